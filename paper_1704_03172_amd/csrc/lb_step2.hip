// lb_step2.hip -- the temporally blocked step kernel (two time steps per
// launch) of the linear LB scheme, for single grids and for the batched
// executor.  The per-node arithmetic is that of the one-step kernel
// (lb_node.h), so both give the same bits.
#include "lb_internal.h"
#include "lb_node.h"

namespace lbw {
namespace {

constexpr int kAdvBlock = 256;

// ---- two time steps per launch ------------------------------------------------
// Temporal blocking: one pass reads h(n) and writes h(n+2), so every
// population element crosses HBM once per two updates.  A wavefront owns a
// strip of columns and a segment of kT2Rows rows: it loads the segment's rows
// of h(n) plus two halo rows on each side, all at once (of the outermost halo
// rows only the population that streams into the segment), then walks down
// the rows computing h(n+1) (from the rows above, at and below, in
// registers) and h(n+2), storing each finished row.  Pulls along x come from
// the neighbouring lane (cross-lane shuffle).  The strip carries kT2Halo halo
// lanes on each side (two columns are needed), chosen so that strip edges
// fall on 64-byte boundaries: measured on MI355X with copy kernels of this
// access pattern, strips whose edges split 32/64-byte words, and waves that
// stream one row at a time, reach only 3-4.5 TB/s, while all-rows-at-once
// loads with aligned edges match a row-major pass (5.5-5.8 TB/s).  Halo rows and lanes are computed
// redundantly and never stored; the halo's h(n+1) is the same arithmetic at
// the same node (rounded to the storage format), so the result equals two
// launches of the one-step kernel bit for bit.  Only rows and columns the
// wave owns are recorded.
constexpr int kT2Block = 256;
constexpr int kT2Halo = 4;    // halo lanes per side

// Rows per segment: all segment rows plus four halo rows sit in registers,
// so the larger states (D2Q9, FP64, FP16 storage with 4 columns per lane)
// take shorter segments.
template <typename S, int Q>
constexpr int t2_rows() { return (Q == 5 && sizeof(S) == 4) ? 8 : 4; }

template <typename S> struct Tb {
    static constexpr int V = sizeof(S) == 8 ? 1 : int(8 / sizeof(S));   // 8-byte lane accesses
    static constexpr int H = kT2Halo;
    static constexpr int OW = (64 - 2 * H) * V;                          // owned columns per wave (448 B)
};

template <int V, typename S> struct LaneVec { typedef S type __attribute__((ext_vector_type(V), aligned(sizeof(S)))); };

// One row (all populations) of the lane's V columns, converted to T.  VEC:
// one vector access at the lane's wrapped first column xv (the lane's
// columns are contiguous after the wrap when nx is a multiple of V);
// otherwise element accesses at the wrapped columns xw.
template <typename U>
__device__ inline U ld_hint(const U *p, bool keep) {
    return keep ? *p : __builtin_nontemporal_load(p);
}

template <bool VEC, int SEL, bool KEEP, typename S, typename T, int Q, int V>
__device__ inline void load_row2(const S *__restrict__ base, int64_t pstride, int64_t rowoff, int xv,
                                 const int (&xw)[V], T (&out)[Q][V]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if ((SEL > 0 && cyv<Q>(i) <= 0) || (SEL < 0 && cyv<Q>(i) >= 0)) {   // not needed from this row
#pragma unroll
            for (int j = 0; j < V; ++j) out[i][j] = T(0);
            continue;
        }
        const S *r = base + i * pstride + rowoff;
        if constexpr (VEC && V > 1) {
            typedef typename LaneVec<V, S>::type vt;
            vt t = ld_hint(reinterpret_cast<const vt *>(r + xv), KEEP);
#pragma unroll
            for (int j = 0; j < V; ++j) out[i][j] = T(t[j]);
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) out[i][j] = T(ld_hint(r + xw[j], KEEP));
        }
    }
}

template <bool VEC, bool KEEP, typename T, int V>
__device__ inline void load_c2row(const T *__restrict__ c2, int64_t rowoff, int xv, const int (&xw)[V], T (&out)[V]) {
    if constexpr (VEC && V > 1) {
        typedef typename LaneVec<V, T>::type vt;
        vt t = ld_hint(reinterpret_cast<const vt *>(c2 + rowoff + xv), KEEP);
#pragma unroll
        for (int j = 0; j < V; ++j) out[j] = t[j];
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) out[j] = ld_hint(c2 + rowoff + xw[j], KEEP);
    }
}

// Whole-wave lane shifts by one lane (DPP wave_shr:1 / wave_shl:1, GFX9
// encodings 0x138 / 0x130): from_lower(v) in lane l is v of lane l - 1,
// from_upper(v) is v of lane l + 1 (the end lanes keep their own value;
// they are halo lanes).
template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL, typename T>
__device__ inline T dpp_shift(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = dpp_u32<CTRL>((uint32_t)u), hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}
template <typename T> __device__ inline T from_lower(T v) { return dpp_shift<0x138>(v); }
template <typename T> __device__ inline T from_upper(T v) { return dpp_shift<0x130>(v); }

// Pulled (pre-collision) state of one row from the rows above (U, y - 1),
// at (C) and below (D, y + 1) it: g_i(x) = h_i(x - c_i).
template <typename T, int Q, int V>
__device__ inline void pull_row2(const T (&U)[Q][V], const T (&C)[Q][V], const T (&D)[Q][V], T (&g)[Q][V]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T r[V];
#pragma unroll
        for (int j = 0; j < V; ++j) r[j] = cyv<Q>(i) > 0 ? U[i][j] : cyv<Q>(i) < 0 ? D[i][j] : C[i][j];
        if (cxv<Q>(i) > 0) {          // from x - 1
            const T l = from_lower(r[V - 1]);
#pragma unroll
            for (int j = V - 1; j > 0; --j) g[i][j] = r[j - 1];
            g[i][0] = l;
        } else if (cxv<Q>(i) < 0) {   // from x + 1
            const T rr = from_upper(r[0]);
#pragma unroll
            for (int j = 0; j < V - 1; ++j) g[i][j] = r[j + 1];
            g[i][V - 1] = rr;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) g[i][j] = r[j];
        }
    }
}

// Blocks are dealt to the 8 XCDs round-robin (block b on XCD b mod 8);
// renumbered, each XCD takes a contiguous range of strips and segments, whose
// shared halo rows then meet in that XCD's L2.
__device__ inline int xcd_block() {
    const int nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, b = blockIdx.x, x8 = b % 8;
    return x8 * q8 + min(x8, r8) + b / 8;
}

// Wave `wave` (of nstrip * nseg for this grid) of a two-step launch; wib: the
// wave's index in its block.  single: take one step only (h(n+1) is stored).
template <typename S, int Q, int KIND, bool VEC>
__device__ inline void step2_wave(const StepParams &p, int wave, int wib, bool single) {
    using T = typename Tr<S>::T;
    constexpr int V = Tb<S>::V, H = Tb<S>::H, OW = Tb<S>::OW, LY = t2_rows<S, Q>(), K = LY + 4;
    const int nx = p.nx, ny = p.ny;
    const int nstrip = (nx + OW - 1) / OW;
    const int nseg = (ny + LY - 1) / LY;
    if ((int64_t)wave >= (int64_t)nstrip * nseg) return;   // whole waves
    const int lane = threadIdx.x & 63;
    const int sx = wave % nstrip, sy = wave / nstrip;
    const int xl = sx * OW - H * V + lane * V;   // first column of this lane
    const int y0 = sy * LY, y1 = min(y0 + LY, ny);
    int xw[V];
    bool own[V];
    const bool own_lane = lane >= H && lane < 64 - H;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        xw[j] = wrapi(xl + j, nx);
        own[j] = own_lane && xl + j < nx;
    }
    const int xv = xw[0];   // VEC: the lane's columns are xv .. xv + V - 1
    int dxw[V];             // distance of each column to the nearest side edge
#pragma unroll
    for (int j = 0; j < V; ++j) dxw[j] = min(xw[j], nx - 1 - xw[j]);
    const S *src = reinterpret_cast<const S *>(p.src);
    S *dst = reinterpret_cast<S *>(p.dst);
    const T *c2 = reinterpret_cast<const T *>(p.c2);
    Receivers rec2 = p.rec;
    rec2.col = p.rec.col + 1;

    // all rows of h(n) at once: R[k] is row y0 - 2 + k (wrapped).  Rows that
    // the neighbouring segments also read (the two halo rows and the two edge
    // rows on each side) are loaded with the ordinary cache policy, so that
    // the segment loaded second finds them in L2; the others stream
    // (nontemporal).
    T R[K][Q][V], C[K][V];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t ro = (int64_t)wrapi(y0 - 2 + k, ny) * nx;
        if (k == 0) {
            load_row2<VEC, 1, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, R[k]);
        } else if (k == K - 1) {
            load_row2<VEC, -1, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, R[k]);
        } else if (k < 4 || k >= K - 4) {
            load_row2<VEC, 0, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, R[k]);
            load_c2row<VEC, true, T, V>(c2, ro, xv, xw, C[k]);
        } else {
            load_row2<VEC, 0, false, S, T, Q, V>(src, p.pstride, ro, xv, xw, R[k]);
            load_c2row<VEC, false, T, V>(c2, ro, xv, xw, C[k]);
        }
    }
    // this segment's slice of the receiver row table, in LDS (a vector-memory
    // load of it would make the arithmetic below wait for every row load)
    __shared__ int32_t s_rows[kT2Block / 64][LY + 1];
    int32_t *rows = s_rows[wib];
    const bool has_rec = p.rec.row_ptr != nullptr;
    if (has_rec) {
        if (lane <= y1 - y0) rows[lane] = p.rec.row_ptr[y0 + lane];
        __builtin_amdgcn_wave_barrier();
    }

    T H1[K][Q][V];   // h(n+1) rows 1 .. K-2 (same indexing as R)
#pragma unroll
    for (int k = 2; k < K; ++k) {
        {
            // h(n+1) at row m = k - 1 from h(n) rows m-1, m, m+1
            const int m = k - 1;
            const int gm = y0 - 2 + m;   // unwrapped row
            const int wm = wrapi(gm, ny);
            T g[Q][V];
            pull_row2<T, Q, V>(R[m - 1], R[m], R[m + 1], g);
            int rb = 0, re = 0;
            if (has_rec && gm >= y0 && gm < y1) {
                rb = rows[gm - y0];
                re = rows[gm - y0 + 1];
            }
#pragma unroll
            for (int j = 0; j < V; ++j) {
                T gj[Q], po[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
                if (rb < re && own[j]) record_node<T, Q>(p.rec, rb, re, xw[j], gj, C[m][j]);
                post_node<T, Q, KIND>(p, gj, C[m][j], xw[j], wm, min(dxw[j], min(wm, ny - 1 - wm)), p.s_n, po);
                // rounded to the storage format, as a stored h(n+1) would be
#pragma unroll
                for (int i = 0; i < Q; ++i) H1[m][i][j] = T(to_store<S>(po[i]));
            }
            if (single && gm >= y0 && gm < y1) {   // one step: h(n+1) is the result
                const int64_t ro = (int64_t)gm * nx;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    S *r = dst + i * p.pstride + ro;
#pragma unroll
                    for (int j = 0; j < V; ++j)
                        if (own[j]) __builtin_nontemporal_store(S(H1[m][i][j]), r + xw[j]);
                }
            }
        }
        if (k >= 4 && !single) {
            // h(n+2) at row mm = k - 2 from h(n+1) rows mm-1, mm, mm+1
            const int mm = k - 2;
            const int gm = y0 - 2 + mm;   // in [y0, y0 + LY)
            if (gm < y1) {
                T g[Q][V];
                pull_row2<T, Q, V>(H1[mm - 1], H1[mm], H1[mm + 1], g);
                int rb = 0, re = 0;
                if (has_rec) {
                    rb = rows[gm - y0];
                    re = rows[gm - y0 + 1];
                }
                S outv[Q][V];
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    T gj[Q], po[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
                    if (rb < re && own[j]) record_node<T, Q>(rec2, rb, re, xw[j], gj, C[mm][j]);
                    post_node<T, Q, KIND>(p, gj, C[mm][j], xw[j], gm, min(dxw[j], min(gm, ny - 1 - gm)), p.s_n2, po);
#pragma unroll
                    for (int i = 0; i < Q; ++i) outv[i][j] = to_store<S>(po[i]);
                }
                const int64_t ro = (int64_t)gm * nx;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    S *r = dst + i * p.pstride + ro;
                    if constexpr (VEC && V > 1) {
                        if (own[0]) {   // nx is a multiple of V: an owned lane owns all its columns
                            typedef typename LaneVec<V, S>::type vt;
                            vt t;
#pragma unroll
                            for (int j = 0; j < V; ++j) t[j] = outv[i][j];
                            __builtin_nontemporal_store(t, reinterpret_cast<vt *>(r + xv));
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j)
                            if (own[j]) __builtin_nontemporal_store(outv[i][j], r + xw[j]);
                    }
                }
            }
        }
    }
}

template <typename S, int Q, int KIND, bool VEC>
__global__ __launch_bounds__(kT2Block) void k_step2(StepParams p) {
    // wave-uniform (so that the row and loop arithmetic is scalar)
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    step2_wave<S, Q, KIND, VEC>(p, xcd_block() * (kT2Block / 64) + wib, wib, false);
}

// Two steps (one for a shot with one step left) of every active shot in one
// launch: wave w belongs to the active shot a with wprefix[a] <= w <
// wprefix[a+1] (waves of nstrip x nseg per shot).
template <typename S, int Q, int KIND>
__global__ __launch_bounds__(kT2Block) void k_step2_batch(BatchParams bp) {
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)xcd_block() * (kT2Block / 64) + wib;
    if (w >= bp.wprefix[bp.nact]) return;
    int lo = 0, hi = bp.nact - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bp.wprefix[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int slot = bp.order[lo];
    const ShotState ss = bp.state[slot];
    if (!ss.active || ss.t >= ss.t_end) return;
    const ShotEntry &e = bp.table[slot];
    StepParams p;
    p.src = ss.cur ? e.pop1 : e.pop0;
    p.dst = ss.cur ? e.pop0 : e.pop1;
    p.c2 = e.c2;
    p.nx = e.nx;
    p.ny = e.ny;
    p.pstride = e.pstride;
    p.q = Q;
    p.coll = bp.coll;
    p.sponge_width = e.sponge_width;
    p.sponge_smax = e.sponge_smax;
    p.src_x = e.src_x;
    p.src_y = e.src_y;
    const int64_t tn = ss.t + 1;
    p.s_n = tn < e.wavelet_len ? e.wavelet[tn] : 0.0;
    p.s_n2 = tn + 1 < e.wavelet_len ? e.wavelet[tn + 1] : 0.0;
    p.rec = e.rec;
    p.rec.col = tn;
    const bool single = ss.t_end - ss.t == 1;
    const int lw = int(w - bp.wprefix[lo]);
    if (e.nx % Tb<S>::V == 0) step2_wave<S, Q, KIND, true>(p, lw, wib, single);
    else step2_wave<S, Q, KIND, false>(p, lw, wib, single);
}

// After a two-step batch launch: each active shot advanced by min(2, steps
// left) in one buffer swap.
__global__ __launch_bounds__(kAdvBlock) void k_batch_advance2(ShotState *state, const int32_t *order, int nact) {
    int a = blockIdx.x * kAdvBlock + threadIdx.x;
    if (a >= nact) return;
    ShotState &ss = state[order[a]];
    if (ss.active && ss.t < ss.t_end) {
        ss.t += min<int64_t>(2, ss.t_end - ss.t);
        ss.cur ^= 1;
    }
}

}  // namespace

template <typename S>
static hipError_t step2_dispatch(const StepParams &p, hipStream_t s) {
    constexpr int OW = Tb<S>::OW;
    const int ly = p.q == 5 ? t2_rows<S, 5>() : t2_rows<S, 9>();
    const int64_t waves = (int64_t)((p.nx + OW - 1) / OW) * ((p.ny + ly - 1) / ly);
    dim3 grid((unsigned)((waves + kT2Block / 64 - 1) / (kT2Block / 64)));
    const int kind = p.coll.kind;
    // vector accesses need every lane's columns contiguous after the wrap
    const bool vec = p.nx % Tb<S>::V == 0;
#define LBW_L2(QQ, KK)                                                                        \
    do {                                                                                      \
        if (vec) hipLaunchKernelGGL((k_step2<S, QQ, KK, true>), grid, dim3(kT2Block), 0, s, p);  \
        else hipLaunchKernelGGL((k_step2<S, QQ, KK, false>), grid, dim3(kT2Block), 0, s, p);     \
    } while (0)
    if (p.q == 5) { if (kind == 0) LBW_L2(5, 0); else LBW_L2(5, 1); }
    else if constexpr (sizeof(S) != 2) { if (kind == 0) LBW_L2(9, 0); else LBW_L2(9, 1); }
    else return hipErrorInvalidValue;   // not offered: see step2_supported
#undef LBW_L2
    return hipGetLastError();
}

hipError_t launch_step2(int storage, const StepParams &p, hipStream_t s) {
    if (p.nx < 1 || p.ny < 1) return hipErrorInvalidValue;
    switch (storage) {
    case ST_F32: return step2_dispatch<float>(p, s);
    case ST_F64: return step2_dispatch<double>(p, s);
    case ST_F16: return step2_dispatch<_Float16>(p, s);
    }
    return hipErrorInvalidValue;
}

int step2_owned_columns(int storage) {
    return storage == ST_F32 ? Tb<float>::OW : storage == ST_F64 ? Tb<double>::OW : Tb<_Float16>::OW;
}

bool step2_supported(int storage, int q) {
    // FP16 storage with D2Q9 would hold its 4-column lanes' rows in scratch
    return !(storage == ST_F16 && q == 9);
}

int64_t step2_waves(int storage, int q, int32_t nx, int32_t ny) {
    const int ow = step2_owned_columns(storage);
    int ly;
    if (storage == ST_F32) ly = q == 5 ? t2_rows<float, 5>() : t2_rows<float, 9>();
    else if (storage == ST_F64) ly = q == 5 ? t2_rows<double, 5>() : t2_rows<double, 9>();
    else ly = q == 5 ? t2_rows<_Float16, 5>() : t2_rows<_Float16, 9>();
    return (int64_t)((nx + ow - 1) / ow) * ((ny + ly - 1) / ly);
}

hipError_t launch_step2_batch(int storage, int q, const BatchParams &bp, int64_t nwaves, hipStream_t s) {
    if (nwaves <= 0 || bp.nact <= 0) return hipSuccess;
    if (!step2_supported(storage, q)) return hipErrorInvalidValue;
    dim3 grid((unsigned)((nwaves + kT2Block / 64 - 1) / (kT2Block / 64)));
    const bool mrt = bp.coll.kind == 1;
#define LBW_B2(SS, QQ)                                                                             \
    do {                                                                                           \
        if (mrt) hipLaunchKernelGGL((k_step2_batch<SS, QQ, 1>), grid, dim3(kT2Block), 0, s, bp);   \
        else hipLaunchKernelGGL((k_step2_batch<SS, QQ, 0>), grid, dim3(kT2Block), 0, s, bp);       \
    } while (0)
    if (storage == ST_F32) { if (q == 5) LBW_B2(float, 5); else LBW_B2(float, 9); }
    else if (storage == ST_F64) { if (q == 5) LBW_B2(double, 5); else LBW_B2(double, 9); }
    else LBW_B2(_Float16, 5);
#undef LBW_B2
    return hipGetLastError();
}

hipError_t launch_batch_advance2(ShotState *state, const int32_t *order, int nact, hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_advance2, dim3((unsigned)((nact + kAdvBlock - 1) / kAdvBlock)), dim3(kAdvBlock), 0, s, state, order, nact);
    return hipGetLastError();
}

}  // namespace lbw
