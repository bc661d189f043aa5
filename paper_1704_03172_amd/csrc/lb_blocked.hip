// lb_blocked.hip -- the temporally blocked step kernel of the linear LB
// scheme (several time steps per launch), for single grids and for the
// batched executor.  The per-node arithmetic is that of the one-step kernel
// (lb_node.h), so both give the same bits.
#include "lb_internal.h"
#include "lb_node.h"

#include <type_traits>

namespace lbw {
namespace {

constexpr int kAdvBlock = 256;

// ---- NS time steps per launch ---------------------------------------------------
// Temporal blocking: one pass reads h(n) and writes h(n+NS), so every
// population element crosses HBM once per NS updates (NS = 3 for D2Q5 with
// FP32 populations, 2 otherwise).  A wavefront owns a strip of columns and a
// segment of rows: it loads the segment's rows of h(n) plus NS halo rows on
// each side, all at once (of the outermost halo rows only the population
// that streams into the segment), then walks down the rows computing
// h(n+1), ..., h(n+NS) from the rows above, at and below, in registers, and
// stores each finished row.  Pulls along x come from the neighbouring lane
// (DPP lane shifts).  The strip carries kT2Halo halo lanes on each side (NS
// columns are needed), chosen so that strip edges fall on 64-byte
// boundaries: measured on MI355X with copy kernels of this access pattern,
// strips whose edges split 32/64-byte words, and waves that stream one row
// at a time, reach only 3-4.5 TB/s, while all-rows-at-once loads with
// aligned edges match a row-major pass (5.5-5.8 TB/s).  Halo rows and lanes
// are computed redundantly and never stored; the halo's intermediate states
// are the same arithmetic at the same nodes (rounded to the storage format),
// so the result equals NS launches of the one-step kernel bit for bit.  Only
// rows and columns the wave owns are recorded.
constexpr int kT2Block = 256;
constexpr int kT2Halo = 4;    // halo lanes per side

// Rows per segment of the two-step kernel: all segment rows plus four halo
// rows sit in registers, so the larger states (D2Q9, FP64, FP16 storage with
// 4 columns per lane) take shorter segments.
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

// f(integral_constant<int, i>) for i = B .. E-1, unrolled at compile time (a
// loop this large is beyond the unroller's size limit, and runtime row
// indices would put the row arrays in scratch memory).
template <int B, typename F, int... I>
__device__ inline void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, B + I>{}), ...);
}
template <int B, int E, typename F>
__device__ inline void static_for(F &&f) {
    static_for_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

// One of three arrays chosen at compile time (separate arrays per stage stay
// in registers; one array of all stages would be too large to promote).
template <int I, typename A>
__device__ inline A &pick3(A &a0, A &a1, A &a2) {
    if constexpr (I == 0) return a0;
    else if constexpr (I == 1) return a1;
    else return a2;
}

// Steps per launch the blocked kernel offers for a configuration: three for
// D2Q5 with FP32 populations, two for the others (larger per-row state).
template <typename S, int Q>
constexpr int tn_max() { return (Q == 5 && sizeof(S) == 4) ? 3 : 2; }

// Rows per segment for NS steps: all segment rows plus NS halo rows on each
// side sit in registers.
template <typename S, int Q, int NS>
constexpr int tn_rows() { return NS == 3 ? 6 : t2_rows<S, Q>(); }

// Wave `wave` (of nstrip * nseg for this grid) of an NS-step launch; wib: the
// wave's index in its block.  The wave takes nrun <= NS steps: stage s
// (1..nrun) computes h(n+s) from h(n+s-1); the state of stage nrun is stored.
template <typename S, int Q, int KIND, bool VEC, int NS>
__device__ inline void stepn_wave(const StepParams &p, int wave, int wib, int nrun) {
    using T = typename Tr<S>::T;
    constexpr int V = Tb<S>::V, H = Tb<S>::H, OW = Tb<S>::OW, LY = tn_rows<S, Q, NS>(), K = LY + 2 * NS;
    static_assert(H * V >= NS, "the strip halo must cover one column per step");
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
    const double sn[3] = {p.s_n, p.s_n2, p.s_n3};

    // L0[k]: row y0 - NS + k (wrapped) of h(n), all rows loaded at once;
    // L1[k], L2[k]: the same row of h(n+1), h(n+2).  Rows that the neighbouring segments
    // also read (the NS halo rows and the NS edge rows on each side) are
    // loaded with the ordinary cache policy, so that the segment loaded
    // second finds them in L2; the others stream (nontemporal).  Of the
    // outermost rows only the populations that stream into the segment are
    // needed.
    T L0[K][Q][V], L1[K][Q][V], L2[K][Q][V], C[K][V];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t ro = (int64_t)wrapi(y0 - NS + k, ny) * nx;
        if (k == 0) {
            load_row2<VEC, 1, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
        } else if (k == K - 1) {
            load_row2<VEC, -1, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
        } else if (k < 2 * NS || k >= K - 2 * NS) {
            load_row2<VEC, 0, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
            load_c2row<VEC, true, T, V>(c2, ro, xv, xw, C[k]);
        } else {
            load_row2<VEC, 0, false, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
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

    // stage st (1..NS) at row m: h(n+st) from rows m-1, m, m+1 of h(n+st-1)
    auto stage = [&](auto stc, auto mc) __attribute__((always_inline)) {
        constexpr int st = decltype(stc)::value;
        constexpr int m = decltype(mc)::value;
        if (st > nrun) return;
        const int gm = y0 - NS + m;   // unwrapped row
        const bool owned_row = gm >= y0 && gm < y1;
        if (st == nrun && !owned_row) return;   // the last stage computes owned rows only
        auto &A = pick3<st - 1>(L0, L1, L2);
        const int wm = wrapi(gm, ny);
        T g[Q][V];
        pull_row2<T, Q, V>(A[m - 1], A[m], A[m + 1], g);
        int rb = 0, re = 0;
        if (has_rec && owned_row) {
            rb = rows[gm - y0];
            re = rows[gm - y0 + 1];
        }
        Receivers rc = p.rec;
        rc.col = p.rec.col + st - 1;
        T po[Q][V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            T gj[Q], pj[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
            if (rb < re && own[j]) record_node<T, Q>(rc, rb, re, xw[j], gj, C[m][j]);
            post_node<T, Q, KIND>(p, gj, C[m][j], xw[j], wm, min(dxw[j], min(wm, ny - 1 - wm)), sn[st - 1], pj);
            // rounded to the storage format, as a stored h(n+st) would be
#pragma unroll
            for (int i = 0; i < Q; ++i) po[i][j] = T(to_store<S>(pj[i]));
        }
        if (st == nrun) {
            if (owned_row) {   // the result of this launch
                const int64_t ro = (int64_t)gm * nx;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    S *r = dst + i * p.pstride + ro;
                    if constexpr (VEC && V > 1) {
                        if (own[0]) {   // nx is a multiple of V: an owned lane owns all its columns
                            typedef typename LaneVec<V, S>::type vt;
                            vt t;
#pragma unroll
                            for (int j = 0; j < V; ++j) t[j] = S(po[i][j]);
                            __builtin_nontemporal_store(t, reinterpret_cast<vt *>(r + xv));
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j)
                            if (own[j]) __builtin_nontemporal_store(S(po[i][j]), r + xw[j]);
                    }
                }
            }
        } else if constexpr (st < NS) {
            auto &B = pick3<st>(L0, L1, L2);
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int j = 0; j < V; ++j) B[m][i][j] = po[i][j];
        }
    };
    // walk down the rows: at index k, stage st computes row m = k - st (its
    // three source rows of stage st-1 are then complete)
    static_for<2, K>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        if constexpr (k - 1 >= 1 && k - 1 <= K - 2)
            stage(std::integral_constant<int, 1>{}, std::integral_constant<int, k - 1>{});
        if constexpr (NS >= 2 && k - 2 >= 2 && k - 2 <= K - 3)
            stage(std::integral_constant<int, 2>{}, std::integral_constant<int, k - 2>{});
        if constexpr (NS >= 3 && k - 3 >= 3 && k - 3 <= K - 4)
            stage(std::integral_constant<int, 3>{}, std::integral_constant<int, k - 3>{});
    });
}

template <typename S, int Q, int KIND, bool VEC, int NS>
__global__ __launch_bounds__(kT2Block) void k_stepn(StepParams p) {
    // wave-uniform (so that the row and loop arithmetic is scalar)
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    stepn_wave<S, Q, KIND, VEC, NS>(p, xcd_block() * (kT2Block / 64) + wib, wib, p.nrun);
}

// Up to NS steps of every active shot in one launch (a shot takes
// min(NS, bp.max_run, steps left)): wave w belongs to the active shot a with
// wprefix[a] <= w < wprefix[a+1] (waves of nstrip x nseg per shot).
template <typename S, int Q, int KIND, int NS>
__global__ __launch_bounds__(kT2Block) void k_stepn_batch(BatchParams bp) {
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
    p.s_n3 = tn + 2 < e.wavelet_len ? e.wavelet[tn + 2] : 0.0;
    p.rec = e.rec;
    p.rec.col = tn;
    const int nrun = (int)min<int64_t>(min(NS, bp.max_run), ss.t_end - ss.t);
    const int lw = int(w - bp.wprefix[lo]);
    if (e.nx % Tb<S>::V == 0) stepn_wave<S, Q, KIND, true, NS>(p, lw, wib, nrun);
    else stepn_wave<S, Q, KIND, false, NS>(p, lw, wib, nrun);
}

// After a blocked batch launch of up to `run` steps: each active shot
// advanced by min(run, steps left) in one buffer swap.
__global__ __launch_bounds__(kAdvBlock) void k_batch_advance_n(ShotState *state, const int32_t *order, int nact,
                                                               int run) {
    int a = blockIdx.x * kAdvBlock + threadIdx.x;
    if (a >= nact) return;
    ShotState &ss = state[order[a]];
    if (ss.active && ss.t < ss.t_end) {
        ss.t += min<int64_t>(run, ss.t_end - ss.t);
        ss.cur ^= 1;
    }
}

}  // namespace

template <typename S, int NS>
static hipError_t stepn_dispatch(const StepParams &p, hipStream_t s) {
    constexpr int OW = Tb<S>::OW;
    const int ly = p.q == 5 ? tn_rows<S, 5, NS>() : tn_rows<S, 9, NS>();
    const int64_t waves = (int64_t)((p.nx + OW - 1) / OW) * ((p.ny + ly - 1) / ly);
    dim3 grid((unsigned)((waves + kT2Block / 64 - 1) / (kT2Block / 64)));
    const int kind = p.coll.kind;
    // vector accesses need every lane's columns contiguous after the wrap
    const bool vec = p.nx % Tb<S>::V == 0;
#define LBW_LN(QQ, KK)                                                                             \
    do {                                                                                           \
        if (vec) hipLaunchKernelGGL((k_stepn<S, QQ, KK, true, NS>), grid, dim3(kT2Block), 0, s, p);   \
        else hipLaunchKernelGGL((k_stepn<S, QQ, KK, false, NS>), grid, dim3(kT2Block), 0, s, p);      \
    } while (0)
    if (p.q == 5) { if (kind == 0) LBW_LN(5, 0); else LBW_LN(5, 1); }
    else if constexpr (sizeof(S) != 2 && NS == 2) { if (kind == 0) LBW_LN(9, 0); else LBW_LN(9, 1); }
    else return hipErrorInvalidValue;   // not offered: see stepn_max
#undef LBW_LN
    return hipGetLastError();
}

int stepn_max(int storage, int q) {
    if (storage == ST_F16 && q == 9) return 1;   // would hold its 4-column lanes' rows in scratch
    if (storage == ST_F32) return q == 5 ? tn_max<float, 5>() : tn_max<float, 9>();
    if (storage == ST_F64) return q == 5 ? tn_max<double, 5>() : tn_max<double, 9>();
    return tn_max<_Float16, 5>();
}

hipError_t launch_stepn(int storage, const StepParams &p, int ns, hipStream_t s) {
    if (p.nx < 1 || p.ny < 1 || ns < 2 || ns > stepn_max(storage, p.q) || p.nrun < 1 || p.nrun > ns)
        return hipErrorInvalidValue;
    switch (storage) {
    case ST_F32: return ns == 3 ? stepn_dispatch<float, 3>(p, s) : stepn_dispatch<float, 2>(p, s);
    case ST_F64: return stepn_dispatch<double, 2>(p, s);
    case ST_F16: return stepn_dispatch<_Float16, 2>(p, s);
    }
    return hipErrorInvalidValue;
}

int64_t stepn_waves(int storage, int q, int ns, int32_t nx, int32_t ny) {
    int ow, ly;
    if (storage == ST_F32) {
        ow = Tb<float>::OW;
        ly = ns == 3 ? tn_rows<float, 5, 3>() : (q == 5 ? tn_rows<float, 5, 2>() : tn_rows<float, 9, 2>());
    } else if (storage == ST_F64) {
        ow = Tb<double>::OW;
        ly = q == 5 ? tn_rows<double, 5, 2>() : tn_rows<double, 9, 2>();
    } else {
        ow = Tb<_Float16>::OW;
        ly = tn_rows<_Float16, 5, 2>();
    }
    return (int64_t)((nx + ow - 1) / ow) * ((ny + ly - 1) / ly);
}

hipError_t launch_stepn_batch(int storage, int q, int ns, const BatchParams &bp, int64_t nwaves, hipStream_t s) {
    if (nwaves <= 0 || bp.nact <= 0) return hipSuccess;
    if (ns < 2 || ns > stepn_max(storage, q) || bp.max_run < 1 || bp.max_run > ns) return hipErrorInvalidValue;
    dim3 grid((unsigned)((nwaves + kT2Block / 64 - 1) / (kT2Block / 64)));
    const bool mrt = bp.coll.kind == 1;
#define LBW_BN(SS, QQ, NN)                                                                             \
    do {                                                                                               \
        if (mrt) hipLaunchKernelGGL((k_stepn_batch<SS, QQ, 1, NN>), grid, dim3(kT2Block), 0, s, bp);   \
        else hipLaunchKernelGGL((k_stepn_batch<SS, QQ, 0, NN>), grid, dim3(kT2Block), 0, s, bp);       \
    } while (0)
    if (storage == ST_F32) {
        if (q == 5) { if (ns == 3) LBW_BN(float, 5, 3); else LBW_BN(float, 5, 2); }
        else LBW_BN(float, 9, 2);
    } else if (storage == ST_F64) {
        if (q == 5) LBW_BN(double, 5, 2); else LBW_BN(double, 9, 2);
    } else {
        LBW_BN(_Float16, 5, 2);
    }
#undef LBW_BN
    return hipGetLastError();
}

hipError_t launch_batch_advance_n(ShotState *state, const int32_t *order, int nact, int run, hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_advance_n, dim3((unsigned)((nact + kAdvBlock - 1) / kAdvBlock)), dim3(kAdvBlock), 0,
                       s, state, order, nact, run);
    return hipGetLastError();
}

int step2_owned_columns(int storage) {
    return storage == ST_F32 ? Tb<float>::OW : storage == ST_F64 ? Tb<double>::OW : Tb<_Float16>::OW;
}

}  // namespace lbw
