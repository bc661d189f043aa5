// lb_blocked.h -- the temporally blocked step kernel of the linear LB scheme
// (several time steps per launch), for single grids and for the batched
// executor, and its templated launchers.  The per-node arithmetic is that of
// the one-step kernel (lb_node.h), so both give the same bits.  Included by
// one source per storage format and lattice (lb_blocked_*.hip, compiled in
// parallel) and by the dispatcher lb_blocked.hip.  Device code only; not
// part of the public interface.
#pragma once

#include "lb_internal.h"
#include "lb_node.h"

#include <type_traits>

namespace lbw {
namespace {

// ---- NS time steps per launch ---------------------------------------------------
// Temporal blocking: one pass reads h(n) and writes h(n+NS), so every
// population element crosses HBM once per NS updates (NS up to 4, see
// tn_max).  A wavefront owns a strip of columns and a segment of rows: it
// loads the segment's rows of h(n) plus NS halo rows on each side, all at
// once or a few rows ahead of the walk (tn_prefetch; of the outermost halo
// rows only the population that streams into the segment), walks down the
// rows computing h(n+1), ..., h(n+NS) from the rows above, at and below, in
// registers, and stores each finished row.  Pulls along x come from the neighbouring lane
// (DPP lane shifts).  The strip carries H halo lanes on each side (NS
// columns are needed; see Tb).  Measured on MI355X with copy kernels of
// this access pattern, waves that stream one row at a time reach only
// 3-4.5 TB/s, while all-rows-at-once loads match a row-major pass
// (5.5-5.8 TB/s with strip edges on 64-byte boundaries).  Halo rows and lanes
// are computed redundantly and never stored; the halo's intermediate states
// are the same arithmetic at the same nodes (rounded to the storage format),
// so the result equals NS launches of the one-step kernel bit for bit.  Only
// rows and columns the wave owns are recorded.
constexpr int kT2Block = 256;
// Block of the marching kernels: two waves for FP32 (measured at 4096^2:
// 30.48 against 30.71 us per step for four-wave blocks of D2Q5 BGK, 34.80
// for eight), four for FP16 storage and FP64 (FP16 D2Q5 BGK: 583 against
// 607 GLUPS with two-wave blocks).
template <typename S>
constexpr int march_block() { return std::is_same_v<S, float> ? 128 : 256; }

constexpr int kT2Halo = 4;    // halo lanes per side

template <typename S> struct Tb {
    static constexpr int V = sizeof(S) == 8 ? 1 : int(8 / sizeof(S));   // 8-byte lane accesses
    // FP32: two halo lanes (4 columns, enough for 4 steps; strip edges at
    // 480 B, measured 2 % faster than four lanes at 448 B: less redundant
    // work outweighs the unaligned edges once the kernel is not
    // bandwidth-bound)
    static constexpr int H = sizeof(S) == 4 ? 2 : kT2Halo;
    static constexpr int OW = (64 - 2 * H) * V;   // owned columns per wave (480 B for FP32, 448 B otherwise)
};

template <int V, typename S> struct LaneVec { typedef S type __attribute__((ext_vector_type(V), aligned(sizeof(S)))); };

// The populations and c^2 live in global memory.  The walks' accesses say
// so: a batched launch reads the arrays' addresses from memory as generic
// pointers, whose accesses would otherwise take the flat path.
template <typename U>
using GlobalPtr = __attribute__((address_space(1))) U *;

// Load with the ordinary cache policy (keep) or nontemporal.
template <typename U>
__device__ inline U ld_hint(const U *p, bool keep) {
    const GlobalPtr<const U> g = (GlobalPtr<const U>)p;
    return keep ? *g : __builtin_nontemporal_load(g);
}

// Nontemporal store to global memory.
template <typename U>
__device__ inline void st_nt(U v, U *p) {
    __builtin_nontemporal_store(v, (GlobalPtr<U>)p);
}

// Element x of a row as a wave-uniform row pointer plus an unsigned 32-bit
// byte offset per lane, so that the access takes the scalar-base form
// (no per-lane 64-bit address arithmetic).  x >= 0 and x * sizeof(U) < 2^32.
template <typename U, typename E>
__device__ inline U *at_lane(E *row, int x) {
    return reinterpret_cast<U *>(reinterpret_cast<
        std::conditional_t<std::is_const_v<E>, const char, char> *>(row) + (uint32_t)x * (uint32_t)sizeof(E));
}

// One row (all populations) of the lane's V columns, converted to T.  VEC:
// one vector access at the lane's wrapped first column xv (the lane's
// columns are contiguous after the wrap when nx is a multiple of V);
// otherwise element accesses at the wrapped columns xw.  SEL > 0 / < 0:
// only the populations that move toward +y / -y (c_y = +1 / -1).
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
            vt t = ld_hint(at_lane<const vt>(r, xv), KEEP);
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
        vt t = ld_hint(at_lane<const vt>(c2 + rowoff, xv), KEEP);
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

// One of four arrays chosen at compile time (separate arrays per stage stay
// in registers; one array of all stages would be too large to promote).
template <int I, typename A>
__device__ inline A &pick4(A &a0, A &a1, A &a2, A &a3) {
    if constexpr (I == 0) return a0;
    else if constexpr (I == 1) return a1;
    else if constexpr (I == 2) return a2;
    else return a3;
}

// Steps per launch the blocked kernel offers for a configuration: the most
// that measured faster at 4096^2 on MI355X without scratch memory.  1: not
// offered (D2Q9 with FP16 storage, whose 4-column lanes would hold nine
// populations per row).
template <typename S, int Q, int KIND>
constexpr int tn_max() {
    if constexpr (sizeof(S) == 2) return Q == 5 ? 3 : 1;
    else if constexpr (Q == 9 && sizeof(S) == 4) return 3;
    else return 4;
}

// Rows per segment for NS steps: the segment rows plus NS halo rows on each
// side are in flight in registers, so more steps and larger per-row states
// take shorter segments.  Most configurations load their rows a prefetch
// distance ahead of the walk (tn_prefetch), which bounds the rows in flight
// and leaves room for taller segments.  Each height is the tallest that
// measured faster at 4096^2 while the kernel stays at three waves per SIMD
// (at most 168 VGPRs) where it was there before (D2Q5 FP32 6 rows: 9 %
// faster than 4, 7 rows within 0.1 % for BGK at tau = 1/2 and 8 rows no
// faster; D2Q5 FP64 7 rows 2 % faster than 6 (8: MRT at two waves);
// D2Q9 FP32 BGK 5 rows: 7 % faster than 4, 3 rows at three waves
// per SIMD 2.5 % slower; D2Q9 FP32 MRT three steps in 3-row segments, three
// waves per SIMD: 21 % faster than two steps in 4 rows, 4 rows at two waves
// 12 % slower; D2Q9 FP64 BGK 6 rows: 8 %; D2Q9 FP64 MRT 5 rows: 10 %; FP16
// storage with three steps: BGK at tau = 1/2 5 rows, 3 % faster than 4;
// MRT and general BGK 4 rows, three waves per SIMD, 11 % faster than 5).
template <typename S, int Q, int NS, int KIND>
constexpr int tn_rows() {
    if constexpr (Q == 9) return KIND == 1 ? (sizeof(S) == 8 ? 5 : 3) : sizeof(S) == 8 ? 6 : 5;
    else if constexpr (sizeof(S) == 2) return KIND == 2 ? 5 : 4;
    else if constexpr (NS == 4) return sizeof(S) == 8 ? 7 : 6;
    else if constexpr (NS == 2 && sizeof(S) == 4) return 8;
    else if constexpr (NS == 3) return 6;
    else return 4;
}

// Rows the walk keeps loads ahead (0: all rows of the segment at once;
// measured 6 better than 4 or 8).
template <typename S, int Q, int NS, int KIND>
constexpr int tn_prefetch() {
    if constexpr (Q == 9) return KIND == 1 && sizeof(S) == 4 ? 0 : 6;
    else if constexpr (sizeof(S) == 2) return 6;
    else return NS == 4 ? 6 : 0;
}

// Wave `wave` (of nstrip * nseg for this grid) of an NS-step launch.  The
// wave takes nrun <= NS steps (FULL: NS, known at compile time): stage s
// (1..nrun) computes h(n+s) from h(n+s-1); the state of stage nrun is
// stored.
template <typename S, int Q, int KIND, bool VEC, int NS, bool FULL, bool RHO = false>
__device__ __attribute__((always_inline)) inline void stepn_wave(const StepParams &p, int wave, int nrun_arg) {
    using T = typename Tr<S>::T;
    constexpr int V = Tb<S>::V, H = Tb<S>::H, OW = Tb<S>::OW, LY = tn_rows<S, Q, NS, KIND>(), K = LY + 2 * NS;
    constexpr int PD = tn_prefetch<S, Q, NS, KIND>();
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
    const int nrun = FULL ? NS : nrun_arg;
    const int xv = xw[0];   // VEC: the lane's columns are xv .. xv + V - 1
    // whether any column of the strip (halo lanes included, before the wrap)
    // lies within the sponge width of a side edge: else the sponge depends
    // on the row alone
    const int L = p.sponge_width;
    const bool strip_sponge = sx * OW - H * V < L || sx * OW - H * V + 64 * V - 1 >= nx - L;
    int dxw[V];             // distance of each column to the nearest side edge
#pragma unroll
    for (int j = 0; j < V; ++j) dxw[j] = min(xw[j], nx - 1 - xw[j]);
    const S *src = reinterpret_cast<const S *>(p.src);
    S *dst = reinterpret_cast<S *>(p.dst);
    const T *c2 = reinterpret_cast<const T *>(p.c2);
    const double sn[4] = {p.s_n, p.s_n2, p.s_n3, p.s_n4};

    // L0[k]: row y0 - NS + k (wrapped) of h(n), all rows loaded at once;
    // L1[k], L2[k]: the same row of h(n+1), h(n+2).  Rows that the neighbouring segments
    // also read (the NS halo rows and the NS edge rows on each side) are
    // loaded with the ordinary cache policy, so that the segment loaded
    // second finds them in L2; the others stream (nontemporal).  Of the
    // outermost rows only the populations that stream into the segment are
    // needed.
    // this segment's slice of the receiver row table: lane k holds
    // row_ptr[y0 + k], read back per row with readlane (loaded before the
    // rows so that its wait does not hold the arithmetic behind them)
    const bool has_rec = p.rec.row_ptr != nullptr;
    int rowv = 0;
    if (has_rec && lane <= y1 - y0) rowv = p.rec.row_ptr[y0 + lane];

    T L0[K][Q][V], L1[K][Q][V], L2[K][Q][V], L3[K][Q][V], C[K][V];
    // wrapped row of index k: one modulo for the first, then a step with a
    // reset at ny (consecutive rows)
    int wr = wrapi(y0 - NS, ny);
    int wrow[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wrow[k] = wr;
        wr = wr + 1 == ny ? 0 : wr + 1;
    }
    // rows loaded up front: all, or (PD > 0) the first PD + 2, the rest PD
    // rows ahead of the walk (row r is first needed at walk index r)
    constexpr int K0 = (PD > 0 && PD + 2 < K) ? PD + 2 : K;
    auto load_k = [&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        const int64_t ro = (int64_t)wrow[k] * nx;
        if constexpr (k == 0) {
            load_row2<VEC, 1, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
        } else if constexpr (k == K - 1) {
            load_row2<VEC, -1, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
        } else if constexpr (k < 2 * NS || k >= K - 2 * NS) {
            load_row2<VEC, 0, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
            load_c2row<VEC, true, T, V>(c2, ro, xv, xw, C[k]);
        } else {
            load_row2<VEC, 0, false, S, T, Q, V>(src, p.pstride, ro, xv, xw, L0[k]);
            load_c2row<VEC, false, T, V>(c2, ro, xv, xw, C[k]);
        }
    };
    static_for<0, K0>(load_k);

    // stage st (1..NS) at row m: h(n+st) from rows m-1, m, m+1 of h(n+st-1)
    auto stage = [&](auto stc, auto mc) __attribute__((always_inline)) {
        constexpr int st = decltype(stc)::value;
        constexpr int m = decltype(mc)::value;
        if (st > nrun) return;
        const int gm = y0 - NS + m;   // unwrapped row
        const bool owned_row = gm >= y0 && gm < y1;
        if (st == nrun && !owned_row) return;   // the last stage computes owned rows only
        auto &A = pick4<st - 1>(L0, L1, L2, L3);
        const int wm = wrow[m];
        T g[Q][V];
        pull_row2<T, Q, V>(A[m - 1], A[m], A[m + 1], g);
        int rb = 0, re = 0;
        if (has_rec && owned_row) {
            rb = __builtin_amdgcn_readlane(rowv, m - NS);
            re = __builtin_amdgcn_readlane(rowv, m - NS + 1);
        }
        // rho of time n+st (owned nodes), summed as the one-step kernel does
        const bool want_rho = RHO && owned_row;   // RHO: p.rho_out is set
        T *rr = reinterpret_cast<T *>(p.rho_out) + (int64_t)(st - 1) * p.rho_stride + (int64_t)gm * nx;
        T rhov[V];
        Receivers rc = p.rec;
        rc.col = p.rec.col + st - 1;
        // receivers, source and sponge: one wave-uniform test per row, the
        // per-node work (the same as post_node's) only in rows that have it
        if (rb < re) {
            asm volatile("");
#pragma unroll
            for (int j = 0; j < V; ++j) {
                T gj[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
                if (own[j]) record_node<T, Q>(rc, rb, re, xw[j], gj, C[m][j]);
            }
        }
        T pj[V][Q];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            T gj[Q], w[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
            if (want_rho) {
                T rho = T(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) rho += gj[i];
                rhov[j] = rho;
            }
            collide<T, Q, KIND>(gj, C[m][j], p.coll, pj[j], w);
        }
        if (wm == p.src_y) {
            asm volatile("");
#pragma unroll
            for (int j = 0; j < V; ++j) {
                if (xw[j] == p.src_x) {
                    T w[Q];
                    weights<T, Q>(C[m][j], p.coll, w);
                    add_source<T, Q>(w, sn[st - 1], pj[j]);
                }
            }
        }
        const int dy = min(wm, ny - 1 - wm);
        if (strip_sponge || dy < L) {
            asm volatile("");
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int d = min(dxw[j], dy);
                if (d < L) {
                    asm volatile("");
                    apply_sponge<T, Q>(d, L, p.sponge_smax, pj[j]);
                }
            }
        }
        // rounded to the storage format, as a stored h(n+st) would be
        T po[Q][V];
#pragma unroll
        for (int j = 0; j < V; ++j)
#pragma unroll
            for (int i = 0; i < Q; ++i) po[i][j] = T(to_store<S>(pj[j][i]));
        if (want_rho) {
            if constexpr (VEC && V > 1) {
                if (own[0]) {
                    typedef typename LaneVec<V, T>::type rt;
                    rt t;
#pragma unroll
                    for (int j = 0; j < V; ++j) t[j] = rhov[j];
                    *(GlobalPtr<rt>)at_lane<rt>(rr, xv) = t;
                }
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (own[j]) rr[xw[j]] = rhov[j];
            }
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
                            st_nt(t, at_lane<vt>(r, xv));
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < V; ++j)
                            if (own[j]) st_nt(S(po[i][j]), r + xw[j]);
                    }
                }
            }
        } else if constexpr (st < NS) {
            auto &B = pick4<st>(L0, L1, L2, L3);
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
        if constexpr (K0 < K && k + PD < K && k + PD >= K0) load_k(std::integral_constant<int, k + PD>{});
        if constexpr (k - 1 >= 1 && k - 1 <= K - 2)
            stage(std::integral_constant<int, 1>{}, std::integral_constant<int, k - 1>{});
        if constexpr (NS >= 2 && k - 2 >= 2 && k - 2 <= K - 3)
            stage(std::integral_constant<int, 2>{}, std::integral_constant<int, k - 2>{});
        if constexpr (NS >= 3 && k - 3 >= 3 && k - 3 <= K - 4)
            stage(std::integral_constant<int, 3>{}, std::integral_constant<int, k - 3>{});
        if constexpr (NS >= 4 && k - 4 >= 4 && k - 4 <= K - 5)
            stage(std::integral_constant<int, 4>{}, std::integral_constant<int, k - 4>{});
    });
}

// ---- NS steps per launch over tall segments (marching) ---------------------------
// The update of stepn_wave (the same stages in the same order, the same
// per-node arithmetic, so the same bits) over segments of LY rows instead of
// a few, which makes more steps per launch affordable: a segment reads
// LY + 2 NS rows of h(n) and computes NS LY + NS (NS - 1) stage-rows for its
// NS LY owned ones.  The walk is a loop whose body takes U consecutive walk
// indices: row m of h(n) and of every intermediate state sits in ring slot
// m mod U, a compile-time index in each copy of the body, so the rings stay
// in registers.  Row m of h(n) is loaded PD walk indices before stage 1
// first reads it; c^2 of row m, which the stages read at walk indices
// m + 1 .. m + NS, goes through a small per-wave LDS ring (the register ring
// then only spans the prefetch: U > PD + 2).  The strip carries
// ceil(NS / V) halo lanes on each side.  Needs nx a multiple of V (vector
// accesses) and ny >= LY + 2 NS (a row index wraps at most once);
// march_ok() tells.
// FP16 storage takes two columns per lane (4-byte accesses) instead of the
// short-segment kernel's four: its ring rows then hold as many registers as
// FP32's, and four waves fit a SIMD (27.3 against 34.4 us per step for four
// steps with four columns per lane).
template <typename S, int NS> struct MTb {
    static constexpr int V = std::is_same_v<S, _Float16> ? 2 : Tb<S>::V;
    static constexpr int H = (NS + V - 1) / V;
    static constexpr int OW = (64 - 2 * H) * V;
};
// Segment height, prefetch distance and ring length, measured at 4096^2 on
// MI355X (us per step, FP32).  D2Q5 BGK at tau = 1/2: seven steps per launch
// with LY = 20, PD = 2, U = 5 (30.66 at 166 VGPRs: three waves per SIMD;
// LY 25 30.66, LY 15 / 30 / 35: 31.2 / 33.2 / 34.0; U = 6 with LY 18 / 24:
// 30.7 / 31.8; PD 1 with U = 4: 32.7).  The third wave per SIMD is what pays:
// eight steps need 176-187 VGPRs, two waves (33.5 at its best: LY 24, PD 3,
// U 6), six steps run at 36.6 and one column per lane (V = 1, four waves)
// at 35.1-35.9.  D2Q5 MRT: seven steps 37.2 (166 VGPRs), six 39.1 (152;
// 40.5 with U = 6, LY = 24), five 43.5.  D2Q9 BGK at tau = 1/2: six steps
// 63.1 (254 VGPRs, two waves), five 70.2-72.8, four 79.5-80.9 (the
// short-segment kernel, three steps: 102.2).  D2Q9 MRT: five steps 86.4
// (230 VGPRs), four 88.0-89.8, six 87.8 (three steps: 117.0).  D2Q5 with
// FP16 storage, two columns per lane: five steps 27.3 / 35.0 for BGK / MRT
// (120 VGPRs, four waves per SIMD), six 28.4 / 38.0, seven 28.9 / 39.1
// (the short-segment kernel, three steps: 36.0 / 46.4).  FP64, one column
// per lane: D2Q5 BGK eight steps 55.6 (174 VGPRs), seven 58.6, six 62.7,
// four or five 77.5; D2Q5 MRT seven 61.6 (154 VGPRs), eight 70.0, six 64.4;
// D2Q9 four steps 134.5 / 143.8 for BGK / MRT, five 135.4 / 144.8, three
// 212 / 217 (the short-segment kernel, four steps: 76.5 / 79.3 for D2Q5,
// 146.2 / 183.1 for D2Q9).
template <typename S, int Q, int KIND, int NS> struct March {
    static constexpr int LY = 20, PD = 2, U = 5;
    static constexpr int CR = NS <= 4 ? 4 : 8;   // c^2 ring rows (>= NS)
    // Fewest waves for which a single grid's launch plan prefers the
    // marching kernel.  A wave's walk has a latency floor (LY + 2 NS rows one
    // after the other), so a grid with few waves leaves the GPU idle and the
    // short-segment kernel, with more and shorter waves, is faster.  Measured
    // crossovers (square grids): FP32 D2Q5 between 2048^2 (1,957 waves:
    // 14.9 against 13.5 us per step) and 2560^2 (2,944: 17.2 against 18.6);
    // FP32 D2Q9 near 1536^2 (1,078 waves: 17.5 / 17.2); FP64 D2Q5 between
    // 1024^2 (1,144: 9.3 / 7.8) and 1536^2 (2,464: 13.7 / 14.5); FP16 storage
    // between 2048^2 (1,854: 15.0 / 13.6) and 2560^2 (2,944: 16.7 / 17.5).
    // FP64 D2Q9 shares its step count with the short-segment kernel and
    // always marches.  The batched executor, whose marching launch covers
    // every shot's waves at once, marches whatever a shot's size.
    static constexpr int64_t MIN_WAVES = std::is_same_v<S, double> ? (Q == 5 ? 1800 : 0) : Q == 5 ? 2500 : 1100;
};

template <typename S, int Q, int KIND, int NS>
inline bool march_ok(int32_t nx, int32_t ny) {
    return nx % Tb<S>::V == 0 && ny >= March<S, Q, KIND, NS>::LY + 2 * NS;
}

template <typename S, int Q, int KIND, int NS>
inline int64_t march_waves(int32_t nx, int32_t ny) {
    return (int64_t)((nx + MTb<S, NS>::OW - 1) / MTb<S, NS>::OW) *
           ((ny + March<S, Q, KIND, NS>::LY - 1) / March<S, Q, KIND, NS>::LY);
}

// The launch parameters as read inside a rarely taken, wave-uniform branch
// (receivers, source, sponge) of a kernel whose first (only) argument is the
// StepParams: straight from the kernel-argument segment (scalar loads),
// through a pointer whose value the compiler cannot follow, so that the
// fields are loaded where the branch uses them rather than held in scalar
// registers across the whole walk (the march kernel's many stages in flight
// otherwise run out of them and spill).  Taking the address of the by-value
// parameter instead would copy it to scratch memory.
typedef const __attribute__((address_space(4))) StepParams *KernargParams;
__device__ inline KernargParams rare_params() {
    KernargParams q = (KernargParams)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(q));
    return q;
}

// Where the marching walk reads the fields of its rarely taken branches:
// the kernel arguments of a single-grid launch (RareKernarg), or the params
// image of the wave's shot in global memory (a batched launch), through a
// pointer hidden from the compiler for the same reason.
struct RareKernarg {
    __device__ KernargParams operator()() const { return rare_params(); }
};
struct RareGlobal {
    KernargParams img;
    __device__ KernargParams operator()() const {
        KernargParams q = img;
        asm volatile("" : "+s"(q));
        return q;
    }
};

// One of eight arrays chosen at compile time.
template <int I, typename A>
__device__ inline A &pick8(A &a0, A &a1, A &a2, A &a3, A &a4, A &a5, A &a6, A &a7) {
    if constexpr (I < 4) return pick4<I>(a0, a1, a2, a3);
    else return pick4<I - 4>(a4, a5, a6, a7);
}

// RHO: also write rho of each stage's time at the owned nodes (p.rho_out,
// p.rho_stride), summed as the one-step kernel sums it.
template <typename S, int Q, int KIND, int NS, bool RHO = false, typename RARE>
__device__ __attribute__((always_inline)) inline void march_wave(const StepParams &p, int wave,
                                                                 typename Tr<S>::T *c2ring, RARE rare) {
    using T = typename Tr<S>::T;
    using M = March<S, Q, KIND, NS>;
    constexpr int V = MTb<S, NS>::V, H = MTb<S, NS>::H, OW = MTb<S, NS>::OW;
    constexpr int LY = M::LY, PD = M::PD, U = M::U, CR = M::CR;
    constexpr int K = LY + 2 * NS;
    static_assert(NS >= 2 && NS <= 8 && H * V >= NS, "the strip halo must cover one column per step");
    static_assert(U > PD + 2 && PD >= 1, "ring too short for the prefetch distance");
    static_assert(LY % U == 0, "the loop over the walk has no tail");
    static_assert(CR >= NS && (CR & (CR - 1)) == 0, "c^2 ring too short");
    static_assert(LY + 1 <= 64, "the receiver row table of a segment is held one row per lane");
    const int nx = p.nx, ny = p.ny;
    const int nstrip = (nx + OW - 1) / OW;
    const int nseg = (ny + LY - 1) / LY;
    if ((int64_t)wave >= (int64_t)nstrip * nseg) return;
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
    const int xv = xw[0];   // nx is a multiple of V: the lane's columns are xv .. xv + V - 1
    const int L = p.sponge_width;
    const bool strip_sponge = sx * OW - H * V < L || sx * OW - H * V + 64 * V - 1 >= nx - L;
    int dxw[V];
#pragma unroll
    for (int j = 0; j < V; ++j) dxw[j] = min(xw[j], nx - 1 - xw[j]);
    const S *src = reinterpret_cast<const S *>(p.src);
    S *dst = reinterpret_cast<S *>(p.dst);
    const T *c2 = reinterpret_cast<const T *>(p.c2);
    const bool has_rec = p.rec.row_ptr != nullptr;
    int rowv = 0;
    if (has_rec && lane <= y1 - y0) rowv = p.rec.row_ptr[y0 + lane];
    // row m of the segment (0 <= m < K) is unwrapped row y0 - NS + m
    auto wrow = [&](int m) {
        const int r = y0 - NS + m;
        return r < 0 ? r + ny : (r >= ny ? r - ny : r);
    };
    typedef typename LaneVec<V, T>::type ct;
    // this lane's c^2 of row m in the LDS ring (slot m mod CR)
    auto c2slot = [&](int m) { return reinterpret_cast<ct *>(c2ring + ((m & (CR - 1)) * 64 + lane) * V); };

    // R: h(n) rows and their c^2; A1..A7: h(n+1) .. h(n+7) rows; row m in slot m % U
    T R[U][Q][V], C[U][V], A1[U][Q][V], A2[U][Q][V], A3[U][Q][V], A4[U][Q][V], A5[U][Q][V], A6[U][Q][V],
        A7[U][Q][V];
    // rows shared with the neighbouring segments (the NS halo rows and NS edge
    // rows on each side) keep the ordinary cache policy, the others stream
    auto load = [&](auto slc, int m, auto selc) __attribute__((always_inline)) {
        constexpr int SL = decltype(slc)::value, SEL = decltype(selc)::value;
        asm volatile("" : "+s"(m));
        const int64_t ro = (int64_t)wrow(m) * nx;
        if (m < 2 * NS || m >= K - 2 * NS) {
            load_row2<true, SEL, true, S, T, Q, V>(src, p.pstride, ro, xv, xw, R[SL]);
            if constexpr (SEL == 0) load_c2row<true, true, T, V>(c2, ro, xv, xw, C[SL]);
        } else {
            load_row2<true, SEL, false, S, T, Q, V>(src, p.pstride, ro, xv, xw, R[SL]);
            load_c2row<true, false, T, V>(c2, ro, xv, xw, C[SL]);
        }
    };
    // rows 0 .. PD + 1 up front (of row 0 only the populations that stream
    // into the segment)
    static_for<0, PD + 2>([&](auto mc) __attribute__((always_inline)) {
        constexpr int m = decltype(mc)::value;
        load(std::integral_constant<int, m % U>{}, m, std::integral_constant<int, m == 0 ? 1 : 0>{});
    });

    // stage st (1..NS) at walk index k computes row m = k - st from rows
    // m - 1, m, m + 1 of stage st - 1; KM is k mod U, known at compile time
    auto stage = [&](auto stc, auto kmc, int k) __attribute__((always_inline)) {
        constexpr int st = decltype(stc)::value, KM = decltype(kmc)::value;
        constexpr int SM = (KM - st + 8 * U) % U, SU = (SM + U - 1) % U, SD = (SM + 1) % U;
        // the row indices are recomputed in every stage (a few scalar
        // operations): the compiler would otherwise keep each row's values
        // for all the stages that reach it and run out of scalar registers
        asm volatile("" : "+s"(k));
        const int m = k - st;
        const int gm = y0 - NS + m;           // unwrapped row
        const bool owned_row = gm >= y0 && gm < y1;
        if (st == NS && !owned_row) return;   // the last stage computes owned rows only
        auto &A = pick8<st - 1>(R, A1, A2, A3, A4, A5, A6, A7);
        const int wm = wrow(m);
        // c^2 of row m: stage 1 takes it from the loaded row and puts it in
        // the ring for the later stages
        T cm[V];
        if constexpr (st == 1) {
            ct t;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                cm[j] = C[SM][j];
                t[j] = cm[j];
            }
            *c2slot(m) = t;
        } else {
            const ct t = *c2slot(m);
#pragma unroll
            for (int j = 0; j < V; ++j) cm[j] = t[j];
        }
        T g[Q][V];
        pull_row2<T, Q, V>(A[SU], A[SM], A[SD], g);
        if constexpr (RHO) {   // rho of time n+st at the owned nodes
            if (owned_row && own[0]) {
                typedef typename LaneVec<V, T>::type rt;
                rt t;
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    T rho = T(0);
#pragma unroll
                    for (int i = 0; i < Q; ++i) rho += g[i][j];
                    t[j] = rho;
                }
                T *rr = reinterpret_cast<T *>(p.rho_out) + (int64_t)(st - 1) * p.rho_stride + (int64_t)gm * nx;
                *(GlobalPtr<rt>)at_lane<rt>(rr, xv) = t;
            }
        }
        int rb = 0, re = 0;
        if (has_rec && owned_row) {
            rb = __builtin_amdgcn_readlane(rowv, m - NS);
            re = __builtin_amdgcn_readlane(rowv, m - NS + 1);
        }
        if (__builtin_expect(rb < re, 0)) {
            const auto q = rare();
            Receivers rc;   // field by field: no copy constructor from this address space
            rc.row_ptr = q->rec.row_ptr;
            rc.xs = q->rec.xs;
            rc.slot = q->rec.slot;
            rc.traces = q->rec.traces;
            rc.nslots = q->rec.nslots;
            rc.what = q->rec.what;
            rc.cap = q->rec.cap;
            rc.col = q->rec.col + st - 1;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                T gj[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
                if (own[j]) record_node<T, Q>(rc, rb, re, xw[j], gj, cm[j]);
            }
        }
        T pj[V][Q];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            T gj[Q], w[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
            collide<T, Q, KIND>(gj, cm[j], p.coll, pj[j], w);
        }
        if (__builtin_expect(wm == p.src_y, 0)) {
            const auto q = rare();
            const double snv = st == 1 ? q->s_n : st == 2 ? q->s_n2 : st == 3 ? q->s_n3 : st == 4 ? q->s_n4
                                                                                        : q->s_more[(st - 5) & 3];
            const int sxs = q->src_x;
            Collision cl;   // the fields weights() reads
            cl.kw = q->coll.kw;
            cl.ratio = q->coll.ratio;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                if (xw[j] == sxs) {
                    T w[Q];
                    weights<T, Q>(cm[j], cl, w);
                    add_source<T, Q>(w, snv, pj[j]);
                }
            }
        }
        const int dy = min(wm, ny - 1 - wm);
        if (__builtin_expect(strip_sponge || dy < L, 0)) {
            const double smax = rare()->sponge_smax;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int d = min(dxw[j], dy);
                if (d < L) {
                    asm volatile("");
                    apply_sponge<T, Q>(d, L, smax, pj[j]);
                }
            }
        }
        if constexpr (st == NS) {   // owned row: the result of this launch
            const int64_t ro = (int64_t)gm * nx;
            if (own[0]) {
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    typedef typename LaneVec<V, S>::type vt;
                    vt t;
#pragma unroll
                    for (int j = 0; j < V; ++j) t[j] = to_store<S>(pj[j][i]);
                    st_nt(t, at_lane<vt>(dst + i * p.pstride + ro, xv));
                }
            }
        } else {
            // rounded to the storage format, as a stored h(n+st) would be
            auto &B = pick8<st>(R, A1, A2, A3, A4, A5, A6, A7);
#pragma unroll
            for (int j = 0; j < V; ++j)
#pragma unroll
                for (int i = 0; i < Q; ++i) B[SM][i][j] = T(to_store<S>(pj[j][i]));
        }
    };
    // the stages that run at walk index k (stage st from k = 2 st on)
    auto stages = [&](auto kmc, int k, auto firstc) __attribute__((always_inline)) {
        constexpr int FIRST = decltype(firstc)::value;   // -1: all stages run
        static_for<1, NS + 1>([&](auto stc) __attribute__((always_inline)) {
            constexpr int st = decltype(stc)::value;
            if constexpr (FIRST < 0 || FIRST >= 2 * st) stage(stc, kmc, k);
        });
    };

    // walk indices 2 .. 2 NS - 1: the stages start one after the other
    static_for<2, 2 * NS>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        load(std::integral_constant<int, (k + PD) % U>{}, k + PD, std::integral_constant<int, 0>{});
        stages(std::integral_constant<int, k % U>{}, k, std::integral_constant<int, k>{});
    });
    // walk indices 2 NS .. K - 1 (LY of them, U per pass): every stage runs
    // and a row is loaded at every index (past the segment the last row
    // again, an L2 hit), so that no ring slot is written conditionally and
    // the values left in the slots are dead across the loop
    for (int k0 = 2 * NS; k0 < K; k0 += U) {
        static_for<0, U>([&](auto jc) __attribute__((always_inline)) {
            constexpr int J = decltype(jc)::value;
            constexpr int KM = (2 * NS + J) % U;
            const int k = k0 + J;
            load(std::integral_constant<int, (KM + PD) % U>{}, min(k + PD, K - 1), std::integral_constant<int, 0>{});
            stages(std::integral_constant<int, KM>{}, k, std::integral_constant<int, -1>{});
        });
    }
}

template <typename S, int Q, int KIND, int NS>
__global__ __launch_bounds__(march_block<S>()) void k_stepn_march(StepParams p) {
    using T = typename Tr<S>::T;
    constexpr int CR = March<S, Q, KIND, NS>::CR, V = MTb<S, NS>::V;
    __shared__ T c2ring[march_block<S>() / 64][CR * 64 * V];
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    march_wave<S, Q, KIND, NS>(p, xcd_block() * (march_block<S>() / 64) + wib, c2ring[wib], RareKernarg());
}

// The marching launch that also writes rho of every stage's time (the
// forward run that keeps the rho tape, the adjoint's recompute): a kernel of
// its own, so that the forward kernel carries none of its registers.
template <typename S, int Q, int KIND, int NS>
__global__ __launch_bounds__(march_block<S>()) void k_stepn_march_rho(StepParams p) {
    using T = typename Tr<S>::T;
    constexpr int CR = March<S, Q, KIND, NS>::CR, V = MTb<S, NS>::V;
    __shared__ T c2ring[march_block<S>() / 64][CR * 64 * V];
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    march_wave<S, Q, KIND, NS, true>(p, xcd_block() * (march_block<S>() / 64) + wib, c2ring[wib], RareKernarg());
}

template <typename S, int Q, int KIND, bool VEC, int NS, bool RHO>
__global__ __launch_bounds__(kT2Block) void k_stepn(StepParams p) {
    // wave-uniform (so that the row and loop arithmetic is scalar)
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    stepn_wave<S, Q, KIND, VEC, NS, true, RHO>(p, xcd_block() * (kT2Block / 64) + wib, NS);
}

// An NS-step launch of a replayed graph (lane columns contiguous, NS the
// most steps the kernel offers).
template <typename S, int Q, int KIND, int NS>
__global__ __launch_bounds__(kT2Block) void k_stepn_graph(StepParams p) {
    const StepParams q = graph_params(p);
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    stepn_wave<S, Q, KIND, true, NS, true, false>(q, xcd_block() * (kT2Block / 64) + wib, NS);
}

// Up to NS steps of every active shot in one launch (a shot takes
// min(NS, bp.max_run, steps left)): wave w belongs to the active shot a with
// wprefix[a] <= w < wprefix[a+1] (waves of nstrip x nseg per shot).
// FP32 D2Q5: at most 168 VGPRs, three waves per SIMD (its two bodies would
// otherwise take one register more for BGK at tau = 1/2 and halve the
// occupancy); the others keep the compiler's choice.
template <typename S, int Q>
constexpr int batch_min_waves() { return Q == 5 && sizeof(S) == 4 ? 3 : 1; }
template <typename S, int Q, int KIND, int NS>
__global__ __launch_bounds__(kT2Block) __attribute__((amdgpu_waves_per_eu(batch_min_waves<S, Q>())))
void k_stepn_batch(BatchParams bp) {
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)xcd_block() * (kT2Block / 64) + wib;
    if (w >= bp.wprefix[bp.nact]) return;
    int lo = 0, hi = bp.nact - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bp.wprefix[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int slot = bp.order[lo];
    if (bp.img != nullptr && bp.img[slot].nrun > 0) return;   // the round's marching launch takes it
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
    p.s_n4 = tn + 3 < e.wavelet_len ? e.wavelet[tn + 3] : 0.0;
    p.rec = e.rec;
    p.rec.col = tn;
    const int nrun = (int)min<int64_t>(min(NS, bp.max_run), ss.t_end - ss.t);
    const int lw = int(w - bp.wprefix[lo]);
    // a shot taking all NS steps with contiguous lane columns (the common
    // case) runs the body with the step count fixed at compile time; the
    // rest (a shot's last launch, odd widths) the general one
    if (nrun == NS && e.nx % Tb<S>::V == 0) stepn_wave<S, Q, KIND, true, NS, true>(p, lw, NS);
    else stepn_wave<S, Q, KIND, false, NS, false>(p, lw, nrun);
}

// The batched marching launch: wave w belongs to the active shot a with
// mprefix[a] <= w < mprefix[a+1] and walks that shot's grid with the params
// image of the round (shots that sit the round out have no waves of use).
template <typename S, int Q, int KIND, int NS>
__global__ __launch_bounds__(march_block<S>()) void k_stepn_march_batch(BatchParams bp, const StepParams *__restrict__ img) {
    using T = typename Tr<S>::T;
    constexpr int CR = March<S, Q, KIND, NS>::CR, V = MTb<S, NS>::V;
    __shared__ T c2ring[march_block<S>() / 64][CR * 64 * V];
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)xcd_block() * (march_block<S>() / 64) + wib;
    if (w >= bp.mprefix[bp.nact]) return;
    int lo = 0, hi = bp.nact - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bp.mprefix[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int slot = __builtin_amdgcn_readfirstlane(bp.order[lo]);
    // the image through the constant address space: it is read-only while
    // the launch runs, so its fields come in with scalar loads, into scalar
    // registers (through a generic pointer they would be vector loads, and
    // read again after every store of the walk)
    const KernargParams q = (KernargParams)(img + slot);
    if (q->nrun != NS) return;
    StepParams pl;
    pl.src = q->src;
    pl.dst = q->dst;
    pl.c2 = q->c2;
    pl.nx = q->nx;
    pl.ny = q->ny;
    pl.pstride = q->pstride;
    pl.q = q->q;
    pl.coll.kind = q->coll.kind;
    pl.coll.omega = q->coll.omega;
    pl.coll.ratio = q->coll.ratio;
    pl.coll.kw = q->coll.kw;
    pl.coll.kax = q->coll.kax;
    pl.coll.kdg = q->coll.kdg;
    for (int i = 0; i < 9; ++i) pl.coll.srate[i] = q->coll.srate[i];
    pl.sponge_width = q->sponge_width;
    pl.src_y = q->src_y;
    pl.rec.row_ptr = q->rec.row_ptr;
    march_wave<S, Q, KIND, NS>(pl, (int)(w - bp.mprefix[lo]), c2ring[wib], RareGlobal{q});
}

// f(integral_constant<int, ns>()) for 2 <= ns <= the largest tn_max<S, Q, KIND>
// over both collision kinds (else hipErrorInvalidValue); only those step
// counts are instantiated.
template <typename S, int Q, typename F>
hipError_t by_steps(int ns, F &&f) {
    constexpr int m = tn_max<S, Q, 0>() > tn_max<S, Q, 1>() ? tn_max<S, Q, 0>() : tn_max<S, Q, 1>();
    if constexpr (m >= 4) if (ns == 4) return f(std::integral_constant<int, 4>());
    if constexpr (m >= 3) if (ns == 3) return f(std::integral_constant<int, 3>());
    if constexpr (m >= 2) if (ns == 2) return f(std::integral_constant<int, 2>());
    return hipErrorInvalidValue;
}

// Waves of an NS-step launch over an nx x ny grid; kind is the kernel's
// collision kind (step_kind: 0, 1 or 2), whose segment height it takes.
template <typename S, int Q>
int64_t waves_of(int kind, int ns, int32_t nx, int32_t ny) {
    int ly = 1;
    const hipError_t e = by_steps<S, Q>(ns, [&](auto nc) {
        constexpr int NS = decltype(nc)::value;
        ly = kind == 1 ? tn_rows<S, Q, NS, 1>() : kind == 2 ? tn_rows<S, Q, NS, 2>() : tn_rows<S, Q, NS, 0>();
        return hipSuccess;
    });
    if (e != hipSuccess) return 0;   // a step count without a kernel: no waves
    return (int64_t)((nx + Tb<S>::OW - 1) / Tb<S>::OW) * ((ny + ly - 1) / ly);
}

// Steps per launch of the marching kernel (march_wave) for a storage format,
// lattice and collision kind (step_kind()), 0 where it is not instantiated.
// Measured at 4096^2 (D2Q5 FP32 BGK at tau = 1/2): four steps per launch
// marching 24-row segments ran at the speed of the 6-row kernel (45.0
// against 44.4 us per step; both are held by the memory access pattern, not
// by their arithmetic), so the marching kernel only takes the step counts
// that the short segments cannot afford: with FP32 storage seven for D2Q5
// (30.7 us per step for BGK), six for D2Q9 BGK and five for D2Q9 MRT; with
// FP64 eight for D2Q5 BGK, seven for D2Q5 MRT and four for D2Q9; five for
// D2Q5 with FP16 storage (see March).
template <typename S, int Q, int KIND>
constexpr int march_steps() {
    if constexpr (std::is_same_v<S, float>) return Q == 5 ? 7 : KIND == 1 ? 5 : 6;
    else if constexpr (std::is_same_v<S, double>) return Q == 5 ? (KIND == 1 ? 7 : 8) : 4;
    else return Q == 5 ? 5 : 0;
}

// The marching kernel's step count for a grid, 0 if it does not take it
// (pref: also 0 if the grid has fewer waves than the kernel's MIN_WAVES).
template <typename S, int Q>
int march_grid(int kind, int32_t nx, int32_t ny, bool pref = false) {
    auto one = [&](auto kc) {
        constexpr int KK = decltype(kc)::value, MN = march_steps<S, Q, KK>();
        if constexpr (MN == 0) return 0;
        else {
            if (!march_ok<S, Q, KK, MN>(nx, ny)) return 0;
            return !pref || march_waves<S, Q, KK, MN>(nx, ny) >= March<S, Q, KK, MN>::MIN_WAVES ? MN : 0;
        }
    };
    return kind == 1 ? one(std::integral_constant<int, 1>())
         : kind == 2 ? one(std::integral_constant<int, 2>()) : one(std::integral_constant<int, 0>());
}

// MIN_WAVES of the marching kernel for a collision kind (0: none).
template <typename S, int Q>
int64_t march_min_waves_of(int kind) {
    auto one = [&](auto kc) -> int64_t {
        constexpr int KK = decltype(kc)::value, MN = march_steps<S, Q, KK>();
        if constexpr (MN == 0) return 0;
        else return March<S, Q, KK, MN>::MIN_WAVES;
    };
    return kind == 1 ? one(std::integral_constant<int, 1>())
         : kind == 2 ? one(std::integral_constant<int, 2>()) : one(std::integral_constant<int, 0>());
}

// The single-grid NS-step launch for storage S and lattice Q.
template <typename S, int Q>
hipError_t stepn_launch(const StepParams &p, int ns, hipStream_t s) {
    const int kind = step_kind(p.coll);
    const int mn = march_grid<S, Q>(kind, p.nx, p.ny);
    // the marching kernel takes its times from the params only; a launch of
    // a captured chunk takes the short-segment kernel, and so does a launch
    // whose step count both kernels have (FP64 D2Q9) on a grid the marching
    // kernel would leave underfilled
    const int sm = kind == 1 ? tn_max<S, Q, 1>() : kind == 2 ? tn_max<S, Q, 2>() : tn_max<S, Q, 0>();
    if (mn > 0 && ns == mn && p.gtab == nullptr && (ns > sm || march_grid<S, Q>(kind, p.nx, p.ny, true) == mn)) {
        auto launch = [&](auto kc) {
            constexpr int KK = decltype(kc)::value, MN = march_steps<S, Q, KK>();
            if constexpr (MN > 0) {
                const int64_t nw = march_waves<S, Q, KK, MN>(p.nx, p.ny);
                const dim3 mgrid((unsigned)((nw + march_block<S>() / 64 - 1) / (march_block<S>() / 64)));
                if (p.rho_out != nullptr)
                    hipLaunchKernelGGL((k_stepn_march_rho<S, Q, KK, MN>), mgrid, dim3(march_block<S>()), 0, s, p);
                else
                    hipLaunchKernelGGL((k_stepn_march<S, Q, KK, MN>), mgrid, dim3(march_block<S>()), 0, s, p);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        };
        return kind == 1 ? launch(std::integral_constant<int, 1>())
             : kind == 2 ? launch(std::integral_constant<int, 2>()) : launch(std::integral_constant<int, 0>());
    }
    const dim3 grid((unsigned)((waves_of<S, Q>(kind, ns, p.nx, p.ny) + kT2Block / 64 - 1) / (kT2Block / 64)));
    // vector accesses need every lane's columns contiguous after the wrap
    const bool vec = p.nx % Tb<S>::V == 0;
    if (p.gtab) {   // a launch of a captured chunk: its own entry kernel, for the most steps only
        if (!vec || p.rho_out) return hipErrorInvalidValue;
        auto launch = [&](auto kc) {
            constexpr int KK = decltype(kc)::value, NS = tn_max<S, Q, KK>();
            if constexpr (NS >= 2) {
                if (ns != NS) return hipErrorInvalidValue;
                hipLaunchKernelGGL((k_stepn_graph<S, Q, KK, NS>), grid, dim3(kT2Block), 0, s, p);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        };
        return kind == 1 ? launch(std::integral_constant<int, 1>())
             : kind == 2 ? launch(std::integral_constant<int, 2>()) : launch(std::integral_constant<int, 0>());
    }
    return by_steps<S, Q>(ns, [&](auto nc) {
        constexpr int NS = decltype(nc)::value;
        auto launch = [&](auto kc) {
            constexpr int KK = decltype(kc)::value;
            if constexpr (NS <= tn_max<S, Q, KK>()) {
                // the rho-writing variant (the adjoint's recompute) is a kernel of
                // its own, so that the forward kernels carry none of its registers
                if (p.rho_out != nullptr) {
                    if (vec) hipLaunchKernelGGL((k_stepn<S, Q, KK, true, NS, true>), grid, dim3(kT2Block), 0, s, p);
                    else hipLaunchKernelGGL((k_stepn<S, Q, KK, false, NS, true>), grid, dim3(kT2Block), 0, s, p);
                } else {
                    if (vec) hipLaunchKernelGGL((k_stepn<S, Q, KK, true, NS, false>), grid, dim3(kT2Block), 0, s, p);
                    else hipLaunchKernelGGL((k_stepn<S, Q, KK, false, NS, false>), grid, dim3(kT2Block), 0, s, p);
                }
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        };
        return kind == 1 ? launch(std::integral_constant<int, 1>())
             : kind == 2 ? launch(std::integral_constant<int, 2>()) : launch(std::integral_constant<int, 0>());
    });
}

// The batched NS-step launch for storage S and lattice Q.
template <typename S, int Q>
hipError_t stepn_batch_launch(const BatchParams &bp, int ns, int64_t nwaves, hipStream_t s) {
    const dim3 grid((unsigned)((nwaves + kT2Block / 64 - 1) / (kT2Block / 64)));
    const int kind = step_kind(bp.coll);
    return by_steps<S, Q>(ns, [&](auto nc) {
        constexpr int NS = decltype(nc)::value;
        auto launch = [&](auto kc) {
            constexpr int KK = decltype(kc)::value;
            if constexpr (NS <= tn_max<S, Q, KK>()) {
                hipLaunchKernelGGL((k_stepn_batch<S, Q, KK, NS>), grid, dim3(kT2Block), 0, s, bp);
                return hipGetLastError();
            }
            return hipErrorInvalidValue;
        };
        return kind == 1 ? launch(std::integral_constant<int, 1>())
             : kind == 2 ? launch(std::integral_constant<int, 2>()) : launch(std::integral_constant<int, 0>());
    });
}

template <typename S, int Q>
hipError_t stepn_march_batch_launch(const BatchParams &bp, int64_t nwaves, hipStream_t s) {
    const dim3 grid((unsigned)((nwaves + march_block<S>() / 64 - 1) / (march_block<S>() / 64)));
    const int kind = step_kind(bp.coll);
    auto launch = [&](auto kc) {
        constexpr int KK = decltype(kc)::value, MN = march_steps<S, Q, KK>();
        if constexpr (MN > 0) {
            hipLaunchKernelGGL((k_stepn_march_batch<S, Q, KK, MN>), grid, dim3(march_block<S>()), 0, s, bp,
                               (const StepParams *)bp.img);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    };
    return kind == 1 ? launch(std::integral_constant<int, 1>())
         : kind == 2 ? launch(std::integral_constant<int, 2>()) : launch(std::integral_constant<int, 0>());
}

template <typename S, int Q>
int64_t march_waves_of(int kind, int32_t nx, int32_t ny) {
    auto waves = [&](auto kc) -> int64_t {
        constexpr int KK = decltype(kc)::value, MN = march_steps<S, Q, KK>();
        if constexpr (MN > 0) {
            if (!march_ok<S, Q, KK, MN>(nx, ny)) return 0;
            return march_waves<S, Q, KK, MN>(nx, ny);
        }
        return 0;
    };
    return kind == 1 ? waves(std::integral_constant<int, 1>())
         : kind == 2 ? waves(std::integral_constant<int, 2>()) : waves(std::integral_constant<int, 0>());
}

}  // namespace

// One source per storage format and lattice instantiates the kernels with
// LBW_BLOCKED_UNIT; lb_blocked.hip validates and dispatches to them.
#define LBW_BLOCKED_UNIT(SS, QQ, NAME)                                                              \
    hipError_t launch_stepn_##NAME(const StepParams &p, int ns, hipStream_t s) {                    \
        return stepn_launch<SS, QQ>(p, ns, s);                                                      \
    }                                                                                               \
    int march_steps_##NAME(int kind, int32_t nx, int32_t ny, bool pref) {                           \
        return march_grid<SS, QQ>(kind, nx, ny, pref);                                              \
    }                                                                                               \
    int64_t march_min_waves_##NAME(int kind) {                                                      \
        return march_min_waves_of<SS, QQ>(kind);                                                    \
    }                                                                                               \
    hipError_t launch_stepn_march_batch_##NAME(const BatchParams &bp, int64_t nwaves, hipStream_t s) {   \
        return stepn_march_batch_launch<SS, QQ>(bp, nwaves, s);                                     \
    }                                                                                               \
    int64_t march_waves_##NAME(int kind, int32_t nx, int32_t ny) {                                  \
        return march_waves_of<SS, QQ>(kind, nx, ny);                                                \
    }                                                                                               \
    hipError_t launch_stepn_batch_##NAME(const BatchParams &bp, int ns, int64_t nwaves, hipStream_t s) { \
        return stepn_batch_launch<SS, QQ>(bp, ns, nwaves, s);                                       \
    }

#define LBW_BLOCKED_DECL(NAME)                                                                      \
    hipError_t launch_stepn_##NAME(const StepParams &p, int ns, hipStream_t s);                     \
    int march_steps_##NAME(int kind, int32_t nx, int32_t ny, bool pref);                            \
    int64_t march_min_waves_##NAME(int kind);                                                       \
    hipError_t launch_stepn_batch_##NAME(const BatchParams &bp, int ns, int64_t nwaves, hipStream_t s); \
    hipError_t launch_stepn_march_batch_##NAME(const BatchParams &bp, int64_t nwaves, hipStream_t s);   \
    int64_t march_waves_##NAME(int kind, int32_t nx, int32_t ny);
LBW_BLOCKED_DECL(f32_q5)
LBW_BLOCKED_DECL(f32_q9)
LBW_BLOCKED_DECL(f64_q5)
LBW_BLOCKED_DECL(f64_q9)
LBW_BLOCKED_DECL(f16_q5)
#undef LBW_BLOCKED_DECL

}  // namespace lbw
