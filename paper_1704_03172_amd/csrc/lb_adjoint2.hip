// lb_adjoint2.hip -- several backward steps of the discrete adjoint per
// launch (steps n, n-1, .., n-NS+1 of the sweep in lb_adjoint), with the strip
// and segment decomposition of the blocked forward kernel (lb_blocked.h): a
// wavefront loads the rows of lambda(n+1) of its segment plus NS halo rows on
// each side, and stage s (1..NS) computes lambda(n-s+1) on the segment plus
// NS - s halo rows on each side (receiver residuals included, as the later
// stages read them); the last stage stores its own rows.  The FP64 gradient
// of the owned nodes is read once, takes the terms of time n, then n-1, ...
// (the order of one-step launches) and is written once.  Per node the
// arithmetic is adjoint_node (lb_node.h), as in the one-step kernel, so the
// gradient is the same bits; lambda crosses HBM once per NS steps.
#include "lb_blocked.h"

namespace lbw {
namespace {

// Most backward steps per launch, and rows per segment for NS steps (the
// halo rows of each side are computed more than once).  D2Q5 at 2048^2
// (FP32, per 3000-step shot): two steps 89.0 ms, three 71.7 ms (161 VGPRs,
// three waves per SIMD), four 78.1 ms (193 VGPRs, two waves).
template <typename T, int Q>
constexpr int adjn_max() { return Q == 5 ? 3 : 2; }
template <typename T, int Q, int NS>
constexpr int adjn_rows() { return Q == 5 ? 4 : 2; }

// mu_i(x) = lambda_i(n+1)(x + c_i): the transpose of the pull, from the row
// below for c_y = +1 (D), above for c_y = -1 (U), and the lane to the right
// (x + 1) or left (x - 1) along x.
template <typename T, int Q, int V>
__device__ inline void pull_back_row(const T (&U)[Q][V], const T (&C)[Q][V], const T (&D)[Q][V], T (&g)[Q][V]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T r[V];
#pragma unroll
        for (int j = 0; j < V; ++j) r[j] = cyv<Q>(i) > 0 ? D[i][j] : cyv<Q>(i) < 0 ? U[i][j] : C[i][j];
        if (cxv<Q>(i) > 0) {          // from x + 1
            const T rr = from_upper(r[0]);
#pragma unroll
            for (int j = 0; j < V - 1; ++j) g[i][j] = r[j + 1];
            g[i][V - 1] = rr;
        } else if (cxv<Q>(i) < 0) {   // from x - 1
            const T l = from_lower(r[V - 1]);
#pragma unroll
            for (int j = V - 1; j > 0; --j) g[i][j] = r[j - 1];
            g[i][0] = l;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) g[i][j] = r[j];
        }
    }
}

template <typename T, int Q, int KIND, bool VEC, int NS>
__device__ __attribute__((always_inline)) inline void adjn_wave(const AdjointParams &p, int wave) {
    constexpr int V = Tb<T>::V, H = Tb<T>::H, OW = Tb<T>::OW, LY = adjn_rows<T, Q, NS>(), K = LY + 2 * NS;
    static_assert(H * V >= NS, "the strip halo must cover one column per step");
    static_assert(K - 2 <= 64, "the receiver row table of a segment is held one row per lane");
    const int nx = p.nx, ny = p.ny;
    const int nstrip = (nx + OW - 1) / OW;
    const int nseg = (ny + LY - 1) / LY;
    if ((int64_t)wave >= (int64_t)nstrip * nseg) return;   // whole waves
    const int lane = threadIdx.x & 63;
    const int sx = wave % nstrip, sy = wave / nstrip;
    const int xl = sx * OW - H * V + lane * V;
    const int y0 = sy * LY, y1 = min(y0 + LY, ny);
    int xw[V], dxw[V];
    bool own[V];
    const bool own_lane = lane >= H && lane < 64 - H;
    // whether any column of the strip lies within the sponge width of a side
    // edge: else the sponge depends on the row alone
    const int L = p.sponge_width;
    const bool strip_sponge = sx * OW - H * V < L || sx * OW - H * V + 64 * V - 1 >= nx - L;
#pragma unroll
    for (int j = 0; j < V; ++j) {
        xw[j] = wrapi(xl + j, nx);
        own[j] = own_lane && xl + j < nx;
        dxw[j] = min(xw[j], nx - 1 - xw[j]);
    }
    const int xv = xw[0];
    // receiver rows of walk rows 1 .. K-2 (grid rows y0-NS+1 .. y0+LY+NS-2):
    // lane k holds the CSR range of walk row k + 1
    int rb_l = 0, re_l = 0;
    if (p.rec.row_ptr != nullptr && lane < (y1 - y0) + 2 * NS - 2) {
        const int w = wrapi(y0 - NS + 1 + lane, ny);
        rb_l = p.rec.row_ptr[w];
        re_l = p.rec.row_ptr[w + 1];
    }
    int wr = wrapi(y0 - NS, ny);
    int wrow[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wrow[k] = wr;
        wr = wr + 1 == ny ? 0 : wr + 1;
    }
    const T *ln = reinterpret_cast<const T *>(p.lam_next);
    const T *c2 = reinterpret_cast<const T *>(p.c2);
    // L0: lambda(n+1); Ls: lambda(n-s+1) of stage s (the last stage stores)
    T L0[K][Q][V], L1[K][Q][V], L2[K][Q][V], L3[K][Q][V], C[K][V];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t ro = (int64_t)wrow[k] * nx;
        if (k < 2 * NS || k >= K - 2 * NS) load_row2<VEC, 0, true, T, T, Q, V>(ln, p.pstride, ro, xv, xw, L0[k]);
        else load_row2<VEC, 0, false, T, T, Q, V>(ln, p.pstride, ro, xv, xw, L0[k]);
        if (k >= 1 && k <= K - 2) load_c2row<VEC, true, T, V>(c2, ro, xv, xw, C[k]);
    }
    // rho of times n .. n-NS+1 and the FP64 gradient at the owned nodes
    T R[NS][LY][V];
    double G[LY][V];
#pragma unroll
    for (int r = 0; r < LY; ++r) {
        const int gm = min(y0 + r, y1 - 1);   // rows past a short last segment repeat its last row (unused)
        const int64_t ro = (int64_t)gm * nx;
#pragma unroll
        for (int s = 0; s < NS; ++s)
            load_c2row<VEC, false, T, V>(reinterpret_cast<const T *>(p.rho) - s * p.rho_back, ro, xv, xw, R[s][r]);
#pragma unroll
        for (int j = 0; j < V; ++j) G[r][j] = own[j] ? p.grad[ro + xw[j]] : 0.0;
    }

    // step st (1: time n, 2: time n-1, ..) at walk row m (grid row y0 - NS + m)
    auto stage = [&](auto stc, auto mc) __attribute__((always_inline)) {
        constexpr int st = decltype(stc)::value;
        constexpr int m = decltype(mc)::value;
        const int gm = y0 - NS + m;
        const bool owned_row = gm >= y0 && gm < y1;
        if (st == NS && !owned_row) return;
        const int wm = wrow[m];
        auto &A = pick4<st - 1>(L0, L1, L2, L3);
        T mu[Q][V];
        pull_back_row<T, Q, V>(A[m - 1], A[m], A[m + 1], mu);
        // the sponge factor (1 - sigma) on mu: one wave-uniform test per row,
        // the per-node multiply (as adjoint_node's) only in rows that reach it
        const int dy = min(wm, ny - 1 - wm);
        if (strip_sponge || dy < L) {
            asm volatile("");
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int d = min(dxw[j], dy);
                if (d < L) {
                    asm volatile("");
                    T mj[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) mj[i] = mu[i][j];
                    apply_sponge<T, Q>(d, L, p.sponge_smax, mj);
#pragma unroll
                    for (int i = 0; i < Q; ++i) mu[i][j] = mj[i];
                }
            }
        }
        const int rb = __builtin_amdgcn_readlane(rb_l, m - 1), re = __builtin_amdgcn_readlane(re_l, m - 1);
        const int64_t col = p.rec.col - (st - 1);
        const double sn = p.s_back[st - 1];
        const bool initial = p.initial_stage == st;
        T lo[Q][V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            T muj[Q], lam[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) muj[i] = mu[i][j];
            T rho = T(0);   // rho only feeds the gradient, kept at the owned rows
            if constexpr (m >= NS && m - NS < LY) {
                if (owned_row) rho = R[st - 1][m - NS][j];
            }
            const double g = adjoint_node<T, Q, KIND>(p, muj, C[m][j], rho, xw[j], wm, min(dxw[j], dy), rb, re, col, sn,
                                                      initial, lam, false);
            if constexpr (m >= NS && m - NS < LY) {
                if (owned_row && own[j]) G[m - NS][j] += g;
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) lo[i][j] = lam[i];
        }
        if constexpr (st < NS) {
            auto &B = pick4<st>(L0, L1, L2, L3);
#pragma unroll
            for (int i = 0; i < Q; ++i)
#pragma unroll
                for (int j = 0; j < V; ++j) B[m][i][j] = lo[i][j];
        } else {
            T *out = reinterpret_cast<T *>(p.lam);
            const int64_t ro = (int64_t)gm * nx;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                T *r = out + i * p.pstride + ro;
                if constexpr (VEC && V > 1) {
                    if (own[0]) {
                        typedef typename LaneVec<V, T>::type vt;
                        vt t;
#pragma unroll
                        for (int j = 0; j < V; ++j) t[j] = lo[i][j];
                        __builtin_nontemporal_store(t, at_lane<vt>(r, xv));
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < V; ++j)
                        if (own[j]) __builtin_nontemporal_store(lo[i][j], r + xw[j]);
                }
            }
        }
    };
    // walk index k: stage st at row k - st, within the rows st .. K-1-st it
    // computes (stage st - 1 produced row k - st + 1 at this same index)
    static_for<2, K + NS - 1>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        static_for<1, NS + 1>([&](auto stc) __attribute__((always_inline)) {
            constexpr int st = decltype(stc)::value;
            if constexpr (k - st >= st && k - st <= K - 1 - st)
                stage(stc, std::integral_constant<int, k - st>{});
        });
    });
#pragma unroll
    for (int r = 0; r < LY; ++r) {
        if (y0 + r >= y1) continue;
        const int64_t ro = (int64_t)(y0 + r) * nx;
#pragma unroll
        for (int j = 0; j < V; ++j)
            if (own[j]) p.grad[ro + xw[j]] = G[r][j];
    }
}

template <typename T, int Q, int KIND, bool VEC, int NS>
__global__ __launch_bounds__(kT2Block) void k_adjointn(AdjointParams p) {
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    adjn_wave<T, Q, KIND, VEC, NS>(p, xcd_block() * (kT2Block / 64) + wib);
}

template <typename T, int Q, int NS>
hipError_t adjointn_launch(const AdjointParams &p, hipStream_t s) {
    constexpr int OW = Tb<T>::OW, LY = adjn_rows<T, Q, NS>();
    const int64_t waves = (int64_t)((p.nx + OW - 1) / OW) * ((p.ny + LY - 1) / LY);
    const dim3 grid((unsigned)((waves + kT2Block / 64 - 1) / (kT2Block / 64)));
    const bool vec = p.nx % Tb<T>::V == 0, mrt = p.coll.kind == 1;
    if (mrt) {
        if (vec) hipLaunchKernelGGL((k_adjointn<T, Q, 1, true, NS>), grid, dim3(kT2Block), 0, s, p);
        else hipLaunchKernelGGL((k_adjointn<T, Q, 1, false, NS>), grid, dim3(kT2Block), 0, s, p);
    } else {
        if (vec) hipLaunchKernelGGL((k_adjointn<T, Q, 0, true, NS>), grid, dim3(kT2Block), 0, s, p);
        else hipLaunchKernelGGL((k_adjointn<T, Q, 0, false, NS>), grid, dim3(kT2Block), 0, s, p);
    }
    return hipGetLastError();
}

template <typename T, int Q>
hipError_t adjointn_by_steps(const AdjointParams &p, int ns, hipStream_t s) {
    if constexpr (adjn_max<T, Q>() >= 4) if (ns == 4) return adjointn_launch<T, Q, 4>(p, s);
    if constexpr (adjn_max<T, Q>() >= 3) if (ns == 3) return adjointn_launch<T, Q, 3>(p, s);
    if (ns == 2) return adjointn_launch<T, Q, 2>(p, s);
    return hipErrorInvalidValue;
}

}  // namespace

int adjointn_max(int storage, int q) {
    if (storage == ST_F64) return q == 5 ? adjn_max<double, 5>() : adjn_max<double, 9>();
    return q == 5 ? adjn_max<float, 5>() : adjn_max<float, 9>();
}

hipError_t launch_adjointn(int storage, const AdjointParams &p, int ns, hipStream_t s) {
    if (p.nx < 1 || p.ny < 1 || p.terminal || p.rec.col < ns - 1 || (p.q != 5 && p.q != 9) || ns < 2 ||
        ns > adjointn_max(storage, p.q) || p.rho_back <= 0)
        return hipErrorInvalidValue;
    if (storage == ST_F64) return p.q == 5 ? adjointn_by_steps<double, 5>(p, ns, s) : adjointn_by_steps<double, 9>(p, ns, s);
    return p.q == 5 ? adjointn_by_steps<float, 5>(p, ns, s) : adjointn_by_steps<float, 9>(p, ns, s);
}

}  // namespace lbw
