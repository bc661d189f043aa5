// lb_node.h -- the per-node arithmetic of the linear LB step shared by every
// step kernel (one step per launch, several steps per launch, the batched
// executor, the refinement interface): lattice tables, storage traits, the
// collision, source, sponge and receiver recording of one node.  Device
// code only; included by the kernel sources (not part of the public
// interface).
#pragma once

#include "lb_internal.h"

#include <hip/hip_fp16.h>

// No automatic a*b+c contraction in this file: where the compiler forms fused
// multiply-adds depends on the surrounding code, so the same per-node
// arithmetic inlined into different kernels (one step per launch, several
// steps per launch, the batched executor) could round differently.  The fused
// multiply-adds of the collision are written out (fmaT) instead.
#pragma clang fp contract(off)

namespace lbw {
namespace {

// ---- lattice tables (velocity order of Appendix A) -----------------------
template <int Q>
__host__ __device__ constexpr int cxv(int i) {
    return Q == 5 ? (i == 1 ? 1 : i == 3 ? -1 : 0)
                  : (i == 1 || i == 5 || i == 8 ? 1 : i == 3 || i == 6 || i == 7 ? -1 : 0);
}
template <int Q>
__host__ __device__ constexpr int cyv(int i) {
    return Q == 5 ? (i == 2 ? 1 : i == 4 ? -1 : 0)
                  : (i == 2 || i == 5 || i == 6 ? 1 : i == 4 || i == 7 || i == 8 ? -1 : 0);
}

// Rows of the moment matrix of Appendix A (non-conserved rows only are
// used: D2Q5 k = 3 (e), 4 (pxx); D2Q9 k = 3 (e), 4 (pxx), 5 (eps),
// 6 (qx), 7 (qy), 8 (pxy)).
template <int Q>
__host__ __device__ constexpr int mrow(int k, int i) {
    if (Q == 5) {
        if (k == 3) return i == 0 ? -4 : 1;
        if (k == 4) return i == 1 || i == 3 ? 1 : (i == 2 || i == 4 ? -1 : 0);
        return 0;
    }
    switch (k) {
    case 3: return i == 0 ? -4 : (i <= 4 ? -1 : 2);
    case 4: return i == 1 || i == 3 ? 1 : (i == 2 || i == 4 ? -1 : 0);
    case 5: return i == 0 ? 4 : (i <= 4 ? -2 : 1);
    case 6: return i == 1 ? -2 : i == 3 ? 2 : (i == 5 || i == 8 ? 1 : (i == 6 || i == 7 ? -1 : 0));
    case 7: return i == 2 ? -2 : i == 4 ? 2 : (i == 5 || i == 6 ? 1 : (i == 7 || i == 8 ? -1 : 0));
    case 8: return i == 5 || i == 7 ? 1 : (i == 6 || i == 8 ? -1 : 0);
    default: return 0;
    }
}

// ---- storage traits -------------------------------------------------------
template <typename S> struct Tr;
template <> struct Tr<float> {
    using T = float;
    static constexpr int V = 4;
    typedef float vec __attribute__((ext_vector_type(4), aligned(4)));
};
template <> struct Tr<double> {
    using T = double;
    static constexpr int V = 2;
    typedef double vec __attribute__((ext_vector_type(2), aligned(8)));
};
template <> struct Tr<_Float16> {
    using T = float;
    static constexpr int V = 8;
    typedef _Float16 vec __attribute__((ext_vector_type(8), aligned(2)));
};

// Conversion of a computed value to the storage format.  For FP16 storage
// the value is first materialised in FP32 (the empty asm is a value barrier):
// otherwise the compiler may fold the last multiply and the conversion into
// one mixed-precision FMA (a single rounding) in some kernels and not in
// others, and a state stored by different kernels would differ in its bits.
template <typename S, typename T>
__device__ inline S to_store(T v) {
    if constexpr (sizeof(S) < sizeof(T)) asm volatile("" : "+v"(v));
    return S(v);
}

template <typename T>
__device__ inline T fmaT(T a, T b, T c) {
    if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
    else return __builtin_fmaf(a, b, c);
}

__device__ inline int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// V consecutive elements starting at x = xs of one row, periodic in x.
template <typename S, int V>
__device__ inline void load_x(const S *__restrict__ row, int xs, int nx, S (&v)[V]) {
    if (V > 1 && xs >= 0 && xs + V <= nx) {
        typedef typename Tr<S>::vec vt;
        vt t = __builtin_nontemporal_load(reinterpret_cast<const vt *>(row + xs));
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = t[j];
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = row[wrapi(xs + j, nx)];
    }
}

template <typename S, int V>
__device__ inline void store_x(S *__restrict__ row, int x0, int nx, const S (&v)[V]) {
    if (V > 1 && x0 + V <= nx) {
        typedef typename Tr<S>::vec vt;
        vt t;
#pragma unroll
        for (int j = 0; j < V; ++j) t[j] = v[j];
        __builtin_nontemporal_store(t, reinterpret_cast<vt *>(row + x0));
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
            if (x0 + j < nx) row[x0 + j] = v[j];
    }
}

// ---- the per-node update ---------------------------------------------------
// Lattice weights from c^2 (Sec. II C): D2Q5 w_i = c^2/2 for movers,
// w0 = 1 - 2 c^2; D2Q9 w1 = c^2 kw (kw = 1 / (2 + 4r)), w5 = r w1,
// w0 = 1 - 4 w1 - 4 w5.
// (1 - 4 w1 as one fused multiply-add: 4 w1 is exact, so this is the
// rounding of 1 - 4 w1 either way.)
template <typename T, int Q>
__device__ inline void weights(T c2, const Collision &c, T (&w)[Q]) {
    if (Q == 5) {
        T w1 = T(0.5) * c2;
        w[0] = fmaT(T(-4), w1, T(1));
#pragma unroll
        for (int i = 1; i < Q; ++i) w[i] = w1;
    } else {
        T w1 = c2 * T(c.kw);
        T w5 = w1 * T(c.ratio);
        w[0] = fmaT(T(-4), w5, fmaT(T(-4), w1, T(1)));
#pragma unroll
        for (int i = 1; i < Q; ++i) w[i] = i <= 4 ? w1 : w5;
    }
}

// c . J for the velocity (cx, cy) with components 0, +-1 resolved at compile
// time (no multiplications by 0 or 1).
template <typename T>
__device__ inline T cdot(int cx, int cy, T jx, T jy) {
    const T ax = cx > 0 ? jx : -jx, ay = cy > 0 ? jy : -jy;
    return cx != 0 ? (cy != 0 ? ax + ay : ax) : (cy != 0 ? ay : T(0));
}

// D2Q9: the rest population's equilibrium w0 rho written as rho minus the
// movers' rounded rho-parts, rho - 4 (w1 rho) - 4 (w5 rho), so that the
// equilibrium holds the mass rho up to roundings that change with rho.  With
// w0 rho, the rounding of the per-node constant w0 = 1 - 4 w1 - 4 w5 is a
// fixed per-node mass source proportional to rho, the same every step, and
// the error it leaves in FP32 grows with the run (an FP32 emulation of the
// 256^2 layered workload: 3.7e-5 of rho after 1000 steps of D2Q9 BGK,
// 6.8e-6 with this form and the momentum-exact kax, kdg; MRT 6.4e-6 ->
// 4.1e-6).  The value is the same real number.
// D2Q5 keeps w0 rho (its movers' weight c^2 / 2 is exact).
template <typename T, int Q>
__device__ inline T geq_rest(const T (&w)[Q], T rho) {
    if constexpr (Q == 9) return fmaT(T(-4), w[5] * rho, fmaT(T(-4), w[1] * rho, rho));
    else return w[0] * rho;
}

// Collision of one node: out = g - C (g - g^eq) with the linear equilibrium
// g^eq_i = w_i rho + (w_i / c^2)(c_i . J); BGK C = omega I (KIND 0), MRT
// C = M^-1 S M applied through the non-conserved moments only (KIND 1).
// KIND 2 is BGK at omega = 2 (tau = 1/2, the non-dissipative case), where
// g - 2 (g - g^eq) is 2 g^eq - g: one rounding less and fewer operations.
template <typename T, int Q, int KIND>
__device__ inline void collide(const T (&g)[Q], T c2, const Collision &c, T (&out)[Q], T (&w)[Q]) {
    // moments, each sum started from its first term (0 + x is not x for
    // x = -0, so a 0 start would cost an addition the compiler must keep)
    T rho = g[0], jx = T(0), jy = T(0);
    bool hx = false, hy = false;
#pragma unroll
    for (int i = 1; i < Q; ++i) rho += g[i];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cxv<Q>(i) != 0) {
            const T v = cxv<Q>(i) > 0 ? g[i] : -g[i];
            jx = hx ? jx + v : v;
            hx = true;
        }
        if (cyv<Q>(i) != 0) {
            const T v = cyv<Q>(i) > 0 ? g[i] : -g[i];
            jy = hy ? jy + v : v;
            hy = true;
        }
    }
    weights<T, Q>(c2, c, w);
    if constexpr (KIND == 2) {
        if constexpr (Q == 5) {
            // D2Q5: 2 w_i = c^2 and 2 (w_i / c^2)(c_i . J) = c_i . J for the
            // movers (both exact), 2 w_0 = 2 - 4 c^2
            out[0] = fmaT(fmaT(T(-4), c2, T(2)), rho, -g[0]);
#pragma unroll
            for (int i = 1; i < Q; ++i) out[i] = fmaT(c2, rho, cdot<T>(cxv<Q>(i), cyv<Q>(i), jx, jy)) - g[i];
        } else {
            out[0] = fmaT(T(2), geq_rest<T, Q>(w, rho), -g[0]);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int cx = cxv<Q>(i), cy = cyv<Q>(i);
                const bool pos = cx > 0 || (cx == 0 && cy > 0);
                const T kj = i <= 4 ? T(c.kax) : T(c.kdg);
                const T kc = kj * cdot<T>(pos ? cx : -cx, pos ? cy : -cy, jx, jy);
                out[i] = fmaT(T(2), fmaT(w[i], rho, pos ? kc : -kc), -g[i]);
            }
        }
        return;
    }
    T d[Q];
    d[0] = g[0] - geq_rest<T, Q>(w, rho);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        // (w_i / c^2)(c_i . J): opposite velocities share one product
        // (k (-a) is -(k a) exactly), taken for the one whose first nonzero
        // component is positive
        const int cx = cxv<Q>(i), cy = cyv<Q>(i);
        const bool pos = cx > 0 || (cx == 0 && cy > 0);
        const T kj = Q == 5 ? T(0.5) : (i <= 4 ? T(c.kax) : T(c.kdg));
        const T kc = kj * cdot<T>(pos ? cx : -cx, pos ? cy : -cy, jx, jy);
        const T geq = fmaT(w[i], rho, pos ? kc : -kc);
        d[i] = g[i] - geq;
    }
    if (KIND == 0) {
        const T om = T(c.omega);
#pragma unroll
        for (int i = 0; i < Q; ++i) out[i] = fmaT(-om, d[i], g[i]);
    } else {
        T r[9];
#pragma unroll
        for (int k = 3; k < Q; ++k) {
            T m = T(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int a = mrow<Q>(k, i);
                if (a != 0) m += T(a) * d[i];
            }
            r[k] = T(c.srate[k]) * m;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            T acc = T(0);
#pragma unroll
            for (int k = 3; k < Q; ++k) {
                int a = mrow<Q>(k, i);
                if (a != 0) acc += T(a) * r[k];
            }
            out[i] = g[i] - acc;
        }
    }
}

// Sponge factor of a node at distance d (in nodes) from the nearest edge.
template <typename T>
__device__ inline T sponge_at(int d, int L, double smax) {
    if (L <= 0 || d >= L) return T(1);
    T f = T(L - d) / T(L);
    return T(1) - T(smax) * f * f;
}

__device__ inline int edge_dist(int x, int y, int nx, int ny) { return min(min(x, y), min(nx - 1 - x, ny - 1 - y)); }

template <typename T>
__device__ inline T sponge_factor(int x, int y, int nx, int ny, int L, double smax) {
    return sponge_at<T>(edge_dist(x, y, nx, ny), L, smax);
}

template <typename T>
__device__ inline void write_fields(const Receivers &rc, int slot, T rho, T jx, T jy, T c2) {
    T *tr = reinterpret_cast<T *>(rc.traces);
    int f = 0;
    const int64_t plane = (int64_t)rc.nslots * rc.cap;
    const int64_t base = (int64_t)slot * rc.cap + rc.col;
    if (rc.what & 1u) { tr[f * plane + base] = c2 * rho; ++f; }
    if (rc.what & 2u) { tr[f * plane + base] = rho; ++f; }
    if (rc.what & 4u) { tr[f * plane + base] = jx; ++f; }
    if (rc.what & 8u) { tr[f * plane + base] = jy; ++f; }
}

// The params of a launch replayed from a captured graph with its times made
// absolute: the launch holds them relative to the chunk's first time, which
// with the chunk's source amplitudes sits in the chunk table (GraphTab).
// The graph entry kernels run the ordinary bodies on this copy, so the
// kernels of eager launches carry nothing of it.
__device__ inline StepParams graph_params(const StepParams &p) {
    StepParams q = p;
    const GraphTab *g = p.gtab;
    const double *s = g->s + p.goff;
    q.s_n = s[0];
    q.s_n2 = s[1];
    q.s_n3 = s[2];
    q.s_n4 = s[3];
    q.rec.col += g->t0;
    q.gtab = nullptr;
    return q;
}

// Receivers at node x of a row whose CSR entries are [rb, re): record the
// fields of the pre-collision state g.
template <typename T, int Q>
__device__ inline void record_node(const Receivers &rc, int rb, int re, int x, const T (&g)[Q], T c2) {
    T rho = T(0), jx = T(0), jy = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += g[i];
        jx += T(cxv<Q>(i)) * g[i];
        jy += T(cyv<Q>(i)) * g[i];
    }
    int lo = rb, hi = re;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rc.xs[mid] < x) lo = mid + 1; else hi = mid;
    }
    for (; lo < re && rc.xs[lo] == x; ++lo)
        write_fields<T>(rc, rc.slot[lo], rho, jx, jy, c2);
}

// The point source w_i S added to a post-collision state (Sec. II D).
template <typename T, int Q>
__device__ inline void add_source(const T (&w)[Q], double s_n, T (&gs)[Q]) {
    const T sn = T(s_n);
#pragma unroll
    for (int i = 0; i < Q; ++i) gs[i] += w[i] * sn;
}

// The sponge factor of a node at distance d < L from the nearest edge
// applied to its post-collision state.
template <typename T, int Q>
__device__ inline void apply_sponge(int d, int L, double smax, T (&gs)[Q]) {
    const T sf = sponge_at<T>(d, L, smax);
#pragma unroll
    for (int i = 0; i < Q; ++i) gs[i] = gs[i] * sf;
}

// Post-collision state of node (x, y): collision, source w_i S at the source
// node, sponge (dedge: the node's distance to the nearest grid edge).
// maybe_sponge: wave-uniform; false when no node of the wave's current row
// lies in the sponge (dedge is then not looked at).
template <typename T, int Q, int KIND>
__device__ inline void post_node(const StepParams &p, const T (&g)[Q], T c2, int x, int y, int dedge, double s_n,
                                 T (&out)[Q], bool maybe_sponge = true) {
    T gs[Q], w[Q];
    collide<T, Q, KIND>(g, c2, p.coll, gs, w);
    if (y == p.src_y) {   // uniform over a row: only the source row tests x
        // (the empty asm keeps this a branch: otherwise the compiler turns
        // the injection into selects evaluated at every node)
        asm volatile("");
        if (x == p.src_x) add_source<T, Q>(w, s_n, gs);
    }
    // sponge: outside it the factor is 1 and g * 1 = g, so only nodes inside
    // multiply (a branch, kept by the empty asm, rather than selects at
    // every node)
    if (maybe_sponge && dedge < p.sponge_width) {
        asm volatile("");
        apply_sponge<T, Q>(dedge, p.sponge_width, p.sponge_smax, gs);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i] = gs[i];
}

// One node of the backward step of time n (the discrete adjoint; see
// k_adjoint): mu is lambda(n+1) pulled back to the node (before the sponge),
// dedge the node's distance to the nearest edge, [rb, re) its row's
// receiver entries (empty: none), col = n for the residuals, s_n = S(n),
// initial: n = 0.  Writes lambda(n) and returns the node's gradient term of
// time n (FP64).  Shared by the one-step and the two-step adjoint kernels,
// so both give the same bits.
template <typename T, int Q, int KIND>
__device__ inline double adjoint_node(const AdjointParams &p, const T (&mu)[Q], T c2, T rho, int x, int y, int dedge,
                                      int rb, int re, int64_t col, double s_n, bool initial, T (&lam)[Q],
                                      bool sponge = true) {
    const T *res = reinterpret_cast<const T *>(p.rec.traces);
    T m[Q], nu[Q], w[Q];
    // (1 - sigma) P^T lambda: outside the sponge the factor is 1 and
    // mu * 1 = mu, so only nodes inside it multiply (sponge false: the
    // caller has applied the factor to mu already)
    if (sponge && dedge < p.sponge_width) {
        asm volatile("");
        const T sf = sponge_at<T>(dedge, p.sponge_width, p.sponge_smax);
#pragma unroll
        for (int i = 0; i < Q; ++i) m[i] = mu[i] * sf;
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) m[i] = mu[i];
    }
    if (KIND == 0) {
#pragma unroll
        for (int i = 0; i < Q; ++i) nu[i] = T(p.coll.omega) * m[i];
    } else {
        T r[9];
#pragma unroll
        for (int k = 3; k < Q; ++k) {
            T a = T(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int c = mrow<Q>(k, i);
                if (c != 0) a += T(c) * m[i];
            }
            r[k] = T(p.coll.srate[k]) * a;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            T a = T(0);
#pragma unroll
            for (int k = 3; k < Q; ++k) {
                const int c = mrow<Q>(k, i);
                if (c != 0) a += T(c) * r[k];
            }
            nu[i] = a;
        }
    }
    double gacc = 0.0;
    {
        double dn = 0.0, dm = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            dn += p.dw[i] * double(nu[i]);
            dm += p.dw[i] * double(m[i]);
        }
        gacc += double(rho) * dn;
        if (y == p.src_y) {   // uniform over a row: only the source row tests x
            asm volatile("");
            if (x == p.src_x) gacc += s_n * dm;
        }
    }
    weights<T, Q>(c2, p.coll, w);
    T s0 = T(0), sxv = T(0), syv = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        s0 += w[i] * nu[i];
        const T kj = Q == 5 ? T(0.5) : (i <= 4 ? T(p.coll.kax) : T(p.coll.kdg));
        if (i > 0) {
            sxv += kj * T(cxv<Q>(i)) * nu[i];
            syv += kj * T(cyv<Q>(i)) * nu[i];
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        lam[i] = m[i] - nu[i] + s0 + T(cxv<Q>(i)) * sxv + T(cyv<Q>(i)) * syv;
    if (rb < re) {
        int lo = rb, hi = re;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (p.rec.xs[mid] < x) lo = mid + 1; else hi = mid;
        }
        for (; lo < re && p.rec.xs[lo] == x; ++lo) {
            const T rr = res[(int64_t)p.rec.slot[lo] * p.rec.cap + col];
#pragma unroll
            for (int i = 0; i < Q; ++i) lam[i] += c2 * rr;
            gacc += double(rr) * double(rho);
        }
    }
    if (initial) {
        double dl = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) dl += p.dw[i] * double(lam[i]);
        gacc += double(rho) * dl;
    }
    return gacc;
}

}  // namespace
}  // namespace lbw
