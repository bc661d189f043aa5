// lb_kernels.hip -- gfx950 kernels of the linear lattice Boltzmann scheme
// (arXiv:1704.03172).
//
// Storage: populations structure-of-arrays, pop[i][y][x], x fastest, with a
// stride of pstride elements between populations.  The step kernel keeps the
// post-collision state: launch n reads h(n-1) = post-collision populations of
// time n-1, pulls g_i(x, n) = h_i(x - c_i, n-1) (streaming, eq. BGK-LB lhs,
// periodic wrap), records time n, collides (eq. BGK-LB / eq. MRT-LB around
// eq. linear eqm dist), adds w_i S(n) at the source node (eq. MRT-LB linear
// acoustic), damps in the sponge (Sec. IV) and writes h(n) at the node it
// owns.  Every element of every array is read once and written once per
// step: the kernel is HBM-bound (no data reuse to stage in LDS), so it is
// written as a pure streaming pass with 16-byte vector accesses.
//
// Each thread owns V consecutive x-nodes of one row (V * sizeof(storage) =
// 16 bytes).  Pulls along x are offset by one element; gfx950 accepts
// 4-byte-aligned dwordx4 loads, so the shifted pulls are single vector loads
// except at the periodic seam, which takes an element-wise path.  Population
// and c^2 traffic is single-use, so loads and stores carry the nontemporal
// hint (measured on MI355X: +8-11 % HBM throughput over cached accesses for
// this 11-stream pattern, and +7 % for a plain copy).
#include "lb_internal.h"

#include <algorithm>

#include <hip/hip_fp16.h>

// No automatic a*b+c contraction in this file: where the compiler forms fused
// multiply-adds depends on the surrounding code, so the same per-node
// arithmetic inlined into different kernels (one step per launch, two steps
// per launch, the batched executor) could round differently.  The fused
// multiply-adds of the collision are written out (fmaT) instead.
#pragma clang fp contract(off)

namespace lbw {
namespace {

constexpr int kBlock = 256;       // set-up, field and interface kernels
constexpr int kStepBlock = 128;   // fused step (best of a block-size sweep)

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
// w0 = 1 - 2 c^2; D2Q9 w1 = c^2 kax, w5 = r w1, w0 = 1 - 4 w1 - 4 w5.
template <typename T, int Q>
__device__ inline void weights(T c2, const Collision &c, T (&w)[Q]) {
    if (Q == 5) {
        T w1 = T(0.5) * c2;
        w[0] = T(1) - T(4) * w1;
#pragma unroll
        for (int i = 1; i < Q; ++i) w[i] = w1;
    } else {
        T w1 = c2 * T(c.kax);
        T w5 = w1 * T(c.ratio);
        w[0] = T(1) - T(4) * w1 - T(4) * w5;
#pragma unroll
        for (int i = 1; i < Q; ++i) w[i] = i <= 4 ? w1 : w5;
    }
}

// c_i . J with the lattice velocity's components (0, +-1) resolved at compile
// time (no multiplications by 0 or 1).
template <typename T, int Q>
__device__ inline T cdot(int i, T jx, T jy) {
    const int cx = cxv<Q>(i), cy = cyv<Q>(i);
    const T ax = cx > 0 ? jx : -jx, ay = cy > 0 ? jy : -jy;
    return cx != 0 ? (cy != 0 ? ax + ay : ax) : (cy != 0 ? ay : T(0));
}

// Collision of one node: out = g - C (g - g^eq) with the linear equilibrium
// g^eq_i = w_i rho + (w_i / c^2)(c_i . J); BGK C = omega I, MRT
// C = M^-1 S M applied through the non-conserved moments only.
template <typename T, int Q, int KIND>
__device__ inline void collide(const T (&g)[Q], T c2, const Collision &c, T (&out)[Q], T (&w)[Q]) {
    T rho = T(0), jx = T(0), jy = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        rho += g[i];
        if (cxv<Q>(i) > 0) jx += g[i];
        if (cxv<Q>(i) < 0) jx -= g[i];
        if (cyv<Q>(i) > 0) jy += g[i];
        if (cyv<Q>(i) < 0) jy -= g[i];
    }
    weights<T, Q>(c2, c, w);
    T d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T kj = Q == 5 ? T(0.5) : (i <= 4 ? T(c.kax) : T(c.kdg));
        T cj = cdot<T, Q>(i, jx, jy);
        T geq = fmaT(w[i], rho, i == 0 ? T(0) : kj * cj);
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

// Post-collision state of node (x, y): collision, source w_i S at the source
// node, sponge (dedge: the node's distance to the nearest grid edge).
template <typename T, int Q, int KIND>
__device__ inline void post_node(const StepParams &p, const T (&g)[Q], T c2, int x, int y, int dedge, double s_n,
                                 T (&out)[Q]) {
    T gs[Q], w[Q];
    collide<T, Q, KIND>(g, c2, p.coll, gs, w);
    if (y == p.src_y && x == p.src_x) {
        const T sn = T(s_n);
#pragma unroll
        for (int i = 0; i < Q; ++i) gs[i] += w[i] * sn;
    }
    const T sf = sponge_at<T>(dedge, p.sponge_width, p.sponge_smax);
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i] = gs[i] * sf;
}

// ---- refinement interface (D2Q5, factor 2) -------------------------------------
template <typename S, typename T>
__device__ inline void pre_at(const GridRef &r, int x, int y, T (&g)[5]) {
    const S *pop = reinterpret_cast<const S *>(r.pop);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        int xs = r.pre ? x : wrapi(x - cxv<5>(i), r.nx);
        int ys = r.pre ? y : wrapi(y - cyv<5>(i), r.ny);
        g[i] = T(pop[i * r.pstride + (int64_t)ys * r.nx + xs]);
    }
}

// Snapshot layout (written by the coarse step, see update_tile): top row
// (y = Y0, x = X0-1 .. X0+W+1), bottom row (y = Y0+H), left column (x = X0,
// y = Y0-1 .. Y0+H+1), right column (x = X0+W).

// R_f(g) = g^eq(rho(g), J(g)) + f (g - g^eq) with the weights of the
// receiving node's c^2 (eq. coarse-fine dist connect), then the collision
// (and sponge) of the receiving grid; written as the post-collision state at
// node (x, y) of dst.
template <typename S, int KIND>
__device__ inline void rescale_collide(const InterfaceParams &p, typename Tr<S>::T (&gh)[5], int x, int y,
                                       typename Tr<S>::T (&out)[5]) {
    using T = typename Tr<S>::T;
    const int64_t k = (int64_t)y * p.dst_nx + x;
    const T c2 = reinterpret_cast<const T *>(p.dst_c2)[k];
    T rho = T(0), jx = T(0), jy = T(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        rho += gh[i];
        jx += T(cxv<5>(i)) * gh[i];
        jy += T(cyv<5>(i)) * gh[i];
    }
    T w[5];
    weights<T, 5>(c2, p.coll, w);
    T gr[5];
    const T f = T(p.f);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        T geq = w[i] * rho + (i == 0 ? T(0) : T(0.5) * (T(cxv<5>(i)) * jx + T(cyv<5>(i)) * jy));
        gr[i] = geq + f * (gh[i] - geq);
    }
    collide<T, 5, KIND>(gr, c2, p.coll, out, w);
    const T sf = sponge_factor<T>(x, y, p.dst_nx, p.dst_ny, p.sponge_width, p.sponge_smax);
#pragma unroll
    for (int i = 0; i < 5; ++i) out[i] *= sf;
}

template <typename S, int KIND>
__device__ inline void rescale_collide_store_impl(const InterfaceParams &p, typename Tr<S>::T (&gh)[5], int x, int y) {
    using T = typename Tr<S>::T;
    const int64_t k = (int64_t)y * p.dst_nx + x;
    if (p.field) {   // R_f keeps rho and J: the node's fields are those of gh
        T rho = T(0), jx = T(0), jy = T(0);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            rho += gh[i];
            jx += T(cxv<5>(i)) * gh[i];
            jy += T(cyv<5>(i)) * gh[i];
        }
        const T c2 = reinterpret_cast<const T *>(p.dst_c2)[k];
        T v = p.field == 1u ? c2 * rho : p.field == 2u ? rho : p.field == 4u ? jx : jy;
        reinterpret_cast<T *>(p.field_out)[k] = v;
        return;
    }
    T out[5];
    rescale_collide<S, KIND>(p, gh, x, y, out);
    S *dst = reinterpret_cast<S *>(p.dst);
#pragma unroll
    for (int i = 0; i < 5; ++i) dst[i * p.dst_pstride + k] = to_store<S>(out[i]);
}

// Interpolation stencil of fine outer-ring node (i, j): coincident nodes
// copy the coarse node (weight 1 on entry 1, the other entries repeat it with
// weight 0), mid-edge nodes take the cubic (-1, 9, 9, -1)/16 along their
// edge.  nodes_*: coarse nodes; sidx: their ring-line snapshot entries.
template <typename T>
__device__ inline void ring_stencil(const PatchGeom &g, int i, int j, int (&nodes_x)[4], int (&nodes_y)[4],
                                    int (&sidx)[4], T (&wt)[4]) {
    const int nh = g.W + 3, nv = g.H + 3;
    const bool horiz = (j == 0 || j == g.nyf - 1);
    const int hbase = (j == 0) ? 0 : nh;                 // top / bottom arrays
    const int vbase = 2 * nh + ((i == 0) ? 0 : nv);      // left / right arrays
    if ((i & 1) == 0 && (j & 1) == 0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            nodes_x[s] = g.X0 + i / 2;
            nodes_y[s] = g.Y0 + j / 2;
            wt[s] = s == 1 ? T(1) : T(0);
            sidx[s] = horiz ? hbase + i / 2 + 1 : vbase + j / 2 + 1;
        }
    } else if (i & 1) {
        const int a = g.X0 + (i - 1) / 2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            nodes_x[s] = a - 1 + s;
            nodes_y[s] = g.Y0 + j / 2;
            sidx[s] = hbase + (i - 1) / 2 + s;
        }
        wt[0] = wt[3] = T(-1) / T(16);
        wt[1] = wt[2] = T(9) / T(16);
    } else {
        const int b = g.Y0 + (j - 1) / 2;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            nodes_x[s] = g.X0 + i / 2;
            nodes_y[s] = b - 1 + s;
            sidx[s] = vbase + (j - 1) / 2 + s;
        }
        wt[0] = wt[3] = T(-1) / T(16);
        wt[1] = wt[2] = T(9) / T(16);
    }
}

// Coarse state interpolated to fine outer-ring node (i, j) along the edge;
// in time a_snap * (snapshot of T) + a_now * (coarse now).
template <typename S>
__device__ inline void ring_interp(const InterfaceParams &p, int i, int j, typename Tr<S>::T (&gh)[5]) {
    using T = typename Tr<S>::T;
    const PatchGeom &g = p.g;
    int nodes_x[4], nodes_y[4], sidx[4];
    T wt[4];
    ring_stencil<T>(g, i, j, nodes_x, nodes_y, sidx, wt);
#pragma unroll
    for (int q = 0; q < 5; ++q) gh[q] = T(0);
    const T *snap = reinterpret_cast<const T *>(p.snap);
    const T an = T(p.a_now), as = T(p.a_snap);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (wt[s] == T(0)) continue;
        T gn[5];
        pre_at<S, T>(p.coarse, nodes_x[s], nodes_y[s], gn);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            T v = an * gn[q];
            if (p.a_snap != 0.0) v += as * snap[q * g.nsnap + sidx[s]];
            gh[q] += wt[s] * v;
        }
    }
}

// The outer-ring states of the two fine steps of one coarse step T -> T+2,
// one thread per fine ring node: R_{1/2} of the coarse state interpolated to
// the node, at T+1 (mean of the ring-line snapshot of T and the coarse state
// of T+2) and at T+2, each followed by the fine collision.
template <typename S, int KIND>
__device__ inline void prolong_pair_node(const InterfaceParams &p, int r) {
    using T = typename Tr<S>::T;
    const PatchGeom &g = p.g;
    if (r >= g.nring) return;
    int i, j;
    if (r < g.nxf) { i = r; j = 0; }
    else if (r < 2 * g.nxf) { i = r - g.nxf; j = g.nyf - 1; }
    else if (r < 2 * g.nxf + g.nyf - 2) { i = 0; j = 1 + r - 2 * g.nxf; }
    else { i = g.nxf - 1; j = 1 + r - 2 * g.nxf - (g.nyf - 2); }
    int nodes_x[4], nodes_y[4], sidx[4];
    T wt[4];
    ring_stencil<T>(g, i, j, nodes_x, nodes_y, sidx, wt);
    // every load of the node up front (one round of memory latency); the
    // weight-0 entries of a coincident node repeat a valid node
    T gn[4][5], gs[4][5];
    const T *snap = reinterpret_cast<const T *>(p.snap);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        pre_at<S, T>(p.coarse, nodes_x[s], nodes_y[s], gn[s]);
#pragma unroll
        for (int q = 0; q < 5; ++q) gs[s][q] = snap[q * g.nsnap + sidx[s]];
    }
    T mid[5], end[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) mid[q] = end[q] = T(0);
    const T half = T(0.5);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            mid[q] += wt[s] * (half * gn[s][q] + half * gs[s][q]);
            end[q] += wt[s] * gn[s][q];
        }
    }
    T *ro = reinterpret_cast<T *>(p.ring_out);
    T out0[5], out1[5];
    rescale_collide<S, KIND>(p, mid, i, j, out0);
    rescale_collide<S, KIND>(p, end, i, j, out1);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        ro[k * g.nring + r] = out0[k];
        ro[(5 + k) * g.nring + r] = out1[k];
    }
}

// ---- fused step -------------------------------------------------------------
// One thread's share of the update: V consecutive nodes (x0 .. x0+V-1) of row
// y.  Returns the FP64 sum of rho over them when p.partial is set.
template <typename S>
constexpr bool kIsF64 = sizeof(S) == 8;

template <typename S, int Q, int KIND, bool PULL>
__device__ inline double update_tile(const StepParams &p, int x0, int y) {
    using T = typename Tr<S>::T;
    constexpr int V = PULL ? Tr<S>::V : 1;
    const int nx = p.nx, ny = p.ny;
    double local = 0.0;
    if (x0 >= nx) return local;

    const S *src = reinterpret_cast<const S *>(p.src);
    T g[Q][V];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ys = PULL ? wrapi(y - cyv<Q>(i), ny) : y;
        const S *row = src + i * p.pstride + (int64_t)ys * nx;
        S t[V];
        load_x<S, V>(row, PULL ? x0 - cxv<Q>(i) : x0, nx, t);
#pragma unroll
        for (int j = 0; j < V; ++j) g[i][j] = T(t[j]);
    }
    T c2v[V];
    {
        const T *c2row = reinterpret_cast<const T *>(p.c2) + (int64_t)y * nx;
        if (V > 1 && x0 + V <= nx) {
            typedef T ct __attribute__((ext_vector_type(V), aligned(sizeof(T))));
            ct t = __builtin_nontemporal_load(reinterpret_cast<const ct *>(c2row + x0));
#pragma unroll
            for (int j = 0; j < V; ++j) c2v[j] = t[j];
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) c2v[j] = c2row[min(x0 + j, nx - 1)];
        }
    }

    // refinement: the pre-collision state of this time on the coarse ring
    // line feeds the temporal interpolation of the next coarse step
    if (Q == 5 && p.snap) {
        T *snap = reinterpret_cast<T *>(p.snap);
        const int X0 = p.snap_x0, Y0 = p.snap_y0, W = p.snap_w, H = p.snap_h;
        const int nh = W + 3, nv = H + 3;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int x = x0 + j;
            if (x >= nx) break;
            if ((y == Y0 || y == Y0 + H) && x >= X0 - 1 && x <= X0 + W + 1) {
                const int t = (y == Y0 ? 0 : nh) + (x - (X0 - 1));
#pragma unroll
                for (int i = 0; i < Q; ++i) snap[i * p.snap_n + t] = g[i][j];
            }
            if ((x == X0 || x == X0 + W) && y >= Y0 - 1 && y <= Y0 + H + 1) {
                const int t = 2 * nh + (x == X0 ? 0 : nv) + (y - (Y0 - 1));
#pragma unroll
                for (int i = 0; i < Q; ++i) snap[i * p.snap_n + t] = g[i][j];
            }
        }
    }

    // receivers of this row (CSR lookup; rows without receivers cost one
    // uniform pair of loads)
    int rb = 0, re = 0;
    if (p.rec.row_ptr) {
        rb = p.rec.row_ptr[y];
        re = p.rec.row_ptr[y + 1];
    }

    S outv[Q][V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        T gj[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) gj[i] = g[i][j];
        const int x = x0 + j;
        if (rb < re && x < nx) record_node<T, Q>(p.rec, rb, re, x, gj, c2v[j]);
        if ((p.partial || p.rho_out) && x < nx) {
            T rho = T(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) rho += gj[i];
            local += double(rho);
            if (p.rho_out) reinterpret_cast<T *>(p.rho_out)[(int64_t)y * nx + x] = rho;
        }
        T po[Q];
        post_node<T, Q, KIND>(p, gj, c2v[j], x, y, edge_dist(min(x, nx - 1), y, nx, ny), p.s_n, po);
#pragma unroll
        for (int i = 0; i < Q; ++i) outv[i][j] = to_store<S>(po[i]);
        if constexpr (Q == 5) {
            if (p.restrict_on && x < nx && !((x | y) & 1)) {
                // this fine node coincides with a coarse node: on the coarse
                // inner ring, its state (R_2, then the coarse collision)
                // replaces the coarse grid's own
                const PatchGeom &pg = p.iface.g;
                const int X = pg.X0 + (x >> 1), Y = pg.Y0 + (y >> 1);
                if (X >= pg.xa && X <= pg.xb && Y >= pg.ya && Y <= pg.yb &&
                    (X == pg.xa || X == pg.xb || Y == pg.ya || Y == pg.yb))
                    rescale_collide_store_impl<S, KIND>(p.iface, gj, X, Y);
            }
            if (p.ring_buf && x < nx && (y == 0 || y == ny - 1 || x == 0 || x == nx - 1)) {
                // outer ring of a fine grid: the state comes from the coarse
                // grid, not from streaming
                const int r = y == 0 ? x : y == ny - 1 ? nx + x : x == 0 ? 2 * nx + y - 1 : 2 * nx + ny - 2 + y - 1;
                const T *rb = reinterpret_cast<const T *>(p.ring_buf);
#pragma unroll
                for (int i = 0; i < 5; ++i) outv[i][j] = to_store<S>(rb[i * p.ring_n + r]);
            }
        }
    }
    S *dst = reinterpret_cast<S *>(p.dst);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store_x<S, V>(dst + i * p.pstride + (int64_t)y * nx, x0, nx, outv[i]);
    return local;
}

template <typename S, int Q, int KIND, bool PULL>
__global__ __launch_bounds__(kStepBlock) void k_step(StepParams p) {
    constexpr int V = PULL ? Tr<S>::V : 1;
    if constexpr (Q == 5 && !kIsF64<S>) {
        // leading block rows of a coarse launch: the fine outer-ring states
        // of this coarse step (they read only what this launch reads; FP64
        // runs them as a launch of their own, whose registers would lower
        // this kernel's occupancy)
        if ((int)blockIdx.y < p.pre_rows) {
            prolong_pair_node<S, KIND>(p.iface, ((int)blockIdx.y * gridDim.x + blockIdx.x) * kStepBlock + threadIdx.x);
            return;
        }
    }
    const int y = blockIdx.y - p.pre_rows;
    const int x0 = (blockIdx.x * kStepBlock + threadIdx.x) * V;
    double local = update_tile<S, Q, KIND, PULL>(p, x0, y);

    if (p.partial) {   // uniform branch: per-block sum of rho in FP64
        for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off, 64);
        __shared__ double sh[kStepBlock / 64];
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = local;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < kStepBlock / 64; ++k) s += sh[k];
            p.partial[(int64_t)y * gridDim.x + blockIdx.x] = s;
        }
    }
}

// ---- discrete adjoint (gradient of the trace misfit w.r.t. c^2) -----------------
// Backward step n: mu(x) = (1 - sigma(x)) lambda(n+1)(x + c_i) (transpose of
// the pull), nu = C mu (C symmetric; its conserved rows drop out of every
// term below), lambda(n) = mu - nu + E^T nu with
// (E^T nu)_j = sum_i w_i nu_i + c_j . sum_i (w_i / c^2) c_i nu_i, plus the
// receiver residuals c^2(x_r) r_r(n) on every population.  Gradient terms of
// time n: rho(n) dw . nu, S(n) dw . mu at the source node, r_r(n) rho(n) at
// receivers, and at n = 0 rho(0) dw . lambda(0) (g(0) is an equilibrium).
// lambda is single-use per step, so it streams like the forward populations.
template <typename T, int Q, int KIND>
__global__ __launch_bounds__(kStepBlock) void k_adjoint(AdjointParams p) {
    constexpr int V = Tr<T>::V;
    const int y = blockIdx.y;
    const int x0 = (blockIdx.x * kStepBlock + threadIdx.x) * V;
    const int nx = p.nx, ny = p.ny;
    if (x0 >= nx) return;
    T mu[Q][V];
    if (p.terminal) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int j = 0; j < V; ++j) mu[i][j] = T(0);
    } else {
        const T *ln = reinterpret_cast<const T *>(p.lam_next);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int ys = wrapi(y + cyv<Q>(i), ny);
            T t[V];
            load_x<T, V>(ln + i * p.pstride + (int64_t)ys * nx, x0 + cxv<Q>(i), nx, t);
#pragma unroll
            for (int j = 0; j < V; ++j) mu[i][j] = t[j];
        }
    }
    T c2v[V], rhov[V];
    {
        const T *c2row = reinterpret_cast<const T *>(p.c2) + (int64_t)y * nx;
        const T *rrow = reinterpret_cast<const T *>(p.rho) + (int64_t)y * nx;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const int x = min(x0 + j, nx - 1);
            c2v[j] = c2row[x];
            rhov[j] = rrow[x];
        }
    }
    int rb = 0, re = 0;
    if (p.rec.row_ptr) {
        rb = p.rec.row_ptr[y];
        re = p.rec.row_ptr[y + 1];
    }
    const T *res = reinterpret_cast<const T *>(p.rec.traces);
    T outv[Q][V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const int x = x0 + j;
        const T sf = sponge_factor<T>(min(x, nx - 1), y, nx, ny, p.sponge_width, p.sponge_smax);
        T m[Q], nu[Q], w[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) m[i] = mu[i][j] * sf;
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
            gacc += double(rhov[j]) * dn;
            if (y == p.src_y && x == p.src_x) gacc += p.s_n * dm;
        }
        weights<T, Q>(c2v[j], p.coll, w);
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
        T lam[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            lam[i] = m[i] - nu[i] + s0 + T(cxv<Q>(i)) * sxv + T(cyv<Q>(i)) * syv;
        if (rb < re && x < nx) {
            int lo = rb, hi = re;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (p.rec.xs[mid] < x) lo = mid + 1; else hi = mid;
            }
            for (; lo < re && p.rec.xs[lo] == x; ++lo) {
                const T rr = res[(int64_t)p.rec.slot[lo] * p.rec.cap + p.rec.col];
#pragma unroll
                for (int i = 0; i < Q; ++i) lam[i] += c2v[j] * rr;
                gacc += double(rr) * double(rhov[j]);
            }
        }
        if (p.initial) {
            double dl = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) dl += p.dw[i] * double(lam[i]);
            gacc += double(rhov[j]) * dl;
        }
        if (x < nx) p.grad[(int64_t)y * nx + x] += gacc;
#pragma unroll
        for (int i = 0; i < Q; ++i) outv[i][j] = lam[i];
    }
    T *lo = reinterpret_cast<T *>(p.lam);
#pragma unroll
    for (int i = 0; i < Q; ++i) store_x<T, V>(lo + i * p.pstride + (int64_t)y * nx, x0, nx, outv[i]);
}

// Residual r = p - d and misfit phi = 1/2 sum r^2 over columns 0 .. ncols-1
// of every receiver (one block, fixed summation order: deterministic).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_misfit(const T *traces, const T *obs, T *res, int32_t nrec, int64_t cap,
                                                   int64_t ncols, double *phi) {
    double s = 0.0;
    const int64_t n = (int64_t)nrec * ncols;
    for (int64_t k = threadIdx.x; k < n; k += kBlock) {
        const int64_t r = k / ncols, c = k % ncols;
        const int64_t idx = r * cap + c;
        const T d = traces[idx] - obs[idx];
        res[idx] = d;
        s += double(d) * double(d);
    }
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *phi = 0.5 * sh[0];
}

// ---- batched step over many shots (serving) ------------------------------------
// One launch covers every active shot: block b belongs to the shot whose
// block range [prefix[a], prefix[a+1]) holds it; the shot's time and buffer
// parity live in device memory, so the same launch sequence can be captured
// once and replayed.  The per-node update is update_tile(), identical to the
// single-grid step, so a shot's results do not depend on its batch mates.
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

template <typename S, int Q, int KIND>
__global__ __launch_bounds__(kStepBlock) void k_step_batch(BatchParams bp) {
    constexpr int V = Tr<S>::V;
    const int64_t b = blockIdx.x;
    int lo = 0, hi = bp.nact - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bp.prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const int slot = bp.order[lo];
    const ShotState ss = bp.state[slot];
    if (!ss.active || ss.t >= ss.t_end) return;
    const ShotEntry &e = bp.table[slot];
    const int64_t local = b - bp.prefix[lo];
    const int y = int(local / e.bx);
    const int tile = int(local % e.bx);
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
    p.rec = e.rec;
    p.rec.col = tn;
    p.partial = nullptr;
    update_tile<S, Q, KIND, true>(p, (tile * kStepBlock + threadIdx.x) * V, y);
}

// After a batched step: every active, unfinished shot moves to the next time
// and swaps its buffers.
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
__global__ __launch_bounds__(kBlock) void k_batch_advance2(ShotState *state, const int32_t *order, int nact) {
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nact) return;
    ShotState &ss = state[order[a]];
    if (ss.active && ss.t < ss.t_end) {
        ss.t += min<int64_t>(2, ss.t_end - ss.t);
        ss.cur ^= 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_advance(ShotState *state, const int32_t *order, int nact) {
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nact) return;
    ShotState &ss = state[order[a]];
    if (ss.active && ss.t < ss.t_end) {
        ss.t += 1;
        ss.cur ^= 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_finalize(const double *partial, int64_t n, double *out) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) s += partial[i];
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ---- set-up kernels --------------------------------------------------------
template <typename S, int Q>
__global__ __launch_bounds__(kBlock) void k_equilibrium(S *pop, int64_t pstride, const void *c2v,
                                                        const void *rho, const void *jx, const void *jy,
                                                        int in_f64, int64_t n, Collision c) {
    using T = typename Tr<S>::T;
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    auto rd = [&](const void *a) -> double {
        if (!a) return 0.0;
        return in_f64 ? reinterpret_cast<const double *>(a)[k] : double(reinterpret_cast<const float *>(a)[k]);
    };
    T r = T(rd(rho)), x = T(rd(jx)), y = T(rd(jy));
    T c2 = reinterpret_cast<const T *>(c2v)[k];
    T w[Q];
    weights<T, Q>(c2, c, w);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        T kj = Q == 5 ? T(0.5) : (i <= 4 ? T(c.kax) : T(c.kdg));
        T cj = T(cxv<Q>(i)) * x + T(cyv<Q>(i)) * y;
        pop[i * pstride + k] = to_store<S>(w[i] * r + (i == 0 ? T(0) : kj * cj));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_convert_c2(const void *in, int in_f64, T *out, int64_t n,
                                                       double c2max, int32_t *bad) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    double v = in_f64 ? reinterpret_cast<const double *>(in)[k] : double(reinterpret_cast<const float *>(in)[k]);
    if (!(v > 0.0 && v <= c2max)) atomicAdd(bad, 1);
    out[k] = T(v);
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(uint32_t *p, int64_t nwords) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nwords; k += (int64_t)gridDim.x * kBlock)
        p[k] = 0u;
}

typedef float f4a __attribute__((ext_vector_type(4)));
// Reference copy: 16-byte nontemporal loads and stores, the access pattern of
// the fused step reduced to one read and one write stream.
__global__ __launch_bounds__(kBlock) void k_copy(f4a *__restrict__ dst, const f4a *__restrict__ src, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + k), dst + k);
}

// ---- fields of the current state ----------------------------------------------
template <typename S, int Q>
__global__ __launch_bounds__(kBlock) void k_field(FieldParams p) {
    using T = typename Tr<S>::T;
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= (int64_t)p.nx * p.ny) return;
    const int x = int(k % p.nx), y = int(k / p.nx);
    const S *pop = reinterpret_cast<const S *>(p.pop);
    T rho = T(0), jx = T(0), jy = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int xs = p.pre ? x : wrapi(x - cxv<Q>(i), p.nx);
        int ys = p.pre ? y : wrapi(y - cyv<Q>(i), p.ny);
        T gi = T(pop[i * p.pstride + (int64_t)ys * p.nx + xs]);
        rho += gi;
        jx += T(cxv<Q>(i)) * gi;
        jy += T(cyv<Q>(i)) * gi;
    }
    T v = rho;
    if (p.what == 1u) v = reinterpret_cast<const T *>(p.c2)[k] * rho;
    else if (p.what == 4u) v = jx;
    else if (p.what == 8u) v = jy;
    reinterpret_cast<T *>(p.out)[k] = v;
}

// Fine outer ring layout: top row (j = 0), bottom row (j = nyf-1), left
// column (i = 0, j = 1 .. nyf-2), right column (i = nxf-1).
template <typename S, int KIND>
__global__ __launch_bounds__(kBlock) void k_prolong(InterfaceParams p) {
    using T = typename Tr<S>::T;
    int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= p.g.nring) return;
    const PatchGeom &g = p.g;
    int i, j;
    if (r < g.nxf) { i = r; j = 0; }
    else if (r < 2 * g.nxf) { i = r - g.nxf; j = g.nyf - 1; }
    else if (r < 2 * g.nxf + g.nyf - 2) { i = 0; j = 1 + r - 2 * g.nxf; }
    else { i = g.nxf - 1; j = 1 + r - 2 * g.nxf - (g.nyf - 2); }
    T gh[5];
    ring_interp<S>(p, i, j, gh);
    rescale_collide_store_impl<S, KIND>(p, gh, i, j);
}

template <typename S, int KIND>
__global__ __launch_bounds__(kBlock) void k_restrict(InterfaceParams p) {
    using T = typename Tr<S>::T;
    int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= p.g.ninner) return;
    const PatchGeom &g = p.g;
    const int nxr = g.xb - g.xa + 1;
    const int nyr = g.yb - g.ya - 1;
    int x, y;
    if (t < nxr) { x = g.xa + t; y = g.ya; }
    else if (t < 2 * nxr) { x = g.xa + t - nxr; y = g.yb; }
    else if (t < 2 * nxr + nyr) { x = g.xa; y = g.ya + 1 + t - 2 * nxr; }
    else { x = g.xb; y = g.ya + 1 + t - 2 * nxr - nyr; }
    T gf[5];
    pre_at<S, T>(p.fine, 2 * (x - g.X0), 2 * (y - g.Y0), gf);
    rescale_collide_store_impl<S, KIND>(p, gf, x, y);
}

template <typename S, int KIND>
__global__ __launch_bounds__(kBlock) void k_prolong_pair(InterfaceParams p) {
    prolong_pair_node<S, KIND>(p, blockIdx.x * kBlock + threadIdx.x);
}

// ---- dispatch helpers ----------------------------------------------------------
inline unsigned blocks_for(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <typename S>
int vwidth(bool pull) { return pull ? Tr<S>::V : 1; }

template <typename S>
hipError_t step_dispatch(const StepParams &p0, bool pull, hipStream_t s) {
    const int V = vwidth<S>(pull);
    dim3 grid((unsigned)(((int64_t)p0.nx + (int64_t)V * kStepBlock - 1) / ((int64_t)V * kStepBlock)), (unsigned)p0.ny);
    const int kind = p0.coll.kind;
    StepParams p = p0;
    p.pre_rows = 0;
    if (p0.prolong_on) {
        const int64_t per_row = (int64_t)grid.x * kStepBlock;
        const int rows = (int)((p0.iface.g.nring + per_row - 1) / per_row);
        if (!kIsF64<S> && (int64_t)p0.ny + rows <= 65535) {
            p.pre_rows = rows;
            grid.y += (unsigned)rows;
        } else {   // a launch of its own first
            const bool mrt = kind == 1;
            dim3 pg(blocks_for(p0.iface.g.nring));
            if (mrt) hipLaunchKernelGGL((k_prolong_pair<S, 1>), pg, dim3(kBlock), 0, s, p0.iface);
            else hipLaunchKernelGGL((k_prolong_pair<S, 0>), pg, dim3(kBlock), 0, s, p0.iface);
        }
    }
#define LBW_LAUNCH(QQ, KK, PP) \
    hipLaunchKernelGGL((k_step<S, QQ, KK, PP>), grid, dim3(kStepBlock), 0, s, p)
    if (p.q == 5) {
        if (kind == 0) { if (pull) LBW_LAUNCH(5, 0, true); else LBW_LAUNCH(5, 0, false); }
        else { if (pull) LBW_LAUNCH(5, 1, true); else LBW_LAUNCH(5, 1, false); }
    } else {
        if (kind == 0) { if (pull) LBW_LAUNCH(9, 0, true); else LBW_LAUNCH(9, 0, false); }
        else { if (pull) LBW_LAUNCH(9, 1, true); else LBW_LAUNCH(9, 1, false); }
    }
#undef LBW_LAUNCH
    return hipGetLastError();
}

}  // namespace

// ---- launchers -------------------------------------------------------------------
int64_t step_blocks(int storage, int32_t nx, int32_t ny, bool pull) {
    int V = storage == ST_F32 ? vwidth<float>(pull) : storage == ST_F64 ? vwidth<double>(pull) : vwidth<_Float16>(pull);
    return (((int64_t)nx + (int64_t)V * kStepBlock - 1) / ((int64_t)V * kStepBlock)) * ny;
}

hipError_t launch_step(int storage, const StepParams &p, bool pull, hipStream_t s) {
    switch (storage) {
    case ST_F32: return step_dispatch<float>(p, pull, s);
    case ST_F64: return step_dispatch<double>(p, pull, s);
    case ST_F16: return step_dispatch<_Float16>(p, pull, s);
    }
    return hipErrorInvalidValue;
}

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

int step_vwidth(int storage) {
    return storage == ST_F32 ? Tr<float>::V : storage == ST_F64 ? Tr<double>::V : Tr<_Float16>::V;
}

int step_tile_nodes(int storage) { return step_vwidth(storage) * kStepBlock; }

hipError_t launch_step_batch(int storage, int q, const BatchParams &bp, int64_t nblocks, hipStream_t s) {
    if (nblocks <= 0 || bp.nact <= 0) return hipSuccess;
    dim3 grid((unsigned)nblocks);
    const bool mrt = bp.coll.kind == 1;
#define LBW_B(SS, QQ)                                                                              \
    do {                                                                                           \
        if (mrt) hipLaunchKernelGGL((k_step_batch<SS, QQ, 1>), grid, dim3(kStepBlock), 0, s, bp);  \
        else hipLaunchKernelGGL((k_step_batch<SS, QQ, 0>), grid, dim3(kStepBlock), 0, s, bp);      \
    } while (0)
    if (storage == ST_F32) { if (q == 5) LBW_B(float, 5); else LBW_B(float, 9); }
    else if (storage == ST_F64) { if (q == 5) LBW_B(double, 5); else LBW_B(double, 9); }
    else { if (q == 5) LBW_B(_Float16, 5); else LBW_B(_Float16, 9); }
#undef LBW_B
    return hipGetLastError();
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
    hipLaunchKernelGGL(k_batch_advance2, dim3(blocks_for(nact)), dim3(kBlock), 0, s, state, order, nact);
    return hipGetLastError();
}

hipError_t launch_batch_advance(ShotState *state, const int32_t *order, int nact, hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_advance, dim3(blocks_for(nact)), dim3(kBlock), 0, s, state, order, nact);
    return hipGetLastError();
}

hipError_t launch_adjoint(int storage, const AdjointParams &p, hipStream_t s) {
    const bool f64 = storage == ST_F64;
    const int V = f64 ? Tr<double>::V : Tr<float>::V;
    dim3 grid((unsigned)(((int64_t)p.nx + (int64_t)V * kStepBlock - 1) / ((int64_t)V * kStepBlock)), (unsigned)p.ny);
    const bool mrt = p.coll.kind == 1;
#define LBW_A(TT, QQ)                                                                             \
    do {                                                                                          \
        if (mrt) hipLaunchKernelGGL((k_adjoint<TT, QQ, 1>), grid, dim3(kStepBlock), 0, s, p);     \
        else hipLaunchKernelGGL((k_adjoint<TT, QQ, 0>), grid, dim3(kStepBlock), 0, s, p);         \
    } while (0)
    if (f64) { if (p.q == 5) LBW_A(double, 5); else LBW_A(double, 9); }
    else { if (p.q == 5) LBW_A(float, 5); else LBW_A(float, 9); }
#undef LBW_A
    return hipGetLastError();
}

hipError_t launch_misfit(int storage, const void *traces, const void *obs, void *res, int32_t nrec, int64_t cap,
                         int64_t ncols, double *phi, hipStream_t s) {
    if (storage == ST_F64)
        hipLaunchKernelGGL(k_misfit<double>, dim3(1), dim3(kBlock), 0, s, reinterpret_cast<const double *>(traces),
                           reinterpret_cast<const double *>(obs), reinterpret_cast<double *>(res), nrec, cap, ncols, phi);
    else
        hipLaunchKernelGGL(k_misfit<float>, dim3(1), dim3(kBlock), 0, s, reinterpret_cast<const float *>(traces),
                           reinterpret_cast<const float *>(obs), reinterpret_cast<float *>(res), nrec, cap, ncols, phi);
    return hipGetLastError();
}

hipError_t launch_sum_finalize(const double *partial, int64_t nblocks, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_finalize, dim3(1), dim3(kBlock), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_equilibrium(int storage, int32_t q, void *pop, int64_t pstride, const void *c2,
                              const void *rho, const void *jx, const void *jy, int in_f64,
                              int32_t nx, int32_t ny, const Collision &coll, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny;
    dim3 grid(blocks_for(n));
#define LBW_EQ(SS, QQ) hipLaunchKernelGGL((k_equilibrium<SS, QQ>), grid, dim3(kBlock), 0, s, \
                                          reinterpret_cast<SS *>(pop), pstride, c2, rho, jx, jy, in_f64, n, coll)
    if (storage == ST_F32) { if (q == 5) LBW_EQ(float, 5); else LBW_EQ(float, 9); }
    else if (storage == ST_F64) { if (q == 5) LBW_EQ(double, 5); else LBW_EQ(double, 9); }
    else { if (q == 5) LBW_EQ(_Float16, 5); else LBW_EQ(_Float16, 9); }
#undef LBW_EQ
    return hipGetLastError();
}

hipError_t launch_convert_c2(int storage, const void *in, int in_f64, void *out, int64_t n, double c2max,
                             int32_t *bad, hipStream_t s) {
    dim3 grid(blocks_for(n));
    if (storage == ST_F64)
        hipLaunchKernelGGL(k_convert_c2<double>, grid, dim3(kBlock), 0, s, in, in_f64,
                           reinterpret_cast<double *>(out), n, c2max, bad);
    else
        hipLaunchKernelGGL(k_convert_c2<float>, grid, dim3(kBlock), 0, s, in, in_f64,
                           reinterpret_cast<float *>(out), n, c2max, bad);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s) {
    int64_t words = bytes / 4;
    if (words <= 0) return hipSuccess;
    unsigned nb = (unsigned)std::min<int64_t>((words + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(kBlock), 0, s, reinterpret_cast<uint32_t *>(p), words);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    int64_t n = (int64_t)(bytes / 16);
    unsigned nb = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 1 << 20);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(kBlock), 0, s, reinterpret_cast<f4a *>(dst),
                       reinterpret_cast<const f4a *>(src), n);
    return hipGetLastError();
}

hipError_t launch_field(int storage, const FieldParams &p, hipStream_t s) {
    dim3 grid(blocks_for((int64_t)p.nx * p.ny));
#define LBW_F(SS, QQ) hipLaunchKernelGGL((k_field<SS, QQ>), grid, dim3(kBlock), 0, s, p)
    if (storage == ST_F32) { if (p.q == 5) LBW_F(float, 5); else LBW_F(float, 9); }
    else if (storage == ST_F64) { if (p.q == 5) LBW_F(double, 5); else LBW_F(double, 9); }
    else { if (p.q == 5) LBW_F(_Float16, 5); else LBW_F(_Float16, 9); }
#undef LBW_F
    return hipGetLastError();
}

#define LBW_IFACE(KERNEL, N)                                                                       \
    dim3 grid(blocks_for(N));                                                                      \
    const bool mrt = p.coll.kind == 1;                                                             \
    if (storage == ST_F32) { if (mrt) hipLaunchKernelGGL((KERNEL<float, 1>), grid, dim3(kBlock), 0, s, p); \
                             else hipLaunchKernelGGL((KERNEL<float, 0>), grid, dim3(kBlock), 0, s, p); }   \
    else if (storage == ST_F64) { if (mrt) hipLaunchKernelGGL((KERNEL<double, 1>), grid, dim3(kBlock), 0, s, p); \
                                  else hipLaunchKernelGGL((KERNEL<double, 0>), grid, dim3(kBlock), 0, s, p); } \
    else { if (mrt) hipLaunchKernelGGL((KERNEL<_Float16, 1>), grid, dim3(kBlock), 0, s, p);         \
           else hipLaunchKernelGGL((KERNEL<_Float16, 0>), grid, dim3(kBlock), 0, s, p); }           \
    return hipGetLastError();

hipError_t launch_prolong(int storage, const InterfaceParams &p, hipStream_t s) { LBW_IFACE(k_prolong, p.g.nring) }

hipError_t launch_prolong_pair(int storage, const InterfaceParams &p, hipStream_t s) { LBW_IFACE(k_prolong_pair, p.g.nring) }
hipError_t launch_restrict(int storage, const InterfaceParams &p, hipStream_t s) { LBW_IFACE(k_restrict, p.g.ninner) }

}  // namespace lbw
