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
//
// This one-step kernel serves single steps (the last of a call, sum-of-rho
// recording, checkpoint boundaries), the refinement patch, whose interface
// work is fused into it, and the collide-only first step of an adjoint
// segment; runs of steps (the adjoint's recompute included) go to the
// temporally blocked kernel of lb_blocked.h.  Both take their per-node
// arithmetic from lb_node.h.
#include "lb_internal.h"
#include "lb_node.h"

#include <algorithm>

namespace lbw {
namespace {

constexpr int kBlock = 256;       // set-up, field and interface kernels
constexpr int kStepBlock = 128;   // fused step (best of a block-size sweep)

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

// Blocks of NT fine outer-ring nodes: each side of the ring (top, bottom,
// left, right, in the ring's order) in runs of NT, so that no block spans a
// corner.
template <int NT>
__host__ __device__ inline int ring_tile_blocks(const PatchGeom &g) {
    return 2 * ((g.nxf + NT - 1) / NT) + 2 * ((g.nyf - 2 + NT - 1) / NT);
}

// The outer-ring states of the two fine steps of one coarse step T -> T+2:
// R_{1/2} of the coarse state interpolated to each fine ring node, at T+1
// (mean of the ring-line snapshot of T and the coarse state of T+2) and at
// T+2, each followed by the fine collision.  Block b (of ring_tile_blocks)
// takes NT consecutive nodes of one side.  Their stencils (the copy of a
// coincident coarse node, or the cubic (-1, 9, 9, -1)/16 along the side; see
// ring_stencil) cover at most NT/2 + 5 consecutive nodes of that side's
// ring line, which the block first pulls from the coarse state and reads
// from the snapshot into an LDS tile, once each instead of once per stencil
// that reaches them (up to three).  The stencil arithmetic then reads the
// tile.  All NT threads of the block must call this (it synchronises).
template <typename S, int KIND, int NT>
__device__ inline void prolong_pair_tile(const InterfaceParams &p, int b) {
    using T = typename Tr<S>::T;
    constexpr int NE = NT / 2 + 5;
    __shared__ T tn[5][NE], ts[5][NE];
    const PatchGeom &g = p.g;
    const int bh = (g.nxf + NT - 1) / NT, bv = (g.nyf - 2 + NT - 1) / NT;
    int side, c;
    if (b < bh) { side = 0; c = b; }
    else if (b < 2 * bh) { side = 1; c = b - bh; }
    else if (b < 2 * bh + bv) { side = 2; c = b - 2 * bh; }
    else if (b < 2 * bh + 2 * bv) { side = 3; c = b - 2 * bh - bv; }
    else return;   // the whole block
    const bool horiz = side < 2;
    const int nh = g.W + 3, nv = g.H + 3;
    const int nline = horiz ? nh : nv;   // ring-line nodes of the side
    const int lbase = side == 0 ? 0 : side == 1 ? nh : side == 2 ? 2 * nh : 2 * nh + nv;
    // along-side fine index u of thread 0 (i on the top and bottom rows, j
    // on the left and right columns); line node e is coarse node
    // (X0 - 1 + e, row) or (column, Y0 - 1 + e)
    const int u0 = (horiz ? 0 : 1) + c * NT;
    const int e_lo = u0 > 0 ? (u0 - 1) / 2 : 0;
    const int crow = g.Y0 + (side == 1 ? g.H : 0), ccol = g.X0 + (side == 3 ? g.W : 0);
    const T *snap = reinterpret_cast<const T *>(p.snap);
    for (int k = threadIdx.x; k < NE; k += NT) {
        const int e = e_lo + k;
        if (e < nline) {
            T gn[5];
            pre_at<S, T>(p.coarse, horiz ? g.X0 - 1 + e : ccol, horiz ? crow : g.Y0 - 1 + e, gn);
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                tn[q][k] = gn[q];
                ts[q][k] = snap[q * g.nsnap + lbase + e];
            }
        }
    }
    __syncthreads();
    const int u = u0 + (int)threadIdx.x;
    if (c * NT + (int)threadIdx.x >= (horiz ? g.nxf : g.nyf - 2)) return;
    const int i = horiz ? u : (side == 2 ? 0 : g.nxf - 1);
    const int j = horiz ? (side == 0 ? 0 : g.nyf - 1) : u;
    const int r = (side == 0 ? 0 : side == 1 ? g.nxf : side == 2 ? 2 * g.nxf : 2 * g.nxf + g.nyf - 2) + c * NT +
                  (int)threadIdx.x;
    // the stencil of ring_stencil, as tile entries; the weight-0 entries of
    // a coincident node repeat it
    int ek[4];
    T wt[4];
    if ((u & 1) == 0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            ek[s] = u / 2 + 1 - e_lo;
            wt[s] = s == 1 ? T(1) : T(0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) ek[s] = (u - 1) / 2 + s - e_lo;
        wt[0] = wt[3] = T(-1) / T(16);
        wt[1] = wt[2] = T(9) / T(16);
    }
    T gn[4][5], gs[4][5];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            gn[s][q] = tn[q][ek[s]];
            gs[s][q] = ts[q][ek[s]];
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
__device__ __attribute__((always_inline)) inline void step_body(const StepParams &p) {
    constexpr int V = PULL ? Tr<S>::V : 1;
    if constexpr (Q == 5 && !kIsF64<S>) {
        // leading block rows of a coarse launch: the fine outer-ring states
        // of this coarse step (they read only what this launch reads; FP64
        // runs them as a launch of their own, whose registers would lower
        // this kernel's occupancy)
        if ((int)blockIdx.y < p.pre_rows) {
            prolong_pair_tile<S, KIND, kStepBlock>(p.iface, (int)blockIdx.y * gridDim.x + blockIdx.x);
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

template <typename S, int Q, int KIND, bool PULL>
__global__ __launch_bounds__(kStepBlock) void k_step(StepParams p) {
    step_body<S, Q, KIND, PULL>(p);
}

// A one-step launch of a replayed graph (pull-stream, no interface work).
template <typename S, int Q, int KIND>
__global__ __launch_bounds__(kStepBlock) void k_step_graph(StepParams p) {
    const StepParams q = graph_params(p);
    step_body<S, Q, KIND, true>(q);
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
    // the FP64 gradient of these nodes, read before the arithmetic (16-byte
    // accesses where the row and nx allow) and written back after it
    double gv[V];
    double *grow = p.grad + (int64_t)y * nx;
    const bool gvec = x0 + V <= nx && (((int64_t)y * nx + x0) & 1) == 0;
    if (gvec) {
#pragma unroll
        for (int j = 0; j < V; j += 2) {
            const double2 t = *reinterpret_cast<const double2 *>(grow + x0 + j);
            gv[j] = t.x;
            gv[j + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) gv[j] = x0 + j < nx ? grow[x0 + j] : 0.0;
    }
    int rb = 0, re = 0;
    if (p.rec.row_ptr) {
        rb = p.rec.row_ptr[y];
        re = p.rec.row_ptr[y + 1];
    }
    T outv[Q][V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        const int x = x0 + j;
        T muj[Q], lam[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) muj[i] = mu[i][j];
        const double gacc = adjoint_node<T, Q, KIND>(p, muj, c2v[j], rhov[j], x, y, edge_dist(min(x, nx - 1), y, nx, ny),
                                                     x < nx ? rb : 0, x < nx ? re : 0, p.rec.col, p.s_n, p.initial != 0,
                                                     lam);
        gv[j] += gacc;
#pragma unroll
        for (int i = 0; i < Q; ++i) outv[i][j] = lam[i];
    }
    if (gvec) {
#pragma unroll
        for (int j = 0; j < V; j += 2) *reinterpret_cast<double2 *>(grow + x0 + j) = make_double2(gv[j], gv[j + 1]);
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
            if (x0 + j < nx) grow[x0 + j] = gv[j];
    }
    T *lo = reinterpret_cast<T *>(p.lam);
#pragma unroll
    for (int i = 0; i < Q; ++i) store_x<T, V>(lo + i * p.pstride + (int64_t)y * nx, x0, nx, outv[i]);
}

// Sum of a value over the 64 lanes of a wavefront by shuffles (lane 0 gets
// it); the order of the additions is fixed, so the result is reproducible.
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of kBlock threads: wave sums, then the wave partials in
// wave order (thread 0 gets it).
__device__ inline double block_sum(double v) {
    __shared__ double sh[kBlock / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w];
    }
    return s;
}

// Residual r = p - d over columns 0 .. ncols-1 of every receiver (written
// to res) and the per-block partial sums of r^2 in FP64 (partial[b], one per
// block of a grid-stride loop over the nrec x ncols elements).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_misfit_partial(const T *traces, const T *obs, T *res, int32_t nrec,
                                                           int64_t cap, int64_t ncols, double *partial) {
    double s = 0.0;
    const int64_t n = (int64_t)nrec * ncols;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) {
        const int64_t r = k / ncols, c = k - r * ncols;
        const int64_t idx = r * cap + c;
        const T d = traces[idx] - obs[idx];
        res[idx] = d;
        s += double(d) * double(d);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// phi = 1/2 (sum of the nb block partials), one block, fixed order.
__global__ __launch_bounds__(kBlock) void k_misfit_finalize(const double *partial, int32_t nb, double *phi) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) s += partial[i];
    s = block_sum(s);
    if (threadIdx.x == 0) *phi = 0.5 * s;
}

// ---- batched step over many shots (serving) ------------------------------------
// One launch covers every active shot: block b belongs to the shot whose
// block range [prefix[a], prefix[a+1]) holds it; the shot's time and buffer
// parity live in device memory, so the same launch sequence can be captured
// once and replayed.  The per-node update is update_tile(), identical to the
// single-grid step, so a shot's results do not depend on its batch mates.
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
    if (bp.img != nullptr && bp.img[slot].nrun > 0) return;   // the round's marching launch takes it
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
__global__ __launch_bounds__(kBlock) void k_batch_advance(ShotState *state, const int32_t *order, int nact) {
    int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nact) return;
    ShotState &ss = state[order[a]];
    if (ss.active && ss.t < ss.t_end) {
        ss.t += 1;
        ss.cur ^= 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_finalize(const double *partial, int64_t n, double *out,
                                                          const GraphTab *gtab) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) s += partial[i];
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[gtab ? gtab->t0 : 0] = sh[0];
}

// The chunk table of a graph replay, copied from the kernel arguments.
__global__ __launch_bounds__(kBlock) void k_graph_prime(GraphTab *dst, GraphTab val) {
    double *d = reinterpret_cast<double *>(dst);
    const double *v = reinterpret_cast<const double *>(&val);
    for (int i = threadIdx.x; i < (int)(sizeof(GraphTab) / 8); i += kBlock) d[i] = v[i];
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
    prolong_pair_tile<S, KIND, kBlock>(p, blockIdx.x);
}

// ---- dispatch helpers ----------------------------------------------------------
inline unsigned blocks_for(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <typename S>
int vwidth(bool pull) { return pull ? Tr<S>::V : 1; }

template <typename S>
hipError_t step_dispatch(const StepParams &p0, bool pull, hipStream_t s) {
    const int V = vwidth<S>(pull);
    dim3 grid((unsigned)(((int64_t)p0.nx + (int64_t)V * kStepBlock - 1) / ((int64_t)V * kStepBlock)), (unsigned)p0.ny);
    const int kind = step_kind(p0.coll);
    StepParams p = p0;
    p.pre_rows = 0;
    if (p0.prolong_on) {
        const int rows = (int)((ring_tile_blocks<kStepBlock>(p0.iface.g) + grid.x - 1) / grid.x);
        if (!kIsF64<S> && (int64_t)p0.ny + rows <= 65535) {
            p.pre_rows = rows;
            grid.y += (unsigned)rows;
        } else {   // a launch of its own first
            dim3 pg((unsigned)ring_tile_blocks<kBlock>(p0.iface.g));
            if (kind == 1) hipLaunchKernelGGL((k_prolong_pair<S, 1>), pg, dim3(kBlock), 0, s, p0.iface);
            else if (kind == 2) hipLaunchKernelGGL((k_prolong_pair<S, 2>), pg, dim3(kBlock), 0, s, p0.iface);
            else hipLaunchKernelGGL((k_prolong_pair<S, 0>), pg, dim3(kBlock), 0, s, p0.iface);
        }
    }
    if (p.gtab) {   // a launch of a captured chunk: its own entry kernel
        if (!pull || p.prolong_on || p.restrict_on || p.snap || p.ring_buf) return hipErrorInvalidValue;
#define LBW_GRAPH(QQ, KK) hipLaunchKernelGGL((k_step_graph<S, QQ, KK>), grid, dim3(kStepBlock), 0, s, p)
        if (p.q == 5) {
            if (kind == 0) LBW_GRAPH(5, 0); else if (kind == 2) LBW_GRAPH(5, 2); else LBW_GRAPH(5, 1);
        } else {
            if (kind == 0) LBW_GRAPH(9, 0); else if (kind == 2) LBW_GRAPH(9, 2); else LBW_GRAPH(9, 1);
        }
#undef LBW_GRAPH
        return hipGetLastError();
    }
#define LBW_LAUNCH(QQ, KK, PP) \
    hipLaunchKernelGGL((k_step<S, QQ, KK, PP>), grid, dim3(kStepBlock), 0, s, p)
    if (p.q == 5) {
        if (kind == 0) { if (pull) LBW_LAUNCH(5, 0, true); else LBW_LAUNCH(5, 0, false); }
        else if (kind == 2) { if (pull) LBW_LAUNCH(5, 2, true); else LBW_LAUNCH(5, 2, false); }
        else { if (pull) LBW_LAUNCH(5, 1, true); else LBW_LAUNCH(5, 1, false); }
    } else {
        if (kind == 0) { if (pull) LBW_LAUNCH(9, 0, true); else LBW_LAUNCH(9, 0, false); }
        else if (kind == 2) { if (pull) LBW_LAUNCH(9, 2, true); else LBW_LAUNCH(9, 2, false); }
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

int step_vwidth(int storage) {
    return storage == ST_F32 ? Tr<float>::V : storage == ST_F64 ? Tr<double>::V : Tr<_Float16>::V;
}

int step_tile_nodes(int storage) { return step_vwidth(storage) * kStepBlock; }

hipError_t launch_step_batch(int storage, int q, const BatchParams &bp, int64_t nblocks, hipStream_t s) {
    if (nblocks <= 0 || bp.nact <= 0) return hipSuccess;
    dim3 grid((unsigned)nblocks);
    const int kind = step_kind(bp.coll);
#define LBW_B(SS, QQ)                                                                              \
    do {                                                                                           \
        if (kind == 1) hipLaunchKernelGGL((k_step_batch<SS, QQ, 1>), grid, dim3(kStepBlock), 0, s, bp); \
        else if (kind == 2) hipLaunchKernelGGL((k_step_batch<SS, QQ, 2>), grid, dim3(kStepBlock), 0, s, bp); \
        else hipLaunchKernelGGL((k_step_batch<SS, QQ, 0>), grid, dim3(kStepBlock), 0, s, bp);      \
    } while (0)
    if (storage == ST_F32) { if (q == 5) LBW_B(float, 5); else LBW_B(float, 9); }
    else if (storage == ST_F64) { if (q == 5) LBW_B(double, 5); else LBW_B(double, 9); }
    else { if (q == 5) LBW_B(_Float16, 5); else LBW_B(_Float16, 9); }
#undef LBW_B
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

int misfit_blocks(int32_t nrec, int64_t ncols) {
    const int64_t n = (int64_t)nrec * ncols;
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kMisfitMaxBlocks));
}

hipError_t launch_misfit(int storage, const void *traces, const void *obs, void *res, int32_t nrec, int64_t cap,
                         int64_t ncols, double *phi, double *partial, hipStream_t s) {
    const int nb = misfit_blocks(nrec, ncols);
    if (storage == ST_F64)
        hipLaunchKernelGGL(k_misfit_partial<double>, dim3(nb), dim3(kBlock), 0, s,
                           reinterpret_cast<const double *>(traces), reinterpret_cast<const double *>(obs),
                           reinterpret_cast<double *>(res), nrec, cap, ncols, partial);
    else
        hipLaunchKernelGGL(k_misfit_partial<float>, dim3(nb), dim3(kBlock), 0, s,
                           reinterpret_cast<const float *>(traces), reinterpret_cast<const float *>(obs),
                           reinterpret_cast<float *>(res), nrec, cap, ncols, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_misfit_finalize, dim3(1), dim3(kBlock), 0, s, partial, nb, phi);
    return hipGetLastError();
}

hipError_t launch_sum_finalize(const double *partial, int64_t nblocks, double *out, const GraphTab *gtab,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_sum_finalize, dim3(1), dim3(kBlock), 0, s, partial, nblocks, out, gtab);
    return hipGetLastError();
}

hipError_t launch_graph_prime(GraphTab *dst, const GraphTab &val, hipStream_t s) {
    static_assert(sizeof(GraphTab) % 8 == 0 && sizeof(GraphTab) <= 4096, "the table travels as a kernel argument");
    hipLaunchKernelGGL(k_graph_prime, dim3(1), dim3(kBlock), 0, s, dst, val);
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

#define LBW_IFACE_KIND(KERNEL, SS)                                                                 \
    do {                                                                                           \
        if (kind == 1) hipLaunchKernelGGL((KERNEL<SS, 1>), grid, dim3(kBlock), 0, s, p);           \
        else if (kind == 2) hipLaunchKernelGGL((KERNEL<SS, 2>), grid, dim3(kBlock), 0, s, p);      \
        else hipLaunchKernelGGL((KERNEL<SS, 0>), grid, dim3(kBlock), 0, s, p);                     \
    } while (0)
#define LBW_IFACE(KERNEL, N)                                                                       \
    dim3 grid(blocks_for(N));                                                                      \
    const int kind = step_kind(p.coll);                                                            \
    if (storage == ST_F32) LBW_IFACE_KIND(KERNEL, float);                                          \
    else if (storage == ST_F64) LBW_IFACE_KIND(KERNEL, double);                                    \
    else LBW_IFACE_KIND(KERNEL, _Float16);                                                         \
    return hipGetLastError();

hipError_t launch_prolong(int storage, const InterfaceParams &p, hipStream_t s) { LBW_IFACE(k_prolong, p.g.nring) }

hipError_t launch_prolong_pair(int storage, const InterfaceParams &p, hipStream_t s) {
    dim3 grid((unsigned)ring_tile_blocks<kBlock>(p.g));   // one side's nodes per block
    const int kind = step_kind(p.coll);
    if (storage == ST_F32) LBW_IFACE_KIND(k_prolong_pair, float);
    else if (storage == ST_F64) LBW_IFACE_KIND(k_prolong_pair, double);
    else LBW_IFACE_KIND(k_prolong_pair, _Float16);
    return hipGetLastError();
}
hipError_t launch_restrict(int storage, const InterfaceParams &p, hipStream_t s) { LBW_IFACE(k_restrict, p.g.ninner) }

}  // namespace lbw
