// lb_runtime.cpp -- host side of the C-ABI declared in include/lbwave.h:
// descriptor validation, workspace carving, set-up uploads, receiver tables,
// the A/B buffer rotation of the fused step and the coarse/fine refinement
// schedule (arXiv:1704.03172, Sec. IV).  The library never allocates device
// memory; everything lives in the caller's workspace.
#include "lbwave.h"
#include "lb_host.h"
#include "lb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace {

using lbw::Collision;
using lbw::FieldParams;
using lbw::InterfaceParams;
using lbw::PatchGeom;
using lbw::StepParams;

constexpr uint64_t kStateMagic = 0x4c42574156453031ull;  // "LBWAVE01"

using lbw::align_up;
using lbw::compute_bytes;
using lbw::storage_bytes;
using lbw::storage_kind;

double c2_max(const lb_grid_desc *d) { return lbw::c2_max(d->lattice, d->d2q9_ratio); }

bool omega_is_two(const lb_grid_desc *d) {
    if (d->collision == LB_BGK) return d->tau == 0.5;
    return d->s[3] == 2.0 && d->s[4] == 2.0;
}

PatchGeom patch_geom(const lb_grid_desc *d) {
    PatchGeom g;
    const int oo = d->patch_overlap_out, oi = d->patch_overlap_in;
    g.X0 = d->patch_x0 - oo;
    g.Y0 = d->patch_y0 - oo;
    g.W = d->patch_nx + 2 * oo;
    g.H = d->patch_ny + 2 * oo;
    g.nxf = 2 * g.W + 1;
    g.nyf = 2 * g.H + 1;
    g.xa = d->patch_x0 + oi;
    g.xb = d->patch_x0 + d->patch_nx - oi;
    g.ya = d->patch_y0 + oi;
    g.yb = d->patch_y0 + d->patch_ny - oi;
    g.nring = 2 * g.nxf + 2 * (g.nyf - 2);
    g.ninner = 2 * (g.xb - g.xa + 1) + 2 * (g.yb - g.ya - 1);
    g.nsnap = 2 * (g.W + 3) + 2 * (g.H + 3);
    return g;
}

int validate(const lb_grid_desc *d) {
    if (!d) return LB_E_INVALID;
    int rc = lbw::validate_scheme(d);
    if (rc) return rc;
    if (d->nx < 1 || d->ny < 1 || d->ny > 65535 || d->nx > (1 << 24)) return LB_E_RANGE;
    if (d->nbatch != 1) return LB_E_UNSUPPORTED;
    if (d->sponge_width < 0 || !(d->sponge_sigma_max >= 0.0 && d->sponge_sigma_max <= 1.0)) return LB_E_RANGE;
    if (d->trace_capacity < 0 || d->max_receivers < 0) return LB_E_RANGE;
    if (d->ckpt_every < 0 || d->ckpt_capacity < 0) return LB_E_RANGE;
    if (d->ckpt_every > 0 && d->ckpt_capacity < 1) return LB_E_RANGE;
    if (d->ckpt_every > 0 && d->patch_enable) return LB_E_UNSUPPORTED;
    if (d->steps_per_launch < 0 || d->steps_per_launch > 8) return LB_E_RANGE;
    if (d->rho_tape != 0 && d->rho_tape != 1) return LB_E_RANGE;
    if (d->rho_tape && d->patch_enable) return LB_E_UNSUPPORTED;
    if (d->rho_tape && d->trace_capacity < 1) return LB_E_RANGE;
    if (d->patch_enable) {
        if (d->lattice != LB_D2Q5 || d->patch_refine != 2) return LB_E_UNSUPPORTED;
        if (!omega_is_two(d)) return LB_E_UNSUPPORTED;
        if (d->patch_overlap_out < 1 || d->patch_overlap_in < 1) return LB_E_RANGE;
        if (d->patch_nx < 1 || d->patch_ny < 1) return LB_E_RANGE;
        if (2 * d->patch_overlap_in >= std::min(d->patch_nx, d->patch_ny)) return LB_E_RANGE;
        PatchGeom g = patch_geom(d);
        const int L = d->sponge_width;
        // the fine grid and the coarse ring-line stencil stay inside the
        // grid and outside the sponge (the fine grid has no sponge)
        if (g.X0 - 2 < L || g.Y0 - 2 < L) return LB_E_RANGE;
        if (g.X0 + g.W + 2 > d->nx - 1 - L || g.Y0 + g.H + 2 > d->ny - 1 - L) return LB_E_RANGE;
        if (g.nyf > 65535) return LB_E_RANGE;
    }
    return LB_OK;
}

struct Layout {
    int64_t pstride = 0, fpstride = 0;
    int64_t nblocks = 0;
    size_t pop[2] = {0, 0}, c2 = 0, rrow = 0, rxs = 0, rslot = 0;
    size_t frow = 0, fxs = 0, fslot = 0, partial = 0, scratch = 0, misfit = 0;
    size_t fpop[2] = {0, 0}, fc2 = 0, snap = 0, ring = 0, total = 0;
    size_t ckpt = 0, seg = 0, lam[2] = {0, 0};
    size_t gtab = 0, tape = 0;
};

Layout make_layout(const lb_grid_desc *d) {
    Layout L;
    const size_t ss = storage_bytes(d->precision), ts = compute_bytes(d->precision);
    const int64_t n = (int64_t)d->nx * d->ny;
    // population stride: 256-element aligned, skewed by 1024 elements so
    // that the population arrays of power-of-two grids do not alias in the
    // low address bits
    L.pstride = lbw::population_stride(n);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.pop[0] = take((size_t)d->lattice * L.pstride * ss);
    L.pop[1] = take((size_t)d->lattice * L.pstride * ss);
    L.c2 = take((size_t)n * ts);
    L.rrow = take(((size_t)d->ny + 1) * 4);
    L.rxs = take((size_t)std::max(d->max_receivers, 1) * 4);
    L.rslot = take((size_t)std::max(d->max_receivers, 1) * 4);
    // the collide-only launch (one node per thread) has the most blocks
    L.nblocks = lbw::step_blocks(storage_kind(d->precision), d->nx, d->ny, false);
    L.partial = take((size_t)L.nblocks * 8);
    L.scratch = take(256);
    L.misfit = take((size_t)lbw::kMisfitMaxBlocks * 8);
    L.gtab = take(sizeof(lbw::GraphTab));
    if (d->patch_enable) {
        PatchGeom g = patch_geom(d);
        const int64_t nf = (int64_t)g.nxf * g.nyf;
        L.fpstride = lbw::population_stride(nf);
        L.fpop[0] = take(5 * (size_t)L.fpstride * ss);
        L.fpop[1] = take(5 * (size_t)L.fpstride * ss);
        L.fc2 = take((size_t)nf * ts);
        L.frow = take(((size_t)g.nyf + 1) * 4);
        L.fxs = take((size_t)std::max(d->max_receivers, 1) * 4);
        L.fslot = take((size_t)std::max(d->max_receivers, 1) * 4);
        L.snap = take(2 * 5 * (size_t)g.nsnap * ts);   // ping-pong by coarse time parity
        L.ring = take(2 * 5 * (size_t)g.nring * ts);   // fine outer ring at T+1, T+2
    }
    if (d->ckpt_every > 0) {
        L.ckpt = take((size_t)d->ckpt_capacity * d->lattice * L.pstride * ss);
        L.seg = take((size_t)d->ckpt_every * n * ts);
    }
    if (d->ckpt_every > 0 || d->rho_tape) {
        L.lam[0] = take((size_t)d->lattice * L.pstride * ts);
        L.lam[1] = take((size_t)d->lattice * L.pstride * ts);
    }
    if (d->rho_tape) L.tape = take((size_t)d->trace_capacity * n * ts);
    L.total = off;
    return L;
}

// One lattice (the main/coarse grid or the fine grid of a patch).
struct Lattice {
    int32_t nx = 0, ny = 0;
    int64_t pstride = 0;
    void *pop[2] = {nullptr, nullptr};
    int cur = 0;           // buffer with the newest state
    int prev_pre = 0;      // the other buffer holds a pre-collision state
    void *c2 = nullptr;
    bool medium = false;
    int32_t *rrow = nullptr, *rxs = nullptr, *rslot = nullptr;
    bool has_rec = false;
    void *curp() const { return pop[cur]; }
    void *prevp() const { return pop[1 - cur]; }
};

}  // namespace

struct lb_grid {
    lb_grid_desc d;
    hipStream_t stream = nullptr;
    int storage = 0;
    size_t ssize = 4, tsize = 4;
    int q = 5;
    Collision coll;
    Layout L;
    char *ws = nullptr;
    Lattice main, fine;
    bool patch = false;
    PatchGeom geom;
    void *snap = nullptr;
    void *ring = nullptr;              // [2][5][nring] fine outer-ring states
    double *partial = nullptr;
    int32_t *scratch = nullptr;
    int64_t t = 0;
    bool collided = false;
    int32_t sx = -1, sy = -1;
    std::vector<double> wavelet;
    int32_t nrec = 0;
    void *traces = nullptr;
    uint32_t what = 0;
    double *sum_rho = nullptr;
    int sticky = LB_OK;
    // adjoint support
    char *ckpt = nullptr;          // [ckpt_capacity] population states
    void *seg = nullptr;           // [ckpt_every][ny][nx] recomputed rho
    void *lam[2] = {nullptr, nullptr};
    std::vector<char> ckpt_pre;    // slot holds a pre-collision state
    bool ckpt_valid = false;       // checkpoints describe the run since time 0
    void *tape = nullptr;          // [trace_capacity][ny][nx] pre-collision rho of each time
    bool tape_valid = false;       // the tape holds times 0 .. t of the run since time 0
    bool state_lost = false;       // an adjoint overwrote the forward state
    // graph replay of lb_step_n (lb_set_graph): chunks of graph_k steps
    int32_t graph_k = 0;
    int64_t gen = 0;               // bumped by every call that changes what a launch takes
    int64_t graph_base = -1;       // while capturing: the chunk's first time (else -1)
    lbw::GraphTab *gtab = nullptr; // the chunk table in the workspace
    struct Cached {
        hipGraphExec_t exec = nullptr;
        int64_t gen = -1;
        int flips = 0;             // buffer swaps of the chunk
    } gcache[2];                   // by the buffer holding the chunk's first state
    ~lb_grid() {
        for (auto &c : gcache)
            if (c.exec) hipGraphExecDestroy(c.exec);
    }
};

namespace {

int hip_fail(lb_grid *h, hipError_t e) {
    if (e == hipSuccess) return LB_OK;
    h->sticky = LB_E_HIP;
    return LB_E_HIP;
}

#define LB_TRY(h, expr)                                   \
    do {                                                  \
        hipError_t e__ = (expr);                          \
        if (e__ != hipSuccess) return hip_fail((h), e__); \
    } while (0)

double source_at(const lb_grid *h, int64_t n) {
    if (h->sx < 0 || n < 0 || n >= (int64_t)h->wavelet.size()) return 0.0;
    return h->wavelet[(size_t)n];
}

void *snap_buffer(const lb_grid *h, int64_t t) {
    return (char *)h->snap + (size_t)(t & 1) * 5 * h->geom.nsnap * h->tsize;
}

StepParams base_params(const lb_grid *h, const Lattice &g, bool is_main) {
    StepParams p;
    p.nx = g.nx;
    p.ny = g.ny;
    p.pstride = g.pstride;
    p.q = h->q;
    p.coll = h->coll;
    p.c2 = g.c2;
    if (is_main) {
        p.sponge_width = h->d.sponge_width;
        p.sponge_smax = h->d.sponge_sigma_max;
        p.src_x = h->sx;
        p.src_y = h->sy;
    }
    return p;
}

// While a chunk is captured for replay: point the launch at the chunk table
// and make its times relative to the chunk's first time, which is returned
// (0 outside a capture).
int64_t graph_time(const lb_grid *h, StepParams &p, int64_t col) {
    if (h->graph_base < 0) return 0;
    p.gtab = h->gtab;
    p.goff = (int32_t)(col - h->graph_base - 1);
    p.rec.col -= h->graph_base;
    return h->graph_base;
}

// The tape's rho field of time n.
void *tape_field(const lb_grid *h, int64_t n) {
    return (char *)h->tape + (size_t)n * h->main.nx * h->main.ny * h->tsize;
}

void attach_receivers(const lb_grid *h, const Lattice &g, StepParams &p, int64_t col) {
    if (!g.has_rec || h->nrec == 0) return;
    p.rec.row_ptr = g.rrow;
    p.rec.xs = g.rxs;
    p.rec.slot = g.rslot;
    p.rec.traces = h->traces;
    p.rec.nslots = h->nrec;
    p.rec.what = h->what;
    p.rec.cap = h->d.trace_capacity;
    p.rec.col = col;
}

// Launch one update of lattice g: pull-stream + collide (or collide only
// when `pull` is false, for the state at time 0).  Records column `col`.
// A fine launch takes its outer ring from ring_buf and, with `restr`, also
// writes the coarse inner ring; a coarse launch with `pro` also computes the
// fine outer-ring pair.
int launch_update(lb_grid *h, Lattice &g, bool is_main, bool pull, int64_t col, bool record, bool sum,
                  const void *ring_buf = nullptr, const InterfaceParams *restr = nullptr,
                  const InterfaceParams *pro = nullptr) {
    StepParams p = base_params(h, g, is_main);
    p.src = g.curp();
    p.dst = g.prevp();
    if (is_main) p.s_n = source_at(h, col);
    if (record) attach_receivers(h, g, p, col);
    if (sum) p.partial = h->partial;
    if (is_main && h->tape_valid) p.rho_out = tape_field(h, col);
    const int64_t base = graph_time(h, p, col);
    if (is_main && h->patch) {   // keep g(col) on the ring line: snapshot of time col
        p.snap = snap_buffer(h, col);
        p.snap_x0 = h->geom.X0;
        p.snap_y0 = h->geom.Y0;
        p.snap_w = h->geom.W;
        p.snap_h = h->geom.H;
        p.snap_n = h->geom.nsnap;
    }
    if (ring_buf) {
        p.ring_buf = ring_buf;
        p.ring_n = h->geom.nring;
    }
    if (restr) {
        p.restrict_on = 1;
        p.iface = *restr;
    } else if (pro) {
        p.prolong_on = 1;
        p.iface = *pro;
    }
    LB_TRY(h, lbw::launch_step(h->storage, p, pull, h->stream));
    if (sum) {
        const int64_t nb = lbw::step_blocks(h->storage, g.nx, g.ny, pull);
        LB_TRY(h, lbw::launch_sum_finalize(h->partial, nb, h->sum_rho + (col - base), p.gtab, h->stream));
    }
    g.cur = 1 - g.cur;
    g.prev_pre = pull ? 0 : 1;
    return LB_OK;
}

InterfaceParams iface_base(const lb_grid *h) {
    InterfaceParams p;
    p.g = h->geom;
    p.coll = h->coll;
    p.snap = h->snap;
    return p;
}

lbw::GridRef ref_prev(const Lattice &g) {
    lbw::GridRef r;
    r.pop = g.prevp();
    r.pre = g.prev_pre;
    r.c2 = g.c2;
    r.nx = g.nx;
    r.ny = g.ny;
    r.pstride = g.pstride;
    return r;
}

// Outer-ring states of the fine grid for the two fine steps of the coarse
// step from T = t_snap: R_{1/2} of the coarse state interpolated along the
// edges, at T+1 (mean of the ring-line snapshot of T and `coarse`, the
// coarse state of T+2) and at T+2 (`coarse`), then the fine collision.
InterfaceParams prolong_params(lb_grid *h, const lbw::GridRef &coarse, int64_t t_snap) {
    InterfaceParams p = iface_base(h);
    p.coarse = coarse;
    p.snap = snap_buffer(h, t_snap);
    p.dst_c2 = h->fine.c2;
    p.dst_nx = h->fine.nx;
    p.dst_ny = h->fine.ny;
    p.dst_pstride = h->fine.pstride;
    p.f = 0.5;
    p.ring_out = h->ring;
    return p;
}

// Half k (0: T+1, 1: T+2) of the ring states made by prolong_pair.
const void *ring_half(const lb_grid *h, int k) {
    return (const char *)h->ring + (size_t)k * 5 * h->geom.nring * h->tsize;
}

// Restriction at the coarse inner ring, fused into a fine launch: R_2 of the
// coincident fine node's pre-collision state, then the coarse collision,
// written into the coarse post-collision buffer `cur`.
InterfaceParams restrict_params(const lb_grid *h) {
    InterfaceParams p = iface_base(h);
    p.dst = h->main.curp();
    p.dst_c2 = h->main.c2;
    p.dst_nx = h->main.nx;
    p.dst_ny = h->main.ny;
    p.dst_pstride = h->main.pstride;
    p.f = 2.0;
    p.sponge_width = h->d.sponge_width;
    p.sponge_smax = h->d.sponge_sigma_max;
    return p;
}

bool recording(const lb_grid *h) { return h->nrec > 0 && h->traces; }

size_t state_bytes_main(const lb_grid *h) { return (size_t)h->q * h->main.pstride * h->ssize; }

// Save the state needed to restart the forward run at time `tc`: the buffer
// the next launch pulls from (post-collision h(tc-1), or g(0) when pre).
int save_checkpoint(lb_grid *h, int64_t tc, bool pre) {
    const int64_t slot = tc / h->d.ckpt_every;
    LB_TRY(h, lbw::launch_copy(h->ckpt + (size_t)slot * state_bytes_main(h), h->main.curp(), state_bytes_main(h),
                               h->stream));
    h->ckpt_pre[(size_t)slot] = pre ? 1 : 0;
    return LB_OK;
}

int initial_collision(lb_grid *h) {
    int rc;
    const bool rec = recording(h), sum = h->sum_rho != nullptr;
    if (h->d.ckpt_every > 0) {
        h->ckpt_valid = h->t == 0;
        if (h->ckpt_valid && (rc = save_checkpoint(h, 0, true))) return rc;
    }
    h->tape_valid = h->tape != nullptr && h->t == 0;   // this launch writes rho(0)
    if ((rc = launch_update(h, h->main, true, false, h->t, rec, sum))) return rc;
    if (h->patch) {
        // fine state of time 0 with its outer ring from the coarse state
        // g(0) (second half of the pair), and the coarse inner ring from it
        LB_TRY(h, lbw::launch_prolong_pair(h->storage, prolong_params(h, ref_prev(h->main), h->t), h->stream));
        const InterfaceParams rp = restrict_params(h);
        if ((rc = launch_update(h, h->fine, false, false, h->t, rec, false, ring_half(h, 1), &rp))) return rc;
    }
    h->collided = true;
    return LB_OK;
}

int one_step(lb_grid *h) {
    int rc;
    const bool rec = recording(h), sum = h->sum_rho != nullptr;
    const int64_t col = h->t + 1;
    if (!h->patch) {
        if (h->ckpt_valid && col % h->d.ckpt_every == 0 && (rc = save_checkpoint(h, col, false))) return rc;
        if ((rc = launch_update(h, h->main, true, true, col, rec, sum))) return rc;
        h->t = col;
        return LB_OK;
    }
    // Coarse step T -> T+2 in fine time units (Sec. IV schedule), 3 launches:
    // the coarse step, which also keeps the ring-line snapshot of T+2 for the
    // next step and computes the fine outer-ring states of T+1 and T+2 (from
    // h(T), whose pull is g(T+2), and the snapshot of T: both only read by
    // this launch); then two fine steps, the second of which also restricts
    // to the coarse inner ring of T+2.
    lbw::GridRef coarse_src;
    coarse_src.pop = h->main.curp();
    coarse_src.pre = 0;
    coarse_src.c2 = h->main.c2;
    coarse_src.nx = h->main.nx;
    coarse_src.ny = h->main.ny;
    coarse_src.pstride = h->main.pstride;
    const InterfaceParams pp = prolong_params(h, coarse_src, h->t);
    if ((rc = launch_update(h, h->main, true, true, col, rec, false, nullptr, nullptr, &pp))) return rc;
    if ((rc = launch_update(h, h->fine, false, true, col, false, false, ring_half(h, 0)))) return rc;  // T+1
    const InterfaceParams rp = restrict_params(h);
    if ((rc = launch_update(h, h->fine, false, true, col, rec, false, ring_half(h, 1), &rp))) return rc;  // T+2
    h->t = col;
    return LB_OK;
}

int upload_sync(lb_grid *h, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return LB_OK;
    LB_TRY(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
    LB_TRY(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

int set_medium_impl(lb_grid *h, Lattice &g, const void *c2, lb_dtype t, int on_device) {
    if (!h || !c2) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    if (t != LB_F32 && t != LB_F64) return LB_E_INVALID;
    g.medium = false;
    int rc = lbw::upload_c2(h->stream, h->d.precision, h->d.lattice, h->d.d2q9_ratio, g.c2, c2, t, on_device,
                            (int64_t)g.nx * g.ny, h->scratch);
    if (rc == LB_E_HIP) h->sticky = LB_E_HIP;
    if (rc) return rc;
    g.medium = true;
    return LB_OK;
}

int set_state_impl(lb_grid *h, Lattice &g, const void *rho, const void *jx, const void *jy, lb_dtype t,
                   int on_device) {
    if (!h || !rho) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    if (t != LB_F32 && t != LB_F64) return LB_E_INVALID;
    if (!g.medium) return LB_E_STATE;
    const int q = (&g == &h->fine) ? 5 : h->q;
    const int64_t n = (int64_t)g.nx * g.ny;
    g.cur = 0;
    g.prev_pre = 0;
    if (on_device) {
        LB_TRY(h, lbw::launch_equilibrium(h->storage, q, g.pop[0], g.pstride, g.c2, rho, jx, jy, t == LB_F64,
                                          g.nx, g.ny, h->coll, h->stream));
    } else {
        // stage the host fields in the other population buffer, in chunks of
        // nodes that fit it (the equilibrium is node-local)
        const size_t es = t == LB_F64 ? 8 : 4;
        const size_t cap_bytes = (size_t)q * g.pstride * h->ssize;
        const int64_t chunk = (int64_t)(cap_bytes / (3 * es)) / 64 * 64;
        if (chunk < 64) return LB_E_WORKSPACE;
        char *stage = (char *)g.pop[1];
        for (int64_t off = 0; off < n; off += chunk) {
            const int64_t cnt = std::min<int64_t>(chunk, n - off);
            const size_t bytes = (size_t)cnt * es;
            char *s_rho = stage, *s_jx = stage + bytes, *s_jy = stage + 2 * bytes;
            LB_TRY(h, hipMemcpyAsync(s_rho, (const char *)rho + off * es, bytes, hipMemcpyHostToDevice, h->stream));
            if (jx) LB_TRY(h, hipMemcpyAsync(s_jx, (const char *)jx + off * es, bytes, hipMemcpyHostToDevice, h->stream));
            if (jy) LB_TRY(h, hipMemcpyAsync(s_jy, (const char *)jy + off * es, bytes, hipMemcpyHostToDevice, h->stream));
            char *dst = (char *)g.pop[0] + (size_t)off * h->ssize;
            const char *c2p = (const char *)g.c2 + (size_t)off * h->tsize;
            LB_TRY(h, lbw::launch_equilibrium(h->storage, q, dst, g.pstride, c2p, s_rho, jx ? s_jx : nullptr,
                                              jy ? s_jy : nullptr, t == LB_F64, (int32_t)cnt, 1, h->coll,
                                              h->stream));
            LB_TRY(h, hipStreamSynchronize(h->stream));
        }
    }
    if (&g == &h->main) {
        h->t = 0;
        h->collided = false;
        h->state_lost = false;
        h->ckpt_valid = false;
        h->tape_valid = false;
        if (h->patch) {   // the fine grid restarts at rest (lb_set_state_fine may follow)
            Lattice &f = h->fine;
            f.cur = 0;
            f.prev_pre = 0;
            const size_t fb = (size_t)((char *)f.pop[1] - (char *)f.pop[0]) + 5 * (size_t)f.pstride * h->ssize;
            LB_TRY(h, lbw::launch_fill_zero(f.pop[0], (int64_t)fb, h->stream));
        }
    }
    return LB_OK;
}

int get_field_impl(lb_grid *h, Lattice &g, int q, uint32_t what, void *out) {
    if (!h || !out) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    if (what != LB_FIELD_P && what != LB_FIELD_RHO && what != LB_FIELD_JX && what != LB_FIELD_JY)
        return LB_E_INVALID;
    if (!g.medium) return LB_E_STATE;
    FieldParams p;
    if (h->collided) {
        p.pop = g.prevp();
        p.pre = g.prev_pre;
    } else {
        p.pop = g.curp();
        p.pre = 1;
    }
    p.c2 = g.c2;
    p.nx = g.nx;
    p.ny = g.ny;
    p.pstride = g.pstride;
    p.q = q;
    p.what = what;
    p.out = out;
    LB_TRY(h, lbw::launch_field(h->storage, p, h->stream));
    if (h->patch && h->collided) {
        // nodes overwritten by the interface hold R_f of the other grid's
        // state; R_f keeps rho and J, so their fields come from that state
        InterfaceParams ip = iface_base(h);
        ip.field = what;
        ip.field_out = out;
        if (&g == &h->main) {
            ip.fine = ref_prev(h->fine);
            ip.dst_c2 = h->main.c2;
            ip.dst_nx = h->main.nx;
            ip.dst_ny = h->main.ny;
            LB_TRY(h, lbw::launch_restrict(h->storage, ip, h->stream));
        } else {
            ip.coarse = ref_prev(h->main);
            ip.a_snap = 0.0;
            ip.a_now = 1.0;
            ip.dst_c2 = h->fine.c2;
            ip.dst_nx = h->fine.nx;
            ip.dst_ny = h->fine.ny;
            LB_TRY(h, lbw::launch_prolong(h->storage, ip, h->stream));
        }
    }
    return LB_OK;
}

// Receiver tables: CSR over rows, x ascending within a row.
struct Rec { int32_t x, y, slot; };

int upload_receivers(lb_grid *h, Lattice &g, std::vector<Rec> &v) {
    g.has_rec = !v.empty();
    if (v.empty()) return LB_OK;
    std::sort(v.begin(), v.end(), [](const Rec &a, const Rec &b) {
        return a.y != b.y ? a.y < b.y : (a.x != b.x ? a.x < b.x : a.slot < b.slot);
    });
    std::vector<int32_t> row((size_t)g.ny + 1, 0), xs(v.size()), slot(v.size());
    for (const Rec &r : v) row[(size_t)r.y + 1]++;
    for (int y = 0; y < g.ny; ++y) row[(size_t)y + 1] += row[(size_t)y];
    for (size_t k = 0; k < v.size(); ++k) {
        xs[k] = v[k].x;
        slot[k] = v[k].slot;
    }
    int rc;
    if ((rc = upload_sync(h, g.rrow, row.data(), row.size() * 4))) return rc;
    if ((rc = upload_sync(h, g.rxs, xs.data(), xs.size() * 4))) return rc;
    if ((rc = upload_sync(h, g.rslot, slot.data(), slot.size() * 4))) return rc;
    return LB_OK;
}

struct StateHeader {
    uint64_t magic;
    int64_t t;
    int32_t collided, nx, ny, q, precision, patch;
    int32_t main_prev_pre, fine_prev_pre;
    uint64_t bytes;
};

}  // namespace

extern "C" {

void lb_default_desc(lb_grid_desc *d) {
    if (!d) return;
    std::memset(d, 0, sizeof(*d));
    d->nx = 64;
    d->ny = 64;
    d->lattice = LB_D2Q5;
    d->collision = LB_BGK;
    d->precision = LB_F32;
    d->nbatch = 1;
    d->tau = 0.5;
    const double s[9] = {1, 1, 1, 2, 2, 2, 1, 1, 2};
    for (int k = 0; k < 9; ++k) d->s[k] = s[k];
    d->d2q9_ratio = 0.25;
    d->patch_refine = 2;
    d->patch_overlap_out = 2;
    d->patch_overlap_in = 2;
}

int lb_validate_desc(const lb_grid_desc *d) { return validate(d); }

int lb_blocked_steps(const lb_grid_desc *d, int32_t *ns) {
    if (!d || !ns) return LB_E_INVALID;
    int rc = validate(d);
    if (rc) return rc;
    const int sk = lbw::step_kind(lbw::make_collision(d));
    const int st = storage_kind(d->precision);
    int m = lbw::stepn_max_grid(st, d->lattice, sk, d->nx, d->ny, true);
    if (d->steps_per_launch > 0)   // an explicit cap may ask for the marching kernel at any size
        m = lbw::stepn_round(st, d->lattice, sk, d->nx, d->ny,
                             std::min(lbw::stepn_max_grid(st, d->lattice, sk, d->nx, d->ny), (int)d->steps_per_launch));
    if (d->patch_enable) m = 1;
    *ns = m;
    return LB_OK;
}

size_t lb_workspace_bytes(const lb_grid_desc *d) {
    if (validate(d) != LB_OK) return 0;
    return make_layout(d).total;
}

int lb_create_grid(const lb_grid_desc *d, void *d_workspace, size_t ws_bytes, void *stream, lb_grid **out) {
    if (!out) return LB_E_INVALID;
    *out = nullptr;
    int rc = validate(d);
    if (rc) return rc;
    Layout L = make_layout(d);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255u)) return LB_E_WORKSPACE;
    lb_grid *h = new (std::nothrow) lb_grid();
    if (!h) return LB_E_INVALID;
    h->d = *d;
    h->stream = (hipStream_t)stream;
    h->storage = storage_kind(d->precision);
    h->ssize = storage_bytes(d->precision);
    h->tsize = compute_bytes(d->precision);
    h->q = d->lattice;
    h->L = L;
    h->ws = (char *)d_workspace;
    h->coll = lbw::make_collision(d);

    Lattice &m = h->main;
    m.nx = d->nx;
    m.ny = d->ny;
    m.pstride = L.pstride;
    m.pop[0] = h->ws + L.pop[0];
    m.pop[1] = h->ws + L.pop[1];
    m.c2 = h->ws + L.c2;
    m.rrow = (int32_t *)(h->ws + L.rrow);
    m.rxs = (int32_t *)(h->ws + L.rxs);
    m.rslot = (int32_t *)(h->ws + L.rslot);
    h->partial = (double *)(h->ws + L.partial);
    h->scratch = (int32_t *)(h->ws + L.scratch);
    h->gtab = (lbw::GraphTab *)(h->ws + L.gtab);
    size_t zero_bytes = L.pop[1] + (size_t)h->q * L.pstride * h->ssize;   // both buffers
    if (d->patch_enable) {
        h->patch = true;
        h->geom = patch_geom(d);
        Lattice &f = h->fine;
        f.nx = h->geom.nxf;
        f.ny = h->geom.nyf;
        f.pstride = L.fpstride;
        f.pop[0] = h->ws + L.fpop[0];
        f.pop[1] = h->ws + L.fpop[1];
        f.c2 = h->ws + L.fc2;
        f.rrow = (int32_t *)(h->ws + L.frow);
        f.rxs = (int32_t *)(h->ws + L.fxs);
        f.rslot = (int32_t *)(h->ws + L.fslot);
        h->snap = h->ws + L.snap;
        h->ring = h->ws + L.ring;
    }
    if (d->ckpt_every > 0) {
        h->ckpt = h->ws + L.ckpt;
        h->seg = h->ws + L.seg;
        h->ckpt_pre.assign((size_t)d->ckpt_capacity, 0);
    }
    if (d->ckpt_every > 0 || d->rho_tape) {
        h->lam[0] = h->ws + L.lam[0];
        h->lam[1] = h->ws + L.lam[1];
    }
    if (d->rho_tape) h->tape = h->ws + L.tape;
    // the state starts at rest: zero both population buffers of each grid
    hipError_t e = lbw::launch_fill_zero(m.pop[0], (int64_t)zero_bytes, h->stream);
    if (e == hipSuccess && h->patch)
        e = lbw::launch_fill_zero(h->fine.pop[0], (int64_t)(L.fpop[1] - L.fpop[0] + 5 * (size_t)L.fpstride * h->ssize),
                                  h->stream);
    if (e != hipSuccess) {
        delete h;
        return LB_E_HIP;
    }
    *out = h;
    return LB_OK;
}

int lb_destroy_grid(lb_grid *h) {
    if (!h) return LB_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    int rc = h->sticky ? h->sticky : (e == hipSuccess ? LB_OK : LB_E_HIP);
    delete h;
    return rc;
}

int lb_set_medium(lb_grid *h, const void *c2, lb_dtype t, int on_device) {
    if (!h) return LB_E_INVALID;
    return set_medium_impl(h, h->main, c2, t, on_device);
}

int lb_set_medium_fine(lb_grid *h, const void *c2, lb_dtype t, int on_device) {
    if (!h) return LB_E_INVALID;
    if (!h->patch) return LB_E_STATE;
    return set_medium_impl(h, h->fine, c2, t, on_device);
}

int lb_set_state(lb_grid *h, const void *rho, const void *jx, const void *jy, lb_dtype t, int on_device) {
    if (!h) return LB_E_INVALID;
    return set_state_impl(h, h->main, rho, jx, jy, t, on_device);
}

int lb_set_state_fine(lb_grid *h, const void *rho, const void *jx, const void *jy, lb_dtype t, int on_device) {
    if (!h) return LB_E_INVALID;
    if (!h->patch) return LB_E_STATE;
    if (h->collided) return LB_E_STATE;
    return set_state_impl(h, h->fine, rho, jx, jy, t, on_device);
}

int lb_set_source(lb_grid *h, int32_t x, int32_t y, const double *wavelet, int64_t nt) {
    if (!h) return LB_E_INVALID;
    ++h->gen;   // cached graphs of lb_step_n are stale
    if (h->sticky) return h->sticky;
    if (nt < 0 || (nt > 0 && !wavelet)) return LB_E_INVALID;
    if (nt == 0) {
        h->sx = h->sy = -1;
        h->wavelet.clear();
        return LB_OK;
    }
    if (x < 0 || y < 0 || x >= h->d.nx || y >= h->d.ny) return LB_E_RANGE;
    if (h->patch) {
        const PatchGeom &g = h->geom;
        if (x >= g.X0 - 1 && x <= g.X0 + g.W + 1 && y >= g.Y0 - 1 && y <= g.Y0 + g.H + 1) return LB_E_UNSUPPORTED;
    }
    try {
        h->wavelet.assign(wavelet, wavelet + nt);
    } catch (...) {
        return LB_E_INVALID;
    }
    h->sx = x;
    h->sy = y;
    return LB_OK;
}

int lb_record(lb_grid *h, const int32_t *rxy, int32_t nrec, void *d_traces, uint32_t what) {
    if (!h) return LB_E_INVALID;
    ++h->gen;   // cached graphs of lb_step_n are stale
    if (h->sticky) return h->sticky;
    if (nrec == 0) {
        h->nrec = 0;
        h->traces = nullptr;
        h->what = 0;
        h->main.has_rec = h->fine.has_rec = false;
        return LB_OK;
    }
    if (nrec < 0 || !rxy || !d_traces) return LB_E_INVALID;
    if (what == 0 || (what & ~0xFu)) return LB_E_INVALID;
    if (nrec > h->d.max_receivers) return LB_E_RANGE;
    std::vector<Rec> vm, vf;
    const PatchGeom &g = h->geom;
    for (int32_t r = 0; r < nrec; ++r) {
        int32_t x = rxy[2 * r], y = rxy[2 * r + 1];
        if (x < 0 || y < 0 || x >= h->d.nx || y >= h->d.ny) return LB_E_RANGE;
        const bool in_patch = h->patch && x >= h->d.patch_x0 && x < h->d.patch_x0 + h->d.patch_nx &&
                              y >= h->d.patch_y0 && y < h->d.patch_y0 + h->d.patch_ny;
        if (in_patch) vf.push_back({2 * (x - g.X0), 2 * (y - g.Y0), r});
        else vm.push_back({x, y, r});
    }
    int rc;
    if ((rc = upload_receivers(h, h->main, vm))) return rc;
    if (h->patch && (rc = upload_receivers(h, h->fine, vf))) return rc;
    h->nrec = nrec;
    h->traces = d_traces;
    h->what = what;
    return LB_OK;
}

int lb_record_sum_rho(lb_grid *h, double *d_sum) {
    if (!h) return LB_E_INVALID;
    ++h->gen;   // cached graphs of lb_step_n are stale
    if (h->patch && d_sum) return LB_E_UNSUPPORTED;
    h->sum_rho = d_sum;
    return LB_OK;
}

// Steps per launch of the blocked kernels for this grid (1: none): up to
// stepn_max steps, and on grids that the marching kernel takes and fills
// with its waves also its (larger) step count; a descriptor's
// steps_per_launch caps it, and may ask for the marching kernel on any grid
// it takes.
int blocked_max(const lb_grid *h) {
    if (h->patch) return 1;
    const int sk = lbw::step_kind(h->coll);
    int ns = lbw::stepn_max_grid(h->storage, h->q, sk, h->d.nx, h->d.ny, true);
    if (h->d.steps_per_launch > 0)   // an explicit cap may ask for the marching kernel at any size
        ns = lbw::stepn_round(h->storage, h->q, sk, h->d.nx, h->d.ny,
                              std::min(lbw::stepn_max_grid(h->storage, h->q, sk, h->d.nx, h->d.ny),
                                       h->d.steps_per_launch));
    return ns;
}

// Steps the next launch may take: at most blocked_max, and a launch from t
// to t+ns skips the states h(t+1) .. h(t+ns-1), so no checkpoint column
// (whose launch pulls from h(col-1)) may fall in t+2 .. t+ns.  left: steps
// still to take in this call; the last launch of a call takes one step (the
// fields and the saved state of time t are read from h(t-1)).  The count is
// rounded down to one a kernel takes (1 .. stepn_max, or the marching
// kernel's).
int blocked_steps(const lb_grid *h, int64_t left) {
    if (h->patch || h->sum_rho) return 1;
    if (h->graph_base >= 0) {   // a captured chunk: the graph entry kernels' one count, else one step
        const int g = lbw::stepn_graph_steps(h->storage, h->q, lbw::step_kind(h->coll), h->d.nx);
        return std::min(g, blocked_max(h)) == g && left - 1 >= g ? g : 1;
    }
    int ns = blocked_max(h);
    ns = (int)std::min<int64_t>(ns, left - 1);
    if (h->ckpt_valid)
        for (int k = 2; k <= ns; ++k)
            if ((h->t + k) % h->d.ckpt_every == 0) {
                ns = k - 1;
                break;
            }
    if (ns < 2) return 1;
    return lbw::stepn_round(h->storage, h->q, lbw::step_kind(h->coll), h->d.nx, h->d.ny, ns);
}

// Steps t -> t+ns in one launch of the blocked kernel (columns t+1 .. t+ns).
int blocked_launch(lb_grid *h, int ns) {
    const int64_t col = h->t + 1;
    if (h->ckpt_valid && col % h->d.ckpt_every == 0) {
        int rc = save_checkpoint(h, col, false);
        if (rc) return rc;
    }
    Lattice &g = h->main;
    StepParams p = base_params(h, g, true);
    p.src = g.curp();
    p.dst = g.prevp();
    p.s_n = source_at(h, col);
    p.s_n2 = source_at(h, col + 1);
    p.s_n3 = source_at(h, col + 2);
    p.s_n4 = source_at(h, col + 3);
    for (int k = 0; k < 4; ++k) p.s_more[k] = source_at(h, col + 4 + k);
    p.nrun = ns;
    if (recording(h)) attach_receivers(h, g, p, col);
    if (h->tape_valid) {   // rho of times col .. col + ns - 1
        p.rho_out = tape_field(h, col);
        p.rho_stride = (int64_t)g.nx * g.ny;
    }
    graph_time(h, p, col);
    LB_TRY(h, lbw::launch_stepn(h->storage, p, ns, h->stream));
    g.cur = 1 - g.cur;
    g.prev_pre = 0;
    h->t = col + ns - 1;
    return LB_OK;
}

// Whether lb_step_n may replay graphs now: enabled, no patch (three
// launches per coarse step with interface work), no checkpoints (their
// saves depend on the time) and a stream of the caller's (the null stream
// cannot be captured).
bool graph_ok(const lb_grid *h) {
    return h->graph_k > 0 && !h->patch && !h->ckpt_valid && !h->tape && h->stream != nullptr;
}

// One chunk of graph_k steps, replayed from a captured graph.  The chunk's
// launches are those of a call of graph_k steps (blocked launches of at most
// stepn_max steps, the last launch one step) with their times relative to
// the chunk's first time t0; before each replay one small launch writes t0
// and the chunk's source amplitudes into the chunk table.  One graph thus
// serves every chunk that starts from the same buffer; it is captured on
// first use and again after any call that changes what the launches take.
int graph_chunk(lb_grid *h) {
    const int64_t t0 = h->t;
    const int cur0 = h->main.cur;
    lb_grid::Cached &c = h->gcache[cur0];
    lbw::GraphTab tab;
    tab.t0 = t0;
    for (int k = 0; k < h->graph_k; ++k) tab.s[k] = source_at(h, t0 + 1 + k);
    LB_TRY(h, lbw::launch_graph_prime(h->gtab, tab, h->stream));
    if (!c.exec || c.gen != h->gen) {
        if (c.exec) {
            LB_TRY(h, hipGraphExecDestroy(c.exec));
            c.exec = nullptr;
        }
        // the launch functions advance the host state as if the launches
        // ran; it is put back afterwards and advanced once for the replay
        LB_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        h->graph_base = t0;
        int rc = LB_OK;
        for (int64_t k = 0; k < h->graph_k && rc == LB_OK;) {
            const int ns = blocked_steps(h, h->graph_k - k);
            rc = ns > 1 ? blocked_launch(h, ns) : one_step(h);
            k += ns;
        }
        h->graph_base = -1;
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(h->stream, &graph);
        const int flips = h->main.cur != cur0;
        h->t = t0;
        h->main.cur = cur0;
        if (rc != LB_OK || ec != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return rc != LB_OK ? rc : hip_fail(h, ec);
        }
        const hipError_t ei = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            c.exec = nullptr;
            return hip_fail(h, ei);
        }
        c.gen = h->gen;
        c.flips = flips;
    }
    LB_TRY(h, hipGraphLaunch(c.exec, h->stream));
    h->t = t0 + h->graph_k;
    if (c.flips) h->main.cur ^= 1;
    h->main.prev_pre = 0;
    return LB_OK;
}

int lb_step_n(lb_grid *h, int64_t n) {
    if (!h) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    if (n < 0) return LB_E_RANGE;
    if (!h->main.medium || (h->patch && !h->fine.medium) || h->state_lost) return LB_E_STATE;
    if ((recording(h) || h->sum_rho || h->tape_valid || (h->tape && !h->collided && h->t == 0)) &&
        h->t + n >= h->d.trace_capacity)
        return LB_E_RANGE;
    if (h->d.ckpt_every > 0 && (h->t + n) / h->d.ckpt_every >= h->d.ckpt_capacity) return LB_E_RANGE;
    int rc;
    if (!h->collided && (rc = initial_collision(h))) return rc;
    for (int64_t k = 0; k < n;) {
        if (graph_ok(h) && n - k >= h->graph_k) {
            if ((rc = graph_chunk(h))) return rc;
            k += h->graph_k;
            continue;
        }
        const int ns = blocked_steps(h, n - k);
        if (ns > 1) {
            if ((rc = blocked_launch(h, ns))) return rc;
        } else if ((rc = one_step(h))) {
            return rc;
        }
        k += ns;
    }
    return LB_OK;
}

static_assert(LB_GRAPH_MAX_STEPS == lbw::kGraphMaxSteps, "the chunk table holds the largest chunk");

int lb_set_graph(lb_grid *h, int32_t steps) {
    if (!h) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    if (steps != 0 && (steps < 2 || steps > lbw::kGraphMaxSteps)) return LB_E_RANGE;
    if (steps != 0 && (h->patch || h->stream == nullptr)) return LB_E_UNSUPPORTED;
    h->graph_k = steps;
    ++h->gen;
    return LB_OK;
}

int lb_get_time(const lb_grid *h, int64_t *n) {
    if (!h || !n) return LB_E_INVALID;
    *n = h->t;
    return LB_OK;
}

int lb_get_field(lb_grid *h, uint32_t what, void *d_out) {
    if (!h) return LB_E_INVALID;
    return get_field_impl(h, h->main, h->q, what, d_out);
}

int lb_get_field_fine(lb_grid *h, uint32_t what, void *d_out) {
    if (!h) return LB_E_INVALID;
    if (!h->patch) return LB_E_STATE;
    return get_field_impl(h, h->fine, 5, what, d_out);
}

size_t lb_state_bytes(const lb_grid *h) {
    if (!h) return 0;
    size_t b = 256 + 2 * (size_t)h->q * h->main.pstride * h->ssize;
    if (h->patch) b += 2 * 5 * (size_t)h->fine.pstride * h->ssize;
    return b;
}

int lb_get_state(lb_grid *h, void *d_out) {
    if (!h || !d_out) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    StateHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    hd.magic = kStateMagic;
    hd.t = h->t;
    hd.collided = h->collided;
    hd.nx = h->d.nx;
    hd.ny = h->d.ny;
    hd.q = h->q;
    hd.precision = h->d.precision;
    hd.patch = h->patch;
    hd.main_prev_pre = h->main.prev_pre;
    hd.fine_prev_pre = h->fine.prev_pre;
    hd.bytes = lb_state_bytes(h);
    // the whole 256-byte header, zero past the fields, so that equal states
    // give equal blobs
    static_assert(sizeof(StateHeader) <= 256, "the header region holds the header");
    unsigned char head[256] = {};
    std::memcpy(head, &hd, sizeof(hd));
    char *o = (char *)d_out;
    LB_TRY(h, hipMemcpyAsync(o, head, sizeof(head), hipMemcpyHostToDevice, h->stream));
    size_t off = 256;
    const size_t mb = (size_t)h->q * h->main.pstride * h->ssize;
    LB_TRY(h, hipMemcpyAsync(o + off, h->main.curp(), mb, hipMemcpyDeviceToDevice, h->stream));
    LB_TRY(h, hipMemcpyAsync(o + off + mb, h->main.prevp(), mb, hipMemcpyDeviceToDevice, h->stream));
    off += 2 * mb;
    if (h->patch) {
        const size_t fb = 5 * (size_t)h->fine.pstride * h->ssize;
        LB_TRY(h, hipMemcpyAsync(o + off, h->fine.curp(), fb, hipMemcpyDeviceToDevice, h->stream));
        LB_TRY(h, hipMemcpyAsync(o + off + fb, h->fine.prevp(), fb, hipMemcpyDeviceToDevice, h->stream));
    }
    LB_TRY(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_set_raw_state(lb_grid *h, const void *d_in) {
    if (!h || !d_in) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    StateHeader hd;
    LB_TRY(h, hipMemcpyAsync(&hd, d_in, sizeof(hd), hipMemcpyDeviceToHost, h->stream));
    LB_TRY(h, hipStreamSynchronize(h->stream));
    if (hd.magic != kStateMagic || hd.nx != h->d.nx || hd.ny != h->d.ny || hd.q != h->q ||
        hd.precision != h->d.precision || hd.patch != (int32_t)h->patch || hd.bytes != lb_state_bytes(h))
        return LB_E_INVALID;
    const char *in = (const char *)d_in;
    size_t off = 256;
    const size_t mb = (size_t)h->q * h->main.pstride * h->ssize;
    h->main.cur = 0;
    LB_TRY(h, hipMemcpyAsync(h->main.pop[0], in + off, mb, hipMemcpyDeviceToDevice, h->stream));
    LB_TRY(h, hipMemcpyAsync(h->main.pop[1], in + off + mb, mb, hipMemcpyDeviceToDevice, h->stream));
    off += 2 * mb;
    if (h->patch) {
        const size_t fb = 5 * (size_t)h->fine.pstride * h->ssize;
        h->fine.cur = 0;
        LB_TRY(h, hipMemcpyAsync(h->fine.pop[0], in + off, fb, hipMemcpyDeviceToDevice, h->stream));
        LB_TRY(h, hipMemcpyAsync(h->fine.pop[1], in + off + fb, fb, hipMemcpyDeviceToDevice, h->stream));
    }
    LB_TRY(h, hipStreamSynchronize(h->stream));
    h->t = hd.t;
    h->collided = hd.collided != 0;
    h->state_lost = false;
    h->ckpt_valid = false;       // checkpoints of another run do not apply
    h->tape_valid = false;
    h->main.prev_pre = hd.main_prev_pre;
    h->fine.prev_pre = hd.fine_prev_pre;
    return LB_OK;
}

int lb_misfit(lb_grid *h, const void *d_obs, int64_t nt, void *d_res, double *d_phi) {
    if (!h || !d_obs || !d_res || !d_phi) return LB_E_INVALID;
    if (h->sticky) return h->sticky;
    if (!recording(h) || !(h->what & LB_FIELD_P)) return LB_E_STATE;
    if (nt < 0 || nt >= h->d.trace_capacity) return LB_E_RANGE;
    LB_TRY(h, lbw::launch_misfit(h->storage, h->traces, d_obs, d_res, h->nrec, h->d.trace_capacity, nt + 1, d_phi,
                                 (double *)(h->ws + h->L.misfit), h->stream));
    return LB_OK;
}

int lb_trace_misfit(const void *d_traces, const void *d_obs, void *d_res, int32_t nrec, int64_t cap, int64_t ncols,
                    lb_dtype t, double *d_phi, void *d_workspace, size_t ws_bytes, void *stream) {
    const int rc = lbw::check_trace_misfit(d_traces, d_obs, d_res, nrec, cap, ncols, t, d_phi);
    if (rc) return rc;
    if (!d_workspace || ((uintptr_t)d_workspace & 7u) || ws_bytes < (size_t)LB_TRACE_MISFIT_WORKSPACE_BYTES)
        return LB_E_WORKSPACE;
    return lbw::launch_misfit(t == LB_F64 ? lbw::ST_F64 : lbw::ST_F32, d_traces, d_obs, d_res, nrec, cap, ncols, d_phi,
                              (double *)d_workspace, (hipStream_t)stream) == hipSuccess ? LB_OK : LB_E_HIP;
}

// Backward steps n = b, b - 1, .., a of the adjoint, the forward rho of time
// n at rho_base + (n - a) fields; up to adjointn_max steps per launch (capped
// as the forward launches are, so steps_per_launch = 1 gives one step per
// launch) where they lie in [a, b] and not at the terminal time nt.
// cur_lam: the lambda buffer holding lambda(b + 1), updated.
int adjoint_backward(lb_grid *h, lbw::AdjointParams &ap, char *rho_base, int64_t a, int64_t b, int64_t nt,
                     int &cur_lam) {
    const int64_t n_nodes = (int64_t)h->main.nx * h->main.ny;
    const size_t field = (size_t)n_nodes * h->tsize;
    const int nmax = std::min(lbw::adjointn_max(h->storage, h->q), blocked_max(h));
    for (int64_t n = b; n >= a;) {
        ap.rho = rho_base + (size_t)(n - a) * field;
        ap.terminal = n == nt;
        ap.initial = n == 0;
        ap.lam_next = h->lam[cur_lam];
        ap.lam = h->lam[1 - cur_lam];
        ap.s_n = source_at(h, n);
        ap.rec.col = n;
        const int ns = n == nt ? 1 : (int)std::min<int64_t>(nmax, n - a + 1);
        if (ns >= 2) {
            ap.rho_back = n_nodes;
            for (int k = 0; k < 4; ++k) ap.s_back[k] = k < ns ? source_at(h, n - k) : 0.0;
            ap.initial_stage = n < ns ? (int32_t)n + 1 : 0;   // the stage of time 0
            LB_TRY(h, lbw::launch_adjointn(h->storage, ap, ns, h->stream));
        } else {
            LB_TRY(h, lbw::launch_adjoint(h->storage, ap, h->stream));
        }
        n -= ns;
        cur_lam = 1 - cur_lam;
    }
    return LB_OK;
}

int lb_adjoint(lb_grid *h, const void *d_res, int64_t nt, double *d_grad) {
    if (!h || !d_res || !d_grad) return LB_E_INVALID;
    ++h->gen;   // cached graphs of lb_step_n are stale
    if (h->sticky) return h->sticky;
    if (h->patch) return LB_E_UNSUPPORTED;
    const bool tape = h->tape_valid;   // else segments recomputed from checkpoints
    if (!tape && h->d.ckpt_every <= 0) return LB_E_STATE;
    if (!h->collided || !(tape || h->ckpt_valid) || h->state_lost || nt != h->t) return LB_E_STATE;
    if (!recording(h)) return LB_E_STATE;
    Lattice &g = h->main;
    const int64_t n_nodes = (int64_t)g.nx * g.ny;
    const size_t tsz = h->tsize;

    lbw::AdjointParams ap;
    ap.c2 = g.c2;
    ap.grad = d_grad;
    ap.nx = g.nx;
    ap.ny = g.ny;
    ap.pstride = g.pstride;
    ap.q = h->q;
    ap.coll = h->coll;
    if (h->q == 5) {
        const double dw[5] = {-2.0, 0.5, 0.5, 0.5, 0.5};
        for (int i = 0; i < 5; ++i) ap.dw[i] = dw[i];
    } else {
        const double r = h->d.d2q9_ratio, a = 1.0 / (2.0 + 4.0 * r);
        ap.dw[0] = -4.0 * a - 4.0 * r * a;
        for (int i = 1; i < 9; ++i) ap.dw[i] = i <= 4 ? a : r * a;
    }
    ap.sponge_width = h->d.sponge_width;
    ap.sponge_smax = h->d.sponge_sigma_max;
    ap.src_x = h->sx;
    ap.src_y = h->sy;
    if (g.has_rec) {
        ap.rec.row_ptr = g.rrow;
        ap.rec.xs = g.rxs;
        ap.rec.slot = g.rslot;
    }
    ap.rec.traces = const_cast<void *>(d_res);
    ap.rec.nslots = h->nrec;
    ap.rec.cap = h->d.trace_capacity;

    LB_TRY(h, lbw::launch_fill_zero(d_grad, n_nodes * 8, h->stream));
    int cur_lam = 0;     // lam[cur_lam] holds lambda(n+1)
    if (tape) return adjoint_backward(h, ap, (char *)h->tape, 0, nt, nt, cur_lam);
    const int64_t K = h->d.ckpt_every;
    for (int64_t j = nt / K; j >= 0; --j) {
        const int64_t a = j * K, b = std::min(a + K - 1, nt);
        // restore the forward state that the launch of time a pulls from
        LB_TRY(h, lbw::launch_copy(g.pop[0], h->ckpt + (size_t)j * state_bytes_main(h), state_bytes_main(h),
                                   h->stream));
        g.cur = 0;
        // the segment's rho fields, up to blocked_max steps per launch (the
        // collide-only launch of a pre-collision checkpoint takes one)
        for (int64_t m = a; m <= b;) {
            const bool pull = !(m == a && h->ckpt_pre[(size_t)j]);
            StepParams p = base_params(h, g, true);
            p.src = g.curp();
            p.dst = g.prevp();
            p.s_n = source_at(h, m);
            p.rho_out = (char *)h->seg + (size_t)(m - a) * n_nodes * tsz;
            // (rounded down to a count a kernel takes)
            const int ns = pull ? lbw::stepn_round(h->storage, h->q, lbw::step_kind(h->coll), h->d.nx, h->d.ny,
                                                   (int)std::min<int64_t>(blocked_max(h), b - m + 1))
                                : 1;
            if (ns > 1) {
                p.s_n2 = source_at(h, m + 1);
                p.s_n3 = source_at(h, m + 2);
                p.s_n4 = source_at(h, m + 3);
                for (int k = 0; k < 4; ++k) p.s_more[k] = source_at(h, m + 4 + k);
                p.nrun = ns;
                p.rho_stride = n_nodes;
                LB_TRY(h, lbw::launch_stepn(h->storage, p, ns, h->stream));
            } else {
                LB_TRY(h, lbw::launch_step(h->storage, p, pull, h->stream));
            }
            g.cur = 1 - g.cur;
            m += ns;
        }
        int rc = adjoint_backward(h, ap, (char *)h->seg, a, b, nt, cur_lam);
        if (rc) return rc;
    }
    h->state_lost = true;
    return LB_OK;
}

int lb_sync(lb_grid *h) {
    if (!h) return LB_E_INVALID;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) h->sticky = LB_E_HIP;
    return h->sticky;
}

const char *lb_status_string(int code) {
    switch (code) {
    case LB_OK: return "ok";
    case LB_E_INVALID: return "invalid argument";
    case LB_E_RANGE: return "value out of range";
    case LB_E_UNSUPPORTED: return "unsupported combination";
    case LB_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case LB_E_HIP: return "HIP runtime error";
    case LB_E_STATE: return "call out of order";
    default: return "unknown status";
    }
}

int lb_device_copy(void *d_dst, const void *d_src, size_t bytes, void *stream) {
    if (!d_dst || !d_src) return LB_E_INVALID;
    if (((uintptr_t)d_dst & 15u) || ((uintptr_t)d_src & 15u) || (bytes & 15u)) return LB_E_INVALID;
    return lbw::launch_copy(d_dst, d_src, bytes, (hipStream_t)stream) == hipSuccess ? LB_OK : LB_E_HIP;
}

}  // extern "C"

namespace lbw {

// Row norms |M_k|^2 of the moment matrices of Appendix A.
static const double kNormD2Q5[5] = {5, 2, 2, 20, 4};
static const double kNormD2Q9[9] = {9, 6, 6, 36, 4, 36, 12, 12, 4};

// The D2Q9 equilibrium's momentum coefficients w_i / c^2 (kax for the axis
// movers, kdg for the diagonal ones) as numbers of the arithmetic type with
// 2 kax + 4 kdg = 1 exactly, so that sum_i c_i g^eq_i is J with no bias
// (eq. linear eqm dist; the identity is sum_i w_i c_i c_i = c^2 I of eq. LB
// lattice moments).  Rounded to nearest on their own, 1/3 and 1/12 give
// 2 kax + 4 kdg = 1 + 3e-8 in FP32; at omega = 2 the collision then
// multiplies J by 1 + 6e-8 every step, a drift that grows linearly in time
// (measured: 8e-5 of rho after 2000 steps of the 1024^2 layered workload).
// kdg is moved by the fewest units in the last place that make 1 - 4 kdg
// halve into a representable kax.  For large ratios kax is then off
// 1 / (2 + 4r) by up to ~1e-5 relative (it is small beside 4 kdg ~ 1), which
// is why the weights take their own coefficient kw: the axis movers carry a
// share 2 kax ~ 1 / (1 + 2r) of the momentum, so the J term's change is
// below 1e-7 of J.
template <typename F>
static void momentum_exact_pair(double ratio, double *kax, double *kdg) {
    const F d0 = F(ratio / (2.0 + 4.0 * ratio));
    for (int m = 0; m <= 16; ++m) {
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            F d = d0;
            for (int k = 0; k < m; ++k) d = std::nextafter(d, sgn < 0 ? F(0) : F(1));
            // t = 1 - 4d, checked for exactness with an FMA (1 - t is exact
            // for t in [1/2, 1])
            const F t = F(1) - F(4) * d;
            if (std::fma(F(-4), d, F(1) - t) != F(0)) continue;
            const F a = t / F(2);
            if (F(2) * a == t && F(2) * a + F(4) * d == F(1)) {
                *kax = double(a);
                *kdg = double(d);
                return;
            }
            if (m == 0) break;
        }
    }
    *kax = 1.0 / (2.0 + 4.0 * ratio);   // not reached for ratios in use
    *kdg = ratio / (2.0 + 4.0 * ratio);
}

Collision make_collision(const lb_grid_desc *d) {
    Collision c;
    c.kind = d->collision;
    c.omega = 1.0 / d->tau;
    const double *norm = d->lattice == LB_D2Q5 ? kNormD2Q5 : kNormD2Q9;
    for (int k = 0; k < 9; ++k) c.srate[k] = (k >= 3 && k < d->lattice) ? d->s[k] / norm[k] : 0.0;
    c.ratio = d->lattice == LB_D2Q9 ? d->d2q9_ratio : 0.0;
    c.kax = 0.5;
    c.kdg = 0.0;
    c.kw = d->lattice == LB_D2Q9 ? 1.0 / (2.0 + 4.0 * c.ratio) : 0.5;
    if (d->lattice == LB_D2Q9) {
        if (d->precision == LB_F64) momentum_exact_pair<double>(c.ratio, &c.kax, &c.kdg);
        else momentum_exact_pair<float>(c.ratio, &c.kax, &c.kdg);
    }
    return c;
}

int check_trace_misfit(const void *traces, const void *obs, const void *res, int32_t nrec, int64_t cap,
                       int64_t ncols, lb_dtype t, const double *phi) {
    if (!traces || !obs || !res || !phi) return LB_E_INVALID;
    if (t != LB_F32 && t != LB_F64 && t != LB_F16S) return LB_E_INVALID;
    if (nrec < 1 || cap < 1 || ncols < 1 || ncols > cap) return LB_E_RANGE;
    if (cap > INT64_MAX / nrec) return LB_E_RANGE;   // nrec x cap elements must be addressable
    return LB_OK;
}

int validate_scheme(const lb_grid_desc *d) {
    if (d->lattice != LB_D2Q5 && d->lattice != LB_D2Q9) return LB_E_INVALID;
    if (d->collision != LB_BGK && d->collision != LB_MRT) return LB_E_INVALID;
    if (d->precision != LB_F32 && d->precision != LB_F64 && d->precision != LB_F16S) return LB_E_INVALID;
    if (d->collision == LB_BGK) {
        if (!(d->tau >= 0.5) || !std::isfinite(d->tau)) return LB_E_RANGE;
    } else {
        for (int k = 3; k < d->lattice; ++k)
            if (!(d->s[k] > 0.0 && d->s[k] <= 2.0)) return LB_E_RANGE;
    }
    if (d->lattice == LB_D2Q9 && !(d->d2q9_ratio >= 0.0 && std::isfinite(d->d2q9_ratio))) return LB_E_RANGE;
    return LB_OK;
}

int upload_c2(hipStream_t s, int precision, int lattice, double ratio, void *dst, const void *c2, lb_dtype t,
              int on_device, int64_t n, int32_t *scratch) {
    const double cmax = lbw::c2_max(lattice, ratio);
    const bool in64 = t == LB_F64;
    if (!on_device) {
        if (compute_bytes(precision) == 8) {
            std::vector<double> v((size_t)n);
            for (int64_t k = 0; k < n; ++k) {
                double x = in64 ? ((const double *)c2)[k] : (double)((const float *)c2)[k];
                if (!(x > 0.0 && x <= cmax)) return LB_E_RANGE;
                v[(size_t)k] = x;
            }
            if (hipMemcpyAsync(dst, v.data(), (size_t)n * 8, hipMemcpyHostToDevice, s) != hipSuccess) return LB_E_HIP;
            if (hipStreamSynchronize(s) != hipSuccess) return LB_E_HIP;
        } else {
            std::vector<float> v((size_t)n);
            for (int64_t k = 0; k < n; ++k) {
                double x = in64 ? ((const double *)c2)[k] : (double)((const float *)c2)[k];
                if (!(x > 0.0 && x <= cmax)) return LB_E_RANGE;
                v[(size_t)k] = (float)x;
            }
            if (hipMemcpyAsync(dst, v.data(), (size_t)n * 4, hipMemcpyHostToDevice, s) != hipSuccess) return LB_E_HIP;
            if (hipStreamSynchronize(s) != hipSuccess) return LB_E_HIP;
        }
        return LB_OK;
    }
    if (launch_fill_zero(scratch, 256, s) != hipSuccess) return LB_E_HIP;
    if (launch_convert_c2(storage_kind(precision), c2, in64, dst, n, cmax, scratch, s) != hipSuccess) return LB_E_HIP;
    int32_t bad = 0;
    if (hipMemcpyAsync(&bad, scratch, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return LB_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return LB_E_HIP;
    return bad ? LB_E_RANGE : LB_OK;
}

}  // namespace lbw
