// lb_internal.h -- kernel parameter blocks and launchers shared by the
// runtime (lb_runtime.cpp) and the kernels (lb_kernels.hip).  Not part of
// the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lbw {

// Storage formats of the population arrays.
enum Storage : int { ST_F32 = 0, ST_F64 = 1, ST_F16 = 2 };

// Receivers of one grid: a CSR table over rows.  Within row y the entries
// row_ptr[y] .. row_ptr[y+1]-1 hold the receiver x positions in ascending
// order (xs) and the output slot of each (slot).
struct Receivers {
    const int32_t *row_ptr = nullptr;  // [ny + 1]; nullptr: nothing recorded
    const int32_t *xs = nullptr;
    const int32_t *slot = nullptr;
    void *traces = nullptr;            // [nfields][nslots][cap], compute type
    int32_t nslots = 0;                // receivers registered on the handle
    uint32_t what = 0;                 // LB_FIELD_* mask
    int64_t cap = 0;                   // columns per trace
    int64_t col = 0;                   // column written by this launch
};

// Relaxation constants.  For MRT only the non-conserved moments matter:
// srate[k] is s_k / |M_k|^2 for moment k (zero for conserved ones).
struct Collision {
    int32_t kind = 0;                  // LB_BGK or LB_MRT
    double omega = 2.0;                // BGK 1/tau
    double srate[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double kax = 0.5, kdg = 0.0;       // w_i / c^2 for axis / diagonal movers in the
                                       // equilibrium's J term (2 kax + 4 kdg = 1 exactly
                                       // in the arithmetic type)
    double kw = 0.5;                   // D2Q9 weights: w1 = c^2 kw, kw = 1 / (2 + 4r)
    double ratio = 0.0;                // D2Q9 w5 / w1
};

// Collision kind the forward kernels are instantiated for: 0 BGK, 1 MRT,
// 2 BGK with omega = 2 (tau = 1/2), whose collision is written as
// 2 g^eq - g.  The adjoint keeps Collision::kind.
inline int step_kind(const Collision &c) { return c.kind == 1 ? 1 : (c.omega == 2.0 ? 2 : 0); }

// Interface geometry of a factor-2 refinement patch (coarse units).
struct PatchGeom {
    int32_t X0 = 0, Y0 = 0;            // fine node (0, 0) at coarse (X0, Y0)
    int32_t W = 0, H = 0;              // fine grid spans W x H coarse cells
    int32_t nxf = 0, nyf = 0;          // 2W + 1, 2H + 1
    int32_t xa = 0, xb = 0, ya = 0, yb = 0;   // coarse inner ring rectangle
    int32_t nring = 0;                 // fine outer ring nodes
    int32_t ninner = 0;                // coarse inner ring nodes
    int32_t nsnap = 0;                 // coarse ring-line snapshot nodes
};

// A grid as seen by the interface kernels.
struct GridRef {
    const void *pop = nullptr;         // populations to read
    int32_t pre = 0;                   // 1: pop holds the pre-collision state
    const void *c2 = nullptr;
    int32_t nx = 0, ny = 0;
    int64_t pstride = 0;
};

struct InterfaceParams {
    PatchGeom g;
    GridRef coarse;                    // coarse state read
    GridRef fine;                      // fine state read (restriction)
    void *snap = nullptr;              // [5][nsnap] ring-line snapshot of time T
    double a_snap = 0.0, a_now = 1.0;  // prolongation: a_snap*snap + a_now*coarse
    void *dst = nullptr;               // populations written (fine or coarse)
    const void *dst_c2 = nullptr;      // c^2 of the written grid
    int32_t dst_nx = 0, dst_ny = 0;
    int64_t dst_pstride = 0;
    double f = 1.0;                    // non-equilibrium rescaling factor
    Collision coll;                    // collision of the written grid
    int32_t sponge_width = 0;          // sponge of the written grid
    double sponge_smax = 0.0;
    uint32_t field = 0;                // nonzero: write this LB_FIELD_* of the
    void *field_out = nullptr;         // interface state instead of populations
    void *ring_out = nullptr;          // prolongation pair: [2][5][nring] post-collision
                                       // ring states of fine times T+1 (mid), T+2 (end)
};

// Times of the launches of a captured graph that lb_step_n replays: the
// launches carry times relative to the first time t0 of the replayed chunk,
// and t0 and the chunk's source amplitudes s[k] = S(t0 + 1 + k) sit here, in
// device memory that the host fills (one small launch) before each replay.
constexpr int kGraphMaxSteps = 256;
struct GraphTab {
    int64_t t0 = 0;
    int64_t pad = 0;
    double s[kGraphMaxSteps + 8] = {};   // (zeros past the chunk: a launch reads four)
};

// One launch of the fused step (or of the collide-only variant).
struct StepParams {
    const void *src = nullptr;         // populations read
    void *dst = nullptr;               // populations written
    const void *c2 = nullptr;          // c^2 per node, compute type
    int32_t nx = 0, ny = 0;
    int64_t pstride = 0;               // elements between populations
    int32_t q = 5;
    Collision coll;
    int32_t sponge_width = 0;
    double sponge_smax = 0.0;
    int32_t src_x = -1, src_y = -1;    // source node
    double s_n = 0.0;                  // source amplitude of this time
    Receivers rec;
    double *partial = nullptr;         // per-block sums of rho (nullptr: off)
    void *rho_out = nullptr;           // [ny][nx] pre-collision rho (nullptr: off)
    void *snap = nullptr;              // refinement ring-line snapshot [5][snap_n]
    int32_t snap_x0 = 0, snap_y0 = 0;  // ring line: rows Y0, Y0+H over x in
    int32_t snap_w = 0, snap_h = 0;    // [X0-1, X0+W+1]; columns X0, X0+W over
    int32_t snap_n = 0;                // y in [Y0-1, Y0+H+1]
    const void *ring_buf = nullptr;    // fine grid of a patch: post-collision outer-ring
    int32_t ring_n = 0;                // states [5][ring_n] taken from the coarse grid
    int32_t restrict_on = 0;           // fine grid of a patch: also write the coarse
                                       // inner ring from this launch's pre-collision
                                       // state (iface: as for launch_restrict)
    int32_t prolong_on = 0;            // coarse grid of a patch: also compute the fine
                                       // outer-ring pair (iface: as launch_prolong_pair)
    InterfaceParams iface;
    int32_t pre_rows = 0;              // set by launch_step: leading block rows that
                                       // do the prolong_on work
    double s_n2 = 0.0;                 // launch_stepn: source amplitudes of the second,
    double s_n3 = 0.0;                 // third and fourth steps
    double s_n4 = 0.0;
    double s_more[4] = {0, 0, 0, 0};   // ... and of the fifth to eighth
    int32_t nrun = 1;                  // launch_stepn: steps this launch takes (= ns)
    int64_t rho_stride = 0;            // launch_stepn with rho_out: elements between the
                                       // rho fields of consecutive steps
    const GraphTab *gtab = nullptr;    // graph replay: rec.col is relative to gtab->t0 and
    int32_t goff = 0;                  // the source amplitudes are gtab->s[goff ..]
};

// One backward step of the discrete adjoint (misfit gradient w.r.t. c^2):
// lambda(n) = K^T (1 - sigma) P^T lambda(n+1) + r(n), with the gradient
// terms of time n accumulated into grad (FP64).
struct AdjointParams {
    const void *lam_next = nullptr;    // lambda(n+1) [q][pstride], compute type
    void *lam = nullptr;               // lambda(n) written
    const void *rho = nullptr;         // forward pre-collision rho(n) [ny][nx]
    const void *c2 = nullptr;
    double *grad = nullptr;            // [ny][nx]
    int32_t nx = 0, ny = 0;
    int64_t pstride = 0;
    int32_t q = 5;
    Collision coll;
    double dw[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // d w_i / d c^2
    int32_t sponge_width = 0;
    double sponge_smax = 0.0;
    int32_t src_x = -1, src_y = -1;
    double s_n = 0.0;                  // S(n)
    Receivers rec;                     // tables + residual array in `traces`
    int32_t terminal = 0;              // 1: n = N (no step, lambda(N+1) = 0)
    int32_t initial = 0;               // 1: n = 0, add the initial-state term
    // launch_adjointn (steps n = rec.col, n - 1, .., n - ns + 1): the rho of
    // time n - k at rho - k * rho_back elements, S(n - k) in s_back[k], and
    // the stage (k + 1) whose time is 0 (0: none)
    int64_t rho_back = 0;
    double s_back[4] = {0, 0, 0, 0};
    int32_t initial_stage = 0;
};

// Field extraction: one field of the state at the current time.
struct FieldParams {
    const void *pop = nullptr;
    int32_t pre = 0;                   // 1: direct read; 0: pull from post-collision
    const void *c2 = nullptr;
    int32_t nx = 0, ny = 0;
    int64_t pstride = 0;
    int32_t q = 5;
    uint32_t what = 0;
    void *out = nullptr;
};

// One shot of the batched executor (serving).  Static description, written
// by the host when the shot is admitted.
struct ShotEntry {
    void *pop0 = nullptr, *pop1 = nullptr;   // population buffers A / B
    const void *c2 = nullptr;
    const double *wavelet = nullptr;         // S(n), n < wavelet_len
    int64_t wavelet_len = 0;
    Receivers rec;                           // col is set per launch
    int32_t nx = 0, ny = 0;
    int64_t pstride = 0;
    int32_t sponge_width = 0;
    double sponge_smax = 0.0;
    int32_t src_x = -1, src_y = -1;
    int32_t bx = 0;                          // step blocks per row
    int32_t march = 0;                       // 1: the marching kernel takes the shape
};

// Dynamic state of a shot, advanced on the device.
struct ShotState {
    int64_t t = 0;                           // time of the newest state
    int64_t t_end = 0;                       // last time to compute
    int32_t cur = 0;                         // buffer holding h(t): 0 = A
    int32_t active = 0;
};

struct BatchParams {
    const ShotEntry *table = nullptr;        // [max_shots]
    ShotState *state = nullptr;              // [max_shots]
    const int64_t *prefix = nullptr;         // [nact + 1] first block of each active shot
    const int64_t *wprefix = nullptr;        // [nact + 1] first blocked-kernel wave of each active shot
    const int32_t *order = nullptr;          // [nact] slot of each active shot
    int32_t nact = 0;
    int32_t max_run = 1;                     // blocked launch: steps per shot at most
    Collision coll;
    // marching rounds: the first marching wave of each active shot, and the
    // params image of each slot for the round (nrun > 0: the shot takes the
    // marching launch; the round's other launches leave it alone)
    const int64_t *mprefix = nullptr;        // [nact + 1]
    StepParams *img = nullptr;               // [max_shots]; nullptr: no marching round
};

// Launchers (lb_kernels.hip).  All return the launch status.
hipError_t launch_adjoint(int storage, const AdjointParams &p, hipStream_t s);
// ns backward steps (n = p.rec.col down to n - ns + 1, ns - 1 <= n < N) in
// one launch: lambda(n+1) from p.lam_next, lambda(n-ns+1) to p.lam, rho and
// S of each time as in AdjointParams; the gradient gets the terms of n, then
// of n - 1, ... (the order of one-step launches).  2 <= ns <= adjointn_max.
hipError_t launch_adjointn(int storage, const AdjointParams &p, int ns, hipStream_t s);
int adjointn_max(int storage, int q);
// Trace misfit: res = traces - obs over columns 0 .. ncols-1 of nrec rows of
// cap columns, and phi = 1/2 sum res^2 (FP64) through misfit_blocks(nrec,
// ncols) block partials in `partial` (at most kMisfitMaxBlocks doubles), then
// one finalize block; the result depends only on the inputs (fixed order).
constexpr int kMisfitMaxBlocks = 2048;
int misfit_blocks(int32_t nrec, int64_t ncols);
hipError_t launch_misfit(int storage, const void *traces, const void *obs, void *res, int32_t nrec,
                         int64_t cap, int64_t ncols, double *phi, double *partial, hipStream_t s);
int step_vwidth(int storage);
int step_tile_nodes(int storage);   // x-nodes covered by one step block
hipError_t launch_step_batch(int storage, int q, const BatchParams &bp, int64_t nblocks, hipStream_t s);
hipError_t launch_batch_advance(ShotState *state, const int32_t *order, int nact, hipStream_t s);
// Blocked batch launch with the ns-step kernel: every active shot advances
// min(ns, bp.max_run, steps left) steps; then launch_batch_advance_n with
// run = bp.max_run.  nwaves: sum of stepn_waves over the active shots.
int64_t stepn_waves(int storage, int q, int kind, int ns, int32_t nx, int32_t ny);   // kind: step_kind()
hipError_t launch_stepn_batch(int storage, int q, int ns, const BatchParams &bp, int64_t nwaves, hipStream_t s);
hipError_t launch_batch_advance_n(ShotState *state, const int32_t *order, int nact, int run, hipStream_t s);
// Marching round of a batch (ns = stepn_march of the scheme): prep writes
// bp.img for every active shot (nrun = ns for a shot whose shape the
// marching kernel takes, with at least ns steps left; 0 otherwise), the
// marching launch runs those over nwaves = sum of stepn_march_waves, and
// advance_sel moves state: sel = 1 the marching shots by their nrun, sel = 2
// the others by min(run, steps left).  The batched step launches of a round
// (bp.img set) skip the marching shots.
int64_t stepn_march_waves(int storage, int q, int kind, int32_t nx, int32_t ny);
hipError_t launch_batch_march_prep(int q, const BatchParams &bp, int ns, hipStream_t s);
hipError_t launch_stepn_march_batch(int storage, int q, const BatchParams &bp, int64_t nwaves, hipStream_t s);
hipError_t launch_batch_advance_sel(ShotState *state, const int32_t *order, int nact, const StepParams *img, int sel,
                                    int run, hipStream_t s);
hipError_t launch_step(int storage, const StepParams &p, bool pull,
                       hipStream_t s);
// ns pull steps in one launch of the temporally blocked ns-step kernel
// (p.nrun must equal ns): reads h(n) from p.src, writes h(n + ns) to p.dst
// (a buffer other than p.src), records columns p.rec.col .. p.rec.col + ns - 1,
// source amplitudes p.s_n .. p.s_n4, p.s_more; with p.rho_out, the pre-collision rho of
// time n + s (s = 1..ns) goes to p.rho_out + (s - 1) * p.rho_stride.  No
// reduction partials, snapshot or interface work.
// 2 <= ns <= stepn_max(storage, p.q, p.coll.kind), or ns = stepn_march(...)
// without gtab; with gtab ns = stepn_graph_steps(...) only.
hipError_t launch_stepn(int storage, const StepParams &p, int ns, hipStream_t s);
int stepn_max(int storage, int q, int kind);   // steps per launch the blocked kernel offers (1: none)
// Steps of the multi-step launches of a captured chunk (p.gtab set): the
// most the kernel offers, on grids whose width the vector loads take; 1:
// the chunk takes one-step launches only.
int stepn_graph_steps(int storage, int q, int kind, int32_t nx);
// Steps per launch of the marching kernel for an nx x ny grid (kind:
// step_kind()), 0 where it does not apply; it takes exactly that count.
// pref: also 0 where a single grid of that size would leave the GPU
// underfilled with the marching kernel's waves (the launch plan's default).
int stepn_march(int storage, int q, int kind, int32_t nx, int32_t ny, bool pref = false);
// Fewest waves for which a marching launch fills the GPU (the threshold of
// pref above; the batched executor applies it to a round's waves).
int64_t stepn_march_min_waves(int storage, int q, int kind);
// Most steps one launch takes on an nx x ny grid (pref: as the default
// launch plan chooses), and the largest step count a launch can take that
// is at most ns (>= 1); kind is step_kind().
int stepn_max_grid(int storage, int q, int kind, int32_t nx, int32_t ny, bool pref = false);
int stepn_round(int storage, int q, int kind, int32_t nx, int32_t ny, int ns);
int64_t step_blocks(int storage, int32_t nx, int32_t ny, bool pull);
// Sum of the nblocks partials to out[0], or (gtab set: a replayed graph) to
// out[gtab->t0].
hipError_t launch_sum_finalize(const double *partial, int64_t nblocks,
                               double *out, const GraphTab *gtab, hipStream_t s);
// *dst = val on the device, in stream order (before a graph replay).
hipError_t launch_graph_prime(GraphTab *dst, const GraphTab &val, hipStream_t s);
hipError_t launch_equilibrium(int storage, int32_t q, void *pop,
                              int64_t pstride, const void *c2,
                              const void *rho, const void *jx, const void *jy,
                              int in_f64, int32_t nx, int32_t ny,
                              const Collision &coll, hipStream_t s);
hipError_t launch_convert_c2(int storage, const void *in, int in_f64,
                             void *out, int64_t n, double c2max,
                             int32_t *bad_count, hipStream_t s);
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s);
hipError_t launch_field(int storage, const FieldParams &p, hipStream_t s);
hipError_t launch_prolong(int storage, const InterfaceParams &p,
                          hipStream_t s);
hipError_t launch_restrict(int storage, const InterfaceParams &p,
                           hipStream_t s);
// The fine outer-ring states of one coarse step (p.ring_out), see
// InterfaceParams::ring_out.
hipError_t launch_prolong_pair(int storage, const InterfaceParams &p, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes,
                       hipStream_t s);

}  // namespace lbw
