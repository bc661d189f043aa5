/*
 * lbwave.h -- C-ABI of the MI355X (gfx950) linear lattice Boltzmann library
 * for linear acoustic waves.
 *
 * The method is the linear lattice Boltzmann scheme of Dhuri, Hanasoge,
 * Perlekar and Robertsson, "Numerical analysis of the lattice Boltzmann
 * method for simulation of linear acoustic waves" (arXiv:1704.03172):
 * D2Q5 and D2Q9 lattices (Table I, Appendix A), BGK (eq. BGK-LB) and MRT
 * (eq. MRT-LB, moments of eq. D2Q5/D2Q9 moments) collision around the
 * linear equilibrium g_i^eq = (w_i / c^2)(p + c_i . J) (eq. linear eqm
 * dist, p = c^2 rho by eq. state), per-node sound speed through the lattice
 * weights (Sec. II C, eq. LB lattice moments, eq. 0th lattice weight), a
 * point source w_i S(n) (eq. MRT-LB linear acoustic, eq. source), absorbing
 * sponge layers and a coarse/fine grid-refinement interface (Sec. IV,
 * eq. grid refinement eqm dist, eq. coarse-fine dist connect).
 *
 * Conventions shared by every call
 *  - Lattice units: dx = dt = 1.  Fields are row-major [ny][nx] (x fastest);
 *    y is depth, row 0 the top.  Populations are stored structure-of-arrays.
 *  - Every call returns LB_OK (0) or a negative LB_E_* code.  Argument and
 *    range checks happen before anything is enqueued; on error nothing is
 *    enqueued and the handle is unchanged.  An error raised by the HIP
 *    runtime while enqueuing is kept on the handle ("sticky") and returned by
 *    the next call and by lb_sync().  Nothing throws across this interface.
 *  - A handle is bound to one HIP stream (passed as void*, a hipStream_t)
 *    and is not thread-safe; distinct handles are independent.
 *  - Memory: the caller allocates one device workspace of
 *    lb_workspace_bytes() bytes and keeps it alive until lb_destroy_grid();
 *    the library never allocates device memory.  Host arrays passed in are
 *    copied before the call returns.  Device pointers passed in must stay
 *    valid until the stream has executed the work that uses them.
 *  - Time: the state at integer time n is the pre-collision population set.
 *    One step n -> n+1 collides at every node (adding w_i S(n) at the source
 *    node and damping in the sponge) and streams with periodic wrap.  Records
 *    (receiver traces, sum of rho) for time n are written into column n.
 */
#ifndef LBWAVE_H
#define LBWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define LB_OK             0
#define LB_E_INVALID     -1  /* NULL handle/pointer, malformed argument     */
#define LB_E_RANGE       -2  /* value outside its allowed range             */
#define LB_E_UNSUPPORTED -3  /* valid combination this library does not do  */
#define LB_E_WORKSPACE   -4  /* workspace missing or too small              */
#define LB_E_HIP         -5  /* HIP runtime error (sticky on the handle)    */
#define LB_E_STATE       -6  /* call out of order (e.g. step before medium) */

/* ---- enumerations ----------------------------------------------------- */
#define LB_D2Q5 5
#define LB_D2Q9 9
#define LB_BGK  0
#define LB_MRT  1

typedef enum {
    LB_F32 = 0,   /* populations and arithmetic in FP32                     */
    LB_F64 = 1,   /* populations and arithmetic in FP64                     */
    LB_F16S = 2   /* populations stored as FP16, arithmetic in FP32         */
} lb_dtype;

/* field masks for lb_record / lb_get_field */
#define LB_FIELD_P   1u  /* pressure p = c^2 rho (eq. state)                */
#define LB_FIELD_RHO 2u  /* rho = sum_i g_i (eq. macroscopic density)       */
#define LB_FIELD_JX  4u  /* J_x = sum_i c_ix g_i (eq. macroscopic velocity) */
#define LB_FIELD_JY  8u  /* J_y = sum_i c_iy g_i                            */

typedef struct lb_grid lb_grid;

/*
 * Grid descriptor.  Fill with lb_default_desc() and override fields.
 *   nx, ny         lattice nodes (both >= 1, ny <= 65535).
 *   lattice        LB_D2Q5 or LB_D2Q9 (velocity order of Appendix A).
 *   collision      LB_BGK (relaxation time tau, omega = 1/tau; tau = 1/2 is
 *                  the non-dissipative choice of Sec. II C) or LB_MRT.
 *   precision      an lb_dtype.
 *   tau            BGK relaxation time, tau >= 1/2.
 *   s[9]           MRT inverse relaxation times in moment order (D2Q5:
 *                  s_rho, s_v, s_v, s_e, s_p; D2Q9: s_rho, s_v, s_v, s_e,
 *                  s_p, s_eps, s_q, s_q, s_p).  Rates of the conserved
 *                  moments are ignored (they multiply zero); the others must
 *                  lie in (0, 2].
 *   d2q9_ratio     D2Q9 weight family r = w5 / w1 >= 0:
 *                  w1 = c^2 / (2 + 4r), w5 = r w1, w0 = 1 - 4 w1 - 4 w5
 *                  (r = 1/4 gives the conventional 4/9, 1/9, 1/36 at
 *                  c^2 = 1/3; r = 0 gives the D2Q5 weights).
 *   sponge_width   L >= 0: width of the absorbing frame along all four edges.
 *   sponge_sigma_max  in [0, 1]: after each collision a node at distance d
 *                  < L from the nearest edge is multiplied by
 *                  1 - sigma_max ((L - d)/L)^2 (Sec. IV sponge layers).
 *   patch_*        optional factor-2 refinement patch (D2Q5 only, omega = 2:
 *                  BGK tau = 1/2 or MRT s_e = s_p = 2).  The patch covers
 *                  coarse x in [patch_x0, patch_x0 + patch_nx], y likewise;
 *                  the fine grid extends patch_overlap_out coarse cells
 *                  beyond it; the coarse ring patch_overlap_in cells inside
 *                  the patch receives the fine solution.
 *   trace_capacity number of time columns of the trace / sum-rho arrays.
 *   max_receivers  receivers that lb_record may register.
 *   ckpt_every     K > 0 enables lb_adjoint: lb_step_n keeps a checkpoint of
 *                  the state at every time that is a multiple of K (and the
 *                  workspace grows by ckpt_capacity states, K rho fields and
 *                  two adjoint population sets).  0: no checkpoints.
 *   ckpt_capacity  checkpoint slots; a run of N steps needs N / K + 1.
 *   steps_per_launch  0 (default): lb_step_n advances several time steps
 *                  per kernel launch (temporal blocking), wherever it can
 *                  (no patch, no sum-rho recording, no checkpoint falling
 *                  inside a launch; the last launch of each call takes one
 *                  step), which divides the HBM traffic per step
 *                  accordingly; the results equal those of one step per
 *                  launch bit for bit.  The marching kernel, on grids it
 *                  takes that are large enough to fill the GPU with its
 *                  waves (FP32 D2Q5 from about 2350^2, D2Q9 from about
 *                  1570^2; FP64 D2Q5 from about 1300^2, D2Q9 always; FP16
 *                  storage from about 2400^2), takes with FP32 populations
 *                  seven steps for D2Q5 (nx even, ny >= 34), six for D2Q9
 *                  BGK (ny >= 32) and five for D2Q9 MRT (ny >= 30); with
 *                  FP64 eight for D2Q5 BGK (ny >= 36), seven for D2Q5 MRT
 *                  (ny >= 34) and four for D2Q9 (ny >= 28); with FP16
 *                  storage five for D2Q5 (nx a multiple of 4, ny >= 30).
 *                  Otherwise the short-segment kernel takes four steps for
 *                  D2Q5 and for FP64, three for D2Q9 with FP32 populations
 *                  and for D2Q5 with FP16 storage, and one for D2Q9 with
 *                  FP16 storage.  lb_blocked_steps reports the count.
 *                  1 .. 8: at most that many steps per launch (a launch
 *                  takes 1 .. 4 steps, or the marching count, which a cap
 *                  at or above it selects on any grid the marching kernel
 *                  takes).
 *   nbatch         independent shots sharing the grid shape (must be 1).
 *   rho_tape       1: lb_step_n also keeps the pre-collision rho of every
 *                  time 0 .. trace_capacity - 1 of the run since lb_set_state
 *                  (the workspace grows by trace_capacity rho fields), and
 *                  lb_adjoint reads it instead of recomputing segments from
 *                  checkpoints (no ckpt_every needed).  Steps per launch as
 *                  without the tape (the multi-step kernels also write
 *                  rho).  Not with a patch.  0: off.
 */
typedef struct {
    int32_t nx, ny;
    int32_t lattice;
    int32_t collision;
    int32_t precision;
    int32_t nbatch;
    double tau;
    double s[9];
    double d2q9_ratio;
    int32_t sponge_width;
    int32_t _pad0;
    double sponge_sigma_max;
    int32_t patch_enable;
    int32_t patch_x0, patch_y0, patch_nx, patch_ny;
    int32_t patch_refine;
    int32_t patch_overlap_out, patch_overlap_in;
    int64_t trace_capacity;
    int32_t max_receivers;
    int32_t ckpt_every;
    int32_t ckpt_capacity;
    int32_t steps_per_launch;
    int32_t rho_tape;
    int32_t _pad1;
} lb_grid_desc;

/* Fill *d with defaults: 64 x 64 D2Q5 BGK FP32, tau = 1/2, MRT rates
 * (1, 1, 1, 2, 2, 2, 1, 1, 2), ratio 1/4, no sponge, no patch,
 * trace_capacity 0, max_receivers 0, steps_per_launch 0, nbatch 1. */
void lb_default_desc(lb_grid_desc *d);

/* Check a descriptor without a GPU.  Returns LB_OK or the error code that
 * lb_create_grid would return for it. */
int lb_validate_desc(const lb_grid_desc *d);

/* Most time steps one kernel launch of lb_step_n takes for a grid with this
 * descriptor (temporal blocking; see steps_per_launch): the count the
 * blocked kernel offers for the lattice, collision and precision, capped by
 * steps_per_launch; 1 with a patch.  No GPU needed.  Returns LB_OK and
 * writes *ns, or the error lb_validate_desc gives (LB_E_INVALID for NULL). */
int lb_blocked_steps(const lb_grid_desc *d, int32_t *ns);

/* Device bytes the workspace of a grid with this descriptor needs
 * (two population buffers, c^2, receiver tables, reduction partials and,
 * with a patch, the fine grid and its ring buffers).  0 if the descriptor
 * is invalid. */
size_t lb_workspace_bytes(const lb_grid_desc *d);

/* Create a handle over a caller-owned device workspace of ws_bytes bytes
 * (at least lb_workspace_bytes(d), 256-byte aligned) bound to `stream`.
 * The state starts at rest (all populations 0, zeroed by a fill kernel
 * enqueued on the stream) at time 0; c^2 is unset. */
int lb_create_grid(const lb_grid_desc *d, void *d_workspace, size_t ws_bytes,
                   void *stream, lb_grid **out);

/* Release the handle (not the workspace).  NULL-safe; waits for the stream. */
int lb_destroy_grid(lb_grid *h);

/* Squared lattice sound speed per node, [ny][nx] of type t (LB_F32 or
 * LB_F64), on the host (on_device = 0) or device (1).  Rejects values
 * outside (0, c2_max] with LB_E_RANGE, where c2_max = 1/2 for D2Q5
 * (w0 >= 0, Appendix D) and (1 + 2r)/(2 + 2r) for D2Q9.  Synchronises the
 * stream (the range check reads the result back). */
int lb_set_medium(lb_grid *h, const void *c2, lb_dtype t, int on_device);

/* Same for the fine grid of a patch: [nyf][nxf] with nxf = 2 (patch_nx +
 * 2 overlap_out) + 1 and nyf likewise, sampled at the fine node positions
 * (coarse coordinate X0 + i/2, Y0 + j/2, X0 = patch_x0 - overlap_out). */
int lb_set_medium_fine(lb_grid *h, const void *c2, lb_dtype t, int on_device);

/* Initial state g = g^eq(rho, J) at every node at time 0 (Sec. IV first
 * bullet: initialise to equilibrium).  rho [ny][nx] required; jx, jy may be
 * NULL (zero).  Needs the medium.  Resets time to 0 and the step counter. */
int lb_set_state(lb_grid *h, const void *rho, const void *jx, const void *jy,
                 lb_dtype t, int on_device);
int lb_set_state_fine(lb_grid *h, const void *rho, const void *jx,
                      const void *jy, lb_dtype t, int on_device);

/* Point source at node (x, y) with amplitude S(n) = wavelet[n] for
 * 0 <= n < nt and 0 afterwards (host array, copied).  nt = 0 removes it.
 * The amplitude S(n) enters the collision of time n.  With a patch the
 * source must lie outside the fine grid (LB_E_UNSUPPORTED otherwise). */
int lb_set_source(lb_grid *h, int32_t x, int32_t y, const double *wavelet,
                  int64_t nt);

/* Register receivers (host array rxy[nrec][2] of (x, y), copied) and a
 * caller-owned device trace array d_traces of the arithmetic type (float for
 * LB_F32/LB_F16S, double for LB_F64), laid out [nfields][nrec][trace_capacity]
 * where the fields are the bits of `what` in the order P, RHO, JX, JY.
 * Column n receives the value at time n; times >= trace_capacity are an
 * error for lb_step_n.  With a patch, receivers inside the patch read the
 * coincident fine node at coarse times.  nrec = 0 disarms recording. */
int lb_record(lb_grid *h, const int32_t *rxy, int32_t nrec, void *d_traces,
              uint32_t what);

/* Record the sum of rho over the grid at every time into d_sum[trace_capacity]
 * (FP64, fixed reduction order, so bitwise reproducible).  NULL disarms.
 * Not available with a patch. */
int lb_record_sum_rho(lb_grid *h, double *d_sum);

/* Enqueue n time steps (coarse steps with a patch) on the bound stream and
 * return.  The first call after lb_set_state also performs the collision of
 * time 0.  Every launch fuses pull-stream, collision, source, sponge and
 * recording; a launch takes up to lb_blocked_steps() steps (see
 * steps_per_launch), and the last launch of each call takes one.  A coarse
 * step of a patch takes three launches (the coarse step with the interface
 * work, then the two fine sub-steps). */
int lb_step_n(lb_grid *h, int64_t n);

/* Graph replay of lb_step_n, for grids whose steps are too short to hide
 * the cost of issuing their launches one by one (the time loop of the
 * evolution equation, Sec. II B).  steps = 0 turns it off (the default);
 * 2 <= steps <= LB_GRAPH_MAX_STEPS makes lb_step_n run each whole chunk of
 * `steps` steps of a call as one replay of a captured HIP graph, and the
 * rest of the call as before.  A chunk's launches take the most steps the
 * multi-step kernel offers (four; three for D2Q9 FP32 and FP16 storage) or
 * one step, the last launch one step; one-step launches only where
 * steps_per_launch caps the count lower, the width is not a multiple of the
 * kernel's vector width or the sum of rho is recorded.  One small launch
 * before each replay hands the graph the chunk's first time and source
 * amplitudes, so one captured graph serves every chunk.  The graph is
 * captured on the first chunk (and again after lb_set_source, lb_record,
 * lb_record_sum_rho, lb_adjoint or lb_set_graph on the handle) and held
 * until lb_destroy_grid.  The results are the same bits as without replay.
 * Returns LB_E_RANGE for other step counts and LB_E_UNSUPPORTED for a grid
 * with a patch or one bound to the null stream (which cannot be captured);
 * while checkpoints are live, lb_step_n launches as without replay. */
#define LB_GRAPH_MAX_STEPS 256
int lb_set_graph(lb_grid *h, int32_t steps);

/* Current time n of the handle (pre-collision state at time n). */
int lb_get_time(const lb_grid *h, int64_t *n);

/* Write one field (a single LB_FIELD_* bit) of the state at the current time
 * into the device array d_out [ny][nx] of the arithmetic type. */
int lb_get_field(lb_grid *h, uint32_t what, void *d_out);
int lb_get_field_fine(lb_grid *h, uint32_t what, void *d_out);

/* Raw state for checkpoint/resume: lb_state_bytes() bytes of device memory
 * holding both population buffers and the time.  lb_set_raw_state() restores
 * it into a handle with an identical descriptor; continuing from it is
 * bitwise identical to never having stopped. */
size_t lb_state_bytes(const lb_grid *h);
int lb_get_state(lb_grid *h, void *d_out);
int lb_set_raw_state(lb_grid *h, const void *d_in);

/* Misfit of the recorded pressure traces against observed data:
 * res = p - d_obs and phi = 1/2 sum_r sum_{n <= nt} res^2 (FP64, fixed
 * summation order: block partials reduced by wave64 shuffles, then one
 * block adding them in order; the partials live in the grid's workspace).  d_obs and d_res are device arrays [nrec][trace_capacity]
 * of the arithmetic type (columns 0..nt used); d_phi one device double.
 * Needs receivers recorded with LB_FIELD_P. */
int lb_misfit(lb_grid *h, const void *d_obs, int64_t nt, void *d_res,
              double *d_phi);

/* Device workspace bytes lb_trace_misfit needs: FP64 partial sums of at
 * most 2048 blocks. */
#define LB_TRACE_MISFIT_WORKSPACE_BYTES 16384

/* The misfit of lb_misfit for trace arrays that no grid handle owns (for
 * instance the traces of shots run by the batched executor):
 * res = traces - obs and phi = 1/2 sum_r sum_{n < ncols} res^2.
 *   d_traces, d_obs, d_res  device arrays [nrec][cap] of the arithmetic type
 *                  (float for LB_F32 and LB_F16S, double for LB_F64);
 *                  columns 0 .. ncols-1 of each row are read / written.
 *   d_phi          one device double (FP64 sum in a fixed order: the result
 *                  is reproducible bit for bit).
 *   d_workspace    caller-owned device scratch of ws_bytes >=
 *                  LB_TRACE_MISFIT_WORKSPACE_BYTES, 8-byte aligned, for the
 *                  block partials; it must stay untouched until the stream
 *                  has run the call.
 * The reduction takes one partial per block of a grid-stride loop (at most
 * 2048 blocks), wave64 shuffles inside each block, and one block that adds
 * the partials in order.  Enqueued on `stream`; returns without waiting.
 * LB_E_INVALID for NULL pointers or another dtype, LB_E_RANGE unless
 * nrec >= 1 and 1 <= ncols <= cap (and nrec x cap fits int64),
 * LB_E_WORKSPACE for a missing, small or misaligned workspace, LB_E_HIP if
 * the launch fails. */
int lb_trace_misfit(const void *d_traces, const void *d_obs, void *d_res, int32_t nrec, int64_t cap,
                    int64_t ncols, lb_dtype t, double *d_phi, void *d_workspace, size_t ws_bytes, void *stream);

/* lb_trace_misfit with no workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, same kernels and the
 * same bits as lb_trace_misfit; it calls no hipMalloc, hipFree or allocating
 * routine.  The block partials live in a static device array of 2048
 * doubles (16 KiB) that every GPU the library runs on holds until the
 * process ends; its address on the GPU of `stream` is looked up once per
 * device.  That array bounds the number of blocks, not the input: any
 * nrec x ncols is reduced by the grid-stride loop; sizes are rejected only
 * as for lb_trace_misfit (LB_E_RANGE unless nrec >= 1, 1 <= ncols <= cap and
 * nrec x cap fits int64).  Every call on one GPU shares that GPU's array:
 * calls whose execution overlaps on one GPU (different streams, or several
 * host threads) race and may return wrong sums; order them on one stream or
 * synchronise between them.  The array keeps the last call's partials;
 * each call writes every partial it reads, so nothing needs clearing.
 * LB_E_HIP if the device or the array's address cannot be obtained or the
 * launch fails. */
int lb_trace_misfit_static(const void *d_traces, const void *d_obs, void *d_res, int32_t nrec, int64_t cap,
                           int64_t ncols, lb_dtype t, double *d_phi, void *stream);

/* Gradient of a trace misfit with respect to the per-node c^2 by the
 * discrete adjoint of the scheme (the paper's update differentiated exactly:
 * transpose of streaming and collision, source, sponge and receiver terms,
 * and the dependence of the initial equilibrium on the weights).
 * d_res [nrec][trace_capacity] holds dL/dp_r(n) for n = 0..nt (for the L2
 * misfit, the residual of lb_misfit); d_grad receives dL/dc^2 [ny][nx] in
 * FP64.  Needs rho_tape = 1 or ckpt_every > 0, receivers recorded, no
 * patch, and a forward run of exactly nt steps from lb_set_state (or the
 * rest state) with the same medium and source.  With the tape the backward
 * steps read the forward rho it holds and the population state is left as
 * it was.  Otherwise the forward segments are recomputed from the
 * checkpoints (as many steps per launch as lb_step_n takes), and afterwards
 * the population state is no longer the forward state, so stepping again
 * needs lb_set_state or lb_set_raw_state first.  The gradient is the same
 * bits either way and whatever steps_per_launch says. */
int lb_adjoint(lb_grid *h, const void *d_res, int64_t nt, double *d_grad);

/* Wait for all work enqueued by the handle; returns the sticky error. */
int lb_sync(lb_grid *h);

/* Static description of a status code. */
const char *lb_status_string(int code);

/* ---- batched executor (serving many shots at once) --------------------
 *
 * Many independent shots (grids of different sizes, each with its own medium,
 * source, receivers and step count) advance together.  Where the scheme has
 * a marching kernel (see lb_grid_desc) and the active shots give it enough
 * waves together (or steps_per_launch asks for it), one marching launch
 * advances every shot of a shape it takes by its step count; the other
 * shots, and every shot otherwise, take launches of up to four steps (the
 * short-segment kernel's count), a shot with fewer steps left taking those.
 * The shots' times and buffer parities live in device memory, so a tick of
 * k steps is captured once as a HIP graph and replayed until the set of
 * shots changes.  Each shot computes
 * exactly what an lb_grid with the same parameters computes (same per-node
 * update), bitwise, whatever its batch mates.  Shots start at rest.  With
 * graphs on, a fixed block of steps is captured per set of active shots and
 * replayed as often as a tick needs.
 */
typedef struct lb_batch lb_batch;

typedef struct {
    int32_t nx, ny;           /* shot grid, as lb_grid_desc                 */
    int32_t src_x, src_y;     /* source node                                */
    int64_t nsteps;           /* times 0..nsteps are computed and recorded  */
    int32_t sponge_width;     /* as lb_grid_desc                            */
    int32_t nrec;             /* receivers (traces of p only)               */
    double sponge_sigma_max;
} lb_shot_desc;

/* Device bytes of a batch with up to max_shots concurrent shots. */
size_t lb_batch_workspace_bytes(int32_t max_shots);

/* Create a batch executor.  `scheme` supplies lattice, collision, precision,
 * tau, s, d2q9_ratio and steps_per_launch (its grid, sponge, patch and
 * capacity fields are ignored; no patch).  use_graph = 1 captures ticks as HIP graphs (needs a
 * stream other than the legacy default stream), 0 launches them directly. */
int lb_batch_create(const lb_grid_desc *scheme, int32_t max_shots,
                    void *d_workspace, size_t ws_bytes, void *stream,
                    int use_graph, lb_batch **out);

/* Device bytes one shot needs: two population buffers, c^2, the wavelet
 * (nsteps + 1 doubles) and its receiver tables.  The footprint used for
 * admission; the trace buffer [nrec][nsteps + 1] is the caller's. 0 if the
 * shot description is invalid. */
size_t lb_shot_workspace_bytes(const lb_batch *b, const lb_shot_desc *s);

/* Admit a shot into a free slot: c2 [ny][nx] as for lb_set_medium (range
 * checked; a device array must be complete when the call is made), wavelet
 * S(n) for n < nt (host, copied), receivers rxy[nrec][2] (host, copied),
 * caller-owned device traces [nrec][nsteps + 1] of the arithmetic type
 * receiving p at every time (complete before the call, as c2).  Zeroes the
 * state, performs the collision of time 0 and records time 0.  The work
 * runs on an upload stream of the executor, not on `stream`: the ticks in
 * flight keep running, and the call waits only for this shot's uploads
 * (and, when every free slot was freed by a recent lb_batch_remove_shot,
 * for the ticks enqueued before that removal).  The next tick waits for
 * the admission on the device.  *slot receives the slot index.  LB_E_RANGE
 * if no slot is free. */
int lb_batch_add_shot(lb_batch *b, const lb_shot_desc *s, void *d_ws,
                      size_t ws_bytes, const void *c2, lb_dtype t,
                      int on_device, const double *wavelet, int64_t nt,
                      const int32_t *rxy, void *d_traces, int32_t *slot);

/* Retire a shot (finished or not) and free its slot; the ticks enqueued
 * after the call no longer touch the shot's workspace or traces, and those
 * enqueued before it do so only while the shot is unfinished (an
 * unfinished shot is stopped in stream order).  Returns without waiting for
 * the ticks: the caller frees the workspace and reads the traces once the
 * work enqueued so far on `stream` has run (for a finished shot, once
 * lb_batch_completed reports its last time).  */
int lb_batch_remove_shot(lb_batch *b, int32_t slot);

/* Enqueue k time steps for every active shot; shots that reach their last
 * time stop updating inside the tick.  Returns without waiting.  Each tick
 * advances every active shot by min(k, steps left). */
int lb_batch_tick(lb_batch *b, int64_t k);

/* Time every slot reaches once the enqueued ticks have run (host array of
 * max_shots; -1 for free slots).  Returns without waiting. */
int lb_batch_times(lb_batch *b, int64_t *t_out);

/* Time every slot has reached on the device: that of the newest tick known
 * to have completed (host array of max_shots; -1 for free slots and for
 * shots no tick has completed since their admission).  Returns without
 * waiting (it polls the ticks' completion events). */
int lb_batch_completed(lb_batch *b, int64_t *t_out);

/* Wait for all enqueued work; returns the sticky error. */
int lb_batch_sync(lb_batch *b);

/* Release the executor (not the workspaces).  NULL-safe. */
int lb_batch_destroy(lb_batch *b);

/* Plain device copy of `bytes` bytes (16-byte nontemporal vector loads and
 * stores) on a stream: the measured reference for attainable HBM bandwidth.
 * Both pointers 16-byte aligned, bytes a multiple of 16. */
int lb_device_copy(void *d_dst, const void *d_src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBWAVE_H */
