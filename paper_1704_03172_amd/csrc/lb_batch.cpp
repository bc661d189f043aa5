// lb_batch.cpp -- batched executor behind the lb_batch_* calls of
// include/lbwave.h: many independent shots of the linear LB scheme advance
// together, in rounds of the marching kernel's step count where the scheme
// has one (every shot of a shape it takes, with that many steps left, in one
// marching launch) and otherwise up to four steps per launch (the
// temporally blocked kernel; one step per launch for the configuration it
// does not serve),
// with per-shot time and buffer parity kept on the device so that a tick of
// k steps is captured once as a HIP graph and replayed until the set of
// active shots changes.
#include "lbwave.h"
#include "lb_host.h"
#include "lb_internal.h"

#include <algorithm>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

namespace {

constexpr int64_t kGraphSteps = 16;      // steps per captured graph (at least; see graph_steps)
constexpr size_t kStageBytes = 4 << 20;  // pinned staging of the uploads
constexpr int kTickEvents = 64;          // ticks whose completion can be tracked at once

using lbw::align_up;
using lbw::BatchParams;
using lbw::ShotEntry;
using lbw::ShotState;

// Per-set device tables of the active shots (two sets: a rebuild writes the
// set that no tick in flight reads).
struct SetLayout {
    size_t order = 0, prefix = 0, wprefix = 0, mprefix = 0;
};

struct BatchLayout {
    size_t table = 0, state = 0, img = 0, scratch = 0, total = 0;
    SetLayout set[2];
};

BatchLayout batch_layout(int32_t max_shots) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.table = take((size_t)max_shots * sizeof(ShotEntry));
    L.state = take((size_t)max_shots * sizeof(ShotState));
    for (SetLayout &t : L.set) {
        t.order = take((size_t)max_shots * sizeof(int32_t));
        t.prefix = take(((size_t)max_shots + 1) * sizeof(int64_t));
        t.wprefix = take(((size_t)max_shots + 1) * sizeof(int64_t));
        t.mprefix = take(((size_t)max_shots + 1) * sizeof(int64_t));
    }
    L.img = take((size_t)max_shots * sizeof(lbw::StepParams));
    L.scratch = take(256);
    L.total = off;
    return L;
}

struct ShotLayout {
    int64_t pstride = 0;
    size_t pop0 = 0, pop1 = 0, c2 = 0, wavelet = 0, rrow = 0, rxs = 0, rslot = 0, total = 0;
};

struct DeviceSet {
    int32_t *order = nullptr;
    int64_t *prefix = nullptr, *wprefix = nullptr, *mprefix = nullptr;
};

// A tick whose completion is tracked: its event and the host times of every
// slot once it has run (-1: free).
struct TickRecord {
    int64_t id = 0;
    std::vector<int64_t> t;
};

}  // namespace

struct lb_batch {
    lb_grid_desc scheme;
    int q = 5, storage = 0;
    size_t ssize = 4, tsize = 4;
    lbw::Collision coll;
    hipStream_t stream = nullptr;      // ticks
    hipStream_t up = nullptr;          // admission and table uploads
    int use_graph = 0;
    int32_t max_shots = 0;
    ShotEntry *d_table = nullptr;
    ShotState *d_state = nullptr;
    lbw::StepParams *d_img = nullptr;
    int32_t *d_scratch = nullptr;
    DeviceSet dset[2];
    int set = 0;                       // the set the next ticks read
    hipEvent_t ev_set[2] = {nullptr, nullptr};   // last tick that read each set
    hipEvent_t ev_up = nullptr;        // uploads the next tick must wait for
    bool up_pending = false;
    std::vector<hipEvent_t> ev_slot;   // per slot: work enqueued when it was freed
    char *stage = nullptr;             // pinned staging (reused once `up` is idle)
    std::vector<ShotEntry> table;
    std::vector<char> used;
    std::vector<int64_t> ht, hend;     // host-tracked time and last time per slot
    std::vector<int64_t> admit_tick;   // tick counter when the slot's shot was admitted
    std::vector<int32_t> order;
    std::vector<int64_t> prefix, wprefix, mprefix;
    int64_t total_blocks = 0, total_waves = 0, total_mwaves = 0;
    int ns = 1;                        // steps per launch (blocked kernel if > 1)
    int nsm = 0;                       // steps of a marching round (0: none)
    int64_t min_mwaves = 0;            // fewest marching waves for a marching round
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<char> graph_sig;       // per round of the graph: the round's short-shot launches
    // tick completion
    hipEvent_t ev_tick[kTickEvents] = {};
    std::deque<TickRecord> pending;    // enqueued ticks, oldest first
    TickRecord done;                   // the newest completed tick
    int64_t ticks = 0;
    int sticky = LB_OK;
};

namespace {

int fail(lb_batch *b, hipError_t e) {
    if (e == hipSuccess) return LB_OK;
    b->sticky = LB_E_HIP;
    return LB_E_HIP;
}

#define BT_TRY(b, expr)                               \
    do {                                              \
        hipError_t e__ = (expr);                      \
        if (e__ != hipSuccess) return fail((b), e__); \
    } while (0)

int check_shot(const lb_shot_desc *s) {
    if (!s) return LB_E_INVALID;
    if (s->nx < 1 || s->ny < 1 || s->ny > 65535 || s->nx > (1 << 24)) return LB_E_RANGE;
    if (s->nsteps < 0 || s->nrec < 0) return LB_E_RANGE;
    if (s->src_x < 0 || s->src_y < 0 || s->src_x >= s->nx || s->src_y >= s->ny) return LB_E_RANGE;
    if (s->sponge_width < 0 || !(s->sponge_sigma_max >= 0.0 && s->sponge_sigma_max <= 1.0)) return LB_E_RANGE;
    return LB_OK;
}

ShotLayout shot_layout(const lb_batch *b, const lb_shot_desc *s) {
    ShotLayout L;
    const int64_t n = (int64_t)s->nx * s->ny;
    L.pstride = lbw::population_stride(n);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.pop0 = take((size_t)b->q * L.pstride * b->ssize);
    L.pop1 = take((size_t)b->q * L.pstride * b->ssize);
    L.c2 = take((size_t)n * b->tsize);
    L.wavelet = take(((size_t)s->nsteps + 1) * sizeof(double));
    L.rrow = take(((size_t)s->ny + 1) * 4);
    L.rxs = take((size_t)std::max(s->nrec, 1) * 4);
    L.rslot = take((size_t)std::max(s->nrec, 1) * 4);
    L.total = off;
    return L;
}

// Staged copy to the device on the upload stream: host bytes go through the
// pinned staging buffer at *off (advanced), so the copy runs without the
// host waiting on it (a pageable source would make the call wait).
int stage_copy(lb_batch *b, void *dst, const void *src, size_t bytes, size_t *off) {
    if (bytes == 0) return LB_OK;
    if (*off + bytes > kStageBytes) {   // full: let the uploads so far finish
        BT_TRY(b, hipStreamSynchronize(b->up));
        *off = 0;
    }
    std::memcpy(b->stage + *off, src, bytes);
    BT_TRY(b, hipMemcpyAsync(dst, b->stage + *off, bytes, hipMemcpyHostToDevice, b->up));
    *off = align_up(*off + bytes);
    return LB_OK;
}

// Rebuild the compact list of active shots and their wave prefix sums into
// the set that no tick in flight reads, on the upload stream after the last
// tick that read it; the ticks enqueued from now on read it once the upload
// is done.  *off: staging offset in use.
int rebuild(lb_batch *b, size_t *off) {
    b->order.clear();
    b->prefix.assign(1, 0);
    b->wprefix.assign(1, 0);
    b->mprefix.assign(1, 0);
    const int kind = lbw::step_kind(b->coll);
    for (int32_t k = 0; k < b->max_shots; ++k) {
        if (!b->used[(size_t)k]) continue;
        const ShotEntry &e = b->table[(size_t)k];
        b->order.push_back(k);
        b->prefix.push_back(b->prefix.back() + (int64_t)e.bx * e.ny);
        if (b->ns > 1) b->wprefix.push_back(b->wprefix.back() + lbw::stepn_waves(b->storage, b->q, kind, b->ns, e.nx, e.ny));
        b->mprefix.push_back(b->mprefix.back() + (e.march ? lbw::stepn_march_waves(b->storage, b->q, kind, e.nx, e.ny) : 0));
    }
    b->total_blocks = b->prefix.back();
    b->total_waves = b->ns > 1 ? b->wprefix.back() : 0;
    b->total_mwaves = b->nsm > 0 ? b->mprefix.back() : 0;
    const int ns = 1 - b->set;
    const DeviceSet &d = b->dset[ns];
    BT_TRY(b, hipStreamWaitEvent(b->up, b->ev_set[ns], 0));
    int rc;
    if (!b->order.empty()) {
        if ((rc = stage_copy(b, d.order, b->order.data(), b->order.size() * 4, off))) return rc;
        if ((rc = stage_copy(b, d.prefix, b->prefix.data(), b->prefix.size() * 8, off))) return rc;
        if (b->ns > 1 && (rc = stage_copy(b, d.wprefix, b->wprefix.data(), b->wprefix.size() * 8, off))) return rc;
        if ((rc = stage_copy(b, d.mprefix, b->mprefix.data(), b->mprefix.size() * 8, off))) return rc;
    }
    BT_TRY(b, hipEventRecord(b->ev_up, b->up));
    b->up_pending = true;
    b->set = ns;
    b->dirty = true;
    return LB_OK;
}

BatchParams params(const lb_batch *b) {
    const DeviceSet &d = b->dset[b->set];
    BatchParams p;
    p.table = b->d_table;
    p.state = b->d_state;
    p.prefix = d.prefix;
    p.wprefix = d.wprefix;
    p.order = d.order;
    p.nact = (int32_t)b->order.size();
    p.coll = b->coll;
    p.mprefix = d.mprefix;
    return p;
}

// One batched launch of up to `run` steps (the blocked kernel, or one step)
// for the shots it takes, and their state update (sel = 2 in a marching
// round: only the shots outside the marching launch).
int enqueue_launch(lb_batch *b, BatchParams &p, int run, int sel) {
    if (run > 1) {
        p.max_run = run;
        BT_TRY(b, lbw::launch_stepn_batch(b->storage, b->q, b->ns, p, b->total_waves, b->stream));
    } else {
        BT_TRY(b, lbw::launch_step_batch(b->storage, b->q, p, b->total_blocks, b->stream));
    }
    if (sel) BT_TRY(b, lbw::launch_batch_advance_sel(b->d_state, p.order, p.nact, b->d_img, sel, run, b->stream));
    else if (run > 1) BT_TRY(b, lbw::launch_batch_advance_n(b->d_state, p.order, p.nact, run, b->stream));
    else BT_TRY(b, lbw::launch_batch_advance(b->d_state, p.order, p.nact, b->stream));
    return LB_OK;
}

// Whether the marching rounds of the next k steps need the launches for
// shots outside the marching launch, one flag per round, from the host
// times (a shot whose shape the marching kernel does not take, or one with
// fewer than nsm steps left at the round).  No marching rounds (an empty
// list) while the active shots give the marching launch fewer waves than
// fill the GPU: the short-segment launches are faster then.
std::vector<char> round_needs(const lb_batch *b, int64_t k) {
    std::vector<char> need;
    if (b->nsm <= 0 || b->total_mwaves <= 0 || b->total_mwaves < b->min_mwaves) return need;
    std::vector<int64_t> t(b->ht);
    for (int64_t r = 0; r + b->nsm <= k; r += b->nsm) {
        char nd = 0;
        for (int32_t s : b->order) {
            const int64_t left = b->hend[(size_t)s] - t[(size_t)s];
            if (left > 0 && (!b->table[(size_t)s].march || left < b->nsm)) nd = 1;
            t[(size_t)s] += std::min<int64_t>(std::max<int64_t>(left, 0), b->nsm);
        }
        need.push_back(nd);
    }
    return need;
}

// k steps of every active shot (a shot stops at its last step).  Rounds of
// nsm steps while k allows: the shots that the marching kernel takes and
// that have nsm steps left run in one marching launch, the others (where
// `need` says there are any) in launches of up to ns steps; the rest of k
// in launches of ns steps, the remainder in one shorter blocked launch (or,
// with one step left or no blocked kernel, one-step launches).  Every shot
// advances by min(k, steps left) either way.
int enqueue_steps(lb_batch *b, int64_t k, const std::vector<char> &need) {
    BatchParams p = params(b);
    int rc;
    size_t r = 0;
    while (r < need.size() && k >= b->nsm) {
        p.img = b->d_img;
        BT_TRY(b, lbw::launch_batch_march_prep(b->q, p, b->nsm, b->stream));
        BT_TRY(b, lbw::launch_stepn_march_batch(b->storage, b->q, p, b->total_mwaves, b->stream));
        BT_TRY(b, lbw::launch_batch_advance_sel(b->d_state, p.order, p.nact, b->d_img, 1, b->nsm, b->stream));
        if (need[r])
            for (int done = 0; done < b->nsm;) {
                const int run = std::min(b->ns, b->nsm - done);
                if ((rc = enqueue_launch(b, p, run, 2))) return rc;
                done += run;
            }
        p.img = nullptr;
        k -= b->nsm;
        ++r;
    }
    while (k > 0) {
        const int run = (int)std::min<int64_t>(b->ns, k);
        if ((rc = enqueue_launch(b, p, run, 0))) return rc;
        k -= run;
    }
    return LB_OK;
}

void drop_graph(lb_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Steps per captured graph: kGraphSteps rounded up to whole marching rounds.
int64_t graph_steps(const lb_batch *b) {
    return b->nsm > 1 ? (kGraphSteps + b->nsm - 1) / b->nsm * b->nsm : kGraphSteps;
}

int capture(lb_batch *b, const std::vector<char> &need) {
    drop_graph(b);
    BT_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_steps(b, graph_steps(b), need);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    BT_TRY(b, e);
    b->graph = g;
    BT_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_sig = need;
    b->dirty = false;
    return LB_OK;
}

// Host times after k more steps of every active shot.
void advance_host(lb_batch *b, int64_t k) {
    for (int32_t s : b->order) {
        int64_t &t = b->ht[(size_t)s];
        t = std::min(t + k, b->hend[(size_t)s]);
    }
}

// Retire the records of the ticks that have completed (non-blocking).
int collect(lb_batch *b) {
    while (!b->pending.empty()) {
        const hipError_t e = hipEventQuery(b->ev_tick[b->pending.front().id % kTickEvents]);
        if (e == hipErrorNotReady) break;
        BT_TRY(b, e);
        b->done = std::move(b->pending.front());
        b->pending.pop_front();
    }
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lb_batch_workspace_bytes(int32_t max_shots) {
    if (max_shots < 1 || max_shots > (1 << 16)) return 0;
    return batch_layout(max_shots).total;
}

int lb_batch_create(const lb_grid_desc *scheme, int32_t max_shots, void *d_workspace, size_t ws_bytes,
                    void *stream, int use_graph, lb_batch **out) {
    if (!out || !scheme) return LB_E_INVALID;
    *out = nullptr;
    int rc = lbw::validate_scheme(scheme);
    if (rc) return rc;
    if (max_shots < 1 || max_shots > (1 << 16)) return LB_E_RANGE;
    BatchLayout L = batch_layout(max_shots);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255u)) return LB_E_WORKSPACE;
    lb_batch *b = new (std::nothrow) lb_batch();
    if (!b) return LB_E_INVALID;
    b->scheme = *scheme;
    b->q = scheme->lattice;
    b->storage = lbw::storage_kind(scheme->precision);
    b->ssize = lbw::storage_bytes(scheme->precision);
    b->tsize = lbw::compute_bytes(scheme->precision);
    b->coll = lbw::make_collision(scheme);
    b->stream = (hipStream_t)stream;
    b->use_graph = use_graph ? 1 : 0;
    b->max_shots = max_shots;
    b->ns = lbw::stepn_max(b->storage, b->q, b->coll.kind);
    if (scheme->steps_per_launch > 0) b->ns = std::min(b->ns, scheme->steps_per_launch);
    // marching rounds: the marching kernel's step count for this scheme (a
    // shape it takes), unless steps_per_launch caps it lower
    // and, as for a single grid, a cap at or above that count asks for the
    // marching rounds however few waves the active shots give them
    b->nsm = lbw::stepn_march(b->storage, b->q, lbw::step_kind(b->coll), 1024, 1024);
    b->min_mwaves = lbw::stepn_march_min_waves(b->storage, b->q, lbw::step_kind(b->coll));
    if (scheme->steps_per_launch > 0 && scheme->steps_per_launch < b->nsm) b->nsm = 0;
    if (scheme->steps_per_launch > 0) b->min_mwaves = 0;
    char *ws = (char *)d_workspace;
    b->d_table = (ShotEntry *)(ws + L.table);
    b->d_state = (ShotState *)(ws + L.state);
    b->d_img = (lbw::StepParams *)(ws + L.img);
    b->d_scratch = (int32_t *)(ws + L.scratch);
    for (int i = 0; i < 2; ++i) {
        b->dset[i].order = (int32_t *)(ws + L.set[i].order);
        b->dset[i].prefix = (int64_t *)(ws + L.set[i].prefix);
        b->dset[i].wprefix = (int64_t *)(ws + L.set[i].wprefix);
        b->dset[i].mprefix = (int64_t *)(ws + L.set[i].mprefix);
    }
    b->table.assign((size_t)max_shots, ShotEntry());
    b->used.assign((size_t)max_shots, 0);
    b->ht.assign((size_t)max_shots, 0);
    b->hend.assign((size_t)max_shots, 0);
    b->admit_tick.assign((size_t)max_shots, 0);
    b->ev_slot.assign((size_t)max_shots, nullptr);
    bool ok = hipStreamCreateWithFlags(&b->up, hipStreamNonBlocking) == hipSuccess &&
              hipHostMalloc((void **)&b->stage, kStageBytes, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev_up, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < 2; ++i) ok = hipEventCreateWithFlags(&b->ev_set[i], hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < kTickEvents; ++i)
        ok = hipEventCreateWithFlags(&b->ev_tick[i], hipEventDisableTiming) == hipSuccess;
    for (int32_t i = 0; ok && i < max_shots; ++i)
        ok = hipEventCreateWithFlags(&b->ev_slot[(size_t)i], hipEventDisableTiming) == hipSuccess;
    // zeroed slot states; the set events mark that nothing reads either set
    ok = ok && lbw::launch_fill_zero(ws + L.state, (int64_t)((size_t)max_shots * sizeof(ShotState)), b->stream) ==
                   hipSuccess;
    for (int i = 0; ok && i < 2; ++i) ok = hipEventRecord(b->ev_set[i], b->stream) == hipSuccess;
    for (int32_t i = 0; ok && i < max_shots; ++i) ok = hipEventRecord(b->ev_slot[(size_t)i], b->stream) == hipSuccess;
    ok = ok && hipStreamSynchronize(b->stream) == hipSuccess;
    b->done.t.assign((size_t)max_shots, -1);
    if (!ok) {
        lb_batch_destroy(b);
        return LB_E_HIP;
    }
    *out = b;
    return LB_OK;
}

size_t lb_shot_workspace_bytes(const lb_batch *b, const lb_shot_desc *s) {
    if (!b || check_shot(s) != LB_OK) return 0;
    return shot_layout(b, s).total;
}

int lb_batch_add_shot(lb_batch *b, const lb_shot_desc *s, void *d_ws, size_t ws_bytes, const void *c2, lb_dtype t,
                      int on_device, const double *wavelet, int64_t nt, const int32_t *rxy, void *d_traces,
                      int32_t *slot) {
    if (!b || !slot || !c2) return LB_E_INVALID;
    *slot = -1;
    if (b->sticky) return b->sticky;
    int rc = check_shot(s);
    if (rc) return rc;
    if (t != LB_F32 && t != LB_F64) return LB_E_INVALID;
    if (nt < 0 || (nt > 0 && !wavelet)) return LB_E_INVALID;
    if (s->nrec > 0 && (!rxy || !d_traces)) return LB_E_INVALID;
    ShotLayout L = shot_layout(b, s);
    if (!d_ws || ws_bytes < L.total || ((uintptr_t)d_ws & 255u)) return LB_E_WORKSPACE;
    for (int32_t r = 0; r < s->nrec; ++r)
        if (rxy[2 * r] < 0 || rxy[2 * r + 1] < 0 || rxy[2 * r] >= s->nx || rxy[2 * r + 1] >= s->ny) return LB_E_RANGE;
    // a free slot, preferring one whose last ticks have run
    int32_t k = -1;
    for (int32_t i = 0; i < b->max_shots; ++i) {
        if (b->used[(size_t)i]) continue;
        if (k < 0) k = i;
        if (hipEventQuery(b->ev_slot[(size_t)i]) == hipSuccess) {
            k = i;
            break;
        }
    }
    if (k < 0) return LB_E_RANGE;

    // everything below runs on the upload stream, so the ticks in flight
    // keep the GPU busy; the host waits only for this shot's uploads (the
    // range check of c^2)
    BT_TRY(b, hipStreamSynchronize(b->up));   // the staging buffer is free
    size_t off = 0;
    char *ws = (char *)d_ws;
    const int64_t n = (int64_t)s->nx * s->ny;
    if ((rc = lbw::upload_c2(b->up, b->scheme.precision, b->q, b->scheme.d2q9_ratio, ws + L.c2, c2, t, on_device,
                             n, b->d_scratch))) {
        if (rc == LB_E_HIP) b->sticky = LB_E_HIP;
        return rc;
    }
    BT_TRY(b, lbw::launch_fill_zero(ws + L.pop0, (int64_t)(L.c2 - L.pop0), b->up));
    const int64_t nw = std::min<int64_t>(nt, s->nsteps + 1);
    if (nw > 0 && (rc = stage_copy(b, ws + L.wavelet, wavelet, (size_t)nw * 8, &off))) return rc;

    // receiver tables: CSR over rows, x ascending
    struct R { int32_t x, y, slot; };
    std::vector<R> v((size_t)s->nrec);
    for (int32_t r = 0; r < s->nrec; ++r) v[(size_t)r] = {rxy[2 * r], rxy[2 * r + 1], r};
    std::sort(v.begin(), v.end(), [](const R &a, const R &c) {
        return a.y != c.y ? a.y < c.y : (a.x != c.x ? a.x < c.x : a.slot < c.slot);
    });
    std::vector<int32_t> row((size_t)s->ny + 1, 0), xs(v.size()), sl(v.size());
    for (const R &r : v) row[(size_t)r.y + 1]++;
    for (int32_t y = 0; y < s->ny; ++y) row[(size_t)y + 1] += row[(size_t)y];
    for (size_t i = 0; i < v.size(); ++i) {
        xs[i] = v[i].x;
        sl[i] = v[i].slot;
    }
    if (s->nrec > 0) {
        if ((rc = stage_copy(b, ws + L.rrow, row.data(), row.size() * 4, &off))) return rc;
        if ((rc = stage_copy(b, ws + L.rxs, xs.data(), xs.size() * 4, &off))) return rc;
        if ((rc = stage_copy(b, ws + L.rslot, sl.data(), sl.size() * 4, &off))) return rc;
    }

    ShotEntry e;
    e.pop0 = ws + L.pop0;
    e.pop1 = ws + L.pop1;
    e.c2 = ws + L.c2;
    e.wavelet = (const double *)(ws + L.wavelet);
    e.wavelet_len = nw;
    if (s->nrec > 0) {
        e.rec.row_ptr = (const int32_t *)(ws + L.rrow);
        e.rec.xs = (const int32_t *)(ws + L.rxs);
        e.rec.slot = (const int32_t *)(ws + L.rslot);
        e.rec.traces = d_traces;
        e.rec.nslots = s->nrec;
        e.rec.what = LB_FIELD_P;
        e.rec.cap = s->nsteps + 1;
    }
    e.nx = s->nx;
    e.ny = s->ny;
    e.pstride = L.pstride;
    e.sponge_width = s->sponge_width;
    e.sponge_smax = s->sponge_sigma_max;
    e.src_x = s->src_x;
    e.src_y = s->src_y;
    const int64_t tile = lbw::step_tile_nodes(b->storage);
    e.bx = (int32_t)(((int64_t)s->nx + tile - 1) / tile);
    e.march = b->nsm > 0 && lbw::stepn_march(b->storage, b->q, lbw::step_kind(b->coll), s->nx, s->ny) == b->nsm;

    // collision of time 0 (records time 0): pop0 (at rest) -> pop1
    lbw::StepParams p;
    p.src = e.pop0;
    p.dst = e.pop1;
    p.c2 = e.c2;
    p.nx = e.nx;
    p.ny = e.ny;
    p.pstride = e.pstride;
    p.q = b->q;
    p.coll = b->coll;
    p.sponge_width = e.sponge_width;
    p.sponge_smax = e.sponge_smax;
    p.src_x = e.src_x;
    p.src_y = e.src_y;
    p.s_n = nw > 0 ? wavelet[0] : 0.0;
    p.rec = e.rec;
    p.rec.col = 0;
    BT_TRY(b, lbw::launch_step(b->storage, p, false, b->up));

    // the slot's table entry and state, once no tick in flight can read the
    // slot's previous shot
    ShotState st;
    st.t = 0;
    st.t_end = s->nsteps;
    st.cur = 1;
    st.active = 1;
    BT_TRY(b, hipStreamWaitEvent(b->up, b->ev_slot[(size_t)k], 0));
    if ((rc = stage_copy(b, b->d_table + k, &e, sizeof(e), &off))) return rc;
    if ((rc = stage_copy(b, b->d_state + k, &st, sizeof(st), &off))) return rc;
    b->table[(size_t)k] = e;
    b->used[(size_t)k] = 1;
    b->ht[(size_t)k] = 0;
    b->hend[(size_t)k] = s->nsteps;
    b->admit_tick[(size_t)k] = b->ticks;
    if ((rc = rebuild(b, &off))) return rc;
    *slot = k;
    return LB_OK;
}

int lb_batch_remove_shot(lb_batch *b, int32_t slot) {
    if (!b) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    if (slot < 0 || slot >= b->max_shots || !b->used[(size_t)slot]) return LB_E_RANGE;
    // an unfinished shot stops in stream order; the slot stays reserved until
    // the work enqueued so far (which may still read it) has run
    if (b->ht[(size_t)slot] < b->hend[(size_t)slot])
        BT_TRY(b, lbw::launch_fill_zero(&b->d_state[slot].active, 4, b->stream));
    BT_TRY(b, hipEventRecord(b->ev_slot[(size_t)slot], b->stream));
    b->used[(size_t)slot] = 0;
    b->table[(size_t)slot] = ShotEntry();
    BT_TRY(b, hipStreamSynchronize(b->up));   // the staging buffer is free
    size_t off = 0;
    return rebuild(b, &off);
}

int lb_batch_tick(lb_batch *b, int64_t k) {
    if (!b) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    if (k < 0) return LB_E_RANGE;
    if (k == 0 || b->order.empty()) return LB_OK;
    if ((int64_t)b->pending.size() >= kTickEvents) {   // the oldest tracked tick must have run
        BT_TRY(b, hipEventSynchronize(b->ev_tick[b->pending.front().id % kTickEvents]));
        int rc = collect(b);
        if (rc) return rc;
    }
    if (b->up_pending) {   // the tables and shots uploaded since the last tick
        BT_TRY(b, hipStreamWaitEvent(b->stream, b->ev_up, 0));
        b->up_pending = false;
    }
    int rc;
    if (!b->use_graph) {
        if ((rc = enqueue_steps(b, k, round_needs(b, k)))) return rc;
        advance_host(b, k);
    } else {
        // graphs of graph_steps() steps, captured again when the set of
        // active shots changes or a round's short-shot launches come or go,
        // and replayed; the remainder of k runs as direct launches
        const int64_t gs = graph_steps(b);
        for (int64_t i = 0; i < k / gs; ++i) {
            const std::vector<char> need = round_needs(b, gs);
            if (b->dirty || !b->exec || need != b->graph_sig)
                if ((rc = capture(b, need))) return rc;
            BT_TRY(b, hipGraphLaunch(b->exec, b->stream));
            advance_host(b, gs);
        }
        const int64_t r = k % gs;
        if ((rc = enqueue_steps(b, r, round_needs(b, r)))) return rc;
        advance_host(b, r);
    }
    BT_TRY(b, hipEventRecord(b->ev_set[b->set], b->stream));
    TickRecord rec;
    rec.id = ++b->ticks;
    rec.t.assign((size_t)b->max_shots, -1);
    for (int32_t s : b->order) rec.t[(size_t)s] = b->ht[(size_t)s];
    BT_TRY(b, hipEventRecord(b->ev_tick[rec.id % kTickEvents], b->stream));
    b->pending.push_back(std::move(rec));
    return LB_OK;
}

int lb_batch_times(lb_batch *b, int64_t *t_out) {
    if (!b || !t_out) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    for (int32_t k = 0; k < b->max_shots; ++k) t_out[k] = b->used[(size_t)k] ? b->ht[(size_t)k] : -1;
    return LB_OK;
}

int lb_batch_completed(lb_batch *b, int64_t *t_out) {
    if (!b || !t_out) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    int rc = collect(b);
    if (rc) return rc;
    for (int32_t k = 0; k < b->max_shots; ++k) {
        const bool valid = b->used[(size_t)k] && b->done.id > b->admit_tick[(size_t)k] && !b->done.t.empty();
        t_out[k] = valid ? b->done.t[(size_t)k] : -1;
    }
    return LB_OK;
}

int lb_batch_sync(lb_batch *b) {
    if (!b) return LB_E_INVALID;
    if (hipStreamSynchronize(b->up) != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
        b->sticky = LB_E_HIP;
    if (!b->sticky) (void)collect(b);
    return b->sticky;
}

int lb_batch_destroy(lb_batch *b) {
    if (!b) return LB_OK;
    hipError_t e = hipSuccess;
    if (b->stream || b->up) {
        const hipError_t e1 = b->up ? hipStreamSynchronize(b->up) : hipSuccess;
        const hipError_t e2 = hipStreamSynchronize(b->stream);
        e = e1 != hipSuccess ? e1 : e2;
    }
    drop_graph(b);
    for (hipEvent_t &ev : b->ev_tick)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : b->ev_slot)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : b->ev_set)
        if (ev) (void)hipEventDestroy(ev);
    if (b->ev_up) (void)hipEventDestroy(b->ev_up);
    if (b->stage) (void)hipHostFree(b->stage);
    if (b->up) (void)hipStreamDestroy(b->up);
    int rc = b->sticky ? b->sticky : (e == hipSuccess ? LB_OK : LB_E_HIP);
    delete b;
    return rc;
}

}  // extern "C"
