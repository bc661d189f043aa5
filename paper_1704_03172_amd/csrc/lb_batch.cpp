// lb_batch.cpp -- batched executor behind the lb_batch_* calls of
// include/lbwave.h: many independent shots of the linear LB scheme advance
// together, up to four steps per launch (the temporally blocked kernel;
// one step per launch for the configuration it does not serve),
// with per-shot time and buffer parity kept on the device so that a tick of
// k steps is captured once as a HIP graph and replayed until the set of
// active shots changes.
#include "lbwave.h"
#include "lb_host.h"
#include "lb_internal.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int64_t kGraphSteps = 16;   // steps per captured graph

using lbw::align_up;
using lbw::BatchParams;
using lbw::ShotEntry;
using lbw::ShotState;

struct BatchLayout {
    size_t table = 0, state = 0, prefix = 0, wprefix = 0, order = 0, scratch = 0, total = 0;
};

BatchLayout batch_layout(int32_t max_shots) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.table = take((size_t)max_shots * sizeof(ShotEntry));
    L.state = take((size_t)max_shots * sizeof(ShotState));
    L.prefix = take(((size_t)max_shots + 1) * sizeof(int64_t));
    L.wprefix = take(((size_t)max_shots + 1) * sizeof(int64_t));
    L.order = take((size_t)max_shots * sizeof(int32_t));
    L.scratch = take(256);
    L.total = off;
    return L;
}

struct ShotLayout {
    int64_t pstride = 0;
    size_t pop0 = 0, pop1 = 0, c2 = 0, wavelet = 0, rrow = 0, rxs = 0, rslot = 0, total = 0;
};

}  // namespace

struct lb_batch {
    lb_grid_desc scheme;
    int q = 5, storage = 0;
    size_t ssize = 4, tsize = 4;
    lbw::Collision coll;
    hipStream_t stream = nullptr;
    int use_graph = 0;
    int32_t max_shots = 0;
    ShotEntry *d_table = nullptr;
    ShotState *d_state = nullptr;
    int64_t *d_prefix = nullptr;
    int64_t *d_wprefix = nullptr;
    int32_t *d_order = nullptr;
    int32_t *d_scratch = nullptr;
    std::vector<ShotEntry> table;
    std::vector<char> used;
    std::vector<int32_t> order;
    std::vector<int64_t> prefix, wprefix;
    int64_t total_blocks = 0, total_waves = 0;
    int ns = 1;                        // steps per launch (blocked kernel if > 1)
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_k = 0;
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

// Rebuild the compact list of active shots and their block prefix sums, and
// upload both (stream-ordered before any later tick).
int rebuild(lb_batch *b) {
    b->order.clear();
    b->prefix.assign(1, 0);
    b->wprefix.assign(1, 0);
    for (int32_t k = 0; k < b->max_shots; ++k) {
        if (!b->used[(size_t)k]) continue;
        const ShotEntry &e = b->table[(size_t)k];
        b->order.push_back(k);
        b->prefix.push_back(b->prefix.back() + (int64_t)e.bx * e.ny);
        if (b->ns > 1) b->wprefix.push_back(b->wprefix.back() + lbw::stepn_waves(b->storage, b->q, lbw::step_kind(b->coll), b->ns, e.nx, e.ny));
    }
    b->total_blocks = b->prefix.back();
    b->total_waves = b->ns > 1 ? b->wprefix.back() : 0;
    if (!b->order.empty()) {
        BT_TRY(b, hipMemcpyAsync(b->d_order, b->order.data(), b->order.size() * 4, hipMemcpyHostToDevice, b->stream));
        BT_TRY(b, hipMemcpyAsync(b->d_prefix, b->prefix.data(), b->prefix.size() * 8, hipMemcpyHostToDevice,
                                 b->stream));
        if (b->ns > 1)
            BT_TRY(b, hipMemcpyAsync(b->d_wprefix, b->wprefix.data(), b->wprefix.size() * 8, hipMemcpyHostToDevice,
                                     b->stream));
    }
    BT_TRY(b, hipStreamSynchronize(b->stream));
    b->dirty = true;
    return LB_OK;
}

BatchParams params(const lb_batch *b) {
    BatchParams p;
    p.table = b->d_table;
    p.state = b->d_state;
    p.prefix = b->d_prefix;
    p.wprefix = b->d_wprefix;
    p.order = b->d_order;
    p.nact = (int32_t)b->order.size();
    p.coll = b->coll;
    return p;
}

// k steps of every active shot (a shot stops at its last step): launches of
// ns steps, the remainder of k in one shorter blocked launch (or, with one
// step left or no blocked kernel, one-step launches).
int enqueue_steps(lb_batch *b, int64_t k) {
    BatchParams p = params(b);
    while (k > 0) {
        const int run = (int)std::min<int64_t>(b->ns, k);
        if (run > 1) {
            p.max_run = run;
            BT_TRY(b, lbw::launch_stepn_batch(b->storage, b->q, b->ns, p, b->total_waves, b->stream));
            BT_TRY(b, lbw::launch_batch_advance_n(b->d_state, b->d_order, p.nact, run, b->stream));
        } else {
            BT_TRY(b, lbw::launch_step_batch(b->storage, b->q, p, b->total_blocks, b->stream));
            BT_TRY(b, lbw::launch_batch_advance(b->d_state, b->d_order, p.nact, b->stream));
        }
        k -= run;
    }
    return LB_OK;
}

void drop_graph(lb_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_k = 0;
}

int capture(lb_batch *b, int64_t k) {
    drop_graph(b);
    BT_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_steps(b, k);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    BT_TRY(b, e);
    b->graph = g;
    BT_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_k = k;
    b->dirty = false;
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
    char *ws = (char *)d_workspace;
    b->d_table = (ShotEntry *)(ws + L.table);
    b->d_state = (ShotState *)(ws + L.state);
    b->d_prefix = (int64_t *)(ws + L.prefix);
    b->d_wprefix = (int64_t *)(ws + L.wprefix);
    b->d_order = (int32_t *)(ws + L.order);
    b->d_scratch = (int32_t *)(ws + L.scratch);
    b->table.assign((size_t)max_shots, ShotEntry());
    b->used.assign((size_t)max_shots, 0);
    if (lbw::launch_fill_zero(ws + L.state, (int64_t)(L.prefix - L.state), b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        delete b;
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
    int32_t k = -1;
    for (int32_t i = 0; i < b->max_shots; ++i)
        if (!b->used[(size_t)i]) { k = i; break; }
    if (k < 0) return LB_E_RANGE;

    char *ws = (char *)d_ws;
    const int64_t n = (int64_t)s->nx * s->ny;
    if ((rc = lbw::upload_c2(b->stream, b->scheme.precision, b->q, b->scheme.d2q9_ratio, ws + L.c2, c2, t, on_device,
                             n, b->d_scratch))) {
        if (rc == LB_E_HIP) b->sticky = LB_E_HIP;
        return rc;
    }
    BT_TRY(b, lbw::launch_fill_zero(ws + L.pop0, (int64_t)(L.c2 - L.pop0), b->stream));
    const int64_t nw = std::min<int64_t>(nt, s->nsteps + 1);
    if (nw > 0)
        BT_TRY(b, hipMemcpyAsync(ws + L.wavelet, wavelet, (size_t)nw * 8, hipMemcpyHostToDevice, b->stream));

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
        BT_TRY(b, hipMemcpyAsync(ws + L.rrow, row.data(), row.size() * 4, hipMemcpyHostToDevice, b->stream));
        BT_TRY(b, hipMemcpyAsync(ws + L.rxs, xs.data(), xs.size() * 4, hipMemcpyHostToDevice, b->stream));
        BT_TRY(b, hipMemcpyAsync(ws + L.rslot, sl.data(), sl.size() * 4, hipMemcpyHostToDevice, b->stream));
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
    BT_TRY(b, lbw::launch_step(b->storage, p, false, b->stream));

    ShotState st;
    st.t = 0;
    st.t_end = s->nsteps;
    st.cur = 1;
    st.active = 1;
    BT_TRY(b, hipMemcpyAsync(b->d_table + k, &e, sizeof(e), hipMemcpyHostToDevice, b->stream));
    BT_TRY(b, hipMemcpyAsync(b->d_state + k, &st, sizeof(st), hipMemcpyHostToDevice, b->stream));
    BT_TRY(b, hipStreamSynchronize(b->stream));
    b->table[(size_t)k] = e;
    b->used[(size_t)k] = 1;
    if ((rc = rebuild(b))) return rc;
    *slot = k;
    return LB_OK;
}

int lb_batch_remove_shot(lb_batch *b, int32_t slot) {
    if (!b) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    if (slot < 0 || slot >= b->max_shots || !b->used[(size_t)slot]) return LB_E_RANGE;
    const int32_t zero = 0;
    BT_TRY(b, hipMemcpyAsync(&b->d_state[slot].active, &zero, 4, hipMemcpyHostToDevice, b->stream));
    BT_TRY(b, hipStreamSynchronize(b->stream));
    b->used[(size_t)slot] = 0;
    b->table[(size_t)slot] = ShotEntry();
    return rebuild(b);
}

int lb_batch_tick(lb_batch *b, int64_t k) {
    if (!b) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    if (k < 0) return LB_E_RANGE;
    if (k == 0 || b->order.empty()) return LB_OK;
    if (!b->use_graph) return enqueue_steps(b, k);
    // a graph of kGraphSteps steps, captured once per set of active shots
    // (cheap to re-capture when shots come and go) and replayed; the
    // remainder of k runs as direct launches
    if (b->dirty || !b->exec) {
        int rc = capture(b, kGraphSteps);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < k / kGraphSteps; ++i) BT_TRY(b, hipGraphLaunch(b->exec, b->stream));
    return enqueue_steps(b, k % kGraphSteps);
}

int lb_batch_times(lb_batch *b, int64_t *t_out) {
    if (!b || !t_out) return LB_E_INVALID;
    if (b->sticky) return b->sticky;
    std::vector<ShotState> st((size_t)b->max_shots);
    BT_TRY(b, hipMemcpyAsync(st.data(), b->d_state, st.size() * sizeof(ShotState), hipMemcpyDeviceToHost, b->stream));
    BT_TRY(b, hipStreamSynchronize(b->stream));
    for (int32_t k = 0; k < b->max_shots; ++k) t_out[k] = b->used[(size_t)k] ? st[(size_t)k].t : -1;
    return LB_OK;
}

int lb_batch_sync(lb_batch *b) {
    if (!b) return LB_E_INVALID;
    if (hipStreamSynchronize(b->stream) != hipSuccess) b->sticky = LB_E_HIP;
    return b->sticky;
}

int lb_batch_destroy(lb_batch *b) {
    if (!b) return LB_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    drop_graph(b);
    int rc = b->sticky ? b->sticky : (e == hipSuccess ? LB_OK : LB_E_HIP);
    delete b;
    return rc;
}

}  // extern "C"
