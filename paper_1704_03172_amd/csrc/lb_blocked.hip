// lb_blocked.hip -- dispatch of the temporally blocked step kernel
// (lb_blocked.h; instantiated per storage format and lattice in
// lb_blocked_*.hip): step counts, wave counts, argument checks, and the
// batched executor's per-shot advance after a blocked launch.
#include "lb_blocked.h"

#include <algorithm>

namespace lbw {
namespace {

constexpr int kAdvBlock = 256;

// After a blocked batch launch of up to `run` steps: each active shot
// advanced by min(run, steps left) in one buffer swap.
__global__ __launch_bounds__(kAdvBlock) void k_batch_advance_n(ShotState *state, const int32_t *order, int nact,
                                                               int run) {
    int a = blockIdx.x * kAdvBlock + threadIdx.x;
    if (a >= nact) return;
    ShotState &ss = state[order[a]];
    if (ss.active && ss.t < ss.t_end) {
        ss.t += min<int64_t>(run, ss.t_end - ss.t);
        ss.cur ^= 1;
    }
}

// Params images of a marching round (see launch_batch_march_prep).
__global__ __launch_bounds__(kAdvBlock) void k_batch_march_prep(BatchParams bp, int q, int ns) {
    const int a = blockIdx.x * kAdvBlock + threadIdx.x;
    if (a >= bp.nact) return;
    const int slot = bp.order[a];
    const ShotState ss = bp.state[slot];
    const ShotEntry &e = bp.table[slot];
    StepParams p;
    p.src = ss.cur ? e.pop1 : e.pop0;
    p.dst = ss.cur ? e.pop0 : e.pop1;
    p.c2 = e.c2;
    p.nx = e.nx;
    p.ny = e.ny;
    p.pstride = e.pstride;
    p.q = q;
    p.coll = bp.coll;
    p.sponge_width = e.sponge_width;
    p.sponge_smax = e.sponge_smax;
    p.src_x = e.src_x;
    p.src_y = e.src_y;
    const int64_t tn = ss.t + 1;
    auto wv = [&](int64_t n) { return n < e.wavelet_len ? e.wavelet[n] : 0.0; };
    p.s_n = wv(tn);
    p.s_n2 = wv(tn + 1);
    p.s_n3 = wv(tn + 2);
    p.s_n4 = wv(tn + 3);
    for (int k = 0; k < 4; ++k) p.s_more[k] = wv(tn + 4 + k);
    p.rec = e.rec;
    p.rec.col = tn;
    p.nrun = e.march && ss.active && ss.t_end - ss.t >= ns ? ns : 0;
    bp.img[slot] = p;
}

// State after the launches of a marching round (see launch_batch_advance_sel).
__global__ __launch_bounds__(kAdvBlock) void k_batch_advance_sel(ShotState *state, const int32_t *order, int nact,
                                                                 const StepParams *img, int sel, int run) {
    const int a = blockIdx.x * kAdvBlock + threadIdx.x;
    if (a >= nact) return;
    const int slot = order[a];
    ShotState &ss = state[slot];
    const int nr = img[slot].nrun;
    if (sel == 1) {
        if (nr > 0) {
            ss.t += nr;
            ss.cur ^= 1;
        }
    } else if (nr == 0 && ss.active && ss.t < ss.t_end) {
        ss.t += min<int64_t>(run, ss.t_end - ss.t);
        ss.cur ^= 1;
    }
}

// f(S(), integral_constant<int, Q>()) for the storage format and lattice.
template <typename F>
static auto by_config(int storage, int q, F &&f) {
    using Q5 = std::integral_constant<int, 5>;
    using Q9 = std::integral_constant<int, 9>;
    if (storage == ST_F64) return q == 5 ? f(double(), Q5()) : f(double(), Q9());
    if (storage == ST_F16) return q == 5 ? f(_Float16(), Q5()) : f(_Float16(), Q9());
    return q == 5 ? f(float(), Q5()) : f(float(), Q9());
}

}  // namespace

int stepn_max(int storage, int q, int kind) {
    return by_config(storage, q, [&](auto sv, auto qc) {
        using S = decltype(sv);
        constexpr int Q = decltype(qc)::value;
        return kind == 1 ? tn_max<S, Q, 1>() : tn_max<S, Q, 0>();
    });
}

int stepn_graph_steps(int storage, int q, int kind, int32_t nx) {
    return by_config(storage, q, [&](auto sv, auto qc) {
        using S = decltype(sv);
        constexpr int Q = decltype(qc)::value;
        const int m = kind == 1 ? tn_max<S, Q, 1>() : tn_max<S, Q, 0>();
        return m >= 2 && nx % Tb<S>::V == 0 ? m : 1;
    });
}

int stepn_march(int storage, int q, int kind, int32_t nx, int32_t ny, bool pref) {
    if (nx < 1 || ny < 1) return 0;
    if (storage == ST_F32)
        return q == 5 ? march_steps_f32_q5(kind, nx, ny, pref) : march_steps_f32_q9(kind, nx, ny, pref);
    if (storage == ST_F64)
        return q == 5 ? march_steps_f64_q5(kind, nx, ny, pref) : march_steps_f64_q9(kind, nx, ny, pref);
    if (storage == ST_F16 && q == 5) return march_steps_f16_q5(kind, nx, ny, pref);
    return 0;
}

int64_t stepn_march_min_waves(int storage, int q, int kind) {
    if (storage == ST_F32) return q == 5 ? march_min_waves_f32_q5(kind) : march_min_waves_f32_q9(kind);
    if (storage == ST_F64) return q == 5 ? march_min_waves_f64_q5(kind) : march_min_waves_f64_q9(kind);
    if (storage == ST_F16 && q == 5) return march_min_waves_f16_q5(kind);
    return 0;
}

int stepn_max_grid(int storage, int q, int kind, int32_t nx, int32_t ny, bool pref) {
    return std::max(stepn_max(storage, q, kind == 1 ? 1 : 0), stepn_march(storage, q, kind, nx, ny, pref));
}

int stepn_round(int storage, int q, int kind, int32_t nx, int32_t ny, int ns) {
    const int mn = stepn_march(storage, q, kind, nx, ny);
    if (mn > 0 && ns >= mn) return mn;
    return std::max(1, std::min(ns, stepn_max(storage, q, kind == 1 ? 1 : 0)));
}

int64_t stepn_waves(int storage, int q, int kind, int ns, int32_t nx, int32_t ny) {
    return by_config(storage, q, [&](auto sv, auto qc) {
        return waves_of<decltype(sv), decltype(qc)::value>(kind, ns, nx, ny);
    });
}

hipError_t launch_stepn(int storage, const StepParams &p, int ns, hipStream_t s) {
    if (p.nx < 1 || p.ny < 1 || (p.q != 5 && p.q != 9) || ns < 2 || p.nrun != ns) return hipErrorInvalidValue;
    const int kind = step_kind(p.coll);
    const bool march = ns == stepn_march(storage, p.q, kind, p.nx, p.ny);
    if (!march && ns > stepn_max(storage, p.q, p.coll.kind)) return hipErrorInvalidValue;
    if (storage == ST_F32) return p.q == 5 ? launch_stepn_f32_q5(p, ns, s) : launch_stepn_f32_q9(p, ns, s);
    if (storage == ST_F64) return p.q == 5 ? launch_stepn_f64_q5(p, ns, s) : launch_stepn_f64_q9(p, ns, s);
    if (storage == ST_F16 && p.q == 5) return launch_stepn_f16_q5(p, ns, s);
    return hipErrorInvalidValue;
}

hipError_t launch_stepn_batch(int storage, int q, int ns, const BatchParams &bp, int64_t nwaves, hipStream_t s) {
    if (nwaves <= 0 || bp.nact <= 0) return hipSuccess;
    if ((q != 5 && q != 9) || ns < 2 || ns > stepn_max(storage, q, bp.coll.kind) || bp.max_run < 1 ||
        bp.max_run > ns)
        return hipErrorInvalidValue;
    if (storage == ST_F32) return q == 5 ? launch_stepn_batch_f32_q5(bp, ns, nwaves, s)
                                         : launch_stepn_batch_f32_q9(bp, ns, nwaves, s);
    if (storage == ST_F64) return q == 5 ? launch_stepn_batch_f64_q5(bp, ns, nwaves, s)
                                         : launch_stepn_batch_f64_q9(bp, ns, nwaves, s);
    if (storage == ST_F16 && q == 5) return launch_stepn_batch_f16_q5(bp, ns, nwaves, s);
    return hipErrorInvalidValue;
}

int64_t stepn_march_waves(int storage, int q, int kind, int32_t nx, int32_t ny) {
    if (nx < 1 || ny < 1) return 0;
    if (storage == ST_F32) return q == 5 ? march_waves_f32_q5(kind, nx, ny) : march_waves_f32_q9(kind, nx, ny);
    if (storage == ST_F64) return q == 5 ? march_waves_f64_q5(kind, nx, ny) : march_waves_f64_q9(kind, nx, ny);
    if (storage == ST_F16 && q == 5) return march_waves_f16_q5(kind, nx, ny);
    return 0;
}

hipError_t launch_batch_march_prep(int q, const BatchParams &bp, int ns, hipStream_t s) {
    if (bp.nact <= 0) return hipSuccess;
    if (bp.img == nullptr || ns < 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_march_prep, dim3((unsigned)((bp.nact + kAdvBlock - 1) / kAdvBlock)), dim3(kAdvBlock),
                       0, s, bp, q, ns);
    return hipGetLastError();
}

hipError_t launch_stepn_march_batch(int storage, int q, const BatchParams &bp, int64_t nwaves, hipStream_t s) {
    if (nwaves <= 0 || bp.nact <= 0) return hipSuccess;
    if (bp.img == nullptr || bp.mprefix == nullptr || (q != 5 && q != 9)) return hipErrorInvalidValue;
    if (storage == ST_F32) return q == 5 ? launch_stepn_march_batch_f32_q5(bp, nwaves, s)
                                         : launch_stepn_march_batch_f32_q9(bp, nwaves, s);
    if (storage == ST_F64) return q == 5 ? launch_stepn_march_batch_f64_q5(bp, nwaves, s)
                                         : launch_stepn_march_batch_f64_q9(bp, nwaves, s);
    if (storage == ST_F16 && q == 5) return launch_stepn_march_batch_f16_q5(bp, nwaves, s);
    return hipErrorInvalidValue;
}

hipError_t launch_batch_advance_sel(ShotState *state, const int32_t *order, int nact, const StepParams *img, int sel,
                                    int run, hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    if (img == nullptr || (sel != 1 && sel != 2)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_advance_sel, dim3((unsigned)((nact + kAdvBlock - 1) / kAdvBlock)), dim3(kAdvBlock), 0,
                       s, state, order, nact, img, sel, run);
    return hipGetLastError();
}

hipError_t launch_batch_advance_n(ShotState *state, const int32_t *order, int nact, int run, hipStream_t s) {
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_advance_n, dim3((unsigned)((nact + kAdvBlock - 1) / kAdvBlock)), dim3(kAdvBlock), 0,
                       s, state, order, nact, run);
    return hipGetLastError();
}

}  // namespace lbw
