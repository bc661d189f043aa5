// lb_host.h -- small host-side helpers shared by the runtime files.
#pragma once

#include "lbwave.h"
#include "lb_internal.h"

#include <cstddef>
#include <cstdint>

namespace lbw {

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }
inline size_t storage_bytes(int p) { return p == LB_F64 ? 8 : (p == LB_F16S ? 2 : 4); }
inline size_t compute_bytes(int p) { return p == LB_F64 ? 8 : 4; }
inline int storage_kind(int p) { return p == LB_F64 ? ST_F64 : (p == LB_F16S ? ST_F16 : ST_F32); }

// Population stride: 256-element aligned, skewed by 1024 elements so that the
// population arrays of power-of-two grids do not alias in the low address bits.
inline int64_t population_stride(int64_t n) { return (int64_t)align_up((size_t)n + 1024, 256); }

// Largest squared sound speed with non-negative weights: 1/2 for D2Q5
// (w0 = 1 - 2 c^2), (1 + 2r)/(2 + 2r) for the D2Q9 family w5 = r w1.
inline double c2_max(int lattice, double ratio) {
    if (lattice == LB_D2Q5) return 0.5;
    return (1.0 + 2.0 * ratio) / (2.0 + 2.0 * ratio);
}

// Collision constants of a scheme descriptor (MRT rates divided by the row
// norms |M_k|^2 of the moment matrices of Appendix A).
Collision make_collision(const lb_grid_desc *d);

// Argument checks shared by the trace-misfit entry points (lb_trace_misfit
// and its variant without workspace): LB_OK, LB_E_INVALID or LB_E_RANGE.
int check_trace_misfit(const void *traces, const void *obs, const void *res, int32_t nrec, int64_t cap,
                       int64_t ncols, lb_dtype t, const double *phi);

// Validate the scheme part of a descriptor (lattice, collision, precision,
// rates, D2Q9 ratio).
int validate_scheme(const lb_grid_desc *d);

// Convert/validate a c^2 field into the compute type at dst (n values):
// host arrays are checked and converted on the host, device arrays by a
// kernel whose failure count lands in `scratch`.  Synchronises the stream.
int upload_c2(hipStream_t s, int precision, int lattice, double ratio, void *dst, const void *c2,
              lb_dtype t, int on_device, int64_t n, int32_t *scratch);

}  // namespace lbw
