// fem_internal.h -- host-side helpers shared by the library's translation
// units: error reporting, launch configuration, device properties,
// workspace carving and the small utility kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

#include "../../include/fem.h"

namespace fem {

// Thread-local last-error message; returns `code` for convenience.
int set_error(int code, const char* fmt, ...);
void clear_error();

#define FEM_HIP_CHECK(expr)                                                                        \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::fem::set_error(FEM_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                    __FILE__, __LINE__);                                           \
    } while (0)

// Compute units of the current device (cached per device id).
int device_cu_count();

// Launch configuration in effect for a kernel / precision.
fem_launch launch_config(int kernel, int prec);

// Number of workgroups of a persistent launch over n_tiles tiles.
int persistent_grid(const fem_launch& cfg, int64_t n_tiles);

// Bump allocator over a caller-provided workspace (256-byte aligned pieces).
struct WsCarver {
    char* base;
    size_t cap, used;
    explicit WsCarver(void* p, size_t c) : base(static_cast<char*>(p)), cap(c), used(0) {}
    template <typename T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return (used <= cap && base) ? reinterpret_cast<T*>(base + off) : nullptr;
    }
    bool ok() const { return used <= cap; }
};

// Size a carver would need for the same sequence of takes (base == nullptr).
struct WsCounter {
    size_t used = 0;
    template <typename T>
    void take(size_t count) {
        used = ((used + 255) & ~size_t(255)) + count * sizeof(T);
    }
};

// Zero `bytes` bytes at p on stream s with a kernel (no memset node, so a
// captured graph may replay it).
hipError_t zero_bytes(void* p, size_t bytes, hipStream_t s);

// Zero two small int32 arrays (up to 64 entries each; either may be null) in
// one launch.
hipError_t zero_counters(int32_t* a, int na, int32_t* b, int nb, hipStream_t s);

// Kernel timing (fem_timing_enable): returns true if enabled; then
// timing_begin / timing_end bracket one launch on stream s.
bool timing_on();
void* timing_begin(hipStream_t s);
void timing_end(void* token, int kernel, hipStream_t s);

// out[3I + c] = sum of the element vectors Re[e][3i + c] over the incident
// entries 8e + i of node I (the residual assembly without constraints or norm)
hipError_t gather_node_vectors(int32_t n_nodes, const int32_t* ne_ptr, const int32_t* ne_list, const double* Re,
                               double* out, hipStream_t s);

// g_uniform[s][k] = sum over the elements of specimen s of g_elem[k][e]
// (fixed order; off = NULL for one specimen)
hipError_t reduce_g_uniform(const double* g_elem, int64_t n_elems, const int64_t* off, int n_spec,
                            double* g_uniform, hipStream_t s);

// Aggregation multigrid (amg.hip) as fem_solve_amg drives it: numeric
// set-up for K, then one cycle z = M b per call on stream s (a V-cycle, or
// a K-cycle, which varies between calls: amg_cycle_type).  With
// presmoothed, amg_level0_x already holds M_0 b (M_0 = amg_smoother0, the
// finest level's 3x3 smoother blocks), as the solver's fused update kernels
// write it.  Every cycle kernel returns at once when *stop is nonzero (stop
// may be NULL).
int amg_update(fem_amg* h, const void* K, fem_precision prec, hipStream_t s);
hipError_t amg_apply_cycle(fem_amg* h, const double* b, double* z, bool presmoothed, const int32_t* stop, hipStream_t s);
const double* amg_smoother0(const fem_amg* h);
double* amg_level0_x(fem_amg* h);
bool amg_matches(const fem_amg* h, const fem_csr* csr);
fem_amg_cycle amg_cycle_type(const fem_amg* h);

}  // namespace fem
