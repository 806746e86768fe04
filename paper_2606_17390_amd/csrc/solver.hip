// solver.hip -- the linear solve of the global Newton iteration (Sec. 2.2.4:
// K du = -R with the Dirichlet rows of App. E replaced by identity rows, so
// K is not symmetric): CSR matrix-vector product and BiCGSTAB with a Jacobi
// preconditioner (the inverse of the diagonal of K).
//
// The matrix is the CSR pattern of fem_csr_pattern (rows 3I+a; the three
// rows of a node are consecutive and share their sorted column list).
// Vectors are FP64; the matrix values are FP64 or FP32 (the mixed form keeps
// K in FP32 and solves in FP64).  Every reduction is a fixed two-stage tree,
// so a solve is bitwise reproducible.  The iteration runs on the host: the
// scalars stay in device memory and the residual norm is read back once per
// iteration for the convergence test.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fem_internal.h"

namespace fem {
namespace {

constexpr int kSpmvLanes = 32;    // lanes per node (3 rows) of the matrix-vector product
constexpr int kVecThreads = 256;  // vector kernels
constexpr int kDotBlocks = 256;   // fixed grid of the first reduction stage

// y = K x over the pattern of fem_csr_pattern, where the three rows of a node
// are consecutive, equally long and share their column list: 32 lanes per
// node, lane l takes columns l, l + 32, ... of the node's rows, reading each
// column index and x value once for the three rows, then a butterfly over
// the 32 lanes (fixed order).
template <typename RV>
__global__ __launch_bounds__(256) void spmv_kernel(int32_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, const RV* __restrict__ val,
                                                   const double* __restrict__ x, double* __restrict__ y) {
    const int64_t node = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSpmvLanes;
    const int l = (int)(threadIdx.x & (kSpmvLanes - 1));
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (node < n_nodes) {
        const int32_t b = row_ptr[3 * node], len = row_ptr[3 * node + 1] - b;
        const int32_t* __restrict__ ci = col_idx + b;
        const RV* __restrict__ v = val + b;
        for (int32_t k = l; k < len; k += kSpmvLanes) {
            const double xv = x[ci[k]];
            s0 += (double)v[k] * xv;
            s1 += (double)v[len + k] * xv;
            s2 += (double)v[2 * len + k] * xv;
        }
    }
#pragma unroll
    for (int m = 1; m < kSpmvLanes; m <<= 1) {
        s0 += __shfl_xor(s0, m, kSpmvLanes);
        s1 += __shfl_xor(s1, m, kSpmvLanes);
        s2 += __shfl_xor(s2, m, kSpmvLanes);
    }
    if (node < n_nodes && l < 3) y[3 * node + l] = (l == 0 ? s0 : (l == 1 ? s1 : s2));
}

// KT = K^T on the same (structurally symmetric) pattern: one wave per node I,
// lane r < deg(I) copies the 3x3 block (J, I)^T of the r-th neighbour J, whose
// slot in J's sorted column list comes from a binary search; rows of
// constrained dofs become identity rows.
template <typename RV>
__global__ __launch_bounds__(256) void transpose_kernel(int32_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        const RV* __restrict__ K, const uint8_t* __restrict__ bc,
                                                        RV* __restrict__ KT) {
    const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t r = (int32_t)(threadIdx.x & 63);
    if (I >= n_nodes) return;
    const int32_t bI = row_ptr[3 * I], degI = (row_ptr[3 * I + 1] - bI) / 3;
    if (r >= degI) return;
    const int32_t J = col_idx[bI + 3 * r] / 3;
    const int32_t bJ = row_ptr[3 * J], degJ = (row_ptr[3 * J + 1] - bJ) / 3;
    int32_t a0 = 0, a1 = degJ - 1;
    while (a0 < a1) {
        const int32_t mid = (a0 + a1) >> 1;
        if (col_idx[bJ + 3 * mid] < 3 * I) a0 = mid + 1;
        else a1 = mid;
    }
    // a0 = slot of I in J's list (present: the pattern is symmetric)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            RV v = K[(int64_t)bJ + (int64_t)b * 3 * degJ + 3 * a0 + a];
            if (bc && bc[3 * I + a]) v = (J == I && a == b) ? RV(1) : RV(0);
            KT[(int64_t)bI + (int64_t)a * 3 * degI + 3 * r + b] = v;
        }
}

// dinv[i] = 1 / K_ii (1 where the diagonal entry is absent or zero)
template <typename RV>
__global__ void diag_inv_kernel(int32_t n_rows, const int32_t* __restrict__ row_ptr,
                                const int32_t* __restrict__ col_idx, const RV* __restrict__ val,
                                double* __restrict__ dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rows) return;
    int32_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col_idx[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    const double dii = (lo <= hi && col_idx[lo] == i) ? (double)val[lo] : 0.0;
    dinv[i] = (dii != 0.0) ? 1.0 / dii : 1.0;
}

// ---- fixed-order reductions: kDotBlocks partials (grid-stride over the
// vector), then one workgroup adds them in a fixed tree.

__device__ inline void block_sum_to(double v, double* __restrict__ out) {
    __shared__ double sh[kVecThreads];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kVecThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ __launch_bounds__(kVecThreads) void dot_partial(int64_t n, const double* __restrict__ a,
                                                           const double* __restrict__ b, double* __restrict__ part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kVecThreads)
        s += a[i] * b[i];
    block_sum_to(s, part + blockIdx.x);
}

__global__ __launch_bounds__(kVecThreads) void dot_final(const double* __restrict__ part, double* __restrict__ out) {
    block_sum_to(part[threadIdx.x], out);  // kDotBlocks == kVecThreads
}

// Scalars of the iteration, in device memory.
enum { S_RHO, S_RHO_NEW, S_ALPHA, S_OMEGA, S_RV, S_TS, S_TT, S_RR, S_BB, S_COUNT };

// r = b - y, rh = r, p = v = 0; rho = alpha = omega = 1
__global__ void init_kernel(int64_t n, const double* __restrict__ b, const double* __restrict__ y,
                            double* __restrict__ r, double* __restrict__ rh, double* __restrict__ p,
                            double* __restrict__ v, double* __restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        sc[S_RHO] = 1.0;
        sc[S_ALPHA] = 1.0;
        sc[S_OMEGA] = 1.0;
    }
    if (i >= n) return;
    const double ri = b[i] - y[i];
    r[i] = ri;
    rh[i] = ri;
    p[i] = 0.0;
    v[i] = 0.0;
}

// p = r + beta (p - omega v), beta = (rho_new / rho)(alpha / omega); ph = dinv p
__global__ void update_p(int64_t n, const double* __restrict__ r, const double* __restrict__ v,
                         const double* __restrict__ dinv, double* __restrict__ p, double* __restrict__ ph,
                         const double* __restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double beta = (sc[S_RHO_NEW] / sc[S_RHO]) * (sc[S_ALPHA] / sc[S_OMEGA]);
    const double pi = r[i] + beta * (p[i] - sc[S_OMEGA] * v[i]);
    p[i] = pi;
    ph[i] = dinv[i] * pi;
}

// alpha = rho_new / (rh, v); s = r - alpha v; sh = dinv s
__global__ void update_s(int64_t n, const double* __restrict__ r, const double* __restrict__ v,
                         const double* __restrict__ dinv, double* __restrict__ s, double* __restrict__ sh,
                         double* __restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double alpha = sc[S_RHO_NEW] / sc[S_RV];
    if (i == 0) sc[S_ALPHA] = alpha;  // read by later kernels only
    if (i >= n) return;
    const double si = r[i] - alpha * v[i];
    s[i] = si;
    sh[i] = dinv[i] * si;
}

// omega = (t, s) / (t, t); x += alpha ph + omega sh; r = s - omega t
__global__ void update_x(int64_t n, const double* __restrict__ ph, const double* __restrict__ sh,
                         const double* __restrict__ s, const double* __restrict__ t, double* __restrict__ x,
                         double* __restrict__ r, const double* __restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double omega = sc[S_TT] > 0.0 ? sc[S_TS] / sc[S_TT] : 0.0;
    x[i] += sc[S_ALPHA] * ph[i] + omega * sh[i];
    r[i] = s[i] - omega * t[i];
}

// the scalars that carry over to the next iteration
__global__ void roll_scalars(double* __restrict__ sc) {
    sc[S_OMEGA] = sc[S_TT] > 0.0 ? sc[S_TS] / sc[S_TT] : 0.0;
    sc[S_RHO] = sc[S_RHO_NEW];
}

struct SolverWs {
    double *r, *rh, *p, *ph, *v, *s, *sh, *t, *y, *dinv, *part, *sc;
};

template <typename C>
void carve_solver(C& c, int32_t n, SolverWs* w) {
    SolverWs o;
    o.r = c.template take<double>((size_t)n + 1);
    o.rh = c.template take<double>((size_t)n + 1);
    o.p = c.template take<double>((size_t)n + 1);
    o.ph = c.template take<double>((size_t)n + 1);
    o.v = c.template take<double>((size_t)n + 1);
    o.s = c.template take<double>((size_t)n + 1);
    o.sh = c.template take<double>((size_t)n + 1);
    o.t = c.template take<double>((size_t)n + 1);
    o.y = c.template take<double>((size_t)n + 1);
    o.dinv = c.template take<double>((size_t)n + 1);
    o.part = c.template take<double>(kDotBlocks);
    o.sc = c.template take<double>(S_COUNT);
    if (w) *w = o;
}

struct CountAdapterS {
    WsCounter cnt;
    template <typename T>
    T* take(size_t n) {
        cnt.take<T>(n);
        return nullptr;
    }
};

hipError_t spmv(const fem_csr* csr, const void* vals, fem_precision prec, const double* x, double* y,
                hipStream_t s) {
    const int32_t nn = csr->n_rows / 3;
    if (nn <= 0) return hipSuccess;
    const unsigned nb = (unsigned)(((int64_t)nn * kSpmvLanes + 255) / 256);
    if (prec == FEM_FP64)
        hipLaunchKernelGGL(spmv_kernel<double>, dim3(nb), dim3(256), 0, s, nn, csr->row_ptr, csr->col_idx,
                           static_cast<const double*>(vals), x, y);
    else
        hipLaunchKernelGGL(spmv_kernel<float>, dim3(nb), dim3(256), 0, s, nn, csr->row_ptr, csr->col_idx,
                           static_cast<const float*>(vals), x, y);
    return hipGetLastError();
}

hipError_t dot(int64_t n, const double* a, const double* b, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(dot_partial, dim3(kDotBlocks), dim3(kVecThreads), 0, s, n, a, b, part);
    hipLaunchKernelGGL(dot_final, dim3(1), dim3(kVecThreads), 0, s, part, out);
    return hipGetLastError();
}

int check_csr(const fem_csr* csr, const void* vals, const char* who) {
    if (!csr || !vals) return set_error(FEM_EINVAL, "%s: csr and K values must not be NULL", who);
    if (csr->n_rows < 0 || csr->n_rows % 3) return set_error(FEM_EINVAL, "%s: n_rows must be 3 n_nodes", who);
    if (csr->n_rows > 0 && (!csr->row_ptr || !csr->col_idx))
        return set_error(FEM_EINVAL, "%s: row_ptr and col_idx must not be NULL", who);
    return FEM_OK;
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" size_t fem_solver_workspace_bytes(int32_t n_rows) {
    if (n_rows < 0) return 0;
    CountAdapterS c;
    carve_solver(c, n_rows, (SolverWs*)nullptr);
    return c.cnt.used + 256;
}

extern "C" int fem_csr_spmv(const fem_csr* csr, const void* K_vals, fem_precision prec, const double* x, double* y,
                            void* stream) {
    clear_error();
    if (int rc = check_csr(csr, K_vals, "fem_csr_spmv")) return rc;
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED) return set_error(FEM_EINVAL, "fem_csr_spmv: bad precision");
    if (csr->n_rows > 0 && (!x || !y)) return set_error(FEM_EINVAL, "fem_csr_spmv: x and y must not be NULL");
    FEM_HIP_CHECK(spmv(csr, K_vals, prec, x, y, (hipStream_t)stream));
    return FEM_OK;
}

extern "C" int fem_csr_transpose(const fem_csr* csr, const void* K_vals, fem_precision prec, const uint8_t* bc_mask,
                                 void* KT_vals, void* stream) {
    clear_error();
    if (int rc = check_csr(csr, K_vals, "fem_csr_transpose")) return rc;
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED) return set_error(FEM_EINVAL, "fem_csr_transpose: bad precision");
    if (csr->n_rows > 0 && !KT_vals) return set_error(FEM_EINVAL, "fem_csr_transpose: KT_vals must not be NULL");
    if (KT_vals == K_vals && csr->n_rows > 0)
        return set_error(FEM_EINVAL, "fem_csr_transpose: KT_vals must not alias K_vals");
    const int32_t nn = csr->n_rows / 3;
    if (nn == 0) return FEM_OK;
    const unsigned nb = (unsigned)(((int64_t)nn * 64 + 255) / 256);
    hipStream_t s = (hipStream_t)stream;
    if (prec == FEM_FP64)
        hipLaunchKernelGGL(transpose_kernel<double>, dim3(nb), dim3(256), 0, s, nn, csr->row_ptr, csr->col_idx,
                           static_cast<const double*>(K_vals), bc_mask, static_cast<double*>(KT_vals));
    else
        hipLaunchKernelGGL(transpose_kernel<float>, dim3(nb), dim3(256), 0, s, nn, csr->row_ptr, csr->col_idx,
                           static_cast<const float*>(K_vals), bc_mask, static_cast<float*>(KT_vals));
    FEM_HIP_CHECK(hipGetLastError());
    return FEM_OK;
}

extern "C" int fem_solve(const fem_csr* csr, const void* K_vals, fem_precision prec, const double* b, double* x,
                         int32_t max_iter, double rtol, int32_t* iters, double* rel_res, void* ws, size_t ws_bytes,
                         void* stream) {
    clear_error();
    if (int rc = check_csr(csr, K_vals, "fem_solve")) return rc;
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED) return set_error(FEM_EINVAL, "fem_solve: bad precision");
    if (max_iter < 0 || !(rtol >= 0.0)) return set_error(FEM_EINVAL, "fem_solve: max_iter >= 0 and rtol >= 0");
    const int32_t n = csr->n_rows;
    if (iters) *iters = 0;
    if (rel_res) *rel_res = 0.0;
    if (n == 0) return FEM_OK;
    if (!b || !x) return set_error(FEM_EINVAL, "fem_solve: b and x must not be NULL");
    const size_t need = fem_solver_workspace_bytes(n);
    if (!ws || ws_bytes < need)
        return set_error(FEM_ENOMEM, "fem_solve: workspace of %zu bytes required, %zu given", need, ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    WsCarver c(ws, ws_bytes);
    SolverWs w;
    carve_solver(c, n, &w);
    const unsigned nb = (unsigned)(((int64_t)n + kVecThreads - 1) / kVecThreads);
    if (prec == FEM_FP64)
        hipLaunchKernelGGL(diag_inv_kernel<double>, dim3(nb), dim3(kVecThreads), 0, s, n, csr->row_ptr,
                           csr->col_idx, static_cast<const double*>(K_vals), w.dinv);
    else
        hipLaunchKernelGGL(diag_inv_kernel<float>, dim3(nb), dim3(kVecThreads), 0, s, n, csr->row_ptr,
                           csr->col_idx, static_cast<const float*>(K_vals), w.dinv);
    FEM_HIP_CHECK(dot(n, b, b, w.part, w.sc + S_BB, s));
    FEM_HIP_CHECK(spmv(csr, K_vals, prec, x, w.y, s));
    hipLaunchKernelGGL(init_kernel, dim3(nb), dim3(kVecThreads), 0, s, (int64_t)n, b, w.y, w.r, w.rh, w.p, w.v,
                       w.sc);
    FEM_HIP_CHECK(dot(n, w.r, w.r, w.part, w.sc + S_RR, s));
    double hs[2];
    FEM_HIP_CHECK(hipMemcpyAsync(hs, w.sc + S_RR, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    FEM_HIP_CHECK(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(hs[1]);
    double res = (bnorm > 0.0) ? std::sqrt(hs[0]) / bnorm : std::sqrt(hs[0]);
    if (rel_res) *rel_res = res;
    if (bnorm == 0.0 && hs[0] == 0.0) return FEM_OK;  // x already solves K x = 0
    int32_t it = 0;
    while (res > rtol && it < max_iter) {
        FEM_HIP_CHECK(dot(n, w.rh, w.r, w.part, w.sc + S_RHO_NEW, s));
        hipLaunchKernelGGL(update_p, dim3(nb), dim3(kVecThreads), 0, s, (int64_t)n, w.r, w.v, w.dinv, w.p, w.ph,
                           w.sc);
        FEM_HIP_CHECK(spmv(csr, K_vals, prec, w.ph, w.v, s));
        FEM_HIP_CHECK(dot(n, w.rh, w.v, w.part, w.sc + S_RV, s));
        hipLaunchKernelGGL(update_s, dim3(nb), dim3(kVecThreads), 0, s, (int64_t)n, w.r, w.v, w.dinv, w.s, w.sh,
                           w.sc);
        FEM_HIP_CHECK(spmv(csr, K_vals, prec, w.sh, w.t, s));
        FEM_HIP_CHECK(dot(n, w.t, w.s, w.part, w.sc + S_TS, s));
        FEM_HIP_CHECK(dot(n, w.t, w.t, w.part, w.sc + S_TT, s));
        hipLaunchKernelGGL(update_x, dim3(nb), dim3(kVecThreads), 0, s, (int64_t)n, w.ph, w.sh, w.s, w.t, x, w.r,
                           w.sc);
        hipLaunchKernelGGL(roll_scalars, dim3(1), dim3(1), 0, s, w.sc);
        FEM_HIP_CHECK(dot(n, w.r, w.r, w.part, w.sc + S_RR, s));
        double rr = 0.0, chk[2];
        FEM_HIP_CHECK(hipMemcpyAsync(&rr, w.sc + S_RR, sizeof(double), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipMemcpyAsync(chk, w.sc + S_RHO, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        FEM_HIP_CHECK(hipStreamSynchronize(s));
        ++it;
        res = (bnorm > 0.0) ? std::sqrt(rr) / bnorm : std::sqrt(rr);
        if (!std::isfinite(res) || chk[0] == 0.0) break;  // breakdown (rho = 0) or non-finite values
    }
    if (iters) *iters = it;
    if (rel_res) *rel_res = res;
    if (!(res <= rtol))
        return set_error(FEM_ENOCONV, "fem_solve: relative residual %.3e after %d iterations (rtol %.3e)", res, it,
                         rtol);
    return FEM_OK;
}
