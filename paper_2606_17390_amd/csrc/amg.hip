// amg.hip -- aggregation multigrid preconditioner for the Krylov solve of the
// global Newton iteration (Sec. 2.2.5 / App. F: the linear systems are solved
// by a Krylov method preconditioned with algebraic multigrid).
//
// Levels are node-block operators in the layout of fem_csr_pattern (rows 3I+a
// of a node consecutive, sharing one column list of whole 3x3 blocks).  The
// set-up splits into
//   - a symbolic part on the host, once per pattern: aggregation by repeated
//     greedy heaviest-edge matching on the node graph weighted by block
//     norms, the coarse patterns, and for every coarse block the list of fine
//     blocks that sum into it (with the 9-bit mask of free row/column dofs);
//   - a numeric part on the device, once per matrix: Galerkin block sums
//     (one thread per coarse block, fixed order), 3x3 block-Jacobi inverses
//     (32 lanes per node) damped by (4/3) / rho from a power iteration, and
//     the dense inverse of the coarsest operator (one workgroup, Gauss-Jordan
//     in LDS).
// One application is a V(1,1)-cycle: per level a residual product, a
// restriction fused with the next level's first smoothing sweep, and on the
// way up a prolongation and a post-smoothing product; or a K-cycle, whose
// coarse levels above the single-workgroup tail replace the coarse
// correction by two minimal-residual steps (for a flexible outer method).
// Vectors are FP64; the finest operator is K as given (FP64 or FP32), the
// coarse ones FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fem_internal.h"

namespace {

constexpr int kLanes = 32;                       // lanes per node of the block products
constexpr int kDenseMax = 3 * FEM_AMG_DENSE_NODES;  // dofs of a dense coarsest level
constexpr double kStall = 0.85;                  // stop when a level keeps more nodes than this
constexpr int kPostGrid = 2048;                  // workgroup cap of the persistent level products

struct Level {
    int32_t n = 0;           // nodes
    int64_t nb = 0;          // 3x3 blocks
    const int32_t* row_ptr = nullptr;  // device [3n + 1] (level 0: the caller's)
    int32_t* ncol = nullptr;           // device [nb] node column of each block
    float* vals = nullptr;             // device [9 nb] (levels >= 1)
    double* minv = nullptr;            // device [9 n] smoother blocks
    uint8_t* mask = nullptr;           // device [3 n] 1 = free dof
    double *b = nullptr, *x = nullptr, *r = nullptr, *y = nullptr;  // device [3 n]
    // transfer from the level above (levels >= 1)
    int32_t* agg = nullptr;    // [n_fine] aggregate of each fine node
    int32_t* mptr = nullptr;   // [n + 1] members of each aggregate ...
    int32_t* mem = nullptr;    // [n_fine] ... (fine nodes)
    int32_t* gptr = nullptr;   // [nb + 1] fine blocks of each coarse block ...
    int32_t* goff = nullptr;   // [nb_fine] entry offset of the fine block's (0,0) entry
    uint16_t* glen = nullptr;  // [nb_fine] row length of the fine block's rows
    uint16_t* gmask = nullptr; // [nb_fine] bit 3a+c: fine row dof a and column dof c both free
    int32_t* gdst = nullptr;   // [nb] entry offset of the coarse block's (0,0) entry
    uint16_t* gdlen = nullptr; // [nb] row length of the coarse block's rows
    uint8_t* gfix = nullptr;   // [nb] bit a: identity on row a (diagonal block, no free fine dof)
    // K-cycle steps on this level (levels >= 1)
    double* kc1 = nullptr;     // [3 n] first cycle result c1
    double* kv1 = nullptr;     // [3 n] A c1
    double* kpart = nullptr;   // [3 kPostGrid] workgroup partial sums
    double* ksc = nullptr;     // [4] (v1, v1), a1, then the coefficients e1, e2 of c1 and c2
};

}  // namespace

struct fem_amg {
    int device = 0;
    int32_t n_rows = 0;
    int64_t nnz = 0;
    int nl = 0;
    bool dense = false;
    int nd = 0;                // dofs of the dense coarsest level
    double* cinv = nullptr;    // device [nd][nd]
    double* om = nullptr;      // device [FEM_AMG_MAX_LEVELS] smoother damping per level
    double* sc = nullptr;      // device [2 FEM_AMG_MAX_LEVELS] power-iteration norms
    double* part = nullptr;    // device partial sums of the power iteration
    int npart = 0;
    Level L[FEM_AMG_MAX_LEVELS];
    void* mem = nullptr;       // one device allocation for everything above
    const void* K = nullptr;   // values of the last fem_amg_update
    fem_precision prec = FEM_FP64;
    bool updated = false;
    fem_amg_cycle cycle = FEM_AMG_CYCLE_V;
    int32_t kmin = 0;          // K-cycle steps on levels of at least this many nodes
};

namespace fem {
namespace {

__device__ inline bool stopped(const int32_t* fl) { return fl && fl[0]; }

// ---- set-up kernels

// ncol[row_ptr[3I]/9 + k] = J and nrm[...] = Frobenius norm of block (I, J)
template <typename RV>
__global__ __launch_bounds__(256) void cols_norms_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col_idx,
                                                         const RV* __restrict__ val, int32_t* __restrict__ ncol,
                                                         float* __restrict__ nrm) {
    const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
    const int l = (int)(threadIdx.x & (kLanes - 1));
    if (I >= n) return;
    const int32_t b = row_ptr[3 * I], len = row_ptr[3 * I + 1] - b, deg = len / 3;
    for (int32_t k = l; k < deg; k += kLanes) {
        ncol[b / 9 + k] = col_idx[b + 3 * k] / 3;
        if (nrm) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double v = (double)val[(int64_t)b + (int64_t)a * len + 3 * k + c];
                    s += v * v;
                }
            nrm[b / 9 + k] = (float)sqrt(s);
        }
    }
}

// minv[9I..] = inverse of D_I, the diagonal 3x3 block of node I (32 lanes
// per node find it; a singular block falls back to the inverse of its
// diagonal, zero -> 1).  The damping factor is applied afterwards.
template <typename RV>
__global__ __launch_bounds__(256) void bj_minv_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ ncol, const RV* __restrict__ val,
                                                      double* __restrict__ minv) {
    const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes;
    const int l = (int)(threadIdx.x & (kLanes - 1));
    if (I >= n) return;  // whole 32-lane groups leave together
    const int32_t b = row_ptr[3 * I], len = row_ptr[3 * I + 1] - b, deg = len / 3;
    const int32_t* __restrict__ nc = ncol + b / 9;
    int32_t kd = -1;
    for (int32_t k = l; k < deg; k += kLanes)
        if (nc[k] == I) kd = k;
#pragma unroll
    for (int m = 1; m < kLanes; m <<= 1) kd = max(kd, __shfl_xor(kd, m, kLanes));
    if (l != 0) return;
    double D[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    if (kd >= 0)
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) D[a][c] = (double)val[(int64_t)b + (int64_t)a * len + 3 * kd + c];
    const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
    const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
    const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
    const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
    const double scale = fabs(D[0][0] * D[1][1] * D[2][2]);
    double M[9];
    if (det != 0.0 && fabs(det) > 1e-12 * scale && isfinite(1.0 / det)) {
        const double id = 1.0 / det;
        M[0] = c00 * id;
        M[1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
        M[2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
        M[3] = c01 * id;
        M[4] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
        M[5] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
        M[6] = c02 * id;
        M[7] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
        M[8] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
    } else {
        for (int k = 0; k < 9; ++k) M[k] = 0.0;
        for (int a = 0; a < 3; ++a) M[4 * a] = D[a][a] != 0.0 ? 1.0 / D[a][a] : 1.0;
    }
    for (int k = 0; k < 9; ++k) minv[9 * I + k] = M[k];
}

// Galerkin block sums: coarse block q = sum over its fine blocks g of the
// masked 3x3 entries (fixed order, FP64 accumulation, FP32 result).
template <typename RV>
__global__ __launch_bounds__(256) void galerkin_kernel(int64_t nb, const int32_t* __restrict__ gptr,
                                                       const int32_t* __restrict__ goff,
                                                       const uint16_t* __restrict__ glen,
                                                       const uint16_t* __restrict__ gmask,
                                                       const int32_t* __restrict__ gdst,
                                                       const uint16_t* __restrict__ gdlen,
                                                       const uint8_t* __restrict__ gfix, const RV* __restrict__ fine,
                                                       float* __restrict__ coarse) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nb) return;
    double s[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t g = gptr[q]; g < gptr[q + 1]; ++g) {
        const int64_t off = goff[g];
        const int32_t len = glen[g];
        const uint32_t m = gmask[g];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((m >> (3 * a + c)) & 1u) s[3 * a + c] += (double)fine[off + (int64_t)a * len + c];
    }
    const uint32_t fix = gfix[q];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if ((fix >> a) & 1u) s[4 * a] = 1.0;
    const int64_t d = gdst[q];
    const int32_t dl = gdlen[q];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) coarse[d + (int64_t)a * dl + c] = (float)s[3 * a + c];
}

// Explicit inverse of a dense operator of nd <= kDenseMax dofs given in
// node-block CSR (one workgroup): Gauss-Jordan in place with partial
// pivoting, then the column swaps in reverse.  A pivot of magnitude at most
// 1e-13 times the largest diagonal entry drops its dof (zero row and column).
template <typename RV>
__global__ __launch_bounds__(256) void dense_inverse_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ ncol,
                                                            const RV* __restrict__ val, double* __restrict__ out) {
    __shared__ double A[kDenseMax * kDenseMax];
    __shared__ double fcol[kDenseMax];
    __shared__ double rv[256];
    __shared__ int ri[256];
    __shared__ int perm[kDenseMax];
    const int nd = 3 * n, t = threadIdx.x;
    for (int i = t; i < nd * nd; i += 256) A[i] = 0.0;
    __syncthreads();
    for (int I = t; I < n; I += 256) {
        const int32_t b = row_ptr[3 * I], len = row_ptr[3 * I + 1] - b, deg = len / 3;
        for (int k = 0; k < deg; ++k) {
            const int J = ncol[b / 9 + k];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) A[(3 * I + a) * nd + 3 * J + c] = (double)val[b + a * len + 3 * k + c];
        }
    }
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < nd; ++i) dmax = fmax(dmax, fabs(A[i * nd + i]));
    const double tiny = 1e-13 * dmax;
    for (int k = 0; k < nd; ++k) {
        // pivot: largest |A(i, k)|, i >= k (smallest index on ties)
        double bv = -1.0;
        int bi = k;
        for (int i = k + t; i < nd; i += 256) {
            const double v = fabs(A[i * nd + k]);
            if (v > bv) {
                bv = v;
                bi = i;
            }
        }
        rv[t] = bv;
        ri[t] = bi;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) {
                const double v2 = rv[t + o];
                const int i2 = ri[t + o];
                if (v2 > rv[t] || (v2 == rv[t] && i2 < ri[t])) {
                    rv[t] = v2;
                    ri[t] = i2;
                }
            }
            __syncthreads();
        }
        const int p = ri[0];
        if (t == 0) perm[k] = p;
        if (p != k)
            for (int j = t; j < nd; j += 256) {
                const double tmp = A[k * nd + j];
                A[k * nd + j] = A[p * nd + j];
                A[p * nd + j] = tmp;
            }
        __syncthreads();
        const double piv = A[k * nd + k];
        const double pinv = (fabs(piv) > tiny && isfinite(1.0 / piv)) ? 1.0 / piv : 0.0;
        for (int i = t; i < nd; i += 256) fcol[i] = A[i * nd + k];
        __syncthreads();
        for (int j = t; j < nd; j += 256) A[k * nd + j] = (j == k ? 1.0 : A[k * nd + j]) * pinv;
        __syncthreads();
        for (int e = t; e < nd * nd; e += 256) {
            const int i = e / nd, j = e - i * nd;
            if (i != k) A[e] = (j == k ? 0.0 : A[e]) - fcol[i] * A[k * nd + j];
        }
        __syncthreads();
    }
    for (int k = nd - 1; k >= 0; --k) {
        const int p = perm[k];
        if (p != k)
            for (int i = t; i < nd; i += 256) {
                const double tmp = A[i * nd + k];
                A[i * nd + k] = A[i * nd + p];
                A[i * nd + p] = tmp;
            }
        __syncthreads();
    }
    for (int i = t; i < nd * nd; i += 256) out[i] = A[i];
}

// ---- cycle kernels

// x = M b (first smoothing sweep from zero), one thread per node
__global__ __launch_bounds__(256) void smooth0_kernel(int32_t n, const double* __restrict__ minv,
                                                      const double* __restrict__ b, double* __restrict__ x,
                                                      const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    const double* m = minv + 9 * I;
    const double b0 = b[3 * I], b1 = b[3 * I + 1], b2 = b[3 * I + 2];
#pragma unroll
    for (int a = 0; a < 3; ++a) x[3 * I + a] = m[3 * a] * b0 + m[3 * a + 1] * b1 + m[3 * a + 2] * b2;
}

// Second sweep: out = x + M (b - A x); 32 lanes per node over a fixed grid
// of at most kPostGrid workgroups (8 nodes per workgroup and round),
// butterfly over the lanes in a fixed order

template <typename RV>
__global__ __launch_bounds__(256) void post_kernel(int32_t n, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ ncol, const RV* __restrict__ val,
                                                   const double* __restrict__ x, const double* __restrict__ b,
                                                   const double* __restrict__ minv, double* __restrict__ out,
                                                   const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    const int l = (int)(threadIdx.x & (kLanes - 1));
    for (int64_t base = (int64_t)blockIdx.x * 8; base < n; base += (int64_t)gridDim.x * 8) {
        const int64_t I = base + (threadIdx.x >> 5);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (I < n) {
            const int32_t bs = row_ptr[3 * I], len = row_ptr[3 * I + 1] - bs, deg = len / 3;
            const int32_t* __restrict__ nc = ncol + bs / 9;
            for (int32_t k = l; k < deg; k += kLanes) {
                const int64_t J = nc[k];
                const double x0 = x[3 * J], x1 = x[3 * J + 1], x2 = x[3 * J + 2];
                const RV* __restrict__ v = val + bs + 3 * k;
                s0 += (double)v[0] * x0 + (double)v[1] * x1 + (double)v[2] * x2;
                s1 += (double)v[len] * x0 + (double)v[len + 1] * x1 + (double)v[len + 2] * x2;
                s2 += (double)v[2 * len] * x0 + (double)v[2 * len + 1] * x1 + (double)v[2 * len + 2] * x2;
            }
        }
#pragma unroll
        for (int m = 1; m < kLanes; m <<= 1) {
            s0 += __shfl_xor(s0, m, kLanes);
            s1 += __shfl_xor(s1, m, kLanes);
            s2 += __shfl_xor(s2, m, kLanes);
        }
        if (I < n && l < 3) {
            const double r0 = b[3 * I] - s0, r1 = b[3 * I + 1] - s1, r2 = b[3 * I + 2] - s2;
            const double* m = minv + 9 * I;
            out[3 * I + l] = x[3 * I + l] + m[3 * l] * r0 + m[3 * l + 1] * r1 + m[3 * l + 2] * r2;
        }
    }
}

// Residual and restriction in one pass: workgroup C takes the (at most
// eight) nodes of aggregate C, 32 lanes per node compute r = b - A x on its
// rows, and the masked sums over the aggregate give the coarse right-hand
// side cb = P^T r; then the first coarse sweep cx = M_c cb.  The fine
// residual itself is never stored.
template <typename RV>
__global__ __launch_bounds__(256) void resid_restrict_kernel(const int32_t* __restrict__ mptr,
                                                             const int32_t* __restrict__ mem,
                                                             const uint8_t* __restrict__ fmask,
                                                             const int32_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ ncol,
                                                             const RV* __restrict__ val, const double* __restrict__ x,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ cminv, double* __restrict__ cb,
                                                             double* __restrict__ cx, const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    __shared__ double part[8][3];
    const int64_t C = blockIdx.x;
    const int g = (int)(threadIdx.x >> 5), l = (int)(threadIdx.x & (kLanes - 1));
    const int32_t m0 = mptr[C], cnt = mptr[C + 1] - m0;
    int64_t I = -1;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (g < cnt) {
        I = mem[m0 + g];
        const int32_t bs = row_ptr[3 * I], len = row_ptr[3 * I + 1] - bs, deg = len / 3;
        const int32_t* __restrict__ nc = ncol + bs / 9;
        for (int32_t k = l; k < deg; k += kLanes) {
            const int64_t J = nc[k];
            const double x0 = x[3 * J], x1 = x[3 * J + 1], x2 = x[3 * J + 2];
            const RV* __restrict__ v = val + bs + 3 * k;
            s0 += (double)v[0] * x0 + (double)v[1] * x1 + (double)v[2] * x2;
            s1 += (double)v[len] * x0 + (double)v[len + 1] * x1 + (double)v[len + 2] * x2;
            s2 += (double)v[2 * len] * x0 + (double)v[2 * len + 1] * x1 + (double)v[2 * len + 2] * x2;
        }
    }
#pragma unroll
    for (int m = 1; m < kLanes; m <<= 1) {
        s0 += __shfl_xor(s0, m, kLanes);
        s1 += __shfl_xor(s1, m, kLanes);
        s2 += __shfl_xor(s2, m, kLanes);
    }
    if (g < cnt && l < 3) {
        const double ra = b[3 * I + l] - (l == 0 ? s0 : (l == 1 ? s1 : s2));
        part[g][l] = fmask[3 * I + l] ? ra : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < cnt; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a) r[a] += part[k][a];
        const double* m = cminv + 9 * C;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cb[3 * C + a] = r[a];
            cx[3 * C + a] = m[3 * a] * r[0] + m[3 * a + 1] * r[1] + m[3 * a + 2] * r[2];
        }
    }
}

// The levels t, ..., nl - 1 of at most kTailNodes nodes each in one
// workgroup of 1024 threads (that part of the cycle is bound by launch
// latency, not by work): on entry level t holds its right-hand side b and
// first sweep x = M b; on exit its post-smoothed iterate y (or, when level t
// is the dense coarsest level, x = Cinv b).  Phases are separated by
// workgroup barriers.
constexpr int kTailNodes = 512;

struct TailLevel {
    int32_t n;
    const int32_t* row_ptr;
    const int32_t* ncol;
    const float* vals;
    const double* minv;
    const uint8_t* mask;
    double *b, *x, *r, *y;
    const int32_t *agg, *mptr, *mem;  // transfer from the level above (unused at level t)
};

struct TailArgs {
    int nlv;    // levels in the tail
    int dense;  // last one inverted exactly
    int nd;
    const double* cinv;
    TailLevel L[FEM_AMG_MAX_LEVELS];
};

// POST = 0: r = b - A x;  POST = 1: y = x + M (b - A x); kTailLanes lanes
// per node (coarse rows hold some 15 to 25 blocks: 128 nodes per round
// keeps the dependent-load rounds few)
constexpr int kTailLanes = 8;

template <int POST>
__device__ inline void tail_sweep(const TailLevel& F, int tid) {
    const int g = tid / kTailLanes, l = tid & (kTailLanes - 1);
    for (int64_t base = 0; base < F.n; base += 1024 / kTailLanes) {
        const int64_t I = base + g;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (I < F.n) {
            const int32_t bs = F.row_ptr[3 * I], len = F.row_ptr[3 * I + 1] - bs, deg = len / 3;
            for (int32_t k = l; k < deg; k += kTailLanes) {
                const int64_t J = F.ncol[bs / 9 + k];
                const double x0 = F.x[3 * J], x1 = F.x[3 * J + 1], x2 = F.x[3 * J + 2];
                const float* v = F.vals + bs + 3 * k;
                s0 += (double)v[0] * x0 + (double)v[1] * x1 + (double)v[2] * x2;
                s1 += (double)v[len] * x0 + (double)v[len + 1] * x1 + (double)v[len + 2] * x2;
                s2 += (double)v[2 * len] * x0 + (double)v[2 * len + 1] * x1 + (double)v[2 * len + 2] * x2;
            }
        }
#pragma unroll
        for (int m = 1; m < kTailLanes; m <<= 1) {
            s0 += __shfl_xor(s0, m, kTailLanes);
            s1 += __shfl_xor(s1, m, kTailLanes);
            s2 += __shfl_xor(s2, m, kTailLanes);
        }
        if (I < F.n && l < 3) {
            const double r0 = F.b[3 * I] - s0, r1 = F.b[3 * I + 1] - s1, r2 = F.b[3 * I + 2] - s2;
            if (POST) {
                const double* m = F.minv + 9 * I;
                F.y[3 * I + l] = F.x[3 * I + l] + m[3 * l] * r0 + m[3 * l + 1] * r1 + m[3 * l + 2] * r2;
            } else {
                F.r[3 * I + l] = l == 0 ? r0 : (l == 1 ? r1 : r2);
            }
        }
    }
}

__global__ __launch_bounds__(1024) void tail_kernel(TailArgs A, const int32_t* fl) {
    if (stopped(fl)) return;
    const int tid = threadIdx.x;
    const int nlv = A.nlv;
    for (int l = 0; l + 1 < nlv; ++l) {
        const TailLevel& F = A.L[l];
        const TailLevel& C = A.L[l + 1];
        tail_sweep<0>(F, tid);
        __syncthreads();
        // restriction: 8 lanes per coarse node, lane j its member j (an
        // aggregate holds at most 8 nodes), butterfly sums in a fixed order
        for (int64_t base = 0; base < C.n; base += 1024 / 8) {
            const int64_t c = base + (tid >> 3);
            const int j = tid & 7;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            if (c < C.n) {
                const int32_t k0 = C.mptr[c];
                if (j < C.mptr[c + 1] - k0) {
                    const int64_t i = C.mem[k0 + j];
                    if (F.mask[3 * i]) s0 = F.r[3 * i];
                    if (F.mask[3 * i + 1]) s1 = F.r[3 * i + 1];
                    if (F.mask[3 * i + 2]) s2 = F.r[3 * i + 2];
                }
            }
#pragma unroll
            for (int m = 1; m < 8; m <<= 1) {
                s0 += __shfl_xor(s0, m, 8);
                s1 += __shfl_xor(s1, m, 8);
                s2 += __shfl_xor(s2, m, 8);
            }
            if (c < C.n && j < 3) {
                const double* m = C.minv + 9 * c;
                C.b[3 * c + j] = j == 0 ? s0 : (j == 1 ? s1 : s2);
                C.x[3 * c + j] = m[3 * j] * s0 + m[3 * j + 1] * s1 + m[3 * j + 2] * s2;
            }
        }
        __syncthreads();
    }
    const TailLevel& K = A.L[nlv - 1];
    if (A.dense) {
        for (int i = tid; i < A.nd; i += 1024) {
            double s = 0.0;
            for (int j = 0; j < A.nd; ++j) s += A.cinv[(int64_t)i * A.nd + j] * K.b[j];
            K.x[i] = s;
        }
    } else {
        tail_sweep<1>(K, tid);
    }
    __syncthreads();
    const double* yc = A.dense ? K.x : K.y;
    for (int l = nlv - 2; l >= 0; --l) {
        const TailLevel& F = A.L[l];
        const TailLevel& C = A.L[l + 1];
        for (int64_t i = tid; i < F.n; i += 1024) {
            const int64_t c = C.agg[i];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (F.mask[3 * i + a]) F.x[3 * i + a] += yc[3 * c + a];
        }
        __syncthreads();
        tail_sweep<1>(F, tid);
        __syncthreads();
        yc = F.y;
    }
}

// Dense coarsest level (one workgroup): x = Cinv b with b = P^T r (mptr
// given) or b = r (mptr NULL: the finest level is the dense one)
__global__ __launch_bounds__(256) void dense_apply_kernel(int32_t n, const int32_t* __restrict__ mptr,
                                                          const int32_t* __restrict__ mem,
                                                          const uint8_t* __restrict__ fmask,
                                                          const double* __restrict__ r,
                                                          const double* __restrict__ cinv, double* __restrict__ x,
                                                          const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    __shared__ double bs[kDenseMax];
    const int nd = 3 * n, t = threadIdx.x;
    if (t < nd) {
        double s = 0.0;
        if (mptr) {
            const int C = t / 3, a = t - 3 * (t / 3);
            for (int32_t k = mptr[C]; k < mptr[C + 1]; ++k) {
                const int64_t i = mem[k];
                if (fmask[3 * i + a]) s += r[3 * i + a];
            }
        } else {
            s = r[t];
        }
        bs[t] = s;
    }
    __syncthreads();
    if (t < nd) {
        double s = 0.0;
        for (int j = 0; j < nd; ++j) s += cinv[t * nd + j] * bs[j];
        x[t] = s;
    }
}

// x_fine += P y (masked)
__global__ __launch_bounds__(256) void prolong_kernel(int32_t n, const int32_t* __restrict__ agg,
                                                      const uint8_t* __restrict__ fmask, const double* __restrict__ y,
                                                      double* __restrict__ x, const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t C = agg[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (fmask[3 * i + a]) x[3 * i + a] += y[3 * C + a];
}

// ---- damping of the smoother: omega_l = kOmegaNum / rho_l with rho_l the
// spectral radius of D_l^-1 A_l estimated by kPowerSteps power steps from a
// fixed pseudo-random start vector (zero on constrained dofs), so that the
// set-up is deterministic.
constexpr int kPowerSteps = 10;
constexpr double kOmegaNum = 4.0 / 3.0;
constexpr double kOmegaFallback = 0.5;  // for a non-positive or non-finite estimate

// Fixed-order sum of one value per thread of a 256-thread block.
__device__ inline double block_sum256(double v) {
    __shared__ double sh[256];
    __syncthreads();
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    return sh[0];
}

// v[i] = value in [-1, 1) from an integer hash of i (a SplitMix64-style
// finaliser) on free dofs, 0 on constrained ones; part = block sums of v.v
__global__ __launch_bounds__(256) void power_init(int64_t n3, const uint8_t* __restrict__ mask,
                                                  double* __restrict__ v, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x = 0.0;
    if (i < n3) {
        uint64_t h = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        h *= 0x94D049BB133111EBull;
        h ^= h >> 32;
        x = mask[i] ? 2.0 * ((double)(h >> 11) * 0x1.0p-53) - 1.0 : 0.0;
        v[i] = x;
    }
    const double t = block_sum256(x * x);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// w = D^-1 A (sc[1] v), 32 lanes per node over a fixed grid of
// kPowerGrid workgroups (8 nodes per workgroup and round); part = one sum
// of w.w per workgroup
constexpr int kPowerGrid = 2048;

template <typename RV>
__global__ __launch_bounds__(256) void power_apply(int32_t n, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ ncol, const RV* __restrict__ val,
                                                   const double* __restrict__ minv, const double* __restrict__ v,
                                                   const double* __restrict__ sc, double* __restrict__ w,
                                                   double* __restrict__ part) {
    const int l = (int)(threadIdx.x & (kLanes - 1));
    const double scale = sc[1];
    double ww = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 8; base < n; base += (int64_t)gridDim.x * 8) {
        const int64_t I = base + (threadIdx.x >> 5);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (I < n) {
            const int32_t bs = row_ptr[3 * I], len = row_ptr[3 * I + 1] - bs, deg = len / 3;
            const int32_t* __restrict__ nc = ncol + bs / 9;
            for (int32_t k = l; k < deg; k += kLanes) {
                const int64_t J = nc[k];
                const double x0 = v[3 * J], x1 = v[3 * J + 1], x2 = v[3 * J + 2];
                const RV* __restrict__ q = val + bs + 3 * k;
                s0 += (double)q[0] * x0 + (double)q[1] * x1 + (double)q[2] * x2;
                s1 += (double)q[len] * x0 + (double)q[len + 1] * x1 + (double)q[len + 2] * x2;
                s2 += (double)q[2 * len] * x0 + (double)q[2 * len + 1] * x1 + (double)q[2 * len + 2] * x2;
            }
        }
#pragma unroll
        for (int m = 1; m < kLanes; m <<= 1) {
            s0 += __shfl_xor(s0, m, kLanes);
            s1 += __shfl_xor(s1, m, kLanes);
            s2 += __shfl_xor(s2, m, kLanes);
        }
        if (I < n && l < 3) {
            const double* m = minv + 9 * I;
            const double wl = scale * (m[3 * l] * s0 + m[3 * l + 1] * s1 + m[3 * l + 2] * s2);
            w[3 * I + l] = wl;
            ww += wl * wl;
        }
    }
    const double t = block_sum256(ww);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// sc[0] = sqrt(sum of part), sc[1] = 1 / sc[0] (0 for a zero norm)
__global__ __launch_bounds__(256) void power_norm(const double* __restrict__ part, int np, double* __restrict__ sc) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    const double t = block_sum256(s);
    if (threadIdx.x == 0) {
        const double nr = sqrt(t);
        sc[0] = nr;
        sc[1] = nr > 0.0 ? 1.0 / nr : 0.0;
    }
}

// minv *= omega = kOmegaNum / rho, rho = sc[0] (the norm of D^-1 A v for a
// unit v after the last step); om = omega
__global__ __launch_bounds__(256) void power_finish(int32_t n, const double* __restrict__ sc,
                                                    double* __restrict__ minv, double* __restrict__ om) {
    const double rho = sc[0];
    const double omega = (rho > 0.0 && isfinite(kOmegaNum / rho)) ? kOmegaNum / rho : kOmegaFallback;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < 9 * (int64_t)n) minv[i] *= omega;
    if (i == 0) om[0] = omega;
}

// ---- K-cycle (recursive Krylov-accelerated cycle): on a coarse level c the
// coarse-grid correction is not one cycle B_c rc but the minimal-residual
// combination of two: c1 = B_c rc, v1 = A_c c1, a1 = (v1, rc) / (v1, v1),
// r2 = rc - a1 v1, c2 = B_c r2, v2 = A_c c2, g = (v2, v1) / (v1, v1) and
// a2 = (v2, r2) / ((v2, v2) - g (v2, v1)); the correction
// (a1 - a2 g) c1 + a2 c2 minimises |rc - A_c e| over e in span{c1, c2}
// (two steps of GCR; (v1, r2) = 0 gives the short forms).  The cycle then
// varies from one application to the next, so the outer Krylov method must
// be a flexible one.

// STEP 1: v1 = A c (stored), part = workgroup sums of (v1, b), (v1, v1).
// STEP 2: v2 = A c (not stored), part = workgroup sums of (v2, v1),
// (v2, v2), (v2, b).  Rows by 32 lanes as in post_kernel.
template <int STEP>
__global__ __launch_bounds__(256) void kstep_product(int32_t n, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ ncol, const float* __restrict__ val,
                                                     const double* __restrict__ c, const double* __restrict__ b,
                                                     double* __restrict__ v1, double* __restrict__ part,
                                                     const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    const int l = (int)(threadIdx.x & (kLanes - 1));
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 8; base < n; base += (int64_t)gridDim.x * 8) {
        const int64_t I = base + (threadIdx.x >> 5);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (I < n) {
            const int32_t bs = row_ptr[3 * I], len = row_ptr[3 * I + 1] - bs, deg = len / 3;
            const int32_t* __restrict__ nc = ncol + bs / 9;
            for (int32_t k = l; k < deg; k += kLanes) {
                const int64_t J = nc[k];
                const double x0 = c[3 * J], x1 = c[3 * J + 1], x2 = c[3 * J + 2];
                const float* __restrict__ v = val + bs + 3 * k;
                s0 += (double)v[0] * x0 + (double)v[1] * x1 + (double)v[2] * x2;
                s1 += (double)v[len] * x0 + (double)v[len + 1] * x1 + (double)v[len + 2] * x2;
                s2 += (double)v[2 * len] * x0 + (double)v[2 * len + 1] * x1 + (double)v[2 * len + 2] * x2;
            }
        }
#pragma unroll
        for (int m = 1; m < kLanes; m <<= 1) {
            s0 += __shfl_xor(s0, m, kLanes);
            s1 += __shfl_xor(s1, m, kLanes);
            s2 += __shfl_xor(s2, m, kLanes);
        }
        if (I < n && l < 3) {
            const int64_t k = 3 * I + l;
            const double va = l == 0 ? s0 : (l == 1 ? s1 : s2);
            if (STEP == 1) {
                v1[k] = va;
                d0 += va * b[k];
                d1 += va * va;
            } else {
                d0 += va * v1[k];
                d1 += va * va;
                d2 += va * b[k];
            }
        }
    }
    const double t0 = block_sum256(d0), t1 = block_sum256(d1), t2 = STEP == 2 ? block_sum256(d2) : 0.0;
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = t0;
        part[3 * blockIdx.x + 1] = t1;
        part[3 * blockIdx.x + 2] = t2;
    }
}

// One workgroup: the sums of the np workgroup partials (fixed order), then
// STEP 1: ksc[0] = (v1, v1), ksc[1] = a1;  STEP 2: ksc[2] = a1 - a2 g,
// ksc[3] = a2 (zero where a denominator is not positive)
template <int STEP>
__global__ __launch_bounds__(256) void kstep_scalars(int np, const double* __restrict__ part, double* __restrict__ ksc,
                                                     const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    for (int k = (int)threadIdx.x; k < np; k += 256) {
        q0 += part[3 * k];
        q1 += part[3 * k + 1];
        q2 += part[3 * k + 2];
    }
    const double u0 = block_sum256(q0), u1 = block_sum256(q1), u2 = block_sum256(q2);
    if (threadIdx.x != 0) return;
    if (STEP == 1) {
        ksc[0] = u1;
        ksc[1] = u1 > 0.0 ? u0 / u1 : 0.0;
    } else {
        const double vv1 = ksc[0], a1 = ksc[1];
        const double g = vv1 > 0.0 ? u0 / vv1 : 0.0;
        const double den = u1 - g * u0;
        const double a2 = den > 0.0 ? u2 / den : 0.0;
        ksc[2] = a1 - a2 * g;
        ksc[3] = a2;
    }
}

// b -= a1 v1 (b becomes r2) and the first sweep x = M b, one thread per node
__global__ __launch_bounds__(256) void kstep_update(int32_t n, const double* __restrict__ v1,
                                                    const double* __restrict__ ksc, const double* __restrict__ minv,
                                                    double* __restrict__ b, double* __restrict__ x,
                                                    const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n) return;
    const double a1 = ksc[1];
    double r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r[a] = b[3 * I + a] - a1 * v1[3 * I + a];
        b[3 * I + a] = r[a];
    }
    const double* m = minv + 9 * I;
#pragma unroll
    for (int a = 0; a < 3; ++a) x[3 * I + a] = m[3 * a] * r[0] + m[3 * a + 1] * r[1] + m[3 * a + 2] * r[2];
}

// x_fine += P (e1 c1 + e2 c2) (masked), e1, e2 = ksc[2], ksc[3] of the coarse level
__global__ __launch_bounds__(256) void kprolong_kernel(int32_t n, const int32_t* __restrict__ agg,
                                                       const uint8_t* __restrict__ fmask, const double* __restrict__ c1,
                                                       const double* __restrict__ c2, const double* __restrict__ ksc,
                                                       double* __restrict__ x, const int32_t* __restrict__ fl) {
    if (stopped(fl)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double e1 = ksc[2], e2 = ksc[3];
    const int64_t C = agg[i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (fmask[3 * i + a]) x[3 * i + a] += e1 * c1[3 * C + a] + e2 * c2[3 * C + a];
}

inline unsigned blocks_for(int64_t threads) { return (unsigned)((threads + 255) / 256); }

// ---- host-side symbolic set-up

struct HostLevel {
    int32_t n = 0;
    std::vector<int64_t> bptr;    // [n + 1] first block of each node
    std::vector<int32_t> ncol;    // [nb]
    std::vector<double> s;        // [nb] block strengths
    std::vector<uint8_t> mask;    // [3n]
    // transfer from the level above
    std::vector<int32_t> agg, mptr, mem, gptr, goff, gdst;
    std::vector<uint16_t> glen, gmask, gdlen;
    std::vector<uint8_t> gfix;
};

struct Graph {
    int32_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
    std::vector<double> w;
};

// Diagonal strengths (0 where a node has no diagonal block)
std::vector<double> diag_strength(const Graph& g) {
    std::vector<double> d(g.n, 0.0);
    for (int32_t i = 0; i < g.n; ++i)
        for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k)
            if (g.adj[k] == i) d[i] = g.w[k];
    return d;
}

// One greedy matching pass: nodes in index order take their unmatched
// neighbour of largest w_ij / sqrt(w_ii w_jj) (> 0; smallest index on ties).
std::vector<int32_t> match_pass(const Graph& g, int32_t& nc) {
    const std::vector<double> d = diag_strength(g);
    std::vector<int32_t> m(g.n, -1);
    nc = 0;
    for (int32_t i = 0; i < g.n; ++i) {
        if (m[i] >= 0) continue;
        int32_t best = -1;
        double bw = 0.0;
        for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) {
            const int32_t j = g.adj[k];
            if (j == i || m[j] >= 0) continue;
            const double dd = d[i] * d[j];
            if (!(dd > 0.0)) continue;
            const double wij = g.w[k] / std::sqrt(dd);
            if (wij > bw) {
                bw = wij;
                best = j;
            }
        }
        m[i] = nc;
        if (best >= 0) m[best] = nc;
        ++nc;
    }
    return m;
}

// Graph of the aggregates of map m (nc of them): summed strengths, columns ascending.
Graph contract(const Graph& g, const std::vector<int32_t>& m, int32_t nc) {
    std::vector<int32_t> cnt(nc + 1, 0), mem(g.n);
    for (int32_t i = 0; i < g.n; ++i) ++cnt[m[i] + 1];
    for (int32_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < g.n; ++i) mem[fill[m[i]]++] = i;
    Graph o;
    o.n = nc;
    o.ptr.assign(nc + 1, 0);
    std::vector<int32_t> mark(nc, -1);
    std::vector<double> acc(nc, 0.0);
    std::vector<int32_t> cols;
    for (int32_t c = 0; c < nc; ++c) {
        cols.clear();
        for (int32_t t = cnt[c]; t < cnt[c + 1]; ++t) {
            const int32_t i = mem[t];
            for (int64_t k = g.ptr[i]; k < g.ptr[i + 1]; ++k) {
                const int32_t dcol = m[g.adj[k]];
                if (mark[dcol] != c) {
                    mark[dcol] = c;
                    acc[dcol] = 0.0;
                    cols.push_back(dcol);
                }
                acc[dcol] += g.w[k];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t dcol : cols) {
            o.adj.push_back(dcol);
            o.w.push_back(acc[dcol]);
        }
        o.ptr[c + 1] = (int64_t)o.adj.size();
    }
    return o;
}

// Aggregates of a level: three matching passes composed.
std::vector<int32_t> aggregate(const HostLevel& f, int32_t& nc) {
    Graph g;
    g.n = f.n;
    g.ptr = f.bptr;
    g.adj = f.ncol;
    g.w = f.s;
    std::vector<int32_t> agg(f.n);
    for (int32_t i = 0; i < f.n; ++i) agg[i] = i;
    nc = f.n;
    for (int pass = 0; pass < 3; ++pass) {
        int32_t nn = 0;
        const std::vector<int32_t> m = match_pass(g, nn);
        for (int32_t i = 0; i < f.n; ++i) agg[i] = m[agg[i]];
        if (pass < 2) g = contract(g, m, nn);
        nc = nn;
    }
    return agg;
}

// Coarse level of aggregates `agg` (nc of them) of level f.
bool build_coarse(const HostLevel& f, std::vector<int32_t>&& agg, int32_t nc, HostLevel& c) {
    c.n = nc;
    c.agg = std::move(agg);
    c.mptr.assign(nc + 1, 0);
    c.mem.resize(f.n);
    for (int32_t i = 0; i < f.n; ++i) ++c.mptr[c.agg[i] + 1];
    for (int32_t k = 0; k < nc; ++k) {
        if (c.mptr[k + 1] > 8) return false;  // three pairings: at most eight nodes (one workgroup row each)
        c.mptr[k + 1] += c.mptr[k];
    }
    {
        std::vector<int32_t> fill(c.mptr.begin(), c.mptr.end() - 1);
        for (int32_t i = 0; i < f.n; ++i) c.mem[fill[c.agg[i]]++] = i;
    }
    c.mask.assign(3 * (size_t)nc, 0);
    for (int32_t i = 0; i < f.n; ++i)
        for (int a = 0; a < 3; ++a) c.mask[3 * (size_t)c.agg[i] + a] |= f.mask[3 * (size_t)i + a];
    const int64_t nbf = f.bptr[f.n];
    c.bptr.assign(nc + 1, 0);
    c.gptr.assign(1, 0);
    c.goff.resize(nbf);
    c.glen.resize(nbf);
    c.gmask.resize(nbf);
    std::vector<int32_t> mark(nc, -1), pos(nc, 0), cols, cnt, next;
    int64_t gfill = 0;
    for (int32_t C = 0; C < nc; ++C) {
        cols.clear();
        for (int32_t t = c.mptr[C]; t < c.mptr[C + 1]; ++t) {
            const int32_t i = c.mem[t];
            for (int64_t q = f.bptr[i]; q < f.bptr[i + 1]; ++q) {
                const int32_t D = c.agg[f.ncol[q]];
                if (mark[D] != C) {
                    mark[D] = C;
                    cols.push_back(D);
                }
            }
        }
        std::sort(cols.begin(), cols.end());
        const int32_t deg = (int32_t)cols.size();
        if (3 * (int64_t)deg > 65535) return false;
        for (int32_t r = 0; r < deg; ++r) pos[cols[r]] = r;
        const int64_t b0 = c.bptr[C];
        c.bptr[C + 1] = b0 + deg;
        cnt.assign(deg, 0);
        for (int32_t t = c.mptr[C]; t < c.mptr[C + 1]; ++t) {
            const int32_t i = c.mem[t];
            for (int64_t q = f.bptr[i]; q < f.bptr[i + 1]; ++q) ++cnt[pos[c.agg[f.ncol[q]]]];
        }
        next.assign(deg, 0);
        for (int32_t r = 0; r < deg; ++r) {
            next[r] = (int32_t)gfill;
            gfill += cnt[r];
            c.gptr.push_back((int32_t)gfill);
            c.ncol.push_back(cols[r]);
            c.s.push_back(0.0);
            c.gdst.push_back((int32_t)(9 * b0 + 3 * (int64_t)r));
            c.gdlen.push_back((uint16_t)(3 * deg));
            uint8_t fix = 0;
            if (cols[r] == C)
                for (int a = 0; a < 3; ++a)
                    if (!c.mask[3 * (size_t)C + a]) fix |= (uint8_t)(1u << a);
            c.gfix.push_back(fix);
        }
        for (int32_t t = c.mptr[C]; t < c.mptr[C + 1]; ++t) {
            const int32_t i = c.mem[t];
            const int64_t fdeg = f.bptr[i + 1] - f.bptr[i];
            for (int64_t q = f.bptr[i]; q < f.bptr[i + 1]; ++q) {
                const int32_t j = f.ncol[q];
                const int32_t r = pos[c.agg[j]];
                const int32_t g = next[r]++;
                c.goff[g] = (int32_t)(9 * f.bptr[i] + 3 * (q - f.bptr[i]));
                c.glen[g] = (uint16_t)(3 * fdeg);
                uint16_t mb = 0;
                for (int a = 0; a < 3; ++a)
                    for (int cc = 0; cc < 3; ++cc)
                        if (f.mask[3 * (size_t)i + a] && f.mask[3 * (size_t)j + cc]) mb |= (uint16_t)(1u << (3 * a + cc));
                c.gmask[g] = mb;
                c.s[b0 + r] += f.s[q];
            }
        }
    }
    return 9 * c.bptr[nc] < (int64_t)INT32_MAX;
}

// s(I, J) = s(J, I) = the larger of the two (row elimination of constrained
// dofs zeroes their rows, not their columns: a clamped node still couples
// to its neighbours through the columns and must be able to join an
// aggregate; the pattern is structurally symmetric, columns ascending).
void symmetrize_strength(HostLevel& f) {
    for (int32_t I = 0; I < f.n; ++I)
        for (int64_t q = f.bptr[I]; q < f.bptr[I + 1]; ++q) {
            const int32_t J = f.ncol[q];
            if (J <= I) continue;
            const int32_t* b0 = f.ncol.data() + f.bptr[J];
            const int32_t* b1 = f.ncol.data() + f.bptr[J + 1];
            const int32_t* it = std::lower_bound(b0, b1, I);
            if (it == b1 || *it != I) continue;
            const int64_t qt = f.bptr[J] + (it - b0);
            const double m = std::max(f.s[q], f.s[qt]);
            f.s[q] = m;
            f.s[qt] = m;
        }
}

// Levels below H[0] (host): aggregate until at most FEM_AMG_DENSE_NODES
// nodes remain, the coarsening stalls or FEM_AMG_MAX_LEVELS is reached.
bool build_hierarchy(std::vector<HostLevel>& H) {
    symmetrize_strength(H[0]);
    while ((int)H.size() < FEM_AMG_MAX_LEVELS && H.back().n > FEM_AMG_DENSE_NODES) {
        int32_t nc = 0;
        std::vector<int32_t> agg = aggregate(H.back(), nc);
        if ((double)nc > kStall * H.back().n) break;
        H.emplace_back();
        if (!build_coarse(H[H.size() - 2], std::move(agg), nc, H.back())) return false;
    }
    return true;
}

// Damped block-Jacobi blocks of level l (values V): the inverses of the
// diagonal blocks, then omega_l from the power iteration (levels that are
// inverted exactly keep omega = 1: their smoother is not used).
template <typename V>
void smoother_setup(fem_amg* h, int l, const V* vals, hipStream_t s) {
    Level& L = h->L[l];
    const unsigned nbl = blocks_for((int64_t)L.n * kLanes);
    hipLaunchKernelGGL(bj_minv_kernel<V>, dim3(nbl), dim3(256), 0, s, L.n, L.row_ptr, L.ncol, vals, L.minv);
    if (h->dense && l == h->nl - 1) return;
    double* sc = h->sc + 2 * l;
    const unsigned nbi = blocks_for(3 * (int64_t)L.n);
    hipLaunchKernelGGL(power_init, dim3(nbi), dim3(256), 0, s, 3 * (int64_t)L.n, L.mask, L.r, h->part);
    hipLaunchKernelGGL(power_norm, dim3(1), dim3(256), 0, s, h->part, (int)nbi, sc);
    const unsigned npg = std::min<unsigned>(kPowerGrid, blocks_for((int64_t)L.n * kLanes));
    for (int k = 0; k < kPowerSteps; ++k) {
        const double* v = (k & 1) ? L.y : L.r;
        double* w = (k & 1) ? L.r : L.y;
        hipLaunchKernelGGL(power_apply<V>, dim3(npg), dim3(256), 0, s, L.n, L.row_ptr, L.ncol, vals, L.minv, v, sc, w,
                           h->part);
        hipLaunchKernelGGL(power_norm, dim3(1), dim3(256), 0, s, h->part, (int)npg, sc);
    }
    hipLaunchKernelGGL(power_finish, dim3(blocks_for(9 * (int64_t)L.n)), dim3(256), 0, s, L.n, sc, L.minv, h->om + l);
}

template <typename RV>
hipError_t update_typed(fem_amg* h, const RV* K, hipStream_t s) {
    smoother_setup(h, 0, K, s);
    for (int l = 1; l < h->nl; ++l) {
        Level& c = h->L[l];
        const Level& f = h->L[l - 1];
        if (l == 1)
            hipLaunchKernelGGL(galerkin_kernel<RV>, dim3(blocks_for(c.nb)), dim3(256), 0, s, c.nb, c.gptr, c.goff,
                               c.glen, c.gmask, c.gdst, c.gdlen, c.gfix, K, c.vals);
        else
            hipLaunchKernelGGL(galerkin_kernel<float>, dim3(blocks_for(c.nb)), dim3(256), 0, s, c.nb, c.gptr, c.goff,
                               c.glen, c.gmask, c.gdst, c.gdlen, c.gfix, (const float*)f.vals, c.vals);
        smoother_setup(h, l, (const float*)c.vals, s);
    }
    if (h->dense) {
        const Level& c = h->L[h->nl - 1];
        if (h->nl == 1)
            hipLaunchKernelGGL(dense_inverse_kernel<RV>, dim3(1), dim3(256), 0, s, c.n, c.row_ptr, c.ncol, K, h->cinv);
        else
            hipLaunchKernelGGL(dense_inverse_kernel<float>, dim3(1), dim3(256), 0, s, c.n, c.row_ptr, c.ncol,
                               (const float*)c.vals, h->cinv);
    }
    return hipGetLastError();
}

template <typename RV>
void launch_post(const Level& L, const RV* vals, const double* x, const double* b, double* out, const int32_t* fl,
                 hipStream_t s) {
    const unsigned nb = std::min<unsigned>(kPostGrid, blocks_for((int64_t)L.n * kLanes));
    hipLaunchKernelGGL(post_kernel<RV>, dim3(nb), dim3(256), 0, s, L.n, L.row_ptr, L.ncol, vals, x, b, L.minv, out, fl);
}

// out = x + M_l (b - A_l x) on level l (the finest level reads K)
void level_post(const fem_amg* h, int l, const double* x, const double* b, double* out, const int32_t* fl,
                hipStream_t s) {
    const Level& L = h->L[l];
    if (l > 0)
        launch_post<float>(L, L.vals, x, b, out, fl, s);
    else if (h->prec == FEM_FP64)
        launch_post<double>(L, static_cast<const double*>(h->K), x, b, out, fl, s);
    else
        launch_post<float>(L, static_cast<const float*>(h->K), x, b, out, fl, s);
}

}  // namespace

// ---- internal interface (fem_solve_amg)

int amg_update(fem_amg* h, const void* K, fem_precision prec, hipStream_t s) {
    if (!h || !K) return set_error(FEM_EINVAL, "fem_amg_update: handle and K values must not be NULL");
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED) return set_error(FEM_EINVAL, "fem_amg_update: bad precision");
    h->K = K;
    h->prec = prec;
    const hipError_t e = prec == FEM_FP64 ? update_typed(h, static_cast<const double*>(K), s)
                                          : update_typed(h, static_cast<const float*>(K), s);
    if (e != hipSuccess) return set_error(FEM_EHIP, "fem_amg_update: %s", hipGetErrorString(e));
    h->updated = true;
    return FEM_OK;
}

const double* amg_smoother0(const fem_amg* h) { return h->L[0].minv; }
double* amg_level0_x(fem_amg* h) { return h->L[0].x; }
fem_amg_cycle amg_cycle_type(const fem_amg* h) { return h->cycle; }
bool amg_matches(const fem_amg* h, const fem_csr* csr) {
    return h && csr && h->n_rows == csr->n_rows && h->nnz == csr->nnz && h->L[0].row_ptr == csr->row_ptr;
}

namespace {

// first level of the single-workgroup tail (nl if no level is small enough)
int tail_start(const fem_amg* h) {
    for (int l = 1; l < h->nl; ++l)
        if (h->L[l].n <= kTailNodes) return l;
    return h->nl;
}

// level c takes the two K-cycle steps: a level above the tail, not the
// coarsest, with at least kmin nodes, in a K-cycle hierarchy
bool krylov_level(const fem_amg* h, int c, int t) {
    return h->cycle == FEM_AMG_CYCLE_K && c >= 1 && c < t && c < h->nl - 1 && h->L[c].n >= h->kmin;
}

// The cycle from level l down: on entry bl is level l's right-hand side and
// L[l].x its first sweep M_l bl; the result is written to out (levels above
// the tail; at the tail start and below, the tail's own buffers) and
// returned.
const double* cycle_from(fem_amg* h, int l, const double* bl, double* out, int t, const int32_t* fl, hipStream_t s) {
    Level* L = h->L;
    const int nl = h->nl;
    if (l >= t) {  // levels t, ..., nl - 1 in one workgroup
        TailArgs A;
        A.nlv = nl - t;
        A.dense = h->dense ? 1 : 0;
        A.nd = h->nd;
        A.cinv = h->cinv;
        for (int k = t; k < nl; ++k) {
            const Level& S = L[k];
            TailLevel& T = A.L[k - t];
            T.n = S.n;
            T.row_ptr = S.row_ptr;
            T.ncol = S.ncol;
            T.vals = S.vals;
            T.minv = S.minv;
            T.mask = S.mask;
            T.b = S.b;
            T.x = S.x;
            T.r = S.r;
            T.y = S.y;
            T.agg = S.agg;
            T.mptr = S.mptr;
            T.mem = S.mem;
        }
        hipLaunchKernelGGL(tail_kernel, dim3(1), dim3(1024), 0, s, A, fl);
        return (t == nl - 1 && h->dense) ? L[t].x : L[t].y;
    }
    if (l == nl - 1) {  // coarsest level, not inverted and too large for the tail: the second sweep
        level_post(h, l, L[l].x, bl, out, fl, s);
        return out;
    }
    // residual, restriction and the first sweep of level c
    const int c = l + 1;
    Level& C = L[c];
    if (l > 0)
        hipLaunchKernelGGL(resid_restrict_kernel<float>, dim3(C.n), dim3(256), 0, s, C.mptr, C.mem, L[l].mask,
                           L[l].row_ptr, L[l].ncol, (const float*)L[l].vals, L[l].x, bl, C.minv, C.b, C.x, fl);
    else if (h->prec == FEM_FP64)
        hipLaunchKernelGGL(resid_restrict_kernel<double>, dim3(C.n), dim3(256), 0, s, C.mptr, C.mem, L[0].mask,
                           L[0].row_ptr, L[0].ncol, static_cast<const double*>(h->K), L[0].x, bl, C.minv, C.b, C.x,
                           fl);
    else
        hipLaunchKernelGGL(resid_restrict_kernel<float>, dim3(C.n), dim3(256), 0, s, C.mptr, C.mem, L[0].mask,
                           L[0].row_ptr, L[0].ncol, static_cast<const float*>(h->K), L[0].x, bl, C.minv, C.b, C.x,
                           fl);
    if (krylov_level(h, c, t)) {
        const unsigned ng = std::min<unsigned>(kPostGrid, blocks_for((int64_t)C.n * kLanes));
        cycle_from(h, c, C.b, C.kc1, t, fl, s);
        hipLaunchKernelGGL(kstep_product<1>, dim3(ng), dim3(256), 0, s, C.n, C.row_ptr, C.ncol,
                           (const float*)C.vals, (const double*)C.kc1, (const double*)C.b, C.kv1, C.kpart, fl);
        hipLaunchKernelGGL(kstep_scalars<1>, dim3(1), dim3(256), 0, s, (int)ng, (const double*)C.kpart, C.ksc, fl);
        hipLaunchKernelGGL(kstep_update, dim3(blocks_for(C.n)), dim3(256), 0, s, C.n, (const double*)C.kv1,
                           (const double*)C.ksc, (const double*)C.minv, C.b, C.x, fl);
        cycle_from(h, c, C.b, C.y, t, fl, s);
        hipLaunchKernelGGL(kstep_product<2>, dim3(ng), dim3(256), 0, s, C.n, C.row_ptr, C.ncol,
                           (const float*)C.vals, (const double*)C.y, (const double*)C.b, C.kv1, C.kpart, fl);
        hipLaunchKernelGGL(kstep_scalars<2>, dim3(1), dim3(256), 0, s, (int)ng, (const double*)C.kpart, C.ksc, fl);
        hipLaunchKernelGGL(kprolong_kernel, dim3(blocks_for(L[l].n)), dim3(256), 0, s, L[l].n, C.agg, L[l].mask,
                           (const double*)C.kc1, (const double*)C.y, (const double*)C.ksc, L[l].x, fl);
    } else {
        const double* yc = cycle_from(h, c, C.b, C.y, t, fl, s);
        hipLaunchKernelGGL(prolong_kernel, dim3(blocks_for(L[l].n)), dim3(256), 0, s, L[l].n, C.agg, L[l].mask, yc,
                           L[l].x, fl);
    }
    level_post(h, l, L[l].x, bl, out, fl, s);
    return out;
}

}  // namespace

hipError_t amg_apply_cycle(fem_amg* h, const double* b, double* z, bool presmoothed, const int32_t* fl, hipStream_t s) {
    Level* L = h->L;
    const int nl = h->nl;
    if (nl == 1 && h->dense) {
        hipLaunchKernelGGL(dense_apply_kernel, dim3(1), dim3(256), 0, s, L[0].n, nullptr, nullptr, nullptr, b,
                           h->cinv, z, fl);
        return hipGetLastError();
    }
    if (!presmoothed)
        hipLaunchKernelGGL(smooth0_kernel, dim3(blocks_for(L[0].n)), dim3(256), 0, s, L[0].n, L[0].minv, b, L[0].x,
                           fl);
    if (nl == 1) {  // one level, not inverted: the two sweeps
        level_post(h, 0, L[0].x, b, z, fl, s);
        return hipGetLastError();
    }
    cycle_from(h, 0, b, z, tail_start(h), fl, s);
    return hipGetLastError();
}

}  // namespace fem

using namespace fem;

extern "C" int fem_amg_create(const fem_csr* csr, const void* K_vals, fem_precision prec, const uint8_t* bc_mask,
                              fem_amg** out, void* stream) {
    clear_error();
    if (!out) return set_error(FEM_EINVAL, "fem_amg_create: out must not be NULL");
    *out = nullptr;
    if (!csr || !K_vals) return set_error(FEM_EINVAL, "fem_amg_create: csr and K values must not be NULL");
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED) return set_error(FEM_EINVAL, "fem_amg_create: bad precision");
    if (csr->n_rows <= 0 || csr->n_rows % 3 || !csr->row_ptr || !csr->col_idx)
        return set_error(FEM_EINVAL, "fem_amg_create: a non-empty fem_csr_pattern is required");
    if (csr->nnz <= 0 || csr->nnz % 9 || csr->nnz > (int64_t)INT32_MAX)
        return set_error(FEM_EINVAL, "fem_amg_create: nnz must be a positive multiple of 9 below 2^31");
    hipStream_t s = (hipStream_t)stream;
    const int32_t n0 = csr->n_rows / 3;
    const int64_t nb0 = csr->nnz / 9;

    // level 0 graph on the host: block columns, block norms, mask
    std::vector<HostLevel> H(1);
    HostLevel& h0 = H[0];
    h0.n = n0;
    std::vector<int32_t> rp(csr->n_rows + 1);
    std::vector<float> nrm(nb0);
    h0.ncol.resize(nb0);
    h0.mask.assign(3 * (size_t)n0, 1);
    {
        int32_t* dcol = nullptr;
        float* dnrm = nullptr;
        FEM_HIP_CHECK(hipMalloc(&dcol, nb0 * sizeof(int32_t)));
        if (hipMalloc(&dnrm, nb0 * sizeof(float)) != hipSuccess) {
            (void)hipFree(dcol);
            return set_error(FEM_ENOMEM, "fem_amg_create: device allocation of %lld bytes failed",
                             (long long)(nb0 * 4));
        }
        const unsigned nbl = blocks_for((int64_t)n0 * kLanes);
        if (prec == FEM_FP64)
            hipLaunchKernelGGL(cols_norms_kernel<double>, dim3(nbl), dim3(256), 0, s, n0, csr->row_ptr, csr->col_idx,
                               static_cast<const double*>(K_vals), dcol, dnrm);
        else
            hipLaunchKernelGGL(cols_norms_kernel<float>, dim3(nbl), dim3(256), 0, s, n0, csr->row_ptr, csr->col_idx,
                               static_cast<const float*>(K_vals), dcol, dnrm);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(rp.data(), csr->row_ptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h0.ncol.data(), dcol, nb0 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(nrm.data(), dnrm, nb0 * sizeof(float), hipMemcpyDeviceToHost, s);
        std::vector<uint8_t> bc;
        if (e == hipSuccess && bc_mask) {
            bc.resize(csr->n_rows);
            e = hipMemcpyAsync(bc.data(), bc_mask, bc.size(), hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(dcol);
        (void)hipFree(dnrm);
        if (e != hipSuccess) return set_error(FEM_EHIP, "fem_amg_create: %s", hipGetErrorString(e));
        for (size_t i = 0; i < bc.size(); ++i) h0.mask[i] = bc[i] ? 0 : 1;
    }
    h0.bptr.resize(n0 + 1);
    for (int32_t I = 0; I <= n0; ++I) h0.bptr[I] = rp[3 * (size_t)I] / 9;
    if (h0.bptr[n0] != nb0) return set_error(FEM_EINVAL, "fem_amg_create: row_ptr does not match nnz");
    for (int32_t I = 0; I < n0; ++I)
        if (3 * (h0.bptr[I + 1] - h0.bptr[I]) > 65535)
            return set_error(FEM_EINVAL, "fem_amg_create: node %d has more than 21845 neighbours", I);
    h0.s.assign(nrm.begin(), nrm.end());
    nrm.clear();
    nrm.shrink_to_fit();

    if (!build_hierarchy(H))
        return set_error(FEM_EINVAL, "fem_amg_create: a coarse node has more than 21845 neighbours (or an "
                                     "aggregate more than eight nodes)");
    const int nl = (int)H.size();
    const bool dense = H.back().n <= FEM_AMG_DENSE_NODES;

    // one device allocation
    auto sizes = [&](WsCounter& c) {
        for (int l = 0; l < nl; ++l) {
            const HostLevel& hl = H[l];
            const size_t n = hl.n, nb = hl.bptr[hl.n];
            if (l == 0) c.take<int32_t>(nb);
            else {
                c.take<int32_t>(3 * n + 1);
                c.take<int32_t>(nb);
                c.take<float>(9 * nb);
            }
            c.take<double>(9 * n);
            c.take<uint8_t>(3 * n);
            for (int k = 0; k < 4; ++k) c.take<double>(3 * n);
            if (l > 0) {
                const size_t nf = H[l - 1].n, nbf = H[l - 1].bptr[H[l - 1].n];
                c.take<int32_t>(nf);
                c.take<int32_t>(n + 1);
                c.take<int32_t>(nf);
                c.take<int32_t>(nb + 1);
                c.take<int32_t>(nbf);
                c.take<uint16_t>(nbf);
                c.take<uint16_t>(nbf);
                c.take<int32_t>(nb);
                c.take<uint16_t>(nb);
                c.take<uint8_t>(nb);
                c.take<double>(3 * n);
                c.take<double>(3 * n);
                c.take<double>(3 * kPostGrid);
                c.take<double>(4);
            }
        }
        if (dense) c.take<double>((size_t)9 * H.back().n * H.back().n);
        c.take<double>(FEM_AMG_MAX_LEVELS);
        c.take<double>(2 * FEM_AMG_MAX_LEVELS);
        c.take<double>(std::max<int64_t>(blocks_for(3 * (int64_t)H[0].n), kPowerGrid) + 1);
    };
    WsCounter cnt;
    sizes(cnt);
    fem_amg* h = new (std::nothrow) fem_amg();
    if (!h) return set_error(FEM_ENOMEM, "fem_amg_create: host allocation failed");
    (void)hipGetDevice(&h->device);
    const size_t bytes = cnt.used + 256;
    if (hipMalloc(&h->mem, bytes) != hipSuccess) {
        delete h;
        (void)hipGetLastError();
        return set_error(FEM_ENOMEM, "fem_amg_create: device allocation of %zu bytes failed", bytes);
    }
    h->n_rows = csr->n_rows;
    h->nnz = csr->nnz;
    h->nl = nl;
    h->dense = dense;
    h->nd = 3 * H.back().n;
    WsCarver cv(h->mem, bytes);
    double ones[FEM_AMG_MAX_LEVELS];  // initial damping (kept alive until the synchronisation below)
    for (double& o : ones) o = 1.0;
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t nbytes) {
        if (e == hipSuccess && nbytes) e = hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, s);
    };
    std::vector<std::vector<int32_t>> rowps(nl);
    for (int l = 0; l < nl; ++l) {
        const HostLevel& hl = H[l];
        Level& L = h->L[l];
        const size_t n = hl.n, nb = hl.bptr[hl.n];
        L.n = hl.n;
        L.nb = (int64_t)nb;
        if (l == 0) {
            L.row_ptr = csr->row_ptr;
            L.ncol = cv.take<int32_t>(nb);
        } else {
            int32_t* rpd = cv.take<int32_t>(3 * n + 1);
            L.row_ptr = rpd;
            L.ncol = cv.take<int32_t>(nb);
            L.vals = cv.take<float>(9 * nb);
            std::vector<int32_t>& r = rowps[l];
            r.resize(3 * n + 1);
            for (size_t C = 0; C < n; ++C) {
                const int64_t deg = hl.bptr[C + 1] - hl.bptr[C];
                for (int a = 0; a < 3; ++a) r[3 * C + a] = (int32_t)(9 * hl.bptr[C] + a * 3 * deg);
            }
            r[3 * n] = (int32_t)(9 * nb);
            up(rpd, r.data(), r.size() * 4);
        }
        up(L.ncol, hl.ncol.data(), nb * 4);
        L.minv = cv.take<double>(9 * n);
        L.mask = cv.take<uint8_t>(3 * n);
        up(L.mask, hl.mask.data(), 3 * n);
        L.b = cv.take<double>(3 * n);
        L.x = cv.take<double>(3 * n);
        L.r = cv.take<double>(3 * n);
        L.y = cv.take<double>(3 * n);
        if (l > 0) {
            const size_t nf = H[l - 1].n, nbf = H[l - 1].bptr[H[l - 1].n];
            L.agg = cv.take<int32_t>(nf);
            L.mptr = cv.take<int32_t>(n + 1);
            L.mem = cv.take<int32_t>(nf);
            L.gptr = cv.take<int32_t>(nb + 1);
            L.goff = cv.take<int32_t>(nbf);
            L.glen = cv.take<uint16_t>(nbf);
            L.gmask = cv.take<uint16_t>(nbf);
            L.gdst = cv.take<int32_t>(nb);
            L.gdlen = cv.take<uint16_t>(nb);
            L.gfix = cv.take<uint8_t>(nb);
            L.kc1 = cv.take<double>(3 * n);
            L.kv1 = cv.take<double>(3 * n);
            L.kpart = cv.take<double>(3 * kPostGrid);
            L.ksc = cv.take<double>(4);
            up(L.agg, hl.agg.data(), nf * 4);
            up(L.mptr, hl.mptr.data(), (n + 1) * 4);
            up(L.mem, hl.mem.data(), nf * 4);
            up(L.gptr, hl.gptr.data(), (nb + 1) * 4);
            up(L.goff, hl.goff.data(), nbf * 4);
            up(L.glen, hl.glen.data(), nbf * 2);
            up(L.gmask, hl.gmask.data(), nbf * 2);
            up(L.gdst, hl.gdst.data(), nb * 4);
            up(L.gdlen, hl.gdlen.data(), nb * 2);
            up(L.gfix, hl.gfix.data(), nb);
        }
    }
    if (dense) h->cinv = cv.take<double>((size_t)h->nd * h->nd);
    h->om = cv.take<double>(FEM_AMG_MAX_LEVELS);
    h->sc = cv.take<double>(2 * FEM_AMG_MAX_LEVELS);
    h->npart = (int)std::max<int64_t>(blocks_for(3 * (int64_t)n0), kPowerGrid) + 1;
    h->part = cv.take<double>(h->npart);
    up(h->om, ones, sizeof ones);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host vectors are freed on return
    if (e != hipSuccess || !cv.ok()) {
        (void)hipFree(h->mem);
        delete h;
        return set_error(FEM_EHIP, "fem_amg_create: upload failed: %s", hipGetErrorString(e));
    }
    *out = h;
    return FEM_OK;
}

extern "C" int fem_amg_plan_host(int32_t n_nodes, const int64_t* bptr, const int32_t* ncol, const float* strength,
                                 const uint8_t* bc_mask, int32_t* n_levels, int32_t* nodes, int64_t* blocks,
                                 int32_t* agg) {
    clear_error();
    if (n_nodes <= 0 || !bptr || !ncol || !strength || !n_levels)
        return set_error(FEM_EINVAL, "fem_amg_plan_host: n_nodes > 0, bptr, ncol, strength and n_levels required");
    const int64_t nb = bptr[n_nodes];
    if (bptr[0] != 0 || nb <= 0 || 9 * nb > (int64_t)INT32_MAX)
        return set_error(FEM_EINVAL, "fem_amg_plan_host: bptr must start at 0 and end below 2^31 / 9");
    for (int32_t I = 0; I < n_nodes; ++I) {
        if (bptr[I + 1] < bptr[I]) return set_error(FEM_EINVAL, "fem_amg_plan_host: bptr not ascending");
        if (3 * (bptr[I + 1] - bptr[I]) > 65535)
            return set_error(FEM_EINVAL, "fem_amg_plan_host: node %d has more than 21845 neighbours", I);
    }
    for (int64_t q = 0; q < nb; ++q)
        if (ncol[q] < 0 || ncol[q] >= n_nodes) return set_error(FEM_EINVAL, "fem_amg_plan_host: ncol out of range");
    std::vector<HostLevel> H(1);
    HostLevel& h0 = H[0];
    h0.n = n_nodes;
    h0.bptr.assign(bptr, bptr + n_nodes + 1);
    h0.ncol.assign(ncol, ncol + nb);
    h0.s.assign(strength, strength + nb);
    h0.mask.assign(3 * (size_t)n_nodes, 1);
    if (bc_mask)
        for (size_t i = 0; i < h0.mask.size(); ++i) h0.mask[i] = bc_mask[i] ? 0 : 1;
    if (!build_hierarchy(H))
        return set_error(FEM_EINVAL, "fem_amg_plan_host: a coarse node has more than 21845 neighbours");
    *n_levels = (int32_t)H.size();
    size_t off = 0;
    for (size_t l = 0; l < H.size(); ++l) {
        if (nodes) nodes[l] = H[l].n;
        if (blocks) blocks[l] = H[l].bptr[H[l].n];
        if (agg && l > 0) {
            std::copy(H[l].agg.begin(), H[l].agg.end(), agg + off);
            off += H[l].agg.size();
        }
    }
    return FEM_OK;
}

extern "C" int fem_amg_update(fem_amg* amg, const void* K_vals, fem_precision prec, void* stream) {
    clear_error();
    return amg_update(amg, K_vals, prec, (hipStream_t)stream);
}

extern "C" int fem_amg_set_cycle(fem_amg* amg, fem_amg_cycle cycle, int32_t k_min_nodes) {
    clear_error();
    if (!amg) return set_error(FEM_EINVAL, "fem_amg_set_cycle: handle must not be NULL");
    if (cycle != FEM_AMG_CYCLE_V && cycle != FEM_AMG_CYCLE_K)
        return set_error(FEM_EINVAL, "fem_amg_set_cycle: bad cycle type");
    if (k_min_nodes < 0) return set_error(FEM_EINVAL, "fem_amg_set_cycle: k_min_nodes must be >= 0");
    amg->cycle = cycle;
    amg->kmin = k_min_nodes;
    return FEM_OK;
}

extern "C" int fem_amg_apply(fem_amg* amg, const double* r, double* z, void* stream) {
    clear_error();
    if (!amg || !r || !z) return set_error(FEM_EINVAL, "fem_amg_apply: handle, r and z must not be NULL");
    if (r == z) return set_error(FEM_EINVAL, "fem_amg_apply: r and z must not alias");
    if (!amg->updated) return set_error(FEM_EINVAL, "fem_amg_apply: fem_amg_update has not been called");
    FEM_HIP_CHECK(amg_apply_cycle(amg, r, z, false, nullptr, (hipStream_t)stream));
    return FEM_OK;
}

extern "C" int fem_amg_info(const fem_amg* amg, int32_t* n_levels, int32_t* nodes, int64_t* blocks, int32_t* dense,
                            double* omega) {
    clear_error();
    if (!amg) return set_error(FEM_EINVAL, "fem_amg_info: handle must not be NULL");
    if (n_levels) *n_levels = amg->nl;
    if (dense) *dense = amg->dense ? 1 : 0;
    for (int l = 0; l < amg->nl; ++l) {
        if (nodes) nodes[l] = amg->L[l].n;
        if (blocks) blocks[l] = amg->L[l].nb;
    }
    if (omega) FEM_HIP_CHECK(hipMemcpy(omega, amg->om, amg->nl * sizeof(double), hipMemcpyDeviceToHost));
    return FEM_OK;
}

extern "C" int fem_amg_aggregates(const fem_amg* amg, int32_t level, int32_t* agg) {
    clear_error();
    if (!amg || !agg) return set_error(FEM_EINVAL, "fem_amg_aggregates: handle and agg must not be NULL");
    if (level < 1 || level >= amg->nl)
        return set_error(FEM_EINVAL, "fem_amg_aggregates: level %d outside [1, %d)", level, amg->nl);
    FEM_HIP_CHECK(hipMemcpy(agg, amg->L[level].agg, (size_t)amg->L[level - 1].n * sizeof(int32_t),
                            hipMemcpyDeviceToHost));
    return FEM_OK;
}

extern "C" int fem_amg_destroy(fem_amg* amg) {
    clear_error();
    if (!amg) return FEM_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != amg->device) (void)hipSetDevice(amg->device);
    const hipError_t e = hipFree(amg->mem);
    if (cur != amg->device) (void)hipSetDevice(cur);
    delete amg;
    if (e != hipSuccess) return set_error(FEM_EHIP, "fem_amg_destroy: %s", hipGetErrorString(e));
    return FEM_OK;
}
