// solver.hip -- the linear solve of the global Newton iteration (Sec. 2.2.4:
// K du = -R with the Dirichlet rows of App. E replaced by identity rows, so
// K is not symmetric): CSR matrix-vector product, BiCGSTAB, and conjugate
// gradients for a symmetric tangent, preconditioned by the inverse diagonal
// of K or by the inverses of its 3x3 node blocks.
//
// The matrix is the CSR pattern of fem_csr_pattern (rows 3I+a; the three
// rows of a node are consecutive and share their sorted column list, which
// runs over whole node blocks 3J, 3J+1, 3J+2).  Vectors are FP64; the matrix
// values are FP64 or FP32 (the mixed form keeps K in FP32 and solves in FP64).
//
// Solve layout: a node-column list (one index J per 3x3 block, a ninth of
// col_idx) is built once per solve, so the iteration's matrix products read
// the values, one index per block and three consecutive x values per block.
// The dot products are fused into the kernels that produce their operands
// and reduced in two fixed stages (fixed grids), so a solve is bitwise
// reproducible.  Scalars, the iteration count and a stop flag live in device
// memory: every kernel of an iteration returns at once when the flag is set,
// and the host reads the flag back once per chunk of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fem_internal.h"

namespace fem {
namespace {

constexpr int kSpmvLanes = 32;    // lanes per node (3 rows) of the matrix-vector product

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

constexpr int kGrid = 1024;      // blocks of the fused vector kernels (fixed: reproducible reductions)
constexpr int kSpmvGrid = 2048;  // blocks of the fused matrix-vector products
constexpr int kParts = kSpmvGrid > kGrid ? kSpmvGrid : kGrid;
constexpr int kChunk = 32;       // iterations enqueued between two reads of the stop flag
constexpr int kChunkAmg = 4;     // the same with a multigrid cycle per iteration

// Scalars of the iteration (device memory) and integer flags.
enum { S_RHO, S_RHO_NEW, S_ALPHA, S_OMEGA, S_BETA, S_RR, S_BB, S_RES, S_COUNT };
enum { F_STOP, F_ITER, F_CYC, F_J, F_COUNT };  // F_CYC: the GMRES cycle has ended; F_J: its length

// ncol[row_ptr[3I]/9 + k] = J, the node of the k-th 3x3 block of node I's rows
// (each row of node I has 3 deg(I) entries, so row_ptr[3I] is a multiple of 9).
__global__ __launch_bounds__(256) void node_cols_kernel(int32_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        int32_t* __restrict__ ncol) {
    const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSpmvLanes;
    const int l = (int)(threadIdx.x & (kSpmvLanes - 1));
    if (I >= n_nodes) return;
    const int32_t b = row_ptr[3 * I], deg = (row_ptr[3 * I + 1] - b) / 3;
    for (int32_t k = l; k < deg; k += kSpmvLanes) ncol[b / 9 + k] = col_idx[b + 3 * k] / 3;
}

// minv[9I + 3a + c] = preconditioner block of node I: the inverse of the 3x3
// diagonal block K[3I+a][3I+c] (block = 1), or the inverse of its diagonal
// (block = 0).  A zero diagonal entry gives 1; a singular block (or a block
// whose determinant underflows against its diagonal) falls back to its
// diagonal.
template <typename RV>
__global__ __launch_bounds__(256) void precond_kernel(int32_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ ncol, const RV* __restrict__ val,
                                                      int block, double* __restrict__ minv) {
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= n_nodes) return;
    const int32_t b = row_ptr[3 * I], deg = (row_ptr[3 * I + 1] - b) / 3;
    const int32_t* __restrict__ nc = ncol + b / 9;
    int32_t lo = 0, hi = deg - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (nc[mid] < I) lo = mid + 1;
        else hi = mid;
    }
    double D[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    if (deg > 0 && nc[lo] == I)
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) D[a][c] = (double)val[(int64_t)b + (int64_t)a * 3 * deg + 3 * lo + c];
    double M[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool done = false;
    if (block) {
        const double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
        const double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
        const double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
        const double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
        const double scale = fabs(D[0][0] * D[1][1] * D[2][2]);
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
            done = true;
        }
    }
    if (!done)
        for (int a = 0; a < 3; ++a) M[4 * a] = D[a][a] != 0.0 ? 1.0 / D[a][a] : 1.0;
    for (int k = 0; k < 9; ++k) minv[9 * I + k] = M[k];
}

// Fixed-order block sum of one value per thread (256 threads); every thread
// gets the result.
__device__ inline double block_sum(double v) {
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

// Second stage: the sum of n partials in a fixed order (one 256-thread block).
__device__ inline double sum_parts(const double* __restrict__ part, int n) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    return block_sum(s);
}

// y = K x on node blocks with the fused partial dot products
//   ND >= 1: part0[block] = sum of w . y over the block's rows
//   ND == 2: part1[block] = sum of y . y
// 32 lanes per node, lane k takes the 3x3 blocks k, k + 32 of the node's rows;
// fixed grid kSpmvGrid, 8 nodes per block and round.  Skipped when the stop
// flag is set (if `fl` is given).
template <typename RV, int ND>
__global__ __launch_bounds__(256) void spmv_dot_kernel(int32_t n_nodes, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ ncol,
                                                       const RV* __restrict__ val, const double* __restrict__ x,
                                                       double* __restrict__ y, const double* __restrict__ w,
                                                       double* __restrict__ part0, double* __restrict__ part1,
                                                       const int32_t* __restrict__ fl) {
    if (fl && fl[F_STOP]) return;
    const int l = (int)(threadIdx.x & (kSpmvLanes - 1));
    double d0 = 0.0, d1 = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 8; base < n_nodes; base += (int64_t)kSpmvGrid * 8) {
        const int64_t node = base + (threadIdx.x >> 5);
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (node < n_nodes) {
            const int32_t b = row_ptr[3 * node], len = row_ptr[3 * node + 1] - b, deg = len / 3;
            const int32_t* __restrict__ nc = ncol + b / 9;
            for (int32_t k = l; k < deg; k += kSpmvLanes) {
                const int64_t J = nc[k];
                const double x0 = x[3 * J], x1 = x[3 * J + 1], x2 = x[3 * J + 2];
                const RV* __restrict__ v = val + b + 3 * k;
                s0 += (double)v[0] * x0 + (double)v[1] * x1 + (double)v[2] * x2;
                s1 += (double)v[len] * x0 + (double)v[len + 1] * x1 + (double)v[len + 2] * x2;
                s2 += (double)v[2 * len] * x0 + (double)v[2 * len + 1] * x1 + (double)v[2 * len + 2] * x2;
            }
        }
#pragma unroll
        for (int m = 1; m < kSpmvLanes; m <<= 1) {
            s0 += __shfl_xor(s0, m, kSpmvLanes);
            s1 += __shfl_xor(s1, m, kSpmvLanes);
            s2 += __shfl_xor(s2, m, kSpmvLanes);
        }
        if (node < n_nodes && l < 3) {
            const double yl = l == 0 ? s0 : (l == 1 ? s1 : s2);
            y[3 * node + l] = yl;
            if (ND >= 1) d0 += w[3 * node + l] * yl;
            if (ND == 2) d1 += yl * yl;
        }
    }
    if (ND >= 1) {
        const double t0 = block_sum(d0);
        if (threadIdx.x == 0) part0[blockIdx.x] = t0;
    }
    if (ND == 2) {
        const double t1 = block_sum(d1);
        if (threadIdx.x == 0) part1[blockIdx.x] = t1;
    }
}

__device__ inline void apply_minv(const double* __restrict__ minv, int64_t I, const double q[3], double* out) {
    const double* m = minv + 9 * I;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[3 * I + a] = m[3 * a] * q[0] + m[3 * a + 1] * q[1] + m[3 * a + 2] * q[2];
}

__global__ void reset_flags(int32_t* __restrict__ fl) {
    for (int k = 0; k < F_COUNT; ++k) fl[k] = 0;
}

// r = b - y, rh = r, p = v = 0; part0 = partials of r . r, part1 = of b . b
__global__ __launch_bounds__(256) void init_kernel(int64_t n, const double* __restrict__ b,
                                                   const double* __restrict__ y, double* __restrict__ r,
                                                   double* __restrict__ rh, double* __restrict__ p,
                                                   double* __restrict__ v, double* __restrict__ part0,
                                                   double* __restrict__ part1) {
    double rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kGrid * 256) {
        const double bi = b[i], ri = bi - y[i];
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        rr += ri * ri;
        bb += bi * bi;
    }
    const double t0 = block_sum(rr);
    const double t1 = block_sum(bb);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = t0;
        part1[blockIdx.x] = t1;
    }
}

__device__ inline double rel_of(double rr, double bb) {
    const double bn = sqrt(bb);
    return bn > 0.0 ? sqrt(rr) / bn : sqrt(rr);
}

__global__ __launch_bounds__(256) void fin_init(const double* __restrict__ part0, const double* __restrict__ part1,
                                                double* __restrict__ sc, int32_t* __restrict__ fl, double rtol,
                                                int32_t max_iter) {
    const double rr = sum_parts(part0, kGrid);
    const double bb = sum_parts(part1, kGrid);
    if (threadIdx.x == 0) {
        const double res = rel_of(rr, bb);
        sc[S_RHO] = 1.0;
        sc[S_ALPHA] = 1.0;
        sc[S_OMEGA] = 1.0;
        sc[S_RHO_NEW] = rr;  // (rh, r) with rh = r
        sc[S_BETA] = 0.0;    // p = v = 0: the first direction is r
        sc[S_RR] = rr;
        sc[S_BB] = bb;
        sc[S_RES] = res;
        fl[F_ITER] = 0;
        fl[F_STOP] = (res <= rtol || !isfinite(res) || max_iter <= 0 || (bb == 0.0 && rr == 0.0)) ? 1 : 0;
    }
}

// p = r + beta (p - omega v); ph = M p   (one thread per node)
__global__ __launch_bounds__(256) void update_p(int32_t n_nodes, const double* __restrict__ r,
                                                const double* __restrict__ v, const double* __restrict__ minv,
                                                double* __restrict__ p, double* __restrict__ ph,
                                                const double* __restrict__ sc, const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double beta = sc[S_BETA], omega = sc[S_OMEGA];
    for (int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x; I < n_nodes; I += (int64_t)kGrid * 256) {
        double q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a] = r[3 * I + a] + beta * (p[3 * I + a] - omega * v[3 * I + a]);
            p[3 * I + a] = q[a];
        }
        apply_minv(minv, I, q, ph);
    }
}

// alpha = rho_new / (rh, v) (breakdown if (rh, v) = 0 or alpha is not finite)
__global__ __launch_bounds__(256) void fin_alpha(const double* __restrict__ part0, double* __restrict__ sc,
                                                 int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double rv = sum_parts(part0, kSpmvGrid);
    if (threadIdx.x == 0) {
        const double alpha = sc[S_RHO_NEW] / rv;
        if (rv == 0.0 || !isfinite(alpha)) fl[F_STOP] = 1;
        else sc[S_ALPHA] = alpha;
    }
}

// s = r - alpha v; sh = M s
__global__ __launch_bounds__(256) void update_s(int32_t n_nodes, const double* __restrict__ r,
                                                const double* __restrict__ v, const double* __restrict__ minv,
                                                double* __restrict__ s, double* __restrict__ sh,
                                                const double* __restrict__ sc, const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double alpha = sc[S_ALPHA];
    for (int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x; I < n_nodes; I += (int64_t)kGrid * 256) {
        double q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a] = r[3 * I + a] - alpha * v[3 * I + a];
            s[3 * I + a] = q[a];
        }
        apply_minv(minv, I, q, sh);
    }
}

// omega = (t, s) / (t, t) (0 if t = 0)
__global__ __launch_bounds__(256) void fin_omega(const double* __restrict__ part0, const double* __restrict__ part1,
                                                 double* __restrict__ sc, const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double ts = sum_parts(part0, kSpmvGrid);
    const double tt = sum_parts(part1, kSpmvGrid);
    if (threadIdx.x == 0) sc[S_OMEGA] = tt > 0.0 ? ts / tt : 0.0;
}

// x += alpha ph + omega sh; r = s - omega t; part0 = partials of (rh, r),
// part1 = of (r, r)
__global__ __launch_bounds__(256) void update_x(int64_t n, const double* __restrict__ ph,
                                                const double* __restrict__ sh, const double* __restrict__ s,
                                                const double* __restrict__ t, const double* __restrict__ rh,
                                                double* __restrict__ x, double* __restrict__ r,
                                                double* __restrict__ part0, double* __restrict__ part1,
                                                const double* __restrict__ sc, const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
    double d0 = 0.0, d1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kGrid * 256) {
        x[i] += alpha * ph[i] + omega * sh[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        d0 += rh[i] * ri;
        d1 += ri * ri;
    }
    const double t0 = block_sum(d0);
    const double t1 = block_sum(d1);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = t0;
        part1[blockIdx.x] = t1;
    }
}

// end of an iteration: rho, rho_new, the residual, beta for the next
// direction; stop on convergence, a non-finite residual, a breakdown
// (rho_new = 0 or omega = 0) or the iteration limit
__global__ __launch_bounds__(256) void fin_rho(const double* __restrict__ part0, const double* __restrict__ part1,
                                               double* __restrict__ sc, int32_t* __restrict__ fl, double rtol,
                                               int32_t max_iter) {
    if (fl[F_STOP]) return;
    const double rho_new = sum_parts(part0, kGrid);
    const double rr = sum_parts(part1, kGrid);
    if (threadIdx.x == 0) {
        const double rho = sc[S_RHO_NEW], alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
        const double res = rel_of(rr, sc[S_BB]);
        const int32_t it = fl[F_ITER] + 1;
        sc[S_RHO] = rho;
        sc[S_RHO_NEW] = rho_new;
        sc[S_RR] = rr;
        sc[S_RES] = res;
        sc[S_BETA] = (rho_new / rho) * (alpha / omega);
        fl[F_ITER] = it;
        if (res <= rtol || !isfinite(res) || rho_new == 0.0 || omega == 0.0 || it >= max_iter) fl[F_STOP] = 1;
    }
}

// ---- preconditioned conjugate gradients (symmetric K: the tangent without
// F-bar; identity rows of constrained dofs with x = b = 0 there keep every
// iterate zero on them, so the iteration runs on the free-free block)

// r = b - y; z = M r; p = z; part0 = partials of (r, z), part1 = of (r, r),
// part2 = of (b, b)   (one thread per node)
__global__ __launch_bounds__(256) void cg_init(int32_t n_nodes, const double* __restrict__ b,
                                               const double* __restrict__ y, const double* __restrict__ minv,
                                               double* __restrict__ r, double* __restrict__ z,
                                               double* __restrict__ p, double* __restrict__ part0,
                                               double* __restrict__ part1, double* __restrict__ part2) {
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x; I < n_nodes; I += (int64_t)kGrid * 256) {
        double q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double bi = b[3 * I + a];
            q[a] = bi - y[3 * I + a];
            r[3 * I + a] = q[a];
            rr += q[a] * q[a];
            bb += bi * bi;
        }
        apply_minv(minv, I, q, z);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double zi = z[3 * I + a];
            p[3 * I + a] = zi;
            rz += q[a] * zi;
        }
    }
    const double t0 = block_sum(rz), t1 = block_sum(rr), t2 = block_sum(bb);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = t0;
        part1[blockIdx.x] = t1;
        part2[blockIdx.x] = t2;
    }
}

__global__ __launch_bounds__(256) void cg_fin_init(const double* __restrict__ part0, const double* __restrict__ part1,
                                                   const double* __restrict__ part2, double* __restrict__ sc,
                                                   int32_t* __restrict__ fl, double rtol, int32_t max_iter) {
    const double rz = sum_parts(part0, kGrid);
    const double rr = sum_parts(part1, kGrid);
    const double bb = sum_parts(part2, kGrid);
    if (threadIdx.x == 0) {
        const double res = rel_of(rr, bb);
        sc[S_RHO] = rz;
        sc[S_RR] = rr;
        sc[S_BB] = bb;
        sc[S_RES] = res;
        fl[F_ITER] = 0;
        fl[F_STOP] = (res <= rtol || !isfinite(res) || max_iter <= 0 || rz == 0.0) ? 1 : 0;
    }
}

// alpha = rho / (p, K p); stop if (p, K p) <= 0 (K not positive definite on
// the search space) or alpha is not finite
__global__ __launch_bounds__(256) void cg_fin_alpha(const double* __restrict__ part0, double* __restrict__ sc,
                                                    int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double pq = sum_parts(part0, kSpmvGrid);
    if (threadIdx.x == 0) {
        const double alpha = sc[S_RHO] / pq;
        if (!(pq > 0.0) || !isfinite(alpha)) fl[F_STOP] = 1;
        else sc[S_ALPHA] = alpha;
    }
}

// x += alpha p; r -= alpha q; z = M r; part0 = partials of (r, z), part1 =
// of (r, r)   (one thread per node)
__global__ __launch_bounds__(256) void cg_update(int32_t n_nodes, const double* __restrict__ p,
                                                 const double* __restrict__ q, const double* __restrict__ minv,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ z, double* __restrict__ part0,
                                                 double* __restrict__ part1, const double* __restrict__ sc,
                                                 const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double alpha = sc[S_ALPHA];
    double rz = 0.0, rr = 0.0;
    for (int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x; I < n_nodes; I += (int64_t)kGrid * 256) {
        double ri[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            x[3 * I + a] += alpha * p[3 * I + a];
            ri[a] = r[3 * I + a] - alpha * q[3 * I + a];
            r[3 * I + a] = ri[a];
            rr += ri[a] * ri[a];
        }
        const double* m = minv + 9 * I;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double zi = m[3 * a] * ri[0] + m[3 * a + 1] * ri[1] + m[3 * a + 2] * ri[2];
            z[3 * I + a] = zi;
            rz += ri[a] * zi;
        }
    }
    const double t0 = block_sum(rz), t1 = block_sum(rr);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = t0;
        part1[blockIdx.x] = t1;
    }
}

// end of a CG iteration: beta = rho_new / rho, the residual, stop tests
__global__ __launch_bounds__(256) void cg_fin_beta(const double* __restrict__ part0, const double* __restrict__ part1,
                                                   double* __restrict__ sc, int32_t* __restrict__ fl, double rtol,
                                                   int32_t max_iter) {
    if (fl[F_STOP]) return;
    const double rz = sum_parts(part0, kGrid);
    const double rr = sum_parts(part1, kGrid);
    if (threadIdx.x == 0) {
        const double res = rel_of(rr, sc[S_BB]);
        const int32_t it = fl[F_ITER] + 1;
        sc[S_BETA] = rz / sc[S_RHO];
        sc[S_RHO] = rz;
        sc[S_RR] = rr;
        sc[S_RES] = res;
        fl[F_ITER] = it;
        if (res <= rtol || !isfinite(res) || rz == 0.0 || it >= max_iter) fl[F_STOP] = 1;
    }
}

// p = z + beta p
__global__ __launch_bounds__(256) void cg_update_p(int64_t n, const double* __restrict__ z, double* __restrict__ p,
                                                   const double* __restrict__ sc, const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    const double beta = sc[S_BETA];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kGrid * 256) p[i] = z[i] + beta * p[i];
}

// ---- kernels of the multigrid-preconditioned iterations (z = V-cycle of r
// computed between them)

// p = z; part0 = partials of (r, z)
__global__ __launch_bounds__(256) void cg_amg_start(int64_t n, const double* __restrict__ z,
                                                    const double* __restrict__ r, double* __restrict__ p,
                                                    double* __restrict__ part0, const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    double d = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kGrid * 256) {
        const double zi = z[i];
        p[i] = zi;
        d += r[i] * zi;
    }
    const double t0 = block_sum(d);
    if (threadIdx.x == 0) part0[blockIdx.x] = t0;
}

// part0 = partials of (a, b)
__global__ __launch_bounds__(256) void dot_kernel(int64_t n, const double* __restrict__ a,
                                                  const double* __restrict__ b, double* __restrict__ part0,
                                                  const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    double d = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kGrid * 256) d += a[i] * b[i];
    const double t0 = block_sum(d);
    if (threadIdx.x == 0) part0[blockIdx.x] = t0;
}

// ---- restarted GMRES(kGmresM), right-preconditioned (K M y = b, x = M y):
// Arnoldi by classical Gram-Schmidt with fused dot products (fixed-order
// two-stage sums), Givens rotations of the Hessenberg column on the device,
// the solution formed at the end of each cycle and the true residual
// recomputed for the restart.  The flexible variant (FGMRES, Saad 1993)
// keeps z_j = M v_j of every step and forms x += Z y, so M may change from
// step to step (a K-cycle).  Inner kernels return at once when the cycle
// has ended (F_CYC, passed as the flag pointer), end-of-cycle kernels when
// it had no step (F_J = 0).
constexpr int kGmresM = FEM_GMRES_RESTART;

// v = scale v (scale = sc[S_BETA]); mx = M0 v (node blocks)
__global__ __launch_bounds__(256) void gm_normalize(int32_t n_nodes, double* __restrict__ v,
                                                    const double* __restrict__ minv, double* __restrict__ mx,
                                                    const double* __restrict__ sc, const int32_t* __restrict__ fl) {
    if (fl[0]) return;
    const double scale = sc[S_BETA];
    for (int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x; I < n_nodes; I += (int64_t)kGrid * 256) {
        double q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q[a] = scale * v[3 * I + a];
            v[3 * I + a] = q[a];
        }
        apply_minv(minv, I, q, mx);
    }
}

// hpart[i][block] = partial of (w, v_i), i = 0..j
__global__ __launch_bounds__(256) void gm_dots(int64_t n, int j, const double* __restrict__ V, int64_t ldv,
                                               const double* __restrict__ w, double* __restrict__ hpart,
                                               const int32_t* __restrict__ fl) {
    if (fl[0]) return;
    for (int i = 0; i <= j; ++i) {
        const double* __restrict__ vi = V + (int64_t)i * ldv;
        double d = 0.0;
        for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)kGrid * 256) d += w[k] * vi[k];
        const double t = block_sum(d);
        if (threadIdx.x == 0) hpart[(int64_t)i * kGrid + blockIdx.x] = t;
    }
}

// H(i, j) = sum of hpart[i][*], one block per i
__global__ __launch_bounds__(256) void gm_hreduce(const double* __restrict__ hpart, int j, double* __restrict__ H,
                                                  const int32_t* __restrict__ fl) {
    if (fl[0]) return;
    const int i = blockIdx.x;
    const double t = sum_parts(hpart + (int64_t)i * kGrid, kGrid);
    if (threadIdx.x == 0) H[(int64_t)j * (kGmresM + 1) + i] = t;
}

// w -= sum_i H(i, j) v_i; part0 = partials of (w, w)
__global__ __launch_bounds__(256) void gm_update(int64_t n, int j, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ H, double* __restrict__ w,
                                                 double* __restrict__ part0, const int32_t* __restrict__ fl) {
    if (fl[0]) return;
    const double* __restrict__ h = H + (int64_t)j * (kGmresM + 1);
    double d = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)kGrid * 256) {
        double wk = w[k];
        for (int i = 0; i <= j; ++i) wk -= h[i] * V[(int64_t)i * ldv + k];
        w[k] = wk;
        d += wk * wk;
    }
    const double t = block_sum(d);
    if (threadIdx.x == 0) part0[blockIdx.x] = t;
}

// End of step j: H(j+1, j) = ||w||, the earlier rotations applied to column
// j, a new rotation zeroing H(j+1, j), g rotated; |g(j+1)| / ||b|| is the
// residual of the cycle's least-squares solution.  The cycle ends on
// convergence, a breakdown (H(j+1, j) = 0: the solution is in the space),
// a non-finite value, the iteration limit or after kGmresM steps.
__global__ __launch_bounds__(256) void gm_finish(const double* __restrict__ part0, int j, double* __restrict__ H,
                                                 double* __restrict__ cs, double* __restrict__ sn,
                                                 double* __restrict__ g, double* __restrict__ sc,
                                                 int32_t* __restrict__ fl, double rtol, int32_t max_iter) {
    if (fl[F_CYC]) return;
    const double ww = sum_parts(part0, kGrid);
    if (threadIdx.x != 0) return;
    double* h = H + (int64_t)j * (kGmresM + 1);
    const double hn = sqrt(ww);
    h[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = h[i], b = h[i + 1];
        h[i] = cs[i] * a + sn[i] * b;
        h[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = h[j], b = h[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, sgn = r > 0.0 ? b / r : 0.0;
    cs[j] = c;
    sn[j] = sgn;
    h[j] = r;
    h[j + 1] = 0.0;
    const double gj = g[j];
    g[j] = c * gj;
    g[j + 1] = -sgn * gj;
    const double bn = sqrt(sc[S_BB]);
    const double res = bn > 0.0 ? fabs(g[j + 1]) / bn : fabs(g[j + 1]);
    const int32_t it = fl[F_ITER] + 1;
    fl[F_ITER] = it;
    fl[F_J] = j + 1;
    sc[S_RES] = res;
    sc[S_BETA] = hn > 0.0 ? 1.0 / hn : 0.0;
    const bool stop = res <= rtol || !isfinite(res) || hn == 0.0 || !(r > 0.0) || it >= max_iter;
    if (stop) fl[F_STOP] = 1;
    if (stop || j + 1 == kGmresM) fl[F_CYC] = 1;
}

// y = R^-1 g over the cycle's F_J steps (upper triangular H), one thread
__global__ void gm_solve_y(const double* __restrict__ H, const double* __restrict__ g, double* __restrict__ y,
                           const int32_t* __restrict__ fl) {
    const int m = fl[F_J];
    for (int i = m - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < m; ++k) t -= H[(int64_t)k * (kGmresM + 1) + i] * y[k];
        const double d = H[(int64_t)i * (kGmresM + 1) + i];
        y[i] = d != 0.0 ? t / d : 0.0;
    }
}

// u = sum_{i < F_J} y_i v_i (zero if the cycle had no step)
__global__ __launch_bounds__(256) void gm_combine(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                  const double* __restrict__ y, double* __restrict__ u,
                                                  const int32_t* __restrict__ fl) {
    const int m = fl[F_J];
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)kGrid * 256) {
        double t = 0.0;
        for (int i = 0; i < m; ++i) t += y[i] * V[(int64_t)i * ldv + k];
        u[k] = t;
    }
}

// z = M0 u (node blocks: the block-Jacobi preconditioner)
__global__ __launch_bounds__(256) void gm_apply_minv(int32_t n_nodes, const double* __restrict__ minv,
                                                     const double* __restrict__ u, double* __restrict__ z) {
    for (int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x; I < n_nodes; I += (int64_t)kGrid * 256) {
        const double q[3] = {u[3 * I], u[3 * I + 1], u[3 * I + 2]};
        apply_minv(minv, I, q, z);
    }
}

// x += z
__global__ __launch_bounds__(256) void gm_addx(int64_t n, const double* __restrict__ z, double* __restrict__ x) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)kGrid * 256) x[k] += z[k];
}

// v0 = b - y (y = K x); part0 = partials of (v0, v0), part1 = of (b, b)
__global__ __launch_bounds__(256) void gm_residual(int64_t n, const double* __restrict__ b,
                                                   const double* __restrict__ y, double* __restrict__ v0,
                                                   double* __restrict__ part0, double* __restrict__ part1,
                                                   const int32_t* __restrict__ fl) {
    if (fl[F_STOP]) return;
    double rr = 0.0, bb = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)kGrid * 256) {
        const double bk = b[k], rk = bk - y[k];
        v0[k] = rk;
        rr += rk * rk;
        bb += bk * bk;
    }
    const double t0 = block_sum(rr), t1 = block_sum(bb);
    if (threadIdx.x == 0) {
        part0[blockIdx.x] = t0;
        part1[blockIdx.x] = t1;
    }
}

// start of a cycle: beta = ||v0||, g = beta e1, S_BETA = 1/beta (||b||
// taken on the first start only); stops on a converged or non-finite
// residual or max_iter <= 0
__global__ __launch_bounds__(256) void gm_start(const double* __restrict__ part0, const double* __restrict__ part1,
                                                double* __restrict__ g, double* __restrict__ sc,
                                                int32_t* __restrict__ fl, double rtol, int32_t max_iter,
                                                int first) {
    if (fl[F_STOP]) return;
    const double rr = sum_parts(part0, kGrid);
    const double bb = first ? sum_parts(part1, kGrid) : 0.0;
    if (threadIdx.x != 0) return;
    if (first) sc[S_BB] = bb;
    const double beta = sqrt(rr);
    const double res = rel_of(rr, sc[S_BB]);
    for (int i = 0; i <= kGmresM; ++i) g[i] = 0.0;
    g[0] = beta;
    sc[S_RES] = res;
    sc[S_BETA] = beta > 0.0 ? 1.0 / beta : 0.0;
    fl[F_J] = 0;
    fl[F_CYC] = 0;
    if (res <= rtol || !isfinite(res) || beta == 0.0 || max_iter <= 0 || fl[F_ITER] >= max_iter) {
        fl[F_STOP] = 1;
        fl[F_CYC] = 1;
    }
}

struct GmresWs {
    double *V, *Z, *H, *cs, *sn, *g, *y, *hpart;
    int64_t ldv;
};

// flexible: also the preconditioned vectors z_j = M_j v_j (FGMRES)
template <typename C>
void carve_gmres(C& c, int32_t n, bool flexible, GmresWs* w) {
    GmresWs o;
    o.ldv = ((int64_t)n + 31) / 32 * 32;
    o.V = c.template take<double>((size_t)o.ldv * (kGmresM + 1));
    o.Z = flexible ? c.template take<double>((size_t)o.ldv * kGmresM) : nullptr;
    o.H = c.template take<double>((size_t)(kGmresM + 1) * kGmresM);
    o.cs = c.template take<double>(kGmresM + 1);
    o.sn = c.template take<double>(kGmresM + 1);
    o.g = c.template take<double>(kGmresM + 1);
    o.y = c.template take<double>(kGmresM + 1);
    o.hpart = c.template take<double>((size_t)(kGmresM + 1) * kGrid);
    if (w) *w = o;
}

struct SolverWs {
    double *r, *rh, *p, *ph, *v, *s, *sh, *t, *minv, *part0, *part1, *part2, *sc;
    int32_t *ncol, *fl;
};

template <typename C>
void carve_solver(C& c, int32_t n, int64_t nnz, SolverWs* w) {
    SolverWs o;
    o.r = c.template take<double>((size_t)n + 1);
    o.rh = c.template take<double>((size_t)n + 1);
    o.p = c.template take<double>((size_t)n + 1);
    o.ph = c.template take<double>((size_t)n + 1);
    o.v = c.template take<double>((size_t)n + 1);
    o.s = c.template take<double>((size_t)n + 1);
    o.sh = c.template take<double>((size_t)n + 1);
    o.t = c.template take<double>((size_t)n + 1);
    o.minv = c.template take<double>(3 * (size_t)n + 1);
    o.part0 = c.template take<double>(kParts);
    o.part1 = c.template take<double>(kParts);
    o.part2 = c.template take<double>(kParts);
    o.sc = c.template take<double>(S_COUNT);
    o.ncol = c.template take<int32_t>((size_t)(nnz / 9) + 1);
    o.fl = c.template take<int32_t>(F_COUNT);
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

template <int ND>
void spmv_dot(const fem_csr* csr, const int32_t* ncol, const void* vals, fem_precision prec, const double* x,
              double* y, const double* w, double* part0, double* part1, const int32_t* fl, hipStream_t s) {
    const int32_t nn = csr->n_rows / 3;
    if (prec == FEM_FP64)
        hipLaunchKernelGGL((spmv_dot_kernel<double, ND>), dim3(kSpmvGrid), dim3(256), 0, s, nn, csr->row_ptr, ncol,
                           static_cast<const double*>(vals), x, y, w, part0, part1, fl);
    else
        hipLaunchKernelGGL((spmv_dot_kernel<float, ND>), dim3(kSpmvGrid), dim3(256), 0, s, nn, csr->row_ptr, ncol,
                           static_cast<const float*>(vals), x, y, w, part0, part1, fl);
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

extern "C" size_t fem_solver_workspace_bytes_method(int32_t n_rows, int64_t nnz, fem_krylov method) {
    if (n_rows < 0 || nnz < 0) return 0;
    CountAdapterS c;
    carve_solver(c, n_rows, nnz, (SolverWs*)nullptr);
    if (method == FEM_KRYLOV_GMRES || method == FEM_KRYLOV_FGMRES)
        carve_gmres(c, n_rows, method == FEM_KRYLOV_FGMRES, (GmresWs*)nullptr);
    return c.cnt.used + 256;
}

extern "C" size_t fem_solver_workspace_bytes(int32_t n_rows, int64_t nnz) {
    return fem_solver_workspace_bytes_method(n_rows, nnz, FEM_KRYLOV_BICGSTAB);
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

namespace {

// The Krylov iterations of fem_solve (amg NULL: Jacobi or block Jacobi by pc)
// and fem_solve_amg (M = one V-cycle of amg).
int krylov_solve(const char* who, const fem_csr* csr, const void* K_vals, fem_precision prec, fem_krylov method,
                 fem_precond pc, fem_amg* amg, const double* b, double* x, int32_t max_iter, double rtol,
                 int32_t* iters, double* rel_res, void* ws, size_t ws_bytes, void* stream) {
    if (int rc = check_csr(csr, K_vals, who)) return rc;
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED) return set_error(FEM_EINVAL, "%s: bad precision", who);
    if (!amg && pc != FEM_PC_JACOBI && pc != FEM_PC_BLOCK_JACOBI)
        return set_error(FEM_EINVAL, "%s: bad preconditioner", who);
    if (method != FEM_KRYLOV_BICGSTAB && method != FEM_KRYLOV_CG && method != FEM_KRYLOV_GMRES &&
        method != FEM_KRYLOV_FGMRES)
        return set_error(FEM_EINVAL, "%s: bad Krylov method", who);
    if (amg && amg_cycle_type(amg) == FEM_AMG_CYCLE_K && method != FEM_KRYLOV_FGMRES)
        return set_error(FEM_EINVAL, "%s: a K-cycle preconditioner varies between applications and needs the "
                                     "flexible method FEM_KRYLOV_FGMRES", who);
    if (max_iter < 0 || !(rtol >= 0.0)) return set_error(FEM_EINVAL, "%s: max_iter >= 0 and rtol >= 0", who);
    const int32_t n = csr->n_rows, nn = n / 3;
    if (iters) *iters = 0;
    if (rel_res) *rel_res = 0.0;
    if (n == 0) return FEM_OK;
    if (!b || !x) return set_error(FEM_EINVAL, "%s: b and x must not be NULL", who);
    if (csr->nnz < 0 || csr->nnz % 9) return set_error(FEM_EINVAL, "%s: nnz must be a multiple of 9", who);
    if (amg && !amg_matches(amg, csr))
        return set_error(FEM_EINVAL, "%s: the multigrid handle was built on another pattern", who);
    const size_t need = fem_solver_workspace_bytes_method(n, csr->nnz, method);
    if (!ws || ws_bytes < need)
        return set_error(FEM_ENOMEM, "%s: workspace of %zu bytes required, %zu given", who, need, ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    WsCarver c(ws, ws_bytes);
    SolverWs w;
    carve_solver(c, n, csr->nnz, &w);
    const unsigned nbl = (unsigned)(((int64_t)nn * kSpmvLanes + 255) / 256);
    const unsigned nbn = (unsigned)(((int64_t)nn + 255) / 256);
    const int block = pc == FEM_PC_BLOCK_JACOBI ? 1 : 0;
    hipLaunchKernelGGL(node_cols_kernel, dim3(nbl), dim3(256), 0, s, nn, csr->row_ptr, csr->col_idx, w.ncol);
    // with multigrid the fused update kernels write the first smoothing sweep
    // M_0 q into the cycle's finest iterate (mx) and the cycle writes M q
    const double* minv = w.minv;
    double* mx = nullptr;
    if (amg) {
        if (int rc = amg_update(amg, K_vals, prec, s)) return rc;
        minv = amg_smoother0(amg);
        mx = amg_level0_x(amg);
    } else if (prec == FEM_FP64) {
        hipLaunchKernelGGL(precond_kernel<double>, dim3(nbn), dim3(256), 0, s, nn, csr->row_ptr, w.ncol,
                           static_cast<const double*>(K_vals), block, w.minv);
    } else {
        hipLaunchKernelGGL(precond_kernel<float>, dim3(nbn), dim3(256), 0, s, nn, csr->row_ptr, w.ncol,
                           static_cast<const float*>(K_vals), block, w.minv);
    }
    hipLaunchKernelGGL(reset_flags, dim3(1), dim3(1), 0, s, w.fl);
    spmv_dot<0>(csr, w.ncol, K_vals, prec, x, w.t, nullptr, nullptr, nullptr, nullptr, s);
    if (method == FEM_KRYLOV_GMRES || method == FEM_KRYLOV_FGMRES) {
        const bool flex = method == FEM_KRYLOV_FGMRES;
        GmresWs g;
        carve_gmres(c, n, flex, &g);
        // M v: with multigrid the normalisation writes the first sweep M_0 v
        // into the cycle's finest iterate and the cycle writes M v to ph (to
        // z_j when flexible); with block Jacobi the normalisation writes M v
        // there itself
        const int32_t* cyc = w.fl + F_CYC;
        const int32_t* stp = w.fl + F_STOP;
        hipLaunchKernelGGL(gm_residual, dim3(kGrid), dim3(256), 0, s, (int64_t)n, b, w.t, g.V, w.part0, w.part1,
                           w.fl);
        hipLaunchKernelGGL(gm_start, dim3(1), dim3(256), 0, s, w.part0, w.part1, g.g, w.sc, w.fl, rtol, max_iter, 1);
        FEM_HIP_CHECK(hipGetLastError());
        int32_t flh[F_COUNT];
        double res = 0.0;
        auto read_back = [&]() -> hipError_t {
            hipError_t e = hipMemcpyAsync(flh, w.fl, sizeof(flh), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipMemcpyAsync(&res, w.sc + S_RES, sizeof(double), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            return e;
        };
        auto read_flags = [&]() -> hipError_t {  // within a cycle: the flags only
            hipError_t e = hipMemcpyAsync(flh, w.fl, sizeof(flh), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            return e;
        };
        FEM_HIP_CHECK(read_back());
        while (!flh[F_STOP]) {
            for (int j = 0; j < kGmresM; ++j) {
                double* vj = g.V + (int64_t)j * g.ldv;
                double* vn = g.V + (int64_t)(j + 1) * g.ldv;
                double* zj = flex ? g.Z + (int64_t)j * g.ldv : w.ph;
                hipLaunchKernelGGL(gm_normalize, dim3(kGrid), dim3(256), 0, s, nn, vj, minv, amg ? mx : zj, w.sc,
                                   cyc);
                if (amg) FEM_HIP_CHECK(amg_apply_cycle(amg, vj, zj, true, cyc, s));
                spmv_dot<0>(csr, w.ncol, K_vals, prec, zj, vn, nullptr, nullptr, nullptr, cyc, s);
                hipLaunchKernelGGL(gm_dots, dim3(kGrid), dim3(256), 0, s, (int64_t)n, j, g.V, g.ldv, vn, g.hpart, cyc);
                hipLaunchKernelGGL(gm_hreduce, dim3(j + 1), dim3(256), 0, s, g.hpart, j, g.H, cyc);
                hipLaunchKernelGGL(gm_update, dim3(kGrid), dim3(256), 0, s, (int64_t)n, j, g.V, g.ldv, g.H, vn,
                                   w.part0, cyc);
                hipLaunchKernelGGL(gm_finish, dim3(1), dim3(256), 0, s, w.part0, j, g.H, g.cs, g.sn, g.g, w.sc, w.fl,
                                   rtol, max_iter);
                // a multigrid step costs far more than a stream synchronisation:
                // stop launching once the cycle has ended
                if (amg) {
                    FEM_HIP_CHECK(hipGetLastError());
                    FEM_HIP_CHECK(read_flags());
                    if (flh[F_CYC]) break;
                }
            }
            // x += M (V y) (flexible: x += Z y); then the true residual of the restart
            hipLaunchKernelGGL(gm_solve_y, dim3(1), dim3(1), 0, s, g.H, g.g, g.y, w.fl);
            if (flex) {
                hipLaunchKernelGGL(gm_combine, dim3(kGrid), dim3(256), 0, s, (int64_t)n, g.Z, g.ldv, g.y, w.sh,
                                   w.fl);
            } else {
                hipLaunchKernelGGL(gm_combine, dim3(kGrid), dim3(256), 0, s, (int64_t)n, g.V, g.ldv, g.y, w.p,
                                   w.fl);
                if (amg)
                    FEM_HIP_CHECK(amg_apply_cycle(amg, w.p, w.sh, false, nullptr, s));
                else
                    hipLaunchKernelGGL(gm_apply_minv, dim3(kGrid), dim3(256), 0, s, nn, minv, w.p, w.sh);
            }
            hipLaunchKernelGGL(gm_addx, dim3(kGrid), dim3(256), 0, s, (int64_t)n, w.sh, x);
            spmv_dot<0>(csr, w.ncol, K_vals, prec, x, w.t, nullptr, nullptr, nullptr, stp, s);
            hipLaunchKernelGGL(gm_residual, dim3(kGrid), dim3(256), 0, s, (int64_t)n, b, w.t, g.V, w.part0, w.part1,
                               w.fl);
            hipLaunchKernelGGL(gm_start, dim3(1), dim3(256), 0, s, w.part0, w.part1, g.g, w.sc, w.fl, rtol, max_iter,
                               0);
            FEM_HIP_CHECK(hipGetLastError());
            FEM_HIP_CHECK(read_back());
        }
        if (iters) *iters = flh[F_ITER];
        if (rel_res) *rel_res = res;
        if (!(res <= rtol))
            return set_error(FEM_ENOCONV, "%s: relative residual %.3e after %d iterations (rtol %.3e)", who, res,
                             flh[F_ITER], rtol);
        return FEM_OK;
    }
    const bool cg = method == FEM_KRYLOV_CG;
    if (cg && amg) {
        // r = b - K x, mx = M_0 r; z (in s) = M r; p = z; (r, z)
        hipLaunchKernelGGL(cg_init, dim3(kGrid), dim3(256), 0, s, nn, b, w.t, minv, w.r, mx, w.p, w.part0, w.part1,
                           w.part2);
        FEM_HIP_CHECK(amg_apply_cycle(amg, w.r, w.s, true, w.fl, s));
        hipLaunchKernelGGL(cg_amg_start, dim3(kGrid), dim3(256), 0, s, (int64_t)n, w.s, w.r, w.p, w.part0, w.fl);
        hipLaunchKernelGGL(cg_fin_init, dim3(1), dim3(256), 0, s, w.part0, w.part1, w.part2, w.sc, w.fl, rtol,
                           max_iter);
    } else if (cg) {
        hipLaunchKernelGGL(cg_init, dim3(kGrid), dim3(256), 0, s, nn, b, w.t, w.minv, w.r, w.s, w.p, w.part0, w.part1,
                           w.part2);
        hipLaunchKernelGGL(cg_fin_init, dim3(1), dim3(256), 0, s, w.part0, w.part1, w.part2, w.sc, w.fl, rtol,
                           max_iter);
    } else {
        hipLaunchKernelGGL(init_kernel, dim3(kGrid), dim3(256), 0, s, (int64_t)n, b, w.t, w.r, w.rh, w.p, w.v,
                           w.part0, w.part1);
        hipLaunchKernelGGL(fin_init, dim3(1), dim3(256), 0, s, w.part0, w.part1, w.sc, w.fl, rtol, max_iter);
    }
    FEM_HIP_CHECK(hipGetLastError());
    int32_t fl[F_COUNT];
    double res = 0.0;
    auto read_back = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(fl, w.fl, sizeof(fl), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&res, w.sc + S_RES, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    };
    FEM_HIP_CHECK(read_back());
    while (!fl[F_STOP] && fl[F_ITER] < max_iter) {
        const int32_t chunk = std::min<int32_t>(amg ? kChunkAmg : kChunk, max_iter - fl[F_ITER]);
        for (int32_t k = 0; cg && k < chunk; ++k) {
            spmv_dot<1>(csr, w.ncol, K_vals, prec, w.p, w.v, w.p, w.part0, nullptr, w.fl, s);
            hipLaunchKernelGGL(cg_fin_alpha, dim3(1), dim3(256), 0, s, w.part0, w.sc, w.fl);
            hipLaunchKernelGGL(cg_update, dim3(kGrid), dim3(256), 0, s, nn, w.p, w.v, minv, x, w.r, amg ? mx : w.s,
                               w.part0, w.part1, w.sc, w.fl);
            if (amg) {
                FEM_HIP_CHECK(amg_apply_cycle(amg, w.r, w.s, true, w.fl, s));
                hipLaunchKernelGGL(dot_kernel, dim3(kGrid), dim3(256), 0, s, (int64_t)n, w.r, w.s, w.part0, w.fl);
            }
            hipLaunchKernelGGL(cg_fin_beta, dim3(1), dim3(256), 0, s, w.part0, w.part1, w.sc, w.fl, rtol, max_iter);
            hipLaunchKernelGGL(cg_update_p, dim3(kGrid), dim3(256), 0, s, (int64_t)n, w.s, w.p, w.sc, w.fl);
        }
        for (int32_t k = 0; !cg && k < chunk; ++k) {
            hipLaunchKernelGGL(update_p, dim3(kGrid), dim3(256), 0, s, nn, w.r, w.v, minv, w.p, amg ? mx : w.ph, w.sc,
                               w.fl);
            if (amg) FEM_HIP_CHECK(amg_apply_cycle(amg, w.p, w.ph, true, w.fl, s));
            spmv_dot<1>(csr, w.ncol, K_vals, prec, w.ph, w.v, w.rh, w.part0, nullptr, w.fl, s);
            hipLaunchKernelGGL(fin_alpha, dim3(1), dim3(256), 0, s, w.part0, w.sc, w.fl);
            hipLaunchKernelGGL(update_s, dim3(kGrid), dim3(256), 0, s, nn, w.r, w.v, minv, w.s, amg ? mx : w.sh, w.sc,
                               w.fl);
            if (amg) FEM_HIP_CHECK(amg_apply_cycle(amg, w.s, w.sh, true, w.fl, s));
            spmv_dot<2>(csr, w.ncol, K_vals, prec, w.sh, w.t, w.s, w.part0, w.part1, w.fl, s);
            hipLaunchKernelGGL(fin_omega, dim3(1), dim3(256), 0, s, w.part0, w.part1, w.sc, w.fl);
            hipLaunchKernelGGL(update_x, dim3(kGrid), dim3(256), 0, s, (int64_t)n, w.ph, w.sh, w.s, w.t, w.rh, x, w.r,
                               w.part0, w.part1, w.sc, w.fl);
            hipLaunchKernelGGL(fin_rho, dim3(1), dim3(256), 0, s, w.part0, w.part1, w.sc, w.fl, rtol, max_iter);
        }
        FEM_HIP_CHECK(hipGetLastError());
        FEM_HIP_CHECK(read_back());
    }
    if (iters) *iters = fl[F_ITER];
    if (rel_res) *rel_res = res;
    if (!(res <= rtol))
        return set_error(FEM_ENOCONV, "%s: relative residual %.3e after %d iterations (rtol %.3e)", who, res,
                         fl[F_ITER], rtol);
    return FEM_OK;
}

}  // namespace

extern "C" int fem_solve(const fem_csr* csr, const void* K_vals, fem_precision prec, fem_krylov method,
                         fem_precond pc, const double* b, double* x, int32_t max_iter, double rtol, int32_t* iters,
                         double* rel_res, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    return krylov_solve("fem_solve", csr, K_vals, prec, method, pc, nullptr, b, x, max_iter, rtol, iters, rel_res, ws,
                        ws_bytes, stream);
}

extern "C" int fem_solve_amg(const fem_csr* csr, const void* K_vals, fem_precision prec, fem_krylov method,
                             fem_amg* amg, const double* b, double* x, int32_t max_iter, double rtol, int32_t* iters,
                             double* rel_res, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!amg) return set_error(FEM_EINVAL, "fem_solve_amg: the multigrid handle must not be NULL");
    return krylov_solve("fem_solve_amg", csr, K_vals, prec, method, FEM_PC_AMG, amg, b, x, max_iter, rtol, iters,
                        rel_res, ws, ws_bytes, stream);
}
