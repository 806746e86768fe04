// vjp.hip -- parameter vector-Jacobian product g = lambda^T dR/dtheta for
// theta = (F, G, H, N, K, eps0, n), or (F, G, H, N, sig0, Q, b) with Voce
// hardening (Alg. 1 "Evaluate VJP", Eq. (main_grad)).
//
// R_Ia = sum_e sum_g w detJ0 P_aA dN_I/dX_A, P = F (P_L : T), and only the
// logarithmic stress T depends on theta, through the converged local update
// (F-bar: F is Fbar throughout, which does not depend on theta).
// Per Gauss point:
//   Lambda = sum_I lambda_I (x) grad N_I,  Tbar = P_L : sym(F^T Lambda),
//   thetabar_k = w detJ0 Tbar : dT/dtheta_k.
// dT/dtheta follows from differentiating the converged closest-point
// equations (App. D); here it is applied in reverse mode, in closed form:
//   u = Xi Tbar,  Xi = (E^-1 + dgamma dN/dT)^-1,  D = N.Xi.N + sigma_y',
//   thetabar = -dgamma u.N_theta
//              - (u.N / D) (-dgamma (Xi N).N_theta + phi_theta - sigma_y,theta).
// The local state is recomputed from d and hist_n (no tape is stored).
// Elastic Gauss points contribute exactly zero.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "fem_device.h"
#include "fem_internal.h"

namespace fem {
namespace {

struct VjpArgs {
    int32_t n_nodes, n_elems;
    const double* X;
    const int32_t* conn;
    const double* prm[FEM_NPARAM];
    uint32_t pe_mask, ps_mask;
    uint32_t model;          // FEM_MODEL_* flags
    const double* orient;    // material orientation(s), or null
    int32_t orient_pe;       // orient holds one rotation per element
    int32_t n_spec;
    const int64_t* elem_off;
    const double* d;
    const double* hist_n;
    const double* lam;
    double* g_elem;  // [7][n_elems]
    int32_t* diag;
    int64_t n_gp;
    int64_t n_tiles;
    int32_t xcd_remap;
    int32_t* fix_list;   // mixed precision: guard-band elements, recomputed in FP64
    int32_t* fix_count;
};

__device__ inline int spec_of_v(const int64_t* __restrict__ off, int n_spec, int64_t e) {
    int lo = 0, hi = n_spec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline Mat load_material_v(const VjpArgs& a, int64_t e) {
    int sp = 0;
    if (a.ps_mask) sp = spec_of_v(a.elem_off, a.n_spec, e);
    double v[FEM_NPARAM];
#pragma unroll
    for (int k = 0; k < FEM_NPARAM; ++k) {
        const int64_t idx = ((a.pe_mask >> k) & 1u) ? e : (((a.ps_mask >> k) & 1u) ? (int64_t)sp : 0);
        v[k] = a.prm[k][idx];
    }
    Mat m;
    m.E = v[0]; m.nu = v[1]; m.F = v[2]; m.G = v[3]; m.H = v[4]; m.L = v[5];
    m.M = v[6]; m.N = v[7]; m.K = v[8]; m.eps0 = v[9]; m.nexp = v[10];
    m.voce = 0;  // set by the kernel from its variant
    return m;
}

// compile-time variants (bit flags, as in the forward kernel)
constexpr int kVarOrientV = 1;
constexpr int kVarFbarV = 2;
constexpr int kVarVoceV = 4;

__device__ inline void tile_range_v(int64_t n_tiles, int remap, int64_t& first, int64_t& end, int64_t& step) {
    const int nb = gridDim.x, b = blockIdx.x;
    if (remap && (nb % 8) == 0 && nb >= 8) {
        const int x = b & 7, k = b >> 3, per = nb >> 3;
        const int64_t chunk = (n_tiles + 7) / 8;
        first = (int64_t)x * chunk + k;
        end = min((int64_t)(x + 1) * chunk, n_tiles);
        step = per;
    } else {
        first = b;
        end = n_tiles;
        step = nb;
    }
}

template <typename R>
struct GPv {
    R g[8][3];
    R detJ;
    R H[3][3];   // displacement gradient, F = I + H
    R Q[3][3];
    R mu[3];
    R eh[3];
};

// FBAR: the material sees Fbar = beta F (fbar_gradient); s.H becomes Fbar - I.
template <typename R, bool FBAR>
__device__ inline void kin_log_v(const double (*nd)[9], int gp, GPv<R>& s, double eps[6]) {
    kinematics_lds<R, 9>(nd, gp, s.g, s.detJ, s.H);
    if constexpr (FBAR) {
        R beta, cw, jm1;
        fbar_gradient<R>(s.detJ, s.H, beta, cw, jm1);
    }
    R M[3][3];
    cauchy_green_minus_identity<R>(s.H, M);
    eig_sym3<R>(M, s.mu, s.Q);
#pragma unroll
    for (int a = 0; a < 3; ++a) s.eh[a] = R(0.5) * m_log1p(s.mu[a]);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int i = mi(k), j = mj(k);
        R v = s.Q[i][0] * s.eh[0] * s.Q[j][0] + s.Q[i][1] * s.eh[1] * s.Q[j][1] + s.Q[i][2] * s.eh[2] * s.Q[j][2];
        eps[k] = (double)(mw<R>(k) * v);
    }
}

// The FP32 form is held to two waves per SIMD (a few registers spill; measured
// faster than one wave per SIMD without spills).
template <typename R, int BLOCK, bool FIXUP, int VAR>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(std::is_same<R, float>::value && !FIXUP ? 2 : 1)))
void vjp_kernel(const VjpArgs a) {
    constexpr int EPB = BLOCK / 8;
    constexpr bool FLAG = std::is_same<R, float>::value && !FIXUP;
    constexpr bool ORIENT = (VAR & kVarOrientV) != 0;
    __shared__ double sN[EPB][8][9];
    __shared__ double red[7][BLOCK + 1];
    __shared__ int sFlag[EPB];
    // per lane, across the local update (registers are the limit there): the
    // frame gradients g^ = Q^T grad N and H, Q
    __shared__ R sG[EPB][8][25];   // odd row lengths: the lanes spread over the LDS banks
    __shared__ R sHQ[EPB][8][19];
    const int tid = threadIdx.x;
    const int slot = tid >> 3, gp = tid & 7;
    int32_t cnt_fail = 0, cnt_j0 = 0;

    int64_t t0, t1, ts;
    int64_t n_work = a.n_elems;
    if constexpr (FIXUP) {
        n_work = *a.fix_count;
        t0 = blockIdx.x;
        t1 = (n_work + EPB - 1) / EPB;
        ts = gridDim.x;
    } else {
        tile_range_v(a.n_tiles, a.xcd_remap, t0, t1, ts);
    }
    for (int64_t tile = t0; tile < t1; tile += ts) {
        const int64_t e_raw = tile * EPB + slot;
        const bool valid = e_raw < n_work;
        int64_t e;
        if constexpr (FIXUP) e = a.fix_list[valid ? e_raw : 0];
        else e = valid ? e_raw : (int64_t)a.n_elems - 1;
        const int64_t q = e * 8 + gp;
        if (FLAG && gp == 0) sFlag[slot] = 0;
        int32_t node = a.conn[q];
        if ((uint32_t)node >= (uint32_t)a.n_nodes) node = 0;  // out-of-range id: stay in bounds
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sN[slot][gp][c] = a.X[3 * (int64_t)node + c];
            sN[slot][gp][3 + c] = a.d[3 * (int64_t)node + c];
            sN[slot][gp][6 + c] = a.lam[3 * (int64_t)node + c];
        }
        double hn[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) hn[k] = a.hist_n[k * a.n_gp + q];
        Mat mat = load_material_v(a, e);
        mat.voce = (VAR & kVarVoceV) ? 1 : 0;
        __syncthreads();

        GPv<R> s;
        double eps[6];
        kin_log_v<R, (VAR & kVarFbarV) != 0>(sN[slot], gp, s, eps);
#pragma unroll
        for (int I = 0; I < 8; ++I)
#pragma unroll
            for (int p = 0; p < 3; ++p)
                sG[slot][gp][3 * I + p] = s.g[I][0] * s.Q[0][p] + s.g[I][1] * s.Q[1][p] + s.g[I][2] * s.Q[2][p];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                sHQ[slot][gp][3 * i + j] = s.H[i][j];
                sHQ[slot][gp][9 + 3 * i + j] = s.Q[i][j];
            }
        asm volatile("" ::: "memory");  // the parked values are re-read, not kept in registers
        const int64_t oidx = a.orient_pe ? e : 0;
        if constexpr (ORIENT) {
            // local update and adjoint in the material frame
            double Th[3][3];
            load_rotation(a.orient, oidx, Th);
            rotate_sym<true>(Th, eps, kSqrt2);
            rotate_sym<true>(Th, hn, 1.0);
        }
        Modes md;
        hill_modes(mat, md);
        Local loc;
        local_update(eps, hn, mat, md, loc);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                s.H[i][j] = sHQ[slot][gp][3 * i + j];
                s.Q[i][j] = sHQ[slot][gp][9 + 3 * i + j];
            }
        if constexpr (FLAG) {
            // guard band: the element is recomputed in FP64 (fixup launch)
            if (valid && fabs(loc.ftr) < 2e-4 * loc.sy_n) sFlag[slot] = 1;
        }
        if (valid && !FIXUP) {
            cnt_fail += loc.converged ? 0 : 1;
            cnt_j0 += (s.detJ <= R(0)) ? 1 : 0;
        }
        double gbar[7] = {0, 0, 0, 0, 0, 0, 0};
        if (loc.plastic) {
            // Tbar = P_L : sym(F^T Lambda) in the eigenframe of C
            const R* gh = sG[slot][gp];  // g^_Iq at 3 I + q
            R Lh[3][3];  // Lambda^_aq = sum_I lambda_Ia g^_Iq
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    R v = R(0);
#pragma unroll
                    for (int I = 1; I < 8; ++I) v += (R)(sN[slot][I][6 + i] - sN[slot][0][6 + i]) * gh[3 * I + p];
                    Lh[i][p] = v;
                }
            R fh[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    fh[i][p] = s.Q[i][p] + (s.H[i][0] * s.Q[0][p] + s.H[i][1] * s.Q[1][p] + s.H[i][2] * s.Q[2][p]);
            R Tb[3][3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int r = p; r < 3; ++r) {
                    R x = R(0.5) * (fh[0][p] * Lh[0][r] + fh[1][p] * Lh[1][r] + fh[2][p] * Lh[2][r] +
                                    fh[0][r] * Lh[0][p] + fh[1][r] * Lh[1][p] + fh[2][r] * Lh[2][p]);
                    const R f1 = (p == r) ? R(0.5) / (R(1) + s.mu[p]) : dd1<R>(s.mu[p], s.mu[r], s.eh[p], s.eh[r]);
                    Tb[p][r] = Tb[r][p] = R(2) * f1 * x;
                }
            R tbm[6];
            frame_to_mandel<R>(s.Q, Tb, tbm);
            double tb[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) tb[k] = (double)tbm[k];
            if constexpr (ORIENT) {
                double Th[3][3];
                load_rotation(a.orient, oidx, Th);
                rotate_sym<true>(Th, tb, kSqrt2);
            }

            // ---- reverse-mode adjoint of the local update (double)
            const double lam = loc.lam, dg = loc.dgamma, phi = loc.phi, sv = loc.svar;
            const double om = 1.0 / (1.0 - lam * sv);
            double tmod[5];
            const double tbh = (tb[0] + tb[1] + tb[2]) * kInvSqrt3;
            tmod[0] = md.v1[0] * tb[0] + md.v1[1] * tb[1] + md.v1[2] * tb[2];
            tmod[1] = md.v2[0] * tb[0] + md.v2[1] * tb[1] + md.v2[2] * tb[2];
            tmod[2] = tb[3];
            tmod[3] = tb[4];
            tmod[4] = tb[5];
            double mT = 0.0;
#pragma unroll
            for (int i = 0; i < 5; ++i) mT += loc.mvec[i] * tmod[i];
            double u[5], xin[5], uN = 0.0;
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const double ai = md.mu2 / (1.0 + md.mu2 * lam * md.eta[i]);
                u[i] = ai * tmod[i] + lam * loc.mvec[i] * mT * om;
                xin[i] = loc.mvec[i] * om;
                uN += u[i] * loc.Nm[i];
            }
            const double uh = md.k3 * tbh;
            const double Dn = sv * om + loc.dsig;
            const double xN = sv * om;
            // Cartesian Mandel of u and Xi N
            double uc[6], xc[6];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                uc[k] = uh * kInvSqrt3 + u[0] * md.v1[k] + u[1] * md.v2[k];
                xc[k] = xin[0] * md.v1[k] + xin[1] * md.v2[k];
            }
            uc[3] = u[2]; uc[4] = u[3]; uc[5] = u[4];
            xc[3] = xin[2]; xc[4] = xin[3]; xc[5] = xin[4];
            const double* T = loc.T;
            // Hill parameters F, G, H, N: (H_theta T) and T.H_theta.T
            double hv[4][6] = {{0, T[1] - T[2], T[2] - T[1], 0, 0, 0},
                               {T[0] - T[2], 0, T[2] - T[0], 0, 0, 0},
                               {T[0] - T[1], T[1] - T[0], 0, 0, 0, 0},
                               {0, 0, 0, 0, 0, T[5]}};
            const double tht[4] = {(T[1] - T[2]) * (T[1] - T[2]), (T[0] - T[2]) * (T[0] - T[2]),
                                   (T[0] - T[1]) * (T[0] - T[1]), T[5] * T[5]};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double uh_ = 0.0, xh_ = 0.0;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    uh_ += uc[c] * hv[k][c];
                    xh_ += xc[c] * hv[k][c];
                }
                const double dphi = tht[k] / (2.0 * phi);
                const double uNt = uh_ / phi - uN * dphi / phi;
                const double xNt = xh_ / phi - xN * dphi / phi;
                gbar[k] = -dg * uNt - (uN / Dn) * (-dg * xNt + dphi);
            }
            // hardening parameters at alpha_{n+1}: Swift (K, eps0, n) or Voce (sig0, Q, b)
            const double alpha = loc.hist[6];
            double d0, d1, d2;
            if (mat.voce) {
                const double ex = exp(-mat.nexp * alpha);
                d0 = 1.0;
                d1 = 1.0 - ex;
                d2 = mat.eps0 * alpha * ex;
            } else {
                d0 = loc.sig / mat.K;
                d1 = loc.dsig;
                d2 = loc.sig * log(mat.eps0 + alpha);
            }
            gbar[4] = (uN / Dn) * d0;
            gbar[5] = (uN / Dn) * d1;
            gbar[6] = (uN / Dn) * d2;
            const double w = (double)s.detJ;
#pragma unroll
            for (int k = 0; k < 7; ++k) gbar[k] *= w;
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) red[k][tid] = gbar[k];
        __syncthreads();
        if (valid && gp < 7) {
            double sum = 0.0;
#pragma unroll
            for (int g2 = 0; g2 < 8; ++g2) sum += red[gp][slot * 8 + g2];
            a.g_elem[(int64_t)gp * a.n_elems + e] = sum;
        }
        if constexpr (FLAG) {
            if (valid && gp == 7 && sFlag[slot]) a.fix_list[atomicAdd(a.fix_count, 1)] = (int32_t)e;
        }
        __syncthreads();
    }
    if (a.diag && !FIXUP) {
        if (cnt_fail) atomicAdd(a.diag + 0, cnt_fail);
        if (cnt_j0) atomicAdd(a.diag + 1, cnt_j0);
    }
}

// g_uniform[s][k] = sum over the elements of specimen s of g_elem[k][e]; one
// workgroup per (s, k): thread t adds elements t, t + T, t + 2T, ... of the
// specimen into 8 chains (element t + mT into chain m mod 8), then a fixed
// tree (deterministic).
constexpr int kRedThreads = 1024;
__global__ __launch_bounds__(kRedThreads) void reduce_uniform(const double* __restrict__ g_elem, int64_t n_elems,
                                                              const int64_t* __restrict__ off,
                                                              double* __restrict__ g_uniform) {
    __shared__ double sh[kRedThreads];
    const int sidx = blockIdx.x / FEM_NGRAD, k = blockIdx.x % FEM_NGRAD;
    const int64_t b = off ? off[sidx] : 0, en = off ? off[sidx + 1] : n_elems;
    const double* __restrict__ gk = g_elem + (int64_t)k * n_elems;
    double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t e = b + threadIdx.x;
    for (; e + 7 * kRedThreads < en; e += 8 * kRedThreads) {
#pragma unroll
        for (int m = 0; m < 8; ++m) c[m] += gk[e + m * kRedThreads];
    }
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if (e + m * kRedThreads < en) c[m] += gk[e + m * kRedThreads];
    sh[threadIdx.x] = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
    __syncthreads();
    for (int o = kRedThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) g_uniform[(int64_t)sidx * FEM_NGRAD + k] = sh[0];
}

template <typename R, int BLOCK, bool FIXUP, int VAR>
hipError_t launch_vjp_one(const VjpArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((vjp_kernel<R, BLOCK, FIXUP, VAR>), dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

inline int variant_of_v(const VjpArgs& a) {
    return (a.orient ? kVarOrientV : 0) | ((a.model & FEM_MODEL_FBAR) ? kVarFbarV : 0) |
           ((a.model & FEM_MODEL_VOCE) ? kVarVoceV : 0);
}

// Variant 0 in every tuned workgroup size; the model variants with 64 threads.
template <typename R, bool FIXUP>
hipError_t launch_vjp_variant(const VjpArgs& a, int block, int grid, hipStream_t s) {
    switch (variant_of_v(a)) {
        case 0:
            if (FIXUP || block == 64) return launch_vjp_one<R, 64, FIXUP, 0>(a, grid, s);
            if (block == 256) return launch_vjp_one<R, 256, FIXUP, 0>(a, grid, s);
            return launch_vjp_one<R, 128, FIXUP, 0>(a, grid, s);
        case 1: return launch_vjp_one<R, 64, FIXUP, 1>(a, grid, s);
        case 2: return launch_vjp_one<R, 64, FIXUP, 2>(a, grid, s);
        case 3: return launch_vjp_one<R, 64, FIXUP, 3>(a, grid, s);
        case 4: return launch_vjp_one<R, 64, FIXUP, 4>(a, grid, s);
        case 5: return launch_vjp_one<R, 64, FIXUP, 5>(a, grid, s);
        case 6: return launch_vjp_one<R, 64, FIXUP, 6>(a, grid, s);
        default: return launch_vjp_one<R, 64, FIXUP, 7>(a, grid, s);
    }
}

template <typename R>
hipError_t launch_vjp(const VjpArgs& a, int block, int grid, hipStream_t s) {
    return launch_vjp_variant<R, false>(a, block, grid, s);
}

// FP64 recomputation of the guard-band elements of a mixed call
hipError_t launch_vjp_fixup(const VjpArgs& a, hipStream_t s) { return launch_vjp_variant<double, true>(a, 64, 1024, s); }

}  // namespace

hipError_t reduce_g_uniform(const double* g_elem, int64_t n_elems, const int64_t* off, int n_spec,
                            double* g_uniform, hipStream_t s) {
    hipLaunchKernelGGL(reduce_uniform, dim3(n_spec * FEM_NGRAD), dim3(kRedThreads), 0, s, g_elem, n_elems, off,
                       g_uniform);
    return hipGetLastError();
}

}  // namespace fem

using namespace fem;

// workspace: [g_elem when the caller passes none][fix list][fix count]
extern "C" size_t fem_vjp_workspace_bytes(int32_t n_elems, int32_t n_spec) {
    (void)n_spec;
    if (n_elems < 0) return 0;
    return sizeof(double) * (size_t)FEM_NGRAD * ((size_t)n_elems + 1) + sizeof(int32_t) * ((size_t)n_elems + 1) +
           1024;
}

extern "C" int fem_residual_vjp(const fem_mesh* mesh, const fem_batch* batch, const fem_params* params,
                                const double* d, const double* hist_n, const double* lam, fem_precision prec,
                                double* g_uniform, double* g_elem, int32_t* diag, void* ws, size_t ws_bytes,
                                void* stream) {
    clear_error();
    if (!mesh || !params) return set_error(FEM_EINVAL, "fem_residual_vjp: mesh and params must not be NULL");
    if (mesh->n_nodes < 0 || mesh->n_elems < 0) return set_error(FEM_EINVAL, "fem_residual_vjp: negative sizes");
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED)
        return set_error(FEM_EINVAL, "fem_residual_vjp: unknown precision %d", (int)prec);
    const int64_t ne = mesh->n_elems;
    if (ne > 0 && (!mesh->X || !mesh->conn || !d || !hist_n || !lam))
        return set_error(FEM_EINVAL, "fem_residual_vjp: X, conn, d, hist_n and lam must not be NULL");
    for (int k = 0; k < FEM_NPARAM; ++k)
        if (!params->p[k]) return set_error(FEM_EINVAL, "fem_residual_vjp: parameter %d is NULL", k);
    if (batch && (batch->n_spec < 1 || !batch->elem_off))
        return set_error(FEM_EINVAL, "fem_residual_vjp: invalid batch");
    if (params->per_spec_mask && !batch)
        return set_error(FEM_EINVAL, "fem_residual_vjp: per-specimen parameters need a batch");
    if (params->model & FEM_MODEL_BARLAT)
        return set_error(FEM_EINVAL, "fem_residual_vjp: the Barlat yield function is available in the forward call only");
    if (params->model & ~(uint32_t)(FEM_MODEL_VOCE | FEM_MODEL_FBAR))
        return set_error(FEM_EINVAL, "fem_residual_vjp: unknown model flags 0x%x", params->model);
    const int n_spec = batch ? batch->n_spec : 1;
    hipStream_t s = (hipStream_t)stream;
    const size_t need = fem_vjp_workspace_bytes(mesh->n_elems, n_spec);
    if (!ws || ws_bytes < need)
        return set_error(FEM_ENOMEM, "fem_residual_vjp: workspace of %zu bytes required", need);
    WsCarver cv(ws, ws_bytes);
    double* ge_ws = cv.take<double>((size_t)FEM_NGRAD * ((size_t)mesh->n_elems + 1));
    int32_t* fix_list = cv.take<int32_t>((size_t)mesh->n_elems + 1);
    int32_t* fix_count = cv.take<int32_t>(4);
    double* ge = g_elem ? g_elem : ge_ws;
    // diag, and the guard-band counter of a mixed call, start at zero
    FEM_HIP_CHECK(zero_counters(diag, 4, (ne > 0 && prec == FEM_FP32_MIXED) ? fix_count : nullptr, 1, s));
    if (ne > 0) {
        fem_launch cfg = launch_config(FEM_KERNEL_VJP, prec);
        if (params->model || params->orient) cfg.block = 64;  // model variants: 64-thread workgroups
        VjpArgs a;
        a.n_nodes = mesh->n_nodes;
        a.n_elems = mesh->n_elems;
        a.X = mesh->X;
        a.conn = mesh->conn;
        for (int k = 0; k < FEM_NPARAM; ++k) a.prm[k] = params->p[k];
        a.pe_mask = params->per_elem_mask;
        a.ps_mask = params->per_spec_mask & ~params->per_elem_mask;
        a.model = params->model;
        a.orient = params->orient;
        a.orient_pe = params->orient_per_elem ? 1 : 0;
        a.n_spec = n_spec;
        a.elem_off = batch ? batch->elem_off : nullptr;
        a.d = d;
        a.hist_n = hist_n;
        a.lam = lam;
        a.g_elem = ge;
        a.diag = diag;
        a.n_gp = 8 * ne;
        const int epb = cfg.block / 8;
        a.n_tiles = (ne + epb - 1) / epb;
        a.xcd_remap = cfg.xcd_remap;
        a.fix_list = fix_list;
        a.fix_count = fix_count;
        const int grid = persistent_grid(cfg, a.n_tiles);
        void* tk = timing_begin(s);
        hipError_t e = (prec == FEM_FP64) ? launch_vjp<double>(a, cfg.block, grid, s)
                                          : launch_vjp<float>(a, cfg.block, grid, s);
        timing_end(tk, FEM_KERNEL_VJP, s);
        if (e != hipSuccess) return set_error(FEM_EHIP, "vjp kernel launch failed: %s", hipGetErrorString(e));
        if (prec == FEM_FP32_MIXED) FEM_HIP_CHECK(launch_vjp_fixup(a, s));
    }
    if (g_uniform) {
        if (ne == 0) {
            FEM_HIP_CHECK(zero_bytes(g_uniform, sizeof(double) * FEM_NGRAD * n_spec, s));
        } else {
            hipLaunchKernelGGL(reduce_uniform, dim3(n_spec * FEM_NGRAD), dim3(kRedThreads), 0, s, ge, ne,
                               batch ? batch->elem_off : nullptr, g_uniform);
            FEM_HIP_CHECK(hipGetLastError());
        }
    }
    return FEM_OK;
}

// ---- fem_residual_vjp_noalloc: the same call with its workspace in a
// file-scope device array (no allocation by the library or the caller).
namespace {

constexpr size_t kVjpScratchBytes = (size_t)FEM_VJP_SCRATCH_MAX_BYTES;
// One copy per device the library runs on, resident until the process ends.
// Host code never passes this symbol itself: the device address of the
// current device's copy is taken once per device with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kVjpScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// device address of the current device's scratch array (nullptr on failure,
// with the error set)
void* scratch_address(int* status) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *status = set_error(FEM_EHIP, "fem_residual_vjp_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *status = set_error(FEM_EINVAL, "fem_residual_vjp_noalloc: device %d out of range", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *status = set_error(FEM_EHIP, "fem_residual_vjp_noalloc: hipGetSymbolAddress failed: %s",
                                hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int fem_residual_vjp_noalloc(const fem_mesh* mesh, const fem_batch* batch, const fem_params* params,
                                        const double* d, const double* hist_n, const double* lam,
                                        fem_precision prec, double* g_uniform, double* g_elem, int32_t* diag,
                                        void* stream) {
    clear_error();
    if (!mesh) return set_error(FEM_EINVAL, "fem_residual_vjp_noalloc: mesh must not be NULL");
    if (mesh->n_elems < 0) return set_error(FEM_EINVAL, "fem_residual_vjp_noalloc: negative sizes");
    const int n_spec = batch ? batch->n_spec : 1;
    const size_t need = fem_vjp_workspace_bytes(mesh->n_elems, n_spec);
    if (need > kVjpScratchBytes)
        return set_error(FEM_ENOMEM,
                         "fem_residual_vjp_noalloc: %d elements need %zu bytes of scratch, the maximum is %zu "
                         "(use fem_residual_vjp with a workspace)",
                         mesh->n_elems, need, kVjpScratchBytes);
    int status = FEM_OK;
    void* ptr = scratch_address(&status);
    if (!ptr) return status;
    return fem_residual_vjp(mesh, batch, params, d, hist_n, lam, prec, g_uniform, g_elem, diag, ptr,
                            kVjpScratchBytes, stream);
}
