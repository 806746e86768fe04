// adjoint.hip -- one load step of the time-history adjoint (Sec. 2.3,
// Eqs. (Lagrangian) ... (dR_u), Alg. 1) for the time-discrete problem in
// which the history h^n of every Gauss point is the local update
// H^n(u^n, h^{n-1}, theta) of the converged step.
//
// For cotangents lambda (of R^n, per node) and mu (of h^n, per Gauss point)
// the call returns
//   g    = lambda^T dR^n/dtheta + mu^T dH^n/dtheta         (per element, summed)
//   hbar = lambda^T dR^n/dh^{n-1} + mu^T dH^n/dh^{n-1}      (per Gauss point)
//   ubar = mu^T dH^n/du^n                                    (per node)
// The lambda part of the displacement cotangent is K^T lambda, applied with
// the assembled tangent (fem_csr_transpose) by the caller.
//
// Per Gauss point the local update is reversed in closed form in the common
// eigenbasis of isotropic elasticity and Hill-48 (hydrostatic + 5 modes), the
// reverse of the closest-point equations G(y; eps, h_n, theta) = 0 of
// App. D with y = (T, alpha, dgamma):
//   output cotangents  Tbar, ebar (of eps^p_{n+1}), abar (of alpha_{n+1}),
//   ybar = (Tbar + dgamma dN/dT ebar, abar, N . ebar),
//   w_dg = (N . Xi ybar_T - ybar_a - ybar_dg) / (N . Xi N + sigma_y'),
//   v    = Xi (ybar_T - N w_dg),  w_a = ybar_a + sigma_y' w_dg,
//   epsbar = v,  eps^p_n bar = ebar - v,  alpha_n bar = w_a,
//   thetabar = -dgamma (v - ebar) . N_theta - w_dg (phi_theta - sigma_y,theta),
// with Xi = (E^-1 + dgamma dN/dT)^-1 applied by Sherman-Morrison.  epsbar
// goes back to the nodes through eps = 1/2 ln C: Fbar = F (P_L : epsbar).
#include <hip/hip_runtime.h>

#include "fem_device.h"
#include "fem_internal.h"

namespace fem {
namespace {

constexpr int kVarOrientA = 1;
constexpr int kVarFbarA = 2;
constexpr int kVarVoceA = 4;
constexpr int kAdjBlock = 64;  // 8 elements per workgroup
constexpr int kAdjEpb = kAdjBlock / 8;

struct AdjArgs {
    int32_t n_nodes, n_elems;
    const double* X;
    const int32_t* conn;
    const double* prm[FEM_NPARAM];
    uint32_t pe_mask;
    const double* orient;
    int32_t orient_pe;
    const double* d;
    const double* hist_n;
    const double* lam;  // [3 n_nodes] or null
    const double* mu;   // [7][n_gp] or null
    double* g_elem;     // [7][n_elems]
    double* hbar;       // [7][n_gp] or null
    double* ue;         // [n_elems][24] or null
    int32_t* diag;
    int64_t n_gp;
};

__device__ inline Mat load_material_a(const AdjArgs& a, int64_t e, int voce) {
    double v[FEM_NPARAM];
#pragma unroll
    for (int k = 0; k < FEM_NPARAM; ++k) v[k] = a.prm[k][((a.pe_mask >> k) & 1u) ? e : 0];
    Mat m;
    m.E = v[0]; m.nu = v[1]; m.F = v[2]; m.G = v[3]; m.H = v[4]; m.L = v[5];
    m.M = v[6]; m.N = v[7]; m.K = v[8]; m.eps0 = v[9]; m.nexp = v[10];
    m.voce = voce;
    return m;
}

// modal coordinates (hydrostatic, 5 Hill modes) of a Cartesian Mandel vector
__device__ inline void to_modal(const Modes& md, const double x[6], double& xh, double xm[5]) {
    xh = (x[0] + x[1] + x[2]) * kInvSqrt3;
    xm[0] = md.v1[0] * x[0] + md.v1[1] * x[1] + md.v1[2] * x[2];
    xm[1] = md.v2[0] * x[0] + md.v2[1] * x[1] + md.v2[2] * x[2];
    xm[2] = x[3];
    xm[3] = x[4];
    xm[4] = x[5];
}

__device__ inline void from_modal(const Modes& md, double xh, const double xm[5], double x[6]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = xh * kInvSqrt3 + xm[0] * md.v1[k] + xm[1] * md.v2[k];
    x[3] = xm[2];
    x[4] = xm[3];
    x[5] = xm[4];
}

// v = Xi (yT - N wdg) for a plastic point (modal), returns wdg and w_a
__device__ inline void reverse_plastic(const Modes& md, const Local& loc, double yh, const double ym[5], double ya,
                                       double ydg, double& vh, double vm[5], double& wdg, double& wa) {
    const double lam = loc.lam, om = 1.0 / (1.0 - lam * loc.svar);
    double my = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) my += loc.mvec[i] * ym[i];
    wdg = (my * om - ya - ydg) / (loc.svar * om + loc.dsig);
    wa = ya + loc.dsig * wdg;
    double z[5], mz = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        z[i] = ym[i] - loc.Nm[i] * wdg;
        mz += loc.mvec[i] * z[i];
    }
    vh = md.k3 * yh;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double ai = md.mu2 / (1.0 + md.mu2 * lam * md.eta[i]);
        vm[i] = ai * z[i] + lam * loc.mvec[i] * mz * om;
    }
}

template <int VAR>
__global__ __launch_bounds__(kAdjBlock) void hadj_kernel(const AdjArgs a) {
    constexpr bool ORIENT = (VAR & kVarOrientA) != 0;
    constexpr bool FBAR = (VAR & kVarFbarA) != 0;
    constexpr int EPB = kAdjEpb;
    __shared__ double sN[EPB][8][9];   // X, d, lambda of the element's nodes
    __shared__ double sG[EPB][8][25];  // g^ = Q^T grad N per Gauss point (odd row length: no bank conflicts)
    __shared__ double red[24][kAdjBlock + 1];
    __shared__ double sQb[FBAR ? EPB : 1][24];
    const int tid = threadIdx.x, slot = tid >> 3, gp = tid & 7;
    const int64_t e_raw = (int64_t)blockIdx.x * EPB + slot;
    const bool valid = e_raw < a.n_elems;
    const int64_t e = valid ? e_raw : (int64_t)a.n_elems - 1;
    const int64_t q = e * 8 + gp;

    int32_t node = a.conn[q];
    if ((uint32_t)node >= (uint32_t)a.n_nodes) node = 0;  // out-of-range id: stay in bounds
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sN[slot][gp][c] = a.X[3 * (int64_t)node + c];
        sN[slot][gp][3 + c] = a.d[3 * (int64_t)node + c];
        sN[slot][gp][6 + c] = a.lam ? a.lam[3 * (int64_t)node + c] : 0.0;
    }
    double hn[7], mu[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        hn[k] = a.hist_n[k * a.n_gp + q];
        mu[k] = a.mu ? a.mu[k * a.n_gp + q] : 0.0;
    }
    const Mat mat = load_material_a(a, e, (VAR & kVarVoceA) ? 1 : 0);
    __syncthreads();

    // ---- kinematics (F-bar: Fbar = beta F), log strain
    double g[8][3], detJ, H[3][3];
    kinematics_lds<double, 9>(sN[slot], gp, g, detJ, H);
    double beta = 1.0, cw = 0.0, jm1 = 0.0;
    if constexpr (FBAR) fbar_gradient<double>(detJ, H, beta, cw, jm1);
    double M[3][3], Q[3][3], mu_c[3], eh[3];
    cauchy_green_minus_identity<double>(H, M);
    eig_sym3<double>(M, mu_c, Q);
#pragma unroll
    for (int p = 0; p < 3; ++p) eh[p] = 0.5 * log1p(mu_c[p]);
    double eps[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int i = mi(k), j = mj(k);
        eps[k] = mw<double>(k) * (Q[i][0] * eh[0] * Q[j][0] + Q[i][1] * eh[1] * Q[j][1] + Q[i][2] * eh[2] * Q[j][2]);
    }
#pragma unroll
    for (int I = 0; I < 8; ++I)
#pragma unroll
        for (int p = 0; p < 3; ++p) sG[slot][gp][3 * I + p] = g[I][0] * Q[0][p] + g[I][1] * Q[1][p] + g[I][2] * Q[2][p];
    double fh[3][3];  // Fbar Q
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int p = 0; p < 3; ++p) fh[i][p] = Q[i][p] + (H[i][0] * Q[0][p] + H[i][1] * Q[1][p] + H[i][2] * Q[2][p]);
    double f1[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int r = 0; r < 3; ++r) f1[p][r] = (p == r) ? 0.5 / (1.0 + mu_c[p]) : dd1<double>(mu_c[p], mu_c[r], eh[p], eh[r]);
    __syncthreads();

    // ---- local update (material frame with an orientation)
    const int64_t oidx = a.orient_pe ? e : 0;
    double Th[3][3];
    if constexpr (ORIENT) {
        load_rotation(a.orient, oidx, Th);
        rotate_sym<true>(Th, eps, kSqrt2);
        rotate_sym<true>(Th, hn, 1.0);
    }
    Modes md;
    hill_modes(mat, md);
    Local loc;
    local_update(eps, hn, mat, md, loc);

    // ---- output cotangents: Tbar = w detJ0 P_L : sym(Fbar^T Lambda) (Cartesian
    // Mandel), ebar (Mandel) and abar from mu
    double tb[6];
    {
        double Lh[3][3];  // Lambda Q
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                double v = 0.0;
#pragma unroll
                for (int I = 0; I < 8; ++I) v += sN[slot][I][6 + i] * sG[slot][gp][3 * I + p];
                Lh[i][p] = v;
            }
        double Tbh[3][3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = p; r < 3; ++r) {
                const double x = 0.5 * (fh[0][p] * Lh[0][r] + fh[1][p] * Lh[1][r] + fh[2][p] * Lh[2][r] +
                                        fh[0][r] * Lh[0][p] + fh[1][r] * Lh[1][p] + fh[2][r] * Lh[2][p]);
                Tbh[p][r] = Tbh[r][p] = 2.0 * f1[p][r] * x * detJ;
            }
        frame_to_mandel<double>(Q, Tbh, tb);
    }
    double eb[6] = {mu[0], mu[1], mu[2], mu[3] * kInvSqrt2, mu[4] * kInvSqrt2, mu[5] * kInvSqrt2};
    if constexpr (ORIENT) {
        rotate_sym<true>(Th, tb, kSqrt2);
        rotate_sym<true>(Th, eb, kSqrt2);
    }
    const double ab = mu[6];

    // ---- reverse of the local update (material frame)
    double th_bar[7] = {0, 0, 0, 0, 0, 0, 0};
    double v[6], vmu[6], hb_a;
    {
        double tbh_, tbm[5], ebh, ebm[5];
        to_modal(md, tb, tbh_, tbm);
        to_modal(md, eb, ebh, ebm);
        double vh, vm[5], vh_mu, vm_mu[5];
        if (loc.plastic) {
            const double dg = loc.dgamma, phi = loc.phi;
            double NE = 0.0;
#pragma unroll
            for (int i = 0; i < 5; ++i) NE += loc.Nm[i] * ebm[i];
            double yT[5], yTmu[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const double dNe = (md.eta[i] * ebm[i] - loc.Nm[i] * NE) / phi;  // dN/dT ebar
                yTmu[i] = dg * dNe;
                yT[i] = tbm[i] + yTmu[i];
            }
            double wdg, wa, wdg_mu, wa_mu;
            reverse_plastic(md, loc, tbh_, yT, ab, NE, vh, vm, wdg, wa);
            reverse_plastic(md, loc, 0.0, yTmu, ab, NE, vh_mu, vm_mu, wdg_mu, wa_mu);
            hb_a = wa;
            // thetabar: Hill parameters F, G, H, N (material frame T)
            double vmE[6], vme[5];
#pragma unroll
            for (int i = 0; i < 5; ++i) vme[i] = vm[i] - ebm[i];
            from_modal(md, vh - ebh, vme, vmE);  // v - ebar, Cartesian material Mandel
            double vN = 0.0;
#pragma unroll
            for (int i = 0; i < 5; ++i) vN += vme[i] * loc.Nm[i];
            const double* T = loc.T;
            const double hv[4][6] = {{0, T[1] - T[2], T[2] - T[1], 0, 0, 0},
                                     {T[0] - T[2], 0, T[2] - T[0], 0, 0, 0},
                                     {T[0] - T[1], T[1] - T[0], 0, 0, 0, 0},
                                     {0, 0, 0, 0, 0, T[5]}};
            const double tht[4] = {(T[1] - T[2]) * (T[1] - T[2]), (T[0] - T[2]) * (T[0] - T[2]),
                                   (T[0] - T[1]) * (T[0] - T[1]), T[5] * T[5]};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double vh_ = 0.0;
#pragma unroll
                for (int c = 0; c < 6; ++c) vh_ += vmE[c] * hv[k][c];
                const double dphi = tht[k] / (2.0 * phi);
                const double vNt = vh_ / phi - vN * dphi / phi;
                th_bar[k] = -dg * vNt - wdg * dphi;
            }
            // hardening parameters at alpha_{n+1}
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
            th_bar[4] = wdg * d0;
            th_bar[5] = wdg * d1;
            th_bar[6] = wdg * d2;
        } else {
            // elastic: T = E : (eps - eps^p_n), history unchanged
            vh = md.k3 * tbh_;
#pragma unroll
            for (int i = 0; i < 5; ++i) vm[i] = md.mu2 * tbm[i];
            vh_mu = 0.0;
#pragma unroll
            for (int i = 0; i < 5; ++i) vm_mu[i] = 0.0;
            hb_a = ab;
        }
        from_modal(md, vh, vm, v);
        from_modal(md, vh_mu, vm_mu, vmu);
    }
    if constexpr (ORIENT) {
        rotate_sym<false>(Th, v, kSqrt2);
        rotate_sym<false>(Th, vmu, kSqrt2);
    }
    if (valid && !loc.converged) atomicAdd(a.diag + 0, 1);
    if (valid && detJ <= 0.0) atomicAdd(a.diag + 1, 1);
    // history cotangent: eps^p_n bar (stored components) = mu - W v, alpha_n bar = w_a
    if (valid && a.hbar) {
#pragma unroll
        for (int k = 0; k < 6; ++k) a.hbar[k * a.n_gp + q] = mu[k] - mw<double>(k) * v[k];
        a.hbar[6 * a.n_gp + q] = hb_a;
    }
    // thetabar summed over the element's Gauss points
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k][tid] = th_bar[k];
    __syncthreads();
    if (valid && gp < 7) {
        double s = 0.0;
#pragma unroll
        for (int g2 = 0; g2 < 8; ++g2) s += red[gp][slot * 8 + g2];
        a.g_elem[(int64_t)gp * a.n_elems + e] = s;
    }
    __syncthreads();
    if (!a.ue) return;  // uniform over the launch

    // ---- displacement cotangent of the history part: Xf = Fbar (P_L : epsbar_mu)
    double Xh[3][3];
    {
        double Yh[3][3];
        mandel_to_frame<double>(Q, vmu, Yh);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int p = 0; p < 3; ++p)
                Xh[i][p] = fh[i][0] * 2.0 * f1[0][p] * Yh[0][p] + fh[i][1] * 2.0 * f1[1][p] * Yh[1][p] +
                           fh[i][2] * 2.0 * f1[2][p] * Yh[2][p];
    }
    double sg = 0.0;
    if constexpr (FBAR) {
        // F-bar: ubar_Jb = sum_g beta (Xf grad N_J)_b + sg (qbar_Jb - q_g,Jb),
        // sg = (Xf : Fbar) / 3, q_g = beta g^ (f^/c)^T, qbar = sum_g cw q_g
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int p = 0; p < 3; ++p) sg += Xh[i][p] * fh[i][p];
        sg *= 1.0 / 3.0;
#pragma unroll
        for (int J = 0; J < 8; ++J)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double x = 0.0;
#pragma unroll
                for (int s2 = 0; s2 < 3; ++s2) x += sG[slot][gp][3 * J + s2] * fh[b][s2] / (1.0 + mu_c[s2]);
                red[3 * J + b][tid] = cw * beta * x;
            }
        __syncthreads();
        if (gp < 8) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
#pragma unroll
                for (int g2 = 0; g2 < 8; ++g2) s += red[3 * gp + b][slot * 8 + g2];
                sQb[slot][3 * gp + b] = s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int J = 0; J < 8; ++J)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double x = Xh[b][0] * sG[slot][gp][3 * J] + Xh[b][1] * sG[slot][gp][3 * J + 1] +
                       Xh[b][2] * sG[slot][gp][3 * J + 2];
            if constexpr (FBAR) {
                double qg = 0.0;
#pragma unroll
                for (int s2 = 0; s2 < 3; ++s2) qg += sG[slot][gp][3 * J + s2] * fh[b][s2] / (1.0 + mu_c[s2]);
                x = beta * x - sg * beta * qg;
            }
            red[3 * J + b][tid] = x;
        }
    __syncthreads();
    const double S = FBAR ? sum8(sg) : 0.0;
    if (valid) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
#pragma unroll
            for (int g2 = 0; g2 < 8; ++g2) s += red[3 * gp + b][slot * 8 + g2];
            if constexpr (FBAR) s += S * sQb[slot][3 * gp + b];
            a.ue[e * 24 + 3 * gp + b] = s;
        }
    }
}

template <int VAR>
hipError_t launch_hadj(const AdjArgs& a, hipStream_t s) {
    const unsigned nb = (unsigned)((a.n_elems + kAdjEpb - 1) / kAdjEpb);
    hipLaunchKernelGGL((hadj_kernel<VAR>), dim3(nb), dim3(kAdjBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_hadj_variant(const AdjArgs& a, int var, hipStream_t s) {
    switch (var) {
        case 0: return launch_hadj<0>(a, s);
        case 1: return launch_hadj<1>(a, s);
        case 2: return launch_hadj<2>(a, s);
        case 3: return launch_hadj<3>(a, s);
        case 4: return launch_hadj<4>(a, s);
        case 5: return launch_hadj<5>(a, s);
        case 6: return launch_hadj<6>(a, s);
        default: return launch_hadj<7>(a, s);
    }
}

}  // namespace
}  // namespace fem

using namespace fem;

extern "C" size_t fem_history_adjoint_workspace_bytes(int32_t n_nodes, int32_t n_elems) {
    (void)n_nodes;
    if (n_elems < 0) return 0;
    return sizeof(double) * ((size_t)FEM_NGRAD + 24) * ((size_t)n_elems + 1) + 1024;
}

extern "C" int fem_history_adjoint(const fem_mesh* mesh, const fem_csr* csr, const fem_params* params,
                                   const double* d, const double* hist_n, const double* lam, const double* mu,
                                   double* g_uniform, double* g_elem, double* hbar, double* ubar, int32_t* diag,
                                   void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!mesh || !params) return set_error(FEM_EINVAL, "fem_history_adjoint: mesh and params must not be NULL");
    if (mesh->n_nodes < 0 || mesh->n_elems < 0) return set_error(FEM_EINVAL, "fem_history_adjoint: negative sizes");
    const int64_t ne = mesh->n_elems;
    if (ne > 0 && (!mesh->X || !mesh->conn || !d || !hist_n))
        return set_error(FEM_EINVAL, "fem_history_adjoint: X, conn, d and hist_n must not be NULL");
    for (int k = 0; k < FEM_NPARAM; ++k)
        if (!params->p[k]) return set_error(FEM_EINVAL, "fem_history_adjoint: parameter %d is NULL", k);
    if (params->per_spec_mask) return set_error(FEM_EINVAL, "fem_history_adjoint: per-specimen parameters unsupported");
    if (params->model & FEM_MODEL_BARLAT)
        return set_error(FEM_EINVAL, "fem_history_adjoint: the Barlat yield function is available in the forward call only");
    if (params->model & ~(uint32_t)(FEM_MODEL_VOCE | FEM_MODEL_FBAR))
        return set_error(FEM_EINVAL, "fem_history_adjoint: unknown model flags 0x%x", params->model);
    if (ubar && mesh->n_nodes > 0 && (!csr || !csr->node_elem_ptr || !csr->node_elem))
        return set_error(FEM_EINVAL, "fem_history_adjoint: ubar needs the node incidence of the CSR pattern");
    const size_t need = fem_history_adjoint_workspace_bytes(mesh->n_nodes, mesh->n_elems);
    if (!ws || ws_bytes < need)
        return set_error(FEM_ENOMEM, "fem_history_adjoint: workspace of %zu bytes required, %zu given", need, ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    WsCarver cv(ws, ws_bytes);
    double* ge_ws = cv.take<double>((size_t)FEM_NGRAD * ((size_t)ne + 1));
    double* ue = cv.take<double>((size_t)24 * ((size_t)ne + 1));
    double* ge = g_elem ? g_elem : ge_ws;
    FEM_HIP_CHECK(zero_counters(diag, 4, nullptr, 0, s));
    if (ne > 0) {
        AdjArgs a;
        a.n_nodes = mesh->n_nodes;
        a.n_elems = mesh->n_elems;
        a.X = mesh->X;
        a.conn = mesh->conn;
        for (int k = 0; k < FEM_NPARAM; ++k) a.prm[k] = params->p[k];
        a.pe_mask = params->per_elem_mask;
        a.orient = params->orient;
        a.orient_pe = params->orient_per_elem ? 1 : 0;
        a.d = d;
        a.hist_n = hist_n;
        a.lam = lam;
        a.mu = mu;
        a.g_elem = ge;
        a.hbar = hbar;
        a.ue = ubar ? ue : nullptr;
        a.diag = diag;
        a.n_gp = 8 * ne;
        const int var = (params->orient ? kVarOrientA : 0) | ((params->model & FEM_MODEL_FBAR) ? kVarFbarA : 0) |
                        ((params->model & FEM_MODEL_VOCE) ? kVarVoceA : 0);
        if (!diag) {
            // the kernel counts into diag unconditionally: use the workspace tail
            a.diag = reinterpret_cast<int32_t*>(cv.take<int32_t>(4));
            FEM_HIP_CHECK(zero_counters(a.diag, 4, nullptr, 0, s));
        }
        FEM_HIP_CHECK(launch_hadj_variant(a, var, s));
    }
    if (g_uniform) {
        if (ne == 0) FEM_HIP_CHECK(zero_bytes(g_uniform, sizeof(double) * FEM_NGRAD, s));
        else FEM_HIP_CHECK(reduce_g_uniform(ge, ne, nullptr, 1, g_uniform, s));
    }
    if (ubar && mesh->n_nodes > 0) {
        if (ne == 0) FEM_HIP_CHECK(zero_bytes(ubar, sizeof(double) * 3 * (size_t)mesh->n_nodes, s));
        else FEM_HIP_CHECK(gather_node_vectors(mesh->n_nodes, csr->node_elem_ptr, csr->node_elem, ue, ubar, s));
    }
    return FEM_OK;
}
