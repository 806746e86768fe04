// barlat.h -- Barlat Yld2004-18p yield function (Eq. Phi_barlat, App. A) and
// its closest-point return map (App. B line search, App. C Alg. C2) for one
// Gauss point, FP64, in the material frame.
//
// phi(T) = [1/4 sum_ij |s'_i - s''_j|^m]^(1/m), s'_i, s''_j the principal
// values of s' = C' : P : T and s'' = C'' : P : T (P the deviatoric
// projector).  Flow N = dphi/dT and dN/dT come from the principal-value
// derivatives lifted to tensors (spectral gradient and Hessian with divided
// differences; coincident values take their limit).  Unlike Hill-48, the
// closest-point equations have no closed-form reduction: a Newton iteration
// on (T, dgamma) (alpha = alpha_n + dgamma) solves the symmetric bordered
// system [[E^-1 + dgamma dN/dT, N], [N^T, -sigma_y']] by a 6x6 Cholesky
// factorisation, damped by the line search of App. B.
#pragma once

#include "fem_device.h"

namespace fem {

// 18 coefficients c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55 c'66, the same nine
// for c'', and the exponent m; mi = m - 2 when m is an integer in [2, 64]
// (the published fits use m = 8), else -1
struct BarlatCoef {
    double c[2][9];
    double m;
    int mi;
};

__device__ inline void load_barlat(const double* __restrict__ p, BarlatCoef& b) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        b.c[0][k] = p[k];
        b.c[1][k] = p[9 + k];
    }
    b.m = p[18];
    b.mi = (b.m >= 2.0 && b.m <= 64.0 && b.m == floor(b.m)) ? (int)b.m - 2 : -1;
}

// |d|^(m-2): by repeated squaring for an integer exponent (the same for every
// lane, so the branch is uniform), else pow; 1 at d = 0 for m = 2
__device__ inline double abs_pow_m2(double ad, const BarlatCoef& b) {
    if (b.mi >= 0) {
        double r = 1.0, x = ad;
        for (int k = b.mi; k; k >>= 1) {
            if (k & 1) r *= x;
            x *= x;
        }
        return r;
    }
    return pow(ad, b.m - 2.0);
}

// s = C : P : t as a symmetric 3x3 (t Mandel)
__device__ inline void barlat_apply(const double* c, const double t[6], double S[3][3]) {
    const double tr = (t[0] + t[1] + t[2]) * (1.0 / 3.0);
    const double s0 = t[0] - tr, s1 = t[1] - tr, s2 = t[2] - tr;
    S[0][0] = -c[0] * s1 - c[1] * s2;
    S[1][1] = -c[2] * s0 - c[3] * s2;
    S[2][2] = -c[4] * s0 - c[5] * s1;
    S[1][2] = S[2][1] = c[6] * t[3] * kInvSqrt2;
    S[0][2] = S[2][0] = c[7] * t[4] * kInvSqrt2;
    S[0][1] = S[1][0] = c[8] * t[5] * kInvSqrt2;
}

// Mandel vector of (C : P)^T : X for a symmetric X = Mandel x
__device__ inline void barlat_apply_T(const double* c, const double x[6], double out[6]) {
    // C^T x (normal block transposed, shear diagonal), then the deviator
    const double y0 = -c[2] * x[1] - c[4] * x[2];
    const double y1 = -c[0] * x[0] - c[5] * x[2];
    const double y2 = -c[1] * x[0] - c[3] * x[1];
    const double tr = (y0 + y1 + y2) * (1.0 / 3.0);
    out[0] = y0 - tr;
    out[1] = y1 - tr;
    out[2] = y2 - tr;
    out[3] = c[6] * x[3];
    out[4] = c[7] * x[4];
    out[5] = c[8] * x[5];
}

// Principal values of both transformed deviators, their eigenvectors, and the
// gradient g / Hessian h of phi with respect to lam = (s'_1..3, s''_1..3).
struct BarlatState {
    double lam[6];
    double P[2][3][3];  // eigenvectors (columns)
    double g[6];
    double phi;
};

// Symmetric 3x3 eigen-decomposition started from an orthonormal basis Q
// (columns) close to the eigenvectors: cyclic Jacobi on Q^T S Q, which is
// nearly diagonal, then Q <- Q Q'.  Between Newton iterates and line-search
// trials the transformed deviators turn little, so one or two sweeps replace
// the four to six of a start from the identity.
__device__ inline void eig_sym3_from(const double S[3][3], double mu[3], double Q[3][3]) {
    double W[3][3], B[3][3], Qs[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) W[i][q] = S[i][0] * Q[0][q] + S[i][1] * Q[1][q] + S[i][2] * Q[2][q];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = p; q < 3; ++q) {
            const double v = Q[0][p] * W[0][q] + Q[1][p] * W[1][q] + Q[2][p] * W[2][q];
            B[p][q] = v;
            B[q][p] = v;
        }
    eig_sym3<double>(B, mu, Qs);
    double Qn[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Qn[i][j] = Q[i][0] * Qs[0][j] + Q[i][1] * Qs[1][j] + Q[i][2] * Qs[2][j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[i][j] = Qn[i][j];
}

// warm: st.P holds eigenvectors of nearby deviators to start from
__device__ inline double barlat_principal(const BarlatCoef& b, const double t[6], BarlatState& st,
                                          bool warm = false) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        double S[3][3], mu[3];
        barlat_apply(b.c[a], t, S);
        if (warm) eig_sym3_from(S, mu, st.P[a]);
        else eig_sym3<double>(S, mu, st.P[a]);
        st.lam[3 * a] = mu[0];
        st.lam[3 * a + 1] = mu[1];
        st.lam[3 * a + 2] = mu[2];
    }
    double Phi = 0.0, dPhi[6] = {0, 0, 0, 0, 0, 0};
    const double m = b.m;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double d = st.lam[i] - st.lam[3 + j], ad = fabs(d);
            const double p2 = abs_pow_m2(ad, b);  // |d|^(m-2)
            Phi += 0.25 * p2 * ad * ad;
            const double t1 = 0.25 * m * d * p2;
            dPhi[i] += t1;
            dPhi[3 + j] -= t1;
        }
    st.phi = exp(log(Phi) / m);
    const double f = st.phi / (m * Phi);
#pragma unroll
    for (int a = 0; a < 6; ++a) st.g[a] = f * dPhi[a];
    return st.phi;
}

// Hessian of phi in lam (6x6), from the principal values held in st
__device__ inline void barlat_hessian(const BarlatCoef& b, const BarlatState& st, double h[6][6]) {
    const double m = b.m;
    double Phi = 0.0, dPhi[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int c = 0; c < 6; ++c) h[a][c] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double d = st.lam[i] - st.lam[3 + j], ad = fabs(d);
            const double p2 = abs_pow_m2(ad, b);
            Phi += 0.25 * p2 * ad * ad;
            const double t1 = 0.25 * m * d * p2, t2 = 0.25 * m * (m - 1.0) * p2;
            dPhi[i] += t1;
            dPhi[3 + j] -= t1;
            h[i][i] += t2;
            h[3 + j][3 + j] += t2;
            h[i][3 + j] -= t2;
            h[3 + j][i] -= t2;
        }
    const double f = st.phi / (m * Phi), c2 = (1.0 / m - 1.0) / Phi;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int c = 0; c < 6; ++c) h[a][c] = f * (h[a][c] + c2 * dPhi[a] * dPhi[c]);
}

// Mandel vector of P diag(v) P^T + (off-diagonal X in the eigenbasis)
__device__ inline void from_eigenbasis(const double P[3][3], const double Xh[3][3], double out[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int i = mi(k), j = mj(k);
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) s += P[i][p] * Xh[p][q] * P[j][q];
        out[k] = mw<double>(k) * s;
    }
}

// N = dphi/dt (Mandel)
__device__ inline void barlat_flow(const BarlatCoef& b, const BarlatState& st, double N[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) N[k] = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        double D[3][3] = {{st.g[3 * a], 0, 0}, {0, st.g[3 * a + 1], 0}, {0, 0, st.g[3 * a + 2]}};
        double n[6], o[6];
        from_eigenbasis(st.P[a], D, n);
        barlat_apply_T(b.c[a], n, o);
#pragma unroll
        for (int k = 0; k < 6; ++k) N[k] += o[k];
    }
}

// dN/dt (Mandel 6x6), column by column: for a direction e_K, ds = L e_K in
// each eigenbasis, dlam = diagonal, dg = h dlam, the spectral derivative
// P (diag(dg) + theta o offdiag(P^T ds P)) P^T, mapped back by L^T.
__device__ inline void barlat_dflow(const BarlatCoef& b, const BarlatState& st, double dN[6][6]) {
    double h[6][6];
    barlat_hessian(b, st, h);
    double th[2][3][3];  // divided differences of g within each block
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const double* l = st.lam + 3 * a;
        const double scale = fabs(l[0]) + fabs(l[1]) + fabs(l[2]) + 1e-300;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double v = 0.0;
                if (i != k) {
                    if (fabs(l[i] - l[k]) > 1e-9 * scale) v = (st.g[3 * a + i] - st.g[3 * a + k]) / (l[i] - l[k]);
                    else v = h[3 * a + i][3 * a + i] - h[3 * a + i][3 * a + k];
                }
                th[a][i][k] = v;
            }
    }
    for (int K = 0; K < 6; ++K) {
        double e[6] = {0, 0, 0, 0, 0, 0};
        e[K] = 1.0;
        double Dh[2][3][3], dl[6];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            double S[3][3];
            barlat_apply(b.c[a], e, S);
            // P^T S P
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) s += st.P[a][i][p] * S[i][j] * st.P[a][j][q];
                    Dh[a][p][q] = s;
                }
            dl[3 * a] = Dh[a][0][0];
            dl[3 * a + 1] = Dh[a][1][1];
            dl[3 * a + 2] = Dh[a][2][2];
        }
        double col[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            double X[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    if (i == k) {
                        double s = 0.0;
#pragma unroll
                        for (int c = 0; c < 6; ++c) s += h[3 * a + i][c] * dl[c];
                        X[i][i] = s;
                    } else {
                        X[i][k] = th[a][i][k] * Dh[a][i][k];
                    }
                }
            double n[6], o[6];
            from_eigenbasis(st.P[a], X, n);
            barlat_apply_T(b.c[a], n, o);
#pragma unroll
            for (int k = 0; k < 6; ++k) col[k] += o[k];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) dN[k][K] = col[k];
    }
}

// Cholesky factor (lower) of a symmetric positive definite 6x6, in place
__device__ inline void chol6(double A[6][6]) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double s = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= A[j][k] * A[j][k];
        const double d = sqrt(s);
        A[j][j] = d;
        const double id = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double x = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) x -= A[i][k] * A[j][k];
            A[i][j] = x * id;
        }
    }
}

__device__ inline void chol6_solve(const double L[6][6], double x[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * x[k];
        x[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = x[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
}

// Result of the Barlat local update (material frame); the algorithmic
// tangent goes to the caller's array cep[21] (upper triangle, row by row)
struct LocalB {
    double T[6];
    double hist[7];
    double ftr, sy_n;
    int plastic, converged;
};

// E^-1 x for isotropic elasticity (Mandel)
__device__ inline void elastic_compliance(const Modes& h, const double x[6], double y[6]) {
    const double hm = (x[0] + x[1] + x[2]) * (1.0 / 3.0);
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = (k < 3 ? (x[k] - hm) : x[k]) / h.mu2;
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] += hm / h.k3;  // (3 kappa)^-1 on the spherical part
}

// E : x for isotropic elasticity (Mandel)
__device__ inline void elastic_stiffness(const Modes& h, const double x[6], double y[6]) {
    const double tr = x[0] + x[1] + x[2];
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = h.mu2 * x[k] + (k < 3 ? h.lam * tr : 0.0);
}

// Residual of the reduced closest-point equations at (T, dg), alpha = alpha_n + dg:
//   G1 = E^-1 (T - t_tr) + dg N(T)  (strain),  G3 = phi(T) - sigma_y(alpha_n + dg),
// and the merit of Eq. (merit), psi = 1/2 G^T G with the stress rows
// T - t_tr + dg E : N = E : G1 and the yield row G3 (both in stress units).
__device__ inline double barlat_residual(const BarlatCoef& b, const Mat& m, const Modes& md, const double t_tr[6],
                                         double alpha_n, const double T[6], double dg, double G[7],
                                         BarlatState& st, double& dsig) {
    barlat_principal(b, T, st, true);  // st.P: eigenvectors at a nearby stress
    double N[6], dT[6], c[6];
    barlat_flow(b, st, N);
#pragma unroll
    for (int k = 0; k < 6; ++k) dT[k] = T[k] - t_tr[k];
    elastic_compliance(md, dT, c);
#pragma unroll
    for (int k = 0; k < 6; ++k) G[k] = c[k] + dg * N[k];
    double Eg[6];
    elastic_stiffness(md, G, Eg);
    double psi = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) psi += Eg[k] * Eg[k];
    const double sy = hardening(m, alpha_n + dg, dsig);
    G[6] = st.phi - sy;
    psi += G[6] * G[6];
    return 0.5 * psi;
}

__device__ inline void local_update_barlat(const double eps[6], const double* hist_n, const Mat& m, const Modes& md,
                                           const BarlatCoef& b, LocalB& o, double* __restrict__ cep) {
    double ee[6];
    ee[0] = eps[0] - hist_n[0];
    ee[1] = eps[1] - hist_n[1];
    ee[2] = eps[2] - hist_n[2];
    ee[3] = eps[3] - kSqrt2 * hist_n[3];
    ee[4] = eps[4] - kSqrt2 * hist_n[4];
    ee[5] = eps[5] - kSqrt2 * hist_n[5];
    const double tr = ee[0] + ee[1] + ee[2];
    double t_tr[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) t_tr[i] = md.mu2 * ee[i] + (i < 3 ? md.lam * tr : 0.0);
    const double alpha_n = hist_n[6];
    double dsig_n;
    o.sy_n = hardening(m, alpha_n, dsig_n);
    BarlatState st;
    const double phi_tr = barlat_principal(b, t_tr, st);
    o.ftr = phi_tr - o.sy_n;
    if (!(o.ftr > 0.0)) {
        o.plastic = 0;
        o.converged = 1;
#pragma unroll
        for (int i = 0; i < 6; ++i) o.T[i] = t_tr[i];
#pragma unroll
        for (int i = 0; i < 7; ++i) o.hist[i] = hist_n[i];
        int c = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) cep[c++] = ((i < 3 && j < 3) ? md.lam : 0.0) + ((i == j) ? md.mu2 : 0.0);
        return;
    }
    o.plastic = 1;
    // start on the current yield surface: phi is homogeneous of degree one, so
    // T0 = t_tr sigma_y(alpha_n) / phi(t_tr), and dgamma0 from the flow rule
    // projected on N(T0) (the root is unique, the start only saves iterations)
    double T[6], dg, G[7], dsig;
    {
        const double r = o.sy_n / phi_tr;
        double N0[6], c[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) T[i] = r * t_tr[i];
        barlat_principal(b, T, st, true);  // T0 is a multiple of t_tr: the same eigenvectors
        barlat_flow(b, st, N0);
        elastic_compliance(md, t_tr, c);
        double nc = 0.0, nn = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            nc += N0[i] * c[i];
            nn += N0[i] * N0[i];
        }
        dg = (1.0 - r) * nc / nn;
        if (!(dg > 0.0)) dg = 0.0;
    }
    double psi = barlat_residual(b, m, md, t_tr, alpha_n, T, dg, G, st, dsig);
    double prev = __builtin_inf();
    int conv = 0;
    for (int it = 0; it < 60; ++it) {
        // scaled residual: stress rows E : G1 over mu, the yield row over
        // sigma_y(alpha_n); converged at 1e-14, or at the rounding floor (a
        // step below 1e-9 that does not halve it; the floor grows with the
        // stress, so no fixed level detects it)
        double gn = 0.0;
        {
            double Eg[6];
            elastic_stiffness(md, G, Eg);
#pragma unroll
            for (int k = 0; k < 6; ++k) gn = fmax(gn, fabs(Eg[k]) * (2.0 / md.mu2));
        }
        gn = fmax(gn, fabs(G[6]) / o.sy_n);
        if (!(gn == gn)) break;
        if (gn <= 1e-14 || (gn <= 1e-9 && gn >= 0.5 * prev)) {
            conv = 1;
            break;
        }
        prev = gn;
        // Newton step of the bordered system
        double N[6], A[6][6];
        barlat_flow(b, st, N);
        barlat_dflow(b, st, A);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
#pragma unroll
            for (int j = 0; j < 6; ++j) A[i][j] *= dg;
        }
        // + E^-1
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double e[6] = {0, 0, 0, 0, 0, 0}, c[6];
            e[j] = 1.0;
            elastic_compliance(md, e, c);
#pragma unroll
            for (int i = 0; i < 6; ++i) A[i][j] += c[i];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j) {
                const double s = 0.5 * (A[i][j] + A[j][i]);
                A[i][j] = A[j][i] = s;
            }
        chol6(A);
        double u[6], w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            u[k] = G[k];
            w[k] = N[k];
        }
        chol6_solve(A, u);  // A^-1 G1
        chol6_solve(A, w);  // A^-1 N
        double NAu = 0.0, NAw = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            NAu += N[k] * u[k];
            NAw += N[k] * w[k];
        }
        const double ddg = (G[6] - NAu) / (NAw + dsig);
        double dT[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) dT[k] = -u[k] - w[k] * ddg;
        // line search of App. B on the merit of Eq. (merit)
        double Tt[6], Gt[7], dsg_t;
        BarlatState stt = st;  // trial states start their eigen-solves from the current one
#pragma unroll
        for (int k = 0; k < 6; ++k) Tt[k] = T[k] + dT[k];
        double psi1 = barlat_residual(b, m, md, t_tr, alpha_n, Tt, dg + ddg, Gt, stt, dsg_t);
        double zeta = 1.0;
        if (!(psi1 < (1.0 - 2.0 * 1e-4) * psi)) {
            double zj = psi / (psi + psi1);
            if (!(zj == zj)) zj = 0.1;
            for (int j = 0; j <= 20; ++j) {
#pragma unroll
                for (int k = 0; k < 6; ++k) Tt[k] = T[k] + zj * dT[k];
                const double psij = barlat_residual(b, m, md, t_tr, alpha_n, Tt, dg + zj * ddg, Gt, stt, dsg_t);
                double zn = fmax(0.1 * zj, psi / (psi + psij));
#pragma unroll
                for (int k = 0; k < 6; ++k) Tt[k] = T[k] + zn * dT[k];
                psi1 = barlat_residual(b, m, md, t_tr, alpha_n, Tt, dg + zn * ddg, Gt, stt, dsg_t);
                zeta = zn;
                if (psi1 < (1.0 - 2.0 * 1e-4 * zn) * psi) break;
                zj = zn;
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) T[k] += zeta * dT[k];
        dg += zeta * ddg;
        psi = barlat_residual(b, m, md, t_tr, alpha_n, T, dg, G, st, dsig);
    }
    o.converged = conv;
    // recovery and algorithmic tangent at the converged state
    double N[6], A[6][6];
    barlat_flow(b, st, N);
    barlat_dflow(b, st, A);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) A[i][j] *= dg;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double e[6] = {0, 0, 0, 0, 0, 0}, c[6];
        e[j] = 1.0;
        elastic_compliance(md, e, c);
#pragma unroll
        for (int i = 0; i < 6; ++i) A[i][j] += c[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            const double s = 0.5 * (A[i][j] + A[j][i]);
            A[i][j] = A[j][i] = s;
        }
    chol6(A);
    // Xi = A^-1 column by column, Xi N
    double XN[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) XN[k] = N[k];
    chol6_solve(A, XN);
    double NXN = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) NXN += N[k] * XN[k];
    const double den = 1.0 / (NXN + dsig);
    // column j of Xi, entries i <= j of Cep (symmetric)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double x[6] = {0, 0, 0, 0, 0, 0};
        x[j] = 1.0;
        chol6_solve(A, x);
#pragma unroll
        for (int i = 0; i <= j; ++i) cep[i * 6 - (i * (i - 1)) / 2 + (j - i)] = x[i] - XN[i] * XN[j] * den;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) o.T[k] = T[k];
    // eps^p_{n+1} = eps^p_n + dg N (tensor components), alpha_{n+1} = alpha_n + dg
#pragma unroll
    for (int k = 0; k < 6; ++k) o.hist[k] = hist_n[k] + dg * N[k] / mw<double>(k);
    o.hist[6] = alpha_n + dg;
}

}  // namespace fem
