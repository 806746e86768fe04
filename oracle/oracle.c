/*
 * oracle.c -- plain FP64 CPU reference of the finite-strain Hill-48 hex8 path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the HIP library; the product
 * never links it.  It shares no code, header, table or helper with the HIP
 * path.  Written for clarity, not speed: every step follows the paper's
 * formulation in its own order and notation.
 *
 * Paper passages followed (JAX-FEM-ANISO, arXiv 2606.17390):
 *   Sec. 2.2.2(a) geometric preprocessor, Eq. (c_decomp): eps = 1/2 ln C
 *   Sec. 2.2.2(b) additive split and linear log-space elasticity, Eq. (T)
 *   Eq. (Phi_hill) and App. A: Hill-48 effective stress phi = sqrt(T:H:T)
 *   Eqs. (ep_evol), (KT): associative flow, Kuhn-Tucker conditions
 *   Sec. 2.2.3 Eqs. (Tr_stress) ... (local_solver): elastic predictor and
 *       closest-point projection with unknowns y = [T, alpha, dgamma]
 *   App. B Eqs. (merit) ... (alpha_safeguard): line search (beta, eta)
 *   App. C Alg. C1 / C2: global stress update and local return mapping
 *   App. D: implicit differentiation of the converged local update
 *   Sec. 2.2.2(c), Eqs. (proj_lagrange), (pk_stress): S = P_L:T, P = F S
 *   Sec. 2.2.4: hex8 residual R^e_I = int P . grad N_I dV, K^e = dR^e/dd^e
 *   App. E Alg. E1: CSR assembly, Dirichlet rows set to identity
 *   Sec. 2.3 Eq. (main_grad), Alg. 1: the VJP term lambda^T dR/dtheta
 *
 *   Eq. (Hard): Voce hardening (model option); App. A: orientation of the
 *       Hill tensor; Sec. 2.2.4: F-bar deformation gradient (model option)
 *   Eq. (Phi_barlat), App. A: Barlat Yld2004-18p yield function (model
 *       option), phi from the principal values of two transformed deviators
 *
 * Readings where the paper is silent or inconsistent (listed in the design
 * notes): Swift hardening sigma_y = K (eps0+alpha)^n by default, Voce as
 * sigma_y = sig0 + Q (1 - exp(-b alpha)) in uniaxial-stress units; the Hill
 * function is written with F,G,H,L,M,N so that it reduces to von Mises at
 * F=G=H=1/2, L=M=N=3/2, with W = 1 in alpha_{n+1} = alpha_n + W dgamma;
 * isotropic elasticity; eps = sum 1/2 ln(c_a) N_a (x) N_a with c_a the
 * eigenvalues of C; F-bar as R^e_I = int P(Fbar) . grad N_I dV with K^e its
 * exact derivative (not symmetric).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { P_E, P_NU, P_F, P_G, P_H, P_L, P_M, P_N, P_K, P_EPS0, P_NEXP };

static const double SQRT2 = 1.41421356237309504880168872420969808;

/* local Newton constants: App. B gives the two line-search constants; the
 * paper fixes no tolerance and no iteration limit for the element runs.  The
 * limit is generous: with the merit of Eq. (merit) an extreme increment
 * (stretches 3 and 0.2 in one step) needs about 130 damped iterations. */
static const double LS_BETA = 1e-4; /* App. B, Goldstein constant */
static const double LS_ETA = 0.1;   /* App. B, step safeguard     */
enum { KMAX = 500, JMAX = 20 };
static const double LOCAL_TOL = 1e-14;

/* Mandel index pairs: (11, 22, 33, 23, 13, 12) */
static const int MI[6] = {0, 1, 2, 1, 0, 0};
static const int MJ[6] = {0, 1, 2, 2, 2, 1};

/* ------------------------------------------------------------------ */
/* small tensor helpers                                                */
/* ------------------------------------------------------------------ */

static void sym_to_mandel(const double M[9], double v[6]) {
    for (int k = 0; k < 6; ++k) {
        double c = (k < 3) ? 1.0 : SQRT2;
        v[k] = c * M[3 * MI[k] + MJ[k]];
    }
}

static void mandel_to_sym(const double v[6], double M[9]) {
    for (int k = 0; k < 6; ++k) {
        double c = (k < 3) ? 1.0 : 1.0 / SQRT2;
        M[3 * MI[k] + MJ[k]] = c * v[k];
        M[3 * MJ[k] + MI[k]] = c * v[k];
    }
}

/* R = Q^T M Q */
static void rot_to_frame(const double Q[9], const double M[9], double R[9]) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) s += Q[3 * i + a] * M[3 * i + j] * Q[3 * j + b];
            R[3 * a + b] = s;
        }
}

/* M = Q R Q^T */
static void rot_from_frame(const double Q[9], const double R[9], double M[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) s += Q[3 * i + a] * R[3 * a + b] * Q[3 * j + b];
            M[3 * i + j] = s;
        }
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static double det3(const double A[9]) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void inv3(const double A[9], double B[9]) {
    double d = det3(A);
    B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

/* Solve A x = b (n x n, row-major) by Gaussian elimination with partial
 * pivoting.  A and b are overwritten; the solution is returned in b. */
static int solve_dense(int n, double *A, double *b) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) {
                best = fabs(A[i * n + k]);
                p = i;
            }
        if (best == 0.0) return 1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[p * n + j];
                A[p * n + j] = t;
            }
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
        b[i] = s / A[i * n + i];
    }
    return 0;
}

/* Inverse of an n x n matrix, column by column through solve_dense. */
static int invert_dense(int n, const double *A, double *Ainv) {
    double W[64], e[8];
    for (int c = 0; c < n; ++c) {
        memcpy(W, A, sizeof(double) * n * n);
        for (int i = 0; i < n; ++i) e[i] = (i == c) ? 1.0 : 0.0;
        if (solve_dense(n, W, e)) return 1;
        for (int i = 0; i < n; ++i) Ainv[i * n + c] = e[i];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* symmetric eigen-decomposition: cyclic Jacobi to machine precision    */
/* ------------------------------------------------------------------ */

void oracle_eig_sym3(const double Ain[9], double w[3], double Q[9]) {
    double A[9];
    memcpy(A, Ain, sizeof A);
    for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = fabs(A[1]) + fabs(A[2]) + fabs(A[5]);
        if (off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                double app = A[3 * p + p], aqq = A[3 * q + q];
                /* an off-diagonal entry below the rounding of both diagonal
                 * entries is set to zero */
                if (sweep > 3 && fabs(app) + 100.0 * fabs(apq) == fabs(app) &&
                    fabs(aqq) + 100.0 * fabs(apq) == fabs(aqq)) {
                    A[3 * p + q] = A[3 * q + p] = 0.0;
                    continue;
                }
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = c * akp - s * akq;
                    A[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = c * apk - s * aqk;
                    A[3 * q + k] = s * apk + c * aqk;
                }
                A[3 * p + q] = A[3 * q + p] = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double qkp = Q[3 * k + p], qkq = Q[3 * k + q];
                    Q[3 * k + p] = c * qkp - s * qkq;
                    Q[3 * k + q] = s * qkp + c * qkq;
                }
            }
    }
    w[0] = A[0];
    w[1] = A[4];
    w[2] = A[8];
}

/* ------------------------------------------------------------------ */
/* divided differences of f(c) = 1/2 ln c, written in mu = c - 1        */
/* ------------------------------------------------------------------ */

/* f1(x, y) = (f(x) - f(y)) / (x - y), f1(x, x) = f'(x) = 1/(2x). */
static double dd1(double mx, double my) {
    double x = 1.0 + mx, y = 1.0 + my;
    if (mx == my) return 0.5 / x;
    double z = (mx - my) / (x + y);
    return atanh(z) / (z * (x + y));
}

/* f2(x, y, z): second divided difference.  For a small spread it is the
 * Taylor series of the divided difference about the mean m,
 * f[x0,x1,x2] = sum_j f^(j+2)(m)/(j+2)! h_j(x - m),  h_j complete
 * homogeneous symmetric polynomials, f^(k)(m)/k! = (-1)^(k-1) / (2 k m^k). */
static double dd2(double m1, double m2, double m3) {
    double v[3] = {m1, m2, m3};
    for (int i = 0; i < 2; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (v[j] < v[i]) {
                double t = v[i];
                v[i] = v[j];
                v[j] = t;
            }
    double mean_mu = (v[0] + v[1] + v[2]) / 3.0;
    double m = 1.0 + mean_mu;
    if (v[2] - v[0] < 1e-3 * m) {
        double dl[3] = {v[0] - mean_mu, v[1] - mean_mu, v[2] - mean_mu};
        double p[9], h[9];
        for (int k = 1; k <= 8; ++k) p[k] = pow(dl[0], k) + pow(dl[1], k) + pow(dl[2], k);
        h[0] = 1.0;
        for (int j = 1; j <= 8; ++j) {
            double s = 0.0;
            for (int i = 1; i <= j; ++i) s += p[i] * h[j - i];
            h[j] = s / j;
        }
        double sum = 0.0;
        for (int j = 0; j <= 8; ++j) {
            int k = j + 2;
            double ck = ((k - 1) % 2 == 0 ? 1.0 : -1.0) / (2.0 * k * pow(m, k));
            sum += ck * h[j];
        }
        return sum;
    }
    return (dd1(v[0], v[1]) - dd1(v[1], v[2])) / (v[0] - v[2]);
}

/* ------------------------------------------------------------------ */
/* material: elasticity, Hill-48, Swift                                */
/* ------------------------------------------------------------------ */

static void elastic_mandel(const double prm[11], double Em[36]) {
    double E = prm[P_E], nu = prm[P_NU];
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    memset(Em, 0, 36 * sizeof(double));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Em[6 * i + j] = lam;
    for (int i = 0; i < 6; ++i) Em[6 * i + i] += 2.0 * mu;
}

/* phi^2 = F(T22-T33)^2 + G(T33-T11)^2 + H(T11-T22)^2 + 2L T23^2 + 2M T13^2 + 2N T12^2
 *       = t . Hm . t  with t the Mandel vector of T. */
static void hill_mandel(const double prm[11], double Hm[36]) {
    double F = prm[P_F], G = prm[P_G], H = prm[P_H];
    memset(Hm, 0, 36 * sizeof(double));
    Hm[0] = G + H;
    Hm[7] = F + H;
    Hm[14] = F + G;
    Hm[1] = Hm[6] = -H;
    Hm[2] = Hm[12] = -G;
    Hm[8] = Hm[13] = -F;
    Hm[21] = prm[P_L];
    Hm[28] = prm[P_M];
    Hm[35] = prm[P_N];
}

static double hill_phi(const double Hm[36], const double t[6]) {
    double s = 0.0;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) s += t[i] * Hm[6 * i + j] * t[j];
    return sqrt(s);
}

/* Hardening law and its derivative: Swift sigma_y = K (eps0 + alpha)^n, or
 * (voce != 0) Voce sigma_y = sig0 + Q (1 - exp(-b alpha)) of Eq. (Hard) with
 * (sig0, Q, b) in the slots of (K, eps0, n). */
static double hardening(const double prm[11], int voce, double alpha, double *dsig) {
    if (voce) {
        double ex = exp(-prm[P_NEXP] * alpha);
        if (dsig) *dsig = prm[P_EPS0] * prm[P_NEXP] * ex;
        return prm[P_K] + prm[P_EPS0] * (1.0 - ex);
    }
    double base = prm[P_EPS0] + alpha;
    double s = prm[P_K] * pow(base, prm[P_NEXP]);
    if (dsig) *dsig = prm[P_NEXP] * s / base;
    return s;
}

/* Mandel 6x6 <-> fourth-order tensor with both minor symmetries
 * (T[27a+9b+3c+d]); Mandel weights 1 on normal and sqrt2 on shear slots. */
static void mandel_to_4th(const double Mm[36], double T4[81]) {
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            double v = Mm[6 * I + J] / ((I < 3 ? 1.0 : SQRT2) * (J < 3 ? 1.0 : SQRT2));
            int a = MI[I], b = MJ[I], c = MI[J], d = MJ[J];
            T4[27 * a + 9 * b + 3 * c + d] = v;
            T4[27 * b + 9 * a + 3 * c + d] = v;
            T4[27 * a + 9 * b + 3 * d + c] = v;
            T4[27 * b + 9 * a + 3 * d + c] = v;
        }
}

static void fourth_to_mandel(const double T4[81], double Mm[36]) {
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J)
            Mm[6 * I + J] = (I < 3 ? 1.0 : SQRT2) * (J < 3 ? 1.0 : SQRT2) *
                            T4[27 * MI[I] + 9 * MJ[I] + 3 * MI[J] + MJ[J]];
}

/* App. A: H_global = Theta Theta : H_local : Theta^T Theta^T, i.e.
 * H_ijkl = sum Theta_ia Theta_jb Theta_kc Theta_ld H_abcd (in place, Mandel). */
static void rotate_hill(const double *Theta, double Hm[36]) {
    if (!Theta) return;
    double L4[81], G4[81];
    mandel_to_4th(Hm, L4);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double v = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            for (int c = 0; c < 3; ++c)
                                for (int d = 0; d < 3; ++d)
                                    v += Theta[3 * i + a] * Theta[3 * j + b] * Theta[3 * k + c] *
                                         Theta[3 * l + d] * L4[27 * a + 9 * b + 3 * c + d];
                    G4[27 * i + 9 * j + 3 * k + l] = v;
                }
    fourth_to_mandel(G4, Hm);
}

/* ------------------------------------------------------------------ */
/* Barlat Yld2004-18p, Eq. (Phi_barlat) and App. A                      */
/* ------------------------------------------------------------------ */

/* coefficients c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55 c'66, the same for
 * c'', and the exponent m (set by oracle_set_barlat; read-only during calls) */
static double g_barlat[19];

void oracle_set_barlat(const double coef[19]) { memcpy(g_barlat, coef, sizeof g_barlat); }

/* L = C : P (Mandel; C and P are block diagonal, so their Voigt and Mandel
 * matrices coincide): s' = L' t, s'' = L'' t for the Mandel stress t. */
static void barlat_transform(const double *c9, double L[36]) {
    double C[36] = {0}, P[36] = {0};
    C[1] = -c9[0];
    C[2] = -c9[1];
    C[6] = -c9[2];
    C[8] = -c9[3];
    C[12] = -c9[4];
    C[13] = -c9[5];
    C[21] = c9[6];
    C[28] = c9[7];
    C[35] = c9[8];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P[6 * i + j] = (i == j ? 2.0 : -1.0) / 3.0;
    for (int i = 3; i < 6; ++i) P[6 * i + i] = 1.0;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double v = 0.0;
            for (int k = 0; k < 6; ++k) v += C[6 * i + k] * P[6 * k + j];
            L[6 * i + j] = v;
        }
}

/* phi and, optionally, its gradient g[6] and Hessian h[36] with respect to the
 * principal values lam = (s'_1..3, s''_1..3):
 *   Phi = 1/4 sum_ij |s'_i - s''_j|^m,  phi = Phi^(1/m) */
static double barlat_principal(const double lam[6], double m, double *g, double *h) {
    double Phi = 0.0, dPhi[6] = {0}, d2Phi[36] = {0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double d = lam[i] - lam[3 + j], ad = fabs(d);
            Phi += 0.25 * pow(ad, m);
            double t1 = 0.25 * m * d * pow(ad, m - 2.0);       /* d/dlam'_i of |d|^m / 4 */
            double t2 = 0.25 * m * (m - 1.0) * pow(ad, m - 2.0); /* second derivative */
            dPhi[i] += t1;
            dPhi[3 + j] -= t1;
            d2Phi[6 * i + i] += t2;
            d2Phi[6 * (3 + j) + 3 + j] += t2;
            d2Phi[6 * i + 3 + j] -= t2;
            d2Phi[6 * (3 + j) + i] -= t2;
        }
    double phi = pow(Phi, 1.0 / m);
    if (g)
        for (int a = 0; a < 6; ++a) g[a] = phi / (m * Phi) * dPhi[a];
    if (h)
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b)
                h[6 * a + b] = phi / (m * Phi) * (d2Phi[6 * a + b] + (1.0 / m - 1.0) * dPhi[a] * dPhi[b] / Phi);
    return phi;
}

/* Gradient (tensor) of a spectral function with principal derivatives g over
 * the eigen-basis Q (columns): sum_i g_i q_i (x) q_i, as a Mandel vector. */
static void spectral_gradient(const double Q[9], const double g[3], double out[6]) {
    double M[9] = {0}, D[9] = {0};
    for (int i = 0; i < 3; ++i) D[4 * i] = g[i];
    rot_from_frame(Q, D, M);
    sym_to_mandel(M, out);
}

/* Mandel 6x6 of the derivative of sum_i g_i q_i (x) q_i (the eigenvalues of
 * the first argument A, basis QA) with respect to the second argument B
 * (basis QB, eigenvalues lb), where g depends on the principal values:
 *   d/dB = sum_ik dg_i/dlb_k (q_k . dB q_k) P_i  [+ for A = B: sum_{i!=k}
 *   theta_ik P_i dB P_k, theta_ik = (g_i - g_k)/(l_i - l_k), or dg_i/dl_i -
 *   dg_i/dl_k where the two values coincide] */
static void spectral_block(const double QA[9], const double QB[9], const double la[3], const double ga[3],
                           const double hab[9], int same, double out[36]) {
    for (int K = 0; K < 6; ++K) {
        double e[6] = {0}, dB[9], dBh[9], R[9] = {0}, Rh[9] = {0}, v[6];
        e[K] = 1.0;
        mandel_to_sym(e, dB);
        rot_to_frame(QB, dB, dBh); /* dBh_kk = q_k . dB q_k */
        for (int i = 0; i < 3; ++i) {
            double x = 0.0;
            for (int k = 0; k < 3; ++k) x += hab[3 * i + k] * dBh[4 * k];
            Rh[4 * i] = x;
        }
        if (same) {
            double scale = fabs(la[0]) + fabs(la[1]) + fabs(la[2]) + 1e-300;
            for (int i = 0; i < 3; ++i)
                for (int k = 0; k < 3; ++k) {
                    if (i == k) continue;
                    double th;
                    if (fabs(la[i] - la[k]) > 1e-9 * scale) th = (ga[i] - ga[k]) / (la[i] - la[k]);
                    else th = hab[3 * i + i] - hab[3 * i + k];
                    Rh[3 * i + k] += th * dBh[3 * i + k];
                }
        }
        memcpy(R, Rh, sizeof R);
        double Rg[9];
        rot_from_frame(QA, R, Rg);
        sym_to_mandel(Rg, v);
        for (int I = 0; I < 6; ++I) out[6 * I + K] = v[I];
    }
}

/* Barlat phi(t), N = dphi/dt and dN/dt (Mandel), with L1 = L', L2 = L'' */
static double barlat_eval(const double L1[36], const double L2[36], double m, const double t[6], double *N,
                          double *dNdT) {
    double s1[6], s2[6], S1[9], S2[9], Q1[9], Q2[9], lam[6];
    for (int i = 0; i < 6; ++i) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < 6; ++j) {
            a += L1[6 * i + j] * t[j];
            b += L2[6 * i + j] * t[j];
        }
        s1[i] = a;
        s2[i] = b;
    }
    mandel_to_sym(s1, S1);
    mandel_to_sym(s2, S2);
    oracle_eig_sym3(S1, lam, Q1);
    oracle_eig_sym3(S2, lam + 3, Q2);
    double g[6], h[36];
    double phi = barlat_principal(lam, m, g, h);
    if (N) {
        double n1[6], n2[6];
        spectral_gradient(Q1, g, n1);
        spectral_gradient(Q2, g + 3, n2);
        for (int i = 0; i < 6; ++i) {
            double v = 0.0;
            for (int j = 0; j < 6; ++j) v += L1[6 * j + i] * n1[j] + L2[6 * j + i] * n2[j];
            N[i] = v;
        }
    }
    if (dNdT) {
        double H11[36], H12[36], H21[36], H22[36], hb[9];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) hb[3 * i + k] = h[6 * i + k];
        spectral_block(Q1, Q1, lam, g, hb, 1, H11);
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) hb[3 * i + k] = h[6 * i + 3 + k];
        spectral_block(Q1, Q2, lam, g, hb, 0, H12);
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) hb[3 * i + k] = h[6 * (3 + i) + k];
        spectral_block(Q2, Q1, lam + 3, g + 3, hb, 0, H21);
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) hb[3 * i + k] = h[6 * (3 + i) + 3 + k];
        spectral_block(Q2, Q2, lam + 3, g + 3, hb, 1, H22);
        /* dN/dt = L1^T (H11 L1 + H12 L2) + L2^T (H21 L1 + H22 L2) */
        double A1[36], A2[36];
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double a = 0.0, b = 0.0;
                for (int k = 0; k < 6; ++k) {
                    a += H11[6 * i + k] * L1[6 * k + j] + H12[6 * i + k] * L2[6 * k + j];
                    b += H21[6 * i + k] * L1[6 * k + j] + H22[6 * i + k] * L2[6 * k + j];
                }
                A1[6 * i + j] = a;
                A2[6 * i + j] = b;
            }
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double v = 0.0;
                for (int k = 0; k < 6; ++k) v += L1[6 * k + i] * A1[6 * k + j] + L2[6 * k + i] * A2[6 * k + j];
                dNdT[6 * i + j] = v;
            }
    }
    return phi;
}

/* ------------------------------------------------------------------ */
/* closest-point projection, Eq. (local_cpp): y = [T(6), alpha, dgamma] */
/* ------------------------------------------------------------------ */

typedef struct {
    double Em[36], Hm[36];
    double ee_tr[6]; /* Mandel eps_{n+1} - eps^p_n */
    double alpha_n;
    const double *prm;
    int voce;
    const double *Theta; /* orientation, or NULL */
    int barlat;          /* Barlat Yld2004-18p instead of Hill-48 */
    double L1[36], L2[36], mexp;
} cpp_ctx;

/* Effective stress phi(t), flow direction N = dphi/dt and dN/dt (the last two
 * may be NULL) of the context's yield function. */
static double yield_eval(const cpp_ctx *c, const double t[6], double *N, double *dNdT) {
    if (c->barlat) return barlat_eval(c->L1, c->L2, c->mexp, t, N, dNdT);
    double phi = hill_phi(c->Hm, t);
    double Nl[6];
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += c->Hm[6 * i + j] * t[j];
        Nl[i] = s / phi;
    }
    if (N) memcpy(N, Nl, sizeof Nl);
    if (dNdT)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) dNdT[6 * i + j] = (c->Hm[6 * i + j] - Nl[i] * Nl[j]) / phi;
    return phi;
}

static void cpp_residual(const cpp_ctx *c, const double y[8], double G[8]) {
    const double *t = y;
    double alpha = y[6], dg = y[7];
    double N[6];
    double phi = yield_eval(c, t, N, NULL);
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += c->Em[6 * i + j] * (c->ee_tr[j] - dg * N[j]);
        G[i] = t[i] - s;
    }
    G[6] = alpha - c->alpha_n - dg;
    G[7] = phi - hardening(c->prm, c->voce, alpha, NULL);
}

/* analytic J^G = dG/dy */
static void cpp_jacobian(const cpp_ctx *c, const double y[8], double J[64]) {
    double alpha = y[6], dg = y[7];
    double N[6], dN[36];
    yield_eval(c, y, N, dN);
    memset(J, 0, 64 * sizeof(double));
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += c->Em[6 * i + k] * dN[6 * k + j];
            J[8 * i + j] = (i == j ? 1.0 : 0.0) + dg * s;
        }
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += c->Em[6 * i + k] * N[k];
        J[8 * i + 7] = s;
    }
    J[8 * 6 + 6] = 1.0;
    J[8 * 6 + 7] = -1.0;
    double dsig;
    hardening(c->prm, c->voce, alpha, &dsig);
    for (int j = 0; j < 6; ++j) J[8 * 7 + j] = N[j];
    J[8 * 7 + 6] = -dsig;
}

/* merit psi = 1/2 |D G|^2, Eq. (merit), on the scaled residual */
static double cpp_merit(const cpp_ctx *c, const double y[8], const double D[8]) {
    double G[8];
    cpp_residual(c, y, G);
    double s = 0.0;
    for (int i = 0; i < 8; ++i) s += (D[i] * G[i]) * (D[i] * G[i]);
    return 0.5 * s;
}

/* Options of the local Newton iteration: the line search of App. B on or off
 * (off: every step is the full Newton step, the "standard Newton method" of
 * App. B's comparison), the iteration limit k_max, the merit scaling (1: the
 * scaled residual D G of the design notes; 0: psi = 1/2 G^T G exactly as in
 * Eq. (merit)), and an optional per-iteration trace (ORACLE_TRACE_REC doubles
 * per outer iteration, layout in oracle.h). */
typedef struct {
    int line_search, kmax, scaled;
    double *trace;
    int trace_cap, n_rec;
} cpp_opts;

static cpp_opts default_opts(void) {
    cpp_opts o = {1, KMAX, 0, NULL, 0, 0};
    return o;
}

/* Alg. C2: Newton with the line search of App. B.  Returns the iteration
 * count (negative if not converged).  Line search (App. B): the full step is
 * taken if psi(1) < (1 - 2 beta) psi(0) (Goldstein); otherwise the first
 * candidate minimises the quadratic model through psi(0), psi'(0) = -2 psi(0)
 * and psi(1), Eq. (alpha_init), and is taken if it passes the Goldstein test
 * with its own step length; each further candidate minimises the model
 * through psi(0) and the merit at the previous candidate, Eq.
 * (alpha_update_ls), bounded below by eta times the previous candidate, Eq.
 * (alpha_safeguard), and is taken once it passes the Goldstein test.  After
 * j_max rejected updates the last candidate is taken.  The merit is
 * psi = 1/2 G^T G of Eq. (merit) unless the options ask for the scaled
 * residual. */
static int cpp_solve(const cpp_ctx *c, double y[8], cpp_opts *o) {
    double mu = c->Em[35] / 2.0;
    double sy_n = hardening(c->prm, c->voce, c->alpha_n, NULL);
    double D[8] = {1 / mu, 1 / mu, 1 / mu, 1 / mu, 1 / mu, 1 / mu, 1.0, 1.0 / sy_n};
    double Dm[8];
    for (int i = 0; i < 8; ++i) Dm[i] = o->scaled ? D[i] : 1.0;
    double prev = INFINITY, best = INFINITY, ybest[8];
    for (int k = 0; k <= o->kmax; ++k) {
        double G[8], J[64], dy[8];
        cpp_residual(c, y, G);
        double gn = 0.0;
        for (int i = 0; i < 8; ++i) gn = fmax(gn, fabs(D[i] * G[i]));
        if (!(gn == gn)) return -(k + 1);
        if (gn <= LOCAL_TOL) return k;
        /* rounding floor reached: a step below 1e-9 that does not halve the
         * residual; the best iterate is kept.  The floor grows with the size
         * of the stress (about 1.5e-12 at a hydrostatic stress of -8.5e4 MPa),
         * so it is detected by the stalled decrease, not by a fixed level. */
        if (gn <= 1e-9 && gn >= 0.5 * prev) {
            if (best < gn)
                for (int i = 0; i < 8; ++i) y[i] = ybest[i];
            return k;
        }
        if (gn < best) {
            best = gn;
            for (int i = 0; i < 8; ++i) ybest[i] = y[i];
        }
        if (k == o->kmax) break;
        prev = gn;
        cpp_jacobian(c, y, J);
        for (int i = 0; i < 8; ++i) dy[i] = -G[i];
        if (solve_dense(8, J, dy)) return -(k + 1);
        double psi0 = 0.0;
        for (int i = 0; i < 8; ++i) psi0 += (Dm[i] * G[i]) * (Dm[i] * G[i]);
        psi0 *= 0.5;
        double yt[8];
        for (int i = 0; i < 8; ++i) yt[i] = y[i] + dy[i];
        double psi1 = cpp_merit(c, yt, Dm);
        double zeta = 1.0;
        double zs[JMAX + 2], ps[JMAX + 2];
        int m = 0; /* candidates evaluated */
        if (o->line_search && !(psi1 < (1.0 - 2.0 * LS_BETA) * psi0)) {
            zs[0] = psi0 / (psi0 + psi1); /* Eq. (alpha_init) */
            if (!(zs[0] == zs[0])) zs[0] = LS_ETA;
            for (int i = 0; i < 8; ++i) yt[i] = y[i] + zs[0] * dy[i];
            ps[0] = cpp_merit(c, yt, Dm);
            m = 1;
            zeta = zs[0];
            /* App. B: the initial trial step is kept if it passes the Goldstein
             * test; only otherwise is the quadratic model updated */
            if (!(ps[0] < (1.0 - 2.0 * LS_BETA * zs[0]) * psi0)) {
                for (int jj = 0; jj <= JMAX; ++jj) {
                    double zn = psi0 / (psi0 + ps[jj]); /* Eq. (alpha_update_ls) */
                    zn = fmax(LS_ETA * zs[jj], zn);      /* Eq. (alpha_safeguard) */
                    for (int i = 0; i < 8; ++i) yt[i] = y[i] + zn * dy[i];
                    zs[jj + 1] = zn;
                    ps[jj + 1] = cpp_merit(c, yt, Dm);
                    m = jj + 2;
                    zeta = zn;
                    if (ps[jj + 1] < (1.0 - 2.0 * LS_BETA * zn) * psi0) break; /* Goldstein */
                }
            }
        }
        if (o->trace && o->n_rec < o->trace_cap) {
            double *r = o->trace + (size_t)o->n_rec * ORACLE_TRACE_REC;
            memset(r, 0, ORACLE_TRACE_REC * sizeof(double));
            r[0] = k;
            r[1] = gn;
            r[2] = psi0;
            r[3] = psi1;
            r[4] = zeta;
            r[5] = m;
            for (int i = 0; i < 8; ++i) r[6 + i] = y[i];
            for (int i = 0; i < 8; ++i) r[14 + i] = dy[i];
            for (int j = 0; j < m; ++j) {
                r[22 + j] = zs[j];
                r[22 + (JMAX + 2) + j] = ps[j];
            }
            ++o->n_rec;
        }
        for (int i = 0; i < 8; ++i) y[i] += zeta * dy[i];
    }
    return -(o->kmax + 1);
}

/* Sets up the local system of a material point from the Mandel logarithmic
 * strain eps_{n+1}, the Mandel plastic strain eps^p_n and alpha_n. */
static void cpp_ctx_init(cpp_ctx *c, const double eps_m[6], const double epsp_n[6], double alpha_n,
                         const double prm[11], int model, const double *Theta) {
    elastic_mandel(prm, c->Em);
    hill_mandel(prm, c->Hm);
    rotate_hill(Theta, c->Hm);
    c->prm = prm;
    c->voce = (model & ORACLE_MODEL_VOCE) != 0;
    c->Theta = Theta;
    c->barlat = (model & ORACLE_MODEL_BARLAT) != 0;
    if (c->barlat) {
        barlat_transform(g_barlat, c->L1);
        barlat_transform(g_barlat + 9, c->L2);
        rotate_hill(Theta, c->L1); /* the same rotation of a fourth-order tensor */
        rotate_hill(Theta, c->L2);
        c->mexp = g_barlat[18];
    }
    c->alpha_n = alpha_n;
    for (int i = 0; i < 6; ++i) c->ee_tr[i] = eps_m[i] - epsp_n[i];
}

/* ------------------------------------------------------------------ */
/* material point, Alg. C1                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    /* kinematics */
    double F[9], Q[9], mu[3], f1[9];
    /* constitutive state */
    double T[9], Tm[6], S[9], P[9];
    double hist[7];
    double Cep[36], Cep_impl[36];
    int plastic, iters, converged;
    double dgamma, ftr, sy_n;
    /* converged local system, kept for the VJP */
    cpp_ctx ctx;
    double y[8];
} mp_state;

static void mp_update(const double F[9], const double hist_n[7], const double prm[11], int model,
                      const double *Theta, mp_state *s) {
    memcpy(s->F, F, 9 * sizeof(double));
    /* C - I = H + H^T + H^T H with H = F - I (no cancellation against I) */
    double H[9], M[9];
    for (int i = 0; i < 9; ++i) H[i] = F[i] - ((i % 4 == 0) ? 1.0 : 0.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double hth = 0.0;
            for (int k = 0; k < 3; ++k) hth += H[3 * k + i] * H[3 * k + j];
            M[3 * i + j] = H[3 * i + j] + H[3 * j + i] + hth;
        }
    oracle_eig_sym3(M, s->mu, s->Q);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s->f1[3 * a + b] = dd1(s->mu[a], s->mu[b]);

    /* eps = sum_a 1/2 ln(c_a) N_a (x) N_a, Eq. (c_decomp) */
    double eps[9], epshat[9] = {0};
    for (int a = 0; a < 3; ++a) epshat[4 * a] = 0.5 * log1p(s->mu[a]);
    rot_from_frame(s->Q, epshat, eps);
    double eps_m[6], epsp_n[6], epsp_t[9];
    sym_to_mandel(eps, eps_m);
    double hp[9];
    hp[0] = hist_n[0];
    hp[4] = hist_n[1];
    hp[8] = hist_n[2];
    hp[5] = hp[7] = hist_n[3];
    hp[2] = hp[6] = hist_n[4];
    hp[1] = hp[3] = hist_n[5];
    sym_to_mandel(hp, epsp_n);
    (void)epsp_t;

    cpp_ctx *c = &s->ctx;
    cpp_ctx_init(c, eps_m, epsp_n, hist_n[6], prm, model, Theta);

    /* elastic predictor, Eq. (Tr_stress) */
    double ttr[6];
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += c->Em[6 * i + j] * c->ee_tr[j];
        ttr[i] = acc;
    }
    s->sy_n = hardening(prm, c->voce, c->alpha_n, NULL);
    s->ftr = yield_eval(c, ttr, NULL, NULL) - s->sy_n;

    double epsp_np1[6];
    double alpha_np1;
    if (s->ftr <= 0.0) {
        s->plastic = 0;
        s->iters = 0;
        s->converged = 1;
        s->dgamma = 0.0;
        memcpy(s->Tm, ttr, sizeof ttr);
        memcpy(epsp_np1, epsp_n, sizeof epsp_np1);
        alpha_np1 = c->alpha_n;
        memcpy(s->Cep, c->Em, sizeof s->Cep);
        memcpy(s->Cep_impl, c->Em, sizeof s->Cep_impl);
        for (int i = 0; i < 6; ++i) s->y[i] = ttr[i];
        s->y[6] = c->alpha_n;
        s->y[7] = 0.0;
    } else {
        s->plastic = 1;
        double *y = s->y;
        for (int i = 0; i < 6; ++i) y[i] = ttr[i];
        y[6] = c->alpha_n;
        y[7] = 0.0;
        cpp_opts o = default_opts();
        int it = cpp_solve(c, y, &o);
        s->converged = it >= 0;
        s->iters = it >= 0 ? it : -it;
        s->dgamma = y[7];
        alpha_np1 = y[6];
        /* recovery step of Alg. C2 */
        double N[6], dNdT[36];
        yield_eval(c, y, N, dNdT);
        for (int i = 0; i < 6; ++i) epsp_np1[i] = epsp_n[i] + s->dgamma * N[i];
        for (int i = 0; i < 6; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 6; ++j) acc += c->Em[6 * i + j] * (eps_m[j] - epsp_np1[j]);
            s->Tm[i] = acc;
        }
        /* closed-form algorithmic tangent:
         *   Xi = (E^-1 + dgamma dN/dT)^-1,  Cep = Xi - (Xi N)(Xi N)^T / (N.Xi.N + sigma_y') */
        double Einv[36], Am[36], Xi[36];
        invert_dense(6, c->Em, Einv);
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j)
                Am[6 * i + j] = Einv[6 * i + j] + s->dgamma * dNdT[6 * i + j];
        invert_dense(6, Am, Xi);
        double v[6], nxn = 0.0, dsig;
        hardening(prm, c->voce, alpha_np1, &dsig);
        for (int i = 0; i < 6; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 6; ++j) acc += Xi[6 * i + j] * N[j];
            v[i] = acc;
            nxn += N[i] * acc;
        }
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) s->Cep[6 * i + j] = Xi[6 * i + j] - v[i] * v[j] / (nxn + dsig);
        /* App. D: J_y ydot = -dG/deps, one solve per Mandel direction */
        double J[64];
        cpp_jacobian(c, y, J);
        for (int col = 0; col < 6; ++col) {
            double W[64], rhs[8];
            memcpy(W, J, sizeof W);
            for (int i = 0; i < 6; ++i) rhs[i] = c->Em[6 * i + col];
            rhs[6] = rhs[7] = 0.0;
            solve_dense(8, W, rhs);
            for (int i = 0; i < 6; ++i) s->Cep_impl[6 * i + col] = rhs[i];
        }
    }
    mandel_to_sym(s->Tm, s->T);
    if (s->plastic) {
        double ep[9];
        mandel_to_sym(epsp_np1, ep);
        s->hist[0] = ep[0];
        s->hist[1] = ep[4];
        s->hist[2] = ep[8];
        s->hist[3] = ep[5];
        s->hist[4] = ep[2];
        s->hist[5] = ep[1];
        s->hist[6] = alpha_np1;
    } else {
        memcpy(s->hist, hist_n, 7 * sizeof(double)); /* Alg. C1: history unchanged */
    }

    /* geometric postprocessor: S = P_L : T, P = F S.  In the eigenframe of
     * C, (P_L : T)^_ab = 2 f1(c_a, c_b) T^_ab. */
    double That[9], Shat[9];
    rot_to_frame(s->Q, s->T, That);
    for (int i = 0; i < 9; ++i) Shat[i] = 2.0 * s->f1[i] * That[i];
    rot_from_frame(s->Q, Shat, s->S);
    matmul3(F, s->S, s->P);
}

/* Lagrangian tangent C = 2 dS/dC as a Mandel 6x6 matrix:
 *   dS = P_L : Cep : (1/2 P_L : dC) + d(P_L) : T,
 *   (d(P_L):T)^_ab = 2 sum_r f2(c_a,c_b,c_r) (dC^_ar T^_rb + T^_ar dC^_rb). */
static void mp_lagrangian_tangent(const mp_state *s, double Cm[36]) {
    double That[9];
    rot_to_frame(s->Q, s->T, That);
    double f2[27];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int r = 0; r < 3; ++r) f2[9 * a + 3 * b + r] = dd2(s->mu[a], s->mu[b], s->mu[r]);
    for (int col = 0; col < 6; ++col) {
        double e[6] = {0}, dC[9], dCh[9], deh[9], de[9], dem[6], dTm[6], dT[9], dTh[9], dSh[9],
               dS[9];
        e[col] = 1.0;
        mandel_to_sym(e, dC);
        rot_to_frame(s->Q, dC, dCh);
        for (int i = 0; i < 9; ++i) deh[i] = s->f1[i] * dCh[i];
        rot_from_frame(s->Q, deh, de);
        sym_to_mandel(de, dem);
        for (int i = 0; i < 6; ++i) {
            double acc = 0.0;
            for (int j = 0; j < 6; ++j) acc += s->Cep[6 * i + j] * dem[j];
            dTm[i] = acc;
        }
        mandel_to_sym(dTm, dT);
        rot_to_frame(s->Q, dT, dTh);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double x = 0.0;
                for (int r = 0; r < 3; ++r)
                    x += f2[9 * a + 3 * b + r] * (dCh[3 * a + r] * That[3 * r + b] +
                                                  That[3 * a + r] * dCh[3 * r + b]);
                dSh[3 * a + b] = 2.0 * s->f1[3 * a + b] * dTh[3 * a + b] + 2.0 * x;
            }
        rot_from_frame(s->Q, dSh, dS);
        for (int i = 0; i < 9; ++i) dS[i] *= 2.0;
        double v[6];
        sym_to_mandel(dS, v);
        for (int i = 0; i < 6; ++i) Cm[6 * i + col] = v[i];
    }
}

/* A_aAbB = delta_ab S_AB + F_aC F_bD Cfull_CADB,  Cfull from Mandel */
static void mp_nominal_tangent(const mp_state *s, const double Cm[36], double A[81]) {
    double C4[81];
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            double cI = I < 3 ? 1.0 : SQRT2, cJ = J < 3 ? 1.0 : SQRT2;
            double v = Cm[6 * I + J] / (cI * cJ);
            int a = MI[I], b = MJ[I], c = MI[J], d = MJ[J];
            C4[27 * a + 9 * b + 3 * c + d] = v;
            C4[27 * b + 9 * a + 3 * c + d] = v;
            C4[27 * a + 9 * b + 3 * d + c] = v;
            C4[27 * b + 9 * a + 3 * d + c] = v;
        }
    const double *F = s->F;
    for (int a = 0; a < 3; ++a)
        for (int A_ = 0; A_ < 3; ++A_)
            for (int b = 0; b < 3; ++b)
                for (int B = 0; B < 3; ++B) {
                    double v = (a == b) ? s->S[3 * A_ + B] : 0.0;
                    for (int C = 0; C < 3; ++C)
                        for (int D = 0; D < 3; ++D)
                            v += F[3 * a + C] * F[3 * b + D] * C4[27 * C + 9 * A_ + 3 * D + B];
                    A[27 * a + 9 * A_ + 3 * b + B] = v;
                }
}

int oracle_material_point(const double F[9], const double hist_n[7], const double prm[11],
                          int model, const double *Theta, double *S, double *P, double *T,
                          double *hist_np1, double *A, double *Cep, double *Cep_implicit,
                          double *Cmat, double *info) {
    mp_state s;
    mp_update(F, hist_n, prm, model, Theta, &s);
    double Cm[36];
    mp_lagrangian_tangent(&s, Cm);
    if (S) memcpy(S, s.S, 9 * sizeof(double));
    if (P) memcpy(P, s.P, 9 * sizeof(double));
    if (T) memcpy(T, s.T, 9 * sizeof(double));
    if (hist_np1) memcpy(hist_np1, s.hist, 7 * sizeof(double));
    if (Cep) memcpy(Cep, s.Cep, 36 * sizeof(double));
    if (Cep_implicit) memcpy(Cep_implicit, s.Cep_impl, 36 * sizeof(double));
    if (Cmat) memcpy(Cmat, Cm, 36 * sizeof(double));
    if (A) mp_nominal_tangent(&s, Cm, A);
    if (info) {
        info[0] = s.plastic;
        info[1] = s.iters;
        info[2] = s.converged;
        info[3] = s.dgamma;
        info[4] = s.ftr;
        info[5] = s.sy_n;
    }
    return s.converged ? 0 : 1;
}

/* hist_n (stored: eps^p tensor components 11,22,33,23,13,12, alpha) to the
 * Mandel plastic strain */
static void hist_to_mandel(const double hist_n[7], double epsp_n[6]) {
    double hp[9];
    hp[0] = hist_n[0];
    hp[4] = hist_n[1];
    hp[8] = hist_n[2];
    hp[5] = hp[7] = hist_n[3];
    hp[2] = hp[6] = hist_n[4];
    hp[1] = hp[3] = hist_n[5];
    sym_to_mandel(hp, epsp_n);
}

typedef char trace_rec_size_check[(ORACLE_TRACE_JMAX2 == JMAX + 2) ? 1 : -1];

int oracle_local_return(const double eps_m[6], const double hist_n[7], const double prm[11], int model,
                        const double *Theta, int line_search, int kmax, int merit_scaled, double y[8],
                        double *trace, int trace_cap, int *n_rec) {
    cpp_ctx c;
    double epsp_n[6];
    hist_to_mandel(hist_n, epsp_n);
    cpp_ctx_init(&c, eps_m, epsp_n, hist_n[6], prm, model, Theta);
    for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += c.Em[6 * i + j] * c.ee_tr[j];
        y[i] = acc; /* trial stress, Eq. (Tr_stress) */
    }
    y[6] = c.alpha_n;
    y[7] = 0.0;
    cpp_opts o = {line_search != 0, kmax, merit_scaled != 0, trace, trace_cap, 0};
    int it = cpp_solve(&c, y, &o);
    if (n_rec) *n_rec = o.n_rec;
    return it;
}

double oracle_local_merit(const double eps_m[6], const double hist_n[7], const double prm[11], int model,
                          const double *Theta, int merit_scaled, const double y[8]) {
    cpp_ctx c;
    double epsp_n[6];
    hist_to_mandel(hist_n, epsp_n);
    cpp_ctx_init(&c, eps_m, epsp_n, hist_n[6], prm, model, Theta);
    double mu = c.Em[35] / 2.0, sy_n = hardening(prm, c.voce, c.alpha_n, NULL);
    double D[8] = {1 / mu, 1 / mu, 1 / mu, 1 / mu, 1 / mu, 1 / mu, 1.0, 1.0 / sy_n};
    if (!merit_scaled)
        for (int i = 0; i < 8; ++i) D[i] = 1.0;
    return cpp_merit(&c, y, D);
}

void oracle_local_return_batch(int32_t n, const double *eps_m, const double hist_n[7], const double prm[11],
                               int model, const double *Theta, int line_search, int kmax, int merit_scaled,
                               int32_t *iters, int n_threads) {
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int32_t q = 0; q < n; ++q) {
        double y[8];
        iters[q] = oracle_local_return(eps_m + 6 * (size_t)q, hist_n, prm, model, Theta, line_search, kmax,
                                       merit_scaled, y, NULL, 0, NULL);
    }
}

double oracle_effective_stress(const double T[9], const double prm[11], int model, const double *Theta,
                               double N[9]) {
    mp_state ref;
    double F0[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, h0[7] = {0, 0, 0, 0, 0, 0, 0};
    mp_update(F0, h0, prm, model, Theta, &ref); /* sets up the yield function */
    double t[6], Nm[6];
    sym_to_mandel(T, t);
    double phi = yield_eval(&ref.ctx, t, Nm, NULL);
    if (N) mandel_to_sym(Nm, N);
    return phi;
}

void oracle_log_strain(const double F[9], double eps[9]) {
    double M[9], mu[3], Q[9], eh[9] = {0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double hth = 0.0;
            for (int k = 0; k < 3; ++k) {
                double hki = F[3 * k + i] - (k == i), hkj = F[3 * k + j] - (k == j);
                hth += hki * hkj;
            }
            M[3 * i + j] = (F[3 * i + j] - (i == j)) + (F[3 * j + i] - (i == j)) + hth;
        }
    oracle_eig_sym3(M, mu, Q);
    for (int a = 0; a < 3; ++a) eh[4 * a] = 0.5 * log1p(mu[a]);
    rot_from_frame(Q, eh, eps);
}

/* ------------------------------------------------------------------ */
/* hex8 element, Sec. 2.2.4                                            */
/* ------------------------------------------------------------------ */

static const double XI_S[8] = {-1, 1, 1, -1, -1, 1, 1, -1};
static const double ETA_S[8] = {-1, -1, 1, 1, -1, -1, 1, 1};
static const double ZETA_S[8] = {-1, -1, -1, -1, 1, 1, 1, 1};

/* dN_I/dxi_j at the natural point (xi, eta, zeta) */
static void shape_grad_ref(double xi, double eta, double zeta, double dN[24]) {
    for (int I = 0; I < 8; ++I) {
        double a = 1.0 + XI_S[I] * xi, b = 1.0 + ETA_S[I] * eta, c = 1.0 + ZETA_S[I] * zeta;
        dN[3 * I + 0] = 0.125 * XI_S[I] * b * c;
        dN[3 * I + 1] = 0.125 * a * ETA_S[I] * c;
        dN[3 * I + 2] = 0.125 * a * b * ZETA_S[I];
    }
}

/* Gauss point g = i + 2j + 4k at (+-1/sqrt3)^3, weight 1: returns detJ0 and
 * the physical gradients gradN[8][3] */
static double gp_gradients(const double X[24], int g, double gradN[24]) {
    double r = 1.0 / sqrt(3.0);
    double xi = (g & 1) ? r : -r, eta = (g & 2) ? r : -r, zeta = (g & 4) ? r : -r;
    double dN[24], J0[9] = {0}, J0i[9];
    shape_grad_ref(xi, eta, zeta, dN);
    for (int I = 0; I < 8; ++I)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J0[3 * i + j] += X[3 * I + i] * dN[3 * I + j];
    double det = det3(J0);
    inv3(J0, J0i);
    for (int I = 0; I < 8; ++I)
        for (int A = 0; A < 3; ++A) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += J0i[3 * j + A] * dN[3 * I + j];
            gradN[3 * I + A] = s;
        }
    return det;
}

static int all_finite(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Deformation gradients of the element's Gauss points and, with F-bar
 * (Sec. 2.2.4), the modified gradients Fbar_g = (Jbar / J_g)^(1/3) F_g with
 * Jbar = sum_g w detJ0_g J_g / sum_g w detJ0_g, and their derivatives
 * dFm[g][9 * 24] = dFbar_g(cD) / dd(Jb) (the plain dF/dd without F-bar). */
static void element_kinematics(const double X[24], const double d[24], int fbar,
                               double gradN[8][24], double detJ0[8], double F[8][9],
                               double Fm[8][9], double *dFm) {
    double Jg[8], Ve = 0.0, VJ = 0.0;
    for (int g = 0; g < 8; ++g) {
        detJ0[g] = gp_gradients(X, g, gradN[g]);
        for (int a = 0; a < 3; ++a)
            for (int A = 0; A < 3; ++A) {
                double s = (a == A) ? 1.0 : 0.0;
                for (int I = 0; I < 8; ++I) s += d[3 * I + a] * gradN[g][3 * I + A];
                F[g][3 * a + A] = s;
            }
        Jg[g] = det3(F[g]);
        Ve += detJ0[g]; /* Gauss weight 1 */
        VJ += detJ0[g] * Jg[g];
    }
    double Jbar = VJ / Ve;
    /* dJ_g/dd_Jb = J_g (F_g^-T)_bE dN_J/dX_E; dJbar/dd = sum_g w detJ0_g dJ_g/dd / V_e */
    double dJ[8][24], dJbar[24] = {0};
    if (fbar)
        for (int g = 0; g < 8; ++g) {
            double Fi[9];
            inv3(F[g], Fi);
            for (int J = 0; J < 8; ++J)
                for (int b = 0; b < 3; ++b) {
                    double v = 0.0;
                    for (int E = 0; E < 3; ++E) v += Fi[3 * E + b] * gradN[g][3 * J + E];
                    dJ[g][3 * J + b] = Jg[g] * v;
                    dJbar[3 * J + b] += detJ0[g] * Jg[g] * v / Ve;
                }
        }
    for (int g = 0; g < 8; ++g) {
        double beta = fbar ? cbrt(Jbar / Jg[g]) : 1.0;
        for (int i = 0; i < 9; ++i) Fm[g][i] = beta * F[g][i];
        if (!dFm) continue;
        double *D = dFm + 216 * g;
        for (int c = 0; c < 3; ++c)
            for (int Dd = 0; Dd < 3; ++Dd)
                for (int J = 0; J < 8; ++J)
                    for (int b = 0; b < 3; ++b) {
                        double v = (c == b) ? gradN[g][3 * J + Dd] : 0.0;
                        if (fbar)
                            v += F[g][3 * c + Dd] / 3.0 *
                                 (dJbar[3 * J + b] / Jbar - dJ[g][3 * J + b] / Jg[g]);
                        D[24 * (3 * c + Dd) + 3 * J + b] = beta * v;
                    }
    }
}

void oracle_element(const double X[24], const double d[24], const double hist[56],
                    const double prm[11], int model, const double *Theta, double R[24],
                    double K[576], double hist_np1[56], int32_t diag[4]) {
    memset(R, 0, 24 * sizeof(double));
    if (K) memset(K, 0, 576 * sizeof(double));
    double gradN[8][24], detJ0[8], F[8][9], Fm[8][9];
    double *dFm = K ? malloc(sizeof(double) * 8 * 216) : NULL;
    element_kinematics(X, d, (model & ORACLE_MODEL_FBAR) != 0, gradN, detJ0, F, Fm, dFm);
    for (int g = 0; g < 8; ++g) {
        if (detJ0[g] <= 0.0) diag[1]++;
        if (det3(F[g]) <= 0.0) diag[2]++;
        mp_state s;
        mp_update(Fm[g], hist + 7 * g, prm, model, Theta, &s);
        if (!s.converged) diag[0]++;
        if (hist_np1) memcpy(hist_np1 + 7 * g, s.hist, 7 * sizeof(double));
        double w = detJ0[g]; /* Gauss weight 1 */
        for (int I = 0; I < 8; ++I)
            for (int a = 0; a < 3; ++a) {
                double r = 0.0;
                for (int A = 0; A < 3; ++A) r += s.P[3 * a + A] * gradN[g][3 * I + A];
                R[3 * I + a] += w * r;
            }
        int fin = all_finite(s.P, 9);
        if (K) {
            /* K^e_IaJb = sum_g w detJ0 dN_I/dX_A A_aAcD dF_cD/dd_Jb */
            double Cm[36], A4[81];
            mp_lagrangian_tangent(&s, Cm);
            mp_nominal_tangent(&s, Cm, A4);
            fin = fin && all_finite(A4, 81);
            const double *D = dFm + 216 * g;
            for (int I = 0; I < 8; ++I)
                for (int a = 0; a < 3; ++a)
                    for (int col = 0; col < 24; ++col) {
                        double k = 0.0;
                        for (int A = 0; A < 3; ++A)
                            for (int c = 0; c < 3; ++c)
                                for (int Dd = 0; Dd < 3; ++Dd)
                                    k += gradN[g][3 * I + A] * A4[27 * a + 9 * A + 3 * c + Dd] *
                                         D[24 * (3 * c + Dd) + col];
                        K[24 * (3 * I + a) + col] += w * k;
                    }
        }
        if (!fin) diag[3]++;
    }
    free(dFm);
}

/* ------------------------------------------------------------------ */
/* CSR pattern, App. E                                                 */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* sorted, unique neighbour list of every node (the node itself included) */
static int build_adjacency(int32_t n_nodes, int32_t n_elems, const int32_t *conn,
                           int32_t **adj_ptr_out, int32_t **adj_out) {
    *adj_ptr_out = NULL;
    *adj_out = NULL;
    int32_t *cnt = calloc((size_t)n_nodes + 1, sizeof(int32_t));
    for (int64_t e = 0; e < n_elems; ++e)
        for (int i = 0; i < 8; ++i) {
            int32_t n = conn[8 * e + i];
            if (n < 0 || n >= n_nodes) {
                free(cnt);
                return -5;
            }
            cnt[n + 1] += 8;
        }
    for (int32_t n = 0; n < n_nodes; ++n) cnt[n + 1] += cnt[n];
    int32_t *cand = malloc(sizeof(int32_t) * ((size_t)cnt[n_nodes] + 1));
    int32_t *fill = calloc((size_t)n_nodes, sizeof(int32_t));
    for (int64_t e = 0; e < n_elems; ++e)
        for (int i = 0; i < 8; ++i) {
            int32_t n = conn[8 * e + i];
            for (int j = 0; j < 8; ++j) cand[cnt[n] + fill[n]++] = conn[8 * e + j];
        }
    int32_t *adj_ptr = calloc((size_t)n_nodes + 1, sizeof(int32_t));
    int rc = 0;
    for (int32_t n = 0; n < n_nodes; ++n) {
        int32_t *list = cand + cnt[n];
        int32_t len = cnt[n + 1] - cnt[n];
        if (len == 0) rc = -5; /* orphan node */
        qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
        int32_t u = 0;
        for (int32_t k = 0; k < len; ++k)
            if (u == 0 || list[k] != list[u - 1]) list[u++] = list[k];
        adj_ptr[n + 1] = u;
    }
    for (int32_t n = 0; n < n_nodes; ++n) adj_ptr[n + 1] += adj_ptr[n];
    int32_t *adj = malloc(sizeof(int32_t) * ((size_t)adj_ptr[n_nodes] + 1));
    for (int32_t n = 0; n < n_nodes; ++n)
        memcpy(adj + adj_ptr[n], cand + cnt[n], sizeof(int32_t) * (adj_ptr[n + 1] - adj_ptr[n]));
    free(cand);
    free(fill);
    free(cnt);
    *adj_ptr_out = adj_ptr;
    *adj_out = adj;
    return rc;
}

int oracle_csr_pattern(int32_t n_nodes, int32_t n_elems, const int32_t *conn, int64_t *nnz,
                       int32_t *row_ptr, int32_t *col_idx, uint8_t *elem_rank) {
    int32_t *adj_ptr, *adj;
    int rc = build_adjacency(n_nodes, n_elems, conn, &adj_ptr, &adj);
    if (rc) {
        free(adj_ptr);
        free(adj);
        return rc;
    }
    /* rows 3I+a, columns {3J+b : J in adj(I), b = 0..2} ascending */
    int64_t total = 0;
    row_ptr[0] = 0;
    for (int32_t n = 0; n < n_nodes; ++n) {
        int32_t deg = adj_ptr[n + 1] - adj_ptr[n];
        for (int a = 0; a < 3; ++a) {
            total += 3 * (int64_t)deg;
            row_ptr[3 * n + a + 1] = (int32_t)total;
        }
    }
    *nnz = total;
    if (col_idx) {
        for (int32_t n = 0; n < n_nodes; ++n)
            for (int a = 0; a < 3; ++a) {
                int32_t p = row_ptr[3 * n + a];
                for (int32_t k = adj_ptr[n]; k < adj_ptr[n + 1]; ++k)
                    for (int b = 0; b < 3; ++b) col_idx[p++] = 3 * adj[k] + b;
            }
        if (elem_rank)
            for (int64_t e = 0; e < n_elems; ++e)
                for (int i = 0; i < 8; ++i)
                    for (int j = 0; j < 8; ++j) {
                        int32_t ni = conn[8 * e + i], nj = conn[8 * e + j];
                        int32_t r = 0;
                        while (adj[adj_ptr[ni] + r] != nj) ++r;
                        elem_rank[64 * e + 8 * i + j] = (uint8_t)r;
                    }
    }
    free(adj_ptr);
    free(adj);
    return 0;
}

/* CSR slot of (row, col) by binary search */
static int64_t csr_find(const int32_t *row_ptr, const int32_t *col_idx, int32_t row, int32_t col) {
    int32_t lo = row_ptr[row], hi = row_ptr[row + 1] - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] == col) return mid;
        if (col_idx[mid] < col)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* global residual / tangent / Dirichlet / norm                        */
/* ------------------------------------------------------------------ */

static void gather_element(int64_t e, const double *X, const int32_t *conn, const double *d,
                           const double *hist_n, int64_t n_gp, double Xe[24], double de[24],
                           double he[56]) {
    for (int I = 0; I < 8; ++I) {
        int32_t n = conn[8 * e + I];
        for (int a = 0; a < 3; ++a) {
            Xe[3 * I + a] = X[3 * (int64_t)n + a];
            de[3 * I + a] = d[3 * (int64_t)n + a];
        }
    }
    for (int g = 0; g < 8; ++g)
        for (int k = 0; k < 7; ++k) he[7 * g + k] = hist_n[k * n_gp + 8 * e + g];
}

int oracle_residual_tangent(int32_t n_nodes, int32_t n_elems, const double *X,
                            const int32_t *conn, const int32_t *row_ptr, const int32_t *col_idx,
                            const double *prm, int model, const double *orient,
                            const double *d, const double *hist_n, const uint8_t *bc_mask, double *R, double *K, double *hist_np1,
                            double *rnorm2, int32_t *diag, int n_threads) {
    int64_t n_dof = 3 * (int64_t)n_nodes, n_gp = 8 * (int64_t)n_elems;
    int64_t nnz = row_ptr ? row_ptr[n_dof] : 0;
    memset(R, 0, sizeof(double) * n_dof);
    if (K) memset(K, 0, sizeof(double) * nnz);
    int32_t dg[4] = {0, 0, 0, 0};
    const int64_t CH = 2048;
    double *Rb = malloc(sizeof(double) * 24 * CH);
    double *Kb = K ? malloc(sizeof(double) * 576 * CH) : NULL;
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    for (int64_t e0 = 0; e0 < n_elems; e0 += CH) {
        int64_t ne = (n_elems - e0 < CH) ? n_elems - e0 : CH;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : dg[:4])
        for (int64_t k = 0; k < ne; ++k) {
            int64_t e = e0 + k;
            double Xe[24], de[24], he[56], hn[56];
            int32_t dl[4] = {0, 0, 0, 0};
            gather_element(e, X, conn, d, hist_n, n_gp, Xe, de, he);
            oracle_element(Xe, de, he, prm + 11 * e, model, orient ? orient + 9 * e : NULL,
                           Rb + 24 * k, Kb ? Kb + 576 * k : NULL, hn, dl);
            for (int i = 0; i < 4; ++i) dg[i] += dl[i];
            if (hist_np1)
                for (int g = 0; g < 8; ++g)
                    for (int c = 0; c < 7; ++c) hist_np1[c * n_gp + 8 * e + g] = hn[7 * g + c];
        }
        /* assembly in element order, slot found by binary search */
        for (int64_t k = 0; k < ne; ++k) {
            int64_t e = e0 + k;
            for (int I = 0; I < 8; ++I)
                for (int a = 0; a < 3; ++a) {
                    int32_t row = 3 * conn[8 * e + I] + a;
                    R[row] += Rb[24 * k + 3 * I + a];
                    if (!Kb) continue;
                    for (int J = 0; J < 8; ++J)
                        for (int b = 0; b < 3; ++b) {
                            int64_t slot = csr_find(row_ptr, col_idx, row, 3 * conn[8 * e + J] + b);
                            if (slot < 0) {
                                bad = 1;
                                continue;
                            }
                            K[slot] += Kb[576 * k + 24 * (3 * I + a) + 3 * J + b];
                        }
                }
        }
    }
    free(Rb);
    free(Kb);
    /* Dirichlet rows, Alg. E1: identity row in K, zero residual */
    if (bc_mask)
        for (int64_t r = 0; r < n_dof; ++r) {
            if (!bc_mask[r]) continue;
            R[r] = 0.0;
            if (K)
                for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
                    K[p] = (col_idx[p] == r) ? 1.0 : 0.0;
        }
    if (rnorm2) {
        double s = 0.0;
        long double sl = 0.0L;
        for (int64_t r = 0; r < n_dof; ++r) {
            s += R[r] * R[r];
            sl += (long double)R[r] * (long double)R[r];
        }
        rnorm2[0] = s;
        rnorm2[1] = (double)sl;
    }
    if (diag)
        for (int i = 0; i < 4; ++i) diag[i] = dg[i];
    return bad ? -1 : 0;
}

void oracle_trial_yield(int32_t n_nodes, int32_t n_elems, const double *X, const int32_t *conn,
                        const double *prm, int model, const double *orient, const double *d,
                        const double *hist_n, uint8_t *flag, int n_threads) {
    (void)n_nodes;
    int64_t n_gp = 8 * (int64_t)n_elems;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_elems; ++e) {
        double Xe[24], de[24], he[56];
        gather_element(e, X, conn, d, hist_n, n_gp, Xe, de, he);
        const double *p = prm + 11 * e;
        double Em[36];
        elastic_mandel(p, Em);
        /* the yield function of the material point update, at alpha_n */
        mp_state ref;
        double F0[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, h0[7] = {0, 0, 0, 0, 0, 0, 0};
        mp_update(F0, h0, p, model, orient ? orient + 9 * e : NULL, &ref);
        double gradN[8][24], detJ0[8], F[8][9], Fm[8][9];
        element_kinematics(Xe, de, (model & ORACLE_MODEL_FBAR) != 0, gradN, detJ0, F, Fm, NULL);
        for (int g = 0; g < 8; ++g) {
            double eps[9], em[6], hp[9], pm[6], t[6];
            oracle_log_strain(Fm[g], eps);
            sym_to_mandel(eps, em);
            const double *h = he + 7 * g;
            hp[0] = h[0];
            hp[4] = h[1];
            hp[8] = h[2];
            hp[5] = hp[7] = h[3];
            hp[2] = hp[6] = h[4];
            hp[1] = hp[3] = h[5];
            sym_to_mandel(hp, pm);
            for (int i = 0; i < 6; ++i) {
                double s = 0.0;
                for (int j = 0; j < 6; ++j) s += Em[6 * i + j] * (em[j] - pm[j]);
                t[i] = s;
            }
            double ftr = yield_eval(&ref.ctx, t, NULL, NULL) - hardening(p, (model & ORACLE_MODEL_VOCE) != 0, h[6], NULL);
            flag[8 * e + g] = ftr > 0.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* parameter VJP: forward-mode implicit differentiation (App. D)       */
/* ------------------------------------------------------------------ */

/* Derivatives of phi(T) and N(T) = H T / phi with respect to the Hill
 * parameter k in (F, G, H, N) at fixed T (Mandel t). */
static void hill_param_derivative(const cpp_ctx *c, const double t[6], int k, double dNv[6], double *dphi_out) {
    double phi = hill_phi(c->Hm, t);
    double N[6], dH[36] = {0};
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += c->Hm[6 * i + j] * t[j];
        N[i] = s / phi;
    }
    if (k == 0) { /* F: H22 = F+H, H33 = F+G, H23 = -F */
        dH[7] = dH[14] = 1.0;
        dH[8] = dH[13] = -1.0;
    } else if (k == 1) { /* G: H11 = G+H, H33 = F+G, H13 = -G */
        dH[0] = dH[14] = 1.0;
        dH[2] = dH[12] = -1.0;
    } else if (k == 2) { /* H: H11, H22, H12 = -H */
        dH[0] = dH[7] = 1.0;
        dH[1] = dH[6] = -1.0;
    } else { /* N: shear 12 */
        dH[35] = 1.0;
    }
    rotate_hill(c->Theta, dH); /* the rotation of App. A is linear in H */
    double dHt[6], tdHt = 0.0;
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += dH[6 * i + j] * t[j];
        dHt[i] = s;
        tdHt += t[i] * s;
    }
    double dphi = tdHt / (2.0 * phi);
    for (int i = 0; i < 6; ++i) dNv[i] = dHt[i] / phi - N[i] * dphi / phi;
    *dphi_out = dphi;
}

/* dG/dtheta_k at the converged local solution, k in (F, G, H, N, K, eps0, n)
 * or, with Voce hardening, (F, G, H, N, sig0, Q, b) */
static void cpp_dG_dparam(const cpp_ctx *c, const double y[8], int k, double dG[8]) {
    const double *t = y;
    double alpha = y[6], dg = y[7];
    memset(dG, 0, 8 * sizeof(double));
    if (k <= 3 && c->barlat) return; /* the Hill parameters do not enter Barlat's function */
    if (k <= 3) {
        /* derivative of the Hill matrix with respect to F, G, H or N */
        double dNv[6], dphi;
        hill_param_derivative(c, t, k, dNv, &dphi);
        for (int i = 0; i < 6; ++i) {
            double s = 0.0;
            for (int j = 0; j < 6; ++j) s += c->Em[6 * i + j] * dNv[j];
            dG[i] = dg * s;
        }
        dG[7] = dphi;
    } else if (c->voce) {
        /* sigma_y = sig0 + Q (1 - exp(-b alpha)): d/dsig0, d/dQ, d/db */
        const double *p = c->prm;
        double ex = exp(-p[P_NEXP] * alpha);
        double dsy;
        if (k == 4)
            dsy = 1.0;
        else if (k == 5)
            dsy = 1.0 - ex;
        else
            dsy = p[P_EPS0] * alpha * ex;
        dG[7] = -dsy;
    } else {
        const double *p = c->prm;
        double base = p[P_EPS0] + alpha;
        double sy = p[P_K] * pow(base, p[P_NEXP]);
        double dsy;
        if (k == 4)
            dsy = pow(base, p[P_NEXP]);
        else if (k == 5)
            dsy = p[P_K] * p[P_NEXP] * pow(base, p[P_NEXP] - 1.0);
        else
            dsy = sy * log(base);
        dG[7] = -dsy;
    }
}

/* ------------------------------------------------------------------ */
/* Jacobian of the local update and the element adjoint (App. D)        */
/* ------------------------------------------------------------------ */

/* dz/dp of the local update at a material point, forward mode of App. D:
 * one solve J_y ydot = -dG/dp pdot per input direction, then the output
 * formulas.  Inputs p (20): eps (Mandel 6), hist_n (7 stored components:
 * eps^p 11,22,33,23,13,12 and alpha), theta (7).  Outputs z (13): T (Mandel
 * 6), hist_{n+1} (7 stored components).  Jz is row-major [13][20]. */
static void mp_local_jacobian(const mp_state *s, const double hist_n[7], double Jz[260]) {
    (void)hist_n;
    static const double W[6] = {1.0, 1.0, 1.0, SQRT2, SQRT2, SQRT2}; /* stored -> Mandel */
    const cpp_ctx *c = &s->ctx;
    memset(Jz, 0, 260 * sizeof(double));
    if (!s->plastic) {
        /* T = E : (eps - eps^p_n), history unchanged */
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                Jz[20 * i + j] = c->Em[6 * i + j];
                Jz[20 * i + 6 + j] = -c->Em[6 * i + j] * W[j];
            }
        for (int r = 0; r < 7; ++r) Jz[20 * (6 + r) + 6 + r] = 1.0;
        return;
    }
    const double *y = s->y;
    double dg = y[7];
    double N[6], dNdT[36];
    yield_eval(c, y, N, dNdT);
    double J[64];
    cpp_jacobian(c, y, J);
    for (int k = 0; k < 20; ++k) {
        double Gd[8] = {0}, ep_dot[6] = {0}, dNth[6] = {0};
        if (k < 6) {
            for (int i = 0; i < 6; ++i) Gd[i] = -c->Em[6 * i + k];
        } else if (k < 12) {
            int j = k - 6;
            for (int i = 0; i < 6; ++i) Gd[i] = c->Em[6 * i + j] * W[j];
            ep_dot[j] = W[j];
        } else if (k == 12) {
            Gd[6] = -1.0;
        } else {
            cpp_dG_dparam(c, y, k - 13, Gd);
            if (k - 13 <= 3) {
                double dphi;
                hill_param_derivative(c, y, k - 13, dNth, &dphi);
            }
        }
        double Wm[64], yd[8];
        memcpy(Wm, J, sizeof Wm);
        for (int i = 0; i < 8; ++i) yd[i] = -Gd[i];
        solve_dense(8, Wm, yd);
        for (int i = 0; i < 6; ++i) Jz[20 * i + k] = yd[i];
        /* eps^p_{n+1} = eps^p_n + dgamma N(T; theta) */
        for (int i = 0; i < 6; ++i) {
            double v = ep_dot[i] + yd[7] * N[i] + dg * dNth[i];
            for (int j = 0; j < 6; ++j) v += dg * dNdT[6 * i + j] * yd[j];
            Jz[20 * (6 + i) + k] = v / W[i];
        }
        Jz[20 * 12 + k] = yd[6];
    }
}

int oracle_local_jacobian(const double F[9], const double hist_n[7], const double prm[11], int model,
                          const double *Theta, double Jz[260]) {
    mp_state s;
    mp_update(F, hist_n, prm, model, Theta, &s);
    mp_local_jacobian(&s, hist_n, Jz);
    return s.converged ? 0 : 1;
}

/* P_L : X for a symmetric X, in the eigenframe of C: (P_L : X)^_ab = 2 f1(c_a, c_b) X^_ab */
static void apply_PL(const mp_state *s, const double X[9], double Y[9]) {
    double Xh[9], Yh[9];
    rot_to_frame(s->Q, X, Xh);
    for (int i = 0; i < 9; ++i) Yh[i] = 2.0 * s->f1[i] * Xh[i];
    rot_from_frame(s->Q, Yh, Y);
}

void oracle_element_adjoint(const double X[24], const double d[24], const double hist[56],
                            const double prm[11], int model, const double *Theta, const double *lam,
                            const double *mu, double theta_bar[7], double hbar[56], double ubar[24]) {
    double gradN[8][24], detJ0[8], F[8][9], Fm[8][9];
    double *dFm = malloc(sizeof(double) * 8 * 216);
    element_kinematics(X, d, (model & ORACLE_MODEL_FBAR) != 0, gradN, detJ0, F, Fm, dFm);
    for (int k = 0; k < 7; ++k) theta_bar[k] = 0.0;
    for (int i = 0; i < 24; ++i) ubar[i] = 0.0;
    for (int g = 0; g < 8; ++g) {
        mp_state s;
        mp_update(Fm[g], hist + 7 * g, prm, model, Theta, &s);
        double Jz[260];
        mp_local_jacobian(&s, hist + 7 * g, Jz);
        /* output cotangent: Tbar from lambda^T R = sum_g w detJ0 Lambda : P(Fm) with
         * P = Fm (P_L : T):  Tbar = w detJ0 P_L : sym(Fm^T Lambda); mu for the history */
        double zb[13] = {0};
        if (lam) {
            double Lg[9], FtL[9], Xs[9], Tb[9];
            for (int a = 0; a < 3; ++a)
                for (int A = 0; A < 3; ++A) {
                    double l = 0.0;
                    for (int I = 0; I < 8; ++I) l += lam[3 * I + a] * gradN[g][3 * I + A];
                    Lg[3 * a + A] = l;
                }
            for (int A = 0; A < 3; ++A)
                for (int B = 0; B < 3; ++B) {
                    double v = 0.0;
                    for (int a = 0; a < 3; ++a) v += Fm[g][3 * a + A] * Lg[3 * a + B];
                    FtL[3 * A + B] = v;
                }
            for (int A = 0; A < 3; ++A)
                for (int B = 0; B < 3; ++B) Xs[3 * A + B] = 0.5 * (FtL[3 * A + B] + FtL[3 * B + A]);
            apply_PL(&s, Xs, Tb);
            sym_to_mandel(Tb, zb);
            for (int i = 0; i < 6; ++i) zb[i] *= detJ0[g];
        }
        if (mu)
            for (int r = 0; r < 7; ++r) zb[6 + r] = mu[7 * g + r];
        /* input cotangent p_bar = Jz^T z_bar */
        double pb[20] = {0}, eb_mu[6] = {0};
        for (int k = 0; k < 20; ++k) {
            double v = 0.0;
            for (int r = 0; r < 13; ++r) v += Jz[20 * r + k] * zb[r];
            pb[k] = v;
        }
        for (int k = 0; k < 6; ++k) {
            double v = 0.0;
            for (int r = 6; r < 13; ++r) v += Jz[20 * r + k] * zb[r];
            eb_mu[k] = v;
        }
        for (int k = 0; k < 7; ++k) theta_bar[k] += pb[13 + k];
        for (int r = 0; r < 7; ++r) hbar[7 * g + r] = pb[6 + r];
        /* u_bar from the history cotangent only: eps_bar -> Fm_bar = Fm (P_L : eps_bar)
         * -> u_bar = dFm/dd^T Fm_bar (the F-bar chain is in dFm) */
        double Xe[9], Ye[9], Fb[9];
        mandel_to_sym(eb_mu, Xe);
        apply_PL(&s, Xe, Ye);
        matmul3(Fm[g], Ye, Fb);
        const double *D = dFm + 216 * g;
        for (int col = 0; col < 24; ++col) {
            double v = 0.0;
            for (int i = 0; i < 9; ++i) v += Fb[i] * D[24 * i + col];
            ubar[col] += v;
        }
    }
    free(dFm);
}

int oracle_residual_vjp(int32_t n_nodes, int32_t n_elems, const double *X, const int32_t *conn,
                        const double *prm, int model, const double *orient, const double *d,
                        const double *hist_n, const double *lam, double *g_uniform,
                        double *g_elem, int32_t *diag, int n_threads) {
    (void)n_nodes;
    int64_t n_gp = 8 * (int64_t)n_elems;
    double *ge = malloc(sizeof(double) * 7 * ((size_t)n_elems + 1));
    int32_t dgc[4] = {0, 0, 0, 0};
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : dgc[:4])
    for (int64_t e = 0; e < n_elems; ++e) {
        double Xe[24], de[24], he[56], le[24];
        gather_element(e, X, conn, d, hist_n, n_gp, Xe, de, he);
        for (int I = 0; I < 8; ++I)
            for (int a = 0; a < 3; ++a) le[3 * I + a] = lam[3 * (int64_t)conn[8 * e + I] + a];
        double acc[7] = {0};
        double gradNe[8][24], detJ0e[8], Fe[8][9], Fme[8][9];
        element_kinematics(Xe, de, (model & ORACLE_MODEL_FBAR) != 0, gradNe, detJ0e, Fe, Fme, NULL);
        const double *Th = orient ? orient + 9 * e : NULL;
        for (int g = 0; g < 8; ++g) {
            const double *gradN = gradNe[g], *F = Fme[g]; /* the material sees Fbar */
            double Lg[9];
            double detJ0 = detJ0e[g];
            if (detJ0 <= 0.0) dgc[1]++;
            for (int a = 0; a < 3; ++a)
                for (int A = 0; A < 3; ++A) {
                    double l = 0.0;
                    for (int I = 0; I < 8; ++I) l += le[3 * I + a] * gradN[3 * I + A];
                    Lg[3 * a + A] = l;
                }
            mp_state s;
            mp_update(F, he + 7 * g, prm + 11 * e, model, Th, &s);
            if (!s.converged) dgc[0]++;
            if (!s.plastic) continue; /* elastic T does not depend on theta */
            /* Tbar = P_L : sym(F^T Lambda) (F = Fbar with F-bar: lambda^T R = sum w detJ0 Lambda : P(Fbar)) */
            double FtL[9], X9[9], Xh[9], Tbh[9], Tb[9], Tbm[6];
            for (int A = 0; A < 3; ++A)
                for (int B = 0; B < 3; ++B) {
                    double v = 0.0;
                    for (int a = 0; a < 3; ++a) v += F[3 * a + A] * Lg[3 * a + B];
                    FtL[3 * A + B] = v;
                }
            for (int A = 0; A < 3; ++A)
                for (int B = 0; B < 3; ++B) X9[3 * A + B] = 0.5 * (FtL[3 * A + B] + FtL[3 * B + A]);
            rot_to_frame(s.Q, X9, Xh);
            for (int i = 0; i < 9; ++i) Tbh[i] = 2.0 * s.f1[i] * Xh[i];
            rot_from_frame(s.Q, Tbh, Tb);
            sym_to_mandel(Tb, Tbm);
            double J[64];
            cpp_jacobian(&s.ctx, s.y, J);
            for (int k = 0; k < 7; ++k) {
                double W[64], rhs[8];
                cpp_dG_dparam(&s.ctx, s.y, k, rhs);
                for (int i = 0; i < 8; ++i) rhs[i] = -rhs[i];
                memcpy(W, J, sizeof W);
                solve_dense(8, W, rhs);
                double v = 0.0;
                for (int i = 0; i < 6; ++i) v += Tbm[i] * rhs[i];
                acc[k] += detJ0 * v;
            }
        }
        for (int k = 0; k < 7; ++k) ge[7 * e + k] = acc[k];
    }
    if (g_elem)
        for (int64_t e = 0; e < n_elems; ++e)
            for (int k = 0; k < 7; ++k) g_elem[k * (int64_t)n_elems + e] = ge[7 * e + k];
    if (g_uniform)
        for (int k = 0; k < 7; ++k) {
            double s = 0.0;
            for (int64_t e = 0; e < n_elems; ++e) s += ge[7 * e + k];
            g_uniform[k] = s;
        }
    free(ge);
    if (diag)
        for (int i = 0; i < 4; ++i) diag[i] = dgc[i];
    return 0;
}
