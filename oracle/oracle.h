/*
 * oracle.h -- FP64 CPU reference for the hex8 finite-strain Hill-48 residual,
 * consistent tangent, CSR assembly and parameter VJP.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path.
 *
 * Conventions (all arrays row-major, host memory, double precision):
 *   node coordinates / displacements : [n_nodes][3]
 *   connectivity                     : [n_elems][8], VTK hex order, 0-based
 *   parameters                       : [n_elems][11]
 *        (E, nu, F, G, H, L, M, N, K, eps0, n)  in MPa / mm
 *   history (per Gauss point q=8e+g) : [7][8*n_elems]
 *        eps_p 11,22,33,23,13,12 (tensor components), alpha
 *   3x3 tensors                      : [9], entry (i,j) at 3*i+j
 *   Mandel 6-vectors                 : (11,22,33,sqrt2*23,sqrt2*13,sqrt2*12)
 */
#ifndef FEM_ORACLE_H
#define FEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_NPARAM 11
#define ORACLE_NGRAD 7

/* Model options (bit flags, argument `model`):
 *   ORACLE_MODEL_VOCE  Voce hardening sigma_y = sig0 + Q (1 - exp(-b alpha)),
 *                      Eq. (Hard) in uniaxial-stress units; parameter slots
 *                      (K, eps0, n) hold (sig0, Q, b) and so do the last three
 *                      VJP entries.  Otherwise Swift sigma_y = K (eps0 + alpha)^n.
 *   ORACLE_MODEL_FBAR  F-bar element (Sec. 2.2.4): the material sees
 *                      Fbar = (Jbar / J)^(1/3) F, Jbar = (1/V_e) int J dV.
 * Orientation (argument `Theta`, or `orient` per element): NULL for the
 * identity, else a row-major 3x3 rotation whose columns are the orthotropy
 * axes in global coordinates; the Hill tensor is rotated as in App. A,
 * H_global,ijkl = Theta_ia Theta_jb Theta_kc Theta_ld H_local,abcd.  The
 * plastic strain history is kept in global components. */
#define ORACLE_MODEL_VOCE 1
#define ORACLE_MODEL_FBAR 2
/*   ORACLE_MODEL_BARLAT  Barlat Yld2004-18p yield function (Eq. Phi_barlat,
 *                      App. A) instead of Hill-48, with the coefficients of
 *                      oracle_set_barlat; the Hill slots are ignored and their
 *                      gradient entries are zero. */
#define ORACLE_MODEL_BARLAT 4

/* Barlat coefficients c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55 c'66, the same
 * nine for c'', and the exponent m (process-wide; set before the calls). */
void oracle_set_barlat(const double coef[19]);

/* Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations. */
void oracle_eig_sym3(const double A[9], double w[3], double Q[9]);

/* Effective stress phi(T) of the model's yield function (Hill-48 or Barlat,
 * with the orientation) and its gradient N = dphi/dT (tensor, may be NULL). */
double oracle_effective_stress(const double T[9], const double prm[11], int model, const double *Theta,
                               double N[9]);

/* Logarithmic strain eps = 1/2 ln(F^T F). */
void oracle_log_strain(const double F[9], double eps[9]);

/* Material point: geometric preprocessor, Hill-48/Swift return map and
 * geometric postprocessor.  Outputs (any may be NULL):
 *   S, P, T       second/first Piola-Kirchhoff and logarithmic stress [9]
 *   hist_np1      updated (eps_p, alpha) [7]
 *   A             dP_aA/dF_bB at index ((a*3+A)*3+b)*3+B  [81]
 *   Cep           closed-form algorithmic tangent dT/deps (Mandel) [36]
 *   Cep_implicit  the same tangent by implicit differentiation [36]
 *   Cmat          Lagrangian tangent 2 dS/dC (Mandel) [36]
 *   info          [0]=plastic flag, [1]=local iterations, [2]=converged,
 *                 [3]=delta gamma, [4]=trial yield value f_tr, [5]=sigma_y(alpha_n)
 * Returns 0 on success, 1 if the local Newton did not converge. */
int oracle_material_point(const double F[9], const double hist_n[7], const double prm[11],
                          int model, const double *Theta, double *S, double *P, double *T, double *hist_np1, double *A,
                          double *Cep, double *Cep_implicit, double *Cmat, double *info);

/* Local return map at one material point (App. C Alg. C2 with the line search
 * of App. B) from the Mandel logarithmic strain eps_m[6] and the stored
 * history hist_n[7], starting at y^0 = [T^tr, alpha_n, 0].  Options:
 * line_search (0: full Newton steps, the standard Newton method of App. B's
 * comparison), kmax (iteration limit; the default of the other calls is 100),
 * merit_scaled (1: psi = 1/2 |D G|^2 on the scaled residual
 * D = (1/mu, ..., 1/mu, 1, 1/sigma_y(alpha_n)) used by the other calls; 0:
 * psi = 1/2 G^T G as printed in Eq. (merit)).  The convergence test always
 * uses the scaled residual.  y[8] = [T Mandel, alpha, dgamma] on return.
 * Returns the number of Newton iterations, or -(kmax + 1) (or -(k + 1) on a
 * singular Jacobian / non-finite residual) if not converged.  If trace is
 * non-NULL, one record of ORACLE_TRACE_REC doubles per Newton step (at most
 * trace_cap), count in *n_rec:
 *   [0] k   [1] scaled max-norm of G(y^k)   [2] psi(0)   [3] psi(1)
 *   [4] step length zeta^k taken   [5] m = line-search candidates evaluated
 *   [6..13] y^k   [14..21] delta y^k
 *   [22 + j] candidate zeta^(j), j < m (zeta^(0) from Eq. (alpha_init))
 *   [22 + ORACLE_TRACE_JMAX2 + j] psi(zeta^(j)) */
#define ORACLE_TRACE_JMAX2 22
#define ORACLE_TRACE_REC (22 + 2 * ORACLE_TRACE_JMAX2)
int oracle_local_return(const double eps_m[6], const double hist_n[7], const double prm[11], int model,
                        const double *Theta, int line_search, int kmax, int merit_scaled, double y[8],
                        double *trace, int trace_cap, int *n_rec);

/* The merit psi(y) of the same local system (scaled or as printed). */
double oracle_local_merit(const double eps_m[6], const double hist_n[7], const double prm[11], int model,
                          const double *Theta, int merit_scaled, const double y[8]);

/* oracle_local_return for n strains eps_m[n][6] sharing hist_n: iters[q] as
 * returned there (no trace). */
void oracle_local_return_batch(int32_t n, const double *eps_m, const double hist_n[7], const double prm[11],
                               int model, const double *Theta, int line_search, int kmax, int merit_scaled,
                               int32_t *iters, int n_threads);

/* Element residual R[24] (index 3*I+a) and tangent K[576] (row 3*I+a, col 3*J+b)
 * from node coordinates X[8][3], displacements d[8][3] and per-GP history
 * hist[8][7] (GP-major).  hist_np1[8][7] may be NULL.  diag[4] accumulates
 * (local Newton failures, detJ0<=0, detF<=0, non-finite). */
void oracle_element(const double X[24], const double d[24], const double hist[56],
                    const double prm[11], int model, const double *Theta, double R[24], double K[576], double hist_np1[56],
                    int32_t diag[4]);

/* CSR pattern.  Phase 1 (col_idx == NULL): fills row_ptr[3*n_nodes+1] and *nnz.
 * Phase 2: fills col_idx[nnz] and, if elem_rank != NULL, elem_rank[n_elems][64]
 * with rank(I,J) = position of node conn[e][J] in the sorted adjacency of conn[e][I].
 * Returns 0, or -5 if a node belongs to no element / an index is out of range. */
int oracle_csr_pattern(int32_t n_nodes, int32_t n_elems, const int32_t *conn,
                       int64_t *nnz, int32_t *row_ptr, int32_t *col_idx, uint8_t *elem_rank);

/* Global residual / tangent.  R[3n] (required), K[nnz] (may be NULL),
 * hist_np1 (may be NULL), bc_mask[3n] (may be NULL), rnorm2[2] (may be NULL:
 * [0] = double sum of R^2, [1] = long-double sum rounded to double),
 * diag[4] (may be NULL).  n_threads <= 0 uses the OpenMP default. */
int oracle_residual_tangent(int32_t n_nodes, int32_t n_elems, const double *X,
                            const int32_t *conn, const int32_t *row_ptr, const int32_t *col_idx,
                            const double *prm, int model, const double *orient,
                            const double *d, const double *hist_n, const uint8_t *bc_mask, double *R, double *K, double *hist_np1,
                            double *rnorm2, int32_t *diag, int n_threads);

/* Trial-state yield test only: flag[q] = 1 if f_tr > 0 at Gauss point q. */
void oracle_trial_yield(int32_t n_nodes, int32_t n_elems, const double *X, const int32_t *conn,
                        const double *prm, int model, const double *orient, const double *d, const double *hist_n,
                        uint8_t *flag, int n_threads);

/* Parameter VJP  g_elem[7][n_elems] = lam^T dR/dtheta_e for the 7 parameters
 * (F, G, H, N, K, eps0, n) (Voce: F, G, H, N, sig0, Q, b), by forward-mode implicit differentiation of the
 * local update; g_uniform[7] = sum over elements (either may be NULL). */
int oracle_residual_vjp(int32_t n_nodes, int32_t n_elems, const double *X, const int32_t *conn,
                        const double *prm, int model, const double *orient, const double *d, const double *hist_n,
                        const double *lam, double *g_uniform, double *g_elem, int32_t *diag,
                        int n_threads);

/* Jacobian of the local update at a material point (App. D, forward mode):
 * Jz[13][20] = dz/dp, z = (T Mandel 6, hist_{n+1} stored 7), p = (eps Mandel
 * 6, hist_n stored 7, theta 7).  Returns 0, or 1 if the local Newton did not
 * converge. */
int oracle_local_jacobian(const double F[9], const double hist_n[7], const double prm[11], int model,
                          const double *Theta, double Jz[260]);

/* Element adjoint of one load step for cotangents lam[24] (of R^e, node-major,
 * may be NULL) and mu[8][7] (of hist_{n+1}, GP-major, may be NULL):
 *   theta_bar[7] = lam^T dR^e/dtheta + mu^T dH/dtheta,
 *   hbar[8][7]   = lam^T dR^e/dh_n + mu^T dH/dh_n   (cotangent of hist_n),
 *   ubar[24]     = mu^T dH/dd^e                      (the lam part, K^T lam, is not included). */
void oracle_element_adjoint(const double X[24], const double d[24], const double hist[56],
                            const double prm[11], int model, const double *Theta, const double *lam,
                            const double *mu, double theta_bar[7], double hbar[56], double ubar[24]);

#ifdef __cplusplus
}
#endif
#endif
