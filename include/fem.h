/*
 * fem.h -- C ABI of libfem.so, the MI355X (gfx950) library for the hot path of
 * a finite-strain anisotropic-plasticity finite-element step:
 *
 *   per hex8 element and each of its 2x2x2 Gauss points: logarithmic strain
 *   from C = F^T F (or the F-bar gradient), Hill-48 return mapping (optional
 *   orientation) with Swift or Voce isotropic hardening,
 *   second and first Piola-Kirchhoff stress, element residual R^e and
 *   consistent tangent K^e = dR^e/dd^e, assembled into a fixed CSR pattern;
 *   and the vector-Jacobian product lambda^T dR/dtheta for material parameters.
 *
 * It follows the discrete equilibrium problem of JAX-FEM-ANISO (arXiv
 * 2606.17390): R(d) = A_e R^e(d^e; h_n, theta) with
 * R^e_I = int P(F, h_n) . grad N_I dV (Sec. 2.2.4, element residual), K = dR/dd
 * (Sec. 2.2.4, global tangent), history h_n = (eps^p_n, alpha_n) from the last
 * converged increment (Sec. 2.2.4), the constitutive update of Sec. 2.2.2-2.2.3
 * and App. C (Alg. C1, C2), Dirichlet rows by row elimination (App. E,
 * Alg. E1) and the VJP term (dR/dtheta)^T lambda of Alg. 1 / Eq. (main_grad).
 *
 * Memory: every pointer marked "device" is HIP device memory owned by the
 * caller; the library never frees or retains it (except the multigrid
 * handle of fem_amg_create, which keeps the pattern and matrix pointers it
 * is given and owns the device memory of its hierarchy).  Host pointers are marked
 * "host".  All work is enqueued on `stream` (a hipStream_t; NULL = the null
 * stream) and is asynchronous unless stated otherwise; output arrays are
 * overwritten, never accumulated into.  Scratch space comes from the caller
 * through a workspace pointer whose size the *_workspace_bytes functions
 * return.  Functions return FEM_OK or a negative fem_status; the message of
 * the last error on the calling thread is returned by fem_last_error().
 * Numerical trouble (non-converged local Newton, inverted elements,
 * non-finite values) never aborts: it is counted in the optional diag[4]
 * array.  Calls on different streams that write the same buffers race.
 *
 * Units: mm and MPa.  Layouts:
 *   X, d, R, lam : node-major [n_nodes][3] doubles; dof index = 3*node + comp
 *   conn         : element-major [n_elems][8] int32, VTK hex corner order:
 *                  (-,-,-) (+,-,-) (+,+,-) (-,+,-) (-,-,+) (+,-,+) (+,+,+) (-,+,+)
 *   Gauss points : g = i + 2j + 4k at (xi, eta, zeta) = ((2i-1), (2j-1), (2k-1))/sqrt3,
 *                  weight 1; Gauss point q = 8*e + g
 *   hist         : [7][8*n_elems] doubles: eps^p 11, 22, 33, 23, 13, 12 (tensor
 *                  components of the logarithmic plastic strain), alpha
 *   params       : FEM_P_* below; Hill-48 in the F,G,H,L,M,N form
 *                  phi^2 = F(T22-T33)^2 + G(T33-T11)^2 + H(T11-T22)^2
 *                          + 2L T23^2 + 2M T13^2 + 2N T12^2,
 *                  Swift sigma_y = K (eps0 + alpha)^n (or Voce, FEM_MODEL_VOCE),
 *                  alpha_{n+1} = alpha_n + dgamma
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FEM_OK = 0,
    FEM_EINVAL = -1,    /* invalid argument (NULL where required, bad size, bad enum) */
    FEM_EHIP = -2,      /* a HIP runtime call failed */
    FEM_ENOMEM = -3,    /* workspace smaller than required */
    FEM_EOVERFLOW = -4, /* nnz does not fit in int32 */
    FEM_EMESH = -5,     /* node index out of range, orphan node, more than 64 neighbours */
    FEM_ENOCONV = -6    /* fem_solve: the relative residual did not reach rtol */
} fem_status;

typedef enum {
    FEM_FP64 = 0,      /* everything in FP64 */
    FEM_FP32_MIXED = 1, /* kinematics, log strain, stress pull-back, B^T C B and
                          assembly in FP32; trial stress, yield function, local
                          return-mapping Newton and residual norm in FP64;
                          K_vals is float */
    FEM_FP64_K32 = 2    /* fem_residual_tangent only: FP64 arithmetic as
                          FEM_FP64 (R, history and norm identical), K_vals
                          rounded to float once per entry of K^e and assembled
                          in float: an exact residual for the global Newton
                          iteration with the Krylov solve reading half the
                          matrix bytes */
} fem_precision;

enum {
    FEM_P_E, FEM_P_NU, FEM_P_F, FEM_P_G, FEM_P_H, FEM_P_L, FEM_P_M, FEM_P_N,
    FEM_P_K, FEM_P_EPS0, FEM_P_NEXP, FEM_NPARAM
};
/* with FEM_MODEL_VOCE the three hardening slots hold (sig0, Q, b) */
enum { FEM_P_SIG0 = FEM_P_K, FEM_P_Q = FEM_P_EPS0, FEM_P_B = FEM_P_NEXP };
/* differentiated parameters, in this order (Voce: F, G, H, N, sig0, Q, b) */
enum { FEM_G_F, FEM_G_G, FEM_G_H, FEM_G_N, FEM_G_K, FEM_G_EPS0, FEM_G_NEXP, FEM_NGRAD };
enum { FEM_G_SIG0 = FEM_G_K, FEM_G_Q = FEM_G_EPS0, FEM_G_B = FEM_G_NEXP };

/* Model options (fem_params.model, bit flags; 0 = Swift hardening, plain hex8):
 *   FEM_MODEL_VOCE  Voce isotropic hardening of Eq. (Hard), read in
 *                   uniaxial-stress units as sigma_y = sig0 + Q (1 - exp(-b alpha))
 *                   (the same normalisation as phi and the Swift law).
 *   FEM_MODEL_FBAR  F-bar element of Sec. 2.2.4: the material sees
 *                   Fbar = (Jbar / J)^(1/3) F at each Gauss point, with
 *                   Jbar = (1/V_e) int J dV over the element; R^e_I =
 *                   int P(Fbar) . grad N_I dV and K^e = dR^e/dd^e (not symmetric). */
enum { FEM_MODEL_VOCE = 1u, FEM_MODEL_FBAR = 2u, FEM_MODEL_BARLAT = 4u };
/*   FEM_MODEL_BARLAT Barlat Yld2004-18p yield function (Eq. Phi_barlat, App. A)
 *                   instead of Hill-48: phi = [1/4 sum_ij |s'_i - s''_j|^m]^(1/m)
 *                   over the principal values of C':P:T and C'':P:T, with the
 *                   coefficients of fem_params.barlat (the Hill slots are
 *                   ignored); closest-point Newton iteration with the line
 *                   search of App. B; FP64 local update and tangent in both
 *                   precision forms (FP32_MIXED stores K in FP32).  Forward
 *                   call only (fem_residual_vjp and fem_history_adjoint
 *                   reject it). */

typedef struct {
    int32_t n_nodes, n_elems;
    const double *X;     /* device [n_nodes][3] reference coordinates */
    const int32_t *conn; /* device [n_elems][8] */
} fem_mesh;

/* Parameter k is read from p[k] (device): one value, or n_elems values if
 * bit k of per_elem_mask is set, or n_spec values indexed by specimen if bit k
 * of per_spec_mask is set (batched calls).  per_elem wins if both are set.
 * model: FEM_MODEL_* flags.  orient: material orientation Theta of the Hill
 * tensor (App. A: H_global = Theta Theta : H_local : Theta^T Theta^T), NULL
 * for the identity, else device row-major 3x3 rotations whose columns are
 * the orthotropy axes in global coordinates: one ([9]) or, if
 * orient_per_elem is nonzero, one per element ([n_elems][9]).  Theta must be
 * a proper rotation (not checked).  The plastic strain history is always in
 * global components. */
typedef struct {
    const double *p[FEM_NPARAM];
    uint32_t per_elem_mask;
    uint32_t per_spec_mask;
    uint32_t model;
    uint32_t orient_per_elem;
    const double *orient;
    const double *barlat; /* device [19]: c'12 c'13 c'21 c'23 c'31 c'32 c'44 c'55 c'66,
                             the same nine for c'', m; required with FEM_MODEL_BARLAT */
} fem_params;

/* CSR matrix of the tangent, 3x3 node blocks: row 3I+a holds columns 3J+b
 * for every node J sharing an element with I (I included), ascending.
 * elem_rank[64*e + 8*i + j] = position of node conn[e][j] in the sorted
 * neighbour list of node conn[e][i], so that K(3I+a, 3J+b) sits at
 * row_ptr[3I+a] + 3*rank + b.  node_elem lists, for every node I, the
 * conn entries 8*e + i with conn[e][i] = I, in ascending order, at
 * [node_elem_ptr[I], node_elem_ptr[I+1]) (node -> element incidence used by
 * the row-owner assembly). */
typedef struct {
    int32_t n_rows;         /* 3 * n_nodes */
    int64_t nnz;            /* set by fem_csr_pattern */
    int32_t *row_ptr;       /* device [n_rows + 1] */
    int32_t *col_idx;       /* device [nnz] */
    uint8_t *elem_rank;     /* device [n_elems][64] */
    int32_t *node_elem_ptr; /* device [n_nodes + 1] */
    int32_t *node_elem;     /* device [8 * n_elems] */
} fem_csr;

/* Batched mode: n_spec specimens concatenated (node ids in conn already
 * offset); elements of specimen s are [elem_off[s], elem_off[s+1]).  A NULL
 * fem_batch* means a single specimen. */
typedef struct {
    int32_t n_spec;
    const int64_t *elem_off; /* device [n_spec + 1], elem_off[0] = 0, elem_off[n_spec] = n_elems */
} fem_batch;

/* Launch configuration of the element kernels (set by the autotuner). */
typedef struct {
    int32_t block;         /* threads per workgroup: 64, 128 or 256 (8 per element) */
    int32_t waves_per_cu;  /* persistent grid = waves_per_cu * CUs * 64 / block workgroups */
    int32_t xcd_remap;     /* 1: consecutive tiles stay on one XCD's L2 */
} fem_launch;

/* Kernel ids: the two element kernels (launch configuration and timing) and
 * the two assembly kernels of fem_residual_tangent (timing only). */
enum { FEM_KERNEL_FORWARD = 0, FEM_KERNEL_VJP = 1, FEM_KERNEL_ASSEMBLE_K = 2, FEM_KERNEL_ASSEMBLE_R = 3 };

/* Library version (major*10000 + minor*100 + patch). */
int fem_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *fem_last_error(void);

/* Set (cfg != NULL) or reset (cfg == NULL) the launch configuration of an
 * element kernel (FEM_KERNEL_FORWARD or FEM_KERNEL_VJP) for a precision;
 * process-wide; FEM_FP64_K32 shares the FEM_FP64 setting (it runs the same
 * element kernels).  Defaults: {64, 8, 1} for both.  Returns FEM_EINVAL for
 * bad values. */
int fem_set_launch(int kernel, fem_precision prec, const fem_launch *cfg);
int fem_get_launch(int kernel, fem_precision prec, fem_launch *cfg);

/* Workspace bytes for each operation (host-only query, no GPU work). */
size_t fem_csr_workspace_bytes(int32_t n_nodes, int32_t n_elems);
size_t fem_forward_workspace_bytes(int32_t n_nodes, int32_t n_elems, fem_precision prec);
size_t fem_vjp_workspace_bytes(int32_t n_elems, int32_t n_spec);

/*
 * fem_csr_pattern -- build the CSR pattern of K from the connectivity
 * (App. E, Alg. E1; the pattern is built once per mesh and reused).
 * Two calls:
 *   csr->col_idx == NULL : fills csr->row_ptr (device, [3*n_nodes+1]) and
 *                          csr->nnz; synchronises `stream` to read nnz back.
 *   csr->col_idx != NULL : fills col_idx [nnz] and, if non-NULL, elem_rank,
 *                          node_elem_ptr and node_elem (all three are needed
 *                          by fem_residual_tangent).
 * ws: device workspace of at least fem_csr_workspace_bytes(n_nodes, n_elems)
 * bytes.  Errors: FEM_EINVAL (NULL pointers, negative sizes), FEM_ENOMEM,
 * FEM_EMESH (node id out of range, orphan node, more than 64 neighbours),
 * FEM_EOVERFLOW (nnz >= 2^31), FEM_EHIP.
 */
int fem_csr_pattern(const fem_mesh *mesh, fem_csr *csr, void *ws, size_t ws_bytes, void *stream);

/*
 * fem_residual_tangent -- one residual + tangent + assembly pass
 * (Sec. 2.2.4 element residual and stiffness, App. C Alg. C1/C2 at every
 * Gauss point, App. E row elimination).  Assembly is row-owner and
 * write-once: the element kernel stores R^e and K^e in the workspace, and
 * every entry of R and K is then written exactly once as the sum of its
 * element contributions in ascending element order (no atomics, no prior
 * zeroing, bitwise reproducible for any launch configuration).
 *   csr      complete pattern of this mesh (row_ptr, col_idx, elem_rank,
 *            node_elem_ptr, node_elem), also for a residual-only pass
 *   d        device [n_nodes][3] current displacement
 *   hist_n   device [7][8*n_elems] history of the last converged increment
 *   bc_mask  device [3*n_nodes] uint8 (1 = constrained dof) or NULL: rows of
 *            constrained dofs become identity rows of K and R is zeroed there
 *   prec     FEM_FP64 or FEM_FP32_MIXED
 *   R        device [3*n_nodes] residual, or NULL (then rnorm2 must be NULL)
 *   K_vals   device [nnz] double (FEM_FP64) or float (FEM_FP32_MIXED), or NULL
 *            for a residual-only pass
 *   hist_np1 device [7][8*n_elems] updated history for this d (never committed
 *            by the library), or NULL
 *   rnorm2   device [1] FP64 sum of R_i^2 after row elimination, or NULL
 *   diag     device [4] int32 counters of Gauss points (zeroed by the call):
 *            local Newton not converged, detJ0 <= 0, det F <= 0,
 *            non-finite stress or tangent (also counted: a node id out of
 *            range, replaced by node 0); or NULL
 *   ws       device workspace of fem_forward_workspace_bytes(n_nodes, n_elems,
 *            prec) bytes (element residuals and tangents: 192 + 576*sizeof(K)
 *            bytes per element)
 * Errors: FEM_EINVAL, FEM_ENOMEM, FEM_EHIP.
 */
int fem_residual_tangent(const fem_mesh *mesh, const fem_batch *batch, const fem_csr *csr,
                         const fem_params *params, const double *d, const double *hist_n,
                         const uint8_t *bc_mask, fem_precision prec, double *R, void *K_vals,
                         double *hist_np1, double *rnorm2, int32_t *diag, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * fem_residual_vjp -- g = lam^T dR/dtheta for theta = (F, G, H, N, K, eps0, n)
 * (Alg. 1 "Evaluate VJP", Eq. (main_grad); the derivative of the converged
 * local update follows App. D, applied in reverse mode; the local state is
 * recomputed from d and hist_n, nothing is stored between calls).
 *   lam       device [n_nodes][3] cotangent
 *   g_uniform device [n_spec][7] (n_spec = 1 without batch): sum of g_elem over
 *             the specimen's elements, i.e. the gradient for parameters that are
 *             uniform over the specimen; or NULL
 *   g_elem    device [7][n_elems] per-element gradient, or NULL
 *   ws        device workspace of fem_vjp_workspace_bytes(n_elems, n_spec) bytes
 * The reduction to g_uniform is deterministic.  Elastic Gauss points
 * contribute exactly zero.  Errors: FEM_EINVAL, FEM_ENOMEM, FEM_EHIP.
 */
int fem_residual_vjp(const fem_mesh *mesh, const fem_batch *batch, const fem_params *params,
                     const double *d, const double *hist_n, const double *lam, fem_precision prec,
                     double *g_uniform, double *g_elem, int32_t *diag, void *ws, size_t ws_bytes,
                     void *stream);

/*
 * fem_residual_vjp_noalloc -- fem_residual_vjp without a workspace argument,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace is a file-scope device array of FEM_VJP_SCRATCH_MAX_BYTES bytes,
 * one per device the library runs on, held until the process ends; the call
 * itself allocates nothing.  Arguments, outputs and results are those of
 * fem_residual_vjp (the same kernels run).
 * Limit: fem_vjp_workspace_bytes(n_elems, n_spec) must not exceed
 * FEM_VJP_SCRATCH_MAX_BYTES (about 1.1 million elements); larger meshes get
 * FEM_ENOMEM and must use fem_residual_vjp.
 * All calls on one device share its array: calls that overlap on one device
 * (on different streams, or from different threads) race and give undefined
 * results.  Errors: as fem_residual_vjp, plus FEM_ENOMEM (too large) and
 * FEM_EHIP (the array's device address could not be taken).
 */
#define FEM_VJP_SCRATCH_MAX_BYTES (64u << 20)
int fem_residual_vjp_noalloc(const fem_mesh *mesh, const fem_batch *batch, const fem_params *params,
                             const double *d, const double *hist_n, const double *lam,
                             fem_precision prec, double *g_uniform, double *g_elem, int32_t *diag,
                             void *stream);

/*
 * Linear solve of the global Newton iteration (Sec. 2.2.4: K du = -R, with
 * the Dirichlet rows of App. E as identity rows, so K is not symmetric).
 *
 * fem_csr_spmv -- y = K x for a pattern csr made by fem_csr_pattern (the three
 * rows 3I, 3I+1, 3I+2 of a node are consecutive and share their columns; only
 * row_ptr, col_idx and n_rows are read) and
 * values K_vals (double for FEM_FP64, float for FEM_FP32_MIXED, as written by
 * fem_residual_tangent); x, y device [n_rows] doubles (not aliased).  Errors:
 * FEM_EINVAL, FEM_EHIP.
 *
 * fem_solve -- K x = b (the linear solve of the global Newton iteration,
 * Sec. 2.2.4 / Eq. (Stiffness_mat); Sec. 2.2.5 lists CG and BiCGSTAB) by
 *   FEM_KRYLOV_BICGSTAB  BiCGSTAB, right-preconditioned by M (any K)
 *   FEM_KRYLOV_GMRES     restarted GMRES(FEM_GMRES_RESTART), right-
 *                        preconditioned (any K): classical Gram-Schmidt with
 *                        fused dot products, Givens rotations on the device,
 *                        the solution formed at the end of each cycle and
 *                        the true residual recomputed for the next; the
 *                        reported residual is the cycle's least-squares
 *                        residual |g_{j+1}| / ||b||; workspace of
 *                        fem_solver_workspace_bytes_method (about
 *                        FEM_GMRES_RESTART + 1 more vectors)
 *   FEM_KRYLOV_FGMRES    flexible GMRES(FEM_GMRES_RESTART) (Saad's FGMRES):
 *                        as FEM_KRYLOV_GMRES but keeps z_j = M v_j of every
 *                        step and forms x += Z y, so M may change between
 *                        steps (required by a K-cycle multigrid); the
 *                        workspace holds FEM_GMRES_RESTART more vectors
 *   FEM_KRYLOV_CG        preconditioned conjugate gradients, for a K that is
 *                        symmetric positive definite on the free dofs (the
 *                        tangent without F-bar) with identity rows on the
 *                        constrained ones, and x = b there on entry (the
 *                        Newton correction: both zero); the iterates then
 *                        stay on the free-free block.  Ends (FEM_ENOCONV) if
 *                        a search direction has p.Kp <= 0.
 * with the preconditioner M:
 *   FEM_PC_JACOBI        M = inverse of the diagonal of K
 *   FEM_PC_BLOCK_JACOBI  M = inverses of the 3x3 node blocks K[3I+a][3I+b]
 *                        (a singular block falls back to its diagonal)
 * The CSR must be a pattern of fem_csr_pattern (node blocks, nnz a multiple
 * of 9).  Vectors and scalars are FP64 whatever the type of K.
 *   b        device [n_rows]
 *   x        device [n_rows], initial guess in, solution out
 *   max_iter iteration limit (>= 0); rtol: stop at ||b - K x|| <= rtol ||b||
 *            (||b - K x|| if b = 0), with ||b - K x|| the recursive residual
 *   iters, rel_res  host outputs (iterations done, final relative residual),
 *            or NULL
 *   ws       device workspace of fem_solver_workspace_bytes(n_rows, nnz) bytes
 *            (GMRES, FGMRES: fem_solver_workspace_bytes_method(n_rows, nnz,
 *            method))
 * The reductions are fixed-order (bitwise reproducible).  The iteration state
 * stays on the device; the host reads the stop flag once per 32 iterations
 * (4 with fem_solve_amg; GMRES: once per restart cycle, after every step
 * with fem_solve_amg), one stream synchronisation each.  A breakdown (a zero inner product) or
 * a non-finite residual ends the iteration.  ||b - K x|| is the recursive
 * residual of the method.
 * Returns FEM_ENOCONV if rtol is not reached (x holds the last iterate).
 * Errors: FEM_EINVAL, FEM_ENOMEM, FEM_EHIP, FEM_ENOCONV.
 */
typedef enum { FEM_PC_JACOBI = 0, FEM_PC_BLOCK_JACOBI = 1, FEM_PC_AMG = 2 /* fem_solve_amg only */ } fem_precond;
typedef enum {
    FEM_KRYLOV_BICGSTAB = 0,
    FEM_KRYLOV_CG = 1,
    FEM_KRYLOV_GMRES = 2,
    FEM_KRYLOV_FGMRES = 3
} fem_krylov;
#define FEM_GMRES_RESTART 30
size_t fem_solver_workspace_bytes(int32_t n_rows, int64_t nnz);        /* CG, BiCGSTAB */
size_t fem_solver_workspace_bytes_method(int32_t n_rows, int64_t nnz, fem_krylov method);
int fem_csr_spmv(const fem_csr *csr, const void *K_vals, fem_precision prec, const double *x, double *y,
                 void *stream);
int fem_solve(const fem_csr *csr, const void *K_vals, fem_precision prec, fem_krylov method, fem_precond pc,
              const double *b, double *x, int32_t max_iter, double rtol, int32_t *iters, double *rel_res,
              void *ws, size_t ws_bytes, void *stream);

/*
 * fem_csr_transpose -- KT_vals = values of K^T on the same pattern (the
 * pattern of fem_csr_pattern is structurally symmetric), the matrix of the
 * adjoint solve of Alg. 1 / Eq. (dR_u).  If bc_mask (device [n_rows], may be
 * NULL) marks a dof, row i of KT becomes an identity row, so that solving
 * KT lambda = v with v_i = 0 there gives lambda_i = 0 and the free-free block
 * of K^T for the rest (for a K whose constrained rows are identity rows).
 * K_vals / KT_vals: device [nnz], double (FEM_FP64) or float
 * (FEM_FP32_MIXED), must not alias.  Asynchronous on `stream`.
 */
int fem_csr_transpose(const fem_csr *csr, const void *K_vals, fem_precision prec, const uint8_t *bc_mask,
                      void *KT_vals, void *stream);

/*
 * Aggregation multigrid preconditioner of the Newton solve (Sec. 2.2.5 and
 * App. F solve the linear systems with an algebraic-multigrid-preconditioned
 * Krylov method).  The hierarchy works on 3x3 node blocks:
 *   - aggregation: each level pairs nodes three times by greedy matching
 *     along the strongest connection (Frobenius norm of the block of K,
 *     the larger of the blocks (I, J) and (J, I), over the geometric mean of
 *     the two diagonal-block norms; nodes visited in index order), so an
 *     aggregate holds up to eight nodes; levels are added
 *     until at most FEM_AMG_DENSE_NODES nodes remain or a level keeps more
 *     than 85 % of the nodes of the one above (or FEM_AMG_MAX_LEVELS);
 *   - prolongation P: piecewise-constant per displacement component (the
 *     three translations of each aggregate), zero on constrained dofs;
 *   - coarse operators A_{l+1} = P^T A_l P, sums of masked 3x3 blocks in
 *     FP32 (fixed order); a coarse dof without a free fine dof gets an
 *     identity row;
 *   - smoother: one damped block-Jacobi sweep before and after the coarse
 *     correction, M_l = omega_l D_I^-1 per node (3x3 inverse of the
 *     diagonal block; a singular block falls back to its diagonal), with
 *     omega_l = (4/3) / rho_l and rho_l the spectral radius of D_l^-1 A_l
 *     estimated by 10 power steps from a fixed pseudo-random start vector
 *     (zero on constrained dofs; the set-up is deterministic); omega_l = 0.5
 *     if the estimate is not positive and finite;
 *   - coarsest level: its explicit inverse (Gauss-Jordan with partial
 *     pivoting in FP64; a pivot below 1e-13 of the largest diagonal entry
 *     drops that dof) when it has at most FEM_AMG_DENSE_NODES nodes, else
 *     one smoothing sweep pair.
 * One application z = M r is one V(1,1)-cycle (the default); for a
 * symmetric K it is a symmetric operator (usable with CG).  In a K-cycle
 * (Notay and Vassilevski's recursive Krylov-based cycle) every level c that
 * has at least k_min_nodes nodes, lies above the levels of at most 512 nodes
 * and is not the coarsest replaces its coarse correction by two
 * minimal-residual steps with the cycle below as preconditioner:
 * c1 = B_c rc, v1 = A_c c1, a1 = (v1, rc) / (v1, v1), r2 = rc - a1 v1,
 * c2 = B_c r2, v2 = A_c c2, g = (v2, v1) / (v1, v1),
 * a2 = (v2, r2) / ((v2, v2) - g (v2, v1)), correction (a1 - a2 g) c1 + a2 c2
 * (zero coefficients where a denominator is not positive).  A K-cycle is
 * not a fixed linear operator: fem_solve_amg accepts it with
 * FEM_KRYLOV_FGMRES only.
 *
 * fem_amg_create -- aggregation and coarse patterns, built on the host from
 *   the pattern of csr (fem_csr_pattern) and the block norms of K_vals
 *   (device [nnz], double for FEM_FP64, float for FEM_FP32_MIXED), then
 *   uploaded.  bc_mask: device [n_rows] uint8, nonzero on constrained dofs
 *   (their rows of K are identity rows, as fem_residual_tangent writes
 *   them), or NULL (no constrained dofs).  The handle keeps csr's device
 *   pointers (they must stay valid) and owns device memory allocated here
 *   (freed by fem_amg_destroy); the coarse values are not computed yet
 *   (fem_amg_update).  Synchronises `stream`.
 *   Errors: FEM_EINVAL (bad arguments, a node with more than 21845
 *   neighbours), FEM_ENOMEM (host or device allocation), FEM_EHIP.
 * fem_amg_update -- numeric set-up for values K_vals on the same pattern
 *   (any precision above): Galerkin operators, smoother blocks and their
 *   damping (power iteration), and the coarsest inverse.  The handle keeps K_vals (it must stay valid while
 *   fem_amg_apply / fem_solve_amg use it).  Asynchronous on `stream`.
 * fem_amg_apply -- z = M r, device [n_rows] each (FP64; must not alias).
 *   Asynchronous on `stream`; calls on one handle must not overlap.
 * fem_amg_info -- number of levels and, per level (up to
 *   FEM_AMG_MAX_LEVELS entries each, any may be NULL), nodes, 3x3 blocks and
 *   the smoother damping omega_l of the last fem_amg_update (1 before it and
 *   on a level inverted exactly; host copy, synchronous); dense = 1 if the
 *   coarsest level is inverted exactly.
 * fem_amg_aggregates -- agg (host [nodes of level - 1]) = the aggregate, a
 *   node of `level` (1 <= level < n_levels), of each node of the level above.
 *   Synchronous.
 * fem_amg_plan_host -- the aggregation of fem_amg_create on host arrays
 *   only (no device work): node-block pattern bptr (host [n_nodes + 1],
 *   int64, first block of each node), ncol (host [bptr[n_nodes]], node column
 *   of each block), strength (host, the block norms), bc_mask (host [3
 *   n_nodes] or NULL).  Outputs: n_levels; nodes and blocks per level (host
 *   [FEM_AMG_MAX_LEVELS] each, may be NULL); agg (host, at least 7 n_nodes
 *   entries, or NULL) = the aggregate maps of levels 1, ..., n_levels - 1
 *   one after the other.  fem_amg_create with the same strengths builds the
 *   same hierarchy.
 * fem_amg_set_cycle -- the cycle of later applications: FEM_AMG_CYCLE_V, or
 *   FEM_AMG_CYCLE_K with the two Krylov steps on levels of at least
 *   k_min_nodes (>= 0) nodes.  Host only.  Errors: FEM_EINVAL.
 * fem_solve_amg -- fem_solve (same arguments, workspace and stop rules)
 *   with M = one cycle of amg, after fem_amg_update(amg, K_vals, prec).
 *   csr must be the pattern amg was created on; a K-cycle needs method
 *   FEM_KRYLOV_FGMRES (else FEM_EINVAL).
 */
#define FEM_AMG_MAX_LEVELS 12
#define FEM_AMG_DENSE_NODES 32
typedef struct fem_amg fem_amg;
typedef enum { FEM_AMG_CYCLE_V = 0, FEM_AMG_CYCLE_K = 1 } fem_amg_cycle;
int fem_amg_create(const fem_csr *csr, const void *K_vals, fem_precision prec, const uint8_t *bc_mask,
                   fem_amg **out, void *stream);
int fem_amg_update(fem_amg *amg, const void *K_vals, fem_precision prec, void *stream);
int fem_amg_apply(fem_amg *amg, const double *r, double *z, void *stream);
int fem_amg_info(const fem_amg *amg, int32_t *n_levels, int32_t *nodes, int64_t *blocks, int32_t *dense,
                 double *omega);
int fem_amg_aggregates(const fem_amg *amg, int32_t level, int32_t *agg);
int fem_amg_plan_host(int32_t n_nodes, const int64_t *bptr, const int32_t *ncol, const float *strength,
                      const uint8_t *bc_mask, int32_t *n_levels, int32_t *nodes, int64_t *blocks, int32_t *agg);
int fem_amg_set_cycle(fem_amg *amg, fem_amg_cycle cycle, int32_t k_min_nodes);
int fem_amg_destroy(fem_amg *amg);
int fem_solve_amg(const fem_csr *csr, const void *K_vals, fem_precision prec, fem_krylov method, fem_amg *amg,
                  const double *b, double *x, int32_t max_iter, double rtol, int32_t *iters, double *rel_res,
                  void *ws, size_t ws_bytes, void *stream);

/*
 * fem_history_adjoint -- one load step of the time-history adjoint (Sec. 2.3,
 * Eqs. (Lagrangian)-(dR_u), Alg. 1) of the time-discrete problem whose
 * history h^n is produced by the local update H^n(u^n, h^{n-1}, theta) of
 * the converged step.  For the state (d = u^n, hist_n = h^{n-1}) of step n
 * and the cotangents lam (of R^n, device [n_nodes][3], or NULL = 0) and mu
 * (of h^n, device [7][8 n_elems] in the hist layout, or NULL = 0):
 *   g_elem [7][n_elems], g_uniform [7]: lam^T dR^n/dtheta + mu^T dH^n/dtheta
 *   hbar [7][8 n_elems]: lam^T dR^n/dh^{n-1} + mu^T dH^n/dh^{n-1} (the mu of
 *                        step n-1)
 *   ubar [n_nodes][3]:   mu^T dH^n/du^n (the lam part is K^T lam; apply it
 *                        with fem_csr_transpose and the assembled tangent)
 * Any output may be NULL (ubar needs csr's node incidence).  FP64 only;
 * model options and orientation as in fem_residual_tangent; no per-specimen
 * parameters.  diag[4] as in fem_residual_vjp (zeroed by the call) or NULL.
 * ws: device workspace of fem_history_adjoint_workspace_bytes bytes.
 * Errors: FEM_EINVAL, FEM_ENOMEM, FEM_EHIP.
 */
size_t fem_history_adjoint_workspace_bytes(int32_t n_nodes, int32_t n_elems);
int fem_history_adjoint(const fem_mesh *mesh, const fem_csr *csr, const fem_params *params, const double *d,
                        const double *hist_n, const double *lam, const double *mu, double *g_uniform,
                        double *g_elem, double *hbar, double *ubar, int32_t *diag, void *ws, size_t ws_bytes,
                        void *stream);

/*
 * Kernel timing for benchmarks: while enabled, every launch of kernel
 * `kernel` (FEM_KERNEL_FORWARD / FEM_KERNEL_VJP: the main element kernel, not
 * the FP64 guard-band re-run; FEM_KERNEL_ASSEMBLE_K / _R: the tangent and
 * residual assembly kernels) is bracketed by a pair of HIP events recorded on
 * the launch stream.  fem_timing_read waits
 * for the recorded events, returns the summed elapsed milliseconds and the
 * number of launches since the previous read, and releases the events.
 * Do not enable while capturing a graph.
 */
int fem_timing_enable(int on);
int fem_timing_read(int kernel, double *total_ms, int32_t *launches);

/*
 * HIP graph helpers for launch-bound callers (e.g. many small specimens):
 * capture the library calls issued on `stream` between begin and end into an
 * executable graph.  The library issues no memset nodes (buffers are cleared
 * by kernels), so a graph may be replayed any number of times.
 */
int fem_graph_begin(void *stream);
int fem_graph_end(void *stream, void **graph_exec);
int fem_graph_launch(void *graph_exec, void *stream);
int fem_graph_destroy(void *graph_exec);

#ifdef __cplusplus
}
#endif
#endif /* FEM_H */
