// forward.hip -- residual + consistent tangent + CSR assembly pass.
//
// One lane per Gauss point, 8 lanes per element, BLOCK/8 elements per
// workgroup; a persistent grid walks element tiles (XCD-aware order so that
// neighbouring elements, which share CSR entries, stay on one L2).
//
// Per Gauss point (Sec. 2.2.2-2.2.4, App. C Alg. C1):
//   gather node coordinates / displacements of the element through LDS,
//   F = I + sum d_I (x) grad N_I, C - I, Jacobi eigen-decomposition,
//   eps = sum 1/2 ln(c_a) N_a (x) N_a, elastic predictor and Hill-48 return
//   map (always FP64), S = P_L : T, P = F S, and the Lagrangian tangent
//   C = P_L : Cep : P_L + T : L_L assembled in the eigenframe of C.
// The element residual and the 24x24 tangent
//   R^e_Ia  = sum_g w detJ0 P_aA dN_I/dX_A,
//   K^e_IaJb = sum_g w detJ0 dN_I/dX_A (delta_ab S_AB + F_aC C_CADB F_bD) dN_J/dX_B
// are formed per Gauss point in the eigenframe (g^ = Q^T grad N, f^ = F Q),
// summed over the 8 lanes of an element through LDS and stored, with
// coalesced stores, as the element's 24 residual entries and its 24x24
// tangent, row by row, in a workspace.
//
// Assembly (App. E, Alg. E1, without triplets or atomics): the owner of each
// node gathers, in ascending element order, the blocks of the elements
// around it and writes its three CSR rows (and residual entries) exactly
// once, applying the Dirichlet row elimination on the fly; the FP64 residual
// norm is reduced in two fixed-order stages.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "barlat.h"
#include "fem_device.h"
#include "fem_internal.h"

namespace fem {
namespace {

struct FwdArgs {
    int32_t n_nodes, n_elems;
    const double* X;
    const int32_t* conn;
    const double* prm[FEM_NPARAM];
    uint32_t pe_mask, ps_mask;
    uint32_t model;          // FEM_MODEL_* flags
    const double* orient;    // material orientation(s), or null
    int32_t orient_pe;       // orient holds one rotation per element
    const double* barlat;    // Yld2004-18p coefficients (Barlat variant)
    int32_t n_spec;
    const int64_t* elem_off;
    const double* d;
    const double* hist_n;
    double* Re;      // [n_elems][24] element residuals
    void* Ke;        // [n_elems][576] element tangent rows (RO), or null
    double* hist_np1;
    int32_t* diag;
    int64_t n_gp;
    int64_t n_tiles;
    int32_t xcd_remap;
    // mixed precision: elements with a Gauss point in the guard band are
    // appended here by the FP32 kernel and recomputed by the FP64 kernel
    int32_t* fix_list;
    int32_t* fix_count;
};

// specimen of element e (elem_off has n_spec + 1 prefix entries)
__device__ inline int spec_of(const int64_t* __restrict__ off, int n_spec, int64_t e) {
    int lo = 0, hi = n_spec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename A>
__device__ inline Mat load_material(const A& a, int64_t e) {
    int sp = 0;
    if (a.ps_mask) sp = spec_of(a.elem_off, a.n_spec, e);
    double v[FEM_NPARAM];
#pragma unroll
    for (int k = 0; k < FEM_NPARAM; ++k) {
        const int64_t idx = ((a.pe_mask >> k) & 1u) ? e : (((a.ps_mask >> k) & 1u) ? (int64_t)sp : 0);
        v[k] = a.prm[k][idx];
    }
    Mat m;
    m.E = v[0];
    m.nu = v[1];
    m.F = v[2];
    m.G = v[3];
    m.H = v[4];
    m.L = v[5];
    m.M = v[6];
    m.N = v[7];
    m.K = v[8];
    m.eps0 = v[9];
    m.nexp = v[10];
    m.voce = 0;  // set by the kernel from its variant
    return m;
}

// Compile-time element variants (bit flags): kVarOrient (a material
// orientation is given), kVarFbar (F-bar element), kVarVoce (Voce hardening).
// Variant 0 is the plain Swift / hex8 kernel.
constexpr int kVarOrient = 1;
constexpr int kVarFbar = 2;
constexpr int kVarVoce = 4;
constexpr int kVarBarlat = 8;  // FP64 kernel only (R = double)

// The element tangent is stored per element as its 9 component blocks
// K^e_{Ia,Jb}, (a, b) row-major, each an 8x8 node block, row-major: offset
// 64 (3a + b) + 8 I + J of the element's 576.  Both triangles are stored, so
// the assembly of node I's rows reads, for each block, 8 consecutive entries
// of row I per incident element (and no entry twice); the element kernel
// writes each block as 8 consecutive rows.  (Storing only the six blocks
// a <= b of a symmetric K^e was measured: the assembly then reads three
// blocks by columns, 8 sectors per row, and took 22 % longer in FP64 and
// 14 % longer in FP32 than it saved in bytes.)
constexpr int kKeStride = 576;
__host__ __device__ constexpr int pair_index(int a, int b) { return a * 3 - (a * (a - 1)) / 2 + (b - a); }
__host__ __device__ constexpr int pair_a(int p) { return p < 3 ? 0 : (p < 5 ? 1 : 2); }
__host__ __device__ constexpr int pair_b(int p) { return p < 3 ? p : (p < 5 ? p - 2 : 2); }
__host__ __device__ constexpr int ke_offset(int I, int a, int b, int J) { return 64 * (3 * a + b) + 8 * I + J; }
// slot of an off-diagonal pair (0,1), (0,2), (1,2) in the transpose hand-off
__host__ __device__ constexpr int offdiag_slot(int p) { return p == 1 ? 0 : (p == 2 ? 1 : 2); }

// Tile range of this workgroup in a persistent launch.  Workgroups are
// dispatched round-robin over the 8 XCDs; with xcd_remap the tiles are cut in
// 8 contiguous chunks and chunk x is walked by the workgroups of XCD x.
__device__ inline void tile_range(int64_t n_tiles, int remap, int64_t& first, int64_t& end, int64_t& step) {
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

// Everything one lane needs after the constitutive update, in working type R.
template <typename R>
struct GP {
    R g[8][3];   // grad N_I (physical)
    R detJ;
    R H[3][3];   // displacement gradient, F = I + H
    R Q[3][3];   // eigenvectors of C (columns)
    R mu[3];     // eigenvalues of C - I
    R eh[3];     // 1/2 ln c_a
};

// FBAR: the material sees Fbar = beta F (fbar_gradient); s.H becomes
// Fbar - I and beta, cw, jm1 = J - 1 are returned for the tangent.
template <typename R, bool FBAR, int W>
__device__ inline void kin_and_log(const double (*nd)[W], int gp, GP<R>& s, double eps[6], R& beta, R& cw, R& jm1) {
    kinematics_lds<R, W>(nd, gp, s.g, s.detJ, s.H);
    if constexpr (FBAR) fbar_gradient<R>(s.detJ, s.H, beta, cw, jm1);
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

// R: working type of kinematics, pull-back and contraction; RO: type of the
// stored element tangent blocks; FIXUP: walk the element list of the guard
// band instead of all elements (FP64 recomputation for the mixed path).
// The FP32 model variants are held to two waves per SIMD (the plain kernel
// fits there by itself).  The FP64 kernel runs one wave per SIMD: held to
// two (at most 256 registers, 20 KB of LDS, only Q parked across the local
// update) it spilled about 100 registers to scratch and took 10 % longer.
template <typename R, typename RO, int BLOCK, bool FIXUP, int VAR>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(std::is_same<R, float>::value && !FIXUP && VAR != 0 ? 2 : 1)))
void fwd_kernel(const FwdArgs a) {
    constexpr int EPB = BLOCK / 8;
    constexpr bool FLAG = std::is_same<R, float>::value && !FIXUP;
    constexpr bool ORIENT = (VAR & kVarOrient) != 0;
    constexpr bool FBAR = (VAR & kVarFbar) != 0;
    constexpr bool BARLAT = (VAR & kVarBarlat) != 0;
    static_assert(!BARLAT || std::is_same<R, double>::value, "the Barlat variant runs in FP64");
    // LDS: node coordinates and displacements of the tile; the frame
    // gradients g^ of every Gauss point; and one buffer used in turn for H
    // and Q (F-bar: and beta, cw) across the local update, the residual
    // reduction and the tangent hand-off (the 3 blocks A^ of one phase per
    // Gauss point; F-bar: first the element sums of the rank-one term).
    // Every per-lane row has an odd length (in values), so that the 64 lanes
    // of a wave, each at its own row, spread over the LDS banks (even
    // strides cost up to 16-way bank conflicts); a row read by the 8 lanes
    // of an element at once is a broadcast.  The Barlat kernel keeps even
    // node and hand-off rows: its LDS (with the parked Cep) must stay within
    // 40 KB for four workgroups per CU, worth more to it than the conflicts.
    constexpr int kHQ = FBAR ? 21 : 19;
    constexpr int kRed = 24 * (BLOCK + 1);
    constexpr int kHandW = BARLAT ? 28 : 29;
    constexpr int kXDW = BARLAT ? 6 : 7;
    constexpr int kHand = EPB * 8 * kHandW;
    constexpr int kPark = EPB * 8 * kHQ;
    constexpr int kBuf = kRed > kHand ? (kRed > kPark ? kRed : kPark) : (kHand > kPark ? kHand : kPark);
    __shared__ double sXD[EPB][8][kXDW];                       // [slot][node][X 3, d 3, pad]
    __shared__ __attribute__((aligned(16))) R sG[EPB][8][25];  // [slot][g][3 I + q] (+1 pad)
    __shared__ __attribute__((aligned(16))) R sbuf[kBuf];
    __shared__ int sFlag[EPB];
    __shared__ R sQb[FBAR ? EPB : 1][24];                      // F-bar: qbar of the element
    __shared__ double sCep[BARLAT ? EPB : 1][8][BARLAT ? 21 : 1];  // Barlat: Cep (upper triangle, material frame)
    R (*sHQ)[8][kHQ] = reinterpret_cast<R (*)[8][kHQ]>(sbuf);   // [slot][g][H 9, Q 9 (, beta, cw)]
    R (*red)[BLOCK + 1] = reinterpret_cast<R (*)[BLOCK + 1]>(sbuf);
    R (*sA)[8][kHandW] = reinterpret_cast<R (*)[8][kHandW]>(sbuf);  // [slot][g][9 k + 3 q + s]

    const int tid = threadIdx.x;
    const int slot = tid >> 3, gp = tid & 7;
    const bool want_K = a.Ke != nullptr;
    int32_t cnt_fail = 0, cnt_j0 = 0, cnt_jf = 0, cnt_nan = 0;

    int64_t t0, t1, ts;
    int64_t n_work = a.n_elems;
    if constexpr (FIXUP) {
        n_work = *a.fix_count;
        t0 = blockIdx.x;
        t1 = (n_work + EPB - 1) / EPB;
        ts = gridDim.x;
    } else {
        tile_range(a.n_tiles, a.xcd_remap, t0, t1, ts);
    }
    for (int64_t tile = t0; tile < t1; tile += ts) {
        const int64_t e_raw = tile * EPB + slot;
        const bool valid = e_raw < n_work;
        int64_t e;
        if constexpr (FIXUP) e = a.fix_list[valid ? e_raw : 0];
        else e = valid ? e_raw : (int64_t)a.n_elems - 1;
        const int64_t q = e * 8 + gp;
        if (FLAG && gp == 0) sFlag[slot] = 0;

        // ---- gather (own node through LDS); an out-of-range node id is
        // replaced by node 0 and counted, so no access leaves its buffer
        int32_t node = a.conn[q];
        if ((uint32_t)node >= (uint32_t)a.n_nodes) {
            if (valid) ++cnt_nan;
            node = 0;
        }
        sXD[slot][gp][0] = a.X[3 * (int64_t)node + 0];
        sXD[slot][gp][1] = a.X[3 * (int64_t)node + 1];
        sXD[slot][gp][2] = a.X[3 * (int64_t)node + 2];
        sXD[slot][gp][3] = a.d[3 * (int64_t)node + 0];
        sXD[slot][gp][4] = a.d[3 * (int64_t)node + 1];
        sXD[slot][gp][5] = a.d[3 * (int64_t)node + 2];
        double hn[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) hn[k] = a.hist_n[k * a.n_gp + q];
        Mat mat = load_material(a, e);
        mat.voce = (VAR & kVarVoce) ? 1 : 0;
        __syncthreads();

        // ---- kinematics, log strain (R), local update (double)
        GP<R> s;
        double eps[6];
        R fb_beta = R(1), fb_cw = R(0), fb_jm1 = R(0);
        kin_and_log<R, FBAR, kXDW>(sXD[slot], gp, s, eps, fb_beta, fb_cw, fb_jm1);
        if constexpr (FBAR) {
            // det F <= 0 is counted on F (s.H now holds Fbar - I)
            if (valid && !FIXUP) cnt_jf += (fb_jm1 <= R(-1)) ? 1 : 0;
            sHQ[slot][gp][18] = fb_beta;
            sHQ[slot][gp][19] = fb_cw;
        }
        // g^_Iq = grad N_IA Q_Aq, parked in LDS (read back by the residual and
        // the tangent hand-off; keeps registers free for the local update)
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
            // the local update runs in the material frame
            double Th[3][3];
            load_rotation(a.orient, oidx, Th);
            rotate_sym<true>(Th, eps, kSqrt2);
            rotate_sym<true>(Th, hn, 1.0);
        }
        Modes md;
        hill_modes(mat, md);
        Local loc;
        if constexpr (BARLAT) {
            BarlatCoef bco;
            load_barlat(a.barlat, bco);
            LocalB lb;
            local_update_barlat(eps, hn, mat, md, bco, lb, &sCep[slot][gp][0]);
#pragma unroll
            for (int k = 0; k < 6; ++k) loc.T[k] = lb.T[k];
#pragma unroll
            for (int k = 0; k < 7; ++k) loc.hist[k] = lb.hist[k];
            loc.plastic = lb.plastic;
            loc.converged = lb.converged;
            loc.ftr = lb.ftr;
            loc.sy_n = lb.sy_n;
        } else {
            local_update(eps, hn, mat, md, loc);
        }
        if constexpr (ORIENT) {
            double Th[3][3];
            load_rotation(a.orient, oidx, Th);
            rotate_sym<false>(Th, loc.T, kSqrt2);
            rotate_sym<false>(Th, loc.hist, 1.0);
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                s.H[i][j] = sHQ[slot][gp][3 * i + j];
                s.Q[i][j] = sHQ[slot][gp][9 + 3 * i + j];
            }
        if constexpr (FBAR) {
            fb_beta = sHQ[slot][gp][18];
            fb_cw = sHQ[slot][gp][19];
        }
        __syncthreads();  // the parking area becomes the residual buffer
        if constexpr (FLAG) {
            // guard band: a trial state this close to the yield surface is
            // left to the FP64 recomputation of its element, so that the
            // elastic/plastic decision and the stress are those of FP64
            if (valid && fabs(loc.ftr) < 2e-4 * loc.sy_n) sFlag[slot] = 1;
        }
        if (valid && !FIXUP) {
            cnt_fail += loc.converged ? 0 : 1;
            cnt_j0 += (s.detJ <= R(0)) ? 1 : 0;
            R F[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) F[i][j] = s.H[i][j] + ((i == j) ? R(1) : R(0));
            const R detF = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                           F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
            if constexpr (!FBAR) cnt_jf += (detF <= R(0)) ? 1 : 0;
        }
        if (valid && a.hist_np1) {
#pragma unroll
            for (int k = 0; k < 7; ++k) a.hist_np1[k * a.n_gp + q] = loc.hist[k];
        }

        // ---- pull-back in the eigenframe of C
        R Th[3][3];
        {
            R Tm[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) Tm[k] = (R)loc.T[k];
            mandel_to_frame<R>(s.Q, Tm, Th);
        }
        R f1[3][3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = p; r < 3; ++r) {
                const R v = (p == r) ? R(0.5) / (R(1) + s.mu[p]) : dd1<R>(s.mu[p], s.mu[r], s.eh[p], s.eh[r]);
                f1[p][r] = v;
                f1[r][p] = v;
            }
        R Sh[3][3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = 0; r < 3; ++r) Sh[p][r] = R(2) * f1[p][r] * Th[p][r];
        R fh[3][3];  // f^_ap = F_aC Q_Cp
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int p = 0; p < 3; ++p) fh[i][p] = s.Q[i][p] + (s.H[i][0] * s.Q[0][p] + s.H[i][1] * s.Q[1][p] + s.H[i][2] * s.Q[2][p]);
        const R wdet = s.detJ;

        // ---- residual: R_Ia = w detJ0 sum_q (f^ S^)_aq g^_Iq
        bool finite_gp = true;  // P (and the tangent) of this Gauss point finite
        {
            R Ph[3][3];
            bool fin = true;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    Ph[i][p] = wdet * (fh[i][0] * Sh[0][p] + fh[i][1] * Sh[1][p] + fh[i][2] * Sh[2][p]);
                    fin = fin && isfinite((double)Ph[i][p]);
                }
            finite_gp = fin;
#pragma unroll
            for (int I = 0; I < 8; ++I)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    red[3 * I + i][tid] = Ph[i][0] * sG[slot][gp][3 * I] + Ph[i][1] * sG[slot][gp][3 * I + 1] +
                                          Ph[i][2] * sG[slot][gp][3 * I + 2];
            __syncthreads();
            if (valid) {
                // lane gp owns node gp of the element: R^e_{gp,0..2}
                double* dst = a.Re + e * 24 + 3 * gp;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    R sum = R(0);
#pragma unroll
                    for (int g2 = 0; g2 < 8; ++g2) sum += red[3 * gp + i][slot * 8 + g2];
                    dst[i] = (double)sum;
                }
                if constexpr (FLAG) {
                    if (gp == 0 && sFlag[slot]) a.fix_list[atomicAdd(a.fix_count, 1)] = (int32_t)e;
                }
            }
            __syncthreads();
        }

        if (want_K) {
            // ---- Cep rotated to the eigenframe: E + sum coef_i b^_i b^_i^T - beta m^ m^^T
            R Ch[6][6];
            {
                const R lamL = (R)md.lam, mu2 = (R)md.mu2;
#pragma unroll
                for (int I = 0; I < 6; ++I)
#pragma unroll
                    for (int J = 0; J < 6; ++J) Ch[I][J] = ((I < 3 && J < 3) ? lamL : R(0)) + ((I == J) ? mu2 : R(0));
                if constexpr (BARLAT) {
                    // dense Cep (material frame) to the eigenframe of C: Ch = M Cep M^T,
                    // column k of M the eigenframe image of Mandel basis tensor k
                    R Qm[3][3];
                    if constexpr (ORIENT) material_frame<R>(a.orient, oidx, s.Q, Qm);
                    const R(*Qb)[3] = ORIENT ? Qm : s.Q;
                    R Mb[6][6];
                    const R u0[3] = {R(1), R(0), R(0)}, u1[3] = {R(0), R(1), R(0)}, u2[3] = {R(0), R(0), R(1)};
                    rot_diag<R>(Qb, u0, Mb[0]);
                    rot_diag<R>(Qb, u1, Mb[1]);
                    rot_diag<R>(Qb, u2, Mb[2]);
                    rot_shear<R, 1, 2>(Qb, Mb[3]);
                    rot_shear<R, 0, 2>(Qb, Mb[4]);
                    rot_shear<R, 0, 1>(Qb, Mb[5]);
                    R Cp[6][6];
                    {
                        int c = 0;
#pragma unroll
                        for (int i = 0; i < 6; ++i)
#pragma unroll
                            for (int j = i; j < 6; ++j) {
                                const R v = (R)sCep[slot][gp][c++];
                                Cp[i][j] = v;
                                Cp[j][i] = v;
                            }
                    }
                    R W[6][6];  // Cep M^T
#pragma unroll
                    for (int k = 0; k < 6; ++k)
#pragma unroll
                        for (int J = 0; J < 6; ++J) {
                            R x = R(0);
#pragma unroll
                            for (int l = 0; l < 6; ++l) x += Cp[k][l] * Mb[l][J];
                            W[k][J] = x;
                        }
#pragma unroll
                    for (int I = 0; I < 6; ++I)
#pragma unroll
                        for (int J = 0; J < 6; ++J) {
                            R x = R(0);
#pragma unroll
                            for (int k = 0; k < 6; ++k) x += Mb[k][I] * W[k][J];
                            Ch[I][J] = x;
                        }
                } else if (loc.plastic) {
                    // Hill eigen-basis (material frame) in the eigenframe of C
                    R Qm[3][3];
                    if constexpr (ORIENT) material_frame<R>(a.orient, oidx, s.Q, Qm);
                    const R(*Qb)[3] = ORIENT ? Qm : s.Q;
                    R B[5][6];
                    R v1[3] = {(R)md.v1[0], (R)md.v1[1], (R)md.v1[2]};
                    R v2[3] = {(R)md.v2[0], (R)md.v2[1], (R)md.v2[2]};
                    rot_diag<R>(Qb, v1, B[0]);
                    rot_diag<R>(Qb, v2, B[1]);
                    rot_shear<R, 1, 2>(Qb, B[2]);
                    rot_shear<R, 0, 2>(Qb, B[3]);
                    rot_shear<R, 0, 1>(Qb, B[4]);
                    R mh[6];
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        R v = R(0);
#pragma unroll
                        for (int i = 0; i < 5; ++i) v += (R)loc.mvec[i] * B[i][k];
                        mh[k] = v;
                    }
                    const R beta = (R)loc.beta;
#pragma unroll
                    for (int I = 0; I < 6; ++I)
#pragma unroll
                        for (int J = I; J < 6; ++J) {
                            R v = -beta * mh[I] * mh[J];
#pragma unroll
                            for (int i = 0; i < 5; ++i) v += (R)loc.coef[i] * B[i][I] * B[i][J];
                            Ch[I][J] += v;
                            if (J != I) Ch[J][I] += v;
                        }
                }
            }
            // ---- second divided differences f2(c_a, c_b, c_r)
            R f2[3][3][3];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const R cp = R(1) + s.mu[p];
                f2[p][p][p] = R(-0.25) / (cp * cp);
            }
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    if (r != p) {
                        const R v = dd2_pair<R>(s.mu[p], s.mu[r], s.eh[p], s.eh[r]);
                        f2[p][p][r] = f2[p][r][p] = f2[r][p][p] = v;
                    }
            {
                const R v = dd2_triple<R>(s.mu[0], s.mu[1], s.mu[2], s.eh[0], s.eh[1], s.eh[2]);
                f2[0][1][2] = f2[0][2][1] = f2[1][0][2] = f2[1][2][0] = f2[2][0][1] = f2[2][1][0] = v;
            }
            // ---- Lagrangian tangent (Mandel, eigenframe):
            //      Cm = P^ Ch P^ + L,  P^_I = 2 f1(I),  (L:dC)_ab = 4 sum_r f2_abr (dC_ar T_rb + T_ar dC_rb)
            R Cm[6][6];
#pragma unroll
            for (int J = 0; J < 6; ++J) {
                const int c = mi(J), d = mj(J);
                const R ev = (c == d) ? R(1) : R(kInvSqrt2);
#pragma unroll
                for (int I = 0; I <= J; ++I) {
                    const int p = mi(I), r = mj(I);
                    // L(E_J)_pr with E_J = ev (e_c e_d + e_d e_c) (or e_c e_c)
                    R x = R(0);
#pragma unroll
                    for (int t = 0; t < 3; ++t) {
                        R Ept = R(0), Etr = R(0);
                        if ((p == c && t == d) || (p == d && t == c)) Ept = ev;
                        if ((t == c && r == d) || (t == d && r == c)) Etr = ev;
                        if (c == d) {
                            Ept = (p == c && t == c) ? R(1) : R(0);
                            Etr = (t == c && r == c) ? R(1) : R(0);
                        }
                        x += f2[p][r][t] * (Ept * Th[t][r] + Th[p][t] * Etr);
                    }
                    const R Pi = R(2) * f1[p][r], Pj = R(2) * f1[c][d];
                    Cm[I][J] = Pi * Ch[I][J] * Pj + R(4) * mw<R>(I) * x;
                    Cm[J][I] = Cm[I][J];  // the tangent is symmetric
                }
            }
            bool fin = true;
#pragma unroll
            for (int I = 0; I < 6; ++I) fin = fin && isfinite((double)Cm[I][I]);
            finite_gp = finite_gp && fin;
            // tensor components C4(p,q,r,s) = Cm[I][J] / (w_I w_J) (Mandel weights)
            R C4[6][6];
#pragma unroll
            for (int I = 0; I < 6; ++I)
#pragma unroll
                for (int J = I; J < 6; ++J) {
                    constexpr R h = R(0.5), r2 = R(kInvSqrt2);
                    const R sc = (I < 3 && J < 3) ? R(1) : ((I < 3 || J < 3) ? r2 : h);
                    C4[I][J] = C4[J][I] = (I < 3 && J < 3) ? Cm[I][J] : sc * Cm[I][J];
                }

            if constexpr (FBAR) {
            // ---- F-bar tangent, all 9 blocks (not symmetric):
            //   K^e_{Ia,Jb} = sum_g g^_Iq A~(a,b)_qs g^_Js + Ubar_Ia qbar_Jb
            //   A~(a,b)_qs = beta w detJ0 (A^(a,b)_qs - Y^_aq (f^_bs / c_s) / 3)
            // in the eigenframe of Cbar (c_s its eigenvalues), with
            //   Y^ = f^ (S^ + (C:Cbar)^)      (Abar : Fbar = Fbar S + Fbar (C : Cbar)),
            //   Ubar_Ia = sum_g w detJ0 / 3 Y^_ap g^_Ip,
            //   qbar_Jb = sum_g cw beta g^_Js f^_bs / c_s   (= dJbar/dd_Jb / Jbar);
            // the A~ part carries d(Fbar)/dd at fixed Jbar and the per-point
            // -dJ/J term, Ubar qbar the element's dJbar/Jbar term.
            const R wK = wdet * fb_beta;
            R Yh[3][3], fc[3][3];
            {
                R Wc[6];
#pragma unroll
                for (int I = 0; I < 6; ++I)
                    Wc[I] = Cm[I][0] * (R(1) + s.mu[0]) + Cm[I][1] * (R(1) + s.mu[1]) + Cm[I][2] * (R(1) + s.mu[2]);
                const R r2 = R(kInvSqrt2);
                const R Wm[3][3] = {{Wc[0], Wc[5] * r2, Wc[4] * r2}, {Wc[5] * r2, Wc[1], Wc[3] * r2},
                                    {Wc[4] * r2, Wc[3] * r2, Wc[2]}};
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        Yh[i][p] = fh[i][0] * (Sh[0][p] + Wm[0][p]) + fh[i][1] * (Sh[1][p] + Wm[1][p]) +
                                   fh[i][2] * (Sh[2][p] + Wm[2][p]);
                        fc[i][p] = fh[i][p] / (R(1) + s.mu[p]);
                    }
            }
            // element sums Ubar (row gp) and qbar through the hand-off area, in
            // Gauss point order
            R (*sU)[8][25] = reinterpret_cast<R (*)[8][25]>(sbuf);
            {
                const R w3 = wdet * R(1.0 / 3.0);
#pragma unroll
                for (int I = 0; I < 8; ++I)
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        sU[slot][gp][3 * I + i] = w3 * (Yh[i][0] * sG[slot][gp][3 * I] + Yh[i][1] * sG[slot][gp][3 * I + 1] +
                                                         Yh[i][2] * sG[slot][gp][3 * I + 2]);
            }
            __syncthreads();
            R ub[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                R x = R(0);
#pragma unroll
                for (int g = 0; g < 8; ++g) x += sU[slot][g][3 * gp + i];
                ub[i] = x;
            }
            __syncthreads();
            {
                const R cb = fb_cw * fb_beta;
#pragma unroll
                for (int J = 0; J < 8; ++J)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        sU[slot][gp][3 * J + b] = cb * (sG[slot][gp][3 * J] * fc[b][0] + sG[slot][gp][3 * J + 1] * fc[b][1] +
                                                        sG[slot][gp][3 * J + 2] * fc[b][2]);
            }
            __syncthreads();
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                R x = R(0);
#pragma unroll
                for (int g = 0; g < 8; ++g) x += sU[slot][g][3 * gp + b];
                sQb[slot][3 * gp + b] = x;
            }
            __syncthreads();
            // three phases: blocks (a, 0), (a, 1), (a, 2) for a = 0, 1, 2
            static_for<0, 3>([&](auto AA) {
                constexpr int aa = decltype(AA)::value;
                R Y[3][3][3];
#pragma unroll
                for (int qq = 0; qq < 3; ++qq)
#pragma unroll
                    for (int r = 0; r < 3; ++r)
#pragma unroll
                        for (int ss = 0; ss < 3; ++ss) {
                            const int J = midx(r, ss);
                            R v = fh[aa][0] * C4[midx(0, qq)][J];
                            v = m_fma(fh[aa][1], C4[midx(1, qq)][J], v);
                            Y[qq][r][ss] = m_fma(fh[aa][2], C4[midx(2, qq)][J], v);
                        }
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                    for (int qq = 0; qq < 3; ++qq)
#pragma unroll
                        for (int ss = 0; ss < 3; ++ss) {
                            R v = fh[bb][0] * Y[qq][0][ss] + fh[bb][1] * Y[qq][1][ss] + fh[bb][2] * Y[qq][2][ss];
                            if (aa == bb) v += Sh[qq][ss];
                            v -= R(1.0 / 3.0) * Yh[aa][qq] * fc[bb][ss];
                            sA[slot][gp][9 * bb + 3 * qq + ss] = wK * v;
                        }
                __syncthreads();
                R acc[3][8];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int J = 0; J < 8; ++J) acc[k][J] = R(0);
#pragma unroll 2
                for (int g = 0; g < 8; ++g) {
                    R G[24], A[28], gi[3];
#pragma unroll
                    for (int t = 0; t < 24; ++t) G[t] = sG[slot][g][t];
#pragma unroll
                    for (int t = 0; t < 28; ++t) A[t] = sA[slot][g][t];
#pragma unroll
                    for (int q = 0; q < 3; ++q) gi[q] = sG[slot][g][3 * gp + q];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        R t3[3];
#pragma unroll
                        for (int ss = 0; ss < 3; ++ss)
                            t3[ss] = m_fma(gi[2], A[9 * k + 6 + ss], m_fma(gi[1], A[9 * k + 3 + ss], gi[0] * A[9 * k + ss]));
#pragma unroll
                        for (int J = 0; J < 8; ++J) {
                            R v = m_fma(t3[0], G[3 * J], acc[k][J]);
                            v = m_fma(t3[1], G[3 * J + 1], v);
                            acc[k][J] = m_fma(t3[2], G[3 * J + 2], v);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int J = 0; J < 8; ++J) acc[k][J] = m_fma(ub[aa], sQb[slot][3 * J + k], acc[k][J]);
                if (valid) {
                    RO* Kd = reinterpret_cast<RO*>(a.Ke) + e * kKeStride;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        RO* row = Kd + ke_offset(gp, aa, k, 0);
                        RO v4[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) v4[j] = (RO)acc[k][j];
                        store4<RO>(row, v4);
#pragma unroll
                        for (int j = 0; j < 4; ++j) v4[j] = (RO)acc[k][4 + j];
                        store4<RO>(row + 4, v4);
                    }
                }
                __syncthreads();
            });
            } else {
            // ---- element tangent blocks K^e(a,b), a <= b:
            //      K^e_{Ia,Jb} = sum_g w detJ0 g^_Iq A^(a,b)_qs g^_Js  (per Gauss point g)
            // Each lane hands its g^ and A^ over through LDS, then lane I
            // sums row I of the blocks over the element's 8 Gauss points, in
            // order.  Two phases of 3 blocks: (0,0),(0,1),(0,2); (1,1),(1,2),(2,2).
            R keep[3][8];  // rows I of the blocks (0,1), (0,2), (1,2)
            static_for<0, 2>([&](auto PH) {
                constexpr int ph = decltype(PH)::value;
                static_for<ph, ph + 1 + ph>([&](auto AA) {
                    constexpr int aa = decltype(AA)::value;
                    // Y[q][r][s] = sum_p f^_ap C4(p,q,r,s), C4 = the tensor components of Cm
                    R Y[3][3][3];
#pragma unroll
                    for (int qq = 0; qq < 3; ++qq)
#pragma unroll
                        for (int r = 0; r < 3; ++r)
#pragma unroll
                            for (int ss = 0; ss < 3; ++ss) {
                                const int J = midx(r, ss);
                                R v = fh[aa][0] * C4[midx(0, qq)][J];
                                v = m_fma(fh[aa][1], C4[midx(1, qq)][J], v);
                                Y[qq][r][ss] = m_fma(fh[aa][2], C4[midx(2, qq)][J], v);
                            }
                    static_for<aa, 3>([&](auto BB) {
                        constexpr int bb = decltype(BB)::value;
                        constexpr int k = pair_index(aa, bb) - 3 * ph;
#pragma unroll
                        for (int qq = 0; qq < 3; ++qq)
#pragma unroll
                            for (int ss = 0; ss < 3; ++ss) {
                                R v = fh[bb][0] * Y[qq][0][ss] + fh[bb][1] * Y[qq][1][ss] + fh[bb][2] * Y[qq][2][ss];
                                if (aa == bb) v += Sh[qq][ss];
                                sA[slot][gp][9 * k + 3 * qq + ss] = wdet * v;
                            }
                    });
                });
                __syncthreads();
                // lane gp = row I
                R acc[3][8];
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int J = 0; J < 8; ++J) acc[k][J] = R(0);
#pragma unroll 2
                for (int g = 0; g < 8; ++g) {
                    R G[24], A[28], gi[3];
#pragma unroll
                    for (int t = 0; t < 24; ++t) G[t] = sG[slot][g][t];
#pragma unroll
                    for (int t = 0; t < 28; ++t) A[t] = sA[slot][g][t];
#pragma unroll
                    for (int q = 0; q < 3; ++q) gi[q] = sG[slot][g][3 * gp + q];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        R t3[3];
#pragma unroll
                        for (int ss = 0; ss < 3; ++ss)
                            t3[ss] = m_fma(gi[2], A[9 * k + 6 + ss], m_fma(gi[1], A[9 * k + 3 + ss], gi[0] * A[9 * k + ss]));
#pragma unroll
                        for (int J = 0; J < 8; ++J) {
                            R v = m_fma(t3[0], G[3 * J], acc[k][J]);
                            v = m_fma(t3[1], G[3 * J + 1], v);
                            acc[k][J] = m_fma(t3[2], G[3 * J + 2], v);
                        }
                    }
                }
                if (valid) {
                    // row I = gp of the blocks (a, b), a <= b, p = 3 ph + k
                    RO* Kd = reinterpret_cast<RO*>(a.Ke) + e * kKeStride;
                    static_for<0, 3>([&](auto KK) {
                        constexpr int k = decltype(KK)::value;
                        constexpr int p = 3 * ph + k;
                        RO* row = Kd + ke_offset(gp, pair_a(p), pair_b(p), 0);
                        RO v4[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) v4[j] = (RO)acc[k][j];
                        store4<RO>(row, v4);
#pragma unroll
                        for (int j = 0; j < 4; ++j) v4[j] = (RO)acc[k][4 + j];
                        store4<RO>(row + 4, v4);
                    });
                }
                // the off-diagonal rows are kept for the transpose below
                static_for<0, 3>([&](auto KK) {
                    constexpr int k = decltype(KK)::value;
                    constexpr int p = 3 * ph + k;
                    if constexpr (pair_a(p) != pair_b(p)) {
#pragma unroll
                        for (int J = 0; J < 8; ++J) keep[offdiag_slot(p)][J] = acc[k][J];
                    }
                });
                __syncthreads();
            });
            // blocks (b, a), a < b: row I of (b, a) is column I of (a, b),
            // handed over through the hand-off area (free after the two phases)
            R* tt = &sA[slot][0][0];  // [3][8 I][9] (216 <= 8 x 28 values)
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int J = 0; J < 8; ++J) tt[72 * t + 9 * gp + J] = keep[t][J];
            __syncthreads();
            if (valid) {
                RO* Kd = reinterpret_cast<RO*>(a.Ke) + e * kKeStride;
                static_for<0, 3>([&](auto TT) {
                    constexpr int t = decltype(TT)::value;
                    constexpr int p = t == 0 ? 1 : (t == 1 ? 2 : 4);
                    RO* row = Kd + ke_offset(gp, pair_b(p), pair_a(p), 0);
                    RO v4[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) v4[j] = (RO)tt[72 * t + 9 * j + gp];
                    store4<RO>(row, v4);
#pragma unroll
                    for (int j = 0; j < 4; ++j) v4[j] = (RO)tt[72 * t + 9 * (4 + j) + gp];
                    store4<RO>(row + 4, v4);
                });
            }
            }  // F-bar / symmetric tangent
        }
        if (valid && !finite_gp && !FIXUP) ++cnt_nan;
        __syncthreads();
    }
    if (a.diag && !FIXUP) {
        if (cnt_fail) atomicAdd(a.diag + 0, cnt_fail);
        if (cnt_j0) atomicAdd(a.diag + 1, cnt_j0);
        if (cnt_jf) atomicAdd(a.diag + 2, cnt_jf);
        if (cnt_nan) atomicAdd(a.diag + 3, cnt_nan);
    }
}

// ---- row-owner assembly


// R_I = sum of R^e_i over the elements around node I; 8 lanes per node, lane
// k taking incident elements k, k+8, ... in ascending order, then a fixed
// butterfly over the 8 lanes (bitwise reproducible).  Dirichlet dofs are
// zeroed; per-workgroup partial sums of R^2 go to `part` for the norm.
// Workgroups are mapped to 8 contiguous node ranges, one per XCD.
constexpr int kResThreads = 256;  // 32 nodes per workgroup
__global__ __launch_bounds__(kResThreads) void assemble_residual(
    int32_t n_nodes, int64_t n_chunk, const int32_t* __restrict__ ne_ptr, const int32_t* __restrict__ ne_list,
    const double* __restrict__ Re, const uint8_t* __restrict__ bc, double* __restrict__ Rv,
    double* __restrict__ part) {
    __shared__ double sh[kResThreads];
    const int64_t grp = (int64_t)(blockIdx.x & 7) * n_chunk + (blockIdx.x >> 3);
    const int64_t n = grp * (kResThreads / 8) + (threadIdx.x >> 3);
    const int k = (int)(threadIdx.x & 7);
    double acc[3] = {0.0, 0.0, 0.0};
    if (n < n_nodes) {
        const int32_t k1 = ne_ptr[n + 1];
        for (int32_t c = ne_ptr[n] + k; c < k1; c += 8) {
            const int64_t v = ne_list[c];  // 8 e + i
            const double* src = Re + (v >> 3) * 24 + 3 * (v & 7);
            acc[0] += src[0];
            acc[1] += src[1];
            acc[2] += src[2];
        }
    }
#pragma unroll
    for (int m = 1; m < 8; m <<= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], m, 8);
    double sq = 0.0;
    if (n < n_nodes && k < 3) {
        const int64_t dof = 3 * n + k;
        const double val = (bc && bc[dof]) ? 0.0 : (k == 0 ? acc[0] : (k == 1 ? acc[1] : acc[2]));
        Rv[dof] = val;
        sq = val * val;
    }
    if (part) {
        sh[threadIdx.x] = sq;
        __syncthreads();
        for (int off = kResThreads / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
    }
}

// Orders a wave's LDS stores before loads of the same addresses by other
// lanes of that wave.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kTanWaves = 4;  // nodes (waves) per workgroup of assemble_tangent
constexpr int kSlot = 12;     // LDS slot of a parked 3x3 block (padded for 16-byte reads)

// Rows 3I+a of K, one wave per node I.  The node's incident elements are
// taken 8 at a time: lane (k, j) loads the 3x3 block (i_k, j) of element k
// (i_k = local index of I in it; per load, the 8 lanes of an element read 8
// consecutive entries of row i_k of one component block) and parks it in
// LDS, and records j in a table at [r][k], r = elem_rank of node j in
// element k (the column block of node j in row I).  Lane r, owner of column
// block r (the r-th neighbour J of I in ascending order), then reads its 8
// table entries at once and adds the parked blocks they name, in ascending
// element order.  The node's 3 rows are 9 deg consecutive values of K; they
// are staged in LDS and stored by all 64 lanes, constrained rows replaced by
// identity rows.  Every entry of K is written exactly once.  Workgroups are
// mapped to 8 contiguous node ranges, one per XCD, so the elements shared by
// neighbouring nodes are re-read from the same L2.
template <typename R>
__global__ __launch_bounds__(64 * kTanWaves) void assemble_tangent(
    int32_t n_nodes, int64_t n_chunk, const int32_t* __restrict__ ne_ptr, const int32_t* __restrict__ ne_list,
    const uint8_t* __restrict__ elem_rank, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
    const R* __restrict__ Ke, const uint8_t* __restrict__ bc, R* __restrict__ K) {
    __shared__ __attribute__((aligned(16))) R sv[kTanWaves][64 * kSlot];
    __shared__ uint64_t stab[kTanWaves][64];  // [r]: byte k = j of element k with rank r, 0xff if none
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t grp = (int64_t)(blockIdx.x & 7) * n_chunk + (blockIdx.x >> 3);
    const int64_t n = grp * kTanWaves + w;
    if (n >= n_nodes) return;  // the whole wave; no workgroup barrier below
    R* vals = sv[w];
    uint8_t* tab = reinterpret_cast<uint8_t*>(stab[w]);
    const int32_t rs = row_ptr[3 * n];
    const int32_t len = row_ptr[3 * n + 1] - rs;  // 3 deg
    const int deg = len / 3;
    const int32_t k0 = ne_ptr[n], k1 = ne_ptr[n + 1];
    // constrained rows of the node (bit a: row 3n + a), fetched up front
    uint32_t bcm = 0;
    if (bc) bcm = (bc[3 * n] ? 1u : 0u) | (bc[3 * n + 1] ? 2u : 0u) | (bc[3 * n + 2] ? 4u : 0u);
    const int kk = lane >> 3, j = lane & 7;
    R acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = R(0);
    for (int32_t c = k0; c < k1; c += 8) {
        stab[w][lane] = ~0ull;
        wave_sync();
        if (c + kk < k1) {
            const int64_t v = ne_list[c + kk];  // 8 e + i
            const int i = (int)(v & 7);
            const R* row = Ke + (v >> 3) * kKeStride + ke_offset(i, 0, 0, j);
            R* dst = vals + lane * kSlot;
#pragma unroll
            for (int ab = 0; ab < 9; ++ab) dst[ab] = row[64 * ab];
            tab[8 * elem_rank[8 * v + j] + kk] = (uint8_t)j;
        }
        wave_sync();
        if (lane < deg) {
            const int nk = min(8, k1 - c);
            const uint64_t word = stab[w][lane];
            for (int q = 0; q < nk; ++q) {
                const uint32_t jj = (uint32_t)(word >> (8 * q)) & 0xffu;
                if (jj != 0xffu) {
                    const R* src = vals + (q * 8 + (int)jj) * kSlot;
#pragma unroll
                    for (int t = 0; t < 9; ++t) acc[t] += src[t];
                }
            }
        }
        wave_sync();
    }
    if (lane < deg) {
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) vals[aa * len + 3 * lane + bb] = acc[aa * 3 + bb];
    }
    wave_sync();
    R* __restrict__ Kn = K + rs;  // the node's 3 rows, wave-uniform base
    const int tot = 3 * len;
    if (bcm == 0) {
        for (int t = lane; t < tot; t += 64) Kn[t] = vals[t];
    } else {
        const int32_t* __restrict__ cn = col_idx + rs;
        for (int t = lane; t < tot; t += 64) {
            const int aa = (t >= len) + (t >= 2 * len);
            R val = vals[t];
            if ((bcm >> aa) & 1u) val = (cn[t] == 3 * n + aa) ? R(1) : R(0);
            Kn[t] = val;
        }
    }
}

// ||R||^2 = sum of the residual workgroups' partial sums: each thread adds a
// fixed strided subset (4 independent chains), then a fixed tree.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void norm_final(const double* __restrict__ part, int nb,
                                                         double* __restrict__ out) {
    __shared__ double sh[kFinThreads];
    const int t = (int)threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = t;
    for (; i + 3 * kFinThreads < nb; i += 4 * kFinThreads) {
        s0 += part[i];
        s1 += part[i + kFinThreads];
        s2 += part[i + 2 * kFinThreads];
        s3 += part[i + 3 * kFinThreads];
    }
    for (; i < nb; i += kFinThreads) s0 += part[i];
    sh[t] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int off = kFinThreads / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    if (t == 0) out[0] = sh[0];
}

template <typename R, typename RO, int BLOCK, bool FIXUP, int VAR>
hipError_t launch_fwd(const FwdArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((fwd_kernel<R, RO, BLOCK, FIXUP, VAR>), dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// element variant of a call
inline int variant_of(const FwdArgs& a) {
    return (a.orient ? kVarOrient : 0) | ((a.model & FEM_MODEL_FBAR) ? kVarFbar : 0) |
           ((a.model & FEM_MODEL_VOCE) ? kVarVoce : 0) | ((a.model & FEM_MODEL_BARLAT) ? kVarBarlat : 0);
}

// Variant 0 in every tuned workgroup size; the model variants with 64 threads.
// Barlat variants: FP64 element kernel, K stored in the call's type RO
template <typename RO>
hipError_t launch_fwd_barlat(const FwdArgs& a, int grid, hipStream_t s) {
    switch (variant_of(a) & ~kVarBarlat) {
        case 0: return launch_fwd<double, RO, 64, false, 8>(a, grid, s);
        case 1: return launch_fwd<double, RO, 64, false, 9>(a, grid, s);
        case 2: return launch_fwd<double, RO, 64, false, 10>(a, grid, s);
        case 3: return launch_fwd<double, RO, 64, false, 11>(a, grid, s);
        case 4: return launch_fwd<double, RO, 64, false, 12>(a, grid, s);
        case 5: return launch_fwd<double, RO, 64, false, 13>(a, grid, s);
        case 6: return launch_fwd<double, RO, 64, false, 14>(a, grid, s);
        default: return launch_fwd<double, RO, 64, false, 15>(a, grid, s);
    }
}

template <typename R, typename RO, bool FIXUP>
hipError_t launch_fwd_variant(const FwdArgs& a, int block, int grid, hipStream_t s) {
    if (variant_of(a) & kVarBarlat) {
        if constexpr (FIXUP) return hipSuccess;  // no guard band: the Barlat kernel is FP64
        else return launch_fwd_barlat<RO>(a, grid, s);
    }
    switch (variant_of(a)) {
        case 0:
            if (FIXUP || block == 64) return launch_fwd<R, RO, 64, FIXUP, 0>(a, grid, s);
            if (block == 256) return launch_fwd<R, RO, 256, FIXUP, 0>(a, grid, s);
            return launch_fwd<R, RO, 128, FIXUP, 0>(a, grid, s);
        case 1: return launch_fwd<R, RO, 64, FIXUP, 1>(a, grid, s);
        case 2: return launch_fwd<R, RO, 64, FIXUP, 2>(a, grid, s);
        case 3: return launch_fwd<R, RO, 64, FIXUP, 3>(a, grid, s);
        case 4: return launch_fwd<R, RO, 64, FIXUP, 4>(a, grid, s);
        case 5: return launch_fwd<R, RO, 64, FIXUP, 5>(a, grid, s);
        case 6: return launch_fwd<R, RO, 64, FIXUP, 6>(a, grid, s);
        default: return launch_fwd<R, RO, 64, FIXUP, 7>(a, grid, s);
    }
}

template <typename R>
hipError_t launch_fwd_main(const FwdArgs& a, int block, int grid, hipStream_t s) {
    return launch_fwd_variant<R, R, false>(a, block, grid, s);
}

hipError_t launch_fixup(const FwdArgs& a, int grid, hipStream_t s);

// FP64 recomputation of the guard-band elements of a mixed pass
constexpr int kFixBlock = 64;
constexpr int kFixGrid = 1024;

hipError_t launch_fixup(const FwdArgs& a, int grid, hipStream_t s) {
    return launch_fwd_variant<double, float, true>(a, kFixBlock, grid, s);
}

// Workgroups of assemble_residual (= partial sums of the norm) for n nodes.
inline int64_t residual_blocks(int64_t n_nodes) {
    const int64_t n_chunk = ((n_nodes + kResThreads / 8 - 1) / (kResThreads / 8) + 7) / 8;
    return 8 * n_chunk;
}

struct FwdWs {
    double* Re;
    void* Ke;
    double* part;
    int32_t* fix_list;
    int32_t* fix_count;
};

template <typename C>
void carve_forward(C& c, int32_t n_nodes, int32_t n_elems, fem_precision prec, FwdWs* w) {
    const size_t kb = (prec == FEM_FP64) ? sizeof(double) : sizeof(float);
    auto re = c.template take<double>((size_t)n_elems * 24 + 1);
    auto ke = c.template take<char>((size_t)n_elems * kKeStride * kb + 16);
    auto pa = c.template take<double>((size_t)residual_blocks(n_nodes) + 1);
    auto fl = c.template take<int32_t>(prec == FEM_FP32_MIXED ? (size_t)n_elems + 1 : 1);
    auto fc = c.template take<int32_t>(4);
    if (w) *w = FwdWs{re, (void*)ke, pa, fl, fc};
}

struct CountAdapterF {
    WsCounter cnt;
    template <typename T>
    T* take(size_t n) {
        cnt.take<T>(n);
        return nullptr;
    }
};

}  // namespace

hipError_t gather_node_vectors(int32_t n_nodes, const int32_t* ne_ptr, const int32_t* ne_list, const double* Re,
                               double* out, hipStream_t s) {
    if (n_nodes <= 0) return hipSuccess;
    const int64_t nb = residual_blocks(n_nodes), n_chunk = nb / 8;
    hipLaunchKernelGGL(assemble_residual, dim3((unsigned)nb), dim3(kResThreads), 0, s, n_nodes, n_chunk, ne_ptr,
                       ne_list, Re, (const uint8_t*)nullptr, out, (double*)nullptr);
    return hipGetLastError();
}

}  // namespace fem

using namespace fem;

extern "C" size_t fem_forward_workspace_bytes(int32_t n_nodes, int32_t n_elems, fem_precision prec) {
    if (n_nodes < 0 || n_elems < 0) return 0;
    CountAdapterF c;
    carve_forward(c, n_nodes, n_elems, prec, (FwdWs*)nullptr);
    return c.cnt.used + 256;
}

extern "C" int fem_residual_tangent(const fem_mesh* mesh, const fem_batch* batch, const fem_csr* csr,
                                    const fem_params* params, const double* d, const double* hist_n,
                                    const uint8_t* bc_mask, fem_precision prec, double* R, void* K_vals,
                                    double* hist_np1, double* rnorm2, int32_t* diag, void* ws, size_t ws_bytes,
                                    void* stream) {
    clear_error();
    if (!mesh || !params) return set_error(FEM_EINVAL, "fem_residual_tangent: mesh and params must not be NULL");
    if (mesh->n_nodes < 0 || mesh->n_elems < 0) return set_error(FEM_EINVAL, "fem_residual_tangent: negative sizes");
    if (prec != FEM_FP64 && prec != FEM_FP32_MIXED && prec != FEM_FP64_K32)
        return set_error(FEM_EINVAL, "fem_residual_tangent: unknown precision %d", (int)prec);
    const int64_t ne = mesh->n_elems, n_dof = 3 * (int64_t)mesh->n_nodes;
    if (rnorm2 && !R && n_dof > 0) return set_error(FEM_EINVAL, "fem_residual_tangent: rnorm2 requires R");
    if (ne > 0 && (!mesh->X || !mesh->conn || !d || !hist_n))
        return set_error(FEM_EINVAL, "fem_residual_tangent: X, conn, d and hist_n must not be NULL");
    const bool assemble = (R || K_vals) && n_dof > 0;
    if (assemble && (!csr || !csr->row_ptr || !csr->node_elem_ptr || !csr->node_elem))
        return set_error(FEM_EINVAL, "fem_residual_tangent: assembly needs csr row_ptr and the node incidence");
    if (K_vals && (!csr->col_idx || !csr->elem_rank))
        return set_error(FEM_EINVAL, "fem_residual_tangent: K_vals requires a complete CSR pattern");
    if (assemble && csr->n_rows != n_dof)
        return set_error(FEM_EINVAL, "fem_residual_tangent: csr->n_rows = %d, expected %lld", csr->n_rows,
                         (long long)n_dof);
    for (int k = 0; k < FEM_NPARAM; ++k)
        if (!params->p[k]) return set_error(FEM_EINVAL, "fem_residual_tangent: parameter %d is NULL", k);
    if (params->per_spec_mask && (!batch || batch->n_spec < 1 || !batch->elem_off))
        return set_error(FEM_EINVAL, "fem_residual_tangent: per-specimen parameters need a batch");
    if (params->model & ~(uint32_t)(FEM_MODEL_VOCE | FEM_MODEL_FBAR | FEM_MODEL_BARLAT))
        return set_error(FEM_EINVAL, "fem_residual_tangent: unknown model flags 0x%x", params->model);
    if ((params->model & FEM_MODEL_BARLAT) && !params->barlat)
        return set_error(FEM_EINVAL, "fem_residual_tangent: FEM_MODEL_BARLAT needs the coefficients");
    if (batch && (batch->n_spec < 1 || !batch->elem_off))
        return set_error(FEM_EINVAL, "fem_residual_tangent: invalid batch");
    const size_t need = fem_forward_workspace_bytes(mesh->n_nodes, mesh->n_elems, prec);
    if (!ws || ws_bytes < need)
        return set_error(FEM_ENOMEM, "fem_residual_tangent: workspace of %zu bytes required, %zu given", need,
                         ws_bytes);
    hipStream_t s = (hipStream_t)stream;
    WsCarver cv(ws, ws_bytes);
    FwdWs w;
    carve_forward(cv, mesh->n_nodes, mesh->n_elems, prec, &w);
    // diag, and the guard-band counter of a mixed pass, start at zero
    FEM_HIP_CHECK(zero_counters(diag, 4, (ne > 0 && prec == FEM_FP32_MIXED) ? w.fix_count : nullptr, 1, s));

    if (ne > 0) {
        fem_launch cfg = launch_config(FEM_KERNEL_FORWARD, prec == FEM_FP32_MIXED ? FEM_FP32_MIXED : FEM_FP64);
        if (params->model || params->orient) cfg.block = 64;  // model variants: 64-thread workgroups
        FwdArgs a;
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
        a.barlat = params->barlat;
        a.n_spec = batch ? batch->n_spec : 1;
        a.elem_off = batch ? batch->elem_off : nullptr;
        a.d = d;
        a.hist_n = hist_n;
        a.Re = w.Re;
        a.Ke = K_vals ? w.Ke : nullptr;
        a.hist_np1 = hist_np1;
        a.diag = diag;
        a.n_gp = 8 * ne;
        const int epb = cfg.block / 8;
        a.n_tiles = (ne + epb - 1) / epb;
        a.xcd_remap = cfg.xcd_remap;
        a.fix_list = w.fix_list;
        a.fix_count = w.fix_count;
        const int grid = persistent_grid(cfg, a.n_tiles);
        void* tk = timing_begin(s);
        hipError_t e = (prec == FEM_FP64)        ? launch_fwd_main<double>(a, cfg.block, grid, s)
                       : (prec == FEM_FP64_K32) ? launch_fwd_variant<double, float, false>(a, cfg.block, grid, s)
                                                : launch_fwd_main<float>(a, cfg.block, grid, s);
        timing_end(tk, FEM_KERNEL_FORWARD, s);
        if (e != hipSuccess) return set_error(FEM_EHIP, "forward kernel launch failed: %s", hipGetErrorString(e));
        if (prec == FEM_FP32_MIXED) {
            e = launch_fixup(a, kFixGrid, s);
            if (e != hipSuccess) return set_error(FEM_EHIP, "fixup kernel launch failed: %s", hipGetErrorString(e));
        }
    } else if (assemble) {
        // no elements: every residual entry and K entry is zero (or an identity row)
        FEM_HIP_CHECK(zero_bytes(w.Re, sizeof(double) * 24, s));
    }
    const int nn = mesh->n_nodes;
    if (R && nn > 0) {
        const int64_t nb = residual_blocks(nn), n_chunk = nb / 8;
        void* tr = timing_begin(s);
        hipLaunchKernelGGL(assemble_residual, dim3((unsigned)nb), dim3(kResThreads), 0, s, nn, n_chunk, csr->node_elem_ptr,
                           csr->node_elem, w.Re, bc_mask, R, rnorm2 ? w.part : nullptr);
        timing_end(tr, FEM_KERNEL_ASSEMBLE_R, s);
        FEM_HIP_CHECK(hipGetLastError());
        if (rnorm2) {
            hipLaunchKernelGGL(norm_final, dim3(1), dim3(kFinThreads), 0, s, w.part, (int)nb, rnorm2);
            FEM_HIP_CHECK(hipGetLastError());
        }
    } else if (rnorm2) {
        FEM_HIP_CHECK(zero_bytes(rnorm2, sizeof(double), s));
    }
    if (K_vals && nn > 0 && csr->nnz > 0) {
        const int64_t n_chunk = ((nn + kTanWaves - 1) / kTanWaves + 7) / 8;
        const unsigned nb = (unsigned)(8 * n_chunk);
        void* tk = timing_begin(s);
        if (prec == FEM_FP64)
            hipLaunchKernelGGL(assemble_tangent<double>, dim3(nb), dim3(64 * kTanWaves), 0, s, nn, n_chunk,
                               csr->node_elem_ptr, csr->node_elem, csr->elem_rank, csr->row_ptr, csr->col_idx,
                               reinterpret_cast<const double*>(w.Ke), bc_mask, reinterpret_cast<double*>(K_vals));
        else
            hipLaunchKernelGGL(assemble_tangent<float>, dim3(nb), dim3(64 * kTanWaves), 0, s, nn, n_chunk,
                               csr->node_elem_ptr, csr->node_elem, csr->elem_rank, csr->row_ptr, csr->col_idx,
                               reinterpret_cast<const float*>(w.Ke), bc_mask, reinterpret_cast<float*>(K_vals));
        timing_end(tk, FEM_KERNEL_ASSEMBLE_K, s);
        FEM_HIP_CHECK(hipGetLastError());
    }
    return FEM_OK;
}
