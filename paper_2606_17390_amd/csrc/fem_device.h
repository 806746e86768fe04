// fem_device.h -- per-Gauss-point device math of the hex8 finite-strain
// Hill-48 path (kinematics, spectral log strain, return map, pull-back and
// tangent pieces).  Templated on the working type R (double for the FP64
// path, float for the kinematics / pull-back / contraction of the mixed
// path); the trial stress, yield function and return map are always double.
//
// Paper passages: Sec. 2.2.2 (a)-(c) geometric pre/postprocessor and
// constitutive model, Sec. 2.2.3 elastic predictor / plastic corrector,
// App. A Hill-48, App. C Alg. C1, App. D (tangent of the converged update),
// Sec. 2.2.4 hex8 element.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fem {

constexpr double kSqrt2 = 1.41421356237309504880168872;
constexpr double kInvSqrt2 = 0.70710678118654752440084436;
constexpr double kInvSqrt3 = 0.57735026918962576450914878;
constexpr double kInvSqrt6 = 0.40824829046386301636621401;

// Mandel ordering (11, 22, 33, 23, 13, 12)
__host__ __device__ constexpr int mi(int k) { return k < 3 ? k : (k == 3 ? 1 : 0); }
__host__ __device__ constexpr int mj(int k) { return k < 3 ? k : (k == 5 ? 1 : 2); }
__host__ __device__ constexpr int midx(int a, int b) {
    return a == b ? a : ((a + b) == 3 ? 3 : ((a + b) == 2 ? 4 : 5));
}
// Mandel weight: 1 on the diagonal, sqrt2 on shear entries
template <typename R>
__host__ __device__ constexpr R mw(int k) { return k < 3 ? R(1) : R(kSqrt2); }

// ---------------------------------------------------------------- math shims
__device__ inline float m_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ inline double m_sqrt(double x) { return __builtin_sqrt(x); }
__device__ inline float m_rsqrt(float x) { return 1.0f / __builtin_sqrtf(x); }
__device__ inline double m_rsqrt(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ inline float m_log1p(float x) { return log1pf(x); }
__device__ inline double m_log1p(double x) { return log1p(x); }
__device__ inline float m_abs(float x) { return __builtin_fabsf(x); }
__device__ inline double m_abs(double x) { return __builtin_fabs(x); }
__device__ inline float m_sinh(float x) { return sinhf(x); }
__device__ inline double m_sinh(double x) { return sinh(x); }
__device__ inline float m_expm1(float x) { return expm1f(x); }
__device__ inline double m_expm1(double x) { return expm1(x); }
__device__ inline float m_cbrt(float x) { return cbrtf(x); }
__device__ inline double m_cbrt(double x) { return cbrt(x); }
// 1/x and 1/sqrt(x) in FP64 for the local update: the hardware estimate
// refined by two Newton-Raphson steps (quadratic convergence; the result is
// within about an ulp, for the finite positive normal arguments used here).
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ inline double rsqrt_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-x * r, r, 1.0);  // 1 - x r^2
    r = __builtin_fma(0.5 * r, e, r);
    e = __builtin_fma(-x * r, r, 1.0);
    return __builtin_fma(0.5 * r, e, r);
}
// c + a b as one fused multiply-add
__device__ inline float m_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double m_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R> struct Eps;
template <> struct Eps<double> {
    static constexpr double jacobi = 4e-16;   // relative off-diagonal stop (~2 ulp)
    static constexpr int sweeps = 10;
    static constexpr double series = 0.02;    // use series below this relative spread
    static constexpr int terms = 11;
};
template <> struct Eps<float> {
    static constexpr float jacobi = 2e-7f;
    static constexpr int sweeps = 8;
    static constexpr float series = 0.02f;
    static constexpr int terms = 6;
};

// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, typename Fn>
__device__ inline void static_for(Fn&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// 4 consecutive values with vector stores (16-byte aligned destination)
template <typename R>
__device__ inline void store4(R* p, const R v[4]);
template <>
__device__ inline void store4<float>(float* p, const float v[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
template <>
__device__ inline void store4<double>(double* p, const double v[4]) {
    reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// ---------------------------------------------------------------- kinematics

// Corner signs of the VTK hex (xi, eta, zeta) of node I.
__host__ __device__ constexpr int sgx(int I) { return (I == 1 || I == 2 || I == 5 || I == 6) ? 1 : -1; }
__host__ __device__ constexpr int sgy(int I) { return (I == 2 || I == 3 || I == 6 || I == 7) ? 1 : -1; }
__host__ __device__ constexpr int sgz(int I) { return I >= 4 ? 1 : -1; }

// Shape-function gradients at Gauss point gp, reference Jacobian and the
// displacement gradient H = grad u (F = I + H is never formed in storage, so
// that H keeps its relative precision in FP32 at small strains).
// xs, ds: node coordinates / displacements relative to node 0 (translations
// drop out of both J0 and grad u because the dN sum to zero).
template <typename R>
__device__ inline void kinematics(const R xs[8][3], const R ds[8][3], int gp, R g[8][3], R& detJ,
                                  R Hd[3][3]) {
    const R r = R(kInvSqrt3);
    const R xi = (gp & 1) ? r : -r, eta = (gp & 2) ? r : -r, zeta = (gp & 4) ? r : -r;
    R dN[8][3];
#pragma unroll
    for (int I = 0; I < 8; ++I) {
        const R a = R(1) + R(sgx(I)) * xi, b = R(1) + R(sgy(I)) * eta, c = R(1) + R(sgz(I)) * zeta;
        dN[I][0] = R(0.125) * R(sgx(I)) * b * c;
        dN[I][1] = R(0.125) * a * R(sgy(I)) * c;
        dN[I][2] = R(0.125) * a * b * R(sgz(I));
    }
    R J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            R s = R(0);
#pragma unroll
            for (int I = 1; I < 8; ++I) s += xs[I][i] * dN[I][j];
            J[i][j] = s;
        }
    const R c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const R c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const R c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    detJ = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const R id = R(1) / detJ;
    // Jinv[j][A]
    R Ji[3][3];
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
    for (int I = 0; I < 8; ++I)
#pragma unroll
        for (int A = 0; A < 3; ++A) g[I][A] = Ji[0][A] * dN[I][0] + Ji[1][A] * dN[I][1] + Ji[2][A] * dN[I][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int A = 0; A < 3; ++A) {
            R s = R(0);
#pragma unroll
            for (int I = 1; I < 8; ++I) s += ds[I][a] * g[I][A];
            Hd[a][A] = s;
        }
}

// Same as kinematics(), reading the element's node coordinates and
// displacements (nd[I][0..2] = X_I, nd[I][3..5] = d_I, FP64 in LDS) as they
// are needed, relative to node 0.
template <typename R, int W>
__device__ inline void kinematics_lds(const double (*nd)[W], int gp, R g[8][3], R& detJ, R Hd[3][3]) {
    const R r = R(kInvSqrt3);
    const R xi = (gp & 1) ? r : -r, eta = (gp & 2) ? r : -r, zeta = (gp & 4) ? r : -r;
    R dN[8][3];
#pragma unroll
    for (int I = 0; I < 8; ++I) {
        const R a = R(1) + R(sgx(I)) * xi, b = R(1) + R(sgy(I)) * eta, c = R(1) + R(sgz(I)) * zeta;
        dN[I][0] = R(0.125) * R(sgx(I)) * b * c;
        dN[I][1] = R(0.125) * a * R(sgy(I)) * c;
        dN[I][2] = R(0.125) * a * b * R(sgz(I));
    }
    R J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double x0 = nd[0][i];
#pragma unroll
        for (int j = 0; j < 3; ++j) J[i][j] = R(0);
#pragma unroll
        for (int I = 1; I < 8; ++I) {
            const R x = (R)(nd[I][i] - x0);
#pragma unroll
            for (int j = 0; j < 3; ++j) J[i][j] += x * dN[I][j];
        }
    }
    const R c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const R c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const R c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    detJ = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const R id = R(1) / detJ;
    R Ji[3][3];
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int A = 0; A < 3; ++A) Hd[a][A] = R(0);
#pragma unroll
    for (int I = 0; I < 8; ++I) {
#pragma unroll
        for (int A = 0; A < 3; ++A) g[I][A] = Ji[0][A] * dN[I][0] + Ji[1][A] * dN[I][1] + Ji[2][A] * dN[I][2];
        if (I > 0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R dv = (R)(nd[I][3 + a] - nd[0][3 + a]);
#pragma unroll
                for (int A = 0; A < 3; ++A) Hd[a][A] += dv * g[I][A];
            }
        }
    }
}

// ---------------------------------------------------------------- F-bar (Sec. 2.2.4)

// det(I + H) - 1 as tr H + (sum of principal 2x2 minors) + det H (no
// cancellation against 1 at small strain)
template <typename R>
__device__ inline R det_minus_one(const R H[3][3]) {
    const R m2 = (H[0][0] * H[1][1] - H[0][1] * H[1][0]) + (H[0][0] * H[2][2] - H[0][2] * H[2][0]) +
                 (H[1][1] * H[2][2] - H[1][2] * H[2][1]);
    const R d3 = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1]) - H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0]) +
                 H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
    return (H[0][0] + H[1][1] + H[2][2]) + m2 + d3;
}

// Sum over the 8 lanes of an element (xor butterfly; every lane gets the
// same bits, as each stage adds the same two values in either order).
template <typename R>
__device__ inline R sum8(R v) {
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    return v;
}

// Per Gauss point of the F-bar element: Fbar = beta F with
// beta = (Jbar / J)^(1/3), Jbar = sum_g w detJ0_g J_g / sum_g w detJ0_g
// (weights 1).  Replaces H by Hbar = Fbar - I = beta H + (beta - 1) I and
// returns beta and cw = w detJ0 J / (V_e Jbar), the weight of this Gauss
// point's dJ in dJbar / Jbar.  Called by all 8 lanes of the element.
// beta - 1 comes from logarithms of J and Jbar (accurate at small volume
// change); a non-positive J or Jbar takes the plain cube root.
template <typename R>
__device__ inline void fbar_gradient(R detJ0, R H[3][3], R& beta, R& cw, R& jm1) {
    jm1 = det_minus_one(H);
    const R V = sum8(detJ0);
    const R jbm1 = sum8(detJ0 * jm1) / V;
    R bm1;
    if (jm1 > R(-1) && jbm1 > R(-1)) bm1 = m_expm1((m_log1p(jbm1) - m_log1p(jm1)) * R(1.0 / 3.0));
    else bm1 = m_cbrt((R(1) + jbm1) / (R(1) + jm1)) - R(1);
    beta = R(1) + bm1;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) H[i][j] = beta * H[i][j] + ((i == j) ? bm1 : R(0));
    cw = detJ0 * (R(1) + jm1) / (V * (R(1) + jbm1));
}

// C - I = H + H^T + H^T H
template <typename R>
__device__ inline void cauchy_green_minus_identity(const R H[3][3], R M[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            R s = H[i][j] + H[j][i];
#pragma unroll
            for (int k = 0; k < 3; ++k) s += H[k][i] * H[k][j];
            M[i][j] = s;
            M[j][i] = s;
        }
}

// ---------------------------------------------------------------- eigen

template <typename R, int p, int q>
__device__ inline void jacobi_rotate(R a[3][3], R Q[3][3]) {
    constexpr int r = 3 - p - q;
    const R apq = a[p][q];
    if (apq == R(0)) return;
    const R theta = (a[q][q] - a[p][p]) / (R(2) * apq);
    const R at = m_abs(theta);
    // tan of the rotation angle, the smaller root; for a huge theta the
    // entry is negligible and t -> 1/(2 theta)
    R t = (at < R(1e18)) ? R(1) / (at + m_sqrt(at * at + R(1))) : R(0.5) / at;
    t = (theta < R(0)) ? -t : t;
    const R c = m_rsqrt(t * t + R(1));
    const R s = t * c;
    a[p][p] -= t * apq;
    a[q][q] += t * apq;
    a[p][q] = a[q][p] = R(0);
    const R arp = a[r][p], arq = a[r][q];
    a[r][p] = a[p][r] = c * arp - s * arq;
    a[r][q] = a[q][r] = s * arp + c * arq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R qp = Q[k][p], qq = Q[k][q];
        Q[k][p] = c * qp - s * qq;
        Q[k][q] = s * qp + c * qq;
    }
}

// Cyclic Jacobi on a symmetric 3x3 (destroyed): eigenvalues mu, eigenvectors
// in the columns of Q.
template <typename R>
__device__ inline void eig_sym3(R a[3][3], R mu[3], R Q[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? R(1) : R(0);
    for (int sw = 0; sw < Eps<R>::sweeps; ++sw) {
        const R off = m_abs(a[0][1]) + m_abs(a[0][2]) + m_abs(a[1][2]);
        const R dg = m_abs(a[0][0]) + m_abs(a[1][1]) + m_abs(a[2][2]);
        if (off <= Eps<R>::jacobi * dg) break;
        jacobi_rotate<R, 0, 1>(a, Q);
        jacobi_rotate<R, 0, 2>(a, Q);
        jacobi_rotate<R, 1, 2>(a, Q);
    }
    mu[0] = a[0][0];
    mu[1] = a[1][1];
    mu[2] = a[2][2];
}

// ---------------------------------------------------------------- divided differences of f(c) = 1/2 ln c

// sinh(u)/u
template <typename R>
__device__ inline R sinhc(R u) {
    const R au = m_abs(u);
    if (au < R(0.5)) {
        const R u2 = u * u;
        // 1 + u^2/3! + u^4/5! + ... (Horner, to u^16)
        R s = R(1.0 / 355687428096000.0);  // 1/17!
        s = s * u2 + R(1.0 / 1307674368000.0);
        s = s * u2 + R(1.0 / 6227020800.0);
        s = s * u2 + R(1.0 / 39916800.0);
        s = s * u2 + R(1.0 / 362880.0);
        s = s * u2 + R(1.0 / 5040.0);
        s = s * u2 + R(1.0 / 120.0);
        s = s * u2 + R(1.0 / 6.0);
        return s * u2 + R(1);
    }
    return m_sinh(u) / u;
}

// f1(c_a, c_b) = (f(c_a) - f(c_b)) / (c_a - c_b) with c = 1 + mu, e = 1/2 ln c:
// = 1 / (2 sqrt(c_a c_b) sinhc(e_a - e_b)); no cancellation.
template <typename R>
__device__ inline R dd1(R mua, R mub, R ea, R eb) {
    return R(0.5) * m_rsqrt((R(1) + mua) * (R(1) + mub)) / sinhc(ea - eb);
}

// f2(c_a, c_a, c_b) = (f'(c_a) - f1(c_a, c_b)) / (c_a - c_b)
//                   = -(r - ln(1+r)) / (2 c_a^2 r^2),  r = (c_b - c_a)/c_a
template <typename R>
__device__ inline R dd2_pair(R mua, R mub, R ea, R eb) {
    const R ca = R(1) + mua;
    const R r = (mub - mua) / ca;
    R v;
    if (m_abs(r) < Eps<R>::series) {
        // sum_j (-r)^j / (j+2)
        R s = R(0);
#pragma unroll
        for (int j = Eps<R>::terms; j >= 0; --j) s = s * (-r) + R(1) / R(j + 2);
        v = s;
    } else {
        const R lg = R(2) * (eb - ea);  // ln(c_b / c_a)
        v = (r - lg) / (r * r);
    }
    return R(-0.5) * v / (ca * ca);
}

// f2 of three (possibly close) arguments; Taylor series of the divided
// difference about the mean for a small spread, else the sorted quotient.
template <typename R>
__device__ inline R dd2_triple(R m0, R m1, R m2, R e0, R e1, R e2) {
    // sort by mu
    R x0 = m0, x1 = m1, x2 = m2, y0 = e0, y1 = e1, y2 = e2, t;
    if (x1 < x0) { t = x0; x0 = x1; x1 = t; t = y0; y0 = y1; y1 = t; }
    if (x2 < x1) { t = x1; x1 = x2; x2 = t; t = y1; y1 = y2; y2 = t; }
    if (x1 < x0) { t = x0; x0 = x1; x1 = t; t = y0; y0 = y1; y1 = t; }
    const R mean = (x0 + x1 + x2) / R(3);
    const R m = R(1) + mean;
    if (x2 - x0 < Eps<R>::series * m) {
        const R im = R(1) / m;
        const R d0 = (x0 - mean) * im, d1 = (x1 - mean) * im, d2 = (x2 - mean) * im;
        // complete homogeneous symmetric polynomials h_j of the scaled deltas
        // via power sums; f2 = sum_j (-1)^(j+1) h_j / (2 (j+2) m^(j+2)) ... in scaled form
        constexpr int NT = Eps<R>::terms;
        R p[NT + 1], h[NT + 1];
        R q0 = d0, q1 = d1, q2 = d2;
#pragma unroll
        for (int k = 1; k <= NT; ++k) {
            p[k] = q0 + q1 + q2;
            q0 *= d0;
            q1 *= d1;
            q2 *= d2;
        }
        h[0] = R(1);
#pragma unroll
        for (int j = 1; j <= NT; ++j) {
            R s = R(0);
#pragma unroll
            for (int i = 1; i <= j; ++i) s += p[i] * h[j - i];
            h[j] = s / R(j);
        }
        R sum = R(0);
#pragma unroll
        for (int j = NT; j >= 0; --j) {
            const R ck = ((j % 2) == 0 ? R(-1) : R(1)) / R(2 * (j + 2));
            sum += ck * h[j];
        }
        return sum * im * im;
    }
    return (dd1(x0, x1, y0, y1) - dd1(x1, x2, y1, y2)) / (x0 - x2);
}

// ---------------------------------------------------------------- material

struct Mat {
    double E, nu, F, G, H, L, M, N, K, eps0, nexp;  // Voce: (K, eps0, nexp) = (sig0, Q, b)
    int voce;
};

// Hill-48 in its eigen-modes: hydrostatic direction (eigenvalue 0), two
// deviatoric normal modes v1, v2 (eigenvalues h1, h2) and the three shear
// Mandel directions (L, M, N); isotropic elasticity is diagonal in the same
// basis (3 kappa, 2 mu x 5).
struct Modes {
    double lam, mu2, k3;
    double v1[3], v2[3];
    double eta[5];
};

__device__ inline void hill_modes(const Mat& m, Modes& h) {
    const double mu = m.E / (2.0 * (1.0 + m.nu));
    h.mu2 = 2.0 * mu;
    h.lam = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
    h.k3 = m.E / (1.0 - 2.0 * m.nu);
    // normal block of the Hill matrix in the basis ea = (1,-1,0)/sqrt2, eb = (1,1,-2)/sqrt6
    const double h00 = 0.5 * (m.F + m.G + 4.0 * m.H);
    const double h11 = 1.5 * (m.F + m.G);
    const double h01 = 0.86602540378443864676 * (m.G - m.F);
    const double dd = 0.5 * (h00 - h11);
    const double rr = sqrt(dd * dd + h01 * h01);
    double c = 1.0, s = 0.0;  // v1 = c ea + s eb
    if (rr > 0.0) {
        // eigenvector of the larger eigenvalue, from the better-conditioned form
        double x, y;
        if (dd >= 0.0) { x = rr + dd; y = h01; }
        else { x = h01; y = rr - dd; }
        const double inv = 1.0 / sqrt(x * x + y * y);
        c = x * inv;
        s = y * inv;
    }
    const double mid = 0.5 * (h00 + h11);
    h.eta[0] = mid + rr;
    h.eta[1] = mid - rr;
    h.eta[2] = m.L;
    h.eta[3] = m.M;
    h.eta[4] = m.N;
    const double ea[3] = {kInvSqrt2, -kInvSqrt2, 0.0};
    const double eb[3] = {kInvSqrt6, kInvSqrt6, -2.0 * kInvSqrt6};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        h.v1[i] = c * ea[i] + s * eb[i];
        h.v2[i] = -s * ea[i] + c * eb[i];
    }
}

// Isotropic hardening sigma_y(alpha) and its slope: Swift K (eps0 + alpha)^n,
// or Voce sig0 + Q (1 - exp(-b alpha)) (Eq. Hard, in uniaxial-stress units)
// with (sig0, Q, b) in the slots of (K, eps0, n).  The law is the same for
// every element of a launch, so the branch is uniform.
__device__ inline double hardening(const Mat& m, double alpha, double& dsig) {
    if (m.voce) {
        const double ex = exp(-m.nexp * alpha);
        dsig = m.eps0 * m.nexp * ex;
        return m.K + m.eps0 * (1.0 - ex);
    }
    const double base = m.eps0 + alpha;
    const double s = m.K * exp(m.nexp * log(base));
    dsig = m.nexp * s * recip(base);
    return s;
}

// Result of the local update at one Gauss point.
struct Local {
    double T[6];      // Cartesian Mandel logarithmic stress
    double hist[7];   // updated eps^p (tensor comps) and alpha
    double coef[5];   // a_i - 2 mu, a_i = 2 mu / (1 + 2 mu lambda eta_i)
    double mvec[5];   // m_i = a_i N_i (modal)
    double beta;      // Cep = E + sum coef_i b_i b_i^T - beta m m^T (modal basis b)
    // kept for the adjoint
    double lam, dgamma, phi, dsig, sig, svar, Nm[5], tb_h;
    double ftr, sy_n;
    int plastic, converged;
};

// Elastic predictor, yield check and return map (Sec. 2.2.3, Alg. C1).
// eps: Cartesian Mandel total log strain; hist_n: eps^p tensor comps, alpha.
// The plastic corrector solves the closest-point equations for the isotropic
// elasticity / Hill-48 pair in its common eigenbasis: with lambda = dgamma/phi,
// tau_i = s_i / (1 + 2 mu lambda eta_i) and the scalar consistency condition
// phi(lambda) - sigma_y(alpha_n + lambda phi(lambda)) = 0 is solved by a
// bracketed Newton iteration.
__device__ inline void local_update(const double eps[6], const double* hist_n, const Mat& m,
                                    const Modes& h, Local& o) {
    double ee[6];
    ee[0] = eps[0] - hist_n[0];
    ee[1] = eps[1] - hist_n[1];
    ee[2] = eps[2] - hist_n[2];
    ee[3] = eps[3] - kSqrt2 * hist_n[3];
    ee[4] = eps[4] - kSqrt2 * hist_n[4];
    ee[5] = eps[5] - kSqrt2 * hist_n[5];
    const double tr = ee[0] + ee[1] + ee[2];
    double t[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) t[i] = h.mu2 * ee[i] + (i < 3 ? h.lam * tr : 0.0);
    // modal coordinates of the trial stress
    const double th = (t[0] + t[1] + t[2]) * kInvSqrt3;
    double s[5];
    s[0] = h.v1[0] * t[0] + h.v1[1] * t[1] + h.v1[2] * t[2];
    s[1] = h.v2[0] * t[0] + h.v2[1] * t[1] + h.v2[2] * t[2];
    s[2] = t[3];
    s[3] = t[4];
    s[4] = t[5];
    double phi2 = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) phi2 += h.eta[i] * s[i] * s[i];
    // phi_tr = sqrt(phi2) (phi2 = 0 only for a zero deviatoric trial stress)
    const double phi_tr = phi2 > 0.0 ? phi2 * rsqrt_nr(phi2) : 0.0;
    double dsig_n;
    const double alpha_n = hist_n[6];
    o.sy_n = hardening(m, alpha_n, dsig_n);
    o.ftr = phi_tr - o.sy_n;
    o.tb_h = th;
    if (!(o.ftr > 0.0)) {
        o.plastic = 0;
        o.converged = 1;
#pragma unroll
        for (int i = 0; i < 6; ++i) o.T[i] = t[i];
#pragma unroll
        for (int i = 0; i < 7; ++i) o.hist[i] = hist_n[i];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            o.coef[i] = 0.0;
            o.mvec[i] = 0.0;
            o.Nm[i] = 0.0;
        }
        o.beta = 0.0;
        o.lam = o.dgamma = 0.0;
        o.phi = phi_tr;
        o.sig = o.sy_n;
        o.dsig = dsig_n;
        o.svar = 0.0;
        return;
    }
    o.plastic = 1;
    const double mu2 = h.mu2;
    // Newton on psi(lambda) = (1 + 2 mu etab lambda) g(lambda): the factor is
    // positive, so psi and g share their root, and for a single active Hill
    // mode with linear hardening psi is linear in lambda (one step).  etab is
    // the trial-stress weighted mean Hill eigenvalue.
    double num = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) num += h.eta[i] * h.eta[i] * s[i] * s[i];
    const double etab = num * recip(phi2);
    double lam = 0.0, lo = 0.0, hi = __builtin_inf();
    double phi = phi_tr, sig = o.sy_n, dsig = dsig_n;
    int conv = 0;
    for (int it = 0; it < 40; ++it) {
        double p2 = 0.0, dp = 0.0;
        const double c = mu2 * lam;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const double den = recip(1.0 + c * h.eta[i]);
            const double ti = s[i] * den;
            const double e2 = h.eta[i] * ti * ti;
            p2 += e2;
            dp -= mu2 * h.eta[i] * e2 * den;
        }
        const double iphi = rsqrt_nr(p2);
        phi = p2 * iphi;
        dp *= iphi;
        sig = hardening(m, alpha_n + lam * phi, dsig);
        const double g = phi - sig;
        if (g > 0.0) lo = lam; else hi = lam;
        // converged at the rounding level of sigma_y
        if (fabs(g) <= 1e-15 * sig) { conv = 1; break; }
        const double gp = dp - dsig * (phi + lam * dp);
        const double f = 1.0 + mu2 * etab * lam;
        const double step = -(f * g) * recip(mu2 * etab * g + f * gp);
        double ln = lam + step;
        if (!(ln > lo && ln < hi)) ln = (hi < __builtin_inf()) ? 0.5 * (lo + hi) : 2.0 * lam + 1e-300;
        // step or bracket at the rounding level of lambda
        if (fabs(ln - lam) <= 2e-15 * lam || hi - lo <= 4e-16 * lam) { lam = ln; conv = 1; break; }
        lam = ln;
    }
    // final state at lambda
    double tau[5], den[5], p2 = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        den[i] = recip(1.0 + mu2 * lam * h.eta[i]);
        tau[i] = s[i] * den[i];
        p2 += h.eta[i] * tau[i] * tau[i];
    }
    const double iphi = rsqrt_nr(p2);
    phi = p2 * iphi;
    const double dg = lam * phi;
    const double alpha = alpha_n + dg;
    sig = hardening(m, alpha, dsig);
    o.converged = conv;
    o.lam = lam;
    o.dgamma = dg;
    o.phi = phi;
    o.sig = sig;
    o.dsig = dsig;
    double N[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) N[i] = h.eta[i] * tau[i] * iphi;
    // stress (Cartesian Mandel)
#pragma unroll
    for (int k = 0; k < 3; ++k) o.T[k] = th * kInvSqrt3 + tau[0] * h.v1[k] + tau[1] * h.v2[k];
    o.T[3] = tau[2];
    o.T[4] = tau[3];
    o.T[5] = tau[4];
    // eps^p_{n+1} = eps^p_n + dgamma N (tensor components)
#pragma unroll
    for (int k = 0; k < 3; ++k) o.hist[k] = hist_n[k] + dg * (N[0] * h.v1[k] + N[1] * h.v2[k]);
    o.hist[3] = hist_n[3] + dg * N[2] * kInvSqrt2;
    o.hist[4] = hist_n[4] + dg * N[3] * kInvSqrt2;
    o.hist[5] = hist_n[5] + dg * N[4] * kInvSqrt2;
    o.hist[6] = alpha;
    // algorithmic tangent in the modal basis:
    //   Cep = diag(3k, a_i) - beta m m^T,  m = A^-1 N,  s = N.m,
    //   beta = (1 - lambda sigma_y') / (s + sigma_y' (1 - lambda s))
    double sv = 0.0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const double a = mu2 * den[i];
        o.coef[i] = -mu2 * (mu2 * lam * h.eta[i]) * den[i];
        o.mvec[i] = a * N[i];
        o.Nm[i] = N[i];
        sv += o.mvec[i] * N[i];
    }
    o.svar = sv;
    o.beta = (1.0 - lam * dsig) * recip(sv + dsig * (1.0 - lam * sv));
}

// ---------------------------------------------------------------- orientation (App. A)

// Theta: row-major rotation whose columns are the orthotropy axes in global
// coordinates; a symmetric tensor A has material-frame components
// Theta^T A Theta.  The Hill tensor is given in the material frame, so the
// local update runs there (isotropic elasticity is unchanged by the
// rotation) and its results are rotated back.
__device__ inline void load_rotation(const double* __restrict__ orient, int64_t idx, double Th[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Th[i][j] = orient[9 * idx + 3 * i + j];
}

// Symmetric tensor with components v = (11, 22, 33, 23, 13, 12) scaled by w on
// the shear entries (w = 1: tensor components, w = sqrt2: Mandel), rotated:
// Theta^T A Theta (TO_MAT) or Theta A Theta^T.
template <bool TO_MAT>
__device__ inline void rotate_sym(const double Th[3][3], double v[6], double w) {
    const double iw = 1.0 / w;
    const double A[3][3] = {{v[0], v[5] * iw, v[4] * iw}, {v[5] * iw, v[1], v[3] * iw}, {v[4] * iw, v[3] * iw, v[2]}};
    double W[3][3];  // A R with R = Theta (TO_MAT) or Theta^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double x = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) x += A[i][k] * (TO_MAT ? Th[k][q] : Th[q][k]);
            W[i][q] = x;
        }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = mi(k), q = mj(k);
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) x += (TO_MAT ? Th[i][p] : Th[p][i]) * W[i][q];
        v[k] = (k < 3) ? x : w * x;
    }
}

// Qm = Theta^T Q: the eigenvectors of C in material-frame components
template <typename R>
__device__ inline void material_frame(const double* __restrict__ orient, int64_t idx, const R Q[3][3], R Qm[3][3]) {
    R Th[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Th[i][j] = (R)orient[9 * idx + 3 * i + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Qm[i][j] = Th[0][i] * Q[0][j] + Th[1][i] * Q[1][j] + Th[2][i] * Q[2][j];
}

// ---------------------------------------------------------------- frame helpers

// Mandel vector of Q^T B Q for B = diag(v)
template <typename R>
__device__ inline void rot_diag(const R Q[3][3], const R v[3], R out[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = mi(k), q = mj(k);
        R s = v[0] * Q[0][p] * Q[0][q] + v[1] * Q[1][p] * Q[1][q] + v[2] * Q[2][p] * Q[2][q];
        out[k] = mw<R>(k) * s;
    }
}

// Mandel vector of Q^T B Q for B = the unit Mandel shear tensor on (i, j)
template <typename R, int i, int j>
__device__ inline void rot_shear(const R Q[3][3], R out[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = mi(k), q = mj(k);
        R s = (Q[i][p] * Q[j][q] + Q[j][p] * Q[i][q]) * R(kInvSqrt2);
        out[k] = mw<R>(k) * s;
    }
}

// Q^T S Q (S given as Cartesian Mandel) -> symmetric 3x3 in the eigenframe
template <typename R>
__device__ inline void mandel_to_frame(const R Q[3][3], const R v[6], R out[3][3]) {
    R S[3][3];
    S[0][0] = v[0];
    S[1][1] = v[1];
    S[2][2] = v[2];
    S[1][2] = S[2][1] = v[3] * R(kInvSqrt2);
    S[0][2] = S[2][0] = v[4] * R(kInvSqrt2);
    S[0][1] = S[1][0] = v[5] * R(kInvSqrt2);
    R W[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) W[i][q] = S[i][0] * Q[0][q] + S[i][1] * Q[1][q] + S[i][2] * Q[2][q];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = p; q < 3; ++q) {
            R s = Q[0][p] * W[0][q] + Q[1][p] * W[1][q] + Q[2][p] * W[2][q];
            out[p][q] = s;
            out[q][p] = s;
        }
}

// Q X Q^T (X symmetric in the eigenframe) -> Cartesian Mandel
template <typename R>
__device__ inline void frame_to_mandel(const R Q[3][3], const R X[3][3], R v[6]) {
    R W[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int b = 0; b < 3; ++b) W[i][b] = Q[i][0] * X[0][b] + Q[i][1] * X[1][b] + Q[i][2] * X[2][b];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int i = mi(k), j = mj(k);
        R s = W[i][0] * Q[j][0] + W[i][1] * Q[j][1] + W[i][2] * Q[j][2];
        v[k] = mw<R>(k) * s;
    }
}

}  // namespace fem
