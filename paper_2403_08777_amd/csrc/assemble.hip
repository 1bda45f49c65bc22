// Momentum right-hand-side assembly over linear tetrahedra and its velocity
// vector-Jacobian product: element math and the two scatter strategies.
//
// Element math (one thread per element, everything in registers):
//   geometry in FP64: J columns d_k = x_k - x_0, rows of adj(J) c_1 = d_2 x d_3,
//   c_2 = d_3 x d_1, c_3 = d_1 x d_2, det J = d_1 . c_1, grad N_k = c_k / det J,
//   grad N_0 = -(grad N_1 + grad N_2 + grad N_3), V = |det J| / 6.
//
//   The paper integrates with four Gauss points on P1 tetrahedra (Sec. V-B).
//   Because grad N, G = grad u and q = grad p are constant on the element, the
//   Gauss sums collapse exactly: with N_a(g) = alpha (a == g) or beta, weight
//   V/4, one has sum_g (V/4) N_a(g) = V/4 and sum_g (V/4) N_a(g) N_b(g) =
//   (V/4)(alpha^2 + 3 beta^2) = V/10 for a == b, (V/4)(2 alpha beta + 2 beta^2)
//   = V/20 otherwise.  So
//     sum_g (V/4) N_a(g) [-rho G u^g - q + rho f]
//       = -(rho V / 20) G (u_a + U) + (V/4)(rho f - q),   U = sum_b u_b,
//   and adding the viscous term -mu_e V G grad N_a gives
//     R^e_a = b - G y_a,   b = (V/4)(rho f - q),
//     y_a = (rho V / 20)(u_a + U) + mu_e V grad N_a.
//   This is the paper's restructuring (compute each RHS entry directly, few
//   live intermediates; Sec. V-A) carried one step further: the four Gauss
//   points are summed symbolically, not numerically.
//
//   VJP, g = (dR/du)^T lambda, per element with L = sum_a lambda_a,
//   P = sum_a lambda_a (x) u_a, Lambda = sum_a lambda_a (x) grad N_a:
//     g_b = -M grad N_b - (rho V / 20) G^T (lambda_b + L),
//     M = (rho V / 20)(P + L (x) U) + mu_e V Lambda + V Phi D = sum_a lambda_a (x) y_a + V Phi D,
//   where Phi = Lambda : G = sum_a lambda_a . G grad N_a and D = d mu_t / d G
//   (for Smagorinsky rho (cs Delta)^2 2 S / |S|, 0 if |S| = 0).
//
// Scatter strategies:
//   ATOMIC: one thread per element, 12 global atomic adds.
//   PATCH:  one workgroup per patch of <= 256 consecutive (Hilbert-ordered)
//           elements; the patch's <= 256 distinct nodes are loaded once into
//           LDS, element contributions are summed per node in LDS (slot runs,
//           no LDS atomics), and each patch node gets one global atomic add
//           per component.
//   PATCH_GATHER: as PATCH, but the per-patch node sums go to a partial-sum
//           buffer and a node-parallel kernel adds them in patch order: no
//           atomics anywhere, bitwise reproducible, no zero-fill.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <type_traits>

#include <hip/hip_ext.h>

#include "internal.hpp"

namespace nsasm {
namespace {

constexpr int kThreads = 256;
// What a launch computes.  Node fields: A (vector), B (vector), C (scalar).
//   kForward: A = u, C = p            -> rhs (3 per node)
//   kVjp:     A = u, B = adjoint      -> (d rhs / d u)^T adjoint (3)
//   kVjpP:    B = adjoint             -> (d rhs / d p)^T adjoint (1)
//   kJvp:     A = u, B = du, C = dp   -> (d rhs / d u) du + (d rhs / d p) dp (3)
//   kMass:    no fields               -> lumped volume V^L (1), once per mesh
enum Mode { kForward = 0, kVjp = 1, kVjpP = 2, kJvp = 3, kMass = 4 };

template <int MODE>
struct Fields {
    static constexpr int NA = (MODE == kVjpP || MODE == kMass) ? 0 : 3;
    static constexpr int NB = (MODE == kForward || MODE == kMass) ? 0 : 3;
    static constexpr int NC = (MODE == kForward || MODE == kJvp) ? 1 : 0;
    static constexpr int NOUT = (MODE == kVjpP || MODE == kMass) ? 1 : 3;
};

template <typename T>
struct KParams {
    T rho;
    T mu;
    T rho_c;       // rho * model constant: cs^2 (Smagorinsky) or 2.5 cs^2 (Vreman)
    T rho_f[3];    // rho * f
    T conv_a;      // convective form c = G u + conv_a tr(G) u + conv_b G^T u
    T conv_b;
};

// Convective form: kAdvective is c = G u; kGeneral adds conv_a tr(G) u +
// conv_b G^T u (divergence, skew-symmetric, rotational and EMAC forms).
enum ConvForm { kAdvective = 0, kGeneral = 1 };

// ------------------------------------------------------------ atomics

__device__ inline void global_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void global_add(float *p, float v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Delta^2 = V^(2/3), the squared filter width of the eddy viscosity, from an
// estimate y of V^(-1/3) built with the hardware base-2 logarithm and
// exponential, then V^(2/3) = V y.
// FP64: V = w 2^(3q), q = (21846 e) >> 16 for V's binary exponent e (e / 3
// rounded down, or one below it for the negative multiples of 3), so that w
// lies in [1/2, 8) and y estimates w^(-1/3) to about 2^-22; one step of the
// binomial series (1 - r)^(-1/3) = 1 + h + 2 h^2 + 14 h^3 / 3 + ...,
// r = 1 - w y^3, h = r / 3, taken to second order then leaves about
// 14 |h|^3 / 3 with |h| about 2^-22, far below rounding;
// V^(2/3) = (w y) 2^(2q).
// FP32 (the mixed path): y <- y (4 - V y^3) / 3, one Newton step (the
// estimate's error, about 1e-6 for small V, is squared).  Volumes below
// 2^-100 are scaled by 2^96 first (2^64 after the power), so that the
// logarithm never sees a denormal.
__device__ inline double filter_width_sq(double v) {
    const int q = __mul24(__builtin_amdgcn_frexp_exp(v), 21846) >> 16;
    const double w = ldexp(v, -3 * q);
    double y = static_cast<double>(
        __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(static_cast<float>(w)) * (-1.0f / 3.0f)));
    const double h = fma(-w, y * y * y, 1.0) * (1.0 / 3.0);
    y = fma(y, h * fma(h, 2.0, 1.0), y);
    return ldexp(w * y, 2 * q);
}
__device__ inline float filter_width_sq(float v) {
    const bool tiny = v < 0x1p-100f;
    const float w = tiny ? v * 0x1p96f : v;
    float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(w) * (-1.0f / 3.0f));
    y = y * (4.0f - w * (y * y * y)) * (1.0f / 3.0f);
    const float d2 = w * y;
    return tiny ? d2 * 0x1p-64f : d2;
}

// 1 / sqrt(x) for x > 0.  FP32: the hardware reciprocal square root (1 ulp).
// FP64 (normal or not): x = w 4^p with
// p = floor(e/2) for x's binary exponent e, so that w lies in [1/2, 2); the
// hardware FP32 reciprocal square root of w (about 2^-22 after the
// conversions) and one step of the binomial series
// (1 - t)^(-1/2) = 1 + h + 3 h^2 / 2 + 5 h^3 / 2 + ..., t = 1 - w y^2,
// h = t / 2, to second order (leaving about 5 |h|^3 / 2, |h| about 2^-22);
// then 1 / sqrt(x) = y 2^-p.
__device__ inline double inv_root(double x) {
    const int p = __builtin_amdgcn_frexp_exp(x) >> 1;
    const double w = ldexp(x, -2 * p);
    double y = static_cast<double>(__builtin_amdgcn_rsqf(static_cast<float>(w)));
    const double h = fma(-w, y * y, 1.0) * 0.5;
    y = fma(y, h * fma(h, 1.5, 1.0), y);
    return ldexp(y, -p);
}
__device__ inline float inv_root(float x) { return __builtin_amdgcn_rsqf(x); }

// sqrt in FP32: the hardware square root (1 ulp).
__device__ inline float root(float v) { return __builtin_amdgcn_sqrtf(v); }

// a / b for the eddy model's ratios of normal, finite operands: a times 1/b.
// FP64: the hardware reciprocal estimate refined by two Newton-Raphson steps
// (as for 1/det J), within about one ulp, so the ratio is within two.  FP32
// (the mixed path, whose error is measured, not bounded): the hardware
// reciprocal (1 ulp).
__device__ inline double quotient(double a, double b) {
    double inv = __builtin_amdgcn_rcp(b);
    inv = fma(inv, fma(-b, inv, 1.0), inv);
    inv = fma(inv, fma(-b, inv, 1.0), inv);
    return a * inv;
}
__device__ inline float quotient(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// ----------------------------------------------------------- element math

// Shape-function gradients and volume, always in FP64.  1/det is the
// hardware reciprocal estimate refined by NEWTON Newton-Raphson steps, each
// of which squares the relative error: two are enough for full double
// precision (the finite, non-zero determinants a validated mesh has), as
// they are for the library's own FP64 division, so the estimate is good to
// about 2^-13.5; the mixed path rounds the gradients to FP32 afterwards, and
// after one step (error below 2^-26) it takes only that one.
template <int NEWTON = 2>
__device__ inline void tet_geometry(const double (&xe)[4][3], double (&gN)[4][3], double &vol) {
    double c1[3], c2[3], c3[3], d1[3];
    const double det = tet_adjugate(xe, c1, c2, c3, d1);
    double inv = __builtin_amdgcn_rcp(det);
#pragma unroll
    for (int k = 0; k < NEWTON; ++k) inv = fma(inv, fma(-det, inv, 1.0), inv);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gN[1][i] = c1[i] * inv;
        gN[2][i] = c2[i] * inv;
        gN[3][i] = c3[i] * inv;
        gN[0][i] = -(gN[1][i] + gN[2][i] + gN[3][i]);
    }
    vol = fabs(det) * (1.0 / 6.0);
}

// G[i][j] = d v_i / d x_j for a nodal vector field v.
template <typename T>
__device__ inline void vector_gradient(const T (&gN)[4][3], const T (&ve)[4][3], T (&G)[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T d1 = ve[1][i] - ve[0][i], d2 = ve[2][i] - ve[0][i], d3 = ve[3][i] - ve[0][i];
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j] = d1 * gN[1][j] + d2 * gN[2][j] + d3 * gN[3][j];
    }
}

enum EddyModel { kNoEddy = 0, kSmagorinsky = 1, kVreman = 2 };

// Cofactor matrix of G: C_ij = G_{i+1,j+1} G_{i+2,j+2} - G_{i+1,j+2} G_{i+2,j+1}
// (indices mod 3), the 2x2 minors of G with their signs.
template <typename T>
__device__ inline void cofactors(const T (&G)[3][3], T (&C)[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i][j] = G[i1][j1] * G[i2][j2] - G[i1][j2] * G[i2][j1];
        }
}

// d mu_t / d G is rebuilt from G where it is used (eddy_d), from a few
// scalars, so that its nine entries need not stay live:
//   Smagorinsky D_ij = k (G_ij + G_ji)              (k = c / |S|),
//   Vreman      D_ij = k (N_ij / A - s2 G_ij)       (k = c / s, s2 = s^2 / A),
// with N = (tr(P) I - P) G, P = G G^T, evaluated as the cofactor contraction
// N_kl = G_{k1 l1} C_{k2 l2} - G_{k1 l2} C_{k2 l1} - G_{k2 l1} C_{k1 l2} + G_{k2 l2} C_{k1 l1}
// (k1 = k+1, k2 = k+2 mod 3; C the cofactors of G), N / A from the cofactors
// scaled by ia = 1 / A.  Dividing both terms by A, rather than the factor
// k (which would then be c / (A s)), keeps every intermediate within a few
// powers of the element size h (c / (A s) grows as h^5 and its product with
// the VJP's weights as h^7, beyond the double range some 2^140 from unit scale).
template <typename T>
struct EddyD {
    T k;
    T s2;
    T ia;
};

// Vreman's B_beta / Delta^4 = e2(P) equals, by the Cauchy-Binet formula, the
// sum of the squared 2x2 minors of G, |cof G|^2, and (1/2) dB/dG = N above.
// Both forms are used here instead of minors of P: when G is close to rank
// one in a scaled direction (elements squashed along one axis), the minors of
// P cancel to far below their terms while the minors of G do not, so the
// result keeps its accuracy in FP64 and stays meaningful in FP32.
template <typename T, int EDDY>
__device__ inline T eddy_viscosity_k(const T (&G)[3][3], T vol, T rho_c, EddyD<T> &ed) {
    ed.k = T(0);
    ed.s2 = T(0);
    ed.ia = T(0);
    if (EDDY == kNoEddy) return T(0);
    const T c = rho_c * filter_width_sq(vol);
    if (EDDY == kSmagorinsky) {
        // 2 S:S = sum_ij (G_ij + G_ji)^2 / 2 = sum_i 2 G_ii^2 + sum_{i<j} (G_ij + G_ji)^2
        T ss = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const T d = G[i][i];
            ss += T(2) * d * d;
#pragma unroll
            for (int j = i + 1; j < 3; ++j) {
                const T o = G[i][j] + G[j][i];
                ss += o * o;
            }
        }
        if constexpr (std::is_same<T, double>::value) {
            // |S| = ss / sqrt(ss) and c / |S| = c / sqrt(ss): one reciprocal
            // square root, no division; 0 for a uniform velocity (ss = 0)
            const bool live = ss > 0.0;
            const double ir = inv_root(ss);
            ed.k = live ? c * ir : 0.0;
            return live ? c * (ss * ir) : 0.0;
        } else {
            const T smag = root(ss);
            ed.k = (smag > T(0)) ? quotient(c, smag) : T(0);
            return c * smag;
        }
    }
    T C[3][3];
    cofactors(G, C);
    T A = T(0), B = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            A += G[i][j] * G[i][j];
            B += C[i][j] * C[i][j];
        }
    // s = sqrt(B / A) and c / s from one reciprocal square root; 0 where the
    // model is (G of rank one or zero)
    const bool live = (A > T(0)) && (B > T(0));
    const T ia = live ? quotient(T(1), A) : T(0);
    const T q = B * ia;
    const T r = inv_root(q);
    ed.k = live ? c * r : T(0);
    ed.s2 = q * ia;
    ed.ia = ia;
    return live ? c * (q * r) : T(0);
}

// All of D = d mu_t / d G from G and the scalars of eddy_viscosity_k.
template <typename T, int EDDY>
__device__ inline void eddy_d(const T (&G)[3][3], const EddyD<T> &ed, T (&D)[3][3]) {
    if (EDDY == kSmagorinsky) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) D[i][j] = ed.k * (G[i][j] + G[j][i]);
    }
    if (EDDY == kVreman) {
        T C[3][3];
        cofactors(G, C);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) C[i][j] *= ed.ia;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const int k1 = (k + 1) % 3, k2 = (k + 2) % 3, l1 = (l + 1) % 3, l2 = (l + 2) % 3;
                const T n = (G[k1][l1] * C[k2][l2] - G[k1][l2] * C[k2][l1]) +
                            (G[k2][l2] * C[k1][l1] - G[k2][l1] * C[k1][l2]);
                D[k][l] = ed.k * (n - ed.s2 * G[k][l]);
            }
    }
}

// M += s D with D = d mu_t / d G rebuilt from G as in eddy_d, the factor s
// folded into the scalars (Smagorinsky: the symmetric sums G_ij + G_ji once
// per pair, one fused multiply-add per entry).
template <typename T, int EDDY>
__device__ inline void add_scaled_eddy_d(const T (&G)[3][3], const EddyD<T> &ed, T s, T (&M)[3][3]) {
    const T f = s * ed.k;
    if (EDDY == kSmagorinsky) {
        const T f2 = f + f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            M[i][i] += f2 * G[i][i];
#pragma unroll
            for (int j = i + 1; j < 3; ++j) {
                const T o = G[i][j] + G[j][i];
                M[i][j] += f * o;
                M[j][i] += f * o;
            }
        }
    }
    if (EDDY == kVreman) {
        EddyD<T> e{f, ed.s2, ed.ia};
        T D[3][3];
        eddy_d<T, EDDY>(G, e, D);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) M[k][l] += D[k][l];
    }
}

// Eddy viscosity mu_t of the element's constant velocity gradient G, with
// filter width Delta = V^(1/3) and c = rho_c Delta^2; with WANT_D also
// D = d mu_t / d G (0 where the model is not differentiable).
//   Smagorinsky: mu_t = c |S|, S = (G + G^T)/2, |S| = sqrt(2 S:S),
//                D = (2c / |S|) S.
//   Vreman (alpha = G^T, beta = Delta^2 alpha^T alpha): with P = G G^T,
//                A = tr P = alpha:alpha and B = e2(P) (sum of the principal
//                2x2 minors, Vreman's B_beta / Delta^4), mu_t = c s with
//                s = sqrt(B / A); since dA/dG = 2G and dB/dG = 2(tr(P) I - P)G,
//                D = c / (A s) ((tr(P) I - P) G - s^2 G).
template <typename T, int EDDY, bool WANT_D>
__device__ inline T eddy_viscosity(const T (&G)[3][3], T vol, T rho_c, T (&D)[3][3]) {
    EddyD<T> ed;
    const T mu_t = eddy_viscosity_k<T, EDDY>(G, vol, rho_c, ed);
    if (WANT_D) eddy_d<T, EDDY>(G, ed, D);
    return mu_t;
}

// ldu(a, i) returns u_a[i]; it is called for G and U and again where u_a
// enters y_a (see element_vjp on why a caller may read it from LDS twice).
template <typename T, int EDDY, int CONV, typename LdU, typename Sink>
__device__ inline void element_rhs(const T (&gN)[4][3], T vol, LdU &&ldu, const T (&pe)[4], const KParams<T> &P,
                                   Sink &&emit) {
    T G[3][3], U[3];
    {
        T ue[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) ue[a][i] = ldu(a, i);
        vector_gradient(gN, ue, G);
#pragma unroll
        for (int i = 0; i < 3; ++i) U[i] = ue[0][i] + ue[1][i] + ue[2][i] + ue[3][i];
    }
    asm volatile("" ::: "memory");
    T q[3];
    {
        const T d1 = pe[1] - pe[0], d2 = pe[2] - pe[0], d3 = pe[3] - pe[0];
#pragma unroll
        for (int j = 0; j < 3; ++j) q[j] = d1 * gN[1][j] + d2 * gN[2][j] + d3 * gN[3][j];
    }
    T unused[3][3];
    const T mu_e = P.mu + eddy_viscosity<T, EDDY, false>(G, vol, P.rho_c, unused);
    const T sc = P.rho * vol * T(0.05);
    const T sv = mu_e * vol;
    const T w4 = vol * T(0.25);
    T b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        b[i] = w4 * (P.rho_f[i] - q[i]);
    }
    const T at = (CONV == kGeneral) ? P.conv_a * (G[0][0] + G[1][1] + G[2][2]) : T(0);
    // z_a = (rho V / 20)(u_a + U) = sc u_a + sc U: one FMA per component.
    T scU[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) scU[i] = sc * U[i];
    // Vertices 1..3 directly; vertex 0 from the element sum
    //   sum_a R^e_a = 4 b - 5 (rho V / 20) K U   (sum_a grad N_a = 0,
    //   sum_a (u_a + U) = 5 U), K = G (+ conv_a tr(G) I + conv_b G^T),
    // so that neither u_0 nor grad N_0 is needed after G and U.
    T rsum[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T ku = G[i][0] * scU[0] + G[i][1] * scU[1] + G[i][2] * scU[2];
        if (CONV == kGeneral) ku += at * scU[i] + P.conv_b * (G[0][i] * scU[0] + G[1][i] * scU[1] + G[2][i] * scU[2]);
        rsum[i] = T(4) * b[i] - T(5) * ku;
    }
#pragma unroll
    for (int a = 1; a < 4; ++a) {
        T z[3], y[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            z[j] = sc * ldu(a, j) + scU[j];
            y[j] = z[j] + sv * gN[a][j];
        }
        T re[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            // b - G y as a chain of fused multiply-subtracts from b
            T r = b[i];
            r -= G[i][0] * y[0];
            r -= G[i][1] * y[1];
            r -= G[i][2] * y[2];
            if (CONV == kGeneral) {
                r -= at * z[i];
                r -= P.conv_b * (G[0][i] * z[0] + G[1][i] * z[1] + G[2][i] * z[2]);
            }
            re[i] = r;
            rsum[i] -= r;
        }
        emit(a, re);
    }
    emit(0, rsum);
}

// ldu(a, i) and ldl(a, i) return u_a[i] and lambda_a[i].  Each is called
// where its value is used: u_a for G and U and again in the accumulation of M,
// lambda_a there and again in the per-vertex terms, so a caller that reads
// them from LDS keeps one vertex's values live instead of all four; the
// compiler barriers keep the second reads from being merged with the first.
// Vertex 0 comes from the element sum  sum_b g_b = -5 (rho V / 20) K^T L
// (sum_b grad N_b = 0, sum_b (lambda_b + L) = 5 L).
template <typename T, int EDDY, int CONV, typename LdU, typename LdL, typename Sink>
__device__ inline void element_vjp(const T (&gN)[4][3], T vol, LdU &&ldu, LdL &&ldl, const KParams<T> &P,
                                   Sink &&emit) {
    T G[3][3], U[3];
    {
        T ue[4][3];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) ue[a][i] = ldu(a, i);
        vector_gradient(gN, ue, G);
#pragma unroll
        for (int i = 0; i < 3; ++i) U[i] = ue[0][i] + ue[1][i] + ue[2][i] + ue[3][i];
    }
    asm volatile("" ::: "memory");
    const T sc = P.rho * vol * T(0.05);
    EddyD<T> ed;
    const T mu_e = P.mu + eddy_viscosity_k<T, EDDY>(G, vol, P.rho_c, ed);
    const T sv = mu_e * vol;
    T scU[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) scU[i] = sc * U[i];
    // M = sum_a lambda_a (x) y_a with y_a = (rho V / 20)(u_a + U) + mu_e V grad N_a
    // (the forward's y_a): the convective part (rho V / 20)(P + L (x) U) and the
    // viscous part mu_e V Lambda in one accumulation.  W = sum_a lambda_a (x) z_a,
    // z_a = (rho V / 20)(u_a + U), is the convective part alone, which a general
    // form K = G + conv_a tr(G) I + conv_b G^T turns into
    // W + conv_a tr(W) I + conv_b W^T.  Phi = Lambda : G = sum_a lambda_a . G grad N_a
    // weighs d mu_t / d G.
    T M[3][3] = {}, W[3][3] = {}, phi = T(0), L[3] = {};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        T la[3], z[3], y[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            la[j] = ldl(a, j);
            L[j] += la[j];
            z[j] = sc * ldu(a, j) + scU[j];
            y[j] = z[j] + sv * gN[a][j];
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                M[k][j] += la[k] * y[j];
                if (CONV == kGeneral) W[k][j] += la[k] * z[j];
            }
        if (EDDY != kNoEddy) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                phi += la[i] * (G[i][0] * gN[a][0] + G[i][1] * gN[a][1] + G[i][2] * gN[a][2]);
        }
    }
    asm volatile("" ::: "memory");
    if (CONV == kGeneral) {
        const T atw = P.conv_a * (W[0][0] + W[1][1] + W[2][2]);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int j = 0; j < 3; ++j) M[k][j] += P.conv_b * W[j][k];
            M[k][k] += atw;
        }
    }
    if (EDDY != kNoEddy) add_scaled_eddy_d<T, EDDY>(G, ed, vol * phi, M);
    const T at = (CONV == kGeneral) ? P.conv_a * (G[0][0] + G[1][1] + G[2][2]) : T(0);
    // (K^T w)_k = (G^T w)_k + conv_a tr(G) w_k + conv_b (G w)_k
    auto kt = [&](const T (&w)[3], T (&kw)[3]) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            kw[k] = G[0][k] * w[0] + G[1][k] * w[1] + G[2][k] * w[2];
            if (CONV == kGeneral) kw[k] += at * w[k] + P.conv_b * (G[k][0] * w[0] + G[k][1] * w[1] + G[k][2] * w[2]);
        }
    };
    // K^T (lambda_b + L) = K^T lambda_b + K^T L, and sum_b g_b = -5 (rho V / 20) K^T L
    T c0[3], gsum[3];
    kt(L, c0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c0[k] *= sc;
        gsum[k] = T(-5) * c0[k];
    }
#pragma unroll
    for (int b = 1; b < 4; ++b) {
        T lb[3], kw[3], ge[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) lb[j] = ldl(b, j);
        kt(lb, kw);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T g = -c0[k];
            g -= sc * kw[k];
            g -= M[k][0] * gN[b][0];
            g -= M[k][1] * gN[b][1];
            g -= M[k][2] * gN[b][2];
            ge[k] = g;
            gsum[k] -= g;
        }
        emit(b, ge);
    }
    emit(0, gsum);
}

// Pressure VJP: the pressure term -(V/4) q at every vertex is linear in p,
// so lambda . R^p = -(V/4) L . q with L = sum_a lambda_a and
// d/dp_b = -(V/4) L . grad N_b.
template <typename T, typename Sink>
__device__ inline void element_vjp_p(const T (&gN)[4][3], T vol, const T (&le)[4][3], Sink &&emit) {
    const T w = -vol * T(0.25);
    T L[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) L[i] = le[0][i] + le[1][i] + le[2][i] + le[3][i];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const T gp[3] = {w * (L[0] * gN[b][0] + L[1] * gN[b][1] + L[2] * gN[b][2]), T(0), T(0)};
        emit(b, gp);
    }
}

// JVP: directional derivative of R^e_a = b - G y_a along (du, dp):
//   dR^e_a = -(V/4) dq - dG y_a - G dy_a,
//   dy_a = (rho V / 20)(du_a + dU) + V (D : dG) grad N_a,
// with dG = grad du, dq = grad dp and D = d mu_t / d G.
template <typename T, int EDDY, int CONV, typename Sink>
__device__ inline void element_jvp(const T (&gN)[4][3], T vol, const T (&ue)[4][3], const T (&due)[4][3],
                                   const T (&dpe)[4], const KParams<T> &P, Sink &&emit) {
    T G[3][3], dG[3][3], dq[3];
    vector_gradient(gN, ue, G);
    vector_gradient(gN, due, dG);
    {
        const T d1 = dpe[1] - dpe[0], d2 = dpe[2] - dpe[0], d3 = dpe[3] - dpe[0];
#pragma unroll
        for (int j = 0; j < 3; ++j) dq[j] = d1 * gN[1][j] + d2 * gN[2][j] + d3 * gN[3][j];
    }
    T D[3][3];
    const T mu_e = P.mu + eddy_viscosity<T, EDDY, true>(G, vol, P.rho_c, D);
    T dmu = T(0);
    if (EDDY != kNoEddy) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) dmu += D[i][j] * dG[i][j];
    }
    const T sc = P.rho * vol * T(0.05);
    const T sv = mu_e * vol, dsv = dmu * vol, w4 = vol * T(0.25);
    T U[3], dU[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        U[i] = ue[0][i] + ue[1][i] + ue[2][i] + ue[3][i];
        dU[i] = due[0][i] + due[1][i] + due[2][i] + due[3][i];
    }
    // general form: the extra term E z_a, E = conv_a tr(G) I + conv_b G^T,
    // z_a = (rho V / 20)(u_a + U), differentiates to dE z_a + E dz_a
    const T at = (CONV == kGeneral) ? P.conv_a * (G[0][0] + G[1][1] + G[2][2]) : T(0);
    const T dat = (CONV == kGeneral) ? P.conv_a * (dG[0][0] + dG[1][1] + dG[2][2]) : T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        T z[3], dz[3], y[3], dy[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            z[j] = sc * (ue[a][j] + U[j]);
            dz[j] = sc * (due[a][j] + dU[j]);
            y[j] = z[j] + sv * gN[a][j];
            dy[j] = dz[j] + dsv * gN[a][j];
        }
        T dr[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            dr[i] = -w4 * dq[i] - (dG[i][0] * y[0] + dG[i][1] * y[1] + dG[i][2] * y[2]) -
                    (G[i][0] * dy[0] + G[i][1] * dy[1] + G[i][2] * dy[2]);
            if (CONV == kGeneral)
                dr[i] -= dat * z[i] + at * dz[i] +
                            P.conv_b * (dG[0][i] * z[0] + dG[1][i] * z[1] + dG[2][i] * z[2] +
                                        G[0][i] * dz[0] + G[1][i] * dz[1] + G[2][i] * dz[2]);
        }
        emit(a, dr);
    }
}

// The element operation of a launch mode on gathered vertex data.  Each
// vertex's contribution is handed to emit(a, value[3]) as soon as it is
// known, so that it need not stay in registers until the element is done.
template <typename T, int EDDY, int CONV, int MODE, typename Sink>
__device__ inline void element_op(const T (&gN)[4][3], T vol, const T (&ea)[4][3], const T (&eb)[4][3],
                                  const T (&ec)[4], const KParams<T> &P, Sink &&emit) {
    if constexpr (MODE == kForward)
        element_rhs<T, EDDY, CONV>(gN, vol, [&](int a, int i) { return ea[a][i]; }, ec, P, emit);
    if constexpr (MODE == kVjp)
        element_vjp<T, EDDY, CONV>(
            gN, vol, [&](int a, int i) { return ea[a][i]; }, [&](int a, int i) { return eb[a][i]; }, P, emit);
    if constexpr (MODE == kVjpP) element_vjp_p(gN, vol, eb, emit);
    if constexpr (MODE == kJvp) element_jvp<T, EDDY, CONV>(gN, vol, ea, eb, ec, P, emit);
    if constexpr (MODE == kMass) {
        // row-sum lumping of the P1 mass matrix: sum_b int N_a N_b = V/4
        const T w[3] = {vol * T(0.25), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < 4; ++a) emit(a, w);
    }
}

// The geometry in the field precision.  In FP32, grad N_0 = -(grad N_1 +
// grad N_2 + grad N_3) is formed from the rounded gradients (three
// conversions fewer; its FP64 value is then never computed).
template <typename T>
__device__ inline void to_field(const double (&g64)[4][3], double vol64, T (&gN)[4][3], T &vol) {
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) gN[a][i] = static_cast<T>(g64[a][i]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
        gN[0][i] = std::is_same<T, double>::value ? static_cast<T>(g64[0][i]) : -(gN[1][i] + gN[2][i] + gN[3][i]);
    vol = static_cast<T>(vol64);
}

// Newton steps of the reciprocal in tet_geometry for field type T.
template <typename T>
constexpr int kGeomNewton = std::is_same<T, double>::value ? 2 : 1;

// ------------------------------------------------------------- kernels

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_zero(T *p, int64_t n) {
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; k < n;
         k += static_cast<int64_t>(gridDim.x) * kThreads)
        p[k] = T(0);
}

// Node fields of a launch (see Mode); fc may be null (read as 0).
template <typename T>
struct NodeFields {
    const T *fa;
    const T *fb;
    const T *fc;
};

// One thread per element, NOUT global atomic adds per vertex.
template <typename T, int EDDY, int CONV, int MODE>
__global__ __launch_bounds__(kThreads) void k_assemble_atomic(int64_t ne, const int4 *__restrict__ conn,
                                                               const double *__restrict__ x, NodeFields<T> F,
                                                               KParams<T> P, T *__restrict__ out) {
    using FL = Fields<MODE>;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t e = tile * kThreads + threadIdx.x;
    if (e >= ne) return;
    const int4 c = conn[e];
    const int64_t ids[4] = {c.x, c.y, c.z, c.w};
    double xe[4][3];
    T ea[4][3] = {}, eb[4][3] = {}, ec[4] = {};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            xe[a][i] = x[3 * ids[a] + i];
            if (FL::NA) ea[a][i] = F.fa[3 * ids[a] + i];
            if (FL::NB) eb[a][i] = F.fb[3 * ids[a] + i];
        }
        if (FL::NC) ec[a] = F.fc ? F.fc[ids[a]] : T(0);
    }
    double g64[4][3], vol64;
    tet_geometry<kGeomNewton<T>>(xe, g64, vol64);
    T gN[4][3], vol;
    to_field(g64, vol64, gN, vol);
    element_op<T, EDDY, CONV, MODE>(gN, vol, ea, eb, ec, P, [&](int a, const T (&r)[3]) {
#pragma unroll
        for (int i = 0; i < FL::NOUT; ++i) global_add(&out[FL::NOUT * ids[a] + i], r[i]);
    });
}

// acc = sum of the slots [beg, end) of every component, in a fixed order.
// FP64: chunks of four whose loads are independent (the run is read in
// parallel, not one LDS round trip per slot); a read past the run's end is
// pointed at slot ZERO, which holds 0, so that every load is unconditional
// and no value needs masking.  FP32: blocks of four slots, then at most one
// pair and one single slot (fewer instructions; in FP64 these tails measured
// slower, as they add dependent LDS round trips).
template <typename T, int NOUT, int KS, int ZERO>
__device__ inline void run_sum(const T (*sval)[KS], int beg, int end, T (&acc)[NOUT]) {
#pragma unroll
    for (int i = 0; i < NOUT; ++i) acc[i] = T(0);
    if constexpr (std::is_same<T, double>::value) {
        for (int k = beg; k < end; k += 4) {
            T v[4][NOUT];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int kk = k + j < end ? k + j : ZERO;
#pragma unroll
                for (int i = 0; i < NOUT; ++i) v[j][i] = sval[i][kk];
            }
#pragma unroll
            for (int i = 0; i < NOUT; ++i) acc[i] += (v[0][i] + v[1][i]) + (v[2][i] + v[3][i]);
        }
    } else {
        int k = beg;
        for (; k + 4 <= end; k += 4) {
#pragma unroll
            for (int i = 0; i < NOUT; ++i)
                acc[i] += (sval[i][k] + sval[i][k + 1]) + (sval[i][k + 2] + sval[i][k + 3]);
        }
        if (k + 2 <= end) {
#pragma unroll
            for (int i = 0; i < NOUT; ++i) acc[i] += sval[i][k] + sval[i][k + 1];
            k += 2;
        }
        if (k < end) {
#pragma unroll
            for (int i = 0; i < NOUT; ++i) acc[i] += sval[i][k];
        }
    }
}

// One workgroup per patch (see the file header).  Thread t loads patch
// record t (node id, slot run, LDS position; records are padded to a fixed
// stride) and stages the node's coordinates and fields at that position;
// element t reads its vertices at the positions elem_loc gives (chosen at
// mesh creation to spread LDS banks).  Then, reusing the same bytes, the
// element contributions go to their precomputed slots: slots are sorted by
// node, so each node's contributions form one contiguous run that one thread
// sums in a fixed order.  GATHER = false adds each node sum to `out` with a
// global atomic; GATHER = true stores it to the node-major partial-sum buffer
// (position patch_ref of the record), for k_gather_partials.
// Minimum waves per SIMD the register allocator is held to: every FP64
// forward fits six (its LDS allows six workgroups per CU) and the FP64
// advective VJP without eddy viscosity five, without spilling; the advective
// Smagorinsky VJP runs five too, spilling 12 bytes per lane (2-4 % faster
// than four waves without spills); the other FP64 VJPs would spill more and
// the FP32 kernels need no hint, so the compiler chooses.
template <typename T, int EDDY, int CONV, int MODE>
constexpr int kPatchMinWaves =
    (std::is_same<T, double>::value && MODE == kForward)                                        ? 6
    : (std::is_same<T, double>::value && MODE == kVjp && EDDY != kVreman && CONV == kAdvective) ? 5
                                                                                                : 1;

template <typename T, int EDDY, int CONV, int MODE, bool GATHER>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kPatchMinWaves<T, EDDY, CONV, MODE>))) void k_assemble_patch(
    int64_t ne, int64_t np, int32_t patch_elems, int32_t stride, const int2 *__restrict__ patch_rec,
    const int32_t *__restrict__ patch_ref, const ushort4 *__restrict__ elem_pos,
    const uchar4 *__restrict__ elem_loc, const double *__restrict__ x,
    NodeFields<T> F, KParams<T> P, T *__restrict__ out) {
    using FL = Fields<MODE>;
    // kS slots per component, then (FP64) a zero slot that reads past a run
    // end are pointed at; rows padded to keep 16-byte alignment
    constexpr int kN = kMaxPatchNodes, kS = 4 * kMaxPatchElems;
    constexpr int kSP = std::is_same<T, double>::value ? kS + 8 : kS;
    constexpr int kNF = FL::NA + FL::NB + FL::NC;
    // The forwards and the FP64 velocity and pressure VJPs pad each row of
    // the node arrays by 32 floats / 16 doubles, so that the fields of one node lie in different
    // LDS bank pairs: with 256-entry rows the compiler pairs the reads of two
    // fields of a vertex into one instruction whose two addresses share a
    // bank pair.  Measured at 96^3 / 160^3: FP64 forward 66.8 -> 63.9 us, with
    // Smagorinsky 96-102 -> 91-92 us (once its eddy model lost its library
    // calls), FP64 advective VJP 81.2 -> 78.9 us (held to five waves, see
    // kPatchMinWaves), FP64 VJPs with an eddy model -5 to -9 %, with the
    // other convective forms -1 to -7 %, FP64 pressure VJP -4 %, FP32
    // forward -2 %.  The FP32 VJPs measured slower with it (instruction mix,
    // registers) and keep 256-entry rows; the FP64 JVPs would lose a wave
    // per SIMD (or spill) and keep them too.
    constexpr bool kPadRows =
        MODE == kForward ||
        (std::is_same<T, double>::value && (MODE == kVjp || MODE == kVjpP));
    constexpr int kNR = kN + (kPadRows ? (std::is_same<T, double>::value ? 16 : 32) : 0);
    constexpr size_t kNodeBytes = 3 * kNR * sizeof(double) + kNF * kNR * sizeof(T);
    constexpr size_t kSlotBytes = FL::NOUT * kSP * sizeof(T);
    // The FP64 forward and VJP read u_a (and lambda_a) from LDS where they use
    // them (twice each) instead of holding all four vertices in registers,
    // which keeps the forward at six waves per SIMD (five otherwise) and the
    // VJP at five (four otherwise).  The FP32 kernels hold them in registers
    // and still run seven or eight waves, except the VJP of a general
    // convective form with an eddy model, which would lose a wave.
    constexpr bool kLds = ((MODE == kForward || MODE == kVjp) && std::is_same<T, double>::value) ||
                          (MODE == kVjp && EDDY != kNoEddy && CONV == kGeneral);
    __shared__ __align__(16) unsigned char smem[kNodeBytes > kSlotBytes ? kNodeBytes : kSlotBytes];
    double(*sx)[kNR] = reinterpret_cast<double(*)[kNR]>(smem);
    T(*sf)[kNR] = reinterpret_cast<T(*)[kNR]>(smem + 3 * kNR * sizeof(double));  // A, then B, then C
    T(*sval)[kSP] = reinterpret_cast<T(*)[kSP]>(smem);

    const int64_t patch = xcd_tile(blockIdx.x, gridDim.x);
    if (patch >= np) return;
    const int t = threadIdx.x;
    const int64_t first = patch * static_cast<int64_t>(patch_elems);
    const int nel = static_cast<int>(min<int64_t>(patch_elems, ne - first));
    // Every load of the patch's description is independent of the others, so
    // all three are issued at once, unconditionally (indices clamped into the
    // patch: a patch has at least one element and its record stride is at
    // least 8; lanes beyond them discard what they read).  The record comes
    // first, as the node loads depend on it, and the element tables stay
    // packed words until after the node staging, so that waiting for the
    // record does not wait for them: unpacked at the load, they cost every
    // workgroup one more memory round trip before its node loads could start.
    const int2 rec = patch_rec[patch * stride + min(t, stride - 1)];
    const int64_t te = first + min(t, nel - 1);
    const uint2 pos_w = reinterpret_cast<const uint2 *>(elem_pos)[te];   // four 16-bit slot positions
    const uint32_t loc_w = reinterpret_cast<const uint32_t *>(elem_loc)[te];  // four 8-bit LDS positions
    int32_t slot = 0, s_beg = 0, s_end = 0;
    const int64_t node = t < stride ? rec.x : -1;
    const int lp = static_cast<int>(static_cast<uint32_t>(rec.y) >> 22);  // the node's LDS position
    const bool has_node = node >= 0;
    if (has_node) {
        // every load of the node before the first LDS store, so that they
        // form one round trip (the scalar field's null check would otherwise
        // hold its load back until the others had been stored)
        double xv[3];
        T av[3] = {}, bv[3] = {}, cv = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            xv[i] = x[3 * node + i];
            if (FL::NA) av[i] = F.fa[3 * node + i];
            if (FL::NB) bv[i] = F.fb[3 * node + i];
        }
        if (FL::NC && F.fc) cv = F.fc[node];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            sx[i][lp] = xv[i];
            if (FL::NA) sf[i][lp] = av[i];
            if (FL::NB) sf[FL::NA + i][lp] = bv[i];
        }
        if (FL::NC) sf[FL::NA + FL::NB][lp] = cv;
    }
    __syncthreads();

    T r[4][3];
    if (t < nel) {
        const int la[4] = {static_cast<int>(loc_w & 0xffu), static_cast<int>((loc_w >> 8) & 0xffu),
                           static_cast<int>((loc_w >> 16) & 0xffu), static_cast<int>(loc_w >> 24)};
        double xe[4][3];
        T ea[4][3] = {}, eb[4][3] = {}, ec[4] = {};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                xe[a][i] = sx[i][la[a]];
                if (FL::NA && !kLds) ea[a][i] = sf[i][la[a]];
                if (FL::NB && !kLds) eb[a][i] = sf[FL::NA + i][la[a]];
            }
            if (FL::NC) ec[a] = sf[FL::NA + FL::NB][la[a]];
        }
        double g64[4][3], vol64;
        tet_geometry<kGeomNewton<T>>(xe, g64, vol64);
        T gN[4][3], vol;
        to_field(g64, vol64, gN, vol);
        auto sink = [&](int a, const T (&v)[3]) {
#pragma unroll
            for (int i = 0; i < FL::NOUT; ++i) r[a][i] = v[i];
        };
        auto ldu = [&](int a, int i) { return sf[i][la[a]]; };
        if constexpr (kLds && MODE == kForward)
            element_rhs<T, EDDY, CONV>(gN, vol, ldu, ec, P, sink);
        else if constexpr (kLds && MODE == kVjp)
            element_vjp<T, EDDY, CONV>(gN, vol, ldu, [&](int a, int i) { return sf[3 + i][la[a]]; }, P, sink);
        else
            element_op<T, EDDY, CONV, MODE>(gN, vol, ea, eb, ec, P, sink);
    }
    __syncthreads();  // node data is dead from here on; its bytes become slots
    if (t < nel) {
        const int sl[4] = {static_cast<int>(pos_w.x & 0xffffu), static_cast<int>(pos_w.x >> 16),
                           static_cast<int>(pos_w.y & 0xffffu), static_cast<int>(pos_w.y >> 16)};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < FL::NOUT; ++i) sval[i][sl[a]] = r[a][i];
    }
    if (kSP > kS && t < FL::NOUT) sval[t][kS] = T(0);
    __syncthreads();
    // the slot run comes from the record word loaded at the start; the
    // partial-sum position is loaded now (an L2 hit) and first used after
    // the run reduction, which hides its latency
    if (GATHER && has_node) slot = patch_ref[patch * stride + t];
    s_beg = rec.y & 0x7ff;
    s_end = (rec.y >> 11) & 0x7ff;
    if (has_node) {
        T acc[FL::NOUT];
        run_sum<T, FL::NOUT, kSP, kS>(sval, s_beg, s_end, acc);
        if (GATHER) {
#pragma unroll
            for (int i = 0; i < FL::NOUT; ++i) out[FL::NOUT * static_cast<int64_t>(slot) + i] = acc[i];
        } else {
#pragma unroll
            for (int i = 0; i < FL::NOUT; ++i) global_add(&out[FL::NOUT * node + i], acc[i]);
        }
    }
}

// acc = sum of the partial sums [kb, ke), in a fixed order: chunks of four
// whose loads are all issued before any is used (most nodes have at most four
// partial sums, so one round trip to memory); an index past the run is
// clamped to its first entry (the loop body runs only when the run is not
// empty) and the value masked.  Reference indices fit int32 (at most 2 Ne <
// 2^30); the element offsets are formed in 64 bits.
template <typename T, int NOUT>
__device__ inline void gather_sum(const T *__restrict__ partial, int kb, int ke, T (&acc)[NOUT]) {
#pragma unroll
    for (int i = 0; i < NOUT; ++i) acc[i] = T(0);
    for (int k = kb; k < ke; k += 4) {
        T v[4][NOUT];
        bool in[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            in[j] = k + j < ke;
            const int kk = in[j] ? k + j : kb;
#pragma unroll
            for (int i = 0; i < NOUT; ++i) v[j][i] = partial[NOUT * static_cast<int64_t>(kk) + i];
        }
#pragma unroll
        for (int i = 0; i < NOUT; ++i)
            acc[i] += (v[0][i] + (in[1] ? v[1][i] : T(0))) + ((in[2] ? v[2][i] : T(0)) + (in[3] ? v[3][i] : T(0)));
    }
}

// out[n] (+)= sum of node n's patch partial sums, which are stored
// contiguously (node-major, patch order) at [ref_off[n], ref_off[n+1]).
template <typename T, int NOUT>
__global__ __launch_bounds__(kThreads) void k_gather_partials(int64_t nn, const int32_t *__restrict__ ref_off,
                                                               const T *__restrict__ partial, T *__restrict__ out,
                                                               int accumulate) {
    const int64_t n = xcd_tile(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (n >= nn) return;
    T acc[NOUT];
    gather_sum<T, NOUT>(partial, ref_off[n], ref_off[n + 1], acc);
#pragma unroll
    for (int i = 0; i < NOUT; ++i) out[NOUT * n + i] = accumulate ? out[NOUT * n + i] + acc[i] : acc[i];
}

// dt / (rho V^L_n), the explicit-update weight of node n; 0 for a node that no
// element references (V^L_n = 0: no mass and no residual, so u stays).
template <typename T>
__device__ inline T update_weight(double lumped, double rho, double dt) {
    return lumped > 0.0 ? static_cast<T>(dt / (rho * lumped)) : T(0);
}

// Explicit momentum stage fused into the gather: rhs_n is summed from the
// patch partials as in k_gather_partials, optionally stored, and
//   u_new[n, i] = u[n, i] + dt rhs[n, i] / (rho V^L_n)
// for components whose bit i of mask[n] is clear (u_new[n, i] = u[n, i]
// otherwise, and at nodes with V^L_n = 0).  u_new may be u itself: each thread reads and writes only its
// own node.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_update(int64_t nn, const int32_t *__restrict__ ref_off,
                                                            const T *__restrict__ partial,
                                                            const double *__restrict__ lumped, double rho,
                                                            double dt, const T *u, const uint8_t *__restrict__ mask,
                                                            T *__restrict__ rhs, T *u_new) {
    const int64_t n = xcd_tile(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (n >= nn) return;
    T acc[3];
    gather_sum<T, 3>(partial, ref_off[n], ref_off[n + 1], acc);
    if (rhs) {
#pragma unroll
        for (int i = 0; i < 3; ++i) rhs[3 * n + i] = acc[i];
    }
    const T w = update_weight<T>(lumped[n], rho, dt);
    const unsigned fixed = mask ? mask[n] : 0u;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T ui = u[3 * n + i];
        u_new[3 * n + i] = ((fixed >> i) & 1u) ? ui : ui + w * acc[i];
    }
}

// The same update from an assembled rhs (atomic and patch scatters).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_update(int64_t nn, const T *__restrict__ rhs,
                                                     const double *__restrict__ lumped, double rho, double dt,
                                                     const T *u, const uint8_t *__restrict__ mask, T *u_new) {
    const int64_t n = xcd_tile(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (n >= nn) return;
    const T w = update_weight<T>(lumped[n], rho, dt);
    const unsigned fixed = mask ? mask[n] : 0u;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T ui = u[3 * n + i];
        u_new[3 * n + i] = ((fixed >> i) & 1u) ? ui : ui + w * rhs[3 * n + i];
    }
}

// ---------------------------------------------------------- host side

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + nb && pb < pa + na;
}

nsasm_status check_params(const nsasm_params *p) {
    if (!p) return fail(NSASM_ERR_INVALID_ARGUMENT, "params is NULL");
    const double vals[6] = {p->rho, p->mu, p->smagorinsky_cs, p->body_force[0], p->body_force[1],
                            p->body_force[2]};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(NSASM_ERR_INVALID_ARGUMENT, "parameters must be finite");
    if (!(p->rho > 0.0)) return fail(NSASM_ERR_INVALID_ARGUMENT, "rho must be > 0");
    if (p->mu < 0.0) return fail(NSASM_ERR_INVALID_ARGUMENT, "mu must be >= 0");
    if (p->smagorinsky_cs < 0.0) return fail(NSASM_ERR_INVALID_ARGUMENT, "smagorinsky_cs must be >= 0");
    if (p->flags & ~NSASM_ACCUMULATE) return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", p->flags);
    if (p->eddy_model != NSASM_EDDY_SMAGORINSKY && p->eddy_model != NSASM_EDDY_VREMAN)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown eddy_model %u", p->eddy_model);
    if (p->convective_form > NSASM_CONVECTIVE_EMAC)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown convective_form %u", p->convective_form);
    if (p->reserved != 0) return fail(NSASM_ERR_INVALID_ARGUMENT, "reserved must be 0");
    return NSASM_OK;
}

template <typename T>
KParams<T> kernel_params(const nsasm_params &p) {
    KParams<T> k;
    k.rho = static_cast<T>(p.rho);
    k.mu = static_cast<T>(p.mu);
    const double c = (p.eddy_model == NSASM_EDDY_VREMAN ? 2.5 : 1.0) * p.smagorinsky_cs * p.smagorinsky_cs;
    k.rho_c = static_cast<T>(p.rho * c);
    for (int i = 0; i < 3; ++i) k.rho_f[i] = static_cast<T>(p.rho * p.body_force[i]);
    // c = G u + a tr(G) u + b G^T u, from div(u (x) u) = G u + tr(G) u and
    // (curl u) x u = G u - G^T u
    static const double kForm[5][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.5, 0.0}, {0.0, -1.0}, {1.0, 1.0}};
    k.conv_a = static_cast<T>(kForm[p.convective_form][0]);
    k.conv_b = static_cast<T>(kForm[p.convective_form][1]);
    return k;
}

// Explicit-update epilogue of a forward launch (see k_gather_update).
template <typename T>
struct Update {
    double rho, dt;
    const T *u;
    const uint8_t *mask;
    T *rhs;  // may be null
    T *u_new;
};

// One kernel launch of kThreads-wide workgroups on `s`.  With a start or
// stop event (nsasm_set_kernel_events) it goes through hipExtLaunchKernelGGL,
// which records the events at the kernel's own start and end.
template <typename... KArgs, typename... Args>
nsasm_status launch_kernel(void (*kernel)(KArgs...), unsigned grid, hipStream_t s, hipEvent_t start,
                           hipEvent_t stop, const char *what, Args... args) {
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), 0, s, start, stop, 0, args...);
    else
        kernel<<<grid, kThreads, 0, s>>>(args...);
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? NSASM_OK : hip_fail(err, what);
}

// With the gather scatter and `up` set, the gather kernel applies the
// explicit update instead of writing `out`.  `ev` times the element kernel
// and the gather kernel (events may be null).  `partial` (may be null: the
// mesh's own buffer) receives the per-patch node sums of the gather scatter.
template <typename T, int EDDY, int CONV, int MODE>
nsasm_status launch(const nsasm_mesh *m, const KParams<T> &kp, NodeFields<T> F, T *out, bool accumulate,
                    const Update<T> *up, const KernelEvents &ev, hipStream_t s, T *partial = nullptr) {
    constexpr int NOUT = Fields<MODE>::NOUT;
    if (m->scatter == NSASM_SCATTER_PATCH_GATHER) {
        if (!partial) partial = reinterpret_cast<T *>(m->partial);
        NSASM_TRY(launch_kernel(k_assemble_patch<T, EDDY, CONV, MODE, true>, xcd_grid(m->n_patches), s,
                                ev.element_start, ev.element_stop, "patch kernel launch", m->n_elems, m->n_patches,
                                m->patch_elems, m->patch_stride, m->patch_rec, m->patch_ref, m->elem_pos,
                                m->elem_loc, m->x, F, kp, partial));
        const int64_t tiles = (m->n_nodes + kThreads - 1) / kThreads;
        if constexpr (MODE == kForward) {
            if (up)
                return launch_kernel(k_gather_update<T>, xcd_grid(tiles), s, ev.gather_start, ev.gather_stop,
                                     "update kernel launch", m->n_nodes, m->node_ref_off, partial, m->lumped, up->rho,
                                     up->dt, up->u, up->mask, up->rhs, up->u_new);
        }
        return launch_kernel(k_gather_partials<T, NOUT>, xcd_grid(tiles), s, ev.gather_start, ev.gather_stop,
                             "gather kernel launch", m->n_nodes, m->node_ref_off, partial, out, accumulate ? 1 : 0);
    }
    if (m->scatter == NSASM_SCATTER_PATCH)
        return launch_kernel(k_assemble_patch<T, EDDY, CONV, MODE, false>, xcd_grid(m->n_patches), s,
                             ev.element_start, ev.element_stop, "patch kernel launch", m->n_elems, m->n_patches,
                             m->patch_elems, m->patch_stride, m->patch_rec, m->patch_ref, m->elem_pos, m->elem_loc,
                             m->x, F, kp, out);
    const int64_t tiles = (m->n_elems + kThreads - 1) / kThreads;
    return launch_kernel(k_assemble_atomic<T, EDDY, CONV, MODE>, xcd_grid(tiles), s, ev.element_start,
                         ev.element_stop, "assembly kernel launch", m->n_elems, m->conn, m->x, F, kp, out);
}

template <typename T, int CONV, int MODE>
nsasm_status launch_eddy(const nsasm_mesh *m, const nsasm_params &p, const KParams<T> &kp, NodeFields<T> F, T *o,
                         const Update<T> *up, const KernelEvents &ph, hipStream_t s, T *partial) {
    const bool accumulate = (p.flags & NSASM_ACCUMULATE) != 0;
    if (p.smagorinsky_cs > 0.0 && p.eddy_model == NSASM_EDDY_VREMAN)
        return launch<T, kVreman, CONV, MODE>(m, kp, F, o, accumulate, up, ph, s, partial);
    if (p.smagorinsky_cs > 0.0)
        return launch<T, kSmagorinsky, CONV, MODE>(m, kp, F, o, accumulate, up, ph, s, partial);
    return launch<T, kNoEddy, CONV, MODE>(m, kp, F, o, accumulate, up, ph, s, partial);
}

// Physics selection (convective form, eddy viscosity) of a launch.
template <typename T, int MODE>
nsasm_status dispatch(const nsasm_mesh *m, const nsasm_params &p, NodeFields<T> F, T *o, const Update<T> *up,
                      const KernelEvents &ph, hipStream_t s, T *partial = nullptr) {
    const KParams<T> kp = kernel_params<T>(p);
    if constexpr (MODE == kVjpP) {
        // the pressure term depends on neither the viscosity nor the convective form
        return launch<T, kNoEddy, kAdvective, MODE>(m, kp, F, o, (p.flags & NSASM_ACCUMULATE) != 0, up, ph, s,
                                                    partial);
    } else {
        if (p.convective_form != NSASM_CONVECTIVE_ADVECTIVE)
            return launch_eddy<T, kGeneral, MODE>(m, p, kp, F, o, up, ph, s, partial);
        return launch_eddy<T, kAdvective, MODE>(m, p, kp, F, o, up, ph, s, partial);
    }
}

template <typename T>
nsasm_status fill_zero(T *o, int64_t n, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
    k_fill_zero<T><<<static_cast<unsigned>(blocks), kThreads, 0, s>>>(o, n);
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? NSASM_OK : hip_fail(err, "fill kernel launch");
}

template <typename T, int MODE>
nsasm_status run(const nsasm_mesh *m, const nsasm_params &p, const void *fa, const void *fb, const void *fc,
                 void *out, const KernelEvents &ph, hipStream_t s, void *partial) {
    T *o = static_cast<T *>(out);
    const bool accumulate = (p.flags & NSASM_ACCUMULATE) != 0;
    // the gather kernel writes every node, so it needs no zero-fill
    if (!accumulate && m->scatter != NSASM_SCATTER_PATCH_GATHER)
        NSASM_TRY(fill_zero(o, Fields<MODE>::NOUT * m->n_nodes, s));
    const NodeFields<T> F{static_cast<const T *>(fa), static_cast<const T *>(fb), static_cast<const T *>(fc)};
    return dispatch<T, MODE>(m, p, F, o, nullptr, ph, s, static_cast<T *>(partial));
}

// ------------------------------------------------ allocation-free variant
// The partial sums of nsasm_assemble_rhs_noalloc live in this fixed region
// rather than in the mesh's buffer.  Each GPU holds its own copy from the
// library's module load until the process ends.  In host code `scratch` is
// only a host-side handle of the symbol: its device address on the current
// GPU comes from hipGetSymbolAddress and is what the kernels receive.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
std::atomic<void *> g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device, resolved once per
// device (with that device current) and kept.
nsasm_status scratch_address(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(NSASM_ERR_UNSUPPORTED, "device %d is beyond the %d devices the library tracks", device,
                    kMaxDevices);
    void *p = g_scratch_ptr[device].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        p = g_scratch_ptr[device].load(std::memory_order_relaxed);
        if (!p) {
            hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (err != hipSuccess || !p) {
                (void)hipGetLastError();
                return fail(NSASM_ERR_DEVICE, "hipGetSymbolAddress of the scratch region failed: %s",
                            hipGetErrorString(err));
            }
            g_scratch_ptr[device].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return NSASM_OK;
}

// Forward assembly and the explicit update: fused into the gather kernel with
// the gather scatter, else assembled into `rhs` and updated by k_update.
template <typename T>
nsasm_status run_update(const nsasm_mesh *m, const nsasm_params &p, double dt, const void *u, const void *pr,
                        const uint8_t *mask, void *rhs, void *u_new, const KernelEvents &ph, hipStream_t s) {
    const NodeFields<T> F{static_cast<const T *>(u), nullptr, static_cast<const T *>(pr)};
    T *r = static_cast<T *>(rhs);
    const Update<T> up{p.rho, dt, static_cast<const T *>(u), mask, r, static_cast<T *>(u_new)};
    if (m->scatter == NSASM_SCATTER_PATCH_GATHER) return dispatch<T, kForward>(m, p, F, nullptr, &up, ph, s);
    NSASM_TRY(fill_zero(r, 3 * m->n_nodes, s));
    NSASM_TRY((dispatch<T, kForward>(m, p, F, r, nullptr, ph, s)));
    const int64_t tiles = (m->n_nodes + kThreads - 1) / kThreads;
    return launch_kernel(k_update<T>, xcd_grid(tiles), s, ph.gather_start, ph.gather_stop, "update kernel launch",
                         m->n_nodes, static_cast<const T *>(r), static_cast<const double *>(m->lumped), p.rho, dt,
                         up.u, mask, up.u_new);
}

// One device array argument of an entry point: name, pointer, components per
// node (0: not used by the mode), whether NULL is allowed.
struct Arg {
    const char *name;
    const void *ptr;
    int ncomp;
    bool nullable;
};

// With `no_alloc` the gather scatter's partial sums go to the static scratch
// region instead of the mesh's buffer.
template <int MODE>
nsasm_status entry(const nsasm_mesh *m, const nsasm_params *params, nsasm_precision prec, Arg a, Arg b, Arg c,
                   Arg out, void *stream, bool no_alloc = false) {
    const KernelEvents ph = take_kernel_events();  // consumed by this call, whatever its outcome
    if (!m) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    NSASM_TRY(check_params(params));
    if (prec != NSASM_FP64 && prec != NSASM_MIXED)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown precision %d", static_cast<int>(prec));
    const size_t es = (prec == NSASM_FP64) ? sizeof(double) : sizeof(float);
    const Arg inputs[3] = {a, b, c};
    NSASM_TRY(check_device_ptr(out.ptr, out.name));
    const size_t out_bytes = static_cast<size_t>(out.ncomp) * m->n_nodes * es;
    for (const Arg &in : inputs) {
        if (in.ncomp == 0 || (in.nullable && in.ptr == nullptr)) continue;
        NSASM_TRY(check_device_ptr(in.ptr, in.name));
        if (overlaps(out.ptr, out_bytes, in.ptr, static_cast<size_t>(in.ncomp) * m->n_nodes * es))
            return fail(NSASM_ERR_INVALID_ARGUMENT, "%s overlaps %s", out.name, in.name);
    }
    void *partial = nullptr;
    if (no_alloc && m->scatter == NSASM_SCATTER_PATCH_GATHER) {
        int dev = 0;
        NSASM_HIP(hipGetDevice(&dev));
        if (dev != m->device)
            return fail(NSASM_ERR_INVALID_ARGUMENT, "the current device (%d) is not the mesh's device (%d)", dev,
                        m->device);
        const size_t need = static_cast<size_t>(Fields<MODE>::NOUT) * static_cast<size_t>(m->patch_node_refs) * es;
        if (need > kScratchBytes)
            return fail(NSASM_ERR_UNSUPPORTED,
                        "the mesh needs %zu bytes of partial sums; the allocation-free call holds at most %zu",
                        need, kScratchBytes);
        NSASM_TRY(scratch_address(dev, &partial));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *o = const_cast<void *>(out.ptr);
    const nsasm_status st = (prec == NSASM_FP64)
                                ? run<double, MODE>(m, *params, a.ptr, b.ptr, c.ptr, o, ph, s, partial)
                                : run<float, MODE>(m, *params, a.ptr, b.ptr, c.ptr, o, ph, s, partial);
    if (st == NSASM_OK) clear_error();
    return st;
}

nsasm_status update_entry(const nsasm_mesh *m, const nsasm_params *params, nsasm_precision prec, double dt,
                          const void *u, const void *p, const uint8_t *mask, void *rhs, void *u_new, void *stream) {
    const KernelEvents ph = take_kernel_events();  // consumed by this call, whatever its outcome
    if (!m) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    NSASM_TRY(check_params(params));
    if (params->flags != 0) return fail(NSASM_ERR_INVALID_ARGUMENT, "flags must be 0 for the explicit update");
    if (prec != NSASM_FP64 && prec != NSASM_MIXED)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown precision %d", static_cast<int>(prec));
    if (!std::isfinite(dt)) return fail(NSASM_ERR_INVALID_ARGUMENT, "dt must be finite");
    const size_t es = (prec == NSASM_FP64) ? sizeof(double) : sizeof(float);
    const size_t vec = 3 * es * m->n_nodes, sca = es * m->n_nodes, mb = static_cast<size_t>(m->n_nodes);
    NSASM_TRY(check_device_ptr(u, "u"));
    NSASM_TRY(check_device_ptr(p, "p"));
    NSASM_TRY(check_device_ptr(u_new, "u_new"));
    if (mask) NSASM_TRY(check_device_ptr(mask, "dirichlet_mask"));
    if (rhs) {
        NSASM_TRY(check_device_ptr(rhs, "rhs"));
    } else if (m->scatter != NSASM_SCATTER_PATCH_GATHER) {
        return fail(NSASM_ERR_INVALID_ARGUMENT, "rhs is required unless the mesh uses the gather scatter");
    }
    if (u_new != u && overlaps(u_new, vec, u, vec))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "u_new must be u itself or not overlap it");
    if (overlaps(u_new, vec, p, sca) || (mask && overlaps(u_new, vec, mask, mb)))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "u_new overlaps p or dirichlet_mask");
    if (rhs && (overlaps(rhs, vec, u, vec) || overlaps(rhs, vec, p, sca) || overlaps(rhs, vec, u_new, vec) ||
                (mask && overlaps(rhs, vec, mask, mb))))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "rhs overlaps another argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const nsasm_status st = (prec == NSASM_FP64) ? run_update<double>(m, *params, dt, u, p, mask, rhs, u_new, ph, s)
                                                 : run_update<float>(m, *params, dt, u, p, mask, rhs, u_new, ph, s);
    if (st == NSASM_OK) clear_error();
    return st;
}

}  // namespace

// V^L_n = sum over elements containing n of V_e / 4, in mesh order, through
// the mesh's own scatter (deterministic with the gather scatter).
nsasm_status compute_lumped_volume(nsasm_mesh *m, hipStream_t s) {
    NSASM_TRY(device_alloc(&m->lumped, static_cast<size_t>(m->n_nodes), "lumped volume"));
    if (m->scatter != NSASM_SCATTER_PATCH_GATHER) NSASM_TRY(fill_zero(m->lumped, m->n_nodes, s));
    const KParams<double> kp{};
    const NodeFields<double> F{nullptr, nullptr, nullptr};
    return launch<double, kNoEddy, kAdvective, kMass>(m, kp, F, m->lumped, false, nullptr, KernelEvents{}, s);
}

}  // namespace nsasm

extern "C" nsasm_status nsasm_assemble_rhs(const nsasm_mesh *mesh, const nsasm_params *params,
                                           nsasm_precision precision, const void *u, const void *p,
                                           void *rhs, void *stream) {
    using namespace nsasm;
    return entry<kForward>(mesh, params, precision, {"u", u, 3, false}, {"unused", nullptr, 0, true},
                           {"p", p, 1, false}, {"rhs", rhs, 3, false}, stream);
}

extern "C" nsasm_status nsasm_assemble_rhs_noalloc(const nsasm_mesh *mesh, const nsasm_params *params,
                                                   nsasm_precision precision, const void *u, const void *p,
                                                   void *rhs, void *stream) {
    using namespace nsasm;
    return entry<kForward>(mesh, params, precision, {"u", u, 3, false}, {"unused", nullptr, 0, true},
                           {"p", p, 1, false}, {"rhs", rhs, 3, false}, stream, true);
}

extern "C" nsasm_status nsasm_assemble_rhs_vjp(const nsasm_mesh *mesh, const nsasm_params *params,
                                               nsasm_precision precision, const void *u,
                                               const void *adjoint, void *grad_u, void *stream) {
    using namespace nsasm;
    return entry<kVjp>(mesh, params, precision, {"u", u, 3, false}, {"adjoint", adjoint, 3, false},
                       {"unused", nullptr, 0, true}, {"grad_u", grad_u, 3, false}, stream);
}

extern "C" nsasm_status nsasm_assemble_rhs_vjp_p(const nsasm_mesh *mesh, const nsasm_params *params,
                                                 nsasm_precision precision, const void *adjoint, void *grad_p,
                                                 void *stream) {
    using namespace nsasm;
    return entry<kVjpP>(mesh, params, precision, {"unused", nullptr, 0, true}, {"adjoint", adjoint, 3, false},
                        {"unused", nullptr, 0, true}, {"grad_p", grad_p, 1, false}, stream);
}

extern "C" nsasm_status nsasm_assemble_rhs_jvp(const nsasm_mesh *mesh, const nsasm_params *params,
                                               nsasm_precision precision, const void *u, const void *du,
                                               const void *dp, void *drhs, void *stream) {
    using namespace nsasm;
    return entry<kJvp>(mesh, params, precision, {"u", u, 3, false}, {"du", du, 3, false}, {"dp", dp, 1, true},
                       {"drhs", drhs, 3, false}, stream);
}

extern "C" nsasm_status nsasm_explicit_update(const nsasm_mesh *mesh, const nsasm_params *params,
                                              nsasm_precision precision, double dt, const void *u, const void *p,
                                              const uint8_t *dirichlet_mask, void *rhs, void *u_new,
                                              void *stream) {
    return nsasm::update_entry(mesh, params, precision, dt, u, p, dirichlet_mask, rhs, u_new, stream);
}
