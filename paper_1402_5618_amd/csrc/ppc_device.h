// Device building blocks of the compact-WENO line operator for gfx950.
//
// Everything here is per-lane arithmetic; the kernels that arrange lanes,
// LDS and HBM traffic live in ppcweno.hip.  Section and equation names refer
// to arXiv 1402.5618 (Guo, Xiong & Shi).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ppc {

// ------------------------------------------------------------ reductions
// Order-preserving map of a double onto int64 so that global atomicMin/Max on
// 64-bit integers give exact, order-independent min/max of doubles.
__device__ __forceinline__ long long ord_enc(double x) {
    long long i = __double_as_longlong(x);
    return i >= 0 ? i : (i ^ 0x7fffffffffffffffLL);
}
__device__ __forceinline__ double ord_dec(long long i) {
    return __longlong_as_double(i >= 0 ? i : (i ^ 0x7fffffffffffffffLL));
}
constexpr long long kEncPosInf = 0x7ff0000000000000LL;  // ord_enc(+inf)
constexpr long long kEncZero = 0;                       // ord_enc(+0.0)

// Reciprocal: hardware estimate refined by Newton steps (two in double,
// one in float) to within an ulp or two; shorter dependency chains than
// the IEEE division sequence.
// A zero or infinite estimate (x = +-0, +-inf) is returned as is, like the
// IEEE quotient, instead of letting the Newton step turn it into NaN.
__device__ __forceinline__ double rcp_t(double x) {
    const double r0 = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r0, 1.0);
    double r = fma(r0, e, r0);
    e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    return (r0 == 0.0 || isinf(r0)) ? r0 : r;
}
// Reciprocal of a finite non-zero value (weight sums, pivots): the same
// estimate and Newton steps without the zero / infinity pass-through.
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
// Square root of a non-negative value (sound speeds, density ratios, the
// limiter's discriminant): the hardware reciprocal-square-root estimate, one
// Goldschmidt iteration for sqrt(x) and 1/(2 sqrt(x)) together, then one
// residual correction g += (x - g^2) h (Markstein's formulation).  x = 0
// returns 0.  Arguments below 2^-767 are outside its design range (the
// products would lose precision); none arise from physical states here.
__device__ __forceinline__ double sqrt_nn(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : x;
}
__device__ __forceinline__ float rcp_t(float x) {
    const float r0 = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r0, 1.0f);
    const float r = fmaf(r0, e, r0);
    return (r0 == 0.0f || isinf(r0)) ? r0 : r;
}

// ------------------------------------------------------- Sec 2.2 weights
// Smoothness indicators of the three candidates of the "-" side at node
// j+1/2 from v0..v4 = ubar_{j-2..j+2}, then WENO-Z weights (power 2) with the
// three divisions of eq. (weight) folded into one reciprocal:
//   alpha_k ~ c_k (d_k^2 + tau^2) * prod_{l != k} d_l^2,  d_k = beta_k + eps.
// Exact in real arithmetic.  In FP64 the products grow like beta^6, so they
// stay finite while differences of neighbouring averages stay below about
// 1e25 (beta below ~1e51); eps keeps them far from underflow.
template <typename T>
__device__ __forceinline__ void wenoz_weights(T v0, T v1, T v2, T v3, T v4, T eps, T& w0, T& w1,
                                              T& w2) {
    const T k13 = T(13) / T(12), k14 = T(0.25);
    T s0 = v0 - T(2) * v1 + v2, t0 = v0 - T(4) * v1 + T(3) * v2;
    T s1 = v1 - T(2) * v2 + v3, t1 = v1 - v3;
    T s2 = v2 - T(2) * v3 + v4, t2 = T(3) * v2 - T(4) * v3 + v4;
    T b0 = k13 * s0 * s0 + k14 * t0 * t0;
    T b1 = k13 * s1 * s1 + k14 * t1 * t1;
    T b2 = k13 * s2 * s2 + k14 * t2 * t2;
    T tau = b2 - b0;
    T tt = tau * tau;
    T d0 = b0 + eps, d1 = b1 + eps, d2 = b2 + eps;
    T e0 = d0 * d0, e1 = d1 * d1, e2 = d2 * d2;
    T a0 = T(0.2) * (e0 + tt) * (e1 * e2);
    T a1 = T(0.5) * (e1 + tt) * (e0 * e2);
    T a2 = T(0.3) * (e2 + tt) * (e0 * e1);
    T inv = rcp_t(a0 + a1 + a2);
    w0 = a0 * inv;
    w1 = a1 * inv;
    w2 = a2 * inv;
}

// Float WENO-Z weights: the product form above under/overflows in float
// (d^6 spans far more than the float range), so evaluate q_k = tau/(beta_k+eps),
// scale by m = max(1, q_0, q_1, q_2) and use alpha_k ~ c_k (1/m^2 + (q_k/m)^2):
// every term stays in [0, 1] and the normalised weights are unchanged.
template <>
__device__ __forceinline__ void wenoz_weights<float>(float v0, float v1, float v2, float v3,
                                                     float v4, float eps, float& w0, float& w1,
                                                     float& w2) {
    const float k13 = 13.0f / 12.0f, k14 = 0.25f;
    const float s0 = v0 - 2.0f * v1 + v2, t0 = v0 - 4.0f * v1 + 3.0f * v2;
    const float s1 = v1 - 2.0f * v2 + v3, t1 = v1 - v3;
    const float s2 = v2 - 2.0f * v3 + v4, t2 = 3.0f * v2 - 4.0f * v3 + v4;
    const float b0 = k13 * s0 * s0 + k14 * t0 * t0;
    const float b1 = k13 * s1 * s1 + k14 * t1 * t1;
    const float b2 = k13 * s2 * s2 + k14 * t2 * t2;
    const float tau = fabsf(b2 - b0);
    const float q0 = tau * rcp_t(b0 + eps), q1 = tau * rcp_t(b1 + eps), q2 = tau * rcp_t(b2 + eps);
    const float m = fmaxf(fmaxf(q0, q1), fmaxf(q2, 1.0f));
    const float is = rcp_t(m);
    const float r0 = q0 * is, r1 = q1 * is, r2 = q2 * is, s2m = is * is;
    const float a0 = 0.2f * (s2m + r0 * r0), a1 = 0.5f * (s2m + r1 * r1), a2 = 0.3f * (s2m + r2 * r2);
    const float inv = rcp_t(a0 + a1 + a2);
    w0 = a0 * inv;
    w1 = a1 * inv;
    w2 = a2 * inv;
}

// Row of eq. (CWENO-FV) at node j+1/2 ("-" side): a u~_{j-1/2} + b u~_{j+1/2}
// + c u~_{j+3/2} = r, right side from ubar_{j-1}, ubar_j, ubar_{j+1}.  The "+"
// side is the same row on the mirrored line.
template <typename T>
__device__ __forceinline__ void cweno_row(T w0, T w1, T w2, T um1, T u0, T up1, T& a, T& b, T& c,
                                          T& r) {
    const T third = T(1) / T(3), sixth = T(1) / T(6);
    a = (T(2) * w0 + w1) * third;
    b = (w0 + T(2) * (w1 + w2)) * third;
    c = w2 * third;
    r = (w0 * um1 + (T(5) * (w0 + w1) + w2) * u0 + (w1 + T(5) * w2) * up1) * sixth;
}

// Closure of a non-periodic line: explicit fifth-order WENO-Z value at node
// j+1/2 ("-" side) from ubar_{j-2..j+2}, linear weights (0.1, 0.6, 0.3).
__device__ __forceinline__ double weno5z_value(double v0, double v1, double v2, double v3,
                                               double v4, double eps) {
    const double k13 = 13.0 / 12.0;
    double s0 = v0 - 2.0 * v1 + v2, t0 = v0 - 4.0 * v1 + 3.0 * v2;
    double s1 = v1 - 2.0 * v2 + v3, t1 = v1 - v3;
    double s2 = v2 - 2.0 * v3 + v4, t2 = 3.0 * v2 - 4.0 * v3 + v4;
    double b0 = k13 * s0 * s0 + 0.25 * t0 * t0;
    double b1 = k13 * s1 * s1 + 0.25 * t1 * t1;
    double b2 = k13 * s2 * s2 + 0.25 * t2 * t2;
    double tau = b2 - b0;
    double q0 = tau / (b0 + eps), q1 = tau / (b1 + eps), q2 = tau / (b2 + eps);
    double a0 = 0.1 * (1.0 + q0 * q0), a1 = 0.6 * (1.0 + q1 * q1), a2 = 0.3 * (1.0 + q2 * q2);
    double p0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) / 6.0;
    double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) / 6.0;
    double p2 = (2.0 * v2 + 5.0 * v3 - v4) / 6.0;
    return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

// The explicit comparison schemes of Sec 3: the classical fifth-order WENO
// value at node j+1/2 ("-" side) from v0..v4 = ubar_{j-2..j+2}, with the
// Jiang-Shu weights alpha_k = d_k / (beta_k + 1e-6)^2 (JS = true; Jiang and
// Shu's epsilon, the paper states none) or the WENO-Z weights of eq. (weight)
// with the linear weights d = (0.1, 0.6, 0.3) (JS = false, epsilon eps).
// As in wenoz_weights, the three weight divisions share one denominator:
//   JS: alpha_k ~ d_k prod_{l != k} e_l,   Z: alpha_k ~ d_k (e_k + tau^2) prod_{l != k} e_l,
// e_k = (beta_k + eps)^2, so one reciprocal normalises them.
constexpr double kWenoJsEps = 1e-6;
template <bool JS>
__device__ __forceinline__ double weno5_explicit(double v0, double v1, double v2, double v3,
                                                 double v4, double eps) {
    const double k13 = 13.0 / 12.0, sixth = 1.0 / 6.0;
    const double s0 = v0 - 2.0 * v1 + v2, t0 = v0 - 4.0 * v1 + 3.0 * v2;
    const double s1 = v1 - 2.0 * v2 + v3, t1 = v1 - v3;
    const double s2 = v2 - 2.0 * v3 + v4, t2 = 3.0 * v2 - 4.0 * v3 + v4;
    const double b0 = k13 * s0 * s0 + 0.25 * t0 * t0;
    const double b1 = k13 * s1 * s1 + 0.25 * t1 * t1;
    const double b2 = k13 * s2 * s2 + 0.25 * t2 * t2;
    const double ep = JS ? kWenoJsEps : eps;
    const double d0 = b0 + ep, d1 = b1 + ep, d2 = b2 + ep;
    const double e0 = d0 * d0, e1 = d1 * d1, e2 = d2 * d2;
    double a0 = 0.1 * (e1 * e2), a1 = 0.6 * (e0 * e2), a2 = 0.3 * (e0 * e1);
    if constexpr (!JS) {
        const double tau = b2 - b0, tt = tau * tau;
        a0 *= e0 + tt;
        a1 *= e1 + tt;
        a2 *= e2 + tt;
    }
    const double p0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * sixth;
    const double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) * sixth;
    const double p2 = (2.0 * v2 + 5.0 * v3 - v4) * sixth;
    return (a0 * p0 + a1 * p1 + a2 * p2) * rcp_t(a0 + a1 + a2);
}

// ------------------------------------------------------------- Sec 2.3
// 3x3 blocks of the characteristic system, row-major in registers.
__device__ __forceinline__ void mm3(const double (&A)[9], const double (&B)[9], double (&C)[9]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = fma(A[3 * i], B[j], fma(A[3 * i + 1], B[3 + j], A[3 * i + 2] * B[6 + j]));
}
__device__ __forceinline__ void mv3(const double (&A)[9], const double (&x)[3], double (&y)[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = fma(A[3 * i], x[0], fma(A[3 * i + 1], x[1], A[3 * i + 2] * x[2]));
}
// Inverse by the adjugate; the pivot blocks of the chase are nonsingular
// for the scheme's rows (diagonal blocks b_k l^(k) dominate).
__device__ __forceinline__ void inv3(const double (&M)[9], double (&I)[9]) {
    const double c0 = M[4] * M[8] - M[5] * M[7];
    const double c1 = M[5] * M[6] - M[3] * M[8];
    const double c2 = M[3] * M[7] - M[4] * M[6];
    const double id = rcp_t(M[0] * c0 + M[1] * c1 + M[2] * c2);
    I[0] = c0 * id;
    I[1] = (M[2] * M[7] - M[1] * M[8]) * id;
    I[2] = (M[1] * M[5] - M[2] * M[4]) * id;
    I[3] = c1 * id;
    I[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    I[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    I[6] = c2 * id;
    I[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    I[8] = (M[0] * M[4] - M[1] * M[3]) * id;
}

// Left eigenvectors of the Euler Jacobian at the Roe average of Ua and Ub
// (rho, rho u, E): rows l^(1), l^(2), l^(3) of L for the fields u - a, u,
// u + a.  A Roe sound speed that is not positive leaves the node
// component-wise (L = I).
__device__ __forceinline__ void roe_left(double g, const double (&Ua)[3], const double (&Ub)[3],
                                         double (&L)[9]) {
    const double ira = rcp_t(Ua[0]), irb = rcp_t(Ub[0]);
    const double ua = Ua[1] * ira, ub = Ub[1] * irb;
    const double pa = (g - 1.0) * (Ua[2] - 0.5 * Ua[1] * ua);
    const double pb = (g - 1.0) * (Ub[2] - 0.5 * Ub[1] * ub);
    const double Ha = (Ua[2] + pa) * ira, Hb = (Ub[2] + pb) * irb;
    const double sa = sqrt_nn(Ua[0]), sb = sqrt_nn(Ub[0]);
    const double iw = rcp_t(sa + sb);
    const double u = (sa * ua + sb * ub) * iw, H = (sa * Ha + sb * Hb) * iw;
    const double a2 = (g - 1.0) * (H - 0.5 * u * u);
    if (!(a2 > 0.0)) {
#pragma unroll
        for (int i = 0; i < 9; ++i) L[i] = (i % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    const double ia2 = rcp_t(a2);
    const double ia = sqrt_nn(a2) * ia2;   // 1/a
    const double c1 = (g - 1.0) * ia2, c2 = 0.5 * u * u * c1;
    L[0] = 0.5 * (c2 + u * ia);
    L[1] = 0.5 * (-c1 * u - ia);
    L[2] = 0.5 * c1;
    L[3] = 1.0 - c2;
    L[4] = c1 * u;
    L[5] = -c1;
    L[6] = 0.5 * (c2 - u * ia);
    L[7] = 0.5 * (-c1 * u + ia);
    L[8] = 0.5 * c1;
}

// Blocks of NB x NB (NB = 3 on 1D lines, 4 on the lines of the 2D
// operator), row-major in registers.  The NB = 3 forms are the ones above.
template <int NB>
__device__ __forceinline__ double dotN(const double* a, int sa, const double* b, int sb) {
    double s = a[(NB - 1) * sa] * b[(NB - 1) * sb];
#pragma unroll
    for (int q = NB - 2; q >= 0; --q) s = fma(a[q * sa], b[q * sb], s);
    return s;
}
template <int NB>
__device__ __forceinline__ void mmN(const double (&A)[NB * NB], const double (&B)[NB * NB],
                                    double (&C)[NB * NB]) {
    if constexpr (NB == 3) {
        mm3(A, B, C);
    } else {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) C[NB * i + j] = dotN<NB>(&A[NB * i], 1, &B[j], NB);
    }
}
template <int NB>
__device__ __forceinline__ void mvN(const double (&A)[NB * NB], const double (&x)[NB],
                                    double (&y)[NB]) {
    if constexpr (NB == 3) {
        mv3(A, x, y);
    } else {
#pragma unroll
        for (int i = 0; i < NB; ++i) y[i] = dotN<NB>(&A[NB * i], 1, x, 1);
    }
}
// 4x4 inverse by cofactors, from the twelve 2x2 minors of the top and the
// bottom row pairs (Laplace expansion along those pairs).
__device__ __forceinline__ void inv4(const double (&M)[16], double (&I)[16]) {
    const double s0 = M[0] * M[5] - M[4] * M[1], s1 = M[0] * M[6] - M[4] * M[2];
    const double s2 = M[0] * M[7] - M[4] * M[3], s3 = M[1] * M[6] - M[5] * M[2];
    const double s4 = M[1] * M[7] - M[5] * M[3], s5 = M[2] * M[7] - M[6] * M[3];
    const double c5 = M[10] * M[15] - M[14] * M[11], c4 = M[9] * M[15] - M[13] * M[11];
    const double c3 = M[9] * M[14] - M[13] * M[10], c2 = M[8] * M[15] - M[12] * M[11];
    const double c1 = M[8] * M[14] - M[12] * M[10], c0 = M[8] * M[13] - M[12] * M[9];
    const double id = rcp_t(s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0);
    I[0] = (M[5] * c5 - M[6] * c4 + M[7] * c3) * id;
    I[1] = (-M[1] * c5 + M[2] * c4 - M[3] * c3) * id;
    I[2] = (M[13] * s5 - M[14] * s4 + M[15] * s3) * id;
    I[3] = (-M[9] * s5 + M[10] * s4 - M[11] * s3) * id;
    I[4] = (-M[4] * c5 + M[6] * c2 - M[7] * c1) * id;
    I[5] = (M[0] * c5 - M[2] * c2 + M[3] * c1) * id;
    I[6] = (-M[12] * s5 + M[14] * s2 - M[15] * s1) * id;
    I[7] = (M[8] * s5 - M[10] * s2 + M[11] * s1) * id;
    I[8] = (M[4] * c4 - M[5] * c2 + M[7] * c0) * id;
    I[9] = (-M[0] * c4 + M[1] * c2 - M[3] * c0) * id;
    I[10] = (M[12] * s4 - M[13] * s2 + M[15] * s0) * id;
    I[11] = (-M[8] * s4 + M[9] * s2 - M[11] * s0) * id;
    I[12] = (-M[4] * c3 + M[5] * c1 - M[6] * c0) * id;
    I[13] = (M[0] * c3 - M[1] * c1 + M[2] * c0) * id;
    I[14] = (-M[12] * s3 + M[13] * s1 - M[14] * s0) * id;
    I[15] = (M[8] * s3 - M[9] * s1 + M[10] * s0) * id;
}
template <int NB>
__device__ __forceinline__ void invN(const double (&M)[NB * NB], double (&I)[NB * NB]) {
    if constexpr (NB == 3) inv3(M, I);
    else inv4(M, I);
}

// Left eigenvectors for a line of the 2D operator, in the line's own
// component order (rho, normal momentum, tangential momentum, E): the Roe
// average of Ua and Ub and, there, the rows for the fields u_n - a, u_n
// (entropy), u_n (shear, carrying u_t) and u_n + a.  With q^2 = u_n^2 +
// u_t^2, b1 = (gamma - 1) / a^2 and b2 = b1 q^2 / 2 the rows are
// ((b2 + u_n/a)/2, -(b1 u_n + 1/a)/2, -b1 u_t/2, b1/2), (1 - b2, b1 u_n,
// b1 u_t, -b1), (-u_t, 0, 1, 0) and ((b2 - u_n/a)/2, (1/a - b1 u_n)/2,
// -b1 u_t/2, b1/2).  A Roe sound speed that is not positive leaves the
// node component-wise (L = I).
__device__ __forceinline__ void roe_left4(double g, const double (&Ua)[4], const double (&Ub)[4],
                                          double (&L)[16]) {
    const double ira = rcp_t(Ua[0]), irb = rcp_t(Ub[0]);
    const double una = Ua[1] * ira, unb = Ub[1] * irb, uta = Ua[2] * ira, utb = Ub[2] * irb;
    const double pa = (g - 1.0) * (Ua[3] - 0.5 * fma(Ua[1], una, Ua[2] * uta));
    const double pb = (g - 1.0) * (Ub[3] - 0.5 * fma(Ub[1], unb, Ub[2] * utb));
    const double Ha = (Ua[3] + pa) * ira, Hb = (Ub[3] + pb) * irb;
    const double sa = sqrt_nn(Ua[0]), sb = sqrt_nn(Ub[0]);
    const double iw = rcp_t(sa + sb);
    const double un = (sa * una + sb * unb) * iw, ut = (sa * uta + sb * utb) * iw;
    const double H = (sa * Ha + sb * Hb) * iw;
    const double q2 = fma(un, un, ut * ut);
    const double a2 = (g - 1.0) * (H - 0.5 * q2);
    if (!(a2 > 0.0)) {
#pragma unroll
        for (int i = 0; i < 16; ++i) L[i] = (i % 5 == 0) ? 1.0 : 0.0;
        return;
    }
    const double ia2 = rcp_t(a2);
    const double ia = sqrt_nn(a2) * ia2;   // 1/a
    const double b1 = (g - 1.0) * ia2, b2 = 0.5 * q2 * b1;
    L[0] = 0.5 * (b2 + un * ia);
    L[1] = 0.5 * (-b1 * un - ia);
    L[2] = -0.5 * b1 * ut;
    L[3] = 0.5 * b1;
    L[4] = 1.0 - b2;
    L[5] = b1 * un;
    L[6] = b1 * ut;
    L[7] = -b1;
    L[8] = -ut;
    L[9] = 0.0;
    L[10] = 1.0;
    L[11] = 0.0;
    L[12] = 0.5 * (b2 - un * ia);
    L[13] = 0.5 * (-b1 * un + ia);
    L[14] = -0.5 * b1 * ut;
    L[15] = 0.5 * b1;
}

// ------------------------------------------------------------- Sec 2.4
// HLLC flux across a face with normal momentum component NRM (1: x, 2: y).
// Contact speed with rho_r in its right term, S_R = max of its candidates,
// sound speeds from max(p, 0), and the vacuum midpoint when the contact-speed
// denominator vanishes (two separating states of zero sound speed).
template <int NC, int NRM>
__device__ __forceinline__ void hllc_flux(double g, const double (&Ul)[NC], const double (&Ur)[NC],
                                          double (&F)[NC]) {
    constexpr int IE = NC - 1;
    constexpr int TG = (NC == 4) ? 3 - NRM : -1;
    const double rl = Ul[0], rr = Ur[0];
    const double irl = rcp_t(rl), irr = rcp_t(rr);
    const double ul = Ul[NRM] * irl, ur = Ur[NRM] * irr;
    double vl = 0.0, vr = 0.0;
    if constexpr (TG > 0) {
        vl = Ul[TG] * irl;
        vr = Ur[TG] * irr;
    }
    const double El = Ul[IE], Er = Ur[IE];
    const double pl = (g - 1.0) * (El - 0.5 * rl * fma(ul, ul, vl * vl));
    const double pr = (g - 1.0) * (Er - 0.5 * rr * fma(ur, ur, vr * vr));
    const double al = sqrt_nn(g * fmax(pl, 0.0) * irl), ar = sqrt_nn(g * fmax(pr, 0.0) * irr);
    const double Hl = (El + pl) * irl, Hr = (Er + pr) * irr;
    const double R = sqrt_nn(rr * irl);
    const double i1R = rcp_t(1.0 + R);
    const double ut = (ul + ur * R) * i1R, vt = (vl + vr * R) * i1R, Ht = (Hl + Hr * R) * i1R;
    const double at = sqrt_nn(fmax((g - 1.0) * (Ht - 0.5 * fma(ut, ut, vt * vt)), 0.0));
    const double SL = fmin(ul - al, ut - at);
    const double SR = fmax(ur + ar, ut + at);
    const double den = rr * (SR - ur) - rl * (SL - ul);
    const double SM =
        den > 0.0 ? (rr * ur * (SR - ur) - rl * ul * (SL - ul) + pl - pr) * rcp_t(den)
                  : 0.5 * (SL + SR);
    if (SL > 0.0) {
        F[0] = rl * ul;
        F[NRM] = rl * ul * ul + pl;
        if constexpr (TG > 0) F[TG] = rl * ul * vl;
        F[IE] = ul * (El + pl);
    } else if (SM > 0.0) {
        const double id = rcp_t(SL - SM);
        const double ps = rl * (ul - SL) * (ul - SM) + pl;
        const double s0 = rl * (SL - ul) * id;
        const double sn = ((SL - ul) * rl * ul + (ps - pl)) * id;
        const double se = ((SL - ul) * El - pl * ul + ps * SM) * id;
        F[0] = rl * ul + SL * (s0 - rl);
        F[NRM] = rl * ul * ul + pl + SL * (sn - Ul[NRM]);
        if constexpr (TG > 0) F[TG] = rl * ul * vl + SL * (s0 * vl - Ul[TG]);
        F[IE] = ul * (El + pl) + SL * (se - El);
    } else if (SR >= 0.0 && SR > SM) {
        const double id = rcp_t(SR - SM);
        const double ps = rr * (ur - SR) * (ur - SM) + pr;
        const double s0 = rr * (SR - ur) * id;
        const double sn = ((SR - ur) * rr * ur + (ps - pr)) * id;
        const double se = ((SR - ur) * Er - pr * ur + ps * SM) * id;
        F[0] = rr * ur + SR * (s0 - rr);
        F[NRM] = rr * ur * ur + pr + SR * (sn - Ur[NRM]);
        if constexpr (TG > 0) F[TG] = rr * ur * vr + SR * (s0 * vr - Ur[TG]);
        F[IE] = ur * (Er + pr) + SR * (se - Er);
    } else {
        F[0] = rr * ur;
        F[NRM] = rr * ur * ur + pr;
        if constexpr (TG > 0) F[TG] = rr * ur * vr;
        F[IE] = ur * (Er + pr);
    }
}

// Local Lax-Friedrichs flux, the more dissipative alternative the paper
// names for Example 3.6 (not defined there): F = (f(Ul) + f(Ur))/2 -
// alpha (Ur - Ul)/2 with alpha = max(|u| + a) over the two states, sound
// speeds from max(p, 0) as in HLLC.
template <int NC, int NRM>
__device__ __forceinline__ void lf_flux(double g, const double (&Ul)[NC], const double (&Ur)[NC],
                                        double (&F)[NC]) {
    constexpr int IE = NC - 1;
    constexpr int TG = (NC == 4) ? 3 - NRM : -1;
    const double rl = Ul[0], rr = Ur[0];
    const double irl = rcp_t(rl), irr = rcp_t(rr);
    const double ul = Ul[NRM] * irl, ur = Ur[NRM] * irr;
    double vl = 0.0, vr = 0.0;
    if constexpr (TG > 0) {
        vl = Ul[TG] * irl;
        vr = Ur[TG] * irr;
    }
    const double El = Ul[IE], Er = Ur[IE];
    const double pl = (g - 1.0) * (El - 0.5 * rl * fma(ul, ul, vl * vl));
    const double pr = (g - 1.0) * (Er - 0.5 * rr * fma(ur, ur, vr * vr));
    const double al = sqrt_nn(g * fmax(pl, 0.0) * irl), ar = sqrt_nn(g * fmax(pr, 0.0) * irr);
    const double alpha = fmax(fabs(ul) + al, fabs(ur) + ar);
    double Fl[NC], Fr[NC];
    Fl[0] = rl * ul;
    Fl[NRM] = rl * ul * ul + pl;
    Fl[IE] = ul * (El + pl);
    Fr[0] = rr * ur;
    Fr[NRM] = rr * ur * ur + pr;
    Fr[IE] = ur * (Er + pr);
    if constexpr (TG > 0) {
        Fl[TG] = rl * ul * vl;
        Fr[TG] = rr * ur * vr;
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) F[k] = 0.5 * (Fl[k] + Fr[k]) - 0.5 * alpha * (Ur[k] - Ul[k]);
}

// Mixed precision HLLC: primitives (rho, u_n, u_t, p) and E are formed in
// double from the limited conserved states (so p never suffers float
// cancellation near vacuum), then the wave speeds, contact, star states and
// flux are evaluated in float; the flux is returned in double.
template <int NC, int NRM>
__device__ __forceinline__ void hllc_flux_f32(double gd, const double (&Uld)[NC],
                                              const double (&Urd)[NC], double (&Fd)[NC]) {
    constexpr int IE = NC - 1;
    constexpr int TG = (NC == 4) ? 3 - NRM : -1;
    const double irld = 1.0 / Uld[0], irrd = 1.0 / Urd[0];
    const double uld = Uld[NRM] * irld, urd = Urd[NRM] * irrd;
    double vld = 0.0, vrd = 0.0;
    if constexpr (TG > 0) {
        vld = Uld[TG] * irld;
        vrd = Urd[TG] * irrd;
    }
    const double pld = (gd - 1.0) * (Uld[IE] - 0.5 * Uld[0] * (uld * uld + vld * vld));
    const double prd = (gd - 1.0) * (Urd[IE] - 0.5 * Urd[0] * (urd * urd + vrd * vrd));
    const float g = (float)gd;
    const float rl = (float)Uld[0], rr = (float)Urd[0];
    const float ul = (float)uld, ur = (float)urd, vl = (float)vld, vr = (float)vrd;
    const float pl = (float)pld, pr = (float)prd, El = (float)Uld[IE], Er = (float)Urd[IE];
    const float irl = rcp_t(rl), irr = rcp_t(rr);
    const float al = sqrtf(g * fmaxf(pl, 0.0f) * irl), ar = sqrtf(g * fmaxf(pr, 0.0f) * irr);
    const float Hl = (El + pl) * irl, Hr = (Er + pr) * irr;
    const float R = sqrtf(rr * irl);
    const float i1R = rcp_t(1.0f + R);
    const float ut = (ul + ur * R) * i1R, vt = (vl + vr * R) * i1R, Ht = (Hl + Hr * R) * i1R;
    const float at = sqrtf(fmaxf((g - 1.0f) * (Ht - 0.5f * (ut * ut + vt * vt)), 0.0f));
    const float SL = fminf(ul - al, ut - at);
    const float SR = fmaxf(ur + ar, ut + at);
    const float den = rr * (SR - ur) - rl * (SL - ul);
    const float SM = den > 0.0f ? (rr * ur * (SR - ur) - rl * ul * (SL - ul) + pl - pr) * rcp_t(den)
                                : 0.5f * (SL + SR);
    float F[NC];
    const float mnl = rl * ul, mnr = rr * ur;
    if (SL > 0.0f) {
        F[0] = mnl;
        F[NRM] = mnl * ul + pl;
        if constexpr (TG > 0) F[TG] = mnl * vl;
        F[IE] = ul * (El + pl);
    } else if (SM > 0.0f) {
        const float id = rcp_t(SL - SM);
        const float ps = rl * (ul - SL) * (ul - SM) + pl;
        const float s0 = rl * (SL - ul) * id;
        const float sn = ((SL - ul) * mnl + (ps - pl)) * id;
        const float se = ((SL - ul) * El - pl * ul + ps * SM) * id;
        F[0] = mnl + SL * (s0 - rl);
        F[NRM] = mnl * ul + pl + SL * (sn - mnl);
        if constexpr (TG > 0) F[TG] = mnl * vl + SL * (s0 * vl - rl * vl);
        F[IE] = ul * (El + pl) + SL * (se - El);
    } else if (SR >= 0.0f && SR > SM) {
        const float id = rcp_t(SR - SM);
        const float ps = rr * (ur - SR) * (ur - SM) + pr;
        const float s0 = rr * (SR - ur) * id;
        const float sn = ((SR - ur) * mnr + (ps - pr)) * id;
        const float se = ((SR - ur) * Er - pr * ur + ps * SM) * id;
        F[0] = mnr + SR * (s0 - rr);
        F[NRM] = mnr * ur + pr + SR * (sn - mnr);
        if constexpr (TG > 0) F[TG] = mnr * vr + SR * (s0 * vr - rr * vr);
        F[IE] = ur * (Er + pr) + SR * (se - Er);
    } else {
        F[0] = mnr;
        F[NRM] = mnr * ur + pr;
        if constexpr (TG > 0) F[TG] = mnr * vr;
        F[IE] = ur * (Er + pr);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) Fd[k] = (double)F[k];
}

// a . b over the momentum components, the normal one (NRM) first: a sweep
// along y of a 2D state and a sweep along x of its mirror image (x and y and
// the two momenta exchanged) then round identically, so the 2D operator keeps
// a state's diagonal mirror symmetry exactly (the fluxes spell their sums of
// squared velocities the same way).
template <int NC, int NRM>
__device__ __forceinline__ double mom_dot(const double (&a)[NC], const double (&b)[NC]) {
    // the fused form is spelled out: left to the compiler, which product is
    // fused may differ between the two instantiations
    if constexpr (NC == 4) return fma(a[NRM], b[NRM], a[3 - NRM] * b[3 - NRM]);
    else return fma(a[1], b[1], 0.0);   // one momentum: rounded once, and not
                                        // fused into the caller's next operation
}

// e = E/rho - |m|^2 / (2 rho^2), the specific internal energy of the set G.
template <int NC, int NRM = 1>
__device__ __forceinline__ double spec_e(const double (&U)[NC]) {
    const double m2 = mom_dot<NC, NRM>(U, U);
    return U[NC - 1] / U[0] - 0.5 * m2 / (U[0] * U[0]);
}

// Limiter step 4 test "rho <= 0 or e(W) < eps" without divisions:
// for rho > 0, e < eps  <=>  rho E - |m|^2/2 < eps rho^2.
template <int NC, int NRM = 1>
__device__ __forceinline__ bool below_eps(double eps, const double (&U)[NC]) {
    const double m2 = mom_dot<NC, NRM>(U, U);
    return !(U[0] > 0.0) || (U[0] * U[NC - 1] - 0.5 * m2 < eps * U[0] * U[0]);
}

// Limiter step 4: root t in [0, 1] of e(Ubar + t (W - Ubar)) = eps via
// rho E - |m|^2/2 - eps rho^2 = A t^2 + B t + C, t = 2C / (-B + sqrt(B^2 - 4AC)).
template <int NC, int NRM = 1>
__device__ __forceinline__ double pp_root(double eps, const double (&Ub)[NC],
                                          const double (&W)[NC]) {
    constexpr int IE = NC - 1;
    double D[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) D[k] = W[k] - Ub[k];
    const double dm2 = mom_dot<NC, NRM>(D, D), mdm = mom_dot<NC, NRM>(Ub, D);
    const double m2 = mom_dot<NC, NRM>(Ub, Ub);
    const double A = D[0] * D[IE] - 0.5 * dm2 - eps * D[0] * D[0];
    const double B = Ub[0] * D[IE] + Ub[IE] * D[0] - mdm - 2.0 * eps * Ub[0] * D[0];
    const double C = Ub[0] * Ub[IE] - 0.5 * m2 - eps * Ub[0] * Ub[0];
    if (C <= 0.0) return 0.0;
    const double disc = fmax(B * B - 4.0 * A * C, 0.0);
    double t = 2.0 * C / (-B + sqrt_nn(disc));
    if (!(t >= 0.0)) t = 0.0;
    return fmin(t, 1.0);
}

// Positivity-preserving limiter of one cell (Sec 2.4, steps 1-4): Um = U-_{j+1/2},
// Up = U+_{j-1/2}, limited in place.  Returns 1 if anything changed.
template <int NC, int NRM = 1>
__device__ __forceinline__ int pp_limit(double w1, double i12, double eps_rho, double eps_e,
                                        const double (&Ub)[NC], double (&Um)[NC],
                                        double (&Up)[NC]) {
    int active = 0;   // i12 = 1 / (1 - 2 w1)
    const double rmid = (Ub[0] - w1 * Up[0] - w1 * Um[0]) * i12;
    const double rmin = fmin(fmin(Um[0], Up[0]), rmid);
    if (rmin < eps_rho) {
        const double th1 = fmin((Ub[0] - eps_rho) / (Ub[0] - rmin), 1.0);
        if (th1 < 1.0) {
            Um[0] = th1 * (Um[0] - Ub[0]) + Ub[0];
            Up[0] = th1 * (Up[0] - Ub[0]) + Ub[0];
            active = 1;
        }
    }
    double W3[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) W3[k] = (Ub[k] - w1 * Up[k] - w1 * Um[k]) * i12;
    double th2 = 1.0;
    if (below_eps<NC, NRM>(eps_e, Um)) th2 = fmin(th2, pp_root<NC, NRM>(eps_e, Ub, Um));
    if (below_eps<NC, NRM>(eps_e, Up)) th2 = fmin(th2, pp_root<NC, NRM>(eps_e, Ub, Up));
    if (below_eps<NC, NRM>(eps_e, W3)) th2 = fmin(th2, pp_root<NC, NRM>(eps_e, Ub, W3));
    if (th2 < 1.0) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            Um[k] = th2 * (Um[k] - Ub[k]) + Ub[k];
            Up[k] = th2 * (Up[k] - Ub[k]) + Ub[k];
        }
        active = 1;
    }
    return active;
}

// Limiter steps 2-4 over the node states of one cell of the Gauss-node 2D
// operator: Nm[k] the three nodes of its right face (U-), Np[k] those of its
// left face (U+), limited in place against the cell average Ub.  The middle
// state is Ub = w1 sum_k g_k (Nm_k + Np_k) + (1 - 2 w1) mid, the Gauss-weighted
// form of the 1D decomposition; i12 = 1 / (1 - 2 w1).  Returns 1 if anything
// changed.
template <int NC, int NRM = 1>
__device__ __forceinline__ int pp_limit_nodes(double w1, double i12, const double (&g)[3],
                                              double eps_rho, double eps_e,
                                              const double (&Ub)[NC], double (&Nm)[3][NC],
                                              double (&Np)[3][NC]) {
    auto middle = [&](double (&mid)[NC]) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) s += g[k] * (Nm[k][c] + Np[k][c]);
            mid[c] = (Ub[c] - w1 * s) * i12;
        }
    };
    int active = 0;
    double mid[NC];
    middle(mid);
    double rmin = mid[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) rmin = fmin(rmin, fmin(Nm[k][0], Np[k][0]));
    if (rmin < eps_rho) {
        const double th1 = fmin((Ub[0] - eps_rho) / (Ub[0] - rmin), 1.0);
        if (th1 < 1.0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                Nm[k][0] = th1 * (Nm[k][0] - Ub[0]) + Ub[0];
                Np[k][0] = th1 * (Np[k][0] - Ub[0]) + Ub[0];
            }
            active = 1;
        }
    }
    middle(mid);
    double th2 = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (below_eps<NC, NRM>(eps_e, Nm[k])) th2 = fmin(th2, pp_root<NC, NRM>(eps_e, Ub, Nm[k]));
        if (below_eps<NC, NRM>(eps_e, Np[k])) th2 = fmin(th2, pp_root<NC, NRM>(eps_e, Ub, Np[k]));
    }
    if (below_eps<NC, NRM>(eps_e, mid)) th2 = fmin(th2, pp_root<NC, NRM>(eps_e, Ub, mid));
    if (th2 < 1.0) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Nm[k][c] = th2 * (Nm[k][c] - Ub[c]) + Ub[c];
                Np[k][c] = th2 * (Np[k][c] - Ub[c]) + Ub[c];
            }
        active = 1;
    }
    return active;
}

// |u_n| + a of a state, a pressure negative by roundoff counting as 0.
template <int NC, int NRM>
__device__ __forceinline__ double wave_speed(double g, const double (&U)[NC]) {
    const double m2 = mom_dot<NC, NRM>(U, U);
    const double ir = rcp_t(U[0]);
    const double p = (g - 1.0) * (U[NC - 1] - 0.5 * m2 * ir);
    return fabs(U[NRM] * ir) + sqrt_nn(g * fmax(p, 0.0) * ir);
}

}  // namespace ppc
