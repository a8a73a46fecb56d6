// fv_physics.h -- point-wise device functions of the fused finite-volume stage
// for gfx950: equation of state, primitive/conservative maps, WENO5-Z
// reconstruction with smoothness indicators shared between the two faces of a
// cell, TENO6-A face reconstruction, characteristic projection, the HLLC flux
// and the 4th-order central viscous flux.
//
// Notation follows arXiv:2402.05193: W primitive, U conservative (Sec. 2.1,
// 2.3), stiffened gas and isobaric mixture closure (Sec. 2.4), WENO5-Z and
// HLLC (Sec. 3.2 and the HLLC appendix), admissible sets (Sec. 3.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fv {

enum { EULER = 0, NS = 1, DIM = 2 };
enum { PERIODIC = 0, ZEROGRAD = 1, SYMMETRY = 2 };

template <int MODEL>
struct Layout;
template <>
struct Layout<EULER> {
    static constexpr int NC = 5, V = 1, P = 4, A = -1;
};
template <>
struct Layout<NS> {
    static constexpr int NC = 5, V = 1, P = 4, A = -1;
};
template <>
struct Layout<DIM> {
    static constexpr int NC = 7, V = 2, P = 5, A = 6;
};

// Material constants in the form the device uses.
//   single phase:  p = gm1 (E - ke) - gpinf,  rho e = iG p + PI,  rho c^2 = gamma (p + pinf)
//   mixture:       Gamma(a1) = a1 iG1 + (1-a1) iG2,  Pi(a1) = a1 PI1 + (1-a1) PI2,
//                  p = (rho e - Pi)/Gamma,  rho c^2 = ((Gamma+1) p + Pi)/Gamma
template <typename Real>
struct Material {
    Real gamma, pinf, gm1, gpinf;  // fluid 1 (single phase)
    Real iG1, PI1, iG2, PI2;       // 1/(gamma_k-1), gamma_k pinf_k/(gamma_k-1)
};

template <typename Real>
struct Tolerances {
    Real eps_rho, eps_rhoc2, eps_alpha;
};

// Dynamic viscosity law (Sec. 2.5, material properties), in terms of theta =
// p / rho = R T: law 0 constant mu; 1 power law mu (T/T_ref)^0.7; 2 Sutherland
// mu (T/T_ref)^1.5 (T_ref + C)/(T + C).  kfac = gamma/((gamma-1) Pr) gives the
// heat-flux coefficient kfac mu (constant Prandtl number; R cancels).
template <typename Real>
struct ViscLaw {
    int law;
    Real mu, kfac;
    Real inv_th_ref;  // 1/(R T_ref)
    Real th_c;        // R C
    Real th_ref_c;    // R (T_ref + C)
};

// ---------------------------------------------------------------- arithmetic helpers
// 1/x and 1/sqrt(x) from the hardware estimates (relative error below 2^-24
// on gfx950, measured) with one third-order correction: for r = 1/x (1 - e),
// 1/x = r (1 + e + e^2 + O(e^3)); for y = (1 - e)^(1/2) / sqrt(x) with
// e = 1 - x y^2, 1/sqrt(x) = y (1 + e/2 + 3 e^2/8 + O(e^3)).  The O(e^3) terms
// are below 2^-70, so the FP64 results are good to about an ulp for the
// positive normal arguments used here.  FP32 uses the estimates as they are.
__device__ __forceinline__ double rcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double rsqrt(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}
__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// sqrt(x) = x / sqrt(x), with one Newton correction of the product
__device__ __forceinline__ double sqrt_fast(double x)
{
    const double y = rsqrt(x);
    const double s = x * y;
    return fma(0.5 * y, fma(-s, s, x), s);
}
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------- EOS / maps
template <typename Real, int MODEL>
__device__ __forceinline__ Real density(const Real* w)
{
    if constexpr (MODEL == DIM) return w[0] + w[1];
    else return w[0];
}

// Gamma = 1/(gamma-1) and Pi = gamma pinf/(gamma-1) of the mixture at a1.
template <typename Real>
__device__ __forceinline__ void mixture(const Material<Real>& m, Real a1, Real& G, Real& Pi)
{
    const Real a2 = Real(1) - a1;
    G = a1 * m.iG1 + a2 * m.iG2;
    Pi = a1 * m.PI1 + a2 * m.PI2;
}

// rho e from the primitive state
template <typename Real, int MODEL>
__device__ __forceinline__ Real rho_e(const Material<Real>& mat, const Real* w)
{
    constexpr int P = Layout<MODEL>::P;
    if constexpr (MODEL == DIM) {
        Real G, Pi;
        mixture(mat, w[6], G, Pi);
        return G * w[P] + Pi;
    } else {
        return (w[P] + mat.gpinf) * mat.iG1;
    }
}

// rho c^2 (Sec. 3.3 helper variable)
template <typename Real, int MODEL>
__device__ __forceinline__ Real rhoc2(const Material<Real>& mat, const Real* w)
{
    constexpr int P = Layout<MODEL>::P;
    if constexpr (MODEL == DIM) {
        Real G, Pi;
        mixture(mat, w[6], G, Pi);
        return ((G + Real(1)) * w[P] + Pi) * rcp(G);
    } else {
        return mat.gamma * (w[P] + mat.pinf);
    }
}

// L_{U->W}
template <typename Real, int MODEL>
__device__ __forceinline__ void cons_to_prim(const Material<Real>& mat, const Real* u, Real* w)
{
    constexpr int V = Layout<MODEL>::V, P = Layout<MODEL>::P;
    Real rho;
    if constexpr (MODEL == DIM) {
        w[0] = u[0];
        w[1] = u[1];
        w[6] = u[6];
        rho = u[0] + u[1];
    } else {
        w[0] = u[0];
        rho = u[0];
    }
    const Real ir = rcp(rho);
    w[V] = u[V] * ir;
    w[V + 1] = u[V + 1] * ir;
    w[V + 2] = u[V + 2] * ir;
    const Real ke = Real(0.5) * rho * (w[V] * w[V] + w[V + 1] * w[V + 1] + w[V + 2] * w[V + 2]);
    const Real re = u[P] - ke;
    if constexpr (MODEL == DIM) {
        Real G, Pi;
        mixture(mat, u[6], G, Pi);
        w[P] = (re - Pi) * rcp(G);
    } else {
        w[P] = mat.gm1 * re - mat.gpinf;
    }
}

// L_{U->W} that also returns 1/rho
template <typename Real, int MODEL>
__device__ __forceinline__ Real cons_to_prim_ir(const Material<Real>& mat, const Real* u, Real* w)
{
    cons_to_prim<Real, MODEL>(mat, u, w);
    return rcp(density<Real, MODEL>(w));
}

// L_{W->U}
template <typename Real, int MODEL>
__device__ __forceinline__ void prim_to_cons(const Material<Real>& mat, const Real* w, Real* u)
{
    constexpr int V = Layout<MODEL>::V, P = Layout<MODEL>::P;
    const Real rho = density<Real, MODEL>(w);
    if constexpr (MODEL == DIM) {
        u[0] = w[0];
        u[1] = w[1];
        u[6] = w[6];
    } else {
        u[0] = w[0];
    }
    u[V] = rho * w[V];
    u[V + 1] = rho * w[V + 1];
    u[V + 2] = rho * w[V + 2];
    const Real ke = Real(0.5) * rho * (w[V] * w[V] + w[V + 1] * w[V + 1] + w[V + 2] * w[V + 2]);
    u[P] = rho_e<Real, MODEL>(mat, w) + ke;
}

// ---------------------------------------------------------------- WENO5-Z
// Both one-sided WENO5-Z values of cell i from v_{i-2..i+2} = a,b,c,d,e:
//   vm = v^-_{i+1/2} (left-biased, stencils {i-2..i}, {i-1..i+1}, {i..i+2},
//        linear weights 1/10, 6/10, 3/10),
//   vp = v^+_{i-1/2} (the mirror image: same smoothness indicators in
//        reverse order).
// Weights alpha_k = d_k (1 + tau / (beta_k + eps)) with tau = |beta0 - beta2|
// (WENO-Z, exponent 1).  The 1/(beta_k + eps) and the factors
// g_k = 1 + tau/(beta_k + eps) are computed once for both sides.
// WENO-Z weights (q = 1) in FP32 for data of any magnitude: g_k = 1 + tau / e_k
// (e_k = beta_k + eps) overflows once tau exceeds ~1e8 with eps = 1e-30 (a jump
// of ~2e4 in the reconstructed variable, e.g. a pressure jump in pascals).  The
// weights divided by the largest one, s_k = g_k / max g = A + (e_min C) / e_k with
// A = e_min / (e_min + tau) and C = tau / (e_min + tau) = 1 - A, normalise to the
// same nonlinear weights, stay in [0, 1] and keep s = 1 for the smoothest
// candidate when A underflows (tau / e_min beyond the FP32 range; e_min C stays
// near e_min >= eps).  Weights of order one also keep the weighted sums of
// small-valued fields out of the denormal range, which weights scaled by e_min
// do not.  FP64 (eps = 1e-40) keeps the plain form.
__device__ __forceinline__ void weno_z_scaled(float tau, float e0, float e1, float e2, float& s0, float& s1,
                                              float& s2)
{
    const float em = fminf(fminf(e0, e1), e2);
    const float inv = rcp(em + tau);
    const float A = em * inv, Cm = em * (tau * inv);
    s0 = fmaf(Cm, rcp(e0), A);
    s1 = fmaf(Cm, rcp(e1), A);
    s2 = fmaf(Cm, rcp(e2), A);
}

template <typename Real>
__device__ __forceinline__ void weno5z_pair(Real a, Real b, Real c, Real d, Real e, Real eps, Real& vm,
                                            Real& vp)
{
    const Real k13 = Real(13.0 / 12.0), q = Real(0.25);
    const Real t0 = a - Real(2) * b + c;
    const Real s0 = a - Real(4) * b + Real(3) * c;
    const Real t1 = b - Real(2) * c + d;
    const Real s1 = b - d;
    const Real t2 = c - Real(2) * d + e;
    const Real s2 = Real(3) * c - Real(4) * d + e;
    const Real b0 = k13 * t0 * t0 + q * s0 * s0;
    const Real b1 = k13 * t1 * t1 + q * s1 * s1;
    const Real b2 = k13 * t2 * t2 + q * s2 * s2;
    const Real tau = fabs(b0 - b2);
    const Real e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
    Real g0, g1, g2;
    if constexpr (sizeof(Real) == 8) {
        // one reciprocal for the three indicators: 1/e_k from 1/(e0 e1 e2)
        const Real p01 = e0 * e1;
        const Real R = rcp(p01 * e2);
        const Real t = e2 * R;
        const Real r2 = p01 * R;
        const Real r0 = e1 * t;
        const Real r1 = e0 * t;
        g0 = fma(tau, r0, Real(1));
        g1 = fma(tau, r1, Real(1));
        g2 = fma(tau, r2, Real(1));
    } else {
        weno_z_scaled(tau, e0, e1, e2, g0, g1, g2);
    }
    // candidate values (times 6)
    const Real p0 = Real(2) * a - Real(7) * b + Real(11) * c;
    const Real p1 = -b + Real(5) * c + Real(2) * d;
    const Real p2 = Real(2) * c + Real(5) * d - e;
    const Real u0 = Real(2) * e - Real(7) * d + Real(11) * c;
    const Real u1 = -d + Real(5) * c + Real(2) * b;
    const Real u2 = Real(2) * c + Real(5) * b - a;
    // alpha scaled by 10: (1, 6, 3) g for vm and (3, 6, 1) g reversed for vp
    const Real m1 = Real(6) * g1, m2 = Real(3) * g2, n2 = Real(3) * g0;
    const Real dm = Real(6) * (g0 + m1 + m2);
    const Real dp = Real(6) * (g2 + m1 + n2);
    Real idm, idp;
    if constexpr (sizeof(Real) == 8) {
        const Real R = rcp(dm * dp);
        idm = dp * R;
        idp = dm * R;
    } else {
        idm = rcp(dm);
        idp = rcp(dp);
    }
    vm = (g0 * p0 + m1 * p1 + m2 * p2) * idm;
    vp = (g2 * u0 + m1 * u1 + n2 * u2) * idp;
}

// One-sided WENO5-Z value v^-_{i+1/2} from v_{i-2..i+2} = a,b,c,d,e (the v^+
// value of a face is the same function of the mirrored stencil).
template <typename Real>
__device__ __forceinline__ Real weno5z_one(Real a, Real b, Real c, Real d, Real e, Real eps)
{
    const Real k13 = Real(13.0 / 12.0), q = Real(0.25);
    const Real t0 = a - Real(2) * b + c;
    const Real s0 = a - Real(4) * b + Real(3) * c;
    const Real t1 = b - Real(2) * c + d;
    const Real s1 = b - d;
    const Real t2 = c - Real(2) * d + e;
    const Real s2 = Real(3) * c - Real(4) * d + e;
    const Real b0 = k13 * t0 * t0 + q * s0 * s0;
    const Real b1 = k13 * t1 * t1 + q * s1 * s1;
    const Real b2 = k13 * t2 * t2 + q * s2 * s2;
    const Real tau = fabs(b0 - b2);
    const Real e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
    Real g0, g1, g2;
    if constexpr (sizeof(Real) == 8) {
        const Real p01 = e0 * e1;
        const Real R = rcp(p01 * e2);
        const Real t = e2 * R;
        const Real r2 = p01 * R;
        const Real r0 = e1 * t;
        const Real r1 = e0 * t;
        g0 = fma(tau, r0, Real(1));
        g1 = fma(tau, r1, Real(1));
        g2 = fma(tau, r2, Real(1));
    } else {
        weno_z_scaled(tau, e0, e1, e2, g0, g1, g2);
    }
    const Real m1 = Real(6) * g1;
    const Real m2 = Real(3) * g2;
    const Real p0 = Real(2) * a - Real(7) * b + Real(11) * c;
    const Real p1 = -b + Real(5) * c + Real(2) * d;
    const Real p2 = Real(2) * c + Real(5) * d - e;
    return (g0 * p0 + m1 * p1 + m2 * p2) * rcp(Real(6) * (g0 + m1 + m2));
}

// ---------------------------------------------------------------- TENO6-A
// Six-point targeted ENO reconstruction with adaptive dissipation (Sec. 3.2
// step 3; the candidate stencils are those of the reconstruction schematic:
// S0 = {i-2,i-1,i}, S1 = {i-1,i,i+1}, S2 = {i,i+1,i+2}, S3 = {i,..,i+3}).
// A face between cells i and i+1 reads v_{i-2..i+3} = a..f for both states.
//
// Cut-off C_T = 10^-floor(beta_bar), beta_bar = 10.5 - 3.5 (1 - g(m)),
// g(m) = (1 - m)^4 (1 + 4 m), m = 1 - min(1, eta / 0.17), eta the smallest
// cell indicator (|2 D- D+| + e) / (D-^2 + D+^2 + e) of cells i-1 .. i+2
// (e = 0.9 * 0.17 * 1e-6 / (1 - 0.9 * 0.17)).  The indicator set is the same
// for both face states.  All four indicators at or above 0.17 give m = 0 and
// C_T = 1e-10 without a division.
template <typename Real>
__device__ __forceinline__ Real teno6a_cutoff(Real a, Real b, Real c, Real d, Real e, Real f)
{
    const Real cr = Real(0.17);
    const Real ee = Real(0.9 * 0.17 / (1.0 - 0.9 * 0.17) * 1e-6);
    const Real d0 = b - a, d1 = c - b, d2 = d - c, d3 = e - d, d4 = f - e;
    const Real n0 = fabs(Real(2) * d0 * d1) + ee, q0 = fma(d0, d0, fma(d1, d1, ee));
    const Real n1 = fabs(Real(2) * d1 * d2) + ee, q1 = fma(d1, d1, fma(d2, d2, ee));
    const Real n2 = fabs(Real(2) * d2 * d3) + ee, q2 = fma(d2, d2, fma(d3, d3, ee));
    const Real n3 = fabs(Real(2) * d3 * d4) + ee, q3 = fma(d3, d3, fma(d4, d4, ee));
    if (n0 >= cr * q0 && n1 >= cr * q1 && n2 >= cr * q2 && n3 >= cr * q3) return Real(1e-10);
    const Real eta = fmin(fmin(n0 * rcp(q0), n1 * rcp(q1)), fmin(n2 * rcp(q2), n3 * rcp(q3)));
    const Real m = Real(1) - fmin(Real(1), eta * Real(1.0 / 0.17));
    const Real om = Real(1) - m, om2 = om * om;
    const Real g = om2 * om2 * fma(Real(4), m, Real(1));
    const Real bbar = Real(10.5) - Real(3.5) * (Real(1) - g);
    return bbar >= Real(10) ? Real(1e-10) : bbar >= Real(9) ? Real(1e-9) : bbar >= Real(8) ? Real(1e-8) : Real(1e-7);
}

// Left-biased TENO6-A value at x_{i+1/2} from v_{i-2..i+3} = a..f (the right
// state of the face is the same function of the mirrored stencil).
//  * Jiang-Shu smoothness indicators beta_0..beta_3 of the candidates and
//    beta_6 of the six-cell polynomial, over cell i; the 4- and 6-cell ones
//    are written with values relative to v_i (they see differences only), so
//    their rounding scales with the data's variation, not its magnitude.
//  * tau_6 = |beta_6 - (beta_0 + 4 beta_1 + beta_2) / 6|.
//  * stencil k is dropped when gamma_k / sum gamma < C_T, gamma_k =
//    (1 + tau_6 / (beta_k + eps))^6; evaluated as s_k^6 < C_T sum s^6 with
//    s_k = gamma_k^(1/6) / max gamma^(1/6) = A + A tau_6 / (beta_k + eps),
//    A = e_min / (e_min + tau_6), which stays finite where gamma overflows
//    (FP32: A + C e_min / e_k with C = tau_6 / (e_min + tau_6), the same value,
//    which keeps s = 1 for the smoothest candidate where A underflows).
//  * kept stencils combine with the linear weights (1, 9, 6, 4) / 20.
template <typename Real>
__device__ __forceinline__ Real teno6a_one(Real a, Real b, Real c, Real d, Real e, Real f, Real eps, Real ct)
{
    const Real k13 = Real(13.0 / 12.0), q = Real(0.25);
    const Real t0 = a - Real(2) * b + c, s0 = a - Real(4) * b + Real(3) * c;
    const Real t1 = b - Real(2) * c + d, s1 = b - d;
    const Real t2 = c - Real(2) * d + e, s2 = Real(3) * c - Real(4) * d + e;
    const Real b0 = k13 * t0 * t0 + q * s0 * s0;
    const Real b1 = k13 * t1 * t1 + q * s1 * s1;
    const Real b2 = k13 * t2 * t2 + q * s2 * s2;
    const Real A = a - c, B = b - c, D = d - c, E = e - c, F = f - c;
    const Real b3 = (D * (Real(11003) * D - Real(17246) * E + Real(4642) * F) + E * (Real(7043) * E - Real(3882) * F) +
                     Real(547) * F * F) *
                    Real(1.0 / 240.0);
    const Real b6 = (A * (Real(271779) * A - Real(2380800) * B - Real(3462252) * D + Real(1458762) * E -
                          Real(245620) * F) +
                     B * (Real(5653317) * B + Real(17905032) * D - Real(7727988) * E + Real(1325006) * F) +
                     D * (Real(17195652) * D - Real(15880404) * E + Real(2863984) * F) +
                     E * (Real(3824847) * E - Real(1429976) * F) + Real(139633) * F * F) *
                    Real(1.0 / 120960.0);
    const Real tau = fabs(b6 - (b0 + Real(4) * b1 + b2) * Real(1.0 / 6.0));
    const Real e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps, e3 = b3 + eps;
    Real r0, r1, r2, r3;
    if constexpr (sizeof(Real) == 8) {
        const Real p01 = e0 * e1, p23 = e2 * e3;
        const Real R = rcp(p01 * p23);
        const Real u = p23 * R, v = p01 * R;
        r0 = e1 * u;
        r1 = e0 * u;
        r2 = e3 * v;
        r3 = e2 * v;
    } else {
        r0 = rcp(e0);
        r1 = rcp(e1);
        r2 = rcp(e2);
        r3 = rcp(e3);
    }
    const Real em = fmin(fmin(e0, e1), fmin(e2, e3));
    auto pow6 = [](Real x) {
        const Real x2 = x * x;
        return x2 * x2 * x2;
    };
    Real g0, g1, g2, g3;
    if constexpr (sizeof(Real) == 8) {
        const Real An = em * rcp(em + tau), Bn = An * tau;
        g0 = pow6(fma(Bn, r0, An));
        g1 = pow6(fma(Bn, r1, An));
        g2 = pow6(fma(Bn, r2, An));
        g3 = pow6(fma(Bn, r3, An));
    } else {
        const Real inv = rcp(em + tau);
        const Real An = em * inv, Cm = em * (tau * inv);
        g0 = pow6(fma(Cm, r0, An));
        g1 = pow6(fma(Cm, r1, An));
        g2 = pow6(fma(Cm, r2, An));
        g3 = pow6(fma(Cm, r3, An));
    }
    const Real thr = ct * (g0 + g1 + g2 + g3);
    const Real w0 = g0 >= thr ? Real(1) : Real(0), w1 = g1 >= thr ? Real(9) : Real(0);
    const Real w2 = g2 >= thr ? Real(6) : Real(0), w3 = g3 >= thr ? Real(4) : Real(0);
    // candidates: 6 p_0..2 and 12 p_3
    const Real p0 = Real(2) * a - Real(7) * b + Real(11) * c;
    const Real p1 = -b + Real(5) * c + Real(2) * d;
    const Real p2 = Real(2) * c + Real(5) * d - e;
    const Real p3 = Real(3) * c + Real(13) * d - Real(5) * e + f;
    const Real num = Real(2) * (w0 * p0 + w1 * p1 + w2 * p2) + w3 * p3;
    return num * rcp(Real(12) * (w0 + w1 + w2 + w3));
}

// Both TENO6-A states of the face between cells i and i+1 from v_{i-2..i+3}.
template <typename Real>
__device__ __forceinline__ void teno6a_pair(Real a, Real b, Real c, Real d, Real e, Real f, Real eps, Real& vl,
                                            Real& vr)
{
    const Real ct = teno6a_cutoff(a, b, c, d, e, f);
    vl = teno6a_one(a, b, c, d, e, f, eps, ct);
    vr = teno6a_one(f, e, d, c, b, a, eps, ct);
}

// Face states by WENO5-Z or TENO6-A of characteristic variables (Sec. 3.2 steps 1-4 and
// the appendix eigenvectors).  st(s, m): component m of W at stencil slot s,
// slots 0..5 = cells f-3 .. f+2 around the face between cells f-1 and f.  The
// frozen face state is the mean of cells f-1 and f.  With rho c the acoustic
// impedance and rho c^2 taken there, the projection K^{-1} W gives the
// acoustic variables (p -/+ (rho c) u_n) / (2 rho c^2), the densities minus
// their acoustic part (rho_k - (rho_k / (rho c^2)) p), and the tangential
// velocities and the volume fraction unchanged; each is reconstructed from both
// sides and mapped back with K.  (WENO5-Z does not see a per-field scale;
// TENO6-A's cut-off does, so the variables are K^{-1} W exactly.)
template <typename Real, int MODEL, int DIR, bool TENO, typename Stencil>
__device__ __forceinline__ void char_face_states(const Material<Real>& mat, Stencil st, Real eps, Real* wl, Real* wr)
{
    constexpr int NC = Layout<MODEL>::NC, V = Layout<MODEL>::V, P = Layout<MODEL>::P;
    constexpr int UN = V + DIR, T1 = V + (DIR + 1) % 3, T2 = V + (DIR + 2) % 3;
    constexpr int ND = MODEL == DIM ? 2 : 1;  // density fields
    Real wf[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) wf[m] = Real(0.5) * (st(2, m) + st(3, m));
    const Real rc2 = rhoc2<Real, MODEL>(mat, wf);
    const Real irc2 = rcp(rc2);
    const Real z = sqrt_fast(density<Real, MODEL>(wf) * rc2);  // rho c
    const Real hh = Real(0.5) * irc2, zh = z * hh;             // 1/(2 rho c^2), 1/(2 c)
    const Real cs = rc2 * rcp(z);                              // c
    Real g[ND];
#pragma unroll
    for (int k = 0; k < ND; k++) g[k] = wf[k] * irc2;
    auto both = [&](auto field, Real& L, Real& R) {
        Real q[6];
#pragma unroll
        for (int s = 0; s < 6; s++) q[s] = field(s);
        if constexpr (TENO) {
            teno6a_pair(q[0], q[1], q[2], q[3], q[4], q[5], eps, L, R);
        } else {
            L = weno5z_one(q[0], q[1], q[2], q[3], q[4], eps);
            R = weno5z_one(q[5], q[4], q[3], q[2], q[1], eps);
        }
    };
    Real amL, amR, apL, apR;
    both([&](int s) { return fma(-zh, st(s, UN), hh * st(s, P)); }, amL, amR);
    both([&](int s) { return fma(zh, st(s, UN), hh * st(s, P)); }, apL, apR);
    const Real pL = rc2 * (amL + apL), pR = rc2 * (amR + apR);
    wl[P] = pL;
    wr[P] = pR;
    wl[UN] = (apL - amL) * cs;
    wr[UN] = (apR - amR) * cs;
#pragma unroll
    for (int k = 0; k < ND; k++) {
        Real eL, eR;
        both([&](int s) { return st(s, k) - g[k] * st(s, P); }, eL, eR);
        wl[k] = eL + g[k] * pL;
        wr[k] = eR + g[k] * pR;
    }
    both([&](int s) { return st(s, T1); }, wl[T1], wr[T1]);
    both([&](int s) { return st(s, T2); }, wl[T2], wr[T2]);
    if constexpr (MODEL == DIM) both([&](int s) { return st(s, 6); }, wl[6], wr[6]);
}

// ---------------------------------------------------------------- THINC
// Interface capturing of the five-equation model (Sec. 3.2, after the
// reconstruction).  A cell is an interface cell when eps <= a0 <= 1 - eps
// (eps = 1e-4) and the volume fraction is monotone through it along the face
// normal (am, a0, ap).  Its profile over the cell, xt in [0, 1] from its -d
// face, is (1 + theta tanh(beta (xt + x_c))) / 2 with theta = sgn(ap - am),
// beta = |n_d| + 0.01 (n = grad psi / |grad psi| of the smoothed volume fraction
// of Sec. 3.7, see thinc_psi; g_d and gn2 = |grad psi|^2 in any common scale) and
// x_c such that the profile's mean is a0:
//   T = tanh(beta x_c) = (exp(theta beta (2 a0 - 1)) - cosh beta) / sinh beta.
// Face values: (1 + theta T) / 2 at the -d face (side 0) and
// (1 + theta tanh(beta + beta x_c)) / 2 at the +d face (side 1), the latter
// from the addition theorem.  Returns false (af untouched) outside interface cells.
// Smoothed volume fraction from which the interface normal is taken (Sec. 3.7):
// psi = a^0.1 / (a^0.1 + (1 - a)^0.1), with a clamped to [0, 1] (rounding can
// leave it a few ulps outside, where the power is undefined).  In FP32 evaluated as
// 1 / (1 + 2^(0.1 log2((1 - a) / a))), one logarithm and one exponential instead of
// two powers (a = 0 and a = 1 give 0 and 1 through the infinities of the quotient and
// the logarithm): the five-equation THINC stage at 256x128x128 took 0.57 against
// 0.67 ms.  In FP64 that form has a quarter of the arithmetic (187 against 442
// instructions) but raised the stage kernel's register spills (172 -> 214 VGPRs) and
// its time (1.45 against 1.42 ms), so FP64 keeps the two powers.
template <typename Real>
__device__ __forceinline__ Real thinc_psi(Real a)
{
    a = fmin(Real(1), fmax(Real(0), a));
    if constexpr (sizeof(Real) == 4) {
        return Real(1) / (Real(1) + exp2(Real(0.1) * log2((Real(1) - a) / a)));
    } else {
        const Real p = pow(a, Real(0.1)), q = pow(Real(1) - a, Real(0.1));
        return p / (p + q);
    }
}

template <typename Real>
__device__ __forceinline__ bool thinc_face(Real am, Real a0, Real ap, Real gd, Real gn2, int side, Real& af)
{
    if (!(a0 >= Real(1e-4) && a0 <= Real(1) - Real(1e-4) && (ap - a0) * (a0 - am) > Real(0))) return false;
    const Real theta = ap > am ? Real(1) : Real(-1);
    const Real beta = fabs(gd) * rsqrt(gn2) + Real(0.01);
    const Real eb = exp(beta), ieb = rcp(eb);
    const Real ch = Real(0.5) * (eb + ieb), sh = Real(0.5) * (eb - ieb);
    const Real Q = exp(theta * beta * (Real(2) * a0 - Real(1)));
    const Real T = (Q - ch) * rcp(sh);
    Real t = T;
    if (side) {
        const Real tb = sh * rcp(ch);
        t = (tb + T) * rcp(Real(1) + tb * T);
    }
    af = Real(0.5) * (Real(1) + theta * t);
    return true;
}

// THINC face state of a cell (five-equation layout): volume fraction af and the
// partial densities from the cell's phase densities rho_k = (alpha_k rho_k) / alpha_k;
// velocity and pressure keep the reconstructed values.
template <typename Real>
__device__ __forceinline__ void thinc_state(Real af, Real ar1, Real ar2, Real a0, Real* w)
{
    w[6] = af;
    w[0] = af * (ar1 * rcp(a0));
    w[1] = (Real(1) - af) * (ar2 * rcp(Real(1) - a0));
}

// ---------------------------------------------------------------- HLLC
// Face normal to direction DIR.  wl, wr: primitive states.  F: flux F^c in
// the global frame; uh: upwinded normal velocity u^HLLC.  Wave speeds:
// Einfeldt with Roe-averaged u-bar and c-bar, s* after Batten.  sgn(0) = 0:
// for s* == 0 both star-side fluxes are averaged.
template <typename Real, int MODEL, int DIR>
__device__ __forceinline__ void hllc_side(const Material<Real>& mat, const Real* w, Real rho, Real un, Real sK,
                                          Real sw, Real sstar, Real* F, Real& uh)
{
    constexpr int V = Layout<MODEL>::V, P = Layout<MODEL>::P;
    const Real p = w[P];
    const Real r = rcp(sK - sstar);
    const Real fac = (sK - un) * r;           // (s^K - u^K)/(s^K - s*)
    const Real q = un + sw * (fac - Real(1));  // flux of any advected density per unit density
    const Real ke = Real(0.5) * rho * (w[V] * w[V] + w[V + 1] * w[V + 1] + w[V + 2] * w[V + 2]);
    const Real E = rho_e<Real, MODEL>(mat, w) + ke;
    if constexpr (MODEL == DIM) {
        F[0] = w[0] * q;
        F[1] = w[1] * q;
        F[6] = w[6] * q;
    } else {
        F[0] = rho * q;
    }
#pragma unroll
    for (int m = 0; m < 3; m++) {
        if (m == DIR) continue;
        F[V + m] = rho * w[V + m] * q;
    }
    // normal momentum: rho u^2 + p + sw (fac rho s* - rho u)
    F[V + DIR] = rho * un * un + p + sw * (fac * rho * sstar - rho * un);
    // energy: u (E + p) + sw (E* - E),
    //   E* = fac (E + (s* - u)(rho s* + p/(s^K - u))) = fac (E + (s*-u) rho s*) + (s*-u) p r
    const Real ds = sstar - un;
    const Real Estar = fac * (E + ds * rho * sstar) + ds * p * r;
    F[P] = un * (E + p) + sw * (Estar - E);
    uh = q;
}

template <typename Real, int MODEL, int DIR>
__device__ __forceinline__ void hllc(const Material<Real>& mat, const Real* wl, const Real* wr, Real* F, Real& uh)
{
    constexpr int V = Layout<MODEL>::V, P = Layout<MODEL>::P, NC = Layout<MODEL>::NC;
    const Real rhoL = density<Real, MODEL>(wl), rhoR = density<Real, MODEL>(wr);
    const Real uL = wl[V + DIR], uR = wr[V + DIR];
    const Real pL = wl[P], pR = wr[P];
    // sqrt(rho) and 1/rho from one reciprocal square root per side
    const Real yL = rsqrt(rhoL), yR = rsqrt(rhoR);
    const Real sqL = rhoL * yL, sqR = rhoR * yR;
    const Real rc2L = rhoc2<Real, MODEL>(mat, wl), rc2R = rhoc2<Real, MODEL>(mat, wr);
    const Real c2L = rc2L * (yL * yL), c2R = rc2R * (yR * yR);
    const Real cL = sqrt_fast(rc2L) * yL, cR = sqrt_fast(rc2R) * yR;
    const Real isum = rcp(sqL + sqR);
    const Real ubar = (sqL * uL + sqR * uR) * isum;
    const Real du = uR - uL;
    const Real cbar2 = (sqL * c2L + sqR * c2R) * isum + Real(0.5) * sqL * sqR * isum * isum * du * du;
    const Real cbar = sqrt_fast(cbar2);
    const Real sL = fmin(ubar - cbar, uL - cL);
    const Real sR = fmax(ubar + cbar, uR + cR);
    const Real mL = rhoL * (sL - uL), mR = rhoR * (sR - uR);
    const Real sstar = ((pR - pL) + (mL * uL - mR * uR)) * rcp(mL - mR);
    const Real sminus = fmin(Real(0), sL), splus = fmax(Real(0), sR);
    // upwind side by operand selection (sgn(0) = 0 averages both sides below)
    const bool left = !(sstar < Real(0));
    Real ws[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) ws[m] = left ? wl[m] : wr[m];
    Real Fa[NC];
    Real uha;
    hllc_side<Real, MODEL, DIR>(mat, ws, left ? rhoL : rhoR, left ? uL : uR, left ? sL : sR,
                                left ? sminus : splus, sstar, Fa, uha);
    if (sstar == Real(0)) {
        Real Fb[NC];
        Real uhb;
        hllc_side<Real, MODEL, DIR>(mat, wr, rhoR, uR, sR, splus, sstar, Fb, uhb);
#pragma unroll
        for (int m = 0; m < NC; m++) Fa[m] = Real(0.5) * Fa[m] + Real(0.5) * Fb[m];
        uha = Real(0.5) * uha + Real(0.5) * uhb;
    }
#pragma unroll
    for (int m = 0; m < NC; m++) F[m] = Fa[m];
    uh = uha;
}

// ---------------------------------------------------------------- admissibility
// 1 if the primitive state violates any loop of the interpolation limiter
// (densities, volume fraction, rho c^2).
template <typename Real, int MODEL>
__device__ __forceinline__ bool inadmissible_w(const Material<Real>& mat, const Tolerances<Real>& tol,
                                               const Real* w)
{
    bool bad;
    if constexpr (MODEL == DIM) {
        bad = (w[0] < tol.eps_rho) || (w[1] < tol.eps_rho) || (w[6] < tol.eps_alpha) ||
              (w[6] > Real(1) - tol.eps_alpha);
    } else {
        bad = w[0] < tol.eps_rho;
    }
    return bad || (rhoc2<Real, MODEL>(mat, w) < tol.eps_rhoc2);
}

// Convective flux F^c of a primitive state in direction DIR.
template <typename Real, int MODEL, int DIR>
__device__ __forceinline__ void physical_flux(const Material<Real>& mat, const Real* w, Real* F)
{
    constexpr int V = Layout<MODEL>::V, P = Layout<MODEL>::P;
    const Real rho = density<Real, MODEL>(w);
    const Real un = w[V + DIR];
    if constexpr (MODEL == DIM) {
        F[0] = w[0] * un;
        F[1] = w[1] * un;
        F[6] = w[6] * un;
    } else {
        F[0] = rho * un;
    }
#pragma unroll
    for (int m = 0; m < 3; m++) F[V + m] = rho * un * w[V + m];
    F[V + DIR] += w[P];
    const Real ke = Real(0.5) * rho * (w[V] * w[V] + w[V + 1] * w[V + 1] + w[V + 2] * w[V + 2]);
    F[P] = un * (rho_e<Real, MODEL>(mat, w) + ke + w[P]);
}

// Flux limiter test (Sec. 3.3 item 2): split forward-Euler states of the two
// cells adjacent to the face, U_i - lam (F - F(U_i)) and U_{i+1} + lam (F -
// F(U_{i+1})) with lam = 2 D dt/dx; the volume fraction uses its
// quasi-conservative split with the u^HLLC source.  Returns true if either
// state violates a loop's tolerance.
template <typename Real, int MODEL, int DIR>
__device__ __forceinline__ bool flux_limiter_trips(const Material<Real>& mat, const Tolerances<Real>& tol,
                                                   const Real* wi, const Real* wj, const Real* F, Real uh,
                                                   Real lam)
{
    constexpr int NC = Layout<MODEL>::NC;
    bool bad = false;
#pragma unroll
    for (int side = 0; side < 2; side++) {
        const Real* w = side == 0 ? wi : wj;
        const Real sg = side == 0 ? -lam : lam;
        Real u[NC], f[NC], us[NC], ws[NC];
        prim_to_cons<Real, MODEL>(mat, w, u);
        physical_flux<Real, MODEL, DIR>(mat, w, f);
#pragma unroll
        for (int m = 0; m < NC; m++) us[m] = u[m] + sg * (F[m] - f[m]);
        if constexpr (MODEL == DIM) us[6] = u[6] + sg * (F[6] - u[6] * uh);
        cons_to_prim<Real, MODEL>(mat, us, ws);
        bad = bad || inadmissible_w<Real, MODEL>(mat, tol, ws);
    }
    return bad;
}

// ---------------------------------------------------------------- viscous
template <typename Real>
__device__ __forceinline__ Real visc_mu(const ViscLaw<Real>& v, Real theta)
{
    if (v.law == 0) return v.mu;
    const Real x = theta * v.inv_th_ref;  // T / T_ref
    if (v.law == 1) return v.mu * pow(x, Real(0.7));
    return v.mu * (x * sqrt_fast(x)) * (v.th_ref_c * rcp(theta + v.th_c));
}

// 4th-order central stencils:
//   face normal derivative  ((q_{-1} - q_{+2}) + 27 (q_{+1} - q_0)) / (24 h)
//   cell derivative         ((q_{-2} - q_{+2}) + 8 (q_{+1} - q_{-1})) / (12 h)
//   face interpolation      (9 (q_0 + q_{+1}) - (q_{-1} + q_{+2})) / 16
template <typename Real>
__device__ __forceinline__ Real dface(Real a, Real b, Real c, Real d, Real inv24h)
{
    return ((a - d) + Real(27) * (c - b)) * inv24h;
}
template <typename Real>
__device__ __forceinline__ Real dcell(Real m2, Real m1, Real p1, Real p2, Real inv12h)
{
    return ((m2 - p2) + Real(8) * (p1 - m1)) * inv12h;
}
template <typename Real>
__device__ __forceinline__ Real ifc(Real a, Real b, Real c, Real d)
{
    return (Real(9) * (b + c) - (a + d)) * Real(0.0625);
}

// Dissipative flux F^d at a face normal to DIR.
//  q[s][0..3] = (u, v, w, T) at the four cells -1, 0, +1, +2 across the face
//  (T = p / rho; the gas constant cancels in kappa = mu gamma/((gamma-1) Pr)),
//  dt1n[s] = d u_n / d x_t1, dt2n[s] = d u_n / d x_t2, dt1t1[s] = d u_t1 / d x_t1,
//  dt2t2[s] = d u_t2 / d x_t2 at those cells (t1, t2 = the tangential axes in
//  increasing order).  Output Fd[0..3] = (tau_n1, tau_n2, tau_n3, sum_i u_i tau_ni - q_n).
template <typename Real, int DIR>
__device__ __forceinline__ void viscous_flux(const Real (*q)[4], const Real* dt1n, const Real* dt2n,
                                             const Real* dt1t1, const Real* dt2t2, Real mu, Real kappa,
                                             Real inv24h, Real* Fd)
{
    constexpr int T1 = DIR == 0 ? 1 : 0;
    constexpr int T2 = DIR == 2 ? 1 : 2;
    Real dn[4];
#pragma unroll
    for (int c = 0; c < 4; c++) dn[c] = dface(q[0][c], q[1][c], q[2][c], q[3][c], inv24h);
    Real vf[3];
#pragma unroll
    for (int c = 0; c < 3; c++) vf[c] = ifc(q[0][c], q[1][c], q[2][c], q[3][c]);
    const Real g_t1n = ifc(dt1n[0], dt1n[1], dt1n[2], dt1n[3]);
    const Real g_t2n = ifc(dt2n[0], dt2n[1], dt2n[2], dt2n[3]);
    const Real g_t1t1 = ifc(dt1t1[0], dt1t1[1], dt1t1[2], dt1t1[3]);
    const Real g_t2t2 = ifc(dt2t2[0], dt2t2[1], dt2t2[2], dt2t2[3]);
    const Real div = dn[DIR] + g_t1t1 + g_t2t2;
    Real tau[3];
    tau[DIR] = mu * (Real(2) * dn[DIR]) - Real(2.0 / 3.0) * mu * div;
    tau[T1] = mu * (g_t1n + dn[T1]);
    tau[T2] = mu * (g_t2n + dn[T2]);
    Fd[0] = tau[0];
    Fd[1] = tau[1];
    Fd[2] = tau[2];
    Fd[3] = vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2] + kappa * dn[3];
}

// The flux from face gradients already formed: dn[c] = d q_c / d x_n (c = u, v,
// w, T), vf = face velocity, and the interpolated tangential derivatives
// g_t1n = d u_n/d x_t1, g_t2n = d u_n/d x_t2, g_t1t1, g_t2t2.
template <typename Real, int DIR>
__device__ __forceinline__ void viscous_flux_from_gradients(const Real* dn, const Real* vf, Real g_t1n, Real g_t2n,
                                                            Real g_t1t1, Real g_t2t2, Real mu, Real kappa, Real* Fd)
{
    constexpr int T1 = DIR == 0 ? 1 : 0;
    constexpr int T2 = DIR == 2 ? 1 : 2;
    const Real div = dn[DIR] + g_t1t1 + g_t2t2;
    Real tau[3];
    tau[DIR] = mu * (Real(2) * dn[DIR]) - Real(2.0 / 3.0) * mu * div;
    tau[T1] = mu * (g_t1n + dn[T1]);
    tau[T2] = mu * (g_t2n + dn[T2]);
    Fd[0] = tau[0];
    Fd[1] = tau[1];
    Fd[2] = tau[2];
    Fd[3] = vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2] + kappa * dn[3];
}

// The same flux reading its inputs from LDS one quantity at a time.
//  vel: &u at the first of the four cells (u, v, w are `fstride` apart),
//  temp: &T at the first cell; consecutive cells are `cstride` apart.
//  t1n, t2n, t1t1, t2t2: d u_n/d x_t1, d u_n/d x_t2, d u_t1/d x_t1, d u_t2/d x_t2
//  at the first cell, consecutive cells `dstride` apart.
template <typename Real, int DIR>
__device__ __forceinline__ void viscous_flux_lds(const Real* vel, const Real* temp, int cstride, int fstride,
                                                 const Real* t1n, const Real* t2n, const Real* t1t1,
                                                 const Real* t2t2, int dstride, Real mu, Real kappa, Real inv24h,
                                                 Real* Fd)
{
    constexpr int T1 = DIR == 0 ? 1 : 0;
    constexpr int T2 = DIR == 2 ? 1 : 2;
    Real dn[4], vf[3];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const Real* q = c < 3 ? vel + c * fstride : temp;
        const Real a = q[0], b = q[cstride], cc = q[2 * cstride], d = q[3 * cstride];
        dn[c] = dface(a, b, cc, d, inv24h);
        if (c < 3) vf[c] = ifc(a, b, cc, d);
    }
    auto itp = [&](const Real* t) { return ifc(t[0], t[dstride], t[2 * dstride], t[3 * dstride]); };
    const Real g_t1n = itp(t1n), g_t2n = itp(t2n), g_t1t1 = itp(t1t1), g_t2t2 = itp(t2t2);
    const Real div = dn[DIR] + g_t1t1 + g_t2t2;
    Real tau[3];
    tau[DIR] = mu * (Real(2) * dn[DIR]) - Real(2.0 / 3.0) * mu * div;
    tau[T1] = mu * (g_t1n + dn[T1]);
    tau[T2] = mu * (g_t2n + dn[T2]);
    Fd[0] = tau[0];
    Fd[1] = tau[1];
    Fd[2] = tau[2];
    Fd[3] = vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2] + kappa * dn[3];
}

// ---------------------------------------------------------------- boundary mapping
// Index of the interior cell that supplies global index g along an axis of n
// cells; toggles flip when a symmetry mirror was crossed.  Indices further out
// than a mirror image (only reached by cells of ragged tiles that lie outside
// the domain and are never written) are clamped.
__device__ __forceinline__ int map_index(int g, int n, int lo, int hi, bool& flip)
{
    if (g < 0) {
        if (lo == PERIODIC) {
            int r = g % n;
            return r < 0 ? r + n : r;
        }
        if (lo == ZEROGRAD) return 0;
        flip = !flip;
        int r = -g - 1;
        return r < n ? r : n - 1;
    }
    if (g >= n) {
        if (hi == PERIODIC) return g % n;
        if (hi == ZEROGRAD) return n - 1;
        flip = !flip;
        int r = 2 * n - 1 - g;
        return r >= 0 ? r : 0;
    }
    return g;
}

}  // namespace fv
