// fv_adjoint.hip -- discrete adjoint of the single-phase Euler right-hand side
// (vector-Jacobian product of Eq. (FVD) with WENO5-Z and HLLC, Sec. 3.2) and
// of the TVD-RK3 step at a fixed time step (Sec. 3.4), the reverse sweep that
// the paper obtains by automatic differentiation (Sec. 6).
//
// One thread per face: it rebuilds the face's six-cell stencil (boundary
// conditions by index mapping, as the stage kernel reads them), the two WENO
// face states and the HLLC flux, then pulls the face cotangent
//   Fbar_f = (Rbar_f - Rbar_{f-1}) / h        (R_i = -(F_{i+1/2} - F_{i-1/2}) / h)
// back through HLLC, WENO5-Z and the U -> W map (reverse sweeps written out
// below), and adds the six cells' cotangents to Ubar with atomic adds.
// Non-differentiable points take the conventions of the adjoint's reference:
// |x|' = sgn(x) with sgn(0) = 0; min / max at a tie split the cotangent evenly; the
// upwind switch of the HLLC flux (the sign of s*) is piecewise constant; the
// hardware-estimate helpers rcp, rsqrt and sqrt_fast are differentiated exactly
// (d(1/x) = -dx/x^2, ...), not through their refinement steps.  The order of the atomic additions is not fixed, so
// the result is reproducible to round-off, not bitwise.
#include <hip/hip_runtime.h>

#include "fv_kernels.h"

namespace fv {

namespace {

constexpr int ADJ_THREADS = 128;

// Reverse sweep of weno5z_one: adds vb * d v / d(a, b, c, d, e) to g[0..4].
// The forward steps are those of weno5z_one (fv_physics.h): smoothness
// indicators, the WENO-Z factors g_k = 1 + tau/(beta_k + eps), weights scaled
// by 10 (1, 6, 3) g_k, candidate values scaled by 6, v = N / D.
__device__ __forceinline__ void weno5z_one_vjp(double a, double b, double c, double d, double e, double eps,
                                               double vb, double* g)
{
    const double k13 = 13.0 / 12.0, q = 0.25;
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = b - d;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double b0 = k13 * t0 * t0 + q * s0 * s0;
    const double b1 = k13 * t1 * t1 + q * s1 * s1;
    const double b2 = k13 * t2 * t2 + q * s2 * s2;
    const double diff = b0 - b2;
    const double tau = ::fabs(diff);
    const double r0 = rcp(b0 + eps), r1 = rcp(b1 + eps), r2 = rcp(b2 + eps);
    const double al0 = 1.0 + tau * r0, al1 = 6.0 * (1.0 + tau * r1), al2 = 3.0 * (1.0 + tau * r2);
    const double p0 = 2.0 * a - 7.0 * b + 11.0 * c;
    const double p1 = -b + 5.0 * c + 2.0 * d;
    const double p2 = 2.0 * c + 5.0 * d - e;
    const double iD = rcp(6.0 * (al0 + al1 + al2));
    const double v = (al0 * p0 + al1 * p1 + al2 * p2) * iD;
    // reverse
    const double Nb = vb * iD;
    const double Db6 = -6.0 * vb * v * iD;  // 6 * dL/dD
    const double ab0 = Nb * p0 + Db6, ab1 = Nb * p1 + Db6, ab2 = Nb * p2 + Db6;
    const double pb0 = Nb * al0, pb1 = Nb * al1, pb2 = Nb * al2;
    const double gb0 = ab0, gb1 = 6.0 * ab1, gb2 = 3.0 * ab2;  // dL/d(1 + tau r_k)
    const double taub = gb0 * r0 + gb1 * r1 + gb2 * r2;
    const double sg = diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0);
    const double bb0 = -gb0 * tau * r0 * r0 + sg * taub;
    const double bb1 = -gb1 * tau * r1 * r1;
    const double bb2 = -gb2 * tau * r2 * r2 - sg * taub;
    const double tb0 = 2.0 * k13 * t0 * bb0, sb0 = 2.0 * q * s0 * bb0;
    const double tb1 = 2.0 * k13 * t1 * bb1, sb1 = 2.0 * q * s1 * bb1;
    const double tb2 = 2.0 * k13 * t2 * bb2, sb2 = 2.0 * q * s2 * bb2;
    g[0] += 2.0 * pb0 + tb0 + sb0;
    g[1] += -7.0 * pb0 - pb1 - 2.0 * tb0 - 4.0 * sb0 + tb1 + sb1;
    g[2] += 11.0 * pb0 + 5.0 * pb1 + 2.0 * pb2 + tb0 + 3.0 * sb0 - 2.0 * tb1 + tb2 + 3.0 * sb2;
    g[3] += 2.0 * pb1 + 5.0 * pb2 + tb1 - sb1 - 2.0 * tb2 - 4.0 * sb2;
    g[4] += -pb2 + tb2 + sb2;
}

// Reverse sweep of the single-phase U -> W map: Ub = (dW/dU)^T Wb.
__device__ __forceinline__ void cons_to_prim_vjp(const Material<double>& mat, const double* w, const double* wb,
                                                 double* ub)
{
    const double ir = rcp(w[0]);
    const double gm1 = mat.gm1;
    const double ke = 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    ub[0] = wb[0] - (wb[1] * w[1] + wb[2] * w[2] + wb[3] * w[3]) * ir + wb[4] * gm1 * ke;
#pragma unroll
    for (int i = 0; i < 3; i++) ub[1 + i] = wb[1 + i] * ir - wb[4] * gm1 * w[1 + i];
    ub[4] = wb[4] * gm1;
}

// Reverse sweep of one star-side flux of hllc (hllc_side in fv_physics.h, single-phase
// layout): G is the cotangent of that side's flux; adds G . dF/dw to wb and returns the
// cotangents of the side's wave speed sK, its upwind factor sw and s*.
template <int DIR>
__device__ __forceinline__ void hllc_side_vjp(const Material<double>& mat, const double* w, double sK, double sw,
                                              double sstar, const double* G, double* wb, double& sKb, double& swb,
                                              double& sstarb)
{
    constexpr int V = 1, P = 4;
    const double rho = w[0], un = w[V + DIR], p = w[P];
    const double r = rcp(sK - sstar);
    const double fac = (sK - un) * r;
    const double q = un + sw * (fac - 1.0);
    const double v2 = w[V] * w[V] + w[V + 1] * w[V + 1] + w[V + 2] * w[V + 2];
    const double E = (p + mat.gpinf) * mat.iG1 + 0.5 * rho * v2;
    const double ds = sstar - un;
    const double Estar = fac * (E + ds * rho * sstar) + ds * p * r;
    const double Gn = G[V + DIR], Ge = G[P];
    // F[0] = rho q; tangential momenta rho u_t q
    double qb = G[0] * rho, rhob = G[0] * q;
#pragma unroll
    for (int m = 0; m < 3; m++) {
        if (m == DIR) continue;
        rhob += G[V + m] * w[V + m] * q;
        wb[V + m] += G[V + m] * rho * q;
        qb += G[V + m] * rho * w[V + m];
    }
    // normal momentum rho un^2 + p + sw (fac rho s* - rho un)
    rhob += Gn * (un * un + sw * (fac * sstar - un));
    double unb = Gn * (2.0 * rho * un - sw * rho);
    double pb = Gn;
    swb = Gn * (fac * rho * sstar - rho * un);
    double facb = Gn * sw * rho * sstar;
    sstarb = Gn * sw * fac * rho;
    // energy un (E + p) + sw (E* - E), E* = fac (E + ds rho s*) + ds p r
    unb += Ge * (E + p);
    double Eb = Ge * (un - sw);
    pb += Ge * un;
    swb += Ge * (Estar - E);
    const double Esb = Ge * sw;
    facb += Esb * (E + ds * rho * sstar);
    Eb += Esb * fac;
    const double dsb = Esb * (fac * rho * sstar + p * r);
    rhob += Esb * fac * ds * sstar;
    sstarb += Esb * fac * ds * rho;
    pb += Esb * ds * r;
    double rb = Esb * ds * p;
    sstarb += dsb;
    unb -= dsb;
    // E = (p + gpinf) / (gamma - 1) + rho |u|^2 / 2
    pb += Eb * mat.iG1;
    rhob += Eb * 0.5 * v2;
#pragma unroll
    for (int m = 0; m < 3; m++) wb[V + m] += Eb * rho * w[V + m];
    // q = un + sw (fac - 1); fac = (sK - un) r; r = 1 / (sK - s*)
    unb += qb;
    swb += qb * (fac - 1.0);
    facb += qb * sw;
    sKb = facb * r;
    unb -= facb * r;
    rb += facb * (sK - un);
    const double dKb = -rb * r * r;
    sKb += dKb;
    sstarb -= dKb;
    wb[0] += rhob;
    wb[V + DIR] += unb;
    wb[P] += pb;
}

// Reverse sweep of hllc<double, EULER, DIR> (fv_physics.h): adds g . dF/d(wl, wr) to
// wlb, wrb, the flux recomputed once and pulled back step by step in reverse order
// (s* = 0 averages the two star-side fluxes, so both are pulled back with half the
// cotangent).  Replaces ten forward-mode tangent evaluations of the flux (one per
// face-state input): the RHS adjoint at 64^3 took 0.25 against 0.34 ms.
template <int DIR>
__device__ __forceinline__ void hllc_vjp(const Material<double>& mat, const double* wl, const double* wr,
                                         const double* g, double* wlb, double* wrb)
{
    constexpr int V = 1, P = 4, NC = 5;
    // forward
    const double rhoL = wl[0], rhoR = wr[0], uL = wl[V + DIR], uR = wr[V + DIR], pL = wl[P], pR = wr[P];
    const double yL = rsqrt(rhoL), yR = rsqrt(rhoR);
    const double sqL = rhoL * yL, sqR = rhoR * yR;
    const double rc2L = mat.gamma * (pL + mat.pinf), rc2R = mat.gamma * (pR + mat.pinf);
    const double c2L = rc2L * (yL * yL), c2R = rc2R * (yR * yR);
    const double srL = sqrt_fast(rc2L), srR = sqrt_fast(rc2R);
    const double cL = srL * yL, cR = srR * yR;
    const double isum = rcp(sqL + sqR);
    const double ubar = (sqL * uL + sqR * uR) * isum;
    const double du = uR - uL;
    const double A = sqL * c2L + sqR * c2R;
    const double cbar2 = A * isum + 0.5 * sqL * sqR * isum * isum * du * du;
    const double cbar = sqrt_fast(cbar2);
    const double aL = ubar - cbar, bL = uL - cL, aR = ubar + cbar, bR = uR + cR;
    const double sL = ::fmin(aL, bL), sR = ::fmax(aR, bR);
    const double mL = rhoL * (sL - uL), mR = rhoR * (sR - uR);
    const double num = (pR - pL) + (mL * uL - mR * uR);
    const double rd = rcp(mL - mR);
    const double sstar = num * rd;
    const double sminus = ::fmin(0.0, sL), splus = ::fmax(0.0, sR);
    // star-side fluxes
    double sLb = 0.0, sRb = 0.0, smb = 0.0, spb = 0.0, sstarb = 0.0;
    if (sstar == 0.0) {
        double gh[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) gh[m] = 0.5 * g[m];
        double kb, wb, sb;
        hllc_side_vjp<DIR>(mat, wl, sL, sminus, sstar, gh, wlb, kb, wb, sb);
        sLb += kb;
        smb += wb;
        sstarb += sb;
        hllc_side_vjp<DIR>(mat, wr, sR, splus, sstar, gh, wrb, kb, wb, sb);
        sRb += kb;
        spb += wb;
        sstarb += sb;
    } else if (!(sstar < 0.0)) {
        hllc_side_vjp<DIR>(mat, wl, sL, sminus, sstar, g, wlb, sLb, smb, sstarb);
    } else {
        hllc_side_vjp<DIR>(mat, wr, sR, splus, sstar, g, wrb, sRb, spb, sstarb);
    }
    // s^- = min(0, sL), s^+ = max(0, sR)
    sLb += smb * (sL < 0.0 ? 1.0 : (sL == 0.0 ? 0.5 : 0.0));
    sRb += spb * (sR > 0.0 ? 1.0 : (sR == 0.0 ? 0.5 : 0.0));
    // s* = ((pR - pL) + mL uL - mR uR) / (mL - mR)
    const double numb = sstarb * rd;
    const double denb = -sstarb * num * rd * rd;
    double pLb = -numb, pRb = numb;
    const double mLb = numb * uL + denb, mRb = -numb * uR - denb;
    double uLb = numb * mL, uRb = -numb * mR;
    // m_K = rho_K (s_K - u_K)
    double rhoLb = mLb * (sL - uL), rhoRb = mRb * (sR - uR);
    sLb += mLb * rhoL;
    uLb -= mLb * rhoL;
    sRb += mRb * rhoR;
    uRb -= mRb * rhoR;
    // sL = min(ubar - cbar, uL - cL), sR = max(ubar + cbar, uR + cR)
    const double kL = aL < bL ? 1.0 : (bL < aL ? 0.0 : 0.5);
    const double kR = aR > bR ? 1.0 : (bR > aR ? 0.0 : 0.5);
    const double aLb = sLb * kL, bLb = sLb * (1.0 - kL), aRb = sRb * kR, bRb = sRb * (1.0 - kR);
    const double ubarb = aLb + aRb, cbarb = aRb - aLb;
    uLb += bLb;
    uRb += bRb;
    const double cLb = -bLb, cRb = bRb;
    // cbar = sqrt(cbar2), cbar2 = A isum + sqL sqR isum^2 du^2 / 2
    const double c2b = cbarb * 0.5 * rsqrt(cbar2);
    const double t = 0.5 * isum * isum * du * du;
    double sqLb = c2b * (sqR * t + c2L * isum), sqRb = c2b * (sqL * t + c2R * isum);
    double isumb = c2b * (A + sqL * sqR * isum * du * du);
    const double dub = c2b * sqL * sqR * isum * isum * du;
    const double c2Lb = c2b * isum * sqL, c2Rb = c2b * isum * sqR;
    uRb += dub;
    uLb -= dub;
    // ubar = (sqL uL + sqR uR) isum
    sqLb += ubarb * uL * isum;
    sqRb += ubarb * uR * isum;
    uLb += ubarb * sqL * isum;
    uRb += ubarb * sqR * isum;
    isumb += ubarb * (sqL * uL + sqR * uR);
    // isum = 1 / (sqL + sqR)
    const double ssb = -isumb * isum * isum;
    sqLb += ssb;
    sqRb += ssb;
    // c_K = sqrt(rc2_K) y_K, c2_K = rc2_K y_K^2, sq_K = rho_K y_K, y_K = rho_K^-1/2
    const double rc2Lb = cLb * yL * 0.5 * rsqrt(rc2L) + c2Lb * yL * yL;
    const double rc2Rb = cRb * yR * 0.5 * rsqrt(rc2R) + c2Rb * yR * yR;
    const double yLb = cLb * srL + c2Lb * 2.0 * rc2L * yL + sqLb * rhoL;
    const double yRb = cRb * srR + c2Rb * 2.0 * rc2R * yR + sqRb * rhoR;
    rhoLb += sqLb * yL - 0.5 * yLb * yL * yL * yL;
    rhoRb += sqRb * yR - 0.5 * yRb * yR * yR * yR;
    pLb += rc2Lb * mat.gamma;
    pRb += rc2Rb * mat.gamma;
    wlb[0] += rhoLb;
    wlb[V + DIR] += uLb;
    wlb[P] += pLb;
    wrb[0] += rhoRb;
    wrb[V + DIR] += uRb;
    wrb[P] += pRb;
}

template <int DIR>
__device__ __forceinline__ void face_adjoint_body(const AdjointArgs& a, const double ih, const long long t,
                                                  const double* __restrict__ U, const double* __restrict__ Rbar,
                                                  double* __restrict__ Ubar)
{
    constexpr int NC = 5, V = 1;
    const int n = DIR == 0 ? a.nx : (DIR == 1 ? a.ny : a.nz);
    const long long lines = a.ncell / n;
    if (t >= lines * (n + 1)) return;
    // consecutive threads take consecutive x: along the line for x faces, across the
    // lines for y and z faces (coalesced loads and accumulations)
    int f;           // face f lies between cells f-1 and f of the line
    int ci, cj, ck;  // coordinates of the line's cells; the DIR one is set per cell below
    if (DIR == 0) {
        f = (int)(t % (n + 1));
        const long long line = t / (n + 1);
        ci = 0;
        cj = (int)(line % a.ny);
        ck = (int)(line / a.ny);
    } else {
        ci = (int)(t % a.nx);
        const long long r = t / a.nx;
        f = (int)(r % (n + 1));
        const int o = (int)(r / (n + 1));
        cj = DIR == 1 ? 0 : o;
        ck = DIR == 1 ? o : 0;
    }
    const long long stride = DIR == 0 ? 1 : (DIR == 1 ? (long long)a.nx : (long long)a.nx * a.ny);
    const long long base = ((long long)ck * a.ny + cj) * a.nx + ci;  // cell 0 of the line
    const int blo = a.bc[2 * DIR], bhi = a.bc[2 * DIR + 1];
    const Material<double> mat = a.mat;

    // stencil cells f-3 .. f+2: mapped index, mirror flag and primitive state
    long long q[6];
    bool flip[6];
    double w[6][NC];
#pragma unroll
    for (int s = 0; s < 6; s++) {
        bool fl = false;
        const int g = map_index(f - 3 + s, n, blo, bhi, fl);
        q[s] = base + g * stride;
        flip[s] = fl;
        double u[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) u[m] = U[m * a.ncell + q[s]];
        if (fl) u[V + DIR] = -u[V + DIR];
        cons_to_prim<double, EULER>(mat, u, w[s]);
    }
    // cotangent of the face flux
    double g[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        double v = 0.0;
        if (f < n) v += Rbar[m * a.ncell + base + f * stride];
        if (f >= 1) v -= Rbar[m * a.ncell + base + (f - 1) * stride];
        g[m] = v * ih;
    }
    // face states: left = v^- of cell f-1 (stencil slots 0..4), right = v^+ of cell f (slots
    // 1..5, the mirrored stencil); the same values as the stage kernel's pair reconstruction
    double wl[NC], wr[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        double vm, vp, x0, x1;
        weno5z_pair(w[0][m], w[1][m], w[2][m], w[3][m], w[4][m], a.weps, vm, x0);
        weno5z_pair(w[1][m], w[2][m], w[3][m], w[4][m], w[5][m], a.weps, x1, vp);
        wl[m] = vm;
        wr[m] = vp;
    }
    // HLLC: cotangents of the two face states
    double wlb[NC], wrb[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) {
        wlb[m] = 0.0;
        wrb[m] = 0.0;
    }
    hllc_vjp<DIR>(mat, wl, wr, g, wlb, wrb);
    // WENO5-Z: cotangents of the stencil's primitive states (reverse sweeps)
    double wb[6][NC];
#pragma unroll
    for (int s = 0; s < 6; s++)
#pragma unroll
        for (int m = 0; m < NC; m++) wb[s][m] = 0.0;
#pragma unroll
    for (int m = 0; m < NC; m++) {
        double gl[5] = {0, 0, 0, 0, 0}, gr[5] = {0, 0, 0, 0, 0};
        weno5z_one_vjp(w[0][m], w[1][m], w[2][m], w[3][m], w[4][m], a.weps, wlb[m], gl);
        weno5z_one_vjp(w[5][m], w[4][m], w[3][m], w[2][m], w[1][m], a.weps, wrb[m], gr);
#pragma unroll
        for (int k = 0; k < 5; k++) {
            wb[k][m] += gl[k];
            wb[5 - k][m] += gr[k];
        }
    }
    // U -> W, then the boundary mapping
#pragma unroll
    for (int s = 0; s < 6; s++) {
        double ub[NC];
        cons_to_prim_vjp(mat, w[s], wb[s], ub);
        if (flip[s]) ub[V + DIR] = -ub[V + DIR];
#pragma unroll
        for (int m = 0; m < NC; m++) atomicAdd(&Ubar[m * a.ncell + q[s]], ub[m]);
    }
}

// The three directions in one launch: blocks [0, b1) take the x faces, [b1, b2) the y
// faces, the rest the z faces.  At one wave per SIMD a 64^3 direction alone fills about
// four rounds of workgroups and a nearly empty fifth; one launch for all three leaves a
// single partial round (RHS adjoint at 64^3 0.257 -> 0.222 ms).
__global__ void __launch_bounds__(ADJ_THREADS) face_adjoint_all(const AdjointArgs a, const unsigned b1, const unsigned b2,
                                                                const double* __restrict__ U,
                                                                const double* __restrict__ Rbar,
                                                                double* __restrict__ Ubar)
{
    const unsigned b = blockIdx.x;
    if (b < b1) face_adjoint_body<0>(a, a.idx, (long long)b * ADJ_THREADS + threadIdx.x, U, Rbar, Ubar);
    else if (b < b2) face_adjoint_body<1>(a, a.idy, (long long)(b - b1) * ADJ_THREADS + threadIdx.x, U, Rbar, Ubar);
    else face_adjoint_body<2>(a, a.idz, (long long)(b - b2) * ADJ_THREADS + threadIdx.x, U, Rbar, Ubar);
}

__global__ void fill_zero_kernel(double* __restrict__ p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// out = c0 x0 + c1 x1 + c2 x2 + c3 x3 (null x terms are skipped); out may alias an input
__global__ void lincomb_kernel(double* out, long long n, double c0, const double* x0, double c1, const double* x1,
                               double c2, const double* x2, double c3, const double* x3)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double v = c0 * x0[i];
        if (x1) v += c1 * x1[i];
        if (x2) v += c2 * x2[i];
        if (x3) v += c3 * x3[i];
        out[i] = v;
    }
}

int grid_for(long long n, int threads)
{
    long long b = (n + threads - 1) / threads;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_rhs_adjoint(const AdjointArgs& a, const double* U, const double* Rbar, double* Ubar, hipStream_t st)
{
    const long long total = a.ncell * 5;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(total, 256)), dim3(256), 0, st, Ubar, total);
    unsigned blocks[3];
    for (int d = 0; d < 3; d++) {
        const int n = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
        const long long faces = a.ncell / n * (n + 1);
        blocks[d] = (unsigned)((faces + ADJ_THREADS - 1) / ADJ_THREADS);
    }
    hipLaunchKernelGGL(face_adjoint_all, dim3(blocks[0] + blocks[1] + blocks[2]), dim3(ADJ_THREADS), 0, st, a, blocks[0],
                       blocks[0] + blocks[1], U, Rbar, Ubar);
    return hipGetLastError();
}

hipError_t launch_lincomb(double* out, long long n, double c0, const double* x0, double c1, const double* x1, double c2,
                          const double* x2, double c3, const double* x3, hipStream_t st)
{
    hipLaunchKernelGGL(lincomb_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, out, n, c0, x0, c1, x1, c2, x2, c3,
                       x3);
    return hipGetLastError();
}

}  // namespace fv
