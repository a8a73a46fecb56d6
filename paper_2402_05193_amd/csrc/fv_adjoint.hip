// fv_adjoint.hip -- discrete adjoint of the single-phase Euler right-hand side
// (vector-Jacobian product of Eq. (FVD) with WENO5-Z and HLLC, Sec. 3.2) and
// of the TVD-RK3 step at a fixed time step (Sec. 3.4), the reverse sweep that
// the paper obtains by automatic differentiation (Sec. 6).
//
// One thread per face: it rebuilds the face's six-cell stencil (boundary
// conditions by index mapping, as the stage kernel reads them), the two WENO
// face states and the HLLC flux, then pulls the face cotangent
//   Fbar_f = (Rbar_f - Rbar_{f-1}) / h        (R_i = -(F_{i+1/2} - F_{i-1/2}) / h)
// back through HLLC (forward-mode tangents of the same device function,
// fv_dual.h, one per face-state input), WENO5-Z and the U -> W map (reverse
// sweeps written out below), and adds the six cells' cotangents to Ubar with
// atomic adds.  The order of the atomic additions is not fixed, so
// the result is reproducible to round-off, not bitwise.
#include <hip/hip_runtime.h>

#include "fv_dual.h"
#include "fv_kernels.h"

namespace fv {

namespace {

constexpr int ADJ_THREADS = 128;

using D = Dual<double>;

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

template <int DIR>
__global__ void __launch_bounds__(ADJ_THREADS) face_adjoint_kernel(const AdjointArgs a, const double* __restrict__ U,
                                                                   const double* __restrict__ Rbar,
                                                                   double* __restrict__ Ubar)
{
    constexpr int NC = 5, V = 1;
    const int n = DIR == 0 ? a.nx : (DIR == 1 ? a.ny : a.nz);
    const long long lines = a.ncell / n;
    const long long t = (long long)blockIdx.x * ADJ_THREADS + threadIdx.x;
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
    const Material<D> dmat = dual_material(mat);

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
        g[m] = v * a.ih;
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
    // HLLC: cotangents of the two face states, one tangent per input
    double wlb[NC], wrb[NC];
#pragma unroll 1
    for (int jdx = 0; jdx < 2 * NC; jdx++) {
        D dl[NC], dr[NC], F[NC], uh;
#pragma unroll
        for (int m = 0; m < NC; m++) {
            dl[m] = D(wl[m], jdx == m ? 1.0 : 0.0);
            dr[m] = D(wr[m], jdx == NC + m ? 1.0 : 0.0);
        }
        hllc<D, EULER, DIR>(dmat, dl, dr, F, uh);
        double sacc = 0.0;
#pragma unroll
        for (int m = 0; m < NC; m++) sacc += g[m] * F[m].d;
        if (jdx < NC) wlb[jdx] = sacc;
        else wrb[jdx - NC] = sacc;
    }
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
    for (int d = 0; d < 3; d++) {
        const int n = d == 0 ? a.nx : (d == 1 ? a.ny : a.nz);
        AdjointArgs ad = a;
        ad.ih = d == 0 ? a.idx : (d == 1 ? a.idy : a.idz);
        const long long faces = a.ncell / n * (n + 1);
        const dim3 grid((unsigned)((faces + ADJ_THREADS - 1) / ADJ_THREADS));
        switch (d) {
        case 0: hipLaunchKernelGGL(face_adjoint_kernel<0>, grid, dim3(ADJ_THREADS), 0, st, ad, U, Rbar, Ubar); break;
        case 1: hipLaunchKernelGGL(face_adjoint_kernel<1>, grid, dim3(ADJ_THREADS), 0, st, ad, U, Rbar, Ubar); break;
        default: hipLaunchKernelGGL(face_adjoint_kernel<2>, grid, dim3(ADJ_THREADS), 0, st, ad, U, Rbar, Ubar); break;
        }
    }
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
