// fv_adjoint.hip -- discrete adjoint of the single-phase Euler right-hand side
// (vector-Jacobian product of Eq. (FVD) with WENO5-Z and HLLC, Sec. 3.2) and
// of the TVD-RK3 step at a fixed time step (Sec. 3.4), the reverse sweep that
// the paper obtains by automatic differentiation (Sec. 6).
//
// One thread per face: it rebuilds the face's six-cell stencil (boundary
// conditions by index mapping, as the stage kernel reads them), the two WENO
// face states and the HLLC flux, then pulls the face cotangent
//   Fbar_f = (Rbar_f - Rbar_{f-1}) / h        (R_i = -(F_{i+1/2} - F_{i-1/2}) / h)
// back through HLLC, WENO5-Z and the U -> W map with forward-mode tangents of
// the same device functions (fv_dual.h), and adds the six cells' cotangents to
// Ubar with atomic adds.  The order of the atomic additions is not fixed, so
// the result is reproducible to round-off, not bitwise.
#include <hip/hip_runtime.h>

#include "fv_dual.h"
#include "fv_kernels.h"

namespace fv {

namespace {

constexpr int ADJ_THREADS = 128;

using D = Dual<double>;

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
    const int f = (int)(t % (n + 1));  // face f lies between cells f-1 and f of the line
    const long long line = t / (n + 1);
    int ci, cj, ck;  // coordinates of the line's cells; the DIR one is set per cell below
    if (DIR == 0) {
        ci = 0;
        cj = (int)(line % a.ny);
        ck = (int)(line / a.ny);
    } else if (DIR == 1) {
        ci = (int)(line % a.nx);
        cj = 0;
        ck = (int)(line / a.nx);
    } else {
        ci = (int)(line % a.nx);
        cj = (int)(line / a.nx);
        ck = 0;
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
    // face states: left = v^- of cell f-1 (stencil slots 0..4), right = v^+ of cell f (slots 1..5)
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
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < NC; m++) s += g[m] * F[m].d;
        if (jdx < NC) wlb[jdx] = s;
        else wrb[jdx - NC] = s;
    }
    // WENO5-Z: cotangents of the stencil's primitive states
    double wb[6][NC];
#pragma unroll
    for (int s = 0; s < 6; s++)
#pragma unroll
        for (int m = 0; m < NC; m++) wb[s][m] = 0.0;
#pragma unroll
    for (int m = 0; m < NC; m++) {
#pragma unroll 1
        for (int k = 0; k < 5; k++) {
            D st[6];
#pragma unroll
            for (int s = 0; s < 6; s++) st[s] = D(w[s][m], 0.0);
            D vm, vp, y0, y1;
            // tangent at slot k of the left stencil and at slot k+1 of the right one
            st[k].d = 1.0;
            weno5z_pair(st[0], st[1], st[2], st[3], st[4], D(a.weps), vm, y0);
            st[k].d = 0.0;
            st[k + 1].d = 1.0;
            weno5z_pair(st[1], st[2], st[3], st[4], st[5], D(a.weps), y1, vp);
            wb[k][m] += wlb[m] * vm.d;
            wb[k + 1][m] += wrb[m] * vp.d;
        }
    }
    // U -> W: cotangents of the conservative states, then the boundary mapping
#pragma unroll
    for (int s = 0; s < 6; s++) {
        double u[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) u[m] = U[m * a.ncell + q[s]];
        if (flip[s]) u[V + DIR] = -u[V + DIR];
        double ub[NC];
#pragma unroll 1
        for (int jdx = 0; jdx < NC; jdx++) {
            D du[NC], dw[NC];
#pragma unroll
            for (int m = 0; m < NC; m++) du[m] = D(u[m], jdx == m ? 1.0 : 0.0);
            cons_to_prim<D, EULER>(dmat, du, dw);
            double sacc = 0.0;
#pragma unroll
            for (int m = 0; m < NC; m++) sacc += wb[s][m] * dw[m].d;
            ub[jdx] = sacc;
        }
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
