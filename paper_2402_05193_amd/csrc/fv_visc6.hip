// fv_visc6.hip -- sixth-order central viscous fluxes for gfx950 (Sec. 2.1
// dissipative fluxes; the single-phase simulations of the paper use 6th-order
// central stencils for them).
//
// The fused stage kernel marches in z with the tangential derivatives of a z
// face one plane behind; sixth-order face interpolation would need them two
// planes ahead.  Instead the viscous part runs as three passes whose result
// the stage adds when it finalises a cell:
//   1. q = (u, v, w, theta = p/rho) on the box padded by 3 cells, boundary
//      conditions by index mapping (the normal velocity negated across
//      symmetry planes), one thread per padded cell;
//   2. the velocity gradient du_c/dx_e at cell centres,
//      (45 (q+1 - q-1) - 9 (q+2 - q-2) + (q+3 - q-3)) / (60 h), for every
//      padded cell whose e-coordinate is interior (the only ones read);
//   3. per interior cell and direction d, the fluxes of its two d-faces from
//      the six cells across each face: face values
//      (3 q-2 - 25 q-1 + 150 q0 + 150 q1 - 25 q2 + 3 q3) / 256, normal
//      derivatives (2250 (q1 - q0) - 125 (q2 - q-1) + 9 (q3 - q-2)) / (1920 h),
//      tangential derivatives interpolated from the gradients of pass 2; the
//      stress tensor with the viscosity of the face temperature, the heat flux
//      with the constant-Prandtl conductivity; then their divergence.
// Pass 2 runs once per axis on line tiles staged in LDS (16 lines of 32 cells
// plus the 3-cell halo), so that each value is read from memory about once per
// axis.  Pass 3 is two kernels marching along y (with the x faces) and along z,
// each with the marched axis' stencils in registers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fv_kernels.h"
#include "fv_physics.h"

namespace fv {
namespace {

template <typename Real>
__device__ __forceinline__ Real ifc6(const Real* q)
{
    return (Real(150) * (q[2] + q[3]) - Real(25) * (q[1] + q[4]) + Real(3) * (q[0] + q[5])) * Real(1.0 / 256.0);
}

template <typename Real>
__device__ __forceinline__ Real dface6(const Real* q, Real ih)
{
    return (Real(2250) * (q[3] - q[2]) - Real(125) * (q[4] - q[1]) + Real(9) * (q[5] - q[0])) *
           (ih * Real(1.0 / 1920.0));
}

template <typename Real>
__global__ void __launch_bounds__(256) visc6_q_kernel(const Visc6Args<Real> a, const Real* __restrict__ U,
                                                      Real* __restrict__ Q)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.npad) return;
    const int px = a.nx + 6, py = a.ny + 6;
    const int i = (int)(t % px) - 3;
    const long long r = t / px;
    const int j = (int)(r % py) - 3, k = (int)(r / py) - 3;
    bool fx = false, fy = false, fz = false;
    const int ii = map_index(i, a.nx, a.bc[0], a.bc[1], fx);
    const int jj = map_index(j, a.ny, a.bc[2], a.bc[3], fy);
    const int kk = map_index(k, a.nz, a.bc[4], a.bc[5], fz);
    const long long q = ((long long)kk * a.ny + jj) * a.nx + ii;
    Real u[5], w[5];
#pragma unroll
    for (int m = 0; m < 5; m++) u[m] = U[m * a.ncell + q];
    if (fx) u[1] = -u[1];
    if (fy) u[2] = -u[2];
    if (fz) u[3] = -u[3];
    cons_to_prim<Real, NS>(a.mat, u, w);
    Q[t] = w[1];
    Q[a.npad + t] = w[2];
    Q[2 * a.npad + t] = w[3];
    Q[3 * a.npad + t] = w[4] * rcp(w[0]);
}

// ---- line tiles: a workgroup stages LNS lines of SPAN cells along one axis in LDS
// (the LEN cells it works on and 3 on either side) and reads every stencil there.
// Lines run along AX; the line coordinate is y for AX = 0 and x otherwise, the
// third coordinate z for AX = 0, 1 and y for AX = 2.  Consecutive lanes take
// consecutive x: along the line for AX = 0, across the lines otherwise.
constexpr int LNS = 16, LEN = 32, SPAN = LEN + 6, NTT = 256;

template <int AX>
__device__ __forceinline__ void tile_cell(int ax, int line, int third, int& x, int& y, int& z)
{
    if constexpr (AX == 0) { x = ax; y = line; z = third; }
    else if constexpr (AX == 1) { x = line; y = ax; z = third; }
    else { x = line; y = third; z = ax; }
}

template <typename Real>
__device__ __forceinline__ long long padded_index(const Visc6Args<Real>& a, int x, int y, int z)
{
    return ((long long)(z + 3) * (a.ny + 6) + (y + 3)) * (a.nx + 6) + (x + 3);
}

// (line slot, position) of item `it` of a tile: x fastest across the lanes
template <int AX, int NP>
__device__ __forceinline__ void tile_item(int it, int& l, int& p)
{
    if constexpr (AX == 0) { p = it % NP; l = it / NP; }
    else { l = it % LNS; p = it / LNS; }
}

// du_c/dx_E (c = 0, 1, 2) at the padded cells whose E-coordinate is interior, over the
// whole padded range of the other two coordinates
template <typename Real, int E>
__global__ void __launch_bounds__(NTT) visc6_grad_kernel(const Visc6Args<Real> a, const Real* __restrict__ Q,
                                                         Real* __restrict__ G)
{
    __shared__ Real S[3][LNS][SPAN];
    const int n3[3] = {a.nx, a.ny, a.nz};
    const int nax = n3[E], nline = E == 0 ? a.ny : a.nx;  // lines over the padded range [-3, nline + 3)
    const int a0 = blockIdx.x * LEN, l0 = (int)blockIdx.y * LNS - 3, third = (int)blockIdx.z - 3;
    for (int it = threadIdx.x; it < 3 * LNS * SPAN; it += NTT) {
        const int c = it / (LNS * SPAN);
        int l, p;
        tile_item<E, SPAN>(it - c * LNS * SPAN, l, p);
        const int ax = a0 + p - 3, line = l0 + l;
        if (ax > nax + 2 || line >= nline + 3) continue;  // beyond the padded box
        int x, y, z;
        tile_cell<E>(ax, line, third, x, y, z);
        S[c][l][p] = Q[c * a.npad + padded_index(a, x, y, z)];
    }
    __syncthreads();
    const Real f = a.ih[E] * Real(1.0 / 60.0);
    for (int it = threadIdx.x; it < LNS * LEN; it += NTT) {
        int l, p;
        tile_item<E, LEN>(it, l, p);
        const int ax = a0 + p, line = l0 + l;
        if (ax >= nax || line >= nline + 3) continue;
        int x, y, z;
        tile_cell<E>(ax, line, third, x, y, z);
        const long long q = padded_index(a, x, y, z);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const Real* v = &S[c][l][p + 3];
            G[(3 * c + E) * a.npad + q] = (Real(45) * (v[1] - v[-1]) - Real(9) * (v[2] - v[-2]) + (v[3] - v[-3])) * f;
        }
    }
}

// viscous flux (tau_x, tau_y, tau_z, u . tau + kappa dtheta/dn) of a d-face from its
// face values vf, normal derivatives dn (u, v, w, theta), face temperature thf and the
// interpolated tangential derivatives t_de1, t_de2 (d u_D / d x_E), t_e1, t_e2 (d u_E / d x_E)
template <typename Real, int D, int LAW>
__device__ __forceinline__ void face6(const Visc6Args<Real>& a, const Real* vf, const Real* dn, Real thf,
                                      Real t_de1, Real t_de2, Real t_e1, Real t_e2, Real* F)
{
    constexpr int E1 = (D + 1) % 3, E2 = (D + 2) % 3;
    const Real div = dn[D] + t_e1 + t_e2;
    // constant viscosity without the law's code (the power law's pow, inlined at six
    // faces, would take the registers of the whole kernel)
    Real mu;
    if constexpr (LAW == 0) mu = a.vl.mu;
    else mu = visc_mu(a.vl, thf);
    const Real kap = mu * a.vl.kfac;
    Real tau[3];
    tau[D] = mu * (Real(2) * dn[D] - Real(2.0 / 3.0) * div);
    tau[E1] = mu * (t_de1 + dn[E1]);
    tau[E2] = mu * (t_de2 + dn[E2]);
    F[0] = tau[0];
    F[1] = tau[1];
    F[2] = tau[2];
    F[3] = vf[0] * tau[0] + vf[1] * tau[1] + vf[2] * tau[2] + kap * dn[3];
}

// both d-faces of the cell at padded index tp (axis stride s): the seven cells along
// the axis are read one field at a time and reduced to the two faces' values at once,
// so that only one field's stencil is live
template <typename Real, int D, int LAW>
__device__ __forceinline__ void direction6(const Visc6Args<Real>& a, const Real* __restrict__ Q,
                                           const Real* __restrict__ G, long long tp, long long s, Real* acc)
{
    constexpr int E1 = (D + 1) % 3, E2 = (D + 2) % 3;
    Real vf[2][3], dn[2][4], th[2], t[4][2];
    auto load7 = [&](const Real* base, Real* v) {
#pragma unroll
        for (int o = 0; o < 7; o++) v[o] = base[tp + (o - 3) * s];
    };
#pragma unroll
    for (int c = 0; c < 4; c++) {
        Real v[7];
        load7(Q + c * a.npad, v);
#pragma unroll
        for (int b = 0; b < 2; b++) {
            dn[b][c] = dface6(v + b, a.ih[D]);
            if (c < 3) vf[b][c] = ifc6(v + b);
            else th[b] = ifc6(v + b);
        }
        __builtin_amdgcn_sched_barrier(0);  // one field's stencil live at a time
    }
    const int gi[4] = {3 * D + E1, 3 * D + E2, 3 * E1 + E1, 3 * E2 + E2};
#pragma unroll
    for (int g = 0; g < 4; g++) {
        Real v[7];
        load7(G + gi[g] * a.npad, v);
#pragma unroll
        for (int b = 0; b < 2; b++) t[g][b] = ifc6(v + b);
        __builtin_amdgcn_sched_barrier(0);
    }
    Real Fl[4], Fu[4];
    face6<Real, D, LAW>(a, vf[0], dn[0], th[0], t[0][0], t[1][0], t[2][0], t[3][0], Fl);  // face between cells -1, 0
    face6<Real, D, LAW>(a, vf[1], dn[1], th[1], t[0][1], t[1][1], t[2][1], t[3][1], Fu);  // face between cells 0, +1
#pragma unroll
    for (int c = 0; c < 4; c++) acc[c] += (Fu[c] - Fl[c]) * a.ih[D];
}

// ---- the flux pass in two kernels, each marching along one axis with that axis'
// stencils in registers: one thread per line, the six cells k-2 .. k+3 of q and of the
// four gradient fields of the faces normal to the axis in a window (the next cell loads
// one step ahead), one face per step, the lower one carried.  The first kernel marches
// along y (lanes along x) and also takes the x faces, whose stencils it reads directly
// (neighbouring lanes share them through the vector cache); it writes (0 + x part) +
// y part.  The second marches along z and adds the z part in place.  The sums are
// formed in the order x, y, z.
constexpr int MCH = 32;  // cells per marched chunk

// the face normal to D between window cells 2 and 3 from cells 0 .. 5 (q: 0 .. 3; the
// gradient fields du_D/dx_E1, du_D/dx_E2, du_E1/dx_E1, du_E2/dx_E2: 4 .. 7), the same
// arithmetic as the upper face of direction6
template <typename Real, int D, int LAW>
__device__ __forceinline__ void window_face6(const Visc6Args<Real>& a, const Real (*w)[8], Real* F)
{
    Real vf[3], dn[4], th, t[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        Real v[6];
#pragma unroll
        for (int o = 0; o < 6; o++) v[o] = w[o][c];
        dn[c] = dface6(v, a.ih[D]);
        if (c < 3) vf[c] = ifc6(v);
        else th = ifc6(v);
    }
#pragma unroll
    for (int f = 0; f < 4; f++) {
        Real v[6];
#pragma unroll
        for (int o = 0; o < 6; o++) v[o] = w[o][4 + f];
        t[f] = ifc6(v);
    }
    face6<Real, D, LAW>(a, vf, dn, th, t[0], t[1], t[2], t[3], F);
}

// march along D (1: y, lanes along x, lines over (x, z); 2: z, lanes along x, lines over
// (x, y)) through chunk blockIdx.y of MCH cells
template <typename Real, int D, int LAW>
__global__ void __launch_bounds__(256) visc6_flux_march_kernel(const Visc6Args<Real> a, const Real* __restrict__ Q,
                                                               const Real* __restrict__ G, Real* __restrict__ Rv)
{
    static_assert(D == 1 || D == 2, "march along y or z");
    constexpr int E1 = (D + 1) % 3, E2 = (D + 2) % 3;
    constexpr int GF[4] = {3 * D + E1, 3 * D + E2, 3 * E1 + E1, 3 * E2 + E2};
    const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nd = D == 1 ? a.ny : a.nz, no = D == 1 ? a.nz : a.ny;  // marched axis, other axis
    if (line >= (long long)a.nx * no) return;
    const int i = (int)(line % a.nx), o = (int)(line / a.nx);
    const int c0 = (int)blockIdx.y * MCH, c1 = min(c0 + MCH, nd);
    const int px = a.nx + 6, py = a.ny + 6;
    // padded index of the cell at position d along the marched axis
    const long long sd = D == 1 ? (long long)px : (long long)px * py;
    const long long base = D == 1 ? ((long long)(o + 3) * py + 3) * px + (i + 3) : (long long)(o + 3) * px + 3 * sd + (i + 3);
    auto load = [&](int d, Real* v) {
        const long long p = base + (long long)d * sd;
#pragma unroll
        for (int c = 0; c < 4; c++) v[c] = Q[c * a.npad + p];
#pragma unroll
        for (int f = 0; f < 4; f++) v[4 + f] = G[GF[f] * a.npad + p];
    };
    Real w[6][8], nxt[8];
#pragma unroll
    for (int p = 0; p < 6; p++) load(c0 - 3 + p, w[p]);  // cells c0-3 .. c0+2
    Real Fl[4];
    window_face6<Real, D, LAW>(a, w, Fl);                 // the face below c0
    load(c0 + 3, nxt);
    for (int d = c0; d < c1; d++) {
#pragma unroll
        for (int p = 0; p < 5; p++)
#pragma unroll
            for (int f = 0; f < 8; f++) w[p][f] = w[p + 1][f];
#pragma unroll
        for (int f = 0; f < 8; f++) w[5][f] = nxt[f];
        if (d + 1 < c1) load(d + 4, nxt);  // up to c1+2, inside the padded box
        const int j = D == 1 ? d : o, k = D == 1 ? o : d;
        const long long t = ((long long)k * a.ny + j) * a.nx + i;
        Real acc[4];
        if constexpr (D == 1) {
            acc[0] = acc[1] = acc[2] = acc[3] = Real(0);
            direction6<Real, 0, LAW>(a, Q, G, base + (long long)d * sd, 1, acc);
        } else {
#pragma unroll
            for (int c = 0; c < 4; c++) acc[c] = Rv[c * a.ncell + t];
        }
        Real Fu[4];
        window_face6<Real, D, LAW>(a, w, Fu);
#pragma unroll
        for (int c = 0; c < 4; c++) {
            Rv[c * a.ncell + t] = acc[c] + (Fu[c] - Fl[c]) * a.ih[D];
            Fl[c] = Fu[c];
        }
    }
}

}  // namespace

template <typename Real>
hipError_t launch_visc6(const Visc6Args<Real>& a, const Real* U, Real* Q, Real* G, Real* Rv, hipStream_t st)
{
    const long long bp = (a.npad + NTT - 1) / NTT;
    hipLaunchKernelGGL(visc6_q_kernel<Real>, dim3((unsigned)bp), dim3(NTT), 0, st, a, U, Q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // gradients along x (lines along x over the padded y, z range), along y and z (lines
    // along those axes, across the padded x range)
    hipLaunchKernelGGL((visc6_grad_kernel<Real, 0>), dim3((a.nx + LEN - 1) / LEN, (a.ny + 6 + LNS - 1) / LNS, a.nz + 6),
                       dim3(NTT), 0, st, a, (const Real*)Q, G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((visc6_grad_kernel<Real, 1>), dim3((a.ny + LEN - 1) / LEN, (a.nx + 6 + LNS - 1) / LNS, a.nz + 6),
                       dim3(NTT), 0, st, a, (const Real*)Q, G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((visc6_grad_kernel<Real, 2>), dim3((a.nz + LEN - 1) / LEN, (a.nx + 6 + LNS - 1) / LNS, a.ny + 6),
                       dim3(NTT), 0, st, a, (const Real*)Q, G);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // fluxes: the march along y with the x faces, then the march along z
    const unsigned by = (unsigned)(((long long)a.nx * a.nz + NTT - 1) / NTT);
    const unsigned bz = (unsigned)(((long long)a.nx * a.ny + NTT - 1) / NTT);
    const unsigned cy = (unsigned)((a.ny + MCH - 1) / MCH), cz = (unsigned)((a.nz + MCH - 1) / MCH);
    if (a.vl.law == 0) {
        hipLaunchKernelGGL((visc6_flux_march_kernel<Real, 1, 0>), dim3(by, cy), dim3(NTT), 0, st, a, (const Real*)Q,
                           (const Real*)G, Rv);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((visc6_flux_march_kernel<Real, 2, 0>), dim3(bz, cz), dim3(NTT), 0, st, a, (const Real*)Q,
                           (const Real*)G, Rv);
    } else {
        hipLaunchKernelGGL((visc6_flux_march_kernel<Real, 1, 1>), dim3(by, cy), dim3(NTT), 0, st, a, (const Real*)Q,
                           (const Real*)G, Rv);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((visc6_flux_march_kernel<Real, 2, 1>), dim3(bz, cz), dim3(NTT), 0, st, a, (const Real*)Q,
                           (const Real*)G, Rv);
    }
    return hipGetLastError();
}

template hipError_t launch_visc6<double>(const Visc6Args<double>&, const double*, double*, double*, double*,
                                         hipStream_t);
template hipError_t launch_visc6<float>(const Visc6Args<float>&, const float*, float*, float*, float*, hipStream_t);

}  // namespace fv
