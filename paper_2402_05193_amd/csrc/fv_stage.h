// fv_stage.h -- the fused finite-volume RHS / TVD-RK3 stage kernel for gfx950.
// Instantiated per precision and model by fv_stage_inst.hip (the kernels of a
// variant family) and fv_stage_launch.hip (dispatch and the batched kernels),
// so that the instantiations compile in parallel.
//
// One kernel evaluates R_NSE (arXiv:2402.05193 Eq. (FVD), plus the volume
// fraction source of Sec. 3.7) for a block of cells and applies one Shu-Osher
// stage (Sec. 3.4) -- or writes R itself.  Face states and fluxes never
// leave the chip.
//
// Work decomposition ("2.5-D z-march"):
//  * a workgroup owns a BX x BY column tile and a chunk of z-planes and marches
//    through them plane by plane;
//  * each thread owns one (x, y) column and keeps a 6-plane register window of
//    primitive states W(s-3..s+2) of that column: the z-direction
//    reconstruction, Riemann solve and viscous flux run entirely in registers;
//  * the current plane s, with a 3-cell ring of x/y halo cells mapped through
//    the boundary conditions, is staged in LDS as primitives; x- and y-face
//    work runs as flat task lists over LDS (cell reconstructions write both
//    face states of a cell, sharing the smoothness indicators; face tasks
//    solve the Riemann problem in place);
//  * z-faces complete one plane behind, so cell s-2 is finalised at step s
//    (combined with U^n and written once, coalesced, x fastest).
#pragma once

#include <hip/hip_runtime.h>

#include "fv_kernels.h"
#include "fv_physics.h"

namespace fv {

template <typename Real>
__device__ __forceinline__ void load_cell(const StageArgs<Real>& a, const Real* __restrict__ U, int gi, int gj,
                                          int gk, Real* u, int nc, int V, bool interior_xy)
{
    bool fx = false, fy = false, fz = false;
    int i = gi, j = gj;
    if (!interior_xy) {
        i = map_index(gi, a.nx, a.bc[0], a.bc[1], fx);
        j = map_index(gj, a.ny, a.bc[2], a.bc[3], fy);
    }
    const int k = map_index(gk, a.nz, a.bc[4], a.bc[5], fz);
    const long long q = ((long long)k * a.ny + j) * a.nx + i;
    for (int m = 0; m < nc; m++) u[m] = U[m * a.ncell + q];
    if (fx) u[V] = -u[V];
    if (fy) u[V + 1] = -u[V + 1];
    if (fz) u[V + 2] = -u[V + 2];
}

// The same load without the reflections: returns which velocity components to
// negate (bit 0: x, 1: y, 2: z), so that the caller can apply them after its other
// loads are issued (a negation right after a load waits for that load)
template <typename Real>
__device__ __forceinline__ int load_cell_raw(const StageArgs<Real>& a, const Real* __restrict__ U, int gi, int gj,
                                             int gk, Real* u, int nc, bool interior_xy)
{
    bool fx = false, fy = false, fz = false;
    int i = gi, j = gj;
    if (!interior_xy) {
        i = map_index(gi, a.nx, a.bc[0], a.bc[1], fx);
        j = map_index(gj, a.ny, a.bc[2], a.bc[3], fy);
    }
    const int k = map_index(gk, a.nz, a.bc[4], a.bc[5], fz);
    const long long q = ((long long)k * a.ny + j) * a.nx + i;
    for (int m = 0; m < nc; m++) u[m] = U[m * a.ncell + q];
    return (fx ? 1 : 0) | (fy ? 2 : 0) | (fz ? 4 : 0);
}

template <typename Real>
__device__ __forceinline__ void apply_reflections(Real* u, int V, int mask)
{
    if (mask & 1) u[V] = -u[V];
    if (mask & 2) u[V + 1] = -u[V + 1];
    if (mask & 4) u[V + 2] = -u[V + 2];
}

// Write R (mode 0) or the Shu-Osher stage combination of cell q (modes 1..3)
// from the preloaded U^(k) (uk) and U^n (un) of the cell; the written values
// are returned in `out` for the optional CFL reduction.
template <typename Real, int NC>
__device__ __forceinline__ void store_cell_impl(const StageArgs<Real>& a, long long q, const Real* r, Real dt,
                                                const Real* uk, const Real* un, Real* out)
{
    if (a.mode == 0) {
#pragma unroll
        for (int m = 0; m < NC; m++) out[m] = r[m];
    } else if (a.mode == 1) {
#pragma unroll
        for (int m = 0; m < NC; m++) out[m] = uk[m] + dt * r[m];
    } else if (a.mode == 2) {
        const Real c1 = Real(0.75), c2 = Real(0.25);
#pragma unroll
        for (int m = 0; m < NC; m++) out[m] = c1 * un[m] + c2 * uk[m] + (c2 * dt) * r[m];
    } else {
        const Real c1 = Real(1.0 / 3.0), c2 = Real(2.0 / 3.0);
#pragma unroll
        for (int m = 0; m < NC; m++) out[m] = c1 * un[m] + c2 * uk[m] + (c2 * dt) * r[m];
    }
#pragma unroll
    for (int m = 0; m < NC; m++) a.out[m * a.ncell + q] = out[m];
}

// Inverse CFL time step of a conservative state: max(max_d (|u_d| + c)/dx_d, kvisc/rho).
template <typename Real, int MODEL, bool VLAW>
__device__ __forceinline__ double inverse_dt(const StageArgs<Real>& a, const Real* u)
{
    constexpr int NC = Layout<MODEL>::NC, V = Layout<MODEL>::V;
    Real w[NC];
    cons_to_prim<Real, MODEL>(a.mat, u, w);
    const Real ir = rcp(density<Real, MODEL>(w));
    const Real c = sqrt_fast(rhoc2<Real, MODEL>(a.mat, w) * ir);
    Real v = fmax((fabs(w[V]) + c) * a.idx, fmax((fabs(w[V + 1]) + c) * a.idy, (fabs(w[V + 2]) + c) * a.idz));
    if constexpr (MODEL == NS) {
        Real kv = Real(a.kvisc);
        if constexpr (VLAW) kv = visc_mu(a.vl, w[Layout<MODEL>::P] * ir) * Real(a.kvisc_h);
        v = fmax(v, kv * ir);
    }
    const double d = (double)v;
    return d >= 0.0 ? d : __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf
}

// LDS geometry of one tile of BX x BY cells worked on by NTH threads
// (NTH >= BX * BY; the x/y task lists are sized to fit NTH in one round)
template <typename Real, int MODEL, int BX, int BY, int NTH, bool VISC_ = (MODEL == NS), bool THINC_ = false>
struct Tile {
    static constexpr int NC = Layout<MODEL>::NC;
    static constexpr bool VISC = VISC_;  // the stage computes viscous fluxes itself
    static constexpr bool THINC = THINC_;  // interface capturing (five-equation model)
    static constexpr int NT = NTH;
    static constexpr int NCELL = BX * BY;
    // primitives of the LDS plane, plus T = p/rho (viscous) or the smoothed volume
    // fraction psi of the interface normal (THINC)
    static constexpr int NW = NC + ((VISC || THINC) ? 1 : 0);
    static constexpr int PX = BX + 6, PY = BY + 6;  // plane with 3-cell halo
    static constexpr int NFX = (BX + 1) * BY, NFY = BX * (BY + 1);
    static constexpr int NFMAX = NFX > NFY ? NFX : NFY;
    static constexpr int WP_SIZE = NW * PY * PX;
    static constexpr int FB_SIZE = 2 * NC * NFMAX;       // face states (left, right), fluxes in place
    static constexpr int UH_SIZE = MODEL == DIM ? NFMAX : 0;
    static constexpr int RX = (BX + 4) * BY, RY = BX * (BY + 4);  // viscous cell regions
    static constexpr int DZ_SIZE = VISC ? 2 * RX + 2 * RY : 0;    // d/dz of (u,w) on RX, (v,w) on RY
    static constexpr int DT_SIZE = VISC ? 2 * (RX > RY ? RX : RY) : 0;  // in-plane tangential d/dx_t
    // halo ring of the plane; corners: 2 deep for the viscous cross terms, 1 deep
    // for the volume-fraction gradient of THINC
    static constexpr int NHALO = 6 * BY + 6 * BX + (VISC ? 16 : (THINC ? 4 : 0));
    // THINC: d(psi)/dz at the plane for the tile and its 1-cell ring
    static constexpr int AZ_SIZE = THINC ? (BX + 2) * (BY + 2) : 0;
    static constexpr int NRING = 2 * BX + 2 * BY + 4;
    // THINC in FP32: psi of each 1-cell ring cell at two consecutive planes (slot =
    // plane & 1), carried by the thread that owns the ring cell
    static constexpr bool PSI_CARRY = THINC && sizeof(Real) == 4;
    static constexpr int PSQ_SIZE = PSI_CARRY ? 2 * NRING : 0;
    // per-thread x/y partial sums of R for planes s-2 / s-1 (two slots); the
    // five-equation model (LDS budget) keeps even planes in one LDS slot and odd planes
    // in registers
    static constexpr bool ACC_LDS = MODEL != DIM;
    static constexpr bool ACC_HALF = MODEL == DIM;
    static constexpr int ACC_SIZE = ACC_LDS ? 2 * NC * NCELL : (ACC_HALF ? NC * NCELL : 0);
    static constexpr size_t bytes()
    {
        return sizeof(Real) * (size_t)(WP_SIZE + FB_SIZE + UH_SIZE + DZ_SIZE + DT_SIZE + ACC_SIZE + AZ_SIZE + PSQ_SIZE);
    }
};

// One workgroup of the fused stage: tile column `bid` of the problem described by `a`.
template <typename Real, int MODEL, int POS, int REC, int VMODE, int BX, int BY, int NTH>
__device__ __forceinline__ void stage_body(const StageArgs<Real>& a, const int bid, unsigned char* smem_raw)
{
    using L = Layout<MODEL>;
    constexpr bool THINC = MODEL == DIM && VMODE == XM_THINC;
    using TL = Tile<Real, MODEL, BX, BY, NTH, MODEL == NS && VMODE != VM_EXT && VMODE != VM_EXT_LAW, THINC>;
    constexpr bool VLAW = MODEL == NS && VMODE == VM_LAW;
    constexpr int NC = L::NC, V = L::V, P = L::P;
    constexpr bool VISC = TL::VISC;
    constexpr bool ACC_LDS = TL::ACC_LDS;
    constexpr bool ACC_HALF = TL::ACC_HALF;
    constexpr int PX = TL::PX, PY = TL::PY;
    constexpr int NT = NTH;
    constexpr int NCELL = BX * BY;
    constexpr int PLANE = PY * PX;
    static_assert(NT >= NCELL && NT % 64 == 0, "threads must cover the tile");
    // POS: 0 limiters off, 1 on, 2 on and every face's decisions written to a.flags
    // (bit 0: interpolation limiter on the left state, bit 1: on the right state,
    // bit 2: flux limiter), per direction [d][k][j][i] with the face index fastest
    // along d (the x block (nx+1) ny nz bytes, then y, then z)
    constexpr bool REC_FLAGS = POS == 2;

    Real* Wp = reinterpret_cast<Real*>(smem_raw);
    Real* FB = Wp + TL::WP_SIZE;
    Real* UHB = FB + TL::FB_SIZE;
    Real* DZX = UHB + TL::UH_SIZE;  // [2][BY][BX+4]   (u, w) d/dz, x-face region
    Real* DZY = DZX + 2 * TL::RX;   // [2][BY+4][BX]   (v, w) d/dz, y-face region
    Real* DT = DZX + TL::DZ_SIZE;   // [2][region]     in-plane tangential derivatives
    Real* ACC = DT + TL::DT_SIZE;   // [2][NC][NCELL]  x/y partial sums of R
    Real* AZ = ACC + TL::ACC_SIZE;  // [BY+2][BX+2]    THINC: d(psi)/dz, tile and 1-cell ring
    Real* PSQ = AZ + TL::AZ_SIZE;   // [2][NRING]      THINC FP32: psi of the ring cells, two planes

    const Material<Real> mat = a.mat;
    const Tolerances<Real> tol = a.tol;
    const Real weps = a.weno_eps;
    const Real dt = a.dt_dev ? Real(*a.dt_dev) : Real(a.dt);

    const int tid = threadIdx.x;
    const bool has_cell = tid < NCELL;  // threads beyond the tile only take x/y tasks
    const int tx = tid % BX, ty = has_cell ? tid / BX : 0;
    // task lists have a few tasks more than threads; the wave that takes the
    // remainder rotates with the workgroup so co-resident groups spread it over SIMDs
    const int rt = (tid + 64 * (bid & 3)) % NT;
    int b = bid;
    // blocks of one tile column are consecutive; consecutive tiles share an XCD's L2
    const int chunk = b % a.nchunks;
    b /= a.nchunks;
    const int tileX = b % a.tiles_x;
    const int tileY = b / a.tiles_x;
    const int x0 = tileX * BX, y0 = tileY * BY;
    const int z0 = chunk * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own_valid = has_cell && gx < a.nx && gy < a.ny;
    // the tile and its 3-cell x/y halo lie inside the domain: no boundary mapping in x, y
    const bool interior_xy = x0 >= 3 && x0 + BX + 3 <= a.nx && y0 >= 3 && y0 + BY + 3 <= a.ny;

    auto wp = [&](int f, int i, int j) -> Real& { return Wp[f * PLANE + (j + 3) * PX + (i + 3)]; };

    // primitive state of an arbitrary (possibly outside) cell
    auto load_w = [&](int gi, int gj, int gk, Real* w) {
        Real u[NC];
        load_cell<Real>(a, a.Uk, gi, gj, gk, u, NC, V, interior_xy);
        cons_to_prim<Real, MODEL>(mat, u, w);
    };
    auto stage_w = [&](int i, int j, const Real* w, Real psi, bool with_psi = true) {
#pragma unroll
        for (int f = 0; f < NC; f++) wp(f, i, j) = w[f];
        if constexpr (VISC) wp(NC, i, j) = w[P] * rcp(w[0]);  // T = p / rho
        if constexpr (THINC) {
            if (with_psi) wp(NC, i, j) = psi;
        }
    };

    // reconstruction variant: WENO5-Z of primitive variables per cell (both faces of a
    // cell share the smoothness indicators), or per face (characteristic variables,
    // TENO6-A): then a z face reads six planes and the window holds seven
    constexpr bool FACE = REC != REC_WENO_PRIM;
    constexpr bool CHARV = REC == REC_WENO_CHAR || REC == REC_TENO_CHAR;
    constexpr bool TENO = REC == REC_TENO_PRIM || REC == REC_TENO_CHAR;
    // register window W(s-3 .. s+2) of the own column
    constexpr int NWIN = FACE ? 7 : 6, WO = FACE ? 1 : 0;  // face tasks need s-4 .. s+2
    Real win[NWIN][NC];
    // THINC: psi of the window's volume fractions (thinc_psi), computed once per plane
    Real psw[THINC ? NWIN : 1];
    // viscous: two warm-up planes for the in-plane derivatives of the first z faces;
    // THINC: one, for the in-plane volume-fraction gradient of cell z0-1
    const int s_begin = VISC ? z0 - 2 : (THINC ? z0 - 1 : z0);
#pragma unroll
    for (int q = 0; q < NWIN - 1; q++) {
        if (has_cell) load_w(gx, gy, s_begin - 3 - WO + q, win[q]);
        else
#pragma unroll
            for (int f = 0; f < NC; f++) win[q][f] = Real(1);
        if constexpr (THINC) psw[q] = thinc_psi(win[q][6]);
    }

    Real vminus[NC];          // v^-_{s-3/2} from the reconstruction of cell s-2
    Real accA[NC], accB[NC];  // x/y part of R of cells s-2, s-1 (registers; ACC_HALF: accA the odd planes')
    Real srcA = 0, srcB = 0;  // DIM: x/y part of sum_d (uh_r - uh_l)/dx_d of cells s-2 and s-1
    Real Fzl[NC];             // flux at the lower z face of cell s-2 (face s-5/2)
    Real uhzl = 0;            // its upwinded normal velocity (DIM)
    Real Dc[3][4];            // NS: (dw/dx, du/dx, dw/dy, dv/dy) at planes s-3, s-2, s-1
    Real Ag[2][2] = {{0, 0}, {0, 0}};  // THINC: (d psi/dx, d psi/dy) of the own column at planes s-2, s-1
#pragma unroll
    for (int m = 0; m < NC; m++) {
        vminus[m] = 0;
        accA[m] = 0;
        accB[m] = 0;
        Fzl[m] = 0;
    }
#pragma unroll
    for (int q = 0; q < 3; q++)
#pragma unroll
        for (int c = 0; c < 4; c++) Dc[q][c] = 0;

    double tmax = 0.0;  // CFL reduction over the finalised cells (stage 3)
    const Real idx = a.idx, idy = a.idy, idz = a.idz;
    const Real lamx = Real(2 * a.ndim) * dt * idx;
    const Real lamy = Real(2 * a.ndim) * dt * idy;
    const Real lamz = Real(2 * a.ndim) * dt * idz;

    // THINC: the 1-cell ring cell of one of the highest-numbered threads, for d(psi)/dz
    // of the ring.  FP32 (PSI_CARRY): these threads also stage the ring's psi in the
    // plane, and psi of the cell at planes s-1 and s is carried in PSQ from the two
    // previous steps, so each step evaluates it once (0.67 -> 0.56 ms per stage for the
    // five-equation THINC stage at 256x128x128, with the cheaper psi of FP32); halo
    // threads evaluate psi only where it is read.  FP64 evaluates psi of the ring at s-1
    // and s+1 in every step and of every halo cell: the carry, or only the skipped halo
    // cells and the ring's coordinates set once, measured 1.45 against 1.42 ms there.
    constexpr bool PSI_CARRY = TL::PSI_CARRY;
    const int rh = NT - 1 - tid;
    const bool carry_ring = PSI_CARRY && rh < TL::NRING;
    int cr_i = 0, cr_j = 0;     // the ring cell (tile coordinates) and its column
    long long cr_col = 0;
    auto ring_alpha = [&](int k) {
        bool fz = false;
        const int kk = map_index(k, a.nz, a.bc[4], a.bc[5], fz);
        return a.Uk[6 * a.ncell + (long long)kk * a.ny * a.nx + cr_col];
    };
    if (carry_ring) {
        if (rh < 2 * BY) {
            cr_j = rh >> 1;
            cr_i = (rh & 1) ? BX : -1;
        } else if (rh < 2 * BY + 2 * BX) {
            const int hh = rh - 2 * BY;
            cr_i = hh >> 1;
            cr_j = (hh & 1) ? BY : -1;
        } else {
            const int hh = rh - 2 * BY - 2 * BX;
            cr_i = (hh & 1) ? BX : -1;
            cr_j = (hh & 2) ? BY : -1;
        }
        bool fx = false, fy = false;
        const int ii = map_index(x0 + cr_i, a.nx, a.bc[0], a.bc[1], fx);
        const int jj = map_index(y0 + cr_j, a.ny, a.bc[2], a.bc[3], fy);
        cr_col = (long long)jj * a.nx + ii;
        PSQ[((s_begin - 1) & 1) * TL::NRING + rh] = thinc_psi(ring_alpha(s_begin - 1));
        PSQ[(s_begin & 1) * TL::NRING + rh] = thinc_psi(ring_alpha(s_begin));
    }

    for (int s = s_begin; s <= z1 + 1; s++) {
        // own column, plane s+2.  Without viscous fluxes it is not read before the next
        // step: the five-equation and Euler kernels load it after the z work and convert it
        // at the end of the step (OWN_AFTER_Z), so that neither the loaded nor the converted
        // values are live during the z faces and the load's latency is covered by the x/y
        // phases (five-equation FP64: VGPR spills 106 -> 93, and its loads no longer wait at
        // the end of the previous step to be spilled: 0.914 -> 0.888 ms per stage at
        // 256x128x128, THINC 1.357 -> 1.316, FP32 1-2 % faster; Euler 256^3 1.673 -> 1.649
        // ms, FP32 0.953 -> 0.934, characteristic 2.274 -> 2.246).  The five-equation FP64
        // TENO6-A and characteristic kernels and the Euler TENO6-A kernels measured 0.2-2 %
        // slower so and keep an early load.  An early load is issued after the step's other
        // loads for the remaining FP64 single-phase kernels (LATE_OWN: its conversion waits
        // for it and would hold them back), else at the start of the step (measured faster
        // so); either way it is converted once those loads are issued.
        constexpr bool OWN_AFTER_Z =
            (MODEL == DIM && (sizeof(Real) == 4 || REC == REC_WENO_PRIM)) || (MODEL == EULER && !TENO);
        constexpr bool LATE_OWN = MODEL != DIM && sizeof(Real) == 8 && !OWN_AFTER_Z;
        Real raw[NC];
        int rrefl = 0;
        auto load_own = [&]() {
            if (has_cell) rrefl = load_cell_raw<Real>(a, a.Uk, gx, gy, s + 2, raw, NC, interior_xy);
            else
#pragma unroll
                for (int f = 0; f < NC; f++) raw[f] = Real(1);
        };
        auto convert_own = [&]() {
            if constexpr (LATE_OWN) load_own();
            apply_reflections(raw, V, rrefl);
            cons_to_prim<Real, MODEL>(mat, raw, win[NWIN - 1]);
            if constexpr (THINC) psw[NWIN - 1] = thinc_psi(win[NWIN - 1][6]);
        };
        if constexpr (!LATE_OWN && !OWN_AFTER_Z) load_own();
        const bool xy = (s >= z0) && (s < z1);
        // THINC also stages plane z1 (the cell above the last z face of the chunk)
        const bool need_plane = xy || (VISC && s >= z0 - 2) || (THINC && s >= z0 - 1 && s <= z1);
        Real accC[NC];
        Real srcC = 0;
        Real Dnew[4] = {0, 0, 0, 0};
        Real Anew[2] = {0, 0};
#pragma unroll
        for (int m = 0; m < NC; m++) accC[m] = 0;

        // U^(k), U^n of the cell finalised in this step (s-2)
        Real pre_k[NC], pre_n[NC];


        if (need_plane) {
            // halo cell of this thread (at most one: NHALO <= NT), loaded before the barrier
            static_assert(TL::NHALO <= NT, "one halo cell per thread");
            Real vz[2][3];           // viscous halo column: (rho, rho u_a, rho w) at two planes
            int vrefl = 0;           // negate rho u_a (bit 0), rho w at plane p (bit 1 + p)
            int vc_i = 0, vc_j = 0;  // its tile coordinates
            int hi = 0, hj = 0;
            Real hu[NC];
            int hrefl = 0;
            // THINC: psi is read on the tile, the 1-cell ring (staged by the ring's
            // threads with PSI_CARRY) and the second ring's arms; a halo thread evaluates
            // it only there
            bool hpsi_needed = true;
            // FP64 five-equation WENO5-Z kernels: the halo index passes through an empty asm
            // here, so that the halo loads are issued in this step; the compiler otherwise
            // moved them to the end of the previous step, where their values, live across
            // the loop's back edge, were spilled as they arrived (each spill waiting for its
            // load).  Spills 93 -> 76 VGPRs, 0.889 -> 0.830 ms per stage at 256x128x128,
            // THINC 1.314 -> 1.295 ms; the other kernels measured equal or 0.3-1.2 % slower
            // with it.
            constexpr bool HALO_IN_STEP = MODEL == DIM && REC == REC_WENO_PRIM && sizeof(Real) == 8;
            int hsel = tid;
            if constexpr (HALO_IN_STEP) asm volatile("" : "+v"(hsel));
            const bool has_halo = hsel < TL::NHALO;
            if (has_halo) {
                const int h = hsel;
                if (h < 6 * BY) {
                    hj = h / 6;
                    const int k = h % 6;
                    hi = k < 3 ? k - 3 : BX + k - 3;
                    if constexpr (PSI_CARRY) hpsi_needed = k == 1 || k == 4;
                } else if (h < 6 * BY + 6 * BX) {
                    const int hh = h - 6 * BY;
                    hi = hh % BX;
                    const int k = hh / BX;
                    hj = k < 3 ? k - 3 : BY + k - 3;
                    if constexpr (PSI_CARRY) hpsi_needed = k == 1 || k == 4;
                } else if constexpr (VISC) {
                    const int hh = h - 6 * BY - 6 * BX;  // 2-deep corners (viscous cross terms)
                    const int ci = hh & 3, cj = hh >> 2;
                    hi = ci < 2 ? ci - 2 : BX + ci - 2;
                    hj = cj < 2 ? cj - 2 : BY + cj - 2;
                } else {
                    const int hh = h - 6 * BY - 6 * BX;  // 1-deep corners (THINC gradient)
                    hi = (hh & 1) ? BX : -1;
                    hj = (hh & 2) ? BY : -1;
                    if constexpr (PSI_CARRY) hpsi_needed = false;  // a ring cell
                }
                hrefl = load_cell_raw<Real>(a, a.Uk, x0 + hi, y0 + hj, s, hu, NC, interior_xy);
            }
            // viscous: the halo columns of the viscous regions need d/dz of two velocity
            // components at plane s; a pair of threads shares a column, the even one
            // loading planes s-2, s-1 and the odd one s+1, s+2 (issued here, reduced
            // after the halo ring is staged)
            if constexpr (VISC) {
                static_assert(2 * (4 * BY + 4 * BX) <= NT, "two threads per viscous halo column");
                if (xy && tid < 2 * (4 * BY + 4 * BX)) {
                    const int h = tid >> 1, odd = tid & 1;
                    int i, j;
                    if (h < 4 * BY) {
                        j = h / 4;
                        const int k = h % 4;
                        i = k < 2 ? k - 2 : BX + k - 2;
                    } else {
                        const int hh = h - 4 * BY;
                        i = hh % BX;
                        const int k = hh / BX;
                        j = k < 2 ? k - 2 : BY + k - 2;
                    }
                    vc_i = i;
                    vc_j = j;
                    const int ca = h < 4 * BY ? V : V + 1;  // u on the x region, v on the y region; then w
                    bool fx = false, fy = false;
                    const int ii = interior_xy ? x0 + i : map_index(x0 + i, a.nx, a.bc[0], a.bc[1], fx);
                    const int jj = interior_xy ? y0 + j : map_index(y0 + j, a.ny, a.bc[2], a.bc[3], fy);
                    const bool fa = h < 4 * BY ? fx : fy;
#pragma unroll
                    for (int p = 0; p < 2; p++) {
                        bool fz = false;
                        const int kk = map_index(s + (odd ? p + 1 : p - 2), a.nz, a.bc[4], a.bc[5], fz);
                        const long long qq = ((long long)kk * a.ny + jj) * a.nx + ii;
                        vz[p][0] = a.Uk[qq];
                        vz[p][1] = a.Uk[ca * a.ncell + qq];
                        vz[p][2] = a.Uk[(V + 2) * a.ncell + qq];
                        vrefl |= (fa ? 1 : 0) | (fz ? 2 << p : 0);
                    }
                } else {
#pragma unroll
                    for (int p = 0; p < 2; p++)
#pragma unroll
                        for (int c = 0; c < 3; c++) vz[p][c] = Real(1);
                }
            }
            // the plane buffer is overwritten below: after a step with x/y phases their
            // barriers already ordered every read of it; after a warm-up step (only the
            // in-plane derivatives read it) a barrier is needed here
            // THINC: alpha of the ring cell at plane s+1 (and s-1 without PSI_CARRY) for
            // d(psi)/dz at plane s, issued with the step's other loads
            Real ring_am = 0, ring_ap = 0;
            int ring_i = 0, ring_j = 0;
            if constexpr (PSI_CARRY) {
                if (carry_ring) ring_ap = ring_alpha(s + 1);
            } else if constexpr (THINC) {
                const int h = NT - 1 - tid;
                if (h < TL::NRING) {
                    if (h < 2 * BY) {
                        ring_j = h >> 1;
                        ring_i = (h & 1) ? BX : -1;
                    } else if (h < 2 * BY + 2 * BX) {
                        const int hh = h - 2 * BY;
                        ring_i = hh >> 1;
                        ring_j = (hh & 1) ? BY : -1;
                    } else {
                        const int hh = h - 2 * BY - 2 * BX;
                        ring_i = (hh & 1) ? BX : -1;
                        ring_j = (hh & 2) ? BY : -1;
                    }
                    bool fx = false, fy = false, fz = false;
                    const int ii = map_index(x0 + ring_i, a.nx, a.bc[0], a.bc[1], fx);
                    const int jj = map_index(y0 + ring_j, a.ny, a.bc[2], a.bc[3], fy);
                    const int km = map_index(s - 1, a.nz, a.bc[4], a.bc[5], fz);
                    const int kp = map_index(s + 1, a.nz, a.bc[4], a.bc[5], fz);
                    const long long col = (long long)jj * a.nx + ii, plane = (long long)a.ny * a.nx;
                    ring_am = a.Uk[6 * a.ncell + km * plane + col];
                    ring_ap = a.Uk[6 * a.ncell + kp * plane + col];
                }
            }
            // THINC FP64 with primitive WENO5-Z: after a step with x/y phases the plane buffer
            // is free here (its last reader, the y reconstructions, ended at a barrier), so the
            // halo cell is converted and staged at once instead of being held through the
            // ring's psi (the compiler otherwise spilled its loads one by one as they arrived):
            // 1.297 -> 1.266 ms per stage for the five-equation THINC shock-bubble at
            // 256x128x128; with THINC the other reconstruction families measured equal or
            // 0.7-1.3 % slower so
            constexpr bool HALO_EARLY = THINC && sizeof(Real) == 8 && REC == REC_WENO_PRIM;
            bool halo_done = false;  // uniform: the previous step had x/y phases
            if constexpr (HALO_EARLY) {
                if ((s - 1 >= z0) && (s - 1 < z1)) {
                    if (has_halo) {
                        Real w[NC];
                        apply_reflections(hu, V, hrefl);
                        cons_to_prim<Real, MODEL>(mat, hu, w);
                        Real hpsi = 0;
                        if (hpsi_needed) hpsi = thinc_psi(w[6]);
                        stage_w(hi, hj, w, hpsi, hpsi_needed);
                    }
                    halo_done = true;
                }
            }
            if constexpr (!OWN_AFTER_Z) convert_own();
            const bool prev_xy = (s - 1 >= z0) && (s - 1 < z1);
            if (!prev_xy) __syncthreads();
            // ---- P0: stage plane s in LDS (own cell from the window, halo ring from memory)
            if (has_cell) stage_w(tx, ty, win[3 + WO], psw[THINC ? 3 + WO : 0]);
            if constexpr (THINC) {
                // d(psi)/dz at plane s (second-order central): own column from the
                // window, the 1-cell ring from PSQ and memory (highest-numbered threads),
                // which also stage the ring's psi at plane s
                const Real hz = Real(0.5) * idz;
                if (has_cell) AZ[(ty + 1) * (BX + 2) + tx + 1] = (psw[4 + WO] - psw[2 + WO]) * hz;
                if constexpr (PSI_CARRY) {
                    if (carry_ring) {
                        const Real pm = PSQ[((s - 1) & 1) * TL::NRING + rh];
                        const Real p0 = PSQ[(s & 1) * TL::NRING + rh];
                        const Real pp = thinc_psi(ring_ap);
                        AZ[(cr_j + 1) * (BX + 2) + cr_i + 1] = (pp - pm) * hz;
                        wp(NC, cr_i, cr_j) = p0;
                        PSQ[((s + 1) & 1) * TL::NRING + rh] = pp;  // the slot of plane s-1
                    }
                } else if (NT - 1 - tid < TL::NRING) {
                    AZ[(ring_j + 1) * (BX + 2) + ring_i + 1] = (thinc_psi(ring_ap) - thinc_psi(ring_am)) * hz;
                }
            }
            if (!(HALO_EARLY && halo_done)) {
                if (has_halo) {
                    Real w[NC];
                    apply_reflections(hu, V, hrefl);
                    cons_to_prim<Real, MODEL>(mat, hu, w);
                    Real hpsi = 0;
                    if constexpr (THINC) {
                        if (hpsi_needed) hpsi = thinc_psi(w[6]);
                    }
                    stage_w(hi, hj, w, hpsi, hpsi_needed);
                }
            }
            if constexpr (VISC) {
                if (xy) {
                    // d/dz of the velocity at plane s: own column from the window
                    const Real i12 = a.inv12dz;
                    if (has_cell) {
                        Real dz[3];
#pragma unroll
                        for (int c = 0; c < 3; c++)
                            dz[c] = dcell(win[1 + WO][V + c], win[2 + WO][V + c], win[4 + WO][V + c], win[5 + WO][V + c], i12);
                        DZX[0 * TL::RX + ty * (BX + 4) + tx + 2] = dz[0];
                        DZX[1 * TL::RX + ty * (BX + 4) + tx + 2] = dz[2];
                        DZY[0 * TL::RY + (ty + 2) * BX + tx] = dz[1];
                        DZY[1 * TL::RY + (ty + 2) * BX + tx] = dz[2];
                    }
                    // halo columns of the viscous regions (loads issued at the start of the
                    // step): velocities at the thread's two planes, then the pair swaps half
                    // of them so that the even thread differentiates the first component
                    // (u or v) and the odd one w, each from all four planes
                    const int odd = tid & 1;
                    Real va[2], vb[2];
#pragma unroll
                    for (int p = 0; p < 2; p++) {
                        const Real ir = rcp(vz[p][0]);
                        va[p] = ((vrefl & 1) ? -vz[p][1] : vz[p][1]) * ir;
                        vb[p] = ((vrefl & (2 << p)) ? -vz[p][2] : vz[p][2]) * ir;
                    }
                    const Real y0 = __shfl_xor(odd ? va[0] : vb[0], 1, 64);
                    const Real y1 = __shfl_xor(odd ? va[1] : vb[1], 1, 64);
                    if (tid < 2 * (4 * BY + 4 * BX)) {
                        const Real d = odd ? dcell(y0, y1, vb[0], vb[1], i12) : dcell(va[0], va[1], y0, y1, i12);
                        if ((tid >> 1) < 4 * BY) DZX[odd * TL::RX + vc_j * (BX + 4) + vc_i + 2] = d;
                        else DZY[odd * TL::RY + (vc_j + 2) * BX + vc_i] = d;
                    }
                }
            }
            __syncthreads();
            if (VISC && has_cell) {
                // in-plane derivatives of the own column for the z faces
                const Real i12x = a.inv12dx, i12y = a.inv12dy;
                Dnew[0] = dcell(wp(V + 2, tx - 2, ty), wp(V + 2, tx - 1, ty), wp(V + 2, tx + 1, ty), wp(V + 2, tx + 2, ty), i12x);
                Dnew[1] = dcell(wp(V, tx - 2, ty), wp(V, tx - 1, ty), wp(V, tx + 1, ty), wp(V, tx + 2, ty), i12x);
                Dnew[2] = dcell(wp(V + 2, tx, ty - 2), wp(V + 2, tx, ty - 1), wp(V + 2, tx, ty + 1), wp(V + 2, tx, ty + 2), i12y);
                Dnew[3] = dcell(wp(V + 1, tx, ty - 2), wp(V + 1, tx, ty - 1), wp(V + 1, tx, ty + 1), wp(V + 1, tx, ty + 2), i12y);
            }
            if (THINC && has_cell) {
                // in-plane gradient of psi of the own column (THINC at the z faces)
                Anew[0] = (wp(NC, tx + 1, ty) - wp(NC, tx - 1, ty)) * (Real(0.5) * idx);
                Anew[1] = (wp(NC, tx, ty + 1) - wp(NC, tx, ty - 1)) * (Real(0.5) * idy);
            }
        } else if constexpr (!OWN_AFTER_Z) {
            convert_own();
        }

        // ---- z work of the own column (registers only): finalises cell s-2
        if (has_cell && s >= z0) {
            // primitive variables: the reconstruction of cell s-1 from W(s-3 .. s+1) gives
            // its face values at s-3/2 (used now) and s-1/2 (carried to the next step)
            Real vm_new[NC], vp[NC];
            if constexpr (!FACE) {
#pragma unroll
                for (int m = 0; m < NC; m++)
                    weno5z_pair(win[0][m], win[1][m], win[2][m], win[3][m], win[4][m], weps, vm_new[m], vp[m]);
            }
            if (s >= z0 + 1) {
                // z face s-3/2 between cells s-2 (win[1]) and s-1 (win[2])
                Real Fd[4];
                if constexpr (VISC) {
                    // viscous part first: its inputs are the window and the carried derivatives
                    const Real i24 = a.inv24dz;
                    Real dn[4], vf[3];
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const Real q0 = win[WO][V + c], q1 = win[1 + WO][V + c], q2 = win[2 + WO][V + c], q3 = win[3 + WO][V + c];
                        dn[c] = dface(q0, q1, q2, q3, i24);
                        vf[c] = ifc(q0, q1, q2, q3);
                    }
                    const Real th0 = win[WO][P] * rcp(win[WO][0]), th1 = win[1 + WO][P] * rcp(win[1 + WO][0]);
                    const Real th2 = win[2 + WO][P] * rcp(win[2 + WO][0]), th3 = win[3 + WO][P] * rcp(win[3 + WO][0]);
                    dn[3] = dface(th0, th1, th2, th3, i24);
                    Real muf = a.mu, kf = a.kappa;
                    if constexpr (VLAW) {
                        muf = visc_mu(a.vl, ifc(th0, th1, th2, th3));
                        kf = muf * a.vl.kfac;
                    }
                    const Real g_xw = ifc(Dc[0][0], Dc[1][0], Dc[2][0], Dnew[0]);  // dw/dx
                    const Real g_yw = ifc(Dc[0][2], Dc[1][2], Dc[2][2], Dnew[2]);  // dw/dy
                    const Real g_xu = ifc(Dc[0][1], Dc[1][1], Dc[2][1], Dnew[1]);  // du/dx
                    const Real g_yv = ifc(Dc[0][3], Dc[1][3], Dc[2][3], Dnew[3]);  // dv/dy
                    viscous_flux_from_gradients<Real, 2>(dn, vf, g_xw, g_yw, g_xu, g_yv, muf, kf, Fd);
                    __builtin_amdgcn_sched_barrier(0);  // keep the two flux parts from interleaving (registers)
                }
                Real wl[NC], wr[NC], F[NC], uh;
                if constexpr (CHARV) {
                    // characteristic variables of the face's frozen state, stencil s-4 .. s+1
                    char_face_states<Real, MODEL, 2, TENO>(mat, [&](int q, int m) { return win[q][m]; }, weps, wl, wr);
                } else if constexpr (TENO) {
#pragma unroll
                    for (int m = 0; m < NC; m++)
                        teno6a_pair(win[0][m], win[1][m], win[2][m], win[3][m], win[4][m], win[5][m], weps, wl[m], wr[m]);
                } else {
#pragma unroll
                    for (int m = 0; m < NC; m++) {
                        wl[m] = vminus[m];
                        wr[m] = vp[m];
                    }
                }
                if constexpr (THINC) {
                    // interface cells s-2 (its +z face) and s-1 (its -z face)
                    const Real hz = Real(0.5) * idz;
                    const Real a0 = win[WO][6], a1 = win[1 + WO][6], a2 = win[2 + WO][6], a3 = win[3 + WO][6];
                    Real af, gz = (psw[2 + WO] - psw[WO]) * hz;
                    if (thinc_face(a0, a1, a2, gz, Ag[0][0] * Ag[0][0] + Ag[0][1] * Ag[0][1] + gz * gz, 1, af))
                        thinc_state(af, win[1 + WO][0], win[1 + WO][1], a1, wl);
                    gz = (psw[3 + WO] - psw[1 + WO]) * hz;
                    if (thinc_face(a1, a2, a3, gz, Ag[1][0] * Ag[1][0] + Ag[1][1] * Ag[1][1] + gz * gz, 0, af))
                        thinc_state(af, win[2 + WO][0], win[2 + WO][1], a2, wr);
                }
                if constexpr (POS) {
                    const bool il = inadmissible_w<Real, MODEL>(mat, tol, wl);
                    if (il)
#pragma unroll
                        for (int m = 0; m < NC; m++) wl[m] = win[1 + WO][m];
                    const bool ir = inadmissible_w<Real, MODEL>(mat, tol, wr);
                    if (ir)
#pragma unroll
                        for (int m = 0; m < NC; m++) wr[m] = win[2 + WO][m];
                    hllc<Real, MODEL, 2>(mat, wl, wr, F, uh);
                    const bool fl = flux_limiter_trips<Real, MODEL, 2>(mat, tol, win[1 + WO], win[2 + WO], F, uh, lamz);
                    if (fl) hllc<Real, MODEL, 2>(mat, win[1 + WO], win[2 + WO], F, uh);
                    if constexpr (REC_FLAGS) {
                        // z face s-1 (between cells s-2 and s-1)
                        if (own_valid)
                            a.flags[a.flag_off[2] + ((long long)(s - 1) * a.ny + gy) * a.nx + gx] =
                                (unsigned char)((il ? 1 : 0) | (ir ? 2 : 0) | (fl ? 4 : 0));
                    }
                } else {
                    hllc<Real, MODEL, 2>(mat, wl, wr, F, uh);
                }
                if constexpr (VISC) {
                    F[V] -= Fd[0];
                    F[V + 1] -= Fd[1];
                    F[V + 2] -= Fd[2];
                    F[P] -= Fd[3];
                }
                if (s >= z0 + 2 && own_valid) {
                    // finalise cell s-2: R = (x/y part) - (F_{s-3/2} - F_{s-5/2}) / dz
                    const long long q = ((long long)(s - 2) * a.ny + gy) * a.nx + gx;
                    Real r[NC];
                    if constexpr (ACC_LDS) {
                        const Real* slot = ACC + (s & 1) * NC * NCELL + tid;
#pragma unroll
                        for (int m = 0; m < NC; m++) r[m] = slot[m * NCELL] - (F[m] - Fzl[m]) * idz;
                    } else if constexpr (ACC_HALF) {
                        if (s & 1) {
#pragma unroll
                            for (int m = 0; m < NC; m++) r[m] = accA[m] - (F[m] - Fzl[m]) * idz;
                        } else {
#pragma unroll
                            for (int m = 0; m < NC; m++) r[m] = ACC[m * NCELL + tid] - (F[m] - Fzl[m]) * idz;
                        }
                    } else {
#pragma unroll
                        for (int m = 0; m < NC; m++) r[m] = accA[m] - (F[m] - Fzl[m]) * idz;
                    }
                    if constexpr (MODEL == DIM) r[6] += win[1 + WO][6] * (srcA + (uh - uhzl) * idz);
                    if constexpr (MODEL == NS && (VMODE == VM_EXT || VMODE == VM_EXT_LAW)) {
                        // divergence of the sixth-order viscous fluxes (separate passes)
#pragma unroll
                        for (int c = 0; c < 3; c++) r[V + c] += a.rvisc[c * a.ncell + q];
                        r[P] += a.rvisc[3 * a.ncell + q];
                    }
                    Real unew[NC];
                    if (a.mode != 0) {
#pragma unroll
                        for (int m = 0; m < NC; m++) {
                            pre_k[m] = a.Uk[m * a.ncell + q];
                            pre_n[m] = a.mode >= 2 ? a.Un[m * a.ncell + q] : Real(0);
                        }
                    }
                    store_cell_impl<Real, NC>(a, q, r, dt, pre_k, pre_n, unew);
                    if (a.inv_max) tmax = fmax(tmax, inverse_dt<Real, MODEL, MODEL == NS && (VMODE == VM_LAW || VMODE == VM_EXT_LAW)>(a, unew));
                }
#pragma unroll
                for (int m = 0; m < NC; m++) Fzl[m] = F[m];
                uhzl = uh;
            }
            if constexpr (!FACE) {
#pragma unroll
                for (int m = 0; m < NC; m++) vminus[m] = vm_new[m];
            }
        }

        if constexpr (OWN_AFTER_Z) load_own();
        if (xy) {
            Real* slot = ACC + (s & 1) * NC * NCELL + tid;  // partial sums of cell s (ACC_LDS)
            // FP64: waves with more work than the others in a phase (the remainder of a task
            // list) take a higher issue priority on their SIMD until the phase's barrier, over
            // the co-resident workgroup's waves, so that the workgroup reaches the barrier
            // sooner: the reconstruction phases' remainder waves priority 1, the face phases'
            // remainder wave priority 2.  NS 256^3 2.260 -> 2.18 ms per stage, five-equation
            // 256x128x128 0.949 -> 0.914 ms, Euler equal; FP32 (three workgroups per CU)
            // measured 0.4-2 % slower with it and keeps the default priority.
            constexpr int P1_ITEMS = CHARV ? TL::NFX : (TENO ? NC * TL::NFX : NC * (BX + 2) * BY);
            constexpr int P4_ITEMS = CHARV ? TL::NFY : (TENO ? NC * TL::NFY : NC * BX * (BY + 2));
            const bool prio_p1 = sizeof(Real) == 8 && (rt >> 6) < ((P1_ITEMS % NT) + 63) / 64;
            const bool prio_p4 = sizeof(Real) == 8 && (rt >> 6) < ((P4_ITEMS % NT) + 63) / 64;
            // ---- P1: x reconstructions (cells -1 .. BX of each row) [+ d/dy on the x region]
            if (prio_p1) __builtin_amdgcn_s_setprio(1);
            Real* FL = FB;
            Real* FR = FB + NC * TL::NFX;
            if constexpr (CHARV) {
                // one task per x face: characteristic reconstruction of both face states
                for (int t = rt; t < TL::NFX; t += NT) {
                    const int j = t / (BX + 1), f = t - j * (BX + 1);
                    Real wl[NC], wr[NC];
                    char_face_states<Real, MODEL, 0, TENO>(mat, [&](int q, int m) { return wp(m, f - 3 + q, j); }, weps,
                                                           wl, wr);
#pragma unroll
                    for (int m = 0; m < NC; m++) {
                        FL[m * TL::NFX + t] = wl[m];
                        FR[m * TL::NFX + t] = wr[m];
                    }
                }
            } else if constexpr (TENO) {
                // one item = one component of one x face (faces between cells f-1 and f)
                for (int it = rt; it < NC * TL::NFX; it += NT) {
                    const int m = it / TL::NFX, t = it - m * TL::NFX;
                    const int j = t / (BX + 1), f = t - j * (BX + 1);
                    const Real* c = &wp(m, f - 3, j);
                    teno6a_pair(c[0], c[1], c[2], c[3], c[4], c[5], weps, FL[it], FR[it]);
                }
            } else {
                // one item = one component of one cell; consecutive lanes take consecutive cells
                constexpr int NTX = (BX + 2) * BY;
                auto item = [&](int it) {
                    const int m = it / NTX, t = it - m * NTX;
                    const int j = t / (BX + 2), i = t - j * (BX + 2) - 1;
                    const Real* c = &wp(m, i, j);
                    Real vm, vp;
                    weno5z_pair(c[-2], c[-1], c[0], c[1], c[2], weps, vm, vp);
                    if (i < BX) FL[m * TL::NFX + j * (BX + 1) + i + 1] = vm;
                    if (i >= 0) FR[m * TL::NFX + j * (BX + 1) + i] = vp;
                };
#pragma unroll 1
                for (int it = rt; it < NC * NTX; it += NT) item(it);
            }
            if constexpr (VISC) {
                // d/dy of u (c = 0) and v (c = 1) on the x-face region
                const Real i12 = a.inv12dy;
                for (int it = rt; it < 2 * TL::RX; it += NT) {
                    const int c = it >= TL::RX, t = it - c * TL::RX;
                    const int j = t / (BX + 4), i = t % (BX + 4) - 2;
                    DT[it] = dcell(wp(V + c, i, j - 2), wp(V + c, i, j - 1), wp(V + c, i, j + 1), wp(V + c, i, j + 2), i12);
                }
            }
            if (prio_p1) __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            // ---- P2: x faces f = 0 .. BX (between cells f-1 and f)
            // the wave holding rt = 0 also runs the remainder round of the x and y face lists
            const bool prio_tail = sizeof(Real) == 8 && (rt >> 6) == 0;  // wave-uniform
            if (prio_tail) __builtin_amdgcn_s_setprio(2);
            for (int t = rt; t < TL::NFX; t += NT) {
                const int j = t / (BX + 1), f = t % (BX + 1);
                Real wl[NC], wr[NC], F[NC], uh;
#pragma unroll
                for (int m = 0; m < NC; m++) {
                    wl[m] = FL[m * TL::NFX + t];
                    wr[m] = FR[m * TL::NFX + t];
                }
                if constexpr (THINC) {
                    // interface cells f-1 (its +x face) and f (its -x face)
                    const Real hx = Real(0.5) * idx, hy = Real(0.5) * idy;
                    const Real am = wp(6, f - 2, j), a0 = wp(6, f - 1, j), a1 = wp(6, f, j), ap = wp(6, f + 1, j);
                    Real af, gx = (wp(NC, f, j) - wp(NC, f - 2, j)) * hx;
                    Real gy = (wp(NC, f - 1, j + 1) - wp(NC, f - 1, j - 1)) * hy, gz = AZ[(j + 1) * (BX + 2) + f];
                    if (thinc_face(am, a0, a1, gx, gx * gx + gy * gy + gz * gz, 1, af))
                        thinc_state(af, wp(0, f - 1, j), wp(1, f - 1, j), a0, wl);
                    gx = (wp(NC, f + 1, j) - wp(NC, f - 1, j)) * hx;
                    gy = (wp(NC, f, j + 1) - wp(NC, f, j - 1)) * hy;
                    gz = AZ[(j + 1) * (BX + 2) + f + 1];
                    if (thinc_face(a0, a1, ap, gx, gx * gx + gy * gy + gz * gz, 0, af))
                        thinc_state(af, wp(0, f, j), wp(1, f, j), a1, wr);
                }
                if constexpr (POS) {
                    Real wi[NC], wj[NC];
#pragma unroll
                    for (int m = 0; m < NC; m++) {
                        wi[m] = wp(m, f - 1, j);
                        wj[m] = wp(m, f, j);
                    }
                    const bool il = inadmissible_w<Real, MODEL>(mat, tol, wl);
                    if (il)
#pragma unroll
                        for (int m = 0; m < NC; m++) wl[m] = wi[m];
                    const bool ir = inadmissible_w<Real, MODEL>(mat, tol, wr);
                    if (ir)
#pragma unroll
                        for (int m = 0; m < NC; m++) wr[m] = wj[m];
                    hllc<Real, MODEL, 0>(mat, wl, wr, F, uh);
                    const bool fl = flux_limiter_trips<Real, MODEL, 0>(mat, tol, wi, wj, F, uh, lamx);
                    if (fl) hllc<Real, MODEL, 0>(mat, wi, wj, F, uh);
                    if constexpr (REC_FLAGS) {
                        // x face x0+f (between cells x0+f-1 and x0+f) of row y0+j, plane s
                        if (x0 + f <= a.nx && y0 + j < a.ny)
                            a.flags[a.flag_off[0] + ((long long)s * a.ny + y0 + j) * (a.nx + 1) + x0 + f] =
                                (unsigned char)((il ? 1 : 0) | (ir ? 2 : 0) | (fl ? 4 : 0));
                    }
                } else {
                    hllc<Real, MODEL, 0>(mat, wl, wr, F, uh);
                }
                if constexpr (VISC) {
                    const int r0 = j * (BX + 4) + f;  // region index of cell f-2
                    Real Fd[4];
                    Real muf = a.mu, kf = a.kappa;
                    if constexpr (VLAW) {
                        const Real* th = &wp(NC, f - 2, j);
                        muf = visc_mu(a.vl, ifc(th[0], th[1], th[2], th[3]));
                        kf = muf * a.vl.kfac;
                    }
                    viscous_flux_lds<Real, 0>(&wp(V, f - 2, j), &wp(NC, f - 2, j), 1, PLANE, DT + r0, DZX + r0,
                                              DT + TL::RX + r0, DZX + TL::RX + r0, 1, muf, kf, a.inv24dx, Fd);
                    F[V] -= Fd[0];
                    F[V + 1] -= Fd[1];
                    F[V + 2] -= Fd[2];
                    F[P] -= Fd[3];
                }
#pragma unroll
                for (int m = 0; m < NC; m++) FL[m * TL::NFX + t] = F[m];
                if constexpr (MODEL == DIM) UHB[t] = uh;
            }
            if (prio_tail) __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            // ---- P3: x divergence of the own cell
            if (has_cell) {
                const int fl = ty * (BX + 1) + tx;
#pragma unroll
                for (int m = 0; m < NC; m++) {
                    const Real v = -(FL[m * TL::NFX + fl + 1] - FL[m * TL::NFX + fl]) * idx;
                    if constexpr (ACC_LDS) slot[m * NCELL] = v;
                    else accC[m] = v;
                }
                if constexpr (MODEL == DIM) srcC = (UHB[fl + 1] - UHB[fl]) * idx;
            }
            __syncthreads();
            // ---- P4: y reconstructions (rows -1 .. BY of each column) [+ d/dx on the y region]
            if (prio_p4) __builtin_amdgcn_s_setprio(1);
            Real* GL = FB;
            Real* GR = FB + NC * TL::NFY;
            if constexpr (CHARV) {
                for (int t = rt; t < TL::NFY; t += NT) {
                    const int f = t / BX, i = t - f * BX;
                    Real wl[NC], wr[NC];
                    char_face_states<Real, MODEL, 1, TENO>(mat, [&](int q, int m) { return wp(m, i, f - 3 + q); }, weps,
                                                           wl, wr);
#pragma unroll
                    for (int m = 0; m < NC; m++) {
                        GL[m * TL::NFY + t] = wl[m];
                        GR[m * TL::NFY + t] = wr[m];
                    }
                }
            } else if constexpr (TENO) {
                // one item = one component of one y face (faces between rows f-1 and f)
                for (int it = rt; it < NC * TL::NFY; it += NT) {
                    const int m = it / TL::NFY, t = it - m * TL::NFY;
                    const int f = t / BX, i = t - f * BX;
                    const Real* c = &wp(m, i, f - 3);
                    teno6a_pair(c[0], c[PX], c[2 * PX], c[3 * PX], c[4 * PX], c[5 * PX], weps, GL[it], GR[it]);
                }
            } else {
                // one item = one component of one cell; consecutive lanes take consecutive cells
                constexpr int NTY = BX * (BY + 2);
                auto item = [&](int it) {
                    const int m = it / NTY, t = it - m * NTY;
                    const int jj = t / BX, i = t - jj * BX, j = jj - 1;
                    const Real* c = &wp(m, i, j);
                    Real vm, vp;
                    weno5z_pair(c[-2 * PX], c[-PX], c[0], c[PX], c[2 * PX], weps, vm, vp);
                    if (j < BY) GL[m * TL::NFY + (j + 1) * BX + i] = vm;
                    if (j >= 0) GR[m * TL::NFY + j * BX + i] = vp;
                };
#pragma unroll 1
                for (int it = rt; it < NC * NTY; it += NT) item(it);
            }
            if constexpr (VISC) {
                // d/dx of v (c = 0) and u (c = 1) on the y-face region
                const Real i12 = a.inv12dx;
                for (int it = rt; it < 2 * TL::RY; it += NT) {
                    const int c = it >= TL::RY, t = it - c * TL::RY;
                    const int i = t % BX, j = t / BX - 2;
                    const int f = V + 1 - c;
                    DT[it] = dcell(wp(f, i - 2, j), wp(f, i - 1, j), wp(f, i + 1, j), wp(f, i + 2, j), i12);
                }
            }
            if (prio_p4) __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            // ---- P5: y faces f = 0 .. BY (between rows f-1 and f)
            if (prio_tail) __builtin_amdgcn_s_setprio(2);
            for (int t = rt; t < TL::NFY; t += NT) {
                const int i = t % BX, f = t / BX;
                Real wl[NC], wr[NC], F[NC], uh;
#pragma unroll
                for (int m = 0; m < NC; m++) {
                    wl[m] = GL[m * TL::NFY + t];
                    wr[m] = GR[m * TL::NFY + t];
                }
                if constexpr (THINC) {
                    // interface cells of rows f-1 (its +y face) and f (its -y face)
                    const Real hx = Real(0.5) * idx, hy = Real(0.5) * idy;
                    const Real am = wp(6, i, f - 2), a0 = wp(6, i, f - 1), a1 = wp(6, i, f), ap = wp(6, i, f + 1);
                    Real af, gy = (wp(NC, i, f) - wp(NC, i, f - 2)) * hy;
                    Real gx = (wp(NC, i + 1, f - 1) - wp(NC, i - 1, f - 1)) * hx, gz = AZ[f * (BX + 2) + i + 1];
                    if (thinc_face(am, a0, a1, gy, gx * gx + gy * gy + gz * gz, 1, af))
                        thinc_state(af, wp(0, i, f - 1), wp(1, i, f - 1), a0, wl);
                    gy = (wp(NC, i, f + 1) - wp(NC, i, f - 1)) * hy;
                    gx = (wp(NC, i + 1, f) - wp(NC, i - 1, f)) * hx;
                    gz = AZ[(f + 1) * (BX + 2) + i + 1];
                    if (thinc_face(a0, a1, ap, gy, gx * gx + gy * gy + gz * gz, 0, af))
                        thinc_state(af, wp(0, i, f), wp(1, i, f), a1, wr);
                }
                if constexpr (POS) {
                    Real wi[NC], wj[NC];
#pragma unroll
                    for (int m = 0; m < NC; m++) {
                        wi[m] = wp(m, i, f - 1);
                        wj[m] = wp(m, i, f);
                    }
                    const bool il = inadmissible_w<Real, MODEL>(mat, tol, wl);
                    if (il)
#pragma unroll
                        for (int m = 0; m < NC; m++) wl[m] = wi[m];
                    const bool ir = inadmissible_w<Real, MODEL>(mat, tol, wr);
                    if (ir)
#pragma unroll
                        for (int m = 0; m < NC; m++) wr[m] = wj[m];
                    hllc<Real, MODEL, 1>(mat, wl, wr, F, uh);
                    const bool fl = flux_limiter_trips<Real, MODEL, 1>(mat, tol, wi, wj, F, uh, lamy);
                    if (fl) hllc<Real, MODEL, 1>(mat, wi, wj, F, uh);
                    if constexpr (REC_FLAGS) {
                        // y face y0+f (between rows y0+f-1 and y0+f) of column x0+i, plane s
                        if (y0 + f <= a.ny && x0 + i < a.nx)
                            a.flags[a.flag_off[1] + ((long long)s * (a.ny + 1) + y0 + f) * a.nx + x0 + i] =
                                (unsigned char)((il ? 1 : 0) | (ir ? 2 : 0) | (fl ? 4 : 0));
                    }
                } else {
                    hllc<Real, MODEL, 1>(mat, wl, wr, F, uh);
                }
                if constexpr (VISC) {
                    const int r0 = f * BX + i;  // region index of cell f-2
                    Real Fd[4];
                    Real muf = a.mu, kf = a.kappa;
                    if constexpr (VLAW) {
                        const Real* th = &wp(NC, i, f - 2);
                        muf = visc_mu(a.vl, ifc(th[0], th[PX], th[2 * PX], th[3 * PX]));
                        kf = muf * a.vl.kfac;
                    }
                    viscous_flux_lds<Real, 1>(&wp(V, i, f - 2), &wp(NC, i, f - 2), PX, PLANE, DT + r0, DZY + r0,
                                              DT + TL::RY + r0, DZY + TL::RY + r0, BX, muf, kf, a.inv24dy, Fd);
                    F[V] -= Fd[0];
                    F[V + 1] -= Fd[1];
                    F[V + 2] -= Fd[2];
                    F[P] -= Fd[3];
                }
#pragma unroll
                for (int m = 0; m < NC; m++) GL[m * TL::NFY + t] = F[m];
                if constexpr (MODEL == DIM) UHB[t] = uh;
            }
            if (prio_tail) __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            // ---- P6: y divergence of the own cell
            if (has_cell) {
                const int fl = ty * BX + tx;
#pragma unroll
                for (int m = 0; m < NC; m++) {
                    const Real d = (GL[m * TL::NFY + fl + BX] - GL[m * TL::NFY + fl]) * idy;
                    if constexpr (ACC_LDS) slot[m * NCELL] -= d;
                    else accC[m] -= d;
                }
                if constexpr (MODEL == DIM) srcC += (UHB[fl + BX] - UHB[fl]) * idy;
            }
        }
        // rotate carries
        if constexpr (ACC_HALF) {
            // plane s: odd into the register slot, even into the thread's LDS slot
            if (s & 1) {
#pragma unroll
                for (int m = 0; m < NC; m++) accA[m] = accC[m];
            } else if (has_cell) {
#pragma unroll
                for (int m = 0; m < NC; m++) ACC[m * NCELL + tid] = accC[m];
            }
        } else if constexpr (!ACC_LDS) {
#pragma unroll
            for (int m = 0; m < NC; m++) {
                accA[m] = accB[m];
                accB[m] = accC[m];
            }
        }
        srcA = srcB;
        srcB = srcC;
        if constexpr (VISC) {
#pragma unroll
            for (int c = 0; c < 4; c++) {
                Dc[0][c] = Dc[1][c];
                Dc[1][c] = Dc[2][c];
                Dc[2][c] = Dnew[c];
            }
        }
        if constexpr (THINC) {
#pragma unroll
            for (int c = 0; c < 2; c++) {
                Ag[0][c] = Ag[1][c];
                Ag[1][c] = Anew[c];
            }
        }
        if constexpr (OWN_AFTER_Z) convert_own();
#pragma unroll
        for (int q = 0; q < NWIN - 1; q++)
#pragma unroll
            for (int f = 0; f < NC; f++) win[q][f] = win[q + 1][f];
        if constexpr (THINC) {
#pragma unroll
            for (int q = 0; q < NWIN - 1; q++) psw[q] = psw[q + 1];
        }
    }
    if (a.inv_max) {
        // block maximum of the inverse time step, one atomic per workgroup
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tmax = fmax(tmax, __shfl_xor(tmax, o, 64));
        __syncthreads();
        double* red = reinterpret_cast<double*>(smem_raw);
        if ((tid & 63) == 0) red[tid >> 6] = tmax;
        __syncthreads();
        if (tid == 0) {
            double m = red[0];
            for (int k = 1; k < NT / 64; k++) m = fmax(m, red[k]);
            atomicMax(a.inv_max, (unsigned long long)__double_as_longlong(m));
        }
    }
}

// Waves per SIMD the stage kernels are compiled for: two in FP64 (256 registers per
// lane), three in FP32 (168), where the narrower state leaves room for a third
template <typename Real>
constexpr int stage_waves()
{
    return sizeof(Real) == 4 ? WAVES_PER_EU_F32 : WAVES_PER_EU;
}

template <typename Real, int MODEL, int POS, int REC, int VMODE, int BX, int BY, int NTH>
__global__ void __launch_bounds__(NTH, stage_waves<Real>()) stage_kernel(const StageArgs<Real> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // the argument block read in place from the kernel-argument segment (fewer scalar
    // registers than a copy)
    const StageArgs<Real>* pa = (const StageArgs<Real>*)__builtin_amdgcn_kernarg_segment_ptr();
    stage_body<Real, MODEL, POS, REC, VMODE, BX, BY, NTH>(*pa, (int)blockIdx.x, smem_raw);
}

// Many independent problems in one launch: the workgroups of problem r are
// first[r] .. first[r+1]-1; args[r] describes problem r (same model, precision,
// limiter setting, reconstruction family and viscosity / interface variant for every
// problem of the launch); *count = n, read from the device table so that a captured
// launch serves any membership (workgroups beyond first[n] return at once).
template <typename Real, int MODEL, int POS, int REC, int VMODE, int BX, int BY, int NTH>
__global__ void __launch_bounds__(NTH, stage_waves<Real>())
    batch_stage_kernel(const StageArgs<Real>* __restrict__ args, const int* __restrict__ first,
                       const int* __restrict__ count)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = (int)blockIdx.x;
    const int n = *count;
    if (n <= 0 || b >= first[n]) return;
    int lo = 0, hi = n - 1;  // last r with first[r] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    // the argument block is read through the constant address space, as the single-problem
    // kernel reads its kernel-argument segment: the table does not change during the launch,
    // so the compiler may load its fields with scalar loads wherever it needs them
    using CArgs = const __attribute__((address_space(4))) StageArgs<Real>;
    const StageArgs<Real>* pa = (const StageArgs<Real>*)(CArgs*)(args + lo);
    stage_body<Real, MODEL, POS, REC, VMODE, BX, BY, NTH>(*pa, b - first[lo], smem_raw);
}

// ------------------------------------------------------------------ launchers
template <typename Real, int MODEL, int POS, int REC, int VMODE, int BX, int BY, int NTH>
static hipError_t launch_tile(const StageArgs<Real>& args, const LaunchGeom& g, hipStream_t st)
{
    using TL = Tile<Real, MODEL, BX, BY, NTH, MODEL == NS && VMODE != VM_EXT && VMODE != VM_EXT_LAW,
                    MODEL == DIM && VMODE == XM_THINC>;
    const size_t lds = TL::bytes();
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)stage_kernel<Real, MODEL, POS, REC, VMODE, BX, BY, NTH>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((stage_kernel<Real, MODEL, POS, REC, VMODE, BX, BY, NTH>), dim3(g.nblocks), dim3(NTH), lds,
                       st, args);
    return hipGetLastError();
}

template <typename Real, int MODEL, int REC, int VMODE>
static hipError_t launch_pos(const StageArgs<Real>& args, const LaunchGeom& g, hipStream_t st)
{
    if (args.positivity) {
        if (args.flags) return launch_tile<Real, MODEL, 2, REC, VMODE, TILE_BX, TILE_BY, TILE_NT>(args, g, st);
        return launch_tile<Real, MODEL, 1, REC, VMODE, TILE_BX, TILE_BY, TILE_NT>(args, g, st);
    }
    return launch_tile<Real, MODEL, 0, REC, VMODE, TILE_BX, TILE_BY, TILE_NT>(args, g, st);
}

// every variant of one precision, model and reconstruction (explicitly instantiated
// per reconstruction in fv_stage_inst.hip, so that the families compile separately and
// each with its own code-generation options)
template <typename Real, int MODEL, int REC>
hipError_t launch_rec(const StageArgs<Real>& args, const LaunchGeom& g, hipStream_t st)
{
    // a viscosity law is a separate instantiation (viscous model only): the law's
    // pow() must not weigh on the constant-viscosity kernel; sixth-order viscous
    // fluxes come from separate passes (the stage adds them)
    if constexpr (MODEL == NS) {
        if (args.rvisc)
            return args.vl.law != 0 ? launch_pos<Real, MODEL, REC, VM_EXT_LAW>(args, g, st)
                                    : launch_pos<Real, MODEL, REC, VM_EXT>(args, g, st);
        if (args.vl.law != 0) return launch_pos<Real, MODEL, REC, VM_LAW>(args, g, st);
    }
    if constexpr (MODEL == DIM) {
        if (args.thinc) return launch_pos<Real, MODEL, REC, XM_THINC>(args, g, st);
    }
    return launch_pos<Real, MODEL, REC, VM_CONST>(args, g, st);
}

template <typename Real, int MODEL>
size_t stage_lds_bytes()
{
    return Tile<Real, MODEL, TILE_BX, TILE_BY, TILE_NT>::bytes();
}

template <typename Real, int MODEL>
hipError_t launch_model(const StageArgs<Real>& args, const LaunchGeom& g, hipStream_t st)
{
    switch (args.recon) {
    case REC_WENO_CHAR: return launch_rec<Real, MODEL, REC_WENO_CHAR>(args, g, st);
    case REC_TENO_PRIM: return launch_rec<Real, MODEL, REC_TENO_PRIM>(args, g, st);
    case REC_TENO_CHAR: return launch_rec<Real, MODEL, REC_TENO_CHAR>(args, g, st);
    default: return launch_rec<Real, MODEL, REC_WENO_PRIM>(args, g, st);
    }
}

template <typename Real, int MODEL, int POS, int REC, int VMODE>
static hipError_t launch_batch_tile(const StageArgs<Real>* args, const int* first, const int* count, int nblocks,
                                    hipStream_t st)
{
    using TL = Tile<Real, MODEL, TILE_BX, TILE_BY, TILE_NT, MODEL == NS && VMODE != VM_EXT && VMODE != VM_EXT_LAW,
                    MODEL == DIM && VMODE == XM_THINC>;
    const size_t lds = TL::bytes();
    auto* k = batch_stage_kernel<Real, MODEL, POS, REC, VMODE, TILE_BX, TILE_BY, TILE_NT>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (nblocks <= 0) return hipSuccess;  // attribute set-up only
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(TILE_NT), lds, st, args, first, count);
    return hipGetLastError();
}

// the batched kernels of one precision, model and reconstruction family, instantiated
// with that family's single-problem kernels in fv_stage_inst.hip (so that they are
// compiled with the same code-generation options as the kernels they share their body
// with); variant: 0 constant viscosity / no THINC, 1 a viscosity law (NS) or THINC
// (five-equation model)
template <typename Real, int MODEL, int REC>
hipError_t launch_batch_rec(bool pos, int variant, const StageArgs<Real>* args, const int* first, const int* count,
                            int nblocks, hipStream_t st)
{
    if constexpr (MODEL != EULER) {
        if (variant) {
            constexpr int VM = MODEL == DIM ? XM_THINC : VM_LAW;
            return pos ? launch_batch_tile<Real, MODEL, 1, REC, VM>(args, first, count, nblocks, st)
                       : launch_batch_tile<Real, MODEL, 0, REC, VM>(args, first, count, nblocks, st);
        }
    }
    return pos ? launch_batch_tile<Real, MODEL, 1, REC, VM_CONST>(args, first, count, nblocks, st)
               : launch_batch_tile<Real, MODEL, 0, REC, VM_CONST>(args, first, count, nblocks, st);
}

template <typename Real, int MODEL>
hipError_t launch_batch_model(int rec, bool pos, int variant, const StageArgs<Real>* args, const int* first,
                              const int* count, int nblocks, hipStream_t st)
{
    switch (rec) {
    case REC_WENO_CHAR: return launch_batch_rec<Real, MODEL, REC_WENO_CHAR>(pos, variant, args, first, count, nblocks, st);
    case REC_TENO_PRIM: return launch_batch_rec<Real, MODEL, REC_TENO_PRIM>(pos, variant, args, first, count, nblocks, st);
    case REC_TENO_CHAR: return launch_batch_rec<Real, MODEL, REC_TENO_CHAR>(pos, variant, args, first, count, nblocks, st);
    default: return launch_batch_rec<Real, MODEL, REC_WENO_PRIM>(pos, variant, args, first, count, nblocks, st);
    }
}

template <typename Real>
hipError_t launch_batch_stage(int model, int rec, bool pos, int variant, const StageArgs<Real>* args, const int* first,
                              const int* count, int nblocks, hipStream_t st)
{
    switch (model) {
    case EULER: return launch_batch_model<Real, EULER>(rec, pos, 0, args, first, count, nblocks, st);
    case NS: return launch_batch_model<Real, NS>(rec, pos, variant, args, first, count, nblocks, st);
    default: return launch_batch_model<Real, DIM>(rec, pos, variant, args, first, count, nblocks, st);
    }
}

template <typename Real>
hipError_t launch_stage(int model, const StageArgs<Real>& args, const LaunchGeom& g, hipStream_t st)
{
    switch (model) {
    case EULER: return launch_model<Real, EULER>(args, g, st);
    case NS: return launch_model<Real, NS>(args, g, st);
    default: return launch_model<Real, DIM>(args, g, st);
    }
}

}  // namespace fv
