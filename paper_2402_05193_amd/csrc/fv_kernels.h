// fv_kernels.h -- kernel argument blocks and launchers shared by the HIP
// sources of the library (internal; the public interface is include/fvrk3.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fv_physics.h"

#ifndef TILE_BX
#define TILE_BX 16
#endif
#ifndef TILE_BY
#define TILE_BY 16
#endif
#ifndef TILE_NT
#define TILE_NT 256
#endif
#ifndef WAVES_PER_EU
#define WAVES_PER_EU 2
#endif
#ifndef WAVES_PER_EU_F32
#define WAVES_PER_EU_F32 3
#endif

namespace fv {

// Reconstruction variants of the stage kernel: WENO5-Z or TENO6-A (Sec. 3.2
// step 3) of primitive or characteristic variables (value: recon + 2 scheme).
enum { REC_WENO_PRIM = 0, REC_WENO_CHAR = 1, REC_TENO_PRIM = 2, REC_TENO_CHAR = 3 };
// Viscous variants of the viscous model: constant viscosity, a viscosity law
// (both 4th-order fluxes inside the stage), or sixth-order fluxes from the
// separate passes of fv_visc6.hip (constant viscosity / a law: the law only
// enters the stage's CFL reduction)
enum { VM_CONST = 0, VM_LAW = 1, VM_EXT = 2, VM_EXT_LAW = 3 };
// and of the five-equation model: THINC interface capturing off / on
enum { XM_PLAIN = 0, XM_THINC = 1 };

// Arguments of the fused stage kernel (passed by value).
template <typename Real>
struct StageArgs {
    const Real* Uk;      // state the RHS is evaluated on
    const Real* Un;      // Runge-Kutta base state (stages 2, 3)
    Real* out;           // R (mode 0) or the new stage state
    const double* dt_dev;// device dt (or null: use dt)
    double dt;
    int mode;            // 0: R, 1..3: Shu-Osher stage
    int nx, ny, nz;
    long long ncell;     // component stride
    int bc[6];
    int tiles_x, tiles_y, zchunk, nchunks;
    int positivity, ndim;
    int recon;           // reconstruction variant REC_* (variables and scheme)
    Material<Real> mat;
    Tolerances<Real> tol;
    Real weno_eps;
    Real idx, idy, idz;
    Real inv12dx, inv12dy, inv12dz, inv24dx, inv24dy, inv24dz;
    Real mu, kappa;      // kappa = mu gamma / ((gamma-1) Pr)
    // optional CFL reduction over the stage output (stage 3): max over cells of
    // max_d (|u_d| + c)/dx_d and kvisc / rho, as the bit pattern of a double
    unsigned long long* inv_max;
    double kvisc;        // (14/3) mu / dx_min^2 (0 without viscosity)
    double kvisc_h;      // (14/3) / dx_min^2 (viscosity laws)
    ViscLaw<Real> vl;    // viscosity law of the faces (law 0: mu and kappa above)
    // sixth-order viscous fluxes computed by the separate passes of fv_visc6.hip:
    // their divergence [4][ncell] (momentum x, y, z, energy), added when a cell is
    // finalised; null: the stage computes the 4th-order viscous fluxes itself
    const Real* rvisc;
    int thinc;           // five-equation model: THINC volume-fraction faces in interface cells
    // limiter decisions of every face (null: not recorded; with the limiters on, the
    // kernel variant that writes them): one byte per face, the x faces at
    // flags[flag_off[0] + (k ny + j)(nx+1) + i], y at flags[flag_off[1] + (k (ny+1) + j) nx + i],
    // z at flags[flag_off[2] + (k ny + j) nx + i]
    unsigned char* flags;
    long long flag_off[3];
};

struct LaunchGeom {
    int nblocks;
};

template <typename Real>
hipError_t launch_stage(int model, const StageArgs<Real>& args, const LaunchGeom& g, hipStream_t st);

template <typename Real, int MODEL>
size_t stage_lds_bytes();

// Fused stage over n independent problems of one model / precision / limiter
// setting / reconstruction family (rec: REC_*) / variant (1: a viscosity law for NS,
// THINC for the five-equation model): args[r] describes problem r, whose workgroups
// are first[r] .. first[r+1]-1 (device arrays), n = *count (device).  nblocks >=
// first[n] workgroups are launched (the rest return at once); nblocks 0 only prepares
// the kernel's attributes (call before stream capture).
template <typename Real>
hipError_t launch_batch_stage(int model, int rec, bool pos, int variant, const StageArgs<Real>* args, const int* first,
                              const int* count, int nblocks, hipStream_t st);

// Sixth-order central viscous fluxes (fv_visc6.hip), three passes over the
// state U of the viscous model:
//   Q  [4][npad]  u, v, w, theta = p / rho on the box padded by 3 cells
//                 (boundary conditions by index mapping);
//   G  [9][npad]  du_c/dx_e at cell centres (index 3 c + e), where the
//                 e-coordinate of the cell is interior;
//   Rv [4][ncell] divergence of the viscous face fluxes (momentum x, y, z,
//                 energy): R = -div(F^c - F^d) receives +div F^d.
template <typename Real>
struct Visc6Args {
    int nx, ny, nz;
    int bc[6];
    long long ncell, npad;
    Material<Real> mat;
    ViscLaw<Real> vl;
    Real ih[3];  // 1 / dx_d
};

template <typename Real>
hipError_t launch_visc6(const Visc6Args<Real>& a, const Real* U, Real* Q, Real* G, Real* Rv, hipStream_t st);

// Per-problem scalars of a batch in CFL mode.
struct BatchScalars {
    unsigned long long* inv_max;  // stage-3 reduction target
    double* dt;                   // time step of the next step
    double* t_acc;                // simulated time
    double cfl;
};
// for every r < *count (device): t_acc += dt; dt = cfl / inv_max; inv_max = 0; the
// launch covers max_n members
hipError_t launch_batch_dt_finish(const BatchScalars* s, const int* count, int max_n, hipStream_t st);

// Point-wise / reduction kernels (fv_aux.hip)
struct AuxArgs {
    int model, nx, ny, nz;
    long long ncell;
    double dx, dy, dz;
    Material<double> matd;
    Material<float> matf;
    ViscLaw<double> vl;  // viscosity law for the viscous CFL limit
};

template <typename Real>
hipError_t launch_prim_to_cons(const AuxArgs& a, const Real* W, Real* U, hipStream_t st);
template <typename Real>
hipError_t launch_cons_to_prim(const AuxArgs& a, const Real* U, Real* W, hipStream_t st);
template <typename Real>
hipError_t launch_init(const AuxArgs& a, int case_id, const double* params, int nparams, uint64_t seed, Real* U,
                       hipStream_t st);
// max over cells of the inverse CFL time step into *inv_max (uint64 bit pattern of a
// non-negative double); then dt = cfl / max and *t_acc += dt (if t_acc).
template <typename Real>
hipError_t launch_dt(const AuxArgs& a, const Real* U, double mu, double cfl, unsigned long long* inv_max,
                     double* dt_out, double* t_acc, hipStream_t st);
// admissibility / finiteness scan; ws_words: [0] first bad index (int64, init INT64_MAX),
// [1] count, [2] worst code
template <typename Real>
hipError_t launch_check(const AuxArgs& a, const Real* U, long long* ws_words, hipStream_t st);
hipError_t launch_add_scalar(double* t_acc, const double* dt, hipStream_t st);
// *inv_max = 0
hipError_t launch_reset_max(unsigned long long* inv_max, hipStream_t st);
// p[0 .. n) = v (a kernel, so that it can be captured in a graph)
hipError_t launch_fill_u8(unsigned char* p, long long n, unsigned char v, hipStream_t st);
// t_acc (optional) += *dt_prev;  *dt_out = cfl / max;  *inv_max = 0
hipError_t launch_dt_finish(unsigned long long* inv_max, double cfl, double* dt_out, double* t_acc,
                            const double* dt_prev, hipStream_t st);

// Discrete adjoint of the single-phase Euler right-hand side (fv_adjoint.hip).
struct AdjointArgs {
    int nx, ny, nz;
    long long ncell;
    int bc[6];
    Material<double> mat;
    double weps;
    double idx, idy, idz;
};
// Ubar = (dR/dU)^T Rbar (overwritten), FP64
hipError_t launch_rhs_adjoint(const AdjointArgs& a, const double* U, const double* Rbar, double* Ubar, hipStream_t st);
// out = c0 x0 + c1 x1 + c2 x2 + c3 x3 over n values (null x1..x3 skipped; out may alias)
hipError_t launch_lincomb(double* out, long long n, double c0, const double* x0, double c1, const double* x1, double c2,
                          const double* x2, double c3, const double* x3, hipStream_t st);

}  // namespace fv
