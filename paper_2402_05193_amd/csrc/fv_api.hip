// fv_api.hip -- the C ABI declared in include/fvrk3.h: validation, launch
// geometry, workspace layout and error reporting.  No device allocation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/fvrk3.h"
#include "fv_kernels.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(FV_EHIP, "%s: %s", where, hipGetErrorString(e));
}

int ncomp_of(int model) { return model == FV_DIM ? 7 : 5; }

size_t state_bytes(const fv_config* c)
{
    const size_t es = c->dtype == FV_F64 ? 8 : 4;
    return es * (size_t)ncomp_of(c->model) * (size_t)c->nx * (size_t)c->ny * (size_t)c->nz;
}

// workgroups a stage launch aims at (tile columns x z chunks), FP64 and FP32 (its
// kernels hold fewer registers, more workgroups fit a CU).  Measured at 256^3 (NS,
// stage ms): FP64 512 / 1024 / 2048 / 4096 workgroups 2.58 / 2.54 / 2.51 / 2.53;
// FP32 (three waves per SIMD) 3072 / 4096 / 6144 / 8192 workgroups 1.41 / 1.36 /
// 1.36 / 1.36, the Euler and five-equation stages alike within 1 %.
#ifndef FV_TARGET_WORKGROUPS
#define FV_TARGET_WORKGROUPS 2048
#endif
#ifndef FV_TARGET_WORKGROUPS_F32
#define FV_TARGET_WORKGROUPS_F32 4096
#endif
// z chunk of a workgroup (planes): at least FV_MIN_ZCHUNK, unless the launch would then
// have fewer workgroups than the GPU holds at once (2 FP64 or 3 FP32 stage workgroups
// on each of the 256 CUs); then halved down to FV_SMALLEST_ZCHUNK.  Each chunk repeats
// the z-march's start (window loads, two z-only steps; two in-plane warm-up planes for
// the viscous model), which costs more than idle CUs only once they are all busy.
// Measured per stage (ms; chunk 16 / 8 / 4): NS FP64 128^3 0.318 / 0.332 / 0.355,
// 64^3 0.225 / 0.122 / 0.075; five-equation FP32 256x64x64 0.222 / 0.143 / 0.139,
// 128x32x32 0.222 / 0.115 / 0.064; Euler FP32 64^3 0.133 / 0.072 / 0.044.
#ifndef FV_MIN_ZCHUNK
#define FV_MIN_ZCHUNK 16
#endif
#ifndef FV_SMALLEST_ZCHUNK
#define FV_SMALLEST_ZCHUNK 4
#endif
// Five-equation model, single-problem launches: chunks lengthened (never shortened) up to
// FV_DIM_MAX_ZCHUNK planes while the launch still gives every resident workgroup slot a
// workgroup (one round), which saves repeated march starts.  Batched members keep the
// base chunks: with the lengthening the batched serving stream measured 1.5 % lower
// throughput (40.2 against 40.8 requests/s), one-at-a-time solves equal.  Measured at 256x128x128 (ms per stage): FP64 with
// 32-plane chunks (512 workgroups) 0.834 -> 0.814, characteristic 0.981 -> 0.964,
// TENO6-A 1.417 -> 1.407, THINC 1.268 -> 1.244; FP32 with 22-plane chunks (768) 0.496 ->
// 0.482, THINC 0.575 -> 0.562.  (NS 256^3 FP64 measured slower with longer chunks.)
#ifndef FV_DIM_MAX_ZCHUNK
#define FV_DIM_MAX_ZCHUNK 32
#endif
constexpr int RESIDENT_CUS = 256;

constexpr size_t SCALAR_BYTES = 256;  // dt, inverse-dt max, time accumulator, check words

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool visc6(const fv_config* c) { return c->model == FV_NS && c->visc_order == 6; }

long long padded_cells(const fv_config* c) { return (long long)(c->nx + 6) * (c->ny + 6) * (c->nz + 6); }

// workspace of the sixth-order viscous passes: q [4][npad], gradient [9][npad], divergence [4][ncell]
size_t visc6_bytes(const fv_config* c)
{
    if (!visc6(c)) return 0;
    const size_t es = c->dtype == FV_F64 ? 8 : 4;
    const size_t np = (size_t)padded_cells(c), n = (size_t)c->nx * c->ny * c->nz;
    return align256(4 * np * es) + align256(9 * np * es) + align256(4 * n * es);
}

int validate(const fv_config* c)
{
    if (!c) return fail(FV_ENULL, "cfg is NULL");
    if (c->abi_version != FV_ABI_VERSION) return fail(FV_EINVAL, "abi_version %d != %d", c->abi_version, FV_ABI_VERSION);
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(FV_EINVAL, "grid %d x %d x %d must be >= 1", c->nx, c->ny, c->nz);
    if ((long long)c->nx * c->ny * c->nz > (1ll << 40)) return fail(FV_EINVAL, "grid too large");
    if (c->model < FV_EULER || c->model > FV_DIM) return fail(FV_EINVAL, "model %d unknown", c->model);
    if (c->dtype != FV_F64 && c->dtype != FV_F32) return fail(FV_EINVAL, "dtype %d unknown", c->dtype);
    if (c->recon != 0 && c->recon != 1) return fail(FV_EINVAL, "recon must be 0 or 1");
    if (c->scheme != 0 && c->scheme != 1) return fail(FV_EINVAL, "scheme must be 0 (WENO5-Z) or 1 (TENO6-A)");
    if (c->visc_law < 0 || c->visc_law > 2) return fail(FV_EINVAL, "visc_law %d unknown", c->visc_law);
    if (c->visc_law != 0) {
        if (c->model != FV_NS) return fail(FV_EINVAL, "viscosity laws apply to the viscous model");
        if (!(c->T_ref > 0)) return fail(FV_EINVAL, "T_ref must be > 0");
        if (!(c->sutherland >= 0)) return fail(FV_EINVAL, "sutherland must be >= 0");
    }
    if (!(c->gas_R >= 0)) return fail(FV_EINVAL, "gas_R must be >= 0");
    if (c->visc_order != 0 && c->visc_order != 4 && c->visc_order != 6)
        return fail(FV_EINVAL, "visc_order must be 0, 4 or 6");
    if (c->visc_order == 6 && c->model != FV_NS) return fail(FV_EINVAL, "visc_order 6 applies to the viscous model");
    if (c->thinc != 0 && c->thinc != 1) return fail(FV_EINVAL, "thinc must be 0 or 1");
    if (c->thinc && c->model != FV_DIM) return fail(FV_EINVAL, "thinc applies to the five-equation model");
    const int n3[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; a++) {
        for (int s = 0; s < 2; s++) {
            const int b = c->bc[2 * a + s];
            if (b < FV_PERIODIC || b > FV_SYMMETRY) return fail(FV_EINVAL, "bc[%d] = %d unknown", 2 * a + s, b);
            if (b == FV_SYMMETRY && n3[a] < 3) return fail(FV_EINVAL, "symmetry on axis %d needs >= 3 cells", a);
        }
        if ((c->bc[2 * a] == FV_PERIODIC) != (c->bc[2 * a + 1] == FV_PERIODIC))
            return fail(FV_EINVAL, "periodic must be set on both faces of axis %d", a);
    }
    if (!(c->dx > 0) || !(c->dy > 0) || !(c->dz > 0)) return fail(FV_EINVAL, "cell sizes must be > 0");
    if (!(c->gamma1 > 1)) return fail(FV_EINVAL, "gamma1 must be > 1");
    if (c->model == FV_DIM && !(c->gamma2 > 1)) return fail(FV_EINVAL, "gamma2 must be > 1");
    if (c->model == FV_NS && (!(c->mu >= 0) || !(c->prandtl > 0))) return fail(FV_EINVAL, "mu >= 0 and prandtl > 0 required");
    if (c->positivity < -1 || c->positivity > 1) return fail(FV_EINVAL, "positivity must be -1, 0 or 1");
    if (c->eps_rho < 0 || c->eps_rhoc2 < 0 || c->eps_alpha < 0 || c->weno_eps < 0)
        return fail(FV_EINVAL, "tolerances must be >= 0");
    return FV_OK;
}

int check_ptr(const void* p, const char* name)
{
    if (!p) return fail(FV_ENULL, "%s is NULL", name);
    if ((uintptr_t)p % 16) return fail(FV_EALIGN, "%s is not 16-byte aligned", name);
    return FV_OK;
}

template <typename Real>
fv::Material<Real> material(const fv_config* c)
{
    fv::Material<Real> m;
    const double g1 = c->gamma1, g2 = c->model == FV_DIM ? c->gamma2 : c->gamma1;
    const double p1 = c->pinf1, p2 = c->model == FV_DIM ? c->pinf2 : c->pinf1;
    m.gamma = (Real)g1;
    m.pinf = (Real)p1;
    m.gm1 = (Real)(g1 - 1.0);
    m.gpinf = (Real)(g1 * p1);
    m.iG1 = (Real)(1.0 / (g1 - 1.0));
    m.PI1 = (Real)(g1 * p1 / (g1 - 1.0));
    m.iG2 = (Real)(1.0 / (g2 - 1.0));
    m.PI2 = (Real)(g2 * p2 / (g2 - 1.0));
    return m;
}

template <typename Real>
fv::ViscLaw<Real> visc_law(const fv_config* c)
{
    fv::ViscLaw<Real> v;
    const bool ns = c->model == FV_NS;
    const double R = c->gas_R > 0 ? c->gas_R : 1.0;
    v.law = ns ? c->visc_law : 0;
    v.mu = (Real)(ns ? c->mu : 0.0);
    v.kfac = (Real)(ns ? c->gamma1 / ((c->gamma1 - 1.0) * c->prandtl) : 0.0);
    v.inv_th_ref = (Real)(v.law ? 1.0 / (R * c->T_ref) : 0.0);
    v.th_c = (Real)(R * c->sutherland);
    v.th_ref_c = (Real)(R * (c->T_ref + c->sutherland));
    return v;
}

fv::AuxArgs aux_args(const fv_config* c)
{
    fv::AuxArgs a;
    a.model = c->model;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.ncell = (long long)c->nx * c->ny * c->nz;
    a.dx = c->dx;
    a.dy = c->dy;
    a.dz = c->dz;
    a.matd = material<double>(c);
    a.matf = material<float>(c);
    a.vl = visc_law<double>(c);
    return a;
}

bool positivity_on(const fv_config* c)
{
    return c->positivity < 0 ? c->model == FV_DIM : c->positivity == 1;
}

// solo: a single-problem launch (the five-equation chunk lengthening below applies;
// batched members keep the base chunks, which interleave better with the other members)
template <typename Real>
fv::StageArgs<Real> stage_args(const fv_config* c, fv::LaunchGeom& g, bool solo = false)
{
    fv::StageArgs<Real> a;
    memset(&a, 0, sizeof a);
    const bool f64 = c->dtype == FV_F64;
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.ncell = (long long)c->nx * c->ny * c->nz;
    for (int k = 0; k < 6; k++) a.bc[k] = c->bc[k];
    a.tiles_x = (c->nx + TILE_BX - 1) / TILE_BX;
    a.tiles_y = (c->ny + TILE_BY - 1) / TILE_BY;
    // z chunks: enough workgroups to fill 256 CUs several times over
    const long long tiles = (long long)a.tiles_x * a.tiles_y;
    const long long target = f64 ? FV_TARGET_WORKGROUPS : FV_TARGET_WORKGROUPS_F32;
    int nch = (int)((target + tiles - 1) / tiles);
    if (nch < 1) nch = 1;
    int zc = (c->nz + nch - 1) / nch;
    if (zc < FV_MIN_ZCHUNK) {
        zc = FV_MIN_ZCHUNK < c->nz ? FV_MIN_ZCHUNK : c->nz;
        const long long slots = (long long)RESIDENT_CUS * (f64 ? 2 : 3);
        while (zc / 2 >= FV_SMALLEST_ZCHUNK && tiles * ((c->nz + zc - 1) / zc) < slots) zc /= 2;
    }
    if (solo && c->model == FV_DIM) {
        const long long slots = (long long)RESIDENT_CUS * (f64 ? 2 : 3);
        const long long round_chunks = (slots + tiles - 1) / tiles;
        int zl = (int)((c->nz + round_chunks - 1) / round_chunks);
        if (zl > FV_DIM_MAX_ZCHUNK) zl = FV_DIM_MAX_ZCHUNK;
        if (zl > zc && tiles * ((c->nz + zl - 1) / zl) >= slots) zc = zl;
    }
    a.zchunk = zc;
    a.nchunks = (c->nz + zc - 1) / zc;
    g.nblocks = (int)(tiles * a.nchunks);
    a.positivity = positivity_on(c) ? 1 : 0;
    a.recon = c->recon + 2 * c->scheme;  // REC_* variant
    a.thinc = c->model == FV_DIM ? c->thinc : 0;
    a.ndim = (c->nx > 1) + (c->ny > 1) + (c->nz > 1);
    a.mat = material<Real>(c);
    a.tol.eps_rho = (Real)(c->eps_rho > 0 ? c->eps_rho : (f64 ? 1e-12 : 1e-10));
    a.tol.eps_rhoc2 = (Real)(c->eps_rhoc2 > 0 ? c->eps_rhoc2 : (f64 ? 1e-10 : 1e-8));
    a.tol.eps_alpha = (Real)(c->eps_alpha > 0 ? c->eps_alpha : (f64 ? 1e-12 : 1e-10));
    a.weno_eps = (Real)(c->weno_eps > 0 ? c->weno_eps : (f64 ? 1e-40 : 1e-30));
    a.idx = (Real)(1.0 / c->dx);
    a.idy = (Real)(1.0 / c->dy);
    a.idz = (Real)(1.0 / c->dz);
    a.inv12dx = (Real)(1.0 / (12.0 * c->dx));
    a.inv12dy = (Real)(1.0 / (12.0 * c->dy));
    a.inv12dz = (Real)(1.0 / (12.0 * c->dz));
    a.inv24dx = (Real)(1.0 / (24.0 * c->dx));
    a.inv24dy = (Real)(1.0 / (24.0 * c->dy));
    a.inv24dz = (Real)(1.0 / (24.0 * c->dz));
    a.mu = (Real)(c->model == FV_NS ? c->mu : 0.0);
    const double hmin = fmin(c->dx, fmin(c->dy, c->dz));
    a.kvisc = c->model == FV_NS ? (14.0 / 3.0) * c->mu / (hmin * hmin) : 0.0;
    a.kvisc_h = (14.0 / 3.0) / (hmin * hmin);
    a.vl = visc_law<Real>(c);
    a.inv_max = nullptr;
    a.kappa = (Real)(c->model == FV_NS ? c->mu * c->gamma1 / ((c->gamma1 - 1.0) * c->prandtl) : 0.0);
    return a;
}

struct WsLayout {
    char* A;
    char* B;
    double* dt;
    unsigned long long* inv_max;
    double* t_acc;
    long long* check;
    char* vq;  // sixth-order viscous passes (null otherwise)
    char* vg;
    char* vr;
};

WsLayout ws_layout(const fv_config* c, void* ws)
{
    WsLayout w;
    const size_t sb = (state_bytes(c) + 255) & ~(size_t)255;
    w.A = (char*)ws;
    w.B = w.A + sb;
    char* sc = w.B + sb;
    w.dt = (double*)sc;
    w.inv_max = (unsigned long long*)(sc + 8);
    w.t_acc = (double*)(sc + 16);
    w.check = (long long*)(sc + 32);
    w.vq = w.vg = w.vr = nullptr;
    if (visc6(c)) {
        const size_t es = c->dtype == FV_F64 ? 8 : 4;
        const size_t np = (size_t)padded_cells(c);
        w.vq = sc + SCALAR_BYTES;
        w.vg = w.vq + align256(4 * np * es);
        w.vr = w.vg + align256(9 * np * es);
    }
    return w;
}

// bytes of the limiter decision record: one per face, x faces then y then z
void flag_offsets(const fv_config* c, long long off[3], long long* total)
{
    const long long nx = c->nx, ny = c->ny, nz = c->nz;
    off[0] = 0;
    off[1] = (nx + 1) * ny * nz;
    off[2] = off[1] + nx * (ny + 1) * nz;
    *total = off[2] + nx * ny * (nz + 1);
}

template <typename Real>
int stage_impl(const fv_config* c, int mode, const void* Un, const void* Uk, void* out, double dt, const double* dt_dev,
               hipStream_t st, unsigned long long* inv_max, const WsLayout* w, unsigned char* flags = nullptr)
{
    fv::LaunchGeom g;
    fv::StageArgs<Real> a = stage_args<Real>(c, g, true);
    if (flags) {
        long long total;
        flag_offsets(c, a.flag_off, &total);
        a.flags = flags;
    }
    if (visc6(c)) {
        if (!w) return fail(FV_EUNSUPPORTED, "sixth-order viscous fluxes need a workspace");
        fv::Visc6Args<Real> v;
        v.nx = c->nx;
        v.ny = c->ny;
        v.nz = c->nz;
        for (int k = 0; k < 6; k++) v.bc[k] = c->bc[k];
        v.ncell = (long long)c->nx * c->ny * c->nz;
        v.npad = padded_cells(c);
        v.mat = a.mat;
        v.vl = a.vl;
        v.ih[0] = (Real)(1.0 / c->dx);
        v.ih[1] = (Real)(1.0 / c->dy);
        v.ih[2] = (Real)(1.0 / c->dz);
        hipError_t e = fv::launch_visc6<Real>(v, (const Real*)Uk, (Real*)w->vq, (Real*)w->vg, (Real*)w->vr, st);
        if (e != hipSuccess) return hip_fail(e, "viscous passes");
        a.rvisc = (const Real*)w->vr;
    }
    a.inv_max = inv_max;
    a.Uk = (const Real*)Uk;
    a.Un = (const Real*)Un;
    a.out = (Real*)out;
    a.dt = dt;
    a.dt_dev = dt_dev;
    a.mode = mode;
    hipError_t e = fv::launch_stage<Real>(c->model, a, g, st);
    if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
    return FV_OK;
}

int stage_dispatch(const fv_config* c, int mode, const void* Un, const void* Uk, void* out, double dt,
                   const double* dt_dev, hipStream_t st, unsigned long long* inv_max = nullptr,
                   const WsLayout* w = nullptr, unsigned char* flags = nullptr)
{
    if (c->dtype == FV_F64) return stage_impl<double>(c, mode, Un, Uk, out, dt, dt_dev, st, inv_max, w, flags);
    return stage_impl<float>(c, mode, Un, Uk, out, dt, dt_dev, st, inv_max, w, flags);
}

}  // namespace

extern "C" {

int32_t fv_ncomp(const fv_config* cfg)
{
    if (!cfg) return fail(FV_ENULL, "cfg is NULL");
    if (cfg->model < FV_EULER || cfg->model > FV_DIM) return fail(FV_EINVAL, "model unknown");
    return ncomp_of(cfg->model);
}

int workspace_bytes(const fv_config* cfg, size_t* out)
{
    int r = validate(cfg);
    if (r) return r;
    if (!out) return fail(FV_ENULL, "out is NULL");
    *out = 2 * ((state_bytes(cfg) + 255) & ~(size_t)255) + SCALAR_BYTES + visc6_bytes(cfg);
    return FV_OK;
}

int init_state(const fv_config* cfg, int32_t case_id, const double* params, int32_t nparams, uint64_t seed, void* U,
               void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U"))) return r;
    const int nc = ncomp_of(cfg->model);
    int need;
    switch (case_id) {
    case FV_CASE_UNIFORM: need = nc; break;
    case FV_CASE_TGV: need = 3; break;
    case FV_CASE_RIEMANN: need = 2 + 2 * nc; break;
    case FV_CASE_SBI: need = 12; break;
    case FV_CASE_GAUSS_WAVE: need = 3; break;
    case FV_CASE_ISENTROPIC_VORTEX: need = 5; break;
    default: return fail(FV_EINVAL, "case_id %d unknown", case_id);
    }
    if ((case_id == FV_CASE_TGV || case_id == FV_CASE_GAUSS_WAVE || case_id == FV_CASE_ISENTROPIC_VORTEX) &&
        cfg->model == FV_DIM)
        return fail(FV_EINVAL, "case %d is a single-phase case", case_id);
    if (case_id == FV_CASE_SBI && cfg->model != FV_DIM) return fail(FV_EINVAL, "SBI needs the DIM model");
    if (nparams < need) return fail(FV_EINVAL, "case %d needs %d parameters, got %d", case_id, need, nparams);
    if (!params) return fail(FV_ENULL, "params is NULL");
    if ((case_id == FV_CASE_RIEMANN || case_id == FV_CASE_GAUSS_WAVE) && (params[0] < 0 || params[0] > 2))
        return fail(FV_EINVAL, "axis must be 0, 1 or 2");
    const fv::AuxArgs a = aux_args(cfg);
    hipError_t e = cfg->dtype == FV_F64
                       ? fv::launch_init<double>(a, case_id, params, nparams, seed, (double*)U, (hipStream_t)stream)
                       : fv::launch_init<float>(a, case_id, params, nparams, seed, (float*)U, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "init_state");
    return FV_OK;
}

int prim_to_cons(const fv_config* cfg, const void* W, void* U, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(W, "W")) || (r = check_ptr(U, "U"))) return r;
    const fv::AuxArgs a = aux_args(cfg);
    hipError_t e = cfg->dtype == FV_F64 ? fv::launch_prim_to_cons<double>(a, (const double*)W, (double*)U, (hipStream_t)stream)
                                        : fv::launch_prim_to_cons<float>(a, (const float*)W, (float*)U, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "prim_to_cons");
    return FV_OK;
}

int cons_to_prim(const fv_config* cfg, const void* U, void* W, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(W, "W"))) return r;
    const fv::AuxArgs a = aux_args(cfg);
    hipError_t e = cfg->dtype == FV_F64 ? fv::launch_cons_to_prim<double>(a, (const double*)U, (double*)W, (hipStream_t)stream)
                                        : fv::launch_cons_to_prim<float>(a, (const float*)U, (float*)W, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cons_to_prim");
    return FV_OK;
}

int rhs(const fv_config* cfg, const void* U, void* R, double dt, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(R, "R"))) return r;
    if (U == R) return fail(FV_EINVAL, "U and R must not overlap");
    if (!(dt >= 0) || !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite and >= 0");
    if (visc6(cfg)) return fail(FV_EUNSUPPORTED, "visc_order 6 needs a workspace: call rhs_ws");
    return stage_dispatch(cfg, 0, U, U, R, dt, nullptr, (hipStream_t)stream);
}

int rhs_ws(const fv_config* cfg, const void* U, void* R, double dt, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(R, "R")) || (r = check_ptr(ws, "ws"))) return r;
    if (U == R) return fail(FV_EINVAL, "U and R must not overlap");
    if (!(dt >= 0) || !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite and >= 0");
    const WsLayout w = ws_layout(cfg, ws);
    return stage_dispatch(cfg, 0, U, U, R, dt, nullptr, (hipStream_t)stream, nullptr, &w);
}

int limiter_flag_bytes(const fv_config* cfg, size_t* out)
{
    int r = validate(cfg);
    if (r) return r;
    if (!out) return fail(FV_ENULL, "out is NULL");
    long long off[3], total;
    flag_offsets(cfg, off, &total);
    *out = (size_t)total;
    return FV_OK;
}

int stage_workgroups(const fv_config* cfg, int32_t* out)
{
    int r = validate(cfg);
    if (r) return r;
    if (!out) return fail(FV_ENULL, "out is NULL");
    fv::LaunchGeom g;
    if (cfg->dtype == FV_F64) (void)stage_args<double>(cfg, g);
    else (void)stage_args<float>(cfg, g);
    *out = g.nblocks;
    return FV_OK;
}

int rhs_flags(const fv_config* cfg, const void* U, void* R, double dt, uint8_t* flags, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(R, "R"))) return r;
    if (!flags) return fail(FV_ENULL, "flags is NULL");
    if (U == R) return fail(FV_EINVAL, "U and R must not overlap");
    if (!(dt >= 0) || !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite and >= 0");
    hipStream_t st = (hipStream_t)stream;
    WsLayout w;
    const WsLayout* wp = nullptr;
    if (visc6(cfg)) {
        if ((r = check_ptr(ws, "ws"))) return fail(r, "visc_order 6 needs a workspace");
        w = ws_layout(cfg, ws);
        wp = &w;
    }
    if (!positivity_on(cfg)) {
        // no limiter acts: every decision byte is 0
        long long off[3], total;
        flag_offsets(cfg, off, &total);
        hipError_t e = fv::launch_fill_u8(flags, total, 0, st);
        if (e != hipSuccess) return hip_fail(e, "rhs_flags: clear");
        return stage_dispatch(cfg, 0, U, U, R, dt, nullptr, st, nullptr, wp);
    }
    return stage_dispatch(cfg, 0, U, U, R, dt, nullptr, st, nullptr, wp, flags);
}

int rk3_stage(const fv_config* cfg, int32_t stage, const void* Un, const void* Uk, void* Uout, double dt,
              const double* dt_dev, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if (stage < 1 || stage > 3) return fail(FV_EINVAL, "stage must be 1, 2 or 3");
    if ((r = check_ptr(Un, "Un")) || (r = check_ptr(Uk, "Uk")) || (r = check_ptr(Uout, "Uout"))) return r;
    if (Uk == Uout) return fail(FV_EINVAL, "Uout must not overlap Uk");
    if (stage == 1 && Un != Uk) return fail(FV_EINVAL, "stage 1 needs Uk == Un");
    if (!dt_dev && (!(dt > 0) || !isfinite(dt))) return fail(FV_EINVAL, "dt must be finite and > 0");
    if (visc6(cfg)) return fail(FV_EUNSUPPORTED, "visc_order 6 needs a workspace: use rk3_stage3_cfl, rk3_step or advance");
    return stage_dispatch(cfg, stage, Un, Uk, Uout, dt, dt_dev, (hipStream_t)stream);
}

int rk3_stage3_cfl(const fv_config* cfg, const void* Un, const void* Uk, void* Uout, const double* dt_dev,
                   double* dt_next, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(Un, "Un")) || (r = check_ptr(Uk, "Uk")) || (r = check_ptr(Uout, "Uout")) ||
        (r = check_ptr(ws, "ws")))
        return r;
    if (!dt_dev || !dt_next) return fail(FV_ENULL, "dt_dev and dt_next are required");
    if (Uk == Uout) return fail(FV_EINVAL, "Uout must not overlap Uk");
    if (!(cfg->cfl > 0)) return fail(FV_EINVAL, "cfl must be > 0");
    hipStream_t st = (hipStream_t)stream;
    const WsLayout w = ws_layout(cfg, ws);
    hipError_t e = fv::launch_reset_max(w.inv_max, st);
    if (e != hipSuccess) return hip_fail(e, "rk3_stage3_cfl: reset");
    if ((r = stage_dispatch(cfg, 3, Un, Uk, Uout, 0.0, dt_dev, st, w.inv_max, &w))) return r;
    e = fv::launch_dt_finish(w.inv_max, cfg->cfl, dt_next, nullptr, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "rk3_stage3_cfl: finish");
    return FV_OK;
}

static int step_impl(const fv_config* cfg, void* U, double dt, const double* dt_dev, const WsLayout& w, hipStream_t st,
                     unsigned long long* inv_max = nullptr)
{
    int r;
    if ((r = stage_dispatch(cfg, 1, U, U, w.A, dt, dt_dev, st, nullptr, &w))) return r;
    if ((r = stage_dispatch(cfg, 2, U, w.A, w.B, dt, dt_dev, st, nullptr, &w))) return r;
    return stage_dispatch(cfg, 3, U, w.B, U, dt, dt_dev, st, inv_max, &w);
}

int rk3_step(const fv_config* cfg, void* U, double dt, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(ws, "ws"))) return r;
    if (!(dt > 0) || !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite and > 0");
    return step_impl(cfg, U, dt, nullptr, ws_layout(cfg, ws), (hipStream_t)stream);
}

int compute_dt(const fv_config* cfg, const void* U, double* dt_dev, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(ws, "ws"))) return r;
    if (!dt_dev) return fail(FV_ENULL, "dt_dev is NULL");
    if (!(cfg->cfl > 0)) return fail(FV_EINVAL, "cfl must be > 0");
    const WsLayout w = ws_layout(cfg, ws);
    const fv::AuxArgs a = aux_args(cfg);
    const double mu = cfg->model == FV_NS ? cfg->mu : 0.0;
    hipError_t e = cfg->dtype == FV_F64
                       ? fv::launch_dt<double>(a, (const double*)U, mu, cfg->cfl, w.inv_max, dt_dev, nullptr, (hipStream_t)stream)
                       : fv::launch_dt<float>(a, (const float*)U, mu, cfg->cfl, w.inv_max, dt_dev, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "compute_dt");
    return FV_OK;
}

// advance with a validated configuration and workspace (advance, advance_noalloc)
static int advance_impl(const fv_config* cfg, void* U, int32_t nsteps, double dt, double* t_inout, void* ws,
                        hipStream_t st)
{
    int r;
    const bool cfl_mode = !(dt > 0);
    const WsLayout w = ws_layout(cfg, ws);
    const fv::AuxArgs a = aux_args(cfg);
    const double mu = cfg->model == FV_NS ? cfg->mu : 0.0;
    if (cfl_mode && t_inout) {
        hipError_t e = hipMemcpyAsync(w.t_acc, t_inout, sizeof(double), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "advance: t upload");
    }
    if (cfl_mode && nsteps > 0) {
        // dt of the first step from a full reduction; every later dt comes from the
        // reduction fused into the previous step's third stage
        hipError_t e = cfg->dtype == FV_F64
                           ? fv::launch_dt<double>(a, (const double*)U, mu, cfg->cfl, w.inv_max, w.dt, nullptr, st)
                           : fv::launch_dt<float>(a, (const float*)U, mu, cfg->cfl, w.inv_max, w.dt, nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "advance: dt");
    }
    for (int n = 0; n < nsteps; n++) {
        if (cfl_mode) {
            if ((r = step_impl(cfg, U, 0.0, w.dt, w, st, w.inv_max))) return r;
            hipError_t e = fv::launch_dt_finish(w.inv_max, cfg->cfl, w.dt, t_inout ? w.t_acc : nullptr, w.dt, st);
            if (e != hipSuccess) return hip_fail(e, "advance: dt finish");
        } else {
            if ((r = step_impl(cfg, U, dt, nullptr, w, st))) return r;
        }
    }
    if (t_inout) {
        if (cfl_mode) {
            hipError_t e = hipMemcpyAsync(t_inout, w.t_acc, sizeof(double), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "advance: t read-back");
        } else {
            *t_inout += dt * nsteps;
        }
    }
    return FV_OK;
}

int advance(const fv_config* cfg, void* U, int32_t nsteps, double dt, double* t_inout, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(ws, "ws"))) return r;
    if (nsteps < 0) return fail(FV_EINVAL, "nsteps must be >= 0");
    const bool cfl_mode = !(dt > 0);
    if (cfl_mode && !(cfg->cfl > 0)) return fail(FV_EINVAL, "cfl must be > 0 when dt <= 0");
    if (!cfl_mode && !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite");
    return advance_impl(cfg, U, nsteps, dt, t_inout, ws, (hipStream_t)stream);
}

}  // extern "C"

// The workspace of advance_noalloc: one fixed array per device, resident while the
// process lives.  Host code uses its device address from hipGetSymbolAddress (the
// array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[FV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of the current device's scratch array, looked up once per device
int scratch_of_current_device(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "advance_noalloc: hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(FV_EUNSUPPORTED, "device index %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "advance_noalloc: hipGetSymbolAddress");
        if (!ptr || (uintptr_t)ptr % 256) return fail(FV_EHIP, "advance_noalloc: scratch address not usable");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FV_OK;
}

}  // namespace

extern "C" {

int advance_noalloc(const fv_config* cfg, void* U, int32_t nsteps, double dt, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U"))) return r;
    if (nsteps < 0) return fail(FV_EINVAL, "nsteps must be >= 0");
    const bool cfl_mode = !(dt > 0);
    if (cfl_mode && !(cfg->cfl > 0)) return fail(FV_EINVAL, "cfl must be > 0 when dt <= 0");
    if (!cfl_mode && !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite");
    size_t need = 0;
    if ((r = workspace_bytes(cfg, &need))) return r;
    if (need > (size_t)FV_NOALLOC_SCRATCH_BYTES)
        return fail(FV_EINVAL, "advance_noalloc: the problem needs %zu bytes of workspace, more than the %zu of the "
                               "fixed scratch array (use advance with a caller workspace)",
                    need, (size_t)FV_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if ((r = scratch_of_current_device(&ws))) return r;
    return advance_impl(cfg, U, nsteps, dt, nullptr, ws, (hipStream_t)stream);
}

static int adjoint_supported(const fv_config* cfg)
{
    if (cfg->model != FV_EULER) return fail(FV_EUNSUPPORTED, "the adjoint covers the single-phase Euler model");
    if (cfg->dtype != FV_F64) return fail(FV_EUNSUPPORTED, "the adjoint is FP64");
    if (positivity_on(cfg)) return fail(FV_EUNSUPPORTED, "the adjoint needs the positivity limiters off");
    if (cfg->recon != 0) return fail(FV_EUNSUPPORTED, "the adjoint covers primitive-variable reconstruction");
    if (cfg->scheme != 0) return fail(FV_EUNSUPPORTED, "the adjoint covers WENO5-Z reconstruction");
    return FV_OK;
}

static fv::AdjointArgs adjoint_args(const fv_config* c)
{
    fv::AdjointArgs a;
    memset(&a, 0, sizeof a);
    a.nx = c->nx;
    a.ny = c->ny;
    a.nz = c->nz;
    a.ncell = (long long)c->nx * c->ny * c->nz;
    for (int k = 0; k < 6; k++) a.bc[k] = c->bc[k];
    a.mat = material<double>(c);
    a.weps = c->weno_eps > 0 ? c->weno_eps : 1e-40;
    a.idx = 1.0 / c->dx;
    a.idy = 1.0 / c->dy;
    a.idz = 1.0 / c->dz;
    return a;
}

int rhs_adjoint(const fv_config* cfg, const void* U, const void* Rbar, void* Ubar, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = adjoint_supported(cfg))) return r;
    (void)ws;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(Rbar, "Rbar")) || (r = check_ptr(Ubar, "Ubar"))) return r;
    if (Ubar == U || Ubar == Rbar) return fail(FV_EINVAL, "Ubar must not overlap U or Rbar");
    hipError_t e = fv::launch_rhs_adjoint(adjoint_args(cfg), (const double*)U, (const double*)Rbar, (double*)Ubar,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rhs_adjoint");
    return FV_OK;
}

int adjoint_workspace_bytes(const fv_config* cfg, size_t* out)
{
    int r = validate(cfg);
    if (r) return r;
    if (!out) return fail(FV_ENULL, "out is NULL");
    *out = 5 * ((state_bytes(cfg) + 255) & ~(size_t)255);
    return FV_OK;
}

}  // extern "C"

// Reverse sweep of one TVD-RK3 step from its stage states U1, U2 (Sec. 3.4):
// U1 = Un + dt R(Un); U2 = 3/4 Un + 1/4 U1 + 1/4 dt R(U1); U3 = 1/3 Un + 2/3 U2 + 2/3 dt R(U2).
// On entry Ubar holds the cotangent of U3, on return that of Un.  aws holds G2, G1 and T
// at state slots 2, 3 and 4 (slots 0 and 1 are free for the caller's stage states).
static int step_adjoint_sweep(const fv_config* cfg, const void* Un, const void* U1p, const void* U2p, void* Ubar,
                              double dt, void* aws, hipStream_t st)
{
    const size_t sb = (state_bytes(cfg) + 255) & ~(size_t)255;
    const double* U1 = (const double*)U1p;
    const double* U2 = (const double*)U2p;
    double* G2 = (double*)((char*)aws + 2 * sb);
    double* G1 = (double*)((char*)aws + 3 * sb);
    double* T = (double*)((char*)aws + 4 * sb);
    double* G3 = (double*)Ubar;
    const long long n = 5ll * cfg->nx * cfg->ny * cfg->nz;
    const fv::AdjointArgs a = adjoint_args(cfg);
    hipError_t e = fv::launch_rhs_adjoint(a, U2, G3, T, st);
    if (e == hipSuccess) e = fv::launch_lincomb(G2, n, 2.0 / 3.0, G3, 2.0 / 3.0 * dt, T, 0, nullptr, 0, nullptr, st);
    if (e == hipSuccess) e = fv::launch_rhs_adjoint(a, U1, G2, T, st);
    if (e == hipSuccess) e = fv::launch_lincomb(G1, n, 0.25, G2, 0.25 * dt, T, 0, nullptr, 0, nullptr, st);
    if (e == hipSuccess) e = fv::launch_rhs_adjoint(a, (const double*)Un, G1, T, st);
    if (e == hipSuccess) e = fv::launch_lincomb(G3, n, 1.0 / 3.0, G3, 0.75, G2, 1.0, G1, dt, T, st);
    if (e != hipSuccess) return hip_fail(e, "rk3_step_adjoint");
    return FV_OK;
}

extern "C" {

int rk3_step_adjoint(const fv_config* cfg, const void* Un, void* Ubar, double dt, void* aws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = adjoint_supported(cfg))) return r;
    if ((r = check_ptr(Un, "Un")) || (r = check_ptr(Ubar, "Ubar")) || (r = check_ptr(aws, "aws"))) return r;
    if (!(dt > 0) || !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite and > 0");
    hipStream_t st = (hipStream_t)stream;
    const size_t sb = (state_bytes(cfg) + 255) & ~(size_t)255;
    void* U1 = aws;
    void* U2 = (char*)aws + sb;
    // the stages of the forward step, recomputed from U^n
    if ((r = stage_dispatch(cfg, 1, Un, Un, U1, dt, nullptr, st))) return r;
    if ((r = stage_dispatch(cfg, 2, Un, U1, U2, dt, nullptr, st))) return r;
    return step_adjoint_sweep(cfg, Un, U1, U2, Ubar, dt, aws, st);
}

int rk3_step_adjoint_stages(const fv_config* cfg, const void* Un, const void* U1, const void* U2, void* Ubar,
                            double dt, void* aws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = adjoint_supported(cfg))) return r;
    if ((r = check_ptr(Un, "Un")) || (r = check_ptr(U1, "U1")) || (r = check_ptr(U2, "U2")) ||
        (r = check_ptr(Ubar, "Ubar")) || (r = check_ptr(aws, "aws")))
        return r;
    if (Ubar == Un || Ubar == U1 || Ubar == U2) return fail(FV_EINVAL, "Ubar must not overlap Un, U1 or U2");
    if (!(dt > 0) || !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite and > 0");
    return step_adjoint_sweep(cfg, Un, U1, U2, Ubar, dt, aws, (hipStream_t)stream);
}

int check_state(const fv_config* cfg, const void* U, void* ws, fv_report* out, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(ws, "ws"))) return r;
    if (!out) return fail(FV_ENULL, "out is NULL");
    hipStream_t st = (hipStream_t)stream;
    const WsLayout w = ws_layout(cfg, ws);
    const fv::AuxArgs a = aux_args(cfg);
    hipError_t e = cfg->dtype == FV_F64 ? fv::launch_check<double>(a, (const double*)U, w.check, st)
                                        : fv::launch_check<float>(a, (const float*)U, w.check, st);
    long long h[3];
    if (e == hipSuccess) e = hipMemcpyAsync(h, w.check, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "check_state");
    out->first_bad_cell = h[1] ? h[0] : -1;
    out->bad_count_clamped = h[1] > 0x7fffffffll ? 0x7fffffff : (int32_t)h[1];
    out->status = h[2] == 2 ? FV_ENONFINITE : (h[2] == 1 ? FV_EINADMISSIBLE : FV_OK);
    if (out->status != FV_OK)
        fail(out->status, "check_state: %lld bad cells, first at %lld", (long long)h[1], (long long)h[0]);
    return out->status;
}

const char* last_error(void) { return g_err; }

}  // extern "C"

// ------------------------------------------------------------------ batches
// A batch is a set of independent problems advanced together: every RK stage
// is one launch per (model, precision, limiter) group whose workgroups are
// spread over the group's problems through a device table.
//
// Table layout (device, caller-owned), for a batch of capacity C: one region per
// group present, in the order of the group id (model, precision, limiter), each
//   [header: int count][int first[C+1]][StageArgs args[C] for stage 1][.. stage 2][.. stage 3]
// then [header: int n][BatchScalars scal[C]].  The kernels read the counts from the
// table, so a captured step serves any membership with the same groups and grid
// sizes: graphs are cached by (groups, bucketed grid sizes, steps, stream) and
// replayed after later batch_set calls.

namespace {

// group of a member: model x precision x limiter setting x reconstruction family x
// variant (a viscosity law for NS, THINC for the five-equation model)
constexpr int MAX_GROUP_IDS = 3 * 2 * 2 * 4 * 2;
constexpr int MAX_GROUPS = 16;  // groups present in one batch (table regions)
constexpr size_t TAB_ALIGN = 256;
constexpr int MAX_GRAPHS = 16;   // cached step graphs per batch

size_t align_up(size_t v) { return (v + TAB_ALIGN - 1) & ~(TAB_ALIGN - 1); }

struct BatchGroup {
    int gid, model, dtype, pos, rec, variant, count, nblocks;
    size_t hdr_off, first_off, args_off[3];  // byte offsets in the device table
    // a group of one member runs the single-problem stage kernel with these arguments
    // (the same body: the same results, without the table indirection)
    fv::StageArgs<double> solo_d[3];
    fv::StageArgs<float> solo_f[3];
};

struct GraphEntry {
    std::vector<long long> key;  // (group id, bucketed grid) per group, then steps
    hipStream_t stream;
    hipGraphExec_t exec;
    unsigned long long last_use;
};

size_t args_bytes(int capacity) { return align_up((size_t)capacity * sizeof(fv::StageArgs<double>)); }

size_t region_bytes(int capacity)
{
    return TAB_ALIGN + align_up(sizeof(int) * (size_t)(capacity + 1)) + 3 * args_bytes(capacity);
}

size_t table_bound(int capacity)
{
    return (size_t)MAX_GROUPS * region_bytes(capacity) + TAB_ALIGN +
           align_up(sizeof(fv::BatchScalars) * (size_t)capacity);
}

// grid of a captured stage launch: the group's workgroups rounded up to a multiple of
// an eighth of their power-of-two floor (at most 12.5 % spare workgroups, which
// return at once), so that memberships of similar size share a graph
int grid_bucket(int nb)
{
    if (nb <= 8) return nb;
    int q = 1;
    while (q * 2 <= nb) q *= 2;
    const int step = q / 8;
    return (nb + step - 1) / step * step;
}

}  // namespace

struct fv_batch {
    int capacity = 0;
    char* table = nullptr;  // device, caller-owned
    size_t table_bytes = 0;
    char* host[2] = {nullptr, nullptr};  // pinned staging of the table image
    hipEvent_t copied[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    int cur = 0;
    int n = 0;
    std::vector<BatchGroup> groups;
    size_t scal_hdr_off = 0, scal_off = 0;
    std::vector<GraphEntry> graphs;
    unsigned long long uses = 0;
};

namespace {

template <typename Real>
void fill_group_args(const fv_config* c, void* U, void* ws, char* img, const BatchGroup& g, int k, int first_block,
                     int* nblocks)
{
    fv::LaunchGeom geo;
    fv::StageArgs<Real> a = stage_args<Real>(c, geo);
    const WsLayout w = ws_layout(c, ws);
    a.dt_dev = w.dt;
    a.dt = 0.0;
    fv::StageArgs<Real>* st = nullptr;
    for (int s = 0; s < 3; s++) {
        fv::StageArgs<Real> b = a;
        b.mode = s + 1;
        b.Un = (const Real*)U;
        b.Uk = (const Real*)(s == 0 ? U : s == 1 ? (void*)w.A : (void*)w.B);
        b.out = (Real*)(s == 0 ? (void*)w.A : s == 1 ? (void*)w.B : U);
        b.inv_max = s == 2 ? w.inv_max : nullptr;
        st = reinterpret_cast<fv::StageArgs<Real>*>(img + g.args_off[s]);
        st[k] = b;
    }
    reinterpret_cast<int*>(img + g.first_off)[k] = first_block;
    *nblocks = geo.nblocks;
}

int batch_launch_steps(fv_batch* b, int nsteps, hipStream_t st, bool bucketed)
{
    const fv::BatchScalars* scal = reinterpret_cast<const fv::BatchScalars*>(b->table + b->scal_off);
    const int* nmem = reinterpret_cast<const int*>(b->table + b->scal_hdr_off);
    for (int k = 0; k < nsteps; k++) {
        for (int s = 0; s < 3; s++) {
            for (const BatchGroup& g : b->groups) {
                if (!bucketed && g.count == 1) {
                    fv::LaunchGeom geo;
                    geo.nblocks = g.nblocks;
                    hipError_t e = g.dtype == FV_F64 ? fv::launch_stage<double>(g.model, g.solo_d[s], geo, st)
                                                     : fv::launch_stage<float>(g.model, g.solo_f[s], geo, st);
                    if (e != hipSuccess) return hip_fail(e, "batch stage launch (single member)");
                    continue;
                }
                const int* first = reinterpret_cast<const int*>(b->table + g.first_off);
                const int* count = reinterpret_cast<const int*>(b->table + g.hdr_off);
                const int nb = bucketed ? grid_bucket(g.nblocks) : g.nblocks;
                hipError_t e =
                    g.dtype == FV_F64
                        ? fv::launch_batch_stage<double>(g.model, g.rec, g.pos != 0, g.variant,
                                                         reinterpret_cast<const fv::StageArgs<double>*>(b->table + g.args_off[s]),
                                                         first, count, nb, st)
                        : fv::launch_batch_stage<float>(g.model, g.rec, g.pos != 0, g.variant,
                                                        reinterpret_cast<const fv::StageArgs<float>*>(b->table + g.args_off[s]),
                                                        first, count, nb, st);
                if (e != hipSuccess) return hip_fail(e, "batch stage launch");
            }
        }
        hipError_t e = fv::launch_batch_dt_finish(scal, nmem, bucketed ? b->capacity : b->n, st);
        if (e != hipSuccess) return hip_fail(e, "batch dt finish");
    }
    return FV_OK;
}

void drop_graphs(fv_batch* b)
{
    for (GraphEntry& g : b->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

}  // namespace

extern "C" {

int batch_table_bytes(int32_t capacity, size_t* out)
{
    if (!out) return fail(FV_ENULL, "out is NULL");
    if (capacity < 1 || capacity > (1 << 20)) return fail(FV_EINVAL, "capacity %d out of range", capacity);
    *out = table_bound(capacity);
    return FV_OK;
}

int batch_create(int32_t capacity, void* table, size_t table_bytes, fv_batch** out)
{
    if (!out) return fail(FV_ENULL, "out is NULL");
    *out = nullptr;
    if (capacity < 1 || capacity > (1 << 20)) return fail(FV_EINVAL, "capacity %d out of range", capacity);
    int r = check_ptr(table, "table");
    if (r) return r;
    if ((uintptr_t)table % TAB_ALIGN) return fail(FV_EALIGN, "table must be 256-byte aligned");
    if (table_bytes < table_bound(capacity))
        return fail(FV_EINVAL, "table of %zu bytes is smaller than batch_table_bytes (%zu)", table_bytes,
                    table_bound(capacity));
    fv_batch* b = new fv_batch;
    b->capacity = capacity;
    b->table = (char*)table;
    b->table_bytes = table_bytes;
    for (int k = 0; k < 2; k++) {
        hipError_t e = hipHostMalloc((void**)&b->host[k], table_bound(capacity), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            batch_destroy(b);
            return hip_fail(e, "batch_create");
        }
    }
    *out = b;
    return FV_OK;
}

int batch_destroy(fv_batch* b)
{
    if (!b) return FV_OK;
    drop_graphs(b);
    for (int k = 0; k < 2; k++) {
        if (b->copied[k]) {
            if (b->pending[k]) (void)hipEventSynchronize(b->copied[k]);
            (void)hipEventDestroy(b->copied[k]);
        }
        if (b->host[k]) (void)hipHostFree(b->host[k]);
    }
    delete b;
    return FV_OK;
}

int batch_set(fv_batch* b, int32_t n, const fv_config* cfgs, void* const* U, void* const* ws, const int32_t* fresh,
              void* stream)
{
    if (!b) return fail(FV_ENULL, "batch is NULL");
    if (n < 0 || n > b->capacity) return fail(FV_EINVAL, "n = %d outside 0 .. capacity %d", n, b->capacity);
    if (n > 0 && (!cfgs || !U || !ws)) return fail(FV_ENULL, "cfgs, U and ws are required");
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n; i++) {
        int r = validate(&cfgs[i]);
        if (r) return fail(r, "member %d: %s", i, last_error());
        if ((r = check_ptr(U[i], "U")) || (r = check_ptr(ws[i], "ws"))) return fail(r, "member %d: %s", i, last_error());
        if (!(cfgs[i].cfl > 0)) return fail(FV_EINVAL, "member %d: cfl must be > 0", i);
        if (visc6(&cfgs[i])) return fail(FV_EUNSUPPORTED, "member %d: batches use 4th-order viscous fluxes", i);
    }
    // groups present, in the order of their id; members keep their order inside a group
    int gcount[MAX_GROUP_IDS] = {0};
    std::vector<int> gid(n);
    for (int i = 0; i < n; i++) {
        const fv_config* c = &cfgs[i];
        const int variant = (c->model == FV_NS && c->visc_law != 0) || (c->model == FV_DIM && c->thinc) ? 1 : 0;
        gid[i] = (((c->model * 2 + c->dtype) * 2 + (positivity_on(c) ? 1 : 0)) * 4 + c->recon + 2 * c->scheme) * 2 +
                 variant;
        gcount[gid[i]]++;
    }
    int present = 0;
    for (int g = 0; g < MAX_GROUP_IDS; g++) present += gcount[g] ? 1 : 0;
    if (present > MAX_GROUPS)
        return fail(FV_EINVAL, "the members form %d groups (model, precision, limiters, reconstruction, variant); "
                               "a batch holds at most %d",
                    present, MAX_GROUPS);
    std::vector<BatchGroup> groups;
    int pos_of[MAX_GROUP_IDS];
    const size_t rb = region_bytes(b->capacity), ab = args_bytes(b->capacity);
    for (int g = 0; g < MAX_GROUP_IDS; g++) {
        pos_of[g] = -1;
        if (!gcount[g]) continue;
        BatchGroup ng;
        memset(&ng, 0, sizeof ng);
        ng.gid = g;
        ng.variant = g % 2;
        ng.rec = (g / 2) % 4;
        ng.pos = (g / 8) % 2;
        ng.dtype = (g / 16) % 2;
        ng.model = g / 32;
        ng.count = gcount[g];
        ng.hdr_off = groups.size() * rb;
        ng.first_off = ng.hdr_off + TAB_ALIGN;
        for (int s = 0; s < 3; s++)
            ng.args_off[s] = ng.first_off + align_up(sizeof(int) * (size_t)(b->capacity + 1)) + s * ab;
        pos_of[g] = (int)groups.size();
        groups.push_back(ng);
    }
    const size_t scal_hdr_off = groups.size() * rb;
    const size_t scal_off = scal_hdr_off + TAB_ALIGN;
    const size_t end = scal_off + sizeof(fv::BatchScalars) * (size_t)(n > 0 ? n : 1);
    if (end > b->table_bytes || end > table_bound(b->capacity))
        return fail(FV_EINVAL, "batch table too small (%zu > %zu)", end, b->table_bytes);

    // the staging buffer may still feed an earlier copy
    const int k = b->cur;
    if (b->pending[k]) {
        hipError_t e = hipEventSynchronize(b->copied[k]);
        if (e != hipSuccess) return hip_fail(e, "batch_set: staging wait");
        b->pending[k] = false;
    }
    char* img = b->host[k];
    memset(img, 0, end);
    std::vector<int> slot(groups.size(), 0), first(groups.size(), 0);
    fv::BatchScalars* sc = reinterpret_cast<fv::BatchScalars*>(img + scal_off);
    for (int i = 0; i < n; i++) {
        const int p = pos_of[gid[i]];
        BatchGroup& g = groups[p];
        int nb = 0;
        if (g.dtype == FV_F64) fill_group_args<double>(&cfgs[i], U[i], ws[i], img, g, slot[p], first[p], &nb);
        else fill_group_args<float>(&cfgs[i], U[i], ws[i], img, g, slot[p], first[p], &nb);
        slot[p]++;
        first[p] += nb;
        const WsLayout w = ws_layout(&cfgs[i], ws[i]);
        sc[i].inv_max = w.inv_max;
        sc[i].dt = w.dt;
        sc[i].t_acc = w.t_acc;
        sc[i].cfl = cfgs[i].cfl;
    }
    for (size_t p = 0; p < groups.size(); p++) {
        reinterpret_cast<int*>(img + groups[p].hdr_off)[0] = groups[p].count;
        reinterpret_cast<int*>(img + groups[p].first_off)[groups[p].count] = first[p];
        groups[p].nblocks = first[p];
        for (int s = 0; s < 3; s++) {
            if (groups[p].dtype == FV_F64)
                groups[p].solo_d[s] = reinterpret_cast<const fv::StageArgs<double>*>(img + groups[p].args_off[s])[0];
            else
                groups[p].solo_f[s] = reinterpret_cast<const fv::StageArgs<float>*>(img + groups[p].args_off[s])[0];
        }
    }
    reinterpret_cast<int*>(img + scal_hdr_off)[0] = n;
    // kernel attributes before any capture
    for (const BatchGroup& g : groups) {
        hipError_t e = g.dtype == FV_F64
                           ? fv::launch_batch_stage<double>(g.model, g.rec, g.pos != 0, g.variant, nullptr, nullptr,
                                                            nullptr, 0, st)
                           : fv::launch_batch_stage<float>(g.model, g.rec, g.pos != 0, g.variant, nullptr, nullptr,
                                                           nullptr, 0, st);
        if (e != hipSuccess) return hip_fail(e, "batch_set: kernel attributes");
    }
    hipError_t e = hipMemcpyAsync(b->table, img, end, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(b->copied[k], st);
    if (e != hipSuccess) return hip_fail(e, "batch_set: table upload");
    b->pending[k] = true;
    b->cur = 1 - k;
    // new members: first dt from a full reduction, simulated time 0
    for (int i = 0; i < n; i++) {
        if (!fresh || !fresh[i]) continue;
        const fv_config* c = &cfgs[i];
        const WsLayout w = ws_layout(c, ws[i]);
        const fv::AuxArgs a = aux_args(c);
        const double mu = c->model == FV_NS ? c->mu : 0.0;
        e = c->dtype == FV_F64 ? fv::launch_dt<double>(a, (const double*)U[i], mu, c->cfl, w.inv_max, w.dt, nullptr, st)
                               : fv::launch_dt<float>(a, (const float*)U[i], mu, c->cfl, w.inv_max, w.dt, nullptr, st);
        if (e == hipSuccess) e = fv::launch_reset_max((unsigned long long*)w.t_acc, st);
        if (e != hipSuccess) return hip_fail(e, "batch_set: first dt");
    }
    b->groups = groups;
    b->n = n;
    b->scal_hdr_off = scal_hdr_off;
    b->scal_off = scal_off;
    return FV_OK;
}

int batch_step(fv_batch* b, int32_t nsteps, void* stream)
{
    if (!b) return fail(FV_ENULL, "batch is NULL");
    if (nsteps < 0) return fail(FV_EINVAL, "nsteps must be >= 0");
    if (b->n == 0) return FV_OK;
    return batch_launch_steps(b, nsteps, (hipStream_t)stream, false);
}

int batch_step_graph(fv_batch* b, int32_t nsteps, void* stream)
{
    if (!b) return fail(FV_ENULL, "batch is NULL");
    if (nsteps < 1) return fail(FV_EINVAL, "nsteps must be >= 1");
    if (!stream) return fail(FV_EINVAL, "graph capture needs a non-default stream");
    if (b->n == 0) return FV_OK;
    hipStream_t st = (hipStream_t)stream;
    // one member per group: the single-problem kernels, launched directly (a graph of
    // them would have to be captured again for every member)
    bool all_single = true;
    for (const BatchGroup& g : b->groups) all_single = all_single && g.count == 1;
    if (all_single) return batch_launch_steps(b, nsteps, st, false);
    std::vector<long long> key;
    for (const BatchGroup& g : b->groups) {
        key.push_back(g.gid);
        key.push_back(grid_bucket(g.nblocks));
    }
    key.push_back(nsteps);
    GraphEntry* hit = nullptr;
    for (GraphEntry& ge : b->graphs)
        if (ge.stream == st && ge.key == key) hit = &ge;
    if (!hit) {
        if ((int)b->graphs.size() >= MAX_GRAPHS) {
            size_t lru = 0;
            for (size_t i = 1; i < b->graphs.size(); i++)
                if (b->graphs[i].last_use < b->graphs[lru].last_use) lru = i;
            (void)hipGraphExecDestroy(b->graphs[lru].exec);
            b->graphs.erase(b->graphs.begin() + (long)lru);
        }
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "batch_step_graph: begin capture");
        const int r = batch_launch_steps(b, nsteps, st, true);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(st, &graph);
        if (r) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess) return hip_fail(e, "batch_step_graph: end capture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "batch_step_graph: instantiate");
        GraphEntry ge;
        ge.key = key;
        ge.stream = st;
        ge.exec = exec;
        ge.last_use = 0;
        b->graphs.push_back(ge);
        hit = &b->graphs.back();
    }
    hit->last_use = ++b->uses;
    hipError_t e = hipGraphLaunch(hit->exec, st);
    if (e != hipSuccess) return hip_fail(e, "batch_step_graph: launch");
    return FV_OK;
}

int batch_graph_count(const fv_batch* b)
{
    return b ? (int)b->graphs.size() : 0;
}

int workspace_time(const fv_config* cfg, const void* ws, double* t, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(ws, "ws"))) return r;
    if (!t) return fail(FV_ENULL, "t is NULL");
    const WsLayout w = ws_layout(cfg, (void*)ws);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(t, w.t_acc, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "workspace_time");
    return FV_OK;
}

}  // extern "C"
