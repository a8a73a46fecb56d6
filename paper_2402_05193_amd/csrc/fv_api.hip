// fv_api.hip -- the C ABI declared in include/fvrk3.h: validation, launch
// geometry, workspace layout and error reporting.  No device allocation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

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

constexpr size_t SCALAR_BYTES = 256;  // dt, inverse-dt max, time accumulator, check words

int validate(const fv_config* c)
{
    if (!c) return fail(FV_ENULL, "cfg is NULL");
    if (c->abi_version != FV_ABI_VERSION) return fail(FV_EINVAL, "abi_version %d != %d", c->abi_version, FV_ABI_VERSION);
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(FV_EINVAL, "grid %d x %d x %d must be >= 1", c->nx, c->ny, c->nz);
    if ((long long)c->nx * c->ny * c->nz > (1ll << 40)) return fail(FV_EINVAL, "grid too large");
    if (c->model < FV_EULER || c->model > FV_DIM) return fail(FV_EINVAL, "model %d unknown", c->model);
    if (c->dtype != FV_F64 && c->dtype != FV_F32) return fail(FV_EINVAL, "dtype %d unknown", c->dtype);
    if (c->reserved != 0) return fail(FV_EINVAL, "reserved must be 0");
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
    return a;
}

bool positivity_on(const fv_config* c)
{
    return c->positivity < 0 ? c->model == FV_DIM : c->positivity == 1;
}

template <typename Real>
fv::StageArgs<Real> stage_args(const fv_config* c, fv::LaunchGeom& g)
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
    const long long target = 2048;
    int nch = (int)((target + tiles - 1) / tiles);
    if (nch < 1) nch = 1;
    int zc = (c->nz + nch - 1) / nch;
    if (zc < 16) zc = 16 < c->nz ? 16 : c->nz;
    a.zchunk = zc;
    a.nchunks = (c->nz + zc - 1) / zc;
    g.nblocks = (int)(tiles * a.nchunks);
    a.positivity = positivity_on(c) ? 1 : 0;
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
    a.inv_max = nullptr;
    a.kappa = (Real)(c->model == FV_NS ? c->mu * c->gamma1 / ((c->gamma1 - 1.0) * c->prandtl) : 0.0);
    return a;
}

template <typename Real>
int stage_impl(const fv_config* c, int mode, const void* Un, const void* Uk, void* out, double dt, const double* dt_dev,
               hipStream_t st, unsigned long long* inv_max)
{
    fv::LaunchGeom g;
    fv::StageArgs<Real> a = stage_args<Real>(c, g);
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
                   const double* dt_dev, hipStream_t st, unsigned long long* inv_max = nullptr)
{
    if (c->dtype == FV_F64) return stage_impl<double>(c, mode, Un, Uk, out, dt, dt_dev, st, inv_max);
    return stage_impl<float>(c, mode, Un, Uk, out, dt, dt_dev, st, inv_max);
}

struct WsLayout {
    char* A;
    char* B;
    double* dt;
    unsigned long long* inv_max;
    double* t_acc;
    long long* check;
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
    return w;
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
    *out = 2 * ((state_bytes(cfg) + 255) & ~(size_t)255) + SCALAR_BYTES;
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
    default: return fail(FV_EINVAL, "case_id %d unknown", case_id);
    }
    if (case_id == FV_CASE_TGV && cfg->model == FV_DIM) return fail(FV_EINVAL, "TGV is a single-phase case");
    if (case_id == FV_CASE_SBI && cfg->model != FV_DIM) return fail(FV_EINVAL, "SBI needs the DIM model");
    if (nparams < need) return fail(FV_EINVAL, "case %d needs %d parameters, got %d", case_id, need, nparams);
    if (!params) return fail(FV_ENULL, "params is NULL");
    if (case_id == FV_CASE_RIEMANN && (params[0] < 0 || params[0] > 2)) return fail(FV_EINVAL, "axis must be 0, 1 or 2");
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
    return stage_dispatch(cfg, 0, U, U, R, dt, nullptr, (hipStream_t)stream);
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
    if ((r = stage_dispatch(cfg, 3, Un, Uk, Uout, 0.0, dt_dev, st, w.inv_max))) return r;
    e = fv::launch_dt_finish(w.inv_max, cfg->cfl, dt_next, nullptr, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "rk3_stage3_cfl: finish");
    return FV_OK;
}

static int step_impl(const fv_config* cfg, void* U, double dt, const double* dt_dev, const WsLayout& w, hipStream_t st,
                     unsigned long long* inv_max = nullptr)
{
    int r;
    if ((r = stage_dispatch(cfg, 1, U, U, w.A, dt, dt_dev, st))) return r;
    if ((r = stage_dispatch(cfg, 2, U, w.A, w.B, dt, dt_dev, st))) return r;
    return stage_dispatch(cfg, 3, U, w.B, U, dt, dt_dev, st, inv_max);
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

int advance(const fv_config* cfg, void* U, int32_t nsteps, double dt, double* t_inout, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    if ((r = check_ptr(U, "U")) || (r = check_ptr(ws, "ws"))) return r;
    if (nsteps < 0) return fail(FV_EINVAL, "nsteps must be >= 0");
    const bool cfl_mode = !(dt > 0);
    if (cfl_mode && !(cfg->cfl > 0)) return fail(FV_EINVAL, "cfl must be > 0 when dt <= 0");
    if (!cfl_mode && !isfinite(dt)) return fail(FV_EINVAL, "dt must be finite");
    hipStream_t st = (hipStream_t)stream;
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

int rhs_adjoint(const fv_config* cfg, const void* U, const void* Rbar, void* Ubar, void* ws, void* stream)
{
    int r = validate(cfg);
    if (r) return r;
    (void)U;
    (void)Rbar;
    (void)Ubar;
    (void)ws;
    (void)stream;
    return fail(FV_EUNSUPPORTED, "rhs_adjoint is not built in this library");
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
