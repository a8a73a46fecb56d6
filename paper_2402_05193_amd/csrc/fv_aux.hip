// fv_aux.hip -- point-wise and reduction kernels around the fused stage:
// primitive/conservative maps, analytic initial conditions, the CFL time-step
// reduction and the admissibility scan.
#include <hip/hip_runtime.h>

#include "fv_kernels.h"

namespace fv {

template <typename Real>
__device__ __forceinline__ const Material<Real>& mat_of(const AuxArgs& a);
template <>
__device__ __forceinline__ const Material<double>& mat_of<double>(const AuxArgs& a)
{
    return a.matd;
}
template <>
__device__ __forceinline__ const Material<float>& mat_of<float>(const AuxArgs& a)
{
    return a.matf;
}

constexpr int AUX_THREADS = 256;

static inline int aux_blocks(long long n)
{
    long long b = (n + AUX_THREADS - 1) / AUX_THREADS;
    return (int)(b < 1 ? 1 : b);
}

// ------------------------------------------------------------------ W <-> U
template <typename Real, int MODEL, bool TO_CONS>
__global__ void __launch_bounds__(AUX_THREADS) convert_kernel(const AuxArgs a, const Real* __restrict__ in,
                                                              Real* __restrict__ out)
{
    constexpr int NC = Layout<MODEL>::NC;
    const long long q = (long long)blockIdx.x * AUX_THREADS + threadIdx.x;
    if (q >= a.ncell) return;
    Real x[NC], y[NC];
#pragma unroll
    for (int m = 0; m < NC; m++) x[m] = in[m * a.ncell + q];
    if constexpr (TO_CONS) prim_to_cons<Real, MODEL>(mat_of<Real>(a), x, y);
    else cons_to_prim<Real, MODEL>(mat_of<Real>(a), x, y);
#pragma unroll
    for (int m = 0; m < NC; m++) out[m * a.ncell + q] = y[m];
}

template <typename Real, bool TO_CONS>
static hipError_t launch_convert(const AuxArgs& a, const Real* in, Real* out, hipStream_t st)
{
    const int nb = aux_blocks(a.ncell);
    switch (a.model) {
    case EULER: hipLaunchKernelGGL((convert_kernel<Real, EULER, TO_CONS>), dim3(nb), dim3(AUX_THREADS), 0, st, a, in, out); break;
    case NS: hipLaunchKernelGGL((convert_kernel<Real, NS, TO_CONS>), dim3(nb), dim3(AUX_THREADS), 0, st, a, in, out); break;
    default: hipLaunchKernelGGL((convert_kernel<Real, DIM, TO_CONS>), dim3(nb), dim3(AUX_THREADS), 0, st, a, in, out); break;
    }
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_prim_to_cons(const AuxArgs& a, const Real* W, Real* U, hipStream_t st)
{
    return launch_convert<Real, true>(a, W, U, st);
}
template <typename Real>
hipError_t launch_cons_to_prim(const AuxArgs& a, const Real* U, Real* W, hipStream_t st)
{
    return launch_convert<Real, false>(a, U, W, st);
}
template hipError_t launch_prim_to_cons<double>(const AuxArgs&, const double*, double*, hipStream_t);
template hipError_t launch_prim_to_cons<float>(const AuxArgs&, const float*, float*, hipStream_t);
template hipError_t launch_cons_to_prim<double>(const AuxArgs&, const double*, double*, hipStream_t);
template hipError_t launch_cons_to_prim<float>(const AuxArgs&, const float*, float*, hipStream_t);

// ------------------------------------------------------------------ initial conditions
// splitmix64 (Steele, Lea & Flood 2014): output number (n + 1) of the stream seeded by `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform01(uint64_t seed, uint64_t n)
{
    return (double)(splitmix64(seed, n) >> 11) * 0x1.0p-53;
}

struct InitParams {
    int case_id, nparams;
    uint64_t seed;
    double p[40];
};

template <typename Real, int MODEL>
__global__ void __launch_bounds__(AUX_THREADS) init_kernel(const AuxArgs a, const InitParams ip, Real* __restrict__ U)
{
    constexpr int NC = Layout<MODEL>::NC, V = Layout<MODEL>::V, P = Layout<MODEL>::P;
    const long long q = (long long)blockIdx.x * AUX_THREADS + threadIdx.x;
    if (q >= a.ncell) return;
    const int i = (int)(q % a.nx);
    const int j = (int)((q / a.nx) % a.ny);
    const int k = (int)(q / ((long long)a.nx * a.ny));
    const double x = (i + 0.5) * a.dx, y = (j + 0.5) * a.dy, z = (k + 0.5) * a.dz;
    double w[NC];
    for (int m = 0; m < NC; m++) w[m] = 0.0;
    if (ip.case_id == 0) {  // uniform
        for (int m = 0; m < NC; m++) w[m] = ip.p[m];
    } else if (ip.case_id == 1) {  // Taylor-Green vortex + seeded noise (single phase)
        const double ma = ip.p[0], rho0 = ip.p[1], amp = ip.p[2];
        const double gamma = a.matd.gamma;
        w[0] = rho0;
        w[V] = sin(x) * cos(y) * cos(z);
        w[V + 1] = -cos(x) * sin(y) * cos(z);
        w[V + 2] = 0.0;
        w[P] = 1.0 / (gamma * ma * ma) + (cos(2.0 * x) + cos(2.0 * y)) * (cos(2.0 * z) + 2.0) / 16.0;
        if (amp != 0.0) {
            for (int c = 0; c < 3; c++) {
                const uint64_t n = (uint64_t)q * 3ull + (uint64_t)c;
                w[V + c] += amp * (2.0 * uniform01(ip.seed, n) - 1.0);
            }
        }
    } else if (ip.case_id == 2) {  // planar Riemann problem
        const int axis = (int)ip.p[0];
        const double frac = ip.p[1];
        const int idx3[3] = {i, j, k};
        const int n3[3] = {a.nx, a.ny, a.nz};
        const double c = (idx3[axis] + 0.5) / n3[axis];
        const double* src = c < frac ? &ip.p[2] : &ip.p[2 + NC];
        for (int m = 0; m < NC; m++) w[m] = src[m];
    } else if (ip.case_id == 4) {  // density wave of two Gaussians (single phase), exact cell averages
        // rho(s) = 1 + 5 exp(-200 (s - 0.5)^2) + 5 exp(-200 (s - 1.5)^2) along the axis; the
        // cell average from the antiderivative sqrt(pi)/(2 sqrt(200)) erf(sqrt(200)(s - c))
        const int axis = (int)ip.p[0];
        const int idx3[3] = {i, j, k};
        const double hs[3] = {a.dx, a.dy, a.dz};
        const double h = hs[axis], s0 = idx3[axis] * h, s1 = s0 + h;
        const double r = sqrt(200.0);
        double acc = 0.0;
        for (int g = 0; g < 2; g++) {
            const double c = g == 0 ? 0.5 : 1.5;
            acc += erf(r * (s1 - c)) - erf(r * (s0 - c));
        }
        w[0] = 1.0 + 5.0 * sqrt(M_PI) / (2.0 * r) * acc / h;
        w[V + axis] = ip.p[1];
        w[P] = ip.p[2];
    } else if (ip.case_id == 5) {  // isentropic vortex (single phase), z-invariant
        // cell averages of the conservative variables by 5 x 5 Gauss-Legendre points in x, y
        const double eps = ip.p[0], xc = ip.p[1], yc = ip.p[2], uinf = ip.p[3], vinf = ip.p[4];
        const double gamma = a.matd.gamma;
        const double t1 = sqrt(5.0 - 2.0 * sqrt(10.0 / 7.0)) / 3.0, t2 = sqrt(5.0 + 2.0 * sqrt(10.0 / 7.0)) / 3.0;
        const double gx[5] = {-t2, -t1, 0.0, t1, t2};
        const double w1 = (322.0 + 13.0 * sqrt(70.0)) / 900.0, w2 = (322.0 - 13.0 * sqrt(70.0)) / 900.0;
        const double gw[5] = {w2, w1, 128.0 / 225.0, w1, w2};
        double uc[NC];
        for (int m = 0; m < NC; m++) uc[m] = 0.0;
        for (int ga = 0; ga < 5; ga++)
            for (int gb = 0; gb < 5; gb++) {
                const double X = x + 0.5 * gx[ga] * a.dx - xc, Y = y + 0.5 * gx[gb] * a.dy - yc;
                const double wt = 0.25 * gw[ga] * gw[gb];
                const double r2 = X * X + Y * Y;
                const double f = exp(0.5 * (1.0 - r2));
                const double u = uinf - eps / (2.0 * M_PI) * f * Y, v = vinf + eps / (2.0 * M_PI) * f * X;
                const double T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * M_PI * M_PI) * exp(1.0 - r2);
                const double rho = pow(T, 1.0 / (gamma - 1.0));
                const double p = rho * T;
                uc[0] += wt * rho;
                uc[V] += wt * rho * u;
                uc[V + 1] += wt * rho * v;
                uc[P] += wt * (p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v));
            }
#pragma unroll
        for (int m = 0; m < NC; m++) U[m * a.ncell + q] = (Real)uc[m];
        return;
    } else {  // shock-bubble interaction (five-equation model)
        const double xs = ip.p[0], xc = ip.p[1], yc = ip.p[2], zc = ip.p[3], R = ip.p[4], eps = ip.p[5];
        const double rho2 = ip.p[6], u2 = ip.p[7], p2 = ip.p[8], rho_air = ip.p[9], p_air = ip.p[10];
        const double rho_b = ip.p[11];
        const double r = sqrt((x - xc) * (x - xc) + (y - yc) * (y - yc) + (z - zc) * (z - zc));
        const double a1 = eps + (1.0 - 2.0 * eps) * 0.5 * (1.0 - tanh((r - R) / a.dx));
        const bool shocked = x < xs;
        const double rho_a = shocked ? rho2 : rho_air;
        w[0] = a1 * rho_b;
        if constexpr (MODEL == DIM) {
            w[1] = (1.0 - a1) * rho_a;
            w[6] = a1;
        }
        w[V] = shocked ? u2 : 0.0;
        w[P] = shocked ? p2 : p_air;
    }
    Real wr[NC], u[NC];
    for (int m = 0; m < NC; m++) wr[m] = (Real)w[m];
    prim_to_cons<Real, MODEL>(mat_of<Real>(a), wr, u);
#pragma unroll
    for (int m = 0; m < NC; m++) U[m * a.ncell + q] = u[m];
}

template <typename Real>
hipError_t launch_init(const AuxArgs& a, int case_id, const double* params, int nparams, uint64_t seed, Real* U,
                       hipStream_t st)
{
    InitParams ip{};
    ip.case_id = case_id;
    ip.nparams = nparams;
    ip.seed = seed;
    for (int n = 0; n < nparams && n < 40; n++) ip.p[n] = params[n];
    const int nb = aux_blocks(a.ncell);
    switch (a.model) {
    case EULER: hipLaunchKernelGGL((init_kernel<Real, EULER>), dim3(nb), dim3(AUX_THREADS), 0, st, a, ip, U); break;
    case NS: hipLaunchKernelGGL((init_kernel<Real, NS>), dim3(nb), dim3(AUX_THREADS), 0, st, a, ip, U); break;
    default: hipLaunchKernelGGL((init_kernel<Real, DIM>), dim3(nb), dim3(AUX_THREADS), 0, st, a, ip, U); break;
    }
    return hipGetLastError();
}
template hipError_t launch_init<double>(const AuxArgs&, int, const double*, int, uint64_t, double*, hipStream_t);
template hipError_t launch_init<float>(const AuxArgs&, int, const double*, int, uint64_t, float*, hipStream_t);

// ------------------------------------------------------------------ CFL time step
__global__ void add_scalar_kernel_fwd(double* t_acc, const double* dt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *t_acc += *dt;
}

__global__ void reset_u64_kernel(unsigned long long* p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

template <typename Real, int MODEL>
__global__ void __launch_bounds__(AUX_THREADS) inv_dt_kernel(const AuxArgs a, const Real* __restrict__ U, double mu,
                                                             unsigned long long* __restrict__ inv_max)
{
    constexpr int NC = Layout<MODEL>::NC, V = Layout<MODEL>::V;
    __shared__ double red[AUX_THREADS / 64];
    double v = 0.0;
    const double hmin = fmin(a.dx, fmin(a.dy, a.dz));
    for (long long q = (long long)blockIdx.x * AUX_THREADS + threadIdx.x; q < a.ncell;
         q += (long long)gridDim.x * AUX_THREADS) {
        Real u[NC], w[NC];
#pragma unroll
        for (int m = 0; m < NC; m++) u[m] = U[m * a.ncell + q];
        cons_to_prim<Real, MODEL>(mat_of<Real>(a), u, w);
        const double rho = (double)density<Real, MODEL>(w);
        const double c = sqrt((double)rhoc2<Real, MODEL>(mat_of<Real>(a), w) / rho);
        const double s0 = (fabs((double)w[V]) + c) / a.dx;
        const double s1 = (fabs((double)w[V + 1]) + c) / a.dy;
        const double s2 = (fabs((double)w[V + 2]) + c) / a.dz;
        double t = fmax(s0, fmax(s1, s2));
        if (MODEL == NS && mu > 0.0) {
            const double m = a.vl.law == 0 ? mu : visc_mu(a.vl, (double)w[Layout<MODEL>::P] / rho);
            t = fmax(t, m / (3.0 / 14.0 * rho * hmin * hmin));
        }
        if (!(t >= 0.0)) t = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +inf (dt -> 0)
        v = fmax(v, t);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int k = 1; k < AUX_THREADS / 64; k++) m = fmax(m, red[k]);
        atomicMax(inv_max, (unsigned long long)__double_as_longlong(m));
    }
}

// t_acc += *dt_prev (optional); *dt_out = cfl / max; max = 0 for the next reduction
__global__ void dt_finish_kernel(unsigned long long* inv_max, double cfl, double* dt_out, double* t_acc,
                                 const double* dt_prev)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (t_acc && dt_prev) *t_acc += *dt_prev;
        const double m = __longlong_as_double((long long)*inv_max);
        *dt_out = cfl / m;
        *inv_max = 0ull;
    }
}

__global__ void batch_dt_finish_kernel(const BatchScalars* __restrict__ s, const int* __restrict__ count)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < *count) {
        const BatchScalars b = s[r];
        *b.t_acc += *b.dt;
        const double m = __longlong_as_double((long long)*b.inv_max);
        *b.dt = b.cfl / m;
        *b.inv_max = 0ull;
    }
}

hipError_t launch_batch_dt_finish(const BatchScalars* s, const int* count, int max_n, hipStream_t st)
{
    if (max_n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_dt_finish_kernel, dim3((max_n + 63) / 64), dim3(64), 0, st, s, count);
    return hipGetLastError();
}

__global__ void fill_u8_kernel(unsigned char* __restrict__ p, long long n, unsigned char v)
{
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

hipError_t launch_fill_u8(unsigned char* p, long long n, unsigned char v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)nb), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_reset_max(unsigned long long* inv_max, hipStream_t st)
{
    hipLaunchKernelGGL(reset_u64_kernel, dim3(1), dim3(64), 0, st, inv_max);
    return hipGetLastError();
}

hipError_t launch_dt_finish(unsigned long long* inv_max, double cfl, double* dt_out, double* t_acc,
                            const double* dt_prev, hipStream_t st)
{
    hipLaunchKernelGGL(dt_finish_kernel, dim3(1), dim3(64), 0, st, inv_max, cfl, dt_out, t_acc, dt_prev);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_dt(const AuxArgs& a, const Real* U, double mu, double cfl, unsigned long long* inv_max,
                     double* dt_out, double* t_acc, hipStream_t st)
{
    hipLaunchKernelGGL(reset_u64_kernel, dim3(1), dim3(64), 0, st, inv_max);
    long long nb = (a.ncell + AUX_THREADS - 1) / AUX_THREADS;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    switch (a.model) {
    case EULER: hipLaunchKernelGGL((inv_dt_kernel<Real, EULER>), dim3(nb), dim3(AUX_THREADS), 0, st, a, U, mu, inv_max); break;
    case NS: hipLaunchKernelGGL((inv_dt_kernel<Real, NS>), dim3(nb), dim3(AUX_THREADS), 0, st, a, U, mu, inv_max); break;
    default: hipLaunchKernelGGL((inv_dt_kernel<Real, DIM>), dim3(nb), dim3(AUX_THREADS), 0, st, a, U, mu, inv_max); break;
    }
    hipLaunchKernelGGL(dt_finish_kernel, dim3(1), dim3(64), 0, st, inv_max, cfl, dt_out, (double*)nullptr,
                       (const double*)nullptr);
    if (t_acc) hipLaunchKernelGGL(add_scalar_kernel_fwd, dim3(1), dim3(64), 0, st, t_acc, (const double*)dt_out);
    return hipGetLastError();
}
template hipError_t launch_dt<double>(const AuxArgs&, const double*, double, double, unsigned long long*, double*,
                                      double*, hipStream_t);
template hipError_t launch_dt<float>(const AuxArgs&, const float*, double, double, unsigned long long*, double*,
                                     double*, hipStream_t);

__global__ void add_scalar_kernel(double* t_acc, const double* dt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *t_acc += *dt;
}
hipError_t launch_add_scalar(double* t_acc, const double* dt, hipStream_t st)
{
    hipLaunchKernelGGL(add_scalar_kernel, dim3(1), dim3(64), 0, st, t_acc, dt);
    return hipGetLastError();
}

// ------------------------------------------------------------------ admissibility scan
__global__ void reset_check_kernel(long long* w)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        w[0] = 0x7fffffffffffffffll;
        w[1] = 0;
        w[2] = 0;
    }
}

template <typename Real, int MODEL>
__global__ void __launch_bounds__(AUX_THREADS) check_kernel(const AuxArgs a, const Real* __restrict__ U,
                                                            long long* __restrict__ words)
{
    constexpr int NC = Layout<MODEL>::NC;
    const long long q = (long long)blockIdx.x * AUX_THREADS + threadIdx.x;
    if (q >= a.ncell) return;
    Real u[NC], w[NC];
    bool finite = true;
#pragma unroll
    for (int m = 0; m < NC; m++) {
        u[m] = U[m * a.ncell + q];
        finite = finite && isfinite(u[m]);
    }
    int code = 0;
    if (!finite) {
        code = 2;
    } else {
        cons_to_prim<Real, MODEL>(mat_of<Real>(a), u, w);
        bool ok;
        if constexpr (MODEL == DIM) ok = w[0] > Real(0) && w[1] > Real(0) && w[6] >= Real(0) && w[6] <= Real(1);
        else ok = w[0] > Real(0);
        ok = ok && rhoc2<Real, MODEL>(mat_of<Real>(a), w) > Real(0);
        if (!ok) code = 1;
    }
    if (code) {
        atomicMin(&words[0], q);
        atomicAdd((unsigned long long*)&words[1], 1ull);
        atomicMax(&words[2], (long long)code);
    }
}

template <typename Real>
hipError_t launch_check(const AuxArgs& a, const Real* U, long long* words, hipStream_t st)
{
    hipLaunchKernelGGL(reset_check_kernel, dim3(1), dim3(64), 0, st, words);
    const int nb = aux_blocks(a.ncell);
    switch (a.model) {
    case EULER: hipLaunchKernelGGL((check_kernel<Real, EULER>), dim3(nb), dim3(AUX_THREADS), 0, st, a, U, words); break;
    case NS: hipLaunchKernelGGL((check_kernel<Real, NS>), dim3(nb), dim3(AUX_THREADS), 0, st, a, U, words); break;
    default: hipLaunchKernelGGL((check_kernel<Real, DIM>), dim3(nb), dim3(AUX_THREADS), 0, st, a, U, words); break;
    }
    return hipGetLastError();
}
template hipError_t launch_check<double>(const AuxArgs&, const double*, long long*, hipStream_t);
template hipError_t launch_check<float>(const AuxArgs&, const float*, long long*, hipStream_t);

}  // namespace fv
