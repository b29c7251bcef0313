// dugks_api.hip -- host side of the C ABI declared in include/dugks.h:
// configuration checks, mesh metric tables, coefficient set-up and kernel
// launches for gfx950.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dugks.h"
#include "kernels_general.hpp"
#include "ctx.hpp"

using namespace dugks;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_init_err = "no error";

namespace dugks {
int fail(dugks_ctx* ctx, int code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    else g_init_err = msg;
    return code;
}
int hip_check(dugks_ctx* ctx, hipError_t e, const char* what)
{
    if (e == hipSuccess) return DUGKS_OK;
    return fail(ctx, DUGKS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace dugks

extern "C" const char* dugks_version(void) { return "dugks-gfx950 1.0.0"; }

extern "C" const char* dugks_last_error(const dugks_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

// ---------------------------------------------------------------------------
// configuration and mesh metrics
// ---------------------------------------------------------------------------
namespace dugks {

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const dugks_config* c, std::string& why)
{
    if (!c) { why = "null configuration"; return DUGKS_EINVAL; }
    if (c->lattice != DUGKS_D2Q9 && c->lattice != DUGKS_D3Q19 && c->lattice != DUGKS_D3Q27) {
        why = "lattice must be 9, 19 or 27";
        return DUGKS_EINVAL;
    }
    if (c->dtype != DUGKS_F32 && c->dtype != DUGKS_F64) { why = "dtype must be F32 or F64"; return DUGKS_EINVAL; }
    const int D = c->lattice == DUGKS_D2Q9 ? 2 : 3;
    if (D == 2 && c->n[2] != 1) { why = "D2Q9 needs n[2] == 1"; return DUGKS_EINVAL; }
    for (int a = 0; a < D; ++a) {
        if (c->n[a] < 1 || c->n[a] > (1 << 24)) { why = "cell count out of range"; return DUGKS_EINVAL; }
        if (!finite_pos(c->L[a])) { why = "domain length must be positive"; return DUGKS_EINVAL; }
        if (c->mesh[a] != DUGKS_UNIFORM && c->mesh[a] != DUGKS_TANH && c->mesh[a] != DUGKS_CUSTOM) {
            why = "unknown mesh kind";
            return DUGKS_EINVAL;
        }
        if (c->mesh[a] == DUGKS_TANH && !finite_pos(c->k_stretch)) { why = "tanh mesh needs k_stretch > 0"; return DUGKS_EINVAL; }
        if (c->mesh[a] == DUGKS_CUSTOM) {
            const double* X = c->faces[a];
            if (!X) { why = "custom mesh needs its face coordinates"; return DUGKS_EINVAL; }
            if (X[0] != 0.0 || X[c->n[a]] != c->L[a]) {
                why = "custom faces must start at 0 and end at L";
                return DUGKS_EINVAL;
            }
            for (int i = 0; i < c->n[a]; ++i)
                if (!(std::isfinite(X[i + 1]) && X[i + 1] > X[i])) {
                    why = "custom faces must be finite and strictly increasing";
                    return DUGKS_EINVAL;
                }
        }
        const int lo = c->bc[2 * a], hi = c->bc[2 * a + 1];
        for (int s : {lo, hi})
            if (s < DUGKS_PERIODIC || s > DUGKS_BOUNCE_BACK) { why = "unknown boundary kind"; return DUGKS_EINVAL; }
        if ((lo == DUGKS_PERIODIC) != (hi == DUGKS_PERIODIC)) { why = "periodic sides must come in pairs"; return DUGKS_EINVAL; }
        if (lo != DUGKS_PERIODIC && c->n[a] < 2) { why = "wall-bounded axes need at least 2 cells"; return DUGKS_EINVAL; }
    }
    long long cells = 1;
    for (int a = 0; a < D; ++a) cells *= (long long)(c->n[a] + 2);
    if (cells * c->lattice > (1LL << 40)) { why = "problem too large"; return DUGKS_EINVAL; }
    if (c->model != DUGKS_MODEL_INCOMPRESSIBLE && c->model != DUGKS_MODEL_ORIGINAL) { why = "unknown model"; return DUGKS_EINVAL; }
    if (!finite_pos(c->rho0) || !finite_pos(c->RT) || !finite_pos(c->tau) || !finite_pos(c->dt)) {
        why = "rho0, RT, tau, dt must be positive and finite";
        return DUGKS_EINVAL;
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c->G[a])) { why = "non-finite acceleration"; return DUGKS_EINVAL; }
    if (!std::isfinite(c->omega) || !std::isfinite(c->phase)) { why = "non-finite omega/phase"; return DUGKS_EINVAL; }
    for (int s = 0; s < 6; ++s) {
        if (!std::isfinite(c->pw[s]) || !std::isfinite(c->pw_osc[s])) {
            why = "non-finite wall pressure";
            return DUGKS_EINVAL;
        }
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(c->uw[s][a])) { why = "non-finite wall velocity"; return DUGKS_EINVAL; }
    }
    for (int s = 0; s < 2 * D; ++s)
        if (c->bc[s] == DUGKS_NEQ_PRESSURE && c->rho0 + (c->pw[s] - std::fabs(c->pw_osc[s])) / c->RT <= 0) {
            why = "wall pressure gives non-positive density";
            return DUGKS_EINVAL;
        }
    return DUGKS_OK;
}

static void faces_of(const dugks_config* c, int a, std::vector<double>& X)
{
    const int N = c->n[a];
    const double L = c->L[a];
    X.resize(N + 1);
    if (c->mesh[a] == DUGKS_CUSTOM) {
        X.assign(c->faces[a], c->faces[a] + N + 1);
        return;
    }
    for (int i = 0; i <= N; ++i) {
        if (c->mesh[a] == DUGKS_TANH) {
            const double k = c->k_stretch;
            X[i] = L * (0.5 + std::tanh(k * (double(i) / N - 0.5)) / (2.0 * std::tanh(0.5 * k)));
        } else {
            X[i] = L * double(i) / N;
        }
    }
    X[0] = 0.0;
    X[N] = L;
}

// per-axis metric arrays in double (layout of AxisMetric), plus ghost ratios
void axis_metrics(const dugks_config* c, int a, std::vector<double>& out, double& rlo, double& rhi)
{
    const int N = c->n[a];
    const bool per = c->bc[2 * a] == DUGKS_PERIODIC;
    std::vector<double> X;
    faces_of(c, a, X);
    std::vector<double> xc(N + 2);  // xc[i+1] = centre of cell i, i = -1..N
    for (int i = 0; i < N; ++i) xc[i + 1] = 0.5 * (X[i] + X[i + 1]);
    if (per) {
        xc[0] = xc[N] - c->L[a];
        xc[N + 1] = xc[1] + c->L[a];
    } else {
        xc[0] = 2.0 * X[0] - xc[1];
        xc[N + 1] = 2.0 * X[N] - xc[N];
    }
    out.assign(7 * N + 2, 0.0);
    double* w = out.data();
    double* gn = w + (N + 1);
    double* cp = gn + (N + 1);
    double* c0 = cp + N;
    double* cm = c0 + N;
    double* fdx = cm + N;
    double* dl = fdx + N;
    for (int f = 0; f <= N; ++f) {
        const double xl = xc[f], xr = xc[f + 1];  // cells f-1, f
        w[f] = (X[f] - xl) / (xr - xl);
        gn[f] = 1.0 / (xr - xl);
    }
    if (per) {
        w[N] = w[0];
        gn[N] = gn[0];
    }
    for (int i = 0; i < N; ++i) {
        dl[i] = X[i + 1] - X[i];
        cp[i] = w[i + 1] / dl[i];
        c0[i] = (1.0 - w[i + 1] - w[i]) / dl[i];
        cm[i] = -(1.0 - w[i]) / dl[i];
        fdx[i] = c->dt / dl[i];
    }
    rlo = rhi = 0.0;
    if (!per) {
        rlo = (xc[0] - xc[1]) / (xc[2] - xc[1]);
        rhi = (xc[N + 1] - xc[N]) / (xc[N - 1] - xc[N]);
    }
}

double min_width(const dugks_config* c)
{
    const int D = c->lattice == DUGKS_D2Q9 ? 2 : 3;
    double m = 1e300;
    for (int a = 0; a < D; ++a) {
        std::vector<double> X;
        faces_of(c, a, X);
        for (int i = 0; i + 1 < (int)X.size(); ++i) m = std::min(m, X[i + 1] - X[i]);
    }
    return m;
}

// host image of the instance parameters, metric pointers into `met` (device)
template <typename T>
void fill_inst(const dugks_config* c, Inst<T>& P, T* met_dev, std::vector<T>& met_host)
{
    const int D = c->lattice == DUGKS_D2Q9 ? 2 : 3;
    std::memset(&P, 0, sizeof(P));
    size_t tot = 0;
    for (int a = 0; a < 3; ++a) {
        P.n[a] = a < D ? c->n[a] : 1;
        P.E[a] = a < D ? c->n[a] + 2 : 1;
        P.per[a] = a < D ? (c->bc[2 * a] == DUGKS_PERIODIC) : 1;
    }
    for (int s = 0; s < 6; ++s) P.bc[s] = (s / 2 < D) ? c->bc[s] : DUGKS_PERIODIC;
    P.nc = (long long)P.n[0] * P.n[1] * P.n[2];
    P.ne = (long long)P.E[0] * P.E[1] * P.E[2];
    P.off = 0;
    P.foff = -1;
    P.poff = 0;
    const double dt = c->dt, tau = c->tau, h = 0.5 * dt;
    P.rho0 = (T)c->rho0;
    P.RT = (T)c->RT;
    P.c = (T)std::sqrt(3.0 * c->RT);
    P.h = (T)h;
    P.dt = (T)dt;
    P.B1 = (T)(3.0 * h / (2.0 * tau + dt));
    P.C1 = (T)(3.0 * tau * h / (2.0 * tau + dt));
    P.B7 = (T)(h / (2.0 * tau + h));
    P.C7 = (T)(tau * h / (2.0 * tau + h));
    {
        const double b1 = 3.0 * h / (2.0 * tau + dt);
        P.bu_ok = std::fabs(1.0 - b1) >= 0.25 ? 1 : 0;
        P.Bu = P.bu_ok ? (T)(b1 / (3.0 * (1.0 - b1))) : T(0);
    }
    for (int a = 0; a < 3; ++a) P.G0[a] = (T)(a < D ? c->G[a] : 0.0);
    {
        const double cc = std::sqrt(3.0 * c->RT), RT = c->RT, r0 = c->rho0;
        P.crho = (T)(cc / r0);
        P.invRT = (T)(1.0 / RT);
        P.eqH = (T)(r0 / (2.0 * RT));
        P.eqB = (T)(r0 * cc / RT);
        P.eqC = (T)(r0 * cc * cc / (2.0 * RT * RT));
        P.sG = (T)(cc / RT);
        P.orig = c->model == DUGKS_MODEL_ORIGINAL ? 1 : 0;
        P.hRT = (T)(1.0 / (2.0 * RT));
        P.cRT = (T)(cc / RT);
        P.c2RT2 = (T)(cc * cc / (2.0 * RT * RT));
    }
    P.uni = 1;
    for (int a = 0; a < D; ++a) {
        if (c->mesh[a] != DUGKS_UNIFORM) P.uni = 0;
        const double dx = c->L[a] / c->n[a];
        P.ugn[a] = (T)(1.0 / dx);
        P.uct[a] = (T)(0.25 / dx);
        P.ufdx[a] = (T)(dt / dx);
    }
    for (int s = 0; s < 6; ++s) {
        for (int a = 0; a < 3; ++a) P.uw[s][a] = (T)(a < D ? c->uw[s][a] : 0.0);
        P.rhow[s] = (T)(c->rho0 + c->pw[s] / c->RT);
        P.rhowo[s] = (T)(c->pw_osc[s] / c->RT);
    }
    P.omega = c->omega;
    P.phase = c->phase;
    P.dtd = c->dt;
    met_host.clear();
    for (int a = 0; a < D; ++a) {
        std::vector<double> m;
        double rlo, rhi;
        axis_metrics(c, a, m, rlo, rhi);
        P.rlo[a] = (T)rlo;
        P.rhi[a] = (T)rhi;
        const int N = c->n[a];
        T* base = met_dev ? met_dev + tot : nullptr;
        P.m[a].w = base;
        P.m[a].gn = base ? base + (N + 1) : nullptr;
        P.m[a].cp = base ? base + 2 * (N + 1) : nullptr;
        P.m[a].c0 = base ? base + 2 * (N + 1) + N : nullptr;
        P.m[a].cm = base ? base + 2 * (N + 1) + 2 * N : nullptr;
        P.m[a].fdx = base ? base + 2 * (N + 1) + 3 * N : nullptr;
        P.m[a].dl = base ? base + 2 * (N + 1) + 4 * N : nullptr;
        for (double v : m) met_host.push_back((T)v);
        tot += m.size();
    }
}

size_t metric_len(const dugks_config* c)
{
    const int D = c->lattice == DUGKS_D2Q9 ? 2 : 3;
    size_t t = 0;
    for (int a = 0; a < D; ++a) t += 7 * (size_t)c->n[a] + 2;
    return t;
}

template void fill_inst<float>(const dugks_config*, Inst<float>&, float*, std::vector<float>&);
template void fill_inst<double>(const dugks_config*, Inst<double>&, double*, std::vector<double>&);

}  // namespace dugks

extern "C" double dugks_dt_from_cfl(const dugks_config* cfg, double cfl)
{
    std::string why;
    if (validate(cfg, why) != DUGKS_OK || !(cfl > 0)) return -1.0;
    return cfl * min_width(cfg) / std::sqrt(3.0 * cfg->RT);
}

// ---------------------------------------------------------------------------
// single-instance kernels
// ---------------------------------------------------------------------------
namespace dugks {

template <class LAT, typename T, bool ORIG>
__global__ __launch_bounds__(256) void k_phi_one(const Inst<T>* __restrict__ Pp, const T* __restrict__ f, const T* __restrict__ force,
                                                 T* __restrict__ phi, T gt)
{
    const Inst<T>& P = *Pp;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P.ne) return;
    phi_ext_body<LAT, T, ORIG>(P, e, f, force, phi, gt);
}

template <class LAT, typename T, bool ORIG>
__global__ __launch_bounds__(256) void k_update_one(const Inst<T>* __restrict__ Pp, const T* __restrict__ f, const T* __restrict__ force,
                                                    const T* __restrict__ phi, T* __restrict__ fout, T gth)
{
    const Inst<T>& P = *Pp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.nc) return;
    update_body<LAT, T, ORIG>(P, c, f, force, phi, fout, gth);
}

template <class LAT, typename T, bool ORIG>
__global__ __launch_bounds__(256) void k_init_one(const Inst<T>* __restrict__ Pp, const T* rho, const T* u, const T* force, T gt,
                                                  T* fout)
{
    const Inst<T>& P = *Pp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.nc) return;
    init_body<LAT, T, ORIG>(P, c, rho, u, force, gt, fout);
}

// macroscopic fields and per-block partial totals (Eq. macro_values)
template <class LAT, typename T, bool ORIG>
__global__ __launch_bounds__(256) void k_moments_one(const Inst<T>* __restrict__ Pp, const T* __restrict__ f, const T* __restrict__ force,
                                                     T gt, T* rho_o, T* u_o, T* p_o, double* partial)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const Inst<T>& P = *Pp;
    __shared__ double sh[6][256];
    const long long ci = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double loc[6] = {0, 0, 0, 0, 0, 0};
    if (ci < P.nc) {
        int c3[3];
        c3[0] = (int)(ci % P.n[0]);
        long long r = ci / P.n[0];
        c3[1] = (int)(r % P.n[1]);
        c3[2] = (int)(r / P.n[1]);
        double V = 1.0;
        for (int a = 0; a < D; ++a) V *= (double)P.m[a].dl[c3[a]];
        T rho = T(0), j[3] = {T(0), T(0), T(0)};
        int bad = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const T v = f[(long long)q * P.nc + ci];
            if (!isfinite(v)) ++bad;
            rho += v;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (LAT::e(q, a) == 1) j[a] += v;
                if (LAT::e(q, a) == -1) j[a] -= v;
            }
        }
        double k2 = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const T G = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + ci] : T(0)));
            const T ua = vel_from<T, ORIG>(P, rho, j[a], G, P.h);
            if (u_o) u_o[(long long)a * P.nc + ci] = ua;
            k2 += (double)ua * (double)ua;
            loc[1 + a] = V * (double)(P.c * j[a]);
        }
        if (rho_o) rho_o[ci] = rho;
        if (p_o) p_o[ci] = (rho - P.rho0) * P.RT;
        loc[0] = V * (double)rho;
        loc[4] = 0.5 * V * k2;
        loc[5] = (double)bad;
    }
    for (int m = 0; m < 6; ++m) sh[m][threadIdx.x] = loc[m];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int m = 0; m < 6; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int m = 0; m < 6; ++m) partial[(long long)blockIdx.x * 6 + m] = sh[m][0];
}

// fixed-order reduction of the per-block partials (deterministic)
// velocity of cell ci of state f (Eq. macro_values) at time factor gt
template <class LAT, typename T, bool ORIG>
__device__ __forceinline__ void cell_velocity(const Inst<T>& P, const T* __restrict__ f, const T* __restrict__ force,
                                              long long ci, T gt, T* u)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    T rho = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T v = f[(long long)q * P.nc + ci];
        rho += v;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (LAT::e(q, a) == 1) j[a] += v;
            if (LAT::e(q, a) == -1) j[a] -= v;
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T G = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + ci] : T(0)));
        u[a] = vel_from<T, ORIG>(P, rho, j[a], G, P.h);
    }
}

// per-block partial sums of |u_b - u_a|^2 and |u_b|^2 (slots 0 and 1 of 6)
template <class LAT, typename T, bool ORIG>
__global__ __launch_bounds__(256) void k_velocity_change(const Inst<T>* __restrict__ Pp, const T* __restrict__ fa,
                                                         const T* __restrict__ fb, const T* __restrict__ force, T gta,
                                                         T gtb, double* partial)
{
    constexpr int D = LAT::D;
    const Inst<T>& P = *Pp;
    __shared__ double sh[2][256];
    const long long ci = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double d2 = 0.0, b2 = 0.0;
    if (ci < P.nc) {
        T ua[3], ub[3];
        cell_velocity<LAT, T, ORIG>(P, fa, force, ci, gta, ua);
        cell_velocity<LAT, T, ORIG>(P, fb, force, ci, gtb, ub);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double du = (double)ub[a] - (double)ua[a];
            d2 += du * du;
            b2 += (double)ub[a] * (double)ub[a];
        }
    }
    sh[0][threadIdx.x] = d2;
    sh[1][threadIdx.x] = b2;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = partial + (long long)blockIdx.x * 6;
        o[0] = sh[0][0];
        o[1] = sh[1][0];
        o[2] = o[3] = o[4] = o[5] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_reduce6(const double* partial, int nblk, double* out)
{
    __shared__ double sh[6][256];
    double loc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int m = 0; m < 6; ++m) loc[m] += partial[(long long)b * 6 + m];
    for (int m = 0; m < 6; ++m) sh[m][threadIdx.x] = loc[m];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int m = 0; m < 6; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int m = 0; m < 6; ++m) out[m] = sh[m][0];
}

static inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class LAT, typename T>
int launch_step_general(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force,
                        double t, hipStream_t st)
{
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * (double)ctx->cfg.dt);
    if (P.orig) {
        hipLaunchKernelGGL((k_phi_one<LAT, T, true>), dim3(nblocks(P.ne, 256)), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)fin, (const T*)force, (T*)ctx->phi, gt);
        hipLaunchKernelGGL((k_update_one<LAT, T, true>), dim3(nblocks(P.nc, 256)), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)fin, (const T*)force, (const T*)ctx->phi, (T*)fout,
                           gth);
    } else {
        hipLaunchKernelGGL((k_phi_one<LAT, T, false>), dim3(nblocks(P.ne, 256)), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)fin, (const T*)force, (T*)ctx->phi, gt);
        hipLaunchKernelGGL((k_update_one<LAT, T, false>), dim3(nblocks(P.nc, 256)), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)fin, (const T*)force, (const T*)ctx->phi, (T*)fout,
                           gth);
    }
    return hip_check(ctx, hipGetLastError(), "step launch");
}

template <class LAT, typename T>
int launch_init(dugks_ctx* ctx, const Inst<T>& P, const void* rho, const void* u, const void* force, double t0,
                void* fout, hipStream_t st)
{
    if (P.orig)
        hipLaunchKernelGGL((k_init_one<LAT, T, true>), dim3(nblocks(P.nc, 256)), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)rho, (const T*)u, (const T*)force, tfac(P, t0),
                           (T*)fout);
    else
        hipLaunchKernelGGL((k_init_one<LAT, T, false>), dim3(nblocks(P.nc, 256)), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)rho, (const T*)u, (const T*)force, tfac(P, t0),
                           (T*)fout);
    return hip_check(ctx, hipGetLastError(), "init launch");
}

template <class LAT, typename T>
int launch_moments(dugks_ctx* ctx, const Inst<T>& P, const void* f, const void* force, double t, void* rho,
                   void* u, void* p, double* totals, hipStream_t st)
{
    const unsigned nb = nblocks(P.nc, 256);
    if (P.orig)
        hipLaunchKernelGGL((k_moments_one<LAT, T, true>), dim3(nb), dim3(256), 0, st, (const Inst<T>*)ctx->inst_dev,
                           (const T*)f, (const T*)force, tfac(P, t), (T*)rho, (T*)u, (T*)p, ctx->partial);
    else
        hipLaunchKernelGGL((k_moments_one<LAT, T, false>), dim3(nb), dim3(256), 0, st, (const Inst<T>*)ctx->inst_dev,
                           (const T*)f, (const T*)force, tfac(P, t), (T*)rho, (T*)u, (T*)p, ctx->partial);
    hipLaunchKernelGGL(k_reduce6, dim3(1), dim3(256), 0, st, (const double*)ctx->partial, (int)nb, totals);
    return hip_check(ctx, hipGetLastError(), "moments launch");
}

template <class LAT, typename T>
int launch_velocity_change(dugks_ctx* ctx, const Inst<T>& P, const void* fa, const void* fb, const void* force,
                           double ta, double tb, hipStream_t st)
{
    const unsigned nb = nblocks(P.nc, 256);
    if (P.orig)
        hipLaunchKernelGGL((k_velocity_change<LAT, T, true>), dim3(nb), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)fa, (const T*)fb, (const T*)force, tfac(P, ta),
                           tfac(P, tb), ctx->partial);
    else
        hipLaunchKernelGGL((k_velocity_change<LAT, T, false>), dim3(nb), dim3(256), 0, st,
                           (const Inst<T>*)ctx->inst_dev, (const T*)fa, (const T*)fb, (const T*)force, tfac(P, ta),
                           tfac(P, tb), ctx->partial);
    hipLaunchKernelGGL(k_reduce6, dim3(1), dim3(256), 0, st, (const double*)ctx->partial, (int)nb, ctx->totals_dev);
    return hip_check(ctx, hipGetLastError(), "velocity change launch");
}

}  // namespace dugks

// ---------------------------------------------------------------------------
// dispatch on (lattice, dtype)
// ---------------------------------------------------------------------------
#define DUGKS_DISPATCH(ctx, FN, ...)                                                          \
    ((ctx)->cfg.lattice == DUGKS_D2Q9                                                         \
         ? ((ctx)->cfg.dtype == DUGKS_F64 ? FN<D2Q9, double>((ctx), (ctx)->pd, __VA_ARGS__)   \
                                          : FN<D2Q9, float>((ctx), (ctx)->pf, __VA_ARGS__))   \
     : (ctx)->cfg.lattice == DUGKS_D3Q19                                                      \
         ? ((ctx)->cfg.dtype == DUGKS_F64 ? FN<D3Q19, double>((ctx), (ctx)->pd, __VA_ARGS__)  \
                                          : FN<D3Q19, float>((ctx), (ctx)->pf, __VA_ARGS__))  \
         : ((ctx)->cfg.dtype == DUGKS_F64 ? FN<D3Q27, double>((ctx), (ctx)->pd, __VA_ARGS__)  \
                                          : FN<D3Q27, float>((ctx), (ctx)->pf, __VA_ARGS__)))

extern "C" int dugks_init(const dugks_config* cfg, const void* rho, const void* u, const void* force, void* f_out,
                          void* stream, dugks_ctx** out)
{
    if (!out) return fail(nullptr, DUGKS_EINVAL, "null output pointer");
    *out = nullptr;
    std::string why;
    int rc = validate(cfg, why);
    if (rc != DUGKS_OK) return fail(nullptr, rc, why);
    if (!f_out) return fail(nullptr, DUGKS_EINVAL, "null state buffer");
    dugks_ctx* ctx = new dugks_ctx();
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ctx->n_cu = 0;
        ctx->device = dev;
    }
    dugks::adjoint_static_setup();
    ctx->cfg = *cfg;
    for (int a = 0; a < 3; ++a) {
        ctx->cfg.faces[a] = nullptr;
        if (a < (cfg->lattice == DUGKS_D2Q9 ? 2 : 3) && cfg->mesh[a] == DUGKS_CUSTOM) {
            ctx->faces_own[a].assign(cfg->faces[a], cfg->faces[a] + cfg->n[a] + 1);
            ctx->cfg.faces[a] = ctx->faces_own[a].data();
        }
    }
    ctx->D = cfg->lattice == DUGKS_D2Q9 ? 2 : 3;
    ctx->Q = cfg->lattice;
    ctx->esize = cfg->dtype == DUGKS_F64 ? 8 : 4;
    const size_t ml = metric_len(cfg);
    hipError_t e = hipMalloc(&ctx->met, ml * ctx->esize);
    if (e != hipSuccess) { delete ctx; return fail(nullptr, DUGKS_ENOMEM, "metric table allocation failed"); }
    if (cfg->dtype == DUGKS_F64) {
        std::vector<double> mh;
        fill_inst<double>(cfg, ctx->pd, (double*)ctx->met, mh);
        e = hipMemcpy(ctx->met, mh.data(), mh.size() * 8, hipMemcpyHostToDevice);
        ctx->nc = ctx->pd.nc;
        ctx->ne = ctx->pd.ne;
    } else {
        std::vector<float> mh;
        fill_inst<float>(cfg, ctx->pf, (float*)ctx->met, mh);
        e = hipMemcpy(ctx->met, mh.data(), mh.size() * 4, hipMemcpyHostToDevice);
        ctx->nc = ctx->pf.nc;
        ctx->ne = ctx->pf.ne;
    }
    if (e != hipSuccess) { dugks_destroy(ctx); return fail(nullptr, DUGKS_EHIP, "metric upload failed"); }
    {
        const size_t isz = cfg->dtype == DUGKS_F64 ? sizeof(Inst<double>) : sizeof(Inst<float>);
        const void* src = cfg->dtype == DUGKS_F64 ? (const void*)&ctx->pd : (const void*)&ctx->pf;
        if (hipMalloc(&ctx->inst_dev, isz) != hipSuccess) {
            dugks_destroy(ctx);
            return fail(nullptr, DUGKS_ENOMEM, "instance table allocation failed");
        }
        if (hipMemcpy(ctx->inst_dev, src, isz, hipMemcpyHostToDevice) != hipSuccess) {
            dugks_destroy(ctx);
            return fail(nullptr, DUGKS_EHIP, "instance table upload failed");
        }
    }
    ctx->nblk_mom = (int)((ctx->nc + 255) / 256);
    if (hipMalloc(&ctx->partial, (size_t)ctx->nblk_mom * 6 * sizeof(double)) != hipSuccess ||
        hipMalloc(&ctx->totals_dev, 8 * sizeof(double)) != hipSuccess) {
        dugks_destroy(ctx);
        return fail(nullptr, DUGKS_ENOMEM, "reduction scratch allocation failed");
    }
    rc = dugks::setup_fast(ctx);
    if (rc != DUGKS_OK) { std::string m = ctx->err; dugks_destroy(ctx); return fail(nullptr, rc, m); }
    rc = dugks_reset(ctx, rho, u, force, 0.0, f_out, stream);
    if (rc != DUGKS_OK) {
        std::string m = ctx->err;
        dugks_destroy(ctx);
        return fail(nullptr, rc, m);
    }
    *out = ctx;
    return DUGKS_OK;
}

extern "C" int dugks_reset(dugks_ctx* ctx, const void* rho, const void* u, const void* force, double t0,
                           void* f_out, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f_out) return fail(ctx, DUGKS_EINVAL, "null state buffer");
    return DUGKS_DISPATCH(ctx, launch_init, rho, u, force, t0, f_out, (hipStream_t)stream);
}

namespace dugks {
template <class LAT, typename T>
int step_dispatch(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force, double t,
                  hipStream_t st)
{
    bool handled = false;
    const int frc = fast_step(ctx, fin, fout, force, t, st, &handled);
    if (handled) return frc;
    if (!ctx->phi) {
        hipError_t e = hipMalloc(&ctx->phi, (size_t)ctx->ne * ctx->Q * ctx->esize);
        if (e != hipSuccess) {
            ctx->phi = nullptr;
            return fail(ctx, DUGKS_ENOMEM, "scratch allocation failed");
        }
    }
    return launch_step_general<LAT, T>(ctx, P, fin, fout, force, t, st);
}
}  // namespace dugks

extern "C" int dugks_step(dugks_ctx* ctx, const void* f_in, void* f_out, const void* force, double t_n, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f_in || !f_out) return fail(ctx, DUGKS_EINVAL, "null state buffer");
    if (f_in == f_out) return fail(ctx, DUGKS_EINVAL, "f_in and f_out must differ");
    if (!std::isfinite(t_n)) return fail(ctx, DUGKS_EINVAL, "non-finite time");
    return DUGKS_DISPATCH(ctx, step_dispatch, f_in, f_out, force, t_n, (hipStream_t)stream);
}

extern "C" int dugks_run(dugks_ctx* ctx, void* f_a, void* f_b, const void* force, double t0, int nsteps,
                         void* stream, int* which_out)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (nsteps < 0) return fail(ctx, DUGKS_EINVAL, "negative step count");
    void* cur = f_a;
    void* nxt = f_b;
    int which = 0;
    for (int k = 0; k < nsteps; ++k) {
        const int rc = dugks_step(ctx, cur, nxt, force, t0 + k * ctx->cfg.dt, stream);
        if (rc != DUGKS_OK) return rc;
        void* tmp = cur;
        cur = nxt;
        nxt = tmp;
        which ^= 1;
    }
    if (which_out) *which_out = which;
    return DUGKS_OK;
}

extern "C" int dugks_moments(dugks_ctx* ctx, const void* f, const void* force, double t, void* rho, void* u,
                             void* p, double* totals_host, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f) return fail(ctx, DUGKS_EINVAL, "null state buffer");
    const hipStream_t st = (hipStream_t)stream;
    int rc = DUGKS_DISPATCH(ctx, launch_moments, f, force, t, rho, u, p, ctx->totals_dev, st);
    if (rc != DUGKS_OK) return rc;
    if (totals_host) {
        double tmp[8];
        rc = hip_check(ctx, hipMemcpyAsync(tmp, ctx->totals_dev, 6 * sizeof(double), hipMemcpyDeviceToHost, st),
                       "totals copy");
        if (rc != DUGKS_OK) return rc;
        rc = hip_check(ctx, hipStreamSynchronize(st), "moments synchronise");
        if (rc != DUGKS_OK) return rc;
        for (int m = 0; m < 6; ++m) totals_host[m] = tmp[m];
        if (tmp[5] != 0.0) return fail(ctx, DUGKS_ENONFINITE, "non-finite values in the state");
    }
    return DUGKS_OK;
}

extern "C" int dugks_totals_async(dugks_ctx* ctx, const void* f, const void* force, double t, double* totals_dev,
                                  void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f || !totals_dev) return fail(ctx, DUGKS_EINVAL, "null buffer");
    return DUGKS_DISPATCH(ctx, launch_moments, f, force, t, nullptr, nullptr, nullptr, totals_dev, (hipStream_t)stream);
}

extern "C" int dugks_velocity_change(dugks_ctx* ctx, const void* f_a, const void* f_b, const void* force, double t_a,
                                     double t_b, double* out_host, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f_a || !f_b || !out_host) return fail(ctx, DUGKS_EINVAL, "null buffer");
    const hipStream_t st = (hipStream_t)stream;
    int rc = DUGKS_DISPATCH(ctx, launch_velocity_change, f_a, f_b, force, t_a, t_b, st);
    if (rc != DUGKS_OK) return rc;
    double tmp[8];
    rc = hip_check(ctx, hipMemcpyAsync(tmp, ctx->totals_dev, 6 * sizeof(double), hipMemcpyDeviceToHost, st),
                   "monitor copy");
    if (rc != DUGKS_OK) return rc;
    rc = hip_check(ctx, hipStreamSynchronize(st), "monitor synchronise");
    if (rc != DUGKS_OK) return rc;
    out_host[0] = std::sqrt(tmp[0]);
    out_host[1] = std::sqrt(tmp[1]);
    if (!std::isfinite(out_host[0]) || !std::isfinite(out_host[1]))
        return fail(ctx, DUGKS_ENONFINITE, "non-finite velocity in a state");
    return DUGKS_OK;
}

namespace dugks {
int resolve_step_kernel(const dugks_ctx* ctx, bool field);
}
extern "C" int dugks_kernel_variant(const dugks_ctx* ctx) { return ctx ? dugks::resolve_step_kernel(ctx, false) : -1; }

extern "C" void dugks_destroy(dugks_ctx* ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    if (ctx->met) (void)hipFree(ctx->met);
    if (ctx->inst_dev) (void)hipFree(ctx->inst_dev);
    if (ctx->phi) (void)hipFree(ctx->phi);
    if (ctx->partial) (void)hipFree(ctx->partial);
    if (ctx->totals_dev) (void)hipFree(ctx->totals_dev);
    dugks::release_fast(ctx);
    dugks::release_adjoint(ctx);
    delete ctx;
}
