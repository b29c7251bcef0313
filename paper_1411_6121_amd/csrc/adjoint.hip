// adjoint.hip -- reverse mode of one step on a fully periodic mesh, and of
// the initial state; gather form (no atomics), forward intermediates
// recomputed from f_n (no tape).
//
// Forward, per interface b of axis a between cells L and R (step 4 written
// through the cell quantities psi_a(c) = phi(c) - h sum_{t!=a} xi_t d_t(c),
// d_t the cell-centred derivative d_t(c) = cp phi(c+t) + c0 phi(c) + cm phi(c-t)):
//   fbar(b) = (1-w) psi_a(L) + w psi_a(R) - h xi_a g (phi(R) - phi(L)).
// Reverse, with lam the adjoint of f_{n+1}:
//   pass A (per cell R, axis a: its lower face b): recompute fbar(b), its
//     moments and the original f(b); adjoint of the flux terms
//     fhat_q = xi_{q,a} (dt/Delta(R) lam_q(R) - dt/Delta(L) lam_q(L)), of step 7
//     and of the moments -> fbar_hat(b) (all q) and G_hat(b);
//   pass B (per cell): psi_hat_a from the two faces of each axis, the normal
//     terms, d_hat_t = -h xi_t sum_{a!=t} psi_hat_a, and the local part of
//     phi_hat (incl. 4/3 lam from Eq. f_tilde_+);
//   pass C (per cell): phi_hat += cp_t(s-t) d_hat_t(s-t) + cm_t(s+t) d_hat_t(s+t);
//     reverse of Eq. (f_bar_+) and of the macroscopic recovery -> lam_n and
//     the force-field gradient (cell term at t_n, face terms at t_n + h).
#include <hip/hip_runtime.h>

#include "ctx.hpp"
#include "kernels_general.hpp"

namespace dugks {

// d feq_q / d(rho, u) and d S_q / d(rho, u, G) at one point
template <class LAT, typename T>
struct Partials {
    T fe, dfe_dr, dS_dr, dfe_du[3], dS_du[3], dS_dG[3];
};

template <class LAT, typename T>
__device__ __forceinline__ Partials<LAT, T> partials(int q, T rho, const T* u, const T* G, T rho0, T c, T invRT)
{
    constexpr int D = LAT::D;
    Partials<LAT, T> r;
    T xu = T(0), gx = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T xi = xi_of<LAT, T>(q, a, c);
        xu += xi * u[a];
        gx += G[a] * (xi - u[a]);
    }
    const T W = T(LAT::w(q));
    r.fe = feq_q<LAT, T>(q, rho, u, rho0, c, invRT);
    r.dfe_dr = W;
    r.dS_dr = gx * invRT * W;
#pragma unroll
    for (int a = 0; a < 3; ++a) { r.dfe_du[a] = T(0); r.dS_du[a] = T(0); r.dS_dG[a] = T(0); }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T xi = xi_of<LAT, T>(q, a, c);
        r.dfe_du[a] = W * rho0 * invRT * (xi + xu * xi * invRT - u[a]);
        r.dS_du[a] = -G[a] * invRT * r.fe + gx * invRT * r.dfe_du[a];
        r.dS_dG[a] = (xi - u[a]) * invRT * r.fe;
    }
    return r;
}

template <typename T>
__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// pass A: adjoint of the lower face of cell R along axis A
template <class LAT, typename T, int A>
__device__ __forceinline__ void adj_face_body(const Inst<T>& P, long long cidx, const T* __restrict__ phi,
                                              const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                              T* __restrict__ fa, T* __restrict__ ga)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    const long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    GlobalPhi<LAT, T> ph{phi, P.ne, ext_idx<LAT, T>(P, ci[0], ci[1], ci[2]), (long long)P.E[0],
                         (long long)P.E[0] * P.E[1]};
    const CellMetric<T> cx = load_metric(P, 0, ci[0]);
    const CellMetric<T> cy = load_metric(P, 1, ci[1]);
    const CellMetric<T> cz = D == 3 ? load_metric(P, 2, ci[2]) : cy;
    const CellMetric<T>& ma = A == 0 ? cx : (A == 1 ? cy : cz);
    T fb[Q], G[3];
    recon_face_ct<LAT, T, GlobalPhi<LAT, T>, A>(P, ph, false, ma, cx, cy, cz, fb);
    face_force<LAT, T>(P, force, A, ci[A], ma.wl, ci, gth, G);
    T rho, u[3];
    face_moments<LAT, T>(P, fb, G, rho, u);
    // left cell (periodic wrap) and flux scales of both cells
    int cl[3] = {ci[0], ci[1], ci[2]};
    cl[A] = wrapc<T>(ci[A] - 1, P.n[A]);
    const long long lidx = int_idx(P, cl[0], cl[1], cl[2]);
    const T sR = ma.fdx;
    const T sL = P.m[A].fdx[cl[A]];
    const T invRT = T(1) / P.RT;
    T rb = T(0), ub[3] = {T(0), T(0), T(0)}, Gb[3] = {T(0), T(0), T(0)}, fh[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        fh[q] = T(0);
        if (LAT::e(q, A) == 0) continue;
        fh[q] = T(LAT::e(q, A)) * P.c * (sR * lam[(long long)q * P.nc + cidx] - sL * lam[(long long)q * P.nc + lidx]);
        const Partials<LAT, T> pd = partials<LAT, T>(q, rho, u, G, P.rho0, P.c, invRT);
        rb += fh[q] * (P.B7 * pd.dfe_dr + P.C7 * pd.dS_dr);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ub[d] += fh[q] * (P.B7 * pd.dfe_du[d] + P.C7 * pd.dS_du[d]);
            Gb[d] += fh[q] * P.C7 * pd.dS_dG[d];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) Gb[d] += T(0.5) * P.h * ub[d];
    const long long stride = (long long)Q * P.nc;  // per axis block of fa
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T v = (T(1) - P.B7) * fh[q] + rb;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (LAT::e(q, d) == 1) v += P.c / P.rho0 * ub[d];
            if (LAT::e(q, d) == -1) v -= P.c / P.rho0 * ub[d];
        }
        fa[A * stride + (long long)q * P.nc + cidx] = v;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) ga[((long long)A * D + d) * P.nc + cidx] = Gb[d];
}

template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adj_face(const Inst<T>* __restrict__ Pp, const T* __restrict__ phi,
                                                  const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                                  T* __restrict__ fa, T* __restrict__ ga)
{
    const Inst<T>& P = *Pp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.nc) return;
    const int a = blockIdx.y;
    if (a == 0) adj_face_body<LAT, T, 0>(P, c, phi, force, lam, gth, fa, ga);
    else if (a == 1) adj_face_body<LAT, T, 1>(P, c, phi, force, lam, gth, fa, ga);
    else if constexpr (LAT::D == 3) adj_face_body<LAT, T, 2>(P, c, phi, force, lam, gth, fa, ga);
}

// pass B
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adj_cell1(const Inst<T>* __restrict__ Pp, const T* __restrict__ lam,
                                                   const T* __restrict__ fa, T* __restrict__ ph_out,
                                                   T* __restrict__ dt_out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const Inst<T>& P = *Pp;
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= P.nc) return;
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    const long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    const long long stride = (long long)Q * P.nc;
    T psi[3][Q];
    T phat[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) phat[q] = T(4.0 / 3.0) * lam[(long long)q * P.nc + cidx];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const CellMetric<T> m = load_metric(P, a, ci[a]);
        int cu[3] = {ci[0], ci[1], ci[2]};
        cu[a] = wrapc<T>(ci[a] + 1, P.n[a]);
        const long long uidx = int_idx(P, cu[0], cu[1], cu[2]);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const T flo = fa[a * stride + (long long)q * P.nc + cidx];  // lower face (this cell is R)
            const T fup = fa[a * stride + (long long)q * P.nc + uidx];  // upper face (this cell is L)
            psi[a][q] = m.wl * flo + (T(1) - m.wu) * fup;
            phat[q] += psi[a][q] + T(LAT::e(q, a)) * P.h * P.c * (m.gu * fup - m.gl * flo);
        }
    }
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const CellMetric<T> m = load_metric(P, t, ci[t]);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T dh = T(0);
            if (LAT::e(q, t) != 0) {
                T s = T(0);
#pragma unroll
                for (int a = 0; a < D; ++a)
                    if (a != t) s += psi[a][q];
                dh = -P.h * P.c * T(LAT::e(q, t)) * s;
            }
            phat[q] += m.c0 * dh;
            dt_out[t * stride + (long long)q * P.nc + cidx] = dh;
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) ph_out[(long long)q * P.nc + cidx] = phat[q];
}

// pass C
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adj_cell2(const Inst<T>* __restrict__ Pp, const T* __restrict__ f,
                                                   const T* __restrict__ force, const T* __restrict__ lam,
                                                   const T* __restrict__ ph_in, const T* __restrict__ dt_in,
                                                   const T* __restrict__ ga, T gt, T gth, T* __restrict__ lam_out,
                                                   T* __restrict__ grad_force)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const Inst<T>& P = *Pp;
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= P.nc) return;
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    const long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    const long long stride = (long long)Q * P.nc;
    T phat[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) phat[q] = ph_in[(long long)q * P.nc + cidx];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        int cm_[3] = {ci[0], ci[1], ci[2]}, cp_[3] = {ci[0], ci[1], ci[2]};
        cm_[t] = wrapc<T>(ci[t] - 1, P.n[t]);
        cp_[t] = wrapc<T>(ci[t] + 1, P.n[t]);
        const long long im = int_idx(P, cm_[0], cm_[1], cm_[2]), ip = int_idx(P, cp_[0], cp_[1], cp_[2]);
        const T cpm = P.m[t].cp[cm_[t]];  // cp of the cell below: its d_t uses this cell as +t neighbour
        const T cmp = P.m[t].cm[cp_[t]];  // cm of the cell above
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (LAT::e(q, t) == 0) continue;
            phat[q] += cpm * dt_in[t * stride + (long long)q * P.nc + im] +
                       cmp * dt_in[t * stride + (long long)q * P.nc + ip];
        }
    }
    // forward cell quantities (step 1)
    const T invRT = T(1) / P.RT;
    T fv[Q], rho = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        fv[q] = f[(long long)q * P.nc + cidx];
        rho += fv[q];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (LAT::e(q, a) == 1) j[a] += fv[q];
            if (LAT::e(q, a) == -1) j[a] -= fv[q];
        }
    }
    T G[3] = {T(0), T(0), T(0)}, u[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        G[a] = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + cidx] : T(0)));
        u[a] = P.c * j[a] / P.rho0 + P.h * G[a];
    }
    T rb = T(0), ub[3] = {T(0), T(0), T(0)}, Gc[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const Partials<LAT, T> pd = partials<LAT, T>(q, rho, u, G, P.rho0, P.c, invRT);
        rb += phat[q] * (P.B1 * pd.dfe_dr + P.C1 * pd.dS_dr);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ub[d] += phat[q] * (P.B1 * pd.dfe_du[d] + P.C1 * pd.dS_du[d]);
            Gc[d] += phat[q] * P.C1 * pd.dS_dG[d];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) Gc[d] += P.h * ub[d];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T v = (T(1) - P.B1) * phat[q] + rb - T(1.0 / 3.0) * lam[(long long)q * P.nc + cidx];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (LAT::e(q, d) == 1) v += P.c / P.rho0 * ub[d];
            if (LAT::e(q, d) == -1) v -= P.c / P.rho0 * ub[d];
        }
        lam_out[(long long)q * P.nc + cidx] = v;
    }
    if (grad_force) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T gsum = gt * Gc[d];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const CellMetric<T> m = load_metric(P, a, ci[a]);
                int cu[3] = {ci[0], ci[1], ci[2]};
                cu[a] = wrapc<T>(ci[a] + 1, P.n[a]);
                const long long uidx = int_idx(P, cu[0], cu[1], cu[2]);
                gsum += gth * (m.wl * ga[((long long)a * D + d) * P.nc + cidx] +
                               (T(1) - m.wu) * ga[((long long)a * D + d) * P.nc + uidx]);
            }
            grad_force[(long long)d * P.nc + cidx] += gsum;
        }
    }
}

// reverse of the initial state (rho = rho0)
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_init_vjp(const Inst<T>* __restrict__ Pp, const T* __restrict__ u,
                                                  const T* __restrict__ force, const T* __restrict__ lam0, T gt,
                                                  T* __restrict__ grad_u, T* __restrict__ grad_force)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const Inst<T>& P = *Pp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.nc) return;
    const T invRT = T(1) / P.RT;
    T uu[3] = {T(0), T(0), T(0)}, G[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (u) uu[a] = u[(long long)a * P.nc + c];
        G[a] = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + c] : T(0)));
    }
    T gu[3] = {T(0), T(0), T(0)}, gG[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const Partials<LAT, T> pd = partials<LAT, T>(q, P.rho0, uu, G, P.rho0, P.c, invRT);
        const T l = lam0[(long long)q * P.nc + c];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            gu[a] += l * (pd.dfe_du[a] - P.h * pd.dS_du[a]);
            gG[a] += l * (-P.h * pd.dS_dG[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (grad_u) grad_u[(long long)a * P.nc + c] += gu[a];
        if (grad_force) grad_force[(long long)a * P.nc + c] += gt * gG[a];
    }
}

// reverse of the macroscopic read-out (Eq. macro_values)
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_moments_vjp(const Inst<T>* __restrict__ Pp, const T* __restrict__ grho,
                                                     const T* __restrict__ gu, T gt, T* __restrict__ lam,
                                                     T* __restrict__ grad_force)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const Inst<T>& P = *Pp;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.nc) return;
    const T r = grho ? grho[c] : T(0);
    T g[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < D; ++d) g[d] = gu ? gu[(long long)d * P.nc + c] : T(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T v = r;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (LAT::e(q, d) == 1) v += P.c / P.rho0 * g[d];
            if (LAT::e(q, d) == -1) v -= P.c / P.rho0 * g[d];
        }
        lam[(long long)q * P.nc + c] = v;
    }
    if (grad_force)
#pragma unroll
        for (int d = 0; d < D; ++d) grad_force[(long long)d * P.nc + c] += gt * P.h * g[d];
}

template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_phi_adj(const Inst<T>* __restrict__ Pp, const T* __restrict__ f,
                                                 const T* __restrict__ force, T* __restrict__ phi, T gt)
{
    const Inst<T>& P = *Pp;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P.ne) return;
    phi_ext_body<LAT, T>(P, e, f, force, phi, gt);
}

static inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

template <class LAT, typename T>
static int adjoint_step(dugks_ctx* ctx, const Inst<T>& P, const void* fn, const void* force, double t,
                        const void* lam_np1, void* lam_n, void* grad_force, hipStream_t st)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const size_t es = sizeof(T);
    const size_t need = (size_t)P.ne * Q * es              // phi (extended)
                        + (size_t)D * Q * P.nc * es          // face adjoints
                        + (size_t)D * D * P.nc * es          // face force adjoints
                        + (size_t)Q * P.nc * es              // phi_hat partial
                        + (size_t)D * Q * P.nc * es;         // d_hat
    if (ctx->adj_bytes < need) {
        if (ctx->adj) (void)hipFree(ctx->adj);
        ctx->adj = nullptr;
        ctx->adj_bytes = 0;
        if (hipMalloc(&ctx->adj, need) != hipSuccess) return fail(ctx, DUGKS_ENOMEM, "adjoint scratch allocation failed");
        ctx->adj_bytes = need;
    }
    T* base = (T*)ctx->adj;
    T* phi = base;
    T* fa = phi + (size_t)P.ne * Q;
    T* ga = fa + (size_t)D * Q * P.nc;
    T* ph = ga + (size_t)D * D * P.nc;
    T* dh = ph + (size_t)Q * P.nc;
    const Inst<T>* Pd = (const Inst<T>*)ctx->inst_dev;
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * (double)ctx->cfg.dt);
    hipLaunchKernelGGL((k_phi_adj<LAT, T>), dim3(nb256(P.ne)), dim3(256), 0, st, Pd, (const T*)fn, (const T*)force,
                       phi, gt);
    hipLaunchKernelGGL((k_adj_face<LAT, T>), dim3(nb256(P.nc), D), dim3(256), 0, st, Pd, (const T*)phi,
                       (const T*)force, (const T*)lam_np1, gth, fa, ga);
    hipLaunchKernelGGL((k_adj_cell1<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, Pd, (const T*)lam_np1,
                       (const T*)fa, ph, dh);
    hipLaunchKernelGGL((k_adj_cell2<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, Pd, (const T*)fn,
                       (const T*)force, (const T*)lam_np1, (const T*)ph, (const T*)dh, (const T*)ga, gt, gth,
                       (T*)lam_n, (T*)grad_force);
    return hip_check(ctx, hipGetLastError(), "adjoint launch");
}

template <class LAT, typename T>
static int init_vjp(dugks_ctx* ctx, const Inst<T>& P, const void* u, const void* force, double t0, const void* lam0,
                    void* grad_u, void* grad_force, hipStream_t st)
{
    hipLaunchKernelGGL((k_init_vjp<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, (const Inst<T>*)ctx->inst_dev,
                       (const T*)u, (const T*)force, (const T*)lam0, tfac(P, t0), (T*)grad_u, (T*)grad_force);
    return hip_check(ctx, hipGetLastError(), "init vjp launch");
}

template <class LAT, typename T>
static int moments_vjp(dugks_ctx* ctx, const Inst<T>& P, const void* grho, const void* gu, double t, void* lam,
                       void* grad_force, hipStream_t st)
{
    hipLaunchKernelGGL((k_moments_vjp<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, (const Inst<T>*)ctx->inst_dev,
                       (const T*)grho, (const T*)gu, tfac(P, t), (T*)lam, (T*)grad_force);
    return hip_check(ctx, hipGetLastError(), "moments vjp launch");
}

void release_adjoint(dugks_ctx* ctx)
{
    if (ctx->adj) (void)hipFree(ctx->adj);
    ctx->adj = nullptr;
    ctx->adj_bytes = 0;
}

}  // namespace dugks

using namespace dugks;

extern "C" int dugks_step_adjoint(dugks_ctx* ctx, const void* f_n, const void* force, double t_n,
                                  const void* lam_np1, void* lam_n, void* grad_force, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f_n || !lam_np1 || !lam_n) return fail(ctx, DUGKS_EINVAL, "null buffer");
    if (ctx->cfg.model != DUGKS_MODEL_INCOMPRESSIBLE)
        return fail(ctx, DUGKS_EUNSUPPORTED, "the adjoint is derived for the incompressible model");
    if (ctx->cfg.lattice == DUGKS_D3Q27) return fail(ctx, DUGKS_EUNSUPPORTED, "no D3Q27 adjoint");
    if (lam_n == f_n || lam_n == lam_np1) return fail(ctx, DUGKS_EINVAL, "lam_n must not alias f_n or lam_np1");
    for (int s = 0; s < 2 * ctx->D; ++s)
        if (ctx->cfg.bc[s] != DUGKS_PERIODIC)
            return fail(ctx, DUGKS_EUNSUPPORTED, "the adjoint step supports fully periodic meshes only");
    const hipStream_t st = (hipStream_t)stream;
    if (ctx->cfg.lattice == DUGKS_D2Q9) {
        if (ctx->cfg.dtype == DUGKS_F64) return adjoint_step<D2Q9, double>(ctx, ctx->pd, f_n, force, t_n, lam_np1, lam_n, grad_force, st);
        return adjoint_step<D2Q9, float>(ctx, ctx->pf, f_n, force, t_n, lam_np1, lam_n, grad_force, st);
    }
    if (ctx->cfg.dtype == DUGKS_F64) return adjoint_step<D3Q19, double>(ctx, ctx->pd, f_n, force, t_n, lam_np1, lam_n, grad_force, st);
    return adjoint_step<D3Q19, float>(ctx, ctx->pf, f_n, force, t_n, lam_np1, lam_n, grad_force, st);
}

extern "C" int dugks_init_vjp(dugks_ctx* ctx, const void* u, const void* force, double t0, const void* lam0,
                              void* grad_u, void* grad_force, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!lam0) return fail(ctx, DUGKS_EINVAL, "null adjoint state");
    if (ctx->cfg.model != DUGKS_MODEL_INCOMPRESSIBLE)
        return fail(ctx, DUGKS_EUNSUPPORTED, "the adjoint is derived for the incompressible model");
    if (ctx->cfg.lattice == DUGKS_D3Q27) return fail(ctx, DUGKS_EUNSUPPORTED, "no D3Q27 adjoint");
    const hipStream_t st = (hipStream_t)stream;
    if (ctx->cfg.lattice == DUGKS_D2Q9) {
        if (ctx->cfg.dtype == DUGKS_F64) return init_vjp<D2Q9, double>(ctx, ctx->pd, u, force, t0, lam0, grad_u, grad_force, st);
        return init_vjp<D2Q9, float>(ctx, ctx->pf, u, force, t0, lam0, grad_u, grad_force, st);
    }
    if (ctx->cfg.dtype == DUGKS_F64) return init_vjp<D3Q19, double>(ctx, ctx->pd, u, force, t0, lam0, grad_u, grad_force, st);
    return init_vjp<D3Q19, float>(ctx, ctx->pf, u, force, t0, lam0, grad_u, grad_force, st);
}

extern "C" int dugks_moments_vjp(dugks_ctx* ctx, const void* grad_rho, const void* grad_u, double t, void* lam,
                                 void* grad_force, void* stream)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!lam) return fail(ctx, DUGKS_EINVAL, "null adjoint state");
    if (ctx->cfg.model != DUGKS_MODEL_INCOMPRESSIBLE)
        return fail(ctx, DUGKS_EUNSUPPORTED, "the adjoint is derived for the incompressible model");
    if (ctx->cfg.lattice == DUGKS_D3Q27) return fail(ctx, DUGKS_EUNSUPPORTED, "no D3Q27 adjoint");
    const hipStream_t st = (hipStream_t)stream;
    if (ctx->cfg.lattice == DUGKS_D2Q9) {
        if (ctx->cfg.dtype == DUGKS_F64) return moments_vjp<D2Q9, double>(ctx, ctx->pd, grad_rho, grad_u, t, lam, grad_force, st);
        return moments_vjp<D2Q9, float>(ctx, ctx->pf, grad_rho, grad_u, t, lam, grad_force, st);
    }
    if (ctx->cfg.dtype == DUGKS_F64) return moments_vjp<D3Q19, double>(ctx, ctx->pd, grad_rho, grad_u, t, lam, grad_force, st);
    return moments_vjp<D3Q19, float>(ctx, ctx->pf, grad_rho, grad_u, t, lam, grad_force, st);
}
