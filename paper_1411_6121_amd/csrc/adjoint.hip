// adjoint.hip -- reverse mode of one step on a fully periodic mesh, and of
// the initial state; gather form (no atomics), forward intermediates
// recomputed from f_n (no tape).
//
// Forward, per interface b of axis a between cells L and R (Eq. gradient written
// through the cell quantities psi_a(c) = phi(c) - h sum_{t!=a} xi_t d_t(c),
// d_t the cell-centred derivative d_t(c) = cp phi(c+t) + c0 phi(c) + cm phi(c-t)):
//   fbar(b) = (1-w) psi_a(L) + w psi_a(R) - h xi_a g (phi(R) - phi(L)).
// Reverse, with lam the adjoint of f_{n+1}:
//   pass A (per cell R, axis a: its lower face b): recompute fbar(b), its
//     moments and the original f(b); adjoint of the flux terms
//     fhat_q = xi_{q,a} (dt/Delta(R) lam_q(R) - dt/Delta(L) lam_q(L)), of Eq. (original_f)
//     and of the moments -> fbar_hat(b) (all q) and G_hat(b);
//   pass B (per cell): psi_hat_a from the two faces of each axis, the normal
//     terms, d_hat_t = -h xi_t sum_{a!=t} psi_hat_a, and the local part of
//     phi_hat (incl. 4/3 lam from Eq. f_tilde_+);
//   pass C (per cell): phi_hat += cp_t(s-t) d_hat_t(s-t) + cm_t(s+t) d_hat_t(s+t);
//     reverse of Eq. (f_bar_+) and of the macroscopic recovery -> lam_n and
//     the force-field gradient (cell term at t_n, face terms at t_n + h).
// For the 2-D sets passes B and C run as one launch over cell tiles whose
// d_hat (halo included) is formed in LDS, so a step reads and writes main
// memory in three passes (phi, faces, cells) instead of four.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <utility>

#include "ctx.hpp"
#include "kernels_general.hpp"
#include "march.hpp"

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

// pass A: adjoint of the lower face of cell R (coordinates ci, index cidx)
// along axis A; ph reads f-bar-plus around the cell
template <class LAT, typename T, int A, class ACC>
__device__ __forceinline__ void adj_face_core(const Inst<T>& P, const int* ci, long long cidx, const ACC& ph,
                                              const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                              T* __restrict__ fa, T* __restrict__ ga)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const CellMetric<T> cx = load_metric(P, 0, ci[0]);
    const CellMetric<T> cy = load_metric(P, 1, ci[1]);
    const CellMetric<T> cz = D == 3 ? load_metric(P, 2, ci[2]) : cy;
    const CellMetric<T>& ma = A == 0 ? cx : (A == 1 ? cy : cz);
    T fb[Q], G[3];
    recon_face_ct<LAT, T, ACC, A>(P, ph, false, ma, cx, cy, cz, fb);
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

// the same with f-bar-plus from the ghost-extended array in memory
template <class LAT, typename T, int A>
__device__ __forceinline__ void adj_face_body(const Inst<T>& P, long long cidx, const T* __restrict__ phi,
                                              const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                              T* __restrict__ fa, T* __restrict__ ga)
{
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    const long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    GlobalPhi<LAT, T> ph{phi, P.ne, ext_idx<LAT, T>(P, ci[0], ci[1], ci[2]), (long long)P.E[0],
                         (long long)P.E[0] * P.E[1]};
    adj_face_core<LAT, T, A>(P, ci, cidx, ph, force, lam, gth, fa, ga);
}

template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adj_face(const Inst<T>* __restrict__ Pp, const T* __restrict__ phi,
                                                  const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                                  T* __restrict__ fa, T* __restrict__ ga)
{
    // one axis per grid row (blockIdx.y)
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

// reverse of Eq. (f_bar_+) at the cell and of the macroscopic recovery
// (Eqs. macro_values, f_bar_+), given the cell's complete phi-hat: lam_n = phi-hat terms - 1/3
// lam_{n+1} (Eq. f_tilde_+), and the force-field gradient (cell term at t_n,
// face terms at t_n + h from the face adjoints ga)
template <class LAT, typename T>
__device__ __forceinline__ void adj_cell_finish(const Inst<T>& P, const int* ci, long long cidx, T (&phat)[LAT::Q],
                                                const T* __restrict__ f, const T* __restrict__ force,
                                                const T* __restrict__ lam, const T* __restrict__ ga, T gt, T gth,
                                                T* __restrict__ lam_out, T* __restrict__ grad_force)
{
    constexpr int Q = LAT::Q, D = LAT::D;
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
    adj_cell_finish<LAT, T>(P, ci, cidx, phat, f, force, lam, ga, gt, gth, lam_out, grad_force);
}

// passes B and C in one launch for the 2-D sets: a workgroup owns a tile of
// ADJ_TX x ADJ_TY cells, one per thread.  Each thread forms its cell's local
// phi-hat (kept in registers) and d_hat (to LDS); the d_hat of the one-cell
// halo, which the tile's edge cells need from their outer neighbours, is
// formed velocity by velocity by all threads; then each cell adds its
// neighbours' d_hat from LDS.  No phi-hat or d_hat arrays in memory; the
// same operations in the same order as the two passes.
constexpr int ADJ_TX = 32, ADJ_TY = 8;

// slot of velocity q among those with e(q, t) != 0, their count, and the
// velocity of a slot
template <class LAT>
__host__ __device__ constexpr int adj_slot(int q, int t)
{
    int s = 0;
    for (int r = 0; r < q; ++r)
        if (LAT::e(r, t) != 0) ++s;
    return s;
}
template <class LAT>
__host__ __device__ constexpr int adj_nslot(int t)
{
    return adj_slot<LAT>(LAT::Q, t);
}
template <class LAT>
__host__ __device__ constexpr int adj_q_of_slot(int t, int slot)
{
    for (int q = 0; q < LAT::Q; ++q)
        if (LAT::e(q, t) != 0 && adj_slot<LAT>(q, t) == slot) return q;
    return -1;
}

__device__ __forceinline__ int wrap_any(int i, int n) { return ((i % n) + n) % n; }

template <class LAT, typename T>
__global__ __attribute__((amdgpu_flat_work_group_size(1, ADJ_TX * ADJ_TY), amdgpu_waves_per_eu(4))) void k_adj_cell_tile(
    const Inst<T>* __restrict__ Pp, const T* __restrict__ f, const T* __restrict__ force, const T* __restrict__ lam,
    const T* __restrict__ fa, const T* __restrict__ ga, T gt, T gth, int tiles_x, T* __restrict__ lam_out,
    T* __restrict__ grad_force)
{
    static_assert(LAT::D == 2, "2-D sets only");
    constexpr int Q = LAT::Q, D = 2;
    constexpr int RX = ADJ_TX + 2, RY = ADJ_TY + 2, NR = RX * RY, NC = ADJ_TX * ADJ_TY;
    constexpr int NS0 = adj_nslot<LAT>(0), NS1 = adj_nslot<LAT>(1);
    constexpr int NS = NS0 > NS1 ? NS0 : NS1;
    __shared__ T dts[D][NS][NR];  // d_hat_t of the region's cells, velocities with e_t != 0
    const Inst<T>& P = *Pp;
    const long long stride = (long long)Q * P.nc;
    // tiles in XCD order: each XCD takes a contiguous range of tile rows, so
    // tiles sharing halo lines read them through one L2
    const int b = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int x0 = (b % tiles_x) * ADJ_TX, y0 = (b / tiles_x) * ADJ_TY;
    const int tx = (int)threadIdx.x % ADJ_TX, ty = (int)threadIdx.x / ADJ_TX;
    const int rc = (ty + 1) * RX + (tx + 1);  // this thread's cell in the region
    // the thread's cell (the wrapped coordinates past a ragged mesh edge:
    // there the slot serves as halo of the cells before it)
    const int ci[3] = {wrap_any(x0 + tx, P.n[0]), wrap_any(y0 + ty, P.n[1]), 0};
    const bool own = x0 + tx < P.n[0] && y0 + ty < P.n[1];
    const long long cidx = int_idx(P, ci[0], ci[1], ci[2]);
    T phat[Q];
    // (a one-trip loop: a scheduling region of its own, which keeps the
    // compiler from hoisting later stages' loads into it; fewer registers)
#pragma unroll 1
    for (int once = (int)threadIdx.x; once < NC; once += NC) {
        T psi[D][Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) phat[q] = T(4.0 / 3.0) * lam[(long long)q * P.nc + cidx];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            asm volatile("" ::: "memory");  // one axis's face adjoints in flight at a time
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
                    dts[t][adj_slot<LAT>(q, t)][rc] = dh;
                }
                phat[q] += m.c0 * dh;
            }
        }
    }
    // halo: the left/right columns need d_hat_0, the bottom/top rows d_hat_1
    // (corners are nobody's neighbour); one velocity per item.  (The memory
    // clobbers keep the compiler from hoisting the loads of later stages
    // here, which would only hold registers.)
    asm volatile("" ::: "memory");
    constexpr int NX_ITEMS = 2 * ADJ_TY * NS0, N_ITEMS = NX_ITEMS + 2 * ADJ_TX * NS1;
#pragma unroll 1
    for (int i = (int)threadIdx.x; i < N_ITEMS; i += NC) {
        int t, slot, rx, ry;
        if (i < NX_ITEMS) {
            t = 0;
            slot = i % NS0;
            const int k = i / NS0;  // 0 .. 2 ADJ_TY - 1
            rx = (k / ADJ_TY) ? RX - 1 : 0;
            ry = 1 + k % ADJ_TY;
        } else {
            t = 1;
            const int j = i - NX_ITEMS;
            slot = j % NS1;
            const int k = j / NS1;  // 0 .. 2 ADJ_TX - 1
            ry = (k / ADJ_TX) ? RY - 1 : 0;
            rx = 1 + k % ADJ_TX;
        }
        const int a = 1 - t;
        const int q = t == 0 ? adj_q_of_slot<LAT>(0, slot) : adj_q_of_slot<LAT>(1, slot);
        const int hc[3] = {wrap_any(x0 - 1 + rx, P.n[0]), wrap_any(y0 - 1 + ry, P.n[1]), 0};
        int hu[3] = {hc[0], hc[1], 0};
        hu[a] = wrapc<T>(hc[a] + 1, P.n[a]);
        const long long hidx = int_idx(P, hc[0], hc[1], hc[2]), huidx = int_idx(P, hu[0], hu[1], hu[2]);
        const T wl = P.m[a].w[hc[a]], wu = P.m[a].w[hc[a] + 1];
        const T psi = wl * fa[a * stride + (long long)q * P.nc + hidx] +
                      (T(1) - wu) * fa[a * stride + (long long)q * P.nc + huidx];
        T s = T(0);
        s += psi;
        const int e = t == 0 ? LAT::ex(q) : LAT::ey(q);
        dts[t][slot][ry * RX + rx] = -P.h * P.c * T(e) * s;
    }
    __syncthreads();
    asm volatile("" ::: "memory");
    if (!own) return;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const int rm = rc - (t == 0 ? 1 : RX), rp = rc + (t == 0 ? 1 : RX);
        const T cpm = P.m[t].cp[wrapc<T>(ci[t] - 1, P.n[t])];  // cp of the cell below
        const T cmp = P.m[t].cm[wrapc<T>(ci[t] + 1, P.n[t])];  // cm of the cell above
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (LAT::e(q, t) == 0) continue;
            phat[q] += cpm * dts[t][adj_slot<LAT>(q, t)][rm] + cmp * dts[t][adj_slot<LAT>(q, t)][rp];
        }
    }
    adj_cell_finish<LAT, T>(P, ci, cidx, phat, f, force, lam, ga, gt, gth, lam_out, grad_force);
}

// f-bar-plus of a tile's region in LDS, laid out [q][region cell] with rows
// of RX cells; rc: the thread's cell (the accessor recon_face_ct reads)
template <typename T, int RX, int NR>
struct TilePhi {
    const T* s;
    int rc;
    __device__ __forceinline__ int base(int ox, int oy, int) const { return rc + ox + oy * RX; }
    __device__ __forceinline__ int up(int t) const { return t == 0 ? 1 : RX; }
    __device__ __forceinline__ int dn(int t) const { return up(t); }
    __device__ __forceinline__ T get(int q, int b) const { return s[q * NR + b]; }
};

// the f-bar-plus pass and pass A in one launch for the 2-D sets: a workgroup
// forms f-bar-plus (Eq. f_bar_+, from f_n at t_n) of its tile of ADJ_TX x
// ADJ_TY cells and their one-cell halo (periodic wrap) in LDS, then each
// thread takes the lower faces of both axes of its cell from there (no
// f-bar-plus array in memory)
template <class LAT, typename T>
__global__ __launch_bounds__(ADJ_TX * ADJ_TY) void k_adj_face_tile(
    const Inst<T>* __restrict__ Pp, const T* __restrict__ f, const T* __restrict__ force, const T* __restrict__ lam,
    T gt, T gth, int tiles_x, T* __restrict__ fa, T* __restrict__ ga)
{
    static_assert(LAT::D == 2, "2-D sets only");
    constexpr int Q = LAT::Q;
    constexpr int RX = ADJ_TX + 2, RY = ADJ_TY + 2, NR = RX * RY, NC = ADJ_TX * ADJ_TY;
    __shared__ T phs[Q * NR];
    const Inst<T>& P = *Pp;
    // tiles in XCD order: each XCD takes a contiguous range of tile rows, so
    // tiles sharing halo lines read them through one L2
    const int b = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int x0 = (b % tiles_x) * ADJ_TX, y0 = (b / tiles_x) * ADJ_TY;
#pragma unroll 1
    for (int r = (int)threadIdx.x; r < NR; r += NC) {
        const int cx = wrap_any(x0 - 1 + r % RX, P.n[0]), cy = wrap_any(y0 - 1 + r / RX, P.n[1]);
        T out[Q];
        phi_cell<LAT, T>(P, f, force, int_idx(P, cx, cy, 0), gt, out);
#pragma unroll
        for (int q = 0; q < Q; ++q) phs[q * NR + r] = out[q];
    }
    __syncthreads();
    asm volatile("" ::: "memory");
    const int tx = (int)threadIdx.x % ADJ_TX, ty = (int)threadIdx.x / ADJ_TX;
    if (x0 + tx >= P.n[0] || y0 + ty >= P.n[1]) return;
    const int ci[3] = {x0 + tx, y0 + ty, 0};
    const long long cidx = int_idx(P, ci[0], ci[1], 0);
    const TilePhi<T, RX, NR> ph{phs, (ty + 1) * RX + (tx + 1)};
    adj_face_core<LAT, T, 0>(P, ci, cidx, ph, force, lam, gth, fa, ga);
    asm volatile("" ::: "memory");
    adj_face_core<LAT, T, 1>(P, ci, cidx, ph, force, lam, gth, fa, ga);
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

// ---------------------------------------------------------------------------
// Reverse mode on meshes with walls (and any mix of periodic and wall axes).
// Every face of axis a, indices 0..n_a, is its own node (face n_a of a
// periodic axis equals face 0 in the forward step and is transposed as a
// face of its own), and the adjoint of f-bar-plus lives on the whole
// ghost-extended grid; the ghost rule is transposed at the end.
//   face pass   (per face): recompute F (Eq. gradient) and the wall rule
//                (Eqs. BB, NEQ) at wall faces; reverse of the flux (adjacent
//                interior cells only), of Eq. (original_f) and of the face moments ->
//                adjoint of F after the wall rule, and of the face acceleration;
//                At wall faces the same thread transposes the wall rule (bounce-back:
//                a permutation; NEQ: the replaced values depend on the values
//                and moments of the opposite interface x_c of the wall cell,
//                whose share is kept per line and side and added to x_c by
//                the psi pass);
//   psi pass    (per extended point and velocity): psi_hat_a from the two
//                faces of each axis, normal terms, 4/3 lam, d_hat_t; the
//                face-force adjoint;
//   gather pass (per cell and velocity): phi_hat = psi-pass part + cp
//                d_hat(-t) + c0 d_hat + cm d_hat(+t), gathered from the cell
//                and from every ghost the ghost rule builds from it (its
//                transpose, with the tensor-product weights of edges and
//                corners);
//   cell pass   (per cell): reverse of Eq. (f_bar_+) and of the macroscopic
//                recovery -> lam_n and the force-field gradient.
// ---------------------------------------------------------------------------

// faces of axis A: n_A + 1 along A, n_b across
template <typename T>
__device__ __forceinline__ void face_dims(const Inst<T>& P, int A, int* F)
{
#pragma unroll
    for (int b = 0; b < 3; ++b) F[b] = P.n[b] + (b == A ? 1 : 0);
}
template <typename T>
__device__ __forceinline__ long long face_lin(const Inst<T>& P, int A, const int* c)
{
    int F[3];
    face_dims(P, A, F);
    return ((long long)c[2] * F[1] + c[1]) * F[0] + c[0];
}
template <typename T>
__host__ __device__ inline long long face_total(const Inst<T>& P, int A)
{
    long long n = 1;
    for (int b = 0; b < 3; ++b) n *= (long long)(P.n[b] + (b == A ? 1 : 0));
    return n;
}

// index of the line along axis A through the point c (its coordinates
// across A, lowest axis fastest)
template <typename T>
__device__ __forceinline__ long long line_of(const Inst<T>& P, int A, const int* c)
{
    long long li = 0, m = 1;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == A) continue;
        li += m * c[b];
        m *= P.n[b];
    }
    return li;
}

// F of Eq. (gradient) on face c (c[A] = face index) of axis A, all velocities
template <class LAT, typename T, int A>
__device__ __forceinline__ void face_recon_at(const Inst<T>& P, const T* __restrict__ phi, const int* c, T* out)
{
    GlobalPhi<LAT, T> ph{phi, P.ne, ext_idx<LAT, T>(P, c[0], c[1], c[2]), (long long)P.E[0],
                         (long long)P.E[0] * P.E[1]};
    CellMetric<T> ma{};
    ma.wl = P.m[A].w[c[A]];
    ma.gl = P.m[A].gn[c[A]];
    const CellMetric<T> mx = A == 0 ? ma : load_metric(P, 0, c[0]);
    const CellMetric<T> my = A == 1 ? ma : load_metric(P, 1, c[1]);
    const CellMetric<T> mz = (A == 2 || LAT::D == 2) ? ma : load_metric(P, 2, c[2]);
    recon_face_ct<LAT, T, GlobalPhi<LAT, T>, A>(P, ph, false, ma, mx, my, mz, out);
}

template <class LAT, typename T, int A>
__device__ __forceinline__ void adjw_face_body(const Inst<T>& P, long long fi, const T* __restrict__ phi,
                                               const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                               T* __restrict__ fa, T* __restrict__ ga, T* __restrict__ ex,
                                               T* __restrict__ gx)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const long long nf = face_total(P, A);
    if (fi >= nf) return;
    int F[3], c[3];
    face_dims(P, A, F);
    c[0] = (int)(fi % F[0]);
    const long long r = fi / F[0];
    c[1] = (int)(r % F[1]);
    c[2] = (int)(r / F[1]);
    const int n = P.n[A], f = c[A];
    T fb[Q], G[3];
    face_recon_at<LAT, T, A>(P, phi, c, fb);
    const T w = P.m[A].w[f];
    face_force<LAT, T>(P, force, A, f, w, c, gth, G);
    const bool wlo = !P.per[A] && f == 0, whi = !P.per[A] && f == n;
    NeqInfo<LAT, T> info;
    T Go[3] = {T(0), T(0), T(0)};
    if (wlo || whi) {
        int co[3] = {c[0], c[1], c[2]};
        co[A] = wlo ? 1 : n - 1;
        T fo[Q];
        face_recon_at<LAT, T, A>(P, phi, co, fo);
        face_force<LAT, T>(P, force, A, co[A], P.m[A].w[co[A]], co, gth, Go);
        neq_capture<LAT, T>(P, A, fo, Go, info);
        wall_rule<LAT, T>(P, wlo ? 2 * A : 2 * A + 1, fb, info, gth);
    }
    T rho, u[3];
    face_moments<LAT, T>(P, fb, G, rho, u);
    // flux adjoint from the interior cells on either side
    T fh[Q];
    const T invRT = T(1) / P.RT;
    int cl[3] = {c[0], c[1], c[2]};
    cl[A] = f - 1;
    const bool hasL = f >= 1, hasR = f <= n - 1;
    const long long lidx = hasL ? int_idx(P, cl[0], cl[1], cl[2]) : 0;
    const long long ridx = hasR ? int_idx(P, c[0], c[1], c[2]) : 0;
    const T sL_ = P.m[A].fdx[hasL ? f - 1 : 0], sR_ = P.m[A].fdx[hasR ? f : 0];
    const T sL = hasL ? sL_ : T(0), sR = hasR ? sR_ : T(0);
    T rb = T(0), ub[3] = {T(0), T(0), T(0)}, Gb[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        fh[q] = T(0);
        if (LAT::e(q, A) == 0) continue;
        const T lr = sR * lam[(long long)q * P.nc + ridx];
        const T ll = sL * lam[(long long)q * P.nc + lidx];
        fh[q] = T(LAT::e(q, A)) * P.c * (lr - ll);
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
    T vb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T v = (T(1) - P.B7) * fh[q] + rb;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (LAT::e(q, d) == 1) v += P.c / P.rho0 * ub[d];
            if (LAT::e(q, d) == -1) v -= P.c / P.rho0 * ub[d];
        }
        vb[q] = v;
    }
    if (wlo || whi) {
        // transpose of the wall rule: vb becomes the adjoint of the values before the
        // rule; NEQ contributions to the opposite interface x_c go to the
        // line's slot of `ex`/`gx`, added to that face by the psi pass
        const int s = wlo ? 2 * A : 2 * A + 1;
        const int sg = wlo ? -1 : 1;  // outward normal sg e_A
        T rep[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            rep[q] = T(0);
            if (LAT::e(q, A) * sg < 0) {
                rep[q] = vb[q];
                vb[q] = T(0);
            }
        }
        T xo[Q], go[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < Q; ++q) xo[q] = T(0);
        if (P.bc[s] == BC_BOUNCE_BACK) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (LAT::e(q, A) * sg < 0) vb[LAT::opp(q)] += rep[q];
        } else {
            const bool vel = P.bc[s] == BC_NEQ_VELOCITY;
            T ra, ua[3] = {T(0), T(0), T(0)};
            if (vel) {
                ra = info.rc;
#pragma unroll
                for (int d = 0; d < D; ++d) ua[d] = P.uw[s][d];
            } else {
                ra = wall_density(P, s, gth);
#pragma unroll
                for (int d = 0; d < D; ++d) ua[d] = info.uc[d];
            }
            T rcb = T(0), ucb[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (LAT::e(q, A) * sg >= 0) continue;
                const Partials<LAT, T> pa = partials<LAT, T>(q, ra, ua, Go, P.rho0, P.c, invRT);
                if (vel) rcb += rep[q] * pa.dfe_dr;
                else
#pragma unroll
                    for (int d = 0; d < D; ++d) ucb[d] += rep[q] * pa.dfe_du[d];
                const Partials<LAT, T> pc = partials<LAT, T>(q, info.rc, info.uc, Go, P.rho0, P.c, invRT);
                rcb -= rep[q] * pc.dfe_dr;
#pragma unroll
                for (int d = 0; d < D; ++d) ucb[d] -= rep[q] * pc.dfe_du[d];
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                T v = rep[q] + rcb;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (LAT::e(q, d) == 1) v += P.c / P.rho0 * ucb[d];
                    if (LAT::e(q, d) == -1) v -= P.c / P.rho0 * ucb[d];
                }
                xo[q] = v;
            }
#pragma unroll
            for (int d = 0; d < D; ++d) go[d] = T(0.5) * P.h * ucb[d];
        }
        const long long nl = P.nc / n;
        const long long li = line_of(P, A, c);
        const long long slot = (wlo ? 0 : nl) + li;
#pragma unroll
        for (int q = 0; q < Q; ++q) ex[(long long)q * 2 * nl + slot] = xo[q];
#pragma unroll
        for (int d = 0; d < D; ++d) gx[(long long)d * 2 * nl + slot] = go[d];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) fa[(long long)q * nf + fi] = vb[q];
#pragma unroll
    for (int d = 0; d < D; ++d) ga[(long long)d * nf + fi] = Gb[d];
}

// all axes in one launch: blockIdx.y = axis
struct AdjFaces {
    void* fa[3];
    void* ga[3];
    void* ex[3];  // per wall line and side: NEQ part of the adjoint of the opposite interface
    void* gx[3];  // the same for its acceleration
};

template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adjw_face(const Inst<T>* __restrict__ Pp, const T* __restrict__ phi,
                                                   const T* __restrict__ force, const T* __restrict__ lam, T gth,
                                                   AdjFaces AF)
{
    const Inst<T>& P = *Pp;
    const long long fi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (a == 0)
        adjw_face_body<LAT, T, 0>(P, fi, phi, force, lam, gth, (T*)AF.fa[0], (T*)AF.ga[0], (T*)AF.ex[0],
                                  (T*)AF.gx[0]);
    else if (a == 1)
        adjw_face_body<LAT, T, 1>(P, fi, phi, force, lam, gth, (T*)AF.fa[1], (T*)AF.ga[1], (T*)AF.ex[1],
                                  (T*)AF.gx[1]);
    else if constexpr (LAT::D == 3)
        adjw_face_body<LAT, T, 2>(P, fi, phi, force, lam, gth, (T*)AF.fa[2], (T*)AF.ga[2], (T*)AF.ex[2],
                                  (T*)AF.gx[2]);
}

// decode an extended-grid index into coordinates -1..n
template <class LAT, typename T>
__device__ __forceinline__ void ext_coords(const Inst<T>& P, long long e, int* x)
{
    x[0] = (int)(e % P.E[0]) - 1;
    const long long r = e / P.E[0];
    x[1] = (int)(r % P.E[1]) - 1;
    x[2] = LAT::D == 3 ? (int)(r / P.E[1]) - 1 : 0;
}

// psi pass for one velocity q (compile time) at extended point e; the
// threads with q = 0 also gather the face-force adjoint
template <class LAT, typename T, int q>
__device__ __forceinline__ void adjw_psi_q(const Inst<T>& P, const AdjFaces& AF, const T* __restrict__ lam, T gth,
                                           long long e, T* __restrict__ php, T* __restrict__ dhat,
                                           T* __restrict__ gext)
{
    constexpr int D = LAT::D;
    int x[3];
    ext_coords<LAT, T>(P, e, x);
    bool in[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) in[b] = x[b] >= 0 && x[b] < P.n[b];
    const bool interior = in[0] && in[1] && in[2];
    const long long ci = interior ? int_idx(P, x[0], x[1], x[2]) : 0;
    T ph = (interior ? T(4.0 / 3.0) : T(0)) * lam[(long long)q * P.nc + ci];
    T psi[3] = {T(0), T(0), T(0)}, gx[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        bool across = true;
#pragma unroll
        for (int b = 0; b < D; ++b)
            if (b != a && !in[b]) across = false;
        if (!across) continue;
        const T* fa = (const T*)AF.fa[a];
        const long long nf = face_total(P, a);
        // lower face (this point is its right cell) and upper face (left cell)
        const int flo = x[a], fup = x[a] + 1;
        const bool hlo = flo >= 0 && flo <= P.n[a], hup = fup >= 0 && fup <= P.n[a];
        int cf[3] = {x[0], x[1], x[2]};
        cf[a] = flo;
        const long long ilo = hlo ? face_lin(P, a, cf) : 0;
        cf[a] = fup;
        const long long iup = hup ? face_lin(P, a, cf) : 0;
        // branch-free: clamped indices, zero weights where a face is absent
        const T wlo_ = P.m[a].w[hlo ? flo : 0], wup_ = P.m[a].w[hup ? fup : 0];
        const T glo_ = P.m[a].gn[hlo ? flo : 0], gup_ = P.m[a].gn[hup ? fup : 0];
        const T klo = hlo ? T(1) : T(0), kup = hup ? T(1) : T(0);
        const T wlo = klo * wlo_, cup = kup * (T(1) - wup_);
        const T glo = klo * glo_, gup = kup * gup_;
        // NEQ shares of the walls in faces 1 (low wall) and n-1 (high wall)
        T xw[4] = {T(0), T(0), T(0), T(0)};
        long long xs[4] = {0, 0, 0, 0}, nl2 = 0;
        const bool wall_axis = !P.per[a];
        if (wall_axis) {
            const long long nl = P.nc / P.n[a];
            nl2 = 2 * nl;
            const long long li = line_of(P, a, x);
            xs[0] = li;
            xs[1] = nl + li;
            xs[2] = li;
            xs[3] = nl + li;
            xw[0] = (hlo && flo == 1) ? T(1) : T(0);
            xw[1] = (hlo && flo == P.n[a] - 1) ? T(1) : T(0);
            xw[2] = (hup && fup == 1) ? T(1) : T(0);
            xw[3] = (hup && fup == P.n[a] - 1) ? T(1) : T(0);
        }
        T blo = fa[(long long)q * nf + ilo];
        T bup = fa[(long long)q * nf + iup];
        if (wall_axis) {
            const T* eq = (const T*)AF.ex[a] + (long long)q * nl2;
            blo += xw[0] * eq[xs[0]] + xw[1] * eq[xs[1]];
            bup += xw[2] * eq[xs[2]] + xw[3] * eq[xs[3]];
        }
        psi[a] = wlo * blo + cup * bup;
        ph += psi[a] + T(LAT::e(q, a)) * P.h * P.c * (gup * bup - glo * blo);
        if constexpr (q == 0) {
            const T* ga = (const T*)AF.ga[a];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                T glo_d = ga[(long long)d * nf + ilo];
                T gup_d = ga[(long long)d * nf + iup];
                if (wall_axis) {
                    const T* gq = (const T*)AF.gx[a] + (long long)d * nl2;
                    glo_d += xw[0] * gq[xs[0]] + xw[1] * gq[xs[1]];
                    gup_d += xw[2] * gq[xs[2]] + xw[3] * gq[xs[3]];
                }
                gx[d] += gth * (wlo * glo_d + cup * gup_d);
            }
        }
    }
    const long long stride = (long long)LAT::Q * P.ne;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        T dh = T(0);
        if (LAT::e(q, t) != 0) {
            T sp = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a)
                if (a != t) sp += psi[a];
            dh = -P.h * P.c * T(LAT::e(q, t)) * sp;
        }
        dhat[t * stride + (long long)q * P.ne + e] = dh;
    }
    php[(long long)q * P.ne + e] = ph;
    if constexpr (q == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) gext[(long long)d * P.ne + e] = gx[d];
}

template <class LAT, typename T, int... Is>
__device__ __forceinline__ void adjw_psi_dispatch(int q, std::integer_sequence<int, Is...>, const Inst<T>& P,
                                                  const AdjFaces& AF, const T* __restrict__ lam, T gth, long long e,
                                                  T* php, T* dhat, T* gext)
{
    ((q == Is ? adjw_psi_q<LAT, T, Is>(P, AF, lam, gth, e, php, dhat, gext) : void()), ...);
}

// one thread per (extended point, velocity): blockIdx.y = velocity
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adjw_psi(const Inst<T>* __restrict__ Pp, AdjFaces AF,
                                                  const T* __restrict__ lam, T gth, T* __restrict__ php,
                                                  T* __restrict__ dhat, T* __restrict__ gext)
{
    const Inst<T>& P = *Pp;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P.ne) return;
    adjw_psi_dispatch<LAT, T>((int)blockIdx.y, std::make_integer_sequence<int, LAT::Q>{}, P, AF, lam, gth, e, php,
                              dhat, gext);
}

// phi_hat of one velocity at an extended point Y: the psi-pass part plus
//   sum_t cp(Y-t) d_hat_t(Y-t) + c0(Y) d_hat_t(Y) + cm(Y+t) d_hat_t(Y+t)
template <class LAT, typename T, int q>
__device__ __forceinline__ T phi_hat_q(const Inst<T>& P, const T* __restrict__ php, const T* __restrict__ dhat,
                                       long long e, const int* x)
{
    constexpr int D = LAT::D;
    const long long stride = (long long)LAT::Q * P.ne;
    const long long st[3] = {1, (long long)P.E[0], (long long)P.E[0] * P.E[1]};
    T acc = php[(long long)q * P.ne + e];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        if (LAT::e(q, t) == 0) continue;
        const int n = P.n[t], xt = x[t];
        const bool dm = xt - 1 >= 0 && xt - 1 < n;
        const bool d0 = xt >= 0 && xt < n;
        const bool dp = xt + 1 >= 0 && xt + 1 < n;
        // branch-free: clamped indices, zero weights for absent terms
        const T cpm_ = P.m[t].cp[dm ? xt - 1 : 0], c00_ = P.m[t].c0[d0 ? xt : 0], cmp_ = P.m[t].cm[dp ? xt + 1 : 0];
        const T cpm = dm ? cpm_ : T(0), c00 = d0 ? c00_ : T(0), cmp = dp ? cmp_ : T(0);
        const long long em = dm ? e - st[t] : e, ep = dp ? e + st[t] : e;
        const T* dq = dhat + t * stride + (long long)q * P.ne;
        acc += cpm * dq[em] + c00 * dq[e] + cmp * dq[ep];
    }
    return acc;
}

// the points of axis a whose value the ghost rule builds from the
// cell with coordinate x along a, with their weights: the cell itself and
// up to two ghosts (wall: linear extrapolation; periodic: copies)
template <typename T>
__device__ __forceinline__ int ghost_sources(const Inst<T>& P, int a, int x, int* y, T* k)
{
    const int n = P.n[a];
    int m = 0;
    y[m] = x;
    k[m++] = T(1);
    if (P.per[a]) {
        if (x == n - 1) { y[m] = -1; k[m++] = T(1); }
        if (x == 0) { y[m] = n; k[m++] = T(1); }
    } else {
        T kl = T(0), kh = T(0);
        if (x == 0) kl += T(1) - P.rlo[a];
        if (x == 1) kl += P.rlo[a];
        if (x == n - 1) kh += T(1) - P.rhi[a];
        if (x == n - 2) kh += P.rhi[a];
        if (kl != T(0)) { y[m] = -1; k[m++] = kl; }
        if (kh != T(0)) { y[m] = n; k[m++] = kh; }
    }
    return m;
}

// phi_hat of velocity q at an interior cell, gathered from the cell and every
// ghost the ghost rule builds from it (transpose of the ghost rule, tensor-product
// weights); the q = 0 threads gather the force adjoint likewise
template <class LAT, typename T, int q>
__device__ __forceinline__ void adjw_gather_q(const Inst<T>& P, long long cidx, const T* __restrict__ php,
                                              const T* __restrict__ dhat, const T* __restrict__ gext,
                                              T* __restrict__ pin, T* __restrict__ gin)
{
    constexpr int D = LAT::D;
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    const long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    int ys[3][3], ms[3] = {1, 1, 1};
    T ks[3][3];
    ys[2][0] = 0;
    ks[2][0] = T(1);
#pragma unroll
    for (int a = 0; a < D; ++a) ms[a] = ghost_sources(P, a, ci[a], ys[a], ks[a]);
    T pb, gb[3] = {T(0), T(0), T(0)};
    if (ms[0] == 1 && ms[1] == 1 && ms[2] == 1) {  // no ghost is built from this cell
        const long long e = ext_idx<LAT, T>(P, ci[0], ci[1], ci[2]);
        pb = phi_hat_q<LAT, T, q>(P, php, dhat, e, ci);
        if constexpr (q == 0)
#pragma unroll
            for (int d = 0; d < D; ++d) gb[d] = gext[(long long)d * P.ne + e];
    } else {
        pb = T(0);
#pragma unroll 1
        for (int i2 = 0; i2 < ms[2]; ++i2)
#pragma unroll 1
            for (int i1 = 0; i1 < ms[1]; ++i1)
#pragma unroll 1
                for (int i0 = 0; i0 < ms[0]; ++i0) {
                    const int y[3] = {ys[0][i0], ys[1][i1], ys[2][i2]};
                    const T w = ks[0][i0] * ks[1][i1] * ks[2][i2];
                    const long long e = ext_idx<LAT, T>(P, y[0], y[1], y[2]);
                    pb += w * phi_hat_q<LAT, T, q>(P, php, dhat, e, y);
                    if constexpr (q == 0)
#pragma unroll
                        for (int d = 0; d < D; ++d) gb[d] += w * gext[(long long)d * P.ne + e];
                }
    }
    pin[(long long)q * P.nc + cidx] = pb;
    if constexpr (q == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) gin[(long long)d * P.nc + cidx] = gb[d];
}

template <class LAT, typename T, int... Is>
__device__ __forceinline__ void adjw_gather_dispatch(int q, std::integer_sequence<int, Is...>, const Inst<T>& P,
                                                     long long cidx, const T* php, const T* dhat, const T* gext,
                                                     T* pin, T* gin)
{
    ((q == Is ? adjw_gather_q<LAT, T, Is>(P, cidx, php, dhat, gext, pin, gin) : void()), ...);
}

// one thread per (cell, velocity): blockIdx.y = velocity
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adjw_gather(const Inst<T>* __restrict__ Pp, const T* __restrict__ php,
                                                     const T* __restrict__ dhat, const T* __restrict__ gext,
                                                     T* __restrict__ pin, T* __restrict__ gin)
{
    const Inst<T>& P = *Pp;
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= P.nc) return;
    adjw_gather_dispatch<LAT, T>((int)blockIdx.y, std::make_integer_sequence<int, LAT::Q>{}, P, cidx, php, dhat,
                                 gext, pin, gin);
}

// per cell: reverse of Eq. (f_bar_+) and of the macroscopic recovery ->
// lam_n and the force-field gradient
template <class LAT, typename T>
__global__ __launch_bounds__(256) void k_adjw_cell(const Inst<T>* __restrict__ Pp, const T* __restrict__ f,
                                                   const T* __restrict__ force, const T* __restrict__ lam,
                                                   const T* __restrict__ pin, const T* __restrict__ gin, T gt,
                                                   T* __restrict__ lam_out, T* __restrict__ grad_force)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const Inst<T>& P = *Pp;
    const long long cidx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cidx >= P.nc) return;
    T pb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) pb[q] = pin[(long long)q * P.nc + cidx];
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
        rb += pb[q] * (P.B1 * pd.dfe_dr + P.C1 * pd.dS_dr);
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ub[d] += pb[q] * (P.B1 * pd.dfe_du[d] + P.C1 * pd.dS_du[d]);
            Gc[d] += pb[q] * P.C1 * pd.dS_dG[d];
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) Gc[d] += P.h * ub[d];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T v = (T(1) - P.B1) * pb[q] + rb - T(1.0 / 3.0) * lam[(long long)q * P.nc + cidx];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (LAT::e(q, d) == 1) v += P.c / P.rho0 * ub[d];
            if (LAT::e(q, d) == -1) v -= P.c / P.rho0 * ub[d];
        }
        lam_out[(long long)q * P.nc + cidx] = v;
    }
    if (grad_force)
#pragma unroll
        for (int d = 0; d < D; ++d) grad_force[(long long)d * P.nc + cidx] += gt * Gc[d] + gin[(long long)d * P.nc + cidx];
}

static inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

// Scratch of the allocation-free adjoint (dugks_step_adjoint_static): one
// static device area, which every GPU the library runs on holds until the
// process ends.  Host code never uses the array's name as a device address:
// its per-device address comes from hipGetSymbolAddress, looked up once per
// device with that device current (at dugks_init, else at the entry
// point's first call there) and kept in static_scratch_dev.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
static void* static_scratch_dev[kMaxDevices];
static std::mutex static_scratch_mu;

static hipError_t static_scratch_lookup(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(static_scratch_mu);
    if (!static_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        static_scratch_dev[dev] = p;
    }
    *out = static_scratch_dev[dev];
    return hipSuccess;
}

void adjoint_static_setup()
{
    int dev = -1;
    void* p = nullptr;
    // a failed lookup is retried (and reported) by the entry point
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) (void)static_scratch_lookup(dev, &p);
}

// device scratch of `need` bytes for one adjoint step: the context's own
// buffer (allocated on first use, grown when needed), or the static area
static int adjoint_scratch(dugks_ctx* ctx, size_t need, bool stat, void** out)
{
    if (stat) {
        if (need > kStaticScratchBytes)
            return fail(ctx, DUGKS_EINVAL,
                        "the adjoint step needs " + std::to_string(need) +
                            " bytes of scratch, more than the static area of the allocation-free entry point (" +
                            std::to_string(kStaticScratchBytes) + " bytes); use dugks_step_adjoint");
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_check(ctx, e, "current device");
        if (dev != ctx->device) return fail(ctx, DUGKS_EINVAL, "the current device is not the context's device");
        if (dev < 0 || dev >= kMaxDevices) return fail(ctx, DUGKS_EUNSUPPORTED, "device ordinal out of range");
        e = static_scratch_lookup(dev, out);
        return hip_check(ctx, e, "static scratch address");
    }
    if (ctx->adj_bytes < need) {
        if (ctx->adj) (void)hipFree(ctx->adj);
        ctx->adj = nullptr;
        ctx->adj_bytes = 0;
        if (hipMalloc(&ctx->adj, need) != hipSuccess) return fail(ctx, DUGKS_ENOMEM, "adjoint scratch allocation failed");
        ctx->adj_bytes = need;
    }
    *out = ctx->adj;
    return DUGKS_OK;
}

template <class LAT, typename T>
static int adjoint_step(dugks_ctx* ctx, const Inst<T>& P, const void* fn, const void* force, double t,
                        const void* lam_np1, void* lam_n, void* grad_force, hipStream_t st, bool stat)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const size_t es = sizeof(T);
    // 2-D sets: two tiled launches (f-bar-plus with pass A, passes B with C)
    constexpr bool tiled = D == 2;
    const size_t need = (size_t)D * Q * P.nc * es            // face adjoints
                        + (size_t)D * D * P.nc * es          // face force adjoints
                        + (tiled ? 0 : (size_t)P.ne * Q * es)        // phi (extended)
                        + (tiled ? 0 : (size_t)Q * P.nc * es)        // phi_hat partial
                        + (tiled ? 0 : (size_t)D * Q * P.nc * es);   // d_hat
    void* work = nullptr;
    const int src = adjoint_scratch(ctx, need, stat, &work);
    if (src != DUGKS_OK) return src;
    T* fa = (T*)work;
    T* ga = fa + (size_t)D * Q * P.nc;
    const Inst<T>* Pd = (const Inst<T>*)ctx->inst_dev;
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * (double)ctx->cfg.dt);
    if constexpr (tiled) {
        const int tiles_x = (P.n[0] + ADJ_TX - 1) / ADJ_TX, tiles_y = (P.n[1] + ADJ_TY - 1) / ADJ_TY;
        const dim3 grid((unsigned)(tiles_x * tiles_y)), block(ADJ_TX * ADJ_TY);
        hipLaunchKernelGGL((k_adj_face_tile<LAT, T>), grid, block, 0, st, Pd, (const T*)fn, (const T*)force,
                           (const T*)lam_np1, gt, gth, tiles_x, fa, ga);
        hipLaunchKernelGGL((k_adj_cell_tile<LAT, T>), grid, block, 0, st, Pd, (const T*)fn, (const T*)force,
                           (const T*)lam_np1, (const T*)fa, (const T*)ga, gt, gth, tiles_x, (T*)lam_n,
                           (T*)grad_force);
    } else {
        T* phi = ga + (size_t)D * D * P.nc;
        T* ph = phi + (size_t)P.ne * Q;
        T* dh = ph + (size_t)Q * P.nc;
        hipLaunchKernelGGL((k_phi_adj<LAT, T>), dim3(nb256(P.ne)), dim3(256), 0, st, Pd, (const T*)fn,
                           (const T*)force, phi, gt);
        hipLaunchKernelGGL((k_adj_face<LAT, T>), dim3(nb256(P.nc), D), dim3(256), 0, st, Pd, (const T*)phi,
                           (const T*)force, (const T*)lam_np1, gth, fa, ga);
        hipLaunchKernelGGL((k_adj_cell1<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, Pd, (const T*)lam_np1,
                           (const T*)fa, ph, dh);
        hipLaunchKernelGGL((k_adj_cell2<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, Pd, (const T*)fn,
                           (const T*)force, (const T*)lam_np1, (const T*)ph, (const T*)dh, (const T*)ga, gt, gth,
                           (T*)lam_n, (T*)grad_force);
    }
    return hip_check(ctx, hipGetLastError(), "adjoint launch");
}

template <class LAT, typename T>
static int adjoint_step_walls(dugks_ctx* ctx, const Inst<T>& P, const void* fn, const void* force, double t,
                              const void* lam_np1, void* lam_n, void* grad_force, hipStream_t st, bool stat)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const size_t es = sizeof(T);
    size_t nfaces = 0;
    for (int a = 0; a < D; ++a) nfaces += (size_t)face_total(P, a);
    size_t nwall = 0;  // 2 sides x lines of each wall axis
    for (int a = 0; a < D; ++a)
        if (!P.per[a]) nwall += (size_t)(2 * (P.nc / P.n[a]));
    const size_t need = (size_t)P.ne * Q * es        // phi (extended)
                        + nfaces * Q * es            // face adjoints
                        + nfaces * D * es            // face-force adjoints
                        + nwall * (Q + D) * es       // NEQ parts of the opposite interfaces
                        + (size_t)P.ne * Q * es      // phi_hat (extended)
                        + (size_t)D * P.ne * Q * es  // d_hat (extended)
                        + (size_t)P.ne * D * es      // force adjoint (extended)
                        + (size_t)P.nc * (Q + D) * es; // phi_hat and force adjoint gathered per cell
    void* work = nullptr;
    const int src = adjoint_scratch(ctx, need, stat, &work);
    if (src != DUGKS_OK) return src;
    T* p = (T*)work;
    T* phi = p;
    p += (size_t)P.ne * Q;
    AdjFaces AF{};
    T* fa[3] = {nullptr, nullptr, nullptr};
    T* ga[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < D; ++a) {
        fa[a] = p;
        p += (size_t)face_total(P, a) * Q;
    }
    for (int a = 0; a < D; ++a) {
        ga[a] = p;
        p += (size_t)face_total(P, a) * D;
    }
    for (int a = 0; a < 3; ++a) {
        AF.fa[a] = fa[a];
        AF.ga[a] = ga[a];
        AF.ex[a] = nullptr;
        AF.gx[a] = nullptr;
    }
    for (int a = 0; a < D; ++a) {
        if (P.per[a]) continue;
        const size_t nw = (size_t)(2 * (P.nc / P.n[a]));
        AF.ex[a] = p;
        p += nw * Q;
        AF.gx[a] = p;
        p += nw * D;
    }
    T* php = p;
    p += (size_t)P.ne * Q;
    T* dhat = p;
    p += (size_t)D * P.ne * Q;
    T* gext = p;
    p += (size_t)P.ne * D;
    T* pin = p;
    p += (size_t)P.nc * Q;
    T* gin = p;
    const Inst<T>* Pd = (const Inst<T>*)ctx->inst_dev;
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * (double)ctx->cfg.dt);
    const T* lam = (const T*)lam_np1;
    long long maxf = 0;
    for (int a = 0; a < D; ++a) maxf = std::max(maxf, face_total(P, a));
    hipLaunchKernelGGL((k_phi_adj<LAT, T>), dim3(nb256(P.ne)), dim3(256), 0, st, Pd, (const T*)fn, (const T*)force,
                       phi, gt);
    hipLaunchKernelGGL((k_adjw_face<LAT, T>), dim3(nb256(maxf), D), dim3(256), 0, st, Pd, (const T*)phi,
                       (const T*)force, lam, gth, AF);
    hipLaunchKernelGGL((k_adjw_psi<LAT, T>), dim3(nb256(P.ne), Q), dim3(256), 0, st, Pd, AF, lam, gth, php, dhat,
                       gext);
    hipLaunchKernelGGL((k_adjw_gather<LAT, T>), dim3(nb256(P.nc), Q), dim3(256), 0, st, Pd, (const T*)php,
                       (const T*)dhat, (const T*)gext, pin, gin);
    hipLaunchKernelGGL((k_adjw_cell<LAT, T>), dim3(nb256(P.nc)), dim3(256), 0, st, Pd, (const T*)fn, (const T*)force,
                       lam, (const T*)pin, (const T*)gin, gt, (T*)lam_n, (T*)grad_force);
    return hip_check(ctx, hipGetLastError(), "adjoint (walls) launch");
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

namespace dugks {
// checks and kernel choice shared by dugks_step_adjoint and its
// allocation-free variant (stat: scratch in the static area)
static int step_adjoint_any(dugks_ctx* ctx, const void* f_n, const void* force, double t_n, const void* lam_np1,
                            void* lam_n, void* grad_force, void* stream, bool stat)
{
    if (!ctx) return fail(nullptr, DUGKS_EINVAL, "null context");
    if (!f_n || !lam_np1 || !lam_n) return fail(ctx, DUGKS_EINVAL, "null buffer");
    if (ctx->cfg.model != DUGKS_MODEL_INCOMPRESSIBLE)
        return fail(ctx, DUGKS_EUNSUPPORTED, "the adjoint is derived for the incompressible model");
    if (ctx->cfg.lattice == DUGKS_D3Q27) return fail(ctx, DUGKS_EUNSUPPORTED, "no D3Q27 adjoint");
    if (lam_n == f_n || lam_n == lam_np1) return fail(ctx, DUGKS_EINVAL, "lam_n must not alias f_n or lam_np1");
    bool periodic = true;
    for (int s = 0; s < 2 * ctx->D; ++s)
        if (ctx->cfg.bc[s] != DUGKS_PERIODIC) periodic = false;
    const hipStream_t st = (hipStream_t)stream;
    // meshes with walls: the general reverse pass (also taken on periodic
    // meshes when DUGKS_ADJOINT_GENERAL=1, to cross-check it)
    const char* gen = getenv("DUGKS_ADJOINT_GENERAL");
    if (!periodic || (gen && gen[0] == '1')) {
        if (ctx->cfg.lattice == DUGKS_D2Q9) {
            if (ctx->cfg.dtype == DUGKS_F64)
                return adjoint_step_walls<D2Q9, double>(ctx, ctx->pd, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
            return adjoint_step_walls<D2Q9, float>(ctx, ctx->pf, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
        }
        if (ctx->cfg.dtype == DUGKS_F64)
            return adjoint_step_walls<D3Q19, double>(ctx, ctx->pd, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
        return adjoint_step_walls<D3Q19, float>(ctx, ctx->pf, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
    }
    if (ctx->cfg.lattice == DUGKS_D2Q9) {
        if (ctx->cfg.dtype == DUGKS_F64)
            return adjoint_step<D2Q9, double>(ctx, ctx->pd, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
        return adjoint_step<D2Q9, float>(ctx, ctx->pf, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
    }
    if (ctx->cfg.dtype == DUGKS_F64)
        return adjoint_step<D3Q19, double>(ctx, ctx->pd, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
    return adjoint_step<D3Q19, float>(ctx, ctx->pf, f_n, force, t_n, lam_np1, lam_n, grad_force, st, stat);
}
}  // namespace dugks

extern "C" int dugks_step_adjoint(dugks_ctx* ctx, const void* f_n, const void* force, double t_n,
                                  const void* lam_np1, void* lam_n, void* grad_force, void* stream)
{
    return step_adjoint_any(ctx, f_n, force, t_n, lam_np1, lam_n, grad_force, stream, false);
}

extern "C" int dugks_step_adjoint_static(dugks_ctx* ctx, const void* f_n, const void* force, double t_n,
                                         const void* lam_np1, void* lam_n, void* grad_force, void* stream)
{
    return step_adjoint_any(ctx, f_n, force, t_n, lam_np1, lam_n, grad_force, stream, true);
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
