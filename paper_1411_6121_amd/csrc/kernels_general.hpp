// kernels_general.hpp -- general step kernels (any lattice, mesh, wall kind,
// force), used for every configuration and as the batched path.
//
// Pass 1 (k_phi): f-bar-plus (Eq. f_bar_+) on every cell of the ghost-extended
//   grid (Appendix steps 1-2); a ghost takes the linear extrapolation through
//   the two nearest centres of each wall axis (tensor product on edges and
//   corners) or the wrapped cell of a periodic axis.
// Pass 2 (k_update): per interior cell, both faces of every axis are
//   reconstructed from pass 1 (steps 3-4), wall rules applied (step 5),
//   interface moments and the original distribution formed (steps 6-7), and
//   the conservative update written (steps 8-9).  Interior faces are thus
//   evaluated by both neighbours with the same code and operands, so the
//   two sides see bitwise-identical fluxes and conservation holds to
//   rounding.
#pragma once

#include "inst.hpp"

namespace dugks {

template <class LAT, typename T>
__device__ __forceinline__ long long ext_idx(const Inst<T>& P, int i, int j, int k)
{
    const int oz = (LAT::D == 3) ? 1 : 0;
    return ((long long)(k + oz) * P.E[1] + (j + 1)) * P.E[0] + (i + 1);
}

template <typename T>
__device__ __forceinline__ long long int_idx(const Inst<T>& P, int i, int j, int k)
{
    return ((long long)k * P.n[1] + j) * P.n[0] + i;
}

// f-bar-plus of one interior cell (Appendix step 1)
template <class LAT, typename T>
__device__ void phi_cell(const Inst<T>& P, const T* __restrict__ f, const T* __restrict__ force, long long ci,
                         T gt, T* out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const T invRT = T(1) / P.RT;
    T fv[Q];
    T rho = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        fv[q] = f[(long long)q * P.nc + ci];
        rho += fv[q];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (LAT::e(q, a) == 1) j[a] += fv[q];
            if (LAT::e(q, a) == -1) j[a] -= fv[q];
        }
    }
    T G[3], u[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        G[a] = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + ci] : T(0)));
        u[a] = P.c * j[a] / P.rho0 + P.h * G[a];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T fe = feq_q<LAT, T>(q, rho, u, P.rho0, P.c, invRT);
        const T S = src_fac<LAT, T>(q, u, G, P.c, invRT) * fe;
        out[q] = fv[q] + P.B1 * (fe - fv[q]) + P.C1 * S;
    }
}

template <class LAT, typename T>
__device__ void phi_ext_body(const Inst<T>& P, long long e, const T* __restrict__ f, const T* __restrict__ force,
                             T* __restrict__ phi, T gt)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    int c[3];
    c[0] = (int)(e % P.E[0]) - 1;
    long long r = e / P.E[0];
    c[1] = (int)(r % P.E[1]) - 1;
    c[2] = (D == 3) ? (int)(r / P.E[1]) - 1 : 0;
    int idx[3][2];
    T wt[3][2];
    int cnt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int x = c[a], N = P.n[a];
        cnt[a] = 1;
        idx[a][0] = x;
        wt[a][0] = T(1);
        idx[a][1] = 0;
        wt[a][1] = T(0);
        if (a >= D || (x >= 0 && x < N)) {
            if (a >= D) idx[a][0] = 0;
        } else if (P.per[a]) {
            idx[a][0] = x < 0 ? N - 1 : 0;
        } else if (x < 0) {
            cnt[a] = 2;
            idx[a][0] = 0; wt[a][0] = T(1) - P.rlo[a];
            idx[a][1] = 1; wt[a][1] = P.rlo[a];
        } else {
            cnt[a] = 2;
            idx[a][0] = N - 1; wt[a][0] = T(1) - P.rhi[a];
            idx[a][1] = N - 2; wt[a][1] = P.rhi[a];
        }
    }
    T acc[Q];
    if (cnt[0] * cnt[1] * cnt[2] == 1) {
        phi_cell<LAT, T>(P, f, force, int_idx(P, idx[0][0], idx[1][0], idx[2][0]), gt, acc);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] = T(0);
        for (int i2 = 0; i2 < cnt[2]; ++i2)
            for (int i1 = 0; i1 < cnt[1]; ++i1)
                for (int i0 = 0; i0 < cnt[0]; ++i0) {
                    T tmp[Q];
                    phi_cell<LAT, T>(P, f, force, int_idx(P, idx[0][i0], idx[1][i1], idx[2][i2]), gt, tmp);
                    const T w = wt[0][i0] * wt[1][i1] * wt[2][i2];
#pragma unroll
                    for (int q = 0; q < Q; ++q) acc[q] += w * tmp[q];
                }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) phi[(long long)q * P.ne + e] = acc[q];
}

// spatial force component d at the cell whose axis-a coordinate is x (which
// may be a ghost), other coordinates from ci; ghosts follow the phi rule
template <class LAT, typename T>
__device__ __forceinline__ T force_at(const Inst<T>& P, const T* __restrict__ force, int d, int a, int x,
                                      const int* ci)
{
    if (!force) return T(0);
    int cc[3] = {ci[0], ci[1], ci[2]};
    const int N = P.n[a];
    const T* fd = force + (long long)d * P.nc;
    if (x >= 0 && x < N) {
        cc[a] = x;
        return fd[int_idx(P, cc[0], cc[1], cc[2])];
    }
    if (P.per[a]) {
        cc[a] = x < 0 ? N - 1 : 0;
        return fd[int_idx(P, cc[0], cc[1], cc[2])];
    }
    const T r = x < 0 ? P.rlo[a] : P.rhi[a];
    cc[a] = x < 0 ? 0 : N - 1;
    const T v0 = fd[int_idx(P, cc[0], cc[1], cc[2])];
    cc[a] = x < 0 ? 1 : N - 2;
    const T v1 = fd[int_idx(P, cc[0], cc[1], cc[2])];
    return (T(1) - r) * v0 + r * v1;
}

// acceleration on face f of axis a (between cells f-1 and f) at time factor gth
template <class LAT, typename T>
__device__ __forceinline__ void face_force(const Inst<T>& P, const T* __restrict__ force, int a, int f,
                                           const int* ci, T gth, T* G)
{
    const T w = P.m[a].w[f];
#pragma unroll
    for (int d = 0; d < LAT::D; ++d) {
        T gh = T(0);
        if (force) {
            const T gl = force_at<LAT, T>(P, force, d, a, f - 1, ci);
            const T gr = force_at<LAT, T>(P, force, d, a, f, ci);
            gh = gl + w * (gr - gl);
        }
        G[d] = gth * (P.G0[d] + gh);
    }
}

// Appendix steps 3-4 on face f of axis a: the face value of f-bar-plus
// (linear in the normal direction) minus h xi . grad, with the normal
// gradient from the two cells and each tangential gradient from the two
// cells' cell-centred derivatives (bilinear cross-point difference).
template <class LAT, typename T>
__device__ void recon_face(const Inst<T>& P, const T* __restrict__ phi, int a, int f, const int* ci, T* out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    int cl[3] = {ci[0], ci[1], ci[2]}, cr[3] = {ci[0], ci[1], ci[2]};
    cl[a] = f - 1;
    cr[a] = f;
    const long long iL = ext_idx<LAT, T>(P, cl[0], cl[1], cl[2]);
    const long long iR = ext_idx<LAT, T>(P, cr[0], cr[1], cr[2]);
    const T w = P.m[a].w[f];
    const T hg = P.h * P.m[a].gn[f];
    long long st[3];
    st[0] = 1;
    st[1] = P.E[0];
    st[2] = (long long)P.E[0] * P.E[1];
    T cp[3], c0[3], cm[3];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        if (t == a) continue;
        cp[t] = P.m[t].cp[ci[t]];
        c0[t] = P.m[t].c0[ci[t]];
        cm[t] = P.m[t].cm[ci[t]];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T* pq = phi + (long long)q * P.ne;
        const T pL = pq[iL], pR = pq[iR];
        T v = pL + w * (pR - pL) - xi_of<LAT, T>(q, a, P.c) * hg * (pR - pL);
#pragma unroll
        for (int t = 0; t < D; ++t) {
            if (t == a || LAT::e(q, t) == 0) continue;
            const T dL = cp[t] * pq[iL + st[t]] + c0[t] * pL + cm[t] * pq[iL - st[t]];
            const T dR = cp[t] * pq[iR + st[t]] + c0[t] * pR + cm[t] * pq[iR - st[t]];
            v -= P.h * xi_of<LAT, T>(q, t, P.c) * (dL + w * (dR - dL));
        }
        out[q] = v;
    }
}

// interface moments (Appendix step 6): rho, u = j/rho0 + h/2 G
template <class LAT, typename T>
__device__ __forceinline__ void face_moments(const Inst<T>& P, const T* fb, const T* G, T& rho, T* u)
{
    rho = T(0);
    T j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < LAT::Q; ++q) {
        rho += fb[q];
#pragma unroll
        for (int a = 0; a < LAT::D; ++a) {
            if (LAT::e(q, a) == 1) j[a] += fb[q];
            if (LAT::e(q, a) == -1) j[a] -= fb[q];
        }
    }
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) u[a] = P.c * j[a] / P.rho0 + T(0.5) * P.h * G[a];
}

// Appendix step 5 on a wall face of side s.  wall: reconstructed values on
// the wall face (modified in place for the velocities entering the domain);
// oppf: reconstructed values on the opposite interface of the same wall
// cell; Gopp: acceleration there.
template <class LAT, typename T>
__device__ void wall_rule(const Inst<T>& P, int s, T* wall, const T* oppf, const T* Gopp)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const int a = s >> 1;
    const int sg = (s & 1) ? 1 : -1;  // outward normal = sg e_a
    const T invRT = T(1) / P.RT;
    const int kind = P.bc[s];
    if (kind == BC_BOUNCE_BACK) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (LAT::e(q, a) * sg >= 0) continue;
            T xu = T(0);
#pragma unroll
            for (int d = 0; d < D; ++d) xu += xi_of<LAT, T>(q, d, P.c) * P.uw[s][d];
            wall[q] = wall[LAT::opp(q)] + T(2) * P.rho0 * T(LAT::w(q)) * xu * invRT;
        }
        return;
    }
    T rc, uc[3];
    face_moments<LAT, T>(P, oppf, Gopp, rc, uc);
    T ra, ua[3];
    if (kind == BC_NEQ_VELOCITY) {
        ra = rc;
#pragma unroll
        for (int d = 0; d < D; ++d) ua[d] = P.uw[s][d];
    } else {
        ra = P.rhow[s];
#pragma unroll
        for (int d = 0; d < D; ++d) ua[d] = uc[d];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (LAT::e(q, a) * sg >= 0) continue;
        wall[q] = feq_q<LAT, T>(q, ra, ua, P.rho0, P.c, invRT) +
                  (oppf[q] - feq_q<LAT, T>(q, rc, uc, P.rho0, P.c, invRT));
    }
}

// Appendix step 7 for the velocities that cross a face of axis a
template <class LAT, typename T>
__device__ __forceinline__ void face_original(const Inst<T>& P, int a, T* fb, const T* G)
{
    const T invRT = T(1) / P.RT;
    T rho, u[3];
    face_moments<LAT, T>(P, fb, G, rho, u);
#pragma unroll
    for (int q = 0; q < LAT::Q; ++q) {
        if (LAT::e(q, a) == 0) continue;
        const T fe = feq_q<LAT, T>(q, rho, u, P.rho0, P.c, invRT);
        const T S = src_fac<LAT, T>(q, u, G, P.c, invRT) * fe;
        fb[q] = fb[q] + P.B7 * (fe - fb[q]) + P.C7 * S;
    }
}

template <class LAT, typename T>
__device__ void update_body(const Inst<T>& P, long long cidx, const T* __restrict__ f, const T* __restrict__ force,
                            const T* __restrict__ phi, T* __restrict__ fout, T gth)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    const long long ie = ext_idx<LAT, T>(P, ci[0], ci[1], ci[2]);
    T acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T p = phi[(long long)q * P.ne + ie];
        acc[q] = p + (p - f[(long long)q * P.nc + cidx]) * T(1.0 / 3.0);  // Eq. (f_tilde_+)
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T fm[Q], fp[Q], Gm[3], Gp[3];
        const int fmi = ci[a], fpi = ci[a] + 1;
        recon_face<LAT, T>(P, phi, a, fmi, ci, fm);
        recon_face<LAT, T>(P, phi, a, fpi, ci, fp);
        face_force<LAT, T>(P, force, a, fmi, ci, gth, Gm);
        face_force<LAT, T>(P, force, a, fpi, ci, gth, Gp);
        if (!P.per[a]) {
            if (ci[a] == 0) wall_rule<LAT, T>(P, 2 * a, fm, fp, Gp);
            if (ci[a] == P.n[a] - 1) wall_rule<LAT, T>(P, 2 * a + 1, fp, fm, Gm);
        }
        face_original<LAT, T>(P, a, fm, Gm);
        face_original<LAT, T>(P, a, fp, Gp);
        const T s = P.m[a].fdx[ci[a]];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (LAT::e(q, a) == 0) continue;
            const T flux = (fp[q] - fm[q]) * s;
            acc[q] = (LAT::e(q, a) > 0) ? acc[q] - P.c * flux : acc[q] + P.c * flux;
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) fout[(long long)q * P.nc + cidx] = acc[q];
}

template <class LAT, typename T>
__device__ void init_body(const Inst<T>& P, long long ci, const T* rho, const T* u, const T* force, T gt,
                          T* fout)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const T invRT = T(1) / P.RT;
    const T r = rho ? rho[ci] : P.rho0;
    T uu[3] = {T(0), T(0), T(0)}, G[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (u) uu[a] = u[(long long)a * P.nc + ci];
        G[a] = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + ci] : T(0)));
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T fe = feq_q<LAT, T>(q, r, uu, P.rho0, P.c, invRT);
        fout[(long long)q * P.nc + ci] = fe - P.h * src_fac<LAT, T>(q, uu, G, P.c, invRT) * fe;
    }
}

}  // namespace dugks
