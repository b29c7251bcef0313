// kernels_general.hpp -- general step kernels (any lattice, mesh, wall kind,
// force), used for every configuration and as the batched path.
//
// Pass 1 (k_phi): f-bar-plus (Eq. f_bar_+) on every cell of the ghost-extended
//   grid (Eq. f_bar_+ and the ghost rule); a ghost takes the linear extrapolation through
//   the two nearest centres of each wall axis (tensor product on edges and
//   corners) or the wrapped cell of a periodic axis.
// Pass 2 (k_update): per interior cell, both faces of every axis are
//   reconstructed from pass 1 (Eq. gradient), wall rules applied (Eqs. BB, NEQ),
//   interface moments and the original distribution formed (Eq. original_f), and
//   the conservative update written (Eqs. microflux, f_tilde_+).  Interior faces are thus
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

// f-bar-plus of one interior cell (Eq. f_bar_+) from its state fv[Q]
// and its force-field values fg[D] (used if has_field)
template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void phi_from(const Inst<T>& P, const T (&fv)[LAT::Q], const T (&fg)[3], bool has_field,
                                         T gt, T* out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    T rho = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
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
        G[a] = gt * (P.G0[a] + (has_field ? fg[a] : T(0)));
        u[a] = vel_from<T, ORIG>(P, rho, j[a], G[a], P.h);
    }
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, rho, u, G);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T fe = feq_pt<LAT, T, ORIG>(P, E, q);
        const T S = srcf_pt<LAT, T>(P, E, q) * fe;
        out[q] = fv[q] + P.B1 * (fe - fv[q]) + P.C1 * S;
    }
}

// the same, loading the cell's state and force field from HBM
template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void phi_cell(const Inst<T>& P, const T* __restrict__ f, const T* __restrict__ force, long long ci,
                         T gt, T* out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    T fv[Q], fg[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Q; ++q) fv[q] = f[(long long)q * P.nc + ci];
    if (force) {
#pragma unroll
        for (int a = 0; a < D; ++a) fg[a] = force[(long long)a * P.nc + ci];
    }
    phi_from<LAT, T, ORIG>(P, fv, fg, force != nullptr, gt, out);
}

template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void phi_ext_body(const Inst<T>& P, long long e, const T* __restrict__ f, const T* __restrict__ force,
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
        phi_cell<LAT, T, ORIG>(P, f, force, int_idx(P, idx[0][0], idx[1][0], idx[2][0]), gt, acc);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] = T(0);
        for (int i2 = 0; i2 < cnt[2]; ++i2)
            for (int i1 = 0; i1 < cnt[1]; ++i1)
                for (int i0 = 0; i0 < cnt[0]; ++i0) {
                    T tmp[Q];
                    phi_cell<LAT, T, ORIG>(P, f, force, int_idx(P, idx[0][i0], idx[1][i1], idx[2][i2]), gt, tmp);
                    const T w = wt[0][i0] * wt[1][i1] * wt[2][i2];
#pragma unroll
                    for (int q = 0; q < Q; ++q) acc[q] += w * tmp[q];
                }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) phi[(long long)q * P.ne + e] = acc[q];
}

// run-time-axis selects of per-axis fields (no address of the by-value
// kernel argument is taken, so it stays in scalar registers)
#define SEL3(arr, a) ((a) == 0 ? (arr)[0] : ((a) == 1 ? (arr)[1] : (arr)[2]))

// spatial force component d at the cell whose axis-a coordinate is x (which
// may be a ghost), other coordinates from ci; ghosts follow the phi rule
template <class LAT, typename T>
__device__ __forceinline__ T force_at(const Inst<T>& P, const T* __restrict__ force, int d, int a, int x,
                                      const int* ci)
{
    const int N = SEL3(P.n, a);
    const T* fd = force + (long long)d * P.nc;
    const long long sa = a == 0 ? 1LL : (a == 1 ? (long long)P.n[0] : (long long)P.n[0] * P.n[1]);
    const int x0 = ci[0], y0 = ci[1], z0 = ci[2];
    const long long c0 = int_idx(P, x0, y0, z0) - (long long)(a == 0 ? x0 : (a == 1 ? y0 : z0)) * sa;
    if (x >= 0 && x < N) return fd[c0 + x * sa];
    if (SEL3(P.per, a)) return fd[c0 + (x < 0 ? N - 1 : 0) * sa];
    const T r = x < 0 ? SEL3(P.rlo, a) : SEL3(P.rhi, a);
    const T v0 = fd[c0 + (x < 0 ? 0 : N - 1) * sa];
    const T v1 = fd[c0 + (x < 0 ? 1 : N - 2) * sa];
    return (T(1) - r) * v0 + r * v1;
}

// acceleration on face f of axis a (between cells f-1 and f) at time factor
// gth; w = interpolation weight of the face
template <class LAT, typename T>
__device__ __forceinline__ void face_force(const Inst<T>& P, const T* __restrict__ force, int a, int f, T w,
                                           const int* ci, T gth, T* G)
{
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

// Accessor of f-bar-plus in the ghost-extended global array, relative to
// the cell the thread updates: base(ox,oy,oz) gives the element offset of a
// neighbour, up(t)/dn(t) the offset to its +t / -t neighbour, get(q, b) the
// value of velocity q there.
template <class LAT, typename T>
struct GlobalPhi {
    const T* __restrict__ phi;
    long long ne, ie, s1, s2;
    __device__ __forceinline__ long long base(int ox, int oy, int oz) const { return ie + ox + oy * s1 + oz * s2; }
    __device__ __forceinline__ long long up(int t) const { return t == 0 ? 1 : (t == 1 ? s1 : s2); }
    __device__ __forceinline__ long long dn(int t) const { return up(t); }
    __device__ __forceinline__ T get(int q, long long b) const { return phi[(long long)q * ne + b]; }
};

// Metric coefficients one cell needs along one axis, held in registers:
// interpolation weight and normal-difference scale of its two faces, its
// cell-centred derivative coefficients and its flux scale dt/Delta.
template <typename T>
struct CellMetric {
    T wl, wu, gl, gu, cp, c0, cm, fdx;
};

template <typename T>
__device__ __forceinline__ CellMetric<T> load_metric(const Inst<T>& P, int a, int i)
{
    const AxisMetric<T>& m = P.m[a];
    return CellMetric<T>{m.w[i], m.w[i + 1], m.gn[i], m.gn[i + 1], m.cp[i], m.c0[i], m.cm[i], m.fdx[i]};
}

// interface moments (Eq. macro_values at the interface): rho, u = j/rho0 + h/2 G
template <class LAT, typename T, bool ORIG = false>
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
    for (int a = 0; a < LAT::D; ++a) u[a] = vel_from<T, ORIG>(P, rho, j[a], G[a], T(0.5) * P.h);
#pragma unroll
    for (int a = LAT::D; a < 3; ++a) u[a] = T(0);
}

// What the NEQ rule needs from the opposite interface x_c of a wall cell:
// its moments and, for the velocities crossing the axis, the
// non-equilibrium part f-bar - feq(rho_c, u_c).
template <class LAT, typename T>
struct NeqInfo {
    T rc, uc[3];
    T neq[LAT::Q];
};

template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void neq_capture(const Inst<T>& P, int a, const T* oppf, const T* Gopp,
                                            NeqInfo<LAT, T>& I)
{
    face_moments<LAT, T, ORIG>(P, oppf, Gopp, I.rc, I.uc);
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, I.rc, I.uc, nullptr);
#pragma unroll
    for (int q = 0; q < LAT::Q; ++q) {
        if (LAT::e(q, a) == 0) continue;
        I.neq[q] = oppf[q] - feq_pt<LAT, T, ORIG>(P, E, q);
    }
}

// the wall rules of Eqs. (BB), (NEQ) on a wall face of side s, in place on the
// reconstructed values, for the velocities entering the domain.
template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void wall_rule(const Inst<T>& P, int s, T* wall, const NeqInfo<LAT, T>& I, T gth)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const int a = s >> 1;
    const int sg = (s & 1) ? 1 : -1;  // outward normal = sg e_a
    const int kind = P.bc[s];
    if (kind == BC_BOUNCE_BACK) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (LAT::e(q, a) * sg >= 0) continue;
            T xu = T(0);
#pragma unroll
            for (int d = 0; d < D; ++d) xu += xi_of<LAT, T>(q, d, P.c) * P.uw[s][d];
            wall[q] = wall[LAT::opp(q)] + T(2) * P.rho0 * T(LAT::w(q)) * xu * P.invRT;
        }
        return;
    }
    T ra, ua[3];
    if (kind == BC_NEQ_VELOCITY) {
        ra = I.rc;
#pragma unroll
        for (int d = 0; d < D; ++d) ua[d] = P.uw[s][d];
    } else {
        ra = wall_density(P, s, gth);
#pragma unroll
        for (int d = 0; d < D; ++d) ua[d] = I.uc[d];
    }
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, ra, ua, nullptr);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (LAT::e(q, a) * sg >= 0) continue;
        wall[q] = feq_pt<LAT, T, ORIG>(P, E, q) + I.neq[q];
    }
}

// the inverse of Eq. (original_f) for the velocities that cross a face of axis a
template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void face_original(const Inst<T>& P, int a, T* fb, const T* G)
{
    T rho, u[3];
    face_moments<LAT, T, ORIG>(P, fb, G, rho, u);
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, rho, u, G);
#pragma unroll
    for (int q = 0; q < LAT::Q; ++q) {
        if (LAT::e(q, a) == 0) continue;
        const T fe = feq_pt<LAT, T, ORIG>(P, E, q);
        const T S = srcf_pt<LAT, T>(P, E, q) * fe;
        fb[q] = fb[q] + P.B7 * (fe - fb[q]) + P.C7 * S;
    }
}

// Eq. (gradient), compile-time axis A, run-time side (see recon_face)
template <class LAT, typename T, class ACC, int A>
__device__ __forceinline__ void recon_face_ct(const Inst<T>& P, const ACC& ph, bool upper, const CellMetric<T>& ma,
                                              const CellMetric<T>& mx, const CellMetric<T>& my,
                                              const CellMetric<T>& mz, T* out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const int lo = upper ? 0 : -1;
    const auto bL = ph.base(A == 0 ? lo : 0, A == 1 ? lo : 0, A == 2 ? lo : 0);
    const auto bR = ph.base(A == 0 ? lo + 1 : 0, A == 1 ? lo + 1 : 0, A == 2 ? lo + 1 : 0);
    const T w = upper ? ma.wu : ma.wl;
    const T hcg = P.h * P.c * (upper ? ma.gu : ma.gl);
    const T hc = P.h * P.c;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T pL = ph.get(q, bL), pR = ph.get(q, bR);
        T v = pL + w * (pR - pL) - T(LAT::e(q, A)) * hcg * (pR - pL);
#pragma unroll
        for (int t = 0; t < D; ++t) {
            if (t == A || LAT::e(q, t) == 0) continue;
            const CellMetric<T>& mt = t == 0 ? mx : (t == 1 ? my : mz);
            const auto u = ph.up(t), d = ph.dn(t);
            const T dL = mt.cp * ph.get(q, bL + u) + mt.c0 * pL + mt.cm * ph.get(q, bL - d);
            const T dR = mt.cp * ph.get(q, bR + u) + mt.c0 * pR + mt.cm * ph.get(q, bR - d);
            v -= T(LAT::e(q, t)) * hc * (dL + w * (dR - dL));
        }
        out[q] = v;
    }
}

template <class LAT, typename T, class ACC, int A, bool ORIG = false>
__device__ __forceinline__ void axis_fluxes_ct(const Inst<T>& P, const ACC& ph, const T* __restrict__ force,
                                               const int* ci, T gth, const CellMetric<T>& mx,
                                               const CellMetric<T>& my, const CellMetric<T>& mz, T* acc)
{
    constexpr int Q = LAT::Q;
    const CellMetric<T>& ma = A == 0 ? mx : (A == 1 ? my : mz);
    const int ca = ci[A];
    const bool wlo = !P.per[A] && ca == 0;
    const bool whi = !P.per[A] && ca == P.n[A] - 1;
    NeqInfo<LAT, T> info;
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
        // k = 0: the face that is not a wall of this cell (upper face if the
        // lower one is a wall), k = 1: the other one
        const bool upper = wlo ? (k == 0) : (k == 1);
        asm volatile("" ::: "memory");
        T fb[Q], G[3];
        recon_face_ct<LAT, T, ACC, A>(P, ph, upper, ma, mx, my, mz, fb);
        face_force<LAT, T>(P, force, A, upper ? ca + 1 : ca, upper ? ma.wu : ma.wl, ci, gth, G);
        const bool wall_here = upper ? whi : wlo;
        if (k == 0 && (wlo != whi)) neq_capture<LAT, T, ORIG>(P, A, fb, G, info);
        if (wall_here) wall_rule<LAT, T, ORIG>(P, upper ? 2 * A + 1 : 2 * A, fb, info, gth);
        face_original<LAT, T, ORIG>(P, A, fb, G);
        const T s = ma.fdx * P.c;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (LAT::e(q, A) == 0) continue;
            // upper face: outward normal +e_A; lower face: -e_A
            const T fl = (upper ? fb[q] : -fb[q]) * s;
            acc[q] = (LAT::e(q, A) > 0) ? acc[q] - fl : acc[q] + fl;
        }
    }
}

// ---------------------------------------------------------------------------
// faces evaluated once (fused kernel v2): the value of the interface of axis
// A with index f between the cells at offsets off and off+1 (relative to the
// thread's cell), after reconstruction, wall rules and Eq. (original_f); walls handled in place.
// ---------------------------------------------------------------------------

// index of velocity q among the velocities crossing a face of axis A
template <class LAT, int A>
__host__ __device__ constexpr int cross_slot(int q)
{
    int s = 0;
    for (int r = 0; r < q; ++r)
        if (LAT::e(r, A) != 0) ++s;
    return s;
}
template <class LAT, int A>
__host__ __device__ constexpr int cross_count()
{
    return cross_slot<LAT, A>(LAT::Q);
}

template <class LAT, typename T, class ACC, int A, bool UNI>
__device__ __forceinline__ void recon_at(const Inst<T>& P, const ACC& ph, int off, T w, T gn, const CellMetric<T>& mx,
                                         const CellMetric<T>& my, const CellMetric<T>& mz, T* out)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const auto bL = ph.base(A == 0 ? off : 0, A == 1 ? off : 0, A == 2 ? off : 0);
    const auto bR = ph.base(A == 0 ? off + 1 : 0, A == 1 ? off + 1 : 0, A == 2 ? off + 1 : 0);
    const T hcg = P.h * P.c * gn;
    const T hc = P.h * P.c;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T pL = ph.get(q, bL), pR = ph.get(q, bR);
        T v;
        if constexpr (UNI) v = T(0.5) * (pL + pR);
        else v = pL + w * (pR - pL);
        if (LAT::e(q, A) != 0) v -= T(LAT::e(q, A)) * hcg * (pR - pL);
#pragma unroll
        for (int t = 0; t < D; ++t) {
            if (t == A || LAT::e(q, t) == 0) continue;
            const auto u = ph.up(t), d = ph.dn(t);
            if constexpr (UNI) {
                // uniform mesh: (1/2)(d(L) + d(R)), d = (phi(+t) - phi(-t)) / (2 Delta)
                const T s = (ph.get(q, bL + u) - ph.get(q, bL - d)) + (ph.get(q, bR + u) - ph.get(q, bR - d));
                v -= T(LAT::e(q, t)) * (hc * P.uct[t]) * s;
            } else {
                const CellMetric<T>& mt = t == 0 ? mx : (t == 1 ? my : mz);
                const T dL = mt.cp * ph.get(q, bL + u) + mt.c0 * pL + mt.cm * ph.get(q, bL - d);
                const T dR = mt.cp * ph.get(q, bR + u) + mt.c0 * pR + mt.cm * ph.get(q, bR - d);
                v -= T(LAT::e(q, t)) * hc * (dL + w * (dR - dL));
            }
        }
        out[q] = v;
    }
}

// ci: global cell coordinates of the thread's cell (tangential ones are
// used for metrics and force); f: face index along A.  out[cross_slot]
// receives f_q (Eq. original_f inverted) for the velocities crossing the face.
template <class LAT, typename T, class ACC, int A, bool UNI>
__device__ __forceinline__ void face_once(const Inst<T>& P, const ACC& ph, const T* __restrict__ force, const int* ci,
                                          int off, int f, T gth, const CellMetric<T>& mx, const CellMetric<T>& my,
                                          const CellMetric<T>& mz, T* out)
{
    constexpr int Q = LAT::Q;
    const AxisMetric<T>& m = P.m[A];
    const int n = P.n[A];
    const bool wall_lo = !P.per[A] && f == 0;
    const bool wall_hi = !P.per[A] && f == n;
    NeqInfo<LAT, T> info;
    asm volatile("" ::: "memory");
    T fb[Q], G[3];
    if (wall_lo || wall_hi) {
        // the opposite interface of the wall cell (its NEQ information)
        const int fo = wall_lo ? 1 : n - 1;
        const int oo = wall_lo ? off + 1 : off - 1;
        const T wo = UNI ? T(0.5) : m.w[fo];
        recon_at<LAT, T, ACC, A, UNI>(P, ph, oo, wo, UNI ? P.ugn[A] : m.gn[fo], mx, my, mz, fb);
        face_force<LAT, T>(P, force, A, fo, wo, ci, gth, G);
        neq_capture<LAT, T>(P, A, fb, G, info);
        asm volatile("" ::: "memory");
    }
    const T w = UNI ? T(0.5) : m.w[f];
    recon_at<LAT, T, ACC, A, UNI>(P, ph, off, w, UNI ? P.ugn[A] : m.gn[f], mx, my, mz, fb);
    face_force<LAT, T>(P, force, A, f, w, ci, gth, G);
    if (wall_lo) wall_rule<LAT, T>(P, 2 * A, fb, info, gth);
    if (wall_hi) wall_rule<LAT, T>(P, 2 * A + 1, fb, info, gth);
    face_original<LAT, T>(P, A, fb, G);
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (LAT::e(q, A) != 0) out[cross_slot<LAT, A>(q)] = fb[q];
}

// The interface and update stages for one cell: acc holds f~+ on entry (Eq. f_tilde_+) and the
// updated state on exit.  Faces are taken one at a time; on a wall axis the
// opposite (interior) face is evaluated first so that the NEQ rule can use
// its moments and non-equilibrium part.
template <class LAT, typename T, class ACC, bool ORIG = false>
__device__ __forceinline__ void cell_fluxes(const Inst<T>& P, const ACC& ph, const T* __restrict__ force,
                                            const int* ci, T gth, const CellMetric<T> cx, const CellMetric<T> cy,
                                            const CellMetric<T> cz, T* acc)
{
    axis_fluxes_ct<LAT, T, ACC, 0, ORIG>(P, ph, force, ci, gth, cx, cy, cz, acc);
    axis_fluxes_ct<LAT, T, ACC, 1, ORIG>(P, ph, force, ci, gth, cx, cy, cz, acc);
    if constexpr (LAT::D == 3) axis_fluxes_ct<LAT, T, ACC, 2, ORIG>(P, ph, force, ci, gth, cx, cy, cz, acc);
}

template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void update_body(const Inst<T>& P, long long cidx, const T* __restrict__ f, const T* __restrict__ force,
                            const T* __restrict__ phi, T* __restrict__ fout, T gth)
{
    constexpr int Q = LAT::Q;
    int ci[3];
    ci[0] = (int)(cidx % P.n[0]);
    long long r = cidx / P.n[0];
    ci[1] = (int)(r % P.n[1]);
    ci[2] = (int)(r / P.n[1]);
    GlobalPhi<LAT, T> ph{phi, P.ne, ext_idx<LAT, T>(P, ci[0], ci[1], ci[2]), (long long)P.E[0],
                         (long long)P.E[0] * P.E[1]};
    T acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T p = ph.get(q, ph.base(0, 0, 0));
        acc[q] = p + (p - f[(long long)q * P.nc + cidx]) * T(1.0 / 3.0);  // Eq. (f_tilde_+)
    }
    const CellMetric<T> cx = load_metric(P, 0, ci[0]);
    const CellMetric<T> cy = load_metric(P, 1, ci[1]);
    const CellMetric<T> cz = LAT::D == 3 ? load_metric(P, 2, ci[2]) : cy;
    cell_fluxes<LAT, T, GlobalPhi<LAT, T>, ORIG>(P, ph, force, ci, gth, cx, cy, cz, acc);
#pragma unroll
    for (int q = 0; q < Q; ++q) fout[(long long)q * P.nc + cidx] = acc[q];
}

template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ void init_body(const Inst<T>& P, long long ci, const T* rho, const T* u, const T* force, T gt,
                          T* fout)
{
    constexpr int Q = LAT::Q, D = LAT::D;
    const T r = rho ? rho[ci] : P.rho0;
    T uu[3] = {T(0), T(0), T(0)}, G[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (u) uu[a] = u[(long long)a * P.nc + ci];
        G[a] = gt * (P.G0[a] + (force ? force[(long long)a * P.nc + ci] : T(0)));
    }
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, r, uu, G);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T fe = feq_pt<LAT, T, ORIG>(P, E, q);
        fout[(long long)q * P.nc + ci] = fe - P.h * srcf_pt<LAT, T>(P, E, q) * fe;
    }
}

}  // namespace dugks
