// inst.hpp -- per-problem parameters seen by the kernels, and the
// point-local formulas of the scheme (Sec. II) as device functions.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace dugks {

enum { BC_PERIODIC = 0, BC_NEQ_VELOCITY = 1, BC_NEQ_PRESSURE = 2, BC_BOUNCE_BACK = 3 };

// Metric table of one axis with n cells, element type T, stored back to back
// in device memory:
//   w  [n+1]  face f between cells f-1 and f: weight of the right cell in the
//             linear interpolation to the face
//   gn [n+1]  face f: 1/(x_f - x_{f-1})   (normal difference)
//   cp [n], c0 [n], cm [n]
//             cell-centred tangential derivative along this axis:
//             d(i) = cp phi(i+1) + c0 phi(i) + cm phi(i-1); it is the difference
//             of the interpolated values on the two faces of cell i over its
//             width, so the tangential gradient on a face of another axis is
//             (1-w) d(L) + w d(R), the bilinear cross-point difference
//   fdx[n]    dt / Delta_i   (micro-flux scale, s_j/|V| = 1/Delta)
//   dl [n]    Delta_i        (cell width)
// Periodic axes use the wrapped, L-shifted neighbour centres and w[n] = w[0],
// gn[n] = gn[0].  Wall axes use mirrored ghost centres.
template <typename T>
struct AxisMetric {
    const T* w;
    const T* gn;
    const T* cp;
    const T* c0;
    const T* cm;
    const T* fdx;
    const T* dl;
};

template <typename T>
struct Inst {
    int n[3];      // cells per axis (1 on the absent z of 2-D)
    int E[3];      // extended extent n+2 on active axes, 1 otherwise
    int per[3];    // periodic flag (1 on the absent axis)
    int bc[6];
    long long nc;  // interior cells
    long long ne;  // extended cells (with one ghost layer on active axes)
    long long off; // element offset of this instance's state (batched)
    long long foff;// element offset of its force field, -1 = none (batched)
    long long poff;// element offset of its f-bar-plus scratch (batched)
    T rho0, RT, c, h, dt;
    T B1, C1;      // Eq. (f_bar_+) in deviation form: phi = f + B1 (feq - f) + C1 S
    T B7, C7;      // Eq. (original_f) inverted: f = fbar + B7 (feq - fbar) + C7 S
    // update without the cell's own state (no acceleration):
    // f~(n+1) = phi + Bu (feq - phi) - fluxes, Bu = B1 / (3 (1 - B1)), from
    // Eq. (f_tilde_+) with f~ = (phi - B1 feq) / (1 - B1).  Bu has a pole at
    // B1 = 1 (dt = 4 tau) and multiplies the rounding of feq - phi by
    // 1/(1 - B1), so the form is allowed (bu_ok = 1) only for |1 - B1| >= 1/4
    T Bu;
    int bu_ok;
    T G0[3];
    // point-formula constants (host-computed): c / rho0, 1 / RT and the
    // factored Eqs. (icfeq), (S): eqH = rho0 / (2 RT), eqB = rho0 c / RT,
    // eqC = rho0 c^2 / (2 RT^2), sG = c / RT
    T crho, invRT, eqH, eqB, eqC, sG;
    // model 1 (original DUGKS, Eq. feq): the same constants per unit density
    // (hRT = 1 / (2 RT), cRT = c / RT, c2RT2 = c^2 / (2 RT^2)); orig = 1
    int orig;
    T hRT, cRT, c2RT2;
    // uniform mesh (every active axis): uni = 1 and per axis, with
    // Delta = L / N, the face weight is 1/2 and the derivative coefficients
    // are ugn = 1 / Delta (normal difference), uct = 1 / (4 Delta) (the face's
    // tangential derivative times 1/2 per neighbour difference) and
    // ufdx = dt / Delta (flux scale)
    int uni;
    T ugn[3], uct[3], ufdx[3];
    T uw[6][3];
    T rhow[6];     // rho0 + p_w / RT (pressure condition)
    T rhowo[6];    // oscillating part of the wall density: p_w,osc / RT
    T rlo[3], rhi[3]; // ghost(-1) = (1-rlo) phi(0) + rlo phi(1); ghost(n) likewise
    double omega, phase;
    double dtd;    // dt in double (time stamps of the time factor)
    AxisMetric<T> m[3];
};

// per-instance launch geometry of the batched fused kernel
struct BatchGeom {
    int tiles0, tiles1, chunk, pad;
};

template <typename T>
__host__ __device__ inline T tfac(const Inst<T>& P, double t)
{
    return (T)cos(P.omega * t + P.phase);
}

// density of the pressure condition of Eq. (NEQ) on side s, rho0 +
// p_w(t) / RT with p_w(t) = p_w + p_w,osc g(t); gth = g at the interface
// time of the step
template <typename T>
__host__ __device__ inline T wall_density(const Inst<T>& P, int s, T gth)
{
    return P.rhow[s] + P.rhowo[s] * gth;
}

// Eq. (icfeq): incompressible equilibrium, xi.u = c (e.u)
template <class LAT, typename T>
__device__ __forceinline__ T feq_q(int q, T rho, const T* u, T rho0, T c, T invRT)
{
    T eu = T(0), uu = T(0);
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) {
        if (LAT::e(q, a) == 1) eu += u[a];
        if (LAT::e(q, a) == -1) eu -= u[a];
        uu += u[a] * u[a];
    }
    const T xu = c * eu;
    return T(LAT::w(q)) * (rho + rho0 * invRT * (xu + T(0.5) * xu * xu * invRT - T(0.5) * uu));
}

// Eq. (S) with the incompressible equilibrium: G.(xi - u)/RT feq
template <class LAT, typename T>
__device__ __forceinline__ T src_fac(int q, const T* u, const T* G, T c, T invRT)
{
    T s = T(0);
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) {
        const int e = LAT::e(q, a);
        s += G[a] * ((e == 0 ? T(0) : (e > 0 ? c : -c)) - u[a]);
    }
    return s * invRT;
}

// Eqs. (icfeq) and (S) at one point, factored for evaluation over many
// velocities: with eu = e_q . u,
//   feq_q = W_q (a + eu (eqB + eqC eu)),   a = rho - eqH |u|^2,
//   S_q   = (sG e_q . G - g) feq_q,         g = G . u / RT,
// i.e. Eq. (icfeq) with xi = c e expanded in powers of e.u, and Eq. (S)
// with xi . G = c e . G.  Per point: a, g and the vectors; per velocity a
// few fused multiply-adds.
template <typename T>
struct EqPt {
    T a, g;
    T B, C;  // per point in the original model (rho cRT, rho c2RT2)
    T u[3], G[3];
};

// ORIG: the original model's Eq. (feq) = W_q rho [1 + xi.u/RT + (xi.u)^2 /
// (2 RT^2) - |u|^2/(2 RT)], i.e. a = rho (1 - hRT |u|^2), and the eu
// coefficients carry rho instead of rho0.
template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ EqPt<T> eq_point(const Inst<T>& P, T rho, const T* u, const T* G)
{
    EqPt<T> E;
    T uu = T(0), gu = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        E.u[a] = a < LAT::D ? u[a] : T(0);
        E.G[a] = (a < LAT::D && G) ? G[a] : T(0);
    }
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) {
        uu += E.u[a] * E.u[a];
        gu += E.G[a] * E.u[a];
    }
    if constexpr (ORIG) {
        E.a = rho - rho * P.hRT * uu;
        E.B = rho * P.cRT;
        E.C = rho * P.c2RT2;
    } else {
        E.a = rho - P.eqH * uu;
        E.B = P.eqB;
        E.C = P.eqC;
    }
    E.g = gu * P.invRT;
    return E;
}

// e_q . v for a compile-time velocity q
template <class LAT, typename T>
__device__ __forceinline__ T e_dot(int q, const T* v)
{
    T s = T(0);
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) {
        if (LAT::e(q, a) == 1) s += v[a];
        if (LAT::e(q, a) == -1) s -= v[a];
    }
    return s;
}

template <class LAT, typename T, bool ORIG = false>
__device__ __forceinline__ T feq_pt(const Inst<T>& P, const EqPt<T>& E, int q)
{
    const T eu = e_dot<LAT, T>(q, E.u);
    if constexpr (ORIG) return T(LAT::w(q)) * (E.a + eu * (E.B + E.C * eu));
    else return T(LAT::w(q)) * (E.a + eu * (P.eqB + P.eqC * eu));
}

// velocity from the momentum moment j = sum e f (a sum of the state's
// components), the acceleration G and its time weight hw (dt/2 at cells,
// h/2 at faces): u = c j / rho0 + hw G (Eq. macro_values), or, in the
// original model, rho u = c j + rho hw G
template <typename T, bool ORIG = false>
__device__ __forceinline__ T vel_from(const Inst<T>& P, T rho, T j, T G, T hw)
{
    if constexpr (ORIG) return P.c * j / rho + hw * G;
    else return P.crho * j + hw * G;
}

// S_q / feq_q
template <class LAT, typename T>
__device__ __forceinline__ T srcf_pt(const Inst<T>& P, const EqPt<T>& E, int q)
{
    return e_dot<LAT, T>(q, E.G) * P.sG - E.g;
}

template <class LAT, typename T>
__device__ __forceinline__ T xi_of(int q, int a, T c)
{
    const int e = LAT::e(q, a);
    return e == 0 ? T(0) : (e > 0 ? c : -c);
}

}  // namespace dugks
