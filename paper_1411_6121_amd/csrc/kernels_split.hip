// kernels_split.hip -- the fused single-launch step with the velocity set
// split over two lanes per column.
//
// The march is that of the faces-once fused kernel (an LDS ring of three
// f-bar-plus planes, every interface evaluated once, x/y face values
// exchanged through LDS, the march-axis face carried in registers), but each
// column is served by two lanes of one wavefront, l and l^32.  Lane half 0
// owns the velocities q = 0..K-1 (K = index of the rest velocity) and the
// rest velocity; half 1 owns their opposites Q-1-k, whose components are
// -e(k) and whose weights are equal.  All per-velocity work (Eq. f_bar_+,
// reconstruction, equilibria, source, wall rules, fluxes, update) is done by
// the owning lane from the half-0 velocity table with the sign sigma = +-1
// folded into u, G and the xi-weighted coefficients; the velocity moments of
// cells and interfaces are partial sums added across the two lanes.  The
// halves of a column always take the same branches, so both partners of an
// exchange are active.  Halving the per-thread state and doubling the
// threads per tile raises occupancy at the same LDS footprint.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ctx.hpp"
#include "kernels_general.hpp"
#include "march.hpp"

namespace dugks {


// value of the partner lane (same column, other half): v_permlane32_swap
// exchanges lanes 32..63 of its first operand with lanes 0..31 of its second;
// with both operands = v the partner's value is the second result in the
// lower half-wave and the first in the upper one.  Both lanes of a pair are
// always active together.
__device__ __forceinline__ unsigned partner_u32(unsigned v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __lane_id() < 32 ? r[1] : r[0];
}
__device__ __forceinline__ float partner(float v)
{
    return __builtin_bit_cast(float, partner_u32(__builtin_bit_cast(unsigned, v)));
}
__device__ __forceinline__ double partner(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = partner_u32((unsigned)b), hi = partner_u32((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Lane-pair sums of two values at once: v_permlane32_swap(a, b) leaves
// (a(l), b(l-32)) in its first result and (a(l+32), b(l)) in its second, so
// one add gives the pair sum of a in the lower half-wave and that of b in
// the upper one; a second swap of that sum with a copy of itself hands both
// halves to every lane.  Each sum is the lower lane's value plus the upper
// one's, bitwise what both lanes get from v + partner(v).  The copy is made
// opaque to the compiler so that the swap never sees two equal operands.
__device__ __forceinline__ void pair_sum2_u32(unsigned a, unsigned b, unsigned& r0, unsigned& r1)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    r0 = r[0];
    r1 = r[1];
}
// M: how the pair is combined: 0 both sums plain; 1 a plain, b signed (the
// lane's sign sg, +1 in the lower and -1 in the upper half-wave); 2 both
// signed.  A signed sum is that of sg * x: the lower lane's value minus the
// upper one's, bitwise what sg * x + partner(sg * x) gives, since
// multiplying by -1 is exact.
template <int M>
__device__ __forceinline__ float pair_combine(float x0, float x1, float sg)
{
    if constexpr (M == 0) return x0 + x1;
    else if constexpr (M == 1) return __builtin_fmaf(sg, x1, x0);
    else return x0 - x1;
}
template <int M>
__device__ __forceinline__ double pair_combine(double x0, double x1, double sg)
{
    if constexpr (M == 0) return x0 + x1;
    else if constexpr (M == 1) return __builtin_fma(sg, x1, x0);
    else return x0 - x1;
}
template <int M = 0>
__device__ __forceinline__ void pair_sum2(float a, float b, float& sa, float& sb, float sg = 1.0f)
{
    unsigned x0, x1;
    pair_sum2_u32(__float_as_uint(a), __float_as_uint(b), x0, x1);
    const float sum = pair_combine<M>(__uint_as_float(x0), __uint_as_float(x1), sg);
    unsigned c = __float_as_uint(sum);
    asm volatile("" : "+v"(c));
    unsigned y0, y1;
    pair_sum2_u32(__float_as_uint(sum), c, y0, y1);
    sa = __uint_as_float(y0);
    sb = __uint_as_float(y1);
}
template <int M = 0>
__device__ __forceinline__ void pair_sum2(double a, double b, double& sa, double& sb, double sg = 1.0)
{
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    unsigned l0, l1, h0, h1;
    pair_sum2_u32((unsigned)ua, (unsigned)ub, l0, l1);
    pair_sum2_u32((unsigned)(ua >> 32), (unsigned)(ub >> 32), h0, h1);
    const double sum = pair_combine<M>(__longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0)),
                                       __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1)), sg);
    const unsigned long long us = (unsigned long long)__double_as_longlong(sum);
    unsigned clo = (unsigned)us, chi = (unsigned)(us >> 32);
    asm volatile("" : "+v"(clo), "+v"(chi));
    pair_sum2_u32((unsigned)us, clo, l0, l1);
    pair_sum2_u32((unsigned)(us >> 32), chi, h0, h1);
    sa = __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0));
    sb = __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
}
// the moments of a column from the two lanes' partial sums: rho = rh + rh
// of the partner lane, j[a] = the pair sum of sg * sj[a]
template <int D, typename T>
__device__ __forceinline__ void moment_sums(T rh, const T (&sj)[3], T sg, T& rho, T (&j)[3])
{
    pair_sum2<1>(rh, sj[0], rho, j[0], sg);
    if constexpr (D == 3) {
        pair_sum2<2>(sj[1], sj[2], j[1], j[2], sg);
    } else {
        const T x = sg * sj[1];
        j[1] = x + partner(x);
    }
}

// value of lane l + N (N > 0) or l - N (N < 0) of the lane's 16-lane row
// (DPP row shift; a source outside the row leaves an unspecified value)
template <int N>
__device__ __forceinline__ unsigned row_shift_u32(unsigned v)
{
    constexpr int ctrl = N > 0 ? 0x100 + N : 0x110 - N;  // row_shl:N / row_shr:-N
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xf, 0xf, false);
}
template <int N>
__device__ __forceinline__ float row_shift(float v)
{
    return __uint_as_float(row_shift_u32<N>(__float_as_uint(v)));
}
template <int N>
__device__ __forceinline__ double row_shift(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = row_shift_u32<N>((unsigned)b), hi = row_shift_u32<N>((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// number of half-0 velocities crossing a face of axis A, and the slot of k
template <class LAT, int A>
__host__ __device__ constexpr int half_cross_slot(int k)
{
    int s = 0;
    for (int r = 0; r < k; ++r)
        if (LAT::e(r, A) != 0) ++s;
    return s;
}
template <class LAT, int A>
__host__ __device__ constexpr int half_cross_count()
{
    return half_cross_slot<LAT, A>(LAT::REST);
}

// f-bar-plus in the LDS ring.  Slot layout of one plane: half-0 velocities
// k = 0..K-1 in slots 0..K-1, the rest velocity in slot K, half-1 velocities
// in slots K+1..2K; every slot is a BX x BY array of columns.
template <class LAT, typename T, int BX, int BY>
struct HalfPhi {
    const T* s;
    int cur;           // element offset of (current plane, slot 0, this column)
    int hb;            // element offset of this lane's first slot
    int dz_up, dz_dn;  // offset from the current plane to the next / previous
    static constexpr int SQ = BX * BY;
    __device__ __forceinline__ int base(int ox, int oy, int oz) const
    {
        if constexpr (LAT::D == 3) return cur + ox + oy * BX + (oz > 0 ? dz_up : (oz < 0 ? dz_dn : 0));
        else return cur + ox + (oy > 0 ? dz_up : (oy < 0 ? dz_dn : 0));
    }
    __device__ __forceinline__ int up(int t) const
    {
        if constexpr (LAT::D == 3) return t == 0 ? 1 : (t == 1 ? BX : dz_up);
        else return t == 0 ? 1 : dz_up;
    }
    __device__ __forceinline__ int dn(int t) const
    {
        if constexpr (LAT::D == 3) return t == 0 ? 1 : (t == 1 ? BX : -dz_dn);
        else return t == 0 ? 1 : -dz_dn;
    }
    __device__ __forceinline__ T get(int k, int b) const { return s[b + hb + k * SQ]; }
    __device__ __forceinline__ T rest(int b) const { return s[b + LAT::REST * SQ]; }
};

// cell moments and f-bar-plus (Eqs. macro_values, f_bar_+) of the lane's
// velocities; fv: lane velocities, fr: rest velocity (both lanes hold it)
template <class LAT, typename T, bool NOG = false, bool ORIG = false>
__device__ __forceinline__ void phi_half(const Inst<T>& P, const T (&fv)[LAT::REST], T fr, const T (&fg)[3],
                                         bool has_field, T gt, T sg, T (&out)[LAT::REST], T& orest)
{
    constexpr int K = LAT::REST, D = LAT::D;
    T rh = T(0), sj[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        rh += fv[k];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (LAT::e(k, a) == 1) sj[a] += fv[k];
            if (LAT::e(k, a) == -1) sj[a] -= fv[k];
        }
    }
    T rs, js[3];
    moment_sums<D>(rh, sj, sg, rs, js);
    const T rho = rs + fr;
    // original model: u = c j / rho (+ h G), with one division per point
    const T cir = ORIG ? P.c / rho : T(0);
    T G[3] = {T(0), T(0), T(0)}, u[3] = {T(0), T(0), T(0)}, us[3] = {T(0), T(0), T(0)}, Gs[3] = {T(0), T(0), T(0)};
    // without acceleration the lane-frame velocity directly: (sg c / rho0) j,
    // bitwise sg (c j / rho0)
    const T cu = sg * (ORIG ? cir : P.crho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T j = js[a];
        if constexpr (NOG) {
            us[a] = cu * j;
        } else {
            G[a] = gt * (P.G0[a] + (has_field ? fg[a] : T(0)));
            u[a] = ORIG ? cir * j + P.h * G[a] : vel_from<T, false>(P, rho, j, G[a], P.h);
            us[a] = sg * u[a];
        }
        Gs[a] = sg * G[a];
    }
    // NOG: no acceleration at all, the source term of Eq. (S) vanishes
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, rho, us, NOG ? nullptr : Gs);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const T fe = feq_pt<LAT, T, ORIG>(P, E, k);
        if constexpr (NOG) {
            out[k] = fv[k] + P.B1 * (fe - fv[k]);
        } else {
            const T S = srcf_pt<LAT, T>(P, E, k) * fe;
            out[k] = fv[k] + P.B1 * (fe - fv[k]) + P.C1 * S;
        }
    }
    const T fe = feq_pt<LAT, T, ORIG>(P, E, LAT::REST);
    if constexpr (NOG) {
        orest = fr + P.B1 * (fe - fr);
    } else {
        const T S = srcf_pt<LAT, T>(P, E, LAT::REST) * fe;
        orest = fr + P.B1 * (fe - fr) + P.C1 * S;
    }
}

// Eq. (gradient) for the lane's velocities on the interface of axis A
// between the cells at offsets off and off+1 (weight w of the right cell,
// normal-difference scale gn); the rest velocity (no gradient term) too
template <class LAT, typename T, class ACC, int A, bool UNI>
__device__ __forceinline__ void recon_half(const Inst<T>& P, const ACC& ph, int off, T w, T gn,
                                           const CellMetric<T>& mx, const CellMetric<T>& my,
                                           const CellMetric<T>& mz, T sg, T (&out)[LAT::REST], T& orest)
{
    constexpr int K = LAT::REST, D = LAT::D;
    const int bL = ph.base(A == 0 ? off : 0, A == 1 ? off : 0, A == 2 ? off : 0);
    const int bR = ph.base(A == 0 ? off + 1 : 0, A == 1 ? off + 1 : 0, A == 2 ? off + 1 : 0);
    const T hcg = sg * (P.h * P.c * gn);
    const T hc = sg * (P.h * P.c);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const T pL = ph.get(k, bL), pR = ph.get(k, bR);
        T v;
        if constexpr (UNI) v = T(0.5) * (pL + pR);
        else v = pL + w * (pR - pL);
        if (LAT::e(k, A) != 0) v -= T(LAT::e(k, A)) * hcg * (pR - pL);
#pragma unroll
        for (int t = 0; t < D; ++t) {
            if (t == A || LAT::e(k, t) == 0) continue;
            const int u = ph.up(t), d = ph.dn(t);
            if constexpr (UNI) {
                // uniform mesh: (1/2)(d(L) + d(R)), d = (phi(+t) - phi(-t)) / (2 Delta)
                const T s2 = (ph.get(k, bL + u) - ph.get(k, bL - d)) + (ph.get(k, bR + u) - ph.get(k, bR - d));
                v -= T(LAT::e(k, t)) * (hc * P.uct[t]) * s2;
            } else {
                const CellMetric<T>& mt = t == 0 ? mx : (t == 1 ? my : mz);
                const T dL = mt.cp * ph.get(k, bL + u) + mt.c0 * pL + mt.cm * ph.get(k, bL - d);
                const T dR = mt.cp * ph.get(k, bR + u) + mt.c0 * pR + mt.cm * ph.get(k, bR - d);
                v -= T(LAT::e(k, t)) * hc * (dL + w * (dR - dL));
            }
        }
        out[k] = v;
    }
    const T rL = ph.rest(bL), rR = ph.rest(bR);
    if constexpr (UNI) orest = T(0.5) * (rL + rR);
    else orest = rL + w * (rR - rL);
}

// interface moments (Eq. macro_values at the interface) from the two lanes' values
// LANE: u receives the velocity in the lane's frame, sg u (without
// acceleration: (sg c / rho0) j, bitwise sg (c j / rho0))
template <class LAT, typename T, bool NOG = false, bool ORIG = false, bool LANE = false>
__device__ __forceinline__ void moments_half(const Inst<T>& P, const T (&fb)[LAT::REST], T fr, const T* G, T sg,
                                             T& rho, T* u)
{
    constexpr int K = LAT::REST, D = LAT::D;
    T rh = T(0), sj[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        rh += fb[k];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (LAT::e(k, a) == 1) sj[a] += fb[k];
            if (LAT::e(k, a) == -1) sj[a] -= fb[k];
        }
    }
    T rs, js[3];
    moment_sums<D>(rh, sj, sg, rs, js);
    rho = rs + fr;
    const T cir = ORIG ? P.c / rho : T(0);  // original model, as in phi_half
    const T cu = LANE ? sg * (ORIG ? cir : P.crho) : (ORIG ? cir : P.crho);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const T j = js[a];
        if constexpr (NOG) {
            u[a] = cu * j;
        } else {
            const T ua = ORIG ? cir * j + (T(0.5) * P.h) * G[a] : vel_from<T, false>(P, rho, j, G[a], T(0.5) * P.h);
            u[a] = LANE ? sg * ua : ua;
        }
    }
#pragma unroll
    for (int a = D; a < 3; ++a) u[a] = T(0);
}

// what the NEQ rule needs from the opposite interface of a wall cell
template <class LAT, typename T>
struct NeqHalf {
    T rc, uc[3];
    T neq[LAT::REST];
};

template <class LAT, typename T, int A, bool NOG = false, bool ORIG = false>
__device__ __forceinline__ void neq_capture_half(const Inst<T>& P, const T (&fb)[LAT::REST], T fr, const T* G, T sg,
                                                 NeqHalf<LAT, T>& I)
{
    moments_half<LAT, T, NOG, ORIG>(P, fb, fr, G, sg, I.rc, I.uc);
    T us[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) us[a] = sg * I.uc[a];
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, I.rc, us, nullptr);
#pragma unroll
    for (int k = 0; k < LAT::REST; ++k) {
        if (LAT::e(k, A) == 0) continue;
        I.neq[k] = fb[k] - feq_pt<LAT, T, ORIG>(P, E, k);
    }
}

// the wall rules of Eqs. (BB), (NEQ) on a wall face of side s = 2A + (sgs > 0)
// for the lane's velocities entering the domain (sigma e_A sgs < 0)
template <class LAT, typename T, int A, bool ORIG = false>
__device__ __forceinline__ void wall_half(const Inst<T>& P, int s, int sgs, T (&wall)[LAT::REST],
                                          const NeqHalf<LAT, T>& I, T sg, int sgi, T gth)
{
    constexpr int K = LAT::REST, D = LAT::D;
    const int kind = P.bc[s];
    if (kind == BC_BOUNCE_BACK) {
        T other[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (LAT::e(k, A) != 0) other[k] = partner(wall[k]);  // opposite velocity, before the rule
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (LAT::e(k, A) == 0) continue;
            if (sgi * LAT::e(k, A) * sgs >= 0) continue;
            T xu = T(0);
#pragma unroll
            for (int d = 0; d < D; ++d) xu += xi_of<LAT, T>(k, d, P.c) * P.uw[s][d];
            wall[k] = other[k] + T(2) * P.rho0 * T(LAT::w(k)) * (sg * xu) * P.invRT;
        }
        return;
    }
    T ra, ua[3] = {T(0), T(0), T(0)};
    if (kind == BC_NEQ_VELOCITY) {
        ra = I.rc;
#pragma unroll
        for (int d = 0; d < D; ++d) ua[d] = sg * P.uw[s][d];
    } else {
        ra = wall_density(P, s, gth);
#pragma unroll
        for (int d = 0; d < D; ++d) ua[d] = sg * I.uc[d];
    }
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, ra, ua, nullptr);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (LAT::e(k, A) == 0) continue;
        if (sgi * LAT::e(k, A) * sgs >= 0) continue;
        wall[k] = feq_pt<LAT, T, ORIG>(P, E, k) + I.neq[k];
    }
}

// The force field of the three ring planes in LDS (D2Q9 launches with a
// field), laid out [plane slot][component][column]: at(d, A, off) is
// component d at offset off along axis A from the thread's column in the
// current plane.  g == nullptr: the field is read from global memory.
template <typename T, int BX, int BY>
struct RingForce {
    const T* g;
    int cur, dz_up, dz_dn;
    static constexpr int SQ = BX * BY;
    __device__ __forceinline__ T at(int d, int A, int off) const
    {
        return g[cur + d * SQ + (A == 0 ? off : (off > 0 ? dz_up : (off < 0 ? dz_dn : 0)))];
    }
};

// acceleration on the interface of axis A between the cells at offsets off
// and off+1 (weight w of the right one), from the LDS ring; the same
// expression as face_force
template <class LAT, typename T, class GV>
__device__ __forceinline__ void face_force_ring(const Inst<T>& P, const GV& gv, int A, int off, T w, T gth, T* G)
{
#pragma unroll
    for (int d = 0; d < LAT::D; ++d) {
        const T gl = gv.at(d, A, off), gr = gv.at(d, A, off + 1);
        G[d] = gth * (P.G0[d] + (gl + w * (gr - gl)));
    }
}

// The interface of axis A with index f between the cells at offsets off and
// off+1: reconstruction (Eq. gradient), wall rules, interface moments and the
// original distribution (the inverse of Eq. original_f) for the lane's
// velocities; out[half_cross_slot] receives f of the lane's velocities
// crossing the face.
// NW: the caller knows that the face is no wall face (the wall code is
// compiled out)
// RX (x faces of tiles whose rows are 16-lane segments): the NEQ rule's
// values at the opposite interface of a wall cell (interface moments and
// non-equilibrium part) are those of the face that the next lane of the row
// (low wall) or the previous one (high wall) evaluates in the same call; the
// wall face takes them from that lane (DPP row shift) instead of
// reconstructing the interface again.  rxw: the tile has the low (1) and / or
// high (2) wall face of the axis (uniform over the workgroup).
template <class LAT, typename T, class ACC, int A, bool UNI, bool NOG = false, bool ORIG = false, bool NW = false,
          bool RX = false, class GV>
__device__ __forceinline__ void face_half(const Inst<T>& P, const ACC& ph, const T* __restrict__ force, const GV& gv,
                                          const int* ci, int off, int f, T gth, const CellMetric<T>& mx,
                                          const CellMetric<T>& my, const CellMetric<T>& mz, T sg, int sgi, T* out,
                                          int rxw = 0)
{
    constexpr int K = LAT::REST;
    const AxisMetric<T>& m = P.m[A];
    const int n = P.n[A];
    const bool wall_lo = !NW && !P.per[A] && f == 0;
    const bool wall_hi = !NW && !P.per[A] && f == n;
    if constexpr (RX) {
        static_assert(A == 0 && !NW, "row exchange: x faces of the wall body");
        T fb[K], fr, G[3];
        const T w = UNI ? T(0.5) : m.w[f];
        recon_half<LAT, T, ACC, A, UNI>(P, ph, off, w, UNI ? P.ugn[A] : m.gn[f], mx, my, mz, sg, fb, fr);
        if constexpr (NOG) G[0] = G[1] = G[2] = T(0);
        else face_force<LAT, T>(P, force, A, f, w, ci, gth, G);
        T rho, u[3];
        moments_half<LAT, T, NOG, ORIG>(P, fb, fr, G, sg, rho, u);
        T us[3] = {T(0), T(0), T(0)}, Gs[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < LAT::D; ++a) {
            us[a] = sg * u[a];
            Gs[a] = sg * G[a];
        }
        EqPt<T> E = eq_point<LAT, T, ORIG>(P, rho, us, NOG ? nullptr : Gs);
        if (rxw) {
            // every lane of the call takes part in the shifts
            auto take = [&](T x) -> T {
                T r = x;
                if (rxw & 1) {
                    const T sx = row_shift<1>(x);
                    if (wall_lo) r = sx;
                }
                if (rxw & 2) {
                    const T sx = row_shift<-1>(x);
                    if (wall_hi) r = sx;
                }
                return r;
            };
            NeqHalf<LAT, T> info;
            info.rc = take(rho);
#pragma unroll
            for (int a = 0; a < 3; ++a) info.uc[a] = a < LAT::D ? take(u[a]) : T(0);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (LAT::e(k, A) != 0) info.neq[k] = take(fb[k] - feq_pt<LAT, T, ORIG>(P, E, k));
            if (wall_lo || wall_hi) {
                if (wall_lo) wall_half<LAT, T, A, ORIG>(P, 2 * A, -1, fb, info, sg, sgi, gth);
                if (wall_hi) wall_half<LAT, T, A, ORIG>(P, 2 * A + 1, 1, fb, info, sg, sgi, gth);
                moments_half<LAT, T, NOG, ORIG>(P, fb, fr, G, sg, rho, u);
#pragma unroll
                for (int a = 0; a < LAT::D; ++a) us[a] = sg * u[a];
                E = eq_point<LAT, T, ORIG>(P, rho, us, NOG ? nullptr : Gs);
            }
        }
        // feq again from the (wall lanes: updated) interface moments rather
        // than held across the exchange (fewer live registers)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (LAT::e(k, A) == 0) continue;
            const T fe = feq_pt<LAT, T, ORIG>(P, E, k);
            if constexpr (NOG) {
                out[half_cross_slot<LAT, A>(k)] = fb[k] + P.B7 * (fe - fb[k]);
            } else {
                const T S = srcf_pt<LAT, T>(P, E, k) * fe;
                out[half_cross_slot<LAT, A>(k)] = fb[k] + P.B7 * (fe - fb[k]) + P.C7 * S;
            }
        }
        return;
    }
    NeqHalf<LAT, T> info;
    asm volatile("" ::: "memory");
    T fb[K], fr, G[3];
    if (wall_lo || wall_hi) {
        const int fo = wall_lo ? 1 : n - 1;
        const int oo = wall_lo ? off + 1 : off - 1;
        const T wo = UNI ? T(0.5) : m.w[fo];
        recon_half<LAT, T, ACC, A, UNI>(P, ph, oo, wo, UNI ? P.ugn[A] : m.gn[fo], mx, my, mz, sg, fb, fr);
        if constexpr (!NOG) {
            if (LAT::D == 2 && gv.g) face_force_ring<LAT, T>(P, gv, A, oo, wo, gth, G);
            else face_force<LAT, T>(P, force, A, fo, wo, ci, gth, G);
        }
        neq_capture_half<LAT, T, A, NOG, ORIG>(P, fb, fr, G, sg, info);
        asm volatile("" ::: "memory");
    }
    const T w = UNI ? T(0.5) : m.w[f];
    recon_half<LAT, T, ACC, A, UNI>(P, ph, off, w, UNI ? P.ugn[A] : m.gn[f], mx, my, mz, sg, fb, fr);
    if constexpr (NOG) G[0] = G[1] = G[2] = T(0);
    else if (LAT::D == 2 && gv.g) face_force_ring<LAT, T>(P, gv, A, off, w, gth, G);
    else face_force<LAT, T>(P, force, A, f, w, ci, gth, G);
    if (wall_lo) wall_half<LAT, T, A, ORIG>(P, 2 * A, -1, fb, info, sg, sgi, gth);
    if (wall_hi) wall_half<LAT, T, A, ORIG>(P, 2 * A + 1, 1, fb, info, sg, sgi, gth);
    T rho, us[3];
    moments_half<LAT, T, NOG, ORIG, true>(P, fb, fr, G, sg, rho, us);
    T Gs[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < LAT::D; ++a) Gs[a] = sg * G[a];
    const EqPt<T> E = eq_point<LAT, T, ORIG>(P, rho, us, NOG ? nullptr : Gs);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (LAT::e(k, A) == 0) continue;
        const T fe = feq_pt<LAT, T, ORIG>(P, E, k);
        if constexpr (NOG) {
            out[half_cross_slot<LAT, A>(k)] = fb[k] + P.B7 * (fe - fb[k]);  // inverse of Eq. (original_f) without a source
        } else {
            const T S = srcf_pt<LAT, T>(P, E, k) * fe;
            out[half_cross_slot<LAT, A>(k)] = fb[k] + P.B7 * (fe - fb[k]) + P.C7 * S;  // inverse of Eq. (original_f)
        }
    }
}

// Threads of a tile: 2 x NCOL, NCOL = BX*BY rounded up to whole half-waves.
template <int BX, int BY>
__host__ __device__ constexpr int split_threads()
{
    return 2 * ((BX * BY + 31) / 32) * 32;
}

// One workgroup's work: tile `tile` (of tiles0 x tiles1) and march chunk
// `ck` of instance P; fin/fout/force point at the instance's arrays.
// The cell's own f-tilde of Eq. (f_tilde_+) is kept in registers from the
// plane load (OWN) instead of being read a second time, where the registers
// allow it: D2Q9, and D3Q19 on uniform meshes without a force field.
template <class LAT, typename T, bool UNI, bool FF>
constexpr bool own_regs()
{
    return LAT::Q == 9 || (LAT::Q == 19 && UNI && !FF);
}

// NW: the workgroup's tile and chunk touch no wall (no wall faces, ghost
// columns or ghost planes); that code is then compiled out of the body that
// most workgroups of a large mesh run.  Used for D3Q19 launches of instances
// without acceleration (elsewhere the second body costs spilled registers,
// FP32 with acceleration, or gains nothing measurable: D3Q27)
template <class LAT, typename T, int BX, int BY, bool PF, bool UNI, bool OWN, bool NOG = false, bool ORIG = false,
          bool LPF = false, bool NW = false>
__device__ __forceinline__ void split_body(const Inst<T>& P, const T* __restrict__ fin, const T* __restrict__ force,
                                           T* __restrict__ fout, T gt, T gth, int chunk, int tiles0, int tile,
                                           int ck, T* lds)
{
    constexpr int Q = LAT::Q, D = LAT::D, M = D - 1, K = LAT::REST;
    constexpr int NX = half_cross_count<LAT, 0>(), NY = half_cross_count<LAT, 1>();
    constexpr int NM = half_cross_count<LAT, M>();
    constexpr int SQ = BX * BY;
    // PHIU (single-instance launches without acceleration: FP32 D3Q19, and
    // D3Q27): the update needs no own state, since rho and j of f-bar-plus
    // equal those of f-tilde without acceleration: feq follows from the ring
    // and f-tilde(n+1) = phi + B1 / (3 (1 - B1)) (feq - phi) - fluxes.  FP32
    // D3Q19 (4 waves per SIMD, 128 registers) spends the freed own-state
    // registers on the late prefetch; D3Q27, which keeps no own state in
    // registers, saves the second read of it (and takes the late prefetch
    // in both precisions).  The host launches these instances only
    // where |1 - B1| >= 1/4 (Inst::bu_ok); elsewhere it takes the instance
    // with the acceleration terms, whose skipped terms are exact zeros.
    constexpr bool PHIU = NOG && !ORIG && LPF && ((LAT::Q == 19 && sizeof(T) == 4) || LAT::Q == 27);
    constexpr bool OWNR = OWN && !PHIU;
    const T Bu = P.Bu;
    T* fxb = lds + 3 * Q * SQ;   // [2][NX][BY][BX] upper x faces, per half
    T* fyb = fxb + 2 * NX * SQ;  // [2][NY][BY][BX] upper y faces (3-D)
    // D2Q9: the force field of the ring planes, [3][D][BY][BX], after the
    // x faces (no y-face buffer in 2-D)
    T* gring = fxb + 2 * NX * SQ;
    const int tid = threadIdx.x;
    const int h = (tid >> 5) & 1;
    const int col = (tid >> 6) * 32 + (tid & 31);
    const bool in_tile = col < SQ;
    const int tx = in_tile ? col % BX : 0, ty = in_tile ? col / BX : 0;
    const T sg = h ? T(-1) : T(1);
    const int sgi = h ? -1 : 1;
    const int hs = h ? K + 1 : 0;  // first LDS slot of this lane
    const int b0 = tile % tiles0, b1 = tile / tiles0;

    int g[2], kind[2], src[2];
    g[0] = b0 * (BX - 2) - 1 + tx;
    g[1] = (D == 3) ? b1 * (BY - 2) - 1 + ty : 0;
#pragma unroll
    for (int a = 0; a < D - 1; ++a) {
        const int N = P.n[a], x = g[a];
        if (!in_tile) { kind[a] = COL_OUT; src[a] = 0; }
        else if (x >= 0 && x < N) { kind[a] = COL_CELL; src[a] = x; }
        else if (P.per[a] && x == -1) { kind[a] = COL_CELL; src[a] = N - 1; }
        else if (P.per[a] && x == N) { kind[a] = COL_CELL; src[a] = 0; }
        else if (!P.per[a] && x == -1) { kind[a] = COL_GHOST_LO; src[a] = 0; }
        else if (!P.per[a] && x == N) { kind[a] = COL_GHOST_HI; src[a] = N - 1; }
        else { kind[a] = COL_OUT; src[a] = 0; }
    }
    if (D == 2) { kind[1] = in_tile ? COL_CELL : COL_OUT; src[1] = 0; }
    const bool cell_col = kind[0] == COL_CELL && kind[1] == COL_CELL;
    const bool ghost_col = !cell_col && kind[0] != COL_OUT && kind[1] != COL_OUT;
    const bool row_ok = in_tile && ((D == 2) || (g[1] >= 0 && g[1] < P.n[1] && ty >= 1 && ty <= BY - 2));
    const bool col_ok = in_tile && g[0] >= 0 && g[0] < P.n[0] && tx >= 1 && tx <= BX - 2;
    const bool upd_col = cell_col && col_ok && row_ok;
    const bool xface = (cell_col || ghost_col) && row_ok && tx <= BX - 2 && g[0] >= -1 && g[0] <= P.n[0] - 1;
    const bool yface = (D == 3) && (cell_col || ghost_col) && col_ok && ty <= BY - 2 && g[1] >= -1 &&
                       g[1] <= P.n[1] - 1;

    const bool any_ghost = NW ? false : __syncthreads_or(ghost_col) != 0;
    // XSH (3-D tiles 16 columns wide, whose rows are the 16-lane segments of
    // a wave): in a tile whose only ghost columns are those of the x walls,
    // a ghost column extrapolates f-bar-plus from the two cells beside it in
    // its row, taken from their lanes by a shuffle (wave-local, before the
    // plane's barrier) instead of from LDS after a second barrier
    constexpr bool XSH = !NW && D == 3 && BX == 16;
    const bool xsh_tile = XSH && any_ghost && __syncthreads_or(ghost_col && kind[1] != COL_CELL) == 0;
    const bool xg_lo = xsh_tile && !P.per[0] && b0 == 0;
    const bool xg_hi = xsh_tile && !P.per[0] && b0 * (BX - 2) - 1 + (BX - 1) >= P.n[0];
    // the tile's x wall faces, for the row exchange of the x-face stage
    // (D3Q27, whose one wave per SIMD has registers to spare; in D3Q19 FP64,
    // at 256 registers, the second pass spills about what the exchange saves)
    constexpr bool RX = XSH && LAT::Q == 27;
    const int rxw = RX ? ((!P.per[0] && b0 == 0) ? 1 : 0) |
                              ((!P.per[0] && b0 * (BX - 2) - 1 + (BX - 1) >= P.n[0]) ? 2 : 0)
                        : 0;
    const bool gr_on = (D == 2) && force != nullptr;
    auto gslot = [&](int p, int d) { return (ring(p) * D + d) * SQ + ty * BX + tx; };
    const int nM = P.n[M];
    const int p0 = ck * chunk;
    const int p1 = min(p0 + chunk, nM);
    const bool perM = P.per[M] != 0;
    const CellMetric<T> cmx = upd_col_pre(P, 0, g[0]);
    const CellMetric<T> cmy = D == 3 ? upd_col_pre(P, 1, g[1]) : cmx;
    // global element offsets of the lane's velocities: q = k (half 0) or
    // Q-1-k (half 1)
    const long long q0off = h ? (long long)(Q - 1) * P.nc : 0;
    const long long qstep = h ? -P.nc : P.nc;
    const long long roff = (long long)LAT::REST * P.nc;

    // element of (plane p, slot s, this column + (dx, dy))
    auto lds_el = [&](int p, int s, int dx, int dy) -> int { return ((ring(p) * Q + s) * BY + ty + dy) * BX + tx + dx; };

    static_assert(!(PF && OWNR), "the own-state registers assume no plane prefetch");
    T pf[K], prest = T(0), pg[3] = {T(0), T(0), T(0)};
    // OWN: f-tilde of plane hi - 1 (the plane before the last one loaded)
    T fo[K], fore = T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) pf[k] = fo[k] = T(0);
    auto shift_own = [&]() {
        if constexpr (OWNR) {
#pragma unroll
            for (int k = 0; k < K; ++k) fo[k] = pf[k];
            fore = prest;
        }
    };
    auto plane_cell = [&](int p) -> long long {
        const int pp = perM ? ((p % nM) + nM) % nM : p;
        return int_idx(P, src[0], (D == 3) ? src[1] : pp, (D == 3) ? pp : 0);
    };
    auto load_plane = [&](int p) {
        shift_own();
        if (cell_col) {
            const long long ci = plane_cell(p);
            const T* fp = fin + ci + q0off;
#pragma unroll
            for (int k = 0; k < K; ++k) pf[k] = fp[k * qstep];
            prest = fin[ci + roff];
            if (force) {
#pragma unroll
                for (int a = 0; a < D; ++a) pg[a] = force[(long long)a * P.nc + ci];
            }
        }
    };
    // Late prefetch (FP64 with the own state in registers, single-instance
    // launches without a force field): the state of plane z+2 is loaded after
    // the interface stage of plane z, so that its latency overlaps the barrier
    // wait and the update instead of stalling the next f-bar-plus stage (2 %
    // at 128^3; the batched and force-field instances, and FP32 with the
    // own-state ring, run out of registers with it: D2Q9 512^2 with a field
    // 30 -> 39 us).  PHIU launches take it too: FP32 D3Q19 in the registers
    // the own state frees, D3Q27 in both precisions (FP64 D3Q27 runs one
    // wave per SIMD, whose register file has room for it: 3 % at 128^3).
    constexpr bool LP = LPF && ((OWNR && sizeof(T) == 8) || PHIU);
    T pn[K], pnr = T(0), pgn[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < K; ++k) pn[k] = T(0);
    int pn_plane = -0x7fffffff;  // plane held in pn
    auto prefetch = [&](int p) {
        if (cell_col) {
            const long long ci = plane_cell(p);
            const T* fp = fin + ci + q0off;
#pragma unroll
            for (int k = 0; k < K; ++k) pn[k] = fp[k * qstep];
            pnr = fin[ci + roff];
            if (force) {
#pragma unroll
                for (int a = 0; a < D; ++a) pgn[a] = force[(long long)a * P.nc + ci];
            }
        }
        pn_plane = p;
    };
    // load_plane's effect with the prefetched values
    auto take_plane = [&]() {
        shift_own();
#pragma unroll
        for (int k = 0; k < K; ++k) pf[k] = pn[k];
        prest = pnr;
#pragma unroll
        for (int a = 0; a < 3; ++a) pg[a] = pgn[a];
    };
    auto compute_plane = [&](int p) {
        T v[K], vr;
        if (cell_col) {
            phi_half<LAT, T, NOG, ORIG>(P, pf, prest, pg, force != nullptr, gt, sg, v, vr);
#pragma unroll
            for (int k = 0; k < K; ++k) lds[lds_el(p, hs + k, 0, 0)] = v[k];
            if (h == 0) lds[lds_el(p, K, 0, 0)] = vr;
            if (gr_on && h == 0) {
#pragma unroll
                for (int d = 0; d < D; ++d) gring[gslot(p, d)] = pg[d];
            }
        }
        if constexpr (XSH) {
            // the ghost rule (linear extrapolation through the two nearest
            // centres) with the centres' values from lanes +1, +2 (low wall) or
            // -1, -2 (high wall) of the row; every lane of the wave takes part
            auto ghost_x = [&](bool lo, int kindg, T r) {
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    const T x = k < K ? v[k] : vr;
                    const T s1 = lo ? row_shift<1>(x) : row_shift<-1>(x);
                    const T s2 = lo ? row_shift<2>(x) : row_shift<-2>(x);
                    T acc = (T(1) - r) * s1;
                    acc += r * s2;
                    if (ghost_col && kind[0] == kindg) {
                        if (k < K) lds[lds_el(p, hs + k, 0, 0)] = acc;
                        else if (h == 0) lds[lds_el(p, K, 0, 0)] = acc;
                    }
                }
            };
            if (xg_lo) ghost_x(true, COL_GHOST_LO, P.rlo[0]);
            if (xg_hi) ghost_x(false, COL_GHOST_HI, P.rhi[0]);
        }
        __syncthreads();
        if (!any_ghost || xsh_tile) return;
        if (ghost_col) {
            int off[2][2];
            T wt[2][2];
            int cnt[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                cnt[a] = 1;
                off[a][0] = 0; wt[a][0] = T(1);
                off[a][1] = 0; wt[a][1] = T(0);
                if (a < D - 1 && kind[a] == COL_GHOST_LO) {
                    cnt[a] = 2;
                    off[a][0] = 1; wt[a][0] = T(1) - P.rlo[a];
                    off[a][1] = 2; wt[a][1] = P.rlo[a];
                } else if (a < D - 1 && kind[a] == COL_GHOST_HI) {
                    cnt[a] = 2;
                    off[a][0] = -1; wt[a][0] = T(1) - P.rhi[a];
                    off[a][1] = -2; wt[a][1] = P.rhi[a];
                }
            }
            T acc[K + 1];
#pragma unroll
            for (int k = 0; k <= K; ++k) acc[k] = T(0);
            for (int i1 = 0; i1 < cnt[1]; ++i1)
                for (int i0 = 0; i0 < cnt[0]; ++i0) {
                    const T w = wt[0][i0] * wt[1][i1];
#pragma unroll
                    for (int k = 0; k < K; ++k) acc[k] += w * lds[lds_el(p, hs + k, off[0][i0], off[1][i1])];
                    acc[K] += w * lds[lds_el(p, K, off[0][i0], off[1][i1])];
                }
#pragma unroll
            for (int k = 0; k < K; ++k) lds[lds_el(p, hs + k, 0, 0)] = acc[k];
            if (h == 0) lds[lds_el(p, K, 0, 0)] = acc[K];
            if (gr_on && h == 0) {
                // the force field's ghost rule is that of f-bar-plus
                T ga[3] = {T(0), T(0), T(0)};
                for (int i1 = 0; i1 < cnt[1]; ++i1)
                    for (int i0 = 0; i0 < cnt[0]; ++i0) {
                        const T w = wt[0][i0] * wt[1][i1];
#pragma unroll
                        for (int d = 0; d < D; ++d) ga[d] += w * gring[gslot(p, d) + off[1][i1] * BX + off[0][i0]];
                    }
#pragma unroll
                for (int d = 0; d < D; ++d) gring[gslot(p, d)] = ga[d];
            }
        }
        __syncthreads();
    };
    // ghost plane p of a wall march axis: extrapolation through planes a, b
    auto ghost_plane = [&](int p, int a, int b, T r) {
        if (cell_col || ghost_col) {
#pragma unroll
            for (int k = 0; k < K; ++k)
                lds[lds_el(p, hs + k, 0, 0)] =
                    (T(1) - r) * lds[lds_el(a, hs + k, 0, 0)] + r * lds[lds_el(b, hs + k, 0, 0)];
            if (h == 0)
                lds[lds_el(p, K, 0, 0)] = (T(1) - r) * lds[lds_el(a, K, 0, 0)] + r * lds[lds_el(b, K, 0, 0)];
            if (gr_on && h == 0) {
#pragma unroll
                for (int d = 0; d < D; ++d)
                    gring[gslot(p, d)] = (T(1) - r) * gring[gslot(a, d)] + r * gring[gslot(b, d)];
            }
        }
        __syncthreads();
    };
    auto phi_view = [&](int z) {
        const int slot = Q * SQ;
        return HalfPhi<LAT, T, BX, BY>{lds, ring(z) * slot + ty * BX + tx, hs * SQ, (ring(z + 1) - ring(z)) * slot,
                                       (ring(z - 1) - ring(z)) * slot};
    };
    auto gview = [&](int z) {
        return RingForce<T, BX, BY>{gr_on ? gring : nullptr, ring(z) * D * SQ + ty * BX + tx,
                                    (ring(z + 1) - ring(z)) * D * SQ, (ring(z - 1) - ring(z)) * D * SQ};
    };
    auto computed = [&](int p) { return NW || perM || p < nM; };

    int hi;
    if (!NW && !perM && p0 == 0) {
        load_plane(0);
        compute_plane(0);
        load_plane(1);
        compute_plane(1);
        ghost_plane(-1, 0, 1, P.rlo[M]);
        hi = 1;
    } else {
        load_plane(p0 - 1);
        compute_plane(p0 - 1);
        load_plane(p0);
        compute_plane(p0);
        hi = p0;
    }
    if (PF && hi + 1 <= p1 && computed(hi + 1)) load_plane(hi + 1);
    if (LP && hi + 1 <= p1 && computed(hi + 1)) prefetch(hi + 1);
    // lower march-axis face of the first plane
    T zlo[NM > 0 ? NM : 1];
    if (upd_col) {
        int ci[3];
        ci[0] = g[0];
        ci[1] = (D == 3) ? g[1] : p0;
        ci[2] = (D == 3) ? p0 : 0;
        const CellMetric<T> cmm = load_metric(P, M, p0);
        const auto ph = phi_view(p0);
        if constexpr (D == 3) face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, M, UNI, NOG, ORIG, NW>(P, ph, force, gview(p0), ci, -1, p0, gth, cmx, cmy, cmm, sg, sgi, zlo);
        else face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, M, UNI, NOG, ORIG, NW>(P, ph, force, gview(p0), ci, -1, p0, gth, cmx, cmm, cmm, sg, sgi, zlo);
    }
    for (int z = p0; z < p1; ++z) {
        if (hi < z + 1) {
            // No barrier needed here: the ring slot of z+1 (= z-2) was last
            // read by the faces of plane z-1, which every wave finished before
            // the barrier that precedes the update of z-1; the face buffers
            // are rewritten only after the barrier that ends this plane's
            // computation, by which time every wave has left that update.
            if (!computed(z + 1)) {
                shift_own();
                ghost_plane(z + 1, z, z - 1, P.rhi[M]);
            } else {
                if (LP && pn_plane == z + 1) take_plane();
                else if (!PF) load_plane(z + 1);
                compute_plane(z + 1);
            }
            hi = z + 1;
            if (PF && z + 2 <= p1 && computed(z + 2)) load_plane(z + 2);
        } else {
            __syncthreads();
        }
        int ci[3];
        ci[0] = g[0];
        ci[1] = (D == 3) ? g[1] : z;
        ci[2] = (D == 3) ? z : 0;
        const CellMetric<T> cmm = load_metric(P, M, z);
        const auto ph = phi_view(z);
        // the cell's own state for Eq. (f_tilde_+)
        T fz[K], fzr = T(0);
        auto load_own = [&]() {
            if constexpr (OWNR) {  // plane z = hi - 1
#pragma unroll
                for (int k = 0; k < K; ++k) fz[k] = fo[k];
                fzr = fore;
                return;
            }
            const long long cidx = int_idx(P, ci[0], ci[1], ci[2]);
            const T* fp = fin + cidx + q0off;
#pragma unroll
            for (int k = 0; k < K; ++k) fz[k] = fp[k * qstep];
            fzr = fin[cidx + roff];
        };
        if (PF && upd_col) load_own();
        T zhi[NM > 0 ? NM : 1];
        if (xface) {
            T v[NX];
            if constexpr (D == 3) face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, 0, UNI, NOG, ORIG, NW, RX>(P, ph, force, gview(z), ci, 0, g[0] + 1, gth, cmx, cmy, cmm, sg, sgi, v, rxw);
            else face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, 0, UNI, NOG, ORIG, NW>(P, ph, force, gview(z), ci, 0, g[0] + 1, gth, cmx, cmm, cmm, sg, sgi, v);
#pragma unroll
            for (int kc = 0; kc < NX; ++kc) fxb[((h * NX + kc) * BY + ty) * BX + tx] = v[kc];
        }
        if constexpr (D == 3) {
            if (yface) {
                T v[NY];
                face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, 1, UNI, NOG, ORIG, NW>(P, ph, force, gview(z), ci, 0, g[1] + 1, gth, cmx, cmy, cmm, sg, sgi, v);
#pragma unroll
                for (int kc = 0; kc < NY; ++kc) fyb[((h * NY + kc) * BY + ty) * BX + tx] = v[kc];
            }
        }
        if (upd_col) {
            if constexpr (D == 3) face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, M, UNI, NOG, ORIG, NW>(P, ph, force, gview(z), ci, 0, z + 1, gth, cmx, cmy, cmm, sg, sgi, zhi);
            else face_half<LAT, T, HalfPhi<LAT, T, BX, BY>, M, UNI, NOG, ORIG, NW>(P, ph, force, gview(z), ci, 0, z + 1, gth, cmx, cmm, cmm, sg, sgi, zhi);
        }
        if (LP && z + 2 <= p1 && computed(z + 2) && pn_plane != z + 2) prefetch(z + 2);
        __syncthreads();
        if (upd_col) {
            const long long cidx = int_idx(P, ci[0], ci[1], ci[2]);
            T acc[K], accr;
            if constexpr (PHIU) {
                T pv[K];
                T rh = T(0), sj[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    pv[k] = ph.get(k, ph.cur);
                    rh += pv[k];
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        if (LAT::e(k, a) == 1) sj[a] += pv[k];
                        if (LAT::e(k, a) == -1) sj[a] -= pv[k];
                    }
                }
                const T pr = ph.rest(ph.cur);
                T rs, js[3];
                moment_sums<D>(rh, sj, sg, rs, js);
                const T rho = rs + pr;
                T us[3] = {T(0), T(0), T(0)};
#pragma unroll
                for (int a = 0; a < D; ++a) us[a] = sg * (P.crho * js[a]);
                const EqPt<T> E = eq_point<LAT, T, false>(P, rho, us, nullptr);
#pragma unroll
                for (int k = 0; k < K; ++k) acc[k] = pv[k] + Bu * (feq_pt<LAT, T, false>(P, E, k) - pv[k]);
                accr = pr + Bu * (feq_pt<LAT, T, false>(P, E, LAT::REST) - pr);
            } else {
            if (!PF) load_own();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T p = ph.get(k, ph.cur);
                acc[k] = p + (p - fz[k]) * T(1.0 / 3.0);  // Eq. (f_tilde_+)
            }
            const T pr = ph.rest(ph.cur);
            accr = pr + (pr - fzr) * T(1.0 / 3.0);
            }
            const T sx = sg * ((UNI ? P.ufdx[0] : cmx.fdx) * P.c), sm = sg * ((UNI ? P.ufdx[M] : cmm.fdx) * P.c);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (LAT::e(k, 0) != 0) {
                    const int kc = half_cross_slot<LAT, 0>(k);
                    const T d = fxb[((h * NX + kc) * BY + ty) * BX + tx] - fxb[((h * NX + kc) * BY + ty) * BX + tx - 1];
                    acc[k] -= T(LAT::e(k, 0)) * sx * d;
                }
                if constexpr (D == 3) {
                    if (LAT::e(k, 1) != 0) {
                        const int kc = half_cross_slot<LAT, 1>(k);
                        const T d = fyb[((h * NY + kc) * BY + ty) * BX + tx] - fyb[((h * NY + kc) * BY + ty - 1) * BX + tx];
                        acc[k] -= T(LAT::e(k, 1)) * (sg * ((UNI ? P.ufdx[1] : cmy.fdx) * P.c)) * d;
                    }
                }
                if (LAT::e(k, M) != 0) {
                    const int kc = half_cross_slot<LAT, M>(k);
                    acc[k] -= T(LAT::e(k, M)) * sm * (zhi[kc] - zlo[kc]);
                }
            }
            T* fp = fout + cidx + q0off;
#pragma unroll
            for (int k = 0; k < K; ++k) fp[k * qstep] = acc[k];
            if (h == 0) fout[cidx + roff] = accr;
#pragma unroll
            for (int kc = 0; kc < NM; ++kc) zlo[kc] = zhi[kc];
        }
    }
}

// Does the workgroup of tile `tile` and march chunk `ck` (3-D) stay clear of
// every wall?  Along a wall-bounded tile axis its columns (halo included) must
// all be cells, and along a wall-bounded march axis its planes p0 - 1 ..
// p1 must all be cells (no wall face, no ghost column or plane).
template <typename T>
__device__ __forceinline__ bool split_no_wall(const Inst<T>& P, int BX, int BY, int tiles0, int tile, int ck, int chunk)
{
    const int b0 = tile % tiles0, b1 = tile / tiles0;
    const int x0 = b0 * (BX - 2) - 1, y0 = b1 * (BY - 2) - 1;
    if (!P.per[0] && (x0 < 0 || x0 + BX - 1 > P.n[0] - 1)) return false;
    if (!P.per[1] && (y0 < 0 || y0 + BY - 1 > P.n[1] - 1)) return false;
    const int p0 = ck * chunk, p1 = min(p0 + chunk, P.n[2]);
    if (!P.per[2] && (p0 < 1 || p1 > P.n[2] - 1)) return false;
    return true;
}

// FF: the launch carries a force field (without one the kernel is compiled
// with a null field and no field code)
template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF, bool UNI, bool NOG, bool ORIG = false>
__global__ DUGKS_KERNEL_BOUNDS((split_threads<BX, BY>()), MINW, (max_waves_per_eu<LAT, T, true>())) void k_split(const Inst<T>* __restrict__ Pp,
                                                                          const T* __restrict__ fin,
                                                                          const T* __restrict__ force,
                                                                          T* __restrict__ fout, double t, int chunk,
                                                                          int tiles0, int tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Inst<T>& P = *Pp;
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * P.dtd);
    const int b = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int tile = b % tiles, ck = b / tiles;
    constexpr bool OWN = own_regs<LAT, T, UNI, FF>();
    if constexpr (LAT::Q == 19 && NOG) {
        if (split_no_wall(P, BX, BY, tiles0, tile, ck, chunk)) {
            split_body<LAT, T, BX, BY, PF, UNI, OWN, NOG, ORIG, !FF, true>(
                P, fin, FF ? force : nullptr, fout, gt, gth, chunk, tiles0, tile, ck, reinterpret_cast<T*>(smem_raw));
            return;
        }
    }
    split_body<LAT, T, BX, BY, PF, UNI, OWN, NOG, ORIG, !FF>(P, fin, FF ? force : nullptr, fout, gt, gth, chunk, tiles0,
                                                             tile, ck, reinterpret_cast<T*>(smem_raw));
}

// batched form (see k_fused2_batch): workgroup b in XCD order belongs to the
// instance i with bstart[i] <= b < bstart[i+1]
template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF>
__global__ DUGKS_KERNEL_BOUNDS((split_threads<BX, BY>()), MINW, (max_waves_per_eu<LAT, T, true>())) void k_split_batch(
    const Inst<T>* __restrict__ insts, const long long* __restrict__ bstart, const BatchGeom* __restrict__ geom,
    int ninst, const T* __restrict__ fin, const T* __restrict__ forces, T* __restrict__ fout,
    const long long* __restrict__ step0, int step)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const long long b = xcd_order((int)blockIdx.x, (int)gridDim.x);
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bstart[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const Inst<T>& P = insts[lo];
    const BatchGeom g = geom[lo];
    const int local = (int)(b - bstart[lo]);
    const int ntile = g.tiles0 * g.tiles1;
    const double t = (double)(*step0 + step) * P.dtd;
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * P.dtd);
    const T* force = (FF && forces && P.foff >= 0) ? forces + P.foff : nullptr;
    // per instance: the uniform-mesh body where every axis is uniform
    if (P.uni)
        split_body<LAT, T, BX, BY, PF, true, own_regs<LAT, T, true, FF>()>(
            P, fin + P.off, force, fout + P.off, gt, gth, g.chunk, g.tiles0, local % ntile, local / ntile,
            reinterpret_cast<T*>(smem_raw));
    else
        split_body<LAT, T, BX, BY, PF, false, own_regs<LAT, T, false, FF>()>(
            P, fin + P.off, force, fout + P.off, gt, gth, g.chunk, g.tiles0, local % ntile, local / ntile,
            reinterpret_cast<T*>(smem_raw));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class LAT, typename T, int BX, int BY>
static size_t split_lds()
{
    return (size_t)(3 * LAT::Q + 2 * half_cross_count<LAT, 0>() + (LAT::D == 3 ? 2 * half_cross_count<LAT, 1>() : 0) +
                    (LAT::D == 2 ? 3 * LAT::D : 0)) *
           BX * BY * sizeof(T);
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF, bool UNI, bool NOG = false, bool ORIG = false>
static int launch_split_ff(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force, double t,
                           hipStream_t st, int chunk)
{
    constexpr int D = LAT::D, M = D - 1;
    const int tiles0 = (P.n[0] + BX - 3) / (BX - 2);
    const int tiles1 = (D == 3) ? (P.n[1] + BY - 3) / (BY - 2) : 1;
    const size_t lds = split_lds<LAT, T, BX, BY>();
    auto kern = k_split<LAT, T, BX, BY, MINW, PF, FF, UNI, NOG, ORIG>;
    static bool attr_set = false;
    static long long slots = 0;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_check(ctx, e, "split kernel LDS attribute");
        slots = resident_slots(kern, split_threads<BX, BY>(), lds, ctx->n_cu);
        attr_set = true;
    }
    chunk = launch_chunk(chunk, (long long)tiles0 * tiles1, P.n[M], slots);
    const int chunks = (P.n[M] + chunk - 1) / chunk;
    const long long nb = (long long)tiles0 * tiles1 * chunks;
    if (nb > 0x7fffffffLL) return fail(ctx, DUGKS_EUNSUPPORTED, "mesh too large for one launch");
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(split_threads<BX, BY>()), lds, st,
                       (const Inst<T>*)ctx->inst_dev, (const T*)fin, (const T*)force, (T*)fout, t, chunk, tiles0,
                       tiles0 * tiles1);
    return hip_check(ctx, hipGetLastError(), "split step launch");
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF>
static int launch_split(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force, double t,
                        hipStream_t st, int chunk)
{
    // FP32 D3Q19, uniform and field-free: fits four waves per SIMD (two
    // tiles per CU) without spills
    constexpr int MINW_UF = (LAT::Q == 19 && sizeof(T) == 4) ? 4 : MINW;
    // no acceleration at all (G = 0, no field): instances without the
    // source term of Eq. (S) (bitwise the same results, fewer operations).
    // Those of FP32 D3Q19 and of D3Q27 update without the own state, whose
    // coefficient B1 / (3 (1 - B1)) is allowed only away from its pole at
    // B1 = 1; near it the instance with the acceleration terms runs instead
    constexpr bool phiu_lat = (LAT::Q == 19 && sizeof(T) == 4) || LAT::Q == 27;
    const bool nog = !force && P.G0[0] == T(0) && P.G0[1] == T(0) && P.G0[2] == T(0) &&
                     (P.orig || !phiu_lat || P.bu_ok);
    if (P.orig) {
        // the original-model equilibrium (launches without a force field;
        // without acceleration the source-free instances, bitwise the same)
        if (P.uni) {
            if (nog) return launch_split_ff<LAT, T, BX, BY, MINW_UF, PF, false, true, true, true>(ctx, P, fin, fout, force, t, st, chunk);
            return launch_split_ff<LAT, T, BX, BY, MINW_UF, PF, false, true, false, true>(ctx, P, fin, fout, force, t, st, chunk);
        }
        if (nog) return launch_split_ff<LAT, T, BX, BY, MINW, PF, false, false, true, true>(ctx, P, fin, fout, force, t, st, chunk);
        return launch_split_ff<LAT, T, BX, BY, MINW, PF, false, false, false, true>(ctx, P, fin, fout, force, t, st, chunk);
    }
    if (P.uni) {
        if (force) return launch_split_ff<LAT, T, BX, BY, MINW, PF, true, true>(ctx, P, fin, fout, force, t, st, chunk);
        if (nog) return launch_split_ff<LAT, T, BX, BY, MINW_UF, PF, false, true, true>(ctx, P, fin, fout, force, t, st, chunk);
        return launch_split_ff<LAT, T, BX, BY, MINW_UF, PF, false, true>(ctx, P, fin, fout, force, t, st, chunk);
    }
    if (force) return launch_split_ff<LAT, T, BX, BY, MINW, PF, true, false>(ctx, P, fin, fout, force, t, st, chunk);
    if (nog) return launch_split_ff<LAT, T, BX, BY, MINW, PF, false, false, true>(ctx, P, fin, fout, force, t, st, chunk);
    return launch_split_ff<LAT, T, BX, BY, MINW, PF, false, false>(ctx, P, fin, fout, force, t, st, chunk);
}

int split_step(dugks_ctx* ctx, const void* fin, void* fout, const void* force, double t, hipStream_t st, int chunk)
{
    if (ctx->cfg.lattice == DUGKS_D3Q27) {
        // 27 velocities, 16 x 8 column tiles.  FP64: the tile's LDS ring
        // (120 KB) fills a CU, four waves (one per SIMD) whose state fits the
        // register file without scratch; an 18 x 9 tile (six waves) would
        // spill to scratch.  FP32: 60 KB, so two workgroups (eight waves)
        // share a CU, where an 18 x 9 tile (76 KB, six waves at over 170
        // registers) leaves one.
        if (ctx->cfg.dtype == DUGKS_F64)
            return launch_split<D3Q27, double, 16, 8, 1, false>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
        return launch_split<D3Q27, float, 16, 8, 2, false>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
    }
    if (ctx->cfg.lattice == DUGKS_D3Q19) {
        // FP64: a 16 x 8 column tile (78 KB of LDS) lets two workgroups share
        // a CU, so one waits at its barriers while the other computes; that
        // outweighs the larger halo share of the smaller tile (0.499 vs
        // 0.515 ms at 128^3 with 18 x 14)
        if (ctx->cfg.dtype == DUGKS_F64)
            return launch_split<D3Q19, double, 16, 8, 2, false>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
        return launch_split<D3Q19, float, 18, 14, 2, false>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
    }
    if (ctx->cfg.dtype == DUGKS_F64)
        return launch_split<D2Q9, double, 128, 1, 2, false>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
    return launch_split<D2Q9, float, 128, 1, 2, false>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF>
static hipError_t split_batch_launch_ff(const void* insts, const long long* bstart, const BatchGeom* geom, int n,
                                        long long nblocks, const void* fin, const void* forces, void* fout,
                                        const long long* step0, int step, hipStream_t st)
{
    auto kern = k_split_batch<LAT, T, BX, BY, MINW, PF, FF>;
    const size_t lds = split_lds<LAT, T, BX, BY>();
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(split_threads<BX, BY>()), lds, st, (const Inst<T>*)insts,
                       bstart, geom, n, (const T*)fin, (const T*)forces, (T*)fout, step0, step);
    return hipGetLastError();
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF>
static hipError_t split_batch_launch_t(const void* insts, const long long* bstart, const BatchGeom* geom, int n,
                                       long long nblocks, const void* fin, const void* forces, void* fout,
                                       const long long* step0, int step, hipStream_t st)
{
    if (forces)
        return split_batch_launch_ff<LAT, T, BX, BY, MINW, PF, true>(insts, bstart, geom, n, nblocks, fin, forces, fout,
                                                                     step0, step, st);
    return split_batch_launch_ff<LAT, T, BX, BY, MINW, PF, false>(insts, bstart, geom, n, nblocks, fin, forces, fout,
                                                                  step0, step, st);
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF>
static long long split_batch_slots_t(int n_cu)
{
    return resident_slots(k_split_batch<LAT, T, BX, BY, MINW, PF, false>, split_threads<BX, BY>(),
                          split_lds<LAT, T, BX, BY>(), n_cu);
}

// workgroups of the batched two-lane kernel resident on the device at once
long long split_batch_slots(int lattice, int dtype, int variant, int n_cu)
{
    if (lattice == DUGKS_D2Q9) {
        if (dtype == DUGKS_F64) {
            if (variant == 1) return split_batch_slots_t<D2Q9, double, 64, 1, 2, false>(n_cu);
            if (variant == 2) return split_batch_slots_t<D2Q9, double, 256, 1, 2, false>(n_cu);
            return split_batch_slots_t<D2Q9, double, 128, 1, 2, false>(n_cu);
        }
        if (variant == 1) return split_batch_slots_t<D2Q9, float, 64, 1, 2, false>(n_cu);
        if (variant == 2) return split_batch_slots_t<D2Q9, float, 256, 1, 2, false>(n_cu);
        return split_batch_slots_t<D2Q9, float, 128, 1, 2, false>(n_cu);
    }
    return dtype == DUGKS_F64 ? split_batch_slots_t<D3Q19, double, 18, 14, 1, false>(n_cu)
                              : split_batch_slots_t<D3Q19, float, 18, 14, 2, false>(n_cu);
}

hipError_t split_batch_launch(int lattice, int dtype, int variant, const void* insts, const long long* bstart,
                              const BatchGeom* geom, int n, long long nblocks, const void* fin, const void* forces,
                              void* fout, const long long* step0, int step, hipStream_t st)
{
#define DUGKS_SPLIT_ARGS insts, bstart, geom, n, nblocks, fin, forces, fout, step0, step, st
    if (lattice == DUGKS_D2Q9) {
        if (dtype == DUGKS_F64) {
            if (variant == 1) return split_batch_launch_t<D2Q9, double, 64, 1, 2, false>(DUGKS_SPLIT_ARGS);
            if (variant == 2) return split_batch_launch_t<D2Q9, double, 256, 1, 2, false>(DUGKS_SPLIT_ARGS);
            return split_batch_launch_t<D2Q9, double, 128, 1, 2, false>(DUGKS_SPLIT_ARGS);
        }
        if (variant == 1) return split_batch_launch_t<D2Q9, float, 64, 1, 2, false>(DUGKS_SPLIT_ARGS);
        if (variant == 2) return split_batch_launch_t<D2Q9, float, 256, 1, 2, false>(DUGKS_SPLIT_ARGS);
        return split_batch_launch_t<D2Q9, float, 128, 1, 2, false>(DUGKS_SPLIT_ARGS);
    }
    return dtype == DUGKS_F64 ? split_batch_launch_t<D3Q19, double, 18, 14, 1, false>(DUGKS_SPLIT_ARGS)
                              : split_batch_launch_t<D3Q19, float, 18, 14, 2, false>(DUGKS_SPLIT_ARGS);
#undef DUGKS_SPLIT_ARGS
}

}  // namespace dugks
