// kernels_fused.hip -- single-launch step for gfx950.
//
// One workgroup owns a halo-inclusive tile of columns in the plane of the
// first D-1 axes (one thread per column) and marches along the last axis
// (z in 3-D, y in 2-D) over a chunk of planes.  f-bar-plus (Eq. f_bar_+,
// with the ghost rule) of three consecutive planes lives in an LDS ring;
// each new plane is computed from the state once per column (ghost columns
// and ghost planes by extrapolation inside LDS), and every interior thread
// then performs the interface and update stages for its cell from LDS: the
// state is read once from HBM (plus the tile halo, which hits L2) and the new
// state written once.
//
// Faces are evaluated by both neighbouring cells with identical code and
// operands, so the two sides see bitwise-identical fluxes (conservation to
// rounding).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ctx.hpp"
#include "kernels_general.hpp"
#include "march.hpp"

namespace dugks {

// f-bar-plus in the LDS ring, relative to the thread's cell in the current
// plane: ring slot offsets of the neighbouring planes are kept as integer
// element offsets (dz_up, dz_dn), in-plane offsets are +-1 / +-BX.
template <class LAT, typename T, int BX, int BY>
struct LdsPhi {
    const T* s;
    int cur;           // element offset of (current plane, q = 0, this column)
    int dz_up, dz_dn;  // offset from the current plane to the next / previous
    static constexpr int SQ = BX * BY;  // stride between velocity planes
    __device__ __forceinline__ int base(int ox, int oy, int oz) const
    {
        if constexpr (LAT::D == 3) return cur + ox + oy * BX + (oz > 0 ? dz_up : (oz < 0 ? dz_dn : 0));
        else return cur + ox + (oy > 0 ? dz_up : (oy < 0 ? dz_dn : 0));
    }
    // offsets to the +t / -t neighbour of a cell in the current plane
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
    __device__ __forceinline__ T get(int q, int b) const { return s[b + q * SQ]; }
};

// One workgroup's work: tile index `tile` (of tiles0 x tiles1) and march
// chunk `ck` of the instance P; fin/fout/force already point at the
// instance's arrays.
template <class LAT, typename T, int BX, int BY>
__device__ __forceinline__ void fused_body(const Inst<T>& P, const T* __restrict__ fin, const T* __restrict__ force,
                                           T* __restrict__ fout, T gt, T gth, int chunk, int tiles0, int tile,
                                           int ck, T* lds)
{
    constexpr int Q = LAT::Q, D = LAT::D, M = D - 1;  // M: march axis
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int b0 = tile % tiles0, b1 = tile / tiles0;

    // column coordinates (in-plane axes 0 .. D-2), kinds and source cells
    int g[2], kind[2], src[2];
    g[0] = b0 * (BX - 2) - 1 + tx;
    g[1] = (D == 3) ? b1 * (BY - 2) - 1 + ty : 0;
#pragma unroll
    for (int a = 0; a < D - 1; ++a) {
        const int N = P.n[a], x = g[a];
        if (x >= 0 && x < N) { kind[a] = COL_CELL; src[a] = x; }
        else if (P.per[a] && x == -1) { kind[a] = COL_CELL; src[a] = N - 1; }
        else if (P.per[a] && x == N) { kind[a] = COL_CELL; src[a] = 0; }
        else if (!P.per[a] && x == -1) { kind[a] = COL_GHOST_LO; src[a] = 0; }
        else if (!P.per[a] && x == N) { kind[a] = COL_GHOST_HI; src[a] = N - 1; }
        else { kind[a] = COL_OUT; src[a] = 0; }
    }
    if (D == 2) { kind[1] = COL_CELL; src[1] = 0; }
    const bool cell_col = kind[0] == COL_CELL && kind[1] == COL_CELL;
    const bool ghost_col = !cell_col && kind[0] != COL_OUT && kind[1] != COL_OUT;
    const bool upd_col = cell_col && g[0] >= 0 && g[0] < P.n[0] && tx >= 1 && tx <= BX - 2 &&
                         (D == 2 || (g[1] >= 0 && g[1] < P.n[1] && ty >= 1 && ty <= BY - 2));

    const int nM = P.n[M];
    const int p0 = ck * chunk;
    const int p1 = min(p0 + chunk, nM);
    const bool perM = P.per[M] != 0;
    // in-plane metric coefficients of this column are fixed for the march
    const CellMetric<T> cmx = upd_col_pre(P, 0, g[0]);
    const CellMetric<T> cmy = D == 3 ? upd_col_pre(P, 1, g[1]) : cmx;

    auto slot_ptr = [&](int p, int q) -> T* {
        return lds + ((long)(ring(p) * Q + q) * BY + ty) * BX + tx;
    };
    auto lds_at = [&](int p, int q, int dx, int dy) -> T {
        return lds[((long)(ring(p) * Q + q) * BY + (ty + dy)) * BX + (tx + dx)];
    };

    // f-bar-plus of plane p (0 <= p < nM, or wrapped on a periodic march axis)
    auto compute_plane = [&](int p) {
        const int pp = perM ? ((p % nM) + nM) % nM : p;
        if (cell_col) {
            int c3[3];
            c3[0] = src[0];
            c3[1] = (D == 3) ? src[1] : pp;
            c3[2] = (D == 3) ? pp : 0;
            T v[Q];
            phi_cell<LAT, T>(P, fin, force, int_idx(P, c3[0], c3[1], c3[2]), gt, v);
#pragma unroll
            for (int q = 0; q < Q; ++q) slot_ptr(p, q)[0] = v[q];
        }
        __syncthreads();
        if (ghost_col) {
            // tensor-product extrapolation from the cells of the same plane
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
            T acc[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] = T(0);
            for (int i1 = 0; i1 < cnt[1]; ++i1)
                for (int i0 = 0; i0 < cnt[0]; ++i0) {
                    const T w = wt[0][i0] * wt[1][i1];
#pragma unroll
                    for (int q = 0; q < Q; ++q) acc[q] += w * lds_at(p, q, off[0][i0], off[1][i1]);
                }
#pragma unroll
            for (int q = 0; q < Q; ++q) slot_ptr(p, q)[0] = acc[q];
        }
        __syncthreads();
    };
    // ghost plane p of a wall march axis: extrapolation along the march axis
    // through planes a (nearest) and b, column by column
    auto ghost_plane = [&](int p, int a, int b, T r) {
        if (cell_col || ghost_col) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                slot_ptr(p, q)[0] = (T(1) - r) * slot_ptr(a, q)[0] + r * slot_ptr(b, q)[0];
        }
        __syncthreads();
    };

    int hi;
    if (!perM && p0 == 0) {
        compute_plane(0);
        compute_plane(1);
        ghost_plane(-1, 0, 1, P.rlo[M]);
        hi = 1;
    } else {
        compute_plane(p0 - 1);
        compute_plane(p0);
        hi = p0;
    }
    for (int z = p0; z < p1; ++z) {
        if (hi < z + 1) {
            __syncthreads();  // the ring slot of z+1 held plane z-2, read by the last update
            if (!perM && z + 1 == nM) ghost_plane(z + 1, z, z - 1, P.rhi[M]);
            else compute_plane(z + 1);
            hi = z + 1;
        }
        if (upd_col) {
            int ci[3];
            ci[0] = g[0];
            ci[1] = (D == 3) ? g[1] : z;
            ci[2] = (D == 3) ? z : 0;
            const long long cidx = int_idx(P, ci[0], ci[1], ci[2]);
            const int slot = Q * BX * BY;
            LdsPhi<LAT, T, BX, BY> ph{lds, ring(z) * slot + ty * BX + tx, (ring(z + 1) - ring(z)) * slot,
                                      (ring(z - 1) - ring(z)) * slot};
            T acc[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const T p = ph.get(q, ph.cur);
                acc[q] = p + (p - fin[(long long)q * P.nc + cidx]) * T(1.0 / 3.0);  // Eq. (f_tilde_+)
            }
            const CellMetric<T> cmm = load_metric(P, M, z);
            if constexpr (D == 3) cell_fluxes<LAT, T>(P, ph, force, ci, gth, cmx, cmy, cmm, acc);
            else cell_fluxes<LAT, T>(P, ph, force, ci, gth, cmx, cmm, cmm, acc);
#pragma unroll
            for (int q = 0; q < Q; ++q) fout[(long long)q * P.nc + cidx] = acc[q];
        }
    }
}

template <class LAT, typename T, int BX, int BY, int MINW>
__global__ __launch_bounds__(BX* BY, MINW) void k_fused(const Inst<T>* __restrict__ Pp, const T* __restrict__ fin,
                                                         const T* __restrict__ force, T* __restrict__ fout,
                                                         double t, int chunk, int tiles0)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Inst<T>& P = *Pp;
    // time factors evaluated on the device (same code as the batched form)
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * P.dtd);
    fused_body<LAT, T, BX, BY>(P, fin, force, fout, gt, gth, chunk, tiles0, blockIdx.x, blockIdx.y,
                               reinterpret_cast<T*>(smem_raw));
}

// ---------------------------------------------------------------------------
// v2: every interface evaluated once.  Per plane: each column evaluates its
// upper x (and y) interface (tile halo columns included) into an LDS face
// buffer and each updating column its upper march-axis interface (kept in
// registers for the next plane); after a barrier every updating cell takes
// the differences of its two faces per axis (Eqs. microflux, f_tilde_+).
// ---------------------------------------------------------------------------
template <class LAT, typename T, int BX, int BY, bool PF, bool UNI>
__device__ __forceinline__ void fused2_body(const Inst<T>& P, const T* __restrict__ fin, const T* __restrict__ force,
                                            T* __restrict__ fout, T gt, T gth, int chunk, int tiles0, int tile,
                                            int ck, T* lds)
{
    constexpr int Q = LAT::Q, D = LAT::D, M = D - 1;
    constexpr int NX = cross_count<LAT, 0>(), NY = cross_count<LAT, 1>();
    constexpr int NM = cross_count<LAT, (D == 3 ? 2 : 1)>();
    constexpr int SQ = BX * BY;
    T* fxb = lds + 3 * Q * SQ;         // [NX][BY][BX] upper x faces
    T* fyb = fxb + NX * SQ;            // [NY][BY][BX] upper y faces (3-D)
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int b0 = tile % tiles0, b1 = tile / tiles0;

    int g[2], kind[2], src[2];
    g[0] = b0 * (BX - 2) - 1 + tx;
    g[1] = (D == 3) ? b1 * (BY - 2) - 1 + ty : 0;
#pragma unroll
    for (int a = 0; a < D - 1; ++a) {
        const int N = P.n[a], x = g[a];
        if (x >= 0 && x < N) { kind[a] = COL_CELL; src[a] = x; }
        else if (P.per[a] && x == -1) { kind[a] = COL_CELL; src[a] = N - 1; }
        else if (P.per[a] && x == N) { kind[a] = COL_CELL; src[a] = 0; }
        else if (!P.per[a] && x == -1) { kind[a] = COL_GHOST_LO; src[a] = 0; }
        else if (!P.per[a] && x == N) { kind[a] = COL_GHOST_HI; src[a] = N - 1; }
        else { kind[a] = COL_OUT; src[a] = 0; }
    }
    if (D == 2) { kind[1] = COL_CELL; src[1] = 0; }
    const bool cell_col = kind[0] == COL_CELL && kind[1] == COL_CELL;
    const bool ghost_col = !cell_col && kind[0] != COL_OUT && kind[1] != COL_OUT;
    const bool row_ok = (D == 2) || (g[1] >= 0 && g[1] < P.n[1] && ty >= 1 && ty <= BY - 2);
    const bool col_ok = g[0] >= 0 && g[0] < P.n[0] && tx >= 1 && tx <= BX - 2;
    const bool upd_col = cell_col && col_ok && row_ok;
    // upper x face of this column: needed for faces 0..n0 of interior rows
    const bool xface = (cell_col || ghost_col) && row_ok && tx <= BX - 2 && g[0] >= -1 && g[0] <= P.n[0] - 1;
    // upper y face (3-D): faces 0..n1 of interior columns
    const bool yface = (D == 3) && (cell_col || ghost_col) && col_ok && ty <= BY - 2 && g[1] >= -1 &&
                       g[1] <= P.n[1] - 1;

    // workgroup-uniform: does the tile hold ghost columns (wall-side tiles)
    const bool any_ghost = __syncthreads_or(ghost_col) != 0;
    const int nM = P.n[M];
    const int p0 = ck * chunk;
    const int p1 = min(p0 + chunk, nM);
    const bool perM = P.per[M] != 0;
    const CellMetric<T> cmx = upd_col_pre(P, 0, g[0]);
    const CellMetric<T> cmy = D == 3 ? upd_col_pre(P, 1, g[1]) : cmx;

    auto slot_ptr = [&](int p, int q) -> T* { return lds + ((long)(ring(p) * Q + q) * BY + ty) * BX + tx; };
    auto lds_at = [&](int p, int q, int dx, int dy) -> T {
        return lds[((long)(ring(p) * Q + q) * BY + (ty + dy)) * BX + (tx + dx)];
    };
    // state (and force field) of the plane a column computes next, loaded
    // into registers one plane ahead of its use
    T pf[Q], pg[3] = {T(0), T(0), T(0)};
    auto plane_cell = [&](int p) -> long long {
        const int pp = perM ? ((p % nM) + nM) % nM : p;
        return int_idx(P, src[0], (D == 3) ? src[1] : pp, (D == 3) ? pp : 0);
    };
    auto load_plane = [&](int p) {
        if (PF && cell_col) {
            const int pp = perM ? ((p % nM) + nM) % nM : p;
            const long long ci = int_idx(P, src[0], (D == 3) ? src[1] : pp, (D == 3) ? pp : 0);
#pragma unroll
            for (int q = 0; q < Q; ++q) pf[q] = fin[(long long)q * P.nc + ci];
            if (force) {
#pragma unroll
                for (int a = 0; a < D; ++a) pg[a] = force[(long long)a * P.nc + ci];
            }
        }
    };
    // f-bar-plus of plane p from the loaded registers
    auto compute_plane = [&](int p) {
        if (cell_col) {
            T v[Q];
            if constexpr (PF) phi_from<LAT, T>(P, pf, pg, force != nullptr, gt, v);
            else phi_cell<LAT, T>(P, fin, force, plane_cell(p), gt, v);
#pragma unroll
            for (int q = 0; q < Q; ++q) slot_ptr(p, q)[0] = v[q];
        }
        __syncthreads();
        if (!any_ghost) return;
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
            T acc[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] = T(0);
            for (int i1 = 0; i1 < cnt[1]; ++i1)
                for (int i0 = 0; i0 < cnt[0]; ++i0) {
                    const T w = wt[0][i0] * wt[1][i1];
#pragma unroll
                    for (int q = 0; q < Q; ++q) acc[q] += w * lds_at(p, q, off[0][i0], off[1][i1]);
                }
#pragma unroll
            for (int q = 0; q < Q; ++q) slot_ptr(p, q)[0] = acc[q];
        }
        __syncthreads();
    };
    auto ghost_plane = [&](int p, int a, int b, T r) {
        if (cell_col || ghost_col) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                slot_ptr(p, q)[0] = (T(1) - r) * slot_ptr(a, q)[0] + r * slot_ptr(b, q)[0];
        }
        __syncthreads();
    };
    auto phi_view = [&](int z) {
        const int slot = Q * SQ;
        return LdsPhi<LAT, T, BX, BY>{lds, ring(z) * slot + ty * BX + tx, (ring(z + 1) - ring(z)) * slot,
                                      (ring(z - 1) - ring(z)) * slot};
    };

    // a plane computed (not extrapolated) by the march: 0 <= p < nM, or any
    // p on a periodic march axis
    auto computed = [&](int p) { return perM || p < nM; };
    int hi;
    if (!perM && p0 == 0) {
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
    // lower march-axis face of the first plane
    T zlo[NM];
    if (upd_col) {
        int ci[3];
        ci[0] = g[0];
        ci[1] = (D == 3) ? g[1] : p0;
        ci[2] = (D == 3) ? p0 : 0;
        const CellMetric<T> cmm = load_metric(P, M, p0);
        const auto ph = phi_view(p0);
        if constexpr (D == 3) face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, M, UNI>(P, ph, force, ci, -1, p0, gth, cmx, cmy, cmm, zlo);
        else face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, M, UNI>(P, ph, force, ci, -1, p0, gth, cmx, cmm, cmm, zlo);
    }
    for (int z = p0; z < p1; ++z) {
        if (hi < z + 1) {
            // No barrier needed here: the ring slot of z+1 (= z-2) was last
            // read by the faces of plane z-1, which every wave finished before
            // the barrier that precedes the update of z-1; the face buffers
            // are rewritten only after the barrier that ends this plane's
            // computation, by which time every wave has left that update.
            if (!computed(z + 1)) {
                ghost_plane(z + 1, z, z - 1, P.rhi[M]);
            } else {
                if (!PF) load_plane(z + 1);
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
        // the cell's own state for Eq. (f_tilde_+), loaded before the faces
        // (PF) or at the update
        T fz[Q];
        auto load_own = [&]() {
            const long long cidx = int_idx(P, ci[0], ci[1], ci[2]);
#pragma unroll
            for (int q = 0; q < Q; ++q) fz[q] = fin[(long long)q * P.nc + cidx];
        };
        if (PF && upd_col) load_own();
        T zhi[NM];
        if (xface) {
            T v[NX];
            if constexpr (D == 3) face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, 0, UNI>(P, ph, force, ci, 0, g[0] + 1, gth, cmx, cmy, cmm, v);
            else face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, 0, UNI>(P, ph, force, ci, 0, g[0] + 1, gth, cmx, cmm, cmm, v);
#pragma unroll
            for (int k = 0; k < NX; ++k) fxb[(k * BY + ty) * BX + tx] = v[k];
        }
        if constexpr (D == 3) {
            if (yface) {
                T v[NY];
                face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, 1, UNI>(P, ph, force, ci, 0, g[1] + 1, gth, cmx, cmy, cmm, v);
#pragma unroll
                for (int k = 0; k < NY; ++k) fyb[(k * BY + ty) * BX + tx] = v[k];
            }
        }
        if (upd_col) {
            if constexpr (D == 3) face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, M, UNI>(P, ph, force, ci, 0, z + 1, gth, cmx, cmy, cmm, zhi);
            else face_once<LAT, T, LdsPhi<LAT, T, BX, BY>, M, UNI>(P, ph, force, ci, 0, z + 1, gth, cmx, cmm, cmm, zhi);
        }
        __syncthreads();
        if (upd_col) {
            const long long cidx = int_idx(P, ci[0], ci[1], ci[2]);
            T acc[Q];
            if (!PF) load_own();
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const T p = ph.get(q, ph.cur);
                acc[q] = p + (p - fz[q]) * T(1.0 / 3.0);  // Eq. (f_tilde_+)
            }
            const T sx = (UNI ? P.ufdx[0] : cmx.fdx) * P.c, sm = (UNI ? P.ufdx[M] : cmm.fdx) * P.c;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if (LAT::e(q, 0) != 0) {
                    const int k = cross_slot<LAT, 0>(q);
                    const T d = fxb[(k * BY + ty) * BX + tx] - fxb[(k * BY + ty) * BX + tx - 1];
                    acc[q] -= T(LAT::e(q, 0)) * sx * d;
                }
                if constexpr (D == 3) {
                    if (LAT::e(q, 1) != 0) {
                        const int k = cross_slot<LAT, 1>(q);
                        const T d = fyb[(k * BY + ty) * BX + tx] - fyb[(k * BY + ty - 1) * BX + tx];
                        acc[q] -= T(LAT::e(q, 1)) * ((UNI ? P.ufdx[1] : cmy.fdx) * P.c) * d;
                    }
                }
                if (LAT::e(q, M) != 0) {
                    const int k = cross_slot<LAT, M>(q);
                    acc[q] -= T(LAT::e(q, M)) * sm * (zhi[k] - zlo[k]);
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) fout[(long long)q * P.nc + cidx] = acc[q];
#pragma unroll
            for (int k = 0; k < NM; ++k) zlo[k] = zhi[k];
        }
    }
}

// FF: the launch carries a force field (without one the kernel is compiled
// with a null field and no field code)
template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF, bool UNI>
__global__ DUGKS_KERNEL_BOUNDS(BX * BY, MINW, (max_waves_per_eu<LAT, T, false>())) void k_fused2(const Inst<T>* __restrict__ Pp, const T* __restrict__ fin,
                                                          const T* __restrict__ force, T* __restrict__ fout,
                                                          double t, int chunk, int tiles0, int tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Inst<T>& P = *Pp;
    const T gt = tfac(P, t), gth = tfac(P, t + 0.5 * P.dtd);
    const int ntile = (int)tiles;
    const int b = xcd_order((int)blockIdx.x, (int)gridDim.x);
    fused2_body<LAT, T, BX, BY, PF, UNI>(P, fin, FF ? force : nullptr, fout, gt, gth, chunk, tiles0, b % ntile, b / ntile,
                                reinterpret_cast<T*>(smem_raw));
}

// Batched form: workgroup b (in XCD order) belongs to the instance i with
// bstart[i] <= b < bstart[i+1]; the instance table holds each instance's
// state offset, force offset, tile counts and chunk (BatchGeom).  Time of
// instance i at this launch: (step0 + step) * dt_i, with step0 a device
// counter so that a captured graph replays with advancing time.
template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF>
__global__ DUGKS_KERNEL_BOUNDS(BX * BY, MINW, (max_waves_per_eu<LAT, T, false>())) void k_fused2_batch(const Inst<T>* __restrict__ insts,
                                                                const long long* __restrict__ bstart,
                                                                const BatchGeom* __restrict__ geom, int ninst,
                                                                const T* __restrict__ fin, const T* __restrict__ forces,
                                                                T* __restrict__ fout,
                                                                const long long* __restrict__ step0, int step)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const long long b = xcd_order((int)blockIdx.x, (int)gridDim.x);
    int lo = 0, hi = ninst - 1;  // bstart[lo] <= b < bstart[hi+1]
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
        fused2_body<LAT, T, BX, BY, PF, true>(P, fin + P.off, force, fout + P.off, gt, gth, g.chunk, g.tiles0,
                                              local % ntile, local / ntile, reinterpret_cast<T*>(smem_raw));
    else
        fused2_body<LAT, T, BX, BY, PF, false>(P, fin + P.off, force, fout + P.off, gt, gth, g.chunk, g.tiles0,
                                               local % ntile, local / ntile, reinterpret_cast<T*>(smem_raw));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// device copy of the instance parameters of the context (uploaded at init)
static const void* dev_inst(const dugks_ctx* ctx) { return ctx->inst_dev; }

// Plane prefetch (state of plane z+2 loaded during plane z) costs about
// 2Q registers per thread: used where the kernel's occupancy target still
// holds with them (D3Q19 FP64 runs one wave per SIMD anyway, D2Q9 FP32 has
// room), not where it would spill (D3Q19 FP32, D2Q9 FP64 at two waves).
template <class LAT, typename T>
constexpr bool prefetch_planes()
{
    return (LAT::D == 3) == (sizeof(T) == 8);
}

// LDS of the v2 kernels: three f-bar-plus planes and the x (and y) face
// buffers
template <class LAT, typename T, int BX, int BY>
static size_t fused2_lds()
{
    return (size_t)(3 * LAT::Q + cross_count<LAT, 0>() + (LAT::D == 3 ? cross_count<LAT, 1>() : 0)) * BX * BY * sizeof(T);
}

template <class LAT, typename T, int BX, int BY, int MINW>
static int launch_fused(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force, double t,
                        hipStream_t st, int chunk)
{
    constexpr int D = LAT::D, M = D - 1;
    const int tiles0 = (P.n[0] + BX - 3) / (BX - 2);
    const int tiles1 = (D == 3) ? (P.n[1] + BY - 3) / (BY - 2) : 1;
    const size_t lds = (size_t)3 * LAT::Q * BX * BY * sizeof(T);
    auto kern = k_fused<LAT, T, BX, BY, MINW>;
    static bool attr_set = false;
    static long long slots = 0;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_check(ctx, e, "fused kernel LDS attribute");
        slots = resident_slots(kern, BX * BY, lds, ctx->n_cu);
        attr_set = true;
    }
    chunk = launch_chunk(chunk, (long long)tiles0 * tiles1, P.n[M], slots);
    const int chunks = (P.n[M] + chunk - 1) / chunk;
    hipLaunchKernelGGL(kern, dim3(tiles0 * tiles1, chunks), dim3(BX * BY), lds, st, (const Inst<T>*)dev_inst(ctx),
                       (const T*)fin, (const T*)force, (T*)fout, t, chunk, tiles0);
    return hip_check(ctx, hipGetLastError(), "fused step launch");
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF, bool UNI>
static int launch_fused2_ff(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force,
                            double t, hipStream_t st, int chunk)
{
    constexpr int D = LAT::D, M = D - 1;
    const int tiles0 = (P.n[0] + BX - 3) / (BX - 2);
    const int tiles1 = (D == 3) ? (P.n[1] + BY - 3) / (BY - 2) : 1;
    const size_t lds = fused2_lds<LAT, T, BX, BY>();
    auto kern = k_fused2<LAT, T, BX, BY, MINW, PF, FF, UNI>;
    static bool attr_set = false;
    static long long slots = 0;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_check(ctx, e, "fused kernel LDS attribute");
        slots = resident_slots(kern, BX * BY, lds, ctx->n_cu);
        attr_set = true;
    }
    chunk = launch_chunk(chunk, (long long)tiles0 * tiles1, P.n[M], slots);
    const int chunks = (P.n[M] + chunk - 1) / chunk;
    const long long nb = (long long)tiles0 * tiles1 * chunks;
    if (nb > 0x7fffffffLL) return fail(ctx, DUGKS_EUNSUPPORTED, "mesh too large for one launch");
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(BX * BY), lds, st, (const Inst<T>*)dev_inst(ctx),
                       (const T*)fin, (const T*)force, (T*)fout, t, chunk, tiles0, tiles0 * tiles1);
    return hip_check(ctx, hipGetLastError(), "fused step launch");
}

template <class LAT, typename T, int BX, int BY, int MINW, bool PF>
static int launch_fused2(dugks_ctx* ctx, const Inst<T>& P, const void* fin, void* fout, const void* force, double t,
                         hipStream_t st, int chunk)
{
    if (P.uni) {
        if (force) return launch_fused2_ff<LAT, T, BX, BY, MINW, PF, true, true>(ctx, P, fin, fout, force, t, st, chunk);
        return launch_fused2_ff<LAT, T, BX, BY, MINW, PF, false, true>(ctx, P, fin, fout, force, t, st, chunk);
    }
    if (force) return launch_fused2_ff<LAT, T, BX, BY, MINW, PF, true, false>(ctx, P, fin, fout, force, t, st, chunk);
    return launch_fused2_ff<LAT, T, BX, BY, MINW, PF, false, false>(ctx, P, fin, fout, force, t, st, chunk);
}

// Default step kernel (measured on MI355X, 128^3 D3Q19 and 1024^2 D2Q9
// cavities).  The two-lane split (3) doubles the waves per SIMD of the D3Q19
// tile and wins wherever its registers fit the occupancy it is built for;
// with a force field its face-force interpolation spills (D3Q19 FP64), and
// in FP32 only the uniform field-free instance fits four waves per SIMD, so
// those cases take the one-lane kernel (2).  D2Q9 and D3Q27: the split
// everywhere.
int default_step_kernel(int lattice, int dtype, bool uniform, bool field)
{
    if (lattice == DUGKS_D2Q9 || lattice == DUGKS_D3Q27) return 3;
    if (dtype == DUGKS_F64) return field ? 2 : 3;
    return (uniform && !field) ? 3 : 2;
}

int split_step(dugks_ctx* ctx, const void* fin, void* fout, const void* force, double t, hipStream_t st, int chunk);

int setup_fast(dugks_ctx* ctx)
{
    ctx->fast = 0;
    const char* env = getenv("DUGKS_FORCE_GENERAL");
    if (env && env[0] == '1') return DUGKS_OK;
    // 1: every face evaluated by both neighbours; 2: faces evaluated once;
    // 3: faces once, velocity set split over two lanes per column;
    // 4: per launch, the default of default_step_kernel
    ctx->fast = 4;
    const char* v = getenv("DUGKS_FUSED_VARIANT");
    if (v && v[0] == '1') ctx->fast = 1;
    if (v && v[0] == '2') ctx->fast = 2;
    if (v && v[0] == '3') ctx->fast = 3;
    // march length override (tuning sweeps)
    const char* ch = getenv("DUGKS_CHUNK");
    ctx->chunk = ch ? std::max(0, atoi(ch)) : 0;
    return DUGKS_OK;
}

// the step kernel a launch with (without) a force field uses
int resolve_step_kernel(const dugks_ctx* ctx, bool field)
{
    // the original-model variant: the two-lane kernel where it is the
    // incompressible choice and no force field is given, else the general
    // kernels
    if (ctx->cfg.model != DUGKS_MODEL_INCOMPRESSIBLE) {
        if (field || ctx->fast == 0) return 0;
        if (ctx->cfg.lattice == DUGKS_D3Q27) return 3;
        const bool uni = ctx->cfg.dtype == DUGKS_F64 ? ctx->pd.uni != 0 : ctx->pf.uni != 0;
        const int v = ctx->fast != 4 ? ctx->fast : default_step_kernel(ctx->cfg.lattice, ctx->cfg.dtype, uni, false);
        return v == 3 ? 3 : 0;
    }
    // D3Q27 has the split kernel only (the one-lane tile would not fit a CU)
    if (ctx->cfg.lattice == DUGKS_D3Q27) return ctx->fast == 0 ? 0 : 3;
    if (ctx->fast != 4) return ctx->fast;
    const bool uni = ctx->cfg.dtype == DUGKS_F64 ? ctx->pd.uni != 0 : ctx->pf.uni != 0;
    return default_step_kernel(ctx->cfg.lattice, ctx->cfg.dtype, uni, field);
}

int fast_step(dugks_ctx* ctx, const void* fin, void* fout, const void* force, double t, hipStream_t st, bool* handled)
{
    *handled = false;
    const int variant = resolve_step_kernel(ctx, force != nullptr);
    if (variant < 1 || variant > 3) return DUGKS_OK;
    *handled = true;
    // tiles: D3Q19 18 x 14 columns (16 x 12 interior), D2Q9 rows of 128
    // columns (126 interior)
    const int chunk = ctx->chunk;  // 0: chosen per launch (auto_chunk)
    if (variant == 3) return split_step(ctx, fin, fout, force, t, st, chunk);
    if (variant == 2) {
        if (ctx->cfg.lattice == DUGKS_D3Q19) {
            if (ctx->cfg.dtype == DUGKS_F64) return launch_fused2<D3Q19, double, 18, 14, 1, prefetch_planes<D3Q19, double>()>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
            return launch_fused2<D3Q19, float, 18, 14, 2, prefetch_planes<D3Q19, float>()>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
        }
        if (ctx->cfg.dtype == DUGKS_F64) return launch_fused2<D2Q9, double, 128, 1, 2, prefetch_planes<D2Q9, double>()>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
        return launch_fused2<D2Q9, float, 128, 1, 2, prefetch_planes<D2Q9, float>()>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
    }
    if (ctx->cfg.lattice == DUGKS_D3Q19) {
        if (ctx->cfg.dtype == DUGKS_F64) return launch_fused<D3Q19, double, 18, 14, 1>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
        return launch_fused<D3Q19, float, 18, 14, 2>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
    }
    if (ctx->cfg.dtype == DUGKS_F64) return launch_fused<D2Q9, double, 128, 1, 2>(ctx, ctx->pd, fin, fout, force, t, st, chunk);
    return launch_fused<D2Q9, float, 128, 1, 2>(ctx, ctx->pf, fin, fout, force, t, st, chunk);
}

void release_fast(dugks_ctx*) {}

// Tile shapes of the batched kernel: (columns along x, along y) incl. halo.
// D3Q19 has one (18 x 14: the FP64 LDS ring fills a CU); D2Q9 rows of 128
// (default), 64 or 256 columns, chosen per batch by the autotuner.
int fused_tile_variants(int lattice) { return lattice == DUGKS_D3Q19 ? 1 : 3; }

void fused_tile_shape(int lattice, int variant, int* bx, int* by)
{
    if (lattice == DUGKS_D3Q19) {
        *bx = 18;
        *by = 14;
        return;
    }
    *bx = variant == 1 ? 64 : (variant == 2 ? 256 : 128);
    *by = 1;
}


template <class LAT, typename T, int BX, int BY, int MINW, bool PF, bool FF>
static hipError_t fused2_batch_ff(const void* insts, const long long* bstart, const BatchGeom* geom, int n,
                                  long long nblocks, const void* fin, const void* forces, void* fout,
                                  const long long* step0, int step, hipStream_t st)
{
    auto kern = k_fused2_batch<LAT, T, BX, BY, MINW, PF, FF>;
    const size_t lds = fused2_lds<LAT, T, BX, BY>();
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(BX * BY), lds, st, (const Inst<T>*)insts, bstart, geom, n,
                       (const T*)fin, (const T*)forces, (T*)fout, step0, step);
    return hipGetLastError();
}

template <class LAT, typename T, int BX, int BY, int MINW>
static hipError_t fused2_batch_t(const void* insts, const long long* bstart, const BatchGeom* geom, int n,
                                 long long nblocks, const void* fin, const void* forces, void* fout,
                                 const long long* step0, int step, hipStream_t st)
{
    constexpr bool PF = prefetch_planes<LAT, T>();
    if (forces)
        return fused2_batch_ff<LAT, T, BX, BY, MINW, PF, true>(insts, bstart, geom, n, nblocks, fin, forces, fout,
                                                               step0, step, st);
    return fused2_batch_ff<LAT, T, BX, BY, MINW, PF, false>(insts, bstart, geom, n, nblocks, fin, forces, fout, step0,
                                                            step, st);
}

hipError_t split_batch_launch(int lattice, int dtype, int variant, const void* insts, const long long* bstart,
                              const BatchGeom* geom, int n, long long nblocks, const void* fin, const void* forces,
                              void* fout, const long long* step0, int step, hipStream_t st);

long long split_batch_slots(int lattice, int dtype, int variant, int n_cu);

template <class LAT, typename T, int BX, int BY, int MINW>
static long long fused2_batch_slots_t(int n_cu)
{
    constexpr bool PF = prefetch_planes<LAT, T>();
    return resident_slots(k_fused2_batch<LAT, T, BX, BY, MINW, PF, false>, BX * BY, fused2_lds<LAT, T, BX, BY>(), n_cu);
}

// workgroups of the batched step kernel (the one batch_step_launch takes)
// resident on the device at once
long long batch_resident_slots(int lattice, int dtype, bool uniform, int variant, int n_cu)
{
    if (default_step_kernel(lattice, dtype, uniform, false) == 3) return split_batch_slots(lattice, dtype, variant, n_cu);
    if (lattice == DUGKS_D2Q9) {
        if (dtype == DUGKS_F64) {
            if (variant == 1) return fused2_batch_slots_t<D2Q9, double, 64, 1, 2>(n_cu);
            if (variant == 2) return fused2_batch_slots_t<D2Q9, double, 256, 1, 2>(n_cu);
            return fused2_batch_slots_t<D2Q9, double, 128, 1, 2>(n_cu);
        }
        if (variant == 1) return fused2_batch_slots_t<D2Q9, float, 64, 1, 2>(n_cu);
        if (variant == 2) return fused2_batch_slots_t<D2Q9, float, 256, 1, 2>(n_cu);
        return fused2_batch_slots_t<D2Q9, float, 128, 1, 2>(n_cu);
    }
    return dtype == DUGKS_F64 ? fused2_batch_slots_t<D3Q19, double, 18, 14, 1>(n_cu)
                              : fused2_batch_slots_t<D3Q19, float, 18, 14, 2>(n_cu);
}

// one batched step on the default step kernel of the lattice and precision
// (so that batched and single-instance runs give identical states)
hipError_t batch_step_launch(int lattice, int dtype, bool uniform, int variant, const void* insts,
                             const long long* bstart, const BatchGeom* geom, int n, long long nblocks, const void* fin,
                             const void* forces, void* fout, const long long* step0, int step, hipStream_t st)
{
    if (default_step_kernel(lattice, dtype, uniform, forces != nullptr) == 3)
        return split_batch_launch(lattice, dtype, variant, insts, bstart, geom, n, nblocks, fin, forces, fout, step0,
                                  step, st);
#define DUGKS_BATCH_ARGS insts, bstart, geom, n, nblocks, fin, forces, fout, step0, step, st
    if (lattice == DUGKS_D2Q9) {
        if (dtype == DUGKS_F64) {
            if (variant == 1) return fused2_batch_t<D2Q9, double, 64, 1, 2>(DUGKS_BATCH_ARGS);
            if (variant == 2) return fused2_batch_t<D2Q9, double, 256, 1, 2>(DUGKS_BATCH_ARGS);
            return fused2_batch_t<D2Q9, double, 128, 1, 2>(DUGKS_BATCH_ARGS);
        }
        if (variant == 1) return fused2_batch_t<D2Q9, float, 64, 1, 2>(DUGKS_BATCH_ARGS);
        if (variant == 2) return fused2_batch_t<D2Q9, float, 256, 1, 2>(DUGKS_BATCH_ARGS);
        return fused2_batch_t<D2Q9, float, 128, 1, 2>(DUGKS_BATCH_ARGS);
    }
    return dtype == DUGKS_F64 ? fused2_batch_t<D3Q19, double, 18, 14, 1>(DUGKS_BATCH_ARGS)
                              : fused2_batch_t<D3Q19, float, 18, 14, 2>(DUGKS_BATCH_ARGS);
#undef DUGKS_BATCH_ARGS
}

}  // namespace dugks
