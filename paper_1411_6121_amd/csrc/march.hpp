// march.hpp -- helpers shared by the plane-marching step kernels: column
// classification of a tile, the LDS plane ring and the XCD-aware workgroup
// order.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_general.hpp"

namespace dugks {

// ring slot of plane p in a three-plane ring (p may be negative)
__device__ __forceinline__ int ring(int p) { return ((p % 3) + 3) % 3; }

// metric coefficients of column coordinate x along in-plane axis a (clamped
// for halo columns, which never update)
template <typename T>
__device__ __forceinline__ CellMetric<T> upd_col_pre(const Inst<T>& P, int a, int x)
{
    const int i = x < 0 ? 0 : (x >= P.n[a] ? P.n[a] - 1 : x);
    return load_metric(P, a, i);
}

// kinds of a column coordinate along one in-plane axis
enum { COL_CELL = 0, COL_GHOST_LO = 1, COL_GHOST_HI = 2, COL_OUT = 3 };

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that each XCD receives one contiguous range of the
// logical order (tiles fastest): tiles that share halo columns then run on
// the same XCD at about the same time and read the shared lines from one L2.
// A bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_order(int b, int nb)
{
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = b % X, k = b / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Planes marched per workgroup (the chunk) of an automatic launch.  W(c) =
// tiles * ceil(n / c) workgroups run in ceil(W / S) rounds on S resident
// workgroups (CUs x workgroups per CU); a workgroup computes c + 2 planes of
// f-bar-plus and c planes of faces and updates, about 2c + 2 plane stages of
// similar cost.  The chunk minimises rounds x (2c + 2) over c = 1, 2, 4 ..
// 32, the larger c on ties (fewer halo planes recomputed and re-read).
// Small meshes thus march one or two planes per workgroup (the step is then
// bound by the latency of one workgroup), large ones 8 to 16.
inline int auto_chunk(long long tiles, int nM, long long slots)
{
    nM = nM > 1 ? nM : 1;
    slots = slots > 1 ? slots : 1;
    int best = 1;
    double best_cost = 1e300;
    for (int c = 1; c <= 32; c *= 2) {
        const int cc = c < nM ? c : nM;
        const long long W = tiles * ((nM + cc - 1) / cc);
        const double cost = (double)((W + slots - 1) / slots) * (2.0 * cc + 2.0);
        if (cost <= best_cost) {
            best_cost = cost;
            best = cc;
        }
        if (cc >= nM) break;
    }
    return best;
}

// workgroups of a step kernel resident on the whole device at once
template <typename K>
inline long long resident_slots(K kern, int threads, size_t lds, int n_cu)
{
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, lds) != hipSuccess || per < 1) per = 1;
    return (long long)per * (n_cu > 0 ? n_cu : 1);
}

// the chunk of a launch: the context's fixed value, else auto_chunk
inline int launch_chunk(int fixed, long long tiles, int nM, long long slots)
{
    if (fixed > 0) return fixed < nM ? fixed : (nM > 1 ? nM : 1);
    return auto_chunk(tiles, nM, slots);
}

// Occupancy bounds of a step kernel (waves per SIMD), for the attribute
//   amdgpu_waves_per_eu(min, max).
// The LDS ring decides how many workgroups share a CU; stating the true
// maximum keeps the compiler from trading instruction-level parallelism for
// an occupancy the LDS never allows.  D3Q19 one lane per column: FP64 155 KB
// -> one 4-wave workgroup per CU, FP32 78 KB -> two; two lanes per column
// (512 threads): FP64 two waves per SIMD, FP32 up to four.  D2Q9 tiles are
// small: up to 8.
template <class LAT, typename T, bool SPLIT>
__host__ __device__ constexpr int max_waves_per_eu()
{
    if (LAT::D == 2) return 8;
    if (SPLIT) return sizeof(T) == 8 ? 2 : 4;
    return sizeof(T) == 8 ? 1 : 2;
}

#define DUGKS_KERNEL_BOUNDS(NT, MINW, MAXW) \
    __attribute__((amdgpu_flat_work_group_size(1, NT), amdgpu_waves_per_eu(MINW, MAXW)))

}  // namespace dugks
