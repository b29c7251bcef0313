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
