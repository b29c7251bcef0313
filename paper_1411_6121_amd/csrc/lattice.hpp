// lattice.hpp -- discrete velocity sets for the gfx950 kernels.
//
// D2Q9: tensor product of the three-point Gauss-Hermite rule in the order
// printed in Sec. II.C (e_x outer, e_y inner); 1-D weights 2/3 (rest) and
// 1/6 (+-1).  D3Q19: e_x outer, e_y middle, e_z inner, corners dropped,
// weights 1/3, 1/18, 1/36.  Both orders are symmetric: opp(q) = Q-1-q.
// xi_q = c e_q with c = sqrt(3 RT) (applied at run time).
#pragma once

#include <hip/hip_runtime.h>

namespace dugks {

struct D2Q9 {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int REST = 4;
    __host__ __device__ static constexpr int ex(int q) { return q / 3 - 1; }
    __host__ __device__ static constexpr int ey(int q) { return q % 3 - 1; }
    __host__ __device__ static constexpr int ez(int) { return 0; }
    __host__ __device__ static constexpr int e(int q, int a) { return a == 0 ? ex(q) : a == 1 ? ey(q) : 0; }
    __host__ __device__ static constexpr int opp(int q) { return Q - 1 - q; }
    __host__ __device__ static constexpr double w(int q)
    {
        return (ex(q) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (ey(q) == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
    }
};

namespace detail {
// D3Q19 components, listed explicitly in the documented order
__host__ __device__ constexpr int d3q19_e(int q, int a)
{
    constexpr int E[19][3] = {
        {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, 0},
        {0, -1, -1}, {0, -1, 0}, {0, -1, 1}, {0, 0, -1}, {0, 0, 0}, {0, 0, 1}, {0, 1, -1}, {0, 1, 0}, {0, 1, 1},
        {1, -1, 0}, {1, 0, -1}, {1, 0, 0}, {1, 0, 1}, {1, 1, 0}};
    return E[q][a];
}
}  // namespace detail

struct D3Q19 {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int REST = 9;
    __host__ __device__ static constexpr int e(int q, int a) { return detail::d3q19_e(q, a); }
    __host__ __device__ static constexpr int ex(int q) { return e(q, 0); }
    __host__ __device__ static constexpr int ey(int q) { return e(q, 1); }
    __host__ __device__ static constexpr int ez(int q) { return e(q, 2); }
    __host__ __device__ static constexpr int opp(int q) { return Q - 1 - q; }
    __host__ __device__ static constexpr double w(int q)
    {
        return (ex(q) * ex(q) + ey(q) * ey(q) + ez(q) * ez(q)) == 0   ? 1.0 / 3.0
               : (ex(q) * ex(q) + ey(q) * ey(q) + ez(q) * ez(q)) == 1 ? 1.0 / 18.0
                                                                    : 1.0 / 36.0;
    }
};

// D3Q27: the paper's 3-D set (Sec. II.C), the full tensor product of the
// three-point rule, e_x outer, e_y middle, e_z inner; rest at q = 13,
// opp(q) = 26 - q; weights products of 2/3 (rest) and 1/6 (+-1).
struct D3Q27 {
    static constexpr int D = 3;
    static constexpr int Q = 27;
    static constexpr int REST = 13;
    __host__ __device__ static constexpr int ex(int q) { return q / 9 - 1; }
    __host__ __device__ static constexpr int ey(int q) { return (q / 3) % 3 - 1; }
    __host__ __device__ static constexpr int ez(int q) { return q % 3 - 1; }
    __host__ __device__ static constexpr int e(int q, int a) { return a == 0 ? ex(q) : a == 1 ? ey(q) : ez(q); }
    __host__ __device__ static constexpr int opp(int q) { return Q - 1 - q; }
    __host__ __device__ static constexpr double w1(int e) { return e == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr double w(int q) { return w1(ex(q)) * w1(ey(q)) * w1(ez(q)); }
};

}  // namespace dugks
