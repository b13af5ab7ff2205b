// lattice.h -- compile-time description of the D2Q5 / D3Q7 lattices of the
// pseudo-vector lattice-BGK scheme (Section "Lattice BGK formulation").
//
// Velocities: i = 0 rest; i = 1..D move along +axis (i-1); i = D+1..2D move
// along -axis (i-D-1).  In 2D this is the paper's counter-clockwise order
// (1,0), (0,1), (-1,0), (0,-1).
//
// Tensor components: the antisymmetric g_{i,alpha,beta} is stored by its
// independent entries, one per pair p = (alpha < beta): 2D p=0 -> (x,y);
// 3D p=0 -> (x,y), p=1 -> (x,z), p=2 -> (y,z).  gamma(p) is the remaining
// index and sgn(p) = eps_{gamma,alpha,beta}, so that the electric field is
// E_gamma(p) = -sgn(p) Lambda_p (Levi-Civita recovery of the Maxwell section)
// and a source component S_gamma(p) enters pair p as sgn(p) S_gamma.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbem {

template <int D>
struct Lat {
    static constexpr int Q = 2 * D + 1;
    static constexpr int P = D * (D - 1) / 2;
};

__host__ __device__ constexpr int cvel(int D, int i, int a)
{
    return i == 0 ? 0 : (i <= D ? (a == i - 1 ? 1 : 0) : (a == i - D - 1 ? -1 : 0));
}
__host__ __device__ constexpr int opp(int D, int i) { return i == 0 ? 0 : (i <= D ? i + D : i - D); }
// moving axis of velocity i (-1 for rest) and its sign
__host__ __device__ constexpr int vaxis(int D, int i) { return i == 0 ? -1 : (i <= D ? i - 1 : i - D - 1); }
__host__ __device__ constexpr int vsign(int D, int i) { return i == 0 ? 0 : (i <= D ? 1 : -1); }
__host__ __device__ constexpr int pair_a(int D, int p) { return D == 2 ? 0 : (p == 2 ? 1 : 0); }
__host__ __device__ constexpr int pair_b(int D, int p) { return D == 2 ? 1 : (p == 0 ? 1 : 2); }
__host__ __device__ constexpr int pair_g(int D, int p) { return D == 2 ? 2 : (p == 0 ? 2 : (p == 1 ? 1 : 0)); }
__host__ __device__ constexpr int pair_s(int D, int p) { return D == 2 ? 1 : (p == 1 ? -1 : 1); }

// multiply by a compile-time velocity component without a floating multiply
template <typename T>
__host__ __device__ __forceinline__ T cmul(int c, T v)
{
    return c == 0 ? T(0) : (c > 0 ? v : -v);
}

}  // namespace lbem
