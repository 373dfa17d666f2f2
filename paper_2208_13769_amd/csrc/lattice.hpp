// lattice.hpp -- D2Q9 lattice in lattice units and precision traits.
//
// Lattice units: dX = dt = rho0 = 1, lattice speed c = 1 and C_s^2 = 1/3
// (the time step is fixed by dt = dX / (sqrt(3) C_s), Sec. 7). Velocity order
// of this implementation:
//   0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
// Weights: 4/9 for the rest velocity, 1/9 for the axis links, 1/36 for the
// diagonals (the standard D2Q9 set of Sec. 3).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// ---------------------------------------------------------------- precision

// TF: population storage, TU: displacement storage and accumulator,
// TJ: momentum storage, TC: arithmetic.
template <class TF_, class TU_, class TJ_, class TC_>
struct Prec {
    using TF = TF_;
    using TU = TU_;
    using TJ = TJ_;
    using TC = TC_;
};
using PrecF64 = Prec<double, double, double, double>;
using PrecF32 = Prec<float, float, float, float>;
using PrecF16 = Prec<__half, double, float, float>;
using PrecBF16 = Prec<__hip_bfloat16, double, float, float>;

// Populations in 16-bit storage are kept multiplied by a per-plate power of
// two so that their range sits well inside the format; 32/64-bit storage is
// unscaled.
template <class TF>
struct FStore;

template <>
struct FStore<double> {
    __device__ static double load(const double *p, size_t i, double) { return p[i]; }
    __device__ static double cvt(double v, double) { return v; }
    __device__ static double roundtrip(double v, double, double) { return v; }
    __device__ static void store(double *p, size_t i, double v, double) { p[i] = v; }
};
template <>
struct FStore<float> {
    __device__ static float load(const float *p, size_t i, float) { return p[i]; }
    __device__ static float cvt(float v, float) { return v; }
    __device__ static float roundtrip(float v, float, float) { return v; }
    __device__ static void store(float *p, size_t i, float v, float) { p[i] = v; }
};
template <>
struct FStore<__half> {
    __device__ static float load(const __half *p, size_t i, float inv_scale)
    {
        return __half2float(p[i]) * inv_scale;
    }
    __device__ static float cvt(__half v, float inv_scale) { return __half2float(v) * inv_scale; }
    // the value a store followed by a load gives back
    __device__ static float roundtrip(float v, float scale, float inv_scale)
    {
        return __half2float(__float2half_rn(v * scale)) * inv_scale;
    }
    __device__ static void store(__half *p, size_t i, float v, float scale)
    {
        p[i] = __float2half_rn(v * scale);
    }
};
template <>
struct FStore<__hip_bfloat16> {
    __device__ static float load(const __hip_bfloat16 *p, size_t i, float inv_scale)
    {
        return __bfloat162float(p[i]) * inv_scale;
    }
    __device__ static float cvt(__hip_bfloat16 v, float inv_scale) { return __bfloat162float(v) * inv_scale; }
    __device__ static float roundtrip(float v, float scale, float inv_scale)
    {
        return __bfloat162float(__float2bfloat16(v * scale)) * inv_scale;
    }
    __device__ static void store(__hip_bfloat16 *p, size_t i, float v, float scale)
    {
        p[i] = __float2bfloat16(v * scale);
    }
};

// ---------------------------------------------------------------- material

// Reciprocal: the hardware approximation (about 1 ulp) in float, exact
// division in double.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Stress sum K = P(H) + Pbar(H) in lattice units for the plane-strain
// neo-Hooke law (eq. (27)) and the Poisson stress (eq. (15)).
//   P = mu F + c cof F with c = (lam/2 (J^2 - 1) - mu) / J, cof F = J F^-T,
//   Pbar = -mu (H + H^T + tr H I).
// Adding them, the O(1) parts cancel analytically; with d = c + mu =
// (J - 1) (lam/2 (J + 1) + mu) / J and J - 1 = tr H + det H:
//   K11 = d (1 + H22) - 2 mu tr H,   K12 = -d H21,
//   K21 = -d H12,                    K22 = d (1 + H11) - 2 mu tr H.
// This form has no O(1) cancellation, so K stays accurate in float at small
// strain (and is exactly zero for a pure shear u_y(x)). H and K are row-major:
// [0]=11, [1]=12, [2]=21, [3]=22. Returns J.
template <class TC>
__device__ __forceinline__ TC stress_sum(const TC H[4], TC lam, TC mu, TC K[4])
{
    TC tr = H[0] + H[3];
    TC Jm1 = tr + (H[0] * H[3] - H[1] * H[2]);
    TC J = TC(1) + Jm1;
    TC d = Jm1 * (TC(0.5) * lam * (J + TC(1)) + mu) * recip(J);
    TC m2tr = TC(2) * mu * tr;
    K[0] = d * (TC(1) + H[3]) - m2tr;
    K[1] = -d * H[2];
    K[2] = -d * H[1];
    K[3] = d * (TC(1) + H[0]) - m2tr;
    return J;
}

// First Piola-Kirchhoff stress alone, P = mu F + c cof F (lattice units).
template <class TC>
__device__ __forceinline__ TC piola(const TC H[4], TC lam, TC mu, TC P[4])
{
    TC F11 = TC(1) + H[0], F12 = H[1], F21 = H[2], F22 = TC(1) + H[3];
    TC J = F11 * F22 - F12 * F21;
    TC c = (TC(0.5) * lam * (J * J - TC(1)) - mu) / J;
    P[0] = mu * F11 + c * F22;
    P[1] = mu * F12 - c * F21;
    P[2] = mu * F21 - c * F12;
    P[3] = mu * F22 + c * F11;
    return J;
}

// Boundary-rule codes of the y edges (kept in step with lbm_bc).
enum : int { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_NEUMANN = 2 };

}  // namespace lbm
