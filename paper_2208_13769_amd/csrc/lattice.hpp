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
using PrecF32U64 = Prec<float, double, float, float>;

// ---------------------------------------------------------------- rounding

// Stochastic rounding of 16-bit population stores draws its random bits from
// a counter-based hash: the integer mixer "lowbias32" (C. Wellons, 2018:
// xorshift 16, multiply 0x7feb352d, xorshift 15, multiply 0x846ca68b,
// xorshift 16), a bijection of 32-bit words. The counter is (site index,
// population pair) and the key is derived from the plate's seed and the index
// of the state being written, so the bits of a stored value do not depend on
// the block, launch or batch that computes it.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// key of the state with index `state` (the step count after the update)
__host__ __device__ __forceinline__ uint32_t sr_key(unsigned long long seed, long long state)
{
    const uint32_t s = mix32((uint32_t)state ^ mix32((uint32_t)((unsigned long long)state >> 32) + 0x9e3779b9u));
    return mix32(s ^ (uint32_t)seed) ^ mix32((uint32_t)(seed >> 32) ^ s);
}

// 32 random bits for populations 2q and 2q+1 (q = 0..4) of a site: the low
// half word rounds the first, the high half word the second.
__device__ __forceinline__ uint32_t sr_bits(uint32_t key, uint32_t site, int q)
{
    return mix32((site * 5u + (uint32_t)q) ^ key);
}

// x rounded to binary16 up or down (toward or away from zero) with
// probability given by its distance to the two neighbours, using the low 13
// bits of r: adding r below the 13 dropped mantissa bits of |x| and then
// truncating carries into the kept bits exactly in that fraction of the
// 2^13 equally likely values. Applies to the normal binary16 range; smaller
// magnitudes (below 2^-14, far under the scaled population range) and
// non-finite values round to nearest.
__device__ __forceinline__ __half half_sr(float x, uint32_t r)
{
    const uint32_t b = __float_as_uint(x);
    const uint32_t mag = b & 0x7fffffffu;
    if (mag >= 0x38800000u && mag < 0x477fe000u) {  // [2^-14, 65504)
        const uint32_t m = mag + (r & 0x1fffu);
        const unsigned short h = (unsigned short)(((b >> 16) & 0x8000u) | ((m >> 13) - (112u << 10)));
        return __ushort_as_half(h);
    }
    return __float2half_rn(x);
}

// the same for bfloat16 with the low 16 bits of r (16 dropped bits); exact
// for every finite magnitude up to the largest bfloat16
__device__ __forceinline__ __hip_bfloat16 bf16_sr(float x, uint32_t r)
{
    const uint32_t b = __float_as_uint(x);
    const uint32_t mag = b & 0x7fffffffu;
    if (mag < 0x7f7f0000u) {
        const uint32_t m = mag + (r & 0xffffu);
        const unsigned short h = (unsigned short)(((b >> 16) & 0x8000u) | (m >> 16));
        return __ushort_as_bfloat16(h);
    }
    return __float2bfloat16(x);
}

// Populations in 16-bit storage are kept multiplied by a per-plate power of
// two so that their range sits well inside the format, and as deviations
// from a reference equilibrium of the same state (ref_eq below,
// kDeviation); 32/64-bit storage holds the populations themselves, unscaled.
template <class TF>
struct FStore;

template <>
struct FStore<double> {
    __device__ static double load(const double *p, size_t i, double) { return p[i]; }
    __device__ static double cvt(double v, double) { return v; }
    __device__ static double roundtrip(double v, double, double) { return v; }
    __device__ static void store(double *p, size_t i, double v, double) { p[i] = v; }
    __device__ static double conv(double v, double) { return v; }
    static constexpr bool kStochastic = false;
    static constexpr bool kDeviation = false;
    __device__ static double roundtrip_sr(double v, double, double, uint32_t) { return v; }
    __device__ static void store_sr(double *p, size_t i, double v, double, uint32_t) { p[i] = v; }
};
template <>
struct FStore<float> {
    __device__ static float load(const float *p, size_t i, float) { return p[i]; }
    __device__ static float cvt(float v, float) { return v; }
    __device__ static float roundtrip(float v, float, float) { return v; }
    __device__ static void store(float *p, size_t i, float v, float) { p[i] = v; }
    __device__ static float conv(float v, float) { return v; }
    static constexpr bool kStochastic = false;
    static constexpr bool kDeviation = false;
    __device__ static float roundtrip_sr(float v, float, float, uint32_t) { return v; }
    __device__ static void store_sr(float *p, size_t i, float v, float, uint32_t) { p[i] = v; }
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
    // the stored value of v, to nearest and stochastically with the random word r
    __device__ static __half conv(float v, float scale) { return __float2half_rn(v * scale); }
    __device__ static __half conv_sr(float v, float scale, uint32_t r) { return half_sr(v * scale, r); }
    static constexpr bool kStochastic = true;
    static constexpr bool kDeviation = true;
    __device__ static float roundtrip_sr(float v, float scale, float inv_scale, uint32_t r)
    {
        return __half2float(half_sr(v * scale, r)) * inv_scale;
    }
    __device__ static void store_sr(__half *p, size_t i, float v, float scale, uint32_t r)
    {
        p[i] = half_sr(v * scale, r);
    }
    // the stored bit pattern, and the value a bit pattern loads as
    __device__ static uint32_t bits(float v, float scale) { return __half_as_ushort(__float2half_rn(v * scale)); }
    __device__ static uint32_t bits_sr(float v, float scale, uint32_t r)
    {
        return __half_as_ushort(half_sr(v * scale, r));
    }
    __device__ static float from_bits(uint32_t b, float inv_scale)
    {
        return __half2float(__ushort_as_half((unsigned short)b)) * inv_scale;
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
    __device__ static __hip_bfloat16 conv(float v, float scale) { return __float2bfloat16(v * scale); }
    __device__ static __hip_bfloat16 conv_sr(float v, float scale, uint32_t r) { return bf16_sr(v * scale, r); }
    static constexpr bool kStochastic = true;
    static constexpr bool kDeviation = true;
    __device__ static float roundtrip_sr(float v, float scale, float inv_scale, uint32_t r)
    {
        return __bfloat162float(bf16_sr(v * scale, r)) * inv_scale;
    }
    __device__ static void store_sr(__hip_bfloat16 *p, size_t i, float v, float scale, uint32_t r)
    {
        p[i] = bf16_sr(v * scale, r);
    }
    __device__ static uint32_t bits(float v, float scale)
    {
        return __bfloat16_as_ushort(__float2bfloat16(v * scale));
    }
    __device__ static uint32_t bits_sr(float v, float scale, uint32_t r)
    {
        return __bfloat16_as_ushort(bf16_sr(v * scale, r));
    }
    __device__ static float from_bits(uint32_t b, float inv_scale)
    {
        return __bfloat162float(__ushort_as_bfloat16((unsigned short)b)) * inv_scale;
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

// Reference equilibrium of deviation storage: f^eq(r, j, Pbar) of eq. (20)
// with the zeroth moment r = -div u (eq. (18)), the momentum j and the
// Poisson stress Pbar = -mu (H + H^T + tr H I) (eq. (15)), all from the
// stored state of one site and its central-difference gradient H (lattice
// units, where mu = C_s^2 = 1/3 for every material). The populations of a
// smooth field differ from it by their non-equilibrium part and by the
// small gaps between these moments and the populations' own, so storing
// f - ref_eq instead of f shrinks the storage rounding error by that
// ratio. H row-major as in stress_sum.
template <class TC>
__device__ __forceinline__ void ref_eq(const TC H[4], TC jx, TC jy, TC fr[9])
{
    const TC third = TC(1) / TC(3);
    const TC r = -(H[0] + H[3]);
    // A = Pbar - r/3 I
    const TC axx = TC(-2.0 / 3.0) * H[0], ayy = TC(-2.0 / 3.0) * H[3];
    const TC axy = -third * (H[1] + H[2]);
    const TC trA = axx + ayy;
    const TC q0 = -trA * third;
    const TC q13 = axx + q0, q24 = ayy + q0;
    const TC q57 = TC(2) * (trA * third + axy), q68 = TC(2) * (trA * third - axy);
    const TC jx3 = TC(3) * jx, jy3 = TC(3) * jy;
    const TC w0 = TC(4) / TC(9), w1 = TC(1) / TC(9), w5 = TC(1) / TC(36);
    fr[0] = w0 * (r + TC(4.5) * q0);
    const TC b13 = r + TC(4.5) * q13, b24 = r + TC(4.5) * q24;
    const TC b57 = r + TC(4.5) * q57, b68 = r + TC(4.5) * q68;
    fr[1] = w1 * (b13 + jx3);
    fr[3] = w1 * (b13 - jx3);
    fr[2] = w1 * (b24 + jy3);
    fr[4] = w1 * (b24 - jy3);
    fr[5] = w5 * (b57 + (jx3 + jy3));
    fr[7] = w5 * (b57 - (jx3 + jy3));
    fr[6] = w5 * (b68 + (jy3 - jx3));
    fr[8] = w5 * (b68 - (jy3 - jx3));
}

// Boundary-rule codes of the y edges (kept in step with lbm_bc).
enum : int { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_NEUMANN = 2 };

}  // namespace lbm
