// device_common.h -- device helpers shared by the gfx950 kernels of the CRBM
// sampler: Philox4x32-10, uniforms, guarded Bernoulli decisions, wavefront
// and workgroup reductions, per-chain record layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crbm {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// multiply-xor S-box; the two key words advance by the Weyl constants between
// rounds.  Counter (unit>>2, sweep, chain, tag), key = 64-bit seed.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input XOR in one v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// The same generator for a key that is uniform across the wave: the key is kept
// in two scalar registers and advanced per round at every call, instead of a
// twenty-register schedule that the compiler would hold across the caller's loops.
__device__ __forceinline__ u32x4 philox10_uk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1)
{
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
    return philox10(c0, c1, c2, c3, k0, k1);
}

enum : uint32_t { STREAM_INIT = 0, STREAM_HID = 1, STREAM_VIS = 2, STREAM_MH = 3, STREAM_PT = 4 };

__device__ __forceinline__ uint32_t word_of(const u32x4& r, int w)
{
    return w == 0 ? r.x : (w == 1 ? r.y : (w == 2 ? r.z : r.w));
}

// 53-bit uniform of (stream, index t, chain g): words 0,1 of unit group 0
__device__ __forceinline__ double uniform53(uint64_t seed, uint32_t t, uint32_t g, uint32_t stream)
{
    const u32x4 r = philox10(0u, t, g, stream, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t x = ((uint64_t)r.x << 32) | (uint64_t)r.y;
    return ((double)(x >> 11) + 0.5) * 0x1p-53;
}

// MH uniform of (chain, sweep)
__device__ __forceinline__ double mh_uniform(uint64_t seed, uint32_t t, uint32_t g)
{
    return uniform53(seed, t, g, STREAM_MH);
}

// ---------------------------------------------------------------------------
// Bernoulli decision h = [u < sigmoid(a)], u = (x + 0.5) 2^-32.
// Fast path in float32: with e = exp(-a), u < sigmoid(a)  <=>  u (1 + e) - 1 < 0.
// `dA` bounds |a_f32 - a_exact| (float32 summation of the pre-activation).
// The remaining error of the test value is below
//   dA + |a| 2^-22 + 2^-19
// (argument rounding of exp2, exp2 result, product, float conversion of u),
// so outside that band the float32 sign is the exact one; inside it the
// caller re-evaluates in FP64 (`near` is set).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bernoulli_fast(float a, uint32_t x, float dA, bool& near)
{
    const float u = ((float)x + 0.5f) * 0x1p-32f;
    const float e = __builtin_amdgcn_exp2f(-a * 1.44269504088896341f);
    const float tt = fmaf(u, e, u) - 1.0f;
    const float bound = dA + fabsf(a) * 0x1p-22f + 0x1p-19f;
    near = fabsf(tt) <= bound;
    return tt < 0.0f;
}

__device__ __forceinline__ bool bernoulli_exact(double a, uint32_t x)
{
    const double u = ((double)x + 0.5) * 0x1p-32;
    const double p = 1.0 / (1.0 + exp(-a));
    return u < p;
}

__device__ __forceinline__ double softplus_d(double x)
{
    return (x > 0.0 ? x : 0.0) + log1p(exp(-fabs(x)));
}

__device__ __forceinline__ double log2cosh_d(double x)
{
    const double ax = fabs(x);
    return ax + log1p(exp(-2.0 * ax));
}

// gamma_n = n u / (1 - n u), u = 2^-24: bound factor of n-term float32 sums
__host__ __device__ inline float gamma_f32(int n)
{
    const double nu = (double)n * 0x1p-24;
    return (float)(nu / (1.0 - nu));
}

// ---------------------------------------------------------------------------
// Reductions (wave64)
// ---------------------------------------------------------------------------
// Butterfly over each 32-lane half with ds_swizzle (xor mode: and-mask 31,
// xor-mask X), which takes its lane pattern as an immediate, then the two
// half sums via readlane.  Needs the whole wave active; the result is
// wave-uniform and identical in every lane.
template <int X>
__device__ __forceinline__ int swz_xor(int v)
{
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (X << 10));
}

template <int X>
__device__ __forceinline__ long long swz_xor(long long v)
{
    const int lo = swz_xor<X>((int)(uint32_t)v);
    const int hi = swz_xor<X>((int)(v >> 32));
    return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int X>
__device__ __forceinline__ double swz_xor(double v)
{
    return __longlong_as_double(swz_xor<X>(__double_as_longlong(v)));
}

__device__ __forceinline__ int readlane_t(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ long long readlane_t(long long v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l);
    return (long long)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_t(double v, int l)
{
    return __longlong_as_double(readlane_t(__double_as_longlong(v), l));
}

template <typename Tv>
__device__ __forceinline__ Tv wave_sum(Tv v)
{
    v += swz_xor<16>(v);
    v += swz_xor<8>(v);
    v += swz_xor<4>(v);
    v += swz_xor<2>(v);
    v += swz_xor<1>(v);
    return readlane_t(v, 0) + readlane_t(v, 32);
}

// The same sum for a double through DPP lane moves (VALU, no LDS round trips):
// quad xor 1 and 2, the half-row and row mirrors give every lane its 16-lane
// row sum, then the four row sums are read out.  Needs the whole wave active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// sum over the 16 lanes of a DPP row, in every lane of the row
__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}

__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v = row16_sum(v);
    return (readlane_t(v, 0) + readlane_t(v, 16)) + (readlane_t(v, 32) + readlane_t(v, 48));
}

// Workgroup sum; `red` is LDS scratch of >= nwaves entries.  Every thread
// receives the total.  Contains two barriers.
template <typename Tv>
__device__ __forceinline__ Tv block_sum(Tv v, Tv* red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    Tv s = 0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// Per-chain record (same layout as crbm_chain_stats of the C ABI)
// ---------------------------------------------------------------------------
struct ChainRec {
    long long sweeps, n_acc, n_meas, n_recheck;
    long long sumE, sumE2, sumM, sumAbsM, sumM2;
    long long E;
    double F, S, Ef, Cf;
    double kE, kE2, kCf;
    double F_bound;     // bound on |F - F_exact| of the cached F
    long long n_swap;   // accepted temperature swaps
    double S_bound;     // Kitaev: bound on |S - S_exact| of the cached S (0: Jacobi re-check route)
};
static_assert(sizeof(ChainRec) == 160, "record layout");

}  // namespace crbm
