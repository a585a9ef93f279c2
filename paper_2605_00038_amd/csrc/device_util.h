// Device helpers shared by the BP, OSD and comparison kernels (gfx950, wave64):
// wave-wide reductions and scans, the lottery's counter-based generator, and
// the error-free fp32 arithmetic that keeps float lambda exact.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbp {

// Orders the wave's LDS accesses before and after this point (one wave's lanes
// run in lockstep; the fences keep the compiler from moving accesses across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the wave's lanes with DPP moves (VALU, no LDS
// crossbar): four shifts within each 16-lane row, then the rows' totals by the
// row broadcasts of lane 15 (into rows 1 and 3) and lane 31 (into rows 2 and 3).
// A lane whose source is outside its row, or whose row is masked off, adds 0.
__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
    (void)lane;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Sum over the wave's lanes, wave-uniform.
__device__ __forceinline__ int wave_sum(int x) {
    return __builtin_amdgcn_readlane(wave_incl_scan(x, 0), 63);
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11): words 0 (returned) and
// 1 (w1) of the block for counter (ctr0, ctr1, 0, 0) under key (k0, 0).  Ten
// rounds of two 64x64 -> 128-bit products with the published multipliers, the
// key bumped by the published Weyl increments between rounds.  Called with
// wave-uniform arguments it runs on the scalar unit.
__device__ __forceinline__ uint64_t philox_word01(uint64_t k0, uint64_t ctr0, uint64_t ctr1, uint64_t &w1) {
    uint64_t x0 = ctr0, x1 = ctr1, x2 = 0, x3 = 0, ka = k0, kb = 0;
#pragma unroll 1
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0hi = __umul64hi(0xD2E7470EE14C6C93ULL, x0), p0lo = 0xD2E7470EE14C6C93ULL * x0;
        const uint64_t p1hi = __umul64hi(0xCA5A826395121157ULL, x2), p1lo = 0xCA5A826395121157ULL * x2;
        const uint64_t n0 = p1hi ^ x1 ^ ka, n2 = p0hi ^ x3 ^ kb;
        x0 = n0;
        x1 = p1lo;
        x2 = n2;
        x3 = p0lo;
        ka += 0x9E3779B97F4A7C15ULL;
        kb += 0xBB67AE8584CAA73BULL;
    }
    w1 = x1;
    return x0;
}

// Error-free sum of two floats: s + e == a + b exactly (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// The check-node scale applied to a float magnitude, rounded once: sigma_i =
// fl32(1 - 2^-(i+1)) is exact for i <= 23 and 1.0 beyond, and the fma forms
// mag - mag 2^-(i+1) with a single rounding; a constant factor is one product.
__device__ __forceinline__ float scale_float(int scale_mode, float scale_f, int i, float mag) {
    if (scale_mode == 1) return scale_f * mag;
    if (i >= 24) return mag;
    return __builtin_fmaf(-mag, __builtin_ldexpf(1.0f, -(i + 1)), mag);
}

// Hard decision e = [lambda <= 2^-12] on an exact pair lambda = hi + lo (|lo| is
// at most half an ulp of hi, so only hi == threshold needs lo).
__device__ __forceinline__ bool hard_pair(float hi, float lo) {
    constexpr float tau = 1.0f / 4096.0f;
    return hi < tau || (hi == tau && lo <= 0.f);
}

// Q(|lambda|) = floor(|hi + lo| * 2^12) of an exact pair, capped at 4e18 (no
// real lambda comes near; the cap only keeps Q an integer).  Float only: the
// scalings by 2^12 are exact, and when H = |hi| 2^12 is not an integer, H + L
// cannot cross one (|L| is at most half an ulp of H).
__device__ __forceinline__ uint64_t quantized_abs_pair(float hi, float lo) {
    if (hi < 0.f || (hi == 0.f && lo < 0.f)) {
        hi = -hi;
        lo = -lo;
    }
    const float H = hi * 4096.0f, L = lo * 4096.0f;
    if (!(H < 4.0e18f)) return 4000000000000000000ull;
    const float fh = __builtin_floorf(H);
    if (fh == H) return (uint64_t)((int64_t)H + (int64_t)__builtin_floorf(L));  // floor(H + L) = H + floor(L)
    return (uint64_t)fh;
}

}  // namespace lbp
