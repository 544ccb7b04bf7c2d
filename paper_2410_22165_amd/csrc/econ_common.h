// econ_common.h -- internal helpers of the gfx950 economy library (not part
// of the public C ABI): error plumbing, the counter-based generator, wave
// and block primitives.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "econ_mi355x.h"

namespace econ {

// ---------------------------------------------------------------------------
// error plumbing: every entry point returns an EJ_* code; the last HIP error
// is kept per thread for ej_last_hip_error().
// ---------------------------------------------------------------------------
void set_last_hip_error(hipError_t e);

#define EJ_HIP(call)                                   \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) {                        \
            ::econ::set_last_hip_error(_e);            \
            return EJ_EHIP;                            \
        }                                              \
    } while (0)

#define EJ_LAUNCH_CHECK()                              \
    do {                                               \
        hipError_t _e = hipGetLastError();             \
        if (_e != hipSuccess) {                        \
            ::econ::set_last_hip_error(_e);            \
            return EJ_EHIP;                            \
        }                                              \
    } while (0)

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11), host and device.  Keys are
// (seed, purpose); counters are four 64-bit words chosen per purpose.
// ---------------------------------------------------------------------------
enum : uint32_t { PURPOSE_SKILL = 1, PURPOSE_ENV = 2, PURPOSE_ACT = 3, PURPOSE_GOV = 4, PURPOSE_SAMPLE = 5 };

struct u64x4 {
    uint64_t x, y, z, w;
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
#endif
}

__host__ __device__ inline u64x4 philox(uint64_t seed, uint32_t purpose, uint64_t c0, uint64_t c1, uint64_t c2,
                                        uint64_t c3)
{
    uint64_t k0 = seed, k1 = purpose;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        uint64_t hi0 = mulhi64(m0, c0), lo0 = m0 * c0;
        uint64_t hi1 = mulhi64(m1, c2), lo1 = m1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    return u64x4{c0, c1, c2, c3};
}

__host__ __device__ inline uint64_t word_of(const u64x4& v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// round-to-nearest-even float -> bfloat16 bits
__host__ __device__ inline uint16_t f32_to_bf16(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t b)
{
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)(threadIdx.x & 63u); }

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ inline T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

template <typename T>
__device__ inline T wave_min(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// inclusive prefix sum across the 64 lanes
template <typename T>
__device__ inline T wave_inclusive_scan(T v)
{
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

}  // namespace econ
