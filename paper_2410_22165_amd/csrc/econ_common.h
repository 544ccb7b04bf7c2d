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
enum : uint32_t {
    PURPOSE_SKILL = 1,
    PURPOSE_ENV = 2,
    PURPOSE_ACT = 3,
    PURPOSE_GOV = 4,
    PURPOSE_SAMPLE = 5,
    PURPOSE_GOV_SAMPLE = 6
};

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

// round-to-nearest-even float -> bfloat16 bits (the device uses the gfx950
// conversion instruction; the host spells the rounding out)
__host__ __device__ inline uint16_t f32_to_bf16(float f)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
#else
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
#endif
}

__host__ __device__ inline float bf16_to_f32(uint16_t b)
{
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------
// device arrays read with 16-byte vector loads must be 16-byte aligned
__host__ inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

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

// ---------------------------------------------------------------------------
// DPP (data-parallel primitives inside a 16-lane row): no LDS round trip.
// Row = lanes 16r .. 16r + 15 of the wave.
// ---------------------------------------------------------------------------
enum : int {
    DPP_XOR1 = 0xB1,        // quad_perm(1, 0, 3, 2)
    DPP_XOR2 = 0x4E,        // quad_perm(2, 3, 0, 1)
    DPP_ROW_SHR1 = 0x111,
    DPP_ROW_SHR2 = 0x112,
    DPP_ROW_SHR4 = 0x114,
    DPP_ROW_SHR8 = 0x118,
    DPP_ROW_MIRROR = 0x140,
    DPP_ROW_HALF_MIRROR = 0x141,
};

template <int CTRL>
__device__ inline float dpp_f(float v, float fill = 0.f)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, fill),
                                                                 __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline int dpp_i(int v, int fill = 0)
{
    return __builtin_amdgcn_update_dpp(fill, v, CTRL, 0xF, 0xF, false);
}

// Workgroup barrier that orders LDS only: outstanding global loads and
// stores stay in flight across it (a full __syncthreads waits for them).
// For threads that communicate through LDS alone.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// all-reduce over the 16 lanes of each row
__device__ inline float row16_sum(float v)
{
    v += dpp_f<DPP_XOR1>(v);
    v += dpp_f<DPP_XOR2>(v);
    v += dpp_f<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_f<DPP_ROW_MIRROR>(v);
    return v;
}
__device__ inline float row16_max(float v)
{
    v = fmaxf(v, dpp_f<DPP_XOR1>(v));
    v = fmaxf(v, dpp_f<DPP_XOR2>(v));
    v = fmaxf(v, dpp_f<DPP_ROW_HALF_MIRROR>(v));
    v = fmaxf(v, dpp_f<DPP_ROW_MIRROR>(v));
    return v;
}
__device__ inline int row16_min_i(int v)
{
    v = min(v, dpp_i<DPP_XOR1>(v));
    v = min(v, dpp_i<DPP_XOR2>(v));
    v = min(v, dpp_i<DPP_ROW_HALF_MIRROR>(v));
    v = min(v, dpp_i<DPP_ROW_MIRROR>(v));
    return v;
}
__device__ inline int row16_max_i(int v)
{
    v = max(v, dpp_i<DPP_XOR1>(v));
    v = max(v, dpp_i<DPP_XOR2>(v));
    v = max(v, dpp_i<DPP_ROW_HALF_MIRROR>(v));
    v = max(v, dpp_i<DPP_ROW_MIRROR>(v));
    return v;
}
__device__ inline int row16_sum_i(int v)
{
    v += dpp_i<DPP_XOR1>(v);
    v += dpp_i<DPP_XOR2>(v);
    v += dpp_i<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_i<DPP_ROW_MIRROR>(v);
    return v;
}
// inclusive prefix sum inside each 16-lane row
__device__ inline float row16_scan(float v)
{
    v += dpp_f<DPP_ROW_SHR1>(v);
    v += dpp_f<DPP_ROW_SHR2>(v);
    v += dpp_f<DPP_ROW_SHR4>(v);
    v += dpp_f<DPP_ROW_SHR8>(v);
    return v;
}
__device__ inline int row16_scan_i(int v)
{
    v += dpp_i<DPP_ROW_SHR1>(v);
    v += dpp_i<DPP_ROW_SHR2>(v);
    v += dpp_i<DPP_ROW_SHR4>(v);
    v += dpp_i<DPP_ROW_SHR8>(v);
    return v;
}

// sums / maxima over the 4 lanes of a quad
__device__ inline float quad_sum(float v)
{
    v += dpp_f<DPP_XOR1>(v);
    v += dpp_f<DPP_XOR2>(v);
    return v;
}
__device__ inline float quad_max(float v)
{
    v = fmaxf(v, dpp_f<DPP_XOR1>(v));
    v = fmaxf(v, dpp_f<DPP_XOR2>(v));
    return v;
}
__device__ inline int quad_min_i(int v)
{
    v = min(v, dpp_i<DPP_XOR1>(v));
    v = min(v, dpp_i<DPP_XOR2>(v));
    return v;
}
__device__ inline int quad_max_i(int v)
{
    v = max(v, dpp_i<DPP_XOR1>(v));
    v = max(v, dpp_i<DPP_XOR2>(v));
    return v;
}
// inclusive prefix sum over the 4 lanes of a quad (q = lane % 4)
__device__ inline float quad_scan(float v, int q)
{
    const float t1 = dpp_f<DPP_ROW_SHR1>(v);
    v += q >= 1 ? t1 : 0.f;
    const float t2 = dpp_f<DPP_ROW_SHR2>(v);
    v += q >= 2 ? t2 : 0.f;
    return v;
}

// wave-wide (64-lane) versions: rows first, then the four row results
__device__ inline int wave_sum_i(int v)
{
    v = row16_sum_i(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
           __builtin_amdgcn_readlane(v, 48);
}
__device__ inline int wave_max_i(int v)
{
    v = row16_max_i(v);
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline int wave_min_i(int v)
{
    v = row16_min_i(v);
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline int wave_scan_i(int v)
{
    v = row16_scan_i(v);
    const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31),
              t2 = __builtin_amdgcn_readlane(v, 47);
    const int row = lane_id() >> 4;
    return v + (row >= 1 ? t0 : 0) + (row >= 2 ? t1 : 0) + (row >= 3 ? t2 : 0);
}

}  // namespace econ
