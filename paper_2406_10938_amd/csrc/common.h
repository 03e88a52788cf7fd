// Internal device helpers shared by the library's kernels (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DL_WAVE 64

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Order-preserving map between FP32 and uint32 (total order of finite floats,
// -0 < +0 is irrelevant here because keys only compare).
__device__ __forceinline__ uint32_t dl_f2key(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float dl_key2f(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

__device__ __forceinline__ int dl_lane() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int dl_rank_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t dl_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Lanes of this wave whose 8-bit `digit` equals this lane's, among lanes where
// `valid` holds.
__device__ __forceinline__ uint64_t dl_match8(uint32_t digit, bool valid) {
    uint64_t m = dl_ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t bb = dl_ballot(((digit >> b) & 1u) != 0);
        m &= ((digit >> b) & 1u) ? bb : ~bb;
    }
    return m;
}

// Read a value from lane `src` of this wave.
__device__ __forceinline__ uint32_t dl_shfl_u32(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

template <typename T>
__device__ __forceinline__ T dl_wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t dl_wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ float dl_bf16_to_f32(uint16_t h);
__device__ __forceinline__ uint16_t dl_f32_to_bf16(float f);

// Four consecutive elements p[k..k+3] (zero beyond d).  ALIGNED: d and k are
// multiples of 4 (rows 16-byte aligned), so the four lie all inside the row or
// all beyond it, and one vector load from a clamped offset plus a select
// covers both without a branch (a branch here splits the load stream and
// forces waits at its join).
template <bool ALIGNED>
__device__ __forceinline__ floatx4 load4(const float* __restrict__ p, int k, int d) {
    floatx4 r;
    if (ALIGNED) {
        const bool in = k + 4 <= d;
        const float4 v = *reinterpret_cast<const float4*>(p + (in ? k : 0));
        r[0] = in ? v.x : 0.0f; r[1] = in ? v.y : 0.0f; r[2] = in ? v.z : 0.0f; r[3] = in ? v.w : 0.0f;
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = (k + t < d) ? p[k + t] : 0.0f;
    }
    return r;
}

template <bool ALIGNED>
__device__ __forceinline__ shortx4 load4bf(const uint16_t* __restrict__ p, int k, int d) {
    shortx4 r;
    if (ALIGNED) {
        const bool in = k + 4 <= d;
        uint2 v = *reinterpret_cast<const uint2*>(p + (in ? k : 0));
        if (!in) v = make_uint2(0u, 0u);
        r[0] = (short)(v.x & 0xffff); r[1] = (short)(v.x >> 16);
        r[2] = (short)(v.y & 0xffff); r[3] = (short)(v.y >> 16);
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = (k + t < d) ? (short)p[k + t] : (short)0;
    }
    return r;
}


__device__ __forceinline__ float dl_bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}
// Round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t dl_f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

// Block-wide exclusive prefix of a 0/1 flag over 256 threads; returns the
// prefix and writes the block total to *tot.
__device__ __forceinline__ uint32_t block_flag_prefix(bool f, uint32_t* wtot, uint32_t* tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t msk = dl_ballot(f);
    const uint32_t r = (uint32_t)dl_rank_below(msk);
    if (lane == 0) wtot[wave] = (uint32_t)__popcll(msk);
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) pre += wtot[w];
        all += wtot[w];
    }
    *tot = all;
    __syncthreads();
    return pre + r;
}

// Block-wide exclusive prefix of per-thread counts over 256 threads (all
// lanes active); returns the prefix and writes the block total to *tot.
__device__ __forceinline__ uint32_t block_count_prefix(uint32_t c, uint32_t* wtot, uint32_t* tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = dl_shfl_u32(incl, lane >= o ? lane - o : lane);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) pre += wtot[w];
        all += wtot[w];
    }
    *tot = all;
    __syncthreads();
    return pre + incl - c;
}
