// Wavefront-level building blocks for line transforms on gfx950: lane
// exchanges (DPP, ds_swizzle, ds_bpermute), the natural-order Walsh-Hadamard
// transform of a line held in one wave (R consecutive values per lane), and
// the index maps between natural and sequency order (Def. 3.1: the sequency
// index b sits at natural position bitrev(gray(b)); odd phases are mirrored,
// Lemma 3.2, which flips the lowest natural bit).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wh2wav_fast {
namespace wave {

__device__ __forceinline__ int lane_id() { return int(__lane_id()); }

template <int D>
__device__ __forceinline__ int xor_i32(int v) {
  if constexpr (D == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (D == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (D < 32) {
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (D << 10));     // bitmask mode, xor D
  } else {
    return __builtin_amdgcn_ds_bpermute((lane_id() ^ 32) << 2, v);
  }
}

template <int D>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(xor_i32<D>(__float_as_int(v)));
}
template <int D>
__device__ __forceinline__ double lane_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_i32<D>(int(b)), hi = xor_i32<D>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__device__ __forceinline__ float shfl_from(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double shfl_from(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, int(b));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(int(b), l), hi = __builtin_amdgcn_readlane(int(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Keeps a value read from LDS at this point of the program.  Before a
// block-wide barrier after which other waves overwrite the same LDS words,
// every value read from them must be pinned: the machine-level passes do not
// treat s_barrier as a memory operation and may otherwise sink an LDS read
// whose result is used only later past the barrier (observed for the last
// staging round of the adjoint column pass, which then read the next phase's
// values).  The empty asm takes the value as an operand, so the read and its
// wait happen before it.
template <typename T>
__device__ __forceinline__ void pin(T& v) {
  asm volatile("" : "+v"(v));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t bitrev_bits(uint32_t x, int bits) { return __brev(x) >> (32 - bits); }
__device__ __forceinline__ uint32_t gray_inverse(uint32_t x) {
  x ^= x >> 1;
  x ^= x >> 2;
  x ^= x >> 4;
  x ^= x >> 8;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ uint32_t natural_of(uint32_t b, uint32_t s, int j) {
  return bitrev_bits(b ^ (b >> 1), j) ^ (s & 1u);
}
__device__ __forceinline__ uint32_t sequency_of(uint32_t k, uint32_t s, int j) {
  return gray_inverse(bitrev_bits(k ^ (s & 1u), j));
}

// ----------------------------------------------------------- vector I/O
template <typename T, int R>
__device__ __forceinline__ void load_line(const T* __restrict__ src, T (&v)[R]) {
  if constexpr (sizeof(T) == 4 && R % 4 == 0) {
    const float4* p = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int c = 0; c < R / 4; ++c) {
      const float4 f = p[c];
      v[4 * c] = f.x, v[4 * c + 1] = f.y, v[4 * c + 2] = f.z, v[4 * c + 3] = f.w;
    }
  } else if constexpr (sizeof(T) == 4 && R % 2 == 0) {
    const float2* p = reinterpret_cast<const float2*>(src);
#pragma unroll
    for (int c = 0; c < R / 2; ++c) {
      const float2 f = p[c];
      v[2 * c] = f.x, v[2 * c + 1] = f.y;
    }
  } else if constexpr (sizeof(T) == 8 && R % 2 == 0) {
    const double2* p = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int c = 0; c < R / 2; ++c) {
      const double2 f = p[c];
      v[2 * c] = f.x, v[2 * c + 1] = f.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = src[c];
  }
}
template <typename T, int R>
__device__ __forceinline__ void store_line(T* __restrict__ dst, const T (&v)[R]) {
  if constexpr (sizeof(T) == 4 && R % 4 == 0) {
    float4* p = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int c = 0; c < R / 4; ++c) p[c] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  } else if constexpr (sizeof(T) == 4 && R % 2 == 0) {
    float2* p = reinterpret_cast<float2*>(dst);
#pragma unroll
    for (int c = 0; c < R / 2; ++c) p[c] = make_float2(v[2 * c], v[2 * c + 1]);
  } else if constexpr (sizeof(T) == 8 && R % 2 == 0) {
    double2* p = reinterpret_cast<double2*>(dst);
#pragma unroll
    for (int c = 0; c < R / 2; ++c) p[c] = make_double2(v[2 * c], v[2 * c + 1]);
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) dst[c] = v[c];
  }
}

template <typename T, int R>
__device__ __forceinline__ void fwht_regs(T (&v)[R]) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if ((i & h) == 0) {
        const T a = v[i], b = v[i + h];
        v[i] = a + b;
        v[i + h] = a - b;
      }
    }
  }
}

template <int D, typename T, int R>
__device__ __forceinline__ void lane_stage(T (&v)[R], int lane) {
  const T sg = (lane & D) ? T(-1) : T(1);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const T p = lane_xor<D>(v[i]);
    v[i] = fma(sg, v[i], p);
  }
}

template <typename T, int R>
__device__ __forceinline__ void fwht_wave(T (&v)[R], int lane) {
  fwht_regs<T, R>(v);
  lane_stage<1>(v, lane);
  lane_stage<2>(v, lane);
  lane_stage<4>(v, lane);
  lane_stage<8>(v, lane);
  lane_stage<16>(v, lane);
  lane_stage<32>(v, lane);
}

}  // namespace wave
}  // namespace wh2wav_fast
