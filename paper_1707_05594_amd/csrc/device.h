// Device-side helpers shared by the HIP sources of libtucker (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// bfloat16 is carried as its 16-bit pattern.
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}
// Round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T>
struct Elem;
template <>
struct Elem<float> {
  __device__ __forceinline__ static float to_f32(float v) { return v; }
  __device__ __forceinline__ static double to_f64(float v) { return (double)v; }
};
template <>
struct Elem<double> {
  __device__ __forceinline__ static float to_f32(double v) { return (float)v; }
  __device__ __forceinline__ static double to_f64(double v) { return v; }
};
template <>
struct Elem<uint16_t> {
  __device__ __forceinline__ static float to_f32(uint16_t v) { return bf16_to_f32(v); }
  __device__ __forceinline__ static double to_f64(uint16_t v) { return (double)bf16_to_f32(v); }
};
// IEEE half storage (TK_F16): every value is exact in FP32
template <>
struct Elem<_Float16> {
  __device__ __forceinline__ static float to_f32(_Float16 v) { return (float)v; }
  __device__ __forceinline__ static double to_f64(_Float16 v) { return (double)(float)v; }
};

typedef unsigned int u2v __attribute__((ext_vector_type(2)));

// Four consecutive elements starting at a 4-element-aligned index, as FP32.
// NT: non-temporal (streaming) load, for data read once.
template <bool NT = false>
__device__ __forceinline__ f4 load4_f32(const float* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
  else
    return *reinterpret_cast<const f4*>(p);
}
template <bool NT = false>
__device__ __forceinline__ f4 load4_f32(const uint16_t* p) {
  u2v v;
  if constexpr (NT)
    v = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
  else
    v = *reinterpret_cast<const u2v*>(p);
  f4 r;
  r[0] = __uint_as_float(v[0] << 16);
  r[1] = __uint_as_float(v[0] & 0xFFFF0000u);
  r[2] = __uint_as_float(v[1] << 16);
  r[3] = __uint_as_float(v[1] & 0xFFFF0000u);
  return r;
}
template <bool NT = false>
__device__ __forceinline__ f4 load4_f32(const _Float16* p) {
  u2v v;
  if constexpr (NT)
    v = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
  else
    v = *reinterpret_cast<const u2v*>(p);
  f4 r;
  r[0] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[0] & 0xFFFFu));
  r[1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[0] >> 16));
  r[2] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[1] & 0xFFFFu));
  r[3] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[1] >> 16));
  return r;
}

// A pointer read from device memory (a descriptor table) is generic to the
// compiler, which then emits flat loads and stores: those count against the
// LDS wait counter too, so every wait for an LDS read also waits for the
// memory loads in flight.  All device buffers live in the global address
// space; rebuilding the pointer there from its integer value lets the
// compiler use global instructions (a plain cast there and back is folded
// away before the address space is inferred).
template <typename T>
__device__ __forceinline__ T* global_ptr(T* p) {
  typedef __attribute__((address_space(1))) T GT;
  return (T*)(GT*)(uintptr_t)p;
}

// Four consecutive elements as loaded (FP32: four floats; 2-byte types: two
// 32-bit words), and their conversion to FP32: lets a pipeline hold loaded
// rows in their storage width until use.
template <typename T>
struct Raw4 {
  typedef u2v type;
};
template <>
struct Raw4<float> {
  typedef f4 type;
};
template <bool NT = false, typename T>
__device__ __forceinline__ typename Raw4<T>::type load4_raw(const T* p) {
  if constexpr (sizeof(T) == 4) {
    return load4_f32<NT>(p);
  } else {
    static_assert(sizeof(T) == 2, "4- or 2-byte element types only");
    if constexpr (NT)
      return __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
    else
      return *reinterpret_cast<const u2v*>(p);
  }
}
template <typename T>
__device__ __forceinline__ f4 raw4_to_f32(typename Raw4<T>::type v);
template <>
__device__ __forceinline__ f4 raw4_to_f32<float>(f4 v) {
  return v;
}
template <>
__device__ __forceinline__ f4 raw4_to_f32<uint16_t>(u2v v) {
  f4 r;
  r[0] = __uint_as_float(v[0] << 16);
  r[1] = __uint_as_float(v[0] & 0xFFFF0000u);
  r[2] = __uint_as_float(v[1] << 16);
  r[3] = __uint_as_float(v[1] & 0xFFFF0000u);
  return r;
}
template <>
__device__ __forceinline__ f4 raw4_to_f32<_Float16>(u2v v) {
  f4 r;
  r[0] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[0] & 0xFFFFu));
  r[1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[0] >> 16));
  r[2] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[1] & 0xFFFFu));
  r[3] = (float)__builtin_bit_cast(_Float16, (uint16_t)(v[1] >> 16));
  return r;
}

// Wave-level sum (64 lanes) of a double, result valid in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace tk
