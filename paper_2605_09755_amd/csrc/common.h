// Device helpers shared by the HIP kernels of the range finder (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RF_DEV __device__ __forceinline__

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

namespace rf {

// Global-memory pointers.  Kernels that take their arguments from a device array
// (the grouped and batched ones) would otherwise access memory through flat
// instructions, whose waits also cover LDS operations; bodies take these types and
// callers cast the pointers they hold.
// (the host pass, which never runs these bodies, sees plain pointers)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gptr = T __attribute__((address_space(1)))*;
#else
template <class T>
using gptr = T*;
#endif
template <class T>
RF_DEV gptr<const T> as_global(const void* p) {
  return (gptr<const T>)p;
}
template <class T>
RF_DEV gptr<T> as_global_w(void* p) {
  return (gptr<T>)p;
}


// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------------
struct u32x4 { uint32_t x, y, z, w; };

RF_DEV u32x4 philox(uint64_t index, uint32_t stream, uint32_t b, uint64_t seed) {
  uint32_t c0 = (uint32_t)index, c1 = (uint32_t)(index >> 32), c2 = stream, c3 = b;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

// ---- bfloat16 / fp8 conversions ----------------------------------------------
RF_DEV uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
RF_DEV float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Hardware forms of the two conversions, checked on gfx950 to give the same bits
// as f32_to_bf16_rne (all non-NaN inputs of a 2^20 random sample, ties included) and
// as fp8e4m3_to_f32 (all 256 codes):
// two floats -> packed BF16 (round to nearest even), one v_cvt_pk_bf16_f32
typedef float rf_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 rf_bf16x2 __attribute__((ext_vector_type(2)));
RF_DEV uint32_t pk_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((rf_f32x2){a, b}, rf_bf16x2));
}
// the four OCP e4m3 codes in the bytes of w -> floats, two v_cvt_pk_f32_fp8
RF_DEV void fp8x4_to_f32(uint32_t w, float* o) {
  const rf_f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false), hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
  o[0] = lo.x; o[1] = lo.y; o[2] = hi.x; o[3] = hi.y;
}

// OCP FP8 E4M3 (bias 7, no infinities, max 448, 0x7f/0xff = NaN) -> float
RF_DEV float fp8e4m3_to_f32(uint32_t v) {
  uint32_t s = (v & 0x80u) << 24, e = (v >> 3) & 0xfu, m = v & 0x7u;
  float r;
  if (e == 0) r = (float)m * 0.001953125f;                 // subnormal: m * 2^-9
  else if (e == 15 && m == 7) return __uint_as_float(0x7fc00000u);
  else r = __uint_as_float(((e + 120u) << 23) | (m << 20));
  return __uint_as_float(__float_as_uint(r) | s);
}

// ---- reductions ----------------------------------------------------------------
RF_DEV float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
RF_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
RF_DEV float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
RF_DEV double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace rf
