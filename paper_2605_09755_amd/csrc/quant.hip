// Storage forms of A for the precision workload: FP32 -> BF16 (round to nearest,
// ties to even) and FP32 -> OCP FP8 e4m3 with one FP32 scale per 128 x 128 block.
//
// The paper fixes no storage format; these are the forms the mixed-precision
// products read (GEMM dtypes 2 and 6, sketch dtypes 2 and 3).  Both kernels read
// A once (HBM-bound: 4 bytes in, 2 or 1 byte out per element).
//
// e4m3 (OCP 8-bit floating point, E4M3): value = (-1)^s 2^(e-7) (1 + m/8) for
// e >= 1, 2^-6 m/8 for e = 0; S.1111.111 is NaN, no infinities; the largest
// finite magnitude is 448 (code 0x7e).  Block scale = amax / 448 computed in
// FP64 and rounded to FP32 (1 for an all-zero block); each element is divided
// by its block scale in FP64 and rounded to the nearest e4m3 value, ties to the
// even code, magnitudes above 448 saturating to 448.  Non-finite inputs encode
// as NaN and are left out of the block maximum.
#include "common.h"
#include "kernels.h"

namespace rf {

__global__ __launch_bounds__(256) void k_quant_bf16(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                     int64_t lda, uint16_t* __restrict__ out, int64_t ldo) {
  const int64_t r = blockIdx.y;
  for (int64_t c = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4; c < cols; c += (int64_t)gridDim.x * 1024) {
    const float* src = A + r * lda + c;
    uint16_t* dst = out + r * ldo + c;
    if (c + 4 <= cols) {
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = __builtin_nontemporal_load(src + e);
#pragma unroll
      for (int e = 0; e < 4; ++e) dst[e] = f32_to_bf16_rne(v[e]);
    } else {
      for (int64_t e = 0; c + e < cols; ++e) dst[e] = f32_to_bf16_rne(src[e]);
    }
  }
}

// Nearest e4m3 code of x (|x| already divided by the block scale), ties to even.
RF_DEV uint8_t e4m3_rne(double x) {
  const uint8_t sgn = x < 0.0 ? 0x80 : 0x00;  // -0 encodes as +0
  double a = fabs(x);
  if (!isfinite(a)) return 0x7f | sgn;  // NaN and +-Inf: no e4m3 value represents them
  if (a >= 448.0) return 0x7e | sgn;
  if (a < 0.015625) {  // below 2^-6: subnormal grid of 2^-9
    const double q = rint(a * 512.0);  // exact scaling; rint rounds half to even
    return (uint8_t)((int)q) | sgn;    // q = 8 is the smallest normal, code 0x08
  }
  int e;
  (void)frexp(a, &e);  // a = f 2^e, f in [1/2, 1): a in [2^(e-1), 2^e)
  const int E = e - 1;  // a in [2^E, 2^(E+1)), E in [-6, 8]
  const double q = rint(ldexp(a, 3 - E));  // mantissa grid of 2^(E-3): q in [8, 16]
  int qi = (int)q, Ei = E;
  if (qi == 16) {
    qi = 8;
    ++Ei;
  }
  const int code = ((Ei + 7) << 3) | (qi - 8);
  return (uint8_t)(code > 0x7e ? 0x7e : code) | sgn;
}

// One workgroup per 128 x 128 block: the block is held in registers (64 values
// per thread), its |max| reduced over the workgroup, then encoded and written.
constexpr int kQB = 128, kQT = 256;

__global__ __launch_bounds__(kQT) void k_quant_fp8_b128(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                        int64_t lda, uint8_t* __restrict__ out, int64_t ldo,
                                                        float* __restrict__ scales, int64_t ldsc) {
  const int64_t r0 = (int64_t)blockIdx.y * kQB, c0 = (int64_t)blockIdx.x * kQB;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 threads x 4 columns cover a block row
  const int64_t c = c0 + tx * 4;
  float v[kQB / 8][4];
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < kQB / 8; ++i) {
    const int64_t r = r0 + ty + 8 * i;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float x = 0.f;
      if (r < rows && c + e < cols) x = __builtin_nontemporal_load(A + r * lda + c + e);
      v[i][e] = x;
      if (isfinite(x)) amax = fmaxf(amax, fabsf(x));
    }
  }
  amax = wave_max(amax);
  __shared__ float red[kQT / 64];
  __shared__ float sc_sh;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = red[0];
    for (int w = 1; w < kQT / 64; ++w) m = fmaxf(m, red[w]);
    const float sc = m > 0.f ? (float)((double)m / 448.0) : 1.f;
    sc_sh = sc;
    scales[blockIdx.y * ldsc + blockIdx.x] = sc;
  }
  __syncthreads();
  const double sc = (double)sc_sh;
#pragma unroll
  for (int i = 0; i < kQB / 8; ++i) {
    const int64_t r = r0 + ty + 8 * i;
    if (r >= rows) continue;
    uint8_t* dst = out + r * ldo + c;
    if (c + 4 <= cols) {
      uint32_t w = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) w |= (uint32_t)e4m3_rne((double)v[i][e] / sc) << (8 * e);
      if ((((uintptr_t)dst) & 3) == 0) {
        *reinterpret_cast<uint32_t*>(dst) = w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[e] = (uint8_t)(w >> (8 * e));
      }
    } else {
      for (int e = 0; c + e < cols; ++e) dst[e] = e4m3_rne((double)v[i][e] / sc);
    }
  }
}

hipError_t launch_quant_bf16(const float* A, int64_t rows, int64_t cols, int64_t lda, uint16_t* out, int64_t ldo,
                             hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  int64_t gx = (cols + 1023) / 1024;
  if (gx > 64) gx = 64;
  for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
    const int64_t nr = rows - r0 < 65535 ? rows - r0 : 65535;
    hipLaunchKernelGGL(k_quant_bf16, dim3((unsigned)gx, (unsigned)nr), dim3(256), 0, st, A + r0 * lda, nr, cols, lda,
                       out + r0 * ldo, ldo);
  }
  return hipGetLastError();
}

hipError_t launch_quant_fp8_b128(const float* A, int64_t rows, int64_t cols, int64_t lda, uint8_t* out, int64_t ldo,
                                 float* scales, hipStream_t st) {
  if (rows == 0 || cols == 0) return hipSuccess;
  const int64_t bx = (cols + kQB - 1) / kQB, by = (rows + kQB - 1) / kQB;
  if (by > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_quant_fp8_b128, dim3((unsigned)bx, (unsigned)by), dim3(kQT), 0, st, A, rows, cols, lda, out,
                     ldo, scales, bx);
  return hipGetLastError();
}

}  // namespace rf

namespace rf {

// ---- Q in the operand form of the FP8 product A^T Q ----------------------------------
// Q (m x k FP32, ld) -> e4m3 codes with one power-of-two (E8M0) scale per 32 rows and
// column, the codes written in the order the 32x32x64 FP8 MFMA takes its B operand:
//   codes[st][jb][ch][p][lane][e] (st < ceil(m/128), jb < qf8_col_blocks(k), ch, p < 2,
//   lane < 64, e < 16) holds row 128 st + 64 ch + 32 p + 16 (lane / 32) + e, column
//   32 jb + lane % 32;
//   scales[st][jb][lane][ch] (bytes) holds the scale of rows 128 st + 64 ch +
//   32 (lane / 32) + [0, 32), column 32 jb + lane % 32.
// Scale of a 32-row block = the smallest 2^e (-127 <= e <= 127) with 448 2^e >= its
// largest finite |q| (2^-127 for an all-zero block); each element is multiplied by
// 2^-e (exact) and rounded to the nearest e4m3 value, ties to even, saturating at 448;
// non-finite elements encode as NaN.  Rows >= m and columns >= k encode as 0.
RF_DEV int e8m0_exponent(float amax) {
  if (!(amax > 0.f)) return -127;
  const double a = (double)amax;
  int e;
  (void)frexp(a / 448.0, &e);  // a / 448 in [2^(e-1), 2^e)
  // step to the smallest e with 448 2^e >= a (the division above may round)
  while (e > -127 && ldexp(448.0, e - 1) >= a) --e;
  while (e < 127 && ldexp(448.0, e) < a) ++e;
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}

__global__ __launch_bounds__(256) void k_quant_q_fp8(const float* __restrict__ Q, int64_t m, int64_t k, int64_t ldq,
                                                     int njb, uint8_t* __restrict__ codes,
                                                     uint8_t* __restrict__ scales) {
  // thread: one column j and one 32-row block rb
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t rb = blockIdx.y;
  if (j >= (int64_t)njb * 32) return;
  float v[32];
  float amax = 0.f;
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const int64_t row = rb * 32 + r;
    const float x = (row < m && j < k) ? Q[row * ldq + j] : 0.f;
    v[r] = x;
    if (isfinite(x)) amax = fmaxf(amax, fabsf(x));
  }
  const int e = e8m0_exponent(amax);
  const int64_t st = rb >> 2;
  const int ch = (int)((rb >> 1) & 1), p = (int)(rb & 1), jb = (int)(j >> 5), jl = (int)(j & 31);
  uint8_t* base = codes + ((((st * njb + jb) * 2 + ch) * 2 + p) * 64) * 16;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t x = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) x |= (uint32_t)e4m3_rne(ldexp((double)v[16 * h + 4 * q + b], -e)) << (8 * b);
      w[q] = x;
    }
    *reinterpret_cast<uint4*>(base + (32 * h + jl) * 16) = make_uint4(w[0], w[1], w[2], w[3]);
  }
  scales[((st * njb + jb) * 64 + 32 * p + jl) * 2 + ch] = (uint8_t)(e + 127);
}

int qf8_col_blocks(int64_t k) { return (int)((k + 255) / 256) * 8; }
size_t qf8_code_bytes(int64_t m, int64_t k) { return (size_t)((m + 127) / 128) * qf8_col_blocks(k) * 4096; }
size_t qf8_scale_bytes(int64_t m, int64_t k) { return (size_t)((m + 127) / 128) * qf8_col_blocks(k) * 128; }

hipError_t launch_quant_q_fp8(const float* Q, int64_t m, int64_t k, int64_t ldq, uint8_t* codes, uint8_t* scales,
                              hipStream_t st) {
  if (m == 0 || k == 0) return hipSuccess;
  const int njb = qf8_col_blocks(k);
  const int64_t nrb = (m + 127) / 128 * 4;  // 32-row blocks, padded to whole 128-row stages
  if (nrb > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_quant_q_fp8, dim3((unsigned)((njb * 32 + 255) / 256), (unsigned)nrb), dim3(256), 0, st, Q, m,
                     k, ldq, njb, codes, scales);
  return hipGetLastError();
}

}  // namespace rf
