// Sketch families of Lemma 3.2 beyond the sparse sign sketch:
//
//  * item 1, dense sub-Gaussian S (n x r1) with independent entries scaled by
//    1/sqrt(r1): Rademacher (+-1, sign = top bit of word x0 of Philox counter
//    i*r1 + j on stream 4) or Gaussian (N(0,1) from the Box-Muller generator on
//    stream 4).  The entries are written unscaled (+-1 is exact in BF16 as well);
//    A S is then a dense product on MFMA with alpha = 1/sqrt(r1).
//  * item 3, the subsampled randomised Hadamard transform S = D H I_{:,P} / sqrt(r1)
//    on n' = the smallest power of two >= n (A padded with zero columns): D = random
//    signs (top bit of x0 of counter j on stream 5), H the Sylvester-Hadamard matrix
//    (entries +-1), P an r1-subset of [0, n') given by the images of 0..r1-1 under a
//    keyed permutation of [0, n') (four Feistel rounds on an even number of bits,
//    round function = x0 of Philox counter (half | round << 32) on stream 6, walked
//    along its cycle until the value is below n'), sorted ascending.
//
// The SRHT pass reads A once: each row is transformed in registers and LDS
// (O(n' log n') adds, FP32) and only the r1 sampled outputs are written.
#include "common.h"
#include "kernels.h"

namespace rf {

constexpr uint32_t kStreamDense = 4, kStreamSrhtD = 5, kStreamSrhtP = 6;

__global__ void k_dense_rademacher(int64_t total, uint64_t seed, uint32_t b, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const u32x4 x = philox((uint64_t)e, kStreamDense, b, seed);
  out[e] = (x.x >> 31) ? -1.f : 1.f;
}

hipError_t launch_dense_sketch(int kind, int64_t n, int r1, uint64_t seed, uint32_t b, float* out, hipStream_t st) {
  const int64_t total = n * (int64_t)r1;
  if (total == 0) return hipSuccess;
  if (kind == 1) {
    hipLaunchKernelGGL(k_dense_rademacher, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, total, seed, b,
                       out);
    return hipGetLastError();
  }
  if (kind == 2) return launch_gaussian(n, r1, seed, kStreamDense, b, out, r1, st);
  return hipErrorInvalidValue;
}

int64_t srht_size(int64_t n) {
  int64_t p = 1;
  while (p < n) p *= 2;
  return p;
}

// ---- SRHT draws: signs d (n' floats +-1) and the sorted subset picks (r1 ints) ----
RF_DEV uint32_t feistel(uint32_t v, int bits, uint64_t seed, uint32_t b) {
  const int h = bits / 2;
  const uint32_t mask = (1u << h) - 1u;
  uint32_t left = (v >> h) & mask, right = v & mask;
#pragma unroll
  for (int rnd = 0; rnd < 4; ++rnd) {
    const uint32_t f = philox((uint64_t)right | ((uint64_t)rnd << 32), kStreamSrhtP, b, seed).x;
    const uint32_t nr = (left ^ f) & mask;
    left = right;
    right = nr;
  }
  return (left << h) | right;
}

constexpr int kSrhtMaxPicks = 8192;  // picks sorted in one workgroup's LDS

__global__ __launch_bounds__(1024) void k_srht_prep(int64_t n2, int r1, int bits, uint64_t seed, uint32_t b,
                                                    float* __restrict__ d, int* __restrict__ picks) {
  for (int64_t j = threadIdx.x; j < n2; j += blockDim.x)
    d[j] = (philox((uint64_t)j, kStreamSrhtD, b, seed).x >> 31) ? -1.f : 1.f;
  __shared__ int key[kSrhtMaxPicks];
  int P = 1;
  while (P < r1) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    int v = 0x7fffffff;  // padding sorts last
    if (i < r1) {
      uint32_t x = feistel((uint32_t)i, bits, seed, b);
      while ((int64_t)x >= n2) x = feistel(x, bits, seed, b);  // cycle walking: ends (a permutation's cycle)
      v = (int)x;
    }
    key[i] = v;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const int a = key[i], c = key[j];
          if (up ? (a > c) : (a < c)) {
            key[i] = c;
            key[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < r1; i += blockDim.x) picks[i] = key[i];
}

hipError_t launch_srht_prep(int64_t n, int r1, uint64_t seed, uint32_t b, float* d, int* picks, hipStream_t st) {
  const int64_t n2 = srht_size(n);
  if (r1 < 1 || r1 > n2 || r1 > kSrhtMaxPicks) return hipErrorInvalidValue;
  int bits = 2;
  while (((int64_t)1 << bits) < n2) ++bits;
  bits += bits & 1;
  hipLaunchKernelGGL(k_srht_prep, dim3(1), dim3(1024), 0, st, n2, r1, bits, seed, b, d, picks);
  return hipGetLastError();
}

// ---- SRHT rows -------------------------------------------------------------------
// One row per iteration of a workgroup of T = n'/E threads.  Mapping A (thread t
// holds elements t + T e, e < E) does the butterflies over element bits >= log2 T
// in registers; a transpose through LDS gives mapping B (thread t holds E t + e),
// which does element bits < log2 E in registers and bits [log2 E, log2 T) with
// lane exchanges inside the wave (T <= 64 E keeps those partners in the same wave).
// The transformed row goes back to LDS and the r1 sampled entries are gathered.
template <typename TIN>
RF_DEV float srht_load(const TIN* __restrict__ row, const float* __restrict__ sc_row, int64_t j) {
  if constexpr (sizeof(TIN) == 4) {
    return __builtin_nontemporal_load(row + j);
  } else if constexpr (sizeof(TIN) == 2) {
    return bf16_to_f32(row[j]);
  } else {
    return fp8e4m3_to_f32(row[j]) * sc_row[j >> 7];
  }
}

RF_DEV int lds_pad(int i) { return i + (i >> 5); }  // one pad word per 32: spreads the strided reads over banks

template <typename TIN, int E>
__global__ __launch_bounds__(1024) void k_srht_rows(const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales,
                                                    int64_t ldsc, int64_t m, int64_t n, int n2, const float* __restrict__ d,
                                                    const int* __restrict__ picks, int r1, float* __restrict__ out,
                                                    int64_t ldo, float scale) {
  extern __shared__ float buf[];
  const int T = blockDim.x, t = threadIdx.x;
  uint32_t dneg = 0;  // bit e: the sign of D at element t + T e is negative (E <= 32)
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = t + T * e;
    if (j < n2 && d[j] < 0.f) dneg |= 1u << e;
  }
  float x[E];
  auto load_row = [&](int64_t i, float* v) {
    const TIN* row = A + i * lda;
    const float* sc = (sizeof(TIN) == 1) ? scales + (i >> 7) * ldsc : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t j = t + (int64_t)T * e;
      const float a = (j < n) ? srht_load<TIN>(row, sc, j) : 0.f;
      v[e] = ((dneg >> e) & 1u) ? -a : a;
    }
  };
  // the next row is loaded while this one is transformed, when the registers
  // allow it (up to 16 values per thread; 32 would spill under 1024 threads)
  constexpr bool kPrefetch = E <= 16;
  int64_t i = blockIdx.x;
  if (kPrefetch && i < m) load_row(i, x);
  for (; i < m; i += gridDim.x) {
    float xn[kPrefetch ? E : 1];
    const int64_t inext = i + gridDim.x;
    if constexpr (kPrefetch) {
      if (inext < m) load_row(inext, xn);  // in flight while this row is transformed
    } else {
      load_row(i, x);
    }
    // mapping A: element bits >= log2 T are the bits of e
#pragma unroll
    for (int s = E / 2; s >= 1; s >>= 1)
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (!(e & s)) {
          const float u = x[e], v = x[e + s];
          x[e] = u + v;
          x[e + s] = u - v;
        }
#pragma unroll
    for (int e = 0; e < E; ++e) buf[lds_pad(t + T * e)] = x[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = buf[lds_pad(E * t + e)];
    // mapping B: element bits < log2 E in registers
#pragma unroll
    for (int s = E / 2; s >= 1; s >>= 1)
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (!(e & s)) {
          const float u = x[e], v = x[e + s];
          x[e] = u + v;
          x[e + s] = u - v;
        }
    // element bits [log2 E, log2 T): partner thread t ^ s, s < 64, inside the wave
    for (int s = 1; s < T / E && (int64_t)s * E < n2; s <<= 1) {  // T / E <= 64
      const bool hi = (t & s) != 0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float o = __shfl_xor(x[e], s, 64);
        x[e] = hi ? (o - x[e]) : (x[e] + o);
      }
    }
    __syncthreads();  // every thread has read its transpose values
#pragma unroll
    for (int e = 0; e < E; ++e) buf[lds_pad(E * t + e)] = x[e];
    __syncthreads();
    float* orow = out + i * ldo;
    for (int jj = t; jj < r1; jj += T) orow[jj] = buf[lds_pad(picks[jj])] * scale;
    __syncthreads();  // the gather is done before the next row overwrites LDS
    if constexpr (kPrefetch) {
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = xn[e];
    }
  }
}

// E and T for n' = 2^L: the smallest power of two E >= max(1, n'/1024) with
// T = n'/E <= 64 E (the lane-exchange stages stay inside one wave); T >= 64.
static void srht_shape(int64_t n2, int& E, int& T) {
  E = 1;
  while (n2 / E > 1024 || n2 / E > 64 * E) E *= 2;
  T = (int)(n2 / E);
  if (T < 64) T = 64;
}

template <typename TIN, int E>
static hipError_t go_srht(const void* A, int64_t lda, const float* scales, int64_t m, int64_t n, int n2, int T,
                          const float* d, const int* picks, int r1, float* out, int64_t ldo, hipStream_t st) {
  const size_t lds = (size_t)(n2 + n2 / 32 + 64) * sizeof(float);
  auto k = k_srht_rows<TIN, E>;
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int per_cu = lds <= 80 * 1024 ? 2 : 1;
  int64_t grid = (int64_t)cus * per_cu * (T <= 256 ? 4 : 1);
  if (grid > m) grid = m;
  const float sc = 1.0f / sqrtf((float)r1);
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(T), lds, st, (const TIN*)A, lda, scales, (n + 127) / 128, m, n, n2,
                     d, picks, r1, out, ldo, sc);
  return hipGetLastError();
}

template <typename TIN>
static hipError_t srht_dispatch(const void* A, int64_t lda, const float* scales, int64_t m, int64_t n, const float* d,
                                const int* picks, int r1, float* out, int64_t ldo, hipStream_t st) {
  const int64_t n2 = srht_size(n);
  int E, T;
  srht_shape(n2, E, T);
  switch (E) {
    case 1: return go_srht<TIN, 1>(A, lda, scales, m, n, (int)n2, T, d, picks, r1, out, ldo, st);
    case 2: return go_srht<TIN, 2>(A, lda, scales, m, n, (int)n2, T, d, picks, r1, out, ldo, st);
    case 4: return go_srht<TIN, 4>(A, lda, scales, m, n, (int)n2, T, d, picks, r1, out, ldo, st);
    case 8: return go_srht<TIN, 8>(A, lda, scales, m, n, (int)n2, T, d, picks, r1, out, ldo, st);
    case 16: return go_srht<TIN, 16>(A, lda, scales, m, n, (int)n2, T, d, picks, r1, out, ldo, st);
    case 32: return go_srht<TIN, 32>(A, lda, scales, m, n, (int)n2, T, d, picks, r1, out, ldo, st);
  }
  return hipErrorInvalidValue;
}

bool srht_supported(int64_t n, int r1) { return srht_size(n) <= 32768 && r1 <= kSrhtMaxPicks && r1 <= srht_size(n); }

hipError_t launch_srht_rows(int dtype, const void* A, int64_t lda, const float* scales, int64_t m, int64_t n,
                            const float* d, const int* picks, int r1, float* out, int64_t ldo, hipStream_t st) {
  if (m == 0 || r1 == 0) return hipSuccess;
  if (!srht_supported(n, r1)) return hipErrorInvalidValue;
  switch (dtype) {
    case 0: return srht_dispatch<float>(A, lda, scales, m, n, d, picks, r1, out, ldo, st);
    case 2: return srht_dispatch<uint16_t>(A, lda, scales, m, n, d, picks, r1, out, ldo, st);
    case 3: return srht_dispatch<uint8_t>(A, lda, scales, m, n, d, picks, r1, out, ldo, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace rf
