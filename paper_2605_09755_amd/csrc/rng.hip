// K1 sketch table and K2 Gaussian fill.
//
// Sketch S (n x r1) of Lemma 3.2 item 2 ("CountSketch-type", s nonzeros
// +-1/sqrt(s) per row).  Placement reading: block layout, nonzero t of row j
// lies in block [floor(t r1/s), floor((t+1) r1/s)) at a column hashed by
// Philox4x32-10 on counter (j*s+t, stream, b); multiply-shift range
// reduction; sign from the top bit of the second output word.  Omega is
// Gaussian (Algorithm 1; Theorem 2.1) by Box-Muller from Philox words.
#include "common.h"
#include "kernels.h"

namespace rf {

// Integer-exact, bit-identical to the oracle table.
RF_DEV int32_t sketch_entry(int64_t idx, int s, int r1, uint64_t seed, uint32_t stream, uint32_t b) {
  int t = (int)(idx % s);
  uint32_t lo = (uint32_t)(((int64_t)t * r1) / s);
  uint32_t hi = (uint32_t)(((int64_t)(t + 1) * r1) / s);
  u32x4 x = philox((uint64_t)idx, stream, b, seed);
  uint32_t bucket = lo + (uint32_t)(((uint64_t)x.x * (uint64_t)(hi - lo)) >> 32);
  return (int32_t)(bucket | (x.y & 0x80000000u));
}

__global__ void k_sketch_table(int64_t n, int s, int r1, uint64_t seed, uint32_t stream, uint32_t b,
                               int32_t* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  out[idx] = sketch_entry(idx, s, r1, seed, stream, b);
}

// "Ready" table for the sketch-apply kernel: entry (j, q) of lane-permuted
// block t = (lane(j) % s) ^ q, where lane(j) = (j % (64*cpl)) / cpl owns column
// j.  Word = sign<<31 | (b_local * 256 + 4 t): the LDS byte offset of the
// bucket line plus the block's slot, so the kernel adds only the row part.
RF_DEV uint32_t ready_entry(const int32_t* __restrict__ table, int64_t idx, int s, int r1, int cpl) {
  int64_t j = idx / s;
  int qq = (int)(idx % s);
  int lane = (int)((j % (64 * cpl)) / cpl);
  int t = (lane % s) ^ qq;
  uint32_t e = (uint32_t)table[j * s + t];
  uint32_t lo = (uint32_t)(((int64_t)t * r1) / s);
  uint32_t bl = (e & 0x7fffffffu) - lo;
  return (e & 0x80000000u) | (bl * 256u + 4u * (uint32_t)t);
}

__global__ void k_sketch_ready(const int32_t* __restrict__ table, int64_t n, int s, int r1, int cpl,
                               uint32_t* __restrict__ ready) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  ready[idx] = ready_entry(table, idx, s, r1, cpl);
}

// Compact form for sketches of at most 512 lines per block: entry (j, q) is the
// 16-bit word sign<<15 | (b_local * 32 + t) of the same lane-permuted block t, the
// index of the 64-bit LDS word of the bucket line and the block (< 2^14), whose two
// halves hold a pair of rows.
RF_DEV uint16_t ready16_entry(const int32_t* __restrict__ table, int64_t idx, int s, int r1, int cpl) {
  const uint32_t w = ready_entry(table, idx, s, r1, cpl);
  const uint32_t line = (w & 0x7fffffffu) >> 8, t = (w & 0xffu) >> 2;
  return (uint16_t)(((w >> 31) << 15) | (line * 32u + t));
}

__global__ void k_sketch_ready16(const int32_t* __restrict__ table, int64_t n, int s, int r1, int cpl,
                                 uint16_t* __restrict__ ready) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  ready[idx] = ready16_entry(table, idx, s, r1, cpl);
}

RF_DEV void gaussian_quad(int64_t p, int64_t total, uint64_t seed, uint32_t stream, uint32_t b,
                          float* __restrict__ out, int64_t cols, int64_t ldo) {
  u32x4 x = philox((uint64_t)p, stream, b, seed);
  const double sc = 2.3283064365386963e-10;  // 2^-32
  double ua = ((double)x.x + 0.5) * sc, ub = ((double)x.y + 0.5) * sc;
  double uc = ((double)x.z + 0.5) * sc, ud = ((double)x.w + 0.5) * sc;
  double ra = sqrt(-2.0 * log(ua)), rc = sqrt(-2.0 * log(uc));
  const double twopi = 6.283185307179586;
  double z[4] = {ra * cos(twopi * ub), ra * sin(twopi * ub), rc * cos(twopi * ud), rc * sin(twopi * ud)};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int64_t g = p * 4 + e;
    if (g < total) out[(g / cols) * ldo + (g % cols)] = (float)z[e];
  }
}

__global__ void k_gaussian(int64_t total, uint64_t seed, uint32_t stream, uint32_t b,
                           float* __restrict__ out, int64_t cols, int64_t ldo) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // counter index
  if (p * 4 >= total) return;
  gaussian_quad(p, total, seed, stream, b, out, cols, ldo);
}

// ---- batched: one problem per blockIdx.y, grid-stride over its entries -------------
__global__ void k_sketch_table_batched(const RngArgs* __restrict__ as) {
  const RngArgs a = as[blockIdx.y];
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.n * a.s;
       idx += (int64_t)gridDim.x * blockDim.x)
    a.table[idx] = sketch_entry(idx, a.s, a.r1, a.seed, 0, a.b);
}
// Batched ready tables in the compact 16-bit form (the batched pass has s = 4 and
// sketches of at most 1280 columns, 320 lines per block).
__global__ void k_sketch_ready_batched(const RngArgs* __restrict__ as) {
  const RngArgs a = as[blockIdx.y];
  uint16_t* const r16 = reinterpret_cast<uint16_t*>(a.ready);
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.n * a.s;
       idx += (int64_t)gridDim.x * blockDim.x)
    r16[idx] = ready16_entry(a.table, idx, a.s, a.r1, a.cpl);
}
__global__ void k_gaussian_batched(const RngArgs* __restrict__ as) {
  const RngArgs a = as[blockIdx.y];
  const int64_t total = (int64_t)a.r1 * a.k;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p * 4 < total; p += (int64_t)gridDim.x * blockDim.x)
    gaussian_quad(p, total, a.seed, 1, a.b, a.om, a.k, a.k);
}

hipError_t launch_sketch_table(int64_t n, int s, int r1, uint64_t seed, uint32_t stream, uint32_t b,
                               int32_t* out, hipStream_t st) {
  int64_t tot = n * s;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sketch_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, s, r1,
                     seed, stream, b, out);
  return hipGetLastError();
}

hipError_t launch_sketch_ready(const int32_t* table, int64_t n, int s, int r1, int cpl, uint32_t* ready,
                               hipStream_t st) {
  int64_t tot = n * s;
  if (tot == 0) return hipSuccess;
  if (sketch_right_ready16(s, r1))
    hipLaunchKernelGGL(k_sketch_ready16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, table, n, s,
                       r1, cpl, reinterpret_cast<uint16_t*>(ready));
  else
    hipLaunchKernelGGL(k_sketch_ready, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, table, n, s,
                       r1, cpl, ready);
  return hipGetLastError();
}

hipError_t launch_gaussian(int64_t rows, int64_t cols, uint64_t seed, uint32_t stream, uint32_t b, float* out,
                           int64_t ldo, hipStream_t st) {
  int64_t tot = rows * cols;
  if (tot == 0) return hipSuccess;
  int64_t nc = (tot + 3) / 4;
  hipLaunchKernelGGL(k_gaussian, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, tot, seed, stream, b,
                     out, cols, ldo);
  return hipGetLastError();
}

// Caller-given sketch table (rf_range_finder_ex): entry t of row j must lie in
// block t = [floor(t r1/s), floor((t+1) r1/s)), the layout every sketch kernel
// indexes by.  Valid entries are copied; an entry outside its block is replaced
// by the block's first column (keeping its sign) and counted in *bad, so no
// kernel reads or writes outside its buffers whatever the table holds.
__global__ void k_table_sanitize(const int32_t* __restrict__ in, int64_t n, int s, int r1, int32_t* __restrict__ out,
                                 int* bad) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * s) return;
  const int t = (int)(idx % s);
  const uint32_t lo = (uint32_t)(((int64_t)t * r1) / s), hi = (uint32_t)(((int64_t)(t + 1) * r1) / s);
  const uint32_t e = (uint32_t)in[idx], bucket = e & 0x7fffffffu;
  if (bucket >= lo && bucket < hi) {
    out[idx] = (int32_t)e;
  } else {
    out[idx] = (int32_t)((e & 0x80000000u) | lo);
    atomicAdd(bad, 1);
  }
}

hipError_t launch_table_sanitize(const int32_t* in, int64_t n, int s, int r1, int32_t* out, int* bad, hipStream_t st) {
  const int64_t tot = n * s;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_table_sanitize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, in, n, s, r1, out, bad);
  return hipGetLastError();
}

hipError_t launch_rng_batched(const RngArgs* as, int count, int64_t max_entries, hipStream_t st) {
  if (count == 0) return hipSuccess;
  unsigned gx = (unsigned)((max_entries + 255) / 256);
  if (gx > 1024) gx = 1024;
  if (gx == 0) gx = 1;
  hipLaunchKernelGGL(k_sketch_table_batched, dim3(gx, count), dim3(256), 0, st, as);
  hipLaunchKernelGGL(k_sketch_ready_batched, dim3(gx, count), dim3(256), 0, st, as);
  hipLaunchKernelGGL(k_gaussian_batched, dim3(gx, count), dim3(256), 0, st, as);
  return hipGetLastError();
}

}  // namespace rf
