// Sparse A in CSR form.  The paper states every cost in nnz(A) (Theorems 2.1,
// 2.3, 2.5): the sketch At = A S touches each nonzero s times, and the power
// loop then runs on the dense m x r1 sketch exactly as for dense A.  The
// randomised SVD's extra product B^T = A^T Q is a sparse-times-dense product.
//
// * Sketch pass: one wave per row.  The row's r1 outputs are accumulated in LDS
//   as 64-bit integers on a fixed-point grid chosen per row (2^F with
//   nnz_row * max|a| * 2^F < 2^62), so the sums are exact integer sums whatever
//   the order of the atomics (deterministic), each term rounded to at most
//   2^-(61 - log2 nnz_row) of the row's largest |a|.  A row with a non-finite
//   value comes out NaN.
// * B^T = A^T Q: A is transposed to CSC once per call (column counts, scan,
//   scatter, then each column's entries sorted by their CSR position, so the
//   order is fixed), and each output row j sums a_ij Q[i, :] over its column in
//   that order, one wave per column, lanes over the k columns of Q (coalesced).
//
// Entries are checked as they are read: a column index outside [0, n) is skipped
// and counted (the call reports it), row pointers are clamped to [0, nnz].
#include "common.h"
#include "kernels.h"

namespace rf {

RF_DEV int64_t clamp_ptr(int64_t v, int64_t nnz) { return v < 0 ? 0 : (v > nnz ? nnz : v); }

// ---- sketch pass ----------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sketch_csr(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                    const float* __restrict__ val, int64_t m, int64_t n, int64_t nnz,
                                                    const int32_t* __restrict__ table, int s, int r1, int waves,
                                                    float* __restrict__ out, int64_t ldo, float inv_sqrt_s, int* bad) {
  extern __shared__ unsigned long long acc_all[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned long long* acc = acc_all + (size_t)w * r1;
  const int64_t stride = (int64_t)gridDim.x * waves;
  int nbad = 0;
  for (int64_t i = (int64_t)blockIdx.x * waves + w; i < m; i += stride) {
    for (int b = lane; b < r1; b += 64) acc[b] = 0ull;
    const int64_t e0 = clamp_ptr(row_ptr[i], nnz), e1 = clamp_ptr(row_ptr[i + 1], nnz);
    float amax = 0.f;
    bool nonfinite = false;
    for (int64_t e = e0 + lane; e < e1; e += 64) {
      const float a = val[e];
      if (isfinite(a)) amax = fmaxf(amax, fabsf(a));
      else nonfinite = true;
    }
    amax = wave_max(amax);
    nonfinite = __any(nonfinite);
    const int64_t cnt = e1 > e0 ? e1 - e0 : 0;
    // 2^F with cnt * amax * 2^F < 2^62: every partial sum fits in a signed 64-bit word
    int ea = 0, ec = 0;
    (void)frexpf(amax, &ea);                    // amax < 2^ea
    (void)frexp((double)(cnt > 0 ? cnt : 1), &ec);  // cnt < 2^ec
    const int F = 61 - ea - ec;
    __builtin_amdgcn_wave_barrier();
    if (amax > 0.f && !nonfinite) {
      for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int32_t j = col[e];
        if (j < 0 || (int64_t)j >= n) {
          ++nbad;
          continue;
        }
        const long long q = llrint(ldexp((double)val[e], F));
        for (int t = 0; t < s; ++t) {
          const uint32_t ent = (uint32_t)table[(int64_t)j * s + t];
          const unsigned long long v = (ent >> 31) ? (unsigned long long)(-q) : (unsigned long long)q;
          atomicAdd(&acc[ent & 0x7fffffffu], v);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    float* orow = out + i * ldo;
    const double unscale = ldexp(1.0, -F) * (double)inv_sqrt_s;
    for (int b = lane; b < r1; b += 64) {
      float v;
      if (nonfinite) v = __uint_as_float(0x7fc00000u);
      else if (!(amax > 0.f)) v = 0.f;
      else v = (float)((double)(long long)acc[b] * unscale);
      orow[b] = v;
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (nbad) atomicAdd(bad, nbad);
}

size_t sketch_csr_lds(int r1, int& waves) {
  const size_t per = (size_t)r1 * sizeof(unsigned long long);
  waves = (int)((160u * 1024u) / per);
  if (waves > 4) waves = 4;
  return (size_t)waves * per;
}

hipError_t launch_sketch_csr(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m, int64_t n,
                             int64_t nnz, const int32_t* table, int s, int r1, float* out, int64_t ldo, int* bad,
                             hipStream_t st) {
  if (m == 0 || r1 == 0) return hipSuccess;
  int waves = 0;
  const size_t lds = sketch_csr_lds(r1, waves);
  if (waves < 1) return hipErrorInvalidValue;
  (void)hipFuncSetAttribute((const void*)k_sketch_csr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int64_t grid = (m + waves - 1) / waves;
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(k_sketch_csr, dim3((unsigned)grid), dim3(64 * waves), lds, st, row_ptr, col, val, m, n, nnz, table,
                     s, r1, waves, out, ldo, 1.0f / sqrtf((float)s), bad);
  return hipGetLastError();
}

bool sketch_csr_ok(int r1) {
  int waves = 0;
  (void)sketch_csr_lds(r1, waves);
  return waves >= 1;
}

// ---- CSC of A (for A^T Q) ---------------------------------------------------------
__global__ void k_fill_i64(int64_t* p, int64_t count, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// count[j] += 1 per valid entry (count = colptr + 1, so the scan below is in place)
__global__ void k_csc_count(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t m, int64_t n,
                            int64_t nnz, unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const int64_t e0 = clamp_ptr(row_ptr[i], nnz), e1 = clamp_ptr(row_ptr[i + 1], nnz);
  for (int64_t e = e0 + (threadIdx.x & 63); e < e1; e += 64) {
    const int32_t j = col[e];
    if (j >= 0 && (int64_t)j < n) atomicAdd(&cnt[j + 1], 1ull);
  }
}

// inclusive scan of c[0..len) in place, one workgroup (chunks of 1024, carried sum)
__global__ __launch_bounds__(1024) void k_scan_i64(int64_t* c, int64_t len) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < len; base += 1024) {
    const int64_t i = base + threadIdx.x;
    buf[threadIdx.x] = i < len ? c[i] : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t v = threadIdx.x >= (unsigned)o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < len) c[i] = buf[threadIdx.x] + carry;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
}

__global__ void k_csc_scatter(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t m,
                              int64_t n, int64_t nnz, const int64_t* __restrict__ colptr,
                              unsigned long long* __restrict__ cursor, int32_t* __restrict__ csc_pos) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const int64_t e0 = clamp_ptr(row_ptr[i], nnz), e1 = clamp_ptr(row_ptr[i + 1], nnz);
  for (int64_t e = e0 + (threadIdx.x & 63); e < e1; e += 64) {
    const int32_t j = col[e];
    if (j >= 0 && (int64_t)j < n) {
      const unsigned long long slot = atomicAdd(&cursor[j], 1ull);
      csc_pos[colptr[j] + (int64_t)slot] = (int32_t)e;
    }
  }
}

// each column's entries in CSR order (insertion sort on the CSR position: unique
// keys, so the result does not depend on the scatter's atomic order)
__global__ void k_csc_sort(const int64_t* __restrict__ colptr, int64_t n, int32_t* __restrict__ csc_pos) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t a = colptr[j], b = colptr[j + 1];
  for (int64_t x = a + 1; x < b; ++x) {
    const int32_t key = csc_pos[x];
    int64_t y = x - 1;
    while (y >= a && csc_pos[y] > key) {
      csc_pos[y + 1] = csc_pos[y];
      --y;
    }
    csc_pos[y + 1] = key;
  }
}

// row of every CSR position (so a column's entry gives its row without a search)
__global__ void k_csr_rows(const int64_t* __restrict__ row_ptr, int64_t m, int64_t nnz, int32_t* __restrict__ row_of) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const int64_t e0 = clamp_ptr(row_ptr[i], nnz), e1 = clamp_ptr(row_ptr[i + 1], nnz);
  for (int64_t e = e0 + (threadIdx.x & 63); e < e1; e += 64) row_of[e] = (int32_t)i;
}

hipError_t launch_csc_build(const int64_t* row_ptr, const int32_t* col, int64_t m, int64_t n, int64_t nnz,
                            int64_t* colptr, unsigned long long* cursor, int32_t* csc_pos, int32_t* row_of,
                            hipStream_t st) {
  const unsigned gr = (unsigned)((m + 3) / 4);
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, st, colptr, n + 1, (int64_t)0);
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (int64_t*)cursor, n, (int64_t)0);
  if (m > 0) {
    hipLaunchKernelGGL(k_csc_count, dim3(gr), dim3(256), 0, st, row_ptr, col, m, n, nnz,
                       reinterpret_cast<unsigned long long*>(colptr));
    hipLaunchKernelGGL(k_csr_rows, dim3(gr), dim3(256), 0, st, row_ptr, m, nnz, row_of);
  }
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, st, colptr, n + 1);
  if (m > 0) hipLaunchKernelGGL(k_csc_scatter, dim3(gr), dim3(256), 0, st, row_ptr, col, m, n, nnz, colptr, cursor, csc_pos);
  hipLaunchKernelGGL(k_csc_sort, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, colptr, n, csc_pos);
  return hipGetLastError();
}

// ---- B^T = A^T Q ------------------------------------------------------------------
// out (n x k, ldo) row j = sum over column j of A (in CSR order) of a_ij Q[i, :];
// one wave per output row, each lane CPL consecutive columns of a 64*CPL-wide tile.
template <int CPL>
__global__ __launch_bounds__(256) void k_spmm_atq(const int64_t* __restrict__ colptr, const int32_t* __restrict__ csc_pos,
                                                  const int32_t* __restrict__ row_of, const float* __restrict__ val,
                                                  int64_t n, const float* __restrict__ Q, int64_t ldq, int k,
                                                  float* __restrict__ out, int64_t ldo) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const int lane = threadIdx.x & 63;
  const int64_t a = colptr[j], b = colptr[j + 1];
  for (int c0 = 0; c0 < k; c0 += 64 * CPL) {
    float acc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) acc[u] = 0.f;
    for (int64_t x = a; x < b; ++x) {
      const int32_t e = csc_pos[x];
      const float v = val[e];
      const float* qrow = Q + (int64_t)row_of[e] * ldq;
#pragma unroll
      for (int u = 0; u < CPL; ++u) {
        const int c = c0 + lane * CPL + u;
        if (c < k) acc[u] = fmaf(v, qrow[c], acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
      const int c = c0 + lane * CPL + u;
      if (c < k) out[j * ldo + c] = acc[u];
    }
  }
}

hipError_t launch_spmm_atq(const int64_t* colptr, const int32_t* csc_pos, const int32_t* row_of, const float* val,
                           int64_t n, const float* Q, int64_t ldq, int k, float* out, int64_t ldo, hipStream_t st) {
  if (n == 0 || k == 0) return hipSuccess;
  const unsigned g = (unsigned)((n + 3) / 4);
  if (k <= 64) hipLaunchKernelGGL(k_spmm_atq<1>, dim3(g), dim3(256), 0, st, colptr, csc_pos, row_of, val, n, Q, ldq, k, out, ldo);
  else hipLaunchKernelGGL(k_spmm_atq<4>, dim3(g), dim3(256), 0, st, colptr, csc_pos, row_of, val, n, Q, ldq, k, out, ldo);
  return hipGetLastError();
}

}  // namespace rf
