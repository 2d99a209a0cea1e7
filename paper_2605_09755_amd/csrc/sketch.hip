// K3 sketch_right: At = A S, and K4 sketch_left: out = S2^T X.
//
// A S costs O(nnz(A) s) and should run "almost as quickly as it takes to
// read A" (Section 1; cost statement in the proof of Theorem 2.1).  Every
// element A[i,j] is added, with sign, into s buckets of row i of At.
//
// Right sketch design (gfx950): a workgroup owns a band of R = 64/s rows and
// keeps their whole At rows on chip in LDS.  Lanes own columns; every lane
// reads its columns of all R rows (coalesced across lanes) and its columns'
// s table entries once, and the lanes of an instruction visit distinct
// (row, block) slots, so the LDS scatter is free of bank conflicts.  Three
// forms, in the order they are chosen:
//  * k_sketch_right_fx2 / _fx2w (s = 4, 8, 16; at most 256 / 512 lines per
//    block): fixed point with a scale per row, pairs of rows added by one 64-bit
//    LDS atomic, partials folded into the output only when needed;
//  * k_sketch_right_fx (at most 640 lines): fixed point with one scale per band
//    and chunk, folded into register accumulators after every chunk;
//  * k_sketch_right (s = 1 or 2, or larger sketches): LDS float atomics;
//  * k_sketch_right_atomic (any other s): global atomics, the generic fallback.
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rf {

template <typename TIN>
RF_DEV float ld_elem(const TIN* p);
template <>
RF_DEV float ld_elem<float>(const float* p) { return *p; }
template <>
RF_DEV float ld_elem<uint16_t>(const uint16_t* p) { return bf16_to_f32(*p); }
template <>
RF_DEV float ld_elem<uint8_t>(const uint8_t* p) { return fp8e4m3_to_f32(*p); }

// Load CPL consecutive elements starting at column j of row pointer rp (row valid).
template <typename TIN, int CPL>
RF_DEV void ld_cols(const TIN* rp, int64_t j, int64_t n, bool vec_ok, float* out) {
  if (vec_ok && j + CPL <= n) {
    if constexpr (sizeof(TIN) == 4 && CPL == 4) {
      float4 v = *reinterpret_cast<const float4*>(rp + j);
      out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
      return;
    } else if constexpr (sizeof(TIN) == 4 && CPL == 2) {
      float2 v = *reinterpret_cast<const float2*>(rp + j);
      out[0] = v.x; out[1] = v.y;
      return;
    } else if constexpr (sizeof(TIN) == 2 && CPL == 4) {
      uint2 v = *reinterpret_cast<const uint2*>(rp + j);
      out[0] = bf16_to_f32(v.x & 0xffff); out[1] = bf16_to_f32(v.x >> 16);
      out[2] = bf16_to_f32(v.y & 0xffff); out[3] = bf16_to_f32(v.y >> 16);
      return;
    } else if constexpr (sizeof(TIN) == 2 && CPL == 2) {
      uint32_t v = *reinterpret_cast<const uint32_t*>(rp + j);
      out[0] = bf16_to_f32(v & 0xffff); out[1] = bf16_to_f32(v >> 16);
      return;
    } else if constexpr (sizeof(TIN) == 1 && CPL == 4) {
      uint32_t v = *reinterpret_cast<const uint32_t*>(rp + j);
      fp8x4_to_f32(v, out);
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < CPL; ++e) out[e] = (j + e < n) ? ld_elem<TIN>(rp + j + e) : 0.f;
}

// Grid: x = row bands of R rows, y = bucket chunks (CHUNKED).  Block: NW waves.
// LDS: wl lines x 64 slots of float, line = bucket index inside its block.
template <typename TIN, int S, int CPL, int NW, bool CHUNKED>
__global__ __launch_bounds__(NW * 64) void k_sketch_right(
    const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales, int64_t ldsc,
    const uint32_t* __restrict__ ready, int64_t m, int64_t n, int r1, int wl, float* __restrict__ out,
    int64_t ldo, float inv_sqrt_s, bool vec_ok) {
  constexpr int R = 64 / S;
  extern __shared__ float acc[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int c0 = CHUNKED ? (int)blockIdx.y * wl : 0;
  for (int i = threadIdx.x; i < wl * 64; i += NW * 64) acc[i] = 0.f;
  __syncthreads();

  const int rbits = lane / S;
  const uint32_t chunk_lo = (uint32_t)c0 * 256u, chunk_hi = (uint32_t)(c0 + wl) * 256u;
  char* accb = reinterpret_cast<char*>(acc);
  const int64_t ngrp = (n + 64 * CPL - 1) / (64 * CPL);
  for (int64_t g = wave; g < ngrp; g += NW) {
    const int64_t j = g * 64 * CPL + (int64_t)lane * CPL;
    float a[R][CPL];
    uint32_t ent[CPL][S];
    float sc = 1.f;
    if constexpr (sizeof(TIN) == 1) {
      if (j < n) sc = scales[(row0 / 128) * ldsc + j / 128];
    }
#pragma unroll
    for (int p = 0; p < R; ++p) {
      const int64_t row = row0 + (rbits ^ p);
      if (row < m) ld_cols<TIN, CPL>(A + row * lda, j, n, vec_ok, a[p]);
      else {
#pragma unroll
        for (int e = 0; e < CPL; ++e) a[p][e] = 0.f;
      }
    }
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      if (j + e < n) {
        const uint32_t* ep = ready + (j + e) * S;
        if constexpr (S % 4 == 0) {
#pragma unroll
          for (int v = 0; v < S / 4; ++v) {
            uint4 w = reinterpret_cast<const uint4*>(ep)[v];
            ent[e][4 * v] = w.x; ent[e][4 * v + 1] = w.y; ent[e][4 * v + 2] = w.z; ent[e][4 * v + 3] = w.w;
          }
        } else {
#pragma unroll
          for (int qq = 0; qq < S; ++qq) ent[e][qq] = ep[qq];
        }
      } else {
#pragma unroll
        for (int qq = 0; qq < S; ++qq) ent[e][qq] = 0u;
      }
    }
    if constexpr (sizeof(TIN) == 1) {
#pragma unroll
      for (int p = 0; p < R; ++p)
#pragma unroll
        for (int e = 0; e < CPL; ++e) a[p][e] *= sc;
    }
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
#pragma unroll
      for (int qq = 0; qq < S; ++qq) {
        uint32_t base = ent[e][qq] & 0x7fffffffu;
        uint32_t sg = ent[e][qq] & 0x80000000u;
        if (CHUNKED) {
          if (base < chunk_lo || base >= chunk_hi) continue;
          base -= chunk_lo;
        }
#pragma unroll
        for (int p = 0; p < R; ++p) {
          float v = __uint_as_float(__float_as_uint(a[p][e]) ^ sg);
          atomicAdd(reinterpret_cast<float*>(accb + base + (uint32_t)(4 * S * (rbits ^ p))), v);
        }
      }
    }
  }
  __syncthreads();
  // write out: slot = r*S + t, line b -> At[row0 + r][lo_t + c0 + b]
  for (int i = threadIdx.x; i < wl * 64; i += NW * 64) {
    int b = i >> 6, slot = i & 63;
    int r = slot / S, t = slot % S;
    int64_t row = row0 + r;
    if (r >= R || row >= m) continue;
    int lo = (int)(((int64_t)t * r1) / S), hi = (int)(((int64_t)(t + 1) * r1) / S);
    int bb = c0 + b;
    if (bb < hi - lo) out[row * ldo + lo + bb] = acc[i] * inv_sqrt_s;
  }
}

// ---- fixed-point variant with one scale per band and chunk ------------------------------
// LDS float atomics are microcoded on gfx950 (~190 clk per wave instruction against
// ~4 for integer atomics), so the scatter accumulates in int32.  Per column chunk
// the workgroup takes the chunk's max |a| (integer ds_max on the float bits) and
// the chunk's exact maximum bucket occupancy c (from the sketch table), and uses
// the power-of-two scale 2^(30-e) with c * max < 2^e: no partial sum can exceed
// 2^30, and each term is rounded to 2^(e-30) <= 2^-24 c max (a bucket of c terms
// is no less accurate than an FP32 sum of them).  After the chunk the integer
// partials are folded into FP32 accumulators held in registers (each thread owns
// a fixed set of LDS words) and cleared.
template <typename TIN, int S, int CPL, int NW, int G, int FACC>
RF_DEV void sketch_right_fx_body(const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales,
                                 int64_t ldsc, const uint32_t* __restrict__ ready, const int* __restrict__ cmax,
                                 int64_t m, int64_t n, int r1, int wl, float* __restrict__ out, int64_t ldo,
                                 float inv_sqrt_s, bool vec_ok, int band) {
  constexpr int R = 64 / S;
  constexpr int NT = NW * 64;
  constexpr int64_t J = (int64_t)NW * G * 64 * CPL;  // columns per chunk
  static_assert(R <= 32, "row flags are kept in one 32-bit mask");
  extern __shared__ int iacc[];
  __shared__ unsigned wgmax, wgbad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)band * R;
  const int entries = wl * 64;
  for (int i = tid; i < entries; i += NT) iacc[i] = 0;
  if (tid == 0) { wgmax = 0u; wgbad = 0u; }
  unsigned bad = 0u;  // bit r: row row0 + r holds a non-finite value
  float facc[FACC];
#pragma unroll
  for (int i = 0; i < FACC; ++i) facc[i] = 0.f;
  __syncthreads();
  const int rbits = lane / S;
  char* accb = reinterpret_cast<char*>(iacc);
  const int64_t nch = (n + J - 1) / J;
  for (int64_t ch = 0; ch < nch; ++ch) {
    float a[G][R][CPL];
    uint32_t ent[G][CPL][S];
    float mx = 0.f;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t j = ch * J + ((int64_t)(g * NW + wave) * 64 + lane) * CPL;
      float sc = 1.f;
      if constexpr (sizeof(TIN) == 1) {
        if (j < n) sc = scales[(row0 / 128) * ldsc + j / 128];
      }
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const int64_t row = row0 + (rbits ^ p);
        if (row < m && j < n) ld_cols<TIN, CPL>(A + row * lda, j, n, vec_ok, a[g][p]);
        else {
#pragma unroll
          for (int e = 0; e < CPL; ++e) a[g][p][e] = 0.f;
        }
#pragma unroll
        for (int e = 0; e < CPL; ++e) {
          float v = a[g][p][e];
          if constexpr (sizeof(TIN) == 1) v *= sc;
          // non-finite entries are kept out of the integer sums (they would wreck
          // the chunk scale); their rows are set to NaN at the end instead
          const bool fin = isfinite(v);
          bad |= fin ? 0u : (1u << (rbits ^ p));
          a[g][p][e] = fin ? v : 0.f;
          mx = fmaxf(mx, fabsf(a[g][p][e]));
        }
      }
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        if (j + e < n) {
          const uint32_t* ep = ready + (j + e) * S;
          if constexpr (S % 4 == 0) {
#pragma unroll
            for (int v = 0; v < S / 4; ++v) {
              uint4 w = reinterpret_cast<const uint4*>(ep)[v];
              ent[g][e][4 * v] = w.x; ent[g][e][4 * v + 1] = w.y; ent[g][e][4 * v + 2] = w.z; ent[g][e][4 * v + 3] = w.w;
            }
          } else {
#pragma unroll
            for (int qq = 0; qq < S; ++qq) ent[g][e][qq] = ep[qq];
          }
        } else {
#pragma unroll
          for (int qq = 0; qq < S; ++qq) ent[g][e][qq] = 0u;
        }
      }
    }
    // chunk max over the workgroup
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) atomicMax(&wgmax, __float_as_uint(mx));
    __syncthreads();
    const float gmax = __uint_as_float(wgmax);
    const float bound = gmax * (float)max(cmax[ch], 1);
    int e2 = 0;
    frexpf(bound, &e2);                        // bound < 2^e2
    const float scale = (gmax > 0.f && isfinite(bound)) ? ldexpf(1.f, 30 - e2) : 1.f;
    const float inv_scale = (gmax > 0.f && isfinite(bound)) ? ldexpf(1.f, e2 - 30) : 1.f;
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        int xi[R];
#pragma unroll
        for (int p = 0; p < R; ++p) xi[p] = __float2int_rn(a[g][p][e] * scale);
#pragma unroll
        for (int qq = 0; qq < S; ++qq) {
          const uint32_t base = ent[g][e][qq] & 0x7fffffffu;
          const int msk = (int)ent[g][e][qq] >> 31;  // 0 or -1
#pragma unroll
          for (int p = 0; p < R; ++p) {
            const int v = (xi[p] ^ msk) - msk;
            atomicAdd(reinterpret_cast<int*>(accb + base + (uint32_t)(4 * S * (rbits ^ p))), v);
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < FACC; ++i) {
      const int idx = tid + i * NT;
      if (idx < entries) {
        facc[i] += (float)iacc[idx] * inv_scale;
        iacc[idx] = 0;
      }
    }
    if (tid == 0) wgmax = 0u;
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, 64);
  if (lane == 0 && bad) atomicOr(&wgbad, bad);
  __syncthreads();
  const unsigned rows_bad = wgbad;
  // write out: entry idx = b*64 + slot, slot = r*S + t -> At[row0 + r][lo_t + b]
#pragma unroll
  for (int i = 0; i < FACC; ++i) {
    const int idx = tid + i * NT;
    if (idx >= entries) continue;
    const int b = idx >> 6, slot = idx & 63;
    const int r = slot / S, t = slot % S;
    const int64_t row = row0 + r;
    if (r >= R || row >= m) continue;
    const int lo = (int)(((int64_t)t * r1) / S), hi = (int)(((int64_t)(t + 1) * r1) / S);
    const float v = ((rows_bad >> r) & 1u) ? __builtin_nanf("") : facc[i] * inv_sqrt_s;
    if (b < hi - lo) out[row * ldo + lo + b] = v;
  }
}

template <typename TIN, int S, int CPL, int NW, int G, int FACC>
__global__ __launch_bounds__(NW * 64) void k_sketch_right_fx(
    const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales, int64_t ldsc,
    const uint32_t* __restrict__ ready, const int* __restrict__ cmax, int64_t m, int64_t n, int r1, int wl,
    float* __restrict__ out, int64_t ldo, float inv_sqrt_s, bool vec_ok) {
  sketch_right_fx_body<TIN, S, CPL, NW, G, FACC>(A, lda, scales, ldsc, ready, cmax, m, n, r1, wl, out, ldo, inv_sqrt_s,
                                                 vec_ok, blockIdx.x);
}

// Two-workgroups-per-CU form of the fixed-point pass, for sketches of at most 256
// lines per block (64 KiB of integer partials per band; up to 512 lines run one
// workgroup per CU).  It keeps one column group
// per wave (J = 512 CPL columns per chunk) and reads the compact 16-bit table, so a
// thread fits in 128 VGPRs and two workgroups share a CU: one streams its next
// chunk from HBM while the other runs its atomics.
//
// Every row of the band has its own scale 2^E_r, set from that row's chunk maximum,
// so the rounding of a row is relative to the row itself (rows of very different
// size may share a band).  The integer partials are not folded after every chunk:
// a chunk is added at the current scales when, for every row, its values lose at
// most two bits against their own scale and the running bound on the row's partials
// (sum over chunks of c_chunk max_chunk 2^E_r plus c_chunk for the rounding) stays
// below 2^31; otherwise all partials are folded into the FP32 registers first and
// each E_r is reset from this chunk with two bits of headroom
// (2^26 <= c max 2^E_r < 2^28: at least seven chunks fit between folds, and a term
// is rounded to at most c 2^-25 times its chunk's row maximum).  A thread's LDS
// words all belong to row lane / s,
// so a fold needs one scale per thread.  One barrier per chunk (three rotating sets
// of row maxima), a second only on a fold.
template <typename TIN, int S, int CPL, int NW, int FACC>
__device__ __forceinline__ void sketch_right_fx2_body(
    const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales, int64_t ldsc,
    const uint16_t* __restrict__ ready, const int* __restrict__ cmax, int64_t m, int64_t n, int r1, int wl,
    float* __restrict__ out, int64_t ldo, float inv_sqrt_s, bool vec_ok) {
  constexpr int R = 64 / S;
  constexpr int P = R / 2;                  // row pairs of the band
  constexpr int NT = NW * 64;
  constexpr int64_t J = (int64_t)NT * CPL;  // columns per chunk
  static_assert(R <= 32 && R % 2 == 0, "row flags are kept in one 32-bit mask; rows go in pairs");
  static_assert(S % 2 == 0, "table entries are read in pairs");
  // 64-bit LDS atomics need 8-byte aligned addresses: the dynamic array follows the
  // static row maxima, so its own alignment sets where it starts
  extern __shared__ __attribute__((aligned(16))) unsigned long long sk_acc64[];
  int* const iacc = reinterpret_cast<int*>(sk_acc64);
  __shared__ unsigned rowmax[3][R], wgbad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int entries = wl * 64;  // 32-bit words: wl lines of P pairs x S blocks x 2 rows
  for (int i = tid; i < entries; i += NT) iacc[i] = 0;
  if (tid < 3 * R) (&rowmax[0][0])[tid] = 0u;
  if (tid == 0) wgbad = 0u;
  unsigned bad = 0u;  // bit r: row row0 + r holds a non-finite value
  __syncthreads();
  // lane = h * 32 + pbits * S + tbits; both half-waves visit the same slots
  const int pbits = (lane & 31) / S, tbits = lane % S;
  // The thread's 64-bit LDS words are (line tid / 32 + i NT / 32, pair pbits, block
  // tbits), rows 2 pbits and 2 pbits + 1: their FP32 sums live in the output itself,
  // which only this thread touches.
  const int64_t orow0 = row0 + 2 * pbits;
  const int blo = (int)(((int64_t)tbits * r1) / S), bw = (int)(((int64_t)(tbits + 1) * r1) / S) - blo;
  float* const optr0 = out + (orow0 < m ? orow0 : 0) * ldo + blo;
  float* const optr1 = out + (orow0 + 1 < m ? orow0 + 1 : 0) * ldo + blo;
  const bool ow0 = orow0 < m, ow1 = orow0 + 1 < m;
  bool ofirst = true;  // the output holds no folded sums yet
  char* accb = reinterpret_cast<char*>(iacc);
  // Per-row fixed-point state, kept by lane r of every wave for row r (lanes >= R
  // hold copies of nothing in particular); every wave computes the same values.
  int E = 0;           // partials of row `lane` hold sum(x 2^E), rounded per term
  float used = 0.f;    // bound on |partial| of the row in integer units since the last fold
  bool live = false;   // the row holds unfolded terms
  const int myrow = lane < R ? lane : 0;
  const int64_t nch = (n + J - 1) / J;
  for (int64_t ch = 0; ch < nch; ++ch) {
    // Opaque copy of the lane's pair bits: the per-row offsets derived from it are
    // recomputed per chunk instead of being held live across the loop.
    int pb = pbits;
    asm volatile("" : "+v"(pb));
    // register p holds band row 2 (pb ^ p/2) + p % 2: at pair step q the lanes of a
    // half-wave hit P x S distinct (pair, block) slots, one 64-bit bank pair each
    auto rowof = [&](int p) { return 2 * (pb ^ (p >> 1)) + (p & 1); };
    float a[R][CPL];
    uint32_t ent[CPL][S / 2];  // two 16-bit words each
    float mx[R];               // mx[p]: max |a| of row rowof(p) over the lane's columns
    float chk[R];              // chk[p]: sum of a * 0, NaN iff that row has a non-finite value
    const int64_t j = ch * J + ((int64_t)wave * 64 + lane) * CPL;
    float sc = 1.f;
    if constexpr (sizeof(TIN) == 1) {
      if (j < n) sc = scales[(row0 / 128) * ldsc + j / 128];
    }
    // interior chunk of a full band: unconditional vector loads (uniform branch)
    const bool interior = vec_ok && row0 + R <= m && (ch + 1) * J <= n;
    if (interior) {
#pragma unroll
      for (int p = 0; p < R; ++p) ld_cols<TIN, CPL>(A + (row0 + rowof(p)) * lda, j, n, true, a[p]);
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        const uint16_t* ep = ready + (j + e) * S;
        if constexpr (S == 4) {
          const uint2 w = *reinterpret_cast<const uint2*>(ep);
          ent[e][0] = w.x; ent[e][1] = w.y;
        } else {
#pragma unroll
          for (int v = 0; v < S / 8; ++v) {
            const uint4 w = reinterpret_cast<const uint4*>(ep)[v];
            ent[e][4 * v] = w.x; ent[e][4 * v + 1] = w.y; ent[e][4 * v + 2] = w.z; ent[e][4 * v + 3] = w.w;
          }
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const int64_t row = row0 + rowof(p);
        if (row < m && j < n) ld_cols<TIN, CPL>(A + row * lda, j, n, vec_ok, a[p]);
        else {
#pragma unroll
          for (int e = 0; e < CPL; ++e) a[p][e] = 0.f;
        }
      }
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        if (j + e < n) {
          const uint16_t* ep = ready + (j + e) * S;
          if constexpr (S == 4) {
            const uint2 w = *reinterpret_cast<const uint2*>(ep);
            ent[e][0] = w.x; ent[e][1] = w.y;
          } else {
#pragma unroll
            for (int v = 0; v < S / 8; ++v) {
              const uint4 w = reinterpret_cast<const uint4*>(ep)[v];
              ent[e][4 * v] = w.x; ent[e][4 * v + 1] = w.y; ent[e][4 * v + 2] = w.z; ent[e][4 * v + 3] = w.w;
            }
          }
        } else {
#pragma unroll
          for (int v = 0; v < S / 2; ++v) ent[e][v] = 0u;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < R; ++p) {
      mx[p] = 0.f;
      chk[p] = 0.f;
#pragma unroll
      for (int e = 0; e < CPL; ++e) {
        if constexpr (sizeof(TIN) == 1) a[p][e] *= sc;
        // a row holding a non-finite value is set to NaN at the end; its own integer
        // sums are then meaningless, and its scale is kept out of the fold decisions
        chk[p] = fmaf(a[p][e], 0.f, chk[p]);
        mx[p] = fmaxf(mx[p], fabsf(a[p][e]));
      }
      bad |= isfinite(chk[p]) ? 0u : (1u << rowof(p));
    }
    // row maxima: one LDS max (on the float bits, all >= 0) per lane and row; the
    // LDS is otherwise idle in this phase, so this is cheaper than lane shuffles
    const int slot = (int)(ch % 3);
#pragma unroll
    for (int p = 0; p < R; ++p)
      if (mx[p] > 0.f) atomicMax(&rowmax[slot][rowof(p)], __float_as_uint(mx[p]));
    __syncthreads();
    // row maxima of slot (ch + 2) % 3 were last read before this barrier and are next
    // written after the next one
    if (tid < R) rowmax[(slot + 2) % 3][tid] = 0u;
    const int c = max(cmax[ch], 1);
    const int cbits = 32 - __clz(c);  // c < 2^cbits
    // lane r decides for row r; the workgroup folds if any row must
    const float gm = __uint_as_float(rowmax[slot][myrow]);
    const bool nz = lane < R && gm > 0.f && isfinite(gm);
    int eg = 0;
    frexpf(gm, &eg);                                 // gm < 2^eg
    const int enew = min(28 - (eg + cbits), 126);   // 2^26 <= c gm 2^enew < 2^28; 2^enew finite
    const float need = ldexpf(gm * (float)c, E) + (float)c;
    // fold when a row would lose more than two bits at its current scale or could
    // overflow a partial
    const bool want = nz && live && (enew > E + 2 || used + need >= 2.0e9f);
    const bool fold = __any(want);
    if (!__any(nz)) continue;  // all-zero chunk: nothing to add
    if (fold) {
      const int ef0 = __shfl(E, 2 * pbits, 64), ef1 = __shfl(E, 2 * pbits + 1, 64);
      const bool lv0 = __shfl((int)live, 2 * pbits, 64) != 0, lv1 = __shfl((int)live, 2 * pbits + 1, 64) != 0;
      if (lv0 || lv1) {
        for (int i = 0; i < FACC / 2; ++i) {
          const int idx = tid + i * NT;  // 64-bit word
          if (2 * idx >= entries) break;
          const int b = (tid >> 5) + i * (NT / 32);
          unsigned long long* wp = reinterpret_cast<unsigned long long*>(accb) + idx;
          const unsigned long long sum = *wp;
          *wp = 0ull;
          // the 64-bit word holds x_odd 2^32 + x_even summed exactly
          const int s0 = (int)(uint32_t)sum, s1 = (int)(uint32_t)(sum >> 32) + (s0 < 0 ? 1 : 0);
          if (b < bw) {
            const float v0 = lv0 ? ldexpf((float)s0, -ef0) : 0.f, v1 = lv1 ? ldexpf((float)s1, -ef1) : 0.f;
            if (ow0) optr0[b] = ofirst ? v0 : optr0[b] + v0;
            if (ow1) optr1[b] = ofirst ? v1 : optr1[b] + v1;
          }
        }
        ofirst = false;
      }
      live = false;
      __syncthreads();
    }
    if (nz) {
      if (live) {
        used += need;
      } else {
        E = enew;
        used = ldexpf(gm * (float)c, E) + (float)c;
        live = true;
      }
    }
    // the lane's multiplier for row rowof(p)
    float mul[R];
#pragma unroll
    for (int p = 0; p < R; ++p) mul[p] = ldexpf(1.f, __shfl(E, rowof(p), 64));
#pragma unroll
    for (int e = 0; e < CPL; ++e) {
      unsigned long long X[P], NX[P];  // pair terms x_odd 2^32 + x_even and their negations
#pragma unroll
      for (int q = 0; q < P; ++q) {
        int x0, x1;
        // round half up, floor(x + 1/2), in one instruction; |x| < 2^28
        asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(x0) : "v"(a[2 * q][e] * mul[2 * q]));
        asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(x1) : "v"(a[2 * q + 1][e] * mul[2 * q + 1]));
        X[q] = ((unsigned long long)(uint32_t)(x1 + (x0 >> 31)) << 32) | (uint32_t)x0;
        NX[q] = 0ull - X[q];
      }
#pragma unroll
      for (int qq = 0; qq < S; ++qq) {
        const uint32_t w = ent[e][qq >> 1];
        // 64-bit word index of (line, block) and the sign of the entry's 16-bit half
        const uint32_t word = (qq & 1) ? ((w >> 16) & 0x7fffu) : (w & 0x7fffu);
        const bool neg = (qq & 1) ? ((int)w < 0) : ((w & 0x8000u) != 0u);
#pragma unroll
        for (int q = 0; q < P; ++q)
          atomicAdd(reinterpret_cast<unsigned long long*>(accb + (word << 3) + (uint32_t)(8 * S * (pb ^ q))),
                    neg ? NX[q] : X[q]);
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o, 64);
  if (lane == 0 && bad) atomicOr(&wgbad, bad);
  __syncthreads();
  const int ef0 = __shfl(E, 2 * pbits, 64), ef1 = __shfl(E, 2 * pbits + 1, 64);
  const bool lv0 = __shfl((int)live, 2 * pbits, 64) != 0, lv1 = __shfl((int)live, 2 * pbits + 1, 64) != 0;
  const bool bad0 = ((wgbad >> (2 * pbits)) & 1u) != 0u, bad1 = ((wgbad >> (2 * pbits + 1)) & 1u) != 0u;
  for (int i = 0; i < FACC / 2; ++i) {
    const int idx = tid + i * NT;
    if (2 * idx >= entries) break;
    const int b = (tid >> 5) + i * (NT / 32);
    if (b >= bw) continue;
    const unsigned long long sum = reinterpret_cast<const unsigned long long*>(accb)[idx];
    const int s0 = (int)(uint32_t)sum, s1 = (int)(uint32_t)(sum >> 32) + (s0 < 0 ? 1 : 0);
    float v0 = lv0 ? ldexpf((float)s0, -ef0) : 0.f, v1 = lv1 ? ldexpf((float)s1, -ef1) : 0.f;
    if (!ofirst) {
      if (ow0) v0 += optr0[b];
      if (ow1) v1 += optr1[b];
    }
    if (ow0) optr0[b] = bad0 ? __builtin_nanf("") : v0 * inv_sqrt_s;
    if (ow1) optr1[b] = bad1 ? __builtin_nanf("") : v1 * inv_sqrt_s;
  }
}

// Up to 256 lines per block: 64 KiB of partials and 128 VGPRs, two workgroups per CU.
template <typename TIN, int S, int CPL, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sketch_right_fx2(
    const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales, int64_t ldsc,
    const uint16_t* __restrict__ ready, const int* __restrict__ cmax, int64_t m, int64_t n, int r1, int wl,
    float* __restrict__ out, int64_t ldo, float inv_sqrt_s, bool vec_ok) {
  sketch_right_fx2_body<TIN, S, CPL, NW, 32>(A, lda, scales, ldsc, ready, cmax, m, n, r1, wl, out, ldo, inv_sqrt_s,
                                             vec_ok);
}

// 257 to 512 lines per block: up to 128 KiB of partials, one workgroup per CU.
template <typename TIN, int S, int CPL, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_sketch_right_fx2w(
    const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales, int64_t ldsc,
    const uint16_t* __restrict__ ready, const int* __restrict__ cmax, int64_t m, int64_t n, int r1, int wl,
    float* __restrict__ out, int64_t ldo, float inv_sqrt_s, bool vec_ok) {
  sketch_right_fx2_body<TIN, S, CPL, NW, 64>(A, lda, scales, ldsc, ready, cmax, m, n, r1, wl, out, ldo, inv_sqrt_s,
                                             vec_ok);
}

// Batched sketch pass over FP32 matrices with s = 4 (one problem per blockIdx.y): the
// paired-row fixed-point pass, 16-bit tables, chunks of 1024 columns.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_sketch_right_fx_batched(
    const SketchArgs* __restrict__ as) {
  const SketchArgs a = as[blockIdx.y];
  constexpr int R = 64 / 4;
  if ((int64_t)blockIdx.x * R >= a.m) return;
  sketch_right_fx2_body<float, 4, 2, 8, 64>(a.A, a.lda, nullptr, 0, reinterpret_cast<const uint16_t*>(a.ready),
                                            a.cmax, a.m, a.n, a.r1, (a.r1 + 3) / 4, a.out, a.ldo, 0.5f,
                                            a.vec_ok != 0);
}

// Maximum bucket occupancy per column chunk (over the s blocks): one workgroup per chunk.
RF_DEV void chunk_occupancy_body(const int32_t* __restrict__ table, int64_t n, int s, int r1, int64_t J,
                                 int* __restrict__ cmax, int chunk) {
  extern __shared__ int hist[];
  const int64_t j0 = (int64_t)chunk * J, j1 = min(n, j0 + J);
  for (int i = threadIdx.x; i < r1; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  for (int64_t e = j0 * s + threadIdx.x; e < j1 * s; e += blockDim.x)
    atomicAdd(&hist[(uint32_t)table[e] & 0x7fffffffu], 1);
  __syncthreads();
  int mx = 0;
  for (int i = threadIdx.x; i < r1; i += blockDim.x) mx = max(mx, hist[i]);
  mx = max(mx, __shfl_xor(mx, 1, 64));
  mx = max(mx, __shfl_xor(mx, 2, 64));
  mx = max(mx, __shfl_xor(mx, 4, 64));
  mx = max(mx, __shfl_xor(mx, 8, 64));
  mx = max(mx, __shfl_xor(mx, 16, 64));
  mx = max(mx, __shfl_xor(mx, 32, 64));
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) cmax[chunk] = max(max(red[0], red[1]), max(red[2], red[3]));
}

__global__ __launch_bounds__(256) void k_chunk_occupancy(const int32_t* __restrict__ table, int64_t n, int s, int r1,
                                                         int64_t J, int* __restrict__ cmax) {
  chunk_occupancy_body(table, n, s, r1, J, cmax, blockIdx.x);
}

// Batched occupancy for the s = 4 batched sketch pass (chunk J = 512 threads x 2 columns).
__global__ __launch_bounds__(256) void k_chunk_occupancy_batched(const SketchArgs* __restrict__ as) {
  const SketchArgs a = as[blockIdx.y];
  constexpr int64_t J = 512 * 2;
  if ((int64_t)blockIdx.x * J >= a.n) return;
  chunk_occupancy_body(a.table, a.n, 4, a.r1, J, a.cmax, blockIdx.x);
}

// Generic fallback (any s): one thread per element, s global atomics.  Output
// must be zeroed first; scaled by 1/sqrt(s) on the fly.
template <typename TIN>
__global__ void k_sketch_right_atomic(const TIN* __restrict__ A, int64_t lda, const float* __restrict__ scales,
                                      int64_t ldsc, const int32_t* __restrict__ table, int s, int64_t m,
                                      int64_t n, float* __restrict__ out, int64_t ldo, float inv_sqrt_s) {
  const int64_t cb = (n + 255) / 256;
  const int64_t i = (int64_t)blockIdx.x / cb;
  const int64_t j = ((int64_t)blockIdx.x % cb) * 256 + threadIdx.x;
  if (j >= n || i >= m) return;
  float a = ld_elem<TIN>(A + i * lda + j) * inv_sqrt_s;
  if constexpr (sizeof(TIN) == 1) a *= scales[(i / 128) * ldsc + j / 128];
  for (int t = 0; t < s; ++t) {
    uint32_t e = (uint32_t)table[j * s + t];
    float v = (e >> 31) ? -a : a;
    atomicAdd(out + i * ldo + (e & 0x7fffffffu), v);
  }
}

__global__ void k_fill_zero(float* p, int64_t rows, int64_t cols, int64_t ld) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  p[(idx / cols) * ld + idx % cols] = 0.f;
}

// ---- K4: out (r1 x N) = S2^T X for X (M x N) row-major, S2 given by its
// (M x s) table.  Workgroup = (strip of 64 columns, bucket chunk, row split);
// lanes own columns, rows are wave-uniform so each row's s bucket entries are
// uniform and the 64 lanes add into 64 consecutive LDS words (no conflicts).
template <typename TIN, int NW>
__global__ __launch_bounds__(NW * 64) void k_sketch_left(const TIN* __restrict__ X, int64_t ldx,
                                                         const float* __restrict__ bscale, int64_t ldsc,
                                                         const int32_t* __restrict__ table, int s, int64_t M,
                                                         int64_t N, int r1, int cw, int64_t rows_per_split,
                                                         float* __restrict__ out, int64_t ldo,
                                                         float* __restrict__ partial, float scale) {
  extern __shared__ float acc[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + lane;
  const int c0 = blockIdx.y * cw;
  const int64_t rbeg = (int64_t)blockIdx.z * rows_per_split;
  const int64_t rend = min(M, rbeg + rows_per_split);
  for (int i = threadIdx.x; i < cw * 64; i += NW * 64) acc[i] = 0.f;
  __syncthreads();
  for (int64_t i = rbeg + wave; i < rend; i += NW) {
    float x = (col < N) ? ld_elem<TIN>(X + i * ldx + col) : 0.f;
    if constexpr (sizeof(TIN) == 1) x *= (col < N) ? bscale[(i >> 7) * ldsc + (col >> 7)] : 0.f;
    const int32_t* tp = table + i * s;
    for (int t = 0; t < s; ++t) {
      uint32_t e = (uint32_t)tp[t];
      int b = (int)(e & 0x7fffffffu) - c0;
      if (b >= 0 && b < cw) {
        float v = __uint_as_float(__float_as_uint(x) ^ (e & 0x80000000u));
        atomicAdd(&acc[b * 64 + lane], v);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cw * 64; i += NW * 64) {
    int b = i >> 6, l = i & 63;
    int64_t c = (int64_t)blockIdx.x * 64 + l;
    int bb = c0 + b;
    if (c >= N || bb >= r1) continue;
    if (partial)
      partial[((int64_t)blockIdx.z * r1 + bb) * N + c] = acc[i];
    else
      out[bb * ldo + c] = acc[i] * scale;
  }
}

// ---- fixed-point left sketch --------------------------------------------------------
// The float form above pays for LDS float atomics (~190 clk per wave instruction on
// gfx950).  Here every output column j (one lane) has one fixed-point scale for the
// whole pass, set from the column's max |x| over all rows (k_colmax, one extra read
// of X) and the largest bucket occupancy c over all rows (c = the most terms any
// output row receives): 2^e > c max_j and terms are rounded to 2^(e-31), so no
// partial can exceed 2^30 and a term's rounding is at most c 2^-30 of the column
// maximum.  The scatter is then integer ds_add_u32.  A column holding a non-finite
// value comes out NaN.
template <typename TIN>
__global__ __launch_bounds__(256) void k_colmax(const TIN* __restrict__ X, int64_t ldx, const float* __restrict__ bscale,
                                                int64_t ldsc, int64_t M, int64_t N, int64_t rows_per_block,
                                                int* __restrict__ work) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= N) return;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block, r1_ = min(M, r0 + rows_per_block);
  float mx = 0.f;
  bool bad = false;
  for (int64_t i = r0; i < r1_; ++i) {
    float x = ld_elem<TIN>(X + i * ldx + col);
    if constexpr (sizeof(TIN) == 1) x *= bscale[(i >> 7) * ldsc + (col >> 7)];
    bad |= !isfinite(x);
    mx = fmaxf(mx, fabsf(x));
  }
  if (mx > 0.f) atomicMax(reinterpret_cast<unsigned*>(work) + col, __float_as_uint(mx));
  if (bad) atomicOr(work + N + col, 1);
}

// Bucket counts over all rows of an (M x s) table, many workgroups: a histogram per
// workgroup in LDS, added into the global one (r1 ints, zeroed beforehand).
__global__ __launch_bounds__(256) void k_table_hist(const int32_t* __restrict__ table, int64_t M, int s, int r1,
                                                    int64_t rows_per_block, int* __restrict__ ghist) {
  extern __shared__ int hist[];
  for (int i = threadIdx.x; i < r1; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * rows_per_block * s, e1 = min(M, ((int64_t)blockIdx.x + 1) * rows_per_block) * s;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&hist[(uint32_t)table[e] & 0x7fffffffu], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < r1; i += blockDim.x)
    if (hist[i]) atomicAdd(ghist + i, hist[i]);
}
__global__ __launch_bounds__(256) void k_hist_max(const int* __restrict__ ghist, int r1, int* __restrict__ out) {
  int mx = 0;
  for (int i = threadIdx.x; i < r1; i += blockDim.x) mx = max(mx, ghist[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  __shared__ int red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) *out = max(max(red[0], red[1]), max(red[2], red[3]));
}

__global__ void k_fill_int(int* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <typename TIN, int NW>
__global__ __launch_bounds__(NW * 64) void k_sketch_left_fx(const TIN* __restrict__ X, int64_t ldx,
                                                            const float* __restrict__ bscale, int64_t ldsc,
                                                            const int32_t* __restrict__ table, int s, int64_t M,
                                                            int64_t N, int r1, int cw, int chunks,
                                                            int64_t rows_per_split, float* __restrict__ out,
                                                            int64_t ldo, float* __restrict__ partial, float scale,
                                                            const int* __restrict__ work) {
  extern __shared__ int iacc[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // One-dimensional grid of strips x chunks x splits workgroups.  Workgroup g runs on
  // XCD g mod 8; the logical index gives each XCD a contiguous range, chunk fastest,
  // so the chunks of one column strip run at the same time behind one L2 and X is
  // read from HBM about once instead of once per chunk.
  const unsigned G = gridDim.x, g = blockIdx.x;
  const unsigned L = (G & 7u) == 0u ? (g & 7u) * (G >> 3) + (g >> 3) : g;
  const unsigned strips = (unsigned)((N + 63) / 64);
  const unsigned bchunk = L % (unsigned)chunks, bstrip = (L / (unsigned)chunks) % strips,
                 bsplit = L / ((unsigned)chunks * strips);
  const int64_t col = (int64_t)bstrip * 64 + lane;
  const bool colok = col < N;
  const int c0 = (int)bchunk * cw;
  const int64_t rbeg = (int64_t)bsplit * rows_per_split;
  const int64_t rend = min(M, rbeg + rows_per_split);
  for (int i = threadIdx.x; i < cw * 64; i += NW * 64) iacc[i] = 0;
  // the lane's column scale
  const float cm = colok ? __uint_as_float((unsigned)work[col]) : 0.f;
  const int c = max(work[2 * N], 1);
  int e = 0;
  frexpf(cm, &e);                          // cm < 2^e
  e += 32 - __clz(c);                      // c cm < 2^e
  const bool live = cm > 0.f && isfinite(cm);
  const float mul = live ? ldexpf(1.f, 30 - e) : 0.f;
  const float inv = live ? ldexpf(1.f, e - 30) : 0.f;
  __syncthreads();
  auto row_xi = [&](int64_t i) -> int {
    float x = colok ? ld_elem<TIN>(X + i * ldx + col) : 0.f;
    if constexpr (sizeof(TIN) == 1) x *= colok ? bscale[(i >> 7) * ldsc + (col >> 7)] : 0.f;
    return isfinite(x) ? __float2int_rn(x * mul) : 0;
  };
  auto row_add = [&](int64_t i, int xi) {
    const int32_t* tp = table + i * s;
    if (s == 8) {  // the row's entries as two 16-byte groups (wave-uniform address)
      const uint4 e0 = reinterpret_cast<const uint4*>(tp)[0], e1 = reinterpret_cast<const uint4*>(tp)[1];
      const uint32_t en[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int b = (int)(en[t] & 0x7fffffffu) - c0;
        if (b >= 0 && b < cw) atomicAdd(&iacc[b * 64 + lane], (en[t] & 0x80000000u) ? -xi : xi);
      }
    } else {
      for (int t = 0; t < s; ++t) {
        const uint32_t en = (uint32_t)tp[t];
        const int b = (int)(en & 0x7fffffffu) - c0;
        if (b >= 0 && b < cw) atomicAdd(&iacc[b * 64 + lane], (en & 0x80000000u) ? -xi : xi);
      }
    }
  };
  // wave w takes blocks of U consecutive rows, NW blocks apart
  constexpr int U = 8;
  const int64_t step = (int64_t)NW * U;
  int64_t blk = rbeg + (int64_t)wave * U;
  if (s == 8) {
    // software pipeline: the next block's U row values and its 64 table entries (one
    // per lane, read back with readlane) are in flight while this block is scattered
    float xc[U], xn[U];
    uint32_t tc = 0u, tn = 0u;
    auto issue = [&](int64_t b0, float (&x)[U], uint32_t& tv) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = b0 + u;
        x[u] = (colok && i < rend) ? ld_elem<TIN>(X + i * ldx + col) : 0.f;
        if constexpr (sizeof(TIN) == 1) x[u] *= (colok && i < rend) ? bscale[(i >> 7) * ldsc + (col >> 7)] : 0.f;
      }
      const int64_t ti = b0 + (lane >> 3);
      tv = ti < rend ? (uint32_t)table[ti * 8 + (lane & 7)] : 0u;
    };
    if (blk < rend) issue(blk, xc, tc);
    for (; blk < rend; blk += step) {
      if (blk + step < rend) issue(blk + step, xn, tn);
      const int nrow = (int)min((int64_t)U, rend - blk);
      // entries of this block that fall in the chunk, one bit per lane (u * 8 + t):
      // each row visits only its own in-chunk entries (about s cw / r1 of them)
      const int bl = (int)(tc & 0x7fffffffu) - c0;
      unsigned long long inm = __ballot(bl >= 0 && bl < cw);
      if (nrow < U) inm &= (1ull << (nrow * 8)) - 1ull;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int xi = isfinite(xc[u]) ? __float2int_rn(xc[u] * mul) : 0;
        unsigned m = (unsigned)__builtin_amdgcn_readfirstlane((int)((unsigned)(inm >> (u * 8)) & 0xffu));
        while (m) {
          const int t = __builtin_ctz(m);
          m &= m - 1u;
          const uint32_t en = (uint32_t)__builtin_amdgcn_readlane((int)tc, u * 8 + t);
          atomicAdd(&iacc[((int)(en & 0x7fffffffu) - c0) * 64 + lane], (en & 0x80000000u) ? -xi : xi);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xc[u] = xn[u];
      tc = tn;
    }
  } else {
    for (; blk < rend; blk += step) {
      if (blk + U <= rend) {
        int xi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xi[u] = row_xi(blk + u);
#pragma unroll
        for (int u = 0; u < U; ++u) row_add(blk + u, xi[u]);
      } else {
        for (int64_t i = blk; i < rend; ++i) row_add(i, row_xi(i));
      }
    }
  }
  __syncthreads();
  const bool cbad = colok && work[N + col] != 0;
  for (int i = threadIdx.x; i < cw * 64; i += NW * 64) {
    int b = i >> 6, l = i & 63;
    int64_t cc = (int64_t)bstrip * 64 + l;
    int bb = c0 + b;
    if (cc >= N || bb >= r1) continue;
    // every lane reads its own column's words here (i & 63 == lane)
    const float v = cbad ? __builtin_nanf("") : (float)iacc[i] * inv;
    if (partial)
      partial[((int64_t)bsplit * r1 + bb) * N + cc] = v;
    else
      out[bb * ldo + cc] = v * scale;
  }
}

__global__ void k_reduce_partial(const float* __restrict__ partial, int splits, int64_t rows, int64_t cols,
                                 float* __restrict__ out, int64_t ldo, float scale) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += partial[(int64_t)z * rows * cols + idx];
  out[(idx / cols) * ldo + idx % cols] = s * scale;
}

// ---- launchers -------------------------------------------------------------------------
static int g_num_cu = 0;
static int num_cu() {
  if (!g_num_cu) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (g_num_cu <= 0) g_num_cu = 256;
  }
  return g_num_cu;
}

int sketch_right_cpl(int s) { return s >= 8 ? 4 : (s == 4 ? 2 : 1); }

bool sketch_right_fast_ok(int s) { return s == 1 || s == 2 || s == 4 || s == 8 || s == 16; }

template <typename TIN, int S, int CPL>
static hipError_t launch_sr(const void* A, int64_t lda, const float* scales, int64_t ldsc, const uint32_t* ready,
                            int64_t m, int64_t n, int r1, float* out, int64_t ldo, hipStream_t st) {
  constexpr int NW = 8;
  const int R = 64 / S;
  int wmax = (r1 + S - 1) / S;
  const int wl_cap = 640;  // 640 lines * 64 slots * 4 B = 160 KiB
  int chunks = (wmax + wl_cap - 1) / wl_cap;
  int wl = (wmax + chunks - 1) / chunks;
  size_t lds = (size_t)wl * 64 * sizeof(float);
  dim3 grid((unsigned)((m + R - 1) / R), (unsigned)chunks);
  bool vec_ok = (((uintptr_t)A) % (sizeof(TIN) * CPL) == 0) && (lda % CPL == 0);
  float inv = 1.0f / sqrtf((float)S);
  if (chunks == 1) {
    auto k = k_sketch_right<TIN, S, CPL, NW, false>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const TIN*)A, lda, scales, ldsc, ready, m, n, r1, wl,
                       out, ldo, inv, vec_ok);
  } else {
    auto k = k_sketch_right<TIN, S, CPL, NW, true>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const TIN*)A, lda, scales, ldsc, ready, m, n, r1, wl,
                       out, ldo, inv, vec_ok);
  }
  return hipGetLastError();
}

template <typename TIN, int S, int CPL, int G, int FACC>
static hipError_t launch_sr_fx_g(const void* A, int64_t lda, const float* scales, int64_t ldsc, const int32_t* table,
                                 const uint32_t* ready, int* cmax, int64_t m, int64_t n, int r1, float* out,
                                 int64_t ldo, hipStream_t st) {
  constexpr int NW = 8;
  constexpr int64_t J = (int64_t)NW * G * 64 * CPL;
  const int R = 64 / S;
  const int wl = (r1 + S - 1) / S;
  const int64_t nch = (n + J - 1) / J;
  size_t hl = (size_t)r1 * sizeof(int);
  hipFuncSetAttribute((const void*)k_chunk_occupancy, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hl);
  hipLaunchKernelGGL(k_chunk_occupancy, dim3((unsigned)nch), dim3(256), hl, st, table, n, S, r1, J, cmax);
  size_t lds = (size_t)wl * 64 * sizeof(int);
  dim3 grid((unsigned)((m + R - 1) / R));
  bool vec_ok = (((uintptr_t)A) % (sizeof(TIN) * CPL) == 0) && (lda % CPL == 0);
  float inv = 1.0f / sqrtf((float)S);
  auto k = k_sketch_right_fx<TIN, S, CPL, NW, G, FACC>;
  hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const TIN*)A, lda, scales, ldsc, ready, cmax, m, n, r1, wl, out,
                     ldo, inv, vec_ok);
  return hipGetLastError();
}

bool sketch_right_ready16(int s, int r1) { return (s == 4 || s == 8 || s == 16) && (r1 + s - 1) / s <= 512; }

template <typename TIN, int S, int CPL>
static hipError_t launch_sr_fx2(const void* A, int64_t lda, const float* scales, int64_t ldsc, const int32_t* table,
                                const uint16_t* ready, int* cmax, int64_t m, int64_t n, int r1, float* out,
                                int64_t ldo, hipStream_t st) {
  constexpr int NW = 8;
  constexpr int64_t J = (int64_t)NW * 64 * CPL;
  const int R = 64 / S;
  const int wl = (r1 + S - 1) / S;  // <= 512: 32 (64) FP32 accumulators per thread up to 256 (512) lines
  const int64_t nch = (n + J - 1) / J;
  size_t hl = (size_t)r1 * sizeof(int);
  hipFuncSetAttribute((const void*)k_chunk_occupancy, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hl);
  hipLaunchKernelGGL(k_chunk_occupancy, dim3((unsigned)nch), dim3(256), hl, st, table, n, S, r1, J, cmax);
  size_t lds = (size_t)wl * 64 * sizeof(int);
  dim3 grid((unsigned)((m + R - 1) / R));
  bool vec_ok = (((uintptr_t)A) % (sizeof(TIN) * CPL) == 0) && (lda % CPL == 0);
  float inv = 1.0f / sqrtf((float)S);
  auto k = wl <= 256 ? k_sketch_right_fx2<TIN, S, CPL, NW> : k_sketch_right_fx2w<TIN, S, CPL, NW>;
  hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const TIN*)A, lda, scales, ldsc, ready, cmax, m, n, r1, wl, out,
                     ldo, inv, vec_ok);
  return hipGetLastError();
}

// FP32 accumulators per thread: ceil(wl*64/512) <= 40 keeps two column groups per
// wave in flight; larger sketches hold one group to stay within 256 VGPRs.
template <typename TIN, int S, int CPL>
static hipError_t launch_sr_fx(const void* A, int64_t lda, const float* scales, int64_t ldsc, const int32_t* table,
                               const uint32_t* ready, int* cmax, int64_t m, int64_t n, int r1, float* out, int64_t ldo,
                               hipStream_t st) {
  const int wl = (r1 + S - 1) / S;
  if (wl <= 320)
    return launch_sr_fx_g<TIN, S, CPL, 2, 40>(A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
  return launch_sr_fx_g<TIN, S, CPL, 1, 80>(A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
}

size_t sketch_right_cmax_ints(int64_t n) { return (size_t)(n / 1024 + 16); }

hipError_t launch_sketch_right_batched(const SketchArgs* as, int count, int64_t mmax, int64_t nmax, int r1max,
                                       hipStream_t st) {
  if (count == 0) return hipSuccess;
  constexpr int64_t J = 512 * 2;
  const size_t hl = (size_t)r1max * sizeof(int);
  (void)hipFuncSetAttribute((const void*)k_chunk_occupancy_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)hl);
  hipLaunchKernelGGL(k_chunk_occupancy_batched, dim3((unsigned)((nmax + J - 1) / J), count), dim3(256), hl, st, as);
  const int wl = (r1max + 3) / 4;
  const size_t lds = (size_t)wl * 64 * sizeof(int);
  (void)hipFuncSetAttribute((const void*)k_sketch_right_fx_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(k_sketch_right_fx_batched, dim3((unsigned)((mmax + 15) / 16), count), dim3(512), lds, st, as);
  return hipGetLastError();
}

template <typename TIN>
static hipError_t launch_sr_dispatch(int s, const void* A, int64_t lda, const float* scales, int64_t ldsc,
                                     const int32_t* table, const uint32_t* ready, int* cmax, int64_t m, int64_t n,
                                     int r1, float* out, int64_t ldo, hipStream_t st) {
  const int wl = (r1 + s - 1) / s;
  if (sketch_right_ready16(s, r1)) {  // the ready table is in the 16-bit form
    if (!cmax) return hipErrorInvalidValue;
    const uint16_t* r16 = reinterpret_cast<const uint16_t*>(ready);
    switch (s) {
      case 4: return launch_sr_fx2<TIN, 4, 2>(A, lda, scales, ldsc, table, r16, cmax, m, n, r1, out, ldo, st);
      case 8: return launch_sr_fx2<TIN, 8, 4>(A, lda, scales, ldsc, table, r16, cmax, m, n, r1, out, ldo, st);
      case 16: return launch_sr_fx2<TIN, 16, 4>(A, lda, scales, ldsc, table, r16, cmax, m, n, r1, out, ldo, st);
      default: break;
    }
  }
  if (cmax && wl <= 640) {
    switch (s) {
      case 4: return launch_sr_fx<TIN, 4, 2>(A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
      case 8: return launch_sr_fx<TIN, 8, 4>(A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
      case 16: return launch_sr_fx<TIN, 16, 4>(A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
      default: break;
    }
  }
  switch (s) {
    case 1: return launch_sr<TIN, 1, 1>(A, lda, scales, ldsc, ready, m, n, r1, out, ldo, st);
    case 2: return launch_sr<TIN, 2, 1>(A, lda, scales, ldsc, ready, m, n, r1, out, ldo, st);
    case 4: return launch_sr<TIN, 4, 2>(A, lda, scales, ldsc, ready, m, n, r1, out, ldo, st);
    case 8: return launch_sr<TIN, 8, 4>(A, lda, scales, ldsc, ready, m, n, r1, out, ldo, st);
    case 16: return launch_sr<TIN, 16, 4>(A, lda, scales, ldsc, ready, m, n, r1, out, ldo, st);
  }
  return hipErrorInvalidValue;
}

// ---- gather form: s without a fixed-point path (CountSketch s = 1, s = 2, 3, 5, ...,
// and sketches too large for the fixed-point forms' LDS lines) ----------------------
// Atomic-free and deterministic.  The table is first turned into bucket lists: for
// every output column c of At, the columns j of A with a nonzero in c, ascending,
// as 16-bit entries j | sign << 15 (n <= 32768).  A persistent workgroup copies the
// offsets, and the lists when they fit, into LDS once (larger lists are read from
// global memory, where they stay in L2), then streams rows: the next row is
// prefetched into registers while the current row sits in LDS, and thread t forms
// the outputs c = t, t + 256, ... as fixed-order FP32 sums over their lists (one
// broadcast-free LDS read per term).
constexpr int kGatherMaxN = 32768;
constexpr int kGatherLds = 160 * 1024;

// LDS of one gather workgroup: the row, the offsets and, when they fit, the lists
// (otherwise the lists are read from global memory, where they stay in L2).
static bool gather_lists_in_lds(int64_t n, int s, int r1) {
  return (size_t)n * 4 + ((size_t)n * s * 2 + 15) / 16 * 16 + (size_t)(r1 + 1) * 4 <= (size_t)kGatherLds;
}
static size_t gather_lds_bytes(int64_t n, int s, int r1) {
  const size_t lists = gather_lists_in_lds(n, s, r1) ? ((size_t)n * s * 2 + 15) / 16 * 16 : 0;
  return (size_t)n * 4 + lists + (size_t)(r1 + 1) * 4;
}

// s = 4, 8, 16 use the fixed-point forms while their block holds at most 640 bucket
// lines; other s, and larger sketches, the gather form (when a row fits in LDS).
bool sketch_right_gather(int s, int64_t n, int r1) {
  if ((s == 4 || s == 8 || s == 16) && (r1 + s - 1) / s <= 640) return false;
  return n <= kGatherMaxN && (size_t)n * 4 + (size_t)(r1 + 1) * 4 <= (size_t)kGatherLds;
}

size_t sketch_right_work_ints(int64_t n, int s, int r1) {
  const size_t g = (size_t)2 * r1 + 2 + (size_t)n * s + ((size_t)n * s + 1) / 2 + 8;
  const size_t c = sketch_right_cmax_ints(n);
  return g > c ? g : c;
}

__global__ void k_bkt_count(const int32_t* __restrict__ table, int64_t ne, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ne) atomicAdd(&cnt[table[i] & 0x7fffffff], 1);
}

// start[0..r1] = exclusive prefix sum of cnt[0..r1) (in place; one workgroup)
__global__ __launch_bounds__(1024) void k_bkt_scan(int* __restrict__ cnt, int r1) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (r1 + 1023) / 1024, lo = t * per, hi = min(lo + per, r1);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;  // exclusive
  for (int i = lo; i < hi; ++i) {
    const int c = cnt[i];
    cnt[i] = run;
    run += c;
  }
  if (t == 1023) cnt[r1] = part[1023];
}

__global__ void k_bkt_fill(const int32_t* __restrict__ table, int64_t n, int s, const int* __restrict__ start,
                           int* __restrict__ cursor, int32_t* __restrict__ list) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n * s) return;
  const int32_t e = table[p];
  const int c = e & 0x7fffffff;
  const int pos = start[c] + atomicAdd(&cursor[c], 1);
  list[pos] = (int32_t)(p / s) | (e & (int32_t)0x80000000);
}

// each list sorted by column (insertion sort; a column appears at most once per
// list, since the s nonzeros of a column lie in different blocks), then packed
// into 16-bit entries
__global__ void k_bkt_sort(const int* __restrict__ start, int r1, int32_t* __restrict__ list,
                           uint16_t* __restrict__ list16) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= r1) return;
  const int a = start[c], b = start[c + 1];
  for (int i = a + 1; i < b; ++i) {
    const int32_t v = list[i];
    const int key = v & 0x7fffffff;
    int k = i - 1;
    while (k >= a && (list[k] & 0x7fffffff) > key) {
      list[k + 1] = list[k];
      --k;
    }
    list[k + 1] = v;
  }
  for (int i = a; i < b; ++i) {
    const int32_t v = list[i];
    list16[i] = (uint16_t)((v & 0x7fff) | (v < 0 ? 0x8000 : 0));
  }
}

constexpr int kGT = 256;      // threads of the gather workgroup
constexpr int kGQ = 32;       // at most 32 float4 chunks (128 elements) of a row per thread

template <typename TIN, bool LDS_LISTS>
__global__ __launch_bounds__(kGT) void k_sketch_gather(const TIN* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ scales, int64_t ldsc,
                                                       const int* __restrict__ start,
                                                       const uint16_t* __restrict__ list16, int64_t m, int64_t n,
                                                       int ne, int r1, float* __restrict__ out, int64_t ldo,
                                                       float inv_sqrt_s, bool vec_ok) {
  extern __shared__ __attribute__((aligned(16))) unsigned char gsm[];
  float* row = reinterpret_cast<float*>(gsm);
  const size_t lbytes = LDS_LISTS ? ((size_t)ne * 2 + 15) / 16 * 16 : 0;
  uint16_t* lsm = reinterpret_cast<uint16_t*>(gsm + (size_t)n * 4);
  int* st = reinterpret_cast<int*>(gsm + (size_t)n * 4 + lbytes);
  const int tid = threadIdx.x;
  if constexpr (LDS_LISTS)
    for (int i = tid; i < ne; i += kGT) lsm[i] = list16[i];
  const uint16_t* lst = LDS_LISTS ? lsm : list16;
  for (int i = tid; i <= r1; i += kGT) st[i] = start[i];
  // row loader: thread t owns elements 4 (t + kGT q) .. +3 of the row, q < nq
  const int nq = (int)((n + 4 * kGT - 1) / (4 * kGT));
  float pre[kGQ][4];
  auto load_row = [&](int64_t i) {
#pragma unroll
    for (int q = 0; q < kGQ; ++q) {
      if (q < nq) {
        const int64_t j = 4 * ((int64_t)tid + (int64_t)kGT * q);
        if (j < n) {
          ld_cols<TIN, 4>(A + i * lda, j, n, vec_ok, pre[q]);
          if constexpr (sizeof(TIN) == 1) {
            const float sc = scales[(i >> 7) * ldsc + (j >> 7)];  // 4 | 128: one block per chunk
#pragma unroll
            for (int e = 0; e < 4; ++e) pre[q][e] *= sc;
          }
        }
      }
    }
  };
  int64_t i = blockIdx.x;
  if (i < m) load_row(i);
  for (; i < m; i += gridDim.x) {
    __syncthreads();  // the previous row's gathers are done
#pragma unroll
    for (int q = 0; q < kGQ; ++q) {
      if (q < nq) {
        const int64_t j = 4 * ((int64_t)tid + (int64_t)kGT * q);
        if (j + 4 <= n) {
          *reinterpret_cast<float4*>(row + j) = make_float4(pre[q][0], pre[q][1], pre[q][2], pre[q][3]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (j + e < n) row[j + e] = pre[q][e];
        }
      }
    }
    __syncthreads();
    if (i + gridDim.x < m) load_row(i + gridDim.x);
    // two outputs per thread at a time, terms read four at a time: independent LDS
    // reads in flight, each output still summed in ascending column order
    for (int c0 = tid; c0 < r1; c0 += 2 * kGT) {
      const int c1 = c0 + kGT;
      const int a0 = st[c0], b0 = st[c0 + 1];
      const int a1 = c1 < r1 ? st[c1] : 0, b1 = c1 < r1 ? st[c1 + 1] : 0;
      float acc0 = 0.f, acc1 = 0.f;
      int e0 = a0, e1 = a1;
      auto term = [&](uint16_t v) {
        const float x = row[v & 0x7fff];
        return (v & 0x8000) ? -x : x;
      };
      while (e0 + 4 <= b0 && e1 + 4 <= b1) {
        const uint16_t u0 = lst[e0], u1 = lst[e0 + 1], u2 = lst[e0 + 2], u3 = lst[e0 + 3];
        const uint16_t w0 = lst[e1], w1 = lst[e1 + 1], w2 = lst[e1 + 2], w3 = lst[e1 + 3];
        const float x0 = term(u0), x1 = term(u1), x2 = term(u2), x3 = term(u3);
        const float y0 = term(w0), y1 = term(w1), y2 = term(w2), y3 = term(w3);
        acc0 += x0; acc0 += x1; acc0 += x2; acc0 += x3;
        acc1 += y0; acc1 += y1; acc1 += y2; acc1 += y3;
        e0 += 4;
        e1 += 4;
      }
      while (e0 + 4 <= b0) {
        const uint16_t u0 = lst[e0], u1 = lst[e0 + 1], u2 = lst[e0 + 2], u3 = lst[e0 + 3];
        const float x0 = term(u0), x1 = term(u1), x2 = term(u2), x3 = term(u3);
        acc0 += x0; acc0 += x1; acc0 += x2; acc0 += x3;
        e0 += 4;
      }
      while (e1 + 4 <= b1) {
        const uint16_t w0 = lst[e1], w1 = lst[e1 + 1], w2 = lst[e1 + 2], w3 = lst[e1 + 3];
        const float y0 = term(w0), y1 = term(w1), y2 = term(w2), y3 = term(w3);
        acc1 += y0; acc1 += y1; acc1 += y2; acc1 += y3;
        e1 += 4;
      }
      for (; e0 < b0; ++e0) acc0 += term(lst[e0]);
      for (; e1 < b1; ++e1) acc1 += term(lst[e1]);
      out[i * ldo + c0] = acc0 * inv_sqrt_s;
      if (c1 < r1) out[i * ldo + c1] = acc1 * inv_sqrt_s;
    }
  }
}

template <typename TIN>
static hipError_t launch_gather(const void* A, int64_t lda, const float* scales, int64_t ldsc, const int32_t* table,
                                int* work, int s, int64_t m, int64_t n, int r1, float* out, int64_t ldo,
                                hipStream_t st) {
  const int64_t ne = n * s;
  int* start = work;                       // r1 + 1
  int* cursor = start + r1 + 1;            // r1
  int32_t* list = cursor + r1;             // n s
  uint16_t* list16 = reinterpret_cast<uint16_t*>(list + ne);
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((2 * r1 + 1 + 255) / 256)), dim3(256), 0, st, start,
                     (int64_t)(2 * r1 + 1));
  hipLaunchKernelGGL(k_bkt_count, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, table, ne, start);
  hipLaunchKernelGGL(k_bkt_scan, dim3(1), dim3(1024), 0, st, start, r1);
  hipLaunchKernelGGL(k_bkt_fill, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, table, n, s, start, cursor,
                     list);
  hipLaunchKernelGGL(k_bkt_sort, dim3((unsigned)((r1 + 255) / 256)), dim3(256), 0, st, start, r1, list, list16);
  const size_t lds = gather_lds_bytes(n, s, r1);
  const bool in_lds = gather_lists_in_lds(n, s, r1);
  static std::once_flag attr;
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute((const void*)k_sketch_gather<TIN, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kGatherLds);
    (void)hipFuncSetAttribute((const void*)k_sketch_gather<TIN, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kGatherLds);
  });
  const int64_t per_cu = (int64_t)(kGatherLds / lds) < 4 ? (int64_t)(kGatherLds / lds) : 4;  // workgroups per CU
  const int64_t slots = per_cu * num_cu();
  const int64_t grid = m < slots ? m : slots;
  const bool vec_ok = (((uintptr_t)A) % (sizeof(TIN) * 4) == 0) && (lda % 4 == 0);
  auto k = in_lds ? k_sketch_gather<TIN, true> : k_sketch_gather<TIN, false>;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kGT), lds, st, (const TIN*)A, lda, scales, ldsc, start, list16, m,
                     n, (int)ne, r1, out, ldo, 1.0f / sqrtf((float)s), vec_ok);
  return hipGetLastError();
}

hipError_t launch_sketch_right(int dtype, const void* A, int64_t lda, const float* scales, const int32_t* table,
                               const uint32_t* ready, int* cmax, int s, int64_t m, int64_t n, int r1, float* out,
                               int64_t ldo, hipStream_t st) {
  if (m == 0 || n == 0) return hipSuccess;
  int64_t ldsc = (n + 127) / 128;
  if (sketch_right_gather(s, n, r1) && cmax) {
    switch (dtype) {
      case 0: return launch_gather<float>(A, lda, scales, ldsc, table, cmax, s, m, n, r1, out, ldo, st);
      case 2: return launch_gather<uint16_t>(A, lda, scales, ldsc, table, cmax, s, m, n, r1, out, ldo, st);
      case 3: return launch_gather<uint8_t>(A, lda, scales, ldsc, table, cmax, s, m, n, r1, out, ldo, st);
    }
    return hipErrorInvalidValue;
  }
  if (sketch_right_fast_ok(s) && ready) {
    switch (dtype) {
      case 0: return launch_sr_dispatch<float>(s, A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
      case 2: return launch_sr_dispatch<uint16_t>(s, A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
      case 3: return launch_sr_dispatch<uint8_t>(s, A, lda, scales, ldsc, table, ready, cmax, m, n, r1, out, ldo, st);
    }
    return hipErrorInvalidValue;
  }
  int64_t tot = m * r1;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, out, m, (int64_t)r1, ldo);
  dim3 grid((unsigned)(((n + 255) / 256) * m));
  float inv = 1.0f / sqrtf((float)s);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(k_sketch_right_atomic<float>, grid, dim3(256), 0, st, (const float*)A, lda, scales, ldsc,
                         table, s, m, n, out, ldo, inv);
      break;
    case 2:
      hipLaunchKernelGGL(k_sketch_right_atomic<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)A, lda, scales,
                         ldsc, table, s, m, n, out, ldo, inv);
      break;
    case 3:
      hipLaunchKernelGGL(k_sketch_right_atomic<uint8_t>, grid, dim3(256), 0, st, (const uint8_t*)A, lda, scales,
                         ldsc, table, s, m, n, out, ldo, inv);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t sketch_left_partial_floats(int64_t M, int64_t N, int r1) {
  int cw = 512;
  int chunks = (r1 + cw - 1) / cw;
  int64_t strips = (N + 63) / 64;
  int64_t wgs = strips * chunks;
  int splits = 1;
  while (wgs * splits < 2 * num_cu() && splits < 64 && M / (splits * 2) >= 256) splits *= 2;
  return splits > 1 ? (size_t)splits * r1 * N : 0;
}

size_t sketch_left_work_ints(int64_t N, int r1) { return (size_t)(2 * N + 16 + r1); }

hipError_t launch_sketch_left(int dtype, const void* X, int64_t ldx, const int32_t* table, int s, int64_t M,
                              int64_t N, int r1, float* out, int64_t ldo, float* partial, hipStream_t st,
                              const float* scales, int* work) {
  if (N == 0 || r1 == 0) return hipSuccess;
  constexpr int NW = 8;
  int cw = 512;
  int chunks = (r1 + cw - 1) / cw;
  cw = (r1 + chunks - 1) / chunks;
  int64_t strips = (N + 63) / 64;
  int64_t wgs = strips * chunks;
  int splits = 1;
  while (wgs * splits < 2 * num_cu() && splits < 64 && M / (splits * 2) >= 256) splits *= 2;
  if (splits > 1 && !partial) splits = 1;
  int64_t rps = (M + splits - 1) / splits;
  size_t lds = (size_t)cw * 64 * sizeof(float);
  float scale = 1.0f / sqrtf((float)s);
  dim3 grid((unsigned)strips, (unsigned)chunks, (unsigned)splits);
  float* part = splits > 1 ? partial : nullptr;
  const int64_t ldsc = (N + 127) / 128;
  if (work && M > 0 && (dtype == 0 || dtype == 2 || (dtype == 3 && scales))) {
    const int64_t nw = (int64_t)sketch_left_work_ints(N, r1);
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, work, nw);
    // column maxima: 256 columns per workgroup, rows in blocks of 512
    const int64_t rpb = 512;
    dim3 gcm((unsigned)((N + 255) / 256), (unsigned)((M + rpb - 1) / rpb));
    if (dtype == 0)
      hipLaunchKernelGGL(k_colmax<float>, gcm, dim3(256), 0, st, (const float*)X, ldx, scales, ldsc, M, N, rpb, work);
    else if (dtype == 2)
      hipLaunchKernelGGL(k_colmax<uint16_t>, gcm, dim3(256), 0, st, (const uint16_t*)X, ldx, scales, ldsc, M, N, rpb,
                         work);
    else
      hipLaunchKernelGGL(k_colmax<uint8_t>, gcm, dim3(256), 0, st, (const uint8_t*)X, ldx, scales, ldsc, M, N, rpb,
                         work);
    // largest bucket occupancy over all M rows (global histogram after the column flags)
    const size_t hl = (size_t)r1 * sizeof(int);
    const int64_t hrows = 1024;
    hipFuncSetAttribute((const void*)k_table_hist, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hl);
    hipLaunchKernelGGL(k_table_hist, dim3((unsigned)((M + hrows - 1) / hrows)), dim3(256), hl, st, table, M, s, r1,
                       hrows, work + 2 * N + 16);
    hipLaunchKernelGGL(k_hist_max, dim3(1), dim3(256), 0, st, work + 2 * N + 16, r1, work + 2 * N);
    // one workgroup per CU (cw x 64 ints of LDS), 16 waves to keep rows in flight
    constexpr int NWF = 16;
    const dim3 g1((unsigned)(strips * chunks * splits));
    if (dtype == 0) {
      auto k = k_sketch_left_fx<float, NWF>;
      hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k, g1, dim3(NWF * 64), lds, st, (const float*)X, ldx, nullptr, 0, table, s, M, N, r1, cw,
                         chunks, rps, out, ldo, part, scale, work);
    } else if (dtype == 2) {
      auto k = k_sketch_left_fx<uint16_t, NWF>;
      hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k, g1, dim3(NWF * 64), lds, st, (const uint16_t*)X, ldx, nullptr, 0, table, s, M, N, r1,
                         cw, chunks, rps, out, ldo, part, scale, work);
    } else {
      auto k = k_sketch_left_fx<uint8_t, NWF>;
      hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(k, g1, dim3(NWF * 64), lds, st, (const uint8_t*)X, ldx, scales, ldsc, table, s, M, N, r1,
                         cw, chunks, rps, out, ldo, part, scale, work);
    }
    if (splits > 1) {
      int64_t tot = (int64_t)r1 * N;
      hipLaunchKernelGGL(k_reduce_partial, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, partial, splits,
                         (int64_t)r1, N, out, ldo, scale);
    }
    return hipGetLastError();
  }
  if (dtype == 0) {
    auto k = k_sketch_left<float, NW>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const float*)X, ldx, nullptr, 0, table, s, M, N, r1, cw, rps,
                       out, ldo, part, scale);
  } else if (dtype == 2) {
    auto k = k_sketch_left<uint16_t, NW>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const uint16_t*)X, ldx, nullptr, 0, table, s, M, N, r1, cw,
                       rps, out, ldo, part, scale);
  } else if (dtype == 3 && scales) {
    auto k = k_sketch_left<uint8_t, NW>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), lds, st, (const uint8_t*)X, ldx, scales, ldsc, table, s, M, N, r1, cw,
                       rps, out, ldo, part, scale);
  } else {
    return hipErrorInvalidValue;
  }
  if (splits > 1) {
    int64_t tot = (int64_t)r1 * N;
    hipLaunchKernelGGL(k_reduce_partial, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, partial, splits,
                       (int64_t)r1, N, out, ldo, scale);
  }
  return hipGetLastError();
}

}  // namespace rf
