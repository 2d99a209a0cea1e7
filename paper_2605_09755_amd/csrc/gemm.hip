// K5/K6: dense products on MFMA.  C = alpha * op(A) op(B), FP32 accumulation.
//
// These are the tall-skinny contractions of the power loop (At Z over r1,
// At^T Q over m -- Algorithm 1, line 1), the randomised-SVD product Q^T A
// (Section 2), the CholeskyQR apply Y R^{-1}, and the small Ritz products.
//
// Tile: 128 x 128 per workgroup, 4 waves in 2 x 2, each wave 64 x 64 as 2 x 2
// MFMA 32x32 blocks.  FP32 operands use v_mfma_f32_32x32x2f32 (one value per
// lane per block), BF16 operands use v_mfma_f32_32x32x16_bf16 (eight k-consecutive
// values per lane).  Operands are staged global -> registers -> LDS with double
// buffering and one barrier per k-step.  Either operand may be k-contiguous
// ("K" layout) or m/n-contiguous ("T" layout); BF16 T-layout tiles are transposed
// in registers (2 x 8 blocks) on their way into LDS, which always stores BF16
// k-contiguous.  Split-K writes FP32 partials that a second kernel sums in
// fixed order (deterministic).
#include <algorithm>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rf {

constexpr int GBM = 128, GBN = 128;

// x where keep holds, else +0: a bit mask rather than a select, so the compiler
// keeps the load unconditional (a select of a loaded value can become a branch
// around the load, with a wait right after it)
RF_DEV float keep_or_zero(float x, bool keep) { return __uint_as_float(__float_as_uint(x) & (keep ? ~0u : 0u)); }

RF_DEV void tile_coords(int id, int ntm, int ntn, int& tm, int& tn) {
  // XCD-aware order: consecutive workgroup ids go to different XCDs (id % 8);
  // give each XCD whole M-panels and walk their N tiles back to back so the
  // panel stays in that XCD's L2.
  if (ntm % 8 == 0 && ntn > 1) {
    int xcd = id & 7, local = id >> 3;
    tn = local % ntn;
    tm = (local / ntn) * 8 + xcd;
  } else {
    tn = id % ntn;
    tm = id / ntn;
  }
}

RF_DEV void store_out(const GemmArgs& g, int64_t i, int64_t j, float v) {
  if (i >= g.M || j >= g.N) return;
  v *= g.alpha;
  if (g.colscale) v *= as_global<float>(g.colscale)[j];
  if (g.c_bf16) {
    const gptr<uint16_t> C = as_global_w<uint16_t>(g.C);
    C[g.c_trans ? j * g.ldc + i : i * g.ldc + j] = f32_to_bf16_rne(v);
  } else {
    const gptr<float> C = as_global_w<float>(g.C);
    C[g.c_trans ? j * g.ldc + i : i * g.ldc + j] = v;
  }
}

// ---------------- FP32 operands -------------------------------------------------------
// VEC: the launcher has checked that both operands take the 16-byte form (true) or
// runs the element form for both (false); each instance compiles one form only:
// with both forms, the compiler merged them into the same registers and waited for
// each chunk's loads before issuing the next chunk's.
template <bool AKC, bool BKC, bool VEC>
RF_DEV void gemm_f32_body(const GemmArgs& g, int bid, int split) {
  constexpr int BK = 16;          // 32 (two workgroups per CU instead of three) measured slower
  constexpr int NPS = BK / 8;     // load passes per operand and step
  constexpr int TPR = BK / 4;     // threads per row of a k-contiguous tile
  constexpr int RPP = 256 / TPR;  // rows per pass of a k-contiguous tile
  constexpr int AST = AKC ? (BK + 1) : GBM;  // LDS row stride (floats)
  constexpr int BST = BKC ? (BK + 1) : GBN;
  constexpr int ASZ = AKC ? GBM * (BK + 1) : BK * GBM;
  constexpr int BSZ = BKC ? GBN * (BK + 1) : BK * GBN;
  __shared__ float As[2][ASZ];
  __shared__ float Bs[2][BSZ];

  const int ntm = (int)((g.M + GBM - 1) / GBM), ntn = (int)((g.N + GBN - 1) / GBN);
  int tm, tn;
  tile_coords(bid, ntm, ntn, tm, tn);
  const int64_t i0 = (int64_t)tm * GBM, j0 = (int64_t)tn * GBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t kbeg = (int64_t)split * g.kps;
  int64_t kend = min(g.K, kbeg + g.kps);
  if (g.b_upper) kend = min(kend, j0 + GBN);
  const gptr<const float> A = as_global<float>(g.A);
  const gptr<const float> B = as_global<float>(g.B);

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  float ra[NPS][4], rb[NPS][4];
  // 16-byte loads when the operand allows them for every chunk (aligned, and its
  // contiguous extent a multiple of 4, so a chunk is wholly inside or wholly past
  // the edge, and one past the edge is zero without a load); otherwise clamped
  // element loads, zero past the edge.  The choice is uniform over the launch: a
  // per-chunk mix of the two forms made the compiler wait for every outstanding
  // load before each 16-byte one (both write the same registers).
  constexpr bool avec = VEC, bvec = VEC;
  // four consecutive elements of P along the contiguous index (x0 .. x0+3 < xmax)
  // of line y (< ymax: the other index), into d
  auto load4 = [&](gptr<const float> P, int64_t ld, int64_t y, int64_t ymax, int64_t x0, int64_t xmax, bool vec,
                   float* d) {
    if (vec) {
      if (y < ymax && x0 < xmax) {
        const float4 v = *reinterpret_cast<gptr<const float4>>(P + y * ld + x0);
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      } else {
        d[0] = d[1] = d[2] = d[3] = 0.f;
      }
    } else {
      // raw loads from clamped addresses; the entries outside the operand are
      // zeroed by mask4 when the stage is stored, so no load waits before the MFMAs
      const int64_t yc = min(y, ymax - 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) d[e] = P[yc * ld + min(x0 + e, xmax - 1)];
    }
  };
  auto mask4 = [&](int64_t y, int64_t ymax, int64_t x0, int64_t xmax, float* d) {
#pragma unroll
    for (int e = 0; e < 4; ++e) d[e] = keep_or_zero(d[e], y < ymax && x0 + e < xmax);
  };
  int64_t kreg = 0;  // first k of the stage held in ra / rb
  auto gload = [&](int64_t k0) {
    kreg = k0;
#pragma unroll
    for (int ps = 0; ps < NPS; ++ps) {
      if (AKC) {
        int row = tid / TPR + RPP * ps, kc = (tid % TPR) * 4;
        load4(A, g.lda, i0 + row, g.M, k0 + kc, kend, avec, ra[ps]);
      } else {
        int kr = (tid >> 5) + 8 * ps, ic = (tid & 31) * 4;
        load4(A, g.lda, k0 + kr, kend, i0 + ic, g.M, avec, ra[ps]);
      }
      if (BKC) {
        int row = tid / TPR + RPP * ps, kc = (tid % TPR) * 4;
        load4(B, g.ldb, j0 + row, g.N, k0 + kc, kend, bvec, rb[ps]);
      } else {
        int kr = (tid >> 5) + 8 * ps, jc = (tid & 31) * 4;
        load4(B, g.ldb, k0 + kr, kend, j0 + jc, g.N, bvec, rb[ps]);
      }
    }
  };
  auto sstore = [&](int buf) {
    if constexpr (!VEC) {
#pragma unroll
      for (int ps = 0; ps < NPS; ++ps) {
        if (AKC) mask4(i0 + tid / TPR + RPP * ps, g.M, kreg + (tid % TPR) * 4, kend, ra[ps]);
        else mask4(kreg + (tid >> 5) + 8 * ps, kend, i0 + (tid & 31) * 4, g.M, ra[ps]);
        if (BKC) mask4(j0 + tid / TPR + RPP * ps, g.N, kreg + (tid % TPR) * 4, kend, rb[ps]);
        else mask4(kreg + (tid >> 5) + 8 * ps, kend, j0 + (tid & 31) * 4, g.N, rb[ps]);
      }
    }
#pragma unroll
    for (int ps = 0; ps < NPS; ++ps) {
      if (AKC) {
        int row = tid / TPR + RPP * ps, kc = (tid % TPR) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][row * AST + kc + e] = ra[ps][e];
      } else {
        int kr = (tid >> 5) + 8 * ps, ic = (tid & 31) * 4;
        *reinterpret_cast<float4*>(&As[buf][kr * AST + ic]) = make_float4(ra[ps][0], ra[ps][1], ra[ps][2], ra[ps][3]);
      }
      if (BKC) {
        int row = tid / TPR + RPP * ps, kc = (tid % TPR) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) Bs[buf][row * BST + kc + e] = rb[ps][e];
      } else {
        int kr = (tid >> 5) + 8 * ps, jc = (tid & 31) * 4;
        *reinterpret_cast<float4*>(&Bs[buf][kr * BST + jc]) = make_float4(rb[ps][0], rb[ps][1], rb[ps][2], rb[ps][3]);
      }
    }
  };

  const int nk = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kbeg + (int64_t)(kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 2; ++kk) {
      const int kidx = 2 * kk + (lane >> 5);
      float af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        int ii = wm * 64 + a * 32 + (lane & 31);
        af[a] = AKC ? As[buf][ii * AST + kidx] : As[buf][kidx * AST + ii];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        int jj = wn * 64 + b * 32 + (lane & 31);
        bf[b] = BKC ? Bs[buf][jj * BST + kidx] : Bs[buf][kidx * BST + jj];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int64_t i = i0 + wm * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        int64_t j = j0 + wn * 64 + b * 32 + (lane & 31);
        if (g.partial) {
          if (i < g.M && j < g.N) as_global_w<float>(g.partial)[((int64_t)split * g.M + i) * g.N + j] = acc[a][b][r];
        } else {
          store_out(g, i, j, acc[a][b][r]);
        }
      }
}

// ---------------- BF16 operands -------------------------------------------------------
RF_DEV uint32_t pack_lo(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
RF_DEV uint32_t pack_hi(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }

RF_DEV uint32_t pack2_bf16(float a, float b) { return pk_bf16(a, b); }

// AF32: the A operand is FP32 in memory and rounded to BF16 (RNE) as it is loaded.
// DEFER: every operand takes the element form, and the raw loads are masked,
// rounded and packed only when the stage is stored (the loads stay in flight across
// the MFMA phase); the grouped launches run it (their problems are ragged).
template <bool AKC, bool BKC, bool AF32 = false, bool DEFER = false>
RF_DEV void gemm_bf16_body(const GemmArgs& g, int bid, int split) {
  constexpr int BK = 32;
  constexpr int ST = BK + 8;  // bf16 elements per LDS row (80 B)
  __shared__ __attribute__((aligned(16))) uint16_t As[2][GBM * ST];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][GBN * ST];

  const int ntm = (int)((g.M + GBM - 1) / GBM), ntn = (int)((g.N + GBN - 1) / GBN);
  int tm, tn;
  tile_coords(bid, ntm, ntn, tm, tn);
  const int64_t i0 = (int64_t)tm * GBM, j0 = (int64_t)tn * GBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t kbeg = (int64_t)split * g.kps;
  int64_t kend = min(g.K, kbeg + g.kps);
  if (g.b_upper) kend = min(kend, j0 + GBN);
  const gptr<const uint16_t> A = as_global<uint16_t>(g.A);
  const gptr<const uint16_t> B = as_global<uint16_t>(g.B);

  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  // staging registers: 2 x uint4 per operand (16 bf16)
  uint4 sa[2], sb[2];

  // Loads take one form per launch: vector loads when every chunk is either wholly
  // inside the operand or wholly past its edge (aligned, contiguous extent a multiple
  // of the chunk; a chunk past the edge is zero without a load), else clamped
  // element loads, all issued before they are combined.  (Mixing the two forms per
  // chunk made the compiler wait for all outstanding loads at each chunk.)
  // K layout: 128 rows x 32 k; thread: row (tid>>2)+64ps, k chunk (tid&3)*8.
  auto load_kc = [&](gptr<const uint16_t> P, int64_t ld, int64_t r0, int64_t rmax, int64_t k0, uint4* dst, bool vec) {
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
      int row = (tid >> 2) + 64 * ps, kc = (tid & 3) * 8;
      int64_t r = r0 + row, k = k0 + kc;
      if (vec) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r < rmax && k < kend) v = *reinterpret_cast<gptr<const uint4>>(P + r * ld + k);
        dst[ps] = v;
      } else {
        const int64_t rc = min(r, rmax - 1);
        uint32_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = P[rc * ld + min(k + e, kend - 1)];
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (r < rmax && k + e < kend) ? h[e] : 0u;
        dst[ps] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
      }
    }
  };
  // T layout: element (r, k) at P[k*ld + r].  Wave w covers k rows 8w..8w+7,
  // lane covers r pair (2 lane, 2 lane + 1); produces two k-vectors of 8.
  auto load_tc = [&](gptr<const uint16_t> P, int64_t ld, int64_t r0, int64_t rmax, int64_t k0, uint4* dst, bool vec) {
    uint32_t w[8];
    int64_t r = r0 + 2 * lane;
    if (vec) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int64_t k = k0 + 8 * wave + e;
        w[e] = (k < kend && r < rmax) ? *reinterpret_cast<gptr<const uint32_t>>(P + k * ld + r) : 0u;
      }
    } else {
      const int64_t r0c = min(r, rmax - 1), r1c = min(r + 1, rmax - 1);
      uint32_t lo[8], hi[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t kc = min(k0 + 8 * wave + e, kend - 1);
        lo[e] = P[kc * ld + r0c];
        hi[e] = P[kc * ld + r1c];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool kin = k0 + 8 * wave + e < kend;
        w[e] = (kin && r < rmax ? lo[e] : 0u) | ((kin && r + 1 < rmax ? hi[e] : 0u) << 16);
      }
    }
    dst[0] = make_uint4(pack_lo(w[0], w[1]), pack_lo(w[2], w[3]), pack_lo(w[4], w[5]), pack_lo(w[6], w[7]));
    dst[1] = make_uint4(pack_hi(w[0], w[1]), pack_hi(w[2], w[3]), pack_hi(w[4], w[5]), pack_hi(w[6], w[7]));
  };
  auto store_kc = [&](uint16_t* S, const uint4* src) {
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
      int row = (tid >> 2) + 64 * ps, kc = (tid & 3) * 8;
      *reinterpret_cast<uint4*>(S + row * ST + kc) = src[ps];
    }
  };
  auto store_tc = [&](uint16_t* S, const uint4* src) {
    *reinterpret_cast<uint4*>(S + (2 * lane) * ST + 8 * wave) = src[0];
    *reinterpret_cast<uint4*>(S + (2 * lane + 1) * ST + 8 * wave) = src[1];
  };
  // FP32 A, same element positions as load_kc / load_tc, rounded to BF16
  const gptr<const float> Af = as_global<float>(g.A);
  auto load_kc_f32 = [&](int64_t r0, int64_t rmax, int64_t k0, uint4* dst, bool vec) {
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
      int row = (tid >> 2) + 64 * ps, kc = (tid & 3) * 8;
      int64_t r = r0 + row, k = k0 + kc;
      float t[8];
      if (vec) {
        float4 x0 = make_float4(0.f, 0.f, 0.f, 0.f), x1 = x0;
        if (r < rmax && k < kend) {
          x0 = *reinterpret_cast<gptr<const float4>>(Af + r * g.lda + k);
          x1 = *reinterpret_cast<gptr<const float4>>(Af + r * g.lda + k + 4);
        }
        t[0] = x0.x; t[1] = x0.y; t[2] = x0.z; t[3] = x0.w; t[4] = x1.x; t[5] = x1.y; t[6] = x1.z; t[7] = x1.w;
      } else {
        const int64_t rc = min(r, rmax - 1);
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = Af[rc * g.lda + min(k + e, kend - 1)];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = keep_or_zero(t[e], r < rmax && k + e < kend);
      }
      dst[ps] = make_uint4(pack2_bf16(t[0], t[1]), pack2_bf16(t[2], t[3]), pack2_bf16(t[4], t[5]),
                           pack2_bf16(t[6], t[7]));
    }
  };
  auto load_tc_f32 = [&](int64_t r0, int64_t rmax, int64_t k0, uint4* dst, bool vec) {
    uint32_t w[8];
    int64_t r = r0 + 2 * lane;
    float lo[8], hi[8];
    if (vec) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int64_t k = k0 + 8 * wave + e;
        float2 x = make_float2(0.f, 0.f);
        if (k < kend && r < rmax) x = *reinterpret_cast<gptr<const float2>>(Af + k * g.lda + r);
        lo[e] = x.x; hi[e] = x.y;
      }
    } else {
      const int64_t r0c = min(r, rmax - 1), r1c = min(r + 1, rmax - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t kc = min(k0 + 8 * wave + e, kend - 1);
        lo[e] = Af[kc * g.lda + r0c];
        hi[e] = Af[kc * g.lda + r1c];
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool kin = k0 + 8 * wave + e < kend;
        lo[e] = keep_or_zero(lo[e], kin && r < rmax);
        hi[e] = keep_or_zero(hi[e], kin && r + 1 < rmax);
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = pack2_bf16(lo[e], hi[e]);
    dst[0] = make_uint4(pack_lo(w[0], w[1]), pack_lo(w[2], w[3]), pack_lo(w[4], w[5]), pack_lo(w[6], w[7]));
    dst[1] = make_uint4(pack_hi(w[0], w[1]), pack_hi(w[2], w[3]), pack_hi(w[4], w[5]), pack_hi(w[6], w[7]));
  };
  // (k chunks are 8 wide and split parts start on multiples of 32, so a K that is a
  // multiple of 8 keeps every k chunk whole; m/n pairs need an even extent)
  const bool kwhole = (g.K % 8 == 0) && (g.kps % 8 == 0);
  const bool avec = AF32 ? (AKC ? ((((uintptr_t)Af) & 15) == 0 && (g.lda & 3) == 0 && kwhole)
                                : ((((uintptr_t)Af) & 7) == 0 && (g.lda & 1) == 0 && (g.M % 2 == 0)))
                         : (AKC ? ((((uintptr_t)A) & 15) == 0 && (g.lda & 7) == 0 && kwhole)
                                : ((((uintptr_t)A) & 3) == 0 && (g.lda & 1) == 0 && (g.M % 2 == 0)));
  const bool bvec = BKC ? ((((uintptr_t)B) & 15) == 0 && (g.ldb & 7) == 0 && kwhole)
                        : ((((uintptr_t)B) & 3) == 0 && (g.ldb & 1) == 0 && (g.N % 2 == 0));
  // deferred element form: raw 32-bit words (BF16 values or FP32 bits) at the
  // positions load_kc / load_tc use, from clamped addresses
  uint32_t raw_a[16], raw_b[16];
  int64_t kreg = 0;
  auto raw_kc = [&](auto P, int64_t ld, int64_t r0, int64_t rmax, int64_t k0, uint32_t* raw) {
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
      const int64_t rc = min(r0 + (tid >> 2) + 64 * ps, rmax - 1), k = k0 + (tid & 3) * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const auto v = P[rc * ld + min(k + e, kend - 1)];
        if constexpr (sizeof(v) == 4) raw[8 * ps + e] = __float_as_uint(v);
        else raw[8 * ps + e] = v;
      }
    }
  };
  auto raw_tc = [&](auto P, int64_t ld, int64_t r0, int64_t rmax, int64_t k0, uint32_t* raw) {
    const int64_t r = r0 + 2 * lane, r0c = min(r, rmax - 1), r1c = min(r + 1, rmax - 1);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t kc = min(k0 + 8 * wave + e, kend - 1);
      const auto lo = P[kc * ld + r0c], hi = P[kc * ld + r1c];
      if constexpr (sizeof(lo) == 4) {
        raw[e] = __float_as_uint(lo);
        raw[8 + e] = __float_as_uint(hi);
      } else {
        raw[e] = lo;
        raw[8 + e] = hi;
      }
    }
  };
  // two entries (FP32 bits if F32) as a packed BF16 pair, each zero unless kept
  auto pair = [&](uint32_t x, bool kx, uint32_t y, bool ky, bool f32) -> uint32_t {
    if (f32) return pack2_bf16(keep_or_zero(__uint_as_float(x), kx), keep_or_zero(__uint_as_float(y), ky));
    return (kx ? x : 0u) | ((ky ? y : 0u) << 16);
  };
  auto pack_kc = [&](const uint32_t* raw, int64_t r0, int64_t rmax, bool f32, uint4* dst) {
#pragma unroll
    for (int ps = 0; ps < 2; ++ps) {
      const int64_t r = r0 + (tid >> 2) + 64 * ps, k = kreg + (tid & 3) * 8;
      const bool rin = r < rmax;
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w[e] = pair(raw[8 * ps + 2 * e], rin && k + 2 * e < kend, raw[8 * ps + 2 * e + 1], rin && k + 2 * e + 1 < kend, f32);
      dst[ps] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  };
  auto pack_tc = [&](const uint32_t* raw, int64_t r0, int64_t rmax, bool f32, uint4* dst) {
    const int64_t r = r0 + 2 * lane;
    uint32_t w[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const bool kin = kreg + 8 * wave + e < kend;
      w[e] = pair(raw[e], kin && r < rmax, raw[8 + e], kin && r + 1 < rmax, f32);
    }
    dst[0] = make_uint4(pack_lo(w[0], w[1]), pack_lo(w[2], w[3]), pack_lo(w[4], w[5]), pack_lo(w[6], w[7]));
    dst[1] = make_uint4(pack_hi(w[0], w[1]), pack_hi(w[2], w[3]), pack_hi(w[4], w[5]), pack_hi(w[6], w[7]));
  };
  auto gload = [&](int64_t k0) {
    if constexpr (DEFER) {
      kreg = k0;
      if constexpr (AF32) {
        if (AKC) raw_kc(Af, g.lda, i0, g.M, k0, raw_a); else raw_tc(Af, g.lda, i0, g.M, k0, raw_a);
      } else {
        if (AKC) raw_kc(A, g.lda, i0, g.M, k0, raw_a); else raw_tc(A, g.lda, i0, g.M, k0, raw_a);
      }
      if (BKC) raw_kc(B, g.ldb, j0, g.N, k0, raw_b); else raw_tc(B, g.ldb, j0, g.N, k0, raw_b);
      return;
    }
    if constexpr (AF32) {
      if (AKC) load_kc_f32(i0, g.M, k0, sa, avec); else load_tc_f32(i0, g.M, k0, sa, avec);
    } else {
      if (AKC) load_kc(A, g.lda, i0, g.M, k0, sa, avec); else load_tc(A, g.lda, i0, g.M, k0, sa, avec);
    }
    if (BKC) load_kc(B, g.ldb, j0, g.N, k0, sb, bvec); else load_tc(B, g.ldb, j0, g.N, k0, sb, bvec);
  };
  auto sstore = [&](int buf) {
    if constexpr (DEFER) {
      if (AKC) pack_kc(raw_a, i0, g.M, AF32, sa); else pack_tc(raw_a, i0, g.M, AF32, sa);
      if (BKC) pack_kc(raw_b, j0, g.N, false, sb); else pack_tc(raw_b, j0, g.N, false, sb);
    }
    if (AKC) store_kc(As[buf], sa); else store_tc(As[buf], sa);
    if (BKC) store_kc(Bs[buf], sb); else store_tc(Bs[buf], sb);
  };

  const int nk = kend > kbeg ? (int)((kend - kbeg + BK - 1) / BK) : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kbeg + (int64_t)(kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 16; ++kk) {
      const int koff = 16 * kk + 8 * (lane >> 5);
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        int ii = wm * 64 + a * 32 + (lane & 31);
        af[a] = *reinterpret_cast<const bf16x8*>(&As[buf][ii * ST + koff]);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        int jj = wn * 64 + b * 32 + (lane & 31);
        bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[buf][jj * ST + koff]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int64_t i = i0 + wm * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        int64_t j = j0 + wn * 64 + b * 32 + (lane & 31);
        if (g.partial) {
          if (i < g.M && j < g.N) as_global_w<float>(g.partial)[((int64_t)split * g.M + i) * g.N + j] = acc[a][b][r];
        } else {
          store_out(g, i, j, acc[a][b][r]);
        }
      }
}

// ---------------- BF16 operands, 256 x 256 tiles ----------------------------------------
// For the large products (Q^T A, the power-loop products at full size).  4 waves,
// each 128 x 128 = 4 x 4 MFMA 32x32x16 blocks (256 accumulators per lane).  LDS
// keeps every operand tile in the layout it has in memory, so global loads and LDS
// stores are 16-byte vectors on both layouts:
//  * k-contiguous operands: rows of 32 k (+8 pad, 80 B: 16 lanes reading 16 B each
//    hit 16 disjoint bank quads); a lane's 8 k values are one ds_read_b128;
//  * m/n-contiguous operands: rows of 256 (+32 pad, 576 B = 64 mod 256 B, so the 8
//    rows touched by one read fall on two disjoint sets of bank columns); a lane's
//    8 k values come from two ds_read_b64_tr_b16, which hand lane i of a 16-lane
//    group element i%4 of the 8-byte chunks addressed by lanes i/4, i/4+4, i/4+8,
//    i/4+12 -- so when lane s of the group addresses row k0+s/4, column c0+4(s%4),
//    lane i receives column c0+i at rows k0..k0+3.
// With AF32 the A operand is FP32 in memory and rounded to BF16 (RNE) on its way
// into LDS.
typedef __bf16 bf16x4v __attribute__((__vector_size__(4 * sizeof(__bf16))));
constexpr int HB = 256, HBK = 64;  // 64 k-rows per stage keep two stages of loads in flight per CU
constexpr int BT = 512;        // threads of a 256 x 256 workgroup: 8 waves, two per SIMD
constexpr int NCH = HB * HBK / 8 / BT;  // 8-element chunks per thread and operand per stage
constexpr int TRL = HB + 32;   // m/n-contiguous LDS row, bf16 elements
constexpr int KRL = HBK + 8;   // k-contiguous LDS row, bf16 elements (144 B: odd multiple of 16)
constexpr int KCH = HBK / 8;   // 8-element chunks per k-contiguous row

template <bool KC>
constexpr int big_stage_elems() { return KC ? HB * KRL : HBK * TRL; }

RF_DEV bf16x8 big_frag_kc(const uint16_t* S, int row, int k) {
  return *reinterpret_cast<const bf16x8*>(S + row * KRL + k);
}

RF_DEV bf16x8 big_frag_tc(const uint16_t* S, int col0, int k0, int lane) {
  const int g = lane >> 4, s = lane & 15;
  const int col = col0 + 16 * (g & 1) + 4 * (s & 3);
  const int kr = k0 + 8 * (g >> 1) + (s >> 2);
  const uint16_t* p0 = S + kr * TRL + col;
  const uint16_t* p1 = p0 + 4 * TRL;
  bf16x4v lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((__attribute__((address_space(3))) bf16x4v*)p0);
  bf16x4v hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((__attribute__((address_space(3))) bf16x4v*)p1);
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

RF_DEV uint4 pack8_bf16(float4 a, float4 b) {
  return make_uint4(pk_bf16(a.x, a.y), pk_bf16(a.z, a.w), pk_bf16(b.x, b.y), pk_bf16(b.z, b.w));
}

// One operand's share of a stage: NCH chunks of 8 consecutive elements per thread.
// KC: chunk c -> row c/KCH of the tile, k offset 8 (c%KCH) (KCH = HBK/8 chunks per
// row); else k row c/32, column 8 (c%32).
template <bool KC, int MODE>  // MODE 0: BF16, 1: FP32, 2: FP8 e4m3 x block scale (m/n-contiguous only)
struct BigStage {
  static constexpr bool F32 = (MODE == 1);
  static constexpr bool F8 = (MODE == 2);
  static_assert(!(F8 && KC), "FP8 operands are read m/n-contiguous");
  uint4 v[NCH];
  float4 f[NCH][2];
  uint2 b8[NCH];
  float sc[NCH];
  // A chunk wholly outside the operand is zero without a load; a chunk that straddles
  // its edge (or an unaligned operand) reads each element from an address clamped into
  // the operand and zeroes the elements outside it.  Both stay branch-free per lane so
  // the loads of a stage stay in flight together.
  RF_DEV void load(const void* P_, int64_t ld, int64_t r0, int64_t rmax, int64_t k0, int64_t kend, bool vec,
                   int tid, const float* scales = nullptr, int64_t ldsc = 0) {
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = tid + BT * q;
      const int64_t r = KC ? r0 + c / KCH : r0 + 8 * (c & 31);         // first m/n index of the chunk
      const int64_t k = KC ? k0 + 8 * (c % KCH) : k0 + (c >> 5);       // first k index of the chunk
      const bool any = r < rmax && k < kend;
      const bool full = KC ? (r < rmax && k + 8 <= kend) : (k < kend && r + 8 <= rmax);
      // element e of the chunk: in range, and its clamped offset from the operand start
      auto in = [&](int e) { return KC ? (k + e < kend) : (r + e < rmax); };
      auto at = [&](int e) {
        return KC ? r * ld + min(k + e, kend - 1) : k * ld + min(r + e, rmax - 1);
      };
      if constexpr (F8) {
        const gptr<const uint8_t> P = as_global<uint8_t>(P_);
        sc[q] = any ? as_global<float>(scales)[(k >> 7) * ldsc + (r >> 7)] : 0.f;
        if (vec && full) {
          b8[q] = *reinterpret_cast<gptr<const uint2>>(P + k * ld + r);
        } else if (!any) {
          b8[q] = make_uint2(0u, 0u);
        } else {
          uint32_t w[2] = {0u, 0u};
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t b = P[at(e)];
            w[e >> 2] |= (in(e) ? b : 0u) << (8 * (e & 3));
          }
          b8[q] = make_uint2(w[0], w[1]);
        }
      } else if constexpr (F32) {
        const gptr<const float> P = as_global<float>(P_);
        if (vec && full) {
          const gptr<const float> src = KC ? P + r * ld + k : P + k * ld + r;
          f[q][0] = *reinterpret_cast<gptr<const float4>>(src);
          f[q][1] = *reinterpret_cast<gptr<const float4>>(src + 4);
        } else if (!any) {
          f[q][0] = f[q][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
          float t[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float x = P[at(e)];
            t[e] = in(e) ? x : 0.f;
          }
          f[q][0] = make_float4(t[0], t[1], t[2], t[3]);
          f[q][1] = make_float4(t[4], t[5], t[6], t[7]);
        }
      } else {
        const gptr<const uint16_t> P = as_global<uint16_t>(P_);
        if (vec && full) {
          v[q] = *reinterpret_cast<gptr<const uint4>>(KC ? P + r * ld + k : P + k * ld + r);
        } else if (!any) {
          v[q] = make_uint4(0u, 0u, 0u, 0u);
        } else {
          uint32_t h[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint32_t x = P[at(e)];
            h[e] = in(e) ? x : 0u;
          }
          v[q] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
        }
      }
    }
  }
  RF_DEV void store(uint16_t* S, int tid) const {
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = tid + BT * q;
      uint16_t* dst = KC ? S + (c / KCH) * KRL + 8 * (c % KCH) : S + (c >> 5) * TRL + 8 * (c & 31);
      uint4 x;
      if constexpr (F8) {
        float t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = 0.f;
        fp8x4_to_f32(b8[q].x, t);
        fp8x4_to_f32(b8[q].y, t + 4);
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] *= sc[q];
        x = pack8_bf16(make_float4(t[0], t[1], t[2], t[3]), make_float4(t[4], t[5], t[6], t[7]));
      } else if constexpr (F32) {
        x = pack8_bf16(f[q][0], f[q][1]);
      } else {
        x = v[q];
      }
      *reinterpret_cast<uint4*>(dst) = x;
    }
  }
};

// L2 warm-up of a later stage: one byte of each 128-byte line of an operand's stage
// tile (at most one line per thread), so the stage's own loads find the tile in L2.
// Returns the byte, which the caller keeps alive.
template <bool KC, int MODE>
RF_DEV uint32_t big_touch(const void* P_, int64_t ld, int64_t r0, int64_t rmax, int64_t k0, int64_t kend, int tid) {
  constexpr int es = MODE == 1 ? 4 : (MODE == 2 ? 1 : 2);
  constexpr int rowb = (KC ? HBK : HB) * es;        // bytes of one tile row in memory
  constexpr int lpr = rowb >= 128 ? rowb / 128 : 1;  // lines per tile row
  constexpr int nlines = (KC ? HB : HBK) * lpr;
  static_assert(nlines <= BT, "one line per thread");
  if (tid >= nlines) return 0u;
  const int row = tid / lpr, off = (tid % lpr) * (128 / es);
  const int64_t r = KC ? r0 + row : r0 + off, k = KC ? k0 + off : k0 + row;
  if (r >= rmax || k >= kend) return 0u;
  const gptr<const uint8_t> P = as_global<uint8_t>(P_);
  return P[(KC ? r * ld + k : k * ld + r) * es];
}

// Epilogue of the 256 x 256 kernels (wave (wm, wn) holds rows wm*128 + 32a + ..,
// columns wn*64 + 32b + .. in acc[a][b]), through LDS one 64-row slab (rows 32a.. of
// both wave rows) at a time: the accumulator copy is fully unrolled (registers only),
// the global stores are row-contiguous across the workgroup.
// NB: 32-column blocks per wave (wave column wn starts at column 32 NB wn); NT: threads.
template <int NB = 2, int NT = BT>
RF_DEV void big_epilogue(const GemmArgs& g, f32x16 (&acc)[4][NB], int64_t i0, int64_t j0, int split, int wm, int wn,
                         int lane, int tid, void* smem) {
  constexpr int SLD = HB + 8;  // 264 floats: lanes 32..63 (4 rows down) land on the other 32 banks
  float* St = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        St[(wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)) * SLD + wn * 32 * NB + 32 * b + (lane & 31)] =
            acc[a][b][r];
    __syncthreads();
    for (int e = tid; e < 64 * HB; e += NT) {
      const int rr = g.c_trans ? (e & 63) : (e / HB), cc = g.c_trans ? (e >> 6) : (e % HB);
      const int64_t i = i0 + (rr >> 5) * 128 + 32 * a + (rr & 31), j = j0 + cc;
      const float v = St[rr * SLD + cc];
      if (g.partial) {
        if (i < g.M && j < g.N) as_global_w<float>(g.partial)[((int64_t)split * g.M + i) * g.N + j] = v;
      } else {
        store_out(g, i, j, v);
      }
    }
    __syncthreads();
  }
}

template <bool AKC, bool BKC, int AMODE>
RF_DEV void gemm_bf16_big_body(const GemmArgs& g, int bid, int split) {
  extern __shared__ __attribute__((aligned(16))) uint16_t smem[];
  constexpr int AS = big_stage_elems<AKC>(), BS = big_stage_elems<BKC>();
  uint16_t* const A0 = smem;
  uint16_t* const B0 = smem + 2 * AS;

  const int ntm = (int)((g.M + HB - 1) / HB), ntn = (int)((g.N + HB - 1) / HB);
  int tm, tn;
  tile_coords(bid, ntm, ntn, tm, tn);
  const int64_t i0 = (int64_t)tm * HB, j0 = (int64_t)tn * HB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // wave tile: rows wm*128 + [0, 128), columns wn*64 + [0, 64)
  int64_t kbeg = (int64_t)split * g.kps;
  int64_t kend = min(g.K, kbeg + g.kps);
  if (g.b_upper) kend = min(kend, j0 + HB);

  const int aes = AMODE == 1 ? 4 : (AMODE == 2 ? 1 : 2);
  const int aal = AMODE == 2 ? 8 : 16;  // FP8 chunks are 8 bytes
  const bool avec = ((((uintptr_t)g.A) & (aal - 1)) == 0) && ((g.lda * aes) % aal == 0);
  const bool bvec = ((((uintptr_t)g.B) & 15) == 0) && ((g.ldb * 2) % 16 == 0);

  f32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  BigStage<AKC, AMODE> sa;
  BigStage<BKC, 0> sb;
  const int nk = kend > kbeg ? (int)((kend - kbeg + HBK - 1) / HBK) : 0;
  // FP32 A (twice the bytes of a BF16 stage) warms L2 for the stage after next; for
  // BF16 and FP8 A the warm-up measured slower (its wait lands in the next step)
  constexpr int PF = AMODE == 1 ? 1 : 0;
  uint32_t pf_sink = 0, pf_prev = 0;
  if (nk > 0) {
    sa.load(g.A, g.lda, i0, g.M, kbeg, kend, avec, tid, g.a_scales, g.a_ldsc);
    sb.load(g.B, g.ldb, j0, g.N, kbeg, kend, bvec, tid);
    sa.store(A0, tid);
    sb.store(B0, tid);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) {
      const int64_t k1 = kbeg + (int64_t)(kt + 1) * HBK;
      sa.load(g.A, g.lda, i0, g.M, k1, kend, avec, tid, g.a_scales, g.a_ldsc);
      sb.load(g.B, g.ldb, j0, g.N, k1, kend, bvec, tid);
    }
    const uint16_t* A_ = A0 + buf * AS;
    const uint16_t* B_ = B0 + buf * BS;
#pragma unroll
    for (int kk = 0; kk < HBK / 16; ++kk) {
      bf16x8 af[4], bfr[2];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        af[a] = AKC ? big_frag_kc(A_, wm * 128 + 32 * a + (lane & 31), 16 * kk + 8 * (lane >> 5))
                    : big_frag_tc(A_, wm * 128 + 32 * a, 16 * kk, lane);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bfr[b] = BKC ? big_frag_kc(B_, wn * 64 + 32 * b + (lane & 31), 16 * kk + 8 * (lane >> 5))
                     : big_frag_tc(B_, wn * 64 + 32 * b, 16 * kk, lane);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      sa.store(A0 + (buf ^ 1) * AS, tid);
      sb.store(B0 + (buf ^ 1) * BS, tid);
    }
    // issued after this step's stage loads were waited for
    if constexpr (PF > 0) {
      pf_sink += pf_prev;
      pf_prev = 0u;
      if (kt + 1 + PF < nk)
        pf_prev = big_touch<AKC, AMODE>(g.A, g.lda, i0, g.M, kbeg + (int64_t)(kt + 1 + PF) * HBK, kend, tid);
    }
    __syncthreads();
  }

  if constexpr (PF > 0) asm volatile("" ::"v"(pf_sink + pf_prev));
  big_epilogue(g, acc, i0, j0, split, wm, wn, lane, tid, smem);
}

template <bool AKC, bool BKC, bool VEC>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs g) {
  gemm_f32_body<AKC, BKC, VEC>(g, blockIdx.x, blockIdx.y);
}
// whether both operands allow the 16-byte form: aligned, and every chunk wholly inside
// the operand or wholly past its edge
static bool f32_vec_ok(const GemmArgs& g) {
  const int64_t akx = g.a_kc ? g.K : g.M, bkx = g.b_kc ? g.K : g.N;
  return ((uintptr_t)g.A % 16 == 0) && (g.lda % 4 == 0) && (akx % 4 == 0) && ((uintptr_t)g.B % 16 == 0) &&
         (g.ldb % 4 == 0) && (bkx % 4 == 0) && (g.kps % 4 == 0);
}
template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  gemm_bf16_body<AKC, BKC>(g, blockIdx.x, blockIdx.y);
}
template <bool AKC, bool BKC, int AMODE>
__global__ __launch_bounds__(BT, 1) void k_gemm_bf16_big(GemmArgs g) {
  gemm_bf16_big_body<AKC, BKC, AMODE>(g, blockIdx.x, blockIdx.y);
}

// ---------------- FP8 operands: A^T Q with FP8-stored A --------------------------------
// C (M x N) = op(A) op(B) with op(A)(i,k) = A[k*lda+i] * a_scales[(k/128)*a_ldsc + i/128]
// (A stored K x M as e4m3 codes with one FP32 scale per 128 x 128 block) and op(B)(k,j)
// from the Q operand form of launch_quant_q_fp8 (e4m3 codes in MFMA order, one E8M0
// scale per 32 rows and column).  Both operands reach v_mfma_scale_f32_32x32x64_f8f6f4
// as stored, and every scale is applied without touching the codes:
//  * Q scales ride in the instruction (scale of column j, 32-deep k block b: lane 32 b + j);
//  * the A scale is one number per wave and 128-deep stage (a wave's 128 output rows
//    lie in one 128-column block of A).  Written s = 2^e mu (mu in [1/2, 1)), 2^e rides
//    in the instruction as the A-side E8M0 scale and mu is carried by the accumulators:
//    they hold the partial sum divided by the current stage's mu, are multiplied by
//    mu_prev / mu when a stage brings a different mu, and by the last mu at the end
//    (one rounding per change of mu, no second set of accumulators).
// k order inside one MFMA, the same for both operands: lane half h, byte p ->
// k = 32 (p / 16) + 16 h + p % 16 (bytes 16 b .. 16 b + 15 form scale block b).
// Workgroup tile 256 x 256, 8 waves of 128 x 64 (two per SIMD).  The A tile is kept
// in LDS in its memory layout (128 k rows of 256 bytes, pitch 288 = 32 mod 256, so the
// 8 rows x 32 bytes read by two 16-lane groups of one transposed read fall on
// distinct banks) and read
// with ds_read_b64_tr_b8, which hands lane i of a 16-lane group byte i % 8 of the
// 8-byte chunks addressed by lanes i / 8 + 2 t (t = 0..7): when lane s addresses row
// r0 + s / 2, column c0 + 8 (s % 2), lane i receives column c0 + i at rows r0 .. r0+7.
// The Q tile of a stage is one contiguous 32 KB run of its operand form, copied and
// read as 16-byte vectors.
typedef int f8i32x2 __attribute__((ext_vector_type(2)));
constexpr int F8K = 128;                   // k rows per stage: one A scale block
constexpr int F8P = HB + 32;               // LDS pitch of the A tile, bytes
constexpr int F8AS = F8K * F8P;            // A stage bytes
constexpr int F8QS = F8K * HB;             // Q stage bytes (2 chunks x 8 column blocks x 2 KB)
constexpr int F8CH = F8K * HB / 16 / BT;   // 16-byte chunks per thread and operand per stage

struct F8Stage {
  uint4 a[F8CH], q[F8CH];
  uint32_t qs[2];
  float sa;
  RF_DEV void load(const GemmArgs& g, int64_t i0, int64_t j0, int64_t k0, int64_t kend, bool avec, int tid,
                   int wm, int wn, int lane) {
    const uint8_t* A = reinterpret_cast<const uint8_t*>(g.A);
#pragma unroll
    for (int q = 0; q < F8CH; ++q) {
      const int c = tid + BT * q;
      const int64_t k = k0 + (c >> 4), i = i0 + 16 * (c & 15);
      const uint8_t* src = A + k * g.lda + i;
      if (avec && k < kend && i + 16 <= g.M) {
        a[q] = *reinterpret_cast<const uint4*>(src);
      } else {
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (k < kend)
          for (int e = 0; e < 16 && i + e < g.M; ++e) w[e >> 2] |= (uint32_t)src[e] << (8 * (e & 3));
        a[q] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    // Q operand form: stage k0 / 128, column blocks j0 / 32 .. + 8 (always present: padded)
    const int64_t st = k0 >> 7, njb = g.ldb, jb0 = j0 >> 5;
    const uint8_t* Qc = reinterpret_cast<const uint8_t*>(g.B) + (st * njb + jb0) * 4096;
#pragma unroll
    for (int q = 0; q < F8CH; ++q) this->q[q] = *reinterpret_cast<const uint4*>(Qc + 16 * (tid + BT * q));
#pragma unroll
    for (int b = 0; b < 2; ++b)
      qs[b] = *reinterpret_cast<const uint16_t*>(g.b_scales + ((st * njb + jb0 + 2 * wn + b) * 64 + lane) * 2);
    const int64_t ib = (i0 >> 7) + wm;
    sa = ib < g.a_ldsc ? g.a_scales[st * g.a_ldsc + ib] : 0.f;
  }
  RF_DEV void store(uint8_t* SA, uint8_t* SQ, int tid) const {
#pragma unroll
    for (int q = 0; q < F8CH; ++q) {
      const int c = tid + BT * q;
      *reinterpret_cast<uint4*>(SA + (c >> 4) * F8P + 16 * (c & 15)) = a[q];
      *reinterpret_cast<uint4*>(SQ + 16 * c) = this->q[q];
    }
  }
};

// A operand of row block a, chunk ch (k rows 64 ch .. 64 ch + 63 of the stage).
RF_DEV i32x8 f8_frag_a(const uint8_t* S, int wm, int a, int ch, int lane) {
  const int G = lane >> 4, s = lane & 15;
  const int col = wm * 128 + 32 * a + 16 * (G & 1) + 8 * (s & 1);
  const int row = 64 * ch + 16 * (G >> 1) + (s >> 1);
  i32x8 f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint8_t* p = S + (row + 32 * (j >> 1) + 8 * (j & 1)) * F8P + col;
    const f8i32x2 t = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) f8i32x2*)p);
    f[2 * j] = t.x;
    f[2 * j + 1] = t.y;
  }
  return f;
}

// B operand of column block b of wave column wn, chunk ch.
RF_DEV i32x8 f8_frag_q(const uint8_t* S, int wn, int b, int ch, int lane) {
  const uint8_t* p = S + (((2 * wn + b) * 2 + ch) * 2) * 1024 + 16 * lane;
  const uint4 lo = *reinterpret_cast<const uint4*>(p), hi = *reinterpret_cast<const uint4*>(p + 1024);
  i32x8 f;
  f[0] = (int)lo.x; f[1] = (int)lo.y; f[2] = (int)lo.z; f[3] = (int)lo.w;
  f[4] = (int)hi.x; f[5] = (int)hi.y; f[6] = (int)hi.z; f[7] = (int)hi.w;
  return f;
}

// s = 2^e mu with e + 127 a valid E8M0 byte; mu NaN for a non-finite s.
RF_DEV void f8_split_scale(float s, int& e8, float& mu) {
  if (!isfinite(s)) {
    e8 = 127;
    mu = __builtin_nanf("");
    return;
  }
  int e;
  float f = frexpf(s, &e);  // s = f 2^e, |f| in [1/2, 1)
  if (e > 127) { f = ldexpf(f, e - 127); e = 127; }
  if (e < -127) { f = ldexpf(f, e + 127); e = -127; }
  e8 = e + 127;
  mu = f;
}

RF_DEV void gemm_fp8_body(const GemmArgs& g, int bid, int split) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem8[];
  uint8_t* const A0 = smem8;
  uint8_t* const Q0 = smem8 + 2 * F8AS;

  const int ntm = (int)((g.M + HB - 1) / HB), ntn = (int)((g.N + HB - 1) / HB);
  int tm, tn;
  tile_coords(bid, ntm, ntn, tm, tn);
  const int64_t i0 = (int64_t)tm * HB, j0 = (int64_t)tn * HB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // wave tile: rows wm*128 + [0, 128), columns wn*64 + [0, 64)
  const int64_t kbeg = (int64_t)split * g.kps;  // kps is a multiple of 128
  const int64_t kend = min(g.K, kbeg + g.kps);
  const bool avec = ((((uintptr_t)g.A) & 15) == 0) && (g.lda % 16 == 0);

  f32x16 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  F8Stage sg;
  const int nk = kend > kbeg ? (int)((kend - kbeg + F8K - 1) / F8K) : 0;
  uint32_t qs[2] = {0u, 0u};
  float sa = 0.f, mu_acc = 0.f;  // mu_acc: the mu the accumulators are divided by (0: nothing added yet)
  if (nk > 0) {
    sg.load(g, i0, j0, kbeg, kend, avec, tid, wm, wn, lane);
    sg.store(A0, Q0, tid);
    qs[0] = sg.qs[0]; qs[1] = sg.qs[1]; sa = sg.sa;
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) sg.load(g, i0, j0, kbeg + (int64_t)(kt + 1) * F8K, kend, avec, tid, wm, wn, lane);
    // the stage's A scale is the same word for every lane of the wave
    const float s_w = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, sa)));
    if (s_w != 0.f) {
      int e8;
      float mu;
      f8_split_scale(s_w, e8, mu);
      if (mu_acc != 0.f && mu != mu_acc) {
        const float r = mu_acc / mu;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int x = 0; x < 16; ++x) acc[a][b][x] *= r;
      }
      mu_acc = mu;
      const uint8_t* A_ = A0 + buf * F8AS;
      const uint8_t* Q_ = Q0 + buf * F8QS;
#pragma unroll
      for (int ch = 0; ch < 2; ++ch) {
        const i32x8 b0 = f8_frag_q(Q_, wn, 0, ch, lane), b1 = f8_frag_q(Q_, wn, 1, ch, lane);
        const int s0 = (int)((qs[0] >> (8 * ch)) & 0xffu), s1 = (int)((qs[1] >> (8 * ch)) & 0xffu);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const i32x8 af = f8_frag_a(A_, wm, a, ch, lane);
          acc[a][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af, b0, acc[a][0], 0, 0, 0, e8, 0, s0);
          acc[a][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af, b1, acc[a][1], 0, 0, 0, e8, 0, s1);
        }
      }
    }
    if (kt + 1 < nk) {
      sg.store(A0 + (buf ^ 1) * F8AS, Q0 + (buf ^ 1) * F8QS, tid);
      qs[0] = sg.qs[0]; qs[1] = sg.qs[1]; sa = sg.sa;
    }
    __syncthreads();
  }
  if (mu_acc != 0.f && mu_acc != 1.f) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int x = 0; x < 16; ++x) acc[a][b][x] *= mu_acc;
  }
  big_epilogue(g, acc, i0, j0, split, wm, wn, lane, tid, smem8);
}

__global__ __launch_bounds__(BT, 1) void k_gemm_fp8(GemmArgs g) { gemm_fp8_body(g, blockIdx.x, blockIdx.y); }

// ---- grouped launches: many independent products in one grid --------------------
// Work list: group i owns tiles [tile_start[i], tile_start[i+1]) of the flat grid;
// a workgroup finds its group by binary search and runs that group's tile.  All
// groups of one launch share the operand layouts (template) and the tile shape.
RF_DEV int find_group(const int* __restrict__ start, int count, int bid) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= bid) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// (the problems of a group launch take the element form: their shapes are ragged)
template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void k_gemm_f32_grouped(const GemmArgs* __restrict__ gs, const int* tile_start,
                                                          int count) {
  const int i = find_group(tile_start, count, blockIdx.x);
  const GemmArgs g = gs[i];
  if (g.M == 0 || g.N == 0) return;
  gemm_f32_body<AKC, BKC, false>(g, blockIdx.x - tile_start[i], 0);
}
template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void k_gemm_bf16_grouped(const GemmArgs* __restrict__ gs, const int* tile_start,
                                                           int count) {
  const int i = find_group(tile_start, count, blockIdx.x);
  const GemmArgs g = gs[i];
  if (g.M == 0 || g.N == 0) return;
  gemm_bf16_body<AKC, BKC, false, true>(g, blockIdx.x - tile_start[i], 0);
}
template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void k_gemm_bf16a32_grouped(const GemmArgs* __restrict__ gs, const int* tile_start,
                                                              int count) {
  const int i = find_group(tile_start, count, blockIdx.x);
  const GemmArgs g = gs[i];
  if (g.M == 0 || g.N == 0) return;
  gemm_bf16_body<AKC, BKC, true, true>(g, blockIdx.x - tile_start[i], 0);
}
template <bool AKC, bool BKC, int AMODE>
__global__ __launch_bounds__(BT, 1) void k_gemm_bf16_big_grouped(const GemmArgs* __restrict__ gs,
                                                                  const int* tile_start, int count) {
  const int i = find_group(tile_start, count, blockIdx.x);
  const GemmArgs g = gs[i];
  if (g.M == 0 || g.N == 0) return;
  gemm_bf16_big_body<AKC, BKC, AMODE>(g, blockIdx.x - tile_start[i], 0);
}

__global__ void k_gemm_reduce(GemmArgs g, int splits) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.M * g.N) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += g.partial[(int64_t)z * g.M * g.N + idx];
  store_out(g, idx / g.N, idx % g.N, s);
}

static int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (n <= 0) n = 256;
  }
  return n;
}

int gemm_splits(int64_t M, int64_t N, int64_t K) {
  int64_t tiles = ((M + GBM - 1) / GBM) * ((N + GBN - 1) / GBN);
  int s = 1;
  while (tiles * s < 2 * cu_count() && K / (s * 2) >= 512 && s < 64) s *= 2;
  return s;
}

// 256 x 256 tiles: one workgroup per CU, so split K until the CUs are covered.
static int gemm_splits_big(int64_t M, int64_t N, int64_t K) {
  int64_t tiles = ((M + HB - 1) / HB) * ((N + HB - 1) / HB);
  int s = 1;
  while (tiles * s < cu_count() && K / (s * 2) >= 1024 && s < 64) s *= 2;
  return s;
}

// ---- tuning table (written by the autotuner, read on every launch) -------------------
// First rule whose dtype matches and whose bounds hold picks the tile and the split
// count (FP32- or FP8-stored A follow the BF16 rules); no match: the heuristics above.  Split counts are capped at kMaxTunedSplit
// (and at K / 256) so the partial buffer sized by gemm_partial_floats always fits.
constexpr int kMaxRules = 256, kMaxTunedSplit = 16;
static GemmRule g_rules[kMaxRules];
static int g_nrules = 0;

int set_gemm_rules(const GemmRule* rules, int count) {
  if (count < 0 || count > kMaxRules || (count > 0 && !rules)) return -1;
  for (int i = 0; i < count; ++i) {
    const GemmRule& r = rules[i];
    if ((r.dtype != 0 && r.dtype != 2) || (r.tile != 128 && r.tile != 256) || (r.tile == 256 && r.dtype != 2) ||
        r.split < 0 || r.split > kMaxTunedSplit)
      return -1;
  }
  for (int i = 0; i < count; ++i) g_rules[i] = rules[i];
  g_nrules = count;
  return 0;
}

static int tuned_cap(int64_t K) {
  int s = 1;
  while (s < kMaxTunedSplit && K / (2 * s) >= 256) s *= 2;
  return s;
}

static const GemmRule* find_rule(int dtype, int64_t M, int64_t N, int64_t K) {
  for (int i = 0; i < g_nrules; ++i) {
    const GemmRule& r = g_rules[i];
    if (r.dtype == dtype && M <= r.max_m && N <= r.max_n && K <= r.max_k) return &r;
  }
  return nullptr;
}

bool gemm_use_big(int dtype, int64_t M, int64_t N) {
  if (dtype == 4 || dtype == 6 || dtype == 7) return true;
  return dtype == 2 && M >= 512 && N >= 512;
}

size_t gemm_partial_floats(int64_t M, int64_t N, int64_t K) {
  int s = gemm_splits(M, N, K);
  s = std::max(s, gemm_splits_big(M, N, K));
  s = std::max(s, tuned_cap(K));
  return s > 1 ? (size_t)s * M * N : 0;
}

template <bool AKC, bool BKC, int AF32>
static void go_big(const GemmArgs& g, dim3 grid, hipStream_t st) {
  constexpr size_t lds = 2 * (size_t)(big_stage_elems<AKC>() + big_stage_elems<BKC>()) * sizeof(uint16_t);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_gemm_bf16_big<AKC, BKC, AF32>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL((k_gemm_bf16_big<AKC, BKC, AF32>), grid, dim3(BT), lds, st, g);
}

hipError_t launch_gemm(GemmArgs g, int dtype, float* partial, hipStream_t st) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  const GemmRule* rule = (dtype == 0 || dtype == 2) ? find_rule(dtype, g.M, g.N, g.K) : nullptr;
  if (dtype == 4 || dtype == 6) {
    // FP32- and FP8-stored A run the 256-tile BF16 kernel: they take the split of
    // its BF16 rule for the shape, when that rule picks the 256 tile (the FP8 x FP8
    // kernel, dtype 7, keeps the heuristic: its stage time differs)
    const GemmRule* r2 = find_rule(2, g.M, g.N, g.K);
    if (r2 && r2->tile == 256) rule = r2;
  }
  const bool big = rule ? (rule->tile == 256) : gemm_use_big(dtype, g.M, g.N);
  int splits = 1;
  if (partial) {
    if (rule && rule->split > 0) splits = std::min(rule->split, tuned_cap(g.K));
    else splits = big ? gemm_splits_big(g.M, g.N, g.K) : gemm_splits(g.M, g.N, g.K);
  }
  if (g.split_cap > 0) splits = std::min(splits, g.split_cap);
  if (g.b_upper) splits = 1;
  const int64_t bk = dtype == 7 ? F8K : 32;  // FP8 split parts start on A scale blocks
  g.kps = ((g.K + splits - 1) / splits + bk - 1) / bk * bk;
  if (g.kps == 0) g.kps = bk;
  splits = (int)((g.K + g.kps - 1) / g.kps);
  if (splits < 1) splits = 1;
  g.partial = splits > 1 ? partial : nullptr;
  const int64_t bm = big ? HB : GBM, bn = big ? HB : GBN;
  int64_t tiles = ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  dim3 grid((unsigned)tiles, (unsigned)splits);
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, g); };
  if (dtype == 0) {
    if (f32_vec_ok(g)) {
      if (g.a_kc && g.b_kc) go(k_gemm_f32<true, true, true>);
      else if (g.a_kc && !g.b_kc) go(k_gemm_f32<true, false, true>);
      else if (!g.a_kc && g.b_kc) go(k_gemm_f32<false, true, true>);
      else go(k_gemm_f32<false, false, true>);
    } else {
      if (g.a_kc && g.b_kc) go(k_gemm_f32<true, true, false>);
      else if (g.a_kc && !g.b_kc) go(k_gemm_f32<true, false, false>);
      else if (!g.a_kc && g.b_kc) go(k_gemm_f32<false, true, false>);
      else go(k_gemm_f32<false, false, false>);
    }
  } else if (dtype == 2 && big) {
    if (g.a_kc && g.b_kc) go_big<true, true, 0>(g, grid, st);
    else if (g.a_kc && !g.b_kc) go_big<true, false, 0>(g, grid, st);
    else if (!g.a_kc && g.b_kc) go_big<false, true, 0>(g, grid, st);
    else go_big<false, false, 0>(g, grid, st);
  } else if (dtype == 2) {
    if (g.a_kc && g.b_kc) go(k_gemm_bf16<true, true>);
    else if (g.a_kc && !g.b_kc) go(k_gemm_bf16<true, false>);
    else if (!g.a_kc && g.b_kc) go(k_gemm_bf16<false, true>);
    else go(k_gemm_bf16<false, false>);
  } else if (dtype == 6) {
    if (g.a_kc || !g.a_scales) return hipErrorInvalidValue;
    if (g.b_kc) go_big<false, true, 2>(g, grid, st);
    else go_big<false, false, 2>(g, grid, st);
  } else if (dtype == 7) {
    if (g.a_kc || g.b_kc || !g.a_scales || !g.b_scales || g.b_upper || g.ldb != qf8_col_blocks(g.N))
      return hipErrorInvalidValue;
    constexpr int lds = 2 * (F8AS + F8QS);
    static std::once_flag attr;
    std::call_once(attr, [] {
      (void)hipFuncSetAttribute((const void*)k_gemm_fp8, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    });
    hipLaunchKernelGGL(k_gemm_fp8, grid, dim3(BT), lds, st, g);
  } else if (dtype == 4) {
    if (g.a_kc && g.b_kc) go_big<true, true, 1>(g, grid, st);
    else if (g.a_kc && !g.b_kc) go_big<true, false, 1>(g, grid, st);
    else if (!g.a_kc && g.b_kc) go_big<false, true, 1>(g, grid, st);
    else go_big<false, false, 1>(g, grid, st);
  } else {
    return hipErrorInvalidValue;
  }
  if (splits > 1) {
    int64_t tot = g.M * g.N;
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, g, splits);
  }
  return hipGetLastError();
}

// ---- grouped launcher ---------------------------------------------------------------
int gemm_group_tiles(int kind, int64_t M, int64_t N) {
  const int64_t b = (kind == 3 || kind == 4) ? HB : GBM;
  return (int)(((M + b - 1) / b) * ((N + b - 1) / b));
}

template <bool AKC, bool BKC, int AF32>
static void go_big_grouped(const GemmArgs* gs, const int* ts, int count, int tiles, hipStream_t st) {
  constexpr size_t lds = 2 * (size_t)(big_stage_elems<AKC>() + big_stage_elems<BKC>()) * sizeof(uint16_t);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_gemm_bf16_big_grouped<AKC, BKC, AF32>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL((k_gemm_bf16_big_grouped<AKC, BKC, AF32>), dim3((unsigned)tiles), dim3(BT), lds, st, gs, ts,
                     count);
}

hipError_t launch_gemm_grouped(const GemmArgs* gs, const int* tile_start, int count, int total_tiles, int kind,
                               int a_kc, int b_kc, hipStream_t st) {
  if (count == 0 || total_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)total_tiles), blk(256);
  const int sel = (a_kc ? 2 : 0) | (b_kc ? 1 : 0);
  switch (kind) {
    case 0:
      if (sel == 3) hipLaunchKernelGGL((k_gemm_f32_grouped<true, true>), grid, blk, 0, st, gs, tile_start, count);
      else if (sel == 2) hipLaunchKernelGGL((k_gemm_f32_grouped<true, false>), grid, blk, 0, st, gs, tile_start, count);
      else if (sel == 1) hipLaunchKernelGGL((k_gemm_f32_grouped<false, true>), grid, blk, 0, st, gs, tile_start, count);
      else hipLaunchKernelGGL((k_gemm_f32_grouped<false, false>), grid, blk, 0, st, gs, tile_start, count);
      break;
    case 2:
      if (sel == 3) hipLaunchKernelGGL((k_gemm_bf16_grouped<true, true>), grid, blk, 0, st, gs, tile_start, count);
      else if (sel == 2) hipLaunchKernelGGL((k_gemm_bf16_grouped<true, false>), grid, blk, 0, st, gs, tile_start, count);
      else if (sel == 1) hipLaunchKernelGGL((k_gemm_bf16_grouped<false, true>), grid, blk, 0, st, gs, tile_start, count);
      else hipLaunchKernelGGL((k_gemm_bf16_grouped<false, false>), grid, blk, 0, st, gs, tile_start, count);
      break;
    case 5:
      if (sel == 3) hipLaunchKernelGGL((k_gemm_bf16a32_grouped<true, true>), grid, blk, 0, st, gs, tile_start, count);
      else if (sel == 2) hipLaunchKernelGGL((k_gemm_bf16a32_grouped<true, false>), grid, blk, 0, st, gs, tile_start, count);
      else if (sel == 1) hipLaunchKernelGGL((k_gemm_bf16a32_grouped<false, true>), grid, blk, 0, st, gs, tile_start, count);
      else hipLaunchKernelGGL((k_gemm_bf16a32_grouped<false, false>), grid, blk, 0, st, gs, tile_start, count);
      break;
    case 3:
      if (sel == 3) go_big_grouped<true, true, 0>(gs, tile_start, count, total_tiles, st);
      else if (sel == 2) go_big_grouped<true, false, 0>(gs, tile_start, count, total_tiles, st);
      else if (sel == 1) go_big_grouped<false, true, 0>(gs, tile_start, count, total_tiles, st);
      else go_big_grouped<false, false, 0>(gs, tile_start, count, total_tiles, st);
      break;
    case 4:
      if (sel == 3) go_big_grouped<true, true, 1>(gs, tile_start, count, total_tiles, st);
      else if (sel == 2) go_big_grouped<true, false, 1>(gs, tile_start, count, total_tiles, st);
      else if (sel == 1) go_big_grouped<false, true, 1>(gs, tile_start, count, total_tiles, st);
      else go_big_grouped<false, false, 1>(gs, tile_start, count, total_tiles, st);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rf
