// C ABI of the range finder: argument checks, workspace carving and the
// stream-ordered schedule of kernels for Algorithms 1-3 and the randomised
// SVD finisher.  No allocation, no synchronisation, no host round trips.
#include <math.h>
#include <string.h>

#include "../../include/rf.h"
#include "common.h"
#include "kernels.h"

using namespace rf;

namespace {

// ------------------------------------------------------------------ workspace
struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(void* b) : base((char*)b) {}
  template <typename T>
  T* get(size_t count) {
    size_t bytes = ((count * sizeof(T)) + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

struct Dims {
  int64_t m, n;
  int k, r1, s, q;
  int dtype, prec;
  bool classical;  // S = I_n (RF_FLAG_CLASSICAL): At = A, Omega n x k; r1 then sizes S2 only
  int64_t rw;      // rows of Omega, Z and At^T Q: n when classical, else r1
  int family;      // S of Algorithm 1: 0 sparse sign, 1 Rademacher, 2 Gaussian, 3 SRHT (Lemma 3.2)
};

struct RFBufs {
  int32_t* table; uint32_t* ready; int* cmax;
  float* Sd; uint16_t* Sd16;  // dense S (Rademacher / Gaussian), unscaled
  float* srd; int* picks;     // SRHT signs and sampled columns
  float* om; uint16_t* om16;
  float* At; uint16_t* At16;
  float* Ya; float* Yb; uint16_t* Q16;
  float* Zh; float* Z; uint16_t* Z16;
  double* G; double* d0; int* flags; int* counters; float* Rinv; double* triwork; int* cwork;
  double* gpart; float* mpart; double* orth;
};

static size_t max3(size_t a, size_t b, size_t c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

// Buffers of Algorithm 1 (shared by every op).
static RFBufs carve_rf(Arena& ar, const Dims& d) {
  RFBufs b;
  const bool mixed = d.prec == RF_PREC_MIXED;
  const bool sk = !d.classical;  // At = A S exists only for S != I
  const bool sparse = sk && d.family == 0, dense = sk && (d.family == 1 || d.family == 2), srht = sk && d.family == 3;
  b.table = sparse ? ar.get<int32_t>((size_t)d.n * d.s) : nullptr;
  b.ready = sparse ? ar.get<uint32_t>((size_t)d.n * d.s) : nullptr;
  b.cmax = sparse ? ar.get<int>(sketch_right_work_ints(d.n, d.s, d.r1)) : nullptr;
  b.Sd = dense ? ar.get<float>((size_t)d.n * d.r1) : nullptr;
  b.Sd16 = (dense && (mixed || d.dtype == RF_BF16)) ? ar.get<uint16_t>((size_t)d.n * d.r1) : nullptr;
  b.srd = srht ? ar.get<float>((size_t)srht_size(d.n)) : nullptr;
  b.picks = srht ? ar.get<int>((size_t)d.r1) : nullptr;
  b.om = ar.get<float>((size_t)d.rw * d.k);
  b.om16 = mixed ? ar.get<uint16_t>((size_t)d.rw * d.k) : nullptr;
  b.At = sk ? ar.get<float>((size_t)d.m * d.r1) : nullptr;
  b.At16 = (sk && mixed) ? ar.get<uint16_t>((size_t)d.m * d.r1) : nullptr;
  b.Ya = ar.get<float>((size_t)d.m * d.k);
  b.Yb = ar.get<float>((size_t)d.m * d.k);
  b.Q16 = mixed ? ar.get<uint16_t>((size_t)d.m * d.k) : nullptr;
  b.Zh = ar.get<float>((size_t)d.rw * d.k);
  b.Z = ar.get<float>((size_t)d.rw * d.k);
  b.Z16 = mixed ? ar.get<uint16_t>((size_t)d.rw * d.k) : nullptr;
  b.G = ar.get<double>((size_t)d.k * d.k);
  b.d0 = ar.get<double>((size_t)d.k);
  b.flags = ar.get<int>((size_t)d.k);
  b.counters = ar.get<int>(16);
  b.Rinv = ar.get<float>((size_t)d.k * d.k);
  b.triwork = ar.get<double>((size_t)d.k * d.k);
  b.cwork = ar.get<int>(cholinv_work_ints(d.k));
  b.gpart = ar.get<double>(gram_partial_doubles(d.m > d.rw ? d.m : d.rw, d.k, d.k));
  b.mpart = ar.get<float>(gemm_partial_floats(d.rw, d.k, d.m));
  b.orth = ar.get<double>(2);
  return b;
}

struct Ctx {
  hipStream_t st;
  hipError_t err = hipSuccess;
  void chk(hipError_t e) {
    if (e != hipSuccess && err == hipSuccess) err = e;
  }
};

static void gemm(Ctx& c, int dtype, const void* A, int64_t lda, int a_kc, const void* B, int64_t ldb, int b_kc, void* C,
                 int64_t ldc, int64_t M, int64_t N, int64_t K, float* partial, const float* colscale = nullptr,
                 int c_trans = 0, int b_upper = 0, int c_bf16 = 0, const float* a_scales = nullptr,
                 int64_t a_ldsc = 0, int split_cap = 0, float alpha = 1.f, const uint8_t* b_scales = nullptr) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.a_scales = a_scales;
  g.b_scales = b_scales;
  g.a_ldsc = a_ldsc;
  g.A = A; g.lda = lda; g.a_kc = a_kc;
  g.B = B; g.ldb = ldb; g.b_kc = b_kc;
  g.C = C; g.ldc = ldc; g.c_trans = c_trans; g.c_bf16 = c_bf16;
  g.M = M; g.N = N; g.K = K;
  g.alpha = alpha;
  g.colscale = colscale;
  g.b_upper = b_upper;
  g.split_cap = split_cap;
  c.chk(launch_gemm(g, dtype, partial, c.st));
}

// Tolerance on Cholesky pivots relative to the original diagonal: a column whose
// residual is below ~4 sqrt(k) FP32 ulps of its norm is numerically dependent.
static double chol_tol(int k) {
  const double u = 5.9604644775390625e-08;  // 2^-24
  return 16.0 * (double)k * u * u;
}

// One CholeskyQR pass: out = X R^{-1}, X^T X = R^T R.  Dependent columns of X are
// replaced (stream-3 Gaussians) and the factorisation repeated.
static void cholqr_pass(Ctx& c, RFBufs& b, float* X, float* out, int64_t rows, int k, uint64_t seed) {
  c.chk(launch_gram(X, k, 0, X, k, 0, rows, k, k, 1, b.G, k, b.gpart, nullptr, c.st));
  c.chk(launch_cholinv(b.G, k, k, chol_tol(k), b.d0, b.flags, &b.counters[0], &b.counters[2], &b.counters[5], nullptr,
                       b.triwork, k, b.Rinv, k, b.cwork, c.st));
  c.chk(launch_note(b.counters, 0, c.st));
  c.chk(launch_refill(X, k, rows, k, b.flags, &b.counters[4], b.d0, seed, c.st));
  c.chk(launch_gram(X, k, 0, X, k, 0, rows, k, k, 1, b.G, k, b.gpart, &b.counters[4], c.st));
  c.chk(launch_cholinv(b.G, k, k, chol_tol(k), b.d0, b.flags, &b.counters[0], &b.counters[2], &b.counters[5],
                       &b.counters[4], b.triwork, k, b.Rinv, k, b.cwork, c.st));
  c.chk(launch_note(b.counters, 1, c.st));
  gemm(c, 0, X, k, 1, b.Rinv, k, 0, out, k, rows, k, k, nullptr, nullptr, 0, 1);
}

// At = A S (m x r1 FP32, ld r1) for the sketch family of d, drawn from `seed`
// (or from `table_in` for the sparse sign sketch).  One pass over A for the
// sparse sketch and the SRHT; a dense product on MFMA for the dense families
// (A S / sqrt(r1) with S = +-1 or N(0,1): FP32 MFMA in the plain form, BF16 MFMA
// in the mixed form or for BF16-stored A).
static void sketch_right_any(Ctx& c, const rf_matrix* A, const Dims& d, uint64_t seed, RFBufs& b, float* out,
                             int64_t ldo, const int32_t* table_in) {
  const bool mixed = d.prec == RF_PREC_MIXED;
  if (d.family == 1 || d.family == 2) {
    c.chk(launch_dense_sketch(d.family, d.n, d.r1, seed, 0, b.Sd, c.st));
    const float alpha = 1.0f / sqrtf((float)d.r1);
    if (A->dtype == RF_F32 && !mixed) {
      gemm(c, 0, A->data, A->ld, 1, b.Sd, d.r1, 0, out, ldo, d.m, d.r1, d.n, nullptr, nullptr, 0, 0, 0, nullptr, 0, 0,
           alpha);
    } else {
      c.chk(launch_cast_f32_bf16(b.Sd, d.r1, b.Sd16, d.r1, d.n, d.r1, c.st));
      gemm(c, A->dtype == RF_BF16 ? 2 : 4, A->data, A->ld, 1, b.Sd16, d.r1, 0, out, ldo, d.m, d.r1, d.n, nullptr,
           nullptr, 0, 0, 0, nullptr, 0, 0, alpha);
    }
    return;
  }
  if (d.family == 3) {
    c.chk(launch_srht_prep(d.n, d.r1, seed, 0, b.srd, b.picks, c.st));
    c.chk(launch_srht_rows(A->dtype, A->data, A->ld, A->block_scales, d.m, d.n, b.srd, b.picks, d.r1, out, ldo, c.st));
    return;
  }
  const int32_t* table = table_in;
  if (!table) {
    c.chk(launch_sketch_table(d.n, d.s, d.r1, seed, 0, 0, b.table, c.st));
    table = b.table;
  }
  const bool fast = sketch_right_fast_ok(d.s) && !sketch_right_gather(d.s, d.n, d.r1);
  if (fast) c.chk(launch_sketch_ready(table, d.n, d.s, d.r1, sketch_right_cpl(d.s), b.ready, c.st));
  c.chk(launch_sketch_right(A->dtype, A->data, A->ld, A->block_scales, table, fast ? b.ready : nullptr, b.cmax, d.s,
                            d.m, d.n, d.r1, out, ldo, c.st));
}

// Operand At of the power products.  Sketched: At = A S (FP32, and its BF16 copy
// in the mixed form).  Classical (S = I): At = A itself, FP32 operands read as
// stored, BF16 operands by rounding A to BF16 as it is loaded (GEMM dtype 4).
struct AtOp {
  const void* p32; int64_t ld32;           // FP32 operand (GEMM dtype 0)
  const void* p16; int64_t ld16; int dt16;  // BF16 operand (dtype 2, or 4 for FP32 A)
};

// Algorithm 1.  Result (m x k FP32, ld k) in `Qout`; b.Ya/b.Yb are used as scratch.
// table_in / om_in: a caller-given sketch table (already checked for the block
// layout) and Omega (rw x k, ld k), or null to draw them from the seed.
static void range_finder_core(Ctx& c, const rf_matrix* A, const Dims& d, uint64_t seed, RFBufs& b, float* Qout,
                              const int32_t* table_in = nullptr, const float* om_in = nullptr,
                              const rf_csr* csr = nullptr) {
  const bool mixed = d.prec == RF_PREC_MIXED;
  const int k = d.k;
  const int64_t rw = d.rw;
  if (!table_in) c.chk(launch_fill_i32(b.counters, 16, 0, c.st));
  const float* om = om_in;
  if (!om) {
    c.chk(launch_gaussian(rw, k, seed, 1, 0, b.om, k, c.st));
    om = b.om;
  }
  AtOp at;
  if (d.classical) {
    at = AtOp{A->data, A->ld, A->data, A->ld, 4};
  } else if (csr) {
    // sparse A: each nonzero scattered into its s buckets (fixed point, exact sums)
    c.chk(launch_sketch_table(d.n, d.s, d.r1, seed, 0, 0, b.table, c.st));
    c.chk(launch_sketch_csr(csr->row_ptr, csr->col_idx, csr->values, d.m, d.n, csr->nnz, b.table, d.s, d.r1, b.At,
                            d.r1, &b.counters[7], c.st));
    if (mixed) c.chk(launch_cast_f32_bf16(b.At, d.r1, b.At16, d.r1, d.m, d.r1, c.st));
    at = AtOp{b.At, d.r1, b.At16, d.r1, 2};
  } else {
    // At = A S  (one pass over A for the sparse sketch and the SRHT)
    sketch_right_any(c, A, d, seed, b, b.At, d.r1, table_in);
    if (mixed) c.chk(launch_cast_f32_bf16(b.At, d.r1, b.At16, d.r1, d.m, d.r1, c.st));
    at = AtOp{b.At, d.r1, b.At16, d.r1, 2};
  }
  if (mixed) c.chk(launch_cast_f32_bf16(om, k, b.om16, k, rw, k, c.st));
  // Y0 = At Omega
  if (mixed && d.q > 0) gemm(c, at.dt16, at.p16, at.ld16, 1, b.om16, k, 0, b.Ya, k, d.m, k, rw, nullptr);
  else gemm(c, 0, at.p32, at.ld32, 1, om, k, 0, b.Ya, k, d.m, k, rw, nullptr);
  if (d.q == 0) {
    cholqr_pass(c, b, b.Ya, b.Yb, d.m, k, seed);
    cholqr_pass(c, b, b.Yb, Qout, d.m, k, seed);
    return;
  }
  float* Qc = b.Yb;
  cholqr_pass(c, b, b.Ya, Qc, d.m, k, seed);
  for (int j = 1; j <= d.q; ++j) {
    // Zh = At^T Q  (contraction over m, split-K)
    if (mixed) {
      c.chk(launch_cast_f32_bf16(Qc, k, b.Q16, k, d.m, k, c.st));
      gemm(c, at.dt16, at.p16, at.ld16, 0, b.Q16, k, 0, b.Zh, k, rw, k, d.m, b.mpart);
    } else {
      gemm(c, 0, at.p32, at.ld32, 0, Qc, k, 0, b.Zh, k, rw, k, d.m, b.mpart);
    }
    cholqr_pass(c, b, b.Zh, b.Z, rw, k, seed);
    // Y = At Z; the last product is taken in FP32 in both forms
    const bool last = (j == d.q);
    if (mixed && !last) {
      c.chk(launch_cast_f32_bf16(b.Z, k, b.Z16, k, rw, k, c.st));
      gemm(c, at.dt16, at.p16, at.ld16, 1, b.Z16, k, 0, b.Ya, k, d.m, k, rw, nullptr);
    } else {
      gemm(c, 0, at.p32, at.ld32, 1, b.Z, k, 0, b.Ya, k, d.m, k, rw, nullptr);
    }
    if (last) {
      cholqr_pass(c, b, b.Ya, b.Yb, d.m, k, seed);
      cholqr_pass(c, b, b.Yb, Qout, d.m, k, seed);
    } else {
      cholqr_pass(c, b, b.Ya, Qc, d.m, k, seed);
    }
  }
}

// ------------------------------------------------------------------ validation
static bool valid_matrix(const rf_matrix* A) {
  if (!A || !A->data || A->rows < 1 || A->cols < 1 || A->ld < A->cols || A->reserved != 0) return false;
  if (A->dtype != RF_F32 && A->dtype != RF_BF16 && A->dtype != RF_FP8E4M3_B128) return false;
  if ((A->dtype == RF_FP8E4M3_B128) != (A->block_scales != nullptr)) return false;
  return true;
}

static bool valid_params(const rf_matrix* A, const rf_params* p, bool square) {
  if (!p) return false;
  if (p->flags & ~(RF_FLAG_ORTH_ERR | RF_FLAG_CLASSICAL | RF_SKETCH_MASK)) return false;
  if ((p->flags & RF_FLAG_CLASSICAL) && (p->flags & RF_SKETCH_MASK)) return false;  // S = I has no family
  int64_t mn = A->rows < A->cols ? A->rows : A->cols;
  if (square) {
    if (A->rows != A->cols) return false;
    mn = A->cols;
  }
  if (p->k < 1 || p->sketch < p->k || p->sketch > mn) return false;
  if (p->q < 0 || p->q > 1000) return false;
  if (p->nnz_per_col < 1 || p->nnz_per_col > p->sketch) return false;
  if (p->precision != RF_PREC_FP32 && p->precision != RF_PREC_MIXED) return false;
  return true;
}

static Dims dims_of(const rf_matrix* A, const rf_params* p) {
  Dims d;
  d.m = A->rows; d.n = A->cols;
  d.k = p->k; d.r1 = p->sketch; d.s = p->nnz_per_col; d.q = p->q;
  d.dtype = A->dtype; d.prec = p->precision;
  d.classical = (p->flags & RF_FLAG_CLASSICAL) != 0;
  d.rw = d.classical ? d.n : d.r1;
  d.family = (int)((p->flags & RF_SKETCH_MASK) >> 2);
  return d;
}

// A family this build cannot run for A (FP8 storage with a dense S has no
// product kernel; the SRHT needs n' <= 32768 and r1 <= 8192).
static bool family_unsupported(const rf_matrix* A, const Dims& d) {
  if ((d.family == 1 || d.family == 2) && A->dtype == RF_FP8E4M3_B128) return true;
  if (d.family == 3 && !srht_supported(d.n, d.r1)) return true;
  return false;
}

// Split-K parts the B^T = A^T Q product may use (its partial buffer holds this many
// n x k FP32 slices; the tuning table's split is capped to it).
constexpr int kQtaSplitCap = 4;

struct SvdBufs {
  float* Q; float* Bt; double* GB; double* lam; double* Ub; float* Ub32; float* inv; void* eigw; int* signw;
  float* qpart;
  uint8_t* qf8c; uint8_t* qf8s;  // FP8 operand form of Q (FP8-stored A, mixed form)
};
static SvdBufs carve_svd(Arena& ar, const Dims& d) {
  SvdBufs s;
  s.Q = ar.get<float>((size_t)d.m * d.k);
  s.Bt = ar.get<float>((size_t)d.n * d.k);
  s.GB = ar.get<double>((size_t)d.k * d.k);
  s.lam = ar.get<double>(d.k);
  s.Ub = ar.get<double>((size_t)d.k * d.k);
  s.Ub32 = ar.get<float>((size_t)d.k * d.k);
  s.inv = ar.get<float>(d.k);
  s.eigw = ar.get<char>(eig_work_bytes(d.k));
  s.signw = ar.get<int>(3 * (size_t)d.k);
  s.qpart = ar.get<float>((size_t)kQtaSplitCap * d.n * d.k);
  const bool f8 = d.dtype == RF_FP8E4M3_B128 && d.prec == RF_PREC_MIXED;
  s.qf8c = f8 ? ar.get<uint8_t>(qf8_code_bytes(d.m, d.k)) : nullptr;
  s.qf8s = f8 ? ar.get<uint8_t>(qf8_scale_bytes(d.m, d.k)) : nullptr;
  return s;
}
static double* carve_gpart_big(Arena& ar, const Dims& d) {
  return ar.get<double>(gram_partial_doubles(d.n, d.k, d.k));
}

struct LrBufs {
  float* Q; int32_t* table2; float* P; float* T; float* W; float* X1; float* lpart; int* lwork;
};
static LrBufs carve_lr(Arena& ar, const Dims& d) {
  LrBufs l;
  l.Q = ar.get<float>((size_t)d.m * d.k);
  l.table2 = ar.get<int32_t>((size_t)d.m * d.s);
  l.P = ar.get<float>((size_t)d.r1 * d.k);
  l.T = ar.get<float>((size_t)d.r1 * d.n);
  l.W = ar.get<float>((size_t)d.k * d.n);
  l.X1 = ar.get<float>((size_t)d.k * d.n);
  size_t lp = sketch_left_partial_floats(d.m, d.n, d.r1);
  size_t lp2 = sketch_left_partial_floats(d.m, d.k, d.r1);
  l.lpart = ar.get<float>(lp > lp2 ? lp : lp2);
  l.lwork = ar.get<int>(sketch_left_work_ints(d.n > d.k ? d.n : d.k, d.r1));
  return l;
}

struct NyBufs {
  float* Wt; float* Yc; float* Yn; float* T1; double* W64; double* lam; double* V; float* V32; float* scale;
  void* eigw; float* lpart; float* Cbuf; int* lwork;
};
static NyBufs carve_ny(Arena& ar, const Dims& d) {
  NyBufs y;
  y.Wt = ar.get<float>((size_t)d.r1 * d.r1);
  y.Yc = ar.get<float>((size_t)d.r1 * d.k);
  y.Yn = ar.get<float>((size_t)d.r1 * d.k);
  y.T1 = ar.get<float>((size_t)d.r1 * d.k);
  y.W64 = ar.get<double>((size_t)d.k * d.k);
  y.lam = ar.get<double>(d.k);
  y.V = ar.get<double>((size_t)d.k * d.k);
  y.V32 = ar.get<float>((size_t)d.k * d.k);
  y.scale = ar.get<float>(d.k);
  y.eigw = ar.get<char>(eig_work_bytes(d.k));
  y.lpart = ar.get<float>(sketch_left_partial_floats(d.n, d.r1, d.r1));
  y.lwork = ar.get<int>(sketch_left_work_ints(d.r1, d.r1));
  y.Cbuf = ar.get<float>((size_t)d.n * d.k);
  return y;
}

static size_t ws_size(int op, const Dims& d) {
  Arena ar(nullptr);
  carve_rf(ar, d);
  if (op == RF_OP_SVD) {
    carve_svd(ar, d);
    carve_gpart_big(ar, d);
  } else if (op == RF_OP_LOWRANK) {
    carve_lr(ar, d);
  } else if (op == RF_OP_NYSTROM) {
    carve_ny(ar, d);
  } else {
    ar.get<float>((size_t)d.m * d.k);
  }
  return ar.off + 256;
}

static rf_status finish(Ctx& c) { return c.err == hipSuccess ? RF_OK : RF_EHIP; }

static void* align_ws(void* ws) { return (void*)(((uintptr_t)ws + 255) / 256 * 256); }

}  // namespace

extern "C" {

const char* rf_status_string(rf_status s) {
  switch (s) {
    case RF_OK: return "ok";
    case RF_EINVAL: return "invalid argument";
    case RF_EWORKSPACE: return "workspace too small";
    case RF_EUNSUPPORTED: return "unsupported";
    case RF_EHIP: return "HIP launch error";
  }
  return "unknown status";
}

// Buffers of the sketch pass alone (rf_sketch_apply): the At-producing draws of
// carve_rf without the power loop's buffers.
static RFBufs carve_sketch(Arena& ar, const Dims& d) {
  RFBufs b;
  memset(&b, 0, sizeof(b));
  const bool mixed = d.prec == RF_PREC_MIXED;
  const bool sparse = d.family == 0, dense = d.family == 1 || d.family == 2, srht = d.family == 3;
  b.table = sparse ? ar.get<int32_t>((size_t)d.n * d.s) : nullptr;
  b.ready = sparse ? ar.get<uint32_t>((size_t)d.n * d.s) : nullptr;
  b.cmax = sparse ? ar.get<int>(sketch_right_work_ints(d.n, d.s, d.r1)) : nullptr;
  b.Sd = dense ? ar.get<float>((size_t)d.n * d.r1) : nullptr;
  b.Sd16 = (dense && (mixed || d.dtype == RF_BF16)) ? ar.get<uint16_t>((size_t)d.n * d.r1) : nullptr;
  b.srd = srht ? ar.get<float>((size_t)srht_size(d.n)) : nullptr;
  b.picks = srht ? ar.get<int>((size_t)d.r1) : nullptr;
  return b;
}

static bool sketch_apply_args_ok(const rf_matrix* A, const rf_params* p) {
  // the sketch itself needs only 1 <= s <= r1 (any r1, any shape of A)
  if (!valid_matrix(A) || !p || p->sketch < 1 || p->nnz_per_col < 1 || p->nnz_per_col > p->sketch) return false;
  if (p->flags & ~(RF_FLAG_ORTH_ERR | RF_SKETCH_MASK)) return false;
  return p->precision == RF_PREC_FP32 || p->precision == RF_PREC_MIXED;
}

size_t rf_sketch_apply_ws(const rf_matrix* A, const rf_params* p) {
  if (!sketch_apply_args_ok(A, p)) return 0;
  Arena ar(nullptr);
  carve_sketch(ar, dims_of(A, p));
  return ar.off + 256;
}

size_t rf_workspace_size(int op, const rf_matrix* A, const rf_params* p) {
  if (op < RF_OP_RANGE_FINDER || op > RF_OP_NYSTROM) return 0;
  if (!valid_matrix(A) || !valid_params(A, p, op == RF_OP_NYSTROM)) return 0;
  return ws_size(op, dims_of(A, p));
}

rf_status rf_sketch_table(int64_t n, int32_t s, int32_t r1, uint64_t seed, uint32_t stream_id, uint32_t b,
                          int32_t* out, void* stream) {
  if (n < 0 || s < 1 || r1 < s || (!out && n > 0)) return RF_EINVAL;
  return launch_sketch_table(n, s, r1, seed, stream_id, b, out, (hipStream_t)stream) == hipSuccess ? RF_OK : RF_EHIP;
}

rf_status rf_gaussian(int64_t rows, int64_t cols, uint64_t seed, uint32_t stream_id, uint32_t b, float* out,
                      void* stream) {
  if (rows < 0 || cols < 0 || (!out && rows * cols > 0)) return RF_EINVAL;
  return launch_gaussian(rows, cols, seed, stream_id, b, out, cols, (hipStream_t)stream) == hipSuccess ? RF_OK
                                                                                                        : RF_EHIP;
}

rf_status rf_sketch_apply(const rf_matrix* A, const rf_params* p, float* out, int64_t ldo, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!sketch_apply_args_ok(A, p) || !out || ldo < p->sketch) return RF_EINVAL;
  Dims d = dims_of(A, p);
  d.k = 1;
  if (family_unsupported(A, d)) return RF_EUNSUPPORTED;
  if (!ws || ws_bytes < rf_sketch_apply_ws(A, p)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_sketch(ar, d);
  Ctx c;
  c.st = (hipStream_t)stream;
  sketch_right_any(c, A, d, p->seed, b, out, ldo, nullptr);
  return finish(c);
}

// S2^T A as rf_lowrank computes it (Algorithm 2): table of stream 2 over the m rows
static size_t carve_left(Arena& ar, const rf_matrix* A, const rf_params* p, int32_t** table, float** part, int** work) {
  const int64_t m = A->rows, n = A->cols;
  const int r1 = p->sketch, s = p->nnz_per_col;
  *table = ar.get<int32_t>((size_t)m * s);
  *part = ar.get<float>(sketch_left_partial_floats(m, n, r1));
  *work = ar.get<int>(sketch_left_work_ints(n, r1));
  return ar.off + 256;
}

size_t rf_sketch_apply_left_ws(const rf_matrix* A, const rf_params* p) {
  if (!valid_matrix(A) || !p || p->sketch < 1 || p->nnz_per_col < 1 || p->nnz_per_col > p->sketch) return 0;
  Arena ar(nullptr);
  int32_t* t; float* pa; int* w;
  return carve_left(ar, A, p, &t, &pa, &w);
}

rf_status rf_sketch_apply_left(const rf_matrix* A, const rf_params* p, float* out, int64_t ldo, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!valid_matrix(A) || !p || p->sketch < 1 || p->nnz_per_col < 1 || p->nnz_per_col > p->sketch || !out ||
      ldo < A->cols)
    return RF_EINVAL;
  if (!ws || ws_bytes < rf_sketch_apply_left_ws(A, p)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  int32_t* table; float* part; int* work;
  carve_left(ar, A, p, &table, &part, &work);
  Ctx c;
  c.st = (hipStream_t)stream;
  c.chk(launch_sketch_table(A->rows, p->nnz_per_col, p->sketch, p->seed, 2, 0, table, c.st));
  c.chk(launch_sketch_left(A->dtype, A->data, A->ld, table, p->nnz_per_col, A->rows, A->cols, p->sketch, out, ldo,
                           part, c.st, A->block_scales, work));
  return finish(c);
}

// Algorithm 1 as an entry point: rf_range_finder draws S and Omega from the seed,
// rf_range_finder_ex may take either from the caller.
static rf_status range_finder_entry(const rf_matrix* A, const rf_params* p, const int32_t* S_table,
                                    const float* Omega, float* Q, int64_t ldq, void* ws, size_t ws_bytes,
                                    rf_info* info, void* stream) {
  if (!valid_matrix(A) || !valid_params(A, p, false) || !Q || ldq < p->k) return RF_EINVAL;
  Dims d = dims_of(A, p);
  if ((d.classical || d.family != 0) && S_table) return RF_EINVAL;  // only the sparse sign sketch has a table
  if (family_unsupported(A, d)) return RF_EUNSUPPORTED;
  if (d.classical && A->dtype != RF_F32) return RF_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_size(RF_OP_RANGE_FINDER, d)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_rf(ar, d);
  float* Qw = ar.get<float>((size_t)d.m * d.k);
  if (ldq == d.k) Qw = Q;
  Ctx c;
  c.st = (hipStream_t)stream;
  const int32_t* table = nullptr;
  if (S_table) {
    // entries outside their block are replaced and reported (info status bit 8)
    c.chk(launch_fill_i32(b.counters, 16, 0, c.st));
    c.chk(launch_table_sanitize(S_table, d.n, d.s, d.r1, b.table, &b.counters[6], c.st));
    table = b.table;
  }
  range_finder_core(c, A, d, p->seed, b, Qw, table, Omega);
  if (p->flags & RF_FLAG_ORTH_ERR) {
    c.chk(launch_gram(Qw, d.k, 0, Qw, d.k, 0, d.m, d.k, d.k, 1, b.G, d.k, b.gpart, nullptr, c.st));
    c.chk(launch_orth_err(b.G, d.k, d.k, b.orth, c.st));
  }
  if (Qw != Q) c.chk(launch_copy_f32(Qw, d.k, Q, ldq, d.m, d.k, c.st));
  c.chk(launch_info(info, b.counters, d.k, (p->flags & RF_FLAG_ORTH_ERR) ? b.orth : nullptr, c.st));
  return finish(c);
}

rf_status rf_range_finder(const rf_matrix* A, const rf_params* p, float* Q, int64_t ldq, void* ws, size_t ws_bytes,
                          rf_info* info, void* stream) {
  return range_finder_entry(A, p, nullptr, nullptr, Q, ldq, ws, ws_bytes, info, stream);
}

rf_status rf_range_finder_ex(const rf_matrix* A, const int32_t* S_table, const float* Omega, const rf_params* p,
                             float* Q, int64_t ldq, void* ws, size_t ws_bytes, rf_info* info, void* stream) {
  return range_finder_entry(A, p, S_table, Omega, Q, ldq, ws, ws_bytes, info, stream);
}

}  // extern "C"

// Rayleigh-Ritz on B = Q^T A given B^T (s.Bt, n x k) and Q (s.Q): B B^T =
// Ub diag(lam) Ub^T in FP64, sigma = sqrt(lam), U = Q Ub, V^T = Sigma^-1 Ub^T B.
static void svd_tail(Ctx& c, const Dims& d, SvdBufs& s, double* gbig, float* U, int64_t ldu, double* sigma, float* Vt,
                     int64_t ldvt) {
  const int k = d.k;
  c.chk(launch_gram(s.Bt, k, 0, s.Bt, k, 0, d.n, k, k, 1, s.GB, k, gbig, nullptr, c.st));
  c.chk(launch_eig(s.GB, k, k, s.lam, s.Ub, k, s.eigw, c.st, kEigTolFP32));
  c.chk(launch_sigma(s.lam, k, sigma, s.inv, c.st));
  c.chk(launch_cast_f64_f32(s.Ub, k, s.Ub32, k, k, k, c.st));
  // U = Q Ub ; V = B^T Ub Sigma^{-1} stored transposed as Vt
  gemm(c, 0, s.Q, k, 1, s.Ub32, k, 0, U, ldu, d.m, k, k, nullptr);
  gemm(c, 0, s.Bt, k, 1, s.Ub32, k, 0, Vt, ldvt, d.n, k, k, nullptr, s.inv, 1);
  c.chk(launch_sign_fix(U, ldu, d.m, k, Vt, ldvt, d.n, s.signw, c.st));
}

extern "C" {

rf_status rf_svd(const rf_matrix* A, const rf_params* p, float* U, int64_t ldu, double* sigma, float* Vt, int64_t ldvt,
                 void* ws, size_t ws_bytes, rf_info* info, void* stream) {
  if (!valid_matrix(A) || !valid_params(A, p, false) || !U || !sigma || !Vt || ldu < p->k || ldvt < A->cols)
    return RF_EINVAL;
  if (p->k > 4096) return RF_EUNSUPPORTED;
  Dims d = dims_of(A, p);
  if ((d.classical && A->dtype != RF_F32) || family_unsupported(A, d)) return RF_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_size(RF_OP_SVD, d)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_rf(ar, d);
  SvdBufs s = carve_svd(ar, d);
  double* gbig = carve_gpart_big(ar, d);
  Ctx c;
  c.st = (hipStream_t)stream;
  const int k = d.k;
  range_finder_core(c, A, d, p->seed, b, s.Q, nullptr, nullptr);
  if (p->flags & RF_FLAG_ORTH_ERR) {
    c.chk(launch_gram(s.Q, k, 0, s.Q, k, 0, d.m, k, k, 1, b.G, k, b.gpart, nullptr, c.st));
    c.chk(launch_orth_err(b.G, k, k, b.orth, c.st));
  }
  // B^T = A^T Q (n x k): the one extra pass over A of the randomised SVD.  BF16
  // products when A is stored in BF16, or in the mixed form (FP32 A is then
  // rounded to BF16 as it is loaded).
  if (A->dtype == RF_FP8E4M3_B128 && d.prec == RF_PREC_MIXED) {
    // FP8 x FP8 on MFMA: Q rounded to e4m3 (E8M0 scale per 32 rows and column), A's
    // codes and block scales used as stored
    c.chk(launch_quant_q_fp8(s.Q, d.m, k, k, s.qf8c, s.qf8s, c.st));
    gemm(c, 7, A->data, A->ld, 0, s.qf8c, qf8_col_blocks(k), 0, s.Bt, k, d.n, k, d.m, s.qpart, nullptr, 0, 0, 0,
         A->block_scales, (d.n + 127) / 128, kQtaSplitCap, 1.f, s.qf8s);
  } else if (A->dtype == RF_FP8E4M3_B128) {
    // plain form: block-scaled FP8 A is dequantised and rounded to BF16 as it is loaded
    uint16_t* q16 = b.Q16 ? b.Q16 : (uint16_t*)b.Ya;
    c.chk(launch_cast_f32_bf16(s.Q, k, q16, k, d.m, k, c.st));
    gemm(c, 6, A->data, A->ld, 0, q16, k, 0, s.Bt, k, d.n, k, d.m, s.qpart, nullptr, 0, 0, 0, A->block_scales,
         (d.n + 127) / 128, kQtaSplitCap);
  } else if (A->dtype == RF_BF16 || d.prec == RF_PREC_MIXED) {
    uint16_t* q16 = b.Q16 ? b.Q16 : (uint16_t*)b.Ya;
    c.chk(launch_cast_f32_bf16(s.Q, k, q16, k, d.m, k, c.st));
    gemm(c, A->dtype == RF_BF16 ? 2 : 4, A->data, A->ld, 0, q16, k, 0, s.Bt, k, d.n, k, d.m, s.qpart, nullptr, 0, 0,
         0, nullptr, 0, kQtaSplitCap);
  } else {
    gemm(c, 0, A->data, A->ld, 0, s.Q, k, 0, s.Bt, k, d.n, k, d.m, s.qpart, nullptr, 0, 0, 0, nullptr, 0,
         kQtaSplitCap);
  }
  svd_tail(c, d, s, gbig, U, ldu, sigma, Vt, ldvt);
  c.chk(launch_info(info, b.counters, k, (p->flags & RF_FLAG_ORTH_ERR) ? b.orth : nullptr, c.st));
  return finish(c);
}

rf_status rf_lowrank(const rf_matrix* A, const rf_params* p, float* Y, int64_t ldy, float* X, int64_t ldx, void* ws,
                     size_t ws_bytes, rf_info* info, void* stream) {
  if (!valid_matrix(A) || !valid_params(A, p, false) || !Y || !X || ldy < p->k || ldx < A->cols) return RF_EINVAL;
  Dims d = dims_of(A, p);
  if ((d.classical && A->dtype != RF_F32) || family_unsupported(A, d)) return RF_EUNSUPPORTED;
  if (!ws || ws_bytes < ws_size(RF_OP_LOWRANK, d)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_rf(ar, d);
  LrBufs l = carve_lr(ar, d);
  Ctx c;
  c.st = (hipStream_t)stream;
  const int k = d.k, r1 = d.r1;
  range_finder_core(c, A, d, p->seed, b, l.Q, nullptr, nullptr);
  // S2 (m x r1, stream 2): P = S2^T Q (r1 x k), T = S2^T A (r1 x n, second pass over A)
  c.chk(launch_sketch_table(d.m, d.s, r1, p->seed, 2, 0, l.table2, c.st));
  c.chk(launch_sketch_left(0, l.Q, k, l.table2, d.s, d.m, k, r1, l.P, k, l.lpart, c.st, nullptr, l.lwork));
  c.chk(launch_sketch_left(A->dtype, A->data, A->ld, l.table2, d.s, d.m, d.n, r1, l.T, d.n, l.lpart, c.st,
                           A->block_scales, l.lwork));
  // X = (P^T P)^{-1} P^T T with P^T P = R^T R (FP64):  X = Rinv (Rinv^T (P^T T))
  c.chk(launch_gram(l.P, k, 0, l.P, k, 0, r1, k, k, 1, b.G, k, b.gpart, nullptr, c.st));
  c.chk(launch_cholinv(b.G, k, k, chol_tol(k), b.d0, b.flags, &b.counters[0], &b.counters[2], &b.counters[5], nullptr,
                       b.triwork, k, b.Rinv, k, b.cwork, c.st));
  gemm(c, 0, l.P, k, 0, l.T, d.n, 0, l.W, d.n, k, d.n, r1, nullptr);          // W = P^T T
  gemm(c, 0, b.Rinv, k, 0, l.W, d.n, 0, l.X1, d.n, k, d.n, k, nullptr);       // X1 = Rinv^T W
  gemm(c, 0, b.Rinv, k, 1, l.X1, d.n, 0, X, ldx, k, d.n, k, nullptr);         // X = Rinv X1
  c.chk(launch_copy_f32(l.Q, k, Y, ldy, d.m, k, c.st));
  c.chk(launch_info(info, b.counters, k, nullptr, c.st));
  return finish(c);
}

rf_status rf_nystrom(const rf_matrix* A, const rf_params* p, float* C, int64_t ldc, double* W, int64_t ldw, float* F,
                     int64_t ldf, void* ws, size_t ws_bytes, rf_info* info, void* stream) {
  if (!valid_matrix(A) || !valid_params(A, p, true) || !C || !W || ldc < p->k || ldw < p->k || (F && ldf < p->k))
    return RF_EINVAL;
  if (F && p->k > 4096) return RF_EUNSUPPORTED;
  if (p->flags & (RF_FLAG_CLASSICAL | RF_SKETCH_MASK)) return RF_EUNSUPPORTED;  // sparse sign S only
  Dims d = dims_of(A, p);
  if (!ws || ws_bytes < ws_size(RF_OP_NYSTROM, d)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_rf(ar, d);
  NyBufs y = carve_ny(ar, d);
  Ctx c;
  c.st = (hipStream_t)stream;
  const int k = d.k, r1 = d.r1;
  const int64_t n = d.n;
  c.chk(launch_fill_i32(b.counters, 16, 0, c.st));
  // Ct = A S (n x r1), Wt = S^T Ct (r1 x r1), symmetrised
  c.chk(launch_sketch_table(n, d.s, r1, p->seed, 0, 0, b.table, c.st));
  const bool fast = sketch_right_fast_ok(d.s) && !sketch_right_gather(d.s, d.n, d.r1);
  if (fast) c.chk(launch_sketch_ready(b.table, n, d.s, r1, sketch_right_cpl(d.s), b.ready, c.st));
  c.chk(launch_gaussian(r1, k, p->seed, 1, 0, b.om, k, c.st));
  c.chk(launch_sketch_right(A->dtype, A->data, A->ld, A->block_scales, b.table, fast ? b.ready : nullptr, b.cmax, d.s, n, n,
                            r1, b.At, r1, c.st));
  c.chk(launch_sketch_left(0, b.At, r1, b.table, d.s, n, r1, r1, y.Wt, r1, y.lpart, c.st, nullptr, y.lwork));
  c.chk(launch_symmetrize(y.Wt, r1, r1, c.st));
  // Y = Wt^q Omega, re-orthonormalised after every product.  Mixed form: every
  // product but the last on BF16 MFMA (Wt and Y rounded to BF16; the iterate is
  // re-orthonormalised in FP64 Gram/Cholesky afterwards), the last one in FP32
  // so that the span of the final Y, which fixes C and W, carries FP32 rounding
  // only (the same rule as the last power product of Algorithm 1).  C = Ct Y
  // stays FP32 in both forms: C W^+ C^T is quadratic in C.
  const bool mixed = d.prec == RF_PREC_MIXED;
  uint16_t* Wt16 = b.At16;  // n x r1 BF16 buffer of the mixed form, >= r1 x r1
  uint16_t* Y16 = b.om16;   // r1 x k BF16
  if (mixed && d.q > 1) c.chk(launch_cast_f32_bf16(y.Wt, r1, Wt16, r1, r1, r1, c.st));
  c.chk(launch_copy_f32(b.om, k, y.Yc, k, r1, k, c.st));
  for (int j = 0; j < d.q; ++j) {
    if (mixed && j + 1 < d.q) {
      c.chk(launch_cast_f32_bf16(y.Yc, k, Y16, k, r1, k, c.st));
      gemm(c, 2, Wt16, r1, 1, Y16, k, 0, y.T1, k, r1, k, r1, nullptr);
    } else {
      gemm(c, 0, y.Wt, r1, 1, y.Yc, k, 0, y.T1, k, r1, k, r1, nullptr);
    }
    cholqr_pass(c, b, y.T1, y.Yn, r1, k, p->seed);
    float* t = y.Yc; y.Yc = y.Yn; y.Yn = t;
  }
  // C = Ct Y (n x k) ; W = Y^T (Wt Y) in FP64
  gemm(c, 0, b.At, r1, 1, y.Yc, k, 0, y.Cbuf, k, n, k, r1, nullptr);
  gemm(c, 0, y.Wt, r1, 1, y.Yc, k, 0, y.T1, k, r1, k, r1, nullptr);
  c.chk(launch_gram(y.Yc, k, 0, y.T1, k, 0, r1, k, k, 0, y.W64, k, b.gpart, nullptr, c.st));
  c.chk(launch_copy_f32(y.Cbuf, k, C, ldc, n, k, c.st));
  // W to the caller, symmetrised (Y^T Wt Y is symmetric up to rounding)
  c.chk(launch_symmetrize64(y.W64, k, k, c.st));
  c.chk(launch_copy_f64(y.W64, k, W, ldw, k, k, c.st));
  if (F) {
    c.chk(launch_eig(y.W64, k, k, y.lam, y.V, k, y.eigw, c.st, kEigTolFP32));
    c.chk(launch_nystrom_scale(y.lam, k, y.scale, c.st));
    c.chk(launch_cast_f64_f32(y.V, k, y.V32, k, k, k, c.st));
    gemm(c, 0, y.Cbuf, k, 1, y.V32, k, 0, F, ldf, n, k, k, nullptr, y.scale, 0);
  }
  c.chk(launch_info(info, b.counters, k, nullptr, c.st));
  return finish(c);
}

// ------------------------------------------------------------------ sparse A (CSR)
}  // extern "C"

static bool valid_csr(const rf_csr* A) {
  if (!A || !A->row_ptr || A->rows < 1 || A->cols < 1 || A->nnz < 0 || A->nnz >= ((int64_t)1 << 31)) return false;
  if (A->nnz > 0 && (!A->col_idx || !A->values)) return false;
  return true;
}

// The rf_matrix-shaped view of a CSR matrix for the shared checks (dtype FP32).
static rf_matrix csr_shape(const rf_csr* A) {
  rf_matrix v;
  memset(&v, 0, sizeof(v));
  v.data = A->row_ptr;
  v.rows = A->rows;
  v.cols = A->cols;
  v.ld = A->cols;
  v.dtype = RF_F32;
  return v;
}

struct CscBufs { int64_t* colptr; unsigned long long* cursor; int32_t* pos; int32_t* row_of; };
static CscBufs carve_csc(Arena& ar, const rf_csr* A) {
  CscBufs b;
  b.colptr = ar.get<int64_t>((size_t)A->cols + 1);
  b.cursor = ar.get<unsigned long long>((size_t)A->cols);
  b.pos = ar.get<int32_t>((size_t)A->nnz + 1);
  b.row_of = ar.get<int32_t>((size_t)A->nnz + 1);
  return b;
}

// Checks shared by the CSR entry points: the sparse sign sketch only (S = I
// would make the power loop a sparse product and the dense families a dense
// one), FP32 values, r1 small enough for one row's 64-bit accumulators in LDS.
static rf_status csr_check(const rf_csr* A, const rf_params* p, rf_matrix& shape) {
  if (!valid_csr(A)) return RF_EINVAL;
  shape = csr_shape(A);
  if (!valid_params(&shape, p, false)) return RF_EINVAL;
  if (p->flags & (RF_FLAG_CLASSICAL | RF_SKETCH_MASK)) return RF_EUNSUPPORTED;
  if (!sketch_csr_ok(p->sketch)) return RF_EUNSUPPORTED;
  return RF_OK;
}

static size_t csr_ws(int op, const rf_csr* A, const Dims& d) {
  Arena ar(nullptr);
  carve_rf(ar, d);
  if (op == RF_OP_SVD) {
    carve_svd(ar, d);
    carve_gpart_big(ar, d);
    carve_csc(ar, A);
  } else {
    ar.get<float>((size_t)d.m * d.k);
  }
  return ar.off + 256;
}

extern "C" {

size_t rf_workspace_size_csr(int op, const rf_csr* A, const rf_params* p) {
  rf_matrix shape;
  if ((op != RF_OP_RANGE_FINDER && op != RF_OP_SVD) || csr_check(A, p, shape) != RF_OK) return 0;
  return csr_ws(op, A, dims_of(&shape, p));
}

rf_status rf_range_finder_csr(const rf_csr* A, const rf_params* p, float* Q, int64_t ldq, void* ws, size_t ws_bytes,
                              rf_info* info, void* stream) {
  rf_matrix shape;
  const rf_status st = csr_check(A, p, shape);
  if (st != RF_OK) return st;
  if (!Q || ldq < p->k) return RF_EINVAL;
  Dims d = dims_of(&shape, p);
  if (!ws || ws_bytes < csr_ws(RF_OP_RANGE_FINDER, A, d)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_rf(ar, d);
  float* Qw = ar.get<float>((size_t)d.m * d.k);
  if (ldq == d.k) Qw = Q;
  Ctx c;
  c.st = (hipStream_t)stream;
  range_finder_core(c, &shape, d, p->seed, b, Qw, nullptr, nullptr, A);
  if (p->flags & RF_FLAG_ORTH_ERR) {
    c.chk(launch_gram(Qw, d.k, 0, Qw, d.k, 0, d.m, d.k, d.k, 1, b.G, d.k, b.gpart, nullptr, c.st));
    c.chk(launch_orth_err(b.G, d.k, d.k, b.orth, c.st));
  }
  if (Qw != Q) c.chk(launch_copy_f32(Qw, d.k, Q, ldq, d.m, d.k, c.st));
  c.chk(launch_info(info, b.counters, d.k, (p->flags & RF_FLAG_ORTH_ERR) ? b.orth : nullptr, c.st));
  return finish(c);
}

rf_status rf_svd_csr(const rf_csr* A, const rf_params* p, float* U, int64_t ldu, double* sigma, float* Vt,
                     int64_t ldvt, void* ws, size_t ws_bytes, rf_info* info, void* stream) {
  rf_matrix shape;
  const rf_status st = csr_check(A, p, shape);
  if (st != RF_OK) return st;
  if (!U || !sigma || !Vt || ldu < p->k || ldvt < A->cols) return RF_EINVAL;
  if (p->k > 4096) return RF_EUNSUPPORTED;
  Dims d = dims_of(&shape, p);
  if (!ws || ws_bytes < csr_ws(RF_OP_SVD, A, d)) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  RFBufs b = carve_rf(ar, d);
  SvdBufs s = carve_svd(ar, d);
  double* gbig = carve_gpart_big(ar, d);
  CscBufs t = carve_csc(ar, A);
  Ctx c;
  c.st = (hipStream_t)stream;
  const int k = d.k;
  range_finder_core(c, &shape, d, p->seed, b, s.Q, nullptr, nullptr, A);
  if (p->flags & RF_FLAG_ORTH_ERR) {
    c.chk(launch_gram(s.Q, k, 0, s.Q, k, 0, d.m, k, k, 1, b.G, k, b.gpart, nullptr, c.st));
    c.chk(launch_orth_err(b.G, k, k, b.orth, c.st));
  }
  // B^T = A^T Q as a sparse product over the CSC form of A (FP32 in both forms)
  c.chk(launch_csc_build(A->row_ptr, A->col_idx, d.m, d.n, A->nnz, t.colptr, t.cursor, t.pos, t.row_of, c.st));
  c.chk(launch_spmm_atq(t.colptr, t.pos, t.row_of, A->values, d.n, s.Q, k, k, s.Bt, k, c.st));
  svd_tail(c, d, s, gbig, U, ldu, sigma, Vt, ldvt);
  c.chk(launch_info(info, b.counters, k, (p->flags & RF_FLAG_ORTH_ERR) ? b.orth : nullptr, c.st));
  return finish(c);
}

rf_status rf_sketch_apply_csr(const rf_csr* A, const rf_params* p, float* out, int64_t ldo, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!valid_csr(A) || !p || p->sketch < 1 || p->nnz_per_col < 1 || p->nnz_per_col > p->sketch || !out ||
      ldo < p->sketch || p->flags != 0)
    return RF_EINVAL;
  if (!sketch_csr_ok(p->sketch)) return RF_EUNSUPPORTED;
  // workspace: the sketch table and the invalid-entry counter
  const size_t need = ((size_t)A->cols * p->nnz_per_col * sizeof(int32_t) + 255) / 256 * 256 + 512;
  if (!ws || ws_bytes < need) return RF_EWORKSPACE;
  Arena ar(align_ws(ws));
  int32_t* table = ar.get<int32_t>((size_t)A->cols * p->nnz_per_col);
  int* bad = ar.get<int>(1);
  Ctx c;
  c.st = (hipStream_t)stream;
  c.chk(launch_fill_i32(bad, 1, 0, c.st));
  c.chk(launch_sketch_table(A->cols, p->nnz_per_col, p->sketch, p->seed, 0, 0, table, c.st));
  c.chk(launch_sketch_csr(A->row_ptr, A->col_idx, A->values, A->rows, A->cols, A->nnz, table, p->nnz_per_col,
                          p->sketch, out, ldo, bad, c.st));
  return finish(c);
}

// ------------------------------------------------------------------ storage forms
rf_status rf_quantize_bf16(const float* A, int64_t rows, int64_t cols, int64_t lda, uint16_t* out, int64_t ldo,
                           void* stream) {
  if (rows < 0 || cols < 0 || lda < cols || ldo < cols || ((!A || !out) && rows * cols > 0)) return RF_EINVAL;
  return launch_quant_bf16(A, rows, cols, lda, out, ldo, (hipStream_t)stream) == hipSuccess ? RF_OK : RF_EHIP;
}

rf_status rf_quantize_fp8_b128(const float* A, int64_t rows, int64_t cols, int64_t lda, uint8_t* out, int64_t ldo,
                               float* scales, void* stream) {
  if (rows < 0 || cols < 0 || lda < cols || ldo < cols || ((!A || !out || !scales) && rows * cols > 0))
    return RF_EINVAL;
  if ((rows + 127) / 128 > 65535) return RF_EUNSUPPORTED;
  return launch_quant_fp8_b128(A, rows, cols, lda, out, ldo, scales, (hipStream_t)stream) == hipSuccess ? RF_OK
                                                                                                       : RF_EHIP;
}

// ------------------------------------------------------------------ parity hooks
rf_status rf_set_gemm_rules(const rf_gemm_rule* rules, int32_t count) {
  static_assert(sizeof(rf_gemm_rule) == sizeof(GemmRule), "rule layouts differ");
  return set_gemm_rules(reinterpret_cast<const GemmRule*>(rules), count) == 0 ? RF_OK : RF_EINVAL;
}

size_t rf_test_gemm_ws(int64_t M, int64_t N, int64_t K) { return gemm_partial_floats(M, N, K) * sizeof(float) + 256; }

rf_status rf_test_gemm(int dtype, int a_kc, int b_kc, const void* A, int64_t lda, const void* B, int64_t ldb, float* C,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, int b_upper, void* ws, void* stream) {
  if ((dtype != 0 && dtype != 2 && dtype != 4) || !A || !B || !C || M < 0 || N < 0 || K < 0 || ldc < N) return RF_EINVAL;
  if ((a_kc ? lda < K : lda < M) || (b_kc ? ldb < K : ldb < N)) return RF_EINVAL;
  Ctx c;
  c.st = (hipStream_t)stream;
  gemm(c, dtype, A, lda, a_kc ? 1 : 0, B, ldb, b_kc ? 1 : 0, C, ldc, M, N, K, ws ? (float*)align_ws(ws) : nullptr,
       nullptr, 0, b_upper ? 1 : 0);
  return finish(c);
}

rf_status rf_test_gemm_fp8a(const uint8_t* A, int64_t lda, const float* scales, const uint16_t* B, int64_t ldb, int b_kc,
                            float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* stream) {
  if (!A || !scales || !B || !C || M < 0 || N < 0 || K < 0 || ldc < N || lda < M || (b_kc ? ldb < K : ldb < N))
    return RF_EINVAL;
  Ctx c;
  c.st = (hipStream_t)stream;
  gemm(c, 6, A, lda, 0, B, ldb, b_kc ? 1 : 0, C, ldc, M, N, K, nullptr, nullptr, 0, 0, 0, scales, (M + 127) / 128);
  return finish(c);
}

size_t rf_test_qf8_bytes(int64_t m, int64_t k, int which) {
  if (m < 1 || k < 1) return 0;
  return which == 0 ? qf8_code_bytes(m, k) : qf8_scale_bytes(m, k);
}

rf_status rf_test_quant_q_fp8(const float* Q, int64_t m, int64_t k, int64_t ldq, uint8_t* codes, uint8_t* scales,
                              void* stream) {
  if (!Q || !codes || !scales || m < 1 || k < 1 || ldq < k) return RF_EINVAL;
  return launch_quant_q_fp8(Q, m, k, ldq, codes, scales, (hipStream_t)stream) == hipSuccess ? RF_OK : RF_EHIP;
}

size_t rf_test_gemm_fp8_ws(int64_t M, int64_t N, int64_t K) {
  if (M < 1 || N < 1 || K < 1) return 0;
  return gemm_partial_floats(M, N, K) * sizeof(float) + 256;
}

rf_status rf_test_gemm_fp8(const uint8_t* A, int64_t lda, const float* scales, const uint8_t* q_codes,
                           const uint8_t* q_scales, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!A || !scales || !q_codes || !q_scales || !C || M < 1 || N < 1 || K < 1 || lda < M || ldc < N)
    return RF_EINVAL;
  const size_t np = gemm_partial_floats(M, N, K);
  if (ws && ws_bytes < rf_test_gemm_fp8_ws(M, N, K)) return RF_EWORKSPACE;
  Ctx c;
  c.st = (hipStream_t)stream;
  gemm(c, 7, A, lda, 0, q_codes, qf8_col_blocks(N), 0, C, ldc, M, N, K, (ws && np) ? (float*)align_ws(ws) : nullptr,
       nullptr, 0, 0, 0, scales, (M + 127) / 128, 0, 1.f, q_scales);
  return finish(c);
}

size_t rf_test_gram_ws(int64_t K, int64_t M, int64_t N) { return gram_partial_doubles(K, M, N) * sizeof(double) + 256; }

rf_status rf_test_gram(const float* X, const float* Y, int64_t K, int64_t M, int64_t N, int sym, double* C, void* ws,
                       void* stream) {
  if (!X || !Y || !C || K < 0 || M < 0 || N < 0 || (sym && (X != Y || M != N))) return RF_EINVAL;
  return launch_gram(X, M, 0, Y, N, 0, K, M, N, sym ? 1 : 0, C, N, ws ? (double*)align_ws(ws) : nullptr, nullptr,
                     (hipStream_t)stream) == hipSuccess
             ? RF_OK
             : RF_EHIP;
}

size_t rf_test_chol_ws(int64_t N) {
  return (size_t)N * sizeof(double) + ((size_t)N + cholinv_work_ints(N)) * sizeof(int) + 4 * 256;
}

rf_status rf_test_cholqr_factor(double* G, int64_t N, double* Rinv, int32_t* counters, void* ws, void* stream) {
  if (!G || !Rinv || !counters || !ws || N < 1) return RF_EINVAL;
  Arena ar(align_ws(ws));
  double* d0 = ar.get<double>(N);
  int* flags = ar.get<int>(N);
  int* work = ar.get<int>(cholinv_work_ints(N));
  Ctx c;
  c.st = (hipStream_t)stream;
  c.chk(launch_fill_i32(counters, 16, 0, c.st));
  c.chk(launch_cholinv(G, N, N, chol_tol((int)N), d0, flags, &counters[0], &counters[2], &counters[5], nullptr, Rinv,
                       N, nullptr, 0, work, c.st));
  return finish(c);
}

size_t rf_test_eig_ws(int64_t N) { return eig_work_bytes(N) + 256; }

rf_status rf_test_eig(const double* G, int64_t N, double tol, double* lam, double* V, double* sweep_trace, void* ws,
                      void* stream) {
  if (!G || !lam || !V || !ws || N < 1 || !(tol > 0.0)) return RF_EINVAL;
  if (N > 4096) return RF_EUNSUPPORTED;
  return launch_eig(const_cast<double*>(G), N, N, lam, V, N, align_ws(ws), (hipStream_t)stream, tol, sweep_trace) ==
                 hipSuccess
             ? RF_OK
             : RF_EHIP;
}

}  // extern "C"
