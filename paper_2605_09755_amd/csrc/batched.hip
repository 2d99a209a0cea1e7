// Batched randomised SVD: many independent matrices of uneven shape and rank,
// each through the sketch-powered range finder (Algorithm 1) and the Rayleigh-Ritz
// finisher (Section 2), in one stream.
//
// Every stage is one grouped launch over all problems: the large passes (A S,
// the power products, Q^T A, the Grams) walk a flat work list of (problem, tile)
// items (per-stage prefix sums of tile counts, binary-searched by each
// workgroup); the small dense stages (Cholesky and inverse, Jacobi rounds,
// elementwise tails) take one problem per workgroup or grid row.  The
// descriptor arrays of every stage are built once, at plan time, and uploaded
// into the head of the caller's workspace; the launch sequence itself can be
// recorded once into a hipGraph and replayed.
//
// Descriptor "tape": the schedule below runs twice at plan time, once to size and
// fill the host copy of every descriptor array (launch = false) and once per run
// (launch = true, or under stream capture); both walks visit the call sites in
// the same order, so each call site finds its arrays at the same offsets.
#include <cstring>
#include <vector>

#include "kernels.h"
#include "rf.h"

namespace rf {
namespace {

constexpr size_t kAlign = 256;
static size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Tape {
  char* dev = nullptr;         // device base of the descriptor region
  std::vector<char>* host = nullptr;  // filled when building
  size_t off = 0;
  template <typename T>
  const T* put(const std::vector<T>& v) {
    const size_t bytes = round_up(v.size() * sizeof(T) + 1);
    if (host) {
      if (host->size() < off + bytes) host->resize(off + bytes);
      if (!v.empty()) std::memcpy(host->data() + off, v.data(), v.size() * sizeof(T));
    }
    const T* p = reinterpret_cast<const T*>(dev + off);
    off += bytes;
    return p;
  }
};

struct Prob {
  // inputs and outputs
  const float* A; int64_t lda; int64_t m, n; int k, r1, s;
  uint64_t seed;
  float* U; int64_t ldu; double* sigma; float* Vt; int64_t ldvt;
  // workspace
  int32_t* table; uint32_t* ready; int* cmax;
  float* om; uint16_t* om16;
  float* At; uint16_t* At16;
  float* Ya; float* Yb; float* Q; uint16_t* Q16;
  float* Zh; float* Z; uint16_t* Z16;
  double* G; double* d0; int* flags; int* counters; float* Rinv; double* X64; double* gpart;
  float* Bt; double* GB; double* lam; double* Ub; float* Ub32; float* inv; void* eigw; int* signw;
};

constexpr int kCounterStride = 16;

}  // namespace
}  // namespace rf

struct rf_batch_plan {
  int count = 0, q = 0;
  bool mixed = false;
  std::vector<rf::Prob> P;
  char* desc = nullptr;        // descriptor region (device)
  size_t desc_bytes = 0;
  int* counters = nullptr;     // count x 16 ints, contiguous
  int* ks = nullptr;           // device copy of k_i
  void* info = nullptr;
  int64_t mmax = 0, nmax = 0, kmax = 0, r1max = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace rf {
namespace {

struct Sched {
  rf_batch_plan& pl;
  Tape& tp;
  bool launch;
  hipStream_t st;
  hipError_t err = hipSuccess;
  void chk(hipError_t e) {
    if (e != hipSuccess && err == hipSuccess) err = e;
  }
  int count() const { return pl.count; }

  template <typename F>
  void gemm(int kind, int a_kc, int b_kc, F make) {
    std::vector<GemmArgs> gs(count());
    std::vector<int> ts(count() + 1, 0);
    for (int i = 0; i < count(); ++i) {
      GemmArgs g;
      std::memset(&g, 0, sizeof(g));
      g.alpha = 1.f;
      make(i, g);
      g.a_kc = a_kc; g.b_kc = b_kc;
      g.kps = g.K + 64;
      g.partial = nullptr;
      gs[i] = g;
      ts[i + 1] = ts[i] + ((g.M > 0 && g.N > 0) ? gemm_group_tiles(kind, g.M, g.N) : 0);
    }
    const GemmArgs* dg = tp.put(gs);
    const int* dt = tp.put(ts);
    if (launch) chk(launch_gemm_grouped(dg, dt, count(), ts[count()], kind, a_kc, b_kc, st));
  }

  template <typename F>
  void gram(F make) {
    std::vector<GramArgs> gs(count());
    std::vector<int> ts(count() + 1, 0);
    int64_t max_mm = 0;
    bool any_split = false;
    for (int i = 0; i < count(); ++i) {
      GramArgs g = make(i);
      // split-K into the problem's partial buffer (sized for its longest basis)
      int s = pl.P[i].gpart ? gram_group_splits(g.K) : 1;
      if (s > 1) {
        g.kps = ((g.K + s - 1) / s + 31) / 32 * 32;
        s = (int)((g.K + g.kps - 1) / g.kps);
      }
      if (s > 1) {
        g.partial = pl.P[i].gpart;
        g.splits = s;
        any_split = true;
      } else {
        g.partial = nullptr;
        g.splits = 1;
        g.kps = g.K;
      }
      gs[i] = g;
      max_mm = std::max<int64_t>(max_mm, g.M * g.M);
      ts[i + 1] = ts[i] + gram_group_tiles(g.M) * (s > 1 ? s : 1);
    }
    const GramArgs* dg = tp.put(gs);
    const int* dt = tp.put(ts);
    if (launch) chk(launch_gram_grouped(dg, dt, count(), ts[count()], max_mm, any_split, st));
  }

  template <typename F>
  void cast(int f64_to_f32, F make) {
    std::vector<CastArgs> cs(count());
    int64_t mx = 0;
    for (int i = 0; i < count(); ++i) {
      cs[i] = make(i);
      mx = std::max<int64_t>(mx, cs[i].rows * cs[i].cols);
    }
    const CastArgs* dc = tp.put(cs);
    if (launch) chk(launch_cast_batched(dc, count(), mx, f64_to_f32, st));
  }

  // One CholeskyQR pass per problem: out = X R^{-1}, X^T X = R^T R (rows x k).
  template <typename FX, typename FO, typename FR>
  void cholqr(FX X, FO out, FR rows) {
    const double u = 5.9604644775390625e-08;
    gram([&](int i) {
      const Prob& p = pl.P[i];
      return GramArgs{X(i), (int64_t)p.k, rows(i), (int64_t)p.k, p.G, (int64_t)p.k, nullptr};
    });
    std::vector<CholInvArgs> c1(count()), c2(count());
    std::vector<RefillArgs> rf(count());
    int64_t mx = 0;
    for (int i = 0; i < count(); ++i) {
      const Prob& p = pl.P[i];
      const double tol = 16.0 * (double)p.k * u * u;
      c1[i] = cholinv_desc(p.G, p.k, p.k, tol, p.d0, p.flags, &p.counters[0], &p.counters[2], nullptr, p.X64, p.k,
                           p.Rinv, p.k);
      c2[i] = cholinv_desc(p.G, p.k, p.k, tol, p.d0, p.flags, &p.counters[0], &p.counters[2], &p.counters[4], p.X64,
                           p.k, p.Rinv, p.k);
      rf[i] = RefillArgs{X(i), (int64_t)p.k, rows(i), (int64_t)p.k, p.flags, &p.counters[4], p.d0, p.seed, (uint32_t)i};
      mx = std::max<int64_t>(mx, rows(i) * p.k);
    }
    const CholInvArgs* d1 = tp.put(c1);
    const CholInvArgs* d2 = tp.put(c2);
    const RefillArgs* dr = tp.put(rf);
    std::vector<int*> cs(count());
    for (int i = 0; i < count(); ++i) cs[i] = pl.P[i].counters;
    int* const* dcs = tp.put(cs);
    if (launch) {
      chk(launch_cholinv_batched(d1, count(), st));
      chk(launch_note_batched(dcs, count(), 0, st));
      chk(launch_refill_batched(dr, count(), mx, st));
    }
    gram([&](int i) {
      const Prob& p = pl.P[i];
      return GramArgs{X(i), (int64_t)p.k, rows(i), (int64_t)p.k, p.G, (int64_t)p.k, &p.counters[4]};
    });
    if (launch) {
      chk(launch_cholinv_batched(d2, count(), st));
      chk(launch_note_batched(dcs, count(), 1, st));
    }
    gemm(0, 1, 0, [&](int i, GemmArgs& g) {
      const Prob& p = pl.P[i];
      g.A = X(i); g.lda = p.k; g.B = p.Rinv; g.ldb = p.k; g.C = out(i); g.ldc = p.k;
      g.M = rows(i); g.N = p.k; g.K = p.k; g.b_upper = 1;
    });
  }

  void run() {
    const int n = count();
    const bool mixed = pl.mixed;
    auto& P = pl.P;
    // counters of every problem (one contiguous block)
    if (launch) chk(launch_fill_i32(pl.counters, (int64_t)n * kCounterStride, 0, st));
    // sketch tables (stream 0), ready tables, Omega (stream 1); problem index = batch index
    {
      std::vector<RngArgs> ra(n);
      int64_t mx = 0;
      for (int i = 0; i < n; ++i) {
        const Prob& p = P[i];
        ra[i] = RngArgs{p.n, p.s, p.r1, p.k, 2, p.seed, (uint32_t)i, p.table, p.ready, p.om};
        mx = std::max<int64_t>(mx, std::max<int64_t>(p.n * p.s, (int64_t)p.r1 * p.k / 4 + 1));
      }
      const RngArgs* d = tp.put(ra);
      if (launch) chk(launch_rng_batched(d, n, mx, st));
    }
    // At = A S
    {
      std::vector<SketchArgs> sa(n);
      for (int i = 0; i < n; ++i) {
        const Prob& p = P[i];
        const bool vec = ((uintptr_t)p.A % 8 == 0) && (p.lda % 2 == 0);
        sa[i] = SketchArgs{p.A, p.lda, p.table, p.ready, p.cmax, p.m, p.n, p.r1, vec ? 1 : 0, p.At, (int64_t)p.r1};
      }
      const SketchArgs* d = tp.put(sa);
      if (launch) chk(launch_sketch_right_batched(d, n, pl.mmax, pl.nmax, (int)pl.r1max, st));
    }
    if (mixed) {
      cast(0, [&](int i) { const Prob& p = P[i]; return CastArgs{p.At, p.At16, p.m, p.r1, p.r1, p.r1}; });
      cast(0, [&](int i) { const Prob& p = P[i]; return CastArgs{p.om, p.om16, p.r1, p.k, p.k, p.k}; });
    }
    // Y0 = At Omega
    if (mixed && pl.q > 0)
      gemm(2, 1, 0, [&](int i, GemmArgs& g) {
        const Prob& p = P[i];
        g.A = p.At16; g.lda = p.r1; g.B = p.om16; g.ldb = p.k; g.C = p.Ya; g.ldc = p.k; g.M = p.m; g.N = p.k; g.K = p.r1;
      });
    else
      gemm(0, 1, 0, [&](int i, GemmArgs& g) {
        const Prob& p = P[i];
        g.A = p.At; g.lda = p.r1; g.B = p.om; g.ldb = p.k; g.C = p.Ya; g.ldc = p.k; g.M = p.m; g.N = p.k; g.K = p.r1;
      });
    auto rows_m = [&](int i) { return P[i].m; };
    auto rows_r1 = [&](int i) { return (int64_t)P[i].r1; };
    if (pl.q == 0) {
      cholqr([&](int i) { return P[i].Ya; }, [&](int i) { return P[i].Yb; }, rows_m);
      cholqr([&](int i) { return P[i].Yb; }, [&](int i) { return P[i].Q; }, rows_m);
    } else {
      cholqr([&](int i) { return P[i].Ya; }, [&](int i) { return P[i].Yb; }, rows_m);
      for (int j = 1; j <= pl.q; ++j) {
        // Zh = At^T Qc (contraction over m)
        if (mixed) {
          cast(0, [&](int i) { const Prob& p = P[i]; return CastArgs{p.Yb, p.Q16, p.m, p.k, p.k, p.k}; });
          gemm(2, 0, 0, [&](int i, GemmArgs& g) {
            const Prob& p = P[i];
            g.A = p.At16; g.lda = p.r1; g.B = p.Q16; g.ldb = p.k; g.C = p.Zh; g.ldc = p.k;
            g.M = p.r1; g.N = p.k; g.K = p.m;
          });
        } else {
          gemm(0, 0, 0, [&](int i, GemmArgs& g) {
            const Prob& p = P[i];
            g.A = p.At; g.lda = p.r1; g.B = p.Yb; g.ldb = p.k; g.C = p.Zh; g.ldc = p.k; g.M = p.r1; g.N = p.k; g.K = p.m;
          });
        }
        cholqr([&](int i) { return P[i].Zh; }, [&](int i) { return P[i].Z; }, rows_r1);
        const bool last = (j == pl.q);
        if (mixed && !last) {
          cast(0, [&](int i) { const Prob& p = P[i]; return CastArgs{p.Z, p.Z16, p.r1, p.k, p.k, p.k}; });
          gemm(2, 1, 0, [&](int i, GemmArgs& g) {
            const Prob& p = P[i];
            g.A = p.At16; g.lda = p.r1; g.B = p.Z16; g.ldb = p.k; g.C = p.Ya; g.ldc = p.k; g.M = p.m; g.N = p.k; g.K = p.r1;
          });
        } else {
          gemm(0, 1, 0, [&](int i, GemmArgs& g) {
            const Prob& p = P[i];
            g.A = p.At; g.lda = p.r1; g.B = p.Z; g.ldb = p.k; g.C = p.Ya; g.ldc = p.k; g.M = p.m; g.N = p.k; g.K = p.r1;
          });
        }
        if (last) {
          cholqr([&](int i) { return P[i].Ya; }, [&](int i) { return P[i].Yb; }, rows_m);
          cholqr([&](int i) { return P[i].Yb; }, [&](int i) { return P[i].Q; }, rows_m);
        } else {
          cholqr([&](int i) { return P[i].Ya; }, [&](int i) { return P[i].Yb; }, rows_m);
        }
      }
    }
    // B^T = A^T Q (n x k)
    if (mixed) {
      cast(0, [&](int i) { const Prob& p = P[i]; return CastArgs{p.Q, p.Q16, p.m, p.k, p.k, p.k}; });
      // k <= 1024 and mostly small: 128 x 128 tiles waste less of N than 256 x 256
      gemm(pl.kmax > 512 ? 4 : 5, 0, 0, [&](int i, GemmArgs& g) {
        const Prob& p = P[i];
        g.A = p.A; g.lda = p.lda; g.B = p.Q16; g.ldb = p.k; g.C = p.Bt; g.ldc = p.k; g.M = p.n; g.N = p.k; g.K = p.m;
      });
    } else {
      gemm(0, 0, 0, [&](int i, GemmArgs& g) {
        const Prob& p = P[i];
        g.A = p.A; g.lda = p.lda; g.B = p.Q; g.ldb = p.k; g.C = p.Bt; g.ldc = p.k; g.M = p.n; g.N = p.k; g.K = p.m;
      });
    }
    // Ritz: B B^T = Ub diag(lam) Ub^T (FP64)
    gram([&](int i) {
      const Prob& p = P[i];
      return GramArgs{p.Bt, (int64_t)p.k, p.n, (int64_t)p.k, p.GB, (int64_t)p.k, nullptr};
    });
    {
      std::vector<EigBatch> eb(n);
      for (int i = 0; i < n; ++i) {
        const Prob& p = P[i];
        eb[i] = eig_batch_desc(p.GB, p.k, p.k, p.lam, p.Ub, p.k, p.eigw, kEigTolFP32);
      }
      const EigBatch* d = tp.put(eb);
      if (launch) chk(launch_eig_batched(d, n, pl.kmax, st));
    }
    std::vector<SvdTailArgs> ta(n);
    int64_t mx = 0;
    for (int i = 0; i < n; ++i) {
      const Prob& p = P[i];
      ta[i] = SvdTailArgs{p.lam, p.Ub, p.Ub32, p.sigma, p.inv, p.signw, p.U, p.ldu, p.Vt, p.ldvt, p.m, p.n, p.k};
      mx = std::max<int64_t>(mx, (p.m + p.n) * p.k);
    }
    const SvdTailArgs* dta = tp.put(ta);
    if (launch) chk(launch_svd_tail_pre_batched(dta, n, pl.kmax, st));
    // U = Q Ub ; V = B^T Ub Sigma^{-1}, stored transposed
    gemm(0, 1, 0, [&](int i, GemmArgs& g) {
      const Prob& p = P[i];
      g.A = p.Q; g.lda = p.k; g.B = p.Ub32; g.ldb = p.k; g.C = p.U; g.ldc = p.ldu; g.M = p.m; g.N = p.k; g.K = p.k;
    });
    gemm(0, 1, 0, [&](int i, GemmArgs& g) {
      const Prob& p = P[i];
      g.A = p.Bt; g.lda = p.k; g.B = p.Ub32; g.ldb = p.k; g.C = p.Vt; g.ldc = p.ldvt; g.c_trans = 1;
      g.colscale = p.inv; g.M = p.n; g.N = p.k; g.K = p.k;
    });
    if (launch) chk(launch_svd_tail_sign_batched(dta, n, pl.kmax, pl.mmax, mx, st));
    if (launch) chk(launch_info_batched(pl.info, pl.counters, kCounterStride, pl.ks, n, st));
  }
};

// Per-problem buffers, carved from `base` (nullptr: sizing only).
static size_t carve(rf_batch_plan& pl, char* base, size_t off) {
  auto get = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += round_up(bytes);
    return p;
  };
  pl.counters = (int*)get((size_t)pl.count * kCounterStride * sizeof(int));
  pl.ks = (int*)get((size_t)pl.count * sizeof(int));
  for (auto& p : pl.P) {
    const size_t m = p.m, n = p.n, k = p.k, r1 = p.r1, s = p.s;
    p.table = (int32_t*)get(n * s * 4);
    p.ready = (uint32_t*)get(n * s * 4);
    p.cmax = (int*)get(sketch_right_cmax_ints(p.n) * 4);
    p.om = (float*)get(r1 * k * 4);
    p.om16 = pl.mixed ? (uint16_t*)get(r1 * k * 2) : nullptr;
    p.At = (float*)get(m * r1 * 4);
    p.At16 = pl.mixed ? (uint16_t*)get(m * r1 * 2) : nullptr;
    p.Ya = (float*)get(m * k * 4);
    p.Yb = (float*)get(m * k * 4);
    p.Q = (float*)get(m * k * 4);
    p.Q16 = pl.mixed ? (uint16_t*)get(m * k * 2) : nullptr;
    p.Zh = (float*)get(r1 * k * 4);
    p.Z = (float*)get(r1 * k * 4);
    p.Z16 = pl.mixed ? (uint16_t*)get(r1 * k * 2) : nullptr;
    p.G = (double*)get(k * k * 8);
    {
      // split-K parts of the Grams of this problem's bases (m, sketch and n rows)
      const int sp = std::max(gram_group_splits((int64_t)m), std::max(gram_group_splits((int64_t)r1),
                                                                      gram_group_splits((int64_t)n)));
      p.gpart = sp > 1 ? (double*)get((size_t)sp * k * k * 8) : nullptr;
    }
    p.d0 = (double*)get(k * 8);
    p.flags = (int*)get(k * 4);
    p.Rinv = (float*)get(k * k * 4);
    p.X64 = (double*)get(k * k * 8);
    p.Bt = (float*)get(n * k * 4);
    p.GB = (double*)get(k * k * 8);
    p.lam = (double*)get(k * 8);
    p.Ub = (double*)get(k * k * 8);
    p.Ub32 = (float*)get(k * k * 4);
    p.inv = (float*)get(k * 4);
    p.eigw = (void*)get(eig_work_bytes(p.k, true));
    p.signw = (int*)get(3 * k * 4);
  }
  for (int i = 0; i < pl.count; ++i) pl.P[i].counters = pl.counters ? pl.counters + (size_t)i * kCounterStride : nullptr;
  return off;
}

static rf_status build(int32_t count, const rf_matrix* As, const rf_params* ps, float* const* U, const int64_t* ldu,
                       double* const* sigma, float* const* Vt, const int64_t* ldvt, rf_batch_plan& pl) {
  if (count < 1 || !As || !ps) return RF_EINVAL;
  pl.count = count;
  pl.q = ps[0].q;
  pl.mixed = ps[0].precision == RF_PREC_MIXED;
  pl.P.assign(count, Prob{});
  for (int i = 0; i < count; ++i) {
    const rf_matrix& A = As[i];
    const rf_params& p = ps[i];
    if (!A.data || A.rows < 1 || A.cols < 1 || A.ld < A.cols || A.reserved != 0) return RF_EINVAL;
    const int64_t mn = A.rows < A.cols ? A.rows : A.cols;
    if (p.k < 1 || p.sketch < p.k || p.sketch > mn || p.q < 0 || p.q > 1000) return RF_EINVAL;
    if (p.precision != RF_PREC_FP32 && p.precision != RF_PREC_MIXED) return RF_EINVAL;
    if (p.nnz_per_col < 1 || p.nnz_per_col > p.sketch) return RF_EINVAL;
    if (U && (!U[i] || !ldu || ldu[i] < p.k)) return RF_EINVAL;
    if (Vt && (!Vt[i] || !ldvt || ldvt[i] < A.cols)) return RF_EINVAL;
    if (sigma && !sigma[i]) return RF_EINVAL;
    if (A.dtype != RF_F32 || p.nnz_per_col != 4 || p.q != pl.q || (p.precision == RF_PREC_MIXED) != pl.mixed ||
        p.k > 1024 || p.sketch > 1280)
      return RF_EUNSUPPORTED;
    Prob& q = pl.P[i];
    q.A = (const float*)A.data; q.lda = A.ld; q.m = A.rows; q.n = A.cols;
    q.k = p.k; q.r1 = p.sketch; q.s = p.nnz_per_col; q.seed = p.seed;
    q.U = U ? U[i] : nullptr; q.ldu = U ? ldu[i] : 0;
    q.sigma = sigma ? sigma[i] : nullptr;
    q.Vt = Vt ? Vt[i] : nullptr; q.ldvt = Vt ? ldvt[i] : 0;
    pl.mmax = std::max<int64_t>(pl.mmax, q.m);
    pl.nmax = std::max<int64_t>(pl.nmax, q.n);
    pl.kmax = std::max<int64_t>(pl.kmax, q.k);
    pl.r1max = std::max<int64_t>(pl.r1max, q.r1);
  }
  return RF_OK;
}

static size_t desc_bytes(rf_batch_plan& pl) {
  Tape tp;
  Sched s{pl, tp, false, nullptr};
  s.run();
  return round_up(tp.off);
}

}  // namespace
}  // namespace rf

using namespace rf;

extern "C" {

size_t rf_svd_batched_ws(int32_t count, const rf_matrix* As, const rf_params* ps) {
  rf_batch_plan pl;
  if (build(count, As, ps, nullptr, nullptr, nullptr, nullptr, nullptr, pl) != RF_OK) return 0;
  // sizing walk: outputs are not touched
  for (auto& p : pl.P) { p.U = nullptr; p.Vt = nullptr; p.sigma = nullptr; }
  const size_t d = desc_bytes(pl);
  return d + carve(pl, nullptr, 0) + kAlign;
}

rf_status rf_svd_batched_plan(int32_t count, const rf_matrix* As, const rf_params* ps, float* const* U,
                              const int64_t* ldu, double* const* sigma, float* const* Vt, const int64_t* ldvt,
                              rf_info* info, void* ws, size_t ws_bytes, int32_t use_graph, void* stream,
                              rf_batch_plan** plan) {
  if (!plan || !U || !sigma || !Vt || !ldu || !ldvt) return RF_EINVAL;
  *plan = nullptr;
  rf_batch_plan* pl = new rf_batch_plan();
  rf_status st = build(count, As, ps, U, ldu, sigma, Vt, ldvt, *pl);
  if (st != RF_OK) { delete pl; return st; }
  const size_t need = rf_svd_batched_ws(count, As, ps);
  if (!ws || ws_bytes < need) { delete pl; return RF_EWORKSPACE; }
  char* base = (char*)(((uintptr_t)ws + kAlign - 1) / kAlign * kAlign);
  pl->desc = base;
  pl->desc_bytes = desc_bytes(*pl);
  carve(*pl, base + pl->desc_bytes, 0);
  pl->info = info;
  // descriptor walk with the real pointers, then one upload
  std::vector<char> host;
  {
    Tape tp;
    tp.dev = pl->desc;
    tp.host = &host;
    Sched s{*pl, tp, false, (hipStream_t)stream};
    s.run();
  }
  std::vector<int> ks(count);
  for (int i = 0; i < count; ++i) ks[i] = pl->P[i].k;
  hipStream_t hs = (hipStream_t)stream;
  if (hipMemcpyAsync(pl->desc, host.data(), host.size(), hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemcpyAsync(pl->ks, ks.data(), ks.size() * sizeof(int), hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipStreamSynchronize(hs) != hipSuccess) {
    delete pl;
    return RF_EHIP;
  }
  if (use_graph) {
    // captured on a private stream (the caller's may be the legacy default stream,
    // which cannot be captured); the graph is later launched on the caller's stream
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { delete pl; return RF_EHIP; }
    Tape tp;
    tp.dev = pl->desc;
    Sched s{*pl, tp, true, cs};
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      delete pl;
      return RF_EHIP;
    }
    s.run();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess || s.err != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      delete pl;
      return RF_EHIP;
    }
    pl->graph = g;
    if (hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      delete pl;
      return RF_EHIP;
    }
  }
  *plan = pl;
  return RF_OK;
}

rf_status rf_svd_batched_run(rf_batch_plan* plan, void* stream) {
  if (!plan) return RF_EINVAL;
  hipStream_t hs = (hipStream_t)stream;
  if (plan->exec) return hipGraphLaunch(plan->exec, hs) == hipSuccess ? RF_OK : RF_EHIP;
  Tape tp;
  tp.dev = plan->desc;
  Sched s{*plan, tp, true, hs};
  s.run();
  return s.err == hipSuccess ? RF_OK : RF_EHIP;
}

void rf_svd_batched_destroy(rf_batch_plan* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

}  // extern "C"
