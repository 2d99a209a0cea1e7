// FP64 small dense linear algebra on the device: the Gram matrices, Cholesky
// factors and triangular inverses of CholeskyQR2 (re-orthonormalisation after
// each power step, remark after Algorithm 1; "orth" of Algorithm 1, line 2),
// and the symmetric eigensolver of the Rayleigh-Ritz step of the randomised SVD
// (SVD of B = Q^T A through the eigenpairs of B B^T, Section 2) and of the
// Nystrom core W (Algorithm 3).  Everything stays on the stream: no host
// round-trips, conditions are written to device counters.
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace rf {

// ============================== Gram: C = X^T Y (FP64) ==============================
constexpr int GT = 64;  // output tile
constexpr int GK = 16;  // k rows per step

RF_DEV void upper_tile(int id, int nt, int& tm, int& tn) {
  // enumerate tm <= tn row by row
  int r = 0, rem = id;
  while (rem >= nt - r) { rem -= nt - r; ++r; }
  tm = r;
  tn = r + rem;
}

// One k-step of a Gram operand: GKS rows of a 64-column panel, EPT consecutive
// elements per thread (256 threads), held in registers until stored to LDS.
template <typename T, int GKS>
struct GramStage {
  static constexpr int EPT = GKS * GT / 256;
  T v[EPT];
  RF_DEV void load(gptr<const T> P, int64_t ld, int64_t k0, int64_t kend, int64_t c0, int64_t cmax) {
    const int r = threadIdx.x / (GT / EPT), c = (threadIdx.x % (GT / EPT)) * EPT;
    const int64_t k = k0 + r, i = c0 + c;
    const gptr<const T> src = P + k * ld + i;
    if (k < kend && i + EPT <= cmax && (((uintptr_t)src) & 15) == 0) {
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int e = 0; e < EPT; e += 4) {
          const float4 x = *reinterpret_cast<gptr<const float4>>(src + e);
          v[e] = x.x; v[e + 1] = x.y; v[e + 2] = x.z; v[e + 3] = x.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < EPT; e += 2) {
          const double2 x = *reinterpret_cast<gptr<const double2>>(src + e);
          v[e] = x.x; v[e + 1] = x.y;
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = (k < kend && i + e < cmax) ? src[e] : T(0);
    }
  }
  RF_DEV void store(T (*S)[GT]) const {
    const int r = threadIdx.x / (GT / EPT), c = (threadIdx.x % (GT / EPT)) * EPT;
#pragma unroll
    for (int e = 0; e < EPT; ++e) S[r][c + e] = v[e];
  }
};

// C tile (64 x 64) = X[:, i0..]^T Y[:, j0..] over rows [split*kps, +kps) on
// v_mfma_f64_16x16x4f64 (operands widened to FP64 as they leave LDS).  Operand
// panels are staged in LDS in their own type, double-buffered with a register
// prefetch of the next k-step, one barrier per step.
template <typename TX, typename TY>
RF_DEV void gram_body(gptr<const TX> X, int64_t ldx, gptr<const TY> Y, int64_t ldy, int64_t K,
                      int64_t M, int64_t N, int sym, gptr<double> C, int64_t ldc,
                      gptr<double> partial, int64_t kps, int bid, int split) {
  constexpr int GKS = (sizeof(TX) == 4 && sizeof(TY) == 4) ? 32 : 16;  // k rows per step: 32 KB of LDS
  __shared__ TX Xs[2][GKS][GT];
  __shared__ TY Ys[2][GKS][GT];
  const int ntm = (int)((M + GT - 1) / GT), ntn = (int)((N + GT - 1) / GT);
  int tm, tn;
  if (sym) upper_tile(bid, ntm, tm, tn);
  else { tm = bid / ntn; tn = bid % ntn; }
  const int64_t i0 = (int64_t)tm * GT, j0 = (int64_t)tn * GT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const int64_t kbeg = (int64_t)split * kps, kend = min(K, kbeg + kps);
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
  GramStage<TX, GKS> sx;
  GramStage<TY, GKS> sy;
  const int nst = kend > kbeg ? (int)((kend - kbeg + GKS - 1) / GKS) : 0;
  if (nst > 0) {
    sx.load(X, ldx, kbeg, kend, i0, M);
    sy.load(Y, ldy, kbeg, kend, j0, N);
    sx.store(Xs[0]);
    sy.store(Ys[0]);
    __syncthreads();
  }
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) {
      const int64_t k1 = kbeg + (int64_t)(st + 1) * GKS;
      sx.load(X, ldx, k1, kend, i0, M);
      sy.load(Y, ldy, k1, kend, j0, N);
    }
#pragma unroll
    for (int kk = 0; kk < GKS / 4; ++kk) {
      const int kr = 4 * kk + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = (double)Xs[buf][kr][wm * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bf[b] = (double)Ys[buf][kr][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (st + 1 < nst) {
      sx.store(Xs[buf ^ 1]);
      sy.store(Ys[buf ^ 1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64 output: register r of lane l holds row (l/16) + 4r, column l%16
        int64_t i = i0 + wm * 32 + a * 16 + (lane >> 4) + 4 * r;
        int64_t j = j0 + wn * 32 + b * 16 + (lane & 15);
        if (i >= M || j >= N) continue;
        if (sym && i > j) continue;
        double v = acc[a][b][r];
        if (partial) {
          partial[((int64_t)split * M + i) * N + j] = v;
        } else {
          C[i * ldc + j] = v;
          if (sym && i != j) C[j * ldc + i] = v;
        }
      }
}

template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_gram(const TX* __restrict__ X, int64_t ldx, const TY* __restrict__ Y,
                                              int64_t ldy, int64_t K, int64_t M, int64_t N, int sym,
                                              double* __restrict__ C, int64_t ldc, double* __restrict__ partial,
                                              int64_t kps, const int* run_if) {
  if (run_if && *run_if == 0) return;
  gram_body<TX, TY>(as_global<TX>(X), ldx, as_global<TY>(Y), ldy, K, M, N, sym, as_global_w<double>(C), ldc,
                    as_global_w<double>(partial), kps, blockIdx.x, blockIdx.y);
}

// Grouped symmetric Grams C_i = X_i^T X_i (FP32 X_i, K_i x M_i): group i owns the
// items [tile_start[i], tile_start[i+1]) of the flat grid, (part, upper tile) with
// the tile fastest; with more than one part of K each writes its share to the
// group's partial buffer and k_gram_reduce_grouped sums them in part order.
__global__ __launch_bounds__(256) void k_gram_grouped(const GramArgs* __restrict__ gs, const int* tile_start,
                                                      int count) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const GramArgs g = gs[lo];
  if (g.run_if && *g.run_if == 0) return;
  const int local = (int)blockIdx.x - tile_start[lo];
  if (g.splits > 1) {
    const int tiles = gram_group_tiles(g.M);
    gram_body<float, float>(as_global<float>(g.X), g.ldx, as_global<float>(g.X), g.ldx, g.K, g.M, g.M, 1,
                            as_global_w<double>(g.C), g.ldc, as_global_w<double>(g.partial), g.kps, local % tiles,
                            local / tiles);
  } else {
    gram_body<float, float>(as_global<float>(g.X), g.ldx, as_global<float>(g.X), g.ldx, g.K, g.M, g.M, 1,
                            as_global_w<double>(g.C), g.ldc, nullptr, g.K + GK, local, 0);
  }
}

// C_i (upper entries and their mirror) = sum of the parts in order; group i = blockIdx.y.
__global__ void k_gram_reduce_grouped(const GramArgs* __restrict__ gs) {
  const GramArgs g = gs[blockIdx.y];
  if (g.splits <= 1 || (g.run_if && *g.run_if == 0)) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, MM = g.M * g.M;
  if (idx >= MM) return;
  const int64_t i = idx / g.M, j = idx % g.M;
  if (i > j) return;
  double s = 0.0;
  for (int z = 0; z < g.splits; ++z) s += g.partial[(int64_t)z * MM + idx];
  g.C[i * g.ldc + j] = s;
  if (i != j) g.C[j * g.ldc + i] = s;
}

__host__ __device__ int gram_group_tiles(int64_t M) {
  const int64_t nt = (M + GT - 1) / GT;
  return (int)(nt * (nt + 1) / 2);
}

// Parts of K for one grouped Gram: about 1024 rows each, at most 8 (the long
// bases of a batch would otherwise run their tiles one 32-row step at a time
// while the short ones idle).
int gram_group_splits(int64_t K) {
  int64_t s = K / 1024;
  if (s > 8) s = 8;
  return s < 1 ? 1 : (int)s;
}

hipError_t launch_gram_grouped(const GramArgs* gs, const int* tile_start, int count, int total_tiles, int64_t max_mm,
                               bool any_split, hipStream_t st) {
  if (count == 0 || total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_grouped, dim3((unsigned)total_tiles), dim3(256), 0, st, gs, tile_start, count);
  if (any_split)
    hipLaunchKernelGGL(k_gram_reduce_grouped, dim3((unsigned)((max_mm + 255) / 256), (unsigned)count), dim3(256), 0,
                       st, gs);
  return hipGetLastError();
}

__global__ void k_gram_reduce(const double* __restrict__ partial, int splits, int64_t M, int64_t N, int sym,
                              double* __restrict__ C, int64_t ldc, const int* run_if) {
  if (run_if && *run_if == 0) return;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  int64_t i = idx / N, j = idx % N;
  if (sym && i > j) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += partial[(int64_t)z * M * N + idx];
  C[i * ldc + j] = s;
  if (sym && i != j) C[j * ldc + i] = s;
}

static int cus() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (n <= 0) n = 256;
  }
  return n;
}

// Split-K parts: about eight workgroups per CU in all (so that the uneven last share
// of a CU costs little), each part at least 256 rows of K, at most 128 parts.
static int gram_splits(int64_t K, int64_t M, int64_t N, int sym) {
  int64_t ntm = (M + GT - 1) / GT, ntn = (N + GT - 1) / GT;
  int64_t tiles = sym ? ntm * (ntm + 1) / 2 : ntm * ntn;
  int64_t s = (8 * (int64_t)cus() + tiles / 2) / tiles;
  if (s > K / 256) s = K / 256;
  if (s > 128) s = 128;
  return s < 1 ? 1 : (int)s;
}

size_t gram_partial_doubles(int64_t K, int64_t M, int64_t N) {
  int s = gram_splits(K, M, N, 0);
  int s2 = gram_splits(K, M, N, 1);
  if (s2 > s) s = s2;
  return s > 1 ? (size_t)s * M * N : 0;
}

hipError_t launch_gram(const void* X, int64_t ldx, int xdt, const void* Y, int64_t ldy, int ydt, int64_t K, int64_t M,
                       int64_t N, int sym, double* C, int64_t ldc, double* partial, const int* run_if,
                       hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  int splits = partial ? gram_splits(K, M, N, sym) : 1;
  int64_t kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
  if (kps == 0) kps = GK;
  splits = (int)((K + kps - 1) / kps);
  if (splits < 1) splits = 1;
  int64_t ntm = (M + GT - 1) / GT, ntn = (N + GT - 1) / GT;
  int64_t tiles = sym ? ntm * (ntm + 1) / 2 : ntm * ntn;
  double* part = splits > 1 ? partial : nullptr;
  dim3 grid((unsigned)tiles, (unsigned)splits);
  if (xdt == 0 && ydt == 0)
    hipLaunchKernelGGL((k_gram<float, float>), grid, dim3(256), 0, st, (const float*)X, ldx, (const float*)Y, ldy, K,
                       M, N, sym, C, ldc, part, kps, run_if);
  else if (xdt == 1 && ydt == 1)
    hipLaunchKernelGGL((k_gram<double, double>), grid, dim3(256), 0, st, (const double*)X, ldx, (const double*)Y,
                       ldy, K, M, N, sym, C, ldc, part, kps, run_if);
  else if (xdt == 0 && ydt == 1)
    hipLaunchKernelGGL((k_gram<float, double>), grid, dim3(256), 0, st, (const float*)X, ldx, (const double*)Y, ldy,
                       K, M, N, sym, C, ldc, part, kps, run_if);
  else
    hipLaunchKernelGGL((k_gram<double, float>), grid, dim3(256), 0, st, (const double*)X, ldx, (const float*)Y, ldy,
                       K, M, N, sym, C, ldc, part, kps, run_if);
  if (splits > 1) {
    int64_t tot = M * N;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, partial, splits, M, N,
                       sym, C, ldc, run_if);
  }
  return hipGetLastError();
}

// ============================== block-Jacobi eigensolver ==============================
// G (K x K, K = 2 p JB, padded with decoupled -1e300 diagonal) is driven to
// diagonal form by rounds of p independent 64 x 64 subproblems (pairs of 32-wide
// blocks, round-robin "circle" schedule).  Each subproblem takes one sweep of
// two-sided Jacobi rotations in LDS (Golub & Van Loan, sym.schur2): over all of
// its index pairs in the first round of an outer sweep, over the pairs across its
// two blocks in the others.  Its rotation V (64 x 64) is then applied to the
// rows/columns of G and to the eigenvector matrix Z: in the single-problem
// solver within the next round's launch (G into a second buffer, the next
// subproblems built from the previous G and V), in the batched solver by a
// separate in-place launch.  Converged when every off-diagonal entry is <= tol *
// sqrt(|G_ii G_jj| + floor^2).
int eig_block_width(int64_t N);


static EigWork eig_layout(void* work, int64_t N, int JB, bool dbuf = true) {
  EigWork w;
  int64_t K = ((N + 2 * JB - 1) / (2 * JB)) * (2 * JB);
  if (K < 2 * JB) K = 2 * JB;
  w.K = K;
  w.p = (int)(K / (2 * JB));
  const int JS = 2 * JB;
  char* p = (char*)work;
  w.Gp = (double*)p; p += K * K * 8;
  w.Gp2 = nullptr;
  if (dbuf) {
    w.Gp2 = (double*)p;
    p += K * K * 8;
  }
  w.Z = (double*)p; p += K * K * 8;
  w.V = (double*)p; p += (size_t)2 * w.p * JS * JS * 8;  // two slots: rounds alternate
  w.perm = (int*)p; p += ((K * 4 + 255) / 256) * 256;
  w.ident = (int*)p; p += ((2 * w.p * 4 + 255) / 256) * 256;
  w.maxoff = (unsigned long long*)p; p += 256;
  w.conv = (int*)p; p += 256;
  w.floor2 = (double*)p; p += 256;
  w.npart = (double*)p; p += 512;
  w.fabs_ = (double*)p; p += 256;  // last: eig_work_bytes ends the layout here
  return w;
}

// At most 24 outer sweeps (the graph holds them all; sweeps after convergence
// exit at once).  k = 2000 matrices with the spectrum i^-3 need 20.
int eig_max_sweeps() { return 24; }

// Bytes of the layout eig_layout lays out (taken from the layout itself, so the
// two cannot disagree), plus alignment slack.
size_t eig_work_bytes(int64_t N, bool batched) {
  const uintptr_t base = 4096;
  const EigWork w = eig_layout(reinterpret_cast<void*>(base), N, eig_block_width(N), !batched);
  return (size_t)(reinterpret_cast<uintptr_t>(w.fabs_) + 256 - base) + 4096;
}

RF_DEV int circle(int round, int i, int n) {  // position i of round in an n-player circle schedule
  return i == 0 ? 0 : 1 + (i - 1 + round) % (n - 1);
}

RF_DEV void eig_init_body(const double* __restrict__ G, int64_t ld, int64_t N, const EigWork& w, int64_t idx) {
  if (idx == 0) {
    *w.maxoff = 0ull;
    *w.conv = 0;
  }
  if (idx >= w.K * w.K) return;
  int64_t i = idx / w.K, j = idx % w.K;
  double v;
  if (i < N && j < N) v = G[i * ld + j];
  else v = (i == j) ? -1e300 : 0.0;
  w.Gp[idx] = v;
  w.Z[idx] = (i == j) ? 1.0 : 0.0;
}

RF_DEV void eig_floor_body(const double* __restrict__ G, int64_t ld, int64_t N, const EigWork& w) {
  // ||G||_F (single workgroup, fixed summation order) -> rotation floor and
  // absolute convergence floor
  __shared__ double red[1024];
  const int nt = blockDim.x, tc = threadIdx.x % 64, tr = threadIdx.x / 64, rstep = nt / 64;
  double s = 0.0;
  for (int64_t r = tr; r < N; r += rstep) {
    const double* row = G + r * ld;
    for (int64_t c = tc; c < N; c += 64) s = fma(row[c], row[c], s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = nt / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double fro = sqrt(red[0]);
    double f = 1e-15 * fro;
    *w.floor2 = f * f + 1e-300;
    *w.fabs_ = 16.0 * 2.220446049250313e-16 * fro + 1e-300;
  }
}

// Symmetric 2x2 Jacobi rotation (Golub & Van Loan, sym.schur2): J = [c s; -s c]
// zeroes apq in J^T [app apq; apq aqq] J for t = s / c = sign(d) 2 apq /
// (|d| + sqrt(d^2 + 4 apq^2)), d = aqq - app (the smaller root of
// t^2 + 2 tau t - 1 = 0, tau = d / (2 apq)).  The angle is taken in FP32 from d
// and 2 apq scaled by a power of two (no overflow or underflow); (c, s) is then
// normalised in FP64 (c^2 + s^2 = 1 to FP64 rounding, second-order correction of
// 1/sqrt(c0^2 + s0^2)).  Callers apply the rotation exactly, so the FP32 angle
// only leaves a residual of relative size ~1e-7 in the pair for later rotations.
// Pairs with |apq| <= 1e-17 sqrt(|app aqq| + floor2) are left alone.
RF_DEV void jacobi_rot(double app, double aqq, double apq, double floor2, double& c, double& s) {
  if (!(apq * apq > 1e-34 * (fabs(app * aqq) + floor2))) {
    c = 1.0; s = 0.0;
    return;
  }
  const double d = aqq - app, y2 = 2.0 * apq;
  int e;
  (void)frexp(fmax(fabs(d), fabs(y2)), &e);
  const float x = (float)ldexp(d, -e), y = (float)ldexp(y2, -e);  // max(|x|, |y|) in [1/2, 1)
  const float den = fabsf(x) + __builtin_amdgcn_sqrtf(x * x + y * y);
  const float tf = (x >= 0.f ? y : -y) * __builtin_amdgcn_rcpf(den);
  const float c0 = __builtin_amdgcn_rsqf(1.f + tf * tf), s0 = tf * c0;
  const double dc = c0, ds = s0;
  const double del = fma(dc, dc, ds * ds) - 1.0;
  const double f = fma(del, fma(del, 0.375, -0.5), 1.0);
  c = dc * f;
  s = ds * f;
}

template <int JB>
RF_DEV void eig_prologue(const EigWork& w, const double* __restrict__ Gs, int round, int x, int pslot, double* sm);

// One subproblem of the round.  Its 64 x 64 block of G comes straight from w.Gp
// (Gs == nullptr) or, with Gs set, is built from Gs, the G before the previous
// round's update, and that round's rotations in slot pslot (eig_prologue).
template <int JB>
RF_DEV void eig_solve_body(const EigWork& w, int round, bool full, int x, int slot,
                           const double* __restrict__ Gs = nullptr, int pslot = 0) {
  constexpr int JS = 2 * JB;
  // this round's rotations and "unchanged" flags go to slot `slot` (rounds
  // alternate between two, so the eigenvector update of one round can run
  // while the next round is solved)
  int* const ident = w.ident + slot * w.p;
  double* const Vout = w.V + (int64_t)slot * w.p * JS * JS;
  if (*w.conv) {
    if (threadIdx.x == 0) ident[x] = 1;
    return;
  }
  extern __shared__ double sm[];
  double(*M)[JS + 1] = reinterpret_cast<double(*)[JS + 1]>(sm);
  double(*V)[JS + 1] = reinterpret_cast<double(*)[JS + 1]>(sm + JS * (JS + 1));
  __shared__ double2 csn[JS / 2];
  __shared__ int done;
  const int np = 2 * w.p;
  const int P = circle(round, x, np), Q = circle(round, np - 1 - x, np);
  const double floor2 = *w.floor2;
  auto gidx = [&](int a) -> int64_t { return a < JB ? (int64_t)P * JB + a : (int64_t)Q * JB + (a - JB); };
  const double fabs_ = *w.fabs_;
  __shared__ int needed;
  if (threadIdx.x == 0) needed = 0;
  __syncthreads();
  if (Gs) {
    eig_prologue<JB>(w, Gs, round, x, pslot, sm);
    for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) V[e / JS][e % JS] = (e / JS == e % JS) ? 1.0 : 0.0;
  } else {
    for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
      int a = e / JS, b = e % JS;
      M[a][b] = as_global<double>(w.Gp)[gidx(a) * w.K + gidx(b)];
      V[a][b] = (a == b) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  // nothing to do when every off-diagonal entry of the pair already meets the
  // global convergence test and the diagonal is already in the sorted order
  // (square roots of the diagonal taken once)
  __shared__ double sq[JS];
  if (threadIdx.x < JS) sq[threadIdx.x] = sqrt(fabs(M[threadIdx.x][threadIdx.x]));
  __syncthreads();
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
    int a = e / JS, b = e % JS;
    if (a != b) {
      double d = sq[a] * sq[b];
      if (!(fabs(M[a][b]) <= fmax(w.tol * d, fabs_))) needed = 1;
    }
  }
  if (threadIdx.x < JS - 1) {
    const int a = threadIdx.x;
    // descending order within each 32-block and across the pair (lower-index block first)
    const int lo_first = (P < Q);
    if (a != JB - 1) {
      int b = a + 1;
      if (M[a][a] < M[b][b]) needed = 1;
    } else {
      double top = lo_first ? M[JB - 1][JB - 1] : M[JS - 1][JS - 1];
      double bot = lo_first ? M[JB][JB] : M[0][0];
      if (top < bot) needed = 1;
    }
  }
  __syncthreads();
  if (!needed) {
    if (threadIdx.x == 0) ident[x] = 1;
    return;
  }
  if (threadIdx.x == 0) ident[x] = 0;
  // A full round rotates every pair of the subproblem, the others only the pairs
  // across its two blocks.  With the first round of each outer sweep full, every
  // pair of indices is rotated at least once per outer sweep (a cyclic Jacobi
  // sweep in block order), in about half the sequential inner rounds of full
  // subproblem sweeps.
  if (full) {
    // a full cyclic sweep over every pair of the 2 JB indices (the pairs inside
    // each block included)
    // the pairs (lo, hi) of every inner round of the circle schedule, computed once:
    // the inner loop then reads them instead of repeating the modular arithmetic
    __shared__ unsigned char pair_lo[JS - 1][JS / 2], pair_hi[JS - 1][JS / 2];
    for (int e = threadIdx.x; e < (JS - 1) * (JS / 2); e += blockDim.x) {
      const int rr = e / (JS / 2), u = e % (JS / 2);
      int a = circle(rr, u, JS), b = circle(rr, JS - 1 - u, JS);
      if (a > b) { const int t = a; a = b; b = t; }
      pair_lo[rr][u] = (unsigned char)a;
      pair_hi[rr][u] = (unsigned char)b;
    }
    __syncthreads();
    if (threadIdx.x == 0) done = 1;
    __syncthreads();
    for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
      int a = e / JS, b = e % JS;
      if (a < b && fabs(M[a][b]) > 1e-15 * sqrt(fabs(M[a][a]) * fabs(M[b][b]) + floor2)) done = 0;
    }
    __syncthreads();
    // (the pass is skipped when the pair is already diagonal to FP64 rounding)
    for (int rr = 0; rr < (done ? 0 : JS - 1); ++rr) {
      // pair u of inner round rr: (lo, hi) of circle positions u and JS-1-u, from
      // the table; the rotations go through LDS as (c, s) pairs
      auto pair_of = [&](int u, int& a, int& b) {
        a = pair_lo[rr][u];
        b = pair_hi[rr][u];
      };
      if (threadIdx.x < JS / 2) {
        const int u = threadIdx.x;
        int a, b;
        pair_of(u, a, b);
        double c, s;
        jacobi_rot(M[a][a], M[b][b], M[a][b], floor2, c, s);  // FP32 angle, exact FP64 rotation
        csn[u] = double2{c, s};
      }
      __syncthreads();
      // thread t: 2x2 block (u, v) = (t / (JS/2), t % (JS/2)), M' = J_u^T M J_v, and
      // rows t / (JS/2) + 32 h of V <- V J_v (the same pair v)
      for (int e = threadIdx.x; e < (JS / 2) * (JS / 2); e += blockDim.x) {
        const int u = e / (JS / 2), v = e % (JS / 2);
        int a, b, cc, d;
        pair_of(u, a, b);
        pair_of(v, cc, d);
        const double2 ju = csn[u], jv = csn[v];
        const double cu = ju.x, su = ju.y, cv = jv.x, sv = jv.y;
        const double m00 = M[a][cc], m01 = M[a][d], m10 = M[b][cc], m11 = M[b][d];
        double v0[2], v1[2];  // rows u and u + JS/2 of V
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          v0[h] = V[u + (JS / 2) * h][cc];
          v1[h] = V[u + (JS / 2) * h][d];
        }
        const double t00 = cu * m00 - su * m10, t01 = cu * m01 - su * m11;
        const double t10 = su * m00 + cu * m10, t11 = su * m01 + cu * m11;
        M[a][cc] = cv * t00 - sv * t01; M[a][d] = sv * t00 + cv * t01;
        M[b][cc] = cv * t10 - sv * t11; M[b][d] = sv * t10 + cv * t11;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          V[u + (JS / 2) * h][cc] = cv * v0[h] - sv * v1[h];
          V[u + (JS / 2) * h][d] = sv * v0[h] + cv * v1[h];
        }
      }
      __syncthreads();
    }
  } else {
    // cross pairs only: inner round r pairs index u of the first block with index
    // (u + r) mod JB of the second, so the JB rounds meet each cross pair once.
    // Only the upper triangle of M is kept current (M[i][j], i <= j): thread t
    // < JB (JB + 1) / 2 owns the 2 x 2 block of pairs (u, v), u <= v, for the
    // whole sweep, which also stands for its mirror block (v, u).
    constexpr int NUP = JB * (JB + 1) / 2;
    int bu = -1, bv = -1;
    if ((int)threadIdx.x < NUP) upper_tile(threadIdx.x, JB, bu, bv);
    // V in registers: thread (vx, vu) holds rows vx and vx + JB of column vu (x0)
    // and of the second-block column of pair vu in the current inner round (x1).
    // That column moves to the neighbouring pair each round, so after its rotation
    // x1 is passed one lane down within the 32-lane half (vu -> vu - 1 mod JB).
    static_assert(JB == 32, "a pair's lanes are one 32-lane half of a wave");
    const int vu = threadIdx.x & (JB - 1), vx = threadIdx.x / JB;
    const int vsrc = (int)(threadIdx.x & 32) | ((vu + 1) & (JB - 1));  // lane that holds the next column
    double x0[2], x1[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = vx + JB * h;
      x0[h] = row == vu ? 1.0 : 0.0;
      x1[h] = row == JB + vu ? 1.0 : 0.0;
    }
    for (int r = 0; r < JB; ++r) {
      if (threadIdx.x < JB) {
        const int u = threadIdx.x, q = JB + ((u + r) & (JB - 1));
        double c, s;
        jacobi_rot(M[u][u], M[q][q], M[u][q], floor2, c, s);
        csn[u] = double2{c, s};
      }
      __syncthreads();
      if (bu >= 0) {
        const int su_ = (bu + r) & (JB - 1), sv_ = (bv + r) & (JB - 1);
        const int a = bu, b = JB + su_, cc = bv, d = JB + sv_;
        const double2 ju = csn[bu], jv = csn[bv];
        const double cu = ju.x, su = ju.y, cv = jv.x, sv = jv.y;
        if (bu == bv) {
          const double app = M[a][a], apq = M[a][b], aqq = M[b][b];
          const double t00 = cu * app - su * apq, t01 = cu * apq - su * aqq;
          const double t10 = su * app + cu * apq, t11 = su * apq + cu * aqq;
          M[a][a] = cv * t00 - sv * t01;
          M[a][b] = sv * t00 + cv * t01;
          M[b][b] = sv * t10 + cv * t11;
        } else {
          const int dlo = JB + (su_ < sv_ ? su_ : sv_), dhi = JB + (su_ < sv_ ? sv_ : su_);
          // rows (a, b), columns (cc, d); M[b][cc] is kept as M[cc][b] (cc < JB <= b)
          const double m00 = M[a][cc], m01 = M[a][d], m10 = M[cc][b], m11 = M[dlo][dhi];
          const double t00 = cu * m00 - su * m10, t01 = cu * m01 - su * m11;
          const double t10 = su * m00 + cu * m10, t11 = su * m01 + cu * m11;
          M[a][cc] = cv * t00 - sv * t01;
          M[a][d] = sv * t00 + cv * t01;
          M[cc][b] = cv * t10 - sv * t11;
          M[dlo][dhi] = sv * t10 + cv * t11;
        }
      }
      {
        const double2 j = csn[vu];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double y0 = j.x * x0[h] - j.y * x1[h];
          const double y1 = j.y * x0[h] + j.x * x1[h];
          x0[h] = y0;
          x1[h] = __shfl(y1, vsrc, 64);
        }
      }
      __syncthreads();
    }
    // after JB rounds x1 is back at column JB + vu
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = vx + JB * h;
      V[row][vu] = x0[h];
      V[row][JB + vu] = x1[h];
    }
    __syncthreads();
  }
  // Order the subproblem's eigenpairs: the larger half goes to the block with the
  // lower index, so eigenvalues settle in descending order along the diagonal
  // (speeds up convergence on clustered spectra; the padding sinks to the end).
  // (16 threads per entry, each counting over JS/16 others, summed across lanes)
  __shared__ int rnk[JS];
  static_assert(JS * 16 <= 1024, "16 threads per diagonal entry");
  if (threadIdx.x < JS * 16) {
    const int a = threadIdx.x >> 4, c = threadIdx.x & 15;
    const double d = M[a][a];
    int r = 0;
#pragma unroll
    for (int i = 0; i < JS / 16; ++i) {
      const int b = c * (JS / 16) + i;
      const double e = M[b][b];
      r += (e > d || (e == d && b < a)) ? 1 : 0;
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) r += __shfl_xor(r, o, 16);
    if (c == 0) rnk[a] = (P < Q) ? r : (r + JB) % JS;
  }
  __syncthreads();
  double* out = Vout + (int64_t)x * JS * JS;
  const gptr<double> outg = as_global_w<double>(out);
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) outg[(e / JS) * JS + rnk[e % JS]] = V[e / JS][e % JS];
}

// 64 x 64 FP64 products on v_mfma_f64_16x16x4f64, 4 waves, each a 32 x 32
// quadrant of 2 x 2 blocks of 16 x 16.  Operand A (16 x 4 per MFMA, lane l holds
// row l%16, k = l/16) and B (4 x 16, lane l holds column l%16, k = l/16).  The
// result of block (i, j), register r of lane l, is row wm*32 + i*16 + l/16 + 4r,
// column wn*32 + j*16 + l%16.
struct Mfma64 {
  int lane, wm, wn;
  RF_DEV Mfma64() : lane(threadIdx.x & 63), wm((threadIdx.x >> 6) >> 1), wn((threadIdx.x >> 6) & 1) {}
  RF_DEV explicit Mfma64(int tid) : lane(tid & 63), wm((tid >> 6) >> 1), wn((tid >> 6) & 1) {}  // 256-thread group
  RF_DEV int arow(int i) const { return wm * 32 + i * 16 + (lane & 15); }
  RF_DEV int bcol(int j) const { return wn * 32 + j * 16 + (lane & 15); }
  RF_DEV int krow(int kk) const { return 4 * kk + (lane >> 4); }
  // register operands of a row-major 64 x 64 matrix in global memory:
  // B operand (X as B: X[k][col]) or A operand of X^T (X^T[row][k] = X[k][row])
  RF_DEV void load_b(gptr<const double> X, double (&r)[16][2]) const {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int j = 0; j < 2; ++j) r[kk][j] = X[krow(kk) * 64 + bcol(j)];
  }
  RF_DEV void load_at(gptr<const double> X, double (&r)[16][2]) const {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int i = 0; i < 2; ++i) r[kk][i] = X[krow(kk) * 64 + arow(i)];
  }
  // acc = S B with S in LDS (A operand) and B in registers
  RF_DEV void mul_lds_reg(const double (*S)[65], const double (&bv)[16][2], f64x4 (&acc)[2][2]) const {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double af[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = S[arow(i)][krow(kk)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bv[kk][j], acc[i][j], 0, 0, 0);
    }
  }
  // acc = A S with A in registers (A operand) and S in LDS (B operand)
  RF_DEV void mul_reg_lds(const double (&av)[16][2], const double (*S)[65], f64x4 (&acc)[2][2]) const {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double bf[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = S[krow(kk)][bcol(j)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk][i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  RF_DEV void store(const f64x4 (&acc)[2][2], double (*S)[65]) const {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) S[wm * 32 + i * 16 + (lane >> 4) + 4 * r][bcol(j)] = acc[i][j][r];
  }
};

// The same 64 x 64 FP64 products with 16 waves (1024 threads): wave (bi, bj) owns
// the 16 x 16 block (bi, bj), so each wave runs a quarter of the MFMA chain of the
// 4-wave form.  Operand layouts as in Mfma64.
struct Mfma16 {
  int lane, bi, bj;
  RF_DEV Mfma16() : lane(threadIdx.x & 63), bi((threadIdx.x >> 6) >> 2), bj((threadIdx.x >> 6) & 3) {}
  RF_DEV int kr(int kk) const { return 4 * kk + (lane >> 4); }
  // B operand X[k][col] of column block bj, and A operand of X^T (X^T[row][k] = X[k][row]) of row block bi
  RF_DEV void load_b(const double* __restrict__ X, double (&r)[16]) const {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) r[kk] = X[kr(kk) * 64 + bj * 16 + (lane & 15)];
  }
  RF_DEV void load_at(const double* __restrict__ X, double (&r)[16]) const {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) r[kk] = X[kr(kk) * 64 + bi * 16 + (lane & 15)];
  }
  // S B with S in LDS (A operand), and A S with S in LDS (B operand)
  RF_DEV f64x4 mul_lds_reg(const double (*S)[65], const double (&bv)[16]) const {
    f64x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(S[bi * 16 + (lane & 15)][kr(kk)], bv[kk], acc, 0, 0, 0);
    return acc;
  }
  RF_DEV f64x4 mul_reg_lds(const double (&av)[16], const double (*S)[65]) const {
    f64x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], S[kr(kk)][bj * 16 + (lane & 15)], acc, 0, 0, 0);
    return acc;
  }
  RF_DEV void store(const f64x4& acc, double (*S)[65]) const {
#pragma unroll
    for (int r = 0; r < 4; ++r) S[bi * 16 + (lane >> 4) + 4 * r][bj * 16 + (lane & 15)] = acc[r];
  }
  // the same two products with the V operand read from LDS (same values, same
  // instruction order, so the same results bit for bit)
  RF_DEV f64x4 mul_lds_lds(const double (*S)[65], const double (*Vy)[65]) const {
    f64x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(S[bi * 16 + (lane & 15)][kr(kk)], Vy[kr(kk)][bj * 16 + (lane & 15)],
                                                 acc, 0, 0, 0);
    return acc;
  }
  RF_DEV f64x4 mul_ldst_lds(const double (*Vx)[65], const double (*S)[65]) const {
    f64x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Vx[kr(kk)][bi * 16 + (lane & 15)], S[kr(kk)][bj * 16 + (lane & 15)],
                                                 acc, 0, 0, 0);
    return acc;
  }
};

// Subproblem of pair x in round `round` (> 0 within an outer sweep), built from
// Gs, the G before the previous round's update, and that round's rotations (slot
// pslot).  Block P of the pair sat in half hP of the previous round's pair a,
// block Q in half hQ of pair b (a != b: two blocks meet once per sweep), so
//   M = [ X_a^T Gs[I_a, I_a] X_a   X_a^T Gs[I_a, I_b] X_b ]
//       [        (mirror)          X_b^T Gs[I_b, I_b] X_b ]
// with X_a = V_a[:, JB hP : JB hP + JB], X_b likewise (no product where the
// previous solve left the pair unchanged).  Only the three needed quadrants are
// formed, each entry exactly as the tile update forms it (tile orientation,
// operands, MFMA order, symmetrisation of diagonal tiles), so M holds, bit for
// bit, the entries that update writes to the other buffer.  Tile t = 0: (a, a),
// 1: (b, b), 2: (min(a,b), max(a,b)); the update takes W = T X_y (64 x 32) and
// C = X_x^T W (32 x 32).  The tiles are read coalesced and staged in LDS; tiles
// 0 and 1 are formed together (16 waves, one 16 x 16 block each), then tile 2.
// LDS: M at sm, tiles at sm + JS (JS+1) (where V goes afterwards) and sm +
// 2 JS (JS+1) (each W over its tile), then X_a and X_b (JS x JB+1 each).
template <int JB>
RF_DEV void eig_prologue(const EigWork& w, const double* __restrict__ Gs, int round, int x, int pslot, double* sm) {
  constexpr int JS = 2 * JB, LD = JS + 1, LH = JB + 1;
  static_assert(JS == 64, "the MFMA tile product is written for 64 x 64 subproblems");
  double(*M)[LD] = reinterpret_cast<double(*)[LD]>(sm);
  // slot s of the tiles (and of the W over each) computed from sm, not picked
  // from an array of pointers: a pointer array indexed at run time loses the LDS
  // address space and its accesses compile to flat ones
  auto TT = [&](int slot) { return reinterpret_cast<double(*)[LD]>(sm + (1 + slot) * JS * LD); };
  auto WW = [&](int slot) { return reinterpret_cast<double(*)[LH]>(sm + (1 + slot) * JS * LD); };
  double(*XA)[LH] = reinterpret_cast<double(*)[LH]>(sm + 3 * JS * LD);
  double(*XB)[LH] = reinterpret_cast<double(*)[LH]>(sm + 3 * JS * LD + JS * LH);
  const int p = w.p, np = 2 * p, rp = round - 1;
  auto posof = [&](int B) { return B == 0 ? 0 : 1 + ((B - 1 - rp) % (np - 1) + (np - 1)) % (np - 1); };
  const int iP = posof(circle(round, x, np)), iQ = posof(circle(round, np - 1 - x, np));
  const int a = iP < p ? iP : np - 1 - iP, hP = iP < p ? 0 : 1;
  const int b = iQ < p ? iQ : np - 1 - iQ, hQ = iQ < p ? 0 : 1;
  const int* const ident = w.ident + pslot * p;
  const double* const Vp = w.V + (int64_t)pslot * p * JS * JS;
  const bool ida = ident[a] != 0, idb = ident[b] != 0;
  const int Pa = circle(rp, a, np), Qa = circle(rp, np - 1 - a, np);
  const int Pb = circle(rp, b, np), Qb = circle(rp, np - 1 - b, np);
  auto ia = [&](int c) -> int64_t { return c < JB ? (int64_t)Pa * JB + c : (int64_t)Qa * JB + (c - JB); };
  auto ib = [&](int c) -> int64_t { return c < JB ? (int64_t)Pb * JB + c : (int64_t)Qb * JB + (c - JB); };
  const bool alo = a < b;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // every global load first: the three tiles (two double2 per thread each) and
  // the needed halves of V_a and V_b (two doubles per thread each)
  double2 tl[3][2];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = (int)threadIdx.x + h * 1024, r = e >> 5, c = (e & 31) * 2;
      const bool ra = t == 0 || (t == 2 && alo), ca = t == 0 || (t == 2 && !alo);
      tl[t][h] = *reinterpret_cast<const double2*>(Gs + (ra ? ia(r) : ib(r)) * w.K + (ca ? ia(c) : ib(c)));
    }
  double xa[2], xb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = (int)threadIdx.x + h * 1024, r = e >> 5, c = e & 31;
    xa[h] = Vp[(int64_t)a * JS * JS + r * JS + JB * hP + c];
    xb[h] = Vp[(int64_t)b * JS * JS + r * JS + JB * hQ + c];
  }
  auto stage = [&](int t, int slot) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = (int)threadIdx.x + h * 1024, r = e >> 5, c = (e & 31) * 2;
      TT(slot)[r][c] = tl[t][h].x;
      TT(slot)[r][c + 1] = tl[t][h].y;
    }
  };
  stage(0, 0);
  stage(1, 1);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = (int)threadIdx.x + h * 1024, r = e >> 5, c = e & 31;
    if (!ida) XA[r][c] = xa[h];
    if (!idb) XB[r][c] = xb[h];
  }
  __syncthreads();
  // W block (bi, j) of the tile in slot s: T X_y, or T's half hy itself
  auto wblock = [&](int s, int bi, int j, const double (*XY)[LH], bool idy, int hy) {
    f64x4 acc = {0, 0, 0, 0};
    if (!idy) {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(TT(s)[bi * 16 + (lane & 15)][4 * kk + (lane >> 4)],
                                                   XY[4 * kk + (lane >> 4)][16 * j + (lane & 15)], acc, 0, 0, 0);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = TT(s)[bi * 16 + (lane >> 4) + 4 * r][JB * hy + 16 * j + (lane & 15)];
    }
    return acc;
  };
  // C block (ci, cj) of the tile whose W is in slot s: X_x^T W, or W's half hx
  auto cblock = [&](int s, int ci, int cj, const double (*XX)[LH], bool idx, int hx) {
    f64x4 c = {0, 0, 0, 0};
    if (!idx) {
#pragma unroll
      for (int kk = 0; kk < 16; ++kk)
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(XX[4 * kk + (lane >> 4)][16 * ci + (lane & 15)],
                                                 WW(s)[4 * kk + (lane >> 4)][16 * cj + (lane & 15)], c, 0, 0, 0);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) c[r] = WW(s)[JB * hx + 16 * ci + (lane >> 4) + 4 * r][16 * cj + (lane & 15)];
    }
    return c;
  };
  // tiles 0 and 1: W (wave wv: tile wv >> 3, block ((wv >> 1) & 3, wv & 1))
  {
    const int t = wv >> 3, bi = (wv >> 1) & 3, j = wv & 1;
    const f64x4 acc = wblock(t, bi, j, t ? XB : XA, t ? idb : ida, t ? hQ : hP);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) WW(t)[bi * 16 + (lane >> 4) + 4 * r][16 * j + (lane & 15)] = acc[r];
  }
  __syncthreads();
  // tiles 0 and 1: C (waves 0-7: tile wv >> 2, block ((wv >> 1) & 1, wv & 1)) into the diagonal quadrants of M
  if (wv < 8) {
    const int t = wv >> 2, ci = (wv >> 1) & 1, cj = wv & 1, o = JB * t;
    const f64x4 c = cblock(t, ci, cj, t ? XB : XA, t ? idb : ida, t ? hQ : hP);
#pragma unroll
    for (int r = 0; r < 4; ++r) M[o + 16 * ci + (lane >> 4) + 4 * r][o + 16 * cj + (lane & 15)] = c[r];
  }
  __syncthreads();
  // tile 2 into slot 0; the diagonal quadrants are written from their upper half
  stage(2, 0);
  {
    const int i = (int)threadIdx.x >> 5, j = (int)threadIdx.x & 31;  // one entry per thread
    if (i > j) {
      M[i][j] = M[j][i];
      M[JB + i][JB + j] = M[JB + j][JB + i];
    }
  }
  __syncthreads();
  // tile 2 (x side a if alo, else b): W (waves 0-7), then C (waves 0-3) into the off-diagonal block
  {
    const double(*XX)[LH] = alo ? XA : XB;
    const double(*XY)[LH] = alo ? XB : XA;
    const bool idx = alo ? ida : idb, idy = alo ? idb : ida;
    const int hx = alo ? hP : hQ, hy = alo ? hQ : hP;
    f64x4 acc = {0, 0, 0, 0};
    const int bi = (wv >> 1) & 3, j = wv & 1;
    if (wv < 8) acc = wblock(0, bi, j, XY, idy, hy);
    __syncthreads();
    if (wv < 8)
#pragma unroll
      for (int r = 0; r < 4; ++r) WW(0)[bi * 16 + (lane >> 4) + 4 * r][16 * j + (lane & 15)] = acc[r];
    __syncthreads();
    if (wv < 4) {
      const int ci = (wv >> 1) & 1, cj = wv & 1;
      const f64x4 c = cblock(0, ci, cj, XX, idx, hx);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * ci + (lane >> 4) + 4 * r, jj = 16 * cj + (lane & 15);  // C[i][jj]
        if (alo) {
          M[i][JB + jj] = c[r];
          M[JB + jj][i] = c[r];
        } else {
          M[jj][JB + i] = c[r];
          M[JB + i][jj] = c[r];
        }
      }
    }
  }
  __syncthreads();
}

// G tile id < p(p+1)/2 of the round: (x, y), x <= y, G[I_x, I_y] <- V_x^T G[I_x, I_y]
// V_y, written to both (x, y) and (y, x) so G stays exactly symmetric (a diagonal
// tile from its upper half).  1024 threads; the tile is staged in LDS, the V
// operands go from global memory straight to registers.
template <int JB>
RF_DEV void eig_gtile_body(const EigWork& w, int round, int slot, int id, const double* __restrict__ Gs, double* Gd) {
  constexpr int JS = 2 * JB;
  static_assert(JS == 64, "the MFMA tile product is written for 64 x 64 subproblems");
  if (*w.conv) return;
  const int* const ident = w.ident + slot * w.p;
  const double* const Vr = w.V + (int64_t)slot * w.p * JS * JS;
  extern __shared__ double sm[];
  double(*T)[JS + 1] = reinterpret_cast<double(*)[JS + 1]>(sm);
  const int np = 2 * w.p;
  int x, y;
  upper_tile(id, w.p, x, y);
  const int idx_ = ident[x], idy_ = ident[y];
  if (idx_ && idy_ && Gs == Gd) return;  // unchanged in place; into the other buffer it is copied
  const int Px = circle(round, x, np), Qx = circle(round, np - 1 - x, np);
  const int Py = circle(round, y, np), Qy = circle(round, np - 1 - y, np);
  auto ix = [&](int a) -> int64_t { return a < JB ? (int64_t)Px * JB + a : (int64_t)Qx * JB + (a - JB); };
  auto iy = [&](int a) -> int64_t { return a < JB ? (int64_t)Py * JB + a : (int64_t)Qy * JB + (a - JB); };
  const Mfma16 mm;
  double opa[16], opb[16];
  if (!idy_) mm.load_b(as_global<double>(Vr) + (int64_t)y * JS * JS, opb);
  if (!idx_) mm.load_at(as_global<double>(Vr) + (int64_t)x * JS * JS, opa);
  for (int e = threadIdx.x; e < JS * JS / 2; e += blockDim.x) {
    const int a = e >> 5, b = (e & 31) * 2;
    const double2 g = *reinterpret_cast<const double2*>(Gs + ix(a) * w.K + iy(b));
    T[a][b] = g.x;
    T[a][b + 1] = g.y;
  }
  __syncthreads();
  if (!idy_) {  // T <- T V_y
    const f64x4 acc = mm.mul_lds_reg(T, opb);
    __syncthreads();
    mm.store(acc, T);
    __syncthreads();
  }
  if (!idx_) {  // T <- V_x^T T
    const f64x4 acc = mm.mul_reg_lds(opa, T);
    __syncthreads();
    mm.store(acc, T);
    __syncthreads();
  }
  for (int e = threadIdx.x; e < JS * JS / 2; e += blockDim.x) {
    const int a = e >> 5, b = (e & 31) * 2;
    double2 g;
    g.x = (x == y && a > b) ? T[b][a] : T[a][b];
    g.y = (x == y && a > b + 1) ? T[b + 1][a] : T[a][b + 1];
    *reinterpret_cast<double2*>(Gd + ix(a) * w.K + iy(b)) = g;
  }
  if (x != y) {
    for (int e = threadIdx.x; e < JS * JS / 2; e += blockDim.x) {
      const int b = e >> 5, a = (e & 31) * 2;
      *reinterpret_cast<double2*>(Gd + iy(b) * w.K + ix(a)) = double2{T[a][b], T[a + 1][b]};
    }
  }
}

// Z strip zid = rb p + x: Z[rows of strip rb, I_x] <- Z[..] V_x for the round and
// rotation slot given, by a group of 256 threads (tid) staging the strip in T.
// Every thread of the workgroup passes the same barriers whether its group is
// active or not.  No test of the convergence flag: this update may run after
// the flag was set; a round whose solve saw it marked every subproblem unchanged.
template <int JB>
RF_DEV void eig_zstrip_body(const EigWork& w, int round, int slot, int zid, int tid, double (*T)[2 * JB + 1],
                            bool active) {
  constexpr int JS = 2 * JB;
  const int np = 2 * w.p;
  const int x = zid % w.p, rb = zid / w.p;
  active = active && !w.ident[slot * w.p + x];
  const Mfma64 mm(tid);
  f64x4 acc[2][2];
  double opb[16][2];
  const int Px = circle(round, x, np), Qx = circle(round, np - 1 - x, np);
  auto ix = [&](int a) -> int64_t { return a < JB ? (int64_t)Px * JB + a : (int64_t)Qx * JB + (a - JB); };
  const int64_t r0 = (int64_t)rb * JS;  // K is a multiple of JS: the strip is whole
  if (active) {
    mm.load_b(as_global<double>(w.V) + ((int64_t)slot * w.p + x) * JS * JS, opb);
    for (int e = tid; e < JS * JS / 2; e += 256) {
      const int a = e >> 5, b = (e & 31) * 2;
      const double2 z = *reinterpret_cast<gptr<const double2>>(as_global<double>(w.Z) + (r0 + a) * w.K + ix(b));
      T[a][b] = z.x;
      T[a][b + 1] = z.y;
    }
  }
  __syncthreads();
  if (active) mm.mul_lds_reg(T, opb, acc);
  __syncthreads();
  if (active) mm.store(acc, T);
  __syncthreads();
  if (active)
    for (int e = tid; e < JS * JS / 2; e += 256) {
      const int a = e >> 5, b = (e & 31) * 2;
      *reinterpret_cast<gptr<double2>>(as_global_w<double>(w.Z) + (r0 + a) * w.K + ix(b)) = double2{T[a][b], T[a][b + 1]};
    }
}

// Work item id < p(p+1)/2: tile (x, y), x <= y, G[I_x, I_y] <- V_x^T G[I_x, I_y] V_y,
// written to both (x, y) and (y, x) so G stays exactly symmetric.  Other ids:
// Z[rows, I_x] <- Z[rows, I_x] V_x for one 64-row strip.  256 threads; the tile
// is staged in LDS, the V operands go from global memory straight to registers.
template <int JB>
RF_DEV void eig_apply_body(const EigWork& w, int round, int id, int slot) {
  constexpr int JS = 2 * JB;
  static_assert(JS == 64, "the MFMA tile product is written for 64 x 64 subproblems");
  const int* const ident = w.ident + slot * w.p;
  const double* const Vr = w.V + (int64_t)slot * w.p * JS * JS;
  extern __shared__ double sm[];
  double(*T)[JS + 1] = reinterpret_cast<double(*)[JS + 1]>(sm);
  const int np = 2 * w.p;
  const int nsym = w.p * (w.p + 1) / 2;
  const Mfma64 mm;
  f64x4 acc[2][2];
  double opa[16][2], opb[16][2];
  if (id < nsym) {
    if (*w.conv) return;
    int x, y;
    upper_tile(id, w.p, x, y);
    const int idx_ = ident[x], idy_ = ident[y];
    if (idx_ && idy_) return;
    const int Px = circle(round, x, np), Qx = circle(round, np - 1 - x, np);
    const int Py = circle(round, y, np), Qy = circle(round, np - 1 - y, np);
    auto ix = [&](int a) -> int64_t { return a < JB ? (int64_t)Px * JB + a : (int64_t)Qx * JB + (a - JB); };
    auto iy = [&](int a) -> int64_t { return a < JB ? (int64_t)Py * JB + a : (int64_t)Qy * JB + (a - JB); };
    if (!idy_) mm.load_b(as_global<double>(Vr) + (int64_t)y * JS * JS, opb);
    if (!idx_) mm.load_at(as_global<double>(Vr) + (int64_t)x * JS * JS, opa);
    for (int e = threadIdx.x; e < JS * JS / 2; e += blockDim.x) {
      const int a = e >> 5, b = (e & 31) * 2;
      const double2 g = *reinterpret_cast<gptr<const double2>>(as_global<double>(w.Gp) + ix(a) * w.K + iy(b));
      T[a][b] = g.x;
      T[a][b + 1] = g.y;
    }
    __syncthreads();
    if (!idy_) {  // T <- T V_y
      mm.mul_lds_reg(T, opb, acc);
      __syncthreads();
      mm.store(acc, T);
      __syncthreads();
    }
    if (!idx_) {  // T <- V_x^T T
      mm.mul_reg_lds(opa, T, acc);
      __syncthreads();
      mm.store(acc, T);
      __syncthreads();
    }
    for (int e = threadIdx.x; e < JS * JS / 2; e += blockDim.x) {
      const int a = e >> 5, b = (e & 31) * 2;
      double2 g;
      // a diagonal tile is symmetrised from its upper half
      g.x = (x == y && a > b) ? T[b][a] : T[a][b];
      g.y = (x == y && a > b + 1) ? T[b + 1][a] : T[a][b + 1];
      *reinterpret_cast<gptr<double2>>(as_global_w<double>(w.Gp) + ix(a) * w.K + iy(b)) = g;
    }
    if (x != y) {
      for (int e = threadIdx.x; e < JS * JS / 2; e += blockDim.x) {
        const int b = e >> 5, a = (e & 31) * 2;
        *reinterpret_cast<gptr<double2>>(as_global_w<double>(w.Gp) + iy(b) * w.K + ix(a)) = double2{T[a][b], T[a + 1][b]};
      }
    }
  } else {
    eig_zstrip_body<JB>(w, round, slot, id - nsym, threadIdx.x, T, true);
  }
}

// Work items of one apply launch: upper G tiles, then Z strips.
__host__ __device__ inline int eig_apply_items(int p, int64_t K, int JS) { return p * (p + 1) / 2 + (int)(K / JS) * p; }

// Converged when every |g_ij| <= max(tol sqrt|g_ii g_jj|, 16 eps ||G||_F), i.e. the
// largest r_ij = |g_ij| / max(...) is <= 1.  The check keeps the maximum of r_ij^2
// (no square roots per entry; the bits of non-negative doubles order like the
// values) and the decision takes one square root.
constexpr int kCheckPerThread = 8;  // entries per thread in the convergence check (256-thread blocks)

RF_DEV void eig_check_body(const EigWork& w, int block) {
  if (*w.conv) return;
  __shared__ double red[4];
  double r2 = 0.0;
  const int K = (int)w.K;  // K <= 4096
  const double fl = *w.fabs_, tol2 = w.tol * w.tol;
#pragma unroll
  for (int e = 0; e < kCheckPerThread; ++e) {
    const int64_t idx = ((int64_t)block * kCheckPerThread + e) * 256 + threadIdx.x;
    if (idx < (int64_t)K * K) {
      const int i = (int)(idx / K), j = (int)(idx - (int64_t)i * K);
      if (i != j) {
        const double g = w.Gp[idx];
        const double den = fmax(tol2 * fabs(w.Gp[(int64_t)i * K + i] * w.Gp[(int64_t)j * K + j]), fl * fl);
        double q = (g * g) / den;
        if (!(q == q)) q = 4.0;  // NaN: keep iterating (and never claim convergence)
        r2 = fmax(r2, q);
      }
    }
  }
  r2 = wave_max(r2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (m > 0.0) atomicMax(w.maxoff, (unsigned long long)__double_as_longlong(m));
  }
}

__host__ __device__ inline unsigned eig_check_blocks(int64_t K) {
  return (unsigned)((K * K + 256 * kCheckPerThread - 1) / (256 * kCheckPerThread));
}

RF_DEV void eig_decide_body(const EigWork& w, double tol, double* trace, int sw) {
  if (*w.conv) {
    if (trace) trace[sw] = 0.0;
    return;
  }
  const double m = sqrt(__longlong_as_double((long long)*w.maxoff));
  if (trace) trace[sw] = m;
  if (m <= tol) *w.conv = 1;
  *w.maxoff = 0ull;
}

// Sort diag(Gp) descending (bitonic, one workgroup, K <= 4096), gather outputs.
RF_DEV void eig_sort_body(const EigWork& w, int64_t N, double* lam) {
  __shared__ double key[4096];
  __shared__ int idx[4096];
  int Kp = 1;
  while (Kp < w.K) Kp <<= 1;
  for (int i = threadIdx.x; i < Kp; i += blockDim.x) {
    key[i] = (i < w.K) ? w.Gp[(int64_t)i * w.K + i] : -INFINITY;
    idx[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= Kp; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < Kp; i += blockDim.x) {
        int j = i ^ stride;
        if (j > i) {
          bool desc = ((i & size) == 0);
          double a = key[i], b = key[j];
          bool sw = desc ? (a < b || (a == b && idx[i] > idx[j])) : (a > b || (a == b && idx[i] < idx[j]));
          if (sw) {
            key[i] = b; key[j] = a;
            int t = idx[i]; idx[i] = idx[j]; idx[j] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    lam[i] = key[i];
    w.perm[i] = idx[i];
  }
}

RF_DEV void eig_gather_body(const EigWork& w, int64_t N, double* V, int64_t ldv, int64_t e) {
  if (e >= N * N) return;
  int64_t r = e / N, c = e % N;
  V[r * ldv + c] = w.Z[r * w.K + w.perm[c]];
}

__global__ void k_eig_init(const double* __restrict__ G, int64_t ld, int64_t N, EigWork w) {
  eig_init_body(G, ld, N, w, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}
// ||G||_F for the single-problem solver in kNormParts row ranges at once (one
// workgroup reading all of G took 1.1 ms at K = 2048), summed in part order.
constexpr int kNormParts = 64;
__global__ __launch_bounds__(1024) void k_eig_norm_part(const double* __restrict__ G, int64_t ld, int64_t N,
                                                         double* __restrict__ part) {
  __shared__ double red[1024];
  const int64_t rows = (N + kNormParts - 1) / kNormParts;
  const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min(N, r0 + rows);
  const int tc = threadIdx.x % 64, tr = threadIdx.x / 64;
  double s = 0.0;
  for (int64_t r = r0 + tr; r < r1; r += 16) {
    const double* row = G + r * ld;
    for (int64_t c = tc; c < N; c += 64) s = fma(row[c], row[c], s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
// the rotation and convergence floors from the parts (as eig_floor_body sets them)
__global__ void k_eig_floor_fin(EigWork w) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < kNormParts; ++i) s += w.npart[i];
  const double fro = sqrt(s);
  const double f = 1e-15 * fro;
  *w.floor2 = f * f + 1e-300;
  *w.fabs_ = 16.0 * 2.220446049250313e-16 * fro + 1e-300;
}
// work items id0 + blockIdx.x (G tiles first, then Z strips)
template <int JB>
__global__ __launch_bounds__(256) void k_eig_apply(EigWork w, int round, int slot, int id0) {
  eig_apply_body<JB>(w, round, id0 + (int)blockIdx.x, slot);
}
template <int JB>
__global__ __launch_bounds__(1024) void k_eig_gtile(EigWork w, int round, int slot) {
  eig_gtile_body<JB>(w, round, slot, (int)blockIdx.x, w.Gp, w.Gp);  // in place
}

// Dynamic LDS of k_eig_round: the subproblem while it is built (M and two G
// tiles, JS x JS+1 doubles each; two halves of rotation blocks, JS x JB+1 each),
// which also covers four Z strips (JS x JS+1 doubles each).
constexpr size_t eig_round_lds(int JB) {
  return (size_t)(3 * (2 * JB) * (2 * JB + 1) + 2 * (2 * JB) * (JB + 1)) * sizeof(double);
}

// One launch per round r of an outer sweep:
//   workgroups [0, p)           the subproblems of round r; for r > 0 each builds
//                               its block from the G before round r-1's update
//                               (buffer gsrc) and round r-1's rotations;
//   next nzw workgroups         Z <- Z V of round r-1 (four 64-row strips each,
//                               one per 256-thread group);
//   last ntile workgroups       G tiles of round r-1, buffer gsrc -> gdst.
// Everything but the subproblems uses only round r-1's rotations, so the launch
// fills the CUs the p subproblems leave idle and no G update waits between two
// solves.  Rotations alternate between two slots (slot: this round, zslot: the
// previous one).
template <int JB>
__global__ __launch_bounds__(1024) void k_eig_round(EigWork w, int round, int full, int slot, int zround, int zslot,
                                                    int nzw, int gsrc, int gdst) {
  constexpr int JS = 2 * JB;
  const int bid = (int)blockIdx.x;
  const double* Gs = gsrc ? w.Gp2 : w.Gp;
  if (bid < w.p) {
    eig_solve_body<JB>(w, round, full != 0, bid, slot, gsrc >= 0 && round > 0 ? Gs : nullptr, zslot);
    return;
  }
  if (bid < w.p + nzw) {
    extern __shared__ double sm[];
    const int grp = (int)threadIdx.x >> 8;
    double(*T)[JS + 1] = reinterpret_cast<double(*)[JS + 1]>(sm + grp * JS * (JS + 1));
    const int zid = (bid - w.p) * 4 + grp;
    eig_zstrip_body<JB>(w, zround, zslot, zid, (int)threadIdx.x & 255, T, zid < (int)(w.K / JS) * w.p);
    return;
  }
  eig_gtile_body<JB>(w, zround, zslot, bid - w.p - nzw, Gs, gdst ? w.Gp2 : w.Gp);
}

__global__ __launch_bounds__(256) void k_eig_check(EigWork w) { eig_check_body(w, blockIdx.x); }
__global__ void k_eig_decide(EigWork w, double tol, double* trace, int sw) { eig_decide_body(w, tol, trace, sw); }
__global__ __launch_bounds__(1024) void k_eig_sort(EigWork w, int64_t N, double* lam) { eig_sort_body(w, N, lam); }
__global__ void k_eig_gather(EigWork w, int64_t N, double* V, int64_t ldv) {
  eig_gather_body(w, N, V, ldv, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---- batched: one problem per blockIdx.y ------------------------------------------
__global__ void k_eigb_init(const EigBatch* __restrict__ bs) {
  const EigBatch b = bs[blockIdx.y];
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < b.w.K * b.w.K;
       idx += (int64_t)gridDim.x * blockDim.x)
    eig_init_body(b.G, b.ld, b.N, b.w, idx);
}
__global__ __launch_bounds__(1024) void k_eigb_floor(const EigBatch* __restrict__ bs) {
  const EigBatch b = bs[blockIdx.y];
  eig_floor_body(b.G, b.ld, b.N, b.w);
}
template <int JB>
__global__ __launch_bounds__(1024) void k_eigb_solve(const EigBatch* __restrict__ bs, int round) {
  const EigBatch b = bs[blockIdx.y];
  if ((int)blockIdx.x >= b.w.p || round >= 2 * b.w.p - 1) return;
  eig_solve_body<JB>(b.w, round, round == 0, blockIdx.x, 0);
}
template <int JB>
__global__ __launch_bounds__(256) void k_eigb_apply(const EigBatch* __restrict__ bs, int round) {
  const EigBatch b = bs[blockIdx.y];
  if ((int)blockIdx.x >= eig_apply_items(b.w.p, b.w.K, 2 * JB) || round >= 2 * b.w.p - 1) return;
  eig_apply_body<JB>(b.w, round, blockIdx.x, 0);
}
__global__ __launch_bounds__(256) void k_eigb_check(const EigBatch* __restrict__ bs) {
  const EigBatch b = bs[blockIdx.y];
  if (blockIdx.x >= eig_check_blocks(b.w.K)) return;  // uniform per block
  eig_check_body(b.w, blockIdx.x);
}
__global__ void k_eigb_decide(const EigBatch* __restrict__ bs, double tol) {
  const EigBatch b = bs[blockIdx.y];
  eig_decide_body(b.w, tol, nullptr, 0);
}
__global__ __launch_bounds__(1024) void k_eigb_sort(const EigBatch* __restrict__ bs) {
  const EigBatch b = bs[blockIdx.y];
  eig_sort_body(b.w, b.N, b.lam);
}
__global__ void k_eigb_gather(const EigBatch* __restrict__ bs) {
  const EigBatch b = bs[blockIdx.y];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < b.N * b.N; e += (int64_t)gridDim.x * blockDim.x)
    eig_gather_body(b.w, b.N, b.V, b.ldv, e);
}

template <int JB>
static void eig_rounds(EigWork w, int64_t N, hipStream_t st, double* trace) {
  constexpr int JS = 2 * JB;
  const size_t lds_round = eig_round_lds(JB);
  const size_t lds_apply = JS * (JS + 1) * sizeof(double);
  const int rounds = 2 * w.p - 1;  // odd: a sweep's G updates into the other buffer come in pairs
  const int max_sweeps = eig_max_sweeps();
  const int nsym = w.p * (w.p + 1) / 2;
  const int nz = eig_apply_items(w.p, w.K, JS) - nsym;
  const int zgroups = (nz + 3) / 4;
  // G_j (before round j's update) sits in buffer j & 1 within a sweep: round r
  // builds its subproblems from buffer (r-1) & 1 while round r-1's tiles go from
  // there to buffer r & 1.  The last round (even) is updated in place in buffer
  // 0, where the convergence test and the next sweep read G.
  int g = 0, prev = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int r = 0; r < rounds; ++r, ++g) {
      const int slot = g & 1;
      const int nzw = g > 0 ? zgroups : 0;
      const int ntile = r > 0 ? nsym : 0;
      const int full = r == 0;  // more full rounds per sweep were measured no faster
      const int gsrc = r > 0 ? (r - 1) & 1 : -1, gdst = r & 1;
      hipLaunchKernelGGL(k_eig_round<JB>, dim3((unsigned)(w.p + nzw + ntile)), dim3(1024), lds_round, st, w, r, full,
                         slot, prev, slot ^ 1, nzw, gsrc, gdst);
      prev = r;
    }
    hipLaunchKernelGGL(k_eig_gtile<JB>, dim3(nsym), dim3(1024), lds_apply, st, w, prev, (g - 1) & 1);
    hipLaunchKernelGGL(k_eig_check, dim3(eig_check_blocks(w.K)), dim3(256), 0, st, w);
    hipLaunchKernelGGL(k_eig_decide, dim3(1), dim3(1), 0, st, w, 1.0, trace, sw);
  }
  // the Z update of the last round
  if (g > 0) hipLaunchKernelGGL(k_eig_apply<JB>, dim3(nz), dim3(256), lds_apply, st, w, prev, (g - 1) & 1, nsym);
}

// 32-wide blocks (64 x 64 subproblems).  16-wide blocks were measured slower at
// k = 1000: their 31-step subproblem sweep is bound by the per-step latency
// (rotation, two barriers), not by LDS traffic, and twice the rounds double the
// launches and the apply work.
int eig_block_width(int64_t N) { (void)N; return 32; }

// The launch sequence of one eigen-decomposition (about 1300 launches at N = 1000).
static hipError_t eig_sequence(double* G, int64_t ld, int64_t N, double* lam, double* V, int64_t ldv, void* work,
                               hipStream_t st, double tol, double* trace) {
  const int JB = eig_block_width(N);
  EigWork w = eig_layout(work, N, JB);
  w.tol = tol;
  int64_t KK = w.K * w.K;
  hipLaunchKernelGGL(k_eig_init, dim3((unsigned)((KK + 255) / 256)), dim3(256), 0, st, G, ld, N, w);
  hipLaunchKernelGGL(k_eig_norm_part, dim3(kNormParts), dim3(1024), 0, st, G, ld, N, w.npart);
  hipLaunchKernelGGL(k_eig_floor_fin, dim3(1), dim3(64), 0, st, w);
  eig_rounds<32>(w, N, st, trace);
  hipLaunchKernelGGL(k_eig_sort, dim3(1), dim3(1024), 0, st, w, N, lam);
  hipLaunchKernelGGL(k_eig_gather, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, st, w, N, V, ldv);
  return hipGetLastError();
}

// Instantiated graphs of the sequence, keyed by every kernel argument (device
// pointers, sizes, tolerance): a repeated call with the same buffers replays the
// graph instead of issuing the launches one by one, which removes the gaps
// between the short Jacobi kernels.  Each entry records an event after its
// latest launch; an entry is dropped (least recently used first) only once that
// event reports completion, so eviction never waits on the device.  When every
// entry is still in flight the new sequence is launched directly, uncached.
// While the caller's stream is being captured the sequence is launched straight
// into that capture (no private stream, no cache).
namespace {
struct EigGraph {
  int dev;
  const void *G, *lam, *V, *work, *trace;
  int64_t ld, N, ldv;
  double tol;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipEvent_t done;  // recorded after the entry's latest launch
  uint64_t used;
  bool same(const EigGraph& o) const {
    return dev == o.dev && G == o.G && lam == o.lam && V == o.V && work == o.work && trace == o.trace && ld == o.ld &&
           N == o.N && ldv == o.ldv && tol == o.tol;
  }
};
std::mutex g_eig_mu;
std::vector<EigGraph> g_eig_graphs;
uint64_t g_eig_clock = 0;
constexpr size_t kEigGraphs = 8;
constexpr int64_t kEigGraphMinN = 128;  // below this the sequence is short
}  // namespace

hipError_t launch_eig(double* G, int64_t ld, int64_t N, double* lam, double* V, int64_t ldv, void* work,
                      hipStream_t st, double tol, double* trace) {
  if (N == 0) return hipSuccess;
  if (eig_layout(nullptr, N, eig_block_width(N)).K > 4096) return hipErrorInvalidValue;
  {
    // kernel attributes are set once, on the first call
    constexpr int JS = 64;
    static std::once_flag attr;
    std::call_once(attr, [] {
      (void)hipFuncSetAttribute((const void*)k_eig_apply<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(JS * (JS + 1) * sizeof(double)));
      (void)hipFuncSetAttribute((const void*)k_eig_round<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)eig_round_lds(32));
    });
  }
  if (N < kEigGraphMinN) return eig_sequence(G, ld, N, lam, V, ldv, work, st, tol, trace);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return hipErrorInvalidValue;
  if (cap != hipStreamCaptureStatusNone) return eig_sequence(G, ld, N, lam, V, ldv, work, st, tol, trace);
  EigGraph key{};
  (void)hipGetDevice(&key.dev);
  key.G = G; key.lam = lam; key.V = V; key.work = work; key.trace = trace;
  key.ld = ld; key.N = N; key.ldv = ldv; key.tol = tol;
  std::lock_guard<std::mutex> lock(g_eig_mu);
  for (auto& e : g_eig_graphs)
    if (e.same(key)) {
      e.used = ++g_eig_clock;
      const hipError_t le = hipGraphLaunch(e.exec, st);
      if (le != hipSuccess) return le;
      return hipEventRecord(e.done, st);
    }
  // room for the new entry: drop the least recently used entry whose last
  // launch has finished; if none has, run this sequence uncached
  if (g_eig_graphs.size() >= kEigGraphs) {
    ptrdiff_t lru = -1;
    for (size_t i = 0; i < g_eig_graphs.size(); ++i) {
      if (hipEventQuery(g_eig_graphs[i].done) != hipSuccess) continue;
      if (lru < 0 || g_eig_graphs[i].used < g_eig_graphs[(size_t)lru].used) lru = (ptrdiff_t)i;
    }
    (void)hipGetLastError();  // hipEventQuery reports hipErrorNotReady for busy entries
    if (lru < 0) return eig_sequence(G, ld, N, lam, V, ldv, work, st, tol, trace);
    (void)hipGraphExecDestroy(g_eig_graphs[(size_t)lru].exec);
    (void)hipGraphDestroy(g_eig_graphs[(size_t)lru].graph);
    (void)hipEventDestroy(g_eig_graphs[(size_t)lru].done);
    g_eig_graphs.erase(g_eig_graphs.begin() + lru);
  }
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return eig_sequence(G, ld, N, lam, V, ldv, work, st, tol, trace);
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  hipEvent_t ev = nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (ok) {
    const hipError_t le = eig_sequence(G, ld, N, lam, V, ldv, work, cs, tol, trace);
    ok = (hipStreamEndCapture(cs, &g) == hipSuccess) && le == hipSuccess && g != nullptr;
  }
  (void)hipStreamDestroy(cs);
  if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  if (ok) ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    if (ex) (void)hipGraphExecDestroy(ex);
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return eig_sequence(G, ld, N, lam, V, ldv, work, st, tol, trace);
  }
  key.graph = g;
  key.exec = ex;
  key.done = ev;
  key.used = ++g_eig_clock;
  g_eig_graphs.push_back(key);
  const hipError_t le = hipGraphLaunch(ex, st);
  if (le != hipSuccess) return le;
  return hipEventRecord(ev, st);
}

// Batched eigensolver: problem i (G_i N_i x N_i, ld_i, preserved) -> lam_i, V_i.
// work_i: eig_work_bytes(N_i) bytes each; descs: device array of count EigBatch
// written by the caller from eig_batch_desc().  All problems take the same number
// of launches (the largest), smaller ones skip the rounds they do not have and
// stop sweeping when converged.
EigBatch eig_batch_desc(const double* G, int64_t ld, int64_t N, double* lam, double* V, int64_t ldv, void* work,
                        double tol) {
  EigBatch b;
  b.w = eig_layout(work, N, 32, false);
  b.w.tol = tol;
  b.G = G; b.ld = ld; b.N = N; b.lam = lam; b.V = V; b.ldv = ldv;
  return b;
}

hipError_t launch_eig_batched(const EigBatch* descs, int count, int64_t Nmax, hipStream_t st) {
  if (count == 0 || Nmax == 0) return hipSuccess;
  constexpr int JB = 32, JS = 64;
  EigWork shape = eig_layout(nullptr, Nmax, JB, false);
  const int64_t Kmax = shape.K;
  const int pmax = shape.p;
  if (Kmax > 4096) return hipErrorInvalidValue;
  const size_t lds_solve = 2 * JS * (JS + 1) * sizeof(double);
  const size_t lds_apply = JS * (JS + 1) * sizeof(double);
  (void)hipFuncSetAttribute((const void*)k_eigb_solve<JB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_solve);
  (void)hipFuncSetAttribute((const void*)k_eigb_apply<JB>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_apply);
  const int64_t KK = Kmax * Kmax;
  const unsigned gx = (unsigned)((KK + 255) / 256);
  hipLaunchKernelGGL(k_eigb_init, dim3(gx, count), dim3(256), 0, st, descs);
  hipLaunchKernelGGL(k_eigb_floor, dim3(1, count), dim3(1024), 0, st, descs);
  const int rounds = 2 * pmax - 1;
  const int ntile = eig_apply_items(pmax, Kmax, JS);
  for (int sw = 0; sw < eig_max_sweeps(); ++sw) {
    for (int r = 0; r < rounds; ++r) {
      hipLaunchKernelGGL(k_eigb_solve<JB>, dim3(pmax, count), dim3(1024), lds_solve, st, descs, r);
      hipLaunchKernelGGL(k_eigb_apply<JB>, dim3(ntile, count), dim3(256), lds_apply, st, descs, r);
    }
    hipLaunchKernelGGL(k_eigb_check, dim3(eig_check_blocks(Kmax), count), dim3(256), 0, st, descs);
    hipLaunchKernelGGL(k_eigb_decide, dim3(1, count), dim3(1), 0, st, descs, 1.0);
  }
  hipLaunchKernelGGL(k_eigb_sort, dim3(1, count), dim3(1024), 0, st, descs);
  hipLaunchKernelGGL(k_eigb_gather, dim3((unsigned)((Nmax * Nmax + 255) / 256), count), dim3(256), 0, st, descs);
  return hipGetLastError();
}

// ============================== utilities ==============================
// four consecutive columns per thread: one 16-byte load and one 8-byte store where
// both operands allow it (vec), element by element otherwise
__global__ void k_cast_f32_bf16(const float* __restrict__ in, int64_t ldi, uint16_t* __restrict__ out, int64_t ldo,
                                int64_t rows, int64_t cols, bool vec) {
  const int64_t c4 = (cols + 3) / 4;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * c4) return;
  const int64_t i = idx / c4, j = (idx - i * c4) * 4;
  const float* src = in + i * ldi + j;
  uint16_t* dst = out + i * ldo + j;
  if (vec && j + 4 <= cols) {
    const float4 v = *reinterpret_cast<const float4*>(src);
    *reinterpret_cast<uint2*>(dst) =
        make_uint2((uint32_t)f32_to_bf16_rne(v.x) | ((uint32_t)f32_to_bf16_rne(v.y) << 16),
                   (uint32_t)f32_to_bf16_rne(v.z) | ((uint32_t)f32_to_bf16_rne(v.w) << 16));
  } else {
    for (int e = 0; e < 4 && j + e < cols; ++e) dst[e] = f32_to_bf16_rne(src[e]);
  }
}
__global__ void k_cast_f64_f32(const double* __restrict__ in, int64_t ldi, float* __restrict__ out, int64_t ldo,
                               int64_t rows, int64_t cols) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  int64_t i = idx / cols, j = idx % cols;
  out[i * ldo + j] = (float)in[i * ldi + j];
}
__global__ void k_copy_f32(const float* __restrict__ in, int64_t ldi, float* __restrict__ out, int64_t ldo,
                           int64_t rows, int64_t cols) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  int64_t i = idx / cols, j = idx % cols;
  out[i * ldo + j] = in[i * ldi + j];
}
__global__ void k_fill_i32(int* p, int64_t n, int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static inline dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_cast_f32_bf16(const float* in, int64_t ldi, uint16_t* out, int64_t ldo, int64_t rows, int64_t cols,
                                hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  const bool vec = ((uintptr_t)in % 16 == 0) && (ldi % 4 == 0) && ((uintptr_t)out % 8 == 0) && (ldo % 4 == 0);
  hipLaunchKernelGGL(k_cast_f32_bf16, g1(rows * ((cols + 3) / 4)), dim3(256), 0, st, in, ldi, out, ldo, rows, cols, vec);
  return hipGetLastError();
}
hipError_t launch_cast_f64_f32(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                               hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f64_f32, g1(rows * cols), dim3(256), 0, st, in, ldi, out, ldo, rows, cols);
  return hipGetLastError();
}
hipError_t launch_copy_f32(const float* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                           hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f32, g1(rows * cols), dim3(256), 0, st, in, ldi, out, ldo, rows, cols);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, g1(n), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

RF_DEV void refill_entry(float* __restrict__ X, int64_t ldx, int64_t rows, int64_t k, const int* __restrict__ flags,
                         const double* __restrict__ d0, uint64_t seed, uint32_t b, int64_t idx) {
  int64_t i = idx / k, j = idx % k;
  if (!flags[j]) return;
  double dm = 0.0;
  for (int64_t c = 0; c < k; ++c) dm = fmax(dm, d0[c]);
  double sc = sqrt(dm / (double)rows);
  if (!(sc > 0.0) || !isfinite(sc)) sc = 1.0 / sqrt((double)rows);
  // entry (i, j) of a rows x k Gaussian on stream 3
  int64_t e = i * k + j;
  u32x4 x = philox((uint64_t)(e >> 2), 3u, b, seed);
  uint32_t w[4] = {x.x, x.y, x.z, x.w};
  int q = (int)(e & 3);
  const double s32 = 2.3283064365386963e-10;
  double ua = ((double)w[(q >> 1) * 2] + 0.5) * s32, ub = ((double)w[(q >> 1) * 2 + 1] + 0.5) * s32;
  double rad = sqrt(-2.0 * log(ua));
  double z = (q & 1) ? rad * sin(6.283185307179586 * ub) : rad * cos(6.283185307179586 * ub);
  X[i * ldx + j] = (float)(z * sc);
}

__global__ void k_refill(float* __restrict__ X, int64_t ldx, int64_t rows, int64_t k, const int* __restrict__ flags,
                         const int* count, const double* __restrict__ d0, uint64_t seed) {
  if (*count == 0) return;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < rows * k;
       idx += (int64_t)gridDim.x * blockDim.x)
    refill_entry(X, ldx, rows, k, flags, d0, seed, 0u, idx);
}

hipError_t launch_refill(float* X, int64_t ldx, int64_t rows, int64_t k, const int* flags, const int* count,
                         const double* d0, uint64_t seed, hipStream_t st) {
  if (rows * k == 0) return hipSuccess;
  // a bounded grid: usually nothing is flagged and every workgroup returns at once
  const dim3 grid((unsigned)std::min<int64_t>((rows * k + 255) / 256, 4096));
  hipLaunchKernelGGL(k_refill, grid, dim3(256), 0, st, X, ldx, rows, k, flags, count, d0, seed);
  return hipGetLastError();
}

__global__ void k_sigma(const double* lam, int64_t k, double* sigma, float* inv32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double l = lam[i];
  double s = l > 0.0 ? sqrt(l) : 0.0;
  if (sigma) sigma[i] = s;
  if (inv32) inv32[i] = s > 0.0 ? (float)(1.0 / s) : 0.f;
}
hipError_t launch_sigma(const double* lam, int64_t k, double* sigma, float* inv32, hipStream_t st) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sigma, g1(k), dim3(256), 0, st, lam, k, sigma, inv32);
  return hipGetLastError();
}

// key = |u| bits << 32 | (0xffffffff - row): max key = largest |u|, lowest row on ties
__global__ void k_sign_key(const float* __restrict__ U, int64_t ldu, int64_t m, int64_t k,
                           unsigned long long* __restrict__ keys, int64_t rows_per) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  int64_t r0 = (int64_t)blockIdx.y * rows_per, r1 = min(m, r0 + rows_per);
  unsigned long long best = 0ull;
  for (int64_t r = r0; r < r1; ++r) {
    float v = fabsf(U[r * ldu + c]);
    unsigned long long key = ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)r);
    best = key > best ? key : best;
  }
  atomicMax(keys + c, best);
}
__global__ void k_sign_decide(const float* __restrict__ U, int64_t ldu, int64_t k,
                              const unsigned long long* __restrict__ keys, float* __restrict__ sgn) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  int64_t rr = 0xffffffffll - (int64_t)(keys[c] & 0xffffffffull);
  sgn[c] = (U[rr * ldu + c] < 0.f) ? -1.f : 1.f;
}
// four consecutive entries of a row per thread (16-byte accesses where aligned):
// U's columns and Vt's rows take the sign of their column
__global__ void k_sign_apply(float* __restrict__ U, int64_t ldu, int64_t m, int64_t k, float* __restrict__ Vt,
                             int64_t ldvt, int64_t n, const float* __restrict__ sgn, bool uvec, bool vvec) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k4 = (k + 3) / 4, n4 = (n + 3) / 4;
  if (idx < m * k4) {
    const int64_t r = idx / k4, c = (idx - r * k4) * 4;
    float* p = U + r * ldu + c;
    if (uvec && c + 4 <= k) {
      float4 v = *reinterpret_cast<float4*>(p);
      v.x *= sgn[c]; v.y *= sgn[c + 1]; v.z *= sgn[c + 2]; v.w *= sgn[c + 3];
      *reinterpret_cast<float4*>(p) = v;
    } else {
      for (int e = 0; e < 4 && c + e < k; ++e) p[e] *= sgn[c + e];
    }
  } else if (Vt && idx < m * k4 + k * n4) {
    const int64_t e0 = idx - m * k4;
    const int64_t c = e0 / n4, j = (e0 - c * n4) * 4;
    float* p = Vt + c * ldvt + j;
    const float sg = sgn[c];
    if (vvec && j + 4 <= n) {
      float4 v = *reinterpret_cast<float4*>(p);
      v.x *= sg; v.y *= sg; v.z *= sg; v.w *= sg;
      *reinterpret_cast<float4*>(p) = v;
    } else {
      for (int e = 0; e < 4 && j + e < n; ++e) p[e] *= sg;
    }
  }
}

// work: 3 k ints (keys: 2k, signs: k)
hipError_t launch_sign_fix(float* U, int64_t ldu, int64_t m, int64_t k, float* Vt, int64_t ldvt, int64_t n, int* work,
                           hipStream_t st) {
  if (m * k == 0) return hipSuccess;
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(work);
  float* sgn = reinterpret_cast<float*>(work + 2 * k);
  hipLaunchKernelGGL(k_fill_i32, g1(2 * k), dim3(256), 0, st, work, 2 * k, 0);
  int64_t rows_per = 256;
  dim3 grid((unsigned)((k + 255) / 256), (unsigned)((m + rows_per - 1) / rows_per));
  hipLaunchKernelGGL(k_sign_key, grid, dim3(256), 0, st, U, ldu, m, k, keys, rows_per);
  hipLaunchKernelGGL(k_sign_decide, g1(k), dim3(256), 0, st, U, ldu, k, keys, sgn);
  const int64_t tot = m * ((k + 3) / 4) + (Vt ? k * ((n + 3) / 4) : 0);
  const bool uvec = ((uintptr_t)U % 16 == 0) && (ldu % 4 == 0);
  const bool vvec = Vt && ((uintptr_t)Vt % 16 == 0) && (ldvt % 4 == 0);
  hipLaunchKernelGGL(k_sign_apply, g1(tot), dim3(256), 0, st, U, ldu, m, k, Vt, ldvt, n, sgn, uvec, vvec);
  return hipGetLastError();
}

__global__ void k_note_first(int* counters) {
  // after the first factorisation of a pass: remember whether a refill happened
  int c = counters[0];
  counters[4] = c > 0 ? 1 : 0;
  if (c > 0) counters[1] += 1;
}
__global__ void k_note_final(int* counters) { counters[3] = counters[0]; }
hipError_t launch_note(int* counters, int final_, hipStream_t st) {
  if (final_) hipLaunchKernelGGL(k_note_final, dim3(1), dim3(1), 0, st, counters);
  else hipLaunchKernelGGL(k_note_first, dim3(1), dim3(1), 0, st, counters);
  return hipGetLastError();
}

// ---- batched utilities (one problem per blockIdx.y, grid-stride inside) -----------
__global__ void k_cast_batched(const CastArgs* __restrict__ as, int f64_to_f32) {
  const CastArgs a = as[blockIdx.y];
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.rows * a.cols;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / a.cols, j = idx % a.cols;
    if (f64_to_f32)
      reinterpret_cast<float*>(a.out)[i * a.ldo + j] = (float)reinterpret_cast<const double*>(a.in)[i * a.ldi + j];
    else
      reinterpret_cast<uint16_t*>(a.out)[i * a.ldo + j] = f32_to_bf16_rne(reinterpret_cast<const float*>(a.in)[i * a.ldi + j]);
  }
}
__global__ void k_refill_batched(const RefillArgs* __restrict__ as) {
  const RefillArgs a = as[blockIdx.y];
  if (*a.count == 0) return;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < a.rows * a.k;
       idx += (int64_t)gridDim.x * blockDim.x)
    if (a.flags[idx % a.k]) refill_entry(a.X, a.ldx, a.rows, a.k, a.flags, a.d0, a.seed, a.b, idx);
}
__global__ void k_note_batched(int* const* __restrict__ cs, int count, int final_) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int* c = cs[i];
  if (final_) {
    c[3] = c[0];
  } else {
    const int n = c[0];
    c[4] = n > 0 ? 1 : 0;
    if (n > 0) c[1] += 1;
  }
}
__global__ void k_svd_tail_batched(const SvdTailArgs* __restrict__ as, int stage) {
  const SvdTailArgs a = as[blockIdx.z];
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(a.signw);
  float* sgn = reinterpret_cast<float*>(a.signw + 2 * a.k);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (stage == 0) {           // sigma, 1/sigma, FP32 copy of the Ritz vectors, clear the keys
    const int64_t lim = a.k * a.k > 2 * a.k ? a.k * a.k : 2 * a.k;
    for (int64_t i = t; i < lim; i += (int64_t)gridDim.x * blockDim.x) {
      if (i < a.k * a.k) a.Ub32[i] = (float)a.Ub[i];
      if (i < a.k) {
        const double l = a.lam[i];
        const double sv = l > 0.0 ? sqrt(l) : 0.0;
        a.sigma[i] = sv;
        a.inv[i] = sv > 0.0 ? (float)(1.0 / sv) : 0.f;
      }
      if (i < 2 * a.k) a.signw[i] = 0;
    }
  } else if (stage == 1) {    // per column: largest |U| (lowest row on ties), rows split over blockIdx.y
    if (t >= a.k) return;
    const int64_t rows_per = (a.m + gridDim.y - 1) / gridDim.y;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per, r1 = min(a.m, r0 + rows_per);
    unsigned long long best = 0ull;
    for (int64_t r = r0; r < r1; ++r) {
      const float v = fabsf(a.U[r * a.ldu + t]);
      const unsigned long long key =
          ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)r);
      best = key > best ? key : best;
    }
    if (best) atomicMax(keys + t, best);
  } else if (stage == 2) {    // signs
    if (t >= a.k) return;
    const int64_t rr = 0xffffffffll - (int64_t)(keys[t] & 0xffffffffull);
    sgn[t] = (rr < a.m && a.U[rr * a.ldu + t] < 0.f) ? -1.f : 1.f;
  } else {                    // apply to U and V^T
    const int64_t tot = a.m * a.k + a.k * a.n;
    for (int64_t idx = t + (int64_t)blockIdx.y * gridDim.x * blockDim.x; idx < tot;
         idx += (int64_t)gridDim.y * gridDim.x * blockDim.x) {
      if (idx < a.m * a.k) {
        const int64_t r = idx / a.k, c = idx % a.k;
        a.U[r * a.ldu + c] *= sgn[c];
      } else {
        const int64_t e = idx - a.m * a.k, c = e / a.n, j = e % a.n;
        a.Vt[c * a.ldvt + j] *= sgn[c];
      }
    }
  }
}

hipError_t launch_cast_batched(const CastArgs* as, int count, int64_t max_elems, int f64_to_f32, hipStream_t st) {
  if (count == 0 || max_elems == 0) return hipSuccess;
  unsigned gx = (unsigned)((max_elems + 255) / 256);
  if (gx > 2048) gx = 2048;
  hipLaunchKernelGGL(k_cast_batched, dim3(gx, count), dim3(256), 0, st, as, f64_to_f32);
  return hipGetLastError();
}
hipError_t launch_refill_batched(const RefillArgs* as, int count, int64_t max_elems, hipStream_t st) {
  if (count == 0 || max_elems == 0) return hipSuccess;
  unsigned gx = (unsigned)((max_elems + 255) / 256);
  if (gx > 2048) gx = 2048;
  hipLaunchKernelGGL(k_refill_batched, dim3(gx, count), dim3(256), 0, st, as);
  return hipGetLastError();
}
hipError_t launch_note_batched(int* const* cs, int count, int final_, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_note_batched, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, cs, count, final_);
  return hipGetLastError();
}
hipError_t launch_svd_tail_pre_batched(const SvdTailArgs* as, int count, int64_t kmax, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const unsigned g0 = (unsigned)((kmax * kmax + 2 * kmax + 255) / 256);
  hipLaunchKernelGGL(k_svd_tail_batched, dim3(g0, 1, count), dim3(256), 0, st, as, 0);
  return hipGetLastError();
}
hipError_t launch_svd_tail_sign_batched(const SvdTailArgs* as, int count, int64_t kmax, int64_t mmax,
                                        int64_t max_elems, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const unsigned gk = (unsigned)((kmax + 255) / 256);
  const unsigned gr = (unsigned)((mmax + 255) / 256);
  hipLaunchKernelGGL(k_svd_tail_batched, dim3(gk, gr, count), dim3(256), 0, st, as, 1);
  hipLaunchKernelGGL(k_svd_tail_batched, dim3(gk, 1, count), dim3(256), 0, st, as, 2);
  unsigned ga = (unsigned)((max_elems + 255) / 256);
  if (ga > 1024) ga = 1024;
  hipLaunchKernelGGL(k_svd_tail_batched, dim3(ga, 1, count), dim3(256), 0, st, as, 3);
  return hipGetLastError();
}

__global__ void k_nystrom_scale(const double* lam, int64_t k, float* scale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double lmax = lam[0] > 0.0 ? lam[0] : 0.0;
  double cut = (double)k * 2.220446049250313e-16 * lmax;
  double l = lam[i];
  scale[i] = (l > cut && l > 0.0) ? (float)(1.0 / sqrt(l)) : 0.f;
}
hipError_t launch_nystrom_scale(const double* lam, int64_t k, float* scale, hipStream_t st) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nystrom_scale, g1(k), dim3(256), 0, st, lam, k, scale);
  return hipGetLastError();
}

struct InfoOut {
  int32_t status, rank_found, chol_retries, nonfinite;
  double orth_err;
};
RF_DEV void k_info_body(InfoOut* info, const int* counters, int k, const double* orth) {
  int retries = counters[1], nonf = counters[2], last = counters[3], fault = counters[5], bad = counters[6],
      badcsr = counters[7];
  info->status = (retries > 0 ? 1 : 0) | (nonf ? 2 : 0) | (fault ? 4 : 0) | (bad ? 8 : 0) | (badcsr ? 16 : 0);
  info->rank_found = k - last;
  info->chol_retries = retries;
  info->nonfinite = nonf;
  info->orth_err = orth ? *orth : -1.0;
}
__global__ void k_info(InfoOut* info, const int* counters, int k, const double* orth) {
  k_info_body(info, counters, k, orth);
}
__global__ void k_info_batched(InfoOut* infos, const int* counters, int stride, const int* ks, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  k_info_body(&infos[i], counters + (int64_t)i * stride, ks[i], nullptr);
}
hipError_t launch_info_batched(void* infos, const int* counters, int stride, const int* ks, int count, hipStream_t st) {
  if (!infos || count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_info_batched, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, (InfoOut*)infos,
                     counters, stride, ks, count);
  return hipGetLastError();
}
hipError_t launch_info(void* info, const int* counters, int k, const double* orth, hipStream_t st) {
  if (!info) return hipSuccess;
  hipLaunchKernelGGL(k_info, dim3(1), dim3(1), 0, st, (InfoOut*)info, counters, k, orth);
  return hipGetLastError();
}

__global__ void k_orth_err(const double* __restrict__ G, int64_t ld, int64_t N, unsigned long long* out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double r = 0.0;
  if (idx < N * N) {
    int64_t i = idx / N, j = idx % N;
    r = fabs(G[i * ld + j] - (i == j ? 1.0 : 0.0));
    if (!(r == r)) r = INFINITY;
  }
  r = wave_max(r);
  if ((threadIdx.x & 63) == 0 && r > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(r));
}
hipError_t launch_orth_err(const double* G, int64_t ld, int64_t N, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, (int*)out, 2, 0);
  if (N == 0) return hipGetLastError();
  hipLaunchKernelGGL(k_orth_err, g1(N * N), dim3(256), 0, st, G, ld, N, (unsigned long long*)out);
  return hipGetLastError();
}

__global__ void k_symmetrize(float* X, int64_t ld, int64_t N) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * N) return;
  int64_t i = idx / N, j = idx % N;
  if (i < j) {
    float a = X[i * ld + j], b = X[j * ld + i];
    float m = 0.5f * (a + b);
    X[i * ld + j] = m;
    X[j * ld + i] = m;
  }
}
hipError_t launch_symmetrize(float* X, int64_t ld, int64_t N, hipStream_t st) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_symmetrize, g1(N * N), dim3(256), 0, st, X, ld, N);
  return hipGetLastError();
}

__global__ void k_symmetrize64(double* X, int64_t ld, int64_t N) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * N) return;
  int64_t i = idx / N, j = idx % N;
  if (i < j) {
    double m = 0.5 * (X[i * ld + j] + X[j * ld + i]);
    X[i * ld + j] = m;
    X[j * ld + i] = m;
  }
}
hipError_t launch_symmetrize64(double* X, int64_t ld, int64_t N, hipStream_t st) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_symmetrize64, g1(N * N), dim3(256), 0, st, X, ld, N);
  return hipGetLastError();
}
__global__ void k_copy_f64(const double* __restrict__ in, int64_t ldi, double* __restrict__ out, int64_t ldo,
                           int64_t rows, int64_t cols) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  int64_t i = idx / cols, j = idx % cols;
  out[i * ldo + j] = in[i * ldi + j];
}
hipError_t launch_copy_f64(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t rows, int64_t cols,
                           hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f64, g1(rows * cols), dim3(256), 0, st, in, ldi, out, ldo, rows, cols);
  return hipGetLastError();
}

}  // namespace rf
