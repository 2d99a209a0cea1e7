// Cholesky factor and its inverse in one launch: G = R^T R (R upper, in place)
// and X = R^{-1}, for the CholeskyQR passes (Q = Y R^{-1}; Algorithm 1, line 2).
//
// Blocked right-looking factorisation on 64 x 64 tiles, run as a persistent
// kernel over a task list in dependency order.  Step kb has
//   A(kb)     factor the diagonal tile: R_kk and X_kk = R_kk^{-1} (one workgroup);
//   B(kb, j)  panel R_kb,j = X_kk^T G_kb,j for j > kb;
//   X(kb, i)  inverse tile X_i,kb = -T_i,kb X_kk for i < kb;
//   C(kb,i,j) trailing update G_ij -= R_kb,i^T R_kb,j for kb < i <= j;
//   U(kb,i,j) inverse update T_ij += X_i,kb R_kb,j for i <= kb < j.
// T_ij = sum_{l=i..j-1} X_il R_lj (from X R = I: X_ij R_jj = -T_ij) is accumulated
// in the X tile (i, j) as the columns of X become final (right-looking, like the
// factorisation), so the inverse adds two tile products per step to the critical
// path instead of a sum over all earlier columns.
// Workgroups take task tickets from an atomic counter, step by step in the order
// A(kb), B(kb, .), X(kb, .), C(kb, .), U(kb, .), and wait on per-tile counters (the
// dependencies of the tile algorithm, so later steps start as soon as their own
// tiles are ready):
//   gcnt(i,j): trailing updates applied to G tile (i,j); A(kb) waits gcnt(kb,kb) = kb,
//     B(kb,j) waits gcnt(kb,j) = kb, C(kb,i,j) waits gcnt(i,j) = kb (its previous writer);
//   pdone(kb,j): panel R_kb,j written (B(kb,j), or A(kb) for j = kb); C(kb,i,j) waits
//     pdone(kb,i) and pdone(kb,j), U(kb,i,j) waits pdone(kb,j), B and X wait pdone(kb,kb);
//   tcnt(i,j): inverse updates applied to T tile (i,j); X(kb,i) waits tcnt(i,kb) = kb - i,
//     U(kb,i,j) waits tcnt(i,j) = kb - i (its previous writer);
//   xdone(i,kb): X tile (i,kb) final; U(kb,i,j) waits it (i < kb).
// A task only waits on tasks with smaller tickets, which are held by running
// workgroups, so the queue drains without co-residency guarantees; every wait is
// bounded and raises the fault word instead of hanging.
// Completion is published with an agent-scope release (L2 write-back, the
// workgroups sit on different XCDs) and observed with an acquire.
#include "common.h"
#include "kernels.h"

namespace rf {

constexpr int TB = 64;          // tile
constexpr int TLD = TB + 1;     // LDS row stride (doubles)
constexpr unsigned kSpinLimit = 1u << 20;  // polls of ~1 us: a stuck dependency ends the launch in ~1 s


RF_DEV int nC_of(int nb, int kb) { int t = nb - 1 - kb; return t * (t + 1) / 2; }
RF_DEV int nU_of(int nb, int kb) { return (kb + 1) * (nb - 1 - kb); }
RF_DEV int step_tasks(int nb, int kb) { return nb + nC_of(nb, kb) + nU_of(nb, kb); }
static int host_step_tasks(int nb, int kb) {
  const int t = nb - 1 - kb;
  return nb + t * (t + 1) / 2 + (kb + 1) * t;
}

// Called by a whole wave (uniform branch); every lane polls the same word.  Gives
// up after kSpinLimit polls, or at once when another wait has already given up.
RF_DEV void wait_at_least(int* ctr, int target, int* err) {
  unsigned spins = 0;
  // relaxed polls (an acquire per poll would invalidate this XCD's L2 every time)
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
    __builtin_amdgcn_s_sleep(2);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// 256 threads; all 16 loads of a thread are issued before the LDS stores.
RF_DEV void load_tile(double (*T)[TLD], gptr<const double> P, int64_t ld, int64_t r0, int64_t c0, int64_t N) {
  constexpr int NT = 256, IT = TB * TB / NT;
  const int c = threadIdx.x % TB, rr = threadIdx.x / TB;
  double v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int r = rr + it * (NT / TB);
    v[it] = (r0 + r < N && c0 + c < N) ? P[(r0 + r) * ld + c0 + c] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) T[rr + it * (NT / TB)][c] = v[it];
}

// acc (+)= op(P) Q over a 64-deep product of 64 x 64 LDS tiles (op(P) = P^T when
// P_TRANS) on v_mfma_f64_16x16x4f64.  Wave w owns the 32 x 32 quadrant
// (w / 2, w % 2) as 2 x 2 blocks of 16 x 16; register r of lane l of block (i, j)
// holds row tile_row(i, r), column tile_col(j).
RF_DEV int tile_row(int i, int r) {
  return ((threadIdx.x >> 6) >> 1) * 32 + i * 16 + ((threadIdx.x & 63) >> 4) + 4 * r;
}
RF_DEV int tile_col(int j) { return ((threadIdx.x >> 6) & 1) * 32 + j * 16 + (threadIdx.x & 15); }

template <bool P_TRANS>
RF_DEV void tile_mac(f64x4 (&acc)[2][2], double (*P)[TLD], double (*Q)[TLD]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
#pragma unroll 4
  for (int kk = 0; kk < TB / 4; ++kk) {
    const int kr = 4 * kk + (lane >> 4);
    double af[2], bf[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = wm * 32 + i * 16 + (lane & 15);
      af[i] = P_TRANS ? P[kr][row] : P[row][kr];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) bf[j] = Q[kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
  }
}

RF_DEV void acc_zero(f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0, 0, 0, 0};
}

// 1/sqrt(d) for d > 0 to FP64 accuracy: FP32 estimate of the scaled argument, two
// Newton steps r <- r (3 - m r^2) / 2 (each squares the relative error).
RF_DEV double rsqrt_f64(double d) {
  int e;
  (void)frexp(d, &e);
  const int e2 = e & ~1;                  // even exponent: d = m 2^e2, m in [1/4, 1)
  const double m = ldexp(d, -e2);
  double r = (double)__builtin_amdgcn_rsqf((float)m);
  r = r * fma(-0.5 * m, r * r, 1.5);
  r = r * fma(-0.5 * m, r * r, 1.5);
  return ldexp(r, -e2 / 2);
}

RF_DEV void put_x(const CholInvArgs& a, int64_t r, int64_t c, double v) {
  if (r >= a.N || c >= a.N) return;
  as_global_w<double>(a.X64)[r * a.ldx64 + c] = v;
  if (a.X32) as_global_w<float>(a.X32)[r * a.ldx32 + c] = (float)v;
}

// Orders one wave's LDS accesses between the steps of a wave-synchronous loop.
RF_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int SB = 16;  // diagonal sub-block of the inverse

// Inverse of the upper-triangular sub-block [k0, k0 + kn) of R (1 / R_cc in rsv):
// lane j < kn of the calling wave solves column j by back substitution.
RF_DEV void inv_sub(int k0, int kn, double (*R)[TLD], double (*Xs)[TLD], const double* rsv) {
  const int lane = threadIdx.x & 63;
  if (lane < kn) {
    double x[SB];
#pragma unroll
    for (int c = SB - 1; c >= 0; --c) {
      double acc = (c == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int l = c + 1; l < SB; ++l) acc = fma(-R[k0 + c][k0 + l], x[l], acc);  // R is zero beyond kn
      x[c] = (c <= lane) ? acc * rsv[k0 + c] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < SB; ++c)
      if (c <= lane) Xs[k0 + c][k0 + lane] = x[c];
  }
}

// Element (a, b) of a thread's 4 x 4 register block with a runtime row a.
// (value selects, so that the block stays in registers)
RF_DEV double pick_row(const double (&m)[4][4], int a, int b) {
  const double v0 = m[0][b], v1 = m[1][b], v2 = m[2][b], v3 = m[3][b];
  double r = v0;
  r = (a == 1) ? v1 : r;
  r = (a == 2) ? v2 : r;
  r = (a == 3) ? v3 : r;
  return r;
}

// A(kb): R_kk and X_kk = R_kk^{-1}, written to G and X.  The tile lives in
// registers: thread (ty, tx) of 16 x 16 holds entries (ty + 16a, tx + 16b).
// Cholesky, right-looking, one barrier per column: the threads holding row c + 1
// publish it, unscaled, into row c + 1 of R right after their step-c update, and at
// step c + 1 every thread reads it, forms R_c+1,. = G_c+1,. / sqrt(g) in registers
// and updates its entries.  R is scaled by its 1 / sqrt(g) once, after the loop.
// Inverse blocked by 16 (see below).
RF_DEV void task_diag(const CholInvArgs& a, int kb, double (*M)[TLD], double (*R)[TLD], double (*Xs)[TLD]) {
  const int64_t b0 = (int64_t)kb * TB;
  const int nbk = (int)min((int64_t)TB, a.N - b0);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double* rsc = &M[0][0];   // M's LDS is scratch here: 1 / sqrt(g) per column (0 when dependent),
  double* rsv = rsc + TB;   // 1 / R_cc for the inverse, pivot floors
  double* floor_ = rsv + TB;
  if (threadIdx.x < nbk) floor_[threadIdx.x] = a.tol * as_global<double>(a.d0)[b0 + threadIdx.x];
  double m[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ty + 16 * p, j = tx + 16 * q;
      m[p][q] = (i < nbk && j < nbk) ? as_global<double>(a.G)[(b0 + i) * a.ld + b0 + j] : 0.0;
    }
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    R[e / TB][e % TB] = 0.0;
    Xs[e / TB][e % TB] = 0.0;
  }
  __syncthreads();
  if (ty == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) R[0][tx + 16 * q] = m[0][q];
  }
  __syncthreads();
  for (int c = 0; c < nbk; ++c) {
    const double* row = R[c];
    const double d = row[c], fl = floor_[c];
    double vi[4], vj[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) vi[p] = row[ty + 16 * p];   // every index < TB: in the row
#pragma unroll
    for (int q = 0; q < 4; ++q) vj[q] = row[tx + 16 * q];
    const bool fin = isfinite(d);
    const bool bad = !(fin & (d > fl) & (d > 0.0));
    const double rs = bad ? 0.0 : rsqrt_f64(d);
    if (threadIdx.x == 0) {
      if (!fin) *a.nonfinite = 1;
      if (bad) {
        as_global_w<int>(a.flags)[b0 + c] = 1;
        atomicAdd(a.count, 1);
      }
      rsc[c] = rs;
    }
    double ri[4], rj[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = ty + 16 * p;
      ri[p] = (i > c && i < nbk) ? vi[p] * rs : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = tx + 16 * q;
      rj[q] = (j > c && j < nbk) ? vj[q] * rs : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) m[p][q] = fma(-ri[p], rj[q], m[p][q]);
    const int c1 = c + 1;
    if (c1 < nbk && ty == (c1 & 15)) {
#pragma unroll
      for (int q = 0; q < 4; ++q) R[c1][tx + 16 * q] = pick_row(m, c1 >> 4, q);
    }
    __syncthreads();
  }
  // R_cj = g_cj / sqrt(g_cc) above the diagonal, sqrt(g_cc) on it, zero below; a
  // dependent column gets a unit diagonal and a zero row
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int r = e / TB, cc = e % TB;
    if (r >= nbk || cc >= nbk) continue;
    const double rs = rsc[r];
    const double v = R[r][cc];
    R[r][cc] = cc > r ? v * rs : (cc == r ? (rs == 0.0 ? 1.0 : v * rs) : 0.0);
    if (cc == r) rsv[r] = rs == 0.0 ? 1.0 : rs;
  }
  __syncthreads();
  // Inverse, blocked by 16: wave w inverts diagonal sub-block w, then the other
  // blocks follow by block diagonals, X_IJ = -X_II (sum_{L=I+1..J} R_IL X_LJ).
  // Block pair (I, I + d) of diagonal d is one wave's: the sum and the product
  // with X_II are 16 x 16 x 16 MFMA products (v_mfma_f64_16x16x4f64; entries past
  // nbk are zero in R and X, so whole blocks are summed).  The sum stays in the
  // wave's accumulators, whose register kk is the B operand of the product's k-step
  // kk, and the blocks a diagonal writes are not read within it.
  const int nsb = (nbk + SB - 1) / SB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < nsb) inv_sub(wave * SB, min(SB, nbk - wave * SB), R, Xs, rsv);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int d = 1; d < nsb; ++d) {
    const int I = wave, J = wave + d;
    if (J < nsb) {  // wave-uniform
      f64x4 m = f64x4{0, 0, 0, 0};
      for (int L = I + 1; L <= J; ++L)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          m = __builtin_amdgcn_mfma_f64_16x16x4f64(R[I * SB + lr][L * SB + 4 * kk + lk],
                                                   Xs[L * SB + 4 * kk + lk][J * SB + lr], m, 0, 0, 0);
      f64x4 x = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[I * SB + lr][I * SB + 4 * kk + lk], m[kk], x, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) Xs[I * SB + lk + 4 * r][J * SB + lr] = -x[r];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) {
    const int r = e / TB, c = e % TB;
    if (r < nbk && c < nbk) {
      as_global_w<double>(a.G)[(b0 + r) * a.ld + b0 + c] = (c >= r) ? R[r][c] : 0.0;
      put_x(a, b0 + r, b0 + c, (c >= r) ? Xs[r][c] : 0.0);
    }
  }
}

// B(kb, j): G_kb,j <- X_kk^T G_kb,j, rows of dependent columns cleared.
RF_DEV void task_panel(const CholInvArgs& a, int kb, int jb, double (*P)[TLD], double (*Q)[TLD]) {
  const int64_t b0 = (int64_t)kb * TB, c0 = (int64_t)jb * TB;
  load_tile(P, as_global<double>(a.X64), a.ldx64, b0, b0, a.N);
  load_tile(Q, as_global<double>(a.G), a.ld, b0, c0, a.N);
  __syncthreads();
  f64x4 acc[2][2];
  acc_zero(acc);
  tile_mac<true>(acc, P, Q);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = b0 + tile_row(i, q), c = c0 + tile_col(j);
        if (r < a.N && c < a.N) as_global_w<double>(a.G)[r * a.ld + c] = as_global<int>(a.flags)[r] ? 0.0 : acc[i][j][q];
      }
}

// X(kb, i): X_i,kb = -(sum_l X_il R_l,kb) X_kk ; the mirrored lower tile is cleared.
RF_DEV void task_xcol(const CholInvArgs& a, int kb, int ib, double (*P)[TLD], double (*Q)[TLD]) {
  const int64_t b0 = (int64_t)kb * TB, i0 = (int64_t)ib * TB;
  f64x4 acc[2][2];
  acc_zero(acc);
  for (int lb = ib; lb < kb; ++lb) {
    const int64_t l0 = (int64_t)lb * TB;
    __syncthreads();
    load_tile(P, as_global<double>(a.X64), a.ldx64, i0, l0, a.N);
    load_tile(Q, as_global<double>(a.G), a.ld, l0, b0, a.N);
    __syncthreads();
    tile_mac<false>(acc, P, Q);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) P[tile_row(i, q)][tile_col(j)] = acc[i][j][q];
  load_tile(Q, as_global<double>(a.X64), a.ldx64, b0, b0, a.N);
  __syncthreads();
  f64x4 o[2][2];
  acc_zero(o);
  tile_mac<false>(o, P, Q);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = tile_row(i, q), c = tile_col(j);
        put_x(a, i0 + r, b0 + c, -o[i][j][q]);
        put_x(a, b0 + c, i0 + r, 0.0);
      }
}

// X(kb, i) of the task queue: X_i,kb = -T_i,kb X_kk with T_i,kb complete in the X
// tile (i, kb); the mirrored lower tile is cleared.
RF_DEV void task_xfin(const CholInvArgs& a, int kb, int ib, double (*P)[TLD], double (*Q)[TLD]) {
  const int64_t b0 = (int64_t)kb * TB, i0 = (int64_t)ib * TB;
  load_tile(P, as_global<double>(a.X64), a.ldx64, i0, b0, a.N);
  load_tile(Q, as_global<double>(a.X64), a.ldx64, b0, b0, a.N);
  __syncthreads();
  f64x4 o[2][2];
  acc_zero(o);
  tile_mac<false>(o, P, Q);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = tile_row(i, q), c = tile_col(j);
        put_x(a, i0 + r, b0 + c, -o[i][j][q]);
        put_x(a, b0 + c, i0 + r, 0.0);
      }
}

// U(kb, i, j): T_ij += X_i,kb R_kb,j (i <= kb < j), held in the X tile (i, j); the
// first term (kb == i) writes it.
RF_DEV void task_tupd(const CholInvArgs& a, int kb, int ib, int jb, double (*P)[TLD], double (*Q)[TLD]) {
  const int64_t k0 = (int64_t)kb * TB, i0 = (int64_t)ib * TB, c0 = (int64_t)jb * TB;
  load_tile(P, as_global<double>(a.X64), a.ldx64, i0, k0, a.N);
  load_tile(Q, as_global<double>(a.G), a.ld, k0, c0, a.N);
  __syncthreads();
  f64x4 acc[2][2];
  acc_zero(acc);
  tile_mac<false>(acc, P, Q);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = i0 + tile_row(i, q), c = c0 + tile_col(j);
        if (r < a.N && c < a.N) {
          const gptr<double> t = as_global_w<double>(a.X64) + r * a.ldx64 + c;
          *t = (ib == kb) ? acc[i][j][q] : *t + acc[i][j][q];
        }
      }
}

// C(kb, i, j): G_ij -= R_kb,i^T R_kb,j (upper tiles).
RF_DEV void task_update(const CholInvArgs& a, int kb, int ib, int jb, double (*P)[TLD], double (*Q)[TLD]) {
  const int64_t b0 = (int64_t)kb * TB, r0 = (int64_t)ib * TB, c0 = (int64_t)jb * TB;
  load_tile(P, as_global<double>(a.G), a.ld, b0, r0, a.N);
  load_tile(Q, as_global<double>(a.G), a.ld, b0, c0, a.N);
  __syncthreads();
  f64x4 acc[2][2];
  acc_zero(acc);
  tile_mac<true>(acc, P, Q);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + tile_row(i, q), c = c0 + tile_col(j);
        if (r < a.N && c < a.N && c >= r) as_global_w<double>(a.G)[r * a.ld + c] -= acc[i][j][q];
      }
}

__global__ __launch_bounds__(256) void k_cholinv(CholInvArgs a) {
  if (a.run_if && *a.run_if == 0) return;
  extern __shared__ double sm[];
  double(*T0)[TLD] = reinterpret_cast<double(*)[TLD]>(sm);
  double(*T1)[TLD] = reinterpret_cast<double(*)[TLD]>(sm + TB * TLD);
  double(*T2)[TLD] = reinterpret_cast<double(*)[TLD]>(sm + 2 * TB * TLD);
  __shared__ int ticket;
  const int nb = a.nb;
  int* err = a.fault;
  int* gcnt = a.work + 2;        // nb x nb
  int* pdone = gcnt + nb * nb;   // nb x nb
  int* tcnt = pdone + nb * nb;   // nb x nb
  int* xdone = tcnt + nb * nb;   // nb x nb
  int total = 0;
  for (int kb = 0; kb < nb; ++kb) total += step_tasks(nb, kb);
  // Control flow around the barriers must be uniform: the ticket and the waits are
  // handled by wave 0 as a whole (a branch on the wave index, never on the lane),
  // and the ticket is read back as a wave-uniform value.
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  for (;;) {
    if (wave == 0) {
      const int old = __builtin_amdgcn_readfirstlane(atomicAdd(a.work, lane == 0 ? 1 : 0));
      ticket = old;  // every lane of wave 0 stores the same value
    }
    __syncthreads();
    int t = __builtin_amdgcn_readfirstlane(ticket);
    __syncthreads();
    if (t >= total) return;
    int kb = 0;
    for (;; ++kb) {
      const int sz = step_tasks(nb, kb);
      if (t < sz) break;
      t -= sz;
    }
    const int w = nb - 1 - kb;  // tiles right of the diagonal at step kb
    int* done;
    if (t == 0) {  // A(kb)
      if (wave == 0 && kb > 0) wait_at_least(&gcnt[kb * nb + kb], kb, err);
      __syncthreads();
      task_diag(a, kb, T0, T1, T2);
      done = &pdone[kb * nb + kb];
    } else if (t < nb) {  // B(kb, j) or X(kb, i)
      const int u = t - 1;  // 0 .. nb-2
      const bool panel = u < w;
      const int j = kb + 1 + u, i = u - w;
      if (wave == 0) {
        wait_at_least(&pdone[kb * nb + kb], 1, err);
        if (panel) {
          if (kb > 0) wait_at_least(&gcnt[kb * nb + j], kb, err);
        } else {
          wait_at_least(&tcnt[i * nb + kb], kb - i, err);
        }
      }
      __syncthreads();
      if (panel) task_panel(a, kb, j, T0, T1);
      else task_xfin(a, kb, i, T0, T1);
      done = panel ? &pdone[kb * nb + j] : &xdone[i * nb + kb];
    } else if (t < nb + nC_of(nb, kb)) {  // C(kb, i, j), kb < i <= j
      int u = t - nb, ib = kb + 1, ww = w;
      while (u >= ww) { u -= ww; ++ib; --ww; }
      const int jb = ib + u;
      if (wave == 0) {
        wait_at_least(&pdone[kb * nb + ib], 1, err);
        wait_at_least(&pdone[kb * nb + jb], 1, err);
        if (kb > 0) wait_at_least(&gcnt[ib * nb + jb], kb, err);
      }
      __syncthreads();
      task_update(a, kb, ib, jb, T0, T1);
      done = &gcnt[ib * nb + jb];
    } else {  // U(kb, i, j), i <= kb < j
      const int u = t - nb - nC_of(nb, kb), ib = u / w, jb = kb + 1 + u % w;
      if (wave == 0) {
        wait_at_least(ib == kb ? &pdone[kb * nb + kb] : &xdone[ib * nb + kb], 1, err);
        wait_at_least(&pdone[kb * nb + jb], 1, err);
        if (kb > ib) wait_at_least(&tcnt[ib * nb + jb], kb - ib, err);
      }
      __syncthreads();
      task_tupd(a, kb, ib, jb, T0, T1);
      done = &tcnt[ib * nb + jb];
    }
    __syncthreads();
    if (wave == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(done, lane == 0 ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void k_cholinv_prep(const double* __restrict__ G, int64_t ld, int64_t N, double* __restrict__ d0,
                               int* __restrict__ flags, int* count, const int* run_if, int* work, int nwork) {
  if (run_if && *run_if == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *count = 0;
  if (i < N) {
    d0[i] = G[i * ld + i];
    flags[i] = 0;
  }
  if (i < nwork) work[i] = 0;
}

// Batched: one workgroup per problem runs the same tasks in dependency order
// (no queue, no waits); for the small k of a batch of independent matrices.
__global__ __launch_bounds__(256) void k_cholinv_seq_batched(const CholInvArgs* __restrict__ as) {
  const CholInvArgs a = as[blockIdx.x];
  if (a.run_if && *a.run_if == 0) return;
  extern __shared__ double sm[];
  double(*T0)[TLD] = reinterpret_cast<double(*)[TLD]>(sm);
  double(*T1)[TLD] = reinterpret_cast<double(*)[TLD]>(sm + TB * TLD);
  double(*T2)[TLD] = reinterpret_cast<double(*)[TLD]>(sm + 2 * TB * TLD);
  for (int64_t i = threadIdx.x; i < a.N; i += blockDim.x) {
    const_cast<double*>(a.d0)[i] = a.G[i * a.ld + i];
    a.flags[i] = 0;
  }
  if (threadIdx.x == 0) *a.count = 0;
  __syncthreads();
  const int nb = a.nb;
  for (int kb = 0; kb < nb; ++kb) {
    task_diag(a, kb, T0, T1, T2);
    __syncthreads();
    for (int jb = kb + 1; jb < nb; ++jb) {
      task_panel(a, kb, jb, T0, T1);
      __syncthreads();
    }
    for (int ib = 0; ib < kb; ++ib) {
      task_xcol(a, kb, ib, T0, T1);
      __syncthreads();
    }
    for (int ib = kb + 1; ib < nb; ++ib)
      for (int jb = ib; jb < nb; ++jb) {
        task_update(a, kb, ib, jb, T0, T1);
        __syncthreads();
      }
  }
}

CholInvArgs cholinv_desc(double* G, int64_t ld, int64_t N, double tol_ratio, double* d0, int* flags, int* count,
                         int* nonfinite, const int* run_if, double* X64, int64_t ldx64, float* X32, int64_t ldx32) {
  CholInvArgs a;
  a.G = G; a.ld = ld; a.N = N;
  a.tol = tol_ratio; a.d0 = d0; a.flags = flags; a.count = count; a.nonfinite = nonfinite;
  a.run_if = run_if;
  a.X64 = X64; a.ldx64 = ldx64; a.X32 = X32; a.ldx32 = ldx32;
  a.work = nullptr; a.fault = nullptr; a.nb = (int)((N + TB - 1) / TB);
  return a;
}

hipError_t launch_cholinv_batched(const CholInvArgs* as, int count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  const size_t lds = 3 * (size_t)TB * TLD * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_cholinv_seq_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL(k_cholinv_seq_batched, dim3((unsigned)count), dim3(256), lds, st, as);
  return hipGetLastError();
}

size_t cholinv_work_ints(int64_t N) {
  const int64_t nb = (N + TB - 1) / TB;
  return (size_t)(2 + 4 * nb * nb);
}

static int cu_count_ci() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (n <= 0) n = 256;
  }
  return n;
}

hipError_t launch_cholinv(double* G, int64_t ld, int64_t N, double tol_ratio, double* d0, int* flags, int* count,
                          int* nonfinite, int* fault, const int* run_if, double* X64, int64_t ldx64, float* X32,
                          int64_t ldx32, int* work, hipStream_t st) {
  if (N == 0) return hipSuccess;
  const int nb = (int)((N + TB - 1) / TB);
  const int nwork = (int)cholinv_work_ints(N);
  const int64_t nprep = N > nwork ? N : nwork;
  hipLaunchKernelGGL(k_cholinv_prep, dim3((unsigned)((nprep + 255) / 256)), dim3(256), 0, st, G, ld, N, d0, flags,
                     count, run_if, work, nwork);
  CholInvArgs a;
  a.G = G; a.ld = ld; a.N = N;
  a.tol = tol_ratio; a.d0 = d0; a.flags = flags; a.count = count; a.nonfinite = nonfinite;
  a.run_if = run_if;
  a.X64 = X64; a.ldx64 = ldx64; a.X32 = X32; a.ldx32 = ldx32;
  a.work = work; a.fault = fault; a.nb = nb;
  int total = 0;
  for (int kb = 0; kb < nb; ++kb) total += host_step_tasks(nb, kb);
  int grid = cu_count_ci();
  if (grid > total) grid = total;
  const size_t lds = 3 * (size_t)TB * TLD * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_cholinv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  hipLaunchKernelGGL(k_cholinv, dim3((unsigned)grid), dim3(256), lds, st, a);
  return hipGetLastError();
}

}  // namespace rf
