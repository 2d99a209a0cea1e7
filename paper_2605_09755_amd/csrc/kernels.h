// Internal launcher declarations of the HIP kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rf {

// ---- K1 / K2 ----
hipError_t launch_sketch_table(int64_t n, int s, int r1, uint64_t seed, uint32_t stream, uint32_t b, int32_t* out,
                               hipStream_t st);
hipError_t launch_sketch_ready(const int32_t* table, int64_t n, int s, int r1, int cpl, uint32_t* ready,
                               hipStream_t st);
hipError_t launch_gaussian(int64_t rows, int64_t cols, uint64_t seed, uint32_t stream, uint32_t b, float* out,
                           int64_t ldo, hipStream_t st);

// ---- K3 / K4 ----
int sketch_right_cpl(int s);
bool sketch_right_fast_ok(int s);
// dtype: 0 f32, 2 bf16, 3 fp8 e4m3 with 128x128 block scales
// cmax: workspace of sketch_right_cmax_ints(n) ints (per-chunk bucket occupancy)
size_t sketch_right_cmax_ints(int64_t n);
hipError_t launch_sketch_right(int dtype, const void* A, int64_t lda, const float* scales, const int32_t* table,
                               const uint32_t* ready, int* cmax, int s, int64_t m, int64_t n, int r1, float* out,
                               int64_t ldo, hipStream_t st);
size_t sketch_left_partial_floats(int64_t M, int64_t N, int r1);
hipError_t launch_sketch_left(int dtype, const void* X, int64_t ldx, const int32_t* table, int s, int64_t M,
                              int64_t N, int r1, float* out, int64_t ldo, float* partial, hipStream_t st);

// ---- K5 / K6 ----
struct GemmArgs {
  const void* A; int64_t lda; int a_kc;  // a_kc: op(A)(i,k) = A[i*lda+k], else A[k*lda+i]
  const void* B; int64_t ldb; int b_kc;  // b_kc: op(B)(k,j) = B[j*ldb+k], else B[k*ldb+j]
  void* C; int64_t ldc; int c_trans; int c_bf16;
  int64_t M, N, K;
  float alpha;
  const float* colscale;  // optional per-column factor
  int b_upper;            // op(B)(k,j) == 0 for k > j (skip those k)
  int64_t kps;            // set by launcher
  float* partial;         // set by launcher
};
int gemm_splits(int64_t M, int64_t N, int64_t K);
size_t gemm_partial_floats(int64_t M, int64_t N, int64_t K);
// dtype: 0 FP32 operands, 2 BF16 operands.  partial may be NULL (no split-K).
hipError_t launch_gemm(GemmArgs g, int dtype, float* partial, hipStream_t st);

// ---- FP64 small linear algebra ----
// C (M x N, FP64, ldc) = X^T Y with X (K x M), Y (K x N) row-major (xdt/ydt: 0 f32, 1 f64).
// sym: X == Y, M == N; only upper tiles computed, result mirrored.
size_t gram_partial_doubles(int64_t K, int64_t M, int64_t N);
hipError_t launch_gram(const void* X, int64_t ldx, int xdt, const void* Y, int64_t ldy, int ydt, int64_t K,
                       int64_t M, int64_t N, int sym, double* C, int64_t ldc, double* partial, const int* run_if,
                       hipStream_t st);
// In-place upper Cholesky G = R^T R and X = R^{-1} (upper, lower triangle zeroed) in
// one persistent launch.  Pivots below tol_ratio * (original diagonal) are declared
// deficient: flags[c] = 1, row c of R set to e_c, *count += 1; d0 (N doubles)
// receives the original diagonal; *nonfinite = 1 on a non-finite pivot.  X64 (N x N,
// ldx64) is required, X32 optional.  work: device int[cholinv_work_ints(N)].
// *fault = 1 if a bounded wait between tasks gave up.
size_t cholinv_work_ints(int64_t N);
hipError_t launch_cholinv(double* G, int64_t ld, int64_t N, double tol_ratio, double* d0, int* flags, int* count,
                          int* nonfinite, int* fault, const int* run_if, double* X64, int64_t ldx64, float* X32,
                          int64_t ldx32, int* work, hipStream_t st);
// Symmetric eigen-decomposition (block Jacobi).  G (N x N, ld) is destroyed.
// lam (N, descending), V (N x N, ldv, column c = eigenvector of lam[c]).
size_t eig_work_bytes(int64_t N);
// trace (optional, device, >= eig_max_sweeps() doubles): per-sweep convergence measure
// (<= 1 means converged; 0 after convergence).
// Relative tolerance used for FP32 outputs (U, V, F): eigenvalue errors are second
// order in it and the computed V = B^T U Sigma^{-1} is orthonormal to about tol.
constexpr double kEigTolFP32 = 1e-7;
int eig_max_sweeps();
// tol: converged when every |g_ij| <= max(tol sqrt|g_ii g_jj|, 16 eps ||G||_F).
hipError_t launch_eig(double* G, int64_t ld, int64_t N, double* lam, double* V, int64_t ldv, void* work,
                      hipStream_t st, double tol, double* trace = nullptr);

// ---- utilities ----
hipError_t launch_cast_f32_bf16(const float* in, int64_t ldi, uint16_t* out, int64_t ldo, int64_t rows, int64_t cols,
                                hipStream_t st);
hipError_t launch_cast_f64_f32(const double* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                               hipStream_t st);
hipError_t launch_copy_f32(const float* in, int64_t ldi, float* out, int64_t ldo, int64_t rows, int64_t cols,
                           hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t st);
// Replace flagged columns of X (rows x k) by N(0,1) * sqrt(max d0)/sqrt(rows) fill (stream 3).
hipError_t launch_refill(float* X, int64_t ldx, int64_t rows, int64_t k, const int* flags, const int* count,
                         const double* d0, uint64_t seed, hipStream_t st);
// sigma = sqrt(max(lam,0)); inv32 = 1/sigma (0 if sigma == 0)
hipError_t launch_sigma(const double* lam, int64_t k, double* sigma, float* inv32, hipStream_t st);
// SVD sign convention on U (m x k) and Vt (k x n); work: 3k ints.
hipError_t launch_sign_fix(float* U, int64_t ldu, int64_t m, int64_t k, float* Vt, int64_t ldvt, int64_t n,
                           int* work, hipStream_t st);
// Nystrom F scaling: scale[c] = lam[c] > cut ? lam^{-1/2} : 0, cut = k*2^-52*lam_max.
hipError_t launch_nystrom_scale(const double* lam, int64_t k, float* scale, hipStream_t st);
// counters: [0] deficient count of the current factorisation, [1] passes that
// needed refill, [2] nonfinite, [3] final count, [4] refill flag of this pass.
hipError_t launch_note(int* counters, int final_, hipStream_t st);
// info finalisation: writes rf_info from counters.
hipError_t launch_info(void* info, const int* counters, int k, const double* orth, hipStream_t st);
// max |G - I| over an N x N FP64 matrix -> *out
hipError_t launch_orth_err(const double* G, int64_t ld, int64_t N, double* out, hipStream_t st);
hipError_t launch_symmetrize(float* X, int64_t ld, int64_t N, hipStream_t st);
hipError_t launch_symmetrize64(double* X, int64_t ld, int64_t N, hipStream_t st);
hipError_t launch_copy_f64(const double* in, int64_t ldi, double* out, int64_t ldo, int64_t rows, int64_t cols,
                           hipStream_t st);

}  // namespace rf
