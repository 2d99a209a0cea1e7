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
// Copy of a caller-given table with every entry outside its block replaced by the
// block's first column (sign kept); *bad += number of such entries.
hipError_t launch_table_sanitize(const int32_t* in, int64_t n, int s, int r1, int32_t* out, int* bad, hipStream_t st);

// ---- K3 / K4 ----
// Batched sketch tables (stream 0), ready tables and Omega (stream 1, r1 x k, ld k),
// problem index b in the Philox counter.  max_entries: max over problems of
// max(n s, r1 k / 4).
struct RngArgs {
  int64_t n; int s, r1, k, cpl; uint64_t seed; uint32_t b;
  int32_t* table; uint32_t* ready; float* om;
};
hipError_t launch_rng_batched(const RngArgs* as, int count, int64_t max_entries, hipStream_t st);
int sketch_right_cpl(int s);
bool sketch_right_fast_ok(int s);
// The single-problem ready table is written in the compact 16-bit form (and read by
// the two-workgroups-per-CU sketch kernel) when this holds.
bool sketch_right_ready16(int s, int r1);
// dtype: 0 f32, 2 bf16, 3 fp8 e4m3 with 128x128 block scales
// cmax: workspace of sketch_right_cmax_ints(n) ints (per-chunk bucket occupancy)
size_t sketch_right_cmax_ints(int64_t n);
// Batched A_i S_i for FP32 A_i with s = 4 nonzeros per column and r1 <= 1280
// (one problem per grid row): table/ready from the single-problem kernels with
// cpl = 2, cmax: sketch_right_cmax_ints(n_i) ints each.
struct SketchArgs {
  const float* A; int64_t lda;
  const int32_t* table; const uint32_t* ready; int* cmax;
  int64_t m, n; int r1; int vec_ok;
  float* out; int64_t ldo;
};
hipError_t launch_sketch_right_batched(const SketchArgs* as, int count, int64_t mmax, int64_t nmax, int r1max,
                                       hipStream_t st);
// Sketches without a fixed-point path (s other than 4, 8, 16; n <= 32768 and the
// bucket lists fit in LDS) run the atomic-free gather form; `cmax` is then its
// workspace.  Size `cmax` with sketch_right_work_ints, which covers both uses.
bool sketch_right_gather(int s, int64_t n, int r1);
size_t sketch_right_work_ints(int64_t n, int s, int r1);
hipError_t launch_sketch_right(int dtype, const void* A, int64_t lda, const float* scales, const int32_t* table,
                               const uint32_t* ready, int* cmax, int s, int64_t m, int64_t n, int r1, float* out,
                               int64_t ldo, hipStream_t st);
size_t sketch_left_partial_floats(int64_t M, int64_t N, int r1);
// work: sketch_left_work_ints(N, r1) ints (column maxima, column flags, bucket
// occupancy, bucket histogram) for the fixed-point pass; nullptr selects the LDS
// float-atomic pass.
size_t sketch_left_work_ints(int64_t N, int r1);
hipError_t launch_sketch_left(int dtype, const void* X, int64_t ldx, const int32_t* table, int s, int64_t M,
                              int64_t N, int r1, float* out, int64_t ldo, float* partial, hipStream_t st,
                              const float* scales = nullptr, int* work = nullptr);

// ---- sketch families of Lemma 3.2 items 1 and 3 (families.hip) ----
// kind 1: Rademacher +-1, kind 2: N(0,1) (stream 4), n x r1 row-major FP32, unscaled
hipError_t launch_dense_sketch(int kind, int64_t n, int r1, uint64_t seed, uint32_t b, float* out, hipStream_t st);
int64_t srht_size(int64_t n);  // smallest power of two >= n
bool srht_supported(int64_t n, int r1);  // n' <= 32768, r1 <= min(n', 8192)
// d: srht_size(n) floats (+-1), picks: r1 ints (ascending)
hipError_t launch_srht_prep(int64_t n, int r1, uint64_t seed, uint32_t b, float* d, int* picks, hipStream_t st);
// out (m x r1, ldo) = A D H I_{:,picks} / sqrt(r1); dtype 0 FP32, 2 BF16, 3 FP8 with 128x128 scales
hipError_t launch_srht_rows(int dtype, const void* A, int64_t lda, const float* scales, int64_t m, int64_t n,
                            const float* d, const int* picks, int r1, float* out, int64_t ldo, hipStream_t st);

// ---- sparse A in CSR form (csr.hip) ----
// out (m x r1, ldo) = A S / ... for CSR A (table as launch_sketch_right); *bad += invalid column indices
hipError_t launch_sketch_csr(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m, int64_t n,
                             int64_t nnz, const int32_t* table, int s, int r1, float* out, int64_t ldo, int* bad,
                             hipStream_t st);
bool sketch_csr_ok(int r1);  // one row's r1 64-bit accumulators fit in LDS
// CSC of A: colptr (n+1), cursor (n, scratch), csc_pos (nnz: CSR positions by column, in CSR order), row_of (nnz)
hipError_t launch_csc_build(const int64_t* row_ptr, const int32_t* col, int64_t m, int64_t n, int64_t nnz,
                            int64_t* colptr, unsigned long long* cursor, int32_t* csc_pos, int32_t* row_of,
                            hipStream_t st);
// out (n x k, ldo) = A^T Q for Q (m x k, ldq)
hipError_t launch_spmm_atq(const int64_t* colptr, const int32_t* csc_pos, const int32_t* row_of, const float* val,
                           int64_t n, const float* Q, int64_t ldq, int k, float* out, int64_t ldo, hipStream_t st);

// ---- storage forms of A (quant.hip) ----
// out (rows x cols, ldo) = BF16 of A (round to nearest even)
hipError_t launch_quant_bf16(const float* A, int64_t rows, int64_t cols, int64_t lda, uint16_t* out, int64_t ldo,
                             hipStream_t st);
// out = OCP e4m3 codes of A / scale(block), scales: ceil(rows/128) x ceil(cols/128)
// row-major FP32, scale = amax / 448 of the 128 x 128 block (1 if all zero)
hipError_t launch_quant_fp8_b128(const float* A, int64_t rows, int64_t cols, int64_t lda, uint8_t* out, int64_t ldo,
                                 float* scales, hipStream_t st);
// Q (m x k FP32) -> e4m3 codes in the B-operand order of the FP8 product (128-row
// stages x 32-column blocks of 4 KB) and E8M0 scales per 32 rows and column
// (128 bytes per stage and column block); layout in quant.hip.
int qf8_col_blocks(int64_t k);  // 32-column blocks, padded to a multiple of 8
size_t qf8_code_bytes(int64_t m, int64_t k);
size_t qf8_scale_bytes(int64_t m, int64_t k);
hipError_t launch_quant_q_fp8(const float* Q, int64_t m, int64_t k, int64_t ldq, uint8_t* codes, uint8_t* scales,
                              hipStream_t st);

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
  const float* a_scales;  // FP8 A only: 128 x 128 block scales of the stored A (k-block rows)
  int64_t a_ldsc;         //   scale of element (k, i) = a_scales[(k/128) * a_ldsc + i/128]
  int split_cap;          // > 0: at most this many split-K parts (the partial buffer's size)
  const uint8_t* b_scales;  // dtype 7 only: E8M0 scales of the Q operand form (B = its codes, ldb = column blocks)
};
// Tuning rule: dtype 0 (FP32) or 2 (BF16); applies when M <= max_m, N <= max_n,
// K <= max_k; tile 128 or 256 (BF16 only); split 0 (heuristic) or 1..16.
struct GemmRule { int32_t dtype, tile, split, reserved; int64_t max_m, max_n, max_k; };
int set_gemm_rules(const GemmRule* rules, int count);  // 0 ok, -1 invalid (table unchanged)
int gemm_splits(int64_t M, int64_t N, int64_t K);
size_t gemm_partial_floats(int64_t M, int64_t N, int64_t K);
// dtype: 0 FP32 operands, 2 BF16 operands, 4 FP32 A rounded to BF16 on load, 6 FP8
// block-scaled A dequantised to BF16 on load, 7 FP8 block-scaled A times the FP8 Q
// operand form (FP8 MFMA; a_kc = b_kc = 0).  partial may be NULL (no split-K).
hipError_t launch_gemm(GemmArgs g, int dtype, float* partial, hipStream_t st);
// Grouped products: count independent GemmArgs (device array, kps = K, partial = 0)
// in one grid; tile_start (device, count + 1 entries) is the prefix sum of
// gemm_group_tiles(kind, M_i, N_i).  kind: 0 FP32 (128 x 128 tiles), 2 BF16
// (128 x 128), 3 BF16 (256 x 256), 4 BF16 with A FP32 rounded on load (256 x 256),
// 5 BF16 with A FP32 rounded on load (128 x 128).
int gemm_group_tiles(int kind, int64_t M, int64_t N);
hipError_t launch_gemm_grouped(const GemmArgs* gs, const int* tile_start, int count, int total_tiles, int kind,
                               int a_kc, int b_kc, hipStream_t st);

// ---- FP64 small linear algebra ----
// C (M x N, FP64, ldc) = X^T Y with X (K x M), Y (K x N) row-major (xdt/ydt: 0 f32, 1 f64).
// sym: X == Y, M == N; only upper tiles computed, result mirrored.
size_t gram_partial_doubles(int64_t K, int64_t M, int64_t N);
hipError_t launch_gram(const void* X, int64_t ldx, int xdt, const void* Y, int64_t ldy, int ydt, int64_t K,
                       int64_t M, int64_t N, int sym, double* C, int64_t ldc, double* partial, const int* run_if,
                       hipStream_t st);
// ---- batched utilities (device descriptor arrays, one entry per problem) ----
struct CastArgs { const void* in; void* out; int64_t rows, cols, ldi, ldo; };
hipError_t launch_cast_batched(const CastArgs* as, int count, int64_t max_elems, int f64_to_f32, hipStream_t st);
// dependent columns of X replaced (stream 3, problem index b) when *count != 0
struct RefillArgs { float* X; int64_t ldx, rows, k; const int* flags; const int* count; const double* d0;
                    uint64_t seed; uint32_t b; };
hipError_t launch_refill_batched(const RefillArgs* as, int count, int64_t max_elems, hipStream_t st);
hipError_t launch_note_batched(int* const* cs, int count, int final_, hipStream_t st);
// Ritz tail: the "pre" launch writes sigma = sqrt(lam), inv = 1/sigma, Ub32 = Ub and
// clears the sign keys (signw: 3 k ints); after the U and V^T products the "sign"
// launches apply the sign rule (largest |U| entry of each column positive).
struct SvdTailArgs {
  const double* lam; const double* Ub; float* Ub32; double* sigma; float* inv; int* signw;
  float* U; int64_t ldu; float* Vt; int64_t ldvt; int64_t m, n, k;
};
hipError_t launch_svd_tail_pre_batched(const SvdTailArgs* as, int count, int64_t kmax, hipStream_t st);
hipError_t launch_svd_tail_sign_batched(const SvdTailArgs* as, int count, int64_t kmax, int64_t mmax,
                                        int64_t max_elems, hipStream_t st);
// rf_info of problem i from counters + i * stride (k_i from ks, device array).
hipError_t launch_info_batched(void* infos, const int* counters, int stride, const int* ks, int count, hipStream_t st);
// Grouped symmetric Grams: C_i (M_i x M_i FP64, ldc) = X_i^T X_i, X_i (K_i x M_i) FP32
// row-major; skipped when run_if is set and *run_if == 0.  tile_start: prefix sum
// of gram_group_tiles(M_i) (device, count + 1 entries).
struct GramArgs {
  const float* X; int64_t ldx; int64_t K, M;
  double* C; int64_t ldc;
  const int* run_if;
  double* partial;  // splits > 1: splits x M x M doubles of split-K parts (reduced in fixed order)
  int splits;       // parts of K (0 or 1: one)
  int64_t kps;      // rows of K per part
};
__host__ __device__ int gram_group_tiles(int64_t M);
int gram_group_splits(int64_t K);
// total_tiles counts (tile, part) items; max_mm = the largest M x M over the group.
hipError_t launch_gram_grouped(const GramArgs* gs, const int* tile_start, int count, int total_tiles, int64_t max_mm,
                               bool any_split, hipStream_t st);
// In-place upper Cholesky G = R^T R and X = R^{-1} (upper, lower triangle zeroed) in
// one persistent launch.  Pivots below tol_ratio * (original diagonal) are declared
// deficient: flags[c] = 1, row c of R set to e_c, *count += 1; d0 (N doubles)
// receives the original diagonal; *nonfinite = 1 on a non-finite pivot.  X64 (N x N,
// ldx64) is required, X32 optional.  work: device int[cholinv_work_ints(N)].
// *fault = 1 if a bounded wait between tasks gave up.
// Batched: one problem per workgroup (problems of a few 64-wide tiles); descriptors
// from cholinv_desc() in a device array.  Same outputs as launch_cholinv.
struct CholInvArgs {
  double* G; int64_t ld; int64_t N;
  double tol; const double* d0; int* flags; int* count; int* nonfinite;
  const int* run_if;
  double* X64; int64_t ldx64;   // R^{-1} in FP64 (required: later tasks read it)
  float* X32; int64_t ldx32;    // optional FP32 copy
  int* work;                    // [0] ticket, [1] unused, [2..2+nb) doneA, then doneP, doneX, doneC
  int* fault;                   // set to 1 when a bounded wait gives up
  int nb;
};
CholInvArgs cholinv_desc(double* G, int64_t ld, int64_t N, double tol_ratio, double* d0, int* flags, int* count,
                         int* nonfinite, const int* run_if, double* X64, int64_t ldx64, float* X32, int64_t ldx32);
hipError_t launch_cholinv_batched(const CholInvArgs* as, int count, hipStream_t st);
size_t cholinv_work_ints(int64_t N);
hipError_t launch_cholinv(double* G, int64_t ld, int64_t N, double tol_ratio, double* d0, int* flags, int* count,
                          int* nonfinite, int* fault, const int* run_if, double* X64, int64_t ldx64, float* X32,
                          int64_t ldx32, int* work, hipStream_t st);
// Block-Jacobi workspace view (carved from the caller's workspace by the library).
struct EigWork {
  double* Gp;      // K x K
  double* Gp2;     // K x K second buffer (single-problem solver; null for a batched problem)
  double* Z;       // K x K
  double* V;       // p x 64 x 64
  int* perm;       // K
  int* ident;      // p: subproblem x of the current round left its block pair unchanged
  unsigned long long* maxoff;  // 1
  int* conv;       // 1
  double* floor2;  // 1: (1e-15 ||G||_F)^2, regularises rotation thresholds
  double* npart;   // 64: partial sums of squares of G (single-problem solver)
  double* fabs_;   // 1: 16 eps ||G||_F, absolute convergence floor
  double tol;      // relative off-diagonal tolerance
  int64_t K;
  int p;
};

// One problem of a batched eigen-decomposition.
struct EigBatch {
  EigWork w;
  const double* G; int64_t ld; int64_t N;
  double* lam; double* V; int64_t ldv;
};
EigBatch eig_batch_desc(const double* G, int64_t ld, int64_t N, double* lam, double* V, int64_t ldv, void* work,
                        double tol);
hipError_t launch_eig_batched(const EigBatch* descs, int count, int64_t Nmax, hipStream_t st);
// Symmetric eigen-decomposition (block Jacobi).  G (N x N, ld) is destroyed.
// lam (N, descending), V (N x N, ldv, column c = eigenvector of lam[c]).
size_t eig_work_bytes(int64_t N, bool batched = false);
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
