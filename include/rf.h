/*
 * rf.h -- C ABI of the MI355X (gfx950) sketch-powered range finder.
 *
 * Implements the method of Chenakkod & Derezinski, "Accelerating Power Method
 * with Fast Sketching for Stronger Low-Rank Approximation" (arXiv 2605.09755):
 *
 *   Algorithm 1 (Sketch-Powered Range Finder, Section 2):
 *       Q = orth((At At^T)^q At Omega),   At = A S,
 *       S  n x r1 sparse sign sketch, s nonzeros +-1/sqrt(s) per row (Lemma 3.2(2)),
 *       Omega r1 x r2 Gaussian, r1 = sketch size l, r2 = target rank k (Section 4).
 *   Randomised SVD finisher (Section 2, "Sketch-Powered Low-Rank Factorization"):
 *       B = Q^T A = Ub Sigma V^T,  U = Q Ub.
 *   Algorithm 2 (Sketch-Powered Low-Rank Factorization):
 *       X = (S2^T Y)^+ (S2^T A),  S2 m x r1 second sparse sketch.
 *   Algorithm 3 (Sketch-Powered Nystrom Approximation, PSD A):
 *       Ct = A S, Wt = S^T A S, Y = Wt^q Omega, C = Ct Y, W = Y^T Wt Y.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are ROW-MAJOR.  Element (i, j) of a matrix with leading dimension
 *   ld is at offset i*ld + j.  ld >= cols.
 * - Every matrix pointer (A data, block scales, outputs, workspace, info) is a
 *   DEVICE pointer owned by the caller.  The library never allocates, frees or
 *   copies host memory, and never synchronises: calls only enqueue work on
 *   `stream` (a hipStream_t passed as void*; NULL = the null stream).
 * - Argument checking is synchronous: on any error status nothing has been
 *   enqueued.  RF_EINVAL: bad sizes / null pointers / inconsistent dtype.
 *   RF_EWORKSPACE: ws_bytes < rf_workspace_size(...).  RF_EUNSUPPORTED: valid
 *   request this build does not implement.  RF_EHIP: a HIP launch failed.
 * - Conditions found on the device (Cholesky breakdown handled by column
 *   refill, non-finite values) are written to *info (device memory, may be
 *   NULL) and are readable after the stream has been synchronised.
 * - Randomness: S, S2 and Omega are pure functions of (seed, stream id, matrix
 *   index b = 0) through Philox4x32-10 (Salmon et al., SC'11); stream ids:
 *   0 = S (S1), 1 = Omega, 2 = S2, 3 = refill vectors.
 * - Sizes: 1 <= k <= sketch <= min(m, n) (Theorem 2.1 / 2.3 hypotheses;
 *   sketch <= n for Nystrom, Theorem 2.5), q >= 0, 1 <= nnz_per_col <= sketch.
 */
#ifndef RF_H
#define RF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RF_OK = 0,
  RF_EINVAL = 1,
  RF_EWORKSPACE = 2,
  RF_EUNSUPPORTED = 3,
  RF_EHIP = 4
} rf_status;

/* storage type of A */
typedef enum {
  RF_F32 = 0,           /* float */
  RF_F64 = 1,           /* reserved (not accepted for A) */
  RF_BF16 = 2,          /* bfloat16 bits (uint16), round-to-nearest-even from FP32 */
  RF_FP8E4M3_B128 = 3   /* OCP e4m3 bytes with one FP32 scale per 128x128 block:
                           value(i,j) = fp8(i,j) * block_scales[(i/128)*ceil(cols/128) + j/128] */
} rf_dtype;

/* arithmetic form of the big products (A S, At Z, At^T Q, Q^T A) */
typedef enum {
  RF_PREC_FP32 = 0,     /* plain: FP32 operands on FP32 MFMA */
  RF_PREC_MIXED = 1     /* BF16 operands on BF16 MFMA, FP32 accumulate; the last
                           power product At Z stays FP32.  An FP32 A is rounded to
                           BF16 as Q^T A loads it, so sigma and V carry BF16
                           product error (~1e-3 relative) while the range of Q
                           (and U) does not.  FP8 A: in the mixed form Q^T A
                           runs on FP8 MFMA, A's codes and block scales as
                           stored and Q rounded to e4m3 with one power-of-two
                           scale per 32 rows and column (sigma and V then carry
                           e4m3 rounding of Q, ~2^-4 relative per element); in
                           the plain form A is dequantised and rounded to BF16
                           as it is loaded (BF16 MFMA, Q in BF16).  The sketch
                           passes dequantise FP8 A in FP32. */
} rf_precision;
/* In both forms the Gram matrices of CholeskyQR2, the Cholesky factors, the
   triangular inverses and the Rayleigh-Ritz eigenproblem are FP64. */

enum { RF_OP_RANGE_FINDER = 0, RF_OP_SVD = 1, RF_OP_LOWRANK = 2, RF_OP_NYSTROM = 3 };

/* flags */
#define RF_FLAG_ORTH_ERR 1u   /* compute info->orth_err = max |Q^T Q - I| (one extra FP64 Gram) */
#define RF_FLAG_CLASSICAL 2u  /* S = I_n: the classical range finder the paper compares against
                                 (Section 2, "Comparison with Classical Range Finder"; Section 4;
                                 Algorithm 2 with S1 = I in the additional experiments).  At = A,
                                 Omega is n x k, the power products read A itself; p->sketch then
                                 only sizes S2 in rf_lowrank (and must still satisfy k <= sketch
                                 <= min(m, n)).  FP32 A only (RF_EUNSUPPORTED otherwise); in the
                                 mixed form A is rounded to BF16 as the products load it and the
                                 last product At Z stays FP32.  Not accepted by rf_nystrom
                                 (RF_EUNSUPPORTED). */

/* Sketch family of S in Algorithm 1 (Lemma 3.2), in bits 2-3 of rf_params.flags
   (not with RF_FLAG_CLASSICAL; rf_nystrom and the batched path take the sparse
   sign sketch only, RF_EUNSUPPORTED otherwise):
   RF_SKETCH_SPARSE     item 2: s = nnz_per_col nonzeros +-1/sqrt(s) per row (default).
   RF_SKETCH_RADEMACHER item 1: dense, entries +-1/sqrt(r1) (sign = top bit of word x0
                        of Philox counter i*r1 + j, stream 4).
   RF_SKETCH_GAUSSIAN   item 1: dense, entries N(0,1)/sqrt(r1) (the Box-Muller
                        generator of rf_gaussian on stream 4, rounded to FP32).
   RF_SKETCH_SRHT       item 3: S = D H I_{:,P} / sqrt(r1) on n' = the smallest power of
                        two >= n (A padded with zero columns): D signs from stream 5,
                        H Sylvester-Hadamard (+-1), P = the images of 0..r1-1 under a
                        keyed 4-round Feistel permutation of [0, n') (round function
                        from stream 6, cycle walking), sorted.  n' <= 32768 and
                        r1 <= 8192 (RF_EUNSUPPORTED otherwise).
   The dense families run A S as a dense product: FP32 MFMA in the plain form, BF16
   MFMA (A and S rounded to BF16) in the mixed form or for BF16-stored A; FP8-stored
   A is RF_EUNSUPPORTED with them.  nnz_per_col is ignored by the dense families
   and the SRHT (it must still be valid).  rf_range_finder_ex takes a table only
   with RF_SKETCH_SPARSE (RF_EINVAL otherwise). */
#define RF_SKETCH_SPARSE 0u
#define RF_SKETCH_RADEMACHER (1u << 2)
#define RF_SKETCH_GAUSSIAN (2u << 2)
#define RF_SKETCH_SRHT (3u << 2)
#define RF_SKETCH_MASK (3u << 2)

typedef struct {
  const void* data;           /* device, row-major rows x cols, leading dim ld (elements) */
  const float* block_scales;  /* device; required iff dtype == RF_FP8E4M3_B128, else NULL */
  int64_t rows, cols, ld;
  int32_t dtype;              /* rf_dtype */
  int32_t reserved;           /* must be 0 */
} rf_matrix;

typedef struct {
  int32_t k;            /* target rank r2 (columns of Q) */
  int32_t sketch;       /* sketch size r1 = l */
  int32_t q;            /* power steps: 2q+1 products with At */
  int32_t nnz_per_col;  /* s: nonzeros per row of S (per column of A) */
  uint64_t seed;
  int32_t precision;    /* rf_precision */
  uint32_t flags;       /* RF_FLAG_* */
} rf_params;

typedef struct {
  int32_t status;       /* 0 = ok; bit 1 = Cholesky breakdown repaired; bit 2 = non-finite seen;
                           bit 4 = a device task queue gave up waiting (results invalid);
                           bit 8 = a caller-given sketch table had entries outside their
                           block (rf_range_finder_ex; results are not Algorithm 1's);
                           bit 16 = a CSR matrix had column indices outside [0, cols),
                           which were skipped (rf_*_csr) */
  int32_t rank_found;   /* k minus columns refilled during orthonormalisation (last call) */
  int32_t chol_retries; /* number of CholeskyQR passes that needed column refill */
  int32_t nonfinite;    /* 1 if a NaN/Inf was seen in a Gram matrix */
  double orth_err;      /* max |Q^T Q - I| if RF_FLAG_ORTH_ERR, else -1 */
} rf_info;

/* Bytes of device workspace op (RF_OP_*) needs for A and p; 0 if the arguments
   are invalid.  Workspace must be 256-byte aligned. */
size_t rf_workspace_size(int op, const rf_matrix* A, const rf_params* p);

/* Algorithm 1.  Q: m x k FP32 (ldq >= k), orthonormal columns spanning
   (At At^T)^q At Omega, computed by subspace iteration with CholeskyQR
   re-orthonormalisation (exact-arithmetic span unchanged, remark after
   Algorithm 1) and a final CholeskyQR2. */
rf_status rf_range_finder(const rf_matrix* A, const rf_params* p, float* Q, int64_t ldq,
                          void* ws, size_t ws_bytes, rf_info* info, void* stream);

/* Algorithm 1 with caller-given random inputs (its inputs S and Omega, Section 2).
   S_table: device int32[n * s] in the layout rf_sketch_table writes (entry j*s + t =
   bucket | negative << 31, bucket inside block t = [floor(t r1/s), floor((t+1) r1/s)),
   value +-1/sqrt(s)), or NULL to draw S from p->seed; must be NULL with
   RF_FLAG_CLASSICAL (RF_EINVAL otherwise).  Entries outside their block are
   replaced by the block's first column and reported in info->status bit 8 (the
   call stays in bounds, the result is then not the requested sketch's).
   Omega: device FP32 rows x k, row-major with ld = k (rows = r1 = p->sketch, or n
   with RF_FLAG_CLASSICAL), or NULL to draw it from p->seed.  Both are read only,
   in stream order, and must stay alive until the call's work has run.  Otherwise
   as rf_range_finder (same workspace size). */
rf_status rf_range_finder_ex(const rf_matrix* A, const int32_t* S_table, const float* Omega, const rf_params* p,
                             float* Q, int64_t ldq, void* ws, size_t ws_bytes, rf_info* info, void* stream);

/* Randomised SVD on top of Algorithm 1 (Section 2; Section 4 uses r2 = k):
   U m x k FP32, sigma k FP64 descending, Vt k x n FP32 with A ~= U diag(sigma) Vt
   = Q Q^T A.  Sign convention: the largest-magnitude entry of each column of U
   is positive (lowest row index on ties). */
rf_status rf_svd(const rf_matrix* A, const rf_params* p, float* U, int64_t ldu, double* sigma,
                 float* Vt, int64_t ldvt, void* ws, size_t ws_bytes, rf_info* info, void* stream);

/* Algorithm 2.  Y m x k FP32 is returned orthonormalised (Y X is invariant
   under Y -> Y M), X k x n FP32 = (S2^T Y)^+ (S2^T A) by FP64 normal equations
   (S2^T Y is a well-conditioned sketch of an orthonormal basis). */
rf_status rf_lowrank(const rf_matrix* A, const rf_params* p, float* Y, int64_t ldy, float* X,
                     int64_t ldx, void* ws, size_t ws_bytes, rf_info* info, void* stream);

/* Algorithm 3 for square PSD A (n x n).  C n x k FP32, W k x k FP64 (symmetric),
   F n x k FP32 optional (NULL to skip): F = C V+ Lambda+^{-1/2} from the
   eigenpairs of W with eigenvalues > k * 2^-52 * lambda_max, so that
   C W^+ C^T = F F^T (dropped columns are zero).  For q >= 1 the power iterate
   Y is re-orthonormalised after every product with Wt.  RF_PREC_MIXED: the
   first q-1 products Wt Y on BF16 MFMA (FP32 accumulation), the last one and
   C = Ct Y in FP32; Grams, Cholesky, W and its eigenpairs FP64 in both forms. */
rf_status rf_nystrom(const rf_matrix* A, const rf_params* p, float* C, int64_t ldc, double* W,
                     int64_t ldw, float* F, int64_t ldf, void* ws, size_t ws_bytes,
                     rf_info* info, void* stream);

/* ---- sparse A (CSR) ------------------------------------------------------
   The paper states every cost in nnz(A) (Theorems 2.1, 2.3 and 2.5): the sketch
   At = A S touches each nonzero s times and the power loop runs on the dense
   m x r1 At.  A CSR matrix: row_ptr (device int64[rows + 1], row_ptr[0] = 0,
   nondecreasing, row_ptr[rows] = nnz), col_idx (device int32[nnz], in [0, cols)),
   values (device FP32[nnz]); nnz < 2^31.  Entries are read as stored: row
   pointers are clamped to [0, nnz], column indices outside [0, cols) are skipped
   and reported in info->status bit 16 (rf_sketch_apply_csr: not reported).

   rf_range_finder_csr / rf_svd_csr: as rf_range_finder / rf_svd (outputs, sign
   convention, precision forms, workspace from rf_workspace_size_csr with
   RF_OP_RANGE_FINDER / RF_OP_SVD) with the sparse sign sketch only: the sketch
   pass accumulates each row's r1 outputs exactly in 64-bit fixed point (grid
   2^F with nnz_row * max|a| * 2^F < 2^62, so each term is rounded to at most
   2^-(61 - log2 nnz_row) of the row's largest |a|; the sums do not depend on the
   order of the additions); a row holding a non-finite value gives a NaN row.
   B^T = A^T Q is a sparse product over a CSC copy of A built on the device (each
   column in CSR order, FP32 in both forms).  RF_EUNSUPPORTED for RF_FLAG_CLASSICAL,
   a dense sketch family, or a sketch too large for one row's accumulators in LDS
   (r1 > 20480).  rf_sketch_apply_csr: At = A S alone (the parity hook; p->flags
   must be 0), ws >= 4 cols nnz_per_col + 768 bytes. */
typedef struct {
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const float* values;
  int64_t rows, cols, nnz;
} rf_csr;
size_t rf_workspace_size_csr(int op, const rf_csr* A, const rf_params* p);
rf_status rf_range_finder_csr(const rf_csr* A, const rf_params* p, float* Q, int64_t ldq, void* ws, size_t ws_bytes,
                              rf_info* info, void* stream);
rf_status rf_svd_csr(const rf_csr* A, const rf_params* p, float* U, int64_t ldu, double* sigma, float* Vt,
                     int64_t ldvt, void* ws, size_t ws_bytes, rf_info* info, void* stream);
rf_status rf_sketch_apply_csr(const rf_csr* A, const rf_params* p, float* out, int64_t ldo, void* ws, size_t ws_bytes,
                              void* stream);

/* ---- storage forms of A (the precision workload: A stored once in BF16 and
   once in FP8-e4m3 with per-128x128-block scales) -------------------------------

   The paper fixes no storage format.  rf_quantize_bf16: out (rows x cols, ldo >=
   cols, device uint16 BF16 bits) = A rounded to nearest, ties to even (NaN stays
   NaN).  rf_quantize_fp8_b128: out (rows x cols, ldo >= cols, device uint8 OCP
   e4m3 codes) and scales (device FP32, ceil(rows/128) x ceil(cols/128) row-major,
   the block_scales of an RF_FP8E4M3_B128 rf_matrix): scale = amax/448 of the
   block's finite entries, computed in FP64 and rounded to FP32 (1 for an all-zero
   block); code = the e4m3 value nearest to a / scale (FP64 division), ties to the
   even code, saturating at +-448; non-finite entries encode as NaN (0x7f/0xff).
   A: device FP32, lda >= cols.  One pass over A each.  RF_EINVAL for bad sizes
   or null pointers; rf_quantize_fp8_b128 returns RF_EUNSUPPORTED for more than
   65535 row blocks. */
rf_status rf_quantize_bf16(const float* A, int64_t rows, int64_t cols, int64_t lda, uint16_t* out, int64_t ldo,
                           void* stream);
rf_status rf_quantize_fp8_b128(const float* A, int64_t rows, int64_t cols, int64_t lda, uint8_t* out, int64_t ldo,
                               float* scales, void* stream);

/* ---- tuning table for the dense products ---------------------------------

   A product with operands of dtype (0 = FP32, 2 = BF16) and shape M x N x K
   takes the first rule with matching dtype and M <= max_m, N <= max_n,
   K <= max_k: tile = 128 or 256 (workgroup tile edge; 256 only for BF16),
   split = 0 (built-in heuristic) or 1..16 (split-K factor, further capped so
   each split keeps >= 256 values of K).  Without a matching rule the built-in
   heuristics apply.  Products whose A is FP32 or FP8 rounded to BF16 on load
   (the mixed-precision Q^T A) take the split of the BF16 rule for their shape
   when that rule picks the 256 tile.  The rules are copied; count = 0 clears them.  The table
   is process-wide: set it before other calls (it is read on every launch and
   must not change while a call is enqueuing).  Returns RF_EINVAL (table
   unchanged) for a malformed rule or count > 256.  Written by the autotuner
   (paper_2605_09755_amd/autotune.py) as JSON; the Python binding loads the
   table it finds next to the library. */
typedef struct {
  int32_t dtype, tile, split, reserved;
  int64_t max_m, max_n, max_k;
} rf_gemm_rule;
rf_status rf_set_gemm_rules(const rf_gemm_rule* rules, int32_t count);

/* ---- batched randomised SVD (many independent matrices, one stream) -------

   count problems: As[i] (FP32, device), ps[i] with nnz_per_col = 4, the same q
   and precision for every i, k <= 1024, sketch <= 1280; shapes and ranks may
   differ.  Problem i uses seed ps[i].seed with matrix index i in the Philox
   counter (a single rf_svd call uses index 0), so problem 0 of a batch gives the
   same sketch and Omega as rf_svd on the same matrix and seed.  Outputs as for
   rf_svd: U[i] (m_i x k_i, ldu[i]), sigma[i] (k_i), Vt[i] (k_i x n_i, ldvt[i]);
   info: device array of count rf_info (or NULL).  Host arrays As, ps, U, ldu,
   sigma, Vt, ldvt are read during the plan call only.

   The plan call validates synchronously (RF_EINVAL, RF_EWORKSPACE, and
   RF_EUNSUPPORTED for what is outside the limits above), lays out the
   workspace (ws >= rf_svd_batched_ws(count, As, ps) bytes, device, owned by the
   caller and kept alive and untouched while the plan is used), writes the
   per-stage work lists into its head and waits for that upload on `stream`.
   With use_graph != 0 the launch sequence is captured into a hipGraph (no
   work runs during the plan call).  rf_svd_batched_run enqueues one batched
   factorisation on `stream` (a graph launch when captured); runs on one plan
   must not overlap.  Every stage is one grouped launch over all problems. */
typedef struct rf_batch_plan rf_batch_plan;
size_t rf_svd_batched_ws(int32_t count, const rf_matrix* As, const rf_params* ps);
rf_status rf_svd_batched_plan(int32_t count, const rf_matrix* As, const rf_params* ps, float* const* U,
                              const int64_t* ldu, double* const* sigma, float* const* Vt, const int64_t* ldvt,
                              rf_info* info, void* ws, size_t ws_bytes, int32_t use_graph, void* stream,
                              rf_batch_plan** plan);
rf_status rf_svd_batched_run(rf_batch_plan* plan, void* stream);
void rf_svd_batched_destroy(rf_batch_plan* plan);

/* ---- parity hooks (same kernels as the entry points above) ---------------- */

/* Sketch table: out[j*s + t] = bucket | (negative << 31) for j < n, t < s, with
   bucket in block t = [floor(t*r1/s), floor((t+1)*r1/s)).  out: device int32[n*s]. */
rf_status rf_sketch_table(int64_t n, int32_t s, int32_t r1, uint64_t seed, uint32_t stream_id,
                          uint32_t b, int32_t* out, void* stream);

/* Gaussian fill: out (rows x cols, row-major, device float) with entry e
   from Philox counter e/4 via Box-Muller in FP64, rounded to FP32. */
rf_status rf_gaussian(int64_t rows, int64_t cols, uint64_t seed, uint32_t stream_id, uint32_t b,
                      float* out, void* stream);

/* At = A S for the sketch given by (s = p->nnz_per_col, r1 = p->sketch, seed,
   stream id 0, and the family in p->flags, RF_SKETCH_*): out m x r1 FP32
   (ldo >= r1).  Any r1 >= s is accepted (p->k, p->q ignored; p->precision picks
   the product form of the dense families).  ws >= rf_sketch_apply_ws(A, p) bytes.
   The sparse sign sketch is deterministic: fixed-point sums for s = 4, 8, 16 with
   at most 640 buckets per block, otherwise (any s) fixed-order FP32 sums per
   output over its columns in ascending order (gather form) when n <= 32768; only
   wider A with such sketches falls back to float atomics (order-dependent). */
size_t rf_sketch_apply_ws(const rf_matrix* A, const rf_params* p);
rf_status rf_sketch_apply(const rf_matrix* A, const rf_params* p, float* out, int64_t ldo,
                          void* ws, size_t ws_bytes, void* stream);

/* Allocation-free form of rf_sketch_apply, for callers that cannot allocate
   device memory (code under stream capture, tight serving loops, harnesses that
   forbid allocation): same arguments and same result bits, no workspace.  The
   sketch table, its kernel-ready form and the per-chunk occupancy (or, for s
   other than 4, 8, 16, the bucket lists of the gather form) live in a
   library-owned device array of 8 MiB per GPU, held until the process ends.
   Limit: 8 n s + 4 max(n/1024 + 16, 1.5 n s + 2 r1 + 10) bytes, each of the
   three parts rounded up to 256, must fit in 8 MiB (e.g. n = 65536 with s = 8,
   n = 32768 with s = 1); larger requests return RF_EUNSUPPORTED with nothing
   enqueued.  Every call on a
   GPU shares that GPU's array: calls that overlap on one GPU (other streams,
   other threads) race and must be serialised by the caller.  No hipMalloc, no
   synchronisation; RF_EINVAL as rf_sketch_apply, RF_EHIP if the array's device
   address cannot be looked up. */
rf_status rf_sketch_apply_noalloc(const rf_matrix* A, const rf_params* p, float* out, int64_t ldo, void* stream);

/* T = S2^T A, the left sketch of Algorithm 2 (line 2) as rf_lowrank applies it:
   S2 is m x r1 (r1 = p->sketch) with s = p->nnz_per_col entries +-1/sqrt(s) per row,
   drawn from (seed, stream id 2); out r1 x n FP32 row-major (ldo >= n).  Any
   1 <= s <= r1 (p->k, p->q ignored).  Fixed point per output column: every term is
   rounded to 2^(e-30) with 2^e > c max_i |a_ij| (c the largest bucket occupancy);
   a column holding a non-finite value comes out NaN.  ws >= rf_sketch_apply_left_ws
   bytes; RF_EINVAL / RF_EWORKSPACE as the entry points above. */
size_t rf_sketch_apply_left_ws(const rf_matrix* A, const rf_params* p);
rf_status rf_sketch_apply_left(const rf_matrix* A, const rf_params* p, float* out, int64_t ldo,
                               void* ws, size_t ws_bytes, void* stream);

/* Kernel-level hooks used by the parity tests (same kernels as above).
   rf_test_gemm: C (M x N FP32, ldc) = op(A) op(B); dtype 0 = FP32 operands,
     2 = BF16 operands (uint16 bits), 4 = A FP32 rounded to BF16 (RNE) as it is
     loaded with B BF16 (BF16 MFMA, FP32 accumulation); a_kc != 0: op(A)(i,k) = A[i*lda+k] else
     A[k*lda+i]; b_kc != 0: op(B)(k,j) = B[j*ldb+k] else B[k*ldb+j];
     b_upper != 0 promises op(B)(k,j) = 0 for k > j.  ws: >= rf_test_gemm_ws(M,N,K)
     bytes (split-K partials), may be NULL to disable split-K.
   rf_test_gram: C (M x N FP64) = X^T Y, X (K x M) and Y (K x N) row-major FP32;
     sym != 0 requires X == Y.  ws >= rf_test_gram_ws(K,M,N) bytes or NULL.
   rf_test_cholqr_factor: in place upper Cholesky of G (N x N FP64, ld N) and
     Rinv (N x N FP64, ld N) = R^{-1}; counters: device int32[16] ([0] = number
     of pivots declared dependent).  ws >= rf_test_chol_ws(N) bytes.
   rf_test_eig: eigenpairs of symmetric G (N x N FP64, ld N, preserved): lam
     (N, descending), V (N x N, ld N), block Jacobi stopped when every
     |g_ij| <= max(tol sqrt|g_ii g_jj|, 16 eps ||G||_F) (rf_svd and rf_nystrom
     use tol = 1e-7); sweep_trace (device double[32] or NULL) receives the
     per-sweep value of max |g_ij| / max(...) (converged when <= 1; 0 once
     converged).  ws >= rf_test_eig_ws(N) bytes; N <= 4096. */
size_t rf_test_gemm_ws(int64_t M, int64_t N, int64_t K);
rf_status rf_test_gemm(int dtype, int a_kc, int b_kc, const void* A, int64_t lda, const void* B, int64_t ldb,
                       float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, int b_upper, void* ws,
                       void* stream);
/* rf_test_gemm_fp8a: C (M x N FP32, ldc) = op(A) op(B) with A OCP e4m3 bytes stored
   K x M row-major (lda >= M; op(A)(i,k) = A[k*lda+i] * scales[(k/128)*ceil(M/128) + i/128],
   the block-scaled form of rf_dtype RF_FP8E4M3_B128), rounded to BF16 as it is
   loaded, and B BF16 (b_kc as in rf_test_gemm); BF16 MFMA, FP32 accumulation. */
rf_status rf_test_gemm_fp8a(const uint8_t* A, int64_t lda, const float* scales, const uint16_t* B, int64_t ldb,
                            int b_kc, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* stream);
/* rf_test_quant_q_fp8: the FP8 operand form of Q (m x k FP32, ldq) that the FP8
   product A^T Q reads: e4m3 codes (rf_test_qf8_bytes(m, k, 0) bytes) and E8M0
   scales (rf_test_qf8_bytes(m, k, 1) bytes), device buffers.  With
   njb = 8 ceil(k / 256): codes[((((st*njb + jb)*2 + ch)*2 + p)*64 + lane)*16 + e]
   = code of Q[128 st + 64 ch + 32 p + 16 (lane/32) + e][32 jb + lane%32] and
   scales[((st*njb + jb)*64 + lane)*2 + ch] = E8M0 byte (127 + x for 2^x) of rows
   128 st + 64 ch + 32 (lane/32) + [0, 32) of column 32 jb + lane%32: the smallest
   2^x, -127 <= x <= 127, with 448 2^x >= the block's largest finite |q|; codes =
   nearest e4m3 of q 2^-x, ties to even, saturating; non-finite q -> NaN code;
   rows >= m and columns >= k -> code 0 (their blocks scale 2^-127).
   rf_test_gemm_fp8: C (M x N FP32, ldc) = op(A) Q with A as in rf_test_gemm_fp8a
   (e4m3 K x M row-major, 128 x 128 FP32 block scales) and Q (K x N) given in the
   FP8 operand form above (q_codes, q_scales from rf_test_quant_q_fp8 with m = K,
   k = N); both on FP8 MFMA, FP32 accumulation.  ws: >= rf_test_gemm_fp8_ws(M, N, K)
   bytes (split-K partials) or NULL (no split-K). */
size_t rf_test_qf8_bytes(int64_t m, int64_t k, int which);
rf_status rf_test_quant_q_fp8(const float* Q, int64_t m, int64_t k, int64_t ldq, uint8_t* codes, uint8_t* scales,
                              void* stream);
size_t rf_test_gemm_fp8_ws(int64_t M, int64_t N, int64_t K);
rf_status rf_test_gemm_fp8(const uint8_t* A, int64_t lda, const float* scales, const uint8_t* q_codes,
                           const uint8_t* q_scales, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws,
                           size_t ws_bytes, void* stream);
size_t rf_test_gram_ws(int64_t K, int64_t M, int64_t N);
rf_status rf_test_gram(const float* X, const float* Y, int64_t K, int64_t M, int64_t N, int sym, double* C,
                       void* ws, void* stream);
size_t rf_test_chol_ws(int64_t N);
rf_status rf_test_cholqr_factor(double* G, int64_t N, double* Rinv, int32_t* counters, void* ws, void* stream);
size_t rf_test_eig_ws(int64_t N);
rf_status rf_test_eig(const double* G, int64_t N, double tol, double* lam, double* V, double* sweep_trace,
                      void* ws, void* stream);

const char* rf_status_string(rf_status s);

#ifdef __cplusplus
}
#endif
#endif /* RF_H */
