/*
 * sbmm.h — C ABI of libsbmm: randomized block matrix multiplication by
 * sampling on AMD Instinct MI355X (gfx950).
 *
 * Method: Niu & Li, "Optimal Sampling Algorithms for Block Matrix
 * Multiplication" (arXiv 2105.04940). The product MN = sum_k M^k N_k over a
 * partition of the inner dimension into K blocks (eq. 2.3) is estimated by
 * drawing terms with replacement, rescaling each drawn term by 1/sqrt(c p)
 * on both factors (Alg. 1), concatenating the drawn columns of M into C and
 * rows of N into D, and forming CD (Alg. 2, eqs. 3.2-3.3).
 *
 * Two sampling modes share the entry points:
 *   SBMM_MODE_BLOCK       the drawn unit is a whole block; c i.i.d. draws with
 *                         block probabilities (1.4) "norm", (1.2) "exact",
 *                         uniform, or user weights.
 *   SBMM_MODE_STRATIFIED  the paper's Alg. 2: each block is a stratum, the
 *                         drawn unit is one inner index (a column of M and the
 *                         matching row of N), block k receives c_k draws with
 *                         probabilities (3.8) "norm" or 1/n_k "uniform"; c_k
 *                         comes from c/K "uniform", (4.2) "norm", (3.9) "opt",
 *                         the caller, or "two-step" (4.7): the two-step
 *                         Alg. 3, whose block sizes use a pilot sketch
 *                         (sbmm_pilot) in place of ||M^k N_k||_F.
 * An "atom" is the drawn unit (a block, or one inner index); a "stratum" is a
 * group of atoms with its own draw count (the whole problem in block mode,
 * one block in stratified mode).
 *
 * Sampling is bit-reproducible: weights are quantized per stratum to uint64
 * integers W (W = ceil(w * 2^(B-1-e)), e = floor(log2 max w), B = 63 -
 * ceil(log2 A_s) for the A_s atoms of the stratum), the per-stratum CDF is an
 * exact integer running sum with total T, draw j of stratum s reads the
 * Philox4x64-10 stream with counter (j, s, trial, (1 << 32) | block) and key
 * (seed, 0), pairs the words into 128-bit words (first word high), maps them
 * with Lemire's multiply-and-reject to an exactly uniform integer in [0, T),
 * and takes the first atom whose CDF exceeds it. The rescale uses
 * p_hat = W / T, the probability actually sampled.
 *
 * Layout: every matrix is row-major with a leading dimension (elements
 * between consecutive rows). M is m x n (ldm >= n), N is n x p (ldn >= p),
 * C is m x L (ldc >= L), D is L x p (ldd >= p), CD and MN are m x p.
 *
 * Ownership: every data pointer is caller-owned device memory unless marked
 * "host". The library keeps no pointer after a call returns except through
 * work it has enqueued on the given stream; the caller keeps buffers alive
 * until that work completes. The handle owns a device workspace that grows
 * on demand (sbmm_reserve pre-sizes it) and a device status word.
 *
 * Errors: every call returns an sbmm_status and never aborts, exits or
 * throws across the ABI. Arguments are checked on the host before anything
 * is launched. Conditions only the device can see (non-finite inputs or
 * weights, a budget below the number of strata that can be sampled) set the
 * handle's status word; the next synchronizing call (sbmm_plan with a
 * non-NULL L_host, sbmm_sync, sbmm_run) reports it and clears it. HIP errors
 * map to SBMM_E_HIP with the HIP text in sbmm_last_error().
 *
 * Streams and threads: calls are asynchronous on the given stream unless
 * documented as synchronizing. Use one handle per host thread. Calls on one
 * handle share its workspace and its device copy of the last partition: work
 * enqueued through one handle on different streams must not overlap (order
 * the streams, or use one handle per stream).
 */
#ifndef SBMM_H
#define SBMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbmm_handle_s* sbmm_handle;
typedef void* sbmm_stream; /* a hipStream_t; NULL is the default stream */

typedef enum {
  SBMM_OK = 0,
  SBMM_E_ARG = 1,         /* invalid argument (shape, pointer, alignment, partition, enum) */
  SBMM_E_BUDGET = 2,      /* c too small for the strata that can be sampled */
  SBMM_E_NONFINITE = 3,   /* NaN/Inf in the inputs or weights */
  SBMM_E_UNSUPPORTED = 4, /* valid request this build does not implement */
  SBMM_E_NOMEM = 5,       /* device allocation failed */
  SBMM_E_HIP = 6,         /* HIP runtime error; text in sbmm_last_error() */
  SBMM_E_STATE = 7        /* handle used on the wrong device / after destroy */
} sbmm_status;

typedef enum { SBMM_F64 = 0, SBMM_F32 = 1, SBMM_BF16 = 2, SBMM_F8E4M3 = 3 } sbmm_dtype;
typedef enum { SBMM_MODE_BLOCK = 0, SBMM_MODE_STRATIFIED = 1 } sbmm_mode;
typedef enum { SBMM_P_UNIFORM = 0, SBMM_P_NORM = 1, SBMM_P_EXACT = 2, SBMM_P_USER = 3 } sbmm_prob;
typedef enum {
  SBMM_ALLOC_UNIFORM = 0,
  SBMM_ALLOC_NORM = 1,
  SBMM_ALLOC_OPT = 2,
  SBMM_ALLOC_USER = 3,
  SBMM_ALLOC_TWO_STEP = 4
} sbmm_alloc;

/* One sampling problem (Alg. 2 input: M, N, the block sizes n_k, c, the
 * probability rule and, in stratified mode, the block-size rule). */
typedef struct {
  int64_t m, n, p;            /* M is m x n, N is n x p; n >= 1, m, p >= 0 */
  sbmm_dtype in_dtype;        /* dtype of M and N: F64, F32 or BF16 */
  const void* M; int64_t ldm; /* device, row-major, ldm >= n */
  const void* N; int64_t ldn; /* device, row-major, ldn >= p */
  int32_t K;                  /* number of blocks, >= 1 */
  const int64_t* block_off;   /* host, K+1 offsets: 0 = off[0] < ... < off[K] = n */
  int64_t c;                  /* total number of draws, >= 1 */
  sbmm_mode mode;
  sbmm_prob prob;             /* EXACT: block mode only (equals NORM for unit atoms) */
  sbmm_alloc alloc;           /* stratified mode only */
  const double* user_w;       /* device, one weight per atom (K block / n stratified), prob == USER */
  const int64_t* user_ck;     /* host, K draw counts summing to c, alloc == USER */
  const double* blkprod_sq;   /* device, K values ||M^k N_k||_F^2 (from sbmm_exact), prob == EXACT or alloc == OPT */
  uint64_t seed, trial;       /* Philox key word 0 and counter word 2 */
  /* two-step algorithm (Alg. 3), alloc == TWO_STEP only: */
  int64_t c0;                 /* pilot draws; every block that can be sampled gets [c0 / K] (so c0 >= K) */
  sbmm_prob pilot_prob;       /* pilot probabilities p_{0k_i}: UNIFORM (1/n_k, method ONU) or NORM ((3.8), ONMCNR) */
  const double* pilot_sq;     /* device, K pilot estimates ||C^{0k} D_{0k}||_F^2 (from sbmm_pilot); sbmm_run
                                 computes them when NULL */
} sbmm_problem;

/* Sizes derived from a problem (no device work). */
typedef struct {
  int64_t atoms;      /* A: K (block) or n (stratified) */
  int64_t strata;     /* S: 1 (block) or K (stratified) */
  int64_t max_width;  /* widest atom */
  int64_t L_max;      /* c * max_width: upper bound of the sketch width L */
  int64_t L_pad_max;  /* L_max rounded up to the sketch padding (32 columns) */
} sbmm_sizes;

/* Outputs of the planning step. All device, caller-owned. */
typedef struct {
  int32_t* idx;      /* [c]   drawn atom per draw (global atom index), stratum-major then draw order */
  double* scale;     /* [c]   1 / sqrt(c_s * p_hat) of each draw (Alg. 1 step 1(b)) */
  int64_t* col_off;  /* [c+1] first column of C (row of D) of each draw; col_off[c] = L */
  int64_t* ck;       /* [S]   draws per stratum */
  double* p_hat;     /* [A]   optional (may be NULL): W / T of each atom */
  int32_t* colmap;   /* [L_pad_max] inner index feeding each sketch column, -1 in the padding */
  double* colscale;  /* [L_pad_max] scale of each sketch column, 0 in the padding */
} sbmm_plan_out;

/* ------------------------------------------------------------------------ */
/* Handle                                                                    */
/* ------------------------------------------------------------------------ */

/* Create a handle bound to HIP device `device`. */
sbmm_status sbmm_create(sbmm_handle* out, int device);
/* Destroy a handle; waits for nothing (synchronize the streams first). */
sbmm_status sbmm_destroy(sbmm_handle h);
/* Static text of a status code. */
const char* sbmm_status_string(sbmm_status s);
/* Text of the last error on this handle (empty if none); valid until the next call. */
const char* sbmm_last_error(sbmm_handle h);
/* Grow the handle's device workspace to at least `bytes` (synchronizing). */
sbmm_status sbmm_reserve(sbmm_handle h, size_t bytes);
/* Wait for `stream`, then report and clear the device status word. */
sbmm_status sbmm_sync(sbmm_handle h, sbmm_stream stream);
/* Fill `out` from the problem's shape (host only; validates the problem). */
sbmm_status sbmm_query_sizes(const sbmm_problem* prob, sbmm_sizes* out);
/* Host only: *bytes = the device workspace that sbmm_run needs for this
 * problem with sketched-product dtype `compute` and every optional buffer
 * (C, D, MN) left to the library, which also covers sbmm_norms, sbmm_plan,
 * sbmm_exact and sbmm_exact_error (with per-block norms), sbmm_pilot and
 * sbmm_bound of the same problem; *L_max (optional) = c * widest atom. After
 * sbmm_reserve(h, *bytes) none of these calls grows the workspace, so none
 * allocates device memory (the handle also keeps a device copy of the last
 * partition, with room for 1023 blocks from sbmm_create on; a partition of
 * more blocks enlarges it once, by 8 bytes a block). SBMM_E_ARG for an
 * invalid problem or a compute dtype the input dtype does not allow. */
sbmm_status sbmm_workspace_size(const sbmm_problem* prob, sbmm_dtype compute, size_t* bytes, int64_t* L_max);

/* ------------------------------------------------------------------------ */
/* Steps of the path                                                         */
/* ------------------------------------------------------------------------ */

/* Norm pass: col_sq[i] = ||M^(i)||_2^2, row_sq[i] = ||N_(i)||_2^2 (the
 * column and row norms behind (1.1), (1.4), (3.8) and (4.2)), and per block
 * blk[k] = ||M^k||_F^2, blk[K+k] = ||N_k||_F^2, blk[2K+k] = s_k =
 * sum_{i in k} ||M^(i)||_2 ||N_(i)||_2. All float64, accumulated in float64
 * in a fixed order (bitwise reproducible). Sizes: col_sq[n], row_sq[n],
 * blk[3K], device. Sets the status word on a non-finite norm. */
sbmm_status sbmm_norms(sbmm_handle h, const sbmm_problem* prob, double* col_sq,
                       double* row_sq, double* blk, sbmm_stream stream);

/* Exact product MN on matrix cores (the reference the sketch is judged
 * against) with, in the epilogue, mn_sq[0] = ||MN||_F^2 (float64, fixed
 * order). MN (optional, may be NULL) gets the product in the compute dtype
 * (F64 for F64 inputs, else F32). blkprod_sq (optional, device [K]) gets
 * ||M^k N_k||_F^2 per block, the quantity (1.2) and (3.9) need: for F32
 * and BF16 inputs with blocks at most 128 wide (and row strides below 2^22
 * elements) as the inner product of the blocks' float32 Gram matrices (bf16
 * values promoted exactly), summed in float64; otherwise from the block sums
 * of the product itself (F64: the float64 product; F32: the float32 product;
 * BF16: the float32 product over exact float32 copies of M and N that the
 * workspace holds, m n + n p floats). mn_sq: device [1], required. */
sbmm_status sbmm_exact(sbmm_handle h, const sbmm_problem* prob, void* MN,
                       int64_t ldmn, double* blkprod_sq, double* mn_sq,
                       sbmm_stream stream);

/* Design and sampling (Alg. 2 inputs p_{k_i} and c_k; Alg. 1 step 1(a)):
 * weights by the problem's rules from col_sq/row_sq/blk (from sbmm_norms),
 * integer quantization and per-stratum CDF, draw counts, the c draws, their
 * scales and the column map of the sketch. If L_host is non-NULL the call
 * synchronizes, stores the sketch width L and reports the status word;
 * otherwise it is asynchronous and L stays on the device in col_off[c]. */
sbmm_status sbmm_plan(sbmm_handle h, const sbmm_problem* prob,
                      const double* col_sq, const double* row_sq,
                      const double* blk, const sbmm_plan_out* out,
                      int64_t* L_host, sbmm_stream stream);

/* Matrix-core throughput of this device for one operand type, measured (a
 * reference beside the specification's peaks, which assume a clock that the
 * power limit holds lower under matrix work; not part of the method). Four
 * workgroups of four waves per compute unit each run eight independent
 * chains of the dtype's 32x32 matrix instruction on operands held in
 * registers: F32 v_mfma_f32_32x32x2_f32, BF16 v_mfma_f32_32x32x16_bf16,
 * F8E4M3 the block-scaled v_mfma_scale_f32_32x32x64_f8f6f4 of the MX
 * product. One warm-up launch, then one timed with events; *tflops (host)
 * receives the instructions' 2 m n k flops over the elapsed time. Synchronous:
 * waits for the handle's device. SBMM_E_UNSUPPORTED for F64. */
sbmm_status sbmm_peak_probe(sbmm_handle h, sbmm_dtype dtype, double* tflops);

/* sbmm_plan for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels, arguments, outputs and status reporting as sbmm_plan, but every
 * scratch buffer of the design and the draws, and the device copy of the
 * partition, lives in a fixed array of SBMM_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends; the call
 * neither grows nor touches the handle's workspace and calls no allocating
 * routine. The array is shared by every call on that GPU, from any handle or
 * thread, and keeps the last call's contents: calls that overlap on one GPU
 * (different streams, or threads) race and must be ordered by the caller.
 * A problem whose plan needs more scratch than the array holds is rejected
 * with SBMM_E_ARG before anything is enqueued (about 16 bytes per atom plus
 * 48 bytes per stratum and 8 per draw: block mode with up to ~10^6 blocks, or
 * stratified mode with n up to ~10^6). The block offsets are copied from the
 * host with hipMemcpyAsync. */
enum { SBMM_NOALLOC_SCRATCH_BYTES = 16 << 20 };
sbmm_status sbmm_plan_noalloc(sbmm_handle h, const sbmm_problem* prob,
                              const double* col_sq, const double* row_sq,
                              const double* blk, const sbmm_plan_out* out,
                              int64_t* L_host, sbmm_stream stream);

/* Step 1 of the two-step algorithm (Alg. 3): in every block k, Alg. 1 with
 * [c0 / K] draws (prob->c0) and the pilot probabilities prob->pilot_prob
 * (UNIFORM: 1/n_k; NORM: (3.8)), i.e. a stratified plan whose draws read the
 * Philox streams with tag 2 in counter word 3 (tag 1 is the main draws), its
 * sketch C^{0k} (m x [c0/K]), D_{0k}, and pilot_sq[k] = ||C^{0k} D_{0k}||_F^2
 * (float64 reduction of products accumulated in the inputs' product dtype:
 * F64 for F64 inputs, else F32). A block whose pilot weights are all zero
 * gets no draws and pilot_sq 0. The stratified problem's own probability
 * and block-size rules are not used. col_sq / row_sq / blk come from
 * sbmm_norms (row_sq / col_sq only for NORM pilots). pilot_plan (optional,
 * may be NULL; sized for c = c0, L_pad_max = round_up(c0, 32)) receives the
 * pilot draws; draws past sum_k ck[k] have idx -1. pilot_sq: device [K]. Pass
 * pilot_sq as prob->pilot_sq to sbmm_plan with alloc TWO_STEP for step 2. */
sbmm_status sbmm_pilot(sbmm_handle h, const sbmm_problem* prob, const double* col_sq, const double* row_sq,
                       const double* blk, const sbmm_plan_out* pilot_plan, double* pilot_sq,
                       sbmm_stream stream);

/* Gather and rescale (Alg. 1 step 1(b), Alg. 2 step 3): C[:, l] = colscale[l]
 * * M[:, colmap[l]] and D[l, :] = colscale[l] * N[colmap[l], :] for
 * l < L, zero for L <= l < round_up(L, 32). C is m x L_pad (ldc >=
 * L_pad_max), D is L_pad x p (ldd >= p), in out_dtype (F64 from F64 inputs;
 * F32 or BF16 from F32/BF16 inputs). Either of C, D may be NULL. */
sbmm_status sbmm_sketch(sbmm_handle h, const sbmm_problem* prob,
                        const sbmm_plan_out* plan, sbmm_dtype out_dtype,
                        void* C, int64_t ldc, void* D, int64_t ldd,
                        sbmm_stream stream);

/* Sketched product CD = C D (Alg. 2 step 4, eq. 3.3) on matrix cores over
 * the inner extent round_up(*L_dev, 32) (read on the device, at most
 * L_pad_max). dtype is the dtype of C and D: F64 (CD in F64), F32 or BF16
 * (CD in F32, float32 accumulation; bf16 operands use the bf16 matrix
 * instructions). If MN and err_sq are given, the
 * epilogue also writes err_sq[0] = ||MN - CD||_F^2 (float64, fixed order).
 * CD may be NULL when only the error is wanted. */
sbmm_status sbmm_sketch_gemm(sbmm_handle h, int64_t m, int64_t p,
                             int64_t L_pad_max, const int64_t* L_dev,
                             sbmm_dtype dtype, const void* C, int64_t ldc,
                             const void* D, int64_t ldd, void* CD,
                             int64_t ldcd, const void* MN, int64_t ldmn,
                             double* err_sq, sbmm_stream stream);

/* The sketch in OCP MX E4M3 (8-bit floats with a shared power-of-two E8M0
 * scale per 32 consecutive sketch columns; float32 inputs): the float32 sketch
 * values C[:, l], D[l, :] of sbmm_sketch are grouped in blocks of 32 along l;
 * a block's scale is 2^X with X = floor(log2 max|x|) - 8 (the byte X + 127;
 * 1 for an all-zero block) and its elements are x / 2^X clamped to +-448 and
 * rounded to the nearest E4M3 (ties to even). C (m x L_pad bytes, ldc) with
 * scales Cs (m x L_pad/32 bytes, ldcs, blocks of one row); D is written
 * transposed: Dt (p x L_pad bytes, lddt) with scales Ds (p x L_pad/32, ldds,
 * blocks of one column of D). ldc, lddt >= L_pad_max and multiples of 16;
 * ldcs, ldds >= round_up(L_pad_max / 32, 4) and multiples of 4; C, Dt 16-byte
 * and Cs, Ds 4-byte aligned. Either the C or the D pair may be NULL. The
 * scales of the blocks past L_pad up to a multiple of 4 blocks are written as
 * 1 (the product reads scales four at a time). */
sbmm_status sbmm_sketch_mx(sbmm_handle h, const sbmm_problem* prob, const sbmm_plan_out* plan, void* C, int64_t ldc,
                           void* Cs, int64_t ldcs, void* Dt, int64_t lddt, void* Ds, int64_t ldds,
                           sbmm_stream stream);

/* Sketched product CD = C D of an MX E4M3 sketch (from sbmm_sketch_mx) on the
 * block-scaled matrix instruction with float32 accumulation, over the inner
 * extent round_up(*L_dev, 32); CD (m x p, float32) and the optional error
 * against MN as in sbmm_sketch_gemm. */
sbmm_status sbmm_sketch_gemm_mx(sbmm_handle h, int64_t m, int64_t p, int64_t L_pad_max, const int64_t* L_dev,
                                const void* C, int64_t ldc, const void* Cs, int64_t ldcs, const void* Dt,
                                int64_t lddt, const void* Ds, int64_t ldds, float* CD, int64_t ldcd,
                                const float* MN, int64_t ldmn, double* err_sq, sbmm_stream stream);

/* The exact product with the judge in its epilogue (the error of a given
 * estimate): err2_and_mn2[0] = ||MN - CD||_F^2, err2_and_mn2[1] =
 * ||MN||_F^2 (device, float64, fixed order). CD is m x p (ldcd >= p) in the
 * product dtype cd_dtype (F64 for F64 inputs, else F32). MN (optional) and
 * blkprod_sq (optional, device [K]: ||M^k N_k||_F^2) as in sbmm_exact. */
sbmm_status sbmm_exact_error(sbmm_handle h, const sbmm_problem* prob, const void* CD, int64_t ldcd,
                             sbmm_dtype cd_dtype, void* MN, int64_t ldmn, double* blkprod_sq,
                             double* err2_and_mn2, sbmm_stream stream);

/* ||X - Y||_F^2 and ||Y||_F^2 of two m x p matrices (F64 or F32) into
 * out2[0..1] (device, float64, fixed order). */
sbmm_status sbmm_error(sbmm_handle h, int64_t m, int64_t p, sbmm_dtype dtype,
                       const void* X, int64_t ldx, const void* Y, int64_t ldy,
                       double* out2, sbmm_stream stream);

/* The whole forward path, synchronizing: norms, (exact product first when
 * the rules need ||M^k N_k||_F), plan, sketch, sketched product, exact
 * product and the error. compute is the dtype of C, D and the sketched
 * product (F64 for F64 inputs; F32 or BF16 otherwise). C and D (optional)
 * receive the sketch; CD (required) the estimate; MN (optional) the exact
 * product. plan (required) receives the draws. err_host / rel_host / L_host
 * (host, optional) receive ||MN - CD||_F, its ratio to ||MN||_F (0 when
 * both are 0, +inf when only ||MN||_F is 0) and L. */
sbmm_status sbmm_run(sbmm_handle h, const sbmm_problem* prob, sbmm_dtype compute,
                     void* C, int64_t ldc, void* D, int64_t ldd, void* CD,
                     int64_t ldcd, void* MN, int64_t ldmn,
                     const sbmm_plan_out* plan, double* err_host,
                     double* rel_host, int64_t* L_host, sbmm_stream stream);

/* Gradient of <G, CD> with respect to M and N, the draws and p held fixed
 * (CD is bilinear in M and N, eq. 3.3); columns of M / rows of N that no draw
 * touched get 0.
 *   F64 / F32 compute: dC = G D^T and dD = C^T G in a float64-accumulating
 *   kernel, then dM[:, i] = sum of scale_l dC[:, l] over the sketch columns l
 *   fed by column i, dN[i, :] likewise from dD, in draw order; C (m x L,
 *   ldc) and D (L x p, ldd) come from the forward (sbmm_sketch in dtype
 *   `compute`).
 *   BF16 compute: the draws of each atom a are merged, w_a = sum of scale^2
 *   over its draws (in draw order, float64), and for every inner index i of a
 *   dM[:, i] = w_a G N[i, :]^T and dN[i, :] = w_a M[:, i]^T G, on the bf16
 *   matrix instructions (float32 accumulation) over bf16(G) and the bf16
 *   values of M and N (M and N of the problem are read; C and D are not and
 *   may be NULL), each product written by its epilogue. The result is the
 *   gradient of the estimator sum_t scale_t^2 M^{a_t} N_{a_t} itself.
 * plan comes from sbmm_plan; L is the sketch width (host; at most
 * L_pad_max; an L below the plan's width sets the status word). G is m x p
 * (ldg) in F64 for F64 compute, else F32. dM (m x n, lddm) and dN (n x p,
 * lddn) are written in full in the problem's input dtype. */
sbmm_status sbmm_backward(sbmm_handle h, const sbmm_problem* prob, const sbmm_plan_out* plan, int64_t L,
                          sbmm_dtype compute, const void* C, int64_t ldc, const void* D, int64_t ldd,
                          const void* G, int64_t ldg, void* dM, int64_t lddm, void* dN, int64_t lddn,
                          sbmm_stream stream);


/* Probability error bounds of the stratified sampler (Alg. 2 and Alg. 3),
 * evaluated from the data and the design that was sampled, by the problem's
 * block-size rule:
 *   alloc OPT      (3.9): Thm 3.3, the variance bound (3.11) and the
 *                  probability bound (3.12);
 *   alloc NORM     (4.2): Thm 4.2, (4.3) and (4.4);
 *   alloc TWO_STEP (4.7): Thm 4.4, (4.8) and (4.9), with the pilot
 *                  estimates prob->pilot_sq (required) that built the plan.
 * With v_k s_k = ||M^k N_k||_F and s_k = sum_{i in k} ||M^(i)||_2 ||N_(i)||_2,
 * theta_1 / theta_2 are the min / max of 1 - v_k^2 over the blocks with
 * s_k > 0 (Thm 3.3), theta^_1 / theta^_2 those of |1 - v^_k^2| with
 * v^_k s_k = ||C^{0k} D_{0k}||_F (Thm 4.3). beta > 0 is used as given (the
 * caller asserts p_hat >= beta (3.8)); beta = 0 takes the largest value the
 * sampled probabilities satisfy, min over atoms with a_i b_i > 0 of
 * p_hat_i / (a_i b_i / s_k) (at most 1). The exponent of Thm 4.4's
 * denominator is read as 1/4, as in Thm 3.3; its numerator carries theta_2
 * of the exact v_k, as printed.
 * Also returned: E ||MN - CD||_F^2 of the design actually sampled, the sum
 * over the blocks with c_k > 0 of (sum_i a_i^2 b_i^2 / p_hat_i -
 * ||M^k N_k||_F^2) / c_k (the per-entry variances of Thm 3.1 summed).
 * Inputs (device): col_sq, row_sq, blk from sbmm_norms; blkprod_sq [K] from
 * sbmm_exact (required for every rule: theta_1, theta_2 and the expected
 * error need it); plan->p_hat and plan->ck of the plan built for this
 * problem (other plan fields are not read). delta: host, n_delta (0..8)
 * values in (0, 1). out: HOST, SBMM_BOUND_FIXED + 2 n_delta doubles laid out
 * as the SBMM_BOUND_* indices, then eta_j and the bound eta_j^2 / (beta c)
 * ||M||_F^2 ||N||_F^2 for every delta_j; phi and the bounds are +inf when
 * the rule divides by theta_1 = 0 (or theta^_1 = 0), and every field but beta
 * and ||M||^2 ||N||^2 is 0 when no block has s_k > 0. The call
 * synchronizes `stream`. Errors: SBMM_E_ARG for block mode, another
 * block-size rule, a missing input, n_delta outside 0..8, delta outside
 * (0, 1) or beta outside [0, 1]. */
enum {
  SBMM_BOUND_THETA1 = 0, SBMM_BOUND_THETA2 = 1, SBMM_BOUND_THETA1_HAT = 2, SBMM_BOUND_THETA2_HAT = 3,
  SBMM_BOUND_BETA = 4, SBMM_BOUND_MN = 5, SBMM_BOUND_PHI = 6, SBMM_BOUND_VAR = 7,
  SBMM_BOUND_EXPECTED = 8, SBMM_BOUND_FIXED = 9, SBMM_BOUND_MAX_DELTA = 8
};
sbmm_status sbmm_bound(sbmm_handle h, const sbmm_problem* prob, const double* col_sq, const double* row_sq,
                       const double* blk, const double* blkprod_sq, const sbmm_plan_out* plan, double beta,
                       int32_t n_delta, const double* delta, double* out, sbmm_stream stream);


/* ------------------------------------------------------------------------ */
/* Many independent problems in one pass                                     */
/* ------------------------------------------------------------------------ */

/* One problem of a batch: block mode, float32 inputs and products, rule
 * UNIFORM or NORM (1.4). All of Alg. 1 / the block sampler runs for it: norm
 * pass, design, draws (Philox key `seed`, counter word 2 `trial`), the
 * sketched product CD (the drawn columns of M and rows of N are read in
 * place, scaled as the gather would write them) and the exact MN it is
 * judged against. m, n, p >= 1. M (m x n, ldm >= n) and N (n x p, ldn >= p)
 * are device, row-major; CD and MN (m x p, ldcd / ldmn >= p) are device
 * outputs. block_off is host (K + 1 offsets, read during sbmm_batch_create
 * only). Every pointer is kept by the batch: the buffers must stay valid
 * until sbmm_batch_destroy, and their contents may change between runs. */
typedef struct {
  int64_t m, n, p;
  const float* M; int64_t ldm;
  const float* N; int64_t ldn;
  int32_t K; const int64_t* block_off;
  int64_t c;
  sbmm_prob prob;
  uint64_t seed, trial;
  float* CD; int64_t ldcd;
  float* MN; int64_t ldmn;
} sbmm_batch_item;

/* Per-problem results of a batch run (device, caller-owned, kept by the
 * batch like the items' buffers). err2_mn2 [2T] (required): ||MN_t - CD_t||_F^2
 * and ||MN_t||_F^2 of problem t at 2t, 2t + 1. L [T] (optional): sketch width
 * of each problem. idx [sum of c_t] (optional): the drawn blocks, problem t
 * starting at sum_{u<t} c_u. */
typedef struct {
  double* err2_mn2;
  int64_t* L;
  int32_t* idx;
} sbmm_batch_outputs;

typedef struct sbmm_batch_s* sbmm_batch;

/* Tile configuration of the two grouped products (exact MN, sketched CD)
 * and whether their work lists start with the longest inner extents. A tile
 * configuration is one of 128x128, 64x128, 128x64, 64x64 (0..3, a
 * register-staged kernel), 256x256 (4, LDS-direct loads, eight waves per
 * workgroup) and 128x128 (5, LDS-direct loads, four waves per workgroup, two
 * workgroups per compute unit). The sketched product has two forms: cfg 0..3
 * read the drawn columns of M and rows of N in place (the gather fused into
 * the product's loads), cfg 6..11 are tile configurations 0..5 over sketches
 * C, D first gathered into a workspace the batch owns (at most 32 GiB, or one
 * problem's sketches if larger, filled by groups of problems, one gather and
 * one product launch per group); 6..11 exist when that workspace could be
 * allocated at sbmm_batch_create. The LDS-direct configurations (exact 4 and
 * 5, materialized 10 and 11) need every problem's rows to start on 16-byte
 * boundaries and its panels to fit 32-bit offsets. Configurations 0..3 and
 * their materialized forms give the same bits; the LDS-direct tiles sum in
 * another order and agree with them to float32 rounding. The timings are
 * filled by sbmm_batch_tune: ms[g][2 cfg + lpt] for product g (0 exact, 1
 * sketch), -1 where not measured. */
enum { SBMM_BATCH_TUNING_SLOTS = 24 };
typedef struct {
  int32_t cfg[2];
  int32_t lpt[2];
  float ms[2][SBMM_BATCH_TUNING_SLOTS];
} sbmm_batch_tuning;

/* Validate T problems, allocate the batch's device memory (owned by the
 * batch) and upload its argument tables; synchronizing. The starting
 * configuration is 128x128 tiles with longest-first work lists. */
sbmm_status sbmm_batch_create(sbmm_handle h, int32_t T, const sbmm_batch_item* items,
                              const sbmm_batch_outputs* out, sbmm_batch* batch);
sbmm_status sbmm_batch_destroy(sbmm_batch batch);

/* Enqueue one pass over every problem: grouped norm pass, one-workgroup-per-
 * problem plans, grouped exact product, grouped sketched product with the
 * error in its epilogue, per-problem reduction. Asynchronous; makes no
 * allocation, host synchronization or memset, so it can be captured. Device
 * status (non-finite norms) is reported by sbmm_sync. */
sbmm_status sbmm_batch_run(sbmm_handle h, sbmm_batch batch, sbmm_stream stream);

/* Capture sbmm_batch_run into a HIP graph held by the batch (replacing any
 * previous one), on a stream of the library's own; sbmm_batch_replay
 * launches it on `stream`. A later sbmm_batch_tune / _set_tuning drops the
 * graph. */
sbmm_status sbmm_batch_capture(sbmm_handle h, sbmm_batch batch);
sbmm_status sbmm_batch_replay(sbmm_handle h, sbmm_batch batch, sbmm_stream stream);

/* Autotuner: run the pass once, then time each available configuration and
 * work order of the two grouped products on this batch (`reps` launches
 * each, HIP events on `stream`), keep the fastest and report all timings in
 * *out (optional). Synchronizing. Results do not depend on the choice among
 * configurations 0..3 and their materialized forms (same accumulation order
 * per output element); the 256x256 tiles agree to float32 rounding (store a
 * tuning with sbmm_batch_set_tuning to fix the bits across runs). */
sbmm_status sbmm_batch_tune(sbmm_handle h, sbmm_batch batch, int32_t reps, sbmm_batch_tuning* out,
                            sbmm_stream stream);
/* Apply a stored configuration (e.g. from an earlier tuning of the same
 * shapes); synchronizing. */
sbmm_status sbmm_batch_set_tuning(sbmm_handle h, sbmm_batch batch, const sbmm_batch_tuning* t);

#ifdef __cplusplus
}
#endif

#endif /* SBMM_H */
