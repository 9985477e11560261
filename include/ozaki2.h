/*
 * ozaki2.h -- C ABI of libozaki2: FP64 (and FP32) matrix multiplication
 * emulated with INT8 matrix cores by Ozaki scheme II, fast mode with the
 * scale-invariant scaling of Kawakami & Takahashi, "Improved Scaling for Fast
 * Mode of Ozaki Scheme II" (Section 4, Algorithm 2), on AMD Instinct MI355X
 * (gfx950).
 *
 * The product C ~ A B is computed in the four steps of Section 2.2:
 *   1. moduli p_1..p_N (the first N of the list printed in Section 3.1),
 *      P = prod p_t, P_t = P / p_t, q_t = P_t^-1 mod p_t;
 *   2. A' = trunc(diag(mu) A), B' = trunc(B diag(nu)) with mu_i, nu_j powers
 *      of two chosen so that 2 sum_h |a'_ih| |b'_hj| < P (eq. os2-condition);
 *   3. the N products rmod(A', p_t) rmod(B', p_t) on INT8 MFMA with INT32
 *      accumulation, combined by the CRT (Theorem 1) into C'' = A'B';
 *   4. C = diag(mu)^-1 C'' diag(nu)^-1, rounded once to the output format.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major (BLAS): element (i, j) of a matrix with
 *   leading dimension ld is at index i + j * ld.
 * - A, B and C are DEVICE pointers owned by the caller.  The library reads
 *   A and B, writes C(0:m-1, 0:n-1) only, and never touches padding rows of
 *   C (i >= m).  C must not overlap A or B.
 * - All GPU work is enqueued on the library's current stream (see
 *   ozaki2_set_stream) and the call returns without waiting for it.
 * - Return value: 0 on success; -i if argument i (1-based) is invalid, in
 *   the style of BLAS xerbla; a positive OZ2_ERR_* code otherwise.  On any
 *   error nothing is launched and C is untouched.  No exception crosses the
 *   ABI.
 * - Not thread-safe: one host thread drives the library at a time.
 */
#ifndef OZAKI2_H
#define OZAKI2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Scaling modes (how mu and nu of Step 2 are chosen). */
#define OZ2_MODE_REVISED  0 /* Section 4, Algorithm 2: the proposed scaling */
#define OZ2_MODE_ORIGINAL 1 /* Section 2.3, Algorithm 1: original fast mode */
#define OZ2_MODE_ACCURATE 2 /* Section 2.3: accurate mode (extra INT8 GEMM) */
/* Exact mode: an optional variant of Algorithm 2 that is not in the paper.
 * The exponent is the exact maximum of the condition Section 4 derives from
 * Cauchy-Schwarz, e = max{e : 2^(2e+1) S <= P - 1} with S the rounded-up
 * squared norm (Algorithm 2 returns this value, or one less within its
 * binary32 slack); it is exactly scale invariant under powers of two.  Where
 * S overflows binary64 (entries or norms beyond about 1.3e154) the norm is
 * recomputed over the entries scaled by 2^-600 (magnitudes rounded up) and
 * the exponent shifted back by 600, so such rows and columns are computed
 * instead of returned as NaN.  Same cost as OZ2_MODE_REVISED when nothing
 * overflows (two extra launches that exit at once). */
#define OZ2_MODE_EXACT    3

/* Engine flag, or-ed into the mode of ozaki2_dgemm, ozaki2_sgemm,
 * ozaki2_workspace_size and ozaki2_debug_stages: the residue products of
 * Step 3 run on the FP8 (E4M3) matrix engine instead of the INT8 one.  The
 * paper states that its scaling serves Ozaki scheme II on FP8 engines too
 * (Section 1) and leaves that extension open (Section 6).  Everything but
 * the products is the INT8 path's (scaling, integers, residues, CRT,
 * unscaling); each residue r is split as r = 16 h + l (l in [-8, 7]) into
 * two E4M3 operands, 16 h and l, the four digit products of an index are
 * summed in binary32 -- exactly, since 512 indices keep every partial sum
 * below 2^24 -- and each block of 512 indices is added in INT32.  The
 * products, and so C, are bit-identical to the INT8 path's; the engine does
 * four times the INT8 path's MFMA work.  Fast modes only (with
 * OZ2_MODE_ACCURATE the call returns OZ2_ERR_UNSUPPORTED).  The workspace
 * holds two digit planes per modulus and operand besides the INT8 ones
 * (ozaki2_workspace_size with the flag reports it). */
#define OZ2_ENGINE_FP8    16

/* Status codes (positive; argument errors are negative). */
#define OZ2_SUCCESS          0
#define OZ2_ERR_K_TOO_LARGE  1 /* k above OZ2_K_MAX (OZ2_K_MAX_ACCURATE in
                                  accurate mode, OZ2_K_BLOCK per problem of a
                                  batch) */
#define OZ2_ERR_WORKSPACE    2 /* no workspace large enough was set (see
                                  ozaki2_set_workspace_policy), or the
                                  library's own allocation failed */
#define OZ2_ERR_HIP          3 /* a HIP runtime call failed */
#define OZ2_ERR_UNSUPPORTED  4 /* valid request the library does not support */
#define OZ2_ERR_TOO_LARGE    5 /* a size overflows the library's indexing */
#define OZ2_ERR_SCRATCH_TOO_SMALL 6 /* ozaki2_dgemm_noalloc: the problem needs
                                       more than OZ2_NOALLOC_SCRATCH_BYTES */

/* Device status bits reported by ozaki2_get_device_status. */
#define OZ2_STATUS_NONFINITE 1 /* a row/column had a NaN/Inf entry or (other
                                  than in OZ2_MODE_EXACT) a squared norm that
                                  overflowed binary64; its output row/column
                                  was written as NaN */

/* Limits. */
#define OZ2_N_MIN 2
#define OZ2_N_MAX 20
#define OZ2_K_BLOCK 131072        /* 2^17: k per INT8 GEMM launch.  For the
                                     odd moduli the residues lie in
                                     [-(p-1)/2, (p-1)/2] and the INT32
                                     products of one block are exact
                                     (|C_t| <= 2^17 * 127^2 < 2^31).  For p =
                                     256 the residues lie in [-128, 127] and
                                     C_0 can reach 2^17 * 128^2 = 2^31, which
                                     wraps in INT32; C_0 is only used modulo
                                     256 and 2^32 is a multiple of 256, so
                                     the result is unaffected (the debug
                                     product of plane 0 is exact modulo
                                     2^32).  Larger k is summed over blocks
                                     modulo p_t */
#define OZ2_K_MAX 4194304         /* 2^22 (grid limits of the norm and
                                     split kernels) */
#define OZ2_K_MAX_ACCURATE 262144 /* 2^18: accurate mode's bar product (entries
                                     <= 64^2 k) stays exact in INT32 */

/*
 * ozaki2_dgemm -- C ~ A B for binary64 A (m x k, lda) and B (k x n, ldb);
 * C (m x n, ldc) is binary64.
 *
 *   m, n, k   >= 0 (args 1-3); k <= OZ2_K_MAX (OZ2_K_MAX_ACCURATE in
 *             accurate mode).
 *   A, lda    device pointer, lda >= max(1, m) (args 4-5).
 *   B, ldb    device pointer, ldb >= max(1, k) (args 6-7).
 *   C, ldc    device pointer, ldc >= max(1, m) (args 8-9).
 *   N         number of moduli, OZ2_N_MIN..OZ2_N_MAX (arg 10).
 *   mode      OZ2_MODE_* (arg 11).
 *
 * Null pointers are accepted only when the matrix has no elements.  m or n
 * equal to 0 is a quick return; k = 0 writes C = 0.  Each element of C is
 * the single correctly rounded (nearest-even) value of C''_ij * 2^-(e_i+f_j),
 * where C'' = A'B' is exact (Section 2.2, Step 4).
 *
 * Workspace: the device memory set by ozaki2_set_workspace, which must be at
 * least ozaki2_workspace_size bytes; otherwise the call returns
 * OZ2_ERR_WORKSPACE and launches nothing (the library never allocates device
 * memory on this path unless the caller opts in with
 * ozaki2_set_workspace_policy(OZ2_WORKSPACE_LIBRARY)).
 */
int ozaki2_dgemm(int64_t m, int64_t n, int64_t k,
                 const double* A, int64_t lda,
                 const double* B, int64_t ldb,
                 double* C, int64_t ldc,
                 int N, int mode);

/*
 * ozaki2_dgemm_noalloc -- ozaki2_dgemm for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * device allocation).  Same arguments, results (bit for bit), stream and
 * return codes as ozaki2_dgemm, but the workspace is a fixed device array of
 * OZ2_NOALLOC_SCRATCH_BYTES inside the library (one per GPU, held until the
 * process ends) instead of the memory set by ozaki2_set_workspace; the call
 * allocates nothing (no hipMalloc, no library allocation, no events) and
 * launches only kernels (no memset), so it may be captured into a graph.
 * The caller still passes A, B and C.  A problem whose workspace would
 * exceed the array returns OZ2_ERR_SCRATCH_TOO_SMALL and launches nothing;
 * every problem with ozaki2_workspace_size <= OZ2_NOALLOC_SCRATCH_BYTES is
 * accepted (the check uses the layout of the GEMM tile the call picks,
 * which may accept somewhat larger ones), e.g. m = n = k = 1024 at any N.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams, or different host threads) race and must be
 * ordered by the caller.  Stage timing (ozaki2_set_timing) does not apply.
 */
#define OZ2_NOALLOC_SCRATCH_BYTES (64u << 20)
int ozaki2_dgemm_noalloc(int64_t m, int64_t n, int64_t k,
                         const double* A, int64_t lda,
                         const double* B, int64_t ldb,
                         double* C, int64_t ldc,
                         int N, int mode);

/*
 * ozaki2_sgemm -- as ozaki2_dgemm for binary32 A, B and C (Section 5 applies
 * the same scheme to SGEMM).  Squared norms are still summed in binary64
 * with rounding up; C is rounded once to binary32.
 */
int ozaki2_sgemm(int64_t m, int64_t n, int64_t k,
                 const float* A, int64_t lda,
                 const float* B, int64_t ldb,
                 float* C, int64_t ldc,
                 int N, int mode);

/*
 * ozaki2_zgemm -- C ~ A B for complex binary64 matrices (ZGEMM).  The paper
 * states that its scaling serves the complex fast mode as well (Section 1)
 * and leaves the extension to future work (Section 6); the library applies
 * Section 2.2 and Algorithm 2 (or 1) as follows.  A complex row of A (column
 * of B) is scaled as the real vector of its 2k components in storage order
 * (re, im, re, ...): squared norms rounded up over those components in
 * chunks of 64 (32 complex entries), Algorithm 1's maximum over component
 * magnitudes.  Both parts of an entry are truncated with the row's
 * (column's) exponent; the CRT recovers the real and imaginary parts of the
 * complex integer product exactly (both are bounded by ||a'_i|| ||b'_j||,
 * what the scaling keeps below P/2), and each part of C is rounded once.
 * Per modulus the product takes three INT8 GEMMs.
 *
 *   A, B, C   device pointers to interleaved (re, im) binary64 pairs
 *             (the layout of hipDoubleComplex / double _Complex), column-major,
 *             each aligned to 16 bytes (else -4, -6 or -8).
 *   lda, ldb, ldc, m, n, k, N: as ozaki2_dgemm, leading dimensions counted
 *             in complex entries.
 *   mode      OZ2_MODE_REVISED, OZ2_MODE_ORIGINAL or OZ2_MODE_EXACT;
 *             OZ2_MODE_ACCURATE returns OZ2_ERR_UNSUPPORTED.
 *
 * k up to OZ2_K_MAX (k-blocked beyond OZ2_K_BLOCK like ozaki2_dgemm).  A row
 * or column with a non-finite entry or squared norm gives NaN in both parts
 * of its outputs and sets OZ2_STATUS_NONFINITE.  Workspace and stream rules
 * as ozaki2_dgemm (size: ozaki2_zgemm_workspace_size).
 */
int ozaki2_zgemm(int64_t m, int64_t n, int64_t k,
                 const double* A, int64_t lda,
                 const double* B, int64_t ldb,
                 double* C, int64_t ldc,
                 int N, int mode);

/*
 * ozaki2_cgemm -- as ozaki2_zgemm for complex binary32 matrices (CGEMM):
 * pointers to interleaved binary32 pairs aligned to 8 bytes; squared norms in
 * binary64 with rounding up; each part of C rounded once to binary32.
 */
int ozaki2_cgemm(int64_t m, int64_t n, int64_t k,
                 const float* A, int64_t lda,
                 const float* B, int64_t ldb,
                 float* C, int64_t ldc,
                 int N, int mode);

/* Bytes of workspace an ozaki2_zgemm or ozaki2_cgemm call with these
 * arguments needs (written to *bytes).  Returns 0, the argument error code,
 * or OZ2_ERR_UNSUPPORTED for accurate mode. */
int ozaki2_zgemm_workspace_size(int64_t m, int64_t n, int64_t k, int N, int mode,
                                size_t* bytes);

/* Set the HIP stream (a hipStream_t passed as void*; NULL = null stream)
 * used by every later call.  Returns 0. */
int ozaki2_set_stream(void* stream);

/* Bytes of workspace a call with these arguments needs (written to *bytes).
 * Returns 0, or the argument error code as ozaki2_dgemm would. */
int ozaki2_workspace_size(int64_t m, int64_t n, int64_t k, int N, int mode,
                          size_t* bytes);

/* Use caller-owned device memory (256-byte aligned) as workspace for every
 * later call.  The library does not free it.  Pass (NULL, 0) to unset it.
 * The memory must stay valid until replaced and must not be in use by
 * another call in flight on another stream; between calls its contents
 * belong to the library (ozaki2_dgemm_batched keeps tables there), so the
 * caller does not write it.  Returns 0, or -1 if ptr is not 256-byte
 * aligned. */
int ozaki2_set_workspace(void* ptr, size_t bytes);

/* What a call does when the caller's workspace is missing or too small.
 * OZ2_WORKSPACE_CALLER (the default): return OZ2_ERR_WORKSPACE, launch
 * nothing -- no entry point allocates device memory.  OZ2_WORKSPACE_LIBRARY
 * (opt-in convenience): the library allocates its own workspace with
 * hipMalloc (synchronising the device when it grows; kept until
 * ozaki2_finalize).  Returns 0, or -1 for an unknown policy. */
#define OZ2_WORKSPACE_CALLER  0
#define OZ2_WORKSPACE_LIBRARY 1
int ozaki2_set_workspace_policy(int policy);

/* Synchronise the current stream, then report (in *status) and clear the
 * device status bits (OZ2_STATUS_*) written by the most recent GEMM call on
 * the current device.  Returns 0, -1 if status is NULL, or OZ2_ERR_HIP. */
int ozaki2_get_device_status(int* status);

/* Human-readable description of a return code.  Never NULL. */
const char* ozaki2_status_string(int code);

/* Library version and contract constants, e.g. "ozaki2 0.1 kc=64 ...". */
const char* ozaki2_version(void);

/* Free library-owned workspace and events.  Returns 0. */
int ozaki2_finalize(void);

/*
 * ozaki2_query_constants -- host-only: the constants of Step 1 and of the
 * scaling formulas for N moduli, as the library computes them.
 *   moduli[N]       the moduli p_1..p_N (first N of the Section 3.1 list)
 *   p_prime_prop    P'_prop = RD32(log2(P-1)/2 - 0.5) (Section 4; equals
 *                   P'_accu of Section 2.3)
 *   p_prime_fast    P'_fast = RD32(log2(P-1)/2 - 1.5) (Section 2.3)
 *   delta           RU32(0.5 / (1 - 4 u32)), u32 = 2^-24 (Section 2.3)
 *   log2_P          log2(P) as a binary64 approximation (informative)
 * Any output pointer may be NULL.  Returns 0 or -1 if N is out of range.
 */
int ozaki2_query_constants(int N, int32_t* moduli, float* p_prime_prop,
                           float* p_prime_fast, float* delta, double* log2_P);

/*
 * Stage timing.  ozaki2_set_timing(1) makes every later call record HIP
 * events around its stages on the current stream; ozaki2_get_stage_times
 * synchronises the stream and writes into ms[OZ2_NUM_STAGES] the summed
 * milliseconds per stage since timing was enabled (or last read), and into
 * *calls the number of calls timed, then resets the sums.
 * Stages: 0 norms and exponents (K1; in accurate mode also the bar matrices
 * and their INT8 GEMM), 1 convert and split (K2), 2 INT8 GEMMs (K3), 3 CRT
 * and unscale (K4), 4 other (zero fill, bookkeeping).  When the fused kernel
 * for narrow B runs (see ozaki2_set_tile), stage 1 holds K2 for B only and
 * stage 2 the fused conversion of A, products and CRT.
 */
#define OZ2_NUM_STAGES 5
int ozaki2_set_timing(int enable);
int ozaki2_get_stage_times(double* ms, int* calls);

/*
 * GEMM tile of ozaki2_dgemm / ozaki2_sgemm (Step 3's N INT8 products; the
 * batched path always uses 128 x 128).  OZ2_TILE_AUTO (the default) picks per
 * call from m, n, k and N with a cost model of padded work and workgroup
 * rounds; the others force one shape (rows x columns of C per workgroup).
 * Under OZ2_TILE_AUTO a narrow B (n <= 64) with N <= 16, a fast or exact
 * mode and k <= OZ2_K_BLOCK runs a fused kernel instead (conversion of A,
 * the N products on 16 x 16 blocks and the CRT in one pass, nothing
 * materialised for A); a forced tile always runs the separate kernels.
 * Results do not depend on the tile or on the fusion.  ozaki2_set_tile returns 0, or -1 for
 * an unknown value; ozaki2_get_tile writes the tile a call with these sizes
 * would use and returns 0, or minus the index of a bad argument.
 */
#define OZ2_TILE_AUTO    0
#define OZ2_TILE_256x256 1
#define OZ2_TILE_128x128 2
#define OZ2_TILE_256x64  3
int ozaki2_set_tile(int tile);
int ozaki2_get_tile(int64_t m, int64_t n, int64_t k, int N, int* tile);

/*
 * Batched emulated DGEMM.  One problem of a batch, column-major as for
 * ozaki2_dgemm.  N is its number of moduli (OZ2_N_MIN..OZ2_N_MAX), or 0 to
 * let the library pick it for the batch's accuracy target; N_used is
 * written by ozaki2_dgemm_batched (its input value is ignored).
 */
typedef struct oz2_problem {
  int64_t m, n, k;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  int N;
  int N_used;   /* output: the number of moduli used (0 if nothing was computed) */
} oz2_problem;

/*
 * ozaki2_dgemm_batched -- C_i ~ A_i B_i for `batch` independent problems of
 * any shapes and moduli counts (problems[] is a HOST array; the matrices are
 * device memory), with mode OZ2_MODE_REVISED or OZ2_MODE_ORIGINAL.
 *
 * Problems with N = 0 get the smallest N whose calibrated maximum relative
 * error (the library's autotuner, see ozaki2_autotune_N) is at most
 * target_max_rel_err / 4 for their k and for phi estimated from their data
 * (ozaki2_estimate_phi of the rows of A and of the columns of B, the larger
 * of the two); this reads the
 * operands once more and synchronises the stream before the launch.  The
 * target is ignored when every N is given.
 *
 * All problems are computed by one HIP graph launch: the stages of
 * ozaki2_dgemm run once for the whole batch (one grid per stage) and the
 * INT8 GEMMs of every problem and modulus run in one persistent kernel over
 * a shared work list.  k <= OZ2_K_BLOCK per problem.  The graph is built on
 * the first call with a given batch signature (shapes, N, mode, device,
 * workspace address and layout; this call writes the batch's tables into
 * the workspace and synchronises) and replayed afterwards; a replay whose
 * problems moved to other matrices first rewrites those pointers with a
 * small kernel launch (the pointers travel as its arguments).  The tables
 * stay in the workspace between calls: when any other call has used the
 * workspace since, or a different workspace was set, they are written again
 * (and the stream synchronised) before the replay.  Every device buffer of
 * the batch -- status, descriptors, work list, the phi estimate's scratch,
 * the per-problem regions -- lies in the caller's workspace, which must hold
 * ozaki2_dgemm_batched_workspace_size bytes (else OZ2_ERR_WORKSPACE, under
 * the default policy).  With ozaki2_set_timing(1) the same kernels are
 * launched directly instead of the graph, with stage events as for
 * ozaki2_dgemm.  Results are bit-identical to calling ozaki2_dgemm on each
 * problem with its N_used.
 *
 * Returns 0; -1 if batch < 0; -2 if problems is NULL with batch > 0; -3 for
 * an unsupported mode; -4 if some N is 0 and the target is not in (0, 1];
 * or, for the first invalid problem, the code ozaki2_dgemm would return for
 * it, with its index in *bad_index (may be NULL).  Nothing is launched on
 * error.
 */
int ozaki2_dgemm_batched(int batch, oz2_problem* problems, int mode,
                         double target_max_rel_err, int* bad_index);

/* Bytes of workspace an ozaki2_dgemm_batched call with these problems and
 * mode needs (written to *bytes; 0 if nothing would be computed).  Problems
 * with N = 0 are counted with OZ2_N_MAX moduli, so the bound holds for any
 * N the autotuner picks.  Returns 0, -1 batch < 0, -2 problems NULL with
 * batch > 0, -3 unsupported mode, -4 bytes NULL, or the code
 * ozaki2_dgemm_batched would return for the first invalid problem. */
int ozaki2_dgemm_batched_workspace_size(int batch, const oz2_problem* problems, int mode,
                                        size_t* bytes);

/*
 * The autotuner.  The error of the emulated product is set by the number of
 * moduli (wider integers) and the spread of the entry magnitudes; for the
 * distribution of the paper's experiments, (rand - 0.5) exp(phi randn)
 * (Section 3.2), log|a| has variance 1 + phi^2.  The library carries a
 * table of maximum relative errors of ozaki2_dgemm measured on the GPU
 * against exact products, per (k, phi, N) grid point (k 64..16384, phi
 * 0.5..4, N 10..20).
 *
 * ozaki2_autotune_N -- host only: *N = the smallest N whose error estimate
 * is at most target / 4, 20 if none is.  The estimate is an upper envelope of
 * the table: the largest tabulated error over every grid point at or below
 * the grid point that brackets (k, phi) from above, for this N or any larger
 * one (so the pick never falls as k, phi or the accuracy demand grow); for k
 * beyond 16384 it is scaled by sqrt(k / 16384); for phi beyond 4 (outside the
 * calibration) *N = 20.  Returns 0; -1 k < 0; -2 phi not >= 0; -3 target not
 * in (0, 1]; -4 N is NULL.
 *
 * ozaki2_estimate_phi -- phi of a column-major rows x cols binary64 device
 * matrix (leading dimension ld) whose vectors -- the units the scaling
 * treats -- are its rows (vectors = 0, as for A) or its columns (vectors =
 * 1, as for B): sqrt(max(var - 1, 0)) with var the variance of log|x| within
 * the vectors, pooled over them (the sum over vectors of the squared
 * deviations from the vector's mean, over the sum of (count - 1)), on a
 * sample of about 2^20 entries: every vector with its first
 * max(2, 2^20 / (number of vectors)) entries; zeros and non-finite entries
 * are skipped and
 * a vector with fewer than two entries left out (0 when none has two).
 * Scaling rows (columns) by different powers of two leaves it unchanged.
 * Uses the first KiB of the workspace (same workspace rules as ozaki2_dgemm)
 * and synchronises the stream.  Returns 0; -1..-6 for the argument in that
 * position; OZ2_ERR_WORKSPACE; or OZ2_ERR_HIP.
 */
int ozaki2_autotune_N(int64_t k, double phi, double target_max_rel_err, int* N);
int ozaki2_estimate_phi(int64_t rows, int64_t cols, const double* X, int64_t ld, int vectors,
                        double* phi);

/*
 * ozaki2_debug_stages -- run Steps 1-3 of ozaki2_dgemm for binary64 A, B
 * (same argument rules) and copy every intermediate to caller DEVICE
 * buffers (any may be NULL to skip it):
 *   eA[m], eB[n]      int32 log2(mu_i), log2(nu_j)
 *   SA[m], SB[n]      binary64 rounded-up squared norms (0 in accurate mode)
 *   RA[N*m*k]         int8 residues of A': element (t, i, h) at t*m*k + i*k + h
 *   RB[N*n*k]         int8 residues of B': element (t, j, h) at t*n*k + j*k + h
 *   Ct[m*n]           int32 product rmod(A',p_t) rmod(B',p_t) for modulus
 *                     index t (0-based), column-major (i + j*m); only for
 *                     k <= OZ2_K_BLOCK (else OZ2_ERR_UNSUPPORTED); for t = 0
 *                     (p = 256) it is the product modulo 2^32 (see
 *                     OZ2_K_BLOCK)
 * Test hook for stage-by-stage comparison with a reference.  Synchronises
 * the stream before returning.
 */
int ozaki2_debug_stages(int64_t m, int64_t n, int64_t k,
                        const double* A, int64_t lda,
                        const double* B, int64_t ldb,
                        int N, int mode, int t,
                        int32_t* eA, int32_t* eB, double* SA, double* SB,
                        int8_t* RA, int8_t* RB, int32_t* Ct);

/*
 * ozaki2_debug_log2f -- y[i] = the binary32 log2 used by the scaling
 * (correctly rounded to nearest), for n binary32 values x[i] in [1, 2];
 * device pointers.  Test hook.  Synchronises the stream.
 */
int ozaki2_debug_log2f(const float* x, float* y, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* OZAKI2_H */
