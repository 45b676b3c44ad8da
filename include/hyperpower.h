/*
 * hyperpower.h -- C ABI of libhyperpower, an MI355X (gfx950) implementation of
 * the 18th-order hyperpower iteration for outer generalized inverses of
 * Pan, Soleymani and Zhao, "Highly Efficient Computation of Generalized
 * Inverse of a Matrix" (arXiv 1604.07893).
 *
 * Problem (Section 1.2 and Theorem 3.1): given A (m x n) and X0 = alpha*G with
 * R(G) and N(G) fixing the range T and null space S, iterate
 *     R_k = I - A X_k,  X_{k+1} = X_k (I + R_k + ... + R_k^17)
 * evaluated with the seven-product factorisation (PM) of Section 2, or with
 * the stabilised variant (PM-modified) of Section 7, until the stopping test
 * passes. The limit is A^(2)_{R(G),N(G)}: the Moore-Penrose inverse for
 * G = A^T and the Drazin inverse for G = A^l, l >= ind(A) (Section 4).
 *
 * Conventions shared by every call:
 *  - Matrices are real FP64, row-major, with an explicit leading dimension
 *    (elements between the starts of consecutive rows, >= the column count).
 *  - Every matrix and workspace pointer is DEVICE memory owned by the caller;
 *    the library never frees or retains it. Inputs are read-only; outputs are
 *    write-only and must not alias inputs or the workspace.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *    device work is enqueued on it; hp_solve synchronises the stream once per
 *    loop to read the two stopping scalars (with hp_params.device_stop, once
 *    per chunk of loops).
 *  - Return value: HP_OK (0); a positive numerical outcome (the output is
 *    still written); or a negative error (outputs untouched).
 *  - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef HYPERPOWER_H
#define HYPERPOWER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HP_ABI_VERSION 4

/* ---- status codes ------------------------------------------------------ */
#define HP_OK 0
#define HP_MAXITER 1      /* max_iter loops ran without passing the stop test */
#define HP_STAGNATED 2    /* the change stopped decreasing after convergence set
                             in; X is the input of the loop that saw it
                             (Section 6: looping past convergence can diverge) */
#define HP_DIVERGED 3     /* the relative change exceeded diverge_limit before
                             convergence set in (alpha too large, or rounding
                             growing in a null-space block, Section 6); X is
                             the best iterate before the blow-up: the input of
                             the loop with the smallest relative change
                             (hp_solve; batched and served solves return the
                             input of the loop that detected it) */
#define HP_NONFINITE 4    /* a NaN/Inf appeared; X is the best iterate as for
                             HP_DIVERGED if no change below tau_switch had been
                             seen, else the last finite iterate */
#define HP_PENDING 5      /* serving: the request has not finished yet */
#define HP_EINVAL (-1)    /* bad argument (shape, leading dim, alignment, enum) */
#define HP_EWORKSPACE (-2)/* workspace NULL or smaller than hp_workspace_bytes */
#define HP_EBUDGET (-3)   /* serving: a request can never fit the HBM budget */
#define HP_EHIP (-4)      /* a HIP runtime call failed */
#define HP_EUNSUPPORTED (-5) /* valid but not implemented combination */

/* ---- enums --------------------------------------------------------------- */
/* which outer inverse (Section 1.2; X0 rules of Section 4) */
#define HP_KIND_MOORE_PENROSE 0   /* G = A^T, limit A^dagger (any m, n) */
#define HP_KIND_DRAZIN 1          /* G = A^l, limit A^D (m == n, l >= ind(A));
                                     HP_PREC_FP64 only (HP_EUNSUPPORTED otherwise) */

/* scaling alpha of X0 = alpha*G (Section 4) */
#define HP_ALPHA_NORM1INF 0  /* Moore-Penrose: alpha = 1/(||A||_1 ||A||_inf) */
#define HP_ALPHA_USER 1      /* alpha = hp_params.alpha (e.g. 1/sigma_max^2 or
                                2/(sigma_1^2 + sigma_r^2) when known) */
#define HP_ALPHA_TRACE 2     /* Drazin: alpha = 1/Tr(A^{l+1}) */
#define HP_ALPHA_SIGMA_MAX2 3 /* Moore-Penrose: alpha = 1/rho with rho an estimate
                                of sigma_1(A)^2 from 50 power-iteration steps on
                                A^T A on the GPU (a fixed generic start vector;
                                rho <= sigma_1^2, so alpha sigma_1^2 >= 1, and it
                                stays below 2 as long as rho > sigma_1^2 / 2,
                                the convergence condition of Section 4) */
#define HP_ALPHA_DIAG 4      /* Moore-Penrose kind, square A only: X0 =
                                diag(1/a_11, ..., 1/a_nn), the initial matrix
                                (choice3) of Example 8.3 (G = D^{-1}, so the
                                limit is A^{-1} when A is nonsingular and the
                                loops converge, e.g. for a strictly diagonally
                                dominant A); alpha is reported as 1. A zero
                                diagonal entry gives HP_NONFINITE */

/* iteration variant */
#define HP_VARIANT_PLAIN 0       /* (PM), Section 2: 7 products per loop */
#define HP_VARIANT_STABILISED 1  /* (PM) loops until the relative change first
                                    drops below tau_switch, then (PM-modified)
                                    of Section 7 (X <- X A X after each loop):
                                    the switch recipe that closes Section 7 */
#define HP_VARIANT_STAB_ALWAYS 2 /* (PM-modified) from X0 (converges to a
                                    smaller-range {2}-inverse on ill-conditioned
                                    input; kept for completeness) */

/* which side the polynomial in R is evaluated on. X(I-AX)^i = (I-XA)^i X, so
   both give the same iterates in exact arithmetic; the left form works with
   n x n residuals and is cheaper when m > n. */
#define HP_SIDE_AUTO 0   /* left if m > n, else right */
#define HP_SIDE_RIGHT 1  /* R = I - A X (m x m), X_{k+1} = X W: the paper's form */
#define HP_SIDE_LEFT 2   /* R = I - X A (n x n), X_{k+1} = W X */

/* which iteration of the hyperpower family runs each loop. PM is the paper's
   method; the others are the schemes it is compared with (Section 1.3 and
   Section 2), evaluated on the GPU with the same kernels so that the
   comparison of Section 8 can be repeated. Each loop's update is X W (right
   form) or W X (left form) with W a polynomial in R. */
#define HP_METHOD_PM 0 /* (PM), Section 2: order 18, 7 products */
#define HP_METHOD_SM 1 /* Newton-Schulz-Hotelling (schulz): X(2I - AX), order 2,
                          2 products */
#define HP_METHOD_CM 2 /* Chebyshev-Sen-Prabhu (chebyshev): X(3I - AX(3I - AX)),
                          order 3, 3 products */
#define HP_METHOD_FM 3 /* the seventh-order factorisation (SoleymaniN):
                          psi = I - AX, zeta = I + psi + psi^2,
                          upsilon = psi + psi^4, X(I + upsilon zeta); 5 products */
#define HP_METHOD_HM 4 /* (hyper18-2): X(I+R)(R^2-R+I)(R^2+R+I)(R^6-R^3+I)
                          (R^6+R^3+I), order 18, 9 products; the five factors
                          are multiplied together before the update */

/* stopping rule (Section 4, Section 8) */
#define HP_STOP_REL_FRO 0   /* ||X_{k+1}-X_k||_F / ||X_k||_F < tol */
#define HP_STOP_PAPER_4_1 1 /* ||X_{k+1}-X_k||_F / (p^k alpha) < tol, rule
                               (stopreliable) with the Frobenius norm; p is the
                               method's order (18 for PM and HM) and k counts
                               loops from 0 */
#define HP_STOP_ABS_INF 2   /* ||X_{k+1}-X_k||_inf <= tol (Example 8.1) */
#define HP_STOP_REL_FRO_BOUND 3 /* HP_STOP_REL_FRO, and in the final precision
                               stage, before a plain loop that follows a change
                               d with d^p < tol, the loop's residual R is formed
                               first: if ||R||_F / (1 - ||R||_F) < tol, the
                               change that loop would make is below tol
                               (||X(R + R^2 + ...)||_F <= ||X||_F ||R||_2 /
                               (1 - ||R||_2)), so it is skipped and X_{k+1} is
                               returned; otherwise the loop goes on with that R
                               and, with HP_METHOD_PM, runs the scheme with the
                               fewest products (SM, CM, FM, PM) whose order q
                               has ||R||_F^q < tol/2. The check also runs
                               before the first loop of the final stage when a
                               lower stage ended in the converging regime.
                               Saves the confirming loop on nonsingular input
                               (R -> 0); on singular input ||R||_F stays >= 1
                               and the rule is the relative change. An
                               addition to the paper's stopping rules. */

/* arithmetic of the loops */
#define HP_PREC_FP64 0  /* every loop in FP64 (FP64 MFMA, FP64 accumulate) */
#define HP_PREC_FP32 1  /* every loop in FP32 storage and FP32 MFMA; the stop
                           sums in FP64; X returned in FP64. Reaches about
                           kappa(A) * 6e-8, not an FP64 tolerance. */
#define HP_PREC_FP32_FP64 3 /* stage 1 (FP32) then stage 2 (FP64): HP_PREC_MIXED
                               without the 16-bit stage */
#define HP_PREC_MIXED 2 /* stage 0: 16-bit MFMA products (hp_params.low_dtype)
                           on FP32 storage with FP32 accumulation; stage 1:
                           FP32; stage 2: FP64 loops until the stop test
                           passes. A stage ends when its relative change stops
                           halving (below 1), falls under 10x its unit
                           roundoff, or after a loop (not its first) whose
                           change falls below 0.2 (that loop's output is at
                           the stage's floor: about 0.2^18 relative error);
                           the FP64 stage alone applies the stop test
                           and the stagnation guard. For Moore-Penrose input
                           that is not square, or square with
                           ||I - AX||_F^2 >= 0.5 after the lower stage (rank
                           deficient), the FP64 stage starts with
                           X <- (XA)^T X (AX)^T: FP32 error in the parts of X
                           outside R(A^T) x R(A) is not corrected by the loops
                           (an addition to the paper's method, from its third
                           and fourth Penrose equations). */

#define HP_PREC_DELTA32 4 /* every loop in the delta form (an exact
                           re-association of Section 2's products): the
                           residual R = I - AX and the update
                           X_{k+1} = X_k + X_k (W - I) in FP64, the products of
                           the polynomial on R in FP32 (FP32 storage and MFMA),
                           each product forming a b and its epilogue adding
                           a + b for factors I + a, I + b, so that no value
                           I + (small) is rounded to FP32. The FP32 error then
                           enters W - I, not the update or R: on rank-deficient
                           input the null-space block is not seeded by FP32
                           rounding (it grows 18x per plain loop, Theorem 6.2,
                           and all-FP32 loops diverge there), and the error
                           floor is about u_fp32 * kappa-dependent growth of
                           the off-diagonal blocks (not an FP64 tolerance on
                           singular input). HP_METHOD_PM only; single solves */

/* hp_params.low_dtype: operand type of the first mixed stage */
#define HP_LOWP_BF16 0
#define HP_LOWP_F16 1

/* hp_params.flags */
#define HP_FLAG_TIME_KERNELS 1 /* time every GEMM launch with hipEvents on the
                                  solve stream; sums land in hp_result.gemm_ms */
#define HP_FLAG_INF_NORM 2     /* also compute ||X_{k+1}-X_k||_inf each loop
                                  (implied by HP_STOP_ABS_INF); enables coc */
#define HP_FLAG_NO_GRAPH 4     /* batched/served, and hp_solve with
                                  device_stop: launch each loop's kernels one
                                  by one instead of replaying a captured
                                  hipGraph of the loop (hp_solve caches a
                                  graph of two loops per workspace, shape and
                                  loop form in the handle; hp_solve_noalloc
                                  and HP_FLAG_TIME_KERNELS never capture) */
#define HP_FLAG_NO_RETRY 8     /* served: do not retry in FP64 a request whose
                                  lower-precision solve ended other than
                                  HP_OK (see hp_serve_step) */
#define HP_FLAG_SYMMETRIC 16  /* single FP64 Moore-Penrose solves from
                                  X0 = alpha A^T (no caller's X0, no Chop),
                                  when the caller knows that rank(A) equals
                                  the residual's side s (min(m, n) with
                                  HP_SIDE_AUTO): form the loop's s x s
                                  products (R, the polynomials in R, the
                                  middle product X A of the stabilising
                                  step), symmetric in exact arithmetic
                                  because X_k = p(A^T A) A^T, once per pair
                                  (i, j), i <= j, and mirror them
                                  (hp_gemm_sym). Only on the first L loops
                                  with p^L 2^-52 <= 1e-7 (p the order) and,
                                  after the first, while the last change d
                                  has (d/2)^p >= tol: the loop expected to
                                  meet the test forms full products and
                                  corrects what the forced symmetry left.
                                  Ignored in staged precisions (mirroring
                                  their rounding diverges). With
                                  rank(A) < s the forced symmetry feeds the
                                  null-space error block back into the
                                  range block: do not set it */

#define HP_FLAG_FP64_POLY 32   /* HP_PREC_MIXED / HP_PREC_FP32_FP64 single
                                  solves: run the FP64 stage's polynomial in
                                  FP64 too. By default an FP64-stage loop whose
                                  last known residual has ||R||_F < 0.5 (the
                                  loops converge to R = 0: no null space on
                                  the residual's side) runs in the delta form
                                  of HP_PREC_DELTA32: R and the update in FP64,
                                  the polynomial's products in FP32, whose
                                  rounding then scales with ||R||; other FP64
                                  loops form every product in FP64 */

/* GEMM element type for hp_gemm */
#define HP_DTYPE_F64 0 /* FP64 operands, v_mfma_f64_16x16x4f64, FP64 accumulate */
#define HP_DTYPE_F32 1 /* FP32 operands, v_mfma_f32_16x16x4f32, FP32 accumulate */
#define HP_DTYPE_BF16_F32 2 /* FP32 in memory, operands rounded to bf16,
                               v_mfma_f32_16x16x32_bf16, FP32 accumulate and C */
#define HP_DTYPE_F16_F32 3  /* as above with fp16 operands (f16 MFMA) */
#define HP_DTYPE_BF16 4 /* 16-bit operands in memory: A (M x K) bf16 row-major and
                           B passed TRANSPOSED, Bt = B^T (N x K) bf16 row-major
                           (ldb >= K); v_mfma_f32_16x16x32_bf16, FP32 accumulate
                           and C (float). lda, ldb multiples of 8 elements */
#define HP_DTYPE_F16 5  /* as HP_DTYPE_BF16 with fp16 operands */
/* hp_autotune only: the tile of the persistent grouped launch of batched and
   served solves, FP64 or FP32 (returned tile: 0 = 64 x 64, 1 = 128 x 128,
   2 = 32 x 32 with a 4x deeper K-tile), timed on a table of copies of an
   M x N x K product; groups created afterwards use the fastest */
#define HP_DTYPE_GROUPED_F64 6
#define HP_DTYPE_GROUPED_F32 7

typedef struct hp_params {
    int32_t kind;          /* HP_KIND_* */
    int32_t drazin_l;      /* l >= ind(A), Drazin only (caller-supplied) */
    int32_t alpha_rule;    /* HP_ALPHA_* */
    int32_t variant;       /* HP_VARIANT_* */
    double alpha;          /* used with HP_ALPHA_USER */
    double tau_switch;     /* relative change that starts the stabilised loops
                              and arms the stagnation guard (default 0.1; a
                              solve whose last stage is FP32 uses at least
                              0.25: its rounding-seeded null-space block
                              outgrows X a loop earlier, Theorem 6.2). The
                              first stabilised loop after the switch is not
                              tested for stagnation (its change also removes
                              the null-space block, Theorem 7.1) */
    double tol;            /* stopping tolerance (default 1e-12) */
    double diverge_limit;  /* relative change treated as divergence (1e6) */
    int32_t max_iter;      /* loop cap (default 100, as in Section 8) */
    int32_t stop_rule;     /* HP_STOP_* */
    int32_t side;          /* HP_SIDE_* */
    int32_t precision;     /* HP_PREC_* */
    int32_t flags;         /* HP_FLAG_* */
    int32_t low_dtype;     /* HP_LOWP_*, HP_PREC_MIXED only */
    int32_t method;        /* HP_METHOD_* (default PM). Methods other than PM
                              run in HP_PREC_FP64 or HP_PREC_FP32 in hp_solve
                              only (HP_EUNSUPPORTED otherwise) */
    int32_t device_stop;   /* 1: hp_solve enqueues its loops without reading
                              the stopping sums on the host after each
                              loop: a one-thread kernel takes each loop's
                              stop / switch / guard decision from the sums on
                              the device, and every kernel of a later loop
                              (or of the form of a loop not taken: plain or
                              stabilised) reads that decision and returns at
                              once; the host reads the decision state once
                              per chunk of loops (the first 4, then 2 at a
                              time). Same decisions, same iterates, bitwise,
                              as with 0. HP_PREC_FP64 without
                              HP_STOP_REL_FRO_BOUND, HP_FLAG_SYMMETRIC or
                              chop (HP_EUNSUPPORTED otherwise); batched and
                              served solves ignore it. 0: one host read per
                              loop */
    double chop;           /* > 0: at the end of every loop, entries of X_{k+1}
                              with |x| < chop are set to zero before the
                              stopping test measures the change (the sparsity
                              control of Example 8.3); 0 = off. hp_solve with
                              HP_PREC_FP64 or HP_PREC_FP32 and a stopping rule
                              other than HP_STOP_REL_FRO_BOUND only
                              (HP_EUNSUPPORTED otherwise) */
    int32_t reserved[2];   /* must be zero */
} hp_params;

#define HP_HIST 128

typedef struct hp_result {
    int32_t status;        /* as returned */
    int32_t iters;         /* loops run, including the one whose test passed */
    int32_t switch_iter;   /* first loop run stabilised; -1 if none */
    int32_t side_used;     /* HP_SIDE_RIGHT or HP_SIDE_LEFT */
    int32_t gemms;         /* GEMM launches, set-up included */
    int32_t iters_stage[3];/* loops run in the 16-bit, FP32 and FP64 stages */
    double alpha;          /* the alpha of X0 = alpha*G that was used */
    double d_last;         /* last relative Frobenius change */
    double stop_last;      /* last value of the stopping rule's quantity */
    double coc;            /* computational order of convergence (COC) from
                              the last three inf-norm changes; 0 if unknown */
    double gflop;          /* executed GEMM work, 2*M*N*K per launch, GFLOP */
    double time_ms;        /* host wall time of the call */
    double gemm_ms;        /* summed GEMM kernel time (HP_FLAG_TIME_KERNELS) */
    double d_stage[3];     /* last relative change in each stage */
    double gflop_stage[3]; /* executed GEMM work per stage (set-up in stage 2) */
    double queue_ms;       /* served requests: submit -> admission */
    double run_ms;         /* served requests: admission -> result written */
    double d_hist[HP_HIST];    /* relative Frobenius change per loop */
    double dinf_hist[HP_HIST]; /* inf-norm change per loop (HP_FLAG_INF_NORM) */
    int32_t gemms_sym;     /* launches of those that ran symmetric (hp_gemm_sym) */
    int32_t reserved_r;
    double gflop_sym;      /* their work, N*(N+1)*K per launch (included in gflop) */
    double gemm_ms_sym;    /* their kernel time (HP_FLAG_TIME_KERNELS; included
                              in gemm_ms) */
    int32_t iters_delta;   /* loops whose polynomial ran in the delta form */
    int32_t reserved_r2;
    double gflop_engine[3];   /* executed GEMM work by MFMA path: 16-bit
                                 operands, FP32, FP64 (included in gflop) */
    double gemm_ms_engine[3]; /* their kernel time (HP_FLAG_TIME_KERNELS) */
} hp_result;

typedef struct hp_handle hp_handle;

/* ABI version (HP_ABI_VERSION). */
int hp_version(void);

/* Static text for a status code. Never NULL. */
const char* hp_status_string(int status);

/* Fill *p with defaults: Moore-Penrose, alpha 1/(||A||_1||A||_inf), plain
   variant, tau_switch 0.1, tol 1e-12, max_iter 100, relative Frobenius stop,
   side AUTO, FP64. */
void hp_params_default(hp_params* p);

/* Create a handle bound to HIP device `device` (pinned host scratch and
   events are allocated here; no matrix memory). */
int hp_create(hp_handle** h, int device);
int hp_destroy(hp_handle* h);

/* Bytes of device workspace hp_solve needs for this shape and these params. */
int hp_workspace_bytes(const hp_params* p, int64_t m, int64_t n, size_t* bytes);

/* Compute X (n x m, row-major, leading dimension ldx >= m) ~ A^(2)_{R(G),N(G)}
 * for A (m x n, leading dimension lda >= n).
 *  X0: optional device n x m start (leading dimension ldx0); NULL = the rule
 *      in p->alpha_rule (G = A^T for Moore-Penrose, A^l for Drazin). With an
 *      explicit X0, p->alpha (if > 0) is used only by HP_STOP_PAPER_4_1.
 *  workspace: >= hp_workspace_bytes, 256-byte aligned device memory.
 *  out: optional host struct filled on every return >= 0.
 * Errors: HP_EINVAL for m or n outside [1, 65535], Drazin with m != n or l < 1, ld below the
 * column count, a misaligned pointer, or an unknown enum; HP_EWORKSPACE;
 * HP_EHIP. */
int hp_solve(hp_handle* h, const hp_params* p,
             const double* A, int64_t m, int64_t n, int64_t lda,
             const double* X0, int64_t ldx0,
             double* X, int64_t ldx,
             void* workspace, size_t ws_bytes,
             void* stream, hp_result* out);

/* hp_solve for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, with the workspace taken from a fixed array of
 * HP_NOALLOC_SCRATCH_BYTES bytes that the library's device code object holds
 * on each device it runs on, from the first hp_create on that device until
 * the process ends. Arguments and results are those of hp_solve without
 * `workspace`/`ws_bytes`; the caller still passes A, X0 and X. Allocates
 * nothing (no hipMalloc, hipFree or allocating library call). Every call on
 * one device shares that device's array: calls that overlap on a device
 * (another stream, another host thread, another handle) race and must not
 * be issued; a call leaves the array's contents behind, and the next call
 * does not depend on them.
 * Errors: as hp_solve; HP_EWORKSPACE when hp_workspace_bytes(p, m, n)
 * exceeds HP_NOALLOC_SCRATCH_BYTES (e.g. 200 x 100 FP64 needs 1.2 MiB,
 * 512 x 512 FP64 22 MiB, 1024 x 1024 FP64 121 MiB: too large). */
#define HP_NOALLOC_SCRATCH_BYTES (64u << 20)
int hp_solve_noalloc(hp_handle* h, const hp_params* p,
                     const double* A, int64_t m, int64_t n, int64_t lda,
                     const double* X0, int64_t ldx0,
                     double* X, int64_t ldx,
                     void* stream, hp_result* out);

/* Complex A (m x n, interleaved real and imaginary doubles, leading dimension
 * lda >= n in complex elements): X (n x m, interleaved, ldx >= m) ~ the
 * generalized inverse hp_solve defines, with G = A^* (conjugate transpose)
 * for Moore-Penrose and A^l for Drazin (Section 1.2 states the method for
 * complex matrices). Computed through the real 2m x 2n matrix
 * [[Re A, -Im A], [Im A, Re A]]: that map turns products into products and
 * A^* into the transpose, so the loop on it is the complex loop, twice the
 * flops of a complex-arithmetic GEMM. m, n <= 32767; no X0 argument (the
 * rule in p->alpha_rule; alpha from the norms of the real form, which has
 * the singular values of A, each twice). hp_params.chop acts on real and
 * imaginary parts separately (as Chop does on complex numbers). Drazin only
 * with HP_ALPHA_USER and no HP_ALPHA_DIAG (HP_EUNSUPPORTED: those rules of the
 * real form are not the complex rules). Errors as hp_solve. */
int hp_complex_workspace_bytes(const hp_params* p, int64_t m, int64_t n, size_t* bytes);
int hp_solve_complex(hp_handle* h, const hp_params* p, const double* A, int64_t m, int64_t n,
                     int64_t lda, double* X, int64_t ldx, void* workspace, size_t ws_bytes,
                     void* stream, hp_result* out);


/* One matrix product on the library's MFMA GEMM kernel, exposed so that the
 * kernel can be checked and timed on its own:
 *     C = alpha * A B + beta_identity * I      (A M x K, B K x N, C M x N)
 * dtype HP_DTYPE_F64 (A, B, C double) or HP_DTYPE_F32 / HP_DTYPE_BF16_F32 /
 * HP_DTYPE_F16_F32 (A, B, C float). Pointers
 * must be 16-byte aligned and the rows of A and B must start on 16-byte
 * boundaries (lda, ldb multiples of 16 bytes).
 * Errors: HP_EINVAL (shape, ld, alignment, dtype), HP_EHIP. */
int hp_gemm(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K,
            double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
            double beta_identity, void* C, int64_t ldc, void* stream);

/* Workspace that lets hp_gemm_ws split K over several blocks per output tile
 * (the split-K tiles, chosen for products with too few 128 x 128 output tiles
 * to occupy every compute unit); 0 when the product would not split. */
int hp_gemm_workspace_bytes(int dtype, int64_t M, int64_t N, int64_t K, size_t* bytes);

/* hp_gemm with a workspace (device memory, 256-byte aligned). With at least
 * hp_gemm_workspace_bytes for the tile the handle chooses, a split tile stores
 * its partial tiles there and the last block of each output tile adds them in
 * a fixed order, so the result is the same from run to run; with less (or
 * NULL and 0) the product runs unsplit. The workspace's counters are cleared
 * on the stream by every call; calls that share a workspace must not overlap.
 * Errors: as hp_gemm (a misaligned workspace is HP_EINVAL). */
int hp_gemm_ws(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K,
               double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
               double beta_identity, void* C, int64_t ldc, void* workspace, size_t ws_bytes,
               void* stream);

/* Workspace of hp_gemm_sym for an N x N x K product: partial tiles for the
 * blocks that share an output tile, and arrival counters (the size depends on
 * the current device's compute-unit count; 0 when no device is visible, and
 * hp_gemm_sym then forms the full product). dtype HP_DTYPE_F64 or F32.
 * Errors: HP_EINVAL for another dtype, N or K outside [1, 2^24], NULL bytes. */
int hp_gemm_sym_workspace_bytes(int dtype, int64_t N, int64_t K, size_t* bytes);

/* C = alpha A B + beta_identity I (N x N) for a product that the caller knows
 * to be symmetric in exact arithmetic, such as G G^T or a polynomial in a
 * symmetric matrix (the loop products of Section 2 when X A or A X is
 * symmetric). Only the output tiles on and above the diagonal are computed,
 * in one launch that gives every block an equal share of their K-steps; a
 * tile shared by several blocks is finished by the last of them, which adds
 * the pieces in K order (the same result from run to run). Each element
 * (i, j), i <= j, is formed once and stored at (i, j) and (j, i), so C is
 * exactly symmetric; its upper triangle equals the full product's up to the
 * rounding of the summation order. dtype HP_DTYPE_F64 or HP_DTYPE_F32; A, B,
 * lda, ldb, C, ldc as for hp_gemm (A N x K, B K x N). With a workspace of
 * fewer than hp_gemm_sym_workspace_bytes (or NULL and 0) the full product is
 * formed instead. The workspace's counters are cleared on the stream by every
 * call; calls that share a workspace must not overlap.
 * Errors: as hp_gemm; another dtype or a misaligned workspace is HP_EINVAL. */
int hp_gemm_sym(hp_handle* h, int dtype, int64_t N, int64_t K, double alpha, const void* A,
                int64_t lda, const void* B, int64_t ldb, double beta_identity, void* C,
                int64_t ldc, void* workspace, size_t ws_bytes, void* stream);

/* ---- residuals of the defining equations ---------------------------------- */

/* Workspace for hp_residuals. */
int hp_residuals_workspace_bytes(int kind, int l, int64_t m, int64_t n, size_t* bytes);

/* Relative residuals, in FP64 on the GPU, of the equations that define the
 * inverse X (n x m) of A (m x n), Frobenius norms:
 *  HP_KIND_MOORE_PENROSE (the four Penrose equations):
 *    out[0] = ||AXA - A||/||A||, out[1] = ||XAX - X||/||X||,
 *    out[2] = ||AX - (AX)^T||/||AX||, out[3] = ||XA - (XA)^T||/||XA||;
 *  HP_KIND_DRAZIN (m == n, l >= ind(A); Section 1.2):
 *    out[0] = ||A^{l+1} X - A^l||/||A^l||, out[1] = ||XAX - X||/||X||,
 *    out[2] = ||AX - XA||/||AX||, out[3] = 0.
 * A, X: device, row-major, lda >= n, ldx >= m, 16-byte aligned with lda and
 * ldx even. out: host array of 4. Synchronises the stream. Errors: HP_EINVAL,
 * HP_EWORKSPACE, HP_EHIP. */
int hp_residuals(hp_handle* h, int kind, int l, const double* A, int64_t m, int64_t n, int64_t lda,
                 const double* X, int64_t ldx, void* workspace, size_t ws_bytes, void* stream,
                 double out[4]);

/* ---- tile autotuning ------------------------------------------------------ */

/* Scratch hp_autotune needs for this product: the operands and result
 * (rows padded to 16 bytes) and the split-K scratch of the split tiles. */
int hp_autotune_scratch_bytes(int dtype, int64_t M, int64_t N, int64_t K, size_t* bytes);

/* Time every tile configuration of the GEMM kernel for dtype on an M x N x K
 * product (operands filled by the library in `scratch`, device memory of at
 * least hp_autotune_scratch_bytes, 16-byte aligned), `reps` timed launches
 * each after one warm-up, and record the fastest in the handle: later
 * products of exactly this (dtype, M, N, K) use it. Returns the chosen tile
 * index and its mean launch time. The environment variable HP_GEMM_TILE, if
 * set, still overrides every choice. Errors: HP_EINVAL, HP_EWORKSPACE (scratch
 * too small), HP_EHIP. */
int hp_autotune(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, void* scratch,
                size_t scratch_bytes, int reps, void* stream, int* tile, double* ms);

/* The handle's table as rows of 5 int64 (dtype, M, N, K, tile): export
 * copies up to `cap` rows and reports the count; import adds rows (all are
 * checked first: HP_EINVAL and nothing added if one has an unknown dtype or
 * a tile out of range). A grouped row (HP_DTYPE_GROUPED_*) also sets the
 * grouped tile of its precision for groups created afterwards, whatever its
 * sizes; the latest grouped row imported or autotuned wins. */
int hp_tune_export(hp_handle* h, int64_t* rows, int cap, int* count);
int hp_tune_import(hp_handle* h, const int64_t* rows, int count);

/* ---- many problems: batched and served forms --------------------------- */

/* One matrix of a batch or one served request. A (m x n, lda) and the
 * optional X0 (n x m, ldx0) are read-only device memory; X (n x m, ldx) is
 * written when the problem finishes. All three stay owned by the caller and
 * must stay valid until then. */
typedef struct hp_problem {
    const double* A;
    int64_t m, n, lda;
    const double* X0;
    int64_t ldx0;
    double* X;
    int64_t ldx;
} hp_problem;

/* Workspace for hp_solve_batched over these problems. */
int hp_batched_workspace_bytes(const hp_params* p, int count, const hp_problem* probs,
                               size_t* bytes);

/* Solve `count` problems of uneven shapes with the same params. Every loop
 * runs each product of all unfinished problems in one persistent grouped MFMA
 * launch (tiles walked from a device-side table; 64x64 unless hp_autotune or
 * hp_tune_import chose another grouped tile for the precision); each problem
 * stops on its own test. A problem's result is bitwise the same whatever else is in
 * the batch. Precision HP_PREC_FP64, HP_PREC_FP32 or HP_PREC_FP32_FP64;
 * stop rules REL_FRO and PAPER_4_1. outs: `count` results (may be NULL).
 * Returns HP_OK if the call ran (see each outs[i].status), else an error. */
int hp_solve_batched(hp_handle* h, const hp_params* p, int count, const hp_problem* probs,
                     void* workspace, size_t ws_bytes, void* stream, hp_result* outs);

/* Continuous-batching server. Requests are queued by hp_serve_submit and
 * admitted in arrival order while a slot is free and their workspace fits in
 * the server's HBM budget (allocated once here); each hp_serve_step admits
 * what fits, runs one loop of every admitted request (grouped launches as in
 * hp_solve_batched, so a request's result does not depend on its neighbours),
 * and retires the requests that finished, writing their X and freeing their
 * memory. Not thread-safe. */
typedef struct hp_server hp_server;
int hp_serve_create(hp_handle* h, const hp_params* p, size_t hbm_budget, int max_slots,
                    void* stream, hp_server** out);
/* HP_EBUDGET if the request alone exceeds the budget, HP_EINVAL for a bad
 * shape; otherwise queues it and returns a ticket. */
int hp_serve_submit(hp_server* sv, const hp_problem* prob, uint64_t* ticket);
/* One scheduling step; reports the requests running and waiting after it
 * (either pointer may be NULL). A request whose solve with lower-precision
 * loops ends with a status other than HP_OK is run again once, from its X0,
 * in FP64 only (in its own arena space; its result then reports that run),
 * unless HP_FLAG_NO_RETRY is set. A request whose set-up on admission (or on
 * that rerun) fails is finished with the error, which hp_serve_poll then
 * returns; its slot and memory are freed. A negative return is the first
 * error of the step (the rest of the step still ran); after HP_EHIP the
 * device may be unusable: destroy the server. */
int hp_serve_step(hp_server* sv, int* active, int* waiting);
/* HP_PENDING while the request is queued or running; afterwards its final
 * status, or the negative error that ended it (out filled, ticket released).
 * HP_EINVAL for an unknown ticket. */
int hp_serve_poll(hp_server* sv, uint64_t ticket, hp_result* out);
int hp_serve_destroy(hp_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* HYPERPOWER_H */
