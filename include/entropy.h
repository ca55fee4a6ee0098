/*
 * entropy.h -- C ABI of libentropy, an MI355X (gfx950) library for the
 * randomized von Neumann entropy estimators of Kontopoulou, Dexter,
 * Szpankowski, Grama and Drineas (arXiv:1801.01072).
 *
 * Problem (Section 1.1, eqns. (1)-(4)): R is a real symmetric positive
 * semidefinite n x n matrix with unit trace; H(R) = -sum_i p_i ln p_i =
 * -tr(R ln R), p_i the eigenvalues of R, with 0 ln 0 = 0.
 *
 * Conventions for every entry point
 *  - Nothing throws across this boundary.  Every call returns an ent_status;
 *    on failure the status is negative, ent_last_error() describes it, and
 *    the output structures are left untouched.
 *  - Matrices are passed by descriptor (ent_matrix).  Their arrays live in
 *    device memory of the current HIP device, or in host memory: the single-
 *    matrix calls (ent_entropy_estimate(_detail), ent_power_method,
 *    ent_selector_features) first copy every array that lies in host memory
 *    (pageable or pinned) to a library-owned device buffer, the extent the
 *    descriptor states ((n - 1) ld + n elements dense; n + 1, nnz, nnz CSR),
 *    on the call's stream.  That buffer is kept per device for later calls
 *    (released by ent_release_workspace(), counted against the workspace
 *    limit); host extents cannot be checked and are the caller's contract.
 *    The caller owns R and the library never retains a pointer past the call.
 *    Before any kernel runs, each call checks every device array it is given
 *    (matrix arrays, and the device arrays of the MLP calls): memory of
 *    another device is ENT_EINVAL, and so is a descriptor whose extent runs
 *    past the end of the allocation the pointer lies in (where the runtime
 *    reports one).  The batched calls take device (or pinned, device-
 *    readable) arrays only.
 *  - Scalar results are returned in host structures / host arrays owned by
 *    the caller.
 *  - Work is enqueued on opt->stream (a hipStream_t; NULL = the legacy
 *    default stream).  Estimating calls synchronise that stream before they
 *    return.  Distinct threads may call concurrently on distinct streams.
 *  - Workspace (probe blocks, recurrence buffers, partial sums) is owned by
 *    the library, cached per device between calls and released by
 *    ent_release_workspace().  ent_set_workspace_limit() caps it; a call
 *    that would exceed the cap returns ENT_ENOMEM.  A CSR R served by the
 *    banded kernels (ENT_FLAG_CSR_GENERAL, ENT_FLAG_CSR_BANDED) adds its slab
 *    copy to the workspace: 16 + 2 hp values of the compute type per row,
 *    rounded up to 16 rows, rebuilt by every call and never kept past it;
 *    a tridiagonal CSR R its three diagonals (4 values per row, likewise;
 *    Chebyshev: a second copy, the prepared 2X).  The multi-step kernels
 *    (banded FP32 pairs; tridiagonal launches of several steps) add two V
 *    blocks, except a tridiagonal forward estimate whose steps all fit in
 *    one launch; where the additional blocks do not fit, the call runs one
 *    step per launch instead of returning ENT_ENOMEM.
 */
#ifndef ENTROPY_H
#define ENTROPY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ENT_OK = 0,
  ENT_EINVAL = -1,       /* null or inaccessible pointer, descriptor past its
                            allocation, malformed CSR structure, size < 1,
                            unknown enum, bad layout                         */
  ENT_ENOTDENSITY = -2,  /* |tr R - 1| above tolerance (see ent_options), or
                            tr R <= 0 with ENT_FLAG_NORMALIZE              */
  ENT_ENOMEM = -3,       /* device allocation failed or workspace cap reached */
  ENT_EDEVICE = -4,      /* a HIP runtime call failed                          */
  ENT_ENUMERIC = -5,     /* p~1 <= 0, or a non-finite estimate                 */
  ENT_EUNSUPPORTED = -6  /* valid request the library does not implement      */
} ent_status;

/* Estimator (Algorithm 1 = Taylor, Section 2; Algorithm 2 = Chebyshev,
 * Section 3; Algorithm 3 = random projection, Section 5). */
typedef enum {
  ENT_TAYLOR = 0,
  ENT_CHEBYSHEV = 1,
  ENT_RANDPROJ = 2,
  ENT_AUTO = 3      /* learned degree / cutoff selector (see ent_selector_load) */
} ent_method;

/* Arithmetic of the recurrence products R.V.  The power method, the
 * coefficients and every reduction are always FP64. */
typedef enum {
  ENT_F64 = 0,    /* FP64 MFMA                                              */
  ENT_F32 = 1,    /* FP32 MFMA                                              */
  ENT_BF16X3 = 2  /* three BF16 MFMA products (hi.hi + hi.lo + lo.hi) with
                     FP32 accumulation; dense only                          */
} ent_precision;

typedef enum { ENT_DENSE = 0, ENT_CSR = 1 } ent_layout;

/* Storage type of a matrix (independent of the compute precision).  The
 * complex types hold a Hermitian density matrix (Section 4) as interleaved
 * (real, imaginary) pairs; they are accepted by ent_entropy_estimate(_detail)
 * and ent_power_method, dense layout only. */
typedef enum {
  ENT_STORE_F64 = 0,
  ENT_STORE_F32 = 1,
  ENT_STORE_C128 = 2,  /* complex double */
  ENT_STORE_C64 = 3    /* complex float  */
} ent_dtype;

/* Probe vectors g_1..g_s: the paper draws standard Gaussians (Lemma 1);
 * Rademacher signs are the other unbiased choice. */
typedef enum { ENT_RADEMACHER = 0, ENT_GAUSSIAN = 1 } ent_probe_dist;

/* Sketch Pi (n x s) of Algorithm 3 (Section 5.2).  Random draws are
 * Philox4x32-10 with counter (row mod 2^32, 0, stream, row >> 32), key =
 * seed:
 *  GAUSSIAN: Pi_jt = N(0,1)/sqrt(s), the probe generator's Gaussian of
 *            stream 2 at (row j, probe t).
 *  SRHT:     subsampled randomized Hadamard transform sqrt(N/s) D H S,
 *            N = 2^ceil(log2 n), H the normalized Sylvester-Hadamard
 *            matrix: Pi_jt = D_jj (-1)^popcount(j & i_t) / sqrt(s).
 *  COUNT:    input-sparsity transform D S: row j holds D_jj in column h(j)
 *            only.  R Pi is one signed pass over R (FP64 sums of the stored
 *            values; the precision option does not apply).
 * D_jj = -1 iff bit 0 of output word 0 of stream 3 at row j; h(j) =
 * floor(w1 s / 2^32), w1 output word 1 of that block; i_t = output word 0
 * of stream 4 at row t, modulo N. */
typedef enum { ENT_SKETCH_GAUSSIAN = 0, ENT_SKETCH_SRHT = 1, ENT_SKETCH_COUNT = 2 } ent_sketch;

enum {
  ENT_FLAG_SKIP_TRACE_CHECK = 1, /* do not verify tr R = 1                    */
  ENT_FLAG_AUTOTUNE = 2,         /* batches: time the candidate tile shapes on
                                    the batch if no cached choice exists      */
  ENT_FLAG_COMPLEX_POWER = 4,    /* Hermitian R: u = min{1, c p~1} from the
                                    power method instead of the paper's u = 1 */
  ENT_FLAG_CLENSHAW = 8,         /* Chebyshev: evaluate g^T f_m(R) g by the
                                    backward Clenshaw recurrence (Algorithm 5,
                                    Appendix B) instead of the forward three-
                                    term recurrence; see ent_entropy_estimate */
  ENT_FLAG_CSR_GENERAL = 16,     /* CSR R: always the general CSR kernels.  By
                                    default an R whose entries all lie within
                                    one of the diagonal (tridiagonal, at most
                                    3n entries) runs the tridiagonal kernels
                                    (steps and power method) on a
                                    per-estimate copy of its three diagonals,
                                    and one whose entries all lie
                                    within 16 of the diagonal the banded kernels
                                    (steps and power method) on a per-estimate
                                    copy of R in 16-row slabs of 16 + 2 hp
                                    values per row (hp = 4, 8 or 16, the half-
                                    bandwidth rounded up) when that copy has no
                                    more bytes per row than the CSR arrays;
                                    same results within rounding             */
  ENT_FLAG_CSR_BANDED = 32,      /* CSR R within 16 of the diagonal: the banded
                                    kernels whatever the byte counts (also for
                                    a tridiagonal R)                          */
  ENT_FLAG_NORMALIZE = 64,       /* estimate H(R / tr R) instead of requiring
                                    tr R = 1 (Section 1.1: a density matrix
                                    has unit trace).  tr R is computed on the
                                    device (Re tr R for Hermitian storage) and
                                    folded into the product scale, p~1 and the
                                    singular values; R itself is not modified
                                    or copied.  p1_est and u are those of
                                    R / tr R.  tr R <= 0 or non-finite is
                                    ENT_ENOTDENSITY.  Overrides
                                    ENT_FLAG_SKIP_TRACE_CHECK and trace_tol.  */
  ENT_FLAG_BATCH_STEPWISE = 128, /* batches: one grouped launch per recurrence
                                    step instead of the persistent schedule
                                    (see ent_graph_create)                   */
  ENT_FLAG_AUTO_RANDPROJ = 256   /* ENT_AUTO: route an R whose sketch looks
                                    numerically low-rank to Algorithm 3      */
};

/*
 * A density matrix on the device.
 *  layout ENT_DENSE: values -> n x n row-major, leading dimension ld >= n
 *                    elements; row_ptr/col_idx/nnz ignored.
 *  layout ENT_CSR:   row_ptr -> int64[n+1] (row_ptr[0] = 0, non-decreasing,
 *                    row_ptr[n] = nnz), col_idx -> int32[nnz] in [0, n),
 *                    values -> nnz entries; ld ignored.
 *  dtype: ENT_STORE_F64 (double) or ENT_STORE_F32 (float) values; or, dense
 *         only, ENT_STORE_C128 / ENT_STORE_C64: n x n complex entries as
 *         interleaved (re, im) pairs, ld counted in complex entries.
 * R must be symmetric (Hermitian for the complex types); this is not checked
 * (an asymmetric R is used as given in the products R.v).
 */
typedef struct {
  int64_t n;
  int32_t layout;
  int32_t dtype;
  int64_t ld;
  int64_t nnz;
  const void *values;
  const int64_t *row_ptr;
  const int32_t *col_idx;
} ent_matrix;

typedef struct {
  int32_t power_iters;   /* t of Algorithm 4 (default 20)                      */
  int32_t power_trials;  /* q of Algorithm 4 (default 1)                       */
  double u_factor;       /* c in u = min{1, c p~1} (Algorithms 1-2: c = 6)     */
  double u_fixed;        /* > 0: use this u and skip the power method          */
  double cutoff;         /* lower end lo of the Chebyshev interval [lo, u];
                            0 = the paper's [0, u] with the Lemma 3 closed
                            form; > 0 = Chebyshev projection of x ln x on
                            [lo, u] (1024-node Gauss-Chebyshev rule)         */
  int32_t precision;     /* ent_precision (default ENT_F64)                    */
  int32_t probe_dist;    /* ent_probe_dist (default ENT_RADEMACHER)            */
  int32_t rank_k;        /* Algorithm 3: number of singular values kept        */
  int32_t sketch_width;  /* Algorithm 3: columns s of the Gaussian sketch      */
  int32_t flags;         /* ENT_FLAG_* bits                                    */
  int32_t sketch;        /* Algorithm 3: ent_sketch (default ENT_SKETCH_GAUSSIAN) */
  double trace_tol;      /* |tr R - 1| tolerance; 0 = 1e-10 (F64 storage) or
                            1e-4 (F32 storage)                                 */
  void *stream;          /* hipStream_t                                        */
} ent_options;

typedef struct {
  double entropy;   /* H^: mean of the per-probe values h_j                   */
  double std_err;   /* standard error of that mean over the probes           */
  double p1_est;    /* p~1 from the power method (0 if u_fixed was given)    */
  double u;         /* upper end of the approximation interval               */
  double lo;        /* lower end of the approximation interval               */
  int32_t degree;   /* m actually used                                       */
  int32_t probes;   /* s actually used                                       */
  int32_t method;   /* ent_method actually run                               */
  int32_t precision;
  int32_t fell_back; /* ENT_AUTO: 1 if the a-posteriori check failed and the
                        plain schedule was run                                */
  int32_t products;  /* R.V products of the recurrence (all passes)          */
} ent_result;

/* Fill *opt with the defaults listed above. */
void ent_options_default(ent_options *opt);

/*
 * One estimate of H(R) (Algorithms 1 and 2, with Algorithm 4 for p~1).
 *   method  ENT_TAYLOR:    h_j = ln(1/u) + sum_{k=1}^{m} g_j^T R (I - R/u)^k g_j / k
 *           ENT_CHEBYSHEV: h_j = -g_j^T f_m(R) g_j, f_m = sum_w alpha_w T_w
 *                          on [lo, u] (Lemma 3 coefficients when lo = 0)
 *           ENT_RANDPROJ:  Algorithm 3 with the sketch opt->sketch of
 *                          opt->sketch_width columns, top opt->rank_k
 *                          singular values (degree and probes ignored)
 *   degree  m >= 1; probes s >= 1; seed keys the Philox4x32-10 stream of
 *   probes (stream 0), power-method start vectors (stream 1) and sketch
 *   entries (stream 2).
 * opt may be NULL (defaults).  Returns ENT_EINVAL for bad arguments,
 * ENT_ENOTDENSITY if the trace check fails, ENT_ENUMERIC if p~1 <= 0 or the
 * estimate is not finite.
 *
 * ENT_FLAG_CLENSHAW (Chebyshev, single estimates): y_{m+1} = y_{m+2} = 0,
 * y_k = alpha_k g + 2 X y_{k+1} - y_{k+2} for k = m..0 (m + 1 products, the
 * first on y_{m+1} = 0), and g^T f_m(R) g = (alpha_0 g^T g + g^T y_0 -
 * g^T y_2) / 2.  The same estimate as the forward recurrence up to rounding;
 * the moment table then holds g_j^T y_k (k = 0..m) instead of d_{k,j}.
 *
 * Hermitian R (complex storage; Section 4, Algorithms 1c and 2c): the same
 * estimators with h_j = ln(1/u) + sum_k g_j^T Re[R (I - R/u)^k] g_j / k and
 * h_j = -g_j^T Re[f_m(R)] g_j for real probes g_j.  u = 1 as in the paper
 * (no power method) unless opt->u_fixed > 0 or ENT_FLAG_COMPLEX_POWER is set.
 * They run on the real 2n x 2n form [[Re R, -Im R], [Im R, Re R]], built in
 * a library-owned device buffer of 4 n^2 doubles (C128) or floats (C64) that
 * is kept for later calls and released by ent_release_workspace(), with
 * probes [g; 0]; every precision applies.  The trace check is on Re tr R.
 * ENT_RANDPROJ and ENT_AUTO return ENT_EUNSUPPORTED.
 */
ent_status ent_entropy_estimate(const ent_matrix *R, int32_t method, int32_t degree,
                                int32_t probes, uint64_t seed, const ent_options *opt,
                                ent_result *out);

/*
 * Same as ent_entropy_estimate, and also copies per-probe detail to host
 * arrays the caller owns (either may be NULL):
 *   per_probe[j]            = h_j, j < probes
 *   moments[k * probes + j] = Chebyshev: d_{k,j} = g_j^T T_k(X) g_j, k = 0..m,
 *                             X = (2R - (u+lo)I)/(u-lo);
 *                             Taylor: e_{k,j} = g_j^T (R/u)(I - R/u)^k g_j,
 *                             k = 0..m.
 * moments holds (degree + 1) * probes doubles.  ENT_AUTO: the moments of the
 * pass that produced the result (its degree is out->degree), rows k <=
 * min(out->degree, degree); any later rows are set to zero.
 * Used for per-probe parity checks.  RANDPROJ: per_probe[i] = the i-th kept
 * singular value (rank_k entries); moments unused.
 */
ent_status ent_entropy_estimate_detail(const ent_matrix *R, int32_t method, int32_t degree,
                                       int32_t probes, uint64_t seed, const ent_options *opt,
                                       ent_result *out, double *per_probe, double *moments);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Taylor / Chebyshev estimate as ent_entropy_estimate_detail (same kernels,
 * same results), with every workspace buffer carved from a fixed device
 * array of ENT_NOALLOC_SCRATCH_BYTES compiled into the library -- one copy
 * per GPU, held from the library's load until the process ends -- instead of
 * the cached workspace.  No hipMalloc, hipFree or allocating library routine
 * is called, and no phase events are recorded (ent_timing is not updated).
 *  - R must be real (ENT_STORE_F64 / ENT_STORE_F32), dense or CSR, with
 *    every array in device memory of the current device (host arrays would
 *    need a device copy): ENT_EINVAL otherwise.  Hermitian storage,
 *    ENT_RANDPROJ and ENT_AUTO: ENT_EUNSUPPORTED.
 *  - An estimate whose workspace exceeds ENT_NOALLOC_SCRATCH_BYTES returns
 *    ENT_ENOMEM (the message states both sizes) before any kernel runs.
 *    Dense FP64 at n = 8192 with 256 probes and degree 50 needs about 64 MB.
 *  - Every call on one GPU uses that GPU's one array, and the next call
 *    overwrites what the last one left there; the library runs such calls
 *    one at a time (a per-device lock held until the call has synchronised
 *    its stream).  Work enqueued on the same memory by other means would
 *    race with it.
 * Arguments, outputs and errors otherwise as ent_entropy_estimate_detail.
 */
#define ENT_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
ent_status ent_entropy_estimate_noalloc(const ent_matrix *R, int32_t method, int32_t degree,
                                        int32_t probes, uint64_t seed, const ent_options *opt,
                                        ent_result *out, double *per_probe, double *moments);

/*
 * Algorithm 4 (Appendix A): q trials of t power iterations from random sign
 * vectors, each iterate divided by its 2-norm, Rayleigh quotient of the last
 * iterate, maximum over trials.  *p1 (host) receives p~1.  Hermitian R: the
 * iteration runs on the real form, i.e. on the complex iterate
 * x_i = s_i + i s_{n+i} (s the 2n signs of stream 1).
 */
ent_status ent_power_method(const ent_matrix *R, int32_t t, int32_t q, uint64_t seed,
                            void *stream, double *p1);

/*
 * Chebyshev coefficients alpha_0..alpha_m of x ln x on [lo, u], computed in
 * FP64 on the device and copied to alpha (host, m+1 entries).  lo = 0: the
 * closed form of Lemma 3; lo > 0: the projection by the 1024-node
 * Gauss-Chebyshev rule (2(m+1) nodes beyond degree 511).  Requires
 * 0 <= lo < u, m >= 1.
 */
ent_status ent_chebyshev_coeffs(double lo, double u, int32_t m, double *alpha);

/*
 * Learned degree / lower-cutoff selector (not in the paper; the extension of
 * the plain schedule of Theorem 2).  A 16-64-64-2 ReLU MLP in FP32 maps 16
 * features of a cheap sketch -- the power method and a degree-12 Chebyshev
 * moment pass with 16 Rademacher probes on [0, u] -- to (ln m, log10(lo/u)).
 *
 * ent_selector_load: copies the parameters (host, ent_mlp_nparams() floats,
 *   layout W1[64][16], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]) to the
 *   current device.
 * ent_entropy_estimate with method ENT_AUTO: runs the sketch pass.  With
 *   ENT_FLAG_AUTO_RANDPROJ and a dense R whose sketch rank n (1 - mean h(X)),
 *   h(X) = ((1 - X)/2)^12 from the normalised moments, is at most
 *   sketch_width / 8 (sketch_width 0: 128), Algorithm 3 (Section 5) runs
 *   with that width, k = rank_k (0: width / 2) and a Gaussian sketch, and its
 *   result is kept (result.method = ENT_RANDPROJ) if its k singular values
 *   sum to 1 (the unit trace) within 5%; else 1 more product is counted.  The sketch cannot tell zero eigenvalues from
 *   tiny ones (a spectrum p_i ~ i^-2 looks rank 6 to it), whose entropy
 *   Algorithm 3 misses, hence the flag.  Otherwise the network, then
 *   Chebyshev on [lo, u] with the predicted degree m.  The a-posteriori
 *   check requires every moment |d_kj| <= ||g_j||^2 (the spectrum inside
 *   the interval) and |H(m) - H(m-4)| <= 2.5e-4 |H(m)| (converged).  If
 *   only the second part fails, the same recurrence continues to
 *   ceil(1.5 m) and then ceil(2.25 m) (at most 511; ENT_F64 and ENT_F32 --
 *   the moments and the coefficients do not depend on the final degree, so
 *   only the new products are run) and is checked again; result.degree is
 *   the degree reached.  If the check still fails, the plain schedule on
 *   [0, u] with the caller's degree is run instead (result.fell_back = 1).
 *   result.products counts every product of every pass.
 * ent_selector_features: the sketch pass alone; features[16] (host) and, if
 *   outputs is non-NULL, the network's two outputs.
 * ent_mlp_forward / ent_mlp_grad / ent_mlp_train_epoch: the network's
 *   inference, gradient of the mean squared error L = (1/B) sum (y - t)^2,
 *   and minibatch Adam (beta1 0.9, beta2 0.999, eps 1e-8) over samples in
 *   order; all arrays are device pointers (X: count x 16, T and Y: count x 2),
 *   *step counts Adam steps and is advanced, *loss / *mean_loss are host.
 */
int32_t ent_mlp_nparams(void);
ent_status ent_mlp_forward(const float *params, const float *X, int32_t count, float *Y, void *stream);
ent_status ent_mlp_grad(const float *params, const float *X, const float *T, int32_t count,
                        float *grad, double *loss, void *stream);
ent_status ent_mlp_train_epoch(float *params, float *adam_m, float *adam_v, int32_t *step,
                               const float *X, const float *T, int32_t count, int32_t batch,
                               float lr, void *stream, double *mean_loss);
ent_status ent_selector_load(const float *params, int32_t nparams);
ent_status ent_selector_features(const ent_matrix *R, uint64_t seed, const ent_options *opt,
                                 float *features, float *outputs);

/* Parameter rules of the paper (host helpers, no device work). */
int32_t ent_probes_for(double eps, double delta);              /* ceil(20 ln(2/delta)/eps^2), Lemma 1     */
int32_t ent_degree_taylor(double u, double ell, double eps);   /* ceil((u/ell) ln(1/eps)), Theorem 1      */
int32_t ent_degree_chebyshev(double u, double ell, double eps);/* ceil(sqrt(u/(2 eps ell ln(1/(1-ell))))), Theorem 2 */
int32_t ent_power_trials_for(double delta);                    /* ceil(4.82 ln(1/delta)), Lemma 5         */
int32_t ent_power_iters_for(int64_t n);                        /* ceil(ln sqrt(4n)), Lemma 5              */

/*
 * Phase timing of the last estimate made on the calling thread, from HIP
 * events recorded on the estimate's stream between launches (only while
 * enabled on that thread; off by default).  For profiling: the events add a
 * few microseconds per launch.
 */
typedef struct {
  double total_ms;       /* first to last enqueued operation                  */
  double power_ms;       /* power method, all trials                          */
  double steps_ms;       /* the recurrence product kernels R.V, summed        */
  double step_max_ms;    /* longest single product launch                     */
  double epilogue_ms;    /* separate epilogue kernels (BF16x3 path), summed   */
  double other_ms;       /* probes, trace check, setup and reductions         */
  int32_t step_launches;
  int32_t power_launches; /* product launches of the power method: t + 1 per
                            trial, fewer for a banded or tridiagonal CSR R,
                            whose products after a trial's first run up to
                            ENT_POWER_FUSE (1..10, default 10) per launch  */
  int32_t epilogue_launches;
  int32_t csr_band;      /* CSR R: padded half-bandwidth (4, 8 or 16) of the
                            banded step kernel that ran, 1 for the
                            tridiagonal step kernel; 0: the general CSR
                            kernel or a dense path                            */
  int32_t steps_fused;   /* recurrence steps per product launch: 2 for the
                            banded FP32 two-step kernel (the last step of
                            an odd count runs alone, in other_ms;
                            ENT_BAND_PAIRS=0 runs one step per launch); for
                            the tridiagonal kernel the steps of the first
                            launch, the m steps split into launches of at
                            most ENT_TRI_FUSE steps (1..10, default 10) as
                            evenly as possible, longer first (a one-step
                            launch in other_ms); steps_ms and step_launches
                            then cover the multi-step launches; 1
                            otherwise, also where the two more V blocks
                            the multi-step launches need do not fit       */
} ent_timing;

ent_status ent_timing_enable(int32_t on);
ent_status ent_last_timing(ent_timing *out);

/*
 * Batches of dense density matrices (uneven n): every phase of the estimate
 * runs as one grouped launch over all matrices.  Matrix b uses probe seed
 * seed + b.  Precision ENT_F32, ENT_F64 or ENT_BF16X3 (probes <= 256);
 * storage of all matrices must be the same type.  Each matrix is copied into
 * an aligned compute-type buffer (BF16x3: split into bf16 hi/lo) at the start
 * of every run, so later changes of the caller's values are seen by the next
 * launch; the caller's pointers must stay valid while a graph exists.
 *
 * ent_entropy_estimate_batched: one synchronous run; outs[count].
 * ent_graph_create: plans the batch (workspace, descriptor and tile tables,
 *   tile shape and step schedule -- from the autotune cache, or timed on the
 *   batch when ENT_FLAG_AUTOTUNE is set; the cache persists as JSON in the
 *   file named by the environment variable ENT_AUTOTUNE_CACHE), then captures
 *   the whole launch sequence into a hipGraph on a private stream.
 *   The m recurrence steps of every matrix run by default as ONE persistent
 *   launch: its workgroups (as many as are resident at once) take (matrix,
 *   row tile, step) items from a device schedule.  Each matrix belongs to one
 *   XCD and only workgroups on that XCD take its items; per XCD, matrices of
 *   decreasing n enter a window of bounded bytes (1 GB over all XCDs by
 *   default) and advance one step per round.  An item waits until every tile
 *   of its matrix's previous step is done (per-matrix counters); each wait is
 *   bounded (environment variable ENT_SCHED_SPIN_LIMIT polls, default 2^20)
 *   and an expired wait, or an XCD's items left untaken, makes
 *   ent_graph_launch return ENT_EDEVICE.  With ENT_FLAG_BATCH_STEPWISE, or
 *   when the autotuner finds it faster, each step is one grouped launch over
 *   every tile instead.  Both give bit-identical results.
 * ent_graph_launch: replays the graph, synchronises, fills outs[count].
 * ent_graph_per_probe: h_j of the last launch, per_probe[count * probes].
 * ent_graph_time_eager: runs the same sequence without the graph, recording
 *   phase events (for profiling), fills outs and *timing.
 * ent_graph_destroy: releases the graph, its workspace and stream.
 */
typedef struct ent_graph_s *ent_graph;
ent_status ent_entropy_estimate_batched(const ent_matrix *Rs, int32_t count, int32_t method,
                                        int32_t degree, int32_t probes, uint64_t seed,
                                        const ent_options *opt, ent_result *outs);
ent_status ent_graph_create(const ent_matrix *Rs, int32_t count, int32_t method, int32_t degree,
                            int32_t probes, uint64_t seed, const ent_options *opt, ent_graph *graph);
ent_status ent_graph_launch(ent_graph graph, ent_result *outs);
ent_status ent_graph_per_probe(ent_graph graph, double *per_probe);
ent_status ent_graph_time_eager(ent_graph graph, ent_result *outs, ent_timing *timing);
int32_t ent_graph_tile_rows(ent_graph graph);       /* 64 or 128 (chosen tile shape; BF16x3: 128) */
size_t ent_graph_window_bytes(ent_graph graph);     /* window of the persistent schedule; 0: one
                                                       grouped launch per step */
size_t ent_graph_workspace_bytes(ent_graph graph);
ent_status ent_graph_destroy(ent_graph graph);

/* Workspace control (device memory cached between calls, per device). */
ent_status ent_set_workspace_limit(size_t bytes);  /* 0 = no limit */
ent_status ent_release_workspace(void);
size_t ent_workspace_bytes(void);

/* Thread-local description of the last failure on this thread ("" if none).
 * Valid until the next call on this thread. */
const char *ent_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int32_t ent_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ENTROPY_H */
