// kernels.hpp -- host-side launch interface of the libentropy gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace ent {

// Device scalar block (FP64).  The power method, the interval and the
// polynomial coefficients live here so the whole estimate runs without a
// host round trip.
enum ScalarSlot {
  S_P1 = 0,     // p~1
  S_U = 1,      // u
  S_LO = 2,     // lower end of the interval
  S_A = 3,      // product scale: Chebyshev 2/(u-lo), Taylor 1/u
  S_B = 4,      // shift: Chebyshev (u+lo)/(u-lo), Taylor 1
  S_FLAG = 5,   // nonzero: numeric failure (p~1 <= 0 or non-finite)
  S_TRACE = 6,  // tr R
  S_NORM = 7,   // > 0: the estimate is of R / tr R, products scaled by this
                // factor (div / tr R); 0: R as given
  S_ENT = 8,    // estimate
  S_SE = 9,     // standard error
  S_ALPHA = 16  // alpha_0 .. alpha_m (Chebyshev) follow
};

// launch_final's method code for the Clenshaw schedule (0 Taylor, 1 Chebyshev).
constexpr int32_t FINAL_CLENSHAW = 2;

struct DenseStepArgs {
  const void *R;      // n x n, row-major, element type T
  int64_t ldr;
  int64_t n;
  int64_t ldv;        // leading dimension of V buffers (= padded probe count)
  const void *Vk;     // operand block V_k
  const void *Vkm1;   // V_{k-1} (may be null when cw == 0)
  void *Vkp1;         // output block (may be null: no write)
  const void *G;      // probe block g
  const double *scal; // device scalars
  double c1, c2, cw;  // z = c1*y + c2*b*V_k + cw*V_{k-1}, y = a*(R V_k)
  int32_t dot_y;      // 1: dots with y (Taylor), 0: dots with z (Chebyshev)
  int32_t slot;       // partial slot of the main dot
  int32_t slot_gg;    // slot for g.g partials (-1: none)
  double *part;       // partials [slot][row tile][ldv]
  int32_t ntile;      // number of row tiles (partial stride)
  int32_t bn;         // column tile width (64, 128 or 256)
  const double *cg;   // device scalar: z += (*cg) g (Clenshaw's alpha_k term); null: none
  // Split-K (ksplit > 1): the product runs over ksplit ranges of kper
  // columns into party[ks][row][ldv] (element type T, n_pad rows), and a
  // second kernel sums them in split order and applies the epilogue.
  int32_t ksplit;
  int64_t kper;       // multiple of 32
  void *party;
  int32_t nptile;     // split-K: 16-row partial tiles (part is [slot][nptile][ldv])
};

struct CsrStepArgs {
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const void *values;  // element type T
  int64_t n;
  int64_t ldv;         // padded probe count (multiple of 64)
  const void *Vk;      // null: V_k is the sign block (first step)
  const void *Vkm1;    // null: V_{k-1} is the sign block (if cw != 0)
  void *Vkp1;
  const uint32_t *signs;  // Rademacher sign bits [n][ldv/32] (null: Gaussian)
  const void *G;          // Gaussian probe block (null: Rademacher)
  const double *scal;
  double c1, c2, cw;
  int32_t dot_y;
  int32_t slot;
  int32_t slot_gg;
  double *part;
  int32_t nblk;         // persistent grid size (partial stride)
  const int2 *win;      // column window per row chunk (launch_csr_chunk_window)
  const double *cg;     // device scalar: z += (*cg) g (Clenshaw's alpha_k term); null: none
  int32_t s;            // probes in use (<= ldv): columns past s are neither read
                        // nor written, and their dot partials are zero; 0: ldv
};

// Per-matrix descriptor of a batch (device resident).  Offsets are in
// elements of the batch-wide buffers they index.
struct BatchMat {
  const void *src; // caller's matrix (storage type), ld = ldsrc
  int64_t ldsrc;
  const void *R;   // matrix in the compute type, row-major, ld = ldr
  int64_t ldr;
  int64_t n;
  int64_t n_pad;   // rows of this matrix's V blocks
  int64_t voff;    // V / G blocks (n_pad x ldv, row-major)
  int64_t poff;    // step partials [slot][ntile][ldv]
  int64_t xoff;    // power-method vectors
  int64_t pboff;   // power-method partials (3 per block)
  int64_t doff;    // moments [slot][s]
  int64_t hoff;    // per-probe values [s]
  double *scal;    // scalar block
  uint64_t seed;   // probe seed of this matrix
  int32_t ntile;   // row tiles of the step kernel (BF16x3: epilogue blocks)
  int32_t pblk;    // power-method blocks
  int64_t aoff;    // BF16x3: bf16 hi/lo split of R (n_pad x n_pad, fragment-major)
};

struct BatchStepArgs {
  DenseStepArgs base;  // V/G/part are batch base pointers; R, n, ntile, scal per matrix
  const BatchMat *mats;
  const int2 *tiles;   // (matrix, row tile) per workgroup
};

// ---- probes ----------------------------------------------------------------
// G[i][j] (row-major, ld = ldv) for i < n_pad, j < ldv; zero outside n x s.
// Rademacher also writes the sign words signs[i][w] (w < ldv/32) if non-null.
template <typename T>
hipError_t launch_probe_gen(T *G, uint32_t *signs, int64_t n, int64_t n_pad, int32_t s,
                            int64_t ldv, uint64_t seed, int32_t dist, hipStream_t st);
hipError_t launch_sign_gen(uint32_t *signs, int64_t n, int32_t s, int64_t ldv, uint64_t seed,
                           hipStream_t st);

// ---- power method (Algorithm 4) ------------------------------------------
hipError_t launch_power_start(double *x, int64_t n, uint64_t seed, int32_t trial, hipStream_t st);
// y = (R x) / ||x_prev||, ||x_prev||^2 = in_norm[0] (in_norm null: scale 1);
// part3[3*b + {0,1,2}] = per-block sums of y^2, xs.y, xs^2, xs = x/||x_prev||.
// *nblk receives the number of blocks.
int32_t power_blocks_dense(int64_t n);
int32_t power_blocks_csr(int64_t n);
template <typename T>
hipError_t launch_power_gemv(const T *R, int64_t ldr, int64_t n, const double *x,
                             const double *in_norm, double *y, double *part3, int32_t *nblk,
                             hipStream_t st);
template <typename T>
// (nnz only picks the lanes per row: 1, 2, 4 or 8 by the mean row length)
hipError_t launch_power_spmv(const int64_t *rp, const int32_t *ci, const T *val, int64_t n,
                             int64_t nnz, const double *x, const double *in_norm, double *y,
                             double *part3, int32_t *nblk, hipStream_t st);
// norm3[0..2] = fixed-order sums of the nblk block triples.
hipError_t launch_power_reduce(const double *part3, int32_t nblk, double *norm3, hipStream_t st);
// p~ of trial = norm3[1]/norm3[2] of its final product; scal[S_P1] keeps the
// maximum over trials (trial 0 overwrites).
hipError_t launch_power_rq(double *scal, const double *norm3, int32_t trial, hipStream_t st);
// u = u_fixed > 0 ? u_fixed : min(1, c p~1); interval scalars and, for
// Chebyshev, alpha_0..alpha_m (closed form of Lemma 3 when lo = 0,
// interpolant at m+1 Chebyshev points otherwise).
// norm_div > 0: the estimate is of R / tr R; S_NORM = norm_div / scal[S_TRACE]
// (norm_div = the multiple of tr R that the trace kernel measured), p~1 and
// the product scale are multiplied by it.
hipError_t launch_setup_interval(double *scal, int32_t method, int32_t m, double c,
                                 double u_fixed, double lo, hipStream_t st, double norm_div = 0.0);
// S_NORM alone (random projection: singular values scaled by it).
hipError_t launch_set_norm(double *scal, double norm_div, hipStream_t st);

// ---- trace check -----------------------------------------------------------
template <typename T>
hipError_t launch_trace_dense(const T *R, int64_t ldr, int64_t n, double *scal, hipStream_t st);
template <typename T>
hipError_t launch_trace_csr(const int64_t *rp, const int32_t *ci, const T *val, int64_t n, int64_t nnz,
                            double *scal, hipStream_t st);

// CSR structure check; flag[0] |= 1 on any violation (flag must start at 0).
hipError_t launch_validate_csr(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz,
                               int32_t *flag, hipStream_t st);
// The same check and the half-bandwidth max |col - row| (into flag[1], which
// must start at 0; meaningful only if flag[0] stays 0) in one pass, one row
// per thread: for short rows (at most a few entries each on average).
hipError_t launch_validate_csr_rows(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz,
                                    int32_t *flag, hipStream_t st);

// ---- conversion --------------------------------------------------------------
template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin *src, int64_t lds, Tout *dst, int64_t ldd, int64_t rows,
                          int64_t cols, hipStream_t st);

// Real 2n x 2n form [[B, -C], [C, B]] of a Hermitian R = B + iC stored as
// interleaved (re, im) pairs with leading dimension ldr (complex elements);
// M row-major with leading dimension ldm >= 2n (padding columns zeroed).
template <typename Tin, typename Tout>
hipError_t launch_realify(const Tin *Rc, int64_t ldr, int64_t n, Tout *M, int64_t ldm,
                          hipStream_t st);

// ---- recurrence steps --------------------------------------------------------
// One dense step; with a K split (ksplit > 1) the product kernel and then,
// unless epilogue is false, the split epilogue (launch_dense_split_epilogue).
template <typename T>
hipError_t launch_dense_step(const DenseStepArgs &a, hipStream_t st, bool epilogue = true);
template <typename T>
hipError_t launch_dense_split_epilogue(const DenseStepArgs &a, hipStream_t st);
// K-splits for a dense step whose tile grid (ntile x ldv/bn) has fewer than
// 512 workgroups (two per CU): a power of two up to 16 while every split
// keeps >= 256 columns.
int32_t dense_step_splits(int64_t n, int32_t ntile, int64_t ldv, int32_t bn);
template <typename T>
hipError_t launch_csr_step(const CsrStepArgs &a, hipStream_t st);
int32_t csr_step_blocks(int64_t n, int32_t fp64);
// Rows per chunk of the CSR step (FP64 or FP32 compute), and the column
// window (min, max) of every chunk, computed once per estimate.
int32_t csr_chunk_rows(int32_t fp64);
hipError_t launch_csr_chunk_window(const int64_t *rp, const int32_t *ci, int64_t n, int32_t ch,
                                   int2 *win, hipStream_t st);


// ---- tridiagonal CSR (every entry within one of the diagonal) ---------------
// Row r's values as {l_r, d_r, u_r, 0} (4 n elements of type T), duplicate
// entries summed in entry order.  With trace non-null, also the trace (the
// diagonal entries summed in FP64, in a fixed order) into *trace, through
// kTriTraceBlocks partial sums in tmp.
constexpr int32_t kTriTraceBlocks = 2048;
template <typename T>
hipError_t launch_tri_pack(const int64_t *rp, const int32_t *ci, const T *val, int64_t n, T *D, double *tmp,
                           double *trace, hipStream_t st);
struct TriStepArgs {
  const void *diag;    // launch_tri_pack output, element type T
  int64_t n;
  int64_t ldv;         // partial-sum and sign-word row stride: probes rounded up to 64
  int64_t ldb;         // row stride of V_k, V_{k-1}, V_{k+1} and G: >= s, a multiple of 4, <= ldv
  int32_t s;           // probes in use (<= ldb; 0: ldv): later columns are not touched
  const void *Vk;      // null: V_k is the sign block (first step)
  const void *Vkm1;    // null: V_{k-1} is the sign block (if cw != 0)
  void *Vkp1;          // null: no write (last Taylor step)
  const uint32_t *signs;  // Rademacher sign bits [n_pad][ldv/32] (null: Gaussian)
  const void *G;          // Gaussian probe block (null: Rademacher)
  const double *scal;
  double c1, c2, cw;
  int32_t dot_y;
  int32_t slot;
  int32_t slot_gg;
  double *part;        // partials [slot][block][ldv]
  int32_t nblk;        // workgroups of the grid (partial stride), from tri_step_blocks
  const double *cg;    // device scalar: z += (*cg) g (Clenshaw's alpha_k term); null: none
};
int32_t tri_step_blocks(int64_t n, int32_t s, int32_t fp64);
// nf consecutive recurrence steps in one pass (2 <= nf <= kTriMaxFuse).
// Step 0 reads V_k (null: sign block) and V_{k-1} (null with cw[0] != 0:
// sign block); only the results of steps nf - 2 (VoutA) and nf - 1 (VoutB;
// null: no write) are stored; the outputs may not alias the inputs; row
// strides as in TriStepArgs; per-step scalars indexed by step, slot_gg for
// step 0.
constexpr int kTriMaxFuse = 10;
struct TriFusedArgs {
  const void *diag;
  const void *prep;    // Chebyshev and Clenshaw steps: launch_tri_prepare output (2X), required
  int64_t n, ldv, ldb;
  int32_t s;
  const void *Vk;
  const void *Vkm1;
  void *VoutA;
  void *VoutB;
  const uint32_t *signs;
  const void *G;
  const double *scal;
  double c1[kTriMaxFuse], c2[kTriMaxFuse], cw[kTriMaxFuse];
  int32_t dot_y[kTriMaxFuse];
  int32_t slot[kTriMaxFuse];
  int32_t slot_gg;
  const double *cg[kTriMaxFuse];
  double *part;
  int32_t nblk;
};
template <typename T>
hipError_t launch_tri_fused(const TriFusedArgs &a, int32_t nf, hipStream_t st);
// P = 2X = 2(aR - bI) on the packed diagonals (rows {2a l, 2(a d - b), 2a u, 0}),
// a and b read from scal on the device; P may not alias D.
template <typename T>
hipError_t launch_tri_prepare(const T *D, const double *scal, int64_t n, T *P, hipStream_t st);
// Power-method product on the packed diagonals: the contract of
// launch_power_spmv, with nblk workgroups (nblk triples written).
template <typename T>
hipError_t launch_power_tri(const T *D, int64_t n, const double *x, const double *in_norm, double *y,
                            double *part3, int32_t nblk, hipStream_t st);
// k (2..kPowerMaxFuse) consecutive power-method products in one pass: the
// first divides by sqrt(prev3[0]) (the previous product's ||y||^2), the
// middle ones by the previous Rayleigh quotient prev3[1] / prev3[2], the last
// by nothing; y = the last product (may not alias x); nblk triples as
// launch_power_tri, over the last product and its input.  prev3 null: no
// scaling.
constexpr int kPowerMaxFuse = 10;
template <typename T>
hipError_t launch_power_tri_fused(const T *D, int64_t n, const double *x, const double *prev3, double *y,
                                  double *part3, int32_t nblk, int32_t k, hipStream_t st);
template <typename T>
hipError_t launch_tri_step(const TriStepArgs &a, hipStream_t st);

// ---- banded CSR (every entry within HP of the diagonal) -----------------------
// Half-bandwidth max |col - row| of a validated CSR matrix into out[0] (which
// must start at 0); the padded half-bandwidth (4, 8 or 16) the banded step
// serves it with, or 0 if it is wider.
hipError_t launch_csr_half_bandwidth(const int64_t *rp, const int32_t *ci, int64_t n, int32_t *out,
                                     hipStream_t st);
int32_t band_half_width_padded(int32_t hbw);
// Elements of the 16-row slab storage, and the slabs from the CSR arrays.
size_t band_pack_elems(int64_t n, int32_t hp);
template <typename T>
hipError_t launch_band_pack(const int64_t *rp, const int32_t *ci, const T *val, int64_t n, int32_t hp,
                            T *band, hipStream_t st);
struct BandStepArgs {
  const void *band;    // slabs (launch_band_pack), element type T
  int64_t n;
  int64_t ldv;         // padded probe count (multiple of 64)
  const void *Vk;      // null: V_k is the sign block (first step)
  const void *Vkm1;    // null: V_{k-1} is the sign block (if cw != 0)
  void *Vkp1;          // null: no write (last Taylor step)
  const uint32_t *signs;  // Rademacher sign bits [n_pad][ldv/32] (null: Gaussian)
  const void *G;          // Gaussian probe block (null: Rademacher)
  const double *scal;
  double c1, c2, cw;
  int32_t dot_y;
  int32_t slot;
  int32_t slot_gg;
  double *part;        // partials [slot][wave][ldv]
  int32_t nwave;       // waves of the grid (partial stride), from band_step_waves
  const double *cg;    // device scalar: z += (*cg) g (Clenshaw's alpha_k term); null: none
};
int32_t band_step_waves(int64_t n, int32_t hp, int32_t fp64);
// Two consecutive recurrence steps in one pass (FP32): step A reads V_k
// (null: the sign block) and V_{k-1} (null with cw[0] != 0: the sign block)
// and writes V_{k+1} to VoutA; step B reads V_{k+1} and V_k and writes V_{k+2}
// to VoutB (null: no write).  Neither output may alias an input: a wave
// recomputes step A on the block before and after its range (whose V_k and
// V_{k-1} rows other waves read at the same time).  Per-step scalars as in
// BandStepArgs, index 0 for step A and 1 for step B; slot_gg applies to
// step A.
struct BandPairArgs {
  const void *band;
  int64_t n;
  int64_t ldv;
  const void *Vk;
  const void *Vkm1;
  void *VoutA;
  void *VoutB;
  const uint32_t *signs;
  const void *G;
  const double *scal;
  double c1[2], c2[2], cw[2];
  int32_t dot_y[2];
  int32_t slot[2];
  int32_t slot_gg;
  const double *cg[2];
  double *part;        // partials [slot][wave][ldv]
  int32_t nwave;       // waves of the grid (partial stride), from band_step_waves
};
hipError_t launch_band_pair(const BandPairArgs &a, int32_t hp, hipStream_t st);
// Power-method product on the slabs: the contract of launch_power_spmv, with
// nblk workgroups (nblk triples written; power_blocks_csr(n) of them).
template <typename T>
hipError_t launch_power_band(const T *band, int32_t hp, int64_t n, const double *x, const double *in_norm,
                             double *y, double *part3, int32_t nblk, hipStream_t st);
// k (2..kPowerMaxFuse) consecutive power-method products on the slabs in one
// pass: the contract of launch_power_tri_fused, with nblk workgroups from
// power_band_fused_blocks(n) (nblk triples written).
template <typename T>
hipError_t launch_power_band_fused(const T *band, int32_t hp, int64_t n, const double *x, const double *prev3,
                                   double *y, double *part3, int32_t nblk, int32_t k, hipStream_t st);
int32_t power_band_fused_blocks(int64_t n);
template <typename T>
hipError_t launch_band_step(const BandStepArgs &a, int32_t hp, hipStream_t st);

// ---- BF16x3 dense path (probe-major blocks, leading dimension n_pad) ----------
struct Bf16GemmArgs {
  const uint16_t *A_hi, *A_lo;  // n_pad x n_pad, row-major, bf16 bits
  const uint16_t *V_hi, *V_lo;  // ldv x n_pad, probe-major
  float *part_y;                // splits x ldv x n_pad
  int64_t n_pad;                // multiple of 128
  int64_t ldv;                  // multiple of bn
  int64_t k_per_split;          // multiple of 32, splits * k_per_split = n_pad
  int32_t splits;
  int32_t bn;                   // 64, 128 or 256
};
struct Bf16EpiArgs {
  const float *part_y;
  int32_t splits;
  const float *Vk, *Vkm1;       // FP32 probe-major (Vkm1 may be null)
  float *Vkp1;                  // null: no write (last Taylor step)
  uint16_t *V_hi, *V_lo;        // split of V_{k+1}, written in place
  const float *G;
  const double *scal;
  double c1, c2, cw;
  int32_t dot_y, slot, slot_gg;
  int32_t scale_y;              // 1: y *= scal[S_A] (the split is of R itself)
  double *part;                 // [slot][nblk][ldv]
  int32_t nblk;
  int64_t n_pad, ldv;
  const double *cg;             // device scalar: z += (*cg) g (Clenshaw); null: none
};
template <typename Tin>
hipError_t launch_split_matrix(const Tin *R, int64_t ldr, int64_t n, int64_t n_pad,
                               const double *scal, uint16_t *hi, uint16_t *lo, hipStream_t st);
// Probe-major block G[j][i] = scale * (probe of the given stream) and its
// bf16 split.
hipError_t launch_probe_gen_t(float *G, uint16_t *hi, uint16_t *lo, int64_t n, int64_t n_pad,
                              int32_t s, int64_t ldv, uint64_t seed, int32_t dist, hipStream_t st,
                              uint32_t stream = 0, double scale = 1.0);
// Rows of the GEMM's workgroup tile for a padded size (256 when it divides).
int32_t bf16x3_tile_rows(int64_t n_pad);
// K-splits of the GEMM for a grid of `tiles` output tiles (n_pad / splits is
// a multiple of 32).
int32_t bf16x3_splits(int64_t n_pad, int64_t tiles);
hipError_t launch_bf16x3_gemm(const Bf16GemmArgs &a, hipStream_t st);
// Power-method product on the fragment-major bf16 hi/lo split of R; x must
// be zero in [n, n_pad).  power_blocks_split: the most partials it writes.
// power_split_parts: column parts per band (> 1: ypart holds parts x n_pad
// doubles).
int32_t power_blocks_split(int64_t n_pad);
int32_t power_split_parts(int64_t n_pad);
hipError_t launch_power_gemv_split(const uint16_t *hi, const uint16_t *lo, int64_t n_pad, int64_t n,
                                   const double *x, const double *in_norm, double *y, double *part3,
                                   double *ypart, int32_t *nblk, hipStream_t st);
hipError_t launch_bf16x3_epilogue(const Bf16EpiArgs &a, hipStream_t st);
int32_t bf16x3_epilogue_blocks(int64_t n_pad);
// ---- BF16x3 batches (descriptor-driven; tables of (matrix, tile) pairs) ----
// tiles: (matrix, 128-row tile); ptiles: (matrix, 32-row band).  G/V_k are
// FP32 probe-major at M.voff; the bf16 V hi/lo at M.voff and A hi/lo at
// M.aoff are fragment-major.  A step reads V_k hi/lo (vin) and writes
// V_{k+1} hi/lo (base.V_hi/V_lo): they must be different buffers.
template <typename Tin>
hipError_t launch_batch_split(const BatchMat *mats, const int2 *tiles, int32_t ntiles, uint16_t *Ahi,
                              uint16_t *Alo, hipStream_t st);
hipError_t launch_batch_probe_t(const BatchMat *mats, const int2 *tiles, int32_t ntiles, float *G,
                                uint16_t *Vhi, uint16_t *Vlo, int32_t s, int64_t ldv, int32_t dist,
                                hipStream_t st);
hipError_t launch_batch_power_split(const BatchMat *mats, const int2 *ptiles, int32_t nptiles,
                                    const uint16_t *Ahi, const uint16_t *Alo, const double *x,
                                    const double *norm, double *y, double *pout, hipStream_t st);
// ---- persistent batch steps: one launch walks a schedule of work items ------
// Item (matrix b, row tile t, step k, 0).  Every matrix belongs to one XCD and
// its items form part of that XCD's segment of the schedule, which only the
// workgroups running on that XCD take; so a tile's inputs were written by the
// same XCD and the XCD's L2 is their point of coherence.  A segment lists
// every tile of step k - 1 of a matrix before any tile of its step k; an item
// waits until done[b] >= k * ntile_b (all tiles of step k - 1 finished), runs
// the tile, then adds one to done[b].  Waits are bounded: after spin_limit
// polls the item sets *err and every workgroup stops taking items.
constexpr int kMaxXcc = 16;
struct SchedArgs {
  const int4 *items;
  int32_t nitems;
  int32_t spin_limit;
  int32_t nseg;                  // segments (XCDs that hold workgroups)
  int32_t seg_off[kMaxXcc + 1];  // segment s: items [seg_off[s], seg_off[s + 1])
  int32_t seg_of_xcc[kMaxXcc];   // hardware XCC id -> segment (-1: none)
  int32_t *head;   // [nseg] next item of each segment (zeroed before the launch)
  int32_t *done;   // per-matrix finished tiles (zeroed before the launch)
  int32_t *err;    // nonzero: a wait timed out (zeroed before the launch)
};
// XCC id of the workgroups of a grid: ids[blockIdx.x] (one-time probe).
hipError_t launch_xcc_probe(int32_t *ids, int32_t grid, hipStream_t st);
// After a persistent launch: sets bit 1 of *err when a segment's items were
// not all taken (no workgroup of the launch ran on its XCD).
hipError_t launch_sched_check(const SchedArgs &s, hipStream_t st);
// Buffers and recurrence of the batched steps, common to every item.
struct BatchPersistArgs {
  SchedArgs sched;
  const BatchMat *mats;
  int32_t method;    // ENT_TAYLOR / ENT_CHEBYSHEV
  int32_t nsteps;    // m (Chebyshev) or m + 1 (Taylor)
  int64_t ldv;
  const void *G;     // probe block (batch base; FP32 probe-major for BF16x3)
  void *VA, *VB;     // recurrence buffers (batch base)
  double *part;      // step partials (batch base)
  // BF16x3: fragment-major split of every R and the two bf16 hi/lo sets of V
  const uint16_t *Ahi, *Alo;
  uint16_t *Vhi[2], *Vlo[2];
};
// Grid of the persistent step kernels (workgroups resident at once); 0 if the
// runtime cannot tell.
int32_t batch_persistent_grid(int32_t precision, int32_t wr, int64_t ldv);
int32_t bf16x3_persistent_grid(int64_t ldv);
template <typename T>
hipError_t launch_batch_dense_persistent(const BatchPersistArgs &pa, int32_t wr, int32_t grid,
                                         hipStream_t st);
hipError_t launch_batch_bf16x3_persistent(const BatchPersistArgs &pa, int32_t grid, hipStream_t st);

hipError_t launch_batch_bf16x3_step(const Bf16EpiArgs &base, const BatchMat *mats, const int2 *tiles,
                                    int32_t ntiles, const uint16_t *Ahi, const uint16_t *Alo,
                                    const uint16_t *vin_hi, const uint16_t *vin_lo, hipStream_t st);

// ---- batches of dense matrices (one launch per phase over all matrices) ------
template <typename T>
hipError_t launch_batch_dense_step(const BatchStepArgs &ba, int32_t ntiles, int32_t wr,
                                   hipStream_t st);
hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st);
// Zero `bytes` bytes at p (kernel stores, no memset node).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// R (compute copy, ld = ldr, zero columns n..ldr) <- src for every matrix.
template <typename Tin, typename Tout>
hipError_t launch_batch_convert(const BatchMat *mats, int32_t count, int64_t max_elems,
                                hipStream_t st);
template <typename T>
hipError_t launch_batch_trace(const BatchMat *mats, int32_t count, hipStream_t st);
template <typename T>
hipError_t launch_batch_probes(const BatchMat *mats, int32_t count, int64_t max_n_pad, T *G,
                               int32_t s, int64_t ldv, int32_t dist, hipStream_t st);
hipError_t launch_batch_power_start(const BatchMat *mats, int32_t count, int64_t max_n, double *x,
                                    int32_t trial, hipStream_t st);
// norm holds 4 doubles per matrix (reduced triple of the previous product).
template <typename T>
hipError_t launch_batch_power_gemv(const BatchMat *mats, const int2 *ptiles, int32_t nptiles,
                                   const double *x, const double *norm, double *y, double *pout,
                                   hipStream_t st);
hipError_t launch_batch_power_reduce(const BatchMat *mats, int32_t count, const double *p,
                                     double *norm, hipStream_t st);
hipError_t launch_batch_power_rq(const BatchMat *mats, int32_t count, const double *norm,
                                 int32_t trial, hipStream_t st);
hipError_t launch_batch_setup(const BatchMat *mats, int32_t count, int32_t method, int32_t m,
                              double c, double u_fixed, double lo, hipStream_t st,
                              double norm_div = 0.0);
hipError_t launch_batch_reduce(const BatchMat *mats, int32_t count, const double *part,
                               int32_t nslot, int64_t ldv, int32_t s, double *d, hipStream_t st);
hipError_t launch_batch_final(const BatchMat *mats, int32_t count, const double *d, int32_t method,
                              int32_t m, int32_t s, double *h, hipStream_t st);

// ---- random projection (Algorithm 3) -----------------------------------------
template <typename T>
hipError_t launch_sketch_gen(T *P, int64_t n, int64_t n_pad, int32_t s, int64_t ldv, uint64_t seed,
                             int32_t kind, hipStream_t st);
// Input-sparsity sketch for symmetric R.  phase 0: the bucket row lists
// cnt (s), off (s + 1), rows (n) for (seed, n, s); phase 1: Y (s x ldy,
// FP64, row c = bucket c) = (R Pi)^T from those lists.
template <typename T>
hipError_t launch_count_sketch(const T *R, int64_t ldr, int64_t n, int32_t s, uint64_t seed,
                               int32_t *cnt, int64_t *off, int32_t *rows, double *Y, int64_t ldy,
                               hipStream_t st, int phase);
// G = X^T X (s x s, FP64) with X(i, a) at X[i*si + a*sa]; scratch holds
// nsplit * s * s doubles.
template <typename T>
hipError_t launch_gram(const T *X, int64_t si, int64_t sa, int64_t n, int32_t s, double *scratch,
                       int32_t nsplit, double *G, hipStream_t st);
// Eigenvalues of G (tridiagonalization + bisection), sigma = sqrt, top k -> sigma[0..k),
// scal[S_ENT] = sum sigma ln(1/sigma).  work: N*N doubles, eig: N (N = s
// rounded up to even, at most 256).
hipError_t launch_rp_spectrum(const double *G, int32_t s, int32_t k, double *work, double *eig,
                              double *sigma, double *scal, hipStream_t st);

// ---- learned selector (MLP 16-64-64-2, FP32) ----------------------------------
int32_t mlp_nparams();
int32_t mlp_blocks(int32_t B);
hipError_t launch_mlp_forward(const float *P, const float *X, int32_t B, float *Y, hipStream_t st);
// grad (device, nparams) and *loss (device) of the mean squared error;
// gpart holds mlp_blocks(B) * nparams floats, lpart mlp_blocks(B) doubles.
hipError_t launch_mlp_grad(const float *P, const float *X, const float *T, int32_t B, float *gpart,
                           double *lpart, float *grad, double *loss, hipStream_t st);
hipError_t launch_adam(float *P, const float *grad, float *m, float *v, int32_t t, float lr,
                       hipStream_t st);
hipError_t launch_selector_features(const double *scal, const double *d, int32_t mf, int32_t sf,
                                    int64_t n, float *feat, hipStream_t st);

// ---- reductions ---------------------------------------------------------------
// d[k][j] = sum_t part[k][t][j] (fixed order), k < nslot, j < s.
hipError_t launch_reduce_moments(const double *part, int32_t nslot, int32_t ntile, int64_t ldv,
                                 int32_t s, double *d, hipStream_t st);
// Per-probe values and the estimate (Algorithms 1-2 output line).
hipError_t launch_final(const double *d, double *scal, int32_t method, int32_t m, int32_t s,
                        double *h, hipStream_t st);

// ---- fixed scratch of the no-allocation entry point ---------------------------
// Size of the per-device scratch array (ENT_NOALLOC_SCRATCH_BYTES).
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
// This device's copy of the scratch array (looked up once per device, with
// that device current) and the lock that serialises the calls using it.
hipError_t noalloc_scratch(int dev, void **ptr, std::mutex **use);

}  // namespace ent
