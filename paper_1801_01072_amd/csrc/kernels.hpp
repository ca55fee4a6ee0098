// kernels.hpp -- host-side launch interface of the libentropy gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
  S_ENT = 8,    // estimate
  S_SE = 9,     // standard error
  S_ALPHA = 16  // alpha_0 .. alpha_m (Chebyshev) follow
};

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
// y = (R x) / ||x_prev||, with ||x_prev||^2 = sum(in_part[0..in_cnt)) (in_part
// null: scale 1).  part3[3*b + {0,1,2}] = per-block sums of y^2, xs.y, xs^2
// with xs = x/||x_prev||.  Returns the number of blocks in *nblk.
template <typename T>
hipError_t launch_power_gemv(const T *R, int64_t ldr, int64_t n, const double *x,
                             const double *in_part, int32_t in_cnt, double *y, double *part3,
                             int32_t *nblk, hipStream_t st);
template <typename T>
hipError_t launch_power_spmv(const int64_t *rp, const int32_t *ci, const T *val, int64_t n,
                             const double *x, const double *in_part, int32_t in_cnt, double *y,
                             double *part3, int32_t *nblk, hipStream_t st);
// p~ of trial = sum(xs.y)/sum(xs^2) from part3 of the final product; keeps
// the maximum over trials in scal[S_P1] (trial 0 overwrites).
hipError_t launch_power_rq(double *scal, const double *part3, int32_t nblk, int32_t trial,
                           hipStream_t st);
// u = u_fixed > 0 ? u_fixed : min(1, c p~1); interval scalars and, for
// Chebyshev, alpha_0..alpha_m (closed form of Lemma 3 when lo = 0,
// interpolant at m+1 Chebyshev points otherwise).
hipError_t launch_setup_interval(double *scal, int32_t method, int32_t m, double c,
                                 double u_fixed, double lo, hipStream_t st);

// ---- trace check -----------------------------------------------------------
template <typename T>
hipError_t launch_trace_dense(const T *R, int64_t ldr, int64_t n, double *scal, hipStream_t st);
template <typename T>
hipError_t launch_trace_csr(const int64_t *rp, const int32_t *ci, const T *val, int64_t n,
                            double *scal, hipStream_t st);

// CSR structure check; flag[0] |= 1 on any violation (flag must start at 0).
hipError_t launch_validate_csr(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz,
                               int32_t *flag, hipStream_t st);

// ---- conversion --------------------------------------------------------------
template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin *src, int64_t lds, Tout *dst, int64_t ldd, int64_t rows,
                          int64_t cols, hipStream_t st);

// ---- recurrence steps --------------------------------------------------------
template <typename T>
hipError_t launch_dense_step(const DenseStepArgs &a, hipStream_t st);
template <typename T>
hipError_t launch_csr_step(const CsrStepArgs &a, hipStream_t st);
int32_t csr_step_blocks(int64_t n);

// ---- reductions ---------------------------------------------------------------
// d[k][j] = sum_t part[k][t][j] (fixed order), k < nslot, j < s.
hipError_t launch_reduce_moments(const double *part, int32_t nslot, int32_t ntile, int64_t ldv,
                                 int32_t s, double *d, hipStream_t st);
// Per-probe values and the estimate (Algorithms 1-2 output line).
hipError_t launch_final(const double *d, double *scal, int32_t method, int32_t m, int32_t s,
                        double *h, hipStream_t st);

}  // namespace ent
