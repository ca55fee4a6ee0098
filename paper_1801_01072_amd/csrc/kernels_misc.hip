// kernels_misc.hip -- probes, power method (Algorithm 4), interval and
// coefficient setup (Lemma 3), trace check, conversions and the final
// reductions of the Hutchinson estimate (Lemma 1, Algorithms 1-2).
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

// ---------------------------------------------------------------------------
// Probe blocks
// ---------------------------------------------------------------------------
// One thread per (row, 32-probe word): Rademacher signs from one Philox word.
template <typename T>
__global__ void probe_rademacher_kernel(T *__restrict__ G, uint32_t *__restrict__ signs, int64_t n,
                                        int64_t n_pad, int32_t s, int64_t ldv, uint64_t seed) {
  const int32_t nw = (int32_t)(ldv >> 5);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pad * nw) return;
  const int64_t row = t / nw;
  const int32_t word = (int32_t)(t % nw);
  uint32_t bits = 0;
  uint32_t valid = 0;
  if (row < n) {
    bits = rademacher_word(seed, 0u, row, word);
    const int32_t lo = word * 32;
    valid = (s - lo >= 32) ? 0xffffffffu : (s > lo ? ((1u << (s - lo)) - 1u) : 0u);
  }
  if (signs && row < n) signs[row * nw + word] = bits & valid;
  if (G) {
    T *dst = G + row * ldv + (int64_t)word * 32;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
      const bool on = (valid >> b) & 1u;
      dst[b] = on ? (((bits >> b) & 1u) ? T(-1) : T(1)) : T(0);
    }
  }
}

template <typename T>
__global__ void probe_gaussian_kernel(T *__restrict__ G, int64_t n, int64_t n_pad, int32_t s,
                                      int64_t ldv, uint64_t seed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pad * ldv) return;
  const int64_t row = t / ldv;
  const int64_t j = t % ldv;
  G[t] = (row < n && j < s) ? (T)gaussian(seed, 0u, row, j) : T(0);
}

template <typename T>
hipError_t launch_probe_gen(T *G, uint32_t *signs, int64_t n, int64_t n_pad, int32_t s,
                            int64_t ldv, uint64_t seed, int32_t dist, hipStream_t st) {
  if (dist == 0) {
    const int64_t tot = n_pad * (ldv >> 5);
    probe_rademacher_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(G, signs, n, n_pad, s,
                                                                             ldv, seed);
  } else {
    const int64_t tot = n_pad * ldv;
    probe_gaussian_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(G, n, n_pad, s, ldv, seed);
  }
  return hipGetLastError();
}
template hipError_t launch_probe_gen<double>(double *, uint32_t *, int64_t, int64_t, int32_t,
                                             int64_t, uint64_t, int32_t, hipStream_t);
template hipError_t launch_probe_gen<float>(float *, uint32_t *, int64_t, int64_t, int32_t,
                                            int64_t, uint64_t, int32_t, hipStream_t);

hipError_t launch_sign_gen(uint32_t *signs, int64_t n, int32_t s, int64_t ldv, uint64_t seed,
                           hipStream_t st) {
  return launch_probe_gen<float>(nullptr, signs, n, n, s, ldv, seed, 0, st);
}

// ---------------------------------------------------------------------------
// Power method
// ---------------------------------------------------------------------------
__global__ void power_start_kernel(double *__restrict__ x, int64_t n, uint64_t seed, int32_t trial) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = rademacher(seed, 1u, i, trial);
}

hipError_t launch_power_start(double *x, int64_t n, uint64_t seed, int32_t trial, hipStream_t st) {
  power_start_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(x, n, seed, trial);
  return hipGetLastError();
}

// Scale 1/||x_prev|| from the yy entries of the previous product's partials.
__device__ __forceinline__ double block_input_scale(const double *in_part, int32_t in_cnt,
                                                    double *s_scale) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (w == 0) {
    double acc = 0.0;
    if (in_part)
      for (int i = lane; i < in_cnt; i += 64) acc += in_part[3 * i];
    acc = wave_sum(acc);
    if (lane == 0) *s_scale = in_part ? 1.0 / sqrt(acc) : 1.0;
  }
  __syncthreads();
  return *s_scale;
}

// Block sums of y^2, xs.y, xs^2 over the rows a block produced.
__device__ __forceinline__ void block_power_partials(double yy, double xy, double xx,
                                                     double *part3) {
  __shared__ double red[3][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  yy = wave_sum(yy);
  xy = wave_sum(xy);
  xx = wave_sum(xx);
  if (lane == 0) {
    red[0][w] = yy;
    red[1][w] = xy;
    red[2][w] = xx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < nw; ++i) {
      a += red[0][i];
      b += red[1][i];
      c += red[2][i];
    }
    part3[3 * blockIdx.x + 0] = a;
    part3[3 * blockIdx.x + 1] = b;
    part3[3 * blockIdx.x + 2] = c;
  }
}

// Dense: each wave owns 4 consecutive rows; lanes stride over 16-byte
// vectors of those rows (FP64 accumulation).
template <typename T>
__global__ __launch_bounds__(256) void power_gemv_kernel(const T *__restrict__ R, int64_t ldr,
                                                         int64_t n, const double *__restrict__ x,
                                                         const double *__restrict__ in_part,
                                                         int32_t in_cnt, double *__restrict__ y,
                                                         double *__restrict__ part3) {
  __shared__ double s_scale;
  const double sc = block_input_scale(in_part, in_cnt, &s_scale);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int VEC = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t nvec = n / VEC;
  for (int64_t v = lane; v < nvec; v += 64) {
    const int64_t k = v * VEC;
    double xv[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) xv[e] = x[k + e];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      if (r0 + rr < n) {
        const vec_t rv = *(const vec_t *)(R + (r0 + rr) * ldr + k);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[rr] += (double)rv[e] * xv[e];
      }
    }
  }
  for (int64_t k = nvec * VEC + lane; k < n; k += 64) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
      if (r0 + rr < n) acc[rr] += (double)R[(r0 + rr) * ldr + k] * x[k];
  }
  double yy = 0.0, xy = 0.0, xx = 0.0;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const double s = wave_sum(acc[rr]);
    if (r0 + rr < n) {
      const double yv = sc * s;
      const double xs = sc * x[r0 + rr];
      if (lane == 0) {
        y[r0 + rr] = yv;
        yy += yv * yv;
        xy += xs * yv;
        xx += xs * xs;
      }
    }
  }
  block_power_partials(yy, xy, xx, part3);
}

template <typename T>
hipError_t launch_power_gemv(const T *R, int64_t ldr, int64_t n, const double *x,
                             const double *in_part, int32_t in_cnt, double *y, double *part3,
                             int32_t *nblk, hipStream_t st) {
  const int64_t blocks = (n + 15) / 16;
  *nblk = (int32_t)blocks;
  power_gemv_kernel<T><<<(unsigned)blocks, 256, 0, st>>>(R, ldr, n, x, in_part, in_cnt, y, part3);
  return hipGetLastError();
}
template hipError_t launch_power_gemv<double>(const double *, int64_t, int64_t, const double *,
                                              const double *, int32_t, double *, double *,
                                              int32_t *, hipStream_t);
template hipError_t launch_power_gemv<float>(const float *, int64_t, int64_t, const double *,
                                             const double *, int32_t, double *, double *, int32_t *,
                                             hipStream_t);

// CSR: 8 lanes per row, 8 rows per wave, 32 rows per block.
template <typename T>
__global__ __launch_bounds__(256) void power_spmv_kernel(const int64_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const T *__restrict__ val, int64_t n,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ in_part,
                                                         int32_t in_cnt, double *__restrict__ y,
                                                         double *__restrict__ part3) {
  __shared__ double s_scale;
  const double sc = block_input_scale(in_part, in_cnt, &s_scale);
  const int lane = threadIdx.x & 63;
  const int sub = lane & 7;
  const int64_t row = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
  double acc = 0.0;
  if (row < n) {
    const int64_t e1 = rp[row + 1];
    for (int64_t e = rp[row] + sub; e < e1; e += 8) acc += (double)val[e] * x[ci[e]];
  }
#pragma unroll
  for (int off = 4; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  double yy = 0.0, xy = 0.0, xx = 0.0;
  if (row < n && sub == 0) {
    const double yv = sc * acc;
    const double xs = sc * x[row];
    y[row] = yv;
    yy = yv * yv;
    xy = xs * yv;
    xx = xs * xs;
  }
  block_power_partials(yy, xy, xx, part3);
}

template <typename T>
hipError_t launch_power_spmv(const int64_t *rp, const int32_t *ci, const T *val, int64_t n,
                             const double *x, const double *in_part, int32_t in_cnt, double *y,
                             double *part3, int32_t *nblk, hipStream_t st) {
  const int64_t blocks = (n + 31) / 32;
  *nblk = (int32_t)blocks;
  power_spmv_kernel<T><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, x, in_part, in_cnt, y, part3);
  return hipGetLastError();
}
template hipError_t launch_power_spmv<double>(const int64_t *, const int32_t *, const double *,
                                              int64_t, const double *, const double *, int32_t,
                                              double *, double *, int32_t *, hipStream_t);
template hipError_t launch_power_spmv<float>(const int64_t *, const int32_t *, const float *,
                                             int64_t, const double *, const double *, int32_t,
                                             double *, double *, int32_t *, hipStream_t);

__global__ void power_rq_kernel(double *__restrict__ scal, const double *__restrict__ part3,
                                int32_t nblk, int32_t trial) {
  const int lane = threadIdx.x;
  double xy = 0.0, xx = 0.0;
  for (int i = lane; i < nblk; i += 64) {
    xy += part3[3 * i + 1];
    xx += part3[3 * i + 2];
  }
  xy = wave_sum(xy);
  xx = wave_sum(xx);
  if (lane == 0) {
    const double rq = xy / xx;
    if (trial == 0 || rq > scal[S_P1]) scal[S_P1] = rq;
  }
}

hipError_t launch_power_rq(double *scal, const double *part3, int32_t nblk, int32_t trial,
                           hipStream_t st) {
  power_rq_kernel<<<1, 64, 0, st>>>(scal, part3, nblk, trial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interval [lo, u] and Chebyshev coefficients
// ---------------------------------------------------------------------------
__global__ void setup_interval_kernel(double *__restrict__ scal, int32_t method, int32_t m,
                                      double c, double u_fixed, double lo) {
  __shared__ double su;
  if (threadIdx.x == 0) {
    double u;
    if (u_fixed > 0.0) {
      u = u_fixed;
    } else {
      const double p1 = scal[S_P1];
      if (!(p1 > 0.0) || !isfinite(p1)) scal[S_FLAG] = 1.0;
      u = fmin(1.0, c * p1);
    }
    if (!(u > lo)) scal[S_FLAG] = 1.0;
    scal[S_U] = u;
    scal[S_LO] = lo;
    if (method == 0) {  // Taylor: A = R/u, C = I - A
      scal[S_A] = 1.0 / u;
      scal[S_B] = 1.0;
    } else {  // Chebyshev: X = a R - b I maps [lo, u] onto [-1, 1]
      scal[S_A] = 2.0 / (u - lo);
      scal[S_B] = (u + lo) / (u - lo);
    }
    su = u;
  }
  __syncthreads();
  if (method != 1) return;
  const double u = su;
  const double pi = 3.141592653589793238462643383279502884;
  for (int w = threadIdx.x; w <= m; w += blockDim.x) {
    double a;
    if (lo == 0.0) {
      // Lemma 3: alpha_0 = (u/2)(ln(u/4)+1), alpha_1 = (u/4)(2 ln(u/4)+3),
      // alpha_w = (-1)^w u / (w^3 - w)
      if (w == 0) {
        a = 0.5 * u * (log(0.25 * u) + 1.0);
      } else if (w == 1) {
        a = 0.25 * u * (2.0 * log(0.25 * u) + 3.0);
      } else {
        const double dw = (double)w;
        a = ((w & 1) ? -u : u) / (dw * dw * dw - dw);
      }
    } else {
      // interpolant of x ln x at the m+1 Chebyshev points of [lo, u]
      const int N = m + 1;
      double acc = 0.0;
      for (int i = 0; i < N; ++i) {
        const double th = pi * ((double)i + 0.5) / (double)N;
        const double x = 0.5 * (u + lo) + 0.5 * (u - lo) * cos(th);
        const double hx = x > 0.0 ? x * log(x) : 0.0;
        acc += hx * cos((double)w * th);
      }
      a = (2.0 / (double)N) * acc;
      if (w == 0) a *= 0.5;
    }
    scal[S_ALPHA + w] = a;
  }
}

hipError_t launch_setup_interval(double *scal, int32_t method, int32_t m, double c, double u_fixed,
                                 double lo, hipStream_t st) {
  setup_interval_kernel<<<1, 256, 0, st>>>(scal, method, m, c, u_fixed, lo);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Trace of R (input contract: unit trace)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void trace_dense_kernel(const T *__restrict__ R, int64_t ldr, int64_t n,
                                   double *__restrict__ scal) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += (double)R[i * ldr + i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) scal[S_TRACE] = red[0] + red[1] + red[2] + red[3];
}

template <typename T>
hipError_t launch_trace_dense(const T *R, int64_t ldr, int64_t n, double *scal, hipStream_t st) {
  trace_dense_kernel<T><<<1, 256, 0, st>>>(R, ldr, n, scal);
  return hipGetLastError();
}
template hipError_t launch_trace_dense<double>(const double *, int64_t, int64_t, double *, hipStream_t);
template hipError_t launch_trace_dense<float>(const float *, int64_t, int64_t, double *, hipStream_t);

// CSR: diagonal entries found by a scan of each row; per-block partials are
// combined by the last pass in block order.
template <typename T>
__global__ void trace_csr_partial_kernel(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                         const T *__restrict__ val, int64_t n,
                                         double *__restrict__ tmp) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
      if (ci[e] == i) acc += (double)val[e];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) tmp[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void sum_to_slot_kernel(const double *__restrict__ tmp, int32_t cnt, double *dst) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < cnt; i += 64) acc += tmp[i];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) *dst = acc;
}

template <typename T>
hipError_t launch_trace_csr(const int64_t *rp, const int32_t *ci, const T *val, int64_t n,
                            double *scal, hipStream_t st) {
  // scal has room after the coefficient area: use a scratch tail of 1024 doubles
  double *tmp = scal + 4096;
  const int blocks = 1024;
  trace_csr_partial_kernel<T><<<blocks, 256, 0, st>>>(rp, ci, val, n, tmp);
  sum_to_slot_kernel<<<1, 64, 0, st>>>(tmp, blocks, scal + S_TRACE);
  return hipGetLastError();
}
template hipError_t launch_trace_csr<double>(const int64_t *, const int32_t *, const double *,
                                             int64_t, double *, hipStream_t);
template hipError_t launch_trace_csr<float>(const int64_t *, const int32_t *, const float *, int64_t,
                                            double *, hipStream_t);

// ---------------------------------------------------------------------------
// CSR structure check: row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz, and
// every column index in [0, n).  Any violation sets flag[0].
// ---------------------------------------------------------------------------
__global__ void validate_csr_kernel(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                    int64_t n, int64_t nnz, int32_t *__restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  for (int64_t i = t0; i <= n; i += stride) {
    const int64_t v = rp[i];
    if (i == 0 && v != 0) bad = true;
    if (i == n && v != nnz) bad = true;
    if (i < n && rp[i + 1] < v) bad = true;
  }
  for (int64_t e = t0; e < nnz; e += stride) {
    const int32_t c = ci[e];
    if (c < 0 || (int64_t)c >= n) bad = true;
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_validate_csr(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz,
                               int32_t *flag, hipStream_t st) {
  validate_csr_kernel<<<1024, 256, 0, st>>>(rp, ci, n, nnz, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Conversion copies
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ void convert_kernel(const Tin *__restrict__ src, int64_t lds, Tout *__restrict__ dst,
                               int64_t ldd, int64_t rows, int64_t cols) {
  const int64_t r = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ldd;
       c += (int64_t)gridDim.x * blockDim.x)
    dst[r * ldd + c] = (r < rows && c < cols) ? (Tout)src[r * lds + c] : Tout(0);
}

template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin *src, int64_t lds, Tout *dst, int64_t ldd, int64_t rows,
                          int64_t cols, hipStream_t st) {
  dim3 grid((unsigned)((ldd + 255) / 256 < 64 ? (ldd + 255) / 256 : 64), (unsigned)rows);
  convert_kernel<Tin, Tout><<<grid, 256, 0, st>>>(src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}
template hipError_t launch_convert<double, float>(const double *, int64_t, float *, int64_t, int64_t,
                                                  int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float *, int64_t, double *, int64_t, int64_t,
                                                  int64_t, hipStream_t);
template hipError_t launch_convert<double, double>(const double *, int64_t, double *, int64_t,
                                                   int64_t, int64_t, hipStream_t);
template hipError_t launch_convert<float, float>(const float *, int64_t, float *, int64_t, int64_t,
                                                 int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__global__ void reduce_moments_kernel(const double *__restrict__ part, int32_t nslot,
                                      int32_t ntile, int64_t ldv, int32_t s,
                                      double *__restrict__ d) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nslot * s) return;
  const int32_t k = (int32_t)(t / s), j = (int32_t)(t % s);
  const double *p = part + (int64_t)k * ntile * ldv + j;
  double acc = 0.0;
  for (int32_t i = 0; i < ntile; ++i) acc += p[(int64_t)i * ldv];
  d[(int64_t)k * s + j] = acc;
}

hipError_t launch_reduce_moments(const double *part, int32_t nslot, int32_t ntile, int64_t ldv,
                                 int32_t s, double *d, hipStream_t st) {
  const int64_t tot = (int64_t)nslot * s;
  reduce_moments_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(part, nslot, ntile, ldv, s, d);
  return hipGetLastError();
}

// h_j and the mean/standard error.  Chebyshev: h_j = -sum_{k=0}^m alpha_k d_kj.
// Taylor: h_j = ln(1/u) + u sum_{k=1}^m e_kj / k  (e_kj = g^T (R/u) C^k g).
__global__ void final_kernel(const double *__restrict__ d, double *__restrict__ scal, int32_t method,
                             int32_t m, int32_t s, double *__restrict__ h) {
  __shared__ double red[4];
  __shared__ double smean;
  const double u = scal[S_U];
  double acc = 0.0;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    double v;
    if (method == 1) {
      v = 0.0;
      for (int k = 0; k <= m; ++k) v -= scal[S_ALPHA + k] * d[(int64_t)k * s + j];
    } else {
      double t = 0.0;
      for (int k = 1; k <= m; ++k) t += d[(int64_t)k * s + j] / (double)k;
      v = log(1.0 / u) + u * t;
    }
    h[j] = v;
    acc += v;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) smean = (red[0] + red[1] + red[2] + red[3]) / (double)s;
  __syncthreads();
  const double mean = smean;
  double var = 0.0;
  for (int j = threadIdx.x; j < s; j += blockDim.x) var += (h[j] - mean) * (h[j] - mean);
  var = wave_sum(var);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = var;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = red[0] + red[1] + red[2] + red[3];
    scal[S_ENT] = mean;
    scal[S_SE] = s > 1 ? sqrt(v / ((double)s * (double)(s - 1))) : 0.0;
    if (!isfinite(mean)) scal[S_FLAG] = 1.0;
  }
}

hipError_t launch_final(const double *d, double *scal, int32_t method, int32_t m, int32_t s,
                        double *h, hipStream_t st) {
  final_kernel<<<1, 256, 0, st>>>(d, scal, method, m, s, h);
  return hipGetLastError();
}

}  // namespace ent
