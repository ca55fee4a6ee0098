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

// Sign bits only: one thread per row (grid-stride), each Philox block
// giving four consecutive words of the row, the same bits as
// probe_rademacher_kernel.
__global__ __launch_bounds__(256) void sign_words_kernel(uint32_t *__restrict__ signs, int64_t n, int32_t s,
                                                         int32_t nw, uint64_t seed) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    uint32_t *dst = signs + row * nw;
    for (int32_t blk = 0; 4 * blk < nw; ++blk) {
      const U4 o = philox_block(seed, 0u, row, (uint32_t)blk);
      const uint32_t w4[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int32_t word = 4 * blk + k;
        if (word >= nw) break;
        const int32_t lo = word * 32;
        const uint32_t valid = (s - lo >= 32) ? 0xffffffffu : (s > lo ? ((1u << (s - lo)) - 1u) : 0u);
        dst[word] = w4[k] & valid;
      }
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
  if (n < 1 || !signs || ldv % 32 != 0) return hipErrorInvalidValue;
  const int64_t b = (n + 255) / 256;
  sign_words_kernel<<<(unsigned)(b < 8192 ? b : 8192), 256, 0, st>>>(signs, n, s, (int32_t)(ldv >> 5), seed);
  return hipGetLastError();
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

// Dense y = (R x)/||x_prev|| (||x_prev||^2 = in_norm[0]; null: no scaling).
// Each wave owns 2 consecutive rows; lanes stride over 16-byte vectors of
// both rows, two vectors in flight per row (FP64 accumulation).
template <typename T>
__device__ __forceinline__ void power_gemv_body(const T *__restrict__ R, int64_t ldr, int64_t n,
                                                const double *__restrict__ x,
                                                const double *__restrict__ in_norm,
                                                double *__restrict__ y, double *__restrict__ part3,
                                                int64_t blk) {
  const double sc = in_norm ? 1.0 / sqrt(in_norm[0]) : 1.0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int VEC = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  const int64_t r0 = (blk * 4 + w) * 2;
  const bool ok0 = r0 < n, ok1 = r0 + 1 < n;
  const T *R0 = R + (ok0 ? r0 : 0) * ldr;
  const T *R1 = R + (ok1 ? r0 + 1 : 0) * ldr;
  double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
  const int64_t nvec = n / VEC;
  int64_t v = lane;
  for (; v + 64 < nvec; v += 128) {
    const int64_t k = v * VEC, k2 = (v + 64) * VEC;
    vec_t p0 = {}, p1 = {}, q0 = {}, q1 = {};
    if (ok0) {
      p0 = *(const vec_t *)(R0 + k);
      q0 = *(const vec_t *)(R0 + k2);
    }
    if (ok1) {
      p1 = *(const vec_t *)(R1 + k);
      q1 = *(const vec_t *)(R1 + k2);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const double xe = x[k + e], xf = x[k2 + e];
      a0 += (double)p0[e] * xe;
      a1 += (double)p1[e] * xe;
      b0 += (double)q0[e] * xf;
      b1 += (double)q1[e] * xf;
    }
  }
  for (; v < nvec; v += 64) {
    const int64_t k = v * VEC;
    vec_t p0 = {}, p1 = {};
    if (ok0) p0 = *(const vec_t *)(R0 + k);
    if (ok1) p1 = *(const vec_t *)(R1 + k);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      a0 += (double)p0[e] * x[k + e];
      a1 += (double)p1[e] * x[k + e];
    }
  }
  for (int64_t k = nvec * VEC + lane; k < n; k += 64) {
    if (ok0) a0 += (double)R0[k] * x[k];
    if (ok1) a1 += (double)R1[k] * x[k];
  }
  const double s0 = wave_sum(a0 + b0), s1 = wave_sum(a1 + b1);
  double yy = 0.0, xy = 0.0, xx = 0.0;
  if (lane == 0) {
    if (ok0) {
      const double yv = sc * s0, xs = sc * x[r0];
      y[r0] = yv;
      yy += yv * yv;
      xy += xs * yv;
      xx += xs * xs;
    }
    if (ok1) {
      const double yv = sc * s1, xs = sc * x[r0 + 1];
      y[r0 + 1] = yv;
      yy += yv * yv;
      xy += xs * yv;
      xx += xs * xs;
    }
  }
  block_power_partials(yy, xy, xx, part3, blk);
}

template <typename T>
__global__ __launch_bounds__(256) void power_gemv_kernel(const T *__restrict__ R, int64_t ldr,
                                                         int64_t n, const double *__restrict__ x,
                                                         const double *__restrict__ in_norm,
                                                         double *__restrict__ y,
                                                         double *__restrict__ part3) {
  power_gemv_body<T>(R, ldr, n, x, in_norm, y, part3, blockIdx.x);
}

int32_t power_blocks_dense(int64_t n) { return (int32_t)((n + 7) / 8); }
int32_t power_blocks_csr(int64_t n) {
  const int64_t b = (n + 31) / 32;
  return (int32_t)(b < 4096 ? b : 4096);
}

template <typename T>
hipError_t launch_power_gemv(const T *R, int64_t ldr, int64_t n, const double *x,
                             const double *in_norm, double *y, double *part3, int32_t *nblk,
                             hipStream_t st) {
  const int32_t blocks = power_blocks_dense(n);
  *nblk = blocks;
  power_gemv_kernel<T><<<(unsigned)blocks, 256, 0, st>>>(R, ldr, n, x, in_norm, y, part3);
  return hipGetLastError();
}
template hipError_t launch_power_gemv<double>(const double *, int64_t, int64_t, const double *,
                                              const double *, double *, double *, int32_t *,
                                              hipStream_t);
template hipError_t launch_power_gemv<float>(const float *, int64_t, int64_t, const double *,
                                             const double *, double *, double *, int32_t *,
                                             hipStream_t);

// CSR: L lanes per row (L = 1, 2, 4 or 8 by the mean row length), 256 / L
// rows per block per pass, persistent grid-stride over row groups (one
// partial triple per block).
template <typename T, int L>
__global__ __launch_bounds__(256) void power_spmv_kernel(const int64_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const T *__restrict__ val, int64_t n,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ in_norm,
                                                         double *__restrict__ y,
                                                         double *__restrict__ part3) {
  constexpr int RPB = 256 / L;  // rows per block per pass
  const double sc = in_norm ? 1.0 / sqrt(in_norm[0]) : 1.0;
  const int sub = threadIdx.x % L;
  double yy = 0.0, xy = 0.0, xx = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < n; base += (int64_t)gridDim.x * RPB) {
    const int64_t row = base + threadIdx.x / L;
    double acc = 0.0;
    if (row < n) {
      const int64_t e1 = rp[row + 1];
      for (int64_t e = rp[row] + sub; e < e1; e += L) acc += (double)val[e] * x[ci[e]];
    }
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (row < n && sub == 0) {
      const double yv = sc * acc;
      const double xs = sc * x[row];
      y[row] = yv;
      yy += yv * yv;
      xy += xs * yv;
      xx += xs * xs;
    }
  }
  block_power_partials(yy, xy, xx, part3, blockIdx.x);
}

template <typename T>
hipError_t launch_power_spmv(const int64_t *rp, const int32_t *ci, const T *val, int64_t n,
                             int64_t nnz, const double *x, const double *in_norm, double *y,
                             double *part3, int32_t *nblk, hipStream_t st) {
  const int32_t blocks = power_blocks_csr(n);
  *nblk = blocks;
  const double avg = n > 0 ? (double)nnz / (double)n : 0.0;
  if (avg <= 1.5)
    power_spmv_kernel<T, 1><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, x, in_norm, y, part3);
  else if (avg <= 3.0)
    power_spmv_kernel<T, 2><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, x, in_norm, y, part3);
  else if (avg <= 6.0)
    power_spmv_kernel<T, 4><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, x, in_norm, y, part3);
  else
    power_spmv_kernel<T, 8><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, x, in_norm, y, part3);
  return hipGetLastError();
}
template hipError_t launch_power_spmv<double>(const int64_t *, const int32_t *, const double *,
                                              int64_t, int64_t, const double *, const double *,
                                              double *, double *, int32_t *, hipStream_t);
template hipError_t launch_power_spmv<float>(const int64_t *, const int32_t *, const float *,
                                             int64_t, int64_t, const double *, const double *,
                                             double *, double *, int32_t *, hipStream_t);

// Fixed-order sum of the block triples of one product into norm3[0..2].
__device__ __forceinline__ void power_reduce_body(const double *__restrict__ part3, int32_t nblk,
                                                  double *__restrict__ norm3) {
  __shared__ double red[3][4];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    a += part3[3 * i];
    b += part3[3 * i + 1];
    c += part3[3 * i + 2];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    norm3[0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    norm3[1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    norm3[2] = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  }
}

__global__ __launch_bounds__(256) void power_reduce_kernel(const double *__restrict__ part3,
                                                           int32_t nblk, double *__restrict__ norm3) {
  power_reduce_body(part3, nblk, norm3);
}

hipError_t launch_power_reduce(const double *part3, int32_t nblk, double *norm3, hipStream_t st) {
  power_reduce_kernel<<<1, 256, 0, st>>>(part3, nblk, norm3);
  return hipGetLastError();
}

// Rayleigh quotient of a trial from the reduced triple of its final product;
// scal[S_P1] keeps the maximum over trials (trial 0 overwrites).
__device__ __forceinline__ void power_rq_body(double *__restrict__ scal,
                                              const double *__restrict__ norm3, int32_t trial) {
  if (threadIdx.x == 0) {
    const double rq = norm3[1] / norm3[2];
    if (trial == 0 || rq > scal[S_P1]) scal[S_P1] = rq;
  }
}

__global__ void power_rq_kernel(double *__restrict__ scal, const double *__restrict__ norm3,
                                int32_t trial) {
  power_rq_body(scal, norm3, trial);
}

hipError_t launch_power_rq(double *scal, const double *norm3, int32_t trial, hipStream_t st) {
  power_rq_kernel<<<1, 64, 0, st>>>(scal, norm3, trial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interval [lo, u] and Chebyshev coefficients
// ---------------------------------------------------------------------------
__device__ __forceinline__ void setup_interval_body(double *__restrict__ scal, int32_t method,
                                                    int32_t m, double c, double u_fixed, double lo,
                                                    double norm_div) {
  __shared__ double su;
  if (threadIdx.x == 0) {
    // R / tr R (problem statement, unit trace): every eigenvalue, hence p~1,
    // and every product R v are scaled by 1 / tr R
    double nm = 1.0;
    if (norm_div > 0.0) {
      const double tr = scal[S_TRACE] / norm_div;
      nm = 1.0 / tr;
      if (!(tr > 0.0) || !isfinite(nm)) {
        scal[S_FLAG] = 1.0;
        nm = 1.0;
      }
      scal[S_NORM] = nm;
      if (!(u_fixed > 0.0)) scal[S_P1] *= nm;
    }
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
      scal[S_A] = nm / u;
      scal[S_B] = 1.0;
    } else {  // Chebyshev: X = a R - b I maps [lo, u] onto [-1, 1]
      scal[S_A] = nm * 2.0 / (u - lo);
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
      // Chebyshev projection of x ln x on [lo, u] by an N-point Gauss-Chebyshev
      // rule, N = 1024 (2(m+1) beyond degree 511): independent of m, so the
      // partial sums over the degree are nested
      const int N = (m + 1) <= 512 ? 1024 : 2 * (m + 1);
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

__global__ void setup_interval_kernel(double *__restrict__ scal, int32_t method, int32_t m,
                                      double c, double u_fixed, double lo, double norm_div) {
  setup_interval_body(scal, method, m, c, u_fixed, lo, norm_div);
}

hipError_t launch_setup_interval(double *scal, int32_t method, int32_t m, double c, double u_fixed,
                                 double lo, hipStream_t st, double norm_div) {
  setup_interval_kernel<<<1, 256, 0, st>>>(scal, method, m, c, u_fixed, lo, norm_div);
  return hipGetLastError();
}

__global__ void set_norm_kernel(double *__restrict__ scal, double norm_div) {
  if (threadIdx.x != 0) return;
  const double tr = scal[S_TRACE] / norm_div;
  const double nm = 1.0 / tr;
  if (!(tr > 0.0) || !isfinite(nm)) {
    scal[S_FLAG] = 1.0;
    scal[S_NORM] = 1.0;
  } else {
    scal[S_NORM] = nm;
  }
}

hipError_t launch_set_norm(double *scal, double norm_div, hipStream_t st) {
  set_norm_kernel<<<1, 64, 0, st>>>(scal, norm_div);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Trace of R (input contract: unit trace)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void trace_dense_body(const T *__restrict__ R, int64_t ldr, int64_t n,
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
__global__ void trace_dense_kernel(const T *__restrict__ R, int64_t ldr, int64_t n,
                                   double *__restrict__ scal) {
  trace_dense_body<T>(R, ldr, n, scal);
}

template <typename T>
hipError_t launch_trace_dense(const T *R, int64_t ldr, int64_t n, double *scal, hipStream_t st) {
  trace_dense_kernel<T><<<1, 256, 0, st>>>(R, ldr, n, scal);
  return hipGetLastError();
}
template hipError_t launch_trace_dense<double>(const double *, int64_t, int64_t, double *, hipStream_t);
template hipError_t launch_trace_dense<float>(const float *, int64_t, int64_t, double *, hipStream_t);

// CSR: diagonal entries found by a scan of each row, L lanes per row (L by
// the mean row length, as in the power-method product) so that a row's
// column indices are read together; per-block partials are combined by the
// last pass in block order.
template <typename T, int L>
__global__ __launch_bounds__(256) void trace_csr_partial_kernel(const int64_t *__restrict__ rp,
                                                                const int32_t *__restrict__ ci,
                                                                const T *__restrict__ val, int64_t n,
                                                                double *__restrict__ tmp) {
  constexpr int RPB = 256 / L;
  __shared__ double red[4];
  const int sub = threadIdx.x % L;
  double acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * RPB; base < n; base += (int64_t)gridDim.x * RPB) {
    const int64_t row = base + threadIdx.x / L;
    if (row < n) {
      const int64_t e1 = rp[row + 1];
      for (int64_t e = rp[row] + sub; e < e1; e += L)
        if (ci[e] == row) acc += (double)val[e];
    }
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
                            int64_t nnz, double *scal, hipStream_t st) {
  // scal has room after the coefficient area: use a scratch tail of 1024 doubles
  double *tmp = scal + 4096;
  const int blocks = 1024;
  const double avg = n > 0 ? (double)nnz / (double)n : 0.0;
  if (avg <= 1.5)
    trace_csr_partial_kernel<T, 1><<<blocks, 256, 0, st>>>(rp, ci, val, n, tmp);
  else if (avg <= 3.0)
    trace_csr_partial_kernel<T, 2><<<blocks, 256, 0, st>>>(rp, ci, val, n, tmp);
  else if (avg <= 6.0)
    trace_csr_partial_kernel<T, 4><<<blocks, 256, 0, st>>>(rp, ci, val, n, tmp);
  else
    trace_csr_partial_kernel<T, 8><<<blocks, 256, 0, st>>>(rp, ci, val, n, tmp);
  sum_to_slot_kernel<<<1, 64, 0, st>>>(tmp, blocks, scal + S_TRACE);
  return hipGetLastError();
}
template hipError_t launch_trace_csr<double>(const int64_t *, const int32_t *, const double *,
                                             int64_t, int64_t, double *, hipStream_t);
template hipError_t launch_trace_csr<float>(const int64_t *, const int32_t *, const float *, int64_t,
                                            int64_t, double *, hipStream_t);

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
  // column indices, 16 bytes per load when the array allows it (a negative
  // index is a large unsigned one)
  int64_t done = 0;
  if (((uintptr_t)ci & 15) == 0) {
    const int4 *c4 = (const int4 *)ci;
    const int64_t n4 = nnz / 4;
    for (int64_t q = t0; q < n4; q += stride) {
      const int4 v = c4[q];
      if ((int64_t)(uint32_t)v.x >= n || (int64_t)(uint32_t)v.y >= n || (int64_t)(uint32_t)v.z >= n ||
          (int64_t)(uint32_t)v.w >= n)
        bad = true;
    }
    done = n4 * 4;
  }
  for (int64_t e = done + t0; e < nnz; e += stride) {
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

// One row per thread: row_ptr's local conditions (rp[0] = 0, rp[n] = nnz,
// 0 <= rp[r] <= rp[r+1] <= nnz) hold for every row exactly when row_ptr is
// valid, and a row's column indices are read only if its range lies in
// [0, nnz), so the entries of a valid structure are each checked once.
__global__ __launch_bounds__(256) void validate_csr_rows_kernel(const int64_t *__restrict__ rp,
                                                                const int32_t *__restrict__ ci, int64_t n,
                                                                int64_t nnz, int32_t *__restrict__ flag) {
  bool bad = false;
  int64_t hb = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = rp[r], b = rp[r + 1];
    if ((r == 0 && a != 0) || (r == n - 1 && b != nnz) || a < 0 || b < a || b > nnz) {
      bad = true;
      continue;
    }
    for (int64_t e = a; e < b; ++e) {
      const int64_t c = ci[e];
      if (c < 0 || c >= n) {
        bad = true;
      } else {
        const int64_t d = c > r ? c - r : r - c;
        hb = d > hb ? d : hb;
      }
    }
  }
  if (bad) atomicOr(flag, 1);
  // n < 2^31 (int32 column indices), so the half-bandwidth fits
  int32_t h = (int32_t)hb;
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(h, off, 64);
    h = o > h ? o : h;
  }
  if ((threadIdx.x & 63) == 0 && h > 0) atomicMax(flag + 1, h);
}

hipError_t launch_validate_csr_rows(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz,
                                    int32_t *flag, hipStream_t st) {
  if (n < 1) return hipErrorInvalidValue;
  const int64_t b = (n + 255) / 256;
  validate_csr_rows_kernel<<<(unsigned)(b < 4096 ? b : 4096), 256, 0, st>>>(rp, ci, n, nnz, flag);
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
// Hermitian R = B + iC (Section 4): its real form M = [[B, -C], [C, B]]
// (2n x 2n, row-major, leading dimension ldm; columns 2n..ldm-1 are zeroed).
// M [x; y] = [Re(R(x+iy)); Im(R(x+iy))], so the recurrence on M with probes
// [g; 0] is the complex recurrence on R with the real probe g, and
// [g; 0]^T T(M) [g; 0] = g^T Re[T(R)] g.  Every eigenvalue of R appears twice
// in M.  One thread per (row i of R, column j < ldm - n), grid-stride.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ void realify_kernel(const Tin *__restrict__ Rc, int64_t ldr, int64_t n,
                               Tout *__restrict__ M, int64_t ldm) {
  const int64_t cols = ldm - n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * cols;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / cols, j = t % cols;
    Tout *top = M + i * ldm, *bot = M + (i + n) * ldm;
    if (j < n) {
      const Tin re = Rc[2 * (i * ldr + j)], im = Rc[2 * (i * ldr + j) + 1];
      top[j] = (Tout)re;
      top[n + j] = (Tout)(-im);
      bot[j] = (Tout)im;
      bot[n + j] = (Tout)re;
    } else {
      // padding columns 2n..ldm-1 of both rows
      top[n + j] = Tout(0);
      bot[n + j] = Tout(0);
    }
  }
}

template <typename Tin, typename Tout>
hipError_t launch_realify(const Tin *Rc, int64_t ldr, int64_t n, Tout *M, int64_t ldm,
                          hipStream_t st) {
  if (ldm < 2 * n || ldr < n) return hipErrorInvalidValue;
  const int64_t tot = n * (ldm - n);
  const int64_t blocks = (tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536;
  realify_kernel<Tin, Tout><<<(unsigned)blocks, 256, 0, st>>>(Rc, ldr, n, M, ldm);
  return hipGetLastError();
}
template hipError_t launch_realify<double, double>(const double *, int64_t, int64_t, double *, int64_t,
                                                   hipStream_t);
template hipError_t launch_realify<double, float>(const double *, int64_t, int64_t, float *, int64_t,
                                                  hipStream_t);
template hipError_t launch_realify<float, double>(const float *, int64_t, int64_t, double *, int64_t,
                                                  hipStream_t);
template hipError_t launch_realify<float, float>(const float *, int64_t, int64_t, float *, int64_t,
                                                 hipStream_t);

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ void reduce_moments_body(const double *__restrict__ part, int32_t nslot,
                                                    int32_t ntile, int64_t ldv, int32_t s,
                                                    double *__restrict__ d, int64_t t) {
  if (t >= (int64_t)nslot * s) return;
  const int32_t k = (int32_t)(t / s), j = (int32_t)(t % s);
  const double *p = part + (int64_t)k * ntile * ldv + j;
  double acc = 0.0;
  for (int32_t i = 0; i < ntile; ++i) acc += p[(int64_t)i * ldv];
  d[(int64_t)k * s + j] = acc;
}

// One estimate's moments: workgroup = (slot, 64 probes); wave w sums the
// tiles of its contiguous quarter in order, then the quarters are added in
// order (fixed, so repeated runs agree bit for bit).
__global__ __launch_bounds__(256) void reduce_moments_kernel(const double *__restrict__ part, int32_t nslot,
                                                             int32_t ntile, int64_t ldv, int32_t s,
                                                             double *__restrict__ d) {
  __shared__ double q[4][64];
  const int k = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.y * 64 + lane;
  const int32_t per = (ntile + 3) / 4;
  const int32_t i0 = w * per, i1 = i0 + per < ntile ? i0 + per : ntile;
  double acc = 0.0;
  if (j < s) {
    const double *p = part + (int64_t)k * ntile * ldv + j;
    for (int32_t i = i0; i < i1; ++i) acc += p[(int64_t)i * ldv];
  }
  q[w][lane] = acc;
  __syncthreads();
  if (w == 0 && j < s) d[(int64_t)k * s + j] = ((q[0][lane] + q[1][lane]) + q[2][lane]) + q[3][lane];
}

hipError_t launch_reduce_moments(const double *part, int32_t nslot, int32_t ntile, int64_t ldv,
                                 int32_t s, double *d, hipStream_t st) {
  if (nslot < 1 || s < 1) return hipSuccess;
  reduce_moments_kernel<<<dim3((unsigned)nslot, (unsigned)((s + 63) / 64)), 256, 0, st>>>(part, nslot, ntile, ldv,
                                                                                         s, d);
  return hipGetLastError();
}

// h_j and the mean/standard error.  Chebyshev: h_j = -sum_{k=0}^m alpha_k d_kj
// (Clenshaw schedule: from g^T y_0, g^T y_2 and g^T g, see FINAL_CLENSHAW).
// Taylor: h_j = ln(1/u) + u sum_{k=1}^m e_kj / k  (e_kj = g^T (R/u) C^k g).
__device__ __forceinline__ void final_body(const double *__restrict__ d, double *__restrict__ scal,
                                           int32_t method, int32_t m, int32_t s,
                                           double *__restrict__ h) {
  __shared__ double red[4];
  __shared__ double smean;
  const double u = scal[S_U];
  double acc = 0.0;
  for (int j = threadIdx.x; j < s; j += blockDim.x) {
    double v;
    if (method == FINAL_CLENSHAW) {
      // Algorithm 5: g^T f_m g = (alpha_0 g^T g + g^T y_0 - g^T y_2) / 2, with
      // d_k = g^T y_k in slots 0..m (y_2 = 0 for m < 2) and g^T g in slot m+1
      const double gg = d[(int64_t)(m + 1) * s + j];
      const double y2 = m >= 2 ? d[(int64_t)2 * s + j] : 0.0;
      v = -0.5 * (scal[S_ALPHA] * gg + d[j] - y2);
    } else if (method == 1) {
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

__global__ void final_kernel(const double *__restrict__ d, double *__restrict__ scal, int32_t method,
                             int32_t m, int32_t s, double *__restrict__ h) {
  final_body(d, scal, method, m, s, h);
}

hipError_t launch_final(const double *d, double *scal, int32_t method, int32_t m, int32_t s,
                        double *h, hipStream_t st) {
  final_kernel<<<1, 256, 0, st>>>(d, scal, method, m, s, h);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batches: the same phases over many matrices in one launch each.  Blocks map
// to matrices through the descriptor array (grid.y) or a tile table.
// ---------------------------------------------------------------------------
__global__ void fill_kernel(double *__restrict__ p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st) {
  const int64_t blocks = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
  fill_kernel<<<(unsigned)(blocks > 0 ? blocks : 1), 256, 0, st>>>(p, count, v);
  return hipGetLastError();
}

// Zero bytes [p, p + bytes): 16-byte stores over the aligned bulk, byte
// stores for the head and tail.  Used instead of a memset node so that a
// captured sequence clears its buffers with kernels only.
__global__ void zero_kernel(unsigned char *__restrict__ p, int64_t head, int64_t nvec, int64_t bytes) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint4 *v = (uint4 *)(p + head);
  for (int64_t i = tid; i < nvec; i += stride) v[i] = make_uint4(0u, 0u, 0u, 0u);
  const int64_t tail0 = head + 16 * nvec;
  for (int64_t i = tid; i < head; i += stride) p[i] = 0;
  for (int64_t i = tail0 + tid; i < bytes; i += stride) p[i] = 0;
}

__global__ void xcc_probe_kernel(int32_t *ids) {
  if (threadIdx.x == 0) ids[blockIdx.x] = xcc_id();
}

hipError_t launch_xcc_probe(int32_t *ids, int32_t grid, hipStream_t st) {
  xcc_probe_kernel<<<(unsigned)grid, 64, 0, st>>>(ids);
  return hipGetLastError();
}

__global__ void sched_check_kernel(SchedArgs s) {
  const int q = (int)threadIdx.x;
  if (q < s.nseg) {
    const int len = s.seg_off[q + 1] - s.seg_off[q];
    if (len > 0 && __hip_atomic_load(s.head + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < len)
      __hip_atomic_fetch_or(s.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_sched_check(const SchedArgs &s, hipStream_t st) {
  sched_check_kernel<<<1, 64, 0, st>>>(s);
  return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  const uintptr_t a = (uintptr_t)p;
  int64_t head = (int64_t)((16 - (a & 15)) & 15);
  if ((size_t)head > bytes) head = (int64_t)bytes;
  const int64_t nvec = ((int64_t)bytes - head) / 16;
  const int64_t work = nvec > 0 ? nvec : (int64_t)bytes;
  const int64_t blocks = (work + 255) / 256 < 2048 ? (work + 255) / 256 : 2048;
  zero_kernel<<<(unsigned)(blocks > 0 ? blocks : 1), 256, 0, st>>>((unsigned char *)p, head, nvec,
                                                                   (int64_t)bytes);
  return hipGetLastError();
}

template <typename Tin, typename Tout>
__global__ void batch_convert_kernel(const BatchMat *__restrict__ mats) {
  const BatchMat &M = mats[blockIdx.y];
  const Tin *src = (const Tin *)M.src;
  Tout *dst = (Tout *)M.R;
  const int64_t tot = M.n * M.ldr;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / M.ldr, c = t % M.ldr;
    dst[t] = c < M.n ? (Tout)src[r * M.ldsrc + c] : Tout(0);
  }
}

template <typename Tin, typename Tout>
hipError_t launch_batch_convert(const BatchMat *mats, int32_t count, int64_t max_elems,
                                hipStream_t st) {
  const int64_t per = (max_elems + 255) / 256;
  dim3 grid((unsigned)(per < 512 ? per : 512), (unsigned)count);
  batch_convert_kernel<Tin, Tout><<<grid, 256, 0, st>>>(mats);
  return hipGetLastError();
}
template hipError_t launch_batch_convert<double, double>(const BatchMat *, int32_t, int64_t, hipStream_t);
template hipError_t launch_batch_convert<float, float>(const BatchMat *, int32_t, int64_t, hipStream_t);
template hipError_t launch_batch_convert<double, float>(const BatchMat *, int32_t, int64_t, hipStream_t);
template hipError_t launch_batch_convert<float, double>(const BatchMat *, int32_t, int64_t, hipStream_t);

template <typename T>
__global__ void batch_trace_kernel(const BatchMat *__restrict__ mats) {
  const BatchMat &M = mats[blockIdx.x];
  trace_dense_body<T>((const T *)M.R, M.ldr, M.n, M.scal);
}

template <typename T>
hipError_t launch_batch_trace(const BatchMat *mats, int32_t count, hipStream_t st) {
  batch_trace_kernel<T><<<(unsigned)count, 256, 0, st>>>(mats);
  return hipGetLastError();
}
template hipError_t launch_batch_trace<double>(const BatchMat *, int32_t, hipStream_t);
template hipError_t launch_batch_trace<float>(const BatchMat *, int32_t, hipStream_t);

// G of matrix b = its n_pad x ldv region; probes from the matrix's own seed.
template <typename T>
__global__ void batch_probe_kernel(const BatchMat *__restrict__ mats, T *__restrict__ G, int32_t s,
                                   int64_t ldv, int32_t dist) {
  const BatchMat &M = mats[blockIdx.y];
  T *Gb = G + M.voff;
  const int64_t tot = M.n_pad * ldv;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / ldv, j = t % ldv;
    T v = T(0);
    if (row < M.n && j < s)
      v = (T)(dist == 0 ? rademacher(M.seed, 0u, row, j) : gaussian(M.seed, 0u, row, j));
    Gb[t] = v;
  }
}

template <typename T>
hipError_t launch_batch_probes(const BatchMat *mats, int32_t count, int64_t max_n_pad, T *G,
                               int32_t s, int64_t ldv, int32_t dist, hipStream_t st) {
  const int64_t per = (max_n_pad * ldv + 255) / 256;
  dim3 grid((unsigned)(per < 256 ? per : 256), (unsigned)count);
  batch_probe_kernel<T><<<grid, 256, 0, st>>>(mats, G, s, ldv, dist);
  return hipGetLastError();
}
template hipError_t launch_batch_probes<double>(const BatchMat *, int32_t, int64_t, double *, int32_t,
                                                int64_t, int32_t, hipStream_t);
template hipError_t launch_batch_probes<float>(const BatchMat *, int32_t, int64_t, float *, int32_t,
                                               int64_t, int32_t, hipStream_t);

__global__ void batch_power_start_kernel(const BatchMat *__restrict__ mats, double *__restrict__ x,
                                         int32_t trial) {
  const BatchMat &M = mats[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M.n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[M.xoff + i] = rademacher(M.seed, 1u, i, trial);
}

hipError_t launch_batch_power_start(const BatchMat *mats, int32_t count, int64_t max_n, double *x,
                                    int32_t trial, hipStream_t st) {
  const int64_t per = (max_n + 255) / 256;
  dim3 grid((unsigned)(per < 64 ? per : 64), (unsigned)count);
  batch_power_start_kernel<<<grid, 256, 0, st>>>(mats, x, trial);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void batch_power_gemv_kernel(const BatchMat *__restrict__ mats,
                                                               const int2 *__restrict__ ptiles,
                                                               const double *x, const double *norm,
                                                               double *y, double *pout) {
  const int2 t = ptiles[blockIdx.x];
  const BatchMat &M = mats[t.x];
  power_gemv_body<T>((const T *)M.R, M.ldr, M.n, x + M.xoff, norm ? norm + 4 * t.x : nullptr,
                     y + M.xoff, pout + M.pboff, t.y);
}

template <typename T>
hipError_t launch_batch_power_gemv(const BatchMat *mats, const int2 *ptiles, int32_t nptiles,
                                   const double *x, const double *norm, double *y, double *pout,
                                   hipStream_t st) {
  batch_power_gemv_kernel<T><<<(unsigned)nptiles, 256, 0, st>>>(mats, ptiles, x, norm, y, pout);
  return hipGetLastError();
}
template hipError_t launch_batch_power_gemv<double>(const BatchMat *, const int2 *, int32_t,
                                                    const double *, const double *, double *,
                                                    double *, hipStream_t);
template hipError_t launch_batch_power_gemv<float>(const BatchMat *, const int2 *, int32_t,
                                                   const double *, const double *, double *, double *,
                                                   hipStream_t);

// One block per matrix: reduce its block triples into norm[4*b .. 4*b+2].
__global__ __launch_bounds__(256) void batch_power_reduce_kernel(const BatchMat *__restrict__ mats,
                                                                 const double *p, double *norm) {
  const BatchMat &M = mats[blockIdx.x];
  power_reduce_body(p + M.pboff, M.pblk, norm + 4 * blockIdx.x);
}

hipError_t launch_batch_power_reduce(const BatchMat *mats, int32_t count, const double *p,
                                     double *norm, hipStream_t st) {
  batch_power_reduce_kernel<<<(unsigned)count, 256, 0, st>>>(mats, p, norm);
  return hipGetLastError();
}

__global__ void batch_power_rq_kernel(const BatchMat *__restrict__ mats, const double *norm,
                                      int32_t trial) {
  power_rq_body(mats[blockIdx.x].scal, norm + 4 * blockIdx.x, trial);
}

hipError_t launch_batch_power_rq(const BatchMat *mats, int32_t count, const double *norm,
                                 int32_t trial, hipStream_t st) {
  batch_power_rq_kernel<<<(unsigned)count, 64, 0, st>>>(mats, norm, trial);
  return hipGetLastError();
}

__global__ void batch_setup_kernel(const BatchMat *__restrict__ mats, int32_t method, int32_t m,
                                   double c, double u_fixed, double lo, double norm_div) {
  setup_interval_body(mats[blockIdx.x].scal, method, m, c, u_fixed, lo, norm_div);
}

hipError_t launch_batch_setup(const BatchMat *mats, int32_t count, int32_t method, int32_t m,
                              double c, double u_fixed, double lo, hipStream_t st, double norm_div) {
  batch_setup_kernel<<<(unsigned)count, 256, 0, st>>>(mats, method, m, c, u_fixed, lo, norm_div);
  return hipGetLastError();
}

__global__ void batch_reduce_kernel(const BatchMat *__restrict__ mats, const double *part,
                                    int32_t nslot, int64_t ldv, int32_t s, double *d) {
  const BatchMat &M = mats[blockIdx.y];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)nslot * s;
       t += (int64_t)gridDim.x * blockDim.x)
    reduce_moments_body(part + M.poff, nslot, M.ntile, ldv, s, d + M.doff, t);
}

hipError_t launch_batch_reduce(const BatchMat *mats, int32_t count, const double *part,
                               int32_t nslot, int64_t ldv, int32_t s, double *d, hipStream_t st) {
  const int64_t per = ((int64_t)nslot * s + 255) / 256;
  dim3 grid((unsigned)(per < 64 ? per : 64), (unsigned)count);
  batch_reduce_kernel<<<grid, 256, 0, st>>>(mats, part, nslot, ldv, s, d);
  return hipGetLastError();
}

__global__ void batch_final_kernel(const BatchMat *__restrict__ mats, const double *d,
                                   int32_t method, int32_t m, int32_t s, double *h) {
  const BatchMat &M = mats[blockIdx.x];
  final_body(d + M.doff, M.scal, method, m, s, h + M.hoff);
}

hipError_t launch_batch_final(const BatchMat *mats, int32_t count, const double *d, int32_t method,
                              int32_t m, int32_t s, double *h, hipStream_t st) {
  batch_final_kernel<<<(unsigned)count, 256, 0, st>>>(mats, d, method, m, s, h);
  return hipGetLastError();
}

}  // namespace ent
