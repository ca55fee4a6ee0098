// kernels_rp.hip -- random-projection estimator (Algorithm 3, Section 5):
// sketch R~ = R Pi (Gaussian and Hadamard sketches: product on the existing
// MFMA kernels; input-sparsity sketch: one signed pass over R), Gram matrix
// R~^T R~ in FP64, its eigenvalues by Householder tridiagonalization and
// bisection in one workgroup, singular values sigma = sqrt(lambda), the k
// largest kept and H^ = sum sigma ln(1/sigma).
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

// ---------------------------------------------------------------------------
// Sketch Pi, row-major n_pad x ldv: kind 0 entries N(0, 1/s) (Gaussian
// stream 2); kind 1 the subsampled randomized Hadamard transform
// sqrt(N/s) D H S, entries D_jj (-1)^popcount(j & i_t) / sqrt(s).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void sketch_gen_kernel(T *__restrict__ P, int64_t n, int64_t n_pad, int32_t s, int64_t ldv,
                                  uint64_t seed, double scale, int32_t kind) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pad * ldv) return;
  const int64_t i = t / ldv, j = t % ldv;
  T v = T(0);
  if (i < n && j < s)
    v = (T)(scale * (kind == 1 ? srht_entry(seed, i, j, hadamard_order(n)) : gaussian(seed, 2u, i, j)));
  P[t] = v;
}

template <typename T>
hipError_t launch_sketch_gen(T *P, int64_t n, int64_t n_pad, int32_t s, int64_t ldv, uint64_t seed,
                             int32_t kind, hipStream_t st) {
  const int64_t tot = n_pad * ldv;
  sketch_gen_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(P, n, n_pad, s, ldv, seed,
                                                                      1.0 / sqrt((double)s), kind);
  return hipGetLastError();
}
template hipError_t launch_sketch_gen<double>(double *, int64_t, int64_t, int32_t, int64_t, uint64_t,
                                              int32_t, hipStream_t);
template hipError_t launch_sketch_gen<float>(float *, int64_t, int64_t, int32_t, int64_t, uint64_t,
                                             int32_t, hipStream_t);

// ---------------------------------------------------------------------------
// Input-sparsity sketch Pi = D S (one entry D_jj per row, in column h(j)).
// R is symmetric, so (R Pi)^T = Pi^T R: row c of Y = (R Pi)^T is the signed
// sum of the rows j of R with h(j) = c.  The rows of each bucket are listed
// in ascending order (count, offsets, fill: one workgroup per bucket), and
// every row of R is then read exactly once: a single pass over R, as the
// construction's input-sparsity running time promises.  Sums are FP64 in
// ascending row order (deterministic).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cs_count_kernel(uint64_t seed, int64_t n, int32_t s,
                                                       int32_t *__restrict__ cnt) {
  __shared__ int32_t red[4];
  const int32_t c = blockIdx.x;
  int32_t k = 0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) k += sketch_bucket(seed, j, s) == c;
  for (int off = 32; off >= 1; off >>= 1) k += __shfl_xor(k, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = k;
  __syncthreads();
  if (threadIdx.x == 0) cnt[c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void cs_offsets_kernel(const int32_t *__restrict__ cnt, int32_t s, int64_t *__restrict__ off) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t a = 0;
  for (int32_t c = 0; c < s; ++c) {
    off[c] = a;
    a += cnt[c];
  }
  off[s] = a;
}

__global__ __launch_bounds__(256) void cs_fill_kernel(uint64_t seed, int64_t n, int32_t s,
                                                      const int64_t *__restrict__ off,
                                                      int32_t *__restrict__ rows) {
  __shared__ int32_t wcount[4];
  const int32_t c = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t base = off[c];
  for (int64_t j0 = 0; j0 < n; j0 += blockDim.x) {
    const int64_t j = j0 + threadIdx.x;
    const bool in = j < n && sketch_bucket(seed, j, s) == c;
    const uint64_t mask = __ballot(in);
    const int32_t before = (int32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[w] = (int32_t)__popcll(mask);
    __syncthreads();
    int32_t wbase = 0;
    for (int q = 0; q < w; ++q) wbase += wcount[q];
    if (in) rows[base + wbase + before] = (int32_t)j;
    base += wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();
  }
}

// Y[c][col] = sum over the rows j of bucket c of D_jj R[j][col]; workgroup
// (column chunk of 1024, bucket c); thread columns col0 + tid + 256 q.
template <typename T>
__global__ __launch_bounds__(256) void cs_apply_kernel(const T *__restrict__ R, int64_t ldr, int64_t n,
                                                       uint64_t seed, const int64_t *__restrict__ off,
                                                       const int32_t *__restrict__ rows,
                                                       double *__restrict__ Y, int64_t ldy) {
  const int32_t c = blockIdx.y;
  const int64_t col0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t r0 = off[c], r1 = off[c + 1];
  int64_t r = r0;
  // four rows at a time: 16 independent loads per thread in flight
  for (; r + 4 <= r1; r += 4) {
    int64_t j[4];
    double d[4];
    T v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      j[u] = rows[r + u];
      d[u] = sketch_sign(seed, j[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t col = col0 + 256 * q;
        v[u][q] = col < n ? R[j[u] * ldr + col] : T(0);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += d[u] * (double)v[u][q];
  }
  for (; r < r1; ++r) {
    const int64_t j = rows[r];
    const double d = sketch_sign(seed, j);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t col = col0 + 256 * q;
      if (col < n) acc[q] += d * (double)R[j * ldr + col];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t col = col0 + 256 * q;
    if (col < ldy) Y[(int64_t)c * ldy + col] = col < n ? acc[q] : 0.0;
  }
}

template <typename T>
hipError_t launch_count_sketch(const T *R, int64_t ldr, int64_t n, int32_t s, uint64_t seed,
                               int32_t *cnt, int64_t *off, int32_t *rows, double *Y, int64_t ldy,
                               hipStream_t st, int phase) {
  if (s < 1 || ldy < n || ldr < n) return hipErrorInvalidValue;
  if (phase == 0) {
    cs_count_kernel<<<(unsigned)s, 256, 0, st>>>(seed, n, s, cnt);
    cs_offsets_kernel<<<1, 64, 0, st>>>(cnt, s, off);
    cs_fill_kernel<<<(unsigned)s, 256, 0, st>>>(seed, n, s, off, rows);
  } else {
    dim3 grid((unsigned)((ldy + 1023) / 1024), (unsigned)s);
    cs_apply_kernel<T><<<grid, 256, 0, st>>>(R, ldr, n, seed, off, rows, Y, ldy);
  }
  return hipGetLastError();
}
template hipError_t launch_count_sketch<double>(const double *, int64_t, int64_t, int32_t, uint64_t,
                                                int32_t *, int64_t *, int32_t *, double *, int64_t,
                                                hipStream_t, int);
template hipError_t launch_count_sketch<float>(const float *, int64_t, int64_t, int32_t, uint64_t,
                                               int32_t *, int64_t *, int32_t *, double *, int64_t,
                                               hipStream_t, int);

// ---------------------------------------------------------------------------
// Gram matrix G = R~^T R~ (s x s, FP64).  R~(i, a) is at X[i*si + a*sa]
// (row-major R~: sa = 1; probe-major: si = 1).
// Workgroup = 16 x 16 block of G over one K range; partials per K range are
// summed in range order by gram_sum_kernel.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T *__restrict__ X, int64_t si,
                                                           int64_t sa, int64_t n, int32_t s,
                                                           int64_t rows_per, double *__restrict__ gp) {
  __shared__ double xa[64][17], xb[64][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int64_t r0 = (int64_t)blockIdx.z * rows_per;
  const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
  double acc = 0.0;
  for (int64_t base = r0; base < r1; base += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      // consecutive threads take consecutive addresses in either layout
      const int rr = si == 1 ? e % 64 : e / 16, cc = si == 1 ? e / 64 : e % 16;
      const int64_t i = base + rr;
      const bool ok = i < r1;
      xa[rr][cc] = (ok && a0 + cc < s) ? (double)X[i * si + (int64_t)(a0 + cc) * sa] : 0.0;
      xb[rr][cc] = (ok && b0 + cc < s) ? (double)X[i * si + (int64_t)(b0 + cc) * sa] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 64; ++rr) acc += xa[rr][ty] * xb[rr][tx];
    __syncthreads();
  }
  const int a = a0 + ty, b = b0 + tx;
  if (a < s && b < s) gp[((int64_t)blockIdx.z * s + a) * s + b] = acc;
}

__global__ void gram_sum_kernel(const double *__restrict__ gp, int32_t nsplit, int32_t s,
                                double *__restrict__ G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s * s) return;
  double acc = 0.0;
  for (int k = 0; k < nsplit; ++k) acc += gp[(int64_t)k * s * s + t];
  G[t] = acc;
}

template <typename T>
hipError_t launch_gram(const T *X, int64_t si, int64_t sa, int64_t n, int32_t s, double *scratch,
                       int32_t nsplit, double *G, hipStream_t st) {
  const int64_t rows_per = ((n + nsplit - 1) / nsplit + 63) / 64 * 64;
  dim3 grid((unsigned)((s + 15) / 16), (unsigned)((s + 15) / 16), (unsigned)nsplit);
  gram_partial_kernel<T><<<grid, 256, 0, st>>>(X, si, sa, n, s, rows_per, scratch);
  gram_sum_kernel<<<(unsigned)((s * s + 255) / 256), 256, 0, st>>>(scratch, nsplit, s, G);
  return hipGetLastError();
}
template hipError_t launch_gram<double>(const double *, int64_t, int64_t, int64_t, int32_t, double *,
                                        int32_t, double *, hipStream_t);
template hipError_t launch_gram<float>(const float *, int64_t, int64_t, int64_t, int32_t, double *,
                                       int32_t, double *, hipStream_t);

// ---------------------------------------------------------------------------
// Eigenvalues of a symmetric N x N matrix (N <= 256, row-major, overwritten),
// one workgroup of 1024 threads:
//  1. Householder reduction to tridiagonal form T (d on the diagonal, e next
//     to it): for k = 0..N-3 the reflector H = I - beta v v^T that maps
//     column k below the diagonal onto alpha e_1 is applied to the trailing
//     block as A22 -= v w^T + w v^T with p = beta A22 v, w = p - K v,
//     K = (beta/2) v.p (the symmetric rank-2 form of H A22 H; Golub & Van
//     Loan, Section 8.3.1).  Four barriers per step: the threads that update
//     row k+1 also sum the squares the next step needs.
//  2. each eigenvalue of T by multisection on the Sturm count (the number of
//     negative pivots of T - x I is the number of eigenvalues below x): a
//     group of 1024/NMAX threads per eigenvalue evaluates that many points of
//     its interval at once, from the Gershgorin interval down to 2 ulp or
//     1e-22 ||T||.
// Only eigenvalues are formed.  For N <= 128 the matrix lives in LDS (row
// stride N + 1) for the whole reduction, else in the global work buffer.
// ---------------------------------------------------------------------------
template <bool IN_LDS>
__global__ __launch_bounds__(1024) void tridiag_eig_kernel(double *__restrict__ Ag, int32_t N,
                                                           double *__restrict__ eig) {
  constexpr int NMAX = IN_LDS ? 128 : 256;
  constexpr int TPR = 1024 / NMAX;  // threads per row, and per eigenvalue
  __shared__ double As[IN_LDS ? 128 * 129 : 1];
  __shared__ double v[NMAX], w[NMAX], d[NMAX], e[NMAX];
  __shared__ double red[16];
  __shared__ double s_tail, bounds[3];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double *A = IN_LDS ? As : Ag;
  const int ld = IN_LDS ? N + 1 : N;
  if (IN_LDS)
    for (int x = tid; x < N * N; x += 1024) As[(x / N) * ld + x % N] = Ag[x];
  __syncthreads();
  // sum over the block in a fixed order, returned to every thread (one
  // barrier; red is next written only after at least one more barrier)
  auto block_sum = [&](double x) -> double {
    x = wave_sum(x);
    if (lane == 0) red[wv] = x;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q];
    return t;
  };
  // sum of squares of row r right of column c0 (all threads)
  auto row_tail = [&](int r, int c0) -> double {
    double sq = 0.0;
    for (int j = c0 + tid; j < N; j += 1024) sq += A[r * ld + j] * A[r * ld + j];
    return block_sum(sq);
  };
  const int rsub = tid / TPR, part = tid % TPR;
  double tail = N > 2 ? row_tail(0, 2) : 0.0;
  for (int k = 0; k + 2 < N; ++k) {
    const int i0 = k + 1;
    // column k below the diagonal is row k right of it (A is symmetric)
    const double x0 = A[k * ld + i0];
    if (tail == 0.0) {  // already tridiagonal in this column
      if (tid == 0) {
        d[k] = A[k * ld + k];
        e[k] = x0;
      }
      __syncthreads();  // every thread has read red from the previous sum
      tail = k + 3 < N ? row_tail(i0, i0 + 2) : 0.0;
      continue;
    }
    const double alpha = -copysign(sqrt(tail + x0 * x0), x0);
    const double v0 = x0 - alpha;  // no cancellation: x0 and alpha differ in sign
    const double beta = 2.0 / (tail + v0 * v0);
    for (int j = i0 + tid; j < N; j += 1024) v[j] = j == i0 ? v0 : A[k * ld + j];
    __syncthreads();
    // p = beta A22 v, kept in w
    const int i = i0 + rsub;
    double acc = 0.0;
    if (i < N)
      for (int j = i0 + part; j < N; j += TPR) acc += A[i * ld + j] * v[j];
#pragma unroll
    for (int off = TPR / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (i < N && part == 0) w[i] = beta * acc;
    __syncthreads();
    const double K = 0.5 * beta * block_sum(tid + i0 < N ? v[tid + i0] * w[tid + i0] : 0.0);
    // A22 -= v (p - K v)^T + (p - K v) v^T; row i0's group also sums the
    // squares of its new entries right of i0 + 1 (the next step's tail)
    double sq = 0.0;
    if (i < N) {
      const double vi = v[i], wi = w[i] - K * v[i];
      for (int j = i0 + part; j < N; j += TPR) {
        const double a_new = A[i * ld + j] - (vi * (w[j] - K * v[j]) + wi * v[j]);
        A[i * ld + j] = a_new;
        if (j >= i0 + 2) sq += a_new * a_new;
      }
    }
    if (rsub == 0) {
#pragma unroll
      for (int off = TPR / 2; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
      if (part == 0) s_tail = sq;
    }
    if (tid == 0) {
      d[k] = A[k * ld + k];
      e[k] = alpha;
    }
    __syncthreads();
    tail = s_tail;
  }
  if (tid == 0) {
    d[N - 2] = A[(N - 2) * ld + N - 2];
    d[N - 1] = A[(N - 1) * ld + N - 1];
    e[N - 2] = A[(N - 2) * ld + N - 1];
    // Gershgorin interval of T and the pivot floor of the Sturm recurrence
    double lo = 0.0, hi = 0.0, emax2 = 0.0;
    for (int q = 0; q < N; ++q) {
      const double r = (q > 0 ? fabs(e[q - 1]) : 0.0) + (q + 1 < N ? fabs(e[q]) : 0.0);
      lo = q == 0 ? d[q] - r : fmin(lo, d[q] - r);
      hi = q == 0 ? d[q] + r : fmax(hi, d[q] + r);
      if (q + 1 < N) emax2 = fmax(emax2, e[q] * e[q]);
    }
    bounds[0] = lo;
    bounds[1] = hi;
    bounds[2] = 2.2250738585072014e-308 * fmax(1.0, emax2);
  }
  __syncthreads();
  for (int q = tid; q + 1 < N; q += 1024) e[q] = e[q] * e[q];  // the recurrence uses e^2
  __syncthreads();
  // eigenvalue jv (ascending) by the TPR threads of group rsub: each
  // iteration splits [a, b] at TPR points; the group keeps the subinterval
  // whose left end has at most jv eigenvalues below it and whose right end
  // more (a and b stay identical across the group)
  const int jv = rsub;
  if (jv < N) {
    const double pivmin = bounds[2];
    const double tnorm = fmax(fabs(bounds[0]), fabs(bounds[1]));
    double a = bounds[0], b = bounds[1];
    for (int it = 0; it < 64; ++it) {
      if (b - a <= fmax(4.440892098500626e-16 * fmax(fabs(a), fabs(b)), 1e-22 * tnorm)) break;
      const double x = a + (b - a) * (double)(part + 1) / (double)(TPR + 1);
      int cnt = 0;
      double qv = d[0] - x;
      if (fabs(qv) < pivmin) qv = -pivmin;
      cnt += qv < 0.0;
      for (int r = 1; r < N; ++r) {
        qv = d[r] - x - e[r - 1] / qv;
        if (fabs(qv) < pivmin) qv = -pivmin;
        cnt += qv < 0.0;
      }
      double na = cnt > jv ? a : x, nb = cnt > jv ? x : b;
#pragma unroll
      for (int off = TPR / 2; off >= 1; off >>= 1) {
        na = fmax(na, __shfl_xor(na, off, 64));
        nb = fmin(nb, __shfl_xor(nb, off, 64));
      }
      a = na;
      b = nb;
    }
    if (part == 0) eig[jv] = 0.5 * (a + b);
  }
}

// Copy the s x s Gram matrix into an N x N (N even) work matrix.
__global__ void pad_square_kernel(const double *__restrict__ G, int32_t s, double *__restrict__ A,
                                  int32_t N) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N * N; e += gridDim.x * blockDim.x) {
    const int i = e / N, j = e % N;
    A[e] = (i < s && j < s) ? G[i * s + j] : 0.0;
  }
}

// sigma = sqrt(max(lambda, 0)) in descending order (rank by comparison,
// ties by index), the k largest kept, H^ = sum sigma ln(1/sigma).
__global__ void rp_finish_kernel(const double *__restrict__ eig, int32_t N, int32_t k,
                                 double *__restrict__ sigma, double *__restrict__ scal) {
  __shared__ double sv[256];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += blockDim.x) {
    const double lam = eig[i];
    const double si = lam > 0.0 ? sqrt(lam) : 0.0;
    int rank = 0;
    for (int j = 0; j < N; ++j) {
      const double lj = eig[j];
      const double sj = lj > 0.0 ? sqrt(lj) : 0.0;
      if (sj > si || (sj == si && j < i)) ++rank;
    }
    sv[rank] = si;
  }
  __syncthreads();
  if (tid == 0) {
    // S_NORM > 0: singular values of (R / tr R) Pi = those of R Pi / tr R
    const double nm = scal[S_NORM] > 0.0 ? scal[S_NORM] : 1.0;
    double h = 0.0;
    for (int i = 0; i < k && i < N; ++i) {
      const double sg = sv[i] * nm;
      sigma[i] = sg;
      if (sg > 0.0) h += sg * log(1.0 / sg);
    }
    scal[S_ENT] = h;
    scal[S_SE] = 0.0;
    if (!isfinite(h)) scal[S_FLAG] = 1.0;
  }
}

hipError_t launch_rp_spectrum(const double *G, int32_t s, int32_t k, double *work, double *eig,
                              double *sigma, double *scal, hipStream_t st) {
  const int32_t N = (s + 1) / 2 * 2;
  if (N > 256) return hipErrorInvalidValue;
  pad_square_kernel<<<64, 256, 0, st>>>(G, s, work, N);
  if (N <= 128)
    tridiag_eig_kernel<true><<<1, 1024, 0, st>>>(work, N, eig);
  else
    tridiag_eig_kernel<false><<<1, 1024, 0, st>>>(work, N, eig);
  rp_finish_kernel<<<1, 256, 0, st>>>(eig, N, k, sigma, scal);
  return hipGetLastError();
}

}  // namespace ent
