/*
 * oracle.c -- plain, slow, FP64 CPU reference for the randomized von Neumann
 * entropy estimators of Kontopoulou, Dexter, Szpankowski, Grama and Drineas,
 * "Randomized Linear Algebra Approaches to Estimate the Von Neumann Entropy of
 * Density Matrices" (arXiv:1801.01072).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library: the only thing both sides have
 * in common is the *published definition* of the Philox4x32-10 counter-based
 * generator (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11) and the probe-mapping rule written below, each implemented
 * separately.
 *
 * Everything is computed in IEEE double precision with plain loops: no
 * blocking, no fusion, no reordering beyond what the paper states.
 * FP32-stored matrices are widened element by element to double.
 *
 * Parity pins (see tests/test_oracle_*.py): Philox known-answer vectors, closed
 * forms for the Chebyshev coefficients (Lemma 3), the tight truncation bound
 * at x = 0, pure / maximally mixed / diagonal states, the Poisson spectrum
 * (Section 6, tridiagonal experiment), exhaustive 2^n sign enumeration for
 * Hutchinson unbiasedness (Lemma 1), finite differences for the MLP.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Matrix descriptor (the oracle's own; not shared with the GPU library).    */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t n;
  int32_t layout; /* 0 = dense row-major, 1 = CSR                          */
  int32_t dtype;  /* 0 = double, 1 = float                                 */
  int64_t ld;     /* dense leading dimension (elements)                    */
  const void *values;
  const int64_t *row_ptr; /* CSR: n+1 offsets                               */
  const int32_t *col_idx; /* CSR: nnz column indices                        */
} orc_matrix;

typedef struct {
  double entropy;  /* mean of the per-probe values                         */
  double p1_est;   /* power-method estimate of the largest eigenvalue      */
  double u;        /* upper end of the approximation interval              */
  double std_err;  /* sample standard error of the mean over probes        */
} orc_result;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox S-box on a */
/* 128-bit counter with a 64-bit key, key bumped by the Weyl constants      */
/* between rounds.                                                           */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Probe entry g_j[i] (the paper draws i.i.d. Gaussian vectors, Lemma 1 and
 * Algorithms 1-2; Rademacher signs are the other unbiased choice, and the
 * power method starts from a random sign vector, Algorithm 4).
 *   key     = (seed mod 2^32, seed >> 32)
 *   counter = (i mod 2^32, block, stream, i >> 32)
 *   dist 0 (Rademacher): block = j >> 7; word = out[(j >> 5) & 3];
 *                        bit (j & 31) set -> -1, clear -> +1
 *   dist 1 (Gaussian):   block = j >> 1; a = (out1:out0) >> 11,
 *                        b = (out3:out2) >> 11 as 53-bit integers;
 *                        u1 = (a + 1) 2^-53 in (0,1], u2 = b 2^-53 in [0,1);
 *                        r = sqrt(-2 ln u1), theta = 2 pi u2;
 *                        even j -> r cos theta, odd j -> r sin theta.
 * Streams: 0 = trace probes, 1 = power-method start vectors, 2 = sketch.
 */
double orc_probe_value(uint64_t seed, int32_t dist, uint32_t stream, int64_t i,
                       int64_t j) {
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t ctr[4], out[4];
  ctr[0] = (uint32_t)((uint64_t)i & 0xffffffffu);
  ctr[2] = stream;
  ctr[3] = (uint32_t)((uint64_t)i >> 32);
  if (dist == 0) {
    ctr[1] = (uint32_t)((uint64_t)j >> 7);
    orc_philox4x32_10(ctr, key, out);
    uint32_t w = out[(j >> 5) & 3];
    return ((w >> (j & 31)) & 1u) ? -1.0 : 1.0;
  }
  ctr[1] = (uint32_t)((uint64_t)j >> 1);
  orc_philox4x32_10(ctr, key, out);
  uint64_t a = (((uint64_t)out[1] << 32) | out[0]) >> 11;
  uint64_t b = (((uint64_t)out[3] << 32) | out[2]) >> 11;
  double u1 = ((double)a + 1.0) * (1.0 / 9007199254740992.0);
  double u2 = (double)b * (1.0 / 9007199254740992.0);
  double r = sqrt(-2.0 * log(u1));
  double theta = 2.0 * ORC_PI * u2;
  return (j & 1) ? r * sin(theta) : r * cos(theta);
}

/* Fill g (length n) with probe column j. */
void orc_probe_vector(uint64_t seed, int32_t dist, uint32_t stream, int64_t n,
                      int64_t j, double *g) {
  for (int64_t i = 0; i < n; ++i) g[i] = orc_probe_value(seed, dist, stream, i, j);
}

/* ------------------------------------------------------------------------- */
/* y = R x                                                                    */
/* ------------------------------------------------------------------------- */
static double orc_elem_dense(const orc_matrix *R, int64_t i, int64_t j) {
  if (R->dtype == 0) return ((const double *)R->values)[i * R->ld + j];
  return (double)((const float *)R->values)[i * R->ld + j];
}

void orc_matvec(const orc_matrix *R, const double *x, double *y) {
  int64_t n = R->n;
  if (R->layout == 0) {
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int64_t j = 0; j < n; ++j) acc += orc_elem_dense(R, i, j) * x[j];
      y[i] = acc;
    }
  } else {
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int64_t e = R->row_ptr[i]; e < R->row_ptr[i + 1]; ++e) {
        double v = R->dtype == 0 ? ((const double *)R->values)[e]
                                 : (double)((const float *)R->values)[e];
        acc += v * x[R->col_idx[e]];
      }
      y[i] = acc;
    }
  }
}

static double orc_dot(int64_t n, const double *a, const double *b) {
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) acc += a[i] * b[i];
  return acc;
}

/* ------------------------------------------------------------------------- */
/* Power method (Algorithm 4, Appendix A), q trials of t iterations from a   */
/* random sign vector, Rayleigh quotient of the last iterate, max over       */
/* trials.  The iterate is divided by its 2-norm after every product: the    */
/* Rayleigh quotient is scale invariant, so this is the same estimate while  */
/* avoiding under/overflow of p_1^t.                                          */
/* ------------------------------------------------------------------------- */
double orc_power_method(const orc_matrix *R, int32_t t, int32_t q,
                        uint64_t seed) {
  int64_t n = R->n;
  double *x = (double *)malloc(sizeof(double) * n);
  double *y = (double *)malloc(sizeof(double) * n);
  double best = -INFINITY;
  for (int32_t trial = 0; trial < q; ++trial) {
    orc_probe_vector(seed, 0, 1u, n, trial, x);
    for (int32_t it = 0; it < t; ++it) {
      orc_matvec(R, x, y);
      double nrm = sqrt(orc_dot(n, y, y));
      for (int64_t i = 0; i < n; ++i) x[i] = y[i] / nrm;
    }
    orc_matvec(R, x, y);
    double rq = orc_dot(n, x, y) / orc_dot(n, x, x);
    if (rq > best) best = rq;
  }
  free(x);
  free(y);
  return best;
}

/* ------------------------------------------------------------------------- */
/* Chebyshev coefficients of h(x) = x ln x on [0,u] (Lemma 3, Section 3):    */
/*   alpha_0 = (u/2)(ln(u/4) + 1), alpha_1 = (u/4)(2 ln(u/4) + 3),           */
/*   alpha_w = (-1)^w u / (w^3 - w), w >= 2.                                 */
/* ------------------------------------------------------------------------- */
void orc_cheb_coeffs(double u, int32_t m, double *alpha) {
  for (int32_t w = 0; w <= m; ++w) {
    if (w == 0)
      alpha[w] = 0.5 * u * (log(u / 4.0) + 1.0);
    else if (w == 1)
      alpha[w] = 0.25 * u * (2.0 * log(u / 4.0) + 3.0);
    else {
      double dw = (double)w;
      alpha[w] = ((w & 1) ? -u : u) / (dw * dw * dw - dw);
    }
  }
}

/*
 * Chebyshev interpolant of h(x) = x ln x on [lo, u] at the N = m + 1
 * Chebyshev points of the first kind (not in the paper: the "lower spectral
 * cutoff" extension).  x_i = (u+lo)/2 + (u-lo)/2 cos(pi (i + 1/2) / N),
 * c_w = (2/N) sum_i h(x_i) cos(w pi (i + 1/2) / N), c_0 halved.  With lo = 0
 * and N -> infinity this tends to the closed form of Lemma 3.
 */
void orc_cheb_interp_coeffs(double lo, double u, int32_t m, int32_t npts,
                            double *c) {
  int32_t N = npts > 0 ? npts : m + 1;
  for (int32_t w = 0; w <= m; ++w) {
    double acc = 0.0;
    for (int32_t i = 0; i < N; ++i) {
      double th = ORC_PI * ((double)i + 0.5) / (double)N;
      double x = 0.5 * (u + lo) + 0.5 * (u - lo) * cos(th);
      double h = x > 0.0 ? x * log(x) : 0.0;
      acc += h * cos((double)w * th);
    }
    c[w] = (2.0 / (double)N) * acc;
  }
  c[0] *= 0.5;
}

/* Nodes of the lower-cutoff coefficients used by the estimator: a fixed
 * 1024-point rule (2(m+1) beyond degree 511), so the coefficients of degree
 * w do not depend on m and partial sums over the degree are nested. */
int32_t orc_cutoff_nodes(int32_t m) { return (m + 1) <= 512 ? 1024 : 2 * (m + 1); }

/*
 * Scalar Clenshaw (Appendix B): b_k = alpha_k + 2 t b_{k+1} - b_{k+2}, with
 * t = (2x - (u+lo)) / (u - lo) the map of [lo,u] onto [-1,1] (lo = 0 gives
 * the paper's 2x/u - 1), f_m(x) = (alpha_0 + b_0 - b_2) / 2.
 */
double orc_cheb_eval_scalar(const double *alpha, int32_t m, double lo, double u,
                            double x) {
  double t = (2.0 * x - (u + lo)) / (u - lo);
  double b1 = 0.0, b2 = 0.0, b0 = 0.0; /* b_{k+1}, b_{k+2}, b_k */
  double bk2_at_0 = 0.0;               /* b_2 when k reaches 0   */
  for (int32_t k = m; k >= 0; --k) {
    b0 = alpha[k] + 2.0 * t * b1 - b2;
    if (k == 0) bk2_at_0 = b2;
    b2 = b1;
    b1 = b0;
  }
  return 0.5 * (alpha[0] + b0 - bk2_at_0);
}

/*
 * g^T f_m(R) g by the matrix-vector Clenshaw recurrence (Algorithm 5,
 * Appendix B), generalised to [lo, u]:
 *   y_{m+1} = y_{m+2} = 0,
 *   y_k = alpha_k g + 2 X y_{k+1} - y_{k+2},  X = (2R - (u+lo) I)/(u - lo),
 *   g^T f_m(R) g = (alpha_0 g^T g + g^T (y_0 - y_2)) / 2.
 * With lo = 0, 2X y = (4/u) R y - 2 y as in the paper.
 */
double orc_cheb_quadform(const orc_matrix *R, const double *alpha, int32_t m,
                         double lo, double u, const double *g) {
  int64_t n = R->n;
  double *y1 = (double *)calloc(n, sizeof(double)); /* y_{k+1} */
  double *y2 = (double *)calloc(n, sizeof(double)); /* y_{k+2} */
  double *yk = (double *)calloc(n, sizeof(double));
  double *ry = (double *)calloc(n, sizeof(double));
  double *ysave2 = (double *)calloc(n, sizeof(double)); /* y_2 */
  double a = 2.0 / (u - lo);
  double sh = (u + lo) / (u - lo);
  for (int32_t k = m; k >= 0; --k) {
    orc_matvec(R, y1, ry);
    for (int64_t i = 0; i < n; ++i) {
      double xy = a * ry[i] - sh * y1[i]; /* (X y_{k+1})_i */
      yk[i] = alpha[k] * g[i] + 2.0 * xy - y2[i];
    }
    if (k == 2) memcpy(ysave2, yk, sizeof(double) * n);
    double *tmp = y2;
    y2 = y1;
    y1 = yk;
    yk = tmp;
  }
  /* y1 now holds y_0 */
  double gy0 = orc_dot(n, g, y1);
  double gy2 = (m >= 2) ? orc_dot(n, g, ysave2) : 0.0;
  double res = 0.5 * (alpha[0] * orc_dot(n, g, g) + gy0 - gy2);
  free(y1); free(y2); free(yk); free(ry); free(ysave2);
  return res;
}

/*
 * Forward three-term recurrence, used only as a cross-check of Clenshaw:
 * d_k = g^T T_k(X) g for k = 0..m, with T_0 g = g, T_1 g = X g,
 * T_{k+1} g = 2 X T_k g - T_{k-1} g.
 */
void orc_cheb_moments_forward(const orc_matrix *R, double lo, double u,
                              int32_t m, const double *g, double *d) {
  int64_t n = R->n;
  double *tm1 = (double *)malloc(sizeof(double) * n);
  double *tk = (double *)malloc(sizeof(double) * n);
  double *tp1 = (double *)malloc(sizeof(double) * n);
  double *r = (double *)malloc(sizeof(double) * n);
  double a = 2.0 / (u - lo);
  double sh = (u + lo) / (u - lo);
  memcpy(tk, g, sizeof(double) * n);
  d[0] = orc_dot(n, g, tk);
  for (int32_t k = 0; k < m; ++k) {
    orc_matvec(R, tk, r);
    for (int64_t i = 0; i < n; ++i) {
      double xt = a * r[i] - sh * tk[i];
      tp1[i] = (k == 0) ? xt : 2.0 * xt - tm1[i];
    }
    d[k + 1] = orc_dot(n, g, tp1);
    double *tmp = tm1;
    tm1 = tk;
    tk = tp1;
    tp1 = tmp;
  }
  free(tm1); free(tk); free(tp1); free(r);
}

/*
 * The Taylor quadratic form of Algorithm 1 (Section 2), taken literally:
 *   sum_{k=1}^{m} g^T R (I - R/u)^k g / k
 * computed as w = R g; v = g; for k = 1..m: v <- v - (R v)/u, acc += (w.v)/k
 * (R symmetric, so g^T R C^k g = (R g) . (C^k g)).
 */
double orc_taylor_quadform(const orc_matrix *R, double u, int32_t m,
                           const double *g) {
  int64_t n = R->n;
  double *w = (double *)malloc(sizeof(double) * n);
  double *v = (double *)malloc(sizeof(double) * n);
  double *rv = (double *)malloc(sizeof(double) * n);
  orc_matvec(R, g, w);
  memcpy(v, g, sizeof(double) * n);
  double acc = 0.0;
  for (int32_t k = 1; k <= m; ++k) {
    orc_matvec(R, v, rv);
    for (int64_t i = 0; i < n; ++i) v[i] = v[i] - rv[i] / u;
    acc += orc_dot(n, w, v) / (double)k;
  }
  free(w); free(v); free(rv);
  return acc;
}

/*
 * Full estimators (Algorithms 1 and 2).
 *   method 0 (Taylor):    h_j = ln(1/u) + sum_{k=1}^m g_j^T R (I - R/u)^k g_j / k
 *   method 1 (Chebyshev): h_j = -g_j^T f_m(R) g_j,   f_m on [lo, u]
 * u = min{1, c p~1} with p~1 from the power method (t iterations, q trials).
 * If u_override > 0 it replaces the power-method value (used by tests that
 * need the exact interval, e.g. u = p_1).  lo is the lower end of the
 * approximation interval (0 = the paper); lo > 0 uses the Chebyshev
 * projection above with orc_cutoff_nodes(m) nodes.
 * probe_idx selects which probes to evaluate (NULL = 0..s-1); per_probe
 * receives h_j for the selected probes; out->entropy is their mean.
 * Probes are independent, so they run in parallel; the mean is formed in
 * index order afterwards, so the result does not depend on the thread count.
 */
int orc_estimate(const orc_matrix *R, int32_t method, int32_t m, int32_t s,
                 uint64_t seed, int32_t t, int32_t q, double c, int32_t dist,
                 double lo, double u_override, const int32_t *probe_idx,
                 int32_t nsel, double *per_probe, orc_result *out) {
  if (!R || !out || m < 1 || s < 1 || R->n < 1) return -1;
  int64_t n = R->n;
  double p1 = u_override > 0.0 ? u_override : orc_power_method(R, t, q, seed);
  double u = u_override > 0.0 ? u_override : fmin(1.0, c * p1);
  int32_t cnt = probe_idx ? nsel : s;
  double *alpha = (double *)malloc(sizeof(double) * (m + 1));
  if (method == 1) {
    if (lo > 0.0)
      orc_cheb_interp_coeffs(lo, u, m, orc_cutoff_nodes(m), alpha);
    else
      orc_cheb_coeffs(u, m, alpha);
  }
  double *h = (double *)malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t p = 0; p < cnt; ++p) {
    int64_t j = probe_idx ? probe_idx[p] : p;
    double *g = (double *)malloc(sizeof(double) * n);
    orc_probe_vector(seed, dist, 0u, n, j, g);
    if (method == 0)
      h[p] = log(1.0 / u) + orc_taylor_quadform(R, u, m, g);
    else
      h[p] = -orc_cheb_quadform(R, alpha, m, lo, u, g);
    free(g);
  }
  double mean = 0.0;
  for (int32_t p = 0; p < cnt; ++p) mean += h[p];
  mean /= (double)cnt;
  double var = 0.0;
  for (int32_t p = 0; p < cnt; ++p) var += (h[p] - mean) * (h[p] - mean);
  out->entropy = mean;
  out->p1_est = p1;
  out->u = u;
  out->std_err = cnt > 1 ? sqrt(var / ((double)cnt * (double)(cnt - 1))) : 0.0;
  if (per_probe)
    for (int32_t p = 0; p < cnt; ++p) per_probe[p] = h[p];
  free(h);
  free(alpha);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Hermitian density matrices (Section 4).  R = B + iC with B symmetric and  */
/* C skew-symmetric; tr R = tr B (Theorem of Section 4), so Lemma 1 applies */
/* to Re[f(R)] with real probes.  Algorithms 1c / 2c are Algorithms 1 / 2   */
/* with g^T Re[...] g, and with u = 1 in place of the power-method bound.    */
/* Complex arithmetic is C99 double complex, element by element.            */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t n;
  int32_t dtype; /* 0 = complex double, 1 = complex float: interleaved (re, im) */
  int64_t ld;    /* leading dimension in complex elements                     */
  const void *values;
} orc_zmatrix;

static double complex orc_zelem(const orc_zmatrix *R, int64_t i, int64_t j) {
  int64_t o = 2 * (i * R->ld + j);
  if (R->dtype == 0) {
    const double *v = (const double *)R->values;
    return v[o] + I * v[o + 1];
  }
  const float *v = (const float *)R->values;
  return (double)v[o] + I * (double)v[o + 1];
}

/* y = R x, complex x and y. */
void orc_zmatvec(const orc_zmatrix *R, const double complex *x, double complex *y) {
  for (int64_t i = 0; i < R->n; ++i) {
    double complex acc = 0.0;
    for (int64_t j = 0; j < R->n; ++j) acc += orc_zelem(R, i, j) * x[j];
    y[i] = acc;
  }
}

static double orc_znorm2(int64_t n, const double complex *x) {
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) acc += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
  return acc;
}

/*
 * Power method on Hermitian R (Algorithm 4 with a complex iterate): the
 * start vector of trial q is x_i = s_i + i s_{n+i}, s the Rademacher signs of
 * stream 1 at indices 0..2n-1; x <- R x / ||R x|| t times; Rayleigh quotient
 * Re(x^H R x) / x^H x of the last iterate; maximum over trials.  (The paper
 * uses u = 1 for Hermitian R because no accuracy bound is known for this
 * iteration; the estimator calls it only when asked.)
 */
double orc_zpower_method(const orc_zmatrix *R, int32_t t, int32_t q, uint64_t seed) {
  int64_t n = R->n;
  double complex *x = (double complex *)malloc(sizeof(double complex) * n);
  double complex *y = (double complex *)malloc(sizeof(double complex) * n);
  double best = -INFINITY;
  for (int32_t trial = 0; trial < q; ++trial) {
    for (int64_t i = 0; i < n; ++i)
      x[i] = orc_probe_value(seed, 0, 1u, i, trial) + I * orc_probe_value(seed, 0, 1u, n + i, trial);
    for (int32_t it = 0; it < t; ++it) {
      orc_zmatvec(R, x, y);
      double nrm = sqrt(orc_znorm2(n, y));
      for (int64_t i = 0; i < n; ++i) x[i] = y[i] / nrm;
    }
    orc_zmatvec(R, x, y);
    double complex xy = 0.0;
    for (int64_t i = 0; i < n; ++i) xy += conj(x[i]) * y[i];
    double rq = creal(xy) / orc_znorm2(n, x);
    if (rq > best) best = rq;
  }
  free(x);
  free(y);
  return best;
}

/*
 * g^T Re[f_m(R)] g for real g by the vector Clenshaw recurrence (Algorithm 5)
 * with complex y_k:  y_k = alpha_k g + 2 X y_{k+1} - y_{k+2},
 * X = (2R - (u+lo) I)/(u - lo); f_m(R) g = (alpha_0 g + y_0 - y_2)/2, and
 * since g is real, g^T Re[f_m(R)] g = (alpha_0 g^T g + g^T Re(y_0 - y_2))/2.
 */
double orc_zcheb_quadform(const orc_zmatrix *R, const double *alpha, int32_t m, double lo,
                          double u, const double *g) {
  int64_t n = R->n;
  double complex *y1 = (double complex *)calloc(n, sizeof(double complex));
  double complex *y2 = (double complex *)calloc(n, sizeof(double complex));
  double complex *yk = (double complex *)calloc(n, sizeof(double complex));
  double complex *ry = (double complex *)calloc(n, sizeof(double complex));
  double complex *ysave2 = (double complex *)calloc(n, sizeof(double complex));
  double a = 2.0 / (u - lo);
  double sh = (u + lo) / (u - lo);
  for (int32_t k = m; k >= 0; --k) {
    orc_zmatvec(R, y1, ry);
    for (int64_t i = 0; i < n; ++i) yk[i] = alpha[k] * g[i] + 2.0 * (a * ry[i] - sh * y1[i]) - y2[i];
    if (k == 2) memcpy(ysave2, yk, sizeof(double complex) * n);
    double complex *tmp = y2;
    y2 = y1;
    y1 = yk;
    yk = tmp;
  }
  double gg = 0.0, gy0 = 0.0, gy2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    gg += g[i] * g[i];
    gy0 += g[i] * creal(y1[i]);
    if (m >= 2) gy2 += g[i] * creal(ysave2[i]);
  }
  double res = 0.5 * (alpha[0] * gg + gy0 - gy2);
  free(y1); free(y2); free(yk); free(ry); free(ysave2);
  return res;
}

/* d_k = g^T Re[T_k(X)] g, k = 0..m, by the forward three-term recurrence. */
void orc_zcheb_moments_forward(const orc_zmatrix *R, double lo, double u, int32_t m,
                               const double *g, double *d) {
  int64_t n = R->n;
  double complex *tm1 = (double complex *)malloc(sizeof(double complex) * n);
  double complex *tk = (double complex *)malloc(sizeof(double complex) * n);
  double complex *tp1 = (double complex *)malloc(sizeof(double complex) * n);
  double complex *r = (double complex *)malloc(sizeof(double complex) * n);
  double a = 2.0 / (u - lo);
  double sh = (u + lo) / (u - lo);
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    tk[i] = g[i];
    acc += g[i] * g[i];
  }
  d[0] = acc;
  for (int32_t k = 0; k < m; ++k) {
    orc_zmatvec(R, tk, r);
    acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double complex xt = a * r[i] - sh * tk[i];
      tp1[i] = (k == 0) ? xt : 2.0 * xt - tm1[i];
      acc += g[i] * creal(tp1[i]);
    }
    d[k + 1] = acc;
    double complex *tmp = tm1;
    tm1 = tk;
    tk = tp1;
    tp1 = tmp;
  }
  free(tm1); free(tk); free(tp1); free(r);
}

/*
 * The Taylor form of Algorithm 1c generalised to an interval [0, u]:
 *   sum_{k=1}^{m} g^T Re[R (I - R/u)^k] g / k      (u = 1: Algorithm 1c)
 * with v_k = (I - R/u)^k g (complex) and w = R g: R Hermitian means
 * R^T = conj(R), so g^T R v = (R^T g)^T v = sum_i conj(w_i) v_i for real g.
 */
double orc_ztaylor_quadform(const orc_zmatrix *R, double u, int32_t m, const double *g) {
  int64_t n = R->n;
  double complex *w = (double complex *)malloc(sizeof(double complex) * n);
  double complex *v = (double complex *)malloc(sizeof(double complex) * n);
  double complex *rv = (double complex *)malloc(sizeof(double complex) * n);
  for (int64_t i = 0; i < n; ++i) v[i] = g[i];
  orc_zmatvec(R, v, w);
  double acc = 0.0;
  for (int32_t k = 1; k <= m; ++k) {
    orc_zmatvec(R, v, rv);
    for (int64_t i = 0; i < n; ++i) v[i] = v[i] - rv[i] / u;
    double complex wv = 0.0;
    for (int64_t i = 0; i < n; ++i) wv += conj(w[i]) * v[i];
    acc += creal(wv) / (double)k;
  }
  free(w); free(v); free(rv);
  return acc;
}

/*
 * Algorithms 1c (method 0) and 2c (method 1) on Hermitian R: the estimators
 * of orc_estimate with Re[...] quadratic forms.  u_override > 0 sets u (the
 * paper's choice for Hermitian R is u = 1); otherwise u = min{1, c p~1} with
 * p~1 from orc_zpower_method.  probe_idx as in orc_estimate.
 */
int orc_zestimate(const orc_zmatrix *R, int32_t method, int32_t m, int32_t s, uint64_t seed,
                  int32_t t, int32_t q, double c, int32_t dist, double lo, double u_override,
                  const int32_t *probe_idx, int32_t nsel, double *per_probe, orc_result *out) {
  if (!R || !out || m < 1 || s < 1 || R->n < 1) return -1;
  int64_t n = R->n;
  double p1 = u_override > 0.0 ? u_override : orc_zpower_method(R, t, q, seed);
  double u = u_override > 0.0 ? u_override : fmin(1.0, c * p1);
  int32_t cnt = probe_idx ? nsel : s;
  double *alpha = (double *)malloc(sizeof(double) * (m + 1));
  if (method == 1) {
    if (lo > 0.0)
      orc_cheb_interp_coeffs(lo, u, m, orc_cutoff_nodes(m), alpha);
    else
      orc_cheb_coeffs(u, m, alpha);
  }
  double *h = (double *)malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t p = 0; p < cnt; ++p) {
    int64_t j = probe_idx ? probe_idx[p] : p;
    double *g = (double *)malloc(sizeof(double) * n);
    orc_probe_vector(seed, dist, 0u, n, j, g);
    if (method == 0)
      h[p] = log(1.0 / u) + orc_ztaylor_quadform(R, u, m, g);
    else
      h[p] = -orc_zcheb_quadform(R, alpha, m, lo, u, g);
    free(g);
  }
  double mean = 0.0;
  for (int32_t p = 0; p < cnt; ++p) mean += h[p];
  mean /= (double)cnt;
  double var = 0.0;
  for (int32_t p = 0; p < cnt; ++p) var += (h[p] - mean) * (h[p] - mean);
  out->entropy = mean;
  out->p1_est = p1;
  out->u = u;
  out->std_err = cnt > 1 ? sqrt(var / ((double)cnt * (double)(cnt - 1))) : 0.0;
  if (per_probe)
    for (int32_t p = 0; p < cnt; ++p) per_probe[p] = h[p];
  free(h);
  free(alpha);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Exact entropy: eigenvalues by the cyclic Jacobi method, then              */
/* H = -sum p ln p over p above a round-off threshold (eqn. (1): 0 ln 0 = 0) */
/* ------------------------------------------------------------------------- */
/*
 * Cyclic Jacobi for a symmetric n x n matrix (row-major, copied).  Each
 * rotation zeroes A[p][q] with the classical stable choice of tan(theta).
 * Stops when the off-diagonal Frobenius norm is below tol * ||A||_F or after
 * max_sweeps sweeps.  eig receives the diagonal (unsorted).  If V != NULL it
 * receives the accumulated rotations (columns = eigenvectors).  Returns the
 * number of sweeps used.
 */
int orc_jacobi_eigen(int64_t n, const double *Ain, double *eig, double *V,
                     double tol, int32_t max_sweeps) {
  double *A = (double *)malloc(sizeof(double) * n * n);
  memcpy(A, Ain, sizeof(double) * n * n);
  if (V) {
    for (int64_t i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int64_t i = 0; i < n; ++i) V[i * n + i] = 1.0;
  }
  double fro = 0.0;
  for (int64_t i = 0; i < n * n; ++i) fro += A[i] * A[i];
  fro = sqrt(fro);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double off = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i + 1; j < n; ++j) off += 2.0 * A[i * n + j] * A[i * n + j];
    if (sqrt(off) <= tol * fro || fro == 0.0) break;
    for (int64_t p = 0; p < n - 1; ++p) {
      for (int64_t q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double app = A[p * n + p], aqq = A[q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double tt = (theta >= 0.0 ? 1.0 : -1.0) /
                    (fabs(theta) + sqrt(theta * theta + 1.0));
        double cs = 1.0 / sqrt(tt * tt + 1.0);
        double sn = tt * cs;
        /* A <- J^T A J with J the rotation in the (p,q) plane */
        for (int64_t k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int64_t k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
        A[p * n + q] = 0.0;
        A[q * n + p] = 0.0;
        if (V) {
          for (int64_t k = 0; k < n; ++k) {
            double vkp = V[k * n + p], vkq = V[k * n + q];
            V[k * n + p] = cs * vkp - sn * vkq;
            V[k * n + q] = sn * vkp + cs * vkq;
          }
        }
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) eig[i] = A[i * n + i];
  free(A);
  return sweep;
}

/* -sum p ln p over p > tau, tau = n * eps * max p (tiny or negative computed
 * eigenvalues are taken as zero, following the footnote to eqn. (1)). */
double orc_entropy_from_eigs(int64_t n, const double *p) {
  double pmax = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (p[i] > pmax) pmax = p[i];
  double tau = (double)n * 2.220446049250313e-16 * pmax;
  double h = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (p[i] > tau) h -= p[i] * log(p[i]);
  return h;
}

/* Exact entropy of a dense symmetric R (any storage) by Jacobi. */
double orc_exact_entropy(const orc_matrix *R) {
  int64_t n = R->n;
  double *A = (double *)malloc(sizeof(double) * n * n);
  double *e = (double *)malloc(sizeof(double) * n);
  if (R->layout == 0) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) A[i * n + j] = orc_elem_dense(R, i, j);
  } else {
    memset(A, 0, sizeof(double) * n * n);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = R->row_ptr[i]; k < R->row_ptr[i + 1]; ++k)
        A[i * n + R->col_idx[k]] = R->dtype == 0
                                       ? ((const double *)R->values)[k]
                                       : (double)((const float *)R->values)[k];
  }
  orc_jacobi_eigen(n, A, e, NULL, 1e-15, 100);
  double h = orc_entropy_from_eigs(n, e);
  free(A);
  free(e);
  return h;
}

/* ------------------------------------------------------------------------- */
/* Random projection (Algorithm 3, Section 5): R~ = R Pi (n x s), singular   */
/* values of R~ via the eigenvalues of the s x s Gram matrix R~^T R~ (Jacobi),*/
/* keep the k largest, H^ = sum sigma ln(1/sigma).                            */
/* ------------------------------------------------------------------------- */
double orc_rp_entropy_with_pi(const orc_matrix *R, const double *Pi, int32_t s,
                              int32_t k, double *sigma_out) {
  int64_t n = R->n;
  double *Rt = (double *)malloc(sizeof(double) * n * s); /* column-major n x s */
  double *col = (double *)malloc(sizeof(double) * n);
  for (int32_t c = 0; c < s; ++c) {
    for (int64_t i = 0; i < n; ++i) col[i] = Pi[i * s + c];
    orc_matvec(R, col, Rt + (int64_t)c * n);
  }
  double *G = (double *)malloc(sizeof(double) * s * s);
  for (int32_t a = 0; a < s; ++a)
    for (int32_t b = 0; b < s; ++b)
      G[a * s + b] = orc_dot(n, Rt + (int64_t)a * n, Rt + (int64_t)b * n);
  double *e = (double *)malloc(sizeof(double) * s);
  orc_jacobi_eigen(s, G, e, NULL, 1e-15, 100);
  /* sort descending (insertion sort: s is small) */
  for (int32_t a = 1; a < s; ++a) {
    double v = e[a];
    int32_t b = a - 1;
    while (b >= 0 && e[b] < v) {
      e[b + 1] = e[b];
      --b;
    }
    e[b + 1] = v;
  }
  double h = 0.0;
  for (int32_t a = 0; a < k && a < s; ++a) {
    double sg = e[a] > 0.0 ? sqrt(e[a]) : 0.0;
    if (sigma_out) sigma_out[a] = sg;
    if (sg > 0.0) h += sg * log(1.0 / sg);
  }
  free(Rt); free(col); free(G); free(e);
  return h;
}

/* Gaussian sketch, zero mean, variance 1/s (so that E[Pi Pi^T] = I). */
/*
 * Sketch matrices Pi (n x s, row-major) for Algorithm 3:
 *   kind 0, Gaussian:  Pi_jt = N(0,1)/sqrt(s) (probe generator, stream 2).
 *   kind 1, subsampled randomized Hadamard transform (Section 5.2):
 *           Pi = sqrt(N/s) D H S with N = 2^ceil(log2 n) (R padded with
 *           zeros to N), H the normalized Sylvester-Hadamard matrix,
 *           H_ji = (-1)^{popcount(j & i)} / sqrt(N), D_jj = +-1 and S
 *           sampling s columns uniformly with replacement, so
 *           Pi_jt = D_jj (-1)^{popcount(j & i_t)} / sqrt(s).
 *           The sqrt(N/s) scale makes E[Pi Pi^T] = I, the normalization
 *           under which the embedding bound for this construction holds.
 *   kind 2, input-sparsity transform (Section 5.2): Pi = D S with one
 *           entry D_jj in column h(j) of row j, h(j) uniform on 0..s-1.
 * Random draws (Philox4x32-10, counter (row mod 2^32, 0, stream, row >> 32),
 * key = seed): D_jj = -1 iff bit 0 of output word 0 of stream 3 at row j;
 * h(j) = floor(w1 s / 2^32) with w1 output word 1 of the same block
 * (multiply-shift reduction); i_t = output word 0 of stream 4 at row t,
 * reduced mod N (N a power of two).
 */
static void orc_philox_row(uint64_t seed, uint32_t stream, int64_t row, uint32_t out[4]) {
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)((uint64_t)row & 0xffffffffu), 0u, stream,
                     (uint32_t)((uint64_t)row >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

int64_t orc_hadamard_order(int64_t n) {
  int64_t N = 1;
  while (N < n) N *= 2;
  return N;
}

double orc_sketch_sign(uint64_t seed, int64_t j) {
  uint32_t o[4];
  orc_philox_row(seed, 3u, j, o);
  return (o[0] & 1u) ? -1.0 : 1.0;
}

int32_t orc_sketch_bucket(uint64_t seed, int64_t j, int32_t s) {
  uint32_t o[4];
  orc_philox_row(seed, 3u, j, o);
  return (int32_t)(((uint64_t)o[1] * (uint64_t)s) >> 32);
}

int64_t orc_srht_column(uint64_t seed, int64_t t, int64_t N) {
  uint32_t o[4];
  orc_philox_row(seed, 4u, t, o);
  return (int64_t)((uint64_t)o[0] % (uint64_t)N);
}

void orc_sketch_matrix(int32_t kind, uint64_t seed, int64_t n, int32_t s, double *Pi) {
  double scale = 1.0 / sqrt((double)s);
  if (kind == 0) {
    for (int64_t i = 0; i < n; ++i)
      for (int32_t c = 0; c < s; ++c) Pi[i * s + c] = scale * orc_probe_value(seed, 1, 2u, i, c);
  } else if (kind == 1) {
    int64_t N = orc_hadamard_order(n);
    int64_t *col = (int64_t *)malloc(sizeof(int64_t) * s);
    for (int32_t c = 0; c < s; ++c) col[c] = orc_srht_column(seed, c, N);
    for (int64_t j = 0; j < n; ++j) {
      double d = orc_sketch_sign(seed, j);
      for (int32_t c = 0; c < s; ++c) {
        int par = __builtin_popcountll((unsigned long long)(j & col[c])) & 1;
        Pi[j * s + c] = d * (par ? -1.0 : 1.0) * scale;
      }
    }
    free(col);
  } else {
    for (int64_t j = 0; j < n; ++j) {
      for (int32_t c = 0; c < s; ++c) Pi[j * s + c] = 0.0;
      Pi[j * s + orc_sketch_bucket(seed, j, s)] = orc_sketch_sign(seed, j);
    }
  }
}

double orc_rp_entropy_kind(const orc_matrix *R, int32_t kind, int32_t s, int32_t k,
                           uint64_t seed, double *sigma_out) {
  int64_t n = R->n;
  double *Pi = (double *)malloc(sizeof(double) * n * s);
  orc_sketch_matrix(kind, seed, n, s, Pi);
  double h = orc_rp_entropy_with_pi(R, Pi, s, k, sigma_out);
  free(Pi);
  return h;
}

double orc_rp_entropy(const orc_matrix *R, int32_t s, int32_t k, uint64_t seed,
                      double *sigma_out) {
  return orc_rp_entropy_kind(R, 0, s, k, seed, sigma_out);
}

/* ------------------------------------------------------------------------- */
/* Small MLP 16 -> 64 -> 64 -> 2 (ReLU, mean-squared error), FP64.           */
/* Parameter vector layout: W1[64][16], b1[64], W2[64][64], b2[64],          */
/* W3[2][64], b3[2]  (5378 values).                                          */
/* ------------------------------------------------------------------------- */
#define MLP_IN 16
#define MLP_H 64
#define MLP_OUT 2
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT)

int32_t orc_mlp_nparams(void) { return MLP_NPARAM; }

void orc_mlp_forward(const double *P, int32_t B, const double *X, double *Y) {
  const double *W1 = P, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H,
               *b2 = W2 + MLP_H * MLP_H, *W3 = b2 + MLP_H, *b3 = W3 + MLP_OUT * MLP_H;
  double h1[MLP_H], h2[MLP_H];
  for (int32_t r = 0; r < B; ++r) {
    const double *x = X + (int64_t)r * MLP_IN;
    for (int o = 0; o < MLP_H; ++o) {
      double a = b1[o];
      for (int i = 0; i < MLP_IN; ++i) a += W1[o * MLP_IN + i] * x[i];
      h1[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
      double a = b2[o];
      for (int i = 0; i < MLP_H; ++i) a += W2[o * MLP_H + i] * h1[i];
      h2[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
      double a = b3[o];
      for (int i = 0; i < MLP_H; ++i) a += W3[o * MLP_H + i] * h2[i];
      Y[(int64_t)r * MLP_OUT + o] = a;
    }
  }
}

/* Loss L = (1/B) sum_r sum_o (y_ro - t_ro)^2 ; returns L and fills grad. */
double orc_mlp_loss_grad(const double *P, int32_t B, const double *X,
                         const double *T, double *grad) {
  const double *W1 = P, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H,
               *b2 = W2 + MLP_H * MLP_H, *W3 = b2 + MLP_H, *b3 = W3 + MLP_OUT * MLP_H;
  double *gW1 = grad, *gb1 = gW1 + MLP_H * MLP_IN, *gW2 = gb1 + MLP_H,
         *gb2 = gW2 + MLP_H * MLP_H, *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_OUT * MLP_H;
  memset(grad, 0, sizeof(double) * MLP_NPARAM);
  double loss = 0.0;
  double a1[MLP_H], h1[MLP_H], a2[MLP_H], h2[MLP_H], y[MLP_OUT];
  double dy[MLP_OUT], dh2[MLP_H], da2[MLP_H], dh1[MLP_H], da1[MLP_H];
  for (int32_t r = 0; r < B; ++r) {
    const double *x = X + (int64_t)r * MLP_IN;
    for (int o = 0; o < MLP_H; ++o) {
      double a = b1[o];
      for (int i = 0; i < MLP_IN; ++i) a += W1[o * MLP_IN + i] * x[i];
      a1[o] = a;
      h1[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
      double a = b2[o];
      for (int i = 0; i < MLP_H; ++i) a += W2[o * MLP_H + i] * h1[i];
      a2[o] = a;
      h2[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
      double a = b3[o];
      for (int i = 0; i < MLP_H; ++i) a += W3[o * MLP_H + i] * h2[i];
      y[o] = a;
      double d = a - T[(int64_t)r * MLP_OUT + o];
      loss += d * d;
      dy[o] = 2.0 * d / (double)B;
    }
    for (int i = 0; i < MLP_H; ++i) dh2[i] = 0.0;
    for (int o = 0; o < MLP_OUT; ++o) {
      gb3[o] += dy[o];
      for (int i = 0; i < MLP_H; ++i) {
        gW3[o * MLP_H + i] += dy[o] * h2[i];
        dh2[i] += W3[o * MLP_H + i] * dy[o];
      }
    }
    for (int o = 0; o < MLP_H; ++o) da2[o] = a2[o] > 0.0 ? dh2[o] : 0.0;
    for (int i = 0; i < MLP_H; ++i) dh1[i] = 0.0;
    for (int o = 0; o < MLP_H; ++o) {
      gb2[o] += da2[o];
      for (int i = 0; i < MLP_H; ++i) {
        gW2[o * MLP_H + i] += da2[o] * h1[i];
        dh1[i] += W2[o * MLP_H + i] * da2[o];
      }
    }
    for (int o = 0; o < MLP_H; ++o) da1[o] = a1[o] > 0.0 ? dh1[o] : 0.0;
    for (int o = 0; o < MLP_H; ++o) {
      gb1[o] += da1[o];
      for (int i = 0; i < MLP_IN; ++i) gW1[o * MLP_IN + i] += da1[o] * x[i];
    }
  }
  return loss / (double)B;
}

/* Threads the parallel probe loop may use (reported with CPU timings). */
int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
