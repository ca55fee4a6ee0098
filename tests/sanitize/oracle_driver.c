/*
 * Host sanitizer run of the oracle: every exported routine on small inputs
 * (dense FP64 / FP32, CSR, Hermitian, sketches, the MLP), built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
 * The oracle's source is included whole so that its private descriptors are
 * visible; nothing here checks values (the oracle's pins do that): only that
 * no access leaves its buffer and no undefined operation runs.
 */
#include "../../oracle/oracle.c"

#include <stdio.h>

#define N 9

static double A[N * N];
static float Af[N * N];

static void fill_density(void) {
  /* R = V diag(p) V^T with V a product of two Givens-like rotations: any
     symmetric PSD matrix of unit trace serves */
  double p[N], s = 0.0;
  for (int i = 0; i < N; ++i) s += (p[i] = 1.0 + i);
  for (int i = 0; i < N; ++i) p[i] /= s;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double v = 0.0;
      for (int k = 0; k < N; ++k) {
        const double qi = cos(0.3 * (i + 1) * (k + 1)), qj = cos(0.3 * (j + 1) * (k + 1));
        v += qi * p[k] * qj;
      }
      A[i * N + j] = v;
    }
  double tr = 0.0;
  for (int i = 0; i < N; ++i) tr += A[i * N + i];
  for (int i = 0; i < N * N; ++i) {
    A[i] /= tr;
    Af[i] = (float)A[i];
  }
}

int main(void) {
  fill_density();
  double g[N], alpha[64], per[8], d[(40 + 1) * 2], sig[N], eig[N], V[N * N];
  orc_result res;
  uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
  orc_philox4x32_10(ctr, key, out);
  for (int dist = 0; dist < 2; ++dist) orc_probe_vector(42, dist, 0, N, 3, g);

  const orc_matrix Rd = {N, 0, 0, N, A, NULL, NULL};
  const orc_matrix Rf = {N, 0, 1, N, Af, NULL, NULL};
  /* tridiagonal CSR copy of a Poisson-like density (rows 0 .. N-1) */
  int64_t rp[N + 1];
  int32_t ci[3 * N];
  double cv[3 * N];
  int64_t nnz = 0;
  for (int i = 0; i < N; ++i) {
    rp[i] = nnz;
    for (int j = i - 1; j <= i + 1; ++j)
      if (j >= 0 && j < N) {
        ci[nnz] = j;
        cv[nnz++] = (i == j ? 2.0 : -1.0) / (2.0 * N);
      }
  }
  rp[N] = nnz;
  const orc_matrix Rc = {N, 1, 0, 0, cv, rp, ci};

  const orc_matrix *mats[3] = {&Rd, &Rf, &Rc};
  for (int k = 0; k < 3; ++k) {
    const orc_matrix *R = mats[k];
    (void)orc_power_method(R, 5, 3, 7);
    for (int method = 0; method < 2; ++method) {
      if (orc_estimate(R, method, 12, 4, 11, 5, 2, 6.0, 0, 0.0, 0.0, NULL, 0, per, &res)) return 1;
      const int32_t sel[2] = {1, 3};
      if (orc_estimate(R, method, 12, 4, 11, 5, 2, 6.0, 1, method ? 1e-3 : 0.0, 0.9, sel, 2, per, &res))
        return 1;
    }
    orc_cheb_moments_forward(R, 0.0, 1.0, 40, g, d);
    orc_cheb_moments_forward(R, 1e-3, 1.0, 40, g, d + 41);
  }
  orc_cheb_coeffs(0.8, 40, alpha);
  orc_cheb_interp_coeffs(1e-3, 0.8, 40, orc_cutoff_nodes(40), alpha);
  (void)orc_cheb_eval_scalar(alpha, 40, 1e-3, 0.8, 0.25);

  /* Hermitian: R = A + i C with C skew-symmetric and small */
  static double Z[2 * N * N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      Z[2 * (i * N + j)] = A[i * N + j];
      Z[2 * (i * N + j) + 1] = i == j ? 0.0 : 0.01 * (i < j ? 1.0 : -1.0) / N;
    }
  const orc_zmatrix Rz = {N, 0, N, Z};
  (void)orc_zpower_method(&Rz, 5, 2, 3);
  for (int method = 0; method < 2; ++method)
    if (orc_zestimate(&Rz, method, 10, 3, 5, 5, 1, 6.0, 0, 0.0, 0.0, NULL, 0, per, &res)) return 1;
  orc_zcheb_moments_forward(&Rz, 0.0, 1.0, 40, g, d);

  if (orc_jacobi_eigen(N, A, eig, V, 1e-14, 60) < 0) return 1;
  (void)orc_entropy_from_eigs(N, eig);
  (void)orc_exact_entropy(&Rd);
  for (int kind = 0; kind < 3; ++kind) (void)orc_rp_entropy_kind(&Rd, kind, 4, 3, 9, sig);
  (void)orc_rp_entropy(&Rf, 5, 5, 9, sig);

  const int32_t B = 3, np = orc_mlp_nparams();
  double *P = (double *)calloc(np, sizeof(double)), *G = (double *)calloc(np, sizeof(double));
  double X[3 * MLP_IN], Y[3 * MLP_OUT], T[3 * MLP_OUT];
  for (int i = 0; i < np; ++i) P[i] = 0.01 * cos(0.1 * i);
  for (int i = 0; i < 3 * MLP_IN; ++i) X[i] = sin(0.2 * i);
  for (int i = 0; i < 3 * MLP_OUT; ++i) T[i] = 0.5;
  orc_mlp_forward(P, B, X, Y);
  (void)orc_mlp_loss_grad(P, B, X, T, G);
  free(P);
  free(G);
  printf("oracle sanitizer run: ok\n");
  return 0;
}
