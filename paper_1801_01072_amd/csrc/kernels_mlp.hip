// kernels_mlp.hip -- the learned degree / lower-cutoff selector: a 16-64-64-2
// ReLU MLP in FP32 (inference, fused forward + backward for training, Adam),
// and the kernel that turns a cheap sketch (power method + a short Chebyshev
// moment pass) into its 16 input features.
//
// Parameter vector (5378 floats): W1[64][16], b1[64], W2[64][64], b2[64],
// W3[2][64], b3[2].  Loss: L = (1/B) sum_r sum_o (y_ro - t_ro)^2.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

namespace {
constexpr int MI = 16, MH = 64, MO = 2;
constexpr int OW1 = 0, OB1 = OW1 + MH * MI, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH,
              OB3 = OW3 + MO * MH, NPAR = OB3 + MO;
constexpr int SPB = 32;  // samples per workgroup
}  // namespace

// Forward (and optionally backward) over SPB samples per workgroup.  With
// grads: gpart[block][p] = sum over the block's samples of dL/dP_p, and
// lpart[block] = sum of squared errors (both in fixed order).
__global__ __launch_bounds__(256) void mlp_block_kernel(const float *__restrict__ P,
                                                        const float *__restrict__ X,
                                                        const float *__restrict__ T, int32_t B,
                                                        float *__restrict__ Y,
                                                        float *__restrict__ gpart,
                                                        double *__restrict__ lpart) {
  __shared__ float sx[SPB][MI];
  __shared__ float h1[SPB][MH], h2[SPB][MH], d1[SPB][MH], d2[SPB][MH];
  __shared__ float dy[SPB][MO];
  __shared__ double sl[4];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * SPB;
  const int ns = (int)((B - s0) < SPB ? (B - s0) : SPB);
  const bool train = gpart != nullptr;
  for (int e = tid; e < SPB * MI; e += 256) {
    const int s = e / MI, i = e % MI;
    sx[s][i] = s < ns ? X[(s0 + s) * MI + i] : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < SPB * MH; e += 256) {
    const int s = e / MH, o = e % MH;
    float a = P[OB1 + o];
    for (int i = 0; i < MI; ++i) a += P[OW1 + o * MI + i] * sx[s][i];
    h1[s][o] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < SPB * MH; e += 256) {
    const int s = e / MH, o = e % MH;
    float a = P[OB2 + o];
    for (int i = 0; i < MH; ++i) a += P[OW2 + o * MH + i] * h1[s][i];
    h2[s][o] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  double loss = 0.0;
  if (tid < SPB * MO) {
    const int s = tid / MO, o = tid % MO;
    float a = P[OB3 + o];
    for (int i = 0; i < MH; ++i) a += P[OW3 + o * MH + i] * h2[s][i];
    if (s < ns) {
      if (Y) Y[(s0 + s) * MO + o] = a;
      if (train) {
        const float dv = a - T[(s0 + s) * MO + o];
        loss = (double)dv * (double)dv;
        dy[s][o] = 2.f * dv / (float)B;
      }
    } else if (train) {
      dy[s][o] = 0.f;
    }
  }
  if (!train) return;
  loss = wave_sum(loss);
  if ((tid & 63) == 0) sl[tid >> 6] = loss;
  __syncthreads();
  if (tid == 0) lpart[blockIdx.x] = sl[0] + sl[1] + sl[2] + sl[3];
  // backward through layer 3 and the second ReLU
  for (int e = tid; e < SPB * MH; e += 256) {
    const int s = e / MH, i = e % MH;
    float a = 0.f;
    for (int o = 0; o < MO; ++o) a += P[OW3 + o * MH + i] * dy[s][o];
    d2[s][i] = h2[s][i] > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < SPB * MH; e += 256) {
    const int s = e / MH, i = e % MH;
    float a = 0.f;
    for (int o = 0; o < MH; ++o) a += P[OW2 + o * MH + i] * d2[s][o];
    d1[s][i] = h1[s][i] > 0.f ? a : 0.f;
  }
  __syncthreads();
  float *g = gpart + (int64_t)blockIdx.x * NPAR;
  for (int p = tid; p < NPAR; p += 256) {
    float a = 0.f;
    if (p < OB1) {
      const int o = p / MI, i = p % MI;
      for (int s = 0; s < SPB; ++s) a += d1[s][o] * sx[s][i];
    } else if (p < OW2) {
      const int o = p - OB1;
      for (int s = 0; s < SPB; ++s) a += d1[s][o];
    } else if (p < OB2) {
      const int q = p - OW2, o = q / MH, i = q % MH;
      for (int s = 0; s < SPB; ++s) a += d2[s][o] * h1[s][i];
    } else if (p < OW3) {
      const int o = p - OB2;
      for (int s = 0; s < SPB; ++s) a += d2[s][o];
    } else if (p < OB3) {
      const int q = p - OW3, o = q / MH, i = q % MH;
      for (int s = 0; s < SPB; ++s) a += dy[s][o] * h2[s][i];
    } else {
      const int o = p - OB3;
      for (int s = 0; s < SPB; ++s) a += dy[s][o];
    }
    g[p] = a;
  }
}

// grad[p] = sum_b gpart[b][p]; loss = sum_b lpart[b] / B (fixed order).
__global__ void mlp_grad_reduce_kernel(const float *__restrict__ gpart, const double *__restrict__ lpart,
                                       int32_t nblk, int32_t B, float *__restrict__ grad,
                                       double *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPAR) {
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += gpart[(int64_t)b * NPAR + p];
    grad[p] = a;
  }
  if (p == 0 && loss) {
    double l = 0.0;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    *loss = l / (double)B;
  }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// P -= lr * mhat / (sqrt(vhat) + eps), bias-corrected by step t (>= 1).
__global__ void adam_kernel(float *__restrict__ P, const float *__restrict__ grad,
                            float *__restrict__ m, float *__restrict__ v, int32_t t, float lr,
                            float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  const float g = grad[p];
  const float mi = b1 * m[p] + (1.f - b1) * g;
  const float vi = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.f - powf(b1, (float)t));
  const float vh = vi / (1.f - powf(b2, (float)t));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

int32_t mlp_nparams() { return NPAR; }
int32_t mlp_blocks(int32_t B) { return (B + SPB - 1) / SPB; }

hipError_t launch_mlp_forward(const float *P, const float *X, int32_t B, float *Y, hipStream_t st) {
  mlp_block_kernel<<<(unsigned)mlp_blocks(B), 256, 0, st>>>(P, X, nullptr, B, Y, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const float *X, const float *T, int32_t B, float *gpart,
                           double *lpart, float *grad, double *loss, hipStream_t st) {
  const int32_t nb = mlp_blocks(B);
  mlp_block_kernel<<<(unsigned)nb, 256, 0, st>>>(P, X, T, B, nullptr, gpart, lpart);
  mlp_grad_reduce_kernel<<<(unsigned)((NPAR + 255) / 256), 256, 0, st>>>(gpart, lpart, nb, B, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float *P, const float *grad, float *m, float *v, int32_t t, float lr,
                       hipStream_t st) {
  adam_kernel<<<(unsigned)((NPAR + 255) / 256), 256, 0, st>>>(P, grad, m, v, t, lr, 0.9f, 0.999f, 1e-8f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Features of one matrix from its sketch pass (power method + Chebyshev
// moments d[k][j], k = 0..mf, on [0, u], sf Rademacher probes):
//   f0 = ln n / 10, f1 = ln(n p~1) / 10, f2 = ln u / 10,
//   f3..f14 = mu_1..mu_12, mu_k = (1/sf) sum_j d_kj / d_0j,
//   f15 = H^_mf / ln n, the degree-mf Chebyshev estimate from the same moments.
// ---------------------------------------------------------------------------
__global__ void selector_features_kernel(const double *__restrict__ scal, const double *__restrict__ d,
                                         int32_t mf, int32_t sf, int64_t n, float *__restrict__ feat) {
  if (threadIdx.x != 0) return;
  const double ln_n = log((double)n);
  feat[0] = (float)(ln_n / 10.0);
  feat[1] = (float)(log((double)n * scal[S_P1]) / 10.0);
  feat[2] = (float)(log(scal[S_U]) / 10.0);
  double h = 0.0;
  for (int k = 0; k <= mf; ++k) {
    double mu = 0.0, raw = 0.0;
    for (int j = 0; j < sf; ++j) {
      mu += d[(int64_t)k * sf + j] / d[j];
      raw += d[(int64_t)k * sf + j];
    }
    mu /= (double)sf;
    if (k >= 1 && k <= 12) feat[2 + k] = (float)mu;
    h -= scal[S_ALPHA + k] * raw / (double)sf;
  }
  feat[15] = (float)(h / (ln_n > 0.0 ? ln_n : 1.0));
}

hipError_t launch_selector_features(const double *scal, const double *d, int32_t mf, int32_t sf,
                                    int64_t n, float *feat, hipStream_t st) {
  selector_features_kernel<<<1, 64, 0, st>>>(scal, d, mf, sf, n, feat);
  return hipGetLastError();
}

}  // namespace ent
