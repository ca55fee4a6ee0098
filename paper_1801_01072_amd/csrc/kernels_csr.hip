// kernels_csr.hip -- one step of the polynomial recurrence for sparse (CSR)
// R, bandwidth bound: Y = a * (R V_k), Z = c1*Y + c2*b*V_k + cw*V_{k-1},
// per-probe dots with g (same algebra as the dense step).
//
// Mapping: one wave per row, lane = probe (64 probes per wave, one 64-probe
// chunk per grid column), so every V row access is one coalesced 256 B (FP32)
// or 512 B (FP64) transaction.  The row's (column, value) pairs are fetched
// once per wave into lanes and broadcast with readlane.  Workgroups are
// persistent: block b handles 64-row slabs b, b + G, ...; its four waves take
// 16 consecutive rows each, so the V rows of a banded R are reused from
// cache.  Per-probe dot partials stay in registers until the end (one
// partial per block per probe: deterministic, fixed order).
// Rademacher probes are read as packed sign bits; when V_k or V_{k-1} is the
// probe block itself it is expanded from those bits instead of stored.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int q);

template <>
__device__ __forceinline__ float readlane_t<float>(float v, int q) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
}
template <>
__device__ __forceinline__ double readlane_t<double>(double v, int q) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), q);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), q);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ __forceinline__ T sign_of(const uint32_t *__restrict__ signs, int64_t row, int32_t nw,
                                     int32_t probe) {
  const uint32_t wd = signs[row * nw + (probe >> 5)];
  return ((wd >> (probe & 31)) & 1u) ? T(-1) : T(1);
}

template <typename T, bool VK_SIGNS, bool VM1_SIGNS>
__global__ __launch_bounds__(256) void csr_step_kernel(CsrStepArgs a) {
  __shared__ double red[2][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = a.n, ldv = a.ldv;
  const int32_t nw = (int32_t)(ldv >> 5);
  const int32_t probe = (int32_t)blockIdx.y * 64 + lane;
  const int64_t *__restrict__ rp = a.row_ptr;
  const int32_t *__restrict__ ci = a.col_idx;
  const T *__restrict__ val = (const T *)a.values;
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *Vkm1 = (const T *)a.Vkm1;
  T *Vkp1 = (T *)a.Vkp1;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const bool use_m1 = a.cw != 0.0;
  const bool want_gg = a.slot_gg >= 0;

  auto xval = [&](int64_t r) -> T {
    if (VK_SIGNS) return sign_of<T>(signs, r, nw, probe);
    return Vk[r * ldv + probe];
  };

  double ds = 0.0, gs = 0.0;
  for (int64_t slab = blockIdx.x; slab * 64 < n; slab += gridDim.x) {
    const int64_t r_lo = slab * 64 + 16 * w;
    for (int rr = 0; rr < 16; ++rr) {
      const int64_t r = r_lo + rr;
      if (r >= n) break;
      const int64_t e0 = rp[r], e1 = rp[r + 1];
      T acc = T(0);
      for (int64_t base = e0; base < e1; base += 64) {
        const int cnt = (int)((e1 - base) < 64 ? (e1 - base) : 64);
        int mc = 0;
        T mv = T(0);
        if (lane < cnt) {
          mc = ci[base + lane];
          mv = val[base + lane];
        }
        int q = 0;
        for (; q + 4 <= cnt; q += 4) {
          const int c0 = __builtin_amdgcn_readlane(mc, q);
          const int c1 = __builtin_amdgcn_readlane(mc, q + 1);
          const int c2 = __builtin_amdgcn_readlane(mc, q + 2);
          const int c3 = __builtin_amdgcn_readlane(mc, q + 3);
          const T x0 = xval(c0), x1 = xval(c1), x2 = xval(c2), x3 = xval(c3);
          acc += readlane_t(mv, q) * x0;
          acc += readlane_t(mv, q + 1) * x1;
          acc += readlane_t(mv, q + 2) * x2;
          acc += readlane_t(mv, q + 3) * x3;
        }
        for (; q < cnt; ++q) {
          const int c0 = __builtin_amdgcn_readlane(mc, q);
          acc += readlane_t(mv, q) * xval(c0);
        }
      }
      const int64_t off = r * ldv + probe;
      const T y = ta * acc;
      T z = tc1 * y + tb * xval(r);
      if (use_m1) z += tcw * (VM1_SIGNS ? sign_of<T>(signs, r, nw, probe) : Vkm1[off]);
      if (Vkp1) Vkp1[off] = z;
      const T g = signs ? sign_of<T>(signs, r, nw, probe) : G[off];
      ds += (double)g * (double)(a.dot_y ? y : z);
      if (want_gg) gs += (double)g * (double)g;
    }
  }
  red[0][w][lane] = ds;
  red[1][w][lane] = gs;
  __syncthreads();
  if (w == 0) {
    const int64_t base = (int64_t)blockIdx.x * ldv + probe;
    a.part[(int64_t)a.slot * a.nblk * ldv + base] =
        red[0][0][lane] + red[0][1][lane] + red[0][2][lane] + red[0][3][lane];
    if (want_gg)
      a.part[(int64_t)a.slot_gg * a.nblk * ldv + base] =
          red[1][0][lane] + red[1][1][lane] + red[1][2][lane] + red[1][3][lane];
  }
}

int32_t csr_step_blocks(int64_t n) {
  const int64_t slabs = (n + 63) / 64;
  const int64_t cap = 256 * 8;
  return (int32_t)(slabs < cap ? slabs : cap);
}

template <typename T>
hipError_t launch_csr_step(const CsrStepArgs &a, hipStream_t st) {
  dim3 grid((unsigned)a.nblk, (unsigned)(a.ldv / 64));
  const bool vk_signs = a.Vk == nullptr;
  const bool vm1_signs = a.Vkm1 == nullptr && a.cw != 0.0;
  if ((vk_signs || vm1_signs) && !a.signs) return hipErrorInvalidValue;
  if (vk_signs)
    csr_step_kernel<T, true, false><<<grid, 256, 0, st>>>(a);
  else if (vm1_signs)
    csr_step_kernel<T, false, true><<<grid, 256, 0, st>>>(a);
  else
    csr_step_kernel<T, false, false><<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}
template hipError_t launch_csr_step<double>(const CsrStepArgs &, hipStream_t);
template hipError_t launch_csr_step<float>(const CsrStepArgs &, hipStream_t);

}  // namespace ent
