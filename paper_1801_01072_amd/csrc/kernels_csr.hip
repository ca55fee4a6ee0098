// kernels_csr.hip -- one step of the polynomial recurrence for sparse (CSR)
// R, bandwidth bound: Y = a * (R V_k), Z = c1*Y + c2*b*V_k + cw*V_{k-1},
// per-probe dots with g (same algebra as the dense step).
//
// Mapping: lane = probe (64 probes per wave, one 64-probe chunk per grid
// column), so every V row access is one coalesced 256 B (FP32) or 512 B
// (FP64) transaction.  Workgroups are persistent: block b handles a
// contiguous run of 64-row slabs.  For each slab the block first stages, in one burst of
// independent loads, the slab's (column, value) entries and the window of
// V_k rows its columns span (about 96 rows for a banded R) into LDS; each of
// the four waves then computes 16 rows from LDS only, so HBM sees each V_k
// row about once and no load latency sits inside the row loop.  A slab whose
// entries or column span exceed the LDS capacity is computed with direct
// gathers instead (entries broadcast from lanes with readlane), so any CSR
// matrix is accepted.  Per-probe dot partials stay in registers until the end
// (one partial per block per probe: deterministic, fixed order).
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

// LDS capacities per slab: window rows of V_k (64 probes each) and entries.
template <typename T>
struct CsrCaps;
template <>
struct CsrCaps<float> {
  static constexpr int WROWS = 128, ECAP = 2560;
};
template <>
struct CsrCaps<double> {
  static constexpr int WROWS = 96, ECAP = 2304;
};

template <typename T, bool VK_SIGNS, bool VM1_SIGNS>
__global__ __launch_bounds__(256) void csr_step_kernel(CsrStepArgs a) {
  constexpr int WROWS = CsrCaps<T>::WROWS, ECAP = CsrCaps<T>::ECAP;
  __shared__ T win[WROWS * 64];
  __shared__ int32_t s_col[ECAP];
  __shared__ T s_val[ECAP];
  __shared__ int64_t s_rp[65];
  __shared__ int32_t s_min[4], s_max[4];
  __shared__ double red[2][4][64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n = a.n, ldv = a.ldv;
  const int32_t nw = (int32_t)(ldv >> 5);
  const int32_t chunk0 = (int32_t)blockIdx.y * 64;
  const int32_t probe = chunk0 + lane;
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

  auto xglob = [&](int64_t r, int32_t pr) -> T {
    if (VK_SIGNS) return sign_of<T>(signs, r, nw, pr);
    return Vk[r * ldv + pr];
  };

  // contiguous run of slabs per block: neighbouring slabs share V_k rows,
  // which then come from this CU's caches
  const int64_t nslab = (n + 63) / 64;
  const int64_t per = (nslab + gridDim.x - 1) / gridDim.x;
  const int64_t s_beg = (int64_t)blockIdx.x * per;
  const int64_t s_end = s_beg + per < nslab ? s_beg + per : nslab;
  double ds = 0.0, gs = 0.0;
  for (int64_t slab = s_beg; slab < s_end; ++slab) {
    const int64_t r_lo = slab * 64;
    const int nr = (int)((n - r_lo) < 64 ? (n - r_lo) : 64);
    if (tid <= nr) s_rp[tid] = rp[r_lo + tid];
    __syncthreads();
    const int64_t e_lo = s_rp[0];
    const int64_t ne = s_rp[nr] - e_lo;
    const bool stage_e = ne <= ECAP;
    // column range of the slab (its own rows included: the epilogue reads V_k[r])
    int32_t cmin = (int32_t)r_lo, cmax = (int32_t)(r_lo + nr - 1);
    if (stage_e) {
      for (int64_t e = tid; e < ne; e += 256) {
        const int32_t c = ci[e_lo + e];
        s_col[e] = c;
        s_val[e] = val[e_lo + e];
        cmin = c < cmin ? c : cmin;
        cmax = c > cmax ? c : cmax;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int32_t o1 = __shfl_xor(cmin, off, 64), o2 = __shfl_xor(cmax, off, 64);
      cmin = o1 < cmin ? o1 : cmin;
      cmax = o2 > cmax ? o2 : cmax;
    }
    if (lane == 0) {
      s_min[w] = cmin;
      s_max[w] = cmax;
    }
    __syncthreads();
    cmin = s_min[0];
    cmax = s_max[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      cmin = s_min[i] < cmin ? s_min[i] : cmin;
      cmax = s_max[i] > cmax ? s_max[i] : cmax;
    }
    const bool stage_w = stage_e && (cmax - cmin + 1) <= WROWS;
    if (stage_w) {
      const int wn = (cmax - cmin + 1) * 64;
      for (int idx = tid; idx < wn; idx += 256) {
        const int64_t c = cmin + idx / 64;
        win[idx] = xglob(c, chunk0 + (idx & 63));
      }
    }
    __syncthreads();
    // each wave: 16 consecutive rows of the slab
    for (int rr = 0; rr < 16; ++rr) {
      const int rl = 16 * w + rr;
      if (rl >= nr) break;
      const int64_t r = r_lo + rl;
      T acc = T(0);
      if (stage_w) {
        const int64_t eb = s_rp[rl] - e_lo, ee = s_rp[rl + 1] - e_lo;
        int64_t e = eb;
        for (; e + 4 <= ee; e += 4) {
          const T x0 = win[(s_col[e] - cmin) * 64 + lane];
          const T x1 = win[(s_col[e + 1] - cmin) * 64 + lane];
          const T x2 = win[(s_col[e + 2] - cmin) * 64 + lane];
          const T x3 = win[(s_col[e + 3] - cmin) * 64 + lane];
          acc += s_val[e] * x0;
          acc += s_val[e + 1] * x1;
          acc += s_val[e + 2] * x2;
          acc += s_val[e + 3] * x3;
        }
        for (; e < ee; ++e) acc += s_val[e] * win[(s_col[e] - cmin) * 64 + lane];
      } else {
        // slab too wide for LDS: entries broadcast from lanes, V_k gathered
        const int64_t e0 = rp[r], e1 = rp[r + 1];
        for (int64_t base = e0; base < e1; base += 64) {
          const int cnt = (int)((e1 - base) < 64 ? (e1 - base) : 64);
          int mc = 0;
          T mv = T(0);
          if (lane < cnt) {
            mc = ci[base + lane];
            mv = val[base + lane];
          }
          for (int q = 0; q < cnt; ++q) {
            const int c0 = __builtin_amdgcn_readlane(mc, q);
            acc += readlane_t(mv, q) * xglob(c0, probe);
          }
        }
      }
      const int64_t off = r * ldv + probe;
      const T xr = stage_w ? win[(r - cmin) * 64 + lane] : xglob(r, probe);
      const T y = ta * acc;
      T z = tc1 * y + tb * xr;
      if (use_m1) z += tcw * (VM1_SIGNS ? sign_of<T>(signs, r, nw, probe) : Vkm1[off]);
      if (Vkp1) Vkp1[off] = z;
      const T g = signs ? sign_of<T>(signs, r, nw, probe) : G[off];
      ds += (double)g * (double)(a.dot_y ? y : z);
      if (want_gg) gs += (double)g * (double)g;
    }
    __syncthreads();
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

// Two workgroups per CU fit in LDS (FP32); the grid is that resident size.
int32_t csr_step_blocks(int64_t n) {
  const int64_t slabs = (n + 63) / 64;
  const int64_t cap = 256 * 2;
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
