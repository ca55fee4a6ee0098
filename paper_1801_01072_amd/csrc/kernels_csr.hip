// kernels_csr.hip -- one step of the polynomial recurrence for sparse (CSR)
// R, bandwidth bound: Y = a * (R V_k), Z = c1*Y + c2*b*V_k + cw*V_{k-1},
// per-probe dots with g (same algebra as the dense step).
//
// Mapping: lane = probe (64 probes per wave, one 64-probe chunk per grid
// column), so every V row access is one coalesced 256 B (FP32) or 512 B
// (FP64) transaction.  A workgroup owns a contiguous range of rows and its
// waves take interleaved rows of it, so at any time they gather from the same
// few dozen V_k rows of a banded R, which stay in the CU's vector L1.  The
// row's column indices and values are wave-uniform and come through the
// scalar cache, kCsrUnroll at a time, and the V_k gathers of such a group are
// independent of each other, so a wave keeps that many loads in flight.
// Per-probe dot partials stay in registers until the end (one partial per
// block per probe: deterministic, fixed order).
// Rademacher probes are read as packed sign bits; when V_k or V_{k-1} is the
// probe block itself it is expanded from those bits instead of stored.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

template <typename T>
__device__ __forceinline__ T sign_of(const uint32_t *__restrict__ signs, int64_t row, int32_t nw,
                                     int32_t probe) {
  const uint32_t wd = signs[row * nw + (probe >> 5)];
  return ((wd >> (probe & 31)) & 1u) ? T(-1) : T(1);
}

// The CSR arrays are read through the constant address space: nothing
// writes them while the kernel runs, and their wave-uniform loads (row
// offsets, a group's columns and values) then go through the scalar cache as
// wide scalar loads.
template <typename T>
using ConstPtr = __attribute__((address_space(4))) const T *;

namespace {
constexpr int kCsrWaves = 8;        // waves per workgroup
constexpr int kCsrBlocksPerCU = 2;  // resident workgroups per CU (256 CUs)
constexpr int kCsrUnroll = 8;       // independent V_k gathers in flight per wave
}  // namespace

template <typename T, bool VK_SIGNS, bool VM1_SIGNS>
__global__ __launch_bounds__(64 * kCsrWaves) void csr_step_kernel(CsrStepArgs a) {
  __shared__ double red[2][kCsrWaves][64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = a.n, ldv = a.ldv;
  const int32_t nw = (int32_t)(ldv >> 5);
  const int32_t probe = (int32_t)blockIdx.y * 64 + lane;
  const ConstPtr<int64_t> rp = (ConstPtr<int64_t>)a.row_ptr;
  const ConstPtr<int32_t> ci = (ConstPtr<int32_t>)a.col_idx;
  const ConstPtr<T> vals = (ConstPtr<T>)a.values;
  auto val = [&](int64_t e) -> T { return vals[e]; };
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  // V_{k+1} is written over V_{k-1} element by element by the thread that
  // read it, so these two may alias each other (and nothing else)
  const T *Vkm1 = (const T *)a.Vkm1;
  T *Vkp1 = (T *)a.Vkp1;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const bool use_m1 = a.cw != 0.0;
  const bool want_gg = a.slot_gg >= 0;

  auto xglob = [&](int64_t r) -> T {
    if (VK_SIGNS) return sign_of<T>(signs, r, nw, probe);
    return Vk[r * ldv + probe];
  };

  // contiguous row range per block, a multiple of the wave count
  const int64_t per0 = (n + gridDim.x - 1) / gridDim.x;
  const int64_t per = (per0 + kCsrWaves - 1) / kCsrWaves * kCsrWaves;
  const int64_t r_beg = (int64_t)blockIdx.x * per;
  const int64_t r_end = r_beg + per < n ? r_beg + per : n;
  double ds = 0.0, gs = 0.0;
  for (int64_t r = r_beg + w; r < r_end; r += kCsrWaves) {
    // epilogue operands first: independent of the gathers
    const T xr = xglob(r);
    T vm = T(0);
    if (use_m1) vm = VM1_SIGNS ? sign_of<T>(signs, r, nw, probe) : Vkm1[r * ldv + probe];
    const T gv = signs ? sign_of<T>(signs, r, nw, probe) : G[r * ldv + probe];
    const int64_t e0 = rp[r], e1 = rp[r + 1];
    T acc0 = T(0), acc1 = T(0);
    // groups of kCsrUnroll entries: one scalar load of their columns and
    // values, then kCsrUnroll independent V_k gathers
    int64_t e = e0;
    for (; e + kCsrUnroll <= e1; e += kCsrUnroll) {
      T x[kCsrUnroll];
#pragma unroll
      for (int q = 0; q < kCsrUnroll; ++q) x[q] = xglob(ci[e + q]);
#pragma unroll
      for (int q = 0; q < kCsrUnroll; q += 2) {
        acc0 += val(e + q) * x[q];
        acc1 += val(e + q + 1) * x[q + 1];
      }
    }
    if (e + 4 <= e1) {
      T x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = xglob(ci[e + q]);
      acc0 += val(e) * x[0];
      acc1 += val(e + 1) * x[1];
      acc0 += val(e + 2) * x[2];
      acc1 += val(e + 3) * x[3];
      e += 4;
    }
    for (; e < e1; ++e) acc0 += val(e) * xglob(ci[e]);
    const T y = ta * (acc0 + acc1);
    T z = tc1 * y + tb * xr;
    if (use_m1) z += tcw * vm;
    if (Vkp1) Vkp1[r * ldv + probe] = z;
    ds += (double)gv * (double)(a.dot_y ? y : z);
    if (want_gg) gs += (double)gv * (double)gv;
  }
  red[0][w][lane] = ds;
  red[1][w][lane] = gs;
  __syncthreads();
  if (w == 0) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int q = 0; q < kCsrWaves; ++q) {
      t0 += red[0][q][lane];
      t1 += red[1][q][lane];
    }
    const int64_t base = (int64_t)blockIdx.x * ldv + probe;
    a.part[(int64_t)a.slot * a.nblk * ldv + base] = t0;
    if (want_gg) a.part[(int64_t)a.slot_gg * a.nblk * ldv + base] = t1;
  }
}

// Persistent grid: kCsrBlocksPerCU workgroups per CU, fewer for small n.
int32_t csr_step_blocks(int64_t n) {
  const int64_t groups = (n + kCsrWaves - 1) / kCsrWaves;
  const int64_t cap = 256 * kCsrBlocksPerCU;
  return (int32_t)(groups < cap ? groups : cap);
}

template <typename T>
hipError_t launch_csr_step(const CsrStepArgs &a, hipStream_t st) {
  dim3 grid((unsigned)a.nblk, (unsigned)(a.ldv / 64));
  const bool vk_signs = a.Vk == nullptr;
  const bool vm1_signs = a.Vkm1 == nullptr && a.cw != 0.0;
  if ((vk_signs || vm1_signs) && !a.signs) return hipErrorInvalidValue;
  if (vk_signs)
    csr_step_kernel<T, true, false><<<grid, 64 * kCsrWaves, 0, st>>>(a);
  else if (vm1_signs)
    csr_step_kernel<T, false, true><<<grid, 64 * kCsrWaves, 0, st>>>(a);
  else
    csr_step_kernel<T, false, false><<<grid, 64 * kCsrWaves, 0, st>>>(a);
  return hipGetLastError();
}
template hipError_t launch_csr_step<double>(const CsrStepArgs &, hipStream_t);
template hipError_t launch_csr_step<float>(const CsrStepArgs &, hipStream_t);

}  // namespace ent
