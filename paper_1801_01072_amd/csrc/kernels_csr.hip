// kernels_csr.hip -- one step of the polynomial recurrence for sparse (CSR)
// R, bandwidth bound: Y = a * (R V_k), Z = c1*Y + c2*b*V_k + cw*V_{k-1},
// per-probe dots with g (same algebra as the dense step).
//
// Mapping: a row is handled by a group of L lanes, each owning P probes of a
// 64-probe chunk (P = 8, L = 8 in FP32; P = 4, L = 16 in FP64: 32 bytes per
// lane) as two 16-byte pieces, one in each half of the row's segment: lane o
// holds bytes [16 o, 16 o + 16) of both halves.  A wave works on 64 / L rows
// at once, every V row access is one contiguous 256 B (FP32) or 512 B (FP64)
// segment per row, and each 16-byte access of a group covers one half of its
// row without gaps, so the group's LDS reads do not collide on banks.
//
// A workgroup walks a contiguous range of row chunks (CH = rows per wave x
// waves).  The V_k rows a chunk's columns span (its window, found once per
// estimate by csr_chunk_window_kernel) are copied into LDS by direct
// global-to-LDS loads, double buffered: the next chunk's window is in flight
// while the current chunk gathers from LDS, which has twice the bandwidth of
// the vector L1 that per-entry gathers from global memory would saturate.
// A chunk whose window is wider than the buffer gathers from global memory
// instead, so any CSR matrix is accepted.  The row's column indices and
// values are loaded once by the lanes of its group (one entry per lane) and
// passed to the group by lane shuffles; the results of a chunk are stored
// after the next chunk's barrier, so that barrier does not wait on them.
// Per-probe dot partials stay in registers until the end (one partial per
// block per probe: deterministic, fixed order).
// Rademacher probes are read as packed sign bits; when V_k or V_{k-1} is the
// probe block itself it is expanded from those bits instead of stored.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

namespace {
constexpr int kCsrWaves = 4;  // waves per workgroup
}  // namespace

template <typename T>
struct CsrLanes {
  static constexpr int P = 32 / (int)sizeof(T);    // probes per lane (32 bytes)
  static constexpr int L = 64 / P;                 // lanes per row
  static constexpr int RPW = 64 / L;               // rows per wave
  static constexpr int CH = RPW * kCsrWaves;       // rows per chunk
  static constexpr int ROWB = 64 * (int)sizeof(T); // bytes of one V row chunk
  static constexpr int VE = 16 / (int)sizeof(T);   // elements per 16-byte piece
  static constexpr int HALF = ROWB / 2;             // bytes of half a row chunk
  static constexpr int WROWS = 64;                 // window capacity in rows
  static constexpr int WBYTES = WROWS * ROWB;      // one window buffer
};

int32_t csr_chunk_rows(int32_t fp64) { return fp64 ? CsrLanes<double>::CH : CsrLanes<float>::CH; }

// Column window of every chunk of ch rows: win[c] = (min, max) over the
// chunk's column indices and its own rows.  One wave per chunk.
__global__ __launch_bounds__(256) void csr_chunk_window_kernel(const int64_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               int64_t n, int32_t ch,
                                                               int2 *__restrict__ win) {
  const int lane = threadIdx.x & 63;
  const int64_t nch = (n + ch - 1) / ch;
  for (int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < nch; c += (int64_t)gridDim.x * 4) {
    const int64_t r_lo = c * ch;
    const int64_t r_hi = r_lo + ch < n ? r_lo + ch : n;
    int32_t cmin = (int32_t)r_lo, cmax = (int32_t)(r_hi - 1);
    for (int64_t e = rp[r_lo] + lane; e < rp[r_hi]; e += 64) {
      const int32_t col = ci[e];
      cmin = col < cmin ? col : cmin;
      cmax = col > cmax ? col : cmax;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int32_t o1 = __shfl_xor(cmin, off, 64), o2 = __shfl_xor(cmax, off, 64);
      cmin = o1 < cmin ? o1 : cmin;
      cmax = o2 > cmax ? o2 : cmax;
    }
    if (lane == 0) win[c] = make_int2(cmin, cmax);
  }
}

hipError_t launch_csr_chunk_window(const int64_t *rp, const int32_t *ci, int64_t n, int32_t ch,
                                   int2 *win, hipStream_t st) {
  const int64_t nch = (n + ch - 1) / ch;
  const int64_t blocks = (nch + 3) / 4 < 4096 ? (nch + 3) / 4 : 4096;
  csr_chunk_window_kernel<<<(unsigned)blocks, 256, 0, st>>>(rp, ci, n, ch, win);
  return hipGetLastError();
}

// Probe (within the 64-probe chunk) of element e of lane o's P values.
template <typename T>
__device__ __forceinline__ int probe_of(int o, int e) {
  constexpr int VE = CsrLanes<T>::VE;
  return 32 * (e / VE) + VE * o + e % VE;
}

// Lane o's P probes of row r in the chunk starting at probe chunk0 (a
// multiple of 64): from V, or expanded from the sign bits.  A piece whose
// probes all lie past the probes in use (pv[h] false) is not read: zeros.
template <typename T, bool SIGNS>
__device__ __forceinline__ void load_row(const T *__restrict__ V, const uint32_t *__restrict__ signs,
                                         int64_t r, int64_t ldv, int32_t nw, int32_t chunk0, int o,
                                         T *x, const bool *pv) {
  constexpr int VE = CsrLanes<T>::VE;
  if (SIGNS) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t wd = signs[r * nw + (chunk0 >> 5) + h] >> (VE * o);
#pragma unroll
      for (int e = 0; e < VE; ++e) x[h * VE + e] = ((wd >> e) & 1u) ? T(-1) : T(1);
    }
  } else {
    typedef T v16 __attribute__((ext_vector_type(VE)));
    const T *src = V + r * ldv + chunk0 + VE * o;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v16 q = {};
      if (pv[h]) q = *(const v16 *)(src + 32 * h);
#pragma unroll
      for (int e = 0; e < VE; ++e) x[h * VE + e] = q[e];
    }
  }
}

// The same P probes from a row in LDS; `row` points at byte 16 o of the row.
template <typename T>
__device__ __forceinline__ void lds_row(const uint8_t *row, T *x) {
  constexpr int VE = CsrLanes<T>::VE;
  typedef T v16 __attribute__((ext_vector_type(VE)));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const v16 q = *(const v16 *)(row + CsrLanes<T>::HALF * h);
#pragma unroll
    for (int e = 0; e < VE; ++e) x[h * VE + e] = q[e];
  }
}

// Lane o's P values z into row r of V (global memory), pieces in use only.
template <typename T>
__device__ __forceinline__ void store_row(T *V, int64_t r, int64_t ldv, int32_t chunk0, int o, const T *z,
                                          const bool *pv) {
  constexpr int VE = CsrLanes<T>::VE;
  typedef T v16 __attribute__((ext_vector_type(VE)));
  T *dst = V + r * ldv + chunk0 + VE * o;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    v16 q;
#pragma unroll
    for (int e = 0; e < VE; ++e) q[e] = z[h * VE + e];
    if (pv[h]) *(v16 *)(dst + 32 * h) = q;
  }
}

// The same into a row in LDS; `row` points at byte 16 o of the row.
template <typename T>
__device__ __forceinline__ void lds_store_row(uint8_t *row, const T *z) {
  constexpr int VE = CsrLanes<T>::VE;
  typedef T v16 __attribute__((ext_vector_type(VE)));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    v16 q;
#pragma unroll
    for (int e = 0; e < VE; ++e) q[e] = z[h * VE + e];
    *(v16 *)(row + CsrLanes<T>::HALF * h) = q;
  }
}

template <typename T>
__device__ __forceinline__ T shfl_t(T v, int src) {
  return __shfl(v, src, 64);
}

// VK_SIGNS: V_k is the sign block.  M1: no V_{k-1} term (0), V_{k-1} stored
// (1) or the sign block (2).  GG: also accumulate g.g (first Chebyshev step).
template <typename T, bool VK_SIGNS, int M1, bool GG>
__global__ __launch_bounds__(64 * kCsrWaves) void csr_step_kernel(CsrStepArgs a) {
  typedef CsrLanes<T> C;
  constexpr int P = C::P, L = C::L, RPW = C::RPW, CH = C::CH, ROWB = C::ROWB;
  constexpr int U = 4;    // entries per gather round
  constexpr int JM = 10;  // rounds whose entries are loaded together
  constexpr bool use_win = !VK_SIGNS;  // a window of the sign block is not needed
  __shared__ __attribute__((aligned(16))) uint8_t wbuf[use_win ? 2 : 1][use_win ? C::WBYTES : 16];
  __shared__ double red[2][kCsrWaves][64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane / L;       // row of the wave's group
  const int o = lane % L;       // probe slot within the row
  const int gl = g * L;         // first lane of the row's group
  const int64_t n = a.n, ldv = a.ldv;
  const int32_t nw = (int32_t)(ldv >> 5);
  const int32_t chunk0 = (int32_t)blockIdx.y * 64;
  // pieces of this lane holding probes in use (the last chunk of a probe
  // count that is not a multiple of 64 skips the rest: no padding traffic)
  const int32_t s_use = a.s > 0 ? a.s : (int32_t)ldv;
  constexpr int VEC = C::VE;
  const bool pv[2] = {chunk0 + VEC * o < s_use, chunk0 + 32 + VEC * o < s_use};
  const int32_t chunk_bytes = (s_use - chunk0 < 64 ? s_use - chunk0 : 64) * (int32_t)sizeof(T);
  const int64_t *__restrict__ rp = a.row_ptr;
  const int32_t *__restrict__ ci = a.col_idx;
  const T *__restrict__ val = (const T *)a.values;
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  const int2 *__restrict__ win = a.win;
  // V_{k+1} is written over V_{k-1} element by element by the thread that
  // read it, so these two may alias each other (and nothing else)
  const T *Vkm1 = (const T *)a.Vkm1;
  T *Vkp1 = (T *)a.Vkp1;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  constexpr bool use_m1 = M1 != 0;
  const bool use_cg = a.cg != nullptr;
  const T tcg = use_cg ? (T)a.cg[0] : T(0);

  // contiguous chunk range per block
  const int64_t nch = (n + CH - 1) / CH;
  const int64_t cper = (nch + gridDim.x - 1) / gridDim.x;
  const int64_t c_beg = (int64_t)blockIdx.x * cper;
  const int64_t c_end = c_beg + cper < nch ? c_beg + cper : nch;
  const int64_t r_lim = c_end * CH < n ? c_end * CH : n;

  // direct global-to-LDS copy of chunk c's window (if it fits) into buffer b
  auto stage = [&](int64_t c, int b) {
    const int2 mw = win[c];
    const int nrows = mw.y - mw.x + 1;
    if (nrows > C::WROWS) return;
    const int ninstr = (nrows * ROWB + 1023) / 1024;
    for (int i = w; i < ninstr; i += kCsrWaves) {
      const int byte = i * 1024 + lane * 16;
      int64_t row = mw.x + byte / ROWB;
      row = row < mw.y ? row : mw.y;
      const uint8_t *src = (const uint8_t *)(Vk + row * ldv + chunk0) + byte % ROWB;
      // 16-byte pieces past the probes in use are not copied (never used)
      if ((byte % ROWB) < chunk_bytes)
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (__attribute__((address_space(3))) void *)(&wbuf[b][0] + i * 1024),
                                         16, 0, 0);
    }
  };

  double ds[P], gs[GG ? P : 1];
#pragma unroll
  for (int e = 0; e < P; ++e) ds[e] = 0.0;
#pragma unroll
  for (int e = 0; e < (GG ? P : 1); ++e) gs[e] = 0.0;
  // results of the previous chunk, stored after the next barrier
  T zs[P];
  int64_t zrow = -1;

  int64_t e0n = 0, e1n = 0;
  {
    const int64_t r = c_beg * CH + RPW * w + g;
    if (c_beg < c_end && r < r_lim) {
      e0n = rp[r];
      e1n = rp[r + 1];
    }
  }
  if (use_win && c_beg < c_end) stage(c_beg, 0);
  __syncthreads();
  for (int64_t c = c_beg; c < c_end; ++c) {
    const int buf = (int)((c - c_beg) & 1);
    if (zrow >= 0 && Vkp1) store_row<T>(Vkp1, zrow, ldv, chunk0, o, zs, pv);
    zrow = -1;
    if (use_win && c + 1 < c_end) stage(c + 1, buf ^ 1);
    int2 mw = make_int2(0, 0);
    bool inlds = false;
    if (use_win) {
      mw = win[c];
      inlds = mw.y - mw.x + 1 <= C::WROWS;
    }
    const uint8_t *wb = &wbuf[use_win ? buf : 0][0] + 16 * o;

    const int64_t r = c * CH + RPW * w + g;
    const bool live = r < r_lim;
    const int64_t rr = live ? r : c * CH;  // a valid row for the loads of idle lanes
    const int64_t e0 = e0n, e1 = e1n;
    const int len = live ? (int)(e1 - e0) : 0;
    const int64_t rn = r + CH;
    if (rn < r_lim) {
      e0n = rp[rn];
      e1n = rp[rn + 1];
    }
    // epilogue operands: independent of the gathers
    T xr[P], vm[P], gv[P];
    if (inlds)
      lds_row<T>(wb + (rr - mw.x) * ROWB, xr);
    else
      load_row<T, VK_SIGNS>(Vk, signs, rr, ldv, nw, chunk0, o, xr, pv);
    if (use_m1) {
      if (M1 == 2)
        load_row<T, true>(nullptr, signs, rr, ldv, nw, chunk0, o, vm, pv);
      else
        load_row<T, false>(Vkm1, nullptr, rr, ldv, nw, chunk0, o, vm, pv);
    } else {
#pragma unroll
      for (int e = 0; e < P; ++e) vm[e] = T(0);
    }
    if (signs)
      load_row<T, true>(nullptr, signs, rr, ldv, nw, chunk0, o, gv, pv);
    else
      load_row<T, false>(G, nullptr, rr, ldv, nw, chunk0, o, gv, pv);
    // longest row of the wave: the number of gather rounds
    int mlen = len;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int t = __shfl_xor(mlen, off, 64);
      mlen = t > mlen ? t : mlen;
    }
    T acc[P];
#pragma unroll
    for (int e = 0; e < P; ++e) acc[e] = T(0);
    for (int jc = 0; jc < mlen; jc += U * JM) {
      // all entries of up to JM rounds at once: lane o (< U) of the group
      // holds entry jc + U t + o of its row; entries past the row's end
      // gather the row itself with weight zero
      int32_t mc[JM];
      T mv[JM];
#pragma unroll
      for (int t = 0; t < JM; ++t) {
        const int j = jc + U * t + o;
        const bool in = o < U && j < len;
        mc[t] = in ? ci[e0 + j] : (int32_t)rr;
        mv[t] = in ? val[e0 + j] : T(0);
      }
#pragma unroll
      for (int t = 0; t < JM; ++t) {
        if (jc + U * t >= mlen) break;
        T x[U][P];
        if (inlds) {
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int32_t col = __shfl(mc[t], gl + q, 64);
            lds_row<T>(wb + (col - mw.x) * ROWB, x[q]);
          }
        } else {
#pragma unroll
          for (int q = 0; q < U; ++q) {
            const int32_t col = __shfl(mc[t], gl + q, 64);
            load_row<T, VK_SIGNS>(Vk, signs, col, ldv, nw, chunk0, o, x[q], pv);
          }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const T v = shfl_t(mv[t], gl + q);
#pragma unroll
          for (int e = 0; e < P; ++e) acc[e] += v * x[q][e];
        }
      }
    }
    if (live) {
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const T y = ta * acc[e];
        T z = tc1 * y + tb * xr[e];
        if (use_m1) z += tcw * vm[e];
        if (use_cg) z += tcg * gv[e];
        zs[e] = z;
        ds[e] += (double)gv[e] * (double)(a.dot_y ? y : z);
        if (GG) gs[GG ? e : 0] += (double)gv[e] * (double)gv[e];
      }
      zrow = r;
    }
    // the next window has landed, and every wave is done with this one
    __syncthreads();
  }
  if (zrow >= 0 && Vkp1) store_row<T>(Vkp1, zrow, ldv, chunk0, o, zs, pv);
  // probes past the ones in use: their window bytes were never copied
#pragma unroll
  for (int e = 0; e < P; ++e)
    if (!pv[e / VEC]) {
      ds[e] = 0.0;
      if (GG) gs[GG ? e : 0] = 0.0;
    }
  // per probe: sum over the wave's rows (lanes o, o+L, ...), then over waves
#pragma unroll
  for (int e = 0; e < P; ++e) {
#pragma unroll
    for (int off = L; off < 64; off <<= 1) {
      ds[e] += __shfl_xor(ds[e], off, 64);
      if (GG) gs[GG ? e : 0] += __shfl_xor(gs[GG ? e : 0], off, 64);
    }
  }
  if (lane < L) {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      red[0][w][probe_of<T>(lane, e)] = ds[e];
      red[1][w][probe_of<T>(lane, e)] = GG ? gs[GG ? e : 0] : 0.0;
    }
  }
  __syncthreads();
  if (w == 0) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int q = 0; q < kCsrWaves; ++q) {
      t0 += red[0][q][lane];
      t1 += red[1][q][lane];
    }
    const int64_t bidx = (int64_t)blockIdx.x * ldv + chunk0 + lane;
    a.part[(int64_t)a.slot * a.nblk * ldv + bidx] = t0;
    if (GG) a.part[(int64_t)a.slot_gg * a.nblk * ldv + bidx] = t1;
  }
}

// Workgroups of one step-kernel instance resident at once on the current
// device: CUs x its per-CU occupancy (registers or LDS bound it).  Every
// workgroup walks an equal share of the chunks, so a grid larger than this
// would finish in a second, partial round that takes as long as the first.
// Each instance is launched with its own count; the partial-sum stride is
// the largest count of any instance (csr_step_blocks), and the partials of
// workgroups an instance does not launch stay zero.
template <typename T, bool VK_SIGNS, int M1, bool GG>
static int32_t csr_instance_blocks() {
  static int32_t cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  if (dev < 64 && cache[dev] > 0) return cache[dev];
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)csr_step_kernel<T, VK_SIGNS, M1, GG>,
                                                   64 * kCsrWaves, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int32_t r = (int32_t)(cus * per_cu);
  if (dev < 64) cache[dev] = r;
  return r;
}

template <typename T>
static int32_t csr_resident_blocks() {
  const int32_t c[] = {csr_instance_blocks<T, true, 0, true>(), csr_instance_blocks<T, false, 0, true>(),
                       csr_instance_blocks<T, true, 0, false>(), csr_instance_blocks<T, false, 0, false>(),
                       csr_instance_blocks<T, false, 1, false>(), csr_instance_blocks<T, false, 2, false>()};
  int32_t r = 1;
  for (int32_t v : c) r = v > r ? v : r;
  return r;
}

// Persistent grid: the resident workgroups, fewer for small n.
int32_t csr_step_blocks(int64_t n, int32_t fp64) {
  const int64_t ch = fp64 ? CsrLanes<double>::CH : CsrLanes<float>::CH;
  const int64_t groups = (n + ch - 1) / ch;
  const int64_t cap = fp64 ? csr_resident_blocks<double>() : csr_resident_blocks<float>();
  return (int32_t)(groups < cap ? groups : cap);
}

template <typename T, bool VK_SIGNS, int M1, bool GG>
static void csr_step_launch(const CsrStepArgs &a, hipStream_t st) {
  const int32_t inst = csr_instance_blocks<T, VK_SIGNS, M1, GG>();
  dim3 grid((unsigned)(a.nblk < inst ? a.nblk : inst), (unsigned)(a.ldv / 64));
  csr_step_kernel<T, VK_SIGNS, M1, GG><<<grid, 64 * kCsrWaves, 0, st>>>(a);
}

// The partial slots written by a launch must be zero beyond its grid (the
// caller clears the partial buffer once per estimate).
template <typename T>
hipError_t launch_csr_step(const CsrStepArgs &a, hipStream_t st) {
  const bool vk_signs = a.Vk == nullptr;
  const int m1 = a.cw == 0.0 ? 0 : (a.Vkm1 == nullptr ? 2 : 1);
  const bool gg = a.slot_gg >= 0;
  if ((vk_signs || m1 == 2) && !a.signs) return hipErrorInvalidValue;
  if (gg) {
    if (m1 != 0) return hipErrorInvalidValue;  // g.g is taken on the first step only
    if (vk_signs)
      csr_step_launch<T, true, 0, true>(a, st);
    else
      csr_step_launch<T, false, 0, true>(a, st);
  } else if (m1 == 0) {
    if (vk_signs)
      csr_step_launch<T, true, 0, false>(a, st);
    else
      csr_step_launch<T, false, 0, false>(a, st);
  } else {
    if (vk_signs) return hipErrorInvalidValue;  // V_k is stored from the second step on
    if (m1 == 2)
      csr_step_launch<T, false, 2, false>(a, st);
    else
      csr_step_launch<T, false, 1, false>(a, st);
  }
  return hipGetLastError();
}
template hipError_t launch_csr_step<double>(const CsrStepArgs &, hipStream_t);
template hipError_t launch_csr_step<float>(const CsrStepArgs &, hipStream_t);

}  // namespace ent
