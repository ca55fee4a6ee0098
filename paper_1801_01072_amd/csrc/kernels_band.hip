// kernels_band.hip -- the recurrence step for a CSR R whose entries all lie
// in a narrow band around the diagonal (|col - row| <= HP, HP = 4, 8 or 16),
// as 16-row products on the FP32/FP64 matrix cores:
//   Y = a * (R V_k), Z = c1*Y + c2*b*V_k + cw*V_{k-1} (+ c_g g),
//   per-probe dots with g (the same algebra as the CSR and dense steps).
//
// Storage (built once per estimate by band_pack_kernel from the caller's
// CSR arrays): 16-row block b of R is the dense 16 x K slab over rows
// 16b .. 16b+15 and columns 16b-HP .. 16b+15+HP (K = 16 + 2 HP; entries
// outside the band are zero), kept in the A-operand order of the 16x16x4
// MFMA.  Lane l of k-step kk holds R[16b + l%16][16b - HP + 4kk + l/16], and
// each lane's KS = K/4 values are contiguous: band[(64 b + l) KS + kk].
// The slab has no column indices, so a step reads fewer matrix bytes than
// the CSR arrays (K values per row against 8 bytes per entry plus row
// pointers: 192 against 272 bytes per row at HP = 16 in FP32).
//
// Step: a wave owns a contiguous range of blocks and one 64-probe chunk.  The
// V_k rows a block needs (K rows) sit in registers as K/4 B-operand fragments
// of four rows each, a ring of KS + 4 fragments: while block b multiplies,
// the four fragments that block b+1 adds (and its slab values) are already
// in flight, so each V_k row is read from HBM once per wave range (plus a
// halo of HP rows at each end).  Probe p of the chunk is column p/4 of
// 16-probe tile p%4, so a lane's four tiles are four consecutive probes of
// one row: every V access (ring fragments, epilogue operands, results) is a
// 16-byte (FP32) or 32-byte (FP64) piece per lane, four whole 256 B rows per
// instruction.  There is no LDS and no barrier; per-probe dot partials stay
// in FP64 registers until the end (one partial per wave per probe, summed in
// fixed order).
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

namespace {

template <int KS>
struct BandShape {
  static constexpr int HP = 2 * KS - 8;          // padded half-bandwidth
  static constexpr int K = 4 * KS;               // slab width (= 16 + 2 HP)
  static constexpr int WF = KS + 4;              // ring: the block's fragments and the next four
};

constexpr int kBandWaves = 4;  // waves per workgroup (independent)

// KS of the instance serving padded half-bandwidth hp
inline int ks_of(int32_t hp) { return (hp + 8) / 2; }

}  // namespace

int32_t band_half_width_padded(int32_t hbw) {
  if (hbw < 0) return 0;
  if (hbw <= 4) return 4;
  if (hbw <= 8) return 8;
  if (hbw <= 16) return 16;
  return 0;
}

size_t band_pack_elems(int64_t n, int32_t hp) {
  const int64_t nb = (n + 15) / 16;
  return (size_t)nb * 64 * (size_t)ks_of(hp);
}

// ---------------------------------------------------------------------------
// Half-bandwidth of a (validated) CSR matrix: out[0] = max |col - row|
// (out[0] must start at 0).  One thread per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void csr_half_bandwidth_kernel(const int64_t *__restrict__ rp,
                                                                 const int32_t *__restrict__ ci,
                                                                 int64_t n, int32_t *__restrict__ out) {
  int32_t m = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e1 = rp[r + 1];
    for (int64_t e = rp[r]; e < e1; ++e) {
      const int64_t d = (int64_t)ci[e] - r;
      const int64_t ad = d < 0 ? -d : d;
      const int32_t a32 = ad > 0x7fffffff ? 0x7fffffff : (int32_t)ad;
      m = a32 > m ? a32 : m;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

hipError_t launch_csr_half_bandwidth(const int64_t *rp, const int32_t *ci, int64_t n, int32_t *out,
                                     hipStream_t st) {
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  csr_half_bandwidth_kernel<<<(unsigned)(blocks > 0 ? blocks : 1), 256, 0, st>>>(rp, ci, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packing: one thread per (block b, lane l) writes that lane's KS slab values.
// Requires |col - row| <= HP for every entry; duplicate entries are summed
// in entry order.
// ---------------------------------------------------------------------------
template <typename T, int KS>
__global__ __launch_bounds__(256) void band_pack_kernel(const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const T *__restrict__ val, int64_t n,
                                                        T *__restrict__ band) {
  constexpr int HP = BandShape<KS>::HP;
  const int64_t nb = (n + 15) / 16;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = idx >> 6;
  if (b >= nb) return;
  const int l = (int)(idx & 63);
  const int q = l >> 4;
  const int64_t row = 16 * b + (l & 15);
  const int64_t base = 16 * b - HP;
  T out[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) out[k] = T(0);
  if (row < n) {
    const int64_t e1 = rp[row + 1];
    for (int64_t e = rp[row]; e < e1; ++e) {
      const int64_t j = (int64_t)ci[e] - base - q;  // slab column minus this lane's k-slot
      if (j < 0 || (j & 3) != 0) continue;
      const int64_t kk = j >> 2;
      const T v = val[e];
#pragma unroll
      for (int k = 0; k < KS; ++k)
        if (k == kk) out[k] += v;
    }
  }
  T *dst = band + idx * KS;
#pragma unroll
  for (int k = 0; k < KS; ++k) dst[k] = out[k];
}

template <typename T>
hipError_t launch_band_pack(const int64_t *rp, const int32_t *ci, const T *val, int64_t n, int32_t hp,
                            T *band, hipStream_t st) {
  const int64_t threads = ((n + 15) / 16) * 64;
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  switch (hp) {
    case 4: band_pack_kernel<T, 6><<<blocks, 256, 0, st>>>(rp, ci, val, n, band); break;
    case 8: band_pack_kernel<T, 8><<<blocks, 256, 0, st>>>(rp, ci, val, n, band); break;
    case 16: band_pack_kernel<T, 12><<<blocks, 256, 0, st>>>(rp, ci, val, n, band); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_band_pack<float>(const int64_t *, const int32_t *, const float *, int64_t, int32_t,
                                            float *, hipStream_t);
template hipError_t launch_band_pack<double>(const int64_t *, const int32_t *, const double *, int64_t, int32_t,
                                             double *, hipStream_t);

// ---------------------------------------------------------------------------
// Row pieces: lane (q, c) of a 64-probe chunk handles probes 4c .. 4c+3.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void load4(const T *__restrict__ V, int64_t row, int64_t ldv, int32_t chunk0, int c,
                                      T *x) {
  typedef T v4t __attribute__((ext_vector_type(4)));
  const v4t v = *(const v4t *)(V + row * ldv + chunk0 + 4 * c);
  x[0] = v[0];
  x[1] = v[1];
  x[2] = v[2];
  x[3] = v[3];
}

template <typename T>
__device__ __forceinline__ void sign4(const uint32_t *__restrict__ signs, int64_t row, int32_t nw, int32_t chunk0,
                                      int c, T *x) {
  const uint32_t wd = signs[row * nw + (chunk0 >> 5) + (c >> 3)] >> ((4 * c) & 31);
#pragma unroll
  for (int t = 0; t < 4; ++t) x[t] = ((wd >> t) & 1u) ? T(-1) : T(1);
}

template <typename T>
__device__ __forceinline__ void store4(T *V, int64_t row, int64_t ldv, int32_t chunk0, int c, const T *z) {
  typedef T v4t __attribute__((ext_vector_type(4)));
  v4t v;
  v[0] = z[0];
  v[1] = z[1];
  v[2] = z[2];
  v[3] = z[3];
  *(v4t *)(V + row * ldv + chunk0 + 4 * c) = v;
}

// V_k (or the sign block) at `row`, zero outside [0, n).
template <typename T>
__device__ __forceinline__ void vk_piece(const T *__restrict__ Vk, const uint32_t *__restrict__ signs, bool from_signs,
                                         int64_t row, int64_t n, int64_t ldv, int32_t nw, int32_t chunk0, int c,
                                         T *x) {
  const bool in = row >= 0 && row < n;
  const int64_t rr = in ? row : 0;
  if (from_signs)
    sign4<T>(signs, rr, nw, chunk0, c, x);
  else
    load4<T>(Vk, rr, ldv, chunk0, c, x);
#pragma unroll
  for (int t = 0; t < 4; ++t) x[t] = in ? x[t] : T(0);
}

// The lane's KS slab values of block b.
template <typename T, int KS>
__device__ __forceinline__ void load_slab(const T *__restrict__ band, int64_t b, int lane, T *a) {
  typedef T v2t __attribute__((ext_vector_type(2)));
  const T *src = band + (64 * b + lane) * KS;
#pragma unroll
  for (int k = 0; k < KS; k += 2) {
    const v2t v = *(const v2t *)(src + k);
    a[k] = v[0];
    a[k + 1] = v[1];
  }
}

template <typename T, int KS>
__global__ __launch_bounds__(64 * kBandWaves) void band_step_kernel(BandStepArgs a) {
  typedef Mfma16<T> M;
  typedef typename M::v4 v4;
  constexpr int HP = BandShape<KS>::HP, WF = BandShape<KS>::WF;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const int64_t wv = (int64_t)blockIdx.x * kBandWaves + (threadIdx.x >> 6);
  const int64_t nwv = (int64_t)gridDim.x * kBandWaves;
  const int64_t n = a.n, ldv = a.ldv;
  const int32_t nw = (int32_t)(ldv >> 5);
  const int32_t chunk0 = (int32_t)blockIdx.y * 64;
  const int64_t nb = (n + 15) >> 4;
  const int64_t per = (nb + nwv - 1) / nwv;
  const int64_t b_beg = wv * per;
  const int64_t b_end = b_beg + per < nb ? b_beg + per : nb;
  const T *__restrict__ band = (const T *)a.band;
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  // V_{k+1} is written over V_{k-1} element by element by the lane that read
  // it, so these two may alias each other (and nothing else)
  const T *Vkm1 = (const T *)a.Vkm1;
  T *Vkp1 = (T *)a.Vkp1;
  const bool vk_signs = Vk == nullptr;
  const int m1 = a.cw == 0.0 ? 0 : (Vkm1 == nullptr ? 2 : 1);
  const bool gg = a.slot_gg >= 0;
  const bool g_signs = signs != nullptr && G == nullptr;
  const bool dot_y = a.dot_y != 0;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const bool use_cg = a.cg != nullptr;
  const T tcg = use_cg ? (T)a.cg[0] : T(0);

  double ds[4] = {0.0, 0.0, 0.0, 0.0}, gs[4] = {0.0, 0.0, 0.0, 0.0};
  T win[WF][4];  // fragments: V_k rows 4f + q, probes 4c .. 4c+3; the block's are 0 .. KS-1
  T an[KS];      // slab values of the next block
  if (b_beg < b_end) {
    const int64_t f0 = 4 * b_beg - HP / 4;
#pragma unroll
    for (int j = 0; j < KS; ++j) vk_piece<T>(Vk, signs, vk_signs, 4 * (f0 + j) + q, n, ldv, nw, chunk0, c, win[j]);
    load_slab<T, KS>(band, b_beg, lane, an);
  }
  for (int64_t b = b_beg; b < b_end; ++b) {
    {
      T ac[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) ac[k] = an[k];
      if (b + 1 < b_end) {
        // the four fragments block b+1 adds, and its slab
        const int64_t fn = 4 * b - HP / 4 + KS;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          vk_piece<T>(Vk, signs, vk_signs, 4 * (fn + j) + q, n, ldv, nw, chunk0, c, win[KS + j]);
        load_slab<T, KS>(band, b + 1, lane, an);
      }
      // epilogue operands of this block's rows (register r holds row drow(q, r))
      T xr[4][4], vm[4][4], gv[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * b + M::drow(q, r);
        vk_piece<T>(Vk, signs, vk_signs, row, n, ldv, nw, chunk0, c, xr[r]);
        if (m1 == 1)
          load4<T>(Vkm1, row, ldv, chunk0, c, vm[r]);
        else if (m1 == 2)
          sign4<T>(signs, row, nw, chunk0, c, vm[r]);
        else {
#pragma unroll
          for (int t = 0; t < 4; ++t) vm[r][t] = T(0);
        }
        if (g_signs)
          sign4<T>(signs, row, nw, chunk0, c, gv[r]);
        else
          load4<T>(G, row, ldv, chunk0, c, gv[r]);
      }
      // Y_b = slab_b x ring, one 16-probe tile per probe of the lane's four
      v4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < KS; ++k) {
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = M::mma(ac[k], win[k][t], acc[t]);
      }
      // slide the ring by one block
#pragma unroll
      for (int j = 0; j < KS; ++j) {
#pragma unroll
        for (int t = 0; t < 4; ++t) win[j][t] = win[j + 4][t];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * b + M::drow(q, r);
        const bool live = row < n;
        T z[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const T y = ta * acc[t][r];
          T zz = tc1 * y + tb * xr[r][t];
          if (m1 != 0) zz += tcw * vm[r][t];
          if (use_cg) zz += tcg * gv[r][t];
          z[t] = zz;
          if (live) {
            ds[t] += (double)gv[r][t] * (double)(dot_y ? y : zz);
            if (gg) gs[t] += (double)gv[r][t] * (double)gv[r][t];
          }
        }
        if (live && Vkp1) store4<T>(Vkp1, row, ldv, chunk0, c, z);
      }
    }
  }
  // per probe: the four row groups (lanes c, c+16, c+32, c+48), fixed order
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ds[t] += __shfl_xor(ds[t], 16, 64);
    ds[t] += __shfl_xor(ds[t], 32, 64);
    gs[t] += __shfl_xor(gs[t], 16, 64);
    gs[t] += __shfl_xor(gs[t], 32, 64);
  }
  if (q == 0) {
    const int64_t bidx = wv * ldv + chunk0 + 4 * c;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a.part[(int64_t)a.slot * a.nwave * ldv + bidx + t] = ds[t];
      if (gg) a.part[(int64_t)a.slot_gg * a.nwave * ldv + bidx + t] = gs[t];
    }
  }
}

// Workgroups of the instance resident at once on the current device.
template <typename T, int KS>
static int32_t band_resident_blocks() {
  static int32_t cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
  if (dev < 64 && cache[dev] > 0) return cache[dev];
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)band_step_kernel<T, KS>,
                                                   64 * kBandWaves, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int32_t r = (int32_t)(cus * per_cu);
  if (dev < 64) cache[dev] = r;
  return r;
}

// Waves of the step grid (the partial stride): the resident waves, or fewer
// so that every wave has at least eight blocks.
int32_t band_step_waves(int64_t n, int32_t hp, int32_t fp64) {
  int32_t res = 0;
  switch (hp) {
    case 4: res = fp64 ? band_resident_blocks<double, 6>() : band_resident_blocks<float, 6>(); break;
    case 8: res = fp64 ? band_resident_blocks<double, 8>() : band_resident_blocks<float, 8>(); break;
    case 16: res = fp64 ? band_resident_blocks<double, 12>() : band_resident_blocks<float, 12>(); break;
    default: return 0;
  }
  const int64_t nb = (n + 15) / 16;
  int64_t blocks = (nb + 8 * kBandWaves - 1) / (8 * kBandWaves);
  if (blocks > res) blocks = res;
  if (blocks < 1) blocks = 1;
  return (int32_t)(blocks * kBandWaves);
}

template <typename T>
hipError_t launch_band_step(const BandStepArgs &a, int32_t hp, hipStream_t st) {
  if (a.nwave <= 0 || a.nwave % kBandWaves != 0 || a.ldv % 64 != 0) return hipErrorInvalidValue;
  if ((a.Vk == nullptr || (a.cw != 0.0 && a.Vkm1 == nullptr)) && !a.signs) return hipErrorInvalidValue;
  if (a.G == nullptr && a.signs == nullptr) return hipErrorInvalidValue;
  dim3 grid((unsigned)(a.nwave / kBandWaves), (unsigned)(a.ldv / 64));
  switch (hp) {
    case 4: band_step_kernel<T, 6><<<grid, 64 * kBandWaves, 0, st>>>(a); break;
    case 8: band_step_kernel<T, 8><<<grid, 64 * kBandWaves, 0, st>>>(a); break;
    case 16: band_step_kernel<T, 12><<<grid, 64 * kBandWaves, 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_band_step<float>(const BandStepArgs &, int32_t, hipStream_t);
template hipError_t launch_band_step<double>(const BandStepArgs &, int32_t, hipStream_t);

}  // namespace ent
