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
// of four rows each, a window of KS + 4 fragments slid by one block after
// each product: while block b multiplies, the four fragments that block b+1
// adds (and its slab values) are already in flight, so each V_k row is read
// from HBM once per wave range (plus a halo of HP rows at each end).  Probe p of the chunk is column p/4 of
// 16-probe tile p%4, so a lane's four tiles are four consecutive probes of
// one row: every V access (window fragments, epilogue operands, results) is
// a 16-byte (FP32) or 32-byte (FP64) piece per lane, four whole 256 B rows per
// instruction.  The epilogue's V_k rows are taken from the window, not read
// again.  There is no LDS and no barrier; per-probe dot partials stay
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
  static constexpr int WF = KS + 4;              // window: the block's fragments and the next four
};

constexpr int kBandWaves = 4;  // waves per workgroup (independent)
constexpr int kBandPairProbes = 2;  // probes per lane of the two-step kernel (32-probe chunks)

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
// Row of entry e among the 16 rows r0 .. r0+15 whose row pointers are bnd[0..16]
// (wave-uniform): the number of row starts after r0 at or before e.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int row_in_block(int64_t e, const int64_t *bnd) {
  int i = 0;
#pragma unroll
  for (int k = 1; k < 16; ++k) i += e >= bnd[k] ? 1 : 0;
  return i;
}

// The row pointers rp[r0 .. r0+16] (clamped at n) of one 16-row block, as
// wave-uniform values.
__device__ __forceinline__ void block_bounds(const int64_t *__restrict__ rp, int64_t r0, int64_t n, int lane,
                                             int64_t *bnd) {
  const int64_t r = r0 + (lane < 16 ? lane : 16);
  const int64_t v = rp[r < n ? r : n];
#pragma unroll
  for (int k = 0; k <= 16; ++k) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v & 0xffffffffu), k);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), k);
    bnd[k] = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
  }
}

// ---------------------------------------------------------------------------
// Half-bandwidth of a (validated) CSR matrix: out[0] = max |col - row|
// (out[0] must start at 0).  One wave per 16-row block, grid-stride: the
// block's entries are read contiguously, and an entry's row is found from
// the block's row pointers.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void csr_half_bandwidth_kernel(const int64_t *__restrict__ rp,
                                                                 const int32_t *__restrict__ ci,
                                                                 int64_t n, int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t nb = (n + 15) / 16;
  int64_t m = 0;
  for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += (int64_t)gridDim.x * 4) {
    int64_t bnd[17];
    block_bounds(rp, 16 * b, n, lane, bnd);
    for (int64_t e = bnd[0] + lane; e < bnd[16]; e += 64) {
      const int64_t d = (int64_t)ci[e] - (16 * b + row_in_block(e, bnd));
      const int64_t ad = d < 0 ? -d : d;
      m = ad > m ? ad : m;
    }
  }
  int32_t m32 = m > 0x7fffffff ? 0x7fffffff : (int32_t)m;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t o = __shfl_xor(m32, off, 64);
    m32 = o > m32 ? o : m32;
  }
  if (lane == 0 && m32 > 0) atomicMax(out, m32);
}

hipError_t launch_csr_half_bandwidth(const int64_t *rp, const int32_t *ci, int64_t n, int32_t *out,
                                     hipStream_t st) {
  const int64_t nb = (n + 15) / 16;
  const int64_t blocks = (nb + 3) / 4 < 4096 ? (nb + 3) / 4 : 4096;
  csr_half_bandwidth_kernel<<<(unsigned)(blocks > 0 ? blocks : 1), 256, 0, st>>>(rp, ci, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packing: one wave per 16-row block.  The block's entries are copied into
// LDS with contiguous loads (when they fit), then lane l gathers the KS slab
// values of row l%16 and k-slot l/16 by walking that row's entries in order
// (duplicate entries are summed in entry order).  Requires |col - row| <= HP
// for every entry.
// ---------------------------------------------------------------------------
template <typename T, int KS>
__global__ __launch_bounds__(256) void band_pack_kernel(const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const T *__restrict__ val, int64_t n,
                                                        T *__restrict__ band) {
  constexpr int HP = BandShape<KS>::HP;
  constexpr int CAP = 1024;  // entries of a block staged in LDS
  __shared__ int32_t scol[4][CAP];
  __shared__ T sval[4][CAP];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, q = l >> 4;
  const int64_t nb = (n + 15) / 16;
  const int64_t b = (int64_t)blockIdx.x * 4 + w;
  const bool live = b < nb;
  int64_t bnd[17];
  bool staged = false;
  if (live) {
    block_bounds(rp, 16 * b, n, l, bnd);
    staged = bnd[16] - bnd[0] <= CAP;
    if (staged) {
      for (int64_t e = bnd[0] + l; e < bnd[16]; e += 64) {
        scol[w][e - bnd[0]] = ci[e];
        sval[w][e - bnd[0]] = val[e];
      }
    }
  }
  __syncthreads();
  if (!live) return;
  const int i = l & 15;
  const int64_t row = 16 * b + i;
  const int64_t base = 16 * b - HP;
  T out[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) out[k] = T(0);
  if (row < n) {
    const int64_t e1 = rp[row + 1];
    for (int64_t e = rp[row]; e < e1; ++e) {
      const int32_t col = staged ? scol[w][e - bnd[0]] : ci[e];
      const int64_t j = (int64_t)col - base - q;  // slab column minus this lane's k-slot
      if (j < 0 || (j & 3) != 0) continue;
      const int64_t kk = j >> 2;
      const T v = staged ? sval[w][e - bnd[0]] : val[e];
#pragma unroll
      for (int k = 0; k < KS; ++k)
        if (k == kk) out[k] += v;
    }
  }
  T *dst = band + (64 * b + l) * KS;
#pragma unroll
  for (int k = 0; k < KS; ++k) dst[k] = out[k];
}

template <typename T>
hipError_t launch_band_pack(const int64_t *rp, const int32_t *ci, const T *val, int64_t n, int32_t hp,
                            T *band, hipStream_t st) {
  const int64_t nb = (n + 15) / 16;
  const unsigned blocks = (unsigned)((nb + 3) / 4);
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

// The block's own V_k rows 16b .. 16b+15 in the MFMA result order, from the
// four window fragments that hold them (fragment j: row 16b + 4j + q at lane
// group q).  FP64 results hold row q + 4r in register r at lane group q: the
// fragments themselves.  FP32 results hold row 4q + r: a transpose of
// (fragment, lane group), done in registers by two rounds of lane-group
// swaps (32-lane halves between fragments j and j+2, then 16-lane rows
// between fragments 2i and 2i+1).
template <typename T>
__device__ __forceinline__ void own_rows(const T *f0, const T *f1, const T *f2, const T *f3, T (*x)[4]) {
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x[0][t] = f0[t];
      x[1][t] = f1[t];
      x[2][t] = f2[t];
      x[3][t] = f3[t];
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      uint32_t m0 = __float_as_uint(f0[t]), m1 = __float_as_uint(f1[t]);
      uint32_t m2 = __float_as_uint(f2[t]), m3 = __float_as_uint(f3[t]);
      const auto a02 = __builtin_amdgcn_permlane32_swap(m0, m2, false, false);
      const auto a13 = __builtin_amdgcn_permlane32_swap(m1, m3, false, false);
      m0 = a02[0];
      m2 = a02[1];
      m1 = a13[0];
      m3 = a13[1];
      const auto b01 = __builtin_amdgcn_permlane16_swap(m0, m1, false, false);
      const auto b23 = __builtin_amdgcn_permlane16_swap(m2, m3, false, false);
      x[0][t] = __uint_as_float(b01[0]);
      x[1][t] = __uint_as_float(b01[1]);
      x[2][t] = __uint_as_float(b23[0]);
      x[3][t] = __uint_as_float(b23[1]);
    }
  }
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

// ---------------------------------------------------------------------------
// Power-method product on the slabs (Algorithm 4): y = (R x) / ||x_prev||
// in FP64, and the block triples (sums of y^2, xs.y, xs^2 with
// xs = x / ||x_prev||) of the CSR product.  A workgroup takes four slab
// blocks (64 rows) per pass, grid-stride; lane l of a block's wave forms
// the partial sum of its k-slot over the KS k-steps of row l%16, and the
// four k-slots are added in fixed order.
// ---------------------------------------------------------------------------
template <typename T, int KS>
__global__ __launch_bounds__(256) void power_band_kernel(const T *__restrict__ band, int64_t n,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ in_norm,
                                                         double *__restrict__ y, double *__restrict__ part3) {
  constexpr int HP = BandShape<KS>::HP;
  const double sc = in_norm ? 1.0 / sqrt(in_norm[0]) : 1.0;
  const int lane = threadIdx.x & 63, q = lane >> 4;
  const int64_t nb = (n + 15) / 16;
  double yy = 0.0, xy = 0.0, xx = 0.0;
  for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nb; b += (int64_t)gridDim.x * 4) {
    T a[KS];
    load_slab<T, KS>(band, b, lane, a);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int64_t col = 16 * b - HP + 4 * k + q;
      const double xv = (col >= 0 && col < n) ? x[col] : 0.0;
      acc += (double)a[k] * xv;
    }
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    const int64_t row = 16 * b + (lane & 15);
    if (q == 0 && row < n) {
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
hipError_t launch_power_band(const T *band, int32_t hp, int64_t n, const double *x, const double *in_norm,
                             double *y, double *part3, int32_t nblk, hipStream_t st) {
  if (nblk < 1) return hipErrorInvalidValue;
  switch (hp) {
    case 4: power_band_kernel<T, 6><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, in_norm, y, part3); break;
    case 8: power_band_kernel<T, 8><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, in_norm, y, part3); break;
    case 16: power_band_kernel<T, 12><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, in_norm, y, part3); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_power_band<float>(const float *, int32_t, int64_t, const double *, const double *,
                                             double *, double *, int32_t, hipStream_t);
template hipError_t launch_power_band<double>(const double *, int32_t, int64_t, const double *, const double *,
                                              double *, double *, int32_t, hipStream_t);

// K consecutive power-method products on the slabs in one pass (temporal
// blocking, as launch_power_tri_fused): a wave owns a contiguous range of
// 16-row blocks; product j runs one block behind product j - 1 (a block's
// stencil reaches at most 16 rows, one block, to each side) and reads product
// j - 1's values of the three blocks around its own from a four-block ring in
// LDS, private to the wave.  Each product reads its block's slab: from HBM for
// product 0, from the caches for the products a few blocks behind.  Scaling
// and the triple as launch_power_tri_fused.
template <typename T, int KS, int K>
__global__ __launch_bounds__(256) void power_band_fused_kernel(const T *__restrict__ band, int64_t n,
                                                               const double *__restrict__ x,
                                                               const double *__restrict__ prev3,
                                                               double *__restrict__ y, double *__restrict__ part3) {
  constexpr int HP = BandShape<KS>::HP;
  __shared__ double ring[4][K][4][16];  // [wave][product][block & 3][row in block]
  const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nb = (n + 15) / 16;
  const int64_t nwave = (int64_t)gridDim.x * 4;
  const int64_t wid = (int64_t)blockIdx.x * 4 + w;
  const int64_t per = (nb + nwave - 1) / nwave;
  const int64_t b_beg = wid * per < nb ? wid * per : nb;
  const int64_t b_end = b_beg + per < nb ? b_beg + per : nb;
  const double sc0 = prev3 ? 1.0 / sqrt(prev3[0]) : 1.0;
  double rinv = 1.0;
  if (prev3) {
    const double rho = prev3[1] / prev3[2];
    if (rho > 0.0 && isfinite(1.0 / rho)) rinv = 1.0 / rho;
  }
  double yy = 0.0, xy = 0.0, xx = 0.0;
  if (b_beg < b_end) {
    for (int i = lane; i < K * 64; i += 64) (&ring[w][0][0][0])[i] = 0.0;
    for (int64_t beta = b_beg - (K - 1); beta - (K - 1) < b_end; ++beta) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int64_t bb = beta - j;
        const bool blk_in = bb >= 0 && bb < nb;
        T a[KS];
        if (blk_in) {
          load_slab<T, KS>(band, bb, lane, a);
        } else {
#pragma unroll
          for (int k = 0; k < KS; ++k) a[k] = T(0);
        }
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
          const int64_t col = 16 * bb - HP + 4 * k + q;
          double xv;
          if (j == 0)
            xv = (col >= 0 && col < n) ? x[col] : 0.0;
          else
            xv = ring[w][j - 1][(col >> 4) & 3][col & 15];
          acc += (double)a[k] * xv;
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        const int64_t row = 16 * bb + c;
        double v = acc;
        if (j == 0) v *= sc0;
        if (j < K - 1) v *= rinv;
        v = (blk_in && row < n) ? v : 0.0;
        if (j == K - 1 && q == 0 && bb >= b_beg && bb < b_end && row < n) {
          const double xin = ring[w][K - 2][bb & 3][c];  // the last product's input row
          y[row] = v;
          yy += v * v;
          xy += xin * v;
          xx += xin * xin;
        }
        if (q == 0) ring[w][j][bb & 3][c] = v;
      }
    }
  }
  block_power_partials(yy, xy, xx, part3, blockIdx.x);
}

template <typename T, int KS>
static void power_band_fused_k(const T *band, int64_t n, const double *x, const double *prev3, double *y,
                               double *part3, int32_t nblk, int32_t k, hipStream_t st) {
  switch (k) {
    case 2: power_band_fused_kernel<T, KS, 2><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 3: power_band_fused_kernel<T, KS, 3><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 4: power_band_fused_kernel<T, KS, 4><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 5: power_band_fused_kernel<T, KS, 5><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 6: power_band_fused_kernel<T, KS, 6><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 7: power_band_fused_kernel<T, KS, 7><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 8: power_band_fused_kernel<T, KS, 8><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    case 9: power_band_fused_kernel<T, KS, 9><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
    default: power_band_fused_kernel<T, KS, 10><<<(unsigned)nblk, 256, 0, st>>>(band, n, x, prev3, y, part3); break;
  }
}

// Workgroups of the fused banded power launch: at most 512 (2048 waves), so
// that a wave's range is long against the K - 1 blocks of lead-in.
int32_t power_band_fused_blocks(int64_t n) {
  const int64_t nb = (n + 15) / 16;
  const int64_t b = (nb + 63) / 64;
  return (int32_t)(b < 1 ? 1 : (b < 512 ? b : 512));
}

template <typename T>
hipError_t launch_power_band_fused(const T *band, int32_t hp, int64_t n, const double *x, const double *prev3,
                                   double *y, double *part3, int32_t nblk, int32_t k, hipStream_t st) {
  if (n < 1 || nblk < 1 || k < 2 || k > kPowerMaxFuse || !band || !x || !y || !part3 || y == x)
    return hipErrorInvalidValue;
  switch (hp) {
    case 4: power_band_fused_k<T, 6>(band, n, x, prev3, y, part3, nblk, k, st); break;
    case 8: power_band_fused_k<T, 8>(band, n, x, prev3, y, part3, nblk, k, st); break;
    case 16: power_band_fused_k<T, 12>(band, n, x, prev3, y, part3, nblk, k, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_power_band_fused<float>(const float *, int32_t, int64_t, const double *, const double *,
                                                   double *, double *, int32_t, int32_t, hipStream_t);
template hipError_t launch_power_band_fused<double>(const double *, int32_t, int64_t, const double *,
                                                    const double *, double *, double *, int32_t, int32_t,
                                                    hipStream_t);

// VKS: V_k is the sign block.  M1: no V_{k-1} term (0), V_{k-1} stored (1)
// or the sign block (2).  GS: the probe rows come from the sign bits.  All
// three are compile-time choices, so a block's row loads issue together
// rather than one branch and wait each.
template <typename T, int KS, bool VKS, int M1, bool GS>
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
  constexpr bool vk_signs = VKS;
  constexpr int m1 = M1;
  const bool gg = a.slot_gg >= 0;
  constexpr bool g_signs = GS;
  const bool dot_y = a.dot_y != 0;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const bool use_cg = a.cg != nullptr;
  const T tcg = use_cg ? (T)a.cg[0] : T(0);

  double ds[4] = {0.0, 0.0, 0.0, 0.0}, gs[4] = {0.0, 0.0, 0.0, 0.0};
  T win[WF][4];  // window fragments: V_k rows 4f + q, probes 4c .. 4c+3; the block's are 0 .. KS-1
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
        // the four fragments block b+1 adds, and its slab.  Loaded from
        // clamped rows and not zeroed, so the loads stay in flight across
        // this block's products: a row outside [0, n) meets zero slab
        // coefficients (the slabs hold no entry outside the matrix)
        const int64_t fn = 4 * b - HP / 4 + KS;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t row = 4 * (fn + j) + q;
          const int64_t rr = row < 0 ? 0 : (row >= n ? n - 1 : row);
          if (vk_signs)
            sign4<T>(signs, rr, nw, chunk0, c, win[KS + j]);
          else
            load4<T>(Vk, rr, ldv, chunk0, c, win[KS + j]);
        }
        load_slab<T, KS>(band, b + 1, lane, an);
      }
      // epilogue operands of this block's rows (register r holds row drow(q, r));
      // the V_k rows come from the window (fragments HP/4 .. HP/4+3)
      T xr[4][4], vm[4][4], gv[4][4];
      own_rows<T>(win[HP / 4], win[HP / 4 + 1], win[HP / 4 + 2], win[HP / 4 + 3], xr);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * b + M::drow(q, r);
        if constexpr (m1 == 1)
          load4<T>(Vkm1, row, ldv, chunk0, c, vm[r]);
        else if constexpr (m1 == 2)
          sign4<T>(signs, row, nw, chunk0, c, vm[r]);
        else {
#pragma unroll
          for (int t = 0; t < 4; ++t) vm[r][t] = T(0);
        }
        if constexpr (g_signs)
          sign4<T>(signs, row, nw, chunk0, c, gv[r]);
        else
          load4<T>(G, row, ldv, chunk0, c, gv[r]);
      }
      // Y_b = slab_b x window, one 16-probe tile per probe of the lane's four
      v4 acc[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < KS; ++k) {
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = M::mma(ac[k], win[k][t], acc[t]);
      }
      // slide the window by one block
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

// ---------------------------------------------------------------------------
// Two steps per pass (FP32).  A wave walks step A over the blocks of its range
// plus one block on each side (V_{k+1} of a neighbouring block is needed by
// step B at the range's edges; those two are computed but neither stored nor
// counted), and step B one block behind: after step A of block b, the V_{k+1}
// fragments of blocks b-2 .. b are in a second register window and step B
// of block b-1 multiplies the slab of b-1 (kept from step A) with them.
// Step B's V_k term is V_{k+1} of its block (step A's result, kept), its
// V_{k-1} term is V_k of its block (step A's window rows, kept), and its
// probe rows are step A's.  So a pair reads each slab, V_k, V_{k-1} and probe
// row once and writes V_{k+1} and V_{k+2}: 4 V row passes per two steps
// instead of 6.  Step A's result rows go from the MFMA result order to the
// B-operand fragment order by the same transpose own_rows does (its own
// inverse).
// ---------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ void pair_load(const float *__restrict__ V, int64_t row, int64_t ldv, int32_t col0, float *x) {
  typedef float vN __attribute__((ext_vector_type(NP)));
  const vN v = *(const vN *)(V + row * ldv + col0);
#pragma unroll
  for (int t = 0; t < NP; ++t) x[t] = v[t];
}
template <int NP>
__device__ __forceinline__ void pair_signs(const uint32_t *__restrict__ signs, int64_t row, int32_t nw, int32_t col0,
                                           float *x) {
  const uint32_t wd = signs[row * nw + (col0 >> 5)] >> (col0 & 31);
#pragma unroll
  for (int t = 0; t < NP; ++t) x[t] = ((wd >> t) & 1u) ? -1.f : 1.f;
}
template <int NP>
__device__ __forceinline__ void pair_store(float *V, int64_t row, int64_t ldv, int32_t col0, const float *z) {
  typedef float vN __attribute__((ext_vector_type(NP)));
  vN v;
#pragma unroll
  for (int t = 0; t < NP; ++t) v[t] = z[t];
  *(vN *)(V + row * ldv + col0) = v;
}
// V_k (or the sign block) at `row`, zero outside [0, n).
template <int NP>
__device__ __forceinline__ void pair_vk(const float *__restrict__ Vk, const uint32_t *__restrict__ signs, bool from_signs,
                                        int64_t row, int64_t n, int64_t ldv, int32_t nw, int32_t col0, float *x) {
  const bool in = row >= 0 && row < n;
  const int64_t rr = in ? row : 0;
  if (from_signs)
    pair_signs<NP>(signs, rr, nw, col0, x);
  else
    pair_load<NP>(Vk, rr, ldv, col0, x);
#pragma unroll
  for (int t = 0; t < NP; ++t) x[t] = in ? x[t] : 0.f;
}
// The block's own rows in the MFMA result order from four fragments (and
// back: the transpose is its own inverse), NP probes per lane.
template <int NP>
__device__ __forceinline__ void pair_own(const float *f0, const float *f1, const float *f2, const float *f3,
                                         float (*x)[NP]) {
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    uint32_t m0 = __float_as_uint(f0[t]), m1 = __float_as_uint(f1[t]);
    uint32_t m2 = __float_as_uint(f2[t]), m3 = __float_as_uint(f3[t]);
    const auto a02 = __builtin_amdgcn_permlane32_swap(m0, m2, false, false);
    const auto a13 = __builtin_amdgcn_permlane32_swap(m1, m3, false, false);
    m0 = a02[0];
    m2 = a02[1];
    m1 = a13[0];
    m3 = a13[1];
    const auto b01 = __builtin_amdgcn_permlane16_swap(m0, m1, false, false);
    const auto b23 = __builtin_amdgcn_permlane16_swap(m2, m3, false, false);
    x[0][t] = __uint_as_float(b01[0]);
    x[1][t] = __uint_as_float(b01[1]);
    x[2][t] = __uint_as_float(b23[0]);
    x[3][t] = __uint_as_float(b23[1]);
  }
}

// NP: probes per lane (4: 64-probe chunks; 2: 32-probe chunks, half the
// per-lane state, the slabs read once per chunk).  GS: the probe rows come
// from the sign bits (Rademacher), else from G; a compile-time choice, so the
// four rows' loads of a block issue together instead of one branch each.
template <int KS, int NP, bool VK_SIGNS, int M1A, bool GG, bool GS>
__global__ __launch_bounds__(64 * kBandWaves) void band_pair_kernel(BandPairArgs a) {
  typedef float T;
  typedef Mfma16<T> M;
  typedef typename M::v4 v4;
  constexpr int HP = BandShape<KS>::HP, WF = BandShape<KS>::WF;
  constexpr int W2 = 4 - HP / 4;  // first fragment of step B's window in the 12-fragment ring
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, c = lane & 15;
  const int64_t wv = (int64_t)blockIdx.x * kBandWaves + (threadIdx.x >> 6);
  const int64_t nwv = (int64_t)gridDim.x * kBandWaves;
  const int64_t n = a.n, ldv = a.ldv;
  const int32_t nw = (int32_t)(ldv >> 5);
  const int32_t chunk0 = (int32_t)blockIdx.y * (16 * NP);
  const int32_t col0 = chunk0 + NP * c;
  const int64_t nb = (n + 15) >> 4;
  const int64_t per = (nb + nwv - 1) / nwv;
  const int64_t b_beg = wv * per < nb ? wv * per : nb;
  const int64_t b_end = b_beg + per < nb ? b_beg + per : nb;
  const T *__restrict__ band = (const T *)a.band;
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *__restrict__ Vkm1 = (const T *)a.Vkm1;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  T *__restrict__ VoutA = (T *)a.VoutA;
  T *__restrict__ VoutB = (T *)a.VoutB;
  constexpr bool g_signs = GS;
  const T ta = (T)a.scal[S_A];
  const T tbA = (T)(a.c2[0] * a.scal[S_B]), tbB = (T)(a.c2[1] * a.scal[S_B]);
  const T c1A = (T)a.c1[0], c1B = (T)a.c1[1], cwA = (T)a.cw[0], cwB = (T)a.cw[1];
  const T cgA = a.cg[0] ? (T)a.cg[0][0] : T(0), cgB = a.cg[1] ? (T)a.cg[1][0] : T(0);
  const bool dyA = a.dot_y[0] != 0, dyB = a.dot_y[1] != 0;

  double dA[NP], dB[NP], gs[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) dA[t] = dB[t] = gs[t] = 0.0;
  if (b_beg < b_end) {
    const int64_t a_beg = b_beg - 1, a_end = b_end + 1;  // step A blocks [a_beg, a_end)
    T win[WF][NP];   // V_k fragments of step A's current block
    T an[KS];       // slab of the next step-A block
    T w2[12][NP];    // V_{k+1} fragments of blocks b-2, b-1, b after step A of block b
    T acp[KS];      // slab of the previous block (step B's)
    T zp[4][NP], xp[4][NP], gp[4][NP];  // previous block: V_{k+1}, V_k, probe rows (result order)
#pragma unroll
    for (int j = 0; j < 12; ++j)
#pragma unroll
      for (int t = 0; t < NP; ++t) w2[j][t] = T(0);
    {
      const int64_t f0 = 4 * a_beg - HP / 4;
#pragma unroll
      for (int j = 0; j < KS; ++j)
        pair_vk<NP>(Vk, signs, VK_SIGNS, 4 * (f0 + j) + q, n, ldv, nw, col0, win[j]);
      if (a_beg >= 0)
        load_slab<T, KS>(band, a_beg, lane, an);
      else {
#pragma unroll
        for (int k = 0; k < KS; ++k) an[k] = T(0);
      }
    }
    for (int64_t b = a_beg; b < a_end; ++b) {
      T ac[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) ac[k] = an[k];
      if (b + 1 < a_end) {
        // the next block's four window fragments, rows 4 fn .. 4 fn + 15,
        // loaded from clamped rows and not zeroed, so the loads stay in
        // flight across this block's products: a row outside [0, n) meets
        // zero slab coefficients (the slabs hold no entry outside the
        // matrix), and rows past n give results that are zeroed before
        // any store or dot product
        const int64_t fn = 4 * b - HP / 4 + KS;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t row = 4 * (fn + j) + q;
          const int64_t rr = row < 0 ? 0 : (row >= n ? n - 1 : row);
          if (VK_SIGNS)
            pair_signs<NP>(signs, rr, nw, col0, win[KS + j]);
          else
            pair_load<NP>(Vk, rr, ldv, col0, win[KS + j]);
        }
        if (b + 1 < nb) {
          load_slab<T, KS>(band, b + 1, lane, an);
        } else {
#pragma unroll
          for (int k = 0; k < KS; ++k) an[k] = T(0);
        }
      }
      // step A on block b
      T xr[4][NP], vm[4][NP], gv[4][NP];
      pair_own<NP>(win[HP / 4], win[HP / 4 + 1], win[HP / 4 + 2], win[HP / 4 + 3], xr);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * b + M::drow(q, r);
        const bool in = row >= 0 && row < n;
        const int64_t rr = in ? row : 0;
        if (M1A == 1)
          pair_load<NP>(Vkm1, rr, ldv, col0, vm[r]);
        else if (M1A == 2)
          pair_signs<NP>(signs, rr, nw, col0, vm[r]);
        if constexpr (g_signs)
          pair_signs<NP>(signs, rr, nw, col0, gv[r]);
        else
          pair_load<NP>(G, rr, ldv, col0, gv[r]);
        // a row outside [0, n) keeps the (finite) values of row rr: its
        // results are zeroed below and it adds to no dot product
        if (M1A == 0) {
#pragma unroll
          for (int t = 0; t < NP; ++t) vm[r][t] = T(0);
        }
      }
      v4 acc[NP];
#pragma unroll
      for (int t = 0; t < NP; ++t) acc[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < KS; ++k) {
#pragma unroll
        for (int t = 0; t < NP; ++t) acc[t] = M::mma(ac[k], win[k][t], acc[t]);
      }
#pragma unroll
      for (int j = 0; j < KS; ++j) {
#pragma unroll
        for (int t = 0; t < NP; ++t) win[j][t] = win[j + 4][t];
      }
      const bool own = b >= b_beg && b < b_end;
      T za[4][NP];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * b + M::drow(q, r);
        const bool in = row >= 0 && row < n;
#pragma unroll
        for (int t = 0; t < NP; ++t) {
          const T y = ta * acc[t][r];
          T z = c1A * y + tbA * xr[r][t];
          if (M1A != 0) z += cwA * vm[r][t];
          z += cgA * gv[r][t];
          za[r][t] = in ? z : T(0);
          if (own && in) {
            dA[t] += (double)gv[r][t] * (double)(dyA ? y : z);
            if (GG) gs[t] += (double)gv[r][t] * (double)gv[r][t];
          }
        }
        if (own && in) pair_store<NP>(VoutA, row, ldv, col0, za[r]);
      }
      // V_{k+1} of block b into the step-B window (fragment order)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
#pragma unroll
        for (int t = 0; t < NP; ++t) w2[j][t] = w2[j + 4][t];
      }
      {
        T fr[4][NP];
        pair_own<NP>(za[0], za[1], za[2], za[3], fr);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int t = 0; t < NP; ++t) w2[8 + j][t] = fr[j][t];
      }
      // step B on block b - 1
      const int64_t cb = b - 1;
      if (cb >= b_beg && cb < b_end) {
        v4 bcc[NP];
#pragma unroll
        for (int t = 0; t < NP; ++t) bcc[t] = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int k = 0; k < KS; ++k) {
#pragma unroll
          for (int t = 0; t < NP; ++t) bcc[t] = M::mma(acp[k], w2[W2 + k][t], bcc[t]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = 16 * cb + M::drow(q, r);
          const bool in = row < n;
          T z4[NP];
#pragma unroll
          for (int t = 0; t < NP; ++t) {
            const T y = ta * bcc[t][r];
            T z = c1B * y + tbB * zp[r][t];
            z += cwB * xp[r][t];
            z += cgB * gp[r][t];
            z4[t] = z;
            if (in) dB[t] += (double)gp[r][t] * (double)(dyB ? y : z);
          }
          if (in && VoutB) pair_store<NP>(VoutB, row, ldv, col0, z4);
        }
      }
      // this block's values for step B at the next block
#pragma unroll
      for (int k = 0; k < KS; ++k) acp[k] = ac[k];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < NP; ++t) {
          zp[r][t] = za[r][t];
          xp[r][t] = xr[r][t];
          gp[r][t] = gv[r][t];
        }
    }
  }
  // per probe: the four row groups (lanes c, c+16, c+32, c+48), fixed order
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    dA[t] += __shfl_xor(dA[t], 16, 64);
    dA[t] += __shfl_xor(dA[t], 32, 64);
    dB[t] += __shfl_xor(dB[t], 16, 64);
    dB[t] += __shfl_xor(dB[t], 32, 64);
    if (GG) {
      gs[t] += __shfl_xor(gs[t], 16, 64);
      gs[t] += __shfl_xor(gs[t], 32, 64);
    }
  }
  if (q == 0) {
    const int64_t bidx = wv * ldv + col0;
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      a.part[(int64_t)a.slot[0] * a.nwave * ldv + bidx + t] = dA[t];
      a.part[(int64_t)a.slot[1] * a.nwave * ldv + bidx + t] = dB[t];
      if (GG) a.part[(int64_t)a.slot_gg * a.nwave * ldv + bidx + t] = gs[t];
    }
  }
}

template <int KS, bool VK_SIGNS, int M1A, bool GG>
static void band_pair_launch(const BandPairArgs &a, hipStream_t st) {
  constexpr int NP = kBandPairProbes;
  dim3 grid((unsigned)(a.nwave / kBandWaves), (unsigned)(a.ldv / (16 * NP)));
  if (a.signs != nullptr && a.G == nullptr)
    band_pair_kernel<KS, NP, VK_SIGNS, M1A, GG, true><<<grid, 64 * kBandWaves, 0, st>>>(a);
  else
    band_pair_kernel<KS, NP, VK_SIGNS, M1A, GG, false><<<grid, 64 * kBandWaves, 0, st>>>(a);
}

template <int KS>
static hipError_t band_pair_dispatch(const BandPairArgs &a, hipStream_t st) {
  const bool vk_signs = a.Vk == nullptr;
  const int m1 = a.cw[0] == 0.0 ? 0 : (a.Vkm1 == nullptr ? 2 : 1);
  const bool gg = a.slot_gg >= 0;
  if (gg) {
    if (m1 != 0) return hipErrorInvalidValue;  // g.g is taken on the first step only
    if (vk_signs)
      band_pair_launch<KS, true, 0, true>(a, st);
    else
      band_pair_launch<KS, false, 0, true>(a, st);
  } else if (m1 == 0) {
    if (vk_signs)
      band_pair_launch<KS, true, 0, false>(a, st);
    else
      band_pair_launch<KS, false, 0, false>(a, st);
  } else {
    if (vk_signs) return hipErrorInvalidValue;  // V_k is stored from the second step on
    if (m1 == 2)
      band_pair_launch<KS, false, 2, false>(a, st);
    else
      band_pair_launch<KS, false, 1, false>(a, st);
  }
  return hipGetLastError();
}

hipError_t launch_band_pair(const BandPairArgs &a, int32_t hp, hipStream_t st) {
  if (a.nwave <= 0 || a.nwave % kBandWaves != 0 || a.ldv % 64 != 0 || !a.VoutA) return hipErrorInvalidValue;
  if ((a.Vk == nullptr || (a.cw[0] != 0.0 && a.Vkm1 == nullptr)) && !a.signs) return hipErrorInvalidValue;
  if (a.G == nullptr && a.signs == nullptr) return hipErrorInvalidValue;
  // outputs must not alias the inputs (other waves read the input rows next
  // to their ranges during the launch)
  const void *outs[2] = {a.VoutA, a.VoutB};
  for (const void *o : outs)
    if (o && (o == a.Vk || o == a.Vkm1 || o == a.G)) return hipErrorInvalidValue;
  switch (hp) {
    case 4: return band_pair_dispatch<6>(a, st);
    case 8: return band_pair_dispatch<8>(a, st);
    case 16: return band_pair_dispatch<12>(a, st);
    default: return hipErrorInvalidValue;
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
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)band_step_kernel<T, KS, false, 1, true>,
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

template <typename T, int KS, bool VKS, int M1>
static hipError_t band_step_launch(const BandStepArgs &a, dim3 grid, hipStream_t st) {
  if (a.signs != nullptr && a.G == nullptr)
    band_step_kernel<T, KS, VKS, M1, true><<<grid, 64 * kBandWaves, 0, st>>>(a);
  else
    band_step_kernel<T, KS, VKS, M1, false><<<grid, 64 * kBandWaves, 0, st>>>(a);
  return hipGetLastError();
}

// V_k is the sign block only on the first step, which has no V_{k-1} term.
template <typename T, int KS>
static hipError_t band_step_dispatch(const BandStepArgs &a, dim3 grid, hipStream_t st) {
  const bool vks = a.Vk == nullptr;
  const int m1 = a.cw == 0.0 ? 0 : (a.Vkm1 == nullptr ? 2 : 1);
  if (vks) return m1 == 0 ? band_step_launch<T, KS, true, 0>(a, grid, st) : hipErrorInvalidValue;
  switch (m1) {
    case 0: return band_step_launch<T, KS, false, 0>(a, grid, st);
    case 1: return band_step_launch<T, KS, false, 1>(a, grid, st);
    default: return band_step_launch<T, KS, false, 2>(a, grid, st);
  }
}

template <typename T>
hipError_t launch_band_step(const BandStepArgs &a, int32_t hp, hipStream_t st) {
  if (a.nwave <= 0 || a.nwave % kBandWaves != 0 || a.ldv % 64 != 0) return hipErrorInvalidValue;
  if ((a.Vk == nullptr || (a.cw != 0.0 && a.Vkm1 == nullptr)) && !a.signs) return hipErrorInvalidValue;
  if (a.G == nullptr && a.signs == nullptr) return hipErrorInvalidValue;
  dim3 grid((unsigned)(a.nwave / kBandWaves), (unsigned)(a.ldv / 64));
  switch (hp) {
    case 4: return band_step_dispatch<T, 6>(a, grid, st);
    case 8: return band_step_dispatch<T, 8>(a, grid, st);
    case 16: return band_step_dispatch<T, 12>(a, grid, st);
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_band_step<float>(const BandStepArgs &, int32_t, hipStream_t);
template hipError_t launch_band_step<double>(const BandStepArgs &, int32_t, hipStream_t);

}  // namespace ent
