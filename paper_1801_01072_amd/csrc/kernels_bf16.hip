// kernels_bf16.hip -- BF16x3 split-precision recurrence step for dense R.
//
// A = R is split once per estimate into bf16 hi = RNE(A), lo = RNE(A - hi)
// (zero padded to n_pad x n_pad; the interval scale a multiplies the FP32
// product in the epilogue, so the power method reads the same split).  Each
// step forms
//     Y = A_hi V_hi + A_hi V_lo + A_lo V_hi          (FP32 accumulation)
// on the gfx950 BF16 matrix cores (v_mfma_f32_32x32x16_bf16), then an
// elementwise epilogue applies the recurrence in FP32, re-splits V_{k+1}
// into hi/lo for the next product and accumulates the per-probe dots in FP64.
//
// Operand layout ("fragment-major"): the bf16 hi and lo arrays of A and of
// V^T are stored in the order the MFMA consumes them.  Element (r, k) of an
// R x K operand (r = matrix row for A, probe for V^T; k = the contraction
// index) lives in 1 KB block (r / 32, k / 16), blocks ordered by r / 32 then
// k / 16, at lane (r % 32) + 32 ((k % 16) / 8), element k % 8.  One block is
// one MFMA operand fragment, so every load of the GEMM reads 1 KB of
// contiguous memory and a workgroup streams each of its 32-row bands as one
// contiguous run.  The FP32 blocks (G, V_k, V_{k+1}, split-K partials) stay
// probe-major ([probe][row], leading dimension n_pad): the epilogue touches
// 8 consecutive rows of one probe per thread, which are also 8 consecutive
// elements of one lane in the fragment-major layout.
//
// MFMA 32x32x16 bf16 layout (lane l, measured on gfx950): A row l%32, k-slots
// 8(l/32)..8(l/32)+7; B column l%32, same k-slots; D register r holds row
// 8(r/4) + 4(l/32) + r%4, column l%32.
//
// GEMM tiling: a workgroup of 2 WM waves owns 64 WM rows (256 when n_pad
// allows, else 128) x BN probes over one K-split; each wave computes 64 rows
// x BN/2 probes.  A and V^T fragments reach LDS by direct global-to-LDS
// loads in a ring of 32-k stages, so A is streamed from HBM once per step.
// Split-K partials go to part_y[split][probe][row]; the epilogue sums them in
// split order (deterministic).  Workgroups are remapped so that those on one
// XCD share a K-split and hence their slice of V^T in that XCD's L2.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even FP32 -> BF16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Element offset of (r, k) in the fragment-major layout (nkb = K / 16).
__device__ __forceinline__ int64_t frag_off(int64_t r, int64_t k, int64_t nkb) {
  return ((r >> 5) * nkb + (k >> 4)) * 512 + ((r & 31) + 32 * ((k >> 3) & 1)) * 8 + (k & 7);
}

// ---------------------------------------------------------------------------
// A = a * R -> hi/lo, fragment-major, zero outside n x n; a = scal[S_A], or 1
// when scal is null (the split is then of R itself and the scale is applied
// to the product in the epilogue).  One wave per 1 KB fragment (32 rows x 16
// columns): lane l reads 8 consecutive columns of row 32 rb + l % 32 and
// writes its 16 bytes at byte 16 l, so each wave stores one contiguous
// fragment of hi and of lo.
// ---------------------------------------------------------------------------
template <typename Tin>
__global__ __launch_bounds__(256) void split_matrix_kernel(const Tin *__restrict__ R, int64_t ldr, int64_t n,
                                                           int64_t n_pad, const double *__restrict__ scal,
                                                           uint16_t *__restrict__ hi, uint16_t *__restrict__ lo) {
  constexpr int VW = 16 / (int)sizeof(Tin);  // elements per 16-byte load
  typedef Tin vec_t __attribute__((ext_vector_type(VW)));
  const double a = scal ? scal[S_A] : 1.0;
  const int64_t nkb = n_pad / 16;
  const int64_t nfrag = (n_pad / 32) * nkb;
  const int lane = threadIdx.x & 63;
  // 16-byte loads when every row start is 16-byte aligned
  const bool vec = ((uintptr_t)R % 16) == 0 && ldr % VW == 0;
  for (int64_t f = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; f < nfrag;
       f += ((int64_t)gridDim.x * blockDim.x) >> 6) {
    const int64_t row = 32 * (f / nkb) + (lane & 31);
    const int64_t c0 = 16 * (f % nkb) + 8 * (lane >> 5);
    Tin x[8];
    if (vec && 32 * (f / nkb) + 32 <= n && 16 * (f % nkb) + 16 <= n) {
      // the fragment lies inside R
      const vec_t *src = (const vec_t *)(R + row * ldr + c0);
#pragma unroll
      for (int q = 0; q < 8 / VW; ++q) {
        const vec_t t = src[q];
#pragma unroll
        for (int e = 0; e < VW; ++e) x[q * VW + e] = t[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (row < n && c0 + e < n) ? R[row * ldr + c0 + e] : Tin(0);
    }
    u16x8 h, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float v = (float)(a * (double)x[e]);
      h[e] = bf16_rne(v);
      l[e] = bf16_rne(v - bf16_to_f32(h[e]));
    }
    const int64_t off = f * 512 + 8 * lane;
    *(u16x8 *)(hi + off) = h;
    *(u16x8 *)(lo + off) = l;
  }
}

template <typename Tin>
hipError_t launch_split_matrix(const Tin *R, int64_t ldr, int64_t n, int64_t n_pad,
                               const double *scal, uint16_t *hi, uint16_t *lo, hipStream_t st) {
  const int64_t nfrag = (n_pad / 32) * (n_pad / 16);
  const int64_t blocks = (nfrag + 3) / 4 < 65536 ? (nfrag + 3) / 4 : 65536;
  split_matrix_kernel<Tin><<<(unsigned)blocks, 256, 0, st>>>(R, ldr, n, n_pad, scal, hi, lo);
  return hipGetLastError();
}
template hipError_t launch_split_matrix<double>(const double *, int64_t, int64_t, int64_t,
                                                const double *, uint16_t *, uint16_t *, hipStream_t);
template hipError_t launch_split_matrix<float>(const float *, int64_t, int64_t, int64_t,
                                               const double *, uint16_t *, uint16_t *, hipStream_t);

// ---------------------------------------------------------------------------
// Probe block: G[j][i] (FP32, probe-major) plus its hi/lo split
// (fragment-major).  Thread = 8 consecutive rows of one probe.
// ---------------------------------------------------------------------------
__global__ void probe_gen_t_kernel(float *__restrict__ G, uint16_t *__restrict__ hi,
                                   uint16_t *__restrict__ lo, int64_t n, int64_t n_pad, int32_t s,
                                   int64_t ldv, uint64_t seed, int32_t dist, uint32_t stream,
                                   double scale) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ldv * (n_pad / 8)) return;
  const int64_t j = t / (n_pad / 8), i0 = (t % (n_pad / 8)) * 8;
  float v[8];
  u16x8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t i = i0 + e;
    v[e] = 0.f;
    if (i < n && j < s)
      v[e] = (float)(scale * (dist == 0   ? rademacher(seed, stream, i, j)
                              : dist == 2 ? srht_entry(seed, i, j, hadamard_order(n))
                                          : gaussian(seed, stream, i, j)));
    h[e] = bf16_rne(v[e]);
    l[e] = bf16_rne(v[e] - bf16_to_f32(h[e]));
  }
  f32x4 *g = (f32x4 *)(G + j * n_pad + i0);
  g[0] = f32x4{v[0], v[1], v[2], v[3]};
  g[1] = f32x4{v[4], v[5], v[6], v[7]};
  const int64_t off = frag_off(j, i0, n_pad / 16);
  *(u16x8 *)(hi + off) = h;
  *(u16x8 *)(lo + off) = l;
}

hipError_t launch_probe_gen_t(float *G, uint16_t *hi, uint16_t *lo, int64_t n, int64_t n_pad,
                              int32_t s, int64_t ldv, uint64_t seed, int32_t dist, hipStream_t st,
                              uint32_t stream, double scale) {
  const int64_t tot = ldv * (n_pad / 8);
  probe_gen_t_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(G, hi, lo, n, n_pad, s, ldv, seed,
                                                                   dist, stream, scale);
  return hipGetLastError();
}

// Batch: split of every matrix (unscaled) and its probe block, one
// workgroup per (matrix, 128-row tile); thread = 8 columns (split) or 8 rows
// of one probe (probes).
template <typename Tin>
__global__ __launch_bounds__(256) void batch_split_kernel(const BatchMat *__restrict__ mats,
                                                          const int2 *__restrict__ tiles,
                                                          uint16_t *Ahi, uint16_t *Alo) {
  const int2 t = tiles[blockIdx.x];
  const BatchMat &M = mats[t.x];
  const Tin *R = (const Tin *)M.src;
  const int64_t n = M.n, n_pad = M.n_pad, nkb = n_pad / 16, cg = n_pad / 8;
  uint16_t *hi = Ahi + M.aoff, *lo = Alo + M.aoff;
  for (int64_t e = threadIdx.x; e < 128 * cg; e += blockDim.x) {
    const int64_t row = (int64_t)t.y * 128 + e / cg, c0 = (e % cg) * 8;
    u16x8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t c = c0 + q;
      const float v = (row < n && c < n) ? (float)R[row * M.ldsrc + c] : 0.f;
      h[q] = bf16_rne(v);
      l[q] = bf16_rne(v - bf16_to_f32(h[q]));
    }
    const int64_t off = frag_off(row, c0, nkb);
    *(u16x8 *)(hi + off) = h;
    *(u16x8 *)(lo + off) = l;
  }
}

template <typename Tin>
hipError_t launch_batch_split(const BatchMat *mats, const int2 *tiles, int32_t ntiles, uint16_t *Ahi,
                              uint16_t *Alo, hipStream_t st) {
  batch_split_kernel<Tin><<<(unsigned)ntiles, 256, 0, st>>>(mats, tiles, Ahi, Alo);
  return hipGetLastError();
}
template hipError_t launch_batch_split<double>(const BatchMat *, const int2 *, int32_t, uint16_t *,
                                               uint16_t *, hipStream_t);
template hipError_t launch_batch_split<float>(const BatchMat *, const int2 *, int32_t, uint16_t *,
                                              uint16_t *, hipStream_t);

__global__ __launch_bounds__(256) void batch_probe_t_kernel(const BatchMat *__restrict__ mats,
                                                            const int2 *__restrict__ tiles, float *G,
                                                            uint16_t *Vhi, uint16_t *Vlo, int32_t s,
                                                            int64_t ldv, int32_t dist) {
  const int2 t = tiles[blockIdx.x];
  const BatchMat &M = mats[t.x];
  const int64_t n_pad = M.n_pad, nkb = n_pad / 16;
  for (int64_t e = threadIdx.x; e < 16 * ldv; e += blockDim.x) {
    const int64_t j = e / 16, i0 = (int64_t)t.y * 128 + (e % 16) * 8;
    float v[8];
    u16x8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + q;
      v[q] = 0.f;
      if (i < M.n && j < s) v[q] = (float)(dist == 0 ? rademacher(M.seed, 0u, i, j) : gaussian(M.seed, 0u, i, j));
      h[q] = bf16_rne(v[q]);
      l[q] = bf16_rne(v[q] - bf16_to_f32(h[q]));
    }
    f32x4 *gp = (f32x4 *)(G + M.voff + j * n_pad + i0);
    gp[0] = f32x4{v[0], v[1], v[2], v[3]};
    gp[1] = f32x4{v[4], v[5], v[6], v[7]};
    const int64_t off = M.voff + frag_off(j, i0, nkb);
    *(u16x8 *)(Vhi + off) = h;
    *(u16x8 *)(Vlo + off) = l;
  }
}

hipError_t launch_batch_probe_t(const BatchMat *mats, const int2 *tiles, int32_t ntiles, float *G,
                                uint16_t *Vhi, uint16_t *Vlo, int32_t s, int64_t ldv, int32_t dist,
                                hipStream_t st) {
  batch_probe_t_kernel<<<(unsigned)ntiles, 256, 0, st>>>(mats, tiles, G, Vhi, Vlo, s, ldv, dist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GEMM: part_y[ks][j][i] = sum_{k in split ks} (A_hi V_hi + A_hi V_lo + A_lo V_hi)[i][j]
//
// Workgroup tile: BM = 64 WM rows x BN probes over one K-split, 2 WM waves
// in a WM x 2 grid (64 rows x BN/2 probes each).  Operand fragments (1 KB
// blocks of the fragment-major layout) reach LDS by direct global-to-LDS
// loads (no registers) in a ring of stages of BK = 32: the next stages are in
// flight while one is computed.  A fragment keeps its layout in LDS (lane l's
// 8 k-values at byte 16 l), so both the loads that fill it and the
// ds_read_b128 that consume it are contiguous per wave.
// ---------------------------------------------------------------------------
namespace {
constexpr int kBK = 32;        // k per stage
constexpr int kKS = kBK / 16;  // MFMA k-steps per stage
constexpr int kNonTemporal = 2;  // cache-policy bits of a load: non-temporal
}  // namespace

template <int BN, int WM>
struct GemmShape {
  static constexpr int WAVES = 2 * WM;
  static constexpr int BM = 64 * WM;
  static constexpr int NRB = BM / 32;                  // row blocks of the tile
  static constexpr int NCB = BN / 32;                  // probe blocks of the tile
  static constexpr int WCB = NCB / 2;                  // probe blocks per wave
  static constexpr int FA = 2 * NRB * kKS;             // A fragments per stage
  static constexpr int FB = 2 * NCB * kKS;             // B fragments per stage
  static constexpr int FST = FA + FB;                  // fragments per stage
  static constexpr int PER_WAVE = FST / WAVES;         // loads per wave per stage
  static constexpr int STAGES = (160 / FST) > 3 ? 3 : (160 / FST);
  static constexpr int LDS_BYTES = STAGES * FST * 1024;
};

// s_waitcnt vmcnt(N) in the gfx9 encoding, expcnt and lgkmcnt left free.
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// One workgroup tile over rows row0..row0+BM-1 and probes col0..col0+BN-1,
// summing k in [kbeg, kbeg + 32 nst).  Without FUSED the tile goes to
// out[col][row] (probe-major, ld = npad).  With FUSED (the tile covers all of
// K) the epilogue of `ep` runs on the accumulators: y = a acc, z = c1 y +
// c2 b V_k + cw V_{k-1}, V_{k+1} = z with its bf16 split (fragment-major), and
// the tile's per-probe dot partials go to ep->part[(slot * nblk + ptile) * ldv
// + probe].
template <int BN, int WM, bool FUSED>
__device__ __forceinline__ void bf16x3_gemm_tile(const uint16_t *__restrict__ A_hi,
                                                 const uint16_t *__restrict__ A_lo,
                                                 const uint16_t *__restrict__ V_hi,
                                                 const uint16_t *__restrict__ V_lo,
                                                 float *__restrict__ out, int64_t npad,
                                                 int64_t kbeg, int nst, int64_t row0, int64_t col0,
                                                 const Bf16EpiArgs *ep, int64_t ptile) {
  typedef GemmShape<BN, WM> S;
  static_assert(S::FST % S::WAVES == 0 && S::FA % S::WAVES == 0,
                "A and B fragments must split evenly over the waves");
  static_assert(S::STAGES >= 2, "at least two stages");
  __shared__ __attribute__((aligned(1024))) uint8_t lds[S::LDS_BYTES];

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w % WM, wc = w / WM;
  const int m32 = lane & 31, kh = lane >> 5;

  // per-lane source of each fragment this wave loads (a stage advances kKS
  // blocks of 512 elements)
  const int64_t nkb = npad / 16;
  const uint16_t *src[S::PER_WAVE];
#pragma unroll
  for (int i = 0; i < S::PER_WAVE; ++i) {
    const int f = w + S::WAVES * i;
    const uint16_t *p;
    if (f < S::FA) {
      const int hl = f / (S::NRB * kKS), rb = (f / kKS) % S::NRB, ks = f % kKS;
      p = (hl ? A_lo : A_hi) + ((row0 / 32 + rb) * nkb + kbeg / 16 + ks) * 512;
    } else {
      const int g = f - S::FA;
      const int hl = g / (S::NCB * kKS), cb = (g / kKS) % S::NCB, ks = g % kKS;
      p = (hl ? V_lo : V_hi) + ((col0 / 32 + cb) * nkb + kbeg / 16 + ks) * 512;
    }
    src[i] = p + 8 * lane;
  }
  // A is streamed once per product: its loads carry the non-temporal hint so
  // they do not displace the probe block (re-read by every row tile of the
  // same K-split on this XCD) or the partial sums the epilogue reads next
  auto issue = [&](int t) {
    uint8_t *base = lds + (t % S::STAGES) * S::FST * 1024;
#pragma unroll
    for (int i = 0; i < S::PER_WAVE; ++i) {
      const void *g = (const void *)(src[i] + (int64_t)t * kKS * 512);
      auto *l = (__attribute__((address_space(3))) void *)(base + (w + S::WAVES * i) * 1024);
      if (i < S::FA / S::WAVES)
        __builtin_amdgcn_global_load_lds(g, l, 16, 0, kNonTemporal);
      else
        __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
    }
  };

  f32x16 acc[2][S::WCB];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < S::WCB; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[r][c][e] = 0.f;

  // prologue: the first STAGES-1 stages in flight
#pragma unroll
  for (int t = 0; t < S::STAGES - 1; ++t)
    if (t < nst) issue(t);
  for (int t = 0; t < nst; ++t) {
    // this wave's loads of stage t are done once at most those of the later
    // stages already issued remain; the barrier then makes every wave's part
    // visible, and also guarantees that the stage whose buffer the next
    // issue reuses has been consumed
    if (t + S::STAGES - 2 < nst)
      wait_vm<S::PER_WAVE * (S::STAGES - 2)>();
    else
      wait_vm<0>();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if (t + S::STAGES - 1 < nst) issue(t + S::STAGES - 1);
    const uint8_t *base = lds + (t % S::STAGES) * S::FST * 1024 + 16 * lane;
#pragma unroll
    for (int ks = 0; ks < kKS; ++ks) {
      bf16x8 ah[2], al[2], bh[S::WCB], bl[S::WCB];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int rb = 2 * wr + r;
        ah[r] = *(const bf16x8 *)(base + ((0 * S::NRB + rb) * kKS + ks) * 1024);
        al[r] = *(const bf16x8 *)(base + ((1 * S::NRB + rb) * kKS + ks) * 1024);
      }
#pragma unroll
      for (int c = 0; c < S::WCB; ++c) {
        const int cb = S::WCB * wc + c;
        bh[c] = *(const bf16x8 *)(base + (S::FA + (0 * S::NCB + cb) * kKS + ks) * 1024);
        bl[c] = *(const bf16x8 *)(base + (S::FA + (1 * S::NCB + cb) * kKS + ks) * 1024);
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < S::WCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[r], bh[c], acc[r][c], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < S::WCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[r], bl[c], acc[r][c], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < S::WCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[r], bh[c], acc[r][c], 0, 0, 0);
    }
  }

  if (!FUSED) {
    // tile -> out[col][row], 4 consecutive rows per store
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int64_t rbase = row0 + 32 * (2 * wr + r) + 4 * kh;
#pragma unroll
      for (int c = 0; c < S::WCB; ++c) {
        const int64_t col = col0 + 32 * (S::WCB * wc + c) + m32;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          f32x4 v = {acc[r][c][4 * g], acc[r][c][4 * g + 1], acc[r][c][4 * g + 2], acc[r][c][4 * g + 3]};
          *(f32x4 *)(out + col * npad + rbase + 8 * g) = v;
        }
      }
    }
    return;
  }
  // fused epilogue: lane (m32, kh) holds rows rbase + 8 g + q (q < 4) of
  // probe col for every (r, c, g)
  const Bf16EpiArgs &e = *ep;
  const float ys = (float)e.scal[S_A];
  const float c1 = (float)e.c1, c2b = (float)(e.c2 * e.scal[S_B]), cw = (float)e.cw;
  const bool use_m1 = e.Vkm1 && e.cw != 0.0;

  double ds[S::WCB], gs[S::WCB];
#pragma unroll
  for (int c = 0; c < S::WCB; ++c) ds[c] = gs[c] = 0.0;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int64_t rbase = row0 + 32 * (2 * wr + r) + 4 * kh;
#pragma unroll
    for (int c = 0; c < S::WCB; ++c) {
      const int64_t col = col0 + 32 * (S::WCB * wc + c) + m32;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int64_t off = col * npad + rbase + 8 * g;
        const f32x4 vk = *(const f32x4 *)(e.Vk + off);
        const f32x4 gv = *(const f32x4 *)(e.G + off);
        f32x4 vm = {0.f, 0.f, 0.f, 0.f};
        if (use_m1) vm = *(const f32x4 *)(e.Vkm1 + off);
        f32x4 z;
        u16x4 zh, zl;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float y = ys * acc[r][c][4 * g + q];
          z[q] = c1 * y + c2b * vk[q] + cw * vm[q];
          zh[q] = bf16_rne(z[q]);
          zl[q] = bf16_rne(z[q] - bf16_to_f32(zh[q]));
          ds[c] += (double)gv[q] * (double)(e.dot_y ? y : z[q]);
          gs[c] += (double)gv[q] * (double)gv[q];
        }
        if (e.Vkp1) {
          *(f32x4 *)(e.Vkp1 + off) = z;
          const int64_t foff = frag_off(col, rbase + 8 * g, nkb);
          *(u16x4 *)(e.V_hi + foff) = zh;
          *(u16x4 *)(e.V_lo + foff) = zl;
        }
      }
    }
  }
  if (e.slot < 0) return;
  // per probe: the two lane halves, then the WM waves of a probe column
  __syncthreads();  // every wave is done with the operand stages
  double *red = (double *)lds;  // [2][WM][BN]
#pragma unroll
  for (int c = 0; c < S::WCB; ++c) {
    ds[c] += __shfl_xor(ds[c], 32, 64);
    gs[c] += __shfl_xor(gs[c], 32, 64);
    if (kh == 0) {
      const int pc = 32 * (S::WCB * wc + c) + m32;
      red[(0 * WM + wr) * BN + pc] = ds[c];
      red[(1 * WM + wr) * BN + pc] = gs[c];
    }
  }
  __syncthreads();
  for (int pc = threadIdx.x; pc < BN; pc += blockDim.x) {
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < WM; ++q) {
      t0 += red[(0 * WM + q) * BN + pc];
      t1 += red[(1 * WM + q) * BN + pc];
    }
    e.part[((int64_t)e.slot * e.nblk + ptile) * e.ldv + col0 + pc] = t0;
    if (e.slot_gg >= 0) e.part[((int64_t)e.slot_gg * e.nblk + ptile) * e.ldv + col0 + pc] = t1;
  }
}

template <int BN, int WM>
__global__ __launch_bounds__(128 * WM) void bf16x3_gemm_kernel(Bf16GemmArgs a) {
  typedef GemmShape<BN, WM> S;
  const int nrt = (int)(a.n_pad / S::BM);
  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  // tile order: row tile fastest, then K-split, then probe tile
  const int rt = b % nrt;
  const int ksp = (b / nrt) % a.splits;
  const int ct = b / (nrt * a.splits);
  bf16x3_gemm_tile<BN, WM, false>(a.A_hi, a.A_lo, a.V_hi, a.V_lo,
                                  a.part_y + (int64_t)ksp * a.ldv * a.n_pad, a.n_pad,
                                  (int64_t)ksp * a.k_per_split, (int)(a.k_per_split / kBK),
                                  (int64_t)rt * S::BM, (int64_t)ct * BN, nullptr, 0);
}

// Batch step: one workgroup per (matrix, 128-row tile) over the matrix's full
// K, with the epilogue fused (the matrix's probe block is one tile of BN =
// ldv probes).  The step reads V_k hi/lo and writes V_{k+1} hi/lo, so the
// two live in separate buffers (vin / vout, alternating by step).  The
// pointers of `base` are batch-wide and offset by the matrix's regions.
template <int BN>
__global__ __launch_bounds__(256) void batch_bf16x3_step_kernel(Bf16EpiArgs base,
                                                                const BatchMat *__restrict__ mats,
                                                                const int2 *__restrict__ tiles,
                                                                const uint16_t *Ahi, const uint16_t *Alo,
                                                                const uint16_t *vin_hi,
                                                                const uint16_t *vin_lo) {
  const int2 t = tiles[blockIdx.x];
  const BatchMat &M = mats[t.x];
  Bf16EpiArgs e = base;
  e.Vk = base.Vk + M.voff;
  e.Vkm1 = base.Vkm1 ? base.Vkm1 + M.voff : nullptr;
  e.Vkp1 = base.Vkp1 ? base.Vkp1 + M.voff : nullptr;
  e.V_hi = base.V_hi + M.voff;
  e.V_lo = base.V_lo + M.voff;
  e.G = base.G + M.voff;
  e.scal = M.scal;
  e.part = base.part + M.poff;
  e.nblk = M.ntile;
  bf16x3_gemm_tile<BN, 2, true>(Ahi + M.aoff, Alo + M.aoff, vin_hi + M.voff, vin_lo + M.voff, nullptr,
                                M.n_pad, 0, (int)(M.n_pad / kBK), (int64_t)t.y * 128, 0, &e, t.y);
}

// Persistent batch steps (BF16x3): each workgroup takes (matrix, 128-row
// tile, step) items in schedule order, waits for the matrix's previous step,
// runs the fused GEMM + epilogue tile of the grouped kernel with that step's
// recurrence (bf16 V sets by step parity), publishes it.
template <int BN>
__global__ __launch_bounds__(256) void batch_bf16x3_persistent_kernel(BatchPersistArgs pa) {
  __shared__ int sh;
  for (;;) {
    const int i = sched_next(pa.sched, &sh);
    if (i < 0) return;
    const int4 it = pa.sched.items[i];
    const BatchMat &M = pa.mats[it.x];
    if (!sched_wait(pa.sched, it.x, it.z * M.ntile, &sh)) return;
    const StepRule r = step_rule(pa.method, it.z, pa.nsteps);
    const float *bufs[3] = {(const float *)pa.G + M.voff, (const float *)pa.VA + M.voff,
                            (const float *)pa.VB + M.voff};
    Bf16EpiArgs e{};
    e.part_y = nullptr;
    e.splits = 1;
    e.Vk = bufs[r.vk];
    e.Vkm1 = r.vkm1 >= 0 ? bufs[r.vkm1] : nullptr;
    e.Vkp1 = r.vout >= 0 ? (float *)bufs[r.vout] : nullptr;
    const int pin = it.z & 1, pout = (it.z + 1) & 1;
    e.V_hi = pa.Vhi[pout] + M.voff;
    e.V_lo = pa.Vlo[pout] + M.voff;
    e.G = bufs[0];
    e.scal = M.scal;
    e.c1 = r.c1; e.c2 = r.c2; e.cw = r.cw;
    e.dot_y = r.dot_y; e.slot = r.slot; e.slot_gg = r.slot_gg;
    e.scale_y = 1;
    e.part = pa.part + M.poff;
    e.nblk = M.ntile;
    e.n_pad = M.n_pad;
    e.ldv = pa.ldv;
    e.cg = nullptr;
    bf16x3_gemm_tile<BN, 2, true>(pa.Ahi + M.aoff, pa.Alo + M.aoff, pa.Vhi[pin] + M.voff,
                                  pa.Vlo[pin] + M.voff, nullptr, M.n_pad, 0, (int)(M.n_pad / kBK),
                                  (int64_t)it.y * 128, 0, &e, it.y);
    sched_release(pa.sched, it.x);
  }
}

hipError_t launch_batch_bf16x3_persistent(const BatchPersistArgs &pa, int32_t grid, hipStream_t st) {
  if (grid < 1) return hipErrorInvalidValue;
  switch (pa.ldv) {
    case 64: batch_bf16x3_persistent_kernel<64><<<(unsigned)grid, 256, 0, st>>>(pa); break;
    case 128: batch_bf16x3_persistent_kernel<128><<<(unsigned)grid, 256, 0, st>>>(pa); break;
    case 256: batch_bf16x3_persistent_kernel<256><<<(unsigned)grid, 256, 0, st>>>(pa); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int32_t bf16x3_persistent_grid(int64_t ldv) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e;
  switch (ldv) {
    case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_bf16x3_persistent_kernel<64>, 256, 0); break;
    case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_bf16x3_persistent_kernel<128>, 256, 0); break;
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_bf16x3_persistent_kernel<256>, 256, 0); break;
    default: return 0;
  }
  if (e != hipSuccess) return 0;
  return cus * (per > 0 ? per : 1);
}

hipError_t launch_batch_bf16x3_step(const Bf16EpiArgs &base, const BatchMat *mats, const int2 *tiles,
                                    int32_t ntiles, const uint16_t *Ahi, const uint16_t *Alo,
                                    const uint16_t *vin_hi, const uint16_t *vin_lo, hipStream_t st) {
  switch (base.ldv) {
    case 64: batch_bf16x3_step_kernel<64><<<(unsigned)ntiles, 256, 0, st>>>(base, mats, tiles, Ahi, Alo, vin_hi, vin_lo); break;
    case 128: batch_bf16x3_step_kernel<128><<<(unsigned)ntiles, 256, 0, st>>>(base, mats, tiles, Ahi, Alo, vin_hi, vin_lo); break;
    case 256: batch_bf16x3_step_kernel<256><<<(unsigned)ntiles, 256, 0, st>>>(base, mats, tiles, Ahi, Alo, vin_hi, vin_lo); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Power-method product on the split of R: y = ((hi + lo) x)/||x_prev|| with
// FP64 accumulation (hi + lo is exact in FP32), reading the fragment-major
// split.  Workgroup = one 32-row band; its W waves take every W-th 16-column
// block, each lane 8 columns of one row; x must be zero beyond n.
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ void power_split_band(const uint16_t *__restrict__ hi,
                                                 const uint16_t *__restrict__ lo, int64_t n_pad,
                                                 int64_t n, const double *__restrict__ x,
                                                 const double *__restrict__ in_norm,
                                                 double *__restrict__ y, double *__restrict__ part3,
                                                 int64_t band) {
  __shared__ double red[W][32];
  const double sc = in_norm ? 1.0 / sqrt(in_norm[0]) : 1.0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nkb = n_pad / 16;
  const uint16_t *H = hi + band * nkb * 512 + 8 * lane;
  const uint16_t *Lo = lo + band * nkb * 512 + 8 * lane;
  const int64_t kofs = 8 * (lane >> 5);
  double acc = 0.0, acc2 = 0.0;
  int64_t kb = w;
  for (; kb + W < nkb; kb += 2 * W) {
    const u16x8 h0 = *(const u16x8 *)(H + kb * 512), l0 = *(const u16x8 *)(Lo + kb * 512);
    const u16x8 h1 = *(const u16x8 *)(H + (kb + W) * 512), l1 = *(const u16x8 *)(Lo + (kb + W) * 512);
    const double *x0 = x + kb * 16 + kofs, *x1 = x + (kb + W) * 16 + kofs;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      acc += (double)(bf16_to_f32(h0[e]) + bf16_to_f32(l0[e])) * x0[e];
      acc2 += (double)(bf16_to_f32(h1[e]) + bf16_to_f32(l1[e])) * x1[e];
    }
  }
  for (; kb < nkb; kb += W) {
    const u16x8 h0 = *(const u16x8 *)(H + kb * 512), l0 = *(const u16x8 *)(Lo + kb * 512);
    const double *x0 = x + kb * 16 + kofs;
#pragma unroll
    for (int e = 0; e < 8; ++e) acc += (double)(bf16_to_f32(h0[e]) + bf16_to_f32(l0[e])) * x0[e];
  }
  acc += acc2;
  acc += __shfl_xor(acc, 32, 64);  // the two 8-column halves of a row
  if (lane < 32) red[w][lane] = acc;
  __syncthreads();
  double yy = 0.0, xy = 0.0, xx = 0.0;
  if (w == 0 && lane < 32) {
    const int64_t r = band * 32 + lane;
    double s = 0.0;
    for (int q = 0; q < W; ++q) s += red[q][lane];
    if (r < n) {
      const double yv = sc * s, xs = sc * x[r];
      y[r] = yv;
      yy = yv * yv;
      xy = xs * yv;
      xx = xs * xs;
    }
  }
  block_power_partials(yy, xy, xx, part3, band);
}

__global__ __launch_bounds__(1024) void power_gemv_split_kernel(const uint16_t *__restrict__ hi,
                                                               const uint16_t *__restrict__ lo,
                                                               int64_t n_pad, int64_t n,
                                                               const double *__restrict__ x,
                                                               const double *__restrict__ in_norm,
                                                               double *__restrict__ y,
                                                               double *__restrict__ part3) {
  power_split_band<16>(hi, lo, n_pad, n, x, in_norm, y, part3, blockIdx.x);
}

// Batch: one workgroup of 4 waves per (matrix, 32-row band) (the matrices are
// at most a few thousand columns wide).
__global__ __launch_bounds__(256) void batch_power_split_kernel(const BatchMat *__restrict__ mats,
                                                                const int2 *__restrict__ ptiles,
                                                                const uint16_t *Ahi,
                                                                const uint16_t *Alo, const double *x,
                                                                const double *norm, double *y,
                                                                double *pout) {
  const int2 t = ptiles[blockIdx.x];
  const BatchMat &M = mats[t.x];
  power_split_band<4>(Ahi + M.aoff, Alo + M.aoff, M.n_pad, M.n, x + M.xoff, norm ? norm + 4 * t.x : nullptr,
                      y + M.xoff, pout + M.pboff, t.y);
}

hipError_t launch_batch_power_split(const BatchMat *mats, const int2 *ptiles, int32_t nptiles,
                                    const uint16_t *Ahi, const uint16_t *Alo, const double *x,
                                    const double *norm, double *y, double *pout, hipStream_t st) {
  batch_power_split_kernel<<<(unsigned)nptiles, 256, 0, st>>>(mats, ptiles, Ahi, Alo, x, norm, y, pout);
  return hipGetLastError();
}

int32_t power_blocks_split(int64_t n_pad) { return (int32_t)(n_pad / 32); }

// One workgroup per band leaves some CUs with two bands when the band count
// is not a multiple of 256 (n_pad = 10240: 320 bands, 3.9 TB/s against 6.2
// at 8192).  Then each band's columns are split into S parts of whole
// 16-column blocks (about 1024 workgroups in all): part p of band b goes to
// ypart[p][row], and a second pass adds the parts in order, scales, and
// forms the norm partials per 256 rows.
int32_t power_split_parts(int64_t n_pad) {
  const int64_t nb = n_pad / 32, nkb = n_pad / 16;
  if (nb % 256 == 0) return 1;
  int64_t p = 1;
  while (nb * p < 1024 && 2 * p * 16 <= nkb) p *= 2;
  return (int32_t)p;
}

__global__ __launch_bounds__(256) void power_split_part_kernel(const uint16_t *__restrict__ hi,
                                                               const uint16_t *__restrict__ lo,
                                                               int64_t n_pad, const double *__restrict__ x,
                                                               double *__restrict__ ypart, int32_t nparts) {
  constexpr int W = 4;
  __shared__ double red[W][32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t band = blockIdx.x, part = blockIdx.y;
  const int64_t nkb = n_pad / 16;
  const int64_t kb0 = part * nkb / nparts, kb1 = (part + 1) * nkb / nparts;
  const uint16_t *H = hi + band * nkb * 512 + 8 * lane;
  const uint16_t *Lo = lo + band * nkb * 512 + 8 * lane;
  const int64_t kofs = 8 * (lane >> 5);
  double acc = 0.0, acc2 = 0.0;
  int64_t kb = kb0 + w;
  for (; kb + W < kb1; kb += 2 * W) {
    const u16x8 h0 = *(const u16x8 *)(H + kb * 512), l0 = *(const u16x8 *)(Lo + kb * 512);
    const u16x8 h1 = *(const u16x8 *)(H + (kb + W) * 512), l1 = *(const u16x8 *)(Lo + (kb + W) * 512);
    const double *x0 = x + kb * 16 + kofs, *x1 = x + (kb + W) * 16 + kofs;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      acc += (double)(bf16_to_f32(h0[e]) + bf16_to_f32(l0[e])) * x0[e];
      acc2 += (double)(bf16_to_f32(h1[e]) + bf16_to_f32(l1[e])) * x1[e];
    }
  }
  for (; kb < kb1; kb += W) {
    const u16x8 h0 = *(const u16x8 *)(H + kb * 512), l0 = *(const u16x8 *)(Lo + kb * 512);
    const double *x0 = x + kb * 16 + kofs;
#pragma unroll
    for (int e = 0; e < 8; ++e) acc += (double)(bf16_to_f32(h0[e]) + bf16_to_f32(l0[e])) * x0[e];
  }
  acc += acc2;
  acc += __shfl_xor(acc, 32, 64);  // the two 8-column halves of a row
  if (lane < 32) red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && lane < 32) {
    double sum = 0.0;
    for (int q = 0; q < W; ++q) sum += red[q][lane];
    ypart[part * n_pad + band * 32 + lane] = sum;
  }
}

__global__ __launch_bounds__(256) void power_split_combine_kernel(const double *__restrict__ ypart,
                                                                  int32_t nparts, int64_t n_pad, int64_t n,
                                                                  const double *__restrict__ x,
                                                                  const double *__restrict__ in_norm,
                                                                  double *__restrict__ y,
                                                                  double *__restrict__ part3) {
  const double sc = in_norm ? 1.0 / sqrt(in_norm[0]) : 1.0;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double yy = 0.0, xy = 0.0, xx = 0.0;
  if (r < n) {
    double sum = 0.0;
    for (int32_t p = 0; p < nparts; ++p) sum += ypart[p * n_pad + r];
    const double yv = sc * sum, xs = sc * x[r];
    y[r] = yv;
    yy = yv * yv;
    xy = xs * yv;
    xx = xs * xs;
  }
  block_power_partials(yy, xy, xx, part3, blockIdx.x);
}

hipError_t launch_power_gemv_split(const uint16_t *hi, const uint16_t *lo, int64_t n_pad, int64_t n,
                                   const double *x, const double *in_norm, double *y, double *part3,
                                   double *ypart, int32_t *nblk, hipStream_t st) {
  const int32_t parts = power_split_parts(n_pad);
  if (parts > 1) {
    if (!ypart) return hipErrorInvalidValue;
    power_split_part_kernel<<<dim3((unsigned)(n_pad / 32), (unsigned)parts), 256, 0, st>>>(hi, lo, n_pad, x, ypart,
                                                                                          parts);
    const int32_t blocks = (int32_t)((n_pad + 255) / 256);
    *nblk = blocks;
    power_split_combine_kernel<<<(unsigned)blocks, 256, 0, st>>>(ypart, parts, n_pad, n, x, in_norm, y, part3);
    return hipGetLastError();
  }
  const int32_t blocks = power_blocks_split(n_pad);
  *nblk = blocks;
  power_gemv_split_kernel<<<(unsigned)blocks, 1024, 0, st>>>(hi, lo, n_pad, n, x, in_norm, y, part3);
  return hipGetLastError();
}

int32_t bf16x3_tile_rows(int64_t n_pad) { return n_pad % 256 == 0 ? 256 : 128; }

// K-splits of the GEMM for `tiles` output tiles.  A workgroup fills a CU (its
// LDS ring), so the grid runs in rounds of 256 workgroups and a split count
// costs rounds(tiles * s) / s of a full-K tile's time; each split also adds
// a partial block for the epilogue to read (weighted 1/64 per split).  Any s
// up to 16 whose column range is a multiple of 32: n_pad = 8192 (32 tiles)
// keeps 8 splits, 10240 (40 tiles) takes 5 (one round of 200) instead of 8
// (320: a second round with 64 workgroups).
int32_t bf16x3_splits(int64_t n_pad, int64_t tiles) {
  int32_t best = 1;
  double best_cost = 1e300;
  for (int32_t sp = 1; sp <= 16; ++sp) {
    if (n_pad % (32 * (int64_t)sp) != 0) continue;
    const double rounds = (double)((tiles * sp + 255) / 256);
    const double cost = rounds / sp + sp / 64.0;
    if (cost < best_cost - 1e-12) {
      best_cost = cost;
      best = sp;
    }
  }
  return best;
}

hipError_t launch_bf16x3_gemm(const Bf16GemmArgs &a, hipStream_t st) {
  const int bm = bf16x3_tile_rows(a.n_pad);
  const int nrt = (int)(a.n_pad / bm), nct = (int)(a.ldv / a.bn);
  const unsigned grid = (unsigned)(nrt * nct * a.splits);
  if (bm == 256) {
    switch (a.bn) {
      case 64: bf16x3_gemm_kernel<64, 4><<<grid, 512, 0, st>>>(a); break;
      case 128: bf16x3_gemm_kernel<128, 4><<<grid, 512, 0, st>>>(a); break;
      case 256: bf16x3_gemm_kernel<256, 4><<<grid, 512, 0, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.bn) {
      case 64: bf16x3_gemm_kernel<64, 2><<<grid, 256, 0, st>>>(a); break;
      case 128: bf16x3_gemm_kernel<128, 2><<<grid, 256, 0, st>>>(a); break;
      case 256: bf16x3_gemm_kernel<256, 2><<<grid, 256, 0, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Epilogue: y = sum_ks part_y[ks]; z = c1*y + c2*b*V_k + cw*V_{k-1};
// V_{k+1} = z (FP32) and its hi/lo split; per-probe dots with g.
// Thread = (probe j, 8 consecutive rows); block = 256 threads of one probe.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bf16x3_epilogue_body(const Bf16EpiArgs &a, int64_t blk, int64_t j) {
  __shared__ double red[2][4];
  const int64_t npad = a.n_pad;
  const int64_t i0 = (blk * blockDim.x + threadIdx.x) * 8;
  const float c1 = (float)a.c1, c2b = (float)(a.c2 * a.scal[S_B]), cw = (float)a.cw;
  const float ys = a.scale_y ? (float)a.scal[S_A] : 1.f;
  const float cg = a.cg ? (float)a.cg[0] : 0.f;
  double ds = 0.0, gs = 0.0;
  if (i0 < npad) {
    const int64_t off = j * npad + i0;
    float y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) y[e] = 0.f;
    for (int ks = 0; ks < a.splits; ++ks) {
      const f32x4 *p = (const f32x4 *)(a.part_y + (int64_t)ks * a.ldv * npad + off);
      const f32x4 p0 = p[0], p1 = p[1];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        y[e] += p0[e];
        y[4 + e] += p1[e];
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) y[e] *= ys;
    const f32x4 *vk = (const f32x4 *)(a.Vk + off);
    const f32x4 vk0 = vk[0], vk1 = vk[1];
    f32x4 vm0 = {0, 0, 0, 0}, vm1 = {0, 0, 0, 0};
    if (a.Vkm1 && a.cw != 0.0) {
      const f32x4 *vm = (const f32x4 *)(a.Vkm1 + off);
      vm0 = vm[0];
      vm1 = vm[1];
    }
    const f32x4 *gp = (const f32x4 *)(a.G + off);
    const f32x4 g0 = gp[0], g1 = gp[1];
    float z[8];
    u16x8 zh, zl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float vke = e < 4 ? vk0[e] : vk1[e - 4];
      const float vme = e < 4 ? vm0[e] : vm1[e - 4];
      const float ge = e < 4 ? g0[e] : g1[e - 4];
      z[e] = c1 * y[e] + c2b * vke + cw * vme;
      if (a.cg) z[e] += cg * ge;
      const uint16_t h = bf16_rne(z[e]);
      zh[e] = h;
      zl[e] = bf16_rne(z[e] - bf16_to_f32(h));
      if (a.slot >= 0) {
        ds += (double)ge * (double)(a.dot_y ? y[e] : z[e]);
        gs += (double)ge * (double)ge;
      }
    }
    if (a.Vkp1) {
      f32x4 *o = (f32x4 *)(a.Vkp1 + off);
      o[0] = f32x4{z[0], z[1], z[2], z[3]};
      o[1] = f32x4{z[4], z[5], z[6], z[7]};
      const int64_t foff = frag_off(j, i0, npad / 16);
      *(u16x8 *)(a.V_hi + foff) = zh;
      *(u16x8 *)(a.V_lo + foff) = zl;
    }
  }
  if (a.slot < 0) return;
  ds = wave_sum(ds);
  gs = wave_sum(gs);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = ds;
    red[1][w] = gs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nwv = blockDim.x >> 6;
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < nwv; ++q) {
      t0 += red[0][q];
      t1 += red[1][q];
    }
    a.part[((int64_t)a.slot * a.nblk + blk) * a.ldv + j] = t0;
    if (a.slot_gg >= 0) a.part[((int64_t)a.slot_gg * a.nblk + blk) * a.ldv + j] = t1;
  }
}

__global__ __launch_bounds__(256) void bf16x3_epilogue_kernel(Bf16EpiArgs a) {
  bf16x3_epilogue_body(a, blockIdx.x, blockIdx.y);
}

int32_t bf16x3_epilogue_blocks(int64_t n_pad) { return (int32_t)((n_pad / 8 + 255) / 256); }

hipError_t launch_bf16x3_epilogue(const Bf16EpiArgs &a, hipStream_t st) {
  dim3 grid((unsigned)a.nblk, (unsigned)a.ldv);
  bf16x3_epilogue_kernel<<<grid, 256, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace ent
