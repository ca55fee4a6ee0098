// tri_fused_impl.hpp -- several steps of the polynomial recurrence for a
// tridiagonal R in one pass over V (temporal blocking of the three-row
// stencil): the step product of Algorithms 1 and 2 (the Taylor and Chebyshev
// recurrences, forward or by Clenshaw's schedule) applied NF times.  Included
// by one translation unit per element type.
//
// Mapping: a wave runs 64 / LS streams of LS lanes, each over its own
// contiguous range of rows; lane p of a stream owns probes 2 p, 2 p + 1, so
// a stream covers 2 LS probes (LS = 16, 32 or 64: the narrowest that covers
// the probes, 128-probe chunks beyond).  With LS = 64 the row index is the
// same across the wave, so the three values of a row come in through scalar
// loads.  A stream computes step 0 on its rows plus NF - 1 rows on each
// side, step j one row behind step j - 1, from the last three rows of step
// j - 1 held in registers (step j's V_{k-1} term is step j - 2's row; step
// 1's is V_k's).  Only the last two steps' rows are stored (the next launch
// needs V_{k+NF-1} and V_{k+NF}): a launch reads V_k, V_{k-1}, the probes and
// the diagonals once and writes two V blocks, four V row passes for NF steps
// instead of 3 NF.  Two probes per lane keep about a dozen registers per
// step, so ten steps fit.  Chebyshev and Clenshaw steps read the prepared
// operator 2X = 2(aR - bI) instead of R's diagonals, so a step is
// z = (2X) v - V_{k-1} (+ alpha_k g); Taylor steps fold the scale into the
// coefficient (z = (c1 a)(R v) + c2 b v) and scale the dot products of the
// product itself once at the end.  Dot partials are FP64, summed
// in a fixed order (rows in order, streams and waves in a fixed order).
#pragma once
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

namespace {
constexpr int kFusedWaves = 4;  // waves per workgroup

// Lanes per stream: the narrowest of 16, 32, 64 whose 2-probe pieces cover s.
inline int tri_fused_lanes(int32_t s) { return s <= 32 ? 16 : (s <= 64 ? 32 : 64); }
}  // namespace

// RAD: Rademacher probes (sign bits), else the Gaussian block G.  VKS: V_k
// is the sign block.  M1: step 0 has a V_{k-1} term (read from Vkm1).  GG:
// accumulate g.g (step 0).  DY: the dot products are of the product R V
// (Taylor), else of the step's result.  CG: a g term with a per-step device
// coefficient (Clenshaw's alpha_k).
template <typename T, int LS, int NF, bool RAD, bool VKS, bool M1, bool GG, bool DY, bool CG>
__global__ __launch_bounds__(64 * kFusedWaves) void tri_fused_kernel(TriFusedArgs a) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  typedef T v4 __attribute__((ext_vector_type(4)));
  constexpr int NSW = 64 / LS;
  constexpr int SPB = NSW * kFusedWaves;
  constexpr int PP = 2 * LS;
  __shared__ double red[kFusedWaves][PP];
  const int tid = threadIdx.x, lane = tid & 63;
  // with one stream per wave every row index is wave-uniform (so the
  // diagonals come in through scalar loads)
  const int w = NSW == 1 ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  const int q = lane / LS, p = lane % LS;
  const int64_t n = a.n, ldb = a.ldb, ldv = a.ldv;
  const int32_t chunk0 = (int32_t)blockIdx.y * PP;
  const int32_t s_use = a.s > 0 ? a.s : (int32_t)ldv;
  const int32_t col = chunk0 + 2 * p;
  const bool pv = col < s_use;
  const int32_t cl = pv ? col : 0;  // loads of lanes past the probes read column 0 (never stored)
  const int64_t nw = ldv >> 5;
  const int32_t wsel = cl >> 5, bsh = cl & 31;
  // Chebyshev / Clenshaw (no dot of the product itself): the prepared 2X
  const T *__restrict__ D = (const T *)(DY ? a.diag : a.prep);
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *__restrict__ Vkm1 = (const T *)a.Vkm1;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  T *__restrict__ VoutA = (T *)a.VoutA;
  T *__restrict__ VoutB = (T *)a.VoutB;
  const double ta = a.scal[S_A];
  T c1t[NF], tb[NF], cw[NF], cg[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) {
    c1t[j] = (T)(a.c1[j] * ta);
    tb[j] = (T)(a.c2[j] * a.scal[S_B]);
    cw[j] = (T)a.cw[j];
    cg[j] = CG ? (T)a.cg[j][0] : T(0);
  }

  const int64_t nstream = (int64_t)gridDim.x * SPB;
  const int64_t sid = (int64_t)blockIdx.x * SPB + w * NSW + q;
  const int64_t share = (n + nstream - 1) / nstream;
  const int64_t r_beg = sid * share < n ? sid * share : n;
  const int64_t r_end = r_beg + share < n ? r_beg + share : n;

  // every load is in bounds: rows clamped to [0, n), columns to the probes
  typedef uint32_t u2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(4))) v4 *dconst;
  auto clampr = [&](int64_t r) -> int64_t { return r < 0 ? 0 : (r >= n ? n - 1 : r); };
  auto ld2 = [&](const T *V, int64_t r) -> v2 { return *(const v2 *)(V + r * ldb + cl); };
  auto ldd = [&](int64_t r) -> v4 {
    if constexpr (NSW == 1)
      return *((dconst)D + r);
    else
      return *((const v4 *)D + r);
  };
  // sign bits of row r as XOR masks on the sign bit of an FP32 value
  auto masks = [&](int64_t r) -> u2 {
    const uint32_t b = signs[r * nw + wsel] >> bsh;
    return u2{b << 31, (b >> 1) << 31};
  };
  auto sgn2 = [&](u2 m) -> v2 { return v2{(T)__uint_as_float(0x3f800000u ^ m[0]), (T)__uint_as_float(0x3f800000u ^ m[1])}; };
  typedef typename std::conditional<RAD, u2, v2>::type GH;
  // dot-product term g * v in FP64 (a sign flip for Rademacher probes)
  auto gdot = [&](const GH &h, int e, T v) -> double {
    if constexpr (RAD) {
      if constexpr (sizeof(T) == 8)
        return __longlong_as_double(__double_as_longlong(v) ^ ((long long)h[e] << 32));
      else
        return (double)__uint_as_float(__float_as_uint(v) ^ h[e]);
    } else {
      return (double)h[e] * (double)v;
    }
  };
  auto g_of = [&](const GH &h) -> v2 {
    if constexpr (RAD)
      return sgn2(h);
    else
      return h;
  };

  double dots[NF][2], gs[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < NF; ++j) dots[j][0] = dots[j][1] = 0.0;
  if (r_beg < r_end) {
    const v2 zero = {T(0), T(0)};
    const int64_t r0 = r_beg - (NF - 1), r1 = r_end + NF - 2;
    auto vk_at = [&](int64_t r) -> v2 {
      if (r < 0 || r >= n) return zero;
      return VKS ? sgn2(masks(r)) : ld2(Vk, r);
    };
    v2 pk = vk_at(r0 - 1), ck = vk_at(r0);  // V_k[r-1], V_k[r]
    v2 ow[NF][3];                           // step j's rows r-j-2, r-j-1, r-j
    GH gh[NF];                              // probe of row r-j
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      ow[j][0] = ow[j][1] = ow[j][2] = zero;
      gh[j] = GH{};
    }
    // one row of every step: step j at row x = r - j from step j - 1's rows
    // x - 1, x, x + 1 and step j - 2's row x (step 0: V_k and V_{k-1}).  EDGE:
    // rows near the ends of the stream's range, where some rows lie outside
    // [0, n) (their results are zero) or outside the range (not stored, not
    // in the dot products).
    auto row = [&](int64_t r, auto edge_tag) {
      constexpr bool EDGE = decltype(edge_tag)::value;
      const int64_t rc = EDGE ? clampr(r) : r;
      const int64_t rn = EDGE ? clampr(r + 1) : r + 1;
      v2 nk = VKS ? sgn2(masks(rn)) : ld2(Vk, rn);
      if (EDGE && (r + 1 < 0 || r + 1 >= n)) nk = zero;
      const v2 m0 = M1 ? ld2(Vkm1, rc) : zero;
      v4 dx[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) dx[j] = ldd(EDGE ? clampr(r - j) : r - j);
#pragma unroll
      for (int j = NF - 1; j > 0; --j) gh[j] = gh[j - 1];
      if constexpr (RAD)
        gh[0] = masks(rc);
      else
        gh[0] = ld2(G, rc);
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int64_t x = r - j;
        const v2 &lo = j == 0 ? pk : ow[j - 1][0];
        const v2 &mid = j == 0 ? ck : ow[j - 1][1];
        const v2 &hi = j == 0 ? nk : ow[j - 1][2];
        const v2 &old = j == 0 ? m0 : (j == 1 ? pk : ow[j - 2][0]);
        const bool in = !EDGE || (x >= 0 && x < n);
        const bool own = !EDGE || (x >= r_beg && x < r_end);
        v2 z;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const T yt = (dx[j][0] * lo[e] + dx[j][1] * mid[e]) + dx[j][2] * hi[e];
          T ze;
          if constexpr (DY)
            ze = c1t[j] * yt + tb[j] * mid[e];
          else  // yt = 2X v; the first forward Chebyshev step is X g
            ze = (j == 0 && GG && !CG) ? T(0.5) * yt : yt;
          if (j > 0 || M1) ze += cw[j] * old[e];
          if (CG) ze += cg[j] * g_of(gh[j])[e];
          z[e] = in ? ze : T(0);
          if (own) {
            dots[j][e] += gdot(gh[j], e, DY ? yt : ze);
            if (GG && j == 0) gs[e] += (double)g_of(gh[j])[e] * (double)g_of(gh[j])[e];
          }
        }
        if (own && pv) {
          if (j == NF - 2) *(v2 *)(VoutA + x * ldb + col) = z;
          if (j == NF - 1 && VoutB) *(v2 *)(VoutB + x * ldb + col) = z;
        }
        ow[j][0] = ow[j][1];
        ow[j][1] = ow[j][2];
        ow[j][2] = z;
      }
      pk = ck;
      ck = nk;
    };
    // steady rows: every step's row inside the range, V_k's next row inside [0, n)
    const int64_t s_lo = r_beg + NF - 1;
    const int64_t s_hi = r_end - 1 < n - 2 ? r_end - 1 : n - 2;
    if (s_lo > s_hi) {
      for (int64_t r = r0; r <= r1; ++r) row(r, std::true_type{});
    } else {
      for (int64_t r = r0; r < s_lo; ++r) row(r, std::true_type{});
#pragma unroll 3
      for (int64_t r = s_lo; r <= s_hi; ++r) row(r, std::false_type{});
      for (int64_t r = s_hi + 1; r <= r1; ++r) row(r, std::true_type{});
    }
  }
  // a dot product of the product itself was taken on R~ v: scale it by a
  if (DY) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      dots[j][0] *= ta;
      dots[j][1] *= ta;
    }
  }
  // streams of a wave, then waves, in a fixed order; one slot at a time
  const int64_t bbase = (int64_t)blockIdx.x * ldv + chunk0;
#pragma unroll
  for (int j = 0; j <= NF; ++j) {
    if (j == NF && !GG) break;
    double v0 = j < NF ? dots[j][0] : gs[0], v1 = j < NF ? dots[j][1] : gs[1];
#pragma unroll
    for (int off = LS; off < 64; off <<= 1) {
      v0 += __shfl_xor(v0, off, 64);
      v1 += __shfl_xor(v1, off, 64);
    }
    if (lane < LS) {
      red[w][2 * p] = v0;
      red[w][2 * p + 1] = v1;
    }
    __syncthreads();
    const int32_t slot = j < NF ? a.slot[j] : a.slot_gg;
    for (int t = tid; t < PP; t += 64 * kFusedWaves) {
      if (chunk0 + t < ldv) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kFusedWaves; ++k) acc += red[k][t];
        a.part[(int64_t)slot * a.nblk * ldv + bbase + t] = acc;
      }
    }
    __syncthreads();
  }
}

namespace {
// Workgroups of one instance resident at once (the grid of one pass, so no
// workgroup waits for a second round), at most the partial stride.
template <typename T, int LS, int NF, bool RAD, bool VKS, bool M1, bool GG, bool DY, bool CG>
int32_t tri_fused_grid(int32_t nblk) {
  static int32_t cap = 0;
  if (cap == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void *)tri_fused_kernel<T, LS, NF, RAD, VKS, M1, GG, DY, CG>, 64 * kFusedWaves, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    cap = cus * per_cu;
  }
  return nblk < cap ? nblk : cap;
}

template <typename T, int LS, int NF, bool RAD, bool VKS, bool M1, bool GG, bool DY, bool CG>
hipError_t tri_fused_launch(const TriFusedArgs &a, int32_t s_use, hipStream_t st) {
  dim3 grid((unsigned)tri_fused_grid<T, LS, NF, RAD, VKS, M1, GG, DY, CG>(a.nblk),
            (unsigned)((s_use + 2 * LS - 1) / (2 * LS)));
  tri_fused_kernel<T, LS, NF, RAD, VKS, M1, GG, DY, CG><<<grid, 64 * kFusedWaves, 0, st>>>(a);
  return hipGetLastError();
}

// The launches the engine makes: Taylor (DY, no V_{k-1} term), forward
// Chebyshev and Clenshaw (CG), each as the first launch (V_k the probe block
// or, for Clenshaw, the zero block; g.g taken) or a later one (V_{k-1} read),
// with either probe kind.
template <typename T, int LS, int NF>
hipError_t tri_fused_dispatch(const TriFusedArgs &a, int32_t s_use, hipStream_t st, bool rad, bool vks, bool m1,
                              bool gg, bool dy, bool cg) {
  const int code = (rad ? 32 : 0) | (vks ? 16 : 0) | (m1 ? 8 : 0) | (gg ? 4 : 0) | (dy ? 2 : 0) | (cg ? 1 : 0);
  switch (code) {
    // Taylor
    case 32 | 16 | 2: return tri_fused_launch<T, LS, NF, true, true, false, false, true, false>(a, s_use, st);
    case 32 | 2: return tri_fused_launch<T, LS, NF, true, false, false, false, true, false>(a, s_use, st);
    case 2: return tri_fused_launch<T, LS, NF, false, false, false, false, true, false>(a, s_use, st);
    // forward Chebyshev
    case 32 | 16 | 4: return tri_fused_launch<T, LS, NF, true, true, false, true, false, false>(a, s_use, st);
    case 32 | 8: return tri_fused_launch<T, LS, NF, true, false, true, false, false, false>(a, s_use, st);
    case 4: return tri_fused_launch<T, LS, NF, false, false, false, true, false, false>(a, s_use, st);
    case 8: return tri_fused_launch<T, LS, NF, false, false, true, false, false, false>(a, s_use, st);
    // Clenshaw
    case 32 | 4 | 1: return tri_fused_launch<T, LS, NF, true, false, false, true, false, true>(a, s_use, st);
    case 32 | 8 | 1: return tri_fused_launch<T, LS, NF, true, false, true, false, false, true>(a, s_use, st);
    case 4 | 1: return tri_fused_launch<T, LS, NF, false, false, false, true, false, true>(a, s_use, st);
    case 8 | 1: return tri_fused_launch<T, LS, NF, false, false, true, false, false, true>(a, s_use, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int NF>
hipError_t tri_fused_width(const TriFusedArgs &a, int32_t s_use, hipStream_t st, bool rad, bool vks, bool m1,
                           bool gg, bool dy, bool cg) {
  switch (tri_fused_lanes(s_use)) {
    case 16: return tri_fused_dispatch<T, 16, NF>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 32: return tri_fused_dispatch<T, 32, NF>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    default: return tri_fused_dispatch<T, 64, NF>(a, s_use, st, rad, vks, m1, gg, dy, cg);
  }
}
}  // namespace

template <typename T>
hipError_t launch_tri_fused(const TriFusedArgs &a, int32_t nf, hipStream_t st) {
  if (nf < 2 || nf > kTriMaxFuse) return hipErrorInvalidValue;
  const bool rad = a.signs != nullptr;
  const bool vks = a.Vk == nullptr;
  const bool m1 = a.cw[0] != 0.0;
  const bool gg = a.slot_gg >= 0;
  const bool dy = a.dot_y[0] != 0;
  const bool cg = a.cg[0] != nullptr;
  // one kind of step throughout; the probe block must exist in the form used
  for (int32_t j = 1; j < nf; ++j)
    if ((a.dot_y[j] != 0) != dy || (a.cg[j] != nullptr) != cg) return hipErrorInvalidValue;
  if ((vks && !rad) || (!rad && !a.G) || (m1 && !a.Vkm1) || (gg && m1)) return hipErrorInvalidValue;
  // Chebyshev / Clenshaw on the prepared 2X: every step is 2X v (c1 = 2,
  // c2 = -2), except the first forward Chebyshev step, X g (c1 = 1, c2 = -1)
  if (!dy) {
    if (!a.prep || a.prep == a.diag) return hipErrorInvalidValue;
    for (int32_t j = 0; j < nf; ++j) {
      const bool half = j == 0 && gg && !cg;
      if (a.c1[j] != (half ? 1.0 : 2.0) || a.c2[j] != -a.c1[j]) return hipErrorInvalidValue;
    }
  }
  const int32_t s_use = a.s > 0 ? a.s : (int32_t)a.ldv;
  if (a.n < 1 || a.nblk < 1 || a.ldv % 64 != 0 || a.ldb % 4 != 0 || a.ldb < s_use || a.ldv < s_use ||
      a.ldb > a.ldv || !a.VoutA || !a.scal || !a.part || !a.diag || (!vks && !a.Vk))
    return hipErrorInvalidValue;
  const void *outs[2] = {a.VoutA, a.VoutB};
  for (const void *o : outs)
    if (o && (o == a.Vk || o == a.Vkm1 || o == a.G || o == a.diag || o == a.prep)) return hipErrorInvalidValue;
  switch (nf) {
    case 2: return tri_fused_width<T, 2>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 3: return tri_fused_width<T, 3>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 4: return tri_fused_width<T, 4>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 5: return tri_fused_width<T, 5>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 6: return tri_fused_width<T, 6>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 7: return tri_fused_width<T, 7>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 8: return tri_fused_width<T, 8>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    case 9: return tri_fused_width<T, 9>(a, s_use, st, rad, vks, m1, gg, dy, cg);
    default: return tri_fused_width<T, 10>(a, s_use, st, rad, vks, m1, gg, dy, cg);
  }
}

}  // namespace ent
