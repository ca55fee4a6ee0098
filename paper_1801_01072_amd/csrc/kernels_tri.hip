// kernels_tri.hip -- one step of the polynomial recurrence for a tridiagonal
// R (every entry within one of the diagonal: the paper's Poisson experiment
// of Section 6 and any R of that pattern), HBM-bound: the product
// (R V)_r = l_r V_{r-1} + d_r V_r + u_r V_{r+1} is a three-row stencil, so
// the step streams V_k, V_{k-1}, the probes and three values per row once and
// writes V_{k+1} once, with no index arrays and no gathers.
//
// Mapping: a wave runs 64 / LS independent streams of LS lanes (LS = 16, 32
// or 64: the narrowest whose 4-probe pieces cover the probes in one pass),
// each over its own contiguous range of rows; lane p of a stream owns probes
// 4 p .. 4 p + 3, and the V blocks are stored with rows of s values rounded
// up to 4 (not to 64), so each row access is one contiguous run of the
// probes in use and consecutive rows follow each other in memory.  A stream
// keeps V_{r-1} and V_r in registers and loads two new rows per iteration, so
// every V_k row is read once; latency is hidden by occupancy (loading the
// next iteration's rows ahead, or four rows per iteration, measured no
// faster).  Per-probe dot partials stay in
// FP64 registers (fixed-order sums: rows in order within a stream, streams
// and waves combined in a fixed order).  Rademacher probes are read as packed
// sign bits, also where V_k or V_{k-1} is the probe block itself.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

namespace {
constexpr int kTriWaves = 4;                 // waves per workgroup
constexpr int kTriRows = 2;                  // rows per stream iteration
}  // namespace

// Tridiagonal values of row r as {l_r, d_r, u_r, 0}; duplicate entries are
// summed in entry order.  One thread per row, grid-stride; with TRACE, each
// workgroup also sums the diagonal entries (FP64) of its rows into tmp.
template <typename T, bool TRACE>
__global__ __launch_bounds__(256) void tri_pack_kernel(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                       const T *__restrict__ val, int64_t n, T *__restrict__ D,
                                                       double *__restrict__ tmp) {
  double tr = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    T l = T(0), d = T(0), u = T(0);
    for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
      const int64_t off = (int64_t)ci[e] - r;
      if (off < 0) {
        l += val[e];
      } else if (off == 0) {
        d += val[e];
        if (TRACE) tr += (double)val[e];
      } else {
        u += val[e];
      }
    }
    D[4 * r] = l;
    D[4 * r + 1] = d;
    D[4 * r + 2] = u;
    D[4 * r + 3] = T(0);
  }
  if (TRACE) {
    __shared__ double red[4];
    tr = wave_sum(tr);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tr;
    __syncthreads();
    if (threadIdx.x == 0) tmp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// The workgroups' partial traces summed in order by one wave.
__global__ void tri_trace_sum_kernel(const double *__restrict__ tmp, int32_t cnt, double *__restrict__ trace) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < cnt; i += 64) acc += tmp[i];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) *trace = acc;
}

template <typename T>
hipError_t launch_tri_pack(const int64_t *rp, const int32_t *ci, const T *val, int64_t n, T *D, double *tmp,
                           double *trace, hipStream_t st) {
  if (n < 1) return hipErrorInvalidValue;
  const int64_t want = (n + 255) / 256;
  const int32_t blocks = (int32_t)(want < kTriTraceBlocks ? want : kTriTraceBlocks);
  if (trace) {
    if (!tmp) return hipErrorInvalidValue;
    tri_pack_kernel<T, true><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, D, tmp);
    tri_trace_sum_kernel<<<1, 64, 0, st>>>(tmp, blocks, trace);
  } else {
    tri_pack_kernel<T, false><<<(unsigned)blocks, 256, 0, st>>>(rp, ci, val, n, D, nullptr);
  }
  return hipGetLastError();
}
template hipError_t launch_tri_pack<double>(const int64_t *, const int32_t *, const double *, int64_t, double *,
                                            double *, double *, hipStream_t);
template hipError_t launch_tri_pack<float>(const int64_t *, const int32_t *, const float *, int64_t, float *,
                                           double *, double *, hipStream_t);

// Power-method product on the packed diagonals: the contract of
// launch_power_spmv (y = (R x) / ||x_prev||, one partial triple per block),
// one row per thread, grid-stride over the rows.
template <typename T>
__global__ __launch_bounds__(256) void power_tri_kernel(const T *__restrict__ D, int64_t n, const double *__restrict__ x,
                                                        const double *__restrict__ in_norm, double *__restrict__ y,
                                                        double *__restrict__ part3) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const double sc = in_norm ? 1.0 / sqrt(in_norm[0]) : 1.0;
  double yy = 0.0, xy = 0.0, xx = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const v4 d = *(const v4 *)(D + 4 * r);
    const double xr = x[r];
    const double xl = r > 0 ? x[r - 1] : 0.0;
    const double xu = r + 1 < n ? x[r + 1] : 0.0;
    const double yv = sc * (((double)d[0] * xl + (double)d[1] * xr) + (double)d[2] * xu);
    const double xs = sc * xr;
    y[r] = yv;
    yy += yv * yv;
    xy += xs * yv;
    xx += xs * xs;
  }
  block_power_partials(yy, xy, xx, part3, blockIdx.x);
}

template <typename T>
hipError_t launch_power_tri(const T *D, int64_t n, const double *x, const double *in_norm, double *y,
                            double *part3, int32_t nblk, hipStream_t st) {
  power_tri_kernel<T><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, in_norm, y, part3);
  return hipGetLastError();
}
template hipError_t launch_power_tri<double>(const double *, int64_t, const double *, const double *, double *,
                                             double *, int32_t, hipStream_t);
template hipError_t launch_power_tri<float>(const float *, int64_t, const double *, const double *, double *,
                                            double *, int32_t, hipStream_t);

// The Chebyshev step operator 2X = 2(aR - bI) on the packed diagonals
// (a = scal[S_A], b = scal[S_B], set once the interval is known): row r of P
// is {2a l_r, 2(a d_r - b), 2a u_r, 0}, so a Chebyshev step is
// z = P v - V_{k-1} (plus Clenshaw's alpha_k g).  One thread per row.
template <typename T>
__global__ __launch_bounds__(256) void tri_prepare_kernel(const T *__restrict__ D, const double *__restrict__ scal,
                                                          int64_t n, T *__restrict__ P) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  typedef T v4 __attribute__((ext_vector_type(4)));
  const double a = scal[S_A], b = scal[S_B];
  const v4 d = *(const v4 *)(D + 4 * r);
  v4 o;
  o[0] = (T)(2.0 * a * (double)d[0]);
  o[1] = (T)(2.0 * (a * (double)d[1] - b));
  o[2] = (T)(2.0 * a * (double)d[2]);
  o[3] = T(0);
  *(v4 *)(P + 4 * r) = o;
}

template <typename T>
hipError_t launch_tri_prepare(const T *D, const double *scal, int64_t n, T *P, hipStream_t st) {
  if (n < 1 || !D || !scal || !P || P == D) return hipErrorInvalidValue;
  tri_prepare_kernel<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(D, scal, n, P);
  return hipGetLastError();
}
template hipError_t launch_tri_prepare<double>(const double *, const double *, int64_t, double *, hipStream_t);
template hipError_t launch_tri_prepare<float>(const float *, const double *, int64_t, float *, hipStream_t);

// K consecutive power-method products on the packed diagonals in one pass
// (temporal blocking of the stencil on one vector).  A wave owns a
// contiguous range of rows and slides a 64-row tile along it: at tile base b
// product j covers rows b - j + lane, one row behind product j - 1, whose
// rows b - j + lane - 1 and b - j + lane are its own values one and two
// lanes down (wave-wide DPP shifts), the first lanes taking lanes 62 and 63
// of its previous tile.  The first product divides by ||x|| (in_norm, as
// launch_power_tri), the products after it by the previous launch's
// Rayleigh quotient x.y / x.x (prev3, if positive: it keeps the values near
// unit size without a norm per product), and the last one by nothing, so the
// triple written (||y||^2, x.y, x.x over the last product and its input) is
// the one launch_power_tri would give for it up to scale: the Rayleigh
// quotient and the next normalization are unchanged.  Only the last
// product is stored.
namespace {
__device__ __forceinline__ double dpp_shr1(double v, double lane0) {
  // lane i takes v of lane i - 1; lane 0 takes lane0
  const int2 a = *(const int2 *)&v, o = *(const int2 *)&lane0;
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(o.x, a.x, 0x138, 0xf, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(o.y, a.y, 0x138, 0xf, 0xf, false);
  return *(const double *)&r;
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const int2 a = *(const int2 *)&v;
  int2 r;
  r.x = __builtin_amdgcn_readlane(a.x, l);
  r.y = __builtin_amdgcn_readlane(a.y, l);
  return *(const double *)&r;
}
}  // namespace

template <typename T, int K>
__global__ __launch_bounds__(256) void power_tri_fused_kernel(const T *__restrict__ D, int64_t n,
                                                              const double *__restrict__ x,
                                                              const double *__restrict__ prev3,
                                                              double *__restrict__ y, double *__restrict__ part3) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwave = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
  const int64_t share = (n + nwave - 1) / nwave;
  const int64_t r_beg = wid * share < n ? wid * share : n;
  const int64_t r_end = r_beg + share < n ? r_beg + share : n;
  const double sc0 = prev3 ? 1.0 / sqrt(prev3[0]) : 1.0;
  double rinv = 1.0;
  if (prev3) {
    const double rho = prev3[1] / prev3[2];
    if (rho > 0.0 && isfinite(1.0 / rho)) rinv = 1.0 / rho;
  }
  double yy = 0.0, xy = 0.0, xx = 0.0;
  if (r_beg < r_end) {
    double cur[K], p62[K], p63[K];  // product j: this tile's value, lanes 62, 63 of the previous tile
#pragma unroll
    for (int j = 0; j < K; ++j) cur[j] = p62[j] = p63[j] = 0.0;
    // loads clamped into [0, n), values outside zeroed: no branches in the loop
    auto clampr = [&](int64_t r) -> int64_t { return r < 0 ? 0 : (r >= n ? n - 1 : r); };
    auto x_at = [&](int64_t r) -> double {
      const double v = x[clampr(r)];
      return r >= 0 && r < n ? v : 0.0;
    };
    for (int64_t b = r_beg - (K - 1); b - (K - 1) < r_end; b += 64) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int64_t xr = b - j + lane;
        double lo, mid, hi;
        if (j == 0) {
          lo = x_at(xr - 1);
          mid = x_at(xr);
          hi = x_at(xr + 1);
        } else {
          hi = cur[j - 1];
          mid = dpp_shr1(cur[j - 1], p63[j - 1]);
          lo = dpp_shr1(mid, p62[j - 1]);
        }
        const bool in = xr >= 0 && xr < n;
        const v4 d = *(const v4 *)(D + 4 * clampr(xr));
        double v = ((double)d[0] * lo + (double)d[1] * mid) + (double)d[2] * hi;
        if (j == 0) v *= sc0;
        if (j < K - 1) v *= rinv;
        v = in ? v : 0.0;
        cur[j] = v;
        if (j == K - 1 && xr >= r_beg && xr < r_end) {
          y[xr] = v;
          yy += v * v;
          xy += mid * v;
          xx += mid * mid;
        }
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        p62[j] = read_lane(cur[j], 62);
        p63[j] = read_lane(cur[j], 63);
      }
    }
  }
  block_power_partials(yy, xy, xx, part3, blockIdx.x);
}

template <typename T>
hipError_t launch_power_tri_fused(const T *D, int64_t n, const double *x, const double *prev3, double *y,
                                  double *part3, int32_t nblk, int32_t k, hipStream_t st) {
  if (n < 1 || nblk < 1 || !D || !x || !y || !part3 || y == x) return hipErrorInvalidValue;
  switch (k) {
    case 2: power_tri_fused_kernel<T, 2><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 3: power_tri_fused_kernel<T, 3><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 4: power_tri_fused_kernel<T, 4><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 5: power_tri_fused_kernel<T, 5><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 6: power_tri_fused_kernel<T, 6><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 7: power_tri_fused_kernel<T, 7><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 8: power_tri_fused_kernel<T, 8><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 9: power_tri_fused_kernel<T, 9><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    case 10: power_tri_fused_kernel<T, 10><<<(unsigned)nblk, 256, 0, st>>>(D, n, x, prev3, y, part3); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_power_tri_fused<double>(const double *, int64_t, const double *, const double *,
                                                   double *, double *, int32_t, int32_t, hipStream_t);
template hipError_t launch_power_tri_fused<float>(const float *, int64_t, const double *, const double *,
                                                  double *, double *, int32_t, int32_t, hipStream_t);

// Lanes per row stream for s probes: the narrowest of 16, 32, 64 whose
// 4-probe pieces cover s in one pass (so a row is read as one contiguous run
// of s values), 16 (64-probe chunks) beyond 256 probes.
__host__ __device__ inline int tri_stream_lanes(int32_t s) { return s <= 64 ? 16 : (s <= 128 ? 32 : (s <= 256 ? 64 : 16)); }

// VK_SIGNS: V_k is the sign block.  M1: no V_{k-1} term (0), V_{k-1} stored
// (1) or the sign block (2).  GG: also accumulate g.g (first Chebyshev step).
// LS: lanes per row stream (64 / LS streams per wave, 4 LS probes per pass).
template <typename T, int LS, bool VK_SIGNS, int M1, bool GG>
__global__ __launch_bounds__(64 * kTriWaves) void tri_step_kernel(TriStepArgs a) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  constexpr int NSW = 64 / LS;          // streams per wave
  constexpr int SPB = NSW * kTriWaves;  // streams per workgroup
  constexpr int PP = 4 * LS;            // probes per pass
  __shared__ double red[2][kTriWaves][PP];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = tid >> 6, q = lane / LS, p = lane % LS;
  const int64_t n = a.n, ldb = a.ldb, ldv = a.ldv;
  const int32_t chunk0 = (int32_t)blockIdx.y * PP;
  const int32_t s_use = a.s > 0 ? a.s : (int32_t)ldv;
  const int32_t col = chunk0 + 4 * p;
  // a lane whose probes all lie past the ones in use reads and writes nothing
  const bool pv = col < s_use;
  const int64_t nw = ldv >> 5;
  const int32_t wsel = col >> 5, bsh = col & 31;
  const T *__restrict__ D = (const T *)a.diag;
  const T *__restrict__ Vk = (const T *)a.Vk;
  const T *__restrict__ G = (const T *)a.G;
  const uint32_t *__restrict__ signs = a.signs;
  // V_{k+1} is written over V_{k-1} element by element by the lane that
  // read it, so these two may alias each other (and nothing else)
  const T *Vkm1 = (const T *)a.Vkm1;
  T *Vkp1 = (T *)a.Vkp1;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const bool use_cg = a.cg != nullptr;
  const T tcg = use_cg ? (T)a.cg[0] : T(0);

  // this stream's rows [r_beg, r_end): equal shares, a multiple of kTriRows
  const int64_t nstream = (int64_t)gridDim.x * SPB;
  const int64_t sid = (int64_t)blockIdx.x * SPB + w * NSW + q;
  int64_t share = (n + nstream - 1) / nstream;
  share = (share + kTriRows - 1) / kTriRows * kTriRows;
  const int64_t r_beg = sid * share < n ? sid * share : n;
  const int64_t r_end = r_beg + share < n ? r_beg + share : n;

  // row r of the sign block as this lane's four probes; zero outside [0, n)
  auto signs_row = [&](int64_t r) -> v4 {
    v4 x = {T(0), T(0), T(0), T(0)};
    if (pv && r >= 0 && r < n) {
      const uint32_t bits = signs[r * nw + wsel] >> bsh;
#pragma unroll
      for (int e = 0; e < 4; ++e) x[e] = ((bits >> e) & 1u) ? T(-1) : T(1);
    }
    return x;
  };
  auto v_row = [&](const T *V, int64_t r) -> v4 {
    v4 x = {T(0), T(0), T(0), T(0)};
    if (pv && r >= 0 && r < n) x = *(const v4 *)(V + r * ldb + col);
    return x;
  };
  auto vk_row = [&](int64_t r) -> v4 { return VK_SIGNS ? signs_row(r) : v_row(Vk, r); };
  auto vm_row = [&](int64_t r) -> v4 {
    if (M1 == 2) return signs_row(r);
    if (M1 == 1) return v_row(Vkm1, r);
    return v4{T(0), T(0), T(0), T(0)};
  };
  auto g_row = [&](int64_t r) -> v4 { return signs ? signs_row(r) : v_row(G, r); };
  auto d_row = [&](int64_t r) -> v4 {
    v4 x = {T(0), T(0), T(0), T(0)};
    if (r < n) x = *(const v4 *)(D + 4 * r);
    return x;
  };

  double ds[4] = {0.0, 0.0, 0.0, 0.0}, gs[4] = {0.0, 0.0, 0.0, 0.0};
  auto row = [&](int64_t r, const v4 &vp, const v4 &vc, const v4 &vn, const v4 &vm, const v4 &gv, const v4 &dd) {
    v4 z;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const T y = ta * ((dd[0] * vp[e] + dd[1] * vc[e]) + dd[2] * vn[e]);
      T ze = tc1 * y + tb * vc[e];
      if (M1 != 0) ze += tcw * vm[e];
      if (use_cg) ze += tcg * gv[e];
      z[e] = ze;
      ds[e] += (double)gv[e] * (double)(a.dot_y ? y : ze);
      if (GG) gs[e] += (double)gv[e] * (double)gv[e];
    }
    if (Vkp1 && pv) *(v4 *)(Vkp1 + r * ldb + col) = z;
  };

  if (r_beg < r_end) {
    v4 vp = vk_row(r_beg - 1), vc = vk_row(r_beg);
    for (int64_t r = r_beg; r < r_end; r += kTriRows) {
      const v4 n1 = vk_row(r + 1), n2 = vk_row(r + 2);
      const v4 m0 = vm_row(r), m1 = vm_row(r + 1);
      const v4 g0 = g_row(r), g1 = g_row(r + 1);
      const v4 d0 = d_row(r), d1 = d_row(r + 1);
      row(r, vp, vc, n1, m0, g0, d0);
      if (r + 1 < r_end) row(r + 1, vc, n1, n2, m1, g1, d1);
      vp = n1;
      vc = n2;
    }
  }
  // per probe: the streams of the wave (lanes p, p + LS, ...), then the
  // waves of the workgroup, in a fixed order
#pragma unroll
  for (int e = 0; e < 4; ++e) {
#pragma unroll
    for (int off = LS; off < 64; off <<= 1) {
      ds[e] += __shfl_xor(ds[e], off, 64);
      if (GG) gs[e] += __shfl_xor(gs[e], off, 64);
    }
  }
  if (lane < LS) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      red[0][w][4 * p + e] = ds[e];
      red[1][w][4 * p + e] = GG ? gs[e] : 0.0;
    }
  }
  __syncthreads();
  for (int t = tid; t < PP; t += 64 * kTriWaves) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < kTriWaves; ++k) {
      t0 += red[0][k][t];
      t1 += red[1][k][t];
    }
    if (chunk0 + t < ldv) {
      const int64_t bidx = (int64_t)blockIdx.x * ldv + chunk0 + t;
      a.part[(int64_t)a.slot * a.nblk * ldv + bidx] = t0;
      if (GG) a.part[(int64_t)a.slot_gg * a.nblk * ldv + bidx] = t1;
    }
  }
}

// Workgroups resident at once (CUs x per-CU occupancy of one instance),
// fewer when the rows give each stream less than 64 rows.
int32_t tri_step_blocks(int64_t n, int32_t s, int32_t fp64) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  const hipError_t e =
      fp64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)tri_step_kernel<double, 32, false, 1, false>,
                                                          64 * kTriWaves, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)tri_step_kernel<float, 32, false, 1, false>,
                                                          64 * kTriWaves, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t cap = (int64_t)cus * per_cu;
  const int64_t spb = (64 / tri_stream_lanes(s)) * kTriWaves;
  const int64_t want = (n + 64 * spb - 1) / (64 * spb);
  return (int32_t)(want < 1 ? 1 : (want < cap ? want : cap));
}

template <typename T, int LS, bool VK_SIGNS, int M1, bool GG>
static void tri_step_launch(const TriStepArgs &a, hipStream_t st) {
  const int32_t s_use = a.s > 0 ? a.s : (int32_t)a.ldv;
  dim3 grid((unsigned)a.nblk, (unsigned)((s_use + 4 * LS - 1) / (4 * LS)));
  tri_step_kernel<T, LS, VK_SIGNS, M1, GG><<<grid, 64 * kTriWaves, 0, st>>>(a);
}

template <typename T, int LS>
static hipError_t tri_step_dispatch(const TriStepArgs &a, hipStream_t st) {
  const bool vk_signs = a.Vk == nullptr;
  const int m1 = a.cw == 0.0 ? 0 : (a.Vkm1 == nullptr ? 2 : 1);
  const bool gg = a.slot_gg >= 0;
  if (gg) {
    if (m1 != 0) return hipErrorInvalidValue;  // g.g is taken on the first step only
    if (vk_signs)
      tri_step_launch<T, LS, true, 0, true>(a, st);
    else
      tri_step_launch<T, LS, false, 0, true>(a, st);
  } else if (m1 == 0) {
    if (vk_signs)
      tri_step_launch<T, LS, true, 0, false>(a, st);
    else
      tri_step_launch<T, LS, false, 0, false>(a, st);
  } else {
    if (vk_signs) return hipErrorInvalidValue;  // V_k is stored from the second step on
    if (m1 == 2)
      tri_step_launch<T, LS, false, 2, false>(a, st);
    else
      tri_step_launch<T, LS, false, 1, false>(a, st);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tri_step(const TriStepArgs &a, hipStream_t st) {
  const bool vk_signs = a.Vk == nullptr;
  const int m1 = a.cw == 0.0 ? 0 : (a.Vkm1 == nullptr ? 2 : 1);
  if ((vk_signs || m1 == 2) && !a.signs) return hipErrorInvalidValue;
  const int32_t s_use = a.s > 0 ? a.s : (int32_t)a.ldv;
  // V rows of ldb >= s values (a multiple of 4: 16- or 32-byte pieces stay
  // aligned); partials and sign words in rows of ldv, a multiple of 64
  if (a.nblk < 1 || a.ldv % 64 != 0 || a.ldb % 4 != 0 || a.ldb < s_use || a.ldv < s_use ||
      a.ldb > a.ldv)
    return hipErrorInvalidValue;
  switch (tri_stream_lanes(s_use)) {
    case 64: return tri_step_dispatch<T, 64>(a, st);
    case 32: return tri_step_dispatch<T, 32>(a, st);
    default: return tri_step_dispatch<T, 16>(a, st);
  }
}
template hipError_t launch_tri_step<double>(const TriStepArgs &, hipStream_t);
template hipError_t launch_tri_step<float>(const TriStepArgs &, hipStream_t);

}  // namespace ent
