// kernels_dense.hip -- one step of the polynomial recurrence for dense R on
// gfx950 matrix cores (FP64 / FP32 MFMA 16x16x4), with the recurrence update
// and the per-probe dot products fused into the epilogue.
//
//   Y = a * (R V_k)                                  (MFMA, K = n)
//   Z = c1*Y + c2*b*V_k + cw*V_{k-1}  -> V_{k+1}      (epilogue)
//   part[slot][tile][j] = sum_{rows of tile} g_ij * (dot_y ? Y : Z)_ij
//
// Chebyshev (Algorithm 2 via the forward three-term recurrence of T_w,
// Section 3 / Appendix B): a = 2/(u-lo), b = (u+lo)/(u-lo); step 0 has
// (c1,c2,cw) = (1,-1,0), later steps (2,-2,-1); dots with Z give
// d_{k+1,j} = g_j^T T_{k+1}(X) g_j.  Taylor (Algorithm 1): a = 1/u, b = 1,
// (c1,c2,cw) = (-1,1,0) so Z = (I - R/u) V_k, dots with Y give
// e_{k,j} = g_j^T (R/u)(I - R/u)^k g_j.
//
// Tiling: a workgroup of 4 waves owns 64*WR rows x BN probe columns; each
// wave owns WR slabs of 16 rows.  K is walked in chunks whose V_k rows and A
// values are loaded straight into LDS three chunks ahead (see
// dense_step_tile).  Row/column padding of the V buffers is zero, so a
// ragged end of K needs no masking of V.
//
// Split-K: when the tile grid is smaller than the chip (n = 4096 with 64
// probes has 64 tiles), each workgroup sums one range of columns into a
// partial block and dense_split_epilogue_kernel adds the partials in split
// order and applies the epilogue, with dot partials per 16 rows.
#include "device_common.hpp"
#include "kernels.hpp"

namespace ent {

// s_waitcnt vmcnt(N) in the gfx9 encoding, expcnt and lgkmcnt left free.
template <int N>
__device__ __forceinline__ void dense_wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// Chunk geometry of the dense step: BK columns of R per chunk (32, 16 or 8),
// KPL = BK/4 of them per lane; one stage holds the chunk's V_k rows (BK x BN,
// shared by the 4 waves) and each wave's A values (WR 16-row slabs x BK); the
// NST stages take at most 60 KB, so two workgroups fit on a CU.
template <typename T, int BN, int WR>
struct DenseChunk {
  static constexpr int NST = 3;                      // stages (prefetch distance NST - 1)
  static constexpr int BUDGET = 61440;
  static_assert(NST >= 3 && NST <= 4, "the waits cover three or four stages");
  static constexpr int ES = (int)sizeof(T);
  static constexpr int VEC = 16 / ES;                // elements per 16-byte piece
  static constexpr int RB = BN * ES;                 // bytes per V row
  static constexpr int stage_bytes(int bk) { return bk * RB + 64 * WR * bk * ES; }
  static constexpr int BK = (NST * stage_bytes(32) <= BUDGET) ? 32
                          : (NST * stage_bytes(16) <= BUDGET || 2 * ES < 16) ? 16 : 8;
  static constexpr int KPL = BK / 4;                 // k values per lane per chunk
  static constexpr int G = RB / 16;                  // 16-byte groups per V row
  static constexpr int VBYTES = BK * RB;
  static constexpr int NVL = BK * G / 256;           // V pieces per wave (direct loads)
  static constexpr int APL = KPL / VEC;              // A pieces per lane and slab
  static constexpr int NAL = WR * APL;               // A direct loads per wave
  static constexpr int ABYTES = 4 * NAL * 1024;      // A of the 4 waves
  static_assert(KPL % VEC == 0, "a lane's A values must be whole 16-byte pieces");
  static_assert((BK * G) % 256 == 0, "V pieces must split over the 4 waves");
  static_assert(4 * ES <= G, "V rows too short for the swizzle");
  // V row r sits at r * RB bytes, its 16-byte groups XOR-swizzled so that
  // the four 16-lane groups of an MFMA B-operand read (rows t, KPL+t, 2KPL+t,
  // 3KPL+t, 16 consecutive probes each) fall on disjoint banks
  __device__ static constexpr int swz(int r) { return ((r / KPL) & 3) * ES; }
  __device__ static int voff(int r, int col) {
    return r * RB + (((col / VEC) ^ swz(r)) << 4) + (col % VEC) * ES;
  }
};

// Body of one tile: rows [64*WR*tm, +64*WR) (wave w owns WR 16-row slabs),
// probe columns [BN*tn, +BN), product columns [kbeg, kend) (kbeg a multiple
// of 32; kend a multiple of 32 or >= n).  Shared by the single-matrix kernel
// and the grouped (batched) kernel.  With yout the raw products go to
// yout[row][ldv] (every row of the tile) instead of the epilogue.
//
// Pipeline over chunks of BK columns, three stages deep: the chunk's V_k rows
// and each wave's A values go from global memory straight into LDS (direct
// loads, no registers), two chunks ahead of the MFMAs that read them; every
// wait on them is explicit (vmcnt), one barrier per chunk.  Lane (m, q) of a
// wave loads R[row m][k0 + KPL q .. + KPL) of each of its slabs, which it
// reads back from its own 16-byte slots: MFMA k-slot q of call t is column
// KPL q + t (the k order inside a chunk is permuted consistently for A and
// B).  A ragged last chunk (n not a multiple of BK) reads A into registers,
// column min(k, n - 1) element by element: V_k is zero in rows k >= n, so
// those products vanish.
template <typename T, int BN, int WR>
__device__ __forceinline__ void dense_step_tile(const DenseStepArgs &a, int tm, int tn, int64_t kbeg,
                                                int64_t kend, T *yout) {
  using M = Mfma16<T>;
  using v4 = typename M::v4;
  using C = DenseChunk<T, BN, WR>;
  constexpr int BM = 64 * WR, BK = C::BK, KPL = C::KPL, VEC = C::VEC;
  constexpr int NSUB = BN / 16;
  constexpr int NVL = C::NVL, NAL = C::NAL, APL = C::APL;
  typedef T vec_t __attribute__((ext_vector_type(VEC)));

  // stage s at lds + s * STAGE: the V_k chunk (VBYTES), then the A values of
  // the 4 waves (ABYTES)
  constexpr int STAGE = C::VBYTES + C::ABYTES, NST = C::NST;
  // one LDS array (the epilogue's per-wave dot sums reuse it after the
  // products): with a single LDS object the compiler adds no waits of its own
  // between the direct loads into one stage and the reads of another
  static_assert(NST * STAGE >= 2 * 4 * BN * 8, "the dot sums fit in the stages");
  __shared__ __attribute__((aligned(1024))) unsigned char lds[NST * STAGE];
  double(*red)[4][BN] = (double(*)[4][BN])lds;

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = a.n, ldv = a.ldv;
  const T *__restrict__ R = (const T *)a.R;
  const T *__restrict__ Vk = (const T *)a.Vk;
  const int64_t col0 = (int64_t)tn * BN;
  const int m16 = lane & 15, kq = lane >> 4;
  const int64_t wrow0 = (int64_t)tm * BM + 16 * WR * w;  // first row of this wave
  // rows beyond n read row n - 1: their products are discarded (zeroed in the
  // epilogue and in yout)
  const T *Arow[WR];
#pragma unroll
  for (int f = 0; f < WR; ++f) {
    const int64_t arow = wrow0 + 16 * f + m16;
    Arow[f] = R + (arow < n ? arow : n - 1) * a.ldr + KPL * kq;
  }
  // V piece q = (i*4 + w)*64 + lane of a chunk: row q / G, swizzled group q % G
  int64_t vsrc[NVL];
#pragma unroll
  for (int i = 0; i < NVL; ++i) {
    const int q = (i * 4 + w) * 64 + lane;
    const int r = q / C::G, gs = q % C::G;
    vsrc[i] = (int64_t)r * ldv + col0 + (int64_t)(gs ^ C::swz(r)) * VEC;
  }

  const int nfull = (int)((kend - kbeg) / BK);
  const bool ragged = kbeg + (int64_t)nfull * BK < kend;

  using LdsPtr = __attribute__((address_space(3))) void *;
  auto issue_v = [&](int c, unsigned char *st) {
    const T *vb = Vk + (kbeg + (int64_t)c * BK) * ldv;
#pragma unroll
    for (int i = 0; i < NVL; ++i)
      __builtin_amdgcn_global_load_lds((const void *)(vb + vsrc[i]), (LdsPtr)(st + (i * 4 + w) * 1024), 16, 0, 0);
  };
  auto issue = [&](int c, unsigned char *st) {
    issue_v(c, st);
    const int64_t kc = kbeg + (int64_t)c * BK;
#pragma unroll
    for (int f = 0; f < WR; ++f)
#pragma unroll
      for (int h = 0; h < APL; ++h)
        __builtin_amdgcn_global_load_lds((const void *)(Arow[f] + kc + h * VEC),
                                         (LdsPtr)(st + C::VBYTES + ((w * WR + f) * APL + h) * 1024), 16, 0, 0);
  };

  v4 acc[WR][NSUB];
#pragma unroll
  for (int f = 0; f < WR; ++f)
#pragma unroll
    for (int c = 0; c < NSUB; ++c) acc[f][c] = v4{0, 0, 0, 0};

  // operands of one chunk in registers: this lane's A values (APL 16-byte
  // pieces per slab) and B values (KPL x NSUB)
  struct Frag {
    vec_t a[WR][APL];
    T b[KPL][NSUB];
  };
  auto read_frag = [&](Frag &fr, const unsigned char *st) {
#pragma unroll
    for (int f = 0; f < WR; ++f)
#pragma unroll
      for (int h = 0; h < APL; ++h)
        fr.a[f][h] = *(const vec_t *)(st + C::VBYTES + ((w * WR + f) * APL + h) * 1024 + 16 * lane);
#pragma unroll
    for (int t = 0; t < KPL; ++t)
#pragma unroll
      for (int c2 = 0; c2 < NSUB; ++c2) fr.b[t][c2] = *(const T *)(st + C::voff(KPL * kq + t, 16 * c2 + m16));
  };
  auto mfma_frag = [&](const Frag &fr) {
#pragma unroll
    for (int t = 0; t < KPL; ++t)
#pragma unroll
      for (int c2 = 0; c2 < NSUB; ++c2)
#pragma unroll
        for (int f = 0; f < WR; ++f) acc[f][c2] = M::mma(fr.a[f][t / VEC][t % VEC], fr.b[t][c2], acc[f][c2]);
  };

  // Chunk j is loaded into stage j % NST at step j - NST (direct loads) and
  // read into registers at step j - 1, after that step's barrier; step j
  // multiplies it.  Step c: wait until this wave's loads of chunk c + 1 have
  // landed and its reads of chunk c have returned, barrier (every wave's part
  // of chunk c + 1 landed; every wave done reading chunk c, whose stage chunk
  // c + NST now takes), issue chunk c + NST, read chunk c + 1, multiply chunk c.
  constexpr int PER = NVL + NAL;  // direct loads per wave per chunk
  for (int c = 0; c < NST; ++c)
    if (c < nfull) issue(c, lds + c * STAGE);
  Frag fx, fy;
  // wait until at most k chunks' loads of this wave are in flight (k < NST)
  auto wait_chunks = [&](int k) {
    if (NST >= 4 && k >= 3)
      dense_wait_vm<(NST >= 4 ? 3 : 0) * PER>();
    else if (k >= 2)
      dense_wait_vm<2 * PER>();
    else if (k >= 1)
      dense_wait_vm<PER>();
    else
      dense_wait_vm<0>();
  };
  auto step = [&](int c, int s0, Frag &cur, Frag &nxt) {
    // chunks issued after chunk c + 1: c + 2 .. min(c + NST - 1, nfull - 1)
    const int ahead = nfull - 2 - c < NST - 2 ? nfull - 2 - c : NST - 2;
    wait_chunks(ahead);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's reads of chunk c returned
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if (c + NST < nfull) issue(c + NST, lds + s0 * STAGE);
    if (c + 1 < nfull) read_frag(nxt, lds + (s0 == NST - 1 ? 0 : s0 + 1) * STAGE);
    mfma_frag(cur);
  };
  if (nfull > 0) {
    wait_chunks(nfull - 1 < NST - 1 ? nfull - 1 : NST - 1);  // chunk 0 landed
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    read_frag(fx, lds);
  }
  int c = 0, s0 = 0;
  for (; c + 1 < nfull; c += 2) {
    step(c, s0, fx, fy);
    s0 = s0 == NST - 1 ? 0 : s0 + 1;
    step(c + 1, s0, fy, fx);
    s0 = s0 == NST - 1 ? 0 : s0 + 1;
  }
  if (c < nfull) {
    step(c, s0, fx, fy);
    s0 = s0 == NST - 1 ? 0 : s0 + 1;
  }
  if (ragged) {
    // the stage this chunk takes (s0) was last read at step nfull - NST - 1,
    // before barriers every wave has passed; its A values come into
    // registers element by element, column min(k, n - 1)
    unsigned char *st = lds + s0 * STAGE;
    dense_wait_vm<0>();
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    issue_v(nfull, st);
    const int64_t k0 = kbeg + (int64_t)nfull * BK + KPL * kq;
    Frag fr;
#pragma unroll
    for (int f = 0; f < WR; ++f)
#pragma unroll
      for (int t = 0; t < KPL; ++t) fr.a[f][t / VEC][t % VEC] = (Arow[f] - KPL * kq)[k0 + t < n ? k0 + t : n - 1];
    dense_wait_vm<0>();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < KPL; ++t)
#pragma unroll
      for (int c2 = 0; c2 < NSUB; ++c2) fr.b[t][c2] = *(const T *)(st + C::voff(KPL * kq + t, 16 * c2 + m16));
    mfma_frag(fr);
  }
  __syncthreads();

  if (yout) {
#pragma unroll
    for (int c = 0; c < NSUB; ++c)
#pragma unroll
      for (int f = 0; f < WR; ++f)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = wrow0 + 16 * f + M::drow(kq, r);
          yout[row * ldv + col0 + 16 * c + m16] = row < n ? acc[f][c][r] : T(0);
        }
    return;
  }
  // ---- epilogue ----
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const T *Vkm1 = (const T *)a.Vkm1;
  const T *__restrict__ G = (const T *)a.G;
  T *Vkp1 = (T *)a.Vkp1;
  const bool use_m1 = (a.cw != 0.0) && Vkm1;
  const bool want_dot = a.slot >= 0;
  const bool want_gg = a.slot_gg >= 0;
  const bool use_cg = a.cg != nullptr;
  const T tcg = use_cg ? (T)a.cg[0] : T(0);
#pragma unroll
  for (int c = 0; c < NSUB; ++c) {
    const int64_t col = col0 + 16 * c + m16;
    double ds = 0.0, gs = 0.0;
#pragma unroll
    for (int f = 0; f < WR; ++f)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = wrow0 + 16 * f + M::drow(kq, r);
      const int64_t off = row * ldv + col;
      const T y = row < n ? ta * acc[f][c][r] : T(0);
      T z = tc1 * y + tb * Vk[off];
      if (use_m1) z += tcw * Vkm1[off];
      if (use_cg) z += tcg * G[off];
      if (Vkp1) Vkp1[off] = z;
      if (want_dot) {
        const T g = G[off];
        ds += (double)g * (double)(a.dot_y ? y : z);
        if (want_gg) gs += (double)g * (double)g;
      }
    }
    ds += __shfl_xor(ds, 16, 64);
    ds += __shfl_xor(ds, 32, 64);
    gs += __shfl_xor(gs, 16, 64);
    gs += __shfl_xor(gs, 32, 64);
    if (kq == 0) {
      red[0][w][16 * c + m16] = ds;
      red[1][w][16 * c + m16] = gs;
    }
  }
  if (!want_dot) return;
  __syncthreads();
  for (int col = tid; col < BN; col += 256) {
    const double s = red[0][0][col] + red[0][1][col] + red[0][2][col] + red[0][3][col];
    a.part[((int64_t)a.slot * a.ntile + tm) * ldv + col0 + col] = s;
    if (want_gg) {
      const double g2 = red[1][0][col] + red[1][1][col] + red[1][2][col] + red[1][3][col];
      a.part[((int64_t)a.slot_gg * a.ntile + tm) * ldv + col0 + col] = g2;
    }
  }
}

template <typename T, int BN, int WR>
__global__ __launch_bounds__(256) void dense_step_kernel(DenseStepArgs a) {
  const int ntn = (int)(a.ldv / BN);
  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  dense_step_tile<T, BN, WR>(a, b / ntn, b % ntn, 0, a.n, nullptr);
}

// Split-K product (a kernel of its own, so the fused kernel's code is not
// shaped by this path): tile order row tile fastest within a K-split, so the
// tiles of one split (same V_k rows) are neighbours.
template <typename T, int BN, int WR>
__global__ __launch_bounds__(256) void dense_step_split_kernel(DenseStepArgs a) {
  const int ntn = (int)(a.ldv / BN);
  const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const int ntl = a.ntile * ntn;
  const int ks = b / ntl, t = b % ntl;
  const int64_t kbeg = (int64_t)ks * a.kper;
  const int64_t kend = kbeg + a.kper < a.n ? kbeg + a.kper : a.n;
  T *yout = (T *)a.party + (int64_t)ks * (int64_t)a.ntile * 64 * a.ldv;
  dense_step_tile<T, BN, WR>(a, t / ntn, t % ntn, kbeg, kend, yout);
}

// Split-K epilogue: y = a sum_ks party[ks] (split order), z = c1 y + c2 b V_k
// + cw V_{k-1} (+ cg g), V_{k+1} = z, and the per-probe dots over each
// 16-row tile (part is [slot][nptile][ldv]).  Workgroup = (16 rows, 64
// probes); thread = one probe of 4 rows, its loads of every split issued
// together.
template <typename T>
__global__ __launch_bounds__(256) void dense_split_epilogue_kernel(DenseStepArgs a) {
  __shared__ double red[2][4][64];
  const int tp = blockIdx.x, tid = threadIdx.x, pl = tid & 63, rq = tid >> 6;
  const int64_t ldv = a.ldv, col = (int64_t)blockIdx.y * 64 + pl;
  const int64_t pstride = (int64_t)a.ntile * 64 * ldv;
  const T *P = (const T *)a.party;
  const T *Vk = (const T *)a.Vk, *Vkm1 = (const T *)a.Vkm1, *G = (const T *)a.G;
  T *Vkp1 = (T *)a.Vkp1;
  const T ta = (T)a.scal[S_A];
  const T tb = (T)(a.c2 * a.scal[S_B]);
  const T tc1 = (T)a.c1, tcw = (T)a.cw;
  const bool use_m1 = (a.cw != 0.0) && Vkm1;
  const bool want_dot = a.slot >= 0, want_gg = a.slot_gg >= 0;
  const bool use_cg = a.cg != nullptr;
  const T tcg = use_cg ? (T)a.cg[0] : T(0);
  int64_t off[4];
  T acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    off[i] = ((int64_t)tp * 16 + rq * 4 + i) * ldv + col;
    acc[i] = T(0);
  }
  for (int ks = 0; ks < a.ksplit; ++ks) {
    T pv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pv[i] = P[ks * pstride + off[i]];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += pv[i];
  }
  double ds = 0.0, gs = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T y = ta * acc[i];
    T z = tc1 * y + tb * Vk[off[i]];
    if (use_m1) z += tcw * Vkm1[off[i]];
    if (use_cg) z += tcg * G[off[i]];
    if (Vkp1) Vkp1[off[i]] = z;
    if (want_dot) {
      const T g = G[off[i]];
      ds += (double)g * (double)(a.dot_y ? y : z);
      if (want_gg) gs += (double)g * (double)g;
    }
  }
  if (!want_dot) return;
  red[0][rq][pl] = ds;
  red[1][rq][pl] = gs;
  __syncthreads();
  if (rq == 0) {
    const double s0 = red[0][0][pl] + red[0][1][pl] + red[0][2][pl] + red[0][3][pl];
    a.part[((int64_t)a.slot * a.nptile + tp) * ldv + col] = s0;
    if (want_gg) {
      const double s1 = red[1][0][pl] + red[1][1][pl] + red[1][2][pl] + red[1][3][pl];
      a.part[((int64_t)a.slot_gg * a.nptile + tp) * ldv + col] = s1;
    }
  }
}

int32_t dense_step_splits(int64_t n, int32_t ntile, int64_t ldv, int32_t bn) {
  const int64_t tiles = (int64_t)ntile * (ldv / bn);
  int32_t ks = 1;
  while (tiles * ks < 512 && ks < 16 && n / (2 * ks) >= 256) ks *= 2;
  return ks;
}

// Grouped step over a batch: block -> (matrix, row tile) from the tile table;
// the batch base pointers are offset by the matrix's region.
template <typename T, int BN, int WR>
__global__ __launch_bounds__(256) void batch_dense_step_kernel(BatchStepArgs ba) {
  const int2 tl = ba.tiles[blockIdx.x];
  const BatchMat &M = ba.mats[tl.x];
  DenseStepArgs a = ba.base;
  a.R = M.R;
  a.ldr = M.ldr;
  a.n = M.n;
  a.Vk = (const T *)ba.base.Vk + M.voff;
  if (ba.base.Vkm1) a.Vkm1 = (const T *)ba.base.Vkm1 + M.voff;
  if (ba.base.Vkp1) a.Vkp1 = (T *)ba.base.Vkp1 + M.voff;
  a.G = (const T *)ba.base.G + M.voff;
  a.part = ba.base.part + M.poff;
  a.ntile = M.ntile;
  a.scal = M.scal;
  dense_step_tile<T, BN, WR>(a, tl.y, 0, 0, a.n, nullptr);
}

// Persistent batch steps: each workgroup takes (matrix, row tile, step)
// items in schedule order, waits for the matrix's previous step, runs the
// tile body of the grouped kernel with that step's recurrence, publishes it.
template <typename T, int WR>
__global__ __launch_bounds__(256) void batch_dense_persistent_kernel(BatchPersistArgs pa) {
  __shared__ int sh;
  for (;;) {
    const int i = sched_next(pa.sched, &sh);
    if (i < 0) return;
    const int4 it = pa.sched.items[i];
    const BatchMat &M = pa.mats[it.x];
    if (!sched_wait(pa.sched, it.x, it.z * M.ntile, &sh)) return;
    const StepRule r = step_rule(pa.method, it.z, pa.nsteps);
    const T *bufs[3] = {(const T *)pa.G + M.voff, (const T *)pa.VA + M.voff, (const T *)pa.VB + M.voff};
    DenseStepArgs a{};
    a.R = M.R;
    a.ldr = M.ldr;
    a.n = M.n;
    a.ldv = pa.ldv;
    a.Vk = bufs[r.vk];
    a.Vkm1 = r.vkm1 >= 0 ? bufs[r.vkm1] : nullptr;
    a.Vkp1 = r.vout >= 0 ? (void *)bufs[r.vout] : nullptr;
    a.G = bufs[0];
    a.scal = M.scal;
    a.c1 = r.c1; a.c2 = r.c2; a.cw = r.cw;
    a.dot_y = r.dot_y; a.slot = r.slot; a.slot_gg = r.slot_gg;
    a.part = pa.part + M.poff;
    a.ntile = M.ntile;
    a.bn = 64;
    dense_step_tile<T, 64, WR>(a, it.y, 0, 0, a.n, nullptr);
    sched_release(pa.sched, it.x);
  }
}

template <typename T>
hipError_t launch_batch_dense_persistent(const BatchPersistArgs &pa, int32_t wr, int32_t grid,
                                         hipStream_t st) {
  if (pa.ldv != 64 || grid < 1) return hipErrorInvalidValue;
  if (wr == 1)
    batch_dense_persistent_kernel<T, 1><<<(unsigned)grid, 256, 0, st>>>(pa);
  else if (wr == 2)
    batch_dense_persistent_kernel<T, 2><<<(unsigned)grid, 256, 0, st>>>(pa);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_batch_dense_persistent<double>(const BatchPersistArgs &, int32_t, int32_t, hipStream_t);
template hipError_t launch_batch_dense_persistent<float>(const BatchPersistArgs &, int32_t, int32_t, hipStream_t);

// Resident workgroups of the persistent step kernels (CUs x occupancy).
int32_t batch_persistent_grid(int32_t precision, int32_t wr, int64_t ldv) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = hipErrorInvalidValue;
  if (precision == 0)
    e = wr == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_dense_persistent_kernel<double, 2>, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_dense_persistent_kernel<double, 1>, 256, 0);
  else if (precision == 1)
    e = wr == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_dense_persistent_kernel<float, 2>, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_dense_persistent_kernel<float, 1>, 256, 0);
  else
    return bf16x3_persistent_grid(ldv);
  if (e != hipSuccess) return 0;
  return cus * (per > 0 ? per : 1);
}

template <typename T>
hipError_t launch_dense_split_epilogue(const DenseStepArgs &a, hipStream_t st) {
  if (a.ksplit < 2 || !a.party || a.nptile != a.ntile * 4) return hipErrorInvalidValue;
  dense_split_epilogue_kernel<T><<<dim3((unsigned)a.nptile, (unsigned)(a.ldv / 64)), 256, 0, st>>>(a);
  return hipGetLastError();
}
template hipError_t launch_dense_split_epilogue<double>(const DenseStepArgs &, hipStream_t);
template hipError_t launch_dense_split_epilogue<float>(const DenseStepArgs &, hipStream_t);

template <typename T>
hipError_t launch_dense_step(const DenseStepArgs &a, hipStream_t st, bool epilogue) {
  const int ntn = (int)(a.ldv / a.bn);
  if (a.ksplit > 1 && (!a.party || a.kper % 32 != 0 || (int64_t)a.ksplit * a.kper < a.n ||
                       a.nptile != a.ntile * 4))
    return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(a.ntile * ntn * (a.ksplit > 1 ? a.ksplit : 1));
  if (a.ksplit > 1) {
    switch (a.bn) {
      case 64: dense_step_split_kernel<T, 64, 1><<<grid, 256, 0, st>>>(a); break;
      case 128: dense_step_split_kernel<T, 128, 1><<<grid, 256, 0, st>>>(a); break;
      case 256: dense_step_split_kernel<T, 256, 1><<<grid, 256, 0, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (a.bn) {
      case 64: dense_step_kernel<T, 64, 1><<<grid, 256, 0, st>>>(a); break;
      case 128: dense_step_kernel<T, 128, 1><<<grid, 256, 0, st>>>(a); break;
      case 256: dense_step_kernel<T, 256, 1><<<grid, 256, 0, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (a.ksplit > 1 && epilogue) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_dense_split_epilogue<T>(a, st);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_dense_step(const BatchStepArgs &ba, int32_t ntiles, int32_t wr,
                                   hipStream_t st) {
  if (ba.base.bn != 64) return hipErrorInvalidValue;
  if (wr == 1)
    batch_dense_step_kernel<T, 64, 1><<<(unsigned)ntiles, 256, 0, st>>>(ba);
  else if (wr == 2)
    batch_dense_step_kernel<T, 64, 2><<<(unsigned)ntiles, 256, 0, st>>>(ba);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template hipError_t launch_batch_dense_step<double>(const BatchStepArgs &, int32_t, int32_t, hipStream_t);
template hipError_t launch_batch_dense_step<float>(const BatchStepArgs &, int32_t, int32_t, hipStream_t);
template hipError_t launch_dense_step<double>(const DenseStepArgs &, hipStream_t, bool);
template hipError_t launch_dense_step<float>(const DenseStepArgs &, hipStream_t, bool);

}  // namespace ent
