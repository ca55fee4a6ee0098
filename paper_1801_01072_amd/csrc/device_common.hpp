// device_common.hpp -- device-side helpers shared by the gfx950 kernels of
// libentropy: the Philox4x32-10 counter generator and the probe mapping,
// wave64 reductions and MFMA wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace ent {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten S-box rounds over a
// 128-bit counter; the 64-bit key is advanced by the two Weyl constants
// between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    U4 n;
    n.x = hi1 ^ c.y ^ k0;
    n.y = lo1;
    n.z = hi0 ^ c.w ^ k1;
    n.w = lo0;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Counter layout: (row mod 2^32, block, stream, row >> 32); key = seed.
__device__ __forceinline__ U4 philox_block(uint64_t seed, uint32_t stream, int64_t row,
                                           uint32_t block) {
  U4 c;
  c.x = (uint32_t)((uint64_t)row & 0xffffffffu);
  c.y = block;
  c.z = stream;
  c.w = (uint32_t)((uint64_t)row >> 32);
  return philox10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
}

// 32 Rademacher signs of probes [32*word, 32*word+32) of one row, as a bit
// mask: bit b set means probe 32*word+b is -1.  One Philox block serves 128
// probes: block = probe >> 7, word index (probe >> 5) & 3.
__device__ __forceinline__ uint32_t rademacher_word(uint64_t seed, uint32_t stream, int64_t row,
                                                    int32_t word) {
  const U4 o = philox_block(seed, stream, row, (uint32_t)word >> 2);
  switch (word & 3) {
    case 0: return o.x;
    case 1: return o.y;
    case 2: return o.z;
    default: return o.w;
  }
}

__device__ __forceinline__ double rademacher(uint64_t seed, uint32_t stream, int64_t row,
                                             int64_t probe) {
  const uint32_t w = rademacher_word(seed, stream, row, (int32_t)(probe >> 5));
  return ((w >> (probe & 31)) & 1u) ? -1.0 : 1.0;
}

// Standard Gaussian by Box-Muller on two 53-bit uniforms of one Philox block
// (block = probe >> 1); even probes take the cosine branch, odd the sine.
__device__ __forceinline__ double gaussian(uint64_t seed, uint32_t stream, int64_t row,
                                           int64_t probe) {
  const U4 o = philox_block(seed, stream, row, (uint32_t)((uint64_t)probe >> 1));
  const uint64_t a = ((((uint64_t)o.y) << 32) | o.x) >> 11;
  const uint64_t b = ((((uint64_t)o.w) << 32) | o.z) >> 11;
  const double u1 = ((double)a + 1.0) * 0x1.0p-53;
  const double u2 = (double)b * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586476925286766559 * u2;
  return (probe & 1) ? r * sin(th) : r * cos(th);
}

// Structured sketches of the random projection (Section 5.2).  Row sign
// D_jj = -1 iff bit 0 of word x of stream 3's block (row j, block 0); the
// input-sparsity bucket of row j is floor(word y * s / 2^32) of the same
// block; the t-th sampled Hadamard column is word x of stream 4's block
// (row t) modulo N, N = 2^ceil(log2 n).
__device__ __forceinline__ double sketch_sign(uint64_t seed, int64_t j) {
  return (philox_block(seed, 3u, j, 0u).x & 1u) ? -1.0 : 1.0;
}
__device__ __forceinline__ int32_t sketch_bucket(uint64_t seed, int64_t j, int32_t s) {
  return (int32_t)(((uint64_t)philox_block(seed, 3u, j, 0u).y * (uint64_t)s) >> 32);
}
__device__ __forceinline__ int64_t hadamard_order(int64_t n) {
  int64_t N = 1;
  while (N < n) N <<= 1;
  return N;
}
// Entry (j, t) of D H S without the 1/sqrt(s) scale: D_jj (-1)^popcount(j & i_t).
__device__ __forceinline__ double srht_entry(uint64_t seed, int64_t j, int64_t t, int64_t N) {
  const int64_t col = (int64_t)((uint64_t)philox_block(seed, 4u, t, 0u).x % (uint64_t)N);
  return (__popcll((unsigned long long)(j & col)) & 1) ? -sketch_sign(seed, j) : sketch_sign(seed, j);
}

// ---------------------------------------------------------------------------
// wave64 reductions (fixed butterfly order: deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// MFMA 16x16x4 for FP64 and FP32.  Operand layout (per lane l of the wave):
//   A: row l%16, k-slot l/16      B: k-slot l/16, column l%16
//   D register r (r = 0..3), column l%16, row:
//     FP32: 4*(l/16) + r      FP64: (l/16) + 4*r
// (measured on gfx950 with a one-wave layout probe against a host product).
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma16;

template <>
struct Mfma16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int drow(int q, int r) { return q + 4 * r; }
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int drow(int q, int r) { return 4 * q + r; }
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// XCD-aware remap of a linear workgroup id: the hardware deals consecutive
// ids round-robin over the 8 XCDs; this gives each XCD a contiguous range of
// logical tiles so that tiles sharing operands share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Block sums of y^2, xs.y, xs^2 over the rows a block produced (fixed order).
__device__ __forceinline__ void block_power_partials(double yy, double xy, double xx,
                                                     double *part3, int64_t blk) {
  __shared__ double red[3][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  yy = wave_sum(yy);
  xy = wave_sum(xy);
  xx = wave_sum(xx);
  if (lane == 0) {
    red[0][w] = yy;
    red[1][w] = xy;
    red[2][w] = xx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < nw; ++i) {
      a += red[0][i];
      b += red[1][i];
      c += red[2][i];
    }
    part3[3 * blk + 0] = a;
    part3[3 * blk + 1] = b;
    part3[3 * blk + 2] = c;
  }
}

// ---------------------------------------------------------------------------
// Persistent batch steps: taking items, waiting for a matrix's previous step,
// publishing a finished tile.  Items are taken from the segment of the XCD
// the workgroup runs on, and every item of a matrix runs on the same XCD, so
// a tile's stores reach the only L2 its consumers read through: publishing
// waits until this workgroup's stores are performed (vmcnt), then one thread
// moves the counter; waiting polls the counter, then invalidates at device
// scope, which drops this CU's L1 (lines that another CU of the XCD has since
// rewritten in L2) and never loses a dirty L2 line.  No L2 write-back is
// needed.  Counters are vector atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kMaxXcc - 1));  // HW_REG_XCC_ID[3:0]
}

// Next item index of this workgroup, or -1 when its XCD's segment is
// exhausted or a wait has failed.  sh: a __shared__ int of the calling kernel.
__device__ __forceinline__ int sched_next(const SchedArgs &s, int *sh) {
  __syncthreads();  // every wave is done with the previous item (and with sh)
  if (threadIdx.x == 0) {
    int i = -1;
    const int seg = s.seg_of_xcc[xcc_id()];
    if (seg >= 0) {
      const int q = __hip_atomic_fetch_add(s.head + seg, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (q < s.seg_off[seg + 1] - s.seg_off[seg] &&
          __hip_atomic_fetch_add(s.err, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        i = s.seg_off[seg] + q;
    }
    *sh = i;
  }
  __syncthreads();
  return *sh;
}

// Waits until done[b] >= need; false (and *err set) after spin_limit polls.
__device__ __forceinline__ bool sched_wait(const SchedArgs &s, int b, int need, int *sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    int polls = 0;
    while (__hip_atomic_fetch_add(s.done + b, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (__hip_atomic_fetch_add(s.err, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          polls++ >= s.spin_limit) {
        __hip_atomic_fetch_or(s.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    *sh = ok;
  }
  __syncthreads();
  asm volatile("buffer_inv sc1" ::: "memory");  // L1 of this CU (device scope: a group-scope invalidate may keep it)
  return *sh != 0;
}

// Publishes one finished tile of matrix b.
__device__ __forceinline__ void sched_release(const SchedArgs &s, int b) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores of the tile are performed in L2
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(s.done + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Recurrence of step k (the host's per-step launches use the same rule):
// Chebyshev forward: V_1 = Y_0 - V_0 (dot slot 1, g.g in slot 0), then
// V_{k+1} = 2 Y_k - 2 V_k - V_{k-1} written over V_{k-1}; Taylor: W_{k+1} =
// W_k - Y_k into alternating buffers, dots with Y_k in slot k, the last step
// writes nothing.  V_0 is the probe block.
struct StepRule {
  double c1, c2, cw;
  int32_t dot_y, slot, slot_gg;
  int vk, vkm1, vout;  // buffer ids: 0 = probe block, 1 = VA, 2 = VB, -1 = none
};
__device__ __forceinline__ StepRule step_rule(int32_t method, int32_t k, int32_t nsteps) {
  StepRule r;
  const int out = 1 + (k & 1), prev = 1 + ((k - 1) & 1);
  if (method == 1) {  // Chebyshev
    r.dot_y = 0;
    r.slot = k + 1;
    if (k == 0) {
      r.c1 = 1.0; r.c2 = -1.0; r.cw = 0.0; r.slot_gg = 0;
      r.vk = 0; r.vkm1 = -1;
    } else {
      r.c1 = 2.0; r.c2 = -2.0; r.cw = -1.0; r.slot_gg = -1;
      r.vk = prev; r.vkm1 = k == 1 ? 0 : out;
    }
    r.vout = out;
  } else {  // Taylor
    r.c1 = -1.0; r.c2 = 1.0; r.cw = 0.0;
    r.dot_y = 1; r.slot = k; r.slot_gg = -1;
    r.vk = k == 0 ? 0 : prev;
    r.vkm1 = -1;
    r.vout = k < nsteps - 1 ? out : -1;
  }
  return r;
}

}  // namespace ent
