// engine.cpp -- C ABI of libentropy: argument validation, workspace, and the
// launch sequence of one estimate (power method -> interval and coefficients
// -> m recurrence steps -> reductions), all enqueued on the caller's stream
// with a single synchronisation at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/entropy.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_last_error;
thread_local bool g_timing_on = false;
thread_local ent_timing g_last_timing = {};

// Events recorded between launches when timing is enabled on this thread.
struct PhaseEvents {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev;
  int power_begin = -1, power_end = -1, steps_begin = -1, steps_end = -1;
  int32_t power_launches = 0;
  int32_t csr_band = 0;  // padded half-bandwidth of the banded CSR step (0: none)
  int32_t logical_steps = 0;  // > 0: the steps span holds this many steps in one launch
  int32_t steps_fused = 1;    // recurrence steps per product launch
  // split steps (product kernel + separate epilogue kernel): event index
  // pairs of the product launches and of the epilogue launches
  std::vector<std::pair<int, int>> main_spans, epi_spans;
  ~PhaseEvents() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  int mark() {
    if (!on) return -1;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      on = false;
      return -1;
    }
    (void)hipEventRecord(e, st);
    ev.push_back(e);
    return (int)ev.size() - 1;
  }
  float between(int a, int b) const {
    float ms = 0.f;
    if (a < 0 || b < 0) return 0.f;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms;
  }
  void finish() {
    if (!on || ev.size() < 2) return;
    ent_timing t{};
    t.total_ms = between(0, (int)ev.size() - 1);
    t.power_ms = between(power_begin, power_end);
    if (main_spans.empty()) {
      t.step_launches = logical_steps > 0 ? logical_steps : steps_end - steps_begin;
      for (int i = steps_begin; i >= 0 && i < steps_end; ++i) {
        const double d = between(i, i + 1);
        t.steps_ms += d;
        if (d > t.step_max_ms) t.step_max_ms = d;
      }
      if (logical_steps > 0) t.step_max_ms = t.steps_ms / logical_steps;
    } else {
      t.step_launches = (int32_t)main_spans.size();
      for (auto &sp : main_spans) {
        const double d = between(sp.first, sp.second);
        t.steps_ms += d;
        if (d > t.step_max_ms) t.step_max_ms = d;
      }
      for (auto &sp : epi_spans) t.epilogue_ms += between(sp.first, sp.second);
      t.epilogue_launches = (int32_t)epi_spans.size();
    }
    t.other_ms = t.total_ms - t.power_ms - t.steps_ms - t.epilogue_ms;
    t.power_launches = power_launches;
    t.csr_band = csr_band;
    t.steps_fused = steps_fused;
    g_last_timing = t;
  }
};

// The banded FP32 two-step launches are on unless the environment variable
// named (ENT_BAND_PAIRS) is 0 (for timing comparisons).
bool step_pairs_enabled(const char *name) {
  const char *e = std::getenv(name);
  return !(e && e[0] == '0');
}

// Recurrence steps per tridiagonal launch: ENT_TRI_FUSE (1 = one step per
// launch, at most kTriMaxFuse), else the most.
constexpr int32_t kTriFuseDefault = ent::kTriMaxFuse;
int32_t tri_fuse_steps() {
  const char *e = std::getenv("ENT_TRI_FUSE");
  if (!e || !*e) return kTriFuseDefault;
  const int v = std::atoi(e);
  return v < 1 ? 1 : (v > ent::kTriMaxFuse ? ent::kTriMaxFuse : v);
}

// Split nsteps recurrence steps into launches of at most nf steps, as even
// as possible, longer launches first (a launch of one step runs the
// single-step kernel).
std::vector<int32_t> fuse_split(int32_t nsteps, int32_t nf) {
  std::vector<int32_t> sizes;
  if (nsteps <= 0) return sizes;
  const int32_t nl = (nsteps + nf - 1) / nf;
  for (int32_t i = 0; i < nl; ++i) sizes.push_back(nsteps / nl + (i < nsteps % nl ? 1 : 0));
  return sizes;
}

ent_status fail(ent_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ENT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------------------
// Workspace: one grow-only device buffer per device, held for the duration of
// a call (calls on one device are serialised on its mutex).
// ---------------------------------------------------------------------------
struct DeviceWorkspace {
  std::mutex mu;
  void *ptr = nullptr;
  size_t bytes = 0;
};

std::mutex g_ws_mu;
std::map<int, DeviceWorkspace *> g_ws;
std::atomic<size_t> g_ws_limit{0};

DeviceWorkspace *workspace_for(int dev) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) return it->second;
  auto *w = new DeviceWorkspace();
  g_ws[dev] = w;
  return w;
}

// Bump allocator over the workspace (256-byte aligned pieces).
struct Carve {
  size_t off = 0;
  std::vector<std::pair<void **, size_t>> items;
  template <typename T>
  void add(T **p, size_t count) {
    items.push_back({(void **)p, count * sizeof(T)});
  }
  size_t total() const {
    size_t t = 0;
    for (auto &it : items) t += (it.second + 255) & ~size_t(255);
    return t;
  }
  void assign(void *base) {
    size_t o = 0;
    for (auto &it : items) {
      *it.first = (char *)base + o;
      o += (it.second + 255) & ~size_t(255);
    }
  }
};

ent_status ensure_workspace(DeviceWorkspace *w, size_t need) {
  if (g_ws_limit && need > g_ws_limit)
    return fail(ENT_ENOMEM, "workspace of %zu bytes exceeds the limit of %zu bytes", need,
                g_ws_limit.load());
  if (w->bytes >= need) return ENT_OK;
  if (w->ptr) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(w->ptr));
    w->ptr = nullptr;
    w->bytes = 0;
  }
  hipError_t e = hipMalloc(&w->ptr, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    w->ptr = nullptr;
    return fail(ENT_ENOMEM, "hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
  }
  w->bytes = need;
  return ENT_OK;
}

// The 2n x 2n real form of a Hermitian R: one grow-only buffer per device,
// separate from the workspace (the estimate that runs on the real form
// carves the workspace from its start).
struct RealFormBuffer {
  std::mutex mu;
  void *ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_rf_mu;
std::map<int, RealFormBuffer *> g_rf;

RealFormBuffer *real_form_for(int dev) {
  std::lock_guard<std::mutex> lk(g_rf_mu);
  auto it = g_rf.find(dev);
  if (it != g_rf.end()) return it->second;
  auto *b = new RealFormBuffer();
  g_rf[dev] = b;
  return b;
}

// Device copies of matrices the caller passes in host memory: one grow-only
// buffer per device, held for the duration of the call that filled it.
struct StagingBuffer {
  std::mutex mu;
  void *ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_stage_mu;
std::map<int, StagingBuffer *> g_stage;

StagingBuffer *staging_for(int dev) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  auto it = g_stage.find(dev);
  if (it != g_stage.end()) return it->second;
  auto *b = new StagingBuffer();
  g_stage[dev] = b;
  return b;
}

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

constexpr int kScalarDoubles = 8192;

bool is_complex(const ent_matrix *R) {
  return R->dtype == ENT_STORE_C128 || R->dtype == ENT_STORE_C64;
}

// allow_complex: the entry point accepts Hermitian (complex) storage.
ent_status validate_matrix(const ent_matrix *R, bool allow_complex = false) {
  if (!R) return fail(ENT_EINVAL, "R is NULL");
  if (R->n < 1) return fail(ENT_EINVAL, "n = %lld < 1", (long long)R->n);
  if (R->n > (int64_t)INT32_MAX - 64)
    return fail(ENT_EINVAL, "n = %lld exceeds the 32-bit column index range", (long long)R->n);
  if (is_complex(R)) {
    if (!allow_complex)
      return fail(ENT_EUNSUPPORTED,
                  "complex (Hermitian) storage is accepted by the estimate and power-method calls only");
    if (R->layout != ENT_DENSE) return fail(ENT_EUNSUPPORTED, "complex (Hermitian) R must be dense");
    if (R->n > (int64_t)INT32_MAX / 2 - 64)
      return fail(ENT_EINVAL, "n = %lld too large for the 2n x 2n real form", (long long)R->n);
  } else if (R->dtype != ENT_STORE_F64 && R->dtype != ENT_STORE_F32) {
    return fail(ENT_EINVAL, "unknown storage dtype %d", R->dtype);
  }
  if (!R->values) return fail(ENT_EINVAL, "R->values is NULL");
  if (R->layout == ENT_DENSE) {
    if (R->ld < R->n) return fail(ENT_EINVAL, "ld = %lld < n", (long long)R->ld);
  } else if (R->layout == ENT_CSR) {
    if (!R->row_ptr || !R->col_idx) return fail(ENT_EINVAL, "CSR row_ptr/col_idx is NULL");
    if (R->nnz < 0) return fail(ENT_EINVAL, "nnz < 0");
  } else {
    return fail(ENT_EINVAL, "unknown layout %d", R->layout);
  }
  return ENT_OK;
}

// The caller's arrays must be memory the current device can read: device
// memory of the current device (or managed / pinned host memory), with the
// bytes the descriptor implies inside one allocation.  Checked on the host
// before any kernel sees the pointers, so a host pointer or a descriptor
// larger than its allocation is an ENT_EINVAL, not a memory fault.
ent_status check_device_range(const void *p, size_t bytes, const char *what) {
  if (!p) return fail(ENT_EINVAL, "%s is NULL", what);
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ENT_EINVAL, "%s is not memory the device can access", what);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged && at.type != hipMemoryTypeHost)
    return fail(ENT_EINVAL, "%s is not memory the device can access (memory type %d)", what, (int)at.type);
  if (at.type == hipMemoryTypeDevice) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (at.device != dev)
      return fail(ENT_EINVAL, "%s is memory of device %d, not of the current device %d", what, at.device, dev);
    // the extent check needs the allocation's range (not every allocator
    // reports one; then only the memory type is checked)
    void *base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess) {
      (void)hipGetLastError();
      return ENT_OK;
    }
    const uintptr_t end = (uintptr_t)base + size, at_p = (uintptr_t)p;
    if (at_p < (uintptr_t)base || bytes > end - at_p)
      return fail(ENT_EINVAL, "%s: the %zu bytes the descriptor implies exceed its allocation (%zu bytes from it)",
                  what, bytes, (size_t)(end - at_p));
  }
  return ENT_OK;
}

// Bytes of each array of R (validate_matrix has accepted R).
ent_status check_matrix_memory(const ent_matrix *R) {
  const int64_t n = R->n;
  const size_t esz = R->dtype == ENT_STORE_F64 ? 8 : R->dtype == ENT_STORE_F32 ? 4 : R->dtype == ENT_STORE_C128 ? 16 : 8;
  if (R->layout == ENT_DENSE) {
    if (R->ld > (INT64_MAX / (int64_t)esz) / n) return fail(ENT_EINVAL, "ld = %lld too large", (long long)R->ld);
    return check_device_range(R->values, (size_t)((n - 1) * R->ld + n) * esz, "R->values");
  }
  ent_status rc = check_device_range(R->row_ptr, (size_t)(n + 1) * sizeof(int64_t), "R->row_ptr");
  if (rc != ENT_OK || R->nnz == 0) return rc;
  rc = check_device_range(R->col_idx, (size_t)R->nnz * sizeof(int32_t), "R->col_idx");
  if (rc != ENT_OK) return rc;
  return check_device_range(R->values, (size_t)R->nnz * esz, "R->values");
}

// Host memory (pageable, or pinned by the HIP runtime): the estimate entry
// points copy such arrays to the device before anything else reads them.
bool is_host_memory(const void *p) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // memory the runtime does not know: pageable host memory
  }
  return at.type == hipMemoryTypeUnregistered || at.type == hipMemoryTypeHost;
}

// Runs body(R') with R' = R, or, when any array of R lies in host memory, a
// descriptor of device copies of those arrays in the device's staging buffer
// (extents as the descriptor states them: (n - 1) ld + n entries dense; n + 1,
// nnz, nnz CSR).  The copies are enqueued on st, so every later use on st
// sees them; the buffer is held until body returns.
template <typename F>
ent_status with_device_copy(const ent_matrix *R, hipStream_t st, F body) {
  const int64_t n = R->n;
  const size_t esz = R->dtype == ENT_STORE_F64 ? 8 : R->dtype == ENT_STORE_F32 ? 4 : R->dtype == ENT_STORE_C128 ? 16 : 8;
  struct Piece {
    const void *src;
    size_t bytes;
    const void **dst;
  };
  ent_matrix M = *R;
  std::vector<Piece> pieces;
  if (R->layout == ENT_DENSE) {
    if (R->ld > (INT64_MAX / (int64_t)esz) / n) return fail(ENT_EINVAL, "ld = %lld too large", (long long)R->ld);
    if (is_host_memory(R->values)) pieces.push_back({R->values, (size_t)((n - 1) * R->ld + n) * esz, &M.values});
  } else {
    if (is_host_memory(R->row_ptr))
      pieces.push_back({R->row_ptr, (size_t)(n + 1) * sizeof(int64_t), (const void **)&M.row_ptr});
    if (R->nnz > 0 && is_host_memory(R->col_idx))
      pieces.push_back({R->col_idx, (size_t)R->nnz * sizeof(int32_t), (const void **)&M.col_idx});
    if (R->nnz > 0 && is_host_memory(R->values))
      pieces.push_back({R->values, (size_t)R->nnz * esz, &M.values});
  }
  if (pieces.empty()) return body(R);
  size_t total = 0;
  for (auto &pc : pieces) total += (pc.bytes + 255) & ~size_t(255);
  if (g_ws_limit && total > g_ws_limit)
    return fail(ENT_ENOMEM, "device copy of the host matrix (%zu bytes) exceeds the workspace limit of %zu bytes",
                total, g_ws_limit.load());
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  StagingBuffer *b = staging_for(dev);
  std::lock_guard<std::mutex> lk(b->mu);
  if (b->bytes < total) {
    if (b->ptr) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(b->ptr));
      b->ptr = nullptr;
      b->bytes = 0;
    }
    if (hipMalloc(&b->ptr, total) != hipSuccess) {
      (void)hipGetLastError();
      b->ptr = nullptr;
      return fail(ENT_ENOMEM, "could not allocate %zu bytes for the device copy of the host matrix", total);
    }
    b->bytes = total;
  }
  size_t off = 0;
  for (auto &pc : pieces) {
    void *d = (char *)b->ptr + off;
    HIP_TRY(hipMemcpyAsync(d, pc.src, pc.bytes, hipMemcpyHostToDevice, st));
    *pc.dst = d;
    off += (pc.bytes + 255) & ~size_t(255);
  }
  const ent_status rc = body(&M);
  // the body synchronises st on success; on failure make sure no copy is
  // still reading the caller's host arrays or writing the buffer
  (void)hipStreamSynchronize(st);
  return rc;
}

struct Opts {
  ent_options o;
  hipStream_t st;
  // Rows of the probe block that carry probes (the rest are zero); -1 = all.
  // The real form of a Hermitian R has 2n rows and probes [g; 0].
  int64_t probe_rows = -1;
  // The matrix's trace is this multiple of tr R (2 for the real form).
  double trace_div = 1.0;
  // The no-allocation entry point: workspace from the fixed scratch array,
  // no phase events.
  bool no_alloc = false;
};

// The memory one estimate carves its buffers from, held (locked) for the
// whole estimate: the device's cached workspace, grown with hipMalloc on
// demand, or -- for the no-allocation entry point -- the device's fixed
// scratch array, whose size is then a hard limit.
struct WsLease {
  DeviceWorkspace *ws = nullptr;
  void *fixed = nullptr;
  std::unique_lock<std::mutex> lk;
  ent_status acquire(int dev, bool no_alloc) {
    if (no_alloc) {
      std::mutex *mu = nullptr;
      const hipError_t e = ent::noalloc_scratch(dev, &fixed, &mu);
      if (e != hipSuccess)
        return fail(ENT_EDEVICE, "address of the fixed scratch array on device %d: %s", dev, hipGetErrorString(e));
      lk = std::unique_lock<std::mutex>(*mu);
      return ENT_OK;
    }
    ws = workspace_for(dev);
    lk = std::unique_lock<std::mutex>(ws->mu);
    return ENT_OK;
  }
  void *ptr() const { return fixed ? fixed : ws->ptr; }
  ent_status ensure(size_t need) {
    if (fixed) {
      if (need > ent::kNoAllocScratchBytes)
        return fail(ENT_ENOMEM, "the estimate needs %zu bytes of workspace; the fixed scratch of the "
                                "no-allocation entry point holds %zu bytes", need, ent::kNoAllocScratchBytes);
      return ENT_OK;
    }
    return ensure_workspace(ws, need);
  }
};

Opts resolve_options(const ent_options *opt) {
  Opts r;
  if (opt)
    r.o = *opt;
  else
    ent_options_default(&r.o);
  r.st = (hipStream_t)r.o.stream;
  return r;
}

ent_status validate_options(const ent_options &o) {
  if (o.power_iters < 0) return fail(ENT_EINVAL, "power_iters < 0");
  if (o.power_trials < 1 && !(o.u_fixed > 0)) return fail(ENT_EINVAL, "power_trials < 1");
  if (!(o.u_factor > 0) && !(o.u_fixed > 0)) return fail(ENT_EINVAL, "u_factor must be > 0");
  if (o.precision < ENT_F64 || o.precision > ENT_BF16X3)
    return fail(ENT_EINVAL, "unknown precision %d", o.precision);
  if (o.probe_dist != ENT_RADEMACHER && o.probe_dist != ENT_GAUSSIAN)
    return fail(ENT_EINVAL, "unknown probe distribution %d", o.probe_dist);
  if (o.cutoff < 0 || !std::isfinite(o.cutoff)) return fail(ENT_EINVAL, "cutoff must be >= 0");
  if (o.u_fixed < 0 || !std::isfinite(o.u_fixed)) return fail(ENT_EINVAL, "u_fixed must be >= 0");
  if (o.u_fixed > 0 && o.cutoff >= o.u_fixed) return fail(ENT_EINVAL, "cutoff must be < u");
  return ENT_OK;
}

// ---------------------------------------------------------------------------
// Power method on the device (Algorithm 4).  Leaves p~1 in scal[S_P1].
// ---------------------------------------------------------------------------
template <typename T>
ent_status enqueue_power(const ent_matrix *R, const T *Rc, int64_t ldr, int32_t t, int32_t q,
                         uint64_t seed, double *x0, double *x1, double *part3, double *norm,
                         double *scal, hipStream_t st, const T *band = nullptr, int32_t hp = 0,
                         const T *trid = nullptr, int32_t *launches = nullptr) {
  const int64_t n = R->n;
  // tridiagonal and banded R: after the first product, the products of a
  // trial in launches of up to pf (ENT_POWER_FUSE, 1 = one per launch)
  int32_t pf = 1;
  if (trid || band) {
    const char *e = std::getenv("ENT_POWER_FUSE");
    pf = e && *e ? std::atoi(e) : ent::kPowerMaxFuse;
    pf = pf < 1 ? 1 : (pf > ent::kPowerMaxFuse ? ent::kPowerMaxFuse : pf);
  }
  int32_t nl = 0;
  for (int32_t trial = 0; trial < q; ++trial) {
    HIP_TRY(ent::launch_power_start(x0, n, seed, trial, st));
    double *xin = x0, *xout = x1;
    const double *in_norm = nullptr;
    for (int32_t it = 0; it <= t;) {  // t iterations + the Rayleigh product
      int32_t nblk = 0;
      const int32_t rem = t + 1 - it;
      ++nl;
      if ((trid || band) && it >= 1 && pf >= 2 && rem >= 2) {
        // the remaining products split as evenly as possible, longer first
        const int32_t nlaunch = (rem + pf - 1) / pf;
        const int32_t k = rem / nlaunch + (rem % nlaunch ? 1 : 0);
        if (trid) {
          nblk = ent::power_blocks_csr(n);
          HIP_TRY(ent::launch_power_tri_fused<T>(trid, n, xin, in_norm, xout, part3, nblk, k, st));
        } else {
          nblk = ent::power_band_fused_blocks(n);
          HIP_TRY(ent::launch_power_band_fused<T>(band, hp, n, xin, in_norm, xout, part3, nblk, k, st));
        }
        HIP_TRY(ent::launch_power_reduce(part3, nblk, norm, st));
        std::swap(xin, xout);
        in_norm = norm;
        it += k;
        continue;
      }
      ++it;
      if (R->layout == ENT_DENSE) {
        HIP_TRY(ent::launch_power_gemv<T>(Rc, ldr, n, xin, in_norm, xout, part3, &nblk, st));
      } else if (band) {
        // banded CSR: the same product on the slabs of the step kernel
        nblk = ent::power_blocks_csr(n);
        HIP_TRY(ent::launch_power_band<T>(band, hp, n, xin, in_norm, xout, part3, nblk, st));
      } else if (trid) {
        // tridiagonal CSR: the same product on the packed diagonals
        nblk = ent::power_blocks_csr(n);
        HIP_TRY(ent::launch_power_tri<T>(trid, n, xin, in_norm, xout, part3, nblk, st));
      } else
        HIP_TRY(ent::launch_power_spmv<T>(R->row_ptr, R->col_idx, (const T *)R->values, n, R->nnz,
                                          xin, in_norm, xout, part3, &nblk, st));
      HIP_TRY(ent::launch_power_reduce(part3, nblk, norm, st));
      std::swap(xin, xout);
      in_norm = norm;
    }
    HIP_TRY(ent::launch_power_rq(scal, norm, trial, st));
  }
  if (launches) *launches = nl;
  return ENT_OK;
}

// The same power method on the bf16 hi/lo split of a dense R.
ent_status enqueue_power_split(const uint16_t *hi, const uint16_t *lo, int64_t n, int64_t n_pad,
                               int32_t t, int32_t q, uint64_t seed, double *x0, double *x1,
                               double *part3, double *norm, double *scal, double *ypart, hipStream_t st) {
  // the split is zero beyond n, and so must be the vectors it multiplies
  HIP_TRY(ent::launch_fill(x0, n_pad, 0.0, st));
  HIP_TRY(ent::launch_fill(x1, n_pad, 0.0, st));
  for (int32_t trial = 0; trial < q; ++trial) {
    HIP_TRY(ent::launch_power_start(x0, n, seed, trial, st));
    double *xin = x0, *xout = x1;
    const double *in_norm = nullptr;
    for (int32_t it = 0; it <= t; ++it) {
      int32_t nblk = 0;
      HIP_TRY(ent::launch_power_gemv_split(hi, lo, n_pad, n, xin, in_norm, xout, part3, ypart, &nblk, st));
      HIP_TRY(ent::launch_power_reduce(part3, nblk, norm, st));
      std::swap(xin, xout);
      in_norm = norm;
    }
    HIP_TRY(ent::launch_power_rq(scal, norm, trial, st));
  }
  return ENT_OK;
}

// Validate a CSR structure on the device before any kernel dereferences its
// indices (one synchronisation).  Uses the first 256 bytes of the workspace.
// With hbw non-null, also measures the half-bandwidth max |col - row| (after
// the structure check, in the same synchronisation).
ent_status check_csr(const ent_matrix *R, void *scratch, hipStream_t st, int32_t *hbw = nullptr,
                     bool short_rows = false) {
  if (R->layout != ENT_CSR) return ENT_OK;
  int32_t *flag = (int32_t *)scratch;
  int32_t h[2] = {0, 0};
  HIP_TRY(ent::launch_zero(flag, 2 * sizeof(int32_t), st));
  if (hbw && short_rows) {
    // a few entries per row: the check and the half-bandwidth in one pass
    HIP_TRY(ent::launch_validate_csr_rows(R->row_ptr, R->col_idx, R->n, R->nnz, flag, st));
    HIP_TRY(hipMemcpyAsync(h, flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h[0]) return fail(ENT_EINVAL, "invalid CSR structure (row_ptr must start at 0, be non-decreasing "
                                      "and end at nnz; column indices must lie in [0, n))");
    *hbw = h[1];
    return ENT_OK;
  }
  HIP_TRY(ent::launch_validate_csr(R->row_ptr, R->col_idx, R->n, R->nnz, flag, st));
  HIP_TRY(hipMemcpyAsync(&h[0], flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h[0]) return fail(ENT_EINVAL, "invalid CSR structure (row_ptr must start at 0, be non-decreasing "
                                    "and end at nnz; column indices must lie in [0, n))");
  if (hbw) {
    HIP_TRY(ent::launch_csr_half_bandwidth(R->row_ptr, R->col_idx, R->n, flag + 1, st));
    HIP_TRY(hipMemcpyAsync(&h[1], flag + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *hbw = h[1];
  }
  return ENT_OK;
}

int64_t power_blocks(const ent_matrix *R) {
  return R->layout == ENT_DENSE ? ent::power_blocks_dense(R->n) : ent::power_blocks_csr(R->n);
}

// Optional work appended to an estimate: selector features and MLP inference
// on the device (feature pass of the learned selector), and a copy of the
// polynomial coefficients for the host-side a-posteriori check.
// Degree stages of one forward Chebyshev estimate (FP64 / FP32 paths): the
// recurrence runs to deg[0]; while check rejects the moments and stages
// remain, the same recurrence continues to the next degree on the same
// interval and probes.  The moments g^T T_k(X) g do not depend on the final
// degree, nor do the coefficients (Lemma 3 on [0, u]; the fixed 1024-node
// projection on [lo, u] up to degree 511), so a stage adds only its new
// products.  The estimate is the one at the degree reached.
struct DegreeStages {
  int32_t count = 0;
  int32_t deg[4] = {};
  // 1: accept, 0: continue to the next stage, -1: reject (no further stage)
  int (*check)(const std::vector<double> &mom, const std::vector<double> &alpha, int32_t m, int32_t s) = nullptr;
  int32_t used = 0;    // out: the degree of the estimate returned
  int32_t passed = 0;  // out: check accepted it
};

struct SelHook {
  float *feat_dev = nullptr;      // 16 features
  const float *params_dev = nullptr;
  float *y_dev = nullptr;         // 2 outputs
  float *y_host = nullptr;
  float *feat_host = nullptr;     // 16 features (optional)
  double *alpha_host = nullptr;   // m + 1 coefficients
  DegreeStages *stages = nullptr; // run_poly only; m is then the last stage's degree
};

// ---------------------------------------------------------------------------
// One polynomial estimate (Algorithms 1-2) in compute type T.
// ---------------------------------------------------------------------------
template <typename T>
ent_status run_poly(const ent_matrix *R, int32_t method, int32_t m, int32_t s, uint64_t seed,
                    const Opts &op, ent_result *out, double *per_probe, double *moments,
                    const SelHook *hook = nullptr) {
  const ent_options &o = op.o;
  hipStream_t st = op.st;
  const int64_t n = R->n;
  const bool dense = R->layout == ENT_DENSE;
  const bool stored_T = (R->dtype == ENT_STORE_F64) == (sizeof(T) == 8);
  const int vec_elems = 16 / (int)sizeof(T);
  bool need_copy = false;
  if (dense) {
    need_copy = !stored_T || (R->ld % vec_elems) != 0 || ((uintptr_t)R->values % 16) != 0;
  } else if (!stored_T) {
    return fail(ENT_EUNSUPPORTED, "CSR values must be stored in the compute precision");
  }
  // dense probe tile: 128 wide when that adds no padding over 64 (at
  // n = 8192, s = 256, with the K split its narrower grid brings in: 2.3%
  // less time per estimate in FP64, 3.5% in FP32)
  const int bn = dense ? (s <= 64 ? 64 : (round_up(s, 128) == round_up(s, 64) ? 128 : 64)) : 64;
  const int64_t ldv = round_up(s, dense ? bn : 64);
  const int64_t n_pad = round_up(n, 64);

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  WsLease ws;
  {
    const ent_status r0 = ws.acquire(dev, op.no_alloc);
    if (r0 != ENT_OK) return r0;
  }

  // CSR: validate the structure, and serve a matrix whose entries all lie
  // within one of the diagonal with the tridiagonal step kernel, within 16
  // with the banded step kernel
  int32_t hp = 0;
  bool tri = false;
  if (!dense) {
    ent_status rc0 = ws.ensure(256);
    if (rc0 != ENT_OK) return rc0;
    // the step streams the matrix once per product: take the slabs (16 + 2 hp
    // values per row) only if they are no larger than the CSR arrays (values,
    // column indices, row pointers), unless the caller asks for them
    const double csr_row = ((double)(sizeof(T) + 4) * (double)R->nnz + 8.0 * (double)(n + 1)) / (double)n;
    const bool forced = (o.flags & ENT_FLAG_CSR_BANDED) != 0;
    const bool want = !(o.flags & ENT_FLAG_CSR_GENERAL) && (forced || 24.0 * sizeof(T) <= csr_row);
    // at most three entries per row (duplicates aside) may be tridiagonal
    const bool maybe_tri = !(o.flags & (ENT_FLAG_CSR_GENERAL | ENT_FLAG_CSR_BANDED)) && R->nnz <= 3 * n;
    int32_t hbw = 0;
    rc0 = check_csr(R, ws.ptr(), st, (want || maybe_tri) ? &hbw : nullptr, maybe_tri);
    if (rc0 != ENT_OK) return rc0;
    tri = maybe_tri && hbw <= 1;
    if (want && !tri) hp = ent::band_half_width_padded(hbw);
    if (hp > 0 && (double)(16 + 2 * hp) * sizeof(T) > csr_row && !forced) hp = 0;
  }
  const bool banded = hp > 0;
  // rows of the V blocks (and of G): the tridiagonal kernel reads each row
  // of up to 256 probes in one pass, so they are s values rounded up to 4;
  // everything else, and the partial sums and sign words, use ldv
  const int64_t ldb = (tri && s <= 256) ? round_up(s, 4) : ldv;
  const int32_t ntile = dense ? (int32_t)(n_pad / 64)
                              : (tri ? ent::tri_step_blocks(n, s, sizeof(T) == 8)
                                     : (banded ? ent::band_step_waves(n, hp, sizeof(T) == 8)
                                               : ent::csr_step_blocks(n, sizeof(T) == 8)));
  // dense steps whose tile grid is smaller than the chip split K
  const int32_t ksplit = dense ? ent::dense_step_splits(n, ntile, ldv, bn) : 1;
  const int64_t kper = round_up((n + ksplit - 1) / ksplit, 32);
  // per-probe dot partials: one per row tile (64 rows), or per 16 rows when
  // the split-K epilogue forms them
  const int32_t npart = ksplit > 1 ? (int32_t)(n_pad / 16) : ntile;
  // Clenshaw (Algorithm 5): slots 0..m hold g^T y_k, slot m+1 holds g^T g
  const bool clenshaw = method == ENT_CHEBYSHEV && (o.flags & ENT_FLAG_CLENSHAW);
  const int32_t nslot = m + 1 + (clenshaw ? 1 : 0);
  const bool rad = o.probe_dist == ENT_RADEMACHER;
  const bool use_power = !(o.u_fixed > 0);
  const int32_t pblk = (int32_t)power_blocks(R);

  double *scal = nullptr, *x0 = nullptr, *x1 = nullptr, *p0 = nullptr, *p1 = nullptr;
  double *part = nullptr, *d = nullptr, *h = nullptr;
  T *Rc = nullptr, *G = nullptr, *VA = nullptr, *VB = nullptr, *band = nullptr, *trid = nullptr;
  // banded FP32 R: two recurrence steps per launch (two more V blocks: a
  // pair's outputs may not overwrite its inputs)
  const int32_t nsteps_all = clenshaw ? m + 1 : (method == ENT_CHEBYSHEV) ? m : m + 1;
  // degree stages (forward Chebyshev): one step per launch, so a stage can
  // end after any step
  DegreeStages *stg = (hook && hook->stages && hook->stages->count > 0 && method == ENT_CHEBYSHEV && !clenshaw)
                          ? hook->stages : nullptr;
  bool band_pairs = banded && sizeof(T) == 4 && nsteps_all >= 2 && !stg && step_pairs_enabled("ENT_BAND_PAIRS");
  // tridiagonal R: up to kTriMaxFuse steps per launch (both precisions)
  const int32_t tri_nf = tri ? tri_fuse_steps() : 1;
  bool tri_fused = tri && nsteps_all >= 2 && tri_nf >= 2 && !stg;
  // all steps in one launch from the probe block: its two outputs are the
  // only V blocks (Clenshaw starts from two zero blocks)
  const bool tri_one_launch = tri_fused && !clenshaw && nsteps_all <= tri_nf;
  T *VC = nullptr, *VD = nullptr, *tprep = nullptr;
  double *ttmp = nullptr;
  uint32_t *signs = nullptr;
  int2 *cwin = nullptr;
  const int32_t ch = ent::csr_chunk_rows(sizeof(T) == 8);
  T *party = nullptr;
  const int64_t ldc = round_up(n, vec_elems);
  auto plan = [&](Carve &cv) {
    cv.add(&scal, kScalarDoubles);
    if (!dense && !banded && !tri) cv.add(&cwin, (size_t)((n + ch - 1) / ch));
    if (banded) cv.add(&band, ent::band_pack_elems(n, hp));
    if (tri) {
      cv.add(&trid, 4 * (size_t)n);
      cv.add(&ttmp, (size_t)ent::kTriTraceBlocks);
    }
    if (tri_fused && method == ENT_CHEBYSHEV) cv.add(&tprep, 4 * (size_t)n);
    if (use_power) {
      cv.add(&x0, n_pad);
      cv.add(&x1, n_pad);
      cv.add(&p0, 3 * (size_t)pblk);
      cv.add(&p1, 4);
    }
    if (need_copy) cv.add(&Rc, (size_t)n * ldc);
    if (dense || !rad) cv.add(&G, (size_t)n_pad * ldb);
    if (!dense && rad) cv.add(&signs, (size_t)n_pad * (ldv / 32));
    cv.add(&VA, (size_t)n_pad * ldb);
    cv.add(&VB, (size_t)n_pad * ldb);
    if (band_pairs || (tri_fused && !tri_one_launch)) {
      cv.add(&VC, (size_t)n_pad * ldb);
      cv.add(&VD, (size_t)n_pad * ldb);
    }
    if (ksplit > 1) cv.add(&party, (size_t)ksplit * n_pad * ldv);
    cv.add(&part, (size_t)nslot * npart * ldv);
    cv.add(&d, (size_t)nslot * s);
    cv.add(&h, (size_t)s);
  };
  Carve cv;
  plan(cv);
  ent_status rc = ws.ensure(cv.total());
  if (rc == ENT_ENOMEM && (band_pairs || tri_fused)) {
    // the multi-step launches need two more V blocks: without room for
    // them, one step per launch
    band_pairs = tri_fused = false;
    cv = Carve();
    plan(cv);
    rc = ws.ensure(cv.total());
  }
  if (rc != ENT_OK) return rc;
  cv.assign(ws.ptr());

  PhaseEvents pe;
  pe.on = g_timing_on && !op.no_alloc;
  pe.st = st;
  pe.csr_band = tri ? 1 : hp;
  pe.mark();
  HIP_TRY(ent::launch_zero(scal, sizeof(double) * 64, st));
  // CSR step launches may use fewer workgroups than the partial stride
  if (!dense) HIP_TRY(ent::launch_zero(part, sizeof(double) * (size_t)nslot * ntile * ldv, st));
  // trace check (or the trace that normalises R)
  const bool normalize = (o.flags & ENT_FLAG_NORMALIZE) != 0;
  const bool check_trace = !(o.flags & ENT_FLAG_SKIP_TRACE_CHECK) && !normalize;
  if (check_trace || normalize) {
    if (dense) {
      if (R->dtype == ENT_STORE_F64)
        HIP_TRY(ent::launch_trace_dense<double>((const double *)R->values, R->ld, n, scal, st));
      else
        HIP_TRY(ent::launch_trace_dense<float>((const float *)R->values, R->ld, n, scal, st));
    } else if (!tri) {  // the tridiagonal pack below sums the diagonal itself
      if (R->dtype == ENT_STORE_F64)
        HIP_TRY(ent::launch_trace_csr<double>(R->row_ptr, R->col_idx, (const double *)R->values, n, R->nnz,
                                              scal, st));
      else
        HIP_TRY(ent::launch_trace_csr<float>(R->row_ptr, R->col_idx, (const float *)R->values, n, R->nnz,
                                             scal, st));
    }
  }
  // matrix in the compute type
  const T *Rt = (const T *)R->values;
  int64_t ldr = R->ld;
  if (need_copy) {
    if (R->dtype == ENT_STORE_F64)
      HIP_TRY((ent::launch_convert<double, T>((const double *)R->values, R->ld, Rc, ldc, n, n, st)));
    else
      HIP_TRY((ent::launch_convert<float, T>((const float *)R->values, R->ld, Rc, ldc, n, n, st)));
    Rt = Rc;
    ldr = ldc;
  }
  if (banded)
    HIP_TRY(ent::launch_band_pack<T>(R->row_ptr, R->col_idx, (const T *)R->values, n, hp, band, st));
  else if (tri)
    HIP_TRY(ent::launch_tri_pack<T>(R->row_ptr, R->col_idx, (const T *)R->values, n, trid, ttmp,
                                    (check_trace || normalize) ? scal + ent::S_TRACE : nullptr, st));
  else if (!dense)
    HIP_TRY(ent::launch_csr_chunk_window(R->row_ptr, R->col_idx, n, ch, cwin, st));
  // probes
  if (dense || !rad)
    HIP_TRY(ent::launch_probe_gen<T>(G, nullptr, op.probe_rows > 0 ? op.probe_rows : n, n_pad, s, ldb,
                                     seed, o.probe_dist, st));
  else
    HIP_TRY(ent::launch_sign_gen(signs, n, s, ldv, seed, st));
  // power method and interval
  if (use_power) {
    pe.power_begin = pe.mark();
    int32_t pl = 0;
    rc = enqueue_power<T>(R, Rt, ldr, o.power_iters, o.power_trials, seed, x0, x1, p0, p1, scal, st, band, hp,
                          trid, &pl);
    if (rc != ENT_OK) return rc;
    pe.power_end = pe.mark();
    pe.power_launches = pl;
  }
  HIP_TRY(ent::launch_setup_interval(scal, method, m, o.u_factor, o.u_fixed, o.cutoff, st,
                                     normalize ? op.trace_div : 0.0));
  // tridiagonal Chebyshev steps run on the prepared 2X = 2(aR - bI)
  if (tprep) HIP_TRY(ent::launch_tri_prepare<T>(trid, scal, n, tprep, st));

  // recurrence
  const int32_t nsteps = clenshaw ? m + 1 : (method == ENT_CHEBYSHEV) ? m : m + 1;
  const T *Vk = dense || !rad ? G : nullptr;  // null: expand the sign block
  const T *Vkm1 = nullptr;
  T *bufs[2] = {VA, VB};
  if (clenshaw) {
    // y_{m+1} = y_{m+2} = 0; y_k = alpha_k g + 2X y_{k+1} - y_{k+2}, k = m..0,
    // each y_k written over y_{k+2} (same element, same thread)
    HIP_TRY(ent::launch_zero(VA, sizeof(T) * (size_t)n_pad * ldb, st));
    HIP_TRY(ent::launch_zero(VB, sizeof(T) * (size_t)n_pad * ldb, st));
    Vk = VA;
    Vkm1 = VB;
  }
  pe.steps_begin = pe.mark();
  // a K-split dense step is timed as its product kernel and its epilogue
  int prev_mark = pe.steps_begin, split_mark = -1;
  auto dense_step = [&](const ent::DenseStepArgs &a) -> hipError_t {
    if (a.ksplit < 2 || !pe.on) return ent::launch_dense_step<T>(a, st);
    const hipError_t e = ent::launch_dense_step<T>(a, st, false);
    if (e != hipSuccess) return e;
    split_mark = pe.mark();
    return ent::launch_dense_split_epilogue<T>(a, st);
  };
  auto end_step = [&](int e) {
    if (split_mark >= 0) {
      pe.main_spans.push_back({prev_mark, split_mark});
      pe.epi_spans.push_back({split_mark, e});
      split_mark = -1;
    }
    prev_mark = e;
  };
  if (band_pairs || tri_fused) {
    // banded: steps k, k + 1 in one launch, the last step of an odd count
    // alone; tridiagonal: launches of up to tri_nf steps
    std::vector<int32_t> sizes;
    if (tri_fused) {
      sizes = fuse_split(nsteps, tri_nf);
    } else {
      for (int32_t k = 0; k < nsteps; k += 2) sizes.push_back(k + 1 < nsteps ? 2 : 1);
    }
    pe.steps_fused = sizes[0];
    T *pool[4] = {VA, VB, VC, VD};
    auto free_buf = [&](const void *x, const void *y, const void *z) -> T * {
      for (T *b : pool)
        if (b && b != x && b != y && b != z) return b;
      return nullptr;
    };
    auto params = [&](int32_t k, double *c1, double *c2, double *cw, int32_t *dot_y, int32_t *slot,
                      int32_t *slot_gg, const double **cg, bool *write) {
      *cg = nullptr;
      *slot_gg = -1;
      *write = true;
      if (clenshaw) {
        const int32_t kk = m - k;
        *c1 = 2.0; *c2 = -2.0; *cw = k == 0 ? 0.0 : -1.0; *dot_y = 0; *slot = kk;
        *slot_gg = k == 0 ? m + 1 : -1;
        *cg = scal + ent::S_ALPHA + kk;
      } else if (method == ENT_CHEBYSHEV) {
        if (k == 0) {
          *c1 = 1.0; *c2 = -1.0; *cw = 0.0; *slot_gg = 0;
        } else {
          *c1 = 2.0; *c2 = -2.0; *cw = -1.0;
        }
        *dot_y = 0;
        *slot = k + 1;
      } else {
        *c1 = -1.0; *c2 = 1.0; *cw = 0.0; *dot_y = 1; *slot = k;
        *write = k < nsteps - 1;
      }
    };
    int32_t k = 0;
    for (const int32_t len : sizes) {
      double c1, c2, cw;
      int32_t dot_y, slot, slot_gg;
      const double *cg;
      bool write;
      params(k, &c1, &c2, &cw, &dot_y, &slot, &slot_gg, &cg, &write);
      if (len >= 2) {
        // per-step scalars of steps k .. k + len - 1
        double c1s[ent::kTriMaxFuse], c2s[ent::kTriMaxFuse], cws[ent::kTriMaxFuse];
        int32_t dys[ent::kTriMaxFuse], slots[ent::kTriMaxFuse];
        const double *cgs[ent::kTriMaxFuse];
        bool last_write = write;
        for (int32_t j = 0; j < len; ++j) {
          int32_t gg;
          params(k + j, &c1s[j], &c2s[j], &cws[j], &dys[j], &slots[j], &gg, &cgs[j], &last_write);
        }
        T *outA = free_buf(Vk, Vkm1, nullptr);
        T *outB = free_buf(Vk, Vkm1, outA);
        const int e0 = pe.mark();
        if (tri_fused) {
          ent::TriFusedArgs ta{};
          ta.diag = trid; ta.prep = tprep; ta.n = n; ta.ldv = ldv; ta.ldb = ldb; ta.s = s;
          ta.Vk = Vk; ta.Vkm1 = cw != 0.0 ? Vkm1 : nullptr;
          ta.VoutA = outA; ta.VoutB = last_write ? outB : nullptr;
          ta.signs = rad ? signs : nullptr; ta.G = rad ? nullptr : G;
          ta.scal = scal; ta.part = part; ta.nblk = ntile; ta.slot_gg = slot_gg;
          for (int32_t j = 0; j < len; ++j) {
            ta.c1[j] = c1s[j]; ta.c2[j] = c2s[j]; ta.cw[j] = cws[j];
            ta.dot_y[j] = dys[j]; ta.slot[j] = slots[j]; ta.cg[j] = cgs[j];
          }
          HIP_TRY(ent::launch_tri_fused<T>(ta, len, st));
        } else {
          ent::BandPairArgs pa{};
          pa.band = band; pa.n = n; pa.ldv = ldv;
          pa.Vk = Vk; pa.Vkm1 = cw != 0.0 ? Vkm1 : nullptr;
          pa.signs = rad ? signs : nullptr; pa.G = rad ? nullptr : G;
          pa.scal = scal; pa.part = part; pa.nwave = ntile; pa.slot_gg = slot_gg;
          for (int32_t j = 0; j < 2; ++j) {
            pa.c1[j] = c1s[j]; pa.c2[j] = c2s[j]; pa.cw[j] = cws[j];
            pa.dot_y[j] = dys[j]; pa.slot[j] = slots[j]; pa.cg[j] = cgs[j];
          }
          pa.VoutA = outA;
          pa.VoutB = last_write ? outB : nullptr;
          HIP_TRY(ent::launch_band_pair(pa, hp, st));
        }
        const int e1 = pe.mark();
        if (pe.on) pe.main_spans.push_back({e0, e1});
        Vkm1 = outA;
        Vk = outB;
        k += len;
      } else if (tri_fused) {
        ent::TriStepArgs a{};
        a.diag = trid; a.n = n; a.ldv = ldv; a.ldb = ldb; a.s = s;
        a.Vk = Vk; a.Vkm1 = cw != 0.0 ? Vkm1 : nullptr;
        a.Vkp1 = write ? free_buf(Vk, Vkm1, nullptr) : nullptr;
        a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
        a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
        a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.nblk = ntile; a.cg = cg;
        HIP_TRY(ent::launch_tri_step<T>(a, st));
        k += 1;
      } else {
        ent::BandStepArgs a{};
        a.band = band; a.n = n; a.ldv = ldv;
        a.Vk = Vk; a.Vkm1 = cw != 0.0 ? Vkm1 : nullptr;
        a.Vkp1 = write ? free_buf(Vk, Vkm1, nullptr) : nullptr;
        a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
        a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
        a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.nwave = ntile; a.cg = cg;
        HIP_TRY(ent::launch_band_step<T>(a, hp, st));
        k += 1;
      }
    }
    pe.steps_end = pe.mark();
  }
  int32_t k_begin = (band_pairs || tri_fused) ? nsteps : 0;
  int32_t m_run = stg ? stg->deg[0] : m;  // degree of the estimate
  int32_t stage = 0;
  for (;;) {
    const int32_t k_end = stg ? m_run : nsteps;
    for (int32_t k = k_begin; k < k_end; ++k) {
      if (clenshaw) {
        const int32_t kk = m - k;  // index of the y computed by this launch
        T *Vout = (T *)Vkm1;
        if (dense) {
          ent::DenseStepArgs a{};
          a.R = Rt; a.ldr = ldr; a.n = n; a.ldv = ldv;
          a.Vk = Vk; a.Vkm1 = Vkm1; a.Vkp1 = Vout; a.G = G;
          a.scal = scal; a.c1 = 2.0; a.c2 = -2.0; a.cw = k == 0 ? 0.0 : -1.0; a.dot_y = 0;
          a.slot = kk; a.slot_gg = k == 0 ? m + 1 : -1; a.part = part; a.ntile = ntile; a.bn = bn;
          a.cg = scal + ent::S_ALPHA + kk;
          a.ksplit = ksplit; a.kper = kper; a.party = party; a.nptile = npart;
          HIP_TRY(dense_step(a));
        } else if (banded) {
          ent::BandStepArgs a{};
          a.band = band; a.n = n; a.ldv = ldv;
          a.Vk = Vk; a.Vkm1 = k == 0 ? nullptr : Vkm1; a.Vkp1 = Vout;
          a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
          a.scal = scal; a.c1 = 2.0; a.c2 = -2.0; a.cw = k == 0 ? 0.0 : -1.0; a.dot_y = 0;
          a.slot = kk; a.slot_gg = k == 0 ? m + 1 : -1; a.part = part; a.nwave = ntile;
          a.cg = scal + ent::S_ALPHA + kk;
          HIP_TRY(ent::launch_band_step<T>(a, hp, st));
        } else if (tri) {
          ent::TriStepArgs a{};
          a.diag = trid; a.n = n; a.ldv = ldv; a.ldb = ldb; a.s = s;
          a.Vk = Vk; a.Vkm1 = k == 0 ? nullptr : Vkm1; a.Vkp1 = Vout;
          a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
          a.scal = scal; a.c1 = 2.0; a.c2 = -2.0; a.cw = k == 0 ? 0.0 : -1.0; a.dot_y = 0;
          a.slot = kk; a.slot_gg = k == 0 ? m + 1 : -1; a.part = part; a.nblk = ntile;
          a.cg = scal + ent::S_ALPHA + kk;
          HIP_TRY(ent::launch_tri_step<T>(a, st));
        } else {
          ent::CsrStepArgs a{};
          a.row_ptr = R->row_ptr; a.col_idx = R->col_idx; a.values = R->values; a.n = n; a.ldv = ldv;
          a.Vk = Vk; a.Vkm1 = k == 0 ? nullptr : Vkm1; a.Vkp1 = Vout;
          a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
          a.scal = scal; a.c1 = 2.0; a.c2 = -2.0; a.cw = k == 0 ? 0.0 : -1.0; a.dot_y = 0;
          a.slot = kk; a.slot_gg = k == 0 ? m + 1 : -1; a.part = part; a.nblk = ntile; a.win = cwin;
          a.cg = scal + ent::S_ALPHA + kk;
          a.s = s;
          HIP_TRY(ent::launch_csr_step<T>(a, st));
        }
        Vkm1 = Vk;
        Vk = Vout;
        const int e = pe.mark();
        if (k == nsteps - 1) pe.steps_end = e;
        end_step(e);
        continue;
      }
      T *Vout = bufs[k & 1];
      double c1, c2, cw;
      int32_t dot_y, slot, slot_gg = -1;
      bool write = true;
      if (method == ENT_CHEBYSHEV) {
        if (k == 0) {
          c1 = 1.0; c2 = -1.0; cw = 0.0;
          slot_gg = 0;
        } else {
          c1 = 2.0; c2 = -2.0; cw = -1.0;
        }
        dot_y = 0;
        slot = k + 1;
      } else {
        c1 = -1.0; c2 = 1.0; cw = 0.0;
        dot_y = 1;
        slot = k;
        write = k < nsteps - 1;
      }
      if (dense) {
        ent::DenseStepArgs a{};
        a.R = Rt; a.ldr = ldr; a.n = n; a.ldv = ldv;
        a.Vk = Vk; a.Vkm1 = Vkm1; a.Vkp1 = write ? Vout : nullptr; a.G = G;
        a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
        a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.ntile = ntile; a.bn = bn;
        a.ksplit = ksplit; a.kper = kper; a.party = party; a.nptile = npart;
        HIP_TRY(dense_step(a));
      } else if (banded) {
        ent::BandStepArgs a{};
        a.band = band; a.n = n; a.ldv = ldv;
        a.Vk = Vk; a.Vkm1 = Vkm1; a.Vkp1 = write ? Vout : nullptr;
        a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
        a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
        a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.nwave = ntile;
        HIP_TRY(ent::launch_band_step<T>(a, hp, st));
      } else if (tri) {
        ent::TriStepArgs a{};
        a.diag = trid; a.n = n; a.ldv = ldv; a.ldb = ldb; a.s = s;
        a.Vk = Vk; a.Vkm1 = Vkm1; a.Vkp1 = write ? Vout : nullptr;
        a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
        a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
        a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.nblk = ntile;
        HIP_TRY(ent::launch_tri_step<T>(a, st));
      } else {
        ent::CsrStepArgs a{};
        a.row_ptr = R->row_ptr; a.col_idx = R->col_idx; a.values = R->values; a.n = n; a.ldv = ldv;
        a.Vk = Vk; a.Vkm1 = Vkm1; a.Vkp1 = write ? Vout : nullptr;
        a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
        a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
        a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.nblk = ntile; a.win = cwin;
        a.s = s;
        HIP_TRY(ent::launch_csr_step<T>(a, st));
      }
      // Chebyshev: V_{k+1} is written over V_{k-1} (same element, same thread),
      // so two buffers plus the probe block suffice.  Taylor: W_{k+1} may not
      // overwrite W_k (read by every tile), so outputs alternate.
      if (method == ENT_CHEBYSHEV) Vkm1 = Vk;
      Vk = Vout;
      const int e = pe.mark();
      if (k == k_end - 1) pe.steps_end = e;
      end_step(e);
    }
    HIP_TRY(ent::launch_reduce_moments(part, stg ? m_run + 1 : nslot, npart, ldv, s, d, st));
    HIP_TRY(ent::launch_final(d, scal, clenshaw ? ent::FINAL_CLENSHAW : method, m_run, s, h, st));
    if (!stg) break;
    // the check on the host; on rejection the recurrence continues from V_k, V_{k-1}
    std::vector<double> smom((size_t)(m_run + 1) * s), salpha(m_run + 1);
    HIP_TRY(hipMemcpyAsync(smom.data(), d, sizeof(double) * smom.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(salpha.data(), scal + ent::S_ALPHA, sizeof(double) * salpha.size(),
                           hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int outcome = stg->check(smom, salpha, m_run, s);
    stg->passed = outcome == 1 ? 1 : 0;
    stg->used = m_run;
    if (outcome != 0 || stage + 1 >= stg->count) break;
    k_begin = k_end;
    m_run = stg->deg[++stage];
  }
  if (hook && hook->feat_dev) {
    HIP_TRY(ent::launch_selector_features(scal, d, m, s, n, hook->feat_dev, st));
    HIP_TRY(ent::launch_mlp_forward(hook->params_dev, hook->feat_dev, 1, hook->y_dev, st));
    HIP_TRY(hipMemcpyAsync(hook->y_host, hook->y_dev, 2 * sizeof(float), hipMemcpyDeviceToHost, st));
    if (hook->feat_host)
      HIP_TRY(hipMemcpyAsync(hook->feat_host, hook->feat_dev, 16 * sizeof(float), hipMemcpyDeviceToHost, st));
  }
  if (hook && hook->alpha_host)
    HIP_TRY(hipMemcpyAsync(hook->alpha_host, scal + ent::S_ALPHA, sizeof(double) * (m_run + 1),
                           hipMemcpyDeviceToHost, st));

  double hs[16];
  HIP_TRY(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, st));
  if (per_probe) HIP_TRY(hipMemcpyAsync(per_probe, h, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  if (moments)
    HIP_TRY(hipMemcpyAsync(moments, d, sizeof(double) * (m_run + 1) * s, hipMemcpyDeviceToHost, st));
  pe.mark();
  HIP_TRY(hipStreamSynchronize(st));
  pe.finish();

  if (check_trace) {
    double tol = o.trace_tol > 0 ? o.trace_tol : (R->dtype == ENT_STORE_F64 ? 1e-10 : 1e-4);
    if (!(std::fabs(hs[ent::S_TRACE] / op.trace_div - 1.0) <= tol))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g, not 1 within %.3g",
                  hs[ent::S_TRACE] / op.trace_div, tol);
  }
  if (normalize) {
    const double tr = hs[ent::S_TRACE] / op.trace_div;
    if (!(tr > 0) || !std::isfinite(1.0 / tr))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g: R cannot be normalised to unit trace", tr);
  }
  if (hs[ent::S_FLAG] != 0.0)
    return fail(ENT_ENUMERIC, "numeric failure: p1~ = %.17g, u = %.17g, estimate = %.17g",
                hs[ent::S_P1], hs[ent::S_U], hs[ent::S_ENT]);
  out->entropy = hs[ent::S_ENT];
  out->std_err = hs[ent::S_SE];
  out->p1_est = use_power ? hs[ent::S_P1] : 0.0;
  out->u = hs[ent::S_U];
  out->lo = hs[ent::S_LO];
  out->degree = m_run;
  out->probes = s;
  out->method = method;
  out->precision = o.precision;
  out->fell_back = 0;
  out->products = (method == ENT_CHEBYSHEV) ? m_run : m_run + 1;
  return ENT_OK;
}


// ---------------------------------------------------------------------------
// BF16x3 dense estimate: A = a R split into bf16 hi/lo once, each step is a
// split-K BF16 MFMA product plus an elementwise FP32 epilogue.
// ---------------------------------------------------------------------------
ent_status run_bf16x3(const ent_matrix *R, int32_t method, int32_t m, int32_t s, uint64_t seed,
                      const Opts &op, ent_result *out, double *per_probe, double *moments,
                      const SelHook *hook = nullptr) {
  const ent_options &o = op.o;
  hipStream_t st = op.st;
  if (R->layout != ENT_DENSE) return fail(ENT_EUNSUPPORTED, "BF16x3 is implemented for dense R only");
  const int64_t n = R->n;
  const bool f64 = R->dtype == ENT_STORE_F64;
  // 256-row GEMM tiles run ~8% faster than 128-row ones (n_pad = 8192,
  // 10240): pad to a multiple of 256 when the extra padded area costs less
  const int64_t p128 = round_up(n, 128), p256 = round_up(n, 256);
  const int64_t n_pad = ((double)p256 * (double)p256 <= 1.07 * (double)p128 * (double)p128) ? p256 : p128;
  const int bn = s <= 64 ? 64 : (s <= 128 ? 128 : 256);
  const int64_t ldv = round_up(s, bn);
  const int64_t tiles = (n_pad / ent::bf16x3_tile_rows(n_pad)) * (ldv / bn);
  const int32_t splits = ent::bf16x3_splits(n_pad, tiles);
  const int64_t kps = n_pad / splits;
  const int32_t nblk = ent::bf16x3_epilogue_blocks(n_pad);
  // Clenshaw (Algorithm 5): slots 0..m hold g^T y_k, slot m+1 holds g^T g
  const bool clenshaw = method == ENT_CHEBYSHEV && (o.flags & ENT_FLAG_CLENSHAW);
  const int32_t nslot = m + 1 + (clenshaw ? 1 : 0);
  const bool use_power = !(o.u_fixed > 0);
  const int32_t pblk = ent::power_blocks_split(n_pad);

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  WsLease ws;
  {
    const ent_status r0 = ws.acquire(dev, op.no_alloc);
    if (r0 != ENT_OK) return r0;
  }
  double *scal = nullptr, *x0 = nullptr, *x1 = nullptr, *p0 = nullptr, *p1 = nullptr, *ypart = nullptr;
  double *part = nullptr, *d = nullptr, *h = nullptr;
  uint16_t *Ahi = nullptr, *Alo = nullptr, *Vhi = nullptr, *Vlo = nullptr;
  float *G = nullptr, *VA = nullptr, *VB = nullptr, *party = nullptr;
  Carve cv;
  cv.add(&scal, kScalarDoubles);
  if (use_power) {
    cv.add(&x0, n_pad);
    cv.add(&x1, n_pad);
    cv.add(&p0, 3 * (size_t)pblk);
    cv.add(&p1, 4);
    const int32_t pparts = ent::power_split_parts(n_pad);
    if (pparts > 1) cv.add(&ypart, (size_t)pparts * n_pad);
  }
  cv.add(&Ahi, (size_t)n_pad * n_pad);
  cv.add(&Alo, (size_t)n_pad * n_pad);
  cv.add(&G, (size_t)ldv * n_pad);
  cv.add(&VA, (size_t)ldv * n_pad);
  cv.add(&VB, (size_t)ldv * n_pad);
  cv.add(&Vhi, (size_t)ldv * n_pad);
  cv.add(&Vlo, (size_t)ldv * n_pad);
  cv.add(&party, (size_t)splits * ldv * n_pad);
  cv.add(&part, (size_t)nslot * nblk * ldv);
  cv.add(&d, (size_t)nslot * s);
  cv.add(&h, (size_t)s);
  ent_status rc = ws.ensure(cv.total());
  if (rc != ENT_OK) return rc;
  cv.assign(ws.ptr());

  PhaseEvents pe;
  pe.on = g_timing_on && !op.no_alloc;
  pe.st = st;
  pe.mark();
  HIP_TRY(ent::launch_zero(scal, sizeof(double) * 64, st));
  const bool normalize = (o.flags & ENT_FLAG_NORMALIZE) != 0;
  const bool check_trace = !(o.flags & ENT_FLAG_SKIP_TRACE_CHECK) && !normalize;
  if (check_trace || normalize) {
    if (f64)
      HIP_TRY(ent::launch_trace_dense<double>((const double *)R->values, R->ld, n, scal, st));
    else
      HIP_TRY(ent::launch_trace_dense<float>((const float *)R->values, R->ld, n, scal, st));
  }
  HIP_TRY(ent::launch_probe_gen_t(G, Vhi, Vlo, op.probe_rows > 0 ? op.probe_rows : n, n_pad, s, ldv, seed,
                                  o.probe_dist, st));
  // split R itself once; the power method reads the split (half the bytes of
  // an FP32 copy), and the interval scale a is applied to each product
  if (f64)
    HIP_TRY(ent::launch_split_matrix<double>((const double *)R->values, R->ld, n, n_pad, nullptr, Ahi, Alo, st));
  else
    HIP_TRY(ent::launch_split_matrix<float>((const float *)R->values, R->ld, n, n_pad, nullptr, Ahi, Alo, st));
  if (use_power) {
    pe.power_begin = pe.mark();
    rc = enqueue_power_split(Ahi, Alo, n, n_pad, o.power_iters, o.power_trials, seed, x0, x1, p0, p1,
                             scal, ypart, st);
    if (rc != ENT_OK) return rc;
    pe.power_end = pe.mark();
    pe.power_launches = o.power_trials * (o.power_iters + 1);
  }
  HIP_TRY(ent::launch_setup_interval(scal, method, m, o.u_factor, o.u_fixed, o.cutoff, st,
                                     normalize ? op.trace_div : 0.0));

  const int32_t nsteps = clenshaw ? m + 1 : (method == ENT_CHEBYSHEV) ? m : m + 1;
  const float *Vk = G, *Vkm1 = nullptr;
  float *bufs[2] = {VA, VB};
  if (clenshaw) {
    // y_{m+1} = y_{m+2} = 0 (and the split of y_{m+1}); see run_poly
    HIP_TRY(ent::launch_zero(VA, sizeof(float) * (size_t)n_pad * ldv, st));
    HIP_TRY(ent::launch_zero(VB, sizeof(float) * (size_t)n_pad * ldv, st));
    HIP_TRY(ent::launch_zero(Vhi, sizeof(uint16_t) * (size_t)n_pad * ldv, st));
    HIP_TRY(ent::launch_zero(Vlo, sizeof(uint16_t) * (size_t)n_pad * ldv, st));
    Vk = VA;
    Vkm1 = VB;
  }
  pe.steps_begin = pe.mark();
  for (int32_t k = 0; k < nsteps; ++k) {
    if (clenshaw) {
      const int32_t kk = m - k;
      float *Vout = (float *)Vkm1;
      ent::Bf16GemmArgs ga{};
      ga.A_hi = Ahi; ga.A_lo = Alo; ga.V_hi = Vhi; ga.V_lo = Vlo; ga.part_y = party;
      ga.n_pad = n_pad; ga.ldv = ldv; ga.k_per_split = kps; ga.splits = splits; ga.bn = bn;
      const int e0 = pe.mark();
      HIP_TRY(ent::launch_bf16x3_gemm(ga, st));
      const int e1 = pe.mark();
      ent::Bf16EpiArgs ea{};
      ea.part_y = party; ea.splits = splits; ea.Vk = Vk; ea.Vkm1 = k == 0 ? nullptr : Vkm1;
      ea.Vkp1 = Vout; ea.V_hi = Vhi; ea.V_lo = Vlo; ea.G = G; ea.scal = scal;
      ea.c1 = 2.0; ea.c2 = -2.0; ea.cw = k == 0 ? 0.0 : -1.0; ea.dot_y = 0; ea.slot = kk;
      ea.slot_gg = k == 0 ? m + 1 : -1; ea.scale_y = 1; ea.cg = scal + ent::S_ALPHA + kk;
      ea.part = part; ea.nblk = nblk; ea.n_pad = n_pad; ea.ldv = ldv;
      HIP_TRY(ent::launch_bf16x3_epilogue(ea, st));
      const int e2 = pe.mark();
      if (pe.on) {
        pe.main_spans.push_back({e0, e1});
        pe.epi_spans.push_back({e1, e2});
      }
      Vkm1 = Vk;
      Vk = Vout;
      continue;
    }
    float *Vout = bufs[k & 1];
    double c1, c2, cw;
    int32_t dot_y, slot, slot_gg = -1;
    bool write = true;
    if (method == ENT_CHEBYSHEV) {
      if (k == 0) {
        c1 = 1.0; c2 = -1.0; cw = 0.0;
        slot_gg = 0;
      } else {
        c1 = 2.0; c2 = -2.0; cw = -1.0;
      }
      dot_y = 0;
      slot = k + 1;
    } else {
      c1 = -1.0; c2 = 1.0; cw = 0.0;
      dot_y = 1;
      slot = k;
      write = k < nsteps - 1;
    }
    ent::Bf16GemmArgs ga{};
    ga.A_hi = Ahi; ga.A_lo = Alo; ga.V_hi = Vhi; ga.V_lo = Vlo; ga.part_y = party;
    ga.n_pad = n_pad; ga.ldv = ldv; ga.k_per_split = kps; ga.splits = splits; ga.bn = bn;
    const int e0 = pe.mark();
    HIP_TRY(ent::launch_bf16x3_gemm(ga, st));
    const int e1 = pe.mark();
    ent::Bf16EpiArgs ea{};
    ea.part_y = party; ea.splits = splits; ea.Vk = Vk; ea.Vkm1 = Vkm1;
    ea.Vkp1 = write ? Vout : nullptr; ea.V_hi = Vhi; ea.V_lo = Vlo; ea.G = G; ea.scal = scal;
    ea.c1 = c1; ea.c2 = c2; ea.cw = cw; ea.dot_y = dot_y; ea.slot = slot; ea.slot_gg = slot_gg;
    ea.scale_y = 1;
    ea.part = part; ea.nblk = nblk; ea.n_pad = n_pad; ea.ldv = ldv;
    HIP_TRY(ent::launch_bf16x3_epilogue(ea, st));
    const int e2 = pe.mark();
    if (pe.on) {
      pe.main_spans.push_back({e0, e1});
      pe.epi_spans.push_back({e1, e2});
    }
    if (method == ENT_CHEBYSHEV) Vkm1 = Vk;
    Vk = Vout;
  }
  pe.steps_end = pe.mark();
  HIP_TRY(ent::launch_reduce_moments(part, nslot, nblk, ldv, s, d, st));
  HIP_TRY(ent::launch_final(d, scal, clenshaw ? ent::FINAL_CLENSHAW : method, m, s, h, st));
  if (hook && hook->alpha_host)
    HIP_TRY(hipMemcpyAsync(hook->alpha_host, scal + ent::S_ALPHA, sizeof(double) * (m + 1),
                           hipMemcpyDeviceToHost, st));
  double hs[16];
  HIP_TRY(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, st));
  if (per_probe) HIP_TRY(hipMemcpyAsync(per_probe, h, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  if (moments)
    HIP_TRY(hipMemcpyAsync(moments, d, sizeof(double) * (m + 1) * s, hipMemcpyDeviceToHost, st));
  pe.mark();
  HIP_TRY(hipStreamSynchronize(st));
  pe.finish();
  if (check_trace) {
    double tol = o.trace_tol > 0 ? o.trace_tol : (f64 ? 1e-10 : 1e-4);
    if (!(std::fabs(hs[ent::S_TRACE] / op.trace_div - 1.0) <= tol))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g, not 1 within %.3g",
                  hs[ent::S_TRACE] / op.trace_div, tol);
  }
  if (normalize) {
    const double tr = hs[ent::S_TRACE] / op.trace_div;
    if (!(tr > 0) || !std::isfinite(1.0 / tr))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g: R cannot be normalised to unit trace", tr);
  }
  if (hs[ent::S_FLAG] != 0.0)
    return fail(ENT_ENUMERIC, "numeric failure: p1~ = %.17g, u = %.17g, estimate = %.17g",
                hs[ent::S_P1], hs[ent::S_U], hs[ent::S_ENT]);
  out->entropy = hs[ent::S_ENT];
  out->std_err = hs[ent::S_SE];
  out->p1_est = use_power ? hs[ent::S_P1] : 0.0;
  out->u = hs[ent::S_U];
  out->lo = hs[ent::S_LO];
  out->degree = m;
  out->probes = s;
  out->method = method;
  out->precision = ENT_BF16X3;
  out->fell_back = 0;
  out->products = (method == ENT_CHEBYSHEV) ? m : m + 1;
  return ENT_OK;
}


// ---------------------------------------------------------------------------
// Learned degree / cutoff selector (ENT_AUTO)
// ---------------------------------------------------------------------------
constexpr int32_t kFeatDegree = 12, kFeatProbes = 16;
constexpr int32_t kRouteSketch = 128;  // random-projection width of the low-rank route

struct SelectorState {
  float *params = nullptr;  // device copy of the MLP parameters
  float *feat = nullptr;    // 16 features
  float *y = nullptr;       // 2 outputs
};
std::mutex g_sel_mu;
std::map<int, SelectorState> g_sel;

ent_status poly_dispatch(const ent_matrix *R, int32_t method, int32_t m, int32_t s, uint64_t seed,
                         const Opts &op, ent_result *out, double *per_probe, double *moments,
                         const SelHook *hook) {
  switch (op.o.precision) {
    case ENT_F64: return run_poly<double>(R, method, m, s, seed, op, out, per_probe, moments, hook);
    case ENT_F32: return run_poly<float>(R, method, m, s, seed, op, out, per_probe, moments, hook);
    default: return run_bf16x3(R, method, m, s, seed, op, out, per_probe, moments, hook);
  }
}

// Highest degree a selector stage reaches (the projection coefficients on
// [lo, u] are independent of the degree up to 511).
constexpr int32_t kStageMaxDegree = 511;

// Maps the network outputs to (m, lo): y0 = ln m*, y1 = log10(lo*/u), where
// lo = 0 is trained as -6 (useful cutoffs lie in [10^-4.75, 10^-1.25] u) and
// decoded below -5.25.  A 25% degree margin and half a decade of cutoff
// margin are applied.
void selector_decode(const float y[2], double u, int32_t *m, double *lo) {
  double md = std::exp((double)y[0]) * 1.25;
  if (!(md > 4.0)) md = 4.0;
  if (md > 400.0) md = 400.0;
  *m = (int32_t)std::ceil(md - 1e-3);  // tolerate FP32 rounding of the output
  const double z = (double)y[1];
  *lo = (z < -5.25) ? 0.0 : u * std::pow(10.0, std::min(z, 0.0) - 0.5);
}

// Numerical rank from the sketch's normalised moments mu_k = feat[2 + k]
// (k = 1..12; mu_0 = 1): the share of the spectrum near 0 is the mean of
// h(X) = ((1 - X) / 2)^12 over the eigenvalues, X = 2R/u - 1 (h = 1 at
// x = 0, (1 - x/u)^12 elsewhere), expanded in Chebyshev polynomials of
// degree <= 12 by repeated products with 0.5 T_0 - 0.5 T_1
// (T_1 T_k = (T_{k+1} + T_{|k-1|}) / 2).  Returns n (1 - that share).
double selector_rank(const float feat[16], int64_t n) {
  double c[kFeatDegree + 2] = {1.0};
  for (int q = 0; q < kFeatDegree; ++q) {
    double nc[kFeatDegree + 2] = {0.0};
    for (int k = 0; k <= q; ++k) {
      nc[k] += 0.5 * c[k];
      nc[k + 1] -= 0.25 * c[k];
      nc[k == 0 ? 1 : k - 1] -= 0.25 * c[k];
    }
    std::memcpy(c, nc, sizeof(c));
  }
  double zero = c[0];
  for (int k = 1; k <= kFeatDegree; ++k) zero += c[k] * (double)feat[2 + k];
  return (double)n * (1.0 - zero);
}

// A-posteriori check: every moment bounded by ||g||^2 (the spectrum stayed in
// [lo, u]) and the partial sums converged: |H(m) - H(m-4)| <= 2.5e-4 |H(m)|.
// The a-posteriori check in two parts: -1 if some |d_kj| exceeds ||g_j||^2
// (an eigenvalue outside the interval: T_k grows there, and a higher degree
// does not help), 0 if the partial sums at degrees m and m - 4 differ by more
// than 2.5e-4 relative (not converged yet), 1 if both pass.
int selector_stage_check(const std::vector<double> &mom, const std::vector<double> &alpha, int32_t m,
                         int32_t s) {
  for (int32_t k = 0; k <= m; ++k)
    for (int32_t j = 0; j < s; ++j)
      if (!(std::fabs(mom[(size_t)k * s + j]) <= (1.0 + 1e-6) * mom[j])) return -1;
  auto partial = [&](int32_t mm) {
    double acc = 0.0;
    for (int32_t j = 0; j < s; ++j) {
      double v = 0.0;
      for (int32_t k = 0; k <= mm; ++k) v -= alpha[k] * mom[(size_t)k * s + j];
      acc += v;
    }
    return acc / s;
  };
  const double hm = partial(m), h4 = partial(std::max(m - 4, 0));
  if (!std::isfinite(hm)) return -1;
  return std::fabs(hm - h4) <= 2.5e-4 * std::fabs(hm) ? 1 : 0;
}

bool selector_check(const std::vector<double> &mom, const std::vector<double> &alpha, int32_t m,
                    int32_t s) {
  return selector_stage_check(mom, alpha, m, s) == 1;
}

// The selector's sketch pass: power method and a degree-12 Chebyshev moment
// pass with 16 Rademacher probes on [0, u], FP32 -- or FP64 for a CSR R
// stored in FP64 (CSR values are read in their stored precision) -- then the
// features and the network on the device; y receives the network's outputs.
ent_status feature_pass(const ent_matrix *R, uint64_t seed, const Opts &op, const SelectorState &st,
                        float y[2], ent_result *fr, float *feat = nullptr) {
  const bool csr64 = R->layout == ENT_CSR && R->dtype == ENT_STORE_F64;
  Opts fo = op;
  fo.o.precision = csr64 ? ENT_F64 : ENT_F32;
  fo.o.u_fixed = 0.0;
  fo.o.cutoff = 0.0;
  fo.o.probe_dist = ENT_RADEMACHER;
  fo.o.flags &= ~ENT_FLAG_CLENSHAW;
  SelHook fh;
  fh.feat_dev = st.feat;
  fh.params_dev = st.params;
  fh.y_dev = st.y;
  fh.y_host = y;
  fh.feat_host = feat;
  const uint64_t fseed = seed ^ 0x5E1EC7ull;
  if (csr64)
    return run_poly<double>(R, ENT_CHEBYSHEV, kFeatDegree, kFeatProbes, fseed, fo, fr, nullptr, nullptr, &fh);
  return run_poly<float>(R, ENT_CHEBYSHEV, kFeatDegree, kFeatProbes, fseed, fo, fr, nullptr, nullptr, &fh);
}

ent_status run_randproj(const ent_matrix *R, uint64_t seed, const Opts &op, ent_result *out,
                        double *sigma_out);

ent_status run_auto(const ent_matrix *R, int32_t m_plain, int32_t s, uint64_t seed, const Opts &op,
                    ent_result *out, double *per_probe, double *moments) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  SelectorState st;
  {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    auto it = g_sel.find(dev);
    if (it == g_sel.end() || !it->second.params)
      return fail(ENT_EINVAL, "ENT_AUTO needs a selector: call ent_selector_load first");
    st = it->second;
  }
  // 1. sketch pass: power method + degree-12 Chebyshev moments with 16 probes
  float y[2] = {0.f, 0.f}, feat[16] = {};
  ent_result fr{};
  ent_status rc = feature_pass(R, seed, op, st, y, &fr, feat);
  if (rc != ENT_OK) return rc;
  // 1b. on request, a numerically low-rank R (sketch rank at most 1/8 of the
  // random projection's width) goes to Algorithm 3 (Section 5): one product;
  // kept if the k singular values hold the unit trace (within 5%)
  int32_t products = kFeatDegree;
  const int32_t s_rp = op.o.sketch_width > 0 ? op.o.sketch_width : kRouteSketch;
  if ((op.o.flags & ENT_FLAG_AUTO_RANDPROJ) && R->layout == ENT_DENSE &&
      selector_rank(feat, R->n) <= s_rp / 8.0) {
    Opts ro = op;
    ro.o.sketch_width = s_rp;
    ro.o.rank_k = op.o.rank_k > 0 ? std::min(op.o.rank_k, s_rp) : s_rp / 2;
    ro.o.sketch = ENT_SKETCH_GAUSSIAN;
    std::vector<double> sig(ro.o.rank_k);
    ent_result r{};
    rc = run_randproj(R, seed, ro, &r, sig.data());
    if (rc != ENT_OK) return rc;
    ++products;
    double held = 0.0;
    for (double v : sig) held += v;
    if (std::fabs(held - 1.0) <= 0.05) {  // tr R = 1 (checked, or normalised)
      r.p1_est = fr.p1_est;
      r.u = fr.u;
      r.method = ENT_RANDPROJ;
      r.fell_back = 0;
      r.products = products;
      if (per_probe) std::fill(per_probe, per_probe + s, r.entropy);
      if (moments) std::fill(moments, moments + (size_t)(m_plain + 1) * s, 0.0);
      *out = r;
      return ENT_OK;
    }
  }
  int32_t m_hat = 0;
  double lo = 0.0;
  selector_decode(y, fr.u, &m_hat, &lo);
  // 2. main pass on [lo, u] with the predicted degree (power method reused).
  // Where the check finds the spectrum inside the interval but the partial
  // sums not converged, the same recurrence continues to 1.5x and then 2.25x
  // the degree (at most kStageMaxDegree, where the coefficients on [lo, u]
  // are still nested) before the fallback; the BF16x3 form has no stages.
  Opts mo = op;
  mo.o.u_fixed = fr.u;
  mo.o.cutoff = lo;
  DegreeStages ds;
  ds.check = selector_stage_check;
  ds.deg[ds.count++] = m_hat;
  if (op.o.precision != ENT_BF16X3) {
    for (double f : {1.5, 2.25}) {
      const int32_t mm = std::min(kStageMaxDegree, (int32_t)std::ceil(f * m_hat));
      if (mm > ds.deg[ds.count - 1]) ds.deg[ds.count++] = mm;
    }
  }
  const int32_t m_top = ds.deg[ds.count - 1];
  std::vector<double> mom((size_t)(m_top + 1) * s), alpha(m_top + 1);
  SelHook mh;
  mh.alpha_host = alpha.data();
  if (op.o.precision != ENT_BF16X3) mh.stages = &ds;
  ent_result r{};
  rc = poly_dispatch(R, ENT_CHEBYSHEV, mh.stages ? m_top : m_hat, s, seed, mo, &r, per_probe, mom.data(), &mh);
  const int32_t m_used = mh.stages ? ds.used : m_hat;
  bool ok = rc == ENT_OK && (mh.stages ? ds.passed != 0 : selector_check(mom, alpha, m_hat, s));
  products += m_used;
  if (ok) {
    // the caller's table has (m_plain + 1) rows: copy the rows that fit
    if (moments) {
      const int32_t rows = std::min(m_used, m_plain) + 1;
      std::memcpy(moments, mom.data(), sizeof(double) * (size_t)rows * s);
      std::fill(moments + (size_t)rows * s, moments + (size_t)(m_plain + 1) * s, 0.0);
    }
  } else {
    // 3. fallback: the plain schedule on [0, u] with the caller's degree
    Opts po = op;
    po.o.u_fixed = fr.u;
    po.o.cutoff = 0.0;
    rc = poly_dispatch(R, ENT_CHEBYSHEV, m_plain, s, seed, po, &r, per_probe, moments, nullptr);
    if (rc != ENT_OK) return rc;
    products += m_plain;
  }
  r.p1_est = fr.p1_est;
  r.method = ENT_AUTO;
  r.fell_back = ok ? 0 : 1;
  r.products = products;
  *out = r;
  return ENT_OK;
}

// ---------------------------------------------------------------------------
// Random projection (Algorithm 3): R~ = R Pi on the MFMA product kernels,
// Gram matrix and its eigenvalues in FP64, top-k singular values.
// ---------------------------------------------------------------------------
ent_status run_randproj(const ent_matrix *R, uint64_t seed, const Opts &op, ent_result *out,
                        double *sigma_out) {
  const ent_options &o = op.o;
  hipStream_t st = op.st;
  const int32_t s = o.sketch_width, k = o.rank_k;
  if (R->layout != ENT_DENSE) return fail(ENT_EUNSUPPORTED, "random projection needs dense R");
  if (s < 1 || s > 256) return fail(ENT_EINVAL, "sketch_width = %d out of range [1, 256]", s);
  if (o.sketch < ENT_SKETCH_GAUSSIAN || o.sketch > ENT_SKETCH_COUNT)
    return fail(ENT_EINVAL, "unknown sketch %d", o.sketch);
  if (k < 1 || k > s) return fail(ENT_EINVAL, "rank_k = %d out of range [1, sketch_width]", k);
  ent_status mrc = check_matrix_memory(R);
  if (mrc != ENT_OK) return mrc;
  const int64_t n = R->n;
  const bool f64 = R->dtype == ENT_STORE_F64;
  const int prec = o.precision;
  const int32_t N = (s + 1) / 2 * 2;
  const int32_t nsplit = 64;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceWorkspace *ws = workspace_for(dev);
  std::lock_guard<std::mutex> lk(ws->mu);
  double *scal = nullptr, *gp = nullptr, *G = nullptr, *work = nullptr, *eig = nullptr, *sig = nullptr;
  Carve cv;
  cv.add(&scal, kScalarDoubles);
  cv.add(&gp, (size_t)nsplit * s * s);
  cv.add(&G, (size_t)s * s);
  cv.add(&work, (size_t)N * N);
  cv.add(&eig, (size_t)N);
  cv.add(&sig, (size_t)k);
  const bool normalize = (o.flags & ENT_FLAG_NORMALIZE) != 0;
  const bool check_trace = !(o.flags & ENT_FLAG_SKIP_TRACE_CHECK) && !normalize;
  PhaseEvents pe;
  pe.on = g_timing_on;
  pe.st = st;
  if (o.sketch == ENT_SKETCH_COUNT) {
    // one signed pass over R into Y = (R Pi)^T, FP64 from the stored values
    // (the precision option does not apply)
    const int64_t ldy = round_up(n, 64);
    int32_t *cnt = nullptr, *rows = nullptr;
    int64_t *off = nullptr;
    double *Y = nullptr;
    cv.add(&cnt, (size_t)s);
    cv.add(&off, (size_t)s + 1);
    cv.add(&rows, (size_t)n);
    cv.add(&Y, (size_t)s * ldy);
    ent_status rc = ensure_workspace(ws, cv.total());
    if (rc != ENT_OK) return rc;
    cv.assign(ws->ptr);
    pe.mark();
    HIP_TRY(ent::launch_fill(scal, 64, 0.0, st));
    if (check_trace || normalize) {
      if (f64)
        HIP_TRY(ent::launch_trace_dense<double>((const double *)R->values, R->ld, n, scal, st));
      else
        HIP_TRY(ent::launch_trace_dense<float>((const float *)R->values, R->ld, n, scal, st));
    }
    if (normalize) HIP_TRY(ent::launch_set_norm(scal, op.trace_div, st));
    if (f64)
      HIP_TRY(ent::launch_count_sketch<double>((const double *)R->values, R->ld, n, s, seed, cnt, off, rows,
                                               Y, ldy, st, 0));
    else
      HIP_TRY(ent::launch_count_sketch<float>((const float *)R->values, R->ld, n, s, seed, cnt, off, rows, Y,
                                              ldy, st, 0));
    pe.steps_begin = pe.mark();
    if (f64)
      HIP_TRY(ent::launch_count_sketch<double>((const double *)R->values, R->ld, n, s, seed, cnt, off, rows,
                                               Y, ldy, st, 1));
    else
      HIP_TRY(ent::launch_count_sketch<float>((const float *)R->values, R->ld, n, s, seed, cnt, off, rows, Y,
                                              ldy, st, 1));
    pe.steps_end = pe.mark();
    HIP_TRY(ent::launch_gram<double>(Y, 1, ldy, n, s, gp, nsplit, G, st));
  } else if (prec == ENT_BF16X3) {
    const int64_t n_pad = round_up(n, 128);
    const int bn = s <= 64 ? 64 : (s <= 128 ? 128 : 256);
    const int64_t ldv = round_up(s, bn);
    const int64_t tiles = (n_pad / ent::bf16x3_tile_rows(n_pad)) * (ldv / bn);
    const int32_t splits = ent::bf16x3_splits(n_pad, tiles);
    uint16_t *Ahi = nullptr, *Alo = nullptr, *Phi = nullptr, *Plo = nullptr;
    float *P = nullptr, *X = nullptr, *party = nullptr;
    cv.add(&Ahi, (size_t)n_pad * n_pad);
    cv.add(&Alo, (size_t)n_pad * n_pad);
    cv.add(&P, (size_t)ldv * n_pad);
    cv.add(&X, (size_t)ldv * n_pad);
    cv.add(&Phi, (size_t)ldv * n_pad);
    cv.add(&Plo, (size_t)ldv * n_pad);
    cv.add(&party, (size_t)splits * ldv * n_pad);
    ent_status rc = ensure_workspace(ws, cv.total());
    if (rc != ENT_OK) return rc;
    cv.assign(ws->ptr);
    pe.mark();
    HIP_TRY(ent::launch_fill(scal, 64, 0.0, st));
    HIP_TRY(ent::launch_fill(scal + ent::S_A, 1, 1.0, st));
    if (check_trace || normalize) {
      if (f64)
        HIP_TRY(ent::launch_trace_dense<double>((const double *)R->values, R->ld, n, scal, st));
      else
        HIP_TRY(ent::launch_trace_dense<float>((const float *)R->values, R->ld, n, scal, st));
    }
    if (normalize) HIP_TRY(ent::launch_set_norm(scal, op.trace_div, st));
    HIP_TRY(ent::launch_probe_gen_t(P, Phi, Plo, n, n_pad, s, ldv, seed,
                                    o.sketch == ENT_SKETCH_SRHT ? 2 : ENT_GAUSSIAN, st, 2u,
                                    1.0 / std::sqrt((double)s)));
    if (f64)
      HIP_TRY(ent::launch_split_matrix<double>((const double *)R->values, R->ld, n, n_pad, scal, Ahi, Alo, st));
    else
      HIP_TRY(ent::launch_split_matrix<float>((const float *)R->values, R->ld, n, n_pad, scal, Ahi, Alo, st));
    pe.steps_begin = pe.mark();
    ent::Bf16GemmArgs ga{};
    ga.A_hi = Ahi; ga.A_lo = Alo; ga.V_hi = Phi; ga.V_lo = Plo; ga.part_y = party;
    ga.n_pad = n_pad; ga.ldv = ldv; ga.k_per_split = n_pad / splits; ga.splits = splits; ga.bn = bn;
    HIP_TRY(ent::launch_bf16x3_gemm(ga, st));
    const int e1 = pe.mark();
    ent::Bf16EpiArgs ea{};
    ea.part_y = party; ea.splits = splits; ea.Vk = P; ea.Vkp1 = X; ea.V_hi = Phi; ea.V_lo = Plo;
    ea.G = P; ea.scal = scal; ea.c1 = 1.0; ea.c2 = 0.0; ea.cw = 0.0; ea.slot = -1; ea.slot_gg = -1;
    ea.nblk = ent::bf16x3_epilogue_blocks(n_pad); ea.n_pad = n_pad; ea.ldv = ldv;
    HIP_TRY(ent::launch_bf16x3_epilogue(ea, st));
    const int e2 = pe.mark();
    if (pe.on) {
      pe.main_spans.push_back({pe.steps_begin, e1});
      pe.epi_spans.push_back({e1, e2});
    }
    pe.steps_end = e2;
    HIP_TRY(ent::launch_gram<float>(X, 1, n_pad, n, s, gp, nsplit, G, st));
  } else {
    const bool d64 = prec == ENT_F64;
    const size_t esz = d64 ? 8 : 4;
    const int ve = d64 ? 2 : 4;
    const bool stored_T = f64 == d64;
    const bool copy = !stored_T || (R->ld % ve) != 0 || ((uintptr_t)R->values % 16) != 0;
    const int64_t n_pad = round_up(n, 64);
    const int bn = s <= 64 ? 64 : (s <= 128 ? 128 : 256);
    const int64_t ldv = round_up(s, bn);
    const int64_t ldc = round_up(n, ve);
    char *Rc = nullptr, *P = nullptr, *X = nullptr;
    if (copy) cv.add(&Rc, (size_t)n * ldc * esz);
    cv.add(&P, (size_t)n_pad * ldv * esz);
    cv.add(&X, (size_t)n_pad * ldv * esz);
    ent_status rc = ensure_workspace(ws, cv.total());
    if (rc != ENT_OK) return rc;
    cv.assign(ws->ptr);
    pe.mark();
    HIP_TRY(ent::launch_fill(scal, 64, 0.0, st));
    HIP_TRY(ent::launch_fill(scal + ent::S_A, 1, 1.0, st));
    if (check_trace || normalize) {
      if (f64)
        HIP_TRY(ent::launch_trace_dense<double>((const double *)R->values, R->ld, n, scal, st));
      else
        HIP_TRY(ent::launch_trace_dense<float>((const float *)R->values, R->ld, n, scal, st));
    }
    if (normalize) HIP_TRY(ent::launch_set_norm(scal, op.trace_div, st));
    const void *Rt = R->values;
    int64_t ldr = R->ld;
    if (copy) {
      if (f64 && d64) HIP_TRY((ent::launch_convert<double, double>((const double *)Rt, R->ld, (double *)Rc, ldc, n, n, st)));
      if (f64 && !d64) HIP_TRY((ent::launch_convert<double, float>((const double *)Rt, R->ld, (float *)Rc, ldc, n, n, st)));
      if (!f64 && d64) HIP_TRY((ent::launch_convert<float, double>((const float *)Rt, R->ld, (double *)Rc, ldc, n, n, st)));
      if (!f64 && !d64) HIP_TRY((ent::launch_convert<float, float>((const float *)Rt, R->ld, (float *)Rc, ldc, n, n, st)));
      Rt = Rc;
      ldr = ldc;
    }
    if (d64)
      HIP_TRY(ent::launch_sketch_gen<double>((double *)P, n, n_pad, s, ldv, seed, o.sketch, st));
    else
      HIP_TRY(ent::launch_sketch_gen<float>((float *)P, n, n_pad, s, ldv, seed, o.sketch, st));
    ent::DenseStepArgs a{};
    a.R = Rt; a.ldr = ldr; a.n = n; a.ldv = ldv; a.Vk = P; a.Vkm1 = nullptr; a.Vkp1 = X; a.G = nullptr;
    a.scal = scal; a.c1 = 1.0; a.c2 = 0.0; a.cw = 0.0; a.dot_y = 0; a.slot = -1; a.slot_gg = -1;
    a.part = nullptr; a.ntile = (int32_t)(n_pad / 64); a.bn = bn;
    pe.steps_begin = pe.mark();
    if (d64)
      HIP_TRY(ent::launch_dense_step<double>(a, st));
    else
      HIP_TRY(ent::launch_dense_step<float>(a, st));
    pe.steps_end = pe.mark();
    if (d64)
      HIP_TRY(ent::launch_gram<double>((const double *)X, ldv, 1, n, s, gp, nsplit, G, st));
    else
      HIP_TRY(ent::launch_gram<float>((const float *)X, ldv, 1, n, s, gp, nsplit, G, st));
  }
  HIP_TRY(ent::launch_rp_spectrum(G, s, k, work, eig, sig, scal, st));
  double hs[16];
  HIP_TRY(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, st));
  if (sigma_out) HIP_TRY(hipMemcpyAsync(sigma_out, sig, sizeof(double) * k, hipMemcpyDeviceToHost, st));
  pe.mark();
  HIP_TRY(hipStreamSynchronize(st));
  pe.finish();
  if (check_trace) {
    const double tol = o.trace_tol > 0 ? o.trace_tol : (f64 ? 1e-10 : 1e-4);
    if (!(std::fabs(hs[ent::S_TRACE] / op.trace_div - 1.0) <= tol))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g, not 1 within %.3g",
                  hs[ent::S_TRACE] / op.trace_div, tol);
  }
  if (normalize) {
    const double tr = hs[ent::S_TRACE] / op.trace_div;
    if (!(tr > 0) || !std::isfinite(1.0 / tr))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g: R cannot be normalised to unit trace", tr);
  }
  if (hs[ent::S_FLAG] != 0.0) return fail(ENT_ENUMERIC, "non-finite random-projection estimate");
  out->entropy = hs[ent::S_ENT];
  out->std_err = 0.0;
  out->p1_est = 0.0;
  out->u = 0.0;
  out->lo = 0.0;
  out->degree = k;
  out->probes = s;
  out->method = ENT_RANDPROJ;
  out->precision = prec;
  out->fell_back = 0;
  out->products = 1;
  return ENT_OK;
}

// ---------------------------------------------------------------------------
// Batches of dense matrices: one launch per phase over every matrix (grouped
// kernels driven by device descriptor and tile tables), captured once into a
// hipGraph.  The step tile shape (64- or 128-row tiles) is chosen by timing
// both on the batch itself.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;  // autotune cache: key -> rows-per-wave factor
bool g_tune_loaded = false;

std::string tune_cache_path() {
  const char *p = std::getenv("ENT_AUTOTUNE_CACHE");
  return p ? std::string(p) : std::string();
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char key[400];
    int v = 0;
    if (std::sscanf(line, " \"%399[^\"]\" : %d", key, &v) == 2) g_tune[key] = v;
  }
  std::fclose(f);
}

void tune_store_locked() {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE *f = std::fopen(path.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (auto &kv : g_tune)
    std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < g_tune.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
}

}  // namespace

struct ent_graph_s {
  int dev = 0;
  hipStream_t stream = nullptr;
  int32_t count = 0, method = 0, m = 0, s = 0, nslot = 0;
  ent_options o{};
  bool src_f64 = false, comp_f64 = false;
  int64_t ldv = 0, sb = 0, max_n = 0, max_npad = 0, max_elems = 0, xlen = 0;
  int32_t wr = 1, ntiles1 = 0, ntiles2 = 0, nptiles = 0;
  std::vector<ent::BatchMat> mats;
  std::vector<int2> tiles1, tiles2, ptiles;
  ent::BatchMat *mats_d = nullptr;
  int2 *tiles1_d = nullptr, *tiles2_d = nullptr, *ptiles_d = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  char *Rc = nullptr, *G = nullptr, *VA = nullptr, *VB = nullptr;
  double *x0 = nullptr, *x1 = nullptr, *p0 = nullptr, *norm = nullptr;
  double *part = nullptr, *d = nullptr, *h = nullptr, *scal = nullptr;
  double *host_scal = nullptr;
  // BF16x3 batches: split of every R, bf16 probe blocks, FP32 products
  bool bf16 = false;
  uint16_t *Ahi = nullptr, *Alo = nullptr, *Vhi[2] = {nullptr, nullptr}, *Vlo[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool launched = false;
  // Recurrence steps: window == 0 runs one grouped launch per step; window
  // > 0 runs one persistent launch that walks a schedule of (matrix, row
  // tile, step) items built with that window (bytes of matrix data in
  // flight), one segment of the schedule per XCD holding workgroups
  size_t window = 0;
  int32_t grid_p = 0, nitems = 0, spin_limit = 1 << 20;
  int32_t nseg = 0;                            // 0: XCDs not probed yet
  int32_t seg_off[ent::kMaxXcc + 1] = {};      // items of segment s: [seg_off[s], seg_off[s + 1])
  int32_t seg_of_xcc[ent::kMaxXcc];            // hardware XCC id -> segment, -1: no workgroups
  int32_t seg_wgs[ent::kMaxXcc] = {};          // workgroups of the grid on each segment's XCD
  int4 *items_d = nullptr;
  int32_t *xcc_d = nullptr;  // [kXccProbe] XCC id of each probe workgroup
  // [0, kMaxXcc) next item of each segment, [kMaxXcc] error flag,
  // [kMaxXcc + 1 + b] finished tiles of matrix b
  int32_t *sched = nullptr;
};

constexpr int32_t kXccProbe = 4096;
constexpr int32_t kSchedErr = ent::kMaxXcc;
constexpr int32_t kSchedDone = ent::kMaxXcc + 1;

namespace {

// The m recurrence steps of an FP32 / FP64 batch as one grouped launch per
// step (every row tile of every matrix).
template <typename T>
ent_status enqueue_steps_grouped(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  const int32_t nsteps = (g->method == ENT_CHEBYSHEV) ? g->m : g->m + 1;
  const T *Vk = (const T *)g->G, *Vkm1 = nullptr;
  T *bufs[2] = {(T *)g->VA, (T *)g->VB};
  if (pe) pe->steps_begin = pe->mark();
  for (int32_t k = 0; k < nsteps; ++k) {
    T *Vout = bufs[k & 1];
    ent::BatchStepArgs ba{};
    ent::DenseStepArgs &a = ba.base;
    a.ldv = g->ldv;
    a.Vk = Vk;
    a.G = g->G;
    a.part = g->part;
    a.bn = 64;
    if (g->method == ENT_CHEBYSHEV) {
      a.dot_y = 0;
      a.slot = k + 1;
      if (k == 0) {
        a.c1 = 1.0; a.c2 = -1.0; a.cw = 0.0;
        a.slot_gg = 0;
      } else {
        a.c1 = 2.0; a.c2 = -2.0; a.cw = -1.0;
        a.slot_gg = -1;
      }
      a.Vkm1 = Vkm1;
      a.Vkp1 = Vout;
    } else {
      a.c1 = -1.0; a.c2 = 1.0; a.cw = 0.0;
      a.dot_y = 1;
      a.slot = k;
      a.slot_gg = -1;
      a.Vkp1 = (k < nsteps - 1) ? Vout : nullptr;
    }
    ba.mats = g->mats_d;
    ba.tiles = g->wr == 2 ? g->tiles2_d : g->tiles1_d;
    HIP_TRY(ent::launch_batch_dense_step<T>(ba, g->wr == 2 ? g->ntiles2 : g->ntiles1, g->wr, st));
    if (g->method == ENT_CHEBYSHEV) Vkm1 = Vk;
    Vk = Vout;
    if (pe) {
      const int e = pe->mark();
      if (k == nsteps - 1) pe->steps_end = e;
    }
  }
  return ENT_OK;
}

// The m recurrence steps of a BF16x3 batch as one grouped launch per step.
ent_status enqueue_steps_grouped_bf16(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  const int32_t nsteps = (g->method == ENT_CHEBYSHEV) ? g->m : g->m + 1;
  const float *Vk = (const float *)g->G, *Vkm1 = nullptr;
  float *bufs[2] = {(float *)g->VA, (float *)g->VB};
  if (pe) pe->steps_begin = pe->mark();
  for (int32_t k = 0; k < nsteps; ++k) {
    float *Vout = bufs[k & 1];
    ent::Bf16EpiArgs ea{};
    bool write = true;
    if (g->method == ENT_CHEBYSHEV) {
      ea.dot_y = 0;
      ea.slot = k + 1;
      if (k == 0) {
        ea.c1 = 1.0; ea.c2 = -1.0; ea.cw = 0.0;
        ea.slot_gg = 0;
      } else {
        ea.c1 = 2.0; ea.c2 = -2.0; ea.cw = -1.0;
        ea.slot_gg = -1;
      }
    } else {
      ea.c1 = -1.0; ea.c2 = 1.0; ea.cw = 0.0;
      ea.dot_y = 1;
      ea.slot = k;
      ea.slot_gg = -1;
      write = k < nsteps - 1;
    }
    // fused step: product + epilogue; V_k hi/lo in set k % 2, V_{k+1} hi/lo to the other
    ea.Vk = Vk;
    ea.Vkm1 = (g->method == ENT_CHEBYSHEV && k > 0) ? Vkm1 : nullptr;
    ea.Vkp1 = write ? Vout : nullptr; ea.V_hi = g->Vhi[(k + 1) & 1]; ea.V_lo = g->Vlo[(k + 1) & 1];
    ea.G = (const float *)g->G; ea.scale_y = 1; ea.part = g->part; ea.ldv = g->ldv;
    HIP_TRY(ent::launch_batch_bf16x3_step(ea, g->mats_d, g->tiles2_d, g->ntiles2, g->Ahi, g->Alo,
                                          g->Vhi[k & 1], g->Vlo[k & 1], st));
    if (pe) {
      const int e = pe->mark();
      if (k == nsteps - 1) pe->steps_end = e;
    }
    if (g->method == ENT_CHEBYSHEV) Vkm1 = Vk;
    Vk = Vout;
  }
  return ENT_OK;
}

// The m recurrence steps as one persistent launch over the batch's schedule
// (counters cleared by a kernel first, so the sequence can be captured).
ent_status enqueue_steps_persistent(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  const int32_t nsteps = (g->method == ENT_CHEBYSHEV) ? g->m : g->m + 1;
  HIP_TRY(ent::launch_zero(g->sched, sizeof(int32_t) * (kSchedDone + (size_t)g->count), st));
  ent::BatchPersistArgs pa{};
  pa.sched.items = g->items_d;
  pa.sched.nitems = g->nitems;
  pa.sched.spin_limit = g->spin_limit;
  pa.sched.nseg = g->nseg;
  for (int q = 0; q <= ent::kMaxXcc; ++q) pa.sched.seg_off[q] = g->seg_off[q];
  for (int q = 0; q < ent::kMaxXcc; ++q) pa.sched.seg_of_xcc[q] = g->seg_of_xcc[q];
  pa.sched.head = g->sched;
  pa.sched.err = g->sched + kSchedErr;
  pa.sched.done = g->sched + kSchedDone;
  pa.mats = g->mats_d;
  pa.method = g->method;
  pa.nsteps = nsteps;
  pa.ldv = g->ldv;
  pa.G = g->G;
  pa.VA = g->VA;
  pa.VB = g->VB;
  pa.part = g->part;
  pa.Ahi = g->Ahi;
  pa.Alo = g->Alo;
  for (int q = 0; q < 2; ++q) {
    pa.Vhi[q] = g->Vhi[q];
    pa.Vlo[q] = g->Vlo[q];
  }
  if (pe) pe->steps_begin = pe->mark();
  if (g->bf16)
    HIP_TRY(ent::launch_batch_bf16x3_persistent(pa, g->grid_p, st));
  else if (g->comp_f64)
    HIP_TRY(ent::launch_batch_dense_persistent<double>(pa, g->wr, g->grid_p, st));
  else
    HIP_TRY(ent::launch_batch_dense_persistent<float>(pa, g->wr, g->grid_p, st));
  HIP_TRY(ent::launch_sched_check(pa.sched, st));  // a segment no workgroup reached is an error
  if (pe) {
    pe->steps_end = pe->mark();
    pe->logical_steps = nsteps;
  }
  return ENT_OK;
}

ent_status batch_enqueue_steps(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  if (g->window > 0) return enqueue_steps_persistent(g, st, pe);
  if (g->bf16) return enqueue_steps_grouped_bf16(g, st, pe);
  return g->comp_f64 ? enqueue_steps_grouped<double>(g, st, pe) : enqueue_steps_grouped<float>(g, st, pe);
}

template <typename T>
ent_status enqueue_batch(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  const ent_options &o = g->o;
  const int32_t count = g->count;
  HIP_TRY(ent::launch_fill(g->scal, (int64_t)count * g->sb, 0.0, st));
  if (g->src_f64)
    HIP_TRY((ent::launch_batch_convert<double, T>(g->mats_d, count, g->max_elems, st)));
  else
    HIP_TRY((ent::launch_batch_convert<float, T>(g->mats_d, count, g->max_elems, st)));
  if (!(o.flags & ENT_FLAG_SKIP_TRACE_CHECK) || (o.flags & ENT_FLAG_NORMALIZE))
    HIP_TRY(ent::launch_batch_trace<T>(g->mats_d, count, st));
  HIP_TRY(ent::launch_batch_probes<T>(g->mats_d, count, g->max_npad, (T *)g->G, g->s, g->ldv,
                                      o.probe_dist, st));
  if (!(o.u_fixed > 0)) {
    if (pe) pe->power_begin = pe->mark();
    for (int32_t trial = 0; trial < o.power_trials; ++trial) {
      HIP_TRY(ent::launch_batch_power_start(g->mats_d, count, g->max_n, g->x0, trial, st));
      double *xin = g->x0, *xout = g->x1;
      const double *in_norm = nullptr;
      for (int32_t it = 0; it <= o.power_iters; ++it) {
        HIP_TRY(ent::launch_batch_power_gemv<T>(g->mats_d, g->ptiles_d, g->nptiles, xin, in_norm,
                                                xout, g->p0, st));
        HIP_TRY(ent::launch_batch_power_reduce(g->mats_d, count, g->p0, g->norm, st));
        std::swap(xin, xout);
        in_norm = g->norm;
      }
      HIP_TRY(ent::launch_batch_power_rq(g->mats_d, count, g->norm, trial, st));
    }
    if (pe) {
      pe->power_end = pe->mark();
      pe->power_launches = o.power_trials * (o.power_iters + 1);
    }
  }
  HIP_TRY(ent::launch_batch_setup(g->mats_d, count, g->method, g->m, o.u_factor, o.u_fixed,
                                  o.cutoff, st, (o.flags & ENT_FLAG_NORMALIZE) ? 1.0 : 0.0));
  ent_status rc = batch_enqueue_steps(g, st, pe);
  if (rc != ENT_OK) return rc;
  HIP_TRY(ent::launch_batch_reduce(g->mats_d, count, g->part, g->nslot, g->ldv, g->s, g->d, st));
  HIP_TRY(ent::launch_batch_final(g->mats_d, count, g->d, g->method, g->m, g->s, g->h, st));
  return ENT_OK;
}

// BF16x3 batch: split each R once (unscaled), power method on the split, then
// per step one grouped GEMM over every (matrix, 128-row tile) and one grouped
// epilogue (the interval scale a is applied there).
ent_status enqueue_batch_bf16(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  const ent_options &o = g->o;
  const int32_t count = g->count;
  HIP_TRY(ent::launch_fill(g->scal, (int64_t)count * g->sb, 0.0, st));
  if (!(o.flags & ENT_FLAG_SKIP_TRACE_CHECK) || (o.flags & ENT_FLAG_NORMALIZE)) {
    if (g->src_f64)
      HIP_TRY(ent::launch_batch_trace<double>(g->mats_d, count, st));
    else
      HIP_TRY(ent::launch_batch_trace<float>(g->mats_d, count, st));
  }
  if (g->src_f64)
    HIP_TRY(ent::launch_batch_split<double>(g->mats_d, g->tiles2_d, g->ntiles2, g->Ahi, g->Alo, st));
  else
    HIP_TRY(ent::launch_batch_split<float>(g->mats_d, g->tiles2_d, g->ntiles2, g->Ahi, g->Alo, st));
  HIP_TRY(ent::launch_batch_probe_t(g->mats_d, g->tiles2_d, g->ntiles2, (float *)g->G, g->Vhi[0],
                                    g->Vlo[0], g->s, g->ldv, o.probe_dist, st));
  if (!(o.u_fixed > 0)) {
    if (pe) pe->power_begin = pe->mark();
    // the split is zero beyond n, and so must be the vectors it multiplies
    HIP_TRY(ent::launch_fill(g->x0, g->xlen, 0.0, st));
    HIP_TRY(ent::launch_fill(g->x1, g->xlen, 0.0, st));
    for (int32_t trial = 0; trial < o.power_trials; ++trial) {
      HIP_TRY(ent::launch_batch_power_start(g->mats_d, count, g->max_n, g->x0, trial, st));
      double *xin = g->x0, *xout = g->x1;
      const double *in_norm = nullptr;
      for (int32_t it = 0; it <= o.power_iters; ++it) {
        HIP_TRY(ent::launch_batch_power_split(g->mats_d, g->ptiles_d, g->nptiles, g->Ahi, g->Alo, xin,
                                              in_norm, xout, g->p0, st));
        HIP_TRY(ent::launch_batch_power_reduce(g->mats_d, count, g->p0, g->norm, st));
        std::swap(xin, xout);
        in_norm = g->norm;
      }
      HIP_TRY(ent::launch_batch_power_rq(g->mats_d, count, g->norm, trial, st));
    }
    if (pe) {
      pe->power_end = pe->mark();
      pe->power_launches = o.power_trials * (o.power_iters + 1);
    }
  }
  HIP_TRY(ent::launch_batch_setup(g->mats_d, count, g->method, g->m, o.u_factor, o.u_fixed,
                                  o.cutoff, st, (o.flags & ENT_FLAG_NORMALIZE) ? 1.0 : 0.0));
  ent_status rc = batch_enqueue_steps(g, st, pe);
  if (rc != ENT_OK) return rc;
  HIP_TRY(ent::launch_batch_reduce(g->mats_d, count, g->part, g->nslot, g->ldv, g->s, g->d, st));
  HIP_TRY(ent::launch_batch_final(g->mats_d, count, g->d, g->method, g->m, g->s, g->h, st));
  return ENT_OK;
}

ent_status batch_enqueue(ent_graph_s *g, hipStream_t st, PhaseEvents *pe) {
  if (g->bf16) return enqueue_batch_bf16(g, st, pe);
  return g->comp_f64 ? enqueue_batch<double>(g, st, pe) : enqueue_batch<float>(g, st, pe);
}

// Bytes a matrix keeps in use while its steps run: R in the compute layout
// (BF16x3: its hi/lo split) and its V blocks.
size_t batch_matrix_bytes(const ent_graph_s *g, const ent::BatchMat &M) {
  const size_t v = (size_t)M.n_pad * (size_t)g->ldv;
  if (g->bf16) return 4 * (size_t)M.n_pad * (size_t)M.n_pad + v * 20;
  const size_t esz = g->comp_f64 ? 8 : 4;
  return esz * ((size_t)M.n * (size_t)M.ldr + 3 * v);
}

// The persistent schedule of one segment: its matrices in decreasing n enter
// a window while their bytes fit `window` (at least one at a time); every
// round emits the next step of each matrix in the window, all its row tiles,
// so a matrix's data is reused across its steps while it stays cached, and a
// step's items come one round after those of the step before.  A matrix
// leaves the window after its last step.
void batch_schedule_segment(const ent_graph_s *g, std::vector<int32_t> order, size_t window,
                            int32_t tile_rows, std::vector<int4> &items) {
  const int32_t nsteps = (g->method == ENT_CHEBYSHEV) ? g->m : g->m + 1;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return g->mats[a].n > g->mats[b].n; });
  struct Active {
    int32_t b, k;
  };
  std::vector<Active> act;
  size_t next = 0, bytes = 0;
  while (next < order.size() || !act.empty()) {
    while (next < order.size()) {
      const size_t mb = batch_matrix_bytes(g, g->mats[order[next]]);
      if (!act.empty() && bytes + mb > window) break;
      act.push_back({order[next], 0});
      bytes += mb;
      ++next;
    }
    for (auto &a : act) {
      const int32_t nt = (int32_t)(g->mats[a.b].n_pad / tile_rows);
      for (int32_t t = 0; t < nt; ++t) items.push_back(make_int4(a.b, t, a.k, 0));
      ++a.k;
    }
    std::vector<Active> keep;
    for (auto &a : act) {
      if (a.k < nsteps)
        keep.push_back(a);
      else
        bytes -= batch_matrix_bytes(g, g->mats[a.b]);
    }
    act.swap(keep);
  }
}

// Matrices to segments (XCDs) by longest processing time first, a matrix's
// cost its bytes (each step streams them once), each segment's load divided
// by its workgroups; then each segment's schedule, its window the segment's
// share of `window`.  Fills seg_off; returns the items, segment by segment.
std::vector<int4> batch_schedule(ent_graph_s *g, size_t window, int32_t tile_rows) {
  const int32_t ns = g->nseg;
  std::vector<int32_t> order(g->count);
  for (int32_t b = 0; b < g->count; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return batch_matrix_bytes(g, g->mats[a]) > batch_matrix_bytes(g, g->mats[b]);
  });
  std::vector<double> load(ns, 0.0);
  std::vector<std::vector<int32_t>> members(ns);
  int64_t wgs = 0;
  for (int32_t q = 0; q < ns; ++q) wgs += g->seg_wgs[q];
  for (int32_t b : order) {
    int32_t best = 0;
    double best_t = 1e300;
    const double c = (double)batch_matrix_bytes(g, g->mats[b]);
    for (int32_t q = 0; q < ns; ++q) {
      const double t = (load[q] + c) / g->seg_wgs[q];
      if (t < best_t) {
        best_t = t;
        best = q;
      }
    }
    load[best] += c;
    members[best].push_back(b);
  }
  std::vector<int4> items;
  for (int32_t q = 0; q < ns; ++q) {
    g->seg_off[q] = (int32_t)items.size();
    const size_t share = (size_t)((double)window * g->seg_wgs[q] / (double)wgs);
    batch_schedule_segment(g, members[q], share, tile_rows, items);
  }
  for (int32_t q = ns; q <= ent::kMaxXcc; ++q) g->seg_off[q] = (int32_t)items.size();
  return items;
}

// Which XCDs the persistent grid's workgroups run on (probed once with a
// grid of the same size; workgroups are dealt to XCDs by index).
ent_status batch_probe_xcc(ent_graph_s *g) {
  const int32_t n = g->grid_p < kXccProbe ? g->grid_p : kXccProbe;
  HIP_TRY(ent::launch_xcc_probe(g->xcc_d, n, g->stream));
  std::vector<int32_t> ids(n);
  HIP_TRY(hipMemcpyAsync(ids.data(), g->xcc_d, sizeof(int32_t) * n, hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  int32_t per[ent::kMaxXcc] = {};
  for (int32_t id : ids) ++per[id & (ent::kMaxXcc - 1)];
  g->nseg = 0;
  for (int32_t x = 0; x < ent::kMaxXcc; ++x) {
    g->seg_of_xcc[x] = -1;
    if (per[x] > 0) {
      g->seg_of_xcc[x] = g->nseg;
      g->seg_wgs[g->nseg++] = per[x];
    }
  }
  if (g->nseg < 1) return fail(ENT_EDEVICE, "XCD probe of the persistent grid found no workgroups");
  return ENT_OK;
}

// Select the step schedule: window 0 = one grouped launch per step; else the
// persistent launch over the schedule built with that window (uploaded here).
ent_status batch_set_schedule(ent_graph_s *g, size_t window) {
  g->window = window;
  if (window == 0) return ENT_OK;
  g->grid_p = ent::batch_persistent_grid(g->bf16 ? ENT_BF16X3 : (g->comp_f64 ? ENT_F64 : ENT_F32), g->wr, g->ldv);
  if (g->grid_p < 1) return fail(ENT_EDEVICE, "no occupancy for the persistent step kernel");
  if (g->nseg == 0) {
    const ent_status rc = batch_probe_xcc(g);
    if (rc != ENT_OK) return rc;
  }
  const std::vector<int4> items = batch_schedule(g, window, g->bf16 ? 128 : 64 * g->wr);
  g->nitems = (int32_t)items.size();
  HIP_TRY(hipMemcpy(g->items_d, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice));
  return ENT_OK;
}

// Upload descriptors with the row-tile count of the chosen tile shape.
ent_status batch_upload(ent_graph_s *g, int wr) {
  for (auto &M : g->mats) M.ntile = (int32_t)(M.n_pad / (64 * wr));
  HIP_TRY(hipMemcpyAsync(g->mats_d, g->mats.data(), sizeof(ent::BatchMat) * g->mats.size(),
                         hipMemcpyHostToDevice, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  g->wr = wr;
  return ENT_OK;
}

// Candidate schedules of the autotuner (bytes of matrix data in flight,
// split over the XCDs; 0 = one grouped launch per step): the 256 MB Infinity
// Cache, two, four and eight times it, and every matrix at once.  Narrow
// windows keep a matrix cached across its steps but leave each XCD few tiles
// per round; on 1024 matrices, n ~ U[64, 2048], s = 64, m = 40, the step time
// per recurrence step was 2.71 / 1.85 / 1.52 / 1.63 / 1.68 ms in BF16x3 for
// 256 MB .. all against 1.64 ms for grouped launches, and 5.15 / 3.01 / 2.06 /
// 2.03 / 2.03 ms in FP32 against 2.04 ms.  The default is 1 GB.
constexpr size_t kWindows[] = {0, (size_t)256 << 20, (size_t)512 << 20, (size_t)1024 << 20,
                               (size_t)2048 << 20, (size_t)65536 << 20};
constexpr int kDefaultWindow = 3;

// Time the recurrence steps of every candidate (tile shape x schedule) on the
// batch's own buffers, after one full run has filled them; keep the fastest.
ent_status batch_autotune(ent_graph_s *g, bool stepwise_only) {
  ent_status rc = batch_upload(g, g->bf16 ? 2 : 1);
  if (rc != ENT_OK) return rc;
  rc = batch_set_schedule(g, 0);
  if (rc != ENT_OK) return rc;
  rc = batch_enqueue(g, g->stream, nullptr);  // fills every buffer with real data
  if (rc != ENT_OK) return rc;
  HIP_TRY(hipStreamSynchronize(g->stream));
  float best = 1e30f;
  int best_wr = g->bf16 ? 2 : 1;
  size_t best_win = 0;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (int wr = g->bf16 ? 2 : 1; wr <= 2 && rc == ENT_OK; ++wr) {
    rc = batch_upload(g, wr);
    for (size_t win : kWindows) {
      if (rc != ENT_OK) break;
      if (stepwise_only && win > 0) continue;
      rc = batch_set_schedule(g, win);
      if (rc != ENT_OK) break;
      rc = batch_enqueue_steps(g, g->stream, nullptr);  // warm
      if (rc != ENT_OK) break;
      (void)hipEventRecord(e0, g->stream);
      rc = batch_enqueue_steps(g, g->stream, nullptr);
      (void)hipEventRecord(e1, g->stream);
      if (rc != ENT_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(ENT_EDEVICE, "autotune timing failed");
        break;
      }
      int32_t err = 0;
      if (win > 0 && hipMemcpy(&err, g->sched + kSchedErr, sizeof(err), hipMemcpyDeviceToHost) == hipSuccess && err)
        continue;  // a bounded wait expired: not a candidate
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        best_wr = wr;
        best_win = win;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != ENT_OK) return rc;
  rc = batch_upload(g, best_wr);
  if (rc != ENT_OK) return rc;
  return batch_set_schedule(g, best_win);
}

std::string batch_tune_key(const ent_graph_s *g) {
  int64_t sum2 = 0;
  for (auto &M : g->mats) sum2 += M.n * M.n;
  int bucket = 0;
  while ((int64_t(1) << (bucket + 1)) <= sum2) ++bucket;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "gfx950|%s|batch|count=%d|log2sum_n2=%d|s=%d|maxn=%lld|m=%d|%s",
                g->bf16 ? "bf16x3" : (g->comp_f64 ? "f64" : "f32"), g->count, bucket, g->s,
                (long long)g->max_n, g->m, (g->o.flags & ENT_FLAG_BATCH_STEPWISE) ? "stepwise" : "any");
  return buf;
}

void batch_free(ent_graph_s *g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->ws) (void)hipFree(g->ws);
  if (g->host_scal) (void)hipHostFree(g->host_scal);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

ent_status batch_create(const ent_matrix *Rs, int32_t count, int32_t method, int32_t m, int32_t s,
                        uint64_t seed, const ent_options *opt, bool capture, ent_graph_s **out) {
  if (!Rs) return fail(ENT_EINVAL, "Rs is NULL");
  if (count < 1) return fail(ENT_EINVAL, "count = %d < 1", count);
  if (method != ENT_TAYLOR && method != ENT_CHEBYSHEV)
    return fail(ENT_EINVAL, "batches support the Taylor and Chebyshev methods");
  if (m < 1 || m > 4000) return fail(ENT_EINVAL, "degree = %d out of range [1, 4000]", m);
  if (s < 1) return fail(ENT_EINVAL, "probes = %d < 1", s);
  Opts op = resolve_options(opt);
  ent_status rc = validate_options(op.o);
  if (rc != ENT_OK) return rc;
  if (method == ENT_TAYLOR && op.o.cutoff > 0)
    return fail(ENT_EINVAL, "cutoff applies to the Chebyshev method only");
  if (op.o.flags & ENT_FLAG_CLENSHAW)
    return fail(ENT_EUNSUPPORTED, "batches use the forward recurrence (no Clenshaw schedule)");
  for (int32_t b = 0; b < count; ++b) {
    rc = validate_matrix(&Rs[b]);
    if (rc != ENT_OK) return fail(rc, "matrix %d: %s", b, g_last_error.c_str());
    if (Rs[b].layout != ENT_DENSE) return fail(ENT_EUNSUPPORTED, "matrix %d: batches are dense only", b);
    if (Rs[b].dtype != Rs[0].dtype) return fail(ENT_EINVAL, "matrix %d: mixed storage types", b);
  }
  for (int32_t b = 0; b < count; ++b) {
    rc = check_matrix_memory(&Rs[b]);
    if (rc != ENT_OK) return fail(rc, "matrix %d: %s", b, g_last_error.c_str());
  }
  auto *g = new ent_graph_s();
  g->count = count;
  g->method = method;
  g->m = m;
  g->s = s;
  g->nslot = m + 1;
  g->o = op.o;
  g->src_f64 = Rs[0].dtype == ENT_STORE_F64;
  g->comp_f64 = op.o.precision == ENT_F64;
  g->bf16 = op.o.precision == ENT_BF16X3;
  const size_t esz = g->comp_f64 ? 8 : 4;
  g->ldv = round_up(s, 64);
  if (g->bf16) {
    // one probe tile per matrix in the grouped GEMM: 64, 128 or 256 probes
    if (s > 256) {
      delete g;
      return fail(ENT_EUNSUPPORTED, "BF16x3 batches take at most 256 probes");
    }
    g->ldv = s <= 64 ? 64 : (s <= 128 ? 128 : 256);
  }
  g->sb = round_up(ent::S_ALPHA + m + 1 + 8, 32);
  auto fail_free = [&](ent_status st) {
    batch_free(g);
    return st;
  };
  if (hipGetDevice(&g->dev) != hipSuccess) return fail_free(fail(ENT_EDEVICE, "hipGetDevice failed"));
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess)
    return fail_free(fail(ENT_EDEVICE, "hipStreamCreate failed"));
  // layout of every per-matrix region
  int64_t roff = 0, voff = 0, poff = 0, xoff = 0, pboff = 0, aoff = 0;
  g->mats.resize(count);
  for (int32_t b = 0; b < count; ++b) {
    ent::BatchMat &M = g->mats[b];
    const int64_t n = Rs[b].n;
    M.src = Rs[b].values;
    M.ldsrc = Rs[b].ld;
    M.ldr = round_up(n, 8);
    M.n = n;
    M.n_pad = round_up(n, 128);
    M.ntile = (int32_t)(M.n_pad / (g->bf16 ? 128 : 64));
    M.pblk = g->bf16 ? ent::power_blocks_split(M.n_pad) : ent::power_blocks_dense(n);
    M.seed = seed + (uint64_t)b;
    M.R = (const void *)(intptr_t)roff;  // offsets for now; rebased below
    M.voff = voff;
    M.poff = poff;
    M.xoff = xoff;
    M.pboff = pboff;
    M.aoff = aoff;
    M.doff = (int64_t)b * g->nslot * s;
    M.hoff = (int64_t)b * s;
    if (g->bf16) {
      // the split reads the caller's matrix; the trace check reads it too
      M.R = Rs[b].values;
      M.ldr = Rs[b].ld;
      aoff += M.n_pad * M.n_pad;
    } else {
      roff += n * M.ldr;
    }
    voff += M.n_pad * g->ldv;
    poff += (int64_t)g->nslot * M.ntile * g->ldv;
    xoff += M.n_pad;
    pboff += 3 * (int64_t)M.pblk;
    g->max_n = std::max(g->max_n, n);
    g->max_npad = std::max(g->max_npad, M.n_pad);
    g->max_elems = std::max(g->max_elems, n * M.ldr);
  }
  // tile tables, largest matrices first (their tiles are the longest)
  std::vector<int32_t> order(count);
  for (int32_t b = 0; b < count; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return g->mats[a].n > g->mats[b].n; });
  for (int32_t b : order) {
    const ent::BatchMat &M = g->mats[b];
    for (int32_t t = 0; t < (int32_t)(M.n_pad / 64); ++t) g->tiles1.push_back(make_int2(b, t));
    for (int32_t t = 0; t < (int32_t)(M.n_pad / 128); ++t) g->tiles2.push_back(make_int2(b, t));
    for (int32_t t = 0; t < M.pblk; ++t) g->ptiles.push_back(make_int2(b, t));
  }
  g->ntiles1 = (int32_t)g->tiles1.size();
  g->ntiles2 = (int32_t)g->tiles2.size();
  g->nptiles = (int32_t)g->ptiles.size();
  g->xlen = xoff;
  Carve cv;
  cv.add(&g->mats_d, (size_t)count);
  cv.add(&g->tiles1_d, g->tiles1.size());
  cv.add(&g->tiles2_d, g->tiles2.size());
  cv.add(&g->ptiles_d, g->ptiles.size());
  if (g->bf16) {
    cv.add(&g->Ahi, (size_t)aoff);
    cv.add(&g->Alo, (size_t)aoff);
    for (int q = 0; q < 2; ++q) {
      cv.add(&g->Vhi[q], (size_t)voff);
      cv.add(&g->Vlo[q], (size_t)voff);
    }
  }
  cv.add(&g->scal, (size_t)count * g->sb);
  if (!g->bf16) cv.add(&g->Rc, (size_t)roff * esz);
  cv.add(&g->G, (size_t)voff * esz);
  cv.add(&g->VA, (size_t)voff * esz);
  cv.add(&g->VB, (size_t)voff * esz);
  cv.add(&g->x0, (size_t)xoff);
  cv.add(&g->x1, (size_t)xoff);
  cv.add(&g->p0, (size_t)pboff);
  cv.add(&g->norm, (size_t)4 * count);
  cv.add(&g->part, (size_t)poff);
  cv.add(&g->d, (size_t)count * g->nslot * s);
  cv.add(&g->h, (size_t)count * s);
  {
    // persistent schedule: every (matrix, row tile, step) item at the
    // smallest tile shape, and the counters
    const int32_t nsteps = (method == ENT_CHEBYSHEV) ? m : m + 1;
    size_t items = 0;
    for (auto &M : g->mats) items += (size_t)(M.n_pad / 64) * nsteps;
    cv.add(&g->items_d, items);
    cv.add(&g->xcc_d, (size_t)kXccProbe);
    cv.add(&g->sched, kSchedDone + (size_t)count);
  }
  g->ws_bytes = cv.total();
  if (g_ws_limit && g->ws_bytes > g_ws_limit)
    return fail_free(fail(ENT_ENOMEM, "batch workspace of %zu bytes exceeds the limit", g->ws_bytes));
  if (hipMalloc(&g->ws, g->ws_bytes) != hipSuccess) {
    (void)hipGetLastError();
    g->ws = nullptr;
    return fail_free(fail(ENT_ENOMEM, "hipMalloc(%zu) for the batch failed", g->ws_bytes));
  }
  cv.assign(g->ws);
  if (hipHostMalloc((void **)&g->host_scal, sizeof(double) * count * g->sb, hipHostMallocDefault) !=
      hipSuccess)
    return fail_free(fail(ENT_ENOMEM, "pinned host buffer allocation failed"));
  for (int32_t b = 0; b < count; ++b) {
    ent::BatchMat &M = g->mats[b];
    if (!g->bf16) M.R = g->Rc + (intptr_t)M.R * esz;
    M.scal = g->scal + (int64_t)b * g->sb;
  }
  if (hipMemcpy(g->tiles1_d, g->tiles1.data(), sizeof(int2) * g->tiles1.size(), hipMemcpyHostToDevice) ||
      hipMemcpy(g->tiles2_d, g->tiles2.data(), sizeof(int2) * g->tiles2.size(), hipMemcpyHostToDevice) ||
      hipMemcpy(g->ptiles_d, g->ptiles.data(), sizeof(int2) * g->ptiles.size(), hipMemcpyHostToDevice))
    return fail_free(fail(ENT_EDEVICE, "descriptor upload failed"));
  // tile shape and step schedule: cached choice, else timed on this batch
  // when asked, else 64-row tiles (BF16x3: 128-row GEMM tiles) and the
  // persistent schedule with a 1 GB window
  if (const char *env = std::getenv("ENT_SCHED_SPIN_LIMIT")) g->spin_limit = std::atoi(env);
  const bool stepwise = (op.o.flags & ENT_FLAG_BATCH_STEPWISE) != 0;
  const std::string key = batch_tune_key(g);
  int choice = -1;  // wr | (window in MB) << 2
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) choice = it->second;
  }
  if (choice < 0 && (op.o.flags & ENT_FLAG_AUTOTUNE)) {
    rc = batch_autotune(g, stepwise);
    if (rc != ENT_OK) return fail_free(rc);
    choice = g->wr | (int)((g->window >> 20) << 2);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = choice;
    tune_store_locked();
  }
  if (choice < 0) choice = (g->bf16 ? 2 : 1) | (stepwise ? 0 : (int)((kWindows[kDefaultWindow] >> 20) << 2));
  rc = batch_upload(g, g->bf16 ? 2 : ((choice & 3) == 2 ? 2 : 1));
  if (rc != ENT_OK) return fail_free(rc);
  rc = batch_set_schedule(g, stepwise ? 0 : ((size_t)(choice >> 2) << 20));
  if (rc != ENT_OK) return fail_free(rc);
  if (capture) {
    if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail_free(fail(ENT_EDEVICE, "hipStreamBeginCapture failed"));
    rc = batch_enqueue(g, g->stream, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(g->stream, &graph);
    if (rc != ENT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail_free(rc);
    }
    if (ce != hipSuccess) return fail_free(fail(ENT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ce)));
    g->graph = graph;
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
      return fail_free(fail(ENT_EDEVICE, "hipGraphInstantiate failed"));
  }
  *out = g;
  return ENT_OK;
}

// Copy the scalar blocks back and fill the results (after the work ran).
ent_status batch_collect(ent_graph_s *g, ent_result *outs) {
  HIP_TRY(hipMemcpyAsync(g->host_scal, g->scal, sizeof(double) * g->count * g->sb,
                         hipMemcpyDeviceToHost, g->stream));
  int32_t sched_err = 0;
  if (g->window > 0)
    HIP_TRY(hipMemcpyAsync(&sched_err, g->sched + kSchedErr, sizeof(sched_err), hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  if (sched_err & 1)
    return fail(ENT_EDEVICE, "a step of the persistent schedule waited longer than its bound (%d polls) "
                             "for its matrix's previous step", g->spin_limit);
  if (sched_err)
    return fail(ENT_EDEVICE, "a segment of the persistent schedule was not run: no workgroup of the launch "
                             "reached its XCD");
  g->launched = true;
  const bool normalize = (g->o.flags & ENT_FLAG_NORMALIZE) != 0;
  const bool check = !(g->o.flags & ENT_FLAG_SKIP_TRACE_CHECK) && !normalize;
  const double tol = g->o.trace_tol > 0 ? g->o.trace_tol : ((g->src_f64 && g->comp_f64) ? 1e-10 : 1e-4);
  for (int32_t b = 0; b < g->count; ++b) {
    const double *hs = g->host_scal + (int64_t)b * g->sb;
    if (check && !(std::fabs(hs[ent::S_TRACE] - 1.0) <= tol))
      return fail(ENT_ENOTDENSITY, "matrix %d: trace %.17g is not 1 within %.3g", b, hs[ent::S_TRACE], tol);
    if (normalize && (!(hs[ent::S_TRACE] > 0) || !std::isfinite(1.0 / hs[ent::S_TRACE])))
      return fail(ENT_ENOTDENSITY, "matrix %d: trace %.17g cannot be normalised to 1", b, hs[ent::S_TRACE]);
    if (hs[ent::S_FLAG] != 0.0)
      return fail(ENT_ENUMERIC, "matrix %d: numeric failure (p1~ = %.17g)", b, hs[ent::S_P1]);
  }
  for (int32_t b = 0; b < g->count; ++b) {
    const double *hs = g->host_scal + (int64_t)b * g->sb;
    ent_result &r = outs[b];
    r.entropy = hs[ent::S_ENT];
    r.std_err = hs[ent::S_SE];
    r.p1_est = (g->o.u_fixed > 0) ? 0.0 : hs[ent::S_P1];
    r.u = hs[ent::S_U];
    r.lo = hs[ent::S_LO];
    r.degree = g->m;
    r.probes = g->s;
    r.method = g->method;
    r.precision = g->o.precision;
    r.fell_back = 0;
    r.products = (g->method == ENT_CHEBYSHEV) ? g->m : g->m + 1;
  }
  return ENT_OK;
}

// ---------------------------------------------------------------------------
// Hermitian R (Section 4, Algorithms 1c / 2c).  R = B + iC is replaced by its
// real form M = [[B, -C], [C, B]] (2n x 2n); the recurrence on M with probes
// [g; 0] equals the complex recurrence on R with the real probe g, and its
// quadratic forms are g^T Re[f(R)] g.  tr M = 2 tr R and lambda_max(M) =
// lambda_max(R).  The interval is [0, 1] (the paper's u = 1 for Hermitian
// inputs) unless the caller fixes u or asks for the power method on M.
// Holds the device's real-form buffer for the duration of `body`.
// ---------------------------------------------------------------------------
template <typename F>
ent_status with_real_form(const ent_matrix *R, hipStream_t st, F body) {
  const int64_t n = R->n, n2 = 2 * n;
  const bool c128 = R->dtype == ENT_STORE_C128;
  const int64_t ldm = round_up(n2, 4);
  const size_t bytes = (size_t)n2 * (size_t)ldm * (c128 ? 8 : 4);
  if (g_ws_limit && bytes > g_ws_limit)
    return fail(ENT_ENOMEM, "real form of %zu bytes exceeds the workspace limit of %zu bytes", bytes,
                g_ws_limit.load());
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  RealFormBuffer *b = real_form_for(dev);
  std::lock_guard<std::mutex> lk(b->mu);
  if (b->bytes < bytes) {
    if (b->ptr) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(b->ptr));
      b->ptr = nullptr;
      b->bytes = 0;
    }
    if (hipMalloc(&b->ptr, bytes) != hipSuccess) {
      (void)hipGetLastError();
      b->ptr = nullptr;
      return fail(ENT_ENOMEM, "could not allocate the %zu-byte real form of R", bytes);
    }
    b->bytes = bytes;
  }
  if (c128)
    HIP_TRY((ent::launch_realify<double, double>((const double *)R->values, R->ld, n, (double *)b->ptr,
                                                 ldm, st)));
  else
    HIP_TRY((ent::launch_realify<float, float>((const float *)R->values, R->ld, n, (float *)b->ptr, ldm,
                                               st)));
  ent_matrix M{};
  M.n = n2;
  M.layout = ENT_DENSE;
  M.dtype = c128 ? ENT_STORE_F64 : ENT_STORE_F32;
  M.ld = ldm;
  M.values = b->ptr;
  return body(M);
}

ent_status run_hermitian(const ent_matrix *R, int32_t method, int32_t m, int32_t s, uint64_t seed,
                         const Opts &op, ent_result *out, double *per_probe, double *moments) {
  if (method != ENT_TAYLOR && method != ENT_CHEBYSHEV)
    return fail(ENT_EUNSUPPORTED, "Hermitian R: Taylor and Chebyshev estimators only");
  Opts mop = op;
  mop.probe_rows = R->n;
  mop.trace_div = 2.0;
  if (!(mop.o.u_fixed > 0) && !(mop.o.flags & ENT_FLAG_COMPLEX_POWER)) mop.o.u_fixed = 1.0;
  return with_real_form(R, op.st, [&](const ent_matrix &M) {
    return poly_dispatch(&M, method, m, s, seed, mop, out, per_probe, moments, nullptr);
  });
}

// Frees the per-device buffers of one map (each after its device is idle);
// the first failure is reported, the remaining buffers are still freed.
template <typename Buf>
ent_status free_buffers(std::mutex &map_mu, std::map<int, Buf *> &bufs) {
  ent_status rc = ENT_OK;
  std::lock_guard<std::mutex> lk(map_mu);
  for (auto &kv : bufs) {
    std::lock_guard<std::mutex> l2(kv.second->mu);
    if (!kv.second->ptr) continue;
    hipError_t e = hipSetDevice(kv.first);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFree(kv.second->ptr);
    if (e != hipSuccess) {
      if (rc == ENT_OK) rc = fail(ENT_EDEVICE, "releasing a buffer on device %d: %s", kv.first, hipGetErrorString(e));
      continue;
    }
    kv.second->ptr = nullptr;
    kv.second->bytes = 0;
  }
  return rc;
}

// Algorithm 4 on a device-resident R (validated, arrays checked).
ent_status power_method_device(const ent_matrix *R, int32_t t, int32_t q, uint64_t seed, void *stream,
                               double *p1) {
  ent_status rc = ENT_OK;
  hipStream_t st = (hipStream_t)stream;
  if (is_complex(R))
    return with_real_form(R, st, [&](const ent_matrix &M) { return power_method_device(&M, t, q, seed, stream, p1); });
  const int64_t n = R->n, n_pad = round_up(n, 64);
  const int32_t pblk = (int32_t)power_blocks(R);
  const bool f64 = R->dtype == ENT_STORE_F64;
  const int ve = f64 ? 2 : 4;
  const bool copy = R->layout == ENT_DENSE && ((R->ld % ve) != 0 || ((uintptr_t)R->values % 16) != 0);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceWorkspace *ws = workspace_for(dev);
  std::lock_guard<std::mutex> lk(ws->mu);
  double *scal, *x0, *x1, *p0, *pp1;
  void *Rc = nullptr;
  const int64_t ldc = round_up(n, ve);
  Carve cv;
  cv.add(&scal, kScalarDoubles);
  cv.add(&x0, n_pad);
  cv.add(&x1, n_pad);
  cv.add(&p0, 3 * (size_t)pblk);
  cv.add(&pp1, 4);
  if (copy) cv.add((char **)&Rc, (size_t)n * ldc * (f64 ? 8 : 4));
  rc = ensure_workspace(ws, cv.total());
  if (rc != ENT_OK) return rc;
  cv.assign(ws->ptr);
  rc = check_csr(R, scal, st);
  if (rc != ENT_OK) return rc;
  if (f64) {
    const double *Rt = (const double *)R->values;
    int64_t ldr = R->ld;
    if (copy) {
      HIP_TRY((ent::launch_convert<double, double>(Rt, R->ld, (double *)Rc, ldc, n, n, st)));
      Rt = (const double *)Rc;
      ldr = ldc;
    }
    rc = enqueue_power<double>(R, Rt, ldr, t, q, seed, x0, x1, p0, pp1, scal, st);
  } else {
    const float *Rt = (const float *)R->values;
    int64_t ldr = R->ld;
    if (copy) {
      HIP_TRY((ent::launch_convert<float, float>(Rt, R->ld, (float *)Rc, ldc, n, n, st)));
      Rt = (const float *)Rc;
      ldr = ldc;
    }
    rc = enqueue_power<float>(R, Rt, ldr, t, q, seed, x0, x1, p0, pp1, scal, st);
  }
  if (rc != ENT_OK) return rc;
  double v = 0;
  HIP_TRY(hipMemcpyAsync(&v, scal + ent::S_P1, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *p1 = v;
  return ENT_OK;
}

static_assert(ENT_NOALLOC_SCRATCH_BYTES == ent::kNoAllocScratchBytes,
              "the header's scratch size is the library's");

// Argument rules shared by the polynomial estimate entry points.
ent_status check_poly_args(int32_t method, int32_t degree, int32_t probes, const Opts &op) {
  if (degree < 1) return fail(ENT_EINVAL, "degree = %d < 1", degree);
  if (degree > 4000) return fail(ENT_EINVAL, "degree = %d > 4000", degree);
  if (probes < 1) return fail(ENT_EINVAL, "probes = %d < 1", probes);
  if (method == ENT_TAYLOR && op.o.cutoff > 0)
    return fail(ENT_EINVAL, "cutoff applies to the Chebyshev method only");
  if ((op.o.flags & ENT_FLAG_CLENSHAW) && method != ENT_CHEBYSHEV)
    return fail(ENT_EINVAL, "the Clenshaw schedule applies to the Chebyshev method only");
  return ENT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void ent_options_default(ent_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->power_iters = 20;
  opt->power_trials = 1;
  opt->u_factor = 6.0;
  opt->precision = ENT_F64;
  opt->probe_dist = ENT_RADEMACHER;
}

ent_status ent_entropy_estimate_detail(const ent_matrix *R, int32_t method, int32_t degree,
                                       int32_t probes, uint64_t seed, const ent_options *opt,
                                       ent_result *out, double *per_probe, double *moments) {
  g_last_error.clear();
  ent_status rc = validate_matrix(R, true);
  if (rc != ENT_OK) return rc;
  if (!out) return fail(ENT_EINVAL, "out is NULL");
  Opts op = resolve_options(opt);
  rc = validate_options(op.o);
  if (rc != ENT_OK) return rc;
  if (is_complex(R) && (method == ENT_RANDPROJ || method == ENT_AUTO))
    return fail(ENT_EUNSUPPORTED, "Hermitian R: Taylor and Chebyshev estimators only");
  if (method == ENT_RANDPROJ) {
    ent_result tmp{};
    rc = with_device_copy(R, op.st, [&](const ent_matrix *D) { return run_randproj(D, seed, op, &tmp, per_probe); });
    if (rc == ENT_OK) *out = tmp;
    return rc;
  }
  if (method != ENT_TAYLOR && method != ENT_CHEBYSHEV && method != ENT_AUTO)
    return fail(ENT_EINVAL, "unknown method %d", method);
  rc = check_poly_args(method, degree, probes, op);
  if (rc != ENT_OK) return rc;
  ent_result tmp{};
  rc = with_device_copy(R, op.st, [&](const ent_matrix *D) {
    ent_status r2 = check_matrix_memory(D);
    if (r2 != ENT_OK) return r2;
    if (is_complex(D)) return run_hermitian(D, method, degree, probes, seed, op, &tmp, per_probe, moments);
    if (method == ENT_AUTO) return run_auto(D, degree, probes, seed, op, &tmp, per_probe, moments);
    return poly_dispatch(D, method, degree, probes, seed, op, &tmp, per_probe, moments, nullptr);
  });
  if (rc == ENT_OK) *out = tmp;
  return rc;
}

ent_status ent_entropy_estimate(const ent_matrix *R, int32_t method, int32_t degree, int32_t probes,
                                uint64_t seed, const ent_options *opt, ent_result *out) {
  return ent_entropy_estimate_detail(R, method, degree, probes, seed, opt, out, nullptr, nullptr);
}

ent_status ent_entropy_estimate_noalloc(const ent_matrix *R, int32_t method, int32_t degree,
                                        int32_t probes, uint64_t seed, const ent_options *opt,
                                        ent_result *out, double *per_probe, double *moments) {
  g_last_error.clear();
  ent_status rc = validate_matrix(R, false);
  if (rc != ENT_OK) return rc;
  if (!out) return fail(ENT_EINVAL, "out is NULL");
  Opts op = resolve_options(opt);
  rc = validate_options(op.o);
  if (rc != ENT_OK) return rc;
  if (method != ENT_TAYLOR && method != ENT_CHEBYSHEV)
    return fail(method == ENT_RANDPROJ || method == ENT_AUTO ? ENT_EUNSUPPORTED : ENT_EINVAL,
                "the no-allocation entry point runs the Taylor and Chebyshev estimators only (method %d)",
                method);
  rc = check_poly_args(method, degree, probes, op);
  if (rc != ENT_OK) return rc;
  // a host array would need a device copy, i.e. an allocation
  const void *arrays[3] = {R->values, R->layout == ENT_CSR ? (const void *)R->row_ptr : nullptr,
                           R->layout == ENT_CSR && R->nnz > 0 ? (const void *)R->col_idx : nullptr};
  for (const void *a : arrays)
    if (a && is_host_memory(a))
      return fail(ENT_EINVAL, "the no-allocation entry point takes device arrays only");
  rc = check_matrix_memory(R);
  if (rc != ENT_OK) return rc;
  op.no_alloc = true;
  ent_result tmp{};
  rc = poly_dispatch(R, method, degree, probes, seed, op, &tmp, per_probe, moments, nullptr);
  if (rc == ENT_OK) *out = tmp;
  return rc;
}

ent_status ent_power_method(const ent_matrix *R, int32_t t, int32_t q, uint64_t seed, void *stream,
                            double *p1) {
  g_last_error.clear();
  ent_status rc = validate_matrix(R, true);
  if (rc != ENT_OK) return rc;
  if (!p1) return fail(ENT_EINVAL, "p1 is NULL");
  if (t < 0 || q < 1) return fail(ENT_EINVAL, "need t >= 0 and q >= 1");
  return with_device_copy(R, (hipStream_t)stream, [&](const ent_matrix *D) {
    ent_status r2 = check_matrix_memory(D);
    if (r2 != ENT_OK) return r2;
    return power_method_device(D, t, q, seed, stream, p1);
  });
}

ent_status ent_chebyshev_coeffs(double lo, double u, int32_t m, double *alpha) {
  g_last_error.clear();
  if (!alpha) return fail(ENT_EINVAL, "alpha is NULL");
  if (m < 1 || m > 4000) return fail(ENT_EINVAL, "m = %d out of range [1, 4000]", m);
  if (!(lo >= 0) || !(u > lo) || !std::isfinite(u)) return fail(ENT_EINVAL, "need 0 <= lo < u");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceWorkspace *ws = workspace_for(dev);
  std::lock_guard<std::mutex> lk(ws->mu);
  ent_status rc = ensure_workspace(ws, sizeof(double) * kScalarDoubles);
  if (rc != ENT_OK) return rc;
  double *scal = (double *)ws->ptr;
  HIP_TRY(ent::launch_setup_interval(scal, ENT_CHEBYSHEV, m, 1.0, u, lo, nullptr));
  HIP_TRY(hipMemcpy(alpha, scal + ent::S_ALPHA, sizeof(double) * (m + 1), hipMemcpyDeviceToHost));
  return ENT_OK;
}

int32_t ent_probes_for(double eps, double delta) {
  if (!(eps > 0) || !(delta > 0) || !(delta < 1)) return -1;
  return (int32_t)std::ceil(20.0 * std::log(2.0 / delta) / (eps * eps));
}

int32_t ent_degree_taylor(double u, double ell, double eps) {
  if (!(ell > 0) || !(u >= ell) || !(eps > 0) || !(eps < 1)) return -1;
  return (int32_t)std::ceil((u / ell) * std::log(1.0 / eps));
}

int32_t ent_degree_chebyshev(double u, double ell, double eps) {
  if (!(ell > 0) || !(ell < 1) || !(u >= ell) || !(eps > 0)) return -1;
  return (int32_t)std::ceil(std::sqrt(u / (2.0 * eps * ell * std::log(1.0 / (1.0 - ell)))));
}

int32_t ent_power_trials_for(double delta) {
  if (!(delta > 0) || !(delta < 1)) return -1;
  return (int32_t)std::ceil(4.82 * std::log(1.0 / delta));
}

int32_t ent_power_iters_for(int64_t n) {
  if (n < 1) return -1;
  return (int32_t)std::ceil(std::log(std::sqrt(4.0 * (double)n)));
}

ent_status ent_graph_create(const ent_matrix *Rs, int32_t count, int32_t method, int32_t degree,
                            int32_t probes, uint64_t seed, const ent_options *opt, ent_graph *graph) {
  g_last_error.clear();
  if (!graph) return fail(ENT_EINVAL, "graph is NULL");
  ent_graph_s *g = nullptr;
  ent_status rc = batch_create(Rs, count, method, degree, probes, seed, opt, true, &g);
  if (rc != ENT_OK) return rc;
  *graph = g;
  return ENT_OK;
}

ent_status ent_graph_launch(ent_graph graph, ent_result *outs) {
  g_last_error.clear();
  if (!graph || !outs) return fail(ENT_EINVAL, "graph or outs is NULL");
  HIP_TRY(hipGraphLaunch(graph->exec, graph->stream));
  return batch_collect(graph, outs);
}

ent_status ent_graph_per_probe(ent_graph graph, double *per_probe) {
  g_last_error.clear();
  if (!graph || !per_probe) return fail(ENT_EINVAL, "graph or per_probe is NULL");
  if (!graph->launched) return fail(ENT_EINVAL, "the graph has not been launched");
  HIP_TRY(hipMemcpyAsync(per_probe, graph->h, sizeof(double) * graph->count * graph->s,
                         hipMemcpyDeviceToHost, graph->stream));
  HIP_TRY(hipStreamSynchronize(graph->stream));
  return ENT_OK;
}

ent_status ent_graph_time_eager(ent_graph graph, ent_result *outs, ent_timing *timing) {
  g_last_error.clear();
  if (!graph || !outs || !timing) return fail(ENT_EINVAL, "NULL argument");
  PhaseEvents pe;
  pe.on = true;
  pe.st = graph->stream;
  pe.mark();
  ent_status rc = batch_enqueue(graph, graph->stream, &pe);
  if (rc != ENT_OK) return rc;
  pe.mark();
  rc = batch_collect(graph, outs);
  if (rc != ENT_OK) return rc;
  pe.finish();
  *timing = g_last_timing;
  return ENT_OK;
}

int32_t ent_graph_tile_rows(ent_graph graph) { return graph ? 64 * graph->wr : -1; }  // BF16x3: 128

size_t ent_graph_window_bytes(ent_graph graph) { return graph ? graph->window : 0; }

size_t ent_graph_workspace_bytes(ent_graph graph) { return graph ? graph->ws_bytes : 0; }

ent_status ent_graph_destroy(ent_graph graph) {
  g_last_error.clear();
  batch_free(graph);
  return ENT_OK;
}

ent_status ent_entropy_estimate_batched(const ent_matrix *Rs, int32_t count, int32_t method,
                                        int32_t degree, int32_t probes, uint64_t seed,
                                        const ent_options *opt, ent_result *outs) {
  g_last_error.clear();
  if (!outs) return fail(ENT_EINVAL, "outs is NULL");
  ent_graph_s *g = nullptr;
  ent_status rc = batch_create(Rs, count, method, degree, probes, seed, opt, false, &g);
  if (rc != ENT_OK) return rc;
  rc = batch_enqueue(g, g->stream, nullptr);
  if (rc == ENT_OK) rc = batch_collect(g, outs);
  batch_free(g);
  return rc;
}

int32_t ent_mlp_nparams(void) { return ent::mlp_nparams(); }

ent_status ent_mlp_forward(const float *params, const float *X, int32_t count, float *Y, void *stream) {
  g_last_error.clear();
  if (!params || !X || !Y) return fail(ENT_EINVAL, "NULL argument");
  if (count < 1) return fail(ENT_EINVAL, "count < 1");
  const size_t np = sizeof(float) * (size_t)ent::mlp_nparams();
  ent_status rc = check_device_range(params, np, "params");
  if (rc == ENT_OK) rc = check_device_range(X, sizeof(float) * 16 * (size_t)count, "X");
  if (rc == ENT_OK) rc = check_device_range(Y, sizeof(float) * 2 * (size_t)count, "Y");
  if (rc != ENT_OK) return rc;
  HIP_TRY(ent::launch_mlp_forward(params, X, count, Y, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return ENT_OK;
}

// Gradient of the mean squared error over count samples (device grad).
ent_status ent_mlp_grad(const float *params, const float *X, const float *T, int32_t count,
                        float *grad, double *loss, void *stream) {
  g_last_error.clear();
  if (!params || !X || !T || !grad || !loss) return fail(ENT_EINVAL, "NULL argument");
  if (count < 1) return fail(ENT_EINVAL, "count < 1");
  {
    const size_t np = sizeof(float) * (size_t)ent::mlp_nparams();
    ent_status rc = check_device_range(params, np, "params");
    if (rc == ENT_OK) rc = check_device_range(grad, np, "grad");
    if (rc == ENT_OK) rc = check_device_range(X, sizeof(float) * 16 * (size_t)count, "X");
    if (rc == ENT_OK) rc = check_device_range(T, sizeof(float) * 2 * (size_t)count, "T");
    if (rc != ENT_OK) return rc;
  }
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceWorkspace *ws = workspace_for(dev);
  std::lock_guard<std::mutex> lk(ws->mu);
  const int32_t nb = ent::mlp_blocks(count);
  float *gpart = nullptr;
  double *lpart = nullptr, *ldev = nullptr;
  Carve cv;
  cv.add(&gpart, (size_t)nb * ent::mlp_nparams());
  cv.add(&lpart, (size_t)nb);
  cv.add(&ldev, 1);
  ent_status rc = ensure_workspace(ws, cv.total());
  if (rc != ENT_OK) return rc;
  cv.assign(ws->ptr);
  HIP_TRY(ent::launch_mlp_grad(params, X, T, count, gpart, lpart, grad, ldev, st));
  HIP_TRY(hipMemcpyAsync(loss, ldev, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return ENT_OK;
}

// One pass of minibatch Adam over the samples in order (the caller shuffles).
ent_status ent_mlp_train_epoch(float *params, float *adam_m, float *adam_v, int32_t *step,
                               const float *X, const float *T, int32_t count, int32_t batch,
                               float lr, void *stream, double *mean_loss) {
  g_last_error.clear();
  if (!params || !adam_m || !adam_v || !step || !X || !T || !mean_loss)
    return fail(ENT_EINVAL, "NULL argument");
  if (count < 1 || batch < 1) return fail(ENT_EINVAL, "count and batch must be >= 1");
  {
    const size_t np = sizeof(float) * (size_t)ent::mlp_nparams();
    ent_status rc = check_device_range(params, np, "params");
    if (rc == ENT_OK) rc = check_device_range(adam_m, np, "adam_m");
    if (rc == ENT_OK) rc = check_device_range(adam_v, np, "adam_v");
    if (rc == ENT_OK) rc = check_device_range(X, sizeof(float) * 16 * (size_t)count, "X");
    if (rc == ENT_OK) rc = check_device_range(T, sizeof(float) * 2 * (size_t)count, "T");
    if (rc != ENT_OK) return rc;
  }
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceWorkspace *ws = workspace_for(dev);
  std::lock_guard<std::mutex> lk(ws->mu);
  const int32_t nb = ent::mlp_blocks(batch);
  const int32_t nsteps = (count + batch - 1) / batch;
  float *gpart = nullptr, *grad = nullptr;
  double *lpart = nullptr, *losses = nullptr;
  Carve cv;
  cv.add(&gpart, (size_t)nb * ent::mlp_nparams());
  cv.add(&lpart, (size_t)nb);
  cv.add(&grad, (size_t)ent::mlp_nparams());
  cv.add(&losses, (size_t)nsteps);
  ent_status rc = ensure_workspace(ws, cv.total());
  if (rc != ENT_OK) return rc;
  cv.assign(ws->ptr);
  const int64_t nin = 16, nout = 2;
  for (int32_t b = 0; b < nsteps; ++b) {
    const int32_t off = b * batch;
    const int32_t cnt = std::min(batch, count - off);
    HIP_TRY(ent::launch_mlp_grad(params, X + (int64_t)off * nin, T + (int64_t)off * nout, cnt, gpart,
                                 lpart, grad, losses + b, st));
    ++*step;
    HIP_TRY(ent::launch_adam(params, grad, adam_m, adam_v, *step, lr, st));
  }
  std::vector<double> lh(nsteps);
  HIP_TRY(hipMemcpyAsync(lh.data(), losses, sizeof(double) * nsteps, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double acc = 0.0;
  for (double v : lh) acc += v;
  *mean_loss = acc / nsteps;
  return ENT_OK;
}

ent_status ent_selector_load(const float *params, int32_t nparams) {
  g_last_error.clear();
  if (!params) return fail(ENT_EINVAL, "params is NULL");
  if (nparams != ent::mlp_nparams())
    return fail(ENT_EINVAL, "expected %d parameters, got %d", ent::mlp_nparams(), nparams);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_sel_mu);
  SelectorState &st = g_sel[dev];
  if (!st.params) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(float) * (nparams + 16 + 2 + 14)) != hipSuccess)
      return fail(ENT_ENOMEM, "selector allocation failed");
    st.params = (float *)p;
    st.feat = st.params + nparams;
    st.y = st.feat + 16;
  }
  HIP_TRY(hipMemcpy(st.params, params, sizeof(float) * nparams, hipMemcpyHostToDevice));
  return ENT_OK;
}

ent_status ent_selector_features(const ent_matrix *R, uint64_t seed, const ent_options *opt,
                                 float *features, float *outputs) {
  g_last_error.clear();
  ent_status rc = validate_matrix(R);
  if (rc != ENT_OK) return rc;
  if (!features) return fail(ENT_EINVAL, "features is NULL");
  Opts op = resolve_options(opt);
  rc = validate_options(op.o);
  if (rc != ENT_OK) return rc;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  SelectorState st;
  {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    auto it = g_sel.find(dev);
    if (it == g_sel.end() || !it->second.params)
      return fail(ENT_EINVAL, "call ent_selector_load first (the features pass also runs the network)");
    st = it->second;
  }
  float y[2];
  ent_result fr{};
  rc = with_device_copy(R, op.st, [&](const ent_matrix *D) {
    ent_status r2 = check_matrix_memory(D);
    if (r2 != ENT_OK) return r2;
    return feature_pass(D, seed, op, st, y, &fr);
  });
  if (rc != ENT_OK) return rc;
  HIP_TRY(hipMemcpy(features, st.feat, sizeof(float) * 16, hipMemcpyDeviceToHost));
  if (outputs) {
    outputs[0] = y[0];
    outputs[1] = y[1];
  }
  return ENT_OK;
}

ent_status ent_timing_enable(int32_t on) {
  g_last_error.clear();
  g_timing_on = on != 0;
  return ENT_OK;
}

ent_status ent_last_timing(ent_timing *out) {
  g_last_error.clear();
  if (!out) return fail(ENT_EINVAL, "out is NULL");
  *out = g_last_timing;
  return ENT_OK;
}

ent_status ent_set_workspace_limit(size_t bytes) {
  g_last_error.clear();
  g_ws_limit = bytes;
  return ENT_OK;
}

// The two maps are released one after the other, never with both map locks
// held: a Hermitian estimate holds its real-form buffer while it takes the
// workspace map lock.
ent_status ent_release_workspace(void) {
  g_last_error.clear();
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  const ent_status r1 = free_buffers(g_ws_mu, g_ws);
  const ent_status r2 = free_buffers(g_rf_mu, g_rf);
  const ent_status r3 = free_buffers(g_stage_mu, g_stage);
  const hipError_t e = hipSetDevice(cur);
  if (r1 != ENT_OK) return r1;
  if (r2 != ENT_OK) return r2;
  if (r3 != ENT_OK) return r3;
  if (e != hipSuccess) return fail(ENT_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  return ENT_OK;
}

size_t ent_workspace_bytes(void) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  size_t t = 0;
  for (auto &kv : g_ws) t += kv.second->bytes;
  return t;
}

const char *ent_last_error(void) { return g_last_error.c_str(); }

int32_t ent_version(void) { return 100; }

}  // extern "C"
