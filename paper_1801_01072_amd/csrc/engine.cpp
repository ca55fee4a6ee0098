// engine.cpp -- C ABI of libentropy: argument validation, workspace, and the
// launch sequence of one estimate (power method -> interval and coefficients
// -> m recurrence steps -> reductions), all enqueued on the caller's stream
// with a single synchronisation at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
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
    t.step_launches = steps_end - steps_begin;
    for (int i = steps_begin; i >= 0 && i < steps_end; ++i) {
      const double d = between(i, i + 1);
      t.steps_ms += d;
      if (d > t.step_max_ms) t.step_max_ms = d;
    }
    t.other_ms = t.total_ms - t.power_ms - t.steps_ms;
    t.power_launches = power_launches;
    g_last_timing = t;
  }
};

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
size_t g_ws_limit = 0;

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
                g_ws_limit);
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

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

constexpr int kScalarDoubles = 8192;

ent_status validate_matrix(const ent_matrix *R) {
  if (!R) return fail(ENT_EINVAL, "R is NULL");
  if (R->n < 1) return fail(ENT_EINVAL, "n = %lld < 1", (long long)R->n);
  if (R->n > (int64_t)INT32_MAX - 64)
    return fail(ENT_EINVAL, "n = %lld exceeds the 32-bit column index range", (long long)R->n);
  if (R->dtype != ENT_STORE_F64 && R->dtype != ENT_STORE_F32)
    return fail(ENT_EINVAL, "unknown storage dtype %d", R->dtype);
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

struct Opts {
  ent_options o;
  hipStream_t st;
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
                         uint64_t seed, double *x0, double *x1, double *p0, double *p1,
                         double *scal, hipStream_t st) {
  const int64_t n = R->n;
  for (int32_t trial = 0; trial < q; ++trial) {
    HIP_TRY(ent::launch_power_start(x0, n, seed, trial, st));
    double *xin = x0, *xout = x1, *pin = nullptr, *pout = p1;
    int32_t in_cnt = 0, nblk = 0;
    for (int32_t it = 0; it <= t; ++it) {  // t iterations + the Rayleigh product
      if (R->layout == ENT_DENSE)
        HIP_TRY(ent::launch_power_gemv<T>(Rc, ldr, n, xin, pin, in_cnt, xout, pout, &nblk, st));
      else
        HIP_TRY(ent::launch_power_spmv<T>(R->row_ptr, R->col_idx, (const T *)R->values, n, xin,
                                          pin, in_cnt, xout, pout, &nblk, st));
      std::swap(xin, xout);
      pin = pout;
      pout = (pout == p1) ? p0 : p1;
      in_cnt = nblk;
    }
    HIP_TRY(ent::launch_power_rq(scal, pin, nblk, trial, st));
  }
  return ENT_OK;
}

// Validate a CSR structure on the device before any kernel dereferences its
// indices (one synchronisation).  Uses the first 256 bytes of the workspace.
ent_status check_csr(const ent_matrix *R, void *scratch, hipStream_t st) {
  if (R->layout != ENT_CSR) return ENT_OK;
  int32_t *flag = (int32_t *)scratch;
  int32_t h = 0;
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  HIP_TRY(ent::launch_validate_csr(R->row_ptr, R->col_idx, R->n, R->nnz, flag, st));
  HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h) return fail(ENT_EINVAL, "invalid CSR structure (row_ptr must start at 0, be non-decreasing "
                                 "and end at nnz; column indices must lie in [0, n))");
  return ENT_OK;
}

int64_t power_blocks(const ent_matrix *R) {
  return R->layout == ENT_DENSE ? (R->n + 15) / 16 : (R->n + 31) / 32;
}

// ---------------------------------------------------------------------------
// One polynomial estimate (Algorithms 1-2) in compute type T.
// ---------------------------------------------------------------------------
template <typename T>
ent_status run_poly(const ent_matrix *R, int32_t method, int32_t m, int32_t s, uint64_t seed,
                    const Opts &op, ent_result *out, double *per_probe, double *moments) {
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
  const int bn = dense ? (s <= 64 ? 64 : (s <= 128 ? 128 : 64)) : 64;
  const int64_t ldv = round_up(s, dense ? bn : 64);
  const int64_t n_pad = round_up(n, 64);
  const int32_t ntile = dense ? (int32_t)(n_pad / 64) : ent::csr_step_blocks(n);
  const int32_t nslot = m + 1;
  const bool rad = o.probe_dist == ENT_RADEMACHER;
  const bool use_power = !(o.u_fixed > 0);
  const int32_t pblk = (int32_t)power_blocks(R);

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceWorkspace *ws = workspace_for(dev);
  std::lock_guard<std::mutex> lk(ws->mu);

  double *scal = nullptr, *x0 = nullptr, *x1 = nullptr, *p0 = nullptr, *p1 = nullptr;
  double *part = nullptr, *d = nullptr, *h = nullptr;
  T *Rc = nullptr, *G = nullptr, *VA = nullptr, *VB = nullptr;
  uint32_t *signs = nullptr;
  Carve cv;
  cv.add(&scal, kScalarDoubles);
  if (use_power) {
    cv.add(&x0, n_pad);
    cv.add(&x1, n_pad);
    cv.add(&p0, 3 * (size_t)pblk);
    cv.add(&p1, 3 * (size_t)pblk);
  }
  const int64_t ldc = round_up(n, vec_elems);
  if (need_copy) cv.add(&Rc, (size_t)n * ldc);
  if (dense || !rad) cv.add(&G, (size_t)n_pad * ldv);
  if (!dense && rad) cv.add(&signs, (size_t)n_pad * (ldv / 32));
  cv.add(&VA, (size_t)n_pad * ldv);
  cv.add(&VB, (size_t)n_pad * ldv);
  cv.add(&part, (size_t)nslot * ntile * ldv);
  cv.add(&d, (size_t)nslot * s);
  cv.add(&h, (size_t)s);
  ent_status rc = ensure_workspace(ws, cv.total());
  if (rc != ENT_OK) return rc;
  cv.assign(ws->ptr);
  rc = check_csr(R, scal, st);
  if (rc != ENT_OK) return rc;

  PhaseEvents pe;
  pe.on = g_timing_on;
  pe.st = st;
  pe.mark();
  HIP_TRY(hipMemsetAsync(scal, 0, sizeof(double) * 64, st));
  // trace check
  const bool check_trace = !(o.flags & ENT_FLAG_SKIP_TRACE_CHECK);
  if (check_trace) {
    if (dense) {
      if (R->dtype == ENT_STORE_F64)
        HIP_TRY(ent::launch_trace_dense<double>((const double *)R->values, R->ld, n, scal, st));
      else
        HIP_TRY(ent::launch_trace_dense<float>((const float *)R->values, R->ld, n, scal, st));
    } else {
      if (R->dtype == ENT_STORE_F64)
        HIP_TRY(ent::launch_trace_csr<double>(R->row_ptr, R->col_idx, (const double *)R->values, n,
                                              scal, st));
      else
        HIP_TRY(ent::launch_trace_csr<float>(R->row_ptr, R->col_idx, (const float *)R->values, n,
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
  // probes
  if (dense || !rad)
    HIP_TRY(ent::launch_probe_gen<T>(G, nullptr, n, n_pad, s, ldv, seed, o.probe_dist, st));
  else
    HIP_TRY(ent::launch_sign_gen(signs, n, s, ldv, seed, st));
  // power method and interval
  if (use_power) {
    pe.power_begin = pe.mark();
    rc = enqueue_power<T>(R, Rt, ldr, o.power_iters, o.power_trials, seed, x0, x1, p0, p1, scal, st);
    if (rc != ENT_OK) return rc;
    pe.power_end = pe.mark();
    pe.power_launches = o.power_trials * (o.power_iters + 1);
  }
  HIP_TRY(ent::launch_setup_interval(scal, method, m, o.u_factor, o.u_fixed, o.cutoff, st));

  // recurrence
  const int32_t nsteps = (method == ENT_CHEBYSHEV) ? m : m + 1;
  const T *Vk = dense || !rad ? G : nullptr;  // null: expand the sign block
  const T *Vkm1 = nullptr;
  T *bufs[2] = {VA, VB};
  pe.steps_begin = pe.mark();
  for (int32_t k = 0; k < nsteps; ++k) {
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
      HIP_TRY(ent::launch_dense_step<T>(a, st));
    } else {
      ent::CsrStepArgs a{};
      a.row_ptr = R->row_ptr; a.col_idx = R->col_idx; a.values = R->values; a.n = n; a.ldv = ldv;
      a.Vk = Vk; a.Vkm1 = Vkm1; a.Vkp1 = write ? Vout : nullptr;
      a.signs = rad ? signs : nullptr; a.G = rad ? nullptr : G;
      a.scal = scal; a.c1 = c1; a.c2 = c2; a.cw = cw; a.dot_y = dot_y;
      a.slot = slot; a.slot_gg = slot_gg; a.part = part; a.nblk = ntile;
      HIP_TRY(ent::launch_csr_step<T>(a, st));
    }
    // Chebyshev: V_{k+1} is written over V_{k-1} (same element, same thread),
    // so two buffers plus the probe block suffice.  Taylor: W_{k+1} may not
    // overwrite W_k (read by every tile), so outputs alternate.
    if (method == ENT_CHEBYSHEV) Vkm1 = Vk;
    Vk = Vout;
    const int e = pe.mark();
    if (k == nsteps - 1) pe.steps_end = e;
  }
  HIP_TRY(ent::launch_reduce_moments(part, nslot, ntile, ldv, s, d, st));
  HIP_TRY(ent::launch_final(d, scal, method, m, s, h, st));

  double hs[16];
  HIP_TRY(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, st));
  if (per_probe) HIP_TRY(hipMemcpyAsync(per_probe, h, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  if (moments)
    HIP_TRY(hipMemcpyAsync(moments, d, sizeof(double) * nslot * s, hipMemcpyDeviceToHost, st));
  pe.mark();
  HIP_TRY(hipStreamSynchronize(st));
  pe.finish();

  if (check_trace) {
    double tol = o.trace_tol > 0 ? o.trace_tol : (R->dtype == ENT_STORE_F64 ? 1e-10 : 1e-4);
    if (!(std::fabs(hs[ent::S_TRACE] - 1.0) <= tol))
      return fail(ENT_ENOTDENSITY, "trace of R is %.17g, not 1 within %.3g", hs[ent::S_TRACE], tol);
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
  out->precision = o.precision;
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
  ent_status rc = validate_matrix(R);
  if (rc != ENT_OK) return rc;
  if (!out) return fail(ENT_EINVAL, "out is NULL");
  Opts op = resolve_options(opt);
  rc = validate_options(op.o);
  if (rc != ENT_OK) return rc;
  if (method == ENT_RANDPROJ) return fail(ENT_EUNSUPPORTED, "random projection is not built yet");
  if (method != ENT_TAYLOR && method != ENT_CHEBYSHEV)
    return fail(ENT_EINVAL, "unknown method %d", method);
  if (degree < 1) return fail(ENT_EINVAL, "degree = %d < 1", degree);
  if (degree > 4000) return fail(ENT_EINVAL, "degree = %d > 4000", degree);
  if (probes < 1) return fail(ENT_EINVAL, "probes = %d < 1", probes);
  if (method == ENT_TAYLOR && op.o.cutoff > 0)
    return fail(ENT_EINVAL, "cutoff applies to the Chebyshev method only");
  ent_result tmp{};
  switch (op.o.precision) {
    case ENT_F64: rc = run_poly<double>(R, method, degree, probes, seed, op, &tmp, per_probe, moments); break;
    case ENT_F32: rc = run_poly<float>(R, method, degree, probes, seed, op, &tmp, per_probe, moments); break;
    default: return fail(ENT_EUNSUPPORTED, "precision %d is not built yet", op.o.precision);
  }
  if (rc == ENT_OK) *out = tmp;
  return rc;
}

ent_status ent_entropy_estimate(const ent_matrix *R, int32_t method, int32_t degree, int32_t probes,
                                uint64_t seed, const ent_options *opt, ent_result *out) {
  return ent_entropy_estimate_detail(R, method, degree, probes, seed, opt, out, nullptr, nullptr);
}

ent_status ent_power_method(const ent_matrix *R, int32_t t, int32_t q, uint64_t seed, void *stream,
                            double *p1) {
  g_last_error.clear();
  ent_status rc = validate_matrix(R);
  if (rc != ENT_OK) return rc;
  if (!p1) return fail(ENT_EINVAL, "p1 is NULL");
  if (t < 0 || q < 1) return fail(ENT_EINVAL, "need t >= 0 and q >= 1");
  hipStream_t st = (hipStream_t)stream;
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
  cv.add(&pp1, 3 * (size_t)pblk);
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

ent_status ent_release_workspace(void) {
  g_last_error.clear();
  std::lock_guard<std::mutex> lk(g_ws_mu);
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  for (auto &kv : g_ws) {
    std::lock_guard<std::mutex> l2(kv.second->mu);
    if (kv.second->ptr) {
      HIP_TRY(hipSetDevice(kv.first));
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(kv.second->ptr));
      kv.second->ptr = nullptr;
      kv.second->bytes = 0;
    }
  }
  HIP_TRY(hipSetDevice(cur));
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
