// C ABI of libcsp: contexts, lattices, states, coefficients and the
// propagation driver (planner + launch sequence).  See include/csp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "csp_internal.h"

using namespace csp;

int csp::ring_parts(int S) {
  for (int g : {3, 4, 2})
    if (S >= g && S % g == 0) return g;
  return 1;
}

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;

csp_status fail(csp_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCALL(x)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      return fail(CSP_EHIP, "%s failed: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                            \
  } while (0)

#define CHECK(x)                          \
  do {                                    \
    csp_status s_ = (x);                  \
    if (s_ != CSP_OK) return s_;          \
  } while (0)

// Makes `dev` current for the scope and restores the previous device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

// ------------------------------------------------------------------ objects
struct csp_context {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  void* ws = nullptr;
  size_t ws_size = 0;
  void* ell_sh = nullptr;           // shadows of explicit-matrix instances (grow-only)
  size_t ell_sh_size = 0;
  std::vector<hipEvent_t> events;   // pool for profiling
  std::map<std::string, csp_tuning> tuned;  // autotuner results per shape
  hipStream_t cap = nullptr;                 // library stream for HIP graph capture
  double* dos_scratch = nullptr;             // this device's csp_dos_noalloc twiddles
};

struct csp_lattice {
  csp_context* ctx = nullptr;
  csp_lattice_desc desc{};
  Geom g{};
  double H0 = 0.0, halfwidth = 0.0, gersh = 0.0;
  double* eps64 = nullptr;
  float* eps32 = nullptr;
  bool has_onsite = false;
  // explicit matrix (kind CSP_SPARSE), [D][N]
  int32_t* ell_col = nullptr;
  double* ell_v64 = nullptr;
  float* ell_v32 = nullptr;
  int ell_D = 0;
  // orbital coordinates of an explicit matrix ([N][2]) and periodic box
  double* pos = nullptr;
  double box[2] = {0.0, 0.0};
  // windowed layout of an explicit matrix (see ell_windows.cpp); null when
  // the matrix's slices are not compact enough for it to pay
  int32_t* ellw_rows = nullptr;
  uint16_t* ellw_loc = nullptr;
  int32_t* ellw_col = nullptr;
  double* ellw_v64 = nullptr;
  float* ellw_v32 = nullptr;
  int64_t* ellw_off = nullptr;
  int32_t* ellw_idx = nullptr;
  std::vector<int32_t> ellw_sizes;   // window size of every slice (host)
  std::vector<int32_t> ellw_sorted;  // the same, ascending
};

namespace {

// Grow-only workspace of the context; contents are not preserved.
csp_status ws_reserve(csp_context* c, size_t bytes) {
  if (bytes <= c->ws_size) return CSP_OK;
  if (c->ws) {
    HIPCALL(hipStreamSynchronize(c->stream));
    HIPCALL(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_size = 0;
  }
  hipError_t e = hipMalloc(&c->ws, bytes);
  if (e != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return fail(CSP_ENOMEM, "workspace of %.3f GB could not be allocated (%s)", bytes / 1e9,
                hipGetErrorString(e));
  }
  c->ws_size = bytes;
  return CSP_OK;
}

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t n) {
    void* p = base + off;
    off += align256(n);
    return p;
  }
};

csp_status hip_event(csp_context* c, size_t i, hipEvent_t* out) {
  while (c->events.size() <= i) {
    hipEvent_t e;
    HIPCALL(hipEventCreate(&e));
    c->events.push_back(e);
  }
  *out = c->events[i];
  return CSP_OK;
}

// The library's own stream, used only to capture HIP graphs (capture is not
// allowed on the legacy null stream a caller may have given).  Default
// priority, non-blocking.
csp_status capture_stream(csp_context* c) {
  if (!c->cap) HIPCALL(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  return CSP_OK;
}

// Device memory the planner may use for the workspace: the cap of the
// parameters, else what is free (plus the workspace already held) less a
// small reserve for the caller's own allocations.
csp_status memory_cap(csp_context* c, uint64_t mem_cap_bytes, size_t* cap) {
  size_t freeb = 0, totalb = 0;
  HIPCALL(hipMemGetInfo(&freeb, &totalb));
  const size_t avail = freeb + c->ws_size;
  const size_t reserve = std::min<size_t>(avail / 32, size_t(4) << 30);
  *cap = mem_cap_bytes ? std::min<size_t>(mem_cap_bytes, avail) : avail - reserve;
  return CSP_OK;
}

int64_t trunc_nmax(double x) { return (int64_t)std::ceil(x + 40.0 + 25.0 * std::cbrt(x + 1.0)); }

// Norm-guard flag: [0] first failing block (INT32_MAX = none), [1] column.
csp_status guard_reset(int* d_flag, hipStream_t s) {
  static const int init[2] = {INT32_MAX, -1};
  HIPCALL(hipMemcpyAsync(d_flag, init, sizeof(init), hipMemcpyHostToDevice, s));
  return CSP_OK;
}

csp_status guard_check(const int* d_flag, hipStream_t s) {
  int h[2] = {0, 0};
  HIPCALL(hipMemcpyAsync(h, d_flag, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCALL(hipStreamSynchronize(s));
  if (h[0] != INT32_MAX)
    return fail(CSP_ENUMERIC,
                "norm guard tripped after time block %d (column %d): the carried state lost "
                "its norm or a correlation is not finite or exceeds <psi0|psi0>",
                h[0], h[1]);
  return CSP_OK;
}

}  // namespace

// ------------------------------------------------------------------ basics
extern "C" int csp_abi_version(void) { return CSP_ABI_VERSION; }
extern "C" const char* csp_last_error(void) { return g_err.c_str(); }

extern "C" csp_status csp_context_create(int device, void* hip_stream, csp_context** out) {
  if (!out) return fail(CSP_EINVAL, "out is NULL");
  int n = 0;
  HIPCALL(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(CSP_EINVAL, "device %d out of range (%d)", device, n);
  DeviceGuard dg(device);
  if (!dg.ok) return fail(CSP_EHIP, "hipSetDevice(%d) failed", device);
  hipDeviceProp_t prop;
  HIPCALL(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(CSP_EUNSUPPORTED, "libcsp is built for gfx950, device is %s", prop.gcnArchName);
  double* scratch = nullptr;
  HIPCALL(dos_noalloc_scratch(device, &scratch));   // once per device, device current
  csp_context* c = new csp_context();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->dos_scratch = scratch;
  *out = c;
  return CSP_OK;
}

extern "C" csp_status csp_context_trim(csp_context* c) {
  if (!c) return fail(CSP_EINVAL, "context is NULL");
  DeviceGuard dg(c->device);
  if (c->ws || c->ell_sh) HIPCALL(hipStreamSynchronize(c->stream));
  if (c->ws) HIPCALL(hipFree(c->ws));
  c->ws = nullptr;
  c->ws_size = 0;
  if (c->ell_sh) HIPCALL(hipFree(c->ell_sh));
  c->ell_sh = nullptr;
  c->ell_sh_size = 0;
  return CSP_OK;
}

extern "C" csp_status csp_context_destroy(csp_context* c) {
  if (!c) return CSP_OK;
  DeviceGuard dg(c->device);
  csp_status st = csp_context_trim(c);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  delete c;
  return st;
}

// ------------------------------------------------------------------ lattices
extern "C" csp_status csp_lattice_create(csp_context* c, const csp_lattice_desc* d,
                                         csp_lattice** out) {
  if (!c || !d || !out) return fail(CSP_EINVAL, "NULL argument");
  if (d->kind < CSP_CHAIN || d->kind > CSP_HONEYCOMB)
    return fail(CSP_EINVAL, "unknown lattice kind %d", d->kind);
  const int64_t Ly = d->kind == CSP_CHAIN ? 1 : d->Ly;
  if (d->Lx < 1 || Ly < 1) return fail(CSP_EINVAL, "lattice sizes must be >= 1");
  {
    const int64_t opr = d->kind == CSP_HONEYCOMB ? 2 * d->Lx : d->Lx;
    if (opr > INT32_MAX || Ly > INT32_MAX || opr * Ly >= ((int64_t)1 << 31))
      return fail(CSP_EUNSUPPORTED, "at most 2^31 - 1 orbitals per lattice");
  }
  if (!std::isfinite(d->t) || !std::isfinite(d->W) || d->W < 0)
    return fail(CSP_EINVAL, "hopping and disorder must be finite, W >= 0");
  DeviceGuard dg(c->device);
  csp_lattice* L = new csp_lattice();
  L->ctx = c;
  L->desc = *d;
  L->g.kind = d->kind;
  L->g.px = d->periodic_x ? 1 : 0;
  L->g.py = (d->kind != CSP_CHAIN && d->periodic_y) ? 1 : 0;
  L->g.Lx = d->Lx;
  L->g.Ly = Ly;
  L->g.opr = d->kind == CSP_HONEYCOMB ? 2 * d->Lx : d->Lx;
  L->g.N = L->g.opr * Ly;
  L->has_onsite = d->W != 0.0;
  L->H0 = d->center;
  auto cleanup = [&](csp_status st) {
    if (L->eps64) (void)hipFree(L->eps64);
    if (L->eps32) (void)hipFree(L->eps32);
    delete L;
    return st;
  };
  if (hipMalloc(&L->eps64, sizeof(double) * L->g.N) != hipSuccess ||
      hipMalloc(&L->eps32, sizeof(float) * L->g.N) != hipSuccess) {
    (void)hipGetLastError();
    return cleanup(fail(CSP_ENOMEM, "on-site arrays of %lld orbitals", (long long)L->g.N));
  }
  hipError_t e = launch_onsite(L->g, d->W, d->disorder_seed, L->eps64, L->eps32, c->stream);
  const int np = 1024;
  double* d_part = nullptr;
  if (e == hipSuccess) e = hipMalloc(&d_part, sizeof(double) * np);
  if (e == hipSuccess) e = launch_gershgorin(L->g, L->eps64, d->t, L->H0, d_part, np, c->stream);
  std::vector<double> part(np);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), d_part, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (d_part) (void)hipFree(d_part);
  if (e != hipSuccess) return cleanup(fail(CSP_EHIP, "lattice set-up: %s", hipGetErrorString(e)));
  double m = 0.0;
  for (double v : part) m = std::max(m, v);
  L->gersh = m;
  const double margin = d->bound_margin > 0 ? d->bound_margin : 1.025;
  L->halfwidth = d->halfwidth_override > 0 ? d->halfwidth_override : margin * m;
  if (!(L->halfwidth > 0)) return cleanup(fail(CSP_EINVAL, "zero spectral half-width (t = W = 0)"));
  *out = L;
  return CSP_OK;
}

extern "C" csp_status csp_lattice_create_sparse(csp_context* c, int64_t N, int32_t D,
                                                const int32_t* col, const double* val,
                                                double margin, csp_lattice** out) {
  if (!c || !col || !val || !out) return fail(CSP_EINVAL, "NULL argument");
  if (N < 1 || N >= ((int64_t)1 << 31)) return fail(CSP_EINVAL, "need 1 <= N < 2^31");
  if (D < 1 || D > 4096) return fail(CSP_EINVAL, "need 1 <= D <= 4096");
  // reorder into slices of 128 rows, [N/128][D][128], on the host, checking
  // the indices; padding entries (and the rows past N of the last slice)
  // hold a valid index and the value 0
  const int64_t n_slices = (N + 127) / 128;
  const size_t n = (size_t)n_slices * D * 128;
  std::vector<int32_t> ct(n, 0);
  std::vector<double> vt(n, 0.0);
  std::vector<float> vf(n, 0.0f);
  for (int64_t sl = 0; sl < n_slices; ++sl) {
    const int64_t s0 = sl * 128, s1 = std::min<int64_t>(N, s0 + 128);
    const size_t o = (size_t)sl * D * 128;
    for (int k = 0; k < D; ++k)
      for (int64_t s = s0; s < s1; ++s) {
        const int32_t j = col[s * D + k];
        if (j >= N) return fail(CSP_EINVAL, "row %lld: column %d out of range", (long long)s, j);
        const double v = j >= 0 ? val[s * D + k] : 0.0;
        if (!std::isfinite(v)) return fail(CSP_EINVAL, "row %lld: non-finite value", (long long)s);
        const size_t e = o + (size_t)k * 128 + (s - s0);
        ct[e] = j < 0 ? static_cast<int32_t>(s) : j;   // padding: 0 x own value
        vt[e] = v;
        vf[e] = static_cast<float>(v);
      }
  }
  DeviceGuard dg(c->device);
  csp_lattice* L = new csp_lattice();
  L->ctx = c;
  L->g.kind = CSP_SPARSE;
  L->g.Lx = N;
  L->g.Ly = 1;
  L->g.opr = N;
  L->g.N = N;
  L->desc.kind = CSP_SPARSE;
  L->desc.Lx = N;
  L->desc.Ly = 1;
  L->ell_D = D;
  auto cleanup = [&](csp_status st) {
    if (L->ell_col) (void)hipFree(L->ell_col);
    if (L->ell_v64) (void)hipFree(L->ell_v64);
    if (L->ell_v32) (void)hipFree(L->ell_v32);
    for (void* q : {(void*)L->ellw_rows, (void*)L->ellw_loc, (void*)L->ellw_col,
                    (void*)L->ellw_v64, (void*)L->ellw_v32, (void*)L->ellw_off,
                    (void*)L->ellw_idx})
      if (q) (void)hipFree(q);
    delete L;
    return st;
  };
  if (hipMalloc(&L->ell_col, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&L->ell_v64, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&L->ell_v32, sizeof(float) * n) != hipSuccess) {
    (void)hipGetLastError();
    return cleanup(fail(CSP_ENOMEM, "explicit matrix of %lld entries", (long long)n));
  }
  hipError_t e = hipMemcpy(L->ell_col, ct.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(L->ell_v64, vt.data(), sizeof(double) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(L->ell_v32, vf.data(), sizeof(float) * n, hipMemcpyHostToDevice);
  const int np = 1024;
  double* d_part = nullptr;
  if (e == hipSuccess) e = hipMalloc(&d_part, sizeof(double) * np);
  if (e == hipSuccess) e = launch_ell_gershgorin(N, D, L->ell_v64, d_part, np, c->stream);
  std::vector<double> part(np);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), d_part, sizeof(double) * np, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (d_part) (void)hipFree(d_part);
  if (e != hipSuccess) return cleanup(fail(CSP_EHIP, "matrix set-up: %s", hipGetErrorString(e)));
  {
    // The windowed layout pays when most slices name few distinct columns:
    // at least half of them with a window that fits a 4-column complex64
    // workgroup's LDS and is read four or more times per step.
    EllWindows w;
    build_ell_windows(N, D, col, val, &w);
    const int64_t cap4 = kEllwLdsBytes / (4 * (int64_t)sizeof(float2));
    int64_t good = 0;
    for (int64_t k = 0; k < w.n_slices; ++k) {
      const int64_t W = w.off[k + 1] - w.off[k];
      if (W > 0 && W <= cap4 && 128 * (int64_t)D >= 4 * W) ++good;
    }
    if (2 * good >= w.n_slices) {
      const size_t ne = w.loc.size();
      auto up = [&](void** dst, const void* src, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(dst, bytes ? bytes : 1);
        if (e == hipSuccess && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
      };
      up((void**)&L->ellw_rows, w.rows.data(), sizeof(int32_t) * w.rows.size());
      up((void**)&L->ellw_loc, w.loc.data(), sizeof(uint16_t) * ne);
      up((void**)&L->ellw_col, w.col.data(), sizeof(int32_t) * ne);
      up((void**)&L->ellw_v64, w.v64.data(), sizeof(double) * ne);
      up((void**)&L->ellw_v32, w.v32.data(), sizeof(float) * ne);
      up((void**)&L->ellw_off, w.off.data(), sizeof(int64_t) * w.off.size());
      up((void**)&L->ellw_idx, w.idx.data(), sizeof(int32_t) * w.idx.size());
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(CSP_ENOMEM, "windowed explicit matrix of %lld entries: %s",
                            (long long)ne, hipGetErrorString(e)));
      }
      L->ellw_sizes.resize(w.n_slices);
      for (int64_t k = 0; k < w.n_slices; ++k)
        L->ellw_sizes[k] = static_cast<int32_t>(w.off[k + 1] - w.off[k]);
      L->ellw_sorted = L->ellw_sizes;
      std::sort(L->ellw_sorted.begin(), L->ellw_sorted.end());
    }
  }
  double m = 0.0;
  for (double v : part) m = std::max(m, v);
  L->gersh = m;
  L->H0 = 0.0;
  L->halfwidth = (margin > 0 ? margin : 1.025) * m;
  if (!(L->halfwidth > 0)) return cleanup(fail(CSP_EINVAL, "zero matrix"));
  *out = L;
  return CSP_OK;
}

extern "C" csp_status csp_lattice_destroy(csp_lattice* L) {
  if (!L) return CSP_OK;
  DeviceGuard dg(L->ctx->device);
  (void)hipStreamSynchronize(L->ctx->stream);
  if (L->eps64) (void)hipFree(L->eps64);
  if (L->eps32) (void)hipFree(L->eps32);
  if (L->ell_col) (void)hipFree(L->ell_col);
  if (L->ell_v64) (void)hipFree(L->ell_v64);
  if (L->ell_v32) (void)hipFree(L->ell_v32);
  if (L->pos) (void)hipFree(L->pos);
  for (void* q : {(void*)L->ellw_rows, (void*)L->ellw_loc, (void*)L->ellw_col,
                  (void*)L->ellw_v64, (void*)L->ellw_v32, (void*)L->ellw_off,
                  (void*)L->ellw_idx})
    if (q) (void)hipFree(q);
  delete L;
  return CSP_OK;
}

extern "C" csp_status csp_lattice_set_positions(csp_lattice* L, const double* pos, double box_x,
                                                double box_y) {
  if (!L || !pos) return fail(CSP_EINVAL, "NULL argument");
  if (L->g.kind != CSP_SPARSE)
    return fail(CSP_EUNSUPPORTED, "stencil lattices have fixed coordinates");
  if (!(box_x >= 0.0) || !(box_y >= 0.0) || !std::isfinite(box_x) || !std::isfinite(box_y))
    return fail(CSP_EINVAL, "box lengths must be finite and >= 0");
  const int64_t N = L->g.N;
  for (int64_t i = 0; i < 2 * N; ++i)
    if (!std::isfinite(pos[i])) return fail(CSP_EINVAL, "coordinate %lld is not finite", (long long)i);
  DeviceGuard dg(L->ctx->device);
  if (!L->pos) {
    if (hipMalloc(&L->pos, sizeof(double) * 2 * N) != hipSuccess) {
      (void)hipGetLastError();
      L->pos = nullptr;
      return fail(CSP_ENOMEM, "coordinates of %lld orbitals", (long long)N);
    }
  }
  HIPCALL(hipMemcpy(L->pos, pos, sizeof(double) * 2 * N, hipMemcpyHostToDevice));
  L->box[0] = box_x;
  L->box[1] = box_y;
  return CSP_OK;
}

extern "C" csp_status csp_lattice_get_info(const csp_lattice* L, csp_lattice_info* o) {
  if (!L || !o) return fail(CSP_EINVAL, "NULL argument");
  o->n_orb = L->g.N;
  o->rows = L->g.Ly;
  o->orb_per_row = L->g.opr;
  o->H0 = L->H0;
  o->halfwidth = L->halfwidth;
  o->gershgorin = L->gersh;
  o->max_degree = L->g.kind == CSP_SPARSE ? L->ell_D : max_degree(L->g.kind);
  o->has_onsite = L->has_onsite ? 1 : 0;
  o->ell_windowed = L->ellw_rows ? 1 : 0;
  int32_t mw = 0;
  for (int32_t W : L->ellw_sizes) mw = std::max(mw, W);
  o->ell_max_window = mw;
  return CSP_OK;
}

extern "C" csp_status csp_lattice_onsite(const csp_lattice* L, double* dev_eps) {
  if (!L || !dev_eps) return fail(CSP_EINVAL, "NULL argument");
  if (L->g.kind == CSP_SPARSE) return fail(CSP_EUNSUPPORTED, "explicit matrix: no on-site array");
  DeviceGuard dg(L->ctx->device);
  HIPCALL(hipMemcpyAsync(dev_eps, L->eps64, sizeof(double) * L->g.N, hipMemcpyDeviceToDevice,
                         L->ctx->stream));
  return CSP_OK;
}

extern "C" csp_status csp_lattice_neighbors(const csp_lattice* L, int64_t* dev_nbr) {
  if (!L || !dev_nbr) return fail(CSP_EINVAL, "NULL argument");
  if (L->g.kind == CSP_SPARSE) return fail(CSP_EUNSUPPORTED, "explicit matrix: no stencil");
  DeviceGuard dg(L->ctx->device);
  HIPCALL(launch_neighbours(L->g, dev_nbr, L->ctx->stream));
  return CSP_OK;
}

// ------------------------------------------------------------------ states
extern "C" csp_status csp_states_random_phase(csp_context* c, int64_t N, int32_t R, uint64_t seed,
                                              int32_t dtype, void* dev_psi, int32_t ld,
                                              int32_t col0) {
  if (!c || !dev_psi) return fail(CSP_EINVAL, "NULL argument");
  if (N < 1 || R < 0 || col0 < 0 || col0 + R > ld)
    return fail(CSP_EINVAL, "bad block shape N=%lld R=%d ld=%d col0=%d", (long long)N, R, ld, col0);
  if (dtype != CSP_C64 && dtype != CSP_C128) return fail(CSP_EINVAL, "bad dtype %d", dtype);
  if (R == 0) return CSP_OK;
  DeviceGuard dg(c->device);
  HIPCALL(launch_random_phase(N, R, seed, dtype, dev_psi, ld, col0, c->stream));
  return CSP_OK;
}

extern "C" csp_status csp_ldos_sites(csp_context* c, int64_t N, int32_t n, uint64_t seed,
                                     int64_t* dev_sites) {
  if (!c || !dev_sites) return fail(CSP_EINVAL, "NULL argument");
  if (n < 0 || n > N || n > 65536) return fail(CSP_EINVAL, "need 0 <= n <= min(N, 65536)");
  if (n == 0) return CSP_OK;
  DeviceGuard dg(c->device);
  HIPCALL(launch_ldos_sites(N, n, seed, dev_sites, c->stream));
  return CSP_OK;
}

extern "C" csp_status csp_states_sites(csp_context* c, int64_t N, int32_t n,
                                       const int64_t* dev_sites, int32_t dtype, void* dev_psi,
                                       int32_t ld, int32_t col0) {
  if (!c || !dev_psi || (n > 0 && !dev_sites)) return fail(CSP_EINVAL, "NULL argument");
  if (N < 1 || n < 0 || col0 < 0 || col0 + n > ld) return fail(CSP_EINVAL, "bad block shape");
  if (dtype != CSP_C64 && dtype != CSP_C128) return fail(CSP_EINVAL, "bad dtype %d", dtype);
  if (n == 0) return CSP_OK;
  DeviceGuard dg(c->device);
  HIPCALL(launch_site_states(N, n, dev_sites, dtype, dev_psi, ld, col0, c->stream));
  return CSP_OK;
}

// ------------------------------------------------------------------ coefficients
extern "C" csp_status csp_chebyshev_coefficients(csp_context* c, double x, double eta,
                                                 int32_t nmax, double* dev_c, int32_t* n_trunc) {
  if (!c || !dev_c) return fail(CSP_EINVAL, "NULL argument");
  if (!(x >= 0) || !std::isfinite(x) || nmax < 0 || !(eta > 0))
    return fail(CSP_EINVAL, "need x >= 0, nmax >= 0, eta > 0");
  DeviceGuard dg(c->device);
  const int64_t nm = std::max<int64_t>(nmax, trunc_nmax(x));
  double* d_a = nullptr;
  int32_t* d_n = nullptr;
  hipError_t e = hipMalloc(&d_a, sizeof(double) * (nm + 1));
  if (e == hipSuccess) e = hipMalloc(&d_n, sizeof(int32_t));
  if (e == hipSuccess) e = launch_bessel(x, 1, (int)nm, eta, false, d_a, d_n, c->stream);
  if (e == hipSuccess) e = launch_complex_coeffs(d_a, nmax, dev_c, c->stream);
  int32_t nt = -1;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&nt, d_n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (d_a) (void)hipFree(d_a);
  if (d_n) (void)hipFree(d_n);
  if (e != hipSuccess) return fail(CSP_EHIP, "coefficients: %s", hipGetErrorString(e));
  if (n_trunc) *n_trunc = nt;
  return CSP_OK;
}

// ------------------------------------------------------------------ recursion helpers
namespace {

struct ChebPlan {
  int vec = 4;          // values per lane and row (strip = 64 vec)
  int kt = 1;           // steps per launch (temporal blocking)
  int seg_rows = 32;    // rows per work item
  int ow = 0;           // owned values per strip
  int64_t total_items = 0;
  std::vector<ChebRun> runs;   // one launch per run of same-class instances
};

// Work items (waves) of the instances for strips of 64 vec values carrying
// kt levels, and segments of seg_rows rows; 0 arguments choose defaults
// (the autotuner passes what it measured).
ChebPlan plan_cheb(std::vector<ChebInst>& insts, bool fp64, bool mom, int n_cu, int vec = 0,
                   int kt = 0, int seg = 0) {
  ChebPlan p;
  p.vec = vec > 0 ? vec : 2;
  p.kt = kt > 0 ? kt : 1;
  for (auto& I : insts)
    if (I.kind == CSP_SPARSE) p.kt = 1;   // explicit matrices: one step per launch
  if (!cheb_shape_supported(fp64, p.vec, p.kt, mom)) {
    p.vec = 2;
    p.kt = 1;
  }
  p.ow = 64 * p.vec - 2 * cheb_margin(p.vec, p.kt);
  int64_t items_rows1 = 0;   // items with one row per segment
  for (auto& I : insts)
    if (I.kind != CSP_SPARSE) items_rows1 += I.Rg * ceil_div(I.opr, p.ow) * I.Ly;
  if (seg > 0) {
    p.seg_rows = seg;
  } else {
    // long segments amortise the 2 kt margin rows; keep >= 8 waves per CU
    p.seg_rows = 64;
    while (p.seg_rows > 4 && items_rows1 / p.seg_rows < (int64_t)n_cu * 8) p.seg_rows /= 2;
  }
  // explicit matrices: a wave owns 128 rows of ell_ct columns; items are
  // the moment records, one per (column, 128-row chunk)
  int64_t t0 = 0, w0 = 0;
  for (size_t k = 0; k < insts.size(); ++k) {
    ChebInst& I = insts[k];
    const bool sparse = I.kind == CSP_SPARSE;
    I.n_strips = sparse ? 1 : ceil_div(I.opr, p.ow);
    I.n_segs = sparse ? ceil_div(I.N, 128) : ceil_div(I.Ly, p.seg_rows);
    I.item0 = t0;
    I.wave0 = w0;
    const int64_t n = (int64_t)I.Rg * I.n_strips * I.n_segs;
    const int ct = sparse ? I.ell_ct : 0;
    const int64_t nw = sparse ? I.n_segs * ceil_div(I.Rg, ct) : 0;
    const bool honey = I.kind == CSP_HONEYCOMB, eps = I.eps != nullptr;
    const bool win = sparse && I.ellw_rows != nullptr;
    if (p.runs.empty() || p.runs.back().honey != honey || p.runs.back().eps != eps ||
        p.runs.back().sparse != sparse || p.runs.back().ct != ct || p.runs.back().win != win)
      p.runs.push_back({(int)k, 0, t0, 0, honey, eps, sparse, ct, w0, 0, win, 0});
    p.runs.back().n_inst += 1;
    if (win)   // LDS values (window entries x columns) of the run's largest tile
      p.runs.back().win_cap = std::max<int64_t>(p.runs.back().win_cap,
                                                I.ellw_lds_cap * std::min(I.ell_ct, I.Rg));
    p.runs.back().n_items += n;
    p.runs.back().n_waves += nw;
    t0 += n;
    w0 += nw;
  }
  p.total_items = t0;
  return p;
}

// Bytes of the per-orbital operands that every recursion launch reads once
// per column group: on-site energies, or the explicit matrix (indices and
// values).
double static_bytes(const csp_lattice* L, bool fp64) {
  const double w = fp64 ? 8 : 4;
  if (L->g.kind == CSP_SPARSE) return (double)L->g.N * L->ell_D * (4 + w);
  return L->has_onsite ? (double)L->g.N * w : 0.0;
}

ChebInst make_inst(const csp_lattice* L, int Rg, bool fp64) {
  ChebInst I{};
  I.kind = L->g.kind;
  I.px = L->g.px;
  I.py = L->g.py;
  I.Rg = Rg;
  I.Ly = L->g.Ly;
  I.opr = L->g.opr;
  I.N = L->g.N;
  I.pitch = L->g.opr;   // unpadded rows (the propagation forms set their own)
  I.cstride = L->g.N;
  I.alpha = 2.0 * (L->g.kind == CSP_SPARSE ? 1.0 : L->desc.t) / L->halfwidth;
  I.beta0 = -2.0 * L->H0 / L->halfwidth;
  I.onsite_scale = 2.0 / L->halfwidth;
  I.eps = L->has_onsite ? (fp64 ? (const void*)L->eps64 : (const void*)L->eps32) : nullptr;
  if (L->g.kind == CSP_SPARSE) {
    I.ell_col = L->ell_col;
    I.ell_val = fp64 ? (const void*)L->ell_v64 : (const void*)L->ell_v32;
    I.ell_D = L->ell_D;
    I.ell_ct = ell_columns_per_wave(fp64, Rg);
    if (L->ellw_rows) {
      const int64_t p97 = L->ellw_sorted[(L->ellw_sorted.size() * 97) / 100];
      I.ell_ct = ellw_columns_per_group(fp64, Rg, p97);
      I.ellw_rows = L->ellw_rows;
      I.ellw_loc = L->ellw_loc;
      I.ellw_col = L->ellw_col;
      I.ellw_val = fp64 ? (const void*)L->ellw_v64 : (const void*)L->ellw_v32;
      I.ellw_off = L->ellw_off;
      I.ellw_idx = L->ellw_idx;
      // LDS of a workgroup: its tile's columns (at most min(ct, Rg)) of the
      // largest window within the budget and the 97th percentile of the
      // window sizes, so that the few slices with far larger windows (they
      // gather from global memory) do not make every workgroup reserve
      // their LDS
      const int64_t ncs = std::min(I.ell_ct, Rg);
      const int64_t cap = kEllwLdsBytes / (ncs * (int64_t)(fp64 ? 16 : 8));
      int64_t best = 0;
      for (int32_t W : L->ellw_sizes)
        if (W <= cap && W <= p97 && W > best) best = W;
      I.ellw_lds_cap = best;
    }
  }
  return I;
}

ChebStep step_args(const ChebPlan& p) {
  ChebStep st{};
  st.seg_rows = p.seg_rows;
  st.ow = p.ow;
  st.total_items = p.total_items;
  st.copy_slot = -1;
  st.sh_in = -1;
  st.sh_out = -1;
  for (int l = 0; l < 8; ++l) st.slot_out[l] = -1;
  return st;
}

// Orbital-major shadows of phi_n for the complex64 explicit-matrix instances
// of two or more columns: two buffers of Rg/2 column pairs each, in the
// context's own grow-only allocation (outside the workspace).  A step
// gathers phi_n from one buffer and writes phi_{n+1} to the other.
csp_status attach_ell_shadows(csp_context* c, std::vector<ChebInst>& sp, bool fp64) {
  size_t need = 0;
  auto wants = [&](const ChebInst& I) {
    return !fp64 && I.kind == CSP_SPARSE && I.Rg >= 2 && !I.ellw_rows;
  };
  for (const ChebInst& I : sp)
    if (wants(I)) need += align256((size_t)(I.Rg / 2) * I.N * 32);
  if (need > c->ell_sh_size) {
    if (c->ell_sh) {
      HIPCALL(hipStreamSynchronize(c->stream));
      HIPCALL(hipFree(c->ell_sh));
      c->ell_sh = nullptr;
      c->ell_sh_size = 0;
    }
    hipError_t e = hipMalloc(&c->ell_sh, need);
    if (e != hipSuccess) {
      c->ell_sh = nullptr;
      (void)hipGetLastError();
      return fail(CSP_ENOMEM, "explicit-matrix shadows of %.3f GB could not be allocated (%s)",
                  need / 1e9, hipGetErrorString(e));
    }
    c->ell_sh_size = need;
  }
  size_t off = 0;
  for (ChebInst& I : sp) {
    I.ell_shadow = nullptr;
    I.sh_pairs = 0;
    if (wants(I)) {
      I.ell_shadow = static_cast<char*>(c->ell_sh) + off;
      I.sh_pairs = I.Rg / 2;
      off += align256((size_t)(I.Rg / 2) * I.N * 32);
    }
  }
  return CSP_OK;
}

// Shadow buffers of the launch that advances phi_n to phi_{n+1}: phi_n's
// shadow sits in buffer n mod 2, except at a block start (phi_0 is new and
// has none).
void set_shadow(ChebStep& st, int64_t n) {
  st.sh_in = st.first ? -1 : static_cast<int32_t>(n & 1);
  st.sh_out = static_cast<int32_t>((n + 1) & 1);
}

}  // namespace

extern "C" csp_status csp_chebyshev_step(csp_context* c, const csp_lattice* L, int32_t R,
                                         int32_t dtype, const void* dev_x, void* dev_y,
                                         int32_t first) {
  if (!c || !L || !dev_x || !dev_y) return fail(CSP_EINVAL, "NULL argument");
  if (R < 1 || R > kMaxStepCols) return fail(CSP_EINVAL, "need 1 <= R <= %d", kMaxStepCols);
  if (dtype != CSP_C64 && dtype != CSP_C128) return fail(CSP_EINVAL, "bad dtype %d", dtype);
  if (dev_x == dev_y) return fail(CSP_EINVAL, "x and y must be distinct");
  if (L->ctx->device != c->device) return fail(CSP_EINVAL, "lattice is on another device");
  DeviceGuard dg(c->device);
  const bool fp64 = dtype == CSP_C128;
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  const int64_t N = L->g.N;
  // the step runs on column-major copies: slot 0 = x, slot 1 = y in, slot 2 = y out
  const int64_t stride = (N * R + 63) / 64 * 64;
  std::vector<ChebInst> insts(1, make_inst(L, R, fp64));
  ChebPlan p = plan_cheb(insts, fp64, false, c->n_cu);
  CHECK(ws_reserve(c, 3 * align256(stride * csz) + align256(sizeof(ChebInst))));
  Carver cv(c->ws);
  char* slots = static_cast<char*>(cv.take(3 * stride * csz));
  ChebInst* d_inst = (ChebInst*)cv.take(sizeof(ChebInst));
  insts[0].base = slots;
  insts[0].slot_stride = stride;
  hipStream_t s = c->stream;
  HIPCALL(launch_gather_cols(N, R, 0, R, dtype, dev_x, fp64, slots, s));
  if (!first) HIPCALL(launch_gather_cols(N, R, 0, R, dtype, dev_y, fp64, slots + stride * csz, s));
  HIPCALL(hipMemcpyAsync(d_inst, insts.data(), sizeof(ChebInst), hipMemcpyHostToDevice, s));
  ChebStep st = step_args(p);
  st.nlev = 1;
  st.first = first ? 1 : 0;
  st.slot_cur = 0;
  st.slot_prev = 1;
  st.slot_out[0] = 2;
  HIPCALL(launch_cheb(fp64, p.vec, p.kt, false, false, d_inst, p.runs, st, s));
  HIPCALL(launch_scatter_cols(N, R, 0, R, dtype, slots + 2 * stride * csz, fp64, dev_y, s));
  HIPCALL(hipStreamSynchronize(s));
  return CSP_OK;
}

// ------------------------------------------------------------------ propagation
namespace {

// One instance of a propagation: columns col_base .. col_base+R-1 of the
// caller's [N][ld] state block and [(Nt+1)][ld] correlation block.
struct InstIn {
  const csp_lattice* lat;
  const void* psi0;
  int R;
  double* corr;
  void* final_out;
  int ld;
  int col_base;
};

struct Group {
  int inst, col0, Rg;
  int64_t M;             // complex values of one Chebyshev slot of the group (Rg x cstride)
  int64_t pitch = 0;     // values between rows (0: vectors of N values, unpadded)
  int64_t cstride = 0;   // values between the group's columns
  // distance between Chebyshev slots: M rounded up to 64 values, so every
  // slot starts 512-byte aligned (16-byte vector loads in the contraction)
  int64_t stride() const { return (M + 63) / 64 * 64; }
  void* slots = nullptr;
  void* psi0g = nullptr;
  void* carry = nullptr;
  double* partial = nullptr;
  int n_wg = 1;
};

// Layout of the propagation forms' vectors: stencil lattices whose rows are
// not a multiple of 16 values get rows padded to one, so every row starts
// 128-byte aligned (measured on 16383^2 against 16384^2: 11 % longer
// recursion launches unaligned); explicit matrices keep N values.
void set_layout(Group& g, const csp_lattice* L) {
  const int64_t opr = L->g.opr, Ly = L->g.Ly, N = L->g.N;
  g.pitch = 0;
  g.cstride = N;
  if (L->g.kind != CSP_SPARSE && opr % 16 != 0) {
    const int64_t pitch = (opr + 15) / 16 * 16;
    if (Ly * pitch < ((int64_t)1 << 31)) {
      g.pitch = pitch;
      g.cstride = Ly * pitch;
    }
  }
  g.M = g.cstride * g.Rg;
}

// The group's layout in a recursion instance.
void apply_layout(ChebInst& I, const Group& g) {
  if (g.pitch > 0) {
    I.pitch = g.pitch;
    I.cstride = g.cstride;
  }
}

struct ChunkTab {
  int n_lo, n_cnt;
  void* bop = nullptr;     // FP32 path
  float* ccf = nullptr;
  double* coef = nullptr;  // FP64 path
  double* ccd = nullptr;
};

struct BlockTab {
  int bk = 0, Nk = 0;
  std::vector<ChunkTab> chunks;
};

// Column groups: powers of two up to kMaxGroupCols for stencil lattices.  An
// explicit matrix is read once per group and step, so it takes groups of any
// size up to kMaxGroupCols (the last wave of a group runs a body for its own
// column count; 5 columns as one group instead of 4 + 1: 3.93 -> 3.83 ms per
// complex128 step at D_H = 121 on MI355X).
std::vector<int> split_columns(int R, bool sparse = false) {
  std::vector<int> g;
  while (R > 0) {
    int p = 1;
    if (sparse) {
      p = std::min(R, kMaxGroupCols);
    } else {
      while (p * 2 <= std::min(R, kMaxGroupCols)) p *= 2;
    }
    g.push_back(p);
    R -= p;
  }
  return g;
}

// Key of the autotuner cache: precision, assembly and, per instance, the
// lattice shape and column count (which fixes the column groups).
std::string shape_key(const std::vector<InstIn>& ins, bool fp64, int assembly) {
  std::string k = fp64 ? "d" : "f";
  k += assembly == CSP_ASSEMBLE_MOMENTS ? "m" : "s";
  char buf[160];
  for (auto& in : ins) {
    const Geom& g = in.lat->g;
    snprintf(buf, sizeof(buf), "|%d:%lld:%lld:%d%d:%d:%d:%d", g.kind, (long long)g.Lx,
             (long long)g.Ly, g.px, g.py, in.lat->has_onsite ? 1 : 0, in.lat->ell_D, in.R);
    k += buf;
  }
  return k;
}

const csp_tuning* find_tuning(const csp_context* c, const std::vector<InstIn>& ins, bool fp64,
                              int assembly) {
  auto it = c->tuned.find(shape_key(ins, fp64, assembly));
  return it == c->tuned.end() ? nullptr : &it->second;
}

void fill_defaults(const csp_params* in, csp_params* p) {
  *p = *in;
  if (!(p->tau_tilde > 0)) p->tau_tilde = M_PI;
  if (!(p->eta > 0)) p->eta = 1e-14;
  if (!(p->norm_tol > 0)) p->norm_tol = 1e-3;
}

struct Profiler {
  csp_context* c;
  bool on;
  size_t next = 0;
  std::vector<std::pair<size_t, int>> spans;  // first event index, kind (0 spmm, 1 contract)
  csp_status begin(int kind, size_t* idx) {
    if (!on) return CSP_OK;
    hipEvent_t e0;
    CHECK(hip_event(c, next, &e0));
    HIPCALL(hipEventRecord(e0, c->stream));
    *idx = next;
    spans.push_back({next, kind});
    next += 2;
    return CSP_OK;
  }
  csp_status end(size_t idx) {
    if (!on) return CSP_OK;
    hipEvent_t e1;
    CHECK(hip_event(c, idx + 1, &e1));
    HIPCALL(hipEventRecord(e1, c->stream));
    return CSP_OK;
  }
  csp_status collect(double* ms_spmm, double* ms_contract) {
    *ms_spmm = 0;
    *ms_contract = 0;
    if (!on) return CSP_OK;
    for (auto& s : spans) {
      float ms = 0.f;
      HIPCALL(hipEventElapsedTime(&ms, c->events[s.first], c->events[s.first + 1]));
      (s.second == 0 ? *ms_spmm : *ms_contract) += ms;
    }
    return CSP_OK;
  }
};

int select_b_rule(const std::vector<int32_t>& ntr_all, int bmax, int64_t Nt, double t_amxsy,
                  double t_axpy, const std::vector<bool>& fits, double* model) {
  // C(b) = N_amxsy(b) t_amxsy + N_axpy(b) t_axpy (Sec. II.B) over the blocks
  // of b steps (last block shorter when b does not divide Nt).
  auto cost = [&](int b) {
    double amxsy = 0, axpy = 0;
    for (int64_t t0 = 0; t0 < Nt; t0 += b) {
      const int bk = (int)std::min<int64_t>(b, Nt - t0);
      amxsy += ntr_all[bk - 1];
      for (int j = 1; j <= bk; ++j) axpy += ntr_all[j - 1];
    }
    return amxsy * t_amxsy + axpy * t_axpy;
  };
  int best = 1;
  double bestc = cost(1);
  for (int b = 1, k = 0; b <= 128; b *= 2, ++k)
    if (model) model[k] = (b <= bmax && b <= (int)ntr_all.size()) ? cost(b) : -1.0;
  for (int b = 2; b <= bmax && b <= (int)ntr_all.size(); ++b) {
    if (!fits[b]) continue;
    const double cb = cost(b);
    if (cb < bestc) {
      bestc = cb;
      best = b;
    }
  }
  return best;
}

}  // namespace

static csp_status propagate_impl(csp_context* c, const std::vector<InstIn>& ins,
                                 const csp_params* params_in, csp_report* rep, bool batch_call,
                                 bool allow_split = true);

extern "C" csp_status csp_propagate(csp_context* c, const csp_lattice* L, const void* dev_psi0,
                                    int32_t R, const csp_params* params, double* dev_corr,
                                    void* dev_final, csp_report* rep) {
  if (!c || !L || !dev_psi0 || !params || !dev_corr) return fail(CSP_EINVAL, "NULL argument");
  std::vector<InstIn> ins(1);
  ins[0] = {L, dev_psi0, R, dev_corr, dev_final, R, 0};
  return propagate_impl(c, ins, params, rep, false);
}

extern "C" csp_status csp_propagate_batch(csp_context* c, int32_t n_inst,
                                          const csp_lattice* const* lats,
                                          const void* const* dev_psi0, const int32_t* R,
                                          const csp_params* params, double* const* dev_corr,
                                          csp_report* rep) {
  if (!c || n_inst < 1 || !lats || !dev_psi0 || !R || !params || !dev_corr)
    return fail(CSP_EINVAL, "NULL argument or n_inst < 1");
  std::vector<InstIn> ins(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    if (!lats[i] || !dev_psi0[i] || !dev_corr[i]) return fail(CSP_EINVAL, "instance %d NULL", i);
    ins[i] = {lats[i], dev_psi0[i], R[i], dev_corr[i], nullptr, R[i], 0};
  }
  return propagate_impl(c, ins, params, rep, true);
}

static csp_status propagate_moments_impl(csp_context* c, const std::vector<InstIn>& ins,
                                         const csp_params& P, double t_start, csp_report* rep);

// Column windows.  Every column is propagated independently, so when even
// the smallest workspace (a 16-order chunk plus psi0 and carry for the
// state assembly, 3 vectors plus psi0 and two carries for the moment
// assembly) of all columns exceeds the memory cap, the columns are run in
// passes over windows of at most w columns (w a power of two) per instance.
static csp_status plan_passes(csp_context* c, const std::vector<InstIn>& ins, const csp_params& P,
                              std::vector<std::vector<InstIn>>* passes) {
  const size_t csz = P.mode == CSP_FP32_CONC ? sizeof(float2) : sizeof(double2);
  const double slots = P.assembly == CSP_ASSEMBLE_MOMENTS ? 6.0 : 18.0;
  size_t cap_b = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap_b));
  const double cap = (double)cap_b;
  auto need = [&](const std::vector<InstIn>& v) {
    double vb = 0;
    for (auto& in : v) vb += (double)in.lat->g.N * in.R * csz;
    return vb * slots + (double)(96u << 20);
  };
  passes->clear();
  if (need(ins) <= cap) {
    passes->push_back(ins);
    return CSP_OK;
  }
  std::vector<InstIn> cur;
  for (auto& in : ins) {
    int w = 32;
    while (w > 1) {
      InstIn x = in;
      x.R = std::min(w, in.R);
      if (need({x}) <= cap) break;
      w /= 2;
    }
    for (int c0 = 0; c0 < in.R; c0 += w) {
      InstIn x = in;
      x.col_base = in.col_base + c0;
      x.R = std::min(w, in.R - c0);
      std::vector<InstIn> trial = cur;
      trial.push_back(x);
      if (!cur.empty() && need(trial) > cap) {
        passes->push_back(cur);
        cur.clear();
      }
      cur.push_back(x);
    }
  }
  if (!cur.empty()) passes->push_back(cur);
  return CSP_OK;
}

static csp_status propagate_impl(csp_context* c, const std::vector<InstIn>& ins,
                                 const csp_params* params_in, csp_report* rep, bool batch_call,
                                 bool allow_split) {
  const double t_start = now_ms();
  csp_params P;
  fill_defaults(params_in, &P);
  if (P.Nt < 0) return fail(CSP_EINVAL, "Nt < 0");
  if (P.mode < CSP_FP64_SEQ || P.mode > CSP_FP32_CONC) return fail(CSP_EINVAL, "bad mode %d", P.mode);
  if (P.assembly != CSP_ASSEMBLE_STATES && P.assembly != CSP_ASSEMBLE_MOMENTS)
    return fail(CSP_EINVAL, "bad assembly %d", P.assembly);
  for (size_t i = 0; i < ins.size(); ++i)
    if (ins[i].R < 1) return fail(CSP_EINVAL, "instance %zu: R must be >= 1", i);
  if (allow_split) {
    std::vector<std::vector<InstIn>> passes;
    {
      DeviceGuard dg0(c->device);
      CHECK(plan_passes(c, ins, P, &passes));
    }
    if (passes.size() > 1) {
      csp_report tot{};
      for (size_t p = 0; p < passes.size(); ++p) {
        csp_report r{};
        CHECK(propagate_impl(c, passes[p], params_in, &r, batch_call, false));
        tot.block_b = r.block_b;
        tot.chunk_K = r.chunk_K;
        tot.n_blocks = r.n_blocks;
        tot.n_groups += r.n_groups;
        tot.amxsy = std::max(tot.amxsy, r.amxsy);
        tot.axpy = std::max(tot.axpy, r.axpy);
        tot.dot = std::max(tot.dot, r.dot);
        tot.spmm_launches += r.spmm_launches;
        tot.contract_launches += r.contract_launches;
        tot.ms_spmm += r.ms_spmm;
        tot.ms_contract += r.ms_contract;
        tot.spmm_bytes += r.spmm_bytes;
        tot.contract_bytes += r.contract_bytes;
        tot.contract_flops += r.contract_flops;
        tot.workspace_bytes = std::max(tot.workspace_bytes, r.workspace_bytes);
        for (int k = 0; k < 8; ++k) tot.model_cost[k] = r.model_cost[k];
        tot.graph_blocks += r.graph_blocks;
        tot.spmm_steps = r.spmm_steps;
      }
      tot.n_passes = (int)passes.size();
      tot.ms_total = now_ms() - t_start;
      if (rep) *rep = tot;
      return CSP_OK;
    }
  }
  if (P.assembly == CSP_ASSEMBLE_MOMENTS) return propagate_moments_impl(c, ins, P, t_start, rep);
  const bool fp64 = P.mode != CSP_FP32_CONC;
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  for (size_t i = 0; i < ins.size(); ++i) {
    if (ins[i].R < 1) return fail(CSP_EINVAL, "instance %zu: R must be >= 1", i);
    if (ins[i].lat->ctx->device != c->device)
      return fail(CSP_EINVAL, "instance %zu: lattice on another device", i);
  }
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;

  // ---------------------------------------------------------- block size
  int bmax = P.mode == CSP_FP64_SEQ ? 1 : (fp64 ? kMaxFp64B : 32 * kMaxJTiles);
  int b = P.mode == CSP_FP64_SEQ ? 1 : P.block_b;
  if (b < 0) return fail(CSP_EINVAL, "block_b < 0");
  if (b > bmax) return fail(CSP_EUNSUPPORTED, "block_b %d above %d for this mode", b, bmax);
  const int64_t Nt = P.Nt;

  // Coefficients for x_j = j tau, j = 1..bmax (all block sizes share them).
  const int ncol = bmax;
  const int nmax = (int)trunc_nmax(ncol * P.tau_tilde);
  const int lda = nmax + 1;
  std::vector<int32_t> ntr(ncol);
  double* d_a = nullptr;
  int32_t* d_ntr = nullptr;
  struct Free {
    std::vector<void*> p;
    ~Free() { for (void* q : p) (void)hipFree(q); }
  } tmp;
  HIPCALL(hipMalloc(&d_a, sizeof(double) * (size_t)ncol * lda));
  tmp.p.push_back(d_a);
  HIPCALL(hipMalloc(&d_ntr, sizeof(int32_t) * ncol));
  tmp.p.push_back(d_ntr);
  HIPCALL(launch_bessel(P.tau_tilde, ncol, nmax, P.eta, true, d_a, d_ntr, s));
  HIPCALL(hipMemcpyAsync(ntr.data(), d_ntr, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, s));
  HIPCALL(hipStreamSynchronize(s));
  for (int j = 0; j < ncol; ++j)
    if (ntr[j] < 1) return fail(CSP_ENUMERIC, "no truncation order for x = %g", (j + 1) * P.tau_tilde);

  // ---------------------------------------------------------- groups & memory
  std::vector<Group> groups;
  int64_t vec_elems = 0;   // complex values of one vector over all groups (rows padded)
  int64_t vec_alg = 0;     // the same without the padding (algorithmic bytes)
  for (size_t i = 0; i < ins.size(); ++i) {
    int col = ins[i].col_base;
    for (int Rg : split_columns(ins[i].R, ins[i].lat->g.kind == CSP_SPARSE)) {
      Group g;
      g.inst = (int)i;
      g.col0 = col;
      g.Rg = Rg;
      set_layout(g, ins[i].lat);
      groups.push_back(g);
      vec_elems += g.M;
      vec_alg += ins[i].lat->g.N * Rg;
      col += Rg;
    }
  }
  size_t cap = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap));
  const size_t vec_bytes = (size_t)vec_elems * csz + 256 * groups.size();
  const csp_tuning* tune = find_tuning(c, ins, fp64, CSP_ASSEMBLE_STATES);
  const int total_wg_target = c->n_cu * (tune ? tune->contract_wg_per_cu : 4);
  const size_t fixed_guess = 2 * vec_bytes + (size_t)total_wg_target * 64 * 16 + (64u << 20);

  // recursion launch shape (steps per launch kt)
  std::vector<ChebInst> sp;
  for (auto& g : groups) {
    sp.push_back(make_inst(ins[g.inst].lat, g.Rg, fp64));
    apply_layout(sp.back(), g);
  }
  const ChebPlan sp_plan = plan_cheb(sp, fp64, false, c->n_cu, tune ? tune->spmm_vec : 0,
                                     tune ? tune->spmm_steps : (fp64 ? 4 : 8),
                                     tune ? tune->spmm_seg_rows : 0);
  const int kt = sp_plan.kt;

  auto fits_b = [&](int bb) {
    // Workspace with every order of a block resident, or at least 16 of them.
    const int need = std::min(ntr[bb - 1] + 1, 16) + kt;
    return fixed_guess + (size_t)need * vec_bytes <= cap;
  };
  if (b == 0 && tune && tune->block_b > 0 && tune->block_b <= bmax && fits_b(tune->block_b)) {
    b = tune->block_b;   // measured by csp_autotune for this shape
    if (rep)
      for (int k = 0; k < 8; ++k) rep->model_cost[k] = tune->model_cost_ms[k];
  } else if (b == 0) {
    std::vector<bool> fits(bmax + 1, false);
    for (int bb = 1; bb <= bmax; ++bb) fits[bb] = fits_b(bb);
    // Without a measurement: the byte model (a recursion step streams 3
    // vectors, one (n, j) pair of the contraction about 1/32 of a vector).
    b = select_b_rule(ntr, bmax, Nt, 3.0, 1.0 / 32.0, fits, rep ? rep->model_cost : nullptr);
  }
  if (Nt > 0) b = (int)std::min<int64_t>(b, Nt);
  b = std::max(b, 1);
  const int b_last = Nt > 0 ? (int)(Nt - (int64_t)(ceil_div(Nt, b) - 1) * b) : b;
  const int jtiles = fp64 ? 1 : (int)ceil_div(b, 32);
  const int N_full = ntr[b - 1];
  const int Ktot = N_full + 1;

  // Chunk size: all orders of a block if they fit, else the largest multiple
  // of 16 that fits.  The ring holds K + kt slots: a launch writes kt orders
  // past the newest one while the chunk in progress must stay intact.
  const size_t tabs_guess = (64u << 20);
  auto ring_slots = [&](int K_) { return std::max(K_ + kt, kt + 2); };
  auto ws_need = [&](int K_, int n_wg_total) {
    size_t by = 0;
    for (auto& g : groups)
      by += align256((size_t)ring_slots(K_) * g.stride() * csz) + 2 * align256(g.M * csz);
    by += align256((size_t)n_wg_total * b * 16) * 2;
    return by + tabs_guess;
  };
  const int wg_bound = total_wg_target + kMaxGroupCols * (int)groups.size();
  const int kcap = fp64 ? 1 << 20 : (496 / jtiles / 16) * 16;   // LDS budget of B operands
  int K = P.chunk_K > 0 ? P.chunk_K : Ktot;
  if (K >= Ktot && Ktot <= kcap && ws_need(Ktot, wg_bound) <= cap) {
    K = Ktot;
  } else {
    K = std::min(std::min(K, Ktot), kcap);
    K = std::max(16, (K / 16) * 16);
    while (K > 16 && ws_need(K, wg_bound) > cap) K -= 16;
  }
  const int S = ring_slots(K);
  const int RG = ring_parts(S);    // ring parts (slot of position k: ring_slot)
  if (ws_need(K, wg_bound) > cap)
    return fail(CSP_ENOMEM, "workspace for b=%d, K=%d exceeds the cap (%.2f GB)", b, K, cap / 1e9);

  // Contraction workgroups: per group proportional to its values, an equal
  // number on each of its columns.
  int64_t Msum = 0;
  for (auto& g : groups) Msum += g.M;
  int total_wg = 0;
  std::vector<int> wpc(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    const int64_t N = g.M / g.Rg;
    const int64_t units = fp64 ? ceil_div(N, kContractThreads) : ceil_div(ceil_div(N, 32), 4);
    const double share = (double)total_wg_target * (double)g.M / (double)Msum / g.Rg;
    wpc[gi] = (int)std::max<int64_t>(1, std::min<int64_t>(std::llround(share), units));
    g.n_wg = g.Rg * wpc[gi];
    total_wg += g.n_wg;
  }

  // ---------------------------------------------------------- block tables
  std::vector<BlockTab> btabs;
  auto make_tab = [&](int bk) {
    BlockTab t;
    t.bk = bk;
    t.Nk = ntr[bk - 1];
    for (int lo = 0; lo <= t.Nk; lo += K) t.chunks.push_back({lo, std::min(K, t.Nk + 1 - lo)});
    return t;
  };
  btabs.push_back(make_tab(b));
  if (b_last != b) btabs.push_back(make_tab(b_last));
  size_t tab_bytes = 0;
  for (auto& t : btabs)
    for (auto& ch : t.chunks)
      tab_bytes += fp64 ? align256(sizeof(double2) * ch.n_cnt * t.bk) + align256(sizeof(double2) * ch.n_cnt)
                        : align256(bop_bytes(jtiles, ch.n_cnt)) + align256(sizeof(float) * 16 * ceil_div(ch.n_cnt, 16));

  // ---------------------------------------------------------- workspace
  size_t need = tab_bytes;
  for (auto& g : groups) {
    need += align256((size_t)S * g.stride() * csz) + 2 * align256(g.M * csz);
    need += align256((size_t)g.n_wg * b * 16);
  }
  const size_t n_sd = 256;   // self-dot partial blocks
  need += align256(sizeof(double) * n_sd * kMaxGroupCols);
  need += align256(2 * sizeof(int)) + align256(2 * sizeof(int64_t));
  need += align256(sizeof(ChebInst) * groups.size()) + align256(sizeof(ContractInst) * groups.size()) +
          align256(sizeof(FinishInst) * groups.size());
  if (need > cap) return fail(CSP_ENOMEM, "workspace %.2f GB exceeds the cap %.2f GB", need / 1e9, cap / 1e9);
  CHECK(ws_reserve(c, need));
  Carver cv(c->ws);
  for (auto& t : btabs)
    for (auto& ch : t.chunks) {
      if (fp64) {
        ch.coef = (double*)cv.take(sizeof(double2) * ch.n_cnt * t.bk);
        ch.ccd = (double*)cv.take(sizeof(double2) * ch.n_cnt);
        HIPCALL(launch_pack_c64(d_a, lda, d_ntr, t.bk, ch.n_lo, ch.n_cnt, ch.coef, ch.ccd, s));
      } else {
        ch.bop = cv.take(bop_bytes(jtiles, ch.n_cnt));
        ch.ccf = (float*)cv.take(sizeof(float) * 16 * ceil_div(ch.n_cnt, 16));
        HIPCALL(launch_pack_bop(d_a, lda, d_ntr, t.bk, jtiles, ch.n_lo, ch.n_cnt, ch.bop, ch.ccf, s));
      }
    }
  for (auto& g : groups) {
    g.slots = cv.take((size_t)S * g.stride() * csz);
    g.psi0g = cv.take(g.M * csz);
    g.carry = cv.take(g.M * csz);
    g.partial = (double*)cv.take((size_t)g.n_wg * b * 16);
    // the contraction reads whole vectors: the row padding of the slots,
    // which the recursion never writes, must hold zeros
    if (g.pitch > 0) {
      const csp_lattice* L = ins[g.inst].lat;
      HIPCALL(launch_zero_pad(g.slots, S, g.stride(), g.Rg, g.cstride, L->g.Ly, L->g.opr, g.pitch,
                              fp64, s));
    }
  }
  double* d_sd = (double*)cv.take(sizeof(double) * n_sd * kMaxGroupCols);
  int* d_flag = (int*)cv.take(2 * sizeof(int));
  int64_t* d_blk = (int64_t*)cv.take(2 * sizeof(int64_t));
  ChebInst* d_spmm = (ChebInst*)cv.take(sizeof(ChebInst) * groups.size());
  ContractInst* d_con = (ContractInst*)cv.take(sizeof(ContractInst) * groups.size());
  FinishInst* d_fin = (FinishInst*)cv.take(sizeof(FinishInst) * groups.size());

  // ---------------------------------------------------------- instance tables
  std::vector<ContractInst> ct;
  std::vector<FinishInst> fi;
  int wg0 = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    const InstIn& in = ins[g.inst];
    ChebInst& I = sp[gi];
    I.base = g.slots;
    I.slot_stride = g.stride();
    I.src = g.carry;
    ContractInst C{};
    C.slots = g.slots;
    C.slot_stride = g.stride();
    C.N = g.M / g.Rg;
    C.Rg = g.Rg;
    C.wpc = wpc[gi];
    C.psi0 = g.psi0g;
    C.carry = g.carry;
    C.partial = g.partial;
    C.wg0 = wg0;
    C.n_wg = g.n_wg;
    wg0 += g.n_wg;
    ct.push_back(C);
    FinishInst F{};
    F.partial = g.partial;
    F.wpc = wpc[gi];
    F.Rg = g.Rg;
    F.corr = in.corr;
    F.ldc = in.ld;
    F.col0 = g.col0;
    fi.push_back(F);
  }
  CHECK(attach_ell_shadows(c, sp, fp64));
  HIPCALL(hipMemcpyAsync(d_spmm, sp.data(), sizeof(ChebInst) * sp.size(), hipMemcpyHostToDevice, s));
  HIPCALL(hipMemcpyAsync(d_con, ct.data(), sizeof(ContractInst) * ct.size(), hipMemcpyHostToDevice, s));
  HIPCALL(hipMemcpyAsync(d_fin, fi.data(), sizeof(FinishInst) * fi.size(), hipMemcpyHostToDevice, s));

  // ---------------------------------------------------------- initial state, C_0
  for (auto& g : groups) {
    const InstIn& in = ins[g.inst];
    const int in_dtype = fp64 ? CSP_C128 : CSP_C64;
    const int64_t N = in.lat->g.N;
    HIPCALL(launch_gather_cols(N, in.ld, g.col0, g.Rg, in_dtype, in.psi0, fp64, g.psi0g, s,
                               in.lat->g.opr, g.pitch));
    HIPCALL(hipMemcpyAsync(g.carry, g.psi0g, g.M * csz, hipMemcpyDeviceToDevice, s));
    // over the padded columns: the padding is zero
    HIPCALL(launch_self_dot(g.cstride, g.Rg, g.psi0g, fp64, in.corr, g.col0, d_sd, (int)n_sd, s));
  }

  // ---------------------------------------------------------- blocks
  if (P.check_norm) CHECK(guard_reset(d_flag, s));
  Profiler prof{c, P.profile != 0};
  int64_t n_spmm = 0, n_con = 0, amxsy = 0, axpy = 0;
  double spmm_bytes = 0, con_bytes = 0, con_flops = 0;
  double eps_bytes = 0;
  for (auto& g : groups)
    eps_bytes += static_bytes(ins[g.inst].lat, fp64);
  const double vbytes = (double)vec_alg * csz;

  ContractArgs ca{};
  ca.n_inst = (int)groups.size();
  ca.S = S;
  ca.G = RG;
  ca.jtiles = jtiles;
  ca.total_wg = total_wg;
  const ChebStep st0 = step_args(sp_plan);

  // One time block: recursion launches of up to kt steps each, with the
  // contraction of every chunk of orders as soon as its last order exists,
  // then the per-column partial sums and the norm guard.  from_dev: the
  // block's time index and number come from the device counter (graph
  // replays), which the block then advances.
  auto enqueue_block = [&](const BlockTab& T, int bk, int64_t t0, hipStream_t strm,
                           bool from_dev) -> csp_status {
    const int Nk = T.Nk;
    size_t ci = 0;
    int produced = 0;
    ContractArgs cab = ca;
    auto run_chunks = [&]() -> csp_status {
      while (ci < T.chunks.size() && T.chunks[ci].n_lo + T.chunks[ci].n_cnt - 1 <= produced) {
        const ChunkTab& ch = T.chunks[ci];
        size_t evc = 0;
        if (!from_dev) CHECK(prof.begin(1, &evc));
        cab.n_lo = ch.n_lo;
        cab.n_cnt = ch.n_cnt;
        cab.first_chunk = ci == 0 ? 1 : 0;
        cab.bcols = bk;
        if (fp64) {
          cab.coef = ch.coef;
          cab.ccarry = ch.ccd;
          HIPCALL(launch_contract_f64(d_con, cab, strm));
        } else {
          cab.bop = ch.bop;
          cab.ccarry = ch.ccf;
          HIPCALL(launch_contract_f32(d_con, cab, strm));
        }
        if (!from_dev) CHECK(prof.end(evc));
        ++ci;
      }
      return CSP_OK;
    };
    while (produced < Nk) {
      ChebStep stb = st0;
      stb.nlev = std::min(kt, Nk - produced);
      if (produced == 0) {
        // block start: phi_0 = carried state (copied to slot 0), phi_1 = H~ phi_0
        stb.first = 1;
        stb.slot_cur = -1;
        stb.copy_slot = 0;
      } else {
        stb.slot_cur = ring_slot(produced % S, S, RG);
        stb.slot_prev = ring_slot((produced - 1) % S, S, RG);
      }
      for (int l = 1; l <= stb.nlev; ++l)
        stb.slot_out[l - 1] = ring_slot((produced + l) % S, S, RG);
      size_t ev = 0;
      if (!from_dev) CHECK(prof.begin(0, &ev));
      set_shadow(stb, produced);
      HIPCALL(launch_cheb(fp64, sp_plan.vec, kt, false, false, d_spmm, sp_plan.runs, stb, strm));
      if (!from_dev) CHECK(prof.end(ev));
      produced += stb.nlev;
      CHECK(run_chunks());
    }
    HIPCALL(launch_finish(d_fin, (int)fi.size(), bk, t0, from_dev ? d_blk : nullptr, strm));
    if (P.check_norm) {
      for (auto& g : groups) {
        const InstIn& in = ins[g.inst];
        HIPCALL(launch_guard(g.cstride, g.Rg, g.carry, fp64, in.corr, in.ld, g.col0, t0, bk,
                             P.norm_tol, (int)(t0 / b), from_dev ? d_blk : nullptr, d_flag, d_sd,
                             (int)n_sd, strm));
      }
    }
    if (from_dev) HIPCALL(launch_advance(d_blk, b, strm));
    return CSP_OK;
  };
  auto count_block = [&](const BlockTab& T, int bk) {
    const int Nk = T.Nk;
    amxsy += Nk;
    for (int j = 1; j <= bk; ++j) axpy += ntr[j - 1];
    // algorithmic bytes of a launch of l steps: read phi_n, phi_{n-1} (the
    // first launch reads phi_0 only and writes it once), write l vectors
    for (int done = 0; done < Nk; done += kt) {
      const int l = std::min(kt, Nk - done);
      ++n_spmm;
      spmm_bytes += vbytes * (done == 0 ? 2.0 + l : 2.0 + l) + eps_bytes;
    }
    for (size_t ci = 0; ci < T.chunks.size(); ++ci) {
      const ChunkTab& ch = T.chunks[ci];
      ++n_con;
      con_bytes += vbytes * (ch.n_cnt + 2 + (ci == 0 ? 0 : 1));
      con_flops += fp64 ? 8.0 * (double)vec_alg * ch.n_cnt * (bk + 1)
                        : 2.0 * 6.0 * 32.0 * 32.0 * 16.0 * jtiles *
                              (double)ceil_div(ch.n_cnt, 16) * (double)ceil_div(vec_alg, 32);
    }
  };

  // Graph replay of the full blocks (state assembly), unless profiling.
  const int64_t n_full = Nt / b;
  bool use_graph = !prof.on && n_full >= 2 &&
                   (P.graph > 0 || (P.graph == 0 && ins.size() > 1 && batch_call));
  hipGraphExec_t gexec = nullptr;
  if (use_graph) {
    const char* force = std::getenv("CSP_FORCE_GRAPH_FAILURE");
    hipGraph_t graph = nullptr;
    bool ok = !(force && force[0] == '1');
    if (ok) ok = capture_stream(c) == CSP_OK;
    if (ok) {
      static const int64_t blk0[2] = {0, 0};
      ok = hipMemcpyAsync(d_blk, blk0, sizeof(blk0), hipMemcpyHostToDevice, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
    }
    if (ok) ok = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const csp_status st_cap = enqueue_block(btabs[0], (int)b, 0, c->cap, true);
      const bool end_ok = hipStreamEndCapture(c->cap, &graph) == hipSuccess;
      ok = st_cap == CSP_OK && end_ok && graph;
    }
    if (ok) ok = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    if (!ok) {
      (void)hipGetLastError();
      if (gexec) (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
      use_graph = false;   // issue the launches directly
    }
  }
  struct ExecGuard {
    hipGraphExec_t e;
    ~ExecGuard() { if (e) (void)hipGraphExecDestroy(e); }
  } exec_guard{gexec};

  int graph_blocks = 0;
  for (int64_t t0 = 0; t0 < Nt; t0 += b) {
    const int bk = (int)std::min<int64_t>(b, Nt - t0);
    const BlockTab& T = (bk == b) ? btabs[0] : btabs.back();
    count_block(T, bk);
    if (use_graph && bk == b) {
      HIPCALL(hipGraphLaunch(gexec, s));
      ++graph_blocks;
    } else {
      CHECK(enqueue_block(T, bk, t0, s, false));
    }
  }

  // ---------------------------------------------------------- final state
  for (auto& g : groups) {
    const InstIn& in = ins[g.inst];
    if (!in.final_out) continue;
    HIPCALL(launch_scatter_cols(in.lat->g.N, in.ld, g.col0, g.Rg, fp64 ? CSP_C128 : CSP_C64,
                                g.carry, fp64, in.final_out, s, in.lat->g.opr, g.pitch));
  }
  HIPCALL(hipStreamSynchronize(s));
  if (P.check_norm) CHECK(guard_check(d_flag, s));

  if (rep) {
    double ms_s = 0, ms_c = 0;
    CHECK(prof.collect(&ms_s, &ms_c));
    rep->block_b = b;
    rep->chunk_K = K;
    rep->n_blocks = (int)(Nt > 0 ? ceil_div(Nt, b) : 0);
    rep->n_groups = (int)groups.size();
    rep->amxsy = amxsy;
    rep->axpy = axpy;
    rep->dot = Nt;
    rep->spmm_launches = n_spmm;
    rep->contract_launches = n_con;
    rep->ms_total = now_ms() - t_start;
    rep->ms_spmm = ms_s;
    rep->ms_contract = ms_c;
    rep->spmm_bytes = spmm_bytes;
    rep->contract_bytes = con_bytes;
    rep->contract_flops = con_flops;
    rep->workspace_bytes = c->ws_size;
    rep->graph_blocks = graph_blocks;
    rep->n_passes = 1;
    rep->spmm_steps = kt;
  }
  return CSP_OK;
}

// ------------------------------------------------------------------ moment form
// Moment-based propagation (Sec. II.A moment-based implementation): per time
// block the recursion runs with the moment epilogue (inner products with
// psi0, and with halving the self products of Eq. cheby_prod), the block
// moments are contracted with the coefficients in FP64, and with more than
// one block the epilogue also accumulates the carried state.  Three
// Chebyshev vectors per column group are kept (Tab. cost: 3 states).
static csp_status propagate_moments_impl(csp_context* c, const std::vector<InstIn>& ins,
                                         const csp_params& P, double t_start, csp_report* rep) {
  const bool fp64 = P.mode != CSP_FP32_CONC;
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  const int64_t Nt = P.Nt;
  for (size_t i = 0; i < ins.size(); ++i) {
    if (ins[i].R < 1) return fail(CSP_EINVAL, "instance %zu: R must be >= 1", i);
    if (ins[i].lat->ctx->device != c->device)
      return fail(CSP_EINVAL, "instance %zu: lattice on another device", i);
  }
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;
  bool want_final = false;
  for (auto& in : ins) want_final |= in.final_out != nullptr;

  // Block size: sequential mode is b = 1; otherwise block_b, 0 = one block.
  int64_t b = P.mode == CSP_FP64_SEQ ? 1 : (P.block_b > 0 ? P.block_b : std::max<int64_t>(Nt, 1));
  if (Nt > 0) b = std::min<int64_t>(b, Nt);
  if (b > (1 << 20)) return fail(CSP_EUNSUPPORTED, "block of %lld steps", (long long)b);
  const bool single = b >= Nt;
  const bool halving = single && !want_final && Nt > 0;
  const bool carry = !single || want_final;
  const int64_t b_last = Nt > 0 ? Nt - (ceil_div(Nt, b) - 1) * b : b;

  // Coefficient table a[j][n], x = (j + 1) tau, j < b.
  const int ncol = (int)b;
  const int nmax = (int)trunc_nmax((double)ncol * P.tau_tilde);
  const int lda = nmax + 1;
  struct Free {
    std::vector<void*> p;
    ~Free() { for (void* q : p) (void)hipFree(q); }
  } tmp;
  double* d_a = nullptr;
  int32_t* d_ntr = nullptr;
  HIPCALL(hipMalloc(&d_a, sizeof(double) * (size_t)ncol * lda));
  tmp.p.push_back(d_a);
  HIPCALL(hipMalloc(&d_ntr, sizeof(int32_t) * ncol));
  tmp.p.push_back(d_ntr);
  HIPCALL(launch_bessel(P.tau_tilde, ncol, nmax, P.eta, true, d_a, d_ntr, s));
  std::vector<int32_t> ntr(ncol);
  HIPCALL(hipMemcpyAsync(ntr.data(), d_ntr, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, s));
  // carry coefficients: rows of the block lengths b and b_last
  std::vector<double> arow_b, arow_last;
  if (carry) {
    arow_b.resize(lda);
    arow_last.resize(lda);
    HIPCALL(hipMemcpyAsync(arow_b.data(), d_a + (size_t)(b - 1) * lda, sizeof(double) * lda,
                           hipMemcpyDeviceToHost, s));
    HIPCALL(hipMemcpyAsync(arow_last.data(), d_a + (size_t)(b_last - 1) * lda,
                           sizeof(double) * lda, hipMemcpyDeviceToHost, s));
  }
  HIPCALL(hipStreamSynchronize(s));
  for (int j = 0; j < ncol; ++j)
    if (ntr[j] < 1) return fail(CSP_ENUMERIC, "no truncation order for x = %g", (j + 1) * P.tau_tilde);
  const int Nk_max = ntr[b - 1];
  const int steps_max = halving ? (Nk_max + 1) / 2 : Nk_max;

  // Column groups (powers of two, <= 32 columns).
  std::vector<Group> groups;
  int64_t vec_alg = 0;     // complex values of one vector over all groups (unpadded)
  int rmax = 1;
  for (size_t i = 0; i < ins.size(); ++i) {
    int col = ins[i].col_base;
    for (int Rg : split_columns(ins[i].R, ins[i].lat->g.kind == CSP_SPARSE)) {
      Group g;
      g.inst = (int)i;
      g.col0 = col;
      g.Rg = Rg;
      set_layout(g, ins[i].lat);
      groups.push_back(g);
      vec_alg += ins[i].lat->g.N * Rg;
      rmax = std::max(rmax, Rg);
      col += Rg;
    }
  }
  std::vector<ChebInst> sp;
  for (auto& g : groups) {
    sp.push_back(make_inst(ins[g.inst].lat, g.Rg, fp64));
    apply_layout(sp.back(), g);
  }
  const csp_tuning* tune = find_tuning(c, ins, fp64, CSP_ASSEMBLE_MOMENTS);
  int vec_want = tune ? tune->spmm_vec : 0;
  // default: 8 steps per launch for the complex64 self-product kernel
  // (halving), 4 where psi0 or the carried state take registers
  int kt_want = tune ? tune->spmm_steps : (halving && !fp64 ? 8 : 4);
  if (carry && !cheb_carry_supported(fp64, 2, kt_want)) kt_want = 4;
  if (carry) vec_want = 2;   // the carried-state kernels hold 2 values per lane
  const ChebPlan sp_plan = plan_cheb(sp, fp64, true, c->n_cu, vec_want, kt_want,
                                     tune ? tune->spmm_seg_rows : 0);
  const int kt = sp_plan.kt;
  const int P_batch = 16;

  // Workspace.
  size_t need = 0;
  const size_t part_bytes = (size_t)P_batch * kt * sp_plan.total_items * 8 * sizeof(double);
  need += align256(part_bytes);
  for (auto& g : groups) {
    need += align256(4 * g.stride() * csz) + align256(g.M * csz);   // ring + psi0
    if (carry) need += 2 * align256(g.M * csz);                      // carry in / out
    need += align256((size_t)(steps_max + 1) * 4 * g.Rg * 16);       // dots
    need += align256((size_t)(Nk_max + 1) * g.Rg * 16);              // mu
  }
  need += align256(sizeof(ChebInst) * groups.size()) + align256(sizeof(MomInst) * groups.size()) +
          align256(sizeof(MomCorrInst) * groups.size()) +
          align256(sizeof(double) * 256 * kMaxGroupCols) + align256(2 * sizeof(int));
  size_t cap = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap));
  if (need > cap)
    return fail(CSP_ENOMEM, "workspace %.2f GB exceeds the cap %.2f GB", need / 1e9, cap / 1e9);
  CHECK(ws_reserve(c, need));
  Carver cv(c->ws);
  double* d_part = (double*)cv.take(part_bytes);
  std::vector<void*> carry_a(groups.size()), carry_b(groups.size());
  std::vector<double*> dots(groups.size()), mus(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    g.slots = cv.take(4 * g.stride() * csz);
    g.psi0g = cv.take(g.M * csz);
    if (carry) {
      carry_a[gi] = cv.take(g.M * csz);
      carry_b[gi] = cv.take(g.M * csz);
      // the recursion writes rows only; the norm guard reads whole vectors
      if (g.pitch > 0) {
        const csp_lattice* L = ins[g.inst].lat;
        HIPCALL(launch_zero_pad(carry_b[gi], 1, 0, g.Rg, g.cstride, L->g.Ly, L->g.opr, g.pitch,
                                fp64, s));
      }
    }
    dots[gi] = (double*)cv.take((size_t)(steps_max + 1) * 4 * g.Rg * 16);
    mus[gi] = (double*)cv.take((size_t)(Nk_max + 1) * g.Rg * 16);
  }
  ChebInst* d_spmm = (ChebInst*)cv.take(sizeof(ChebInst) * groups.size());
  MomInst* d_mi = (MomInst*)cv.take(sizeof(MomInst) * groups.size());
  MomCorrInst* d_mc = (MomCorrInst*)cv.take(sizeof(MomCorrInst) * groups.size());
  double* d_sd = (double*)cv.take(sizeof(double) * 256 * kMaxGroupCols);
  int* d_flag = (int*)cv.take(2 * sizeof(int));
  if (P.check_norm) CHECK(guard_reset(d_flag, s));

  // Initial state, C_0, instance tables.
  std::vector<MomInst> mi;
  std::vector<MomCorrInst> mc;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    const InstIn& in = ins[g.inst];
    const int64_t N = in.lat->g.N;
    HIPCALL(launch_gather_cols(N, in.ld, g.col0, g.Rg, fp64 ? CSP_C128 : CSP_C64, in.psi0, fp64,
                               g.psi0g, s, in.lat->g.opr, g.pitch));
    HIPCALL(launch_self_dot(g.cstride, g.Rg, g.psi0g, fp64, in.corr, g.col0, d_sd, 256, s));
    if (carry)
      HIPCALL(hipMemcpyAsync(carry_a[gi], g.psi0g, g.M * csz, hipMemcpyDeviceToDevice, s));
    ChebInst& I = sp[gi];
    I.base = g.slots;
    I.slot_stride = g.stride();
    I.psi0 = g.psi0g;
    MomInst m{};
    m.tile0 = I.item0;
    m.n_tiles = (int64_t)g.Rg * I.n_strips * I.n_segs;
    m.Rg = g.Rg;
    m.dots = dots[gi];
    mi.push_back(m);
    MomCorrInst q{};
    q.dots = dots[gi];
    q.mu = mus[gi];
    q.corr = in.corr;
    q.ldc = in.ld;
    q.Rg = g.Rg;
    q.col0 = g.col0;
    mc.push_back(q);
  }
  HIPCALL(hipMemcpyAsync(d_mi, mi.data(), sizeof(MomInst) * mi.size(), hipMemcpyHostToDevice, s));
  HIPCALL(hipMemcpyAsync(d_mc, mc.data(), sizeof(MomCorrInst) * mc.size(), hipMemcpyHostToDevice, s));

  Profiler prof{c, P.profile != 0};
  int64_t n_spmm = 0, amxsy = 0, axpy = 0, ndot = 0;
  double spmm_bytes = 0;
  double eps_bytes = 0;
  for (auto& g : groups)
    eps_bytes += static_bytes(ins[g.inst].lat, fp64);
  const double vbytes = (double)vec_alg * csz;

  const ChebStep st0 = step_args(sp_plan);
  int cur_carry = 0;   // carry_a holds s_k when 0
  for (int64_t t0 = 0; t0 < Nt; t0 += b) {
    const int bk = (int)std::min<int64_t>(b, Nt - t0);
    const int Nk = ntr[bk - 1];
    const int steps = halving ? (Nk + 1) / 2 : Nk;
    const std::vector<double>& arow = (bk == b) ? arow_b : arow_last;
    // per-block instance table: source and carry destination
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      ChebInst& I = sp[gi];
      if (carry) {
        I.src = cur_carry == 0 ? carry_a[gi] : carry_b[gi];
        I.carry = cur_carry == 0 ? carry_b[gi] : carry_a[gi];
      } else {
        I.src = groups[gi].psi0g;
        I.carry = nullptr;
      }
    }
    CHECK(attach_ell_shadows(c, sp, fp64));
    HIPCALL(hipMemcpyAsync(d_spmm, sp.data(), sizeof(ChebInst) * sp.size(), hipMemcpyHostToDevice, s));
    // four slots: phi_n, phi_{n-1} and the two newest levels of a launch
    int cur_slot = -1, prev_slot = -1;
    int produced = 0;
    int launches = 0;          // launches in the pending batch of records
    int batch0 = 1;            // order produced by the first level of that batch
    while (produced < steps) {
      ChebStep st = st0;
      st.nlev = std::min(kt, steps - produced);
      int freeb[4], nf = 0;
      for (int q = 0; q < 4; ++q)
        if (q != cur_slot && q != prev_slot) freeb[nf++] = q;
      int new_cur = freeb[0], new_prev;
      if (produced == 0) {
        st.first = 1;
        st.slot_cur = -1;
        if (st.nlev == 1) {
          st.copy_slot = freeb[1];     // phi_0 is the next launch's phi_{n-1}
          new_prev = freeb[1];
        } else {
          new_prev = freeb[1];
        }
      } else {
        st.slot_cur = cur_slot;
        st.slot_prev = prev_slot;
        new_prev = st.nlev == 1 ? cur_slot : freeb[1];
      }
      st.slot_out[st.nlev - 1] = new_cur;
      if (st.nlev >= 2) st.slot_out[st.nlev - 2] = new_prev;
      // With halving every moment above mu_1 comes from the self products
      // <phi_k|phi_k> and <phi_k|phi_k-1> (Eq. cheby_prod): psi0 is read by
      // the first launch only (mu_0, mu_1); the others run the kernel
      // without psi0.
      st.dot_psi0 = (!halving || produced == 0) ? 1 : 0;
      st.dot_self = halving ? 1 : 0;
      st.mom_slot = launches;
      st.partial = d_part;
      if (carry) {
        auto coef = [&](int n, double* out2) {
          const double v = arow[n];
          switch (n & 3) {   // (-i)^n v
            case 0: out2[0] = v; out2[1] = 0.0; break;
            case 1: out2[0] = 0.0; out2[1] = -v; break;
            case 2: out2[0] = -v; out2[1] = 0.0; break;
            default: out2[0] = 0.0; out2[1] = v; break;
          }
        };
        st.carry_mode = produced == 0 ? 1 : 2;
        coef(0, st.cc0);
        for (int l = 1; l <= st.nlev; ++l) coef(produced + l, st.ccl[l - 1]);
        axpy += st.nlev + (produced == 0 ? 1 : 0);
      }
      size_t ev = 0;
      CHECK(prof.begin(0, &ev));
      set_shadow(st, produced);
      HIPCALL(launch_cheb(fp64, sp_plan.vec, kt, true, carry, d_spmm, sp_plan.runs, st, s));
      CHECK(prof.end(ev));
      ++n_spmm;
      amxsy += st.nlev;
      spmm_bytes += vbytes * ((produced == 0 ? 1.0 : 2.0) + std::min(st.nlev, 2) +
                              (st.copy_slot >= 0 ? 1.0 : 0.0) + (st.dot_psi0 ? 1.0 : 0.0) +
                              (carry ? (produced == 0 ? 1.0 : 2.0) : 0.0)) +
                    eps_bytes;
      produced += st.nlev;
      cur_slot = new_cur;
      prev_slot = new_prev;
      ++launches;
      if (launches == P_batch || produced >= steps) {
        HIPCALL(launch_cheb_mom_finish(d_mi, (int)mi.size(), d_part, sp_plan.total_items, kt,
                                       launches, batch0, produced, s));
        batch0 = produced + 1;
        launches = 0;
      }
    }
    ndot += Nk;
    HIPCALL(launch_mom_corr(d_mc, (int)mc.size(), Nk, halving ? 1 : 0, d_a, lda, d_ntr, bk, t0,
                            rmax, s));
    if (P.check_norm) {
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        const InstIn& in = ins[g.inst];
        const void* cy = carry ? (cur_carry == 0 ? carry_b[gi] : carry_a[gi]) : nullptr;
        HIPCALL(launch_guard(g.cstride, g.Rg, cy, fp64, in.corr, in.ld, g.col0, t0, bk,
                             P.norm_tol, (int)(t0 / b), nullptr, d_flag, d_sd, 256, s));
      }
    }
    if (carry) cur_carry ^= 1;
  }
  // final state
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    const InstIn& in = ins[g.inst];
    if (!in.final_out) continue;
    void* fin = cur_carry == 0 ? carry_a[gi] : carry_b[gi];
    HIPCALL(launch_scatter_cols(in.lat->g.N, in.ld, g.col0, g.Rg, fp64 ? CSP_C128 : CSP_C64, fin,
                                fp64, in.final_out, s, in.lat->g.opr, g.pitch));
  }
  HIPCALL(hipStreamSynchronize(s));
  if (P.check_norm) CHECK(guard_check(d_flag, s));
  if (rep) {
    double ms_s = 0, ms_c = 0;
    CHECK(prof.collect(&ms_s, &ms_c));
    rep->block_b = (int)b;
    rep->chunk_K = 3;
    rep->n_blocks = (int)(Nt > 0 ? ceil_div(Nt, b) : 0);
    rep->n_groups = (int)groups.size();
    rep->amxsy = amxsy;
    rep->axpy = axpy;
    rep->dot = ndot;
    rep->spmm_launches = n_spmm;
    rep->contract_launches = 0;
    rep->ms_total = now_ms() - t_start;
    rep->ms_spmm = ms_s;
    rep->ms_contract = ms_c;
    rep->spmm_bytes = spmm_bytes;
    rep->contract_bytes = 0;
    rep->contract_flops = 0;
    rep->workspace_bytes = c->ws_size;
    rep->graph_blocks = 0;
    rep->n_passes = 1;
    rep->spmm_steps = kt;
  }
  return CSP_OK;
}

// ------------------------------------------------------------------ quasi-eigenstates
// QE-Concurrent-E (QE section): the Chebyshev vectors of psi0 up to
// N(Nt tau~) are produced by the recursion into a ring of K + kt slots and
// contracted chunk by chunk with the real coefficients C_n(E) of Eq.
// QE_coeff into one accumulated state per energy and column.
namespace {
// QE-Concurrent-S: forward and backward carried states per column, time
// blocks of b steps; per block one recursion of each carried state into a
// ring and contractions with the block's complex coefficients (energies and
// the next carried state as one more row).  Arguments validated by the caller.
csp_status qe_state_based(csp_context* c, const csp_lattice* L, const void* dev_psi0, int32_t R,
                          const csp_params& P, int nE, const double* energies, void* dev_qe,
                          csp_report* rep, double t_start) {
  const bool fp64 = P.mode == CSP_FP64_CONC;
  hipStream_t s = c->stream;
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  const int Nt = (int)P.Nt;
  const int b = (int)std::min<int64_t>(P.block_b, P.Nt);
  const int64_t N = L->g.N;
  const int rows = nE + 1;
  const double tau = P.tau_tilde / L->halfwidth;
  struct Free {
    std::vector<void*> p;
    ~Free() { for (void* q : p) (void)hipFree(q); }
  } tmp;
  auto alloc = [&](void** ptr, size_t bytes) -> csp_status {
    HIPCALL(hipMalloc(ptr, bytes));
    tmp.p.push_back(*ptr);
    return CSP_OK;
  };
  // Bessel table for x = j tau~, j = 1..b
  const int nmax_tab = (int)trunc_nmax((double)b * P.tau_tilde);
  const int lda = nmax_tab + 1;
  double *d_a = nullptr, *d_E = nullptr, *d_C = nullptr;
  int32_t* d_ntr = nullptr;
  CHECK(alloc((void**)&d_a, sizeof(double) * (size_t)b * lda));
  CHECK(alloc((void**)&d_ntr, sizeof(int32_t) * b));
  HIPCALL(launch_bessel(P.tau_tilde, b, nmax_tab, P.eta, true, d_a, d_ntr, s));
  std::vector<int32_t> ntr(b);
  HIPCALL(hipMemcpyAsync(ntr.data(), d_ntr, sizeof(int32_t) * b, hipMemcpyDeviceToHost, s));
  HIPCALL(hipStreamSynchronize(s));
  const int NkMax = ntr[b - 1];
  if (NkMax < 1) return fail(CSP_ENUMERIC, "no truncation order for x = %g", b * P.tau_tilde);
  CHECK(alloc((void**)&d_E, sizeof(double) * nE));
  CHECK(alloc((void**)&d_C, sizeof(double2) * (size_t)rows * (NkMax + 1)));
  HIPCALL(hipMemcpyAsync(d_E, energies, sizeof(double) * nE, hipMemcpyHostToDevice, s));

  // instances: forward and backward of every column group
  std::vector<Group> groups;
  {
    int col = 0;
    for (int Rg : split_columns(R, L->g.kind == CSP_SPARSE)) {
      Group g;
      g.inst = 0;
      g.col0 = col;
      g.Rg = Rg;
      g.M = N * Rg;
      groups.push_back(g);
      col += Rg;
    }
  }
  std::vector<ChebInst> sp;
  for (auto& g : groups)
    for (int d = 0; d < 2; ++d) sp.push_back(make_inst(L, g.Rg, fp64));
  const ChebPlan sp_plan = plan_cheb(sp, fp64, false, c->n_cu, 2, fp64 ? 4 : 8, 0);
  const int kt = sp_plan.kt;
  int B64 = 1;
  while (B64 < rows) B64 *= 2;
  const int kcap = fp64 ? (int)((60 * 1024) / (sizeof(double2) * B64)) / 16 * 16 : 240;
  size_t cap = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap));
  auto ws_need = [&](int K_) {
    size_t by = 0;
    for (auto& g : groups)
      by += 2 * (align256((size_t)(K_ + kt) * g.stride() * csz) + align256(g.M * csz) +
                 align256((size_t)nE * g.M * csz));
    by += fp64 ? align256(sizeof(double2) * (size_t)K_ * B64)
               : align256((size_t)64 * 64 * ceil_div(K_, 16));
    by += align256(sizeof(ChebInst) * sp.size()) + align256(sizeof(QeInst) * sp.size());
    return by;
  };
  int K = std::min(NkMax + 1, kcap);
  if (K < NkMax + 1) K = std::max(16, K / 16 * 16);
  while (K > 16 && ws_need(K) > cap) K = (K > 32 ? (K - 1) / 16 * 16 : 16);
  if (ws_need(K) > cap)
    return fail(CSP_ENOMEM, "quasi-eigenstate workspace %.2f GB exceeds the cap %.2f GB",
                ws_need(K) / 1e9, cap / 1e9);
  const int S = K + kt;
  const int RG = ring_parts(S);    // ring parts (slot of position k: ring_slot)
  CHECK(ws_reserve(c, ws_need(K)));
  Carver cv(c->ws);
  std::vector<void*> carry(sp.size()), acc(sp.size()), slots(sp.size());
  for (size_t i = 0; i < sp.size(); ++i) {
    const Group& g = groups[i / 2];
    slots[i] = cv.take((size_t)S * g.stride() * csz);
    carry[i] = cv.take(g.M * csz);
    acc[i] = cv.take((size_t)nE * g.M * csz);
  }
  void* d_bop = nullptr;
  double* d_coef = nullptr;
  if (fp64) d_coef = (double*)cv.take(sizeof(double2) * (size_t)K * B64);
  else d_bop = cv.take((size_t)64 * 64 * ceil_div(K, 16));
  ChebInst* d_inst = (ChebInst*)cv.take(sizeof(ChebInst) * sp.size());
  QeInst* d_qi = (QeInst*)cv.take(sizeof(QeInst) * sp.size());

  int64_t Msum = 0;
  for (auto& g : groups) Msum += 2 * g.M;
  std::vector<QeInst> qi;
  int wg0 = 0;
  for (size_t i = 0; i < sp.size(); ++i) {
    const Group& g = groups[i / 2];
    // both carried states start from psi0
    HIPCALL(launch_gather_cols(N, R, g.col0, g.Rg, fp64 ? CSP_C128 : CSP_C64, dev_psi0, fp64,
                               carry[i], s));
    ChebInst& I = sp[i];
    I.base = slots[i];
    I.slot_stride = g.stride();
    I.src = carry[i];
    const int64_t units = fp64 ? ceil_div(N, kContractThreads) : ceil_div(ceil_div(N, 32), 4);
    const double share = (double)c->n_cu * 4.0 * (double)g.M / (double)Msum / g.Rg;
    const int wpc = (int)std::max<int64_t>(1, std::min<int64_t>(std::llround(share), units));
    QeInst q{};
    q.slots = slots[i];
    q.slot_stride = g.stride();
    q.N = N;
    q.Rg = g.Rg;
    q.wpc = wpc;
    q.out = acc[i];
    q.wg0 = wg0;
    q.n_wg = g.Rg * wpc;
    q.carry = carry[i];
    q.conj = (int)(i & 1);                     // odd instances propagate backward
    wg0 += q.n_wg;
    qi.push_back(q);
  }
  CHECK(attach_ell_shadows(c, sp, fp64));
  HIPCALL(hipMemcpyAsync(d_inst, sp.data(), sizeof(ChebInst) * sp.size(), hipMemcpyHostToDevice, s));
  HIPCALL(hipMemcpyAsync(d_qi, qi.data(), sizeof(QeInst) * qi.size(), hipMemcpyHostToDevice, s));

  Profiler prof{c, P.profile != 0};
  int64_t n_spmm = 0, n_con = 0, amxsy = 0, axpy = 0;
  const ChebStep st0 = step_args(sp_plan);
  const int n_blk = (int)ceil_div(Nt, b);
  for (int k = 0; k < n_blk; ++k) {
    const int bk = std::min(b, Nt - k * b);
    const int Nk = ntr[bk - 1];
    HIPCALL(launch_qes_coeffs(d_a, lda, d_ntr, bk, (int64_t)k * b, nE, d_E, L->H0, tau,
                              k == 0 ? 1 : 0, Nk, d_C, s));
    amxsy += 2 * Nk;
    axpy += 2 * (int64_t)(Nk + 1) * rows;
    int produced = 0, n_lo = 0;
    while (n_lo <= Nk) {
      if (produced < Nk) {
        ChebStep st = st0;
        st.nlev = std::min(kt, Nk - produced);
        if (produced == 0) {
          st.first = 1;
          st.slot_cur = -1;
          st.copy_slot = 0;
        } else {
          st.slot_cur = ring_slot(produced % S, S, RG);
          st.slot_prev = ring_slot((produced - 1) % S, S, RG);
        }
        for (int l = 1; l <= st.nlev; ++l)
          st.slot_out[l - 1] = ring_slot((produced + l) % S, S, RG);
        size_t ev = 0;
        CHECK(prof.begin(0, &ev));
        set_shadow(st, produced);
        HIPCALL(launch_cheb(fp64, sp_plan.vec, kt, false, false, d_inst, sp_plan.runs, st, s));
        CHECK(prof.end(ev));
        ++n_spmm;
        produced += st.nlev;
      }
      while (n_lo <= Nk && (n_lo + K - 1 <= produced || produced == Nk)) {
        const int n_cnt = std::min(K, Nk + 1 - n_lo);
        if (fp64) HIPCALL(launch_pack_qes64(d_C, Nk + 1, rows, B64, n_lo, n_cnt, d_coef, s));
        else HIPCALL(launch_pack_qes(d_C, Nk + 1, rows, n_lo, n_cnt, d_bop, s));
        QeArgs qa{};
        qa.n_inst = (int)sp.size();
        qa.n_lo = n_lo;
        qa.n_cnt = n_cnt;
        qa.S = S;
        qa.G = RG;
        qa.first_chunk = (k == 0 && n_lo == 0) ? 1 : 0;
        qa.nE = nE;
        qa.total_wg = wg0;
        qa.cplx = 1;
        qa.carry_first = n_lo == 0 ? 1 : 0;
        qa.bop = d_bop;
        qa.coef = d_coef;
        size_t evc = 0;
        CHECK(prof.begin(1, &evc));
        HIPCALL(launch_contract_qe(fp64, d_qi, qa, s));
        CHECK(prof.end(evc));
        ++n_con;
        n_lo += n_cnt;
      }
    }
  }
  // Psi(E) = forward + backward accumulators, to the caller's layout
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    HIPCALL(launch_add_complex(fp64, (int64_t)nE * groups[gi].M, acc[2 * gi], acc[2 * gi + 1], s));
    HIPCALL(launch_qe_scatter(N, groups[gi].Rg, nE, R, groups[gi].col0, fp64, acc[2 * gi],
                              fp64 ? CSP_C128 : CSP_C64, dev_qe, s));
  }
  HIPCALL(hipStreamSynchronize(s));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    double ms_s = 0, ms_c = 0;
    CHECK(prof.collect(&ms_s, &ms_c));
    rep->block_b = b;
    rep->chunk_K = K;
    rep->n_blocks = n_blk;
    rep->n_groups = (int)groups.size();
    rep->amxsy = amxsy;
    rep->axpy = axpy;
    rep->dot = 0;
    rep->spmm_launches = n_spmm;
    rep->contract_launches = n_con;
    rep->ms_total = now_ms() - t_start;
    rep->ms_spmm = ms_s;
    rep->ms_contract = ms_c;
    rep->spmm_bytes = (double)N * R * csz * ((double)amxsy + 4.0 * n_spmm) +
                      (double)sp.size() * static_bytes(L, fp64) * n_spmm;
    rep->contract_bytes = (double)N * R * csz * ((double)amxsy + 2.0 * n_blk +
                                                 2.0 * 2.0 * rows * n_con);
    rep->contract_flops = 4.0 * 2.0 * (double)N * R * (double)axpy / 2.0 * (fp64 ? 1.0 : 3.0);
    rep->workspace_bytes = c->ws_size;
    rep->n_passes = 1;
    rep->spmm_steps = kt;
  }
  return CSP_OK;
}
}  // namespace

extern "C" csp_status csp_quasi_eigenstates(csp_context* c, const csp_lattice* L,
                                            const void* dev_psi0, int32_t R,
                                            const csp_params* params_in, int32_t n_E,
                                            const double* energies, void* dev_qe,
                                            csp_report* rep) {
  const double t_start = now_ms();
  if (!c || !L || !dev_psi0 || !params_in || !energies || !dev_qe)
    return fail(CSP_EINVAL, "NULL argument");
  csp_params P;
  fill_defaults(params_in, &P);
  if (P.mode != CSP_FP32_CONC && P.mode != CSP_FP64_CONC)
    return fail(CSP_EINVAL, "quasi-eigenstates need CSP_FP32_CONC or CSP_FP64_CONC");
  const bool fp64 = P.mode == CSP_FP64_CONC;
  const int nE = n_E;
  if (nE < 1 || nE > 128) return fail(CSP_EINVAL, "need 1 <= n_E <= 128");
  if (R < 1) return fail(CSP_EINVAL, "R must be >= 1");
  if (P.Nt < 1 || P.Nt > (1 << 20)) return fail(CSP_EINVAL, "need 1 <= Nt <= 2^20");
  if (L->ctx->device != c->device) return fail(CSP_EINVAL, "lattice is on another device");
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(energies[e])) return fail(CSP_EINVAL, "energy %d is not finite", e);
  if (P.block_b < 0) return fail(CSP_EINVAL, "block_b must be >= 0");
  if (P.block_b >= 1 && nE > (fp64 ? 15 : 31))
    return fail(CSP_EINVAL, "the state-based form takes 1 <= n_E <= %d", fp64 ? 15 : 31);
  DeviceGuard dg(c->device);
  if (P.block_b >= 1) return qe_state_based(c, L, dev_psi0, R, P, nE, energies, dev_qe, rep, t_start);
  hipStream_t s = c->stream;
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  const int Nt = (int)P.Nt;
  const int64_t N = L->g.N;

  // Bessel table for x = j tau~, j = 1..Nt, and the coefficients C_n(E).
  const int nmax_tab = (int)trunc_nmax((double)Nt * P.tau_tilde);
  const int lda = nmax_tab + 1;
  struct Free {
    std::vector<void*> p;
    ~Free() { for (void* q : p) (void)hipFree(q); }
  } tmp;
  auto alloc = [&](void** ptr, size_t bytes) -> csp_status {
    HIPCALL(hipMalloc(ptr, bytes));
    tmp.p.push_back(*ptr);
    return CSP_OK;
  };
  double *d_a = nullptr, *d_E = nullptr, *d_cs = nullptr, *d_C = nullptr;
  int32_t *d_ntr = nullptr, *d_ntrq = nullptr;
  CHECK(alloc((void**)&d_a, sizeof(double) * (size_t)Nt * lda));
  CHECK(alloc((void**)&d_ntr, sizeof(int32_t) * Nt));
  HIPCALL(launch_bessel(P.tau_tilde, Nt, nmax_tab, P.eta, true, d_a, d_ntr, s));
  int32_t Nmax = 0;
  HIPCALL(hipMemcpyAsync(&Nmax, d_ntr + (Nt - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCALL(hipStreamSynchronize(s));
  if (Nmax < 1) return fail(CSP_ENUMERIC, "no truncation order for x = %g", Nt * P.tau_tilde);
  const int ldc = Nmax + 1;
  CHECK(alloc((void**)&d_E, sizeof(double) * nE));
  CHECK(alloc((void**)&d_cs, sizeof(double2) * (size_t)nE * Nt));
  CHECK(alloc((void**)&d_C, sizeof(double) * (size_t)nE * ldc));
  CHECK(alloc((void**)&d_ntrq, sizeof(int32_t) * 32));
  HIPCALL(hipMemcpyAsync(d_E, energies, sizeof(double) * nE, hipMemcpyHostToDevice, s));
  {
    std::vector<int32_t> nq(32, Nmax);
    HIPCALL(hipMemcpyAsync(d_ntrq, nq.data(), sizeof(int32_t) * 32, hipMemcpyHostToDevice, s));
    HIPCALL(launch_qe_coeffs(d_a, lda, d_ntr, Nt, nE, d_E, L->H0, P.tau_tilde / L->halfwidth,
                             Nmax, d_cs, d_C, s));
    HIPCALL(hipStreamSynchronize(s));   // nq leaves scope
  }

  // Column groups and the recursion's launch shape.
  std::vector<Group> groups;
  {
    int col = 0;
    for (int Rg : split_columns(R, L->g.kind == CSP_SPARSE)) {
      Group g;
      g.inst = 0;
      g.col0 = col;
      g.Rg = Rg;
      g.M = N * Rg;
      groups.push_back(g);
      col += Rg;
    }
  }
  std::vector<ChebInst> sp;
  for (auto& g : groups) sp.push_back(make_inst(L, g.Rg, fp64));
  const ChebPlan sp_plan = plan_cheb(sp, fp64, false, c->n_cu, 2, fp64 ? 4 : 8, 0);
  const int kt = sp_plan.kt;

  // Orders per contraction chunk: all of them when they fit, else a multiple
  // of 16 (LDS holds the chunk's coefficients of one energy tile; the ring
  // K + kt slots).  Energy tiles of 32 (FP32) or B64 (FP64) energies.
  int B64 = 1;
  while (B64 < nE && B64 < 16) B64 *= 2;
  const int n_et = (int)ceil_div(nE, fp64 ? B64 : 32);
  const int kcap = fp64 ? (int)((60 * 1024) / (sizeof(double2) * B64)) / 16 * 16 : 496;
  size_t cap = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap));
  auto ws_need = [&](int K_) {
    size_t by = 0;
    for (auto& g : groups)
      by += align256((size_t)(K_ + kt) * g.stride() * csz) + align256(g.M * csz) +
            align256((size_t)nE * g.M * csz);
    by += fp64 ? align256(sizeof(double2) * (size_t)K_ * B64 * n_et)
               : align256(bop_bytes(1, K_) * n_et) + align256(sizeof(float) * 16 * ceil_div(K_, 16));
    by += align256(sizeof(ChebInst) * groups.size()) + align256(sizeof(QeInst) * groups.size());
    return by;
  };
  int K = std::min(Nmax + 1, kcap);
  if (K < Nmax + 1) K = std::max(16, K / 16 * 16);
  while (K > 16 && ws_need(K) > cap) K = (K > 32 ? (K - 1) / 16 * 16 : 16);
  if (ws_need(K) > cap)
    return fail(CSP_ENOMEM, "quasi-eigenstate workspace %.2f GB exceeds the cap %.2f GB",
                ws_need(K) / 1e9, cap / 1e9);
  const int S = K + kt;
  const int RG = ring_parts(S);    // ring parts (slot of position k: ring_slot)
  CHECK(ws_reserve(c, ws_need(K)));
  Carver cv(c->ws);
  std::vector<void*> outs(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    g.slots = cv.take((size_t)S * g.stride() * csz);
    g.psi0g = cv.take(g.M * csz);
    outs[gi] = cv.take((size_t)nE * g.M * csz);
  }
  void* d_bop = nullptr;
  float* d_ccd = nullptr;
  double* d_coef = nullptr;
  if (fp64) {
    d_coef = (double*)cv.take(sizeof(double2) * (size_t)K * B64 * n_et);
  } else {
    d_bop = cv.take(bop_bytes(1, K) * n_et);
    d_ccd = (float*)cv.take(sizeof(float) * 16 * ceil_div(K, 16));
  }
  ChebInst* d_inst = (ChebInst*)cv.take(sizeof(ChebInst) * groups.size());
  QeInst* d_qi = (QeInst*)cv.take(sizeof(QeInst) * groups.size());

  // Instance tables (workgroups per column as in the state assembly).
  int64_t Msum = 0;
  for (auto& g : groups) Msum += g.M;
  std::vector<QeInst> qi;
  int wg0 = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    HIPCALL(launch_gather_cols(N, R, g.col0, g.Rg, fp64 ? CSP_C128 : CSP_C64, dev_psi0, fp64,
                               g.psi0g, s));
    ChebInst& I = sp[gi];
    I.base = g.slots;
    I.slot_stride = g.stride();
    I.src = g.psi0g;
    const int64_t units = fp64 ? ceil_div(N, kContractThreads) : ceil_div(ceil_div(N, 32), 4);
    const double share = (double)c->n_cu * 4.0 * (double)g.M / (double)Msum / g.Rg;
    const int wpc = (int)std::max<int64_t>(1, std::min<int64_t>(std::llround(share), units));
    QeInst q{};
    q.slots = g.slots;
    q.slot_stride = g.stride();
    q.N = N;
    q.Rg = g.Rg;
    q.wpc = wpc;
    q.out = outs[gi];
    q.wg0 = wg0;
    q.n_wg = g.Rg * wpc;
    wg0 += q.n_wg;
    qi.push_back(q);
  }
  CHECK(attach_ell_shadows(c, sp, fp64));
  HIPCALL(hipMemcpyAsync(d_inst, sp.data(), sizeof(ChebInst) * sp.size(), hipMemcpyHostToDevice, s));
  HIPCALL(hipMemcpyAsync(d_qi, qi.data(), sizeof(QeInst) * qi.size(), hipMemcpyHostToDevice, s));

  // Recursion launches with a contraction after every completed chunk.
  Profiler prof{c, P.profile != 0};
  int64_t n_spmm = 0, n_con = 0;
  const ChebStep st0 = step_args(sp_plan);
  int produced = 0, n_lo = 0;
  while (produced < Nmax) {
    ChebStep st = st0;
    st.nlev = std::min(kt, Nmax - produced);
    if (produced == 0) {
      st.first = 1;
      st.slot_cur = -1;
      st.copy_slot = 0;
    } else {
      st.slot_cur = ring_slot(produced % S, S, RG);
      st.slot_prev = ring_slot((produced - 1) % S, S, RG);
    }
    for (int l = 1; l <= st.nlev; ++l)
      st.slot_out[l - 1] = ring_slot((produced + l) % S, S, RG);
    size_t ev = 0;
    CHECK(prof.begin(0, &ev));
    set_shadow(st, produced);
    HIPCALL(launch_cheb(fp64, sp_plan.vec, kt, false, false, d_inst, sp_plan.runs, st, s));
    CHECK(prof.end(ev));
    ++n_spmm;
    produced += st.nlev;
    while (n_lo <= Nmax && (n_lo + K - 1 <= produced || produced == Nmax)) {
      const int n_cnt = std::min(K, Nmax + 1 - n_lo);
      for (int t = 0; t < n_et; ++t) {
        const int w = fp64 ? B64 : 32, e0 = t * w, ne = std::min(w, nE - e0);
        if (fp64)
          HIPCALL(launch_pack_qe64(d_C + (size_t)e0 * ldc, ldc, ne, B64, n_lo, n_cnt,
                                   d_coef + 2 * (size_t)t * K * B64, s));
        else
          HIPCALL(launch_pack_bop(d_C + (size_t)e0 * ldc, ldc, d_ntrq, ne, 1, n_lo, n_cnt,
                                  static_cast<char*>(d_bop) + (size_t)t * bop_bytes(1, K), d_ccd,
                                  s));
      }
      QeArgs qa{};
      qa.e_tile_stride = fp64 ? K * B64 : (int)(bop_bytes(1, K) / (2 * 16));
      qa.n_inst = (int)groups.size();
      qa.n_lo = n_lo;
      qa.n_cnt = n_cnt;
      qa.S = S;
      qa.G = RG;
      qa.first_chunk = n_lo == 0 ? 1 : 0;
      qa.nE = nE;
      qa.total_wg = wg0;
      qa.bop = d_bop;
      qa.coef = d_coef;
      size_t evc = 0;
      CHECK(prof.begin(1, &evc));
      HIPCALL(launch_contract_qe(fp64, d_qi, qa, s));
      CHECK(prof.end(evc));
      ++n_con;
      n_lo += n_cnt;
    }
  }
  for (size_t gi = 0; gi < groups.size(); ++gi)
    HIPCALL(launch_qe_scatter(N, groups[gi].Rg, nE, R, groups[gi].col0, fp64, outs[gi],
                              fp64 ? CSP_C128 : CSP_C64, dev_qe, s));
  HIPCALL(hipStreamSynchronize(s));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    double ms_s = 0, ms_c = 0;
    CHECK(prof.collect(&ms_s, &ms_c));
    rep->block_b = Nt;
    rep->chunk_K = K;
    rep->n_blocks = 1;
    rep->n_groups = (int)groups.size();
    rep->amxsy = Nmax;
    rep->axpy = (int64_t)(Nmax + 1) * nE;
    rep->dot = 0;
    rep->spmm_launches = n_spmm;
    rep->contract_launches = n_con;
    rep->ms_total = now_ms() - t_start;
    rep->ms_spmm = ms_s;
    rep->ms_contract = ms_c;
    rep->spmm_bytes = (double)N * R * csz * ((double)Nmax + 2.0 * n_spmm) +
                      (double)groups.size() * static_bytes(L, fp64) * n_spmm;
    rep->contract_bytes = (double)N * R * csz * ((double)Nmax + 1.0 + 2.0 * nE * n_con);
    rep->contract_flops = 2.0 * 2.0 * (double)N * R * (Nmax + 1) * nE * (fp64 ? 1.0 : 3.0);
    rep->workspace_bytes = c->ws_size;
    rep->n_passes = 1;
    rep->spmm_steps = kt;
  }
  return CSP_OK;
}

// ------------------------------------------------------------------ conductivity
namespace {
// J_alpha applied to nvec vectors [nvec][N] of the lattice
hipError_t apply_current(const csp_lattice* L, bool fp64, int alpha, const void* in, void* out,
                         int64_t nvec, hipStream_t s) {
  if (L->g.kind == CSP_SPARSE)
    return launch_current_ell(fp64, L->g.N, L->ell_D, L->ell_col, L->ell_v64, L->pos,
                              L->box[alpha], alpha, in, out, nvec, s);
  return launch_current_stencil(fp64, L->g, L->desc.t, alpha, in, out, nvec, s);
}
}  // namespace

extern "C" csp_status csp_ec_correlation(csp_context* c, const csp_lattice* L, int32_t alpha,
                                         const void* dev_psi0, int32_t R, const void* dev_qe,
                                         const csp_params* params_in, int32_t n_E,
                                         double* dev_corr, csp_report* rep) {
  const double t_start = now_ms();
  if (!c || !L || !dev_psi0 || !dev_qe || !params_in || !dev_corr)
    return fail(CSP_EINVAL, "NULL argument");
  csp_params P;
  fill_defaults(params_in, &P);
  if (P.mode != CSP_FP32_CONC && P.mode != CSP_FP64_CONC)
    return fail(CSP_EINVAL, "the conductivity needs CSP_FP32_CONC or CSP_FP64_CONC");
  const bool fp64 = P.mode == CSP_FP64_CONC;
  const int nE = n_E;
  if (nE < 1 || nE > 128) return fail(CSP_EINVAL, "need 1 <= n_E <= 128");
  const int e_tile = fp64 ? ec64_tile(nE) : 32;
  const int ldp = (int)ceil_div(nE, e_tile) * e_tile;
  if (alpha != 0 && alpha != 1) return fail(CSP_EINVAL, "alpha must be 0 (x) or 1 (y)");
  if (R < 1) return fail(CSP_EINVAL, "R must be >= 1");
  if (P.Nt < 1 || P.Nt > (1 << 20)) return fail(CSP_EINVAL, "need 1 <= Nt <= 2^20");
  if (L->ctx->device != c->device) return fail(CSP_EINVAL, "lattice is on another device");
  if (L->g.kind == CSP_SPARSE && !L->pos)
    return fail(CSP_EINVAL, "explicit matrix without coordinates (csp_lattice_set_positions)");
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  const int Nt = (int)P.Nt;
  const int64_t N = L->g.N;
  const int64_t ldmu = (int64_t)R * nE;
  if ((int64_t)Nt * ldmu > INT32_MAX)
    return fail(CSP_EUNSUPPORTED, "Nt x R x n_E = %lld exceeds 2^31 - 1 (split the columns)",
                (long long)Nt * ldmu);
  const double tau = P.tau_tilde / L->halfwidth;

  struct Free {
    std::vector<void*> p;
    ~Free() { for (void* q : p) (void)hipFree(q); }
  } tmp;
  auto alloc = [&](void** ptr, size_t bytes) -> csp_status {
    HIPCALL(hipMalloc(ptr, bytes));
    tmp.p.push_back(*ptr);
    return CSP_OK;
  };
  // Bessel table for x = j tau~, j = 1..Nt
  const int nmax_tab = (int)trunc_nmax((double)Nt * P.tau_tilde);
  const int lda = nmax_tab + 1;
  double* d_a = nullptr;
  int32_t* d_ntr = nullptr;
  CHECK(alloc((void**)&d_a, sizeof(double) * (size_t)Nt * lda));
  CHECK(alloc((void**)&d_ntr, sizeof(int32_t) * Nt));
  HIPCALL(launch_bessel(P.tau_tilde, Nt, nmax_tab, P.eta, true, d_a, d_ntr, s));
  int32_t Nmax = 0;
  HIPCALL(hipMemcpyAsync(&Nmax, d_ntr + (Nt - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCALL(hipStreamSynchronize(s));
  if (Nmax < 1) return fail(CSP_ENUMERIC, "no truncation order for x = %g", Nt * P.tau_tilde);
  double *d_mu = nullptr, *d_G = nullptr, *d_nrm = nullptr;
  CHECK(alloc((void**)&d_mu, sizeof(double2) * (size_t)(Nmax + 1) * ldmu));
  CHECK(alloc((void**)&d_G, sizeof(double2) * (size_t)(Nt + 1) * ldmu));
  CHECK(alloc((void**)&d_nrm, sizeof(double) * ldmu));

  // Column groups, the recursion's launch shape, slices of the moment
  // contraction (about four workgroups per CU over all columns).
  std::vector<Group> groups;
  {
    int col = 0;
    for (int Rg : split_columns(R, L->g.kind == CSP_SPARSE)) {
      Group g;
      g.inst = 0;
      g.col0 = col;
      g.Rg = Rg;
      g.M = N * Rg;
      groups.push_back(g);
      col += Rg;
    }
  }
  std::vector<ChebInst> sp;
  for (auto& g : groups) sp.push_back(make_inst(L, g.Rg, fp64));
  const ChebPlan sp_plan = plan_cheb(sp, fp64, false, c->n_cu, 2, fp64 ? 4 : 8, 0);
  const int kt = sp_plan.kt;
  const int64_t target_slices = std::max<int64_t>(1, (int64_t)c->n_cu * 4 / R);
  const int64_t slice_len = std::max<int64_t>(512, (ceil_div(N, target_slices) + 7) / 8 * 8);
  const int n_slices = (int)ceil_div(N, slice_len);
  const size_t psz = fp64 ? sizeof(double2) : sizeof(float2);   // partial element

  int K = std::min(Nmax + 1, 128);
  size_t cap = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap));
  auto ws_need = [&](int K_) {
    size_t by = 0;
    for (auto& g : groups)
      by += align256((size_t)(K_ + kt) * g.stride() * csz) + 2 * align256(g.M * csz) +
            2 * align256((size_t)nE * g.M * csz) +
            align256((size_t)g.Rg * n_slices * K_ * ldp * psz);
    by += align256(sizeof(ChebInst) * groups.size()) + align256(sizeof(EcInst) * groups.size()) +
          align256(sizeof(MomCorrInst));
    return by;
  };
  while (K > 16 && ws_need(K) > cap) K = std::max(16, K - 16);
  if (ws_need(K) > cap)
    return fail(CSP_ENOMEM, "conductivity workspace %.2f GB exceeds the cap %.2f GB",
                ws_need(K) / 1e9, cap / 1e9);
  const int S = K + kt;
  const int RG = ring_parts(S);    // ring parts (slot of position k: ring_slot)
  CHECK(ws_reserve(c, ws_need(K)));
  Carver cv(c->ws);
  std::vector<void*> jpsi(groups.size()), qeg(groups.size()), bra(groups.size()),
      part(groups.size());
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    g.slots = cv.take((size_t)S * g.stride() * csz);
    g.psi0g = cv.take(g.M * csz);
    jpsi[gi] = cv.take(g.M * csz);
    qeg[gi] = cv.take((size_t)nE * g.M * csz);
    bra[gi] = cv.take((size_t)nE * g.M * csz);
    part[gi] = cv.take((size_t)g.Rg * n_slices * K * ldp * psz);
  }
  ChebInst* d_inst = (ChebInst*)cv.take(sizeof(ChebInst) * groups.size());
  EcInst* d_ei = (EcInst*)cv.take(sizeof(EcInst) * groups.size());
  MomCorrInst* d_mc = (MomCorrInst*)cv.take(sizeof(MomCorrInst));

  // J psi (recursion start), J Psi(E) (bras), |<psi|Psi(E)>|
  const int dt = fp64 ? CSP_C128 : CSP_C64;
  std::vector<EcInst> ei;
  int wg0 = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    Group& g = groups[gi];
    HIPCALL(launch_gather_cols(N, R, g.col0, g.Rg, dt, dev_psi0, fp64, g.psi0g, s));
    HIPCALL(apply_current(L, fp64, alpha, g.psi0g, jpsi[gi], g.Rg, s));
    for (int e = 0; e < nE; ++e)
      HIPCALL(launch_gather_cols(N, R, g.col0, g.Rg, dt,
                                 static_cast<const char*>(dev_qe) + (size_t)e * N * R * csz, fp64,
                                 static_cast<char*>(qeg[gi]) + (size_t)e * g.M * csz, s));
    HIPCALL(launch_ec_norm(fp64, N, g.Rg, nE, g.psi0g, qeg[gi], d_nrm, g.col0 * nE, s));
    HIPCALL(apply_current(L, fp64, alpha, qeg[gi], bra[gi], (int64_t)nE * g.Rg, s));
    ChebInst& I = sp[gi];
    I.base = g.slots;
    I.slot_stride = g.stride();
    I.src = jpsi[gi];
    EcInst q{};
    q.slots = g.slots;
    q.slot_stride = g.stride();
    q.bra = bra[gi];
    q.partial = part[gi];
    q.N = N;
    q.slice_len = slice_len;
    q.Rg = g.Rg;
    q.n_slices = n_slices;
    q.wg0 = wg0;
    q.n_wg = g.Rg * n_slices;
    q.q0 = g.col0 * nE;
    wg0 += q.n_wg;
    ei.push_back(q);
  }
  CHECK(attach_ell_shadows(c, sp, fp64));
  HIPCALL(hipMemcpyAsync(d_inst, sp.data(), sizeof(ChebInst) * sp.size(), hipMemcpyHostToDevice, s));
  HIPCALL(hipMemcpyAsync(d_ei, ei.data(), sizeof(EcInst) * ei.size(), hipMemcpyHostToDevice, s));
  int rg_max = 1;
  for (auto& g : groups) rg_max = std::max(rg_max, g.Rg);

  // Recursion launches with a moment contraction after every completed chunk.
  Profiler prof{c, P.profile != 0};
  int64_t n_spmm = 0, n_con = 0;
  const ChebStep st0 = step_args(sp_plan);
  int produced = 0, n_lo = 0;
  while (n_lo <= Nmax) {
    if (produced < Nmax) {
      ChebStep st = st0;
      st.nlev = std::min(kt, Nmax - produced);
      if (produced == 0) {
        st.first = 1;
        st.slot_cur = -1;
        st.copy_slot = 0;
      } else {
        st.slot_cur = ring_slot(produced % S, S, RG);
        st.slot_prev = ring_slot((produced - 1) % S, S, RG);
      }
      for (int l = 1; l <= st.nlev; ++l)
        st.slot_out[l - 1] = ring_slot((produced + l) % S, S, RG);
      size_t ev = 0;
      CHECK(prof.begin(0, &ev));
      set_shadow(st, produced);
      HIPCALL(launch_cheb(fp64, sp_plan.vec, kt, false, false, d_inst, sp_plan.runs, st, s));
      CHECK(prof.end(ev));
      ++n_spmm;
      produced += st.nlev;
    }
    while (n_lo <= Nmax && (n_lo + K - 1 <= produced || produced == Nmax)) {
      EcArgs ea{};
      ea.n_inst = (int)groups.size();
      ea.n_lo = n_lo;
      ea.n_cnt = std::min(K, Nmax + 1 - n_lo);
      ea.S = S;
      ea.G = RG;
      ea.nE = nE;
      ea.K = K;
      ea.total_wg = wg0;
      ea.ldp = ldp;
      ea.mu = d_mu;
      ea.ldmu = ldmu;
      size_t evc = 0;
      CHECK(prof.begin(1, &evc));
      HIPCALL(launch_ec_moments(fp64, d_ei, (int)groups.size(), ea, s));
      CHECK(prof.end(evc));
      HIPCALL(launch_ec_mu_finish(fp64, d_ei, (int)groups.size(), rg_max, ea, s));
      ++n_con;
      n_lo += ea.n_cnt;
    }
  }
  // G_j = sum_n c_n(j tau~) mu_n (rows 1..Nt), then C = conj(G) e^{iH0 t} / |<psi|Psi>|
  MomCorrInst mc{};
  mc.mu = d_mu;
  mc.corr = d_G;
  mc.ldc = ldmu;
  mc.Rg = (int32_t)ldmu;
  mc.col0 = 0;
  HIPCALL(hipMemcpyAsync(d_mc, &mc, sizeof(mc), hipMemcpyHostToDevice, s));
  HIPCALL(launch_mom_corr_only(d_mc, 1, d_a, lda, d_ntr, Nt, 0, (int)ldmu, s));
  HIPCALL(launch_ec_finish(Nt, R, nE, d_mu, d_G, d_nrm, L->H0, tau, dev_corr, s));
  HIPCALL(hipStreamSynchronize(s));
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    double ms_s = 0, ms_c = 0;
    CHECK(prof.collect(&ms_s, &ms_c));
    rep->block_b = Nt;
    rep->chunk_K = K;
    rep->n_blocks = 1;
    rep->n_groups = (int)groups.size();
    rep->amxsy = Nmax;
    rep->axpy = 0;
    rep->dot = (int64_t)(Nmax + 1) * nE;
    rep->spmm_launches = n_spmm;
    rep->contract_launches = n_con;
    rep->ms_total = now_ms() - t_start;
    rep->ms_spmm = ms_s;
    rep->ms_contract = ms_c;
    rep->spmm_bytes = (double)N * R * csz * ((double)Nmax + 2.0 * n_spmm) +
                      (double)groups.size() * static_bytes(L, fp64) * n_spmm;
    rep->contract_bytes = (double)N * R * csz * ((double)Nmax + 1.0 + (double)nE * n_con);
    rep->contract_flops = 8.0 * (double)N * R * (Nmax + 1) * nE * (fp64 ? 1.0 : 3.0);
    rep->workspace_bytes = c->ws_size;
    rep->n_passes = 1;
    rep->spmm_steps = kt;
  }
  return CSP_OK;
}

extern "C" csp_status csp_ec_sigma(csp_context* c, const double* dev_corr, int64_t Nt, int32_t R,
                                   int32_t n_E, const double* energies, double halfwidth,
                                   double tau_tilde, const double* dos_over_area,
                                   double* dev_sigma) {
  if (!c || !dev_corr || !energies || !dev_sigma) return fail(CSP_EINVAL, "NULL argument");
  if (Nt < 0 || R < 1 || n_E < 1 || !(halfwidth > 0) || !(tau_tilde > 0))
    return fail(CSP_EINVAL, "need Nt >= 0, R >= 1, n_E >= 1, |H| > 0, tau~ > 0");
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;
  std::vector<double> h(2 * (size_t)n_E);
  for (int e = 0; e < n_E; ++e) {
    h[e] = energies[e];
    h[n_E + e] = dos_over_area ? dos_over_area[e] : 1.0;
    if (!std::isfinite(h[e]) || !std::isfinite(h[n_E + e]))
      return fail(CSP_EINVAL, "energy or D(E)/A %d is not finite", e);
  }
  double* d_h = nullptr;
  HIPCALL(hipMalloc(&d_h, sizeof(double) * h.size()));
  hipError_t e = hipMemcpyAsync(d_h, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_ec_sigma(Nt, R, n_E, dev_corr, d_h, d_h + n_E, tau_tilde / halfwidth, dev_sigma, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_h);
  if (e != hipSuccess) return fail(CSP_EHIP, "conductivity integral: %s", hipGetErrorString(e));
  return CSP_OK;
}

// ------------------------------------------------------------------ DOS
extern "C" csp_status csp_dos(csp_context* c, const double* dev_corr, int64_t Nt, int32_t R,
                              double halfwidth, double center, double tau_tilde, int32_t window,
                              double* dev_E, double* dev_D, double* dev_Dmean) {
  if (!c || !dev_corr || !dev_E || !dev_D) return fail(CSP_EINVAL, "NULL argument");
  if (Nt < 1 || R < 1 || !(halfwidth > 0)) return fail(CSP_EINVAL, "need Nt >= 1, R >= 1, |H| > 0");
  if (!std::isfinite(center)) return fail(CSP_EINVAL, "center is not finite");
  if (window != CSP_WINDOW_HANN && window != CSP_WINDOW_NONE) return fail(CSP_EINVAL, "bad window");
  if (!(tau_tilde > 0)) tau_tilde = M_PI;
  DeviceGuard dg(c->device);
  double* tw = nullptr;
  HIPCALL(hipMalloc(&tw, sizeof(double2) * 2 * Nt));
  hipError_t e = launch_dos(dev_corr, Nt, R, halfwidth, center, tau_tilde, window, dev_E, dev_D,
                            dev_Dmean, tw, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(tw);
  if (e != hipSuccess) return fail(CSP_EHIP, "dos: %s", hipGetErrorString(e));
  return CSP_OK;
}

extern "C" csp_status csp_dos_noalloc(csp_context* c, const double* dev_corr, int64_t Nt,
                                      int32_t R, double halfwidth, double center,
                                      double tau_tilde, int32_t window, double* dev_E,
                                      double* dev_D, double* dev_Dmean) {
  if (!c || !dev_corr || !dev_E || !dev_D) return fail(CSP_EINVAL, "NULL argument");
  if (Nt < 1 || R < 1 || !(halfwidth > 0)) return fail(CSP_EINVAL, "need Nt >= 1, R >= 1, |H| > 0");
  if (Nt > CSP_DOS_NOALLOC_MAX_NT)
    return fail(CSP_EINVAL, "Nt = %lld exceeds the %d time steps of the static twiddle scratch",
                (long long)Nt, CSP_DOS_NOALLOC_MAX_NT);
  if (!std::isfinite(center)) return fail(CSP_EINVAL, "center is not finite");
  if (window != CSP_WINDOW_HANN && window != CSP_WINDOW_NONE) return fail(CSP_EINVAL, "bad window");
  if (!(tau_tilde > 0)) tau_tilde = M_PI;
  if (!c->dos_scratch) return fail(CSP_EHIP, "no scratch address for device %d", c->device);
  DeviceGuard dg(c->device);
  const hipError_t e = launch_dos(dev_corr, Nt, R, halfwidth, center, tau_tilde, window, dev_E,
                                  dev_D, dev_Dmean, c->dos_scratch, c->stream);
  if (e != hipSuccess) return fail(CSP_EHIP, "dos_noalloc: %s", hipGetErrorString(e));
  return CSP_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {

// Median of three launch times (ms) of `launch`, after one untimed launch.
template <typename F>
csp_status time_launch(csp_context* c, F launch, double* ms_out) {
  hipStream_t s = c->stream;
  CHECK(launch());
  double v[3];
  for (int i = 0; i < 3; ++i) {
    hipEvent_t e0, e1;
    CHECK(hip_event(c, 2 * i, &e0));
    CHECK(hip_event(c, 2 * i + 1, &e1));
    HIPCALL(hipEventRecord(e0, s));
    CHECK(launch());
    HIPCALL(hipEventRecord(e1, s));
    HIPCALL(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCALL(hipEventElapsedTime(&ms, e0, e1));
    v[i] = ms;
  }
  std::sort(v, v + 3);
  *ms_out = v[1];
  return CSP_OK;
}

}  // namespace

extern "C" csp_status csp_autotune(csp_context* c, int32_t n_inst, const csp_lattice* const* lats,
                                   const int32_t* R, const csp_params* params_in,
                                   csp_tuning* out) {
  if (!c || n_inst < 1 || !lats || !R || !params_in) return fail(CSP_EINVAL, "NULL argument");
  csp_params P;
  fill_defaults(params_in, &P);
  if (P.mode < CSP_FP64_SEQ || P.mode > CSP_FP32_CONC) return fail(CSP_EINVAL, "bad mode %d", P.mode);
  if (P.assembly != CSP_ASSEMBLE_STATES && P.assembly != CSP_ASSEMBLE_MOMENTS)
    return fail(CSP_EINVAL, "bad assembly %d", P.assembly);
  const bool fp64 = P.mode != CSP_FP32_CONC;
  const bool mom = P.assembly == CSP_ASSEMBLE_MOMENTS;
  // the moment form of one block (no final state) uses the halving identity
  const bool halving_t = mom && P.mode != CSP_FP64_SEQ && (P.block_b <= 0 || P.block_b >= P.Nt);
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  std::vector<InstIn> ins(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    if (!lats[i] || R[i] < 1) return fail(CSP_EINVAL, "instance %d: NULL lattice or R < 1", i);
    if (lats[i]->ctx->device != c->device) return fail(CSP_EINVAL, "instance %d on another device", i);
    ins[i] = {lats[i], nullptr, R[i], nullptr, nullptr, R[i], 0};
  }
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;

  // column groups, as csp_propagate forms them
  std::vector<Group> groups;
  int64_t vec_elems = 0;
  int rmax = 1;
  for (size_t i = 0; i < ins.size(); ++i) {
    int col = ins[i].col_base;
    for (int Rg : split_columns(ins[i].R, ins[i].lat->g.kind == CSP_SPARSE)) {
      Group g;
      g.inst = (int)i;
      g.col0 = col;
      g.Rg = Rg;
      set_layout(g, ins[i].lat);
      groups.push_back(g);
      vec_elems += g.M;
      rmax = std::max(rmax, Rg);
      col += Rg;
    }
  }
  std::vector<ChebInst> sp;
  for (auto& g : groups) {
    sp.push_back(make_inst(ins[g.inst].lat, g.Rg, fp64));
    apply_layout(sp.back(), g);
  }

  // recursion candidates (values per lane, steps per launch, rows per work
  // item) and the largest record buffer among them
  struct Cand { int vec, kt, seg; };
  std::vector<Cand> cands;
  int64_t max_rec = 0;
  bool any_sparse = false;
  for (auto& I : sp) any_sparse = any_sparse || I.kind == CSP_SPARSE;
  for (int v = 2; v <= (any_sparse ? 2 : 4); v *= 2)
    for (int kt = 1; kt <= (any_sparse ? 1 : 8); kt *= 2) {
      if (!cheb_shape_supported(fp64, v, kt, mom)) continue;
      for (int seg = 8; seg <= (any_sparse ? 8 : 128); seg *= 2) {
        std::vector<ChebInst> tmp_sp = sp;
        ChebPlan p = plan_cheb(tmp_sp, fp64, mom, c->n_cu, v, kt, seg);
        if (p.total_items < 1 || ceil_div(p.total_items, 4) > INT32_MAX) continue;
        cands.push_back({v, kt, seg});
        max_rec = std::max(max_rec, p.total_items * kt);
      }
    }

  // coefficient table for the cost model and the contraction operands
  const int bmax = P.mode == CSP_FP64_SEQ ? 1 : (fp64 ? kMaxFp64B : 32 * kMaxJTiles);
  const int ncol = bmax;
  const int nmax = (int)trunc_nmax(ncol * P.tau_tilde);
  const int lda = nmax + 1;
  struct Free {
    std::vector<void*> p;
    ~Free() { for (void* q : p) (void)hipFree(q); }
  } tmp;
  double* d_a = nullptr;
  int32_t* d_ntr = nullptr;
  HIPCALL(hipMalloc(&d_a, sizeof(double) * (size_t)ncol * lda));
  tmp.p.push_back(d_a);
  HIPCALL(hipMalloc(&d_ntr, sizeof(int32_t) * ncol));
  tmp.p.push_back(d_ntr);
  HIPCALL(launch_bessel(P.tau_tilde, ncol, nmax, P.eta, true, d_a, d_ntr, s));
  std::vector<int32_t> ntr(ncol);
  HIPCALL(hipMemcpyAsync(ntr.data(), d_ntr, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, s));
  HIPCALL(hipStreamSynchronize(s));
  for (int j = 0; j < ncol; ++j)
    if (ntr[j] < 1) return fail(CSP_ENUMERIC, "no truncation order for x = %g", (j + 1) * P.tau_tilde);

  // timing workspace: K_t Chebyshev slots per group (3 for the recursion
  // alone), psi0, carry, partial sums, operand tables
  size_t cap = 0;
  CHECK(memory_cap(c, P.mem_cap_bytes, &cap));
  const int wg_max = 8 * c->n_cu + kMaxGroupCols * (int)groups.size();
  auto tune_ws = [&](int S_) {
    size_t by = 0;
    for (auto& g : groups) by += align256((size_t)S_ * g.stride() * csz) + 2 * align256(g.M * csz);
    by += align256((size_t)max_rec * 8 * sizeof(double));                    // moment records
    by += align256((size_t)wg_max * 64 * 16);                                // contraction partials
    by += 2 * align256(bop_bytes(kMaxJTiles, 32)) + 2 * align256(sizeof(double2) * 32 * 17);
    by += align256(sizeof(ChebInst) * groups.size()) + align256(sizeof(ContractInst) * groups.size());
    return by;
  };
  // slots: the recursion writes up to 8 levels after phi_{n-1}, phi_n
  int K_t = (mom || P.mode == CSP_FP64_SEQ) ? 10 : 32;
  while (K_t > 16 && tune_ws(K_t) > cap) K_t -= 16;
  if (K_t > 10 && tune_ws(K_t) > cap) K_t = 10;
  if (tune_ws(K_t) > cap)
    return fail(CSP_ENOMEM, "autotuner workspace %.2f GB exceeds the cap %.2f GB", tune_ws(K_t) / 1e9,
                cap / 1e9);
  CHECK(ws_reserve(c, tune_ws(K_t)));
  Carver cv(c->ws);
  for (auto& g : groups) {
    g.slots = cv.take((size_t)K_t * g.stride() * csz);
    g.psi0g = cv.take(g.M * csz);
    g.carry = cv.take(g.M * csz);
  }
  double* d_part = (double*)cv.take((size_t)max_rec * 8 * sizeof(double));
  double* d_cpart = (double*)cv.take((size_t)wg_max * 64 * 16);
  void* d_bop1 = cv.take(bop_bytes(kMaxJTiles, 32));
  void* d_bop2 = cv.take(bop_bytes(kMaxJTiles, 32));
  float* d_cc1 = (float*)cv.take(sizeof(double2) * 32 * 17);
  float* d_cc2 = (float*)cv.take(sizeof(double2) * 32 * 17);
  ChebInst* d_spmm = (ChebInst*)cv.take(sizeof(ChebInst) * groups.size());
  ContractInst* d_con = (ContractInst*)cv.take(sizeof(ContractInst) * groups.size());
  // state values: random phases in every slot, psi0 and carry
  for (auto& g : groups) {
    const int64_t N = ins[g.inst].lat->g.N;
    for (int k = 0; k < K_t; ++k)
      HIPCALL(launch_random_phase(N, g.Rg, 0x5eed + k, fp64 ? CSP_C128 : CSP_C64,
                                  static_cast<char*>(g.slots) + (size_t)k * g.stride() * csz, g.Rg, 0, s));
    HIPCALL(launch_random_phase(N, g.Rg, 0x1234, fp64 ? CSP_C128 : CSP_C64, g.psi0g, g.Rg, 0, s));
    HIPCALL(launch_random_phase(N, g.Rg, 0x4321, fp64 ? CSP_C128 : CSP_C64, g.carry, g.Rg, 0, s));
  }

  csp_tuning T{};
  // ---- recursion shapes: time per Chebyshev step of a launch of kt steps
  double best_ms = 1e30;
  for (auto& cd : cands) {
    std::vector<ChebInst> tsp = sp;
    ChebPlan p = plan_cheb(tsp, fp64, mom, c->n_cu, cd.vec, cd.kt, cd.seg);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      tsp[gi].base = groups[gi].slots;
      tsp[gi].slot_stride = groups[gi].stride();
      tsp[gi].psi0 = groups[gi].psi0g;
    }
    CHECK(attach_ell_shadows(c, tsp, fp64));
    HIPCALL(hipMemcpyAsync(d_spmm, tsp.data(), sizeof(ChebInst) * tsp.size(),
                           hipMemcpyHostToDevice, s));
    ChebStep st = step_args(p);
    st.nlev = p.kt;
    st.slot_cur = 1;
    st.slot_prev = 0;
    set_shadow(st, 1);   // a step inside a block, as the recursion runs it
    if (mom) {
      // moment form: the two newest levels are kept; one block (halving)
      // runs the self products without psi0, time blocks the products
      // with psi0
      st.slot_out[p.kt - 1] = 2;
      if (p.kt >= 2) st.slot_out[p.kt - 2] = 3;
      st.dot_psi0 = halving_t ? 0 : 1;
      st.dot_self = halving_t ? 1 : 0;
    } else {
      for (int l = 1; l <= p.kt; ++l) st.slot_out[l - 1] = 1 + l;
    }
    st.partial = d_part;
    double ms = 0;
    CHECK(time_launch(c, [&]() -> csp_status {
      HIPCALL(launch_cheb(fp64, p.vec, p.kt, mom, false, d_spmm, p.runs, st, s));
      return CSP_OK;
    }, &ms));
    ms /= p.kt;
    ++T.n_candidates;
    if (ms < best_ms) {
      best_ms = ms;
      T.spmm_vec = p.vec;
      T.spmm_steps = p.kt;
      T.spmm_seg_rows = p.seg_rows;
    }
  }
  T.t_amxsy_us = best_ms * 1000.0;

  // ---- contraction (state assembly)
  T.contract_wg_per_cu = 4;
  T.t_order_us[0] = T.t_order_us[1] = -1.0;
  if (!mom && K_t >= 16) {
    const int jt_max = fp64 ? 1 : kMaxJTiles;
    auto setup = [&](int wpc, int* total) -> csp_status {
      std::vector<ContractInst> ct;
      int64_t Msum = 0;
      for (auto& g : groups) Msum += g.M;
      int wg0 = 0;
      for (auto& g : groups) {
        const int64_t N = g.M / g.Rg;
        const int64_t units = fp64 ? ceil_div(N, kContractThreads) : ceil_div(ceil_div(N, 32), 4);
        const double share = (double)c->n_cu * wpc * (double)g.M / (double)Msum / g.Rg;
        const int w = (int)std::max<int64_t>(1, std::min<int64_t>(std::llround(share), units));
        ContractInst C{};
        C.slots = g.slots;
        C.slot_stride = g.stride();
        C.N = N;
        C.Rg = g.Rg;
        C.wpc = w;
        C.psi0 = g.psi0g;
        C.carry = g.carry;
        C.partial = d_cpart;   // timing only: instances may share it
        C.wg0 = wg0;
        C.n_wg = g.Rg * w;
        wg0 += C.n_wg;
        ct.push_back(C);
      }
      HIPCALL(hipMemcpyAsync(d_con, ct.data(), sizeof(ContractInst) * ct.size(),
                             hipMemcpyHostToDevice, s));
      *total = wg0;
      return CSP_OK;
    };
    const int K = std::min(K_t, 32);
    if (fp64) {
      HIPCALL(launch_pack_c64(d_a, lda, d_ntr, kMaxFp64B, 0, K, (double*)d_bop1, (double*)d_cc1, s));
    } else {
      HIPCALL(launch_pack_bop(d_a, lda, d_ntr, 32, 1, 0, K, d_bop1, d_cc1, s));
      HIPCALL(launch_pack_bop(d_a, lda, d_ntr, 64, 2, 0, K, d_bop2, d_cc2, s));
    }
    auto run = [&](int jt, int total) -> csp_status {
      ContractArgs ca{};
      ca.n_inst = (int)groups.size();
      ca.n_lo = 0;
      ca.n_cnt = K;
      ca.S = K_t;
      ca.G = ring_parts(K_t);
      ca.first_chunk = 0;
      ca.jtiles = jt;
      ca.bcols = fp64 ? kMaxFp64B : 32 * jt;
      ca.total_wg = total;
      if (fp64) {
        ca.coef = d_bop1;
        ca.ccarry = d_cc1;
        HIPCALL(launch_contract_f64(d_con, ca, s));
      } else {
        ca.bop = jt == 1 ? d_bop1 : d_bop2;
        ca.ccarry = jt == 1 ? d_cc1 : d_cc2;
        HIPCALL(launch_contract_f32(d_con, ca, s));
      }
      return CSP_OK;
    };
    double best = 1e30;
    for (int wpc = 2; wpc <= 8; wpc *= 2) {
      int total = 0;
      CHECK(setup(wpc, &total));
      double ms = 0;
      CHECK(time_launch(c, [&]() { return run(1, total); }, &ms));
      if (ms < best) {
        best = ms;
        T.contract_wg_per_cu = wpc;
      }
    }
    T.t_order_us[0] = best * 1000.0 / K;
    if (jt_max > 1) {
      int total = 0;
      CHECK(setup(T.contract_wg_per_cu, &total));
      double ms = 0;
      CHECK(time_launch(c, [&]() { return run(2, total); }, &ms));
      T.t_order_us[1] = ms * 1000.0 / K;
    }
  }

  // ---- time-block size by the cost model
  for (int k = 0; k < 8; ++k) T.model_cost_ms[k] = -1.0;
  T.block_b = 0;
  if (!mom) {
    const int64_t Nt = std::max<int64_t>(P.Nt, 1);
    const int wg_total = c->n_cu * T.contract_wg_per_cu + kMaxGroupCols * (int)groups.size();
    const int kt_best = std::max(1, T.spmm_steps);
    auto state_ws = [&](int K_, int b) {
      const int S_ = std::max(K_ + kt_best, kt_best + 2);
      size_t by = 0;
      for (auto& g : groups) by += align256((size_t)S_ * g.stride() * csz) + 2 * align256(g.M * csz);
      by += align256((size_t)wg_total * b * 16) * 2;
      return by + (64u << 20);
    };
    auto cost = [&](int b) -> double {
      const int jt = fp64 ? 1 : (int)ceil_div(b, 32);
      const double t_ord = T.t_order_us[jt - 1];
      if (t_ord < 0 && b > 1 && P.mode != CSP_FP64_SEQ) return -1.0;
      const int Ktot = ntr[b - 1] + 1;
      const int kcap = fp64 ? (1 << 20) : (496 / jt / 16) * 16;
      int K = std::min(Ktot, kcap);
      if (K < Ktot) K = (K / 16) * 16;
      while (K > 16 && state_ws(K, b) > cap) K = ((K - 1) / 16) * 16;
      if (state_ws(K, b) > cap) return -1.0;
      double us = 0;
      for (int64_t t0 = 0; t0 < Nt; t0 += b) {
        const int bk = (int)std::min<int64_t>(b, Nt - t0);
        const int Nk = ntr[bk - 1];
        const int chunks = (int)ceil_div(Nk + 1, K);
        // the carry is read back and rewritten once per extra chunk
        us += Nk * T.t_amxsy_us + (Nk + 1 + 2 * (chunks - 1)) * std::max(t_ord, 0.0);
      }
      return us / 1000.0;
    };
    double best = 1e300;
    for (int b = 1; b <= bmax; ++b) {
      const double cb = cost(b);
      if (cb >= 0 && cb < best) {
        best = cb;
        T.block_b = b;
      }
    }
    for (int b = 1, k = 0; b <= 128; b *= 2, ++k) T.model_cost_ms[k] = b <= bmax ? cost(b) : -1.0;
  }
  c->tuned[shape_key(ins, fp64, P.assembly)] = T;
  if (out) *out = T;
  return CSP_OK;
}

extern "C" csp_status csp_set_tuning(csp_context* c, int32_t n_inst,
                                      const csp_lattice* const* lats, const int32_t* R,
                                      const csp_params* params_in, const csp_tuning* T) {
  if (!c || n_inst < 1 || !lats || !R || !params_in || !T) return fail(CSP_EINVAL, "NULL argument");
  csp_params P;
  fill_defaults(params_in, &P);
  if (P.mode < CSP_FP64_SEQ || P.mode > CSP_FP32_CONC) return fail(CSP_EINVAL, "bad mode %d", P.mode);
  if (P.assembly != CSP_ASSEMBLE_STATES && P.assembly != CSP_ASSEMBLE_MOMENTS)
    return fail(CSP_EINVAL, "bad assembly %d", P.assembly);
  const bool fp64 = P.mode != CSP_FP32_CONC;
  const bool mom = P.assembly == CSP_ASSEMBLE_MOMENTS;
  if (!cheb_shape_supported(fp64, T->spmm_vec, T->spmm_steps, mom))
    return fail(CSP_EINVAL, "no recursion kernel for %d values per lane, %d steps per launch",
                T->spmm_vec, T->spmm_steps);
  if (T->spmm_seg_rows < 1 || T->contract_wg_per_cu < 1 || T->block_b < 0)
    return fail(CSP_EINVAL, "rows per work item and workgroups per CU must be >= 1, b >= 0");
  std::vector<InstIn> ins(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    if (!lats[i] || R[i] < 1) return fail(CSP_EINVAL, "instance %d: NULL lattice or R < 1", i);
    ins[i] = {lats[i], nullptr, R[i], nullptr, nullptr, R[i], 0};
  }
  c->tuned[shape_key(ins, fp64, P.assembly)] = *T;
  return CSP_OK;
}

extern "C" csp_status csp_select_block(csp_context* c, const csp_lattice* L, int32_t R,
                                       const csp_params* params, int32_t* b_out, csp_report* rep) {
  if (!c || !L || !params || !b_out) return fail(CSP_EINVAL, "NULL argument");
  csp_params P;
  fill_defaults(params, &P);
  P.assembly = CSP_ASSEMBLE_STATES;
  const bool fp64 = P.mode != CSP_FP32_CONC;
  std::vector<InstIn> ins(1);
  ins[0] = {L, nullptr, R, nullptr, nullptr, R, 0};
  csp_tuning T{};
  const csp_tuning* have = find_tuning(c, ins, fp64, CSP_ASSEMBLE_STATES);
  if (have) {
    T = *have;
  } else {
    const csp_lattice* lats[1] = {L};
    CHECK(csp_autotune(c, 1, lats, &R, &P, &T));
  }
  *b_out = T.block_b;
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->block_b = T.block_b;
    for (int k = 0; k < 8; ++k) rep->model_cost[k] = T.model_cost_ms[k];
  }
  return CSP_OK;
}

// ------------------------------------------------------------------ bandwidth probe
extern "C" csp_status csp_bandwidth_probe(csp_context* c, uint64_t bytes, double* gbs_out) {
  if (!c || !gbs_out) return fail(CSP_EINVAL, "NULL argument");
  bytes = (bytes / 4096) * 4096;
  if (bytes < (1u << 20)) return fail(CSP_EINVAL, "need at least 1 MiB per array");
  DeviceGuard dg(c->device);
  hipStream_t s = c->stream;
  CHECK(ws_reserve(c, 3 * bytes + 4096));
  Carver cv(c->ws);
  void* a = cv.take(bytes);
  void* b = cv.take(bytes);
  void* d = cv.take(bytes);
  float* sink = (float*)cv.take(4096);
  const int64_t n16 = (int64_t)(bytes / 16);
  // defined contents for the reads
  HIPCALL(launch_probe(1, nullptr, nullptr, a, sink, n16, 4 * c->n_cu, s));
  HIPCALL(launch_probe(1, nullptr, nullptr, b, sink, n16, 4 * c->n_cu, s));
  for (int kind = 0; kind < 3; ++kind) {
    double best = 0.0;
    for (int wpc = 4; wpc <= 64; wpc *= 2) {
      const int grid = wpc * c->n_cu;
      double ms = 0;
      CHECK(time_launch(c, [&]() -> csp_status {
        HIPCALL(launch_probe(kind, a, b, d, sink, n16, grid, s));
        return CSP_OK;
      }, &ms));
      const double moved = (kind == 2 ? 3.0 : 1.0) * (double)bytes;
      best = std::max(best, moved / (ms * 1e-3) / 1e9);
    }
    gbs_out[kind] = best;
  }
  return CSP_OK;
}
