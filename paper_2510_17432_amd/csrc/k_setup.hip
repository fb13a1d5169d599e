// Set-up and small kernels: on-site disorder, spectral bound, neighbour
// table, random-phase and localized states, column-group gather/scatter,
// <psi0|psi0>, and the DOS transform (Sec. III).
#include <mutex>

#include "csp_internal.h"

namespace csp {

// ------------------------------------------------------------------ lattice
__global__ void k_onsite(int64_t N, double W, uint64_t seed, double* __restrict__ e64,
                         float* __restrict__ e32) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const double e = W * (rng_unit(rng_draw(seed, 0, (uint64_t)s)) - 0.5);
  e64[s] = e;
  e32[s] = static_cast<float>(e);
}

hipError_t launch_onsite(const Geom& g, double W, uint64_t seed, double* d_eps64, float* d_eps32,
                         hipStream_t s) {
  const int64_t nb = ceil_div(g.N, 256);
  hipLaunchKernelGGL(k_onsite, dim3((unsigned)nb), dim3(256), 0, s, g.N, W, seed, d_eps64, d_eps32);
  return hipGetLastError();
}

// Gershgorin row bound max_s (|eps_s - H0| + deg(s) |t|); one max per block.
__global__ void k_gershgorin(Geom g, const double* __restrict__ eps, double t, double H0,
                             double* __restrict__ partial) {
  __shared__ double red[256];
  double m = 0.0;
  const int deg_max = max_degree(g.kind);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < g.N;
       s += (int64_t)gridDim.x * blockDim.x) {
    int deg = 0;
    for (int k = 0; k < deg_max; ++k) deg += neighbour(g, s, k) >= 0 ? 1 : 0;
    const double e = eps ? eps[s] : 0.0;
    double r;
    {
      // No fused multiply-add here: the bound must be reproducible bit for
      // bit by any IEEE implementation of the same expression.
#pragma clang fp contract(off)
      r = fabs(e - H0) + (double)deg * fabs(t);
    }
    m = r > m ? r : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double o = red[threadIdx.x + w];
      red[threadIdx.x] = o > red[threadIdx.x] ? o : red[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_gershgorin(const Geom& g, const double* d_eps, double t, double H0,
                             double* d_partial, int n_partial, hipStream_t s) {
  hipLaunchKernelGGL(k_gershgorin, dim3(n_partial), dim3(256), 0, s, g, d_eps, t, H0, d_partial);
  return hipGetLastError();
}

__global__ void k_neighbours(Geom g, int64_t* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.N) return;
  const int d = max_degree(g.kind);
  for (int k = 0; k < d; ++k) out[s * d + k] = neighbour(g, s, k);
}

hipError_t launch_neighbours(const Geom& g, int64_t* d_nbr, hipStream_t s) {
  hipLaunchKernelGGL(k_neighbours, dim3((unsigned)ceil_div(g.N, 256)), dim3(256), 0, s, g, d_nbr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ states
__global__ void k_random_phase(int64_t N, int R, uint64_t seed, int dtype, void* __restrict__ psi,
                               int ld, int col0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * R) return;
  const int64_t s = e / R;
  const int r = static_cast<int>(e - s * R);
  const double u = rng_unit(rng_draw(seed, (uint64_t)r, (uint64_t)s));
  double sn, cs;
  sincospi(2.0 * u, &sn, &cs);
  const double inv = 1.0 / sqrt(static_cast<double>(N));
  const int64_t at = s * ld + col0 + r;
  if (dtype == CSP_C128)
    static_cast<double2*>(psi)[at] = make_double2(cs * inv, sn * inv);
  else
    static_cast<float2*>(psi)[at] = make_float2(static_cast<float>(cs * inv),
                                                static_cast<float>(sn * inv));
}

hipError_t launch_random_phase(int64_t N, int R, uint64_t seed, int dtype, void* d_psi, int ld,
                               int col0, hipStream_t s) {
  hipLaunchKernelGGL(k_random_phase, dim3((unsigned)ceil_div(N * R, 256)), dim3(256), 0, s, N, R,
                     seed, dtype, d_psi, ld, col0);
  return hipGetLastError();
}

// Sequential by nature (distinct draws in order); one thread.
__global__ void k_ldos_sites(int64_t N, int n, uint64_t seed, int64_t* __restrict__ sites) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int got = 0;
  for (uint64_t i = 0; got < n; ++i) {
    const uint64_t bits = rng_draw(seed, 0, i);
    const int64_t s = static_cast<int64_t>(__umul64hi(bits, static_cast<uint64_t>(N)));
    bool dup = false;
    for (int k = 0; k < got; ++k) dup |= sites[k] == s;
    if (!dup) sites[got++] = s;
  }
}

hipError_t launch_ldos_sites(int64_t N, int n, uint64_t seed, int64_t* d_sites, hipStream_t s) {
  hipLaunchKernelGGL(k_ldos_sites, dim3(1), dim3(1), 0, s, N, n, seed, d_sites);
  return hipGetLastError();
}

__global__ void k_site_states(int64_t N, int n, const int64_t* __restrict__ sites, int dtype,
                              void* __restrict__ psi, int ld, int col0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * n) return;
  const int64_t s = e / n;
  const int k = static_cast<int>(e - s * n);
  const double v = sites[k] == s ? 1.0 : 0.0;
  const int64_t at = s * ld + col0 + k;
  if (dtype == CSP_C128)
    static_cast<double2*>(psi)[at] = make_double2(v, 0.0);
  else
    static_cast<float2*>(psi)[at] = make_float2(static_cast<float>(v), 0.f);
}

hipError_t launch_site_states(int64_t N, int n, const int64_t* d_sites, int dtype, void* d_psi,
                              int ld, int col0, hipStream_t s) {
  hipLaunchKernelGGL(k_site_states, dim3((unsigned)ceil_div(N * n, 256)), dim3(256), 0, s, N, n,
                     d_sites, dtype, d_psi, ld, col0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ column groups
// A column group is stored column-major, [Rg][N]: column c of the group is
// values c*N .. c*N + N - 1 (one lattice vector).  Gather/scatter convert
// from/to the caller's orbital-major [N][ld] blocks.
// Element e of the group: column c, row r, position p (pitch and opr equal
// to N when the group is not padded).
__global__ void k_gather_cols(int64_t N, int ld, int col0, int Rg, int in_dtype,
                              const void* __restrict__ in, int fp64, void* __restrict__ out,
                              int64_t opr, int64_t pitch, int64_t Nc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nc * Rg) return;
  const int64_t c = e / Nc;
  const int64_t q = e - c * Nc;
  const int64_t r = q / pitch;
  const int64_t p = q - r * pitch;
  double x = 0.0, y = 0.0;
  if (p < opr) {
    const int64_t at = (r * opr + p) * ld + col0 + c;
    if (in_dtype == CSP_C128) {
      const double2 v = static_cast<const double2*>(in)[at];
      x = v.x; y = v.y;
    } else {
      const float2 v = static_cast<const float2*>(in)[at];
      x = v.x; y = v.y;
    }
  }
  if (fp64) static_cast<double2*>(out)[e] = make_double2(x, y);
  else static_cast<float2*>(out)[e] = make_float2(static_cast<float>(x), static_cast<float>(y));
}

hipError_t launch_gather_cols(int64_t N, int ld, int col0, int Rg, int in_dtype, const void* d_in,
                              bool fp64, void* d_out, hipStream_t s, int64_t opr, int64_t pitch) {
  if (pitch <= 0) opr = pitch = N;
  if (opr <= 0 || pitch < opr || N % opr != 0) return hipErrorInvalidValue;
  const int64_t Nc = N / opr * pitch;
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)ceil_div(Nc * Rg, 256)), dim3(256), 0, s, N,
                     ld, col0, Rg, in_dtype, d_in, fp64 ? 1 : 0, d_out, opr, pitch, Nc);
  return hipGetLastError();
}

__global__ void k_scatter_cols(int64_t N, int ld, int col0, int Rg, int out_dtype,
                               const void* __restrict__ in, int fp64, void* __restrict__ out,
                               int64_t opr, int64_t pitch, int64_t Nc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Nc * Rg) return;
  const int64_t c = e / Nc;
  const int64_t q = e - c * Nc;
  const int64_t r = q / pitch;
  const int64_t p = q - r * pitch;
  if (p >= opr) return;
  double x, y;
  if (fp64) {
    const double2 v = static_cast<const double2*>(in)[e];
    x = v.x; y = v.y;
  } else {
    const float2 v = static_cast<const float2*>(in)[e];
    x = v.x; y = v.y;
  }
  const int64_t at = (r * opr + p) * ld + col0 + c;
  if (out_dtype == CSP_C128) static_cast<double2*>(out)[at] = make_double2(x, y);
  else static_cast<float2*>(out)[at] = make_float2(static_cast<float>(x), static_cast<float>(y));
}

hipError_t launch_scatter_cols(int64_t N, int ld, int col0, int Rg, int out_dtype, const void* d_in,
                               bool fp64, void* d_out, hipStream_t s, int64_t opr, int64_t pitch) {
  if (pitch <= 0) opr = pitch = N;
  if (opr <= 0 || pitch < opr || N % opr != 0) return hipErrorInvalidValue;
  const int64_t Nc = N / opr * pitch;
  hipLaunchKernelGGL(k_scatter_cols, dim3((unsigned)ceil_div(Nc * Rg, 256)), dim3(256), 0, s, N,
                     ld, col0, Rg, out_dtype, d_in, fp64 ? 1 : 0, d_out, opr, pitch, Nc);
  return hipGetLastError();
}

// One thread per padding value: vector k = slot * Rg + c, row r, position
// opr + p.
__global__ void k_zero_pad(void* __restrict__ base, int64_t n_pad, int Rg, int64_t slot_stride,
                           int64_t cstride, int64_t Ly, int64_t opr, int64_t pitch, int fp64) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pad) return;
  const int64_t w = pitch - opr;
  const int64_t per_vec = Ly * w;
  const int64_t k = e / per_vec;
  const int64_t q = e - k * per_vec;
  const int64_t r = q / w;
  const int64_t p = opr + (q - r * w);
  const int64_t slot = k / Rg, c = k - slot * Rg;
  const int64_t at = slot * slot_stride + c * cstride + r * pitch + p;
  if (fp64) static_cast<double2*>(base)[at] = make_double2(0.0, 0.0);
  else static_cast<float2*>(base)[at] = make_float2(0.f, 0.f);
}

hipError_t launch_zero_pad(void* d_base, int n_slots, int64_t slot_stride, int Rg, int64_t cstride,
                           int64_t Ly, int64_t opr, int64_t pitch, bool fp64, hipStream_t s) {
  if (pitch <= opr || n_slots <= 0) return hipSuccess;
  const int64_t n_pad = (int64_t)n_slots * Rg * Ly * (pitch - opr);
  hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)ceil_div(n_pad, 256)), dim3(256), 0, s, d_base,
                     n_pad, Rg, slot_stride, cstride, Ly, opr, pitch, fp64 ? 1 : 0);
  return hipGetLastError();
}

// <psi_c|psi_c> per column of an [Rg][N] group: workgroup (x, c) sums column
// c with stride gridDim.x * 256 and reduces in a fixed order into
// partial[c * gridDim.x + x] (FP64); one thread per column then adds the
// partials in order.
__global__ void k_self_dot_partial(int64_t N, int Rg, const void* __restrict__ psi, int fp64,
                                   double* __restrict__ partial) {
  __shared__ double red[256];
  const int64_t c = blockIdx.y;
  double acc = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < N; s += (int64_t)gridDim.x * 256) {
    double x, y;
    if (fp64) { const double2 v = static_cast<const double2*>(psi)[c * N + s]; x = v.x; y = v.y; }
    else { const float2 v = static_cast<const float2*>(psi)[c * N + s]; x = v.x; y = v.y; }
    acc = fma(x, x, fma(y, y, acc));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[c * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_self_dot_finish(int n_wg, int Rg, const double* __restrict__ partial,
                                  double* __restrict__ corr, int col0) {
  const int r = threadIdx.x;
  if (r >= Rg) return;
  double s = 0.0;
  for (int w = 0; w < n_wg; ++w) s += partial[(int64_t)r * n_wg + w];
  corr[2 * (col0 + r)] = s;
  corr[2 * (col0 + r) + 1] = 0.0;
}

hipError_t launch_self_dot(int64_t N, int Rg, const void* d_psi, bool fp64, double* d_corr,
                           int col0, double* d_scratch, int n_scratch_wg, hipStream_t s) {
  hipLaunchKernelGGL(k_self_dot_partial, dim3(n_scratch_wg, Rg), dim3(256), 0, s, N, Rg, d_psi,
                     fp64 ? 1 : 0, d_scratch);
  hipLaunchKernelGGL(k_self_dot_finish, dim3(1), dim3(64), 0, s, n_scratch_wg, Rg, d_scratch,
                     d_corr, col0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ norm guard
// After a time block: the carried state must keep the norm of psi0 (the
// propagator is unitary) and every new correlation must be finite with
// |C_j| <= |psi0|^2 (Cauchy-Schwarz).  Thread r checks column r of the group:
// the carry norm from the self-dot partials (when carry_partial is set) and
// the correlation rows t0+1..t0+bk.  A violation stores the block index into
// flag[0] (smallest index wins) and the column into flag[1].
__global__ void k_guard(int n_wg, int Rg, const double* __restrict__ carry_partial,
                        const double* __restrict__ corr, int64_t ldc, int col0, int64_t t0,
                        int bk, double tol, int block, const int64_t* __restrict__ blk_dev,
                        int* __restrict__ flag) {
  const int r = threadIdx.x;
  if (r >= Rg) return;
  if (blk_dev) {
    t0 = blk_dev[0];
    block = static_cast<int>(blk_dev[1]);
  }
  const double2* C = reinterpret_cast<const double2*>(corr);
  const double c0 = C[col0 + r].x;
  bool bad = !(c0 >= 0.0) || !isfinite(c0);
  if (carry_partial) {
    double s = 0.0;
    for (int w = 0; w < n_wg; ++w) s += carry_partial[(int64_t)r * n_wg + w];
    bad |= !isfinite(s) || fabs(s - c0) > tol * c0;
  }
  const double lim = (1.0 + tol) * c0;
  for (int j = 1; j <= bk; ++j) {
    const double2 v = C[(t0 + j) * ldc + col0 + r];
    bad |= !isfinite(v.x) || !isfinite(v.y) || sqrt(v.x * v.x + v.y * v.y) > lim;
  }
  if (bad) {
    if (atomicMin(&flag[0], block) > block) flag[1] = col0 + r;
  }
}

hipError_t launch_guard(int64_t N, int Rg, const void* d_carry, bool fp64, const double* d_corr,
                        int64_t ldc, int col0, int64_t t0, int bk, double tol, int block,
                        const int64_t* blk_dev, int* d_flag, double* d_scratch,
                        int n_scratch_wg, hipStream_t s) {
  if (d_carry)
    hipLaunchKernelGGL(k_self_dot_partial, dim3(n_scratch_wg, Rg), dim3(256), 0, s, N, Rg,
                       d_carry, fp64 ? 1 : 0, d_scratch);
  hipLaunchKernelGGL(k_guard, dim3(1), dim3(64), 0, s, n_scratch_wg, Rg,
                     d_carry ? d_scratch : nullptr, d_corr, ldc, col0, t0, bk, tol, block,
                     blk_dev, d_flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ DOS
// twiddle[m] = exp(i pi m / Nt), m = 0..2Nt-1 (exact arguments via sincospi).
__global__ void k_twiddle(int64_t Nt, double2* __restrict__ tw) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= 2 * Nt) return;
  double sn, cs;
  sincospi(static_cast<double>(m) / static_cast<double>(Nt), &sn, &cs);
  tw[m] = make_double2(cs, sn);
}

// D_r(E_k) for k = -Nt..Nt-1 (index k + Nt), pairing j with -j:
// (tau/2pi) [w_0 Re C_0 + 2 sum_{j=1}^{Nt-1} w_j Re(C_j e^{i pi k j/Nt})
//            + w_{Nt} Re(conj(C_Nt) e^{-i pi k})].
__global__ void k_dos(const double2* __restrict__ corr, int64_t Nt, int R, double pref,
                      int window, const double2* __restrict__ tw, double* __restrict__ D) {
  const int64_t kk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // 0..2Nt-1
  const int r = blockIdx.y;
  if (kk >= 2 * Nt) return;
  const int64_t two = 2 * Nt;
  const int64_t kpos = (kk - Nt + two) % two;   // k mod 2Nt, nonnegative
  auto w = [&](int64_t j) { return window == CSP_WINDOW_HANN ? 0.5 * (1.0 + tw[j].x) : 1.0; };
  double acc = w(0) * corr[r].x;
  int64_t idx = 0;
  for (int64_t j = 1; j < Nt; ++j) {
    idx += kpos;
    if (idx >= two) idx -= two;
    const double2 c = corr[j * R + r];
    const double2 t = tw[idx];
    acc += 2.0 * w(j) * (c.x * t.x - c.y * t.y);
  }
  {
    const double2 c = corr[Nt * R + r];
    const double2 t = tw[(two - (kpos * Nt) % two) % two];   // e^{-i pi k}
    acc += w(Nt) * (c.x * t.x + c.y * t.y);
  }
  D[kk * R + r] = pref * acc;
}

// Column mean, and the energies center + E_k of the centred transform.
__global__ void k_dos_mean(int64_t n, int R, const double* __restrict__ D, double* __restrict__ Dm,
                           double* __restrict__ E, double dE, int64_t Nt, double center) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += D[k * R + r];
  if (Dm) Dm[k] = s / R;
  E[k] = center + dE * static_cast<double>(k - Nt);
}

hipError_t launch_dos(const double* d_corr, int64_t Nt, int R, double halfwidth, double center,
                      double tau_tilde, int window, double* d_E, double* d_D, double* d_Dmean,
                      double* d_twiddle, hipStream_t s) {
  const int64_t n = 2 * Nt;
  double2* tw = reinterpret_cast<double2*>(d_twiddle);
  hipLaunchKernelGGL(k_twiddle, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, Nt, tw);
  const double tau = tau_tilde / halfwidth;
  const double pref = tau / (2.0 * M_PI);
  hipLaunchKernelGGL(k_dos, dim3((unsigned)ceil_div(n, 128), R), dim3(128), 0, s,
                     reinterpret_cast<const double2*>(d_corr), Nt, R, pref, window, tw, d_D);
  const double dE = M_PI / (static_cast<double>(Nt) * tau);
  hipLaunchKernelGGL(k_dos_mean, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, n, R, d_D,
                     d_Dmean, d_E, dE, Nt, center);
  return hipGetLastError();
}

// ------------------------------------------------------------------ DOS without allocation
// The twiddle table of csp_dos_noalloc: a static device array, one copy per
// device for the life of the process.  In host code `scratch` is a host-side
// stand-in; kernels get the device address from hipGetSymbolAddress, looked
// up once per device (that device current) and kept in g_scratch.
static __device__ __align__(256) double2 scratch[2 * CSP_DOS_NOALLOC_MAX_NT];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t dos_noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<double*>(p);
  }
  *out = g_scratch[device];
  return hipSuccess;
}

}  // namespace csp
