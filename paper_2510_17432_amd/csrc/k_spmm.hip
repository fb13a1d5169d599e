// Chebyshev recursion step (amxsy of Sec. II.B): out = s * (2 H~ cur) - prev
// on [N][R] complex blocks, with H~ = (H - H0)/|H| the rescaled lattice
// Hamiltonian of Sec. II.A applied as a stencil (no matrix in memory).
//
// Work decomposition.  A lattice row (fixed y) is a contiguous run of
// rowlen = orbitals_per_row * R complex values.  A workgroup owns a strip of
// W = 256*V values of that run and a segment of seg_rows rows, and marches
// down the rows keeping rows y-1, y, y+1 of `cur` (plus an R-value halo on
// each side) in a three-slot LDS ring.  Every value of `cur` is read from HBM
// once per segment (two extra halo rows per segment), `prev` once and `out`
// written once: 3 vectors of traffic per step, the minimum for this
// recursion.  The next row of `cur` and of `prev` are fetched into registers
// one iteration ahead so that HBM latency overlaps the stencil work.
//
// Thread t handles strip offsets i = v*256 + t (v < V): each wave's loads
// and stores touch consecutive complex values (coalesced) and its LDS reads
// hit consecutive banks.
//
// Neighbours inside a row are at +-R values (one orbital left/right); rows
// y-1 and y+1 carry the vertical bonds.  Square: left, right, down, up.
// Honeycomb (orbital 2x+sigma): A reaches B(x), B(x-1) in its row and
// B(x, y-1); B reaches A(x), A(x+1) and A(x, y+1).  Chain: left, right.
// Open edges read zeros from the halo; periodic edges wrap.
#include "csp_internal.h"

namespace csp {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

template <typename C> __device__ inline C czero() { C z; z.x = 0; z.y = 0; return z; }

template <typename T, int V>
__global__ __launch_bounds__(kSpmmThreads) void k_spmm(const SpmmInst* __restrict__ insts,
                                                       int n_inst, SpmmStep st) {
  using C = typename cplx_of<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  C* lds = reinterpret_cast<C*>(smem);
  constexpr int W = kSpmmThreads * V;
  const int ldsw = W + 2 * st.halo;
  const int tid = threadIdx.x;

  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  int ii = 0;
  while (ii + 1 < n_inst && tile >= insts[ii + 1].tile0) ++ii;
  const SpmmInst& I = insts[ii];

  const int R = I.R;
  const int kind = I.kind;
  const int64_t rowlen = I.rowlen;
  const int64_t Ly = I.Ly;
  const int64_t tl = tile - I.tile0;
  const int64_t strip = tl % I.n_strips;
  const int64_t seg = tl / I.n_strips;
  const int64_t e0 = strip * W;
  const int width = static_cast<int>(rowlen - e0 < W ? rowlen - e0 : W);
  const int64_t y0 = seg * st.seg_rows;
  const int64_t y1 = (y0 + st.seg_rows < Ly) ? y0 + st.seg_rows : Ly;

  C* base = static_cast<C*>(I.base);
  const C* cur = st.cur_from_src ? static_cast<const C*>(I.src) : base + st.slot_cur * I.slot_stride;
  C* out = base + st.slot_out * I.slot_stride;
  const C* prev = base + st.slot_prev * I.slot_stride;
  C* copy = st.copy_cur ? base + st.slot_cur * I.slot_stride : nullptr;
  const T* eps = static_cast<const T*>(I.eps);
  const T alpha = static_cast<T>(I.alpha);
  const T beta0 = static_cast<T>(I.beta0);
  const T oscale = static_cast<T>(I.onsite_scale);
  const T scale = sizeof(T) == 4 ? static_cast<T>(st.scale_f) : static_cast<T>(st.scale_d);
  const bool vertical = kind != CSP_CHAIN;

  // Per-thread element geometry (identical for every row).
  int64_t ev[V];
  int64_t xv[V];
  bool valid[V];
  int sig[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int i = v * kSpmmThreads + tid;
    valid[v] = i < width;
    ev[v] = e0 + i;
    xv[v] = valid[v] ? ev[v] / R : 0;
    sig[v] = static_cast<int>(xv[v] & 1);
  }
  // Halo element handled by this thread (tid < 2R): position in the row or -1.
  int64_t he = -1;
  int hslot = 0;
  if (tid < 2 * R) {
    int64_t e = (tid < R) ? e0 - R + tid : e0 + width + (tid - R);
    if (e < 0) e = I.px ? e + rowlen : -1;
    else if (e >= rowlen) e = I.px ? e - rowlen : -1;
    he = e;
    hslot = (tid < R) ? tid : R + width + (tid - R);
  }

  C cen[V];
  C hal;
  auto fetch = [&](int64_t yy) {
    bool zero = false;
    int64_t yr = yy;
    if (!vertical && yy != 0) zero = true;
    if (yy < 0) { if (I.py) yr = yy + Ly; else zero = true; }
    else if (yy >= Ly) { if (I.py) yr = yy - Ly; else zero = true; }
    const C* rp = cur + yr * rowlen;
#pragma unroll
    for (int v = 0; v < V; ++v) cen[v] = (valid[v] && !zero) ? rp[ev[v]] : czero<C>();
    hal = (he >= 0 && !zero) ? rp[he] : czero<C>();
  };
  auto stash = [&](int slot) {
    C* d = lds + slot * ldsw;
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (valid[v]) d[R + v * kSpmmThreads + tid] = cen[v];
    // The right halo sits just past the valid part of a short strip, where
    // the slots of invalid threads would be: those threads store nothing.
    if (tid < 2 * R) d[hslot] = hal;
  };

  // Ring: row yy lives in slot (yy - y0 + 1) % 3.
  fetch(y0 - 1); stash(0);
  fetch(y0);     stash(1);
  fetch(y0 + 1); stash(2);
  __syncthreads();
  if (y0 + 1 < y1) fetch(y0 + 2);

  C prv[V], prvn[V];
  T ep[V], epn[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    prv[v] = (st.has_prev && valid[v]) ? prev[y0 * rowlen + ev[v]] : czero<C>();
    ep[v] = (eps && valid[v]) ? eps[y0 * I.opr + xv[v]] : T(0);
  }

  int sm = 0, sc = 1, sp = 2;
  for (int64_t y = y0; y < y1; ++y) {
    const bool more = y + 1 < y1;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      prvn[v] = (more && st.has_prev && valid[v]) ? prev[(y + 1) * rowlen + ev[v]] : czero<C>();
      epn[v] = (more && eps && valid[v]) ? eps[(y + 1) * I.opr + xv[v]] : T(0);
    }
    const C* Lm = lds + sm * ldsw + R;
    const C* Lc = lds + sc * ldsw + R;
    const C* Lp = lds + sp * ldsw + R;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (!valid[v]) continue;
      const int i = v * kSpmmThreads + tid;
      const C c = Lc[i];
      const C l = Lc[i - R];
      const C r = Lc[i + R];
      T nx = l.x + r.x, ny = l.y + r.y;
      if (kind == CSP_SQUARE) {
        const C d = Lm[i], u = Lp[i];
        nx += d.x + u.x;
        ny += d.y + u.y;
      } else if (kind == CSP_HONEYCOMB) {
        const C z = sig[v] ? Lp[i - R] : Lm[i + R];
        nx += z.x;
        ny += z.y;
      }
      const T beta = beta0 + oscale * ep[v];
      C o;
      o.x = scale * (alpha * nx + beta * c.x) - prv[v].x;
      o.y = scale * (alpha * ny + beta * c.y) - prv[v].y;
      out[y * rowlen + ev[v]] = o;
      if (copy) copy[y * rowlen + ev[v]] = c;
    }
    if (more) {
      __syncthreads();          // every thread is done with row y-1's slot
      stash(sm);                // row y+2 replaces row y-1
      if (y + 2 < y1) fetch(y + 3);
      __syncthreads();
      const int t = sm; sm = sc; sc = sp; sp = t;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) { prv[v] = prvn[v]; ep[v] = epn[v]; }
  }
}

hipError_t launch_spmm(bool fp64, int vec, const SpmmInst* d_inst, int n_inst,
                       const SpmmStep& st, hipStream_t s) {
  if (st.total_tiles <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(st.total_tiles)), block(kSpmmThreads);
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  const size_t lds = 3 * (size_t)(kSpmmThreads * vec + 2 * st.halo) * csz;
  if (fp64) {
    switch (vec) {
      case 1: hipLaunchKernelGGL((k_spmm<double, 1>), grid, block, lds, s, d_inst, n_inst, st); break;
      case 2: hipLaunchKernelGGL((k_spmm<double, 2>), grid, block, lds, s, d_inst, n_inst, st); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (vec) {
      case 1: hipLaunchKernelGGL((k_spmm<float, 1>), grid, block, lds, s, d_inst, n_inst, st); break;
      case 2: hipLaunchKernelGGL((k_spmm<float, 2>), grid, block, lds, s, d_inst, n_inst, st); break;
      case 4: hipLaunchKernelGGL((k_spmm<float, 4>), grid, block, lds, s, d_inst, n_inst, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace csp
