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
//
// Moment variant (MOM = true, moment-based form of Sec. II.A): the same
// step, plus per-column inner products of the new vector with psi0, of psi0
// with the current vector, and of the new vector with itself and with the
// current vector (the halving identity of Eq. cheby_prod needs the last
// two), and optionally the carried state s_{k+1} = sum_n c_n phi_n of a time
// block.  Every column's products are accumulated by a fixed set of
// threads in FP64 (column = thread % R, since the strip width is a multiple
// of 256 and R a power of two dividing it), reduced per workgroup in a fixed
// order and written as one record per tile; no atomics, so the result is the
// same on every run.
#include <algorithm>

#include "csp_internal.h"

namespace csp {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };

template <typename C> __device__ inline C czero() { C z; z.x = 0; z.y = 0; return z; }

template <typename T, int V, bool MOM>
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

  // Moment epilogue state (compiled out of the plain variant).
  const C* psi0 = static_cast<const C*>(I.psi0);
  C* carry = static_cast<C*>(I.carry_out);
  const bool dpsi = MOM && st.dot_psi0;
  const bool dself = MOM && st.dot_self;
  const int cmode = MOM ? st.carry_mode : 0;
  const T cc0r = static_cast<T>(st.cc0[0]), cc0i = static_cast<T>(st.cc0[1]);
  const T ccr = static_cast<T>(st.cc[0]), cci = static_cast<T>(st.cc[1]);
  double acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = 0.0;
  C p0v[MOM ? V : 1], p0n[MOM ? V : 1], cyv[MOM ? V : 1], cyn[MOM ? V : 1];
  if constexpr (MOM) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      p0v[v] = (dpsi && valid[v]) ? psi0[y0 * rowlen + ev[v]] : czero<C>();
      cyv[v] = (cmode == 2 && valid[v]) ? carry[y0 * rowlen + ev[v]] : czero<C>();
    }
  }

  int sm = 0, sc = 1, sp = 2;
  for (int64_t y = y0; y < y1; ++y) {
    const bool more = y + 1 < y1;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      prvn[v] = (more && st.has_prev && valid[v]) ? prev[(y + 1) * rowlen + ev[v]] : czero<C>();
      epn[v] = (more && eps && valid[v]) ? eps[(y + 1) * I.opr + xv[v]] : T(0);
    }
    if constexpr (MOM) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        p0n[v] = (more && dpsi && valid[v]) ? psi0[(y + 1) * rowlen + ev[v]] : czero<C>();
        cyn[v] = (more && cmode == 2 && valid[v]) ? carry[(y + 1) * rowlen + ev[v]] : czero<C>();
      }
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
      if constexpr (MOM) {
        const double ox = o.x, oy = o.y, cx = c.x, cy = c.y;
        if (dpsi) {
          const double px = p0v[v].x, py = p0v[v].y;
          acc[0] = fma(px, ox, fma(py, oy, acc[0]));      // conj(psi0) out
          acc[1] = fma(px, oy, fma(-py, ox, acc[1]));
          acc[2] = fma(px, cx, fma(py, cy, acc[2]));      // conj(psi0) cur
          acc[3] = fma(px, cy, fma(-py, cx, acc[3]));
        }
        if (dself) {
          acc[4] = fma(ox, ox, fma(oy, oy, acc[4]));      // |out|^2
          acc[6] = fma(ox, cx, fma(oy, cy, acc[6]));      // conj(out) cur
          acc[7] = fma(ox, cy, fma(-oy, cx, acc[7]));
        }
        if (cmode) {
          C b;
          if (cmode == 1) {
            b.x = cc0r * c.x - cc0i * c.y;
            b.y = cc0r * c.y + cc0i * c.x;
          } else {
            b = cyv[v];
          }
          b.x += ccr * o.x - cci * o.y;
          b.y += ccr * o.y + cci * o.x;
          carry[y * rowlen + ev[v]] = b;
        }
      }
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
    if constexpr (MOM) {
#pragma unroll
      for (int v = 0; v < V; ++v) { p0v[v] = p0n[v]; cyv[v] = cyn[v]; }
    }
  }

  if constexpr (MOM) {
    if (dpsi || dself) {
      // Workgroup sum per column in a fixed order: thread r, r + R, ...
      __syncthreads();                 // the LDS ring is no longer read
      double* red = reinterpret_cast<double*>(smem);
#pragma unroll
      for (int k = 0; k < 8; ++k) red[k * kSpmmThreads + tid] = acc[k];
      __syncthreads();
      double* part = st.partial + (((int64_t)st.mom_slot * st.total_tiles + tile) * 4) *
                                      (int64_t)st.rmax * 2;
      for (int q = tid; q < 8 * R; q += kSpmmThreads) {
        const int k = q / R, r = q - k * R;
        double sum = 0.0;
        for (int t = r; t < kSpmmThreads; t += R) sum += red[k * kSpmmThreads + t];
        // record layout [kind][rmax][re, im]
        part[((k >> 1) * st.rmax + r) * 2 + (k & 1)] = sum;
      }
    }
  }
}

hipError_t launch_spmm(bool fp64, int vec, bool mom, const SpmmInst* d_inst, int n_inst,
                       const SpmmStep& st, hipStream_t s) {
  if (st.total_tiles <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(st.total_tiles)), block(kSpmmThreads);
  const size_t csz = fp64 ? sizeof(double2) : sizeof(float2);
  size_t lds = 3 * (size_t)(kSpmmThreads * vec + 2 * st.halo) * csz;
  if (mom) lds = std::max(lds, sizeof(double) * 8 * kSpmmThreads);
#define CSP_SPMM_CASE(T, V, M)                                                              \
  hipLaunchKernelGGL((k_spmm<T, V, M>), grid, block, lds, s, d_inst, n_inst, st)
  if (fp64) {
    switch (vec * 2 + (mom ? 1 : 0)) {
      case 2: CSP_SPMM_CASE(double, 1, false); break;
      case 3: CSP_SPMM_CASE(double, 1, true); break;
      case 4: CSP_SPMM_CASE(double, 2, false); break;
      case 5: CSP_SPMM_CASE(double, 2, true); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (vec * 2 + (mom ? 1 : 0)) {
      case 2: CSP_SPMM_CASE(float, 1, false); break;
      case 3: CSP_SPMM_CASE(float, 1, true); break;
      case 4: CSP_SPMM_CASE(float, 2, false); break;
      case 5: CSP_SPMM_CASE(float, 2, true); break;
      case 8: CSP_SPMM_CASE(float, 4, false); break;
      case 9: CSP_SPMM_CASE(float, 4, true); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef CSP_SPMM_CASE
  return hipGetLastError();
}

}  // namespace csp
