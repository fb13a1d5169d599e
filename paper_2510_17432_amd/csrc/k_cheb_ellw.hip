// Chebyshev step of an explicit matrix in the windowed layout (amxsy of
// Sec. II.B, for matrices of any density D_H):
//   phi_{n+1} = 2 H~ phi_n - phi_{n-1},
// one step per launch.  The layout (built at lattice creation,
// ell_windows.cpp) groups the rows into slices of 128 that are compact in
// the matrix graph and lists, per slice, its window: the distinct columns
// its entries name.
//
// One workgroup of 128 threads owns a slice and a tile of CT columns of a
// column group.  It stages the slice's window of phi_n for its columns in
// LDS (one plane of W complex values per column, coalesced where the
// window's columns run consecutively), then thread t accumulates row t of
// the slice over its D entries, reading the matrix once (16-bit
// window-local columns and values in quads of four entries per load,
// non-temporal: 6 B per entry in complex64 and 10 B in complex128, against
// 8 and 12 B in the slice layout) and gathering every phi_n value from LDS
// instead of the caches.
// A slice whose window exceeds the LDS budget gathers from global memory
// with the entries' global columns.  Rows keep their index in every vector:
// thread t reads and writes row rows[t] of phi_n, phi_{n-1}, phi_{n+1},
// psi0 and the carried state (scattered within the slice's ball of rows).
// Moment epilogue and carried state as the other recursion kernels: one
// record of 8 FP64 sums per (column, slice), the two waves of the
// workgroup added in a fixed order.
#include <algorithm>
#include <type_traits>

#include "csp_internal.h"

#define CSP_GLOBAL __attribute__((address_space(1)))

namespace csp {
namespace ellw {

template <typename T> struct cplx {
  T x, y;
};
typedef float f32x2 __attribute__((ext_vector_type(2), aligned(8)));
typedef double f64x2 __attribute__((ext_vector_type(2), aligned(16)));
typedef float f32x4 __attribute__((ext_vector_type(4), aligned(16)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4), aligned(8)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4), aligned(16)));
template <typename T> struct vec2;
template <> struct vec2<float> { using type = f32x2; };
template <> struct vec2<double> { using type = f64x2; };

template <typename T>
__device__ __forceinline__ cplx<T> ld(const CSP_GLOBAL T* p) {
  const typename vec2<T>::type v = *reinterpret_cast<const CSP_GLOBAL typename vec2<T>::type*>(p);
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st(CSP_GLOBAL T* p, cplx<T> c, bool nt) {
  typename vec2<T>::type v;
  v.x = c.x;
  v.y = c.y;
  CSP_GLOBAL typename vec2<T>::type* q = reinterpret_cast<CSP_GLOBAL typename vec2<T>::type*>(p);
  if (nt) __builtin_nontemporal_store(v, q);
  else *q = v;
}

template <typename T, int CT, bool MOM, bool CARRY>
__global__ __launch_bounds__(128) void k_cheb_ellw(const ChebInst* __restrict__ insts, int n_inst,
                                                   int64_t wg_lo, int64_t wg_hi, ChebStep sp) {
  using C = cplx<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[2][CT][8];                  // record sums of the two waves
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int64_t L = wg_lo + xcd_remap(blockIdx.x, gridDim.x);
  if (L >= wg_hi) return;                           // the whole workgroup
  int ii = 0;
  while (ii + 1 < n_inst && L >= insts[ii + 1].wave0) ++ii;
  const ChebInst& I = insts[ii];
  const int64_t lw = L - I.wave0;
  // the group's columns in n_tiles tiles of as equal size as possible (the
  // first Rg mod n_tiles take one more): CT or CT - 1 columns each
  const int n_tiles = (I.Rg + CT - 1) / CT;
  const int64_t slice = lw / n_tiles;
  const int tile = static_cast<int>(lw - slice * n_tiles);
  const int tb = I.Rg / n_tiles, tr = I.Rg - tb * n_tiles;
  const int c0 = tile * tb + (tile < tr ? tile : tr);
  const int nc = tb + (tile < tr ? 1 : 0);          // columns of this tile
  const int64_t N = I.N;
  const int D = I.ell_D;
  const int32_t row = I.ellw_rows[slice * 128 + t];
  const bool valid = row >= 0;
  const int64_t woff = I.ellw_off[slice];
  const int64_t W = I.ellw_off[slice + 1] - woff;
  const bool staged = W > 0 && W <= I.ellw_lds_cap;   // uniform over the workgroup

  const int64_t cofs = 2 * (int64_t)c0 * N;         // column c0 of the group, in T units
  CSP_GLOBAL T* base = (CSP_GLOBAL T*)(I.base);
  const CSP_GLOBAL T* cur =
      (sp.slot_cur < 0 ? (const CSP_GLOBAL T*)(I.src) : base + 2 * (int64_t)sp.slot_cur * I.slot_stride) +
      cofs;
  const CSP_GLOBAL T* prev =
      sp.first ? nullptr : base + 2 * (int64_t)sp.slot_prev * I.slot_stride + cofs;
  CSP_GLOBAL T* outv =
      sp.slot_out[0] >= 0 ? base + 2 * (int64_t)sp.slot_out[0] * I.slot_stride + cofs : nullptr;
  CSP_GLOBAL T* copyv =
      sp.copy_slot >= 0 ? base + 2 * (int64_t)sp.copy_slot * I.slot_stride + cofs : nullptr;

  // ---- the window of phi_n, one plane of W complex values per column
  // ([nc][W]).  Lanes gather window positions that are close together (the
  // rows of a slice ascend and most matrices name neighbouring columns from
  // neighbouring rows), so with 8-byte planes they hit distinct banks; an
  // interleaved [W][nc] layout put every position with the same residue of
  // 32 / nc on the same banks and serialised the gathers.
  // Each thread loads four window positions of every column before it
  // stores them, so the loads of a thread are in flight together.
  const int Wi = static_cast<int>(W);
  C* win = reinterpret_cast<C*>(smem);
  auto stage = [&](auto nc_tag) {
    constexpr int NC = decltype(nc_tag)::value;
    const CSP_GLOBAL int32_t* wi = (const CSP_GLOBAL int32_t*)(I.ellw_idx) + woff;
    int w = t;
    for (; w + 3 * 128 < Wi; w += 4 * 128) {
      int64_t j[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = wi[w + u * 128];
      C x[4][NC];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) x[u][c] = ld<T>(cur + 2 * ((int64_t)c * N + j[u]));
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) win[c * Wi + w + u * 128] = x[u][c];
    }
    for (; w < Wi; w += 128) {
      const int64_t j = wi[w];
      C x[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) x[c] = ld<T>(cur + 2 * ((int64_t)c * N + j));
#pragma unroll
      for (int c = 0; c < NC; ++c) win[c * Wi + w] = x[c];
    }
    __syncthreads();
  };

  // ---- sum_k H_{row,j_k} phi_n[j_k] for the tile's columns; the entries
  // come in quads (4 indices and 4 values per load), so a thread keeps
  // several quads of the matrix stream in flight.  The loop is compiled for
  // a fixed column count (tiles of a group hold CT or CT - 1 columns): a
  // run-time count would put a branch around every gather and keep the
  // gathers of one entry from being issued together.
  T ar[CT], ai[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) ar[c] = ai[c] = T(0);
  const int D4 = (D + 3) / 4;
  const int64_t qofs = slice * D4 * 512 + 4 * t;    // quad 0 of this row
  const CSP_GLOBAL T* vp = (const CSP_GLOBAL T*)(I.ellw_val) + qofs;
  auto ld_vals = [&](int q, T (&v)[4]) {
    if constexpr (sizeof(T) == 4) {
      const f32x4 a = __builtin_nontemporal_load(
          reinterpret_cast<const CSP_GLOBAL f32x4*>(vp + (int64_t)q * 512));
      v[0] = a.x;
      v[1] = a.y;
      v[2] = a.z;
      v[3] = a.w;
    } else {
      const CSP_GLOBAL f64x2* p = reinterpret_cast<const CSP_GLOBAL f64x2*>(vp + (int64_t)q * 512);
      const f64x2 a = __builtin_nontemporal_load(p), b = __builtin_nontemporal_load(p + 1);
      v[0] = a.x;
      v[1] = a.y;
      v[2] = b.x;
      v[3] = b.y;
    }
  };
  // Entries of quads q .. q + NQ - 1 of the row: window-local indices (or
  // global columns) and values, loaded one group ahead of their use so the
  // matrix stream of the next group is in flight while the current one
  // gathers.  Quads past D4 are not loaded (they would belong to the next
  // slice, or lie past the matrix).
  constexpr int NQ = 2;
  auto accumulate = [&](auto nc_tag) {
    constexpr int NC = decltype(nc_tag)::value;
    if (staged) {
      stage(nc_tag);
      const CSP_GLOBAL u16x4* lp = reinterpret_cast<const CSP_GLOBAL u16x4*>(
          (const CSP_GLOBAL uint16_t*)(I.ellw_loc) + qofs);
      u16x4 la[NQ];
      T va[NQ][4];
#pragma unroll
      for (int p = 0; p < NQ; ++p)
        if (p < D4) {
          la[p] = __builtin_nontemporal_load(lp + (int64_t)p * 128);
          ld_vals(p, va[p]);
        }
#pragma unroll 1
      for (int q0 = 0; q0 < D4; q0 += NQ) {
        u16x4 lb[NQ];
        T vb[NQ][4];
#pragma unroll
        for (int p = 0; p < NQ; ++p)
          if (q0 + NQ + p < D4) {
            lb[p] = __builtin_nontemporal_load(lp + (int64_t)(q0 + NQ + p) * 128);
            ld_vals(q0 + NQ + p, vb[p]);
          }
#pragma unroll
        for (int p = 0; p < NQ; ++p) {
          if (q0 + p < D4) {
            const int li[4] = {la[p].x, la[p].y, la[p].z, la[p].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              C x[NC];
#pragma unroll
              for (int c = 0; c < NC; ++c) x[c] = win[c * Wi + li[e]];
#pragma unroll
              for (int c = 0; c < NC; ++c) {
                ar[c] = fma(va[p][e], x[c].x, ar[c]);
                ai[c] = fma(va[p][e], x[c].y, ai[c]);
              }
            }
          }
        }
#pragma unroll
        for (int p = 0; p < NQ; ++p) {
          la[p] = lb[p];
#pragma unroll
          for (int e = 0; e < 4; ++e) va[p][e] = vb[p][e];
        }
      }
    } else {
      // a window beyond the LDS budget: gather from the vectors, the NC x 4
      // values of a quad issued together
      const CSP_GLOBAL i32x4* gp = reinterpret_cast<const CSP_GLOBAL i32x4*>(
          (const CSP_GLOBAL int32_t*)(I.ellw_col) + qofs);
#pragma unroll 1
      for (int q = 0; q < D4; ++q) {
        const i32x4 j4 = __builtin_nontemporal_load(gp + (int64_t)q * 128);
        T v[4];
        ld_vals(q, v);
        const int64_t jj[4] = {j4.x, j4.y, j4.z, j4.w};
        C x[4][NC];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int c = 0; c < NC; ++c) x[e][c] = ld<T>(cur + 2 * ((int64_t)c * N + jj[e]));
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            ar[c] = fma(v[e], x[e][c].x, ar[c]);
            ai[c] = fma(v[e], x[e][c].y, ai[c]);
          }
      }
    }
  };
  if (nc == CT) {
    accumulate(std::integral_constant<int, CT>{});
  } else if (CT > 1 && nc == CT - 1) {
    accumulate(std::integral_constant<int, (CT > 1 ? CT - 1 : 1)>{});
  } else {
    // other counts (not produced by ellw_columns_per_group): a branch per
    // column
    const CSP_GLOBAL int32_t* gp = (const CSP_GLOBAL int32_t*)(I.ellw_col) + qofs;
    for (int q = 0; q < D4; ++q) {
      T v[4];
      ld_vals(q, v);
      for (int e = 0; e < 4; ++e) {
        const int64_t j = gp[(int64_t)q * 512 + e];
        for (int c = 0; c < nc; ++c) {
          const C x = ld<T>(cur + 2 * ((int64_t)c * N + j));
          ar[c] = fma(v[e], x.x, ar[c]);
          ai[c] = fma(v[e], x.y, ai[c]);
        }
      }
    }
  }

  // ---- phi_{n+1} = 2 H~ phi_n - phi_{n-1} of row `row`, epilogues
  const T scale = sp.first ? T(0.5) : T(1);
  const T alpha = scale * static_cast<T>(I.alpha);
  const T beta0 = scale * static_cast<T>(I.beta0);
  const bool dots = MOM && (sp.dot_psi0 || sp.dot_self);
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    double rec[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (c < nc && valid) {
      const int64_t e = 2 * ((int64_t)c * N + row);
      const C cv = ld<T>(cur + e);
      const C pv = prev ? ld<T>(prev + e) : C{T(0), T(0)};
      C o;
      o.x = alpha * ar[c] + (beta0 * cv.x - pv.x);
      o.y = alpha * ai[c] + (beta0 * cv.y - pv.y);
      if (outv) st<T>(outv + e, o, true);
      if (copyv) st<T>(copyv + e, cv, true);
      if constexpr (CARRY) {
        if (sp.carry_mode && I.carry) {
          const T c0r = static_cast<T>(sp.cc0[0]), c0i = static_cast<T>(sp.cc0[1]);
          const T c1r = static_cast<T>(sp.ccl[0][0]), c1i = static_cast<T>(sp.ccl[0][1]);
          CSP_GLOBAL T* cy = (CSP_GLOBAL T*)(I.carry) + cofs + e;
          C b;
          if (sp.carry_mode == 1) {
            b.x = c0r * cv.x - c0i * cv.y;
            b.y = c0r * cv.y + c0i * cv.x;
          } else {
            b = ld<T>(cy);
          }
          b.x += c1r * o.x - c1i * o.y;
          b.y += c1r * o.y + c1i * o.x;
          st<T>(cy, b, false);
        }
      }
      if constexpr (MOM) {
        if (sp.dot_psi0) {
          const C q = ld<T>((const CSP_GLOBAL T*)(I.psi0) + cofs + e);
          rec[0] = (double)q.x * o.x + (double)q.y * o.y;
          rec[1] = (double)q.x * o.y - (double)q.y * o.x;
          rec[2] = (double)q.x * cv.x + (double)q.y * cv.y;
          rec[3] = (double)q.x * cv.y - (double)q.y * cv.x;
        }
        if (sp.dot_self) {
          rec[4] = (double)o.x * o.x + (double)o.y * o.y;
          rec[6] = (double)o.x * cv.x + (double)o.y * cv.y;
          rec[7] = (double)o.x * cv.y - (double)o.y * cv.x;
        }
      }
    }
    if constexpr (MOM) {
      if (dots) {
        // [kind][re, im]: <psi0|out>, <psi0|cur>, <out|out>, <out|cur>,
        // summed over the wave by a fixed butterfly
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double x = rec[q];
#pragma unroll
          for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
          if (lane == q) red[wave][c][q] = x;
        }
      }
    }
  }
  if constexpr (MOM) {
    if (dots) {
      __syncthreads();
      if (t < 8 * CT) {
        const int c = t >> 3, q = t & 7;
        if (c < nc) {
          const int64_t item = I.item0 + (int64_t)(c0 + c) * I.n_segs + slice;
          sp.partial[((int64_t)sp.mom_slot * sp.total_items + item) * 8 + q] =
              red[0][c][q] + red[1][c][q];
        }
      }
    }
  }
}

}  // namespace ellw

// Columns per workgroup (tile width CT): the group's columns in as few tiles
// as possible, split evenly (10 columns: two tiles of 5; 25: 7 + 6 + 6 + 6),
// so the matrix is read once per step per tile and every tile holds CT or
// CT - 1 columns.  A tile holds at most 8 columns, and at most as many as
// fit the LDS budget with a window of `window` positions.
int ellw_columns_per_group(bool fp64, int Rg, int64_t window) {
  const int64_t fit = kEllwLdsBytes / (std::max<int64_t>(window, 1) * (fp64 ? 16 : 8));
  const int cap = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(8, fit)));
  if (Rg < 1) return 1;
  const int tiles = (Rg + cap - 1) / cap;
  return (Rg + tiles - 1) / tiles;
}

hipError_t launch_cheb_ellw(bool fp64, bool mom, bool carry, int ct, int64_t lds_cap,
                            const ChebInst* d_inst, int n_inst, int64_t wg_lo, int64_t wg_hi,
                            const ChebStep& st, hipStream_t s) {
  const int64_t n = wg_hi - wg_lo;
  if (n <= 0) return hipSuccess;
  if (st.nlev != 1 || (carry && !mom)) return hipErrorInvalidValue;
  if (ct < 1 || ct > 8) return hipErrorInvalidValue;
  // LDS: the largest staged window of the run's instances times its
  // columns (lds_cap complex values)
  const size_t lds = (size_t)(lds_cap > 0 ? lds_cap : 1) * (fp64 ? 16 : 8);
  if (lds > (size_t)kEllwLdsBytes) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(n)), block(128);
#define CSP_ELLW(T, CT, M, CY) \
  hipLaunchKernelGGL((ellw::k_cheb_ellw<T, CT, M, CY>), grid, block, lds, s, d_inst, n_inst, wg_lo, wg_hi, st)
#define CSP_ELLW_CT(T, M, CY)      \
  do {                             \
    switch (ct) {                  \
      case 1: CSP_ELLW(T, 1, M, CY); break; \
      case 2: CSP_ELLW(T, 2, M, CY); break; \
      case 3: CSP_ELLW(T, 3, M, CY); break; \
      case 4: CSP_ELLW(T, 4, M, CY); break; \
      case 5: CSP_ELLW(T, 5, M, CY); break; \
      case 6: CSP_ELLW(T, 6, M, CY); break; \
      case 7: CSP_ELLW(T, 7, M, CY); break; \
      default: CSP_ELLW(T, 8, M, CY); break; \
    }                              \
  } while (0)
  if (fp64) {
    if (carry) CSP_ELLW_CT(double, true, true);
    else if (mom) CSP_ELLW_CT(double, true, false);
    else CSP_ELLW_CT(double, false, false);
  } else {
    if (carry) CSP_ELLW_CT(float, true, true);
    else if (mom) CSP_ELLW_CT(float, true, false);
    else CSP_ELLW_CT(float, false, false);
  }
#undef CSP_ELLW_CT
#undef CSP_ELLW
  return hipGetLastError();
}

}  // namespace csp
