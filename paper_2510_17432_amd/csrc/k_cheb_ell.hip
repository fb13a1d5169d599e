// Chebyshev recursion (amxsy of Sec. II.B) for a Hamiltonian given
// explicitly in ELL form, for matrices of any density D_H (Sec. II.B: the
// paper's speedups are measured at D_H = 60..230, where the recursion
// dominates):
//   phi_{n+1} = 2 H~ phi_n - phi_{n-1},  H~ = (H - H0)/|H|,
// one step per launch (the neighbours of a row are arbitrary, so no
// temporal blocking).
//
// Layout.  The matrix is stored in slices of 128 rows, [N/128][D][128]
// (sliced ELL): entry k of the 128 rows of a slice is contiguous, and a
// slice's D entries follow each other, so the wave that owns a slice
// streams one contiguous block.  A row with fewer than D entries, and every
// row s >= N of the last slice, is padded with a valid column index and a
// zero value, so the entry loop has no branch.  At D_H in the tens to hundreds
// the matrix is most of the bytes of a step (D (4 + sizeof(T)) per row
// against 24..48 B per row and column for the three vectors), so the kernel
// is built around streaming it once per step:
//   - a wave owns a slice (128 rows) and CT columns of a column group: the
//     matrix entries loaded once serve the gathers of all CT columns;
//   - lane l owns rows l and l + 64 of the slice, so every matrix load and
//     every gather of the 64 lanes covers consecutive elements;
//   - the index and value loads of the next U entries are issued after the
//     gathers of the current ones, so the HBM latency of the matrix stream
//     overlaps the (mostly cache-hit) vector gathers.
//   - complex64: the gathers read an orbital-major copy of phi_n ("shadow",
//     [pairs][N][2] complex values), so one 16-byte load per row serves two
//     columns; each step writes phi_{n+1}'s copy beside its column-major
//     store, into the other of two buffers.  A block's first step (phi_0
//     new) and an odd last column gather from the column-major vectors.
// Measured on MI355X (D_H = 233, 4.76 M rows, two columns): the matrix
// stream alone runs at the read ceiling (about 6 TB/s); the gathers set the
// pace.  The cost follows both the load instructions and the cache lines
// they touch: two columns in one 16-byte load (1 KB per wave, 8 lines) beat
// two 8-byte loads (2 x 4 lines) by 15-19 % in isolation, whereas four
// columns in two 16-byte loads (16 half-used lines each) lost to four
// 8-byte loads; interleaved row pairs, deeper pipelines and other block
// sizes changed nothing.
// Moment epilogue and carried state as the stencil kernel: one record of 8
// FP64 sums per (column, 128-row chunk), record index column-major.
#include <type_traits>

#include "csp_internal.h"

#define CSP_GLOBAL __attribute__((address_space(1)))

namespace csp {
namespace ell {

// complex values as element-aligned 2-vectors (a column of a group starts
// at c N values)
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2), aligned(4)));
typedef double f64x2 __attribute__((ext_vector_type(2), aligned(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct vt;
template <> struct vt<float> { using v2 = f32x2; };
template <> struct vt<double> { using v2 = f64x2; };

// the complex values of a lane's two rows in one column
template <typename T> struct pair2 { T r0, i0, r1, i1; };

// one complex value
template <typename T>
__device__ __forceinline__ typename vt<T>::v2 ld_c(const CSP_GLOBAL T* p) {
  return *reinterpret_cast<const CSP_GLOBAL typename vt<T>::v2*>(p);
}
template <typename T>
__device__ __forceinline__ void st_c(CSP_GLOBAL T* p, T re, T im, bool nt) {
  typename vt<T>::v2 t;
  t.x = re;
  t.y = im;
  if (nt) __builtin_nontemporal_store(t, reinterpret_cast<CSP_GLOBAL typename vt<T>::v2*>(p));
  else *reinterpret_cast<CSP_GLOBAL typename vt<T>::v2*>(p) = t;
}
// rows s0, s1 of one column (zeros for rows past N)
template <typename T>
__device__ __forceinline__ pair2<T> ld_rows(const CSP_GLOBAL T* col, int64_t s0, int64_t s1,
                                            bool v0, bool v1) {
  pair2<T> r{T(0), T(0), T(0), T(0)};
  if (v0) {
    const typename vt<T>::v2 a = ld_c(col + 2 * s0);
    r.r0 = a.x;
    r.i0 = a.y;
  }
  if (v1) {
    const typename vt<T>::v2 b = ld_c(col + 2 * s1);
    r.r1 = b.x;
    r.i1 = b.y;
  }
  return r;
}
template <typename T>
__device__ __forceinline__ void st_rows(CSP_GLOBAL T* col, int64_t s0, int64_t s1, bool v0, bool v1,
                                        const pair2<T>& v, bool nt) {
  if (v0) st_c(col + 2 * s0, v.r0, v.i0, nt);
  if (v1) st_c(col + 2 * s1, v.r1, v.i1, nt);
}

// Matrix entries per pipelined block and blocks the matrix loads run ahead
// (measured on MI355X at D_H = 233: FP32 4 entries, FP64 2 entries, one
// block ahead; deeper pipelines bought nothing, as the gathers rather than
// the index latency set the pace).
template <typename T> constexpr int ell_block() { return sizeof(T) == 4 ? 4 : 2; }
constexpr int PD = 1;

// The matrix is read once per step and never again before every other
// cache line of the step has passed: non-temporal loads, which leave the
// L2 to the gathered vectors (each vector value is gathered D times).
template <typename V>
__device__ __forceinline__ V ld_stream(const CSP_GLOBAL V* p) {
  return __builtin_nontemporal_load(p);
}

// One wave: rows chunk * 128 + lane and + 64 of the CT columns c0 .. c0 +
// CT - 1 of its group (c0 even when CT >= 2).  SH: the gathers of the column
// pairs (c0 + 2p, c0 + 2p + 1) read the orbital-major shadow of phi_n, one
// 16-byte load per row for both columns (complex64 only); an odd last column
// is gathered from its column-major vector.
template <typename T, int CT, bool MOM, bool CARRY, bool SH>
__device__ __forceinline__ void ell_wave(const ChebInst& I, int64_t chunk, int c0, int lane,
                                         const ChebStep& st) {
  using V2 = typename vt<T>::v2;
  constexpr int U = ell_block<T>();
  static_assert(!SH || std::is_same<T, float>::value, "shadows hold complex64 values");
  constexpr int NP = SH ? CT / 2 : 0;               // column pairs read from the shadow
  const int64_t N = I.N;
  const int D = I.ell_D;
  const int64_t s0 = chunk * 128 + lane, s1 = s0 + 64;
  const bool v0 = s0 < N, v1 = s1 < N;

  const int64_t cofs = 2 * (int64_t)c0 * N;         // column c0 of the group, in T units
  CSP_GLOBAL T* base = (CSP_GLOBAL T*)(I.base);
  const CSP_GLOBAL T* cur =
      (st.slot_cur < 0 ? (const CSP_GLOBAL T*)(I.src) : base + 2 * (int64_t)st.slot_cur * I.slot_stride) +
      cofs;
  const CSP_GLOBAL T* prev = st.first ? nullptr : base + 2 * (int64_t)st.slot_prev * I.slot_stride + cofs;
  CSP_GLOBAL T* outv =
      st.slot_out[0] >= 0 ? base + 2 * (int64_t)st.slot_out[0] * I.slot_stride + cofs : nullptr;
  CSP_GLOBAL T* copyv =
      st.copy_slot >= 0 ? base + 2 * (int64_t)st.copy_slot * I.slot_stride + cofs : nullptr;

  // entry k of rows s0, s1: slice start + k * 128 + row inside the slice
  const int64_t mofs = chunk * D * 128 + lane;
  const CSP_GLOBAL int32_t* cp = (const CSP_GLOBAL int32_t*)(I.ell_col) + mofs;
  const CSP_GLOBAL T* vp = (const CSP_GLOBAL T*)(I.ell_val) + mofs;
  auto ld_entry = [&](int k, i32x2& j, V2& v) {
    const int64_t e = (int64_t)k * 128;
    j.x = ld_stream(cp + e);
    j.y = ld_stream(cp + e + 64);
    v.x = ld_stream(vp + e);
    v.y = ld_stream(vp + e + 64);
  };

  // sum_k H_{s,j_k} phi_n[j_k] for rows s0, s1 of each column
  T ar0[CT], ai0[CT], ar1[CT], ai1[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) ar0[c] = ai0[c] = ar1[c] = ai1[c] = T(0);

  const CSP_GLOBAL T* xcol[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) xcol[c] = cur + 2 * (int64_t)c * N;
  const CSP_GLOBAL f32x4* xsh[NP > 0 ? NP : 1];
#pragma unroll
  for (int q = 0; q < NP; ++q)
    xsh[q] = (const CSP_GLOBAL f32x4*)(I.ell_shadow) +
             ((int64_t)st.sh_in * I.sh_pairs + c0 / 2 + q) * N;
  // phi_n[j] of column c for rows s0 (j.x) and s1 (j.y)
  auto gather = [&](const i32x2 j, V2 (&xu)[CT][2]) {
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      if (c < 2 * NP) {
        if (c % 2 == 0) {
          const f32x4 p = xsh[c / 2][j.x], q = xsh[c / 2][j.y];
          xu[c][0].x = p.x;
          xu[c][0].y = p.y;
          xu[c + 1][0].x = p.z;
          xu[c + 1][0].y = p.w;
          xu[c][1].x = q.x;
          xu[c][1].y = q.y;
          xu[c + 1][1].x = q.z;
          xu[c + 1][1].y = q.w;
        }
      } else {
        xu[c][0] = ld_c(xcol[c] + 2 * (int64_t)j.x);
        xu[c][1] = ld_c(xcol[c] + 2 * (int64_t)j.y);
      }
    }
  };

  auto fma_rows = [&](int c, const V2 v, const V2 x0, const V2 x1) {
    ar0[c] = fma(v.x, x0.x, ar0[c]);
    ai0[c] = fma(v.x, x0.y, ai0[c]);
    ar1[c] = fma(v.y, x1.x, ar1[c]);
    ai1[c] = fma(v.y, x1.y, ai1[c]);
  };

  if constexpr (SH) {
    // Two columns per 16-byte gather: a plain loop unrolled by 4 lets the
    // compiler batch the loads of four entries (measured faster here than
    // the explicit pipeline below: 1.92 against 1.95 ms per step at D_H =
    // 233, 1.93 against 2.06 ms at D_H = 61 with 10 columns).
#pragma unroll 4
    for (int k = 0; k < D; ++k) {
      i32x2 j;
      V2 v;
      ld_entry(k, j, v);
      V2 x[CT][2];
      gather(j, x);
#pragma unroll
      for (int c = 0; c < CT; ++c) fma_rows(c, v, x[c][0], x[c][1]);
    }
  } else {
    // Blocks of U entries, the matrix loads running PD blocks ahead of the
    // gathers.  In each block the gathers (which need the block's indices)
    // are issued first and the matrix loads of block kb + PD U after them;
    // loads complete in issue order, so waiting for the gathers waits for the
    // matrix loads issued before them (blocks up to kb + (PD - 1) U) and
    // leaves the newest in flight.
    const int Dm = D - D % U;
    i32x2 jb[PD][U];
    V2 vb[PD][U];
    if (Dm > 0) {
#pragma unroll
      for (int d = 0; d < PD; ++d) {
        const int k0 = d * U < Dm ? d * U : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) ld_entry(k0 + u, jb[d][u], vb[d][u]);
      }
    }
    for (int kb = 0; kb < Dm; kb += U) {
      V2 x[U][CT][2];
#pragma unroll
      for (int u = 0; u < U; ++u) gather(jb[0][u], x[u]);
      // block kb + PD U (past the end: the current block again, cached, no branch)
      const int kn = kb + PD * U < Dm ? kb + PD * U : kb;
      i32x2 jn[U];
      V2 vn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) ld_entry(kn + u, jn[u], vn[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < CT; ++c) fma_rows(c, vb[0][u], x[u][c][0], x[u][c][1]);
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          jb[d][u] = jb[d + 1][u];
          vb[d][u] = vb[d + 1][u];
        }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        jb[PD - 1][u] = jn[u];
        vb[PD - 1][u] = vn[u];
      }
    }
    for (int k = Dm; k < D; ++k) {
      i32x2 j;
      V2 v;
      ld_entry(k, j, v);
      V2 x[CT][2];
      gather(j, x);
#pragma unroll
      for (int c = 0; c < CT; ++c) fma_rows(c, v, x[c][0], x[c][1]);
    }
  }

  const T scale = st.first ? T(0.5) : T(1);
  const T alpha = scale * static_cast<T>(I.alpha);
  const T beta0 = scale * static_cast<T>(I.beta0);
  double rec[CT][8];
  pair2<T> outs[CT];

#pragma unroll
  for (int c = 0; c < CT; ++c) {
#pragma unroll
    for (int q = 0; q < 8; ++q) rec[c][q] = 0.0;
    if (!v0) continue;
    const int64_t co = 2 * (int64_t)c * N;          // column c0 + c, in T units
    // phi_n and phi_{n-1} at rows s0, s1 (zeros past N)
    const pair2<T> cv = ld_rows<T>(cur + co, s0, s1, v0, v1);
    const pair2<T> pv = prev ? ld_rows<T>(prev + co, s0, s1, v0, v1)
                             : pair2<T>{T(0), T(0), T(0), T(0)};
    pair2<T> o;
    o.r0 = alpha * ar0[c] + (beta0 * cv.r0 - pv.r0);
    o.i0 = alpha * ai0[c] + (beta0 * cv.i0 - pv.i0);
    o.r1 = v1 ? alpha * ar1[c] + (beta0 * cv.r1 - pv.r1) : T(0);
    o.i1 = v1 ? alpha * ai1[c] + (beta0 * cv.i1 - pv.i1) : T(0);
    outs[c] = o;
    if (outv) st_rows<T>(outv + co, s0, s1, v0, v1, o, true);
    if (copyv) st_rows<T>(copyv + co, s0, s1, v0, v1, cv, true);

    if constexpr (CARRY) {
      if (st.carry_mode && I.carry) {
        const T c0r = static_cast<T>(st.cc0[0]), c0i = static_cast<T>(st.cc0[1]);
        const T c1r = static_cast<T>(st.ccl[0][0]), c1i = static_cast<T>(st.ccl[0][1]);
        CSP_GLOBAL T* carry = (CSP_GLOBAL T*)(I.carry) + cofs + co;
        pair2<T> b;
        if (st.carry_mode == 1) {
          b.r0 = c0r * cv.r0 - c0i * cv.i0;
          b.i0 = c0r * cv.i0 + c0i * cv.r0;
          b.r1 = c0r * cv.r1 - c0i * cv.i1;
          b.i1 = c0r * cv.i1 + c0i * cv.r1;
        } else {
          b = ld_rows<T>(carry, s0, s1, v0, v1);
        }
        b.r0 += c1r * o.r0 - c1i * o.i0;
        b.i0 += c1r * o.i0 + c1i * o.r0;
        b.r1 += c1r * o.r1 - c1i * o.i1;
        b.i1 += c1r * o.i1 + c1i * o.r1;
        st_rows<T>(carry, s0, s1, v0, v1, b, false);
      }
    }

    if constexpr (MOM) {
      if (st.dot_psi0) {
        const pair2<T> q =
            ld_rows<T>((const CSP_GLOBAL T*)(I.psi0) + cofs + co, s0, s1, v0, v1);
        rec[c][0] = ((double)q.r0 * o.r0 + (double)q.i0 * o.i0) +
                    ((double)q.r1 * o.r1 + (double)q.i1 * o.i1);
        rec[c][1] = ((double)q.r0 * o.i0 - (double)q.i0 * o.r0) +
                    ((double)q.r1 * o.i1 - (double)q.i1 * o.r1);
        rec[c][2] = ((double)q.r0 * cv.r0 + (double)q.i0 * cv.i0) +
                    ((double)q.r1 * cv.r1 + (double)q.i1 * cv.i1);
        rec[c][3] = ((double)q.r0 * cv.i0 - (double)q.i0 * cv.r0) +
                    ((double)q.r1 * cv.i1 - (double)q.i1 * cv.r1);
      }
      if (st.dot_self) {
        rec[c][4] = ((double)o.r0 * o.r0 + (double)o.i0 * o.i0) +
                    ((double)o.r1 * o.r1 + (double)o.i1 * o.i1);
        rec[c][6] = ((double)o.r0 * cv.r0 + (double)o.i0 * cv.i0) +
                    ((double)o.r1 * cv.r1 + (double)o.i1 * cv.i1);
        rec[c][7] = ((double)o.r0 * cv.i0 - (double)o.i0 * cv.r0) +
                    ((double)o.r1 * cv.i1 - (double)o.i1 * cv.r1);
      }
    }
  }

  // phi_{n+1} of the column pairs into the other shadow buffer, for the
  // next step's gathers (complex64 instances with a shadow)
  if constexpr (std::is_same<T, float>::value && CT >= 2) {
    if (st.sh_out >= 0 && I.ell_shadow && v0) {
#pragma unroll
      for (int q = 0; q < CT / 2; ++q) {
        CSP_GLOBAL f32x4* d = (CSP_GLOBAL f32x4*)(I.ell_shadow) +
                              ((int64_t)st.sh_out * I.sh_pairs + c0 / 2 + q) * N;
        const pair2<T>& a0 = outs[2 * q];
        const pair2<T>& a1 = outs[2 * q + 1];
        d[s0] = f32x4{a0.r0, a0.i0, a1.r0, a1.i0};
        if (v1) d[s1] = f32x4{a0.r1, a0.i1, a1.r1, a1.i1};
      }
    }
  }

  if constexpr (MOM) {
    if (st.dot_psi0 || st.dot_self) {
      // records [kind][re, im]: <psi0|out>, <psi0|cur>, <out|out>, <out|cur>,
      // one per column, summed over the wave by a fixed butterfly
#pragma unroll
      for (int c = 0; c < CT; ++c) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          double x = rec[c][q];
#pragma unroll
          for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
          rec[c][q] = x;
        }
        if (lane < 8) {
          double val = rec[c][0];
#pragma unroll
          for (int q = 1; q < 8; ++q) val = lane == q ? rec[c][q] : val;
          const int64_t item = I.item0 + (int64_t)(c0 + c) * I.n_segs + chunk;
          st.partial[((int64_t)st.mom_slot * st.total_items + item) * 8 + lane] = val;
        }
      }
    }
  }
}

// Waves of CT columns; the last tile of a group whose size is not a
// multiple of CT runs a body for its own column count (wave-uniform
// branch), so no wave gathers for a column it does not have.
template <typename T, int CT, bool MOM, bool CARRY, bool SH>
__global__ __launch_bounds__(256) void k_cheb_ell(const ChebInst* __restrict__ insts, int n_inst,
                                                  int64_t wave_lo, int64_t wave_hi, ChebStep st) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t w = wave_lo + xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= wave_hi) return;                         // a whole wave
  int ii = 0;
  while (ii + 1 < n_inst && w >= insts[ii + 1].wave0) ++ii;
  const ChebInst& I = insts[ii];
  const int64_t lw = w - I.wave0;
  const int n_tiles = (I.Rg + CT - 1) / CT;
  const int64_t chunk = lw / n_tiles;               // the slice of 128 rows
  const int c0 = static_cast<int>(lw - chunk * n_tiles) * CT;
  const int nc = I.Rg - c0 < CT ? I.Rg - c0 : CT;   // columns of this wave
  if (nc >= CT) {
    ell_wave<T, CT, MOM, CARRY, SH>(I, chunk, c0, lane, st);
  } else if constexpr (CT >= 2) {
    if (nc == 1) {
      ell_wave<T, 1, MOM, CARRY, false>(I, chunk, c0, lane, st);
    } else if constexpr (CT >= 4) {
      if (nc == 2)
        ell_wave<T, 2, MOM, CARRY, SH>(I, chunk, c0, lane, st);
      else
        ell_wave<T, 3, MOM, CARRY, SH>(I, chunk, c0, lane, st);
    }
  }
}

}  // namespace ell

// Up to four columns per wave in both precisions (measured on MI355X at
// D_H = 121 with 5 columns, complex128: 4.63 ms per step with two-column
// waves, 3.83 ms with four).
int ell_columns_per_wave(bool fp64, int Rg) {
  (void)fp64;
  int ct = 1;
  while (ct * 2 <= Rg && ct * 2 <= 4) ct *= 2;
  return ct;
}

hipError_t launch_cheb_ell(bool fp64, bool mom, bool carry, int ct, const ChebInst* d_inst,
                           int n_inst, int64_t wave_lo, int64_t wave_hi, const ChebStep& st,
                           hipStream_t s) {
  const int64_t n = wave_hi - wave_lo;
  if (n <= 0) return hipSuccess;
  if (st.nlev != 1 || (carry && !mom)) return hipErrorInvalidValue;
  if (ct != 1 && ct != 2 && ct != 4) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(ceil_div(n, 4))), block(256);
  // complex64 waves of two or four columns gather phi_n from its shadow
  // when the previous step wrote one
  const bool sh = !fp64 && ct >= 2 && st.sh_in >= 0;
#define CSP_ELL(T, CT, M, CY, SH)                                                                 \
  hipLaunchKernelGGL((ell::k_cheb_ell<T, CT, M, CY, SH>), grid, block, 0, s, d_inst, n_inst,      \
                     wave_lo, wave_hi, st)
#define CSP_ELL_CT(T, M, CY, SH)                \
  do {                                          \
    if (ct == 1) CSP_ELL(T, 1, M, CY, false);   \
    else if (ct == 2) CSP_ELL(T, 2, M, CY, SH); \
    else CSP_ELL(T, 4, M, CY, SH);              \
  } while (0)
  if (fp64) {
    if (carry) CSP_ELL_CT(double, true, true, false);
    else if (mom) CSP_ELL_CT(double, true, false, false);
    else CSP_ELL_CT(double, false, false, false);
  } else if (sh) {
    if (carry) CSP_ELL_CT(float, true, true, true);
    else if (mom) CSP_ELL_CT(float, true, false, true);
    else CSP_ELL_CT(float, false, false, true);
  } else {
    if (carry) CSP_ELL_CT(float, true, true, false);
    else if (mom) CSP_ELL_CT(float, true, false, false);
    else CSP_ELL_CT(float, false, false, false);
  }
#undef CSP_ELL_CT
#undef CSP_ELL
  return hipGetLastError();
}

// Gershgorin row bound of an explicit matrix (H0 = 0): max_s sum_k |val_sk|,
// each row summed in k order with plain additions (padding values are 0);
// one maximum per block.
__global__ void k_ell_gershgorin(int64_t N, int D, const double* __restrict__ val,
                                 double* __restrict__ partial) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    const double* row = val + (s >> 7) * D * 128 + (s & 127);
    double r = 0.0;
    for (int k = 0; k < D; ++k) r = r + fabs(row[(int64_t)k * 128]);
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

hipError_t launch_ell_gershgorin(int64_t N, int D, const double* d_val, double* d_partial,
                                 int n_partial, hipStream_t s) {
  hipLaunchKernelGGL(k_ell_gershgorin, dim3(n_partial), dim3(256), 0, s, N, D, d_val, d_partial);
  return hipGetLastError();
}

}  // namespace csp
