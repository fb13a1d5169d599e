// Chebyshev recursion (amxsy of Sec. II.B), several steps per pass over
// memory:  phi_{n+l} = 2 H~ phi_{n+l-1} - phi_{n+l-2},  l = 1..nlev (nlev <=
// KT), with H~ = (H - H0)/|H| the rescaled lattice Hamiltonian of Sec. II.A
// applied as a stencil (no matrix in memory).  The first step of a time
// block is phi_1 = H~ phi_0.
//
// Layout.  A column group is stored column-major: column c of the group is
// one lattice vector, cstride values from the previous one, rows of `opr`
// values in the orbital order of the lattice and `pitch` values apart, so
// the in-row stencil neighbours are at +-1 and the vertical ones one row up
// or down.  The propagation forms pad rows whose length is not a multiple
// of 16 values to one, so that rows start 128-byte aligned (unaligned rows
// measured about a tenth slower); vectors the caller passes in are unpadded
// (pitch = opr).
//
// Work decomposition.  One wave (64 lanes) owns a strip of a row segment of
// one column and is independent of every other wave: no LDS, no barriers.
// Lane l holds the V consecutive positions p0 + V l .. p0 + V l + V - 1 of
// the strip, so a lane loads and stores V values with wide accesses and the
// whole wave touches 64 V consecutive values.  In-row neighbours are in the
// lane's own registers except at its two ends, which come from the adjacent
// lane by a DPP wavefront shift.  On the honeycomb lattice the vertical
// partner of an orbital is the other orbital of its (even, odd) pair one row
// up or down, which is in the same lane (V is even, p0 is even).
//
// The strip covers [os - MG, os - MG + 64 V); each level is valid one
// position further inside on each side than the one before, so after up to
// KT <= MG levels the owned positions [os, os + 64 V - 2 MG) are exact and
// neighbouring strips overlap by 2 MG positions that both compute (the
// redundant-margin form of temporal blocking).  MG is KT rounded up to a
// multiple of V, so every lane is either wholly owned or wholly margin.
// The wave marches down the rows y0 - nlev .. y1 + nlev - 1 of its segment
// keeping, for every level, the last three rows in registers; level l
// computes row r0 - l while level 0 loads row r0, so all levels advance
// together and only the owned rows [y0, y1) of every level are written.
// Per pass the memory traffic is one read of phi_n and phi_{n-1} (plus the
// 2 nlev-row segment margins) and one write per level kept, instead of two
// reads and one write per step.
//
// Moment variants (moment-based form of Sec. II.A).  MOM = kMomBra: for every
// level and owned value the epilogue accumulates <psi0|phi_{n+l}>,
// <psi0|phi_n> (first level only), <phi_{n+l}|phi_{n+l}> and
// <phi_{n+l}|phi_{n+l-1}> (the products of Eq. cheby_prod), each kind when
// its flag is set; it can also accumulate the carried state
// s_{k+1} = sum_n c_n phi_n of a time block.  MOM = kMomSelf (one block with
// bra = ket, Sec. III DOS-Concurrent-M): only |phi_{n+l}|^2 and
// Re <phi_{n+l}|phi_{n+l-1}>, the two products that give every moment above
// the first two; psi0 is not read and holds no registers.  Products over the
// V values of a lane are summed in the working precision, then in FP64 over
// rows; each wave reduces with a fixed butterfly and writes one record per
// level, so the sums do not depend on the run.
#pragma once

#include <type_traits>

#include "csp_internal.h"

#define CSP_GLOBAL __attribute__((address_space(1)))

namespace csp {
namespace cheb {

// moment epilogue of the recursion kernel (template argument MOM)
constexpr int kMomNone = 0;   // state form: no inner products
constexpr int kMomBra = 1;    // products with psi0 and the self products, by flags
constexpr int kMomSelf = 2;   // self products only (bra = ket, one block)

template <typename T> struct cx {
  T x, y;
};

typedef float f32x4u __attribute__((ext_vector_type(4), aligned(8)));
typedef float f32x2u __attribute__((ext_vector_type(2), aligned(4)));
typedef float f32x4w __attribute__((ext_vector_type(4), aligned(4)));
typedef double f64x2u __attribute__((ext_vector_type(2), aligned(8)));

// ---- V consecutive complex values of one lane (T units: 2 per value)
template <int V>
__device__ __forceinline__ void ldv(const CSP_GLOBAL float* p, cx<float> (&d)[V]) {
  const CSP_GLOBAL f32x4u* q = reinterpret_cast<const CSP_GLOBAL f32x4u*>(p);
#pragma unroll
  for (int k = 0; k < V / 2; ++k) {
    const f32x4u t = q[k];
    d[2 * k] = {t.x, t.y};
    d[2 * k + 1] = {t.z, t.w};
  }
}
template <int V>
__device__ __forceinline__ void stv(CSP_GLOBAL float* p, const cx<float> (&d)[V]) {
  CSP_GLOBAL f32x4u* q = reinterpret_cast<CSP_GLOBAL f32x4u*>(p);
#pragma unroll
  for (int k = 0; k < V / 2; ++k) {
    f32x4u t;
    t.x = d[2 * k].x;
    t.y = d[2 * k].y;
    t.z = d[2 * k + 1].x;
    t.w = d[2 * k + 1].y;
    q[k] = t;
  }
}
// Chebyshev vectors are written once and read back only after many other
// vectors have streamed through the caches: non-temporal stores.
#ifndef CSP_CHEB_NT
#define CSP_CHEB_NT 1
#endif
template <int V>
__device__ __forceinline__ void stv_nt(CSP_GLOBAL float* p, const cx<float> (&d)[V]) {
  CSP_GLOBAL f32x4u* q = reinterpret_cast<CSP_GLOBAL f32x4u*>(p);
#pragma unroll
  for (int k = 0; k < V / 2; ++k) {
    f32x4u t;
    t.x = d[2 * k].x;
    t.y = d[2 * k].y;
    t.z = d[2 * k + 1].x;
    t.w = d[2 * k + 1].y;
#if CSP_CHEB_NT
    __builtin_nontemporal_store(t, q + k);
#else
    q[k] = t;
#endif
  }
}
template <int V>
__device__ __forceinline__ void ldv(const CSP_GLOBAL double* p, cx<double> (&d)[V]) {
  const CSP_GLOBAL f64x2u* q = reinterpret_cast<const CSP_GLOBAL f64x2u*>(p);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const f64x2u t = q[v];
    d[v] = {t.x, t.y};
  }
}
template <int V>
__device__ __forceinline__ void stv(CSP_GLOBAL double* p, const cx<double> (&d)[V]) {
  CSP_GLOBAL f64x2u* q = reinterpret_cast<CSP_GLOBAL f64x2u*>(p);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    f64x2u t;
    t.x = d[v].x;
    t.y = d[v].y;
    q[v] = t;
  }
}
template <int V>
__device__ __forceinline__ void stv_nt(CSP_GLOBAL double* p, const cx<double> (&d)[V]) {
  CSP_GLOBAL f64x2u* q = reinterpret_cast<CSP_GLOBAL f64x2u*>(p);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    f64x2u t;
    t.x = d[v].x;
    t.y = d[v].y;
#if CSP_CHEB_NT
    __builtin_nontemporal_store(t, q + v);
#else
    q[v] = t;
#endif
  }
}
__device__ __forceinline__ cx<float> ld1(const CSP_GLOBAL float* p) {
  const f32x2u t = *reinterpret_cast<const CSP_GLOBAL f32x2u*>(p);
  return {t.x, t.y};
}
__device__ __forceinline__ void st1(CSP_GLOBAL float* p, cx<float> v) {
  f32x2u t;
  t.x = v.x;
  t.y = v.y;
  *reinterpret_cast<CSP_GLOBAL f32x2u*>(p) = t;
}
__device__ __forceinline__ cx<double> ld1(const CSP_GLOBAL double* p) {
  const f64x2u t = *reinterpret_cast<const CSP_GLOBAL f64x2u*>(p);
  return {t.x, t.y};
}
__device__ __forceinline__ void st1(CSP_GLOBAL double* p, cx<double> v) {
  f64x2u t;
  t.x = v.x;
  t.y = v.y;
  *reinterpret_cast<CSP_GLOBAL f64x2u*>(p) = t;
}
// V consecutive on-site energies
template <int V>
__device__ __forceinline__ void ldr(const CSP_GLOBAL float* p, float (&d)[V]) {
  if constexpr (V == 4) {
    const f32x4w t = *reinterpret_cast<const CSP_GLOBAL f32x4w*>(p);
    d[0] = t.x;
    d[1] = t.y;
    d[2] = t.z;
    d[3] = t.w;
  } else {
#pragma unroll
    for (int k = 0; k < V / 2; ++k) {
      const f32x2u t = reinterpret_cast<const CSP_GLOBAL f32x2u*>(p)[k];
      d[2 * k] = t.x;
      d[2 * k + 1] = t.y;
    }
  }
}
template <int V>
__device__ __forceinline__ void ldr(const CSP_GLOBAL double* p, double (&d)[V]) {
#pragma unroll
  for (int k = 0; k < V / 2; ++k) {
    const f64x2u t = reinterpret_cast<const CSP_GLOBAL f64x2u*>(p)[k];
    d[2 * k] = t.x;
    d[2 * k + 1] = t.y;
  }
}

// ---- wavefront shifts by one lane (DPP): lane l receives lane l - 1 (shr)
// or lane l + 1 (shl); the lane without a source receives 0.
__device__ __forceinline__ int dpp_shr1_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_shl1_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float shr1(float x) {
  return __builtin_bit_cast(float, dpp_shr1_i(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ float shl1(float x) {
  return __builtin_bit_cast(float, dpp_shl1_i(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double shr1(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)dpp_shr1_i((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_shr1_i((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double shl1(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)dpp_shl1_i((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_shl1_i((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int V, int KT> struct Shape {
  static constexpr int MG = ((KT + V - 1) / V) * V;   // margin positions per side
  static constexpr int OW = 64 * V - 2 * MG;          // owned positions per strip
};

// insts: the instances of this launch (consecutive items item_lo..item_hi-1).
template <typename T, int V, int KT, bool HONEY, bool EPS, int MOM, bool CARRY>
__global__ __launch_bounds__(256) void k_cheb(const ChebInst* __restrict__ insts, int n_inst,
                                              int64_t item_lo, int64_t item_hi, ChebStep st) {
  static_assert(V % 2 == 0, "lanes hold whole (even, odd) orbital pairs");
  static_assert(!CARRY || MOM == kMomBra, "the carried state comes with the bra moments");
  using C = cx<T>;
  using gT = CSP_GLOBAL T;
  constexpr int MG = Shape<V, KT>::MG;
  constexpr int OW = Shape<V, KT>::OW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t item = item_lo + xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (item >= item_hi) return;                     // a whole wave; no barriers below
  int ii = 0;
  while (ii + 1 < n_inst && item >= insts[ii + 1].item0) ++ii;
  const ChebInst& I = insts[ii];

  // ---- geometry of this work item (wave-uniform)
  const int64_t per_col = I.n_strips * I.n_segs;
  const int64_t local = item - I.item0;
  const int64_t col = local / per_col;
  const int64_t rem = local - col * per_col;
  const int64_t seg = rem / I.n_strips;
  const int64_t strip = rem - seg * I.n_strips;
  // positions, rows and offsets inside one lattice vector fit in 32 bits
  // (the host checks N < 2^31)
  const int opr = static_cast<int>(I.opr), Ly = static_cast<int>(I.Ly);
  const int os = static_cast<int>(strip) * OW;       // first owned position
  const int p0 = os - MG;                            // first position of the strip
  const bool fast = p0 >= 0 && p0 + 64 * V <= opr;   // no wrap, every position a site
  const int y0 = static_cast<int>(seg) * st.seg_rows;
  const int y1 = (y0 + st.seg_rows < Ly) ? y0 + st.seg_rows : Ly;
  const int nlev = st.nlev;
  const int py = I.py;
  const int64_t coff = 2 * col * I.cstride;          // column offset in T units

  // ---- per-lane positions
  const int lq = V * lane;
  const bool lane_own = lq >= MG && lq < MG + OW;
  int wpos[V];          // position inside the row (wrapped), valid when present
  bool pres[V];         // position is a site of the lattice
  bool own[V];          // position owned by this strip
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int p = p0 + lq + v;
    if (I.px) {
      int w = p % opr;
      if (w < 0) w += opr;
      wpos[v] = static_cast<int>(w);
      pres[v] = true;
    } else {
      pres[v] = p >= 0 && p < opr;
      wpos[v] = pres[v] ? static_cast<int>(p) : 0;
    }
    own[v] = lane_own && p >= 0 && p < opr;
  }
  auto row_of = [&](int r, bool& present) -> int {
    if (py) {
      while (r < 0) r += Ly;
      while (r >= Ly) r -= Ly;
      present = true;
      return r;
    }
    present = static_cast<unsigned>(r) < static_cast<unsigned>(Ly);
    return r;
  };
  // T offset of row rw (inside the lattice) in a column of the group's
  // vectors (rows pitch values apart); the on-site energies are packed
  const int64_t pitch = I.pitch;
  auto row_off = [&](int rw) -> int64_t { return 2 * static_cast<int64_t>(rw) * pitch; };

  gT* base = (gT*)(I.base);
  const gT* curv = (st.slot_cur < 0 ? (const gT*)(I.src)
                                    : base + 2 * (int64_t)st.slot_cur * I.slot_stride) + coff;
  const gT* prevv = st.first ? nullptr : base + 2 * (int64_t)st.slot_prev * I.slot_stride + coff;
  gT* copyv = st.copy_slot >= 0 ? base + 2 * (int64_t)st.copy_slot * I.slot_stride + coff
                                : nullptr;
  const gT* eps = (const gT*)(I.eps);
  const gT* psi0 = (const gT*)(I.psi0) + coff;
  gT* carry = CARRY && I.carry ? (gT*)(I.carry) + coff : nullptr;

  // output slot of each level (nullptr: not stored)
  gT* outv[KT];
#pragma unroll
  for (int l = 0; l < KT; ++l)
    outv[l] = st.slot_out[l] >= 0 ? base + 2 * (int64_t)st.slot_out[l] * I.slot_stride + coff
                                  : nullptr;

  // ---- register rows: rr[l][.] = the last three rows of level l.  With ROT
  // (the self-product kernel, whose pace is set by its instruction count)
  // the three slots rotate with the row index: before an iteration of phase
  // P = i mod 3, slot P holds the oldest row, P + 1 the middle and P + 2 the
  // newest; the iteration overwrites slot P with the new row, and the row
  // loop is unrolled by three so every slot index is a constant (rotation by
  // renaming, no register moves).  Without ROT every iteration moves the
  // rows down one slot and writes the new row into slot 2.  At 8 steps per
  // launch only the honeycomb lattice without on-site energies rotates:
  // unrolled, the others take 186-214 VGPRs (2 waves per SIMD instead of 3).
  constexpr bool ROT = MOM == kMomSelf && (KT <= 4 || (HONEY && !EPS));
  C rr[KT][3][V];
#pragma unroll
  for (int l = 0; l < KT; ++l)
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int v = 0; v < V; ++v) rr[l][k][v] = {T(0), T(0)};
  T er[EPS ? KT + 1 : 1][V];                         // on-site energies of rows r0 - k
#pragma unroll
  for (int k = 0; k < (EPS ? KT + 1 : 1); ++k)
#pragma unroll
    for (int v = 0; v < V; ++v) er[k][v] = T(0);

  // Moment sums.  kMomBra: quantity q = 5 (l - 1) + j for level l: j = 0, 1
  // <psi0|out>, 2 |out|^2, 3, 4 <out|cur>; q = 5 KT + 0, 1: <psi0|cur> of
  // the first level.  kMomSelf: q = 2 (l - 1) + j: j = 0 |out|^2, 1
  // Re <out|cur>.  sq holds this lane's working-precision sums of the last
  // rows; every kFlush rows each is summed over the wave and added in FP64
  // into accq of lane q.
  constexpr int kFlush = 16;
  constexpr int NQ = MOM == kMomBra ? 5 * KT + 2 : (MOM == kMomSelf ? 2 * KT : 1);
  T sq[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) sq[k] = T(0);
  double accq = 0.0;
  // psi0 rows r0 - k (moment epilogue)
  C pq[MOM == kMomBra ? KT + 1 : 1][V];
#pragma unroll
  for (int k = 0; k < (MOM == kMomBra ? KT + 1 : 1); ++k)
#pragma unroll
    for (int v = 0; v < V; ++v) pq[k][v] = {T(0), T(0)};
  const bool dots = MOM == kMomSelf || (MOM == kMomBra && (st.dot_psi0 || st.dot_self));
  const bool want_psi0 = MOM == kMomBra && st.dot_psi0;
  // carried state: partial sums of rows r0 - 1 - j (j < KT) in registers;
  // a row is read (carry_mode 2), completed and written once per launch
  const bool carry_on = CARRY && carry && st.carry_mode != 0;
  const bool carry_in = CARRY && carry && st.carry_mode == 2;
  C cpr[CARRY ? KT : 1][V];
#pragma unroll
  for (int k = 0; k < (CARRY ? KT : 1); ++k)
#pragma unroll
    for (int v = 0; v < V; ++v) cpr[k][v] = {T(0), T(0)};

  const T alpha = static_cast<T>(I.alpha);
  const T beta0 = static_cast<T>(I.beta0);
  const T oscale = static_cast<T>(I.onsite_scale);
  const bool vert = I.kind != CSP_CHAIN;
  // iterations: the segment's rows and nlev margin rows on each side; with
  // ROT rounded up to a multiple of three (the extra iterations compute rows
  // past the segment, which are neither stored nor summed, from loads of
  // rows that are inside the lattice or absent and read as zero)
  const int n_iter = ROT ? ((y1 - y0) + 2 * nlev + 2) / 3 * 3 : (y1 - y0) + 2 * nlev;
  const int rbase = y0 - nlev;                       // level-0 row of iteration 0

  // The row loop, compiled twice: FAST for strips inside the row (no wrap,
  // every position a site: wide loads and stores, whole lanes owned), and
  // the general form with per-position wrap, presence and ownership.
  auto run = [&](auto fast_tag) {
    constexpr bool FAST = decltype(fast_tag)::value;
    auto load_row = [&](const gT* vec, int r, C (&d)[V]) {
      bool rp;
      const int rw = row_of(r, rp);
      if (!rp) {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = {T(0), T(0)};
        return;
      }
      const gT* rowp = vec + row_off(rw);
      if constexpr (FAST) {
        ldv<V>(rowp + 2 * p0 + 2 * lq, d);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = pres[v] ? ld1(rowp + 2 * wpos[v]) : C{T(0), T(0)};
      }
    };
    auto load_eps = [&](int r, T (&d)[V]) {
      bool rp;
      const int rw = row_of(r, rp);
      if (!rp) {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = T(0);
        return;
      }
      const gT* rowp = eps + static_cast<int64_t>(rw) * opr;
      if constexpr (FAST) {
        ldr<V>(rowp + p0 + lq, d);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) d[v] = pres[v] ? rowp[wpos[v]] : T(0);
      }
    };
    // row rw must be inside [0, Ly); nt: non-temporal (Chebyshev slots)
    auto store_row = [&](gT* vec, int rw, const C (&o)[V], bool nt) {
      gT* rowp = vec + row_off(rw);
      if constexpr (FAST) {
        if (lane_own) {
          if (nt) stv_nt<V>(rowp + 2 * p0 + 2 * lq, o);
          else stv<V>(rowp + 2 * p0 + 2 * lq, o);
        }
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (own[v]) st1(rowp + 2 * wpos[v], o[v]);
      }
    };

    C ncur[V], nprev[V], pv[V], npq[V], ncar[V], car[V];
    T neps[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      nprev[v] = {T(0), T(0)};
      npq[v] = {T(0), T(0)};
      ncar[v] = {T(0), T(0)};
    }
    load_row(curv, rbase, ncur);
    if (prevv) load_row(prevv, rbase - 1, nprev);
    if constexpr (EPS) load_eps(rbase, neps);
    if (want_psi0) load_row(psi0, rbase, npq);
    if (carry_in) load_row(carry, rbase - nlev, ncar);

    int flush_in = kFlush;                           // rows left before the next flush
    // one iteration: level 0 takes row r0 = rbase + i, level l computes row
    // r0 - l; the phase selects the register slots.  STEADY iterations are
    // those in which all KT levels run and compute rows of the segment
    // (i in [2 KT, H + KT + 1) with nlev = KT): no level or row tests, and
    // those rows are inside the lattice.
    auto iter = [&](auto phase_tag, auto steady_tag, int i) {
      constexpr int P = ROT ? decltype(phase_tag)::value : 2;
      constexpr bool STEADY = decltype(steady_tag)::value;
      // slots after this iteration's new rows: oldest, middle, newest
      constexpr int SLO = (P + 1) % 3, SMI = (P + 2) % 3, SHI = P;
      // without ROT a level moves its rows down one slot before it writes
      // its new row
      auto shift_down = [&](int l) {
        if constexpr (!ROT) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            rr[l][0][v] = rr[l][1][v];
            rr[l][1][v] = rr[l][2][v];
          }
        }
      };
      const int r0 = rbase + i;
      shift_down(0);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        rr[0][SHI][v] = ncur[v];
        pv[v] = nprev[v];
      }
      if constexpr (EPS) {
#pragma unroll
        for (int k = KT; k >= 1; --k)
#pragma unroll
          for (int v = 0; v < V; ++v) er[k][v] = er[k - 1][v];
#pragma unroll
        for (int v = 0; v < V; ++v) er[0][v] = neps[v];
      }
      if constexpr (MOM == kMomBra) {
#pragma unroll
        for (int k = KT; k >= 1; --k)
#pragma unroll
          for (int v = 0; v < V; ++v) pq[k][v] = pq[k - 1][v];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          pq[0][v] = npq[v];
          car[v] = ncar[v];
        }
      }
      if constexpr (CARRY) {
#pragma unroll
        for (int k = KT - 1; k >= 1; --k)
#pragma unroll
          for (int v = 0; v < V; ++v) cpr[k][v] = cpr[k - 1][v];
#pragma unroll
        for (int v = 0; v < V; ++v) cpr[0][v] = {T(0), T(0)};
      }
      if (i + 1 < n_iter) {
        load_row(curv, r0 + 1, ncur);
        if (prevv) load_row(prevv, r0, nprev);
        if constexpr (EPS) load_eps(r0 + 1, neps);
        if (want_psi0) load_row(psi0, r0 + 1, npq);
        if (carry_in) load_row(carry, r0 + 1 - nlev, ncar);
      }
      // phi_n itself for the contraction (order 0 of a block)
      if (copyv && r0 >= y0 && r0 < y1) store_row(copyv, r0, rr[0][SHI], true);

#pragma unroll
      for (int l = 1; l <= KT; ++l) {
        if constexpr (!STEADY) {
          if (l > nlev || i < 2 * l) break;
        }
        const int r = r0 - l;
        bool rp = true;
        const int rw = STEADY ? r : row_of(r, rp);
        // With ROT a row outside the lattice (rp false) gets zero
        // coefficients: its phi_{n+l-1} and phi_{n+l-2} rows are zero, so o
        // is zero without a branch.  The other kernels branch (measured
        // faster there).
        const T scale = (ROT && !rp) ? T(0) : ((l == 1 && st.first) ? T(0.5) : T(1));
        const T as = scale * alpha, bs = scale * beta0, os_ = scale * oscale;
        // level l-1 rows r - 1, r, r + 1 and level l-2 row r (phi_{n+l-2})
        const C(&up)[V] = rr[l - 1][SLO];
        const C(&c)[V] = rr[l - 1][SMI];
        const C(&dn)[V] = rr[l - 1][SHI];
        C o[V];
        if (ROT || rp) {
          const T lx = shr1(c[V - 1].x), ly = shr1(c[V - 1].y);
          const T rx = shl1(c[0].x), ry = shl1(c[0].y);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            T nx = (v > 0 ? c[v - 1].x : lx) + (v < V - 1 ? c[v + 1].x : rx);
            T ny = (v > 0 ? c[v - 1].y : ly) + (v < V - 1 ? c[v + 1].y : ry);
            if constexpr (HONEY) {
              // even orbital: partner one row up (pos + 1); odd: one row down (pos - 1)
              if (v % 2 == 0) {
                nx += up[v + 1].x;
                ny += up[v + 1].y;
              } else {
                nx += dn[v - 1].x;
                ny += dn[v - 1].y;
              }
            } else {
              if (vert) {
                nx += up[v].x + dn[v].x;
                ny += up[v].y + dn[v].y;
              }
            }
            const C p = l == 1 ? pv[v] : rr[l - 2 >= 0 ? l - 2 : 0][SLO][v];
            T beta = bs;
            if constexpr (EPS) beta = bs + os_ * er[l][v];
            o[v].x = as * nx + (beta * c[v].x - p.x);
            o[v].y = as * ny + (beta * c[v].y - p.y);
          }
          if constexpr (!FAST) {
#pragma unroll
            for (int v = 0; v < V; ++v)
              if (!pres[v]) o[v] = {T(0), T(0)};
          }
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) o[v] = {T(0), T(0)};
        }
        if (l < KT) {
          shift_down(l);
#pragma unroll
          for (int v = 0; v < V; ++v) rr[l][SHI][v] = o[v];
        }
        if (STEADY || (r >= y0 && r < y1)) {
          if (outv[l - 1]) store_row(outv[l - 1], rw, o, true);
          if constexpr (MOM == kMomSelf) {
            const int q0 = 2 * (l - 1);
#pragma unroll
            for (int v = 0; v < V; ++v) {
              const bool w = FAST ? true : own[v];
              const C oo = w ? o[v] : C{T(0), T(0)};
              // one accumulating FMA per product
              sq[q0] += oo.x * oo.x;
              sq[q0] += oo.y * oo.y;
              sq[q0 + 1] += oo.x * c[v].x;
              sq[q0 + 1] += oo.y * c[v].y;
            }
          }
          if constexpr (MOM == kMomBra) {
            if (dots) {
              // values outside the owned positions take no part in the sums
              // (interior strips: whole lanes, masked when the sums are
              // flushed)
              C oo[V], cc[V];
#pragma unroll
              for (int v = 0; v < V; ++v) {
                const bool w = FAST ? true : own[v];
                oo[v] = w ? o[v] : C{T(0), T(0)};
                cc[v] = w ? c[v] : C{T(0), T(0)};
              }
              const C(&q)[V] = pq[l];
              const int q0 = 5 * (l - 1);
#pragma unroll
              for (int v = 0; v < V; ++v) {
                if (want_psi0) {
                  sq[q0] += q[v].x * oo[v].x;
                  sq[q0] += q[v].y * oo[v].y;
                  sq[q0 + 1] += q[v].x * oo[v].y;
                  sq[q0 + 1] -= q[v].y * oo[v].x;
                  if (l == 1) {
                    sq[5 * KT] += q[v].x * cc[v].x;
                    sq[5 * KT] += q[v].y * cc[v].y;
                    sq[5 * KT + 1] += q[v].x * cc[v].y;
                    sq[5 * KT + 1] -= q[v].y * cc[v].x;
                  }
                }
                if (st.dot_self) {
                  sq[q0 + 2] += oo[v].x * oo[v].x;
                  sq[q0 + 2] += oo[v].y * oo[v].y;
                  sq[q0 + 3] += oo[v].x * c[v].x;
                  sq[q0 + 3] += oo[v].y * c[v].y;
                  sq[q0 + 4] += oo[v].x * c[v].y;
                  sq[q0 + 4] -= oo[v].y * c[v].x;
                }
              }
            }
          }
          if constexpr (CARRY) {
            // level l adds c_{n+l} phi_{n+l} (and the first launch of a
            // block c_n phi_n) to the partial carried row r = r0 - l
            if (carry_on) {
              const T clr = static_cast<T>(st.ccl[l - 1][0]), cli = static_cast<T>(st.ccl[l - 1][1]);
              const T c0r = static_cast<T>(st.cc0[0]), c0i = static_cast<T>(st.cc0[1]);
#pragma unroll
              for (int v = 0; v < V; ++v) {
                C& b = cpr[l - 1][v];
                b.x += clr * o[v].x - cli * o[v].y;
                b.y += clr * o[v].y + cli * o[v].x;
                if (l == 1 && st.carry_mode == 1) {
                  b.x += c0r * c[v].x - c0i * c[v].y;
                  b.y += c0r * c[v].y + c0i * c[v].x;
                }
              }
              if (l == nlev) {                       // row r is complete
                C b[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                  b[v] = cpr[l - 1][v];
                  if (st.carry_mode == 2) {
                    b[v].x += car[v].x;
                    b[v].y += car[v].y;
                  }
                }
                store_row(carry, rw, b, false);
              }
            }
          }
        }
      }
      if constexpr (MOM != kMomNone) {
        if (dots && (--flush_in == 0 || i + 1 == n_iter)) {
          flush_in = kFlush;
#pragma unroll
          for (int k = 0; k < NQ; ++k) {
            T x = (FAST && !lane_own) ? T(0) : sq[k];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
            if (lane == k) accq += static_cast<double>(x);
            sq[k] = T(0);
          }
        }
      }
    };
    // iterations [i0, i1) (with ROT multiples of three)
    auto iter_range = [&](auto steady_tag, int i0, int i1) {
      if constexpr (ROT) {
#pragma unroll 1
        for (int i = i0; i < i1; i += 3) {
          iter(std::integral_constant<int, 0>{}, steady_tag, i);
          iter(std::integral_constant<int, 1>{}, steady_tag, i + 1);
          iter(std::integral_constant<int, 2>{}, steady_tag, i + 2);
        }
      } else {
#pragma unroll 1
        for (int i = i0; i < i1; ++i) iter(std::integral_constant<int, 2>{}, steady_tag, i);
      }
    };
    // steady iterations [ia, ib), rounded inwards to multiples of three
    // with ROT; the others take the general form.  Only the ROT kernels
    // have a steady form: in the others a second copy of the row loop costs
    // registers (occupancy) that the shorter scalar path does not repay.
    int ia = n_iter, ib = n_iter;
    if (nlev == KT) {
      ia = 2 * KT;
      ib = (y1 - y0) + KT + 1;
      if constexpr (ROT) {
        ia = (ia + 2) / 3 * 3;
        ib = ib / 3 * 3;
      }
      if (ib < ia) ib = ia;
    }
    if constexpr (ROT) {
      iter_range(std::false_type{}, 0, ia);
      iter_range(std::true_type{}, ia, ib);
      iter_range(std::false_type{}, ib, n_iter);
    } else {
      iter_range(std::false_type{}, 0, n_iter);
    }
  };
  if (fast) run(std::true_type{});
  else run(std::false_type{});

  if constexpr (MOM != kMomNone) {
    if (dots) {
      // one record of 8 doubles per level, [kind][re, im] with kinds
      // <psi0|out>, <psi0|cur> (first level only), <out|out>, <out|cur>
      // (kMomSelf: the real parts of the last two, zeros elsewhere);
      // lane m writes element m % 8 of level m / 8
      const int m = lane;
      const int l = m >> 3, slot = m & 7;
      int q = -1;
      if constexpr (MOM == kMomSelf) {
        if (slot == 4) q = 2 * l;
        else if (slot == 6) q = 2 * l + 1;
      } else {
        if (slot == 0 || slot == 1) q = 5 * l + slot;
        else if (slot == 4) q = 5 * l + 2;
        else if (slot == 6 || slot == 7) q = 5 * l + slot - 3;
        else if ((slot == 2 || slot == 3) && l == 0) q = 5 * KT + slot - 2;
      }
      const double val = __shfl(accq, q < 0 ? 0 : q);
      if (l < nlev && l < KT) {
        double* out = st.partial + (((int64_t)st.mom_slot * KT + l) * st.total_items + item) * 8;
        out[slot] = q < 0 ? 0.0 : val;
      }
    }
  }
}

}  // namespace cheb
}  // namespace csp

// Launch helper for one instantiation file: (V, KT) pairs are listed by the
// including file.
#define CSP_CHEB_LAUNCH(T, V, KT, MOM, CARRY)                                                  \
  do {                                                                                         \
    if (honey) {                                                                               \
      if (eps) hipLaunchKernelGGL((cheb::k_cheb<T, V, KT, true, true, MOM, CARRY>), grid,      \
                                  block, 0, s, d_inst, n_inst, item_lo, item_hi, st);          \
      else hipLaunchKernelGGL((cheb::k_cheb<T, V, KT, true, false, MOM, CARRY>), grid, block,  \
                              0, s, d_inst, n_inst, item_lo, item_hi, st);                     \
    } else {                                                                                   \
      if (eps) hipLaunchKernelGGL((cheb::k_cheb<T, V, KT, false, true, MOM, CARRY>), grid,     \
                                  block, 0, s, d_inst, n_inst, item_lo, item_hi, st);          \
      else hipLaunchKernelGGL((cheb::k_cheb<T, V, KT, false, false, MOM, CARRY>), grid, block, \
                              0, s, d_inst, n_inst, item_lo, item_hi, st);                     \
    }                                                                                          \
  } while (0)
