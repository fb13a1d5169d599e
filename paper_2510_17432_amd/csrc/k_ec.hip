// Electronic conductivity (EC section) by the moment-based concurrent form
// EC-Concurrent-M:
//   C(t, E) = <psi|J e^{iHt} J|Psi(E)> / |<psi|Psi(E)>|        (Eq. dc_corr)
//   m_n(E)  = <J psi|T_n(H~)|J Psi(E)>                          (Eq. dc_mom)
//   C(t, E) = e^{iH0 t} sum_n c_n(t~)^* m_n(E) / |<psi|Psi(E)>|
//   sigma(E) = D(E)/A int_0^T Re[e^{-iEt} C(t, E)] dt             (Eq. DC)
// with J = i [H, X_alpha].  The recursion of J psi is the ordinary
// Chebyshev kernel writing into a ring of orders; here are the current
// operator, the moment contraction of a chunk of orders against all n_E
// bras J Psi(E) at once, and the FP64 assembly.
//
// Moment contraction (FP32 path).  For a chunk of up to 128 orders,
//   mu_n(E) = <X_E|phi_n> = sum_s conj(X_E[s]) phi_n[s],  X_E = J Psi(E),
// is a GEMM reducing over the orbitals.  Viewing a complex vector as 2N
// floats (re, im), Re mu = phi' . X' and Im mu = phi' . Z' with Z = i X
// (floats (-Xi, Xr)), so both are real GEMMs [orders x 2N] x [2N x energies]
// on v_mfma_f32_32x32x16_bf16 with split hi + lo bf16 operands (three
// products each) and FP32 accumulation: A = 32 orders x 8 orbitals (each
// lane 4 consecutive complex values of one order), B = 8 orbitals x 32
// energies (4 consecutive values of one bra; Z formed in registers).  A
// workgroup owns one column, one slice of orbitals and one tile of 32
// energies (grid y); it stages 32-orbital tiles of the chunk's orders and
// of the bras in LDS with coalesced loads (one ring slot per order, so a
// load instruction whose lanes each read a different order would touch 32
// pages), and each of its four waves multiplies one tile of 32 orders.
// The FP32 tiles of all slices are summed in FP64 in slice order (no
// atomics).  The FP64 path stages the same tiles and forms the sums with
// FMAs.  m_n = conj(mu_n).
#include "csp_internal.h"

namespace csp {

typedef __bf16 ebf16x8 __attribute__((ext_vector_type(8)));
typedef float ef32x16 __attribute__((ext_vector_type(16)));
typedef float ef32x2 __attribute__((ext_vector_type(2), aligned(8)));
typedef __attribute__((address_space(1))) ef32x2 gef2;

// ------------------------------------------------------------------ current operator
// Bond vectors r_j - r_s of the neighbours of orbital s (stencil
// conventions of the lattice; a bond closing a periodic boundary has the
// vector of its kind).  (J psi)_s = i t sum_nb v_alpha psi_j.
template <typename T>
__global__ void k_current_stencil(Geom g, double t, int alpha, const T* __restrict__ in,
                                  T* __restrict__ out, int64_t nvec) {
  const int64_t total = nvec * g.N;
  const double r3h = 0.86602540378443864676;   // sqrt(3) / 2
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = i / g.N, s = i - v * g.N;
    const T* x = in + 2 * v * g.N;
    int64_t nb[3];
    double vv[3];
    int n = 0;
    auto add = [&](int64_t j, double vx, double vy) {
      nb[n] = j;
      vv[n] = alpha == 0 ? vx : vy;
      ++n;
    };
    if (g.kind == CSP_CHAIN) {
      const int64_t ix = s;
      if (ix + 1 < g.Lx) add(s + 1, 1.0, 0.0);
      else if (g.px) add(s + 1 - g.Lx, 1.0, 0.0);
      if (ix >= 1) add(s - 1, -1.0, 0.0);
      else if (g.px) add(s + g.Lx - 1, -1.0, 0.0);
    } else if (g.kind == CSP_SQUARE) {
      const int64_t iy = s / g.Lx, ix = s - iy * g.Lx;
      // four neighbours: summed directly (the table above holds three)
      double acc_r = 0.0, acc_i = 0.0;
      auto take = [&](int64_t j, double w) {
        acc_r += w * (double)x[2 * j];
        acc_i += w * (double)x[2 * j + 1];
      };
      const double wx = alpha == 0 ? 1.0 : 0.0, wy = alpha == 1 ? 1.0 : 0.0;
      if (ix + 1 < g.Lx) take(s + 1, wx);
      else if (g.px) take(s + 1 - g.Lx, wx);
      if (ix >= 1) take(s - 1, -wx);
      else if (g.px) take(s + g.Lx - 1, -wx);
      if (iy + 1 < g.Ly) take(s + g.Lx, wy);
      else if (g.py) take(ix, wy);
      if (iy >= 1) take(s - g.Lx, -wy);
      else if (g.py) take(s + (g.Ly - 1) * g.Lx, -wy);
      // i t (acc_r + i acc_i)
      out[2 * i] = static_cast<T>(-t * acc_i);
      out[2 * i + 1] = static_cast<T>(t * acc_r);
      continue;
    } else {
      const int64_t cell = s >> 1, iy = cell / g.Lx, ix = cell - iy * g.Lx;
      if ((s & 1) == 0) {                          // A
        add(s + 1, r3h, 0.5);
        if (ix >= 1) add(2 * (cell - 1) + 1, -r3h, 0.5);
        else if (g.px) add(2 * (iy * g.Lx + g.Lx - 1) + 1, -r3h, 0.5);
        if (iy >= 1) add(2 * (cell - g.Lx) + 1, 0.0, -1.0);
        else if (g.py) add(2 * ((g.Ly - 1) * g.Lx + ix) + 1, 0.0, -1.0);
      } else {                                     // B
        add(s - 1, -r3h, -0.5);
        if (ix + 1 < g.Lx) add(2 * (cell + 1), r3h, -0.5);
        else if (g.px) add(2 * (iy * g.Lx), r3h, -0.5);
        if (iy + 1 < g.Ly) add(2 * (cell + g.Lx), 0.0, 1.0);
        else if (g.py) add(2 * ix, 0.0, 1.0);
      }
    }
    double acc_r = 0.0, acc_i = 0.0;
    for (int k = 0; k < n; ++k) {
      acc_r += vv[k] * (double)x[2 * nb[k]];
      acc_i += vv[k] * (double)x[2 * nb[k] + 1];
    }
    out[2 * i] = static_cast<T>(-t * acc_i);
    out[2 * i + 1] = static_cast<T>(t * acc_r);
  }
}

hipError_t launch_current_stencil(bool fp64, const Geom& g, double t, int alpha, const void* in,
                                  void* out, int64_t nvec, hipStream_t s) {
  const int64_t total = nvec * g.N;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 65536);
  if (fp64)
    hipLaunchKernelGGL(k_current_stencil<double>, dim3(grid), dim3(256), 0, s, g, t, alpha,
                       static_cast<const double*>(in), static_cast<double*>(out), nvec);
  else
    hipLaunchKernelGGL(k_current_stencil<float>, dim3(grid), dim3(256), 0, s, g, t, alpha,
                       static_cast<const float*>(in), static_cast<float*>(out), nvec);
  return hipGetLastError();
}

// Explicit matrix in slices of 128 rows ([N/128][D][128]); padding entries
// have the value 0.  (J psi)_s = i sum_k H_{s,j_k} (x_{j_k} - x_s) psi_{j_k}.
// A thread owns row s of up to 8 vectors, so each matrix entry and its
// displacement serve 8 gathers.
constexpr int kCurVec = 8;

template <typename T>
__global__ void k_current_ell(int64_t N, int D, const int32_t* __restrict__ col,
                              const double* __restrict__ val, const double* __restrict__ pos,
                              double box, int alpha, const T* __restrict__ in,
                              T* __restrict__ out, int64_t nvec) {
  const int64_t n_vt = (nvec + kCurVec - 1) / kCurVec;
  const int64_t total = n_vt * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t vt = i / N, s = i - vt * N;
    const int64_t v0 = vt * kCurVec;
    const int nv = nvec - v0 < kCurVec ? static_cast<int>(nvec - v0) : kCurVec;
    const int64_t base = (s >> 7) * (int64_t)D * 128 + (s & 127);
    const double xs = pos[2 * s + alpha];
    double acc_r[kCurVec], acc_i[kCurVec];
#pragma unroll
    for (int v = 0; v < kCurVec; ++v) acc_r[v] = acc_i[v] = 0.0;
    for (int k = 0; k < D; ++k) {
      const int64_t j = col[base + (int64_t)k * 128];
      const double h = val[base + (int64_t)k * 128];
      double d = pos[2 * j + alpha] - xs;
      if (box > 0.0) d -= box * rint(d / box);
      const double w = h * d;
#pragma unroll
      for (int v = 0; v < kCurVec; ++v) {
        if (v < nv) {
          const T* x = in + 2 * ((v0 + v) * N + j);
          acc_r[v] += w * (double)x[0];
          acc_i[v] += w * (double)x[1];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < kCurVec; ++v) {
      if (v < nv) {
        T* o = out + 2 * ((v0 + v) * N + s);
        o[0] = static_cast<T>(-acc_i[v]);
        o[1] = static_cast<T>(acc_r[v]);
      }
    }
  }
}

hipError_t launch_current_ell(bool fp64, int64_t N, int D, const int32_t* ell_col,
                              const double* ell_v64, const double* pos, double box, int alpha,
                              const void* in, void* out, int64_t nvec, hipStream_t s) {
  const int64_t total = ceil_div(nvec, kCurVec) * N;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(total, 256), 65536);
  if (fp64)
    hipLaunchKernelGGL(k_current_ell<double>, dim3(grid), dim3(256), 0, s, N, D, ell_col,
                       ell_v64, pos, box, alpha, static_cast<const double*>(in),
                       static_cast<double*>(out), nvec);
  else
    hipLaunchKernelGGL(k_current_ell<float>, dim3(grid), dim3(256), 0, s, N, D, ell_col,
                       ell_v64, pos, box, alpha, static_cast<const float*>(in),
                       static_cast<float*>(out), nvec);
  return hipGetLastError();
}

// ------------------------------------------------------------------ norms
// Sum of 256 FP64 values of a workgroup: wave butterfly, then the four wave
// sums in order.
__device__ inline double block_sum256(double x, double* red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// workgroup per (c, e)
template <typename T>
__global__ __launch_bounds__(256) void k_ec_norm(int64_t N, int Rg, int nE,
                                                 const T* __restrict__ psi,
                                                 const T* __restrict__ qe,
                                                 double* __restrict__ nrm, int q0) {
  __shared__ double red[4];
  const int c = blockIdx.x / nE, e = blockIdx.x - c * nE;
  const T* p = psi + 2 * (int64_t)c * N;
  const T* q = qe + 2 * ((int64_t)e * Rg + c) * N;
  double sr = 0.0, si = 0.0;
  for (int64_t s = threadIdx.x; s < N; s += 256) {
    const double pr = p[2 * s], pi = p[2 * s + 1], qr = q[2 * s], qi = q[2 * s + 1];
    sr += pr * qr + pi * qi;
    si += pr * qi - pi * qr;
  }
  sr = block_sum256(sr, red);
  si = block_sum256(si, red);
  if (threadIdx.x == 0) nrm[q0 + c * nE + e] = sqrt(sr * sr + si * si);
}

hipError_t launch_ec_norm(bool fp64, int64_t N, int Rg, int nE, const void* psi, const void* qe,
                          double* nrm, int q0, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_ec_norm<double>, dim3(Rg * nE), dim3(256), 0, s, N, Rg, nE,
                       static_cast<const double*>(psi), static_cast<const double*>(qe), nrm, q0);
  else
    hipLaunchKernelGGL(k_ec_norm<float>, dim3(Rg * nE), dim3(256), 0, s, N, Rg, nE,
                       static_cast<const float*>(psi), static_cast<const float*>(qe), nrm, q0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ moments, FP32
__device__ __forceinline__ void split8(const float (&f)[8], ebf16x8& hi, ebf16x8& lo) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const __bf16 h = static_cast<__bf16>(f[v]);
    hi[v] = h;
    lo[v] = static_cast<__bf16>(f[v] - static_cast<float>(h));
  }
}

typedef float ef32x4 __attribute__((ext_vector_type(4), aligned(8)));
typedef __attribute__((address_space(1))) ef32x4 gef4;
typedef float lf32x4 __attribute__((ext_vector_type(4)));

constexpr int kEcOrb = 32;           // orbitals per staged tile
constexpr int kEcLds = 2 * kEcOrb + 8;   // floats per LDS row (padded)

// Two complex values (orbitals o, o + 1) of a column, zeros past s_end.
__device__ __forceinline__ ef32x4 ld2c(const gef2* p, int64_t o, int64_t s_end, bool ok) {
  ef32x4 r = {0.f, 0.f, 0.f, 0.f};
  if (ok && o + 1 < s_end) {
    r = *reinterpret_cast<const gef4*>(p + o);
  } else if (ok && o < s_end) {
    const ef32x2 z = p[o];
    r.x = z.x;
    r.y = z.y;
  }
  return r;
}

// Workgroup -> (instance, column c, slice) and tile of 32 energies
// (grid y).  Per step of 32 orbitals the workgroup stages the 128 orders x
// 32 orbitals of the chunk and the 32 bras x 32 orbitals in LDS with
// coalesced loads (16 lanes read one 256-byte row), then wave w multiplies
// orders 32 w .. 32 w + 31 by the 32 bras in four MFMA k-steps of 8
// orbitals.  MFMA lane (il, h): A = order il, B = bra il, floats
// 16 kk + 8 h .. + 7 of the staged row (orbitals 8 kk + 4 h .. + 3);
// accumulator v = (order 8 (v / 4) + 4 h + v % 4, energy il).
__global__ __launch_bounds__(256) void k_ec_moments_f32(const EcInst* __restrict__ insts,
                                                        EcArgs a) {
  __shared__ __align__(16) float sa[128 * kEcLds];
  __shared__ __align__(16) float sb[32 * kEcLds];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(tid >> 6));
  const int il = lane & 31, h = lane >> 5;
  // logical workgroup (slice, energy tile), the tiles of a slice adjacent:
  // they land on one XCD at the same time and stream the same orders, which
  // the second and later tiles find in that XCD's L2
  const int n_et = (a.nE + 31) / 32;
  const int64_t lwg = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t wg = lwg / n_et;
  const int e_tile = 32 * static_cast<int>(lwg - wg * n_et);
  int ii = 0;
  while (ii + 1 < a.n_inst && wg >= insts[ii + 1].wg0) ++ii;
  const EcInst& I = insts[ii];
  const int64_t wgl = wg - I.wg0;
  const int c = static_cast<int>(wgl / I.n_slices);
  const int sl = static_cast<int>(wgl - (int64_t)c * I.n_slices);
  const int64_t N = I.N;
  const int64_t s_beg = (int64_t)sl * I.slice_len;
  const int64_t s_end = s_beg + I.slice_len < N ? s_beg + I.slice_len : N;

  // staging roles: row (lane >> 4) of each group of four, 2 orbitals at 2 (lane & 15)
  const int sub = lane >> 4, ch = lane & 15;
  const gef2* arow[8];
  bool aok[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int r = wave * 32 + j * 4 + sub;
    aok[j] = r < a.n_cnt;
    arow[j] = (const gef2*)(I.slots) +
              (int64_t)ring_slot((a.n_lo + (aok[j] ? r : 0)) % a.S, a.S, a.G) * I.slot_stride +
              (int64_t)c * N;
  }
  const gef2* brow[2];
  bool bok[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int e = e_tile + (wave * 2 + j) * 4 + sub;
    bok[j] = e < a.nE;
    brow[j] = (const gef2*)(I.bra) + ((int64_t)(bok[j] ? e : 0) * I.Rg + c) * N;
  }
  ef32x4 ra[8], rb[2];
  auto fetch = [&](int64_t s) {
    const int64_t o = s + 2 * ch;
#pragma unroll
    for (int j = 0; j < 8; ++j) ra[j] = ld2c(arow[j], o, s_end, aok[j]);
#pragma unroll
    for (int j = 0; j < 2; ++j) rb[j] = ld2c(brow[j], o, s_end, bok[j]);
  };

  ef32x16 accR, accI;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    accR[v] = 0.f;
    accI[v] = 0.f;
  }
  const bool active = 32 * wave < a.n_cnt;           // wave-uniform
  if (s_beg < s_end) fetch(s_beg);
  for (int64_t s = s_beg; s < s_end; s += kEcOrb) {
    __syncthreads();                                 // previous tile consumed
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const ef32x4 v = ra[j];
      *reinterpret_cast<lf32x4*>(&sa[(wave * 32 + j * 4 + sub) * kEcLds + 4 * ch]) =
          lf32x4{v.x, v.y, v.z, v.w};
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const ef32x4 v = rb[j];
      *reinterpret_cast<lf32x4*>(&sb[((wave * 2 + j) * 4 + sub) * kEcLds + 4 * ch]) =
          lf32x4{v.x, v.y, v.z, v.w};
    }
    __syncthreads();
    if (s + kEcOrb < s_end) fetch(s + kEcOrb);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const float* pa = &sa[(wave * 32 + il) * kEcLds + 16 * kk + 8 * h];
        const float* pb = &sb[il * kEcLds + 16 * kk + 8 * h];
        const lf32x4 a0 = *reinterpret_cast<const lf32x4*>(pa);
        const lf32x4 a1 = *reinterpret_cast<const lf32x4*>(pa + 4);
        const lf32x4 b0 = *reinterpret_cast<const lf32x4*>(pb);
        const lf32x4 b1 = *reinterpret_cast<const lf32x4*>(pb + 4);
        const float fa[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const float fx[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
        // Z = i X: (-Xi, Xr) per complex value
        const float fz[8] = {-b0.y, b0.x, -b0.w, b0.z, -b1.y, b1.x, -b1.w, b1.z};
        ebf16x8 ah, al, xh, xl, zh, zl;
        split8(fa, ah, al);
        split8(fx, xh, xl);
        split8(fz, zh, zl);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, zh, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, zh, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, zl, accI, 0, 0, 0);
      }
    }
  }
  const int e = e_tile + il;
  if (active && e < a.nE) {
    gef2* out = (gef2*)(I.partial) + ((int64_t)c * I.n_slices + sl) * a.K * a.ldp;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 32 * wave + 8 * (v >> 2) + 4 * h + (v & 3);
      if (r < a.n_cnt) {
        ef32x2 o;
        o.x = accR[v];
        o.y = accI[v];
        out[(int64_t)r * a.ldp + e] = o;
      }
    }
  }
}

// ------------------------------------------------------------------ moments, FP64
// Workgroup per (instance, column, slice) and tile of up to 16 energies, or
// 24 when there are more than 16 (the energies split evenly over the tiles).
// Per step of 32 orbitals the chunk's 128 orders and the tile's bras are
// staged in LDS with coalesced loads (32 lanes read one 512-byte row);
// thread t accumulates energies t % 8 + 8 q (q < 2, or 3 with 24-energy
// tiles) against orders t / 8 + 32 p, p = 0..3, with FMAs: six LDS reads per
// eight complex products with two energies (the kernel is bound by LDS
// reads; one energy against eight orders took nine).
constexpr int kEc64Row = 33;         // complex values per LDS row (padded)

template <int NE>
__global__ __launch_bounds__(256) void k_ec_moments_f64(const EcInst* __restrict__ insts,
                                                        EcArgs a) {
  constexpr int NQ = NE > 16 ? 3 : NE > 8 ? 2 : 1;  // energies per thread
  constexpr int TILE = ec64_tile(NE);                 // energies a tile can hold
  __shared__ double2 sa[128 * kEc64Row];
  __shared__ double2 sb[8 * NQ * kEc64Row];
  const int tid = threadIdx.x;
  // logical workgroup (slice, energy tile), the tiles of a slice adjacent
  // (one XCD, the same orders at the same time: L2 hits after the first);
  // the energies split evenly over the tiles (49: 17 + 16 + 16)
  const int n_et = (a.nE + TILE - 1) / TILE;
  const int tw = (a.nE + n_et - 1) / n_et;
  const int64_t lwg = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t wg = lwg / n_et;
  const int e0 = tw * static_cast<int>(lwg - wg * n_et);
  int ii = 0;
  while (ii + 1 < a.n_inst && wg >= insts[ii + 1].wg0) ++ii;
  const EcInst& I = insts[ii];
  const int64_t wgl = wg - I.wg0;
  const int c = static_cast<int>(wgl / I.n_slices);
  const int sl = static_cast<int>(wgl - (int64_t)c * I.n_slices);
  const int64_t N = I.N;
  const int64_t s_beg = (int64_t)sl * I.slice_len;
  const int64_t s_end = s_beg + I.slice_len < N ? s_beg + I.slice_len : N;
  const int col = tid & 31, rsub = tid >> 5;        // staging: orbital col of row 8 j + rsub

  const double2* arow[16];
  bool aok[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int r = 8 * j + rsub;
    aok[j] = r < a.n_cnt;
    arow[j] = static_cast<const double2*>(I.slots) +
              (int64_t)ring_slot((a.n_lo + (aok[j] ? r : 0)) % a.S, a.S, a.G) * I.slot_stride +
              (int64_t)c * N;
  }
  const double2* brow[NQ];
  bool bok[NQ];
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    const int e = e0 + 8 * j + rsub;
    bok[j] = e < a.nE && 8 * j + rsub < tw;
    brow[j] = static_cast<const double2*>(I.bra) + ((int64_t)(bok[j] ? e : 0) * I.Rg + c) * N;
  }
  double2 ra[16], rb[NQ];
  auto fetch = [&](int64_t s) {
    const int64_t o = s + col;
    const bool in = o < s_end;
#pragma unroll
    for (int j = 0; j < 16; ++j) ra[j] = (aok[j] && in) ? arow[j][o] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < NQ; ++j) rb[j] = (bok[j] && in) ? brow[j][o] : make_double2(0.0, 0.0);
  };

  const int eq = tid & 7, og = tid >> 3;           // energies eq + 8 q, orders og + 32 p
  double sr[NQ][4], si[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) sr[q][p] = si[q][p] = 0.0;
  if (s_beg < s_end) fetch(s_beg);
  for (int64_t s = s_beg; s < s_end; s += 32) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) sa[(8 * j + rsub) * kEc64Row + col] = ra[j];
#pragma unroll
    for (int j = 0; j < NQ; ++j) sb[(8 * j + rsub) * kEc64Row + col] = rb[j];
    __syncthreads();
    if (s + 32 < s_end) fetch(s + 32);
    if (eq < NE) {
      for (int o = 0; o < 32; ++o) {
        double2 x[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) x[q] = sb[(eq + 8 * q) * kEc64Row + o];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const double2 f = sa[(og + 32 * p) * kEc64Row + o];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            sr[q][p] = fma(x[q].x, f.x, fma(x[q].y, f.y, sr[q][p]));
            si[q][p] = fma(x[q].x, f.y, fma(-x[q].y, f.x, si[q][p]));
          }
        }
      }
    }
  }
  double2* out = static_cast<double2*>(I.partial) + ((int64_t)c * I.n_slices + sl) * a.K * a.ldp;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = eq + 8 * q;
    if (e < tw && e0 + e < a.nE) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int r = og + 32 * p;
        if (r < a.n_cnt) out[(int64_t)r * a.ldp + e0 + e] = make_double2(sr[q][p], si[q][p]);
      }
    }
  }
}

// mu[n_lo + rel][q0 + c nE + e] = sum over slices (in order), FP64
template <typename P>
__global__ void k_ec_mu_finish(const EcInst* __restrict__ insts, EcArgs a) {
  const EcInst& I = insts[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)a.n_cnt * I.Rg * a.nE;
  if (t >= per) return;
  const int rel = static_cast<int>(t / ((int64_t)I.Rg * a.nE));
  const int rest = static_cast<int>(t - (int64_t)rel * I.Rg * a.nE);
  const int c = rest / a.nE, e = rest - c * a.nE;
  const P* part = static_cast<const P*>(I.partial);
  double sr = 0.0, si = 0.0;
  for (int sl = 0; sl < I.n_slices; ++sl) {
    const P* p = part + 2 * ((((int64_t)c * I.n_slices + sl) * a.K + rel) * a.ldp + e);
    sr += (double)p[0];
    si += (double)p[1];
  }
  double* m = a.mu + 2 * ((int64_t)(a.n_lo + rel) * a.ldmu + I.q0 + c * a.nE + e);
  m[0] = sr;
  m[1] = si;
}

hipError_t launch_ec_moments(bool fp64, const EcInst* d_inst, int n_inst, const EcArgs& a,
                             hipStream_t s) {
  const int tile = fp64 ? ec64_tile(a.nE) : 32;
  const int n_et = (int)ceil_div(a.nE, tile);
  if (a.n_cnt < 1 || a.n_cnt > a.K || a.K > 128 || a.nE < 1 || a.ldp != n_et * tile)
    return hipErrorInvalidValue;
  if (fp64) {
    int ne = 1;
    while (ne < std::min(a.nE, 16)) ne *= 2;
    if (a.nE > 16) ne = 24;
#define CSP_EC64(NE) \
  hipLaunchKernelGGL(k_ec_moments_f64<NE>, dim3(a.total_wg * n_et), dim3(256), 0, s, d_inst, a)
    switch (ne) {
      case 1: CSP_EC64(1); break;
      case 2: CSP_EC64(2); break;
      case 4: CSP_EC64(4); break;
      case 8: CSP_EC64(8); break;
      case 16: CSP_EC64(16); break;
      default: CSP_EC64(24); break;
    }
#undef CSP_EC64
  } else {
    hipLaunchKernelGGL(k_ec_moments_f32, dim3(a.total_wg * n_et), dim3(256), 0, s, d_inst, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_ec_mu_finish(bool fp64, const EcInst* d_inst, int n_inst, int rg_max,
                               const EcArgs& a, hipStream_t s) {
  const int64_t per = (int64_t)a.n_cnt * rg_max * a.nE;
  const dim3 grid((unsigned)ceil_div(per, 256), n_inst);
  if (fp64) hipLaunchKernelGGL(k_ec_mu_finish<double>, grid, dim3(256), 0, s, d_inst, a);
  else hipLaunchKernelGGL(k_ec_mu_finish<float>, grid, dim3(256), 0, s, d_inst, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ assembly
// out[(e (Nt+1) + j) R + r] = conj(G_j[r nE + e]) e^{i H0 j tau} / nrm[r nE + e]
__global__ void k_ec_finish(int Nt, int R, int nE, const double2* __restrict__ mu,
                            const double2* __restrict__ g, const double* __restrict__ nrm,
                            double H0, double tau, double2* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nE * (Nt + 1) * R;
  if (t >= total) return;
  const int r = static_cast<int>(t % R);
  const int64_t ej = t / R;
  const int j = static_cast<int>(ej % (Nt + 1));
  const int e = static_cast<int>(ej / (Nt + 1));
  const int q = r * nE + e;
  const double2 G = j == 0 ? mu[q] : g[(int64_t)j * R * nE + q];
  double sn, cn;
  sincos(H0 * ((double)j * tau), &sn, &cn);
  const double inv = 1.0 / nrm[q];
  // conj(G) (cn + i sn)
  out[t] = make_double2((G.x * cn + G.y * sn) * inv, (G.x * sn - G.y * cn) * inv);
}

hipError_t launch_ec_finish(int Nt, int R, int nE, const double* mu, const double* g,
                            const double* nrm, double H0, double tau, double* out, hipStream_t s) {
  const int64_t total = (int64_t)nE * (Nt + 1) * R;
  hipLaunchKernelGGL(k_ec_finish, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, Nt, R,
                     nE, reinterpret_cast<const double2*>(mu), reinterpret_cast<const double2*>(g),
                     nrm, H0, tau, reinterpret_cast<double2*>(out));
  return hipGetLastError();
}

// workgroup per (e, r): tau sum_j w_j Re[e^{-i E t_j} C_j] times D(E)/A
__global__ __launch_bounds__(256) void k_ec_sigma(int64_t Nt, int R, int nE,
                                                  const double2* __restrict__ corr,
                                                  const double* __restrict__ E,
                                                  const double* __restrict__ dA, double tau,
                                                  double* __restrict__ sigma) {
  __shared__ double red[4];
  const int e = blockIdx.x / R, r = blockIdx.x - e * R;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j <= Nt; j += 256) {
    const double2 C = corr[((int64_t)e * (Nt + 1) + j) * R + r];
    double sn, cn;
    sincos(E[e] * ((double)j * tau), &sn, &cn);
    const double w = (j == 0 || j == Nt) ? 0.5 : 1.0;
    acc += w * (C.x * cn + C.y * sn);              // Re[(cn - i sn) C]
  }
  acc = block_sum256(acc, red);
  if (threadIdx.x == 0) sigma[(int64_t)e * R + r] = (Nt == 0 ? 0.0 : dA[e] * tau * acc);
}

hipError_t launch_ec_sigma(int64_t Nt, int R, int nE, const double* corr, const double* E,
                           const double* dA, double tau, double* sigma, hipStream_t s) {
  hipLaunchKernelGGL(k_ec_sigma, dim3(nE * R), dim3(256), 0, s, Nt, R, nE,
                     reinterpret_cast<const double2*>(corr), E, dA, tau, sigma);
  return hipGetLastError();
}

}  // namespace csp
