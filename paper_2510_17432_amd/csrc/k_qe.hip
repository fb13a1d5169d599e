// Quasi-eigenstates by the energy-based concurrent form (QE section,
// QE-Concurrent-E): the forward and backward time integrals of Eq. QE are
// merged into real, energy-dependent expansion coefficients (Eq. QE_coeff),
//   C_n(E) = tau [ delta_n0 + sum_{j >= 1, n <= N(j tau~)} 2 a_n(j tau~) Re((-i)^n e^{i E' t_j}) ],
// (c_n(-x) = conj(c_n(x)) turns the pair e^{iE't} c_n(t~) + e^{-iE't} c_n(-t~)
// into twice a real part), t_j = j tau, E' = E - H0, and the states are one
// contraction of the Chebyshev vectors of psi0,
//   Psi(E) = sum_{n=0}^{N(Nt tau~)} C_n(E) T_n(H~) psi0,
// over chunks of orders as the recursion produces them.
//
// FP32 path: the contraction runs on v_mfma_f32_32x32x16_bf16 with the
// split hi + lo bf16 operands of the state assembly, here with the
// coefficients as the A operand (32 energies x 16 orders) and the Chebyshev
// values as the B operand (16 orders x 32 values), so that the accumulator
// holds, per lane, one value and 16 energies and the states are stored with
// 256-byte coalesced writes.  The FP64 path multiplies complex128 values by
// the real coefficients with FMAs.  Coefficients are FP64 on the GPU, summed
// over j in a fixed order.
#include <type_traits>

#include "csp_internal.h"

namespace csp {

typedef __bf16 qbf16x8 __attribute__((ext_vector_type(8)));
typedef float qf32x16 __attribute__((ext_vector_type(16)));
typedef float qf32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) qf32x2 gq2;

struct QeBop {
  qbf16x8 hi;
  qbf16x8 lo;
};
// complex A operand of the state-based form: real and imaginary parts
struct QeBop4 {
  qbf16x8 rhi, rlo, ihi, ilo;
};
typedef unsigned short qu16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ qbf16x8 neg_bf16(qbf16x8 x) {
  qu16x8 u = __builtin_bit_cast(qu16x8, x);
  u ^= (unsigned short)0x8000;
  return __builtin_bit_cast(qbf16x8, u);
}

// cs[e][j-1] = (cos, sin) of (E_e - H0) j tau, j = 1..Nt
__global__ void k_qe_phase(int nE, int Nt, const double* __restrict__ E, double H0, double tau,
                           double2* __restrict__ cs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nE * Nt) return;
  const int e = (int)(i / Nt), j = (int)(i - (int64_t)e * Nt) + 1;
  const double th = (E[e] - H0) * ((double)j * tau);
  double sn, cn;
  sincos(th, &sn, &cn);
  cs[i] = make_double2(cn, sn);
}

// C[e][n], n = 0..nmax: thread per (n, e); a is the Bessel table of
// launch_bessel (row j-1 for x = j tau~), ntr its truncation orders.
__global__ void k_qe_coeffs(const double* __restrict__ a, int lda, const int32_t* __restrict__ ntr,
                            int Nt, int nE, const double2* __restrict__ cs, double tau, int nmax,
                            double* __restrict__ C) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (n > nmax || e >= nE) return;
  double s = 0.0;
  const double2* ce = cs + (int64_t)e * Nt;
  for (int j = 1; j <= Nt; ++j) {
    if (n > ntr[j - 1]) continue;                 // order n not yet in the expansion
    const double an = a[(int64_t)(j - 1) * lda + n];
    const double2 t = ce[j - 1];
    double r;
    switch (n & 3) {                              // Re((-i)^n e^{i th})
      case 0: r = t.x; break;
      case 1: r = t.y; break;
      case 2: r = -t.x; break;
      default: r = -t.y; break;
    }
    s = fma(2.0 * an, r, s);
  }
  C[(int64_t)e * (nmax + 1) + n] = tau * ((n == 0 ? 1.0 : 0.0) + s);
}

hipError_t launch_qe_coeffs(const double* d_a, int lda, const int32_t* d_ntr, int Nt, int nE,
                            const double* d_E, double H0, double tau, int nmax, double* d_cs,
                            double* d_C, hipStream_t s) {
  const int64_t np = (int64_t)nE * Nt;
  hipLaunchKernelGGL(k_qe_phase, dim3((unsigned)ceil_div(np, 256)), dim3(256), 0, s, nE, Nt, d_E,
                     H0, tau, reinterpret_cast<double2*>(d_cs));
  hipLaunchKernelGGL(k_qe_coeffs, dim3((unsigned)ceil_div(nmax + 1, 128), nE), dim3(128), 0, s,
                     d_a, lda, d_ntr, Nt, nE, reinterpret_cast<const double2*>(d_cs), tau, nmax,
                     d_C);
  return hipGetLastError();
}

// FP64 table coef[rel][e] = C[e][n_lo + rel] (imaginary part 0), e < B.
__global__ void k_pack_qe64(const double* __restrict__ C, int ldc, int nE, int B, int n_lo,
                            int n_cnt, double2* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cnt * B) return;
  const int rel = i / B, e = i - rel * B;
  coef[i] = make_double2(e < nE ? C[(int64_t)e * ldc + n_lo + rel] : 0.0, 0.0);
}

hipError_t launch_pack_qe64(const double* d_C, int ldc, int nE, int B, int n_lo, int n_cnt,
                            double* d_coef, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_qe64, dim3((unsigned)ceil_div(n_cnt * B, 256)), dim3(256), 0, s, d_C,
                     ldc, nE, B, n_lo, n_cnt, reinterpret_cast<double2*>(d_coef));
  return hipGetLastError();
}

// ------------------------------------------------------------------ state-based form
// QE-Concurrent-S: within a time block starting at t_{J0} from the carried
// states s^+ = psi(t_{J0}) and s^- = psi(-t_{J0}),
//   psi(+-t_{J0+j}) = sum_n c_n(j tau~)^{(*)} T_n(H~) s^+-,
// so the block's share of Eq. QE is sum_n C_n(E) T_n s^+ + conj(C_n(E)) T_n s^-
// with the complex block coefficients below (the j = 0 term tau psi0 rides
// on C_0 of the first block, tau/2 on each side), and the next carried states take the
// coefficients c_n(bk tau~) (and their conjugates) as one more row.
__global__ void k_qes_coeffs(const double* __restrict__ a, int lda, const int32_t* __restrict__ ntr,
                             int bk, int64_t J0, int nE, const double* __restrict__ E, double H0,
                             double tau, int first, int Nk, double2* __restrict__ C) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (n > Nk || e > nE) return;
  double2 out = make_double2(0.0, 0.0);
  if (e == nE) {                                  // carry row: c_n(bk tau~)
    if (n <= ntr[bk - 1]) {
      const double an = a[(int64_t)(bk - 1) * lda + n];
      switch (n & 3) {                            // (-i)^n an
        case 0: out = make_double2(an, 0.0); break;
        case 1: out = make_double2(0.0, -an); break;
        case 2: out = make_double2(-an, 0.0); break;
        default: out = make_double2(0.0, an); break;
      }
    }
  } else {
    double sr = 0.0, si = 0.0;
    for (int j = 1; j <= bk; ++j) {
      if (n > ntr[j - 1]) continue;
      const double an = a[(int64_t)(j - 1) * lda + n];
      double sn, cn;
      sincos((E[e] - H0) * ((double)(J0 + j) * tau), &sn, &cn);
      double xr, xi;                              // (-i)^n (cn + i sn)
      switch (n & 3) {
        case 0: xr = cn; xi = sn; break;
        case 1: xr = sn; xi = -cn; break;
        case 2: xr = -cn; xi = -sn; break;
        default: xr = -sn; xi = cn; break;
      }
      sr = fma(an, xr, sr);
      si = fma(an, xi, si);
    }
    // j = 0: (1/2)(psi0 + psi0), half on the forward and half on the backward side
    out = make_double2(tau * ((first && n == 0 ? 0.5 : 0.0) + sr), tau * si);
  }
  C[(int64_t)e * (Nk + 1) + n] = out;
}

hipError_t launch_qes_coeffs(const double* d_a, int lda, const int32_t* d_ntr, int bk,
                             int64_t J0, int nE, const double* d_E, double H0, double tau,
                             int first, int Nk, double* d_C, hipStream_t s) {
  hipLaunchKernelGGL(k_qes_coeffs, dim3((unsigned)ceil_div(Nk + 1, 128), nE + 1), dim3(128), 0, s,
                     d_a, lda, d_ntr, bk, J0, nE, d_E, H0, tau, first, Nk,
                     reinterpret_cast<double2*>(d_C));
  return hipGetLastError();
}

// entry (kb, lane): row il of orders n_lo + 16 kb + 8 h .. + 7, split hi + lo
__global__ void k_pack_qes(const double2* __restrict__ C, int ldc, int rows, int n_lo, int n_cnt,
                           QeBop4* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n_kb = (n_cnt + 15) >> 4;
  if (i >= n_kb * 64) return;
  const int kb = i >> 6, lane = i & 63, il = lane & 31, h = lane >> 5;
  QeBop4 b;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int rel = 16 * kb + 8 * h + v;
    double2 c = make_double2(0.0, 0.0);
    if (il < rows && rel < n_cnt) c = C[(int64_t)il * ldc + n_lo + rel];
    const float re = static_cast<float>(c.x), im = static_cast<float>(c.y);
    const __bf16 rh = static_cast<__bf16>(re), ih = static_cast<__bf16>(im);
    b.rhi[v] = rh;
    b.rlo[v] = static_cast<__bf16>(re - static_cast<float>(rh));
    b.ihi[v] = ih;
    b.ilo[v] = static_cast<__bf16>(im - static_cast<float>(ih));
  }
  out[i] = b;
}

hipError_t launch_pack_qes(const double* d_C, int ldc, int rows, int n_lo, int n_cnt,
                           void* d_bop, hipStream_t s) {
  const int n = 64 * ((n_cnt + 15) >> 4);
  hipLaunchKernelGGL(k_pack_qes, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(d_C), ldc, rows, n_lo, n_cnt,
                     static_cast<QeBop4*>(d_bop));
  return hipGetLastError();
}

__global__ void k_pack_qes64(const double2* __restrict__ C, int ldc, int rows, int B, int n_lo,
                             int n_cnt, double2* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_cnt * B) return;
  const int rel = i / B, e = i - rel * B;
  coef[i] = e < rows ? C[(int64_t)e * ldc + n_lo + rel] : make_double2(0.0, 0.0);
}

hipError_t launch_pack_qes64(const double* d_C, int ldc, int rows, int B, int n_lo, int n_cnt,
                             double* d_coef, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_qes64, dim3((unsigned)ceil_div(n_cnt * B, 256)), dim3(256), 0, s,
                     reinterpret_cast<const double2*>(d_C), ldc, rows, B, n_lo, n_cnt,
                     reinterpret_cast<double2*>(d_coef));
  return hipGetLastError();
}

template <typename T>
__global__ void k_add_complex(int64_t n, T* __restrict__ a, const T* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] += b[i];
}

hipError_t launch_add_complex(bool fp64, int64_t n, void* d_a, const void* d_b, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(2 * n, 256), 65536);
  if (fp64)
    hipLaunchKernelGGL(k_add_complex<double>, dim3(grid), dim3(256), 0, s, n,
                       static_cast<double*>(d_a), static_cast<const double*>(d_b));
  else
    hipLaunchKernelGGL(k_add_complex<float>, dim3(grid), dim3(256), 0, s, n,
                       static_cast<float*>(d_a), static_cast<const float*>(d_b));
  return hipGetLastError();
}

// ------------------------------------------------------------------ FP32 contraction
// Workgroup -> (instance, column, sub) as in the state assembly; each wave
// owns one 32-value tile of its column at a time.  Lane (i, h): B operand =
// value i of orders 8h..8h+7 of a 16-order step; A operand (LDS) =
// C_n(E_i) for the same orders; accumulator = Psi(E_e) at value i for
// e = 8(v/4) + 4h + v%4.  CPLX: complex coefficients (state-based form),
// conjugated for backward instances, and row nE the carried state.
template <bool CPLX>
__global__ __launch_bounds__(kContractThreads) void k_contract_qe_f32(
    const QeInst* __restrict__ insts, QeArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using Bop = typename std::conditional<CPLX, QeBop4, QeBop>::type;
  const int n_kb = (a.n_cnt + 15) >> 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int il = lane & 31, h = lane >> 5;
  Bop* sb = reinterpret_cast<Bop*>(smem);
  // logical workgroup (tile of values, energy tile), the energy tiles of a
  // value tile adjacent: they run on one XCD at the same time and read the
  // same Chebyshev values, which the later tiles find in that XCD's L2
  const int n_et = (a.nE + (a.cplx ? 1 : 0) + 31) / 32;
  const int64_t lwg = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t wg = lwg / n_et;
  const int et = static_cast<int>(lwg - wg * n_et);
  const int e_base = 32 * et;                         // energy tile
  {
    const Bop* gb = static_cast<const Bop*>(a.bop) + (int64_t)et * a.e_tile_stride;
    for (int e = tid; e < n_kb * 64; e += kContractThreads) sb[e] = gb[e];
  }
  __syncthreads();

  int ii = 0;
  while (ii + 1 < a.n_inst && wg >= insts[ii + 1].wg0) ++ii;
  const QeInst& I = insts[ii];
  const int64_t wgl = wg - I.wg0;
  const int64_t col = wgl / I.wpc, sub = wgl - col * I.wpc;
  const int64_t N = I.N;
  const gq2* slots = (const gq2*)(I.slots) + col * N;
  gq2* out = (gq2*)(I.out) + col * (int64_t)a.nE * N;
  const int64_t n_tiles = ceil_div(N, 32);
  const int64_t sstr = I.slot_stride;

  const int64_t stride_tiles = (int64_t)I.wpc * 4;
  for (int64_t tile = sub * 4 + wave; tile < n_tiles; tile += stride_tiles) {
    const int64_t m = tile * 32 + il;
    const bool mv = m < N;
    qf32x16 accR, accI;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      accR[v] = 0.f;
      accI[v] = 0.f;
    }
    qf32x2 xn[8];
    // order n in slot ring_slot(n % S)
    const int part = a.S / a.G;
    auto load_step = [&](int kb) {
      const int rel0 = kb * 16 + h * 8;
      int k = (a.n_lo + rel0) % a.S;
      int ps = ring_slot(k, a.S, a.G);
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        qf32x2 z;
        z.x = 0.f;
        z.y = 0.f;
        xn[v] = (mv && rel0 + v < a.n_cnt) ? slots[(int64_t)ps * sstr + m] : z;
        // next position (S wraps to 0) and its slot, without branches
        const int kn = k + 1, pn = ps + part;
        ps = kn == a.S ? 0 : (pn >= a.S ? pn - (a.S - 1) : pn);
        k = kn == a.S ? 0 : kn;
      }
    };
    load_step(0);
    for (int kb = 0; kb < n_kb; ++kb) {
      qbf16x8 phi, plo, qhi, qlo;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const float p = xn[v].x, q = xn[v].y;
        const __bf16 ph = static_cast<__bf16>(p);
        const __bf16 qh = static_cast<__bf16>(q);
        phi[v] = ph;
        qhi[v] = qh;
        plo[v] = static_cast<__bf16>(p - static_cast<float>(ph));
        qlo[v] = static_cast<__bf16>(q - static_cast<float>(qh));
      }
      if (kb + 1 < n_kb) load_step(kb + 1);
      if constexpr (!CPLX) {
        const QeBop be = sb[kb * 64 + lane];
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.hi, phi, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.lo, phi, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.hi, plo, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.hi, qhi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.lo, qhi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.hi, qlo, accI, 0, 0, 0);
      } else {
        // (Cr + i Ci)(p + i q): Re = Cr p - Ci q, Im = Cr q + Ci p, with Ci
        // negated for the conjugate coefficients of a backward instance
        const QeBop4 be = sb[kb * 64 + lane];
        const qbf16x8 ip_h = I.conj ? neg_bf16(be.ihi) : be.ihi;
        const qbf16x8 ip_l = I.conj ? neg_bf16(be.ilo) : be.ilo;
        const qbf16x8 im_h = neg_bf16(ip_h), im_l = neg_bf16(ip_l);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.rhi, phi, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.rlo, phi, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.rhi, plo, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(im_h, qhi, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(im_l, qhi, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f32_32x32x16_bf16(im_h, qlo, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.rhi, qhi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.rlo, qhi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(be.rhi, qlo, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ip_h, phi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ip_l, phi, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ip_h, plo, accI, 0, 0, 0);
      }
    }
    if (mv) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int e = e_base + 8 * (v >> 2) + 4 * h + (v & 3);
        gq2* p = nullptr;
        bool first = a.first_chunk != 0;
        if (e < a.nE) {
          p = out + (int64_t)e * N + m;
        } else if (CPLX && a.cplx && e == a.nE && I.carry) {
          p = (gq2*)(I.carry) + col * N + m;
          first = a.carry_first != 0;
        }
        if (p) {
          qf32x2 o;
          o.x = accR[v];
          o.y = accI[v];
          if (!first) {
            const qf32x2 old = *p;
            o.x += old.x;
            o.y += old.y;
          }
          *p = o;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ FP64 contraction
// One value per thread, B (>= nE) energy columns in registers, complex
// coefficients (imaginary part 0) in LDS.
template <int B>
__global__ __launch_bounds__(kContractThreads) void k_contract_qe_f64(
    const QeInst* __restrict__ insts, QeArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2* scoef = reinterpret_cast<double2*>(smem);   // [n_cnt][B]
  const int tid = threadIdx.x;
  // logical workgroup (tile of values, energy tile), energy tiles adjacent
  // (one XCD, the same Chebyshev values at the same time: L2 hits)
  const int n_et = (a.nE + (a.cplx ? 1 : 0) + B - 1) / B;
  const int64_t lwg = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t wg = lwg / n_et;
  const int et = static_cast<int>(lwg - wg * n_et);
  const int e_base = B * et;                           // energy tile
  {
    const double2* gc = static_cast<const double2*>(a.coef) + (int64_t)et * a.e_tile_stride;
    for (int e = tid; e < a.n_cnt * B; e += kContractThreads) scoef[e] = gc[e];
  }
  __syncthreads();
  int ii = 0;
  while (ii + 1 < a.n_inst && wg >= insts[ii + 1].wg0) ++ii;
  const QeInst& I = insts[ii];
  const int64_t wgl = wg - I.wg0;
  const int64_t col = wgl / I.wpc, sub = wgl - col * I.wpc;
  const int64_t N = I.N;
  const double2* slots = static_cast<const double2*>(I.slots) + col * N;
  double2* out = static_cast<double2*>(I.out) + col * (int64_t)a.nE * N;
  const int64_t step = (int64_t)I.wpc * kContractThreads;
  for (int64_t m = sub * kContractThreads + tid; m < N; m += step) {
    double2 acc[B];
#pragma unroll
    for (int e = 0; e < B; ++e) acc[e] = make_double2(0.0, 0.0);
    for (int rel = 0; rel < a.n_cnt; ++rel) {
      const double2 x =
          slots[(int64_t)ring_slot((a.n_lo + rel) % a.S, a.S, a.G) * I.slot_stride + m];
#pragma unroll
      for (int e = 0; e < B; ++e) {
        const double2 c = scoef[rel * B + e];
        const double ci = I.conj ? -c.y : c.y;
        acc[e].x = fma(c.x, x.x, fma(-ci, x.y, acc[e].x));
        acc[e].y = fma(c.x, x.y, fma(ci, x.x, acc[e].y));
      }
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
      double2* p = nullptr;
      bool first = a.first_chunk != 0;
      if (e_base + e < a.nE) {
        p = out + (int64_t)(e_base + e) * N + m;
      } else if (a.cplx && e_base + e == a.nE && I.carry) {
        p = static_cast<double2*>(I.carry) + col * N + m;
        first = a.carry_first != 0;
      }
      if (p) {
        double2 o = acc[e];
        if (!first) {
          const double2 old = *p;
          o.x += old.x;
          o.y += old.y;
        }
        *p = o;
      }
    }
  }
}

hipError_t launch_contract_qe(bool fp64, const QeInst* d_inst, const QeArgs& a, hipStream_t s) {
  if (a.total_wg <= 0 || a.n_cnt <= 0) return hipSuccess;
  const dim3 block(kContractThreads);
  const int rows = a.nE + (a.cplx ? 1 : 0);          // energies (+ the carried state)
  if (a.nE < 1 || rows > 129 || (a.cplx && rows > (fp64 ? 16 : 32))) return hipErrorInvalidValue;
  if (!fp64) {
    const dim3 g2((unsigned)(a.total_wg * ceil_div(rows, 32)));
    if (a.cplx) {
      const size_t lds = sizeof(QeBop4) * 64 * (size_t)ceil_div(a.n_cnt, 16);
      hipLaunchKernelGGL(k_contract_qe_f32<true>, g2, block, lds, s, d_inst, a);
    } else {
      const size_t lds = sizeof(QeBop) * 64 * (size_t)ceil_div(a.n_cnt, 16);
      hipLaunchKernelGGL(k_contract_qe_f32<false>, g2, block, lds, s, d_inst, a);
    }
    return hipGetLastError();
  }
  int B = 1;
  while (B < rows && B < 16) B *= 2;
  const dim3 grid2((unsigned)(a.total_wg * ceil_div(rows, B)));
  const size_t lds = sizeof(double2) * (size_t)a.n_cnt * B;
  switch (B) {
    case 1: hipLaunchKernelGGL(k_contract_qe_f64<1>, grid2, block, lds, s, d_inst, a); break;
    case 2: hipLaunchKernelGGL(k_contract_qe_f64<2>, grid2, block, lds, s, d_inst, a); break;
    case 4: hipLaunchKernelGGL(k_contract_qe_f64<4>, grid2, block, lds, s, d_inst, a); break;
    case 8: hipLaunchKernelGGL(k_contract_qe_f64<8>, grid2, block, lds, s, d_inst, a); break;
    case 16: hipLaunchKernelGGL(k_contract_qe_f64<16>, grid2, block, lds, s, d_inst, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ output layout
// in: [Rg][nE][N] (the group's accumulators); out: [nE][N][ld], columns
// col0 .. col0 + Rg - 1, complex64 or complex128.
__global__ void k_qe_scatter(int64_t N, int Rg, int nE, int ld, int col0, int fp64_in,
                             const void* __restrict__ in, int out_dtype, void* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = N * Rg * nE;
  if (i >= total) return;
  // i runs over (e, s, c) with c fastest, so the writes of a row are contiguous
  const int64_t c = i % Rg;
  const int64_t rest = i / Rg;
  const int64_t s = rest % N;
  const int64_t e = rest / N;
  const int64_t src = (c * nE + e) * N + s;
  double x, y;
  if (fp64_in) {
    const double2 v = static_cast<const double2*>(in)[src];
    x = v.x;
    y = v.y;
  } else {
    const float2 v = static_cast<const float2*>(in)[src];
    x = v.x;
    y = v.y;
  }
  const int64_t dst = (e * N + s) * ld + col0 + c;
  if (out_dtype == CSP_C128) static_cast<double2*>(out)[dst] = make_double2(x, y);
  else static_cast<float2*>(out)[dst] = make_float2(static_cast<float>(x), static_cast<float>(y));
}

hipError_t launch_qe_scatter(int64_t N, int Rg, int nE, int ld, int col0, bool fp64_in,
                             const void* d_in, int out_dtype, void* d_out, hipStream_t s) {
  const int64_t total = N * Rg * nE;
  hipLaunchKernelGGL(k_qe_scatter, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, N, Rg,
                     nE, ld, col0, fp64_in ? 1 : 0, d_in, out_dtype, d_out);
  return hipGetLastError();
}

}  // namespace csp
