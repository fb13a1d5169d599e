// Chebyshev expansion coefficients of the propagator (App. B):
//   exp(-i x y) = sum_n c_n(x) T_n(y),  c_0 = J_0(x),  c_n = 2 (-i)^n J_n(x),
// in FP64 on the GPU, and the truncation order N(x) of Sec. II.A.
//
// J_n(x) by Miller's backward recurrence (J. C. P. Miller, 1952): start far
// above both the wanted orders and x with an arbitrary seed, run
// J_{k-1} = (2k/x) J_k - J_{k+1} down to k = 0 (the recurrence is stable in
// that direction for the decaying solution), and fix the overall factor with
// the Neumann identity J_0 + 2 (J_2 + J_4 + ...) = 1.  Growth in the
// evanescent region n > x is kept in range by rescaling by 2^-600 whenever a
// value exceeds 2^600, applied to the running sum and to every stored order.
#include "csp_internal.h"

namespace csp {

__global__ void k_bessel(double tau, int nx, int nmax, double eta, int clip,
                         double* __restrict__ out, int32_t* __restrict__ ntrunc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nx) return;
  const double x = tau * (double)(j + 1);
  double* a = out + (size_t)j * (nmax + 1);
  if (!(x > 0.0)) {
    a[0] = 1.0;
    for (int n = 1; n <= nmax; ++n) a[n] = 0.0;
    ntrunc[j] = 0;
    return;
  }
  // With clip, only the orders this argument needs are computed: past its
  // truncation order (bounded by x + 40 + 25 x^(1/3)) the coefficients are
  // below 1e-14 and stored as 0.  Arguments far below the table's largest
  // then avoid a long, repeatedly rescaled recurrence.
  const int need = (int)ceil(x + 40.0 + 25.0 * cbrt(x + 1.0));
  const int top = (clip && need < nmax) ? need : nmax;   // highest order stored
  for (int n = top + 1; n <= nmax; ++n) a[n] = 0.0;
  // Start order: beyond the stored orders and the turning point x by a
  // margin that grows like x^(1/3) (the width of the transition region of
  // J_n near n = x); even, so that the Neumann sum ends on an even order.
  int M = (int)ceil((x > (double)top ? x : (double)top) + 24.0 + 18.0 * cbrt(x + 1.0));
  M += M & 1;
  const double big = 0x1p600, small = 0x1p-600;
  const double inv_x = 1.0 / x;
  double up = 0.0;        // J_{k+1}
  double cur = 0x1p-300;  // J_k, arbitrary seed at k = M
  double even_sum = 0.0;  // sum of J_k over even k >= 2 seen so far
  for (int k = M; k >= 1; --k) {
    if (k <= top) a[k] = cur;
    if ((k & 1) == 0) even_sum += cur;
    const double down = (2.0 * (double)k * inv_x) * cur - up;
    up = cur;
    cur = down;
    if (fabs(cur) > big) {
      cur *= small;
      up *= small;
      even_sum *= small;
      for (int n = k; n <= top; ++n) a[n] *= small;  // orders stored so far
    }
  }
  // cur now holds J_0 (unnormalised).
  a[0] = cur;
  const double norm = cur + 2.0 * even_sum;
  const double inv = 1.0 / norm;
  for (int n = 0; n <= top; ++n) a[n] *= (n == 0 ? inv : 2.0 * inv);
  // Truncation: first order above x with |c_n| = a_n <= eta.
  int N = -1;
  for (int n = (int)floor(x) + 1; n <= top; ++n)
    if (fabs(a[n]) <= eta) { N = n; break; }
  ntrunc[j] = N;
}

hipError_t launch_bessel(double tau, int nx, int nmax, double eta, bool clip, double* d_a,
                         int32_t* d_ntrunc, hipStream_t s) {
  hipLaunchKernelGGL(k_bessel, dim3((nx + 63) / 64), dim3(64), 0, s, tau, nx, nmax, eta,
                     clip ? 1 : 0, d_a, d_ntrunc);
  return hipGetLastError();
}

__global__ void k_complex_coeffs(const double* __restrict__ a, int nmax, double2* __restrict__ c) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n > nmax) return;
  const double v = a[n];
  double2 o;
  switch (n & 3) {               // (-i)^n
    case 0: o = make_double2(v, 0.0); break;
    case 1: o = make_double2(0.0, -v); break;
    case 2: o = make_double2(-v, 0.0); break;
    default: o = make_double2(0.0, v); break;
  }
  c[n] = o;
}

hipError_t launch_complex_coeffs(const double* d_a, int nmax, double* d_c, hipStream_t s) {
  hipLaunchKernelGGL(k_complex_coeffs, dim3((nmax + 256) / 256), dim3(256), 0, s, d_a, nmax,
                     reinterpret_cast<double2*>(d_c));
  return hipGetLastError();
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
struct BopEntryP {
  bf16x8 hi;
  bf16x8 lo;
};

// One thread per (16-order step kb, time tile jt, lane): lane (j, h) holds
// a_{n, j+1} for n = n_lo + 16 kb + 8 h + v, v = 0..7, split into bf16 hi/lo.
__global__ void k_pack_bop(const double* __restrict__ a, int lda, const int32_t* __restrict__ ntr,
                           int bcols, int jtiles, int n_lo, int n_cnt, BopEntryP* __restrict__ bop,
                           float* __restrict__ ccarry) {
  const int n_kb = (n_cnt + 15) / 16;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_kb * 16) {
    const int n = n_lo + e;
    float v = 0.f;
    if (e < n_cnt && n <= ntr[bcols - 1]) v = (float)a[(size_t)(bcols - 1) * lda + n];
    ccarry[e] = v;
  }
  if (e >= n_kb * jtiles * 64) return;
  const int lane = e & 63;
  const int jt = (e >> 6) % jtiles;
  const int kb = (e >> 6) / jtiles;
  const int j = jt * 32 + (lane & 31);
  BopEntryP out;
  for (int v = 0; v < 8; ++v) {
    const int rel = kb * 16 + (lane >> 5) * 8 + v;
    const int n = n_lo + rel;
    double val = 0.0;
    if (j < bcols && rel < n_cnt && n <= ntr[j]) val = a[(size_t)j * lda + n];
    const __bf16 hi = static_cast<__bf16>(static_cast<float>(val));
    const double rest = val - static_cast<double>(static_cast<float>(hi));
    out.hi[v] = hi;
    out.lo[v] = static_cast<__bf16>(static_cast<float>(rest));
  }
  bop[(kb * jtiles + jt) * 64 + lane] = out;
}

hipError_t launch_pack_bop(const double* d_a, int lda, const int32_t* d_ntrunc, int bcols,
                           int jtiles, int n_lo, int n_cnt, void* d_bop, float* d_ccarry,
                           hipStream_t s) {
  const int n_kb = (n_cnt + 15) / 16;
  const int total = n_kb * jtiles * 64 > n_kb * 16 ? n_kb * jtiles * 64 : n_kb * 16;
  hipLaunchKernelGGL(k_pack_bop, dim3((total + 255) / 256), dim3(256), 0, s, d_a, lda, d_ntrunc,
                     bcols, jtiles, n_lo, n_cnt, static_cast<BopEntryP*>(d_bop), d_ccarry);
  return hipGetLastError();
}

__global__ void k_pack_c64(const double* __restrict__ a, int lda, const int32_t* __restrict__ ntr,
                           int bcols, int n_lo, int n_cnt, double2* __restrict__ coef,
                           double2* __restrict__ ccarry) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_cnt * bcols) return;
  const int rel = e / bcols, j = e - rel * bcols;
  const int n = n_lo + rel;
  const double v = n <= ntr[j] ? a[(size_t)j * lda + n] : 0.0;
  double2 o;
  switch (n & 3) {
    case 0: o = make_double2(v, 0.0); break;
    case 1: o = make_double2(0.0, -v); break;
    case 2: o = make_double2(-v, 0.0); break;
    default: o = make_double2(0.0, v); break;
  }
  coef[e] = o;
  if (j == bcols - 1) ccarry[rel] = o;
}

hipError_t launch_pack_c64(const double* d_a, int lda, const int32_t* d_ntrunc, int bcols,
                           int n_lo, int n_cnt, double* d_coef, double* d_ccarry,
                           hipStream_t s) {
  const int total = n_cnt * bcols;
  hipLaunchKernelGGL(k_pack_c64, dim3((total + 255) / 256), dim3(256), 0, s, d_a, lda, d_ntrunc,
                     bcols, n_lo, n_cnt, reinterpret_cast<double2*>(d_coef),
                     reinterpret_cast<double2*>(d_ccarry));
  return hipGetLastError();
}

}  // namespace csp
