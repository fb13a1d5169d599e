// Moment-based form (Sec. II.A, moment-based implementation; Sec. III
// DOS-Concurrent-M): the per-order inner products (the recursion kernel's
// moment records, summed per column by k_cheb_mom_finish) are turned into
// the block moments mu_n = <psi0|T_n(H~) s_k> (directly, or with halving
// every moment above mu_1 from the self products of Eq. cheby_prod), and contracted
// with the expansion coefficients into correlations
//   C(t_{kb+j}) = sum_{n=0}^{N(j tau)} c_n(j tau) mu_n,   c_n = (-i)^n a_n.
// Everything here is FP64 and summed in a fixed order.
#include "csp_internal.h"

namespace csp {

// mu_n for n = 0..Nk of one instance.  dots row n holds the sums of the step
// that produced order n: [0] <psi0|phi_n>, [1] <psi0|phi_{n-1}>,
// [2] <phi_n|phi_n>, [3] <phi_n|phi_{n-1}>.
__global__ void k_mom_assemble(const MomCorrInst* __restrict__ mc, int Nk, int halving) {
  const MomCorrInst& M = mc[blockIdx.y];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (Nk + 1) * M.Rg) return;
  const int n = e / M.Rg, r = e - n * M.Rg;
  const int Rg = M.Rg;
  auto dot = [&](int row, int kind) {
    const double* p = M.dots + ((int64_t)row * 4 * Rg + kind * Rg + r) * 2;
    return make_double2(p[0], p[1]);
  };
  double2 mu;
  if (n == 0) {
    mu = dot(1, 1);                       // <psi0|s_k>
  } else if (!halving || n == 1) {
    mu = dot(n, 0);
  } else if ((n & 1) == 0) {              // mu_2k = 2 <phi_k|phi_k> - mu_0
    const double2 a = dot(n / 2, 2), m0 = dot(1, 1);
    mu = make_double2(2.0 * a.x - m0.x, 2.0 * a.y - m0.y);
  } else {                                // mu_2k+1 = 2 <phi_k+1|phi_k> - mu_1
    const double2 a = dot((n + 1) / 2, 3), m1 = dot(1, 0);
    mu = make_double2(2.0 * a.x - m1.x, 2.0 * a.y - m1.y);
  }
  reinterpret_cast<double2*>(M.mu)[(int64_t)n * Rg + r] = mu;
}

// corr[(t0 + 1 + j) * ldc + col0 + r] = sum_{n <= N((j+1) tau)} (-i)^n a[j][n] mu_n[r]
__global__ void k_mom_corr(const MomCorrInst* __restrict__ mc, const double* __restrict__ a,
                           int lda, const int32_t* __restrict__ ntr, int bk, int64_t t0) {
  const MomCorrInst& M = mc[blockIdx.y];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= bk * M.Rg) return;
  const int j = e / M.Rg, r = e - j * M.Rg;
  const double* aj = a + (int64_t)j * lda;
  const double2* mu = reinterpret_cast<const double2*>(M.mu);
  double sx = 0.0, sy = 0.0;
  const int nt = ntr[j];
  for (int n = 0; n <= nt; ++n) {
    const double c = aj[n];
    const double2 m = mu[(int64_t)n * M.Rg + r];
    switch (n & 3) {                      // (-i)^n (m.x + i m.y)
      case 0: sx += c * m.x; sy += c * m.y; break;
      case 1: sx += c * m.y; sy -= c * m.x; break;
      case 2: sx -= c * m.x; sy -= c * m.y; break;
      default: sx -= c * m.y; sy += c * m.x; break;
    }
  }
  reinterpret_cast<double2*>(M.corr)[(t0 + 1 + j) * M.ldc + M.col0 + r] = make_double2(sx, sy);
}

hipError_t launch_mom_corr(const MomCorrInst* d_mc, int n_inst, int Nk, int halving,
                           const double* d_a, int lda, const int32_t* d_ntrunc, int bk,
                           int64_t t0, int rg_max, hipStream_t s) {
  const int na = (Nk + 1) * rg_max;
  hipLaunchKernelGGL(k_mom_assemble, dim3((unsigned)ceil_div(na, 256), n_inst), dim3(256), 0, s,
                     d_mc, Nk, halving);
  const int nc = bk * rg_max;
  hipLaunchKernelGGL(k_mom_corr, dim3((unsigned)ceil_div(nc, 256), n_inst), dim3(256), 0, s,
                     d_mc, d_a, lda, d_ntrunc, bk, t0);
  return hipGetLastError();
}

// Correlations from moments that are already assembled (M.mu filled by the
// caller): rows t0 + 1 .. t0 + bk of M.corr.
hipError_t launch_mom_corr_only(const MomCorrInst* d_mc, int n_inst, const double* d_a, int lda,
                                const int32_t* d_ntrunc, int bk, int64_t t0, int rg_max,
                                hipStream_t s) {
  const int64_t nc = (int64_t)bk * rg_max;
  hipLaunchKernelGGL(k_mom_corr, dim3((unsigned)ceil_div(nc, 256), n_inst), dim3(256), 0, s,
                     d_mc, d_a, lda, d_ntrunc, bk, t0);
  return hipGetLastError();
}

}  // namespace csp
