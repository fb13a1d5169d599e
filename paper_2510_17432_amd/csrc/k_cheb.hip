// Chebyshev recursion launches: the kernel itself (k_cheb_body.h) is
// instantiated per precision and epilogue in k_cheb_f32*.hip and
// k_cheb_f64*.hip; this file picks the instantiation for each run of
// instances with the same lattice class, and sums the moment records.
#include "csp_internal.h"

namespace csp {

#define CSP_CHEB_LAUNCHER(name)                                                                 \
  hipError_t name(int vec, int kt, bool honey, bool eps, const ChebInst* d_inst, int n_inst,   \
                  int64_t item_lo, int64_t item_hi, const ChebStep& st, hipStream_t s);
CSP_CHEB_LAUNCHER(launch_cheb_f32)
CSP_CHEB_LAUNCHER(launch_cheb_f32m)
CSP_CHEB_LAUNCHER(launch_cheb_f64)
CSP_CHEB_LAUNCHER(launch_cheb_f64m)
CSP_CHEB_LAUNCHER(launch_cheb_f32mc)
CSP_CHEB_LAUNCHER(launch_cheb_f64mc)
CSP_CHEB_LAUNCHER(launch_cheb_f32s)
CSP_CHEB_LAUNCHER(launch_cheb_f64s)
#undef CSP_CHEB_LAUNCHER

bool cheb_shape_supported(bool fp64, int vec, int kt, bool mom) {
  if (fp64) return vec == 2 && (kt == 1 || kt == 2 || kt == 4);
  if (vec != 2 && vec != 4) return false;
  return kt == 1 || kt == 2 || kt == 4 || (kt == 8 && (!mom || vec == 2));
}

bool cheb_carry_supported(bool fp64, int vec, int kt) {
  return vec == 2 && (kt == 1 || kt == 2 || kt == 4 || (kt == 8 && !fp64));
}

int cheb_margin(int vec, int kt) { return (kt + vec - 1) / vec * vec; }

hipError_t launch_cheb(bool fp64, int vec, int kt, bool mom, bool carry, const ChebInst* d_inst,
                       const std::vector<ChebRun>& runs, const ChebStep& st, hipStream_t s) {
  if (st.nlev < 1 || st.nlev > kt) return hipErrorInvalidValue;
  if (!cheb_shape_supported(fp64, vec, kt, mom)) return hipErrorInvalidValue;
  if (carry && (!mom || !cheb_carry_supported(fp64, vec, kt))) return hipErrorInvalidValue;
  // only the self products (one block, bra = ket): the kernel without psi0
  const bool self = mom && !carry && !st.dot_psi0 && st.dot_self;
  if (st.ow != 64 * vec - 2 * cheb_margin(vec, kt)) return hipErrorInvalidValue;
  for (const ChebRun& r : runs) {
    const ChebInst* di = d_inst + r.inst0;
    const int64_t lo = r.item0, hi = r.item0 + r.n_items;
    hipError_t e;
    if (r.sparse && r.win)
      e = launch_cheb_ellw(fp64, mom, carry, r.ct, r.win_cap, di, r.n_inst, r.wave0,
                           r.wave0 + r.n_waves, st, s);
    else if (r.sparse)
      e = launch_cheb_ell(fp64, mom, carry, r.ct, di, r.n_inst, r.wave0, r.wave0 + r.n_waves, st,
                          s);
    else if (fp64)
      e = carry  ? launch_cheb_f64mc(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s)
          : self ? launch_cheb_f64s(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s)
          : mom  ? launch_cheb_f64m(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s)
                 : launch_cheb_f64(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s);
    else
      e = carry  ? launch_cheb_f32mc(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s)
          : self ? launch_cheb_f32s(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s)
          : mom  ? launch_cheb_f32m(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s)
                 : launch_cheb_f32(vec, kt, r.honey, r.eps, di, r.n_inst, lo, hi, st, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ moment sums
// One workgroup per (launch slot, level) and instance: thread t handles
// value t % (8 Rg) (kind, column, re/im) of the per-column sums and adds the
// records of that column's work items lane, lane + lanes, ... in eight
// interleaved partial sums; the lanes are then added in order.
__global__ __launch_bounds__(256) void k_cheb_mom_finish(const MomInst* __restrict__ mi,
                                                         const double* __restrict__ partial,
                                                         int64_t total_items, int kt, int n0,
                                                         int max_row) {
  __shared__ double red[256];
  const int sl = blockIdx.x;                     // slot * kt + level
  const int row = n0 + sl;                       // order produced by that level
  const MomInst& M = mi[blockIdx.y];
  const int nval = 8 * M.Rg;
  const int lanes = 256 / nval;
  const int t = threadIdx.x;
  const int lanei = t / nval, vi = t - lanei * nval;
  const int kindk = vi / (2 * M.Rg);
  const int rem = vi - kindk * 2 * M.Rg;
  const int c = rem >> 1, comp = rem & 1;
  double s = 0.0;
  if (lanei < lanes && row <= max_row) {
    const int64_t ipc = M.n_tiles / M.Rg;        // work items per column
    const double* base = partial + ((int64_t)sl * total_items + M.tile0 + c * ipc) * 8 +
                         kindk * 2 + comp;
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t k = lanei;
    for (; k + 7 * lanes < ipc; k += 8 * lanes) {
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] += base[(k + u * lanes) * 8];
    }
    for (int u = 0; k < ipc; k += lanes, ++u) q[u & 7] += base[k * 8];
    s = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
  }
  red[t] = s;
  __syncthreads();
  if (t < nval && row <= max_row) {
    double sum = 0.0;
    for (int l = 0; l < lanes; ++l) sum += red[l * nval + t];
    // dots row `row`, layout [kind][Rg][re, im]
    M.dots[(int64_t)row * nval + (kindk * M.Rg + c) * 2 + comp] = sum;
  }
}

hipError_t launch_cheb_mom_finish(const MomInst* d_mi, int n_inst, const double* partial,
                                  int64_t total_items, int kt, int n_slots, int n0, int max_row,
                                  hipStream_t s) {
  if (n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cheb_mom_finish, dim3(n_slots * kt, n_inst), dim3(256), 0, s, d_mi,
                     partial, total_items, kt, n0, max_row);
  return hipGetLastError();
}

}  // namespace csp
