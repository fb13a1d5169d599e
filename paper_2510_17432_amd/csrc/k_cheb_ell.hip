// Chebyshev recursion (amxsy of Sec. II.B) for a Hamiltonian given
// explicitly in ELL form, for matrices of any density D_H (Sec. II.B: the
// paper's speedups are measured at D_H = 60..230, where the recursion
// dominates):
//   phi_{n+1} = 2 H~ phi_n - phi_{n-1},  H~ = (H - H0)/|H|,
// one step per launch (the neighbours of a row are arbitrary, so no
// temporal blocking).  The matrix is stored [D][N] (entry k of every row
// contiguous; a row with fewer entries is padded with its own index and a
// zero value), so a wave reading entry k of its 64 rows reads 256 B of
// indices and 256-512 B of values; the vector gathers go through the caches.
// One wave handles 64 rows of one column; the waves of the columns of one
// row chunk are scheduled together so that they share the matrix rows in
// the caches (the matrix is read from HBM about once per step, not once per
// column).  The moment epilogue and the carried state follow the stencil
// kernel (records of 8 FP64 sums per wave, fixed butterfly).
#include <type_traits>

#include "csp_internal.h"

namespace csp {

template <typename T, bool MOM, bool CARRY>
__global__ __launch_bounds__(256) void k_cheb_ell(const ChebInst* __restrict__ insts, int n_inst,
                                                  int64_t item_lo, int64_t item_hi, ChebStep st) {
  using C = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int64_t w = item_lo + xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= item_hi) return;                         // a whole wave
  int ii = 0;
  while (ii + 1 < n_inst && w >= insts[ii + 1].item0) ++ii;
  const ChebInst& I = insts[ii];
  const int64_t lw = w - I.item0;
  const int64_t col = lw % I.Rg, chunk = lw / I.Rg;
  const int64_t item = I.item0 + col * I.n_segs + chunk;   // record index: column-major
  const int64_t N = I.N;
  const int64_t s = chunk * 64 + lane;
  const bool valid = s < N;
  const int64_t coff = col * N;

  C* base = static_cast<C*>(I.base);
  const C* cur = (st.slot_cur < 0 ? static_cast<const C*>(I.src)
                                  : base + (int64_t)st.slot_cur * I.slot_stride) + coff;
  const C* prev = st.first ? nullptr : base + (int64_t)st.slot_prev * I.slot_stride + coff;
  C* outv = st.slot_out[0] >= 0 ? base + (int64_t)st.slot_out[0] * I.slot_stride + coff : nullptr;
  C* copyv = st.copy_slot >= 0 ? base + (int64_t)st.copy_slot * I.slot_stride + coff : nullptr;
  const T* val = static_cast<const T*>(I.ell_val);
  const int D = I.ell_D;
  const T scale = st.first ? T(0.5) : T(1);
  const T alpha = scale * static_cast<T>(I.alpha);
  const T beta0 = scale * static_cast<T>(I.beta0);

  C c, o;
  c.x = c.y = o.x = o.y = T(0);
  if (valid) {
    c = cur[s];
    // padding entries hold (own index, 0), so the loop has no branch and
    // its gathers can be issued ahead
    T ax = T(0), ay = T(0);
    const int32_t* cp = I.ell_col + s;
    const T* vp = val + s;
#pragma unroll 4
    for (int k = 0; k < D; ++k) {
      const int32_t j = cp[(int64_t)k * N];
      const T v = vp[(int64_t)k * N];
      const C x = cur[j];
      ax = fma(v, x.x, ax);
      ay = fma(v, x.y, ay);
    }
    C p;
    p.x = p.y = T(0);
    if (prev) p = prev[s];
    o.x = alpha * ax + (beta0 * c.x - p.x);
    o.y = alpha * ay + (beta0 * c.y - p.y);
    if (outv) outv[s] = o;
    if (copyv) copyv[s] = c;
  }

  if constexpr (CARRY) {
    if (valid && st.carry_mode && I.carry) {
      C* carry = static_cast<C*>(I.carry) + coff;
      const T c0r = static_cast<T>(st.cc0[0]), c0i = static_cast<T>(st.cc0[1]);
      const T c1r = static_cast<T>(st.ccl[0][0]), c1i = static_cast<T>(st.ccl[0][1]);
      C b;
      if (st.carry_mode == 1) {
        b.x = c0r * c.x - c0i * c.y;
        b.y = c0r * c.y + c0i * c.x;
      } else {
        b = carry[s];
      }
      b.x += c1r * o.x - c1i * o.y;
      b.y += c1r * o.y + c1i * o.x;
      carry[s] = b;
    }
  }

  if constexpr (MOM) {
    if (st.dot_psi0 || st.dot_self) {
      double r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (valid) {
        const double ox = o.x, oy = o.y, cx = c.x, cy = c.y;
        if (st.dot_psi0) {
          const C q = static_cast<const C*>(I.psi0)[coff + s];
          const double qx = q.x, qy = q.y;
          r[0] = qx * ox + qy * oy;
          r[1] = qx * oy - qy * ox;
          r[2] = qx * cx + qy * cy;
          r[3] = qx * cy - qy * cx;
        }
        if (st.dot_self) {
          r[4] = ox * ox + oy * oy;
          r[6] = ox * cx + oy * cy;
          r[7] = ox * cy - oy * cx;
        }
      }
      // record [kind][re, im]: <psi0|out>, <psi0|cur>, <out|out>, <out|cur>
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        double x = r[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
        r[k] = x;
      }
      if (lane == 0) {
        double* out = st.partial + ((int64_t)st.mom_slot * st.total_items + item) * 8;
#pragma unroll
        for (int k = 0; k < 8; ++k) out[k] = r[k];
      }
    }
  }
}

hipError_t launch_cheb_ell(bool fp64, bool mom, bool carry, const ChebInst* d_inst, int n_inst,
                           int64_t item_lo, int64_t item_hi, const ChebStep& st, hipStream_t s) {
  const int64_t n = item_hi - item_lo;
  if (n <= 0) return hipSuccess;
  if (st.nlev != 1 || (carry && !mom)) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(ceil_div(n, 4))), block(256);
#define CSP_ELL(T, M, CY) \
  hipLaunchKernelGGL((k_cheb_ell<T, M, CY>), grid, block, 0, s, d_inst, n_inst, item_lo, item_hi, st)
  if (fp64) {
    if (carry) CSP_ELL(double, true, true);
    else if (mom) CSP_ELL(double, true, false);
    else CSP_ELL(double, false, false);
  } else {
    if (carry) CSP_ELL(float, true, true);
    else if (mom) CSP_ELL(float, true, false);
    else CSP_ELL(float, false, false);
  }
#undef CSP_ELL
  return hipGetLastError();
}

// Gershgorin row bound of an explicit matrix (H0 = 0): max_s sum_k |val_sk|,
// each row summed in k order with plain additions (padding values are 0);
// one maximum per block.
__global__ void k_ell_gershgorin(int64_t N, int D, const double* __restrict__ val, double* __restrict__ partial) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    double r = 0.0;
    for (int k = 0; k < D; ++k)
      r = r + fabs(val[(int64_t)k * N + s]);
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

hipError_t launch_ell_gershgorin(int64_t N, int D, const int32_t* d_col, const double* d_val,
                                 double* d_partial, int n_partial, hipStream_t s) {
  (void)d_col;
  hipLaunchKernelGGL(k_ell_gershgorin, dim3(n_partial), dim3(256), 0, s, N, D, d_val, d_partial);
  return hipGetLastError();
}

}  // namespace csp
