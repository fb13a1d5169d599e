// Instantiations of the Chebyshev recursion kernel: complex128, plain recursion and moment epilogue.
#include "k_cheb_body.h"

namespace csp {

hipError_t launch_cheb_f64(int vec, int kt, bool honey, bool eps, const ChebInst* d_inst, int n_inst,
                           int64_t item_lo, int64_t item_hi, const ChebStep& st, hipStream_t s) {
  const int64_t n = item_hi - item_lo;
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(ceil_div(n, 4))), block(256);
  switch (vec * 100 + kt) {
    case 201: CSP_CHEB_LAUNCH(double, 2, 1, cheb::kMomNone, false); break;
    case 202: CSP_CHEB_LAUNCH(double, 2, 2, cheb::kMomNone, false); break;
    case 204: CSP_CHEB_LAUNCH(double, 2, 4, cheb::kMomNone, false); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cheb_f64m(int vec, int kt, bool honey, bool eps, const ChebInst* d_inst, int n_inst,
                            int64_t item_lo, int64_t item_hi, const ChebStep& st, hipStream_t s) {
  const int64_t n = item_hi - item_lo;
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(ceil_div(n, 4))), block(256);
  switch (vec * 100 + kt) {
    case 201: CSP_CHEB_LAUNCH(double, 2, 1, cheb::kMomBra, false); break;
    case 202: CSP_CHEB_LAUNCH(double, 2, 2, cheb::kMomBra, false); break;
    case 204: CSP_CHEB_LAUNCH(double, 2, 4, cheb::kMomBra, false); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace csp
