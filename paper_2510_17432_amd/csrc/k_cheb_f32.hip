// Instantiations of the Chebyshev recursion kernel: complex64, plain recursion.
#include "k_cheb_body.h"

namespace csp {

hipError_t launch_cheb_f32(int vec, int kt, bool honey, bool eps, const ChebInst* d_inst, int n_inst,
                           int64_t item_lo, int64_t item_hi, const ChebStep& st, hipStream_t s) {
  const int64_t n = item_hi - item_lo;
  if (n <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(ceil_div(n, 4))), block(256);
  switch (vec * 100 + kt) {
    case 201: CSP_CHEB_LAUNCH(float, 2, 1, cheb::kMomNone, false); break;
    case 202: CSP_CHEB_LAUNCH(float, 2, 2, cheb::kMomNone, false); break;
    case 204: CSP_CHEB_LAUNCH(float, 2, 4, cheb::kMomNone, false); break;
    case 208: CSP_CHEB_LAUNCH(float, 2, 8, cheb::kMomNone, false); break;
    case 401: CSP_CHEB_LAUNCH(float, 4, 1, cheb::kMomNone, false); break;
    case 402: CSP_CHEB_LAUNCH(float, 4, 2, cheb::kMomNone, false); break;
    case 404: CSP_CHEB_LAUNCH(float, 4, 4, cheb::kMomNone, false); break;
    case 408: CSP_CHEB_LAUNCH(float, 4, 8, cheb::kMomNone, false); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace csp
