// Masked orthonormal 2-D DFT operator (compressive sensing): H^T y, |H(w)|^2
// and H^T H v = Re(F^H diag(mask) F v), built on a hand-written FFT.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "lik.h"

namespace eptv {

hipError_t dft_setup(LikCtx& lc, const LikInstInfo* li, int n, hipStream_t s, std::string& err);
hipError_t dft_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s);
// mode 0: q = A x; mode 1: p_out = z + beta p_in, q = A p_out (with v.q partials)
hipError_t dft_apply(LikCtx& lc, int mode, hipStream_t s);
void dft_destroy(LikCtx& lc);

}  // namespace eptv
