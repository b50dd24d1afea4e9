// Hand-written FFT and what is built on it: the masked orthonormal 2-D DFT
// operator (compressive sensing: H^T y, |H(w)|^2, H^T H v) and the circulant
// CG preconditioner (H^T H / xi + d_bar I)^{-1}.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "lik.h"

namespace eptv {

hipError_t dft_setup(LikCtx& lc, const LikInstInfo* li, int n, size_t fft_bytes, hipStream_t s,
                     std::string& err);
hipError_t dft_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s);
// H^T v of the masked-DFT instance with likelihood index li (v: interleaved
// complex observation-space array) into the pixel plane `out`
hipError_t dft_back_project_inst(LikCtx& lc, int li, const float* v, float* out, hipStream_t s);
// mode 0: q = A x; mode 1: p_out = z + beta p_in, q = A p_out (with v.q partials)
hipError_t dft_apply(LikCtx& lc, int mode, hipStream_t s);
void dft_destroy(LikCtx& lc);
// z = M^{-1} r with the circulant M = H^T H / xi + d_bar I, for instances
// whose preconditioner is PRECOND_CIRCULANT
hipError_t fft_precondition(LikCtx& lc, hipStream_t s);
// z = M^{-1} r through a real-input transform (half spectra, three row passes
// and two transposes), writing r.z and r.r partials at [tile0, tile0 + npart)
// (update = 1: first the CG step x += alpha p, r -= alpha q, fused into the
// first pass)
hipError_t rfft_precondition(LikCtx& lc, int update, hipStream_t s);
// masked-DFT instances: p_out = z + beta p_in and q = (H^T H / xi + diag tau_c)
// p_out by the real transform, with p.q partials at [tile0, tile0 + npart)
hipError_t rfft_product(LikCtx& lc, hipStream_t s);
int rfft_partials(int H, int W);

}  // namespace eptv
