// Subsampled Paley-ordered 2-D Walsh-Hadamard sensing operator (compressive
// sensing, Sec. II-A case (iii) with the Hadamard matrix of the CS experiment,
// Sec. V): H^T y, H^T H v, and the CG preconditioner that is diagonal in the
// Walsh basis.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "lik.h"

namespace eptv {

// p.q partials one product writes (one per LDS block; never more than the
// instance's likelihood tiles)
int wht_partials(int H, int W);
hipError_t wht_setup(LikCtx& lc, const LikInstInfo* li, int n, size_t wht_bytes, hipStream_t s,
                     std::string& err);
// H^T y into the H^T y plane and the pixel-space observation
hipError_t wht_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s);
// H^T v of the Walsh-Hadamard instance with likelihood index li (v: Paley-ordered
// coefficients) into the pixel plane `out`
hipError_t wht_back_project_inst(LikCtx& lc, int li, const float* v, float* out, hipStream_t s);
// mode 0: q = A x; mode 1: p_out = z + beta p_in, q = A p_out; with p.q partials
hipError_t wht_apply(LikCtx& lc, int mode, hipStream_t s);
// z = M^{-1} r, M = W^T diag(mask / xi + d_bar) W, for instances whose
// preconditioner is the transform-diagonal one
hipError_t wht_precondition(LikCtx& lc, hipStream_t s);

}  // namespace eptv
