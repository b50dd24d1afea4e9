// Gaussian i.i.d. compressive sensing (Sec. II-A case (iii), the CS experiment
// of Sec. V): a dense M x N sensing matrix H, whose likelihood site gets its
// mean and variances from the Woodbury identity (Sec. III-C, for low-rank
// H^T H):
//   S = xi I_M + H D^-1 H^T = L L^T (blocked Cholesky),  Z^T = H^T L^-T,
//   v_i = 1/d_i - |Z^T_i|^2 / d_i^2,  E_i = (b_i - Z^T_i . t) / d_i,  t = Z (b / d),
// with D = diag(tau_c) the cavity precisions and b = H^T y / xi + eta_c.  All
// of it in FP64 (the subtraction in v_i cancels when d_i is small), the
// products on v_mfma_f64_16x16x4f64.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "lik.h"

namespace eptv {

hipError_t gauss_setup(LikCtx& lc, const LikInstInfo* li, int n, hipStream_t s, std::string& err);
// H^T y into the H^T y plane and the pixel-space observation.
hipError_t gauss_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s);
// The Woodbury moments of every Gaussian-CS instance whose likelihood site is
// updated in this sweep (host state `hst` current): E into the x plane, v into
// the variance plane.
hipError_t gauss_update(LikCtx& lc, const InstState* hst, hipStream_t s);

}  // namespace eptv
