#include "lik.h"

namespace eptv {

hipError_t lik_create(LikCtx& lc, const LikInstInfo* li, int n, char*, const LikLayout&, long long,
                      InstDev*, InstState*, int4*, int, float*, hipStream_t,
                      std::string& err) {
  for (int i = 0; i < n; ++i)
    if (li[i].op != OP_IDENTITY) {
      err = "operator not available in this build";
      return hipErrorNotSupported;
    }
  lc.any = false;
  return hipSuccess;
}
hipError_t lik_set_observation(LikCtx&, const float* const*, hipStream_t) { return hipSuccess; }
hipError_t lik_reset(LikCtx&, hipStream_t) { return hipSuccess; }
hipError_t lik_resume(LikCtx&, hipStream_t) { return hipSuccess; }
hipError_t lik_update(LikCtx&, float2* const*, hipStream_t) { return hipSuccess; }
void lik_destroy(LikCtx&) {}
void lik_timing(LikCtx&, bool, bool) {}
hipError_t lik_timing_read(LikCtx&, double& ms, int& n) { ms = 0; n = 0; return hipSuccess; }

}  // namespace eptv
