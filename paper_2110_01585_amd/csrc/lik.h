// Likelihood-site update q_{x,0} (Eqs. (tilted_P_1) and (update_q0_x)) for the
// non-identity operators: interface between the host schedule and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "ep_tv_internal.h"

namespace eptv {

constexpr int kMaxTaps = 17;

inline bool fft_size_ok(int n) { return n >= 4 && n <= 4096 && (n & (n - 1)) == 0; }

struct LikInstInfo {
  int op = 0, H = 0, W = 0, pitch = 0;
  long long off = 0;
  double xi = 1.0, damping = 1.0;
  const float* taps = nullptr;
  int th = 0, tw = 0;
  const uint8_t* mask = nullptr;
  int tile0 = 0, ntiles = 0;
};

struct LikLayout {
  size_t planes[8]{};
  int nplanes = 0;
  size_t extra = 0;
};

template <class Take>
void lik_layout(const LikInstInfo* li, int n, long long plane, Take&& take, LikLayout& L) {
  bool any = false;
  for (int i = 0; i < n; ++i) any = any || li[i].op != OP_IDENTITY;
  L.nplanes = any ? 6 : 0;
  for (int k = 0; k < L.nplanes; ++k) L.planes[k] = take(sizeof(float) * (size_t)plane);
  L.extra = take(4096);
}

struct LikCtx {
  bool any = false;
};

hipError_t lik_create(LikCtx& lc, const LikInstInfo* li, int n, char* ws, const LikLayout& L,
                      long long plane, InstDev* d_inst, InstState* d_st, int4* d_tiles, int ntiles,
                      float* ypix, hipStream_t s, std::string& err);
hipError_t lik_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s);
hipError_t lik_reset(LikCtx& lc, hipStream_t s);
hipError_t lik_resume(LikCtx& lc, hipStream_t s);
hipError_t lik_update(LikCtx& lc, float2* const S[5], hipStream_t s);
void lik_destroy(LikCtx& lc);
void lik_timing(LikCtx& lc, bool enable, bool clear);
hipError_t lik_timing_read(LikCtx& lc, double& ms, int& launches);

}  // namespace eptv
