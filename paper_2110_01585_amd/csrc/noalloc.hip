// Denoising (H = I, l1-TV) without any allocation: the entry point
// ep_tv_denoise_noalloc of include/ep_tv.h.  It runs the same kernels as a
// context created for one identity-operator instance (cold start, sweeps,
// finalisation, gather), with every per-call buffer in one file-scope device
// array instead of a caller workspace, for callers that cannot allocate (code
// under HIP graph capture, tight serving loops).  Each device holds its own copy
// of the array until the process ends; calls on one device share it, so calls
// that overlap on one device race.
#include <mutex>

#include "ep_tv.h"
#include "ep_tv_internal.h"

namespace eptv {

constexpr int kNoAllocMaxSide = 512;
constexpr int kNoAllocRows = 8;   // sweep tile height a context of this size starts with
constexpr size_t kNoAllocBytes = 24u << 20;

// 9 site planes (float2) + the observation plane of a 512 x 512 image at its
// 576-element row pitch come to 22.4 MB; the tile list and partials add < 64 KB.
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once per device).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

size_t take(size_t& cur, size_t bytes) {
  const size_t at = cur;
  cur = (cur + bytes + 255) / 256 * 256;
  return at;
}

// Instance descriptor, state and tile list written on the device, so that the
// call records only kernels and device-to-device copies.
__global__ void k_noalloc_setup(InstDev* inst, InstState* st, int4* tiles, float** tab0,
                                float** tab1, InstDev I, double lam, float* mean, float* var) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *inst = I;
    InstState s{};
    s.lam = s.lam_prev = lam;
    s.active = 1u;
    *st = s;
    tab0[0] = mean;
    tab1[0] = var;
  }
  if (t < I.ntiles) tiles[t] = make_int4(0, t / I.chunks, t % I.chunks, 0);
}

}  // namespace
}  // namespace eptv

using namespace eptv;

extern "C" int ep_tv_denoise_noalloc(int32_t height, int32_t width, int32_t boundary,
                                     double noise_var, double lambda, double damping,
                                     int32_t n_sweeps, int32_t em_enabled, const float* d_y,
                                     float* d_mean, float* d_var, void* hip_stream) {
  if (height < 1 || width < 1 || height > kNoAllocMaxSide || width > kNoAllocMaxSide)
    return EP_TV_E_ARG;
  if (boundary != EP_TV_BND_FREE && boundary != EP_TV_BND_PERIODIC) return EP_TV_E_ARG;
  if (boundary == EP_TV_BND_PERIODIC && (height % 2 || width % 2 || height < 2 || width < 2))
    return EP_TV_E_ARG;
  if (!(noise_var > 0.0) || !(noise_var < HUGE_VAL) || !(lambda > 0.0) || !(lambda < HUGE_VAL) ||
      !(damping > 0.0 && damping <= 1.0) || n_sweeps < 0 || !d_y || !d_mean || !d_var)
    return EP_TV_E_ARG;
  const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  char* base = nullptr;
  if (scratch_ptr(reinterpret_cast<void**>(&base)) != hipSuccess) return EP_TV_E_HIP;

  // layout of one instance (the same pitch and tiling as a context's)
  InstDev I{};
  I.H = height;
  I.W = width;
  I.pitch = (width + 1 + 63) / 64 * 64;
  I.bnd = boundary;
  I.off = 0;
  I.op = OP_IDENTITY;
  I.strips = (width + kStripInt - 1) / kStripInt;
  I.chunks = (height + kNoAllocRows - 1) / kNoAllocRows;
  I.tile0 = 0;
  I.ntiles = I.strips * I.chunks;
  I.chunk_rows = kNoAllocRows;
  I.npix = height * width;
  I.xi = (float)noise_var;
  I.inv_xi = (float)(1.0 / noise_var);
  I.alpha = (float)damping;
  const size_t plane = (size_t)I.pitch * height;
  size_t cur = 0;
  const size_t o_s0 = take(cur, sizeof(float2) * plane);
  size_t o_sb[2][4];
  for (int b = 0; b < 2; ++b)
    for (int k = 0; k < 4; ++k) o_sb[b][k] = take(cur, sizeof(float2) * plane);
  const size_t o_y = take(cur, sizeof(float) * plane);
  const size_t o_inst = take(cur, sizeof(InstDev));
  const size_t o_st = take(cur, sizeof(InstState));
  const size_t o_tiles = take(cur, sizeof(int4) * I.ntiles);
  const size_t o_pe = take(cur, sizeof(double) * I.ntiles);
  const size_t o_pm = take(cur, sizeof(float) * I.ntiles);
  const size_t o_pv = take(cur, sizeof(float) * I.ntiles);
  const size_t o_pc = take(cur, sizeof(unsigned) * I.ntiles);
  const size_t o_pf = take(cur, sizeof(unsigned) * I.ntiles);
  const size_t o_t0 = take(cur, sizeof(float*));
  const size_t o_t1 = take(cur, sizeof(float*));
  if (cur > kNoAllocBytes) return EP_TV_E_ARG;

  float2* S0 = reinterpret_cast<float2*>(base + o_s0);
  float2* SB[2][4];
  for (int b = 0; b < 2; ++b)
    for (int k = 0; k < 4; ++k) SB[b][k] = reinterpret_cast<float2*>(base + o_sb[b][k]);
  float* ypix = reinterpret_cast<float*>(base + o_y);
  InstDev* d_inst = reinterpret_cast<InstDev*>(base + o_inst);
  InstState* d_st = reinterpret_cast<InstState*>(base + o_st);
  int4* d_tiles = reinterpret_cast<int4*>(base + o_tiles);
  float** tab0 = reinterpret_cast<float**>(base + o_t0);
  float** tab1 = reinterpret_cast<float**>(base + o_t1);

  hipLaunchKernelGGL(k_noalloc_setup, dim3((I.ntiles + 255) / 256), dim3(256), 0, s, d_inst, d_st,
                     d_tiles, tab0, tab1, I, lambda, d_mean, d_var);
  if (hipGetLastError() != hipSuccess) return EP_TV_E_HIP;
  if (hipMemcpy2DAsync(ypix, sizeof(float) * I.pitch, d_y, sizeof(float) * width,
                       sizeof(float) * width, height, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return EP_TV_E_HIP;
  if (launch_yrange(ypix, d_inst, d_st, 1, d_tiles, I.ntiles, reinterpret_cast<float*>(base + o_pm),
                    reinterpret_cast<float*>(base + o_pv), s) != hipSuccess)
    return EP_TV_E_HIP;
  int par = 0;
  float2* S[5] = {S0, SB[0][0], SB[0][1], SB[0][2], SB[0][3]};
  if (launch_init_cold(S, ypix, d_inst, d_st, d_tiles, I.ntiles, s) != hipSuccess) return EP_TV_E_HIP;

  SweepArgs a{};
  a.S0 = S0;
  a.inst = d_inst;
  a.st = d_st;
  a.tiles = d_tiles;
  a.ntiles = I.ntiles;
  a.part_eabs = reinterpret_cast<double*>(base + o_pe);
  a.part_dmu = reinterpret_cast<float*>(base + o_pm);
  a.part_dv = reinterpret_cast<float*>(base + o_pv);
  a.part_clamp = reinterpret_cast<unsigned*>(base + o_pc);
  a.part_flags = reinterpret_cast<unsigned*>(base + o_pf);
  a.part_mu = a.part_dmu;   // never read: an identity instance has no likelihood tiles
  a.prior = PRIOR_L1;
  for (int t = 0; t < n_sweeps; ++t) {
    a.I1 = SB[par][0]; a.I2 = SB[par][1]; a.I3 = SB[par][2]; a.I4 = SB[par][3];
    a.O1 = SB[par ^ 1][0]; a.O2 = SB[par ^ 1][1]; a.O3 = SB[par ^ 1][2]; a.O4 = SB[par ^ 1][3];
    if (launch_tv_sweep(a, false, s) != hipSuccess) return EP_TV_E_HIP;
    if (launch_finalize(d_inst, d_st, 1, a, em_enabled ? 1 : 0, 0.0, s) != hipSuccess)
      return EP_TV_E_HIP;
    par ^= 1;
  }
  for (int k = 0; k < 4; ++k) S[k + 1] = SB[par][k];
  if (launch_marginals(S, d_inst, d_tiles, I.ntiles, tab0, tab1, s) != hipSuccess) return EP_TV_E_HIP;
  return EP_TV_OK;
}
