// Learned warm start: a 6-layer 3x3 convolutional network (channels 1 -> 32 ->
// 32 -> 32 -> 32 -> 32 -> 2, ReLU after layers 1..5, zero padding) that maps a
// normalised observation x0 = (y - m) / s (m, s: image mean and standard
// deviation) to o = (o0, o1), read as the posterior mean m + s o0 and the
// posterior variance xi exp(o1).  Inference, loss gradient and Adam updates.
//
// Precision: weights, activations and back-propagated activation gradients are
// stored in bfloat16 (round to nearest even), every sum is accumulated in
// float32, per-block partial sums of weight gradients are reduced in float64 in
// a fixed order, master weights and Adam moments are float32.
//
// Layouts: activations are NHWC with 32 channels (64 bytes per pixel).  The
// 32 -> 32 layers run on v_mfma_f32_16x16x32_bf16 (lane l of a wave holds row
// l%16 and k-slice 8*(l/16)..+7 of A, the same k-slice and column l%16 of B, and
// rows 4*(l/16)..+3 of column l%16 of D):
//   forward / input gradient: D[out channel][pixel] = sum over taps of
//     W_tap[out][in] x X[in][pixel], A = weights (per-wave registers, all 9 taps),
//     B = 16 pixels x 8 channels read from the block's input tile staged in LDS;
//   weight gradient: D[in][out] = sum over pixels X[pixel + tap][in] G[pixel][out],
//     with both operands transposed through LDS (pixels contiguous).
// The 1 -> 32 and 32 -> 2 layers are plain float32 FMAs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ep_tv_net.h"

namespace eptv_net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int C = 32;                 // hidden channels
constexpr int kW1 = 9 * 1 * C;        // 288
constexpr int kW32 = 9 * C * C;       // 9216
constexpr int kW6 = 9 * C * 2;        // 576
// canonical parameter offsets (W then b per layer)
constexpr int kOffW1 = 0, kOffB1 = kW1;
constexpr int kOff2 = kW1 + C;                     // layer 2 weights
constexpr int kStride32 = kW32 + C;                // one 32 -> 32 layer
constexpr int kOffW6 = kOff2 + 4 * kStride32, kOffB6 = kOffW6 + kW6;
constexpr int kParams = kOffB6 + 2;                // 37890
constexpr int kTile = 32;                          // weight-gradient block tile (pixels per side)
constexpr int kPartStride = kW32 + C;              // floats per block partial (largest layer)
constexpr float kSFloor = 1e-6f;

static_assert(kParams == 37890, "parameter count");

// ---------------------------------------------------------------- bf16 helpers
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t h) { return h != 0 && !(h & 0x8000u); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

struct NetDev {
  const float* master;       // canonical float32 parameters (caller-owned)
  uint16_t* wf;              // 4 x [9][32 out][32 in]: forward A operands, layers 2..5
  uint16_t* wd;              // 4 x [9][32 in][32 out]: input-gradient A operands (taps reversed)
  float* w1r;                // [9][32] layer-1 weights rounded to bf16
  float* w6r;                // [9][32][2] layer-6 weights rounded to bf16
  float* grad;               // canonical gradient
  float* adam_m;
  float* adam_v;
  float2* stats;             // per image (m, s)
  uint16_t* act[5];          // a1..a5
  float* o;                  // layer-6 output / loss gradient (float2 per pixel)
  uint16_t* g[2];            // activation gradients (ping-pong)
  float* part;               // weight-gradient partials
  double* loss_part;
  double2* stats_part;       // per image and stats block: (sum y, sum y^2)
  double* red_part;          // per chunk of weight-gradient partial blocks and parameter
};

// partial blocks per image of the statistics pass, chunks of the weight-gradient
// partial blocks summed in the first reduction step
constexpr int kStatBlocks = 256;
constexpr int kRedChunks = 32;

// ---------------------------------------------------------------- image statistics
// Mean and standard deviation of each image, in two steps so that the whole
// chip reads the images: kStatBlocks blocks per image sum contiguous slices
// (FP64, a wave butterfly and the four wave totals in a fixed order), then one
// block per image sums those partials in a fixed order.
__device__ __forceinline__ void block_sum2(double& s1, double& s2) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
  }
  __shared__ double a[4], b[4];
  if ((threadIdx.x & 63) == 0) {
    a[threadIdx.x >> 6] = s1;
    b[threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  s1 = (a[0] + a[1]) + (a[2] + a[3]);
  s2 = (b[0] + b[1]) + (b[2] + b[3]);
}

__global__ __launch_bounds__(256) void k_stats_part(const float* __restrict__ y, int H, int W,
                                                    double2* __restrict__ part) {
  const int n = blockIdx.y;
  const long long np = (long long)H * W;
  const long long per = (np + kStatBlocks - 1) / kStatBlocks;
  const long long i0 = (long long)blockIdx.x * per;
  const long long i1 = i0 + per < np ? i0 + per : np;
  const float* yi = y + (long long)n * np;
  double s1 = 0.0, s2 = 0.0;
  constexpr int kU = 8;   // loads in flight per thread
  for (long long b = i0 + threadIdx.x; b < i1; b += kU * 256) {
    float v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long i = b + (long long)u * 256;
      v[u] = i < i1 ? yi[i] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      s1 += (double)v[u];
      s2 += (double)v[u] * (double)v[u];
    }
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) part[(long long)n * kStatBlocks + blockIdx.x] = make_double2(s1, s2);
}

__global__ __launch_bounds__(256) void k_stats_fin(const double2* __restrict__ part, int H, int W,
                                                   float2* __restrict__ stats) {
  static_assert(kStatBlocks == 256, "one partial per thread");
  const int n = blockIdx.x;
  const long long np = (long long)H * W;
  const double2 p = part[(long long)n * kStatBlocks + threadIdx.x];
  double s1 = p.x, s2 = p.y;
  block_sum2(s1, s2);
  if (threadIdx.x == 0) {
    const double m = s1 / (double)np;
    double var = s2 / (double)np - m * m;
    // second pass is not needed at the precision the network uses; guard round-off
    if (var < 0.0) var = 0.0;
    double sd = sqrt(var);
    if (sd < kSFloor) sd = kSFloor;
    stats[n] = make_float2((float)m, (float)sd);
  }
}

// ---------------------------------------------------------------- layer 1 (1 -> 32)
__global__ __launch_bounds__(256) void k_conv1(const float* __restrict__ y,
                                               const float2* __restrict__ stats,
                                               const float* __restrict__ w1r,
                                               const float* __restrict__ b1,
                                               uint16_t* __restrict__ out, int B, int H, int W) {
  __shared__ float sw[kW1 + C];
  for (int i = threadIdx.x; i < kW1 + C; i += blockDim.x) sw[i] = i < kW1 ? w1r[i] : b1[i - kW1];
  __syncthreads();
  const long long np = (long long)H * W;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)B * np) return;
  const int n = (int)(gid / np);
  const int rem = (int)(gid % np);
  const int r = rem / W, c = rem % W;
  const float2 ms = stats[n];
  const float* yi = y + (long long)n * np;
  float x[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int rr = r + a - 1, cc = c + b - 1;
      x[3 * a + b] = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? (yi[rr * W + cc] - ms.x) / ms.y : 0.f;
    }
  uint16_t* po = out + gid * C;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint16_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int co = 8 * q + e;
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < 9; ++t) acc += x[t] * sw[t * C + co];
      h[e] = f2bf(fmaxf(acc + sw[kW1 + co], 0.f));
    }
    uint4 v;
    v.x = h[0] | ((uint32_t)h[1] << 16);
    v.y = h[2] | ((uint32_t)h[3] << 16);
    v.z = h[4] | ((uint32_t)h[5] << 16);
    v.w = h[6] | ((uint32_t)h[7] << 16);
    *reinterpret_cast<uint4*>(po + 8 * q) = v;
  }
}

// ---------------------------------------------------------------- 32 -> 32 conv on MFMA
enum { EPI_RELU = 0, EPI_MASK = 1 };

// grid (ceil(W / 64), ceil(H / 16), B), 256 threads.  A block takes columns
// 64 * blockIdx.x .. +63 of rows 16 * blockIdx.y .. +15 in four steps of four
// rows; in each step wave w takes row +w, in four groups of 16 columns.  The
// weights of all nine taps stay in registers across the steps.  Each step's
// input tile (rows -1 .. +4 and columns -1 .. +64 around its outputs, zero
// outside the image: 6 x 66 pixels x 64 bytes) is staged in LDS as 16-byte
// words ordered [k-slice][row][column], so the 16 lanes of a k-slice read 16
// consecutive words for each tap instead of gathering them from global memory
// nine times.
constexpr int kConvTR = 6, kConvTC = 66;                 // staged tile rows, columns
constexpr int kConvWords = 4 * kConvTR * kConvTC;        // 16-byte words per tile (1,584, 25,344 bytes)
constexpr int kConvSteps = 4;                            // four-row steps per block
static_assert(kConvWords <= 8 * 256, "two staging rounds of four words per thread");
template <int EPI>
__global__ __launch_bounds__(256) void k_conv32(const uint16_t* __restrict__ in,
                                                const uint16_t* __restrict__ wa,
                                                const float* __restrict__ bias,
                                                const uint16_t* __restrict__ mask,
                                                uint16_t* __restrict__ out, int H, int W) {
  // two tile buffers: a step stages into one while slower waves may still read
  // the previous step's tile from the other; the barrier after staging step s
  // is passed only once every wave has finished step s - 1, so step s + 1 can
  // overwrite that step's buffer
  __shared__ bf16x8 X[2][kConvWords];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, pl = lane & 15;
  const int n = blockIdx.z;
  const int c0 = blockIdx.x * 64;
  const long long img = (long long)n * H * W;
  bf16x8 A[9][2];
  float bv[2][4];
  for (int step = 0; step < kConvSteps; ++step) {
    const int r0 = (blockIdx.y * kConvSteps + step) * 4;
    if (r0 >= H) break;                           // uniform over the block
    const int r = r0 + wave;
    bf16x8* T = X[step & 1];
    // stage: word w = (tile row, tile column, k-slice) in global order (a tile
    // row's 66 pixels are contiguous in NHWC), stored at [k-slice][row][column]
    // in two rounds of four words per thread, each round's loads in flight
    // together (the weights stay in registers, so the rounds are kept short)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int w = (int)threadIdx.x + 256 * (4 * h + u);
        v[u] = zero8();
        if (w >= kConvWords) continue;
        const int tr = w / (4 * kConvTC), rem = w - tr * (4 * kConvTC);
        const int rr = r0 - 1 + tr, cc = c0 - 1 + (rem >> 2);
        if (rr >= 0 && rr < H && cc >= 0 && cc < W)
          v[u] = ld8(in + (img + (long long)rr * W + cc) * C + 8 * (rem & 3));
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int w = (int)threadIdx.x + 256 * (4 * h + u);
        if (w >= kConvWords) continue;
        const int tr = w / (4 * kConvTC), rem = w - tr * (4 * kConvTC);
        T[((rem & 3) * kConvTR + tr) * kConvTC + (rem >> 2)] = v[u];
      }
    }
    if (step == 0) {
#pragma unroll
      for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) A[t][mb] = ld8(wa + ((t * C + 16 * mb + pl) * C + 8 * q));
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[mb][i] = EPI == EPI_RELU ? bias[16 * mb + 4 * q + i] : 0.f;
    }
    __syncthreads();
    for (int g = 0; g < 4; ++g) {
      const int c = c0 + 16 * g + pl;
      if (c0 + 16 * g >= W) break;                // the whole group is right of the image
      f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          // tap (a, b) of output column c reads tile row wave + a, column 16 g + pl + b
          const bf16x8 xb = T[(q * kConvTR + wave + a) * kConvTC + 16 * g + pl + b];
          acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[3 * a + b][0], xb, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[3 * a + b][1], xb, acc1, 0, 0, 0);
        }
      }
      if (r >= H || c >= W) continue;
      const long long px = img + (long long)r * W + c;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const f4 acc = mb ? acc1 : acc0;
        const int ch = 16 * mb + 4 * q;
        uint16_t h[4];
        if (EPI == EPI_RELU) {
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = f2bf(fmaxf(acc[i] + bv[mb][i], 0.f));
        } else {
          const uint2 mv = *reinterpret_cast<const uint2*>(mask + px * C + ch);
          const uint16_t m4[4] = {(uint16_t)(mv.x & 0xffff), (uint16_t)(mv.x >> 16),
                                  (uint16_t)(mv.y & 0xffff), (uint16_t)(mv.y >> 16)};
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = bf_pos(m4[i]) ? f2bf(acc[i]) : (uint16_t)0;
        }
        uint2 v;
        v.x = h[0] | ((uint32_t)h[1] << 16);
        v.y = h[2] | ((uint32_t)h[3] << 16);
        *reinterpret_cast<uint2*>(out + px * C + ch) = v;
      }
    }
  }
}

// ---------------------------------------------------------------- layer 6 (32 -> 2) + outputs / loss
// One thread per pixel.  mode 0: write mu_hat = m + s o0, var_hat = xi exp(o1).
// mode 1: targets t0 = (mu - m) / s, t1 = log(v / xi); write dL/do = 2 (o - t) / N_total
// into o_out and per-block loss partials.
__global__ __launch_bounds__(256) void k_conv6(const uint16_t* __restrict__ a5,
                                               const float* __restrict__ w6r,
                                               const float* __restrict__ b6,
                                               const float2* __restrict__ stats, int B, int H, int W,
                                               float xi, int mode, float* __restrict__ mu_out,
                                               float* __restrict__ var_out,
                                               const float* __restrict__ mu_t,
                                               const float* __restrict__ v_t,
                                               float* __restrict__ g_out,
                                               double* __restrict__ loss_part) {
  __shared__ float sw[kW6 + 2];
  for (int i = threadIdx.x; i < kW6 + 2; i += blockDim.x) sw[i] = i < kW6 ? w6r[i] : b6[i - kW6];
  __syncthreads();
  const long long np = (long long)H * W;
  const long long total = (long long)B * np;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double lpart = 0.0;
  if (gid < total) {
    const int n = (int)(gid / np);
    const int rem = (int)(gid % np);
    const int r = rem / W, c = rem % W;
    float o0 = sw[kW6], o1 = sw[kW6 + 1];
    for (int a = 0; a < 3; ++a) {
      const int rr = r + a - 1;
      if (rr < 0 || rr >= H) continue;
      for (int b = 0; b < 3; ++b) {
        const int cc = c + b - 1;
        if (cc < 0 || cc >= W) continue;
        const uint16_t* px = a5 + ((long long)n * np + (long long)rr * W + cc) * C;
        const float* wt = sw + (3 * a + b) * C * 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint4 v = *reinterpret_cast<const uint4*>(px + 8 * q);
          const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float x = bf2f((uint16_t)((wv[e >> 1] >> (16 * (e & 1))) & 0xffff));
            o0 += x * wt[(8 * q + e) * 2];
            o1 += x * wt[(8 * q + e) * 2 + 1];
          }
        }
      }
    }
    const float2 ms = stats[n];
    if (mode == 0) {
      mu_out[gid] = ms.x + ms.y * o0;
      var_out[gid] = xi * expf(o1);
    } else {
      const float t0 = (mu_t[gid] - ms.x) / ms.y;
      const float t1 = logf(v_t[gid] / xi);
      const float d0 = o0 - t0, d1 = o1 - t1;
      const float sc = 2.0f / (float)total;
      g_out[2 * gid] = sc * d0;
      g_out[2 * gid + 1] = sc * d1;
      lpart = (double)d0 * d0 + (double)d1 * d1;
    }
  }
  if (mode == 1) {
    __shared__ double red[256];
    red[threadIdx.x] = lpart;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
  }
}

// input gradient of layer 6: g5[p][i] = sum_{a,b,o} g6[p - (a-1, b-1)][o] W6[a][b][i][o],
// times the ReLU mask of a5, stored bf16.  One thread per pixel.
__global__ __launch_bounds__(256) void k_dgrad6(const float* __restrict__ g6,
                                                const float* __restrict__ w6r,
                                                const uint16_t* __restrict__ a5,
                                                uint16_t* __restrict__ g5, int B, int H, int W) {
  __shared__ float sw[kW6];
  for (int i = threadIdx.x; i < kW6; i += blockDim.x) sw[i] = w6r[i];
  __syncthreads();
  const long long np = (long long)H * W;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)B * np) return;
  const int n = (int)(gid / np);
  const int rem = (int)(gid % np);
  const int r = rem / W, c = rem % W;
  float acc[C];
#pragma unroll
  for (int i = 0; i < C; ++i) acc[i] = 0.f;
  for (int a = 0; a < 3; ++a) {
    const int rr = r - a + 1;
    if (rr < 0 || rr >= H) continue;
    for (int b = 0; b < 3; ++b) {
      const int cc = c - b + 1;
      if (cc < 0 || cc >= W) continue;
      const float2 gv = *reinterpret_cast<const float2*>(g6 + 2 * ((long long)n * np + (long long)rr * W + cc));
      const float* wt = sw + (3 * a + b) * C * 2;
#pragma unroll
      for (int i = 0; i < C; ++i) acc[i] += gv.x * wt[2 * i] + gv.y * wt[2 * i + 1];
    }
  }
  const uint16_t* mp = a5 + gid * C;
  uint16_t* po = g5 + gid * C;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint4 mv = *reinterpret_cast<const uint4*>(mp + 8 * q);
    const uint32_t mw[4] = {mv.x, mv.y, mv.z, mv.w};
    uint32_t ow[4];
#pragma unroll
    for (int e2 = 0; e2 < 4; ++e2) {
      const uint16_t m0 = (uint16_t)(mw[e2] & 0xffff), m1 = (uint16_t)(mw[e2] >> 16);
      const uint16_t h0 = bf_pos(m0) ? f2bf(acc[8 * q + 2 * e2]) : (uint16_t)0;
      const uint16_t h1 = bf_pos(m1) ? f2bf(acc[8 * q + 2 * e2 + 1]) : (uint16_t)0;
      ow[e2] = h0 | ((uint32_t)h1 << 16);
    }
    *reinterpret_cast<uint4*>(po + 8 * q) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
  }
}

// ---------------------------------------------------------------- weight gradients
// Block tile: 32 x 32 output pixels of one image, processed as four 8-row
// sub-tiles; grid (ceil(W / 32), ceil(H / 32), B).  Partial sums per block are
// written in canonical order ([tap][in][out] then bias[out]).
__device__ __forceinline__ int part_block() {
  return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

// 32 -> 32 layers on MFMA.  XT[s][ch][hr][c] holds X[r0 - 1 + hr][c0 - 1 + c + s]
// (three column shifts so every 8-pixel k-slice is 16-byte aligned), GT[ch][row][c]
// holds G[r0 + row][c0 + c].
__global__ __launch_bounds__(256) void k_wgrad32(const uint16_t* __restrict__ x,
                                                 const uint16_t* __restrict__ g,
                                                 float* __restrict__ part, int H, int W) {
  __shared__ __attribute__((aligned(16))) uint16_t XT[3 * C * 10 * 32];
  __shared__ __attribute__((aligned(16))) uint16_t GT[C * 8 * 32];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, pl = lane & 15;
  const int cb = wave >> 1, ob = wave & 1;   // in-channel block, out-channel block of this wave
  const int n = blockIdx.z;
  const long long img = (long long)n * H * W;
  f4 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = (f4){0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  for (int s = 0; s < 4; ++s) {
    const int r0 = blockIdx.y * kTile + 8 * s, c0 = blockIdx.x * kTile;
    __syncthreads();
    for (int it = tid; it < 10 * 34 * 4; it += 256) {
      const int hr = it / 136, rem = it % 136, hc = rem >> 2, qq = rem & 3;
      const int rr = r0 - 1 + hr, cc = c0 - 1 + hc;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (rr >= 0 && rr < H && cc >= 0 && cc < W)
        v = *reinterpret_cast<const uint4*>(x + (img + (long long)rr * W + cc) * C + 8 * qq);
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int sh = 0; sh < 3; ++sh) {
        const int cp = hc - sh;
        if (cp < 0 || cp >= 32) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          XT[((sh * C + 8 * qq + e) * 10 + hr) * 32 + cp] = (uint16_t)((w4[e >> 1] >> (16 * (e & 1))) & 0xffff);
      }
    }
    for (int it = tid; it < 8 * 32 * 4; it += 256) {
      const int row = it >> 7, rem = it & 127, col = rem >> 2, qq = rem & 3;
      const int rr = r0 + row, cc = c0 + col;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (rr < H && cc < W) v = *reinterpret_cast<const uint4*>(g + (img + (long long)rr * W + cc) * C + 8 * qq);
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 8; ++e)
        GT[((8 * qq + e) * 8 + row) * 32 + col] = (uint16_t)((w4[e >> 1] >> (16 * (e & 1))) & 0xffff);
    }
    __syncthreads();
    if (tid < C) {
      const uint16_t* gp = GT + tid * 8 * 32;
      for (int k = 0; k < 8 * 32; ++k) bsum += bf2f(gp[k]);
    }
    for (int i = 0; i < 8; ++i) {
      const bf16x8 bop = ld8(GT + ((16 * ob + pl) * 8 + i) * 32 + 8 * q);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const bf16x8 aop = ld8(XT + ((b * C + 16 * cb + pl) * 10 + i + a) * 32 + 8 * q);
          acc[3 * a + b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[3 * a + b], 0, 0, 0);
        }
    }
  }
  float* pp = part + (long long)part_block() * kPartStride;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) pp[(t * C + 16 * cb + 4 * q + i) * C + 16 * ob + pl] = acc[t][i];
  if (tid < C) pp[kW32 + tid] = bsum;
}

// layer 6: dW6[a][b][i][o] = sum_p a5[p + (a-1, b-1)][i] g6[p][o]; thread = (tap, i) pair
__global__ __launch_bounds__(256) void k_wgrad6(const uint16_t* __restrict__ x,
                                                const float* __restrict__ g6,
                                                float* __restrict__ part, int H, int W) {
  __shared__ float XS[10 * 34 * C];
  __shared__ float GS[8 * 32 * 2];
  const int tid = threadIdx.x;
  const int n = blockIdx.z;
  const long long img = (long long)n * H * W;
  float acc[2][2] = {{0.f, 0.f}, {0.f, 0.f}};   // up to two (tap, i) pairs per thread
  float bs0 = 0.f, bs1 = 0.f;
  for (int s = 0; s < 4; ++s) {
    const int r0 = blockIdx.y * kTile + 8 * s, c0 = blockIdx.x * kTile;
    __syncthreads();
    for (int it = tid; it < 10 * 34 * C; it += 256) {
      const int hr = it / (34 * C), rem = it % (34 * C), hc = rem / C, ch = rem % C;
      const int rr = r0 - 1 + hr, cc = c0 - 1 + hc;
      XS[it] = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? bf2f(x[(img + (long long)rr * W + cc) * C + ch]) : 0.f;
    }
    for (int it = tid; it < 8 * 32 * 2; it += 256) {
      const int row = it / 64, rem = it % 64, col = rem >> 1, o = rem & 1;
      const int rr = r0 + row, cc = c0 + col;
      GS[it] = (rr < H && cc < W) ? g6[2 * (img + (long long)rr * W + cc) + o] : 0.f;
    }
    __syncthreads();
    for (int pi = 0; pi < 2; ++pi) {
      const int pair = tid + 256 * pi;
      if (pair >= 9 * C) break;
      const int t = pair / C, i = pair % C, a = t / 3, b = t % 3;
      float s0 = 0.f, s1 = 0.f;
      for (int row = 0; row < 8; ++row)
        for (int col = 0; col < 32; ++col) {
          const float xv = XS[((row + a) * 34 + col + b) * C + i];
          s0 += xv * GS[(row * 32 + col) * 2];
          s1 += xv * GS[(row * 32 + col) * 2 + 1];
        }
      acc[pi][0] += s0;
      acc[pi][1] += s1;
    }
    if (tid < 2) {
      float sb = 0.f;
      for (int k = 0; k < 256; ++k) sb += GS[2 * k + tid];
      if (tid == 0) bs0 += sb; else bs1 += sb;
    }
  }
  float* pp = part + (long long)part_block() * kPartStride;
  for (int pi = 0; pi < 2; ++pi) {
    const int pair = tid + 256 * pi;
    if (pair >= 9 * C) break;
    pp[2 * pair] = acc[pi][0];
    pp[2 * pair + 1] = acc[pi][1];
  }
  if (tid == 0) pp[kW6] = bs0;
  if (tid == 1) pp[kW6 + 1] = bs1;
}

// layer 1: dW1[a][b][0][o] = sum_p x0[p + (a-1, b-1)] g1[p][o]; thread = (tap, o) pair
__global__ __launch_bounds__(256) void k_wgrad1(const float* __restrict__ y,
                                                const float2* __restrict__ stats,
                                                const uint16_t* __restrict__ g1,
                                                float* __restrict__ part, int H, int W) {
  __shared__ float XS[10 * 34];
  __shared__ float GS[8 * 32 * C];
  const int tid = threadIdx.x;
  const int n = blockIdx.z;
  const long long img = (long long)n * H * W;
  const float2 ms = stats[n];
  float acc[2] = {0.f, 0.f};
  float bsum = 0.f;
  for (int s = 0; s < 4; ++s) {
    const int r0 = blockIdx.y * kTile + 8 * s, c0 = blockIdx.x * kTile;
    __syncthreads();
    for (int it = tid; it < 10 * 34; it += 256) {
      const int hr = it / 34, hc = it % 34;
      const int rr = r0 - 1 + hr, cc = c0 - 1 + hc;
      XS[it] = (rr >= 0 && rr < H && cc >= 0 && cc < W) ? (y[img + (long long)rr * W + cc] - ms.x) / ms.y : 0.f;
    }
    for (int it = tid; it < 8 * 32 * C; it += 256) {
      const int row = it / (32 * C), rem = it % (32 * C), col = rem / C, ch = rem % C;
      const int rr = r0 + row, cc = c0 + col;
      GS[it] = (rr < H && cc < W) ? bf2f(g1[(img + (long long)rr * W + cc) * C + ch]) : 0.f;
    }
    __syncthreads();
    for (int pi = 0; pi < 2; ++pi) {
      const int pair = tid + 256 * pi;
      if (pair >= 9 * C) break;
      const int t = pair / C, o = pair % C, a = t / 3, b = t % 3;
      float sacc = 0.f;
      for (int row = 0; row < 8; ++row)
        for (int col = 0; col < 32; ++col) sacc += XS[(row + a) * 34 + col + b] * GS[(row * 32 + col) * C + o];
      acc[pi] += sacc;
    }
    if (tid < C) {
      float sb = 0.f;
      for (int k = 0; k < 256; ++k) sb += GS[k * C + tid];
      bsum += sb;
    }
  }
  float* pp = part + (long long)part_block() * kPartStride;
  for (int pi = 0; pi < 2; ++pi) {
    const int pair = tid + 256 * pi;
    if (pair >= 9 * C) break;
    pp[pair] = acc[pi];
  }
  if (tid < C) pp[kW1 + tid] = bsum;
}

// Fixed-order float64 sum of the per-block partials into the canonical
// gradient, in two steps: chunk c of kRedChunks sums its contiguous range of
// partial blocks in ascending order, then the chunk sums are added in
// ascending chunk order.
__global__ __launch_bounds__(256) void k_reduce_chunks(const float* __restrict__ part, int nblocks,
                                                       int count, double* __restrict__ red) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int per = (nblocks + kRedChunks - 1) / kRedChunks;
  const int b0 = blockIdx.y * per, b1 = min(b0 + per, nblocks);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += part[(long long)b * kPartStride + k];
  red[(long long)blockIdx.y * count + k] = s;
}

__global__ __launch_bounds__(256) void k_reduce_fin(const double* __restrict__ red, int count,
                                                    float* __restrict__ grad_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  double s = 0.0;
#pragma unroll 8
  for (int c = 0; c < kRedChunks; ++c) s += red[(long long)c * count + k];
  grad_out[k] = (float)s;
}

__global__ __launch_bounds__(256) void k_loss_sum(const double* __restrict__ lp, int n, double scale,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += lp[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] * scale;
}

// ---------------------------------------------------------------- optimiser and weight copies
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ w, uint16_t* __restrict__ wf,
                                              uint16_t* __restrict__ wd, float* __restrict__ w1r,
                                              float* __restrict__ w6r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kW1) w1r[i] = bf2f(f2bf(w[kOffW1 + i]));
  if (i < kW6) w6r[i] = bf2f(f2bf(w[kOffW6 + i]));
  if (i < 4 * kW32) {
    const int l = i / kW32, k = i % kW32;          // canonical [t][in][out]
    const int t = k / (C * C), ci = (k / C) % C, co = k % C;
    const uint16_t h = f2bf(w[kOff2 + l * kStride32 + k]);
    wf[l * kW32 + (t * C + co) * C + ci] = h;              // [t][out][in]
    wd[l * kW32 + ((8 - t) * C + ci) * C + co] = h;        // [8 - t][in][out]
  }
}

}  // namespace eptv_net

// ==================================================================== host side
using namespace eptv_net;

struct ep_tv_net {
  NetDev d{};
  float* master = nullptr;
  int max_batch = 0, max_h = 0, max_w = 0;
  long long max_px = 0;
  int adam_t = 0;
  bool have_grad = false;
  hipStream_t stream = nullptr;
  std::string err;
  double* d_loss = nullptr;
};

namespace {

constexpr size_t kAlign = 256;
size_t rup(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct NetLayout {
  size_t wf, wd, w1r, w6r, grad, am, av, stats, act[5], o, g[2], part, loss_part, loss, stats_part,
      red_part, total;
  long long nblk, nloss;
};

bool net_layout(int max_batch, int max_h, int max_w, NetLayout& L) {
  if (max_batch < 1 || max_h < 1 || max_w < 1 || max_batch > 65535 || max_h > 16384 || max_w > 16384)
    return false;
  const long long P = (long long)max_batch * max_h * max_w;
  L.nblk = (long long)max_batch * ((max_h + kTile - 1) / kTile) * ((max_w + kTile - 1) / kTile);
  L.nloss = (P + 255) / 256;
  size_t cur = 0;
  auto take = [&](size_t b) { size_t at = cur; cur = rup(cur + b); return at; };
  L.wf = take(4 * kW32 * 2);
  L.wd = take(4 * kW32 * 2);
  L.w1r = take(kW1 * 4);
  L.w6r = take(kW6 * 4);
  L.grad = take(kParams * 4);
  L.am = take(kParams * 4);
  L.av = take(kParams * 4);
  L.stats = take((size_t)max_batch * 8);
  for (int k = 0; k < 5; ++k) L.act[k] = take((size_t)P * C * 2);
  L.o = take((size_t)P * 8);
  L.g[0] = take((size_t)P * C * 2);
  L.g[1] = take((size_t)P * C * 2);
  L.part = take((size_t)L.nblk * kPartStride * 4);
  L.loss_part = take((size_t)L.nloss * 8);
  L.loss = take(8);
  L.stats_part = take((size_t)max_batch * kStatBlocks * 16);
  L.red_part = take((size_t)kRedChunks * kStride32 * 8);
  L.total = cur;
  return true;
}

int fail(ep_tv_net* n, int code, const std::string& m) {
  if (n) n->err = m;
  return code;
}

int hipchk(ep_tv_net* n, hipError_t e, const char* what) {
  if (e == hipSuccess) return EP_TV_OK;
  return fail(n, EP_TV_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define NCHK(n, expr)                                   \
  do {                                                  \
    int _rc = hipchk((n), (expr), #expr);               \
    if (_rc != EP_TV_OK) return _rc;                \
  } while (0)

int check_shape(ep_tv_net* n, int batch, int h, int w) {
  if (batch < 1 || h < 1 || w < 1 || batch > n->max_batch || h > n->max_h || w > n->max_w)
    return fail(n, EP_TV_E_ARG, "batch / size outside the limits the network was created for");
  return EP_TV_OK;
}

hipError_t pack(ep_tv_net* n) {
  hipLaunchKernelGGL(k_pack, dim3((4 * kW32 + 255) / 256), dim3(256), 0, n->stream, n->master, n->d.wf,
                     n->d.wd, n->d.w1r, n->d.w6r);
  return hipGetLastError();
}

// canonical gradient of `count` parameters from the nblk per-block partials
void reduce_grad(ep_tv_net* n, int nblk, int count, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_chunks, dim3((count + 255) / 256, kRedChunks), dim3(256), 0, s, n->d.part,
                     nblk, count, n->d.red_part);
  hipLaunchKernelGGL(k_reduce_fin, dim3((count + 255) / 256), dim3(256), 0, s, n->d.red_part, count, out);
}

// forward pass up to a5 (stats, layers 1..5)
hipError_t forward5(ep_tv_net* n, const float* y, int B, int H, int W) {
  const hipStream_t s = n->stream;
  const long long P = (long long)B * H * W;
  hipLaunchKernelGGL(k_stats_part, dim3(kStatBlocks, B), dim3(256), 0, s, y, H, W, n->d.stats_part);
  hipLaunchKernelGGL(k_stats_fin, dim3(B), dim3(256), 0, s, n->d.stats_part, H, W, n->d.stats);
  hipLaunchKernelGGL(k_conv1, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, y, n->d.stats, n->d.w1r,
                     n->master + kOffB1, n->d.act[0], B, H, W);
  const dim3 g((W + 63) / 64, (H + 4 * kConvSteps - 1) / (4 * kConvSteps), B);
  for (int l = 0; l < 4; ++l)
    hipLaunchKernelGGL((k_conv32<EPI_RELU>), g, dim3(256), 0, s, n->d.act[l], n->d.wf + l * kW32,
                       n->master + kOff2 + l * kStride32 + kW32, (const uint16_t*)nullptr, n->d.act[l + 1],
                       H, W);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int ep_tv_net_param_count(void) { return kParams; }

int ep_tv_net_workspace_bytes(int32_t max_batch, int32_t max_h, int32_t max_w, size_t* bytes) {
  if (!bytes) return EP_TV_E_ARG;
  NetLayout L;
  if (!net_layout(max_batch, max_h, max_w, L)) return EP_TV_E_ARG;
  *bytes = L.total;
  return EP_TV_OK;
}

int ep_tv_net_create(float* d_params, void* d_ws, size_t ws_bytes, int32_t max_batch, int32_t max_h,
                     int32_t max_w, void* hip_stream, ep_tv_net** out) {
  if (!out) return EP_TV_E_ARG;
  *out = nullptr;
  if (!d_params || !d_ws || reinterpret_cast<uintptr_t>(d_ws) % kAlign) return EP_TV_E_ARG;
  NetLayout L;
  if (!net_layout(max_batch, max_h, max_w, L)) return EP_TV_E_ARG;
  if (ws_bytes < L.total) return EP_TV_E_OOM;
  ep_tv_net* n = new ep_tv_net();
  char* ws = reinterpret_cast<char*>(d_ws);
  n->master = d_params;
  n->max_batch = max_batch; n->max_h = max_h; n->max_w = max_w;
  n->max_px = (long long)max_batch * max_h * max_w;
  n->stream = reinterpret_cast<hipStream_t>(hip_stream);
  NetDev& d = n->d;
  d.master = d_params;
  d.wf = reinterpret_cast<uint16_t*>(ws + L.wf);
  d.wd = reinterpret_cast<uint16_t*>(ws + L.wd);
  d.w1r = reinterpret_cast<float*>(ws + L.w1r);
  d.w6r = reinterpret_cast<float*>(ws + L.w6r);
  d.grad = reinterpret_cast<float*>(ws + L.grad);
  d.adam_m = reinterpret_cast<float*>(ws + L.am);
  d.adam_v = reinterpret_cast<float*>(ws + L.av);
  d.stats = reinterpret_cast<float2*>(ws + L.stats);
  for (int k = 0; k < 5; ++k) d.act[k] = reinterpret_cast<uint16_t*>(ws + L.act[k]);
  d.o = reinterpret_cast<float*>(ws + L.o);
  d.g[0] = reinterpret_cast<uint16_t*>(ws + L.g[0]);
  d.g[1] = reinterpret_cast<uint16_t*>(ws + L.g[1]);
  d.part = reinterpret_cast<float*>(ws + L.part);
  d.loss_part = reinterpret_cast<double*>(ws + L.loss_part);
  d.stats_part = reinterpret_cast<double2*>(ws + L.stats_part);
  d.red_part = reinterpret_cast<double*>(ws + L.red_part);
  n->d_loss = reinterpret_cast<double*>(ws + L.loss);
  int rc = ep_tv_net_sync(n);
  if (rc != EP_TV_OK) {
    delete n;
    return rc;
  }
  *out = n;
  return EP_TV_OK;
}

int ep_tv_net_sync(ep_tv_net* n) {
  if (!n) return EP_TV_E_ARG;
  NCHK(n, hipMemsetAsync(n->d.adam_m, 0, kParams * 4, n->stream));
  NCHK(n, hipMemsetAsync(n->d.adam_v, 0, kParams * 4, n->stream));
  n->adam_t = 0;
  n->have_grad = false;
  NCHK(n, pack(n));
  return EP_TV_OK;
}

int ep_tv_net_infer(ep_tv_net* n, const float* d_y, int32_t batch, int32_t h, int32_t w, double noise_var,
                    float* d_mu_hat, float* d_var_hat) {
  if (!n || !d_y || !d_mu_hat || !d_var_hat || !(noise_var > 0.0)) return EP_TV_E_ARG;
  int rc = check_shape(n, batch, h, w);
  if (rc) return rc;
  NCHK(n, forward5(n, d_y, batch, h, w));
  const long long P = (long long)batch * h * w;
  hipLaunchKernelGGL(k_conv6, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, n->stream, n->d.act[4],
                     n->d.w6r, n->master + kOffB6, n->d.stats, batch, h, w, (float)noise_var, 0, d_mu_hat,
                     d_var_hat, (const float*)nullptr, (const float*)nullptr, (float*)nullptr,
                     (double*)nullptr);
  NCHK(n, hipGetLastError());
  return EP_TV_OK;
}

int ep_tv_net_loss_grad(ep_tv_net* n, const float* d_y, const float* d_mu_t, const float* d_var_t,
                        int32_t batch, int32_t h, int32_t w, double noise_var, float* d_grad,
                        double* loss_out) {
  if (!n || !d_y || !d_mu_t || !d_var_t || !(noise_var > 0.0)) return EP_TV_E_ARG;
  int rc = check_shape(n, batch, h, w);
  if (rc) return rc;
  const hipStream_t s = n->stream;
  NCHK(n, forward5(n, d_y, batch, h, w));
  const long long P = (long long)batch * h * w;
  const unsigned nl = (unsigned)((P + 255) / 256);
  hipLaunchKernelGGL(k_conv6, dim3(nl), dim3(256), 0, s, n->d.act[4], n->d.w6r, n->master + kOffB6,
                     n->d.stats, batch, h, w, (float)noise_var, 1, (float*)nullptr, (float*)nullptr, d_mu_t,
                     d_var_t, n->d.o, n->d.loss_part);
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, s, n->d.loss_part, (int)nl, 1.0 / (double)P,
                     n->d_loss);
  const dim3 gt((w + kTile - 1) / kTile, (h + kTile - 1) / kTile, batch);
  const int nblk = (int)(gt.x * gt.y * gt.z);
  const dim3 gc((w + 63) / 64, (h + 4 * kConvSteps - 1) / (4 * kConvSteps), batch);
  // layer 6: weight gradient, input gradient (masked by a5)
  hipLaunchKernelGGL(k_wgrad6, gt, dim3(256), 0, s, n->d.act[4], n->d.o, n->d.part, h, w);
  reduce_grad(n, nblk, kW6 + 2, n->d.grad + kOffW6, s);
  hipLaunchKernelGGL(k_dgrad6, dim3(nl), dim3(256), 0, s, n->d.o, n->d.w6r, n->d.act[4], n->d.g[0], batch, h,
                     w);
  // layers 5..2: weight gradient from (a_{l-1}, g_l), then g_{l-1} = W_l^T g_l masked by a_{l-1}
  int cur = 0;
  for (int l = 3; l >= 0; --l) {           // l = index of the 32 -> 32 layer (layer l + 2)
    const uint16_t* xin = n->d.act[l];
    hipLaunchKernelGGL(k_wgrad32, gt, dim3(256), 0, s, xin, n->d.g[cur], n->d.part, h, w);
    reduce_grad(n, nblk, kStride32, n->d.grad + kOff2 + l * kStride32, s);
    hipLaunchKernelGGL((k_conv32<EPI_MASK>), gc, dim3(256), 0, s, n->d.g[cur], n->d.wd + l * kW32,
                       (const float*)nullptr, xin, n->d.g[cur ^ 1], h, w);
    cur ^= 1;
  }
  // layer 1
  hipLaunchKernelGGL(k_wgrad1, gt, dim3(256), 0, s, d_y, n->d.stats, n->d.g[cur], n->d.part, h, w);
  reduce_grad(n, nblk, kW1 + C, n->d.grad + kOffW1, s);
  NCHK(n, hipGetLastError());
  if (d_grad) NCHK(n, hipMemcpyAsync(d_grad, n->d.grad, kParams * 4, hipMemcpyDeviceToDevice, s));
  n->have_grad = true;
  if (loss_out) {
    NCHK(n, hipMemcpyAsync(loss_out, n->d_loss, 8, hipMemcpyDeviceToHost, s));
    NCHK(n, hipStreamSynchronize(s));
  }
  return EP_TV_OK;
}

int ep_tv_net_adam_step(ep_tv_net* n, float lr) {
  if (!n || !(lr > 0.f)) return EP_TV_E_ARG;
  if (!n->have_grad) return fail(n, EP_TV_E_STATE, "no gradient computed");
  n->adam_t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, n->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, n->adam_t)));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, n->stream, n->master, n->d.adam_m,
                     n->d.adam_v, n->d.grad, kParams, lr, (float)b1, (float)b2, 1e-8f, c1, c2);
  NCHK(n, hipGetLastError());
  NCHK(n, pack(n));
  return EP_TV_OK;
}

int ep_tv_net_train_step(ep_tv_net* n, const float* d_y, const float* d_mu_t, const float* d_var_t,
                         int32_t batch, int32_t h, int32_t w, double noise_var, float lr,
                         double* loss_out) {
  int rc = ep_tv_net_loss_grad(n, d_y, d_mu_t, d_var_t, batch, h, w, noise_var, nullptr, loss_out);
  if (rc) return rc;
  return ep_tv_net_adam_step(n, lr);
}

int ep_tv_net_adam_count(const ep_tv_net* n) { return n ? n->adam_t : -1; }

const char* ep_tv_net_last_error(const ep_tv_net* n) { return n ? n->err.c_str() : "null network"; }

void ep_tv_net_destroy(ep_tv_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  delete n;
}

}  // extern "C"
