// Subsampled Paley-ordered 2-D Walsh-Hadamard operator on the device.
//
// The orthonormal 2-D Walsh transform of an H x W image in natural (Sylvester)
// order is the 1-D Walsh-Hadamard transform of length N = H W of its row-major
// flattening: the Sylvester matrix of order H W is the Kronecker product of
// those of orders H and W, and with W a power of two the row-major index
// r W + c splits into the bits of r above those of c.  The Paley order of the
// observations only relabels coefficients: Paley row k is natural row
// bitreverse(k) along each axis, which the host applies to the mask and the
// observation gather applies to y.
//
// The transform runs over the bits of the flattened index in groups:
//   * the low lb = min(log2 N, 12) bits, a contiguous run of up to 4096
//     elements, in LDS (radix-4 butterflies, one barrier per two bits);
//   * the remaining bits in groups of at most 5, each thread holding the
//     2^g elements of one group in registers; consecutive threads take
//     consecutive low indices, so every load and store is coalesced.
// H^T H = W^T diag(mask) W: a product is pre-op, forward groups, the mask
// multiply and the inverse (the same transform) of the last group fused into
// one pass, the remaining groups again, and the post-op.  Butterflies are
// unnormalised; the 1 / N of the orthonormal pair is folded into the multiply.
#include "wht.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace eptv {

namespace wht {

constexpr int kLowBits = 12;      // elements of the LDS group: 4096 floats
constexpr int kHighBits = 5;      // elements of a register group: at most 32
constexpr int kThreads = 256;

enum { WSRC_DIRECTION = 0, WSRC_REAL, WSRC_OBS, WSRC_WORK };
enum { WMUL_NONE = 0, WMUL_MASK, WMUL_PRECOND, WMUL_SCALE };
enum { WDST_WORK = 0, WDST_Q, WDST_REAL };

struct WhtArgs {
  int logW, logH, logN, lb;
  long long off;             // plane offset of pixel (0, 0)
  int pitch, inst;
  float inv_xi, scale;
  // pitched planes
  const float* z; const float* x; const float* p_in; float* p_out; const float* tauc;
  const float* real_in; float* real_out; const float* pvec;
  const InstState* st;
  int mode0;                 // WSRC_DIRECTION: the vector is x (product for the CG start)
  const float* obs;          // WSRC_OBS: user coefficients, dense H x W, Paley order
  const float* eig;          // mask in natural order (0 or 1), compact N
  float* work;               // compact N
  int src, mul, dst;
  int fwd, inv;              // transform before / after the multiply
  int b;                     // register group: lowest bit
  double* part;              // WDST_Q: one p.q partial per LDS block
};

__device__ __forceinline__ long long plane_index(const WhtArgs& a, int n) {
  const int r = n >> a.logW, c = n & ((1 << a.logW) - 1);
  return a.off + (long long)r * a.pitch + c;
}

__device__ __forceinline__ float mul_factor(const WhtArgs& a, int n, float dbar) {
  if (a.mul == WMUL_MASK) return a.eig[n] * a.scale;
  if (a.mul == WMUL_PRECOND) return a.scale / (a.eig[n] * a.inv_xi + dbar);
  return a.scale;   // WMUL_SCALE
}

__device__ __forceinline__ float load_src(const WhtArgs& a, int n) {
  if (a.src == WSRC_WORK) return a.work[n];
  const long long p = plane_index(a, n);
  if (a.src == WSRC_REAL) return a.real_in[p];
  if (a.src == WSRC_OBS) {
    if (a.eig[n] == 0.f) return 0.f;
    const unsigned r = (unsigned)(n >> a.logW), c = (unsigned)(n & ((1 << a.logW) - 1));
    const unsigned rp = __brev(r) >> (32 - a.logH), cp = __brev(c) >> (32 - a.logW);
    return a.obs[(rp << a.logW) + cp];
  }
  // WSRC_DIRECTION
  if (a.mode0) return a.x[p];
  const InstState& st = a.st[a.inst];
  const float z = a.z[p];
  const float v = st.cg_it == 0 ? z : z + (float)st.cg_beta * a.p_in[p];
  a.p_out[p] = v;
  return v;
}

// Four consecutive elements n .. n + 3 (n a multiple of 4, so they share a row
// and, with 256-byte aligned rows, form one 16-byte word of every plane).
__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

__device__ __forceinline__ float4 load_src4(const WhtArgs& a, int n) {
  if (a.src == WSRC_WORK) return ld4(a.work + n);
  if (a.src == WSRC_OBS)
    return make_float4(load_src(a, n), load_src(a, n + 1), load_src(a, n + 2), load_src(a, n + 3));
  const long long p = plane_index(a, n);
  if (a.src == WSRC_REAL) return ld4(a.real_in + p);
  if (a.mode0) return ld4(a.x + p);
  const InstState& st = a.st[a.inst];
  float4 v = ld4(a.z + p);
  if (st.cg_it != 0) {
    const float beta = (float)st.cg_beta;
    const float4 q = ld4(a.p_in + p);
    v = make_float4(v.x + beta * q.x, v.y + beta * q.y, v.z + beta * q.z, v.w + beta * q.w);
  }
  st4(a.p_out + p, v);
  return v;
}

// In-place unnormalised Walsh-Hadamard transform of X[0, 2^lb) (natural
// order), lb >= 2.
__device__ void lds_wht(float* X, int lb) {
  int s = 0;
  const int nq = 1 << (lb - 2);
  for (; s + 2 <= lb; s += 2) {
    const int S = 1 << s;
    for (int q = threadIdx.x; q < nq; q += kThreads) {
      const int i0 = ((q >> s) << (s + 2)) | (q & (S - 1));
      const float a0 = X[i0], a1 = X[i0 + S], a2 = X[i0 + 2 * S], a3 = X[i0 + 3 * S];
      const float b0 = a0 + a1, b1 = a0 - a1, b2 = a2 + a3, b3 = a2 - a3;
      X[i0] = b0 + b2;
      X[i0 + S] = b1 + b3;
      X[i0 + 2 * S] = b0 - b2;
      X[i0 + 3 * S] = b1 - b3;
    }
    __syncthreads();
  }
  if (s < lb) {   // odd lb: one radix-2 stage
    const int S = 1 << s;
    for (int q = threadIdx.x; q < (1 << (lb - 1)); q += kThreads) {
      const int i0 = ((q >> s) << (s + 1)) | (q & (S - 1));
      const float a0 = X[i0], a1 = X[i0 + S];
      X[i0] = a0 + a1;
      X[i0 + S] = a0 - a1;
    }
    __syncthreads();
  }
}

// One block per run of 2^lb contiguous flattened indices.
__global__ __launch_bounds__(kThreads) void k_wht_low(WhtArgs a) {
  __shared__ __align__(16) float X[1 << kLowBits];
  float4* X4 = reinterpret_cast<float4*>(X);
  const int C = 1 << a.lb, C4 = C >> 2;   // lb >= 4
  const int n0 = blockIdx.x << a.lb;
  for (int i = threadIdx.x; i < C4; i += kThreads) X4[i] = load_src4(a, n0 + 4 * i);
  __syncthreads();
  if (a.fwd) lds_wht(X, a.lb);
  if (a.mul != WMUL_NONE) {
    const float dbar = a.mul == WMUL_PRECOND ? (float)a.st[a.inst].dbar : 0.f;
    for (int i = threadIdx.x; i < C; i += kThreads) X[i] *= mul_factor(a, n0 + i, dbar);
    __syncthreads();
  }
  if (a.inv) lds_wht(X, a.lb);
  if (a.dst == WDST_WORK) {
    for (int i = threadIdx.x; i < C4; i += kThreads) st4(a.work + n0 + 4 * i, X4[i]);
    return;
  }
  if (a.dst == WDST_REAL) {
    for (int i = threadIdx.x; i < C4; i += kThreads) st4(a.real_out + plane_index(a, n0 + 4 * i), X4[i]);
    return;
  }
  // q = A p with this block's p.q partial (dst is uniform over the block)
  double acc = 0.0;
  for (int i = threadIdx.x; i < C4; i += kThreads) {
    const long long p = plane_index(a, n0 + 4 * i);
    const float4 pv = ld4(a.pvec + p), tc = ld4(a.tauc + p), v = X4[i];
    const float4 qv = make_float4(v.x * a.inv_xi + tc.x * pv.x, v.y * a.inv_xi + tc.y * pv.y,
                                  v.z * a.inv_xi + tc.z * pv.z, v.w * a.inv_xi + tc.w * pv.w);
    st4(a.real_out + p, qv);
    acc += ((double)pv.x * (double)qv.x + (double)pv.y * (double)qv.y) +
           ((double)pv.z * (double)qv.z + (double)pv.w * (double)qv.w);
  }
  #pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ double wsum[kThreads / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    a.part[blockIdx.x] = a.st[a.inst].cg_done ? 0.0 : (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

template <int G>
__device__ __forceinline__ void reg_wht(float (&v)[1 << G]) {
  #pragma unroll
  for (int s = 1; s < (1 << G); s <<= 1) {
    #pragma unroll
    for (int i = 0; i < (1 << G); ++i) {
      if (i & s) continue;
      const float x = v[i], y = v[i + s];
      v[i] = x + y;
      v[i + s] = x - y;
    }
  }
}

// Bits [b, b + G) of the flattened index, in place on the work buffer.
// N <= 2^24, so element indices fit 32 bits.
template <int G>
__global__ __launch_bounds__(kThreads) void k_wht_high(WhtArgs a) {
  constexpr int M = 1 << G;
  const int T = 1 << (a.logN - G);
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= T) return;
  const int n0 = (t & ((1 << a.b) - 1)) | ((t >> a.b) << (a.b + G));
  const int S = 1 << a.b;
  float* w = a.work + n0;
  float v[M];
  #pragma unroll
  for (int i = 0; i < M; ++i) v[i] = w[i * S];
  reg_wht<G>(v);
  if (a.mul != WMUL_NONE) {
    const float dbar = a.mul == WMUL_PRECOND ? (float)a.st[a.inst].dbar : 0.f;
    #pragma unroll
    for (int i = 0; i < M; ++i) v[i] *= mul_factor(a, n0 + i * S, dbar);
  }
  if (a.inv) reg_wht<G>(v);
  #pragma unroll
  for (int i = 0; i < M; ++i) w[i * S] = v[i];
}

// All high bits [lb, logN) at once, hb = logN - lb <= kMidBits, in place on
// the work buffer: a block takes kMidCols consecutive low indices and every
// value of the high bits (2^hb x kMidCols elements, 64 KB at hb = 10) into LDS
// as X[h][l], transforms along h, applies the multiply, and (two-sided)
// transforms along h again.  This replaces the register groups' separate
// passes over the high bits (two-sided: four passes become one).  Along h the
// transform runs in register groups of up to 16 elements (radix 16, 16, 4 at
// hb = 10), one LDS round trip and barrier per group.  Row h of X starts at
// kMidCols (h + h / 16): one spare row every 16, so the 16-element groups of
// the first stage (rows 16 apart in a wave) fall on different banks.
constexpr int kMidBits = 10;
constexpr int kMidCols = 16;      // 64-byte runs of each row h
constexpr int kMidThreads = 1024; // one block per CU at hb = 10: every wave it can hold
constexpr int kMidRows = (1 << kMidBits) + (1 << kMidBits) / 16;

__device__ __forceinline__ int mid_off(int h, int l) { return kMidCols * (h + (h >> 4)) + l; }

// One register-group stage along h: bits [s, s + G) of h.
template <int G>
__device__ __forceinline__ void mid_stage(float* X, int R, int s) {
  constexpr int M = 1 << G;
  const int S = 1 << s;
  for (int q = threadIdx.x; q < (R >> G) * kMidCols; q += kMidThreads) {
    const int l = q & (kMidCols - 1), b = q / kMidCols;
    const int h0 = ((b >> s) << (s + G)) | (b & (S - 1));
    float v[M];
#pragma unroll
    for (int i = 0; i < M; ++i) v[i] = X[mid_off(h0 + (i << s), l)];
    reg_wht<G>(v);
#pragma unroll
    for (int i = 0; i < M; ++i) X[mid_off(h0 + (i << s), l)] = v[i];
  }
  __syncthreads();
}

__device__ __forceinline__ void mid_wht(float* X, int hb) {
  const int R = 1 << hb;
  for (int s = 0; s < hb;) {
    const int g = hb - s < 4 ? hb - s : 4;
    if (g == 4) mid_stage<4>(X, R, s);
    else if (g == 3) mid_stage<3>(X, R, s);
    else if (g == 2) mid_stage<2>(X, R, s);
    else mid_stage<1>(X, R, s);
    s += g;
  }
}

__global__ __launch_bounds__(kMidThreads) void k_wht_mid(WhtArgs a) {
  __shared__ __align__(16) float X[kMidCols * kMidRows];
  const int hb = a.logN - a.lb;
  const int R = 1 << hb;                       // rows h
  const int n4 = R * (kMidCols / 4);           // float4 words of the tile
  const int low0 = blockIdx.x * kMidCols;
  // word i: row h = i / 4, columns l = 4 (i % 4) .. + 3 <-> work[(h << lb) + low0 + l]
  auto widx = [&](int i) { return ((i >> 2) << a.lb) + low0 + 4 * (i & 3); };
  auto xw = [&](int i) -> float4& {
    return *reinterpret_cast<float4*>(X + mid_off(i >> 2, 4 * (i & 3)));
  };
  constexpr int kW = (kMidCols << kMidBits) / 4 / kMidThreads;   // words per thread at most
  float4 ev[kW];
  const bool need_eig = a.mul == WMUL_MASK || a.mul == WMUL_PRECOND;
#pragma unroll
  for (int u = 0; u < kW; ++u) {
    const int i = threadIdx.x + u * kMidThreads;
    if (i < n4) {
      xw(i) = ld4(a.work + widx(i));
      if (need_eig) ev[u] = ld4(a.eig + widx(i));
    }
  }
  __syncthreads();
  if (a.fwd) mid_wht(X, hb);
  if (a.mul != WMUL_NONE) {
    const float dbar = a.mul == WMUL_PRECOND ? (float)a.st[a.inst].dbar : 0.f;
#pragma unroll
    for (int u = 0; u < kW; ++u) {
      const int i = threadIdx.x + u * kMidThreads;
      if (i >= n4) continue;
      const float e4[4] = {ev[u].x, ev[u].y, ev[u].z, ev[u].w};
      float m[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        m[k] = a.mul == WMUL_MASK ? e4[k] * a.scale
             : a.mul == WMUL_PRECOND ? a.scale / (e4[k] * a.inv_xi + dbar) : a.scale;
      const float4 v = xw(i);
      xw(i) = make_float4(v.x * m[0], v.y * m[1], v.z * m[2], v.w * m[3]);
    }
    __syncthreads();
  }
  if (a.inv) mid_wht(X, hb);
#pragma unroll
  for (int u = 0; u < kW; ++u) {
    const int i = threadIdx.x + u * kMidThreads;
    if (i < n4) st4(a.work + widx(i), xw(i));
  }
}

// mask in natural order -> spectrum plane (the spectral variance estimator
// reads the eigenvalues of H^T H from it)
__global__ void k_wht_spec(const float* __restrict__ eig, float* __restrict__ spec, long long off,
                           int pitch, int logW, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  spec[off + (long long)(n >> logW) * pitch + (n & ((1 << logW) - 1))] = eig[n];
}

int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

hipError_t launch_high(const WhtArgs& a, int g, hipStream_t s) {
  const int T = 1 << (a.logN - g);
  const dim3 grid((unsigned)((T + kThreads - 1) / kThreads)), blk(kThreads);
  switch (g) {
    case 1: hipLaunchKernelGGL(k_wht_high<1>, grid, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_wht_high<2>, grid, blk, 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_wht_high<3>, grid, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_wht_high<4>, grid, blk, 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_wht_high<5>, grid, blk, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// src -> W -> multiply -> (W again if two_sided) -> dst, over the bit groups.
hipError_t run(const WhtPlan& P, WhtArgs a, bool two_sided, hipStream_t s) {
  a.logW = P.logW; a.logH = P.logH; a.logN = P.logN; a.lb = P.lb;
  a.eig = P.eig; a.work = P.work;
  const unsigned nblk = 1u << (P.logN - P.lb);
  hipError_t e;
  if (P.logN == P.lb) {   // one LDS pass
    a.fwd = 1; a.inv = two_sided ? 1 : 0;
    hipLaunchKernelGGL(k_wht_low, dim3(nblk), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  }
  const int hb = P.logN - P.lb, ng = (hb + kHighBits - 1) / kHighBits;
  if (hb <= kMidBits && P.lb >= 4) {
    // low bits, then every high bit in one LDS pass (multiply and, two-sided,
    // the inverse included), then the low bits again (two-sided) and the post-op
    WhtArgs first = a;
    first.fwd = 1; first.inv = 0; first.mul = WMUL_NONE; first.dst = WDST_WORK;
    hipLaunchKernelGGL(k_wht_low, dim3(nblk), dim3(kThreads), 0, s, first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    WhtArgs m = a;
    m.fwd = 1; m.inv = two_sided ? 1 : 0;
    hipLaunchKernelGGL(k_wht_mid, dim3((1u << P.lb) / kMidCols), dim3(kMidThreads), 0, s, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    WhtArgs last = a;
    last.src = WSRC_WORK; last.fwd = two_sided ? 1 : 0; last.inv = 0; last.mul = WMUL_NONE;
    hipLaunchKernelGGL(k_wht_low, dim3(nblk), dim3(kThreads), 0, s, last);
    return hipGetLastError();
  }
  int gb[4], gg[4];
  for (int k = 0, b = P.lb; k < ng; ++k) {
    gg[k] = hb / ng + (k < hb % ng ? 1 : 0);
    gb[k] = b;
    b += gg[k];
  }
  WhtArgs first = a;
  first.fwd = 1; first.inv = 0; first.mul = WMUL_NONE; first.dst = WDST_WORK;
  hipLaunchKernelGGL(k_wht_low, dim3(nblk), dim3(kThreads), 0, s, first);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k = 0; k < ng; ++k) {
    WhtArgs h = a;
    h.b = gb[k];
    const bool last = k == ng - 1;
    h.mul = last ? a.mul : WMUL_NONE;
    h.inv = (last && two_sided) ? 1 : 0;
    if ((e = launch_high(h, gg[k], s)) != hipSuccess) return e;
  }
  if (two_sided) {
    for (int k = ng - 2; k >= 0; --k) {
      WhtArgs h = a;
      h.b = gb[k]; h.mul = WMUL_NONE; h.inv = 0;
      if ((e = launch_high(h, gg[k], s)) != hipSuccess) return e;
    }
  }
  WhtArgs last = a;
  last.src = WSRC_WORK; last.fwd = two_sided ? 1 : 0; last.inv = 0; last.mul = WMUL_NONE;
  hipLaunchKernelGGL(k_wht_low, dim3(nblk), dim3(kThreads), 0, s, last);
  return hipGetLastError();
}

WhtArgs base(const LikCtx& lc, const LikInst& L) {
  WhtArgs a;
  std::memset(&a, 0, sizeof(a));
  a.off = L.off; a.pitch = L.pitch; a.inst = L.inst; a.inv_xi = L.inv_xi;
  a.st = lc.d_st;
  a.tauc = lc.planes[LP_TAUC];
  return a;
}

}  // namespace wht

using namespace wht;

int wht_partials(int H, int W) {
  const int logN = ilog2i(H) + ilog2i(W);
  return 1 << (logN - (logN < kLowBits ? logN : kLowBits));
}

hipError_t wht_setup(LikCtx& lc, const LikInstInfo* li, int n, size_t wht_bytes, hipStream_t s,
                     std::string& err) {
  (void)n;
  lc.wht.clear();
  char* cur = reinterpret_cast<char*>(lc.whtbuf);
  size_t used = 0;
  std::vector<std::vector<float>> host;   // kept until the copies finish
  for (size_t k = 0; k < lc.hinst.size(); ++k) {
    const LikInst& L = lc.hinst[k];
    if (L.op != OP_HAD) continue;
    const LikInstInfo& I = li[L.inst];
    WhtPlan P;
    P.li = (int)k;
    P.logH = ilog2i(L.H); P.logW = ilog2i(L.W); P.logN = P.logH + P.logW;
    P.lb = P.logN < kLowBits ? P.logN : kLowBits;
    const size_t N = (size_t)L.H * L.W;
    if ((1 << P.logH) != L.H || (1 << P.logW) != L.W || P.logH < 2 || P.logW < 2 ||
        P.logN > 24) {
      err = "Walsh-Hadamard operator needs power-of-two sizes in [4, 4096]";
      return hipErrorInvalidValue;
    }
    const size_t bytes = (N * sizeof(float) + 255) / 256 * 256;
    P.work = reinterpret_cast<float*>(cur + used);
    P.eig = reinterpret_cast<float*>(cur + used + bytes);
    used += 2 * bytes;
    if (used > wht_bytes) {
      err = "Walsh-Hadamard workspace layout mismatch";
      return hipErrorInvalidValue;
    }
    // mask (Paley order, user layout) -> natural order
    host.emplace_back(N);
    std::vector<float>& m = host.back();
    for (int r = 0; r < L.H; ++r)
      for (int c = 0; c < L.W; ++c) {
        int rp = 0, cp = 0;
        for (int b = 0; b < P.logH; ++b) rp |= ((r >> b) & 1) << (P.logH - 1 - b);
        for (int b = 0; b < P.logW; ++b) cp |= ((c >> b) & 1) << (P.logW - 1 - b);
        m[(size_t)r * L.W + c] = I.mask[(size_t)rp * L.W + cp] ? 1.f : 0.f;
      }
    hipError_t e = hipMemcpyAsync(P.eig, m.data(), N * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wht_spec, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, P.eig,
                       lc.planes[LP_SPEC], L.off, L.pitch, P.logW, (int)N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    lc.wht.push_back(P);
  }
  return host.empty() ? hipSuccess : hipStreamSynchronize(s);
}

// H^T v = W^T (mask v) of a Paley-ordered coefficient array v into the pixel
// plane `out`: one transform of the masked, reordered coefficients.
static hipError_t wht_back_project(LikCtx& lc, const WhtPlan& P, const float* v, float* out,
                                   hipStream_t s) {
  const LikInst& L = lc.hinst[P.li];
  WhtArgs a = base(lc, L);
  a.src = WSRC_OBS; a.obs = v;
  a.mul = WMUL_SCALE; a.scale = (float)(1.0 / std::sqrt((double)L.H * L.W));
  a.dst = WDST_REAL; a.real_out = out;
  return run(P, a, false, s);
}

hipError_t wht_back_project_inst(LikCtx& lc, int li, const float* v, float* out, hipStream_t s) {
  for (const WhtPlan& P : lc.wht)
    if (P.li == li) return wht_back_project(lc, P, v, out, s);
  return hipErrorInvalidValue;
}

hipError_t wht_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s) {
  for (const WhtPlan& P : lc.wht) {
    const LikInst& L = lc.hinst[P.li];
    hipError_t e = wht_back_project(lc, P, d_y[L.inst], lc.planes[LP_HTY], s);
    if (e != hipSuccess) return e;
    // the cold start and the observation range use H^T y as the pixel-space observation
    e = hipMemcpy2DAsync(lc.ypix + L.off, sizeof(float) * L.pitch, lc.planes[LP_HTY] + L.off,
                         sizeof(float) * L.pitch, sizeof(float) * L.W, L.H,
                         hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t wht_apply(LikCtx& lc, int mode, hipStream_t s) {
  for (const WhtPlan& P : lc.wht) {
    const LikInst& L = lc.hinst[P.li];
    float* p_in = lc.planes[lc.pcur ? LP_P1 : LP_P0];
    float* p_out = lc.planes[lc.pcur ? LP_P0 : LP_P1];
    WhtArgs a = base(lc, L);
    a.src = WSRC_DIRECTION; a.mode0 = mode == 0;
    a.z = lc.planes[LP_Z]; a.x = lc.planes[LP_X]; a.p_in = p_in; a.p_out = p_out;
    a.mul = WMUL_MASK; a.scale = (float)(1.0 / ((double)L.H * L.W));
    a.dst = WDST_Q; a.real_out = lc.planes[LP_Q];
    a.pvec = mode == 0 ? lc.planes[LP_X] : p_out;
    a.part = lc.part0 + L.tile0;
    hipError_t e = run(P, a, true, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t wht_precondition(LikCtx& lc, hipStream_t s) {
  for (const WhtPlan& P : lc.wht) {
    const LikInst& L = lc.hinst[P.li];
    if (L.precond != PRECOND_CIRCULANT) continue;
    WhtArgs a = base(lc, L);
    a.src = WSRC_REAL; a.real_in = lc.planes[LP_R];
    a.mul = WMUL_PRECOND; a.scale = (float)(1.0 / ((double)L.H * L.W));
    a.dst = WDST_REAL; a.real_out = lc.planes[LP_Z];
    hipError_t e = run(P, a, true, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace eptv
