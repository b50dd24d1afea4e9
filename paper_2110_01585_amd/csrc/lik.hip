// Likelihood-site update q_{x,0} for deconvolution (periodic blur).
//
// Eq. (tilted_P_1): the tilted distribution P_0 has mean
//   E = (H^T H / xi + diag(tau_c))^{-1} (H^T y / xi + eta_c),
// where (tau_c, eta_c) are the natural parameters of the cavity Q^{\0} (the sum
// of the four colour-class sites).  E is found by Jacobi-preconditioned
// conjugate gradients, warm-started from the previous sweep's E (the paper
// notes that only products with the inverse covariance are needed).  The
// diagonal of Cov_{P_0} is estimated spectrally: with the cavity precision
// replaced by its mean d, the covariance is circulant with constant diagonal
// c = mean_w 1 / (|H(w)|^2 / xi + d), giving the site precision
// gamma = 1/c - d for every pixel.  Eq. (update_q0_x) then gives
//   tau_0 = gamma,  eta_0 = (gamma + tau_c) E - eta_c,
// clamped and damped like the colour-class sites.
//
// H^T H x for a periodic convolution is a periodic convolution with the
// autocorrelation of the taps (radius kh-1, kw-1).  It is applied on 64 x 16
// output tiles staged through LDS with the halo: two 1-D passes when the taps
// are separable (rank one, e.g. Gaussian), otherwise H followed by H^T as two
// 2-D passes.  Reductions (dot products, means) are per-tile FP64 partials
// summed in a fixed order by one block per instance.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.h"
#include "fft.h"
#include "lik.h"
#include "wht.h"

namespace eptv {

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

struct LikArgs {
  const LikInst* inst;
  const int4* tiles;         // {lik index, tile x, tile y, 0}
  int ntiles;
  InstState* st;
  double* part0;
  double* part1;
  float* part_mu;
  const float* taps;
  float* hty; float* tauc; float* etac; float* b; float* x; float* r; float* z;
  float* p_in; float* p_out; float* q; float* spec; float* xprev;
  int r_from_apply;          // the separable H^T H kernel writes the CG start r = b - A x itself
  // RBMC: accumulated squared off-diagonal sums, the mean solve's E, and the
  // planes of the current sample (H^T e1, e2, last solution)
  float* acc; float* esave;
  const float* g_s; const float* e2_s; float* xs_s;
  int sample;
  float* var;                // Gaussian CS: the Woodbury variances
};

// The likelihood site is updated in this sweep (every sweep but the first of a
// cold start, on active instances).
__device__ __forceinline__ bool lik_now(const InstState& st) {
  return st.active && (st.sweeps > 0 || st.warm);
}

// Instance L solves for RBMC sample `s` in this sweep.
__device__ __forceinline__ bool rbmc_now(const LikInst& L, const InstState& st, int s) {
  return L.rbmc_ns > s && lik_now(st);
}

// Deterministic block sum of two doubles (256 threads): a butterfly over the
// 64 lanes of each wave (every lane ends with the same bits, since each step
// adds the same two numbers on both lanes), then the four wave totals in a
// fixed order.  One barrier instead of one per tree level.
__device__ __forceinline__ void block_sum2(double a, double b, double* out_a, double* out_b) {
  __shared__ double wa[4], wb[4];
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
  }
  const int w = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) {
    wa[w] = a;
    wb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *out_a = (wa[0] + wa[1]) + (wa[2] + wa[3]);
    *out_b = (wb[0] + wb[1]) + (wb[2] + wb[3]);
  }
}

struct TileXY {
  int r0, c0, r1, c1;
};

__device__ __forceinline__ TileXY lik_tile(const int4 td, const LikInst& L) {
  TileXY t;
  t.c0 = td.y * kLikTW;
  t.r0 = td.z * kLikTH;
  t.c1 = min(t.c0 + kLikTW, L.W);
  t.r1 = min(t.r0 + kLikTH, L.H);
  return t;
}

// Element-wise work on one tile in two phases: load(u, p) for every pixel of
// the tile (u < kTileItems, p its plane index), then op(u, p).  Every load of
// the tile is in flight before the first store, which the compiler would not
// arrange itself: a store through one plane may alias the others as far as it
// knows.  Launched with 256 threads.
constexpr int kTileItems = kLikTH * kLikTW / 256;
// QUAD: a full tile gives each thread four adjacent pixels of one row instead
// (the compiler then merges a kernel's per-pixel loads into 16-byte words; it
// pays where the stores merge too, or where there are none).
template <bool QUAD = false, class Load, class Op>
__device__ __forceinline__ void tile_two_phase(const TileXY& t, const LikInst& L, Load&& load,
                                               Op&& op) {
  const int cols = t.c1 - t.c0;
  const int n = cols * (t.r1 - t.r0);
  static_assert(kTileItems == 4 && kLikTW % 4 == 0, "four adjacent pixels per thread");
  if (QUAD && n == kLikTH * kLikTW) {
    const int r = t.r0 + 4 * (int)threadIdx.x / kLikTW, c = t.c0 + 4 * (int)threadIdx.x % kLikTW;
    const long long p0 = L.off + (long long)r * L.pitch + c;
#pragma unroll
    for (int u = 0; u < 4; ++u) load(u, p0 + u);
#pragma unroll
    for (int u = 0; u < 4; ++u) op(u, p0 + u);
    return;
  }
  long long pp[kTileItems];
#pragma unroll
  for (int u = 0; u < kTileItems; ++u) {
    const int i = threadIdx.x + 256 * u;
    pp[u] = -1;
    if (i < n) {
      const int r = t.r0 + i / cols, c = t.c0 + i % cols;
      pp[u] = L.off + (long long)r * L.pitch + c;
      load(u, pp[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < kTileItems; ++u)
    if (pp[u] >= 0) op(u, pp[u]);
}

// ---------------------------------------------------------------------------
// 1. cavity of site 0, right-hand side, CG starting point (and d_bar, ||b||^2
//    partials).  The start is the mean of the global approximation when no
//    earlier solve exists, the last solve's E after one solve, and the linear
//    extrapolation 2 E_1 - E_2 of the last two solves after that: the sites move
//    smoothly from sweep to sweep (damped updates), so the extrapolated point
//    is closer to the new solution and the CG needs fewer iterations; the
//    solution itself is fixed by the residual tolerance, not by the start.
__global__ __launch_bounds__(256) void k_lik_prep(LikArgs A, const float2* __restrict__ S0,
                                                  const float2* __restrict__ S1,
                                                  const float2* __restrict__ S2,
                                                  const float2* __restrict__ S3,
                                                  const float2* __restrict__ S4) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  double at = 0.0, ab = 0.0;
  if (st.active && (st.sweeps > 0 || st.warm)) {
    const TileXY t = lik_tile(td, L);
    const bool init_x = !st.x_valid;
    const bool extrap = st.x_valid && st.xprev_valid;
    float2 s1[kTileItems], s2[kTileItems], s3[kTileItems], s4[kTileItems], s0[kTileItems];
    float hy[kTileItems], xv[kTileItems], xp[kTileItems];
    tile_two_phase(
        t, L,
        [&](int u, long long p) {
          s1[u] = S1[p]; s2[u] = S2[p]; s3[u] = S3[p]; s4[u] = S4[p];
          hy[u] = A.hty[p];
          if (init_x) s0[u] = S0[p];
          if (!init_x) xv[u] = A.x[p];
          if (extrap) xp[u] = A.xprev[p];
        },
        [&](int u, long long p) {
          const double tc = (double)s1[u].x + (double)s2[u].x + (double)s3[u].x + (double)s4[u].x;
          const double ec = (double)s1[u].y + (double)s2[u].y + (double)s3[u].y + (double)s4[u].y;
          const float bv = (float)((double)hy[u] * (double)L.inv_xi + ec);
          A.tauc[p] = (float)tc;
          A.etac[p] = (float)ec;
          A.b[p] = bv;
          if (init_x) {
            A.x[p] = (float)(((double)s0[u].y + ec) / ((double)s0[u].x + tc));
          } else {
            A.xprev[p] = xv[u];
            if (extrap) A.x[p] = 2.0f * xv[u] - xp[u];
          }
          at += tc;
          ab += (double)bv * (double)bv;
        });
  }
  block_sum2(at, ab, &A.part0[tile], &A.part1[tile]);
}

// ---------------------------------------------------------------------------
// 2. per-instance finalisation of the partial sums (one block per instance)
__global__ __launch_bounds__(256) void k_lik_fin(LikArgs A, int stage) {
  const LikInst L = A.inst[blockIdx.x];
  InstState& st = A.st[L.inst];
  double s0 = 0.0, s1 = 0.0;
  // number of partials this stage sums (one per tile, or one per row block of the
  // real-transform passes), chosen on the host
  const int cnt = A.inst[blockIdx.x].fin_count[stage];
  // 16 partials per thread are requested before the first is added (the sum
  // is still taken in ascending order), so their latencies overlap
  constexpr int kU = 16;
  for (int t0 = threadIdx.x; t0 < cnt; t0 += kU * 256) {
    double v0[kU], v1[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + u * 256;
      v0[u] = t < cnt ? A.part0[L.tile0 + t] : 0.0;
      v1[u] = t < cnt ? A.part1[L.tile0 + t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      s0 += v0[u];
      s1 += v1[u];
    }
  }
  __shared__ double r0, r1;
  block_sum2(s0, s1, &r0, &r1);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double N = (double)L.H * (double)L.W;
  switch (stage) {
    case FIN_PREP:
      if (!st.active || (st.sweeps == 0 && !st.warm)) {
        st.cg_done = 1;          // nothing to do this sweep
        break;
      }
      st.dbar = r0 / N;
      st.cg_bb = r1;
      st.pc_scaled = (L.op == OP_BLUR && st.cg_last > kCgScaleAbove) ? 1 : 0;
      st.cg_it = 0;
      st.cg_done = L.op == OP_GAUSS ? 1 : 0;   // the dense Woodbury path replaces the CG
      st.xprev_valid = st.x_valid;   // prep has just kept the last solve's E
      st.x_valid = 1;
      break;
    case FIN_SPEC:
      if (st.cg_done) break;
      st.gamma = 1.0 / (r0 / N) - st.dbar;
      break;
    case FIN_INIT:
      if (st.cg_done) break;
      st.cg_rz = r0;
      st.cg_rr = r1;
      st.cg_beta = 0.0;
      // stop at the tolerance, or (cg_reduce > 0) once the residual has fallen
      // by cg_reduce from where this solve started, whichever comes first
      st.cg_stop2 = L.cg_tol2;
      if (st.cg_bb > 0.0) st.cg_stop2 = fmax(L.cg_tol2, L.cg_reduce2 * st.cg_rr / st.cg_bb);
      if (!(st.cg_rr > L.cg_tol2 * st.cg_bb)) st.cg_done = 1;
      break;
    case FIN_ALPHA:
      if (st.cg_done) break;
      st.cg_alpha = (r0 != 0.0) ? st.cg_rz / r0 : 0.0;
      break;
    case FIN_SAMPLE:
      // start of the CG solve of RBMC sample A.sample: ||b||^2 of its right-hand side
      if (!rbmc_now(L, st, A.sample)) {
        st.cg_done = 1;
        break;
      }
      st.cg_bb = r1;
      st.cg_it = 0;
      st.cg_done = 0;
      break;
    case FIN_BETA:
      if (st.cg_done) break;
      st.cg_beta = (st.cg_rz != 0.0) ? r0 / st.cg_rz : 0.0;
      st.cg_rz = r0;
      st.cg_rr = r1;
      st.cg_it += 1;
      if (!(st.cg_rr > st.cg_stop2 * st.cg_bb) || st.cg_it >= L.cg_max_iters) st.cg_done = 1;
      break;
  }
}

// ---------------------------------------------------------------------------
// 3. spectral diagonal: partial sums of 1 / (|H(w)|^2 / xi + d_bar)
__global__ __launch_bounds__(256) void k_lik_spec(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  double acc = 0.0;
  if (!st.cg_done) {
    const TileXY t = lik_tile(td, L);
    const double d = st.dbar;
    const double ix = (double)L.inv_xi;
    float sp[kTileItems];
    tile_two_phase<true>(
        t, L, [&](int u, long long p) { sp[u] = A.spec[p]; },
        [&](int u, long long) { acc += 1.0 / ((double)sp[u] * ix + d); });
  }
  block_sum2(acc, 0.0, &A.part0[tile], &A.part1[tile]);
}

// ---------------------------------------------------------------------------
// 4. q = (H^T H / xi + diag(tau_c)) v on a tile, with v either the warm start x
//    (MODE 0) or the new search direction p = z + beta p_old, z = r / diag(A)
//    (MODE 1, p written to p_out).  Partial sums of v . q.
template <int MODE>
__device__ __forceinline__ float direction(const LikArgs& A, const LikInst& L, const InstState& st,
                                           long long p) {
  if (MODE == 0) return A.x[p];
  const float z = A.z[p];
  return st.cg_it == 0 ? z : z + (float)st.cg_beta * A.p_in[p];
}

// General (non-separable) taps: H then H^T with the original taps (kh x kw,
// centred at (kh/2, kw/2)) as two 2-D passes through LDS.
template <int MODE>
__global__ __launch_bounds__(256) void k_apply(LikArgs A) {
  constexpr int EWMAX = kLikTW + 2 * kMaxRadius;
  constexpr int EHMAX = kLikTH + 2 * kMaxRadius;
  __shared__ float P[EHMAX * EWMAX];          // v on the tile plus halo
  __shared__ float T[EHMAX * EWMAX];          // first-pass result
  const int tile = xcd_remap(blockIdx.x, gridDim.x);   // neighbours share an L2
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  if (L.op != OP_BLUR) return;   // masked-DFT tiles: q and partials come from the FFT path
  // a finished solve's partials are not read (every finishing stage skips it)
  if (st.cg_done) return;
  const TileXY t = lik_tile(td, L);
  const int Rr = L.Rr, Rc = L.Rc;
  const int EH = kLikTH + 2 * Rr, EW = kLikTW + 2 * Rc;
  for (int i = threadIdx.x; i < EH * EW; i += blockDim.x) {
    const int er = i / EW, ec = i % EW;
    const int gr = wrapi(t.r0 - Rr + er, L.H), gc = wrapi(t.c0 - Rc + ec, L.W);
    const long long p = L.off + (long long)gr * L.pitch + gc;
    const float v = direction<MODE>(A, L, st, p);
    P[er * EW + ec] = v;
    if (MODE == 1) {
      const int lr = er - Rr, lc = ec - Rc;
      if (lr >= 0 && lr < kLikTH && lc >= 0 && lc < kLikTW && t.r0 + lr < L.H && t.c0 + lc < L.W)
        A.p_out[p] = v;
    }
  }
  __syncthreads();
  const float* k = A.taps + L.k_off;
  const int ch = L.kh / 2, cw = L.kw / 2;
  const int TH = kLikTH + 2 * ch, TW = kLikTW + 2 * cw;
  for (int i = threadIdx.x; i < TH * TW; i += blockDim.x) {
    const int tr = i / TW, tc = i % TW;
    float acc = 0.f;
    for (int a = 0; a < L.kh; ++a)
      for (int b2 = 0; b2 < L.kw; ++b2)
        acc += k[a * L.kw + b2] * P[(tr - a + 2 * ch) * EW + (tc - b2 + 2 * cw)];
    T[tr * TW + tc] = acc;
  }
  __syncthreads();
  double dot = 0.0;
  for (int i = threadIdx.x; i < kLikTH * kLikTW; i += blockDim.x) {
    const int orow = i / kLikTW, oc = i % kLikTW;
    if (t.r0 + orow >= L.H || t.c0 + oc >= L.W) continue;
    float acc = 0.f;
    for (int a = 0; a < L.kh; ++a)
      for (int b2 = 0; b2 < L.kw; ++b2) acc += k[a * L.kw + b2] * T[(orow + a) * TW + (oc + b2)];
    const long long p = L.off + (long long)(t.r0 + orow) * L.pitch + (t.c0 + oc);
    const float v = P[(orow + Rr) * EW + oc + Rc];
    const float qv = acc * L.inv_xi + A.tauc[p] * v;
    A.q[p] = qv;
    dot += (double)v * (double)qv;
  }
  block_sum2(dot, 0.0, &A.part0[tile], &A.part1[tile]);
}

// Separable taps (rank one, e.g. Gaussian): H^T H is the separable periodic
// convolution with the autocorrelations g_r (rows) and g_c (columns) of the two
// factors, radius RI <= RT each.  RT is a compile-time bound (taps beyond an
// instance's own radius are zero), so the tile geometry and index arithmetic are
// constants: the 64 x 16 output tile plus an RT halo is staged in LDS (periodic
// wrap only on border tiles), filtered along rows into a second LDS array, then
// along columns.
template <int RT, int MODE>
__global__ __launch_bounds__(256) void k_hth_sep(LikArgs A) {
  constexpr int EW = kLikTW + 2 * RT, EH = kLikTH + 2 * RT, NT = 2 * RT + 1;
  __shared__ __align__(16) float P[EH * EW];
  __shared__ __align__(16) float T[EH * kLikTW];
  __shared__ float gr[NT], gc[NT];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);   // neighbours share an L2
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  if (L.op != OP_BLUR) return;   // masked-DFT tiles: the FFT path writes q and partials
  // a finished solve's partials are not read (every finishing stage skips it)
  if (st.cg_done) return;
  if (threadIdx.x < NT) {
    const int d = (int)threadIdx.x - RT;       // offset -RT..RT
    gr[threadIdx.x] = (d >= -L.Rr && d <= L.Rr) ? A.taps[L.gr_off + d + L.Rr] : 0.f;
    gc[threadIdx.x] = (d >= -L.Rc && d <= L.Rc) ? A.taps[L.gc_off + d + L.Rc] : 0.f;
  }
  const TileXY t = lik_tile(td, L);
  const bool inner = t.r0 >= RT && t.c0 >= RT && t.r0 + kLikTH + RT <= L.H && t.c0 + kLikTW + RT <= L.W;
  const bool first = st.cg_it == 0;
  const float beta = (float)st.cg_beta;
  // Every global load of the tile is issued before the first store (a store to
  // p_out or q may alias the loaded planes as far as the compiler knows, so
  // interleaving them would serialise the loads on memory latency).
  constexpr int NL = (EH * EW + 255) / 256;          // halo elements per thread
  constexpr int NQ = kLikTH * kLikTW / 4 / 256;      // output quads (4 columns) per thread
  auto halo_index = [&](int i) {
    const int er = i / EW, ec = i - (i / EW) * EW;
    int gy = t.r0 - RT + er, gx = t.c0 - RT + ec;
    if (!inner) {   // periodic wrap; images smaller than the halo wrap more than once
      gy = wrapi(gy, L.H);
      gx = wrapi(gx, L.W);
    }
    return L.off + (long long)gy * L.pitch + gx;
  };
  // output quad u of this thread: row qrow(u), columns qcol(u) .. qcol(u) + 3
  auto qrow = [&](int u) { return (int)(threadIdx.x + 256 * u) / (kLikTW / 4); };
  auto qcol = [&](int u) { return 4 * ((int)(threadIdx.x + 256 * u) % (kLikTW / 4)); };
  auto qfull = [&](int u) { return t.r0 + qrow(u) < L.H && t.c0 + qcol(u) + 3 < L.W; };
  // Tiles whose halo lies inside the image (no wrap) load it as 16-byte words:
  // the halo starts RT columns left of a 64-column tile boundary, and planes
  // and their row pitch are 64-float aligned, so every word is aligned.
  static_assert(RT % 4 == 0 && EW % 4 == 0 && kLikTW % 4 == 0, "16-byte halo words");
  constexpr int EW4 = EW / 4;
  constexpr int NL4 = (EH * EW4 + 255) / 256;        // halo words per thread
  float4 zv4[NL4], pv4[NL4];
  float zv[NL], pv[NL];
  float4 tc[NQ], bq[NQ];
  if (inner) {
#pragma unroll
    for (int u = 0; u < NL4; ++u) {
      const int i = threadIdx.x + 256 * u;
      zv4[u] = pv4[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i < EH * EW4) {
        const int er = i / EW4, ec = 4 * (i - (i / EW4) * EW4);
        const long long p = L.off + (long long)(t.r0 - RT + er) * L.pitch + (t.c0 - RT + ec);
        if (MODE == 0) {
          zv4[u] = *reinterpret_cast<const float4*>(A.x + p);
        } else {
          zv4[u] = *reinterpret_cast<const float4*>(A.z + p);
          if (!first) pv4[u] = *reinterpret_cast<const float4*>(A.p_in + p);
        }
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int i = threadIdx.x + 256 * u;
      zv[u] = 0.f;
      pv[u] = 0.f;
      if (i < EH * EW) {
        const long long p = halo_index(i);
        if (MODE == 0) {
          zv[u] = A.x[p];
        } else {
          zv[u] = A.z[p];
          if (!first) pv[u] = A.p_in[p];
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const long long p = L.off + (long long)(t.r0 + qrow(u)) * L.pitch + (t.c0 + qcol(u));
    float e[4] = {0.f, 0.f, 0.f, 0.f}, f[4] = {0.f, 0.f, 0.f, 0.f};
    if (qfull(u)) {
      tc[u] = *reinterpret_cast<const float4*>(A.tauc + p);
      if (MODE == 0 && A.r_from_apply) bq[u] = *reinterpret_cast<const float4*>(A.b + p);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (t.r0 + qrow(u) < L.H && t.c0 + qcol(u) + k < L.W) {
          e[k] = A.tauc[p + k];
          if (MODE == 0 && A.r_from_apply) f[k] = A.b[p + k];
        }
      tc[u] = make_float4(e[0], e[1], e[2], e[3]);
      if (MODE == 0 && A.r_from_apply) bq[u] = make_float4(f[0], f[1], f[2], f[3]);
    }
  }
  if (inner) {
#pragma unroll
    for (int u = 0; u < NL4; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (i >= EH * EW4) continue;
      float4 v = zv4[u];
      const int er = i / EW4, ec = 4 * (i - (i / EW4) * EW4);
      if (MODE == 1) {
        if (!first) {
          v.x = zv4[u].x + beta * pv4[u].x;
          v.y = zv4[u].y + beta * pv4[u].y;
          v.z = zv4[u].z + beta * pv4[u].z;
          v.w = zv4[u].w + beta * pv4[u].w;
        }
        const int lr = er - RT, lc = ec - RT;   // a word is all inside or all outside the tile
        if (lr >= 0 && lr < kLikTH && lc >= 0 && lc < kLikTW) {
          const long long p = L.off + (long long)(t.r0 + lr) * L.pitch + (t.c0 + lc);
          *reinterpret_cast<float4*>(A.p_out + p) = v;
        }
      }
      *reinterpret_cast<float4*>(P + er * EW + ec) = v;
    }
  } else {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (i >= EH * EW) continue;
      float v = zv[u];
      if (MODE == 1) {
        v = first ? zv[u] : zv[u] + beta * pv[u];
        const int er = i / EW, ec = i - (i / EW) * EW;
        const int lr = er - RT, lc = ec - RT;
        if (lr >= 0 && lr < kLikTH && lc >= 0 && lc < kLikTW && t.r0 + lr < L.H && t.c0 + lc < L.W)
          A.p_out[halo_index(i)] = v;
      }
      P[i] = v;
    }
  }
  __syncthreads();
  // row pass, four adjacent outputs per work item from 128-bit LDS reads
  constexpr int NW = (NT + 3 + 3) / 4;               // float4 words of the input window
  for (int w = threadIdx.x; w < EH * kLikTW / 4; w += 256) {
    const int er = w / (kLikTW / 4), oc = 4 * (w % (kLikTW / 4));
    float win[4 * NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const float4 x = *reinterpret_cast<const float4*>(P + er * EW + oc + 4 * q);
      win[4 * q] = x.x; win[4 * q + 1] = x.y; win[4 * q + 2] = x.z; win[4 * q + 3] = x.w;
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < NT; ++d) {
      const float g = gc[d];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += g * win[k + d];
    }
    *reinterpret_cast<float4*>(T + er * kLikTW + oc) = make_float4(acc[0], acc[1], acc[2], acc[3]);
  }
  __syncthreads();
  // column pass and q = H^T H p / xi + tau_c p, four adjacent columns per item
  double dot = 0.0;
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int orow = qrow(u), oc = qcol(u);
    if (t.r0 + orow >= L.H || t.c0 + oc >= L.W) continue;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < NT; ++d) {
      const float g = gr[d];
      const float4 x = *reinterpret_cast<const float4*>(T + (orow + d) * kLikTW + oc);
      acc[0] += g * x.x; acc[1] += g * x.y; acc[2] += g * x.z; acc[3] += g * x.w;
    }
    const float4 v4 = *reinterpret_cast<const float4*>(P + (orow + RT) * EW + oc + RT);
    const float v[4] = {v4.x, v4.y, v4.z, v4.w};
    const float tq[4] = {tc[u].x, tc[u].y, tc[u].z, tc[u].w};
    float qv[4], ov[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qv[k] = acc[k] * L.inv_xi + tq[k] * v[k];
    // MODE 0 with r_from_apply: the CG start r = b - A x goes out instead of A x
    const bool wr = MODE == 0 && A.r_from_apply;
    const float bb[4] = {bq[u].x, bq[u].y, bq[u].z, bq[u].w};
#pragma unroll
    for (int k = 0; k < 4; ++k) ov[k] = wr ? bb[k] - qv[k] : qv[k];
    float* out = wr ? A.r : A.q;
    const long long p = L.off + (long long)(t.r0 + orow) * L.pitch + (t.c0 + oc);
    if (qfull(u)) {
      *reinterpret_cast<float4*>(out + p) = make_float4(ov[0], ov[1], ov[2], ov[3]);
#pragma unroll
      for (int k = 0; k < 4; ++k) dot += (double)v[k] * (double)qv[k];
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (t.c0 + oc + k >= L.W) continue;
        out[p + k] = ov[k];
        dot += (double)v[k] * (double)qv[k];
      }
    }
  }
  block_sum2(dot, 0.0, &A.part0[tile], &A.part1[tile]);
}

// ---------------------------------------------------------------------------
// 5. CG start: r = b - A x (q holds A x); blur tiles whose product kernel
//    wrote r itself are skipped
__global__ __launch_bounds__(256) void k_cg_init(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  if (st.cg_done || (A.r_from_apply && L.op == OP_BLUR)) return;
  const TileXY t = lik_tile(td, L);
  float bv[kTileItems], qv[kTileItems];
  tile_two_phase(
      t, L, [&](int u, long long p) { bv[u] = A.b[p]; qv[u] = A.q[p]; },
      [&](int u, long long p) { A.r[p] = bv[u] - qv[u]; });
}

// 5b. z = M^{-1} r (Jacobi instances: here; circulant instances: z was written
//     by the FFT pipeline) and partial sums of r.z and r.r
__global__ __launch_bounds__(256) void k_precond_dot(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  if (st.cg_done) return;   // its partials are not read (every finishing stage skips it)
  double rz = 0.0, rr = 0.0;
  {
    const TileXY t = lik_tile(td, L);
    const bool jac = L.precond == PRECOND_JACOBI;
    float rv[kTileItems], wv[kTileItems];   // r, and tau_c (Jacobi) or z
    tile_two_phase(
        t, L,
        [&](int u, long long p) {
          rv[u] = A.r[p];
          wv[u] = jac ? A.tauc[p] : A.z[p];
        },
        [&](int u, long long p) {
          float zv;
          if (jac) {
            zv = rv[u] / (L.diagA + wv[u]);
            A.z[p] = zv;
          } else {
            zv = wv[u];
          }
          rz += (double)rv[u] * (double)zv;
          rr += (double)rv[u] * (double)rv[u];
        });
  }
  block_sum2(rz, rr, &A.part0[tile], &A.part1[tile]);
}

// 6. CG step: x += alpha p, r -= alpha q
__global__ __launch_bounds__(256) void k_cg_update(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  if (st.cg_done) return;
  const float alpha = (float)st.cg_alpha;
  const TileXY t = lik_tile(td, L);
  float xv[kTileItems], pv[kTileItems], rv[kTileItems], qv[kTileItems];
  tile_two_phase(
      t, L,
      [&](int u, long long p) { xv[u] = A.x[p]; pv[u] = A.p_out[p]; rv[u] = A.r[p]; qv[u] = A.q[p]; },
      [&](int u, long long p) {
        A.x[p] = xv[u] + alpha * pv[u];
        A.r[p] = rv[u] - alpha * qv[u];
      });
}

// 6b. The CG step and the Jacobi preconditioner in one pass, for contexts whose
//     every instance is Jacobi-preconditioned: x += alpha p, r -= alpha q,
//     z = r / diag(A), and partial sums of r.z and r.r (what k_cg_update and
//     k_precond_dot do, without writing r and reading it back).
__global__ __launch_bounds__(256) void k_cg_update_jacobi(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  if (st.cg_done) return;   // its partials are not read (every finishing stage skips it)
  double rz = 0.0, rr = 0.0;
  {
    const float alpha = (float)st.cg_alpha;
    const TileXY t = lik_tile(td, L);
    float xv[kTileItems], pv[kTileItems], rv[kTileItems], qv[kTileItems], tv[kTileItems];
    tile_two_phase<true>(
        t, L,
        [&](int u, long long p) {
          xv[u] = A.x[p]; pv[u] = A.p_out[p]; rv[u] = A.r[p]; qv[u] = A.q[p]; tv[u] = A.tauc[p];
        },
        [&](int u, long long p) {
          const float rn = rv[u] - alpha * qv[u];
          const float zv = rn / (L.diagA + tv[u]);
          A.x[p] = xv[u] + alpha * pv[u];
          A.r[p] = rn;
          A.z[p] = zv;
          rz += (double)rn * (double)zv;
          rr += (double)rn * (double)rn;
        });
  }
  block_sum2(rz, rr, &A.part0[tile], &A.part1[tile]);
}

// Deterministic block maximum (256 threads), written by thread 0.
__device__ __forceinline__ void block_max(float v, float* out) {
  __shared__ float wm[4];
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  if (threadIdx.x % kWave == 0) wm[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

// 7. site update q_{x,0} from E = x (Eq. (update_q0_x)), clamp, damping; the
//    tile's largest |mean| of the global approximation after the update feeds
//    the divergence rule
__global__ __launch_bounds__(256) void k_lik_site(LikArgs A, float2* __restrict__ S0) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  InstState& st = A.st[L.inst];
  if (!st.active || (st.sweeps == 0 && !st.warm)) {
    if (threadIdx.x == 0) A.part_mu[tile] = 0.f;
    return;
  }
  const TileXY t = lik_tile(td, L);
  const float a = L.alpha;
  if (L.op == OP_GAUSS) {
    // Woodbury variances and mean from the dense path
    float tcv[kTileItems], ev[kTileItems], ecv[kTileItems], vv[kTileItems];
    float2 ov[kTileItems];
    float mx = 0.f;
    tile_two_phase<true>(
        t, L,
        [&](int u, long long p) {
          tcv[u] = A.tauc[p]; ev[u] = A.x[p]; ecv[u] = A.etac[p]; vv[u] = A.var[p]; ov[u] = S0[p];
        },
        [&](int u, long long p) {
          double tn = 1.0 / (double)vv[u] - (double)tcv[u];
          if (!(tn >= (double)kPrecFloor)) tn = (double)kPrecFloor;
          const float tau_new = (float)tn;
          const float eta_new = (float)((tn + (double)tcv[u]) * (double)ev[u] - (double)ecv[u]);
          const float2 s0 = make_float2(a * tau_new + (1.f - a) * ov[u].x, a * eta_new + (1.f - a) * ov[u].y);
          S0[p] = s0;
          mx = fmaxf(mx, fabsf((s0.y + ecv[u]) / (s0.x + tcv[u])));
        });
    block_max(mx, &A.part_mu[tile]);
    return;
  }
  if (L.rbmc_ns) {
    // RBMC: per-pixel tilted variance V = 1/Q_ii + acc / (Ns Q_ii^2), Q_ii = diag
    // (H^T H)/xi + tau_c; E is the mean solve's, restored into x for the next
    // sweep's CG start
    if (tile == L.tile0 && threadIdx.x == 0) st.xs_valid = 1;
    const double inv_ns = 1.0 / (double)L.rbmc_ns;
    float tcv[kTileItems], ev[kTileItems], ecv[kTileItems], acv[kTileItems];
    float2 ov[kTileItems];
    float mx = 0.f;
    tile_two_phase<true>(
        t, L,
        [&](int u, long long p) {
          tcv[u] = A.tauc[p]; ev[u] = A.esave[p]; ecv[u] = A.etac[p]; acv[u] = A.acc[p]; ov[u] = S0[p];
        },
        [&](int u, long long p) {
          const double q = (double)L.diagA + (double)tcv[u];
          const double v = 1.0 / q + (double)acv[u] * inv_ns / (q * q);
          double tn = 1.0 / v - (double)tcv[u];
          if (!(tn >= (double)kPrecFloor)) tn = (double)kPrecFloor;
          const float tau_new = (float)tn;
          const float eta_new = (float)((tn + (double)tcv[u]) * (double)ev[u] - (double)ecv[u]);
          const float2 s0 = make_float2(a * tau_new + (1.f - a) * ov[u].x, a * eta_new + (1.f - a) * ov[u].y);
          S0[p] = s0;
          A.x[p] = ev[u];
          mx = fmaxf(mx, fabsf((s0.y + ecv[u]) / (s0.x + tcv[u])));
        });
    block_max(mx, &A.part_mu[tile]);
    return;
  }
  if (tile == L.tile0 && threadIdx.x == 0) {
    st.cg_last = st.cg_it;
    st.cg_total += st.cg_it;
  }
  float tau_new = (float)st.gamma;
  if (!(tau_new >= kPrecFloor)) tau_new = kPrecFloor;
  float tcv[kTileItems], xv[kTileItems], ecv[kTileItems];
  float2 ov[kTileItems];
  float mx = 0.f;
  tile_two_phase<true>(
      t, L,
      [&](int u, long long p) { tcv[u] = A.tauc[p]; xv[u] = A.x[p]; ecv[u] = A.etac[p]; ov[u] = S0[p]; },
      [&](int u, long long p) {
        const float eta_new = (float)(((double)tau_new + (double)tcv[u]) * (double)xv[u] - (double)ecv[u]);
        const float2 s0 = make_float2(a * tau_new + (1.f - a) * ov[u].x, a * eta_new + (1.f - a) * ov[u].y);
        S0[p] = s0;
        mx = fmaxf(mx, fabsf((s0.y + ecv[u]) / (s0.x + tcv[u])));
      });
  block_max(mx, &A.part_mu[tile]);
}

// ---------------------------------------------------------------------------
// RBMC variance estimator (Siden et al. 2018, named for general H in Sec.
// III-C): after the mean solve, each sample s solves Q x = z with
// z = H^T e1 / sqrt(xi) + sqrt(tau_c) e2 ~ N(0, Q) (perturbation-optimisation),
// then sum_{j != i} Q_ij x_j = (Q x)_i - Q_ii x_i = b_i - r_i - Q_ii x_i is
// squared into acc.  The mean solve's E is kept aside meanwhile.

// 8a. keep E, clear the accumulator
__global__ __launch_bounds__(256) void k_rbmc_begin(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  InstState& st = A.st[L.inst];
  if (!rbmc_now(L, st, 0)) return;
  if (tile == L.tile0 && threadIdx.x == 0) {   // the mean solve's iterations
    st.cg_last = st.cg_it;
    st.cg_total += st.cg_it;
  }
  const TileXY t = lik_tile(td, L);
  float xv[kTileItems];
  tile_two_phase<true>(
      t, L, [&](int u, long long p) { xv[u] = A.x[p]; },
      [&](int u, long long p) {
        A.esave[p] = xv[u];
        A.acc[p] = 0.f;
      });
}

// 8b. right-hand side of sample A.sample and its CG start (the sample's last
//     solution, or 0), with the ||b||^2 partials
__global__ __launch_bounds__(256) void k_rbmc_rhs(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  const InstState& st = A.st[L.inst];
  double bb = 0.0;
  if (rbmc_now(L, st, A.sample)) {
    const TileXY t = lik_tile(td, L);
    const bool start = st.xs_valid;
    const float isx = L.inv_sqrt_xi;
    float gv[kTileItems], ev[kTileItems], tv[kTileItems], xv[kTileItems];
    tile_two_phase<true>(
        t, L,
        [&](int u, long long p) {
          gv[u] = A.g_s[p]; ev[u] = A.e2_s[p]; tv[u] = A.tauc[p];
          if (start) xv[u] = A.xs_s[p];
        },
        [&](int u, long long p) {
          const float bv = (float)((double)gv[u] * (double)isx + sqrt((double)tv[u]) * (double)ev[u]);
          A.b[p] = bv;
          A.x[p] = start ? xv[u] : 0.f;
          bb += (double)bv * (double)bv;
        });
  }
  block_sum2(0.0, bb, &A.part0[tile], &A.part1[tile]);
}

// 8c. after the sample's solve: keep its solution, accumulate the squared
//     off-diagonal sum
__global__ __launch_bounds__(256) void k_rbmc_acc(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  InstState& st = A.st[L.inst];
  if (!rbmc_now(L, st, A.sample)) return;
  if (tile == L.tile0 && threadIdx.x == 0) st.cg_total += st.cg_it;
  const TileXY t = lik_tile(td, L);
  float xv[kTileItems], bv[kTileItems], rv[kTileItems], tv[kTileItems], av[kTileItems];
  tile_two_phase<true>(
      t, L,
      [&](int u, long long p) {
        xv[u] = A.x[p]; bv[u] = A.b[p]; rv[u] = A.r[p]; tv[u] = A.tauc[p]; av[u] = A.acc[p];
      },
      [&](int u, long long p) {
        const double q = (double)L.diagA + (double)tv[u];
        const double off = (double)bv[u] - (double)rv[u] - q * (double)xv[u];
        A.xs_s[p] = xv[u];
        A.acc[p] = (float)((double)av[u] + off * off);
      });
}

// ---------------------------------------------------------------------------
// one-time kernels: H^T y (correlation with the taps) and |H(w)|^2
__global__ __launch_bounds__(256) void k_hty_blur(LikArgs A, const float* __restrict__ ypix) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  if (L.op != OP_BLUR) return;
  const TileXY t = lik_tile(td, L);
  const int cols = t.c1 - t.c0;
  const int n = cols * (t.r1 - t.r0);
  const float* k = A.taps + L.k_off;
  const int ch = L.kh / 2, cw = L.kw / 2;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = t.r0 + i / cols, c = t.c0 + i % cols;
    double acc = 0.0;
    for (int a = 0; a < L.kh; ++a)
      for (int b2 = 0; b2 < L.kw; ++b2) {
        const int gr = wrapi(r + a - ch, L.H), gc = wrapi(c + b2 - cw, L.W);
        acc += (double)k[a * L.kw + b2] * (double)ypix[L.off + (long long)gr * L.pitch + gc];
      }
    A.hty[L.off + (long long)r * L.pitch + c] = (float)acc;
  }
}

// |K(w)|^2 of a separable kernel u v^T is |U(r)|^2 |V(c)|^2, and each factor
// is the real transform of the factor's autocorrelation g (symmetric):
// g(0) + 2 sum_{d>0} g(d) cos(2 pi w d / n), the phase reduced exactly; a
// power spectrum, so a value rounding has pushed below zero is taken as zero.
__device__ double autocorr_spectrum(const float* g, int k, int w, int n) {
  const double two_pi = 6.283185307179586476925;
  double acc = (double)g[k - 1];
  for (int d = 1; d < k; ++d)
    acc += 2.0 * (double)g[k - 1 + d] * cos(two_pi * (double)(((long long)w * d) % n) / n);
  return fmax(acc, 0.0);
}

__global__ __launch_bounds__(256) void k_spectrum_blur(LikArgs A) {
  const int tile = blockIdx.x;
  const int4 td = A.tiles[tile];
  const LikInst L = A.inst[td.x];
  if (L.op != OP_BLUR) return;
  const TileXY t = lik_tile(td, L);
  const int cols = t.c1 - t.c0;
  const int n = cols * (t.r1 - t.r0);
  if (L.sep) {
    // separable taps: one 1-D spectrum value per tile row and per tile column
    __shared__ double gr[kLikTH], gc[kLikTW];
    const int tid = threadIdx.x;
    if (tid < t.r1 - t.r0) gr[tid] = autocorr_spectrum(A.taps + L.gr_off, L.kh, t.r0 + tid, L.H);
    else if (tid >= kLikTH && tid - kLikTH < cols)
      gc[tid - kLikTH] = autocorr_spectrum(A.taps + L.gc_off, L.kw, t.c0 + tid - kLikTH, L.W);
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      const int r = i / cols, c = i % cols;
      A.spec[L.off + (long long)(t.r0 + r) * L.pitch + t.c0 + c] = (float)(gr[r] * gc[c]);
    }
    return;
  }
  const float* k = A.taps + L.k_off;
  const double two_pi = 6.283185307179586476925;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = t.r0 + i / cols, c = t.c0 + i % cols;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < L.kh; ++a)
      for (int b2 = 0; b2 < L.kw; ++b2) {
        // phase of tap offset (a - kh/2, b - kw/2) at frequency (r, c), reduced exactly
        const long long ph_r = ((long long)(a - L.kh / 2) * r) % L.H;
        const long long ph_c = ((long long)(b2 - L.kw / 2) * c) % L.W;
        const double ang = two_pi * ((double)ph_r / L.H + (double)ph_c / L.W);
        double sn, cs;
        sincos(ang, &sn, &cs);
        re += (double)k[a * L.kw + b2] * cs;
        im -= (double)k[a * L.kw + b2] * sn;
      }
    A.spec[L.off + (long long)r * L.pitch + c] = (float)(re * re + im * im);
  }
}

// ---------------------------------------------------------------------------
// host side

// Blur instances go to the separable H^T H kernel when all of them have
// separable taps (one kernel per launch), else to the general one.
static bool blur_all_sep(const LikCtx& lc) {
  for (const LikInst& d : lc.hinst)
    if (d.op == OP_BLUR && !d.sep) return false;
  return true;
}

static LikArgs make_args(LikCtx& lc) {
  LikArgs A;
  A.r_from_apply = blur_all_sep(lc) ? 1 : 0;
  A.inst = lc.d_inst;
  A.tiles = lc.d_tiles;
  A.ntiles = lc.ntiles;
  A.st = lc.d_st;
  A.part0 = lc.part0;
  A.part1 = lc.part1;
  A.part_mu = lc.part_mu;
  A.taps = lc.taps;
  A.hty = lc.planes[LP_HTY];
  A.tauc = lc.planes[LP_TAUC];
  A.etac = lc.planes[LP_ETAC];
  A.b = lc.planes[LP_B];
  A.x = lc.planes[LP_X];
  A.r = lc.planes[LP_R];
  A.z = lc.planes[LP_Z];
  A.p_in = lc.planes[lc.pcur ? LP_P1 : LP_P0];
  A.p_out = lc.planes[lc.pcur ? LP_P0 : LP_P1];
  A.q = lc.planes[LP_Q];
  A.spec = lc.planes[LP_SPEC];
  A.xprev = lc.planes[LP_XPREV];
  A.acc = lc.planes[LP_ACC];
  A.esave = lc.planes[LP_ESAVE];
  A.var = lc.planes[LP_VAR];
  A.sample = lc.sample;
  const size_t off = (size_t)lc.plane * (size_t)lc.sample;
  A.g_s = lc.rbmc_g ? lc.rbmc_g + off : nullptr;
  A.e2_s = lc.rbmc_e2 ? lc.rbmc_e2 + off : nullptr;
  A.xs_s = lc.rbmc_x ? lc.rbmc_x + off : nullptr;
  return A;
}

hipError_t lik_create(LikCtx& lc, const LikInstInfo* li, int n, char* ws, const LikLayout& L,
                      long long plane, InstDev* d_inst, InstState* d_st, int4* d_tiles, int ntiles,
                      float* ypix, hipStream_t s, std::string& err) {
  (void)d_tiles; (void)ntiles;
  lc = LikCtx();
  lc.n_all = n;
  lc.nlik = L.nlik;
  lc.ntiles = L.ntiles;
  lc.d_st = d_st;
  lc.d_idev = d_inst;
  lc.ypix = ypix;
  if (lc.nlik == 0) return hipSuccess;
  for (int k = 0; k < LP_COUNT; ++k)
    lc.planes[k] = k < L.nplanes ? reinterpret_cast<float*>(ws + L.planes[k]) : nullptr;
  lc.plane = plane;
  lc.rbmc_ns_max = L.rbmc_ns_max;
  if (L.rbmc_ns_max) {
    lc.rbmc_g = reinterpret_cast<float*>(ws + L.rbmc_g);
    lc.rbmc_e2 = reinterpret_cast<float*>(ws + L.rbmc_e2);
    lc.rbmc_x = reinterpret_cast<float*>(ws + L.rbmc_x);
  }
  lc.d_inst = reinterpret_cast<LikInst*>(ws + L.inst);
  lc.d_tiles = reinterpret_cast<int4*>(ws + L.tiles);
  lc.part0 = reinterpret_cast<double*>(ws + L.part0);
  lc.part1 = reinterpret_cast<double*>(ws + L.part1);
  lc.part_mu = reinterpret_cast<float*>(ws + L.part_mu);
  lc.taps = reinterpret_cast<float*>(ws + L.taps);
  lc.fft = reinterpret_cast<float2*>(ws + L.fft);
  lc.whtbuf = reinterpret_cast<float*>(ws + L.wht);
  std::vector<float> taps;
  std::vector<int4> tiles;
  for (int i = 0; i < n; ++i) {
    const LikInstInfo& I = li[i];
    if (I.op == OP_IDENTITY) continue;
    LikInst d;
    std::memset(&d, 0, sizeof(d));
    d.H = I.H; d.W = I.W; d.pitch = I.pitch; d.op = I.op; d.off = I.off; d.inst = i;
    d.tile0 = (int)tiles.size();
    d.tiles_x = (I.W + kLikTW - 1) / kLikTW;
    const int ty = (I.H + kLikTH - 1) / kLikTH;
    d.ntiles = d.tiles_x * ty;
    d.inv_xi = (float)(1.0 / I.xi);
    d.inv_sqrt_xi = (float)(1.0 / std::sqrt(I.xi));
    d.rbmc_ns = I.rbmc_ns;
    d.alpha = (float)I.damping;
    d.cg_tol2 = I.cg_tol * I.cg_tol;
    d.cg_reduce2 = I.cg_reduce * I.cg_reduce;
    d.cg_max_iters = I.cg_max_iters;
    d.precond = I.op == OP_GAUSS ? PRECOND_JACOBI : lik_precond(I.op, I.H, I.W, I.precond_req);
    d.npart = (d.precond == PRECOND_CIRCULANT && I.op != OP_HAD) ? rfft_partials(I.H, I.W) : d.ntiles;
    if (d.npart > d.ntiles) return hipErrorInvalidValue;   // partial slots are per tile
    lc.max_iters = std::max(lc.max_iters, I.cg_max_iters);
    const int li_idx = (int)lc.hinst.size();
    for (int yy = 0; yy < ty; ++yy)
      for (int xx = 0; xx < d.tiles_x; ++xx) tiles.push_back(make_int4(li_idx, xx, yy, 0));
    if (I.op == OP_BLUR) {
      const int kh = I.th, kw = I.tw;
      d.kh = kh; d.kw = kw;
      d.Rr = kh - 1; d.Rc = kw - 1;
      d.k_off = (int)taps.size();
      double ksq = 0.0, kmax = 0.0;
      int a0 = 0, b0 = 0;
      for (int a = 0; a < kh; ++a)
        for (int b2 = 0; b2 < kw; ++b2) {
          const double v = I.taps[a * kw + b2];
          taps.push_back((float)v);
          ksq += v * v;
          if (std::fabs(v) > kmax) { kmax = std::fabs(v); a0 = a; b0 = b2; }
        }
      d.diagA = (float)(ksq / I.xi);
      // rank-one test: taps == u v^T with u = column b0, v = row a0 / taps[a0][b0]
      bool sep = kmax > 0.0;
      std::vector<double> u(kh), v(kw);
      if (sep) {
        for (int a = 0; a < kh; ++a) u[a] = I.taps[a * kw + b0];
        for (int b2 = 0; b2 < kw; ++b2) v[b2] = I.taps[a0 * kw + b2] / I.taps[a0 * kw + b0];
        for (int a = 0; a < kh && sep; ++a)
          for (int b2 = 0; b2 < kw; ++b2)
            if (std::fabs(u[a] * v[b2] - I.taps[a * kw + b2]) > 1e-6 * kmax) { sep = false; break; }
      }
      d.sep = sep ? 1 : 0;
      // autocorrelations g(d) = sum_t u(t) u(t + d), d = -(kh-1) .. kh-1 (same for v)
      d.gr_off = (int)taps.size();
      for (int dd = -(kh - 1); dd <= kh - 1; ++dd) {
        double acc = 0.0;
        for (int a = 0; a < kh; ++a)
          if (a + dd >= 0 && a + dd < kh) acc += u[a] * u[a + dd];
        taps.push_back((float)(sep ? acc : 0.0));
      }
      d.gc_off = (int)taps.size();
      for (int dd = -(kw - 1); dd <= kw - 1; ++dd) {
        double acc = 0.0;
        for (int b2 = 0; b2 < kw; ++b2)
          if (b2 + dd >= 0 && b2 + dd < kw) acc += v[b2] * v[b2 + dd];
        taps.push_back((float)(sep ? acc : 0.0));
      }
    } else if (I.op == OP_DFT || I.op == OP_HAD) {
      d.Rr = 0; d.Rc = 0; d.sep = 0; d.kh = 1; d.kw = 1;
      // H^T H of a masked orthonormal transform whose basis vectors have
      // entries of modulus 1 / sqrt(N) (Fourier, Walsh): its diagonal is the
      // kept fraction
      int kept = 0;
      for (long long q = 0; q < (long long)I.H * I.W; ++q) kept += I.mask[q] ? 1 : 0;
      d.diagA = (float)((double)kept / ((double)I.H * I.W) / I.xi);
    }
    lc.hinst.push_back(d);
    lc.inst_of.push_back(i);
  }
  lc.fast = !lc.hinst.empty();
  lc.all_jacobi = !lc.hinst.empty();
  for (const LikInst& d : lc.hinst) lc.all_jacobi = lc.all_jacobi && d.precond == PRECOND_JACOBI;
  for (const LikInst& d : lc.hinst) {
    lc.fast = lc.fast && d.precond == PRECOND_CIRCULANT && d.op != OP_HAD && d.op != OP_GAUSS &&
              d.npart <= d.ntiles;
  }
  // partial counts per finalisation stage: r.z / r.r (and p.q of masked-DFT
  // instances) come from the real-transform passes in the fast CG, everything
  // else from one partial per tile
  for (LikInst& d : lc.hinst) {
    const int tr = lc.fast ? d.npart : d.ntiles;
    d.fin_count[FIN_PREP] = d.ntiles;
    d.fin_count[FIN_SPEC] = d.ntiles;
    d.fin_count[FIN_INIT] = tr;
    d.fin_count[FIN_ALPHA] = (lc.fast && d.op == OP_DFT) ? d.npart : d.ntiles;
    if (d.op == OP_HAD) d.fin_count[FIN_ALPHA] = wht_partials(d.H, d.W);   // from the last transform pass
    d.fin_count[FIN_BETA] = tr;
    d.fin_count[FIN_SAMPLE] = d.ntiles;
  }
  if ((int)taps.size() > L.ntaps || (int)tiles.size() != L.ntiles) {
    err = "likelihood layout mismatch (taps or tiles)";
    return hipErrorInvalidValue;
  }
  hipError_t e = hipMemcpyAsync(lc.d_inst, lc.hinst.data(), sizeof(LikInst) * lc.hinst.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lc.d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !taps.empty())
    e = hipMemcpyAsync(lc.taps, taps.data(), sizeof(float) * taps.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // host vectors go out of scope
  if (e != hipSuccess) {
    err = hipGetErrorString(e);
    return e;
  }
  LikArgs A = make_args(lc);
  hipLaunchKernelGGL(k_spectrum_blur, dim3(lc.ntiles), dim3(256), 0, s, A);
  e = hipGetLastError();
  if (e == hipSuccess) e = dft_setup(lc, li, n, L.fft_bytes, s, err);
  if (e == hipSuccess) e = wht_setup(lc, li, n, L.wht_bytes, s, err);
  lc.gaussbuf = ws + L.gauss;
  if (e == hipSuccess) e = gauss_setup(lc, li, n, s, err);
  if (e != hipSuccess && err.empty()) err = hipGetErrorString(e);
  return e;
}

hipError_t lik_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  LikArgs A = make_args(lc);
  hipLaunchKernelGGL(k_hty_blur, dim3(lc.ntiles), dim3(256), 0, s, A, lc.ypix);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = dft_set_observation(lc, d_y, s)) != hipSuccess) return e;
  if ((e = gauss_set_observation(lc, d_y, s)) != hipSuccess) return e;
  return wht_set_observation(lc, d_y, s);
}

static hipError_t set_x_invalid(LikCtx& lc, hipStream_t s);

// Floats of one instance's observation: H x W, complex (two floats) for the DFT.
static long long obs_floats(const LikInst& L) {
  return (long long)L.H * L.W * (L.op == OP_DFT ? 2 : 1);
}

hipError_t lik_set_rbmc_noise(LikCtx& lc, const float* const* d_noise, hipStream_t s) {
  if (lc.nlik == 0 || lc.rbmc_ns_max == 0) return hipSuccess;
  hipError_t e;
  for (int k = 0; k < lc.rbmc_ns_max; ++k) {
    const size_t off = (size_t)lc.plane * (size_t)k;
    bool any_blur = false;
    for (int li = 0; li < (int)lc.hinst.size(); ++li) {
      const LikInst& L = lc.hinst[li];
      if (L.rbmc_ns <= k) continue;
      const long long nobs = obs_floats(L), npx = (long long)L.H * L.W;
      const float* e1 = d_noise[L.inst] + (size_t)k * (size_t)(nobs + npx);
      const float* e2 = e1 + nobs;
      // e2: white noise in pixel space, into its pitched plane
      e = hipMemcpy2DAsync(lc.rbmc_e2 + off + L.off, sizeof(float) * L.pitch, e2,
                           sizeof(float) * L.W, sizeof(float) * L.W, L.H, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
      // H^T e1 (unscaled; 1/sqrt(xi) is applied with every right-hand side)
      if (L.op == OP_BLUR) {
        // staged in the q plane (scratch between solves), correlated below
        e = hipMemcpy2DAsync(lc.planes[LP_Q] + L.off, sizeof(float) * L.pitch, e1,
                             sizeof(float) * L.W, sizeof(float) * L.W, L.H, hipMemcpyDeviceToDevice, s);
        any_blur = true;
      } else if (L.op == OP_DFT) {
        e = dft_back_project_inst(lc, li, e1, lc.rbmc_g + off, s);
      } else {
        e = wht_back_project_inst(lc, li, e1, lc.rbmc_g + off, s);
      }
      if (e != hipSuccess) return e;
    }
    if (any_blur) {
      LikArgs A = make_args(lc);
      A.hty = lc.rbmc_g + off;
      hipLaunchKernelGGL(k_hty_blur, dim3(lc.ntiles), dim3(256), 0, s, A, (const float*)lc.planes[LP_Q]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return set_x_invalid(lc, s);
}

hipError_t lik_reset(LikCtx& lc, hipStream_t s) { return set_x_invalid(lc, s); }
hipError_t lik_resume(LikCtx& lc, hipStream_t s) { return set_x_invalid(lc, s); }

__global__ void k_x_invalid(InstState* st, const LikInst* inst, int nlik) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nlik) {
    st[inst[i].inst].x_valid = 0;
    st[inst[i].inst].xprev_valid = 0;
    st[inst[i].inst].xs_valid = 0;
  }
}

static hipError_t set_x_invalid(LikCtx& lc, hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  hipLaunchKernelGGL(k_x_invalid, dim3((lc.nlik + 255) / 256), dim3(256), 0, s, lc.d_st, lc.d_inst,
                     lc.nlik);
  return hipGetLastError();
}

// q = A v on every blur tile (v = x for mode 0, the new direction for mode 1)
static hipError_t launch_apply_blur(LikCtx& lc, int mode, hipStream_t s) {
  const LikArgs A = make_args(lc);
  bool any_blur = false, all_sep = true;
  int rmax = 0;
  for (const LikInst& d : lc.hinst) {
    if (d.op != OP_BLUR) continue;
    any_blur = true;
    all_sep = all_sep && d.sep;
    rmax = std::max(rmax, std::max(d.Rr, d.Rc));
  }
  if (!any_blur) return hipSuccess;
  const dim3 g(lc.ntiles), b(256);
  if (!all_sep) {
    if (mode == 0) hipLaunchKernelGGL((k_apply<0>), g, b, 0, s, A);
    else hipLaunchKernelGGL((k_apply<1>), g, b, 0, s, A);
  } else if (rmax <= 8) {
    if (mode == 0) hipLaunchKernelGGL((k_hth_sep<8, 0>), g, b, 0, s, A);
    else hipLaunchKernelGGL((k_hth_sep<8, 1>), g, b, 0, s, A);
  } else {
    if (mode == 0) hipLaunchKernelGGL((k_hth_sep<kMaxRadius, 0>), g, b, 0, s, A);
    else hipLaunchKernelGGL((k_hth_sep<kMaxRadius, 1>), g, b, 0, s, A);
  }
  return hipGetLastError();
}

static hipError_t launch_apply(LikCtx& lc, int mode, hipStream_t s) {
  bool any_dft = false;
  for (const LikInst& d : lc.hinst) any_dft = any_dft || d.op == OP_DFT;
  return lik_timed(lc, KT_APPLY, s, [&]() -> hipError_t {
    if (any_dft) {
      hipError_t e = dft_apply(lc, mode, s);
      if (e != hipSuccess) return e;
    }
    if (!lc.wht.empty()) {
      hipError_t e = wht_apply(lc, mode, s);
      if (e != hipSuccess) return e;
    }
    return launch_apply_blur(lc, mode, s);
  });
}

static hipError_t fin(LikCtx& lc, int stage, hipStream_t s) {
  return lik_timed(lc, KT_FIN, s, [&]() {
    hipLaunchKernelGGL(k_lik_fin, dim3(lc.nlik), dim3(256), 0, s, make_args(lc), stage);
    return hipGetLastError();
  });
}

// One element-wise / reduction kernel of the likelihood update on every tile,
// timed in the KT_OTHER bucket.
template <class K, class... Args>
static hipError_t other(LikCtx& lc, hipStream_t s, K kernel, Args... args) {
  return lik_timed(lc, KT_OTHER, s, [&]() {
    hipLaunchKernelGGL(kernel, dim3(lc.ntiles), dim3(256), 0, s, args...);
    return hipGetLastError();
  });
}

// CG start for the right-hand side in b and the start in x: q = A x, r = b - q,
// z = M^{-1} r, r.z and r.r.
static hipError_t cg_start(LikCtx& lc, hipStream_t s) {
  hipError_t e;
  lc.pcur = 0;   // the first iteration sets p = z whatever the p planes hold
  if ((e = launch_apply(lc, 0, s)) != hipSuccess) return e;
  bool cg_init_needed = !blur_all_sep(lc);
  for (const LikInst& d : lc.hinst) cg_init_needed = cg_init_needed || d.op != OP_BLUR;
  if (cg_init_needed && (e = other(lc, s, k_cg_init, make_args(lc))) != hipSuccess) return e;
  if (lc.fast) {
    if ((e = rfft_precondition(lc, 0, s)) != hipSuccess) return e;
  } else {
    if ((e = fft_precondition(lc, s)) != hipSuccess) return e;
    if ((e = wht_precondition(lc, s)) != hipSuccess) return e;
    if ((e = other(lc, s, k_precond_dot, make_args(lc))) != hipSuccess) return e;
  }
  return fin(lc, FIN_INIT, s);
}

hipError_t lik_head(LikCtx& lc, float2* const S[5], hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  hipError_t e;
  lc.sample = 0;
  lc.pcur = 0;   // the first iteration sets p = z whatever the p planes hold
  if ((e = other(lc, s, k_lik_prep, make_args(lc), (const float2*)S[0], (const float2*)S[1],
                 (const float2*)S[2], (const float2*)S[3], (const float2*)S[4])) != hipSuccess)
    return e;
  if ((e = fin(lc, FIN_PREP, s)) != hipSuccess) return e;
  if ((e = other(lc, s, k_lik_spec, make_args(lc))) != hipSuccess) return e;
  if ((e = fin(lc, FIN_SPEC, s)) != hipSuccess) return e;
  return cg_start(lc, s);
}

hipError_t lik_iterations(LikCtx& lc, int n, hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  hipError_t e;
  const dim3 g(lc.ntiles), b(256);
  if (lc.fast) {
    for (int it = 0; it < n; ++it) {
      // p_out = z + beta p_in and q = A p_out: blur tiles by the direct
      // H^T H kernel, masked-DFT instances by the real transform
      e = lik_timed(lc, KT_APPLY, s, [&]() -> hipError_t {
        hipError_t e2 = launch_apply_blur(lc, 1, s);
        return e2 != hipSuccess ? e2 : rfft_product(lc, s);
      });
      if (e != hipSuccess) return e;
      // alpha = r.z / p.q is formed by every workgroup of the first transform
      // pass from the p.q partials, so no finishing kernel runs in between
      e = lik_timed(lc, KT_PRECOND, s, [&]() { return rfft_precondition(lc, 1, s); });   // with x, r update
      if (e != hipSuccess) return e;
      if ((e = fin(lc, FIN_BETA, s)) != hipSuccess) return e;
      lc.pcur ^= 1;
    }
    return hipGetLastError();
  }
  for (int it = 0; it < n; ++it) {
    if ((e = launch_apply(lc, 1, s)) != hipSuccess) return e;   // p_out = z + beta p_in, q = A p_out
    if ((e = fin(lc, FIN_ALPHA, s)) != hipSuccess) return e;
    if (lc.all_jacobi) {
      if ((e = other(lc, s, k_cg_update_jacobi, make_args(lc))) != hipSuccess) return e;
      if ((e = fin(lc, FIN_BETA, s)) != hipSuccess) return e;
      lc.pcur ^= 1;
      continue;
    }
    if ((e = other(lc, s, k_cg_update, make_args(lc))) != hipSuccess) return e;
    if ((e = fft_precondition(lc, s)) != hipSuccess) return e;
    if ((e = wht_precondition(lc, s)) != hipSuccess) return e;
    if ((e = other(lc, s, k_precond_dot, make_args(lc))) != hipSuccess) return e;
    if ((e = fin(lc, FIN_BETA, s)) != hipSuccess) return e;
    lc.pcur ^= 1;
  }
  return hipSuccess;
}

hipError_t lik_poll(LikCtx& lc, hipStream_t s, bool& all_done) {
  all_done = true;
  if (lc.nlik == 0) return hipSuccess;
  if (!lc.hst) {   // pinned, so the copy goes straight to host memory
    const hipError_t ea = hipHostMalloc(reinterpret_cast<void**>(&lc.hst),
                                        sizeof(InstState) * (size_t)std::max(lc.n_all, 1));
    if (ea != hipSuccess) {
      lc.hst = nullptr;
      return ea;
    }
  }
  hipError_t e = hipMemcpyAsync(lc.hst, lc.d_st, sizeof(InstState) * lc.n_all,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int i : lc.inst_of) all_done = all_done && lc.hst[i].cg_done;
  return hipSuccess;
}

// CG poll word for graph replays: the last kernel of a captured run of CG
// iterations writes to pinned host memory a sequence number one above the one
// it finds there (bits 0-31), whether every instance's solve has stopped (bit
// 32) and the largest iteration count of the instances' current solves (bits
// 33-62), so the host waits for the word to change instead of copying the flags
// back and synchronising the stream.  One block of 256 threads reduces the
// instances' flags and counts (each thread a strided share, then the block);
// thread 0's 64-bit system-scope store makes all fields visible to the host at
// once.
__global__ __launch_bounds__(256) void k_cg_poll_word(const LikInst* __restrict__ inst, int nlik,
                                                      const InstState* __restrict__ st,
                                                      long long* word) {
  int done = 1, iters = 0;
  for (int j = threadIdx.x; j < nlik; j += blockDim.x) {
    const InstState& s = st[inst[j].inst];
    done &= s.cg_done ? 1 : 0;
    iters = max(iters, s.cg_it);
  }
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    done &= __shfl_xor(done, off, kWave);
    iters = max(iters, __shfl_xor(iters, off, kWave));
  }
  __shared__ int wd[4], wi[4];
  if (threadIdx.x % kWave == 0) {
    wd[threadIdx.x / kWave] = done;
    wi[threadIdx.x / kWave] = iters;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  long long all = 1, most = 0;
  for (int k = 0; k < 4; ++k) {
    all &= wd[k];
    most = wi[k] > most ? wi[k] : most;
  }
  most = most < 0x3fffffff ? most : 0x3fffffff;
  const long long w = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  const unsigned seq = (unsigned)w + 1u;
  __hip_atomic_store(word, (most << 33) | (all << 32) | (long long)seq, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t lik_poll_word_alloc(LikCtx& lc) {
  if (lc.poll_word) return hipSuccess;
  void* h = nullptr;
  hipError_t e = hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return e;
  void* d = nullptr;
  e = hipHostGetDevicePointer(&d, h, 0);
  if (e != hipSuccess) {
    (void)hipHostFree(h);
    return e;
  }
  lc.poll_word = static_cast<long long*>(h);
  lc.poll_word_dev = static_cast<long long*>(d);
  __atomic_store_n(lc.poll_word, 0LL, __ATOMIC_RELEASE);
  return hipSuccess;
}

hipError_t lik_poll_word_launch(LikCtx& lc, hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  if (!lc.poll_word_dev) return hipErrorInvalidValue;   // lik_poll_word_alloc first
  hipLaunchKernelGGL(k_cg_poll_word, dim3(1), dim3(256), 0, s, lc.d_inst, lc.nlik,
                     (const InstState*)lc.d_st, lc.poll_word_dev);
  return hipGetLastError();
}

unsigned lik_poll_word_seq(const LikCtx& lc) {
  return lc.poll_word ? (unsigned)__atomic_load_n(lc.poll_word, __ATOMIC_ACQUIRE) : 0u;
}

hipError_t lik_poll_word_wait(LikCtx& lc, hipStream_t s, unsigned seq0, bool& all_done,
                              int& max_iters) {
  all_done = true;
  max_iters = 0;
  if (lc.nlik == 0) return hipSuccess;
  if (!lc.poll_word) return hipErrorInvalidValue;
  auto fresh = [&](bool& done) {
    const long long w = __atomic_load_n(lc.poll_word, __ATOMIC_ACQUIRE);
    if ((unsigned)w == seq0) return false;
    done = ((w >> 32) & 1) != 0;
    max_iters = (int)(w >> 33);
    return true;
  };
  for (unsigned spin = 1;; ++spin) {
    if (fresh(all_done)) return hipSuccess;
    if (spin % 256 == 0) {
      // the stream has drained without a new word only if the poll kernel
      // did not run; wait for the stream once and look again before failing
      const hipError_t q = hipStreamQuery(s);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return q;
      const hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      return fresh(all_done) ? hipSuccess : hipErrorUnknown;
    }
  }
}

hipError_t lik_tail(LikCtx& lc, float2* S0, hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  return other(lc, s, k_lik_site, make_args(lc), S0);
}

// CG iterations until every instance's solve has stopped (host polls).
static hipError_t iterate_to_done(LikCtx& lc, hipStream_t s) {
  hipError_t e;
  for (int it = 0; it < lc.max_iters; it += kCgPoll) {
    if ((e = lik_iterations(lc, kCgPoll, s)) != hipSuccess) return e;
    bool done = false;
    if ((e = lik_poll(lc, s, done)) != hipSuccess) return e;
    if (done) break;
  }
  return hipSuccess;
}

// RBMC sample solves after the mean solve (instances with rbmc_ns > 0).
static hipError_t rbmc_samples(LikCtx& lc, hipStream_t s) {
  hipError_t e;
  lc.sample = 0;
  if ((e = other(lc, s, k_rbmc_begin, make_args(lc))) != hipSuccess) return e;
  for (int k = 0; k < lc.rbmc_ns_max; ++k) {
    lc.sample = k;
    if ((e = other(lc, s, k_rbmc_rhs, make_args(lc))) != hipSuccess) return e;
    if ((e = fin(lc, FIN_SAMPLE, s)) != hipSuccess) return e;
    if ((e = cg_start(lc, s)) != hipSuccess) return e;
    if ((e = iterate_to_done(lc, s)) != hipSuccess) return e;
    if ((e = other(lc, s, k_rbmc_acc, make_args(lc))) != hipSuccess) return e;
  }
  lc.sample = 0;
  return hipSuccess;
}

hipError_t lik_update(LikCtx& lc, float2* const S[5], hipStream_t s) {
  if (lc.nlik == 0) return hipSuccess;
  hipError_t e = lik_head(lc, S, s);
  if (e != hipSuccess) return e;
  if ((e = iterate_to_done(lc, s)) != hipSuccess) return e;
  if (lc.rbmc_ns_max && (e = rbmc_samples(lc, s)) != hipSuccess) return e;
  // the host state was pulled by the last CG poll, after this sweep's preparation
  if (!lc.gauss.empty() && (e = gauss_update(lc, lc.hst, s)) != hipSuccess) return e;
  return lik_tail(lc, S[0], s);
}

void lik_destroy(LikCtx& lc) {
  for (hipEvent_t e : lc.ev) (void)hipEventDestroy(e);
  lc.ev.clear();
  if (lc.hst) (void)hipHostFree(lc.hst);
  lc.hst = nullptr;
  if (lc.poll_word) (void)hipHostFree(lc.poll_word);
  lc.poll_word = lc.poll_word_dev = nullptr;
  dft_destroy(lc);
}

void lik_timing(LikCtx& lc, bool enable, bool clear) {
  lc.timing = enable;
  if (clear) {
    lc.ev_used = 0;
    for (auto& b : lc.ev_k) b.clear();
    lc.dgemm_flops = 0.0;
  }
}

static hipError_t sum_events(LikCtx& lc, const std::vector<std::pair<int, int>>& b, double& ms, int& n) {
  ms = 0.0;
  n = 0;
  for (auto& pr : b) {
    float t = 0.f;
    hipError_t e = hipEventElapsedTime(&t, lc.ev[pr.first], lc.ev[pr.second]);
    if (e != hipSuccess) return e;
    ms += t;
    n += 1;
  }
  return hipSuccess;
}

hipError_t lik_timing_read(LikCtx& lc, double* ms, int* launches) {
  for (int k = 0; k < KT_COUNT; ++k) {
    hipError_t e = sum_events(lc, lc.ev_k[k], ms[k], launches[k]);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace eptv
