// Element-wise and reduction kernels around the sweep: cold initialisation
// (initialisation line of Algorithm 1), per-instance finalisation of a sweep
// (EM update lambda = N / a_bar_u of Algorithm 2 and the convergence rule),
// the gather of the global approximation (Eq. (Q_x_final)), site checkpoint
// copies and the observation range.
//
// Element-wise kernels walk the same tile list as the sweep (one tile = the
// 124 interior columns of a strip times one chunk of rows), one block per tile.
#include "ep_tv_internal.h"

namespace eptv {

struct TileBox {
  int c0, c1, r0, r1;
};

__device__ __forceinline__ TileBox tile_box(const int4 td, const InstDev& I) {
  TileBox b;
  b.c0 = td.y * kStripInt;
  b.c1 = min(b.c0 + kStripInt, I.W);
  b.r0 = td.z * I.chunk_rows;
  b.r1 = min(b.r0 + I.chunk_rows, I.H);
  return b;
}

// Pixel (r, c) is touched by some pair of colour class k (0-based kk = k-1).
__device__ __forceinline__ bool covered(int kk, int r, int c, const InstDev& I) {
  if (I.bnd == BND_PERIODIC) return true;
  switch (kk) {
    case 0: return (c & 1) ? true : (c + 1 < I.W);
    case 1: return (c & 1) ? (c + 1 < I.W) : (c >= 1);
    case 2: return (r & 1) ? true : (r + 1 < I.H);
    default: return (r & 1) ? (r + 1 < I.H) : (r >= 1);
  }
}

struct SitePtrs {
  float2* S[5];
};

__global__ __launch_bounds__(256) void k_init_cold(SitePtrs sp, const float* __restrict__ y_pix,
                                                   const InstDev* __restrict__ inst,
                                                   const InstState* __restrict__ st,
                                                   const int4* __restrict__ tiles, int only_restart,
                                                   const float* __restrict__ wpix) {
  const int4 td = tiles[blockIdx.x];
  if (only_restart && !st[td.x].restart) return;
  const InstDev I = inst[td.x];
  const TileBox b = tile_box(td, I);
  const int cols = b.c1 - b.c0;
  const int n = cols * (b.r1 - b.r0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = b.r0 + i / cols;
    const int c = b.c0 + i % cols;
    const long long p = I.off + (long long)r * I.pitch + c;
    const float yv = y_pix[p];
    const float w = I.wmap ? wpix[p] : I.inv_xi;   // noise precision of the pixel
    sp.S[0][p] = make_float2(w, yv * w);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      sp.S[kk + 1][p] = covered(kk, r, c, I) ? make_float2(kSiteInitPrec, 0.f) : make_float2(0.f, 0.f);
  }
}

hipError_t launch_init_cold(float2* const S[5], const float* y_pix, const InstDev* inst,
                            InstState* st, const int4* tiles, int ntiles, hipStream_t s,
                            bool only_restart, const float* wpix) {
  SitePtrs sp;
  for (int k = 0; k < 5; ++k) sp.S[k] = S[k];
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_cold, dim3(ntiles), dim3(256), 0, s, sp, y_pix, inst, st, tiles,
                     only_restart ? 1 : 0, wpix);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Warm start from a predicted posterior N(mu_hat, diag var_hat).  The sites are
// chosen so that the global approximation (Eq. (Q_x_final)) equals the
// prediction: for H = I the likelihood site is exact and keeps (1/xi, y/xi) and
// the rest of the precision (at least 1e-8 per class) is split equally over the
// covering colour classes; otherwise precision and eta are split equally over
// the likelihood site and the covering classes.  lambda_0 follows option 1 of
// the EM approximations of a_0 (Sec. IV-B): a_x = sum over pairs of E|x_i - x_j|
// under the prediction (a folded-normal mean), lambda_0 = scale * (N / a_x)^power.
__device__ __forceinline__ double folded_mean(double d, double var) {
  const double sd = sqrt(var);
  return d * erf(d / (sd * 1.4142135623730951)) + sd * 0.7978845608028654 * exp(-d * d / (2.0 * var));
}

__device__ __forceinline__ bool pred_ok(float m, float v) {
  return isfinite(m) && isfinite(v) && v > 0.f;
}

__global__ __launch_bounds__(256) void k_warm_scan(const InstDev* __restrict__ inst,
                                                   const int4* __restrict__ tiles,
                                                   const float* const* __restrict__ mu_tab,
                                                   const float* const* __restrict__ var_tab,
                                                   double* __restrict__ part_a,
                                                   unsigned* __restrict__ part_f) {
  const int4 td = tiles[blockIdx.x];
  const InstDev I = inst[td.x];
  const TileBox b = tile_box(td, I);
  const float* mu = mu_tab[td.x];
  const float* va = var_tab[td.x];
  const int cols = b.c1 - b.c0;
  const int n = cols * (b.r1 - b.r0);
  double acc = 0.0;
  unsigned bad = 0u;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = b.r0 + i / cols, c = b.c0 + i % cols;
    const long long p = (long long)r * I.W + c;
    const float m0 = mu[p], v0 = va[p];
    if (!pred_ok(m0, v0)) {
      bad = 1u;
      continue;
    }
    // pairs owned by this pixel: to the right and downwards (wrapping when periodic)
    int cr = c + 1, rd = r + 1;
    if (I.bnd == BND_PERIODIC) {
      cr = cr == I.W ? 0 : cr;
      rd = rd == I.H ? 0 : rd;
    }
    if (cr < I.W) {
      const long long q = (long long)r * I.W + cr;
      const float m1 = mu[q], v1 = va[q];
      if (pred_ok(m1, v1)) acc += folded_mean((double)m0 - m1, (double)v0 + v1);
    }
    if (rd < I.H) {
      const long long q = (long long)rd * I.W + c;
      const float m1 = mu[q], v1 = va[q];
      if (pred_ok(m1, v1)) acc += folded_mean((double)m0 - m1, (double)v0 + v1);
    }
  }
  __shared__ double sa[256];
  __shared__ unsigned sf[256];
  sa[threadIdx.x] = acc;
  sf[threadIdx.x] = bad;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sf[threadIdx.x] |= sf[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_a[blockIdx.x] = sa[0];
    part_f[blockIdx.x] = sf[0];
  }
}

__global__ __launch_bounds__(256) void k_warm_fin(const InstDev* __restrict__ inst,
                                                  InstState* __restrict__ st,
                                                  const double* __restrict__ part_a,
                                                  const unsigned* __restrict__ part_f, double scale,
                                                  double power) {
  const InstDev I = inst[blockIdx.x];
  InstState& S = st[blockIdx.x];
  __shared__ double sa[256];
  __shared__ unsigned sf[256];
  double a = 0.0;
  unsigned f = 0u;
  for (int t = threadIdx.x; t < I.ntiles; t += blockDim.x) {
    a += part_a[I.tile0 + t];
    f |= part_f[I.tile0 + t];
  }
  sa[threadIdx.x] = a;
  sf[threadIdx.x] = f;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sf[threadIdx.x] |= sf[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (sf[0]) {
    S.warm = 0;
    S.warm_ok = 0;
    return;
  }
  S.warm = 1;
  S.warm_ok = 1;
  if (scale > 0.0 && sa[0] > 0.0) {
    S.lam = scale * pow((double)I.npix / sa[0], power);
    S.lam_prev = S.lam;
  }
}

__global__ __launch_bounds__(256) void k_warm_write(SitePtrs sp, const float* __restrict__ y_pix,
                                                    const InstDev* __restrict__ inst,
                                                    const InstState* __restrict__ st,
                                                    const int4* __restrict__ tiles,
                                                    const float* const* __restrict__ mu_tab,
                                                    const float* const* __restrict__ var_tab,
                                                    const float* __restrict__ wpix) {
  const int4 td = tiles[blockIdx.x];
  if (!st[td.x].warm_ok) return;                 // rejected: the cold sites stay
  const InstDev I = inst[td.x];
  const TileBox b = tile_box(td, I);
  const float* mu = mu_tab[td.x];
  const float* va = var_tab[td.x];
  const int cols = b.c1 - b.c0;
  const int n = cols * (b.r1 - b.r0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = b.r0 + i / cols, c = b.c0 + i % cols;
    const long long p = I.off + (long long)r * I.pitch + c;
    const float m = mu[(long long)r * I.W + c];
    const float prec = 1.f / va[(long long)r * I.W + c];
    bool cov[4];
    int cnt = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      cov[kk] = covered(kk, r, c, I);
      cnt += cov[kk] ? 1 : 0;
    }
    float tk, ek;
    if (I.op == OP_IDENTITY) {
      const float yv = y_pix[p];
      const float w = I.wmap ? wpix[p] : I.inv_xi;
      sp.S[0][p] = make_float2(w, yv * w);
      const float rest = fmaxf(prec - w, (float)cnt * kSiteInitPrec);
      const float rest_eta = m * (w + rest) - yv * w;
      const float share = cnt ? 1.f / (float)cnt : 0.f;
      tk = rest * share;
      ek = rest_eta * share;
    } else {
      const float share = 1.f / (float)(1 + cnt);
      tk = prec * share;
      ek = m * prec * share;
      sp.S[0][p] = make_float2(tk, ek);
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) sp.S[kk + 1][p] = cov[kk] ? make_float2(tk, ek) : make_float2(0.f, 0.f);
  }
}

hipError_t launch_init_warm(float2* const S[5], const float* y_pix, const InstDev* inst,
                            InstState* st, int n, const int4* tiles, int ntiles,
                            const float* const* mu_tab, const float* const* var_tab,
                            double lambda_scale, double lambda_power, double* part_a,
                            unsigned* part_f, hipStream_t s, const float* wpix) {
  if (ntiles == 0) return hipSuccess;
  SitePtrs sp;
  for (int k = 0; k < 5; ++k) sp.S[k] = S[k];
  hipLaunchKernelGGL(k_warm_scan, dim3(ntiles), dim3(256), 0, s, inst, tiles, mu_tab, var_tab, part_a,
                     part_f);
  hipLaunchKernelGGL(k_warm_fin, dim3(n), dim3(256), 0, s, inst, st, part_a, part_f, lambda_scale,
                     lambda_power);
  hipLaunchKernelGGL(k_warm_write, dim3(ntiles), dim3(256), 0, s, sp, y_pix, inst, st, tiles, mu_tab,
                     var_tab, wpix);
  return hipGetLastError();
}

// Option 1 of the approximations of a_0: every pixel of the tile adds its edge
// to the right neighbour and to the lower one (with the wrap-around pairs of a
// periodic boundary), E|x_i - x_j| under Q(x) = N(mu, diag v).  Block sums in
// a fixed order.
__global__ __launch_bounds__(256) void k_em_ax(SitePtrs sp, const InstDev* __restrict__ inst,
                                               const InstState* __restrict__ st,
                                               const int4* __restrict__ tiles, double* part) {
  __shared__ double red[256];
  const int4 td = tiles[blockIdx.x];
  const InstDev I = inst[td.x];
  double acc = 0.0;
  if (st[td.x].active) {
    const TileBox b = tile_box(td, I);
    const bool per = I.bnd == BND_PERIODIC;
    const int cols = b.c1 - b.c0;
    const int n = cols * (b.r1 - b.r0);
    auto moments = [&](int r, int c, double& mu, double& v) {
      const long long p = I.off + (long long)r * I.pitch + c;
      double t = 0.0, e = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const float2 s2 = sp.S[k][p];
        t += (double)s2.x;
        e += (double)s2.y;
      }
      mu = e / t;
      v = 1.0 / t;
    };
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int r = b.r0 + i / cols, c = b.c0 + i % cols;
      double m0, v0, m1, v1;
      moments(r, c, m0, v0);
      if (c + 1 < I.W || (per && I.W > 1)) {
        moments(r, c + 1 < I.W ? c + 1 : 0, m1, v1);
        acc += folded_mean(m0 - m1, v0 + v1);
      }
      if (r + 1 < I.H || (per && I.H > 1)) {
        moments(r + 1 < I.H ? r + 1 : 0, c, m1, v1);
        acc += folded_mean(m0 - m1, v0 + v1);
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

hipError_t launch_em_ax(float2* const S[5], const InstDev* inst, const InstState* st,
                        const int4* tiles, int ntiles, double* part, hipStream_t s) {
  SitePtrs sp;
  for (int k = 0; k < 5; ++k) sp.S[k] = S[k];
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_em_ax, dim3(ntiles), dim3(256), 0, s, sp, inst, st, tiles, part);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_noise_prec(float* __restrict__ wpix,
                                                    const InstDev* __restrict__ inst,
                                                    const int4* __restrict__ tiles,
                                                    const float* const* __restrict__ var_tab) {
  const int4 td = tiles[blockIdx.x];
  const InstDev I = inst[td.x];
  const float* v = var_tab[td.x];
  if (!I.wmap || !v) return;
  const TileBox b = tile_box(td, I);
  const int cols = b.c1 - b.c0;
  const int n = cols * (b.r1 - b.r0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = b.r0 + i / cols, c = b.c0 + i % cols;
    wpix[I.off + (long long)r * I.pitch + c] = 1.f / v[(long long)r * I.W + c];
  }
}

hipError_t launch_noise_prec(float* wpix, const InstDev* inst, const int4* tiles, int ntiles,
                             const float* const* var_tab, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_noise_prec, dim3(ntiles), dim3(256), 0, s, wpix, inst, tiles, var_tab);
  return hipGetLastError();
}

// One block per instance: deterministic fixed-shape reduction of the sweep's
// per-tile partials, then lambda / convergence / counters.
__global__ __launch_bounds__(256) void k_finalize(const InstDev* __restrict__ inst,
                                                  InstState* __restrict__ st, SweepArgs a, int em,
                                                  double tol) {
  __shared__ double se[256];
  __shared__ float sm[256], sv[256];
  __shared__ unsigned sc[256], sf[256];
  const int i = blockIdx.x;
  const InstDev I = inst[i];
  InstState& S = st[i];
  if (!S.active) return;   // frozen before this sweep: nothing ran
  double e = 0.0;
  float dm = 0.f, dv = 0.f;
  unsigned cl = 0u, fl = 0u;
  // kU partials per thread are requested before the first is folded in (each
  // thread still takes its partials in ascending order), so their latencies
  // overlap instead of adding up
  constexpr int kU = 8;
  for (int t0 = threadIdx.x; t0 < I.ntiles; t0 += kU * 256) {
    double ve[kU];
    float vm[kU], vv[kU];
    unsigned vc[kU], vf[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + 256 * u;
      const int g = I.tile0 + (t < I.ntiles ? t : 0);
      ve[u] = a.part_eabs[g];
      vm[u] = a.part_dmu[g];
      vv[u] = a.part_dv[g];
      vc[u] = a.part_clamp[g];
      vf[u] = a.part_flags[g];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (t0 + 256 * u >= I.ntiles) break;
      e += ve[u];
      dm = fmaxf(dm, vm[u]);
      dv = fmaxf(dv, vv[u]);
      cl += vc[u];
      fl |= vf[u];
    }
  }
  // divergence rule: the global mean after this sweep's likelihood-site update
  float mm = 0.f;
  for (int t0 = threadIdx.x; t0 < I.lik_ntiles; t0 += kU * 256) {
    float vu[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = t0 + 256 * u;
      vu[u] = t < I.lik_ntiles ? a.part_mu[I.lik_tile0 + t] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) mm = fmaxf(mm, vu[u]);
  }
  if (I.lik_ntiles > 0 && !(mm <= (float)(kDivergeFactor * S.yscale))) fl |= FLAG_DIVERGED;
  se[threadIdx.x] = e; sm[threadIdx.x] = dm; sv[threadIdx.x] = dv; sc[threadIdx.x] = cl;
  sf[threadIdx.x] = fl;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      se[threadIdx.x] += se[threadIdx.x + w];
      sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
      sv[threadIdx.x] = fmaxf(sv[threadIdx.x], sv[threadIdx.x + w]);
      sc[threadIdx.x] += sc[threadIdx.x + w];
      sf[threadIdx.x] |= sf[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double abar = se[0];
    S.abar = abar;
    S.clamps += sc[0];
    S.flags |= sf[0];
    S.sweeps += 1;
    S.lam_prev = S.lam;
    if (em && abar > 0.0) S.lam = (double)I.npix / abar;
    S.dmu = (double)sm[0] / (S.yrange > 0.0 ? S.yrange : 1.0);
    S.dv = (double)sv[0];
    if (S.flags & (FLAG_NONFINITE | FLAG_DIVERGED)) {
      S.active = 0u;
    } else if (tol > 0.0) {
      const double dl = fabs(S.lam / S.lam_prev - 1.0);
      if (S.dmu <= tol && S.dv <= 10.0 * tol && (!em || dl <= tol)) {
        S.converged = 1;
        S.active = 0u;
      }
    }
  }
}

hipError_t launch_finalize(const InstDev* inst, InstState* st, int n, const SweepArgs& a, int em,
                           double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(n), dim3(256), 0, s, inst, st, a, em, tol);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_marginals(SitePtrs sp, const InstDev* __restrict__ inst,
                                                   const int4* __restrict__ tiles,
                                                   float* const* __restrict__ mean_tab,
                                                   float* const* __restrict__ var_tab) {
  const int4 td = tiles[blockIdx.x];
  const InstDev I = inst[td.x];
  const TileBox b = tile_box(td, I);
  float* mo = mean_tab ? mean_tab[td.x] : nullptr;
  float* vo = var_tab ? var_tab[td.x] : nullptr;
  const int cols = b.c1 - b.c0;
  const int n = cols * (b.r1 - b.r0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = b.r0 + i / cols;
    const int c = b.c0 + i % cols;
    const long long p = I.off + (long long)r * I.pitch + c;
    double t = 0.0, e = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const float2 v = sp.S[k][p];
      t += (double)v.x;
      e += (double)v.y;
    }
    const long long q = (long long)r * I.W + c;
    if (mo) mo[q] = (float)(e / t);
    if (vo) vo[q] = (float)(1.0 / t);
  }
}

hipError_t launch_marginals(float2* const S[5], const InstDev* inst, const int4* tiles, int ntiles,
                            float* const* d_mean_tab, float* const* d_var_tab, hipStream_t s) {
  SitePtrs sp;
  for (int k = 0; k < 5; ++k) sp.S[k] = S[k];
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_marginals, dim3(ntiles), dim3(256), 0, s, sp, inst, tiles, d_mean_tab,
                     d_var_tab);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sites_io(SitePtrs sp, const InstDev* __restrict__ inst,
                                                  const int4* __restrict__ tiles,
                                                  float* const* __restrict__ tab, int to_user) {
  const int4 td = tiles[blockIdx.x];
  const InstDev I = inst[td.x];
  const TileBox b = tile_box(td, I);
  float* u = tab[td.x];
  const long long plane = (long long)I.H * I.W;
  const int cols = b.c1 - b.c0;
  const int n = cols * (b.r1 - b.r0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = b.r0 + i / cols;
    const int c = b.c0 + i % cols;
    const long long p = I.off + (long long)r * I.pitch + c;
    const long long q = (long long)r * I.W + c;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      if (to_user) {
        const float2 v = sp.S[k][p];
        u[(2 * k) * plane + q] = v.x;
        u[(2 * k + 1) * plane + q] = v.y;
      } else {
        sp.S[k][p] = make_float2(u[(2 * k) * plane + q], u[(2 * k + 1) * plane + q]);
      }
    }
  }
}

hipError_t launch_sites_io(float2* const S[5], const InstDev* inst, const int4* tiles, int ntiles,
                           float* const* d_tab, int to_user, hipStream_t s) {
  SitePtrs sp;
  for (int k = 0; k < 5; ++k) sp.S[k] = S[k];
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sites_io, dim3(ntiles), dim3(256), 0, s, sp, inst, tiles, d_tab, to_user);
  return hipGetLastError();
}

// Range and scale of the pixel-space observation, in two steps so that the
// whole chip reads it: every sweep tile reduces its pixels to a min and a max
// (partials at the tile's index), then one block per instance reduces its
// tiles' partials.  Min and max do not depend on the order.
__device__ __forceinline__ void block_minmax(float& lo, float& hi) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, off, kWave));
  }
  __shared__ float wl[4], wh[4];
  if (threadIdx.x % kWave == 0) {
    wl[threadIdx.x / kWave] = lo;
    wh[threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  lo = fminf(fminf(wl[0], wl[1]), fminf(wl[2], wl[3]));
  hi = fmaxf(fmaxf(wh[0], wh[1]), fmaxf(wh[2], wh[3]));
}

__global__ __launch_bounds__(256) void k_yrange_tiles(const float* __restrict__ y_pix,
                                                      const InstDev* __restrict__ inst,
                                                      const int4* __restrict__ tiles,
                                                      float* __restrict__ plo,
                                                      float* __restrict__ phi) {
  const int tile = blockIdx.x;
  const int4 td = tiles[tile];
  const InstDev I = inst[td.x];
  const int c0 = td.y * kStripInt, c1 = min(c0 + kStripInt, I.W);
  const int r0 = td.z * I.chunk_rows, r1 = min(r0 + I.chunk_rows, I.H);
  const int cols = c1 - c0, n = cols * (r1 - r0);
  float lo = 3.0e38f, hi = -3.0e38f;
  // up to 8 loads per thread in flight before the first comparison
  constexpr int kU = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += kU * 256) {
    float v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * 256;
      const int ii = i < n ? i : i0;   // a repeated pixel leaves min and max unchanged
      v[u] = y_pix[I.off + (long long)(r0 + ii / cols) * I.pitch + c0 + ii % cols];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      lo = fminf(lo, v[u]);
      hi = fmaxf(hi, v[u]);
    }
  }
  block_minmax(lo, hi);
  if (threadIdx.x == 0) {
    plo[tile] = lo;
    phi[tile] = hi;
  }
}

__global__ __launch_bounds__(256) void k_yrange_fin(const InstDev* __restrict__ inst,
                                                    InstState* __restrict__ st,
                                                    const float* __restrict__ plo,
                                                    const float* __restrict__ phi) {
  const InstDev I = inst[blockIdx.x];
  float lo = 3.0e38f, hi = -3.0e38f;
  for (int t = threadIdx.x; t < I.ntiles; t += 256) {
    lo = fminf(lo, plo[I.tile0 + t]);
    hi = fmaxf(hi, phi[I.tile0 + t]);
  }
  block_minmax(lo, hi);
  if (threadIdx.x == 0) {
    const double lo_d = (double)lo, hi_d = (double)hi;
    st[blockIdx.x].yrange = hi_d - lo_d;
    st[blockIdx.x].yscale = fmax(hi_d - lo_d, fmax(fabs(lo_d), fabs(hi_d)));
  }
}

hipError_t launch_yrange(const float* y_pix, const InstDev* inst, InstState* st, int n,
                         const int4* tiles, int ntiles, float* plo, float* phi, hipStream_t s) {
  if (n <= 0 || ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_yrange_tiles, dim3(ntiles), dim3(256), 0, s, y_pix, inst, tiles, plo, phi);
  hipLaunchKernelGGL(k_yrange_fin, dim3(n), dim3(256), 0, s, inst, st, plo, phi);
  return hipGetLastError();
}

}  // namespace eptv

