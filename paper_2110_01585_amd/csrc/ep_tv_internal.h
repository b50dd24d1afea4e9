// Internal declarations shared by the HIP translation units of libeptv.
// Device data layout (all in the caller-provided workspace):
//   * per-pixel state of every instance lives in "planes": one plane holds all
//     instances back to back, instance i at element offset InstDev::off, rows of
//     InstDev::pitch elements (pitch a multiple of 64, so every row starts
//     256-byte aligned and a lane's pixel pair is 16-byte aligned);
//   * the five EP sites are float2 planes of (tau, eta) (natural parameters,
//     Sec. III-A); q_{x,0} is S0, the colour-class sites S1..S4 exist twice
//     (ping-pong between sweeps);
//   * per-instance scalars (lambda, convergence, likelihood-site scalars) are in
//     an InstState array; per-tile partial sums are in plain arrays.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eptv {

constexpr int kWave = 64;
constexpr int kStripPx = 2 * kWave;       // columns a wave holds (2 per lane)
constexpr int kStripInt = kStripPx - 4;   // interior columns per strip (2-px halo each side)
constexpr int kWavesPerBlock = 4;
constexpr float kPrecFloor = 1e-8f;       // clamp: site variance < 0 or > 1e8 -> 1e8
constexpr float kSiteInitPrec = 1e-8f;    // initial TV-site variance 1e8

enum { OP_IDENTITY = 0, OP_BLUR = 1, OP_DFT = 2, OP_HAD = 3, OP_GAUSS = 4 };
enum { BND_FREE = 0, BND_PERIODIC = 1 };

struct InstDev {
  int H, W, pitch, bnd;
  long long off;             // element offset of pixel (0, 0) in every plane
  int op, strips, chunks, tile0;
  int ntiles, chunk_rows, npix, wmap;     // wmap: per-pixel noise precisions (identity operator)
  float xi, inv_xi, alpha, pad1;
  int lik_tile0, lik_ntiles;               // likelihood-kernel tiles (non-identity operators)
  int pad2, pad3;
  float mix_dla, mix_dv, mix_v1, mix_v2;   // mixture factor: log(a2/a1), v1 - v2, v1, v2
};

// factor kinds (the sweep is compiled once per kind; a context uses one)
enum { PRIOR_L1 = 0, PRIOR_MOG2 = 1, PRIOR_BG = 2 };

struct InstState {
  double lam, lam_prev;      // current / previous lambda
  double abar;               // a_bar_u of the last sweep
  double yrange;             // max y - min y (pixel-space observation)
  double dmu, dv;            // last sweep's relative deltas
  double gamma, dbar;        // likelihood site: spectral precision, mean cavity precision
  double cg_rr, cg_bb;       // CG residual / rhs squared norms
  double cg_rz, cg_alpha, cg_beta;
  double cg_stop2;           // this solve's stopping threshold on ||r||^2 / ||b||^2
  unsigned clamps, flags, active, sweeps;
  int cg_last, cg_total, converged, cg_done;
  int cg_it, x_valid, warm, warm_ok;   // warm: sites were set from a prediction (no skipped q0)
  int xprev_valid, restart;            // restart: cold re-initialisation pending (host-set)
  double yscale;                       // max(range, max |.|) of the pixel-space observation
  int cold_restarts, xs_valid;         // xs_valid: the RBMC sample solutions hold the last solves
  int pc_scaled;                       // this solve's circulant preconditioner is diagonally scaled
};

// FLAG_DIVERGED: the global mean after a likelihood-site update left
// kDivergeFactor times the observation's scale (EP is not guaranteed to converge;
// the spectral variance estimator can run away on sparse masks).
enum { FLAG_NONFINITE = 1u, FLAG_DIVERGED = 2u };
constexpr double kDivergeFactor = 1e3;

// The sweep reads the TV sites of the previous sweep from one buffer and writes
// the new ones to the other (ping-pong): a wave's halo pixels are interior
// pixels of its neighbours, which must be read before anyone rewrites them.
struct SweepArgs {
  const float2* S0;
  const float2* I1; const float2* I2; const float2* I3; const float2* I4;   // in
  float2* O1; float2* O2; float2* O3; float2* O4;                           // out
  const InstDev* inst;
  InstState* st;
  const int4* tiles;         // {instance, strip, chunk, 0}
  int ntiles;
  double* part_eabs;
  float* part_dmu;
  float* part_dv;
  unsigned* part_clamp;
  unsigned* part_flags;
  const float* part_mu;      // per likelihood tile: max |mu| after the likelihood-site update
  int prior;                 // PRIOR_* of every instance of the context
  int em_opt;                // EM approximation of a_0 (Sec. IV): 1, 2 or 3 (l1 only)
  int persistent;            // 1: one resident grid loops over the tile blocks
};

// Map a block index so that consecutive tiles land on the same XCD (workgroups
// are dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int nx = 8;
  int q = nb / nx, r = nb % nx;
  int x = bid % nx, j = bid / nx;
  int base = (x < r) ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return base + j;
}

// ---- launchers (defined in the .hip files) ----
hipError_t launch_tv_sweep(const SweepArgs& a, bool want_delta, hipStream_t s);

hipError_t launch_tilted(int n, const float* m, const float* s, float lam, float* rho, float* del,
                         float* eabs, hipStream_t st);
hipError_t launch_tilted_mixture(int n, const float* m, const float* s, float dla, float dv,
                                 float v1, float v2, float* rho, float* del, float* eabs,
                                 hipStream_t st);
// only_restart: re-initialise only the instances whose InstState::restart is set.
// wpix: per-pixel noise precisions of instances with InstDev::wmap (else unused).
hipError_t launch_init_cold(float2* const S[5], const float* y_pix, const InstDev* inst,
                            InstState* st, const int4* tiles, int ntiles, hipStream_t s,
                            bool only_restart = false, const float* wpix = nullptr);
// Option 1 of the EM approximations of a_0 (Sec. IV): per sweep tile, the sum
// over the edges owned by its pixels (right and lower neighbour) of
// E|x_i - x_j| under the global Q(x) of the sites S, into part.
hipError_t launch_em_ax(float2* const S[5], const InstDev* inst, const InstState* st,
                        const int4* tiles, int ntiles, double* part, hipStream_t s);
// 1 / var into the per-pixel noise-precision plane, for the given instances.
hipError_t launch_noise_prec(float* wpix, const InstDev* inst, const int4* tiles, int ntiles,
                             const float* const* var_tab, hipStream_t s);
hipError_t launch_finalize(const InstDev* inst, InstState* st, int n, const SweepArgs& a,
                           int em, double tol, hipStream_t s);
hipError_t launch_marginals(float2* const S[5], const InstDev* inst, const int4* tiles, int ntiles,
                            float* const* d_mean_tab, float* const* d_var_tab, hipStream_t s);
hipError_t launch_sites_io(float2* const S[5], const InstDev* inst, const int4* tiles, int ntiles,
                           float* const* d_tab, int to_user, hipStream_t s);
hipError_t launch_yrange(const float* y_pix, const InstDev* inst, InstState* st, int n,
                         const int4* tiles, int ntiles, float* plo, float* phi, hipStream_t s);
// Warm start from predicted marginals (device pointer tables, one per instance):
// validates the prediction, computes lambda_0 = scale * (N / a_x)^power (a_x: sum
// over pairs of the folded-normal mean of x_i - x_j under the prediction) when
// scale > 0, and overwrites the sites of every accepted instance.
hipError_t launch_init_warm(float2* const S[5], const float* y_pix, const InstDev* inst,
                            InstState* st, int n, const int4* tiles, int ntiles,
                            const float* const* mu_tab, const float* const* var_tab,
                            double lambda_scale, double lambda_power, double* part_a,
                            unsigned* part_f, hipStream_t s, const float* wpix = nullptr);

}  // namespace eptv
