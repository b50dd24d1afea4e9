// Likelihood-site update q_{x,0} (Eqs. (tilted_P_1) and (update_q0_x)) for the
// non-identity operators: interface between the host schedule and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ep_tv_internal.h"

namespace eptv {

constexpr int kMaxTaps = 17;
constexpr int kLikTW = 64;       // likelihood-kernel tile: 64 columns x 16 rows
constexpr int kLikTH = 16;
constexpr int kMaxRadius = kMaxTaps - 1;   // radius of the combined H^T H kernel
// Iteration cap of one likelihood solve.  It binds only in the first sweeps
// from a cold start, whose solves cannot reach the tolerance in any affordable
// number of iterations (thousands, with tau_c spanning ten decades) and whose
// error EP forgets; the solves near the fixed point need a few iterations.
constexpr int kCgMaxIters = 50;
constexpr double kCgTol = 1e-8;            // relative residual ||r|| / ||b||
constexpr int kCgPoll = 4;                 // CG iterations between convergence checks (even)
constexpr int kCgHeadShort = 2;            // CG iterations of the short head graph (even)
// A blur instance's circulant preconditioner is diagonally scaled for a solve
// whose predecessor needed more than this many iterations (far from the fixed
// point, where the cavity precisions vary most and the scaling pays).
constexpr int kCgScaleAbove = 10;

inline bool fft_size_ok(int n) { return n >= 4 && n <= 4096 && (n & (n - 1)) == 0; }

// Likelihood-kernel tiles of an H x W instance (64 x 16 pixels each).
inline int lik_tile_count(int H, int W) { return ((W + 63) / 64) * ((H + 15) / 16); }

// Preconditioner request per instance (the ABI's EP_TV_PRECOND_* values).
enum { PRECOND_REQ_AUTO = 0, PRECOND_REQ_JACOBI = 1, PRECOND_REQ_CIRCULANT = 2 };

struct LikInstInfo {
  int op = 0, H = 0, W = 0, pitch = 0;
  long long off = 0;
  double xi = 1.0, damping = 1.0;
  double cg_tol = kCgTol;
  double cg_reduce = 0.0;
  int cg_max_iters = kCgMaxIters;
  int precond_req = PRECOND_REQ_AUTO;
  int rbmc_ns = 0;           // RBMC samples of the variance estimator (0: spectral)
  const float* sense = nullptr;   // Gaussian CS: host M x N sensing matrix
  int sense_rows = 0;
  const float* taps = nullptr;
  int th = 0, tw = 0;
  const uint8_t* mask = nullptr;
  int tile0 = 0, ntiles = 0;
};

// Device description of one instance with a non-identity operator.
// stages of the per-instance finishing kernel (index into LikInst::fin_count)
enum { FIN_PREP = 0, FIN_SPEC, FIN_INIT, FIN_ALPHA, FIN_BETA, FIN_SAMPLE, FIN_COUNT };

struct LikInst {
  int H, W, pitch, op;
  long long off;             // element offset in the pixel planes
  int inst;                  // index into InstDev / InstState
  int tile0, ntiles, tiles_x;
  int sep, Rr, Rc, kh, kw;   // separable taps?, combined-kernel radii, tap sizes
  int k_off, gr_off, gc_off; // offsets into the taps buffer
  float inv_xi, alpha, diagA, pad;   // diagA = sum of squared taps / xi (diagonal of H^T H / xi)
  double cg_tol2;            // squared relative residual tolerance
  double cg_reduce2;         // squared residual reduction at which a solve may stop (0: off)
  int cg_max_iters;
  int precond;               // PRECOND_JACOBI or PRECOND_CIRCULANT
  int npart;                 // partial-sum slots of the real-transform passes (fast CG)
  int fin_count[FIN_COUNT];  // partial sums each finalisation stage reduces (set on the host)
  int rbmc_ns;               // RBMC samples (0: spectral variance estimator)
  float inv_sqrt_xi;
};

enum {
  LP_HTY = 0, LP_TAUC, LP_ETAC, LP_B, LP_X, LP_R, LP_Z, LP_P0, LP_P1, LP_Q, LP_SPEC, LP_XPREV,
  LP_ACC, LP_ESAVE,            // RBMC: sum of squared off-diagonal terms, the mean solve's E
  LP_VAR,                      // Gaussian CS: the Woodbury variances
  LP_COUNT
};

enum { PRECOND_JACOBI = 0, PRECOND_CIRCULANT = 1 };

// The circulant preconditioner needs power-of-two FFT sizes; AUTO takes it
// whenever the sizes allow.
inline int lik_precond(int op, int H, int W, int req) {
  if (req == PRECOND_REQ_JACOBI) return PRECOND_JACOBI;
  return (fft_size_ok(H) && fft_size_ok(W)) ? PRECOND_CIRCULANT : PRECOND_JACOBI;
}

// FFT plans: the masked-DFT operator, and the circulant preconditioner.
inline bool lik_uses_fft(int op, int H, int W, int req) {
  return op == OP_DFT || (op == OP_BLUR && lik_precond(op, H, W, req) == PRECOND_CIRCULANT);
}

struct LikLayout {
  size_t planes[LP_COUNT]{};
  int nplanes = 0;
  // RBMC planes, rbmc_ns_max of each: H^T e1 of every sample (unscaled), the
  // pixel-space noise e2, and the sample's last solution (the next CG start)
  int rbmc_ns_max = 0;
  size_t rbmc_g = 0, rbmc_e2 = 0, rbmc_x = 0;
  size_t inst = 0, tiles = 0, part0 = 0, part1 = 0, part_mu = 0, taps = 0, fft = 0;
  int nlik = 0, ntiles = 0, ntaps = 0;
  size_t fft_bytes = 0;
  size_t wht = 0, wht_bytes = 0;
  size_t gauss = 0, gauss_bytes = 0;
};

// Bytes of the dense buffers of a Gaussian-CS instance (M sensing rows, N
// pixels), each rounded up to 256 bytes: H and H^T (float), S and Z^T (double),
// the vectors d, 1/d, b (N), t (M), the partial sums of t, the inverses of the
// diagonal Cholesky blocks and the observation.
constexpr int kGaussChunk = 256;   // rows per partial sum of t = Z (b / d)
// Leading dimension of S and Z^T: M rounded up to an even number, so that every
// row starts on a 16-byte boundary (the GEMM then reads rows as 16-byte words).
inline int gauss_ld(int M) { return (M + 1) / 2 * 2; }

inline size_t gauss_bytes_of(int M, int N) {
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t m = (size_t)M, nn = (size_t)N, nchunk = (nn + kGaussChunk - 1) / kGaussChunk;
  const size_t ld = (size_t)gauss_ld(M);
  return 2 * r(m * nn * 4) + r(m * ld * 8) + r(nn * ld * 8) + 3 * r(nn * 8) + r(m * 8) +
         r(nchunk * m * 8) + r((m + 63) / 64 * 64 * 64 * 8) + r(m * 4);
}

// Number of likelihood tiles and taps floats for the layout.
inline void lik_counts(const LikInstInfo* li, int n, int& nlik, int& ntiles, int& ntaps,
                       long long& fft_elems) {
  nlik = 0; ntiles = 0; ntaps = 0; fft_elems = 0;
  for (int i = 0; i < n; ++i) {
    if (li[i].op == OP_IDENTITY) continue;
    ++nlik;
    ntiles += ((li[i].W + kLikTW - 1) / kLikTW) * ((li[i].H + kLikTH - 1) / kLikTH);
    if (li[i].op == OP_BLUR) ntaps += li[i].th * li[i].tw + 2 * li[i].th + 2 * li[i].tw;
    if (li[i].op == OP_DFT || li[i].op == OP_HAD) fft_elems = std::max<long long>(fft_elems, (long long)li[i].H * li[i].W);
  }
}

template <class Take>
void lik_layout(const LikInstInfo* li, int n, long long plane, Take&& take, LikLayout& L) {
  long long fft_elems = 0;
  lik_counts(li, n, L.nlik, L.ntiles, L.ntaps, fft_elems);
  L.rbmc_ns_max = 0;
  bool any_gauss = false;
  for (int i = 0; i < n; ++i) {
    if (li[i].op != OP_IDENTITY) L.rbmc_ns_max = std::max(L.rbmc_ns_max, li[i].rbmc_ns);
    any_gauss = any_gauss || li[i].op == OP_GAUSS;
  }
  L.nplanes = L.nlik ? ((L.rbmc_ns_max || any_gauss) ? LP_COUNT : LP_ACC) : 0;
  for (int k = 0; k < L.nplanes; ++k) L.planes[k] = take(sizeof(float) * (size_t)plane);
  if (L.rbmc_ns_max) {
    L.rbmc_g = take(sizeof(float) * (size_t)plane * L.rbmc_ns_max);
    L.rbmc_e2 = take(sizeof(float) * (size_t)plane * L.rbmc_ns_max);
    L.rbmc_x = take(sizeof(float) * (size_t)plane * L.rbmc_ns_max);
  }
  L.inst = take(sizeof(LikInst) * (size_t)std::max(L.nlik, 1));
  L.tiles = take(sizeof(int4) * (size_t)std::max(L.ntiles, 1));
  L.part0 = take(sizeof(double) * (size_t)std::max(L.ntiles, 1));
  L.part1 = take(sizeof(double) * (size_t)std::max(L.ntiles, 1));
  L.part_mu = take(sizeof(float) * (size_t)std::max(L.ntiles, 1));
  L.taps = take(sizeof(float) * (size_t)std::max(L.ntaps, 1));
  // FFT work buffers, per DFT instance: two complex planes, twiddles, the
  // transposed spectrum and the mask (each rounded up to 256 bytes)
  L.fft_bytes = 0;
  for (int i = 0; i < n; ++i) {
    if (li[i].op == OP_IDENTITY || !lik_uses_fft(li[i].op, li[i].H, li[i].W, li[i].precond_req)) continue;
    const size_t N = (size_t)li[i].H * li[i].W;
    auto r256 = [](size_t b) { return (b + 255) / 256 * 256; };
    L.fft_bytes += 2 * r256(N * 8) + r256((size_t)li[i].W * 8) + r256((size_t)li[i].H * 8) +
                   r256(N * 4) + r256(N);
  }
  (void)fft_elems;
  L.fft = take(std::max<size_t>(L.fft_bytes, 256));
  // Walsh-Hadamard instances: a work vector and the reordered mask, N floats each
  L.wht_bytes = 0;
  for (int i = 0; i < n; ++i) {
    if (li[i].op != OP_HAD) continue;
    const size_t N = (size_t)li[i].H * li[i].W;
    L.wht_bytes += 2 * ((N * sizeof(float) + 255) / 256 * 256);
  }
  L.wht = take(std::max<size_t>(L.wht_bytes, 256));
  // Gaussian-CS instances: H, H^T, S, Z^T and the vectors of the Woodbury moments
  L.gauss_bytes = 0;
  for (int i = 0; i < n; ++i)
    if (li[i].op == OP_GAUSS) L.gauss_bytes += gauss_bytes_of(li[i].sense_rows, li[i].H * li[i].W);
  L.gauss = take(std::max<size_t>(L.gauss_bytes, 256));
}

// FFT work buffers of one instance that uses the FFT (masked DFT operator,
// and the circulant preconditioner), all in the workspace.
struct DftPlan {
  int li = 0;                // index into LikCtx::hinst
  int H = 0, W = 0, logH = 0, logW = 0;
  float2* A = nullptr;       // H x W complex
  float2* B = nullptr;       // W x H complex (transposed layout)
  float2* twW = nullptr;     // W twiddles e^{-2 pi i t / W}
  float2* twH = nullptr;     // H twiddles
  float* specT = nullptr;    // W x H eigenvalues of H^T H (transposed layout)
  uint8_t* mask = nullptr;   // H x W
};

// Walsh-Hadamard work buffers of one instance with that operator.
struct WhtPlan {
  int li = 0;                // index into LikCtx::hinst
  int logH = 0, logW = 0, logN = 0, lb = 0;   // lb: bits of the LDS group
  float* work = nullptr;     // N floats, natural order
  float* eig = nullptr;      // N floats: the mask in natural order
};

// Device buffers of one Gaussian-CS instance (all in the workspace).
struct GaussPlan {
  int li = 0;                  // index into LikCtx::hinst
  int M = 0, N = 0;            // sensing rows, pixels
  float* Hm = nullptr;         // M x N, row-major (as given)
  float* HT = nullptr;         // N x M, its transpose
  int ld = 0;                  // leading dimension of S and ZT (gauss_ld)
  double* S = nullptr;         // M x M (lower triangle used), then its Cholesky factor
  double* ZT = nullptr;        // N x M
  double* d = nullptr;         // N: cavity precisions (flat, row-major pixels)
  double* w = nullptr;         // N: 1 / d
  double* b = nullptr;         // N: right-hand side
  double* t = nullptr;         // M
  double* tpart = nullptr;     // nchunk x M partial sums of t
  double* Linv = nullptr;      // ceil(M / 64) blocks of 64 x 64: inverses of the diagonal Cholesky blocks
  float* y = nullptr;          // M: the observation
  int nchunk = 0;
};

struct LikCtx {
  int nlik = 0, ntiles = 0;
  std::vector<DftPlan> dft;
  std::vector<WhtPlan> wht;
  std::vector<GaussPlan> gauss;
  char* gaussbuf = nullptr;
  double dgemm_flops = 0.0;          // flops of the FP64 GEMMs launched while timing
  float* whtbuf = nullptr;
  std::vector<LikInst> hinst;
  std::vector<int> inst_of;          // lik index -> instance index
  LikInst* d_inst = nullptr;
  int4* d_tiles = nullptr;
  double* part0 = nullptr;
  double* part1 = nullptr;
  float* part_mu = nullptr;          // per tile: max |mu| after the likelihood-site update
  float* taps = nullptr;
  float* planes[LP_COUNT]{};
  float2* fft = nullptr;
  InstState* d_st = nullptr;
  const InstDev* d_idev = nullptr;
  float* ypix = nullptr;
  long long plane = 0;               // elements per plane
  int rbmc_ns_max = 0;               // RBMC: largest sample count of any instance (0: none)
  float* rbmc_g = nullptr;           // rbmc_ns_max planes each
  float* rbmc_e2 = nullptr;
  float* rbmc_x = nullptr;
  int pcur = 0;                      // which p plane holds the current search direction
  int sample = 0;                    // RBMC sample whose planes the kernels address
  bool fast = false;                 // every instance circulant: CG products and preconditioner by real FFTs
  bool all_jacobi = false;           // every instance Jacobi: CG step and preconditioner in one pass
  int max_iters = kCgMaxIters;       // largest per-instance CG cap
  InstState* hst = nullptr;          // pinned host staging for CG polls (allocated on first poll)
  long long* poll_word = nullptr;    // pinned host word of graph-replay polls (host address)
  long long* poll_word_dev = nullptr;  // the same word as the device addresses it
  int n_all = 0;
  // kernel timing (event pairs per bucket, KT_*)
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  std::vector<std::pair<int, int>> ev_k[9];
};

// Timing buckets of the likelihood-site update.  KT_APPLY and KT_PRECOND each
// bracket a group of launches (the product with A inside CG; the fast CG's
// whole preconditioner with its x, r update); the others bracket single
// launches: the three real-transform passes, the per-instance finishing
// kernels, and everything else (cavity / right-hand side, spectral sum, CG
// start, Jacobi kernels, site update); KT_DGEMM brackets every FP64 GEMM of the
// Gaussian-CS Woodbury moments.
enum { KT_APPLY = 0, KT_PRECOND, KT_RF_FWD, KT_RF_FILT, KT_RF_INV, KT_FIN, KT_OTHER, KT_DGEMM,
       KT_COUNT };
static_assert(KT_COUNT <= 9, "timing buckets");
constexpr size_t kMaxTimingEvents = 1u << 17;

// Run `body` between two timing events (when timing is on), recording the pair
// in bucket `kt`.
template <class F>
hipError_t lik_timed(LikCtx& lc, int kt, hipStream_t s, F&& body) {
  const bool tm = lc.timing && lc.ev_used + 2 <= kMaxTimingEvents;
  int i0 = 0, i1 = 0;
  if (tm) {
    while (lc.ev_used + 2 > lc.ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
      lc.ev.push_back(e);
    }
    i0 = (int)lc.ev_used++;
    i1 = (int)lc.ev_used++;
    const hipError_t e0 = hipEventRecord(lc.ev[i0], s);
    if (e0 != hipSuccess) return e0;
  }
  hipError_t e = body();
  if (e != hipSuccess) return e;
  if (tm) {
    const hipError_t e1 = hipEventRecord(lc.ev[i1], s);
    if (e1 != hipSuccess) return e1;
    lc.ev_k[kt].emplace_back(i0, i1);
  }
  return hipGetLastError();
}

hipError_t lik_create(LikCtx& lc, const LikInstInfo* li, int n, char* ws, const LikLayout& L,
                      long long plane, InstDev* d_inst, InstState* d_st, int4* d_tiles, int ntiles,
                      float* ypix, hipStream_t s, std::string& err);
hipError_t lik_set_observation(LikCtx& lc, const float* const* d_y, hipStream_t s);
hipError_t lik_reset(LikCtx& lc, hipStream_t s);
hipError_t lik_resume(LikCtx& lc, hipStream_t s);
hipError_t lik_update(LikCtx& lc, float2* const S[5], hipStream_t s);
// The pieces of lik_update, for graph capture: head (cavity, rhs, spectral
// precision, CG start), n CG iterations (no host synchronisation; converged
// instances are skipped on the device), a host poll of the CG flags, and the
// site update.  n must be even for a captured sequence to be replayable.
hipError_t lik_head(LikCtx& lc, float2* const S[5], hipStream_t s);
hipError_t lik_iterations(LikCtx& lc, int n, hipStream_t s);
hipError_t lik_poll(LikCtx& lc, hipStream_t s, bool& all_done);
// The poll of graph replays: lik_poll_word_launch queues (for capture at the end
// of a run of CG iterations) a kernel that writes {sequence number + 1, all
// solves stopped, largest iteration count of the current solves} to a pinned
// host word; the host reads the sequence number before launching such a replay
// (lik_poll_word_seq) and waits for it to change (lik_poll_word_wait, which
// spins on the word and falls back to the stream's completion if the stream
// drains without a new word).
hipError_t lik_poll_word_alloc(LikCtx& lc);   // before capture: no allocation while capturing
hipError_t lik_poll_word_launch(LikCtx& lc, hipStream_t s);
unsigned lik_poll_word_seq(const LikCtx& lc);
hipError_t lik_poll_word_wait(LikCtx& lc, hipStream_t s, unsigned seq0, bool& all_done,
                              int& max_iters);
hipError_t lik_tail(LikCtx& lc, float2* S0, hipStream_t s);
// RBMC: the white noise of every RBMC instance (host array of device pointers,
// one per instance of the context; NULL for instances without RBMC): H^T e1 and
// e2 of every sample into the workspace.  The sample solutions restart from 0.
hipError_t lik_set_rbmc_noise(LikCtx& lc, const float* const* d_noise, hipStream_t s);
void lik_destroy(LikCtx& lc);
void lik_timing(LikCtx& lc, bool enable, bool clear);
// Total milliseconds and launch counts per bucket (arrays of KT_COUNT).
hipError_t lik_timing_read(LikCtx& lc, double* ms, int* launches);

}  // namespace eptv
