// Host side of the C ABI declared in include/ep_tv.h: argument validation,
// workspace layout, the tile list, and the per-sweep launch schedule.
#include "ep_tv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ep_tv_internal.h"
#include "lik.h"

using namespace eptv;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct InstHost {
  ep_tv_problem p{};
  std::vector<float> taps;
  std::vector<uint8_t> mask;
  int pitch = 0;
  long long off = 0;
  int strips = 0, chunks = 0, chunk_rows = 0, tile0 = 0, ntiles = 0;
};

struct Layout {
  long long plane = 0;       // elements per plane (all instances)
  int ntiles = 0;            // tiles at the initial tile height
  int tile_cap = 0;          // tiles at the smallest tile height (sizes the tile arrays)
  size_t S0 = 0, SB[2][4]{}, ypix = 0, wpix = 0, inst = 0, st = 0, tiles = 0;
  size_t part_e = 0, part_m = 0, part_v = 0, part_c = 0, part_f = 0, tab0 = 0, tab1 = 0;
  LikLayout lik;
  size_t total = 0;
};

// Tile heights (rows per sweep tile) the autotuner tries; all even, since the
// sweep marches row pairs.
constexpr int kTuneRows[] = {8, 10, 12, 14, 16, 18, 20, 24, 28, 32, 40, 48, 64, 96, 128};
constexpr int kNumTuneRows = 15;
constexpr int kMinChunkRows = 8;

int env_chunk_rows() {
  if (const char* e = std::getenv("EPTV_CHUNK_ROWS")) {
    int v = std::atoi(e);
    if (v >= 2 && v <= 4096 && v % 2 == 0) return v;
  }
  return 0;
}

// Default tile height for a batch: the tallest of 32/16/8 rows that still gives
// >= 8192 tiles (32 waves per CU) over the whole batch.
int default_chunk_rows(const std::vector<ep_tv_problem>& ps) {
  if (int v = env_chunk_rows()) return v;
  int ch = 32;
  while (ch > kMinChunkRows) {
    long long tiles = 0;
    for (const auto& p : ps)
      tiles += (long long)((p.width + kStripInt - 1) / kStripInt) * ((p.height + ch - 1) / ch);
    if (tiles >= 8192) break;
    ch /= 2;
  }
  return ch;
}

int count_tiles(const std::vector<InstHost>& ih, int rows) {
  long long t = 0;
  for (const auto& h : ih)
    t += (long long)((h.p.width + kStripInt - 1) / kStripInt) * ((h.p.height + rows - 1) / rows);
  return (int)std::min<long long>(t, 1LL << 30);
}

// Assign tile ranges for tile height `rows` (same height for every instance).
void assign_tiles(std::vector<InstHost>& ih, int rows) {
  int tiles = 0;
  for (auto& h : ih) {
    h.chunk_rows = rows;
    h.strips = (h.p.width + kStripInt - 1) / kStripInt;
    h.chunks = (h.p.height + rows - 1) / rows;
    h.tile0 = tiles;
    h.ntiles = h.strips * h.chunks;
    tiles += h.ntiles;
  }
}

const char* validate(const ep_tv_problem& p) {
  if (p.height < 1 || p.width < 1 || p.height > 16384 || p.width > 16384)
    return "height and width must be in [1, 16384]";
  if (p.op < EP_TV_OP_IDENTITY || p.op > EP_TV_OP_GAUSS_CS) return "unknown operator";
  if (p.op == EP_TV_OP_GAUSS_CS) {
    if (!p.sense_matrix) return "the Gaussian CS operator needs sense_matrix";
    if (p.sense_rows < 1 || p.sense_rows > 32768) return "sense_rows must be in [1, 32768]";
    if ((long long)p.height * p.width > 65536) return "the Gaussian CS operator needs at most 65536 pixels";
    if (p.var_estimator != EP_TV_VAR_SPECTRAL)
      return "the Gaussian CS operator computes its variances exactly (Woodbury)";
  }
  if (p.boundary != EP_TV_BND_FREE && p.boundary != EP_TV_BND_PERIODIC) return "unknown boundary";
  if (p.boundary == EP_TV_BND_PERIODIC && (p.height % 2 || p.width % 2 || p.height < 2 || p.width < 2))
    return "periodic boundary needs even height and width";
  if (!(p.noise_var > 0.0) || !std::isfinite(p.noise_var)) return "noise_var must be > 0";
  if (!(p.lambda0 > 0.0) || !std::isfinite(p.lambda0)) return "lambda0 must be > 0";
  if (!(p.damping > 0.0 && p.damping <= 1.0)) return "damping must be in (0, 1]";
  if (!(p.cg_tol >= 0.0 && p.cg_tol < 1.0)) return "cg_tol must be in [0, 1)";
  if (!(p.cg_reduce >= 0.0 && p.cg_reduce < 1.0)) return "cg_reduce must be in [0, 1)";
  if (p.prior < EP_TV_PRIOR_L1 || p.prior > EP_TV_PRIOR_BG) return "prior must be one of EP_TV_PRIOR_*";
  if (p.prior != EP_TV_PRIOR_L1) {
    if (!(p.prior_omega > 0.0 && p.prior_omega <= 1.0)) return "prior_omega must be in (0, 1]";
    if (!(p.prior_s1sq > 0.0) || !std::isfinite(p.prior_s1sq)) return "prior_s1sq must be > 0";
    if (p.prior == EP_TV_PRIOR_MOG2 && (!(p.prior_s2sq > 0.0) || !std::isfinite(p.prior_s2sq)))
      return "prior_s2sq must be > 0";
  }
  if (p.cg_max_iters < 0 || p.cg_max_iters > 100000) return "cg_max_iters must be in [0, 100000]";
  if (p.var_estimator != EP_TV_VAR_SPECTRAL && p.var_estimator != EP_TV_VAR_RBMC)
    return "var_estimator must be one of EP_TV_VAR_*";
  if (p.var_estimator == EP_TV_VAR_RBMC && (p.rbmc_samples < 1 || p.rbmc_samples > 64))
    return "rbmc_samples must be in [1, 64]";
  if (p.noise_map != 0 && p.noise_map != 1) return "noise_map must be 0 or 1";
  if (p.noise_map && p.op != EP_TV_OP_IDENTITY)
    return "per-pixel noise variances are supported for the identity operator";
  if (p.cg_precond < EP_TV_PRECOND_AUTO || p.cg_precond > EP_TV_PRECOND_CIRCULANT)
    return "cg_precond must be one of EP_TV_PRECOND_*";
  if (p.cg_precond == EP_TV_PRECOND_CIRCULANT && p.op != EP_TV_OP_IDENTITY &&
      !(fft_size_ok(p.height) && fft_size_ok(p.width)))
    return "the circulant preconditioner needs power-of-two sizes in [4, 4096]";
  if (p.op == EP_TV_OP_BLUR_PERIODIC) {
    if (!p.blur_taps) return "blur operator needs blur_taps";
    if (p.blur_h < 1 || p.blur_w < 1 || p.blur_h % 2 == 0 || p.blur_w % 2 == 0 ||
        p.blur_h > kMaxTaps || p.blur_w > kMaxTaps)
      return "blur taps must have odd sizes <= 17";
    if (p.blur_h > p.height || p.blur_w > p.width) return "blur kernel larger than the image";
  }
  if (p.op == EP_TV_OP_DFT_MASK) {
    if (!p.dft_mask) return "DFT operator needs dft_mask";
    if (!fft_size_ok(p.height) || !fft_size_ok(p.width))
      return "DFT operator needs power-of-two sizes in [4, 4096]";
  }
  if (p.op == EP_TV_OP_HADAMARD_MASK) {
    if (!p.dft_mask) return "Walsh-Hadamard operator needs dft_mask";
    if (!fft_size_ok(p.height) || !fft_size_ok(p.width))
      return "Walsh-Hadamard operator needs power-of-two sizes in [4, 4096]";
  }
  if (p.reserved != 0) return "reserved must be 0";
  return nullptr;
}

// RBMC samples of an instance (0: the spectral estimator, or H = I).
int rbmc_ns(const ep_tv_problem& p) {
  return (p.op != EP_TV_OP_IDENTITY && p.var_estimator == EP_TV_VAR_RBMC) ? p.rbmc_samples : 0;
}

void make_layout(std::vector<InstHost>& ih, int rows, Layout& L) {
  long long off = 0;
  for (auto& h : ih) {
    const int H = h.p.height, W = h.p.width;
    h.pitch = (int)align_up((size_t)W + 1, 64);   // +1: a lane's pixel pair never leaves the row
    h.off = off;
    off += (long long)h.pitch * H;
    off = (long long)align_up((size_t)off, 64);
  }
  assign_tiles(ih, rows);
  L.plane = std::max<long long>(off, 64);
  L.ntiles = count_tiles(ih, rows);
  L.tile_cap = std::max(L.ntiles, count_tiles(ih, std::min(rows, kMinChunkRows)));
  const int tiles = L.tile_cap;
  const int n = (int)ih.size();
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t at = cur;
    cur = align_up(cur + bytes, kAlign);
    return at;
  };
  L.S0 = take(sizeof(float2) * (size_t)L.plane);
  for (int b = 0; b < 2; ++b)
    for (int k = 0; k < 4; ++k) L.SB[b][k] = take(sizeof(float2) * (size_t)L.plane);
  L.ypix = take(sizeof(float) * (size_t)L.plane);
  bool any_map = false;
  for (const auto& h : ih) any_map = any_map || h.p.noise_map;
  L.wpix = any_map ? take(sizeof(float) * (size_t)L.plane) : 0;
  L.inst = take(sizeof(InstDev) * n);
  L.st = take(sizeof(InstState) * n);
  L.tiles = take(sizeof(int4) * (size_t)std::max(tiles, 1));
  L.part_e = take(sizeof(double) * (size_t)std::max(tiles, 1));
  L.part_m = take(sizeof(float) * (size_t)std::max(tiles, 1));
  L.part_v = take(sizeof(float) * (size_t)std::max(tiles, 1));
  L.part_c = take(sizeof(unsigned) * (size_t)std::max(tiles, 1));
  L.part_f = take(sizeof(unsigned) * (size_t)std::max(tiles, 1));
  L.tab0 = take(sizeof(float*) * n);
  L.tab1 = take(sizeof(float*) * n);
  std::vector<LikInstInfo> li(n);
  for (int i = 0; i < n; ++i) {
    li[i].op = ih[i].p.op;
    li[i].H = ih[i].p.height;
    li[i].W = ih[i].p.width;
    li[i].th = ih[i].p.op == EP_TV_OP_BLUR_PERIODIC ? ih[i].p.blur_h : 0;
    li[i].tw = ih[i].p.op == EP_TV_OP_BLUR_PERIODIC ? ih[i].p.blur_w : 0;
    li[i].precond_req = ih[i].p.cg_precond;
    li[i].rbmc_ns = rbmc_ns(ih[i].p);
    li[i].sense_rows = ih[i].p.op == EP_TV_OP_GAUSS_CS ? ih[i].p.sense_rows : 0;
  }
  lik_layout(li.data(), n, L.plane, take, L.lik);
  L.total = cur;
}

}  // namespace

// Captured launch sequences (hipGraph) of one sweep, replayed on the caller's
// stream.  The TV-site buffers alternate between sweeps, so the pieces that
// read or write them exist once per buffer parity.
struct Graphs {
  bool valid = false;
  int em = -1;
  bool delta = false;
  double tol = 0.0;
  hipGraphExec_t head[2]{};    // likelihood head + kCgPoll CG iterations
  hipGraphExec_t head_short[2]{};  // likelihood head + kCgHeadShort CG iterations
  hipGraphExec_t cg = nullptr; // kCgPoll CG iterations
  hipGraphExec_t cg8 = nullptr, cg16 = nullptr;  // 2 and 4 times as many
  hipGraphExec_t tail[2]{};    // likelihood site + TV sweep + finalize (one sweep)
  hipGraphExec_t multi[2]{};   // kGraphSweeps whole sweeps (identity operators only)
};

constexpr int kGraphSweeps = 8;   // even: a multi-sweep graph ends on the parity it starts on

struct ep_tv_ctx {
  int n = 0;
  std::vector<InstDev> idev_host;
  std::vector<int4> tiles_host;
  std::vector<InstHost> ih;
  Layout L;
  int ntiles = 0;            // current sweep tile count
  int chunk_rows = 0;        // current sweep tile height
  bool use_graph = false;
  Graphs g;
  int cg_iters_prev = 1 << 30;   // largest CG iteration count of the last graph-replayed sweep
  hipStream_t cap = nullptr; // private stream used only to capture graphs
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  float2* S0 = nullptr;
  float2* SB[2][4]{};
  int cur = 0;   // which TV-site buffer holds the current state
  float* ypix = nullptr;
  float* wpix = nullptr;             // per-pixel noise precisions (noise_map instances)
  bool any_noise_map = false;
  bool noise_set = false;
  InstDev* d_inst = nullptr;
  InstState* d_st = nullptr;
  int4* d_tiles = nullptr;
  SweepArgs sa{};
  float** d_tab0 = nullptr;
  float** d_tab1 = nullptr;
  LikCtx lik;
  bool has_obs = false;
  bool any_lik = false;
  bool warm_started = false;         // init_warm / set_sites since the last cold start
  bool rbmc_noise_set = false;       // RBMC contexts: white noise uploaded
  std::vector<InstState> host_st;
  InstState* pull_st = nullptr;      // pinned host staging for state pulls (allocated on first pull)
  std::vector<float*> tab_host0, tab_host1;
  double last_elapsed_ms = 0.0;
  std::string err;
  // measurement: event pairs around sweep launches and likelihood updates
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_sweep, ev_lik;   // indices into ev_pool
  size_t ev_used = 0;
};

struct CurSites {
  float2* S[5];
};

static CurSites cur_sites(const ep_tv_ctx* c) {
  CurSites r;
  r.S[0] = c->S0;
  for (int k = 0; k < 4; ++k) r.S[k + 1] = c->SB[c->cur][k];
  return r;
}

static hipEvent_t next_event(ep_tv_ctx* c, int& idx) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  idx = (int)c->ev_used;
  return c->ev_pool[c->ev_used++];
}

static void timing_clear(ep_tv_ctx* c) {
  c->ev_sweep.clear();
  c->ev_lik.clear();
  c->ev_used = 0;
}

static int fail(ep_tv_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

static int hip_check(ep_tv_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return EP_TV_OK;
  return fail(c, EP_TV_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                              \
  do {                                               \
    int _rc = hip_check((c), (expr), #expr);         \
    if (_rc != EP_TV_OK) return _rc;                 \
  } while (0)

// ---- tile-height choice shared by every context with the same instance sizes
// (filled by ep_tv_autotune, read by ep_tv_workspace_bytes / ep_tv_create)
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune_rows;

static std::string shape_key(const ep_tv_problem* p, int n) {
  std::vector<std::pair<int, int>> v(n);
  for (int i = 0; i < n; ++i) v[i] = {p[i].height, p[i].width};
  std::sort(v.begin(), v.end());
  std::string k;
  for (auto& hw : v) k += std::to_string(hw.first) + "x" + std::to_string(hw.second) + ";";
  return k;
}

static int initial_rows(const ep_tv_problem* p, int n) {
  if (int v = env_chunk_rows()) return v;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_rows.find(shape_key(p, n));
    if (it != g_tune_rows.end()) return it->second;
  }
  return default_chunk_rows(std::vector<ep_tv_problem>(p, p + n));
}

// Per-instance device descriptors and the sweep tile list for the current
// tile height.  Asynchronous uploads from host vectors that live in the ctx.
static int upload_tiles(ep_tv_ctx* c) {
  const int n = c->n;
  c->idev_host.assign(n, InstDev{});
  c->tiles_host.clear();
  int lik_tiles = 0;   // likelihood tiles are numbered in instance order, as lik_create does
  for (int i = 0; i < n; ++i) {
    const InstHost& h = c->ih[i];
    InstDev& d = c->idev_host[i];
    std::memset(&d, 0, sizeof(d));
    d.H = h.p.height; d.W = h.p.width; d.pitch = h.pitch; d.bnd = h.p.boundary;
    d.off = h.off; d.op = h.p.op; d.strips = h.strips; d.chunks = h.chunks; d.tile0 = h.tile0;
    d.ntiles = h.ntiles; d.chunk_rows = h.chunk_rows; d.npix = h.p.height * h.p.width;
    d.wmap = h.p.noise_map ? 1 : 0;
    if (h.p.op != EP_TV_OP_IDENTITY) {
      d.lik_tile0 = lik_tiles;
      d.lik_ntiles = lik_tile_count(h.p.height, h.p.width);
      lik_tiles += d.lik_ntiles;
    }
    d.xi = (float)h.p.noise_var; d.inv_xi = (float)(1.0 / h.p.noise_var);
    d.alpha = (float)h.p.damping;
    if (h.p.prior != EP_TV_PRIOR_L1) {
      // phi = a1 N(0, v1) + a2 N(0, v2): MoG2 (omega, 1 - omega; s1^2, s2^2), BG (v2 = 0)
      const double a1 = h.p.prior_omega, a2 = 1.0 - h.p.prior_omega;
      const double v1 = h.p.prior_s1sq, v2 = h.p.prior == EP_TV_PRIOR_MOG2 ? h.p.prior_s2sq : 0.0;
      d.mix_dla = (float)(a2 > 0.0 ? std::log(a2 / a1) : -HUGE_VAL);
      d.mix_dv = (float)(v1 - v2);
      d.mix_v1 = (float)v1;
      d.mix_v2 = (float)v2;
    }
    for (int st = 0; st < h.strips; ++st)
      for (int ch = 0; ch < h.chunks; ++ch) c->tiles_host.push_back(make_int4(i, st, ch, 0));
  }
  if ((int)c->tiles_host.size() > c->L.tile_cap)
    return fail(c, EP_TV_E_ARG, "tile count exceeds the workspace's tile capacity");
  c->ntiles = (int)c->tiles_host.size();
  c->sa.ntiles = c->ntiles;
  HIPCHK(c, hipMemcpyAsync(c->d_inst, c->idev_host.data(), sizeof(InstDev) * n,
                           hipMemcpyHostToDevice, c->stream));
  if (!c->tiles_host.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_tiles, c->tiles_host.data(), sizeof(int4) * c->tiles_host.size(),
                             hipMemcpyHostToDevice, c->stream));
  return EP_TV_OK;
}

static void drop_graphs(ep_tv_ctx* c) {
  Graphs& g = c->g;
  hipGraphExec_t* all[] = {&g.head[0], &g.head[1], &g.head_short[0], &g.head_short[1], &g.cg,
                           &g.cg8, &g.cg16, &g.tail[0], &g.tail[1], &g.multi[0], &g.multi[1]};
  for (hipGraphExec_t* e : all)
    if (*e) {
      (void)hipGraphExecDestroy(*e);
      *e = nullptr;
    }
  g.valid = false;
}

static int set_rows(ep_tv_ctx* c, int rows) {
  assign_tiles(c->ih, rows);
  c->chunk_rows = rows;
  drop_graphs(c);
  return upload_tiles(c);
}

static int set_tab(ep_tv_ctx* c, float* const* host, float** dev, std::vector<float*>& keep);
static int pull_states(ep_tv_ctx* c);

extern "C" {

const char* ep_tv_version(void) { return "eptv-gfx950 0.2"; }

int ep_tv_workspace_bytes(const ep_tv_problem* p, int32_t n, size_t* bytes) {
  if (!p || !bytes || n < 1 || n > 4096) return EP_TV_E_ARG;
  std::vector<InstHost> ih(n);
  for (int i = 0; i < n; ++i) {
    if (validate(p[i])) return EP_TV_E_ARG;
    if (p[i].prior != p[0].prior) return EP_TV_E_ARG;   // as ep_tv_create
    ih[i].p = p[i];
  }
  Layout L;
  make_layout(ih, initial_rows(p, n), L);
  *bytes = L.total;
  return EP_TV_OK;
}

int ep_tv_create(const ep_tv_problem* p, int32_t n, void* d_ws, size_t ws_bytes, void* stream,
                 ep_tv_ctx** out) {
  if (!out) return EP_TV_E_ARG;
  *out = nullptr;
  if (!p || n < 1 || n > 4096 || !d_ws) return EP_TV_E_ARG;
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return EP_TV_E_ARG;
  ep_tv_ctx* c = new ep_tv_ctx();
  c->n = n;
  c->ih.resize(n);
  for (int i = 0; i < n; ++i) {
    if (const char* m = validate(p[i])) {
      delete c;
      return EP_TV_E_ARG;
    }
    c->ih[i].p = p[i];
    if (p[i].op == EP_TV_OP_BLUR_PERIODIC) {
      c->ih[i].taps.assign(p[i].blur_taps, p[i].blur_taps + (size_t)p[i].blur_h * p[i].blur_w);
      c->ih[i].p.blur_taps = nullptr;
    }
    if (p[i].op == EP_TV_OP_DFT_MASK || p[i].op == EP_TV_OP_HADAMARD_MASK) {
      c->ih[i].mask.assign(p[i].dft_mask, p[i].dft_mask + (size_t)p[i].height * p[i].width);
      c->ih[i].mask[0] = 1;   // DC always observed
      c->ih[i].p.dft_mask = nullptr;
    }
    if (p[i].op != EP_TV_OP_IDENTITY) c->any_lik = true;
    if (p[i].prior != p[0].prior) {   // the sweep is compiled per factor kind
      delete c;
      return EP_TV_E_ARG;
    }
  }
  c->sa.prior = p[0].prior;
  c->sa.em_opt = 3;
  make_layout(c->ih, initial_rows(p, n), c->L);
  c->chunk_rows = c->ih[0].chunk_rows;
  if (ws_bytes < c->L.total) {
    delete c;
    return EP_TV_E_OOM;
  }
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(d_ws);
  c->S0 = reinterpret_cast<float2*>(c->ws + c->L.S0);
  for (int b = 0; b < 2; ++b)
    for (int k = 0; k < 4; ++k) c->SB[b][k] = reinterpret_cast<float2*>(c->ws + c->L.SB[b][k]);
  c->ypix = reinterpret_cast<float*>(c->ws + c->L.ypix);
  for (int i = 0; i < n; ++i) c->any_noise_map = c->any_noise_map || p[i].noise_map;
  c->wpix = c->any_noise_map ? reinterpret_cast<float*>(c->ws + c->L.wpix) : nullptr;
  c->d_inst = reinterpret_cast<InstDev*>(c->ws + c->L.inst);
  c->d_st = reinterpret_cast<InstState*>(c->ws + c->L.st);
  c->d_tiles = reinterpret_cast<int4*>(c->ws + c->L.tiles);
  c->d_tab0 = reinterpret_cast<float**>(c->ws + c->L.tab0);
  c->d_tab1 = reinterpret_cast<float**>(c->ws + c->L.tab1);
  SweepArgs& a = c->sa;
  a.S0 = c->S0;
  a.inst = c->d_inst;
  a.st = c->d_st;
  a.tiles = c->d_tiles;
  a.part_eabs = reinterpret_cast<double*>(c->ws + c->L.part_e);
  a.part_dmu = reinterpret_cast<float*>(c->ws + c->L.part_m);
  a.part_dv = reinterpret_cast<float*>(c->ws + c->L.part_v);
  a.part_clamp = reinterpret_cast<unsigned*>(c->ws + c->L.part_c);
  a.part_flags = reinterpret_cast<unsigned*>(c->ws + c->L.part_f);
  int rc = upload_tiles(c);
  if (rc == EP_TV_OK) {
    std::vector<LikInstInfo> li(n);
    for (int i = 0; i < n; ++i) {
      li[i].op = c->ih[i].p.op;
      li[i].H = c->ih[i].p.height;
      li[i].W = c->ih[i].p.width;
      li[i].pitch = c->ih[i].pitch;
      li[i].off = c->ih[i].off;
      li[i].xi = c->ih[i].p.noise_var;
      li[i].damping = c->ih[i].p.damping;
      li[i].cg_tol = c->ih[i].p.cg_tol > 0.0 ? c->ih[i].p.cg_tol : kCgTol;
      li[i].cg_max_iters = c->ih[i].p.cg_max_iters > 0 ? c->ih[i].p.cg_max_iters : kCgMaxIters;
      li[i].cg_reduce = c->ih[i].p.cg_reduce;
      li[i].precond_req = c->ih[i].p.cg_precond;
      li[i].taps = c->ih[i].taps.empty() ? nullptr : c->ih[i].taps.data();
      li[i].th = c->ih[i].p.blur_h;
      li[i].tw = c->ih[i].p.blur_w;
      li[i].mask = c->ih[i].mask.empty() ? nullptr : c->ih[i].mask.data();
      li[i].rbmc_ns = rbmc_ns(c->ih[i].p);
      li[i].sense = c->ih[i].p.sense_matrix;
      li[i].sense_rows = c->ih[i].p.sense_rows;
      li[i].tile0 = c->ih[i].tile0;
      li[i].ntiles = c->ih[i].ntiles;
    }
    std::string e;
    if (lik_create(c->lik, li.data(), n, c->ws, c->L.lik, c->L.plane, c->d_inst, c->d_st,
                   c->d_tiles, c->ntiles, c->ypix, c->stream, e) != hipSuccess)
      rc = fail(c, EP_TV_E_HIP, "likelihood-site setup: " + e);
    // the finalisation reads it only for instances with likelihood tiles
    a.part_mu = c->lik.part_mu ? c->lik.part_mu : a.part_dmu;
  }
  if (rc == EP_TV_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "create sync");
  if (rc != EP_TV_OK) {
    delete c;
    return rc;
  }
  c->host_st.resize(n);
  *out = c;
  return EP_TV_OK;
}

static int reset_states(ep_tv_ctx* c) {
  for (int i = 0; i < c->n; ++i) {
    InstState& s = c->host_st[i];
    std::memset(&s, 0, sizeof(s));
    s.lam = s.lam_prev = c->ih[i].p.lambda0;
    s.active = 1u;
  }
  HIPCHK(c, hipMemcpyAsync(c->d_st, c->host_st.data(), sizeof(InstState) * c->n,
                           hipMemcpyHostToDevice, c->stream));
  return EP_TV_OK;
}

int ep_tv_init_cold(ep_tv_ctx* c) {
  if (!c) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  if (c->any_noise_map && !c->noise_set)
    return fail(c, EP_TV_E_STATE, "per-pixel noise variances not set (ep_tv_set_noise_variance)");
  int rc = reset_states(c);
  if (rc) return rc;
  // the sweep's per-tile partial arrays serve as the range partials (no sweep runs meanwhile)
  HIPCHK(c, launch_yrange(c->ypix, c->d_inst, c->d_st, c->n, c->d_tiles, c->ntiles,
                          c->sa.part_dmu, c->sa.part_dv, c->stream));
  c->cur = 0;
  c->warm_started = false;
  HIPCHK(c, launch_init_cold(cur_sites(c).S, c->ypix, c->d_inst, c->d_st, c->d_tiles, c->ntiles,
                             c->stream, false, c->wpix));
  HIPCHK(c, lik_reset(c->lik, c->stream));
  return EP_TV_OK;
}

int ep_tv_init_warm(ep_tv_ctx* c, const float* const* d_mu_hat, const float* const* d_var_hat,
                    double lambda_scale, double lambda_power) {
  if (!c || !d_mu_hat || !d_var_hat || !std::isfinite(lambda_scale) || !std::isfinite(lambda_power) ||
      !(lambda_power > 0.0))
    return EP_TV_E_ARG;
  for (int i = 0; i < c->n; ++i)
    if (!d_mu_hat[i] || !d_var_hat[i]) return fail(c, EP_TV_E_ARG, "null prediction pointer");
  int rc = ep_tv_init_cold(c);
  if (rc) return rc;
  rc = set_tab(c, const_cast<float* const*>(d_mu_hat), c->d_tab0, c->tab_host0);
  if (rc) return rc;
  rc = set_tab(c, const_cast<float* const*>(d_var_hat), c->d_tab1, c->tab_host1);
  if (rc) return rc;
  HIPCHK(c, launch_init_warm(cur_sites(c).S, c->ypix, c->d_inst, c->d_st, c->n, c->d_tiles, c->ntiles,
                             c->d_tab0, c->d_tab1, lambda_scale, lambda_power, c->sa.part_eabs,
                             c->sa.part_flags, c->stream, c->wpix));
  rc = pull_states(c);
  if (rc) return rc;
  c->warm_started = true;
  int rejected = 0;
  for (int i = 0; i < c->n; ++i) rejected += c->host_st[i].warm_ok ? 0 : 1;
  if (rejected) {
    c->err = std::to_string(rejected) + " instance(s) had a non-finite or non-positive prediction and "
             "start cold";
    return EP_TV_W_WARM_FALLBACK;
  }
  return EP_TV_OK;
}

int ep_tv_set_observation(ep_tv_ctx* c, const float* const* d_y) {
  if (!c || !d_y) return EP_TV_E_ARG;
  for (int i = 0; i < c->n; ++i) {
    if (!d_y[i]) return fail(c, EP_TV_E_ARG, "null observation pointer");
    const InstHost& h = c->ih[i];
    if (h.p.op == EP_TV_OP_DFT_MASK || h.p.op == EP_TV_OP_HADAMARD_MASK || h.p.op == EP_TV_OP_GAUSS_CS)
      continue;   // the likelihood setup writes H^T y as the pixel-space observation
    HIPCHK(c, hipMemcpy2DAsync(c->ypix + h.off, sizeof(float) * h.pitch, d_y[i],
                               sizeof(float) * h.p.width, sizeof(float) * h.p.width, h.p.height,
                               hipMemcpyDeviceToDevice, c->stream));
  }
  HIPCHK(c, lik_set_observation(c->lik, d_y, c->stream));
  c->has_obs = true;
  if (c->any_noise_map && !c->noise_set) return EP_TV_OK;   // cold start once the map is set
  return ep_tv_init_cold(c);
}

int ep_tv_set_noise_variance(ep_tv_ctx* c, const float* const* d_var) {
  if (!c || !d_var) return EP_TV_E_ARG;
  if (!c->any_noise_map) return fail(c, EP_TV_E_ARG, "no instance has noise_map = 1");
  for (int i = 0; i < c->n; ++i)
    if (c->ih[i].p.noise_map && !d_var[i]) return fail(c, EP_TV_E_ARG, "null noise-variance pointer");
  int rc = set_tab(c, const_cast<float* const*>(d_var), c->d_tab1, c->tab_host1);
  if (rc) return rc;
  HIPCHK(c, launch_noise_prec(c->wpix, c->d_inst, c->d_tiles, c->ntiles, c->d_tab1, c->stream));
  c->noise_set = true;
  return c->has_obs ? ep_tv_init_cold(c) : EP_TV_OK;
}

int ep_tv_set_rbmc_noise(ep_tv_ctx* c, const float* const* d_noise) {
  if (!c || !d_noise) return EP_TV_E_ARG;
  if (!c->lik.rbmc_ns_max) return fail(c, EP_TV_E_ARG, "no instance uses the RBMC estimator");
  for (int i = 0; i < c->n; ++i)
    if (rbmc_ns(c->ih[i].p) && !d_noise[i]) return fail(c, EP_TV_E_ARG, "null RBMC noise pointer");
  HIPCHK(c, lik_set_rbmc_noise(c->lik, d_noise, c->stream));
  c->rbmc_noise_set = true;
  return EP_TV_OK;
}

static CurSites sites_at(const ep_tv_ctx* c, int par) {
  CurSites r;
  r.S[0] = c->S0;
  for (int k = 0; k < 4; ++k) r.S[k + 1] = c->SB[par][k];
  return r;
}

// TV sweep reading the sites of buffer `par`, writing buffer par ^ 1, then the
// per-instance finalisation (EM, convergence).
static int enqueue_tv(ep_tv_ctx* c, int par, int em, bool delta, double tol, hipStream_t s) {
  SweepArgs a = c->sa;
  float2* const* in = c->SB[par];
  float2* const* out = c->SB[par ^ 1];
  a.I1 = in[0]; a.I2 = in[1]; a.I3 = in[2]; a.I4 = in[3];
  a.O1 = out[0]; a.O2 = out[1]; a.O3 = out[2]; a.O4 = out[3];
  HIPCHK(c, launch_tv_sweep(a, delta, s));
  if (em && a.em_opt == 1)
    HIPCHK(c, launch_em_ax(sites_at(c, par ^ 1).S, c->d_inst, c->d_st, c->d_tiles, c->ntiles,
                           a.part_eabs, s));
  HIPCHK(c, launch_finalize(c->d_inst, c->d_st, c->n, a, em, tol, s));
  return EP_TV_OK;
}

static int one_sweep(ep_tv_ctx* c, int em, bool delta, double tol) {
  const bool tm = c->timing && c->ev_used + 4 <= kMaxTimingEvents;
  int i0 = 0, i1 = 0;
  if (c->any_lik) {
    if (tm) HIPCHK(c, hipEventRecord(next_event(c, i0), c->stream));
    HIPCHK(c, lik_update(c->lik, cur_sites(c).S, c->stream));
    if (tm) {
      HIPCHK(c, hipEventRecord(next_event(c, i1), c->stream));
      c->ev_lik.emplace_back(i0, i1);
    }
  }
  if (tm) HIPCHK(c, hipEventRecord(next_event(c, i0), c->stream));
  SweepArgs& a = c->sa;
  float2* const* in = c->SB[c->cur];
  float2* const* out = c->SB[c->cur ^ 1];
  a.I1 = in[0]; a.I2 = in[1]; a.I3 = in[2]; a.I4 = in[3];
  a.O1 = out[0]; a.O2 = out[1]; a.O3 = out[2]; a.O4 = out[3];
  HIPCHK(c, launch_tv_sweep(a, delta, c->stream));
  c->cur ^= 1;
  if (tm) {
    HIPCHK(c, hipEventRecord(next_event(c, i1), c->stream));
    c->ev_sweep.emplace_back(i0, i1);
  }
  if (em && a.em_opt == 1)
    HIPCHK(c, launch_em_ax(cur_sites(c).S, c->d_inst, c->d_st, c->d_tiles, c->ntiles, a.part_eabs,
                           c->stream));
  HIPCHK(c, launch_finalize(c->d_inst, c->d_st, c->n, c->sa, em, tol, c->stream));
  return EP_TV_OK;
}

// ---- graph capture: the sequences are recorded on a private stream (nothing
// runs while capturing) and replayed on the caller's stream.
static int capture(ep_tv_ctx* c, hipGraphExec_t* out, const std::function<int(hipStream_t)>& body) {
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  const bool lt = c->lik.timing;
  c->lik.timing = false;
  int rc = body(c->cap);
  c->lik.timing = lt;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc == EP_TV_OK) rc = hip_check(c, e, "hipStreamEndCapture");
  if (rc == EP_TV_OK) rc = hip_check(c, hipGraphInstantiate(out, g, nullptr, nullptr, 0),
                                     "hipGraphInstantiate");
  if (g) (void)hipGraphDestroy(g);
  return rc;
}

static int build_graphs(ep_tv_ctx* c, int em, bool delta, double tol) {
  Graphs& g = c->g;
  if (g.valid && g.em == em && g.delta == delta && g.tol == tol) return EP_TV_OK;
  drop_graphs(c);
  if (c->any_lik) HIPCHK(c, lik_poll_word_alloc(c->lik));
  int rc = EP_TV_OK;
  for (int par = 0; par < 2 && rc == EP_TV_OK; ++par) {
    if (c->any_lik) {
      rc = capture(c, &g.head[par], [&](hipStream_t s) -> int {
        HIPCHK(c, lik_head(c->lik, sites_at(c, par).S, s));
        HIPCHK(c, lik_iterations(c->lik, kCgPoll, s));
        HIPCHK(c, lik_poll_word_launch(c->lik, s));
        return EP_TV_OK;
      });
      if (rc == EP_TV_OK)
        rc = capture(c, &g.head_short[par], [&](hipStream_t s) -> int {
          HIPCHK(c, lik_head(c->lik, sites_at(c, par).S, s));
          HIPCHK(c, lik_iterations(c->lik, kCgHeadShort, s));
          HIPCHK(c, lik_poll_word_launch(c->lik, s));
          return EP_TV_OK;
        });
      if (rc == EP_TV_OK)
        rc = capture(c, &g.tail[par], [&](hipStream_t s) -> int {
          HIPCHK(c, lik_tail(c->lik, c->S0, s));
          return enqueue_tv(c, par, em, delta, tol, s);
        });
    } else {
      rc = capture(c, &g.tail[par], [&](hipStream_t s) -> int { return enqueue_tv(c, par, em, delta, tol, s); });
      if (rc == EP_TV_OK)
        rc = capture(c, &g.multi[par], [&](hipStream_t s) -> int {
          for (int t = 0; t < kGraphSweeps; ++t) {
            int r = enqueue_tv(c, par ^ (t & 1), em, delta, tol, s);
            if (r) return r;
          }
          return EP_TV_OK;
        });
    }
  }
  if (rc == EP_TV_OK && c->any_lik)
    rc = capture(c, &g.cg, [&](hipStream_t s) -> int {
      HIPCHK(c, lik_iterations(c->lik, kCgPoll, s));
      HIPCHK(c, lik_poll_word_launch(c->lik, s));
      return EP_TV_OK;
    });
  if (rc == EP_TV_OK && c->any_lik)
    rc = capture(c, &g.cg8, [&](hipStream_t s) -> int {
      HIPCHK(c, lik_iterations(c->lik, 2 * kCgPoll, s));
      HIPCHK(c, lik_poll_word_launch(c->lik, s));
      return EP_TV_OK;
    });
  if (rc == EP_TV_OK && c->any_lik)
    rc = capture(c, &g.cg16, [&](hipStream_t s) -> int {
      HIPCHK(c, lik_iterations(c->lik, 4 * kCgPoll, s));
      HIPCHK(c, lik_poll_word_launch(c->lik, s));
      return EP_TV_OK;
    });
  if (rc != EP_TV_OK) {
    drop_graphs(c);
    return rc;
  }
  g.valid = true;
  g.em = em;
  g.delta = delta;
  g.tol = tol;
  return EP_TV_OK;
}

// One sweep from the graphs: the CG runs kCgPoll iterations per replay until
// every instance's solve has converged, which the last kernel of each replay
// reports in the pinned poll word the host waits on.  The head replay carries
// kCgHeadShort iterations instead when the previous sweep's solves all
// stopped within that many (near the fixed point they need about two), so
// fewer launches of a finished solve's iterations run.
static int graph_sweep(ep_tv_ctx* c) {
  Graphs& g = c->g;
  if (c->any_lik) {
    unsigned seq = lik_poll_word_seq(c->lik);
    const bool short_head = c->cg_iters_prev <= kCgHeadShort;
    HIPCHK(c, hipGraphLaunch(short_head ? g.head_short[c->cur] : g.head[c->cur], c->stream));
    int iters = short_head ? kCgHeadShort : kCgPoll;
    bool done = false;
    int used = 0;
    HIPCHK(c, lik_poll_word_wait(c->lik, c->stream, seq, done, used));
    while (!done && iters < c->lik.max_iters) {
      // as many iterations per replay as the previous sweep's solves still
      // needed at this point (the counts change slowly from sweep to sweep),
      // so long solves wait on fewer polls
      const int ahead = c->cg_iters_prev - iters;
      const int n = ahead >= 4 * kCgPoll ? 4 * kCgPoll : ahead >= 2 * kCgPoll ? 2 * kCgPoll : kCgPoll;
      seq = lik_poll_word_seq(c->lik);
      HIPCHK(c, hipGraphLaunch(n == 4 * kCgPoll ? g.cg16 : n == 2 * kCgPoll ? g.cg8 : g.cg, c->stream));
      iters += n;
      HIPCHK(c, lik_poll_word_wait(c->lik, c->stream, seq, done, used));
    }
    c->cg_iters_prev = used;
  }
  HIPCHK(c, hipGraphLaunch(g.tail[c->cur], c->stream));
  c->cur ^= 1;
  return EP_TV_OK;
}

// Run n sweeps with the given finalisation settings (direct launches or graphs;
// RBMC sample solves are launched directly).
static int advance(ep_tv_ctx* c, int n, int em, bool delta, double tol) {
  if (c->lik.rbmc_ns_max && !c->rbmc_noise_set)
    return fail(c, EP_TV_E_STATE, "the RBMC estimator needs ep_tv_set_rbmc_noise first");
  if (c->any_noise_map && !c->noise_set)
    return fail(c, EP_TV_E_STATE, "per-pixel noise variances not set (ep_tv_set_noise_variance)");
  if (!c->use_graph || c->lik.rbmc_ns_max || !c->lik.gauss.empty()) {
    for (int t = 0; t < n; ++t) {
      int rc = one_sweep(c, em, delta, tol);
      if (rc) return rc;
    }
    return EP_TV_OK;
  }
  int rc = build_graphs(c, em, delta, tol);
  if (rc) return rc;
  int t = 0;
  if (!c->any_lik)
    for (; t + kGraphSweeps <= n; t += kGraphSweeps)
      HIPCHK(c, hipGraphLaunch(c->g.multi[c->cur], c->stream));
  for (; t < n; ++t) {
    rc = graph_sweep(c);
    if (rc) return rc;
  }
  return EP_TV_OK;
}

int ep_tv_run(ep_tv_ctx* c, int32_t n_sweeps, int32_t em) {
  if (!c || n_sweeps < 0) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  if (em && c->sa.prior != PRIOR_L1) return fail(c, EP_TV_E_ARG, "EM is defined for the l1 factor only");
  return advance(c, n_sweeps, em ? 1 : 0, false, 0.0);
}

static int pull_states(ep_tv_ctx* c) {
  if (!c->pull_st) {   // pinned, so the copy goes straight to host memory
    if (hipHostMalloc(reinterpret_cast<void**>(&c->pull_st), sizeof(InstState) * (size_t)c->n) !=
        hipSuccess) {
      c->pull_st = nullptr;
      return fail(c, EP_TV_E_HIP, "hipHostMalloc of the state staging buffer failed");
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->pull_st, c->d_st, sizeof(InstState) * c->n, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(c->host_st.data(), c->pull_st, sizeof(InstState) * c->n);
  return EP_TV_OK;
}

int ep_tv_em_step(ep_tv_ctx* c, int32_t n_ep, double* lambda_out) {
  if (!c || n_ep < 1) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  if (c->lik.rbmc_ns_max && !c->rbmc_noise_set)
    return fail(c, EP_TV_E_STATE, "the RBMC estimator needs ep_tv_set_rbmc_noise first");
  if (c->any_noise_map && !c->noise_set)
    return fail(c, EP_TV_E_STATE, "per-pixel noise variances not set (ep_tv_set_noise_variance)");
  if (c->sa.prior != PRIOR_L1) return fail(c, EP_TV_E_ARG, "EM is defined for the l1 factor only");
  for (int t = 0; t < n_ep; ++t) {
    int rc = one_sweep(c, t == n_ep - 1 ? 1 : 0, false, 0.0);
    if (rc) return rc;
  }
  if (lambda_out) {
    int rc = pull_states(c);
    if (rc) return rc;
    for (int i = 0; i < c->n; ++i) lambda_out[i] = c->host_st[i].lam;
  }
  return EP_TV_OK;
}

static int set_tab(ep_tv_ctx* c, float* const* host, float** dev, std::vector<float*>& keep) {
  keep.assign(host, host + c->n);
  HIPCHK(c, hipMemcpyAsync(dev, keep.data(), sizeof(float*) * c->n, hipMemcpyHostToDevice,
                           c->stream));
  return EP_TV_OK;
}

int ep_tv_marginals(ep_tv_ctx* c, float* const* d_mean, float* const* d_var) {
  if (!c) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  if (!d_mean && !d_var) return EP_TV_OK;
  if (d_mean) {
    int rc = set_tab(c, d_mean, c->d_tab0, c->tab_host0);
    if (rc) return rc;
  }
  if (d_var) {
    int rc = set_tab(c, d_var, c->d_tab1, c->tab_host1);
    if (rc) return rc;
  }
  HIPCHK(c, launch_marginals(cur_sites(c).S, c->d_inst, c->d_tiles, c->ntiles, d_mean ? c->d_tab0 : nullptr,
                             d_var ? c->d_tab1 : nullptr, c->stream));
  return EP_TV_OK;
}

static void fill_stats(ep_tv_ctx* c, ep_tv_stats* s) {
  for (int i = 0; i < c->n; ++i) {
    const InstState& h = c->host_st[i];
    ep_tv_stats& o = s[i];
    o.sweeps_done = (int32_t)h.sweeps;
    o.cg_iters_last = h.cg_last;
    o.cg_iters_total = h.cg_total;
    o.clamp_count = (int32_t)h.clamps;
    o.converged = h.converged;
    o.status = (h.flags & FLAG_NONFINITE)   ? EP_TV_E_NONFINITE
               : (h.flags & FLAG_DIVERGED)  ? EP_TV_E_DIVERGED
               : !h.converged               ? EP_TV_W_NOT_CONVERGED
               : h.cold_restarts            ? EP_TV_W_WARM_FALLBACK
                                            : EP_TV_OK;
    o.cold_restarts = h.cold_restarts;
    o.reserved_ = 0;
    o.lambda = h.lam;
    o.a_bar_u = h.abar;
    o.max_dmu_rel = h.dmu;
    o.max_dv_rel = h.dv;
    o.elapsed_ms = c->last_elapsed_ms;
    o.lik_precision = h.gamma;
    o.cavity_precision_mean = h.dbar;
    o.cg_rel_residual = h.cg_bb > 0.0 ? std::sqrt(h.cg_rr / h.cg_bb) : 0.0;
  }
}

// An instance started from a prediction (ep_tv_init_warm) or restored sites
// (ep_tv_set_sites) that went non-finite or diverged is re-initialised cold,
// once, and keeps sweeping; the host state is current (pulled by the caller).
static int restart_failed_warm(ep_tv_ctx* c) {
  int nrestart = 0;
  for (int i = 0; i < c->n; ++i) {
    InstState& s = c->host_st[i];
    if (!(s.flags & (FLAG_NONFINITE | FLAG_DIVERGED)) || !s.warm || s.cold_restarts > 0) continue;
    const double yr = s.yrange, ys = s.yscale;
    std::memset(&s, 0, sizeof(s));
    s.lam = s.lam_prev = c->ih[i].p.lambda0;
    s.yrange = yr;
    s.yscale = ys;
    s.active = 1u;
    s.restart = 1;
    s.cold_restarts = 1;
    ++nrestart;
  }
  if (!nrestart) return EP_TV_OK;
  HIPCHK(c, hipMemcpyAsync(c->d_st, c->host_st.data(), sizeof(InstState) * c->n,
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_init_cold(cur_sites(c).S, c->ypix, c->d_inst, c->d_st, c->d_tiles, c->ntiles,
                             c->stream, true, c->wpix));
  for (int i = 0; i < c->n; ++i) c->host_st[i].restart = 0;
  HIPCHK(c, hipMemcpyAsync(c->d_st, c->host_st.data(), sizeof(InstState) * c->n,
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));   // the host state array is rewritten by later pulls
  return EP_TV_OK;
}

int ep_tv_solve(ep_tv_ctx* c, int32_t max_sweeps, double tol, int32_t em, float* const* d_mean,
                float* const* d_var, ep_tv_stats* stats) {
  if (!c || max_sweeps < 0) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  if (em && c->sa.prior != PRIOR_L1) return fail(c, EP_TV_E_ARG, "EM is defined for the l1 factor only");
  const auto t0 = std::chrono::steady_clock::now();
  const bool use_tol = tol > 0.0;
  const int check_every = kGraphSweeps;
  int rc = EP_TV_OK;
  for (int t = 0; t < max_sweeps; t += check_every) {
    rc = advance(c, std::min(check_every, max_sweeps - t), em ? 1 : 0, true, use_tol ? tol : 0.0);
    if (rc) return rc;
    if (use_tol || c->warm_started) {
      rc = pull_states(c);
      if (rc) return rc;
      if (c->warm_started) {
        rc = restart_failed_warm(c);
        if (rc) return rc;
      }
      bool any = false;
      for (int i = 0; i < c->n; ++i) any = any || c->host_st[i].active;
      if (use_tol && !any) break;
    }
  }
  rc = ep_tv_marginals(c, d_mean, d_var);
  if (rc) return rc;
  rc = pull_states(c);
  if (rc) return rc;
  c->last_elapsed_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) fill_stats(c, stats);
  bool nonfinite = false, diverged = false, notconv = false, restarted = false;
  for (int i = 0; i < c->n; ++i) {
    nonfinite = nonfinite || (c->host_st[i].flags & FLAG_NONFINITE);
    diverged = diverged || (c->host_st[i].flags & FLAG_DIVERGED);
    notconv = notconv || !c->host_st[i].converged;
    restarted = restarted || c->host_st[i].cold_restarts > 0;
  }
  if (nonfinite) return fail(c, EP_TV_E_NONFINITE, "non-finite EP state");
  if (diverged) return fail(c, EP_TV_E_DIVERGED, "EP diverged (the global mean left 1e3 times the "
                                                 "observation's scale)");
  if (use_tol && notconv) return EP_TV_W_NOT_CONVERGED;
  if (restarted) {
    c->err = "a warm-started instance failed and was restarted cold";
    return EP_TV_W_WARM_FALLBACK;
  }
  return EP_TV_OK;
}

int ep_tv_get_sites(ep_tv_ctx* c, float* const* d_out) {
  if (!c || !d_out) return EP_TV_E_ARG;
  int rc = set_tab(c, d_out, c->d_tab0, c->tab_host0);
  if (rc) return rc;
  HIPCHK(c, launch_sites_io(cur_sites(c).S, c->d_inst, c->d_tiles, c->ntiles, c->d_tab0, 1,
                            c->stream));
  return EP_TV_OK;
}

int ep_tv_set_sites(ep_tv_ctx* c, const float* const* d_in, const double* lambda) {
  if (!c || !d_in) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  int rc = pull_states(c);
  if (rc) return rc;
  for (int i = 0; i < c->n; ++i) {
    InstState& s = c->host_st[i];
    if (lambda) {
      if (!(lambda[i] > 0.0)) return fail(c, EP_TV_E_ARG, "lambda must be > 0");
      s.lam = s.lam_prev = lambda[i];
    }
    s.active = 1u;
    s.converged = 0;
    s.sweeps = 0u;
    s.clamps = 0u;
    s.flags = 0u;
    s.cg_total = 0;
    s.warm = 1;               // restored sites are informative: no skipped q0 update
    s.warm_ok = 1;
  }
  HIPCHK(c, hipMemcpyAsync(c->d_st, c->host_st.data(), sizeof(InstState) * c->n,
                           hipMemcpyHostToDevice, c->stream));
  rc = set_tab(c, const_cast<float* const*>(d_in), c->d_tab0, c->tab_host0);
  if (rc) return rc;
  HIPCHK(c, launch_sites_io(cur_sites(c).S, c->d_inst, c->d_tiles, c->ntiles, c->d_tab0, 0,
                            c->stream));
  HIPCHK(c, lik_resume(c->lik, c->stream));
  c->warm_started = true;
  return EP_TV_OK;
}

int ep_tv_get_stats(ep_tv_ctx* c, ep_tv_stats* stats) {
  if (!c || !stats) return EP_TV_E_ARG;
  int rc = pull_states(c);
  if (rc) return rc;
  fill_stats(c, stats);
  return EP_TV_OK;
}

int ep_tv_get_lik_planes(ep_tv_ctx* c, int32_t instance, float* d_out) {
  if (!c || !d_out || instance < 0 || instance >= c->n) return EP_TV_E_ARG;
  const InstHost& h = c->ih[instance];
  if (h.p.op == EP_TV_OP_IDENTITY) return fail(c, EP_TV_E_ARG, "identity operator has no likelihood planes");
  const int which[10] = {LP_X, LP_TAUC, LP_ETAC, LP_B, LP_R, LP_Z, LP_SPEC, LP_P0, LP_P1, LP_Q};
  const size_t plane = (size_t)h.p.height * h.p.width;
  for (int k = 0; k < 10; ++k)
    HIPCHK(c, hipMemcpy2DAsync(d_out + k * plane, sizeof(float) * h.p.width,
                               c->lik.planes[which[k]] + h.off, sizeof(float) * h.pitch,
                               sizeof(float) * h.p.width, h.p.height, hipMemcpyDeviceToDevice,
                               c->stream));
  return EP_TV_OK;
}

int ep_tv_tilted_moments(int32_t n, const float* d_m, const float* d_s, float lambda, float* d_rho,
                         float* d_delta, float* d_eabs, void* stream) {
  if (n < 0 || (n > 0 && (!d_m || !d_s || !d_rho || !d_delta || !d_eabs)) || !(lambda >= 0.f))
    return EP_TV_E_ARG;
  if (launch_tilted(n, d_m, d_s, lambda, d_rho, d_delta, d_eabs,
                    reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return EP_TV_E_HIP;
  return EP_TV_OK;
}

int ep_tv_tilted_moments_prior(int32_t prior, const double* theta, int32_t n, const float* d_m,
                               const float* d_s, float* d_rho, float* d_delta, float* d_eabs,
                               void* stream) {
  if (!theta || n < 0 || (n > 0 && (!d_m || !d_s || !d_rho || !d_delta || !d_eabs)))
    return EP_TV_E_ARG;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  if (prior == EP_TV_PRIOR_L1) {
    if (!(theta[0] >= 0.0) || !std::isfinite(theta[0])) return EP_TV_E_ARG;
    e = launch_tilted(n, d_m, d_s, (float)theta[0], d_rho, d_delta, d_eabs, s);
  } else if (prior == EP_TV_PRIOR_MOG2 || prior == EP_TV_PRIOR_BG) {
    const double om = theta[0], v1 = theta[1];
    const double v2 = prior == EP_TV_PRIOR_MOG2 ? theta[2] : 0.0;
    if (!(om > 0.0 && om <= 1.0) || !(v1 > 0.0) || !std::isfinite(v1)) return EP_TV_E_ARG;
    if (prior == EP_TV_PRIOR_MOG2 && (!(v2 > 0.0) || !std::isfinite(v2))) return EP_TV_E_ARG;
    const double a2 = 1.0 - om;
    e = launch_tilted_mixture(n, d_m, d_s, (float)(a2 > 0.0 ? std::log(a2 / om) : -HUGE_VAL),
                              (float)(v1 - v2), (float)v1, (float)v2, d_rho, d_delta, d_eabs, s);
  } else {
    return EP_TV_E_ARG;
  }
  return e == hipSuccess ? EP_TV_OK : EP_TV_E_HIP;
}

int ep_tv_set_timing(ep_tv_ctx* c, int32_t enable) {
  if (!c) return EP_TV_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  timing_clear(c);
  lik_timing(c->lik, enable != 0, true);
  c->timing = enable != 0;
  return EP_TV_OK;
}

int ep_tv_get_timing(ep_tv_ctx* c, ep_tv_timing* out) {
  if (!c || !out) return EP_TV_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memset(out, 0, sizeof(*out));
  for (auto& pr : c->ev_sweep) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[pr.first], c->ev_pool[pr.second]));
    out->sweep_ms += ms;
    out->sweep_launches += 1;
  }
  for (auto& pr : c->ev_lik) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[pr.first], c->ev_pool[pr.second]));
    out->lik_ms += ms;
    out->lik_updates += 1;
  }
  double ms[KT_COUNT] = {};
  int n[KT_COUNT] = {};
  HIPCHK(c, lik_timing_read(c->lik, ms, n));
  out->apply_ms = ms[KT_APPLY];
  out->apply_launches = n[KT_APPLY];
  out->precond_ms = ms[KT_PRECOND];
  out->precond_launches = n[KT_PRECOND];
  out->rf_fwd_ms = ms[KT_RF_FWD];
  out->rf_fwd_launches = n[KT_RF_FWD];
  out->rf_filt_ms = ms[KT_RF_FILT];
  out->rf_filt_launches = n[KT_RF_FILT];
  out->rf_inv_ms = ms[KT_RF_INV];
  out->rf_inv_launches = n[KT_RF_INV];
  out->fin_ms = ms[KT_FIN];
  out->fin_launches = n[KT_FIN];
  out->lik_other_ms = ms[KT_OTHER];
  out->lik_other_launches = n[KT_OTHER];
  out->dgemm_ms = ms[KT_DGEMM];
  out->dgemm_launches = n[KT_DGEMM];
  out->dgemm_flops = c->lik.dgemm_flops;
  return EP_TV_OK;
}

int ep_tv_set_option(ep_tv_ctx* c, int32_t option, int64_t value) {
  if (!c) return EP_TV_E_ARG;
  switch (option) {
    case EP_TV_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(c, EP_TV_E_ARG, "graph option must be 0 or 1");
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->use_graph = value != 0;
      if (!c->use_graph) drop_graphs(c);
      return EP_TV_OK;
    case EP_TV_OPT_EM_OPTION:
      if (value < 1 || value > 3) return fail(c, EP_TV_E_ARG, "EM option must be 1, 2 or 3");
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->sa.em_opt = (int)value;
      drop_graphs(c);
      return EP_TV_OK;
    case EP_TV_OPT_PERSISTENT:
      if (value != 0 && value != 1) return fail(c, EP_TV_E_ARG, "persistent option must be 0 or 1");
      HIPCHK(c, hipStreamSynchronize(c->stream));
      c->sa.persistent = (int)value;
      drop_graphs(c);
      return EP_TV_OK;
    case EP_TV_OPT_TILE_ROWS: {
      if (value < 2 || value > 4096 || value % 2)
        return fail(c, EP_TV_E_ARG, "tile rows must be even and in [2, 4096]");
      std::vector<InstHost> probe = c->ih;
      if (count_tiles(probe, (int)value) > c->L.tile_cap)
        return fail(c, EP_TV_E_ARG, "tile rows below the workspace's tile capacity");
      HIPCHK(c, hipStreamSynchronize(c->stream));
      return set_rows(c, (int)value);
    }
    default:
      return fail(c, EP_TV_E_ARG, "unknown option");
  }
}

int ep_tv_get_option(ep_tv_ctx* c, int32_t option, int64_t* value) {
  if (!c || !value) return EP_TV_E_ARG;
  switch (option) {
    case EP_TV_OPT_GRAPH: *value = c->use_graph ? 1 : 0; return EP_TV_OK;
    case EP_TV_OPT_TILE_ROWS: *value = c->chunk_rows; return EP_TV_OK;
    case EP_TV_OPT_EM_OPTION: *value = c->sa.em_opt; return EP_TV_OK;
    case EP_TV_OPT_PERSISTENT: *value = c->sa.persistent; return EP_TV_OK;
    default: return fail(c, EP_TV_E_ARG, "unknown option");
  }
}

int ep_tv_autotune(ep_tv_ctx* c, int32_t repeats, ep_tv_tune_result* out) {
  if (!c || repeats < 1 || repeats > 1000) return EP_TV_E_ARG;
  if (!c->has_obs) return fail(c, EP_TV_E_STATE, "no observation set");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  ep_tv_tune_result r;
  std::memset(&r, 0, sizeof(r));
  const int rows0 = c->chunk_rows;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  int rc = hip_check(c, hipEventCreate(&e1), "hipEventCreate");
  // the sweep kernel alone reads the current sites and writes the other buffer
  // and the per-tile partials, so timing it leaves the EP state unchanged
  SweepArgs a = c->sa;
  float2* const* in = c->SB[c->cur];
  float2* const* o = c->SB[c->cur ^ 1];
  a.I1 = in[0]; a.I2 = in[1]; a.I3 = in[2]; a.I4 = in[3];
  a.O1 = o[0]; a.O2 = o[1]; a.O3 = o[2]; a.O4 = o[3];
  int last_tiles = -1;
  double best = 1e300;
  int best_rows = rows0;
  for (int k = 0; k < kNumTuneRows && rc == EP_TV_OK; ++k) {
    const int rows = kTuneRows[k];
    const int nt = count_tiles(c->ih, rows);
    if (nt > c->L.tile_cap || nt == last_tiles) continue;   // same tiling as a smaller height
    last_tiles = nt;
    rc = set_rows(c, rows);
    if (rc) break;
    a.ntiles = c->ntiles;
    rc = hip_check(c, launch_tv_sweep(a, true, c->stream), "tune warm-up");
    if (rc == EP_TV_OK) rc = hip_check(c, hipEventRecord(e0, c->stream), "hipEventRecord");
    for (int t = 0; t < repeats && rc == EP_TV_OK; ++t)
      rc = hip_check(c, launch_tv_sweep(a, true, c->stream), "tune launch");
    if (rc == EP_TV_OK) rc = hip_check(c, hipEventRecord(e1, c->stream), "hipEventRecord");
    if (rc == EP_TV_OK) rc = hip_check(c, hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    if (rc == EP_TV_OK) rc = hip_check(c, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (rc != EP_TV_OK) break;
    const double per = ms / repeats;
    if (r.candidates < 16) {
      r.rows[r.candidates] = rows;
      r.ms[r.candidates] = per;
      r.candidates += 1;
    }
    if (rows == rows0) r.default_ms = per;
    if (per < best) {
      best = per;
      best_rows = rows;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  int rc2 = set_rows(c, rc == EP_TV_OK ? best_rows : rows0);
  if (rc != EP_TV_OK) return rc;
  if (rc2 != EP_TV_OK) return rc2;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  r.tile_rows = best_rows;
  r.best_ms = best;
  {
    std::vector<ep_tv_problem> ps(c->n);
    for (int i = 0; i < c->n; ++i) ps[i] = c->ih[i].p;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_rows[shape_key(ps.data(), c->n)] = best_rows;
  }
  if (out) *out = r;
  return EP_TV_OK;
}

const char* ep_tv_last_error(const ep_tv_ctx* c) { return c ? c->err.c_str() : "null context"; }

void ep_tv_destroy(ep_tv_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  lik_destroy(c->lik);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->pull_st) (void)hipHostFree(c->pull_st);
  delete c;
}

}  // extern "C"
