// Host-side checks of the C ABI under AddressSanitizer (built by
// tests/test_host_asan.py with the library's host code instrumented).  Every
// call below returns before its first HIP call (argument validation, workspace
// layout, error returns), so it needs no GPU and touches none: the validation,
// layout and error paths of include/ep_tv.h and include/ep_tv_net.h execute
// under the sanitizer.  Prints one line per failed expectation and exits
// non-zero if there was one.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ep_tv.h"
#include "ep_tv_net.h"

static int g_fail = 0;

#define EXPECT(cond, what)                                    \
  do {                                                        \
    if (!(cond)) {                                            \
      std::printf("FAILED: %s (line %d)\n", what, __LINE__); \
      ++g_fail;                                               \
    }                                                         \
  } while (0)

static ep_tv_problem base(int h, int w) {
  ep_tv_problem p;
  std::memset(&p, 0, sizeof(p));
  p.height = h;
  p.width = w;
  p.op = EP_TV_OP_IDENTITY;
  p.boundary = EP_TV_BND_FREE;
  p.noise_var = 1e-2;
  p.lambda0 = 1.0;
  p.damping = 0.5;
  return p;
}

int main() {
  EXPECT(ep_tv_version() != nullptr && std::strlen(ep_tv_version()) > 0, "version string");
  EXPECT(std::strlen(ep_tv_last_error(nullptr)) > 0, "last_error(NULL)");
  ep_tv_destroy(nullptr);

  // operator variants the layout must accept
  std::vector<float> taps(9 * 9, 1.0f / 81.0f), taps_ns(5 * 3, 0.0f);
  taps_ns[0] = 0.5f;
  taps_ns[7] = 0.25f;
  taps_ns[14] = 0.25f;   // not separable
  std::vector<uint8_t> mask64(64 * 64), mask5(4 * 4);
  for (size_t i = 0; i < mask64.size(); ++i) mask64[i] = (i * 2654435761u >> 7) % 3 == 0;
  for (size_t i = 0; i < mask5.size(); ++i) mask5[i] = i % 2;
  const int gh = 12, gw = 10, gm = 36;
  std::vector<float> sense((size_t)gm * gh * gw);
  for (size_t i = 0; i < sense.size(); ++i) sense[i] = (float)std::sin(0.37 * (double)i) * 0.2f;

  std::vector<ep_tv_problem> ok;
  ok.push_back(base(1, 1));
  ok.push_back(base(37, 91));
  {
    ep_tv_problem p = base(64, 64);
    p.boundary = EP_TV_BND_PERIODIC;
    ok.push_back(p);
  }
  {
    ep_tv_problem p = base(70, 52);
    p.op = EP_TV_OP_BLUR_PERIODIC;
    p.blur_taps = taps.data();
    p.blur_h = p.blur_w = 9;
    ok.push_back(p);
    p.blur_taps = taps_ns.data();
    p.blur_h = 5;
    p.blur_w = 3;
    ok.push_back(p);
    p.var_estimator = EP_TV_VAR_RBMC;
    p.rbmc_samples = 4;
    ok.push_back(p);
  }
  {
    ep_tv_problem p = base(64, 64);
    p.op = EP_TV_OP_DFT_MASK;
    p.dft_mask = mask64.data();
    ok.push_back(p);
    p.op = EP_TV_OP_HADAMARD_MASK;
    ok.push_back(p);
    ep_tv_problem q = base(4, 4);
    q.op = EP_TV_OP_HADAMARD_MASK;
    q.dft_mask = mask5.data();
    ok.push_back(q);
  }
  {
    ep_tv_problem p = base(gh, gw);
    p.op = EP_TV_OP_GAUSS_CS;
    p.sense_matrix = sense.data();
    p.sense_rows = gm;
    ok.push_back(p);
  }
  {
    ep_tv_problem p = base(30, 40);
    p.noise_map = 1;
    ok.push_back(p);
    p.noise_map = 0;
    p.prior = EP_TV_PRIOR_MOG2;
    p.prior_omega = 0.3;
    p.prior_s1sq = 0.1;
    p.prior_s2sq = 1e-3;
    ok.push_back(p);
  }
  size_t total = 0;
  for (size_t i = 0; i < ok.size(); ++i) {
    size_t b = 0;
    const int rc = ep_tv_workspace_bytes(&ok[i], 1, &b);
    char what[64];
    std::snprintf(what, sizeof(what), "valid problem %zu accepted", i);
    EXPECT(rc == EP_TV_OK && b > 0, what);
    total += b;
  }
  {
    // several instances in one context (one mixture kind rules out the MoG2 one)
    std::vector<ep_tv_problem> batch(ok.begin(), ok.end() - 1);
    size_t b = 0;
    EXPECT(ep_tv_workspace_bytes(batch.data(), (int)batch.size(), &b) == EP_TV_OK && b > 0,
           "mixed batch accepted");
  }

  // invalid problems: each must be rejected by validation, with no memory error
  std::vector<ep_tv_problem> bad;
  auto add = [&](ep_tv_problem p) { bad.push_back(p); };
  { ep_tv_problem p = base(0, 5); add(p); }
  { ep_tv_problem p = base(5, 16385); add(p); }
  { ep_tv_problem p = base(5, 5); p.noise_var = 0.0; add(p); }
  { ep_tv_problem p = base(5, 5); p.noise_var = NAN; add(p); }
  { ep_tv_problem p = base(5, 5); p.lambda0 = -1.0; add(p); }
  { ep_tv_problem p = base(5, 5); p.damping = 0.0; add(p); }
  { ep_tv_problem p = base(5, 5); p.damping = 1.5; add(p); }
  { ep_tv_problem p = base(5, 5); p.boundary = EP_TV_BND_PERIODIC; add(p); }   // odd sizes
  { ep_tv_problem p = base(5, 5); p.boundary = 7; add(p); }
  { ep_tv_problem p = base(5, 5); p.op = 9; add(p); }
  { ep_tv_problem p = base(5, 5); p.op = EP_TV_OP_BLUR_PERIODIC; add(p); }     // no taps
  {
    ep_tv_problem p = base(5, 5);
    p.op = EP_TV_OP_BLUR_PERIODIC;
    p.blur_taps = taps.data();
    p.blur_h = 8;
    p.blur_w = 9;   // even tap size
    add(p);
  }
  { ep_tv_problem p = base(48, 48); p.op = EP_TV_OP_DFT_MASK; p.dft_mask = mask64.data(); add(p); }
  { ep_tv_problem p = base(64, 64); p.op = EP_TV_OP_HADAMARD_MASK; add(p); }   // no mask
  { ep_tv_problem p = base(gh, gw); p.op = EP_TV_OP_GAUSS_CS; p.sense_rows = gm; add(p); }
  {
    ep_tv_problem p = base(gh, gw);
    p.op = EP_TV_OP_GAUSS_CS;
    p.sense_matrix = sense.data();
    p.sense_rows = 0;
    add(p);
  }
  { ep_tv_problem p = base(5, 5); p.cg_tol = -1.0; add(p); }
  { ep_tv_problem p = base(5, 5); p.cg_max_iters = -3; add(p); }
  { ep_tv_problem p = base(5, 5); p.cg_precond = 5; add(p); }
  { ep_tv_problem p = base(5, 5); p.cg_reduce = 1.0; add(p); }
  { ep_tv_problem p = base(5, 5); p.prior = 4; add(p); }
  { ep_tv_problem p = base(5, 5); p.prior = EP_TV_PRIOR_BG; p.prior_omega = 0.0; add(p); }
  {
    ep_tv_problem p = base(70, 52);
    p.op = EP_TV_OP_BLUR_PERIODIC;
    p.blur_taps = taps.data();
    p.blur_h = p.blur_w = 9;
    p.var_estimator = EP_TV_VAR_RBMC;
    p.rbmc_samples = 0;
    add(p);
  }
  {
    ep_tv_problem p = base(70, 52);
    p.op = EP_TV_OP_BLUR_PERIODIC;
    p.blur_taps = taps.data();
    p.blur_h = p.blur_w = 9;
    p.noise_map = 1;   // identity operator only
    add(p);
  }
  { ep_tv_problem p = base(5, 5); p.reserved = 1; add(p); }
  for (size_t i = 0; i < bad.size(); ++i) {
    size_t b = 12345;
    const int rc = ep_tv_workspace_bytes(&bad[i], 1, &b);
    char what[64];
    std::snprintf(what, sizeof(what), "invalid problem %zu rejected", i);
    EXPECT(rc != EP_TV_OK, what);
  }
  {
    size_t b = 0;
    EXPECT(ep_tv_workspace_bytes(nullptr, 1, &b) != EP_TV_OK, "null problem array");
    EXPECT(ep_tv_workspace_bytes(ok.data(), 0, &b) != EP_TV_OK, "zero problems");
    EXPECT(ep_tv_workspace_bytes(ok.data(), 1, nullptr) != EP_TV_OK, "null byte count");
    // two different mixture kinds in one context
    ep_tv_problem mix[2] = {ok.back(), ok.back()};
    mix[1].prior = EP_TV_PRIOR_BG;
    mix[1].prior_omega = 0.5;
    mix[1].prior_s1sq = 0.2;
    EXPECT(ep_tv_workspace_bytes(mix, 2, &b) != EP_TV_OK, "two factor kinds in one context");
  }

  // create: invalid arguments and a short workspace return before any device call
  // (the partly built context is released)
  {
    ep_tv_ctx* c = nullptr;
    size_t b = 0;
    ep_tv_workspace_bytes(&ok[3], 1, &b);
    // never dereferenced: every call below returns before its first device call
    void* fake = reinterpret_cast<void*>(uintptr_t(1) << 20);
    void* misaligned = reinterpret_cast<void*>((uintptr_t(1) << 20) + 8);
    EXPECT(ep_tv_create(&ok[3], 1, nullptr, b, nullptr, &c) == EP_TV_E_ARG && c == nullptr,
           "create without a workspace");
    EXPECT(ep_tv_create(&ok[3], 1, misaligned, b, nullptr, &c) == EP_TV_E_ARG && c == nullptr,
           "create with a misaligned workspace");
    EXPECT(ep_tv_create(&ok[3], 1, fake, 16, nullptr, &c) == EP_TV_E_OOM && c == nullptr,
           "create with a short workspace");
    EXPECT(ep_tv_create(&ok[3], 1, fake, b, nullptr, nullptr) == EP_TV_E_ARG,
           "create without an output handle");
    EXPECT(ep_tv_create(&bad[4], 1, fake, b, nullptr, &c) == EP_TV_E_ARG && c == nullptr,
           "create with an invalid problem");
  }

  // calls on a null context
  {
    double lam = 0.0;
    ep_tv_stats st;
    int64_t v = 0;
    EXPECT(ep_tv_init_cold(nullptr) != EP_TV_OK, "init_cold(NULL)");
    EXPECT(ep_tv_run(nullptr, 1, 0) != EP_TV_OK, "run(NULL)");
    EXPECT(ep_tv_em_step(nullptr, 1, &lam) != EP_TV_OK, "em_step(NULL)");
    EXPECT(ep_tv_get_stats(nullptr, &st) != EP_TV_OK, "get_stats(NULL)");
    EXPECT(ep_tv_get_option(nullptr, EP_TV_OPT_GRAPH, &v) != EP_TV_OK, "get_option(NULL)");
    EXPECT(ep_tv_set_option(nullptr, EP_TV_OPT_GRAPH, 1) != EP_TV_OK, "set_option(NULL)");
    EXPECT(ep_tv_solve(nullptr, 10, 1e-5, 0, nullptr, nullptr, &st) != EP_TV_OK, "solve(NULL)");
    EXPECT(ep_tv_tilted_moments(-1, nullptr, nullptr, 1.0f, nullptr, nullptr, nullptr, nullptr) !=
               EP_TV_OK,
           "tilted moments with n < 0");
  }

  // the allocation-free entry point validates before touching the device
  {
    std::vector<float> y(16), m(16), v(16);
    EXPECT(ep_tv_denoise_noalloc(0, 4, EP_TV_BND_FREE, 0.01, 1.0, 0.5, 5, 0, y.data(), m.data(),
                                 v.data(), nullptr) == EP_TV_E_ARG,
           "noalloc with height 0");
    EXPECT(ep_tv_denoise_noalloc(600, 4, EP_TV_BND_FREE, 0.01, 1.0, 0.5, 5, 0, y.data(),
                                 m.data(), v.data(), nullptr) == EP_TV_E_ARG,
           "noalloc above its size limit");
    EXPECT(ep_tv_denoise_noalloc(4, 4, EP_TV_BND_FREE, 0.01, 1.0, 0.0, 5, 0, y.data(), m.data(),
                                 v.data(), nullptr) == EP_TV_E_ARG,
           "noalloc with damping 0");
    EXPECT(ep_tv_denoise_noalloc(4, 4, EP_TV_BND_FREE, 0.01, 1.0, 0.5, 5, 0, nullptr, m.data(),
                                 v.data(), nullptr) == EP_TV_E_ARG,
           "noalloc without an observation");
  }

  // the warm-start network's host checks
  {
    size_t b = 0;
    EXPECT(ep_tv_net_param_count() > 0, "net parameter count");
    EXPECT(ep_tv_net_workspace_bytes(2, 64, 48, &b) == EP_TV_OK && b > 0, "net workspace");
    EXPECT(ep_tv_net_workspace_bytes(0, 64, 48, &b) != EP_TV_OK, "net workspace, batch 0");
    EXPECT(ep_tv_net_workspace_bytes(2, 64, 20000, &b) != EP_TV_OK, "net workspace, too wide");
    EXPECT(std::strlen(ep_tv_net_last_error(nullptr)) > 0, "net last_error(NULL)");
    EXPECT(ep_tv_net_adam_count(nullptr) < 0, "net adam_count(NULL)");
    ep_tv_net_destroy(nullptr);
  }

  std::printf("%s: %zu valid and %zu invalid problems, workspace bytes summed %zu\n",
              g_fail ? "FAILED" : "ok", ok.size(), bad.size(), total);
  return g_fail ? 1 : 0;
}
