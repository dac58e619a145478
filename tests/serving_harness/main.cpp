// Serving harness: drives the request server of serve.cpp and the C ABI of
// capi.cpp (real code) over the host stand-ins of the HIP runtime and of the
// kernel launchers, in the pattern of the GPU serving test, under
// ThreadSanitizer.  Phases, repeated:
//   1. six requests one at a time (one worker), then all six with up to four
//      running, on fresh servers: every E_c the same alone and in the mix;
//   2. six requests with up to three running while every third contraction
//      fails after queueing its kernel: failed requests report
//      SSRPA_ERR_NOMEM, the others finish, and no buffer of a failed solve
//      reaches another request while its kernel still runs;
//   3. a description with a repeated plane wave is refused before any
//      device work.
// Exit status 0 when every check holds; ThreadSanitizer reports races.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../include/ssrpa.h"

extern std::atomic<int> g_fail_herk_every;

namespace {

struct Sys {
  std::vector<int32_t> miller;
  std::vector<double> coeff, energy;
  ssrpa_system_desc d{};
};

// Plane waves |n_i| <= 2 in a 16^3 box, chi0 set |n|^2 <= 2 (alias bound
// 2*2 + 1 + 1 = 6 <= 16).
Sys make_sys(int n_v, int n_c, unsigned seed) {
  Sys s;
  for (int a = -2; a <= 2; ++a)
    for (int b = -2; b <= 2; ++b)
      for (int c = -2; c <= 2; ++c) s.miller.insert(s.miller.end(), {a, b, c});
  const int n_pw = (int)s.miller.size() / 3, nb = n_v + n_c;
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  s.coeff.resize(2 * (size_t)n_pw * nb);
  for (auto &x : s.coeff) x = u(rng);
  for (int i = 0; i < n_v; ++i) s.energy.push_back(-1.0 + 0.01 * i);
  for (int i = 0; i < n_c; ++i) s.energy.push_back(0.5 + 0.01 * i);
  const double a = 8.0;
  double lat[9] = {a, 0, 0, 0, a, 0, 0, 0, a};
  for (int i = 0; i < 9; ++i) s.d.lattice[i] = lat[i];
  s.d.fft[0] = s.d.fft[1] = s.d.fft[2] = 16;
  s.d.n_pw = n_pw;
  s.d.miller = s.miller.data();
  s.d.n_v = n_v;
  s.d.n_c = n_c;
  s.d.coeff = s.coeff.data();
  s.d.coeff_on_device = 0;
  s.d.energy = s.energy.data();
  const double g1 = 2.0 * M_PI / a;
  s.d.ecut_chi = 0.5 * 2.5 * g1 * g1;  // |n|^2 <= 2
  return s;
}

int failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

std::vector<double> run_stream(ssrpa_context *ctx, std::vector<Sys> &sys,
                               int max_running, bool one_at_a_time,
                               std::vector<int> *states = nullptr,
                               std::vector<int> *statuses = nullptr) {
  const int nf = 8;
  std::vector<double> om(nf), wt(nf);
  ssrpa_frequency_grid(nf, 1.0, om.data(), wt.data());
  ssrpa_server *srv = nullptr;
  CHECK(ssrpa_server_create(ctx, max_running, 0.5, &srv) == SSRPA_OK);
  std::vector<uint64_t> ids;
  for (size_t i = 0; i < sys.size(); ++i) {
    uint64_t id = 0;
    CHECK(ssrpa_server_submit(srv, &sys[i].d, 3 + (int)i, nf, om.data(),
                              wt.data(), i % 2 ? SSRPA_BF16X3 : SSRPA_FP64,
                              &id) == SSRPA_OK);
    ids.push_back(id);
    if (one_at_a_time) CHECK(ssrpa_server_drain(srv) == SSRPA_OK);
  }
  CHECK(ssrpa_server_drain(srv) == SSRPA_OK);
  std::vector<double> ec;
  for (auto id : ids) {
    int st = -1;
    ssrpa_status status = SSRPA_OK;
    double e = 0.0, t0, t1, t2, d0 = -1, d1 = -1;
    CHECK(ssrpa_server_poll(srv, id, &st, &status, &e, &t0, &t1, &t2) == SSRPA_OK);
    CHECK(ssrpa_server_device_times(srv, id, &d0, &d1) == SSRPA_OK);
    CHECK(d0 >= 0.0 && d1 >= d0);
    if (states) states->push_back(st);
    if (statuses) statuses->push_back((int)status);
    ec.push_back(e);
  }
  CHECK(ssrpa_server_destroy(srv) == SSRPA_OK);
  return ec;
}

}  // namespace

int main(int argc, char **argv) {
  const int rounds = argc > 1 ? std::atoi(argv[1]) : 4;
  ssrpa_context *ctx = nullptr;
  CHECK(ssrpa_context_create(0, size_t(2) << 30, &ctx) == SSRPA_OK);
  std::vector<Sys> sys;
  const int shapes[6][2] = {{4, 28}, {6, 40}, {3, 21}, {8, 56}, {5, 37}, {2, 30}};
  for (int i = 0; i < 6; ++i) sys.push_back(make_sys(shapes[i][0], shapes[i][1], 900 + i));
  for (int r = 0; r < rounds; ++r) {
    // 1. alone vs mixed
    const auto alone = run_stream(ctx, sys, 1, true);
    const auto mixed = run_stream(ctx, sys, 4, false);
    for (size_t i = 0; i < sys.size(); ++i) {
      CHECK(alone[i] == mixed[i]);
      CHECK(alone[i] < 0.0);
    }
    // 2. failures while other requests run
    g_fail_herk_every.store(3);
    std::vector<int> states, statuses;
    run_stream(ctx, sys, 3, false, &states, &statuses);
    g_fail_herk_every.store(0);
    int failed = 0, done = 0;
    for (size_t i = 0; i < states.size(); ++i) {
      if (states[i] == SSRPA_REQ_FAILED) {
        ++failed;
        CHECK(statuses[i] == SSRPA_ERR_NOMEM);
      } else {
        CHECK(states[i] == SSRPA_REQ_DONE);
        ++done;
      }
    }
    CHECK(failed > 0 && done > 0);
    // 3. a repeated plane wave is refused on the host
    Sys bad = make_sys(2, 5, 7);
    bad.miller[3] = bad.miller[0];
    bad.miller[4] = bad.miller[1];
    bad.miller[5] = bad.miller[2];
    ssrpa_system *s = nullptr;
    CHECK(ssrpa_system_create(ctx, &bad.d, nullptr, &s) == SSRPA_ERR_ARG);
    CHECK(s == nullptr);
    std::printf("round %d: alone == mixed for %zu requests; %d failed, %d done "
                "under injected failures\n", r, sys.size(), failed, done);
    std::fflush(stdout);
  }
  size_t in_use = 0, hw = 0;
  CHECK(ssrpa_context_memory(ctx, &in_use, &hw) == SSRPA_OK);
  CHECK(ssrpa_context_destroy(ctx) == SSRPA_OK);
  std::printf("%s\n", failures ? "FAILED" : "OK");
  return failures ? 1 : 0;
}
