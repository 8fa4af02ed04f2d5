// Host-side checks of the C ABI's argument validation and of the serving scheduler's pool
// allocator, meant to be built with the address and undefined-behaviour sanitizers on every host
// translation unit of the library.  No GPU is needed: every ABI call made here returns before it
// reaches a device.  Prints one line per group of checks and exits non-zero on the first failed
// group.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <utility>
#include <vector>

#include "crypto_serve.h"
#include "finrl_mi.h"
#include "learner.h"
#include "pool_alloc.h"

static int g_failures = 0;
#define CHECK(c)                                                                      \
  do {                                                                                \
    if (!(c)) {                                                                       \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c);     \
      ++g_failures;                                                                   \
    }                                                                                 \
  } while (0)

// The allocator against a byte-map model: first fit (lowest offset of a free run long enough),
// no overlap, and everything coalesced back into one range at the end.
static void pool_against_model(unsigned seed) {
  const size_t unit = 256, units = 512, size = unit * units;
  fm::cx::PoolAlloc pool;
  pool.reset(size);
  std::vector<char> used(units, 0);
  std::vector<std::pair<size_t, size_t>> live;
  std::mt19937 rng(seed);
  for (int op = 0; op < 20000; ++op) {
    if (live.empty() || rng() % 100 < 55) {
      const size_t n = 1 + rng() % 32;  // in units
      size_t want = units;
      for (size_t s = 0; s + n <= units && want == units; ++s) {
        size_t k = 0;
        while (k < n && !used[s + k]) ++k;
        if (k == n) want = s;
      }
      size_t off = 0;
      const bool ok = pool.alloc(n * unit, &off);
      CHECK(ok == (want != units));
      if (!ok) continue;
      CHECK(off == want * unit);
      if (off != want * unit) return;
      for (size_t k = 0; k < n; ++k) used[want + k] = 1;
      live.emplace_back(off, n * unit);
    } else {
      const size_t i = rng() % live.size();
      pool.release(live[i].first, live[i].second);
      for (size_t k = 0; k < live[i].second / unit; ++k) used[live[i].first / unit + k] = 0;
      live[i] = live.back();
      live.pop_back();
    }
  }
  for (const auto& r : live) pool.release(r.first, r.second);
  size_t off = 1;
  CHECK(pool.alloc(size, &off) && off == 0);  // one coalesced range
  CHECK(!pool.alloc(unit, &off));             // and nothing left
}

static fm_env_config tiny_config() {
  fm_env_config c;
  std::memset(&c, 0, sizeof(c));
  c.n_envs = 16;
  c.n_stocks = 30;
  c.n_ind = 5;
  c.n_days = 30;
  c.hmax = 100;
  c.init_cash = 1e6;
  c.cost_rate = 1e-3;
  c.reward_scale = std::ldexp(1.0, -12);
  c.cash_obs_scale = std::ldexp(1.0f, -20);
  c.price_obs_scale = std::ldexp(1.0f, -8);
  c.hold_obs_scale = std::ldexp(1.0f, -10);
  return c;
}

static void env_validation() {
  fm_env_config c = tiny_config();
  CHECK(env_workspace_bytes(&c) > 0 && env_workspace_bytes(&c) % 256 == 0);
  CHECK(env_workspace_bytes(nullptr) == 0);
  fm_env_config bad = c;
  bad.n_stocks = 0;
  CHECK(env_workspace_bytes(&bad) == 0);
  bad = c;
  bad.cost_rate = 1.0;
  CHECK(env_workspace_bytes(&bad) == 0);
  bad = c;
  bad.reward_scale = std::nan("");
  CHECK(env_workspace_bytes(&bad) == 0);
  fm_env* env = reinterpret_cast<fm_env*>(0x1);
  CHECK(env_create(&c, nullptr, nullptr, nullptr, 0, nullptr, &env) == FM_ERR_INVALID && env == nullptr);
  CHECK(std::strstr(fm_last_error(), "NULL") != nullptr);
  float* const fake = reinterpret_cast<float*>(256);
  CHECK(env_create(&c, fake, fake, reinterpret_cast<void*>(1028), size_t{1} << 30, nullptr, &env) == FM_ERR_INVALID);
  CHECK(std::strstr(fm_last_error(), "aligned") != nullptr);
  CHECK(env_create(&c, fake, fake, reinterpret_cast<void*>(1024), 16, nullptr, &env) == FM_ERR_INVALID);
  CHECK(std::strstr(fm_last_error(), "small") != nullptr);
  CHECK(env_reset(nullptr, nullptr) == FM_ERR_INVALID);
  CHECK(env_step(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == FM_ERR_INVALID);
  CHECK(env_rollout(nullptr, nullptr, 1, nullptr) == FM_ERR_INVALID);
  CHECK(env_day(nullptr) == -1);
  CHECK(env_set_tile(nullptr, 8, nullptr) == FM_ERR_INVALID);
  CHECK(env_set_fused_tuning(nullptr, 0, 0, 0) == FM_ERR_INVALID);
  CHECK(env_read_state(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == FM_ERR_INVALID);
  CHECK(env_write_state(nullptr, nullptr, nullptr, nullptr, nullptr, 0) == FM_ERR_INVALID);
  env_destroy(nullptr);
}

static void ensemble_validation() {
  CHECK(ensemble_workspace_bytes(3, 211, 256, 30, FM_BF16, 2048) > 0);
  CHECK(ensemble_workspace_bytes(0, 211, 256, 30, FM_F32, 1) == 0);
  CHECK(ensemble_workspace_bytes(3, 211, 250, 30, FM_F32, 1) == 0);
  CHECK(ensemble_workspace_bytes(3, 211, 256, 30, 2, 1) == 0);
  fm_ensemble* e = nullptr;
  CHECK(ensemble_create(3, 211, 100, 30, FM_F32, reinterpret_cast<float*>(256), nullptr, 16,
                        reinterpret_cast<void*>(1024), size_t{1} << 30, nullptr, &e) == FM_ERR_INVALID);
  CHECK(std::strstr(fm_last_error(), "hidden") != nullptr);
  CHECK(ensemble_act(nullptr, nullptr, 1, 0.0f, 0, 0, 0, nullptr, nullptr, nullptr) == FM_ERR_INVALID);
  ensemble_destroy(nullptr);
}

static void sharpe_weights() {
  const double s[4] = {1.0, 0.5, -0.2, 2.0};
  float w[4] = {0, 0, 0, 0};
  CHECK(fm_sharpe_weights(s, 4, 0.0, w) == FM_OK);
  CHECK(w[2] == 0.0f && w[3] > w[0] && w[0] > w[1]);
  CHECK(std::fabs(w[0] + w[1] + w[3] - 1.0f) < 1e-6f);
  const double low[3] = {-3.0, -1.0, -2.0};
  CHECK(fm_sharpe_weights(low, 3, 0.0, w) == FM_OK && w[1] == 1.0f && w[0] == 0.0f && w[2] == 0.0f);
  const double nan2[2] = {std::nan(""), 1.0};
  CHECK(fm_sharpe_weights(nan2, 2, 0.0, w) == FM_ERR_INVALID);
  CHECK(fm_sharpe_weights(nullptr, 2, 0.0, w) == FM_ERR_INVALID);
}

static void batch_and_learner_validation() {
  CHECK(fm_batch_workspace_bytes(nullptr, 0) == 0);
  fm_batch_group g;
  std::memset(&g, 0, sizeof(g));
  CHECK(fm_batch_workspace_bytes(&g, 1) == 0);
  fm_batch* b = nullptr;
  CHECK(fm_batch_create(nullptr, 1, reinterpret_cast<void*>(256), 1 << 20, nullptr, &b) == FM_ERR_INVALID);
  CHECK(fm_batch_tune(nullptr, nullptr, nullptr) == FM_ERR_INVALID);
  CHECK(fm_batch_set_tiling(nullptr, 16, 256) == FM_ERR_INVALID);
  CHECK(fm_batch_run(nullptr, 0) == FM_ERR_INVALID);
  fm_batch_destroy(nullptr);
  CHECK(fm_pg_workspace_bytes(3, 211, 256, 30, 2048, 252) > 0);
  CHECK(fm_pg_workspace_bytes(9, 211, 256, 30, 2048, 252) == 0);
  CHECK(fm_pg_workspace_bytes(3, 211, 2048, 30, 16, 4) == 0);
  CHECK(fm_policy_gradient(3, 211, 256, 30, nullptr, nullptr, 0, nullptr, nullptr, 16, 4, 0.1f, 1, 0, 0, 0.0f,
                           nullptr, nullptr, 0, nullptr) == FM_ERR_INVALID);
  CHECK(fm_noise(7, 0, 4, 0, 30, nullptr, nullptr, nullptr) == FM_ERR_INVALID);
}

static void serve_validation() {
  fm_serve_config c;
  std::memset(&c, 0, sizeof(c));
  CHECK(fm_serve_workspace_bytes(&c) == 0);  // NULL tick table
  std::vector<float> w(5 * (16 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3), 0.0f);
  c.d_mid = reinterpret_cast<const double*>(256);
  c.d_feat = reinterpret_cast<const float*>(256);
  c.n_ticks = 1000;
  c.n_agents = 5;
  c.h_weights = w.data();
  c.rule = 0;
  c.eps = 0.0f;
  c.fee = 2e-4;
  c.cash0 = 1e5;
  c.tile_rows = 64;
  c.chunk_ticks = 256;
  c.max_requests = 16;
  c.max_active_envs = 4096;
  c.d_pool = reinterpret_cast<void*>(256);
  c.pool_bytes = 1 << 20;
  CHECK(fm_serve_workspace_bytes(&c) > 5 * 32 * 1024);
  fm_serve_config bad = c;
  bad.tile_rows = 32;
  CHECK(fm_serve_workspace_bytes(&bad) == 0);
  fm_serve* s = nullptr;
  CHECK(fm_serve_create(&bad, nullptr, &s) == FM_ERR_INVALID && s == nullptr);
  bad = c;
  bad.eps = 1.5f;
  CHECK(fm_serve_workspace_bytes(&bad) == 0);
  CHECK(fm_serve_request_bytes(0) == 0 && fm_serve_request_bytes(100) == 6400);
  int32_t n = 0;
  CHECK(fm_serve_poll(nullptr, 0, nullptr, 0, &n) == FM_ERR_INVALID);
  CHECK(fm_serve_step(nullptr, nullptr, nullptr, nullptr) == FM_ERR_INVALID);
  fm_serve_destroy(nullptr);
}

int main() {
  struct Group {
    const char* name;
    void (*fn)();
  };
  const Group groups[] = {
      {"pool allocator against a byte-map model", [] {
         for (unsigned seed = 1; seed <= 4; ++seed) pool_against_model(seed);
       }},
      {"environment argument validation", env_validation},
      {"ensemble argument validation", ensemble_validation},
      {"softmax-of-Sharpe weights", sharpe_weights},
      {"batch, learner and noise argument validation", batch_and_learner_validation},
      {"serving argument validation", serve_validation},
  };
  for (const Group& g : groups) {
    const int before = g_failures;
    g.fn();
    std::printf("%s: %s\n", g.name, g_failures == before ? "ok" : "FAILED");
    std::fflush(stdout);
    if (g_failures != before) return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
