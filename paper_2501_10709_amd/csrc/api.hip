// The C ABI (include/finrl_mi.h): argument validation, workspace layout, handles and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <algorithm>

#include "../../include/finrl_mi.h"
#include "fused.h"
#include "launch.h"
#include "status.h"

namespace {

thread_local std::string g_last_error;

fm_status fail(fm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

fm_status device_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return FM_OK;
  return fail(FM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

// Environments per workgroup of the environment kernels by problem size (measured on MI355X,
// D = 30, driven rollouts): tiles of 8 spread the serial trading chains over every compute unit
// while the grid does not fill the GPU, and from 8192 environments the kernel runs them three to
// a compute unit; from 16384, tiles of 16, also three to a compute unit (the per-step cost of a
// workgroup grows much slower than its tile).  The tile is capped by the kernel's LDS budget.
int env_tile(int N) {
  if (N >= 16384) return 16;
  return 8;
}

struct EnvLayout {
  size_t cash, asset, cumrew, hold, act, obs, eps, mt, total;
};

EnvLayout env_layout(const fm_env_config& c) {
  const int S = (c.n_ind + 2) * c.n_stocks + 1;
  EnvLayout L{};
  size_t off = 0;
  L.cash = off;
  off = align_up(off + sizeof(double) * c.n_envs);
  L.asset = off;
  off = align_up(off + sizeof(double) * c.n_envs);
  L.cumrew = off;
  off = align_up(off + sizeof(double) * c.n_envs);
  L.hold = off;
  off = align_up(off + sizeof(int32_t) * static_cast<size_t>(c.n_stocks) * c.n_envs);
  L.act = off;
  off = align_up(off + sizeof(float) * static_cast<size_t>(c.n_stocks) * c.n_envs);
  L.obs = off;
  off = align_up(off + sizeof(float) * static_cast<size_t>(S) * c.n_envs);
  // Scratch of the fused rollout's streamed schedule (noise and market table of a chunk).
  L.eps = off;
  off = align_up(off + sizeof(float) * fm::fused_eps_floats(c.n_envs, c.n_stocks));
  L.mt = off;
  off = align_up(off + sizeof(float) * fm::fused_table_floats());
  L.total = off;
  return L;
}

std::string validate_config(const fm_env_config* c) {
  if (!c) return "config is NULL";
  if (c->n_envs < 1 || c->n_envs > (1 << 24)) return "n_envs must be in 1..2^24";
  if (c->n_stocks < 1 || c->n_stocks > 128) return "n_stocks must be in 1..128";
  if (c->n_ind < 0 || c->n_ind > 16) return "n_ind must be in 0..16";
  if (c->n_days < 1 || c->n_days > (1 << 20)) return "n_days must be in 1..2^20";
  if (c->hmax < 1 || c->hmax > (1 << 20)) return "hmax must be in 1..2^20";
  if (!(c->init_cash >= 0.0) || !std::isfinite(c->init_cash)) return "init_cash must be finite and >= 0";
  if (!(c->cost_rate >= 0.0 && c->cost_rate < 1.0)) return "cost_rate must be in [0, 1)";
  if (!std::isfinite(c->reward_scale)) return "reward_scale must be finite";
  if (!std::isfinite(c->cash_obs_scale) || !std::isfinite(c->price_obs_scale) ||
      !std::isfinite(c->hold_obs_scale))
    return "state scales must be finite";
  const size_t S = static_cast<size_t>(c->n_ind + 2) * c->n_stocks + 1;
  if (S * static_cast<size_t>(c->n_envs) * c->n_days > (static_cast<size_t>(1) << 46))
    return "trajectory too large";
  return "";
}

using fm::DeviceGuard;

}  // namespace

namespace fm {
fm_status set_error(fm_status s, const std::string& msg) { return fail(s, msg); }
fm_status device_error(hipError_t e, const char* what) { return device_status(e, what); }
}  // namespace fm

struct fm_env {
  fm_env_config cfg;
  fm::EnvConst C;
  fm::EnvState st;
  float* act_stage;
  float* obs_stage;
  float* eps_chunk;
  float* mt_chunk;
  hipStream_t stream;
  int device;
  int day;
  int tile;
  int step_kernel;    // 0 by shape and size, 1 the tile kernel, 2 the lane kernel, 3 the row kernel
  int lane_envs;      // environments per wavefront of the lane kernel (0: by N)
  fm::FusedTuning fused;  // fused-rollout tuning (schedule, row tiles, environments per workgroup)
};

struct fm_ensemble {
  int K, S, H, A, dtype, max_batch, device;
  fm::EnsDev E;
  float* mu;  // [K][max_batch][A]
};

namespace {

struct EnsLayout {
  int S_pad, A_pad, split_a, ke_pad;
  size_t w1, w2, w3, b1, b2, b3, actor, mix, mu, w1e, w1m, total;
};

// The split first layer applies to bfloat16 ensembles over a trading state
// [cash, closes(A), holdings(A), indicators(I*A)].
bool splits_first_layer(int S, int A, int dtype) {
  return dtype == FM_BF16 && A >= 1 && (S - 1) % A == 0 && (S - 1) / A >= 2 && 1 + A <= 128;
}

EnsLayout ens_layout(int K, int S, int H, int A, int dtype, int max_batch) {
  EnsLayout L{};
  const int kg = dtype == FM_F32 ? 16 : 32;
  const size_t es = dtype == FM_F32 ? 4 : 2;
  L.S_pad = fm::round_up(S, kg);
  L.A_pad = fm::round_up(A, 16);
  size_t off = 0;
  L.w1 = off;
  off = align_up(off + es * L.S_pad * H);
  L.w2 = off;
  off = align_up(off + es * static_cast<size_t>(H) * H);
  L.w3 = off;
  off = align_up(off + es * static_cast<size_t>(H) * L.A_pad);
  L.b1 = off;
  off = align_up(off + 4 * H);
  L.b2 = off;
  off = align_up(off + 4 * H);
  L.b3 = off;
  off = align_up(off + 4 * L.A_pad);
  L.actor = off;
  L.mix = L.actor * K;
  L.mu = align_up(L.mix + 4 * 8);
  off = align_up(L.mu + sizeof(float) * static_cast<size_t>(K) * max_batch * A);
  if (splits_first_layer(S, A, dtype)) {
    L.split_a = A;
    L.ke_pad = fm::round_up(1 + A, 32);
    L.w1e = off;
    off = align_up(off + 2 * static_cast<size_t>(K) * H * L.ke_pad);
    L.w1m = off;
    off = align_up(off + 2 * static_cast<size_t>(K) * (S - 1 - A) * H);
  }
  L.total = off;
  return L;
}

std::string validate_ensemble(int K, int S, int H, int A, int dtype, int max_batch) {
  if (K < 1 || K > 8) return "n_actors must be in 1..8";
  if (S < 1 || S > 1024) return "in_dim must be in 1..1024";
  if (H < 32 || H > 512 || H % 32 != 0) return "hidden must be a multiple of 32 in 32..512";
  if (A < 1 || A > 128) return "out_dim must be in 1..128";
  if (dtype != FM_F32 && dtype != FM_BF16) return "dtype must be FM_F32 or FM_BF16";
  if (max_batch < 1 || max_batch > (1 << 24)) return "max_batch must be in 1..2^24";
  return "";
}

}  // namespace

extern "C" {

const char* fm_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------------------------------
// Uneven batch
// ------------------------------------------------------------------------------------------
}  // extern "C"

struct fm_batch {
  int n_groups = 0, device = 0, n_chunks = 0, rows = 16, blocks = 0;
  hipStream_t stream = nullptr;
  std::vector<fm_batch_group> groups;
  std::vector<int> start_day;
  size_t desc_bytes = 0, lds = 0, items_cap = 0;
  unsigned char* d_desc = nullptr;  // [n_chunks][n_groups] descriptors
  int* d_items = nullptr;           // [n_chunks][items_cap] int2
  int* d_counter = nullptr;
  unsigned char* d_save = nullptr;  // state copies for the autotuner
  std::vector<float*> d_mt;         // per group: its chunk's market table (split first layer), or null
  std::vector<int> n_items;         // per chunk, for the current rows: all work items
  std::vector<int> n_wide;          // per chunk: the first n_wide items run 32-row tiles
  size_t lds_wide = 0;              // dynamic LDS of the 32-row and 16-row launches
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;  // private stream the chunk launches are captured on
};

namespace {

constexpr int kBatchChunk = 64;

struct BatchLayout {
  size_t desc, items, counter, save, mt, total, items_cap;
  int n_chunks;
};

// Floats of a group's market-table slot: the chunk's days x actors x hidden units.
size_t batch_table_floats(const fm_batch_group& g) {
  const fm::EnsDev& E = g.ens->E;
  return E.split_a > 0 ? static_cast<size_t>(kBatchChunk) * E.K * E.H : 0;
}

std::string validate_batch(const fm_batch_group* g, int n, int device) {
  if (!g) return "groups is NULL";
  if (n < 1 || n > 4096) return "n_groups must be in 1..4096";
  for (int i = 0; i < n; ++i) {
    const fm_batch_group& b = g[i];
    const std::string at = " (group " + std::to_string(i) + ")";
    if (!b.env || !b.ens) return "env and ensemble are required" + at;
    if (b.ens->dtype != FM_BF16) return "the batch runs bfloat16 ensembles" + at;
    if (b.ens->S != b.env->C.S || b.ens->A != b.env->C.D) return "ensemble in_dim/out_dim do not match" + at;
    if (b.ens->H > 256) return "hidden must be <= 256" + at;
    if (b.env->device != device || b.ens->device != device) return "all groups must be on the current device" + at;
    if (b.n_steps < 0 || b.env->day + b.n_steps > b.env->C.T) return "n_steps out of range" + at;
    if (!(b.sigma >= 0.0f) || !std::isfinite(b.sigma)) return "sigma must be finite and >= 0" + at;
    if (fm::batched_lds_bytes(16, b.env->C, b.ens->E) > fm::batched_max_lds()) return "state too wide for the LDS budget" + at;
  }
  return "";
}

BatchLayout batch_layout(const fm_batch_group* g, int n) {
  BatchLayout L{};
  int max_steps = 0;
  size_t items = 0, save = 0;
  for (int i = 0; i < n; ++i) {
    max_steps = std::max(max_steps, g[i].n_steps);
    items += static_cast<size_t>((g[i].env->C.N + 15) / 16);
    save += align_up(sizeof(double) * 3 * g[i].env->C.N) +
            align_up(sizeof(int32_t) * static_cast<size_t>(g[i].env->C.D) * g[i].env->C.N);
  }
  L.n_chunks = std::max(1, (max_steps + kBatchChunk - 1) / kBatchChunk);
  L.items_cap = items;
  size_t off = 0;
  L.desc = off;
  off = align_up(off + fm::batched_group_desc_bytes() * n * L.n_chunks);
  L.items = off;
  off = align_up(off + sizeof(int) * 2 * items * L.n_chunks);
  L.counter = off;
  off = align_up(off + 256);
  L.save = off;
  off = align_up(off + save);
  L.mt = off;
  for (int i = 0; i < n; ++i) off = align_up(off + sizeof(float) * batch_table_floats(g[i]));
  L.total = off;
  return L;
}

// A group's tile rows for the batch's rows setting: 32 when its 32-row tile fits the LDS budget.
int group_rows(const fm_batch_group& G, int rows) {
  return rows == 32 && fm::batched_lds_bytes(32, G.env->C, G.ens->E) <= fm::batched_max_lds() ? 32 : 16;
}

// Work lists of every chunk for the given tile rows: (group, tile), the 32-row items first, each
// part most expensive first.
fm_status batch_items(fm_batch* b, int rows) {
  std::vector<int> host;
  b->n_items.assign(b->n_chunks, 0);
  b->n_wide.assign(b->n_chunks, 0);
  for (int c = 0; c < b->n_chunks; ++c) {
    struct It { double cost; int g, tile, wide; };
    std::vector<It> list;
    for (int g = 0; g < b->n_groups; ++g) {
      const fm_batch_group& G = b->groups[g];
      const int n = std::min(kBatchChunk, G.n_steps - c * kBatchChunk);
      if (n <= 0) continue;
      const fm::EnsDev& E = G.ens->E;
      const int kin1 = E.split_a > 0 ? E.ke_pad : E.S_pad;
      const double per_step = static_cast<double>(E.K) *
                              (static_cast<double>(kin1) * E.H + static_cast<double>(E.H) * E.H +
                               static_cast<double>(E.H) * E.A_pad) + 64.0 * G.env->C.D;
      const int gr = group_rows(G, rows);
      const int tiles = (G.env->C.N + gr - 1) / gr;
      for (int t = 0; t < tiles; ++t) list.push_back({per_step * n * gr, g, t, gr == 32 ? 1 : 0});
    }
    std::stable_sort(list.begin(), list.end(),
                     [](const It& x, const It& y) { return x.wide != y.wide ? x.wide > y.wide : x.cost > y.cost; });
    b->n_items[c] = static_cast<int>(list.size());
    for (const It& it : list) b->n_wide[c] += it.wide;
    host.resize(2 * b->items_cap);
    for (size_t i = 0; i < list.size(); ++i) {
      host[2 * i] = list[i].g;
      host[2 * i + 1] = list[i].tile;
    }
    hipError_t e = hipMemcpyAsync(b->d_items + 2 * b->items_cap * c, host.data(), sizeof(int) * 2 * list.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return device_status(e, "fm_batch (work lists)");
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return device_status(e, "fm_batch (work lists)");
  }
  b->rows = rows;
  size_t lds = 0, lds_wide = 0;
  for (const fm_batch_group& G : b->groups) {
    const int gr = group_rows(G, rows);
    size_t& l = gr == 32 ? lds_wide : lds;
    l = std::max(l, fm::batched_lds_bytes(gr, G.env->C, G.ens->E));
  }
  b->lds = lds;
  b->lds_wide = lds_wide;
  return device_status(fm::prepare_batched(std::max(lds, lds_wide)), "fm_batch (LDS limit)");
}

void batch_drop_graph(fm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

hipError_t batch_enqueue(fm_batch* b, int n_chunks, hipStream_t stream) {
  for (int c = 0; c < n_chunks; ++c) {
    if (b->n_items[c] == 0) continue;
    // The chunk's market tables of the groups that split their first layer.
    for (int g = 0; g < b->n_groups; ++g) {
      const fm_batch_group& G = b->groups[g];
      const int n = std::min(kBatchChunk, G.n_steps - c * kBatchChunk);
      if (n <= 0 || !b->d_mt[g]) continue;
      const hipError_t e = fm::launch_market_table(G.env->C, G.ens->E, b->start_day[g] + c * kBatchChunk, n,
                                                   b->d_mt[g], stream);
      if (e != hipSuccess) return e;
    }
    // The 32-row items, then the 16-row ones: one persistent launch each, with its own counter.
    const unsigned char* desc = b->d_desc + b->desc_bytes * b->n_groups * c;
    const int* items = b->d_items + 2 * b->items_cap * c;
    const int nw = b->n_wide[c], nn = b->n_items[c] - nw;
    hipError_t e = hipSuccess;
    if (nw > 0) e = fm::launch_batched(32, b->blocks, b->lds_wide, desc, items, nw, b->d_counter, stream);
    if (e == hipSuccess && nn > 0)
      e = fm::launch_batched(16, b->blocks, b->lds, desc, items + 2 * nw, nn, b->d_counter + 1, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Copies every group's trading state to (save) or from (restore) the batch's save area.
hipError_t batch_state_copy(fm_batch* b, bool save) {
  unsigned char* p = b->d_save;
  for (const fm_batch_group& G : b->groups) {
    const size_t N = G.env->C.N, D = G.env->C.D;
    const size_t nd = align_up(sizeof(double) * 3 * N), nh = sizeof(int32_t) * D * N;
    const fm::EnvState& st = G.env->st;
    void* src[4] = {st.cash, st.asset, st.cumrew, st.hold};
    const size_t sz[4] = {sizeof(double) * N, sizeof(double) * N, sizeof(double) * N, nh};
    size_t off[4] = {0, sizeof(double) * N, 2 * sizeof(double) * N, nd};
    for (int k = 0; k < 4; ++k) {
      const hipError_t e = save ? hipMemcpyAsync(p + off[k], src[k], sz[k], hipMemcpyDeviceToDevice, b->stream)
                                : hipMemcpyAsync(src[k], p + off[k], sz[k], hipMemcpyDeviceToDevice, b->stream);
      if (e != hipSuccess) return e;
    }
    p += nd + align_up(nh);
  }
  return hipSuccess;
}

// Default environment-step kernels by batch size (measured on MI355X, D = 30): up to
// kRowMaxEnvs environments the row kernel (a 16-lane row per environment) has the shortest
// per-step latency, since its cash chain is split over the row's lanes; from kLaneMinEnvs the lane
// kernel (one lane per environment) holds enough environments per SIMD to hide its chains'
// instruction stream and streams the state rows at the HBM rate; between them the tile kernel.
constexpr int kRowMaxEnvs = 12288;
constexpr int kLaneMinEnvs = 24576;

bool row_kernel(const fm_env* env) {
  if (!fm::env_lane_shape(env->C)) return false;
  return env->step_kernel == 3 || (env->step_kernel == 0 && env->C.N <= kRowMaxEnvs);
}

bool lane_kernel(const fm_env* env) {
  if (env->step_kernel == 1 || env->step_kernel == 3 || !fm::env_lane_shape(env->C)) return false;
  return env->step_kernel == 2 || env->C.N >= kLaneMinEnvs;
}

// The plain path's one-step launches (ensemble means, noise and clip, then the trade): the row
// kernel up to kRowMaxEnvs environments (at most 8 actors), else the lane kernel at every size its
// shape allows; both fetch the actors' means and the market rows under the noise generation, and
// beat the tile kernel on MI355X from 1024 to 65536 environments (D = 30, K = 3).
bool row_kernel_means(const fm_env* env, int K) { return K <= 8 && row_kernel(env); }

// Environments per wavefront of the row kernel: the caller's choice (env_set_step_kernel), else 2.
int row_envs(const fm_env* env) { return env->lane_envs == 1 || env->lane_envs == 2 ? env->lane_envs : 2; }

bool lane_kernel_means(const fm_env* env) {
  return (env->step_kernel == 0 || env->step_kernel == 2) && fm::env_lane_shape(env->C);
}

// The caller's actions over n_steps days from day t0, by the chosen environment-step kernel.
hipError_t launch_given(const fm_env* env, int t0, int n_steps, const float* act, float* obs, double* rew,
                        int* qty, hipStream_t stream) {
  if (row_kernel(env))
    return fm::launch_env_row_given(env->C, env->st, t0, n_steps, act, obs, rew, qty, row_envs(env), stream);
  if (lane_kernel(env))
    return fm::launch_env_lane_given(env->C, env->st, t0, n_steps, act, obs, rew, qty, env->lane_envs, stream);
  return fm::launch_env_given(env->C, env->st, t0, n_steps, act, obs, rew, qty, env->tile, stream);
}

}  // namespace

extern "C" {

size_t fm_batch_workspace_bytes(const fm_batch_group* h_groups, int32_t n_groups) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (!validate_batch(h_groups, n_groups, dev).empty()) return 0;
  return batch_layout(h_groups, n_groups).total;
}

fm_status fm_batch_create(const fm_batch_group* h_groups, int32_t n_groups, void* d_workspace,
                          size_t workspace_bytes, hipStream_t stream, fm_batch** out) {
  if (!out) return fail(FM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const std::string why = validate_batch(h_groups, n_groups, dev);
  if (!why.empty()) return fail(FM_ERR_INVALID, why);
  if (!d_workspace) return fail(FM_ERR_INVALID, "d_workspace is NULL");
  if (!aligned(d_workspace)) return fail(FM_ERR_INVALID, "d_workspace must be 256-byte aligned");
  const BatchLayout L = batch_layout(h_groups, n_groups);
  if (workspace_bytes < L.total) return fail(FM_ERR_INVALID, "workspace too small");
  fm_batch* b = new (std::nothrow) fm_batch();
  if (!b) return fail(FM_ERR_DEVICE, "host allocation failed");
  unsigned char* base = static_cast<unsigned char*>(d_workspace);
  b->n_groups = n_groups;
  b->device = dev;
  b->stream = stream;
  b->groups.assign(h_groups, h_groups + n_groups);
  b->n_chunks = L.n_chunks;
  b->items_cap = L.items_cap;
  b->desc_bytes = fm::batched_group_desc_bytes();
  b->d_desc = base + L.desc;
  b->d_items = reinterpret_cast<int*>(base + L.items);
  b->d_counter = reinterpret_cast<int*>(base + L.counter);
  b->d_save = base + L.save;
  {
    size_t off = L.mt;
    for (int g = 0; g < n_groups; ++g) {
      const size_t f = batch_table_floats(h_groups[g]);
      b->d_mt.push_back(f > 0 ? reinterpret_cast<float*>(base + off) : nullptr);
      off = align_up(off + sizeof(float) * f);
    }
  }
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  b->blocks = cus;
  // Descriptors of every (chunk, group): the chunk's first day, its steps and trajectory rows.
  std::vector<unsigned char> host(b->desc_bytes * n_groups * L.n_chunks);
  for (int c = 0; c < L.n_chunks; ++c)
    for (int g = 0; g < n_groups; ++g) {
      const fm_batch_group& G = h_groups[g];
      const fm::EnvConst& C = G.env->C;
      const int n = std::max(0, std::min(kBatchChunk, G.n_steps - c * kBatchChunk));
      const size_t r0 = static_cast<size_t>(c) * kBatchChunk;
      const size_t N = C.N, D = C.D, S = C.S;
      fm::batched_group_desc(C, G.env->st, G.ens->E, G.env->day + c * kBatchChunk, n, G.sigma, G.noise_key,
                             G.env_offset, G.d_obs_traj && n ? G.d_obs_traj + r0 * N * S : nullptr,
                             G.d_act_traj && n ? G.d_act_traj + r0 * N * D : nullptr,
                             G.d_rew_traj && n ? G.d_rew_traj + r0 * N : nullptr,
                             G.d_qty_traj && n ? G.d_qty_traj + r0 * N * D : nullptr, b->d_mt[g],
                             host.data() + b->desc_bytes * (static_cast<size_t>(c) * n_groups + g));
    }
  for (int g = 0; g < n_groups; ++g) b->start_day.push_back(h_groups[g].env->day);
  DeviceGuard guard(dev);
  hipError_t e = hipMemcpyAsync(b->d_desc, host.data(), host.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    delete b;
    return device_status(e, "fm_batch_create");
  }
  const fm_status s = batch_items(b, 16);
  if (s != FM_OK) {
    delete b;
    return s;
  }
  *out = b;
  return FM_OK;
}

fm_status fm_batch_tune(fm_batch* b, int32_t* h_rows, int32_t* h_blocks) {
  if (!b) return fail(FM_ERR_INVALID, "batch is NULL");
  DeviceGuard guard(b->device);
  batch_drop_graph(b);
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) cus = 256;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(FM_ERR_DEVICE, "fm_batch_tune: event creation failed");
  int best_rows = b->rows, best_blocks = b->blocks;
  float best_ms = -1.0f;
  fm_status status = FM_OK;
  for (int rows : {16, 32}) {
    status = batch_items(b, rows);
    if (status != FM_OK) break;
    for (int blocks : {cus / 2, cus, 2 * cus}) {
      b->blocks = blocks;
      hipError_t e = batch_state_copy(b, true);
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = batch_enqueue(b, 1, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = batch_state_copy(b, false);
      }
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
      if (e != hipSuccess) {
        status = device_status(e, "fm_batch_tune");
        break;
      }
      if (best_ms < 0.0f || ms < best_ms) {
        best_ms = ms;
        best_rows = rows;
        best_blocks = blocks;
      }
    }
    if (status != FM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != FM_OK) return status;
  b->blocks = best_blocks;
  status = batch_items(b, best_rows);
  if (status != FM_OK) return status;
  if (h_rows) *h_rows = b->rows;
  if (h_blocks) *h_blocks = b->blocks;
  return FM_OK;
}

fm_status fm_batch_set_tiling(fm_batch* b, int32_t rows, int32_t blocks) {
  if (!b) return fail(FM_ERR_INVALID, "batch is NULL");
  if (rows != 16 && rows != 32) return fail(FM_ERR_INVALID, "fm_batch_set_tiling: rows must be 16 or 32");
  if (blocks < 1 || blocks > 65536) return fail(FM_ERR_INVALID, "fm_batch_set_tiling: blocks must be in 1..65536");
  DeviceGuard guard(b->device);
  batch_drop_graph(b);
  b->blocks = blocks;
  return batch_items(b, rows);
}

fm_status fm_batch_run(fm_batch* b, int32_t use_graph) {
  if (!b) return fail(FM_ERR_INVALID, "batch is NULL");
  for (int g = 0; g < b->n_groups; ++g)
    if (b->groups[g].env->day != b->start_day[g])
      return fail(FM_ERR_STATE, "an environment is not at the day the batch was created for (group " +
                                    std::to_string(g) + ")");
  DeviceGuard guard(b->device);
  hipError_t e = hipSuccess;
  if (use_graph) {
    if (!b->exec) {
      // Captured on a private stream (the caller's may be the legacy default stream, which cannot
      // capture) and launched on the caller's.
      if (!b->capture) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        const hipError_t le = batch_enqueue(b, b->n_chunks, b->capture);
        e = hipStreamEndCapture(b->capture, &b->graph);
        if (le != hipSuccess) e = le;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        batch_drop_graph(b);
        return device_status(e, "fm_batch_run (graph capture)");
      }
    }
    e = hipGraphLaunch(b->exec, b->stream);
  } else {
    e = batch_enqueue(b, b->n_chunks, b->stream);
  }
  if (e != hipSuccess) return device_status(e, "fm_batch_run");
  for (fm_batch_group& G : b->groups) G.env->day += G.n_steps;
  return FM_OK;
}

void fm_batch_destroy(fm_batch* b) {
  if (!b) return;
  batch_drop_graph(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

const char* fm_version(void) { return "finrl_mi 0.1 gfx950"; }

size_t env_workspace_bytes(const fm_env_config* cfg) {
  if (!validate_config(cfg).empty()) return 0;
  return env_layout(*cfg).total;
}

fm_status env_create(const fm_env_config* cfg, const float* d_close, const float* d_ind,
                     void* d_workspace, size_t workspace_bytes, hipStream_t stream,
                     fm_env** out) {
  if (!out) return fail(FM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  const std::string why = validate_config(cfg);
  if (!why.empty()) return fail(FM_ERR_INVALID, why);
  if (!d_close) return fail(FM_ERR_INVALID, "d_close is NULL");
  if (!d_ind && cfg->n_ind > 0) return fail(FM_ERR_INVALID, "d_ind is NULL");
  if (!d_workspace) return fail(FM_ERR_INVALID, "d_workspace is NULL");
  if (!aligned(d_workspace)) return fail(FM_ERR_INVALID, "d_workspace must be 256-byte aligned");
  const EnvLayout L = env_layout(*cfg);
  if (workspace_bytes < L.total) return fail(FM_ERR_INVALID, "workspace too small");
  fm_env* e = new (std::nothrow) fm_env();
  if (!e) return fail(FM_ERR_DEVICE, "host allocation failed");
  e->cfg = *cfg;
  fm::EnvConst& C = e->C;
  C.N = cfg->n_envs;
  C.D = cfg->n_stocks;
  C.I = cfg->n_ind;
  C.T = cfg->n_days;
  C.S = (cfg->n_ind + 2) * cfg->n_stocks + 1;
  C.hmax = cfg->hmax;
  C.hmax_f = static_cast<float>(cfg->hmax);
  C.cash_scale = cfg->cash_obs_scale;
  C.price_scale = cfg->price_obs_scale;
  C.hold_scale = cfg->hold_obs_scale;
  C.init_cash = cfg->init_cash;
  C.one_m = 1.0 - cfg->cost_rate;
  C.one_p = 1.0 + cfg->cost_rate;
  C.reward_scale = cfg->reward_scale;
  C.close = d_close;
  C.ind = d_ind;
  unsigned char* base = static_cast<unsigned char*>(d_workspace);
  e->st.cash = reinterpret_cast<double*>(base + L.cash);
  e->st.asset = reinterpret_cast<double*>(base + L.asset);
  e->st.cumrew = reinterpret_cast<double*>(base + L.cumrew);
  e->st.hold = reinterpret_cast<int*>(base + L.hold);
  e->act_stage = reinterpret_cast<float*>(base + L.act);
  e->obs_stage = reinterpret_cast<float*>(base + L.obs);
  e->eps_chunk = reinterpret_cast<float*>(base + L.eps);
  e->mt_chunk = reinterpret_cast<float*>(base + L.mt);
  e->stream = stream;
  if (hipGetDevice(&e->device) != hipSuccess) e->device = 0;
  e->day = 0;
  e->tile = env_tile(C.N);
  e->step_kernel = 0;
  e->lane_envs = 0;
  *out = e;
  return FM_OK;
}

fm_status env_reset(fm_env* env, float* d_obs) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  DeviceGuard g(env->device);
  fm_status s = device_status(fm::launch_env_reset(env->C, env->st, d_obs, env->tile, env->stream),
                              "env_reset");
  if (s == FM_OK) env->day = 0;
  return s;
}

fm_status env_step(fm_env* env, const float* d_act, float* d_obs, double* d_reward,
                   int32_t* d_exec_qty, int32_t* h_done) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (!d_act) return fail(FM_ERR_INVALID, "d_act is NULL");
  if (!d_reward) return fail(FM_ERR_INVALID, "d_reward is NULL");
  if (env->day >= env->C.T) return fail(FM_ERR_STATE, "environment is at the last day; reset first");
  DeviceGuard g(env->device);
  fm_status s = device_status(launch_given(env, env->day, 1, d_act, d_obs, d_reward, d_exec_qty, env->stream),
                              "env_step");
  if (s != FM_OK) return s;
  env->day += 1;
  if (h_done) *h_done = env->day == env->C.T ? 1 : 0;
  return FM_OK;
}

fm_status env_rollout(fm_env* env, const fm_ensemble* ens, int32_t n_steps,
                      const fm_rollout_opts* opts) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (!opts) return fail(FM_ERR_INVALID, "opts is NULL");
  if (n_steps < 0) return fail(FM_ERR_INVALID, "n_steps must be >= 0");
  if (opts->path != FM_PATH_PLAIN && opts->path != FM_PATH_FUSED)
    return fail(FM_ERR_INVALID, "path must be FM_PATH_PLAIN or FM_PATH_FUSED");
  if (env->day + n_steps > env->C.T)
    return fail(FM_ERR_STATE, "rollout would run past the last day");
  if (n_steps == 0) return FM_OK;
  const fm::EnvConst& C = env->C;
  const size_t N = C.N, D = C.D, S = C.S;
  DeviceGuard g(env->device);
  hipStream_t st = env->stream;
  if (opts->d_actions) {  // driven mode: one launch over all steps
    fm_status s = device_status(launch_given(env, env->day, n_steps, opts->d_actions, opts->d_obs_traj,
                                             opts->d_rew_traj, opts->d_qty_traj, st),
                                "env_rollout (driven)");
    if (s != FM_OK) return s;
    if (opts->d_act_traj) {
      s = device_status(hipMemcpyAsync(opts->d_act_traj, opts->d_actions,
                                       sizeof(float) * N * D * n_steps, hipMemcpyDeviceToDevice, st),
                        "env_rollout (copy actions)");
      if (s != FM_OK) return s;
    }
    env->day += n_steps;
    return FM_OK;
  }
  if (!ens) return fail(FM_ERR_INVALID, "closed-loop rollout needs an ensemble");
  if (ens->S != C.S || ens->A != C.D)
    return fail(FM_ERR_INVALID, "ensemble in_dim/out_dim do not match the environment state/action");
  if (!(opts->sigma >= 0.0f) || !std::isfinite(opts->sigma)) return fail(FM_ERR_INVALID, "sigma must be finite and >= 0");
  if (ens->device != env->device) return fail(FM_ERR_INVALID, "ensemble and environment are on different devices");
  if (opts->path == FM_PATH_FUSED) {
    if (ens->dtype != FM_BF16) return fail(FM_ERR_UNSUPPORTED, "the fused path runs bfloat16 ensembles");
    std::string why;
    const hipError_t e = fm::launch_fused_rollout(C, env->st, ens->E, env->day, n_steps, opts->sigma,
                                                  opts->noise_key, opts->env_offset, opts->d_obs_traj,
                                                  opts->d_act_traj, opts->d_rew_traj, opts->d_qty_traj,
                                                  env->eps_chunk, env->mt_chunk, st, &why, env->fused);
    if (!why.empty()) return fail(FM_ERR_UNSUPPORTED, why);
    fm_status s = device_status(e, "env_rollout (fused)");
    if (s != FM_OK) return s;
    env->day += n_steps;
    return FM_OK;
  }
  if (static_cast<size_t>(ens->max_batch) < N)
    return fail(FM_ERR_INVALID, "ensemble max_batch is smaller than n_envs");
  // Plain path: the current state, then per step the ensemble MLP and the env step.
  fm_status s = device_status(fm::launch_env_observe(C, env->st, env->day, env->obs_stage, env->tile, st),
                              "env_rollout (observe)");
  if (s != FM_OK) return s;
  const float* obs_in = env->obs_stage;
  for (int i = 0; i < n_steps; ++i) {
    const int t = env->day + i;
    s = device_status(fm::launch_mlp(ens->dtype, ens->E, obs_in, C.N, ens->mu, st), "env_rollout (mlp)");
    if (s != FM_OK) return s;
    float* obs_out = opts->d_obs_traj ? opts->d_obs_traj + static_cast<size_t>(i) * N * S : env->obs_stage;
    float* act_out = opts->d_act_traj ? opts->d_act_traj + static_cast<size_t>(i) * N * D : nullptr;
    double* rew = opts->d_rew_traj ? opts->d_rew_traj + static_cast<size_t>(i) * N : nullptr;
    int* qty = opts->d_qty_traj ? opts->d_qty_traj + static_cast<size_t>(i) * N * D : nullptr;
    const hipError_t e =
        row_kernel_means(env, ens->K)
            ? fm::launch_env_row_ensemble_step(C, env->st, t, ens->mu, ens->E.mix, ens->K, opts->sigma,
                                               opts->noise_key, opts->env_offset, obs_out, act_out, rew, qty,
                                               row_envs(env), st)
        : lane_kernel_means(env)
            ? fm::launch_env_lane_ensemble_step(C, env->st, t, ens->mu, ens->E.mix, ens->K, opts->sigma,
                                                opts->noise_key, opts->env_offset, obs_out, act_out, rew, qty,
                                                env->lane_envs, st)
            : fm::launch_env_ensemble_step(C, env->st, t, ens->mu, ens->E.mix, ens->K, opts->sigma,
                                           opts->noise_key, opts->env_offset, obs_out, act_out, rew, qty,
                                           env->tile, st);
    s = device_status(e, "env_rollout (step)");
    if (s != FM_OK) return s;
    obs_in = obs_out;
  }
  env->day += n_steps;
  return FM_OK;
}

fm_status env_read_state(const fm_env* env, double* d_cash, int32_t* d_hold, double* d_asset,
                         double* d_cumrew, int32_t* h_day) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (h_day) *h_day = env->day;
  if (!d_cash && !d_hold && !d_asset && !d_cumrew) return FM_OK;
  DeviceGuard g(env->device);
  return device_status(fm::launch_read_state(env->C, env->st, d_cash, d_hold, d_asset, d_cumrew, env->stream),
                       "env_read_state");
}

fm_status env_write_state(fm_env* env, const double* d_cash, const int32_t* d_hold,
                          const double* d_asset, const double* d_cumrew, int32_t day) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (!d_cash || !d_hold || !d_asset || !d_cumrew) return fail(FM_ERR_INVALID, "all state buffers are required");
  if (day < 0 || day > env->C.T) return fail(FM_ERR_INVALID, "day must be in 0..T");
  DeviceGuard g(env->device);
  fm_status s = device_status(
      fm::launch_write_state(env->C, env->st, d_cash, d_hold, d_asset, d_cumrew, env->stream), "env_write_state");
  if (s == FM_OK) env->day = day;
  return s;
}

int32_t env_day(const fm_env* env) { return env ? env->day : -1; }

fm_status env_set_tile(fm_env* env, int32_t envs_per_group, int32_t* h_tile) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (envs_per_group < 0 || envs_per_group > 64) return fail(FM_ERR_INVALID, "envs_per_group must be in 0..64");
  env->tile = envs_per_group == 0 ? env_tile(env->C.N) : envs_per_group;
  if (h_tile) *h_tile = env->tile;
  return FM_OK;
}

fm_status env_set_step_kernel(fm_env* env, int32_t kernel, int32_t envs_per_wave) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (kernel < 0 || kernel > 3)
    return fail(FM_ERR_INVALID, "kernel must be 0 (by shape and size), 1 (tile), 2 (lane) or 3 (row)");
  if (envs_per_wave < 0 || envs_per_wave > 64) return fail(FM_ERR_INVALID, "envs_per_wave must be in 0..64");
  if (kernel == 3 && envs_per_wave > 2) return fail(FM_ERR_INVALID, "the row kernel takes 1 or 2 environments per wavefront");
  if ((kernel == 2 || kernel == 3) && !fm::env_lane_shape(env->C))
    return fail(FM_ERR_UNSUPPORTED, "the lane and row kernels take at most 32 stocks and (2 + n_ind) * n_stocks < 256");
  env->step_kernel = kernel;
  env->lane_envs = envs_per_wave;
  return FM_OK;
}

fm_status env_set_fused_tuning(fm_env* env, int32_t schedule, int32_t row_tiles, int32_t tile_envs) {
  if (!env) return fail(FM_ERR_INVALID, "env is NULL");
  if (schedule < 0 || schedule > 3)
    return fail(FM_ERR_INVALID, "schedule must be 0 (by shape and size), 1 (streamed), 2 (generic) or 3 (resident)");
  if (row_tiles < 0 || row_tiles > 2) return fail(FM_ERR_INVALID, "row_tiles must be 0, 1 or 2");
  if (tile_envs < 0 || tile_envs > 32) return fail(FM_ERR_INVALID, "tile_envs must be in 0..32");
  env->fused.schedule = schedule;
  env->fused.row_tiles = row_tiles;
  env->fused.tile_envs = tile_envs;
  return FM_OK;
}

void env_destroy(fm_env* env) { delete env; }

size_t ensemble_workspace_bytes(int32_t n_actors, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                int32_t dtype, int32_t max_batch) {
  if (!validate_ensemble(n_actors, in_dim, hidden, out_dim, dtype, max_batch).empty()) return 0;
  return ens_layout(n_actors, in_dim, hidden, out_dim, dtype, max_batch).total;
}

fm_status ensemble_create(int32_t K, int32_t S, int32_t H, int32_t A, int32_t dtype, const float* d_w,
                          const float* h_mix, int32_t max_batch, void* d_workspace, size_t workspace_bytes,
                          hipStream_t stream, fm_ensemble** out) {
  if (!out) return fail(FM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  const std::string why = validate_ensemble(K, S, H, A, dtype, max_batch);
  if (!why.empty()) return fail(FM_ERR_INVALID, why);
  if (!d_w) return fail(FM_ERR_INVALID, "d_w is NULL");
  if (!d_workspace) return fail(FM_ERR_INVALID, "d_workspace is NULL");
  if (!aligned(d_workspace)) return fail(FM_ERR_INVALID, "d_workspace must be 256-byte aligned");
  const EnsLayout L = ens_layout(K, S, H, A, dtype, max_batch);
  if (workspace_bytes < L.total) return fail(FM_ERR_INVALID, "workspace too small");
  float mix[8];
  for (int k = 0; k < K; ++k) {
    mix[k] = h_mix ? h_mix[k] : 1.0f / static_cast<float>(K);
    if (!std::isfinite(mix[k])) return fail(FM_ERR_INVALID, "mix weights must be finite");
  }
  fm_ensemble* e = new (std::nothrow) fm_ensemble();
  if (!e) return fail(FM_ERR_DEVICE, "host allocation failed");
  e->K = K;
  e->S = S;
  e->H = H;
  e->A = A;
  e->dtype = dtype;
  e->max_batch = max_batch;
  if (hipGetDevice(&e->device) != hipSuccess) e->device = 0;
  unsigned char* base = static_cast<unsigned char*>(d_workspace);
  fm::EnsDev& E = e->E;
  E.K = K;
  E.S = S;
  E.H = H;
  E.A = A;
  E.S_pad = L.S_pad;
  E.A_pad = L.A_pad;
  E.base = base;
  E.actor_stride = L.actor;
  E.off_w1 = L.w1;
  E.off_w2 = L.w2;
  E.off_w3 = L.w3;
  E.off_b1 = L.b1;
  E.off_b2 = L.b2;
  E.off_b3 = L.b3;
  E.mix = reinterpret_cast<const float*>(base + L.mix);
  E.split_a = L.split_a;
  E.ke_pad = L.ke_pad;
  E.off_w1e = L.w1e;
  E.off_w1m = L.w1m;
  e->mu = reinterpret_cast<float*>(base + L.mu);
  // Master layout per actor: W1[S][H], b1[H], W2[H][H], b2[H], W3[H][A], b3[A].
  const size_t per_actor = static_cast<size_t>(S) * H + H + static_cast<size_t>(H) * H + H +
                           static_cast<size_t>(H) * A + A;
  hipError_t err = hipSuccess;
  for (int k = 0; k < K && err == hipSuccess; ++k) {
    const float* src = d_w + per_actor * k;
    unsigned char* dst = base + L.actor * k;
    const float* w1 = src;
    const float* b1 = w1 + static_cast<size_t>(S) * H;
    const float* w2 = b1 + H;
    const float* b2 = w2 + static_cast<size_t>(H) * H;
    const float* w3 = b2 + H;
    const float* b3 = w3 + static_cast<size_t>(H) * A;
    err = fm::launch_pack_matrix(dtype, w1, S, H, L.S_pad, H, dst + L.w1, stream);
    if (err == hipSuccess) err = fm::launch_pack_matrix(dtype, w2, H, H, H, H, dst + L.w2, stream);
    if (err == hipSuccess) err = fm::launch_pack_matrix(dtype, w3, H, A, H, L.A_pad, dst + L.w3, stream);
    if (err == hipSuccess) err = fm::launch_copy_pad(b1, H, H, reinterpret_cast<float*>(dst + L.b1), stream);
    if (err == hipSuccess) err = fm::launch_copy_pad(b2, H, H, reinterpret_cast<float*>(dst + L.b2), stream);
    if (err == hipSuccess) err = fm::launch_copy_pad(b3, A, L.A_pad, reinterpret_cast<float*>(dst + L.b3), stream);
    if (err == hipSuccess && L.split_a > 0) {
      err = fm::launch_pack_env_rows(w1, A, H, L.ke_pad, base + L.w1e + 2 * static_cast<size_t>(k) * H * L.ke_pad,
                                     stream);
      if (err == hipSuccess)
        err = fm::launch_gather_market_rows(w1, S, H, A,
                                            reinterpret_cast<__bf16*>(base + L.w1m) +
                                                static_cast<size_t>(k) * (S - 1 - A) * H,
                                            stream);
    }
  }
  if (err == hipSuccess)
    err = hipMemcpyAsync(base + L.mix, mix, sizeof(float) * K, hipMemcpyHostToDevice, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  if (err != hipSuccess) {
    delete e;
    return device_status(err, "ensemble_create");
  }
  *out = e;
  return FM_OK;
}

fm_status ensemble_act(const fm_ensemble* ens, const float* d_obs, int32_t n, float sigma, uint64_t noise_key,
                       int32_t t, int64_t env_offset, float* d_mean, float* d_act, hipStream_t stream) {
  if (!ens) return fail(FM_ERR_INVALID, "ensemble is NULL");
  if (!d_obs || !d_act) return fail(FM_ERR_INVALID, "d_obs and d_act are required");
  if (n < 0 || n > ens->max_batch) return fail(FM_ERR_INVALID, "n must be in 0..max_batch");
  if (!(sigma >= 0.0f) || !std::isfinite(sigma)) return fail(FM_ERR_INVALID, "sigma must be finite and >= 0");
  if (t < 0) return fail(FM_ERR_INVALID, "t must be >= 0");
  if (env_offset < 0) return fail(FM_ERR_INVALID, "env_offset must be >= 0");
  if (n == 0) return FM_OK;
  DeviceGuard g(ens->device);
  fm_status s = device_status(fm::launch_mlp(ens->dtype, ens->E, d_obs, n, ens->mu, stream), "ensemble_act (mlp)");
  if (s != FM_OK) return s;
  return device_status(fm::launch_combine(ens->K, n, ens->A, ens->mu, ens->E.mix, sigma, noise_key, t, env_offset,
                                          d_mean, d_act, stream),
                       "ensemble_act (combine)");
}

void ensemble_destroy(fm_ensemble* ens) { delete ens; }

fm_status fm_backtest_metrics(const double* d_rew, int32_t n_steps, int32_t n_envs, double init_asset,
                              const double* d_init_asset, double reward_scale, double periods_per_year,
                              double risk_free, double* d_out, hipStream_t stream) {
  if (!d_rew || !d_out) return fail(FM_ERR_INVALID, "d_rew and d_out are required");
  if (n_steps < 1 || n_envs < 0) return fail(FM_ERR_INVALID, "n_steps must be >= 1 and n_envs >= 0");
  if (!(reward_scale != 0.0) || !std::isfinite(reward_scale)) return fail(FM_ERR_INVALID, "reward_scale must be finite and nonzero");
  if (!(periods_per_year > 0.0) || !std::isfinite(periods_per_year)) return fail(FM_ERR_INVALID, "periods_per_year must be > 0");
  if (!std::isfinite(risk_free) || !std::isfinite(init_asset)) return fail(FM_ERR_INVALID, "risk_free and init_asset must be finite");
  if (n_envs == 0) return FM_OK;
  return device_status(fm::launch_metrics(d_rew, n_steps, n_envs, init_asset, d_init_asset, reward_scale,
                                          periods_per_year, risk_free, d_out, stream),
                       "fm_backtest_metrics");
}

fm_status fm_sharpe_weights(const double* h_sharpe, int32_t n_actors, double min_sharpe, float* h_mix) {
  if (!h_sharpe || !h_mix) return fail(FM_ERR_INVALID, "h_sharpe and h_mix are required");
  if (n_actors < 1 || n_actors > 8) return fail(FM_ERR_INVALID, "n_actors must be in 1..8");
  int best = 0;
  double top = -INFINITY;
  bool any = false;
  for (int k = 0; k < n_actors; ++k) {
    if (std::isnan(h_sharpe[k])) return fail(FM_ERR_INVALID, "Sharpe ratios must not be NaN");
    if (h_sharpe[k] > h_sharpe[best]) best = k;
    if (h_sharpe[k] >= min_sharpe) {
      any = true;
      top = std::fmax(top, h_sharpe[k]);
    }
  }
  if (!any) {
    for (int k = 0; k < n_actors; ++k) h_mix[k] = k == best ? 1.0f : 0.0f;
    return FM_OK;
  }
  double e[8], total = 0.0;
  for (int k = 0; k < n_actors; ++k) {
    e[k] = h_sharpe[k] >= min_sharpe ? std::exp(h_sharpe[k] - top) : 0.0;
    total += e[k];
  }
  for (int k = 0; k < n_actors; ++k) h_mix[k] = static_cast<float>(e[k] / total);
  return FM_OK;
}

fm_status fm_noise(uint64_t noise_key, int64_t env_offset, int32_t n, int32_t t, int32_t n_stocks,
                   uint64_t* d_words, float* d_eps, hipStream_t stream) {
  if (!d_eps) return fail(FM_ERR_INVALID, "d_eps is NULL");
  if (n < 0 || n_stocks < 1 || n_stocks > 1024 || t < 0 || env_offset < 0)
    return fail(FM_ERR_INVALID, "bad sizes");
  if (n == 0) return FM_OK;
  return device_status(fm::launch_noise(noise_key, env_offset, n, t, n_stocks, d_words, d_eps, stream), "fm_noise");
}

}  // extern "C"
