// The single-asset crypto task served with continuous batching (include/crypto_serve.h):
// the per-chunk policy + environment kernel and the request scheduler.
//
// Kernel.  A workgroup of five wavefronts runs a work item = ROWS environments of one request
// for up to chunk_ticks ticks.  The agents' weights stay on chip for the whole launch: MLP
// wavefront w (0..3) owns hidden units 32w..32w+31 of every agent, with its slice of W2 in
// registers and W1, W3 and the biases in LDS; wavefront 4 holds the environments.  All three layers run transposed on MFMA (outputs x environments), so
// a wavefront's layer-1 and layer-2 accumulators are directly the B operands of the next layer
// once its k-slots are read in the order the weights were packed:
//   k-slot 8g + j of wavefront w  <->  hidden unit 32w + 16 (j / 4) + 4g + (j % 4).
// Per tick: layer 1 (16 -> 128, v_mfma_f32_16x16x16_bf16) and an LDS exchange of the hidden
// units; layer 2 (v_mfma_f32_16x16x32_bf16, W2 from registers) and the wavefront's share of
// layer 3 (its 32 units) into LDS partial sums; then one lane of the environment wavefront per
// environment adds the four partial sums in a fixed order, applies the ensemble rule and the
// exploration draw (computed while the MLP ran), trades in float64, updates the running
// statistics and writes the next state row.  Three workgroup barriers per tick.  The
// environment's state stays in that lane's registers for the item.
//
// Scheduler.  Host-side: a FIFO queue, a first-fit allocator over the caller's device pool, the
// active set, and per-chunk lists of (request, tile) items copied from pinned staging.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/crypto_serve.h"
#include "device_common.h"
#include "pool_alloc.h"
#include "mlp_device.h"
#include "status.h"

namespace fm {
namespace cx {

constexpr int kF = 16;    // agent input width
constexpr int kH = 128;   // hidden units
constexpr int kA = 3;     // actions
constexpr int kNW = 4;    // MLP wavefronts per workgroup
constexpr int kNT = 64 * (kNW + 1);   // plus the environment wavefront

typedef __attribute__((ext_vector_type(4))) short s16x4;

struct ReqDesc {
  int64_t start_tick, horizon, t0;
  int32_t n_envs, stride;
  uint64_t key;
  fm_crypto_result* state;
  fm_crypto_result* result;
  int8_t* act;
  float* prob;
};

// Packed agents (device), all agents back to back.
struct PolicyDev {
  const bf16x8* w2;   // [K][4 waves][2 tiles][4 k-steps][64 lanes]
  const s16x4* w1;    // [K][4 waves][2 tiles][64 lanes]
  const bf16x8* w3;   // [K][4 waves][64 lanes]
  const float* b1;    // [K][128]
  const float* b2;    // [K][128]
  const float* b3;    // [K][4] (padded)
  const float* mix;   // [K]
};

struct ChunkArgs {
  const double* mid;
  const float* feat;
  PolicyDev P;
  int rule;
  float eps;
  double fee, cash0;
  const ReqDesc* reqs;
  const int2* items;
  int n_items;
  int* counter;
  int chunk;
};

typedef __attribute__((ext_vector_type(8))) short s16x8;

// relu(x) rounded to bfloat16 for eight accumulators.  Rounding keeps the sign, so the ReLU is
// applied after it as a signed 16-bit max with zero on the bfloat16 bit patterns (negative
// values, -0 included, have the sign bit set).
__device__ __forceinline__ bf16x8 pack_relu(floatx4 a, floatx4 b) {
  bf16x8 r;
  r[0] = static_cast<__bf16>(a[0]);
  r[1] = static_cast<__bf16>(a[1]);
  r[2] = static_cast<__bf16>(a[2]);
  r[3] = static_cast<__bf16>(a[3]);
  r[4] = static_cast<__bf16>(b[0]);
  r[5] = static_cast<__bf16>(b[1]);
  r[6] = static_cast<__bf16>(b[2]);
  r[7] = static_cast<__bf16>(b[3]);
  const s16x8 m = __builtin_elementwise_max(__builtin_bit_cast(s16x8, r), s16x8{0, 0, 0, 0, 0, 0, 0, 0});
  return __builtin_bit_cast(bf16x8, m);
}

__device__ __forceinline__ floatx4 mfma16(s16x4 a, s16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// The state row x = fl32([b 2^-17, p 2^-16, h, f]) rounded to bfloat16, into LDS row xr[16].
__device__ __forceinline__ void write_state_row(__bf16* xr, double cash, double p, int pos, const float4 (&f)[4]) {
  bf16x8 lo, hi;
  lo[0] = static_cast<__bf16>(static_cast<float>(cash * 0x1p-17));
  lo[1] = static_cast<__bf16>(static_cast<float>(p * 0x1p-16));
  lo[2] = static_cast<__bf16>(static_cast<float>(pos));
  lo[3] = static_cast<__bf16>(f[0].w);
  lo[4] = static_cast<__bf16>(f[1].x);
  lo[5] = static_cast<__bf16>(f[1].y);
  lo[6] = static_cast<__bf16>(f[1].z);
  lo[7] = static_cast<__bf16>(f[1].w);
  hi[0] = static_cast<__bf16>(f[2].x);
  hi[1] = static_cast<__bf16>(f[2].y);
  hi[2] = static_cast<__bf16>(f[2].z);
  hi[3] = static_cast<__bf16>(f[2].w);
  hi[4] = static_cast<__bf16>(f[3].x);
  hi[5] = static_cast<__bf16>(f[3].y);
  hi[6] = static_cast<__bf16>(f[3].z);
  hi[7] = static_cast<__bf16>(f[3].w);
  reinterpret_cast<bf16x8*>(xr)[0] = lo;
  reinterpret_cast<bf16x8*>(xr)[1] = hi;
}

__device__ __forceinline__ void load_feat(const float* feat, int64_t tick, float4 (&f)[4]) {
  const float4* src = reinterpret_cast<const float4*>(feat + tick * kF);
#pragma unroll
  for (int i = 0; i < 4; ++i) f[i] = src[i];
}

#pragma clang fp contract(off)
template <int R, int K>
__global__ __launch_bounds__(kNT, 1) void crypto_chunk_kernel(ChunkArgs a) {
  constexpr int ROWS = 16 * R;
  // Separate LDS objects, so that the compiler can see that the layer phases' loads and stores
  // never alias and keep several blocks' MFMA chains in flight.
  __shared__ s16x4 w1s[K * kNW * 2 * 64];
  __shared__ bf16x8 w3s[K * kNW * 12];   // lanes (g, r < 3) of the layer-3 A fragments
  __shared__ __align__(16) float b1s[K * kH];
  __shared__ __align__(16) float b2s[K * kH];
  __shared__ float b3s[K * 4];
  __shared__ float mixs[K];
  __shared__ __align__(16) __bf16 xs[R * 16 * kF];
  __shared__ bf16x8 hs[K * kNW * R * 64];
  __shared__ floatx4 ps[kNW * K * R * 16];
  __shared__ floatx4 pk[K * ROWS];   // per-agent weighted probabilities or votes
  // The environments' state between ticks (kept out of registers that the MLP wavefronts need).
  __shared__ double s_cash[ROWS], s_value[ROWS], s_sum[ROWS], s_sum2[ROWS], s_peak[ROWS], s_mdd[ROWS];
  __shared__ int s_pos[ROWS], s_trades[ROWS];
  __shared__ double sp[ROWS], sp1[ROWS];
  __shared__ float4 sf[ROWS * 4];
  __shared__ int s_item;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, e16 = lane & 15;
  const bool mlp_wave = wave < kNW;

  // Agents into LDS (W1, W3, biases) and registers (each MLP wavefront's W2 slice).
  for (int i = tid; i < K * kNW * 2 * 64; i += kNT) w1s[i] = a.P.w1[i];
  for (int i = tid; i < K * kNW * 12; i += kNT) {
    const int kw = i / 12, gr = i % 12;   // fragment rows 3..15 are zero and not stored
    w3s[i] = a.P.w3[kw * 64 + (gr / 3) * 16 + gr % 3];
  }
  for (int i = tid; i < K * kH; i += kNT) {
    b1s[i] = a.P.b1[i];
    b2s[i] = a.P.b2[i];
  }
  for (int i = tid; i < K * 4; i += kNT) b3s[i] = a.P.b3[i];
  for (int i = tid; i < K; i += kNT) mixs[i] = a.P.mix[i];
  bf16x8 w2[K][2][4];
  {
    const int wl = mlp_wave ? wave : 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int tt = 0; tt < 2; ++tt)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) w2[k][tt][kk] = a.P.w2[(((k * kNW + wl) * 2 + tt) * 4 + kk) * 64 + lane];
  }

  // The environment wavefront: lane ce < ROWS owns environment ce of the work item.
  const bool env_lane = wave == kNW && lane < ROWS;
  const int ce = lane;

  for (;;) {
    __syncthreads();
    if (tid == 0) s_item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= a.n_items) break;
    const int2 it = a.items[item];
    const ReqDesc d = a.reqs[it.x];
    const int n0 = it.y * ROWS;
    const int nvalid = min(ROWS, d.n_envs - n0);
    const int64_t t0 = d.t0;
    const int nt = static_cast<int>(min(static_cast<int64_t>(a.chunk), d.horizon - t0));
    const bool valid = env_lane && ce < nvalid;
    const int64_t n = n0 + ce;

    const int64_t tick0 = d.start_tick + n * d.stride + t0;   // this environment's tick at t0
    if (valid) {
      double cash = a.cash0, value = a.cash0, sum = 0.0, sum2 = 0.0, peak = a.cash0, mdd = 0.0;
      int pos = 0, trades = 0;
      if (t0 != 0) {
        const fm_crypto_result* r = d.state + n;
        cash = r->cash;
        value = r->value;
        sum = r->sum_r;
        sum2 = r->sum_r2;
        peak = r->peak;
        mdd = r->max_drawdown;
        pos = r->position;
        trades = r->trades;
      }
      s_cash[ce] = cash;
      s_value[ce] = value;
      s_sum[ce] = sum;
      s_sum2[ce] = sum2;
      s_peak[ce] = peak;
      s_mdd[ce] = mdd;
      s_pos[ce] = pos;
      s_trades[ce] = trades;
      const double p = a.mid[tick0];
      sp[ce] = p;
      float4 f[4];
      load_feat(a.feat, tick0, f);
      write_state_row(xs + ce * kF, cash, p, pos, f);
    } else if (env_lane) {
      const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      float4 f[4] = {z, z, z, z};
      write_state_row(xs + ce * kF, 0.0, 0.0, 0, f);
    }
    __syncthreads();

    for (int s = 0; s < nt; ++s) {
      const int64_t t = t0 + s;
      if (mlp_wave) {
        // Layer 1: hidden units 32w.. of every agent for every block of 16 environments.
        s16x4 xb[R];
#pragma unroll
        for (int b = 0; b < R; ++b) xb[b] = *reinterpret_cast<const s16x4*>(xs + (b * 16 + e16) * kF + 4 * g);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const s16x4 wa0 = w1s[((k * kNW + wave) * 2 + 0) * 64 + lane];
          const s16x4 wa1 = w1s[((k * kNW + wave) * 2 + 1) * 64 + lane];
          const floatx4 c0 = *reinterpret_cast<const floatx4*>(b1s + k * kH + 32 * wave + 4 * g);
          const floatx4 c1 = *reinterpret_cast<const floatx4*>(b1s + k * kH + 32 * wave + 16 + 4 * g);
#pragma unroll
          for (int b = 0; b < R; ++b)
            hs[((k * kNW + wave) * R + b) * 64 + lane] = pack_relu(mfma16(wa0, xb[b], c0), mfma16(wa1, xb[b], c1));
        }
      } else if (valid) {
        // Next tick's market row, staged in LDS while the MLP runs.
        const int64_t tick = tick0 + s;
        sp1[ce] = a.mid[tick + 1];
        float4 f[4];
        load_feat(a.feat, tick + 1, f);
#pragma unroll
        for (int i = 0; i < 4; ++i) sf[ce * 4 + i] = f[i];
      }
      __syncthreads();
      int explore_act = -1;
      if (mlp_wave) {
        // Layer 2 (this wavefront's 32 units) and its share of layer 3.
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const floatx4 c0 = *reinterpret_cast<const floatx4*>(b2s + k * kH + 32 * wave + 4 * g);
          const floatx4 c1 = *reinterpret_cast<const floatx4*>(b2s + k * kH + 32 * wave + 16 + 4 * g);
          bf16x8 w3 = {};
          if (e16 < kA) w3 = w3s[(k * kNW + wave) * 12 + g * 3 + e16];
#pragma unroll
          for (int b = 0; b < R; ++b) {
            bf16x8 hc[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) hc[kk] = hs[((k * kNW + kk) * R + b) * 64 + lane];
            floatx4 acc0 = c0, acc1 = c1;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              acc0 = mfma_bf16(w2[k][0][kk], hc[kk], acc0);
              acc1 = mfma_bf16(w2[k][1][kk], hc[kk], acc1);
            }
            const floatx4 q = mfma_bf16(w3, pack_relu(acc0, acc1), floatx4{0.0f, 0.0f, 0.0f, 0.0f});
            if (lane < 16) ps[((wave * K + k) * R + b) * 16 + lane] = q;
          }
        }
      } else if (valid && a.eps > 0.0f) {
        // Exploration draw for this tick, while the MLP runs.
        uint64_t c0 = static_cast<uint64_t>(n), c1 = static_cast<uint64_t>(t), c2 = 0, c3 = 0;
        philox4x64_10(c0, c1, c2, c3, d.key, 1);
        if (uniform_from_word(c0) < a.eps) explore_act = static_cast<int>(static_cast<uint32_t>(c1 >> 32) % 3u);
      }
      __syncthreads();
      // One thread per (agent, environment): the agent's action values from the four partial
      // sums (fixed order) and its weighted softmax, or its vote.
      if (tid < K * ROWS) {
        const int k = tid / ROWS, c = tid % ROWS, b = c >> 4, e = c & 15;
        floatx4 q = ps[((0 * K + k) * R + b) * 16 + e];
#pragma unroll
        for (int w = 1; w < kNW; ++w) {
          const floatx4 pw = ps[((w * K + k) * R + b) * 16 + e];
          q[0] = q[0] + pw[0];
          q[1] = q[1] + pw[1];
          q[2] = q[2] + pw[2];
        }
        const float q0 = q[0] + b3s[4 * k], q1 = q[1] + b3s[4 * k + 1], q2 = q[2] + b3s[4 * k + 2];
        floatx4 out;
        if (a.rule == FM_RULE_AVG_SOFTMAX) {
          const float m = fmaxf(q0, fmaxf(q1, q2));
          const float e0 = __expf(q0 - m), e1 = __expf(q1 - m), e2 = __expf(q2 - m);
          const float inv = __builtin_amdgcn_rcpf((e0 + e1) + e2);
          const float wk = mixs[k];
          out = floatx4{wk * (e0 * inv), wk * (e1 * inv), wk * (e2 * inv), 0.0f};
        } else {
          const int j = (q0 >= q1 && q0 >= q2) ? 0 : (q1 >= q2 ? 1 : 2);
          out = floatx4{j == 0 ? 1.0f : 0.0f, j == 1 ? 1.0f : 0.0f, j == 2 ? 1.0f : 0.0f, 0.0f};
        }
        pk[k * ROWS + c] = out;
      }
      __syncthreads();
      // One lane per environment: ensemble rule, exploration, trade, statistics, next state row.
      if (valid) {
        float avg[kA] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const floatx4 v = pk[k * ROWS + ce];
          avg[0] = avg[0] + v[0];
          avg[1] = avg[1] + v[1];
          avg[2] = avg[2] + v[2];
        }
        // Averaged probabilities, or vote counts (exact small integers).
        int act = (avg[0] >= avg[1] && avg[0] >= avg[2]) ? 0 : (avg[1] >= avg[2] ? 1 : 2);
        float out[kA];
        if (a.rule == FM_RULE_AVG_SOFTMAX) {
          out[0] = avg[0];
          out[1] = avg[1];
          out[2] = avg[2];
        } else {
          out[0] = avg[0] / K;
          out[1] = avg[1] / K;
          out[2] = avg[2] / K;
        }
        if (explore_act >= 0) act = explore_act;
        // Trade at p, mark at p1 (float64, one rounding per operation).
        const double p = sp[ce], p1 = sp1[ce];
        const int pos1 = act - 1;
        const int delta = pos1 - s_pos[ce];
        const double cash1 = (s_cash[ce] - static_cast<double>(delta) * p) -
                             (static_cast<double>(delta < 0 ? -delta : delta) * p) * a.fee;
        const double v1 = cash1 + static_cast<double>(pos1) * p1;
        const double r = v1 - s_value[ce];
        s_sum[ce] = s_sum[ce] + r;
        s_sum2[ce] = s_sum2[ce] + r * r;
        const double peak = fmax(s_peak[ce], v1);
        s_peak[ce] = peak;
        s_mdd[ce] = fmax(s_mdd[ce], peak - v1);
        s_trades[ce] += delta != 0;
        s_cash[ce] = cash1;
        s_pos[ce] = pos1;
        s_value[ce] = v1;
        sp[ce] = p1;
        const int64_t o = t * d.n_envs + n;
        if (d.act) d.act[o] = static_cast<int8_t>(act);
        if (d.prob) {
          d.prob[3 * o] = out[0];
          d.prob[3 * o + 1] = out[1];
          d.prob[3 * o + 2] = out[2];
        }
        float4 f[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) f[i] = sf[ce * 4 + i];
        write_state_row(xs + ce * kF, cash1, p1, pos1, f);
      }
      __syncthreads();
    }
    if (valid) {
      const bool last = t0 + nt == d.horizon;
      for (int o = 0; o < (last ? 2 : 1); ++o) {
        fm_crypto_result* r = o == 0 ? d.state + n : d.result + n;
        r->cash = s_cash[ce];
        r->value = s_value[ce];
        r->sum_r = s_sum[ce];
        r->sum_r2 = s_sum2[ce];
        r->peak = s_peak[ce];
        r->max_drawdown = s_mdd[ce];
        r->position = s_pos[ce];
        r->trades = s_trades[ce];
        r->ticks = t0 + nt;
      }
    }
  }
}

__global__ void zero_counter(int* c) {
  if (threadIdx.x == 0) *c = 0;
}

template <int R, int K>
hipError_t launch(const ChunkArgs& a, int grid, hipStream_t stream) {
  zero_counter<<<1, 64, 0, stream>>>(a.counter);
  crypto_chunk_kernel<R, K><<<grid, kNT, 0, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_chunk(int rows, int K, const ChunkArgs& a, int grid, hipStream_t stream) {
  if (rows == 64) {
    if (K == 5) return launch<4, 5>(a, grid, stream);
    if (K == 3) return launch<4, 3>(a, grid, stream);
    if (K == 1) return launch<4, 1>(a, grid, stream);
  } else if (rows == 16) {
    if (K == 5) return launch<1, 5>(a, grid, stream);
    if (K == 3) return launch<1, 3>(a, grid, stream);
    if (K == 1) return launch<1, 1>(a, grid, stream);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------------
// Host: agent packing.
// ---------------------------------------------------------------------------------------------

// float32 -> bfloat16 bits, nearest with ties to even (NaN kept quiet).
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return static_cast<uint16_t>((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// Hidden unit behind k-slot (g, j) of wavefront w.
int unit_of(int w, int g, int j) { return 32 * w + 16 * (j / 4) + 4 * g + (j % 4); }

constexpr size_t kParamsPerAgent = size_t(kF) * kH + kH + size_t(kH) * kH + kH + size_t(kH) * kA + kA;

struct PackLayout {
  size_t w2, w1, w3, b1, b2, b3, mix, counter, reqs, items, total;
};

PackLayout pack_layout(int K, int max_requests, int64_t max_items) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  PackLayout L{};
  size_t o = 0;
  L.w2 = o;
  o = al(o + size_t(K) * kNW * 2 * 4 * 64 * 16);
  L.w1 = o;
  o = al(o + size_t(K) * kNW * 2 * 64 * 8);
  L.w3 = o;
  o = al(o + size_t(K) * kNW * 64 * 16);
  L.b1 = o;
  o = al(o + size_t(K) * kH * 4);
  L.b2 = o;
  o = al(o + size_t(K) * kH * 4);
  L.b3 = o;
  o = al(o + size_t(K) * 16);
  L.mix = o;
  o = al(o + size_t(K) * 4);
  L.counter = o;
  o = al(o + 4);
  L.reqs = o;
  o = al(o + sizeof(ReqDesc) * max_requests);
  L.items = o;
  o = al(o + sizeof(int2) * static_cast<size_t>(max_items));
  L.total = o;
  return L;
}

// Host image of the packed agents (everything before the counter).
std::vector<unsigned char> pack_agents(const fm_serve_config& c, const PackLayout& L) {
  const int K = c.n_agents;
  std::vector<unsigned char> img(L.counter, 0);
  auto put16 = [&](size_t off, uint16_t v) { std::memcpy(&img[off], &v, 2); };
  auto putf = [&](size_t off, float v) { std::memcpy(&img[off], &v, 4); };
  for (int k = 0; k < K; ++k) {
    const float* W1 = c.h_weights + k * kParamsPerAgent;
    const float* b1 = W1 + kF * kH;
    const float* W2 = b1 + kH;
    const float* b2 = W2 + kH * kH;
    const float* W3 = b2 + kH;
    const float* b3 = W3 + kH * kA;
    for (int w = 0; w < kNW; ++w)
      for (int lane = 0; lane < 64; ++lane) {
        const int g = lane >> 4, r = lane & 15;
        for (int tt = 0; tt < 2; ++tt) {
          const int unit = 32 * w + 16 * tt + r;  // output row of layers 1 and 2
          for (int kk = 0; kk < 4; ++kk)
            for (int j = 0; j < 8; ++j)
              put16(L.w2 + ((((size_t(k) * kNW + w) * 2 + tt) * 4 + kk) * 64 + lane) * 16 + 2 * j,
                    bf16_bits(W2[size_t(unit_of(kk, g, j)) * kH + unit]));
          for (int j = 0; j < 4; ++j)
            put16(L.w1 + (((size_t(k) * kNW + w) * 2 + tt) * 64 + lane) * 8 + 2 * j,
                  bf16_bits(W1[size_t(4 * g + j) * kH + unit]));
        }
        for (int j = 0; j < 8; ++j)
          put16(L.w3 + ((size_t(k) * kNW + w) * 64 + lane) * 16 + 2 * j,
                r < kA ? bf16_bits(W3[size_t(unit_of(w, g, j)) * kA + r]) : 0);
      }
    for (int i = 0; i < kH; ++i) {
      putf(L.b1 + (size_t(k) * kH + i) * 4, b1[i]);
      putf(L.b2 + (size_t(k) * kH + i) * 4, b2[i]);
    }
    for (int j = 0; j < kA; ++j) putf(L.b3 + (size_t(k) * 4 + j) * 4, b3[j]);
    putf(L.mix + size_t(k) * 4, c.h_mix ? c.h_mix[k] : 1.0f / K);
  }
  return img;
}


}  // namespace cx
}  // namespace fm

using fm::cx::ReqDesc;

struct fm_serve {
  struct Req {
    int64_t id;
    fm_serve_request r;
    size_t pool_off = 0, pool_len = 0;
    int64_t done = 0;
  };
  fm_serve_config cfg{};
  fm::cx::PackLayout L{};
  unsigned char* ws = nullptr;
  int rows = 64, grid = 0;
  int64_t max_items = 0;
  ReqDesc* h_reqs[2] = {nullptr, nullptr};
  int2* h_items[2] = {nullptr, nullptr};
  static constexpr int kEvents = 4;
  hipEvent_t ev[kEvents] = {};
  int64_t launched = 0;      // chunks launched
  int64_t completed = 0;     // chunks known complete
  hipStream_t stream = nullptr;
  bool stream_set = false;
  std::deque<Req> queue;
  std::vector<Req> active;
  int64_t active_envs = 0;
  fm::cx::PoolAlloc pool;
  std::deque<std::pair<int64_t, std::vector<int64_t>>> finishing;  // (chunk, ids)
  std::vector<int64_t> done;
  int64_t next_id = 0;
};

namespace {

using fm::set_error;

size_t request_bytes(int64_t n) { return n < 1 ? 0 : (sizeof(fm_crypto_result) * n + 255) / 256 * 256; }

std::string check_config(const fm_serve_config* c) {
  if (!c) return "config is NULL";
  if (!c->d_mid || !c->d_feat) return "tick table pointers are NULL";
  if (reinterpret_cast<uintptr_t>(c->d_feat) % 16 || reinterpret_cast<uintptr_t>(c->d_mid) % 8)
    return "tick table pointers must be 16-byte (features) and 8-byte (mid) aligned";
  if (c->n_ticks < 2) return "n_ticks must be >= 2";
  if (c->n_agents != 1 && c->n_agents != 3 && c->n_agents != 5) return "n_agents must be 1, 3 or 5";
  if (!c->h_weights) return "h_weights is NULL";
  if (c->rule != FM_RULE_AVG_SOFTMAX && c->rule != FM_RULE_MAJORITY_VOTE) return "unknown ensemble rule";
  if (!(c->eps >= 0.0f && c->eps <= 1.0f)) return "eps must be in [0, 1]";
  if (!(c->fee >= 0.0 && c->fee < 1.0)) return "fee must be in [0, 1)";
  if (!std::isfinite(c->cash0)) return "cash0 must be finite";
  if (c->tile_rows != 16 && c->tile_rows != 64) return "tile_rows must be 16 or 64";
  if (c->chunk_ticks < 1 || c->chunk_ticks > 65536) return "chunk_ticks must be in 1..65536";
  if (c->max_requests < 1 || c->max_requests > 65536) return "max_requests must be in 1..65536";
  if (c->max_active_envs < 1 || c->max_active_envs > (int64_t(1) << 30)) return "max_active_envs must be in 1..2^30";
  if (c->grid < 0 || c->grid > 65536) return "grid must be in 0..65536";
  if (!c->d_pool || reinterpret_cast<uintptr_t>(c->d_pool) % 256) return "d_pool must be non-NULL and 256-byte aligned";
  if (c->pool_bytes < request_bytes(1)) return "pool_bytes too small for one environment";
  return "";
}

int64_t items_cap(const fm_serve_config* c) {
  return c->max_active_envs / c->tile_rows + c->max_requests + 1;
}

}  // namespace

extern "C" {

size_t fm_serve_request_bytes(int32_t n_envs) { return request_bytes(n_envs); }

size_t fm_serve_workspace_bytes(const fm_serve_config* cfg) {
  if (!check_config(cfg).empty()) return 0;
  return fm::cx::pack_layout(cfg->n_agents, cfg->max_requests, items_cap(cfg)).total;
}

fm_status fm_serve_create(const fm_serve_config* cfg, hipStream_t stream, fm_serve** out) {
  if (!out) return set_error(FM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  const std::string why = check_config(cfg);
  if (!why.empty()) return set_error(FM_ERR_INVALID, "fm_serve_create: " + why);
  for (int k = 0; k < cfg->n_agents; ++k)
    for (size_t i = 0; i < fm::cx::kParamsPerAgent; ++i)
      if (!std::isfinite(cfg->h_weights[k * fm::cx::kParamsPerAgent + i]))
        return set_error(FM_ERR_INVALID, "fm_serve_create: weights must be finite");
  const fm::cx::PackLayout L = fm::cx::pack_layout(cfg->n_agents, cfg->max_requests, items_cap(cfg));
  if (!cfg->d_workspace || reinterpret_cast<uintptr_t>(cfg->d_workspace) % 256 || cfg->workspace_bytes < L.total)
    return set_error(FM_ERR_INVALID, "fm_serve_create: workspace NULL, unaligned or smaller than fm_serve_workspace_bytes");
  fm::DeviceGuard guard(cfg->device);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != cfg->device)
    return set_error(FM_ERR_DEVICE, "fm_serve_create: cannot select the device");
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fm::device_error(e, "fm_serve_create (device properties)");

  fm_serve* s = new (std::nothrow) fm_serve();
  if (!s) return set_error(FM_ERR_INVALID, "fm_serve_create: out of host memory");
  s->cfg = *cfg;
  s->cfg.h_weights = nullptr;
  s->cfg.h_mix = nullptr;
  s->L = L;
  s->ws = static_cast<unsigned char*>(cfg->d_workspace);
  s->rows = cfg->tile_rows;
  s->grid = cfg->grid > 0 ? cfg->grid : prop.multiProcessorCount;
  s->max_items = items_cap(cfg);
  s->pool.reset(cfg->pool_bytes / 256 * 256);
  auto cleanup = [&](fm_status st) {
    fm_serve_destroy(s);
    return st;
  };
  for (int i = 0; i < 2; ++i) {
    e = hipHostMalloc(reinterpret_cast<void**>(&s->h_reqs[i]), sizeof(ReqDesc) * cfg->max_requests, hipHostMallocDefault);
    if (e != hipSuccess) return cleanup(fm::device_error(e, "fm_serve_create (pinned staging)"));
    e = hipHostMalloc(reinterpret_cast<void**>(&s->h_items[i]), sizeof(int2) * s->max_items, hipHostMallocDefault);
    if (e != hipSuccess) return cleanup(fm::device_error(e, "fm_serve_create (pinned staging)"));
  }
  for (int i = 0; i < fm_serve::kEvents; ++i) {
    e = hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming);
    if (e != hipSuccess) return cleanup(fm::device_error(e, "fm_serve_create (events)"));
  }
  const std::vector<unsigned char> img = fm::cx::pack_agents(*cfg, L);
  e = hipMemcpyAsync(s->ws, img.data(), img.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return cleanup(fm::device_error(e, "fm_serve_create (agents)"));
  *out = s;
  return FM_OK;
}

fm_status fm_serve_submit(fm_serve* s, const fm_serve_request* r, int64_t* id) {
  if (!s || !r) return set_error(FM_ERR_INVALID, "fm_serve_submit: NULL argument");
  if (r->n_envs < 1 || r->n_envs > (1 << 24)) return set_error(FM_ERR_INVALID, "fm_serve_submit: n_envs must be in 1..2^24");
  if (r->stride < 0 || r->horizon < 1 || r->start_tick < 0)
    return set_error(FM_ERR_INVALID, "fm_serve_submit: stride >= 0, horizon >= 1, start_tick >= 0 required");
  const int64_t last = r->start_tick + int64_t(r->stride) * (r->n_envs - 1) + r->horizon;
  if (last > s->cfg.n_ticks - 1)
    return set_error(FM_ERR_INVALID, "fm_serve_submit: start_tick + (n_envs-1) stride + horizon exceeds n_ticks - 1");
  if (!r->d_result) return set_error(FM_ERR_INVALID, "fm_serve_submit: d_result is NULL");
  if (request_bytes(r->n_envs) > s->cfg.pool_bytes / 256 * 256 || r->n_envs > s->cfg.max_active_envs)
    return set_error(FM_ERR_INVALID, "fm_serve_submit: request larger than the pool or the active-environment limit");
  if (int64_t(r->n_envs) * r->horizon > (int64_t(1) << 40))
    return set_error(FM_ERR_INVALID, "fm_serve_submit: n_envs * horizon too large");
  fm_serve::Req q;
  q.id = s->next_id++;
  q.r = *r;
  s->queue.push_back(q);
  if (id) *id = q.id;
  return FM_OK;
}

static void collect(fm_serve* s, bool wait) {
  while (!s->finishing.empty()) {
    const int64_t chunk = s->finishing.front().first;
    hipEvent_t ev = s->ev[chunk % fm_serve::kEvents];
    if (wait) (void)hipEventSynchronize(ev);
    else if (hipEventQuery(ev) != hipSuccess) break;
    for (int64_t id : s->finishing.front().second) s->done.push_back(id);
    s->finishing.pop_front();
  }
}

fm_status fm_serve_step(fm_serve* s, hipStream_t stream, int32_t* n_active, int32_t* n_queued) {
  if (!s) return set_error(FM_ERR_INVALID, "fm_serve_step: server is NULL");
  if (s->stream_set && stream != s->stream)
    return set_error(FM_ERR_INVALID, "fm_serve_step: every step of a server must use the same stream");
  fm::DeviceGuard guard(s->cfg.device);
  const int buf = static_cast<int>(s->launched & 1);
  if (s->launched >= 2) {
    // The staging buffer of this parity was read by the copy of chunk launched - 2.
    const hipError_t e = hipEventSynchronize(s->ev[(s->launched - 2) % fm_serve::kEvents]);
    if (e != hipSuccess) return fm::device_error(e, "fm_serve_step (wait)");
  }
  // Admission in arrival order.
  while (!s->queue.empty() && static_cast<int>(s->active.size()) < s->cfg.max_requests) {
    fm_serve::Req& q = s->queue.front();
    if (s->active_envs + q.r.n_envs > s->cfg.max_active_envs) break;
    const size_t need = request_bytes(q.r.n_envs);
    size_t off = 0;
    if (!s->pool.alloc(need, &off)) break;
    q.pool_off = off;
    q.pool_len = need;
    s->active_envs += q.r.n_envs;
    s->active.push_back(q);
    s->queue.pop_front();
  }
  if (n_queued) *n_queued = static_cast<int32_t>(s->queue.size());
  if (s->active.empty()) {
    if (n_active) *n_active = 0;
    collect(s, false);
    return FM_OK;
  }
  // Work list: every tile of every active request, longest remaining chunk first.
  ReqDesc* hr = s->h_reqs[buf];
  int2* hi = s->h_items[buf];
  int64_t n_items = 0;
  const int chunk = s->cfg.chunk_ticks;
  std::vector<int> order(s->active.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return std::min<int64_t>(chunk, s->active[x].r.horizon - s->active[x].done) >
           std::min<int64_t>(chunk, s->active[y].r.horizon - s->active[y].done);
  });
  for (size_t i = 0; i < s->active.size(); ++i) {
    const fm_serve::Req& q = s->active[i];
    ReqDesc& d = hr[i];
    d.start_tick = q.r.start_tick;
    d.horizon = q.r.horizon;
    d.t0 = q.done;
    d.n_envs = q.r.n_envs;
    d.stride = q.r.stride;
    d.key = q.r.key;
    d.state = reinterpret_cast<fm_crypto_result*>(static_cast<unsigned char*>(s->cfg.d_pool) + q.pool_off);
    d.result = q.r.d_result;
    d.act = q.r.d_act;
    d.prob = q.r.d_prob;
  }
  for (int i : order) {
    const int tiles = (s->active[i].r.n_envs + s->rows - 1) / s->rows;
    for (int t = 0; t < tiles; ++t) hi[n_items++] = make_int2(i, t);
  }
  hipError_t e = hipMemcpyAsync(s->ws + s->L.reqs, hr, sizeof(ReqDesc) * s->active.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ws + s->L.items, hi, sizeof(int2) * n_items, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fm::device_error(e, "fm_serve_step (work lists)");
  fm::cx::ChunkArgs a{};
  a.mid = s->cfg.d_mid;
  a.feat = s->cfg.d_feat;
  a.P.w2 = reinterpret_cast<const fm::bf16x8*>(s->ws + s->L.w2);
  a.P.w1 = reinterpret_cast<const fm::cx::s16x4*>(s->ws + s->L.w1);
  a.P.w3 = reinterpret_cast<const fm::bf16x8*>(s->ws + s->L.w3);
  a.P.b1 = reinterpret_cast<const float*>(s->ws + s->L.b1);
  a.P.b2 = reinterpret_cast<const float*>(s->ws + s->L.b2);
  a.P.b3 = reinterpret_cast<const float*>(s->ws + s->L.b3);
  a.P.mix = reinterpret_cast<const float*>(s->ws + s->L.mix);
  a.rule = s->cfg.rule;
  a.eps = s->cfg.eps;
  a.fee = s->cfg.fee;
  a.cash0 = s->cfg.cash0;
  a.reqs = reinterpret_cast<const ReqDesc*>(s->ws + s->L.reqs);
  a.items = reinterpret_cast<const int2*>(s->ws + s->L.items);
  a.n_items = static_cast<int>(n_items);
  a.counter = reinterpret_cast<int*>(s->ws + s->L.counter);
  a.chunk = chunk;
  const int grid = static_cast<int>(std::min<int64_t>(s->grid, n_items));
  e = fm::cx::launch_chunk(s->rows, s->cfg.n_agents, a, grid, stream);
  if (e != hipSuccess) return fm::device_error(e, "fm_serve_step (launch)");
  const int64_t k = s->launched;
  e = hipEventRecord(s->ev[k % fm_serve::kEvents], stream);
  if (e != hipSuccess) return fm::device_error(e, "fm_serve_step (event)");
  s->launched = k + 1;
  s->stream = stream;
  s->stream_set = true;
  // Retire what this chunk finishes; its pool space is reusable by the next chunk.
  std::vector<int64_t> fin;
  std::vector<fm_serve::Req> keep;
  keep.reserve(s->active.size());
  for (fm_serve::Req& q : s->active) {
    q.done += std::min<int64_t>(chunk, q.r.horizon - q.done);
    if (q.done == q.r.horizon) {
      fin.push_back(q.id);
      s->pool.release(q.pool_off, q.pool_len);
      s->active_envs -= q.r.n_envs;
    } else {
      keep.push_back(q);
    }
  }
  s->active.swap(keep);
  if (!fin.empty()) s->finishing.emplace_back(k, std::move(fin));
  if (n_active) *n_active = static_cast<int32_t>(s->active.size());
  collect(s, false);
  return FM_OK;
}

fm_status fm_serve_poll(fm_serve* s, int32_t wait, int64_t* h_ids, int32_t cap, int32_t* n) {
  if (!s || !n || cap < 0 || (cap > 0 && !h_ids)) return set_error(FM_ERR_INVALID, "fm_serve_poll: bad arguments");
  fm::DeviceGuard guard(s->cfg.device);
  collect(s, wait != 0);
  const int32_t m = static_cast<int32_t>(std::min<size_t>(cap, s->done.size()));
  for (int32_t i = 0; i < m; ++i) h_ids[i] = s->done[i];
  s->done.erase(s->done.begin(), s->done.begin() + m);
  *n = m;
  return FM_OK;
}

void fm_serve_destroy(fm_serve* s) {
  if (!s) return;
  fm::DeviceGuard guard(s->cfg.device);
  if (s->launched > 0) (void)hipEventSynchronize(s->ev[(s->launched - 1) % fm_serve::kEvents]);
  for (int i = 0; i < fm_serve::kEvents; ++i)
    if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
  for (int i = 0; i < 2; ++i) {
    if (s->h_reqs[i]) (void)hipHostFree(s->h_reqs[i]);
    if (s->h_items[i]) (void)hipHostFree(s->h_items[i]);
  }
  delete s;
}

}  // extern "C"
