// Fused rollout: one launch runs every step of a closed-loop rollout for a tile of MR = 16*ROWT
// environments per workgroup.  Per step, inside the workgroup:
//   1. the K actors' three bfloat16 MFMA layers over the tile's state rows (activations in LDS,
//      weights streamed from L2), accumulating a_bar = sum_k w_k mu_k in float32;
//   2. Gaussian noise (Philox4x64-10 + Box-Muller) and a = clip(a_bar + sigma * eps, -1, 1);
//   3. the trading chain (lane m of wavefront 0 owns environment m): orders, sells, buys, the new
//      day's value in float64, reward, cumulative reward;
//   4. the next state, written once as bfloat16 into LDS for the next step's first layer and, if
//      requested, as float32 into the [T][N][S] trajectory.
// Environments are independent, so workgroups never communicate.
//
// Two MLP schedules:
//   * streamed (the 211 -> 256 -> 256 -> 30, K = 3 shape): eight wavefronts; every wavefront
//     owns fixed output tiles and walks a compile-time sequence of weight fragments (all layers
//     of all actors), keeping DEPTH k-steps of fragments in flight in registers.  The sequence
//     wraps around, so the first fragments of the next step load while the trading chain runs.
//   * generic (any supported shape): four wavefronts, runtime loops, one fragment at a time.
#include <algorithm>
#include <cstring>
#include <utility>

#include "device_common.h"
#include "fused.h"
#include "mlp_device.h"

namespace fm {

namespace {


// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1, fully unrolled.
template <class Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>());
}

// LDS layout shared by both schedules.
struct FusedLds {
  __bf16 *x0, *x1, *x2;  // state rows, layer-1 and layer-2 outputs
  float* abar;           // [MR][DS] ensemble mean
  float* act;            // [MR][D] noisy clipped action
  int* hold;             // [MR][D] holdings (the trading state, resident for the whole rollout)
  int* qty;              // [MR][D] executed shares
  float* env;            // [MR][DS] cash entry, holdings entries of the state rows
  float *px, *pn;        // closes of the trading day ([DP], entries beyond D unused) / new day [D]
  float* mkt;            // [(1+I)*D] scaled new close, new indicators
  ChainLds chain;        // the chain's scratch and the views above

  __host__ __device__ static size_t bytes(int MR, int st0, int sth, int D, int I) {
    const ChainShape Z = ChainShape::of(D);
    const size_t DS = D + 1;
    size_t b = Z.scratch_bytes(MR);
    b += sizeof(__bf16) * MR * (static_cast<size_t>(st0) + 2 * sth);
    b += sizeof(float) * MR * DS * 2 + sizeof(int) * MR * D * 2 + sizeof(float) * MR * D;
    b += sizeof(float) * (Z.DP + D + (1 + I) * D);
    return (b + 64 + 15) / 16 * 16;
  }
  __device__ void carve(unsigned char* smem, int MR, int st0, int sth, int D) {
    const ChainShape Z = ChainShape::of(D);
    const int DS = D + 1;
    unsigned char* p = chain.carve_scratch(smem, Z, MR);
    // 16-byte alignment for the bf16 MFMA operand rows.
    const size_t off = (static_cast<size_t>(p - smem) + 15) / 16 * 16;
    x0 = reinterpret_cast<__bf16*>(smem + off);
    x1 = x0 + MR * st0;
    x2 = x1 + MR * sth;
    abar = reinterpret_cast<float*>(x2 + MR * sth);
    env = abar + MR * DS;
    act = env + MR * DS;
    hold = reinterpret_cast<int*>(act + MR * D);
    qty = hold + MR * D;
    // px: 16-byte aligned for the serial phase's vector reads.
    const size_t poff = (reinterpret_cast<uintptr_t>(qty + MR * D) - reinterpret_cast<uintptr_t>(smem) + 15) / 16 * 16;
    px = reinterpret_cast<float*>(smem + poff);
    pn = px + Z.DP;
    mkt = pn + D;
    chain.act = act;
    chain.hold = hold;
    chain.qty = qty;
    chain.env = env;
    chain.px = px;
    chain.pn = pn;
  }
};

// Global-memory view of a pointer.  The batched form reads its groups' pointers from memory, and
// the compiler would access memory through such pointers with flat instructions, which also
// count on the LDS counter, so that the step's LDS waits would also wait for them.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// The environment half of a step, shared by both schedules.  NT threads per workgroup.
template <int NT>
struct EnvPhase {
  const EnvConst& C;
  const FusedArgs& F;
  FusedLds& L;
  int tid, lane, wave, n0, M, S_pad, st0;
  float inv_d, inv_g;
  int G;

  // Market rows of day tn (and the trading day tn-1 when trading) into LDS.
  __device__ void stage_market(int tn, bool with_trade_day) {
    const int D = C.D;
    for (int d = tid; d < D; d += NT) {
      if (with_trade_day) L.px[d] = gbl(C.close)[static_cast<size_t>(tn - 1) * D + d];
      const float pn = gbl(C.close)[static_cast<size_t>(tn) * D + d];
      L.pn[d] = pn;
      L.mkt[d] = pn * C.price_scale;
    }
    for (int i = tid; i < C.I * D; i += NT) L.mkt[D + i] = gbl(C.ind)[static_cast<size_t>(tn) * C.I * D + i];
  }

  // a = clip(a_bar + sigma * eps, -1, 1) into LDS (and the action trajectory).
  __device__ void actions(int t, size_t row_base) {
    const int D = C.D, DS = D + 1;
    for (int i = tid; i < M * G; i += NT) {
      const int m = div_small(i, inv_g);
      const int g = i - m * G;
      float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (F.sigma != 0.0f)
        noise_block(F.key, static_cast<uint64_t>(F.env_offset + n0 + m), static_cast<uint64_t>(t),
                    static_cast<uint64_t>(g), z);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = 4 * g + r;
        if (d < D) {
          float a = L.abar[m * DS + d];
          if (F.sigma != 0.0f) a = a + F.sigma * z[r];
          a = fminf(fmaxf(a, -1.0f), 1.0f);
          L.act[m * D + d] = a;
          if (F.act_traj) gbl(F.act_traj)[(row_base + m) * D + d] = a;
        }
      }
    }
  }

  // Cash and holdings entries of the state rows (owner lanes).
  __device__ void env_entries(bool owner, double cash) {
    if (!owner) return;
    const int D = C.D, DS = D + 1;
    float* erow = L.env + lane * DS;
    const int* hrow = L.hold + lane * D;
    erow[0] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
    for (int d = 0; d < D; ++d) erow[1 + d] = static_cast<float>(hrow[d]) * C.hold_scale;
  }

  // One step of the trading chain: parallel pre-terms (all threads), the serial cash recurrence
  // (owner lanes), parallel post-terms (all threads).  Returns the reward in the owner lanes.
  // Entered and left with all threads synchronised.
  __device__ double chain(bool owner, double& cash, double& asset, double& cumrew) {
    const ChainShape Z = ChainShape::of(C.D);
    const ChainLds& CL = L.chain;
    chain_day_terms(CL, Z, tid, NT, C.one_p);
    chain_pairs_a(CL, Z, M, tid, NT, C.hmax_f, C.one_m, C.one_p);
    __syncthreads();
    if (owner)
      chain_serial(cash, CL.pro + lane * Z.RD, CL.deb + lane * Z.RD, CL.c1, CL.rc1, CL.qd + lane * Z.RI, CL.px,
                   CL.kq + lane * Z.RI, Z.DP, C.one_p);
    __syncthreads();
    chain_pairs_c(CL, Z, M, tid, NT, C.hold_scale);
    __syncthreads();
    double r = 0.0;
    if (owner) {
      const double v_new = chain_value(cash, CL.val + lane * Z.RD, Z.DP);
      r = (v_new - asset) * C.reward_scale;
      cumrew = cumrew + r;
      asset = v_new;
      L.env[lane * Z.DS] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
    }
    return r;
  }

  // State rows: bfloat16 into x0 for the next first layer, float32 into the trajectory.  With
  // the split first layer (split_pad > 0) x0 holds only the per-environment entries [cash,
  // holdings] in split_pad columns; the market entries reach layer 1 through the day's table.
  // The (row, column) pairs are spread over all threads: consecutive threads write consecutive
  // entries of the tile's contiguous trajectory rows.
  __device__ void assemble(float* traj, int split_pad = 0) {
    const int D = C.D, DS = D + 1, S = C.S;
    const int W = split_pad > 0 ? S : S_pad;  // columns visited per row
    const float inv_w = 1.0f / static_cast<float>(W);
#pragma unroll 2
    for (int i = tid; i < M * W; i += NT) {
      const int m = div_small(i, inv_w);
      const int f = i - m * W;
      float v = 0.0f;
      if (f < S) {
        if (f == 0) v = L.env[m * DS];
        else if (f <= D) v = L.mkt[f - 1];
        else if (f <= 2 * D) v = L.env[m * DS + f - D];
        else v = L.mkt[f - 1 - D];
        if (traj) gbl(traj)[static_cast<size_t>(m) * S + f] = v;
      }
      if (split_pad == 0) L.x0[m * st0 + f] = static_cast<__bf16>(v);
    }
    if (split_pad > 0) {
      const float inv_p = 1.0f / static_cast<float>(split_pad);
      for (int i = tid; i < M * split_pad; i += NT) {
        const int m = div_small(i, inv_p);
        const int f = i - m * split_pad;
        L.x0[m * st0 + f] = static_cast<__bf16>(f <= D ? L.env[m * DS + f] : 0.0f);
      }
    }
  }

  __device__ void quantities(size_t row_base) {
    if (!F.qty_traj) return;
    const int D = C.D;
    for (int i = tid; i < M * D; i += NT) gbl(F.qty_traj)[row_base * D + i] = L.qty[i];
  }

  // Load the tile's state into the owner lanes (holdings into LDS).
  __device__ void load_state(bool owner, const EnvState& st, double& cash, double& asset, double& cumrew) {
    if (!owner) return;
    const int D = C.D, N = C.N, n = n0 + lane;
    cash = st.cash[n];
    asset = st.asset[n];
    cumrew = st.cumrew[n];
    for (int d = 0; d < D; ++d) L.hold[lane * D + d] = st.hold[static_cast<size_t>(d) * N + n];
  }
  __device__ void store_state(bool owner, const EnvState& st, double cash, double asset, double cumrew) {
    if (!owner) return;
    const int D = C.D, N = C.N, n = n0 + lane;
    st.cash[n] = cash;
    st.asset[n] = asset;
    st.cumrew[n] = cumrew;
    for (int d = 0; d < D; ++d) st.hold[static_cast<size_t>(d) * N + n] = L.hold[lane * D + d];
  }
};

// ------------------------------------------------------------------------------------------
// Generic MLP schedule (runtime shapes): wavefront w owns output tiles w, w+4, ...; the weight
// fragments of the next four k-steps are in flight in a register ring while the current ones are
// multiplied (the ensemble MLP's layer loop).  The epilogue gets (row tile, slot i, tile c).
// ------------------------------------------------------------------------------------------
template <int ROWT, int TMAX, class Epi>
__device__ __forceinline__ void layer_bf16(const __bf16* sin, int ist, int kin_pad, const bf16x8* W,
                                           int ntiles, int wave, int lane, Epi epi) {
  mlp_layer<kBF16, TMAX, ROWT, 4, Epi, 4>(sin, ist, kin_pad, W, ntiles, wave, lane, epi);
}

// ------------------------------------------------------------------------------------------
// Streamed MLP schedule for K = 3, H = 256, A_pad = 32 over the split first layer: layer 1 runs
// on the per-environment entries only (KKE k-steps of 32 rows: cash, holdings, zero padding),
// its market share comes from the day's table.  NWAVES wavefronts; in layers 1 and 2 wavefront w
// owns output tiles w, w+NWAVES, ...; layer 3 (two output tiles) is split over the K dimension:
// wavefront w takes k-blocks w*L3 .. w*L3+L3-1 of both tiles and leaves partial sums, which the
// action phase adds up.  Every wavefront requests the same number of fragments at every
// position, so the wait counts of the register ring are exact.  Its weight fragments form a
// fixed sequence of NS k-steps per environment step; fragments for k-step s+DEPTH are requested
// when k-step s is consumed.
// ------------------------------------------------------------------------------------------
template <int KKE, int ROWT, int DEPTH, int NWAVES>
struct Streamed {
  static constexpr int K = 3, KK2 = 8, HT = 16, AT = 2, NW = NWAVES, TW = HT / NWAVES;
  static constexpr int L3 = KK2 / NWAVES;          // layer-3 k-steps per wavefront
  static constexpr int SPA = KKE + KK2 + L3;       // k-steps per actor
  static constexpr int NS = K * SPA;               // k-steps per environment step
  static_assert(TW >= AT, "a ring slot holds the layer-3 fragments of both tiles");
  // The schedule walks NSP >= NS positions per step, a multiple of DEPTH, so that k-step j always
  // uses ring slot j % DEPTH, also across the wrap into the next step; positions >= NS are idle.
  static constexpr int NSP = (NS + DEPTH - 1) / DEPTH * DEPTH;

  // Packed-ensemble layout of this shape (bytes; checked against the workspace on the host):
  // per actor W1 (224 rows), W2, W3, b1, b2, b3; the env-row fragments of all actors elsewhere.
  static constexpr size_t kW2 = 224 * 256 * 2, kW3 = kW2 + 256 * 256 * 2;
  static constexpr size_t kB1 = kW3 + 256 * 32 * 2, kB2 = kB1 + 1024, kB3 = kB2 + 1024;
  static constexpr size_t kActor = kB3 + 256;
  static constexpr size_t kW1eActor = static_cast<size_t>(KKE) * HT * 1024;

  // Weight fragments of k-step S2 for wavefront wv (uniform); voff = lane * 16.
  template <int S2>
  static __device__ __forceinline__ void load(bf16x8 (&b)[TW], const unsigned char* wb, const unsigned char* w1e,
                                              int wv, int voff) {
    if constexpr (S2 >= NS) return;  // idle position
    constexpr int actor = S2 / SPA, r = S2 % SPA;
    if constexpr (r < KKE) {
      const unsigned char* P = w1e + kW1eActor * actor;
#pragma unroll
      for (int i = 0; i < TW; ++i)
        b[i] = *reinterpret_cast<const bf16x8*>(P + static_cast<size_t>((wv + NW * i) * KKE + r) * 1024 + voff);
    } else if constexpr (r < KKE + KK2) {
      constexpr int kk = r - KKE;
      const unsigned char* P = wb + kActor * actor;
#pragma unroll
      for (int i = 0; i < TW; ++i)
        b[i] = *reinterpret_cast<const bf16x8*>(P + kW2 + static_cast<size_t>((wv + NW * i) * KK2 + kk) * 1024 + voff);
    } else {
      constexpr int j = r - KKE - KK2;
      const int kk = wv * L3 + j;
      const unsigned char* P = wb + kActor * actor;
#pragma unroll
      for (int c = 0; c < AT; ++c)
        b[c] = *reinterpret_cast<const bf16x8*>(P + kW3 + static_cast<size_t>(c * KK2 + kk) * 1024 + voff);
    }
  }
};

// ------------------------------------------------------------------------------------------
// Per-chunk tables of the streamed kernel, made before it by two small kernels:
//   mt[c][k][j]: actor k's layer-1 pre-activation share of the market entries of state s_t
//     (t = t0 + c), b1_k[j] + sum_f bf16(x_f) * W1m_k[f][j] in float32 -- the same for every
//     environment of day t, so it is computed once per day instead of once per environment;
//   eps[c][n][d]: the noise of step t for environment n (Philox4x64-10 + Box-Muller).
// ------------------------------------------------------------------------------------------
// One workgroup per (kMtDays days, actor), thread j per hidden unit: each weight load serves
// kMtDays days, and the weights are requested 64 at a time before they are used, so the load
// latency is paid a few times per unit rather than once per few entries.  Each sum still runs
// over f in ascending order, one rounding per product and per addition; the entries are padded
// with zeros to whole batches (a zero product added to a sum that starts at +0 changes nothing).
constexpr int kMtDays = 2, kMtBatch = 64;
__host__ __device__ constexpr int mt_row(int Fm) { return (Fm + kMtBatch - 1) / kMtBatch * kMtBatch; }
// A few hundred workgroups at most: registers for the batch matter more than occupancy.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
void market_table_kernel(EnvConst C, EnsDev E, int t0, int n_days, float* __restrict__ mt) {
  extern __shared__ float xs[];  // [kMtDays][Fp]: the days' market entries, bfloat16-rounded, zero-padded
  const int c0 = blockIdx.x * kMtDays, k = blockIdx.y;
  const int D = C.D, I = C.I, Fm = (1 + I) * D, H = E.H, Fp = mt_row(Fm);
  for (int i = threadIdx.x; i < kMtDays * Fp; i += blockDim.x) {
    const int dd = i / Fp, f = i - dd * Fp, t = t0 + c0 + dd;
    float v = 0.0f;
    if (c0 + dd < n_days && f < Fm)
      v = f < D ? C.close[static_cast<size_t>(t) * D + f] * C.price_scale
                : C.ind[static_cast<size_t>(t) * I * D + (f - D)];
    xs[i] = static_cast<float>(static_cast<__bf16>(v));
  }
  __syncthreads();
  const __bf16* w = reinterpret_cast<const __bf16*>(E.base + E.off_w1m) + static_cast<size_t>(k) * Fm * H;
  const float* b1 = reinterpret_cast<const float*>(E.base + k * E.actor_stride + E.off_b1);
  for (int j = threadIdx.x; j < H; j += blockDim.x) {
    float acc[kMtDays];
#pragma unroll
    for (int dd = 0; dd < kMtDays; ++dd) acc[dd] = 0.0f;
    for (int f0 = 0; f0 < Fm; f0 += kMtBatch) {
      float wv[kMtBatch];
#pragma unroll
      for (int q = 0; q < kMtBatch; ++q) wv[q] = static_cast<float>(w[static_cast<size_t>(min(f0 + q, Fm - 1)) * H + j]);
#pragma unroll
      for (int q = 0; q < kMtBatch; ++q)
#pragma unroll
        for (int dd = 0; dd < kMtDays; ++dd) acc[dd] = acc[dd] + xs[dd * Fp + f0 + q] * wv[q];
    }
#pragma unroll
    for (int dd = 0; dd < kMtDays; ++dd)
      if (c0 + dd < n_days) mt[(static_cast<size_t>(c0 + dd) * E.K + k) * H + j] = acc[dd] + b1[j];
  }
}

__global__ void noise_chunk_kernel(uint64_t key, int64_t env_offset, int t0, int n_days, int N, int D,
                                   float* __restrict__ eps) {
  const int G = (D + 3) >> 2;
  const size_t total = static_cast<size_t>(n_days) * N * G;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int g = static_cast<int>(i % G);
  const size_t rest = i / G;
  const int n = static_cast<int>(rest % N);
  const int c = static_cast<int>(rest / N);
  float z[4];
  noise_block(key, static_cast<uint64_t>(env_offset + n), static_cast<uint64_t>(t0 + c), static_cast<uint64_t>(g), z);
  float* row = eps + (static_cast<size_t>(c) * N + n) * D;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (4 * g + r < D) row[4 * g + r] = z[r];
}

// ------------------------------------------------------------------------------------------
// Streamed kernel.  Five wavefronts with two roles:
//   wavefronts 0-3 (MLP): the three layers of the K actors for the tile's state rows, weight
//     fragments streamed through a register ring; then the trading chain: the parallel phases
//     over (env, stock) pairs (actions, orders and sells; buys applied, holdings entries of the
//     next state rows) and the serial ones, where lane l of wavefront w runs environment
//     w*MR/4 + l (the cash recurrence, then the value and reward);
//   wavefront 4 (memory): during the MLP of step t, the staging of step t+1's inputs (market
//     rows, noise, market table) from registers into LDS and the requests for step t+2's; while
//     the cash recurrences of step t run, the stores of step t-1's results.  Its vector-memory
//     traffic never delays the MLP wavefronts' weight waits, which count only their own
//     requests.
// The two roles run separate loops that pass the same sequence of workgroup barriers per step.
// The trading state (cash, value, cumulative reward, holdings) stays in LDS for the launch.
// State rows, actions, quantities, state entries, rewards, noise and table rows are
// double-buffered by step parity; the market rows [close[t] | close[t+1] | ind[t+1]] are
// triple-buffered by step (the results of step t read them during step t+1).
// ------------------------------------------------------------------------------------------
constexpr int kMlpWaves = 4;
constexpr int kStreamThreads = 64 * (kMlpWaves + 1);
constexpr int kStreamK = 3, kStreamH = 256;
constexpr int kBiasStride = 2 * kStreamH;  // b2 | b3 (padded) per actor
constexpr int kMktStage = 10;              // registers per lane: (2 + I) * D <= 640
constexpr int kTabStage = kStreamK * kStreamH / 64;

struct StreamLds {
  // Double- and triple-buffered regions are a base and a buffer stride (in elements): buffer b
  // starts at base + b * stride.
  __bf16* x0_;    // [2][MR][ST0] state-row entries of the environments (cash, holdings)
  __bf16* x1;     // [MR][STH]
  __bf16* x2;     // [MR][STH]
  float* bias;    // [K][kBiasStride]
  float* mix;     // [K]
  float* part;    // [K][NW][MR][32] layer-3 partial sums by actor and wavefront
  float* eps_;    // [2][MR][D] noise
  float* mt_;     // [2][K][H] layer-1 market share
  float* act_;    // [2][MR][D]
  int* qty_;      // [2][MR][D]
  float* env_;    // [2][MR][DS] cash entry, holdings entries
  double* rew_;   // [2][MR]
  int* hold;      // [MR][D]
  double* cash;   // [MR] the trading state: cash, pre-trade value, cumulative reward
  double* asset;  // [MR]
  double* cumrew; // [MR]
  float* in_;     // [3][IN] market rows of a step
  int x0s, epss, mts, acts, qtys, envs, rews, ins;
  ChainLds chain;

  __device__ __bf16* x0(int b) const { return x0_ + b * x0s; }
  __device__ float* eps(int b) const { return eps_ + b * epss; }
  __device__ float* mt(int b) const { return mt_ + b * mts; }
  __device__ float* act(int b) const { return act_ + b * acts; }
  __device__ int* qty(int b) const { return qty_ + b * qtys; }
  __device__ float* env(int b) const { return env_ + b * envs; }
  __device__ double* rew(int b) const { return rew_ + b * rews; }
  __device__ float* in(int b) const { return in_ + b * ins; }

  static __host__ __device__ size_t a16(size_t b) { return (b + 15) / 16 * 16; }
  // Byte offsets of the regions and the total.
  struct Offsets {
    size_t sc, x0, x1, x2, bias, mix, part, eps, mt, act, qty, env, rew, hold, state, in, total;
    size_t x0b, epsb, mtb, actb, qtyb, envb, rewb, inb;  // bytes per buffer
  };
  __host__ __device__ static Offsets offsets(int MR, int st0, int sth, int D, int I) {
    const ChainShape Z = ChainShape::of(D);
    const size_t DS = D + 1;
    Offsets o{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
      const size_t a = a16(p);
      p = a + bytes;
      return a;
    };
    o.x0b = a16(sizeof(__bf16) * MR * st0);
    o.epsb = a16(sizeof(float) * MR * D);
    o.mtb = a16(sizeof(float) * kStreamK * kStreamH);
    o.actb = a16(sizeof(float) * MR * D);
    o.qtyb = a16(sizeof(int) * MR * D);
    o.envb = a16(sizeof(float) * MR * DS);
    o.rewb = a16(sizeof(double) * MR);
    const size_t nin = static_cast<size_t>(2 + I) * D;
    o.inb = a16(sizeof(float) * (nin > static_cast<size_t>(Z.DP) ? nin : static_cast<size_t>(Z.DP)));
    // The chain's scratch (used after the MLP) shares its region with the layer-1/2 outputs
    // (used during the MLP only).
    const size_t xb = a16(sizeof(__bf16) * MR * sth);
    const size_t region = Z.scratch_bytes(MR) > 2 * xb ? Z.scratch_bytes(MR) : 2 * xb;
    o.sc = take(region);
    o.x1 = o.sc;
    o.x2 = o.sc + xb;
    o.x0 = take(2 * o.x0b);
    o.bias = take(sizeof(float) * kStreamK * kBiasStride);
    o.mix = take(sizeof(float) * kStreamK);
    o.part = take(sizeof(float) * kStreamK * kMlpWaves * MR * 32);
    o.eps = take(2 * o.epsb);
    o.mt = take(2 * o.mtb);
    o.act = take(2 * o.actb);
    o.qty = take(2 * o.qtyb);
    o.env = take(2 * o.envb);
    o.rew = take(2 * o.rewb);
    o.hold = take(sizeof(int) * MR * D);
    o.state = take(sizeof(double) * 3 * MR);
    o.in = take(3 * o.inb);
    o.total = a16(p);
    return o;
  }
  __device__ void carve(unsigned char* smem, int MR, int st0, int sth, int D, int I) {
    const Offsets o = offsets(MR, st0, sth, D, I);
    x0_ = reinterpret_cast<__bf16*>(smem + o.x0);
    x1 = reinterpret_cast<__bf16*>(smem + o.x1);
    x2 = reinterpret_cast<__bf16*>(smem + o.x2);
    bias = reinterpret_cast<float*>(smem + o.bias);
    mix = reinterpret_cast<float*>(smem + o.mix);
    part = reinterpret_cast<float*>(smem + o.part);
    eps_ = reinterpret_cast<float*>(smem + o.eps);
    mt_ = reinterpret_cast<float*>(smem + o.mt);
    act_ = reinterpret_cast<float*>(smem + o.act);
    qty_ = reinterpret_cast<int*>(smem + o.qty);
    env_ = reinterpret_cast<float*>(smem + o.env);
    rew_ = reinterpret_cast<double*>(smem + o.rew);
    hold = reinterpret_cast<int*>(smem + o.hold);
    cash = reinterpret_cast<double*>(smem + o.state);
    asset = cash + MR;
    cumrew = asset + MR;
    in_ = reinterpret_cast<float*>(smem + o.in);
    x0s = static_cast<int>(o.x0b / sizeof(__bf16));
    epss = static_cast<int>(o.epsb / sizeof(float));
    mts = static_cast<int>(o.mtb / sizeof(float));
    acts = static_cast<int>(o.actb / sizeof(float));
    qtys = static_cast<int>(o.qtyb / sizeof(int));
    envs = static_cast<int>(o.envb / sizeof(float));
    rews = static_cast<int>(o.rewb / sizeof(double));
    ins = static_cast<int>(o.inb / sizeof(float));
    chain.carve_scratch(smem + o.sc, ChainShape::of(D), MR);
    chain.hold = hold;
  }
};

template <int ROWT, int KKE, int DEPTH>
__global__ __launch_bounds__(kStreamThreads) void fused_streamed_kernel(EnvConst C, EnvState st, EnsDev E,
                                                                        FusedArgs F) {
  using SP = Streamed<KKE, ROWT, DEPTH, kMlpWaves>;
  constexpr int MR = 16 * ROWT, TW = SP::TW, NW = SP::NW, NT = kStreamThreads;
  constexpr int KK2 = SP::KK2, SPA = SP::SPA, NS = SP::NS, NSP = SP::NSP;
  constexpr int H = kStreamH, K = kStreamK;
  constexpr int ST0 = 32 * KKE + 8, STH = H + 8;
  constexpr int NBAR = 2 * K + 1;                 // layer-end barriers per step
  constexpr int EPS_STAGE = (MR * 32 + 63) / 64;  // registers per lane for a step's noise (D <= 32)
  constexpr int SPW = MR / kMlpWaves;             // environments per MLP wavefront in the serial phases
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int D = C.D, N = C.N, DS = D + 1, S = C.S, I = C.I;
  // A workgroup owns tile_envs <= MR environments; the MFMA rows beyond them stay zero, as in a
  // ragged last tile.  Smaller tiles spread a small N over every compute unit.
  const int n0 = blockIdx.x * F.tile_envs;
  const int M = min(F.tile_envs, N - n0);
  const ChainShape Z = ChainShape::of(D);

  StreamLds L;
  L.carve(smem, MR, ST0, STH, D, I);

  // Zero both state-row buffers (padding columns and the rows of absent environments stay
  // zero); layer-2/3 biases and mixing weights into LDS.
  for (int b = 0; b < 2; ++b)
    for (int i = tid; i < MR * ST0; i += NT) L.x0(b)[i] = static_cast<__bf16>(0.0f);
  for (int i = tid; i < K * kBiasStride; i += NT) {
    const int a = i / kBiasStride, c = i - a * kBiasStride;
    const size_t off = c < H ? SP::kB2 + 4 * c : SP::kB3 + 4 * (c - H);
    L.bias[i] = (c < H + 32) ? *reinterpret_cast<const float*>(E.base + SP::kActor * a + off) : 0.0f;
  }
  for (int i = tid; i < K; i += NT) L.mix[i] = E.mix[i];
  __syncthreads();

  if (wave < NW) {
    // ---------------------------------------------------------------- MLP wavefronts
    const int wv = wave;
    const int voff = lane * 16;
    bf16x8 ring[DEPTH][TW];
    static_for<DEPTH>([&](auto sc) __attribute__((always_inline)) {
      constexpr int s = decltype(sc)::value;
      SP::template load<s>(ring[s], E.base, E.base + E.off_w1e, wv, voff);
    });
    const int row_q = 4 * (lane >> 4), col_l = lane & 15, row = lane & 15, grp = lane >> 4;
    const float sigma = F.sigma;
    __syncthreads();  // the first state rows and inputs are staged

    for (int it = 0; it < F.n_steps; ++it) {
      __syncthreads();  // T: state rows of step it complete
      // The weight bases are offset by an opaque zero every step, so that no fragment address
      // is hoisted out of the step loop (there are hundreds of them).  Laundering an integer
      // rather than the pointer keeps the loads in the global address space (flat loads would
      // also count against the LDS wait counter).
      int opaque_zero = 0;
      asm volatile("" : "+s"(opaque_zero));
      const unsigned char* wb = E.base + opaque_zero;
      const unsigned char* w1e = E.base + (E.off_w1e + opaque_zero);
      const __bf16* xin = L.x0(it & 1);
      const float* mtab = L.mt(it & 1);

      floatx4 acc[ROWT][TW];
      static_for<NSP>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        // Keep the k-steps in program order: the scheduler would otherwise hoist every load of
        // a layer to its top and run out of registers.
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (s >= NS) {
          SP::template load<(s + DEPTH) % NSP>(ring[s % DEPTH], wb, w1e, wv, voff);
          return;
        }
        constexpr int actor = s / SPA, r = s % SPA;
        constexpr int layer = r < KKE ? 1 : (r < KKE + KK2 ? 2 : 3);
        constexpr int kk = layer == 1 ? r : (layer == 2 ? r - KKE : r - KKE - KK2);
        constexpr int first = layer == 1 ? 0 : (layer == 2 ? KKE : KKE + KK2);
        constexpr int last = layer == 1 ? KKE - 1 : (layer == 2 ? KKE + KK2 - 1 : SPA - 1);
        if constexpr (r == first) {
#pragma unroll
          for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
            for (int i = 0; i < TW; ++i) acc[rt][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        bf16x8 cur[TW];
#pragma unroll
        for (int i = 0; i < TW; ++i) cur[i] = ring[s % DEPTH][i];
        SP::template load<(s + DEPTH) % NSP>(ring[s % DEPTH], wb, w1e, wv, voff);

        const __bf16* src = layer == 1 ? xin : (layer == 2 ? L.x1 : L.x2);
        constexpr int ist = layer == 1 ? ST0 : STH;
        const int kcol = layer == 3 ? 32 * (wv * SP::L3 + kk) : 32 * kk;
        bf16x8 a[ROWT];
#pragma unroll
        for (int rt = 0; rt < ROWT; ++rt)
          a[rt] = *reinterpret_cast<const bf16x8*>(src + (rt * 16 + row) * ist + kcol + 8 * grp);
        if constexpr (layer < 3) {
#pragma unroll
          for (int i = 0; i < TW; ++i)
#pragma unroll
            for (int rt = 0; rt < ROWT; ++rt) acc[rt][i] = mfma_bf16(a[rt], cur[i], acc[rt][i]);
        } else {
#pragma unroll
          for (int c = 0; c < SP::AT; ++c)
#pragma unroll
            for (int rt = 0; rt < ROWT; ++rt) acc[rt][c] = mfma_bf16(a[rt], cur[c], acc[rt][c]);
        }

        if constexpr (r == last) {
          if constexpr (layer < 3) {
            // Layer 1 adds the day's market share (bias included); layer 2 its bias.
            const float* b = layer == 1 ? mtab + actor * H : L.bias + actor * kBiasStride;
            __bf16* out = layer == 1 ? L.x1 : L.x2;
#pragma unroll
            for (int i = 0; i < TW; ++i) {
              const int col = 16 * (wv + NW * i) + col_l;
              const float bc = b[col];
#pragma unroll
              for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                  out[(rt * 16 + row_q + q) * STH + col] = static_cast<__bf16>(fast_tanh(acc[rt][i][q] + bc));
            }
            __syncthreads();  // layer end
          } else {
            // This wavefront's share of the layer-3 sums of this actor.
            float* pp = L.part + (actor * NW + wv) * MR * 32;
#pragma unroll
            for (int c = 0; c < SP::AT; ++c)
#pragma unroll
              for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) pp[(rt * 16 + row_q + q) * 32 + 16 * c + col_l] = acc[rt][c][q];
            if constexpr (actor == K - 1) __syncthreads();  // all partial sums written
          }
        }
      });

      // Actions a = clip(a_bar + sigma * eps), orders, sells, debits; the day's reciprocals.
      const float* in = L.in(it % 3);
      const float* eps = L.eps(it & 1);
      ChainLds CL = L.chain;
      CL.px = in;
      CL.pn = in + D;
      CL.qty = L.qty(it & 1);
      CL.env = L.env(it & 1);
      float* actb = L.act(it & 1);
      chain_day_terms(CL, Z, tid, 64 * NW, C.one_p);
      chain_pairs_a(CL, Z, M, tid, 64 * NW, C.hmax_f, C.one_m, C.one_p, [&](int m, int d, int e) {
        // a_bar = sum_k w_k tanh(z_k + b3_k), z_k the sum of the wavefronts' partial sums.
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float* pk = L.part + k * NW * MR * 32 + m * 32 + d;
          float z = pk[0];
#pragma unroll
          for (int w = 1; w < NW; ++w) z = z + pk[w * MR * 32];
          const float v = L.mix[k] * fast_tanh(z + L.bias[k * kBiasStride + H + d]);
          a = k == 0 ? v : a + v;
        }
        if (sigma != 0.0f) a = a + sigma * eps[e];
        a = fminf(fmaxf(a, -1.0f), 1.0f);
        actb[e] = a;
        return a;
      });
      __syncthreads();  // A
      // The cash recurrences: lane l of wavefront w runs environment w*SPW + l.
      const int me = wv * SPW + lane;
      const bool mine = lane < SPW && me < M;
      if (mine) {
        double cash = L.cash[me];
        chain_serial<4>(cash, CL.pro + me * Z.RD, CL.deb + me * Z.RD, CL.c1, CL.rc1, CL.qd + me * Z.RI, in,
                        CL.kq + me * Z.RI, Z.DP, C.one_p);
        L.cash[me] = cash;
      }
      __syncthreads();  // S
      __bf16* xn = L.x0((it + 1) & 1);
      chain_pairs_c(CL, Z, M, tid, 64 * NW, C.hold_scale,
                    [&](int m, int d, float he) { xn[m * ST0 + 1 + d] = static_cast<__bf16>(he); });
      __syncthreads();  // C
      if (mine) {
        const double cash = L.cash[me];
        const double v_new = chain_value<4>(cash, CL.val + me * Z.RD, Z.DP);
        const double r = (v_new - L.asset[me]) * C.reward_scale;
        L.cumrew[me] = L.cumrew[me] + r;
        L.asset[me] = v_new;
        const float ce = static_cast<float>(cash * static_cast<double>(C.cash_scale));
        CL.env[me * DS] = ce;
        xn[me * ST0] = static_cast<__bf16>(ce);
        L.rew(it & 1)[me] = r;
      }
    }
    __syncthreads();  // end
    return;
  }

  // ------------------------------------------------------------------ memory wavefront
  const bool owner = lane < M;
  const int n = n0 + lane;
  if (owner) {
    L.cash[lane] = st.cash[n];
    L.asset[lane] = st.asset[n];
    L.cumrew[lane] = st.cumrew[n];
    for (int d = 0; d < D; ++d) L.hold[lane * D + d] = st.hold[static_cast<size_t>(d) * N + n];
  }
  const int n_mkt = (2 + I) * D, MD = M * D;
  // Inputs of step j: market rows close[t] | close[t+1] | ind[t+1] (t = t0 + j), the tile's noise
  // rows, the market table of day t.
  float stg_m[kMktStage], stg_e[EPS_STAGE], stg_t[kTabStage];
  auto issue = [&](int j) {
    const int t = F.t0 + j;
#pragma unroll
    for (int r = 0; r < kMktStage; ++r) {
      const int i = lane + 64 * r;
      float v = 0.0f;
      if (i < D) v = C.close[static_cast<size_t>(t) * D + i];
      else if (i < 2 * D) v = C.close[static_cast<size_t>(t + 1) * D + (i - D)];
      else if (i < n_mkt) v = C.ind[static_cast<size_t>(t + 1) * I * D + (i - 2 * D)];
      stg_m[r] = v;
    }
    const float* e = F.eps + (static_cast<size_t>(j) * N + n0) * D;
#pragma unroll
    for (int r = 0; r < EPS_STAGE; ++r) {
      const int i = lane + 64 * r;
      stg_e[r] = i < MD ? e[i] : 0.0f;
    }
    const float* tb = F.mt + static_cast<size_t>(j) * K * H;
#pragma unroll
    for (int r = 0; r < kTabStage; ++r) stg_t[r] = tb[lane + 64 * r];
  };
  auto commit = [&](int j) {
    float* in = L.in(j % 3);
#pragma unroll
    for (int r = 0; r < kMktStage; ++r) {
      const int i = lane + 64 * r;
      if (i < n_mkt) in[i] = stg_m[r];
    }
    float* e = L.eps(j & 1);
#pragma unroll
    for (int r = 0; r < EPS_STAGE; ++r) {
      const int i = lane + 64 * r;
      if (i < MD) e[i] = stg_e[r];
    }
    float* tb = L.mt(j & 1);
#pragma unroll
    for (int r = 0; r < kTabStage; ++r) tb[lane + 64 * r] = stg_t[r];
  };
  auto results = [&](int j) {
    const size_t row0 = static_cast<size_t>(j) * N + n0;
    if (F.rew_traj && owner) F.rew_traj[row0 + lane] = L.rew(j & 1)[lane];
    if (F.act_traj) {
      const float* a = L.act(j & 1);
      wave_store_row(F.act_traj + row0 * D, MD, lane, [&](int i) { return a[i]; });
    }
    if (F.qty_traj) {
      const int* q = L.qty(j & 1);
      wave_store_row(F.qty_traj + row0 * D, MD, lane, [&](int i) { return q[i]; });
    }
    if (F.obs_traj) store_state_rows(F.obs_traj + row0 * S, M, S, D, L.env(j & 1), DS, L.in(j % 3), C.price_scale, lane);
  };

  // The first state rows: the cash and holdings entries.
  if (owner) {
    __bf16* x = L.x0(0) + lane * ST0;
    x[0] = static_cast<__bf16>(static_cast<float>(L.cash[lane] * static_cast<double>(C.cash_scale)));
    for (int d = 0; d < D; ++d) x[1 + d] = static_cast<__bf16>(static_cast<float>(L.hold[lane * D + d]) * C.hold_scale);
  }
  issue(0);
  commit(0);
  if (F.n_steps > 1) issue(1);
  __syncthreads();  // the first state rows and inputs are staged

  for (int it = 0; it < F.n_steps; ++it) {
    __syncthreads();  // T
    // During layer 1 of the first actor: step it+1's inputs into LDS (no HBM traffic).
    if (it + 1 < F.n_steps) commit(it + 1);
    __syncthreads();  // end of layer 1 of the first actor
    // During layer 2: the requests for step it+2's inputs.
    if (it + 2 < F.n_steps) issue(it + 2);
    for (int b = 1; b < NBAR; ++b) __syncthreads();  // the other layer ends
    __syncthreads();                                 // A
    if (it >= 1) results(it - 1);                    // while the cash recurrences run
    __syncthreads();  // S
    __syncthreads();  // C
  }
  __syncthreads();  // end
  if (F.n_steps >= 1) results(F.n_steps - 1);
  if (owner) {
    st.cash[n] = L.cash[lane];
    st.asset[n] = L.asset[lane];
    st.cumrew[n] = L.cumrew[lane];
    for (int d = 0; d < D; ++d) st.hold[static_cast<size_t>(d) * N + n] = L.hold[lane * D + d];
  }
}

// One tile (16*ROWT environments starting at tile*16*ROWT) through the steps of F, generic
// schedule: the body of the generic kernel and of the batched persistent kernel.
template <int ROWT, int TMAX>
__device__ __forceinline__ void generic_tile(const EnvConst& C, const EnvState& st, const EnsDev& E,
                                             const FusedArgs& F, int tile, unsigned char* smem) {
  constexpr int NT = 256, MR = 16 * ROWT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int D = C.D, N = C.N, DS = D + 1;
  const int n0 = tile * MR;
  const int M = min(MR, N - n0);
  // Split first layer when the day's market tables come with the launch (F.mt, [n_steps][K][H],
  // bias included): layer 1 runs on the ke_pad per-environment entries only.
  const int split_pad = F.mt != nullptr ? E.ke_pad : 0;
  const int st0 = (split_pad > 0 ? split_pad : E.S_pad) + 8, sth = E.H + 8;

  FusedLds L;
  L.carve(smem, MR, st0, sth, D);
  EnvPhase<NT> P{C, F, L, tid, lane, wave, n0, M, E.S_pad, st0, 1.0f / static_cast<float>(D),
                 1.0f / static_cast<float>((D + 3) >> 2), (D + 3) >> 2};

  for (int i = tid; i < MR * st0; i += NT) L.x0[i] = static_cast<__bf16>(0.0f);

  const bool owner = wave == 0 && lane < M;
  const int n = n0 + lane;
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  P.load_state(owner, st, cash, asset, cumrew);

  P.stage_market(F.t0, false);
  P.env_entries(owner, cash);
  __syncthreads();
  P.assemble(nullptr, split_pad);

  const int row_q = 4 * (lane >> 4), col_l = lane & 15;
  const int ht = E.H / 16, at = E.A_pad / 16;
  // Layer 3's k-range slices: the wavefronts left over by its output tiles (partial tiles of
  // sl3 * at * ROWT * 1024 bytes in the layer-1 output area).
  const int kk3 = E.H / 32;
  int sl3 = at < 4 ? min(4 / at, kk3) : 1;
  while (sl3 > 1 && sl3 * at * ROWT * 1024 > MR * sth * 2) --sl3;

  for (int it = 0; it < F.n_steps; ++it) {
    const int t = F.t0 + it;
    const size_t row_base = static_cast<size_t>(it) * N + n0;
    __syncthreads();
    P.stage_market(t + 1, true);

    for (int k = 0; k < E.K; ++k) {
      const unsigned char* PA = E.base + static_cast<size_t>(k) * E.actor_stride;
      const float* b1 = reinterpret_cast<const float*>(PA + E.off_b1);
      const float* b2 = reinterpret_cast<const float*>(PA + E.off_b2);
      const float* b3 = reinterpret_cast<const float*>(PA + E.off_b3);
      const float wk = gbl(E.mix)[k];
      // Layer 1's bias, or with the split layer the day's market share (bias included).
      const float* b1t = split_pad > 0 ? F.mt + (static_cast<size_t>(it) * E.K + k) * E.H : b1;
      const bf16x8* W1 = split_pad > 0
                             ? reinterpret_cast<const bf16x8*>(E.base + E.off_w1e +
                                                               static_cast<size_t>(k) * E.H * split_pad * 2)
                             : reinterpret_cast<const bf16x8*>(PA + E.off_w1);
      // Each layer's biases for the wavefront's output tiles are requested before its k loop, so
      // that the epilogues do not wait for them (up to four tiles per wavefront; with eight the
      // registers are short, and the epilogue reads its bias).
      constexpr bool kPre = TMAX <= 4;
      float bv[TMAX];
      const float* bsrc = nullptr;
      auto bias = [&](const float* b, int ntiles, int n) {  // n: the layer's outputs
        bsrc = b;
        if constexpr (kPre) {
#pragma unroll
          for (int i = 0; i < TMAX; ++i) {
            const int c = wave + 4 * i;
            bv[i] = c < ntiles && 16 * c + col_l < n ? gbl(b)[16 * c + col_l] : 0.0f;
          }
        }
      };
      auto bias_of = [&](int i, int col) -> float {
        if constexpr (kPre) return bv[i];
        else return gbl(bsrc)[col];
      };
      bias(b1t, ht, E.H);
      layer_bf16<ROWT, TMAX>(L.x0, st0, split_pad > 0 ? split_pad : E.S_pad, W1, ht, wave, lane,
                             [&](int rt, int i, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               const float b = bias_of(i, col);
#pragma unroll
                               for (int q = 0; q < 4; ++q)
                                 L.x1[(rt * 16 + row_q + q) * sth + col] = static_cast<__bf16>(fast_tanh(acc[q] + b));
                             });
      bias(b2, ht, E.H);
      __syncthreads();
      layer_bf16<ROWT, TMAX>(L.x1, sth, E.H, reinterpret_cast<const bf16x8*>(PA + E.off_w2), ht, wave, lane,
                             [&](int rt, int i, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               const float b = bias_of(i, col);
#pragma unroll
                               for (int q = 0; q < 4; ++q)
                                 L.x2[(rt * 16 + row_q + q) * sth + col] = static_cast<__bf16>(fast_tanh(acc[q] + b));
                             });
      bias(b3, at, E.A);
      __syncthreads();
      auto out3 = [&](int rt, int i, int c, floatx4 acc) {
        const int col = 16 * c + col_l;
        if (col >= E.A) return;
        const float b = bias_of(i, col);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float* dst = &L.abar[(rt * 16 + row_q + q) * DS + col];
          const float v = wk * fast_tanh(acc[q] + b);
          *dst = (k == 0) ? v : (*dst + v);
        }
      };
      const bf16x8* W3 = reinterpret_cast<const bf16x8*>(PA + E.off_w3);
      if (sl3 == 1) {
        layer_bf16<ROWT, TMAX>(L.x2, sth, E.H, W3, at, wave, lane, out3);
      } else {
        // Fewer output tiles than wavefronts: the k range is split over them, the partial tiles
        // meet in LDS over layer 1's outputs (read by now) and are summed in slice order.
        floatx4* part = reinterpret_cast<floatx4*>(L.x1);  // [sl3][at][ROWT][64]
        const int c3 = wave % at, q3 = wave / at;
        auto e3 = [&](int rt, int, int, floatx4 acc) { part[((q3 * at + c3) * ROWT + rt) * 64 + lane] = acc; };
        if (q3 < sl3)
          mlp_layer<kBF16, 1, ROWT, 1, decltype(e3), 4>(L.x2, sth, E.H, W3, at, c3, lane, e3, q3 * kk3 / sl3,
                                                        (q3 + 1) * kk3 / sl3);
        __syncthreads();
        if (wave < at) {
#pragma unroll
          for (int rt = 0; rt < ROWT; ++rt) {
            floatx4 acc = part[(wave * ROWT + rt) * 64 + lane];
            for (int q = 1; q < sl3; ++q) {
              const floatx4 p = part[((q * at + wave) * ROWT + rt) * 64 + lane];
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[r] = acc[r] + p[r];
            }
            out3(rt, 0, wave, acc);  // tile c = wave: slot 0 of the wavefront's biases
          }
        }
      }
      __syncthreads();
    }

    P.actions(t, row_base);
    __syncthreads();
    const double rwd = P.chain(owner, cash, asset, cumrew);
    if (owner && F.rew_traj) gbl(F.rew_traj)[static_cast<size_t>(it) * N + n] = rwd;
    __syncthreads();
    P.quantities(row_base);
    P.assemble(F.obs_traj ? F.obs_traj + row_base * C.S : nullptr, split_pad);
  }

  P.store_state(owner, st, cash, asset, cumrew);
}

template <int ROWT, int TMAX>
__global__ __launch_bounds__(256) void fused_generic_kernel(EnvConst C, EnvState st, EnsDev E,
                                                            FusedArgs F) {
  extern __shared__ __align__(16) unsigned char smem[];
  generic_tile<ROWT, TMAX>(C, st, E, F, blockIdx.x, smem);
}

// Batched persistent kernel (uneven groups): every workgroup takes work items -- (group, tile)
// pairs, ordered by decreasing cost -- from a counter until none is left, and runs each item's
// steps with the generic schedule.  The item counter is reset by zero_counter_kernel before each
// launch (a kernel, not a memset, so that the pair can be captured in a graph).
constexpr size_t kBatchedMaxLds = 160 * 1024 - 256;  // the kernel's own item slot takes a little

struct GroupDesc {
  EnvConst C;
  EnvState st;
  EnsDev E;
  FusedArgs F;
};

template <int ROWT, int TMAX>
__global__ __launch_bounds__(256) void fused_batched_kernel(const GroupDesc* __restrict__ groups,
                                                            const int2* __restrict__ items, int n_items,
                                                            int* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= n_items) break;
    const int2 gt = items[item];
    const GroupDesc G = groups[gt.x];
    if (G.F.n_steps > 0) generic_tile<ROWT, TMAX>(G.C, G.st, G.E, G.F, gt.y, smem);
  }
}

__global__ void zero_counter_kernel(int* counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

template <class Kern>
hipError_t go(Kern kern, int grid, int threads, size_t lds, hipStream_t stream, const EnvConst& C,
              const EnvState& st, const EnsDev& E, const FusedArgs& F) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, stream, C, st, E, F);
  return hipGetLastError();
}

hipError_t launch_generic(const EnvConst& C, const EnvState& st, const EnsDev& E, const FusedArgs& F,
                          hipStream_t stream, std::string* why) {
  const size_t lds = FusedLds::bytes(16, E.S_pad + 8, E.H + 8, C.D, C.I);
  if (lds > 160 * 1024) {
    *why = "fused rollout: state and hidden sizes exceed the LDS budget";
    return hipSuccess;
  }
  const int grid = (C.N + 15) / 16;
  const int tiles_per_wave = (E.H / 16 + 3) / 4;
  if (tiles_per_wave <= 2) return go(fused_generic_kernel<1, 2>, grid, 256, lds, stream, C, st, E, F);
  if (tiles_per_wave <= 4) return go(fused_generic_kernel<1, 4>, grid, 256, lds, stream, C, st, E, F);
  return go(fused_generic_kernel<1, 8>, grid, 256, lds, stream, C, st, E, F);
}

// Ring depth (k-steps of weight fragments in flight) by row tiles: the register budget of five
// wavefronts per workgroup is 256 per lane.
template <int ROWT>
constexpr int streamed_depth() { return ROWT == 1 ? 6 : 5; }

template <int ROWT, int KKE>
size_t streamed_lds_bytes(const EnvConst& C) {
  return StreamLds::offsets(16 * ROWT, 32 * KKE + 8, kStreamH + 8, C.D, C.I).total;
}

template <int ROWT, int KKE>
hipError_t launch_streamed_kernel(const EnvConst& C, const EnvState& st, const EnsDev& E, const FusedArgs& F,
                                  hipStream_t stream) {
  const size_t lds = streamed_lds_bytes<ROWT, KKE>(C);
  if (F.tile_envs < 1 || F.tile_envs > 16 * ROWT) return hipErrorInvalidValue;
  const int grid = (C.N + F.tile_envs - 1) / F.tile_envs;
  return go(fused_streamed_kernel<ROWT, KKE, streamed_depth<ROWT>()>, grid, kStreamThreads, lds, stream, C, st,
            E, F);
}

// The streamed schedule over a rollout: per chunk of at most kFusedChunk steps, the chunk's
// market table and noise, then the fused kernel for the chunk's steps.
hipError_t launch_streamed(const EnvConst& C, const EnvState& st, const EnsDev& E, FusedArgs F, int rowt,
                           float* eps_chunk, float* mt_chunk, hipStream_t stream) {
  const int t_end = F.t0 + F.n_steps;
  const size_t N = C.N, D = C.D, S = C.S;
  for (int t = F.t0; t < t_end; t += kFusedChunk) {
    const int n = t_end - t < kFusedChunk ? t_end - t : kFusedChunk;
    const size_t i0 = static_cast<size_t>(t - F.t0);
    hipError_t err = launch_chunk_inputs(C, E, t, n, F.sigma, F.key, F.env_offset, eps_chunk, mt_chunk, stream);
    if (err != hipSuccess) return err;
    FusedArgs Fc = F;
    Fc.t0 = t;
    Fc.n_steps = n;
    Fc.eps = eps_chunk;
    Fc.mt = mt_chunk;
    Fc.obs_traj = F.obs_traj ? F.obs_traj + i0 * N * S : nullptr;
    Fc.act_traj = F.act_traj ? F.act_traj + i0 * N * D : nullptr;
    Fc.rew_traj = F.rew_traj ? F.rew_traj + i0 * N : nullptr;
    Fc.qty_traj = F.qty_traj ? F.qty_traj + i0 * N * D : nullptr;
    const int kke = E.ke_pad / 32;
    if (rowt == 2)
      err = kke == 1 ? launch_streamed_kernel<2, 1>(C, st, E, Fc, stream) : launch_streamed_kernel<2, 2>(C, st, E, Fc, stream);
    else
      err = kke == 1 ? launch_streamed_kernel<1, 1>(C, st, E, Fc, stream) : launch_streamed_kernel<1, 2>(C, st, E, Fc, stream);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}


}  // namespace


hipError_t launch_chunk_inputs(const EnvConst& C, const EnsDev& E, int t, int n, float sigma, uint64_t key,
                               int64_t env_offset, float* eps_chunk, float* mt_chunk, hipStream_t stream) {
  const int Fm = (1 + C.I) * C.D;
  hipLaunchKernelGGL(market_table_kernel, dim3((n + kMtDays - 1) / kMtDays, E.K), dim3(kStreamH),
                     sizeof(float) * kMtDays * mt_row(Fm), stream, C, E, t, n, mt_chunk);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || sigma == 0.0f) return err;
  const size_t total = static_cast<size_t>(n) * C.N * ((C.D + 3) / 4);
  hipLaunchKernelGGL(noise_chunk_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, stream, key,
                     env_offset, t, n, C.N, C.D, eps_chunk);
  return hipGetLastError();
}

bool fused_streamed_shape(const EnvConst& C, const EnsDev& E) {
  using SP = Streamed<1, 1, streamed_depth<1>(), kMlpWaves>;
  if (!(E.K == kStreamK && E.H == kStreamH && E.S_pad == 224 && E.A_pad == 32 && C.D >= 1 && C.D <= 32 &&
        E.split_a == C.D && (E.ke_pad == 32 || E.ke_pad == 64) && (2 + C.I) * C.D <= 64 * kMktStage))
    return false;
  if (streamed_lds_bytes<2, 2>(C) > 160 * 1024) return false;
  return E.off_w1 == 0 && E.off_w2 == SP::kW2 && E.off_w3 == SP::kW3 && E.off_b1 == SP::kB1 &&
         E.off_b2 == SP::kB2 && E.off_b3 == SP::kB3 && E.actor_stride == SP::kActor;
}

size_t batched_lds_bytes(int rows, const EnvConst& C, const EnsDev& E) {
  return FusedLds::bytes(rows, (E.split_a > 0 ? E.ke_pad : E.S_pad) + 8, E.H + 8, C.D, C.I);
}

hipError_t launch_market_table(const EnvConst& C, const EnsDev& E, int t, int n, float* mt, hipStream_t stream) {
  const int Fm = (1 + C.I) * C.D;
  hipLaunchKernelGGL(market_table_kernel, dim3((n + kMtDays - 1) / kMtDays, E.K), dim3(kStreamH),
                     sizeof(float) * kMtDays * mt_row(Fm), stream, C, E, t, n, mt);
  return hipGetLastError();
}

size_t batched_max_lds() { return kBatchedMaxLds; }

size_t batched_group_desc_bytes() { return sizeof(GroupDesc); }

void batched_group_desc(const EnvConst& C, const EnvState& st, const EnsDev& E, int t0, int n_steps, float sigma,
                        uint64_t key, int64_t env_offset, float* obs_traj, float* act_traj, double* rew_traj,
                        int* qty_traj, const float* mt, void* out) {
  GroupDesc G{C, st, E, FusedArgs{t0, n_steps, sigma, key, env_offset, obs_traj, act_traj, rew_traj, qty_traj,
                                  nullptr, E.split_a > 0 ? mt : nullptr}};
  std::memcpy(out, &G, sizeof(GroupDesc));
}

hipError_t prepare_batched(size_t lds) {
  for (const void* k : {reinterpret_cast<const void*>(fused_batched_kernel<1, 4>),
                        reinterpret_cast<const void*>(fused_batched_kernel<2, 4>)}) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_batched(int rows, int blocks, size_t lds, const void* groups, const int* items, int n_items,
                          int* counter, hipStream_t stream) {
  if (lds > kBatchedMaxLds) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const GroupDesc* g = static_cast<const GroupDesc*>(groups);
  const int2* it = reinterpret_cast<const int2*>(items);
  if (rows == 32)
    hipLaunchKernelGGL((fused_batched_kernel<2, 4>), dim3(blocks), dim3(256), lds, stream, g, it, n_items, counter);
  else
    hipLaunchKernelGGL((fused_batched_kernel<1, 4>), dim3(blocks), dim3(256), lds, stream, g, it, n_items, counter);
  return hipGetLastError();
}

hipError_t launch_fused_rollout(const EnvConst& C, const EnvState& st, const EnsDev& E, int t0, int n_steps,
                                float sigma, uint64_t key, int64_t env_offset, float* obs_traj, float* act_traj,
                                double* rew_traj, int* qty_traj, float* eps_chunk, float* mt_chunk,
                                hipStream_t stream, std::string* why, FusedTuning tune) {
  why->clear();
  if (E.A != C.D || E.S != C.S) {
    *why = "fused rollout: ensemble shape does not match the environment";
    return hipSuccess;
  }
  FusedArgs F{t0, n_steps, sigma, key, env_offset, obs_traj, act_traj, rew_traj, qty_traj, nullptr, nullptr};
  int rowt = tune.row_tiles;
  if (rowt <= 0) rowt = C.N >= 4096 ? 2 : 1;
  rowt = rowt >= 2 ? 2 : 1;
  // Environments per workgroup: a full 16 * rowt rows, or fewer when that leaves compute units
  // idle (one workgroup fits a compute unit).
  F.tile_envs = 16 * rowt;
  if (tune.tile_envs > 0) {
    F.tile_envs = std::min(tune.tile_envs, 16 * rowt);
  } else {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      const int per_cu = (C.N + cus - 1) / cus;
      if (per_cu < F.tile_envs) F.tile_envs = std::max(per_cu, 1);
    }
  }
  int cus = 0;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
  }
  // The resident schedule runs one workgroup of up to eight environments per compute unit; past
  // one workgroup per compute unit the streamed schedule's wider tiles do better.
  const bool resident = fused_resident_shape(C, E) &&
                        (tune.schedule == 3 || (tune.schedule == 0 && cus > 0 && C.N <= kResRows * cus));
  if (resident) {
    // Up to eight environments per workgroup, fewer when that leaves compute units idle.
    F.tile_envs = kResRows;
    if (tune.tile_envs > 0)
      F.tile_envs = std::min(tune.tile_envs, kResRows);
    else if (cus > 0)
      F.tile_envs = std::max(1, std::min(kResRows, (C.N + cus - 1) / cus));
    return launch_resident(C, st, E, F, eps_chunk, mt_chunk, stream);
  }
  if (tune.schedule != 2 && fused_streamed_shape(C, E))
    return launch_streamed(C, st, E, F, rowt, eps_chunk, mt_chunk, stream);
  if (C.D > 128) {
    *why = "fused rollout: at most 128 stocks";
    return hipSuccess;
  }
  return launch_generic(C, st, E, F, stream, why);
}

}  // namespace fm
