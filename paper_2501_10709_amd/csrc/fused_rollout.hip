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
#include <utility>

#include "device_common.h"
#include "fused.h"
#include "mlp_device.h"

namespace fm {

namespace {

struct FusedArgs {
  int t0, n_steps;
  float sigma;
  uint64_t key;
  int64_t env_offset;
  float* obs_traj;
  float* act_traj;
  double* rew_traj;
  int* qty_traj;
};

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
      if (with_trade_day) L.px[d] = C.close[static_cast<size_t>(tn - 1) * D + d];
      const float pn = C.close[static_cast<size_t>(tn) * D + d];
      L.pn[d] = pn;
      L.mkt[d] = pn * C.price_scale;
    }
    for (int i = tid; i < C.I * D; i += NT) L.mkt[D + i] = C.ind[static_cast<size_t>(tn) * C.I * D + i];
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
          if (F.act_traj) F.act_traj[(row_base + m) * D + d] = a;
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
    chain_pairs_a(CL, Z, M, tid, NT, C.hmax_f, C.one_m, C.one_p);
    __syncthreads();
    if (owner)
      chain_serial(cash, CL.pro + lane * Z.RD, CL.deb + lane * Z.RD, CL.val + lane * Z.RD, CL.qd + lane * Z.RI,
                   CL.px, CL.kq + lane * Z.RI, Z.DP, C.one_p);
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

  // State rows: bfloat16 into x0 for the next first layer, float32 into the trajectory.
  __device__ void assemble(float* traj) {
    const int D = C.D, DS = D + 1, S = C.S;
    for (int m = 0; m < M; ++m) {
      for (int f = tid; f < S_pad; f += NT) {
        float v = 0.0f;
        if (f < S) {
          if (f == 0) v = L.env[m * DS];
          else if (f <= D) v = L.mkt[f - 1];
          else if (f <= 2 * D) v = L.env[m * DS + f - D];
          else v = L.mkt[f - 1 - D];
          if (traj) traj[static_cast<size_t>(m) * S + f] = v;
        }
        L.x0[m * st0 + f] = static_cast<__bf16>(v);
      }
    }
  }

  __device__ void quantities(size_t row_base) {
    if (!F.qty_traj) return;
    const int D = C.D;
    for (int i = tid; i < M * D; i += NT) F.qty_traj[row_base * D + i] = L.qty[i];
  }

  // Load the tile's state into the owner lanes (holdings into LDS).
  __device__ void load_state(bool owner, const EnvState& st, double& cash, double& asset, double& cumrew) {
    if (!owner) return;
    const int D = C.D, N = C.N, DS = D + 1, n = n0 + lane;
    cash = st.cash[n];
    asset = st.asset[n];
    cumrew = st.cumrew[n];
    for (int d = 0; d < D; ++d) L.hold[lane * D + d] = st.hold[static_cast<size_t>(d) * N + n];
  }
  __device__ void store_state(bool owner, const EnvState& st, double cash, double asset, double cumrew) {
    if (!owner) return;
    const int D = C.D, N = C.N, DS = D + 1, n = n0 + lane;
    st.cash[n] = cash;
    st.asset[n] = asset;
    st.cumrew[n] = cumrew;
    for (int d = 0; d < D; ++d) st.hold[static_cast<size_t>(d) * N + n] = L.hold[lane * D + d];
  }
};

// ------------------------------------------------------------------------------------------
// Generic MLP schedule (runtime shapes): wavefront w owns output tiles w, w+4, ...
// ------------------------------------------------------------------------------------------
template <int ROWT, int TMAX, class Epi>
__device__ __forceinline__ void layer_bf16(const __bf16* sin, int ist, int kin_pad, const bf16x8* W,
                                           int ntiles, int wave, int lane, Epi epi) {
  floatx4 acc[ROWT][TMAX];
#pragma unroll
  for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
    for (int i = 0; i < TMAX; ++i) acc[rt][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const int row = lane & 15, grp = lane >> 4;
  const int KK = kin_pad / 32;
  for (int kk = 0; kk < KK; ++kk) {
    bf16x8 a[ROWT];
#pragma unroll
    for (int rt = 0; rt < ROWT; ++rt)
      a[rt] = *reinterpret_cast<const bf16x8*>(sin + (rt * 16 + row) * ist + 32 * kk + 8 * grp);
#pragma unroll
    for (int i = 0; i < TMAX; ++i) {
      const int c = wave + 4 * i;
      if (c < ntiles) {
        const bf16x8 b = W[(static_cast<size_t>(c) * KK + kk) * 64 + lane];
#pragma unroll
        for (int rt = 0; rt < ROWT; ++rt) acc[rt][i] = mfma_bf16(a[rt], b, acc[rt][i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TMAX; ++i) {
    const int c = wave + 4 * i;
    if (c < ntiles) {
#pragma unroll
      for (int rt = 0; rt < ROWT; ++rt) epi(rt, c, acc[rt][i]);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Streamed MLP schedule for K = 3, S_pad = 32*KK1, H = 256, A_pad = 32 with eight wavefronts.
// Wavefront w owns layer-1/2 output tiles w and w+8 and, if w < 2, layer-3 tile w.  Its weight
// fragments form a fixed sequence of NS k-steps per environment step; fragments for k-step
// s+DEPTH are requested when k-step s is consumed.
// ------------------------------------------------------------------------------------------
template <int KK1, int ROWT, int DEPTH, int NWAVES>
struct Streamed {
  static constexpr int K = 3, KK2 = 8, HT = 16, AT = 2, NW = NWAVES, TW = HT / NWAVES;
  static constexpr int SPA = KK1 + 2 * KK2;  // k-steps per actor
  static constexpr int NS = K * SPA;         // k-steps per environment step
  // The schedule walks NSP >= NS positions per step, a multiple of DEPTH, so that k-step j always
  // uses ring slot j % DEPTH, also across the wrap into the next step; positions >= NS are idle.
  static constexpr int NSP = (NS + DEPTH - 1) / DEPTH * DEPTH;

  // Packed-ensemble layout of this shape (bytes; checked against the workspace on the host).
  static constexpr size_t kW1 = 0, kW2 = 32 * KK1 * 256 * 2, kW3 = kW2 + 256 * 256 * 2;
  static constexpr size_t kB1 = kW3 + 256 * 32 * 2, kB2 = kB1 + 1024, kB3 = kB2 + 1024;
  static constexpr size_t kActor = kB3 + 256;

  // Weight fragments of k-step S2 for wavefront wv (uniform); voff = lane * 16.
  template <int S2>
  static __device__ __forceinline__ void load(bf16x8 (&b)[TW], const unsigned char* wb, int wv, int voff) {
    if constexpr (S2 >= NS) return;  // idle position
    constexpr int actor = S2 / SPA, r = S2 % SPA;
    const unsigned char* P = wb + kActor * actor;
    if constexpr (r < KK1) {
#pragma unroll
      for (int i = 0; i < TW; ++i)
        b[i] = *reinterpret_cast<const bf16x8*>(P + kW1 + static_cast<size_t>((wv + NW * i) * KK1 + r) * 1024 + voff);
    } else if constexpr (r < KK1 + KK2) {
      constexpr int kk = r - KK1;
#pragma unroll
      for (int i = 0; i < TW; ++i)
        b[i] = *reinterpret_cast<const bf16x8*>(P + kW2 + static_cast<size_t>((wv + NW * i) * KK2 + kk) * 1024 + voff);
    } else {
      constexpr int kk = r - KK1 - KK2;
      if (wv < AT) b[0] = *reinterpret_cast<const bf16x8*>(P + kW3 + static_cast<size_t>(wv * KK2 + kk) * 1024 + voff);
    }
  }
};

template <int ROWT, int KK1, int DEPTH, int NWAVES>
__global__ __launch_bounds__(64 * NWAVES) void fused_streamed_kernel(EnvConst C, EnvState st, EnsDev E,
                                                                     FusedArgs F) {
  using SP = Streamed<KK1, ROWT, DEPTH, NWAVES>;
  constexpr int NT = 64 * NWAVES, MR = 16 * ROWT, TW = SP::TW, NW = SP::NW;
  constexpr int KK2 = SP::KK2, SPA = SP::SPA, NS = SP::NS, NSP = SP::NSP;
  constexpr int S_PAD = 32 * KK1, H = 256;
  constexpr int ST0 = S_PAD + 8, STH = H + 8;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int D = C.D, N = C.N, DS = D + 1;
  const int n0 = blockIdx.x * MR;
  const int M = min(MR, N - n0);

  FusedLds L;
  L.carve(smem, MR, ST0, STH, D);
  EnvPhase<NT> P{C, F, L, tid, lane, wave, n0, M, S_PAD, ST0, 1.0f / static_cast<float>(D),
                 1.0f / static_cast<float>((D + 3) >> 2), (D + 3) >> 2};

  for (int i = tid; i < MR * ST0; i += NT) L.x0[i] = static_cast<__bf16>(0.0f);

  const bool owner = wave == 0 && lane < M;
  const int n = n0 + lane;
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  P.load_state(owner, st, cash, asset, cumrew);

  P.stage_market(F.t0, false);
  P.env_entries(owner, cash);
  __syncthreads();
  P.assemble(nullptr);

  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int voff = lane * 16;
  bf16x8 ring[DEPTH][TW];
  static_for<DEPTH>([&](auto sc) __attribute__((always_inline)) {
    constexpr int s = decltype(sc)::value;
    SP::template load<s>(ring[s], E.base, wv, voff);
  });

  const int row_q = 4 * (lane >> 4), col_l = lane & 15, row = lane & 15, grp = lane >> 4;
  const float* mix = E.mix;

  for (int it = 0; it < F.n_steps; ++it) {
    const int t = F.t0 + it;
    const size_t row_base = static_cast<size_t>(it) * N + n0;
    __syncthreads();                       // x0 complete; LDS market rows free
    P.stage_market(t + 1, true);
    // The weight base is offset by an opaque zero every step, so that no fragment address is
    // hoisted out of the step loop (there are hundreds of them).  Laundering an integer rather
    // than the pointer keeps the loads in the global address space (flat loads would also count
    // against the LDS wait counter and stall every LDS read behind the whole weight pipeline).
    int opaque_zero = 0;
    asm volatile("" : "+s"(opaque_zero));
    const unsigned char* wb = E.base + opaque_zero;

    floatx4 acc[ROWT][TW];
    static_for<NSP>([&](auto sc) __attribute__((always_inline)) {
      constexpr int s = decltype(sc)::value;
      // Keep the k-steps in program order: the scheduler would otherwise hoist every load of a
      // layer to its top and run out of registers.
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (s >= NS) {
        SP::template load<(s + DEPTH) % NSP>(ring[s % DEPTH], wb, wv, voff);
        return;
      }
      constexpr int actor = s / SPA, r = s % SPA;
      constexpr int layer = r < KK1 ? 1 : (r < KK1 + KK2 ? 2 : 3);
      constexpr int kk = layer == 1 ? r : (layer == 2 ? r - KK1 : r - KK1 - KK2);
      constexpr int first = layer == 1 ? 0 : (layer == 2 ? KK1 : KK1 + KK2);
      constexpr int last = layer == 1 ? KK1 - 1 : (layer == 2 ? KK1 + KK2 - 1 : SPA - 1);
      if constexpr (r == first) {
#pragma unroll
        for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
          for (int i = 0; i < TW; ++i) acc[rt][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
      }
      bf16x8 cur[TW];
#pragma unroll
      for (int i = 0; i < TW; ++i) cur[i] = ring[s % DEPTH][i];
      SP::template load<(s + DEPTH) % NSP>(ring[s % DEPTH], wb, wv, voff);

      const __bf16* src = layer == 1 ? L.x0 : (layer == 2 ? L.x1 : L.x2);
      constexpr int ist = layer == 1 ? ST0 : STH;
      bf16x8 a[ROWT];
#pragma unroll
      for (int rt = 0; rt < ROWT; ++rt)
        a[rt] = *reinterpret_cast<const bf16x8*>(src + (rt * 16 + row) * ist + 32 * kk + 8 * grp);
      if constexpr (layer < 3) {
#pragma unroll
        for (int i = 0; i < TW; ++i)
#pragma unroll
          for (int rt = 0; rt < ROWT; ++rt) acc[rt][i] = mfma_bf16(a[rt], cur[i], acc[rt][i]);
      } else {
        if (wave < SP::AT) {
#pragma unroll
          for (int rt = 0; rt < ROWT; ++rt) acc[rt][0] = mfma_bf16(a[rt], cur[0], acc[rt][0]);
        }
      }

      if constexpr (r == last) {
        const unsigned char* PA = wb + SP::kActor * actor;
        if constexpr (layer < 3) {
          const float* bias = reinterpret_cast<const float*>(PA + (layer == 1 ? SP::kB1 : SP::kB2));
          __bf16* out = layer == 1 ? L.x1 : L.x2;
#pragma unroll
          for (int i = 0; i < TW; ++i) {
            const int col = 16 * (wave + NW * i) + col_l;
            const float b = bias[col];
#pragma unroll
            for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                out[(rt * 16 + row_q + q) * STH + col] = static_cast<__bf16>(fast_tanh(acc[rt][i][q] + b));
          }
        } else {
          if (wave < SP::AT) {
            const float* b3 = reinterpret_cast<const float*>(PA + SP::kB3);
            const int col = 16 * wave + col_l;
            if (col < E.A) {
              const float b = b3[col];
              const float wk = mix[actor];
#pragma unroll
              for (int rt = 0; rt < ROWT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  float* dst = &L.abar[(rt * 16 + row_q + q) * DS + col];
                  const float v = wk * fast_tanh(acc[rt][0][q] + b);
                  *dst = (actor == 0) ? v : (*dst + v);
                }
            }
          }
        }
        __syncthreads();
      }
    });

    P.actions(t, row_base);
    __syncthreads();
    const double rwd = P.chain(owner, cash, asset, cumrew);
    if (owner && F.rew_traj) F.rew_traj[static_cast<size_t>(it) * N + n] = rwd;
    __syncthreads();
    P.quantities(row_base);
    P.assemble(F.obs_traj ? F.obs_traj + row_base * C.S : nullptr);
  }

  P.store_state(owner, st, cash, asset, cumrew);
}

template <int ROWT, int TMAX>
__global__ __launch_bounds__(256) void fused_generic_kernel(EnvConst C, EnvState st, EnsDev E,
                                                            FusedArgs F) {
  constexpr int NT = 256, MR = 16 * ROWT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int D = C.D, N = C.N, DS = D + 1;
  const int n0 = blockIdx.x * MR;
  const int M = min(MR, N - n0);
  const int st0 = E.S_pad + 8, sth = E.H + 8;

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
  P.assemble(nullptr);

  const int row_q = 4 * (lane >> 4), col_l = lane & 15;
  const int ht = E.H / 16, at = E.A_pad / 16;

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
      const float wk = E.mix[k];
      layer_bf16<ROWT, TMAX>(L.x0, st0, E.S_pad, reinterpret_cast<const bf16x8*>(PA + E.off_w1), ht, wave, lane,
                             [&](int rt, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               const float b = b1[col];
#pragma unroll
                               for (int q = 0; q < 4; ++q)
                                 L.x1[(rt * 16 + row_q + q) * sth + col] = static_cast<__bf16>(fast_tanh(acc[q] + b));
                             });
      __syncthreads();
      layer_bf16<ROWT, TMAX>(L.x1, sth, E.H, reinterpret_cast<const bf16x8*>(PA + E.off_w2), ht, wave, lane,
                             [&](int rt, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               const float b = b2[col];
#pragma unroll
                               for (int q = 0; q < 4; ++q)
                                 L.x2[(rt * 16 + row_q + q) * sth + col] = static_cast<__bf16>(fast_tanh(acc[q] + b));
                             });
      __syncthreads();
      layer_bf16<ROWT, TMAX>(L.x2, sth, E.H, reinterpret_cast<const bf16x8*>(PA + E.off_w3), at, wave, lane,
                             [&](int rt, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               if (col >= E.A) return;
                               const float b = b3[col];
#pragma unroll
                               for (int q = 0; q < 4; ++q) {
                                 float* dst = &L.abar[(rt * 16 + row_q + q) * DS + col];
                                 const float v = wk * fast_tanh(acc[q] + b);
                                 *dst = (k == 0) ? v : (*dst + v);
                               }
                             });
      __syncthreads();
    }

    P.actions(t, row_base);
    __syncthreads();
    const double rwd = P.chain(owner, cash, asset, cumrew);
    if (owner && F.rew_traj) F.rew_traj[static_cast<size_t>(it) * N + n] = rwd;
    __syncthreads();
    P.quantities(row_base);
    P.assemble(F.obs_traj ? F.obs_traj + row_base * C.S : nullptr);
  }

  P.store_state(owner, st, cash, asset, cumrew);
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

constexpr int kDepth = 6;
constexpr int kWaves = 4;

template <int ROWT>
hipError_t launch_streamed(const EnvConst& C, const EnvState& st, const EnsDev& E, const FusedArgs& F,
                           hipStream_t stream) {
  const size_t lds = FusedLds::bytes(16 * ROWT, 224 + 8, 256 + 8, C.D, C.I);
  const int grid = (C.N + 16 * ROWT - 1) / (16 * ROWT);
  return go(fused_streamed_kernel<ROWT, 7, kDepth, kWaves>, grid, 64 * kWaves, lds, stream, C, st, E, F);
}

}  // namespace

bool fused_streamed_shape(const EnvConst& C, const EnsDev& E) {
  using SP = Streamed<7, 1, kDepth, kWaves>;
  return E.K == 3 && E.H == 256 && E.S_pad == 224 && E.A_pad == 32 && C.D >= 1 && C.D <= 32 &&
         E.off_w1 == SP::kW1 && E.off_w2 == SP::kW2 && E.off_w3 == SP::kW3 && E.off_b1 == SP::kB1 &&
         E.off_b2 == SP::kB2 && E.off_b3 == SP::kB3 && E.actor_stride == SP::kActor;
}

hipError_t launch_fused_rollout(const EnvConst& C, const EnvState& st, const EnsDev& E, int t0, int n_steps,
                                float sigma, uint64_t key, int64_t env_offset, float* obs_traj, float* act_traj,
                                double* rew_traj, int* qty_traj, hipStream_t stream, std::string* why,
                                FusedTuning tune) {
  why->clear();
  if (E.A != C.D || E.S != C.S) {
    *why = "fused rollout: ensemble shape does not match the environment";
    return hipSuccess;
  }
  FusedArgs F{t0, n_steps, sigma, key, env_offset, obs_traj, act_traj, rew_traj, qty_traj};
  int rowt = tune.row_tiles;
  if (rowt <= 0) rowt = C.N >= 4096 ? 2 : 1;
  rowt = rowt >= 2 ? 2 : 1;
  if (tune.schedule != 2 && fused_streamed_shape(C, E))
    return rowt == 2 ? launch_streamed<2>(C, st, E, F, stream) : launch_streamed<1>(C, st, E, F, stream);
  if (C.D > 128) {
    *why = "fused rollout: at most 128 stocks";
    return hipSuccess;
  }
  return launch_generic(C, st, E, F, stream, why);
}

}  // namespace fm
