// Fused rollout: one launch runs every step of a closed-loop rollout for a tile of 16*ROWT
// environments per workgroup.  Per step, inside the workgroup and without leaving the chip for
// anything but the weights and the trajectory stores:
//   1. Gaussian noise for the tile (Philox4x64-10 + Box-Muller) into LDS;
//   2. for each actor k: three bfloat16 MFMA layers over the tile's state rows (activations in
//      LDS, weights streamed from L2 in the packed B-operand layout), accumulating
//      a_bar = sum_k w_k mu_k in float32;
//   3. a = clip(a_bar + sigma * eps, -1, 1);
//   4. the trading chain (lane m of wavefront 0 owns environment m): orders, sells, buys, the new
//      day's value in float64, reward, cumulative reward;
//   5. the next state, written once as bfloat16 into LDS for the next step's first layer and, if
//      requested, as float32 into the [T][N][S] trajectory.
// Environments are independent, so workgroups never communicate.
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

template <int DMAX, int ROWT, int TMAX>
__global__ __launch_bounds__(256) void fused_rollout_kernel(EnvConst C, EnvState st, EnsDev E,
                                                            FusedArgs F) {
  constexpr int MR = 16 * ROWT;  // rows per workgroup
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int D = C.D, S = C.S, N = C.N, I = C.I;
  const int n0 = blockIdx.x * MR;
  const int M = min(MR, N - n0);
  const int st0 = E.S_pad + 8, sth = E.H + 8;
  const int DS = D + 1;
  const float inv_d = 1.0f / static_cast<float>(D);
  const int G = (D + 3) >> 2;
  const float inv_g = 1.0f / static_cast<float>(G);

  // LDS carve-up.
  __bf16* x0 = reinterpret_cast<__bf16*>(smem);
  __bf16* x1 = x0 + MR * st0;
  __bf16* x2 = x1 + MR * sth;
  float* s_abar = reinterpret_cast<float*>(x2 + MR * sth);
  float* s_eps = s_abar + MR * DS;
  float* s_act = s_eps + MR * DS;
  float* s_env = s_act + MR * DS;               // [MR][D+1]: cash entry, holdings entries
  int* s_qty = reinterpret_cast<int*>(s_env + MR * DS);
  float* s_px = reinterpret_cast<float*>(s_qty + MR * DS);
  float* s_pn = s_px + D;
  float* s_mkt = s_pn + D;                      // [(1+I)*D]: scaled close, indicators

  for (int i = tid; i < MR * st0; i += 256) x0[i] = static_cast<__bf16>(0.0f);

  // Trading state of environment n0+lane lives in wavefront 0's registers for the whole rollout.
  const bool owner = wave == 0 && lane < M;
  const int n = n0 + lane;
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  int h[DMAX], x[DMAX];
#pragma unroll
  for (int d = 0; d < DMAX; ++d) {
    h[d] = 0;
    x[d] = 0;
  }
  if (owner) {
    cash = st.cash[n];
    asset = st.asset[n];
    cumrew = st.cumrew[n];
#pragma unroll
    for (int d = 0; d < DMAX; ++d)
      if (d < D) h[d] = st.hold[static_cast<size_t>(d) * N + n];
  }

  // Market rows of day tn into s_pn / s_mkt (and of day tn-1 into s_px when trading).
  auto stage_market = [&](int tn, bool with_trade_day) {
    for (int d = tid; d < D; d += 256) {
      if (with_trade_day) s_px[d] = C.close[static_cast<size_t>(tn - 1) * D + d];
      const float pn = C.close[static_cast<size_t>(tn) * D + d];
      s_pn[d] = pn;
      s_mkt[d] = pn * C.price_scale;
    }
    for (int i = tid; i < I * D; i += 256) s_mkt[D + i] = C.ind[static_cast<size_t>(tn) * I * D + i];
  };
  auto write_env_entries = [&]() {
    if (owner) {
      s_env[lane * DS] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
#pragma unroll
      for (int d = 0; d < DMAX; ++d)
        if (d < D) s_env[lane * DS + 1 + d] = static_cast<float>(h[d]) * C.hold_scale;
    }
  };
  // State rows: bfloat16 into x0 for the next first layer, float32 into the trajectory.
  auto assemble = [&](float* traj) {
    for (int m = 0; m < M; ++m) {
      for (int f = tid; f < E.S_pad; f += 256) {
        float v = 0.0f;
        if (f < S) {
          if (f == 0) v = s_env[m * DS];
          else if (f <= D) v = s_mkt[f - 1];
          else if (f <= 2 * D) v = s_env[m * DS + f - D];
          else v = s_mkt[f - 1 - D];
          if (traj) traj[static_cast<size_t>(m) * S + f] = v;
        }
        x0[m * st0 + f] = static_cast<__bf16>(v);
      }
    }
  };

  stage_market(F.t0, false);
  write_env_entries();
  __syncthreads();
  assemble(nullptr);
  __syncthreads();

  const int row_q = 4 * (lane >> 4), col_l = lane & 15;
  const int ht = E.H / 16, at = E.A_pad / 16;

  for (int it = 0; it < F.n_steps; ++it) {
    const int t = F.t0 + it;
    const size_t row_base = static_cast<size_t>(it) * N + n0;
    stage_market(t + 1, true);
    if (F.sigma != 0.0f) {
      for (int i = tid; i < M * G; i += 256) {
        const int m = div_small(i, inv_g);
        const int g = i - m * G;
        float z[4];
        noise_block(F.key, static_cast<uint64_t>(F.env_offset + n0 + m), static_cast<uint64_t>(t),
                    static_cast<uint64_t>(g), z);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * g + r < D) s_eps[m * DS + 4 * g + r] = z[r];
      }
    }

    for (int k = 0; k < E.K; ++k) {
      const unsigned char* P = E.base + static_cast<size_t>(k) * E.actor_stride;
      const float* b1 = reinterpret_cast<const float*>(P + E.off_b1);
      const float* b2 = reinterpret_cast<const float*>(P + E.off_b2);
      const float* b3 = reinterpret_cast<const float*>(P + E.off_b3);
      const float wk = E.mix[k];
      layer_bf16<ROWT, TMAX>(x0, st0, E.S_pad, reinterpret_cast<const bf16x8*>(P + E.off_w1), ht, wave, lane,
                             [&](int rt, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               const float b = b1[col];
#pragma unroll
                               for (int r = 0; r < 4; ++r)
                                 x1[(rt * 16 + row_q + r) * sth + col] = static_cast<__bf16>(fast_tanh(acc[r] + b));
                             });
      __syncthreads();
      layer_bf16<ROWT, TMAX>(x1, sth, E.H, reinterpret_cast<const bf16x8*>(P + E.off_w2), ht, wave, lane,
                             [&](int rt, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               const float b = b2[col];
#pragma unroll
                               for (int r = 0; r < 4; ++r)
                                 x2[(rt * 16 + row_q + r) * sth + col] = static_cast<__bf16>(fast_tanh(acc[r] + b));
                             });
      __syncthreads();
      layer_bf16<ROWT, TMAX>(x2, sth, E.H, reinterpret_cast<const bf16x8*>(P + E.off_w3), at, wave, lane,
                             [&](int rt, int c, floatx4 acc) {
                               const int col = 16 * c + col_l;
                               if (col >= E.A) return;
                               const float b = b3[col];
#pragma unroll
                               for (int r = 0; r < 4; ++r) {
                                 float* dst = &s_abar[(rt * 16 + row_q + r) * DS + col];
                                 const float v = wk * fast_tanh(acc[r] + b);
                                 *dst = (k == 0) ? v : (*dst + v);
                               }
                             });
      __syncthreads();
    }

    // Noisy, clipped action.
    for (int i = tid; i < M * D; i += 256) {
      const int m = div_small(i, inv_d);
      const int d = i - m * D;
      float a = s_abar[m * DS + d];
      if (F.sigma != 0.0f) a = a + F.sigma * s_eps[m * DS + d];
      a = fminf(fmaxf(a, -1.0f), 1.0f);
      s_act[m * DS + d] = a;
      if (F.act_traj) F.act_traj[row_base * D + i] = a;
    }
    __syncthreads();

    if (owner) {
      trade<DMAX>(cash, h, x, &s_act[lane * DS], s_px, D, C.hmax_f, C.one_m, C.one_p);
      const double v_new = portfolio_value<DMAX>(cash, h, s_pn, D);
      const double r = (v_new - asset) * C.reward_scale;
      cumrew = cumrew + r;
      asset = v_new;
      if (F.rew_traj) F.rew_traj[static_cast<size_t>(it) * N + n] = r;
#pragma unroll
      for (int d = 0; d < DMAX; ++d)
        if (d < D) s_qty[lane * DS + d] = x[d];
    }
    write_env_entries();
    __syncthreads();

    if (F.qty_traj)
      for (int i = tid; i < M * D; i += 256) {
        const int m = div_small(i, inv_d);
        F.qty_traj[row_base * D + i] = s_qty[m * DS + (i - m * D)];
      }
    assemble(F.obs_traj ? F.obs_traj + row_base * S : nullptr);
    __syncthreads();
  }

  if (owner) {
    st.cash[n] = cash;
    st.asset[n] = asset;
    st.cumrew[n] = cumrew;
#pragma unroll
    for (int d = 0; d < DMAX; ++d)
      if (d < D) st.hold[static_cast<size_t>(d) * N + n] = h[d];
  }
}

size_t fused_lds_bytes(const EnvConst& C, const EnsDev& E, int rowt) {
  const int MR = 16 * rowt;
  const size_t DS = C.D + 1;
  size_t b = sizeof(__bf16) * MR * (static_cast<size_t>(E.S_pad + 8) + 2 * (E.H + 8));
  b += sizeof(float) * MR * DS * 5;  // abar, eps, act, env, qty
  b += sizeof(float) * (2 * C.D + (1 + C.I) * C.D);
  return b;
}

template <int DMAX, int ROWT>
hipError_t launch_rowt(const EnvConst& C, const EnvState& st, const EnsDev& E, const FusedArgs& F,
                       hipStream_t stream, std::string* why) {
  const size_t lds = fused_lds_bytes(C, E, ROWT);
  if (lds > 160 * 1024) {
    *why = "fused rollout: state and hidden sizes exceed the LDS budget";
    return hipSuccess;
  }
  const int grid = (C.N + 16 * ROWT - 1) / (16 * ROWT);
  const int tiles_per_wave = (E.H / 16 + 3) / 4;
  auto go = [&](auto kern) -> hipError_t {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, stream, C, st, E, F);
    return hipGetLastError();
  };
  if (tiles_per_wave <= 2) return go(fused_rollout_kernel<DMAX, ROWT, 2>);
  if (tiles_per_wave <= 4) return go(fused_rollout_kernel<DMAX, ROWT, 4>);
  return go(fused_rollout_kernel<DMAX, ROWT, 8>);
}

template <int DMAX>
hipError_t launch_dmax(const EnvConst& C, const EnvState& st, const EnsDev& E, const FusedArgs& F, int rowt,
                       hipStream_t stream, std::string* why) {
  if (rowt == 1) return launch_rowt<DMAX, 1>(C, st, E, F, stream, why);
  return launch_rowt<DMAX, 2>(C, st, E, F, stream, why);
}

}  // namespace

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
  if (rowt <= 0) rowt = C.N >= 8192 ? 2 : 1;
  if (C.D <= 8) return launch_dmax<8>(C, st, E, F, rowt, stream, why);
  if (C.D <= 16) return launch_dmax<16>(C, st, E, F, rowt, stream, why);
  if (C.D <= 32) return launch_dmax<32>(C, st, E, F, rowt, stream, why);
  if (C.D <= 64) return launch_dmax<64>(C, st, E, F, rowt, stream, why);
  if (C.D <= 128) return launch_dmax<128>(C, st, E, F, rowt, stream, why);
  *why = "fused rollout: at most 128 stocks";
  return hipSuccess;
}

}  // namespace fm
