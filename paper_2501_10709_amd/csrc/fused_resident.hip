// The resident schedule of the fused rollout: the K = 3, H = 256 ensemble over a trading state
// of D <= 31 stocks, with every weight on chip for the whole launch.
//
// A workgroup owns up to eight environments (one compute unit; N = 2048 fills 256 of them) and
// runs four wavefronts:
//   * W2 of all three actors (384 KB in bfloat16) lives in registers: wavefront w holds the
//     fragments of output tiles 4w .. 4w+3 of every actor, two actors' worth in the accumulation
//     registers (read in place by the MFMAs) and one in the vector registers;
//   * W1e (the first layer's rows for the cash and holdings entries) and W3 live in LDS; the
//     first layer's market rows are folded into the day's table (bias included), made per chunk
//     by market_table_kernel, because the closes and indicators are the same for every
//     environment on a day (Section 3.1 state, shared market data of Section 4.2).
// The layers run transposed (units x environments, weights as the A operand); the 8 environments
// fill half of each accumulator's columns, and two accumulators are merged by a DPP row shift
// before an epilogue, so each tanh is evaluated once per value.
//
// Per step, four workgroup barriers close the phases:
//   L1    all wavefronts.  A: W1e, B: the state rows' cash and holdings entries; the
//         accumulators start from the day's table row;
//   L2    all wavefronts, A from registers;
//   L3    wavefront a < 3 computes actor a's two output tiles and leaves w_a tanh(z + b3_a);
//   trade every wavefront trades two environments, one per 16-lane row (rows 2 and 3 repeat
//         rows 0 and 1), lane j of a row owning stocks j and j + 16: the action (actor sum,
//         noise, clip), the order and the sale, then the cash recurrence of Section 3.1 --
//         sells, then buys, in ascending stock order -- which every lane of the row computes on
//         terms broadcast from the owning lane (DPP row broadcasts, no LDS round trip), keeping
//         the fills of its own stocks; holdings, position values, the new value and reward, the
//         next state row, and the trajectory stores of actions, quantities and rewards straight
//         from registers.
// The step's noise (drawn per chunk by noise_chunk_kernel) is requested at the top of a step and
// used after the MLP.  The inputs travel by buffer loads that write LDS directly: the next step's
// table row, a third by each of wavefronts 0-2 at the top of a step (waited for after the third
// barrier; double-buffered), and the market rows two steps ahead by wavefront 3, which has no
// actor in L3, in that phase (waited for in the next step's L3; triple-buffered).  The state rows
// of a step are assembled as a float32 image in LDS -- the market entries by every wavefront in
// L3, the cash and holdings by the trading lanes -- and stored whole by wavefront 3 in the next
// step's L3.
#include <cstring>
#include <utility>

#include "device_common.h"
#include "fused.h"
#include "mlp_device.h"
#include "row_chain.h"



namespace fm {

namespace {

constexpr int kRT = 256;     // threads per workgroup
constexpr int kRK = 3, kRH = 256, kRKK = 8;
constexpr int kRX0 = 40;     // state-row stride (bfloat16): cash, <= 31 holdings, zeros
constexpr int kRXS = 264;    // hidden-row stride (bfloat16)
constexpr int kRIn = 256;    // market entries per day, (2 + I) * D <= 256
// An input buffer in LDS: close[t] | close[t+1] in floats 0 .. 2D-1, ind[t+1] from float kRInd
// (the fetch writes whole runs of 64 floats, so the two parts do not overlap).
constexpr int kRInd = 64;
constexpr int kRInBuf = kRInd + 256;
// A float32 image of a step's state rows ([8][S], S = 1 + (2 + I) D <= 1 + kRIn), padded to whole
// 16-byte units.
constexpr int kRImg = kResRows * (kRIn + 4);

constexpr size_t r16(size_t b) { return (b + 15) / 16 * 16; }

// LDS regions (byte offsets) of the resident kernel.
struct RLds {
  static constexpr size_t w1e = 0;                                                 // [K][16][64] bf16x8
  static constexpr size_t w3 = w1e + sizeof(bf16x8) * kRK * 16 * 64;               // [K][2][8][64] bf16x8
  static constexpr size_t xb = r16(sizeof(__bf16) * kRK * kResRows * kRXS);
  static constexpr size_t x1 = w3 + sizeof(bf16x8) * kRK * 2 * kRKK * 64;          // [K][8][264] bf16
  static constexpr size_t mu = x1;                                                 // [K][8][32] f32 (after L2)
  static constexpr size_t x2 = x1 + xb;                                            // [K][8][264] bf16
  static constexpr size_t x0 = x2 + xb;                                            // [8][40] bf16
  static constexpr size_t b2 = x0 + r16(sizeof(__bf16) * kResRows * kRX0);         // [K][256] f32
  static constexpr size_t b3 = b2 + sizeof(float) * kRK * kRH;                     // [K][32] f32
  static constexpr size_t mix = b3 + sizeof(float) * kRK * 32;                     // [4] f32
  static constexpr size_t mt = mix + 16;                                           // [2][K][256] f32
  static constexpr size_t in = mt + sizeof(float) * 2 * kRK * kRH;                 // [3][320] f32
  static constexpr size_t state = in + sizeof(float) * 3 * kRInBuf;                // [8] {cash, value, cumrew, 0} f64
  static constexpr size_t img = state + sizeof(double) * 4 * kResRows;              // [2][8][S] f32
  static constexpr size_t total = img + sizeof(float) * 2 * kRImg;
  static_assert(sizeof(float) * kRK * kResRows * 32 <= xb, "the actor means fit the layer-1 region");
};
static_assert(RLds::total <= 160 * 1024, "LDS budget");
static_assert(kRK * kRH % (64 * 3) == 0, "wavefronts 0-2 fetch equal shares of a table row");

// An opaque zero: values derived from it are recomputed where they are used instead of being
// hoisted out of the step loop and held in registers.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// The layers run transposed: out[unit][env] = W^T x, the packed weight fragment as the A
// operand and the activation rows as the B operand, so lane l of an accumulator holds units
// 4(l/16) .. 4(l/16)+3 of its 16-unit tile for environment l mod 16.  The activation rows of the
// 8 environments fill B columns 0-7 and repeat in 8-15, so lanes with l mod 16 >= 8 duplicate
// those below.  Two tiles are merged into one register set by a DPP row shift: lane l then holds
// tile q1 for environment l mod 8 when l mod 16 >= 8, else tile q0.  The accumulator starts from
// the bias, so the epilogue is the activation alone.
__device__ __forceinline__ floatx4 merge_tiles(const floatx4& q0, const floatx4& q1) {
  floatx4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = __builtin_amdgcn_update_dpp(q0[i], q1[i], 0x118, 0xf, 0xf, false);  // row_shr:8
  return r;
}

// tanh(x) = 2 / (1 + e^{-2x}) - 1 from one exponential and one reciprocal; absolute error about
// 2e-7 (the tanh of the library agrees to within 1e-6).
__device__ __forceinline__ float tanh_sig(float x) {
  const float t = __builtin_amdgcn_exp2f(-2.8853900817779268f * x);  // e^{-2x}
  return fmaf(2.0f, __builtin_amdgcn_rcpf(1.0f + t), -1.0f);
}

// Four activations as bfloat16 (round to nearest even), 8 bytes.
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d) {
  typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
  const bf16x2 lo = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
  const bf16x2 hi = {static_cast<__bf16>(c), static_cast<__bf16>(d)};
  return uint2{__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
}

// Trajectory stores go through buffer resources that cover the tile's rows of one step: a lane
// with nothing to store passes an offset beyond the range, which the hardware drops, so the
// stores need no branches; a trajectory that is not requested gets an empty range.
constexpr int kNoStore = 1 << 30;  // beyond every range; adding a row offset stays below 2^31
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const void* base, size_t elem_offset, size_t elem_bytes,
                                                            int n_elems) {
  if (!base) return __builtin_amdgcn_make_buffer_rsrc(nullptr, 0, 0, 0x00020000);
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(static_cast<const char*>(base)) + elem_offset * elem_bytes, 0,
      static_cast<int>(elem_bytes * n_elems), 0x00020000);
}
__device__ __forceinline__ void store_f32(__amdgpu_buffer_rsrc_t r, int byte_off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, 0, 0);
}
// A load through such a resource returns 0 beyond its range.
__device__ __forceinline__ float load_f32(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// The three layers of one step for the wavefront's tiles.  Lane l's B operand is activation
// row l mod 8 (the environment), entries 8(l/16) .. +7 of each 32-entry k-step; after a merge,
// lane l holds tile (l / 8) mod 2 of a pair, environment l mod 8, units 4(l/16) .. +3.  The LDS
// regions are passed as distinct (restrict) pointers, so the compiler may move the loads of
// later tiles above the stores of earlier ones.
__device__ __forceinline__ void layer1(const bf16x8* __restrict__ w1e, const float* __restrict__ mt,
                                       const __bf16* __restrict__ x0, __bf16* __restrict__ x1, int wave, int lane) {
  constexpr int K = kRK, H = kRH, MR = kResRows;
  const int bev = lane & 7, bgrp = lane >> 4, pair_t = (lane >> 3) & 1;
  const bf16x8 X = *reinterpret_cast<const bf16x8*>(x0 + bev * kRX0 + 8 * bgrp);
  // Six (actor, tile pair) stages: stage i requests the operands of pair i + 2 (the weight
  // fragments and the day's table entries, which the accumulators start from), issues the MFMAs
  // of pair i + 1 and then the epilogue of pair i, fenced so that the activations run while the
  // matrix cores work and no LDS latency sits between a load and its use.
  constexpr int NP = 2 * K;
  floatx4 T[NP][2], acc[NP][2];
  bf16x8 Wf[NP][2];
  auto ld = [&](int i) {
    const int a = i >> 1, p = i & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = 4 * wave + 2 * p + h;
      T[i][h] = *reinterpret_cast<const floatx4*>(mt + a * H + 16 * c + 4 * bgrp);
      Wf[i][h] = w1e[(a * 16 + c) * 64 + lane];
    }
  };
  auto mm = [&](int i) {
#pragma unroll
    for (int h = 0; h < 2; ++h) acc[i][h] = mfma_bf16(Wf[i][h], X, T[i][h]);
  };
  auto epi = [&](int i) {
    const int a = i >> 1, p = i & 1;
    const floatx4 v = merge_tiles(acc[i][0], acc[i][1]);
    const int u0 = 16 * (4 * wave + 2 * p + pair_t) + 4 * bgrp;
    *reinterpret_cast<uint2*>(x1 + a * MR * kRXS + bev * kRXS + u0) =
        pack_bf16x4(tanh_sig(v[0]), tanh_sig(v[1]), tanh_sig(v[2]), tanh_sig(v[3]));
  };
  ld(0);
  ld(1);
  mm(0);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    if (i + 2 < NP) ld(i + 2);
    if (i + 1 < NP) mm(i + 1);
    epi(i);
    __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ void layer2(const bf16x8 (&w2)[kRK][kRKK][4], const float* __restrict__ b2,
                                       const __bf16* __restrict__ x1, __bf16* __restrict__ x2, int wave, int lane) {
  constexpr int K = kRK, H = kRH, KK = kRKK, MR = kResRows;
  const int bev = lane & 7, bgrp = lane >> 4, pair_t = (lane >> 3) & 1;
  // Software-pipelined over (actor, tile pair): the MFMAs of one pair are issued between the
  // slices of the previous pair's epilogue (its activations), so the vector work runs while the
  // matrix cores are busy.  Each accumulator still sums its k-steps in the same order.
  // Actor a's activations: X[a & 1], requested one stage before the first use.
  bf16x8 X[2][KK];
  floatx4 acc[4];
  auto load_x = [&](int a) {
    const __bf16* src = x1 + a * MR * kRXS + bev * kRXS + 8 * bgrp;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) X[a & 1][kk] = *reinterpret_cast<const bf16x8*>(src + 32 * kk);
  };
  auto epilogue = [&](int a, int p) {
    const floatx4 v = merge_tiles(acc[2 * p], acc[2 * p + 1]);
    const int u0 = 16 * (4 * wave + 2 * p + pair_t) + 4 * bgrp;
    *reinterpret_cast<uint2*>(x2 + a * MR * kRXS + bev * kRXS + u0) =
        pack_bf16x4(tanh_sig(v[0]), tanh_sig(v[1]), tanh_sig(v[2]), tanh_sig(v[3]));
  };
  // Stage (a, p): the MFMAs of pair (a, p), k-step by k-step, each k-step followed by a slice of
  // the previous pair (pa, pp)'s epilogue (merge, one activation, the pack, the store) and a
  // scheduling fence: left to itself the scheduler issues the MFMAs of several pairs back to back
  // and the epilogues after them, with nothing overlapped.
  auto stage = [&](int a, int p, int pa, int pp, bool epi, int pre) {
    floatx4 v;
    float t[4];
    uint2 packed;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
#pragma unroll
      for (int i = 2 * p; i < 2 * p + 2; ++i)
        acc[i] = kk == 0 ? mfma_bf16(w2[a][0][i], X[a & 1][0], *reinterpret_cast<const floatx4*>(b2 + a * H + 16 * (4 * wave + i) + 4 * bgrp))
                         : mfma_bf16(w2[a][kk][i], X[a & 1][kk], acc[i]);
      // The next actor's activations, requested after this stage's bias loads so that waiting
      // for those does not wait for these.
      if (kk == 0 && pre >= 0) load_x(pre);
      if (epi) {
        if (kk == 0) v = merge_tiles(acc[2 * pp], acc[2 * pp + 1]);
        if (kk >= 1 && kk <= 4) t[kk - 1] = tanh_sig(v[kk - 1]);
        if (kk == 5) packed = pack_bf16x4(t[0], t[1], t[2], t[3]);
        if (kk == 6) {
          const int u0 = 16 * (4 * wave + 2 * pp + pair_t) + 4 * bgrp;
          *reinterpret_cast<uint2*>(x2 + pa * MR * kRXS + bev * kRXS + u0) = packed;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  load_x(0);
  stage(0, 0, 0, 0, false, -1);
#pragma unroll
  for (int a = 0; a < K; ++a) {
    stage(a, 1, a, 0, true, a + 1 < K ? a + 1 : -1);
    if (a + 1 < K) stage(a + 1, 0, a, 1, true, -1);
  }
  epilogue(K - 1, 1);
}

// Actor a = wave's two output tiles, w_a tanh(z + b3_a) into mu[a][env][dim].
__device__ __forceinline__ void layer3(const bf16x8* __restrict__ w3, const float* __restrict__ b3,
                                       const float* __restrict__ mix, const __bf16* __restrict__ x2,
                                       float* __restrict__ mu, int wave, int lane) {
  constexpr int KK = kRKK, MR = kResRows;
  const int bev = lane & 7, bgrp = lane >> 4, pair_t = (lane >> 3) & 1;
  const int a = wave;
  const __bf16* src = x2 + a * MR * kRXS + bev * kRXS + 8 * bgrp;
  // The operands of k-step kk + kRL3 are requested before the products of k-step kk, so the LDS
  // latency is paid once rather than per k-step.
  constexpr int kRL3 = 4;
  floatx4 acc[2];
  bf16x8 X[KK], W[2][KK];
  auto load = [&](int kk) {
    X[kk] = *reinterpret_cast<const bf16x8*>(src + 32 * kk);
#pragma unroll
    for (int h = 0; h < 2; ++h) W[h][kk] = w3[((a * 2 + h) * KK + kk) * 64 + lane];
  };
#pragma unroll
  for (int h = 0; h < 2; ++h) acc[h] = *reinterpret_cast<const floatx4*>(b3 + a * 32 + 16 * h + 4 * bgrp);
#pragma unroll
  for (int kk = 0; kk < kRL3; ++kk) load(kk);
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) {
    if (kk + kRL3 < KK) load(kk + kRL3);
#pragma unroll
    for (int h = 0; h < 2; ++h) acc[h] = mfma_bf16(W[h][kk], X[kk], acc[h]);
    __builtin_amdgcn_sched_barrier(0);
  }
  const floatx4 v = merge_tiles(acc[0], acc[1]);
  const float wk = mix[a];
  *reinterpret_cast<float4*>(mu + a * MR * 32 + bev * 32 + 16 * pair_t + 4 * bgrp) =
      float4{wk * tanh_sig(v[0]), wk * tanh_sig(v[1]), wk * tanh_sig(v[2]), wk * tanh_sig(v[3])};
}

__global__ __launch_bounds__(kRT) __attribute__((amdgpu_waves_per_eu(1, 1)))
void fused_resident_kernel(EnvConst C, EnvState st, EnsDev E, FusedArgs F) {
  constexpr int K = kRK, H = kRH, KK = kRKK, MR = kResRows;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane0 = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int D = C.D, N = C.N, I = C.I, S = C.S;
  const int n0 = blockIdx.x * F.tile_envs;
  const int M = min(F.tile_envs, N - n0);
  const int n_mkt = (1 + I) * D;  // market entries of a state row: closes, indicators

  // ---------------------------------------------------------------- set-up
  // W2 fragments of this wavefront's output tiles.  Actors 0 and 1 are placed in the
  // accumulation registers (the MFMAs read them there), actor 2 in the vector registers.
  bf16x8 w2[K][KK][4];
#pragma unroll
  for (int a = 0; a < K; ++a)
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        w2[a][kk][i] = *reinterpret_cast<const bf16x8*>(E.base + a * E.actor_stride + E.off_w2 +
                                                        static_cast<size_t>((4 * wave + i) * KK + kk) * 1024 + lane0 * 16);
        if (a < 2) asm volatile("" : "+a"(w2[a][kk][i]));
      }
  // Entry i of step t's input buffer: close[t] | close[t+1] (i < 2D), ind[t+1] (from kRInd).
  auto load_in = [&](int t, int i) -> float {
    if (i < D) return C.close[static_cast<size_t>(t) * D + i];
    if (i < 2 * D) return C.close[static_cast<size_t>(t + 1) * D + (i - D)];
    if (i >= kRInd && i - kRInd < I * D) return C.ind[static_cast<size_t>(t + 1) * I * D + (i - kRInd)];
    return 0.0f;
  };
  {
    bf16x8* s_w1e = reinterpret_cast<bf16x8*>(smem + RLds::w1e);
    bf16x8* s_w3 = reinterpret_cast<bf16x8*>(smem + RLds::w3);
    float* s_b2 = reinterpret_cast<float*>(smem + RLds::b2);
    float* s_b3 = reinterpret_cast<float*>(smem + RLds::b3);
    float* s_mix = reinterpret_cast<float*>(smem + RLds::mix);
    __bf16* s_x0 = reinterpret_cast<__bf16*>(smem + RLds::x0);
    float* s_mt = reinterpret_cast<float*>(smem + RLds::mt);
    float* s_in = reinterpret_cast<float*>(smem + RLds::in);
    for (int f = wave; f < K * 16; f += 4)
      s_w1e[f * 64 + lane0] = *reinterpret_cast<const bf16x8*>(E.base + E.off_w1e + static_cast<size_t>(f) * 1024 + lane0 * 16);
    for (int f = wave; f < K * 2 * KK; f += 4) {
      const int a = f / (2 * KK), r = f - a * 2 * KK;
      s_w3[f * 64 + lane0] = *reinterpret_cast<const bf16x8*>(E.base + a * E.actor_stride + E.off_w3 +
                                                              static_cast<size_t>(r) * 1024 + lane0 * 16);
    }
    for (int i = tid; i < K * H; i += kRT) {
      const int a = i / H, c = i - a * H;
      s_b2[i] = reinterpret_cast<const float*>(E.base + a * E.actor_stride + E.off_b2)[c];
    }
    if (tid < K * 32) {
      const int a = tid / 32, c = tid - a * 32;
      s_b3[tid] = reinterpret_cast<const float*>(E.base + a * E.actor_stride + E.off_b3)[c];
    }
    if (tid < K) s_mix[tid] = E.mix[tid];
    for (int i = tid; i < MR * kRX0; i += kRT) s_x0[i] = static_cast<__bf16>(0.0f);
    // Input buffers of the first two steps (later ones are fetched two steps ahead).
    for (int i = tid; i < kRInBuf; i += kRT) {
      s_in[i] = load_in(F.t0, i);
      if (F.n_steps > 1) s_in[kRInBuf + i] = load_in(F.t0 + 1, i);
    }
#pragma unroll
    for (int r = 0; r < K; ++r) s_mt[tid + kRT * r] = F.mt[tid + kRT * r];
  }
  __syncthreads();

  // The trading state.  Wavefront w trades environments 2w and 2w+1: 16-lane row r of the
  // wavefront works on environment 2w + (r & 1) (rows 2 and 3 repeat rows 0 and 1), lane j of a
  // row on stocks j and j + 16.  Holdings live in the lanes' registers; cash, value and
  // cumulative reward live in LDS between steps.
  const int tm = 2 * wave + ((lane0 >> 4) & 1), tj = lane0 & 15;
  const bool tenv = tm < M;
  int hold[2] = {0, 0};
  if (tenv) {
    const double cash = st.cash[n0 + tm];
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (tj + 16 * s < D) hold[s] = st.hold[static_cast<size_t>(tj + 16 * s) * N + n0 + tm];
    if (lane0 < 32) {
      __bf16* s_x0 = reinterpret_cast<__bf16*>(smem + RLds::x0);
#pragma unroll
      for (int s = 0; s < 2; ++s)
        if (tj + 16 * s < D)
          s_x0[tm * kRX0 + 1 + tj + 16 * s] = static_cast<__bf16>(static_cast<float>(hold[s]) * C.hold_scale);
      if (tj == 0) {
        s_x0[tm * kRX0] = static_cast<__bf16>(static_cast<float>(cash * static_cast<double>(C.cash_scale)));
        double* s_state = reinterpret_cast<double*>(smem + RLds::state) + 4 * tm;
        s_state[0] = cash;
        s_state[1] = st.asset[n0 + tm];
        s_state[2] = st.cumrew[n0 + tm];
      }
    }
  }
  __syncthreads();

  // The state rows of a step are assembled in LDS as float32 images (double-buffered): the market
  // entries (closes, indicators) of step jj's rows from its market rows, 64 entries by each
  // wavefront at the end of the step's layer 3 (wavefronts 0-2 would otherwise wait there for
  // wavefront 3's stores), and the cash and holdings entries by the trading lanes.  The tile's
  // rows of a step are contiguous in the trajectory, so the image is stored whole, with
  // 16-byte stores where the rows start on a 16-byte boundary, during the next step's layer 3
  // (and after the loop for the last step).
  const bool obs_on = F.obs_traj != nullptr;
  // No per-row branches: rows past M are filled too and never stored.
  static_assert(kRIn == 64 * 4, "one 64-entry chunk of the market entries per wavefront");
  auto fill_image = [&](const float* in_jj, float* img_jj, int lane_, int k) {
    const int u = lane_ + 64 * k;  // market entry u of a state row: close[t+1] (u < D), then ind[t+1]
    if (u < n_mkt) {
      const bool cl = u < D;
      const float x = in_jj[cl ? D + u : kRInd + u - D];
      const float v = x * (cl ? C.price_scale : 1.0f);  // closes scaled, indicators as they are
      const int pos = 1 + u + (cl ? 0 : D);             // closes at entries 1 .. D, indicators from 1 + 2D
#pragma unroll
      for (int e = 0; e < MR; ++e) img_jj[e * S + pos] = v;
    }
  };
  auto store_image = [&](int jj, const float* img_jj, int lane_) {
    const int total = M * S;
    const size_t base = (static_cast<size_t>(jj) * N + n0) * S;
    const __amdgpu_buffer_rsrc_t r = rows_rsrc(F.obs_traj, base, 4, total);
    if ((reinterpret_cast<uintptr_t>(F.obs_traj + base) & 15) == 0 && (total & 3) == 0) {
      typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
      constexpr int kQ = (kRImg / 4 + 63) / 64;
      u32x4 v[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) v[q] = reinterpret_cast<const u32x4*>(img_jj)[min(lane_ + 64 * q, kRImg / 4 - 1)];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int i4 = lane_ + 64 * q;
        __builtin_amdgcn_raw_buffer_store_b128(v[q], r, 4 * i4 < total ? 16 * i4 : kNoStore, 0, 0);
      }
    } else {
      for (int q = 0; 64 * q < total; ++q) {
        const int i = lane_ + 64 * q;
        store_f32(r, i < total ? 4 * i : kNoStore, img_jj[min(i, kRImg - 1)]);
      }
    }
  };
  // Every set-up load has landed: a load still counted as pending on entry would make the
  // compiler wait for all memory operations, stores included, at the top of every step.
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  for (int j = 0; j < F.n_steps; ++j) {
    const int b = j & 1;       // this step's table row buffer
    const int bi = j % 3;      // this step's market-row buffer
    const bool nxt = j + 1 < F.n_steps;
    // Addresses derived from the lane and the LDS base are recomputed every step rather than
    // held across the loop: the weights leave few registers for loop-invariant values.
    const int z = opaque_zero();
    const int lane = threadIdx.x % 64 + z;
    unsigned char* sm = smem + z;
    const bf16x8* s_w1e = reinterpret_cast<const bf16x8*>(sm + RLds::w1e);
    const bf16x8* s_w3 = reinterpret_cast<const bf16x8*>(sm + RLds::w3);
    __bf16* s_x1 = reinterpret_cast<__bf16*>(sm + RLds::x1);
    float* s_mu = reinterpret_cast<float*>(sm + RLds::mu);
    __bf16* s_x2 = reinterpret_cast<__bf16*>(sm + RLds::x2);
    __bf16* s_x0 = reinterpret_cast<__bf16*>(sm + RLds::x0);
    const float* s_b2 = reinterpret_cast<const float*>(sm + RLds::b2);
    const float* s_b3 = reinterpret_cast<const float*>(sm + RLds::b3);
    const float* s_mix = reinterpret_cast<const float*>(sm + RLds::mix);
    float* s_mt = reinterpret_cast<float*>(sm + RLds::mt);
    float* s_in = reinterpret_cast<float*>(sm + RLds::in);
    double* s_state = reinterpret_cast<double*>(sm + RLds::state);
    float* s_img = reinterpret_cast<float*>(sm + RLds::img);
    // This step's noise and the next step's inputs, requested now, used after the MLP.
    const int m = 2 * wave + ((lane >> 4) & 1), jl = lane & 15;
    const bool env_ok = m < M;
    // Loads through buffer resources: out-of-range lanes read 0, so no branches.
    float eps[2];
    {
      const __amdgpu_buffer_rsrc_t r =
          rows_rsrc(F.sigma != 0.0f ? F.eps : nullptr, (static_cast<size_t>(j) * N + n0) * D, 4, M * D);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int d = jl + 16 * s;
        eps[s] = load_f32(r, env_ok && d < D ? 4 * (m * D + d) : kNoStore);
      }
    }
    // The next step's table row, straight into LDS, 64 floats per load, a third by each of
    // wavefronts 0-2 (wavefront 3 fetches the market rows, two steps ahead, in layer 3).
    if (nxt && wave < K) {
      constexpr int kPer = K * H / 64 / 3;  // 64-float runs of the table row per wavefront
      const __amdgpu_buffer_rsrc_t rm = rows_rsrc(F.mt, static_cast<size_t>(j + 1) * K * H, 4, K * H);
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int o = 64 * (kPer * wave + q);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rm, s_mt + (b ^ 1) * K * H + o, 4, 4 * (lane + o), 0, 0, 0);
      }
    }
    // ------------------------------------------------------------ L1
    layer1(s_w1e, s_mt + b * K * H, s_x0, s_x1, wave, lane);
    __syncthreads();  // 1: layer-1 outputs complete
    // ------------------------------------------------------------ L2
    layer2(w2, s_b2, s_x1, s_x2, wave, lane);
    __syncthreads();  // 2: layer-2 outputs complete
    // ------------------------------------------------------------ L3: actor a on wavefront a
    if (wave < K) {
      layer3(s_w3, s_b3, s_mix, s_x2, s_mu, wave, lane);
    } else {
      // The next step's market rows (requested in the previous step's layer 3) have landed in
      // LDS, visible to all after the barriers below; then the market rows two steps ahead are
      // requested, and the previous step's state rows go out from their image.
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      if (j + 2 < F.n_steps) {
        // The market rows close[t] | close[t+1] | ind[t+1] of step j + 2 into its input buffer
        // (last read in step j - 1), 64 floats per load, lanes past a range writing zeros;
        // waited for in step j + 1's layer 3.
        const int t = F.t0 + j + 2;
        float* in_n = s_in + ((j + 2) % 3) * kRInBuf;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rows_rsrc(C.close, static_cast<size_t>(t) * D, 4, 2 * D), in_n, 4,
                                                 4 * lane, 0, 0, 0);
        const __amdgpu_buffer_rsrc_t ri = rows_rsrc(C.ind, static_cast<size_t>(t + 1) * I * D, 4, I * D);
        for (int q = 0; 64 * q < I * D; ++q)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(ri, in_n + kRInd + 64 * q, 4, 4 * (lane + 64 * q), 0, 0, 0);
      }
      if (obs_on && j >= 1) store_image(j - 1, s_img + ((j - 1) & 1) * kRImg, lane);
    }
    // This step's image receives its market entries, chunk `wave` of them.
    if (obs_on) fill_image(s_in + bi * kRInBuf, s_img + (j & 1) * kRImg, lane, wave);
    __syncthreads();  // 3: the actors' weighted means complete
    // Wavefronts 0-2: their share of the next table row has landed in LDS (requested at the top of
    // the step, so this wait costs nothing; it precedes the trade's stores, which it would
    // otherwise also wait for at the end of the step).
    if (wave < K) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    {
      // ---------------------------------------------------------- the trading step
#pragma clang fp contract(off)
      const float* in = s_in + bi * kRInBuf;
      const size_t row = static_cast<size_t>(j) * N + n0 + m;
      const bool store_row = env_ok && lane < 32;  // rows 2 and 3 repeat rows 0 and 1
      const size_t row0 = static_cast<size_t>(j) * N + n0;  // the tile's first row of step j
      const int em = m * D;                                 // environment m's first entry in [M][D]
      double cash = s_state[4 * m];
      int sold[2];
      BuySet B[2];
      double pro[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int d = jl + 16 * s;
        const bool on = env_ok && d < D;
        // Action: a_bar = sum_k w_k tanh(z_k + b3_k) in actor order, noise, clip (Section 5.2.1).
        // Formed on every lane (m < 8 and d < 32 stay inside the means) and kept where on: the
        // noise load is then consumed on every path, and no load is left pending at the next step.
        const float* mk = s_mu + m * 32 + d;
        const float mean = (mk[0] + mk[MR * 32]) + mk[2 * MR * 32];
        const float noisy = F.sigma != 0.0f ? mean + F.sigma * eps[s] : mean;
        const float act = on ? fminf(fmaxf(noisy, -1.0f), 1.0f) : 0.0f;
        store_f32(rows_rsrc(F.act_traj, row0 * D, 4, M * D), on && lane < 32 ? 4 * (em + d) : kNoStore, act);
        // Order and sale of stock d; the whole-order and one-share debits.
        const float p = on ? in[d] : 0.0f;
        const int q = on ? order_from_action(act, C.hmax_f) : 0;
        sold[s] = q < 0 ? min(hold[s], -q) : 0;
        hold[s] -= sold[s];
        const double pd = static_cast<double>(p);
        const int qd = q > 0 ? q : 0;
        pro[s] = (pd * static_cast<double>(sold[s])) * C.one_m;
        B[s].deb = (pd * static_cast<double>(qd)) * C.one_p;
        B[s].c1 = pd * C.one_p;
        B[s].pq = pack_pq(p, qd);
      }
      // The cash recurrence: all sells in ascending stock order, then the buys (Section 3.1,
      // readings 5-7); stocks beyond D carry zero terms, which leave the cash unchanged.
      cash = row_sum(cash, pro[0]);
      cash = row_sum(cash, pro[1]);
      int kown[2] = {0, 0};
      buy_all_seg(cash, kown, lane, B, C.one_p);
      // Holdings, executed quantities, the new day's position values, value and reward
      // (Section 3.1 reward, reading 8).
      double val[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int d = jl + 16 * s;
        const bool on = env_ok && d < D;
        hold[s] += kown[s];
        const float pn = on ? in[D + d] : 0.0f;
        val[s] = static_cast<double>(pn) * static_cast<double>(hold[s]);
        const float he = static_cast<float>(hold[s]) * C.hold_scale;
        if (on) s_x0[m * kRX0 + 1 + d] = static_cast<__bf16>(he);
        const bool st_on = on && lane < 32;
        store_f32(rows_rsrc(F.qty_traj, row0 * D, 4, M * D), st_on ? 4 * (em + d) : kNoStore,
                  __int_as_float(kown[s] - sold[s]));
        if (st_on) s_img[(j & 1) * kRImg + m * S + 1 + D + d] = he;
      }
      double v_new = row_sum(cash, val[0]);
      v_new = row_sum(v_new, val[1]);
      if (store_row && jl == 0) {
        const double r = (v_new - s_state[4 * m + 1]) * C.reward_scale;
        const float ce = static_cast<float>(cash * static_cast<double>(C.cash_scale));
        s_state[4 * m] = cash;
        s_state[4 * m + 1] = v_new;
        s_state[4 * m + 2] = s_state[4 * m + 2] + r;
        s_x0[m * kRX0] = static_cast<__bf16>(ce);
        typedef __attribute__((ext_vector_type(2))) unsigned u32x2;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, r), rows_rsrc(F.rew_traj, row0, 8, M), 8 * m, 0, 0);
        s_img[(j & 1) * kRImg + m * S] = ce;
      }
    }
    __syncthreads();  // 4: the next state rows and inputs are in LDS
  }
  if (obs_on && F.n_steps >= 1 && wave == 3)
    store_image(F.n_steps - 1, reinterpret_cast<const float*>(smem + RLds::img) + ((F.n_steps - 1) & 1) * kRImg, lane0);
  // The trading state back to HBM.
  if (tenv && lane0 < 32) {
    if (tj == 0) {
      const double* s_state = reinterpret_cast<const double*>(smem + RLds::state) + 4 * tm;
      st.cash[n0 + tm] = s_state[0];
      st.asset[n0 + tm] = s_state[1];
      st.cumrew[n0 + tm] = s_state[2];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (tj + 16 * s < D) st.hold[static_cast<size_t>(tj + 16 * s) * N + n0 + tm] = hold[s];
  }
}

}  // namespace

bool fused_resident_shape(const EnvConst& C, const EnsDev& E) {
  return fused_streamed_shape(C, E) && C.D <= 31 && E.ke_pad == 32 && (2 + C.I) * C.D <= kRIn;
}

// Per chunk of at most kFusedChunk steps: the chunk's market table and noise, then the resident
// kernel for the chunk's steps.
hipError_t launch_resident(const EnvConst& C, const EnvState& st, const EnsDev& E, FusedArgs F, float* eps_chunk,
                           float* mt_chunk, hipStream_t stream) {
  if (F.tile_envs < 1 || F.tile_envs > kResRows) return hipErrorInvalidValue;
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(fused_resident_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(RLds::total));
  if (err != hipSuccess) return err;
  const int t_end = F.t0 + F.n_steps;
  const size_t N = C.N, D = C.D, S = C.S;
  const int grid = (C.N + F.tile_envs - 1) / F.tile_envs;
  for (int t = F.t0; t < t_end; t += kFusedChunk) {
    const int n = t_end - t < kFusedChunk ? t_end - t : kFusedChunk;
    const size_t i0 = static_cast<size_t>(t - F.t0);
    err = launch_chunk_inputs(C, E, t, n, F.sigma, F.key, F.env_offset, eps_chunk, mt_chunk, stream);
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
    hipLaunchKernelGGL(fused_resident_kernel, dim3(grid), dim3(kRT), RLds::total, stream, C, st, E, Fc);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace fm
