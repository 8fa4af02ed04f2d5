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
//         next state row, and the trajectory stores straight from registers.
// The step's noise (drawn per chunk by noise_chunk_kernel) and the next step's market rows and
// table row are requested at the top of a step and used after the MLP.
#include <cstring>
#include <utility>

#include "device_common.h"
#include "fused.h"
#include "mlp_device.h"

namespace fm {

namespace {

constexpr int kRT = 256;     // threads per workgroup
constexpr int kRK = 3, kRH = 256, kRKK = 8;
constexpr int kRX0 = 40;     // state-row stride (bfloat16): cash, <= 31 holdings, zeros
constexpr int kRXS = 264;    // hidden-row stride (bfloat16)
constexpr int kRIn = 256;    // market entries per day, (2 + I) * D <= 256

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
  static constexpr size_t mt = mix + 16;                                           // [K][256] f32
  static constexpr size_t in = mt + sizeof(float) * kRK * kRH;                     // [2][256] f32
  static constexpr size_t state = in + sizeof(float) * 2 * kRIn;                   // [8] {cash, value, cumrew, 0} f64
  static constexpr size_t total = state + sizeof(double) * 4 * kResRows;
  static_assert(sizeof(float) * kRK * kResRows * 32 <= xb, "the actor means fit the layer-1 region");
};
static_assert(RLds::total <= 160 * 1024, "LDS budget");

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

// Lane L of each 16-lane row, broadcast to the whole row (64-bit DPP row broadcast).
template <int L>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(__builtin_nondeterministic_value(v), v, 0x150 + L, 0xf, 0xf, true);
}
template <int L>
__device__ __forceinline__ long row_bcast(long v) {
  return __builtin_amdgcn_update_dpp(__builtin_nondeterministic_value(v), v, 0x150 + L, 0xf, 0xf, true);
}

// acc + v(lane 0) + v(lane 1) + ... + v(lane 15) of the row, in lane order.
template <int... L>
__device__ __forceinline__ double row_sum_impl(double acc, double v, std::integer_sequence<int, L...>) {
#pragma clang fp contract(off)
  ((acc = acc + row_bcast<L>(v)), ...);
  return acc;
}
__device__ __forceinline__ double row_sum(double acc, double v) {
  return row_sum_impl(acc, v, std::make_integer_sequence<int, 16>());
}

template <class Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>());
}

// One stock's buy terms, owned by one lane of the row: the whole order's debit (p q)(1+c), the
// one-share debit (p 1)(1+c), and the price and order packed as {float bits, int}.
struct BuySet {
  double deb, c1;
  long pq;
};
__device__ __forceinline__ long pack_pq(float p, int q) {
  return static_cast<long>((static_cast<unsigned long>(static_cast<unsigned>(q)) << 32) | __float_as_uint(p));
}
__device__ __forceinline__ float pq_price(long pq) { return __uint_as_float(static_cast<unsigned>(pq)); }
__device__ __forceinline__ int pq_order(long pq) { return static_cast<int>(static_cast<unsigned long>(pq) >> 32); }

// The buy of one stock whose whole order of q shares does not fit the cash while one share does
// (Section 3.1, reading 7): the largest k in [0, q-1] with debit(k) = (p k)(1+c) <= cash.  The
// estimate kd = floor(cash / c1), from the refined reciprocal of the one-share debit c1 and
// clamped to [0, q-1], is at most one share off; the debits of kd-1 .. kd+2 are formed side by
// side and the answer is the largest of kd-1, kd, kd+1 that fits.  If the answer were not in
// that range (kd-1 does not fit, or kd+2 does), ok is false and the caller takes unit steps.
__device__ __forceinline__ int partial_fill_sel(double cash, double p, double c1, int q, double one_p, double& debit,
                                               bool& ok) {
#pragma clang fp contract(off)
  double rc1 = __builtin_amdgcn_rcp(c1);
  rc1 = fma(fma(-c1, rc1, 1.0), rc1, rc1);
  const double kd = fmax(fmin(floor(cash * rc1), static_cast<double>(q - 1)), 0.0);
  const double dm = (p * (kd - 1.0)) * one_p, d0 = (p * kd) * one_p;
  const double dp = (p * (kd + 1.0)) * one_p, dpp = (p * (kd + 2.0)) * one_p;
  const bool fm = kd <= 1.0 || dm <= cash, f0 = kd <= 0.0 || d0 <= cash, fp = dp <= cash, fpp = dpp <= cash;
  ok = fm && !fpp;
  const int k = static_cast<int>(kd);
  debit = fp ? dp : (f0 ? d0 : (k >= 2 ? dm : 0.0));
  return fp ? k + 1 : (f0 ? k : (k >= 1 ? k - 1 : 0));
}

// Buy of stock N of the row's environment (Section 3.1, readings 5-7), every lane of the row
// computing the same recurrence on terms broadcast from the lane that owns the stock; lane j
// keeps the fills of stocks j and j + 16 in k[0], k[1].  A buy fills whole when its debit fits
// the cash and not at all when one share does not (selects); the partial fill is evaluated, for
// the whole wavefront, only at a stock where some row needs it.
template <int N>
__device__ __forceinline__ void buy_stock(double& cash, int (&k)[2], int j, const BuySet (&B)[2], double one_p) {
#pragma clang fp contract(off)
  constexpr int s = N / 16, L = N % 16;
  const double deb = row_bcast<L>(B[s].deb), c1 = row_bcast<L>(B[s].c1);
  const long pq = row_bcast<L>(B[s].pq);
  const bool fits = deb <= cash;
  const bool need = !fits && c1 <= cash;
  int kj = fits ? pq_order(pq) : 0;
  double debit = fits ? deb : 0.0;
  if (__builtin_amdgcn_ballot_w64(need) != 0) {
    bool ok = true;
    double dpart;
    const int kp = partial_fill_sel(cash, static_cast<double>(pq_price(pq)), c1, pq_order(pq), one_p, dpart, ok);
    if (need) {
      kj = kp;
      debit = dpart;
    }
    if (__builtin_amdgcn_ballot_w64(need && !ok) != 0) {
      if (need && !ok) {
        double rc1 = __builtin_amdgcn_rcp(c1);
        rc1 = fma(fma(-c1, rc1, 1.0), rc1, rc1);
        kj = partial_fill(cash, static_cast<double>(pq_price(pq)), rc1, pq_order(pq), one_p, debit);
      }
    }
  }
  cash = cash - debit;
  k[s] = j == L ? kj : k[s];
}

// Stocks 4C .. 4C+3, unless no row of the wavefront can still buy: once the cash is below the
// day's lowest price (a lower bound of every one-share debit), no later order fills even in
// part, and the remaining stocks leave cash and fills unchanged.
template <int C>
__device__ __forceinline__ void buy_chunk(double& cash, int (&k)[2], int j, const BuySet (&B)[2], double one_p,
                                          double p_min, bool& live) {
  if (!live) return;
  buy_stock<4 * C>(cash, k, j, B, one_p);
  buy_stock<4 * C + 1>(cash, k, j, B, one_p);
  buy_stock<4 * C + 2>(cash, k, j, B, one_p);
  buy_stock<4 * C + 3>(cash, k, j, B, one_p);
  live = __builtin_amdgcn_ballot_w64(cash >= p_min) != 0;
}

template <int... C>
__device__ __forceinline__ void buy_all(double& cash, int (&k)[2], int j, const BuySet (&B)[2], double one_p,
                                        double p_min, std::integer_sequence<int, C...>) {
  bool live = __builtin_amdgcn_ballot_w64(cash >= p_min) != 0;
  (buy_chunk<C>(cash, k, j, B, one_p, p_min, live), ...);
}

// Minimum over the 16 lanes of each row (DPP row rotations).
__device__ __forceinline__ float row_min(float v) {
  v = fminf(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false));  // row_ror:8
  v = fminf(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xf, 0xf, false));  // row_ror:4
  v = fminf(v, __builtin_amdgcn_update_dpp(v, v, 0x122, 0xf, 0xf, false));  // row_ror:2
  v = fminf(v, __builtin_amdgcn_update_dpp(v, v, 0x121, 0xf, 0xf, false));  // row_ror:1
  return v;
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
  const int n_in = (2 + I) * D;
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
  // Market rows close[t] | close[t+1] | ind[t+1] of step t's trade (entry tid of the row).
  auto load_in = [&](int t) -> float {
    const int i = tid;
    if (i < D) return C.close[static_cast<size_t>(t) * D + i];
    if (i < 2 * D) return C.close[static_cast<size_t>(t + 1) * D + (i - D)];
    if (i < n_in) return C.ind[static_cast<size_t>(t + 1) * I * D + (i - 2 * D)];
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
    s_in[tid] = load_in(F.t0);
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

  for (int j = 0; j < F.n_steps; ++j) {
    const int b = j & 1;
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
    // This step's noise and the next step's inputs, requested now, used after the MLP.
    const int m = 2 * wave + ((lane >> 4) & 1), jl = lane & 15;
    const bool env_ok = m < M;
    float eps[2] = {0.0f, 0.0f};
    if (env_ok && F.sigma != 0.0f) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
        if (jl + 16 * s < D) eps[s] = F.eps[(static_cast<size_t>(j) * N + n0 + m) * D + jl + 16 * s];
    }
    float p_in = 0.0f, p_mt[K] = {0.0f, 0.0f, 0.0f};
    if (nxt) {
      p_in = load_in(F.t0 + j + 1);
#pragma unroll
      for (int r = 0; r < K; ++r) p_mt[r] = F.mt[static_cast<size_t>(j + 1) * K * H + tid + kRT * r];
    }
    // ------------------------------------------------------------ L1
    // Lane l's B operand: state row of environment l mod 8, entries 8(l/16) .. +7.  Lane l's
    // results: tile T = (l / 8) mod 2 of the wavefront's pair, environment l mod 8, units
    // u0 .. u0+3.
    const int bev = lane & 7, bgrp = lane >> 4;
    const int pair_t = (lane >> 3) & 1;
    {
      const bf16x8 X = *reinterpret_cast<const bf16x8*>(s_x0 + bev * kRX0 + 8 * bgrp);
#pragma unroll
      for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          floatx4 acc[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int c = 4 * wave + 2 * p + h;
            acc[h] = mfma_bf16(s_w1e[(a * 16 + c) * 64 + lane], X,
                               *reinterpret_cast<const floatx4*>(s_mt + a * H + 16 * c + 4 * bgrp));
          }
          const floatx4 v = merge_tiles(acc[0], acc[1]);
          const int u0 = 16 * (4 * wave + 2 * p + pair_t) + 4 * bgrp;
          *reinterpret_cast<uint2*>(s_x1 + a * MR * kRXS + bev * kRXS + u0) =
              pack_bf16x4(tanh_sig(v[0]), tanh_sig(v[1]), tanh_sig(v[2]), tanh_sig(v[3]));
        }
      }
    }
    __syncthreads();  // 1: layer-1 outputs complete
    // ------------------------------------------------------------ L2
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const __bf16* src = s_x1 + a * MR * kRXS + bev * kRXS + 8 * bgrp;
      bf16x8 X[KK];
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) X[kk] = *reinterpret_cast<const bf16x8*>(src + 32 * kk);
      floatx4 acc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i] = mfma_bf16(w2[a][0][i], X[0], *reinterpret_cast<const floatx4*>(s_b2 + a * H + 16 * (4 * wave + i) + 4 * bgrp));
#pragma unroll
      for (int kk = 1; kk < KK; ++kk)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = mfma_bf16(w2[a][kk][i], X[kk], acc[i]);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const floatx4 v = merge_tiles(acc[2 * p], acc[2 * p + 1]);
        const int u0 = 16 * (4 * wave + 2 * p + pair_t) + 4 * bgrp;
        *reinterpret_cast<uint2*>(s_x2 + a * MR * kRXS + bev * kRXS + u0) =
            pack_bf16x4(tanh_sig(v[0]), tanh_sig(v[1]), tanh_sig(v[2]), tanh_sig(v[3]));
      }
    }
    __syncthreads();  // 2: layer-2 outputs complete
    // ------------------------------------------------------------ L3: actor a on wavefront a
    if (wave < K) {
      const int a = wave;
      const __bf16* src = s_x2 + a * MR * kRXS + bev * kRXS + 8 * bgrp;
      floatx4 acc[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h] = *reinterpret_cast<const floatx4*>(s_b3 + a * 32 + 16 * h + 4 * bgrp);
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) {
        const bf16x8 X = *reinterpret_cast<const bf16x8*>(src + 32 * kk);
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[h] = mfma_bf16(s_w3[((a * 2 + h) * KK + kk) * 64 + lane], X, acc[h]);
      }
      const floatx4 v = merge_tiles(acc[0], acc[1]);
      const float wk = s_mix[a];
      *reinterpret_cast<float4*>(s_mu + a * MR * 32 + bev * 32 + 16 * pair_t + 4 * bgrp) =
          float4{wk * tanh_sig(v[0]), wk * tanh_sig(v[1]), wk * tanh_sig(v[2]), wk * tanh_sig(v[3])};
    }
    __syncthreads();  // 3: the actors' weighted means complete
    {
      // ---------------------------------------------------------- the trading step
#pragma clang fp contract(off)
      const float* in = s_in + b * kRIn;
      const size_t row = static_cast<size_t>(j) * N + n0 + m;
      const bool store_row = env_ok && lane < 32;  // rows 2 and 3 repeat rows 0 and 1
      // The new state row's market entries (closes, indicators) do not depend on the trades:
      // stored first, by both rows of the environment.
      float* o = F.obs_traj ? F.obs_traj + row * S : nullptr;
      if (env_ok && o) {
        const int t32 = ((lane >> 5) << 4) | jl;  // 0 .. 31 over the environment's two rows
        float v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {  // (1 + I) D <= 255
          const int u = t32 + 32 * r;
          v[r] = u < n_mkt ? in[D + u] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int u = t32 + 32 * r;
          if (u < D) o[1 + u] = v[r] * C.price_scale;
          else if (u < n_mkt) o[1 + D + u] = v[r];
        }
      }
      double cash = s_state[4 * m];
      int sold[2];
      BuySet B[2];
      double pro[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int d = jl + 16 * s;
        const bool on = env_ok && d < D;
        // Action: a_bar = sum_k w_k tanh(z_k + b3_k) in actor order, noise, clip (Section 5.2.1).
        float act = 0.0f;
        if (on) {
          const float* mk = s_mu + m * 32 + d;
          act = (mk[0] + mk[MR * 32]) + mk[2 * MR * 32];
          if (F.sigma != 0.0f) act = act + F.sigma * eps[s];
          act = fminf(fmaxf(act, -1.0f), 1.0f);
          if (F.act_traj && lane < 32) F.act_traj[row * D + d] = act;
        }
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
      const float p_min = row_min(fminf(jl < D ? in[jl] : __builtin_inff(), jl + 16 < D ? in[jl + 16] : __builtin_inff()));
      buy_all(cash, kown, jl, B, C.one_p, static_cast<double>(p_min), std::make_integer_sequence<int, 8>());
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
        if (on && lane < 32) {
          s_x0[m * kRX0 + 1 + d] = static_cast<__bf16>(he);
          if (F.qty_traj) F.qty_traj[row * D + d] = kown[s] - sold[s];
          if (o) o[1 + D + d] = he;
        }
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
        if (F.rew_traj) F.rew_traj[row] = r;
        if (o) o[0] = ce;
      }
    }
    if (nxt) {
      s_in[(b ^ 1) * kRIn + tid] = p_in;
#pragma unroll
      for (int r = 0; r < K; ++r) s_mt[tid + kRT * r] = p_mt[r];
    }
    __syncthreads();  // 4: the next state rows and inputs are in LDS
  }
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
