// Device-side building blocks shared by the environment, ensemble and fused rollout kernels:
// the Philox4x64-10 noise generator, the Box-Muller map, and the per-environment trading chain.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

// ------------------------------------------------------------------------------------------
// Environment constants as the kernels see them.
// ------------------------------------------------------------------------------------------
struct EnvConst {
  int N, D, I, T, S, hmax;
  float hmax_f, cash_scale, price_scale, hold_scale;
  double init_cash, one_m, one_p, reward_scale;
  const float* close;  // [T+1][D]
  const float* ind;    // [T+1][I][D]
};

// Environment state in the workspace, structure-of-arrays with the env index fastest.
struct EnvState {
  double* cash;    // [N]
  double* asset;   // [N]  v_t, the pre-trade value at the current day's close
  double* cumrew;  // [N]
  int* hold;       // [D][N]
};

// ------------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 64x64->128 multiplies
// of counter words 0 and 2, XOR of the high halves with words 1 and 3 and the round key, and a
// Weyl increment of the key between rounds.
// ------------------------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;  // golden ratio
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;  // sqrt(3) - 1

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                              uint64_t& c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// Top 23 bits of the word, centred: ((w >> 41) + 0.5) * 2^-23, exact in float32, in (0, 1).
__device__ __forceinline__ float uniform_from_word(uint64_t w) {
  return (static_cast<float>(static_cast<uint32_t>(w >> 41)) + 0.5f) * 0x1p-23f;
}

// Box-Muller: two standard normals from two uniforms.  cos/sin of 2*pi*u use the pi-scaled
// forms so that the argument 2u is exact.
__device__ __forceinline__ void box_muller(float ua, float ub, float& z0, float& z1) {
  const float r = sqrtf(-2.0f * logf(ua));
  float s, c;
  sincospif(2.0f * ub, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// The noise block for environment n, day t, stock group j (stocks 4j..4j+3): key
// (noise_key, 0), counter (n, t, j, 0).  Writes the raw words if w != nullptr.
__device__ __forceinline__ void noise_block(uint64_t key, uint64_t n, uint64_t t, uint64_t j,
                                            float z[4], uint64_t* w = nullptr) {
  uint64_t c0 = n, c1 = t, c2 = j, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, key, 0);
  if (w) {
    w[0] = c0;
    w[1] = c1;
    w[2] = c2;
    w[3] = c3;
  }
  box_muller(uniform_from_word(c0), uniform_from_word(c1), z[0], z[1]);
  box_muller(uniform_from_word(c2), uniform_from_word(c3), z[2], z[3]);
}

// ------------------------------------------------------------------------------------------
// Orders and the trading chain.  Every float64 operation below rounds once: the library is
// built with contraction off and the pragma repeats that for these functions.
// ------------------------------------------------------------------------------------------

// q = trunc(fl32(clamp(a, -1, 1) * hmax)); NaN -> 0.
__device__ __forceinline__ int order_from_action(float a, float hmax_f) {
#pragma clang fp contract(off)
  a = (a == a) ? fminf(fmaxf(a, -1.0f), 1.0f) : 0.0f;
  const float prod = a * hmax_f;
  return static_cast<int>(truncf(prod));
}

// Largest k in [0, q] with (p*k)*one_p <= cash, for the case (p*q)*one_p > cash.  The debit is
// monotone in k, so a quotient estimate (from an approximate reciprocal) followed by unit steps
// in both directions is exact whatever the estimate's error; the steps are bounded by q.
__device__ __forceinline__ int partial_fill(double cash, double p, int q, double one_p) {
#pragma clang fp contract(off)
  const double c1 = p * one_p;
  if (!(c1 <= cash)) return 0;
  const double est = floor(cash * __builtin_amdgcn_rcp(c1));
  int k = static_cast<int>(fmin(fmax(est, 0.0), static_cast<double>(q)));
  while (k < q && (p * static_cast<double>(k + 1)) * one_p <= cash) ++k;
  while (k > 0 && (p * static_cast<double>(k)) * one_p > cash) --k;
  return k;
}

// One day's trades for one environment held in registers: all sells in ascending stock order,
// then all buys in ascending stock order, at prices px (float32, day t).  a, px: this env's
// actions and the day's closes, zero-padded beyond the real stock count; a padded stock has no
// order, so it adds +0.0 to (and subtracts +0.0 from) a non-negative cash, which leaves it
// unchanged bit for bit.  x: executed shares (signed).
template <int DMAX>
__device__ __forceinline__ void trade(double& cash, int (&h)[DMAX], int (&x)[DMAX],
                                      const float (&a)[DMAX], const float (&px)[DMAX],
                                      float hmax_f, double one_m, double one_p) {
#pragma clang fp contract(off)
  int q[DMAX];
#pragma unroll
  for (int d = 0; d < DMAX; ++d) q[d] = order_from_action(a[d], hmax_f);
  // Sells: proceeds (p*s)*(1-c); a zero sale adds +0.0.
#pragma unroll
  for (int d = 0; d < DMAX; ++d) {
    const int s = q[d] < 0 ? min(h[d], -q[d]) : 0;
    const double proceeds = (static_cast<double>(px[d]) * static_cast<double>(s)) * one_m;
    cash = cash + proceeds;
    h[d] -= s;
    x[d] = -s;
  }
  // Buys: the whole order if its debit fits, otherwise the largest affordable part.
#pragma unroll
  for (int d = 0; d < DMAX; ++d) {
    const int qd = q[d] > 0 ? q[d] : 0;
    const double p = static_cast<double>(px[d]);
    double debit = (p * static_cast<double>(qd)) * one_p;
    int k = qd;
    if (!(debit <= cash)) {
      k = partial_fill(cash, p, qd, one_p);
      debit = (p * static_cast<double>(k)) * one_p;
    }
    cash = cash - debit;
    h[d] += k;
    x[d] += k;
  }
}

// v = b + p^T h, accumulated in ascending stock order (zero-padded stocks add +0.0).
template <int DMAX>
__device__ __forceinline__ double portfolio_value(double cash, const int (&h)[DMAX],
                                                  const float (&px)[DMAX]) {
#pragma clang fp contract(off)
  double acc = cash;
#pragma unroll
  for (int d = 0; d < DMAX; ++d) acc = acc + static_cast<double>(px[d]) * static_cast<double>(h[d]);
  return acc;
}

// DMAX consecutive floats from a 16-byte-aligned LDS row.
template <int DMAX>
__device__ __forceinline__ void lds_row(float (&v)[DMAX], const float* row) {
  static_assert(DMAX % 4 == 0, "rows are read four floats at a time");
#pragma unroll
  for (int d = 0; d < DMAX; d += 4) {
    const float4 t = *reinterpret_cast<const float4*>(row + d);
    v[d] = t.x;
    v[d + 1] = t.y;
    v[d + 2] = t.z;
    v[d + 3] = t.w;
  }
}

// Exact floor(i / D) for 0 <= i < 2^20 and 1 <= D <= 1024, via a float reciprocal: i/D is at
// least 1/(2D) away from the next integer above it and the float error is far smaller.
__device__ __forceinline__ int div_small(int i, float inv_d) {
  return static_cast<int>((static_cast<float>(i) + 0.5f) * inv_d);
}

// Writes the values val(e), e = 0..total-1, to dst[0..total-1] with one wavefront (lane =
// 0..63): 16-byte stores for the 16-byte-aligned body, single stores for the unaligned head and
// the tail.  val is evaluated for every element exactly once.
template <class T, class Val>
__device__ __forceinline__ void wave_store_row(T* dst, int total, int lane, Val val) {
  static_assert(sizeof(T) == 4, "four-byte elements");
  const int head = min(total, static_cast<int>(((16 - (reinterpret_cast<uintptr_t>(dst) & 15)) & 15) / 4));
  if (lane < head) dst[lane] = val(lane);
  const int nvec = (total - head) / 4;
  T* body = dst + head;
#pragma unroll 2
  for (int q = lane; q < nvec; q += 64) {
    const int e = head + 4 * q;
    T v0 = val(e), v1 = val(e + 1), v2 = val(e + 2), v3 = val(e + 3);
    typedef __attribute__((ext_vector_type(4))) T T4;
    T4 v;
    v.x = v0;
    v.y = v1;
    v.z = v2;
    v.w = v3;
    *reinterpret_cast<T4*>(body + 4 * q) = v;
  }
  const int done = head + 4 * nvec;
  if (done + lane < total) dst[done + lane] = val(done + lane);
}

// ------------------------------------------------------------------------------------------
// The chain of a tile of M environments, split so that only the cash recurrence is serial.
// Every per-stock quantity that does not depend on cash (orders, the sale size, proceeds, the
// debit of the whole order, the new day's position values) is computed by all threads of the
// group over the M*D (env, stock) pairs; one lane per environment then runs the float64 cash
// recurrence in ascending stock order, reading the precomputed terms.  The arithmetic and its
// order are exactly those of trade() / portfolio_value().
//
// LDS rows (stride DS = D + 1 for per-env rows, D for scratch):
//   act[m][d] actions, hold[m][d] holdings (updated), qty[m][d] executed shares (written),
//   env[m][0..D] state entries (written: cash * scale, holdings * scale)
//   pro[m][d], deb[m][d], val[m][d] float64 scratch; qd[m][d], kq[m][d] int scratch
// ------------------------------------------------------------------------------------------
struct ChainLds {
  const float* act;
  int* hold;
  int* qty;
  float* env;
  const float* px;  // trading day closes [D]
  const float* pn;  // new day closes [D]
  double* pro;
  double* deb;
  double* val;
  int* qd;
  int* kq;
};

// Phase A (all threads, pairs i = first, first + stride, ...): orders, sells, whole-order debit.
__device__ __forceinline__ void chain_pairs_a(const ChainLds& L, int M, int D, int first, int stride,
                                              float inv_d, float hmax_f, double one_m, double one_p) {
#pragma clang fp contract(off)
  const int DS = D + 1;
#pragma unroll 4
  for (int i = first; i < M * D; i += stride) {
    const int m = div_small(i, inv_d);
    const int d = i - m * D;
    const int q = order_from_action(L.act[m * DS + d], hmax_f);
    const int h = L.hold[m * DS + d];
    const int s = q < 0 ? min(h, -q) : 0;
    const double p = static_cast<double>(L.px[d]);
    L.hold[m * DS + d] = h - s;
    L.qty[m * DS + d] = -s;
    L.pro[i] = (p * static_cast<double>(s)) * one_m;
    const int qd = q > 0 ? q : 0;
    L.qd[i] = qd;
    L.deb[i] = (p * static_cast<double>(qd)) * one_p;
    L.val[i] = p * one_p;  // debit of one share, (p*1)*(1+c); the slot is reused in phase C
  }
}

// Phase B (lane m of the owner group): the cash recurrence of environment m.  A buy that does not
// fit is filled partially only when at least one share is affordable; that is the one rare,
// divergent branch (the common cases are a whole fill or no fill, both branch-free selects).
__device__ __forceinline__ void chain_serial(double& cash, const double* __restrict__ pro,
                                             const double* __restrict__ deb, const double* __restrict__ c1s,
                                             const int* __restrict__ qd, const float* __restrict__ px,
                                             int* __restrict__ kq, int D, double one_p) {
#pragma clang fp contract(off)
#pragma unroll 8
  for (int d = 0; d < D; ++d) cash = cash + pro[d];  // sells, ascending stock order
#pragma unroll 4
  for (int d = 0; d < D; ++d) {                       // buys, ascending stock order
    const double debit_q = deb[d];
    const double c1 = c1s[d];
    const int q = qd[d];
    const bool fits = debit_q <= cash;
    int k = fits ? q : 0;
    double debit = fits ? debit_q : 0.0;
    if (!fits && c1 <= cash) {
      const double p = static_cast<double>(px[d]);
      k = partial_fill(cash, p, q, one_p);
      debit = (p * static_cast<double>(k)) * one_p;
    }
    cash = cash - debit;
    kq[d] = k;
  }
}

// Phase C (all threads): apply the buys, state entries of the holdings, new-day position values.
__device__ __forceinline__ void chain_pairs_c(const ChainLds& L, int M, int D, int first, int stride,
                                              float inv_d, float hold_scale) {
#pragma clang fp contract(off)
  const int DS = D + 1;
#pragma unroll 4
  for (int i = first; i < M * D; i += stride) {
    const int m = div_small(i, inv_d);
    const int d = i - m * D;
    const int k = L.kq[i];
    const int h = L.hold[m * DS + d] + k;
    L.hold[m * DS + d] = h;
    L.qty[m * DS + d] += k;
    L.env[m * DS + 1 + d] = static_cast<float>(h) * hold_scale;
    L.val[i] = static_cast<double>(L.pn[d]) * static_cast<double>(h);
  }
}

// Phase D (lane m): v = cash + sum_d p'_d h_d in ascending stock order.
__device__ __forceinline__ double chain_value(double cash, const double* __restrict__ val, int D) {
#pragma clang fp contract(off)
  double acc = cash;
#pragma unroll 8
  for (int d = 0; d < D; ++d) acc = acc + val[d];
  return acc;
}

// Holdings entries and values without trading (reset / observe): all threads.
__device__ __forceinline__ void chain_pairs_hold(const ChainLds& L, int M, int D, int first, int stride,
                                                 float inv_d, float hold_scale) {
#pragma clang fp contract(off)
  const int DS = D + 1;
  for (int i = first; i < M * D; i += stride) {
    const int m = div_small(i, inv_d);
    const int d = i - m * D;
    const int h = L.hold[m * DS + d];
    L.env[m * DS + 1 + d] = static_cast<float>(h) * hold_scale;
    L.val[i] = static_cast<double>(L.pn[d]) * static_cast<double>(h);
  }
}

// Synchronisation of one wavefront's LDS traffic between the phases (no hardware barrier:
// a wavefront's LDS operations complete in order; this stops the compiler reordering them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace fm
