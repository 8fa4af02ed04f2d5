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
// debit of the whole order and of one share, the new day's position values) is computed by all
// threads of the group over the (env, stock) pairs; one lane per environment then runs the
// float64 cash recurrence in ascending stock order over the precomputed terms, eight stocks per
// register chunk, with the next chunk's terms read from LDS while the current one is consumed.
//
// LDS rows:
//   act[m][d], hold[m][d], qty[m][d]: stride D (dense, as the tile's rows in HBM);
//   env[m][0..D]: stride D + 1, the cash entry then the holdings entries of the state row;
//   pro/deb/val[m][d] float64 scratch: stride RD; qd/kq[m][d] int scratch: stride RI.
// Scratch rows hold DP >= D stocks, DP a multiple of the chunk; stocks d >= D carry a zero
// order (proceeds 0, debit 0, order 0), and adding or subtracting +0.0 leaves a non-negative
// cash (and a value) unchanged bit for bit, so the recurrence may run over whole chunks.  The
// scratch strides are offset from a multiple of 64 bytes by 16 bytes, so that the lanes of the
// serial phase, each reading its own row, start in different LDS banks.
// ------------------------------------------------------------------------------------------
constexpr int kChunk = 8;

struct ChainShape {
  int D, DP, RD, RI, DS;
  float inv_dp;
  __host__ __device__ static ChainShape of(int D) {
    ChainShape z;
    z.D = D;
    z.DP = (D + kChunk - 1) / kChunk * kChunk;
    z.RD = z.DP + 2;
    z.RI = z.DP + 4;
    z.DS = D + 1;
    z.inv_dp = 1.0f / static_cast<float>(z.DP);
    return z;
  }
  // LDS bytes of the scratch of M rows and the per-day terms (16-byte multiple).
  __host__ __device__ size_t scratch_bytes(int M) const {
    return sizeof(double) * 3 * static_cast<size_t>(M) * RD + sizeof(int) * 2 * static_cast<size_t>(M) * RI +
           sizeof(double) * 2 * DP;
  }
};

struct ChainLds {
  const float* act;
  int* hold;
  int* qty;
  float* env;
  const float* px;  // trading day closes, >= DP readable entries (those beyond D unused)
  const float* pn;  // new day closes [D]
  double* pro;
  double* deb;
  double* val;
  int* qd;
  int* kq;
  double* c1;   // [DP] per day: the one-share debit (p*1)*(1+c) of each stock
  double* rc1;  // [DP] per day: its reciprocal (an estimate's input)
  // Carves the scratch (16-byte aligned base) of M rows; returns the first byte after it.
  __host__ __device__ unsigned char* carve_scratch(unsigned char* base, const ChainShape& Z, int M) {
    pro = reinterpret_cast<double*>(base);
    deb = pro + M * Z.RD;
    val = deb + M * Z.RD;
    qd = reinterpret_cast<int*>(val + M * Z.RD);
    kq = qd + M * Z.RI;
    c1 = reinterpret_cast<double*>(kq + M * Z.RI);
    rc1 = c1 + Z.DP;
    return reinterpret_cast<unsigned char*>(rc1 + Z.DP);
  }
};

// Per-day terms (threads first, first + stride, ... over DP): c1[d] = (p_d*1)*(1+c) and
// rc1[d] ~ 1/c1[d], the hardware reciprocal refined by one Newton step -- only the input of an
// estimate; zero beyond D.
__device__ __forceinline__ void chain_day_terms(const ChainLds& L, const ChainShape& Z, int first, int stride,
                                                double one_p) {
#pragma clang fp contract(off)
  for (int d = first; d < Z.DP; d += stride) {
    double c = 0.0, r = 0.0;
    if (d < Z.D) {
      c = static_cast<double>(L.px[d]) * one_p;
      r = __builtin_amdgcn_rcp(c);
      r = fma(fma(-c, r, 1.0), r, r);
    }
    L.c1[d] = c;
    L.rc1[d] = r;
  }
}

// Phase A (all threads, pairs i = first, first + stride, ... over M*DP): orders, sells and the
// whole-order debit.  act(m, d, e) yields the action of env m, stock d (e = m*D + d).
template <class Act>
__device__ __forceinline__ void chain_pairs_a(const ChainLds& L, const ChainShape& Z, int M, int first,
                                              int stride, float hmax_f, double one_m, double one_p, Act act) {
#pragma clang fp contract(off)
#pragma unroll 4
  for (int i = first; i < M * Z.DP; i += stride) {
    const int m = div_small(i, Z.inv_dp);
    const int d = i - m * Z.DP;
    double pro = 0.0, deb = 0.0;
    int qd = 0;
    if (d < Z.D) {
      const int e = m * Z.D + d;
      const int q = order_from_action(act(m, d, e), hmax_f);
      const int h = L.hold[e];
      const int s = q < 0 ? min(h, -q) : 0;
      const double p = static_cast<double>(L.px[d]);
      L.hold[e] = h - s;
      L.qty[e] = -s;
      pro = (p * static_cast<double>(s)) * one_m;
      qd = q > 0 ? q : 0;
      deb = (p * static_cast<double>(qd)) * one_p;
    }
    L.pro[m * Z.RD + d] = pro;
    L.deb[m * Z.RD + d] = deb;
    L.qd[m * Z.RI + d] = qd;
  }
}
__device__ __forceinline__ void chain_pairs_a(const ChainLds& L, const ChainShape& Z, int M, int first,
                                              int stride, float hmax_f, double one_m, double one_p) {
  chain_pairs_a(L, Z, M, first, stride, hmax_f, one_m, one_p, [&](int, int, int e) { return L.act[e]; });
}

// The buy of one stock that does not fit whole: (p*q)*one_p > cash.  The answer is the largest k
// in [0, q-1] with (p*k)*one_p <= cash (a zero-share buy debits nothing; q <= 0 gives 0).  The
// debit is monotone in k.  The estimate k = floor(cash * rc1), rc1 ~ 1/((p*1)*one_p) (relative
// error below 2^-44), clamped to [0, max(q-1, 0)], is kept when the debits of k and k+1 bracket
// cash; otherwise unit steps from it reach the answer, whatever the estimate's error (for orders
// below 2^20 shares the estimate is at most one share off, so at most one step is taken).  k stays
// in float64 (an exact small integer) on the common path.
__device__ __forceinline__ int partial_fill(double cash, double p, double rc1, int q, double one_p,
                                           double& debit) {
#pragma clang fp contract(off)
  const double qm1 = static_cast<double>(q - 1);
  const double kd = fmax(fmin(floor(cash * rc1), qm1), 0.0);
  double dk = kd > 0.0 ? (p * kd) * one_p : 0.0;
  const double dk1 = (p * (kd + 1.0)) * one_p;
  int k = static_cast<int>(kd);
  if (!(dk <= cash) || (kd < qm1 && dk1 <= cash)) {
#pragma clang loop unroll(disable)
    while (k + 1 < q && (p * static_cast<double>(k + 1)) * one_p <= cash) ++k;
#pragma clang loop unroll(disable)
    while (k > 0 && !((p * static_cast<double>(k)) * one_p <= cash)) --k;
    dk = k > 0 ? (p * static_cast<double>(k)) * one_p : 0.0;
  }
  debit = dk;
  return k;
}

// CH (a multiple of 4) float64 / int / float entries from a 16-byte-aligned LDS address.
template <int CH>
__device__ __forceinline__ void lds_vec(double (&v)[CH], const double* src) {
#pragma unroll
  for (int j = 0; j < CH / 2; ++j) {
    const double2 t = reinterpret_cast<const double2*>(src)[j];
    v[2 * j] = t.x;
    v[2 * j + 1] = t.y;
  }
}
template <int CH>
__device__ __forceinline__ void lds_vec(int (&v)[CH], const int* src) {
#pragma unroll
  for (int j = 0; j < CH / 4; ++j) {
    const int4 t = reinterpret_cast<const int4*>(src)[j];
    v[4 * j] = t.x;
    v[4 * j + 1] = t.y;
    v[4 * j + 2] = t.z;
    v[4 * j + 3] = t.w;
  }
}
template <int CH>
__device__ __forceinline__ void lds_vec(float (&v)[CH], const float* src) {
#pragma unroll
  for (int j = 0; j < CH / 4; ++j) {
    const float4 t = reinterpret_cast<const float4*>(src)[j];
    v[4 * j] = t.x;
    v[4 * j + 1] = t.y;
    v[4 * j + 2] = t.z;
    v[4 * j + 3] = t.w;
  }
}

// acc + v[0] + ... + v[DP-1] in index order, the terms read CH at a time one chunk ahead.
template <int CH = kChunk>
__device__ __forceinline__ double chain_sum(double acc, const double* __restrict__ v, int DP) {
#pragma clang fp contract(off)
  double cur[CH];
  lds_vec<CH>(cur, v);
  for (int d0 = 0; d0 < DP; d0 += CH) {
    double nxt[CH];
    lds_vec<CH>(nxt, v + (d0 + CH < DP ? d0 + CH : d0));
#pragma unroll
    for (int j = 0; j < CH; ++j) acc = acc + cur[j];
#pragma unroll
    for (int j = 0; j < CH; ++j) cur[j] = nxt[j];
  }
  return acc;
}

template <int CH>
struct BuyChunk {
  double deb[CH], c1[CH], rc1[CH];
  int q[CH];
  float p[CH];
  __device__ __forceinline__ void load(const double* deb_, const double* c1_, const double* rc1_, const int* q_,
                                       const float* p_) {
    lds_vec<CH>(deb, deb_);
    lds_vec<CH>(c1, c1_);
    lds_vec<CH>(rc1, rc1_);
    lds_vec<CH>(q, q_);
    lds_vec<CH>(p, p_);
  }
};

// Phase B (lane m of the owner group): the cash recurrence of environment m -- all sells, then
// all buys, in ascending stock order.  A buy fills whole when its debit fits the cash and not at
// all when one share does not (selects); otherwise the partial fill decides (the one divergent
// branch).  c1s, rc1s: the day's one-share debits and their reciprocals (shared by all
// environments).  CH stocks per register chunk (DP is a multiple of CH).  With PF the next
// chunk's terms are read while the current one is consumed; without, after it (fewer registers).
template <int CH = kChunk, bool PF = true>
__device__ __forceinline__ void chain_serial(double& cash, const double* __restrict__ pro,
                                             const double* __restrict__ deb, const double* __restrict__ c1s,
                                             const double* __restrict__ rc1s, const int* __restrict__ qd,
                                             const float* __restrict__ px, int* __restrict__ kq, int DP,
                                             double one_p) {
#pragma clang fp contract(off)
  static_assert(CH % 4 == 0 && kChunk % CH == 0, "chunks of 4 or 8 stocks");
  cash = chain_sum<CH>(cash, pro, DP);
  BuyChunk<CH> cur;
  cur.load(deb, c1s, rc1s, qd, px);
  for (int d0 = 0; d0 < DP; d0 += CH) {
    BuyChunk<CH> nxt;
    const int dn = d0 + CH < DP ? d0 + CH : d0;
    if constexpr (PF) nxt.load(deb + dn, c1s + dn, rc1s + dn, qd + dn, px + dn);
    int k[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const bool fits = cur.deb[j] <= cash;
      int kj = fits ? cur.q[j] : 0;
      double debit = fits ? cur.deb[j] : 0.0;
      if (!fits && cur.c1[j] <= cash)
        kj = partial_fill(cash, static_cast<double>(cur.p[j]), cur.rc1[j], cur.q[j], one_p, debit);
      cash = cash - debit;
      k[j] = kj;
    }
#pragma unroll
    for (int j = 0; j < CH / 4; ++j)
      reinterpret_cast<int4*>(kq + d0)[j] = int4{k[4 * j], k[4 * j + 1], k[4 * j + 2], k[4 * j + 3]};
    if constexpr (PF)
      cur = nxt;
    else
      cur.load(deb + dn, c1s + dn, rc1s + dn, qd + dn, px + dn);
  }
}

// Phase C (all threads, pairs over M*DP): apply the buys, the holdings entries of the state
// rows (also passed to entry(m, d, value)), and the new day's position values p'_d h_d (zero
// beyond D).
template <class Entry>
__device__ __forceinline__ void chain_pairs_c(const ChainLds& L, const ChainShape& Z, int M, int first,
                                              int stride, float hold_scale, Entry entry) {
#pragma clang fp contract(off)
#pragma unroll 4
  for (int i = first; i < M * Z.DP; i += stride) {
    const int m = div_small(i, Z.inv_dp);
    const int d = i - m * Z.DP;
    double v = 0.0;
    if (d < Z.D) {
      const int e = m * Z.D + d;
      const int k = L.kq[m * Z.RI + d];
      const int h = L.hold[e] + k;
      L.hold[e] = h;
      L.qty[e] += k;
      const float he = static_cast<float>(h) * hold_scale;
      L.env[m * Z.DS + 1 + d] = he;
      entry(m, d, he);
      v = static_cast<double>(L.pn[d]) * static_cast<double>(h);
    }
    L.val[m * Z.RD + d] = v;
  }
}
__device__ __forceinline__ void chain_pairs_c(const ChainLds& L, const ChainShape& Z, int M, int first,
                                              int stride, float hold_scale) {
  chain_pairs_c(L, Z, M, first, stride, hold_scale, [](int, int, float) {});
}

// Phase D (lane m): v = cash + sum_d p'_d h_d in ascending stock order.
template <int CH = kChunk>
__device__ __forceinline__ double chain_value(double cash, const double* __restrict__ val, int DP) {
  return chain_sum<CH>(cash, val, DP);
}

// Holdings entries and position values without trading (reset / observe): all threads.
__device__ __forceinline__ void chain_pairs_hold(const ChainLds& L, const ChainShape& Z, int M, int first,
                                                 int stride, float hold_scale) {
#pragma clang fp contract(off)
  for (int i = first; i < M * Z.DP; i += stride) {
    const int m = div_small(i, Z.inv_dp);
    const int d = i - m * Z.DP;
    double v = 0.0;
    if (d < Z.D) {
      const int h = L.hold[m * Z.D + d];
      L.env[m * Z.DS + 1 + d] = static_cast<float>(h) * hold_scale;
      v = static_cast<double>(L.pn[d]) * static_cast<double>(h);
    }
    L.val[m * Z.RD + d] = v;
  }
}

// The state rows s_{t+1} = [cash, new closes, holdings, new indicators] of M environments from
// LDS into dst[m][0..S) (row stride S), with one wavefront: lane f writes entry f (f, f+64, ...) of
// every row, so each store instruction covers 64 consecutive entries.  env[m][0..D]: cash entry,
// holdings entries (row stride DS); in: [close[t] (D) | close[t+1] (D) | ind[t+1] (I*D)].  Rows go
// in batches of 8: all eight LDS reads are issued before the first store, so the LDS latency is
// paid once per batch rather than once per entry.
__device__ __forceinline__ void store_state_rows(float* dst, int M, int S, int D, const float* env, int DS,
                                                 const float* in, float price_scale, int lane) {
  constexpr int B = 8;
  for (int f = lane; f < S; f += 64) {
    const float* src;
    int stride = 0;
    float scale = 1.0f;
    if (f == 0) {
      src = env;
      stride = DS;
    } else if (f <= D) {
      src = in + D + (f - 1);
      scale = price_scale;
    } else if (f <= 2 * D) {
      src = env + (f - D);
      stride = DS;
    } else {
      src = in + (f - 1);  // ind[t+1][f-1-2D]
    }
    float* o = dst + f;
    for (int m0 = 0; m0 < M; m0 += B) {
      float v[B];
#pragma unroll
      for (int j = 0; j < B; ++j) v[j] = src[min(m0 + j, M - 1) * stride];  // rows past M: row M-1
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (m0 + j < M) o[static_cast<size_t>(m0 + j) * S] = v[j] * scale;
    }
  }
}

// Synchronisation of one wavefront's LDS traffic between the phases (no hardware barrier:
// a wavefront's LDS operations complete in order; this stops the compiler reordering them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace fm
