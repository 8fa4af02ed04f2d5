// The trading chain of Section 3.1 run by a 16-lane row of a wavefront: lane j of the row owns
// stocks j and j + 16 (at most 32 stocks); the serial cash recurrences (the sells' proceeds, the
// buys, the value) run on terms broadcast along the row by DPP row broadcasts, in stock order, so
// every lane of the row holds the same cash.  Used by the resident fused rollout and by the row
// variant of the environment step.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "device_common.h"

namespace fm {

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

// acc - v(lane 0) - v(lane 1) - ... - v(lane 15) of the row, in lane order.
template <int... L>
__device__ __forceinline__ double row_sub_impl(double acc, double v, std::integer_sequence<int, L...>) {
#pragma clang fp contract(off)
  ((acc = acc - row_bcast<L>(v)), ...);
  return acc;
}

// The buys of the wavefront's two environments (Section 3.1, readings 5-7).
// If every row's cash covers the sum of its whole orders with a margin far above the rounding of
// 32 subtractions, every whole order fits in sequence: the debits are subtracted in stock order
// and every order fills.  Otherwise the buys run as a sequence of events, both rows in step: with
// cash C, the next stock (in ascending order) that can change anything is the first one with a
// buy order whose one-share debit fits C -- the stocks before it fill nothing and leave C as it
// is.  A ballot per stock slot finds each row's next event; the lane owning that stock fills it
// (the whole order if its debit fits C, else the partial fill) and keeps the fill, and its debit
// reaches the rest of the row by a lane permute.
__device__ __forceinline__ void buy_all(double& cash, int (&kown)[2], int lane, const BuySet (&B)[2], double one_p) {
#pragma clang fp contract(off)
  const int jl = lane & 15, rl = (lane >> 4) & 1, rbase = lane & 48;
  const double total = row_sum(0.0, B[0].deb + B[1].deb);  // any order: only a bound
  if (__builtin_amdgcn_ballot_w64(!(cash >= total * (1.0 + 0x1p-40))) == 0) {
    cash = row_sub_impl(cash, B[0].deb, std::make_integer_sequence<int, 16>());
    cash = row_sub_impl(cash, B[1].deb, std::make_integer_sequence<int, 16>());
    kown[0] = pq_order(B[0].pq);
    kown[1] = pq_order(B[1].pq);
    return;
  }
  const bool buy0 = pq_order(B[0].pq) > 0, buy1 = pq_order(B[1].pq) > 0;
  int dn = 0;  // the row's next stock to consider
  for (int it = 0; it < 32; ++it) {
    const unsigned long long b0 = __builtin_amdgcn_ballot_w64(buy0 && B[0].c1 <= cash && jl >= dn);
    const unsigned long long b1 = __builtin_amdgcn_ballot_w64(buy1 && B[1].c1 <= cash && jl + 16 >= dn);
    const unsigned m0 = static_cast<unsigned>(b0 & 0xffffu) | (static_cast<unsigned>(b1 & 0xffffu) << 16);
    const unsigned m1 = static_cast<unsigned>((b0 >> 16) & 0xffffu) | (static_cast<unsigned>((b1 >> 16) & 0xffffu) << 16);
    if ((m0 | m1) == 0) break;
    const unsigned mine = rl == 0 ? m0 : m1;
    const int e = mine != 0 ? __builtin_ctz(mine) : 64;  // the row's event stock (64: none)
    const bool hi = e >= 16;
    const bool owner = (e & 15) == jl && e < 32;
    // The owner's fill of stock e: whole, or partial when only part of the order fits.
    const double deb = hi ? B[1].deb : B[0].deb;
    const long pq = hi ? B[1].pq : B[0].pq;
    const bool fits = deb <= cash;
    int k = fits ? pq_order(pq) : 0;
    double debit = fits ? deb : 0.0;
    if (owner && !fits) {
      const double c1 = hi ? B[1].c1 : B[0].c1;
      bool ok = true;
      k = partial_fill_sel(cash, static_cast<double>(pq_price(pq)), c1, pq_order(pq), one_p, debit, ok);
      if (!ok) {
        double rc1 = __builtin_amdgcn_rcp(c1);
        rc1 = fma(fma(-c1, rc1, 1.0), rc1, rc1);
        k = partial_fill(cash, static_cast<double>(pq_price(pq)), rc1, pq_order(pq), one_p, debit);
      }
    }
    if (owner) kown[hi ? 1 : 0] = k;
    const int src = rbase + (e & 15);
    const long dbits = __builtin_bit_cast(long, debit);
    const int lo = __builtin_amdgcn_ds_bpermute(4 * src, static_cast<int>(dbits));
    const int hb = __builtin_amdgcn_ds_bpermute(4 * src, static_cast<int>(dbits >> 32));
    const double d_e = __builtin_bit_cast(
        double, static_cast<long>((static_cast<unsigned long>(static_cast<unsigned>(hb)) << 32) | static_cast<unsigned>(lo)));
    if (e < 32) {
      cash = cash - d_e;
      dn = e + 1;
    }
  }
}

// The row's cash before each lane's stock under the serial recurrence P(j + 1) = P(j) - x(j),
// P(0) = start, x(j) held by lane j: carried along the row one lane per round by DPP row shifts
// (lane 0 has no source and keeps start), so lane j's value is the exact serial result of j
// subtractions in lane order.  total receives P(16).
__device__ __forceinline__ double row_shr1(double keep, double v) {
  return __builtin_amdgcn_update_dpp(keep, v, 0x111, 0xf, 0xf, false);
}
__device__ __forceinline__ double row_prefix(double start, double x, double& total) {
#pragma clang fp contract(off)
  double t = start;
#pragma unroll
  for (int r = 0; r < 15; ++r) t = row_shr1(t, t - x);
  total = row_bcast<15>(t - x);
  return t;
}

// The buys of the wavefront's two environments (Section 3.1, readings 5-7), by segments.
// Fast path as in buy_all.  Otherwise, with cash C at the start of a segment, the candidates are
// the stocks from dn on with a buy order whose one-share debit fits C (the others cannot buy: the
// cash only falls during the buys).  Every candidate is assumed to fill its whole order; the row
// prefix of their debits gives the cash each one meets, exactly as the serial recurrence would,
// up to the first candidate e whose whole order does not fit that cash.  The candidates before e
// fill whole; e buys what its cash allows (a partial fill, or nothing when one share does not
// fit); the next segment starts after e.  A segment therefore covers a run of whole fills at the
// cost of one prefix, where buy_all spends one event per stock.
__device__ __forceinline__ void buy_all_seg(double& cash, int (&kown)[2], int lane, const BuySet (&B)[2],
                                            double one_p) {
#pragma clang fp contract(off)
  const int jl = lane & 15, rl = (lane >> 4) & 1, rbase = lane & 48;
  const double total = row_sum(0.0, B[0].deb + B[1].deb);  // any order: only a bound
  if (__builtin_amdgcn_ballot_w64(!(cash >= total * (1.0 + 0x1p-40))) == 0) {
    cash = row_sub_impl(cash, B[0].deb, std::make_integer_sequence<int, 16>());
    cash = row_sub_impl(cash, B[1].deb, std::make_integer_sequence<int, 16>());
    kown[0] = pq_order(B[0].pq);
    kown[1] = pq_order(B[1].pq);
    return;
  }
  const int q0 = pq_order(B[0].pq), q1 = pq_order(B[1].pq);
  const int rsh = lane & 48;  // this lane's row's bits in a ballot
  int dn = 0;  // the row's next stock to consider
  for (int it = 0; it <= 32; ++it) {
    const bool c0 = q0 > 0 && B[0].c1 <= cash && jl >= dn;
    const bool c1 = q1 > 0 && B[1].c1 <= cash && jl + 16 >= dn;
    const unsigned long long b0 = __builtin_amdgcn_ballot_w64(c0);
    if ((b0 | __builtin_amdgcn_ballot_w64(c1)) == 0) break;
    // A prefix is formed only where some row needs it: stocks 0-15 when a row has candidates
    // there; stocks 16-31 when a row without a failure among stocks 0-15 has candidates there.
    double mid = cash, end, p0 = cash, p1;
    if (b0 != 0) p0 = row_prefix(cash, c0 ? B[0].deb : 0.0, mid);
    const unsigned long long f0 = __builtin_amdgcn_ballot_w64(c0 && !(B[0].deb <= p0));
    const bool own_f0 = ((f0 >> rsh) & 0xffffu) != 0;
    unsigned long long f1 = 0;
    end = mid;
    p1 = mid;
    if (__builtin_amdgcn_ballot_w64(c1 && !own_f0) != 0) {
      p1 = row_prefix(mid, c1 ? B[1].deb : 0.0, end);
      f1 = __builtin_amdgcn_ballot_w64(c1 && !(B[1].deb <= p1));
    }
    const unsigned m0 = static_cast<unsigned>(f0 & 0xffffu) | (static_cast<unsigned>(f1 & 0xffffu) << 16);
    const unsigned m1 = static_cast<unsigned>((f0 >> 16) & 0xffffu) | (static_cast<unsigned>((f1 >> 16) & 0xffffu) << 16);
    const unsigned mine = rl == 0 ? m0 : m1;
    const int e = mine != 0 ? __builtin_ctz(mine) : 32;  // the row's first failure (32: none)
    if (c0 && jl < e) kown[0] = q0;
    if (c1 && jl + 16 < e) kown[1] = q1;
    if ((f0 | f1) == 0) {  // every row filled all its candidates whole
      cash = end;
      break;
    }
    const bool hi = e >= 16;
    const bool owner = e < 32 && (e & 15) == jl;
    double nc = end;  // a row without a failure: all its candidates filled
    if (owner) {
      const double pe = hi ? p1 : p0, c1e = hi ? B[1].c1 : B[0].c1;
      const long pq = hi ? B[1].pq : B[0].pq;
      int k = 0;
      double debit = 0.0;
      if (c1e <= pe) {
        bool ok = true;
        k = partial_fill_sel(pe, static_cast<double>(pq_price(pq)), c1e, pq_order(pq), one_p, debit, ok);
        if (!ok) {
          double rc1 = __builtin_amdgcn_rcp(c1e);
          rc1 = fma(fma(-c1e, rc1, 1.0), rc1, rc1);
          k = partial_fill(pe, static_cast<double>(pq_price(pq)), rc1, pq_order(pq), one_p, debit);
        }
      }
      kown[hi ? 1 : 0] = k;
      nc = pe - debit;
    }
    const int src = e < 32 ? rbase + (e & 15) : lane;
    const long nbits = __builtin_bit_cast(long, nc);
    const int lo = __builtin_amdgcn_ds_bpermute(4 * src, static_cast<int>(nbits));
    const int hb = __builtin_amdgcn_ds_bpermute(4 * src, static_cast<int>(nbits >> 32));
    cash = __builtin_bit_cast(
        double, static_cast<long>((static_cast<unsigned long>(static_cast<unsigned>(hb)) << 32) | static_cast<unsigned>(lo)));
    dn = e < 32 ? e + 1 : 32;
  }
}

}  // namespace fm
