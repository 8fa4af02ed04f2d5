// The environment step with one lane per environment, for up to 32 stocks (Section 3.1's
// market step; Sections 4.2-4.3: the vectorised environments on the GPU).
//
// Each lane holds its environment's whole trading state in registers (cash, total asset and
// cumulative reward in float64, the holdings as int32) and runs the step's serial chain --
// orders, the sells, the buys against the cash, the new holdings, the position values and the
// reward -- without any cross-lane traffic: the 64 lanes of a wavefront advance 64 chains at
// once, so the serial recurrence costs one instruction stream per wavefront rather than one per
// environment.  A wavefront owns M consecutive environments; it needs no workgroup barrier, so
// the four wavefronts of a workgroup run free of each other.
//
// Per step a wavefront
//   1. waits for the step's inputs, requested one step ahead straight from HBM into its LDS
//      area (buffer loads with an LDS destination: the market rows and, driven, the tile of
//      actions, 64 consecutive floats per instruction), and spreads the actions into
//      per-environment rows;
//   2. requests the next step's inputs;
//   3. runs the chains: lane m reads its action row and the day's prices from LDS;
//   4. writes the state rows' cash and holdings entries and the executed quantities to LDS;
//   5. stores the tile's state rows, quantities and rewards as wave-wide runs of addresses.
// HBM sees each trajectory byte once: the actions are read and the states, quantities and
// rewards written, nothing else (the per-environment state stays in registers across steps).
#include "device_common.h"
#include "launch.h"
#include "row_chain.h"

namespace fm {

namespace {

constexpr int kWaves = 4;       // wavefronts per workgroup
constexpr int kRow = 33;        // LDS stride of the per-environment rows: lane m's reads of its
                                // own row fall in distinct banks
constexpr int kMaxMkt = 256;    // market floats staged per step, (2 + I) * D
constexpr int kMaxEnvs = 64;    // environments per wavefront
constexpr int kColGroups = kMaxMkt / 64;             // 64-column groups of a state row (S <= 256)
constexpr int kNoStore = 1 << 30;                     // a byte offset beyond any store range

enum LaneMode { kDriven = 0, kMeans = 1 };

struct LaneArgs {
  int t0, n_steps, M;
  const float* act;   // kDriven: [n_steps][N][D]
  const float* mu;    // kMeans: [K][N][D] actor means
  const float* mix;   // kMeans: [K] weights w_k (device)
  int K;
  float sigma;
  uint64_t noise_key;
  int64_t env_offset;
  float* obs;         // [n_steps][N][S] or null
  float* act_out;     // kMeans: [N][D] or null
  double* rew;        // [n_steps][N] or null
  int* qty;           // [n_steps][N][D] or null
  int stage;          // LDS floats of a wavefront's staging area
  int mu_slot;        // kMeans: staging floats per actor when the means go through LDS, else 0
};

constexpr int kMktClose = 64;   // LDS floats per buffer of close[t] | close[t+1] (2D <= 64)
constexpr int kMktInd = 256;    // LDS floats per buffer of ind[t+1] (I*D < 256)
constexpr int kWaitVm0 = 0x0F70;    // s_waitcnt vmcnt(0)
constexpr int kWaitLgkm0 = 0xC07F;  // s_waitcnt lgkmcnt(0)

constexpr int kMuStage = 4096;      // LDS floats per wavefront for the actor means' tiles

// LDS floats of a tile of M environments of D stocks fetched 64 floats per instruction, and of a
// wavefront's whole area with a staging area of `stage` floats.
__host__ __device__ inline int stage_floats(int M, int D) { return (M * D + 63) / 64 * 64; }
__host__ __device__ inline int wave_floats(int M, int stage) {
  return 2 * kMktClose + 2 * kMktInd + stage + 2 * (M + 1) * kRow;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t range_rsrc(const float* base, int n_floats) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, 4 * n_floats, 0x00020000);
}
// Beyond the resource's range a load returns 0.
__device__ __forceinline__ float range_load(__amdgpu_buffer_rsrc_t r, int i) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, 4 * i, 0, 0));
}

// The day's trading chain of one environment (Section 3.1) over its lane's LDS rows: row holds
// the actions on entry and the executed quantities on exit (signed orders in between), ent
// receives the state row's cash and holdings entries.  The pointers are restrict-qualified (the
// rows, the prices and the entries never overlap), so the compiler may issue the LDS reads
// ahead of the writes.  Returns the new value v' = cash + sum_d p'_d h_d.
template <int DP>
__device__ __forceinline__ double lane_chain(double& cash, int (&hold)[DP], float* __restrict__ row,
                                             float* __restrict__ ent, const float* __restrict__ px,
                                             const float* __restrict__ pn, int D, const EnvConst& C) {
#pragma clang fp contract(off)
  const double one_p = C.one_p;
  // Orders and all sells in ascending stock order.
  float a[DP];
#pragma unroll
  for (int d = 0; d < DP; ++d) a[d] = row[d];
#pragma unroll
  for (int d = 0; d < DP; ++d) {
    const int q = order_from_action(a[d], C.hmax_f);
    const int s = q < 0 ? min(hold[d], -q) : 0;
    hold[d] -= s;
    row[d] = __int_as_float(q < 0 ? -s : q);
    cash = cash + (static_cast<double>(px[d]) * static_cast<double>(s)) * C.one_m;
  }
  // All buys in ascending order, each whole when its debit fits the cash, else the largest
  // affordable part: one loop body for every stock (the partial fill is long and rarely taken),
  // the next stock's order and price read one iteration ahead (entry D of a row and of the
  // prices exists).
  int od = __float_as_int(row[0]);
  float pf = px[0];
#pragma clang loop unroll(disable)
  for (int d = 0; d < D; ++d) {
    const int od_next = __float_as_int(row[d + 1]);
    const float pf_next = px[d + 1];
    const int qd = od > 0 ? od : 0;
    const double p = static_cast<double>(pf);
    const double deb = (p * static_cast<double>(qd)) * one_p;
    const bool fits = deb <= cash;
    int k = fits ? qd : 0;
    double debit = fits ? deb : 0.0;
    if (!fits) {
      const double c1 = p * one_p;
      if (c1 <= cash) {
        double rc = __builtin_amdgcn_rcp(c1);
        rc = fma(fma(-c1, rc, 1.0), rc, rc);
        k = partial_fill(cash, p, rc, qd, one_p, debit);
      }
    }
    cash = cash - debit;
    if (qd > 0) row[d] = __int_as_float(k);
    od = od_next;
    pf = pf_next;
  }
  // Holdings, the state row's entries and the value in ascending stock order.
  double v = cash;
#pragma unroll
  for (int d = 0; d < DP; ++d) {
    const int e = __float_as_int(row[d]);
    hold[d] += e > 0 ? e : 0;
    v = v + static_cast<double>(pn[d]) * static_cast<double>(hold[d]);
    ent[1 + d] = static_cast<float>(hold[d]) * C.hold_scale;
  }
  ent[0] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
  return v;
}

// DP: stocks per chain in registers (D <= DP); the entries d >= D carry a zero action, hence a
// zero order, a zero sale and debit and a zero position value, and leave the cash and the value
// unchanged bit for bit (adding +0.0 to a non-negative float64).
template <int MODE, int DP>
__global__ __launch_bounds__(kWaves * 64) void env_lane_kernel(EnvConst C, EnvState st, LaneArgs A) {
  extern __shared__ __align__(16) float lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int MM = A.M;
  const int n0 = (blockIdx.x * kWaves + wave) * MM;
  if (n0 >= C.N) return;  // the whole wavefront; no barrier follows
  const int N = C.N, D = C.D, S = C.S, ID = C.I * D;
  const int M = min(MM, N - n0);
  const int MD = M * D;
  const float inv_d = 1.0f / static_cast<float>(D);
  float* mcl = lds + wave * wave_floats(MM, A.stage);  // [2][64]: close[t] | close[t+1], zero from 2D
  float* mind = mcl + 2 * kMktClose;                   // [2][256]: ind[t+1]
  float* stage = mind + 2 * kMktInd;  // the driven tile, or the K actors' mean tiles, as fetched
  // Rows of kRow floats, M + 1 of each (idle lanes work on the spare last row):
  float* tile = stage + A.stage;  // actions / actor means, then orders, then quantities
  float* ent = tile + (MM + 1) * kRow;        // noise, then the state rows' cash and holdings entries
  const bool active = lane < M;
  const int n = n0 + lane;

  // The holdings through a buffer resource over [D][N]: rows d >= D read 0 and are not stored.
  const __amdgpu_buffer_rsrc_t hr = range_rsrc(reinterpret_cast<const float*>(st.hold), D * N);
  double cash = 0.0, asset = 0.0, cumrew = 0.0;
  int hold[DP];
#pragma unroll
  for (int d = 0; d < DP; ++d) hold[d] = active ? __float_as_int(range_load(hr, d * N + n)) : 0;
  if (active) {
    cash = st.cash[n];
    asset = st.asset[n];
    cumrew = st.cumrew[n];
  }
  // Entries d >= D of the LDS rows stay zero: they are written only with the zero actions,
  // orders and quantities of those stocks.
  for (int i = lane; i < 2 * (MM + 1) * kRow; i += 64) tile[i] = 0.0f;

  // Inside the step loop the lane index L is re-derived each step through an opaque copy, so
  // the per-lane addresses and masks are recomputed rather than held in registers.
  int L = lane;
  // Step it's inputs go from HBM straight into LDS buffer it & 1 (the market rows; lanes past
  // the ranges write zeros) and, driven, into the staging area (64 floats per instruction,
  // consecutive lanes on consecutive floats of the tile's contiguous block).
  auto fetch = [&](int it) {
    const int t = A.t0 + it, b = it & 1;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(range_rsrc(C.close + static_cast<size_t>(t) * D, 2 * D),
                                             mcl + b * kMktClose, 4, 4 * L, 0, 0, 0);
    const __amdgpu_buffer_rsrc_t ri = range_rsrc(C.ind + static_cast<size_t>(t + 1) * ID, ID);
    for (int j = 0; 64 * j < ID; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ri, mind + b * kMktInd + 64 * j, 4, 4 * (L + 64 * j), 0, 0, 0);
    if (MODE == kDriven) {
      const __amdgpu_buffer_rsrc_t ra = range_rsrc(A.act + (static_cast<size_t>(it) * N + n0) * D, MD);
      for (int j = 0; 64 * j < MD; ++j)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, stage + 64 * j, 4, 4 * (L + 64 * j), 0, 0, 0);
    } else if (A.mu_slot > 0) {
      for (int k = 0; k < A.K; ++k) {
        const __amdgpu_buffer_rsrc_t rk = range_rsrc(A.mu + (static_cast<size_t>(k) * N + n0) * D, MD);
        for (int j = 0; 64 * j < MD; ++j)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rk, stage + k * A.mu_slot + 64 * j, 4, 4 * (L + 64 * j), 0, 0, 0);
      }
    }
  };
  // Tile float i = m * D + d goes to row m, entry d.
  auto tile_put = [&](const float (&v)[DP]) {
    int md = MD;
    __asm__ volatile("" : "+s"(md));
#pragma unroll
    for (int j = 0; j < DP; ++j) {
      const int i = L + 64 * j;
      if (64 * j < md && i < md) {
        const int m = div_small(i, inv_d);
        tile[m * kRow + (i - m * D)] = v[j];
      }
    }
  };
  auto tile_get = [&](int i) {
    const int m = div_small(i, inv_d);
    return tile[m * kRow + (i - m * D)];
  };
  // The fetched tile at src (float i = m * D + d) into the rows.
  auto tile_from = [&](const float* src) {
    for (int i = L; i < MD; i += 64) {
      const int m = div_small(i, inv_d);
      tile[m * kRow + (i - m * D)] = src[i];
    }
  };

  fetch(0);
  for (int it = 0; it < A.n_steps; ++it) {
#pragma clang fp contract(off)
    const int t = A.t0 + it, b = it & 1;
    const size_t row0 = static_cast<size_t>(it) * N + n0;
    L = lane;
    __asm__ volatile("" : "+v"(L));
    const int LR = L < M ? L : MM;
    const float* px = mcl + b * kMktClose;  // close[t][d]; entries from D on are finite
    const float* pn = px + D;               // close[t+1][d]; entries from D on are finite
    const float* ind = mind + b * kMktInd;
    if (MODE == kMeans) {
      // The noise (Section 5.2.1) while the inputs are in flight: one Philox block per
      // (environment, group of four stocks), spread over the lanes; the noise rows' entries
      // from D on are zero.
      const int G = (D + 3) >> 2;
      for (int i = L; i < M * 8; i += 64) {
        const int m = i >> 3;
        const int g = i & 7;
        float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (g < G && A.sigma != 0.0f)
          noise_block(A.noise_key, static_cast<uint64_t>(A.env_offset + n0 + m), static_cast<uint64_t>(t),
                      static_cast<uint64_t>(g), z);
#pragma unroll
        for (int r = 0; r < 4; ++r) ent[m * kRow + 4 * g + r] = 4 * g + r < D ? z[r] : 0.0f;
      }
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm0);  // step it's inputs have landed in LDS
    if (MODE == kDriven) tile_from(stage);
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);  // the staging area is read before it is refilled
    if (it + 1 < A.n_steps) fetch(it + 1);
    wave_lds_sync();

    // Actions (Section 5.2.1 for the ensemble's: a = clip(sum_k w_k mu_k + sigma eps)) in the
    // lanes' tile rows.
    if (MODE == kMeans) {
      float acc[DP];
#pragma unroll
      for (int d = 0; d < DP; ++d) acc[d] = 0.0f;
      for (int k = 0; k < A.K; ++k) {
        const float w = A.mix[k];
        if (A.mu_slot > 0) {
          wave_lds_sync();  // the previous actor's rows have been read
          tile_from(stage + k * A.mu_slot);
        } else {
          const __amdgpu_buffer_rsrc_t r = range_rsrc(A.mu + (static_cast<size_t>(k) * N + n0) * D, MD);
          int md = MD;
          __asm__ volatile("" : "+s"(md));
          float v[DP];
#pragma unroll
          for (int j = 0; j < DP; ++j) v[j] = 64 * j < md ? range_load(r, L + 64 * j) : 0.0f;
          wave_lds_sync();  // the previous actor's rows have been read
          tile_put(v);
        }
        wave_lds_sync();
#pragma unroll
        for (int d = 0; d < DP; ++d) acc[d] = acc[d] + w * tile[LR * kRow + d];
      }
      wave_lds_sync();
#pragma unroll
      for (int d = 0; d < DP; ++d) {
        float x = acc[d];
        if (A.sigma != 0.0f) x = acc[d] + A.sigma * ent[LR * kRow + d];
        tile[LR * kRow + d] = fminf(fmaxf(x, -1.0f), 1.0f);
      }
      wave_lds_sync();
      if (A.act_out) wave_store_row(A.act_out + static_cast<size_t>(n0) * D, MD, L, tile_get);
    }

    // The chain (Section 3.1); the lane's tile row turns from actions into executed quantities.
    const double v = lane_chain<DP>(cash, hold, tile + LR * kRow, ent + LR * kRow, px, pn, D, C);
    const double r = (v - asset) * C.reward_scale;
    cumrew = cumrew + r;
    asset = v;
    if (A.rew && L < M) A.rew[row0 + L] = r;

    // The tile's stores.
    wave_lds_sync();
    if (A.qty)
      wave_store_row(A.qty + row0 * D, MD, L, [&](int i) { return __float_as_int(tile_get(i)); });
    if (A.obs) {
      // The state rows [cash, close[t+1] (D), holdings (D), ind[t+1] (I*D)]: lane column
      // f = L + 64 g of row m is read from LDS at src + m * stride -- the environment's entries
      // row for the cash and holdings columns, a market row (stride 0) otherwise -- scaled, and
      // stored at byte 4 f of the row; columns past S store nowhere (an offset beyond every
      // range of at most 64 rows).  Four rows per batch: every read is issued before the first
      // store; rows past M read row M - 1 and store beyond the range.
      const __amdgpu_buffer_rsrc_t orow = range_rsrc(A.obs + row0 * S, M * S);
      // Per lane and column group: the LDS byte address of the column's value for row 0, a mask
      // that keeps the row's byte offset for the environment's own entries (zero for market
      // columns, shared by all rows), the scale, and the column's byte offset in a row.  The
      // row offsets are wave-uniform, so each value costs an and, two adds, a read, a multiply
      // and a store.
      int src[kColGroups], own[kColGroups], cb[kColGroups];
      float scale[kColGroups];
      const int ent_o = static_cast<int>(ent - mcl), pn_o = static_cast<int>(pn - mcl);
      const int ind_o = static_cast<int>(ind - mcl);
#pragma unroll
      for (int g = 0; g < kColGroups; ++g) {
        const int f = L + 64 * g;
        const bool o = f == 0 || (f > D && f <= 2 * D);
        src[g] = 4 * (o ? ent_o + (f == 0 ? 0 : f - D) : (f <= D ? pn_o + f - 1 : ind_o + min(f, S - 1) - 1 - 2 * D));
        own[g] = o ? -1 : 0;
        scale[g] = (f >= 1 && f <= D) ? C.price_scale : 1.0f;
        cb[g] = f < S ? 4 * f : kNoStore;
      }
      const char* lbase = reinterpret_cast<const char*>(mcl);
      for (int m0 = 0; m0 < M; m0 += 4) {
        float x[4][kColGroups];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ro = 4 * kRow * min(m0 + r, M - 1);  // rows past M read row M - 1
#pragma unroll
          for (int g = 0; g < kColGroups; ++g)
            x[r][g] = *reinterpret_cast<const float*>(lbase + src[g] + (own[g] & ro));
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int so = 4 * (m0 + r) * S;  // rows past M store beyond the range
#pragma unroll
          for (int g = 0; g < kColGroups; ++g)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[r][g] * scale[g]), orow, so + cb[g], 0, 0);
        }
      }
    }
    wave_lds_sync();  // the stores have read the LDS rows before the next step rewrites them
  }

  if (active) {
    st.cash[n] = cash;
    st.asset[n] = asset;
    st.cumrew[n] = cumrew;
#pragma unroll
    for (int d = 0; d < DP; ++d) __builtin_amdgcn_raw_buffer_store_b32(hold[d], hr, 4 * (d * N + n), 0, 0);
  }
}

template <int MODE, int DP>
hipError_t launch_dp(const EnvConst& C, const EnvState& st, const LaneArgs& A, hipStream_t stream) {
  const int waves = (C.N + A.M - 1) / A.M;
  const int grid = (waves + kWaves - 1) / kWaves;
  const size_t lds = sizeof(float) * kWaves * wave_floats(A.M, A.stage);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(env_lane_kernel<MODE, DP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((env_lane_kernel<MODE, DP>), dim3(grid), dim3(kWaves * 64), lds, stream, C, st, A);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Row variant (D <= 32): E = 1 or 2 environments per wavefront, one per 16-lane row (the other
// rows repeat them and store nothing), lane j of a row owning stocks j and j + 16.  The step's chain is the
// resident fused rollout's: the independent per-stock work spread over the row's lanes, the
// serial cash recurrences on terms broadcast along the row (row_chain.h).  At small batches this
// shortens a step: the 16 lanes of a row share an environment's instruction stream instead of
// one lane issuing all of it.
// ------------------------------------------------------------------------------------------
constexpr int kRowEnvs = 2;  // the most environments per wavefront

__host__ __device__ inline int row_wave_floats() { return 2 * kMktClose + 2 * kMktInd + 2 * (kRowEnvs + 1) * kRow; }

template <int MODE, int E>
__global__ __launch_bounds__(kWaves * 64) void env_row_kernel(EnvConst C, EnvState st, LaneArgs A) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) float lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n0 = (blockIdx.x * kWaves + wave) * E;
  if (n0 >= C.N) return;  // the whole wavefront; no barrier follows
  const int N = C.N, D = C.D, S = C.S, ID = C.I * D;
  const int M = min(E, N - n0);
  const int jl = lane & 15, m = (lane >> 4) & (E - 1);
  const bool lead = lane < 16 * E;  // the rows that store their environment's results
  const bool env_ok = m < M;
  const int n = n0 + (env_ok ? m : 0);  // an idle row repeats environment n0 and stores nothing
  float* mcl = lds + wave * row_wave_floats();  // [2][64]: close[t] | close[t+1], zero from 2D
  float* mind = mcl + 2 * kMktClose;            // [2][256]: ind[t+1]
  float* ent = mind + 2 * kMktInd;              // [2 + 1][kRow] the state rows' own entries
  float* zrow = ent + (kRowEnvs + 1) * kRow;    // [2 + 1][kRow] noise (ensemble mode)

  // The trading state: every lane of a row holds its environment's cash, value and cumulative
  // reward; lane j the holdings of stocks j and j + 16 (zero beyond D).
  double cash = st.cash[n], asset = st.asset[n], cumrew = st.cumrew[n];
  const __amdgpu_buffer_rsrc_t hr = range_rsrc(reinterpret_cast<const float*>(st.hold), D * N);
  int hold[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int d = jl + 16 * s;
    hold[s] = __float_as_int(range_load(hr, d < D ? d * N + n : D * N));
  }

  auto fetch = [&](int it) {
    const int t = A.t0 + it, b = it & 1;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(range_rsrc(C.close + static_cast<size_t>(t) * D, 2 * D),
                                             mcl + b * kMktClose, 4, 4 * lane, 0, 0, 0);
    const __amdgpu_buffer_rsrc_t ri = range_rsrc(C.ind + static_cast<size_t>(t + 1) * ID, ID);
    for (int j = 0; 64 * j < ID; ++j)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ri, mind + b * kMktInd + 64 * j, 4, 4 * (lane + 64 * j), 0, 0, 0);
  };
  // Per-lane element of the wavefront's [M][D] block (the resources below cover the whole block,
  // so their base stays wave-uniform); stocks beyond D index past the block and read zero.
  auto blk = [&](int s) { return jl + 16 * s < D ? m * D + jl + 16 * s : M * D; };
  // Driven: the row's actions of step it, one step ahead in registers (zero beyond D).
  float pa[2] = {0.0f, 0.0f};
  auto fetch_act = [&](int it) {
    const __amdgpu_buffer_rsrc_t ra = range_rsrc(A.act + (static_cast<size_t>(it) * N + n0) * D, M * D);
#pragma unroll
    for (int s = 0; s < 2; ++s) pa[s] = range_load(ra, blk(s));
  };

  fetch(0);
  if (MODE == kDriven) fetch_act(0);
  for (int it = 0; it < A.n_steps; ++it) {
    const int t = A.t0 + it, b = it & 1;
    const size_t row0 = static_cast<size_t>(it) * N + n0;
    const float* px = mcl + b * kMktClose;
    const float* ind = mind + b * kMktInd;
    float a[2];
    if (MODE == kDriven) {
      a[0] = pa[0];
      a[1] = pa[1];
      __builtin_amdgcn_s_waitcnt(kWaitVm0);  // step it's inputs have landed
      if (it + 1 < A.n_steps) {
        fetch(it + 1);
        fetch_act(it + 1);
      }
    } else {
      // Ensemble means, then the noise (Section 5.2.1): one Philox block per (environment, group
      // of four stocks), lanes 0..7 of rows 0 and 1, through LDS to the lanes owning the stocks.
      float acc[2] = {0.0f, 0.0f};
      float mu[8][2];
      const int K = min(A.K, 8);
      for (int k = 0; k < K; ++k) {
        const __amdgpu_buffer_rsrc_t rk = range_rsrc(A.mu + (static_cast<size_t>(k) * N + n0) * D, M * D);
        mu[k][0] = range_load(rk, blk(0));
        mu[k][1] = range_load(rk, blk(1));
      }
      if (A.sigma != 0.0f && lead && 4 * jl < D) {
        float z[4];
        noise_block(A.noise_key, static_cast<uint64_t>(A.env_offset + n), static_cast<uint64_t>(t),
                    static_cast<uint64_t>(jl), z);
#pragma unroll
        for (int r = 0; r < 4; ++r) zrow[m * kRow + 4 * jl + r] = z[r];
      }
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      for (int k = 0; k < K; ++k) {
        const float w = A.mix[k];
        acc[0] = acc[0] + w * mu[k][0];
        acc[1] = acc[1] + w * mu[k][1];
      }
      wave_lds_sync();
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int d = jl + 16 * s;
        float x = acc[s];
        if (A.sigma != 0.0f) x = acc[s] + A.sigma * zrow[m * kRow + min(d, kRow - 1)];
        a[s] = d < D ? fminf(fmaxf(x, -1.0f), 1.0f) : 0.0f;
        if (A.act_out && env_ok && lead && d < D)
          A.act_out[static_cast<size_t>(n) * D + d] = a[s];
      }
    }

    // The chain (Section 3.1): orders and sells, the sells' proceeds summed in stock order; the
    // buys in stock order (events); holdings, the position values and the value in stock order.
    int sold[2], q[2];
    BuySet B[2];
    double pro[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int d = jl + 16 * s;
      const float p = d < D ? px[d] : 0.0f;
      q[s] = d < D ? order_from_action(a[s], C.hmax_f) : 0;
      sold[s] = q[s] < 0 ? min(hold[s], -q[s]) : 0;
      hold[s] -= sold[s];
      const double pd = static_cast<double>(p);
      const int qd = q[s] > 0 ? q[s] : 0;
      pro[s] = (pd * static_cast<double>(sold[s])) * C.one_m;
      B[s].deb = (pd * static_cast<double>(qd)) * C.one_p;
      B[s].c1 = pd * C.one_p;
      B[s].pq = pack_pq(p, qd);
    }
    cash = row_sum(cash, pro[0]);
    cash = row_sum(cash, pro[1]);
    int kown[2] = {0, 0};
    buy_all_seg(cash, kown, lane, B, C.one_p);
    double val[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int d = jl + 16 * s;
      hold[s] += kown[s];
      const float pn = d < D ? px[D + d] : 0.0f;
      val[s] = static_cast<double>(pn) * static_cast<double>(hold[s]);
    }
    double v = row_sum(cash, val[0]);
    v = row_sum(v, val[1]);
    const double r = (v - asset) * C.reward_scale;
    cumrew = cumrew + r;
    asset = v;

    // Results: quantities and rewards straight from the owning lanes; the state rows' own
    // entries through LDS, then the rows by column groups as in the lane kernel.
    const bool own = env_ok && lead;
    if (A.qty) {
      const __amdgpu_buffer_rsrc_t rq = range_rsrc(reinterpret_cast<const float*>(A.qty) + row0 * D, M * D);
#pragma unroll
      for (int s = 0; s < 2; ++s)
        __builtin_amdgcn_raw_buffer_store_b32(q[s] < 0 ? -sold[s] : kown[s], rq, own ? 4 * blk(s) : kNoStore, 0, 0);
    }
    if (A.rew && own && jl == 0) A.rew[row0 + m] = r;
    wave_lds_sync();  // the previous step's rows have been stored
    if (jl == 0) ent[m * kRow] = static_cast<float>(cash * static_cast<double>(C.cash_scale));
#pragma unroll
    for (int s = 0; s < 2; ++s) ent[m * kRow + 1 + jl + 16 * s] = static_cast<float>(hold[s]) * C.hold_scale;
    wave_lds_sync();
    if (A.obs) {
      const __amdgpu_buffer_rsrc_t orow = range_rsrc(A.obs + row0 * S, M * S);
      const int ent_o = static_cast<int>(ent - mcl), pn_o = static_cast<int>(px - mcl) + D;
      const int ind_o = static_cast<int>(ind - mcl);
#pragma unroll
      for (int g = 0; g < kColGroups; ++g) {
        const int f = lane + 64 * g;
        const bool own_col = f == 0 || (f > D && f <= 2 * D);
        const int src = own_col ? ent_o + (f == 0 ? 0 : f - D) : (f <= D ? pn_o + f - 1 : ind_o + min(f, S - 1) - 1 - 2 * D);
        const float scale = (f >= 1 && f <= D) ? C.price_scale : 1.0f;
        const int cb = f < S ? 4 * f : kNoStore;
        const float x0 = mcl[src], x1 = mcl[src + (own_col ? kRow : 0)];
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x0 * scale), orow, cb, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x1 * scale), orow, 4 * S + cb, 0, 0);
      }
    }
  }

  if (env_ok && lead) {
    if (jl == 0) {
      st.cash[n] = cash;
      st.asset[n] = asset;
      st.cumrew[n] = cumrew;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int d = jl + 16 * s;
      __builtin_amdgcn_raw_buffer_store_b32(hold[s], hr, d < D ? 4 * (d * N + n) : kNoStore, 0, 0);
    }
  }
}

template <int MODE, int E>
hipError_t launch_row_e(const EnvConst& C, const EnvState& st, const LaneArgs& A, hipStream_t stream) {
  const int waves = (C.N + E - 1) / E;
  const int grid = (waves + kWaves - 1) / kWaves;
  const size_t lds = sizeof(float) * kWaves * row_wave_floats();
  hipLaunchKernelGGL((env_row_kernel<MODE, E>), dim3(grid), dim3(kWaves * 64), lds, stream, C, st, A);
  return hipGetLastError();
}

// A.M: environments per wavefront, 1 or 2 (0: by N).
template <int MODE>
hipError_t launch_row(const EnvConst& C, const EnvState& st, const LaneArgs& A, hipStream_t stream) {
  if (!env_lane_shape(C) || (MODE == kMeans && A.K > 8) || A.M < 0 || A.M > kRowEnvs) return hipErrorInvalidValue;
  if (A.n_steps <= 0 || C.N <= 0) return hipSuccess;
  return A.M == 1 ? launch_row_e<MODE, 1>(C, st, A, stream) : launch_row_e<MODE, 2>(C, st, A, stream);
}

template <int MODE>
hipError_t launch_mode(const EnvConst& C, const EnvState& st, LaneArgs A, hipStream_t stream) {
  if (!env_lane_shape(C)) return hipErrorInvalidValue;
  if (A.n_steps <= 0 || C.N <= 0) return hipSuccess;
  if (A.M <= 0) {
    // One wavefront per SIMD (four per compute unit) when the batch allows, up to 64 lanes each.
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    A.M = (C.N + 4 * cus - 1) / (4 * cus);
  }
  A.M = max(1, min(A.M, kMaxEnvs));
  // The staging area: the driven tile, or all K actors' mean tiles when they fit (fetched with
  // the market rows, under the noise); larger batches read the means into registers per actor.
  const int slot = stage_floats(A.M, C.D);
  A.mu_slot = (MODE == kMeans && A.K * slot <= kMuStage) ? slot : 0;
  A.stage = MODE == kDriven ? slot : (A.mu_slot > 0 ? A.K * slot : 64);
  if (C.D <= 8) return launch_dp<MODE, 8>(C, st, A, stream);
  if (C.D <= 16) return launch_dp<MODE, 16>(C, st, A, stream);
  return launch_dp<MODE, 32>(C, st, A, stream);
}

}  // namespace

bool env_lane_shape(const EnvConst& C) {
  return C.D >= 1 && C.D <= 32 && (2 + C.I) * C.D < kMaxMkt;
}

hipError_t launch_env_lane_given(const EnvConst& C, const EnvState& st, int t0, int n_steps, const float* act,
                                 float* obs, double* rew, int* qty, int envs_per_wave, hipStream_t stream) {
  LaneArgs A{};
  A.t0 = t0;
  A.n_steps = n_steps;
  A.M = envs_per_wave;
  A.act = act;
  A.obs = obs;
  A.rew = rew;
  A.qty = qty;
  return launch_mode<kDriven>(C, st, A, stream);
}

hipError_t launch_env_row_given(const EnvConst& C, const EnvState& st, int t0, int n_steps, const float* act,
                                float* obs, double* rew, int* qty, int envs_per_wave, hipStream_t stream) {
  LaneArgs A{};
  A.M = envs_per_wave;
  A.t0 = t0;
  A.n_steps = n_steps;
  A.act = act;
  A.obs = obs;
  A.rew = rew;
  A.qty = qty;
  return launch_row<kDriven>(C, st, A, stream);
}

hipError_t launch_env_row_ensemble_step(const EnvConst& C, const EnvState& st, int t, const float* mu,
                                        const float* mix, int K, float sigma, uint64_t key, int64_t env_offset,
                                        float* obs, float* act_out, double* rew, int* qty, int envs_per_wave,
                                        hipStream_t stream) {
  LaneArgs A{};
  A.M = envs_per_wave;
  A.t0 = t;
  A.n_steps = 1;
  A.mu = mu;
  A.mix = mix;
  A.K = K;
  A.sigma = sigma;
  A.noise_key = key;
  A.env_offset = env_offset;
  A.obs = obs;
  A.act_out = act_out;
  A.rew = rew;
  A.qty = qty;
  return launch_row<kMeans>(C, st, A, stream);
}

hipError_t launch_env_lane_ensemble_step(const EnvConst& C, const EnvState& st, int t, const float* mu,
                                         const float* mix, int K, float sigma, uint64_t key, int64_t env_offset,
                                         float* obs, float* act_out, double* rew, int* qty, int envs_per_wave,
                                         hipStream_t stream) {
  LaneArgs A{};
  A.t0 = t;
  A.n_steps = 1;
  A.M = envs_per_wave;
  A.mu = mu;
  A.mix = mix;
  A.K = K;
  A.sigma = sigma;
  A.noise_key = key;
  A.env_offset = env_offset;
  A.obs = obs;
  A.act_out = act_out;
  A.rew = rew;
  A.qty = qty;
  return launch_mode<kMeans>(C, st, A, stream);
}

}  // namespace fm
