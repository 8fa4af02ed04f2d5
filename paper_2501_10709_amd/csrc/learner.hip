// The learner that consumes the rollout's samples (include/learner.h): the policy gradient of
// eq. (4) with the agent-diversity term of eq. (5), by the chain rule through agent i's network.
//
// Pipeline, all on the caller's stream: the K actors' forward passes over the T*N sample rows
// (agent i last, so its layer activations stay in the workspace); the returns R_n; per row the
// derivative of the objective with respect to mu_i, times tanh' (the layer-3 delta); then back
// through layers 3, 2, 1: each weight and bias gradient [X | 1]^T G is a reduction over the rows,
// split over row chunks into float32 partial products and summed in float64 in chunk order; each
// delta of the layer below is (G W^T) * (1 - X^2), written over the activation it masks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/learner.h"
#include "device_common.h"
#include "mlp_device.h"
#include "status.h"

namespace fm {
namespace lrn {

constexpr int kTile = 128, kBK = 16, kThreads = 256, kMaxK = 8;

enum Epilogue { kBiasTanh = 0, kMaskTanhGrad = 1, kStore = 2 };

// C(m, n) = sum_k A(m, k) B(k, n) over k in the block's range, with element (m, k) of A at
// A[m * sam + k * sak] and (k, n) of B at B[k * sbk + n * sbn].  blockIdx.z selects a chunk of
// kc values of k (split reductions) and offsets C by z * scz.  Epilogues: kBiasTanh,
// C = tanh(acc + bias[n]) (from one exp2 and one reciprocal, absolute error below 1e-6); kMaskTanhGrad, C = acc * (1 - X^2) with X at the same place as C (C may
// be X itself: each element is read and written by one thread); kStore, C = acc.  A workgroup
// computes a 128 x TN tile: for TN = 128 each of its four wavefronts a 64 x 64 quarter, for
// TN = 32 (outputs at most 32 wide) a 32 x 32 quarter of the rows, as blocks of float32 MFMAs
// (16 x 16 x 4), accumulating over k in ascending order of 4-element steps.  The tile width
// changes only which threads compute an element, not its arithmetic.
struct Gemm {
  const float* A;
  long sam, sak;
  const float* B;
  long sbk, sbn;
  float* C;
  long scm, scn, scz;
  const float* bias;
  const float* X;
  int M, N, K, kc;
  int ones_row;  // rows m >= ones_row of A read as 1 (appends the column sums of B: bias gradients)
  // colsum: the workgroups of row tile 0 also sum B's columns over their k range (ascending k,
  // float32) and store them as row bias_row of C -- the column sums without a row tile of their
  // own when M is a multiple of the tile height.
  int colsum, bias_row;
};

template <int EPI, int TN>
__global__ __launch_bounds__(kThreads) void gemm_kernel(Gemm g) {
  static_assert(TN == kTile || TN == 32, "tiles 128 x 128 or 128 x 32");
  // Wavefronts along n (WN) and m; each owns BI x BJ blocks of 16 x 16.
  constexpr int WN = TN == kTile ? 2 : 1, BI = kTile / (4 / WN) / 16, BJ = TN / WN / 16;
  // Rows padded by 16 floats: the two k rows a half-wavefront reads sit 16 banks apart.
  __shared__ float As[kBK][kTile + 16];
  __shared__ float Bs[kBK][TN + 16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * TN;
  const int wm = (wave / WN) * 16 * BI, wn = (wave % WN) * 16 * BJ;  // this wavefront's quarter
  const int k_begin = blockIdx.z * g.kc, k_end = min(g.K, k_begin + g.kc);
  // Loads walk the operand's unit-stride index across neighbouring threads (coalesced).  Thread
  // tid moves elements e = 0..kPerA-1 of A's k-block (am, ak) and 0..kPerB-1 of B's (bk, bn).
  constexpr int kPerA = kTile * kBK / kThreads, kPerB = TN * kBK / kThreads;
  const bool a_kfast = g.sak == 1, b_kfast = g.sbk == 1;
  const int am0 = a_kfast ? tid / kBK : tid % kTile, ak0 = a_kfast ? tid % kBK : tid / kTile;
  const int bn0 = b_kfast ? tid / kBK : tid % TN, bk0 = b_kfast ? tid % kBK : tid / TN;
  constexpr int kStepFast = kThreads / kBK, kStepSlowA = kThreads / kTile, kStepSlowB = kThreads / TN;
  auto a_at = [&](int e, int& am, int& ak) {
    am = a_kfast ? am0 + kStepFast * e : am0;
    ak = a_kfast ? ak0 : ak0 + kStepSlowA * e;
  };
  auto b_at = [&](int e, int& bk, int& bn) {
    bn = b_kfast ? bn0 + kStepFast * e : bn0;
    bk = b_kfast ? bk0 : bk0 + kStepSlowB * e;
  };
  // The next k-block is read into registers while the current one is multiplied.
  float ra[kPerA], rb[kPerB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < kPerA; ++e) {
      int am, ak;
      a_at(e, am, ak);
      const int m = m0 + am, k = k0 + ak;
      ra[e] = (m < g.M && k < k_end) ? (m < g.ones_row ? g.A[m * g.sam + k * g.sak] : 1.0f) : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < kPerB; ++e) {
      int bk, bn;
      b_at(e, bk, bn);
      const int n = n0 + bn, kb = k0 + bk;
      rb[e] = (n < g.N && kb < k_end) ? g.B[kb * g.sbk + n * g.sbn] : 0.0f;
    }
  };
  floatx4 acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const bool do_colsum = g.colsum && blockIdx.x == 0 && tid < TN;
  float csum = 0.0f;
  if (k_begin < k_end) fetch(k_begin);
  for (int k0 = k_begin; k0 < k_end; k0 += kBK) {
#pragma unroll
    for (int e = 0; e < kPerA; ++e) {
      int am, ak;
      a_at(e, am, ak);
      As[ak][am] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < kPerB; ++e) {
      int bk, bn;
      b_at(e, bk, bn);
      Bs[bk][bn] = rb[e];
    }
    __syncthreads();
    if (k0 + kBK < k_end) fetch(k0 + kBK);
    if (do_colsum) {
      // Rows beyond k_end were stored as zero, so they add nothing.
#pragma unroll
      for (int kk = 0; kk < kBK; ++kk) csum = csum + Bs[kk][tid];
    }
    // v_mfma_f32_16x16x4_f32: lane l supplies A[row l%16][k l/16] and B[k l/16][col l%16].
#pragma unroll
    for (int kq = 0; kq < kBK; kq += 4) {
      float a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = As[kq + (lane >> 4)][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = Bs[kq + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // Lane l holds column l%16 and rows 4(l/16)..4(l/16)+3 of each 16 x 16 block.
  float* C = g.C + blockIdx.z * g.scz;
  if (do_colsum && n0 + tid < g.N) C[static_cast<long>(g.bias_row) * g.scm + (n0 + tid) * g.scn] = csum;
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
      if (n >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (m >= g.M) continue;
        const long o = m * g.scm + n * g.scn;
        const float v = acc[i][j][r];
        if (EPI == kBiasTanh) {
          C[o] = fast_tanh(v + g.bias[n]);
        } else if (EPI == kMaskTanhGrad) {
          const float x = g.X[o];
          C[o] = v * (1.0f - x * x);
        } else {
          C[o] = v;
        }
      }
    }
}

// R_n = sum_t r[t][n] in ascending t.
__global__ void returns_kernel(const double* rew, int T, int N, double* R) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double acc = 0.0;
  // Unrolled so that the loads issue ahead of the additions, which stay in ascending t.
#pragma unroll 8
  for (int t = 0; t < T; ++t) acc = acc + rew[static_cast<size_t>(t) * N + n];
  R[n] = acc;
}

struct Mix {
  float w[kMaxK];
};

// Layer-3 delta of agent i for row r = t*N + n and actions 4j..4j+3 (one noise block):
//   u = (R_n / N) (abar + sigma eps - mu_i) / sigma^2 + lambda/(N T) sum_{k != i} (mu_i - mu_k) / sigma^2
//   G3 = u (1 - mu_i^2).
__global__ void delta3_kernel(const float* mu, int K, int agent, Mix mix, int rows, int N, int T, int A,
                              const double* R, float sigma, uint64_t key, int64_t env_offset, int t0,
                              float lambda_kl, float* G3) {
  const int G = (A + 3) / 4;
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<long>(rows) * G) return;
  const int r = static_cast<int>(i / G), j = static_cast<int>(i % G);
  const int t = r / N, n = r % N;
  float z[4];
  // Row t of the samples was drawn on day t0 + t: the noise is keyed by the absolute day.
  noise_block(key, static_cast<uint64_t>(env_offset + n), static_cast<uint64_t>(t0 + t), static_cast<uint64_t>(j), z);
  const float inv_s2 = 1.0f / (sigma * sigma);
  const float rn = static_cast<float>(R[n] / N);
  const float kl = lambda_kl / (static_cast<float>(N) * static_cast<float>(T));
  for (int q = 0; q < 4; ++q) {
    const int a = 4 * j + q;
    if (a >= A) break;
    const size_t off = static_cast<size_t>(r) * A + a;
    const size_t plane = static_cast<size_t>(rows) * A;
    const float mi = mu[agent * plane + off];
    float abar = 0.0f, div = 0.0f;
    for (int k = 0; k < K; ++k) {
      const float mk = mu[k * plane + off];
      abar = abar + mix.w[k] * mk;
      if (k != agent) div = div + (mi - mk);
    }
    const float u = rn * ((abar + sigma * z[q]) - mi) * inv_s2 + kl * div * inv_s2;
    G3[off] = u * (1.0f - mi * mi);
  }
}

// out[i] = sum over chunks c (ascending) of P[c][i], in float64, rounded once.
__global__ void reduce_kernel(const float* P, int len, int n_chunks, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = 0.0;
#pragma unroll 8
  for (int c = 0; c < n_chunks; ++c) acc = acc + static_cast<double>(P[static_cast<size_t>(c) * len + i]);
  out[i] = static_cast<float>(acc);
}

struct Layout {
  size_t mu, x1, x2, g3, R, P, total;
  int rows, chunk, n_chunks;
};

Layout layout(int K, int S, int H, int A, int N, int T) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  Layout L{};
  L.rows = N * T;
  L.chunk = std::max(2048, (L.rows + 255) / 256);
  L.n_chunks = (L.rows + L.chunk - 1) / L.chunk;
  const size_t rows = L.rows;
  size_t o = 0;
  L.mu = o;
  o = al(o + sizeof(float) * K * rows * A);
  L.x1 = o;
  o = al(o + sizeof(float) * rows * H);
  L.x2 = o;
  o = al(o + sizeof(float) * rows * H);
  L.g3 = o;
  o = al(o + sizeof(float) * rows * A);
  L.R = o;
  o = al(o + sizeof(double) * N);
  const size_t pmax = std::max({static_cast<size_t>(S + 1) * H, static_cast<size_t>(H + 1) * H,
                                static_cast<size_t>(H + 1) * A});
  L.P = o;
  o = al(o + sizeof(float) * L.n_chunks * pmax);
  L.total = o;
  return L;
}

// Outputs at most 32 wide (the action layer) take 128 x 32 tiles instead of padding to 128.
template <int EPI>
hipError_t gemm(const Gemm& g, int z, hipStream_t stream) {
  if (g.N <= 32) {
    const dim3 grid((g.M + kTile - 1) / kTile, 1, z);
    hipLaunchKernelGGL((gemm_kernel<EPI, 32>), grid, dim3(kThreads), 0, stream, g);
  } else {
    const dim3 grid((g.M + kTile - 1) / kTile, (g.N + kTile - 1) / kTile, z);
    hipLaunchKernelGGL((gemm_kernel<EPI, kTile>), grid, dim3(kThreads), 0, stream, g);
  }
  return hipGetLastError();
}

// Weight and bias gradients [X | 1]^T G: Xr [rows][kin] (row stride ldx), Gr [rows][kout]; the
// result [kin + 1][kout] (weights, then the bias as the row of ones) into out, which is the
// layout of W followed by b in the master weights.
hipError_t weight_grad(const Layout& L, const float* Xr, int kin, int ldx, const float* Gr, int kout, float* P,
                       float* out, hipStream_t stream) {
  Gemm g{};
  g.A = Xr;
  g.sam = 1;
  g.sak = ldx;
  g.B = Gr;
  g.sbk = kout;
  g.sbn = 1;
  g.C = P;
  g.scm = kout;
  g.scn = 1;
  g.scz = static_cast<long>(kin + 1) * kout;
  // With kin a multiple of the tile height the bias row (the column sums of G) would take a row
  // tile of its own; the first row tile's workgroups sum the columns instead.
  const bool own = kin % kTile == 0;
  g.M = own ? kin : kin + 1;
  g.N = kout;
  g.K = L.rows;
  g.kc = L.chunk;
  g.ones_row = kin;
  g.colsum = own ? 1 : 0;
  g.bias_row = kin;
  hipError_t e = gemm<kStore>(g, L.n_chunks, stream);
  if (e != hipSuccess) return e;
  const int len = (kin + 1) * kout;
  hipLaunchKernelGGL(reduce_kernel, dim3((len + 255) / 256), dim3(256), 0, stream, P, len, L.n_chunks, out);
  return hipGetLastError();
}

// Delta of the layer below: Gout [rows][kin] = (Gin [rows][kout] W^T) * (1 - X^2), W [kin][kout],
// written over X [rows][kin].
hipError_t back_delta(const Layout& L, const float* Gin, int kout, const float* W, int kin, float* X,
                      hipStream_t stream) {
  Gemm g{};
  g.A = Gin;
  g.sam = kout;
  g.sak = 1;
  g.B = W;
  g.sbk = 1;
  g.sbn = kout;
  g.C = X;
  g.scm = kin;
  g.scn = 1;
  g.X = X;
  g.M = L.rows;
  g.N = kin;
  g.K = kout;
  g.kc = kout;
  g.ones_row = g.M;
  return gemm<kMaskTanhGrad>(g, 1, stream);
}

// Y [rows][kout] = tanh(X [rows][kin] W + b).
hipError_t layer(const Layout& L, const float* X, int kin, const float* W, const float* b, int kout, float* Y,
                 hipStream_t stream) {
  Gemm g{};
  g.A = X;
  g.sam = kin;
  g.sak = 1;
  g.B = W;
  g.sbk = kout;
  g.sbn = 1;
  g.C = Y;
  g.scm = kout;
  g.scn = 1;
  g.bias = b;
  g.M = L.rows;
  g.N = kout;
  g.K = kin;
  g.kc = kin;
  g.ones_row = g.M;
  return gemm<kBiasTanh>(g, 1, stream);
}

bool dims_ok(int K, int S, int H, int A, int N, int T) {
  if (K < 1 || K > kMaxK || S < 1 || S > 1024 || H < 1 || H > 1024 || A < 1 || A > 128 || N < 1 || T < 1)
    return false;
  return static_cast<int64_t>(N) * T <= (int64_t(1) << 26);
}

}  // namespace lrn
}  // namespace fm

extern "C" {

size_t fm_pg_workspace_bytes(int32_t K, int32_t S, int32_t H, int32_t A, int32_t N, int32_t T) {
  if (!fm::lrn::dims_ok(K, S, H, A, N, T)) return 0;
  return fm::lrn::layout(K, S, H, A, N, T).total;
}

fm_status fm_policy_gradient(int32_t K, int32_t S, int32_t H, int32_t A, const float* d_w, const float* h_mix,
                             int32_t agent, const float* d_states, const double* d_rew, int32_t N, int32_t T,
                             float sigma, uint64_t noise_key, int64_t env_offset, int32_t t0, float lambda_kl,
                             float* d_grad, void* d_workspace, size_t workspace_bytes, hipStream_t stream) {
  using namespace fm::lrn;
  if (!dims_ok(K, S, H, A, N, T))
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: sizes out of range (K 1..8, S/H 1..1024, A 1..128, N*T <= 2^26)");
  if (agent < 0 || agent >= K) return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: agent out of range");
  if (!d_w || !d_states || !d_rew || !d_grad || !d_workspace)
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: NULL buffer");
  if (!(sigma > 0.0f) || !std::isfinite(sigma)) return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: sigma must be finite and > 0");
  if (!(lambda_kl >= 0.0f) || !std::isfinite(lambda_kl))
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: lambda_kl must be finite and >= 0");
  if (env_offset < 0) return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: env_offset must be >= 0");
  if (t0 < 0 || static_cast<int64_t>(t0) + T > (int64_t{1} << 31) - 1)
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: t0 must be >= 0 and t0 + T must fit int32");
  const Layout L = layout(K, S, H, A, N, T);
  if (workspace_bytes < L.total || reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: workspace smaller than fm_pg_workspace_bytes or not 256-byte aligned");
  Mix mix{};
  for (int k = 0; k < K; ++k) {
    mix.w[k] = h_mix ? h_mix[k] : 1.0f / K;
    if (!std::isfinite(mix.w[k])) return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient: mix weights must be finite");
  }
  unsigned char* ws = static_cast<unsigned char*>(d_workspace);
  float* mu = reinterpret_cast<float*>(ws + L.mu);
  float* x1 = reinterpret_cast<float*>(ws + L.x1);
  float* x2 = reinterpret_cast<float*>(ws + L.x2);
  float* g3 = reinterpret_cast<float*>(ws + L.g3);
  double* R = reinterpret_cast<double*>(ws + L.R);
  float* P = reinterpret_cast<float*>(ws + L.P);
  const size_t per = static_cast<size_t>(S) * H + H + static_cast<size_t>(H) * H + H + static_cast<size_t>(H) * A + A;
  const size_t oW1 = 0, ob1 = static_cast<size_t>(S) * H, oW2 = ob1 + H, ob2 = oW2 + static_cast<size_t>(H) * H,
               oW3 = ob2 + H, ob3 = oW3 + static_cast<size_t>(H) * A;
  hipError_t e = hipSuccess;
  // Forward passes, agent i last so that x1, x2 hold its activations.
  for (int step = 0; step < K && e == hipSuccess; ++step) {
    const int k = step < K - 1 ? (step < agent ? step : step + 1) : agent;
    const float* w = d_w + per * k;
    e = layer(L, d_states, S, w + oW1, w + ob1, H, x1, stream);
    if (e == hipSuccess) e = layer(L, x1, H, w + oW2, w + ob2, H, x2, stream);
    if (e == hipSuccess) e = layer(L, x2, H, w + oW3, w + ob3, A, mu + static_cast<size_t>(k) * L.rows * A, stream);
  }
  if (e != hipSuccess) return fm::device_error(e, "fm_policy_gradient (forward)");
  hipLaunchKernelGGL(returns_kernel, dim3((N + 255) / 256), dim3(256), 0, stream, d_rew, T, N, R);
  const long nd = static_cast<long>(L.rows) * ((A + 3) / 4);
  hipLaunchKernelGGL(delta3_kernel, dim3(static_cast<unsigned>((nd + 255) / 256)), dim3(256), 0, stream, mu, K,
                     agent, mix, L.rows, N, T, A, R, sigma, noise_key, env_offset, t0, lambda_kl, g3);
  e = hipGetLastError();
  if (e != hipSuccess) return fm::device_error(e, "fm_policy_gradient (delta)");
  const float* wi = d_w + per * agent;
  // Layer 3, then the delta of layer 2 over x2, layer 2, the delta of layer 1 over x1, layer 1.
  e = weight_grad(L, x2, H, H, g3, A, P, d_grad + oW3, stream);
  if (e == hipSuccess) e = back_delta(L, g3, A, wi + oW3, H, x2, stream);
  if (e == hipSuccess) e = weight_grad(L, x1, H, H, x2, H, P, d_grad + oW2, stream);
  if (e == hipSuccess) e = back_delta(L, x2, H, wi + oW2, H, x1, stream);
  if (e == hipSuccess) e = weight_grad(L, d_states, S, S, x1, H, P, d_grad + oW1, stream);
  if (e != hipSuccess) return fm::device_error(e, "fm_policy_gradient (backward)");
  return FM_OK;
}

// ------------------------------------------------------------------------------------------
// The allocation-free variant: the same computation with its workspace in a file-scope device
// array instead of a caller buffer.  Each device the library runs on holds its own copy of the
// array; its address is looked up once per device (the array's name is a host-side stand-in, not
// a device address) and kept.  Every call on a device shares that device's array, so calls that
// overlap on one device race.  The workspace needs no clearing: every region is written before
// it is read within a call.
// ------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FM_PG_NOALLOC_MAX_BYTES];

fm_status fm_policy_gradient_noalloc(int32_t K, int32_t S, int32_t H, int32_t A, const float* d_w, const float* h_mix,
                                     int32_t agent, const float* d_states, const double* d_rew, int32_t N, int32_t T,
                                     float sigma, uint64_t noise_key, int64_t env_offset, int32_t t0, float lambda_kl,
                                     float* d_grad, hipStream_t stream) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  const size_t need = fm_pg_workspace_bytes(K, S, H, A, N, T);
  if (need == 0)
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient_noalloc: sizes out of range (K 1..8, S/H 1..1024, A 1..128, N*T <= 2^26)");
  if (need > FM_PG_NOALLOC_MAX_BYTES)
    return fm::set_error(FM_ERR_INVALID, "fm_policy_gradient_noalloc: the problem needs " + std::to_string(need) +
                                             " bytes of workspace, more than the " +
                                             std::to_string(FM_PG_NOALLOC_MAX_BYTES) + " the library holds");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fm::device_error(e, "fm_policy_gradient_noalloc (hipGetDevice)");
  if (dev < 0 || dev >= kMaxDevices) return fm::set_error(FM_ERR_UNSUPPORTED, "fm_policy_gradient_noalloc: device index above 63");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return fm::device_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                         "fm_policy_gradient_noalloc (hipGetSymbolAddress)");
      addr[dev] = p;
    }
    ws = addr[dev];
  }
  return fm_policy_gradient(K, S, H, A, d_w, h_mix, agent, d_states, d_rew, N, T, sigma, noise_key, env_offset, t0,
                            lambda_kl, d_grad, ws, FM_PG_NOALLOC_MAX_BYTES, stream);
}

}  // extern "C"
