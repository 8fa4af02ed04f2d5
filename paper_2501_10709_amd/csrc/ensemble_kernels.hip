// Ensemble kernels: weight packing, the per-actor MLP over 16- or 32-row tiles, and the combine step
// (weighted average of the actor means, Gaussian noise, clip) used by ensemble_act.
#include <algorithm>

#include "device_common.h"
#include "launch.h"
#include "mlp_device.h"

namespace fm {

namespace {

// Pack one float32 matrix W [kin][nout] (row-major) into the MFMA B-operand layout of DT.
template <int DT>
__global__ void pack_matrix_kernel(const float* __restrict__ w, int kin, int nout, int kin_pad,
                                   int nout_pad, void* __restrict__ out) {
  const size_t total = static_cast<size_t>(kin_pad) * nout_pad;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int k, col;
  if constexpr (DT == kF32) {
    // i = ((c * KQ + kq) * 64 + lane) * 4 + e
    const int e = static_cast<int>(i & 3);
    const int lane = static_cast<int>((i >> 2) & 63);
    const size_t rest = i >> 8;
    const int KQ = kin_pad / 16;
    const int kq = static_cast<int>(rest % KQ);
    const int c = static_cast<int>(rest / KQ);
    k = 16 * kq + 4 * e + (lane >> 4);
    col = 16 * c + (lane & 15);
    static_cast<float*>(out)[i] = (k < kin && col < nout) ? w[static_cast<size_t>(k) * nout + col] : 0.0f;
  } else {
    // i = ((c * KK + kk) * 64 + lane) * 8 + j
    const int j = static_cast<int>(i & 7);
    const int lane = static_cast<int>((i >> 3) & 63);
    const size_t rest = i >> 9;
    const int KK = kin_pad / 32;
    const int kk = static_cast<int>(rest % KK);
    const int c = static_cast<int>(rest / KK);
    k = 32 * kk + 8 * (lane >> 4) + j;
    col = 16 * c + (lane & 15);
    const float v = (k < kin && col < nout) ? w[static_cast<size_t>(k) * nout + col] : 0.0f;
    static_cast<__bf16*>(out)[i] = static_cast<__bf16>(v);  // round to nearest even
  }
}

// Rows 0 and A+1..2A of W1 [S][H] (cash, holdings) as bfloat16 MFMA fragments over ke_pad rows.
__global__ void pack_env_rows_kernel(const float* __restrict__ w1, int A, int H, int ke_pad,
                                     __bf16* __restrict__ out) {
  const size_t total = static_cast<size_t>(ke_pad) * H;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  // i = ((c * KK + kk) * 64 + lane) * 8 + j
  const int j = static_cast<int>(i & 7);
  const int lane = static_cast<int>((i >> 3) & 63);
  const size_t rest = i >> 9;
  const int KK = ke_pad / 32;
  const int kk = static_cast<int>(rest % KK);
  const int c = static_cast<int>(rest / KK);
  const int k = 32 * kk + 8 * (lane >> 4) + j;
  const int col = 16 * c + (lane & 15);
  const int row = k == 0 ? 0 : (k <= A ? A + k : -1);
  const float v = (row >= 0 && col < H) ? w1[static_cast<size_t>(row) * H + col] : 0.0f;
  out[i] = static_cast<__bf16>(v);
}

// Rows 1..A and 2A+1..S-1 of W1 [S][H] (closes, indicators) as bfloat16 [S-1-A][H].
__global__ void gather_market_rows_kernel(const float* __restrict__ w1, int S, int H, int A,
                                          __bf16* __restrict__ out) {
  const size_t total = static_cast<size_t>(S - 1 - A) * H;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int f = static_cast<int>(i / H), col = static_cast<int>(i - static_cast<size_t>(f) * H);
  const int row = f < A ? 1 + f : A + 1 + f;
  out[i] = static_cast<__bf16>(w1[static_cast<size_t>(row) * H + col]);
}

__global__ void copy_pad_kernel(const float* __restrict__ src, int n, int n_pad,
                                float* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_pad) dst[i] = i < n ? src[i] : 0.0f;
}

// The MLP of actor blockIdx.y on rows [16 RT blockIdx.x, +16 RT) of obs [n][S]; writes tanh
// outputs to mu [K][n][A].
template <int DT, int TMAX, int RT, int NW>
__global__ __launch_bounds__(64 * NW) void mlp_kernel(EnsDev E, const float* __restrict__ obs, int n,
                                                  float* __restrict__ mu) {
  using act_t = typename MT<DT>::act_t;
  constexpr int R = 16 * RT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = blockIdx.y;
  const int row0 = blockIdx.x * R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int st0 = act_stride<DT>(E.S_pad), sth = act_stride<DT>(E.H);
  // Two LDS regions: the state tile, then layer 2's outputs, in the first; layer 1's in the second.
  act_t* x0 = reinterpret_cast<act_t*>(smem);
  act_t* x1 = x0 + R * max(st0, sth);
  act_t* x2 = x0;

  // Stage the state tile, zero-padded to S_pad columns and R rows.
  for (int i = threadIdx.x; i < R * E.S_pad; i += 64 * NW) {
    const int r = i / E.S_pad, c = i - r * E.S_pad;
    float v = 0.0f;
    if (c < E.S && row0 + r < n) v = obs[static_cast<size_t>(row0 + r) * E.S + c];
    x0[r * st0 + c] = static_cast<act_t>(v);
  }
  __syncthreads();

  const unsigned char* P = E.base + static_cast<size_t>(k) * E.actor_stride;
  const float* b1 = reinterpret_cast<const float*>(P + E.off_b1);
  const float* b2 = reinterpret_cast<const float*>(P + E.off_b2);
  const float* b3 = reinterpret_cast<const float*>(P + E.off_b3);
  const int row_q = 4 * (lane >> 4), col_l = lane & 15;

  // Each layer's biases for the wavefront's output tiles are requested before its k loop, so that
  // the epilogue does not wait a memory round trip for them.
  const int ht = E.H / 16;
  float bv[TMAX];
  auto bias = [&](const float* b, int ntiles, int nout) {
#pragma unroll
    for (int i = 0; i < TMAX; ++i) {
      const int col = 16 * (wave + NW * i) + col_l;
      bv[i] = wave + NW * i < ntiles && col < nout ? b[col] : 0.0f;
    }
  };
  auto hidden_epi = [&](act_t* out, int ost) {
    return [=, &bv](int rt, int i, int c, floatx4 acc) {
      const int col = 16 * c + col_l;
      const float b = bv[i];
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(16 * rt + row_q + r) * ost + col] = static_cast<act_t>(fast_tanh(acc[r] + b));
    };
  };
  bias(b1, ht, E.H);
  mlp_layer<DT, TMAX, RT, NW>(x0, st0, E.S_pad, P + E.off_w1, ht, wave, lane, hidden_epi(x1, sth));
  bias(b2, ht, E.H);
  __syncthreads();
  mlp_layer<DT, TMAX, RT, NW>(x1, sth, E.H, P + E.off_w2, ht, wave, lane, hidden_epi(x2, sth));
  __syncthreads();
  float* mu_k = mu + static_cast<size_t>(k) * n * E.A;
  // Layer 3's bias of this wavefront's output tile (slot 0: tile c = wave in both forms below).
  const float b3v = wave < E.A_pad / 16 && 16 * wave + col_l < E.A ? b3[16 * wave + col_l] : 0.0f;
  auto out_epi = [&](int rt, floatx4 acc, int c) {
    const int col = 16 * c + col_l;
    if (col >= E.A) return;
    const float b = c == wave ? b3v : b3[col];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + 16 * rt + row_q + r;
      if (row < n) mu_k[static_cast<size_t>(row) * E.A + col] = fast_tanh(acc[r] + b);
    }
  };
  // Layer 3 has few output tiles (A_pad / 16): its k range is split over the otherwise idle
  // wavefronts, whose partial tiles meet in LDS (over layer 1's outputs, no longer needed) and
  // are summed in slice order.
  const int nt3 = E.A_pad / 16;
  const int nk3 = E.H / MT<DT>::kKGroup;
  const int cap = R * sth * static_cast<int>(sizeof(act_t)) / (nt3 * RT * 1024);
  const int slices = max(1, min(min(NW / nt3, nk3), cap));
  if (slices == 1) {
    mlp_layer<DT, TMAX, RT, NW>(x2, sth, E.H, P + E.off_w3, nt3, wave, lane,
                                [&](int rt, int, int c, floatx4 acc) { out_epi(rt, acc, c); });
    return;
  }
  floatx4* part = reinterpret_cast<floatx4*>(x1);  // [slices][nt3][RT][64]
  const int c3 = wave % nt3, sl = wave / nt3;
  if (sl < slices)
    mlp_layer<DT, 1, RT, 1>(x2, sth, E.H, P + E.off_w3, nt3, c3, lane,
                            [&](int rt, int, int, floatx4 acc) { part[((sl * nt3 + c3) * RT + rt) * 64 + lane] = acc; },
                            sl * nk3 / slices, (sl + 1) * nk3 / slices);
  __syncthreads();
  if (wave < nt3) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      floatx4 acc = part[(wave * RT + rt) * 64 + lane];
      for (int q = 1; q < slices; ++q) {
        const floatx4 p = part[((q * nt3 + wave) * RT + rt) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = acc[r] + p[r];
      }
      out_epi(rt, acc, wave);
    }
  }
}

// a_bar = sum_k w_k mu_k; a = clip(a_bar + sigma * eps, -1, 1).  One thread per (row, group of
// four outputs) so each Philox block is drawn once.
__global__ void combine_kernel(int K, int n, int A, const float* __restrict__ mu,
                               const float* __restrict__ mix, float sigma, uint64_t key, int t,
                               int64_t env_offset, float* __restrict__ mean,
                               float* __restrict__ act) {
  const int G = (A + 3) >> 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * G) return;
  const int row = i / G, g = i - row * G;
  float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (sigma != 0.0f)
    noise_block(key, static_cast<uint64_t>(env_offset + row), static_cast<uint64_t>(t),
                static_cast<uint64_t>(g), z);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int d = 4 * g + r;
    if (d >= A) break;
    const size_t o = static_cast<size_t>(row) * A + d;
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) acc = acc + mix[k] * mu[static_cast<size_t>(k) * n * A + o];
    if (mean) mean[o] = acc;
    float a = acc;
    if (sigma != 0.0f) a = acc + sigma * z[r];
    act[o] = fminf(fmaxf(a, -1.0f), 1.0f);
  }
}

template <int DT>
hipError_t launch_mlp_dt(const EnsDev& E, const float* obs, int n, float* mu, hipStream_t stream) {
  const int st0 = act_stride<DT>(E.S_pad), sth = act_stride<DT>(E.H);
  // Tiles of 32 rows (each weight fragment serves two row tiles) on sixteen wavefronts, each
  // owning one or two output column tiles of every layer; a single 16-row tile on four
  // wavefronts when the batch fits one.  Measured on MI355X (float32, hidden 256, N = 2048):
  // 32 rows on 16 wavefronts beat 16 rows on 4 (the former schedule) by 15% per rollout, although
  // they leave a quarter of the compute units idle.
  const bool two = n > 16;
  const int rt = two ? 2 : 1;
  const size_t lds = static_cast<size_t>(16 * rt) * (std::max(st0, sth) + sth) * MT<DT>::kElem;
  const dim3 grid((n + 16 * rt - 1) / (16 * rt), E.K);
  auto go = [&](auto kern, int waves) -> hipError_t {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(64 * waves), lds, stream, E, obs, n, mu);
    return hipGetLastError();
  };
  if (two) {
    const int tiles_per_wave = (E.H / 16 + 15) / 16;
    if (tiles_per_wave <= 2) return go(mlp_kernel<DT, 2, 2, 16>, 16);
    return go(mlp_kernel<DT, 4, 2, 16>, 16);
  }
  const int tiles_per_wave = (E.H / 16 + 3) / 4;
  if (tiles_per_wave <= 2) return go(mlp_kernel<DT, 2, 1, 4>, 4);
  if (tiles_per_wave <= 4) return go(mlp_kernel<DT, 4, 1, 4>, 4);
  return go(mlp_kernel<DT, 8, 1, 4>, 4);
}

}  // namespace

hipError_t launch_pack_matrix(int dtype, const float* w, int kin, int nout, int kin_pad,
                              int nout_pad, void* out, hipStream_t stream) {
  const size_t total = static_cast<size_t>(kin_pad) * nout_pad;
  const dim3 grid(static_cast<unsigned>((total + 255) / 256));
  if (dtype == kF32)
    hipLaunchKernelGGL(pack_matrix_kernel<kF32>, grid, dim3(256), 0, stream, w, kin, nout, kin_pad,
                       nout_pad, out);
  else
    hipLaunchKernelGGL(pack_matrix_kernel<kBF16>, grid, dim3(256), 0, stream, w, kin, nout, kin_pad,
                       nout_pad, out);
  return hipGetLastError();
}

hipError_t launch_pack_env_rows(const float* w1, int A, int H, int ke_pad, void* out, hipStream_t stream) {
  const size_t total = static_cast<size_t>(ke_pad) * H;
  hipLaunchKernelGGL(pack_env_rows_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, stream,
                     w1, A, H, ke_pad, static_cast<__bf16*>(out));
  return hipGetLastError();
}

hipError_t launch_gather_market_rows(const float* w1, int S, int H, int A, __bf16* out, hipStream_t stream) {
  const size_t total = static_cast<size_t>(S - 1 - A) * H;
  hipLaunchKernelGGL(gather_market_rows_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                     stream, w1, S, H, A, out);
  return hipGetLastError();
}

hipError_t launch_copy_pad(const float* src, int n, int n_pad, float* dst, hipStream_t stream) {
  hipLaunchKernelGGL(copy_pad_kernel, dim3((n_pad + 255) / 256), dim3(256), 0, stream, src, n, n_pad,
                     dst);
  return hipGetLastError();
}

hipError_t launch_mlp(int dtype, const EnsDev& E, const float* obs, int n, float* mu,
                      hipStream_t stream) {
  return dtype == kF32 ? launch_mlp_dt<kF32>(E, obs, n, mu, stream)
                       : launch_mlp_dt<kBF16>(E, obs, n, mu, stream);
}

hipError_t launch_combine(int K, int n, int A, const float* mu, const float* mix, float sigma,
                          uint64_t key, int t, int64_t env_offset, float* mean, float* act,
                          hipStream_t stream) {
  const int total = n * ((A + 3) >> 2);
  hipLaunchKernelGGL(combine_kernel, dim3((total + 255) / 256), dim3(256), 0, stream, K, n, A, mu, mix,
                     sigma, key, t, env_offset, mean, act);
  return hipGetLastError();
}

}  // namespace fm
