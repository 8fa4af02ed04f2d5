// Ensemble MLP building blocks on MFMA (gfx950).
//
// Each actor is S -> H -> H -> A with tanh after every layer.  A workgroup evaluates one layer
// for a tile of 16 or 32 states: the tile's activations sit in LDS (row-major, padded rows), the
// layer's weights are pre-packed so that every lane of a wavefront fetches the B-operand of an
// MFMA with one contiguous load, and the wavefronts of the workgroup split the layer's
// 16-column output tiles between them.
//
//   float32:  v_mfma_f32_16x16x4_f32, B packed [col tile][k/16][lane][4]
//             (element e of lane l is W[16 kq + 4 e + l/16][16 c + l%16])
//   bfloat16: v_mfma_f32_16x16x32_bf16, B packed [col tile][k/32][lane][8]
//             (element j of lane l is W[32 kk + 8 (l/16) + j][16 c + l%16])
//
// In both, lane l holds rows 4(l/16)..4(l/16)+3 of column l%16 of the 16x16 accumulator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;

enum { kF32 = 0, kBF16 = 1 };

template <int DT>
struct MT;
template <>
struct MT<kF32> {
  using act_t = float;
  static constexpr int kKGroup = 16;  // k covered by one packed load per lane
  static constexpr int kElem = 4;     // bytes per weight
};
template <>
struct MT<kBF16> {
  using act_t = __bf16;
  static constexpr int kKGroup = 32;
  static constexpr int kElem = 2;
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Row stride (elements) of an LDS activation tile with kin_pad columns: keeps the MFMA
// A-operand reads free of bank conflicts.
template <int DT>
__host__ __device__ inline int act_stride(int kin_pad) {
  return DT == kF32 ? round_up(kin_pad, 32) + 2 : kin_pad + 8;
}

// Device view of a packed ensemble.
struct EnsDev {
  int K, S, H, A;
  int S_pad, A_pad;  // layer-1 input and layer-3 output, padded
  const unsigned char* base;
  size_t actor_stride;
  size_t off_w1, off_w2, off_w3, off_b1, off_b2, off_b3;
  const float* mix;  // [K]
  // Split first layer (bfloat16 ensembles whose input is a trading state [cash, closes(A),
  // holdings(A), indicators]): W1 = W1e (rows of the per-environment entries: cash, holdings)
  // + W1m (rows of the market entries shared by all environments of a day).  split_a = A when
  // present, else 0.  Regions hold all actors back to back, from base.
  int split_a;
  int ke_pad;           // per-environment rows padded to a multiple of 32
  size_t off_w1e;       // [K][H/16][ke_pad/32][64][8] bfloat16 MFMA fragments
  size_t off_w1m;       // [K][S-1-A][H] bfloat16, row-major
};

// tanh from one exponential and one reciprocal: tanh|x| = (1 - e^{-2|x|}) / (1 + e^{-2|x|}).
// Absolute error below 1e-6 over the whole range.
__device__ __forceinline__ float fast_tanh(float x) {
  const float t = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(x));  // e^{-2|x|}
  const float y = (1.0f - t) * __builtin_amdgcn_rcpf(1.0f + t);
  return copysignf(y, x);
}

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// One layer for RT row tiles of 16 and the wavefront's column tiles c = wave, wave + NW, ...
// (< ntiles; NW wavefronts per workgroup).  sin: LDS tile [16 RT][in_stride] holding kin_pad
// valid (zero-padded) columns.  Calls epi(r, i, c, acc) for every (row tile r, column tile c) the
// wave owns.  Each B-operand fragment serves all RT row tiles; the fragments of the next RING
// k-steps are in flight while the current k-step's MFMAs run.  [kbeg, kend) restricts the sum to
// those k-steps (16 k for float32, 32 for bfloat16; kend < 0: to the end).
// The bfloat16 weights are read through a global-address-space pointer: a pointer that reached
// the kernel through memory (the batched form's group table) would otherwise be read with flat
// loads, which also count on the LDS counter, so that each wait for an activation fragment in
// LDS would wait for the weight prefetch as well.
template <int DT, int TMAX, int RT, int NW, class Epi, int RING = 4>
__device__ __forceinline__ void mlp_layer(const typename MT<DT>::act_t* sin, int in_stride,
                                          int kin_pad, const void* wp, int ntiles, int wave,
                                          int lane, Epi epi, int kbeg = 0, int kend = -1) {
  floatx4 acc[RT][TMAX];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int i = 0; i < TMAX; ++i) acc[r][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const int row = lane & 15, grp = lane >> 4;
  if constexpr (DT == kF32) {
    const float4* W = static_cast<const float4*>(wp);
    const int KQ = kin_pad / 16, K1 = kend < 0 ? KQ : min(kend, KQ);
    float4 ring[RING][TMAX];
    auto fetch = [&](float4 (&dst)[TMAX], int kq) {
#pragma unroll
      for (int i = 0; i < TMAX; ++i) {
        const int c = wave + NW * i;
        if (c < ntiles && kq < K1) dst[i] = W[(static_cast<size_t>(c) * KQ + kq) * 64 + lane];
      }
    };
#pragma unroll
    for (int j = 0; j < RING; ++j) fetch(ring[j], kbeg + j);
    for (int kq0 = kbeg; kq0 < K1; kq0 += RING) {
#pragma unroll
      for (int j = 0; j < RING; ++j) {
        const int kq = kq0 + j;
        if (kq < K1) {
          float4 b[TMAX];
#pragma unroll
          for (int i = 0; i < TMAX; ++i) b[i] = ring[j][i];
          fetch(ring[j], kq + RING);
          float a[RT][4];
#pragma unroll
          for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) a[r][e] = sin[(16 * r + row) * in_stride + 16 * kq + 4 * e + grp];
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int i = 0; i < TMAX; ++i) {
              if (wave + NW * i < ntiles) {
                const float bv = e == 0 ? b[i].x : e == 1 ? b[i].y : e == 2 ? b[i].z : b[i].w;
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r][i] = mfma_f32(a[r][e], bv, acc[r][i]);
              }
            }
        }
      }
    }
  } else {
    const __attribute__((address_space(1))) bf16x8* W = (const __attribute__((address_space(1))) bf16x8*)wp;
    const int KK = kin_pad / 32, K1 = kend < 0 ? KK : min(kend, KK);
    bf16x8 ring[RING][TMAX];
    auto fetch = [&](bf16x8 (&dst)[TMAX], int kk) {
#pragma unroll
      for (int i = 0; i < TMAX; ++i) {
        const int c = wave + NW * i;
        if (c < ntiles && kk < K1) dst[i] = W[(static_cast<size_t>(c) * KK + kk) * 64 + lane];
      }
    };
#pragma unroll
    for (int j = 0; j < RING; ++j) fetch(ring[j], kbeg + j);
    for (int kk0 = kbeg; kk0 < K1; kk0 += RING) {
#pragma unroll
      for (int j = 0; j < RING; ++j) {
        const int kk = kk0 + j;
        if (kk < K1) {
          bf16x8 b[TMAX];
#pragma unroll
          for (int i = 0; i < TMAX; ++i) b[i] = ring[j][i];
          fetch(ring[j], kk + RING);
          bf16x8 a[RT];
#pragma unroll
          for (int r = 0; r < RT; ++r)
            a[r] = *reinterpret_cast<const bf16x8*>(sin + (16 * r + row) * in_stride + 32 * kk + 8 * grp);
#pragma unroll
          for (int i = 0; i < TMAX; ++i)
            if (wave + NW * i < ntiles)
#pragma unroll
              for (int r = 0; r < RT; ++r) acc[r][i] = mfma_bf16(a[r], b[i], acc[r][i]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int i = 0; i < TMAX; ++i) {
      const int c = wave + NW * i;
      if (c < ntiles) epi(r, i, c, acc[r][i]);
    }
}

}  // namespace fm
