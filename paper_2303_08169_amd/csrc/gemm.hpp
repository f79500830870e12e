// Edge-batched matrix-core products for the per-edge MLPs (gfx950 MFMA).
//
// Every per-edge linear map of the model is y = x W over a batch of edges: a
// tall [E, K] x [K, N] product with K, N <= 1024 and E in the millions. One
// workgroup (4 wavefronts) owns BM edge rows and ALL N output columns, so the
// A rows are read once and an epilogue may read and overwrite them in place.
// K is walked in LDS-staged steps; W is tiny and stays L2-resident.
//   * BF16: v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation.
//   * FP32: v_mfma_f32_16x16x4_f32.
// A is produced by an ALoad functor (plain, SiLU of a stored pre-activation,
// concatenation of two sources, or an adjoint g * c * rowscale * SiLU'(a)) and
// results leave through an Epi functor (store, SiLU + cutoff scaling, residual
// update, adjoint split, accumulate), so each MLP layer and its adjoint are one
// launch each with no separate elementwise passes.
#pragma once

#include "nq_internal.hpp"

namespace nq {

__device__ inline float sigmoidf_(float a) { return 1.0f / (1.0f + __expf(-a)); }
__device__ inline float siluf(float a) { return a * sigmoidf_(a); }
__device__ inline float dsiluf(float a) {
  float s = sigmoidf_(a);
  return s * (1.0f + a * (1.0f - s));
}

constexpr float kInvSqrt2 = 0.70710678118654752f;

enum ALoadMode { A_PLAIN = 0, A_SILU = 1, A_CAT = 2, A_GRADSILU = 3 };

struct ALoad {
  int mode;
  const float* p0; int ld0; int K0;  // primary source
  const float* p1; int ld1; int K1;  // concatenated source, or the pre-activation for A_GRADSILU
  const float* rs; int rs_ld;        // optional per-row scale (the cutoff u)
  float c;                           // constant factor (A_GRADSILU)
  __device__ inline float operator()(int64_t r, int k) const {
    switch (mode) {
      case A_PLAIN: return k < K0 ? p0[r * ld0 + k] : 0.f;
      case A_SILU: return k < K0 ? siluf(p0[r * ld0 + k]) : 0.f;
      case A_CAT:
        if (k < K0) return p0[r * ld0 + k];
        if (k < K0 + K1) return p1[r * ld1 + (k - K0)];
        return 0.f;
      default: {
        if (k >= K0) return 0.f;
        float g = p0[r * ld0 + k] * c;
        if (rs) g *= rs[r * rs_ld];
        return g * dsiluf(p1[r * ld1 + k]);
      }
    }
  }
};

enum EpiMode { E_STORE = 0, E_STORE_X0 = 1, E_RESIDUAL = 2, E_LATENT_BWD = 3, E_ADD = 4 };

struct Epi {
  int mode;
  float* o0; int ld0; int N0;
  float* o1; int ld1;
  const float* x; int ldx;
  const float* rs; int rs_ld;
  int D;
  template <int MODE>
  __device__ inline void apply(int64_t r, int c, float v) const {
    if (c >= N0) return;
    if constexpr (MODE == E_STORE) {
      o0[r * ld0 + c] = v;
    } else if constexpr (MODE == E_STORE_X0) {
      o0[r * ld0 + c] = v;
      o1[r * ld1 + c] = rs[r * rs_ld] * siluf(v);
    } else if constexpr (MODE == E_RESIDUAL) {
      o0[r * ld0 + c] = v;
      o1[r * ld1 + c] = (x[r * ldx + c] + rs[r * rs_ld] * siluf(v)) * kInvSqrt2;
    } else if constexpr (MODE == E_LATENT_BWD) {
      if (c < D) {
        float* q = o0 + r * ld0 + c;
        *q = *q * kInvSqrt2 + v;
      } else {
        o1[r * ld1 + (c - D)] = v;
      }
    } else {
      o0[r * ld0 + c] += v;
    }
  }
};

// Writes the accumulator tiles of one wavefront through epilogue mode MODE.
// Lane l holds rows 4*(l/16)+q, column l%16 of every 16x16 tile.
template <int MODE, int MI, int NI>
__device__ inline void store_tiles(const Epi& ep, const floatx4 (&acc)[MI][NI], int64_t rbase, int cbase,
                                   int lane, int64_t nrows) {
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = rbase + i * 16 + (lane / 16) * 4 + q;
        const int col = cbase + j * 16 + lane % 16;
        if (row < nrows) ep.apply<MODE>(row, col, acc[i][j][q]);
      }
}

template <typename T> struct MfmaTraits;

template <> struct MfmaTraits<bf16> {
  static constexpr int BK = 32;
  static constexpr int PAD = 8;
};
template <> struct MfmaTraits<float> {
  static constexpr int BK = 16;
  static constexpr int PAD = 4;
};

// C[rows, NP] = A[rows, Kp] * Bt[NP, Kp]^T.  4 wavefronts as WM x WN.
template <typename T, int BM, int NP, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm(int Kp, const T* __restrict__ Bt,
                                              const int* __restrict__ nrows_p, ALoad ld, Epi ep) {
  constexpr int BK = MfmaTraits<T>::BK;
  constexpr int LDK = BK + MfmaTraits<T>::PAD;
  constexpr int RW = BM / WM;  // rows per wave
  constexpr int CW = NP / WN;  // cols per wave
  constexpr int MI = RW / 16;
  constexpr int NI = CW / 16;
  static_assert(WM * WN == 4, "4 wavefronts");
  static_assert(RW % 16 == 0 && CW % 16 == 0, "16x16 tiles");
  __shared__ __attribute__((aligned(16))) T As[BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[NP * LDK];

  const int64_t nrows = *nrows_p;
  const int64_t r0 = (int64_t)blockIdx.x * BM;
  if (r0 >= nrows) return;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int wm = wave / WN, wn = wave % WN;

  floatx4 acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < Kp; k0 += BK) {
    // stage A (BM x BK) through the loader
    for (int idx = tid; idx < BM * BK; idx += 256) {
      const int rr = idx / BK, kk = idx % BK;
      const int64_t row = r0 + rr;
      float v = (row < nrows) ? ld(row, k0 + kk) : 0.f;
      As[rr * LDK + kk] = (T)v;
    }
    // stage B (NP x BK), 16-byte chunks
    constexpr int CHUNKS = BK * (int)sizeof(T) / 16;  // 4
    for (int idx = tid; idx < NP * CHUNKS; idx += 256) {
      const int n = idx / CHUNKS, ch = idx % CHUNKS;
      const uint4 v = *reinterpret_cast<const uint4*>(Bt + (int64_t)n * Kp + k0 + ch * (16 / sizeof(T)));
      *reinterpret_cast<uint4*>(&Bs[n * LDK + ch * (16 / sizeof(T))]) = v;
    }
    __syncthreads();
    if constexpr (sizeof(T) == 2) {
      bf16x8 a[MI];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * RW + i * 16 + lane % 16) * LDK + (lane / 16) * 8]);
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        const bf16x8 b =
            *reinterpret_cast<const bf16x8*>(&Bs[(wn * CW + j * 16 + lane % 16) * LDK + (lane / 16) * 8]);
#pragma unroll
        for (int i = 0; i < MI; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) a[i] = As[(wm * RW + i * 16 + lane % 16) * LDK + kk + lane / 16];
#pragma unroll
        for (int j = 0; j < NI; ++j) {
          const float b = Bs[(wn * CW + j * 16 + lane % 16) * LDK + kk + lane / 16];
#pragma unroll
          for (int i = 0; i < MI; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  const int64_t rb = r0 + wm * RW;
  const int cb = wn * CW;
  switch (ep.mode) {
    case E_STORE: store_tiles<E_STORE>(ep, acc, rb, cb, lane, nrows); break;
    case E_STORE_X0: store_tiles<E_STORE_X0>(ep, acc, rb, cb, lane, nrows); break;
    case E_RESIDUAL: store_tiles<E_RESIDUAL>(ep, acc, rb, cb, lane, nrows); break;
    case E_LATENT_BWD: store_tiles<E_LATENT_BWD>(ep, acc, rb, cb, lane, nrows); break;
    default: store_tiles<E_ADD>(ep, acc, rb, cb, lane, nrows); break;
  }
}

}  // namespace nq
