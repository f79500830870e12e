// Column-stationary channel mixing on the matrix cores for the l <= 2,
// 32-channel model (the benchmark shape).
//
// The mixing of layer t is, for each output order l3, a small product
//   forward: V[e][l3 m][c'] = sum_{p in l3, c} T[e][p][m][c] W_l3[(p, c)][c']
//   adjoint: gT[e][p][m][c] = sum_{c'} gV[e][l3 m][c'] W_l3[(p, c)][c']
// with rows (edge, m). The weights never change, so every wavefront owns a
// fixed set of 16-column output tiles and keeps their B fragments in registers
// for the whole (persistent) kernel; per edge group only the A fragments are
// read from LDS. The assignment balances matrix-core work over the 4 waves:
// forward tiles (l3, c' half) weighted by row tiles x K steps, adjoint tiles
// (l3, 16 columns of (p, c)) weighted by row tiles.
#pragma once

#include "gemm.hpp"

namespace nq {
namespace mix32 {

constexpr int C = 32, CP = C + 4, EPB = 256 / C, NT = 35, NY = 9;
constexpr int NP[3] = {3, 4, 4};          // coupling paths per l3 (l <= 2)
constexpr int TOFF[3][4] = {{0, 12, 29, -1}, {1, 9, 18, 26}, {4, 13, 21, 30}};  // T offsets per (l3, path)
constexpr int MOFF[3] = {0, 3, 7};        // mixing block offsets in units of C*C
constexpr int RT[3] = {1, 2, 3};          // 16-row tiles of EPB * (2 l3 + 1) rows

struct Tile {
  int l3, ct;
};
// forward: column tiles (l3, c' half); adjoint: column tiles (l3, 16 of P_l3*C)
constexpr Tile kFwd[4][2] = {{{2, 0}, {-1, 0}}, {{2, 1}, {-1, 0}}, {{1, 0}, {0, 0}}, {{1, 1}, {0, 1}}};
constexpr int kFwdN[4] = {1, 1, 2, 2};
constexpr Tile kBwd[4][8] = {{{2, 0}, {2, 1}, {2, 2}, {2, 3}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}},
                             {{2, 4}, {2, 5}, {2, 6}, {2, 7}, {-1, 0}, {-1, 0}, {-1, 0}, {-1, 0}},
                             {{1, 0}, {1, 1}, {1, 2}, {1, 3}, {1, 4}, {1, 5}, {-1, 0}, {-1, 0}},
                             {{1, 6}, {1, 7}, {0, 0}, {0, 1}, {0, 2}, {0, 3}, {0, 4}, {0, 5}}};
constexpr int kBwdN[4] = {4, 4, 6, 8};

// One B fragment: this lane's share of a 32-deep slice of a 16-column tile.
template <int KIND> struct Frag;
template <> struct Frag<G_F32> {
  float b[8];  // k = 4 j + lane/16, j = 0..7
};
template <> struct Frag<G_BF16> {
  bf16x8 hi;
};
template <> struct Frag<G_BF16X3> {
  bf16x8 hi, lo;
};

// Loads the fragment of column n (this lane), K offset k0, from a row-major
// [n][K] weight block (K contiguous).
template <int KIND>
__device__ inline void load_frag(Frag<KIND>& f, const void* base, int64_t lo_off, int64_t row_off, int k0,
                                 int lane) {
  if constexpr (KIND == G_F32) {
    const float* p = static_cast<const float*>(base) + row_off + k0 + (lane >> 4);
#pragma unroll
    for (int j = 0; j < 8; ++j) f.b[j] = p[4 * j];
  } else {
    const bf16* p = static_cast<const bf16*>(base) + row_off + k0 + (lane >> 4) * 8;
    f.hi = *reinterpret_cast<const bf16x8*>(p);
    if constexpr (KIND == G_BF16X3) f.lo = *reinterpret_cast<const bf16x8*>(p + lo_off);
  }
}

// A fragment: this lane's row of a 32-deep slice (F32: values 4 j + lane/16;
// BF16: values 8 (lane/16) .. +8, split into hi and lo for BF16X3).
template <int KIND> struct AFrag;
template <> struct AFrag<G_F32> {
  float v[8];
};
template <> struct AFrag<G_BF16> {
  bf16x8 h;
};
template <> struct AFrag<G_BF16X3> {
  bf16x8 h, l;
};

// `a` points at the 32 consecutive K values of this lane's row; an invalid row
// gives zeros.
template <int KIND>
__device__ inline AFrag<KIND> load_a(const float* a, bool valid, int lane) {
  AFrag<KIND> A;
  if constexpr (KIND == G_F32) {
#pragma unroll
    for (int j = 0; j < 8; ++j) A.v[j] = valid ? a[4 * j + (lane >> 4)] : 0.f;
  } else {
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (valid) {
      *reinterpret_cast<float4*>(&v[0]) = *reinterpret_cast<const float4*>(a + (lane >> 4) * 8);
      *reinterpret_cast<float4*>(&v[4]) = *reinterpret_cast<const float4*>(a + (lane >> 4) * 8 + 4);
    }
    if constexpr (KIND == G_BF16) {
#pragma unroll
      for (int k = 0; k < 8; ++k) A.h[k] = (bf16)v[k];
    } else {
      split_bf16(v, A.h, A.l);
    }
  }
  return A;
}

// acc += A x B for one 32-deep slice.
template <int KIND>
__device__ inline floatx4 mma_frag(floatx4 acc, const AFrag<KIND>& A, const Frag<KIND>& f) {
  if constexpr (KIND == G_F32) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.v[j], f.b[j], acc, 0, 0, 0);
  } else if constexpr (KIND == G_BF16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, f.hi, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.l, f.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, f.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, f.hi, acc, 0, 0, 0);
  }
  return acc;
}

template <int KIND>
__device__ inline floatx4 mma32(floatx4 acc, const float* a, bool valid, const Frag<KIND>& f, int lane) {
  return mma_frag<KIND>(acc, load_a<KIND>(a, valid, lane), f);
}

// Forward B fragments of wave W: for each owned tile (l3, ct) and K slice ks,
// column c' = 16 ct + lane % 16 of the transposed block [c'][(p, c)].
template <int KIND, int W>
struct FwdB {
  static constexpr int NF = 8;  // up to 2 tiles x 4 slices
  Frag<KIND> f[NF];
  __device__ inline void load(const void* wT, int64_t lo_off, int lane) {
#pragma unroll
    for (int j = 0; j < kFwdN[W]; ++j) {
      const int l3 = kFwd[W][j].l3, ct = kFwd[W][j].ct;
      const int K = NP[l3] * C;
      const int64_t row = (int64_t)MOFF[l3] * C * C + (int64_t)(16 * ct + (lane & 15)) * K;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        if (ks * 32 < K) load_frag<KIND>(f[j * 4 + ks], wT, lo_off, row, ks * 32, lane);
    }
  }
};

template <int KIND, int W>
struct BwdB {
  static constexpr int NF = 8;
  Frag<KIND> f[NF];
  __device__ inline void load(const void* wN, int64_t lo_off, int lane) {
#pragma unroll
    for (int j = 0; j < kBwdN[W]; ++j) {
      const int l3 = kBwd[W][j].l3, ct = kBwd[W][j].ct;
      const int64_t row = (int64_t)MOFF[l3] * C * C + (int64_t)(16 * ct + (lane & 15)) * C;
      load_frag<KIND>(f[j], wN, lo_off, row, 0, lane);
    }
  }
};

// Forward mixing of one group of EPB edges (rows (edge, m)) from T in LDS
// ([edge][NT][CP]) straight to V_t in HBM, through a buffer over the group's
// rows below ne (stores past them are dropped: no branches around them).
template <int KIND, int W>
__device__ inline void mix_fwd(const FwdB<KIND, W>& B, const float* Tl, int64_t e0, int64_t ne,
                               float* __restrict__ vout, int lane) {
  const __amdgpu_buffer_rsrc_t VR = buffer_rsrc(vout + e0 * NY * C, (ne - e0 < EPB ? ne - e0 : EPB) * NY * C * 4);
#pragma unroll
  for (int j = 0; j < kFwdN[W]; ++j) {
    const int l3 = kFwd[W][j].l3, ct = kFwd[W][j].ct, nm = 2 * l3 + 1, R = EPB * nm;
    const int n = 16 * ct + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT[l3]; ++rt) {
      const int r = rt * 16 + (lane & 15);
      const bool rv = r < R;
      const int el = rv ? r / nm : 0, m = rv ? r % nm : 0;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        if (ks >= NP[l3]) continue;  // 32-deep slice ks covers path p = ks
        const float* a = Tl + (el * NT + TOFF[l3][ks] + m) * CP;
        acc = mma32<KIND>(acc, a, rv, B.f[j * 4 + ks], lane);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = rt * 16 + 4 * (lane >> 4) + q;
        const unsigned off = rr < R ? (unsigned)(((rr / nm) * NY + l3 * l3 + rr % nm) * C + n) * 4 : kOutOfRange;
        buf_store(acc[q], VR, off);
      }
    }
  }
}

// mix_fwd from T already split into BF16 in LDS: hi rows [edge][NT][CPH]
// (CPH = C + 8 values) and, for BF16X3, lo rows tlo values further. The
// fragments are the same values load_a would split, so the products are too.
template <int KIND, int W>
__device__ inline void mix_fwd_split(const FwdB<KIND, W>& B, const bf16* Th, int tlo, int64_t e0, int64_t ne,
                                     float* __restrict__ vout, int lane) {
  static_assert(KIND == G_BF16 || KIND == G_BF16X3, "BF16 kinds only");
  constexpr int CPH = C + 8;
  const __amdgpu_buffer_rsrc_t VR = buffer_rsrc(vout + e0 * NY * C, (ne - e0 < EPB ? ne - e0 : EPB) * NY * C * 4);
#pragma unroll
  for (int j = 0; j < kFwdN[W]; ++j) {
    const int l3 = kFwd[W][j].l3, ct = kFwd[W][j].ct, nm = 2 * l3 + 1, R = EPB * nm;
    const int n = 16 * ct + (lane & 15);
#pragma unroll
    for (int rt = 0; rt < RT[l3]; ++rt) {
      const int r = rt * 16 + (lane & 15);
      const bool rv = r < R;
      const int el = rv ? r / nm : 0, m = rv ? r % nm : 0;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        if (ks >= NP[l3]) continue;  // 32-deep slice ks covers path p = ks
        const bf16* h = Th + (el * NT + TOFF[l3][ks] + m) * CPH + (lane >> 4) * 8;
        AFrag<KIND> A;
        bf16x8 z;
#pragma unroll
        for (int k = 0; k < 8; ++k) z[k] = (bf16)0.f;
        A.h = rv ? *reinterpret_cast<const bf16x8*>(h) : z;
        if constexpr (KIND == G_BF16X3) A.l = rv ? *reinterpret_cast<const bf16x8*>(h + tlo) : z;
        acc = mma_frag<KIND>(acc, A, B.f[j * 4 + ks]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = rt * 16 + 4 * (lane >> 4) + q;
        const unsigned off = rr < R ? (unsigned)(((rr / nm) * NY + l3 * l3 + rr % nm) * C + n) * 4 : kOutOfRange;
        buf_store(acc[q], VR, off);
      }
    }
  }
}

constexpr bool bwd_has(int W, int l3) {
  for (int j = 0; j < kBwdN[W]; ++j)
    if (kBwd[W][j].l3 == l3) return true;
  return false;
}

// Adjoint mixing of one group: gV in LDS ([edge][NY][CP]) -> gT in LDS. The
// wave's column tiles of one l3 share their A fragments (rows (edge, m) of
// dE/dV), so each row tile's fragment is loaded and split once.
template <int KIND, int W>
__device__ inline void mix_bwd(const BwdB<KIND, W>& B, const float* gVl, float* gTl, int lane) {
#pragma unroll
  for (int l3 = 2; l3 >= 0; --l3) {
    if (!bwd_has(W, l3)) continue;
    const int nm = 2 * l3 + 1, R = EPB * nm;
#pragma unroll
    for (int rt = 0; rt < RT[l3]; ++rt) {
      const int r = rt * 16 + (lane & 15);
      const bool rv = r < R;
      const int el = rv ? r / nm : 0, m = rv ? r % nm : 0;
      const AFrag<KIND> A = load_a<KIND>(gVl + (el * NY + l3 * l3 + m) * CP, rv, lane);
      int dst[4];  // LDS row offsets of this lane's four output rows (-1: past the group)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = rt * 16 + 4 * (lane >> 4) + q;
        dst[q] = rr < R ? ((rr / nm) * NT + rr % nm) * CP : -1;
      }
#pragma unroll
      for (int j = 0; j < kBwdN[W]; ++j) {
        if (kBwd[W][j].l3 != l3) continue;
        const int n = 16 * kBwd[W][j].ct + (lane & 15), p = n / C, c = n % C;
        const floatx4 acc = mma_frag<KIND>(floatx4{0.f, 0.f, 0.f, 0.f}, A, B.f[j]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (dst[q] >= 0) gTl[dst[q] + TOFF[l3][p] * CP + c] = acc[q];
      }
    }
  }
}

// mix_bwd from dE/dV already split into BF16 in LDS: hi rows [edge][NY][CPH]
// (CPH = C + 8 values) and, for BF16X3, lo rows glo values further. The
// fragments are the same values load_a would split, so the products are too.
template <int KIND, int W>
__device__ inline void mix_bwd_split(const BwdB<KIND, W>& B, const bf16* gVh, int glo, float* gTl, int lane) {
  static_assert(KIND == G_BF16 || KIND == G_BF16X3, "BF16 kinds only");
  constexpr int CPH = C + 8;
#pragma unroll
  for (int l3 = 2; l3 >= 0; --l3) {
    if (!bwd_has(W, l3)) continue;
    const int nm = 2 * l3 + 1, R = EPB * nm;
#pragma unroll
    for (int rt = 0; rt < RT[l3]; ++rt) {
      const int r = rt * 16 + (lane & 15);
      const bool rv = r < R;
      const int el = rv ? r / nm : 0, m = rv ? r % nm : 0;
      const bf16* h = gVh + (el * NY + l3 * l3 + m) * CPH + (lane >> 4) * 8;
      AFrag<KIND> A;
      bf16x8 z;
#pragma unroll
      for (int k = 0; k < 8; ++k) z[k] = (bf16)0.f;
      A.h = rv ? *reinterpret_cast<const bf16x8*>(h) : z;
      if constexpr (KIND == G_BF16X3) A.l = rv ? *reinterpret_cast<const bf16x8*>(h + glo) : z;
      int dst[4];  // LDS row offsets of this lane's four output rows (-1: past the group)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = rt * 16 + 4 * (lane >> 4) + q;
        dst[q] = rr < R ? ((rr / nm) * NT + rr % nm) * CP : -1;
      }
#pragma unroll
      for (int j = 0; j < kBwdN[W]; ++j) {
        if (kBwd[W][j].l3 != l3) continue;
        const int n = 16 * kBwd[W][j].ct + (lane & 15), p = n / C, c = n % C;
        const floatx4 acc = mma_frag<KIND>(floatx4{0.f, 0.f, 0.f, 0.f}, A, B.f[j]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (dst[q] >= 0) gTl[dst[q] + TOFF[l3][p] * CP + c] = acc[q];
      }
    }
  }
}

}  // namespace mix32
}  // namespace nq
