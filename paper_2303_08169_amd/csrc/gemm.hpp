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

// Logistic function with the hardware reciprocal (1 ulp) instead of an IEEE
// division, which expands to about ten instructions per call.
__device__ inline float sigmoidf_(float a) { return __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }
__device__ inline float siluf(float a) { return a * sigmoidf_(a); }
__device__ inline float dsiluf(float a) {
  float s = sigmoidf_(a);
  return s * (1.0f + a * (1.0f - s));
}

constexpr float kInvSqrt2 = 0.70710678118654752f;

// Element operations shared by the product kernels, written with explicit
// fused multiply-adds so that every kernel rounds them the same way (the
// compiler would otherwise contract them differently in different contexts).
// Adjoint of SiLU scaled by f: g f SiLU'(a), with s = sigmoid(a).
__device__ inline float gradsilu_scale(float g, float a, float s, float f) {
  return g * (f * s * __builtin_fmaf(a, 1.f - s, 1.f));
}
// Row-scale derivative share of four values: sum g SiLU(a).
__device__ inline float gradsilu_part(const float4& g, const float4& a, float sx, float sy, float sz, float sw) {
  float p = (g.x * a.x) * sx;
  p = __builtin_fmaf(g.y * a.y, sy, p);
  p = __builtin_fmaf(g.z * a.z, sz, p);
  return __builtin_fmaf(g.w * a.w, sw, p);
}
// Residual update (x + u SiLU(y)) / sqrt 2 and its adjoint g / sqrt 2 + y.
__device__ inline float residual_update(float x, float u, float y) { return __builtin_fmaf(u, siluf(y), x) * kInvSqrt2; }
__device__ inline float residual_adjoint(float g, float y) { return __builtin_fmaf(g, kInvSqrt2, y); }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// A_SILU_U: u SiLU(a) with u the row scale, i.e. the two-body output x0
// formed at use from its stored pre-activation; A_CAT_SILU_U: [u SiLU(a) | s].
enum ALoadMode { A_PLAIN = 0, A_SILU = 1, A_CAT = 2, A_GRADSILU = 3, A_SILU_U = 4, A_CAT_SILU_U = 5 };

// Raw loads of four consecutive A values of one row, kept in registers until
// the tile is written to LDS (a K step later), so the loads stay in flight
// while the matrix cores work.
struct ARaw {
  float4 v, a;  // source values; the stored pre-activation (A_GRADSILU)
  float f;      // row scale (A_GRADSILU)
};

struct ALoad {
  int mode;
  const float* p0; int ld0; int K0;  // primary source
  const float* p1; int ld1; int K1;  // concatenated source, or the pre-activation for A_GRADSILU
  const float* rs; int rs_ld;        // optional per-row scale (the cutoff u)
  float c;                           // constant factor (A_GRADSILU)
  float* gu;                         // A_GRADSILU, optional: gu[r] += c * sum_k g[r][k] SiLU(a[r][k])
  // Issues the loads of columns k..k+3 of row r (k % 4 == 0; widths and
  // leading dimensions are multiples of 4, so each access is one aligned
  // 16-byte load). r must be a valid row; a column beyond the source width
  // reads column 0 and is zeroed by finish(). Only uniform branches, so the
  // loads of several K steps can be in flight together.
  __device__ inline void fetch(int64_t r, int k, ARaw& o) const {
    if (mode == A_CAT || mode == A_CAT_SILU_U) {
      const bool second = k >= K0;
      const int k1 = k - K0 < K1 ? k - K0 : 0;
      const float* p = second ? p1 + r * ld1 + k1 : p0 + r * ld0 + k;
      o.v = *reinterpret_cast<const float4*>(p);
      if (mode == A_CAT_SILU_U) o.f = rs[r * rs_ld];
    } else {
      const int kk = k < K0 ? k : 0;
      o.v = *reinterpret_cast<const float4*>(p0 + r * ld0 + kk);
      if (mode == A_GRADSILU) {
        o.a = *reinterpret_cast<const float4*>(p1 + r * ld1 + kk);
        o.f = rs ? rs[r * rs_ld] : 1.f;
      } else if (mode == A_SILU_U) {
        o.f = rs[r * rs_ld];
      }
    }
  }
  // The A values from the raw loads: zero outside the rows or columns,
  // SiLU, or the adjoint g * c * rowscale * SiLU'(a).
  // With gu set, rd accumulates this chunk's share of sum_k g SiLU(a), the
  // derivative with respect to the row scale, from the same loaded values.
  __device__ inline float4 finish(const ARaw& o, bool row_ok, int k, float& rd) const {
    const bool ok = row_ok && k < ((mode == A_CAT || mode == A_CAT_SILU_U) ? K0 + K1 : K0);
    float4 v = o.v;
    if (mode == A_SILU) {
      v.x = siluf(v.x);
      v.y = siluf(v.y);
      v.z = siluf(v.z);
      v.w = siluf(v.w);
    } else if (mode == A_SILU_U || (mode == A_CAT_SILU_U && k < K0)) {
      v.x = o.f * siluf(v.x);
      v.y = o.f * siluf(v.y);
      v.z = o.f * siluf(v.z);
      v.w = o.f * siluf(v.w);
    } else if (mode == A_GRADSILU) {
      const float f = c * o.f;
      const float sx = sigmoidf_(o.a.x), sy = sigmoidf_(o.a.y), sz = sigmoidf_(o.a.z), sw = sigmoidf_(o.a.w);
      if (gu) {
        const float part = gradsilu_part(v, o.a, sx, sy, sz, sw);
        rd += ok ? part : 0.f;
      }
      v.x = gradsilu_scale(v.x, o.a.x, sx, f);
      v.y = gradsilu_scale(v.y, o.a.y, sy, f);
      v.z = gradsilu_scale(v.z, o.a.z, sz, f);
      v.w = gradsilu_scale(v.w, o.a.w, sw, f);
    }
    return ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
  }
};

// The dE/du row sum of a 256-wide A row whose 64 four-value chunks are held
// one per lane of a wavefront (lane l: chunk l = 8 s + j, K step s, position
// j in it): per position the shares of K steps 0..7 in order, then the 8
// positions pairwise; every product kernel adds in this order. Done with
// cross-lane register moves (DPP row shifts and quad permutes, row and half
// swaps) instead of LDS round trips; the result is in lane 0.
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ inline float row_share_sum(float x) {
  constexpr int kShl8 = 0x108, kShl4 = 0x104, kSwap1 = 0xB1, kSwap2 = 0x4E;  // row_shl:8, row_shl:4, quad_perm
  const unsigned xi = __float_as_uint(x);
  // y: lane j holds the share of lane j + 16; z: of lane j + 32; w: of lane j + 48
  const float y = __uint_as_float(__builtin_amdgcn_permlane16_swap(xi, xi, false, false)[1]);
  const unsigned zi = __builtin_amdgcn_permlane32_swap(xi, xi, false, false)[1];
  const float z = __uint_as_float(zi);
  const float w = __uint_as_float(__builtin_amdgcn_permlane16_swap(zi, zi, false, false)[1]);
  float s = 0.f + x;
  s += dpp_f<kShl8>(x);
  s += y;
  s += dpp_f<kShl8>(y);
  s += z;
  s += dpp_f<kShl8>(z);
  s += w;
  s += dpp_f<kShl8>(w);
  s += dpp_f<kSwap1>(s);
  s += dpp_f<kSwap2>(s);
  s += dpp_f<kShl4>(s);
  return s;
}

enum EpiMode { E_STORE = 0, E_STORE_X0 = 1, E_RESIDUAL = 2, E_LATENT_BWD = 3, E_ADD = 4 };

struct Epi {
  int mode;
  float* o0; int ld0; int N0;
  float* o1; int ld1;
  const float* x; int ldx;
  const float* rs; int rs_ld;
  int D;
  int xsilu;  // E_RESIDUAL: x holds a pre-activation; the residual input is u SiLU(x)
};

// Writes the accumulator tiles of one wavefront through epilogue mode MODE.
// Lane l holds rows 4*(l/16)+q, column l%16 of every 16x16 tile. The values
// an epilogue reads (which may alias what it writes) are loaded for a block
// of up to 4 tiles before any of its stores, with indices clamped into range,
// so those loads are in flight together; only the stores are guarded.
template <int MODE, int MI, int NI>
__device__ inline void store_tiles(const Epi& ep, const floatx4 (&acc)[MI][NI], int64_t rbase, int cbase,
                                   int lane, int64_t nrows) {
  constexpr bool kRS = MODE == E_STORE_X0 || MODE == E_RESIDUAL;
  constexpr bool kIN = MODE == E_RESIDUAL || MODE == E_LATENT_BWD || MODE == E_ADD;
  constexpr int JC = NI < 4 ? NI : 4;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    // row base addresses, once per row (64-bit), column offsets 32-bit
    int64_t rr[4];
    bool rok[4];
    float rsv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = rbase + i * 16 + (lane / 16) * 4 + q;
      rok[q] = r < nrows;
      rr[q] = rok[q] ? r : nrows - 1;
      if constexpr (kRS) rsv[q] = ep.rs[rr[q] * ep.rs_ld];
    }
#pragma unroll
    for (int j0 = 0; j0 < NI; j0 += JC) {
      float in[JC][4];
      if constexpr (kIN) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float* src = MODE == E_RESIDUAL ? ep.x + rr[q] * ep.ldx : ep.o0 + rr[q] * ep.ld0;
#pragma unroll
          for (int jj = 0; jj < JC; ++jj) {
            if (j0 + jj >= NI) continue;
            const int c = cbase + (j0 + jj) * 16 + lane % 16;
            int cc = c < ep.N0 ? c : 0;
            if constexpr (MODE == E_LATENT_BWD) cc = cc < ep.D ? cc : 0;
            in[jj][q] = src[cc];
            if (MODE == E_RESIDUAL && ep.xsilu) in[jj][q] = rsv[q] * siluf(in[jj][q]);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!rok[q]) continue;
        float* o0 = ep.o0 + rr[q] * ep.ld0;
        float* o1 = (MODE == E_STORE_X0 || MODE == E_RESIDUAL || MODE == E_LATENT_BWD) ? ep.o1 + rr[q] * ep.ld1
                                                                                          : nullptr;
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
          const int j = j0 + jj;
          if (j >= NI) continue;
          const int c = cbase + j * 16 + lane % 16;
          if (c >= ep.N0) continue;
          const float v = acc[i][j][q];
          if constexpr (MODE == E_STORE) {
            o0[c] = v;
          } else if constexpr (MODE == E_STORE_X0) {
            o0[c] = v;
            o1[c] = rsv[q] * siluf(v);
          } else if constexpr (MODE == E_RESIDUAL) {
            o0[c] = v;
            o1[c] = residual_update(in[jj][q], rsv[q], v);
          } else if constexpr (MODE == E_LATENT_BWD) {
            if (c < ep.D)
              o0[c] = residual_adjoint(in[jj][q], v);
            else
              o1[c - ep.D] = v;
          } else {
            o0[c] = in[jj][q] + v;
          }
        }
      }
    }
  }
}

// Kinds of matrix-core product.
enum GemmKind { G_F32 = 0, G_BF16 = 1, G_BF16X3 = 2 };

template <int KIND> struct GemmTraits;
template <> struct GemmTraits<G_F32> {  // A, B: f32 in LDS; v_mfma_f32_16x16x4_f32
  typedef float AT;
  typedef float BT;
  static constexpr int BK = 16, LDA = 20, LDB = 20, BHALVES = 1;
};
template <> struct GemmTraits<G_BF16> {  // A, B: bf16 in LDS; v_mfma_f32_16x16x32_bf16
  typedef bf16 AT;
  typedef bf16 BT;
  static constexpr int BK = 32, LDA = 40, LDB = 40, BHALVES = 1;
};
template <> struct GemmTraits<G_BF16X3> {  // A: f32 in LDS split on load; B: bf16 hi and lo
  typedef float AT;
  typedef bf16 BT;
  static constexpr int BK = 32, LDA = 36, LDB = 40, BHALVES = 2;
};

__device__ inline void split_bf16(const float* v, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bf16 h = (bf16)v[k];
    hi[k] = h;
    lo[k] = (bf16)(v[k] - (float)h);
  }
}

// C[rows, NP] = A[rows, Kp] * Bt[NP, Kp]^T.  4 wavefronts as WM x WN.
// For BF16X3, Bt holds two [NP][Kp] halves (hi, lo) and the product is
// A_hi B_hi + A_lo B_hi + A_hi B_lo. The loads of the next K step's A and B
// tiles are issued right after the barrier and consumed only after the
// current step's matrix-core work (raw values in registers, transformed when
// written to LDS), so HBM and L2 latency overlap the products.
template <int KIND, int BM, int NP, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm(int Kp, const typename GemmTraits<KIND>::BT* __restrict__ Bt,
                                              const int* __restrict__ nrows_p, ALoad ld, Epi ep) {
  typedef GemmTraits<KIND> Tr;
  typedef typename Tr::AT AT;
  typedef typename Tr::BT BT;
  constexpr int BK = Tr::BK, LDA = Tr::LDA, LDB = Tr::LDB;
  constexpr int RW = BM / WM;  // rows per wave
  constexpr int CW = NP / WN;  // cols per wave
  constexpr int MI = RW / 16;
  constexpr int NI = CW / 16;
  constexpr int A4 = BM * BK / 4;                      // float4 chunks of one A tile
  constexpr int NA = (A4 + 255) / 256;                 // ... per thread
  constexpr int CPR = BK * (int)sizeof(BT) / 16;       // 16-byte chunks per B row
  constexpr int EPC = 16 / (int)sizeof(BT);            // elements per chunk
  constexpr int B16 = Tr::BHALVES * NP * CPR;          // chunks of one B tile
  constexpr int NB = (B16 + 255) / 256;
  static_assert(WM * WN == 4, "4 wavefronts");
  static_assert(RW % 16 == 0 && CW % 16 == 0, "16x16 tiles");
  // BF16 weight rows (32 values, four 16-byte chunks) are stored unpadded with
  // the chunk index XORed by (row / 4) % 4, which keeps both the 16-byte
  // fragment reads of 16 consecutive rows and the tile stores free of bank
  // conflicts; FP32 rows keep a padded stride.
  constexpr bool SWZ = sizeof(BT) == 2;
  constexpr int LDBS = SWZ ? BK : LDB;
  constexpr int ABUF = BM * LDA, BBUF = Tr::BHALVES * NP * LDBS;
  __shared__ __attribute__((aligned(16))) AT As[ABUF];
  __shared__ __attribute__((aligned(16))) BT Bs[BBUF];

  const int64_t nrows = *nrows_p;
  const int64_t r0 = (int64_t)blockIdx.x * BM;
  if (r0 >= nrows) return;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t half = (int64_t)NP * Kp;
  const int nsteps = Kp / BK;

  floatx4 acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  ARaw ra[NA];
  u32x4 rb[NB];
  float rd[NA];  // row-scale derivative partial sums (ld.gu)
#pragma unroll
  for (int q = 0; q < NA; ++q) rd[q] = 0.f;
#define NQ_GEMM_FETCH_A(K0)                                                                        \
  {                                                                                               \
    _Pragma("unroll") for (int q = 0; q < NA; ++q) {                                              \
      const int idx = (tid + 256 * q) % A4;                                                       \
      const int rr = idx / (BK / 4), kk = (idx % (BK / 4)) * 4;                                   \
      const int64_t row = r0 + rr < nrows ? r0 + rr : nrows - 1;                                  \
      ld.fetch(row, (K0) + kk, ra[q]);                                                            \
    }                                                                                             \
  }
#define NQ_GEMM_FETCH_B(K0)                                                                        \
  {                                                                                               \
    _Pragma("unroll") for (int q = 0; q < NB; ++q) {                                              \
      const int idx = tid + 256 * q;                                                              \
      if (idx < B16) {                                                                            \
        const int h = idx / (NP * CPR), rem = idx % (NP * CPR);                                   \
        const int n = rem / CPR, ch = rem % CPR;                                                  \
        rb[q] = *reinterpret_cast<const u32x4*>(Bt + h * half + (int64_t)n * Kp + (K0) + ch * EPC); \
      }                                                                                           \
    }                                                                                             \
  }
#define NQ_GEMM_SWZ(N, CH) (SWZ ? ((CH) ^ (((N) >> 2) & (CPR - 1))) : (CH))
  // Writes the fetched tiles of K step ST into LDS.
#define NQ_GEMM_STORE(ST)                                                                         \
  {                                                                                               \
    AT* as_ = As;                                                                                 \
    BT* bs_ = Bs;                                                                                 \
    _Pragma("unroll") for (int q = 0; q < NA; ++q) {                                              \
      const int idx = tid + 256 * q;                                                              \
      if (idx < A4) {                                                                             \
        const int rr = idx / (BK / 4), kk = (idx % (BK / 4)) * 4;                                 \
        const float4 v = ld.finish(ra[q], r0 + rr < nrows, (ST) * BK + kk, rd[q]);               \
        if constexpr (sizeof(AT) == 4) {                                                          \
          *reinterpret_cast<float4*>(&as_[rr * LDA + kk]) = v;                                    \
        } else {                                                                                  \
          typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));                              \
          bf16x4 b4;                                                                              \
          b4[0] = (bf16)v.x;                                                                      \
          b4[1] = (bf16)v.y;                                                                      \
          b4[2] = (bf16)v.z;                                                                      \
          b4[3] = (bf16)v.w;                                                                      \
          *reinterpret_cast<bf16x4*>(&as_[rr * LDA + kk]) = b4;                                   \
        }                                                                                         \
      }                                                                                           \
    }                                                                                             \
    _Pragma("unroll") for (int q = 0; q < NB; ++q) {                                              \
      const int idx = tid + 256 * q;                                                              \
      if (idx < B16) {                                                                            \
        const int h = idx / (NP * CPR), rem = idx % (NP * CPR);                                   \
        const int n = rem / CPR, ch = rem % CPR;                                                  \
        *reinterpret_cast<u32x4*>(&bs_[(h * NP + n) * LDBS + NQ_GEMM_SWZ(n, ch) * EPC]) = rb[q];  \
      }                                                                                           \
    }                                                                                             \
  }
  // Matrix-core products of the tiles in LDS.
#define NQ_GEMM_COMPUTE()                                                                           \
  {                                                                                               \
    const AT* as_ = As;                                                                           \
    const BT* bs_ = Bs;                                                                           \
    if constexpr (KIND == G_BF16) {                                                               \
      bf16x8 a[MI];                                                                               \
      _Pragma("unroll") for (int i = 0; i < MI; ++i) a[i] =                                       \
          *reinterpret_cast<const bf16x8*>(&as_[(wm * RW + i * 16 + lane % 16) * LDA + (lane / 16) * 8]); \
      _Pragma("unroll") for (int j = 0; j < NI; ++j) {                                            \
        const int n = wn * CW + j * 16 + lane % 16;                                               \
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&bs_[n * LDBS + NQ_GEMM_SWZ(n, lane / 16) * 8]); \
        _Pragma("unroll") for (int i = 0; i < MI; ++i) acc[i][j] =                                \
            __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);                 \
      }                                                                                           \
    } else if constexpr (KIND == G_BF16X3) {                                                      \
      bf16x8 ahi[MI], alo[MI];                                                                    \
      _Pragma("unroll") for (int i = 0; i < MI; ++i) {                                            \
        const float* src = &as_[(wm * RW + i * 16 + lane % 16) * LDA + (lane / 16) * 8];          \
        float v[8];                                                                               \
        *reinterpret_cast<float4*>(&v[0]) = *reinterpret_cast<const float4*>(src);                \
        *reinterpret_cast<float4*>(&v[4]) = *reinterpret_cast<const float4*>(src + 4);            \
        split_bf16(v, ahi[i], alo[i]);                                                            \
      }                                                                                           \
      _Pragma("unroll") for (int j = 0; j < NI; ++j) {                                            \
        const int n = wn * CW + j * 16 + lane % 16;                                               \
        const int nb = n * LDBS + NQ_GEMM_SWZ(n, lane / 16) * 8;                                  \
        const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(&bs_[nb]);                            \
        const bf16x8 blo = *reinterpret_cast<const bf16x8*>(&bs_[NP * LDBS + nb]);                \
        _Pragma("unroll") for (int i = 0; i < MI; ++i) {                                          \
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[i], bhi, acc[i][j], 0, 0, 0);   \
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], blo, acc[i][j], 0, 0, 0);   \
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi[i], bhi, acc[i][j], 0, 0, 0);   \
        }                                                                                         \
      }                                                                                           \
    } else {                                                                                      \
      _Pragma("unroll") for (int kk = 0; kk < BK; kk += 4) {                                      \
        float a[MI];                                                                              \
        _Pragma("unroll") for (int i = 0; i < MI; ++i) a[i] =                                     \
            as_[(wm * RW + i * 16 + lane % 16) * LDA + kk + lane / 16];                           \
        _Pragma("unroll") for (int j = 0; j < NI; ++j) {                                          \
          const float b = bs_[(wn * CW + j * 16 + lane % 16) * LDBS + kk + lane / 16];            \
          _Pragma("unroll") for (int i = 0; i < MI; ++i) acc[i][j] =                              \
              __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b, acc[i][j], 0, 0, 0);                  \
        }                                                                                         \
      }                                                                                           \
    }                                                                                             \
  }
  NQ_GEMM_FETCH_A(0);
  NQ_GEMM_FETCH_B(0);
  // store, barrier, fetch the next step, products, barrier (a second LDS
  // buffer with one barrier per step was measured no faster: it halves the
  // workgroups resident per CU)
  for (int st = 0; st < nsteps; ++st) {
    NQ_GEMM_STORE(st);
    __syncthreads();
    if (st + 1 < nsteps) {
      NQ_GEMM_FETCH_A((st + 1) * BK);
      NQ_GEMM_FETCH_B((st + 1) * BK);
    }
    NQ_GEMM_COMPUTE();
    __syncthreads();
  }
#undef NQ_GEMM_STORE
#undef NQ_GEMM_COMPUTE
#undef NQ_GEMM_SWZ
#undef NQ_GEMM_FETCH_A
#undef NQ_GEMM_FETCH_B
  if (ld.gu) {
    // the BK / 4 lanes that loaded one row are consecutive
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      float r = rd[q];
#pragma unroll
      for (int o = 1; o < BK / 4; o <<= 1) r += __shfl_xor(r, o);
      const int idx = tid + 256 * q;
      if (idx < A4 && idx % (BK / 4) == 0) {
        const int64_t row = r0 + idx / (BK / 4);
        if (row < nrows) ld.gu[row] += ld.c * r;
      }
    }
  }
  const int64_t rbase = r0 + wm * RW;
  const int cbase = wn * CW;
  switch (ep.mode) {
    case E_STORE: store_tiles<E_STORE>(ep, acc, rbase, cbase, lane, nrows); break;
    case E_STORE_X0: store_tiles<E_STORE_X0>(ep, acc, rbase, cbase, lane, nrows); break;
    case E_RESIDUAL: store_tiles<E_RESIDUAL>(ep, acc, rbase, cbase, lane, nrows); break;
    case E_LATENT_BWD: store_tiles<E_LATENT_BWD>(ep, acc, rbase, cbase, lane, nrows); break;
    default: store_tiles<E_ADD>(ep, acc, rbase, cbase, lane, nrows); break;
  }
}

// Raw buffer resource over [base, base + bytes): loads beyond it return 0 and
// stores beyond it are dropped by the hardware, which lets a kernel guard
// its memory operations by offset instead of by branches.
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr unsigned kOutOfRange = 0x80000000u;
// 32-bit buffer load / store of a float at a byte offset (the builtins move
// raw 32-bit words).
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// Weight-stationary persistent variant for the BF16 kinds. One workgroup of
// 8 wavefronts per CU keeps the whole weight matrix in registers as
// matrix-core B fragments (wavefront w owns the NTW 16-column output tiles
// starting at column 16 NTW w, for all KS K steps), so no weight tile is
// staged through LDS again; workgroups then loop over 16-row edge tiles. The
// A tile of the next row tile is loaded into registers while the current one
// is multiplied from LDS (two LDS buffers, one barrier per row tile). The A
// tile is split into its BF16 halves once, when written to LDS, instead of by
// every wavefront that reads it. K steps, the split and the product order per
// step are those of k_gemm, so the products are bitwise identical to it.
// Loader and epilogue modes are compile-time, and every global address is a
// per-tile uniform base plus a 32-bit lane offset, which keeps the registers
// beside the weights within budget. The residual update and the latent
// adjoint read their FP32 inputs (x, the first D columns of [x | s]; the raw
// g rows) from a third LDS tile, so those epilogues do no global loads that
// could alias their stores.
// With ld.gu set, Kp must be 256: one wavefront's load then covers one row
// (eight K steps of eight chunks).
template <int KIND, int NTW, int KS, int AMODE, int EMODE, int PF, int EPI>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemm_ws(int NP, const bf16* __restrict__ Bt, const int* __restrict__ nrows_p,
                                                 ALoad ld, Epi ep) {
  static_assert(KIND == G_BF16 || KIND == G_BF16X3, "BF16 kinds only");
  constexpr int H = KIND == G_BF16X3 ? 2 : 1;  // weight halves (hi, lo)
  constexpr int RT = 16;                       // rows per tile
  constexpr int Kp = KS * 32;
  constexpr int LDH = Kp + 8;                  // LDS row stride of the BF16 halves
  constexpr int LDW = Kp + 4;                  // ... of the FP32 copy
  constexpr int CPR = Kp / 4;                  // float4 chunks per row
  constexpr int A4 = RT * CPR;                 // ... per tile
  constexpr int NA = (A4 + 511) / 512;
  constexpr bool GR = AMODE == A_GRADSILU;
  constexpr bool CAT = AMODE == A_CAT || AMODE == A_CAT_SILU_U;
  constexpr bool SU = AMODE == A_SILU_U || AMODE == A_CAT_SILU_U;  // u SiLU(a) of the (first) source
  constexpr bool XIN = EMODE == E_RESIDUAL || EMODE == E_LATENT_BWD;  // FP32 copy of the primary source
  __shared__ __attribute__((aligned(16))) bf16 As[2][H * RT * LDH];
  __shared__ __attribute__((aligned(16))) float Xs[XIN ? 2 : 1][XIN ? RT * LDW : 4];
  constexpr bool RS = EMODE == E_STORE_X0 || EMODE == E_RESIDUAL;  // epilogue row scale, staged too
  __shared__ float Us[2][RT];
  constexpr int LDO = 8 * NTW * 16 + 4;  // products of one row tile, all wavefronts' columns
  constexpr int NE = NTW;                // float4 output chunks per thread (RT * 8 NTW * 16 / 4 / 512)
  __shared__ __attribute__((aligned(16))) float Os[EPI == 1 ? RT * LDO : 4];
  constexpr bool ADD = EMODE == E_ADD && EPI == 1;  // the accumulated rows are staged like A
  constexpr bool GU = GR && KS == 8;  // dE/du row sums (the launcher passes gu only when Kp = 256)
  __shared__ float Rs[GU ? 2 : 1][GU ? RT : 4];  // dE/du row sums of the staged tile
  __shared__ __attribute__((aligned(16))) float Is[ADD ? 2 : 1][ADD ? RT * LDO : 4];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int64_t nrows = *nrows_p;
  const int64_t ntiles = (nrows + RT - 1) / RT;
  const int nt = NP / 16;
  const int my0 = __builtin_amdgcn_readfirstlane(wave * NTW);
  const int my_nt = my0 >= nt ? 0 : (nt - my0 < NTW ? nt - my0 : NTW);

  bf16x8 bw[NTW][KS][H];
#pragma unroll
  for (int j = 0; j < NTW; ++j)
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int h = 0; h < H; ++h) {
        bf16x8 z;
#pragma unroll
        for (int e = 0; e < 8; ++e) z[e] = (bf16)0.f;
        if (j < my_nt)
          z = *reinterpret_cast<const bf16x8*>(Bt + (int64_t)h * NP * Kp + ((my0 + j) * 16 + lane % 16) * Kp + s * 32 +
                                               (lane / 16) * 8);
        bw[j][s][h] = z;
      }

  // staged raw A values of one row tile (chunk q: row idx / CPR, columns
  // 4 (idx % CPR) .. +3 with idx = tid + 512 q)
  struct Stage {
    float4 rv[NA], rg[GR ? NA : 1], in[ADD ? NE : 1];
    float rf[GR || SU ? NA : 1], ru;  // ru: the epilogue row scale, or dE/du of rows (wave + 8 lane) (GR)
  };
  Stage s0, s1;  // s1 is used only with two tiles in flight (PF = 2)
  // dE/du of the rows of a tile (empty without gu)
  auto gu_rsrc = [&](int64_t row0) {
    return buffer_rsrc(ld.gu ? ld.gu + row0 : nullptr, ld.gu ? (nrows - row0 < RT ? nrows - row0 : RT) * 4 : 0);
  };
  auto fetch = [&](int64_t tile, int t, Stage& S) {
    const int64_t row0 = tile * RT;
    const int lim = (int)(nrows - 1 - row0 < RT ? nrows - 1 - row0 : RT - 1);
    const float* b0 = ld.p0 + row0 * ld.ld0;
    const float* b1 = ld.p1 + row0 * ld.ld1;
    // without a row scale the (unused) scale load reads a valid address
    const float* brs = ld.rs ? ld.rs + row0 * ld.rs_ld : ld.p1;
    const int rsl = ld.rs ? ld.rs_ld : 0;
    if constexpr (RS) S.ru = ep.rs[(row0 + (t % RT < lim ? t % RT : lim)) * ep.rs_ld];
    if constexpr (GU) S.ru = buf_load(gu_rsrc(row0), (unsigned)(t % RT) * 4);
    if constexpr (ADD) {
      const int cpr = ep.N0 / 4;
      const float* bo = ep.o0 + row0 * ep.ld0;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int idx = (t + 512 * e) % (RT * cpr);
        const int r = idx / cpr < lim ? idx / cpr : lim;
        S.in[e] = *reinterpret_cast<const float4*>(bo + (unsigned)(r * ep.ld0 + (idx % cpr) * 4));
      }
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int idx = (t + 512 * q) % A4;
      const int r = idx / CPR < lim ? idx / CPR : lim;
      const int k = (idx % CPR) * 4;
      if constexpr (CAT) {
        const float* p = k >= ld.K0 ? b1 + (unsigned)(r * ld.ld1 + (k - ld.K0 < ld.K1 ? k - ld.K0 : 0))
                                    : b0 + (unsigned)(r * ld.ld0 + k);
        S.rv[q] = *reinterpret_cast<const float4*>(p);
        if constexpr (SU) S.rf[q] = brs[(unsigned)(r * rsl)];
      } else {
        const int kk = k < ld.K0 ? k : 0;
        S.rv[q] = *reinterpret_cast<const float4*>(b0 + (unsigned)(r * ld.ld0 + kk));
        if constexpr (GR) {
          S.rg[q] = *reinterpret_cast<const float4*>(b1 + (unsigned)(r * ld.ld1 + kk));
          S.rf[q] = brs[(unsigned)(r * rsl)];
        }
        if constexpr (SU) S.rf[q] = brs[(unsigned)(r * rsl)];
      }
    }
  };
  auto store = [&](int64_t tile, int it1, int t, const Stage& S) {
    bf16* dst = As[it1];
    float* xdst = Xs[XIN ? it1 : 0];
    float* udst = Us[it1];
    const int64_t row0 = tile * RT;
    if ((RS || GU) && t < RT) udst[t] = S.ru;
    if constexpr (ADD) {
      const int cpr = ep.N0 / 4;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int idx = t + 512 * e;
        if (idx < RT * cpr) *reinterpret_cast<float4*>(&Is[it1][(idx / cpr) * LDO + (idx % cpr) * 4]) = S.in[e];
      }
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int idx = t + 512 * q;
      const int i2 = idx % A4, rr = i2 / CPR, k = (i2 % CPR) * 4;
      const bool ok = row0 + rr < nrows && k < (CAT ? ld.K0 + ld.K1 : ld.K0);
      float4 v = S.rv[q];
      // x0 = u SiLU(a) is formed before the FP32 copy (the residual's input)
      if constexpr (SU) {
        if (AMODE == A_SILU_U || k < ld.K0) {
          v.x = S.rf[q] * siluf(v.x);
          v.y = S.rf[q] * siluf(v.y);
          v.z = S.rf[q] * siluf(v.z);
          v.w = S.rf[q] * siluf(v.w);
        }
      }
      if constexpr (XIN)
        if (idx < A4 && k < ld.K0)
          *reinterpret_cast<float4*>(&xdst[rr * LDW + k]) = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
      float rd = 0.f;
      if constexpr (AMODE == A_SILU) {
        v.x = siluf(v.x);
        v.y = siluf(v.y);
        v.z = siluf(v.z);
        v.w = siluf(v.w);
      } else if constexpr (GR) {
        const float4 a = S.rg[q];
        const float f = ld.c * (ld.rs ? S.rf[q] : 1.f);
        const float sx = sigmoidf_(a.x), sy = sigmoidf_(a.y), sz = sigmoidf_(a.z), sw = sigmoidf_(a.w);
        rd = ok ? gradsilu_part(v, a, sx, sy, sz, sw) : 0.f;
        v.x = gradsilu_scale(v.x, a.x, sx, f);
        v.y = gradsilu_scale(v.y, a.y, sy, f);
        v.z = gradsilu_scale(v.z, a.z, sz, f);
        v.w = gradsilu_scale(v.w, a.w, sw, f);
      }
      if (idx < A4) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        const float e[4] = {ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f};
        bf16x4 hi, lo;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          hi[u] = (bf16)e[u];
          lo[u] = (bf16)(e[u] - (float)hi[u]);
        }
        *reinterpret_cast<bf16x4*>(&dst[rr * LDH + k]) = hi;
        if constexpr (H == 2) *reinterpret_cast<bf16x4*>(&dst[RT * LDH + rr * LDH + k]) = lo;
      }
      // the row's dE/du sum (a wavefront's 64 lanes hold one row: Kp = 256),
      // added to dE/du by the tile's iteration
      if constexpr (GU) {
        const float sum = row_share_sum(rd);
        if (lane == 0) Rs[it1][rr] = sum;
      }
    }
  };

  const int64_t G = gridDim.x;
  auto clampt = [&](int64_t tl) { return tl < ntiles ? tl : ntiles - 1; };
  // One row tile: the next tile's staged values into the other buffer and
  // the tile PF steps ahead into the same staging registers, then the
  // products from LDS buffer it & 1 and the epilogue. Returns false after
  // the last tile.
  auto one = [&](int it, int64_t tile, Stage& S) -> bool {
    // The lane-dependent offsets below are loop-invariant; recomputing them
    // from an opaque copy of the thread index each iteration is cheaper than
    // the registers that hoisting them out of the loop would take.
    int t = tid;
    asm volatile("" : "+v"(t));
    const int ln = t % 64;
    // the next tile's staged values into the other buffers first (last read
    // before the previous barrier; past the last tile they are never read)
    // and the loads PF tiles ahead into the staging registers, so that this
    // element work interleaves with the products below; the loads keep the
    // same distance as when issued after the epilogue
    const int64_t next = tile + G;
    store(next, (it + 1) & 1, t, S);
    fetch(clampt(tile + (PF + 1) * G), t, S);
    const bf16* a_ = As[it & 1] + (ln % 16) * LDH + (ln / 16) * 8;
    floatx4 acc[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      // tiles a wavefront does not own hold zero weights: no branches here
      const bf16x8 ahi = *reinterpret_cast<const bf16x8*>(a_ + s * 32);
      if constexpr (KIND == G_BF16X3) {
        const bf16x8 alo = *reinterpret_cast<const bf16x8*>(a_ + RT * LDH + s * 32);
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bw[j][s][0], acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bw[j][s][H - 1], acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bw[j][s][0], acc[j], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int j = 0; j < NTW; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bw[j][s][0], acc[j], 0, 0, 0);
      }
    }
    if constexpr (GU) {
      // dE/du of the tile's rows: row t's sum (formed when the tile was
      // staged, in k_gemm's order, so dE/du is bitwise identical too) added
      // to the staged dE/du; the store is unconditional (dropped for t >= 16)
      float val = 0.f;
      unsigned off = kOutOfRange;
      if (t < RT) {
        val = Us[it & 1][t] + ld.c * Rs[it & 1][t];
        off = (unsigned)t * 4;
      }
      buf_store(val, gu_rsrc(tile * RT), off);
    }
    if constexpr (EPI == 0) {
      // epilogue: lane holds rows 4 (ln / 16) + q, column ln % 16 of each
      // tile; buffer stores drop rows past the end and columns past N0
      {
        const int64_t row0 = tile * RT;
        const int nvalid = (int)(nrows - row0 < RT ? nrows - row0 : RT);
        const __amdgpu_buffer_rsrc_t R0 = buffer_rsrc(ep.o0 + row0 * ep.ld0, (int64_t)nvalid * ep.ld0 * 4);
        __amdgpu_buffer_rsrc_t R1 = R0;
        if constexpr (EMODE == E_STORE_X0 || EMODE == E_RESIDUAL || EMODE == E_LATENT_BWD)
          R1 = buffer_rsrc(ep.o1 + row0 * ep.ld1, (int64_t)nvalid * ep.ld1 * 4);
        const float* lin = Xs[XIN ? it & 1 : 0];
        float rsv[4];
  #pragma unroll
        for (int q = 0; q < 4; ++q) rsv[q] = RS ? Us[it & 1][(ln / 16) * 4 + q] : 0.f;
  #pragma unroll
        for (int j = 0; j < NTW; ++j) {
          const int c0 = (my0 + j) * 16;  // first column of the tile (uniform)
          const int c = c0 + ln % 16;
          const bool cok = j < my_nt && c < ep.N0;
          const int cl = cok ? c : 0;  // in-range column for LDS reads
          float in[4];
          if constexpr (EMODE == E_ADD) {
  #pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = (ln / 16) * 4 + q;
              in[q] = buf_load(R0, cok ? (unsigned)(r * ep.ld0 + c) * 4 : kOutOfRange);
            }
          }
  #pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = (ln / 16) * 4 + q;
            const float v = acc[j][q];
            const unsigned off0 = cok ? (unsigned)(r * ep.ld0 + c) * 4 : kOutOfRange;
            const unsigned off1 = cok ? (unsigned)(r * ep.ld1 + c) * 4 : kOutOfRange;
            if constexpr (EMODE == E_STORE) {
              buf_store(v, R0, off0);
            } else if constexpr (EMODE == E_STORE_X0) {
              buf_store(v, R0, off0);
              buf_store(rsv[q] * siluf(v), R1, off1);
            } else if constexpr (EMODE == E_RESIDUAL) {
              buf_store(v, R0, off0);
              buf_store(residual_update(lin[r * LDW + cl], rsv[q], v), R1, off1);
            } else if constexpr (EMODE == E_LATENT_BWD) {
              // columns below D update g in place, the rest are the scalar adjoint
              const bool lo = c0 < ep.D;
              const unsigned off = !cok ? kOutOfRange : lo ? off0 : (unsigned)(r * ep.ld1 + c - ep.D) * 4;
              buf_store(lo ? residual_adjoint(lin[r * LDW + (lo ? cl : 0)], v) : v, lo ? R0 : R1, off);
            } else {
              buf_store(in[q] + v, R0, off0);
            }
          }
        }
      }
    } else {
      // epilogue: the products go to LDS (lane holds rows 4 (ln / 16) + q,
      // column ln % 16 of each 16x16 tile), then every thread finishes whole
      // 16-byte chunks of rows, so the stores are contiguous row segments;
      // buffer stores drop rows past the end
  #pragma unroll
      for (int j = 0; j < NTW; ++j)
  #pragma unroll
        for (int q = 0; q < 4; ++q) Os[((ln / 16) * 4 + q) * LDO + (my0 + j) * 16 + ln % 16] = acc[j][q];
      __syncthreads();
      {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        const int64_t row0 = tile * RT;
        const int nvalid = (int)(nrows - row0 < RT ? nrows - row0 : RT);
        const __amdgpu_buffer_rsrc_t R0 = buffer_rsrc(ep.o0 + row0 * ep.ld0, (int64_t)nvalid * ep.ld0 * 4);
        __amdgpu_buffer_rsrc_t R1 = R0;
        if constexpr (EMODE == E_STORE_X0 || EMODE == E_RESIDUAL || EMODE == E_LATENT_BWD)
          R1 = buffer_rsrc(ep.o1 + row0 * ep.ld1, (int64_t)nvalid * ep.ld1 * 4);
        const float* lin = Xs[XIN ? it & 1 : 0];
        const int cpr = ep.N0 / 4;  // chunks per output row
  #pragma unroll
        for (int e = 0; e < NE; ++e) {
          const int idx = t + 512 * e;
          const bool ok = idx < RT * cpr;
          const int i2 = ok ? idx : 0;
          const int r = i2 / cpr, c = (i2 % cpr) * 4;
          const float4 v = *reinterpret_cast<const float4*>(&Os[r * LDO + c]);
          const unsigned off0 = ok ? (unsigned)(r * ep.ld0 + c) * 4 : kOutOfRange;
          const unsigned off1 = ok ? (unsigned)(r * ep.ld1 + c) * 4 : kOutOfRange;
          float4 w;
          if constexpr (EMODE == E_STORE) {
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), R0, off0, 0, 0);
          } else if constexpr (EMODE == E_STORE_X0) {
            const float u = Us[it & 1][r];
            w = make_float4(u * siluf(v.x), u * siluf(v.y), u * siluf(v.z), u * siluf(v.w));
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), R0, off0, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), R1, off1, 0, 0);
          } else if constexpr (EMODE == E_RESIDUAL) {
            const float u = Us[it & 1][r];
            const float4 x = *reinterpret_cast<const float4*>(&lin[r * LDW + c]);
            w = make_float4(residual_update(x.x, u, v.x), residual_update(x.y, u, v.y), residual_update(x.z, u, v.z),
                            residual_update(x.w, u, v.w));
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), R0, off0, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), R1, off1, 0, 0);
          } else if constexpr (EMODE == E_LATENT_BWD) {
            // columns below D update g in place, the rest are the scalar adjoint
            const bool lo = c < ep.D;
            const float4 g = *reinterpret_cast<const float4*>(&lin[r * LDW + (lo ? c : 0)]);
            w = lo ? make_float4(residual_adjoint(g.x, v.x), residual_adjoint(g.y, v.y), residual_adjoint(g.z, v.z),
                                 residual_adjoint(g.w, v.w))
                   : v;
            const unsigned off = !ok ? kOutOfRange : lo ? off0 : (unsigned)(r * ep.ld1 + c - ep.D) * 4;
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), lo ? R0 : R1, off, 0, 0);
          } else {
            const float4 in = *reinterpret_cast<const float4*>(&Is[it & 1][r * LDO + c]);
            w = make_float4(in.x + v.x, in.y + v.y, in.z + v.z, in.w + v.w);
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), R0, off0, 0, 0);
          }
        }
      }
    }
    return next < ntiles;
  };

  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  // fetches are unconditional (a tile past the end is replaced by the last
  // one, loaded and never used) so every path issues the same memory
  // operations and the compiler's wait counts stay exact
  fetch(tile, tid, s0);
  store(tile, 0, tid, s0);
  if constexpr (PF == 1) {
    fetch(clampt(tile + G), tid, s0);
    __syncthreads();
    for (int it = 0;; ++it, tile += G) {
      if (!one(it, tile, s0)) break;
      __syncthreads();
    }
  } else {
    fetch(clampt(tile + G), tid, s1);
    fetch(clampt(tile + 2 * G), tid, s0);
    __syncthreads();
    for (int it = 0;; it += 2) {
      if (!one(it, tile, s1)) break;
      __syncthreads();
      tile += G;
      if (!one(it + 1, tile, s0)) break;
      __syncthreads();
      tile += G;
    }
  }
}

// Weight-stationary launch of one product (gemm_ws.hip) with epilogue form 0
// or 1. Returns whether the product's signature has a compiled kernel;
// launches it only when asked.
bool gemm_ws(bool launch, int form, int kind, hipStream_t s, int num_cu, int NP, int Kp, const void* Bt,
             const int* nrows, const ALoad& ld, const Epi& ep);

}  // namespace nq
