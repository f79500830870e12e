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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

enum ALoadMode { A_PLAIN = 0, A_SILU = 1, A_CAT = 2, A_GRADSILU = 3 };

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
    if (mode == A_CAT) {
      const bool second = k >= K0;
      const int k1 = k - K0 < K1 ? k - K0 : 0;
      const float* p = second ? p1 + r * ld1 + k1 : p0 + r * ld0 + k;
      o.v = *reinterpret_cast<const float4*>(p);
    } else {
      const int kk = k < K0 ? k : 0;
      o.v = *reinterpret_cast<const float4*>(p0 + r * ld0 + kk);
      if (mode == A_GRADSILU) {
        o.a = *reinterpret_cast<const float4*>(p1 + r * ld1 + kk);
        o.f = rs ? rs[r * rs_ld] : 1.f;
      }
    }
  }
  // The A values from the raw loads: zero outside the rows or columns,
  // SiLU, or the adjoint g * c * rowscale * SiLU'(a).
  // With gu set, rd accumulates this chunk's share of sum_k g SiLU(a), the
  // derivative with respect to the row scale, from the same loaded values.
  __device__ inline float4 finish(const ARaw& o, bool row_ok, int k, float& rd) const {
    const bool ok = row_ok && k < (mode == A_CAT ? K0 + K1 : K0);
    float4 v = o.v;
    if (mode == A_SILU) {
      v.x = siluf(v.x);
      v.y = siluf(v.y);
      v.z = siluf(v.z);
      v.w = siluf(v.w);
    } else if (mode == A_GRADSILU) {
      const float f = c * o.f;
      const float sx = sigmoidf_(o.a.x), sy = sigmoidf_(o.a.y), sz = sigmoidf_(o.a.z), sw = sigmoidf_(o.a.w);
      if (gu) {
        const float part = v.x * o.a.x * sx + v.y * o.a.y * sy + v.z * o.a.z * sz + v.w * o.a.w * sw;
        rd += ok ? part : 0.f;
      }
      v.x *= f * sx * (1.f + o.a.x * (1.f - sx));
      v.y *= f * sy * (1.f + o.a.y * (1.f - sy));
      v.z *= f * sz * (1.f + o.a.z * (1.f - sz));
      v.w *= f * sw * (1.f + o.a.w * (1.f - sw));
    }
    return ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
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
            o1[c] = (in[jj][q] + rsv[q] * siluf(v)) * kInvSqrt2;
          } else if constexpr (MODE == E_LATENT_BWD) {
            if (c < ep.D)
              o0[c] = in[jj][q] * kInvSqrt2 + v;
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

}  // namespace nq
