// The two-body MLP of the edge latents (paper Sec. 2.1: the initial scalar
// latent of an edge is an MLP of the two species and the radial basis) as one
// persistent kernel per direction, for the benchmark shape: input row h0
// [32] (one-hot species of i and j, 8 Bessel terms, padding), layers
// 32 -> 64 -> 128 -> 256 with SiLU after each.
//
// Forward: only the last pre-activation a2 leaves the kernel (x0 = u SiLU(a2)
// is formed by its readers); a0 and a1 stay in LDS. Adjoint: a0 and a1 are
// recomputed from h0 in the same way, then dE/da2 = g u SiLU'(a2) (with the
// row sums dE/du += sum g SiLU(a2)) is taken back through the three layers to
// dE/dh0; dE/ds1 and dE/ds0 stay in LDS. Against one launch per layer this
// saves writing and reading back a0, a1, dE/ds1 and dE/ds0 (3.7 KB per edge).
//
// Every product is the one the per-layer kernels compute: the same BF16
// splits of the same FP32 values, the same 32-deep K steps in the same order,
// the same three BF16X3 products per step in the same order, and the same
// element functions; the row sums are added in the per-layer kernels' order.
// So the results are bitwise those of the per-layer path.
//
// One workgroup of 8 wavefronts per CU takes 16-row edge tiles in turn. The
// largest weight matrix (128 x 256) is held in registers as matrix-core B
// fragments (forward: wavefront w owns output columns 32 w .. 32 w + 31;
// adjoint: dE/ds1 columns 16 w .. 16 w + 15); the two small ones live in LDS. A lane holds rows 4 (lane / 16) + q, column lane % 16 of
// each 16 x 16 product tile.
#include "gemm.hpp"

namespace nq {
namespace tb {

constexpr int RT = 16, NTH = 512;
constexpr int K0 = 32, N0 = 64, N1 = 128, N2 = 256;  // padded input and layer widths
// LDS row strides in BF16 values (8 more than the row: 16-byte aligned rows,
// fewer bank conflicts between the 16 rows a fragment load spans)
constexpr int L0 = K0 + 8, L1 = N0 + 8, L2 = N1 + 8, LG = N2 + 8;
// FP32 row strides
constexpr int F1 = N0 + 4, F2 = N1 + 4;

struct Args {
  const int* nrows;
  const float* h0;  // [E][32]
  const float* u;   // cutoff u of row e at u[e * ldu]
  int ldu;
  const bf16* w0;   // forward B operands [N][K], BF16 hi then lo
  const bf16* w1;
  const bf16* w2;
  const bf16* b0;   // adjoint B operands [K][N] (W itself), BF16 hi then lo
  const bf16* b1;
  const bf16* b2;
  float* a2;        // [E][256] forward output (pre-activation)
  const float* g;   // [E][ldg] dE/dx0 (adjoint input)
  int ldg;
  float* gu;        // [E] dE/du, added to
  float* gh0;       // [E][ldgh] dE/dh0 (adjoint output, n_in columns)
  int ldgh, n_in;
};

// One 16-row tile of A (hi and lo rows of stride L) times one 16-column B
// fragment set, K = 32 S, in K order with the BF16X3 product order.
template <int KIND, int S>
__device__ inline floatx4 mma_lds(const bf16* A, int la, int alo, const bf16* B, int lb, int blo, int n0, int lane) {
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const bf16* ar = A + (lane % 16) * la + (lane / 16) * 8;
  const bf16* br = B + (n0 + lane % 16) * lb + (lane / 16) * 8;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ar + s * 32);
    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(br + s * 32);
    if constexpr (KIND == G_BF16X3) {
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(ar + alo + s * 32);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(br + blo + s * 32);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    } else {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    }
  }
  return acc;
}

// v into row r, column c of a split tile (hi rows at T, lo rows lo further).
// v is pinned to a rounded register value first: otherwise the compiler may
// fuse the product that made v (SiLU's last multiply) with the residual
// v - hi into one FMA, and the low half would differ from the per-layer
// kernels', which split values that went through memory.
template <int KIND>
__device__ inline void put_split(bf16* T, int lo, int idx, float v) {
  asm volatile("" : "+v"(v));
  const bf16 h = (bf16)v;
  T[idx] = h;
  if constexpr (KIND == G_BF16X3) T[lo + idx] = (bf16)(v - (float)h);
}

// Copies a [N][K] BF16 operand (hi then lo, nh halves) into LDS rows of stride L.
__device__ inline void stage_w(bf16* dst, const bf16* src, int N, int K, int L, int nh, int tid) {
  const int per = N * K / 8;
  for (int i = tid; i < nh * per; i += NTH) {
    const int h = i / per, r = i % per, n = r / (K / 8), k = (r % (K / 8)) * 8;
    *reinterpret_cast<bf16x8*>(dst + h * N * L + n * L + k) =
        *reinterpret_cast<const bf16x8*>(src + (int64_t)h * N * K + n * K + k);
  }
}

// h0 rows of a tile into the first layer's A tile: 128 chunks of 4, one per
// thread below 128 (rows past the end are zero).
template <int KIND>
__device__ inline void put_h0(bf16* A0, const float4& v, bool ok, int tid) {
  if (tid < RT * K0 / 4) {
    const int r = tid / (K0 / 4), k = (tid % (K0 / 4)) * 4;
    const float e[4] = {ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) put_split<KIND>(A0, RT * L0, r * L0 + k + q, e[q]);
  }
}

__device__ inline float4 load_h0(const Args& a, int64_t tile, int64_t nrows, int tid) {
  const int r = tid / (K0 / 4), k = (tid % (K0 / 4)) * 4;
  int64_t row = tile * RT + (tid < RT * K0 / 4 ? r : 0);
  row = row < nrows ? row : nrows - 1;
  return *reinterpret_cast<const float4*>(a.h0 + row * K0 + k);
}

// a0 = A0 W0 (waves 0..3, one 16-column tile each) and a1 = SiLU(a0) W1
// (all 8 waves, one tile each). Forward: s1 = SiLU(a1) into S1. Adjoint
// (ADJ): the FP32 pre-activations a0, a1 into A0f, A1f. Ends with a barrier.
template <int KIND, bool ADJ>
__device__ inline void layers01(const bf16* A0, const bf16* W0s, const bf16* W1s, bf16* S0, float* A0f, bf16* S1,
                                float* A1f, int wave, int lane) {
  if (wave < N0 / 16) {
    const floatx4 acc = mma_lds<KIND, K0 / 32>(A0, L0, RT * L0, W0s, L0, N0 * L0, wave * 16, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * (lane / 16) + q, c = wave * 16 + lane % 16;
      if constexpr (ADJ) A0f[r * F1 + c] = acc[q];
      put_split<KIND>(S0, RT * L1, r * L1 + c, siluf(acc[q]));
    }
  }
  __syncthreads();
  {
    const floatx4 acc = mma_lds<KIND, N0 / 32>(S0, L1, RT * L1, W1s, L1, N1 * L1, wave * 16, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 4 * (lane / 16) + q, c = wave * 16 + lane % 16;
      if constexpr (ADJ)
        A1f[r * F2 + c] = acc[q];
      else
        put_split<KIND>(S1, RT * L2, r * L2 + c, siluf(acc[q]));
    }
  }
  __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_tb_fwd(Args a) {
  constexpr int H = KIND == G_BF16X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) bf16 W0s[H * N0 * L0];
  __shared__ __attribute__((aligned(16))) bf16 W1s[H * N1 * L1];
  __shared__ __attribute__((aligned(16))) bf16 A0[H * RT * L0];
  __shared__ __attribute__((aligned(16))) bf16 S0[H * RT * L1];
  __shared__ __attribute__((aligned(16))) bf16 S1[H * RT * L2];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int64_t nrows = *a.nrows, ntiles = (nrows + RT - 1) / RT;
  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  stage_w(W0s, a.w0, N0, K0, L0, H, tid);
  stage_w(W1s, a.w1, N1, N0, L1, H, tid);
  // the last layer's weights as B fragments: wave w, column tiles 2 w, 2 w + 1
  bf16x8 bw[2][N1 / 32][H];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int s = 0; s < N1 / 32; ++s)
#pragma unroll
      for (int h = 0; h < H; ++h)
        bw[j][s][h] = *reinterpret_cast<const bf16x8*>(a.w2 + (int64_t)h * N2 * N1 +
                                                        ((2 * wave + j) * 16 + lane % 16) * N1 + s * 32 + (lane / 16) * 8);
  float4 hv = load_h0(a, tile, nrows, tid);
  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * RT;
    put_h0<KIND>(A0, hv, row0 + tid / (K0 / 4) < nrows, tid);
    const int64_t next = tile + gridDim.x;
    hv = load_h0(a, next < ntiles ? next : ntiles - 1, nrows, tid);
    __syncthreads();
    layers01<KIND, false>(A0, W0s, W1s, S0, nullptr, S1, nullptr, wave, lane);
    // a2 = s1 W2, stored as the forward output
    floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    const bf16* ar = S1 + (lane % 16) * L2 + (lane / 16) * 8;
#pragma unroll
    for (int s = 0; s < N1 / 32; ++s) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ar + s * 32);
      if constexpr (KIND == G_BF16X3) {
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(ar + RT * L2 + s * 32);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bw[j][s][0], acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[j][s][H - 1], acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[j][s][0], acc[j], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[j][s][0], acc[j], 0, 0, 0);
      }
    }
    const int nvalid = (int)(nrows - row0 < RT ? nrows - row0 : RT);
    const __amdgpu_buffer_rsrc_t R = buffer_rsrc(a.a2 + row0 * N2, (int64_t)nvalid * N2 * 4);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * (lane / 16) + q, c = (2 * wave + j) * 16 + lane % 16;
        buf_store(acc[j][q], R, (unsigned)(r * N2 + c) * 4);
      }
    // S1 is next written after the next tile's first barrier, by which time
    // every wavefront has read it
  }
}

template <int KIND>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_tb_bwd(Args a) {
  constexpr int H = KIND == G_BF16X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) bf16 W0s[H * N0 * L0];   // forward W0 [64][32]
  __shared__ __attribute__((aligned(16))) bf16 W1s[H * N1 * L1];   // forward W1 [128][64]
  __shared__ __attribute__((aligned(16))) bf16 B1s[H * N0 * L2];   // adjoint W1 [64][128]
  __shared__ __attribute__((aligned(16))) bf16 B0s[H * 16 * L1];   // adjoint W0 [16][64]
  __shared__ __attribute__((aligned(16))) bf16 A0[H * RT * L0];
  __shared__ __attribute__((aligned(16))) bf16 S0[H * RT * L1];
  __shared__ __attribute__((aligned(16))) float A0f[RT * F1];      // a0 (FP32)
  __shared__ __attribute__((aligned(16))) float A1f[RT * F2];      // a1 (FP32)
  __shared__ __attribute__((aligned(16))) bf16 G2[H * RT * LG];    // dE/da2 (split)
  __shared__ __attribute__((aligned(16))) bf16 G1[H * RT * L2];    // dE/da1 (split)
  __shared__ __attribute__((aligned(16))) bf16 G0[H * RT * L1];    // dE/da0 (split)
  __shared__ float Rd[RT * 64];                                    // dE/du shares per 4-chunk
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int64_t nrows = *a.nrows, ntiles = (nrows + RT - 1) / RT;
  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  stage_w(W0s, a.w0, N0, K0, L0, H, tid);
  stage_w(W1s, a.w1, N1, N0, L1, H, tid);
  stage_w(B1s, a.b1, N0, N1, L2, H, tid);
  stage_w(B0s, a.b0, 16, N0, L1, H, tid);
  // the adjoint of the last layer as B fragments: wave w, column tile w of
  // dE/ds1 (128 columns), K = 256
  bf16x8 bw[N2 / 32][H];
#pragma unroll
  for (int s = 0; s < N2 / 32; ++s)
#pragma unroll
    for (int h = 0; h < H; ++h)
      bw[s][h] = *reinterpret_cast<const bf16x8*>(a.b2 + (int64_t)h * N1 * N2 + (wave * 16 + lane % 16) * N2 + s * 32 +
                                                  (lane / 16) * 8);
  // dE/da2 inputs: wavefront w holds rows w and w + 8, lane l their 4-chunk l
  // (columns 4 l .. 4 l + 3: K step l / 8, position l % 8 in it)
  float4 gv[2], av[2];
  float uv[2], guv = 0.f;
  auto load_g = [&](int64_t t) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int64_t row = t * RT + wave + 8 * q;
      row = row < nrows ? row : nrows - 1;
      gv[q] = *reinterpret_cast<const float4*>(a.g + row * a.ldg + 4 * lane);
      av[q] = *reinterpret_cast<const float4*>(a.a2 + row * N2 + 4 * lane);
      uv[q] = a.u[row * a.ldu];
    }
    int64_t row = t * RT + (tid < RT ? tid : 0);
    row = row < nrows ? row : nrows - 1;
    guv = a.gu[row];
  };
  float4 hv = load_h0(a, tile, nrows, tid);
  load_g(tile);
  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * RT;
    const int nvalid = (int)(nrows - row0 < RT ? nrows - row0 : RT);
    put_h0<KIND>(A0, hv, tid / (K0 / 4) < nvalid, tid);
    // dE/da2 = g u SiLU'(a2) into G2; each 4-chunk's share of sum g SiLU(a2)
    // into Rd
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = wave + 8 * q;
      const bool ok = r < nvalid;
      const float4 g4 = gv[q], a4 = av[q];
      const float sx = sigmoidf_(a4.x), sy = sigmoidf_(a4.y), sz = sigmoidf_(a4.z), sw = sigmoidf_(a4.w);
      const float e[4] = {gradsilu_scale(g4.x, a4.x, sx, uv[q]), gradsilu_scale(g4.y, a4.y, sy, uv[q]),
                          gradsilu_scale(g4.z, a4.z, sz, uv[q]), gradsilu_scale(g4.w, a4.w, sw, uv[q])};
#pragma unroll
      for (int k = 0; k < 4; ++k) put_split<KIND>(G2, RT * LG, r * LG + 4 * lane + k, ok ? e[k] : 0.f);
      Rd[r * 64 + lane] = ok ? gradsilu_part(g4, a4, sx, sy, sz, sw) : 0.f;
    }
    const float gu_old = guv;
    const int64_t next = tile + gridDim.x;
    hv = load_h0(a, next < ntiles ? next : ntiles - 1, nrows, tid);
    load_g(next < ntiles ? next : ntiles - 1);
    __syncthreads();
    // dE/du of row tid: the shares of each position summed over the K steps
    // in order, then the 8 positions pairwise (the per-layer kernels' order)
    if (tid < nvalid) {
      const float* rp = Rd + tid * 64;
      float r[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) r[j] = 0.f;
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] += rp[s2 * 8 + j];
      a.gu[row0 + tid] = gu_old + 1.f * (((r[0] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7])));
    }
    // a0, a1 again from h0 (FP32 in LDS)
    layers01<KIND, true>(A0, W0s, W1s, S0, A0f, nullptr, A1f, wave, lane);
    // dE/ds1 = dE/da2 W2^T (wave w: columns 16 w ..), then dE/da1 = dE/ds1 SiLU'(a1)
    {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      const bf16* ar = G2 + (lane % 16) * LG + (lane / 16) * 8;
#pragma unroll
      for (int s = 0; s < N2 / 32; ++s) {
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ar + s * 32);
        if constexpr (KIND == G_BF16X3) {
          const bf16x8 al = *reinterpret_cast<const bf16x8*>(ar + RT * LG + s * 32);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bw[s][0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[s][H - 1], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[s][0], acc, 0, 0, 0);
        } else {
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[s][0], acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * (lane / 16) + q, c = wave * 16 + lane % 16;
        const float a1 = A1f[r * F2 + c];
        put_split<KIND>(G1, RT * L2, r * L2 + c, r < nvalid ? gradsilu_scale(acc[q], a1, sigmoidf_(a1), 1.f) : 0.f);
      }
    }
    __syncthreads();
    // dE/ds0 = dE/da1 W1^T (waves 0..3), then dE/da0 = dE/ds0 SiLU'(a0)
    if (wave < N0 / 16) {
      const floatx4 acc = mma_lds<KIND, N1 / 32>(G1, L2, RT * L2, B1s, L2, N0 * L2, wave * 16, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * (lane / 16) + q, c = wave * 16 + lane % 16;
        const float a0 = A0f[r * F1 + c];
        put_split<KIND>(G0, RT * L1, r * L1 + c, r < nvalid ? gradsilu_scale(acc[q], a0, sigmoidf_(a0), 1.f) : 0.f);
      }
    }
    __syncthreads();
    // dE/dh0 = dE/da0 W0^T (wave 0), the first n_in columns stored
    if (wave == 0) {
      const floatx4 acc = mma_lds<KIND, N0 / 32>(G0, L1, RT * L1, B0s, L1, 16 * L1, 0, lane);
      const __amdgpu_buffer_rsrc_t R = buffer_rsrc(a.gh0 + row0 * a.ldgh, (int64_t)nvalid * a.ldgh * 4);
      const int c = lane % 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 4 * (lane / 16) + q;
        buf_store(acc[q], R, c < a.n_in ? (unsigned)(r * a.ldgh + c) * 4 : kOutOfRange);
      }
    }
    // the LDS tiles of this tile are rewritten only after the next tile's
    // first barrier (A0, G2, Rd) or later ones
  }
}

}  // namespace tb

// True when the two-body MLP of this model runs as the two kernels above on
// this context: the automatic path, a BF16 kind for every two-body product,
// and the compiled widths.
bool tb_fused(const nq_ctx* ctx, const nq_model* m) {
  const Dims& d = m->dims;
  if (ctx->path != NQ_PATH_AUTO) return false;
  if (d.prec != NQ_PRECISION_BF16 && d.prec != NQ_PRECISION_BF16X3) return false;
  if (d.n_tb != 3 || d.tb[0] != tb::N0 || d.tb[1] != tb::N1 || d.tb[2] != tb::N2 || d.D != tb::N2) return false;
  if (ctx->ws.K0p != tb::K0 || d.n_in2b > 16 || ctx->ws.maxw < 16) return false;
  const Lin &L0 = *m->tb[0], &L1 = *m->tb[1], &L2 = *m->tb[2];
  if (L0.kp_f != tb::K0 || L0.np_f != tb::N0 || L1.kp_f != tb::N0 || L1.np_f != tb::N1 || L2.kp_f != tb::N1 ||
      L2.np_f != tb::N2 || L2.kp_b != tb::N2 || L2.np_b != tb::N1 || L1.kp_b != tb::N1 || L1.np_b != tb::N0 ||
      L0.kp_b != tb::N0 || L0.np_b != 16)
    return false;
  for (const auto& kv : m->site_prec)
    if (kv.first.find("twobody") != std::string::npos && kv.second != d.prec) return false;
  return true;
}

namespace {
tb::Args tb_args(nq_ctx* ctx, const nq_model* m) {
  const Workspace& ws = ctx->ws;
  const Dims& d = m->dims;
  tb::Args a{};
  a.nrows = ws.v_nedge;
  a.h0 = ws.h0;
  a.u = ws.geo + 1;
  a.ldu = 16;
  a.w0 = m->tb[0]->bf_fwd.as<bf16>();
  a.w1 = m->tb[1]->bf_fwd.as<bf16>();
  a.w2 = m->tb[2]->bf_fwd.as<bf16>();
  a.b0 = m->tb[0]->bf_bwd.as<bf16>();
  a.b1 = m->tb[1]->bf_bwd.as<bf16>();
  a.b2 = m->tb[2]->bf_bwd.as<bf16>();
  a.a2 = ws.a_tb[2];
  a.g = ws.gx;
  a.ldg = d.D;
  a.gu = ws.gu;
  a.gh0 = ws.gh[0];
  a.ldgh = (int)ws.maxw;
  a.n_in = d.n_in2b;
  return a;
}

template <class K>
unsigned tb_grid(K kernel, int num_cu, int64_t cap) {
  int per_cu = 0;
  NQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, tb::NTH, 0));
  const int64_t tiles = (cap + tb::RT - 1) / tb::RT;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)std::max(per_cu, 1) * num_cu));
}
}  // namespace

void tb_fwd_async(nq_ctx* ctx, const nq_model* m) {
  const tb::Args a = tb_args(ctx, m);
  // per edge: h0 and a2; the three products
  const double fl = 2.0 * (tb::K0 * tb::N0 + tb::N0 * tb::N1 + tb::N1 * tb::N2);
  const int sp = span_begin(ctx, "fwd.twobody", fl, 4.0 * (tb::K0 + tb::N2), 0, 0, fl);
  if (m->dims.prec == NQ_PRECISION_BF16X3)
    tb::k_tb_fwd<G_BF16X3><<<tb_grid(tb::k_tb_fwd<G_BF16X3>, ctx->num_cu, ctx->ws.cap), tb::NTH, 0, ctx->stream>>>(a);
  else
    tb::k_tb_fwd<G_BF16><<<tb_grid(tb::k_tb_fwd<G_BF16>, ctx->num_cu, ctx->ws.cap), tb::NTH, 0, ctx->stream>>>(a);
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

void tb_bwd_async(nq_ctx* ctx, const nq_model* m) {
  const tb::Args a = tb_args(ctx, m);
  // per edge: h0, dE/dx0, a2, u, dE/du (read and written), dE/dh0; the
  // recomputed first two products and the three adjoint products
  const double fl = 2.0 * (tb::K0 * tb::N0 + tb::N0 * tb::N1 + tb::N1 * tb::N2);
  const int sp = span_begin(ctx, "bwd.twobody", 2.0 * fl - 2.0 * tb::N1 * tb::N2,
                            4.0 * (tb::K0 + 2 * tb::N2 + 1 + 2 + m->dims.n_in2b), 0, 0, fl);
  if (m->dims.prec == NQ_PRECISION_BF16X3)
    tb::k_tb_bwd<G_BF16X3><<<tb_grid(tb::k_tb_bwd<G_BF16X3>, ctx->num_cu, ctx->ws.cap), tb::NTH, 0, ctx->stream>>>(a);
  else
    tb::k_tb_bwd<G_BF16><<<tb_grid(tb::k_tb_bwd<G_BF16>, ctx->num_cu, ctx->ws.cap), tb::NTH, 0, ctx->stream>>>(a);
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

}  // namespace nq
