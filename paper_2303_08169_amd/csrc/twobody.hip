// The two-body MLP of the edge latents (paper Sec. 2.1: the initial scalar
// latent of an edge is an MLP of the two species and the radial basis) as one
// persistent kernel per direction, for the benchmark shape: input row h0
// [32] (one-hot species of i and j, 8 Bessel terms, padding), layers
// 32 -> 64 -> 128 -> 256 with SiLU after each.
//
// Forward: only the last pre-activation a2 leaves the kernel (x0 = u SiLU(a2)
// is formed by its readers); s0 = SiLU(a0) and s1 stay in LDS. Adjoint: a0 and a1 are
// recomputed from h0 in the same way, then dE/da2 = g u SiLU'(a2) (with the
// row sums dE/du += sum g SiLU(a2)) is taken back through the three layers to
// dE/dh0; dE/da1 and dE/da0 stay in LDS. Against one launch per layer this
// saves writing and reading back a0, a1, dE/ds1 and dE/ds0 (3.7 KB per edge).
//
// Every product is the one the per-layer kernels compute: the same BF16
// splits of the same FP32 values, the same 32-deep K steps in the same order,
// the same three BF16X3 products per step in the same order, and the same
// element functions; the row sums are added in the per-layer kernels' order.
// So the results are bitwise those of the per-layer path.
//
// One workgroup of 8 wavefronts per CU takes 32-row edge tiles (two 16-row
// matrix-core tiles) in turn. The largest weight matrix (128 x 256) is held in
// registers as matrix-core B fragments (forward: wavefront w owns output
// columns 32 w .. 32 w + 31; adjoint: dE/ds1 columns 16 w .. 16 w + 15), as is
// the first layer's adjoint; the other weights live in LDS. A wavefront keeps
// the a0 and a1 tiles it recomputes in the adjoint in registers, because it is
// also the one that forms dE/da0 and dE/da1 at the same elements. A lane holds
// rows 4 (lane / 16) + q, column lane % 16 of each 16 x 16 product tile.
#include "gemm.hpp"

namespace nq {
namespace tb {

constexpr int RT = 32, NTH = 512;  // rows per tile (two 16-row MFMA tiles), threads
constexpr int K0 = 32, N0 = 64, N1 = 128, N2 = 256;  // padded input and layer widths
// LDS row strides in BF16 values (8 more than the row: 16-byte aligned rows,
// fewer bank conflicts between the 16 rows a fragment load spans)
constexpr int L0 = K0 + 8, L1 = N0 + 8, L2 = N1 + 8, LG = N2 + 8;

struct Args {
  const int* nrows;
  const float* h0;  // [E][32]
  const float* u;   // cutoff u of row e at u[e * ldu]
  int ldu;
  const bf16* w0;   // forward B operands [N][K], BF16 hi then lo
  const bf16* w1;
  const bf16* w2;
  const bf16* b0;   // adjoint B operands: W as [fan-in][fan-out], BF16 hi then lo
  const bf16* b1;
  const bf16* b2;
  float* a2;        // [E][256] forward output (pre-activation)
  const float* g;   // [E][ldg] dE/dx0 (adjoint input)
  int ldg;
  float* gu;        // [E] dE/du, added to
  float* gh0;       // [E][ldgh] dE/dh0 (adjoint output, n_in columns)
  int ldgh, n_in;
};

// NR consecutive 16-row tiles of A (hi rows of stride la, lo rows alo
// further) times one 16-column fragment set of B (rows n0 .., stride lb, lo
// blo further), K = 32 S, in K order with the BF16X3 product order per step.
template <int KIND, int S, int NR>
__device__ inline void mma_lds(const bf16* A, int la, int alo, const bf16* B, int lb, int blo, int n0, int lane,
                               floatx4 (&acc)[NR]) {
  const bf16* ar = A + (lane % 16) * la + (lane / 16) * 8;
  const bf16* br = B + (n0 + lane % 16) * lb + (lane / 16) * 8;
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(br + s * 32);
    bf16x8 bl = bh;
    if constexpr (KIND == G_BF16X3) bl = *reinterpret_cast<const bf16x8*>(br + blo + s * 32);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ar + i * 16 * la + s * 32);
      if constexpr (KIND == G_BF16X3) {
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(ar + i * 16 * la + alo + s * 32);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[i], 0, 0, 0);
      }
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[i], 0, 0, 0);
    }
  }
}

// The same with B as register fragments bw[s][half].
template <int KIND, int S, int NR, int H>
__device__ inline void mma_reg(const bf16* A, int la, int alo, const bf16x8 (&bw)[S][H], int lane, floatx4 (&acc)[NR]) {
  const bf16* ar = A + (lane % 16) * la + (lane / 16) * 8;
#pragma unroll
  for (int i = 0; i < NR; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(ar + i * 16 * la + s * 32);
      if constexpr (KIND == G_BF16X3) {
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(ar + i * 16 * la + alo + s * 32);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bw[s][0], acc[i], 0, 0, 0);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[s][H - 1], acc[i], 0, 0, 0);
      }
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw[s][0], acc[i], 0, 0, 0);
    }
}

// v into a split tile (hi at T[idx], lo at T[lo + idx]). v is pinned to a
// rounded register value first: otherwise the compiler may fuse the product
// that made v (SiLU's last multiply) with the residual v - hi into one FMA,
// and the low half would differ from the per-layer kernels', which split
// values that went through memory.
template <int KIND>
__device__ inline void put_split(bf16* T, int lo, int idx, float v) {
  asm volatile("" : "+v"(v));
  const bf16 h = (bf16)v;
  T[idx] = h;
  if constexpr (KIND == G_BF16X3) T[lo + idx] = (bf16)(v - (float)h);
}

// Four consecutive values into a split tile as one 8-byte store per half
// (idx a multiple of 4), each value pinned as in put_split.
template <int KIND>
__device__ inline void put_split4(bf16* T, int lo, int idx, const float (&v)[4]) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 h, l;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float x = v[k];
    asm volatile("" : "+v"(x));
    h[k] = (bf16)x;
    l[k] = (bf16)(x - (float)h[k]);
  }
  *reinterpret_cast<bf16x4*>(T + idx) = h;
  if constexpr (KIND == G_BF16X3) *reinterpret_cast<bf16x4*>(T + lo + idx) = l;
}

// B fragments of a [N][K] operand (hi then lo) for column tile n0, K = 32 S.
template <int S, int H>
__device__ inline void load_frags(bf16x8 (&bw)[S][H], const bf16* src, int N, int K, int n0, int lane) {
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int h = 0; h < H; ++h)
      bw[s][h] = *reinterpret_cast<const bf16x8*>(src + (int64_t)h * N * K + (n0 + lane % 16) * K + s * 32 +
                                                  (lane / 16) * 8);
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

// The input rows of a tile, one 4-chunk per thread (row tid / 8, columns
// 4 (tid % 8) ..): loads (rows past the end read the last row) and the split
// into the first layer's A tile (rows past the end are zero).
__device__ inline float4 load_h0(const Args& a, int64_t tile, int64_t nrows, int tid) {
  int64_t row = tile * RT + tid / (K0 / 4);
  row = row < nrows ? row : nrows - 1;
  return *reinterpret_cast<const float4*>(a.h0 + row * K0 + (tid % (K0 / 4)) * 4);
}
template <int KIND>
__device__ inline void put_h0(bf16* A0, const float4& v, bool ok, int tid) {
  const int r = tid / (K0 / 4), k = (tid % (K0 / 4)) * 4;
  const float e[4] = {ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f};
  put_split4<KIND>(A0, RT * L0, r * L0 + k, e);
}

// Output element q of a 16 x 16 product tile: row 4 (lane / 16) + q, column lane % 16.
__device__ inline int orow(int lane, int q) { return 4 * (lane / 16) + q; }

// Wavefront w's part of the first layer: a0 of column tile w % 4 and row
// tile w / 4, kept in a0 with its sigmoid in sg0 (SiLU(a) = a sigmoid(a));
// s0 = SiLU(a0) split into S0.
template <int KIND>
__device__ inline void layer0(const bf16* A0, const bf16* W0s, bf16* S0, int wave, int lane, floatx4 (&a0)[1],
                              floatx4& sg0) {
  const int rt = wave / 4, c0 = (wave % 4) * 16;
  mma_lds<KIND, K0 / 32, 1>(A0 + rt * 16 * L0, L0, RT * L0, W0s, L0, N0 * L0, c0, lane, a0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    sg0[q] = sigmoidf_(a0[0][q]);
    put_split<KIND>(S0, RT * L1, (rt * 16 + orow(lane, q)) * L1 + c0 + lane % 16, a0[0][q] * sg0[q]);
  }
}

// Wavefront w's part of the second layer: a1 of column tile w, both row
// tiles, kept in a1; with S1 given, s1 = SiLU(a1) split into it.
template <int KIND>
__device__ inline void layer1(const bf16* S0, const bf16* W1s, bf16* S1, int wave, int lane, floatx4 (&a1)[2]) {
  mma_lds<KIND, N0 / 32, 2>(S0, L1, RT * L1, W1s, L1, N1 * L1, wave * 16, lane, a1);
  if (S1) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        put_split<KIND>(S1, RT * L2, (i * 16 + orow(lane, q)) * L2 + wave * 16 + lane % 16, siluf(a1[i][q]));
  }
}

// The workgroups take tiles blockIdx.x, + gridDim.x, ... Both kernels are
// software-pipelined over a workgroup's tiles so that independent products of
// consecutive tiles share the phases between two barriers.

// Forward, per tile i: phase 1 = layer 0 of tile i and the last layer of
// tile i - 1 (four independent accumulation chains per wavefront); phase 2 =
// layer 1 of tile i (into S1 buffer i % 2) and the input rows of tile i + 1
// into A0. A final pass of both phases ends tile i - 1 alone.
template <int KIND>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_tb_fwd(Args a) {
  constexpr int H = KIND == G_BF16X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) bf16 W0s[H * N0 * L0];
  __shared__ __attribute__((aligned(16))) bf16 W1s[H * N1 * L1];
  __shared__ __attribute__((aligned(16))) bf16 A0[H * RT * L0];
  __shared__ __attribute__((aligned(16))) bf16 S0[H * RT * L1];
  __shared__ __attribute__((aligned(16))) bf16 S1[2][H * RT * L2];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int64_t nrows = *a.nrows, ntiles = (nrows + RT - 1) / RT, G = gridDim.x;
  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  stage_w(W0s, a.w0, N0, K0, L0, H, tid);
  stage_w(W1s, a.w1, N1, N0, L1, H, tid);
  // the last layer's weights as B fragments: wavefront w, column tiles 2 w, 2 w + 1
  bf16x8 bw[2][N1 / 32][H];
  load_frags(bw[0], a.w2, N2, N1, 32 * wave, lane);
  load_frags(bw[1], a.w2, N2, N1, 32 * wave + 16, lane);
  auto clampt = [&](int64_t t) { return t < ntiles ? t : ntiles - 1; };
  float4 hv = load_h0(a, tile, nrows, tid & 255);
  if (tid < RT * K0 / 4) put_h0<KIND>(A0, hv, tile * RT + tid / (K0 / 4) < nrows, tid);
  hv = load_h0(a, clampt(tile + G), nrows, tid & 255);
  __syncthreads();
  // a2 = s1 W2 of tile t, column half j (s1: that tile's S1 buffer), stored;
  // t < 0 stores nothing (a buffer of no rows)
  auto last_layer = [&](int64_t t, int j, const bf16* s1) {
    const int64_t row0 = t < 0 ? 0 : t * RT;
    const int nvalid = t < 0 ? 0 : (int)(nrows - row0 < RT ? nrows - row0 : RT);
    const __amdgpu_buffer_rsrc_t R = buffer_rsrc(a.a2 + row0 * N2, nvalid * N2 * 4);
    floatx4 acc[2];
    mma_reg<KIND, N1 / 32, 2, H>(s1, L2, RT * L2, bw[j], lane, acc);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        buf_store(acc[i][q], R, (unsigned)((i * 16 + orow(lane, q)) * N2 + 32 * wave + 16 * j + lane % 16) * 4);
  };
  int64_t prev = -1;
  for (int it = 0;; ++it) {
    const bool cur = tile < ntiles;  // uniform
    floatx4 a0[1], a1[2], sg0;
    // branch-free, so that the two interleave: on the last pass layer 0 works
    // on a stale input tile whose s0 is never read, on the first the last
    // layer on an unset S1 buffer and stores nothing
    layer0<KIND>(A0, W0s, S0, wave, lane, a0, sg0);
    last_layer(prev, 0, S1[(it + 1) & 1]);
    last_layer(prev, 1, S1[(it + 1) & 1]);
    __syncthreads();
    layer1<KIND>(S0, W1s, S1[it & 1], wave, lane, a1);
    const int64_t next = tile + G;
    // (past the last tile: zero rows into A0, for the stale last pass)
    if (tid < RT * K0 / 4) put_h0<KIND>(A0, hv, next * RT + tid / (K0 / 4) < nrows, tid);
    hv = load_h0(a, clampt(next + G), nrows, tid & 255);
    __syncthreads();
    if (!cur) break;
    prev = tile;
    tile = next;
  }
}

// Adjoint, per tile i: phase 1 = a1 of tile i recomputed (registers), dE/da2
// and dE/du of tile i, and dE/dh0 of tile i - 1 (wavefronts 0 and 1); phase 2
// = dE/ds1 -> dE/da1 of tile i into G1 and the input rows of tile i + 1 into
// A0; phase 3 = dE/ds0 -> dE/da0 of tile i into G0 and a0 of tile i + 1
// recomputed (registers, s0 into S0). A last phase 1 ends tile i - 1 alone.
template <int KIND>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_tb_bwd(Args a) {
  constexpr int H = KIND == G_BF16X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) bf16 W0s[H * N0 * L0];   // forward W0 [64][32]
  __shared__ __attribute__((aligned(16))) bf16 W1s[H * N1 * L1];   // forward W1 [128][64]
  __shared__ __attribute__((aligned(16))) bf16 B1s[H * N0 * L2];   // adjoint W1 [64][128]
  __shared__ __attribute__((aligned(16))) bf16 A0[H * RT * L0];
  __shared__ __attribute__((aligned(16))) bf16 S0[H * RT * L1];
  __shared__ __attribute__((aligned(16))) bf16 G2[H * RT * LG];    // dE/da2 (split)
  __shared__ __attribute__((aligned(16))) bf16 G1[H * RT * L2];    // dE/da1 (split)
  __shared__ __attribute__((aligned(16))) bf16 G0[H * RT * L1];    // dE/da0 (split)
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int64_t nrows = *a.nrows, ntiles = (nrows + RT - 1) / RT, G = gridDim.x;
  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  stage_w(W0s, a.w0, N0, K0, L0, H, tid);
  stage_w(W1s, a.w1, N1, N0, L1, H, tid);
  stage_w(B1s, a.b1, N0, N1, L2, H, tid);
  // register B fragments: the last layer's adjoint for column tile w of
  // dE/ds1 (K = 256), the first layer's (16 columns, K = 64)
  bf16x8 bw[N2 / 32][H], b0w[N0 / 32][H];
  load_frags(bw, a.b2, N1, N2, 16 * wave, lane);
  load_frags(b0w, a.b0, 16, N0, 0, lane);
  auto clampt = [&](int64_t t) { return t < ntiles ? t : ntiles - 1; };
  // dE/da2 inputs: wavefront w holds rows w + 8 q (q < 4), lane l their
  // 4-chunk l (columns 4 l .. 4 l + 3: K step l / 8, position l % 8 in it)
  float4 gv[4], av[4];
  float uv[4], guv[4];
  auto load_g = [&](int64_t t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t row = t * RT + wave + 8 * q;
      row = row < nrows ? row : nrows - 1;
      gv[q] = *reinterpret_cast<const float4*>(a.g + row * a.ldg + 4 * lane);
      av[q] = *reinterpret_cast<const float4*>(a.a2 + row * N2 + 4 * lane);
      uv[q] = a.u[row * a.ldu];
      guv[q] = a.gu[row];
    }
  };
  // dE/dh0 = dE/da0 W0^T of tile t (wavefronts 0 and 1: row tile w), the first n_in columns stored
  auto first_layer_adjoint = [&](int64_t t) {
    if (wave < 2) {  // (t < 0: a buffer of no rows, nothing stored)
      const int64_t row0 = t < 0 ? 0 : t * RT;
      const int nvalid = t < 0 ? 0 : (int)(nrows - row0 < RT ? nrows - row0 : RT);
      floatx4 acc[1];
      mma_reg<KIND, N0 / 32, 1, H>(G0 + wave * 16 * L1, L1, RT * L1, b0w, lane, acc);
      const __amdgpu_buffer_rsrc_t R = buffer_rsrc(a.gh0 + row0 * a.ldgh, nvalid * a.ldgh * 4);
      const int c = lane % 16;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        buf_store(acc[0][q], R, c < a.n_in ? (unsigned)((wave * 16 + orow(lane, q)) * a.ldgh + c) * 4 : kOutOfRange);
    }
  };
  load_g(tile);
  float4 hv = load_h0(a, tile, nrows, tid & 255);
  if (tid < RT * K0 / 4) put_h0<KIND>(A0, hv, tile * RT + tid / (K0 / 4) < nrows, tid);
  hv = load_h0(a, clampt(tile + G), nrows, tid & 255);
  __syncthreads();
  floatx4 a0[1], sg0;  // a0 of the current tile (column tile w % 4, row tile w / 4), its sigmoid
  layer0<KIND>(A0, W0s, S0, wave, lane, a0, sg0);
  __syncthreads();
  int64_t prev = -1;
  for (;;) {
    const bool cur = tile < ntiles;  // uniform
    const int64_t next = tile + G;
    const int64_t row0 = tile * RT;
    const int nvalid = (int)(nrows - row0 < RT ? nrows - row0 : RT);
    // a1 again (registers; S0 was written before the last barrier), beside
    // the element work of dE/da2
    floatx4 a1[2];
    layer1<KIND>(S0, W1s, nullptr, wave, lane, a1);
    {
      // dE/da2 = g u SiLU'(a2) into G2, and dE/du += sum g SiLU(a2) in the
      // per-layer kernels' order (past the last tile: stale inputs, no valid
      // rows, nothing stored)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wave + 8 * q;
        const bool ok = r < nvalid;
        const float4 g4 = gv[q], a4 = av[q];
        const float sx = sigmoidf_(a4.x), sy = sigmoidf_(a4.y), sz = sigmoidf_(a4.z), sw = sigmoidf_(a4.w);
        const float e[4] = {ok ? gradsilu_scale(g4.x, a4.x, sx, uv[q]) : 0.f, ok ? gradsilu_scale(g4.y, a4.y, sy, uv[q]) : 0.f,
                            ok ? gradsilu_scale(g4.z, a4.z, sz, uv[q]) : 0.f, ok ? gradsilu_scale(g4.w, a4.w, sw, uv[q]) : 0.f};
        put_split4<KIND>(G2, RT * LG, r * LG + 4 * lane, e);
        const float rj = row_share_sum(ok ? gradsilu_part(g4, a4, sx, sy, sz, sw) : 0.f);
        if (ok && lane == 0) a.gu[row0 + r] = guv[q] + 1.f * rj;
      }
      load_g(clampt(next));
    }
    first_layer_adjoint(prev);
    __syncthreads();
    if (!cur) break;
    // dE/ds1 = dE/da2 W2^T (column tile w, both row tiles) and
    // dE/da1 = dE/ds1 SiLU'(a1) into G1
    {
      floatx4 acc[2];
      mma_reg<KIND, N2 / 32, 2, H>(G2, LG, RT * LG, bw, lane, acc);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = i * 16 + orow(lane, q);
          const float x = a1[i][q];
          put_split<KIND>(G1, RT * L2, r * L2 + wave * 16 + lane % 16,
                          r < nvalid ? gradsilu_scale(acc[i][q], x, sigmoidf_(x), 1.f) : 0.f);
        }
    }
    if (tid < RT * K0 / 4) put_h0<KIND>(A0, hv, next * RT + tid / (K0 / 4) < nrows, tid);
    hv = load_h0(a, clampt(next + G), nrows, tid & 255);
    __syncthreads();
    // dE/ds0 = dE/da1 W1^T (column tile w % 4, row tile w / 4), then
    // dE/da0 = dE/ds0 SiLU'(a0) into G0; a0 of the next tile
    {
      const int rt = wave / 4, c0 = (wave % 4) * 16;
      floatx4 acc[1];
      mma_lds<KIND, N1 / 32, 1>(G1 + rt * 16 * L2, L2, RT * L2, B1s, L2, N0 * L2, c0, lane, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = rt * 16 + orow(lane, q);
        put_split<KIND>(G0, RT * L1, r * L1 + c0 + lane % 16,
                        r < nvalid ? gradsilu_scale(acc[0][q], a0[0][q], sg0[q], 1.f) : 0.f);
      }
    }
    // (after the last tile: a stale input tile, whose a0 and s0 are never used)
    layer0<KIND>(A0, W0s, S0, wave, lane, a0, sg0);
    __syncthreads();
    prev = tile;
    tile = next;
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

// FLOPs per edge of the three products, at the model's input width
double tb_flop(const nq_model* m) { return 2.0 * (m->dims.n_in2b * tb::N0 + tb::N0 * tb::N1 + tb::N1 * tb::N2); }

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
  // per edge: h0 and a2; the three products of the model
  const double fl = tb_flop(m);
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
  // model's three input-gradient products (the recomputed forward products
  // are not counted as the method's work)
  const double fl = tb_flop(m);
  const int sp = span_begin(ctx, "bwd.twobody", fl, 4.0 * (tb::K0 + 2 * tb::N2 + 1 + 2 + m->dims.n_in2b), 0, 0, fl);
  if (m->dims.prec == NQ_PRECISION_BF16X3)
    tb::k_tb_bwd<G_BF16X3><<<tb_grid(tb::k_tb_bwd<G_BF16X3>, ctx->num_cu, ctx->ws.cap), tb::NTH, 0, ctx->stream>>>(a);
  else
    tb::k_tb_bwd<G_BF16><<<tb_grid(tb::k_tb_bwd<G_BF16>, ctx->num_cu, ctx->ws.cap), tb::NTH, 0, ctx->stream>>>(a);
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

}  // namespace nq
