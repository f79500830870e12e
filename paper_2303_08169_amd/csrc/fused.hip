// Fused per-centre evaluation of energy and forces (gfx950): one persistent
// kernel runs the whole forward pass and its hand-written adjoint for one
// centre atom at a time and writes only E_i and g_ij = dE/dr_ij.
//
// Allegro is strictly local (paper Sec. 2.1: E is a sum of pair energies E_ij
// within the cutoff, built from equivariant features of the pair and of the
// centre's environment), so the only couplings between the edges of a centre
// are its environment sums Gamma_i (one per layer) and, in the adjoint, their
// gradients dE/dGamma_i. A workgroup owns a centre; its edges are processed in
// blocks of 64 rows, and each phase below ends where a sum over all of the
// centre's edges has to be complete:
//   F1   geometry, two-body MLP -> x0, [w0 | e1] = x0 [W_V0 | W_env1]  => Gamma_1
//   F2   tensor product (V0 = w0 Y, Gamma_1) -> s1 and mixing -> V1;
//        two-body MLP again -> x0; x1 = (x0 + u MLP([x0 | s1])) / sqrt2;
//        e2 = x1 W_env2                                                 => Gamma_2
//   F3B1 s2 from (V1, Gamma_2); x2 = (x1 + u MLP([x1 | s2])) / sqrt2;
//        edge MLP -> E_ij, E_i; then at once the adjoint of these steps:
//        dE/dx2, dE/dx1 (partial), dE/ds2 -> dE/dV1, dE/dGamma_2 shares  => dGamma_2
//   B2   dE/de2 from dGamma_2 -> dE/dx1; adjoint of the first latent MLP ->
//        dE/dx0 (partial), dE/ds1; mixing and tensor-product adjoint
//        -> dE/dw0, dE/dY, dE/dGamma_1 shares                          => dGamma_1
//   B3   dE/de1; adjoint of [W_V0 | W_env1] -> dE/dx0; two-body MLP again
//        and its adjoint -> dE/db, dE/du; geometry adjoint -> g_ij
// Within a block every matrix-core product reads its A operand from LDS
// (split into BF16 hi and lo parts once, by the producer) and its weights
// straight from global memory (L2-resident), and its epilogue writes the next
// product's A operand back into LDS, so the edge activations of a chain of
// products never leave the chip. What crosses a phase boundary (w0, e_t, s1,
// V1, x1, the latent pre-activation of layer 1 and the adjoints that cross
// dGamma) goes to a scratch region private to the workgroup, reused centre
// after centre. Every sum over edges or channels runs in a fixed order, so the
// results do not depend on timing.
//
// Compiled for the model shape of the benchmark workloads (l <= 2, two
// layers, 32 channels, two-body MLP 14 -> 64 -> 128 -> 256, one latent layer
// 352 -> 256, edge MLP 256 -> 128 -> 1); other shapes use the layered path.
#include "cg_const.hpp"
#include "gemm.hpp"
#include "mix32.hpp"
#include "nq_internal.hpp"

namespace nq {

namespace fz {

constexpr int RB = 64;        // rows (edges) per block
constexpr int AST = 360;      // LDS row stride of the A operand, BF16 elements (352 + 8)
constexpr int NTH = 512;      // threads per workgroup (8 wavefronts)
constexpr int D = 256, C = 32, NY = 9, NW = 96, NS = 3, NT = 35, K0P = 32;
constexpr int TB0 = 64, TB1 = 128, EDGE = 128, KLAT = D + NS * C;  // 352
constexpr int TCP = 36;       // LDS row stride (floats) of tensor-product components
constexpr int GL = NY * C;    // 288 floats of Gamma

// scratch columns per edge row, one region per quantity
enum : int {
  S_W0E1 = 0,            // [w0 | e1] 192
  S_V1 = S_W0E1 + 192,   // V1 288 ([lm][c])
  S_AL1 = S_V1 + 288,    // first latent pre-activation 256
  S_X1 = S_AL1 + 256,    // x1 256
  S_E2 = S_X1 + 256,     // e2 96
  S_GX1 = S_E2 + 96,     // dE/dx1 (adjoint of the second layer) 256
  S_GV1 = S_GX1 + 256,   // dE/dV1 288
  S_GX0 = S_GV1 + 288,   // dE/dx0 (adjoint of the first latent layer) 256
  S_GW0 = S_GX0 + 256,   // dE/dw0 96
  S_GYU = S_GW0 + 96,    // dE/dY (0..8), dE/du (9) 16
  S_WPR = S_GYU + 16     // 2000 floats per row
};

// One weight operand of a matrix-core product: [N][kp] BF16 hi, then lo.
struct WOp {
  const bf16* p;
  int kp;
  int64_t lo;
};

struct Args {
  int64_t n;              // atoms; every atom is a tile (atoms without edges get E_i = 0)
  int64_t n_centres;      // atoms >= n_centres are ghosts (no edges)
  const int* nedge;       // total edges of the list
  const int* eoff;        // [n + 1] CSR offsets by centre
  const int* ej;
  const float4* rij;      // (x, y, z, d) per edge
  const int32_t* species;
  int S, nb, p;
  float rc, inv_sqrt_nu, sigma;
  WOp tbf[3], tbb[3], v0f, v0b, envf, envb, latf[2], latb[2], edf, edb;
  const float* wout;
  const bf16* mixT;       // mixing weights of layer 1, transposed blocks (forward)
  const bf16* mixN;       // ... natural blocks (adjoint)
  int64_t mixlo;
  float* scratch;         // per workgroup: ksc rows x S_WPR floats
  int64_t ksc;
  float4* gr;             // dE/dr_ij per edge
  double* atomE;
  double* atom_out;       // optional copy of E_i
  int* flags;
};

struct Smem {
  // A operand, BF16 hi and lo planes (also an FP32 pool for tensor-product staging)
  __attribute__((aligned(16))) bf16 ah[RB * AST];
  __attribute__((aligned(16))) bf16 al[RB * AST];
  __attribute__((aligned(16))) float geo[RB * 16];  // per row: d, u, rhat (3), Y (9), pad
  __attribute__((aligned(16))) float gam[2][GL];    // Gamma_1, Gamma_2 of the centre ([lm][c])
  __attribute__((aligned(16))) float dg[2][GL];     // dGamma_2 (index 0), dGamma_1 (index 1), unscaled sums
  __attribute__((aligned(16))) float red[RB * 8];   // per-row partial sums of the 8 wavefronts
  __attribute__((aligned(16))) float aux[12288];    // staging (see the phases)
  double eacc;            // E_i
  Args args;              // the launch arguments (read after barriers, so not hoisted into registers)
};

// threadIdx.x through an empty asm statement: values derived from it are
// computed where they are used instead of being hoisted out of the tile loop
// (which would keep dozens of per-lane addresses live across the whole kernel).
__device__ inline int tid_() {
  int x = threadIdx.x;
  asm volatile("" : "+v"(x));
  return x;
}

// Device memory through address-space-1 pointers: the loads and stores are
// global_* instructions, counted by vmcnt only. (Pointers read from LDS are
// generic, and flat instructions also count against lgkmcnt, so every wait
// for an LDS read would drain the prefetched weight loads too.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GAS __attribute__((address_space(1)))
#else
#define GAS  // the host pass only needs the declarations
#endif
template <class T>
__device__ inline GAS T* gp(T* p) {
  return (GAS T*)p;
}

__device__ inline void sst(GAS float* p, float v) { *p = v; }
__device__ inline float sld(const GAS float* p) { return *p; }
__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ inline void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline float4 ld4(const GAS float* p) { return *reinterpret_cast<const GAS float4*>(p); }
__device__ inline void st4(GAS float* p, float4 v) { *reinterpret_cast<GAS float4*>(p) = v; }
#endif
__device__ inline float4 f4(const floatx4& v) { return make_float4(v[0], v[1], v[2], v[3]); }

// Barrier for LDS traffic only: waits for this wavefront's LDS operations,
// not for its outstanding global loads and stores (__syncthreads drains
// those too). Where one thread reads global data that another thread of the
// workgroup wrote, a full __syncthreads() separates them.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ inline float* apool(Smem& s) { return reinterpret_cast<float*>(s.ah); }

template <int KIND>
__device__ inline void put_a(Smem& s, int row, int col, float v) {
  const bf16 h = (bf16)v;
  s.ah[row * AST + col] = h;
  if constexpr (KIND == G_BF16X3) s.al[row * AST + col] = (bf16)(v - (float)h);
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
// Four consecutive A values of one row (col % 4 == 0): one 8-byte store per plane.
template <int KIND>
__device__ inline void put_a4(Smem& s, int row, int col, float4 v) {
  bf16x4 h, l;
  const float f[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h[k] = (bf16)f[k];
    l[k] = (bf16)(f[k] - (float)h[k]);
  }
  *reinterpret_cast<bf16x4*>(&s.ah[row * AST + col]) = h;
  if constexpr (KIND == G_BF16X3) *reinterpret_cast<bf16x4*>(&s.al[row * AST + col]) = l;
}

// C[rows, N] = A[rows, K] W for the nrt 16-row tiles of the block. The 8
// wavefronts form WC column groups x (8 / WC) row groups; wavefront
// (wc, wr) owns the column tiles wc, wc + WC, ... and the row tiles wr,
// wr + 8/WC, ... A comes from LDS (already split), the weight fragments
// straight from global memory one K step ahead. The matrix cores compute the
// transposed tile (weights as the first operand), so a lane ends up with one
// row and four consecutive columns: epi(i, j, row, c0, v) gets out[row][c0 + q]
// in v[q], and its stores are 8- and 16-byte chunks. Starts with a barrier
// (the caller's writes of A are visible) and ends with one before the
// epilogue (every wavefront is done reading A, so the epilogue may overwrite it).
template <int KIND, int K, int N, int WC, class EPI>
__device__ inline void gemm(Smem& s, const WOp& W, int nrt, EPI&& epi) {
  constexpr int CT = N / 16, WR = 8 / WC, CTW = (CT + WC - 1) / WC, RTW = (4 + WR - 1) / WR, KS = K / 32;
  constexpr bool X3 = KIND == G_BF16X3;
  static_assert(N % 16 == 0 && K % 32 == 0 && 8 % WC == 0, "tile shape");
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int wc = wave % WC, wr = wave / WC;
  nrt = __builtin_amdgcn_readfirstlane(nrt);
  lds_barrier();
  floatx4 acc[RTW][CTW];
#pragma unroll
  for (int i = 0; i < RTW; ++i)
#pragma unroll
    for (int j = 0; j < CTW; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const GAS bf16* bp[CTW];
#pragma unroll
  for (int j = 0; j < CTW; ++j) {
    const int ct = wc + j * WC < CT ? wc + j * WC : CT - 1;
    bp[j] = gp(W.p) + (int64_t)(ct * 16 + (lane & 15)) * W.kp + (lane >> 4) * 8;
  }
  bf16x8 bh[CTW], bl[CTW];
#pragma unroll
  for (int j = 0; j < CTW; ++j) {
    bh[j] = *reinterpret_cast<const GAS bf16x8*>(bp[j]);
    if constexpr (X3) bl[j] = *reinterpret_cast<const GAS bf16x8*>(bp[j] + W.lo);
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 nh[CTW], nl[CTW];
    if (ks + 1 < KS) {
#pragma unroll
      for (int j = 0; j < CTW; ++j) {
        nh[j] = *reinterpret_cast<const GAS bf16x8*>(bp[j] + (ks + 1) * 32);
        if constexpr (X3) nl[j] = *reinterpret_cast<const GAS bf16x8*>(bp[j] + W.lo + (ks + 1) * 32);
      }
    }
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      const int rt = wr + i * WR;
      if (rt < nrt) {
        const int off = (rt * 16 + (lane & 15)) * AST + ks * 32 + (lane >> 4) * 8;
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&s.ah[off]);
        bf16x8 al;
        if constexpr (X3) al = *reinterpret_cast<const bf16x8*>(&s.al[off]);
#pragma unroll
        for (int j = 0; j < CTW; ++j) {
          if (wc + j * WC < CT) {
            if constexpr (X3) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al, acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah, acc[i][j], 0, 0, 0);
            }
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah, acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (ks + 1 < KS) {
#pragma unroll
      for (int j = 0; j < CTW; ++j) {
        bh[j] = nh[j];
        if constexpr (X3) bl[j] = nl[j];
      }
    }
  }
  lds_barrier();
#pragma unroll
  for (int i = 0; i < RTW; ++i) {
    const int rt = wr + i * WR;
    if (rt < nrt)
#pragma unroll
      for (int j = 0; j < CTW; ++j)
        if (wc + j * WC < CT) epi(i, j, rt * 16 + (lane & 15), (wc + j * WC) * 16 + 4 * (lane >> 4), acc[i][j]);
  }
}

// Sum of a per-row value over the four lane groups (lane / 16) that hold the
// row's columns; every lane of the row gets the total.
__device__ inline float sum_row(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// One 16x16 tile of a small product whose A fragment (8 consecutive K values
// of this lane's row, FP32 in LDS) comes from `arow` and whose weight
// fragment from `brow` (K contiguous, global), over K / 32 steps.
template <int KIND, int K, class AR, class BR>
__device__ inline floatx4 small_tile(int64_t lo, AR&& arow, BR&& brow) {
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    float v[8];
    const float* a = arow(k0);
    *reinterpret_cast<float4*>(&v[0]) = *reinterpret_cast<const float4*>(a);
    *reinterpret_cast<float4*>(&v[4]) = *reinterpret_cast<const float4*>(a + 4);
    const GAS bf16* b = brow(k0);
    const bf16x8 bh = *reinterpret_cast<const GAS bf16x8*>(b);
    if constexpr (KIND == G_BF16X3) {
      const bf16x8 bl = *reinterpret_cast<const GAS bf16x8*>(b + lo);
      bf16x8 ah, al;
      split_bf16(v, ah, al);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    } else {
      bf16x8 ah;
#pragma unroll
      for (int k = 0; k < 8; ++k) ah[k] = (bf16)v[k];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    }
  }
  return acc;
}

__device__ inline void sph9(float x, float y, float z, float* Y) {
  const float s3 = 1.7320508075688772f, s5 = 2.2360679774997897f, s15 = 3.872983346207417f;
  Y[0] = 1.f;
  Y[1] = s3 * x;
  Y[2] = s3 * y;
  Y[3] = s3 * z;
  Y[4] = s15 * x * y;
  Y[5] = s15 * y * z;
  Y[6] = 0.5f * s5 * (3.f * z * z - 1.f);
  Y[7] = s15 * x * z;
  Y[8] = 0.5f * s15 * (x * x - y * y);
}

// Polynomial cutoff u(x) and du/dx in the factored form (1-x)^3 q(x), which
// keeps full relative accuracy near x = 1.
__device__ inline void cutoff(float x, int p, float& u, float& du) {
  if (x >= 1.f) {
    u = 0.f;
    du = 0.f;
    return;
  }
  float q = 0.f, xp1 = 1.f;
  for (int k = p - 1; k >= 0; --k) q = q * x + 0.5f * (float)((k + 1) * (k + 2));
  for (int k = 0; k < p - 1; ++k) xp1 *= x;
  const float om = 1.f - x;
  u = om * om * om * q;
  du = -0.5f * (float)(p * (p + 1) * (p + 2)) * xp1 * om * om;
}

__device__ inline void zero3(float (&v)[4][2][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[i][j][q] = 0.f;
}

__device__ inline int lof(int lm) { return lm >= 4 ? 2 : (lm >= 1 ? 1 : 0); }

// Per-tile context.
struct Tile {
  int64_t i;      // centre
  int e0, ne;     // first edge, edge count
  int zi;         // centre species
  GAS float* sc;  // this workgroup's scratch
  int64_t ksc;
  __device__ GAS float* q(int off, int width, int row) const { return sc + ksc * off + (int64_t)row * width; }
};

// Geometry of the block's rows (rows >= nrow are zero): d, u, rhat, Y.
__device__ inline void block_geometry(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  const int row = tid_();
  if (row < RB) {
    float* g = s.geo + row * 16;
    if (row < nrow) {
      const float4 r = gp(a.rij)[t.e0 + r0 + row];
      const float d = r.w, inv = 1.f / d;
      const float x = r.x * inv, y = r.y * inv, z = r.z * inv;
      float u, du;
      cutoff(d / a.rc, a.p, u, du);
      g[0] = d;
      g[1] = u;
      g[2] = x;
      g[3] = y;
      g[4] = z;
      sph9(x, y, z, g + 5);
      g[14] = 0.f;
      g[15] = 0.f;
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) g[k] = 0.f;
    }
  }
}

// Two-body input rows [onehot z_i | onehot z_j | B_n(d) u] into A columns 0..31.
template <int KIND>
__device__ inline void block_h0(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  const int row = tid_();
  if (row >= RB) return;
  float h[K0P];
#pragma unroll
  for (int k = 0; k < K0P; ++k) h[k] = 0.f;
  if (row < nrow) {
    const int e = t.e0 + r0 + row;
    const int zj = gp(a.species)[gp(a.ej)[e]];
    if (t.zi < 0 || t.zi >= a.S || zj < 0 || zj >= a.S) gp(a.flags)[5] = 1;
    const float d = s.geo[row * 16], u = s.geo[row * 16 + 1], inv = 1.f / d;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      h[k] = (k == t.zi) ? 1.f : 0.f;
      h[3 + k] = (k == zj) ? 1.f : 0.f;
    }
    const float pref = 2.f / a.rc, w = 3.14159265358979323846f / a.rc;
    float s1, c1;
    sincosf(w * d, &s1, &c1);
    float sn = s1, cn = c1;
#pragma unroll
    for (int n = 1; n <= 8; ++n) {
      h[5 + n] = pref * sn * inv * u;
      const float tt = sn * c1 + cn * s1;
      cn = cn * c1 - sn * s1;
      sn = tt;
    }
  }
#pragma unroll
  for (int k = 0; k < K0P; k += 4) put_a4<KIND>(s, row, k, make_float4(h[k], h[k + 1], h[k + 2], h[k + 3]));
}

// FP32 rows of a scratch quantity into A columns [c0, c0 + width).
template <int KIND, class P>
__device__ inline void stage_rows(Smem& s, P src, int width, int c0, int nrow) {
  const int cpr = width / 4;
  for (int idx = tid_(); idx < RB * cpr; idx += NTH) {
    const int row = idx / cpr, k = (idx % cpr) * 4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < nrow) v = ld4(src + (int64_t)row * width + k);
    put_a4<KIND>(s, row, c0 + k, v);
  }
}

// The two-body MLP of the block (A columns 0..31 hold its input) as far as x0:
// A = SiLU(a0), SiLU(a1), then the last layer's pre-activation goes to epi.
template <int KIND, class EPI0, class EPI1, class EPI2>
__device__ inline void twobody(const Args& a, Smem& s, int nrt, EPI0&& e0, EPI1&& e1, EPI2&& e2) {
  gemm<KIND, K0P, TB0, 4>(s, a.tbf[0], nrt, e0);
  gemm<KIND, TB0, TB1, 8>(s, a.tbf[1], nrt, e1);
  gemm<KIND, TB1, D, 8>(s, a.tbf[2], nrt, e2);
}

__device__ inline float4 silu4(const floatx4& v) { return make_float4(siluf(v[0]), siluf(v[1]), siluf(v[2]), siluf(v[3])); }

// ------------------------------------------------------------------ phases
// F1: Gamma_1 accumulated over the centre's blocks (sums in s.gam[0]).
template <int KIND>
__device__ inline void phase_f1(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  __syncthreads();  // the previous block's reads of geo and the staging areas are done
  const int nrt = (nrow + 15) / 16;
  block_geometry(a, s, t, r0, nrow);
  lds_barrier();
  block_h0<KIND>(a, s, t, r0, nrow);
  auto silu_a = [&](int, int, int row, int c0, const floatx4& v) { put_a4<KIND>(s, row, c0, silu4(v)); };
  auto x0_a = [&](int, int, int row, int c0, const floatx4& v) {
    const float u = s.geo[row * 16 + 1];
    const float4 h = silu4(v);
    put_a4<KIND>(s, row, c0, make_float4(u * h.x, u * h.y, u * h.z, u * h.w));
  };
  twobody<KIND>(a, s, nrt, silu_a, silu_a, x0_a);
  float* est = s.aux;  // e1 of the block [RB][96]
  gemm<KIND, D, 2 * NW, 4>(s, a.v0f, nrt, [&](int, int, int row, int c0, const floatx4& v) {
    const bool ok = row < nrow;
    if (ok) st4(&t.q(S_W0E1, 2 * NW, r0 + row)[c0], f4(v));
    if (c0 >= NW) st4(&est[row * NW + c0 - NW], ok ? f4(v) : make_float4(0.f, 0.f, 0.f, 0.f));
  });
  lds_barrier();
  for (int k = tid_(); k < GL; k += NTH) {
    const int lm = k / C, c = k % C, l = lof(lm);
    float acc = 0.f;
    for (int row = 0; row < nrow; ++row) acc += est[row * NW + l * C + c] * s.geo[row * 16 + 5 + lm];
    s.gam[0][k] += acc;
  }
}

// Forward mixing of one l3 for a group of 16 edges on the matrix cores:
// V[e][l3 m][c'] = sum_{p, c} T[e][toff(p) + m][c] W_l3[(p, c)][c'], rows
// (e, m), 16-column output tiles dealt round-robin to the 8 wavefronts.
template <int KIND, int L3, class OUT>
__device__ inline void mix_fwd_l3(const Args& a, const float* Tst, int& tile, int wave, int lane, OUT&& out) {
  using namespace mix32;
  constexpr int nm = 2 * L3 + 1, K = NP[L3] * C;
  const int64_t woff = (int64_t)MOFF[L3] * C * C;
#pragma unroll
  for (int rt = 0; rt < nm; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct, ++tile) {
      if ((tile & 7) != wave) continue;
      const int r = rt * 16 + (lane & 15), e = r / nm, m = r % nm, n = ct * 16 + (lane & 15);
      auto ar = [&](int k0) -> const float* { return Tst + (e * NT + TOFF[L3][k0 / C] + m) * TCP + (lane >> 4) * 8; };
      auto br = [&](int k0) -> const GAS bf16* { return gp(a.mixT) + woff + (int64_t)n * K + k0 + (lane >> 4) * 8; };
      out(L3, nm, rt, n, small_tile<KIND, K>(a.mixlo, ar, br));
    }
}

// Adjoint mixing of one l3 for a group of 16 edges:
// gT[e][toff(p) + m][c] = sum_{c'} gV[e][l3 m][c'] W_l3[(p, c)][c'].
template <int KIND, int L3>
__device__ inline void mix_bwd_l3(const Args& a, const float* gvst, float* gTst, int& tile, int wave, int lane) {
  using namespace mix32;
  constexpr int nm = 2 * L3 + 1, N = NP[L3] * C;
  const int64_t woff = (int64_t)MOFF[L3] * C * C;
#pragma unroll
  for (int rt = 0; rt < nm; ++rt)
#pragma unroll
    for (int ct = 0; ct < N / 16; ++ct, ++tile) {
      if ((tile & 7) != wave) continue;
      const int r = rt * 16 + (lane & 15), e = r / nm, m = r % nm, n = ct * 16 + (lane & 15);
      auto ar = [&](int k0) -> const float* { return gvst + (e * NY + L3 * L3 + m) * TCP + k0 + (lane >> 4) * 8; };
      auto br = [&](int k0) -> const GAS bf16* { return gp(a.mixN) + woff + (int64_t)n * C + k0 + (lane >> 4) * 8; };
      const floatx4 acc = small_tile<KIND, C>(a.mixlo, ar, br);
      const int p = ct / 2, cc = n % C;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = rt * 16 + 4 * (lane >> 4) + q;
        gTst[((rr / nm) * NT + TOFF[L3][p] + rr % nm) * TCP + cc] = acc[q];
      }
    }
}

// Sum over the 32 lanes of each half wavefront; every lane gets the total.
__device__ inline float sum32(float v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 32);
  return v;
}

// TP1 and mixing for the 16 rows g0 .. g0 + 15 of the block: s1 and V1 to scratch.
template <int KIND>
__device__ inline void tp1_fwd_group(const Args& a, Smem& s, const Tile& t, int r0, int nrow, int g0) {
  using namespace mix32;
  float* Tst = apool(s);  // [16][35][TCP]
  const int el = tid_() / C, c = tid_() % C, row = g0 + el;
  const bool valid = row < nrow;
  {
    float w0[3], V[NY], G[NY];
    const GAS float* w = t.q(S_W0E1, 2 * NW, r0 + (valid ? row : 0));
#pragma unroll
    for (int l = 0; l < 3; ++l) w0[l] = valid ? sld(&w[l * C + c]) : 0.f;
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) {
      V[lm] = w0[lof(lm)] * s.geo[row * 16 + 5 + lm];
      G[lm] = s.gam[0][lm * C + c];
    }
    float* srow = s.aux + row * NW;  // s1 of the block, staged into A after the two-body MLP
    int toff = 0, qs = 0;
#pragma unroll
    for (int l1 = 0; l1 <= 2; ++l1)
#pragma unroll
      for (int l2 = 0; l2 <= 2; ++l2)
#pragma unroll
        for (int l3 = 0; l3 <= 2; ++l3) {
          if (!cgc::natural(l1, l2, l3)) continue;
#pragma unroll
          for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
            float acc = 0.f;
#pragma unroll
            for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
#pragma unroll
              for (int m2 = 0; m2 < 2 * l2 + 1; ++m2) {
                const float cgv = kCG.v[l1][l2][l3][m1][m2][m3];
                if (cgv != 0.f) acc += cgv * V[l1 * l1 + m1] * G[l2 * l2 + m2];
              }
            Tst[(el * NT + toff + m3) * TCP + c] = valid ? acc : 0.f;
            if (l3 == 0 && valid) srow[qs * C + c] = acc;
          }
          toff += 2 * l3 + 1;
          if (l3 == 0) ++qs;
        }
  }
  lds_barrier();
  // mixing: per l3, rows (edge, m) (16 (2 l3 + 1) = 2 l3 + 1 row tiles), K = P_l3 C, N = C
  const int wave = tid_() >> 6, lane = tid_() & 63;
  int tile = 0;
  auto out = [&](int l3, int nm, int rt, int n, const floatx4& acc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = rt * 16 + 4 * (lane >> 4) + q, ee = rr / nm, mm = rr % nm;
      if (g0 + ee < nrow) sst(&t.q(S_V1, GL, r0 + g0 + ee)[(l3 * l3 + mm) * C + n], acc[q]);
    }
  };
  mix_fwd_l3<KIND, 0>(a, Tst, tile, wave, lane, out);
  mix_fwd_l3<KIND, 1>(a, Tst, tile, wave, lane, out);
  mix_fwd_l3<KIND, 2>(a, Tst, tile, wave, lane, out);
  lds_barrier();
}

// F2: V1, x1, the first latent pre-activation and e2 to scratch; Gamma_2
// accumulated in s.gam[1].
template <int KIND>
__device__ inline void phase_f2(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  __syncthreads();  // the previous block's reads of geo and the staging areas are done
  const int nrt = (nrow + 15) / 16;
  block_geometry(a, s, t, r0, nrow);
  lds_barrier();
  for (int g0 = 0; g0 < nrt * 16; g0 += 16) tp1_fwd_group<KIND>(a, s, t, r0, nrow, g0);
  block_h0<KIND>(a, s, t, r0, nrow);
  auto silu_a = [&](int, int, int row, int c0, const floatx4& v) { put_a4<KIND>(s, row, c0, silu4(v)); };
  float x0r[4][2][4];  // x0 at this lane's output positions of the 256-wide products
  zero3(x0r);
  auto x0_a = [&](int i, int j, int row, int c0, const floatx4& v) {
    const float u = s.geo[row * 16 + 1];
#pragma unroll
    for (int q = 0; q < 4; ++q) x0r[i][j][q] = u * siluf(v[q]);
    put_a4<KIND>(s, row, c0, make_float4(x0r[i][j][0], x0r[i][j][1], x0r[i][j][2], x0r[i][j][3]));
  };
  twobody<KIND>(a, s, nrt, silu_a, silu_a, x0_a);
  stage_rows<KIND>(s, s.aux, NS * C, D, nrow);  // s1 (LDS)
  gemm<KIND, KLAT, D, 8>(s, a.latf[0], nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    const float u = s.geo[row * 16 + 1];
    float x1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x1[q] = residual_update(x0r[i][j][q], u, v[q]);
    const float4 x = make_float4(x1[0], x1[1], x1[2], x1[3]);
    if (row < nrow) {
      st4(&t.q(S_AL1, D, r0 + row)[c0], f4(v));
      st4(&t.q(S_X1, D, r0 + row)[c0], x);
    }
    put_a4<KIND>(s, row, c0, x);
  });
  float* est = s.aux;
  gemm<KIND, D, NW, 2>(s, a.envf, nrt, [&](int, int, int row, int c0, const floatx4& v) {
    const bool ok = row < nrow;
    if (ok) st4(&t.q(S_E2, NW, r0 + row)[c0], f4(v));
    st4(&est[row * NW + c0], ok ? f4(v) : make_float4(0.f, 0.f, 0.f, 0.f));
  });
  lds_barrier();
  for (int k = tid_(); k < GL; k += NTH) {
    const int lm = k / C, c = k % C, l = lof(lm);
    float acc = 0.f;
    for (int row = 0; row < nrow; ++row) acc += est[row * NW + l * C + c] * s.geo[row * 16 + 5 + lm];
    s.gam[1][k] += acc;
  }
}

// F3B1: second-layer features, the edge energies and the adjoint of those
// steps; dGamma_2 shares accumulated in s.dg[0].
template <int KIND>
__device__ inline void phase_f3b1(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  __syncthreads();  // the previous block's reads of geo and the staging areas are done
  const int nrt = (nrow + 15) / 16;
  const int wave = tid_() >> 6, lane = tid_() & 63;
  block_geometry(a, s, t, r0, nrow);
  stage_rows<KIND>(s, t.q(S_X1, D, r0), D, 0, nrow);
  lds_barrier();
  // s2 (scalar paths of the last layer) into A columns 256..351
  {
    const int c = tid_() % C;
    for (int row = tid_() / C; row < nrt * 16; row += NTH / C) {
      const bool valid = row < nrow;
      const GAS float* v1 = t.q(S_V1, GL, r0 + (valid ? row : 0));
#pragma unroll
      for (int l = 0; l <= 2; ++l) {
        float acc = 0.f;
#pragma unroll
        for (int m1 = 0; m1 < 2 * l + 1; ++m1)
#pragma unroll
          for (int m2 = 0; m2 < 2 * l + 1; ++m2) {
            const float cgv = kCG.v[l][l][0][m1][m2][0];
            if (cgv != 0.f) acc += cgv * sld(&v1[(l * l + m1) * C + c]) * s.gam[1][(l * l + m2) * C + c];
          }
        put_a<KIND>(s, row, D + l * C + c, valid ? acc : 0.f);
      }
    }
  }
  float al2[4][2][4];
  zero3(al2);
  gemm<KIND, KLAT, D, 8>(s, a.latf[1], nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    const float4 x1 = row < nrow ? ld4(&t.q(S_X1, D, r0 + row)[c0]) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float u = s.geo[row * 16 + 1];
#pragma unroll
    for (int q = 0; q < 4; ++q) al2[i][j][q] = v[q];
    put_a4<KIND>(s, row, c0,
                 make_float4(residual_update(x1.x, u, v[0]), residual_update(x1.y, u, v[1]),
                             residual_update(x1.z, u, v[2]), residual_update(x1.w, u, v[3])));
  });
  // edge MLP: E_ij = sigma sum_k SiLU(a_k) w_out[k]; its adjoint into A
  gemm<KIND, D, EDGE, 8>(s, a.edf, nrt, [&](int, int, int row, int c0, const floatx4& v) {
    const float4 wo4 = ld4(gp(a.wout) + c0);
    const float wo[4] = {wo4.x, wo4.y, wo4.z, wo4.w};
    float part = 0.f, g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      part += siluf(v[q]) * wo[q];
      g[q] = gradsilu_scale(1.f, v[q], sigmoidf_(v[q]), a.sigma * wo[q]);
    }
    part = sum_row(part);
    if (lane < 16) s.red[row * 8 + wave] = part;
    put_a4<KIND>(s, row, c0, make_float4(g[0], g[1], g[2], g[3]));
  });
  lds_barrier();
  if (tid_() < 64) {  // wave 0, lane = row: E_ij, then their sum in a fixed butterfly
    const int row = tid_();
    float p = 0.f;
#pragma unroll
    for (int w = 0; w < 8; ++w) p += s.red[row * 8 + w];
    double e = row < nrow ? (double)(a.sigma * p) : 0.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) e += __shfl_xor(e, o);
    if (row == 0) s.eacc += e;
  }
  // adjoint of the edge MLP -> dE/dx2; residual adjoint into A, dE/du rows
  float gx2[4][2][4];
  zero3(gx2);
  float dur[4] = {0.f, 0.f, 0.f, 0.f};  // this lane's share of dE/du of its rows
  gemm<KIND, EDGE, D, 8>(s, a.edb, nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    const float u = s.geo[row * 16 + 1];
    float g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float al = al2[i][j][q], sg = sigmoidf_(al);
      gx2[i][j][q] = v[q];
      dur[i] += v[q] * (al * sg);
      g[q] = gradsilu_scale(v[q], al, sg, kInvSqrt2 * u);
    }
    put_a4<KIND>(s, row, c0, make_float4(g[0], g[1], g[2], g[3]));
  });
  // dE/du of the residual update: (1/sqrt2) sum_k g SiLU(a)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float p = sum_row(dur[i]);
    if (lane < 16 && i < nrt) s.red[(i * 16 + lane) * 8 + wave] = p;
  }
  lds_barrier();
  if ((int)tid_() < nrow) {
    float p = 0.f;
#pragma unroll
    for (int w = 0; w < 8; ++w) p += s.red[tid_() * 8 + w];
    sst(&t.q(S_GYU, 16, r0 + tid_())[9], kInvSqrt2 * p);
  }
  // adjoint of the second latent layer: dE/dx1 (scratch), dE/ds2 (LDS)
  float* gs2 = s.aux;  // [RB][96]
  gemm<KIND, D, KLAT, 8>(s, a.latb[1], nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    if (j < 2) {
      const int jj = j < 2 ? j : 0;
      if (row < nrow)
        st4(&t.q(S_GX1, D, r0 + row)[c0],
            make_float4(residual_adjoint(gx2[i][jj][0], v[0]), residual_adjoint(gx2[i][jj][1], v[1]),
                        residual_adjoint(gx2[i][jj][2], v[2]), residual_adjoint(gx2[i][jj][3], v[3])));
    } else if (c0 >= D) {
      st4(&gs2[row * NW + c0 - D], f4(v));
    }
  });
  lds_barrier();
  // adjoint of the scalar paths: dE/dV1 (scratch), dGamma_2 shares
  float* dgst = s.aux + RB * NW;  // [16][288]
  const int el = tid_() / C, c = tid_() % C;
  for (int g0 = 0; g0 < nrt * 16; g0 += 16) {
    const int row = g0 + el;
    const bool valid = row < nrow;
    const GAS float* v1 = t.q(S_V1, GL, r0 + (valid ? row : 0));
    float gV[NY], gG[NY];
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) gV[lm] = gG[lm] = 0.f;
#pragma unroll
    for (int l = 0; l <= 2; ++l) {
      const float g = valid ? gs2[row * NW + l * C + c] : 0.f;
#pragma unroll
      for (int m1 = 0; m1 < 2 * l + 1; ++m1)
#pragma unroll
        for (int m2 = 0; m2 < 2 * l + 1; ++m2) {
          const float cgv = kCG.v[l][l][0][m1][m2][0];
          if (cgv != 0.f) {
            const float w = cgv * g;
            gV[l * l + m1] += w * s.gam[1][(l * l + m2) * C + c];
            gG[l * l + m2] += w * sld(&v1[(l * l + m1) * C + c]);
          }
        }
    }
    if (valid) {
      GAS float* gv = t.q(S_GV1, GL, r0 + row);
#pragma unroll
      for (int lm = 0; lm < NY; ++lm) sst(&gv[lm * C + c], gV[lm]);
    }
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) dgst[el * GL + lm * C + c] = valid ? gG[lm] : 0.f;
    lds_barrier();
    for (int k = tid_(); k < GL; k += NTH) {
      float acc = 0.f;
#pragma unroll
      for (int e = 0; e < 16; ++e) acc += dgst[e * GL + k];
      s.dg[0][k] += acc;
    }
    lds_barrier();
  }
}

// Environment-sum adjoint for one layer (dg: unscaled dGamma sums, esrc: the
// layer's e rows in scratch): dE/de into A columns c0 .. c0 + 95, and the
// layer's share of dE/dY added to the scratch rows (or stored when first).
template <int KIND>
__device__ inline void env_adjoint(const Args& a, Smem& s, const Tile& t, int r0, int nrow, const float* dg,
                                   const GAS float* esrc, int lde, int c0, bool first) {
  const float sc = a.inv_sqrt_nu;
  for (int idx = tid_(); idx < RB * NW; idx += NTH) {
    const int row = idx / NW, k = idx % NW, l = k / C, c = k % C;
    float ge = 0.f;
    if (row < nrow) {
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) ge += dg[(l * l + m) * C + c] * s.geo[row * 16 + 5 + l * l + m];
    }
    put_a<KIND>(s, row, c0 + k, sc * ge);
  }
  for (int idx = tid_(); idx < RB * NY; idx += NTH) {
    const int row = idx / NY, lm = idx % NY, l = lof(lm);
    if (row >= nrow) continue;
    const GAS float* e = esrc + (int64_t)(r0 + row) * lde + l * C;
    float acc = 0.f;
    for (int c = 0; c < C; ++c) acc += sld(&e[c]) * dg[lm * C + c];
    GAS float* gy = t.q(S_GYU, 16, r0 + row) + lm;
    sst(gy, first ? sc * acc : sld(gy) + sc * acc);
  }
}

// Mixing adjoint and TP1 adjoint for the 16 rows g0 .. g0 + 15 of the block:
// dE/dw0 to scratch, the w0 share of dE/dY, dGamma_1 shares into s.dg[1].
template <int KIND>
__device__ inline void tp1_bwd_group(const Args& a, Smem& s, const Tile& t, int r0, int nrow, int g0) {
  using namespace mix32;
  float* gs1 = s.aux;                // [RB][96] dE/ds1
  float* gvst = s.aux + RB * NW;     // [16][9][TCP] dE/dV1, then [16][288] dGamma shares
  float* gTst = apool(s);            // [16][35][TCP]
  const int el = tid_() / C, c = tid_() % C, row = g0 + el;
  const bool valid = row < nrow;
  {
    const GAS float* gv = t.q(S_GV1, GL, r0 + (valid ? row : 0));
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) gvst[(el * NY + lm) * TCP + c] = valid ? sld(&gv[lm * C + c]) : 0.f;
  }
  lds_barrier();
  const int wave = tid_() >> 6, lane = tid_() & 63;
  int tile = 0;
  mix_bwd_l3<KIND, 0>(a, gvst, gTst, tile, wave, lane);
  mix_bwd_l3<KIND, 1>(a, gvst, gTst, tile, wave, lane);
  mix_bwd_l3<KIND, 2>(a, gvst, gTst, tile, wave, lane);
  lds_barrier();
  float gV[NY], gG[NY], V[NY], Y[NY], G[NY], w0[3];
  const GAS float* w = t.q(S_W0E1, 2 * NW, r0 + (valid ? row : 0));
#pragma unroll
  for (int l = 0; l < 3; ++l) w0[l] = valid ? sld(&w[l * C + c]) : 0.f;
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) {
    Y[lm] = s.geo[row * 16 + 5 + lm];
    V[lm] = w0[lof(lm)] * Y[lm];
    G[lm] = s.gam[0][lm * C + c];
    gV[lm] = gG[lm] = 0.f;
  }
  {
    int toff = 0, qs = 0;
#pragma unroll
    for (int l1 = 0; l1 <= 2; ++l1)
#pragma unroll
      for (int l2 = 0; l2 <= 2; ++l2)
#pragma unroll
        for (int l3 = 0; l3 <= 2; ++l3) {
          if (!cgc::natural(l1, l2, l3)) continue;
#pragma unroll
          for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
            float g = gTst[(el * NT + toff + m3) * TCP + c];
            if (l3 == 0) g += valid ? gs1[row * NW + qs * C + c] : 0.f;
#pragma unroll
            for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
#pragma unroll
              for (int m2 = 0; m2 < 2 * l2 + 1; ++m2) {
                const float cgv = kCG.v[l1][l2][l3][m1][m2][m3];
                if (cgv != 0.f) {
                  const float wv = cgv * g;
                  gV[l1 * l1 + m1] += wv * G[l2 * l2 + m2];
                  gG[l2 * l2 + m2] += wv * V[l1 * l1 + m1];
                }
              }
          }
          toff += 2 * l3 + 1;
          if (l3 == 0) ++qs;
        }
  }
  // V0 = w0 Y: dE/dw0 per (l, c) and the channel sums of w0 dE/dV0 for dE/dY
  GAS float* gwr = t.q(S_GW0, NW, r0 + (valid ? row : 0));
  GAS float* gyr = t.q(S_GYU, 16, r0 + (valid ? row : 0));
#pragma unroll
  for (int l = 0; l <= 2; ++l) {
    float gw = 0.f;
#pragma unroll
    for (int m = 0; m < 2 * l + 1; ++m) {
      gw += gV[l * l + m] * Y[l * l + m];
      const float part = sum32(w0[l] * gV[l * l + m]);
      if (c == 31 && valid) sst(&gyr[l * l + m], sld(&gyr[l * l + m]) + part);
    }
    if (valid) sst(&gwr[l * C + c], gw);
  }
  lds_barrier();  // every wave is done with gvst before the dGamma shares overwrite it
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) gvst[el * GL + lm * C + c] = valid ? gG[lm] : 0.f;
  lds_barrier();
  for (int k = tid_(); k < GL; k += NTH) {
    float acc = 0.f;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc += gvst[e * GL + k];
    s.dg[1][k] += acc;
  }
  lds_barrier();
}

// B2: dE/dx0 (partial) and dE/dw0 to scratch, dE/dY and dE/du added; dGamma_1
// shares accumulated in s.dg[1].
template <int KIND>
__device__ inline void phase_b2(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  __syncthreads();  // the previous block's reads of geo and the staging areas are done
  const int nrt = (nrow + 15) / 16;
  const int wave = tid_() >> 6, lane = tid_() & 63;
  block_geometry(a, s, t, r0, nrow);
  lds_barrier();
  env_adjoint<KIND>(a, s, t, r0, nrow, s.dg[0], t.q(S_E2, NW, 0), NW, 0, true);
  // adjoint of e2 = x1 W_env2 plus the second layer's dE/dx1, then the first
  // latent layer's residual adjoint into A
  float gx1[4][2][4];
  zero3(gx1);
  float dur[4] = {0.f, 0.f, 0.f, 0.f};
  gemm<KIND, NW, D, 8>(s, a.envb, nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    const bool ok = row < nrow;
    const float4 gp4 = ok ? ld4(&t.q(S_GX1, D, r0 + row)[c0]) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 al4 = ok ? ld4(&t.q(S_AL1, D, r0 + row)[c0]) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float gpv[4] = {gp4.x, gp4.y, gp4.z, gp4.w}, alv[4] = {al4.x, al4.y, al4.z, al4.w};
    const float f = kInvSqrt2 * s.geo[row * 16 + 1];
    float g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float gg = v[q] + gpv[q], sg = sigmoidf_(alv[q]);
      gx1[i][j][q] = gg;
      dur[i] += gg * (alv[q] * sg);
      g[q] = gradsilu_scale(gg, alv[q], sg, f);
    }
    put_a4<KIND>(s, row, c0, make_float4(g[0], g[1], g[2], g[3]));
  });
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float p = sum_row(dur[i]);
    if (lane < 16 && i < nrt) s.red[(i * 16 + lane) * 8 + wave] = p;
  }
  lds_barrier();
  if ((int)tid_() < nrow) {
    float p = 0.f;
#pragma unroll
    for (int w = 0; w < 8; ++w) p += s.red[tid_() * 8 + w];
    GAS float* p_ = &t.q(S_GYU, 16, r0 + tid_())[9];
    sst(p_, sld(p_) + kInvSqrt2 * p);
  }
  float* gs1 = s.aux;  // [RB][96]
  gemm<KIND, D, KLAT, 8>(s, a.latb[0], nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    if (j < 2) {
      const int jj = j < 2 ? j : 0;
      if (row < nrow)
        st4(&t.q(S_GX0, D, r0 + row)[c0],
            make_float4(residual_adjoint(gx1[i][jj][0], v[0]), residual_adjoint(gx1[i][jj][1], v[1]),
                        residual_adjoint(gx1[i][jj][2], v[2]), residual_adjoint(gx1[i][jj][3], v[3])));
    } else if (c0 >= D) {
      st4(&gs1[row * NW + c0 - D], f4(v));
    }
  });
  __syncthreads();  // full: the dE/dY rows stored above are added to by other threads
  for (int g0 = 0; g0 < nrt * 16; g0 += 16) tp1_bwd_group<KIND>(a, s, t, r0, nrow, g0);
}

// B3: dE/dx0 complete, the two-body adjoint and g_ij.
template <int KIND>
__device__ inline void phase_b3(const Args& a, Smem& s, const Tile& t, int r0, int nrow) {
  __syncthreads();  // the previous block's reads of geo and the staging areas are done
  const int nrt = (nrow + 15) / 16;
  const int wave = tid_() >> 6, lane = tid_() & 63;
  block_geometry(a, s, t, r0, nrow);
  lds_barrier();
  block_h0<KIND>(a, s, t, r0, nrow);
  float* a0st = s.aux;             // [RB][64] first two-body pre-activation
  float* a1st = s.aux + RB * TB0;  // [RB][128]
  float a2[4][2][4];
  zero3(a2);
  auto e0 = [&](int, int, int row, int c0, const floatx4& v) {
    st4(&a0st[row * TB0 + c0], f4(v));
    put_a4<KIND>(s, row, c0, silu4(v));
  };
  auto e1 = [&](int, int, int row, int c0, const floatx4& v) {
    st4(&a1st[row * TB1 + c0], f4(v));
    put_a4<KIND>(s, row, c0, silu4(v));
  };
  auto e2 = [&](int i, int j, int, int, const floatx4& v) {
#pragma unroll
    for (int q = 0; q < 4; ++q) a2[i][j][q] = v[q];
  };
  twobody<KIND>(a, s, nrt, e0, e1, e2);
  // A = [dE/dw0 | dE/de1]
  stage_rows<KIND>(s, t.q(S_GW0, NW, r0), NW, 0, nrow);
  env_adjoint<KIND>(a, s, t, r0, nrow, s.dg[1], t.q(S_W0E1, 2 * NW, 0) + NW, 2 * NW, NW, false);
  float dur[4] = {0.f, 0.f, 0.f, 0.f};
  gemm<KIND, 2 * NW, D, 8>(s, a.v0b, nrt, [&](int i, int j, int row, int c0, const floatx4& v) {
    const float4 gp4 = row < nrow ? ld4(&t.q(S_GX0, D, r0 + row)[c0]) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float gpv[4] = {gp4.x, gp4.y, gp4.z, gp4.w};
    const float u = s.geo[row * 16 + 1];
    float g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float gg = v[q] + gpv[q], al = a2[i][j][q], sg = sigmoidf_(al);
      dur[i] += gg * (al * sg);
      g[q] = gradsilu_scale(gg, al, sg, u);
    }
    put_a4<KIND>(s, row, c0, make_float4(g[0], g[1], g[2], g[3]));
  });
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float p = sum_row(dur[i]);
    if (lane < 16 && i < nrt) s.red[(i * 16 + lane) * 8 + wave] = p;
  }
  lds_barrier();
  if ((int)tid_() < nrow) {
    float p = 0.f;
#pragma unroll
    for (int w = 0; w < 8; ++w) p += s.red[tid_() * 8 + w];
    GAS float* p_ = &t.q(S_GYU, 16, r0 + tid_())[9];
    sst(p_, sld(p_) + p);
  }
  auto adj = [&](const float* ast, int width) {
    return [&s, ast, width](int, int, int row, int c0, const floatx4& v) {
      const float4 al4 = ld4(&ast[row * width + c0]);
      const float alv[4] = {al4.x, al4.y, al4.z, al4.w};
      float g[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) g[q] = gradsilu_scale(v[q], alv[q], sigmoidf_(alv[q]), 1.f);
      put_a4<KIND>(s, row, c0, make_float4(g[0], g[1], g[2], g[3]));
    };
  };
  gemm<KIND, D, TB1, 8>(s, a.tbb[2], nrt, adj(a1st, TB1));
  gemm<KIND, TB1, TB0, 4>(s, a.tbb[1], nrt, adj(a0st, TB0));
  float* gh0 = s.aux;  // [RB][16] dE/d(two-body input)
  gemm<KIND, TB0, 16, 1>(s, a.tbb[0], nrt, [&](int, int, int row, int c0, const floatx4& v) {
    st4(&gh0[row * 16 + c0], f4(v));
  });
  __syncthreads();  // full: the dE/dY and dE/du rows were written by other threads
  // geometry adjoint: g_ij from dE/db, dE/du, dE/dY
  const int row = tid_();
  if (row < nrow) {
    const float* g = s.geo + row * 16;
    const float d = g[0], x = g[2], y = g[3], z = g[4];
    float u, dudx;
    cutoff(d / a.rc, a.p, u, dudx);
    const GAS float* gyu = t.q(S_GYU, 16, r0 + row);
    float gut = sld(&gyu[9]), gd = 0.f;
    const float pref = 2.f / a.rc, w = 3.14159265358979323846f / a.rc, inv = 1.f / d;
    float s1, c1;
    sincosf(w * d, &s1, &c1);
    float sn = s1, cs = c1;
#pragma unroll
    for (int n = 1; n <= 8; ++n) {
      const float k = n * w;
      const float B = pref * sn * inv;
      const float dB = pref * (k * cs * inv - sn * inv * inv);
      const float gb = gh0[row * 16 + 5 + n];
      gut += gb * B;
      gd += gb * u * dB;
      const float tt = sn * c1 + cs * s1;
      cs = cs * c1 - sn * s1;
      sn = tt;
    }
    gd += gut * dudx / a.rc;
    float gY[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) gY[k] = sld(&gyu[k]);
    const float s3 = 1.7320508075688772f, s5 = 2.2360679774997897f, s15 = 3.872983346207417f;
    const float ax = s3 * gY[1] + s15 * (y * gY[4] + z * gY[7] + x * gY[8]);
    const float ay = s3 * gY[2] + s15 * (x * gY[4] + z * gY[5] - y * gY[8]);
    const float az = s3 * gY[3] + s15 * (y * gY[5] + x * gY[7]) + 3.f * s5 * z * gY[6];
    const float rad = ax * x + ay * y + az * z;
    gp(a.gr)[t.e0 + r0 + row] = make_float4(gd * x + (ax - rad * x) * inv, gd * y + (ay - rad * y) * inv,
                                            gd * z + (az - rad * z) * inv, 0.f);
  }
}

template <int KIND>
__global__ __launch_bounds__(NTH) void k_fused(Args ka) {
  __shared__ Smem s;
  {
    const unsigned* src = reinterpret_cast<const unsigned*>(&ka);
    unsigned* dst = reinterpret_cast<unsigned*>(&s.args);
    for (int k = tid_(); k < (int)(sizeof(Args) / 4); k += NTH) dst[k] = src[k];
  }
  __syncthreads();
  const Args& a = s.args;
  const int ne_all = __builtin_amdgcn_readfirstlane(*gp(a.nedge));
  Tile t;
  t.sc = gp(a.scratch) + (int64_t)blockIdx.x * a.ksc * S_WPR;
  t.ksc = a.ksc;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    t.i = i;
    const bool centre = i < a.n_centres;
    // uniform values in scalar registers: branches on them stay scalar, so the
    // compiler's wait counts for the products' prefetched loads stay exact
    t.e0 = __builtin_amdgcn_readfirstlane(centre ? min(gp(a.eoff)[i], ne_all) : 0);
    t.ne = __builtin_amdgcn_readfirstlane(centre ? min(gp(a.eoff)[i + 1], ne_all) - t.e0 : 0);
    if (t.ne > a.ksc) {
      if (tid_() == 0) atomicMax(a.flags + 4, t.ne);  // (rare error path)
      t.ne = 0;
    }
    t.zi = __builtin_amdgcn_readfirstlane(gp(a.species)[i]);
    for (int k = tid_(); k < 2 * GL; k += NTH) {
      (&s.gam[0][0])[k] = 0.f;
      (&s.dg[0][0])[k] = 0.f;
    }
    if (tid_() == 0) s.eacc = 0.0;
    __syncthreads();
    if (t.ne > 0) {
      for (int r0 = 0; r0 < t.ne; r0 += RB) phase_f1<KIND>(a, s, t, r0, min(RB, t.ne - r0));
      __syncthreads();
      for (int k = tid_(); k < GL; k += NTH) s.gam[0][k] *= a.inv_sqrt_nu;
      for (int r0 = 0; r0 < t.ne; r0 += RB) phase_f2<KIND>(a, s, t, r0, min(RB, t.ne - r0));
      __syncthreads();
      for (int k = tid_(); k < GL; k += NTH) s.gam[1][k] *= a.inv_sqrt_nu;
      for (int r0 = 0; r0 < t.ne; r0 += RB) phase_f3b1<KIND>(a, s, t, r0, min(RB, t.ne - r0));
      __syncthreads();
      for (int r0 = 0; r0 < t.ne; r0 += RB) phase_b2<KIND>(a, s, t, r0, min(RB, t.ne - r0));
      __syncthreads();
      for (int r0 = 0; r0 < t.ne; r0 += RB) phase_b3<KIND>(a, s, t, r0, min(RB, t.ne - r0));
    }
    __syncthreads();
    if (tid_() == 0) {
      gp(a.atomE)[i] = s.eacc;
      if (a.atom_out) gp(a.atom_out)[i] = s.eacc;
    }
  }
}

}  // namespace fz

// True when the fused kernel is compiled for this model (one precision for
// every product: no per-product overrides).
bool fused_supported(const nq_model* m) {
  const Dims& d = m->dims;
  return d.L == 2 && d.T == 2 && d.C == 32 && d.S == 3 && d.nb == 8 && d.n_tb == 3 && d.tb[0] == fz::TB0 &&
         d.tb[1] == fz::TB1 && d.tb[2] == fz::D && d.n_lat == 1 && d.lat[0] == fz::D && d.n_edge == 1 &&
         d.edge[0] == fz::EDGE && (d.prec == NQ_PRECISION_BF16 || d.prec == NQ_PRECISION_BF16X3) &&
         m->site_prec.empty();
}

namespace {
fz::WOp wop(const Lin& L, bool bwd) {
  const int kp = bwd ? L.kp_b : L.kp_f, np = bwd ? L.np_b : L.np_f;
  return fz::WOp{(bwd ? L.bf_bwd : L.bf_fwd).as<bf16>(), kp, (int64_t)np * kp};
}
}  // namespace

void fused_prepare(nq_ctx* ctx) {
  const size_t need = (size_t)ctx->num_cu * std::max(ctx->nl.k_max, 1) * fz::S_WPR * 4;
  if (ctx->fz_scratch.bytes >= need) return;
  NQ_HIP(hipStreamSynchronize(ctx->stream));
  ctx->fz_scratch.release();
  ctx->fz_scratch.ensure(need);
  ++ctx->gen;
}

void fused_async(nq_ctx* ctx, const nq_model* m, const int32_t* species, double* atom_energy, int64_t n_centres) {
  const Dims& d = m->dims;
  Workspace& ws = ctx->ws;
  NbrList& nl = ctx->nl;
  const int64_t n = ws.n_atoms;
  fz::Args a{};
  a.n = n;
  a.n_centres = n_centres < 0 ? n : n_centres;
  a.nedge = ws.nedge.as<int>();
  a.eoff = ws.eoff.as<int>();
  a.ej = ws.ej.as<int>();
  a.rij = ws.rij.as<float4>();
  a.species = species;
  a.S = d.S;
  a.nb = d.nb;
  a.p = d.p;
  a.rc = (float)d.rc;
  a.inv_sqrt_nu = (float)d.inv_sqrt_nu;
  a.sigma = (float)d.sigma_e;
  for (int k = 0; k < 3; ++k) {
    a.tbf[k] = wop(*m->tb[k], false);
    a.tbb[k] = wop(*m->tb[k], true);
  }
  a.v0f = wop(m->v0e1, false);
  a.v0b = wop(m->v0e1, true);
  a.envf = wop(*m->env[1], false);
  a.envb = wop(*m->env[1], true);
  for (int t = 0; t < 2; ++t) {
    a.latf[t] = wop(*m->lat[t][0], false);
    a.latb[t] = wop(*m->lat[t][0], true);
  }
  a.edf = wop(*m->edge[0], false);
  a.edb = wop(*m->edge[0], true);
  a.wout = m->wout.as<float>();
  a.mixT = m->mixw[0]->bT.as<bf16>();
  a.mixN = m->mixw[0]->bN.as<bf16>();
  a.mixlo = m->mixw[0]->n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ctx->num_cu, n));
  a.ksc = std::max(nl.k_max, 1);
  NQ_REQUIRE(ctx->fz_scratch.bytes >= (size_t)grid * a.ksc * fz::S_WPR * 4, NQ_ERR_DEVICE,
             "fused-kernel scratch not prepared");
  a.scratch = ctx->fz_scratch.as<float>();
  a.gr = ws.grbuf.as<float4>();
  a.atomE = ws.atomE;
  a.atom_out = atom_energy;
  a.flags = nl.flags.as<int>();
  const int sp = span_begin(ctx, "fused", 0, 0, 0, 0, 0);
  if (d.prec == NQ_PRECISION_BF16X3)
    fz::k_fused<G_BF16X3><<<grid, fz::NTH, 0, ctx->stream>>>(a);
  else
    fz::k_fused<G_BF16><<<grid, fz::NTH, 0, ctx->stream>>>(a);
  span_end(ctx, sp);
  NQ_HIP(hipGetLastError());
}

}  // namespace nq
