// Energy and force pipeline of the Allegro-style edge model (gfx950).
//
// The model (paper Sec. 2.1: pairwise embedding energies E_ij within a cutoff,
// E(3)-equivariant tensors up to rank l, tensor products of irreducible
// representations; forces f = -dE/dr, Eq. 1) is evaluated as a chain of
// edge-batched stages over the directed edges sorted by centre atom:
//   geometry   d, rhat, cutoff u, Bessel basis b, spherical harmonics Y
//   two-body   MLP on [onehot z_i | onehot z_j | b], x0 = u * h        (matrix cores)
//   features   [w0 | e1] = x0 [W_V0 | W_env^1]                          (matrix cores)
//   layer t    Gamma_i = nu^-1/2 sum_k e_ik (x) Y_ik   (one wavefront per centre)
//              T = C (V (x) Gamma_i), s = scalar paths (one thread per edge-channel)
//              V_t = mixing of T across channels and paths (t < T)
//              x_t = (x_{t-1} + u MLP([x_{t-1} | s])) / sqrt2            (matrix cores)
//              e_{t+1} = x_t W_env^{t+1}                                (matrix cores)
//   energy     E_ij = sigma_E (SiLU(x_T W_e) w_out); E_i, E (compensated FP64)
// and then its hand-written adjoint in reverse order, which yields
// g_ij = dE/dr_ij per edge; the force on atom a is gathered as
// sum over its edges of g(a,j) - g(j,a) through the reverse-edge index, so no
// atomics are needed and the result is deterministic.
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "cg_const.hpp"
#include "gemm.hpp"
#include "mix32.hpp"
#include "nq_internal.hpp"

namespace nq {

namespace {

constexpr int kGeo = 16;  // geo row: d, u, rhat(3), Y(9), pad
constexpr int kGeoY = 5;


// Real spherical harmonics, component normalised, order l=1: (x,y,z);
// l=2: (xy, yz, 3z^2-1, xz, x^2-y^2) with the factors below.
__device__ inline void sph(float x, float y, float z, float* Y) {
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

// Polynomial cutoff u(x) and du/dx, x = d / r_c. The polynomial
// 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2) has a triple root at
// x = 1 and equals (1-x)^3 * sum_{k<p} (k+1)(k+2)/2 x^k; that factored form
// keeps full relative accuracy near the cutoff, where the expanded one cancels.
__device__ inline void envelope(float x, int p, float& u, float& du) {
  if (x >= 1.f) {
    u = 0.f;
    du = 0.f;
    return;
  }
  float q = 0.f, xp1 = 1.f;  // xp1 = x^(p-1)
  for (int k = p - 1; k >= 0; --k) q = q * x + 0.5f * (float)((k + 1) * (k + 2));
  for (int k = 0; k < p - 1; ++k) xp1 *= x;
  const float om = 1.f - x;
  u = om * om * om * q;
  du = -0.5f * (float)(p * (p + 1) * (p + 2)) * xp1 * om * om;
}

// ------------------------------------------------------------------ geometry
// One thread per edge computes the edge's geometry row and two-body input
// row into LDS (rows padded by one word: no bank conflicts); the block then
// writes its rows as contiguous 16-byte chunks (stored directly, a thread's
// rows are 64 and 128 bytes apart: one 4-byte store per value, the lanes
// of a store 64 or 128 bytes apart).
__global__ __launch_bounds__(256) void k_geometry(const int* __restrict__ nedge_p, const float4* __restrict__ rij,
                                                  const int* __restrict__ ei, const int* __restrict__ ej, int64_t a0,
                                                  const int32_t* __restrict__ species, int S, int nb, int p, float rc,
                                                  int K0p, float* __restrict__ geo, float* __restrict__ h0,
                                                  int* __restrict__ flags) {
  extern __shared__ float gl_lds[];  // [256][kGeo + 1], then [256][K0p + 1]
  const int t = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * 256, ne = *nedge_p;
  if (e0 >= ne) return;  // the whole block
  const int nrow = (int)(ne - e0 < 256 ? ne - e0 : 256);
  float* g = gl_lds + t * (kGeo + 1);
  float* h = gl_lds + 256 * (kGeo + 1) + t * (K0p + 1);
  if (t < nrow) {
    const int64_t e = e0 + t;
    const float4 r = rij[e];
    const float d = r.w, inv = 1.f / d;
    const float x = r.x * inv, y = r.y * inv, z = r.z * inv;
    float u, du;
    envelope(d / rc, p, u, du);
    float Y[9];
    sph(x, y, z, Y);
    g[0] = d;
    g[1] = u;
    g[2] = x;
    g[3] = y;
    g[4] = z;
#pragma unroll
    for (int k = 0; k < 9; ++k) g[kGeoY + k] = Y[k];
    g[14] = 0.f;
    g[15] = 0.f;
    const int zi = species[a0 + ei[e]], zj = species[ej[e]];
    if (zi < 0 || zi >= S || zj < 0 || zj >= S) flags[5] = 1;
    for (int k = 0; k < S; ++k) {
      h[k] = (k == zi) ? 1.f : 0.f;
      h[S + k] = (k == zj) ? 1.f : 0.f;
    }
    const float pref = 2.f / rc, w = 3.14159265358979323846f / rc;
    // sin(n w d) for n = 1..nb by the angle-addition recurrence from one sincos
    float s1, c1;
    sincosf(w * d, &s1, &c1);
    float sn = s1, cn = c1;
    for (int n = 1; n <= nb; ++n) {
      h[2 * S + n - 1] = pref * sn * inv * u;
      const float tt = sn * c1 + cn * s1;
      cn = cn * c1 - sn * s1;
      sn = tt;
    }
    for (int k = 2 * S + nb; k < K0p; ++k) h[k] = 0.f;
  }
  __syncthreads();
  constexpr int GC = kGeo / 4;
  for (int i = t; i < nrow * GC; i += 256) {
    const int rr = i / GC, c = (i % GC) * 4;
    const float* src = gl_lds + rr * (kGeo + 1) + c;
    *reinterpret_cast<float4*>(geo + (e0 + rr) * kGeo + c) = make_float4(src[0], src[1], src[2], src[3]);
  }
  const int HC = K0p / 4;
  for (int i = t; i < nrow * HC; i += 256) {
    const int rr = i / HC, c = (i % HC) * 4;
    const float* src = gl_lds + 256 * (kGeo + 1) + rr * (K0p + 1) + c;
    *reinterpret_cast<float4*>(h0 + (e0 + rr) * K0p + c) = make_float4(src[0], src[1], src[2], src[3]);
  }
}

// ------------------------------------------------------------------ environment sums
// One wavefront per centre i; lane = (channel c, group g), group g owns the
// components lm = g, g+G, ... of Gamma_i[lm][c] (G = 64 / C). The centre's edges
// are taken four at a time with all their loads issued before the sums, and
// components past NY read a valid one and are dropped, so no load sits behind
// a lane-dependent branch.
template <int NY, int C>
__global__ __launch_bounds__(256) void k_env_fwd(int64_t n, const int* __restrict__ nedge_p, const int* __restrict__ eoff,
                                                 const float* __restrict__ esrc, int lde,
                                                 const float* __restrict__ geo, float scale,
                                                 float* __restrict__ gam) {
  constexpr int G = 64 / C, NQ = (NY + G - 1) / G, U = 4;
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= n) return;
  const int lane = threadIdx.x % 64;
  const int c = lane % C, g = lane / C;
  int lmq[NQ], lq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int lm = min(g + q * G, NY - 1);
    lmq[q] = lm;
    lq[q] = lm >= 4 ? 2 : (lm >= 1 ? 1 : 0);
  }
  float acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.f;
  const int ne = *nedge_p;
  const int b = min(eoff[i], ne), e1 = min(eoff[i + 1], ne);
  int e = b;
  for (; e + U <= e1; e += U) {
    float ev[U][NQ], yv[U][NQ];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        ev[u][q] = esrc[(int64_t)(e + u) * lde + lq[q] * C + c];
        yv[u][q] = geo[(int64_t)(e + u) * kGeo + kGeoY + lmq[q]];
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] += ev[u][q] * yv[u][q];
  }
  for (; e < e1; ++e)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      acc[q] += esrc[(int64_t)e * lde + lq[q] * C + c] * geo[(int64_t)e * kGeo + kGeoY + lmq[q]];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    if (g + q * G < NY) gam[(i * NY + g + q * G) * C + c] = acc[q] * scale;
}

// ------------------------------------------------------------------ group sums
constexpr int spread_len(int n, int rounds) {
  for (int r = 0; r < rounds; ++r) n = (n + 1) / 2;
  return n;
}

// Sums N values per lane over each aligned group of W lanes (W a power of two
// dividing 64) by recursive halving: every round trades the half of the
// remaining components this lane does not keep for the partner's copy of the
// half it keeps, so the N sums take about N + log2(W) shuffles instead of
// N log2(W). Afterwards slot s < count of this lane holds the group total of
// component first + s, and every component is held by exactly one lane.
template <int N, int W>
__device__ inline void spread_sum(float (&v)[N], int lane, int& first, int& count) {
  first = 0;
  int len = N;
#pragma unroll
  for (int r = 0; (W >> (r + 1)) >= 1; ++r) {
    const int m = W >> (r + 1);
    const int L = spread_len(N, r), H = (L + 1) / 2;
    const bool up = (lane & m) != 0;
    float nv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) nv[i] = 0.f;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float hi = H + i < L ? v[H + i] : 0.f;
      const float send = up ? v[i] : hi;
      nv[i] = (up ? hi : v[i]) + __shfl_xor(send, m, W);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = nv[i];
    if (up) {
      first += H;
      len -= H;
    } else {
      len = len < H ? len : H;
    }
  }
  count = len > 0 ? len : 0;
}

// Sum of v over each aligned group of 32 lanes with DPP lane moves (no LDS
// round trips): pair, quad, half-row mirror, row mirror, then row 1 (3) adds
// row 0's (2's) lane 15. The total is valid in lanes 16..31 and 48..63.
template <int CTRL, int ROWS>
__device__ inline float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROWS, 0xF, false));
}
__device__ inline float sum32_dpp(float v) {
  v += dpp_mov<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_mov<0x140, 0xF>(v);  // row_mirror
  v += dpp_mov<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  return v;
}

// dst[k] += sum over the C lanes of the group (lane index c) of v[k], k < N.
template <int N>
__device__ inline void add_group_sums(float (&v)[N], int C, int c, float* dst) {
  int first = 0, count = 0;
  switch (C) {
    case 8: spread_sum<N, 8>(v, c, first, count); break;
    case 16: spread_sum<N, 16>(v, c, first, count); break;
    case 32: spread_sum<N, 32>(v, c, first, count); break;
    default: spread_sum<N, 64>(v, c, first, count); break;
  }
#pragma unroll
  for (int k = 0; k < N; ++k)
    if (k < count) dst[first + k] += v[k];
}

// ------------------------------------------------------------------ tensor products
// Compile-time walk over the coupling paths (l1,l2,l3) of one layer in
// lexicographic order. `f(l1,l2,l3,toff,qscal,pidx_in_l3)` is called for each
// path that is needed (all paths, or only l3 == 0 when `scalar_only`); toff is
// the path's offset in the full list of T components, so all offsets are
// compile-time constants after unrolling.
template <int LMAX, class F>
__device__ inline void for_paths(bool scalar_only, F&& f) {
  int toff = 0, qs = 0;
  int pcount[3] = {0, 0, 0};
#pragma unroll
  for (int l1 = 0; l1 <= LMAX; ++l1)
#pragma unroll
    for (int l2 = 0; l2 <= LMAX; ++l2)
#pragma unroll
      for (int l3 = 0; l3 <= LMAX; ++l3) {
        const bool ok = (l1 - l2 <= l3) && (l2 - l1 <= l3) && (l3 <= l1 + l2) && ((l1 + l2 + l3) % 2 == 0);
        if (ok) {
          if (!scalar_only || l3 == 0) f(l1, l2, l3, toff, qs, pcount[l3]);
          toff += 2 * l3 + 1;
          if (l3 == 0) qs++;
          pcount[l3]++;
        }
      }
}

template <int LMAX> struct TPSize {
  static constexpr int NY = (LMAX + 1) * (LMAX + 1);
  static constexpr int NT = LMAX == 1 ? 8 : 35;  // sum over paths of (2 l3 + 1)
};

// Raw loads of V_{t-1} for one (edge, channel), with no arithmetic on the
// loaded values, so the loads of a prefetched group stay in flight until the
// group is processed. First layer: V0[lm] = w0[l] Y[lm] is formed at use
// (vprev_value) from R = Y and W = w0; later layers: R = V_{t-1} (W reads R's
// row and is unused). One 64-bit row address per source, components at fixed
// offsets from it; the uniform selects keep the loads branch-free.
template <int NY, int NL>
__device__ inline void load_vprev(bool first, int64_t e, int c, int C, const float* we1, int ldwe,
                                  const float* vprev, const float* Y, float (&R)[NY], float (&W)[NL]) {
  const float* v = vprev + e * (NY * C) + c;
  const float* rb = first ? Y : v;
  const int rs = first ? 1 : C;
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) R[lm] = rb[lm * rs];
  const float* wb = first ? we1 + e * ldwe + c : v;
  const int ws = first ? C : 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) W[l] = wb[l * ws];
}
template <int NY, int NL>
__device__ inline float vprev_value(bool first, const float (&R)[NY], const float (&W)[NL], int lm) {
  const int l = lm >= 4 ? 2 : (lm >= 1 ? 1 : 0);
  return first ? W[l] * R[lm] : R[lm];
}

// Coupling paths of one l3 group: count, offsets of their components in the
// full T list, and the offset of the group's mixing block (in units of C*C).
struct PathInfo {
  int np[3];
  int toff[3][4];
  int moff[3];
};

template <int LMAX>
constexpr PathInfo make_path_info() {
  PathInfo pi{};
  int toff = 0;
  for (int l1 = 0; l1 <= LMAX; ++l1)
    for (int l2 = 0; l2 <= LMAX; ++l2)
      for (int l3 = 0; l3 <= LMAX; ++l3)
        if ((l1 - l2 <= l3) && (l2 - l1 <= l3) && (l3 <= l1 + l2) && ((l1 + l2 + l3) % 2 == 0)) {
          pi.toff[l3][pi.np[l3]++] = toff;
          toff += 2 * l3 + 1;
        }
  int o = 0;
  for (int l3 = 0; l3 <= LMAX; ++l3) {
    pi.moff[l3] = o;
    o += pi.np[l3];
  }
  return pi;
}

template <int LMAX> struct Paths {
  static constexpr PathInfo pi = make_path_info<LMAX>();
};

// Channel-mixing weights of one layer as the matrix-core kernels read them.
struct MixPtrs {
  const float* fN;   // FP32 [(p, c)][c'] per l3 block
  const float* fT;   // FP32 [c'][(p, c)] per l3 block
  const bf16* bN;    // BF16 hi | lo, natural
  const bf16* bT;    // BF16 hi | lo, transposed
  int64_t n;         // elements per copy (offset of the lo half)
};

__device__ inline void load8(const float* p, float* v) {
  *reinterpret_cast<float4*>(&v[0]) = *reinterpret_cast<const float4*>(p);
  *reinterpret_cast<float4*>(&v[4]) = *reinterpret_cast<const float4*>(p + 4);
}

__device__ inline bf16x8 to_bf16x8(const float* v) {
  bf16x8 r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r[k] = (bf16)v[k];
  return r;
}

// Dynamic LDS of the tensor-product kernels: the edge group's T (forward) or
// gV and gT (adjoint), rows padded to C + 4 floats.
extern __shared__ __attribute__((aligned(16))) float nq_dyn_lds[];

// One 16x16 output tile of a small product on the matrix cores, accumulating
// over K: A(r, k) comes from `afetch(k)` (this lane's row, 1 or 8 values from
// LDS), B(k, n) from `bptr(k)` (this lane's column, contiguous in k, global).
template <int KIND, class AF, class BP>
__device__ inline floatx4 tile_mma(int K, int lane, int64_t lo_off, bool bvalid, AF&& afetch, BP&& bptr) {
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (KIND == G_F32) {
    for (int kk = 0; kk < K; kk += 4) {
      const int k = kk + (lane >> 4);
      float a = 0.f, b = 0.f;
      if (k < K) {
        afetch(k, &a);
        if (bvalid) b = *static_cast<const float*>(bptr(k));
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  } else {
    for (int kk = 0; kk < K; kk += 32) {
      const int k = kk + (lane >> 4) * 8;
      float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bf16x8 bhi = {}, blo = {};
      if (k < K) {
        afetch(k, v);
        if (bvalid) {
          const bf16* bp = static_cast<const bf16*>(bptr(k));
          bhi = *reinterpret_cast<const bf16x8*>(bp);
          if constexpr (KIND == G_BF16X3) blo = *reinterpret_cast<const bf16x8*>(bp + lo_off);
        }
      }
      if constexpr (KIND == G_BF16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(to_bf16x8(v), bhi, acc, 0, 0, 0);
      } else {
        bf16x8 ahi, alo;
        split_bf16(v, ahi, alo);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
      }
    }
  }
  return acc;
}

// Forward channel mixing of one edge group on the matrix cores. For each l3:
// rows (edge, m), K = (path p, channel c), columns c':
// V_t[e][l3 m][c'] = sum_{p, c} T[e][toff(p) + m][c] W_l3[(p, c)][c'].
template <int KIND, int LMAX>
__device__ inline void mix_fwd(const float* Tl, int epb, int C, int64_t e0, int64_t ne, const MixPtrs& W,
                               float* __restrict__ vout) {
  constexpr int NY = (LMAX + 1) * (LMAX + 1), NT = LMAX == 1 ? 8 : 35;
  const PathInfo& pi = Paths<LMAX>::pi;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int tile = 0;
#pragma unroll
  for (int l3 = 0; l3 <= LMAX; ++l3) {
    const int nm = 2 * l3 + 1, R = epb * nm, RT = (R + 15) / 16, CT = (C + 15) / 16, K = pi.np[l3] * C;
    const int64_t woff = (int64_t)pi.moff[l3] * C * C;
    for (int rt = 0; rt < RT; ++rt)
      for (int ct = 0; ct < CT; ++ct, ++tile) {
        if ((tile & 3) != wave) continue;
        const int r = rt * 16 + (lane & 15);
        const bool rv = r < R;
        const int el = rv ? r / nm : 0, m = rv ? r % nm : 0;
        const int n = ct * 16 + (lane & 15);
        auto af = [&](int k, float* v) {
          if (!rv) return;
          const float* src = Tl + (el * NT + pi.toff[l3][k / C] + m) * (C + 4) + (k % C);
          if constexpr (KIND == G_F32) v[0] = *src; else load8(src, v);
        };
        auto bp = [&](int k) -> const void* {
          const int64_t o = woff + (int64_t)n * K + k;
          if constexpr (KIND == G_F32) return W.fT + o;
          else return W.bT + o;
        };
        const floatx4 acc = tile_mma<KIND>(K, lane, W.n, n < C, af, bp);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = rt * 16 + 4 * (lane >> 4) + q;
          if (rr < R && n < C) {
            const int64_t e = e0 + rr / nm;
            if (e < ne) vout[(e * NY + l3 * l3 + rr % nm) * C + n] = acc[q];
          }
        }
      }
  }
}

// Adjoint of the channel mixing for one edge group, into LDS:
// gT[e][toff(p) + m][c] = sum_{c'} gV[e][l3 m][c'] W_l3[(p, c)][c'].
template <int KIND, int LMAX>
__device__ inline void mix_bwd(const float* gVl, float* gTl, int epb, int C, const MixPtrs& W) {
  constexpr int NY = (LMAX + 1) * (LMAX + 1), NT = LMAX == 1 ? 8 : 35;
  const PathInfo& pi = Paths<LMAX>::pi;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int tile = 0;
#pragma unroll
  for (int l3 = 0; l3 <= LMAX; ++l3) {
    const int nm = 2 * l3 + 1, R = epb * nm, RT = (R + 15) / 16, N = pi.np[l3] * C, CT = (N + 15) / 16;
    const int64_t woff = (int64_t)pi.moff[l3] * C * C;
    for (int rt = 0; rt < RT; ++rt)
      for (int ct = 0; ct < CT; ++ct, ++tile) {
        if ((tile & 3) != wave) continue;
        const int r = rt * 16 + (lane & 15);
        const bool rv = r < R;
        const int el = rv ? r / nm : 0, m = rv ? r % nm : 0;
        const int n = ct * 16 + (lane & 15);
        auto af = [&](int k, float* v) {
          if (!rv) return;
          const float* src = gVl + (el * NY + l3 * l3 + m) * (C + 4) + k;
          if constexpr (KIND == G_F32) v[0] = *src; else load8(src, v);
        };
        auto bp = [&](int k) -> const void* {
          const int64_t o = woff + (int64_t)n * C + k;
          if constexpr (KIND == G_F32) return W.fN + o;
          else return W.bN + o;
        };
        const floatx4 acc = tile_mma<KIND>(C, lane, W.n, n < N, af, bp);
        const int p = n / C, c = n % C;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = rt * 16 + 4 * (lane >> 4) + q;
          if (rr < R && n < N) gTl[((rr / nm) * NT + pi.toff[l3][p] + rr % nm) * (C + 4) + c] = acc[q];
        }
      }
  }
}

static_assert(Paths<2>::pi.toff[0][0] == mix32::TOFF[0][0] && Paths<2>::pi.toff[0][1] == mix32::TOFF[0][1] &&
                  Paths<2>::pi.toff[0][2] == mix32::TOFF[0][2] && Paths<2>::pi.toff[1][0] == mix32::TOFF[1][0] &&
                  Paths<2>::pi.toff[1][1] == mix32::TOFF[1][1] && Paths<2>::pi.toff[1][2] == mix32::TOFF[1][2] &&
                  Paths<2>::pi.toff[1][3] == mix32::TOFF[1][3] && Paths<2>::pi.toff[2][0] == mix32::TOFF[2][0] &&
                  Paths<2>::pi.toff[2][1] == mix32::TOFF[2][1] && Paths<2>::pi.toff[2][2] == mix32::TOFF[2][2] &&
                  Paths<2>::pi.toff[2][3] == mix32::TOFF[2][3] && Paths<2>::pi.moff[1] == mix32::MOFF[1] &&
                  Paths<2>::pi.moff[2] == mix32::MOFF[2] && TPSize<2>::NT == mix32::NT,
              "path layout of the 32-channel mixing plan");

// LDS bytes of one tensor-product workgroup: rows of C + 4 floats for the
// group's (256 / C) edges x (NT, plus NY for the adjoint) components.
inline size_t tp_lds_bytes(int C, int L, bool adjoint) {
  const int NT = L == 1 ? 8 : 35, NY = (L + 1) * (L + 1);
  // the adjoint adds two buffers of the group's edge centres (run sums); the
  // forward's T rows are C + 4 floats, or two rows of C + 8 BF16 values
  // (the adjoint's dE/dV rows likewise: two rows of C + 8 BF16 values)
  if (!adjoint) return (size_t)(256 / C) * NT * (C + 8) * sizeof(float);
  return (size_t)(256 / C) * ((C + 8) * NY + (C + 4) * NT + 2) * sizeof(float);
}
// Dynamic LDS of the last layer's 32-channel adjoint: two alternating buffers
// of the group's dE/dGamma contributions and of its edge centres.
inline size_t tp_last_lds_bytes(int C, int L) {
  const int NY = (L + 1) * (L + 1);
  return (size_t)(256 / C) * (2 * NY * (C + 4) + 2) * sizeof(float);
}

struct TpFwdArgs {
  const int* nedge_p;
  const int* ei;
  const float* geo;
  int C, first, last;
  const float* we1;
  int ldwe;
  const float* vprev;
  const float* gam;
  float* s;
  int lds;
  MixPtrs W;
  float* vout;
};

// Inputs of the forward product of one (edge, channel): V_{t-1} (raw, see
// load_vprev) and Gamma_i.
template <int LMAX> struct TpFwdIn {
  static constexpr int NY = TPSize<LMAX>::NY;
  float V[NY], W[LMAX + 1], G[NY];
};

// ctr: the edge's centre (its index load issued a group earlier, so the Gamma
// loads do not wait on it).
template <int LMAX, int CC>
__device__ inline void tp_fwd_load(const TpFwdArgs& a, int64_t e, int ctr, int c, TpFwdIn<LMAX>& in) {
  constexpr int NY = TPSize<LMAX>::NY;
  const int C = CC > 0 ? CC : a.C;
  load_vprev(a.first, e, c, C, a.we1, a.ldwe, a.vprev, a.geo + e * kGeo + kGeoY, in.V, in.W);
  const float* g = a.gam + (int64_t)ctr * (NY * C) + c;
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) in.G[lm] = g[lm * C];
}

// T = C (V (x) Gamma_i) for one (edge, channel), path by path (zero
// coefficients skipped at compile time): each component goes straight to the
// edge's LDS rows Trow (stride CP; zero for a row past the last edge), the
// scalar paths also to s through a buffer over the group's valid rows S (the
// edge is row el of the group; stores past them are dropped, so no branch
// makes the compiler's wait counts for the prefetched loads inexact). CC:
// channel count if known at compile time, else 0.
// TS: the LDS form of T: 0 FP32 rows (stride CP floats); 1 BF16 rows, 2 BF16
// hi rows and, tlo elements further, lo rows (stride CP BF16 values), split
// here once instead of by every wavefront that reads them for the mixing.
template <int LMAX, int CC, int TS = 0>
__device__ inline void tp_fwd_edge(const TpFwdArgs& a, __amdgpu_buffer_rsrc_t S, int el, bool valid, int c,
                                   void* Trow, int CP, const TpFwdIn<LMAX>& in, int tlo = 0) {
  const int C = CC > 0 ? CC : a.C;
  constexpr int NY = TPSize<LMAX>::NY;
  float V[NY];
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) V[lm] = vprev_value(a.first, in.V, in.W, lm);
  const unsigned srow = (unsigned)(el * a.lds + c) * 4;
  for_paths<LMAX>(a.last, [&](int l1, int l2, int l3, int toff, int qs, int) {
#pragma unroll
    for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
      float acc = 0.f;
#pragma unroll
      for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
#pragma unroll
        for (int m2 = 0; m2 < 2 * l2 + 1; ++m2) {
          const float cgv = kCG.v[l1][l2][l3][m1][m2][m3];
          if (cgv != 0.f) acc += cgv * V[l1 * l1 + m1] * in.G[l2 * l2 + m2];
        }
      if (Trow) {  // (null: no mixing follows)
        const float v = valid ? acc : 0.f;
        if constexpr (TS == 0) {
          static_cast<float*>(Trow)[(toff + m3) * CP + c] = v;
        } else {
          bf16* tr = static_cast<bf16*>(Trow) + (toff + m3) * CP + c;
          const bf16 h = (bf16)v;
          tr[0] = h;
          if constexpr (TS == 2) tr[tlo] = (bf16)(v - (float)h);
        }
      }
      if (l3 == 0) buf_store(acc, S, srow + (unsigned)(qs * C) * 4);
    }
  });
}

// Persistent loop of one wavefront over groups of (256 / C) edges x C
// channels: one thread per (edge, channel) computes T, the group's T is staged
// in LDS and mixed across channels and paths on the matrix cores. MW < 0: the
// output tiles are dealt round-robin to the 4 waves and the weights read per
// tile; MW = 0..3: the wave's fixed tiles of the l <= 2, 32-channel plan, with
// their weight fragments loaded once into registers.
template <int KIND, int LMAX, int MW>
__device__ inline void tp_fwd_loop(const TpFwdArgs& a) {
  constexpr int NT = TPSize<LMAX>::NT;
  // MW = -2: the last layer (no mixing) of a 32-channel model
  constexpr int CC = MW >= 0 || MW == -2 ? mix32::C : 0;
  const int C = CC > 0 ? CC : a.C;
  // the 32-channel plan keeps T in LDS already split into the BF16 operand(s)
  // of the mixing (rows of CPH values); otherwise as FP32 rows of CP floats
  constexpr int TS = MW >= 0 && KIND != G_F32 ? (KIND == G_BF16X3 ? 2 : 1) : 0;
  const int epb = 256 / C, CP = C + 4, CPH = C + 8;
  const int el = threadIdx.x / C, c = threadIdx.x % C, lane = threadIdx.x & 63;
  float* Tl = nq_dyn_lds;
  bf16* Th = reinterpret_cast<bf16*>(nq_dyn_lds);
  const int tlo = epb * NT * CPH;  // lo rows after the hi rows
  const int64_t ne = *a.nedge_p;
  const int64_t ngroups = (ne + epb - 1) / epb;
  mix32::FwdB<KIND, (MW < 0 ? 0 : MW)> B;
  if constexpr (MW >= 0) {
    if (!a.last) B.load(KIND == G_F32 ? static_cast<const void*>(a.W.fT) : a.W.bT, a.W.n, lane);
  }
  // Software pipeline over the workgroup's groups: the next group's inputs are
  // loaded while this group is mixed. A row past the last edge reads the last
  // edge and contributes zeros.
  // The centre index of a group is loaded one group earlier still.
  auto edge_of = [&](int64_t g) {
    const int64_t eg = g * epb + el;
    return eg < ne ? eg : ne - 1;
  };
  auto clampg = [&](int64_t g) { return g < ngroups ? g : ngroups - 1; };
  auto issue = [&](int64_t g, int ctr, TpFwdIn<LMAX>& inr) {
    tp_fwd_load<LMAX, CC>(a, edge_of(g), ctr, c, inr);
  };
  TpFwdIn<LMAX> in;
  int64_t grp = blockIdx.x;
  int ctr = 0;
  if (grp < ngroups) {
    issue(grp, a.ei[edge_of(grp)], in);
    ctr = a.ei[edge_of(clampg(grp + gridDim.x))];
  }
  for (; grp < ngroups; grp += gridDim.x) {
    const int64_t e = grp * epb + el, e0 = grp * epb;
    const __amdgpu_buffer_rsrc_t S = buffer_rsrc(a.s + e0 * a.lds, (ne - e0 < epb ? ne - e0 : epb) * a.lds * 4);
    if constexpr (TS == 0)
      tp_fwd_edge<LMAX, CC, 0>(a, S, el, e < ne, c, MW == -2 ? nullptr : Tl + el * NT * CP, CP, in);
    else
      tp_fwd_edge<LMAX, CC, TS>(a, S, el, e < ne, c, Th + el * NT * CPH, CPH, in, tlo);
    issue(clampg(grp + gridDim.x), ctr, in);
    ctr = a.ei[edge_of(clampg(grp + 2 * gridDim.x))];
    if (MW == -2 || a.last) continue;
    __syncthreads();
    if constexpr (TS > 0)
      mix32::mix_fwd_split<KIND, MW>(B, Th, tlo, grp * epb, ne, a.vout, lane);
    else if constexpr (MW >= 0)
      mix32::mix_fwd<KIND, MW>(B, Tl, grp * epb, ne, a.vout, lane);
    else
      mix_fwd<KIND, LMAX>(Tl, epb, C, grp * epb, ne, a.W, a.vout);
    __syncthreads();
  }
}

// Last layer of a 32-channel l <= 2 model (no mixing; see k_tp_bwd_last32).
template <int KIND>
__global__ __launch_bounds__(256) void k_tp_fwd_last32(TpFwdArgs a) {
  tp_fwd_loop<KIND, 2, -2>(a);
}

// Forward tensor product of one layer: s (scalar paths) and, for t < T, the
// mixed features V_t. C32: the l <= 2, 32-channel model, each wave running its
// own mixing plan (the wave index is uniform, every wave passes the same
// barriers).
template <int KIND, int LMAX, bool C32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_tp_fwd(TpFwdArgs a) {
  if constexpr (C32) {
    static_assert(LMAX == 2, "the 32-channel plan is for l <= 2");
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
      case 0: tp_fwd_loop<KIND, LMAX, 0>(a); break;
      case 1: tp_fwd_loop<KIND, LMAX, 1>(a); break;
      case 2: tp_fwd_loop<KIND, LMAX, 2>(a); break;
      default: tp_fwd_loop<KIND, LMAX, 3>(a); break;
    }
  } else {
    tp_fwd_loop<KIND, LMAX, -1>(a);
  }
}

// ------------------------------------------------------------------ energy
// E_ij = sigma_E * sum_k SiLU(a[k]) w_out[k]; 16 lanes per edge.
__global__ __launch_bounds__(256) void k_edge_energy(const int* __restrict__ nedge_p, const float* __restrict__ a,
                                                     int lda, int K, const float* __restrict__ wout, float sigma,
                                                     float* __restrict__ eij) {
  const int64_t e = (int64_t)blockIdx.x * 16 + threadIdx.x / 16;
  const int l = threadIdx.x % 16;
  float acc = 0.f;
  const bool valid = e < *nedge_p;
  // 16-byte loads (K and lda are multiples of 16), two chunks in flight
  if (valid) {
#pragma unroll 2
    for (int k = 4 * l; k < K; k += 64) {
      const float4 v = *reinterpret_cast<const float4*>(a + e * lda + k);
      const float4 w = *reinterpret_cast<const float4*>(wout + k);
      acc += siluf(v.x) * w.x + siluf(v.y) * w.y + siluf(v.z) * w.z + siluf(v.w) * w.w;
    }
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 16);
  if (valid && l == 0) eij[e] = sigma * acc;
}

__global__ void k_atom_energy(int64_t n, const int* __restrict__ nedge_p, const int* __restrict__ eoff,
                              const float* __restrict__ eij, double* __restrict__ atomE, double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int ne = *nedge_p;
  double s = 0.0;
  for (int e = min(eoff[a], ne); e < min(eoff[a + 1], ne); ++e) s += (double)eij[e];
  atomE[a] = s;
  if (out) out[a] = s;
}

// True when the device has flagged a condition that makes this evaluation's
// results wrong (a truncated neighbour row or edge list, a non-finite
// coordinate or coincident atoms, a species out of range): the outputs are
// then poisoned with NaN, so an error reported only at the next nq_stats is
// still visible in the results.
__device__ inline bool results_invalid(const int* flags) {
  return (flags[0] > 0) | (flags[2] != 0) | (flags[4] > 0) | (flags[5] != 0);
}

// Neumaier-compensated FP64 sums of consecutive segments of n values, one
// block per segment (one segment per replica): energy[b] = sum of v[b n, (b+1) n).
__global__ __launch_bounds__(1024) void k_total_energy(int64_t n, const double* __restrict__ v,
                                                       double* __restrict__ energy, const int* __restrict__ flags) {
  __shared__ double hs[1024], hc[1024];
  double s = 0.0, c = 0.0;
  v += (int64_t)blockIdx.x * n;
  energy += blockIdx.x;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const double x = v[k];
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  hs[threadIdx.x] = s;
  hc[threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double a = hs[threadIdx.x], b = hs[threadIdx.x + o];
      const double t = a + b;
      const double err = (fabs(a) >= fabs(b)) ? (a - t) + b : (b - t) + a;
      hs[threadIdx.x] = t;
      hc[threadIdx.x] += hc[threadIdx.x + o] + err;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[0] = results_invalid(flags) ? __builtin_nan("") : hs[0] + hc[0];
}

// ------------------------------------------------------------------ adjoint helpers
__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

struct TpBwdArgs {
  const int* nedge_p;
  const int* e0p;  // global index of edge 0 (the chunk's first edge)
  const int* ei;
  const float* geo;
  int C, first, last;
  const float* we1;
  int ldwe;
  const float* vprev;
  const float* gam;
  const float* gs;
  int ldgs;
  const float* gvin;
  MixPtrs W;
  float* ggc;
  float* gvout;
  float* gew;
  int ldgew;
  float* gY;
  int ldgy;
};

// Workgroup barrier that waits for this wavefront's LDS accesses only: global
// loads in flight (the next group's inputs) stay in flight across it.
__device__ inline void tp_lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Inputs of the adjoint of one (edge, channel) that do not depend on the
// mixing adjoint: V_{t-1}, Gamma_i and dE/ds. They are loaded before the
// group's mixing so that their HBM latency overlaps it.
template <int LMAX> struct TpBwdIn {
  static constexpr int NY = TPSize<LMAX>::NY, NS = LMAX + 1;  // scalar paths: (l, l, 0)
  float V[NY], W[LMAX + 1], G[NY], gs[NS];
};

// ctr as in tp_fwd_load.
template <int LMAX, int CC>
__device__ inline void tp_bwd_load(const TpBwdArgs& a, int64_t e, int ctr, int c, TpBwdIn<LMAX>& in) {
  constexpr int NY = TPSize<LMAX>::NY;
  const int C = CC > 0 ? CC : a.C;
  load_vprev(a.first, e, c, C, a.we1, a.ldwe, a.vprev, a.geo + e * kGeo + kGeoY, in.V, in.W);
  const float* g = a.gam + (int64_t)ctr * (NY * C) + c;
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) in.G[lm] = g[lm * C];
  const float* gsr = a.gs + e * a.ldgs + c;
#pragma unroll
  for (int q = 0; q <= LMAX; ++q) in.gs[q] = gsr[q * C];
}

// Adjoint of the tensor product of one (edge, channel), given dE/dT from the
// mixing adjoint (gTrow: this edge's rows in LDS, unused for the last layer)
// and dE/ds. Writes the edge's contributions to dE/dGamma_i into LDS
// (red[lm * CP + c]: only this thread reads or writes these words before the
// next barrier; the caller sums them over the runs of equal centres), and
// either dE/dV_{t-1} (t > 1) or, for t = 1, dE/dw0 into gew[:, 0:NW] and
// the w0 part of dE/dY into slot 0 of the edge's dE/dY row (a plain store:
// the geometry adjoint adds the slots, and a read-modify-write here would wait
// on every outstanding load of the next group). CC: channel count if known at
// compile time.
template <int LMAX, int CC>
__device__ inline void tp_bwd_edge(const TpBwdArgs& a, int64_t e0, int lo, int hi, int el, int c,
                                   const float* gTrow, int CP, const TpBwdIn<LMAX>& in, float* red) {
  constexpr int NY = TPSize<LMAX>::NY;
  const int C = CC > 0 ? CC : a.C;
  float gV[NY], gG[NY], V[NY];
#pragma unroll
  for (int k = 0; k < NY; ++k) {
    gV[k] = 0.f;
    gG[k] = 0.f;
    V[k] = vprev_value(a.first, in.V, in.W, k);
  }
  for_paths<LMAX>(a.last, [&](int l1, int l2, int l3, int toff, int qs, int) {
#pragma unroll
    for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
      float g = a.last ? 0.f : gTrow[(toff + m3) * CP + c];
      if (l3 == 0) g += in.gs[qs];
#pragma unroll
      for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
#pragma unroll
        for (int m2 = 0; m2 < 2 * l2 + 1; ++m2) {
          const float cgv = kCG.v[l1][l2][l3][m1][m2][m3];
          if (cgv != 0.f) {
            const float w = cgv * g;
            gV[l1 * l1 + m1] += w * in.G[l2 * l2 + m2];
            gG[l2 * l2 + m2] += w * V[l1 * l1 + m1];
          }
        }
    }
  });
  if constexpr (CC == 32) {
    // 32-channel plan (called for valid rows only): plain stores, which keep
    // its register peak lower than buffer offsets do
    const int64_t e = e0 + el;
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) red[lm * CP + c] = gG[lm];
    if (!a.first) {
      float* gvr = a.gvout + e * (NY * C) + c;
#pragma unroll
      for (int lm = 0; lm < NY; ++lm) gvr[lm * C] = gV[lm];
    } else {
      // (the first layer's raw inputs: in.V holds Y, in.W holds w0)
      float* gwr = a.gew + e * a.ldgew + c;
      float* gYr = a.gY + e * a.ldgy;
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        float gw = 0.f;
        const float w0 = in.W[l];
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          gw += gV[l * l + m] * in.V[l * l + m];
          const float part = sum32_dpp(w0 * gV[l * l + m]);
          if (c == 31) gYr[l * l + m] = part;
        }
        gwr[l * C] = gw;
      }
    }
  } else {
    // stores through buffers over the group's valid rows lo .. hi - 1 (edge
    // e0 + el; a row outside them is dropped: its offset, negative before lo,
    // wraps past the range), so no branch guards them
    const int r = el - lo;
    const int64_t eb = e0 + lo;
    const int nval = hi - lo;
    const unsigned rowc = (unsigned)((r * NY * C + c) * 4);
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) red[lm * CP + c] = gG[lm];
    if (!a.first) {
      const __amdgpu_buffer_rsrc_t GV = buffer_rsrc(a.gvout + eb * (NY * C), (int64_t)nval * NY * C * 4);
#pragma unroll
      for (int lm = 0; lm < NY; ++lm) buf_store(gV[lm], GV, rowc + (unsigned)(lm * C) * 4);
    } else {
      // V0[c][lm] = w0[l][c] Y[lm]; each component's channel sum is reduced
      // right away (gathering them first raises the register peak)
      const __amdgpu_buffer_rsrc_t GW = buffer_rsrc(a.gew + eb * a.ldgew, (int64_t)nval * a.ldgew * 4);
      const __amdgpu_buffer_rsrc_t GY = buffer_rsrc(a.gY + eb * a.ldgy, (int64_t)nval * a.ldgy * 4);
      const unsigned gwo = (unsigned)((r * a.ldgew + c) * 4), gyo = (unsigned)(r * a.ldgy * 4);
#pragma unroll
      for (int l = 0; l <= LMAX; ++l) {
        float gw = 0.f;
        const float w0 = in.W[l];
#pragma unroll
        for (int m = 0; m < 2 * l + 1; ++m) {
          gw += gV[l * l + m] * in.V[l * l + m];
          float part = w0 * gV[l * l + m];
          for (int o = C / 2; o >= 1; o >>= 1) part += __shfl_xor(part, o, C);
          buf_store(part, GY, c == 0 ? gyo + (unsigned)(l * l + m) * 4 : kOutOfRange);
        }
        buf_store(gw, GW, gwo + (unsigned)(l * C) * 4);
      }
    }
  }
}

// Persistent loop of one wavefront of the adjoint: the group's dE/dV_t is
// staged in LDS, mixed back to dE/dT on the matrix cores (MW as in
// tp_fwd_loop), then each thread runs the adjoint of its (edge, channel).
template <int KIND, int LMAX, int MW>
__device__ inline void tp_bwd_loop(const TpBwdArgs& a) {
  constexpr int NY = TPSize<LMAX>::NY, NT = TPSize<LMAX>::NT;
  // MW = -2: the last layer (no mixing) of a 32-channel model
  constexpr int CC = MW >= 0 || MW == -2 ? mix32::C : 0;
  constexpr bool LAST = MW == -2;
  const int C = CC > 0 ? CC : a.C;
  // the 32-channel plan stages dE/dV already split into the BF16 operand(s)
  // of the mixing adjoint (rows of CPH values: hi, then lo gtlo further);
  // otherwise as FP32 rows of CP floats. The region holds either.
  constexpr int GS = MW >= 0 && KIND != G_F32 ? (KIND == G_BF16X3 ? 2 : 1) : 0;
  const int epb = 256 / C, CP = C + 4, CPH = C + 8;
  const int el = threadIdx.x / C, c = threadIdx.x % C, lane = threadIdx.x & 63;
  float* gVl = nq_dyn_lds;
  bf16* gVh = reinterpret_cast<bf16*>(nq_dyn_lds);
  const int gtlo = epb * NY * CPH;  // lo rows after the hi rows
  float* gTl = nq_dyn_lds + epb * NY * CPH;
  const int64_t ne = *a.nedge_p;
  // groups of epb edges start at multiples of epb of the global edge index
  // (edge e of a chunk is edge e0 + e of the system), so the run sums below
  // do not depend on how the centres are split into chunks
  const int sh = __builtin_amdgcn_readfirstlane(*a.e0p % epb);
  const int64_t ngroups = ne > 0 ? (ne + sh + epb - 1) / epb : 0;
  mix32::BwdB<KIND, (MW < 0 ? 0 : MW)> B;
  if constexpr (MW >= 0) {
    if (!a.last) B.load(KIND == G_F32 ? static_cast<const void*>(a.W.fN) : a.W.bN, a.W.n, lane);
  }
  // Software pipeline over the workgroup's groups: the loads of the next
  // group (dE/dV_t and the adjoint's other inputs) are issued right after
  // this group's adjoint arithmetic and consumed after the next staging and
  // mixing. A row past the last edge reads the last edge.
  float gv[NY];
  TpBwdIn<LMAX> in;
  // The centre index of a group is loaded one group earlier still.
  auto edge_of = [&](int64_t g) {
    const int64_t eg = g * epb + el - sh;
    return eg < 0 ? 0 : (eg < ne ? eg : ne - 1);
  };
  auto clampg = [&](int64_t g) { return g < ngroups ? g : ngroups - 1; };
  auto issue = [&](int64_t g, int ctr, float (&gvr)[NY], TpBwdIn<LMAX>& inr) {
    const int64_t ec = edge_of(g);
    if (!LAST && !a.last) {
      const float* src = a.gvin + ec * (NY * C) + c;
#pragma unroll
      for (int lm = 0; lm < NY; ++lm) gvr[lm] = src[lm * C];
    }
    tp_bwd_load<LMAX, CC>(a, ec, ctr, c, inr);
  };
  // dE/dGamma: the group's edges put their contributions into LDS and the
  // first edge of every run of equal centres within the group stores the
  // run's sum (in edge order) at its row of ggc; no other row is written:
  // rows are written at each centre's first edge and at every global
  // multiple of epb inside its edges.
  // With mixing the rows go into the edge's own dE/dT rows (read only by the
  // same thread, and rewritten by the next group's mixing only after the next
  // staging barrier); without, into two alternating buffers.
  const bool mixing = !LAST && !a.last;
  float* const redbase = mixing ? gTl : nq_dyn_lds;
  const int rstride = mixing ? NT * CP : NY * CP;
  int* const centbase = reinterpret_cast<int*>(mixing ? gTl + epb * NT * CP : nq_dyn_lds + 2 * epb * NY * CP);
  int64_t grp = blockIdx.x;
  int ctr = 0, cur = 0;
  if (grp < ngroups) {
    cur = a.ei[edge_of(grp)];
    issue(grp, cur, gv, in);
    ctr = a.ei[edge_of(clampg(grp + gridDim.x))];
  }
  for (int it = 0; grp < ngroups; grp += gridDim.x, ++it) {
    const int par = mixing ? 0 : (it & 1);
    float* const red = redbase + par * epb * NY * CP;
    int* const cent = centbase + par * epb;
    const int64_t e0 = grp * epb - sh;
    // valid rows of the group: lo .. hi - 1 (lo > 0 only in the first group)
    const int lo = e0 < 0 ? (int)-e0 : 0, hi = (int)(ne - e0 < epb ? ne - e0 : epb);
    const bool valid = el >= lo && el < hi;
    if (!LAST && !a.last) {
      // The previous group's reads of gTl finished before this barrier pair
      // lets the mixing overwrite it.
#pragma unroll
      for (int lm = 0; lm < NY; ++lm) {
        const float v = valid ? gv[lm] : 0.f;
        if constexpr (GS == 0) {
          gVl[(el * NY + lm) * CP + c] = v;
        } else {
          bf16* gr = gVh + (el * NY + lm) * CPH + c;
          const bf16 h = (bf16)v;
          gr[0] = h;
          if constexpr (GS == 2) gr[gtlo] = (bf16)(v - (float)h);
        }
      }
      __syncthreads();
      if constexpr (GS > 0)
        mix32::mix_bwd_split<KIND, MW>(B, gVh, gtlo, gTl, lane);
      else if constexpr (MW >= 0)
        mix32::mix_bwd<KIND, MW>(B, gVl, gTl, lane);
      else
        mix_bwd<KIND, LMAX>(gVl, gTl, epb, C, a.W);
      __syncthreads();
    }
    // Generic plan: every thread runs the adjoint (a row past the last edge
    // reads the last edge's inputs) and its stores are dropped, so no branch
    // guards the stores. The 32-channel plan keeps the branch: running the
    // extra rows there costs more registers (spills) than the exact wait
    // counts save.
    if (CC == 0 || valid)
      tp_bwd_edge<LMAX, CC>(a, e0, lo, hi, el, c, gTl + el * NT * CP, CP, in, red + el * rstride);
    if (c == 0) cent[el] = cur;
    tp_lds_barrier();
    // Run sums, shared by the whole workgroup: for each run of equal centres
    // (centres are sorted) every thread takes (component, channel) sums of
    // the run's rows, each added in row order, and stores them at the run's
    // first row (one thread per run start serialised the group otherwise)
    // bit k of `starts`: row k begins a run (the same in every wavefront)
    const int lc = lane < epb ? lane : 0;
    uint64_t starts = __ballot(lane >= lo && lane < hi && (lane == lo || cent[lc] != cent[lc > 0 ? lc - 1 : 0]));
    while (starts) {
      const int k = __builtin_ctzll(starts);
      starts &= starts - 1;
      const int end = starts ? __builtin_ctzll(starts) : hi;
      for (int idx = threadIdx.x; idx < NY * C; idx += 256) {
        const int lm = idx / C, cc = idx - lm * C;
        const float* rp = red + k * rstride + lm * CP + cc;
        float sum = rp[0];
#pragma unroll 4
        for (int e2 = 1; e2 < end - k; ++e2) sum += rp[e2 * rstride];
        a.ggc[(e0 + k) * (NY * C) + idx] = sum;
      }
    }
    // The next group's loads go into the same registers once this group's
    // adjoint is done: their latency then overlaps the next group's staging
    // and mixing (or, for the last layer, other wavefronts' work), and only
    // one set of inputs is live at a time (issuing them before the adjoint
    // kept two sets live and spilled the mixing weights).
    issue(clampg(grp + gridDim.x), ctr, gv, in);
    cur = ctr;
    ctr = a.ei[edge_of(clampg(grp + 2 * gridDim.x))];
  }
}

// Last layer of a 32-channel l <= 2 model: no mixing, the channel count known
// at compile time (fewer registers than the generic kernel).
template <int KIND>
__global__ __launch_bounds__(256) void k_tp_bwd_last32(TpBwdArgs a) {
  tp_bwd_loop<KIND, 2, -2>(a);
}

// Adjoint of one layer's tensor product and, for t < T, of its channel mixing.
template <int KIND, int LMAX, bool C32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_tp_bwd(TpBwdArgs a) {
  if constexpr (C32) {
    static_assert(LMAX == 2, "the 32-channel plan is for l <= 2");
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
      case 0: tp_bwd_loop<KIND, LMAX, 0>(a); break;
      case 1: tp_bwd_loop<KIND, LMAX, 1>(a); break;
      case 2: tp_bwd_loop<KIND, LMAX, 2>(a); break;
      default: tp_bwd_loop<KIND, LMAX, 3>(a); break;
    }
  } else {
    tp_bwd_loop<KIND, LMAX, -1>(a);
  }
}

// Adjoint of the environment sum Gamma_i = nu^-1/2 sum_k e_k (x) Y_k for one
// centre per wavefront (lanes: channel c, group g of G = 64 / C):
//   dGamma_i[lm][c] = nu^-1/2 sum_k ggc[k][lm][c]      (groups split the rows)
// where the tensor-product adjoint left ggc rows only at the centre's first
// edge and at every multiple of `run` after it, each holding the sum of the
// contributions up to the next such row;
//   de_k[l][c]      = sum_m dGamma_i[lm][c] Y_k[lm]     -> gew[:, gcol + l*C + c]
//   dY_k[lm]        = sum_c e_k[l][c] dGamma_i[lm][c]   (channel sums spread over lanes)
// dGamma_i stays in registers between the two passes over the centre's edges.
// dY_k goes to this layer's own 16-float slot of the edge's dE/dY row (plain
// stores; the geometry adjoint adds the slots), and the second pass loads the
// next edge's inputs before working on the current one.
template <int NY, int C>
__global__ __launch_bounds__(256) void k_env_adjoint(int64_t n, const int* __restrict__ nedge_p,
                                                     const int* __restrict__ eoff, const int* __restrict__ e0p,
                                                     int run, const float* __restrict__ ggc,
                                                     const float* __restrict__ esrc, int lde,
                                                     const float* __restrict__ geo, float scale,
                                                     float* __restrict__ gew, int ldgew, int gcol,
                                                     float* __restrict__ gY, int ldgy) {
  constexpr int G = 64 / C, L = NY == 9 ? 2 : (NY == 4 ? 1 : 0);
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= n) return;
  const int lane = threadIdx.x % 64;
  const int c = lane % C, g = lane / C;
  const int ne = *nedge_p;
  const int b = min(eoff[i], ne), e1 = min(eoff[i + 1], ne);
  float dg[NY];
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) dg[lm] = 0.f;
  // rows: b, then m0, m0 + run, ... below e1 (m0: the first edge after b
  // whose global index e0 + k is a multiple of run); row q of the centre is
  // b for q = 0, m0 + (q - 1) run after
  const int m0 = b + run - (*e0p + b) % run;
  const int nrow = b < e1 ? 1 + (e1 > m0 ? (e1 - m0 + run - 1) / run : 0) : 0;
  for (int q = g; q < nrow; q += G) {
    const int64_t k = q == 0 ? b : m0 + (int64_t)(q - 1) * run;
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) dg[lm] += ggc[(k * NY + lm) * C + c];
  }
#pragma unroll
  for (int o = C; o < 64; o <<= 1)
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) dg[lm] += __shfl_xor(dg[lm], o);
#pragma unroll
  for (int lm = 0; lm < NY; ++lm) dg[lm] *= scale;
  // inputs of edge kk2 (a row past the centre's last edge reads the last one)
  auto load = [&](int kk2, float (&Yv)[NY], float (&evv)[L + 1]) {
    const int kc = kk2 < e1 ? kk2 : e1 - 1;
    const float* Yr = geo + (int64_t)kc * kGeo + kGeoY;
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) Yv[lm] = Yr[lm];
#pragma unroll
    for (int l = 0; l <= L; ++l) evv[l] = esrc[(int64_t)kc * lde + l * C + c];
  };
  float Yn[NY], evn[L + 1];
  const __amdgpu_buffer_rsrc_t GYr = buffer_rsrc(gY + (int64_t)b * ldgy, (int64_t)(e1 - b) * ldgy * 4);
  if (b + g < e1) load(b + g, Yn, evn);
  for (int kk = b + g; kk < e1; kk += G) {
    float Y[NY], ev[L + 1], prod[NY];
#pragma unroll
    for (int lm = 0; lm < NY; ++lm) Y[lm] = Yn[lm];
#pragma unroll
    for (int l = 0; l <= L; ++l) ev[l] = evn[l];
    load(kk + G, Yn, evn);
#pragma unroll
    for (int l = 0; l <= L; ++l) {
      float ge = 0.f;
#pragma unroll
      for (int m = 0; m < 2 * l + 1; ++m) {
        ge += dg[l * l + m] * Y[l * l + m];
        prod[l * l + m] = ev[l] * dg[l * l + m];
      }
      gew[(int64_t)kk * ldgew + gcol + l * C + c] = ge;
    }
    int first = 0, count = 0;
    spread_sum<NY, C>(prod, c, first, count);
    // a lane holds at most ceil(NY / C) components; the stores are
    // unconditional (dropped by the buffer range for slots holding none), so
    // no branch makes the wait for the next edge's prefetched inputs inexact
#pragma unroll
    for (int q = 0; q < (NY + C - 1) / C; ++q)
      buf_store(prod[q], GYr, q < count ? (unsigned)((kk - b) * ldgy + first + q) * 4 : kOutOfRange);
  }
}

__device__ inline void sph_grad_dot(const float* gY, float x, float y, float z, float& gx, float& gy, float& gz) {
  const float s3 = 1.7320508075688772f, s5 = 2.2360679774997897f, s15 = 3.872983346207417f;
  gx = s3 * gY[1] + s15 * (y * gY[4] + z * gY[7] + x * gY[8]);
  gy = s3 * gY[2] + s15 * (x * gY[4] + z * gY[5] - y * gY[8]);
  gz = s3 * gY[3] + s15 * (y * gY[5] + x * gY[7]) + 3.f * s5 * z * gY[6];
}

// Adjoint of the edge geometry: dE/dr_ij from dE/du, dE/dY (the sum of the
// nslot 16-float slots of the edge's row in gYb: the first tensor product's
// part, then each layer's environment-sum part) and dE/db.
__global__ void k_geometry_bwd(const int* __restrict__ nedge_p, const float* __restrict__ geo,
                               const float* __restrict__ gu, const float* __restrict__ gYb, int nslot,
                               const float* __restrict__ gh0, int ldh0, int boff, int nb, int p, float rc, int NY,
                               const int* __restrict__ e0p, float4* __restrict__ gr) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= *nedge_p) return;
  const float* g = geo + e * kGeo;
  const float d = g[0], x = g[2], y = g[3], z = g[4];
  float u, dudx;
  envelope(d / rc, p, u, dudx);
  float gut = gu[e], gd = 0.f;
  const float pref = 2.f / rc, w = 3.14159265358979323846f / rc, inv = 1.f / d;
  float s1, c1;
  sincosf(w * d, &s1, &c1);
  float sn = s1, cs = c1;  // sin, cos of n w d (angle-addition recurrence)
  for (int n = 1; n <= nb; ++n) {
    const float k = n * w;
    const float B = pref * sn * inv;
    const float dB = pref * (k * cs * inv - sn * inv * inv);
    const float gb = gh0[e * ldh0 + boff + n - 1];
    gut += gb * B;
    gd += gb * u * dB;
    const float t = sn * c1 + cs * s1;
    cs = cs * c1 - sn * s1;
    sn = t;
  }
  gd += gut * dudx / rc;
  float gY[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) gY[k] = 0.f;
  // slots in order, each as three 16-byte loads (components 0..11), all issued
  // before the sums (at most 5 slots: T <= 4)
  float4 q[5][3];
  const float4* row = reinterpret_cast<const float4*>(gYb + e * nslot * 16);
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j) q[r][j] = r < nslot ? row[r * 4 + j] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const float w[4] = {q[r][j].x, q[r][j].y, q[r][j].z, q[r][j].w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j * 4 + u < 9 && j * 4 + u < NY) gY[j * 4 + u] += w[u];
    }
  float ax, ay, az;
  sph_grad_dot(gY, x, y, z, ax, ay, az);
  const float rad = ax * x + ay * y + az * z;
  gr[*e0p + e] = make_float4(gd * x + (ax - rad * x) * inv, gd * y + (ay - rad * y) * inv, gd * z + (az - rad * z) * inv,
                      0.f);
}

// F_a = sum over edges (a, j): g(a,j) - g(j,a)   (F_i += g_ij, F_j -= g_ij)
// F_a = sum over a's edges (a, j) of g(a, j) - g(j, a). A centre's incoming
// edges are the reverses of its own; an atom a >= n_centres (a ghost of a
// spatial domain: no edges of its own) gathers the edges (j, a) of its centre
// neighbours j through its neighbour-list row (binary search in j's edge row).
__global__ void k_forces(int64_t n, int64_t n_centres, const int* __restrict__ nedge_p,
                         const int* __restrict__ eoff, const int* __restrict__ ej, const int* __restrict__ rev,
                         const int* __restrict__ nbr, const int* __restrict__ nbr_cnt, int k_max,
                         const float4* __restrict__ gr, double* __restrict__ F, const int* __restrict__ flags) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  if (results_invalid(flags)) {
    F[3 * a] = F[3 * a + 1] = F[3 * a + 2] = __builtin_nan("");
    return;
  }
  const int ne = *nedge_p;
  double fx = 0, fy = 0, fz = 0;
  if (a < n_centres) {
    for (int e = min(eoff[a], ne); e < min(eoff[a + 1], ne); ++e) {
      const int r = rev[e];
      const float4 g = gr[e], h = (r < ne) ? gr[r] : make_float4(0.f, 0.f, 0.f, 0.f);
      fx += (double)g.x - (double)h.x;
      fy += (double)g.y - (double)h.y;
      fz += (double)g.z - (double)h.z;
    }
  } else {
    const int cnt = nbr_cnt[a];
    for (int s = 0; s < cnt; ++s) {
      const int j = nbr[a * (int64_t)k_max + s];
      if (j >= n_centres) continue;
      int lo = min(eoff[j], ne), hi = min(eoff[j + 1], ne);
      const int end = hi;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ej[mid] < a) lo = mid + 1; else hi = mid;
      }
      if (lo < end && ej[lo] == a) {
        const float4 h = gr[lo];
        fx -= (double)h.x;
        fy -= (double)h.y;
        fz -= (double)h.z;
      }
    }
  }
  F[3 * a] = fx;
  F[3 * a + 1] = fy;
  F[3 * a + 2] = fz;
}

// ------------------------------------------------------------------ GEMM dispatch
template <int KIND, int BM, int NP, int WM, int WN>
void launch_gemm_t(hipStream_t s, int64_t cap, int Kp, const void* Bt, const int* nrows, const ALoad& ld,
                   const Epi& ep) {
  typedef typename GemmTraits<KIND>::BT BT;
  k_gemm<KIND, BM, NP, WM, WN><<<(unsigned)cdiv(cap, BM), 256, 0, s>>>(Kp, static_cast<const BT*>(Bt), nrows, ld,
                                                                       ep);
}

// Tile-shape candidates per output width NP: (rows per workgroup BM, wave grid
// WM x WN). Variant 0 is the default; the
// autotuner (nq_autotune) times all of them on the real shapes and keeps the
// fastest per product. Shapes whose LDS (A and B tiles) would not fit are left
// out for the split-BF16 kind, which keeps both weight halves in LDS.
int gemm_variants(int kind, int NP) {
  const bool x3 = kind == G_BF16X3;
  switch (NP) {
    case 16: case 32: return 3;
    case 48: return 2;
    case 64: case 96: case 128: case 192: case 256: return 4;
    case 352: return x3 ? 2 : 3;
    default: return 1;
  }
}

template <int KIND>
void launch_gemm_np(hipStream_t s, int64_t cap, int NP, int Kp, const void* Bt, const int* nrows, const ALoad& ld,
                    const Epi& ep, int v) {
  constexpr bool X3 = KIND == G_BF16X3;
  v = v % gemm_variants(KIND, NP);
#define NQ_G(BM, N, WM, WN) launch_gemm_t<KIND, BM, N, WM, WN>(s, cap, Kp, Bt, nrows, ld, ep)
  switch (NP) {
    case 16: if (v == 0) NQ_G(128, 16, 4, 1); else if (v == 1) NQ_G(64, 16, 4, 1); else NQ_G(256, 16, 4, 1); break;
    case 32: if (v == 0) NQ_G(128, 32, 4, 1); else if (v == 1) NQ_G(64, 32, 4, 1); else NQ_G(256, 32, 4, 1); break;
    case 48: if (v == 0) NQ_G(128, 48, 4, 1); else NQ_G(64, 48, 4, 1); break;
    case 64:
      if (v == 0) NQ_G(128, 64, 2, 2); else if (v == 1) NQ_G(64, 64, 2, 2);
      else if (v == 2) NQ_G(256, 64, 2, 2); else NQ_G(128, 64, 4, 1);
      break;
    case 96:
      if (v == 0) NQ_G(128, 96, 2, 2); else if (v == 1) NQ_G(64, 96, 2, 2);
      else if (v == 2) NQ_G(256, 96, 4, 1); else NQ_G(128, 96, 4, 1);
      break;
    case 128:
      if (v == 0) NQ_G(128, 128, 2, 2); else if (v == 1) NQ_G(64, 128, 2, 2);
      else if (v == 2) NQ_G(256, 128, 4, 1); else NQ_G(128, 128, 4, 1);
      break;
    case 192:
      if (v == 0) NQ_G(64, 192, 2, 2); else if (v == 1) NQ_G(32, 192, 2, 2);
      else if (v == 2) NQ_G(128, 192, 2, 2); else NQ_G(64, 192, 4, 1);
      break;
    case 256:
      if (v == 0) NQ_G(64, 256, 2, 2); else if (v == 1) NQ_G(32, 256, 2, 2);
      else if (v == 2) NQ_G(128, 256, 2, 2); else NQ_G(64, 256, 4, 1);
      break;
    case 352:
      if constexpr (X3) {
        if (v == 0) NQ_G(32, 352, 2, 2); else NQ_G(64, 352, 2, 2);
      } else {
        if (v == 0) NQ_G(64, 352, 2, 2); else if (v == 1) NQ_G(32, 352, 2, 2); else NQ_G(128, 352, 2, 2);
      }
      break;
    case 384:
      if constexpr (X3) NQ_G(32, 384, 2, 2); else NQ_G(64, 384, 2, 2);
      break;
    case 512:
      if constexpr (X3) NQ_G(32, 512, 2, 2); else NQ_G(64, 512, 2, 2);
      break;
    case 704:
      if constexpr (X3) NQ_G(32, 704, 2, 2); else NQ_G(64, 704, 1, 4);
      break;
    default: throw Error{NQ_ERR_UNSUPPORTED, "no matrix-core kernel for output width " + std::to_string(NP)};
  }
#undef NQ_G
}

// Algorithmic HBM bytes per edge row of one product: every source value of A
// read once, every other value the epilogue reads or writes once.
double gemm_bytes_per_row(const ALoad& ld, const Epi& ep) {
  double a = 0;
  switch (ld.mode) {
    case A_CAT: a = ld.K0 + ld.K1; break;
    case A_CAT_SILU_U: a = ld.K0 + ld.K1 + 1; break;
    case A_SILU_U: a = ld.K0 + 1; break;
    case A_GRADSILU: a = (ld.ld0 ? ld.K0 : 0) + ld.K0 + (ld.rs ? 1 : 0) + (ld.gu ? 2 : 0); break;
    default: a = ld.K0;
  }
  double o = 0;
  switch (ep.mode) {
    case E_STORE: o = ep.N0; break;
    case E_STORE_X0: o = 2.0 * ep.N0 + 1; break;
    case E_RESIDUAL: o = 2.0 * ep.N0 + 1; break;  // x is the first part of A
    case E_LATENT_BWD: o = ep.N0; break;          // g is A's source
    default: o = 2.0 * ep.N0;
  }
  return 4.0 * (a + o);
}

// y = A W (fwd) or gA = gy W^T (bwd) for one stored linear map. The kernel is
// the model's tuned choice for this product (or the one being timed): one of
// the tile shapes of k_gemm or, where compiled, the two epilogue forms of the
// weight-stationary k_gemm_ws (the last two variants).
void gemm(nq_ctx* ctx, const nq_model* m, const Lin& L, bool bwd, const ALoad& ld, const Epi& ep,
          const std::string& name) {
  const Workspace& ws = ctx->ws;
  const double flop = 2.0 * L.fin * L.fout;
  const int sp = span_begin(ctx, name, flop, gemm_bytes_per_row(ld, ep), 0, 0, flop);
  const int NP = bwd ? L.np_b : L.np_f;
  const int Kp = bwd ? L.kp_b : L.kp_f;
  const int* nr = ws.v_nedge;
  int v = 0;
  if (ctx->force_variant >= 0) {
    v = ctx->force_variant;
  } else if (ctx->user_variant >= 0) {
    v = ctx->user_variant;
  } else if (ctx->user_variant == NQ_VARIANT_TUNED) {
    auto it = m->gemm_choice.find(name);
    if (it != m->gemm_choice.end()) v = it->second;
  }
  const int prec = site_precision(m, name);
  const int kind = prec == NQ_PRECISION_BF16X3 ? G_BF16X3 : (prec == NQ_PRECISION_BF16 ? G_BF16 : G_F32);
  const void* Bbf = (bwd ? L.bf_bwd : L.bf_fwd).p;
  const int ntile = gemm_variants(kind, NP);
  const bool has_ws = gemm_ws(false, 0, kind, ctx->stream, ctx->num_cu, NP, Kp, Bbf, nr, ld, ep);
  const int nv = ntile + (has_ws ? 2 : 0);
  ctx->site_np[name] = NP;
  ctx->site_nvar[name] = nv;
  if (ctx->force_variant < 0 && ctx->user_variant <= NQ_VARIANT_LAST)
    v = std::max(0, nv + 1 + ctx->user_variant);  // LAST: nv - 1, LAST2: nv - 2
  else
    v %= nv;
  if (has_ws && v >= ntile) {
    gemm_ws(true, v - ntile, kind, ctx->stream, ctx->num_cu, NP, Kp, Bbf, nr, ld, ep);
    NQ_HIP(hipGetLastError());
    span_end(ctx, sp);
    return;
  }
  switch (prec) {
    case NQ_PRECISION_BF16:
      launch_gemm_np<G_BF16>(ctx->stream, ws.cap, NP, Kp, Bbf, nr, ld, ep, v);
      break;
    case NQ_PRECISION_BF16X3:
      launch_gemm_np<G_BF16X3>(ctx->stream, ws.cap, NP, Kp, Bbf, nr, ld, ep, v);
      break;
    default:
      launch_gemm_np<G_F32>(ctx->stream, ws.cap, NP, Kp, (bwd ? L.f32_bwd : L.f32_fwd).p, nr, ld, ep, v);
  }
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

ALoad a_plain(const float* p, int ld, int K) { return ALoad{A_PLAIN, p, ld, K, nullptr, 0, 0, nullptr, 0, 1.f, nullptr}; }
ALoad a_silu(const float* p, int ld, int K) { return ALoad{A_SILU, p, ld, K, nullptr, 0, 0, nullptr, 0, 1.f, nullptr}; }
// u SiLU(a) of pre-activations a with the row scale u (x0 formed at use)
ALoad a_silu_u(const float* p, int ld, int K, const float* u) {
  return ALoad{A_SILU_U, p, ld, K, nullptr, 0, 0, u, kGeo, 1.f, nullptr};
}
ALoad a_cat(const float* p, int ld, int K, const float* q, int ldq, int Kq) {
  return ALoad{A_CAT, p, ld, K, q, ldq, Kq, nullptr, 0, 1.f, nullptr};
}
// [u SiLU(a) | q]
ALoad a_cat_silu_u(const float* p, int ld, int K, const float* q, int ldq, int Kq, const float* u) {
  return ALoad{A_CAT_SILU_U, p, ld, K, q, ldq, Kq, u, kGeo, 1.f, nullptr};
}
ALoad a_gradsilu(const float* g, int ldg, int K, const float* a, int lda, const float* rs, float c,
                 float* gu = nullptr) {
  return ALoad{A_GRADSILU, g, ldg, K, a, lda, 0, rs, kGeo, c, gu};
}
Epi e_store(float* o, int ld, int N) { return Epi{E_STORE, o, ld, N, nullptr, 0, nullptr, 0, nullptr, 0, 0}; }
Epi e_add(float* o, int ld, int N) { return Epi{E_ADD, o, ld, N, nullptr, 0, nullptr, 0, nullptr, 0, 0}; }

unsigned grid_for(int64_t n, int per_block) { return (unsigned)std::max<int64_t>(1, cdiv(n, per_block)); }

// Calls M(NY, C) with compile-time values for l <= 1 or 2 and C = 8 ... 64.
#define NQ_DISPATCH_NY_C(NYV, CV, M)                                    \
  do {                                                                  \
    const int nq_c_ = (CV);                                             \
    if ((NYV) == 4) {                                                   \
      if (nq_c_ == 8) M(4, 8); else if (nq_c_ == 16) M(4, 16);          \
      else if (nq_c_ == 32) M(4, 32); else M(4, 64);                    \
    } else {                                                            \
      if (nq_c_ == 8) M(9, 8); else if (nq_c_ == 16) M(9, 16);          \
      else if (nq_c_ == 32) M(9, 32); else M(9, 64);                    \
    }                                                                   \
  } while (0)

// ------------------------------------------------------------------ per-edge launches
MixPtrs layer_mix(const nq_model* m, int t) {
  MixPtrs w{nullptr, nullptr, nullptr, nullptr, 0};
  if (t == m->dims.T) return w;
  const MixW& M = *m->mixw[t - 1];
  w.fN = M.fN.as<float>();
  w.fT = M.fT.as<float>();
  w.bN = M.bN.as<bf16>();
  w.bT = M.bT.as<bf16>();
  w.n = M.n;
  return w;
}

// Persistent launches: exactly as many workgroups as the chip holds at once
// (no partial last wave of workgroups), each looping over groups of edges.
template <class K>
unsigned tp_grid(const nq_ctx* ctx, K kernel, size_t lds, int C) {
  static std::map<std::pair<const void*, size_t>, int> cache;  // workgroups per CU
  static std::mutex mu;                                         // contexts may live on several threads
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), lds);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int per_cu = 0;
    NQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, lds));
    it = cache.emplace(key, std::max(per_cu, 1)).first;
  }
  const int64_t resident = (int64_t)it->second * ctx->num_cu;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid_for(ctx->ws.cap, 256 / C), resident));
}

void launch_tp_fwd(nq_ctx* ctx, const nq_model* m, int t) {
  const Dims& d = m->dims;
  Workspace& ws = ctx->ws;
  const bool last = t == d.T;
  const TpFwdArgs a{ws.v_nedge, ws.v_ei, ws.geo, d.C, t == 1, last, ws.we1, 2 * d.NW, ws.V[t - 1], ws.gam[t],
                    ws.s[t], d.nscal * d.C, layer_mix(m, t), ws.V[t]};
  const size_t lds = tp_lds_bytes(d.C, d.L, false);
  // bytes per edge: V_{t-1} (w0 and Y for t = 1), the centre index, s, V_t;
  // per atom: Gamma read once
  const double vin = t == 1 ? 4.0 * (d.NW + d.NY) : 4.0 * d.NY * d.C;
  const double bpe = vin + 4.0 + 4.0 * d.nscal * d.C + (last ? 0.0 : 4.0 * d.NY * d.C);
  const int sp = span_begin(ctx, "tp_fwd" + std::to_string(t), m->tp_flop_fwd[t - 1], bpe, 0,
                            4.0 * d.NY * d.C, m->tp_flop_mix[t - 1]);
  // the last layer has no mixing: a lighter kernel keeps more waves
  const bool c32 = d.L == 2 && d.C == mix32::C && !last, l32 = d.L == 2 && d.C == mix32::C && last;
#define NQ_TPF(K, LM)                                                                             \
  if (LM == 2 && c32)                                                                             \
    k_tp_fwd<K, 2, true><<<tp_grid(ctx, k_tp_fwd<K, 2, true>, lds, d.C), 256, lds, ctx->stream>>>(a); \
  else if (LM == 2 && l32) /* no mixing: no LDS */                                                \
    k_tp_fwd_last32<K><<<tp_grid(ctx, k_tp_fwd_last32<K>, 0, d.C), 256, 0, ctx->stream>>>(a);     \
  else                                                                                            \
    k_tp_fwd<K, LM, false><<<tp_grid(ctx, k_tp_fwd<K, LM, false>, lds, d.C), 256, lds, ctx->stream>>>(a)
  switch (site_precision(m, "tp_fwd" + std::to_string(t)) * 2 + (d.L == 2)) {
    case 0: NQ_TPF(G_F32, 1); break;
    case 1: NQ_TPF(G_F32, 2); break;
    case 2: NQ_TPF(G_BF16, 1); break;
    case 3: NQ_TPF(G_BF16, 2); break;
    case 4: NQ_TPF(G_BF16X3, 1); break;
    default: NQ_TPF(G_BF16X3, 2); break;
  }
#undef NQ_TPF
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

void launch_tp_bwd(nq_ctx* ctx, const nq_model* m, int t, const float* gvin, float* gvout) {
  const Dims& d = m->dims;
  Workspace& ws = ctx->ws;
  const bool last = t == d.T;
  const TpBwdArgs a{ws.v_nedge, ws.v_e0, ws.v_ei, ws.geo, d.C, t == 1, last, ws.we1, 2 * d.NW, ws.V[t - 1], ws.gam[t],
                    ws.gs, d.nscal * d.C, last ? nullptr : gvin, layer_mix(m, t), ws.ggc, gvout, ws.gew,
                    2 * d.NW, ws.gY, 16 * (d.T + 1)};
  const size_t lds = tp_lds_bytes(d.C, d.L, true), llds = tp_last_lds_bytes(d.C, d.L);
  // bytes per edge: dE/dV_t, V_{t-1} (w0 and Y for t = 1), the centre index,
  // dE/ds, the dE/dGamma contributions, and dE/dV_{t-1} (t > 1) or dE/dw0
  // plus the w0 part of dE/dY (t = 1); per atom: Gamma read once
  const double vin = t == 1 ? 4.0 * (d.NW + d.NY) : 4.0 * d.NY * d.C;
  const double vout = t == 1 ? 4.0 * d.NW + 4.0 * d.NY : 4.0 * d.NY * d.C;
  // (the dE/dGamma rows: one run sum per group of 256 / C edges)
  const double bpe =
      (last ? 0.0 : 4.0 * d.NY * d.C) + vin + 4.0 + 4.0 * d.nscal * d.C + 4.0 * d.NY * d.C * d.C / 256.0 + vout;
  const int sp = span_begin(ctx, "tp_bwd" + std::to_string(t), m->tp_flop_bwd[t - 1], bpe, 0,
                            4.0 * d.NY * d.C, m->tp_flop_mix[t - 1]);
  // the last layer has no mixing: a lighter kernel keeps more waves
  const bool c32 = d.L == 2 && d.C == mix32::C && !last, l32 = d.L == 2 && d.C == mix32::C && last;
#define NQ_TPB(K, LM)                                                                             \
  if (LM == 2 && c32)                                                                             \
    k_tp_bwd<K, 2, true><<<tp_grid(ctx, k_tp_bwd<K, 2, true>, lds, d.C), 256, lds, ctx->stream>>>(a); \
  else if (LM == 2 && l32) /* no mixing: LDS for the run sums only */                             \
    k_tp_bwd_last32<K><<<tp_grid(ctx, k_tp_bwd_last32<K>, llds, d.C), 256, llds, ctx->stream>>>(a); \
  else                                                                                            \
    k_tp_bwd<K, LM, false><<<tp_grid(ctx, k_tp_bwd<K, LM, false>, lds, d.C), 256, lds, ctx->stream>>>(a)
  switch (site_precision(m, "tp_bwd" + std::to_string(t)) * 2 + (d.L == 2)) {
    case 0: NQ_TPB(G_F32, 1); break;
    case 1: NQ_TPB(G_F32, 2); break;
    case 2: NQ_TPB(G_BF16, 1); break;
    case 3: NQ_TPB(G_BF16, 2); break;
    case 4: NQ_TPB(G_BF16X3, 1); break;
    default: NQ_TPB(G_BF16X3, 2); break;
  }
#undef NQ_TPB
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

void launch_env_bwd(nq_ctx* ctx, const nq_model* m, int t) {
  const Dims& d = m->dims;
  Workspace& ws = ctx->ws;
  const int64_t n = ws.v_n;
  const float* esrc = t == 1 ? ws.we1 + d.NW : ws.e[t];
  const int lde = t == 1 ? 2 * d.NW : d.NW;
  const float scale = (float)d.inv_sqrt_nu;
  // per edge: the dE/dGamma run sums (one per group of 256 / C edges), e, Y,
  // dE/de and dE/dY written
  const int sp = span_begin(ctx, "env_bwd" + std::to_string(t), 0,
                            4.0 * d.NY * d.C * d.C / 256.0 + 8.0 * d.NW + 4.0 * d.NY + 4.0 * d.NY, 0, 4.0);
#define NQ_ENVB(NYV, CV)                                                                                   \
  k_env_adjoint<NYV, CV><<<grid_for(n, 4), 256, 0, ctx->stream>>>(n, ws.v_nedge, ws.v_eoff, ws.v_e0, 256 / d.C, ws.ggc, esrc, lde, \
                                                                  ws.geo, scale, ws.gew, 2 * d.NW, d.NW,       \
                                                                  ws.gY + 16 * t, 16 * (d.T + 1))
  NQ_DISPATCH_NY_C(d.NY, d.C, NQ_ENVB);
#undef NQ_ENVB
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
}

}  // namespace

// ------------------------------------------------------------------ workspace
namespace {

// Bytes of per-edge activation and adjoint buffers per edge of a chunk.
int64_t bytes_per_edge(const Dims& d, int K0p, int maxw) {
  int64_t w = kGeo + K0p + 2 * d.NW + 1;  // geo, h0, we1, eij
  for (int k = 0; k < d.n_tb; ++k) w += d.tb[k];
  w += d.D;  // x0
  for (int t = 1; t <= d.T; ++t) {
    if (t > 1) w += d.NW;
    w += d.nscal * d.C + d.D;
    for (int k = 0; k < d.n_lat; ++k) w += d.lat[k];
    if (t < d.T) w += d.NY * d.C;
  }
  for (int k = 0; k < d.n_edge; ++k) w += d.edge[k];
  w += d.D + 2 * maxw + d.nscal * d.C + 3 * d.NY * d.C + 2 * d.NW + 16 + 1;  // adjoint
  return w * 4 + 24;  // + chunk-local edge copies
}

// Per-chunk edge views: chunk-local centre index, neighbour, geometry, offsets.
__global__ void k_chunk_edges(const int* __restrict__ eoff, int64_t a0, int64_t a1, int64_t cap,
                              const int* __restrict__ ei, const int* __restrict__ ej, const float4* __restrict__ rij,
                              int* c_ei, int* c_ej, float4* c_rij, int* c_nedge, int* flags) {
  const int64_t e0 = eoff[a0], n = (int64_t)eoff[a1] - e0;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) {
    if (n > cap) flags[4] = (int)n;
    *c_nedge = (int)(n < cap ? n : cap);
  }
  if (e >= n || e >= cap) return;
  c_ei[e] = ei[e0 + e] - (int)a0;
  c_ej[e] = ej[e0 + e];
  c_rij[e] = rij[e0 + e];
}

__global__ void k_chunk_offsets(const int* __restrict__ eoff, int64_t a0, int64_t a1, int* c_eoff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > a1 - a0) return;
  c_eoff[i] = eoff[a0 + i] - eoff[a0];
}

// x0[e][c] = u_e SiLU(a[e][c]) (the stage export of x0; the pipeline forms it
// at use)
__global__ void k_x0(const int* __restrict__ nedge_p, const float* __restrict__ a, int D,
                     const float* __restrict__ geo, float* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = k / D;
  if (e >= *nedge_p) return;
  out[k] = geo[e * kGeo + 1] * siluf(a[k]);
}

}  // namespace

void debug_x0_async(nq_ctx* ctx, const nq_model* m, float* out) {
  const Workspace& ws = ctx->ws;
  const Dims& d = m->dims;
  k_x0<<<(unsigned)cdiv(ws.cap * d.D, 256), 256, 0, ctx->stream>>>(ws.v_nedge, ws.a_tb[d.n_tb - 1], d.D, ws.geo,
                                                                   out);
  NQ_HIP(hipGetLastError());
}

void ws_ensure(nq_ctx* ctx, const nq_model* m, int64_t cap_all, int64_t n_atoms, bool activations) {
  Workspace& ws = ctx->ws;
  cap_all = rup(std::max<int64_t>(cap_all, 1), 128);
  const NbrList& nl = ctx->nl;
  if (ws.model == m && ws.cap_all >= cap_all && ws.n_atoms == n_atoms && !ws.chunks.empty() &&
      (ws.has_act || !activations))
    return;
  ++ctx->gen;
  const Dims& d = m->dims;
  NQ_HIP(hipStreamSynchronize(ctx->stream));
  ws.bufs.clear();
  ws.cap_all = cap_all;
  ws.n_atoms = n_atoms;
  ws.model = m;
  ws.ecnt.ensure(n_atoms * 4);
  ws.eoff.ensure((n_atoms + 1) * 4);
  ws.ei.ensure(cap_all * 4);
  ws.ej.ensure(cap_all * 4);
  ws.rev.ensure(cap_all * 4);
  ws.rij.ensure(cap_all * 16);
  ws.grbuf.ensure(cap_all * 16);
  ws.nedge.ensure(64);
  ws.gr = ws.grbuf.as<float4>();
  ws.has_act = activations;
  if (!activations) {
    // the fused path: energies per atom and the edge list only
    ws.chunks.assign({0, n_atoms});
    ws.cap = cap_all;
    ws.bufs.emplace_back(new DevBuf());
    ws.bufs.back()->ensure((size_t)n_atoms * 8);
    ws.atomE = ws.bufs.back()->as<double>();
    ws.bufs.emplace_back(new DevBuf());
    ws.bufs.back()->ensure(64);
    ws.esum = ws.bufs.back()->as<double>();
    return;
  }
  ws.K0p = (int)rup(d.n_in2b, 32);
  int maxw = d.n_in2b;
  for (int k = 0; k < d.n_tb; ++k) maxw = std::max(maxw, d.tb[k]);
  for (int k = 0; k < d.n_lat; ++k) maxw = std::max(maxw, d.lat[k]);
  for (int k = 0; k < d.n_edge; ++k) maxw = std::max(maxw, d.edge[k]);
  maxw = std::max(maxw, d.D + d.nscal * d.C);
  ws.maxw = (int)rup(maxw, 16);
  // Chunks of consecutive centres whose list entries (an upper bound of their
  // edges, with a margin for rebuilds) fit the activation budget.
  size_t free_b = 0, total_b = 0;
  NQ_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t bpe = bytes_per_edge(d, ws.K0p, ws.maxw);
  int64_t budget = std::min<int64_t>((int64_t)(0.75 * (double)free_b), ctx->ws_budget);
  int64_t cap = std::max<int64_t>(budget / bpe, 1 << 16);
  cap = std::min(cap, cap_all);
  ws.chunks.assign(1, 0);
  if (cap >= cap_all || nl.entry_prefix.size() != (size_t)n_atoms + 1) {
    ws.chunks.push_back(n_atoms);
    cap = cap_all;
  } else {
    const double margin = (double)cap_all / std::max<double>(1.0, (double)nl.n_entries);
    int64_t a = 0;
    while (a < n_atoms) {
      int64_t b = a + 1;
      while (b < n_atoms && (double)(nl.entry_prefix[b + 1] - nl.entry_prefix[a]) * margin <= (double)cap) ++b;
      ws.chunks.push_back(b);
      a = b;
    }
  }
  ws.cap = cap = rup(cap, 128);
  auto fbuf = [&](int64_t rows, int64_t width) -> float* {
    ws.bufs.emplace_back(new DevBuf());
    ws.bufs.back()->ensure((size_t)rows * width * 4);
    return ws.bufs.back()->as<float>();
  };
  if (ws.chunks.size() > 2) {
    ws.c_ei.ensure(cap * 4);
    ws.c_ej.ensure(cap * 4);
    ws.c_rij.ensure(cap * 16);
    ws.c_eoff.ensure((n_atoms + 1) * 4);
    ws.c_nedge.ensure(64);
  }
  ws.geo = fbuf(cap, kGeo);
  ws.h0 = fbuf(cap, ws.K0p);
  ws.a_tb.clear();
  for (int k = 0; k < d.n_tb; ++k) ws.a_tb.push_back(fbuf(cap, d.tb[k]));
  ws.we1 = fbuf(cap, 2 * d.NW);
  ws.x.assign(d.T + 1, nullptr);
  ws.gam.assign(d.T + 1, nullptr);
  ws.s.assign(d.T + 1, nullptr);
  ws.V.assign(d.T + 1, nullptr);
  ws.e.assign(d.T + 1, nullptr);
  ws.a_lat.assign(d.T + 1, {});
  // x[0] stays null: x0 = u SiLU(a) is formed from the two-body pre-activation
  for (int t = 1; t <= d.T; ++t) {
    if (t > 1) ws.e[t] = fbuf(cap, d.NW);
    ws.gam[t] = fbuf(n_atoms, d.NY * d.C);
    ws.s[t] = fbuf(cap, d.nscal * d.C);
    for (int k = 0; k < d.n_lat; ++k) ws.a_lat[t].push_back(fbuf(cap, d.lat[k]));
    ws.x[t] = fbuf(cap, d.D);
    if (t < d.T) ws.V[t] = fbuf(cap, d.NY * d.C);
  }
  ws.a_edge.clear();
  for (int k = 0; k < d.n_edge; ++k) ws.a_edge.push_back(fbuf(cap, d.edge[k]));
  ws.eij = fbuf(cap, 1);
  ws.bufs.emplace_back(new DevBuf());
  ws.bufs.back()->ensure((size_t)n_atoms * 8);
  ws.atomE = ws.bufs.back()->as<double>();
  ws.bufs.emplace_back(new DevBuf());
  ws.bufs.back()->ensure(64);
  ws.esum = ws.bufs.back()->as<double>();
  ws.gx = fbuf(cap, d.D);
  ws.gh[0] = fbuf(cap, ws.maxw);
  ws.gh[1] = fbuf(cap, ws.maxw);
  ws.gs = fbuf(cap, d.nscal * d.C);
  ws.gv[0] = fbuf(cap, d.NY * d.C);
  ws.gv[1] = fbuf(cap, d.NY * d.C);
  ws.ggc = fbuf(cap, d.NY * d.C);
  ws.gew = fbuf(cap, 2 * d.NW);
  ws.gY = fbuf(cap, 16 * (d.T + 1));  // dE/dY: one 16-float slot per contributor
  ws.gu = fbuf(cap, 1);
  ws.gr = ws.grbuf.as<float4>();
}

// Points the pipeline at chunk `c` (centres chunks[c] .. chunks[c+1]); with a
// single chunk the views are the whole-system arrays themselves.
void chunk_view_async(nq_ctx* ctx, int c) {
  Workspace& ws = ctx->ws;
  const int64_t a0 = ws.chunks[c], a1 = ws.chunks[c + 1];
  ws.v_a0 = a0;
  ws.v_n = a1 - a0;
  ws.v_e0 = ws.eoff.as<int>() + a0;
  if (ws.chunks.size() == 2) {
    ws.v_nedge = ws.nedge.as<int>();
    ws.v_ei = ws.ei.as<int>();
    ws.v_ej = ws.ej.as<int>();
    ws.v_rij = ws.rij.as<float4>();
    ws.v_eoff = ws.eoff.as<int>();
    return;
  }
  const int sp = span_begin(ctx, "chunk_view");
  k_chunk_edges<<<grid_for(ws.cap, 256), 256, 0, ctx->stream>>>(
      ws.eoff.as<int>(), a0, a1, ws.cap, ws.ei.as<int>(), ws.ej.as<int>(), ws.rij.as<float4>(), ws.c_ei.as<int>(),
      ws.c_ej.as<int>(), ws.c_rij.as<float4>(), ws.c_nedge.as<int>(), ctx->nl.flags.as<int>());
  k_chunk_offsets<<<grid_for(a1 - a0 + 1, 256), 256, 0, ctx->stream>>>(ws.eoff.as<int>(), a0, a1,
                                                                       ws.c_eoff.as<int>());
  NQ_HIP(hipGetLastError());
  span_end(ctx, sp);
  ws.v_nedge = ws.c_nedge.as<int>();
  ws.v_ei = ws.c_ei.as<int>();
  ws.v_ej = ws.c_ej.as<int>();
  ws.v_rij = ws.c_rij.as<float4>();
  ws.v_eoff = ws.c_eoff.as<int>();
}

// ------------------------------------------------------------------ forward
void forward_async(nq_ctx* ctx, const nq_model* m, const int32_t* species, double* atom_energy) {
  const Dims& d = m->dims;
  Workspace& ws = ctx->ws;
  const int64_t n = ws.v_n;
  hipStream_t s = ctx->stream;
  const int* ne = ws.v_nedge;
  const int64_t cap = ws.cap;
  const float* u = ws.geo + 1;
  {
    // per edge: r_ij and d, indices, species, geo row and two-body input row written
    const int sp_ = span_begin(ctx, "geometry", 0, 16.0 + 8.0 + 8.0 + 4.0 * kGeo + 4.0 * ws.K0p);
    k_geometry<<<grid_for(cap, 256), 256, 256 * (kGeo + 1 + ws.K0p + 1) * sizeof(float), s>>>(
        ne, ws.v_rij, ws.v_ei, ws.v_ej, ws.v_a0,
                                                        species, d.S, d.nb, d.p, (float)d.rc, ws.K0p, ws.geo, ws.h0,
                                                   ctx->nl.flags.as<int>());
    span_end(ctx, sp_);
  }
  // two-body MLP; x0 = u * SiLU(a) of the last layer is not stored: its two
  // readers (the [w0 | e1] product and the first latent layer, operand and
  // residual) form it from the stored pre-activation a
  const bool tb1 = tb_fused(ctx, m);
  if (tb1) tb_fwd_async(ctx, m);
  for (int k = 0; k < d.n_tb && !tb1; ++k) {
    const Lin& L = *m->tb[k];
    ALoad ld = k == 0 ? a_plain(ws.h0, ws.K0p, ws.K0p) : a_silu(ws.a_tb[k - 1], d.tb[k - 1], d.tb[k - 1]);
    gemm(ctx, m, L, false, ld, e_store(ws.a_tb[k], d.tb[k], d.tb[k]), "fwd.twobody." + std::to_string(k));
  }
  const float* a_x0 = ws.a_tb[d.n_tb - 1];
  gemm(ctx, m, m->v0e1, false, a_silu_u(a_x0, d.D, d.D, u), e_store(ws.we1, 2 * d.NW, 2 * d.NW), "fwd.v0env1");
  const float inv_sqrt_nu = (float)d.inv_sqrt_nu;
  for (int t = 1; t <= d.T; ++t) {
    if (t > 1)
      gemm(ctx, m, *m->env[t - 1], false, a_plain(ws.x[t - 1], d.D, d.D), e_store(ws.e[t], d.NW, d.NW),
           "fwd.env" + std::to_string(t));
    const float* esrc = t == 1 ? ws.we1 + d.NW : ws.e[t];
    const int lde = t == 1 ? 2 * d.NW : d.NW;
    {
      const int sp_ = span_begin(ctx, "env_fwd" + std::to_string(t), 0, 4.0 * d.NW + 4.0 * d.NY, 0,
                                 4.0 * d.NY * d.C + 4.0);
#define NQ_ENVF(NYV, CV) \
  k_env_fwd<NYV, CV><<<grid_for(n, 4), 256, 0, s>>>(n, ne, ws.v_eoff, esrc, lde, ws.geo, inv_sqrt_nu, ws.gam[t])
      NQ_DISPATCH_NY_C(d.NY, d.C, NQ_ENVF);
#undef NQ_ENVF
      span_end(ctx, sp_);
    }
    launch_tp_fwd(ctx, m, t);
    NQ_HIP(hipGetLastError());
    // latent MLP on [x | s]; the last layer applies the residual update
    for (int k = 0; k < d.n_lat; ++k) {
      const Lin& L = *m->lat[t - 1][k];
      ALoad ld = k > 0    ? a_silu(ws.a_lat[t][k - 1], d.lat[k - 1], d.lat[k - 1])
                 : t == 1 ? a_cat_silu_u(a_x0, d.D, d.D, ws.s[t], d.nscal * d.C, d.nscal * d.C, u)
                          : a_cat(ws.x[t - 1], d.D, d.D, ws.s[t], d.nscal * d.C, d.nscal * d.C);
      Epi ep = e_store(ws.a_lat[t][k], d.lat[k], d.lat[k]);
      if (k == d.n_lat - 1) {
        ep.mode = E_RESIDUAL;
        ep.o1 = ws.x[t];
        ep.ld1 = d.D;
        ep.x = t == 1 ? a_x0 : ws.x[t - 1];
        ep.ldx = d.D;
        ep.rs = u;
        ep.rs_ld = kGeo;
        ep.xsilu = t == 1;
      }
      gemm(ctx, m, L, false, ld, ep, "fwd.latent" + std::to_string(t) + "." + std::to_string(k));
    }
  }
  for (int k = 0; k < d.n_edge; ++k) {
    ALoad ld = k == 0 ? a_plain(ws.x[d.T], d.D, d.D) : a_silu(ws.a_edge[k - 1], d.edge[k - 1], d.edge[k - 1]);
    gemm(ctx, m, *m->edge[k], false, ld, e_store(ws.a_edge[k], d.edge[k], d.edge[k]), "fwd.edge." + std::to_string(k));
  }
  const int ke = d.n_edge - 1;
  {
    const int sp_ = span_begin(ctx, "edge_energy", 0, 4.0 * d.edge[ke] + 4.0);
    k_edge_energy<<<grid_for(cap, 16), 256, 0, s>>>(ne, ws.a_edge[ke], d.edge[ke], d.edge[ke],
                                                          m->wout.as<float>(), (float)d.sigma_e, ws.eij);
    span_end(ctx, sp_);
  }
  {
    const int sp_ = span_begin(ctx, "atom_energy");
    k_atom_energy<<<grid_for(n, 256), 256, 0, s>>>(n, ne, ws.v_eoff, ws.eij, ws.atomE + ws.v_a0,
                                                   atom_energy ? atom_energy + ws.v_a0 : nullptr);
    span_end(ctx, sp_);
  }
  NQ_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ adjoint
void backward_async(nq_ctx* ctx, const nq_model* m) {
  const Dims& d = m->dims;
  Workspace& ws = ctx->ws;
  hipStream_t s = ctx->stream;
  const int* ne = ws.v_nedge;
  const int64_t cap = ws.cap;
  const float* u = ws.geo + 1;
  {
    const int sp_ = span_begin(ctx, "fill");
    k_fill<<<grid_for(cap, 256), 256, 0, s>>>(ws.gu, cap, 0.f);
    span_end(ctx, sp_);
  }
  // edge MLP: g_a(last) = sigma_E w_out SiLU'(a)
  {
    float* gout = nullptr;
    for (int k = d.n_edge - 1; k >= 0; --k) {
      ALoad ld = k == d.n_edge - 1
                     ? a_gradsilu(m->wout.as<float>(), 0, d.edge[k], ws.a_edge[k], d.edge[k], nullptr,
                                  (float)d.sigma_e)
                     : a_gradsilu(gout, ws.maxw, d.edge[k], ws.a_edge[k], d.edge[k], nullptr, 1.f);
      const int fin = k == 0 ? d.D : d.edge[k - 1];
      float* dst = k == 0 ? ws.gx : ws.gh[k % 2];
      gemm(ctx, m, *m->edge[k], true, ld, e_store(dst, k == 0 ? d.D : ws.maxw, fin), "bwd.edge." + std::to_string(k));
      gout = dst;
    }
  }
  int gvcur = 0;  // ws.gv[gvcur] holds dE/dV_t while processing layer t (t < T)
  for (int t = d.T; t >= 1; --t) {
    const int kl = d.n_lat - 1;
    float* gout = nullptr;
    for (int k = kl; k >= 0; --k) {
      // the first product also adds dE/du of the residual update to gu
      ALoad ld = k == kl ? a_gradsilu(ws.gx, d.D, d.lat[k], ws.a_lat[t][k], d.lat[k], u, kInvSqrt2, ws.gu)
                         : a_gradsilu(gout, ws.maxw, d.lat[k], ws.a_lat[t][k], d.lat[k], nullptr, 1.f);
      Epi ep;
      if (k == 0) {
        ep = Epi{E_LATENT_BWD, ws.gx, d.D, d.D + d.nscal * d.C, ws.gs, d.nscal * d.C, nullptr, 0, nullptr, 0, d.D};
      } else {
        ep = e_store(ws.gh[k % 2], ws.maxw, d.lat[k - 1]);
      }
      gemm(ctx, m, *m->lat[t - 1][k], true, ld, ep, "bwd.latent" + std::to_string(t) + "." + std::to_string(k));
      gout = ws.gh[k % 2];
    }
    // tensor-product adjoint, then the environment-sum adjoint -> gew[:, NW:2NW], gY
    launch_tp_bwd(ctx, m, t, ws.gv[gvcur], ws.gv[1 - gvcur]);
    gvcur = 1 - gvcur;
    launch_env_bwd(ctx, m, t);
    NQ_HIP(hipGetLastError());
    if (t > 1)
      gemm(ctx, m, *m->env[t - 1], true, a_plain(ws.gew + d.NW, 2 * d.NW, d.NW), e_add(ws.gx, d.D, d.D),
           "bwd.env" + std::to_string(t));
    else
      gemm(ctx, m, m->v0e1, true, a_plain(ws.gew, 2 * d.NW, 2 * d.NW), e_add(ws.gx, d.D, d.D), "bwd.v0env1");
  }
  // two-body MLP: x0 = u SiLU(a_last)
  const int kt = d.n_tb - 1;
  float* gout = nullptr;
  const bool tb1 = tb_fused(ctx, m);
  if (tb1) {
    tb_bwd_async(ctx, m);
    gout = ws.gh[0];
  }
  for (int k = kt; k >= 0 && !tb1; --k) {
    // the first product also adds dE/du of x0 = u SiLU(a) to gu
    ALoad ld = k == kt ? a_gradsilu(ws.gx, d.D, d.tb[k], ws.a_tb[k], d.tb[k], u, 1.f, ws.gu)
                       : a_gradsilu(gout, ws.maxw, d.tb[k], ws.a_tb[k], d.tb[k], nullptr, 1.f);
    const int fin = k == 0 ? d.n_in2b : d.tb[k - 1];
    gemm(ctx, m, *m->tb[k], true, ld, e_store(ws.gh[k % 2], ws.maxw, fin), "bwd.twobody." + std::to_string(k));
    gout = ws.gh[k % 2];
  }
  {
    // per edge: geo row, gu, dE/dY (T + 1 parts), dE/db, the edge slot, g_ij written
    const int sp_ = span_begin(ctx, "geometry_bwd", 0,
                               4.0 * kGeo + 4.0 + 4.0 * (d.T + 1) * d.NY + 4.0 * d.nb + 4.0 + 16.0);
    k_geometry_bwd<<<grid_for(cap, 256), 256, 0, s>>>(ne, ws.geo, ws.gu, ws.gY, d.T + 1, gout, ws.maxw, 2 * d.S, d.nb,
                                                            d.p, (float)d.rc, d.NY, ws.v_e0, ws.gr);
    span_end(ctx, sp_);
  }
  NQ_HIP(hipGetLastError());
}

// Whole-system totals after every chunk: compensated energy and force gather.
void finish_async(nq_ctx* ctx, const nq_model* m, double* energy, double* forces, int64_t n_rep,
                  int64_t n_centres) {
  Workspace& ws = ctx->ws;
  hipStream_t s = ctx->stream;
  const int64_t n = ws.n_atoms;
  int sp = span_begin(ctx, "total_energy");
  k_total_energy<<<(unsigned)n_rep, 1024, 0, s>>>(n / n_rep, ws.atomE, energy, ctx->nl.flags.as<int>());
  span_end(ctx, sp);
  sp = span_begin(ctx, "forces");
  const NbrList& nl = ctx->nl;
  k_forces<<<grid_for(n, 256), 256, 0, s>>>(n, n_centres < 0 ? n : n_centres, ws.nedge.as<int>(),
                                            ws.eoff.as<int>(), ws.ej.as<int>(), ws.rev.as<int>(),
                                            nl.nbr.as<int>(), nl.nbr_cnt.as<int>(), nl.k_max, ws.gr, forces,
                                            nl.flags.as<int>());
  span_end(ctx, sp);
  NQ_HIP(hipGetLastError());
}

}  // namespace nq
