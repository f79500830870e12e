// Linked-cell neighbour list and per-evaluation edge list (gfx950).
//
// The paper builds an O(N) linked-list cell decomposition followed by a
// neighbour list (Sec. 2.4); here both live on the GPU. Atoms are binned into
// cells of side >= r_list by a counting sort (histogram, scan, scatter); one
// wavefront per atom scans the neighbouring cells with the minimum-image
// convention, compacts the hits with a ballot prefix count and sorts its row by
// neighbour index, so the list is deterministic. Each evaluation then compacts
// the skin list to the directed edges with d < r_c (edges sorted by (i, j)),
// and finds for every edge (i, j) the slot of its reverse (j, i) by binary
// search, which lets the force assembly gather instead of scatter.
//
// Several independent replicas of one box (ring-polymer beads) can share one
// list: atom a belongs to replica a / n_per, every replica has its own cell
// grid, and only atoms of the same replica are neighbours.
#include <cmath>

#include "nq_internal.hpp"

namespace nq {

namespace {

constexpr int kWave = 64;
constexpr int kRowsPerBlock = 4;  // one wavefront per atom row

struct CellGeom {
  double L[3];
  double inv_cell[3];
  int nc[3];
  int noff[3];
  int off[3][3];
  int ncell;      // cells of one replica
  int64_t n_per;  // atoms of one replica
};

__device__ inline double mic1(double d, double L) { return d - L * rint(d / L); }

__device__ inline double wrap1(double x, double L) {
  double w = x - L * floor(x / L);
  return (w >= L) ? w - L : w;
}

// Make this wavefront's LDS writes visible to all of its lanes.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ void k_zero_i32(int* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_bin(const double* __restrict__ pos, int64_t n, CellGeom g, int* atom_cell,
                      int* cell_count, int* flags, int predicated) {
  if (predicated && flags[1] == 0) return;
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  int c[3];
  for (int k = 0; k < 3; ++k) {
    double x = wrap1(pos[3 * a + k], g.L[k]);
    if (!(x >= 0.0 && x < g.L[k])) {  // NaN or infinite coordinate
      x = 0.0;
      atomicOr((int*)&flags[2], 1);
    }
    int ci = (int)(x * g.inv_cell[k]);
    c[k] = ci < 0 ? 0 : (ci >= g.nc[k] ? g.nc[k] - 1 : ci);
  }
  const int cell = (int)(a / g.n_per) * g.ncell + (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
  atom_cell[a] = cell;
  atomicAdd(&cell_count[cell], 1);
}

// Exclusive scan of a small int array by one block; also zeroes `fill`.
__global__ void k_scan_block(const int* __restrict__ in, int* out, int* fill, int64_t n,
                             const int* flags, int predicated) {
  if (predicated && flags[1] == 0) return;
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + blockDim.x - 1) / blockDim.x;
  const int64_t b = t * per, e = (b + per < n) ? b + per : n;
  int s = 0;
  for (int64_t i = b; i < e; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    int v = (t >= o) ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int64_t i = b; i < e; ++i) {
    out[i] = run;
    run += in[i];
    if (fill) fill[i] = 0;
  }
  if (t == (int)blockDim.x - 1) out[n] = part[t];
}

__global__ void k_scatter(int64_t n, const int* __restrict__ atom_cell, const int* __restrict__ cell_start,
                          int* cell_fill, int* cell_atoms, const int* flags, int predicated) {
  if (predicated && flags[1] == 0) return;
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  int c = atom_cell[a];
  int slot = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + slot] = (int)a;
}

// One wavefront per atom: gather list neighbours, sort the row, store it.
__global__ __launch_bounds__(kWave * kRowsPerBlock) void k_rows(
    const double* __restrict__ pos, int64_t n, CellGeom g, double r2list,
    const int* __restrict__ atom_cell, const int* __restrict__ cell_start,
    const int* __restrict__ cell_atoms, int* nbr, int* nbr_cnt, double* pos_ref, int k_max,
    int* flags, int predicated) {
  if (predicated && flags[1] == 0) return;
  extern __shared__ int rowbuf[];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t a = (int64_t)blockIdx.x * kRowsPerBlock + w;
  if (a >= n) return;
  int* row = rowbuf + w * k_max;
  const double ax = pos[3 * a], ay = pos[3 * a + 1], az = pos[3 * a + 2];
  const int rep0 = atom_cell[a] / g.ncell * g.ncell;  // first cell of this atom's replica
  const int cell = atom_cell[a] - rep0;
  const int cx = cell % g.nc[0], cy = (cell / g.nc[0]) % g.nc[1], cz = cell / (g.nc[0] * g.nc[1]);
  int cnt = 0;
  for (int oz = 0; oz < g.noff[2]; ++oz)
    for (int oy = 0; oy < g.noff[1]; ++oy)
      for (int ox = 0; ox < g.noff[0]; ++ox) {
        int x = (cx + g.off[0][ox] + g.nc[0]) % g.nc[0];
        int y = (cy + g.off[1][oy] + g.nc[1]) % g.nc[1];
        int z = (cz + g.off[2][oz] + g.nc[2]) % g.nc[2];
        int c = rep0 + (z * g.nc[1] + y) * g.nc[0] + x;
        int s = cell_start[c], e = cell_start[c + 1];
        for (int base = s; base < e; base += kWave) {
          int idx = base + lane;
          bool hit = false;
          int b = -1;
          if (idx < e) {
            b = cell_atoms[idx];
            if (b != a) {
              double dx = mic1(pos[3 * b] - ax, g.L[0]);
              double dy = mic1(pos[3 * b + 1] - ay, g.L[1]);
              double dz = mic1(pos[3 * b + 2] - az, g.L[2]);
              hit = dx * dx + dy * dy + dz * dz < r2list;
            }
          }
          uint64_t m = __ballot(hit);
          int slot = cnt + __popcll(m & lanemask_lt());
          if (hit && slot < k_max) row[slot] = b;
          cnt += __popcll(m);
        }
      }
  wave_sync();
  const int kept = cnt < k_max ? cnt : k_max;
  if (cnt > k_max && lane == 0) atomicMax(&flags[0], cnt);
  // rank sort of distinct indices
  for (int i = lane; i < kept; i += kWave) {
    int v = row[i];
    int r = 0;
    for (int k = 0; k < kept; ++k) r += (row[k] < v);
    nbr[a * (int64_t)k_max + r] = v;
  }
  if (lane == 0) {
    nbr_cnt[a] = kept;
    pos_ref[3 * a] = ax;
    pos_ref[3 * a + 1] = ay;
    pos_ref[3 * a + 2] = az;
  }
}

__global__ void k_finish_rebuild(int* flags, int predicated) {
  if (predicated && flags[1] == 0) return;
  flags[1] = 0;
  flags[3] += 1;
}

__global__ void k_displacement(const double* __restrict__ pos, const double* __restrict__ pos_ref,
                               int64_t n, double Lx, double Ly, double Lz, double lim2, int* flags) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double dx = mic1(pos[3 * a] - pos_ref[3 * a], Lx);
  double dy = mic1(pos[3 * a + 1] - pos_ref[3 * a + 1], Ly);
  double dz = mic1(pos[3 * a + 2] - pos_ref[3 * a + 2], Lz);
  double d2 = dx * dx + dy * dy + dz * dz;
  if (d2 > lim2 || !(d2 == d2)) flags[1] = 1;
}

// ---- per-evaluation edge list
// Atoms a >= n_centres (ghosts of a spatial domain) are not centres: their
// edge rows are empty.
__global__ __launch_bounds__(kWave * kRowsPerBlock) void k_edge_count(
    const double* __restrict__ pos, int64_t n, int64_t n_centres, double Lx, double Ly, double Lz, double rc2,
    const int* __restrict__ nbr, const int* __restrict__ nbr_cnt, int k_max, int* ecnt) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t a = (int64_t)blockIdx.x * kRowsPerBlock + w;
  if (a >= n) return;
  const double ax = pos[3 * a], ay = pos[3 * a + 1], az = pos[3 * a + 2];
  const int cnt = a < n_centres ? nbr_cnt[a] : 0;
  int total = 0;
  for (int base = 0; base < cnt; base += kWave) {
    int k = base + lane;
    bool hit = false;
    if (k < cnt) {
      int b = nbr[a * (int64_t)k_max + k];
      double dx = mic1(pos[3 * b] - ax, Lx), dy = mic1(pos[3 * b + 1] - ay, Ly),
             dz = mic1(pos[3 * b + 2] - az, Lz);
      hit = dx * dx + dy * dy + dz * dz < rc2;
    }
    total += __popcll(__ballot(hit));
  }
  if (lane == 0) ecnt[a] = total;
}

__global__ __launch_bounds__(kWave * kRowsPerBlock) void k_edge_fill(
    const double* __restrict__ pos, int64_t n, int64_t n_centres, double Lx, double Ly, double Lz, double rc2,
    const int* __restrict__ nbr, const int* __restrict__ nbr_cnt, int k_max,
    const int* __restrict__ eoff, int64_t cap, int* ei, int* ej, float4* rij, int* flags) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t a = (int64_t)blockIdx.x * kRowsPerBlock + w;
  if (a >= n) return;
  const double ax = pos[3 * a], ay = pos[3 * a + 1], az = pos[3 * a + 2];
  const int cnt = a < n_centres ? nbr_cnt[a] : 0;
  int64_t out = eoff[a];
  for (int base = 0; base < cnt; base += kWave) {
    int k = base + lane;
    bool hit = false;
    int b = 0;
    double dx = 0, dy = 0, dz = 0, d2 = 0;
    if (k < cnt) {
      b = nbr[a * (int64_t)k_max + k];
      dx = mic1(pos[3 * b] - ax, Lx);
      dy = mic1(pos[3 * b + 1] - ay, Ly);
      dz = mic1(pos[3 * b + 2] - az, Lz);
      d2 = dx * dx + dy * dy + dz * dz;
      hit = d2 < rc2;
      if (!(d2 == d2) || (hit && d2 < 1e-2)) flags[2] = 1;  // NaN or d < 0.1 A
    }
    uint64_t m = __ballot(hit);
    int64_t slot = out + __popcll(m & lanemask_lt());
    if (hit && slot < cap) {
      ei[slot] = (int)a;
      ej[slot] = b;
      rij[slot] = make_float4((float)dx, (float)dy, (float)dz, (float)sqrt(d2));
    }
    out += __popcll(m);
  }
}

// Slot of the reverse edge (j, i) of every edge (i, j), or INT_MAX when there
// is none (j is a ghost, which is no centre).
__global__ void k_edge_rev(const int* __restrict__ nedge, const int* __restrict__ ei,
                           const int* __restrict__ ej, const int* __restrict__ eoff, int* rev) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ne = *nedge;
  if (e >= ne) return;
  int i = ei[e], j = ej[e];
  int lo = min(eoff[j], ne), hi = min(eoff[j + 1], ne);
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ej[mid] < i) lo = mid + 1; else hi = mid;
  }
  rev[e] = (lo < min(eoff[j + 1], ne) && ej[lo] == i) ? lo : 0x7fffffff;
}

// nedge = min(total, cap); an overflow is reported through flags[4].
__global__ void k_set_edge_count(const int* __restrict__ total, int* nedge, int64_t cap, int* flags) {
  const int t = *total;
  if (t > cap) flags[4] = t;
  *nedge = t > cap ? (int)cap : t;
}

CellGeom make_geom(const NbrList& nl) {
  CellGeom g{};
  for (int k = 0; k < 3; ++k) {
    g.L[k] = nl.box[k];
    g.nc[k] = nl.nc[k];
    g.inv_cell[k] = nl.nc[k] / nl.box[k];
    if (nl.nc[k] >= 3) {
      g.noff[k] = 3;
      g.off[k][0] = -1; g.off[k][1] = 0; g.off[k][2] = 1;
    } else if (nl.nc[k] == 2) {
      g.noff[k] = 2;
      g.off[k][0] = 0; g.off[k][1] = 1;
    } else {
      g.noff[k] = 1;
      g.off[k][0] = 0;
    }
  }
  g.ncell = nl.nc[0] * nl.nc[1] * nl.nc[2];
  g.n_per = nl.n / nl.n_rep;
  return g;
}

}  // namespace

void nbr_configure(nq_ctx* ctx, int64_t n, const double cell[3], double r_cut, double skin, int64_t n_rep) {
  NbrList& nl = ctx->nl;
  NQ_REQUIRE(n_rep >= 1 && n % n_rep == 0 && n / n_rep > 1, NQ_ERR_ARG, "replicas must split the atoms evenly");
  const double rl = r_cut + skin;
  for (int k = 0; k < 3; ++k)
    NQ_REQUIRE(std::isfinite(cell[k]) && cell[k] > 0 && rl < 0.5 * cell[k], NQ_ERR_ARG,
               "r_cut + skin must be below half of every box length (minimum image)");
  NQ_REQUIRE(r_cut > 0 && skin >= 0, NQ_ERR_ARG, "bad r_cut or skin");
  NQ_REQUIRE(n > 1 && n < (int64_t)1 << 30, NQ_ERR_ARG, "n out of range");
  const bool same = nl.n == n && nl.n_rep == n_rep && nl.box[0] == cell[0] && nl.box[1] == cell[1] &&
                    nl.box[2] == cell[2] && nl.r_cut == r_cut && nl.skin == skin;
  if (same && nl.k_max > 0) return;
  ++ctx->gen;
  nl.n = n;
  nl.n_rep = n_rep;
  for (int k = 0; k < 3; ++k) {
    nl.box[k] = cell[k];
    nl.nc[k] = std::max(1, (int)std::floor(cell[k] / rl));
  }
  nl.r_cut = r_cut;
  nl.skin = skin;
  const double vol = cell[0] * cell[1] * cell[2];
  const double expect = 4.0 / 3.0 * M_PI * rl * rl * rl * (double)(n / n_rep) / vol;
  int kmax = (int)rup((int64_t)(1.5 * expect + 32), 32);
  nl.k_max = (int)std::min<int64_t>(kmax, rup(n / n_rep, 32));
  nl.built = false;
  const int64_t ncell = (int64_t)nl.nc[0] * nl.nc[1] * nl.nc[2] * n_rep;
  NQ_REQUIRE(ncell < ((int64_t)1 << 30), NQ_ERR_ARG, "too many cells");
  nl.cell_count.ensure(ncell * 4);
  nl.cell_start.ensure((ncell + 1) * 4);
  nl.cell_fill.ensure(ncell * 4);
  nl.cell_atoms.ensure(n * 4);
  nl.atom_cell.ensure(n * 4);
  nl.nbr.ensure((size_t)n * nl.k_max * 4);
  nl.nbr_cnt.ensure(n * 4);
  nl.pos_ref.ensure(n * 3 * 8);
  nl.flags.ensure(8 * 4);
  NQ_HIP(hipMemsetAsync(nl.flags.p, 0, 8 * 4, ctx->stream));
}

void nbr_build_async(nq_ctx* ctx, const double* pos, bool predicated) {
  NbrList& nl = ctx->nl;
  NQ_REQUIRE(nl.k_max > 0 && nl.k_max <= 2048, NQ_ERR_CAPACITY, "neighbour row capacity out of range");
  const CellGeom g = make_geom(nl);
  const int64_t ncell = (int64_t)g.ncell * nl.n_rep;
  const int64_t n = nl.n;
  hipStream_t s = ctx->stream;
  int* flags = nl.flags.as<int>();
  const int pr = predicated ? 1 : 0;
  const double rl = nl.r_cut + nl.skin;
  // zeroing is cheap and harmless when the rebuild is skipped
  k_zero_i32<<<cdiv(ncell, 256), 256, 0, s>>>(nl.cell_count.as<int>(), ncell);
  k_bin<<<cdiv(n, 256), 256, 0, s>>>(pos, n, g, nl.atom_cell.as<int>(), nl.cell_count.as<int>(), flags, pr);
  k_scan_block<<<1, 1024, 0, s>>>(nl.cell_count.as<int>(), nl.cell_start.as<int>(), nl.cell_fill.as<int>(),
                                  ncell, flags, pr);
  k_scatter<<<cdiv(n, 256), 256, 0, s>>>(n, nl.atom_cell.as<int>(), nl.cell_start.as<int>(),
                                         nl.cell_fill.as<int>(), nl.cell_atoms.as<int>(), flags, pr);
  const size_t lds = (size_t)nl.k_max * kRowsPerBlock * sizeof(int);
  k_rows<<<cdiv(n, kRowsPerBlock), kWave * kRowsPerBlock, lds, s>>>(
      pos, n, g, rl * rl, nl.atom_cell.as<int>(), nl.cell_start.as<int>(), nl.cell_atoms.as<int>(),
      nl.nbr.as<int>(), nl.nbr_cnt.as<int>(), nl.pos_ref.as<double>(), nl.k_max, flags, pr);
  k_finish_rebuild<<<1, 1, 0, s>>>(flags, pr);
  NQ_HIP(hipGetLastError());
}

void nbr_displacement_check_async(nq_ctx* ctx, const double* pos, double half) {
  NbrList& nl = ctx->nl;
  k_displacement<<<cdiv(nl.n, 256), 256, 0, ctx->stream>>>(pos, nl.pos_ref.as<double>(), nl.n, nl.box[0],
                                                           nl.box[1], nl.box[2], half * half,
                                                           nl.flags.as<int>());
  NQ_HIP(hipGetLastError());
}

void edges_build_async(nq_ctx* ctx, const double* pos, double r_cut, int64_t n_centres) {
  NbrList& nl = ctx->nl;
  Workspace& ws = ctx->ws;
  const int64_t n = nl.n;
  if (n_centres < 0) n_centres = n;
  hipStream_t s = ctx->stream;
  const double rc2 = r_cut * r_cut;
  const int blocks = (int)cdiv(n, kRowsPerBlock);
  k_edge_count<<<blocks, kWave * kRowsPerBlock, 0, s>>>(pos, n, n_centres, nl.box[0], nl.box[1], nl.box[2], rc2,
                                                         nl.nbr.as<int>(), nl.nbr_cnt.as<int>(), nl.k_max,
                                                         ws.ecnt.as<int>());
  k_scan_block<<<1, 1024, 0, s>>>(ws.ecnt.as<int>(), ws.eoff.as<int>(), nullptr, n, nullptr, 0);
  // the total edge count lives in eoff[n]
  k_set_edge_count<<<1, 1, 0, s>>>(ws.eoff.as<int>() + n, ws.nedge.as<int>(), ws.cap_all, nl.flags.as<int>());
  k_edge_fill<<<blocks, kWave * kRowsPerBlock, 0, s>>>(pos, n, n_centres, nl.box[0], nl.box[1], nl.box[2], rc2,
                                                        nl.nbr.as<int>(), nl.nbr_cnt.as<int>(), nl.k_max,
                                                        ws.eoff.as<int>(), ws.cap_all, ws.ei.as<int>(),
                                                        ws.ej.as<int>(), ws.rij.as<float4>(),
                                                        nl.flags.as<int>());
  k_edge_rev<<<cdiv(ws.cap_all, 256), 256, 0, s>>>(ws.nedge.as<int>(), ws.ei.as<int>(), ws.ej.as<int>(),
                                               ws.eoff.as<int>(), ws.rev.as<int>());
  NQ_HIP(hipGetLastError());
}

}  // namespace nq
