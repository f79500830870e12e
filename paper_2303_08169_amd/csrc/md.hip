// Velocity-Verlet integration of Newton's equations (paper Sec. 2.1, Eq. 1) in FP64.
//   v += dt/2 * F/m;  r += dt * v (wrapped into the box);  F = F(r);  v += dt/2 * F/m
// Units: A, fs, amu, eV; 1 eV/(amu A) = 9.648533212e-3 A/fs^2 (CODATA 2018).
#include "nq_internal.hpp"

#include <mutex>

namespace nq {

namespace {

constexpr double kAcc = 9.648533212e-3;          // A/fs^2 per eV/(amu A)
constexpr double kEvPerAmuA2fs2 = 1.0 / kAcc;    // eV per amu A^2/fs^2

__global__ void k_half_kick(double* __restrict__ vel, const double* __restrict__ F,
                            const double* __restrict__ inv_mass, int64_t n, double half_dt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  vel[k] += half_dt * kAcc * F[k] * inv_mass[k / 3];
}

__global__ void k_drift(double* __restrict__ pos, const double* __restrict__ vel, int64_t n, double dt,
                        double Lx, double Ly, double Lz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  const int ax = (int)(k % 3);
  const double L = ax == 0 ? Lx : (ax == 1 ? Ly : Lz);
  double x = pos[k] + dt * vel[k];
  x -= L * floor(x / L);
  if (x >= L) x -= L;
  pos[k] = x;
}

__global__ __launch_bounds__(1024) void k_ekin(const double* __restrict__ vel, const double* __restrict__ inv_mass,
                                               int64_t n, double* __restrict__ out) {
  __shared__ double hs[1024], hc[1024];
  double s = 0.0, c = 0.0;
  for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
    const double vx = vel[3 * a], vy = vel[3 * a + 1], vz = vel[3 * a + 2];
    const double x = 0.5 * (vx * vx + vy * vy + vz * vz) / inv_mass[a] * kEvPerAmuA2fs2;
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
  if (threadIdx.x == 0) out[0] = hs[0] + hc[0];
}

// Appends this step's energies at the device-side step counter and advances it.
__global__ void k_record(const double* __restrict__ epot_now, const double* __restrict__ ekin_now,
                         int* counter, double* epot, double* ekin, int n_steps) {
  const int s = *counter;
  if (s < n_steps) {
    if (epot) epot[s] = epot_now[0];
    if (ekin) ekin[s] = ekin_now[0];
  }
  *counter = s + 1;
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// One Nose-Hoover thermostat half step of length h (constant-temperature
// runs of the robustness protocol, paper Sec. 3.2), single thread. With
// G(K) = (2K - N_f k_B T) / Q:
//   xi += G(K) h/2;  scale = exp(-xi h);  K *= scale^2;  eta += xi h;  xi += G(K) h/2,
// and the velocities are then multiplied by scale (k_scale_vel).
__global__ void k_nh_half(double* __restrict__ xi, double* __restrict__ eta, double* __restrict__ K,
                          double* __restrict__ scale, double nfkT, double Q, double h) {
  double x = xi[0], k = K[0];
  x += (2.0 * k - nfkT) / Q * 0.5 * h;
  const double sc = exp(-x * h);
  k *= sc * sc;
  eta[0] += x * h;
  x += (2.0 * k - nfkT) / Q * 0.5 * h;
  xi[0] = x;
  K[0] = k;
  scale[0] = sc;
}

__global__ void k_scale_vel(double* __restrict__ vel, int64_t n, const double* __restrict__ scale) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 3 * n) vel[k] *= scale[0];
}

// Thermostat energy Q xi^2 / 2 + N_f k_B T eta of the step being recorded.
__global__ void k_nh_record(const double* __restrict__ xi, const double* __restrict__ eta, const int* counter,
                            double* ethermo, int n_steps, double nfkT, double Q) {
  const int s = *counter;
  if (s < n_steps && ethermo) ethermo[s] = 0.5 * Q * xi[0] * xi[0] + nfkT * eta[0];
}

// Force outliers (the robustness measure of paper Sec. 3.2: force values
// beyond 5 sigma): over the 3n components of F, the mean mu and standard
// deviation sigma, then count[0] = #{k : |F_k - mu| > nsigma sigma}. One block.
__global__ __launch_bounds__(1024) void k_force_outliers(const double* __restrict__ F, int64_t m, double nsigma,
                                                         int* __restrict__ count) {
  __shared__ double s1[1024], s2[1024];
  __shared__ int sc[1024];
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < m; k += blockDim.x) {
    a += F[k];
    b += F[k] * F[k];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double mu = s1[0] / (double)m;
  const double var = s2[0] / (double)m - mu * mu;
  const double lim = nsigma * sqrt(var > 0.0 ? var : 0.0);
  int c = 0;
  for (int64_t k = threadIdx.x; k < m; k += blockDim.x) c += fabs(F[k] - mu) > lim;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sc[threadIdx.x] += sc[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[0] = sc[0];
}

__device__ inline double mic(double d, double L) { return d - L * rint(d / L); }

// Harmonic coupling of the R beads (replicas) of every atom into a ring
// (the path-integral ring polymer of the application in paper Sec. 5):
//   E = 1/2 sum_a m_a w^2 sum_k |r_{k+1,a} - r_{k,a}|^2,  bead R = bead 0,
//   F_{k,a} += m_a w^2 ((r_{k-1,a} - r_{k,a}) + (r_{k+1,a} - r_{k,a})),
// bead separations by minimum image. One thread per (bead, atom); e_bond gets
// the (k, k+1) bond energy of each thread.
__global__ void k_ring_polymer(const double* __restrict__ pos, const double* __restrict__ inv_mass, int64_t n,
                               int64_t R, double w2, double Lx, double Ly, double Lz,
                               double* __restrict__ forces, double* __restrict__ e_bond) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * R) return;
  const int64_t k = idx / n, a = idx % n;
  const int64_t prev = ((k + R - 1) % R) * n + a, next = ((k + 1) % R) * n + a;
  const double kappa = w2 / inv_mass[a] * kEvPerAmuA2fs2;  // eV / A^2
  const double L[3] = {Lx, Ly, Lz};
  double e = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double x = pos[3 * idx + c];
    const double dp = mic(pos[3 * prev + c] - x, L[c]), dn = mic(pos[3 * next + c] - x, L[c]);
    forces[3 * idx + c] += kappa * (dp + dn);
    e += dn * dn;
  }
  e_bond[idx] = 0.5 * kappa * e;
}

// Neumaier-compensated FP64 sum of n values by one block.
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ v, int64_t n, double* __restrict__ out) {
  __shared__ double hs[1024], hc[1024];
  double s = 0.0, c = 0.0;
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
      hc[threadIdx.x] += hc[threadIdx.x + o] + ((fabs(a) >= fabs(b)) ? (a - t) + b : (b - t) + a);
      hs[threadIdx.x] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = hs[0] + hc[0];
}

}  // namespace

// Bond energies of nq_ring_polymer_noalloc. A fixed array in device memory:
// every GPU the library runs on holds its own copy, at its own address, until
// the process ends, and every call on that GPU shares it. In host code this
// name is not a device address; kernels get the address that
// ring_polymer_static_scratch() looked up.
static __device__ __align__(256) double scratch[NQ_RING_POLYMER_NOALLOC_MAX];

double* ring_polymer_static_scratch(int device) {
  static std::mutex mu;
  static std::vector<double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
  if (!addr[(size_t)device]) {
    int cur = -1;
    NQ_HIP(hipGetDevice(&cur));
    NQ_REQUIRE(cur == device, NQ_ERR_DEVICE, "ring-polymer scratch looked up with another device current");
    void* p = nullptr;
    NQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    NQ_REQUIRE(p != nullptr, NQ_ERR_DEVICE, "no device address for the ring-polymer scratch");
    addr[(size_t)device] = (double*)p;
  }
  return addr[(size_t)device];
}

void md_half_kick_async(hipStream_t s, double* vel, const double* forces, const double* inv_mass, int64_t n,
                        double half_dt) {
  k_half_kick<<<(unsigned)cdiv(3 * n, 256), 256, 0, s>>>(vel, forces, inv_mass, n, half_dt);
}

void md_drift_async(hipStream_t s, double* pos, const double* vel, int64_t n, double dt, const double box[3]) {
  k_drift<<<(unsigned)cdiv(3 * n, 256), 256, 0, s>>>(pos, vel, n, dt, box[0], box[1], box[2]);
}

void md_ekin_async(hipStream_t s, const double* vel, const double* inv_mass, int64_t n, double* out) {
  k_ekin<<<1, 1024, 0, s>>>(vel, inv_mass, n, out);
}

void md_record_async(hipStream_t s, const double* epot_now, const double* ekin_now, int* counter, double* epot,
                     double* ekin, int n_steps) {
  k_record<<<1, 1, 0, s>>>(epot_now, ekin_now, counter, epot, ekin, n_steps);
}

void md_set_int_async(hipStream_t s, int* p, int v) { k_set_int<<<1, 1, 0, s>>>(p, v); }

void md_nh_half_async(hipStream_t s, double* vel, int64_t n, double* xi, double* eta, double* K, double* scale,
                      double nfkT, double Q, double h) {
  k_nh_half<<<1, 1, 0, s>>>(xi, eta, K, scale, nfkT, Q, h);
  k_scale_vel<<<(unsigned)cdiv(3 * n, 256), 256, 0, s>>>(vel, n, scale);
}

void md_nh_record_async(hipStream_t s, const double* xi, const double* eta, const int* counter, double* ethermo,
                        int n_steps, double nfkT, double Q) {
  k_nh_record<<<1, 1, 0, s>>>(xi, eta, counter, ethermo, n_steps, nfkT, Q);
}

void force_outliers_async(hipStream_t s, const double* forces, int64_t n, double nsigma, int* count) {
  k_force_outliers<<<1, 1024, 0, s>>>(forces, 3 * n, nsigma, count);
}

void ring_polymer_async(hipStream_t s, const double* pos, const double* inv_mass, int64_t n, int64_t R,
                        double omega_p, const double box[3], double* forces, double* e_bond, double* energy) {
  k_ring_polymer<<<(unsigned)cdiv(n * R, 256), 256, 0, s>>>(pos, inv_mass, n, R, omega_p * omega_p, box[0], box[1],
                                                           box[2], forces, e_bond);
  k_sum<<<1, 1024, 0, s>>>(e_bond, n * R, energy);
}

}  // namespace nq
