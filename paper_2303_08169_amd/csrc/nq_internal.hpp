// Internal declarations of the gfx950 energy/force library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/nnqmd.h"

namespace nq {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMaxL = 2;                     // highest irrep order supported
constexpr int kMaxNY = (kMaxL + 1) * (kMaxL + 1);
constexpr int kMaxPaths = 11;

// Error carrying status + message, thrown only inside the library and turned
// into an nq_status at the ABI boundary.
struct Error {
  nq_status status;
  std::string msg;
};

#define NQ_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::nq::Error{e_ == hipErrorOutOfMemory ? NQ_ERR_OOM : NQ_ERR_DEVICE,          \
                        std::string(#call) + ": " + hipGetErrorString(e_)};              \
  } while (0)

#define NQ_REQUIRE(cond, status, msg)                     \
  do {                                                    \
    if (!(cond)) throw ::nq::Error{(status), (msg)};      \
  } while (0)

// A device allocation that grows on demand and frees itself.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t nbytes) {
    if (nbytes <= bytes) return;
    release();
    NQ_HIP(hipMalloc(&p, nbytes ? nbytes : 1));
    bytes = nbytes;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Derived sizes of one model.
struct Dims {
  int S, nb, p, L, T, C, D;
  int NY;      // (L+1)^2 spherical-harmonic components
  int NW;      // (L+1)*C per-edge weights of one l-block
  int nscal;   // number of coupling paths with l3 = 0
  int n_paths; // all coupling paths
  int n_in2b;  // 2S + nb two-body input width
  int n_tb, tb[4], n_lat, lat[4], n_edge, edge[4];
  double rc, inv_sqrt_nu, sigma_e;
  int prec;
  int paths[kMaxPaths][3];
  int path_l3_count[kMaxL + 1];
};

// One linear map y = x W stored for the matrix-core kernels.
//  fwd: B operand of y = x W, laid out [Np][Kp] with K contiguous (W^T), Kp = fin
//       padded to 32, Np = fout padded to 16.
//  bwd: B operand of gx = gy W^T, laid out [Np][Kp] = W with fin padded to 16 rows
//       and fout padded to 32 columns.
//  The BF16 buffers hold two [Np][Kp] halves: hi = rne(w) and lo = rne(w - hi).
struct Lin {
  int fin = 0, fout = 0;
  int kp_f = 0, np_f = 0, kp_b = 0, np_b = 0;
  DevBuf f32_fwd, f32_bwd, bf_fwd, bf_bwd;
};

// Channel-mixing weights of one layer (see upload_mix).
struct MixW {
  int64_t n = 0;               // floats per copy
  DevBuf fN, fT, bN, bT;       // FP32 natural / transposed, BF16 [hi | lo] natural / transposed
};

// Dense real coupling tables C^(l1,l2,l3)[m1][m2][m3], indexed by path triple.
struct CGTable {
  float v[kMaxL + 1][kMaxL + 1][kMaxL + 1][2 * kMaxL + 1][2 * kMaxL + 1][2 * kMaxL + 1];
};

}  // namespace nq

struct nq_model {
  nq_ctx* ctx = nullptr;
  nq_model_desc desc{};
  nq::Dims dims{};
  std::vector<nq::Lin*> tb;                 // two-body layers
  nq::Lin v0e1;                             // [W_V0 | W_env^1]
  std::vector<nq::Lin*> env;                // W_env^t for t >= 2 (index t-1; [0] unused)
  std::vector<std::vector<nq::Lin*>> lat;   // latent layers per layer t (index t-1)
  std::vector<nq::Lin*> edge;               // hidden edge-MLP layers
  nq::DevBuf wout;                          // [edge_last] f32 final edge weights
  std::vector<nq::MixW*> mixw;              // per layer t < T (index t-1)
  std::vector<double> tp_flop_fwd, tp_flop_bwd;  // algorithmic FLOPs per edge of each layer's tensor product
  std::vector<double> tp_flop_mix;               // ... of which the channel mixing (matrix cores), each direction
  mutable std::map<std::string, int> gemm_choice;  // tuned tile shape per matrix-core product
  std::map<std::string, int> site_prec;            // per-product precision (nq_model_set_product_precision)
  int64_t version = 0;  // bumped when a kernel choice or precision changes (part of the MD graph key)
  ~nq_model();
};

namespace nq {

struct NbrList {
  int64_t n = 0;          // atoms of all replicas
  int64_t n_rep = 1;      // independent replicas (same box), n / n_rep atoms each
  double box[3] = {0, 0, 0};
  double r_cut = 0, skin = 0;
  int nc[3] = {0, 0, 0};
  int k_max = 0;
  int64_t n_entries = 0;  // total skin-list entries at the last host-visible build
  std::vector<int64_t> entry_prefix;  // prefix sums of the row counts at that build (host)
  bool built = false;
  DevBuf cell_count, cell_start, cell_fill, cell_atoms, atom_cell;
  DevBuf nbr, nbr_cnt, pos_ref;
  // flags[0] row overflow (largest row), [1] rebuild requested, [2] numeric problem,
  // [3] rebuild count, [4] edge overflow (edge total), [5] species out of range
  DevBuf flags;
};

// Per-edge workspace of the layered pipeline. The edge list of the whole
// system holds up to cap_all edges; the per-edge activations hold `cap` edges,
// one chunk of consecutive centres at a time (one chunk covers the whole system
// when it fits the memory budget).
struct Workspace {
  int64_t cap = 0;       // edges per chunk (activation buffers)
  int64_t cap_all = 0;   // edges of the whole system (edge list, per-edge gradients)
  int64_t n_atoms = 0;
  const nq_model* model = nullptr;
  DevBuf ecnt, eoff, ei, ej, rev, rij, nedge;  // edge list of the whole system
  DevBuf c_ei, c_ej, c_rij, c_eoff, c_nedge;    // chunk-local copies (chunked mode)
  DevBuf grbuf;                                 // dE/dr_ij of every edge
  std::vector<std::unique_ptr<DevBuf>> bufs;    // model-dependent buffers
  std::vector<int64_t> chunks;                  // centre boundaries a_0 = 0 < a_1 < ... = n
  int K0p = 0, maxw = 0;
  bool has_act = false;                         // the layered kernels' buffers exist
  // current chunk view: centres [v_a0, v_a0 + v_n), edges renumbered from 0
  int64_t v_a0 = 0, v_n = 0;
  const int *v_nedge = nullptr, *v_ei = nullptr, *v_ej = nullptr, *v_eoff = nullptr, *v_e0 = nullptr;
  const float4* v_rij = nullptr;
  float *geo = nullptr, *h0 = nullptr, *we1 = nullptr, *eij = nullptr;
  float *gx = nullptr, *gh[2] = {nullptr, nullptr}, *gs = nullptr, *gv[2] = {nullptr, nullptr};
  float *ggc = nullptr, *gew = nullptr, *gY = nullptr, *gu = nullptr;
  float4* gr = nullptr;
  double *atomE = nullptr, *esum = nullptr;
  std::vector<float*> a_tb, a_edge, x, gam, s, V, e;
  std::vector<std::vector<float*>> a_lat;
};

}  // namespace nq

namespace nq {
// One timed launch (or group of launches) recorded while timing is enabled.
struct Span {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  double flop_per_edge = 0, byte_per_edge = 0;  // algorithmic work per in-cutoff edge
  double flop_per_atom = 0, byte_per_atom = 0;  // ... or per atom
  double mfma_flop_per_edge = 0;                // part of flop_per_edge done on the matrix cores
};
}  // namespace nq

struct nq_ctx {
  int device = 0;
  int num_cu = 256;  // compute units of the device
  hipStream_t stream = nullptr;
  std::string last_error;
  nq::NbrList nl;
  nq::Workspace ws;
  // MD graph state
  hipStream_t md_stream = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec = nullptr;
  std::vector<const void*> graph_key;
  // Bumped whenever device buffers or sizes that a captured graph bakes in
  // change (neighbour-list geometry or row capacity, workspace reallocation);
  // part of the graph key, so such a change forces a new capture.
  int64_t gen = 0;
  int64_t graph_captures = 0;
  nq::DevBuf md_scratch;
  nq::DevBuf fz_scratch;  // per-workgroup scratch of the fused kernel
  int path = NQ_PATH_AUTO;  // nq_ctx_set_path
  nq::DevBuf rp_scratch;  // ring-polymer bond energies
  double* rp_static = nullptr;  // this device's fixed bond-energy array (nq_ring_polymer_noalloc)
  int64_t last_edges = 0;
  int64_t ws_budget = (int64_t)160 << 30;  // bytes allowed for per-edge activations
  // per-launch timing with HIP events on the context's stream
  bool timing = false;
  int force_variant = -1;               // >= 0 while the autotuner times one tile shape
  int user_variant = NQ_VARIANT_TUNED;  // nq_ctx_set_variant
  std::map<std::string, int> site_np;   // output width of each named matrix-core product
  std::map<std::string, int> site_nvar; // kernel variants available for it
  std::vector<nq::Span> spans;
  std::vector<hipEvent_t> event_pool;
};

namespace nq {

// ---- neighbour list (neighbor.hip)
void nbr_configure(nq_ctx* ctx, int64_t n, const double cell[3], double r_cut, double skin, int64_t n_rep = 1);
void nbr_build_async(nq_ctx* ctx, const double* pos, bool predicated);
void nbr_displacement_check_async(nq_ctx* ctx, const double* pos, double half_margin);
// Edges of centres a < n_centres (all atoms when n_centres < 0).
void edges_build_async(nq_ctx* ctx, const double* pos, double r_cut, int64_t n_centres = -1);

// ---- model (model.cpp)
Dims make_dims(const nq_model_desc& d);
nq_model* model_create(nq_ctx* ctx, const nq_model_desc* desc, const double* w, int64_t n_w);
void weight_layout(const nq_model_desc& d, std::vector<std::pair<int64_t, int64_t>>& segs);
void derive_cg(CGTable& t);

// ---- pipeline (forward.hip / backward.hip)
// activations: allocate the per-edge buffers of the layered kernels too.
void ws_ensure(nq_ctx* ctx, const nq_model* m, int64_t cap_all, int64_t n_atoms, bool activations);
void chunk_view_async(nq_ctx* ctx, int chunk);
void forward_async(nq_ctx* ctx, const nq_model* m, const int32_t* species, double* atom_energy);
void backward_async(nq_ctx* ctx, const nq_model* m);
// Energies (one per replica) and forces of all atoms; atoms a >= n_centres
// (ghosts) also gather the edges that point at them through the neighbour list.
void finish_async(nq_ctx* ctx, const nq_model* m, double* energy, double* forces, int64_t n_rep = 1,
                  int64_t n_centres = -1);

// ---- fused per-centre kernel (fused.hip)
bool fused_supported(const nq_model* m);
// Sizes the fused kernel's scratch for the current neighbour list (outside graph capture).
void fused_prepare(nq_ctx* ctx);
// E_i (ws.atomE, and atom_energy when not null) and g_ij (ws.grbuf) of the
// whole edge list in one launch; atoms >= n_centres (>= 0) have no edges.
void fused_async(nq_ctx* ctx, const nq_model* m, const int32_t* species, double* atom_energy, int64_t n_centres);


// ---- MD (md.hip)
void md_half_kick_async(hipStream_t s, double* vel, const double* forces, const double* inv_mass,
                        int64_t n, double half_dt);
void md_drift_async(hipStream_t s, double* pos, const double* vel, int64_t n, double dt,
                    const double box[3]);
// Nose-Hoover thermostat half step of length h on vel (xi, eta, K, scale: one
// device double each), and the record of its energy into ethermo[*counter].
void md_nh_half_async(hipStream_t s, double* vel, int64_t n, double* xi, double* eta, double* K, double* scale,
                      double nfkT, double Q, double h);
void md_nh_record_async(hipStream_t s, const double* xi, const double* eta, const int* counter, double* ethermo,
                        int n_steps, double nfkT, double Q);
// count[0] = force components of F[n*3] farther than nsigma standard deviations from their mean.
void force_outliers_async(hipStream_t s, const double* forces, int64_t n, double nsigma, int* count);
// Ring-polymer springs of R beads x n atoms: forces += spring forces (eV/A),
// energy[0] = spring energy (eV); e_bond: n R doubles of scratch.
void ring_polymer_async(hipStream_t s, const double* pos, const double* inv_mass, int64_t n, int64_t R,
                        double omega_p, const double box[3], double* forces, double* e_bond, double* energy);
void md_ekin_async(hipStream_t s, const double* vel, const double* inv_mass, int64_t n,
                   double* out);
// out[e][c] = u_e SiLU(a[e][c]) over the last evaluation's edges: the two-body
// output x0, which the pipeline forms at use instead of storing (stage export).
void debug_x0_async(nq_ctx* ctx, const nq_model* m, float* out);
// Device address of the fixed ring-polymer bond-energy array on `device`
// (NQ_RING_POLYMER_NOALLOC_MAX doubles), looked up once per device; the
// device must be current.
double* ring_polymer_static_scratch(int device);
// The two-body MLP as one kernel per direction (benchmark widths, BF16 kinds,
// automatic path only); bitwise the per-layer products.
bool tb_fused(const nq_ctx* ctx, const nq_model* m);
void tb_fwd_async(nq_ctx* ctx, const nq_model* m);
void tb_bwd_async(nq_ctx* ctx, const nq_model* m);

// Arithmetic of one product site: its override, else the model's precision.
inline int site_precision(const nq_model* m, const std::string& site) {
  auto it = m->site_prec.find(site);
  return it == m->site_prec.end() ? m->dims.prec : it->second;
}

// Start/stop a timed span on ctx->stream (no-ops unless timing is enabled).
int span_begin(nq_ctx* ctx, const std::string& name, double flop_per_edge = 0, double byte_per_edge = 0,
               double flop_per_atom = 0, double byte_per_atom = 0, double mfma_flop_per_edge = 0);
void span_end(nq_ctx* ctx, int idx);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

}  // namespace nq
