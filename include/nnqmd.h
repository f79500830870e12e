/*
 * nnqmd.h - C ABI of the MI355X (gfx950) energy/force library for an
 * Allegro-style neural-network interatomic potential.
 *
 * The library evaluates, for a periodic orthorhombic box of atoms, the total
 * potential energy E built from pairwise embedding energies E_ij of atom pairs
 * within a cutoff, and the forces f_i = -dE/dr_i, and advances Newton's
 * equations m_i d^2 r_i/dt^2 = f_i (paper Sec. 2.1, Eq. 1). Pairs are found
 * with a linked-cell neighbour list (Sec. 2.4). The equivariant edge model
 * (radial Bessel basis with polynomial cutoff, real spherical harmonics Y_l,
 * two-body / latent / edge MLPs, environment sums over neighbours,
 * Clebsch-Gordan tensor products; Sec. 2.1) is written out in the library's
 * design notes; forces come from a hand-written adjoint of every step.
 *
 * Conventions shared by every entry point
 *   - Units: Angstrom, eV, fs, amu. Forces in eV/A.
 *   - Arrays are contiguous, row-major. Unless stated otherwise an array
 *     pointer is a DEVICE pointer (e.g. torch.Tensor.data_ptr() of a CUDA/HIP
 *     tensor) on the context's device, owned by the caller, and must stay valid
 *     until the work queued on the context's stream has finished.
 *   - cell[3] is a HOST array with the three orthorhombic box lengths.
 *   - All GPU work is queued asynchronously on the context's stream; results
 *     are valid after that stream is synchronised. Calls on one context must
 *     not overlap (a context is not thread-safe).
 *   - Errors are returned as nq_status; no C++ exception crosses the ABI. The
 *     message of the last error on a context is available from nq_last_error.
 *   - Model weights are one flat FP64 host blob; each segment is a row-major
 *     [fan_in, fan_out] matrix of a linear map y = x W (no biases), in the order
 *     reported by nq_model_weight_layout.
 */
#ifndef NNQMD_H
#define NNQMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NQ_OK = 0,
  NQ_ERR_ARG = -1,          /* bad pointer, size, species or geometry argument */
  NQ_ERR_UNSUPPORTED = -2,  /* model shape or option the library does not support */
  NQ_ERR_CAPACITY = -3,     /* neighbour-list row or edge capacity exceeded */
  NQ_ERR_NUMERIC = -4,      /* non-finite value or coincident atoms detected */
  NQ_ERR_DEVICE = -5,       /* HIP runtime error */
  NQ_ERR_OOM = -6           /* device allocation failed */
} nq_status;

enum { NQ_PRECISION_FP32 = 0, NQ_PRECISION_BF16 = 1, NQ_PRECISION_BF16X3 = 2 };

typedef struct nq_ctx nq_ctx;
typedef struct nq_model nq_model;

/* Model hyper-parameters. Widths of MLP layers are listed without the input
 * width; twobody[n_twobody-1] is the latent width D and latent[n_latent-1] must
 * equal D. lmax <= 2. n_species <= 8. precision selects the arithmetic of the
 * per-edge MLP products: NQ_PRECISION_FP32 (FP32 operands on the matrix cores),
 * NQ_PRECISION_BF16 (BF16 operands on the matrix cores, FP32 accumulation) or
 * NQ_PRECISION_BF16X3 (each FP32 operand split into BF16 hi + lo parts and the
 * product formed as hi*hi + lo*hi + hi*lo on the matrix cores, FP32
 * accumulation: about FP32 accuracy at three BF16 products' cost). Tensor
 * products, reductions and everything else stay FP32/FP64 in every mode. */
typedef struct {
  int32_t n_species, n_bessel, poly_p, lmax, n_layers, channels;
  int32_t n_twobody, twobody[4];
  int32_t n_latent, latent[4];
  int32_t n_edge, edge[4];
  double r_cut;             /* cutoff r_c in A */
  double avg_num_neighbors; /* nu: environment sums are scaled by nu^-1/2 */
  double energy_scale;      /* sigma_E multiplying every E_ij */
  int32_t precision;
} nq_model_desc;

/* Create a context on HIP device `device` that queues work on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
nq_status nq_ctx_create(int device, void* hip_stream, nq_ctx** out);
/* Change the stream of an existing context. */
nq_status nq_ctx_set_stream(nq_ctx* ctx, void* hip_stream);
void nq_ctx_destroy(nq_ctx* ctx);

/* Host-only: the weight segments a model with this description expects.
 * shapes[2*s] = fan_in, shapes[2*s+1] = fan_out of segment s, for s <
 * min(*n_segments, max_segments). shapes may be NULL to query the count.
 * *n_weights receives the total number of FP64 values. */
nq_status nq_model_weight_layout(const nq_model_desc* desc, int64_t* shapes, int32_t max_segments,
                                 int32_t* n_segments, int64_t* n_weights);

/* Copy a model to the context's device. `weights` is a HOST array of n_weights
 * FP64 values (see nq_model_weight_layout); it is not retained. The model
 * derives its FP32 and BF16 copies (round to nearest even) and its coupling
 * tables itself. */
nq_status nq_model_create(nq_ctx* ctx, const nq_model_desc* desc, const double* weights,
                          int64_t n_weights, nq_model** out);
void nq_model_destroy(nq_model* model);

/* Build the linked-cell neighbour list (Sec. 2.4) of n atoms at positions
 * pos[n*3] (device, FP64) for the list radius r_cut + skin. Rows are sorted by
 * neighbour index. Requires r_cut + skin < min(cell)/2 (minimum image).
 * Returns NQ_ERR_CAPACITY if a row still overflows after the row capacity was
 * grown once. Synchronises the stream once to size the edge workspace. */
nq_status nq_neighbor_build(nq_ctx* ctx, const double* pos, int64_t n, const double cell[3],
                            double r_cut, double skin);

/* Energy and forces (Sec. 2.1, Eq. 1) of the current positions pos[n*3]
 * (device, FP64) with species[n] (device, int32 in [0, n_species)).
 * energy[1] (device, FP64) receives E; forces[n*3] (device, FP64) receives
 * -dE/dr; atom_energy[n] (device, FP64, or NULL) receives E_i = sum_j E_ij.
 * Uses the context's neighbour list; builds it if there is none for this
 * n/cell (list margin min(1.0 A, 0.9 (min(cell)/2 - r_c)): 1.0 A for the
 * 27,648-atom box, 0.315 A for the 64-atom one), and rebuilds it on the device
 * when an atom has moved more than half the margin since the last build.
 * Returns NQ_ERR_ARG if the cutoff does not fit the minimum image.
 * Asynchronous: nothing is synchronised, so conditions the DEVICE detects (a
 * neighbour row longer than the row capacity during an on-device rebuild, more
 * edges than the edge workspace holds, a non-finite coordinate or two atoms
 * closer than 0.1 A, a species outside [0, n_species)) cannot be returned by
 * this call: the outputs of such an evaluation are set to NaN (energy, all
 * forces), and the next nq_stats reports the status (NQ_ERR_CAPACITY,
 * NQ_ERR_NUMERIC, NQ_ERR_ARG). After a capacity error the next evaluation
 * rebuilds the list on the host and grows its capacity. */
nq_status nq_energy_forces(nq_ctx* ctx, const nq_model* model, const double* pos,
                           const int32_t* species, int64_t n, const double cell[3], double* energy,
                           double* forces, double* atom_energy);

/* Energies and forces of n_rep independent replicas (ring-polymer beads of
 * the path-integral application, Sec. 5) of an n-atom system in the same box,
 * in one evaluation: pos[n_rep*n*3] (device, FP64, replica-major), species
 * [n_rep*n] (device, int32), energy[n_rep] (device, FP64: E of each replica),
 * forces[n_rep*n*3] (device, FP64), atom_energy[n_rep*n] (device, FP64, or
 * NULL). Only atoms of the same replica interact; each replica's results are
 * those nq_energy_forces gives for it alone. The neighbour list covers all
 * replicas (rebuilt as in nq_energy_forces). NQ_ERR_ARG for n_rep outside
 * [1, 65536] or n * n_rep outside [2, 2^30). Asynchronous. */
nq_status nq_energy_forces_replicas(nq_ctx* ctx, const nq_model* model, const double* pos,
                                    const int32_t* species, int64_t n, int64_t n_rep,
                                    const double cell[3], double* energy, double* forces,
                                    double* atom_energy);

/* One GPU's share of a spatial decomposition (Sec. 2.4): n_local atoms owned
 * by this domain followed by n_total - n_local ghost atoms (copies of
 * neighbouring domains' atoms within the cutoff). pos[n_total*3] (device,
 * FP64), species[n_total] (device, int32). Only local atoms are centres:
 * energy[1] (device, FP64) = sum of E_i over the local atoms, atom_energy
 * [n_total] (device, FP64, or NULL) is 0 for ghosts, and forces[n_total*3]
 * (device, FP64) holds -dE/dr of this domain's energy for local AND ghost atoms
 * (the ghost rows are what a reverse exchange adds to the owners). The cell
 * must enclose all atoms with at least r_c + skin of empty space around them,
 * so that no periodic image is within reach. Asynchronous. */
nq_status nq_energy_forces_domain(nq_ctx* ctx, const nq_model* model, const double* pos,
                                  const int32_t* species, int64_t n_local, int64_t n_total,
                                  const double cell[3], double* energy, double* forces,
                                  double* atom_energy);

/* Harmonic ring-polymer coupling of the n_rep beads of every atom (the
 * path-integral replicas of Sec. 5; primitive discretisation):
 *   E = 1/2 sum_a m_a w_P^2 sum_k |r_{k+1,a} - r_{k,a}|^2 (bead n_rep = bead 0),
 *   w_P = n_rep k_B T / hbar, bead separations by minimum image.
 * pos[n_rep*n*3] (device, FP64, bead-major), inv_mass[n] (device, FP64,
 * 1/amu, shared by the beads), temperature in K. The spring forces are ADDED
 * to forces[n_rep*n*3] (device, FP64, eV/A); energy[1] (device, FP64)
 * receives E in eV. n_rep = 1 adds nothing. Asynchronous. */
nq_status nq_ring_polymer(nq_ctx* ctx, const double* pos, const double* inv_mass, int64_t n,
                          int64_t n_rep, const double cell[3], double temperature, double* forces,
                          double* energy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as nq_ring_polymer, with the bond energies
 * staged in a fixed device array of NQ_RING_POLYMER_NOALLOC_MAX doubles
 * (8 MiB) that the library holds on every GPU it runs on until the process
 * ends, instead of context memory grown on demand. Allocates nothing: no
 * hipMalloc, hipFree or allocating library call. NQ_ERR_CAPACITY if
 * n * n_rep > NQ_RING_POLYMER_NOALLOC_MAX (nothing is launched), NQ_ERR_ARG as
 * for nq_ring_polymer. Every call on one GPU, from any context, uses the same
 * array: calls that overlap on one GPU (different streams, not ordered by
 * events) race and give wrong energies; calls ordered on one stream do not.
 * Nothing in the array needs to start at zero (each call writes every entry
 * it reads). Asynchronous. */
#define NQ_RING_POLYMER_NOALLOC_MAX ((int64_t)1 << 20)
nq_status nq_ring_polymer_noalloc(nq_ctx* ctx, const double* pos, const double* inv_mass, int64_t n,
                                  int64_t n_rep, const double cell[3], double temperature,
                                  double* forces, double* energy);

/* n_steps velocity-Verlet steps (Eq. 1) of length dt_fs: v += dt/2 F/m;
 * r += dt v (wrapped into the box); F = F(r); v += dt/2 F/m. pos[n*3], vel[n*3]
 * (device, FP64, A and A/fs) are updated in place; inv_mass[n] (device, FP64,
 * 1/amu). forces[n*3] (device, FP64) must hold F(pos) on entry (e.g. from
 * nq_energy_forces) and holds F of the final positions on return. epot/ekin
 * (device, FP64, [n_steps] each, or NULL) receive the potential and kinetic
 * energy after every step. The neighbour list is rebuilt on the device
 * whenever an atom has moved more than half the skin since the last build.
 * One step is captured once as a HIP graph and replayed. */
nq_status nq_step(nq_ctx* ctx, const nq_model* model, double* pos, double* vel,
                  const double* inv_mass, const int32_t* species, int64_t n, const double cell[3],
                  double dt_fs, int32_t n_steps, double* forces, double* epot, double* ekin);

/* n_steps velocity-Verlet steps with one Nose-Hoover thermostat (the NVT
 * thermalisation of the robustness protocol, Sec. 3.2): each step is a
 * thermostat half step, the nq_step velocity-Verlet step, a thermostat half
 * step; a half step of length h = dt/2 with G(K) = (2K - N_f k_B T)/Q,
 * Q = N_f k_B T tau^2, N_f = 3n - 3:
 *   xi += G(K) h/2; v *= exp(-xi h); eta += xi h; xi += G(K) h/2.
 * thermostat[2] (device, FP64, in/out): xi (1/fs) and eta, zero to start.
 * temperature in K, tau_fs > 0. epot/ekin as in nq_step (ekin after the last
 * half step); ethermo[n_steps] (device, FP64, or NULL) receives
 * Q xi^2/2 + N_f k_B T eta, so epot + ekin + ethermo is conserved. Other
 * arguments, graph replay and rebuilds as in nq_step. */
nq_status nq_step_nvt(nq_ctx* ctx, const nq_model* model, double* pos, double* vel,
                      const double* inv_mass, const int32_t* species, int64_t n, const double cell[3],
                      double dt_fs, int32_t n_steps, double temperature, double tau_fs, double* thermostat,
                      double* forces, double* epot, double* ekin, double* ethermo);

/* Outlier count of a force array (the robustness measure of Sec. 3.2, force
 * values beyond 5 sigma): over the 3n components of forces[n*3] (device,
 * FP64), their mean mu and standard deviation sigma; count[1] (device, int32)
 * receives the number of components with |F_k - mu| > nsigma sigma.
 * Asynchronous; nsigma > 0. */
nq_status nq_force_outliers(nq_ctx* ctx, const double* forces, int64_t n, double nsigma, int32_t* count);

/* Number of in-cutoff directed edges of the last nq_energy_forces / nq_step
 * evaluation, and of neighbour-list rebuilds so far. Synchronises the stream.
 * Returns (and clears) the first device-detected error of the evaluations
 * since the last nq_stats, see nq_energy_forces. */
nq_status nq_stats(nq_ctx* ctx, int64_t* n_edges, int64_t* n_rebuilds);

/* Host-only: *captures (host) receives how many times nq_step / nq_step_nvt
 * have captured their HIP graph on this context. A graph is captured again
 * whenever what it bakes in changes: the caller's array pointers, n, dt, the
 * cell, the model, the thermostat, or the context's neighbour-list geometry,
 * row capacity and workspace buffers. For tests of that rule. */
nq_status nq_ctx_graph_captures(const nq_ctx* ctx, int64_t* captures);

/* Copy the directed in-cutoff edges (i, j) of the last evaluation, sorted by
 * (i, j), into ei[cap], ej[cap] (device, int32). *n_edges (host) receives the
 * count; returns NQ_ERR_CAPACITY if it exceeds cap. Synchronises the stream. */
nq_status nq_edges_export(nq_ctx* ctx, int32_t* ei, int32_t* ej, int64_t cap, int64_t* n_edges);

/* Copy a named per-edge or per-atom intermediate of the last evaluation into
 * out[cap] (device, FP32) and report its row count and width (host). Names:
 * "geom" (d, u, Y...), "h0" (two-body input row), "x0", "we1" ([V_0 | w_1]
 * products), "gamma<t>", "s<t>", "x<t>", "V<t>", "eij", "g" (dE/dr_ij), "gu"
 * (dE/du), "gY" (dE/dY parts), "gh0" (dE/dh0 in the first 2 S + n_bessel of
 * its columns). For parity tests of single stages. Synchronises the stream. */
nq_status nq_debug_export(nq_ctx* ctx, const nq_model* model, const char* name, float* out,
                          int64_t cap, int64_t* rows, int64_t* width);

/* Evaluation path of later calls on this context. NQ_PATH_LAYERED: the
 * layered kernels (one launch per stage and product, activations in device
 * memory; the path whose products nq_autotune times and whose intermediates
 * nq_debug_export reads). NQ_PATH_AUTO (default): the same kernels, except
 * that the two-body MLP runs as one kernel per direction (forward: only its
 * last pre-activation is stored; adjoint: the first two layers are
 * recomputed) where that kernel is compiled: two-body widths 64-128-256 on at
 * most 16 inputs padded to 32, latent width 256, precision BF16 or BF16X3 and
 * no per-product override of a two-body product. Its results are bitwise those
 * of NQ_PATH_LAYERED; it is the faster path on the benchmark workload.
 * NQ_PATH_FUSED: one persistent kernel per
 * evaluation that runs the forward pass and its adjoint centre by centre and
 * keeps the edge activations of each 64-edge block on chip; it is compiled
 * for l <= 2, two layers, 32 channels, two-body MLP 64-128-256, one 256-wide
 * latent layer, a 128-wide edge layer, three species, eight Bessel functions
 * and precision BF16 or BF16X3, and the next evaluation returns
 * NQ_ERR_UNSUPPORTED for other models. All paths compute the same function
 * (paper Sec. 2.1, Eq. 1) and agree to rounding. NQ_ERR_ARG for other
 * values. Synchronises the stream and drops the captured MD graph. */
#define NQ_PATH_AUTO 0
#define NQ_PATH_LAYERED 1
#define NQ_PATH_FUSED 2
nq_status nq_ctx_set_path(nq_ctx* ctx, int32_t path);

/* Kernel choice for the matrix-core products of later evaluations on this
 * context: NQ_VARIANT_TUNED (default) uses the model's autotuned choice (or
 * variant 0 before nq_autotune), NQ_VARIANT_LAST and NQ_VARIANT_LAST2 the last
 * and second-to-last variant of every product (the two epilogue forms of the
 * weight-stationary kernel where one is compiled for the product's shape), and
 * v >= 0 variant v modulo each product's count. The energies and forces are
 * bitwise identical for every choice; this exists for tests and measurements.
 * NQ_ERR_ARG for other values. Synchronises the stream and drops the captured
 * MD graph. */
#define NQ_VARIANT_TUNED (-1)
#define NQ_VARIANT_LAST (-2)
#define NQ_VARIANT_LAST2 (-3)
nq_status nq_ctx_set_variant(nq_ctx* ctx, int32_t variant);

/* Upper bound (bytes) of device memory for the per-edge activations of one
 * evaluation (default 160 GiB, further capped at 3/4 of the free memory). When
 * the activations of all edges do not fit, centres are processed in chunks of
 * consecutive atoms, each chunk through the whole forward and adjoint chain;
 * results do not depend on the chunking. Synchronises the stream. */
nq_status nq_ctx_set_workspace_budget(nq_ctx* ctx, int64_t bytes);

/* Autotuner of the matrix-core products: for every per-edge MLP product of
 * one nq_energy_forces evaluation on this system, times each kernel variant
 * (tile shapes of the tiled kernel: rows per workgroup and wave grid; where
 * compiled for the product's shape, the two epilogue forms of the
 * weight-stationary kernel) over `reps` evaluations with HIP events on the
 * context's stream, and keeps the fastest for `model` (later calls use it;
 * an MD graph captured before is captured again). Products run in the
 * precision they have when it is called (nq_model_set_product_precision).
 * Positions/species/cell as in nq_energy_forces. If report is
 * not NULL, a JSON object {"sites": [{"name", "np", "chosen", "ms": [...]}]} is
 * written to report[cap] (host); *len (host, may be NULL) receives its length.
 * Results of the energy/force evaluation do not depend on the choice.
 * Synchronises the stream. */
nq_status nq_autotune(nq_ctx* ctx, nq_model* model, const double* pos, const int32_t* species,
                      int64_t n, const double cell[3], int32_t reps, char* report, int64_t cap,
                      int64_t* len);

/* Sets the kernel variant of one matrix-core product of `model`, as
 * nq_autotune would: `site` is a product name from nq_autotune's report,
 * `variant` >= 0 (taken modulo the product's variant count at launch). Lets a
 * caller replay a recorded tuning in another process; results do not depend on
 * it. Later evaluations use it (an MD graph captured before is captured
 * again). A name that is not a product of the model has no effect. NQ_ERR_ARG
 * for a null or empty name or a negative variant. Not thread-safe against
 * concurrent evaluations. */
nq_status nq_model_set_choice(nq_model* model, const char* site, int32_t variant);

/* Arithmetic of one product of the layered path, overriding the model's
 * precision for it: `site` is a matrix-core product name from nq_autotune's
 * report ("fwd.latent1.0", "bwd.twobody.0", ...) or "tp_fwd<t>" / "tp_bwd<t>"
 * for the channel mixing inside layer t's tensor product (forward / adjoint);
 * `precision` is NQ_PRECISION_FP32, _BF16 or _BF16X3, or -1 to drop the
 * override. Inputs and outputs of every product stay FP32 in memory, so any
 * mixture is valid; the error of the result is what the mixture gives. A name
 * that is not a product of the model has no effect. The fused path does not
 * take overrides: with any set, NQ_PATH_FUSED evaluations return
 * NQ_ERR_UNSUPPORTED. Later evaluations use it (an MD graph captured before is
 * captured again). NQ_ERR_ARG for a null or empty name or another precision. */
nq_status nq_model_set_product_precision(nq_model* model, const char* site, int32_t precision);

/* Per-kernel timing. While enabled, every kernel launch of nq_energy_forces
 * (not of nq_step's graph) is bracketed by HIP events recorded on the
 * context's stream. nq_timing_report synchronises the stream and writes a JSON
 * object {"n_edges": E, "kernels": [{"name", "count", "ms_total",
 * "flop_per_launch", "mfma_flop_per_launch", "bytes_per_launch"}...]}
 * (algorithmic FLOPs, the part of them done on the matrix cores, and HBM bytes
 * of one launch at the last edge count, averaged over the launches: a kernel
 * that runs once per chunk of centres gets its share of the edges) into
 * buf[cap] (host), then clears the record. The record should cover whole
 * evaluations of one system. *len (host) receives the length; NQ_ERR_CAPACITY if buf is too
 * small. */
nq_status nq_timing(nq_ctx* ctx, int enable);
nq_status nq_timing_report(nq_ctx* ctx, char* buf, int64_t cap, int64_t* len);

const char* nq_status_str(nq_status status);
const char* nq_last_error(const nq_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* NNQMD_H */
