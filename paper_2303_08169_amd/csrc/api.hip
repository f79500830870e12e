// C ABI of the library (declared in include/nnqmd.h). Every entry point turns
// internal errors into an nq_status and records the message on the context.
#include <cmath>
#include <cstring>
#include <exception>

#include "nq_internal.hpp"

namespace nq {
void md_record_async(hipStream_t s, const double* epot_now, const double* ekin_now, int* counter, double* epot,
                     double* ekin, int n_steps);
void md_set_int_async(hipStream_t s, int* p, int v);
}  // namespace nq

namespace nq {

static hipEvent_t pool_event(nq_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  NQ_HIP(hipEventCreate(&e));
  return e;
}

int span_begin(nq_ctx* ctx, const std::string& name, double fpe, double bpe, double fpa, double bpa,
               double mfpe) {
  if (!ctx->timing) return -1;
  Span s;
  s.name = name;
  s.a = pool_event(ctx);
  s.b = pool_event(ctx);
  s.flop_per_edge = fpe;
  s.byte_per_edge = bpe;
  s.flop_per_atom = fpa;
  s.byte_per_atom = bpa;
  s.mfma_flop_per_edge = mfpe;
  NQ_HIP(hipEventRecord(s.a, ctx->stream));
  ctx->spans.push_back(s);
  return (int)ctx->spans.size() - 1;
}

void span_end(nq_ctx* ctx, int idx) {
  if (idx < 0 || !ctx->timing) return;
  NQ_HIP(hipEventRecord(ctx->spans[idx].b, ctx->stream));
}

}  // namespace nq

using namespace nq;

namespace {

thread_local std::string g_error;

template <class F>
nq_status guarded(nq_ctx* ctx, F&& f) {
  try {
    f();
    return NQ_OK;
  } catch (const Error& e) {
    (ctx ? ctx->last_error : g_error) = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    (ctx ? ctx->last_error : g_error) = "host allocation failed";
    return NQ_ERR_OOM;
  } catch (const std::exception& e) {
    (ctx ? ctx->last_error : g_error) = e.what();
    return NQ_ERR_DEVICE;
  }
}

void read_flags(nq_ctx* ctx, int* host) {
  NQ_HIP(hipMemcpyAsync(host, ctx->nl.flags.p, 8 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  NQ_HIP(hipStreamSynchronize(ctx->stream));
}

void zero_flags(nq_ctx* ctx) { NQ_HIP(hipMemsetAsync(ctx->nl.flags.p, 0, 8 * sizeof(int), ctx->stream)); }

void check_flags(nq_ctx* ctx) {
  int f[8];
  read_flags(ctx, f);
  if (f[2]) {
    zero_flags(ctx);
    throw Error{NQ_ERR_NUMERIC, "non-finite coordinate or two atoms closer than 0.1 A"};
  }
  if (f[0] > 0) {
    zero_flags(ctx);
    ctx->nl.built = false;  // the list is truncated: the next evaluation rebuilds (and grows) it
    throw Error{NQ_ERR_CAPACITY, "a neighbour-list row overflowed (" + std::to_string(f[0]) + " > " +
                                     std::to_string(ctx->nl.k_max) + ")"};
  }
  if (f[5]) {
    zero_flags(ctx);
    throw Error{NQ_ERR_ARG, "species outside [0, n_species)"};
  }
  if (f[4] > 0) {
    zero_flags(ctx);
    ctx->nl.built = false;  // the edge workspace is resized from a fresh host-visible build
    throw Error{NQ_ERR_CAPACITY, "edge workspace overflowed (" + std::to_string(f[4]) + " edges)"};
  }
}

void neighbor_build_sync(nq_ctx* ctx, const double* pos, int64_t n, const double cell[3], double r_cut,
                         double skin, int64_t n_rep = 1) {
  NQ_HIP(hipSetDevice(ctx->device));
  nbr_configure(ctx, n, cell, r_cut, skin, n_rep);
  NbrList& nl = ctx->nl;
  for (int attempt = 0;; ++attempt) {
    zero_flags(ctx);
    nbr_build_async(ctx, pos, false);
    int f[8];
    read_flags(ctx, f);
    if (f[2]) {
      zero_flags(ctx);
      throw Error{NQ_ERR_NUMERIC, "non-finite coordinate"};
    }
    if (f[0] == 0) break;
    NQ_REQUIRE(attempt == 0, NQ_ERR_CAPACITY,
               "neighbour-list row overflow after growing the row capacity to " + std::to_string(nl.k_max));
    nl.k_max = (int)std::max<int64_t>(rup((int64_t)(1.5 * nl.k_max), 32), rup(f[0] + 16, 32));
    NQ_REQUIRE(nl.k_max <= 2048, NQ_ERR_CAPACITY, "neighbour rows longer than 2048");
    nl.nbr.release();
    nl.nbr.ensure((size_t)n * nl.k_max * 4);
    ++ctx->gen;
  }
  std::vector<int> cnt(n);
  NQ_HIP(hipMemcpy(cnt.data(), nl.nbr_cnt.p, n * sizeof(int), hipMemcpyDeviceToHost));
  nl.entry_prefix.assign(n + 1, 0);
  for (int64_t a = 0; a < n; ++a) nl.entry_prefix[a + 1] = nl.entry_prefix[a] + cnt[a];
  nl.n_entries = nl.entry_prefix[n];
  nl.built = true;
  zero_flags(ctx);
}

double default_skin(const double cell[3], double rc) {
  const double lmin = std::min(cell[0], std::min(cell[1], cell[2]));
  const double room = 0.5 * lmin - rc;
  NQ_REQUIRE(room > 0, NQ_ERR_ARG, "the cutoff must be below half of every box length (minimum image)");
  return std::min(1.0, 0.9 * room);
}

// True when evaluations of this model on this context take the fused kernel.
// The layered kernels are the default: on the benchmark workload they are
// measured faster than the fused kernel, whose per-block weight traffic from
// L2 (the whole weight set once per 64 edges) bounds it.
bool use_fused(const nq_ctx* ctx, const nq_model* m) {
  if (ctx->path != NQ_PATH_FUSED) return false;
  NQ_REQUIRE(fused_supported(m), NQ_ERR_UNSUPPORTED,
             "the fused kernel is not compiled for this model shape or precision");
  return true;
}

// Make sure a neighbour list valid for this model exists and the workspace fits it.
// n counts the atoms of all n_rep replicas.
void ensure_list(nq_ctx* ctx, const nq_model* m, const double* pos, int64_t n, const double cell[3],
                 int64_t n_rep = 1) {
  NbrList& nl = ctx->nl;
  const double rc = m->dims.rc;
  const bool ok = nl.built && nl.n == n && nl.n_rep == n_rep && nl.box[0] == cell[0] && nl.box[1] == cell[1] &&
                  nl.box[2] == cell[2] && nl.r_cut + nl.skin >= rc;
  if (!ok) neighbor_build_sync(ctx, pos, n, cell, rc, default_skin(cell, rc), n_rep);
  const int64_t cap = rup((int64_t)(1.25 * (double)nl.n_entries) + 1024, 128);
  const bool fused = use_fused(ctx, m);
  ws_ensure(ctx, m, cap, n, !fused);
  if (fused) fused_prepare(ctx);
}

void check_common(nq_ctx* ctx, const nq_model* m, const double* pos, const int32_t* species, int64_t n,
                  const double* cell) {
  NQ_REQUIRE(ctx && m && pos && species && cell, NQ_ERR_ARG, "null argument");
  NQ_REQUIRE(m->ctx == ctx, NQ_ERR_ARG, "model belongs to another context");
  NQ_REQUIRE(n >= 2 && n < ((int64_t)1 << 30), NQ_ERR_ARG, "n out of range");
  for (int k = 0; k < 3; ++k) NQ_REQUIRE(std::isfinite(cell[k]) && cell[k] > 0, NQ_ERR_ARG, "bad cell");
}

// n_centres: atoms whose edges are evaluated (the others are ghosts), -1 = all.
void evaluate_async(nq_ctx* ctx, const nq_model* m, const double* pos, const int32_t* species, int64_t n,
                    double* energy, double* forces, double* atom_energy, int64_t n_rep = 1,
                    int64_t n_centres = -1) {
  NbrList& nl = ctx->nl;
  const double half = 0.5 * (nl.r_cut + nl.skin - m->dims.rc);
  int sp = span_begin(ctx, "neighbor_check_rebuild");
  nbr_displacement_check_async(ctx, pos, half);
  nbr_build_async(ctx, pos, true);
  span_end(ctx, sp);
  sp = span_begin(ctx, "edge_list");
  edges_build_async(ctx, pos, m->dims.rc, n_centres);
  span_end(ctx, sp);
  if (use_fused(ctx, m)) {
    fused_async(ctx, m, species, atom_energy, n_centres);
  } else {
    for (int c = 0; c + 1 < (int)ctx->ws.chunks.size(); ++c) {
      chunk_view_async(ctx, c);
      forward_async(ctx, m, species, atom_energy);
      backward_async(ctx, m);
    }
  }
  finish_async(ctx, m, energy, forces, n_rep, n_centres);
}

}  // namespace

extern "C" {

nq_status nq_ctx_create(int device, void* hip_stream, nq_ctx** out) {
  return guarded(nullptr, [&] {
    NQ_REQUIRE(out, NQ_ERR_ARG, "null out");
    int count = 0;
    NQ_HIP(hipGetDeviceCount(&count));
    NQ_REQUIRE(device >= 0 && device < count, NQ_ERR_ARG, "no such device");
    NQ_HIP(hipSetDevice(device));
    nq_ctx* c = new nq_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    NQ_HIP(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device));
    c->rp_static = ring_polymer_static_scratch(device);
    *out = c;
  });
}

nq_status nq_ctx_set_stream(nq_ctx* ctx, void* hip_stream) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx, NQ_ERR_ARG, "null ctx");
    ctx->stream = (hipStream_t)hip_stream;
  });
}

void nq_ctx_destroy(nq_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->md_stream) (void)hipStreamDestroy(ctx->md_stream);
  if (ctx->ev[0]) (void)hipEventDestroy(ctx->ev[0]);
  if (ctx->ev[1]) (void)hipEventDestroy(ctx->ev[1]);
  delete ctx;
}

nq_status nq_model_weight_layout(const nq_model_desc* desc, int64_t* shapes, int32_t max_segments,
                                 int32_t* n_segments, int64_t* n_weights) {
  return guarded(nullptr, [&] {
    NQ_REQUIRE(desc && n_segments && n_weights, NQ_ERR_ARG, "null argument");
    std::vector<std::pair<int64_t, int64_t>> segs;
    weight_layout(*desc, segs);
    *n_segments = (int32_t)segs.size();
    int64_t tot = 0;
    for (size_t s = 0; s < segs.size(); ++s) {
      if (shapes && (int32_t)s < max_segments) {
        shapes[2 * s] = segs[s].first;
        shapes[2 * s + 1] = segs[s].second;
      }
      tot += segs[s].first * segs[s].second;
    }
    *n_weights = tot;
  });
}

nq_status nq_model_create(nq_ctx* ctx, const nq_model_desc* desc, const double* weights, int64_t n_weights,
                          nq_model** out) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && desc && weights && out, NQ_ERR_ARG, "null argument");
    *out = model_create(ctx, desc, weights, n_weights);
  });
}

void nq_model_destroy(nq_model* model) {
  if (!model) return;
  nq_ctx* ctx = model->ctx;
  if (ctx) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws.model == model) {
      ctx->ws.model = nullptr;
      ctx->ws.cap = 0;
      ctx->ws.cap_all = 0;
      ctx->ws.chunks.clear();
      ctx->ws.bufs.clear();
    }
    if (ctx->graph_exec) {
      (void)hipGraphExecDestroy(ctx->graph_exec);
      ctx->graph_exec = nullptr;
      ctx->graph_key.clear();
    }
  }
  delete model;
}

nq_status nq_neighbor_build(nq_ctx* ctx, const double* pos, int64_t n, const double cell[3], double r_cut,
                            double skin) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && pos && cell, NQ_ERR_ARG, "null argument");
    NQ_REQUIRE(std::isfinite(r_cut) && std::isfinite(skin), NQ_ERR_ARG, "bad r_cut or skin");
    neighbor_build_sync(ctx, pos, n, cell, r_cut, skin);
  });
}

nq_status nq_energy_forces(nq_ctx* ctx, const nq_model* model, const double* pos, const int32_t* species,
                           int64_t n, const double cell[3], double* energy, double* forces, double* atom_energy) {
  return guarded(ctx, [&] {
    check_common(ctx, model, pos, species, n, cell);
    NQ_REQUIRE(energy && forces, NQ_ERR_ARG, "null output");
    NQ_HIP(hipSetDevice(ctx->device));
    ensure_list(ctx, model, pos, n, cell);
    evaluate_async(ctx, model, pos, species, n, energy, forces, atom_energy);
  });
}

nq_status nq_energy_forces_replicas(nq_ctx* ctx, const nq_model* model, const double* pos,
                                    const int32_t* species, int64_t n, int64_t n_rep, const double cell[3],
                                    double* energy, double* forces, double* atom_energy) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(n_rep >= 1 && n_rep <= 65536, NQ_ERR_ARG, "n_rep out of range");
    NQ_REQUIRE(n >= 2 && n < ((int64_t)1 << 30) && n * n_rep < ((int64_t)1 << 30), NQ_ERR_ARG,
               "n out of range");
    check_common(ctx, model, pos, species, n * n_rep, cell);
    NQ_REQUIRE(energy && forces, NQ_ERR_ARG, "null output");
    NQ_HIP(hipSetDevice(ctx->device));
    ensure_list(ctx, model, pos, n * n_rep, cell, n_rep);
    evaluate_async(ctx, model, pos, species, n * n_rep, energy, forces, atom_energy, n_rep);
  });
}

nq_status nq_energy_forces_domain(nq_ctx* ctx, const nq_model* model, const double* pos,
                                  const int32_t* species, int64_t n_local, int64_t n_total, const double cell[3],
                                  double* energy, double* forces, double* atom_energy) {
  return guarded(ctx, [&] {
    check_common(ctx, model, pos, species, n_total, cell);
    NQ_REQUIRE(n_local >= 1 && n_local <= n_total, NQ_ERR_ARG, "need 1 <= n_local <= n_total");
    NQ_REQUIRE(energy && forces, NQ_ERR_ARG, "null output");
    NQ_HIP(hipSetDevice(ctx->device));
    ensure_list(ctx, model, pos, n_total, cell);
    evaluate_async(ctx, model, pos, species, n_total, energy, forces, atom_energy, 1, n_local);
  });
}

nq_status nq_force_outliers(nq_ctx* ctx, const double* forces, int64_t n, double nsigma, int32_t* count) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && forces && count, NQ_ERR_ARG, "null argument");
    NQ_REQUIRE(n >= 1 && n < ((int64_t)1 << 30), NQ_ERR_ARG, "n out of range");
    NQ_REQUIRE(std::isfinite(nsigma) && nsigma > 0, NQ_ERR_ARG, "bad nsigma");
    NQ_HIP(hipSetDevice(ctx->device));
    force_outliers_async(ctx->stream, forces, n, nsigma, count);
    NQ_HIP(hipGetLastError());
  });
}

namespace {

// Argument checks shared by both ring-polymer entry points; returns w_P (1/fs).
double ring_polymer_check(nq_ctx* ctx, const double* pos, const double* inv_mass, int64_t n, int64_t n_rep,
                          const double cell[3], double temperature, double* forces, double* energy) {
  NQ_REQUIRE(ctx && pos && inv_mass && cell && forces && energy, NQ_ERR_ARG, "null argument");
  NQ_REQUIRE(n >= 1 && n_rep >= 1 && n * n_rep < ((int64_t)1 << 30), NQ_ERR_ARG, "n or n_rep out of range");
  NQ_REQUIRE(std::isfinite(temperature) && temperature >= 0, NQ_ERR_ARG, "bad temperature");
  for (int k = 0; k < 3; ++k) NQ_REQUIRE(std::isfinite(cell[k]) && cell[k] > 0, NQ_ERR_ARG, "bad cell");
  // w_P = P k_B T / hbar (1/fs): k_B in eV/K, hbar in eV fs (CODATA 2018)
  return (double)n_rep * 8.617333262e-5 * temperature / 0.6582119569;
}

}  // namespace

nq_status nq_ring_polymer(nq_ctx* ctx, const double* pos, const double* inv_mass, int64_t n, int64_t n_rep,
                          const double cell[3], double temperature, double* forces, double* energy) {
  return guarded(ctx, [&] {
    const double omega_p = ring_polymer_check(ctx, pos, inv_mass, n, n_rep, cell, temperature, forces, energy);
    NQ_HIP(hipSetDevice(ctx->device));
    ctx->rp_scratch.ensure((size_t)(n * n_rep) * sizeof(double));
    ring_polymer_async(ctx->stream, pos, inv_mass, n, n_rep, omega_p, cell, forces, ctx->rp_scratch.as<double>(),
                       energy);
    NQ_HIP(hipGetLastError());
  });
}

nq_status nq_ring_polymer_noalloc(nq_ctx* ctx, const double* pos, const double* inv_mass, int64_t n,
                                  int64_t n_rep, const double cell[3], double temperature, double* forces,
                                  double* energy) {
  return guarded(ctx, [&] {
    const double omega_p = ring_polymer_check(ctx, pos, inv_mass, n, n_rep, cell, temperature, forces, energy);
    NQ_REQUIRE(n * n_rep <= NQ_RING_POLYMER_NOALLOC_MAX, NQ_ERR_CAPACITY,
               "n * n_rep exceeds the fixed ring-polymer array (NQ_RING_POLYMER_NOALLOC_MAX)");
    NQ_REQUIRE(ctx->rp_static, NQ_ERR_DEVICE, "ring-polymer array not set up");
    NQ_HIP(hipSetDevice(ctx->device));
    ring_polymer_async(ctx->stream, pos, inv_mass, n, n_rep, omega_p, cell, forces, ctx->rp_static, energy);
    NQ_HIP(hipGetLastError());
  });
}

namespace {

// Thermostat of an NVT run (null for NVE).
struct NhParams {
  double temperature, tau, nfkT, Q;
  double* state;    // device [2]: xi (1/fs), eta
  double* ethermo;  // device [n_steps] or null
};

// n_steps MD steps replayed from one captured HIP graph; see nq_step / nq_step_nvt.
void md_run(nq_ctx* ctx, const nq_model* model, double* pos, double* vel, const double* inv_mass,
            const int32_t* species, int64_t n, const double cell[3], double dt_fs, int32_t n_steps,
            double* forces, double* epot, double* ekin, const NhParams* nh) {
  check_common(ctx, model, pos, species, n, cell);
  NQ_REQUIRE(vel && inv_mass && forces, NQ_ERR_ARG, "null argument");
  NQ_REQUIRE(n_steps >= 0 && std::isfinite(dt_fs) && dt_fs > 0, NQ_ERR_ARG, "bad dt or n_steps");
  if (n_steps == 0) return;
  NQ_HIP(hipSetDevice(ctx->device));
  ensure_list(ctx, model, pos, n, cell);
  if (!ctx->md_stream) {
    NQ_HIP(hipStreamCreateWithFlags(&ctx->md_stream, hipStreamNonBlocking));
    NQ_HIP(hipEventCreateWithFlags(&ctx->ev[0], hipEventDisableTiming));
    NQ_HIP(hipEventCreateWithFlags(&ctx->ev[1], hipEventDisableTiming));
  }
  ctx->md_scratch.ensure(128);
  double* ek_now = ctx->md_scratch.as<double>();
  int* counter = reinterpret_cast<int*>(ctx->md_scratch.as<double>() + 2);
  double* nh_K = ctx->md_scratch.as<double>() + 4;      // kinetic energy tracked by the thermostat
  double* nh_scale = ctx->md_scratch.as<double>() + 5;  // velocity scale of the last half step
  std::vector<const void*> key = {model,  pos,  vel,  inv_mass, species, forces,
                                  epot,   ekin, (const void*)(intptr_t)n,
                                  (const void*)(intptr_t)ctx->ws.cap, (const void*)(intptr_t)n_steps,
                                  (const void*)(intptr_t)ctx->ws.chunks.size(),
                                  ctx->ws.bufs.empty() ? nullptr : ctx->ws.bufs.front()->p,
                                  ctx->md_scratch.p, (const void*)(intptr_t)ctx->gen,
                                  (const void*)(intptr_t)model->version};
  auto push_double = [&](double v) {
    int64_t b;
    std::memcpy(&b, &v, sizeof(double));
    key.push_back((const void*)(intptr_t)b);
  };
  push_double(dt_fs);
  for (int k = 0; k < 3; ++k) push_double(cell[k]);
  key.push_back(nh ? nh->state : nullptr);
  key.push_back(nh ? nh->ethermo : nullptr);
  push_double(nh ? nh->nfkT : 0.0);
  push_double(nh ? nh->Q : 0.0);
  hipStream_t user = ctx->stream;
  if (!ctx->graph_exec || key != ctx->graph_key) {
    if (ctx->graph_exec) {
      (void)hipGraphExecDestroy(ctx->graph_exec);
      ctx->graph_exec = nullptr;
    }
    ctx->stream = ctx->md_stream;
    hipGraph_t graph = nullptr;
    try {
      NQ_HIP(hipStreamBeginCapture(ctx->md_stream, hipStreamCaptureModeThreadLocal));
      const double h = 0.5 * dt_fs;
      if (nh) md_nh_half_async(ctx->md_stream, vel, n, nh->state, nh->state + 1, nh_K, nh_scale, nh->nfkT, nh->Q, h);
      md_half_kick_async(ctx->md_stream, vel, forces, inv_mass, n, 0.5 * dt_fs);
      md_drift_async(ctx->md_stream, pos, vel, n, dt_fs, cell);
      evaluate_async(ctx, model, pos, species, n, ctx->ws.esum, forces, nullptr);
      md_half_kick_async(ctx->md_stream, vel, forces, inv_mass, n, 0.5 * dt_fs);
      if (nh) {
        md_ekin_async(ctx->md_stream, vel, inv_mass, n, nh_K);
        md_nh_half_async(ctx->md_stream, vel, n, nh->state, nh->state + 1, nh_K, nh_scale, nh->nfkT, nh->Q, h);
        md_nh_record_async(ctx->md_stream, nh->state, nh->state + 1, counter, nh->ethermo, n_steps, nh->nfkT,
                           nh->Q);
        md_record_async(ctx->md_stream, ctx->ws.esum, nh_K, counter, epot, ekin, n_steps);
      } else {
        md_ekin_async(ctx->md_stream, vel, inv_mass, n, ek_now);
        md_record_async(ctx->md_stream, ctx->ws.esum, ek_now, counter, epot, ekin, n_steps);
      }
      NQ_HIP(hipStreamEndCapture(ctx->md_stream, &graph));
      NQ_HIP(hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(graph);
    } catch (...) {
      hipGraph_t dummy = nullptr;
      (void)hipStreamEndCapture(ctx->md_stream, &dummy);
      if (dummy) (void)hipGraphDestroy(dummy);
      if (graph) (void)hipGraphDestroy(graph);
      ctx->stream = user;
      throw;
    }
    ctx->stream = user;
    ctx->graph_key = key;
    ++ctx->graph_captures;
  }
  NQ_HIP(hipEventRecord(ctx->ev[0], user));
  NQ_HIP(hipStreamWaitEvent(ctx->md_stream, ctx->ev[0], 0));
  md_set_int_async(ctx->md_stream, counter, 0);
  if (nh) md_ekin_async(ctx->md_stream, vel, inv_mass, n, nh_K);  // K of the starting velocities
  for (int s = 0; s < n_steps; ++s) NQ_HIP(hipGraphLaunch(ctx->graph_exec, ctx->md_stream));
  NQ_HIP(hipEventRecord(ctx->ev[1], ctx->md_stream));
  NQ_HIP(hipStreamWaitEvent(user, ctx->ev[1], 0));
  NQ_HIP(hipStreamSynchronize(ctx->md_stream));
  check_flags(ctx);
}

}  // namespace

nq_status nq_step(nq_ctx* ctx, const nq_model* model, double* pos, double* vel, const double* inv_mass,
                  const int32_t* species, int64_t n, const double cell[3], double dt_fs, int32_t n_steps,
                  double* forces, double* epot, double* ekin) {
  return guarded(ctx, [&] {
    md_run(ctx, model, pos, vel, inv_mass, species, n, cell, dt_fs, n_steps, forces, epot, ekin, nullptr);
  });
}

nq_status nq_step_nvt(nq_ctx* ctx, const nq_model* model, double* pos, double* vel, const double* inv_mass,
                      const int32_t* species, int64_t n, const double cell[3], double dt_fs, int32_t n_steps,
                      double temperature, double tau_fs, double* thermostat, double* forces, double* epot,
                      double* ekin, double* ethermo) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(thermostat, NQ_ERR_ARG, "null thermostat state");
    NQ_REQUIRE(std::isfinite(temperature) && temperature > 0 && std::isfinite(tau_fs) && tau_fs > 0, NQ_ERR_ARG,
               "bad temperature or tau");
    NhParams nh;
    nh.temperature = temperature;
    nh.tau = tau_fs;
    nh.nfkT = (double)(3 * n - 3) * 8.617333262e-5 * temperature;  // k_B in eV/K
    nh.Q = nh.nfkT * tau_fs * tau_fs;
    nh.state = thermostat;
    nh.ethermo = ethermo;
    md_run(ctx, model, pos, vel, inv_mass, species, n, cell, dt_fs, n_steps, forces, epot, ekin, &nh);
  });
}

nq_status nq_ctx_graph_captures(const nq_ctx* ctx, int64_t* captures) {
  return guarded(nullptr, [&] {
    NQ_REQUIRE(ctx && captures, NQ_ERR_ARG, "null argument");
    *captures = ctx->graph_captures;
  });
}

nq_status nq_stats(nq_ctx* ctx, int64_t* n_edges, int64_t* n_rebuilds) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx, NQ_ERR_ARG, "null ctx");
    int ne = 0;
    if (ctx->ws.nedge.p) {
      NQ_HIP(hipMemcpyAsync(&ne, ctx->ws.nedge.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    }
    int f[8] = {0};
    if (ctx->nl.flags.p) read_flags(ctx, f);
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    if (n_edges) *n_edges = ne;
    if (n_rebuilds) *n_rebuilds = f[3];
    if (ctx->nl.flags.p) check_flags(ctx);
  });
}

nq_status nq_edges_export(nq_ctx* ctx, int32_t* ei, int32_t* ej, int64_t cap, int64_t* n_edges) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && ei && ej && n_edges, NQ_ERR_ARG, "null argument");
    NQ_REQUIRE(ctx->ws.nedge.p, NQ_ERR_ARG, "no evaluation yet");
    int ne = 0;
    NQ_HIP(hipMemcpyAsync(&ne, ctx->ws.nedge.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    *n_edges = ne;
    NQ_REQUIRE(ne <= cap, NQ_ERR_CAPACITY, "output too small");
    NQ_HIP(hipMemcpyAsync(ei, ctx->ws.ei.p, (size_t)ne * 4, hipMemcpyDeviceToDevice, ctx->stream));
    NQ_HIP(hipMemcpyAsync(ej, ctx->ws.ej.p, (size_t)ne * 4, hipMemcpyDeviceToDevice, ctx->stream));
    NQ_HIP(hipStreamSynchronize(ctx->stream));
  });
}

nq_status nq_debug_export(nq_ctx* ctx, const nq_model* model, const char* name, float* out, int64_t cap,
                          int64_t* rows, int64_t* width) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && model && name && out && rows && width, NQ_ERR_ARG, "null argument");
    const Workspace& ws = ctx->ws;
    NQ_REQUIRE(ws.model == model && ws.nedge.p, NQ_ERR_ARG, "no evaluation of this model yet");
    NQ_REQUIRE(ws.has_act || std::string(name) == "g", NQ_ERR_ARG,
               "stage intermediates exist only on the layered path (nq_ctx_set_path)");
    const Dims& d = model->dims;
    int ne = 0, ne_all = 0;
    NQ_HIP(hipMemcpyAsync(&ne, ws.v_nedge ? ws.v_nedge : ws.nedge.as<int>(), sizeof(int), hipMemcpyDeviceToHost,
                          ctx->stream));
    NQ_HIP(hipMemcpyAsync(&ne_all, ws.nedge.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    const std::string s(name);
    const float* src = nullptr;
    int64_t r = ne, w = 0;
    auto layer = [&](const char* pre) -> int {
      const size_t k = std::strlen(pre);
      if (s.compare(0, k, pre) != 0 || s.size() == k) return -1;
      return std::atoi(s.c_str() + k);
    };
    int t;
    if (s == "geom") { src = ws.geo; w = 16; }
    else if (s == "h0") { src = ws.h0; w = ws.K0p; }
    else if (s == "we1") { src = ws.we1; w = 2 * d.NW; }
    else if (s == "eij") { src = ws.eij; w = 1; }
    else if (s == "g") { src = reinterpret_cast<const float*>(ws.gr); w = 4; r = ne_all; }
    else if (s == "gu") { src = ws.gu; w = 1; }
    else if (s == "gY") { src = ws.gY; w = 16 * (d.T + 1); }
    else if (s == "gh0") { src = ws.gh[0]; w = ws.maxw; }
    else if ((t = layer("gamma")) >= 1 && t <= d.T) { src = ws.gam[t]; w = d.NY * d.C; r = ws.v_n; }
    else if ((t = layer("s")) >= 1 && t <= d.T) { src = ws.s[t]; w = d.nscal * d.C; }
    else if ((t = layer("V")) >= 1 && t < d.T) { src = ws.V[t]; w = d.NY * d.C; }
    else if ((t = layer("x")) >= 0 && t <= d.T) { src = ws.x[t]; w = d.D; }
    const bool x0 = s == "x0";  // formed from the two-body pre-activation, not stored
    NQ_REQUIRE(src || x0, NQ_ERR_ARG, "unknown buffer name " + s);
    if (x0) w = d.D;
    *rows = r;
    *width = w;
    NQ_REQUIRE(r * w <= cap, NQ_ERR_CAPACITY, "output too small");
    if (x0)
      debug_x0_async(ctx, model, out);
    else
      NQ_HIP(hipMemcpyAsync(out, src, (size_t)r * w * 4, hipMemcpyDeviceToDevice, ctx->stream));
    NQ_HIP(hipStreamSynchronize(ctx->stream));
  });
}

nq_status nq_model_set_choice(nq_model* model, const char* site, int32_t variant) {
  return guarded(nullptr, [&] {
    NQ_REQUIRE(model && site && site[0] && variant >= 0, NQ_ERR_ARG, "bad product name or variant");
    model->gemm_choice[site] = variant;
    ++model->version;
  });
}

nq_status nq_model_set_product_precision(nq_model* model, const char* site, int32_t precision) {
  return guarded(nullptr, [&] {
    NQ_REQUIRE(model && site && site[0], NQ_ERR_ARG, "null or empty product name");
    NQ_REQUIRE(precision == -1 || precision == NQ_PRECISION_FP32 || precision == NQ_PRECISION_BF16 ||
                   precision == NQ_PRECISION_BF16X3,
               NQ_ERR_ARG, "bad precision");
    if (precision < 0)
      model->site_prec.erase(site);
    else
      model->site_prec[site] = precision;
    ++model->version;
  });
}

nq_status nq_ctx_set_variant(nq_ctx* ctx, int32_t variant) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && variant >= NQ_VARIANT_LAST2, NQ_ERR_ARG, "bad kernel variant");
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    ctx->user_variant = variant;
    if (ctx->graph_exec) {
      (void)hipGraphExecDestroy(ctx->graph_exec);
      ctx->graph_exec = nullptr;
      ctx->graph_key.clear();
    }
  });
}

nq_status nq_ctx_set_path(nq_ctx* ctx, int32_t path) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && (path == NQ_PATH_AUTO || path == NQ_PATH_LAYERED || path == NQ_PATH_FUSED), NQ_ERR_ARG,
               "bad path");
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    ctx->path = path;
    if (ctx->graph_exec) {
      (void)hipGraphExecDestroy(ctx->graph_exec);
      ctx->graph_exec = nullptr;
      ctx->graph_key.clear();
    }
  });
}

nq_status nq_ctx_set_workspace_budget(nq_ctx* ctx, int64_t bytes) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && bytes > 0, NQ_ERR_ARG, "bad budget");
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    ctx->ws_budget = bytes;
    ctx->ws.chunks.clear();  // re-plan at the next call
    ctx->ws.model = nullptr;
    if (ctx->graph_exec) {
      (void)hipGraphExecDestroy(ctx->graph_exec);
      ctx->graph_exec = nullptr;
      ctx->graph_key.clear();
    }
  });
}

nq_status nq_autotune(nq_ctx* ctx, nq_model* model, const double* pos, const int32_t* species, int64_t n,
                      const double cell[3], int32_t reps, char* report, int64_t cap, int64_t* len) {
  return guarded(ctx, [&] {
    check_common(ctx, model, pos, species, n, cell);
    NQ_REQUIRE(reps >= 1 && reps <= 100, NQ_ERR_ARG, "reps must be 1..100");
    NQ_HIP(hipSetDevice(ctx->device));
    // the tuned products are the layered kernels'
    const int was_path = ctx->path;
    ctx->path = NQ_PATH_LAYERED;
    struct Restore {
      nq_ctx* c;
      int p;
      ~Restore() { c->path = p; }
    } restore{ctx, was_path};
    ensure_list(ctx, model, pos, n, cell);
    DevBuf scratch;
    scratch.ensure((size_t)(n * 3 + 8) * sizeof(double));
    double* F = scratch.as<double>();
    double* E = F + n * 3;
    const bool was_timing = ctx->timing;
    std::map<std::string, std::vector<double>> ms;  // site -> mean ms per variant
    int nvar = 1;
    try {
      // one evaluation records the products and their kernel variants
      ctx->timing = false;
      evaluate_async(ctx, model, pos, species, n, E, F, nullptr);
      for (const auto& kv : ctx->site_nvar) nvar = std::max(nvar, kv.second);
      for (int v = 0; v < nvar; ++v) {
        ctx->force_variant = v;
        ctx->timing = false;
        evaluate_async(ctx, model, pos, species, n, E, F, nullptr);  // warm-up
        ctx->timing = true;
        ctx->spans.clear();
        for (int r = 0; r < reps; ++r) evaluate_async(ctx, model, pos, species, n, E, F, nullptr);
        NQ_HIP(hipStreamSynchronize(ctx->stream));
        std::map<std::string, double> tot;
        for (const Span& sp : ctx->spans) {
          float t = 0.f;
          NQ_HIP(hipEventElapsedTime(&t, sp.a, sp.b));
          tot[sp.name] += t;
          ctx->event_pool.push_back(sp.a);
          ctx->event_pool.push_back(sp.b);
        }
        ctx->spans.clear();
        for (const auto& kv : ctx->site_np) ms[kv.first].push_back(tot[kv.first] / reps);
      }
    } catch (...) {
      ctx->force_variant = -1;
      ctx->timing = was_timing;
      throw;
    }
    ctx->force_variant = -1;
    ctx->timing = was_timing;
    std::string out = "{\"sites\": [";
    bool first = true;
    for (const auto& kv : ms) {
      const int np = ctx->site_np[kv.first];
      const int nv = ctx->site_nvar[kv.first];
      int best = 0;
      for (int v = 1; v < nv && v < (int)kv.second.size(); ++v)
        if (kv.second[v] < kv.second[best]) best = v;
      model->gemm_choice[kv.first] = best;
      ++model->version;
      out += std::string(first ? "" : ", ") + "{\"name\": \"" + kv.first + "\", \"np\": " + std::to_string(np) +
             ", \"chosen\": " + std::to_string(best) + ", \"ms\": [";
      for (int v = 0; v < nv && v < (int)kv.second.size(); ++v)
        out += (v ? ", " : "") + std::to_string(kv.second[v]);
      out += "]}";
      first = false;
    }
    out += "]}";
    if (len) *len = (int64_t)out.size();
    if (report) {
      NQ_REQUIRE(cap > (int64_t)out.size(), NQ_ERR_CAPACITY, "report buffer too small");
      std::memcpy(report, out.c_str(), out.size() + 1);
    }
  });
}

nq_status nq_timing(nq_ctx* ctx, int enable) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx, NQ_ERR_ARG, "null ctx");
    ctx->timing = enable != 0;
  });
}

nq_status nq_timing_report(nq_ctx* ctx, char* buf, int64_t cap, int64_t* len) {
  return guarded(ctx, [&] {
    NQ_REQUIRE(ctx && len, NQ_ERR_ARG, "null argument");
    NQ_HIP(hipStreamSynchronize(ctx->stream));
    int ne = 0;
    if (ctx->ws.nedge.p) NQ_HIP(hipMemcpy(&ne, ctx->ws.nedge.p, sizeof(int), hipMemcpyDeviceToHost));
    struct Agg {
      int count = 0;
      double ms = 0, flop = 0, byte = 0, mfma = 0;
    };
    std::vector<std::string> order;
    std::vector<Agg> agg;
    for (const Span& s : ctx->spans) {
      float ms = 0.f;
      NQ_HIP(hipEventElapsedTime(&ms, s.a, s.b));
      size_t k = 0;
      while (k < order.size() && order[k] != s.name) ++k;
      if (k == order.size()) {
        order.push_back(s.name);
        agg.push_back(Agg());
      }
      agg[k].count++;
      agg[k].ms += ms;
      // per evaluation: a span inside the centre-chunk loop runs once per
      // chunk and its launches together cover every edge once
      agg[k].flop = s.flop_per_edge * ne + s.flop_per_atom * (double)ctx->ws.n_atoms;
      agg[k].byte = s.byte_per_edge * ne + s.byte_per_atom * (double)ctx->ws.n_atoms;
      agg[k].mfma = s.mfma_flop_per_edge * ne;
      ctx->event_pool.push_back(s.a);
      ctx->event_pool.push_back(s.b);
    }
    ctx->spans.clear();
    // evaluations covered: the launches of the once-per-evaluation energy sum
    int n_eval = 0;
    for (size_t k = 0; k < order.size(); ++k)
      if (order[k] == "total_energy") n_eval = agg[k].count;
    if (n_eval == 0)
      for (const Agg& g : agg) n_eval = n_eval ? std::min(n_eval, g.count) : g.count;
    for (Agg& g : agg) {
      const double per = (double)n_eval / (double)g.count;  // evaluations per launch
      g.flop *= per;
      g.byte *= per;
      g.mfma *= per;
    }
    std::string out = "{\"n_edges\": " + std::to_string(ne) + ", \"kernels\": [";
    char tmp[512];
    for (size_t k = 0; k < order.size(); ++k) {
      std::snprintf(tmp, sizeof(tmp),
                    "%s{\"name\": \"%s\", \"count\": %d, \"ms_total\": %.6f, \"flop_per_launch\": %.6e, "
                    "\"mfma_flop_per_launch\": %.6e, \"bytes_per_launch\": %.6e}",
                    k ? ", " : "", order[k].c_str(), agg[k].count, agg[k].ms, agg[k].flop, agg[k].mfma, agg[k].byte);
      out += tmp;
    }
    out += "]}";
    *len = (int64_t)out.size();
    NQ_REQUIRE(buf && cap > (int64_t)out.size(), NQ_ERR_CAPACITY, "report buffer too small");
    std::memcpy(buf, out.c_str(), out.size() + 1);
  });
}

const char* nq_status_str(nq_status status) {
  switch (status) {
    case NQ_OK: return "ok";
    case NQ_ERR_ARG: return "invalid argument";
    case NQ_ERR_UNSUPPORTED: return "unsupported";
    case NQ_ERR_CAPACITY: return "capacity exceeded";
    case NQ_ERR_NUMERIC: return "numeric error";
    case NQ_ERR_DEVICE: return "device error";
    case NQ_ERR_OOM: return "out of device memory";
  }
  return "unknown status";
}

const char* nq_last_error(const nq_ctx* ctx) { return ctx ? ctx->last_error.c_str() : g_error.c_str(); }

}  // extern "C"
