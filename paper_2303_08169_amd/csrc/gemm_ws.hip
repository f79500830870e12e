// Launchers of the weight-stationary edge products (k_gemm_ws) for the
// product signatures of the Allegro-style model: K steps, output tiles per
// wavefront, loader and epilogue modes. A product whose signature is not
// listed uses the tiled kernels only.
#include <map>
#include <mutex>

#include "gemm.hpp"

namespace nq {

namespace {

// (K steps, 16-column tiles per wavefront, A loader, epilogue, row tiles in
// flight beyond the current one; 1 where the weights leave no room for two).
// Each signature has two epilogue forms (per-lane stores, or whole rows
// through LDS); the autotuner picks one per product.
#define NQ_WS_LIST(X)                     \
  X(11, 2, A_CAT, E_RESIDUAL, 2)          \
  X(11, 2, A_CAT_SILU_U, E_RESIDUAL, 2)   \
  X(8, 3, A_GRADSILU, E_LATENT_BWD, 1)    \
  X(4, 2, A_SILU, E_STORE, 2)             \
  X(8, 2, A_SILU_U, E_STORE, 2)           \
  X(6, 2, A_PLAIN, E_ADD, 2)              \
  X(3, 2, A_PLAIN, E_ADD, 2)              \
  X(8, 1, A_GRADSILU, E_STORE, 2)         \
  X(4, 2, A_GRADSILU, E_STORE, 2)         \
  X(8, 2, A_PLAIN, E_STORE, 2)            \
  X(8, 1, A_PLAIN, E_STORE, 2)

// Workgroups resident at once (occupancy query x CUs), cached per kernel.
template <class K>
unsigned resident(K kernel, int num_cu) {
  static std::map<const void*, int> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  const void* key = reinterpret_cast<const void*>(kernel);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int per_cu = 0;
    NQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 512, 0));
    it = cache.emplace(key, per_cu > 0 ? per_cu : 1).first;
  }
  return (unsigned)(it->second * num_cu);
}

template <int KIND>
bool ws_dispatch(bool launch, int form, hipStream_t s, int num_cu, int NP, int Kp, const void* Bt, const int* nrows,
                 const ALoad& ld, const Epi& ep) {
  if (Kp % 32 != 0 || NP % 16 != 0 || ep.N0 % 4 != 0) return false;
  if (ld.gu && Kp != 256) return false;  // one wavefront's load must cover one row
  const int KS = Kp / 32, NTW = (NP / 16 + 7) / 8;
#define NQ_WS_CASE(ks, ntw, am, em, pf)                                                                    \
  if (KS == ks && NTW == ntw && ld.mode == am && ep.mode == em) {                                          \
    if (launch) {                                                                                          \
      auto kern = form == 0 ? k_gemm_ws<KIND, ntw, ks, am, em, pf, 0> : k_gemm_ws<KIND, ntw, ks, am, em, pf, 1>; \
      kern<<<resident(kern, num_cu), 512, 0, s>>>(NP, static_cast<const bf16*>(Bt), nrows, ld, ep);         \
    }                                                                                                      \
    return true;                                                                                           \
  }
  NQ_WS_LIST(NQ_WS_CASE)
#undef NQ_WS_CASE
  return false;
}

}  // namespace

bool gemm_ws(bool launch, int form, int kind, hipStream_t s, int num_cu, int NP, int Kp, const void* Bt,
             const int* nrows, const ALoad& ld, const Epi& ep) {
  if (kind == G_BF16X3) return ws_dispatch<G_BF16X3>(launch, form, s, num_cu, NP, Kp, Bt, nrows, ld, ep);
  if (kind == G_BF16) return ws_dispatch<G_BF16>(launch, form, s, num_cu, NP, Kp, Bt, nrows, ld, ep);
  return false;
}

}  // namespace nq
