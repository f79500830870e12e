// Model description, weight layout, coupling tables and device upload.
//
// The weight blob is the FP64 source of truth; FP32 and BF16 copies are derived
// by round-to-nearest-even. The coupling tables C^(l1,l2,l3) are the real Gaunt
// integrals (1/4pi) * int Y_l1m1 Y_l2m2 Y_l3m3 dOmega of the library's spherical
// harmonics (tensor products over irreducible representations, Sec. 2.1),
// computed here by exact integration of monomials over the sphere, scaled to
// unit Frobenius norm, with the first non-zero entry in (m1,m2,m3) order made
// positive.
#include <cmath>
#include <cstring>

#include "cg_const.hpp"
#include "nq_internal.hpp"

namespace nq {

namespace {

bool natural_path(int l1, int l2, int l3) {
  return std::abs(l1 - l2) <= l3 && l3 <= l1 + l2 && ((l1 + l2 + l3) % 2 == 0);
}

}  // namespace

Dims make_dims(const nq_model_desc& d) {
  Dims m{};
  NQ_REQUIRE(d.n_species >= 1 && d.n_species <= 8, NQ_ERR_UNSUPPORTED, "n_species must be 1..8");
  NQ_REQUIRE(d.n_bessel >= 1 && d.n_bessel <= 16, NQ_ERR_UNSUPPORTED, "n_bessel must be 1..16");
  NQ_REQUIRE(d.poly_p >= 2 && d.poly_p <= 16, NQ_ERR_UNSUPPORTED, "poly_p must be 2..16");
  NQ_REQUIRE(d.lmax >= 1 && d.lmax <= kMaxL, NQ_ERR_UNSUPPORTED, "lmax must be 1 or 2");
  NQ_REQUIRE(d.n_layers >= 1 && d.n_layers <= 4, NQ_ERR_UNSUPPORTED, "n_layers must be 1..4");
  NQ_REQUIRE(d.channels == 8 || d.channels == 16 || d.channels == 32 || d.channels == 64,
             NQ_ERR_UNSUPPORTED, "channels must be 8, 16, 32 or 64");
  NQ_REQUIRE(d.n_twobody >= 1 && d.n_twobody <= 4, NQ_ERR_UNSUPPORTED, "1..4 two-body layers");
  NQ_REQUIRE(d.n_latent >= 1 && d.n_latent <= 4, NQ_ERR_UNSUPPORTED, "1..4 latent layers");
  NQ_REQUIRE(d.n_edge >= 1 && d.n_edge <= 4, NQ_ERR_UNSUPPORTED, "1..4 hidden edge layers");
  NQ_REQUIRE(d.r_cut > 0 && d.avg_num_neighbors > 0, NQ_ERR_ARG, "r_cut and nu must be > 0");
  NQ_REQUIRE(d.precision == NQ_PRECISION_FP32 || d.precision == NQ_PRECISION_BF16 ||
                 d.precision == NQ_PRECISION_BF16X3,
             NQ_ERR_ARG, "unknown precision");
  m.S = d.n_species;
  m.nb = d.n_bessel;
  m.p = d.poly_p;
  m.L = d.lmax;
  m.T = d.n_layers;
  m.C = d.channels;
  m.n_tb = d.n_twobody;
  m.n_lat = d.n_latent;
  m.n_edge = d.n_edge;
  auto width_ok = [](int w) { return w >= 16 && w <= 1024 && w % 16 == 0; };
  for (int k = 0; k < m.n_tb; ++k) {
    m.tb[k] = d.twobody[k];
    NQ_REQUIRE(width_ok(m.tb[k]), NQ_ERR_UNSUPPORTED, "MLP widths must be multiples of 16 in 16..1024");
  }
  for (int k = 0; k < m.n_lat; ++k) {
    m.lat[k] = d.latent[k];
    NQ_REQUIRE(width_ok(m.lat[k]), NQ_ERR_UNSUPPORTED, "MLP widths must be multiples of 16 in 16..1024");
  }
  for (int k = 0; k < m.n_edge; ++k) {
    m.edge[k] = d.edge[k];
    NQ_REQUIRE(width_ok(m.edge[k]), NQ_ERR_UNSUPPORTED, "MLP widths must be multiples of 16 in 16..1024");
  }
  m.D = m.tb[m.n_tb - 1];
  NQ_REQUIRE(m.lat[m.n_lat - 1] == m.D, NQ_ERR_ARG, "last latent width must equal the two-body output width");
  m.NY = (m.L + 1) * (m.L + 1);
  m.NW = (m.L + 1) * m.C;
  m.n_in2b = 2 * m.S + m.nb;
  m.n_paths = 0;
  m.nscal = 0;
  for (int l = 0; l <= kMaxL; ++l) m.path_l3_count[l] = 0;
  for (int l1 = 0; l1 <= m.L; ++l1)
    for (int l2 = 0; l2 <= m.L; ++l2)
      for (int l3 = 0; l3 <= m.L; ++l3)
        if (natural_path(l1, l2, l3)) {
          m.paths[m.n_paths][0] = l1;
          m.paths[m.n_paths][1] = l2;
          m.paths[m.n_paths][2] = l3;
          m.n_paths++;
          m.path_l3_count[l3]++;
          if (l3 == 0) m.nscal++;
        }
  m.rc = d.r_cut;
  m.inv_sqrt_nu = 1.0 / std::sqrt(d.avg_num_neighbors);
  m.sigma_e = d.energy_scale;
  m.prec = d.precision;
  return m;
}

void weight_layout(const nq_model_desc& d, std::vector<std::pair<int64_t, int64_t>>& segs) {
  Dims m = make_dims(d);
  segs.clear();
  int fin = m.n_in2b;
  for (int k = 0; k < m.n_tb; ++k) {
    segs.push_back({fin, m.tb[k]});
    fin = m.tb[k];
  }
  segs.push_back({m.D, m.NW});  // W_V0
  for (int t = 1; t <= m.T; ++t) {
    segs.push_back({m.D, m.NW});  // W_env^t
    fin = m.D + m.nscal * m.C;
    for (int k = 0; k < m.n_lat; ++k) {
      segs.push_back({fin, m.lat[k]});
      fin = m.lat[k];
    }
    if (t < m.T)
      for (int l3 = 0; l3 <= m.L; ++l3) segs.push_back({(int64_t)m.path_l3_count[l3] * m.C, m.C});
  }
  fin = m.D;
  for (int k = 0; k < m.n_edge; ++k) {
    segs.push_back({fin, m.edge[k]});
    fin = m.edge[k];
  }
  segs.push_back({fin, 1});
}

// ----------------------------------------------------------------- coupling tables
namespace {

struct Mono {
  double c;
  int a, b, e;  // x^a y^b z^e
};

// The library's real spherical harmonics as polynomials in the unit vector.
std::vector<Mono> sh_poly(int l, int m) {
  const double s3 = std::sqrt(3.0), s5 = std::sqrt(5.0), s15 = std::sqrt(15.0);
  if (l == 0) return {{1.0, 0, 0, 0}};
  if (l == 1) {
    if (m == 0) return {{s3, 1, 0, 0}};
    if (m == 1) return {{s3, 0, 1, 0}};
    return {{s3, 0, 0, 1}};
  }
  switch (m) {
    case 0: return {{s15, 1, 1, 0}};
    case 1: return {{s15, 0, 1, 1}};
    case 2: return {{1.5 * s5, 0, 0, 2}, {-0.5 * s5, 0, 0, 0}};
    case 3: return {{s15, 1, 0, 1}};
    default: return {{0.5 * s15, 2, 0, 0}, {-0.5 * s15, 0, 2, 0}};
  }
}

double dfact(int n) {  // n!! with (-1)!! = 0!! = 1
  double r = 1.0;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}

// Mean of x^a y^b z^e over the unit sphere.
double sphere_mean(int a, int b, int e) {
  if ((a | b | e) & 1) return 0.0;
  return dfact(a - 1) * dfact(b - 1) * dfact(e - 1) / dfact(a + b + e + 1);
}

}  // namespace

void derive_cg(CGTable& t) {
  std::memset(&t, 0, sizeof(t));
  for (int l1 = 0; l1 <= kMaxL; ++l1)
    for (int l2 = 0; l2 <= kMaxL; ++l2)
      for (int l3 = 0; l3 <= kMaxL; ++l3) {
        if (!natural_path(l1, l2, l3)) continue;
        double g[5][5][5] = {};
        double nrm = 0.0;
        for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
          for (int m2 = 0; m2 < 2 * l2 + 1; ++m2)
            for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
              double s = 0.0;
              for (const Mono& p : sh_poly(l1, m1))
                for (const Mono& q : sh_poly(l2, m2))
                  for (const Mono& r : sh_poly(l3, m3))
                    s += p.c * q.c * r.c * sphere_mean(p.a + q.a + r.a, p.b + q.b + r.b, p.e + q.e + r.e);
              if (std::fabs(s) < 1e-12) s = 0.0;
              g[m1][m2][m3] = s;
              nrm += s * s;
            }
        nrm = std::sqrt(nrm);
        double sign = 0.0;
        for (int m1 = 0; m1 < 2 * l1 + 1 && sign == 0.0; ++m1)
          for (int m2 = 0; m2 < 2 * l2 + 1 && sign == 0.0; ++m2)
            for (int m3 = 0; m3 < 2 * l3 + 1 && sign == 0.0; ++m3)
              if (g[m1][m2][m3] != 0.0) sign = g[m1][m2][m3] > 0 ? 1.0 : -1.0;
        for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
          for (int m2 = 0; m2 < 2 * l2 + 1; ++m2)
            for (int m3 = 0; m3 < 2 * l3 + 1; ++m3)
              t.v[l1][l2][l3][m1][m2][m3] = (float)(sign * g[m1][m2][m3] / nrm);
      }
}

// ----------------------------------------------------------------- upload
namespace {

uint16_t bf16_bits_rne(double d) {
  float f = (float)d;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf/nan
  uint32_t low = u & 0xffffu;
  uint32_t hi = u >> 16;
  if (low == 0x8000u && (double)f != d) {
    // f sits exactly on a bf16 midpoint only because of the first rounding:
    // round toward the side d lies on.
    bool up = std::fabs(d) > std::fabs((double)f);
    return (uint16_t)(up ? hi + 1 : hi);
  }
  uint32_t r = u + 0x7fffu + (hi & 1u);
  return (uint16_t)(r >> 16);
}

double bf16_value(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

// BF16 copies are stored as [hi | lo] halves: hi = rne(w), lo = rne(w - hi).
void upload_lin(Lin& L, const double* W, int fin, int fout) {
  L.fin = fin;
  L.fout = fout;
  L.kp_f = (int)rup(fin, 32);
  L.np_f = (int)rup(fout, 16);
  L.kp_b = (int)rup(fout, 32);
  L.np_b = (int)rup(fin, 16);
  std::vector<float> ff((size_t)L.np_f * L.kp_f, 0.f), fb((size_t)L.np_b * L.kp_b, 0.f);
  const size_t hf = (size_t)L.np_f * L.kp_f, hb = (size_t)L.np_b * L.kp_b;
  std::vector<uint16_t> bf(2 * hf, 0), bb(2 * hb, 0);
  for (int k = 0; k < fin; ++k)
    for (int n = 0; n < fout; ++n) {
      const double w = W[(size_t)k * fout + n];
      const uint16_t hi = bf16_bits_rne(w);
      const uint16_t lo = bf16_bits_rne(w - bf16_value(hi));
      ff[(size_t)n * L.kp_f + k] = (float)w;
      bf[(size_t)n * L.kp_f + k] = hi;
      bf[hf + (size_t)n * L.kp_f + k] = lo;
      fb[(size_t)k * L.kp_b + n] = (float)w;
      bb[(size_t)k * L.kp_b + n] = hi;
      bb[hb + (size_t)k * L.kp_b + n] = lo;
    }
  L.f32_fwd.ensure(ff.size() * 4);
  L.f32_bwd.ensure(fb.size() * 4);
  L.bf_fwd.ensure(bf.size() * 2);
  L.bf_bwd.ensure(bb.size() * 2);
  NQ_HIP(hipMemcpy(L.f32_fwd.p, ff.data(), ff.size() * 4, hipMemcpyHostToDevice));
  NQ_HIP(hipMemcpy(L.f32_bwd.p, fb.data(), fb.size() * 4, hipMemcpyHostToDevice));
  NQ_HIP(hipMemcpy(L.bf_fwd.p, bf.data(), bf.size() * 2, hipMemcpyHostToDevice));
  NQ_HIP(hipMemcpy(L.bf_bwd.p, bb.data(), bb.size() * 2, hipMemcpyHostToDevice));
}

// Channel-mixing weights of one layer: per l3 a [P_l3*C, C] block W (rows (p, c),
// columns c'), stored natural and with every block transposed to [C, P_l3*C],
// in FP32 and as BF16 hi | lo halves.
void upload_mix(MixW& M, const Dims& d, const std::vector<double>& w) {
  const size_t n = w.size();
  M.n = (int64_t)n;
  std::vector<float> fN(n), fT(n);
  std::vector<uint16_t> bN(2 * n), bT(2 * n);
  size_t off = 0;
  for (int l3 = 0; l3 <= d.L; ++l3) {
    const int rows = d.path_l3_count[l3] * d.C, C = d.C;
    for (int r = 0; r < rows; ++r)
      for (int q = 0; q < C; ++q) {
        const double v = w[off + (size_t)r * C + q];
        const uint16_t hi = bf16_bits_rne(v), lo = bf16_bits_rne(v - bf16_value(hi));
        const size_t in = off + (size_t)r * C + q, it = off + (size_t)q * rows + r;
        fN[in] = (float)v;
        fT[it] = (float)v;
        bN[in] = hi;
        bN[n + in] = lo;
        bT[it] = hi;
        bT[n + it] = lo;
      }
    off += (size_t)rows * C;
  }
  M.fN.ensure(n * 4);
  M.fT.ensure(n * 4);
  M.bN.ensure(n * 4);
  M.bT.ensure(n * 4);
  NQ_HIP(hipMemcpy(M.fN.p, fN.data(), n * 4, hipMemcpyHostToDevice));
  NQ_HIP(hipMemcpy(M.fT.p, fT.data(), n * 4, hipMemcpyHostToDevice));
  NQ_HIP(hipMemcpy(M.bN.p, bN.data(), n * 4, hipMemcpyHostToDevice));
  NQ_HIP(hipMemcpy(M.bT.p, bT.data(), n * 4, hipMemcpyHostToDevice));
}

}  // namespace

}  // namespace nq

nq_model::~nq_model() {
  for (auto* p : tb) delete p;
  for (auto* p : env) delete p;
  for (auto& v : lat)
    for (auto* p : v) delete p;
  for (auto* p : edge) delete p;
  for (auto* p : mixw) delete p;
}

namespace nq {

nq_model* model_create(nq_ctx* ctx, const nq_model_desc* desc, const double* w, int64_t n_w) {
  std::vector<std::pair<int64_t, int64_t>> segs;
  weight_layout(*desc, segs);
  int64_t need = 0;
  for (auto& s : segs) need += s.first * s.second;
  NQ_REQUIRE(n_w == need, NQ_ERR_ARG,
             "weight blob has " + std::to_string(n_w) + " values, layout needs " + std::to_string(need));
  for (int64_t i = 0; i < n_w; ++i)
    NQ_REQUIRE(std::isfinite(w[i]), NQ_ERR_NUMERIC, "non-finite weight");
  NQ_HIP(hipSetDevice(ctx->device));
  nq_model* m = new nq_model();
  try {
    m->ctx = ctx;
    m->desc = *desc;
    m->dims = make_dims(*desc);
    const Dims& d = m->dims;
    size_t seg = 0;
    const double* p = w;
    auto next = [&](int& fin, int& fout) {
      fin = (int)segs[seg].first;
      fout = (int)segs[seg].second;
      const double* q = p;
      p += (size_t)fin * fout;
      seg++;
      return q;
    };
    int fi, fo;
    for (int k = 0; k < d.n_tb; ++k) {
      const double* W = next(fi, fo);
      m->tb.push_back(new Lin());
      upload_lin(*m->tb.back(), W, fi, fo);
    }
    // W_V0 and W_env^1 share their input x0: store them side by side.
    std::vector<double> cat((size_t)d.D * 2 * d.NW);
    const double* Wv0 = next(fi, fo);
    m->env.assign(d.T, nullptr);
    m->lat.assign(d.T, {});
    m->mixw.assign(d.T, nullptr);
    for (int t = 1; t <= d.T; ++t) {
      const double* We = next(fi, fo);
      if (t == 1) {
        for (int k = 0; k < d.D; ++k)
          for (int n = 0; n < d.NW; ++n) {
            cat[(size_t)k * 2 * d.NW + n] = Wv0[(size_t)k * d.NW + n];
            cat[(size_t)k * 2 * d.NW + d.NW + n] = We[(size_t)k * d.NW + n];
          }
        upload_lin(m->v0e1, cat.data(), d.D, 2 * d.NW);
      } else {
        m->env[t - 1] = new Lin();
        upload_lin(*m->env[t - 1], We, fi, fo);
      }
      for (int k = 0; k < d.n_lat; ++k) {
        const double* Wl = next(fi, fo);
        m->lat[t - 1].push_back(new Lin());
        upload_lin(*m->lat[t - 1].back(), Wl, fi, fo);
      }
      if (t < d.T) {
        std::vector<double> mixes;
        for (int l3 = 0; l3 <= d.L; ++l3) {
          const double* Wm = next(fi, fo);
          mixes.insert(mixes.end(), Wm, Wm + (size_t)fi * fo);
        }
        m->mixw[t - 1] = new MixW();
        upload_mix(*m->mixw[t - 1], d, mixes);
      }
    }
    for (int k = 0; k < d.n_edge; ++k) {
      const double* W = next(fi, fo);
      m->edge.push_back(new Lin());
      upload_lin(*m->edge.back(), W, fi, fo);
    }
    const double* Wo = next(fi, fo);
    std::vector<float> wo(fi);
    for (int k = 0; k < fi; ++k) wo[k] = (float)Wo[k];
    m->wout.ensure(wo.size() * 4);
    NQ_HIP(hipMemcpy(m->wout.p, wo.data(), wo.size() * 4, hipMemcpyHostToDevice));
    CGTable cg;
    derive_cg(cg);
    // algorithmic FLOPs per edge of each layer's tensor product (2 per multiply-add
    // over the non-zero coupling coefficients, channel mixing as dense products)
    for (int t = 1; t <= d.T; ++t) {
      double cgf = 0.0, mixf = 0.0;
      for (int p = 0; p < d.n_paths; ++p) {
        const int l1 = d.paths[p][0], l2 = d.paths[p][1], l3 = d.paths[p][2];
        if (t == d.T && l3 != 0) continue;
        int nnz = 0;
        for (int a = 0; a < 2 * l1 + 1; ++a)
          for (int b = 0; b < 2 * l2 + 1; ++b)
            for (int c = 0; c < 2 * l3 + 1; ++c) nnz += cg.v[l1][l2][l3][a][b][c] != 0.f;
        cgf += 2.0 * nnz * d.C;
        if (t < d.T) mixf += 2.0 * (2 * l3 + 1) * d.C * d.C;
      }
      m->tp_flop_fwd.push_back(cgf + mixf);
      m->tp_flop_bwd.push_back(2.0 * cgf + mixf);
      m->tp_flop_mix.push_back(mixf);
    }
    // the kernels carry the compile-time table; it must agree with this derivation
    for (int a = 0; a <= kMaxL; ++a)
      for (int b = 0; b <= kMaxL; ++b)
        for (int c = 0; c <= kMaxL; ++c)
          for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j)
              for (int k = 0; k < 5; ++k)
                NQ_REQUIRE(std::fabs(cg.v[a][b][c][i][j][k] - kCG.v[a][b][c][i][j][k]) < 1e-6f, NQ_ERR_DEVICE,
                           "compile-time coupling table disagrees with the host derivation");
  } catch (...) {
    delete m;
    throw;
  }
  return m;
}

}  // namespace nq
