// Compile-time real Clebsch-Gordan (Gaunt) coupling tables for l <= 2.
//
// Same definition as the host derivation in model.hip: the mean over the unit
// sphere of Y_l1m1 Y_l2m2 Y_l3m3 for the library's component-normalised real
// spherical harmonics, scaled to unit Frobenius norm per path, first non-zero
// entry in (m1,m2,m3) order positive. Evaluated here with constexpr arithmetic
// so that the tensor-product kernels carry the coefficients as immediates and
// skip the zero entries at compile time; model creation checks this table
// against the host derivation.
#pragma once

namespace nq {
namespace cgc {

struct Term {
  double c;
  int a, b, e;  // c * x^a y^b z^e
};
struct Poly {
  Term t[2];
  int n;
};

constexpr double csqrt(double x) {
  double r = x > 1.0 ? x : 1.0;
  for (int k = 0; k < 100; ++k) r = 0.5 * (r + x / r);
  return r;
}

constexpr Poly sh(int l, int m) {
  const double s3 = csqrt(3.0), s5 = csqrt(5.0), s15 = csqrt(15.0);
  if (l == 0) return Poly{{{1.0, 0, 0, 0}, {0, 0, 0, 0}}, 1};
  if (l == 1) {
    if (m == 0) return Poly{{{s3, 1, 0, 0}, {0, 0, 0, 0}}, 1};
    if (m == 1) return Poly{{{s3, 0, 1, 0}, {0, 0, 0, 0}}, 1};
    return Poly{{{s3, 0, 0, 1}, {0, 0, 0, 0}}, 1};
  }
  if (m == 0) return Poly{{{s15, 1, 1, 0}, {0, 0, 0, 0}}, 1};
  if (m == 1) return Poly{{{s15, 0, 1, 1}, {0, 0, 0, 0}}, 1};
  if (m == 2) return Poly{{{1.5 * s5, 0, 0, 2}, {-0.5 * s5, 0, 0, 0}}, 2};
  if (m == 3) return Poly{{{s15, 1, 0, 1}, {0, 0, 0, 0}}, 1};
  return Poly{{{0.5 * s15, 2, 0, 0}, {-0.5 * s15, 0, 2, 0}}, 2};
}

constexpr double dfact(int n) {
  double r = 1.0;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}

constexpr double sphere_mean(int a, int b, int e) {
  return ((a | b | e) & 1) ? 0.0 : dfact(a - 1) * dfact(b - 1) * dfact(e - 1) / dfact(a + b + e + 1);
}

struct Table {
  float v[3][3][3][5][5][5];
};

constexpr bool natural(int l1, int l2, int l3) {
  return (l1 - l2 <= l3) && (l2 - l1 <= l3) && (l3 <= l1 + l2) && ((l1 + l2 + l3) % 2 == 0);
}

constexpr Table make_table() {
  Table t{};
  for (int l1 = 0; l1 < 3; ++l1)
    for (int l2 = 0; l2 < 3; ++l2)
      for (int l3 = 0; l3 < 3; ++l3) {
        if (!natural(l1, l2, l3)) continue;
        double g[5][5][5] = {};
        double nrm = 0.0;
        for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
          for (int m2 = 0; m2 < 2 * l2 + 1; ++m2)
            for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) {
              const Poly p = sh(l1, m1), q = sh(l2, m2), r = sh(l3, m3);
              double s = 0.0;
              for (int i = 0; i < p.n; ++i)
                for (int j = 0; j < q.n; ++j)
                  for (int k = 0; k < r.n; ++k)
                    s += p.t[i].c * q.t[j].c * r.t[k].c *
                         sphere_mean(p.t[i].a + q.t[j].a + r.t[k].a, p.t[i].b + q.t[j].b + r.t[k].b,
                                     p.t[i].e + q.t[j].e + r.t[k].e);
              if (s < 1e-12 && s > -1e-12) s = 0.0;
              g[m1][m2][m3] = s;
              nrm += s * s;
            }
        nrm = csqrt(nrm);
        double sign = 0.0;
        for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
          for (int m2 = 0; m2 < 2 * l2 + 1; ++m2)
            for (int m3 = 0; m3 < 2 * l3 + 1; ++m3)
              if (sign == 0.0 && g[m1][m2][m3] != 0.0) sign = g[m1][m2][m3] > 0 ? 1.0 : -1.0;
        for (int m1 = 0; m1 < 2 * l1 + 1; ++m1)
          for (int m2 = 0; m2 < 2 * l2 + 1; ++m2)
            for (int m3 = 0; m3 < 2 * l3 + 1; ++m3) t.v[l1][l2][l3][m1][m2][m3] = (float)(sign * g[m1][m2][m3] / nrm);
      }
  return t;
}

}  // namespace cgc

constexpr cgc::Table kCG = cgc::make_table();

}  // namespace nq
