// Build-time generator of the real Clebsch-Gordan tables used by the HIP
// kernels. Writes a header of constexpr arrays (path list and nonzero
// coefficients) to the path given on the command line.
//
// Method: for a natural-parity path (l1, l2, l3) (triangle rule, even
// l1+l2+l3; the MACE table of Appendix F excludes pseudotensors) the real
// Gaunt integral G[m1,m2,m3] = (1/4pi) \int Y1 Y2 Y3 dOmega over the real,
// component-normalised harmonics is a rotation-invariant tensor, hence
// proportional to the coupling tensor. Since sum G Y1(n) Y2(n) Y3(n) is
// constant in n and integrates to |G|^2 > 0, the proportionality constant is
// positive, so G / |G| * sqrt(2 l3 + 1) is the coupling tensor normalised to
// sum_{m1 m2} C[m1,m2,m3] C[m1,m2,m3'] = delta and with the sign that makes
// sum C Y1(n) Y2(n) a positive multiple of Y3(n).
//
// The integral is exact: Gauss-Legendre in cos(theta) with 8 nodes (exact to
// degree 15) times 16 uniform azimuths (exact for trigonometric degree < 16);
// the integrand has degree <= 9.
#include <cmath>
#include <cstdio>
#include <vector>

namespace {

constexpr int kLmax = 3;
constexpr int kNc = (kLmax + 1) * (kLmax + 1);

// Real harmonics of the unit vector (x, y, z), component normalised
// (sum_m Y_lm^2 = 2l+1), index l*l + m + l, m = -l..l.
void real_sh(double x, double y, double z, double* Y) {
  const double s3 = std::sqrt(3.0), s15 = std::sqrt(15.0), s5 = std::sqrt(5.0);
  const double s105 = std::sqrt(105.0), s7 = std::sqrt(7.0);
  const double a358 = std::sqrt(35.0 / 8.0), a218 = std::sqrt(21.0 / 8.0);
  Y[0] = 1.0;
  Y[1] = s3 * y;
  Y[2] = s3 * z;
  Y[3] = s3 * x;
  Y[4] = s15 * x * y;
  Y[5] = s15 * y * z;
  Y[6] = 0.5 * s5 * (3.0 * z * z - 1.0);
  Y[7] = s15 * x * z;
  Y[8] = 0.5 * s15 * (x * x - y * y);
  Y[9] = a358 * y * (3.0 * x * x - y * y);
  Y[10] = s105 * x * y * z;
  Y[11] = a218 * y * (5.0 * z * z - 1.0);
  Y[12] = 0.5 * s7 * z * (5.0 * z * z - 3.0);
  Y[13] = a218 * x * (5.0 * z * z - 1.0);
  Y[14] = 0.5 * s105 * z * (x * x - y * y);
  Y[15] = a358 * x * (x * x - 3.0 * y * y);
}

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

struct Nz {
  int m1, m2, m3;
  double c;
};

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: gen_tables <out.inc>\n");
    return 2;
  }
  // Quadrature points and weights normalised to total weight 1 (= 1/4pi dOmega).
  std::vector<double> gx, gw;
  gauss_legendre(8, gx, gw);
  const int nphi = 16;
  std::vector<double> qw;
  std::vector<double> qY;
  for (size_t i = 0; i < gx.size(); ++i) {
    double ct = gx[i], st = std::sqrt(1.0 - ct * ct);
    for (int j = 0; j < nphi; ++j) {
      double ph = 2.0 * M_PI * j / nphi;
      double Y[kNc];
      real_sh(st * std::cos(ph), st * std::sin(ph), ct, Y);
      qY.insert(qY.end(), Y, Y + kNc);
      qw.push_back(gw[i] * 0.5 / nphi);
    }
  }
  const size_t nq = qw.size();

  struct Path {
    int l1, l2, l3;
    std::vector<Nz> nz;
  };
  std::vector<Path> paths;
  for (int l3 = 0; l3 <= kLmax; ++l3)
    for (int l1 = 0; l1 <= kLmax; ++l1)
      for (int l2 = 0; l2 <= kLmax; ++l2) {
        if (l3 < std::abs(l1 - l2) || l3 > l1 + l2 || (l1 + l2 + l3) % 2) continue;
        Path p{l1, l2, l3, {}};
        const int d1 = 2 * l1 + 1, d2 = 2 * l2 + 1, d3 = 2 * l3 + 1;
        std::vector<double> G(d1 * d2 * d3, 0.0);
        for (size_t q = 0; q < nq; ++q) {
          const double* Y = &qY[q * kNc];
          for (int a = 0; a < d1; ++a)
            for (int b = 0; b < d2; ++b)
              for (int c = 0; c < d3; ++c)
                G[(a * d2 + b) * d3 + c] += qw[q] * Y[l1 * l1 + a] * Y[l2 * l2 + b] * Y[l3 * l3 + c];
        }
        double nrm = 0.0;
        for (double g : G) nrm += g * g;
        const double scale = std::sqrt(d3 / nrm);
        for (int a = 0; a < d1; ++a)
          for (int b = 0; b < d2; ++b)
            for (int c = 0; c < d3; ++c) {
              double v = G[(a * d2 + b) * d3 + c] * scale;
              if (std::fabs(v) > 1e-12) p.nz.push_back({a, b, c, v});
            }
        paths.push_back(p);
      }

  FILE* f = std::fopen(argv[1], "w");
  if (!f) {
    std::perror("gen_tables");
    return 1;
  }
  std::fprintf(f, "// Generated by gen_tables.cpp: real Clebsch-Gordan coefficients from exact\n");
  std::fprintf(f, "// quadrature of real Gaunt integrals. Do not edit.\n#pragma once\n\n");
  std::fprintf(f, "namespace e3mi_cg {\n");
  std::fprintf(f, "constexpr int kNumPaths = %zu;  // ordered by (l3, l1, l2)\n", paths.size());
  size_t nnz = 0;
  for (auto& p : paths) nnz += p.nz.size();
  std::fprintf(f, "constexpr int kNumNz = %zu;\n", nnz);
  auto emit_int = [&](const char* name, auto get) {
    std::fprintf(f, "constexpr int %s[kNumPaths] = {", name);
    for (size_t i = 0; i < paths.size(); ++i) std::fprintf(f, "%s%d", i ? ", " : "", get(paths[i]));
    std::fprintf(f, "};\n");
  };
  emit_int("kL1", [](const Path& p) { return p.l1; });
  emit_int("kL2", [](const Path& p) { return p.l2; });
  emit_int("kL3", [](const Path& p) { return p.l3; });
  std::fprintf(f, "constexpr int kNzBegin[kNumPaths + 1] = {");
  size_t acc = 0;
  for (size_t i = 0; i < paths.size(); ++i) {
    std::fprintf(f, "%zu, ", acc);
    acc += paths[i].nz.size();
  }
  std::fprintf(f, "%zu};\n", acc);
  const char* names[3] = {"kM1", "kM2", "kM3"};
  for (int w = 0; w < 3; ++w) {
    std::fprintf(f, "constexpr int %s[kNumNz] = {", names[w]);
    size_t k = 0;
    for (auto& p : paths)
      for (auto& z : p.nz) std::fprintf(f, "%s%d", k++ ? ", " : "", w == 0 ? z.m1 : (w == 1 ? z.m2 : z.m3));
    std::fprintf(f, "};\n");
  }
  std::fprintf(f, "constexpr float kC[kNumNz] = {");
  size_t k = 0;
  for (auto& p : paths)
    for (auto& z : p.nz) std::fprintf(f, "%s%.9ef", k++ ? ", " : "", z.c);
  std::fprintf(f, "};\n");
  std::fprintf(f, "constexpr double kC64[kNumNz] = {");
  k = 0;
  for (auto& p : paths)
    for (auto& z : p.nz) std::fprintf(f, "%s%.17e", k++ ? ", " : "", z.c);
  std::fprintf(f, "};\n}  // namespace e3mi_cg\n");
  std::fclose(f);
  return 0;
}
