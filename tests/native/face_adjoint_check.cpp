// Host-side check of the hand-derived face-flux adjoints (physics_adj.hpp)
// against central differences of the forward code (physics.hpp), for all
// three face orientations and every HLLC wave pattern. Runs on the CPU.
// Prints the worst relative dot-product mismatch per routine; exit 1 on failure.
#include <cmath>
#include <cstdio>
#include <random>

#include "../../paper_2203_13760_amd/csrc/physics_adj.hpp"

using namespace cfd;

static std::mt19937_64 rng(12345);
static double U(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static int fails = 0;
// Fourth-order central difference of f along a direction, at the step in
// {1e-3 .. 1e-8} that agrees best with the adjoint value: truncation falls and
// roundoff grows as the step shrinks, and a wrong adjoint disagrees at every step.
template <class Fn>
static double best_fd(Fn&& f, double ad) {
  double best = 0, err = 1e300;
  for (double h = 1e-3; h > 5e-9; h /= 3.0) {
    const double fd = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h);
    if (std::fabs(fd - ad) < err) { err = std::fabs(fd - ad); best = fd; }
  }
  return best;
}
static void report(const char* what, double fd, double ad) {
  const double rel = std::fabs(fd - ad) / std::fmax(1e-300, std::fmax(std::fabs(fd), std::fabs(ad)));
  if (!(rel < 1e-7)) {
    std::printf("FAIL %s fd=%.12e ad=%.12e rel=%.3e\n", what, fd, ad, rel);
    ++fails;
  }
}

template <int D>
static void check_hllc(int pattern) {
  double WL[5], WR[5];
  // pattern 0: supersonic right-moving, 1: subsonic S*>0, 2: subsonic S*<0, 3: supersonic left
  const double base = pattern == 0 ? 3.0 : pattern == 3 ? -3.0 : (pattern == 1 ? 0.3 : -0.3);
  WL[0] = U(0.5, 2.0); WR[0] = U(0.5, 2.0);
  WL[4] = U(0.5, 2.0); WR[4] = U(0.5, 2.0);
  for (int a = 0; a < 3; ++a) { WL[1 + a] = U(-0.4, 0.4); WR[1 + a] = U(-0.4, 0.4); }
  WL[1 + D] += base; WR[1 + D] += base;
  const double gamma = 1.4, gm1i = 1.0 / 0.4;
  double Fb[5], dL[5], dR[5];
  for (int v = 0; v < 5; ++v) { Fb[v] = U(-1, 1); dL[v] = U(-1, 1); dR[v] = U(-1, 1); }
  double WLb[5] = {0}, WRb[5] = {0};
  hllc_rev<D>(gamma, gm1i, WL, WR, Fb, WLb, WRb);
  // fourth-order central difference along (dL, dR)
  auto dir = [&](double t, double* F) {
    double L[5], R[5];
    for (int v = 0; v < 5; ++v) { L[v] = WL[v] + t * dL[v]; R[v] = WR[v] + t * dR[v]; }
    hllc<D>(gamma, gm1i, L, R, F);
    double s = 0;
    for (int v = 0; v < 5; ++v) s += Fb[v] * F[v];
    return s;
  };
  double F[5];
  double ad = 0;
  for (int v = 0; v < 5; ++v) ad += WLb[v] * dL[v] + WRb[v] * dR[v];
  const double fd = best_fd([&](double t) { return dir(t, F); }, ad);
  char buf[64];
  std::snprintf(buf, sizeof buf, "hllc D=%d pattern=%d", D, pattern);
  report(buf, fd, ad);
}

static void check_weno() {
  for (int t = 0; t < 200; ++t) {
    double s[5], d[5];
    const bool rough = t % 2;
    for (int m = 0; m < 5; ++m) { s[m] = rough ? U(-1, 1) : 1.0 + 0.1 * m + 0.01 * U(-1, 1); d[m] = U(-1, 1); }
    const double qb = U(-1, 1);
    double g[5] = {0};
    weno5_rev(s[0], s[1], s[2], s[3], s[4], qb, g);
    auto dir = [&](double t) {
      return qb * weno5(s[0] + t * d[0], s[1] + t * d[1], s[2] + t * d[2], s[3] + t * d[3], s[4] + t * d[4]);
    };
    double ad = 0;
    for (int m = 0; m < 5; ++m) ad += g[m] * d[m];
    const double fd = best_fd(dir, ad);
    report("weno5", fd, ad);
  }
}

// The cell-centred pair (both face values of the centre cell, shared
// indicators): its reverse against central differences of weno5_pair, and
// against the sum of the two single-face reverses of the same values.
static void check_weno_pair() {
  for (int t = 0; t < 200; ++t) {
    double s[5], d[5];
    const bool rough = t % 2;
    for (int m = 0; m < 5; ++m) { s[m] = rough ? U(-1, 1) : 1.0 + 0.1 * m + 0.01 * U(-1, 1); d[m] = U(-1, 1); }
    const double qrb = U(-1, 1), qlb = U(-1, 1);
    double g[5] = {0}, h[5] = {0};
    weno5_pair_rev(s[0], s[1], s[2], s[3], s[4], qrb, qlb, g);
    weno5_rev(s[0], s[1], s[2], s[3], s[4], qrb, h);
    double hm[5] = {0};
    weno5_rev(s[4], s[3], s[2], s[1], s[0], qlb, hm);
    for (int m = 0; m < 5; ++m) h[m] += hm[4 - m];
    auto dir = [&](double t) {
      double qr, ql;
      weno5_pair(s[0] + t * d[0], s[1] + t * d[1], s[2] + t * d[2], s[3] + t * d[3], s[4] + t * d[4], qr, ql);
      return qrb * qr + qlb * ql;
    };
    double ad = 0;
    for (int m = 0; m < 5; ++m) ad += g[m] * d[m];
    report("weno5_pair", best_fd(dir, ad), ad);
    for (int m = 0; m < 5; ++m) report("weno5_pair vs single", h[m], g[m]);
  }
}

template <int D>
static void check_face(bool shocky) {
  Geom g{};
  for (int a = 0; a < 3; ++a) { g.act[a] = 1; g.dx[a] = 0.1 + 0.05 * a; g.idx[a] = 1.0 / g.dx[a]; }
  g.gamma = 1.4; g.gm1i = 1.0 / 0.4; g.mu = 0.03; g.kappa = 1.4 * 0.03 / (0.4 * 0.72);
  g.inviscid = 1; g.viscous = 1; g.heat = 1;
  FaceWindow w{}, dw{};
  for (int c = 0; c < 6; ++c) {
    w.q[c][0] = shocky ? U(0.3, 2.0) : 1.0 + 0.05 * c;
    w.q[c][4] = shocky ? U(0.3, 2.0) : 1.0 - 0.03 * c;
    for (int a = 0; a < 3; ++a) w.q[c][1 + a] = shocky ? U(-1, 1) : 0.1 * a + 0.02 * c;
    for (int v = 0; v < 5; ++v) dw.q[c][v] = U(-1, 1);
  }
  for (int c = 0; c < 4; ++c) {
    w.T[c] = w.q[c + 1][4] / w.q[c + 1][0];
    dw.T[c] = U(-1, 1);
    for (int k = 0; k < 4; ++k) { w.tg[c][k] = U(-1, 1); dw.tg[c][k] = U(-1, 1); }
  }
  double Gb[5];
  for (int v = 0; v < 5; ++v) Gb[v] = U(-1, 1);
  struct { double qb[6][6]; double tgb[5][4]; void q(int m, int v, double x) { qb[m][v] += x; }
           void tg(int m, int k, double x) { tgb[m][k] += x; } } a{};
  face_flux_rev<D>(g, w, Gb, a);
  auto dir = [&](double t) {
    FaceWindow x = w;
    for (int c = 0; c < 6; ++c)
      for (int v = 0; v < 5; ++v) x.q[c][v] += t * dw.q[c][v];
    for (int c = 0; c < 4; ++c) {
      x.T[c] += t * dw.T[c];
      for (int k = 0; k < 4; ++k) x.tg[c][k] += t * dw.tg[c][k];
    }
    double G[5];
    face_flux<D>(g, x, G);
    double s = 0;
    for (int v = 0; v < 5; ++v) s += Gb[v] * G[v];
    return s;
  };
  double ad = 0;
  for (int c = 0; c < 6; ++c)
    for (int v = 0; v < 5; ++v) ad += a.qb[c][v] * dw.q[c][v];
  for (int c = 0; c < 4; ++c) {
    ad += a.qb[1 + c][5] * dw.T[c];
    for (int k = 0; k < 4; ++k) ad += a.tgb[1 + c][k] * dw.tg[c][k];
  }
  const double fd = best_fd(dir, ad);
  char buf[64];
  std::snprintf(buf, sizeof buf, "face_flux D=%d shocky=%d", D, (int)shocky);
  report(buf, fd, ad);
}

int main() {
  check_weno();
  check_weno_pair();
  for (int t = 0; t < 50; ++t)
    for (int p = 0; p < 4; ++p) {
      check_hllc<0>(p);
      check_hllc<1>(p);
      check_hllc<2>(p);
    }
  for (int t = 0; t < 50; ++t) {
    check_face<0>(t % 2);
    check_face<1>(t % 2);
    check_face<2>(t % 2);
  }
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "OK", fails);
  return fails ? 1 : 0;
}
