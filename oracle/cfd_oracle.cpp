// Serial FP64 reference solver ("oracle") for the finite-volume right-hand
// side of the compressible Navier-Stokes equations in Bezgin, Buhendwa &
// Adams, "JAX-FLUIDS: A fully-differentiable high-order computational fluid
// dynamics solver for compressible two-phase flows" (arXiv:2203.13760).
//
// TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the
// CPU-baseline leg of the benchmark are its only users; the product library
// never includes, links or calls it, and it shares no code with it.
//
// It is deliberately plain: one loop per face, per axis, per variable, in the
// order the method defines the operation, with no blocking or fusion. Each
// step cites the passage of the paper (or of the method the paper cites) that
// defines it. Where the paper does not print a formula, the standard published
// form of the cited method is written out and the reading is named.
//
// Data layout at the C interface: a state is 5 contiguous variables
// (rho, rho*u, rho*v, rho*w, E), each a padded block [Z][Y][X] with x fastest.
// An active axis with n cells carries nh halo cells on each side; an inactive
// axis (n == 1) carries none (§4.1: inactive axes have extent one).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "scalar.hpp"

extern "C" {
typedef struct {
  int32_t n[3];        // interior cells per axis; 1 marks an inactive axis
  int32_t nh;          // halo width on active axes (>= 3)
  double lo[3], hi[3]; // domain box
  double gamma;        // ratio of specific heats (> 1)
  double mu;           // dynamic viscosity (>= 0)
  double prandtl;      // Prandtl number (> 0)
  double cfl;          // CFL number
  int32_t bc[6];       // x-, x+, y-, y+, z-, z+ : 0 periodic, 1 zero gradient, 2 reflecting wall
  uint32_t flags;      // 1 inviscid flux, 2 viscous flux, 4 heat flux, 8 WENO5-Z reconstruction,
                       // 16 Roe flux splitting in characteristic space (the paper's ROE setup),
                       // 32 WENO3-JS reconstruction, 64 Rusanov flux, 128 TVD-RK2 time integration,
                       // 256 Rusanov-NN flux (Rusanov with the learned dissipation of §7.4),
                       // 512 safe reconstruction (first-order states at faces whose
                       // reconstructed rho or p is not positive)
} oracle_cfg;
}

namespace oracle {

enum { BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1, BC_REFLECT = 2 };
enum : uint32_t {
  F_INVISCID = 1u, F_VISCOUS = 2u, F_HEAT = 4u, F_WENOZ = 8u, F_ROE = 16u, F_WENO3 = 32u, F_RUSANOV = 64u,
  F_RK2 = 128u, F_RUSANOV_NN = 256u, F_SAFE_RECON = 512u
};

// --------------------------------------------------------------------------
// Grid: cell (i,j,k), interior indices 0..n-1, halo indices -nh..-1, n..n+nh-1.
// Cell sizes dx_d = (hi_d - lo_d)/n_d (§3.1: cuboid cells on a Cartesian grid).
struct Grid {
  int n[3], h[3], N[3];
  bool act[3];
  double dx[3];
  long ncell;
  explicit Grid(const oracle_cfg& c) {
    for (int d = 0; d < 3; ++d) {
      n[d] = c.n[d];
      act[d] = c.n[d] > 1;
      h[d] = act[d] ? c.nh : 0;
      N[d] = n[d] + 2 * h[d];
      dx[d] = (c.hi[d] - c.lo[d]) / n[d];
    }
    ncell = (long)N[0] * N[1] * N[2];
  }
  long at(int i, int j, int k) const {
    return ((long)(k + h[2]) * N[1] + (j + h[1])) * N[0] + (i + h[0]);
  }
  // Index of the cell displaced by s along axis d from cell (i,j,k).
  long shift(int d, int i, int j, int k, int s) const {
    int q[3] = {i, j, k};
    q[d] += s;
    return at(q[0], q[1], q[2]);
  }
};

// --------------------------------------------------------------------------
// Boundary conditions (§3.7 and Table of numerical methods: periodic and zero
// gradient; the setup file of Appendix A calls zero gradient "neumann" without
// a value; the implosion of §7.4 reflects its shock at walls, read as a slip
// wall: the halo mirrors the interior about the boundary face and the momentum
// normal to it changes sign). Halo layers are filled axis by axis, x then y
// then z; each later axis sweeps the full extent of the earlier axes including
// their halos, so edge and corner halo cells are filled consistently.
template <class R>
void fill_halo(const oracle_cfg& c, const Grid& g, std::vector<R>& U) {
  for (int d = 0; d < 3; ++d) {
    if (!g.act[d]) continue;
    const int n = g.n[d];
    // ranges of the two other axes: interior for later axes, padded for earlier
    int lo[3], hi[3];
    for (int e = 0; e < 3; ++e) {
      if (e < d) { lo[e] = -g.h[e]; hi[e] = g.n[e] + g.h[e]; }
      else       { lo[e] = 0;       hi[e] = g.n[e]; }
    }
    lo[d] = 0; hi[d] = 1;  // the axis itself is looped below
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          for (int m = 1; m <= g.h[d]; ++m) {
            // low side: halo cell -m; high side: halo cell n-1+m
            const int blo = c.bc[2 * d], bhi = c.bc[2 * d + 1];
            const int src_lo = blo == BC_PERIODIC ? n - m : (blo == BC_REFLECT ? m - 1 : 0);
            const int src_hi = bhi == BC_PERIODIC ? m - 1 : (bhi == BC_REFLECT ? n - m : n - 1);
            int q[3] = {i, j, k};
            q[d] = 0;
            for (int v = 0; v < 5; ++v) {
              R* Uv = U.data() + (long)v * g.ncell;
              const double slo = (blo == BC_REFLECT && v == 1 + d) ? -1.0 : 1.0;
              const double shi = (bhi == BC_REFLECT && v == 1 + d) ? -1.0 : 1.0;
              Uv[g.shift(d, q[0], q[1], q[2], -m)] = slo * Uv[g.shift(d, q[0], q[1], q[2], src_lo)];
              Uv[g.shift(d, q[0], q[1], q[2], n - 1 + m)] = shi * Uv[g.shift(d, q[0], q[1], q[2], src_hi)];
            }
          }
        }
  }
}

// --------------------------------------------------------------------------
// Health word of the calling thread, OR-accumulated by the solver and read
// (and cleared) through oracle_status: bit 0 a non-finite conservative value,
// bit 1 rho <= 0, bit 2 p <= 0, in a state a step starts from or produces
// (stage states included); bit 3 a reconstructed face state with rho <= 0 or
// p <= 0, where the Riemann solver's sound speed is undefined. Appendix A
// names an "is_safe_reconstruction" switch for this situation without
// defining it; the reading here flags such faces and repairs nothing.
inline int& health_word() {
  static thread_local int h = 0;
  return h;
}

// --------------------------------------------------------------------------
// Primitive variables W = (rho, u, v, w, p) from U = (rho, rho u, rho v, rho w, E)
// (§2: E = rho e + 1/2 rho u.u; stiffened-gas law p = (gamma-1) rho e - gamma B
// with B = 0, the ideal gas used throughout §5). Also T~ = p/rho, which is the
// temperature times the gas constant; the heat flux below needs only T~.
template <class R>
struct Prims {
  std::vector<R> rho, u[3], p, T;
};

template <class R>
void primitives(const oracle_cfg& c, const Grid& g, const std::vector<R>& U, Prims<R>& W) {
  W.rho.assign(g.ncell, R(0.0));
  for (int d = 0; d < 3; ++d) W.u[d].assign(g.ncell, R(0.0));
  W.p.assign(g.ncell, R(0.0));
  W.T.assign(g.ncell, R(0.0));
  for (long q = 0; q < g.ncell; ++q) {
    const R rho = U[q];
    const R ux = U[1 * g.ncell + q] / rho;
    const R uy = U[2 * g.ncell + q] / rho;
    const R uz = U[3 * g.ncell + q] / rho;
    const R E = U[4 * g.ncell + q];
    const R kin = 0.5 * (U[1 * g.ncell + q] * ux + U[2 * g.ncell + q] * uy + U[3 * g.ncell + q] * uz);
    const R p = (c.gamma - 1.0) * (E - kin);
    W.rho[q] = rho;
    W.u[0][q] = ux;
    W.u[1][q] = uy;
    W.u[2][q] = uz;
    W.p[q] = p;
    W.T[q] = p / rho;
  }
}

// --------------------------------------------------------------------------
// WENO5-JS (Jiang & Shu 1996; the paper's HLLC setup of §5 uses it on the
// primitive variables). Value at the right face of the centre cell c of the
// five-cell stencil (a, b, c, d, e) = (q_{i-2}, ..., q_{i+2}):
// three third-order candidates p_k, smoothness indicators beta_k, linear
// weights (0.1, 0.6, 0.3), nonlinear weights alpha_k = d_k/(eps + beta_k)^2
// with eps = 1e-6, normalised.
template <class R>
R weno5_js(R a, R b, R c, R d, R e) {
  const double eps = 1.0e-6;
  const R beta0 = (13.0 / 12.0) * sq(a - 2.0 * b + c) + 0.25 * sq(a - 4.0 * b + 3.0 * c);
  const R beta1 = (13.0 / 12.0) * sq(b - 2.0 * c + d) + 0.25 * sq(b - d);
  const R beta2 = (13.0 / 12.0) * sq(c - 2.0 * d + e) + 0.25 * sq(3.0 * c - 4.0 * d + e);
  const R p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  const R p1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  const R p2 = (2.0 * c + 5.0 * d - e) / 6.0;
  const R alpha0 = 0.1 / sq(eps + beta0);
  const R alpha1 = 0.6 / sq(eps + beta1);
  const R alpha2 = 0.3 / sq(eps + beta2);
  return (alpha0 * p0 + alpha1 * p1 + alpha2 * p2) / (alpha0 + alpha1 + alpha2);
}

// WENO5-Z (Borges, Carmona, Costa & Don 2008; the paper lists WENO5-JS/Z among
// its reconstructions, §3.3): the same candidates and smoothness indicators,
// with the global indicator tau5 = |beta0 - beta2| and nonlinear weights
// alpha_k = d_k (1 + tau5 / (beta_k + eps)), eps = 1e-40, normalised.
template <class R>
R weno5_z(R a, R b, R c, R d, R e) {
  const double eps = 1.0e-40;
  const R beta0 = (13.0 / 12.0) * sq(a - 2.0 * b + c) + 0.25 * sq(a - 4.0 * b + 3.0 * c);
  const R beta1 = (13.0 / 12.0) * sq(b - 2.0 * c + d) + 0.25 * sq(b - d);
  const R beta2 = (13.0 / 12.0) * sq(c - 2.0 * d + e) + 0.25 * sq(3.0 * c - 4.0 * d + e);
  const R tau5 = abs_(beta0 - beta2);
  const R p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  const R p1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  const R p2 = (2.0 * c + 5.0 * d - e) / 6.0;
  const R alpha0 = 0.1 * (1.0 + tau5 / (beta0 + eps));
  const R alpha1 = 0.6 * (1.0 + tau5 / (beta1 + eps));
  const R alpha2 = 0.3 * (1.0 + tau5 / (beta2 + eps));
  return (alpha0 * p0 + alpha1 * p1 + alpha2 * p2) / (alpha0 + alpha1 + alpha2);
}

// WENO3-JS (Jiang & Shu 1996, r = 2; the implosion of §7.4 reconstructs with
// it): value at the right face of the centre cell b of the stencil (a, b, c) =
// (q_{i-1}, q_i, q_{i+1}): candidates p0 = (3b - a)/2 and p1 = (b + c)/2,
// smoothness indicators (b - a)^2 and (c - b)^2, linear weights (1/3, 2/3),
// alpha_k = d_k/(eps + beta_k)^2 with eps = 1e-6 (reading: as WENO5-JS),
// normalised.
template <class R>
R weno3_js(R a, R b, R c) {
  const double eps = 1.0e-6;
  const R beta0 = sq(b - a);
  const R beta1 = sq(c - b);
  const R p0 = 1.5 * b - 0.5 * a;
  const R p1 = 0.5 * b + 0.5 * c;
  const R alpha0 = (1.0 / 3.0) / sq(eps + beta0);
  const R alpha1 = (2.0 / 3.0) / sq(eps + beta1);
  return (alpha0 * p0 + alpha1 * p1) / (alpha0 + alpha1);
}

// Rusanov (local Lax-Friedrichs) flux of §7.4 across a face normal to axis d
// from the reconstructed primitive states WL, WR:
//   F = (F_L + F_R)/2 - alpha (U_R - U_L)/2,
//   alpha = max(|u_L - c_L|, |u_L + c_L|, |u_R - c_R|, |u_R + c_R|),
// u the face-normal velocity and c the speed of sound of each state.
template <class R>
void rusanov_flux(double gamma, const R WL[5], const R WR[5], int d, R F[5]);

// Rusanov-NN flux of §7.4: the Rusanov form with alpha replaced by the output
// of a multi-layer perceptron. Inputs are the face-normal velocity jump
// |u_R - u_L|, the mean normal velocity (u_L + u_R)/2, the mean speed of sound
// (c_L + c_R)/2 and the entropy jump |s_R - s_L|; three hidden layers of 32
// units with ReLU; one output through exp, so alpha >= 0. The entropy is
// s = ln(p / rho^gamma) / (gamma - 1) (specific entropy in units of c_v, up to
// an additive constant that the jump cancels; the same s as in §7.3).
// Parameters theta, 2305 values in this order: W1 (32 x 4, row-major), b1
// (32), W2 (32 x 32), b2, W3 (32 x 32), b3, W4 (1 x 32), b4 (1); a layer maps
// h -> W h + b.
constexpr int NN_IN = 4, NN_H = 32;
constexpr int NN_PARAMS = NN_H * NN_IN + NN_H + 2 * (NN_H * NN_H + NN_H) + NN_H + 1;

template <class R>
R nn_alpha(const R* th, const R f[NN_IN]) {
  R h[NN_H], g[NN_H];
  for (int o = 0; o < NN_H; ++o) {
    R s = th[NN_H * NN_IN + o];
    for (int i = 0; i < NN_IN; ++i) s = s + th[o * NN_IN + i] * f[i];
    h[o] = max_(s, R(0.0));
  }
  const R* L = th + NN_H * NN_IN + NN_H;
  for (int layer = 0; layer < 2; ++layer, L += NN_H * NN_H + NN_H) {
    for (int o = 0; o < NN_H; ++o) {
      R s = L[NN_H * NN_H + o];
      for (int i = 0; i < NN_H; ++i) s = s + L[o * NN_H + i] * h[i];
      g[o] = max_(s, R(0.0));
    }
    for (int o = 0; o < NN_H; ++o) h[o] = g[o];
  }
  R s = L[NN_H];
  for (int i = 0; i < NN_H; ++i) s = s + L[i] * h[i];
  return exp_(s);
}

// Network weights for the scalar type in use, set by the entry points that
// evaluate the Rusanov-NN flux (the taped entry points hold them as leaves).
template <class R>
const R*& nn_weights() {
  static thread_local const R* w = nullptr;
  return w;
}

template <class R>
void rusanov_nn_flux(double gamma, const R WL[5], const R WR[5], int d, const R* th, R F[5]);

// --------------------------------------------------------------------------
// Einfeldt (1988) signal speeds of the HLLC solver below (the setup file of
// Appendix A selects "EINFELDT"; the formula is not printed, reading: the
// Roe-averaged form with the min/max safety bounds). From the primitive
// states left and right of a face normal to axis d, with r_K = sqrt(rho_K)
// and the sound speeds c_K = sqrt(gamma p_K / rho_K):
//   ubar  = (r_L u_L + r_R u_R) / (r_L + r_R)
//   dbar2 = (r_L c_L^2 + r_R c_R^2) / (r_L + r_R) + eta2 (u_R - u_L)^2,
//   eta2  = 1/2 r_L r_R / (r_L + r_R)^2
//   S_L = min(u_L - c_L, ubar - dbar),  S_R = max(u_R + c_R, ubar + dbar).
template <class R>
void einfeldt_speeds(double gamma, const R WL[5], const R WR[5], int d, R& ubar, R& dbar, R& SL, R& SR) {
  const R rL = WL[0], uL = WL[1 + d], pL = WL[4];
  const R rR = WR[0], uR = WR[1 + d], pR = WR[4];
  const R cL = sqrt_(gamma * pL / rL);
  const R cR = sqrt_(gamma * pR / rR);
  const R sL = sqrt_(rL), sR = sqrt_(rR);
  ubar = (sL * uL + sR * uR) / (sL + sR);
  const R eta2 = 0.5 * sL * sR / sq(sL + sR);
  const R dbar2 = (sL * cL * cL + sR * cR * cR) / (sL + sR) + eta2 * sq(uR - uL);
  dbar = sqrt_(dbar2);
  SL = min_(uL - cL, ubar - dbar);
  SR = max_(uR + cR, ubar + dbar);
}

// --------------------------------------------------------------------------
// HLLC approximate Riemann solver (Toro, Spruce & Speares 1994; §3.3 step 3)
// with the Einfeldt (1988) signal-speed estimate (the setup file of Appendix A
// selects "HLLC" with "EINFELDT"). Inputs are the reconstructed primitive
// states left (L) and right (R) of a face normal to axis d, in physical slot
// order (rho, u, v, w, p). The output F is in physical slot order as well.
template <class R>
void hllc_flux(double gamma, const R WL[5], const R WR[5], int d, R F[5]) {
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  // normal-first ordering of the state (§3.3: dimension-by-dimension)
  const R rL = WL[0], uL = WL[1 + d], aL = WL[1 + t1], bL = WL[1 + t2], pL = WL[4];
  const R rR = WR[0], uR = WR[1 + d], aR = WR[1 + t1], bR = WR[1 + t2], pR = WR[4];
  // step 2 of §3.3: primitive -> conservative face states, and the physical
  // fluxes of §2 (convective flux F, G, H rotated to the face normal)
  const R EL = pL / (gamma - 1.0) + 0.5 * rL * (uL * uL + aL * aL + bL * bL);
  const R ER = pR / (gamma - 1.0) + 0.5 * rR * (uR * uR + aR * aR + bR * bR);
  const R UL[5] = {rL, rL * uL, rL * aL, rL * bL, EL};
  const R UR[5] = {rR, rR * uR, rR * aR, rR * bR, ER};
  const R FL[5] = {rL * uL, rL * uL * uL + pL, rL * uL * aL, rL * uL * bL, uL * (EL + pL)};
  const R FR[5] = {rR * uR, rR * uR * uR + pR, rR * uR * aR, rR * uR * bR, uR * (ER + pR)};
  // Einfeldt: Roe-averaged normal velocity and sound-speed bound
  R ubar, dbar, SL, SR;
  einfeldt_speeds(gamma, WL, WR, d, ubar, dbar, SL, SR);
  // contact wave speed
  const R Sstar = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                  (rL * (SL - uL) - rR * (SR - uR));
  R Fn[5];
  if (0.0 <= val(SL)) {
    for (int v = 0; v < 5; ++v) Fn[v] = FL[v];
  } else if (val(SL) < 0.0 && 0.0 <= val(Sstar)) {
    const R f = rL * (SL - uL) / (SL - Sstar);
    const R Us[5] = {f, f * Sstar, f * aL, f * bL,
                     f * (EL / rL + (Sstar - uL) * (Sstar + pL / (rL * (SL - uL))))};
    for (int v = 0; v < 5; ++v) Fn[v] = FL[v] + SL * (Us[v] - UL[v]);
  } else if (val(Sstar) < 0.0 && 0.0 < val(SR)) {
    const R f = rR * (SR - uR) / (SR - Sstar);
    const R Us[5] = {f, f * Sstar, f * aR, f * bR,
                     f * (ER / rR + (Sstar - uR) * (Sstar + pR / (rR * (SR - uR))))};
    for (int v = 0; v < 5; ++v) Fn[v] = FR[v] + SR * (Us[v] - UR[v]);
  } else {
    for (int v = 0; v < 5; ++v) Fn[v] = FR[v];
  }
  // back to physical slot order
  F[0] = Fn[0];
  F[1 + d] = Fn[1];
  F[1 + t1] = Fn[2];
  F[1 + t2] = Fn[3];
  F[4] = Fn[4];
}

// --------------------------------------------------------------------------
// Flux-splitting approach of §3.3 (the paper's ROE setup of §5: Roe average,
// WENO5-JS flux reconstruction in characteristic space). For the face between
// cells i and i+1 along axis d, in the order the paper lists the steps:
//   1. the Roe average (Roe 1981; Toro 2009, §11.2) of cells i and i+1:
//      sqrt(rho)-weighted velocity and total enthalpy H = (E + p)/rho,
//      a^2 = (gamma - 1)(H - |u|^2/2);
//   2. the eigen-decomposition A = R Lambda R^-1 of the Euler flux Jacobian
//      along d at that state: eigenvalues u_d - a, u_d (three times), u_d + a
//      and the right eigenvectors of Toro 2009, §3.2, with the shear waves
//      carrying the unit vectors of the two tangential axes; R^-1 is formed
//      here by Gauss-Jordan elimination of R (not from its closed form);
//   3. V_j = R^-1 U_j and G_j = R^-1 F_j for the six stencil cells
//      j = i-2 .. i+3, F the Euler flux along d;
//   4. G+-_j = (G_j +- |Lambda| V_j) / 2: the Roe splitting takes the moduli of
//      the face's eigenvalues (reading: no entropy fix);
//   5. WENO5-JS of G+ over cells i-2..i+2 and of G- over cells i+3..i-1
//      (mirrored), characteristic field by field;
//   6. G_face = G+ + G-;
//   7. F_face = R G_face.
template <class R>
void euler_flux(double gamma, const R w[5], int d, R F[5]) {
  const R rho = w[0], un = w[1 + d], p = w[4];
  const R E = p / (gamma - 1.0) + 0.5 * rho * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  F[0] = rho * un;
  for (int a = 0; a < 3; ++a) F[1 + a] = rho * un * w[1 + a] + (a == d ? p : R(0.0));
  F[4] = un * (E + p);
}

template <class R>
void conservative(double gamma, const R w[5], R U[5]) {
  U[0] = w[0];
  for (int a = 0; a < 3; ++a) U[1 + a] = w[0] * w[1 + a];
  U[4] = w[4] / (gamma - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
}

template <class R>
void rusanov_flux(double gamma, const R WL[5], const R WR[5], int d, R F[5]) {
  R UL[5], UR[5], FL[5], FR[5];
  conservative(gamma, WL, UL);
  conservative(gamma, WR, UR);
  euler_flux(gamma, WL, d, FL);
  euler_flux(gamma, WR, d, FR);
  const R cL = sqrt_(gamma * WL[4] / WL[0]), cR = sqrt_(gamma * WR[4] / WR[0]);
  const R uL = WL[1 + d], uR = WR[1 + d];
  const R alpha = max_(max_(abs_(uL - cL), abs_(uL + cL)), max_(abs_(uR - cR), abs_(uR + cR)));
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * alpha * (UR[v] - UL[v]);
}

template <class R>
void rusanov_nn_flux(double gamma, const R WL[5], const R WR[5], int d, const R* th, R F[5]) {
  R UL[5], UR[5], FL[5], FR[5];
  conservative(gamma, WL, UL);
  conservative(gamma, WR, UR);
  euler_flux(gamma, WL, d, FL);
  euler_flux(gamma, WR, d, FR);
  const R cL = sqrt_(gamma * WL[4] / WL[0]), cR = sqrt_(gamma * WR[4] / WR[0]);
  const R uL = WL[1 + d], uR = WR[1 + d];
  const R sL = (log_(WL[4]) - gamma * log_(WL[0])) / (gamma - 1.0);
  const R sR = (log_(WR[4]) - gamma * log_(WR[0])) / (gamma - 1.0);
  const R f[NN_IN] = {abs_(uR - uL), 0.5 * (uL + uR), 0.5 * (cL + cR), abs_(sR - sL)};
  const R alpha = nn_alpha(th, f);
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * alpha * (UR[v] - UL[v]);
}

// Steps 1 and 2 for primitive states wl (cell i) and wr (cell i+1): right
// eigenvectors as the columns of Rm (row-major 5x5), Lm = Rm^-1, eigenvalues lam.
template <class R>
void roe_eigen(double gamma, const R wl[5], const R wr[5], int d, R Rm[25], R Lm[25], R lam[5]) {
  const R sl = sqrt_(wl[0]), sr = sqrt_(wr[0]);
  const R Hl = (gamma / (gamma - 1.0)) * wl[4] / wl[0] + 0.5 * (wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]);
  const R Hr = (gamma / (gamma - 1.0)) * wr[4] / wr[0] + 0.5 * (wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3]);
  R u[3];
  for (int a = 0; a < 3; ++a) u[a] = (sl * wl[1 + a] + sr * wr[1 + a]) / (sl + sr);
  const R H = (sl * Hl + sr * Hr) / (sl + sr);
  const R q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const R c = sqrt_((gamma - 1.0) * (H - 0.5 * q2));
  const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  // columns: acoustic (u_d - a), entropy, shear t1, shear t2, acoustic (u_d + a)
  R col[5][5];
  col[0][0] = R(1.0);
  col[1][0] = R(1.0);
  col[2][0] = R(0.0);
  col[3][0] = R(0.0);
  col[4][0] = R(1.0);
  for (int a = 0; a < 3; ++a) {
    const R n = R(a == d ? 1.0 : 0.0);
    col[0][1 + a] = u[a] - c * n;
    col[1][1 + a] = u[a];
    col[2][1 + a] = R(a == t1 ? 1.0 : 0.0);
    col[3][1 + a] = R(a == t2 ? 1.0 : 0.0);
    col[4][1 + a] = u[a] + c * n;
  }
  col[0][4] = H - u[d] * c;
  col[1][4] = 0.5 * q2;
  col[2][4] = u[t1];
  col[3][4] = u[t2];
  col[4][4] = H + u[d] * c;
  for (int r = 0; r < 5; ++r)
    for (int k = 0; k < 5; ++k) Rm[r * 5 + k] = col[k][r];
  lam[0] = u[d] - c;
  lam[1] = u[d];
  lam[2] = u[d];
  lam[3] = u[d];
  lam[4] = u[d] + c;
  // Gauss-Jordan elimination with partial pivoting on [Rm | I]
  R A[5][10];
  for (int r = 0; r < 5; ++r)
    for (int k = 0; k < 10; ++k) A[r][k] = k < 5 ? Rm[r * 5 + k] : R(k - 5 == r ? 1.0 : 0.0);
  for (int k = 0; k < 5; ++k) {
    int piv = k;
    for (int r = k + 1; r < 5; ++r)
      if (std::fabs(val(A[r][k])) > std::fabs(val(A[piv][k]))) piv = r;
    if (piv != k)
      for (int m = 0; m < 10; ++m) std::swap(A[k][m], A[piv][m]);
    const R inv = 1.0 / A[k][k];
    for (int m = 0; m < 10; ++m) A[k][m] = A[k][m] * inv;
    for (int r = 0; r < 5; ++r) {
      if (r == k) continue;
      const R f = A[r][k];
      for (int m = 0; m < 10; ++m) A[r][m] = A[r][m] - f * A[k][m];
    }
  }
  for (int r = 0; r < 5; ++r)
    for (int k = 0; k < 5; ++k) Lm[r * 5 + k] = A[r][5 + k];
}

// Convective flux by Roe flux splitting from the primitive states of the six
// stencil cells w[0..5] = cells i-2 .. i+3 (steps 1-7 above).
template <class R>
void roe_split_flux(double gamma, const R w[6][5], int d, R F[5]) {
  R Rm[25], Lm[25], lam[5];
  roe_eigen(gamma, w[2], w[3], d, Rm, Lm, lam);
  R Gp[6][5], Gm[6][5];
  for (int j = 0; j < 6; ++j) {
    R U[5], Fj[5];
    conservative(gamma, w[j], U);
    euler_flux(gamma, w[j], d, Fj);
    for (int k = 0; k < 5; ++k) {
      R V = R(0.0), G = R(0.0);
      for (int m = 0; m < 5; ++m) {
        V = V + Lm[k * 5 + m] * U[m];
        G = G + Lm[k * 5 + m] * Fj[m];
      }
      const R al = abs_(lam[k]);
      Gp[j][k] = 0.5 * (G + al * V);
      Gm[j][k] = 0.5 * (G - al * V);
    }
  }
  R Gf[5];
  for (int k = 0; k < 5; ++k) {
    const R plus = weno5_js(Gp[0][k], Gp[1][k], Gp[2][k], Gp[3][k], Gp[4][k]);
    const R minus = weno5_js(Gm[5][k], Gm[4][k], Gm[3][k], Gm[2][k], Gm[1][k]);
    Gf[k] = plus + minus;
  }
  for (int r = 0; r < 5; ++r) {
    R acc = R(0.0);
    for (int k = 0; k < 5; ++k) acc = acc + Rm[r * 5 + k] * Gf[k];
    F[r] = acc;
  }
}

// --------------------------------------------------------------------------
// Dissipative flux at the face between cells i and i+1 along axis d
// (§2: stresses tau with the Stokes hypothesis, Fourier heat flux q = -lambda
// grad T; §3.4: fourth-order central differences).
//  * derivative along the face normal, directly at the face:
//        (psi_{i-1} - 27 psi_i + 27 psi_{i+1} - psi_{i+2}) / (24 dx)
//  * derivative along a tangential axis t: first at the cell centres
//        (psi_{c-2} - 8 psi_{c-1} + 8 psi_{c+1} - psi_{c+2}) / (12 dx_t),
//    for the four cells c = i-1 .. i+2 along d, then interpolated to the face
//    with the fourth-order central interpolation (-D_{i-1} + 9 D_i + 9 D_{i+1} - D_{i+2})/16
//    (reading: the paper's interpolation indices are shifted by one cell; the
//    face i+1/2 sits between cells i and i+1);
//  * face velocities for the work term: the same fourth-order interpolation.
// lambda grad T = gamma mu / ((gamma-1) Pr) grad(p/rho), because
// lambda = mu c_p / Pr and c_p = gamma R/(gamma-1): the gas constant cancels.
template <class R>
void dissipative_flux(const oracle_cfg& c, const Grid& g, const Prims<R>& W, int d,
                      int i, int j, int k, bool viscous, bool heat, R F[5]) {
  const int ii[3] = {i, j, k};
  auto cell = [&](int s) {  // cell displaced by s along d from (i,j,k)
    int q[3] = {ii[0], ii[1], ii[2]};
    q[d] += s;
    return g.at(q[0], q[1], q[2]);
  };
  // normal derivative at the face
  auto dnormal = [&](const std::vector<R>& psi) {
    return (psi[cell(-1)] - 27.0 * psi[cell(0)] + 27.0 * psi[cell(1)] - psi[cell(2)]) / (24.0 * g.dx[d]);
  };
  // tangential derivative along t at the face
  auto dtangent = [&](const std::vector<R>& psi, int t) {
    if (!g.act[t]) return R(0.0);
    R D[4];
    for (int s = -1; s <= 2; ++s) {
      int q[3] = {ii[0], ii[1], ii[2]};
      q[d] += s;
      auto at_t = [&](int o) {
        int r[3] = {q[0], q[1], q[2]};
        r[t] += o;
        return g.at(r[0], r[1], r[2]);
      };
      D[s + 1] = (psi[at_t(-2)] - 8.0 * psi[at_t(-1)] + 8.0 * psi[at_t(1)] - psi[at_t(2)]) / (12.0 * g.dx[t]);
    }
    return (-D[0] + 9.0 * D[1] + 9.0 * D[2] - D[3]) / 16.0;
  };
  auto interp = [&](const std::vector<R>& psi) {
    return (-psi[cell(-1)] + 9.0 * psi[cell(0)] + 9.0 * psi[cell(1)] - psi[cell(2)]) / 16.0;
  };

  for (int v = 0; v < 5; ++v) F[v] = R(0.0);
  if (viscous) {
    // velocity gradient at the face: grad[a][b] = d u_a / d x_b
    R grad[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        grad[a][b] = (b == d) ? dnormal(W.u[a]) : dtangent(W.u[a], b);
    const R div = grad[0][0] + grad[1][1] + grad[2][2];
    R tau[3];  // tau^{d,b}
    for (int b = 0; b < 3; ++b) {
      tau[b] = c.mu * (grad[d][b] + grad[b][d]);
      if (b == d) tau[b] = tau[b] - (2.0 / 3.0) * c.mu * div;
    }
    R uf[3];
    for (int a = 0; a < 3; ++a) uf[a] = interp(W.u[a]);
    F[1] = tau[0];
    F[2] = tau[1];
    F[3] = tau[2];
    F[4] = uf[0] * tau[0] + uf[1] * tau[1] + uf[2] * tau[2];
  }
  if (heat) {
    const double kappa = c.gamma * c.mu / ((c.gamma - 1.0) * c.prandtl);
    // -q_d = lambda dT/dx_d
    F[4] = F[4] + kappa * dnormal(W.T);
  }
}

// --------------------------------------------------------------------------
// Numerical flux G = F - F^d across the face between cells (a) and (a)+1
// along axis d: F is the convective flux of the high-order Godunov approach
// (§3.3: reconstruct W with WENO5-JS left and right of the face, convert,
// HLLC), F^d the dissipative flux.
template <class R>
void face_flux(const oracle_cfg& c, const Grid& g, const Prims<R>& W, int d, const int a[3],
               bool inviscid, bool viscous, bool heat, R G[5]) {
  const std::vector<R>* q[5] = {&W.rho, &W.u[0], &W.u[1], &W.u[2], &W.p};
  R Fc[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
  if (inviscid && (c.flags & F_ROE)) {
    R w[6][5];
    for (int j = 0; j < 6; ++j)
      for (int v = 0; v < 5; ++v) w[j][v] = (*q[v])[g.shift(d, a[0], a[1], a[2], j - 2)];
    roe_split_flux(c.gamma, w, d, Fc);
  } else if (inviscid) {
    R WL[5], WR[5];
    for (int v = 0; v < 5; ++v) {
      const std::vector<R>& s = *q[v];
      auto at = [&](int o) { return s[g.shift(d, a[0], a[1], a[2], o)]; };
      if (c.flags & F_WENO3) {
        WL[v] = weno3_js(at(-1), at(0), at(1));
        WR[v] = weno3_js(at(2), at(1), at(0));
      } else if (c.flags & F_WENOZ) {
        WL[v] = weno5_z(at(-2), at(-1), at(0), at(1), at(2));
        WR[v] = weno5_z(at(3), at(2), at(1), at(0), at(-1));
      } else {
        WL[v] = weno5_js(at(-2), at(-1), at(0), at(1), at(2));
        WR[v] = weno5_js(at(3), at(2), at(1), at(0), at(-1));
      }
    }
    if (!(val(WL[0]) > 0.0) || !(val(WL[4]) > 0.0) || !(val(WR[0]) > 0.0) || !(val(WR[4]) > 0.0)) {
      health_word() |= 8;
      // safe reconstruction (Appendix A's is_safe_reconstruction; reading:
      // both states of the face fall back to the values of the two cells next
      // to it, the first-order reconstruction)
      if (c.flags & F_SAFE_RECON)
        for (int v = 0; v < 5; ++v) {
          const std::vector<R>& s = *q[v];
          WL[v] = s[g.shift(d, a[0], a[1], a[2], 0)];
          WR[v] = s[g.shift(d, a[0], a[1], a[2], 1)];
        }
    }
    if (c.flags & F_RUSANOV_NN) rusanov_nn_flux(c.gamma, WL, WR, d, nn_weights<R>(), Fc);
    else if (c.flags & F_RUSANOV) rusanov_flux(c.gamma, WL, WR, d, Fc);
    else hllc_flux(c.gamma, WL, WR, d, Fc);
  }
  R Fd[5] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
  if (viscous || heat) dissipative_flux(c, g, W, d, a[0], a[1], a[2], viscous, heat, Fd);
  for (int v = 0; v < 5; ++v) G[v] = Fc[v] - Fd[v];
}

// --------------------------------------------------------------------------
// Right-hand side of the semi-discrete finite-volume scheme (§3.1, Eq. FVD):
//   dU_i/dt = - sum_d (G_{i+1/2} - G_{i-1/2}) / dx_d,   G = F - F^d.
// Axes are treated one after the other (dimension by dimension, §3.1).
// Each face flux is computed once and used by both neighbouring cells.
// U is the padded state; its halos are refreshed here (Algorithm 2 refills
// boundaries before every right-hand-side evaluation). R is padded; its halo
// entries are zero.
template <class R>
void rhs(const oracle_cfg& c, const Grid& g, std::vector<R>& U, std::vector<R>& Rhs) {
  fill_halo(c, g, U);
  Prims<R> W;
  primitives(c, g, U, W);
  Rhs.assign(5 * g.ncell, R(0.0));
  const bool inviscid = c.flags & F_INVISCID;
  const bool viscous = (c.flags & F_VISCOUS) && c.mu > 0.0;
  const bool heat = (c.flags & F_HEAT) && c.mu > 0.0;
  for (int d = 0; d < 3; ++d) {
    if (!g.act[d]) continue;
    const int n = g.n[d];
    int ext[3] = {g.n[0], g.n[1], g.n[2]};
    ext[d] = 1;
    std::vector<R> G((size_t)(n + 1) * 5);
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          // faces f = -1 .. n-1, face f between cells f and f+1 of this line
          for (int f = -1; f < n; ++f) {
            int a[3] = {i, j, k};
            a[d] = f;
            face_flux(c, g, W, d, a, inviscid, viscous, heat, &G[(size_t)(f + 1) * 5]);
          }
          for (int m = 0; m < n; ++m) {
            int a[3] = {i, j, k};
            a[d] = m;
            const long cidx = g.at(a[0], a[1], a[2]);
            for (int v = 0; v < 5; ++v) {
              const R diff = (G[(size_t)(m + 1) * 5 + v] - G[(size_t)m * 5 + v]) / g.dx[d];
              Rhs[(long)v * g.ncell + cidx] = Rhs[(long)v * g.ncell + cidx] - diff;
            }
          }
        }
  }
}

// --------------------------------------------------------------------------
// Time step from the CFL criterion (§3.2 cites Hoppe et al. 2022; the formula
// is not printed, reading):
//   convective: s_c = max over interior cells of sum_d (|u_d| + c)/dx_d
//   viscous   : s_v = max over interior cells of 2 (mu/rho) max(4/3, gamma/Pr) sum_d dx_d^-2
//   dt = CFL / max(s_c, s_v), then clipped so that t + dt <= t_end.
inline double cfl_dt(const oracle_cfg& c, const Grid& g, const std::vector<double>& U,
                     double t, double t_end) {
  double sc = 0.0, sv = 0.0;
  const bool visc = ((c.flags & (F_VISCOUS | F_HEAT)) != 0) && c.mu > 0.0;
  double inv2 = 0.0;
  for (int d = 0; d < 3; ++d)
    if (g.act[d]) inv2 += 1.0 / (g.dx[d] * g.dx[d]);
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const long q = g.at(i, j, k);
        const double rho = U[q];
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = U[(1 + d) * g.ncell + q] / rho;
        const double kin = 0.5 * (U[1 * g.ncell + q] * u[0] + U[2 * g.ncell + q] * u[1] +
                                  U[3 * g.ncell + q] * u[2]);
        const double p = (c.gamma - 1.0) * (U[4 * g.ncell + q] - kin);
        const double cs = std::sqrt(c.gamma * p / rho);
        double s = 0.0;
        for (int d = 0; d < 3; ++d)
          if (g.act[d]) s += (std::fabs(u[d]) + cs) / g.dx[d];
        sc = std::max(sc, s);
        if (visc) {
          const double r = std::max(4.0 / 3.0, c.gamma / c.prandtl);
          sv = std::max(sv, 2.0 * (c.mu / rho) * r * inv2);
        }
      }
  double dt = c.cfl / std::max(sc, sv);
  if (t_end > 0.0) dt = std::min(dt, t_end - t);
  return dt;
}

// --------------------------------------------------------------------------
// Third-order TVD Runge-Kutta (Gottlieb & Shu 1998; §3.2), in exactly this form:
//   U1   = Un + dt R(Un)
//   U2   = 3/4 Un + 1/4 (U1 + dt R(U1))
//   Un+1 = 1/3 Un + 2/3 (U2 + dt R(U2))
// dt stays fixed over the three stages. Only interior cells are updated; the
// halos of the result are refreshed afterwards. With F_RK2 the step is the
// second-order TVD Runge-Kutta scheme of the same paper (the implosion of §7.4
// integrates with TVD-RK2):
//   U1   = Un + dt R(Un)
//   Un+1 = 1/2 Un + 1/2 (U1 + dt R(U1))
// Bits 0-2 of the health word for the interior cells of a state.
template <class R>
void note_health(const oracle_cfg& c, const Grid& g, const std::vector<R>& U) {
  int bad = 0;
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const long q = g.at(i, j, k);
        double u[5];
        for (int v = 0; v < 5; ++v) u[v] = val(U[(long)v * g.ncell + q]);
        if (!std::isfinite(u[0]) || !std::isfinite(u[1]) || !std::isfinite(u[2]) || !std::isfinite(u[3]) ||
            !std::isfinite(u[4]))
          bad |= 1;
        if (!(u[0] > 0.0)) bad |= 2;
        const double kin = 0.5 * (u[1] * (u[1] / u[0]) + u[2] * (u[2] / u[0]) + u[3] * (u[3] / u[0]));
        if (!((c.gamma - 1.0) * (u[4] - kin) > 0.0)) bad |= 4;
      }
  health_word() |= bad;
}

template <class R>
void rk3_step(const oracle_cfg& c, const Grid& g, std::vector<R>& U, double dt) {
  std::vector<R> Un = U, U1 = U, U2 = U, Rh;
  auto interior = [&](auto&& body) {
    for (int v = 0; v < 5; ++v)
      for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
          for (int i = 0; i < g.n[0]; ++i) body((long)v * g.ncell + g.at(i, j, k));
  };
  note_health(c, g, Un);
  rhs(c, g, Un, Rh);
  interior([&](long q) { U1[q] = Un[q] + dt * Rh[q]; });
  note_health(c, g, U1);
  if (c.flags & F_RK2) {
    rhs(c, g, U1, Rh);
    interior([&](long q) { U[q] = 0.5 * Un[q] + 0.5 * (U1[q] + dt * Rh[q]); });
    note_health(c, g, U);
    fill_halo(c, g, U);
    return;
  }
  rhs(c, g, U1, Rh);
  interior([&](long q) { U2[q] = 0.75 * Un[q] + 0.25 * (U1[q] + dt * Rh[q]); });
  note_health(c, g, U2);
  rhs(c, g, U2, Rh);
  interior([&](long q) { U[q] = (1.0 / 3.0) * Un[q] + (2.0 / 3.0) * (U2[q] + dt * Rh[q]); });
  note_health(c, g, U);
  fill_halo(c, g, U);
}

// Conservative state from primitive point values, interior cells only (§2).
template <class R>
void state_init(const oracle_cfg& c, const Grid& g, const R* W, std::vector<R>& U) {
  U.assign(5 * g.ncell, R(0.0));
  const long ni = (long)g.n[0] * g.n[1] * g.n[2];
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const long s = ((long)k * g.n[1] + j) * g.n[0] + i;
        const long q = g.at(i, j, k);
        const R rho = W[s], u = W[ni + s], v = W[2 * ni + s], w = W[3 * ni + s], p = W[4 * ni + s];
        U[q] = rho;
        U[g.ncell + q] = rho * u;
        U[2 * g.ncell + q] = rho * v;
        U[3 * g.ncell + q] = rho * w;
        U[4 * g.ncell + q] = p / (c.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
      }
  fill_halo(c, g, U);
}

}  // namespace oracle

// ============================================================================
// C interface for the test suite (ctypes). All arrays are host memory owned by
// the caller; padded arrays have 5 * prod(n_d + 2 h_d) entries. Return 0 on
// success, -1 on an invalid configuration.
using namespace oracle;

static int check_cfg(const oracle_cfg* c) {
  if (!c) return -1;
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 1) return -1;
    if (c->n[d] > 1 && c->n[d] < c->nh) return -1;  // periodic images need n >= nh
    if (!(c->hi[d] > c->lo[d])) return -1;
    if (c->n[d] > 1 && ((c->bc[2 * d] == BC_PERIODIC) != (c->bc[2 * d + 1] == BC_PERIODIC))) return -1;
    if (c->bc[2 * d] < 0 || c->bc[2 * d] > BC_REFLECT || c->bc[2 * d + 1] < 0 || c->bc[2 * d + 1] > BC_REFLECT)
      return -1;
  }
  if (c->nh < 3 || !(c->gamma > 1.0) || !(c->mu >= 0.0) || !(c->prandtl > 0.0)) return -1;
  // the Rusanov-NN flux needs weights (oracle_set_nn) and is not a flux splitting
  if ((c->flags & F_RUSANOV_NN) && (!nn_weights<double>() || (c->flags & F_ROE))) return -1;
  return 0;
}

// Weights of the Rusanov-NN flux for the entry points below (copied).
static std::vector<double>& nn_store() {
  static std::vector<double> w;
  return w;
}

// Taped copies of the network weights: leaves on the active tape while one of
// the reverse-mode entry points runs with the Rusanov-NN flux.
struct NNLeaves {
  std::vector<TVar> th;
  std::vector<int32_t> id;
  explicit NNLeaves(bool on) {
    if (!on) return;
    const std::vector<double>& w = nn_store();
    th.resize(w.size());
    id.resize(w.size());
    for (size_t p = 0; p < w.size(); ++p) { th[p] = TVar::leaf(w[p]); id[p] = th[p].id; }
    nn_weights<TVar>() = th.data();
  }
  ~NNLeaves() { nn_weights<TVar>() = nullptr; }
  void read(const std::vector<double>& adj, double* theta_bar) const {
    if (!theta_bar) return;
    for (size_t p = 0; p < id.size(); ++p) theta_bar[p] = adj[id[p]];
  }
};

extern "C" {

long oracle_state_numel(const oracle_cfg* c) {
  if (check_cfg(c)) return -1;
  return 5 * Grid(*c).ncell;
}

int oracle_state_init(const oracle_cfg* c, const double* W, double* U) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  std::vector<double> u;
  state_init(*c, g, W, u);
  std::memcpy(U, u.data(), sizeof(double) * u.size());
  return 0;
}

int oracle_fill_halo(const oracle_cfg* c, double* U) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  std::vector<double> u(U, U + 5 * g.ncell);
  fill_halo(*c, g, u);
  std::memcpy(U, u.data(), sizeof(double) * u.size());
  return 0;
}

// R = rhs(U); U's halos are refreshed in place.
int oracle_rhs(const oracle_cfg* c, double* U, double* R) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  std::vector<double> u(U, U + 5 * g.ncell), r;
  rhs(*c, g, u, r);
  std::memcpy(U, u.data(), sizeof(double) * u.size());
  std::memcpy(R, r.data(), sizeof(double) * r.size());
  return 0;
}

double oracle_dt(const oracle_cfg* c, const double* U, double t, double t_end) {
  if (check_cfg(c)) return -1.0;
  Grid g(*c);
  std::vector<double> u(U, U + 5 * g.ncell);
  return cfl_dt(*c, g, u, t, t_end);
}

// One TVD-RK3 step; dt <= 0 selects the CFL time step. Writes the dt used.
int oracle_rk3_step(const oracle_cfg* c, double* U, double dt, double* dt_used) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  std::vector<double> u(U, U + 5 * g.ncell);
  fill_halo(*c, g, u);
  if (dt <= 0.0) dt = cfl_dt(*c, g, u, 0.0, 0.0);
  rk3_step(*c, g, u, dt);
  std::memcpy(U, u.data(), sizeof(double) * u.size());
  if (dt_used) *dt_used = dt;
  return 0;
}

// n_steps CFL steps, stopping at t_end (> 0) with a clipped last step.
// fixed_dt > 0 replaces the CFL step. *t is read and updated. Returns the
// number of steps taken.
int oracle_advance(const oracle_cfg* c, double* U, int n_steps, double t_end, double fixed_dt,
                   double* t) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  std::vector<double> u(U, U + 5 * g.ncell);
  fill_halo(*c, g, u);
  double time = t ? *t : 0.0;
  int taken = 0;
  for (int s = 0; s < n_steps; ++s) {
    if (t_end > 0.0 && time >= t_end) break;
    double dt = fixed_dt > 0.0 ? fixed_dt : cfl_dt(*c, g, u, time, t_end);
    if (fixed_dt > 0.0 && t_end > 0.0) dt = std::min(dt, t_end - time);
    rk3_step(*c, g, u, dt);
    time += dt;
    ++taken;
  }
  std::memcpy(U, u.data(), sizeof(double) * u.size());
  if (t) *t = time;
  return taken;
}

// The calling thread's health word (see health_word); clear != 0 resets it.
int oracle_status(int clear) {
  const int h = health_word();
  if (clear) health_word() = 0;
  return h;
}

// Single-face building blocks, for unit tests of the method's pieces.
double oracle_weno5(double a, double b, double c, double d, double e) {
  return weno5_js(a, b, c, d, e);
}
double oracle_weno5z(double a, double b, double c, double d, double e) {
  return weno5_z(a, b, c, d, e);
}
void oracle_hllc(double gamma, const double* WL, const double* WR, int d, double* F) {
  hllc_flux(gamma, WL, WR, d, F);
}
// The Einfeldt speeds HLLC uses at that face: out = (ubar, dbar, S_L, S_R).
void oracle_einfeldt(double gamma, const double* WL, const double* WR, int d, double* out) {
  einfeldt_speeds(gamma, WL, WR, d, out[0], out[1], out[2], out[3]);
}
// Roe average and eigen-decomposition between primitive states wl, wr
// (rho, u, v, w, p) along axis d: Rm, Lm row-major 5x5, lam[5].
void oracle_roe_eigen(double gamma, const double* wl, const double* wr, int d, double* Rm, double* Lm,
                      double* lam) {
  roe_eigen(gamma, wl, wr, d, Rm, Lm, lam);
}
// Roe flux-splitting convective flux from six primitive states w (6 x 5,
// cells i-2 .. i+3) at the face between the third and the fourth.
void oracle_roe_flux(double gamma, const double* w, int d, double* F) {
  double ww[6][5];
  for (int j = 0; j < 6; ++j)
    for (int v = 0; v < 5; ++v) ww[j][v] = w[j * 5 + v];
  roe_split_flux(gamma, ww, d, F);
}
double oracle_weno3(double a, double b, double c) { return weno3_js(a, b, c); }
void oracle_rusanov(double gamma, const double* WL, const double* WR, int d, double* F) {
  rusanov_flux(gamma, WL, WR, d, F);
}
// Euler flux along axis d of one primitive state.
void oracle_euler_flux(double gamma, const double* w, int d, double* F) { euler_flux(gamma, w, d, F); }

// Rusanov-NN weights (2305 values, copied) for every entry point that takes a
// configuration with the Rusanov-NN flux; NULL clears them. Returns the count.
int oracle_set_nn(const double* theta) {
  if (!theta) {
    nn_store().clear();
    nn_weights<double>() = nullptr;
    return NN_PARAMS;
  }
  nn_store().assign(theta, theta + NN_PARAMS);
  nn_weights<double>() = nn_store().data();
  return NN_PARAMS;
}

// Network output alpha for the feature vector f (4 values) with the weights set
// by oracle_set_nn; negative if none are set.
double oracle_nn_alpha(const double* f) {
  if (!nn_weights<double>()) return -1.0;
  return nn_alpha(nn_weights<double>(), f);
}

// Rusanov-NN face flux with the weights set by oracle_set_nn.
int oracle_rusanov_nn(double gamma, const double* WL, const double* WR, int d, double* F) {
  if (!nn_weights<double>()) return -1;
  rusanov_nn_flux(gamma, WL, WR, d, nn_weights<double>(), F);
  return 0;
}

// Operation counts of one right-hand-side evaluation of state U:
// out = {add, mul, div, sqrt, cmp}.
int oracle_opcount(const oracle_cfg* c, const double* U, double* out) {
  if (check_cfg(c) || (c->flags & F_RUSANOV_NN)) return -1;
  Grid g(*c);
  std::vector<OpCount> u(5 * g.ncell), r;
  for (long q = 0; q < 5 * g.ncell; ++q) u[q] = OpCount(U[q]);
  tally() = OpTally();
  rhs(*c, g, u, r);
  const OpTally t = tally();
  out[0] = t.add; out[1] = t.mul; out[2] = t.div; out[3] = t.sqrt; out[4] = t.cmp;
  return 0;
}

// Operation counts (add+mul+div+sqrt) of the parts of one right-hand side,
// evaluated on state U: out[0] primitive conversion per cell, out[1..3] one
// face flux G normal to x, y, z at an interior face (0 for inactive axes).
int oracle_opcount_parts(const oracle_cfg* c, const double* U, double* out) {
  if (check_cfg(c) || (c->flags & F_RUSANOV_NN)) return -1;
  Grid g(*c);
  std::vector<OpCount> u(5 * g.ncell);
  for (long q = 0; q < 5 * g.ncell; ++q) u[q] = OpCount(U[q]);
  fill_halo(*c, g, u);
  auto flops = [](const OpTally& t) { return t.add + t.mul + t.div + t.sqrt; };
  tally() = OpTally();
  Prims<OpCount> W;
  primitives(*c, g, u, W);
  out[0] = flops(tally()) / (double)g.ncell;
  const bool inviscid = c->flags & F_INVISCID;
  const bool viscous = (c->flags & F_VISCOUS) && c->mu > 0.0;
  const bool heat = (c->flags & F_HEAT) && c->mu > 0.0;
  for (int d = 0; d < 3; ++d) {
    out[1 + d] = 0.0;
    if (!g.act[d]) continue;
    int a[3] = {g.n[0] / 2, g.n[1] / 2, g.n[2] / 2};
    OpCount G[5];
    tally() = OpTally();
    face_flux(*c, g, W, d, a, inviscid, viscous, heat, G);
    out[1 + d] = flops(tally());
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Reverse-mode derivatives from the tape (independent of any hand-derived
// adjoint). Each records the forward computation with TVar and reverses it.

// Ubar = (dR/dU)^T Rbar for R = rhs(U). Halo entries of Ubar receive nothing:
// the halo fill overwrites them before they are read.
// With the Rusanov-NN flux, theta_bar (2305 values, may be NULL) receives
// (dR/dtheta)^T Rbar.
int oracle_vjp_rhs_theta(const oracle_cfg* c, const double* U, const double* Rbar, double* Ubar,
                         double* theta_bar) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  Tape tape;
  active_tape() = &tape;
  std::vector<TVar> u(5 * g.ncell), r;
  for (long q = 0; q < 5 * g.ncell; ++q) u[q] = TVar::leaf(U[q]);
  std::vector<int32_t> leaf(5 * g.ncell);
  for (long q = 0; q < 5 * g.ncell; ++q) leaf[q] = u[q].id;
  NNLeaves nn(c->flags & F_RUSANOV_NN);
  rhs(*c, g, u, r);
  std::vector<double> adj(tape.nodes.size(), 0.0);
  for (long q = 0; q < 5 * g.ncell; ++q)
    if (r[q].id >= 0) adj[r[q].id] += Rbar[q];
  tape.reverse(adj);
  for (long q = 0; q < 5 * g.ncell; ++q) Ubar[q] = adj[leaf[q]];
  nn.read(adj, theta_bar);
  active_tape() = nullptr;
  return 0;
}

// Wbar = (dU/dW)^T Ubar for U = state_init(W) (§2, halos filled): W and
// Wbar hold 5 x interior primitives, Ubar a padded state (halo entries count).
int oracle_vjp_state_init(const oracle_cfg* c, const double* W, const double* Ubar, double* Wbar) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  const long ni = (long)g.n[0] * g.n[1] * g.n[2];
  Tape tape;
  active_tape() = &tape;
  std::vector<TVar> w(5 * ni);
  for (long q = 0; q < 5 * ni; ++q) w[q] = TVar::leaf(W[q]);
  std::vector<TVar> u;
  state_init(*c, g, w.data(), u);
  std::vector<double> adj(tape.nodes.size(), 0.0);
  for (long q = 0; q < 5 * g.ncell; ++q)
    if (u[q].id >= 0) adj[u[q].id] += Ubar[q];
  tape.reverse(adj);
  for (long q = 0; q < 5 * ni; ++q) Wbar[q] = adj[w[q].id];
  active_tape() = nullptr;
  return 0;
}

int oracle_vjp_rhs(const oracle_cfg* c, const double* U, const double* Rbar, double* Ubar) {
  return oracle_vjp_rhs_theta(c, U, Rbar, Ubar, nullptr);
}

// Ubar_n = (dU^{n+1}/dU^n)^T Ubar_np1 for one step (TVD-RK3, or TVD-RK2 with
// F_RK2) with fixed dt; with the Rusanov-NN flux theta_bar (may be NULL)
// receives (dU^{n+1}/dtheta)^T Ubar_np1.
int oracle_vjp_step_theta(const oracle_cfg* c, const double* Un, double dt, const double* Ubar_np1,
                          double* Ubar_n, double* theta_bar) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  Tape tape;
  active_tape() = &tape;
  std::vector<TVar> u(5 * g.ncell);
  std::vector<int32_t> leaf(5 * g.ncell);
  for (long q = 0; q < 5 * g.ncell; ++q) { u[q] = TVar::leaf(Un[q]); leaf[q] = u[q].id; }
  NNLeaves nn(c->flags & F_RUSANOV_NN);
  rk3_step(*c, g, u, dt);
  std::vector<double> adj(tape.nodes.size(), 0.0);
  // the result's halo cells are copies of interior cells: seed interior only
  for (int v = 0; v < 5; ++v)
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          const long q = (long)v * g.ncell + g.at(i, j, k);
          if (u[q].id >= 0) adj[u[q].id] += Ubar_np1[q];
        }
  tape.reverse(adj);
  for (long q = 0; q < 5 * g.ncell; ++q) Ubar_n[q] = adj[leaf[q]];
  nn.read(adj, theta_bar);
  active_tape() = nullptr;
  return 0;
}

int oracle_vjp_rk3_step(const oracle_cfg* c, const double* Un, double dt, const double* Ubar_np1,
                        double* Ubar_n) {
  return oracle_vjp_step_theta(c, Un, dt, Ubar_np1, Ubar_n, nullptr);
}

// Loss L = sum over interior cells of 1/2 |rho u|^2 / rho * dV after n_steps
// fixed-dt TVD-RK3 steps from the primitive initial state W0 (5 x interior),
// and its gradient with respect to the initial velocities (3 x interior).
// Forward states are stored; the backward pass tapes one step at a time.
int oracle_grad_ke(const oracle_cfg* c, const double* W0, int n_steps, double dt, double* loss,
                   double* grad_uvw) {
  if (check_cfg(c)) return -1;
  Grid g(*c);
  const long ni = (long)g.n[0] * g.n[1] * g.n[2];
  const double dV = g.dx[0] * g.dx[1] * g.dx[2];
  // forward, keeping every state
  std::vector<std::vector<double>> states;
  {
    std::vector<double> u;
    state_init(*c, g, W0, u);
    states.push_back(u);
    for (int s = 0; s < n_steps; ++s) {
      rk3_step(*c, g, u, dt);
      states.push_back(u);
    }
  }
  // loss and its adjoint at the final state
  std::vector<double> ubar(5 * g.ncell, 0.0);
  {
    Tape tape;
    active_tape() = &tape;
    const std::vector<double>& uN = states.back();
    std::vector<TVar> u(5 * g.ncell);
    std::vector<int32_t> leaf(5 * g.ncell);
    for (long q = 0; q < 5 * g.ncell; ++q) { u[q] = TVar::leaf(uN[q]); leaf[q] = u[q].id; }
    TVar L(0.0);
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          const long q = g.at(i, j, k);
          const TVar m2 = u[g.ncell + q] * u[g.ncell + q] + u[2 * g.ncell + q] * u[2 * g.ncell + q] +
                          u[3 * g.ncell + q] * u[3 * g.ncell + q];
          L = L + 0.5 * m2 / u[q] * dV;
        }
    *loss = L.v;
    std::vector<double> adj(tape.nodes.size(), 0.0);
    adj[L.id] = 1.0;
    tape.reverse(adj);
    for (long q = 0; q < 5 * g.ncell; ++q) ubar[q] = adj[leaf[q]];
    active_tape() = nullptr;
  }
  // backward through the steps
  for (int s = n_steps - 1; s >= 0; --s) {
    std::vector<double> prev(5 * g.ncell);
    oracle_vjp_rk3_step(c, states[s].data(), dt, ubar.data(), prev.data());
    ubar.swap(prev);
  }
  // through the primitive -> conservative map of the initial state, with rho
  // and p held fixed
  {
    Tape tape;
    active_tape() = &tape;
    std::vector<double> Wd(W0, W0 + 5 * ni);
    std::vector<TVar> W(5 * ni);
    std::vector<int32_t> leaf(3 * ni);
    for (long s = 0; s < ni; ++s) {
      W[s] = TVar(Wd[s]);
      W[4 * ni + s] = TVar(Wd[4 * ni + s]);
      for (int a = 0; a < 3; ++a) {
        W[(1 + a) * ni + s] = TVar::leaf(Wd[(1 + a) * ni + s]);
        leaf[a * ni + s] = W[(1 + a) * ni + s].id;
      }
    }
    std::vector<TVar> u;
    state_init(*c, g, W.data(), u);
    std::vector<double> adj(tape.nodes.size(), 0.0);
    for (int v = 0; v < 5; ++v)
      for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
          for (int i = 0; i < g.n[0]; ++i) {
            const long q = (long)v * g.ncell + g.at(i, j, k);
            if (u[q].id >= 0) adj[u[q].id] += ubar[q];
          }
    tape.reverse(adj);
    for (long s = 0; s < 3 * ni; ++s) grad_uvw[s] = adj[leaf[s]];
    active_tape() = nullptr;
  }
  return 0;
}

}  // extern "C"
