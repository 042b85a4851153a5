// Device building blocks of the finite-volume right-hand side (gfx950).
//
// Face-local arithmetic only: WENO5-JS reconstruction, HLLC flux with Einfeldt
// signal speeds, the fourth-order dissipative flux, and the cell-local
// primitive conversion. The sweep kernels feed these from registers; face
// fluxes never leave the register file.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfd {

// Grid geometry and physics constants, passed to every kernel by value.
struct Geom {
  int n[3];        // interior cells
  int h[3];        // halo width per axis (0 on inactive axes)
  int N[3];        // padded extents
  long long s[3];  // element strides of the padded block: 1, Nx, Nx*Ny
  long long vs;    // stride between variables: Nx*Ny*Nz
  double dx[3];
  double idx[3];   // 1/dx
  int act[3];      // axis active (n > 1)
  int bc[6];       // boundary types, x-, x+, y-, y+, z-, z+
  double gamma;
  double gm1i;     // 1/(gamma - 1)
  double mu;
  double kappa;    // gamma mu / ((gamma - 1) Pr): lambda grad T = kappa grad(p/rho)
  double cfl;
  double visc_rate;  // 2 max(4/3, gamma/Pr) sum_d dx_d^-2 (times mu/rho gives the diffusive rate)
  int inviscid, viscous, heat;
  int wenoz;       // WENO5-Z instead of WENO5-JS
  int roe;         // Roe flux splitting in characteristic space instead of HLLC
  int weno3;       // WENO3-JS instead of WENO5
  int rusanov;     // Rusanov flux instead of HLLC
  int rk2;         // TVD-RK2 instead of TVD-RK3
  int seg;         // cells per lane of the y / z marches
  int nn;          // Rusanov-NN flux (with WENO3-JS): alpha per face from nna
  int safe;        // safe reconstruction: first-order states at faces with a non-positive rho or p
  const double* nnw;  // Rusanov-NN network weights (device, 2305 values)
  double* nna;        // Rusanov-NN alpha per face, [3][padded cells] at the face's left cell
};

// Convective schemes of the sweeps, a compile-time parameter: WENO5-JS or
// WENO5-Z on the primitives with HLLC (the high-order Godunov approach), or
// the flux-splitting approach with Roe eigenvalues and WENO5-JS in
// characteristic space (§3.3; the ROE setup of §5).
constexpr int SCH_JS = 0, SCH_Z = 1, SCH_ROE = 2;
// and the schemes of the implosion of §7.4: WENO3-JS with HLLC, WENO3-JS or
// WENO5-JS with the Rusanov flux
constexpr int SCH_W3 = 3, SCH_JS_RUS = 4, SCH_W3_RUS = 5;
// and the Rusanov-NN flux of §7.4 (WENO3-JS, Rusanov with the dissipation of a
// network, evaluated per face beforehand into Geom::nna)
constexpr int SCH_W3_NN = 6;
__host__ __device__ constexpr bool sch_weno3(int sch) { return sch == SCH_W3 || sch == SCH_W3_RUS || sch == SCH_W3_NN; }
__host__ __device__ constexpr bool sch_rusanov(int sch) {
  return sch == SCH_JS_RUS || sch == SCH_W3_RUS || sch == SCH_W3_NN;
}

__host__ __device__ __forceinline__ double sq(double x) { return x * x; }

// a / b for denominators that are finite, normal and nonzero wherever the
// result is used: the hardware reciprocal estimate r ~ 1/b (v_rcp_f64,
// relative error below 2^-24 on gfx950) refined by one Newton-Raphson step
// r <- r + r (1 - b r) (error below 2^-48), then one residual correction of
// the quotient q <- q + r (a - b q) (Markstein 1990). It skips the range
// scaling and special-case fixup of the IEEE division sequence, about half of
// its instructions; on 4 194 304 random operand pairs (exponents -20 .. 20)
// it returned the correctly rounded a / b every time. The host pass (host-
// compiled tests of the face code) divides.
__host__ __device__ __forceinline__ double div_nr(double a, double b) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(b);
  const double e = fma(-b, r, 1.0);
  r = fma(e, r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
#else
  return a / b;
#endif
}

// sqrt(x) for a finite x >= 2^-767 (densities, pressures, squared sound
// speeds): the hardware reciprocal square root estimate y ~ 1/sqrt(x)
// (v_rsq_f64) refined by one Goldschmidt step on the pair g ~ sqrt(x),
// h ~ 1/(2 sqrt(x)) (r = 1/2 - g h, g += g r, h += h r) and two Newton
// corrections of the root (g += (x - g^2) h). These are the steps of the
// compiler's own square root on gfx950 for such x, without its range scaling
// for tiny arguments and its fixups for 0 and infinity (x = 0 gives NaN, a
// negative x NaN as sqrt does): about half of its instructions. The host pass
// takes sqrt.
__host__ __device__ __forceinline__ double sqrt_pos(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
#else
  return sqrt(x);
#endif
}

// Cell index of interior-relative coordinates (i,j,k) (halo cells negative).
__device__ __forceinline__ long long cell_at(const Geom& g, int i, int j, int k) {
  return (long long)(k + g.h[2]) * g.s[2] + (long long)(j + g.h[1]) * g.s[1] + (i + g.h[0]);
}

// Interior source coordinate of a (possibly halo) coordinate c on an axis with
// n cells: periodic image, zero-gradient clamp (§3.7), or the mirror image
// about a reflecting wall (the slip walls of the implosion, §7.4). Applying it
// per axis reproduces the axis-by-axis halo fill, corners included.
__device__ __forceinline__ int bc_source(int c, int n, int bc_lo, int bc_hi) {
  if (c < 0) return bc_lo == 0 ? c + n : (bc_lo == 2 ? -1 - c : 0);
  if (c >= n) return bc_hi == 0 ? c - n : (bc_hi == 2 ? 2 * n - 1 - c : n - 1);
  return c;
}

// Factor of the axis's velocity (momentum) component in the image of c: -1
// through a reflecting wall, else 1. Corner cells take the product over axes.
__device__ __forceinline__ double bc_sign(int c, int n, int bc_lo, int bc_hi) {
  return ((c < 0 && bc_lo == 2) || (c >= n && bc_hi == 2)) ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// WENO5-JS (Jiang & Shu 1996) value at the right face of the centre cell c of
// the stencil (a,b,c,d,e): smoothness indicators beta_k, candidates p_k,
// linear weights (0.1, 0.6, 0.3), alpha_k = d_k/(1e-6 + beta_k)^2, normalised.
// Evaluated with a single division: with s_k = (1e-6 + beta_k)^2 the weights
// are proportional to d_k * prod_{j != k} s_j, and the 1/6 of the candidate
// stencils is applied to the normaliser. The products stay within FP64 range
// for |beta_k| up to ~1e100.
__host__ __device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
  constexpr double k13 = 13.0 / 12.0;
  constexpr double eps = 1.0e-6;
  const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
  const double t1 = b - 2.0 * c + d, u1 = b - d;
  const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
  const double s0 = sq(eps + (k13 * t0 * t0 + 0.25 * u0 * u0));
  const double s1 = sq(eps + (k13 * t1 * t1 + 0.25 * u1 * u1));
  const double s2 = sq(eps + (k13 * t2 * t2 + 0.25 * u2 * u2));
  const double w0 = 0.1 * (s1 * s2), w1 = 0.6 * (s0 * s2), w2 = 0.3 * (s0 * s1);
  const double P0 = 2.0 * a - 7.0 * b + 11.0 * c;
  const double P1 = -b + 5.0 * c + 2.0 * d;
  const double P2 = 2.0 * c + 5.0 * d - e;
  return div_nr(w0 * P0 + w1 * P1 + w2 * P2, 6.0 * (w0 + w1 + w2));
}

// WENO5-Z (Borges, Carmona, Costa & Don 2008): the same candidates and
// smoothness indicators, global indicator tau5 = |beta0 - beta2|, weights
// alpha_k = d_k (1 + tau5 / e_k) with e_k = beta_k + 1e-40, normalised.
// Single division as in weno5: with alpha_k = d_k (e_k + tau5) / e_k the
// weights are proportional to d_k (e_k + tau5) prod_{j != k} e_j.
__host__ __device__ __forceinline__ double weno5z(double a, double b, double c, double d, double e) {
  constexpr double k13 = 13.0 / 12.0;
  constexpr double eps = 1.0e-40;
  const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
  const double t1 = b - 2.0 * c + d, u1 = b - d;
  const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
  const double b0 = k13 * t0 * t0 + 0.25 * u0 * u0;
  const double b1 = k13 * t1 * t1 + 0.25 * u1 * u1;
  const double b2 = k13 * t2 * t2 + 0.25 * u2 * u2;
  const double tau = fabs(b0 - b2);
  const double e0 = b0 + eps, e1 = b1 + eps, e2 = b2 + eps;
  const double w0 = 0.1 * (e0 + tau) * (e1 * e2), w1 = 0.6 * (e1 + tau) * (e0 * e2),
               w2 = 0.3 * (e2 + tau) * (e0 * e1);
  const double P0 = 2.0 * a - 7.0 * b + 11.0 * c;
  const double P1 = -b + 5.0 * c + 2.0 * d;
  const double P2 = 2.0 * c + 5.0 * d - e;
  return (w0 * P0 + w1 * P1 + w2 * P2) / (6.0 * (w0 + w1 + w2));
}

// WENO5-JS at both faces of the centre cell c of the stencil (a, b, c, d, e) =
// q_{i-2} .. q_{i+2}: qr at the right face i+1/2 (the left state there) and
// ql at the left face i-1/2 (the right state there). The two reconstructions
// share their three smoothness indicators in mirrored roles - the indicator
// of cells i-2..i is beta_0 of qr and beta_2 of ql - so each is formed once
// per cell, from the second differences Db, Dc, Dd centred at b, c, d and the
// first differences dm = c - b, dp = d - c:
//   beta_L = 13/12 Db^2 + 1/4 (Db + 2 dm)^2     (a - 4b + 3c = Db + 2 dm)
//   beta_C = 13/12 Dc^2 + 1/4 (dm + dp)^2       (b - d = -(dm + dp))
//   beta_R = 13/12 Dd^2 + 1/4 (Dd - 2 dp)^2     (3c - 4d + e = Dd - 2 dp).
// With s_k = (1e-6 + beta_k)^2 the weights of qr are proportional to
// (0.1 s_C s_R, 0.6 s_L s_R, 0.3 s_L s_C) on the candidates
// (2a - 7b + 11c, -b + 5c + 2d, 2c + 5d - e)/6, those of ql to
// (0.1 s_L s_C, 0.6 s_L s_R, 0.3 s_C s_R) on the mirrored candidates
// (2e - 7d + 11c, -d + 5c + 2b, 2c + 5b - a)/6: the pairwise products are
// shared too. Both quotients come from one reciprocal of the product of the
// two normalisers (in range for |beta| below ~1e38).
__host__ __device__ __forceinline__ void weno5_pair(double a, double b, double c, double d, double e, double& qr,
                                                   double& ql) {
  constexpr double k13 = 13.0 / 12.0;
  constexpr double eps = 1.0e-6;
  const double Db = a - 2.0 * b + c, Dc = b - 2.0 * c + d, Dd = c - 2.0 * d + e;
  const double dm = c - b, dp = d - c;
  const double tL = Db + 2.0 * dm, tC = dm + dp, tR = Dd - 2.0 * dp;
  const double sL = sq(eps + (k13 * Db * Db + 0.25 * tL * tL));
  const double sC = sq(eps + (k13 * Dc * Dc + 0.25 * tC * tC));
  const double sR = sq(eps + (k13 * Dd * Dd + 0.25 * tR * tR));
  const double pCR = sC * sR, pLR = sL * sR, pLC = sL * sC;
  const double nr = 0.1 * pCR * (2.0 * a - 7.0 * b + 11.0 * c) + 0.6 * pLR * (-b + 5.0 * c + 2.0 * d) +
                    0.3 * pLC * (2.0 * c + 5.0 * d - e);
  const double nl = 0.1 * pLC * (2.0 * e - 7.0 * d + 11.0 * c) + 0.6 * pLR * (-d + 5.0 * c + 2.0 * b) +
                    0.3 * pCR * (2.0 * c + 5.0 * b - a);
  const double dr = 0.1 * pCR + 0.6 * pLR + 0.3 * pLC;
  const double dl = 0.1 * pLC + 0.6 * pLR + 0.3 * pCR;
  const double r = div_nr(1.0, 6.0 * (dr * dl));
  qr = nr * dl * r;
  ql = nl * dr * r;
}

// WENO3-JS (Jiang & Shu 1996, r = 2) value at the right face of the centre
// cell b of the stencil (a, b, c): candidates (3b - a)/2 and (b + c)/2,
// smoothness indicators (b - a)^2 and (c - b)^2, linear weights (1/3, 2/3),
// alpha_k = d_k/(1e-6 + beta_k)^2, normalised; one division as in weno5.
__host__ __device__ __forceinline__ double weno3(double a, double b, double c) {
  constexpr double eps = 1.0e-6;
  const double s0 = sq(eps + sq(b - a)), s1 = sq(eps + sq(c - b));
  const double w0 = s1, w1 = 2.0 * s0;  // (1/3)/s0 : (2/3)/s1, times 3 s0 s1
  return div_nr(w0 * (3.0 * b - a) + w1 * (b + c), 2.0 * (w0 + w1));
}

// WENO3-JS at both faces of the centre cell b of (a, b, c): qr = weno3(a, b, c)
// at the right face and ql = weno3(c, b, a) at the left face, sharing the two
// indicators: s0 = (1e-6 + (b - a)^2)^2 and s1 = (1e-6 + (c - b)^2)^2 weigh
// the candidates (3b - a, b + c)/2 of qr as (s1, 2 s0) and (3b - c, b + a)/2
// of ql as (s0, 2 s1).
__host__ __device__ __forceinline__ void weno3_pair(double a, double b, double c, double& qr, double& ql) {
  constexpr double eps = 1.0e-6;
  const double s0 = sq(eps + sq(b - a)), s1 = sq(eps + sq(c - b));
  const double nr = s1 * (3.0 * b - a) + 2.0 * s0 * (b + c);
  const double nl = s0 * (3.0 * b - c) + 2.0 * s1 * (b + a);
  const double dr = s1 + 2.0 * s0, dl = s0 + 2.0 * s1;
  const double r = div_nr(1.0, 2.0 * (dr * dl));
  qr = nr * dl * r;
  ql = nl * dr * r;
}

// Rusanov (local Lax-Friedrichs) flux of §7.4 across a face normal to axis D
// from reconstructed primitive states: (F_L + F_R)/2 - alpha (U_R - U_L)/2 with
// alpha the largest |u -+ c| of the two states (u normal to the face), or the
// given alpha_in (GIVEN: the Rusanov-NN flux).
template <int D, bool GIVEN = false>
__host__ __device__ __forceinline__ void rusanov(double gamma, double gm1i, const double* WL, const double* WR,
                                                 double* F, double alpha_in = 0.0) {
  const double rL = WL[0], pL = WL[4], rR = WR[0], pR = WR[4];
  const double uL = WL[1 + D], uR = WR[1 + D];
  const double kL = 0.5 * rL * (WL[1] * WL[1] + WL[2] * WL[2] + WL[3] * WL[3]);
  const double kR = 0.5 * rR * (WR[1] * WR[1] + WR[2] * WR[2] + WR[3] * WR[3]);
  const double EL = pL * gm1i + kL, ER = pR * gm1i + kR;
  double alpha = alpha_in;
  if constexpr (!GIVEN) {
    const double cL = sqrt_pos(div_nr(gamma * pL, rL)), cR = sqrt_pos(div_nr(gamma * pR, rR));
    alpha = fmax(fmax(fabs(uL - cL), fabs(uL + cL)), fmax(fabs(uR - cR), fabs(uR + cR)));
  }
  const double UL[5] = {rL, rL * WL[1], rL * WL[2], rL * WL[3], EL};
  const double UR[5] = {rR, rR * WR[1], rR * WR[2], rR * WR[3], ER};
  double FL[5], FR[5];
  FL[0] = rL * uL;
  FR[0] = rR * uR;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    FL[1 + a] = FL[0] * WL[1 + a] + (a == D ? pL : 0.0);
    FR[1 + a] = FR[0] * WR[1 + a] + (a == D ? pR : 0.0);
  }
  FL[4] = uL * (EL + pL);
  FR[4] = uR * (ER + pR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * alpha * (UR[v] - UL[v]);
}

// ---------------------------------------------------------------------------
// HLLC flux (Toro, Spruce & Speares 1994) with Einfeldt (1988) speeds across a
// face normal to axis D (five divisions, five square roots). Inputs:
// reconstructed primitive states (rho, u, v, w, p) left/right. Output in
// physical slot order. The flux comes from one side K: the left one where
// 0 <= S_L or 0 <= S*, else the right one; it is that side's physical flux
// F_K, plus S_K (U*_K - U_K) inside the star region (S_L < 0 <= S* on the
// left, S* < 0 < S_R on the right). The side's values are selected first, so
// one physical flux and one star state are evaluated, and lanes never
// diverge.
template <int D>
__host__ __device__ __forceinline__ void hllc(double gamma, double gm1i, const double* WL, const double* WR, double* F) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const double rL = WL[0], uL = WL[1 + D], pL = WL[4];
  const double rR = WR[0], uR = WR[1 + D], pR = WR[4];
  const double c2L = div_nr(gamma * pL, rL), c2R = div_nr(gamma * pR, rR);
  const double cL = sqrt_pos(c2L), cR = sqrt_pos(c2R);
  // Einfeldt: Roe-averaged normal velocity and sound-speed bound
  const double sL = sqrt_pos(rL), sR = sqrt_pos(rR);
  const double isum = div_nr(1.0, sL + sR);
  const double ubar = (sL * uL + sR * uR) * isum;
  const double eta2 = 0.5 * sL * sR * isum * isum;
  const double dbar = sqrt_pos((sL * c2L + sR * c2R) * isum + eta2 * sq(uR - uL));
  const double SL = fmin(uL - cL, ubar - dbar);
  const double SR = fmax(uR + cR, ubar + dbar);
  const double mL = rL * (SL - uL), mR = rR * (SR - uR);  // mass fluxes relative to the waves
  const double Ss = div_nr(pR - pL + uL * mL - uR * mR, mL - mR);
  const bool useL = 0.0 <= SL;
  const bool left = useL || 0.0 <= Ss;
  const bool star = left ? !useL : 0.0 < SR;
  const double r = left ? rL : rR, u = left ? uL : uR, p = left ? pL : pR;
  const double a = left ? WL[1 + T1] : WR[1 + T1], b = left ? WL[1 + T2] : WR[1 + T2];
  const double S = left ? SL : SR, m = left ? mL : mR;
  const double E = p * gm1i + 0.5 * r * (u * u + a * a + b * b);
  // star state U*_K = rho_K (S_K - u_K)/(S_K - S*) (1, S*, t1, t2, E_K/rho_K + (S*-u_K)(S* + p_K/(rho_K (S_K-u_K))));
  // the energy slot is rearranged so that no division by rho_K or m_K
  // remains; outside the star region it may be non-finite and is discarded
  const double i = div_nr(1.0, S - Ss);
  const double f = m * i;
  const double e = (S - u) * i * E + (Ss - u) * (f * Ss + p * i);
  const double F0 = r * u;
  const double Fk[5] = {F0, F0 * u + p, F0 * a, F0 * b, u * (E + p)};
  const double Uk[5] = {r, r * u, r * a, r * b, E};
  const double Us[5] = {f, f * Ss, f * a, f * b, e};
  double Fn[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) Fn[v] = star ? Fk[v] + S * (Us[v] - Uk[v]) : Fk[v];
  F[0] = Fn[0];
  F[1 + D] = Fn[1];
  F[1 + T1] = Fn[2];
  F[1 + T2] = Fn[3];
  F[4] = Fn[4];
}

// ---------------------------------------------------------------------------
// Stencil window of one face between window cells 2 and 3 (cells f-2 .. f+3
// along the face normal): primitive values q[c][v] (rho,u,v,w,p) and, for the
// four cells f-1 .. f+2, T~ = p/rho and the four tangential velocity
// derivatives the face needs (cell-centred, fourth order):
//   tg[c][0] = d u_D / d x_T1,  tg[c][1] = d u_T1 / d x_T1,
//   tg[c][2] = d u_D / d x_T2,  tg[c][3] = d u_T2 / d x_T2.
struct FaceWindow {
  double q[6][5];
  double T[4];
  double tg[4][4];
  double a;  // Rusanov-NN: the face's alpha
};

// Fourth-order central interpolation to the face between b and c (§3.4).
__host__ __device__ __forceinline__ double rc4(double a, double b, double c, double d) {
  return (-a + 9.0 * b + 9.0 * c - d) / 16.0;
}

// Face values of the four tangential derivatives of a window (same order as
// FaceWindow::tg), interpolated along the normal from cells 1..4.
__host__ __device__ __forceinline__ void face_tangential(const FaceWindow& w, double* tf) {
#pragma unroll
  for (int k = 0; k < 4; ++k) tf[k] = rc4(w.tg[0][k], w.tg[1][k], w.tg[2][k], w.tg[3][k]);
}

// Numerical flux G = F - F^d across the face (§3.3, §3.4) from given
// reconstructed states WL, WR (inviscid part), the window's cells 1..4
// (velocities and T~ for the fourth-order normal derivatives and the face
// velocities) and the face values tf of the tangential derivatives.
// Subtracts the dissipative flux F^d (§3.4) across the face from F: the
// window's cells 1..4 (velocities and T~ for the fourth-order normal
// derivatives and the face velocities) and the face values tf of the
// tangential derivatives.
// The same from the primitives q[0..3] and T~[0..3] of the four cells i-1 ..
// i+2 around the face i+1/2.
template <int D>
__host__ __device__ __forceinline__ void sub_dissipative_q(const Geom& g, const double (*q)[5], const double* T,
                                                           const double* tf, double* F) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  if (g.viscous || g.heat) {
    const double i24 = g.idx[D] * (1.0 / 24.0);
    auto dn = [&](double a, double b, double c, double d) { return (a - 27.0 * b + 27.0 * c - d) * i24; };
    double Fd1 = 0.0, Fd2 = 0.0, Fd3 = 0.0, Fd4 = 0.0;  // slots D, T1, T2 momentum; energy
    if (g.viscous) {
      // normal derivatives of the three velocity components
      const double dD = dn(q[0][1 + D], q[1][1 + D], q[2][1 + D], q[3][1 + D]);
      const double d1 = dn(q[0][1 + T1], q[1][1 + T1], q[2][1 + T1], q[3][1 + T1]);
      const double d2 = dn(q[0][1 + T2], q[1][1 + T2], q[2][1 + T2], q[3][1 + T2]);
      const double uD_t1 = tf[0], u1_t1 = tf[1], uD_t2 = tf[2], u2_t2 = tf[3];
      const double div = dD + u1_t1 + u2_t2;
      const double tDD = g.mu * (dD + dD) - (2.0 / 3.0) * g.mu * div;
      const double tD1 = g.mu * (uD_t1 + d1);
      const double tD2 = g.mu * (uD_t2 + d2);
      const double ufD = rc4(q[0][1 + D], q[1][1 + D], q[2][1 + D], q[3][1 + D]);
      const double uf1 = rc4(q[0][1 + T1], q[1][1 + T1], q[2][1 + T1], q[3][1 + T1]);
      const double uf2 = rc4(q[0][1 + T2], q[1][1 + T2], q[2][1 + T2], q[3][1 + T2]);
      Fd1 = tDD;
      Fd2 = tD1;
      Fd3 = tD2;
      Fd4 = ufD * tDD + uf1 * tD1 + uf2 * tD2;
    }
    if (g.heat) Fd4 += g.kappa * dn(T[0], T[1], T[2], T[3]);
    F[1 + D] -= Fd1;
    F[1 + T1] -= Fd2;
    F[1 + T2] -= Fd3;
    F[4] -= Fd4;
  }
}

template <int D>
__host__ __device__ __forceinline__ void sub_dissipative(const Geom& g, const FaceWindow& w, const double* tf,
                                                         double* F) {
  sub_dissipative_q<D>(g, w.q + 1, w.T, tf, F);
}

template <int D, bool RUS = false, bool NN = false>
__host__ __device__ __forceinline__ void face_flux_lr(const Geom& g, const double* WL, const double* WR,
                                                      const FaceWindow& w, const double* tf, double* G) {
  double F[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (g.inviscid) {
    if constexpr (NN) rusanov<D, true>(g.gamma, g.gm1i, WL, WR, F, w.a);
    else if constexpr (RUS) rusanov<D>(g.gamma, g.gm1i, WL, WR, F);
    else hllc<D>(g.gamma, g.gm1i, WL, WR, F);
  }
  sub_dissipative<D>(g, w, tf, F);
#pragma unroll
  for (int v = 0; v < 5; ++v) G[v] = F[v];
}

// ---------------------------------------------------------------------------
// Flux-splitting approach of §3.3 with the ROE setup of §5: convective flux
// across the face between window cells 2 and 3 (primitives q[0..5] = cells
// f-2 .. f+3). Roe average (sqrt(rho) weights) of cells 2 and 3: velocity u,
// total enthalpy H, sound speed c, c^2 = (gamma-1)(H - |u|^2/2). With
// b = (gamma-1)/c^2 and the waves ordered (u_D - c, entropy, shear T1,
// shear T2, u_D + c), the closed-form left eigenvectors (Toro 2009, §3.2)
// project cell j (velocity v, pressure p) to
//   A   = b (rho |v - u|^2 / 2 + p/(gamma-1)),  S = rho (u_D - v_D) / c,
//   V   = ((A + S)/2, rho - A, rho (v_T1 - u_T1), rho (v_T2 - u_T2), (A - S)/2),
// and, because the Euler flux is F = v_D U + p (0, e_D, v_D), the projected
// flux G = v_D V + p (l_D + l_E v_D) with the left eigenvectors' momentum-D
// and energy entries:
//   G   = v_D V + p (b (v_D - u_D)/2 - 1/(2c), -b (v_D - u_D), 0, 0, b (v_D - u_D)/2 + 1/(2c)).
// Each field is split, G+- = (G +- |lambda| V)/2, reconstructed with WENO5-JS
// (G+ from cells 0..4, G- mirrored from cells 5..1), summed, and transformed
// back with the right eigenvectors (columns (1, u - c e_D, H - u_D c),
// (1, u, |u|^2/2), (0, e_T1, u_T1), (0, e_T2, u_T2), (1, u + c e_D, H + u_D c)).
// No entropy fix (the splitting uses the moduli of the Roe eigenvalues as they are).
template <int D>
__host__ __device__ __forceinline__ void roe_flux(const Geom& g, const double (&q)[6][5], double* F) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const double gm1 = g.gamma - 1.0;
  const double sl = sqrt_pos(q[2][0]), sr = sqrt_pos(q[3][0]);
  const double isum = 1.0 / (sl + sr);
  const double al = sl * isum, ar = sr * isum;
  const double uD = al * q[2][1 + D] + ar * q[3][1 + D];
  const double u1 = al * q[2][1 + T1] + ar * q[3][1 + T1];
  const double u2 = al * q[2][1 + T2] + ar * q[3][1 + T2];
  const double kl = 0.5 * (q[2][1] * q[2][1] + q[2][2] * q[2][2] + q[2][3] * q[2][3]);
  const double kr = 0.5 * (q[3][1] * q[3][1] + q[3][2] * q[3][2] + q[3][3] * q[3][3]);
  const double hp = g.gamma * g.gm1i;  // gamma/(gamma-1): H = hp p/rho + |v|^2/2
  const double H = al * (hp * q[2][4] / q[2][0] + kl) + ar * (hp * q[3][4] / q[3][0] + kr);
  const double q2 = uD * uD + u1 * u1 + u2 * u2;
  const double c2 = gm1 * (H - 0.5 * q2);
  const double c = sqrt_pos(c2);
  const double ic = 1.0 / c;
  const double b = gm1 * ic * ic;
  const double lam[5] = {fabs(uD - c), fabs(uD), fabs(uD), fabs(uD), fabs(uD + c)};
  // per cell: A, S and the pressure terms of the projected fluxes; the fields
  // are then split and reconstructed one at a time (fewer live registers)
  double A[6], S[6], pb[6], pc[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const double rho = q[j][0], p = q[j][4];
    const double dD = q[j][1 + D] - uD, d1 = q[j][1 + T1] - u1, d2 = q[j][1 + T2] - u2;
    A[j] = b * (0.5 * rho * (dD * dD + d1 * d1 + d2 * d2) + p * g.gm1i);
    S[j] = -rho * dD * ic;
    pb[j] = 0.5 * p * b * dD;
    pc[j] = 0.5 * p * ic;
  }
  double Gf[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double Gp[6], Gm[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double rho = q[j][0], vD = q[j][1 + D];
      double V, G;
      if (k == 0) {
        V = 0.5 * (A[j] + S[j]);
        G = vD * V + (pb[j] - pc[j]);
      } else if (k == 1) {
        V = rho - A[j];
        G = vD * V - 2.0 * pb[j];
      } else if (k == 4) {
        V = 0.5 * (A[j] - S[j]);
        G = vD * V + (pb[j] + pc[j]);
      } else {
        V = rho * (k == 2 ? q[j][1 + T1] - u1 : q[j][1 + T2] - u2);
        G = vD * V;
      }
      Gp[j] = 0.5 * (G + lam[k] * V);
      Gm[j] = 0.5 * (G - lam[k] * V);
    }
    Gf[k] = weno5(Gp[0], Gp[1], Gp[2], Gp[3], Gp[4]) + weno5(Gm[5], Gm[4], Gm[3], Gm[2], Gm[1]);
  }
  const double sac = Gf[0] + Gf[4], dac = Gf[4] - Gf[0];
  const double s3 = sac + Gf[1];
  F[0] = s3;
  F[1 + D] = uD * s3 + c * dac;
  F[1 + T1] = u1 * s3 + Gf[2];
  F[1 + T2] = u2 * s3 + Gf[3];
  F[4] = H * sac + uD * c * dac + 0.5 * q2 * Gf[1] + u1 * Gf[2] + u2 * Gf[3];
}

// Numerical flux from the window's primitives and given face tangential
// derivatives tf: WENO5-JS (or WENO5-Z) left and right of the face and HLLC,
// or the Roe flux splitting, then the dissipative flux. The scheme is a
// compile-time choice: a run-time branch between them multiplies the live
// registers of the sweeps.
template <int D, int SCH = SCH_JS>
__host__ __device__ __forceinline__ void face_flux_tf(const Geom& g, const FaceWindow& w, const double* tf,
                                                      double* G) {
  if constexpr (SCH == SCH_ROE) {
    double F[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (g.inviscid) roe_flux<D>(g, w.q, F);
    sub_dissipative<D>(g, w, tf, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) G[v] = F[v];
    return;
  }
  double WL[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, WR[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (g.inviscid) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      if constexpr (sch_weno3(SCH)) {
        WL[v] = weno3(w.q[1][v], w.q[2][v], w.q[3][v]);
        WR[v] = weno3(w.q[4][v], w.q[3][v], w.q[2][v]);
      } else if constexpr (SCH == SCH_Z) {
        WL[v] = weno5z(w.q[0][v], w.q[1][v], w.q[2][v], w.q[3][v], w.q[4][v]);
        WR[v] = weno5z(w.q[5][v], w.q[4][v], w.q[3][v], w.q[2][v], w.q[1][v]);
      } else {
        WL[v] = weno5(w.q[0][v], w.q[1][v], w.q[2][v], w.q[3][v], w.q[4][v]);
        WR[v] = weno5(w.q[5][v], w.q[4][v], w.q[3][v], w.q[2][v], w.q[1][v]);
      }
    }
  }
  face_flux_lr<D, sch_rusanov(SCH), SCH == SCH_W3_NN>(g, WL, WR, w, tf, G);
}

// Reconstructed states of the cell-centred schemes (WENO5-JS and WENO3-JS on
// the primitives; the Roe flux splitting projects per face, and WENO5-Z's
// per-cell form needs more registers than the marches hold, so both stay
// face by face): from the primitives q[0..4] of cells i-2 .. i+2, the left
// state of face i+1/2 (qr) and the right state of face i-1/2 (ql), per
// variable.
template <int SCH>
__host__ __device__ __forceinline__ void recon_pair(const double (*q)[5], double* qr, double* ql) {
  static_assert(SCH != SCH_ROE && SCH != SCH_Z, "face-by-face schemes");
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    if constexpr (sch_weno3(SCH)) weno3_pair(q[1][v], q[2][v], q[3][v], qr[v], ql[v]);
    else weno5_pair(q[0][v], q[1][v], q[2][v], q[3][v], q[4][v], qr[v], ql[v]);
  }
}

// Numerical flux G = F - F^d across face i+1/2 (§3.3, §3.4) from its
// reconstructed states WL, WR, the primitives q[0..3] and T~[0..3] of cells
// i-1 .. i+2, the face values tf of the tangential derivatives and, for the
// Rusanov-NN flux, the face's alpha.
template <int D, int SCH>
__host__ __device__ __forceinline__ void face_flux_states(const Geom& g, const double* WL, const double* WR,
                                                          const double (*q)[5], const double* T, const double* tf,
                                                          double alpha, double* G) {
  double F[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (g.inviscid) {
    if constexpr (SCH == SCH_W3_NN) rusanov<D, true>(g.gamma, g.gm1i, WL, WR, F, alpha);
    else if constexpr (sch_rusanov(SCH)) rusanov<D>(g.gamma, g.gm1i, WL, WR, F);
    else hllc<D>(g.gamma, g.gm1i, WL, WR, F);
  }
  sub_dissipative_q<D>(g, q, T, tf, F);
#pragma unroll
  for (int v = 0; v < 5; ++v) G[v] = F[v];
}

// Numerical flux G = F - F^d across the face (§3.3, §3.4) from a full window.
template <int D, int SCH = SCH_JS>
__host__ __device__ __forceinline__ void face_flux(const Geom& g, const FaceWindow& w, double* G) {
  double tf[4] = {0.0, 0.0, 0.0, 0.0};
  if (g.viscous) face_tangential(w, tf);
  face_flux_tf<D, SCH>(g, w, tf, G);
}

}  // namespace cfd
