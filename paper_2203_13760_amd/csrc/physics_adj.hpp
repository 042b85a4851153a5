// Reverse (adjoint) building blocks of the face flux, hand-derived from the
// forward code in physics.hpp: each routine recomputes the forward
// intermediates of one face and propagates output adjoints back to its inputs
// in reverse order. Branches (the HLLC wave pattern, the Einfeldt min/max)
// follow the decisions of the forward evaluation at the same state.
#pragma once
#include "physics.hpp"

namespace cfd {

// q = weno3(a,b,c); g[0..2] += (dq/d(a,b,c)) * qbar.
__host__ __device__ __forceinline__ void weno3_rev(double a, double b, double c, double qbar, double* g) {
  constexpr double eps = 1.0e-6;
  const double d0 = b - a, d1 = c - b;
  const double e0 = eps + d0 * d0, e1 = eps + d1 * d1;
  const double s0 = e0 * e0, s1 = e1 * e1;
  const double w0 = s1, w1 = 2.0 * s0;
  const double A = 3.0 * b - a, B = b + c;
  const double iD = 1.0 / (2.0 * (w0 + w1));
  const double q = (w0 * A + w1 * B) * iD;
  // reverse
  const double Nb = qbar * iD;
  const double Db = -qbar * q * iD;
  const double w0b = Nb * A + 2.0 * Db, w1b = Nb * B + 2.0 * Db;
  const double Ab = Nb * w0, Bb = Nb * w1;
  const double e0b = 2.0 * e0 * (2.0 * w1b), e1b = 2.0 * e1 * w0b;
  const double d0b = 2.0 * d0 * e0b, d1b = 2.0 * d1 * e1b;
  g[0] += -Ab - d0b;
  g[1] += 3.0 * Ab + Bb + d0b - d1b;
  g[2] += Bb + d1b;
}

// q = weno5(a,b,c,d,e); g[0..4] += (dq/d(a..e)) * qbar.
__host__ __device__ __forceinline__ void weno5_rev(double a, double b, double c, double d, double e,
                                                    double qbar, double* g) {
  constexpr double k13 = 13.0 / 12.0;
  constexpr double eps = 1.0e-6;
  const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
  const double t1 = b - 2.0 * c + d, u1 = b - d;
  const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
  const double e0 = eps + (k13 * t0 * t0 + 0.25 * u0 * u0);
  const double e1 = eps + (k13 * t1 * t1 + 0.25 * u1 * u1);
  const double e2 = eps + (k13 * t2 * t2 + 0.25 * u2 * u2);
  const double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
  const double w0 = 0.1 * (s1 * s2), w1 = 0.6 * (s0 * s2), w2 = 0.3 * (s0 * s1);
  const double P0 = 2.0 * a - 7.0 * b + 11.0 * c;
  const double P1 = -b + 5.0 * c + 2.0 * d;
  const double P2 = 2.0 * c + 5.0 * d - e;
  const double Dn = 6.0 * (w0 + w1 + w2);
  const double iD = 1.0 / Dn;
  const double q = (w0 * P0 + w1 * P1 + w2 * P2) * iD;
  // reverse
  const double Nb = qbar * iD;
  const double Db = -qbar * q * iD;
  const double w0b = Nb * P0 + 6.0 * Db, w1b = Nb * P1 + 6.0 * Db, w2b = Nb * P2 + 6.0 * Db;
  const double P0b = Nb * w0, P1b = Nb * w1, P2b = Nb * w2;
  const double s0b = 0.6 * s2 * w1b + 0.3 * s1 * w2b;
  const double s1b = 0.1 * s2 * w0b + 0.3 * s0 * w2b;
  const double s2b = 0.1 * s1 * w0b + 0.6 * s0 * w1b;
  const double b0b = 2.0 * e0 * s0b, b1b = 2.0 * e1 * s1b, b2b = 2.0 * e2 * s2b;
  const double t0b = 2.0 * k13 * t0 * b0b, u0b = 0.5 * u0 * b0b;
  const double t1b = 2.0 * k13 * t1 * b1b, u1b = 0.5 * u1 * b1b;
  const double t2b = 2.0 * k13 * t2 * b2b, u2b = 0.5 * u2 * b2b;
  g[0] += t0b + u0b + 2.0 * P0b;
  g[1] += -2.0 * t0b - 4.0 * u0b - 7.0 * P0b + t1b + u1b - P1b;
  g[2] += t0b + 3.0 * u0b + 11.0 * P0b - 2.0 * t1b + 5.0 * P1b + t2b + 3.0 * u2b + 2.0 * P2b;
  g[3] += t1b - u1b + 2.0 * P1b - 2.0 * t2b - 4.0 * u2b + 5.0 * P2b;
  g[4] += t2b + u2b - P2b;
}

// Reverse of weno5_pair (both face values of the centre cell c of the stencil
// a..e, sharing the three smoothness indicators): given the adjoints qrb of
// the right-face value qr and qlb of the left-face value ql, g[0..4] +=
// (d qr/d(a..e)) qrb + (d ql/d(a..e)) qlb. With qr = nr / (6 dr) and
// ql = nl / (6 dl), one reciprocal 1/(6 dr dl) serves both, as in the forward.
__host__ __device__ __forceinline__ void weno5_pair_rev(double a, double b, double c, double d, double e,
                                                         double qrb, double qlb, double* g) {
  constexpr double k13 = 13.0 / 12.0;
  constexpr double eps = 1.0e-6;
  // ---- forward recompute (same expressions as weno5_pair)
  const double Db = a - 2.0 * b + c, Dc = b - 2.0 * c + d, Dd = c - 2.0 * d + e;
  const double dm = c - b, dp = d - c;
  const double tL = Db + 2.0 * dm, tC = dm + dp, tR = Dd - 2.0 * dp;
  const double eL = eps + (k13 * Db * Db + 0.25 * tL * tL);
  const double eC = eps + (k13 * Dc * Dc + 0.25 * tC * tC);
  const double eR = eps + (k13 * Dd * Dd + 0.25 * tR * tR);
  const double sL = eL * eL, sC = eC * eC, sR = eR * eR;
  const double pCR = sC * sR, pLR = sL * sR, pLC = sL * sC;
  const double PR0 = 2.0 * a - 7.0 * b + 11.0 * c, PR1 = -b + 5.0 * c + 2.0 * d, PR2 = 2.0 * c + 5.0 * d - e;
  const double PL0 = 2.0 * e - 7.0 * d + 11.0 * c, PL1 = -d + 5.0 * c + 2.0 * b, PL2 = 2.0 * c + 5.0 * b - a;
  const double nr = 0.1 * pCR * PR0 + 0.6 * pLR * PR1 + 0.3 * pLC * PR2;
  const double nl = 0.1 * pLC * PL0 + 0.6 * pLR * PL1 + 0.3 * pCR * PL2;
  const double dr = 0.1 * pCR + 0.6 * pLR + 0.3 * pLC;
  const double dl = 0.1 * pLC + 0.6 * pLR + 0.3 * pCR;
  const double r = div_nr(1.0, 6.0 * (dr * dl));
  const double ir = dl * r, il = dr * r;  // 1/(6 dr), 1/(6 dl)
  // ---- reverse
  const double nrb = qrb * ir, nlb = qlb * il;
  const double drb = -6.0 * (nr * ir) * nrb, dlb = -6.0 * (nl * il) * nlb;  // d(n/(6d))/dd = -q/d
  const double pCRb = 0.1 * PR0 * nrb + 0.3 * PL2 * nlb + 0.1 * drb + 0.3 * dlb;
  const double pLRb = 0.6 * (PR1 * nrb + PL1 * nlb + drb + dlb);
  const double pLCb = 0.3 * PR2 * nrb + 0.1 * PL0 * nlb + 0.3 * drb + 0.1 * dlb;
  const double PR0b = 0.1 * pCR * nrb, PR1b = 0.6 * pLR * nrb, PR2b = 0.3 * pLC * nrb;
  const double PL0b = 0.1 * pLC * nlb, PL1b = 0.6 * pLR * nlb, PL2b = 0.3 * pCR * nlb;
  const double sLb = pLRb * sR + pLCb * sC, sCb = pCRb * sR + pLCb * sL, sRb = pCRb * sC + pLRb * sL;
  const double eLb = 2.0 * eL * sLb, eCb = 2.0 * eC * sCb, eRb = 2.0 * eR * sRb;
  const double tLb = 0.5 * tL * eLb, tCb = 0.5 * tC * eCb, tRb = 0.5 * tR * eRb;
  const double Dbb = 2.0 * k13 * Db * eLb + tLb;
  const double Dcb = 2.0 * k13 * Dc * eCb;
  const double Ddb = 2.0 * k13 * Dd * eRb + tRb;
  const double dmb = 2.0 * tLb + tCb, dpb = tCb - 2.0 * tRb;
  g[0] += Dbb + 2.0 * PR0b - PL2b;
  g[1] += -2.0 * Dbb + Dcb - dmb - 7.0 * PR0b - PR1b + 2.0 * PL1b + 5.0 * PL2b;
  g[2] += Dbb - 2.0 * Dcb + Ddb + dmb - dpb + 11.0 * PR0b + 5.0 * PR1b + 2.0 * PR2b + 11.0 * PL0b + 5.0 * PL1b +
          2.0 * PL2b;
  g[3] += Dcb - 2.0 * Ddb + dpb + 2.0 * PR1b + 5.0 * PR2b - 7.0 * PL0b - PL1b;
  g[4] += Ddb - PR2b + 2.0 * PL0b;
}

// Reverse of hllc<D>: given Fbar (physical slot order) accumulate WLb, WRb
// (physical slot order).
template <int D>
__host__ __device__ __forceinline__ void hllc_rev(double gamma, double gm1i, const double* WL, const double* WR,
                                                   const double* Fbar, double* WLb, double* WRb) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  // ---- forward recompute (same expressions as hllc<D>)
  const double rL = WL[0], uL = WL[1 + D], aL = WL[1 + T1], bL = WL[1 + T2], pL = WL[4];
  const double rR = WR[0], uR = WR[1 + D], aR = WR[1 + T1], bR = WR[1 + T2], pR = WR[4];
  const double EL = pL * gm1i + 0.5 * rL * (uL * uL + aL * aL + bL * bL);
  const double ER = pR * gm1i + 0.5 * rR * (uR * uR + aR * aR + bR * bR);
  const double c2L = div_nr(gamma * pL, rL), c2R = div_nr(gamma * pR, rR);
  const double cL = sqrt_pos(c2L), cR = sqrt_pos(c2R);
  const double sL = sqrt_pos(rL), sR = sqrt_pos(rR);
  const double isum = div_nr(1.0, sL + sR);
  const double ubar = (sL * uL + sR * uR) * isum;
  const double eta2 = 0.5 * sL * sR * isum * isum;
  const double Hs = sL * c2L + sR * c2R;
  const double du = uR - uL;
  const double dbar = sqrt_pos(Hs * isum + eta2 * du * du);
  const double candL1 = uL - cL, candL2 = ubar - dbar;
  const double candR1 = uR + cR, candR2 = ubar + dbar;
  const bool firstL = !(candL2 < candL1);  // fmin keeps the first on ties
  const bool firstR = !(candR2 > candR1);
  const double SL = firstL ? candL1 : candL2;
  const double SR = firstR ? candR1 : candR2;
  const double mL = rL * (SL - uL), mR = rR * (SR - uR);
  const double den = mL - mR;
  const double Ss = div_nr(pR - pL + uL * mL - uR * mR, den);
  const bool useL = 0.0 <= SL;
  const bool useSL = !useL && 0.0 <= Ss;
  const bool useSR = !useL && !useSL && 0.0 < SR;
  const bool useR = !useL && !useSL && !useSR;

  const double Fb[5] = {Fbar[0], Fbar[1 + D], Fbar[1 + T1], Fbar[1 + T2], Fbar[4]};
  // adjoints of the normal-first primitives and intermediates
  double rLb = 0, uLb = 0, aLb = 0, bLb = 0, pLb = 0, ELb = 0;
  double rRb = 0, uRb = 0, aRb = 0, bRb = 0, pRb = 0, ERb = 0;
  double SLb = 0, SRb = 0, Ssb = 0, mLb = 0, mRb = 0;
  {
    // The flux takes one side K: F = F_K (supersonic) or F_K + S_K (U*_K - U_K)
    // (star region). The side's inputs are selected first, so that a
    // wavefront whose faces take different sides runs one reverse, not two.
    const bool left = useL || useSL;
    const bool star = useSL || useSR;
    const double rK = left ? rL : rR, uK = left ? uL : uR, aK = left ? aL : aR, bK = left ? bL : bR;
    const double pK = left ? pL : pR, EK = left ? EL : ER, SK = left ? SL : SR, mK = left ? mL : mR;
    double rKb = 0, uKb = 0, aKb = 0, bKb = 0, pKb = 0, EKb = 0, SKb = 0, mKb = 0;
    double FKb[5];
    for (int v = 0; v < 5; ++v) FKb[v] = Fb[v];
    if (star) {
      const double iK = div_nr(1.0, SK - Ss);
      const double fK = mK * iK;
      const double A = SK - uK, C = Ss - uK, B = fK * Ss + pK * iK;
      const double eK = A * iK * EK + C * B;
      const double UsK[5] = {fK, fK * Ss, fK * aK, fK * bK, eK};
      const double UK[5] = {rK, rK * uK, rK * aK, rK * bK, EK};
      double Usb[5], Ukb[5];
      for (int v = 0; v < 5; ++v) {
        SKb += Fb[v] * (UsK[v] - UK[v]);
        Usb[v] = SK * Fb[v];
        Ukb[v] = -SK * Fb[v];
      }
      double fKb = Usb[0] + Usb[1] * Ss + Usb[2] * aK + Usb[3] * bK;
      Ssb += Usb[1] * fK;
      aKb += Usb[2] * fK;
      bKb += Usb[3] * fK;
      const double eKb = Usb[4];
      const double Ab = eKb * iK * EK;
      double iKb = eKb * A * EK;
      EKb += eKb * A * iK;
      const double Cb = eKb * B, Bb = eKb * C;
      fKb += Bb * Ss;
      Ssb += Bb * fK;
      pKb += Bb * iK;
      iKb += Bb * pK;
      SKb += Ab;
      uKb -= Ab;
      Ssb += Cb;
      uKb -= Cb;
      rKb += Ukb[0] + Ukb[1] * uK + Ukb[2] * aK + Ukb[3] * bK;
      uKb += Ukb[1] * rK;
      aKb += Ukb[2] * rK;
      bKb += Ukb[3] * rK;
      EKb += Ukb[4];
      mKb += fKb * iK;
      iKb += fKb * mK;
      SKb -= iKb * iK * iK;
      Ssb += iKb * iK * iK;
    }
    // physical flux F_K
    {
      const double F0 = rK * uK;
      const double F0b = FKb[0] + FKb[1] * uK + FKb[2] * aK + FKb[3] * bK;
      uKb += FKb[1] * F0 + FKb[4] * (EK + pK);
      aKb += FKb[2] * F0;
      bKb += FKb[3] * F0;
      pKb += FKb[1] + FKb[4] * uK;
      EKb += FKb[4] * uK;
      rKb += F0b * uK;
      uKb += F0b * rK;
    }
    // back to the side's own adjoints
    if (left) {
      rLb = rKb; uLb = uKb; aLb = aKb; bLb = bKb; pLb = pKb; ELb = EKb; SLb = SKb; mLb = mKb;
    } else {
      rRb = rKb; uRb = uKb; aRb = aKb; bRb = bKb; pRb = pKb; ERb = EKb; SRb = SKb; mRb = mKb;
    }
  }
  if (!useL && !useR) {
    // contact speed S* = num / den
    const double iden = div_nr(1.0, den);
    const double numb = Ssb * iden;
    const double denb = -Ssb * Ss * iden;
    pRb += numb;
    pLb -= numb;
    uLb += numb * mL;
    mLb += numb * uL + denb;
    uRb -= numb * mR;
    mRb += -numb * uR - denb;
    // m_K = rho_K (S_K - u_K)
    rLb += mLb * (SL - uL);
    SLb += mLb * rL;
    uLb -= mLb * rL;
    rRb += mRb * (SR - uR);
    SRb += mRb * rR;
    uRb -= mRb * rR;
    // Einfeldt speeds
    double cLb = 0, cRb = 0, ubarb = 0, dbarb = 0;
    if (firstL) { uLb += SLb; cLb -= SLb; } else { ubarb += SLb; dbarb -= SLb; }
    if (firstR) { uRb += SRb; cRb += SRb; } else { ubarb += SRb; dbarb += SRb; }
    const double dbar2b = div_nr(0.5 * dbarb, dbar);
    const double Hsb = dbar2b * isum;
    double isumb = dbar2b * Hs;
    const double eta2b = dbar2b * du * du;
    const double dub = dbar2b * eta2 * 2.0 * du;
    double sLb = Hsb * c2L, sRb = Hsb * c2R;
    double c2Lb = Hsb * sL, c2Rb = Hsb * sR;
    uRb += dub;
    uLb -= dub;
    sLb += eta2b * 0.5 * sR * isum * isum;
    sRb += eta2b * 0.5 * sL * isum * isum;
    isumb += eta2b * sL * sR * isum;
    const double Nu = sL * uL + sR * uR;
    const double Nub = ubarb * isum;
    isumb += ubarb * Nu;
    sLb += Nub * uL;
    uLb += Nub * sL;
    sRb += Nub * uR;
    uRb += Nub * sR;
    const double sumb = -isumb * isum * isum;
    sLb += sumb;
    sRb += sumb;
    // 1/sqrt(r) = sqrt(r)/r: one reciprocal of rho per side serves the
    // square-root and sound-speed terms
    const double irL = div_nr(1.0, rL), irR = div_nr(1.0, rR);
    rLb += 0.5 * sLb * sL * irL;
    rRb += 0.5 * sRb * sR * irR;
    c2Lb += div_nr(0.5 * cLb, cL);
    c2Rb += div_nr(0.5 * cRb, cR);
    pLb += c2Lb * gamma * irL;
    rLb -= c2Lb * c2L * irL;
    pRb += c2Rb * gamma * irR;
    rRb -= c2Rb * c2R * irR;
  }
  // total energies
  pLb += ELb * gm1i;
  rLb += ELb * 0.5 * (uL * uL + aL * aL + bL * bL);
  uLb += ELb * rL * uL;
  aLb += ELb * rL * aL;
  bLb += ELb * rL * bL;
  pRb += ERb * gm1i;
  rRb += ERb * 0.5 * (uR * uR + aR * aR + bR * bR);
  uRb += ERb * rR * uR;
  aRb += ERb * rR * aR;
  bRb += ERb * rR * bR;
  WLb[0] += rLb;
  WLb[1 + D] += uLb;
  WLb[1 + T1] += aLb;
  WLb[1 + T2] += bLb;
  WLb[4] += pLb;
  WRb[0] += rRb;
  WRb[1 + D] += uRb;
  WRb[1 + T1] += aRb;
  WRb[1 + T2] += bRb;
  WRb[4] += pRb;
}

// Adjoint of the face window, accumulated in arrays (used by host checks):
// qb[6][6] holds (rho,u,v,w,p,T~) of the six window cells, tgb[4][4] the
// tangential-derivative inputs of window cells 1..4.
struct FaceWindowAdj {
  double qb[6][6];
  double tgb[4][4];
  __host__ __device__ void q(int m, int v, double x) { qb[m][v] += x; }
  __host__ __device__ void tg(int m, int k, double x) { tgb[m][k] += x; }
};

// Reverse of face_flux<D>: given Gbar (physical slot order) hand the adjoints
// of the window inputs to the sink as they become final:
// sink.q(cell m, variable v, value) with v in 0..5 = (rho,u,v,w,p,T~), and
// sink.tg(cell m in 1..4, input k, value).
template <int D, class Sink>
__host__ __device__ __forceinline__ void face_flux_rev(const Geom& g, const FaceWindow& w, const double* Gbar,
                                                        Sink& sink) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  if (g.inviscid) {
    double WL[5], WR[5];
    for (int v = 0; v < 5; ++v) {
      WL[v] = weno5(w.q[0][v], w.q[1][v], w.q[2][v], w.q[3][v], w.q[4][v]);
      WR[v] = weno5(w.q[5][v], w.q[4][v], w.q[3][v], w.q[2][v], w.q[1][v]);
    }
    double WLb[5] = {0, 0, 0, 0, 0}, WRb[5] = {0, 0, 0, 0, 0};
    hllc_rev<D>(g.gamma, g.gm1i, WL, WR, Gbar, WLb, WRb);
    for (int v = 0; v < 5; ++v) {
      double gs[6] = {0, 0, 0, 0, 0, 0};
      weno5_rev(w.q[0][v], w.q[1][v], w.q[2][v], w.q[3][v], w.q[4][v], WLb[v], gs);
      double gr[5] = {0, 0, 0, 0, 0};
      weno5_rev(w.q[5][v], w.q[4][v], w.q[3][v], w.q[2][v], w.q[1][v], WRb[v], gr);
      for (int m = 0; m < 5; ++m) gs[5 - m] += gr[m];
      for (int m = 0; m < 6; ++m) sink.q(m, v, gs[m]);
    }
  }
  if (g.viscous || g.heat) {
    const double i24 = g.idx[D] / 24.0;
    const double cdn[4] = {i24, -27.0 * i24, 27.0 * i24, -i24};                   // normal derivative weights
    const double crc[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};  // face interpolation weights
    // G slots carry -F^d
    const double Fd1b = -Gbar[1 + D], Fd2b = -Gbar[1 + T1], Fd3b = -Gbar[1 + T2], Fd4b = -Gbar[4];
    if (g.heat)
      for (int m = 0; m < 4; ++m) sink.q(1 + m, 5, g.kappa * Fd4b * cdn[m]);
    if (g.viscous) {
      auto dn = [&](int v) {
        return cdn[0] * w.q[1][v] + cdn[1] * w.q[2][v] + cdn[2] * w.q[3][v] + cdn[3] * w.q[4][v];
      };
      auto rc = [&](int v) { return crc[0] * w.q[1][v] + crc[1] * w.q[2][v] + crc[2] * w.q[3][v] + crc[3] * w.q[4][v]; };
      auto rct = [&](int k) { return crc[0] * w.tg[0][k] + crc[1] * w.tg[1][k] + crc[2] * w.tg[2][k] + crc[3] * w.tg[3][k]; };
      const double dD = dn(1 + D), d1 = dn(1 + T1), d2 = dn(1 + T2);
      const double uD_t1 = rct(0), u1_t1 = rct(1), uD_t2 = rct(2), u2_t2 = rct(3);
      const double div = dD + u1_t1 + u2_t2;
      const double tDD = g.mu * (dD + dD) - (2.0 / 3.0) * g.mu * div;
      const double tD1 = g.mu * (uD_t1 + d1);
      const double tD2 = g.mu * (uD_t2 + d2);
      const double ufD = rc(1 + D), uf1 = rc(1 + T1), uf2 = rc(1 + T2);
      const double tDDb = Fd1b + Fd4b * ufD;
      const double tD1b = Fd2b + Fd4b * uf1;
      const double tD2b = Fd3b + Fd4b * uf2;
      const double ufDb = Fd4b * tDD, uf1b = Fd4b * tD1, uf2b = Fd4b * tD2;
      const double divb = -(2.0 / 3.0) * g.mu * tDDb;
      const double dDb = 2.0 * g.mu * tDDb + divb;
      const double d1b = g.mu * tD1b, d2b = g.mu * tD2b;
      const double tgb[4] = {g.mu * tD1b, divb, g.mu * tD2b, divb};
      for (int m = 0; m < 4; ++m) {
        sink.q(1 + m, 1 + D, cdn[m] * dDb + crc[m] * ufDb);
        sink.q(1 + m, 1 + T1, cdn[m] * d1b + crc[m] * uf1b);
        sink.q(1 + m, 1 + T2, cdn[m] * d2b + crc[m] * uf2b);
        for (int k = 0; k < 4; ++k) sink.tg(1 + m, k, crc[m] * tgb[k]);
      }
    }
  }
}

}  // namespace cfd
