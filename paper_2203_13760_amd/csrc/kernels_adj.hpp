// Discrete adjoint of the right-hand side (gfx950).
//
//   1. the primitives P at the state (the forward kernels, or the buffers a
//      forward recompute of the stages leaves);
//   2. the face reverses: the face flux adjoint follows from Rbar
//      (R_i = -(G_{i+1/2} - G_{i-1/2})/dx gives Gbar_{i+1/2} =
//      (Rbar_{i+1} - Rbar_i)/dx); each face recomputes its forward flux and
//      reverses it (physics_adj.hpp), and its contributions go to Wbar
//      (rho,u,v,w,p,T~ of the stencil cells) and Dbar (the adjoints of the
//      centred derivatives) with hardware FP64 atomics. x faces
//      (k_face_adj_inv/dis<0>): one lane per face, the lanes of a wavefront
//      holding consecutive faces of a row, contributions summed per cell by
//      shuffles (one atomic per cell and variable). y and z faces
//      (k_march_adj_inv/dis): marching wavefronts, the reverse of the forward
//      marches. The inviscid and dissipative reverses run on two streams;
//   3. k_adj_dbar (viscous): the transposed centred differences of Dbar,
//      added to Wbar at every padded cell;
//   4. k_adj_halo: the transposed halo fill, every halo cell's Wbar added to
//      its interior source cell;
//   5. k_adj_fold: per interior cell, the transposed primitive map at U gives
//      Ubar.
// The atomics make the summation order, and so the last bits, vary between
// runs; everything else is deterministic.
#pragma once
#include "kernels_fwd.hpp"
#include "physics_adj.hpp"

namespace cfd {

__device__ __forceinline__ void atomic_add(double* p, double v) {
  if (v != 0.0) unsafeAtomicAdd(p, v);
}

// Face numbering for axis D: face f in [0, n_D] lies between cells f-1 and f.
// D = 0: f runs fastest, so the lanes of a wavefront hold consecutive faces of
// a row (col = the row) and also load consecutive cells; D = 1, 2: x runs
// fastest so that lanes load consecutive cells (col = -1: no two lanes of a
// wavefront share a column).
template <int D>
__device__ __forceinline__ bool face_coords(const Geom& g, int t, int& i, int& j, int& k, int& f, int& col) {
  if (D == 0) {
    const int F = g.n[0] + 1;
    col = t / F;
    f = t - col * F;
    k = col / g.n[1];
    j = col - k * g.n[1];
    i = f;
    return k < g.n[2];
  } else if (D == 1) {
    const int F = g.n[1] + 1;
    const int r = t / g.n[0];
    i = t - r * g.n[0];
    k = r / F;
    f = r - k * F;
    j = f;
    col = -1;
    return k < g.n[2];
  } else {
    const int r = t / g.n[0];
    i = t - r * g.n[0];
    f = r / g.n[1];
    j = r - f * g.n[1];
    k = f;
    col = -1;
    return f <= g.n[2];
  }
}

// Summation across a wavefront whose lanes hold consecutive faces of rows.
// A lane's contribution to cell f + d of its row (d in -3..2) belongs to the
// lane holding face f + d of the same row (the cell's "owner"); the owner adds
// up what it receives and adds the total to memory with one atomic. A
// contribution whose owner is not in the wavefront (row ends, wavefront edges,
// halo cells) is added to memory by its lane directly.
struct LaneSum {
  int lane;
  int key;            // column of a lane with a face, -2 without a face
  bool sent[6];       // offset d = idx - 3: the owner lane + d exists
  bool got[6];        //                     the lane - d exists (sends to me)

  // has: the lane holds a face; col: its column, or -1 when the lanes of the
  // wavefront hold faces of different columns (every contribution but the
  // lane's own cell is then added directly)
  __device__ __forceinline__ void init(int lane_, bool has, int col) {
    lane = lane_;
    key = has ? col : -2;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int d = e - 3;
      const int dst = lane + d, src = lane - d;
      const int kd = __shfl(key, dst & 63, 64), ks = __shfl(key, src & 63, 64);
      if (d == 0) {
        sent[e] = got[e] = has;
      } else {
        sent[e] = has && col >= 0 && dst >= 0 && dst < 64 && kd == key;
        got[e] = has && col >= 0 && src >= 0 && src < 64 && ks == key;
      }
    }
  }
  // Contribution x to cell f + d (address addr): returns the share this lane
  // collects as owner from lane - d; adds x to memory when no owner exists.
  __device__ __forceinline__ double pass(double x, int d, double* addr) const {
    const int e = d + 3;
    const double y = __shfl(x, (lane - d) & 63, 64);
    if (key != -2 && !sent[e]) atomic_add(addr, x);
    return got[e] ? y : 0.0;
  }
};
// Face adjoint Gbar from Rbar (read as rscale * Rbar, interior cells only).
template <int D>
__device__ __forceinline__ bool face_gbar(const Geom& g, const double* __restrict__ Rbar, double rscale, long long cf,
                                          int f, double* Gb) {
  const long long st = g.s[D];
  const bool hasL = f >= 1, hasR = f < g.n[D];
  double any = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double rl = hasL ? Rbar[v * g.vs + cf - st] : 0.0;
    const double rr = hasR ? Rbar[v * g.vs + cf] : 0.0;
    Gb[v] = rscale * (rr - rl) * g.idx[D];
    any += fabs(Gb[v]);
  }
  return any != 0.0;
}

// Inviscid part of the face adjoint: WENO5-JS forward, HLLC reverse, then the
// WENO reverse one variable at a time with that variable's stencil reloaded,
// so the window is not held in registers across the HLLC reverse. Every lane
// takes part in the shuffles; lanes without a face (or with a zero face
// adjoint) contribute zeros.
template <int D>
__global__ void __launch_bounds__(kBlock) k_face_adj_inv(const double* P, const double* __restrict__ Rbar,
                                                         double rscale, double* Wbar, Geom g) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int i = 0, j = 0, k = 0, f = 0, col = 0;
  const bool has = face_coords<D>(g, t, i, j, k, f, col);
  if (!has) i = j = k = f = 0;  // a valid cell for the (unused) address arithmetic
  LaneSum ls;
  ls.init(threadIdx.x & 63, has, col);
  const long long st = g.s[D];
  const long long cf = cell_at(g, i, j, k);  // cell f: the face lies between f-1 and f
  const long long c0 = cf - 3 * st;          // window cell 0 = cell f-3
  double Gb[5] = {0, 0, 0, 0, 0};
  const bool active = has && face_gbar<D>(g, Rbar, rscale, cf, f, Gb);
  double WLb[5] = {0, 0, 0, 0, 0}, WRb[5] = {0, 0, 0, 0, 0};
  if (active) {
    double WL[5], WR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double* q = P + v * g.vs + c0;
      const double q0 = q[0], q1 = q[st], q2 = q[2 * st], q3 = q[3 * st], q4 = q[4 * st], q5 = q[5 * st];
      WL[v] = weno5(q0, q1, q2, q3, q4);
      WR[v] = weno5(q5, q4, q3, q2, q1);
    }
    hllc_rev<D>(g.gamma, g.gm1i, WL, WR, Gb, WLb, WRb);
  }
  asm volatile("" ::: "memory");  // reload the stencils below instead of keeping them live
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double gs[6] = {0, 0, 0, 0, 0, 0};
    if (active) {
      const double* q = P + v * g.vs + c0;
      const double q0 = q[0], q1 = q[st], q2 = q[2 * st], q3 = q[3 * st], q4 = q[4 * st], q5 = q[5 * st];
      weno5_rev(q0, q1, q2, q3, q4, WLb[v], gs);
      double gr[5] = {0, 0, 0, 0, 0};
      weno5_rev(q5, q4, q3, q2, q1, WRb[v], gr);
#pragma unroll
      for (int m = 0; m < 5; ++m) gs[5 - m] += gr[m];
    }
    double* wv = Wbar + v * g.vs + c0;
    double own = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) own += ls.pass(gs[m], m - 3, wv + m * st);
    if (has) atomic_add(wv + 3 * st, own);
  }
}

// Dissipative part of the face adjoint (viscous and heat flux).
// The cell-centred tangential derivatives are formed from P as in the forward
// sweeps; their adjoints go to Dbar and are transposed in k_adj_fold. The
// window's adjoints (cells 1..4: u, v, w, T~ and the four derivative inputs)
// are collected in registers, then summed across the wavefront.
template <int D>
__global__ void __launch_bounds__(kBlock) k_face_adj_dis(const double* __restrict__ P,
                                                         const double* __restrict__ Rbar, double rscale,
                                                         double* Wbar, double* Dbar, Geom g) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  int i = 0, j = 0, k = 0, f = 0, col = 0;
  const bool has = face_coords<D>(g, t, i, j, k, f, col);
  if (!has) i = j = k = f = 0;
  LaneSum ls;
  ls.init(threadIdx.x & 63, has, col);
  const long long st = g.s[D];
  const long long cf = cell_at(g, i, j, k);
  const long long c0 = cf - 3 * st;
  double Gb[5] = {0, 0, 0, 0, 0};
  const bool active = has && face_gbar<D>(g, Rbar, rscale, cf, f, Gb);
  struct RegSink {
    double qb[4][4];   // window cells 1..4: u, v, w, T~
    double tgb[4][4];  // window cells 1..4: derivative inputs
    __device__ void q(int m, int v, double x) { qb[m - 1][v == 5 ? 3 : v - 1] += x; }
    __device__ void tg(int m, int kk, double x) { tgb[m - 1][kk] += x; }
  } sink;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) sink.qb[m][v] = sink.tgb[m][v] = 0.0;
  if (active) {
    FaceWindow w;
#pragma unroll
    for (int m = 1; m < 5; ++m)
#pragma unroll
      for (int v = 1; v < 4; ++v) w.q[m][v] = P[v * g.vs + c0 + m * st];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      w.T[m] = P[5 * g.vs + c0 + (1 + m) * st];
      if (g.viscous) tangential_at<D>(g, P, c0 + (1 + m) * st, w.tg[m]);
    }
    Geom gd = g;
    gd.inviscid = 0;  // the inviscid part is k_face_adj_inv
    face_flux_rev<D>(gd, w, Gb, sink);
  }
  // window cell m (1..4) is cell f + (m - 3)
  const int wslot[4] = {1, 2, 3, 5};  // u, v, w, T~ in Wbar
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (v == 3 && !g.heat) continue;
    if (v < 3 && !g.viscous) continue;
    double* wv = Wbar + wslot[v] * g.vs + c0;
    double own = 0.0;
#pragma unroll
    for (int m = 1; m < 5; ++m) own += ls.pass(sink.qb[m - 1][v], m - 3, wv + m * st);
    if (has) atomic_add(wv + 3 * st, own);
  }
  if (g.viscous) {
    const int comp[4] = {D * 3 + T1, T1 * 3 + T1, D * 3 + T2, T2 * 3 + T2};
    const bool act[4] = {g.act[T1] != 0, g.act[T1] != 0, g.act[T2] != 0, g.act[T2] != 0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (!act[kk]) continue;
      double* dv = Dbar + comp[kk] * g.vs + c0;
      double own = 0.0;
#pragma unroll
      for (int m = 1; m < 5; ++m) own += ls.pass(sink.tgb[m - 1][kk], m - 3, dv + m * st);
      if (has) atomic_add(dv + 3 * st, own);
    }
  }
}

// ---------------------------------------------------------------------------
// Marching face reverses along y and z (AX = 1, 2), the reverse counterparts
// of the forward marches: a wavefront holds 64 consecutive x of one column
// (other transverse coordinate, segment of g.seg cells along AX) and walks
// its faces in order, keeping the stencil window in registers, so every cell
// of the column is loaded once per segment instead of once per face that
// touches it, and a cell's adjoint is added to memory once, when the last
// face of the segment that touches it is done (one atomic per cell and
// variable; a cell near a segment end gets a share from each of the two
// segments). Launch shape: sweep_march_blocks<AX>.

// Column, segment and first/last face of the marching wavefront; false for a
// lane without a column. The segment of cells [s0, s1) owns faces s0 .. s1-1,
// and the last segment also face n (the upper boundary).
template <int AX>
__device__ __forceinline__ bool march_adj_column(const Geom& g, int& i, int& o, int& s0, int& fe) {
  constexpr int OT = AX == 1 ? 2 : 1;
  const int logical = xcd_major_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int by = logical / gridDim.x, bx = logical - by * gridDim.x;
  i = bx * 64 + (threadIdx.x & 63);
  const int sl = g.seg;
  const int nseg = (g.n[AX] + sl - 1) / sl;
  const long long col = (long long)by * (kBlock >> 6) + (threadIdx.x >> 6);
  if (i >= g.n[0] || col >= (long long)g.n[OT] * nseg) return false;
  o = (int)(col / nseg);
  const int seg = (int)(col - (long long)o * nseg);
  s0 = seg * sl;
  const int s1 = min(s0 + sl, g.n[AX]);
  fe = s1 == g.n[AX] ? s1 : s1 - 1;
  return true;
}

template <int AX>
__device__ __forceinline__ long long march_adj_cell(const Geom& g, int i, int o, int a) {
  return AX == 1 ? cell_at(g, i, a, o) : cell_at(g, i, o, a);
}

// Inviscid part. Face f (between cells f-1 and f) takes its left state from
// the reconstruction pair of cell f-1 and its right state from that of cell
// f (§3.3): the wavefront computes the pair of cell f at face f, reverses the
// HLLC flux of face f, and then reverses the pair of cell f-1, whose two
// cotangents (from faces f-1 and f) are both known, into cells f-3 .. f+1.
// The window holds cells f-3 .. f+2; the per-cell adjoint sums of the five
// cells a pair reverse touches live in a lane-private LDS ring (the register
// file holds the window and the HLLC reverse). A pair shared with the
// neighbouring segment is reversed in both, each with its own face's share of
// the cotangent (the reverse is linear in it). The window, the HLLC reverse
// and the carried states need about 380 registers: the kernel runs one
// wavefront per SIMD (at two it spills, and ran 1.8x slower).
constexpr int kMarchRing = 5;

template <int AX>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1)))
k_march_adj_inv(const double* __restrict__ P, const double* __restrict__ Rbar, double rscale, double* Wbar,
                Geom g) {
  __shared__ double ring[kMarchRing * 5 * kBlock];
  int i, o, s0, fe;
  if (!march_adj_column<AX>(g, i, o, s0, fe)) return;
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < kMarchRing * 5; ++e) ring[e * kBlock + tid] = 0.0;
  const long long st = g.s[AX], vs = g.vs;
  const int n = g.n[AX];
  const double gs_scale = rscale * g.idx[AX];
  long long c = march_adj_cell<AX>(g, i, o, s0 - 3);  // window cell 0: cell f-3 of face f = s0
  double w[6][5];
#pragma unroll
  for (int m = 0; m < 6; ++m) load_prims(P, vs, c + m * st, w[m]);
  double WLc[5], WRbc[5], rl[5];
  {
    double unused[5];
    double q[5][5];
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) q[m][v] = w[m][v];
    recon_pair<SCH_JS>(q, WLc, unused);  // cell s0-1: left state of face s0
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    WRbc[v] = 0.0;  // face s0-1 belongs to the previous segment
    rl[v] = s0 >= 1 ? Rbar[v * vs + c + 2 * st] : 0.0;
  }
  int r0 = 0;  // ring slot of window cell 0
  for (int f = s0; f <= fe; ++f) {
    const bool more = f < fe;
    double nq[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, rr[5];
    if (more) load_prims(P, vs, c + 6 * st, nq);
#pragma unroll
    for (int v = 0; v < 5; ++v) rr[v] = f < n ? Rbar[v * vs + c + 3 * st] : 0.0;
    double Gb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Gb[v] = gs_scale * (rr[v] - rl[v]);
    // pair of cell f (window cells 1..5): left state of face f+1, right state of face f
    double nWL[5], WR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) weno5_pair(w[1][v], w[2][v], w[3][v], w[4][v], w[5][v], nWL[v], WR[v]);
    double WLb[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, WRb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    hllc_rev<AX>(g.gamma, g.gm1i, WLc, WR, Gb, WLb, WRb);
    // pair of cell f-1 (window cells 0..4) with the cotangents of faces f and f-1
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double gq[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      weno5_pair_rev(w[0][v], w[1][v], w[2][v], w[3][v], w[4][v], WLb[v], WRbc[v], gq);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int slot = r0 + m < kMarchRing ? r0 + m : r0 + m - kMarchRing;
        ring[(slot * 5 + v) * kBlock + tid] += gq[m];
      }
    }
    // cell f-3 is complete for this segment
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      double& a = ring[(r0 * 5 + v) * kBlock + tid];
      atomic_add(Wbar + v * vs + c, a);
      a = 0.0;
    }
    r0 = r0 + 1 < kMarchRing ? r0 + 1 : 0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
#pragma unroll
      for (int m = 0; m < 5; ++m) w[m][v] = w[m + 1][v];
      w[5][v] = nq[v];
      WLc[v] = nWL[v];
      WRbc[v] = WRb[v];
      rl[v] = rr[v];
    }
    c += st;
  }
  // the pair of cell fe (window cells 0..4) with the cotangent of face fe only
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double gq[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    weno5_pair_rev(w[0][v], w[1][v], w[2][v], w[3][v], w[4][v], 0.0, WRbc[v], gq);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const int slot = r0 + m < kMarchRing ? r0 + m : r0 + m - kMarchRing;
      atomic_add(Wbar + v * vs + c + m * st, ring[(slot * 5 + v) * kBlock + tid] + gq[m]);
    }
  }
}

// Dissipative part (viscous and heat flux). Face f reads window cells
// f-2 .. f+1 (u, v, w, T~ and the four tangential-derivative inputs of each,
// formed from P as in the forward marches); the adjoints of those inputs
// (Wbar u, v, w, T~ and Dbar) are summed in registers and cell f-2 is added
// to memory after face f.
template <int AX>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_march_adj_dis(const double* __restrict__ P, const double* __restrict__ Rbar, double rscale, double* Wbar,
                double* Dbar, Geom g) {
  constexpr int T1 = (AX + 1) % 3, T2 = (AX + 2) % 3;
  int i, o, s0, fe;
  if (!march_adj_column<AX>(g, i, o, s0, fe)) return;
  const long long st = g.s[AX], vs = g.vs;
  const int n = g.n[AX];
  const double gs_scale = rscale * g.idx[AX];
  Geom gd = g;
  gd.inviscid = 0;  // the inviscid part is k_march_adj_inv
  long long c = march_adj_cell<AX>(g, i, o, s0 - 2);  // window cell 0: cell f-2 of face f = s0
  // q[1..4] (u, v, w) and tg[0..3]: cells f-2 .. f+1. The heat flux is
  // linear in T~, so its reverse needs no T~ values.
  FaceWindow win;
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int v = 0; v < 5; ++v) win.q[m][v] = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    win.T[m] = 0.0;
#pragma unroll
    for (int v = 1; v < 4; ++v) win.q[1 + m][v] = g.viscous ? P[v * vs + c + m * st] : 0.0;
    if (g.viscous) tangential_at<AX>(g, P, c + m * st, win.tg[m]);
    else
#pragma unroll
      for (int k = 0; k < 4; ++k) win.tg[m][k] = 0.0;
  }
  struct RegSink {
    double qb[4][4];   // window cells 0..3: u, v, w, T~
    double tgb[4][4];  // window cells 0..3: derivative inputs
    __device__ void q(int m, int v, double x) { qb[m - 1][v == 5 ? 3 : v - 1] += x; }
    __device__ void tg(int m, int k, double x) { tgb[m - 1][k] += x; }
  } sink;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) sink.qb[m][v] = sink.tgb[m][v] = 0.0;
  double rl[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) rl[v] = s0 >= 1 ? Rbar[v * vs + c + st] : 0.0;
  const int wslot[4] = {1, 2, 3, 5};  // u, v, w, T~ in Wbar
  const int comp[4] = {AX * 3 + T1, T1 * 3 + T1, AX * 3 + T2, T2 * 3 + T2};
  const bool tact[4] = {g.act[T1] != 0, g.act[T1] != 0, g.act[T2] != 0, g.act[T2] != 0};
  for (int f = s0; f <= fe; ++f) {
    const bool more = f < fe;
    double nq[3] = {0.0, 0.0, 0.0}, ntr[4][4], rr[5];
    if (more && g.viscous) {
#pragma unroll
      for (int v = 1; v < 4; ++v) nq[v - 1] = P[v * vs + c + 4 * st];
      tangential_load<AX>(g, P, c + 4 * st, ntr);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) rr[v] = f < n ? Rbar[v * vs + c + 2 * st] : 0.0;
    double Gb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Gb[v] = gs_scale * (rr[v] - rl[v]);
    face_flux_rev<AX>(gd, win, Gb, sink);
    // cell f-2 is complete for this segment
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (v == 3 ? g.heat : g.viscous) atomic_add(Wbar + wslot[v] * vs + c, sink.qb[0][v]);
    }
    if (g.viscous) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (tact[k]) atomic_add(Dbar + comp[k] * vs + c, sink.tgb[0][k]);
    }
    double ntg[4] = {0.0, 0.0, 0.0, 0.0};
    if (more && g.viscous) tangential_combine<AX>(g, ntr, ntg);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sink.qb[m][v] = sink.qb[m + 1][v];
        sink.tgb[m][v] = sink.tgb[m + 1][v];
        win.tg[m][v] = win.tg[m + 1][v];
      }
#pragma unroll
      for (int v = 1; v < 4; ++v) win.q[1 + m][v] = win.q[2 + m][v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sink.qb[3][v] = sink.tgb[3][v] = 0.0;
      win.tg[3][v] = ntg[v];
    }
#pragma unroll
    for (int v = 1; v < 4; ++v) win.q[4][v] = nq[v - 1];
#pragma unroll
    for (int v = 0; v < 5; ++v) rl[v] = rr[v];
    c += st;
  }
  // cells fe-1 .. fe+1 (window cells 0..2) hold the rest of this segment's sums
#pragma unroll
  for (int m = 0; m < 3; ++m) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (v == 3 ? g.heat : g.viscous) atomic_add(Wbar + wslot[v] * vs + c + m * st, sink.qb[m][v]);
    }
    if (g.viscous) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (tact[k]) atomic_add(Dbar + comp[k] * vs + c + m * st, sink.tgb[m][k]);
    }
  }
}

// Transposed centred differences of Dbar at padded cell cc (coordinates q),
// added to wb[1..3]: phi_bar(m) += (Dbar(m+2) - 8 Dbar(m+1) + 8 Dbar(m-1) -
// Dbar(m-2)) / (12 dx_t). CHECK selects the range checks a halo image needs;
// an interior cell's +-2 neighbours always lie inside the padded block.
template <bool CHECK>
__device__ __forceinline__ void fold_dbar(const Geom& g, const double* __restrict__ Dbar, long long cc,
                                          const int* q, double* wb) {
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (!g.act[t]) continue;
    const long long st = g.s[t];
    const int lo = -g.h[t], hi = g.n[t] + g.h[t];
    const int y = q[t];
    const double i12 = g.idx[t] / 12.0;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const double* Db = Dbar + (comp * 3 + t) * g.vs + cc;
      double acc = 0.0;
      if (!CHECK || y + 2 < hi) acc += Db[2 * st];
      if (!CHECK || y + 1 < hi) acc -= 8.0 * Db[st];
      if (!CHECK || y - 1 >= lo) acc += 8.0 * Db[-st];
      if (!CHECK || y - 2 >= lo) acc -= Db[-2 * st];
      wb[1 + comp] += acc * i12;
    }
  }
}

// Transposed centred differences of Dbar, for every padded cell c:
// Wbar(u, v, w)[c] += the adjoint the tangential derivatives give c. Every
// padded cell is the image of exactly one interior cell, so after this pass
// the fold only sums Wbar over images. Each thread updates its own cell.
__global__ void __launch_bounds__(kBlock) k_adj_dbar(const double* __restrict__ Dbar, double* __restrict__ Wbar,
                                                     Geom g) {
  const PlaneIdx p = plane_index(g, true);
  if (!p.in) return;
  const int q[3] = {p.i, p.j, p.k};
  double wb[4] = {0.0, 0.0, 0.0, 0.0};
  fold_dbar<true>(g, Dbar, p.c, q, wb);
#pragma unroll
  for (int c = 1; c < 4; ++c) Wbar[c * g.vs + p.c] += wb[c];
}

// Transposed halo fill of the primitive adjoints: every halo cell adds its
// adjoint to its interior source cell (the wall-normal velocity's through the
// image's sign at a reflecting wall), with atomics, since an edge cell can
// own several halo cells. One thread per halo cell, numbered as in the
// primitive halo refresh.
__global__ void __launch_bounds__(kBlock) k_adj_halo(double* Wbar, Geom g) {
  int i, j, k;
  if (!halo_cell(g, (long long)blockIdx.x * kBlock + threadIdx.x, i, j, k)) return;
  const int si = bc_source(i, g.n[0], g.bc[0], g.bc[1]);
  const int sj = bc_source(j, g.n[1], g.bc[2], g.bc[3]);
  const int sk = bc_source(k, g.n[2], g.bc[4], g.bc[5]);
  const long long c = cell_at(g, i, j, k), s = cell_at(g, si, sj, sk);
  const double f[6] = {1.0, bc_sign(i, g.n[0], g.bc[0], g.bc[1]), bc_sign(j, g.n[1], g.bc[2], g.bc[3]),
                       bc_sign(k, g.n[2], g.bc[4], g.bc[5]), 1.0, 1.0};
#pragma unroll
  for (int v = 0; v < 6; ++v) atomic_add(Wbar + v * g.vs + s, f[v] * Wbar[v * g.vs + c]);
}

// Per interior cell s, after k_adj_halo (and, with viscous fluxes,
// k_adj_dbar): the transposed primitive map at U[s] applied to Wbar[s];
// Ubar[s] += result. Halo entries of Ubar are not touched.
__global__ void __launch_bounds__(kBlock) k_adj_fold(const double* __restrict__ U, const double* __restrict__ Wbar,
                                                     double* __restrict__ Ubar, Geom g) {
  const PlaneIdx p = plane_index(g, true);
  if (!p.in || p.i < 0 || p.i >= g.n[0] || p.j < 0 || p.j >= g.n[1] || p.k < 0 || p.k >= g.n[2]) return;
  double wb[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) wb[v] = Wbar[v * g.vs + p.c];
  // transposed primitive map at U[s]
  const long long s = p.c;
  const double rho = U[s], m0 = U[g.vs + s], m1 = U[2 * g.vs + s], m2 = U[3 * g.vs + s], E = U[4 * g.vs + s];
  const double ir = 1.0 / rho;
  const double u[3] = {m0 * ir, m1 * ir, m2 * ir};
  const double gm1 = g.gamma - 1.0;
  const double pr = gm1 * (E - 0.5 * (m0 * u[0] + m1 * u[1] + m2 * u[2]));
  // T~ = p / rho
  const double pb = wb[4] + wb[5] * ir;
  double rb = wb[0] - wb[5] * pr * ir * ir;
  // p = (gamma-1)(E - |m|^2 / (2 rho)), u_a = m_a / rho
  const double q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  rb += pb * gm1 * 0.5 * q2;
  double mb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mb[a] = wb[1 + a] * ir - pb * gm1 * u[a];
    rb -= wb[1 + a] * u[a] * ir;
  }
  Ubar[s] += rb;
  Ubar[g.vs + s] += mb[0];
  Ubar[2 * g.vs + s] += mb[1];
  Ubar[3 * g.vs + s] += mb[2];
  Ubar[4 * g.vs + s] += pb * gm1;
}

// out = a X + b Y + c Z over interior cells (null terms are skipped); the halo
// of out is set to zero.
__global__ void __launch_bounds__(kBlock) k_lincomb(double* __restrict__ out, double a, const double* X, double b,
                                                    const double* Y, double c, const double* Z, Geom g) {
  const PlaneIdx p = plane_index(g);
  if (!p.in) return;
  const bool in = p.i >= 0 && p.i < g.n[0] && p.j >= 0 && p.j < g.n[1] && p.k >= 0 && p.k < g.n[2];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long e = v * g.vs + p.c;
    double r = 0.0;
    if (in) {
      if (X) r += a * X[e];
      if (Y) r += b * Y[e];
      if (Z) r += c * Z[e];
    }
    out[e] = r;
  }
}

// Coordinates along one axis (n cells, halo h) whose value in a state with
// filled halos is the image of interior coordinate c: m = 0 is c itself,
// m = 1 .. h the low halo cells -m and m = h+1 .. 2h the high halo cells
// n-1 .. n-1+h; false when halo cell m's boundary source is not c. sg is the
// factor the image applies to the axis's velocity (-1 through a wall).
__device__ __forceinline__ bool halo_preimage(int c, int n, int h, int bc_lo, int bc_hi, int m, int& x, double& sg) {
  if (m == 0) {
    x = c;
    sg = 1.0;
    return true;
  }
  x = m <= h ? -m : n - 1 + (m - h);
  if (bc_source(x, n, bc_lo, bc_hi) != c) return false;
  sg = bc_sign(x, n, bc_lo, bc_hi);
  return true;
}

// Adjoint of the initial state U = S(W) (primitive point values W, 5 x
// interior, to the padded conservative state with filled halos): per interior
// cell, the adjoint of the cell's conservative values gathers Ubar over the
// cell and all its halo images (the transpose of the halo fill, in a fixed
// order, so the result is deterministic), then the transposed map of
// (rho, u, v, w, p) -> (rho, rho u, rho v, rho w, p/(gamma-1) + rho |u|^2/2)
// at W is added to Wbar.
__global__ void __launch_bounds__(kBlock) k_state_init_adj(const double* __restrict__ W,
                                                           const double* __restrict__ Ubar,
                                                           double* __restrict__ Wbar, Geom g) {
  const PlaneIdx p = plane_index(g);
  if (!p.in || p.i < 0 || p.i >= g.n[0] || p.j < 0 || p.j >= g.n[1] || p.k < 0 || p.k >= g.n[2]) return;
  double ub[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int a = 0; a <= 2 * g.h[0]; ++a) {
    int x;
    double sx;
    if (!halo_preimage(p.i, g.n[0], g.h[0], g.bc[0], g.bc[1], a, x, sx)) continue;
    for (int b = 0; b <= 2 * g.h[1]; ++b) {
      int y;
      double sy;
      if (!halo_preimage(p.j, g.n[1], g.h[1], g.bc[2], g.bc[3], b, y, sy)) continue;
      for (int c = 0; c <= 2 * g.h[2]; ++c) {
        int z;
        double sz;
        if (!halo_preimage(p.k, g.n[2], g.h[2], g.bc[4], g.bc[5], c, z, sz)) continue;
        const long long e = cell_at(g, x, y, z);
        ub[0] += Ubar[e];
        ub[1] += sx * Ubar[g.vs + e];
        ub[2] += sy * Ubar[2 * g.vs + e];
        ub[3] += sz * Ubar[3 * g.vs + e];
        ub[4] += Ubar[4 * g.vs + e];
      }
    }
  }
  const long long ni = (long long)g.n[0] * g.n[1] * g.n[2];
  const long long s = ((long long)p.k * g.n[1] + p.j) * g.n[0] + p.i;
  const double rho = W[s], u = W[ni + s], v = W[2 * ni + s], w = W[3 * ni + s];
  Wbar[s] += ub[0] + u * ub[1] + v * ub[2] + w * ub[3] + 0.5 * (u * u + v * v + w * w) * ub[4];
  Wbar[ni + s] += rho * (ub[1] + u * ub[4]);
  Wbar[2 * ni + s] += rho * (ub[2] + v * ub[4]);
  Wbar[3 * ni + s] += rho * (ub[3] + w * ub[4]);
  Wbar[4 * ni + s] += ub[4] * g.gm1i;
}

}  // namespace cfd
