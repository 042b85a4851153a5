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
//      (k_xadj_inv/dis): one lane per cell or face of a row, inputs passed
//      between lanes and contributions summed per cell by wavefront shifts
//      (one atomic per cell and variable). y and z faces
//      (k_march_adj_inv/dis): marching wavefronts, the reverse of the forward
//      marches. The inviscid and dissipative reverses run on two streams;
//   3. k_adj_dbar_halo (viscous): the transposed centred differences of
//      Dbar, added to Wbar at the halo cells (k_adj_fold adds the interior
//      cells' share);
//   4. k_adj_halo: the transposed halo fill, every halo cell's Wbar added to
//      its interior source cell;
//   5. k_adj_fold: per interior cell, the transposed primitive map at the
//      state (from its primitives) gives Ubar.
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

// ---------------------------------------------------------------------------
// x faces: one lane per slot of a row, as in the forward x sweep; the
// neighbouring cells of a row are neighbouring lanes, so a cell's inputs are
// loaded once and passed to the faces that use them, and the contributions to
// a cell are summed across lanes into the lane that owns it (DPP wavefront
// shifts, no LDS), which adds the sum to memory with one atomic per variable.
// Rows are taken in the band-major order of the forward x sweep.

// Inviscid part: the slots of a row are its cells -3 .. n+2 (every cell a
// reconstruction reaches). The lane of cell x forms the reconstruction pair
// of x (cells x-1 .. n have one, §3.3), reverses the HLLC flux of face x
// (between x-1 and x; its left state is the pair of x-1, one lane below), and
// then reverses the pair of x with the cotangents of its faces x (own) and
// x+1 (one lane above), into cells x-2 .. x+2 (lanes -2 .. +2). A wavefront
// takes 64 consecutive slots of which the middle kXInvNew reverse their
// pairs; two slots at each end overlap the neighbouring wavefronts and only
// supply shuffles and collect sums.
constexpr int kXInvNew = 60;

__global__ void __launch_bounds__(kBlock) k_xadj_inv(const double* P, const double* __restrict__ Rbar,
                                                     double rscale, double* Wbar, Geom g) {
  const int lane = threadIdx.x & 63;
  const int wave = (xcd_major_block(blockIdx.x, gridDim.x) * kBlock + (int)threadIdx.x) >> 6;
  const int n = g.n[0];
  const int S = n + 6;
  const int total = S * g.n[1] * g.n[2];
  const int first = wave * kXInvNew;
  if (first >= total) return;  // uniform per wavefront
  const int gs = first - 2 + lane;
  const bool inrange = gs >= 0 && gs < total;
  int x = 0, j = 0, k = 0;
  if (inrange) {
    const int row = gs / S;
    x = gs - row * S - 3;
    x_row(g, row, j, k);
  }
  const bool pair = inrange && x >= -1 && x <= n;     // cell x has a reconstruction pair
  const bool face = inrange && x >= 0 && x <= n && lane >= 1;  // face x, with its left cell in the wavefront
  const bool rev = pair && lane >= 2 && lane < 2 + kXInvNew;
  const long long cx = cell_at(g, x, j, k);
  const long long c0 = cell_at(g, (pair ? x : 0) - 2, j, k);  // window: cells x-2 .. x+2
  const double gsc = rscale * g.idx[0];
  double WLb[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, WRb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  {
    double q[5][5];
#pragma unroll
    for (int m = 0; m < 5; ++m) load_prims(P, g.vs, c0 + m, q[m]);
    double qr[5], ql[5];
    recon_pair<SCH_JS>(q, qr, ql);  // right face of x (left state of face x+1), left face of x
    double WL[5], Gb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double r = inrange && x >= 0 && x < n ? Rbar[v * g.vs + cx] : 0.0;
      Gb[v] = gsc * (r - lane_shr1(r));  // (Rbar_x - Rbar_{x-1}) / dx
      WL[v] = lane_shr1(qr[v]);
    }
    if (face) hllc_rev<0>(g.gamma, g.gm1i, WL, ql, Gb, WLb, WRb);
  }
  asm volatile("" ::: "memory");  // reload the window below instead of keeping it live
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double qrb = lane_shl1(WLb[v]);  // face x+1: cotangent of the right-face value of x
    double gq[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (rev) {
      const double* q = P + v * g.vs + c0;
      weno5_pair_rev(q[0], q[1], q[2], q[3], q[4], qrb, WRb[v], gq);
    }
    // cell x receives gq[4] from lane - 2, gq[3] from lane - 1, gq[2] from
    // itself, gq[1] from lane + 1 and gq[0] from lane + 2
    const double up = lane_shr1(lane_shr1(gq[4]) + gq[3]);
    const double down = lane_shl1(lane_shl1(gq[0]) + gq[1]);
    if (inrange) atomic_add(Wbar + v * g.vs + cx, up + gq[2] + down);
  }
}

// Dissipative part: slot s of a row is face f = s - 3 (f = -3 .. n), and its
// lane loads the inputs of cell f+1 (u, v, w and the four tangential
// derivatives). Face f takes those of cells f-2 .. f+1 from itself and the
// three lanes below, and its contributions to those cells flow back down to
// them. A wavefront takes 64 consecutive slots; the first three overlap its
// predecessor and only supply inputs and collect sums. The heat flux is
// linear in T~, so its reverse needs no T~ values.
constexpr int kXDisCtx = 3;
constexpr int kXDisNew = 64 - kXDisCtx;

__global__ void __launch_bounds__(kBlock) k_xadj_dis(const double* __restrict__ P, const double* __restrict__ Rbar,
                                                     double rscale, double* Wbar, double* Dbar, Geom g) {
  const int lane = threadIdx.x & 63;
  const int wave = (xcd_major_block(blockIdx.x, gridDim.x) * kBlock + (int)threadIdx.x) >> 6;
  const int n = g.n[0];
  const int S = n + 1 + kXDisCtx;
  const int total = S * g.n[1] * g.n[2];
  const int first = wave * kXDisNew;
  if (first >= total) return;  // uniform per wavefront
  const int gs = first - kXDisCtx + lane;
  const bool inrange = gs >= 0 && gs < total;
  int f = 0, j = 0, k = 0;
  if (inrange) {
    const int row = gs / S;
    f = gs - row * S - kXDisCtx;
    x_row(g, row, j, k);
  }
  const bool face = inrange && f >= 0 && lane >= kXDisCtx;
  const long long co = cell_at(g, inrange ? f + 1 : 0, j, k);  // the lane's cell f+1
  // inputs of cell f+1, then of cells f, f-1, f-2 from the lanes below
  double u[4][3], d[4][4], r[3][5];
#pragma unroll
  for (int v = 0; v < 3; ++v) u[3][v] = g.viscous ? P[(1 + v) * g.vs + co] : 0.0;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) d[3][kk] = 0.0;
  if (g.viscous) tangential_at_flat<0>(g, P, co, d[3]);
#pragma unroll
  for (int v = 0; v < 5; ++v) r[0][v] = inrange && f + 1 >= 0 && f + 1 < n ? Rbar[v * g.vs + co] : 0.0;
#pragma unroll
  for (int m = 2; m >= 0; --m) {
#pragma unroll
    for (int v = 0; v < 3; ++v) u[m][v] = lane_shr1(u[m + 1][v]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) d[m][kk] = lane_shr1(d[m + 1][kk]);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    r[1][v] = lane_shr1(r[0][v]);  // cell f
    r[2][v] = lane_shr1(r[1][v]);  // cell f-1
  }
  struct RegSink {
    double qb[4][4];   // cells f-2 .. f+1: u, v, w, T~
    double tgb[4][4];  // cells f-2 .. f+1: derivative inputs
    __device__ void q(int m, int v, double x) { qb[m - 1][v == 5 ? 3 : v - 1] += x; }
    __device__ void tg(int m, int kk, double x) { tgb[m - 1][kk] += x; }
  } sink;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) sink.qb[m][v] = sink.tgb[m][v] = 0.0;
  if (face) {
    FaceWindow w;
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) w.q[m][v] = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      w.T[m] = 0.0;
#pragma unroll
      for (int v = 0; v < 3; ++v) w.q[1 + m][1 + v] = u[m][v];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) w.tg[m][kk] = d[m][kk];
    }
    const double gsc = rscale * g.idx[0];
    double Gb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Gb[v] = gsc * (r[1][v] - r[2][v]);
    Geom gd = g;
    gd.inviscid = 0;  // the inviscid part is k_xadj_inv
    face_flux_rev<0>(gd, w, Gb, sink);
  }
  // cell f+1 collects its share from faces f, f+1, f+2, f+3 (this lane and
  // the three above), up to the end of its row
  const bool above = inrange && f < n;
  auto gather = [&](const double (&c)[4][4], int v) {
    double a = c[0][v];
#pragma unroll
    for (int m = 1; m < 4; ++m) {
      const double b = lane_shl1(a);  // every lane takes part in the shift
      a = (above ? b : 0.0) + c[m][v];
    }
    return a;
  };
  const int wslot[4] = {1, 2, 3, 5};  // u, v, w, T~ in Wbar
  const int comp[4] = {0 * 3 + 1, 1 * 3 + 1, 0 * 3 + 2, 2 * 3 + 2};
  const bool tact[4] = {g.act[1] != 0, g.act[1] != 0, g.act[2] != 0, g.act[2] != 0};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (v == 3 ? !g.heat : !g.viscous) continue;
    const double t = gather(sink.qb, v);
    if (inrange) atomic_add(Wbar + wslot[v] * g.vs + co, t);
  }
  if (g.viscous) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      if (!tact[kk]) continue;
      const double t = gather(sink.tgb, kk);
      if (inrange) atomic_add(Dbar + comp[kk] * g.vs + co, t);
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
// A pair shared with the neighbouring segment is reversed in both, each with
// its own face's share of the cotangent (the reverse is linear in it).
// The window holds cells f-3 .. f+2 in registers, and the per-cell sums of
// the five cells a pair reverse touches live in a lane-private LDS ring.
// Cell offsets are 32-bit (the adjoint requires fewer than 2^31 padded
// cells): one address register per cell instead of one per cell and
// variable. The window, the HLLC reverse and the carried states still need
// about 380 registers, so the kernel runs one wavefront per SIMD; at two it
// spills, and reloading the window at every face instead (which fits two)
// ran 1.3x slower, the reloads' latency exposed.
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
  const int st = (int)g.s[AX];
  const long long vs = g.vs;
  const int n = g.n[AX];
  const double gs_scale = rscale * g.idx[AX];
  int c = (int)march_adj_cell<AX>(g, i, o, s0 - 3);  // window cell 0: cell f-3 of face f = s0
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
  const int st = (int)g.s[AX];  // 32-bit cell offsets, as in k_march_adj_inv
  const long long vs = g.vs;
  const int n = g.n[AX];
  const double gs_scale = rscale * g.idx[AX];
  Geom gd = g;
  gd.inviscid = 0;  // the inviscid part is k_march_adj_inv
  int c = (int)march_adj_cell<AX>(g, i, o, s0 - 2);  // window cell 0: cell f-2 of face f = s0
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

// Transposed centred differences of Dbar at the halo cells: Wbar(u, v, w)[c]
// += the adjoint the tangential derivatives give halo cell c, before
// k_adj_halo adds the halo cells to their interior sources (the interior
// cells' own share is formed in k_adj_fold). One thread per halo cell, each
// updating its own cell.
__global__ void __launch_bounds__(kBlock) k_adj_dbar_halo(const double* __restrict__ Dbar, double* __restrict__ Wbar,
                                                          Geom g) {
  int i, j, k;
  if (!halo_cell(g, (long long)blockIdx.x * kBlock + threadIdx.x, i, j, k)) return;
  const long long c = cell_at(g, i, j, k);
  const int q[3] = {i, j, k};
  double wb[4] = {0.0, 0.0, 0.0, 0.0};
  fold_dbar<true>(g, Dbar, c, q, wb);
#pragma unroll
  for (int v = 1; v < 4; ++v) Wbar[v * g.vs + c] += wb[v];
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

// The destination of a right-hand-side adjoint: out = a X + b Y + c Z + the
// folded adjoint at the interior cells (null terms are skipped; out may be
// one of X, Y, Z), and, with zero_halo, zeros at its halo cells (otherwise
// they are not touched). The linear combinations of the step adjoint's
// stages are formed here, in the pass that writes out anyway.
struct AdjOut {
  double* out;
  double a, b, c;
  const double* X;
  const double* Y;
  const double* Z;
  int zero_halo;
};

// Per cell s, after k_adj_halo (and, with viscous fluxes, k_adj_dbar_halo):
// Wbar[s] plus (Dbar non-null) the transposed centred differences of Dbar at
// s, then the transposed primitive map at the state, given by its primitives
// P[s] (rho, u, v, w, p), into the destination o.
__global__ void __launch_bounds__(kBlock) k_adj_fold(const double* __restrict__ P, const double* __restrict__ Wbar,
                                                     const double* __restrict__ Dbar, AdjOut o, Geom g) {
  const PlaneIdx p = plane_index(g, true);
  if (!p.in) return;
  const long long s = p.c;
  if (p.i < 0 || p.i >= g.n[0] || p.j < 0 || p.j >= g.n[1] || p.k < 0 || p.k >= g.n[2]) {
    if (o.zero_halo)
#pragma unroll
      for (int v = 0; v < 5; ++v) o.out[v * g.vs + s] = 0.0;
    return;
  }
  double base[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long e = v * g.vs + s;
    double r = 0.0;
    if (o.X) r += o.a * o.X[e];
    if (o.Y) r += o.b * o.Y[e];
    if (o.Z) r += o.c * o.Z[e];
    base[v] = r;
  }
  double wb[6];
#pragma unroll
  for (int v = 0; v < 6; ++v) wb[v] = Wbar[v * g.vs + s];
  if (Dbar) {
    // an interior cell's +-2 neighbours lie inside the padded block
    const int q[3] = {p.i, p.j, p.k};
    fold_dbar<false>(g, Dbar, s, q, wb);
  }
  const double rho = P[s], pr = P[4 * g.vs + s];
  const double u[3] = {P[g.vs + s], P[2 * g.vs + s], P[3 * g.vs + s]};
  const double ir = div_nr(1.0, rho);
  const double gm1 = g.gamma - 1.0;
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
  o.out[s] = base[0] + rb;
  o.out[g.vs + s] = base[1] + mb[0];
  o.out[2 * g.vs + s] = base[2] + mb[1];
  o.out[3 * g.vs + s] = base[3] + mb[2];
  o.out[4 * g.vs + s] = base[4] + pb * gm1;
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
