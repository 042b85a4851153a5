// Forward kernels of one right-hand-side evaluation / TVD-RK3 stage (gfx950).
//
// Per stage:  prim  : U_k -> P = (rho,u,v,w,p,T~) on the padded grid, halos by
//                     gather from their interior source cells (so U's own halo
//                     is never read), plus the CFL rate max;
//             sweep : one kernel per active axis; each face flux is computed
//                     once in registers and differenced into its two cells,
//                     the tangential velocity derivatives of the viscous flux
//                     formed from P on the way.
//                     x: one lane per face, wavefront shuffles carry the
//                        left-face flux; y, z: one lane per column segment
//                        marching along the axis with a register window.
//                     The last active axis applies the RK3 stage update and
//                     may also store the primitives of the updated cell for
//                     the next stage (with the CFL rate and health bits), so
//                     that within a run of steps the prim pass reduces to a
//                     halo refresh of P.
#pragma once
#include "physics.hpp"

namespace cfd {

// Device control block of a solver.
struct DevCtl {
  double dt;   // step of the current step (0: step disabled, t_end reached)
  int status;  // health bits, see cfd_check
  int pad;
};

constexpr int kBlock = 256;
constexpr int kGradComps = 9;  // adjoint of d u_a / d x_b accumulated at component a*3+b

// What a sweep does with the divergence D of its axis: MODE_WRITE stores
// R = -D, MODE_ACC R -= D; the RK modes apply the stage update with
// R = -D (MODE_WRITE_RK), R - D (MODE_ACC_RK) or R + R2 - D (MODE_ACC2_RK:
// the two marches before it each wrote their own accumulator, which spares
// the second one a read-modify-write of R).
enum SweepMode { MODE_WRITE = 0, MODE_ACC = 1, MODE_ACC_RK = 2, MODE_WRITE_RK = 3, MODE_ACC2_RK = 4 };
__host__ __device__ constexpr bool mode_rk(int m) { return m == MODE_ACC_RK || m == MODE_WRITE_RK || m == MODE_ACC2_RK; }
__host__ __device__ constexpr bool mode_reads_r(int m) { return m == MODE_ACC || m == MODE_ACC_RK || m == MODE_ACC2_RK; }

struct StageIO {
  double* R;         // right-hand-side accumulator (padded layout)
  const double* R2;  // second accumulator (MODE_ACC2_RK)
  const double* Un;  // state at the start of the step
  const double* Uk;  // stage input state
  double* Uout;      // stage output state (may alias Un in the last stage)
  double a, b;       // Uout = a Un + b (Uk + dt R)
  const double* dtp; // step size; nullptr for a plain right-hand side
  double* Pn;        // primitives of Uout, interior cells (sweeps with PN set)
  double* partial;   // CFL rate slots (PN sweeps with PRIM_CFL in `what`)
  DevCtl* ctl;       // health bits (PN sweeps with PRIM_HEALTH in `what`)
  int what;
};

__device__ __forceinline__ bool step_disabled(const double* dtp) { return dtp != nullptr && *dtp == 0.0; }

// Kernels over the padded grid use a plane-indexed launch: blockIdx.y is the
// padded z index, and threads cover the x-y plane with a 32-bit in-plane index.
struct PlaneIdx {
  int i, j, k;      // interior-relative coordinates (halo cells negative)
  long long c;      // padded cell index
  bool in;          // inside the padded grid
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2). The XCD-major order gives each XCD one contiguous range of logical
// blocks - consecutive planes - so the neighbour planes a stencil re-reads stay
// in that XCD's L2. XCD x receives the hardware blocks b = x, x+8, x+16, ...;
// the first nb % 8 XCDs get one block more, and the map is a permutation.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_major_block(int b, int nb) {
  const int x = b % kXcds, local = b / kXcds;
  const int q = nb / kXcds, r = nb % kXcds;
  return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// bx, by: block coordinates of a plane-indexed launch of gx x gy blocks.
__device__ __forceinline__ PlaneIdx plane_index_at(const Geom& g, int bx, int by, int gx, int gy, bool xcd_major) {
  PlaneIdx p;
  const int plane = g.N[0] * g.N[1];
  if (xcd_major) {
    const int logical = xcd_major_block(by * gx + bx, gx * gy);
    by = logical / gx;
    bx = logical - by * gx;
  }
  const int t = bx * kBlock + threadIdx.x;
  p.in = t < plane;
  const int jj = t / g.N[0];
  const int ii = t - jj * g.N[0];
  p.i = ii - g.h[0];
  p.j = jj - g.h[1];
  p.k = by - g.h[2];
  p.c = (long long)by * plane + t;
  return p;
}

__device__ __forceinline__ PlaneIdx plane_index(const Geom& g, bool xcd_major = false) {
  return plane_index_at(g, blockIdx.x, blockIdx.y, gridDim.x, gridDim.y, xcd_major);
}

// Number of blocks along x of a plane-indexed launch.
__host__ __device__ __forceinline__ int plane_blocks_x(const Geom& g) {
  return (g.N[0] * g.N[1] + kBlock - 1) / kBlock;
}

// ----------------------------------------------------------------------------
// Halo refresh of a padded field of NC components (in place): halo cells copy
// their interior source cell, interior cells do nothing.
template <int NC = 5>
__device__ __forceinline__ void fill_halo_body(double* U, const Geom& g, const PlaneIdx& p) {
  if (!p.in) return;
  const int si = bc_source(p.i, g.n[0], g.bc[0], g.bc[1]);
  const int sj = bc_source(p.j, g.n[1], g.bc[2], g.bc[3]);
  const int sk = bc_source(p.k, g.n[2], g.bc[4], g.bc[5]);
  if (si == p.i && sj == p.j && sk == p.k) return;
  const long long s = cell_at(g, si, sj, sk);
  const double sg[3] = {bc_sign(p.i, g.n[0], g.bc[0], g.bc[1]), bc_sign(p.j, g.n[1], g.bc[2], g.bc[3]),
                        bc_sign(p.k, g.n[2], g.bc[4], g.bc[5])};
#pragma unroll
  for (int v = 0; v < NC; ++v) U[v * g.vs + p.c] = (v >= 1 && v <= 3 ? sg[v - 1] : 1.0) * U[v * g.vs + s];
}

__global__ void __launch_bounds__(kBlock) k_fill_halo(double* U, Geom g) { fill_halo_body<5>(U, g, plane_index(g)); }

// Halo refresh of the primitives P (6 components) after a sweep stored the
// interior ones, one thread per halo cell; skipped with the step. Halo cells
// are numbered slab by slab: the z halo planes (whole padded planes), then
// for interior z the y halo rows (whole padded rows), then for interior z and
// y the x halo cells.
__host__ __device__ __forceinline__ long long halo_cells(const Geom& g) {
  return 2LL * g.h[2] * g.N[0] * g.N[1] + 2LL * g.h[1] * g.N[0] * g.n[2] + 2LL * g.h[0] * g.n[1] * g.n[2];
}

__host__ __device__ __forceinline__ int halo_blocks(const Geom& g) {
  const long long n = halo_cells(g);
  return (int)(n > 0 ? (n + kBlock - 1) / kBlock : 1);
}

// Interior-relative coordinates of halo cell number t (numbered as above);
// false past the last halo cell.
__device__ __forceinline__ bool halo_cell(const Geom& g, long long t, int& i, int& j, int& k) {
  const long long zs = 2LL * g.h[2] * g.N[0] * g.N[1];
  const long long ys = 2LL * g.h[1] * g.N[0] * g.n[2];
  const long long xs = 2LL * g.h[0] * g.n[1] * g.n[2];
  if (t < zs) {
    const long long plane = (long long)g.N[0] * g.N[1];
    const int kk = (int)(t / plane);  // 0 .. 2h-1
    const long long r = t - kk * plane;
    j = (int)(r / g.N[0]) - g.h[1];
    i = (int)(r - (long long)(j + g.h[1]) * g.N[0]) - g.h[0];
    k = kk < g.h[2] ? kk - g.h[2] : g.n[2] + (kk - g.h[2]);
  } else if ((t -= zs) < ys) {
    const long long slab = 2LL * g.h[1] * g.N[0];
    k = (int)(t / slab);
    const long long r = t - k * slab;
    const int jj = (int)(r / g.N[0]);  // 0 .. 2h-1
    i = (int)(r - (long long)jj * g.N[0]) - g.h[0];
    j = jj < g.h[1] ? jj - g.h[1] : g.n[1] + (jj - g.h[1]);
  } else if ((t -= ys) < xs) {
    const long long row = 2LL * g.h[0];
    const long long kj = t / row;
    const int ii = (int)(t - kj * row);
    k = (int)(kj / g.n[1]);
    j = (int)(kj - (long long)k * g.n[1]);
    i = ii < g.h[0] ? ii - g.h[0] : g.n[0] + (ii - g.h[0]);
  } else {
    return false;
  }
  return true;
}

__device__ __forceinline__ void prim_halo_body(double* P, const Geom& g, long long t) {
  int i, j, k;  // interior-relative coordinates of the halo cell
  if (!halo_cell(g, t, i, j, k)) return;
  const int si = bc_source(i, g.n[0], g.bc[0], g.bc[1]);
  const int sj = bc_source(j, g.n[1], g.bc[2], g.bc[3]);
  const int sk = bc_source(k, g.n[2], g.bc[4], g.bc[5]);
  const long long c = cell_at(g, i, j, k), s = cell_at(g, si, sj, sk);
  const double sg[3] = {bc_sign(i, g.n[0], g.bc[0], g.bc[1]), bc_sign(j, g.n[1], g.bc[2], g.bc[3]),
                        bc_sign(k, g.n[2], g.bc[4], g.bc[5])};
  // T~ = p/rho (slot 5) only for the face-by-face schemes, which read it from
  // P; the cell-centred ones form it from the window and do not store it
  const bool with_t = g.roe || g.wenoz;
#pragma unroll
  for (int v = 0; v < 6; ++v)
    if (v < 5 || with_t) P[v * g.vs + c] = (v >= 1 && v <= 3 ? sg[v - 1] : 1.0) * P[v * g.vs + s];
}

__global__ void __launch_bounds__(kBlock) k_prim_halo(double* P, Geom g, const double* dtp) {
  if (step_disabled(dtp)) return;
  prim_halo_body(P, g, (long long)blockIdx.x * kBlock + threadIdx.x);
}

// Conservative interior state from primitive point values W (5 x interior, no halo).
__global__ void __launch_bounds__(kBlock) k_state_init(const double* W, double* U, Geom g) {
  const PlaneIdx p = plane_index(g);
  if (!p.in || p.i < 0 || p.i >= g.n[0] || p.j < 0 || p.j >= g.n[1] || p.k < 0 || p.k >= g.n[2]) return;
  const long long ni = (long long)g.n[0] * g.n[1] * g.n[2];
  const long long s = ((long long)p.k * g.n[1] + p.j) * g.n[0] + p.i;
  const double rho = W[s], u = W[ni + s], v = W[2 * ni + s], w = W[3 * ni + s], pr = W[4 * ni + s];
  U[p.c] = rho;
  U[g.vs + p.c] = rho * u;
  U[2 * g.vs + p.c] = rho * v;
  U[3 * g.vs + p.c] = rho * w;
  U[4 * g.vs + p.c] = pr / (g.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Block maximum (wavefront shuffles, then across the block's wavefronts via
// LDS); the result is valid in thread 0.
__device__ __forceinline__ double block_max(double x) {
  __shared__ double part[kBlock / 64];
  x = wave_max(x);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) x = fmax(x, part[i]);
  }
  __syncthreads();  // part[] may be reused by the block's next reduction
  return x;
}

// CFL rate of an interior cell from its primitives w = (rho, u, v, w, p, p/rho)
// and ir = 1/rho: max(sum_d (|u_d| + c)/dx_d, (mu/rho) visc_rate), c^2 = gamma p/rho.
__device__ __forceinline__ double cfl_rate(const Geom& g, const double* w, double ir) {
  const double c = sqrt_pos(g.gamma * w[5]);
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (g.act[d]) s += (fabs(w[1 + d]) + c) * g.idx[d];
  if (g.viscous || g.heat) s = fmax(s, (g.mu * ir) * g.visc_rate);
  return s;
}

// CFL rate maxima are kept in kCflSlots slots (the bits of non-negative
// doubles order like unsigned integers, so atomicMax on the bits is a max).
// Each block folds its maximum into slot (block index mod kCflSlots), which
// spreads the atomics; k_dt reduces the slots and clears them for the next step.
constexpr int kCflSlots = 256;

__device__ __forceinline__ void publish_rate(double* slots, int block_index, double s) {
  s = block_max(s);
  if (threadIdx.x == 0 && s > 0.0)
    atomicMax(reinterpret_cast<unsigned long long*>(slots) + (block_index & (kCflSlots - 1)),
              (unsigned long long)__double_as_longlong(s));
}

// Primitive variables w = (rho, u, v, w, p, p/rho) of conservative values q;
// returns 1/rho.
__device__ __forceinline__ double cons_to_prim(const Geom& g, const double* q, double* w) {
  const double rho = q[0];
  w[0] = rho;
  const double ir = div_nr(1.0, rho);
  w[1] = q[1] * ir;
  w[2] = q[2] * ir;
  w[3] = q[3] * ir;
  w[4] = (g.gamma - 1.0) * (q[4] - 0.5 * (q[1] * w[1] + q[2] * w[2] + q[3] * w[3]));
  w[5] = w[4] * ir;
  return ir;
}

// Health bits of a cell: 1 non-finite conservative value, 2 rho <= 0, 4 p <= 0;
// and of a face: 8 a reconstructed state with rho <= 0 or p <= 0.
constexpr int kBadFace = 8;

// Face check of the cell-centred schemes: a reconstructed state of the face
// with a non-positive (or non-finite) density or pressure sets kBadFace in
// bad; with safe reconstruction both states then take the values of the two
// cells next to the face (qa left, qb right: the first-order reconstruction).
__device__ __forceinline__ void check_face_states(const Geom& g, bool use, double* WL, double* WR,
                                                  const double* qa, const double* qb, int& bad) {
  const bool ok = WL[0] > 0.0 && WL[4] > 0.0 && WR[0] > 0.0 && WR[4] > 0.0;
  if (use && !ok) {
    bad |= kBadFace;
    if (g.safe) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        WL[v] = qa[v];
        WR[v] = qb[v];
      }
    }
  }
}

// Health bits of a cell: 1 non-finite conservative value, 2 rho <= 0, 4 p <= 0.
__device__ __forceinline__ int health_bits(const double* q, double p) {
  int bad = 0;
  if (!isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2]) || !isfinite(q[3]) || !isfinite(q[4])) bad |= 1;
  if (!(q[0] > 0.0)) bad |= 2;
  if (!(p > 0.0)) bad |= 4;
  return bad;
}

// Primitive variables on the padded grid, gathered through the boundary map.
// Over interior cells, `what` bit 0 adds the CFL rate (block maxima written
// to partial[], one per block) and bit 1 the health bits.
constexpr int PRIM_CFL = 1, PRIM_HEALTH = 2;

__device__ __forceinline__ void prim_body(const double* __restrict__ U, double* __restrict__ P, const Geom& g,
                                          DevCtl* ctl, int what, double* __restrict__ partial, const PlaneIdx& q,
                                          int part_index) {
  double smax = 0.0;
  if (q.in) {
    const int si = bc_source(q.i, g.n[0], g.bc[0], g.bc[1]);
    const int sj = bc_source(q.j, g.n[1], g.bc[2], g.bc[3]);
    const int sk = bc_source(q.k, g.n[2], g.bc[4], g.bc[5]);
    const long long s = cell_at(g, si, sj, sk);
    const long long c = q.c;
    double u[5], w[6];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[v * g.vs + s];
    u[1] *= bc_sign(q.i, g.n[0], g.bc[0], g.bc[1]);
    u[2] *= bc_sign(q.j, g.n[1], g.bc[2], g.bc[3]);
    u[3] *= bc_sign(q.k, g.n[2], g.bc[4], g.bc[5]);
    const double ir = cons_to_prim(g, u, w);
#pragma unroll
    for (int v = 0; v < 6; ++v) P[v * g.vs + c] = w[v];
    if (what && s == c) {
      if (what & PRIM_CFL) smax = cfl_rate(g, w, ir);
      if (what & PRIM_HEALTH) {
        const int bad = health_bits(u, w[4]);
        if (bad) atomicOr(&ctl->status, bad);
      }
    }
  }
  if (what & PRIM_CFL) publish_rate(partial, part_index, smax);
}

__global__ void __launch_bounds__(kBlock) k_prim(const double* __restrict__ U, double* __restrict__ P,
                                                 Geom g, DevCtl* ctl, int what, const double* dtp,
                                                 double* __restrict__ partial) {
  if (step_disabled(dtp)) return;
  prim_body(U, P, g, ctl, what, partial, plane_index(g), blockIdx.y * gridDim.x + blockIdx.x);
}

// CFL rate maxima of a state (interior cells only), for cfd_compute_dt.
__global__ void __launch_bounds__(kBlock) k_cfl(const double* __restrict__ U, Geom g,
                                                double* __restrict__ partial) {
  const PlaneIdx q = plane_index(g);
  double smax = 0.0;
  if (q.in && q.i >= 0 && q.i < g.n[0] && q.j >= 0 && q.j < g.n[1] && q.k >= 0 && q.k < g.n[2]) {
    double u[5], w[6];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[v * g.vs + q.c];
    const double ir = cons_to_prim(g, u, w);
    smax = cfl_rate(g, w, ir);
  }
  publish_rate(partial, blockIdx.y * gridDim.x + blockIdx.x, smax);
}

// Step size of the current step: fixed, or cfl / (max of the npart CFL rate
// partials); clipped to t_end (> 0) and zero once t_end is reached. Advances
// *t. One block of kBlock threads.
__device__ __forceinline__ void dt_body(DevCtl* ctl, double cfl, double fixed_dt, double t_end, double* t,
                                        double* dt_out, double* __restrict__ partial, int npart) {
  double dt = fixed_dt;
  if (!(fixed_dt > 0.0)) {
    double m = 0.0;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) m = fmax(m, partial[i]);
    m = block_max(m);  // every slot has been read once this returns
    for (int i = threadIdx.x; i < npart; i += blockDim.x) partial[i] = 0.0;
    dt = cfl / m;
  }
  if (threadIdx.x != 0) return;
  if (t != nullptr && t_end > 0.0) {
    const double rem = t_end - *t;
    dt = rem > 0.0 ? fmin(dt, rem) : 0.0;
  }
  ctl->dt = dt;
  if (t != nullptr) *t = *t + dt;
  if (dt_out != nullptr) *dt_out = dt;
}

__global__ void __launch_bounds__(kBlock) k_dt(DevCtl* ctl, double cfl, double fixed_dt, double t_end,
                                               double* t, double* dt_out, double* __restrict__ partial,
                                               int npart) {
  dt_body(ctl, cfl, fixed_dt, t_end, t, dt_out, partial, npart);
}

// ----------------------------------------------------------------------------
// ----------------------------------------------------------------------------
// Face window loads.
__device__ __forceinline__ void load_prims(const double* __restrict__ P, long long vs, long long c,
                                           double* q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) q[v] = P[v * vs + c];
}

// Tangential velocity derivatives at a cell for faces normal to D (the
// layout of FaceWindow::tg), fourth-order central differences of the
// primitives across the cell (§3.4):
// d u_D / d x_T1, d u_T1 / d x_T1, d u_D / d x_T2, d u_T2 / d x_T2. The
// tangential coordinates of every cell a face stencil touches are interior, so
// the +-2 neighbours lie inside the padded block.
__device__ __forceinline__ double central4(const double* __restrict__ q, long long st, double i12) {
  return (q[-2 * st] - 8.0 * q[-st] + 8.0 * q[st] - q[2 * st]) * i12;
}

template <int D>
__device__ __forceinline__ void tangential_at(const Geom& g, const double* __restrict__ P, long long c,
                                              double* tg) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const double* uD = P + (1 + D) * g.vs + c;
  if (g.act[T1]) {
    const long long st = g.s[T1];
    const double i12 = g.idx[T1] * (1.0 / 12.0);
    tg[0] = central4(uD, st, i12);
    tg[1] = central4(P + (1 + T1) * g.vs + c, st, i12);
  } else {
    tg[0] = 0.0;
    tg[1] = 0.0;
  }
  if (g.act[T2]) {
    const long long st = g.s[T2];
    const double i12 = g.idx[T2] * (1.0 / 12.0);
    tg[2] = central4(uD, st, i12);
    tg[3] = central4(P + (1 + T2) * g.vs + c, st, i12);
  } else {
    tg[2] = 0.0;
    tg[3] = 0.0;
  }
}

// The same without branches, in two halves: the sixteen loads, and the
// arithmetic. An inactive axis gets stride 0 and weight 0 (the difference of
// a cell with itself is exactly 0). Callers issue all loads before any use (a
// scheduling barrier keeps the compiler from interleaving loads and uses,
// which serialises their latencies).
template <int D>
__device__ __forceinline__ void tangential_load(const Geom& g, const double* __restrict__ P, long long c,
                                                double (&x)[4][4]) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const long long s1 = g.act[T1] ? g.s[T1] : 0, s2 = g.act[T2] ? g.s[T2] : 0;
  const double* q[4] = {P + (1 + D) * g.vs + c, P + (1 + T1) * g.vs + c, P + (1 + D) * g.vs + c,
                        P + (1 + T2) * g.vs + c};
  const long long st[4] = {s1, s1, s2, s2};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    x[m][0] = q[m][-2 * st[m]];
    x[m][1] = q[m][-st[m]];
    x[m][2] = q[m][st[m]];
    x[m][3] = q[m][2 * st[m]];
  }
}

template <int D>
__device__ __forceinline__ void tangential_combine(const Geom& g, const double (&x)[4][4], double* tg) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  const double w1 = g.act[T1] ? g.idx[T1] * (1.0 / 12.0) : 0.0, w2 = g.act[T2] ? g.idx[T2] * (1.0 / 12.0) : 0.0;
  const double w[4] = {w1, w1, w2, w2};
#pragma unroll
  for (int m = 0; m < 4; ++m) tg[m] = (x[m][0] - 8.0 * x[m][1] + 8.0 * x[m][2] - x[m][3]) * w[m];
}

template <int D>
__device__ __forceinline__ void tangential_at_flat(const Geom& g, const double* __restrict__ P, long long c,
                                                   double* tg) {
  double x[4][4];
  tangential_load<D>(g, P, c, x);
  __builtin_amdgcn_sched_barrier(0);
  tangential_combine<D>(g, x, tg);
}

// Writing the divergence contribution D = (G+ - G-)/dx of one cell, in two
// halves so that a marching sweep can issue the loads of the cell's update
// (accumulated R, stage states) before the face arithmetic and store after
// it: EmitIn holds the loaded values. MODE_WRITE / MODE_ACC store R = -D or
// R - D; the RK modes store Uout = a Un + b (Uk + dt R) instead of R.
struct EmitIn {
  double r[5], un[5], uk[5];
};

// A stage whose weight a of U^n is zero (TVD-RK3 stage 1, where U^(k) is
// U^n) does not load U^n.
template <int MODE>
__device__ __forceinline__ void emit_fetch(const StageIO& io, long long vs, long long c, EmitIn& in) {
  const bool with_un = io.a != 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long e = v * vs + c;
    if (MODE == MODE_ACC || MODE == MODE_ACC_RK) in.r[v] = io.R[e];
    if (MODE == MODE_ACC2_RK) in.r[v] = io.R[e] + io.R2[e];
    if (mode_rk(MODE)) {
      in.un[v] = with_un ? io.Un[e] : 0.0;
      in.uk[v] = io.Uk[e];
    }
  }
}

// STORE_T: also store T~ = p/rho with the next primitives (the face-by-face
// sweeps read it from P; the cell-centred ones form it from rho and p).
template <int MODE, bool PN = false, bool STORE_T = true>
__device__ __forceinline__ void emit_put(const StageIO& io, const Geom& g, long long c, const double* D,
                                         const EmitIn& in, double dt, double& smax, int& bad) {
  double uo[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long e = v * g.vs + c;
    const double r = (MODE == MODE_WRITE || MODE == MODE_WRITE_RK) ? -D[v] : in.r[v] - D[v];
    if (MODE == MODE_WRITE || MODE == MODE_ACC) {
      io.R[e] = r;
    } else {
      uo[v] = io.a * in.un[v] + io.b * (in.uk[v] + dt * r);
      io.Uout[e] = uo[v];
    }
  }
  if constexpr (PN && mode_rk(MODE)) {
    double w[6];
    const double ir = cons_to_prim(g, uo, w);
#pragma unroll
    for (int v = 0; v < (STORE_T ? 6 : 5); ++v) io.Pn[v * g.vs + c] = w[v];
    if (io.what & PRIM_CFL) smax = fmax(smax, cfl_rate(g, w, ir));
    if (io.what & PRIM_HEALTH) bad |= health_bits(uo, w[4]);
  }
}

// End of a sweep that stored next-stage primitives: the block's CFL rate
// maximum into its slot, the health bits into the control block. Every thread
// of the block calls it.
__device__ __forceinline__ void finish_prims(const StageIO& io, double smax, int bad) {
  if (io.what & PRIM_CFL) publish_rate(io.partial, blockIdx.y * gridDim.x + blockIdx.x, smax);
  if (bad) atomicOr(&io.ctl->status, bad);
}

// Value of x in the lane below (lane - 1) across the whole wavefront, by one
// DPP move per 32-bit half (wavefront shift right by one lane, a VALU
// operation instead of an LDS permute); lane 0 receives 0.
__device__ __forceinline__ double lane_shr1(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Value of x in the lane above (lane + 1), wavefront shift left by one lane;
// lane 63 receives 0.
__device__ __forceinline__ double lane_shl1(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// x sweep: every interior row holds kXCtx context slots followed by its nx+1
// faces, and the slots of all rows are numbered row-major; slot s of a row is
// face f = s - kXCtx, lying between cells f-1 and f. A wavefront takes 64
// consecutive slots, one per lane. The lane of slot s computes the tangential
// velocity derivatives of cell f+1, and face f takes those of cells f-2..f+1
// from itself and the three lanes below it (context slots only supply the
// first faces of their row); the left-face flux of a cell comes from the lane
// below. The first kXCtx+1 slots of a wavefront overlap its predecessor and
// only seed these shuffles. One slot per lane keeps the kernel at four
// wavefronts per SIMD (126 VGPRs with the default scheme).
constexpr int kXCtx = 3;
constexpr int kXFaces = 64 - (kXCtx + 1);  // faces a wavefront emits

// Interior row `row` (a line of cells along x) of an x sweep in band-major
// order: bands of kXBand consecutive y rows, within a band z outer and y
// inner. The blocks one XCD runs at a time then cover a few planes of a
// narrow band, so the y and z neighbours the tangential stencils read are
// mostly still in that XCD's L2. At 256^3 bands of 32 rows measured 1 %
// faster than 16 or 64 (8: 2 % slower).
constexpr int kXBand = 32;

__device__ __forceinline__ void x_row(const Geom& g, int row, int& j, int& k) {
  const int full = g.n[1] / kXBand;
  const int band_rows = kXBand * g.n[2];
  int band = row / band_rows, h = kXBand;
  if (band >= full) {
    band = full;
    h = g.n[1] - full * kXBand;
  }
  const int r = row - band * band_rows;
  k = r / h;
  j = band * kXBand + (r - k * h);
}

template <int MODE, bool PN, int SCH>
__device__ __forceinline__ void sweep_x_body_face(const double* __restrict__ P, const StageIO& io, const Geom& g,
                                                  int bx) {
  // slot numbering fits in 32 bits (checked when the solver is created)
  const int lane = threadIdx.x & 63;
  const int wave = (bx * kBlock + (int)threadIdx.x) >> 6;
  const int S = g.n[0] + 1 + kXCtx;
  const int total = S * g.n[1] * g.n[2];
  const int first = wave * kXFaces;
  double smax = 0.0;
  int bad = 0;
  if (first < total) {  // uniform per wavefront
    const double dt = mode_rk(MODE) ? *io.dtp : 0.0;
    const int gs = first - (kXCtx + 1) + lane;
    const bool inrange = gs >= 0 && gs < total;
    int f = 0, j = 0, k = 0;
    if (inrange) {
      const int row = gs / S;
      f = gs - row * S - kXCtx;
      x_row(g, row, j, k);
    }
    const bool valid = inrange && f >= 0 && gs >= first - 1;  // lanes whose face flux is used
    // Every lane loads a window inside the padded block (context slots and
    // lanes past the end take face 0 of their row) and computes a flux, so the
    // window loads, the derivative loads and the shuffles need no branch and
    // are in flight together.
    const int fl = f < 0 ? 0 : f;
    const long long c0 = cell_at(g, fl - 3, j, k);
    FaceWindow w;
#pragma unroll
    for (int m = 0; m < 6; ++m) load_prims(P, g.vs, c0 + m, w.q[m]);
#pragma unroll
    for (int m = 0; m < 4; ++m) w.T[m] = P[5 * g.vs + c0 + 1 + m];  // unused without heat flux
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.viscous) tangential_at_flat<0>(g, P, cell_at(g, f + 1, j, k), d);
    // face values of the derivatives from cells f-2..f+1 (lanes - 3 .. lane)
    double tf[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double t2 = lane_shr1(d[v]);
      const double t1 = lane_shr1(t2);
      const double t0 = lane_shr1(t1);
      tf[v] = rc4(t0, t1, t2, d[v]);
    }
    if constexpr (SCH == SCH_W3_NN) w.a = g.nna[c0 + 2];  // alpha of face f (left cell f-1)
    double G[5];
    face_flux_tf<0, SCH>(g, w, tf, G);
    double Gm[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Gm[v] = lane_shr1(G[v]);
    if (valid && gs >= first && f >= 1) {
      double D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v] = (G[v] - Gm[v]) * g.idx[0];
      const long long ce = cell_at(g, f - 1, j, k);
      EmitIn ein;
      emit_fetch<MODE>(io, g.vs, ce, ein);
      emit_put<MODE, PN>(io, g, ce, D, ein, dt, smax, bad);
    }
  }
  if (PN) finish_prims(io, smax, bad);
}

// The same for the cell-centred schemes: the lane of face f reconstructs at
// both faces of cell f (window cells f-2 .. f+2, one smoothness evaluation
// for the two faces) and takes the left state of face f from the lane below,
// which reconstructed cell f-1.
template <int MODE, bool PN, int SCH>
__device__ __forceinline__ void sweep_x_body_pair(const double* __restrict__ P, const StageIO& io, const Geom& g,
                                                  int bx) {
  const int lane = threadIdx.x & 63;
  const int wave = (bx * kBlock + (int)threadIdx.x) >> 6;
  const int S = g.n[0] + 1 + kXCtx;
  const int total = S * g.n[1] * g.n[2];
  const int first = wave * kXFaces;
  double smax = 0.0;
  int bad = 0;
  if (first < total) {  // uniform per wavefront
    const double dt = mode_rk(MODE) ? *io.dtp : 0.0;
    const int gs = first - (kXCtx + 1) + lane;
    const bool inrange = gs >= 0 && gs < total;
    int f = 0, j = 0, k = 0;
    if (inrange) {
      const int row = gs / S;
      f = gs - row * S - kXCtx;
      x_row(g, row, j, k);
    }
    const bool valid = inrange && f >= 0 && gs >= first - 1;  // lanes whose face flux is used
    // every lane loads a window inside the padded block and computes a flux:
    // the context slots before a row's first face reconstruct cell -1 (the
    // left state of face 0 comes from the slot below it), lanes past the end
    // take face 0 of the first row
    const int fl = f < -1 ? -1 : f;
    const long long c0 = cell_at(g, fl - 2, j, k);  // cells f-2 .. f+2
    double q[5][5];
#pragma unroll
    for (int m = 0; m < 5; ++m) load_prims(P, g.vs, c0 + m, q[m]);
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.viscous) tangential_at_flat<0>(g, P, cell_at(g, f + 1, j, k), d);
    // T~ = p/rho of cells f-2 .. f+1 (heat flux only), from the window
    double T[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.heat) {
#pragma unroll
      for (int m = 0; m < 4; ++m) T[m] = div_nr(q[m][4], q[m][0]);
    }
    // face values of the derivatives from cells f-2..f+1 (lanes - 3 .. lane)
    double tf[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double t2 = lane_shr1(d[v]);
      const double t1 = lane_shr1(t2);
      const double t0 = lane_shr1(t1);
      tf[v] = rc4(t0, t1, t2, d[v]);
    }
    double WL[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, WR[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (g.inviscid) {
      double qr[5];
      recon_pair<SCH>(q, qr, WR);
#pragma unroll
      for (int v = 0; v < 5; ++v) WL[v] = lane_shr1(qr[v]);
      check_face_states(g, valid, WL, WR, q[1], q[2], bad);
    }
    double alpha = 0.0;
    if constexpr (SCH == SCH_W3_NN) alpha = g.nna[c0 + 1];  // alpha of face f (left cell f-1)
    double G[5];
    face_flux_states<0, SCH>(g, WL, WR, q, T, tf, alpha, G);
    double Gm[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) Gm[v] = lane_shr1(G[v]);
    if (valid && gs >= first && f >= 1) {
      double D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v] = (G[v] - Gm[v]) * g.idx[0];
      const long long ce = cell_at(g, f - 1, j, k);
      EmitIn ein;
      emit_fetch<MODE>(io, g.vs, ce, ein);
      emit_put<MODE, PN, false>(io, g, ce, D, ein, dt, smax, bad);
    }
  }
  if (PN) finish_prims(io, smax, bad);
  else if (bad && io.ctl) atomicOr(&io.ctl->status, bad);
}

template <int MODE, bool PN = false, int SCH = SCH_JS>
__device__ __forceinline__ void sweep_x_body(const double* __restrict__ P, const StageIO& io, const Geom& g,
                                             int bx) {
  if constexpr (SCH == SCH_ROE || SCH == SCH_Z) sweep_x_body_face<MODE, PN, SCH>(P, io, g, bx);
  else sweep_x_body_pair<MODE, PN, SCH>(P, io, g, bx);
}

// Blocks are taken in XCD-major order, so that the neighbouring rows and
// planes whose velocities the derivative stencils read are being processed in
// the same XCD and stay in its L2.
template <int MODE, bool PN, int SCH>
__global__ void __launch_bounds__(kBlock) k_sweep_x(const double* __restrict__ P, StageIO io, Geom g) {
  if (step_disabled(io.dtp)) return;
  sweep_x_body<MODE, PN, SCH>(P, io, g, xcd_major_block(blockIdx.x, gridDim.x));
}

// Blocks of an x sweep.
__host__ __device__ __forceinline__ int sweep_x_blocks(const Geom& g) {
  const long long slots = (long long)(g.n[0] + 1 + kXCtx) * g.n[1] * g.n[2];
  const long long waves = (slots + kXFaces - 1) / kXFaces;
  return (int)((waves + 3) / 4);
}

// y / z sweep: one lane per (x, other) column segment of Geom::seg cells
// along the axis (kSegSolo for a single grid, kSeg in the serving batch;
// fewer on grids too small to fill the chip with segments that long); lanes
// run along x so every load is coalesced. The segment's first face is
// computed only to seed the left flux.
constexpr int kSeg = 32;
constexpr int kSegSolo = 128;

// y / z sweep body of one lane. Lanes beyond the grid (a partial last block)
// march a valid column too but store nothing, so that every lane reaches the
// block-wide CFL reduction of a sweep that stores next-stage primitives.
template <int AX, int MODE, bool PN, int SCH>
__device__ __forceinline__ void sweep_march_body_face(const double* __restrict__ P, const StageIO& io,
                                                      const Geom& g, int bx, int by) {
  constexpr int OT = AX == 1 ? 2 : 1;  // the other transverse axis
  const int i = bx * 64 + (threadIdx.x & 63);
  const int sl = g.seg;
  const int nseg = (g.n[AX] + sl - 1) / sl;
  const long long col = (long long)by * (kBlock >> 6) + (threadIdx.x >> 6);
  const bool in = i < g.n[0] && col < (long long)g.n[OT] * nseg;
  if (!PN && !in) return;
  double smax = 0.0;
  int bad = 0;
  const long long colc = in ? col : 0;
  const int o = (int)(colc / nseg);
  const int seg = (int)(colc - (long long)o * nseg);
  const int s0 = seg * sl;
  const int s1 = min(s0 + sl, g.n[AX]);
  const long long st = g.s[AX];
  int q3[3];
  q3[0] = in ? i : 0;
  q3[OT] = o;
  q3[AX] = s0 - 3;
  long long c = cell_at(g, q3[0], q3[1], q3[2]);  // window cell 0 (axis index f-2 for face f+1/2)
  const bool dis = g.viscous || g.heat;
  FaceWindow w;
#pragma unroll
  for (int m = 0; m < 6; ++m) load_prims(P, g.vs, c + m * st, w.q[m]);
  if (dis) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      w.T[m] = P[5 * g.vs + c + (1 + m) * st];
      if (g.viscous) tangential_at<AX>(g, P, c + (1 + m) * st, w.tg[m]);
    }
  }
  double Gm[5];
  const double dt = mode_rk(MODE) ? *io.dtp : 0.0;
  for (int f = s0 - 1; f < s1; ++f) {
    // issue the loads of the cell entering the window at the next face, and
    // those of this face's cell update, before this face's arithmetic, so
    // their latency overlaps it
    const bool more = f + 1 < s1;
    EmitIn ein;
    if (f >= s0 && in) emit_fetch<MODE>(io, g.vs, c + 2 * st, ein);  // window cell 2 is cell f
    // The entering cell's derivative stencil: in MODE_WRITE (no update loads
    // in flight) the sixteen raw values are held across the face arithmetic
    // and combined after it, so their latency is hidden; the other modes have
    // no registers to spare for that and combine them at once.
    constexpr bool kDeferTg = MODE == MODE_WRITE;
    double nq[5], nT = 0.0, ntr[4][4], ntg[4] = {0.0, 0.0, 0.0, 0.0};
    if (more) {
      load_prims(P, g.vs, c + 6 * st, nq);
      if (dis) {
        nT = P[5 * g.vs + c + 5 * st];
        if (g.viscous) {
          if (kDeferTg) tangential_load<AX>(g, P, c + 5 * st, ntr);
          else tangential_at<AX>(g, P, c + 5 * st, ntg);
        }
      }
    }
    if (kDeferTg) __builtin_amdgcn_sched_barrier(0);
    if constexpr (SCH == SCH_W3_NN) w.a = g.nna[AX * g.vs + c + 2 * st];  // face f+1/2, left cell f
    double G[5];
    face_flux<AX, SCH>(g, w, G);
    if (f >= s0 && in) {
      double D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v] = (G[v] - Gm[v]) * g.idx[AX];
      emit_put<MODE, PN>(io, g, c + 2 * st, D, ein, dt, smax, bad);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) Gm[v] = G[v];
    if (more) {
      // shift the window by one cell along the axis
#pragma unroll
      for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) w.q[m][v] = w.q[m + 1][v];
#pragma unroll
      for (int v = 0; v < 5; ++v) w.q[5][v] = nq[v];
      c += st;
      if (dis) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          w.T[m] = w.T[m + 1];
#pragma unroll
          for (int v = 0; v < 4; ++v) w.tg[m][v] = w.tg[m + 1][v];
        }
        w.T[3] = nT;
        if (kDeferTg && g.viscous) tangential_combine<AX>(g, ntr, ntg);
#pragma unroll
        for (int v = 0; v < 4; ++v) w.tg[3][v] = ntg[v];
      }
    }
  }
  if (PN) finish_prims(io, smax, bad);
}

// The same for the cell-centred schemes: the lane carries the left state of
// the next face, reconstructed with the right state of the current face from
// the cell between them (one smoothness evaluation for the two faces), so the
// window holds five cells, f-1 .. f+3 for face f+1/2. The segment starts with
// the reconstruction of cell s0-1, for the left state of its first face.
template <int AX, int MODE, bool PN, int SCH>
__device__ __forceinline__ void sweep_march_body_pair(const double* __restrict__ P, const StageIO& io,
                                                      const Geom& g, int bx, int by) {
  constexpr int OT = AX == 1 ? 2 : 1;  // the other transverse axis
  const int i = bx * 64 + (threadIdx.x & 63);
  const int sl = g.seg;
  const int nseg = (g.n[AX] + sl - 1) / sl;
  const long long col = (long long)by * (kBlock >> 6) + (threadIdx.x >> 6);
  const bool in = i < g.n[0] && col < (long long)g.n[OT] * nseg;
  if (!PN && !in) return;
  double smax = 0.0;
  int bad = 0;
  const long long colc = in ? col : 0;
  const int o = (int)(colc / nseg);
  const int seg = (int)(colc - (long long)o * nseg);
  const int s0 = seg * sl;
  const int s1 = min(s0 + sl, g.n[AX]);
  const long long st = g.s[AX];
  int q3[3];
  q3[0] = in ? i : 0;
  q3[OT] = o;
  q3[AX] = s0 - 3;
  long long c = cell_at(g, q3[0], q3[1], q3[2]);  // cell s0-3
  const bool dis = g.viscous || g.heat;
  double q[5][5];   // window: cells f-1 .. f+3 for face f+1/2
  double WLc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // left state of face f+1/2
  {
    double s[5][5];  // cells s0-3 .. s0+1
#pragma unroll
    for (int m = 0; m < 5; ++m) load_prims(P, g.vs, c + m * st, s[m]);
    load_prims(P, g.vs, c + 5 * st, q[4]);
    if (g.inviscid) {
      double unused[5];
      recon_pair<SCH>(s, WLc, unused);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int v = 0; v < 5; ++v) q[m][v] = s[m + 1][v];
  }
  c += st;  // window cell 0: cell f-1 for the first face f = s0-1
  double T[4] = {0.0, 0.0, 0.0, 0.0}, tg[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) tg[m][v] = 0.0;
  if (dis) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (g.heat) T[m] = div_nr(q[m][4], q[m][0]);  // T~ = p/rho from the window
      if (g.viscous) tangential_at<AX>(g, P, c + m * st, tg[m]);
    }
  }
  double Gm[5];
  const double dt = mode_rk(MODE) ? *io.dtp : 0.0;
  for (int f = s0 - 1; f < s1; ++f) {
    // issue the loads of the cell entering the window at the next face, and
    // those of this face's cell update, before this face's arithmetic, so
    // their latency overlaps it
    const bool more = f + 1 < s1;
    EmitIn ein;
    if (f >= s0 && in) emit_fetch<MODE>(io, g.vs, c + st, ein);  // window cell 1 is cell f
    constexpr bool kDeferTg = MODE == MODE_WRITE;
    double nq[5], nT = 0.0, ntr[4][4], ntg[4] = {0.0, 0.0, 0.0, 0.0};
    if (more) {
      load_prims(P, g.vs, c + 5 * st, nq);
      if (dis) {
        if (g.heat) nT = div_nr(q[4][4], q[4][0]);  // cell f+3, window cell 4
        if (g.viscous) {
          if (kDeferTg) tangential_load<AX>(g, P, c + 4 * st, ntr);
          else tangential_at<AX>(g, P, c + 4 * st, ntg);
        }
      }
    }
    if (kDeferTg) __builtin_amdgcn_sched_barrier(0);
    double alpha = 0.0;
    if constexpr (SCH == SCH_W3_NN) alpha = g.nna[AX * g.vs + c + st];  // face f+1/2, left cell f
    double WR[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, qr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double WL[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) WL[v] = WLc[v];
    if (g.inviscid) {
      recon_pair<SCH>(q, qr, WR);  // cell f+1: left state of face f+3/2, right state of f+1/2
      check_face_states(g, true, WL, WR, q[1], q[2], bad);
    }
    double tf[4] = {0.0, 0.0, 0.0, 0.0};
    if (g.viscous) {
#pragma unroll
      for (int v = 0; v < 4; ++v) tf[v] = rc4(tg[0][v], tg[1][v], tg[2][v], tg[3][v]);
    }
    double G[5];
    face_flux_states<AX, SCH>(g, WL, WR, q, T, tf, alpha, G);
    if (f >= s0 && in) {
      double D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v] = (G[v] - Gm[v]) * g.idx[AX];
      emit_put<MODE, PN, false>(io, g, c + st, D, ein, dt, smax, bad);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Gm[v] = G[v];
      WLc[v] = qr[v];
    }
    if (more) {
      // shift the window by one cell along the axis
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) q[m][v] = q[m + 1][v];
#pragma unroll
      for (int v = 0; v < 5; ++v) q[4][v] = nq[v];
      c += st;
      if (dis) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          T[m] = T[m + 1];
#pragma unroll
          for (int v = 0; v < 4; ++v) tg[m][v] = tg[m + 1][v];
        }
        T[3] = nT;
        if (kDeferTg && g.viscous) tangential_combine<AX>(g, ntr, ntg);
#pragma unroll
        for (int v = 0; v < 4; ++v) tg[3][v] = ntg[v];
      }
    }
  }
  if (PN) finish_prims(io, smax, bad);
  else if (bad && io.ctl) atomicOr(&io.ctl->status, bad);
}

template <int AX, int MODE, bool PN = false, int SCH = SCH_JS>
__device__ __forceinline__ void sweep_march_body(const double* __restrict__ P, const StageIO& io,
                                                 const Geom& g, int bx, int by) {
  if constexpr (SCH == SCH_ROE || SCH == SCH_Z) sweep_march_body_face<AX, MODE, PN, SCH>(P, io, g, bx, by);
  else sweep_march_body_pair<AX, MODE, PN, SCH>(P, io, g, bx, by);
}

// The Roe flux splitting does not fit the marching window in the register
// budget of two wavefronts per SIMD; its marches run one wavefront per SIMD,
// which leaves the accumulation registers to the compiler.
template <int AX, int MODE, bool PN, int SCH>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SCH == SCH_ROE ? 1 : 2)))
k_sweep_march(const double* __restrict__ P, StageIO io, Geom g) {
  if (step_disabled(io.dtp)) return;
  // XCD-major block order (see k_sweep_x): consecutive column groups, hence
  // neighbouring planes of the transverse derivatives, share an XCD
  const int logical = xcd_major_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int by = logical / gridDim.x;
  sweep_march_body<AX, MODE, PN, SCH>(P, io, g, logical - by * gridDim.x, by);
}

// Launch shape of a marching sweep along AX (x blocks, y blocks).
template <int AX>
__host__ __device__ __forceinline__ void sweep_march_blocks(const Geom& g, int& gx, int& gy) {
  constexpr int OT = AX == 1 ? 2 : 1;
  const int nseg = (g.n[AX] + g.seg - 1) / g.seg;
  gx = (g.n[0] + 63) / 64;
  gy = (int)(((long long)g.n[OT] * nseg + 3) / 4);
}

// Order of the per-axis sweeps of a stage: y, z, x over the active axes. The
// first writes the right-hand side, the later ones accumulate into it, and x,
// the last whenever it is active, applies the stage update and stores the next
// primitives. The y march goes first because it writes without reading the
// accumulator, which leaves it the registers to hold the loads of its
// tangential stencil (whose z neighbours lie a plane apart) across a face.
constexpr int kSweepAxes[3] = {1, 2, 0};

// Zero a buffer (graph-safe replacement for a memset node).
__global__ void __launch_bounds__(kBlock) k_zero(double* x, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

}  // namespace cfd
