// Forward kernels of one right-hand-side evaluation / TVD-RK3 stage (gfx950).
//
// Per stage:  prim  : U_k -> P = (rho,u,v,w,p,T~) on the padded grid, halos by
//                     gather from their interior source cells (so U's own halo
//                     is never read), plus the CFL rate max in stage 1;
//             grad  : P -> cell-centred velocity gradient (viscous runs only);
//             sweep : one kernel per active axis; each face flux is computed
//                     once in registers and differenced into its two cells.
//                     x: one lane per face, wavefront shuffles carry the
//                        left-face flux; y, z: one lane per column segment
//                        marching along the axis with a register window.
//                     The last active axis applies the RK3 stage update.
#pragma once
#include "physics.hpp"

namespace cfd {

// Device control block of a solver.
struct DevCtl {
  unsigned long long smax;  // max CFL rate of the current step, as the bits of a non-negative double
  double dt;                // step of the current step (0: step disabled, t_end reached)
  int status;               // health bits, see cfd_check
  int pad;
};

constexpr int kBlock = 256;
constexpr int kGradComps = 9;  // d u_a / d x_b stored at component a*3+b

enum SweepMode { MODE_WRITE = 0, MODE_ACC = 1, MODE_ACC_RK = 2, MODE_WRITE_RK = 3 };

struct StageIO {
  double* R;         // right-hand-side accumulator (padded layout)
  const double* Un;  // state at the start of the step
  const double* Uk;  // stage input state
  double* Uout;      // stage output state (may alias Un in the last stage)
  double a, b;       // Uout = a Un + b (Uk + dt R)
  const double* dtp; // step size; nullptr for a plain right-hand side
};

__device__ __forceinline__ bool step_disabled(const double* dtp) { return dtp != nullptr && *dtp == 0.0; }

// ----------------------------------------------------------------------------
// Halo refresh of a padded state (in place). Threads over the padded grid;
// halo cells copy their interior source cell, interior cells do nothing.
__global__ void __launch_bounds__(kBlock) k_fill_halo(double* U, Geom g) {
  const long long total = (long long)g.N[0] * g.N[1] * g.N[2];
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < total;
       c += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(c % g.N[0]) - g.h[0];
    const int j = (int)((c / g.N[0]) % g.N[1]) - g.h[1];
    const int k = (int)(c / ((long long)g.N[0] * g.N[1])) - g.h[2];
    const int si = bc_source(i, g.n[0], g.bc[0], g.bc[1]);
    const int sj = bc_source(j, g.n[1], g.bc[2], g.bc[3]);
    const int sk = bc_source(k, g.n[2], g.bc[4], g.bc[5]);
    if (si == i && sj == j && sk == k) continue;
    const long long s = cell_at(g, si, sj, sk);
#pragma unroll
    for (int v = 0; v < 5; ++v) U[v * g.vs + c] = U[v * g.vs + s];
  }
}

// Conservative interior state from primitive point values W (5 x interior, no halo).
__global__ void __launch_bounds__(kBlock) k_state_init(const double* W, double* U, Geom g) {
  const long long ni = (long long)g.n[0] * g.n[1] * g.n[2];
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < ni;
       s += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(s % g.n[0]);
    const int j = (int)((s / g.n[0]) % g.n[1]);
    const int k = (int)(s / ((long long)g.n[0] * g.n[1]));
    const long long c = cell_at(g, i, j, k);
    const double rho = W[s], u = W[ni + s], v = W[2 * ni + s], w = W[3 * ni + s], p = W[4 * ni + s];
    U[c] = rho;
    U[g.vs + c] = rho * u;
    U[2 * g.vs + c] = rho * v;
    U[3 * g.vs + c] = rho * w;
    U[4 * g.vs + c] = p / (g.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
  }
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// CFL rate of an interior cell: max(sum_d (|u_d| + c)/dx_d, (mu/rho) visc_rate).
__device__ __forceinline__ double cfl_rate(const Geom& g, double rho, const double* u, double p) {
  const double c = sqrt(g.gamma * p / rho);
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (g.act[d]) s += (fabs(u[d]) + c) * g.idx[d];
  if (g.viscous || g.heat) s = fmax(s, (g.mu / rho) * g.visc_rate);
  return s;
}

__device__ __forceinline__ void publish_max(DevCtl* ctl, double s) {
  s = wave_max(s);
  if ((threadIdx.x & 63) == 0 && s > 0.0) atomicMax(&ctl->smax, (unsigned long long)__double_as_longlong(s));
}

// Primitive variables on the padded grid, gathered through the boundary map.
// Over interior cells, `what` bit 0 adds the CFL rate max and bit 1 the health bits.
constexpr int PRIM_CFL = 1, PRIM_HEALTH = 2;

__global__ void __launch_bounds__(kBlock) k_prim(const double* __restrict__ U, double* __restrict__ P,
                                                 Geom g, DevCtl* ctl, int what, const double* dtp) {
  if (step_disabled(dtp)) return;
  const long long total = (long long)g.N[0] * g.N[1] * g.N[2];
  double smax = 0.0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < total;
       c += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(c % g.N[0]) - g.h[0];
    const int j = (int)((c / g.N[0]) % g.N[1]) - g.h[1];
    const int k = (int)(c / ((long long)g.N[0] * g.N[1])) - g.h[2];
    const int si = bc_source(i, g.n[0], g.bc[0], g.bc[1]);
    const int sj = bc_source(j, g.n[1], g.bc[2], g.bc[3]);
    const int sk = bc_source(k, g.n[2], g.bc[4], g.bc[5]);
    const long long s = cell_at(g, si, sj, sk);
    const double rho = U[s];
    const double m0 = U[g.vs + s], m1 = U[2 * g.vs + s], m2 = U[3 * g.vs + s], E = U[4 * g.vs + s];
    const double u[3] = {m0 / rho, m1 / rho, m2 / rho};
    const double p = (g.gamma - 1.0) * (E - 0.5 * (m0 * u[0] + m1 * u[1] + m2 * u[2]));
    P[c] = rho;
    P[g.vs + c] = u[0];
    P[2 * g.vs + c] = u[1];
    P[3 * g.vs + c] = u[2];
    P[4 * g.vs + c] = p;
    P[5 * g.vs + c] = p / rho;
    if (what && s == c) {
      if (what & PRIM_CFL) smax = fmax(smax, cfl_rate(g, rho, u, p));
      if (what & PRIM_HEALTH) {
        int bad = 0;
        if (!isfinite(rho) || !isfinite(m0) || !isfinite(m1) || !isfinite(m2) || !isfinite(E)) bad |= 1;
        if (!(rho > 0.0)) bad |= 2;
        if (!(p > 0.0)) bad |= 4;
        if (bad) atomicOr(&ctl->status, bad);
      }
    }
  }
  if (what & PRIM_CFL) publish_max(ctl, smax);
}

// CFL rate max of a state (interior cells only), for cfd_compute_dt.
__global__ void __launch_bounds__(kBlock) k_cfl(const double* __restrict__ U, Geom g, DevCtl* ctl) {
  const long long ni = (long long)g.n[0] * g.n[1] * g.n[2];
  double smax = 0.0;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ni;
       q += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(q % g.n[0]);
    const int j = (int)((q / g.n[0]) % g.n[1]);
    const int k = (int)(q / ((long long)g.n[0] * g.n[1]));
    const long long s = cell_at(g, i, j, k);
    const double rho = U[s];
    const double m0 = U[g.vs + s], m1 = U[2 * g.vs + s], m2 = U[3 * g.vs + s], E = U[4 * g.vs + s];
    const double u[3] = {m0 / rho, m1 / rho, m2 / rho};
    const double p = (g.gamma - 1.0) * (E - 0.5 * (m0 * u[0] + m1 * u[1] + m2 * u[2]));
    smax = fmax(smax, cfl_rate(g, rho, u, p));
  }
  publish_max(ctl, smax);
}

// Step size of the current step: fixed, or cfl / max rate; clipped to t_end
// (> 0) and zero once t_end is reached. Advances *t, resets the max slot.
__global__ void k_dt(DevCtl* ctl, double cfl, double fixed_dt, double t_end, double* t,
                     double* dt_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double dt = fixed_dt > 0.0 ? fixed_dt : cfl / __longlong_as_double((long long)ctl->smax);
  ctl->smax = 0ull;
  if (t != nullptr && t_end > 0.0) {
    const double rem = t_end - *t;
    dt = rem > 0.0 ? fmin(dt, rem) : 0.0;
  }
  ctl->dt = dt;
  if (t != nullptr) *t = *t + dt;
  if (dt_out != nullptr) *dt_out = dt;
}

// ----------------------------------------------------------------------------
// Cell-centred velocity gradient (fourth-order central, §3.4):
// Gv[a*3+b] = d u_a / d x_b, written wherever coordinate b is interior (the
// only places a face interpolation reads it).
__global__ void __launch_bounds__(kBlock) k_grad(const double* __restrict__ P, double* __restrict__ Gv,
                                                 Geom g, const double* dtp) {
  if (step_disabled(dtp)) return;
  const long long total = (long long)g.N[0] * g.N[1] * g.N[2];
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < total;
       c += (long long)gridDim.x * blockDim.x) {
    const int q[3] = {(int)(c % g.N[0]) - g.h[0], (int)((c / g.N[0]) % g.N[1]) - g.h[1],
                      (int)(c / ((long long)g.N[0] * g.N[1])) - g.h[2]};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (!g.act[b] || q[b] < 0 || q[b] >= g.n[b]) continue;
      const long long st = g.s[b];
      const double i12 = g.idx[b] / 12.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double* u = P + (1 + a) * g.vs + c;
        Gv[(a * 3 + b) * g.vs + c] = (u[-2 * st] - 8.0 * u[-st] + 8.0 * u[st] - u[2 * st]) * i12;
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Face window loads.
__device__ __forceinline__ void load_prims(const double* __restrict__ P, long long vs, long long c,
                                           double* q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) q[v] = P[v * vs + c];
}

// Tangential derivatives at a cell for faces normal to D (see FaceWindow).
template <int D>
__device__ __forceinline__ void load_tangential(const Geom& g, const double* __restrict__ Gv, long long c,
                                                double* tg) {
  constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
  if (g.act[T1]) {
    tg[0] = Gv[(D * 3 + T1) * g.vs + c];
    tg[1] = Gv[(T1 * 3 + T1) * g.vs + c];
  } else {
    tg[0] = 0.0;
    tg[1] = 0.0;
  }
  if (g.act[T2]) {
    tg[2] = Gv[(D * 3 + T2) * g.vs + c];
    tg[3] = Gv[(T2 * 3 + T2) * g.vs + c];
  } else {
    tg[2] = 0.0;
    tg[3] = 0.0;
  }
}

// Write the divergence contribution D = (G+ - G-)/dx of one cell.
template <int MODE>
__device__ __forceinline__ void emit(const StageIO& io, long long vs, long long c, const double* D) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long e = v * vs + c;
    double r;
    if (MODE == MODE_WRITE || MODE == MODE_WRITE_RK) r = -D[v];
    else r = io.R[e] - D[v];
    if (MODE == MODE_WRITE || MODE == MODE_ACC) {
      io.R[e] = r;
    } else {
      const double dt = *io.dtp;
      io.Uout[e] = io.a * io.Un[e] + io.b * (io.Uk[e] + dt * r);
    }
  }
}

// x sweep: faces of all interior rows are numbered row-major, face f of a row
// lying between cells f-1 and f (f = 0..nx). Each wavefront takes
// kXIters*64 consecutive faces, the first of which overlaps the previous
// wavefront's last face and only seeds the carry.
constexpr int kXIters = 4;

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_sweep_x(const double* __restrict__ P,
                                                    const double* __restrict__ Gv, StageIO io, Geom g) {
  if (step_disabled(io.dtp)) return;
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int F = g.n[0] + 1;
  const long long total = (long long)F * g.n[1] * g.n[2];
  constexpr long long Q = 64 * kXIters - 1;
  const long long first = wave * Q;
  if (first >= total) return;  // whole wavefront exits together
  double carry[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < kXIters; ++it) {
    const long long gf = first - 1 + it * 64 + lane;
    const bool valid = gf >= 0 && gf < total;
    double G[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    long long row = 0;
    int f = 0;
    if (valid) {
      row = gf / F;
      f = (int)(gf - row * F);
      const int j = (int)(row % g.n[1]);
      const int k = (int)(row / g.n[1]);
      FaceWindow w;
      const long long c0 = cell_at(g, f - 3, j, k);
#pragma unroll
      for (int m = 0; m < 6; ++m) load_prims(P, g.vs, c0 + m, w.q[m]);
      if (g.viscous || g.heat) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          w.T[m] = P[5 * g.vs + c0 + 1 + m];
          if (g.viscous) load_tangential<0>(g, Gv, c0 + 1 + m, w.tg[m]);
        }
      }
      face_flux<0>(g, w, G);
    }
    double Gm[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double up = __shfl_up(G[v], 1, 64);
      Gm[v] = lane == 0 ? carry[v] : up;
      carry[v] = __shfl(G[v], 63, 64);
    }
    if (valid && gf >= first && f >= 1) {
      const int j = (int)(row % g.n[1]);
      const int k = (int)(row / g.n[1]);
      double D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v] = (G[v] - Gm[v]) * g.idx[0];
      emit<MODE>(io, g.vs, cell_at(g, f - 1, j, k), D);
    }
  }
}

// y / z sweep: one lane per (x, other) column segment of kSeg cells along the
// axis; lanes run along x so every load is coalesced. The segment's first
// face is computed only to seed the left flux.
constexpr int kSeg = 32;

template <int AX, int MODE>
__global__ void __launch_bounds__(kBlock) k_sweep_march(const double* __restrict__ P,
                                                        const double* __restrict__ Gv, StageIO io,
                                                        Geom g) {
  if (step_disabled(io.dtp)) return;
  constexpr int OT = AX == 1 ? 2 : 1;  // the other transverse axis
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int nseg = (g.n[AX] + kSeg - 1) / kSeg;
  const long long col = (long long)blockIdx.y * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= g.n[0] || col >= (long long)g.n[OT] * nseg) return;
  const int o = (int)(col / nseg);
  const int seg = (int)(col - (long long)o * nseg);
  const int s0 = seg * kSeg;
  const int s1 = min(s0 + kSeg, g.n[AX]);
  const long long st = g.s[AX];
  int q3[3];
  q3[0] = i;
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
      if (g.viscous) load_tangential<AX>(g, Gv, c + (1 + m) * st, w.tg[m]);
    }
  }
  double Gm[5];
  for (int f = s0 - 1; f < s1; ++f) {
    double G[5];
    face_flux<AX>(g, w, G);
    if (f >= s0) {
      double D[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v] = (G[v] - Gm[v]) * g.idx[AX];
      emit<MODE>(io, g.vs, c + 2 * st, D);  // window cell 2 is cell f
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) Gm[v] = G[v];
    if (f + 1 < s1) {
      // shift the window by one cell along the axis
#pragma unroll
      for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int v = 0; v < 5; ++v) w.q[m][v] = w.q[m + 1][v];
      c += st;
      load_prims(P, g.vs, c + 5 * st, w.q[5]);
      if (dis) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          w.T[m] = w.T[m + 1];
#pragma unroll
          for (int v = 0; v < 4; ++v) w.tg[m][v] = w.tg[m + 1][v];
        }
        w.T[3] = P[5 * g.vs + c + 4 * st];
        if (g.viscous) load_tangential<AX>(g, Gv, c + 4 * st, w.tg[3]);
      }
    }
  }
}

// Zero a buffer (graph-safe replacement for a memset node).
__global__ void __launch_bounds__(kBlock) k_zero(double* x, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

}  // namespace cfd
