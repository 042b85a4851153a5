// libcfd host side: the C ABI of include/cfd.h over the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cfd.h"
#include "kernels_adj.hpp"
#include "kernels_nn.hpp"
#include "kernels_fwd.hpp"

using namespace cfd;

namespace {

thread_local std::string g_err;

cfd_status fail(cfd_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define CFD_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(CFD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CFD_LAUNCHED()                                                                   \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess) return fail(CFD_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

unsigned grid_for(long long n, long long cap = 1 << 20) {
  long long b = (n + kBlock - 1) / kBlock;
  return (unsigned)std::max(1LL, std::min(b, cap));
}

// Plane-indexed launch over the padded grid (see PlaneIdx).
dim3 plane_grid(const Geom& g) {
  return dim3((unsigned)(((long long)g.N[0] * g.N[1] + kBlock - 1) / kBlock), (unsigned)g.N[2]);
}

}  // namespace

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const void* key[3] = {nullptr, nullptr, nullptr};
  double kd[2] = {0.0, 0.0};
  int mode = -1;
};

// Components of a primitive buffer (rho, u, v, w, p, T~) per padded cell.
constexpr int kPrimComps = 6;

struct cfd_solver {
  cfd_config cfg;
  Geom g;
  long long ncell = 0;  // padded cells
  long long nint = 0;   // interior cells
  double* U1 = nullptr;
  double* U2 = nullptr;
  double* P = nullptr;    // 6 x padded (= Pb[0])
  double* Pb[3] = {nullptr, nullptr, nullptr};  // primitives of the stage inputs of a step
  double* Racc = nullptr; // 5 x padded
  double* Racc2 = nullptr; // 5 x padded: the second march's accumulator (grids with three active axes)
  double* A1 = nullptr;   // adjoint scratch (allocated on the first adjoint call)
  double* A2 = nullptr;
  double* A3 = nullptr;
  double* Wbar = nullptr; // 6 x padded
  double* Dbar = nullptr; // 9 x padded (viscous runs)
  // a second pair, cleared on the side stream during one right-hand-side
  // adjoint for the next one of the same step adjoint (the two swap)
  double* Wbar2 = nullptr;
  double* Dbar2 = nullptr;
  double* partial = nullptr;  // CFL rate maxima slots (kCflSlots)
  double* nna = nullptr;      // Rusanov-NN alpha per face (3 x padded)
  double* nntape = nullptr;   // Rusanov-NN per-face records of the reverse (adjoint scratch)
  double* nnbar = nullptr;    // caller's weight-gradient accumulator (may be NULL)
  NNTape tape{};
  int npart = 0;
  DevCtl* ctl = nullptr;
  hipStream_t cap = nullptr;
  hipStream_t side = nullptr;  // the dissipative face reverses run here, beside the inviscid ones
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  GraphCache graph;
};

static cfd_status validate(const cfd_config* c) {
  if (!c) return fail(CFD_EINVAL, "config is NULL");
  if (c->nh < 3) return fail(CFD_EINVAL, "nh must be >= 3");
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 1) return fail(CFD_EINVAL, "n must be >= 1 on every axis");
    if (c->n[d] > 1 && c->n[d] < c->nh) return fail(CFD_EINVAL, "active axes need n >= nh");
    if (!(c->hi[d] > c->lo[d]) || !std::isfinite(c->hi[d] - c->lo[d]))
      return fail(CFD_EINVAL, "box must satisfy lo < hi");
    for (int s = 0; s < 2; ++s)
      if (c->bc[2 * d + s] != CFD_BC_PERIODIC && c->bc[2 * d + s] != CFD_BC_ZERO_GRADIENT &&
          c->bc[2 * d + s] != CFD_BC_REFLECT)
        return fail(CFD_EINVAL, "unknown boundary type");
    if (c->n[d] > 1 && ((c->bc[2 * d] == CFD_BC_PERIODIC) != (c->bc[2 * d + 1] == CFD_BC_PERIODIC)))
      return fail(CFD_EINVAL, "periodic boundaries come in pairs");
  }
  if (c->n[0] == 1 && c->n[1] == 1 && c->n[2] == 1) return fail(CFD_EINVAL, "no active axis");
  if (!(c->gamma > 1.0)) return fail(CFD_EINVAL, "gamma must be > 1");
  if (!(c->mu >= 0.0)) return fail(CFD_EINVAL, "mu must be >= 0");
  if (!(c->prandtl > 0.0)) return fail(CFD_EINVAL, "prandtl must be > 0");
  if (!(c->cfl > 0.0 && c->cfl <= 1.0)) return fail(CFD_EINVAL, "cfl must lie in (0, 1]");
  if (c->flags & ~1023u) return fail(CFD_EINVAL, "unknown physics flag");
  if ((c->flags & CFD_F_SAFE_RECON) && (c->flags & CFD_F_ROE))
    return fail(CFD_EINVAL, "safe reconstruction applies to reconstructed primitives (flag SAFE_RECON with ROE)");
  if ((c->flags & CFD_F_RUSANOV_NN) &&
      ((c->flags & (CFD_F_ROE | CFD_F_WENOZ | CFD_F_RUSANOV)) || !(c->flags & CFD_F_WENO3)))
    return fail(CFD_EINVAL, "the Rusanov-NN flux runs with WENO3-JS (flag RUSANOV_NN needs WENO3, without ROE, WENOZ, RUSANOV)");
  if ((c->flags & CFD_F_ROE) && (c->flags & (CFD_F_WENOZ | CFD_F_WENO3 | CFD_F_RUSANOV)))
    return fail(CFD_EINVAL, "the Roe flux splitting reconstructs with WENO5-JS (flag WENOZ, WENO3 or RUSANOV with ROE)");
  if ((c->flags & CFD_F_WENOZ) && (c->flags & (CFD_F_WENO3 | CFD_F_RUSANOV)))
    return fail(CFD_EINVAL, "WENO5-Z is combined with HLLC only (flag WENO3 or RUSANOV with WENOZ)");
  // index ranges of the kernels: faces per axis and padded planes in 32 bits,
  // padded z extent within the launch grid's y limit
  long long N[3];
  for (int d = 0; d < 3; ++d) N[d] = c->n[d] > 1 ? c->n[d] + 2LL * c->nh : 1;
  for (int d = 0; d < 3; ++d) {
    // (the x sweep numbers its faces with 3 extra slots per row, the x
    // adjoint its cells with 6)
    long long faces = (long long)c->n[0] * c->n[1] * c->n[2] / c->n[d] * (c->n[d] + (d == 0 ? 6 : 1));
    if (faces >= (1LL << 31)) return fail(CFD_EINVAL, "grid too large: faces per axis must fit in 31 bits");
    if ((c->flags & CFD_F_RUSANOV_NN) && faces >= (1LL << 29))
      return fail(CFD_EINVAL, "grid too large: the Rusanov-NN kernels run four lanes per face (faces per axis < 2^29)");
  }
  if (N[0] * N[1] >= (1LL << 31) || N[2] > 65535) return fail(CFD_EINVAL, "grid too large for the launch shape");
  return CFD_OK;
}

static void make_geom(const cfd_config& c, Geom& g) {
  std::memset(&g, 0, sizeof(g));
  double inv2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c.n[d];
    g.act[d] = c.n[d] > 1;
    g.h[d] = g.act[d] ? c.nh : 0;
    g.N[d] = g.n[d] + 2 * g.h[d];
    g.dx[d] = (c.hi[d] - c.lo[d]) / c.n[d];
    g.idx[d] = 1.0 / g.dx[d];
    if (g.act[d]) inv2 += 1.0 / (g.dx[d] * g.dx[d]);
  }
  for (int s = 0; s < 6; ++s) g.bc[s] = c.bc[s];
  g.s[0] = 1;
  g.s[1] = g.N[0];
  g.s[2] = (long long)g.N[0] * g.N[1];
  g.vs = (long long)g.N[0] * g.N[1] * g.N[2];
  g.gamma = c.gamma;
  g.gm1i = 1.0 / (c.gamma - 1.0);
  g.mu = c.mu;
  g.kappa = c.gamma * c.mu / ((c.gamma - 1.0) * c.prandtl);
  g.cfl = c.cfl;
  g.visc_rate = 2.0 * std::max(4.0 / 3.0, c.gamma / c.prandtl) * inv2;
  g.inviscid = (c.flags & CFD_F_INVISCID) ? 1 : 0;
  g.wenoz = (c.flags & CFD_F_WENOZ) ? 1 : 0;
  g.roe = (c.flags & CFD_F_ROE) ? 1 : 0;
  g.weno3 = (c.flags & CFD_F_WENO3) ? 1 : 0;
  g.rusanov = (c.flags & CFD_F_RUSANOV) ? 1 : 0;
  g.rk2 = (c.flags & CFD_F_RK2) ? 1 : 0;
  g.seg = kSeg;
  g.nn = (c.flags & CFD_F_RUSANOV_NN) ? 1 : 0;
  g.safe = (c.flags & CFD_F_SAFE_RECON) ? 1 : 0;
  g.viscous = ((c.flags & CFD_F_VISCOUS) && c.mu > 0.0) ? 1 : 0;
  g.heat = ((c.flags & CFD_F_HEAT) && c.mu > 0.0) ? 1 : 0;
}

// March segment length of a single-grid solver: kSegSolo, halved (down to 8
// cells) while a y or z march would run fewer than 1024 wavefronts, so that
// small grids spread their marches over more lanes (each segment recomputes
// its seed face and, in the adjoint, a reconstruction pair). Long segments
// pay that less often: at 256^3 the marches run 128-cell segments (2048
// wavefronts, one per wavefront slot at two per SIMD), 2-3 % faster than
// 32-cell ones; 16-cell ones are 4 % slower. The serving batch chooses its
// own (batch_segment): it fills the chip with many grids.
static void choose_segment(Geom& g) {
  auto waves = [&](int seg) {
    long long w = -1;
    for (int ax = 1; ax < 3; ++ax) {
      if (!g.act[ax]) continue;
      const int ot = ax == 1 ? 2 : 1;
      const long long v = (long long)((g.n[0] + 63) / 64) * g.n[ot] * ((g.n[ax] + seg - 1) / seg);
      w = w < 0 ? v : std::min(w, v);
    }
    return w;
  };
  g.seg = kSegSolo;
  while (g.seg > 8 && waves(g.seg) >= 0 && waves(g.seg) < 1024) g.seg /= 2;
}

// ---------------------------------------------------------------------------
// Enqueue the primitive pass of stage input Uk; `what` selects the CFL max
// and the health check (PRIM_* bits).
static cfd_status enqueue_prim(cfd_solver* s, const double* Uk, int what, const double* dtp,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_prim, plane_grid(s->g), dim3(kBlock), 0, st, Uk, s->P, s->g, s->ctl, what, dtp,
                     s->partial);
  CFD_LAUNCHED();
  return CFD_OK;
}

template <int D, bool PN, int SCH>
static void launch_sweep_r(cfd_solver* s, int mode, const double* P, const StageIO& io, hipStream_t st) {
  const Geom& g = s->g;
  if (D == 0) {
    const dim3 grid((unsigned)sweep_x_blocks(g));
    switch (mode) {
      case MODE_WRITE: hipLaunchKernelGGL((k_sweep_x<MODE_WRITE, false, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      case MODE_ACC: hipLaunchKernelGGL((k_sweep_x<MODE_ACC, false, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      case MODE_ACC_RK: hipLaunchKernelGGL((k_sweep_x<MODE_ACC_RK, PN, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      case MODE_ACC2_RK: hipLaunchKernelGGL((k_sweep_x<MODE_ACC2_RK, PN, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      default: hipLaunchKernelGGL((k_sweep_x<MODE_WRITE_RK, PN, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
    }
  } else {
    constexpr int AX = D == 0 ? 1 : D;
    int gx, gy;
    sweep_march_blocks<AX>(g, gx, gy);
    const dim3 grid(gx, gy);
    switch (mode) {
      case MODE_WRITE: hipLaunchKernelGGL((k_sweep_march<AX, MODE_WRITE, false, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      case MODE_ACC: hipLaunchKernelGGL((k_sweep_march<AX, MODE_ACC, false, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      case MODE_ACC_RK: hipLaunchKernelGGL((k_sweep_march<AX, MODE_ACC_RK, PN, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
      default: hipLaunchKernelGGL((k_sweep_march<AX, MODE_WRITE_RK, PN, SCH>), grid, dim3(kBlock), 0, st, P, io, g); break;
    }
  }
}

// The convective scheme (WENO5-JS or WENO5-Z with HLLC, or the Roe flux
// splitting) is a template parameter of the sweep kernels; pick the
// instantiation for the solver's configuration.
template <int D, bool PN>
static void launch_sweep(cfd_solver* s, int mode, const double* P, const StageIO& io, hipStream_t st) {
  const Geom& g = s->g;
  if (g.nn) launch_sweep_r<D, PN, SCH_W3_NN>(s, mode, P, io, st);
  else if (g.roe) launch_sweep_r<D, PN, SCH_ROE>(s, mode, P, io, st);
  else if (g.wenoz) launch_sweep_r<D, PN, SCH_Z>(s, mode, P, io, st);
  else if (g.weno3 && g.rusanov) launch_sweep_r<D, PN, SCH_W3_RUS>(s, mode, P, io, st);
  else if (g.weno3) launch_sweep_r<D, PN, SCH_W3>(s, mode, P, io, st);
  else if (g.rusanov) launch_sweep_r<D, PN, SCH_JS_RUS>(s, mode, P, io, st);
  else launch_sweep_r<D, PN, SCH_JS>(s, mode, P, io, st);
}

template <bool PN>
static void launch_sweep_axis(cfd_solver* s, int d, int mode, const double* P, const StageIO& io, hipStream_t st) {
  if (d == 0) launch_sweep<0, PN>(s, mode, P, io, st);
  else if (d == 1) launch_sweep<1, PN>(s, mode, P, io, st);
  else launch_sweep<2, PN>(s, mode, P, io, st);
}

// A stage of a grid with three active axes splits its accumulator: the y and
// z marches write R and R2, the x sweep reads both (MODE_ACC2_RK).
static bool stage_split(const Geom& g) { return g.act[0] && g.act[1] && g.act[2]; }

// The first and last active axes in sweep order (kSweepAxes).
static void sweep_order(const Geom& g, int& first, int& last) {
  first = last = -1;
  for (int d : kSweepAxes)
    if (g.act[d]) {
      if (first < 0) first = d;
      last = d;
    }
}

// Enqueue the per-axis sweeps over primitives P. With rk set, the last active
// axis applies the stage update into io.Uout (and, with io.Pn set, stores the
// primitives of the updated interior cells into io.Pn, whose halo is then
// refreshed); otherwise io.R receives the full right-hand side.
// Faces normal to axis d (interior cells of the other axes).
static long long faces_of(const Geom& g, int d) {
  return (long long)g.n[0] * g.n[1] * g.n[2] / g.n[d] * (g.n[d] + 1);
}

// Rusanov-NN launch split: 64 faces per block per active axis (the network
// kernels run four lanes per face), record offsets in axis order.
static NNAxes nn_axes(const Geom& g, long long& blocks) {
  NNAxes a{};
  blocks = 0;
  long long off = 0;
  for (int d = 0; d < 3; ++d) {
    const long long F = g.act[d] ? faces_of(g, d) : 0;
    a.blk[d] = (int)((F + 63) / 64);
    a.off[d] = off;
    off += F;
    blocks += a.blk[d];
  }
  return a;
}

// Rusanov-NN: alpha of every face of the active axes from primitives P.
static cfd_status enqueue_nn_alpha(cfd_solver* s, const double* P, hipStream_t st) {
  const Geom& g = s->g;
  if (!g.nnw) return fail(CFD_EINVAL, "Rusanov-NN weights are not set (cfd_set_nn_weights)");
  long long blocks = 0;
  const NNAxes ax = nn_axes(g, blocks);
  hipLaunchKernelGGL(k_nn_alpha, dim3((unsigned)blocks), dim3(kBlock), 0, st, P, g, ax);
  CFD_LAUNCHED();
  return CFD_OK;
}

static cfd_status enqueue_fluxes(cfd_solver* s, const double* P, const StageIO& io, bool rk, hipStream_t st) {
  const Geom& g = s->g;
  if (g.nn) {
    cfd_status rc = enqueue_nn_alpha(s, P, st);
    if (rc) return rc;
  }
  int first = -1, last = -1;
  sweep_order(g, first, last);
  for (int d : kSweepAxes) {
    if (!g.act[d]) continue;
    int mode;
    StageIO iod = io;
    if (d == last && rk) {
      mode = d == first ? MODE_WRITE_RK : (stage_split(g) && d == 0 ? MODE_ACC2_RK : MODE_ACC_RK);
    } else if (rk && stage_split(g)) {
      // the marches before the x sweep each write their own accumulator
      mode = MODE_WRITE;
      if (d != first) iod.R = const_cast<double*>(io.R2);
    } else {
      mode = d == first ? MODE_WRITE : MODE_ACC;
    }
    if (d == last && rk && io.Pn) launch_sweep_axis<true>(s, d, mode, P, iod, st);
    else launch_sweep_axis<false>(s, d, mode, P, iod, st);
    CFD_LAUNCHED();
  }
  if (rk && io.Pn) {
    hipLaunchKernelGGL(k_prim_halo, dim3(halo_blocks(g)), dim3(kBlock), 0, st, io.Pn, g, io.dtp);
    CFD_LAUNCHED();
  }
  return CFD_OK;
}

// Clear the CFL slots before a fresh accumulation: the last step of a run
// leaves the maxima of its final state there, consumed by nobody.
static cfd_status enqueue_clear_slots(cfd_solver* s, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, st, s->partial, (long long)s->npart);
  CFD_LAUNCHED();
  return CFD_OK;
}

// Step prologue: the primitives of U into Pb[0] with the health bits and,
// for a CFL step, the CFL rate maxima of U.
static cfd_status enqueue_step_prologue(cfd_solver* s, const double* U, bool cfl, hipStream_t st) {
  if (cfl) {
    cfd_status rc = enqueue_clear_slots(s, st);
    if (rc) return rc;
  }
  return enqueue_prim(s, U, PRIM_HEALTH | (cfl ? PRIM_CFL : 0), nullptr, st);
}

// Enqueue one TVD-RK3 step on U in place; Pb[0] must hold the primitives of U
// and, for a CFL step, the CFL slots its rate maxima (the prologue, or the
// previous step, leaves both). fixed_dt > 0 fixes the step; otherwise the
// CFL step of Un, clipped against *t_dev and t_end when t_dev is given.
// dt_out (nullable) receives the step. Each stage's last sweep stores the
// primitives of its output for the next stage (Pb[0] -> Pb[1] -> Pb[2] ->
// Pb[0]); the third also the health bits of U^{n+1} and, for CFL steps, its
// CFL rate maxima, so consecutive steps need no separate primitive pass.
// Pst (nullable): the primitives of the three stage inputs are read from and
// written to Pst[0] (which must hold those of Un), Pst[1] and Pst[2] instead
// of the solver's ring; the third stage still writes Pb[0].
static cfd_status enqueue_step(cfd_solver* s, double* U, double fixed_dt, double t_end, double* t_dev,
                               double* dt_out, hipStream_t st, double* U1 = nullptr, double* U2 = nullptr,
                               double* const* Pst = nullptr) {
  if (!U1) U1 = s->U1;
  if (!U2) U2 = s->U2;
  double* const P0 = Pst ? Pst[0] : s->Pb[0];
  double* const P1 = Pst ? Pst[1] : s->Pb[1];
  double* const P2 = Pst ? Pst[2] : s->Pb[2];
  const double* dtp = &s->ctl->dt;
  const bool cfl = !(fixed_dt > 0.0);
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(kBlock), 0, st, s->ctl, s->g.cfl, fixed_dt, t_end, t_dev, dt_out,
                     s->partial, s->npart);
  CFD_LAUNCHED();
  StageIO io{};
  io.R = s->Racc;
  io.R2 = s->Racc2;
  io.Un = U;
  io.dtp = dtp;
  io.partial = s->partial;
  io.ctl = s->ctl;
  cfd_status rc;
  // stage 1: U1 = Un + dt R(Un)
  io.Uk = U;
  io.Uout = U1;
  io.a = 0.0;
  io.b = 1.0;
  io.Pn = P1;
  io.what = PRIM_HEALTH;  // health bits of every stage state
  if ((rc = enqueue_fluxes(s, P0, io, true, st))) return rc;
  if (s->g.rk2) {
    // TVD-RK2, second stage: Un+1 = 1/2 Un + 1/2 (U1 + dt R(U1)), in place on U
    io.Uk = U1;
    io.Uout = U;
    io.a = 0.5;
    io.b = 0.5;
    io.Pn = s->Pb[0];
    io.what = PRIM_HEALTH | (cfl ? PRIM_CFL : 0);
    return enqueue_fluxes(s, P1, io, true, st);
  }
  // stage 2: U2 = 3/4 Un + 1/4 (U1 + dt R(U1))
  io.Uk = U1;
  io.Uout = U2;
  io.a = 0.75;
  io.b = 0.25;
  io.Pn = P2;
  if ((rc = enqueue_fluxes(s, P1, io, true, st))) return rc;
  // stage 3: Un+1 = 1/3 Un + 2/3 (U2 + dt R(U2)), in place on U
  io.Uk = U2;
  io.Uout = U;
  io.a = 1.0 / 3.0;
  io.b = 2.0 / 3.0;
  io.Pn = s->Pb[0];
  io.what = PRIM_HEALTH | (cfl ? PRIM_CFL : 0);
  return enqueue_fluxes(s, P2, io, true, st);
}

static cfd_status enqueue_fill_halo(cfd_solver* s, double* U, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_halo, plane_grid(s->g), dim3(kBlock), 0, st, U, s->g);
  CFD_LAUNCHED();
  return CFD_OK;
}

// Replay `n` copies of a captured single-step graph on stream st. The graph
// is re-captured when its key (pointers and scalars) changes.
static cfd_status run_graph(cfd_solver* s, double* U, int mode, double fixed_dt, double t_end, double* t_dev,
                            int n, hipStream_t st) {
  GraphCache& gc = s->graph;
  const bool hit = gc.exec && gc.mode == mode && gc.key[0] == U && gc.key[1] == t_dev &&
                   gc.kd[0] == fixed_dt && gc.kd[1] == t_end;
  if (!hit) {
    if (gc.exec) {
      CFD_HIP(hipGraphExecDestroy(gc.exec));
      gc.exec = nullptr;
    }
    hipGraph_t graph;
    CFD_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    cfd_status rc = enqueue_step(s, U, fixed_dt, t_end, t_dev, nullptr, s->cap);
    hipError_t ec = hipStreamEndCapture(s->cap, &graph);
    if (rc) return rc;
    if (ec != hipSuccess) return fail(CFD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    hipError_t ei = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      gc.exec = nullptr;
      return fail(CFD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    gc.mode = mode;
    gc.key[0] = U;
    gc.key[1] = t_dev;
    gc.kd[0] = fixed_dt;
    gc.kd[1] = t_end;
  }
  cfd_status rc = enqueue_step_prologue(s, U, !(fixed_dt > 0.0), st);
  if (rc) return rc;
  for (int i = 0; i < n; ++i) CFD_HIP(hipGraphLaunch(gc.exec, st));
  return CFD_OK;
}

// ---------------------------------------------------------------------------
// Adjoint scratch: two adjoint states, the primitive-adjoint and the
// derivative-adjoint accumulators. Allocated on the first adjoint call.
static cfd_status ensure_adjoint_scratch(cfd_solver* s) {
  if (s->A1) return CFD_OK;
  // the marching face reverses address cells with 32-bit offsets
  if (s->ncell >= (1LL << 31)) return fail(CFD_EINVAL, "grid too large for the adjoint (2^31 padded cells or more)");
  const size_t st = sizeof(double) * 5 * (size_t)s->ncell;
  bool ok = hipMalloc(&s->A1, st) == hipSuccess && hipMalloc(&s->A2, st) == hipSuccess &&
            hipMalloc(&s->Wbar, sizeof(double) * 6 * (size_t)s->ncell) == hipSuccess &&
            hipMalloc(&s->Wbar2, sizeof(double) * 6 * (size_t)s->ncell) == hipSuccess;
  if (ok && s->g.viscous)
    ok = hipMalloc(&s->Dbar, sizeof(double) * kGradComps * (size_t)s->ncell) == hipSuccess &&
         hipMalloc(&s->Dbar2, sizeof(double) * kGradComps * (size_t)s->ncell) == hipSuccess;
  long long F = 0;
  if (s->g.nn) {
    for (int d = 0; d < 3; ++d)
      if (s->g.act[d]) F += faces_of(s->g, d);
    ok = ok && hipMalloc(&s->nntape, sizeof(double) * (kNNTapePerFace * (size_t)F + kNNChunks * kNNParams)) ==
                   hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    double* b[] = {s->A1, s->A2, s->Wbar, s->Dbar, s->Wbar2, s->Dbar2, s->nntape};
    for (double* x : b)
      if (x) (void)hipFree(x);
    s->A1 = s->A2 = s->Wbar = s->Dbar = s->Wbar2 = s->Dbar2 = s->nntape = nullptr;
    return fail(CFD_ENOMEM, "adjoint scratch allocation failed");
  }
  if (s->g.nn) {
    NNTape& t = s->tape;
    t.F = F;
    for (int l = 0; l < 3; ++l) {
      t.z[l] = s->nntape + (size_t)l * kNNH * F;
      t.d[l] = s->nntape + (size_t)(3 + l) * kNNH * F;
    }
    t.f = s->nntape + (size_t)6 * kNNH * F;
    t.d4 = t.f + (size_t)kNNIn * F;
    t.part = t.d4 + F;
  }
  return CFD_OK;
}

// The face reverses of axis D: the inviscid part on st, the dissipative part on sd.
template <int D>
static void launch_face_adj(cfd_solver* s, const double* P, const double* Rbar, double rscale, hipStream_t st,
                            hipStream_t sd) {
  const Geom& g = s->g;
  if constexpr (D == 0) {
    const long long rows = (long long)g.n[1] * g.n[2];
    auto blocks = [&](long long slots, int per_wave) {
      const long long waves = (slots + per_wave - 1) / per_wave;
      return dim3((unsigned)((waves + (kBlock / 64) - 1) / (kBlock / 64)));
    };
    if (g.inviscid)
      hipLaunchKernelGGL(k_xadj_inv, blocks((g.n[0] + 6) * rows, kXInvNew), dim3(kBlock), 0, st, P, Rbar, rscale,
                         s->Wbar, g);
    if (g.viscous || g.heat)
      hipLaunchKernelGGL(k_xadj_dis, blocks((g.n[0] + 1 + kXDisCtx) * rows, kXDisNew), dim3(kBlock), 0, sd, P,
                         Rbar, rscale, s->Wbar, s->Dbar, g);
  } else {
    int gx = 0, gy = 0;
    sweep_march_blocks<D>(g, gx, gy);
    if (g.inviscid)
      hipLaunchKernelGGL(k_march_adj_inv<D>, dim3(gx, gy), dim3(kBlock), 0, st, P, Rbar, rscale, s->Wbar, g);
    if (g.viscous || g.heat)
      hipLaunchKernelGGL(k_march_adj_dis<D>, dim3(gx, gy), dim3(kBlock), 0, sd, P, Rbar, rscale, s->Wbar, s->Dbar,
                         g);
  }
}

// out.out = (the combination in out) + (dR/dU(U))^T (rscale Rbar) at the
// interior cells, with U given by its primitives P (padded, halos included;
// rho, u, v, w, p are read).
// Padded cells from which a right-hand-side adjoint uses its second stream.
constexpr long long kAdjForkMinCells = 1LL << 18;

// Clear the accumulators Wbar, Dbar (graph-safe fill kernels).
static void enqueue_clear_adj(cfd_solver* s, double* Wb, double* Db, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(grid_for(6 * s->ncell)), dim3(kBlock), 0, st, Wb, 6 * s->ncell);
  if (s->g.viscous)
    hipLaunchKernelGGL(k_zero, dim3(grid_for(kGradComps * s->ncell)), dim3(kBlock), 0, st, Db,
                       kGradComps * s->ncell);
}

// cleared: s->Wbar, s->Dbar are already zero (cleared on the side stream by
// the previous call of the same step adjoint); clear_next: clear the other
// pair on the side stream, after the face reverses there, for the next call.
// The pairs swap at the end.
static cfd_status enqueue_rhs_adjoint(cfd_solver* s, const double* P, const double* Rbar,
                                      double rscale, const AdjOut& out, hipStream_t st, bool cleared = false,
                                      bool clear_next = false) {
  const Geom& g = s->g;
  // Small grids (a few microseconds per kernel) keep everything on one
  // stream: there the fork and join cost more than the overlap gains, and
  // each call clears its own pair.
  const bool big = s->ncell >= kAdjForkMinCells;
  cleared = cleared && big;
  clear_next = clear_next && big;
  if (!cleared) {
    enqueue_clear_adj(s, s->Wbar, s->Dbar, st);
    CFD_LAUNCHED();
  }
  // the inviscid reverses (FP64-bound) and the dissipative ones (bound by
  // their stencil loads) add to disjoint or commuting entries of Wbar and
  // Dbar: they run side by side on two streams, and the side stream then
  // clears the next pair
  const bool side_faces = big && !g.nn && g.inviscid && (g.viscous || g.heat);
  const bool fork = side_faces || clear_next;
  hipStream_t sd = st;
  if (fork) {
    CFD_HIP(hipEventRecord(s->ev_fork, st));
    CFD_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
    if (side_faces) sd = s->side;
  }
  if (g.nn) {
    // Rusanov-NN faces of every axis in one launch, then the weight gradient
    if (!g.nnw) return fail(CFD_EINVAL, "Rusanov-NN weights are not set (cfd_set_nn_weights)");
    long long blocks = 0;
    const NNAxes ax = nn_axes(g, blocks);
    hipLaunchKernelGGL(k_face_adj_nn, dim3((unsigned)blocks), dim3(kBlock), 0, st, P, Rbar, rscale, s->Wbar, g,
                       s->tape, ax);
    CFD_LAUNCHED();
    if (s->nnbar) {
      hipLaunchKernelGGL(k_nn_wgrad, dim3(kNNRows * kNNChunks), dim3(kBlock), 0, st, s->tape);
      hipLaunchKernelGGL(k_nn_wgrad_sum, dim3((kNNParams + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                         (const double*)s->tape.part, s->nnbar);
      CFD_LAUNCHED();
    }
  } else {
    if (g.act[0]) launch_face_adj<0>(s, P, Rbar, rscale, st, sd);
    if (g.act[1]) launch_face_adj<1>(s, P, Rbar, rscale, st, sd);
    if (g.act[2]) launch_face_adj<2>(s, P, Rbar, rscale, st, sd);
    CFD_LAUNCHED();
  }
  if (fork) {
    if (clear_next) {
      enqueue_clear_adj(s, s->Wbar2, s->Dbar2, s->side);
      CFD_LAUNCHED();
    }
    CFD_HIP(hipEventRecord(s->ev_join, s->side));
    CFD_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
  }
  if (g.viscous) {
    hipLaunchKernelGGL(k_adj_dbar_halo, dim3(halo_blocks(g)), dim3(kBlock), 0, st, (const double*)s->Dbar, s->Wbar,
                       g);
    CFD_LAUNCHED();
  }
  hipLaunchKernelGGL(k_adj_halo, dim3(halo_blocks(g)), dim3(kBlock), 0, st, s->Wbar, g);
  CFD_LAUNCHED();
  hipLaunchKernelGGL(k_adj_fold, plane_grid(g), dim3(kBlock), 0, st, P, (const double*)s->Wbar,
                     (const double*)(g.viscous ? s->Dbar : nullptr), out, g);
  CFD_LAUNCHED();
  std::swap(s->Wbar, s->Wbar2);
  std::swap(s->Dbar, s->Dbar2);
  return CFD_OK;
}

static AdjOut adj_out(double* out, double a, const double* X, double b = 0.0, const double* Y = nullptr,
                      double c = 0.0, const double* Z = nullptr, bool zero_halo = false) {
  AdjOut o;
  o.out = out;
  o.a = a;
  o.b = b;
  o.c = c;
  o.X = X;
  o.Y = Y;
  o.Z = Z;
  o.zero_halo = zero_halo ? 1 : 0;
  return o;
}

// The reverse sweep of a step given the primitives Pk[0..2] of its stage
// inputs Un, U1 (, U2):
//   TVD-RK3  U1 = Un + dt R(Un),  U2 = 3/4 Un + 1/4 (U1 + dt R(U1)),
//            U3 = 1/3 Un + 2/3 (U2 + dt R(U2)):
//     A2 = 2/3 Ubar_3 + (dR/dU(U2))^T (2/3 dt Ubar_3)
//     A1 = 1/4 A2 + (dR/dU(U1))^T (1/4 dt A2)
//     Ubar_n = 1/3 Ubar_3 + 3/4 A2 + A1 + (dR/dU(Un))^T (dt A1)
//   TVD-RK2  U2 = 1/2 Un + 1/2 (U1 + dt R(U1)):
//     A1 = 1/2 Ubar_2 + (dR/dU(U1))^T (1/2 dt Ubar_2)
//     Ubar_n = 1/2 Ubar_2 + A1 + (dR/dU(Un))^T (dt A1)
// Ubar_n's halo entries are set to zero.
static cfd_status enqueue_step_reverse(cfd_solver* s, const double* const* Pk, double dt, const double* Ubar_np1,
                                       double* Ubar_n, hipStream_t st) {
  cfd_status rc;
  if (s->g.rk2) {
    if ((rc = enqueue_rhs_adjoint(s, Pk[1], Ubar_np1, 0.5 * dt, adj_out(s->A1, 0.5, Ubar_np1), st, false, true)))
      return rc;
    return enqueue_rhs_adjoint(s, Pk[0], s->A1, dt, adj_out(Ubar_n, 0.5, Ubar_np1, 1.0, s->A1, 0.0, nullptr, true),
                               st, true, false);
  }
  if ((rc = enqueue_rhs_adjoint(s, Pk[2], Ubar_np1, 2.0 / 3.0 * dt, adj_out(s->A2, 2.0 / 3.0, Ubar_np1), st, false,
                                true)))
    return rc;
  if ((rc = enqueue_rhs_adjoint(s, Pk[1], s->A2, 0.25 * dt, adj_out(s->A1, 0.25, s->A2), st, true, true))) return rc;
  return enqueue_rhs_adjoint(s, Pk[0], s->A1, dt,
                             adj_out(Ubar_n, 1.0 / 3.0, Ubar_np1, 0.75, s->A2, 1.0, s->A1, true), st, true, false);
}

// The adjoint covers WENO5-JS with HLLC (any physics), and WENO3-JS with the
// Rusanov-NN flux (inviscid), with TVD-RK3 or TVD-RK2 and any boundaries.
static bool adjoint_supported(const cfd_solver* s) {
  const Geom& g = s->g;
  if (g.wenoz || g.roe || g.rusanov || g.safe) return false;
  if (g.nn) return !g.viscous && !g.heat;
  return !g.weno3;
}
#define CFD_ADJ_SCOPE "the adjoint covers WENO5-JS + HLLC and WENO3-JS + Rusanov-NN (inviscid), without safe reconstruction"

// ===========================================================================
extern "C" {

const char* cfd_last_error(void) { return g_err.c_str(); }

cfd_status cfd_create(const cfd_config* cfg, cfd_solver** out) {
  if (!out) return fail(CFD_EINVAL, "out is NULL");
  *out = nullptr;
  cfd_status rc = validate(cfg);
  if (rc) return rc;
  cfd_solver* s = new (std::nothrow) cfd_solver();
  if (!s) return fail(CFD_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  make_geom(*cfg, s->g);
  choose_segment(s->g);
  s->ncell = s->g.vs;
  s->nint = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
  const size_t st = sizeof(double) * 5 * (size_t)s->ncell;
  bool ok = hipMalloc(&s->U1, st) == hipSuccess && hipMalloc(&s->U2, st) == hipSuccess &&
            hipMalloc(&s->Racc, st) == hipSuccess &&
            (!stage_split(s->g) || hipMalloc(&s->Racc2, st) == hipSuccess) &&
            hipMalloc(&s->Pb[0], sizeof(double) * 6 * (size_t)s->ncell) == hipSuccess &&
            hipMalloc(&s->Pb[1], sizeof(double) * 6 * (size_t)s->ncell) == hipSuccess &&
            hipMalloc(&s->Pb[2], sizeof(double) * 6 * (size_t)s->ncell) == hipSuccess &&
            hipMalloc(&s->ctl, sizeof(DevCtl)) == hipSuccess;
  s->P = s->Pb[0];
  s->npart = kCflSlots;
  ok = ok && hipMalloc(&s->partial, sizeof(double) * (size_t)s->npart) == hipSuccess;
  if (s->g.nn) {
    ok = ok && hipMalloc(&s->nna, sizeof(double) * 3 * (size_t)s->ncell) == hipSuccess &&
         hipMemset(s->nna, 0, sizeof(double) * 3 * (size_t)s->ncell) == hipSuccess;
    s->g.nna = s->nna;
  }
  if (!ok) {
    (void)hipGetLastError();
    cfd_destroy(s);
    return fail(CFD_ENOMEM, "device allocation failed");
  }
  if (hipMemset(s->ctl, 0, sizeof(DevCtl)) != hipSuccess ||
      hipMemset(s->partial, 0, sizeof(double) * (size_t)s->npart) != hipSuccess ||
      hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    cfd_destroy(s);
    return fail(CFD_EHIP, "solver initialisation failed");
  }
  *out = s;
  return CFD_OK;
}

void cfd_destroy(cfd_solver* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  if (s->graph.exec) (void)hipGraphExecDestroy(s->graph.exec);
  if (s->cap) (void)hipStreamDestroy(s->cap);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  double* bufs[] = {s->U1, s->U2,   s->Pb[0], s->Pb[1], s->Pb[2], s->Racc,    s->Racc2, s->A1,
                    s->A2, s->A3,   s->Wbar,  s->Dbar,  s->Wbar2, s->Dbar2, s->partial, s->nna, s->nntape};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (s->ctl) (void)hipFree(s->ctl);
  delete s;
}

int64_t cfd_state_numel(const cfd_solver* s) { return s ? 5 * (int64_t)s->ncell : -1; }

cfd_status cfd_state_init(cfd_solver* s, const double* W, double* U, void* stream) {
  if (!s || !W || !U) return fail(CFD_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_state_init, plane_grid(s->g), dim3(kBlock), 0, st, W, U, s->g);
  CFD_LAUNCHED();
  return enqueue_fill_halo(s, U, st);
}

cfd_status cfd_state_init_adjoint(cfd_solver* s, const double* W, const double* Ubar, double* Wbar, void* stream) {
  if (!s || !W || !Ubar || !Wbar) return fail(CFD_EINVAL, "NULL argument");
  if (Wbar == W || Wbar == Ubar) return fail(CFD_EINVAL, "Wbar must not alias W or Ubar");
  hipLaunchKernelGGL(k_state_init_adj, plane_grid(s->g), dim3(kBlock), 0, (hipStream_t)stream, W, Ubar, Wbar,
                     s->g);
  CFD_LAUNCHED();
  return CFD_OK;
}

cfd_status cfd_fill_halo(cfd_solver* s, double* U, void* stream) {
  if (!s || !U) return fail(CFD_EINVAL, "NULL argument");
  return enqueue_fill_halo(s, U, (hipStream_t)stream);
}

cfd_status cfd_rhs(cfd_solver* s, double* U, double* R, void* stream) {
  if (!s || !U || !R) return fail(CFD_EINVAL, "NULL argument");
  if (U == R) return fail(CFD_EINVAL, "U and R must not alias");
  hipStream_t st = (hipStream_t)stream;
  cfd_status rc;
  if ((rc = enqueue_fill_halo(s, U, st))) return rc;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(5 * s->ncell)), dim3(kBlock), 0, st, R, 5 * s->ncell);
  CFD_LAUNCHED();
  if ((rc = enqueue_prim(s, U, 0, nullptr, st))) return rc;
  StageIO io{};
  io.R = R;
  io.dtp = nullptr;
  io.ctl = s->ctl;  // faces with non-positive reconstructed states
  return enqueue_fluxes(s, s->P, io, false, st);
}

cfd_status cfd_compute_dt(cfd_solver* s, const double* U, double* dt_dev, void* stream) {
  if (!s || !U || !dt_dev) return fail(CFD_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  cfd_status rc = enqueue_clear_slots(s, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_cfl, plane_grid(s->g), dim3(kBlock), 0, st, U, s->g, s->partial);
  CFD_LAUNCHED();
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(kBlock), 0, st, s->ctl, s->g.cfl, 0.0, 0.0, (double*)nullptr, dt_dev,
                     s->partial, s->npart);
  CFD_LAUNCHED();
  return CFD_OK;
}

cfd_status cfd_rk3_step(cfd_solver* s, double* U, double dt, double* dt_used_dev, void* stream) {
  if (!s || !U) return fail(CFD_EINVAL, "NULL argument");
  if (!std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be finite");
  hipStream_t st = (hipStream_t)stream;
  cfd_status rc = enqueue_step_prologue(s, U, !(dt > 0.0), st);
  if (rc) return rc;
  if ((rc = enqueue_step(s, U, dt > 0.0 ? dt : 0.0, 0.0, nullptr, dt_used_dev, st))) return rc;
  return enqueue_fill_halo(s, U, st);
}

cfd_status cfd_advance(cfd_solver* s, double* U, int32_t n_steps, double t_end, double* t_dev,
                       void* stream) {
  if (!s || !U || !t_dev) return fail(CFD_EINVAL, "NULL argument");
  if (n_steps < 0) return fail(CFD_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return CFD_OK;
  hipStream_t st = (hipStream_t)stream;
  cfd_status rc = run_graph(s, U, 1, 0.0, t_end > 0.0 ? t_end : 0.0, t_dev, n_steps, st);
  if (rc) return rc;
  return enqueue_fill_halo(s, U, st);
}

cfd_status cfd_advance_fixed(cfd_solver* s, double* U, int32_t n_steps, double dt, void* stream) {
  if (!s || !U) return fail(CFD_EINVAL, "NULL argument");
  if (n_steps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fail(CFD_EINVAL, "need n_steps >= 0 and dt > 0");
  if (n_steps == 0) return CFD_OK;
  hipStream_t st = (hipStream_t)stream;
  cfd_status rc = run_graph(s, U, 2, dt, 0.0, nullptr, n_steps, st);
  if (rc) return rc;
  return enqueue_fill_halo(s, U, st);
}

cfd_status cfd_check(cfd_solver* s, int32_t* status_out) {
  if (!s || !status_out) return fail(CFD_EINVAL, "NULL argument");
  CFD_HIP(hipDeviceSynchronize());
  int v = 0;
  CFD_HIP(hipMemcpy(&v, &s->ctl->status, sizeof(int), hipMemcpyDeviceToHost));
  const int zero = 0;
  CFD_HIP(hipMemcpy(&s->ctl->status, &zero, sizeof(int), hipMemcpyHostToDevice));
  *status_out = v;
  return CFD_OK;
}

cfd_status cfd_profile_stage(cfd_solver* s, const double* U, int32_t reps, double* ms_out, void* stream) {
  if (!s || !U || !ms_out || reps < 1 || reps > 4096) return fail(CFD_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  const Geom& g = s->g;
  // a fixed nonzero step so that the stage kernels do their work
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(kBlock), 0, st, s->ctl, g.cfl, 1e-12, 0.0, (double*)nullptr,
                     (double*)nullptr, s->partial, s->npart);
  CFD_LAUNCHED();
  int first = -1, last = -1;
  sweep_order(g, first, last);
  // slots of ms_out: prim pass, x, y, z sweeps, halo refresh of the next
  // primitives. Repetition r runs stage r % 3 + 1 of a step as a run of steps
  // does (the third with the CFL maxima and health bits of its output), into
  // scratch; all repetitions run back to back, each kernel between two events,
  // and the stream is synchronised once at the end.
  constexpr int K = 5;
  std::vector<hipEvent_t> ev((size_t)reps * (K + 1));
  std::vector<int> slot((size_t)reps * (K + 1), -1);
  cfd_status rc = CFD_OK;
  size_t made = 0;
  for (; made < ev.size(); ++made)
    if (hipEventCreate(&ev[made]) != hipSuccess) {
      rc = fail(CFD_EHIP, "hipEventCreate failed");
      break;
    }
  for (int r = 0; r < reps && rc == CFD_OK; ++r) {
    const int stage = r % 3;
    StageIO io{};
    io.R = s->Racc;
    io.R2 = s->Racc2;
    io.Un = U;
    io.Uk = U;
    io.Uout = s->U2;
    io.a = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
    io.b = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
    io.dtp = &s->ctl->dt;
    io.Pn = s->Pb[1];
    io.partial = s->partial;
    io.ctl = s->ctl;
    io.what = stage == 2 ? (PRIM_HEALTH | PRIM_CFL) : 0;
    hipEvent_t* e = ev.data() + (size_t)r * (K + 1);
    int* sl = slot.data() + (size_t)r * (K + 1);
    int n = 0;
    (void)hipEventRecord(e[n], st);
    hipLaunchKernelGGL(k_prim, plane_grid(g), dim3(kBlock), 0, st, U, s->P, g, s->ctl, 0, io.dtp, s->partial);
    sl[n] = 0;
    (void)hipEventRecord(e[++n], st);
    for (int d : kSweepAxes) {
      if (!g.act[d]) continue;
      int mode;
      StageIO iod = io;
      if (d == last) {
        mode = d == first ? MODE_WRITE_RK : (stage_split(g) && d == 0 ? MODE_ACC2_RK : MODE_ACC_RK);
      } else if (stage_split(g)) {
        mode = MODE_WRITE;
        if (d != first) iod.R = const_cast<double*>(io.R2);
      } else {
        mode = d == first ? MODE_WRITE : MODE_ACC;
      }
      if (d == last) launch_sweep_axis<true>(s, d, mode, s->P, iod, st);
      else launch_sweep_axis<false>(s, d, mode, s->P, iod, st);
      sl[n] = 1 + d;
      (void)hipEventRecord(e[++n], st);
    }
    hipLaunchKernelGGL(k_prim_halo, dim3(halo_blocks(g)), dim3(kBlock), 0, st, io.Pn, g, io.dtp);
    sl[n] = 4;
    (void)hipEventRecord(e[++n], st);
    if (hipGetLastError() != hipSuccess) rc = fail(CFD_EHIP, "profiled stage failed");
  }
  double acc[K] = {0, 0, 0, 0, 0};
  if (rc == CFD_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(CFD_EHIP, "profiled stage failed");
  for (int r = 0; r < reps && rc == CFD_OK; ++r)
    for (int k = 0; k < K; ++k) {
      const int sl = slot[(size_t)r * (K + 1) + k];
      if (sl < 0) continue;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[(size_t)r * (K + 1) + k], ev[(size_t)r * (K + 1) + k + 1]);
      acc[sl] += ms;
    }
  for (size_t e = 0; e < made; ++e) (void)hipEventDestroy(ev[e]);
  // the CFL maxima of the third stages are nobody's: clear them
  if (rc == CFD_OK) rc = enqueue_clear_slots(s, st);
  for (int k = 0; k < K; ++k) ms_out[k] = acc[k] / reps;
  return rc;
}

cfd_status cfd_rhs_adjoint(cfd_solver* s, const double* U, const double* Rbar, double* Ubar, void* stream) {
  if (!s || !U || !Rbar || !Ubar) return fail(CFD_EINVAL, "NULL argument");
  if (!adjoint_supported(s)) return fail(CFD_EUNSUPPORTED, CFD_ADJ_SCOPE);
  if (Ubar == U || Ubar == Rbar) return fail(CFD_EINVAL, "Ubar must not alias U or Rbar");
  cfd_status rc = ensure_adjoint_scratch(s);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = enqueue_prim(s, U, 0, nullptr, st))) return rc;
  return enqueue_rhs_adjoint(s, s->P, Rbar, 1.0, adj_out(Ubar, 1.0, Ubar), st);
}

cfd_status cfd_rk3_step_adjoint(cfd_solver* s, const double* Un, double dt, const double* Ubar_np1,
                                double* Ubar_n, void* stream) {
  if (!s || !Un || !Ubar_np1 || !Ubar_n) return fail(CFD_EINVAL, "NULL argument");
  if (!adjoint_supported(s)) return fail(CFD_EUNSUPPORTED, CFD_ADJ_SCOPE);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be > 0");
  if (Ubar_n == Un || Ubar_n == Ubar_np1) return fail(CFD_EINVAL, "Ubar_n must not alias the inputs");
  cfd_status rc = ensure_adjoint_scratch(s);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geom& g = s->g;
  // forward recompute of the stage states U1, U2 with the fixed step; the
  // stage updates leave the primitives of Un, U1, U2 in Pb[0], Pb[1], Pb[2]
  // (rho, u, v, w, p with halos: all the face reverses and the fold read)
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(kBlock), 0, st, s->ctl, g.cfl, dt, 0.0, (double*)nullptr,
                     (double*)nullptr, s->partial, s->npart);
  CFD_LAUNCHED();
  const double* dtp = &s->ctl->dt;
  StageIO io{};
  io.R = s->Racc;
  io.R2 = s->Racc2;
  io.Un = Un;
  io.dtp = dtp;
  io.partial = s->partial;
  io.ctl = s->ctl;
  io.what = 0;
  io.Uk = Un;
  io.Uout = s->U1;
  io.a = 0.0;
  io.b = 1.0;
  io.Pn = s->Pb[1];
  if ((rc = enqueue_prim(s, Un, 0, dtp, st))) return rc;
  if ((rc = enqueue_fluxes(s, s->Pb[0], io, true, st))) return rc;
  if (g.rk2) {
    const double* const Pk[2] = {s->Pb[0], s->Pb[1]};
    return enqueue_step_reverse(s, Pk, dt, Ubar_np1, Ubar_n, st);
  }
  io.Uk = s->U1;
  io.Uout = s->U2;
  io.a = 0.75;
  io.b = 0.25;
  io.Pn = s->Pb[2];
  if ((rc = enqueue_fluxes(s, s->Pb[1], io, true, st))) return rc;
  const double* const Pk[3] = {s->Pb[0], s->Pb[1], s->Pb[2]};
  return enqueue_step_reverse(s, Pk, dt, Ubar_np1, Ubar_n, st);
}

cfd_status cfd_set_nn_weights(cfd_solver* s, const double* theta, double* theta_bar) {
  if (!s) return fail(CFD_EINVAL, "NULL argument");
  if (!s->g.nn) return fail(CFD_EINVAL, "the solver was not created with the Rusanov-NN flux");
  s->g.nnw = theta;
  s->nnbar = theta ? theta_bar : nullptr;
  // a captured step holds the old weight address; it may still be running
  if (s->graph.exec) {
    CFD_HIP(hipDeviceSynchronize());
    CFD_HIP(hipGraphExecDestroy(s->graph.exec));
    s->graph.exec = nullptr;
  }
  return CFD_OK;
}

cfd_status cfd_rk3_step_stages(cfd_solver* s, double* U, double dt, double* U1_out, double* U2_out, void* stream) {
  if (!s || !U || !U1_out || !U2_out) return fail(CFD_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be > 0");
  if (U1_out == U || U2_out == U || U1_out == U2_out) return fail(CFD_EINVAL, "the stage buffers must be distinct");
  if (s->g.rk2) return fail(CFD_EUNSUPPORTED, "the stages kept are those of TVD-RK3");
  hipStream_t st = (hipStream_t)stream;
  cfd_status rc = enqueue_step_prologue(s, U, false, st);
  if (rc) return rc;
  if ((rc = enqueue_step(s, U, dt, 0.0, nullptr, nullptr, st, U1_out, U2_out))) return rc;
  return enqueue_fill_halo(s, U, st);
}

cfd_status cfd_rk3_step_adjoint_stages(cfd_solver* s, const double* Un, const double* U1, const double* U2, double dt,
                                       const double* Ubar_np1, double* Ubar_n, void* stream) {
  if (!s || !Un || !U1 || !U2 || !Ubar_np1 || !Ubar_n) return fail(CFD_EINVAL, "NULL argument");
  if (!adjoint_supported(s)) return fail(CFD_EUNSUPPORTED, CFD_ADJ_SCOPE);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be > 0");
  if (Ubar_n == Un || Ubar_n == U1 || Ubar_n == U2 || Ubar_n == Ubar_np1)
    return fail(CFD_EINVAL, "Ubar_n must not alias the inputs");
  if (s->g.rk2) return fail(CFD_EUNSUPPORTED, "the stages kept are those of TVD-RK3");
  cfd_status rc = ensure_adjoint_scratch(s);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const Geom& g = s->g;
  // primitives of the three stage inputs (halos gathered through the boundary map)
  const double* Us[3] = {Un, U1, U2};
  for (int k = 0; k < 3; ++k) {
    hipLaunchKernelGGL(k_prim, plane_grid(g), dim3(kBlock), 0, st, Us[k], s->Pb[k], g, s->ctl, 0,
                       (const double*)nullptr, s->partial);
    CFD_LAUNCHED();
  }
  const double* const Pk[3] = {s->Pb[0], s->Pb[1], s->Pb[2]};
  return enqueue_step_reverse(s, Pk, dt, Ubar_np1, Ubar_n, st);
}

cfd_status cfd_rk3_step_prims(cfd_solver* s, double* U, double dt, double* P_out, void* stream) {
  if (!s || !U || !P_out) return fail(CFD_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be > 0");
  if (P_out == U) return fail(CFD_EINVAL, "P_out must not alias U");
  if (s->g.rk2) return fail(CFD_EUNSUPPORTED, "the stages kept are those of TVD-RK3");
  hipStream_t st = (hipStream_t)stream;
  const size_t ps = kPrimComps * (size_t)s->ncell;
  double* const Pst[3] = {P_out, P_out + ps, P_out + 2 * ps};
  hipLaunchKernelGGL(k_prim, plane_grid(s->g), dim3(kBlock), 0, st, (const double*)U, Pst[0], s->g, s->ctl,
                     PRIM_HEALTH, (const double*)nullptr, s->partial);
  CFD_LAUNCHED();
  cfd_status rc = enqueue_step(s, U, dt, 0.0, nullptr, nullptr, st, nullptr, nullptr, Pst);
  if (rc) return rc;
  return enqueue_fill_halo(s, U, st);
}

cfd_status cfd_rk3_step_adjoint_prims(cfd_solver* s, const double* P, double dt, const double* Ubar_np1,
                                      double* Ubar_n, void* stream) {
  if (!s || !P || !Ubar_np1 || !Ubar_n) return fail(CFD_EINVAL, "NULL argument");
  if (!adjoint_supported(s)) return fail(CFD_EUNSUPPORTED, CFD_ADJ_SCOPE);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be > 0");
  if (Ubar_n == Ubar_np1 || Ubar_n == P) return fail(CFD_EINVAL, "Ubar_n must not alias the inputs");
  if (s->g.rk2) return fail(CFD_EUNSUPPORTED, "the stages kept are those of TVD-RK3");
  cfd_status rc = ensure_adjoint_scratch(s);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const size_t ps = kPrimComps * (size_t)s->ncell;
  const double* const Pk[3] = {P, P + ps, P + 2 * ps};
  return enqueue_step_reverse(s, Pk, dt, Ubar_np1, Ubar_n, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free TVD-RK3 step. Its scratch (CFL slots, control block, two
// stage states, the right-hand-side accumulator and three primitive buffers)
// lives in one file-scope device array, present on every device the library
// runs on until the process ends. Host code never passes the array's name to
// a kernel (on the host it is only a stand-in symbol): the device address of
// each device's copy is looked up once, on that device's first call, with
// hipGetSymbolAddress and kept per device.
constexpr long long kNoAllocDoubles = 112LL << 17;  // 112 MiB of FP64
constexpr long long kNoAllocHead = kCflSlots + 32;  // CFL slots, then the control block (256 B aligned)
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Padded cells of cfg that fit the scratch array: 38 doubles per padded cell
// (U1, U2 and the two accumulators: 5 each; three primitive buffers: 6 each)
// after the head.
static constexpr long long noalloc_max_cells() { return (kNoAllocDoubles - kNoAllocHead) / 38; }
static_assert(noalloc_max_cells() == CFD_NOALLOC_MAX_PADDED_CELLS, "header limit out of date");

static cfd_status noalloc_scratch(double** out) {
  int dev = -1;
  CFD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(CFD_EUNSUPPORTED, "device index beyond the supported range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CFD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return CFD_OK;
}

extern "C" {

cfd_status cfd_rk3_step_noalloc(const cfd_config* cfg, double* U, double dt, double* dt_used_dev, void* stream) {
  if (!U) return fail(CFD_EINVAL, "NULL argument");
  cfd_status rc = validate(cfg);
  if (rc) return rc;
  if (!std::isfinite(dt)) return fail(CFD_EINVAL, "dt must be finite");
  if (cfg->flags & CFD_F_RUSANOV_NN)
    return fail(CFD_EUNSUPPORTED, "the allocation-free step does not take the Rusanov-NN flux (it needs weights)");
  cfd_solver s{};
  s.cfg = *cfg;
  make_geom(*cfg, s.g);
  choose_segment(s.g);
  s.ncell = s.g.vs;
  s.nint = (long long)cfg->n[0] * cfg->n[1] * cfg->n[2];
  if (s.ncell > noalloc_max_cells())
    return fail(CFD_EINVAL, "grid too large for the allocation-free step: " + std::to_string(s.ncell) +
                                " padded cells, at most " + std::to_string(noalloc_max_cells()));
  double* base = nullptr;
  if ((rc = noalloc_scratch(&base))) return rc;
  const long long nc = s.ncell;
  s.partial = base;
  s.npart = kCflSlots;
  s.ctl = reinterpret_cast<DevCtl*>(base + kCflSlots);
  double* b = base + kNoAllocHead;
  s.U1 = b;
  s.U2 = b + 5 * nc;
  s.Racc = b + 10 * nc;
  s.Racc2 = b + 15 * nc;
  for (int k = 0; k < 3; ++k) s.Pb[k] = b + (20 + 6 * k) * nc;
  s.P = s.Pb[0];
  hipStream_t st = (hipStream_t)stream;
  // the control block (step size, health bits) starts clear on every call;
  // the CFL slots are cleared by the prologue of a CFL step
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, st, base + kCflSlots, 32LL);
  CFD_LAUNCHED();
  if ((rc = enqueue_step_prologue(&s, U, !(dt > 0.0), st))) return rc;
  if ((rc = enqueue_step(&s, U, dt > 0.0 ? dt : 0.0, 0.0, nullptr, dt_used_dev, st))) return rc;
  return enqueue_fill_halo(&s, U, st);
}

}  // extern "C"
#include "batch_host.inc"
