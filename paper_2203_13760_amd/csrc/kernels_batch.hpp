// Batched persistent stage kernels for serving (gfx950).
//
// Many independent grids (mixed sizes, 2D and 3D, different physics) are
// resident at once. For every phase of a TVD-RK3 stage (primitives, step size,
// x/y/z sweeps, primitive halo) one persistent launch covers the work of the
// resident grids of a sub-batch (its width chosen on the host from the
// phase's blocks): the work of grid k is blocks [prefix[k], prefix[k+1]) of
// that phase, and each workgroup takes blocks of the concatenated range, finds
// their grid by binary search, and runs the same per-block body as the
// single-grid kernels. Grids never interact:
// each keeps its own state, scratch and CFL step, so a grid's result does not
// depend on which other grids share the launch.
//
// As in the single-grid step, a grid with an active x axis gets the
// primitives of each stage's output from its x sweep (which applies the stage
// update) plus a halo pass, and the CFL rate maxima of U^{n+1} from the third
// x sweep; its primitives of a new state are formed once, on admission. A grid
// without an x axis takes a primitive pass at the start of every stage.
#pragma once
#include "kernels_fwd.hpp"

namespace cfd {

// PH_SX/SY/SZ: the sweep of that axis where it does not apply the stage
// update except the x sweep (which applies it whenever x is active);
// PH_SLAST: the last march of grids without an x axis, which applies the
// update. Keeping those rare updating marches in a phase of their own keeps
// the y and z phases to one sweep mode and within the register file.
enum BatchPhase { PH_PRIM = 0, PH_DT, PH_SX, PH_SY, PH_SZ, PH_SLAST, PH_HALO, PH_COUNT };

constexpr int kBatchMaxGrids = 512;

struct GridWork {
  Geom g;
  double* U;       // resident state (updated in place by the third stage)
  double* U1;
  double* U2;
  double* Pb[3];   // primitives (6 x padded) of the stage inputs: stage s reads Pb[s-1]
  double* R;       // 5 x padded
  double* R2;      // 5 x padded: the second march's accumulator (grids with three active axes)
  double* partial; // CFL rate slots
  DevCtl* ctl;
  int npart;
  int last_axis;   // the last swept axis (the lowest active one) applies the stage update
  int first_axis;
  int xpn;         // x is active: the x sweep stores the next primitives
  int pgx;         // x blocks of a plane-indexed launch
  int sgx[3], sgy[3];  // launch shapes of the marching sweeps (axes 1, 2)
};

struct BatchTable {
  int ngrids;
  int pad;
  int prefix[PH_COUNT][kBatchMaxGrids + 1];
  GridWork grid[kBatchMaxGrids];
};

__device__ __forceinline__ int find_grid(const int* __restrict__ prefix, int ngrids, int b) {
  int lo = 0, hi = ngrids;  // prefix[lo] <= b < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// PN: the sweep stores the primitives of its output (x sweeps only).
template <int MODE, bool PN>
__device__ __forceinline__ void batch_sweep(int axis, const GridWork& w, const double* P, const StageIO& io,
                                            int local) {
  if (axis == 0) {
    sweep_x_body<MODE, PN>(P, io, w.g, local);
  } else if (axis == 1) {
    const int by = local / w.sgx[1];
    sweep_march_body<1, MODE>(P, io, w.g, local - by * w.sgx[1], by);
  } else {
    const int by = local / w.sgx[2];
    sweep_march_body<2, MODE>(P, io, w.g, local - by * w.sgx[2], by);
  }
}

// Work distribution of a persistent launch: the concatenated block range of a
// phase is cut into kXcds equal chunks, chunk x first served to the workgroups
// of XCD x (hardware block b runs on XCD b % kXcds), so that each XCD works
// through consecutive blocks - neighbouring rows and planes of the same grids,
// whose stencils share its L2. A workgroup takes blocks from a chunk's counter
// one at a time and, once its own chunk is used up, from the other chunks in
// turn, so no XCD idles while work remains. The last workgroup to finish
// clears the counters for the next launch. Each (phase, stage) launch has its
// own kCtrStride counters: kXcds chunk counters and a finished-workgroup count.
// Phases with fewer than kDynamicMin blocks per workgroup (a lone grid of the
// sizes served, small batches) take a fixed stride instead: there the atomic
// round trips would lengthen the launch more than balancing shortens it.
constexpr int kDynamicMin = 8;
constexpr int kCtrStride = 16;
constexpr int kCtrCount = PH_COUNT * 3 * kCtrStride;

// One block of a phase: block b of the concatenated range.
// STAGE 1..3 selects the stage input/output states and the stage weights.
template <int PHASE, int STAGE>
__device__ __forceinline__ void batch_item(const BatchTable* __restrict__ tab, int b) {
  const int ng = tab->ngrids;
  const int* prefix = tab->prefix[PHASE];
  {
    const int k = find_grid(prefix, ng, b);
    const int local = b - prefix[k];
    const GridWork& w = tab->grid[k];
    const Geom& g = w.g;
    StageIO io;
    io.R = w.R;
    io.R2 = w.R2;
    io.Un = w.U;
    io.dtp = &w.ctl->dt;
    io.Uk = STAGE == 1 ? w.U : (STAGE == 2 ? w.U1 : w.U2);
    io.Uout = STAGE == 1 ? w.U1 : (STAGE == 2 ? w.U2 : w.U);
    io.a = STAGE == 1 ? 0.0 : (STAGE == 2 ? 0.75 : 1.0 / 3.0);
    io.b = STAGE == 1 ? 1.0 : (STAGE == 2 ? 0.25 : 2.0 / 3.0);
    io.Pn = w.Pb[STAGE % 3];
    io.partial = w.partial;
    io.ctl = w.ctl;
    io.what = STAGE == 3 ? (PRIM_HEALTH | PRIM_CFL) : PRIM_HEALTH;
    const double* P = w.Pb[STAGE - 1];
    if (PHASE == PH_PRIM) {
      const int by = local / w.pgx;
      const int bx = local - by * w.pgx;
      const PlaneIdx q = plane_index_at(g, bx, by, w.pgx, g.N[2], false);
      prim_body(io.Uk, w.Pb[STAGE - 1], g, w.ctl, STAGE == 1 ? (PRIM_CFL | PRIM_HEALTH) : 0, w.partial, q,
                local);
    } else if (PHASE == PH_DT) {
      dt_body(w.ctl, g.cfl, 0.0, 0.0, nullptr, nullptr, w.partial, w.npart);
    } else if (PHASE == PH_HALO) {
      prim_halo_body(io.Pn, g, (long long)local * kBlock + threadIdx.x);
    } else if (PHASE == PH_SX) {
      // x is the last axis whenever it is active: the stage update
      const bool split = g.act[1] && g.act[2];  // y and z marches wrote R and R2
      if (w.first_axis == 0) batch_sweep<MODE_WRITE_RK, true>(0, w, P, io, local);
      else if (split) batch_sweep<MODE_ACC2_RK, true>(0, w, P, io, local);
      else batch_sweep<MODE_ACC_RK, true>(0, w, P, io, local);
    } else if (PHASE == PH_SLAST) {
      // the last march of a grid without an x axis
      if (w.last_axis == w.first_axis) batch_sweep<MODE_WRITE_RK, false>(w.last_axis, w, P, io, local);
      else batch_sweep<MODE_ACC_RK, false>(w.last_axis, w, P, io, local);
    } else {
      // a march before the update: the first writes R, a second (only with
      // x active) its own accumulator R2
      constexpr int axis = PHASE == PH_SY ? 1 : 2;
      if (axis != w.first_axis) io.R = w.R2;
      batch_sweep<MODE_WRITE, false>(axis, w, P, io, local);
    }
  }
}

template <int PHASE, int STAGE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_batch(const BatchTable* __restrict__ tab, unsigned* ctr) {
  unsigned* c = ctr + (PHASE * 3 + STAGE - 1) * kCtrStride;
  const int total = tab->prefix[PHASE][tab->ngrids];
  if (total < kDynamicMin * (int)gridDim.x) {
    // few blocks per workgroup: a fixed stride, without the counters' latency
    for (int b = blockIdx.x; b < total; b += gridDim.x) batch_item<PHASE, STAGE>(tab, b);
    return;
  }
  const int x0 = blockIdx.x % kXcds;
  __shared__ int next;
  for (int t = 0; t < kXcds; ++t) {
    const int x = (x0 + t) % kXcds;
    const int lo = (int)((long long)total * x / kXcds), hi = (int)((long long)total * (x + 1) / kXcds);
    for (;;) {
      if (threadIdx.x == 0) next = lo + (int)atomicAdd(c + x, 1u);
      __syncthreads();
      const int b = next;
      __syncthreads();  // every wave has read `next` before it is replaced
      if (b >= hi) break;
      batch_item<PHASE, STAGE>(tab, b);
    }
  }
  if (threadIdx.x == 0) {
    // every other workgroup has taken its last (failed) block before counting itself
    __threadfence();
    if (atomicAdd(c + kXcds, 1u) == gridDim.x - 1) {
      for (int x = 0; x <= kXcds; ++x) atomicExch(c + x, 0u);
      __threadfence();
    }
  }
}

}  // namespace cfd
