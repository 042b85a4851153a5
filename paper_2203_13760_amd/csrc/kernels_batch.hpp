// Batched persistent stage kernels for serving (gfx950).
//
// Many independent grids (mixed sizes, 2D and 3D, different physics) are
// resident at once. For every phase of a TVD-RK3 stage (primitives, step size,
// x/y/z sweeps, halo refresh) one persistent launch of a fixed number of
// workgroups covers the work of all resident grids: the work of grid k is
// blocks [prefix[k], prefix[k+1]) of that phase, and each workgroup strides
// over the concatenated block range, finds its grid by binary search, and runs
// the same per-block body as the single-grid kernels. Grids never interact:
// each keeps its own state, scratch and CFL step, so a grid's result does not
// depend on which other grids share the launch.
#pragma once
#include "kernels_fwd.hpp"

namespace cfd {

enum BatchPhase { PH_PRIM = 0, PH_DT, PH_SX, PH_SY, PH_SZ, PH_HALO, PH_COUNT };

constexpr int kBatchMaxGrids = 512;

struct GridWork {
  Geom g;
  double* U;       // resident state (updated in place by the third stage)
  double* U1;
  double* U2;
  double* P;       // 6 x padded
  double* R;       // 5 x padded
  double* partial; // CFL rate slots
  DevCtl* ctl;
  int npart;
  int last_axis;   // the last swept axis (the lowest active one) applies the stage update
  int first_axis;
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

template <int MODE>
__device__ __forceinline__ void batch_sweep(int axis, const GridWork& w, const StageIO& io, int local) {
  if (axis == 0) {
    sweep_x_body<MODE>(w.P, io, w.g, local);
  } else if (axis == 1) {
    const int by = local / w.sgx[1];
    sweep_march_body<1, MODE>(w.P, io, w.g, local - by * w.sgx[1], by);
  } else {
    const int by = local / w.sgx[2];
    sweep_march_body<2, MODE>(w.P, io, w.g, local - by * w.sgx[2], by);
  }
}

// STAGE 1..3 selects the stage input/output states and the stage weights.
template <int PHASE, int STAGE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_batch(const BatchTable* __restrict__ tab) {
  const int ng = tab->ngrids;
  const int* prefix = tab->prefix[PHASE];
  const int total = prefix[ng];
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const int k = find_grid(prefix, ng, b);
    const int local = b - prefix[k];
    const GridWork& w = tab->grid[k];
    const Geom& g = w.g;
    StageIO io;
    io.R = w.R;
    io.Un = w.U;
    io.dtp = &w.ctl->dt;
    io.Uk = STAGE == 1 ? w.U : (STAGE == 2 ? w.U1 : w.U2);
    io.Uout = STAGE == 1 ? w.U1 : (STAGE == 2 ? w.U2 : w.U);
    io.a = STAGE == 1 ? 0.0 : (STAGE == 2 ? 0.75 : 1.0 / 3.0);
    io.b = STAGE == 1 ? 1.0 : (STAGE == 2 ? 0.25 : 2.0 / 3.0);
    if (PHASE == PH_PRIM) {
      const int by = local / w.pgx;
      const int bx = local - by * w.pgx;
      const PlaneIdx q = plane_index_at(g, bx, by, w.pgx, g.N[2], false);
      prim_body(io.Uk, w.P, g, w.ctl, STAGE == 1 ? (PRIM_CFL | PRIM_HEALTH) : 0, w.partial, q, local);
    } else if (PHASE == PH_DT) {
      dt_body(w.ctl, g.cfl, 0.0, 0.0, nullptr, nullptr, w.partial, w.npart);
    } else if (PHASE == PH_HALO) {
      const int by = local / w.pgx;
      const int bx = local - by * w.pgx;
      fill_halo_body(w.U, g, plane_index_at(g, bx, by, w.pgx, g.N[2], false));
    } else {
      const int axis = PHASE - PH_SX;
      const bool last = axis == w.last_axis, first = axis == w.first_axis;
      if (last) {
        if (first) batch_sweep<MODE_WRITE_RK>(axis, w, io, local);
        else batch_sweep<MODE_ACC_RK>(axis, w, io, local);
      } else {
        if (first) batch_sweep<MODE_WRITE>(axis, w, io, local);
        else batch_sweep<MODE_ACC>(axis, w, io, local);
      }
    }
  }
}

}  // namespace cfd
