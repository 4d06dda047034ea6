// les_stage.hpp -- launchers of the fused Runge-Kutta stage kernels.
#pragma once
#include "les_common.hpp"

namespace les {

struct StageArgs {
  Layout L;
  Phys P;
  const double* M;  // metrics [10][fe]
  const double* f;  // source [5][nk][nj] or null
  int i_f;
};

// Number of per-block norm partials written by one fused stage launch.
long long stage_blocks(const Layout& L);

// One FP64 stage: Qout = Q0 - alpha dt R(Qin) on the interior (Qin's ghosts
// already filled).  dtp (device) overrides dt when non-null.  part: norm
// partials (or null).  Q0 and Qout may alias.
hipError_t launch_stage_fp64(hipStream_t s, const StageArgs& a, const double* Qin, const double* Q0, double* Qout,
                             const double* dtp, double dt, double alpha, double* part);

// A whole mixed-precision step (FP32 stage states, FP64 Q^n and update).
hipError_t run_rk_mixed(hipStream_t s, const StageArgs& a, const int bc[3], double* Q, float* Sf[2],
                        const double* dtp, double dt, double* part);

}  // namespace les
