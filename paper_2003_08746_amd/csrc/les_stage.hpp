// les_stage.hpp -- launchers of the fused Runge-Kutta stage kernels.
#pragma once
#include "les_common.hpp"

namespace les {

// The device's compute-unit and XCD (accelerator complex die) counts: the
// persistent stage kernel runs one block per CU and maps consecutive blocks
// to one XCD (each XCD has its own L2).
struct Machine {
  int cus = 256;
  int xcds = 8;
};

struct StageArgs {
  Layout L;
  Phys P;
  const double* M;  // metrics [10][fe]
  const double* f;  // source [5][nk][nj] or null
  int i_f;
  int kchunk;       // k planes per block (from stage_kchunk, fixed per context)
  const double* dyn = nullptr;  // dynamic SGS coefficients per column (P.sgs == 2)
  int axis = 0;                 // j = 0 is the polar axis of an O-grid
  Machine mach;
};

// k planes per block of the fused kernel for this layout (LES_SEG in
// the environment overrides the automatic choice; read once per context).
int stage_kchunk(const Layout& L, const Machine& m);

// Largest number of k planes per segment of the stage kernel's schedule for
// this layout (0: a single k plane is too large for the kernel's 32-bit
// per-thread offsets, which les_create refuses).
int stage_kmax(const Layout& L);

// Number of per-block norm partials written by one fused stage launch.
long long stage_blocks(const Layout& L, int kchunk, const Machine& m);

// One FP64 stage: Qout = Q0 - alpha dt R(Qin) on the interior (Qin's ghosts
// already filled).  dtp (device) overrides dt when non-null.  part: norm
// partials (or null).  cpart (or null): per-block minima of the local CFL
// bound of the updated state (stage_blocks doubles; not together with part).
// Q0 and Qout may alias.
hipError_t launch_stage_fp64(hipStream_t s, const StageArgs& a, const double* Qin, const double* Q0, double* Qout,
                             const double* dtp, double dt, double alpha, double* part, double* cpart);

// One mixed-precision stage: the stencil input is FP64 (Qin64, stage 1) or
// FP32 (Qin32); fluxes and dissipation in FP32; the update Q0 - alpha dt R
// in FP64, written as FP64 (Qout) and/or as an FP32 stage state (Qsh).
hipError_t launch_stage_mixed(hipStream_t s, const StageArgs& a, const double* Qin64, const float* Qin32,
                              const double* Q0, double* Qout, float* Qsh, const double* dtp, double dt, double alpha,
                              double* part, double* cpart);

}  // namespace les
