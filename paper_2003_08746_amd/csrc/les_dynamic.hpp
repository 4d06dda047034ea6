// les_dynamic.hpp -- launchers of the dynamic SGS closure (per-column
// coefficients C and D_T of the eddy viscosity and SGS conductivity).
#pragma once
#include "les_common.hpp"

namespace les {

// Work array (doubles) the closure needs for a layout.
long long dynamic_work_elems(const Layout& L);

// dyn[0 .. ncol) = C, dyn[ncol .. 2 ncol) = D_T per padded column (dyn_col)
// of the state Q (ghosts filled); work: dynamic_work_elems(L) doubles.
hipError_t launch_dynamic(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M,
                          const double* Q, double* work, double* dyn);
hipError_t launch_dynamic_f32(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M,
                              const float* Q, double* work, double* dyn);

}  // namespace les
