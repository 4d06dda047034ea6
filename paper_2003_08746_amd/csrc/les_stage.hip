// les_stage.hip -- Runge-Kutta stage launchers.
#include "les_stage.hpp"
#include "les_launch.hpp"

namespace les {

long long stage_blocks(const Layout& L) { return ref_blocks(L); }

hipError_t launch_stage_fp64(hipStream_t s, const StageArgs& a, const double* Qin, const double* Q0, double* Qout,
                             const double* dtp, double dt, double alpha, double* part) {
  return launch_stage_ref(s, a.L, a.P, a.M, Qin, Q0, Qout, dtp, dt, alpha, a.f, a.i_f, part);
}

hipError_t run_rk_mixed(hipStream_t, const StageArgs&, const int*, double*, float**, const double*, double,
                        double*) {
  return hipErrorNotSupported;
}

}  // namespace les
