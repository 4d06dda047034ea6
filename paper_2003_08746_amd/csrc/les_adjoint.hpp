// les_adjoint.hpp -- reverse-mode (adjoint) of one Runge-Kutta step.
#pragma once
#include "les_common.hpp"
#include "les_faces.hpp"

namespace les {

struct AdjArgs {
  Layout L;
  Phys P;
  const double* M;
  int bc0, bc1, bc2;  // 0 periodic, 1 Dirichlet, 2 periodic with superposed first and last nodes
  int i_f;
  Faces F;            // boundary faces of the Dirichlet directions
  int axis;           // bc1 == 3: j = 0 is the O-grid's polar axis
};

// Device work elements (doubles) needed by run_adjoint_step.
size_t adjoint_work_elems(const Layout& L);

// Qbar = (dR/dQ|Q)^T Rbar on the interior (Q with ghosts filled).
hipError_t run_residual_vjp(hipStream_t s, const AdjArgs& a, const double* Q, const double* Rbar, double* Qbar,
                            double* work);

hipError_t run_adjoint_step(hipStream_t s, const AdjArgs& a, const double* ckpt, double dt, double* Qbar,
                            double* fbar, double* work);

// Reverse of the centerline condition (each axis node takes the mean of the
// ring j = 1 over its nk - 1 distinct azimuths), in place on the interior of
// an adjoint state: the axis adjoints' sum over all nk azimuths, divided by
// nk - 1, is added to every distinct ring node, and the axis adjoints are
// cleared.
hipError_t launch_axis_avg_adjoint(hipStream_t s, const Layout& L, double* qbar);

}  // namespace les
