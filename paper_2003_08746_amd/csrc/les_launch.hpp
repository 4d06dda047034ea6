// les_launch.hpp -- host launchers of the gfx950 kernels (one translation
// unit per kernel family; the C-ABI implementation calls only these).
#pragma once
#include "les_common.hpp"
#include "les_faces.hpp"

namespace les {

hipError_t launch_metrics(hipStream_t s, const Layout& L, const int bc[3], const double* xyz, double* M);
hipError_t launch_metrics_copy(hipStream_t s, const Layout& L, const double* src, double* M);
hipError_t launch_metrics_export(hipStream_t s, const Layout& L, const double* M, double* dst);
long long ghost_count(const Layout& L);
hipError_t launch_ghost_fill(hipStream_t s, const Layout& L, const int bc[3], double* q, const double* frozen, int nf,
                             const Faces& F);
hipError_t launch_ghost_fill_f32(hipStream_t s, const Layout& L, const int bc[3], float* q, const double* frozen,
                                 const Faces& F);
// acc[12][nj][ni] += sums over k of the primitives and their second moments
hipError_t launch_stats(hipStream_t s, const Layout& L, const Phys& P, int nks, const double* Q, double* acc);
hipError_t launch_stats_profiles(hipStream_t s, const Layout& L, const double* acc, double samples, double core_u,
                                 double* prof, unsigned char* core);
// p[0 .. n) = 0 on stream s.
hipError_t launch_zero(hipStream_t s, double* p, long long n);
// Plain copy of n16 16-byte words (instrumentation: achievable stream rate).
hipError_t launch_stream_copy(hipStream_t s, const void* src, void* dst, long long n16);
long long ref_blocks(const Layout& L);
// partials written by the CFL kernel
long long cfl_blocks(const Layout& L);
// dt of the interior of Q into *dt_out (and *also when not null); axis != 0:
// the polar axis (j = 0) is left out
hipError_t launch_cfl(hipStream_t s, const Layout& L, const Phys& P, const double* M, const double* Q, double* part,
                      double* dt_out, int* flag, double* also = nullptr, int axis = 0);
// centerline condition on the axis nodes (j = 0) of a state
hipError_t launch_axis_avg(hipStream_t s, const Layout& L, double* q);
hipError_t launch_axis_avg_f32(hipStream_t s, const Layout& L, float* q);
// dt = cfl * min of np per-block CFL bounds (e.g. the stage kernel's)
hipError_t launch_cfl_final(hipStream_t s, const double* part, long long np, double cfl, double* dt_out,
                            double* also, int* flag);
hipError_t launch_residual_ref(hipStream_t s, const Layout& L, const Phys& P, const double* M, const double* Q,
                               const double* f, int i_f, double* R, double* part, const double* dyn, int axis);
hipError_t launch_stage_ref(hipStream_t s, const Layout& L, const Phys& P, const double* M, const double* Qin,
                            const double* Q0, double* Qout, const double* dtp, double dt, double alpha,
                            const double* f, int i_f, double* part, const double* dyn, int axis);
hipError_t launch_norm_final(hipStream_t s, const double* part, long long np, double count, double* norms, int* flag);
hipError_t launch_probe(hipStream_t s, const Layout& L, const Phys& P, int nks, const double* Q, int i_p,
                        double p_inf, double weight, double* Jacc, double* Qbar, double* part);

}  // namespace les
