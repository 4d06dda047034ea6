// les_common.hpp -- types and device building blocks shared by the gfx950
// kernels of the LES residual / Runge-Kutta library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace les {

constexpr int GH = 2;    // ghost layers per side (Sec. 4, Fig. 3)
constexpr int LEAD = 9;  // element offset of interior i = 0 inside a row (node i = -1 at 64 B)

// Library layout of one field (see include/les.h).
struct Layout {
  int ni, nj, nk;
  long long sj, sk;  // element strides of j and k (stride of i is 1)
  long long fe;      // field pitch in elements
  long long o;       // element offset of interior node (0, 0, 0)
  __host__ __device__ long long at(int i, int j, int k) const {
    return o + (long long)i + (long long)j * sj + (long long)k * sk;
  }
};

inline Layout make_layout(int ni, int nj, int nk) {
  Layout L;
  L.ni = ni; L.nj = nj; L.nk = nk;
  long long pitch = ((long long)LEAD + ni + GH + 15) / 16 * 16;
  L.sj = pitch;
  L.sk = pitch * (nj + 2 * GH);
  L.fe = (L.sk * (nk + 2 * GH) + 31) / 32 * 32;
  L.o = LEAD + GH * L.sj + GH * L.sk;
  return L;
}

// Dense padded layout [nk+4][nj+4][ni+4].
struct Dense {
  int ni, nj, nk;
  __host__ __device__ long long at(int i, int j, int k) const {
    return ((long long)(k + GH) * (nj + 2 * GH) + (j + GH)) * (long long)(ni + 2 * GH) + (i + GH);
  }
  __host__ __device__ long long n() const { return (long long)(ni + 4) * (nj + 4) * (nk + 4); }
};

// Flow / scheme constants, derived once on the host.
struct Phys {
  double gamma, gm1, inv_R, Cp_over_Pr, Cp_over_Prsgs;
  double mu_ref, inv_Tref, S, one_plus_S;
  double Cs2;  // Cs^2
  double k2, k4, alpha;
  double cfl, nu_fac;  // nu_fac = max(4/3, gamma/Pr)
  int sgs;         // 0 none, 1 static Smagorinsky, 2 dynamic coefficients per column
  int alpha_half;  // alpha == 1/2: Lam_d = lam_d + sqrt(lam_d)(sqrt(lam_e) + sqrt(lam_f))
  double gamma_R;  // gamma * R (c^2 = gamma R T)
  double CI43;     // (4/3) CI: sigma_kk / 3 = CI43 rho D^2 S_ij S_ij (0 = no isotropic SGS stress)
  double Cp;
};

// Per-column dynamic coefficients (sgs == 2): C at dyn[c], D_T at
// dyn[ncol + c], c = (j + 2)(ni + 4) + (i + 2) for nodes with i, j in
// [-2, n+1] (ghost columns included).
__host__ __device__ inline long long dyn_col(const Layout& L, int i, int j) {
  return (long long)(j + 2) * (L.ni + 4) + (i + 2);
}
__host__ __device__ inline long long dyn_ncol(const Layout& L) { return (long long)(L.nj + 4) * (L.ni + 4); }

// Runge-Kutta coefficients of the five-stage scheme.
__host__ __device__ inline double rk_alpha(int l) {
  return l == 0 ? 0.25 : l == 1 ? (1.0 / 6.0) : l == 2 ? 0.375 : l == 3 ? 0.5 : 1.0;
}

// ---------------------------------------------------------------------------
// Pointwise physics (templated on the compute type T).
// ---------------------------------------------------------------------------
// Primitive variables from Q (Eq. 2, 7): u, v, w, p, T.
template <class T>
__device__ __forceinline__ void prim_from_q(T q0, T q1, T q2, T q3, T q4, const Phys& P, T& u, T& v, T& w, T& p,
                                            T& tem) {
  T ir = T(1) / q0;
  u = q1 * ir;
  v = q2 * ir;
  w = q3 * ir;
  p = T(P.gm1) * (q4 - T(0.5) * q0 * (u * u + v * v + w * w));
  tem = p * ir * T(P.inv_R);
}

// Sutherland's law (Eq. 6): mu_ref (T/T_ref)^{3/2} (1+S)/(T/T_ref + S).
template <class T>
__device__ __forceinline__ T sutherland(T tem, const Phys& P) {
  T th = tem * T(P.inv_Tref);
  return T(P.mu_ref * P.one_plus_S) * th * sqrt(th) / (th + T(P.S));
}

// Anisotropic spectral-radius scaling of Turkel and Vatsa for direction d
// given lam_d and the other two radii.
template <class T>
__device__ __forceinline__ T aniso(T ld, T le, T lf, const Phys& P) {
  if (P.alpha_half) {
    T sd = sqrt(ld);
    return ld + sd * (sqrt(le) + sqrt(lf));
  }
  return ld * (T(1) + pow(le / ld, T(P.alpha)) + pow(lf / ld, T(P.alpha)));
}

template <class T>
__device__ __forceinline__ T tmax(T a, T b) { return a >= b ? a : b; }

// ---------------------------------------------------------------------------
// Short reciprocal / square-root sequences for the stage kernel: the
// hardware approximation refined by Newton steps, without the scaling and
// special-value handling of the IEEE sequences.  Valid for finite, normal,
// positive arguments (rcp: nonzero); the result is within a few ulp.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
// sqrt(x), x > 0: y ~ 1/sqrt(x) refined once (y += y (1 - x y^2) / 2), then
// s = x y corrected once (s += (x - s^2) y / 2).
__device__ __forceinline__ double sqrt_pos(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hy = 0.5 * y;
  y = fma(hy, fma(-x * y, y, 1.0), y);
  double s = x * y;
  return fma(0.5 * y, fma(-s, s, x), s);
}
__device__ __forceinline__ float sqrt_pos(float x) { return __builtin_amdgcn_sqrtf(x); }
// sqrt(x) for x >= 0 (0 at 0)
template <class T>
__device__ __forceinline__ T sqrt_nn(T x) { return x > T(0) ? sqrt_pos(x) : T(0); }

// J^(-1/3), J > 0: single-precision seed 2^(-log2(J)/3), then two Newton
// steps y += y (1 - J y^3) / 3 (each squares the relative error).
__device__ __forceinline__ double icbrt(double J) {
  const float jf = (float)J;
  double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(jf) * (-1.0f / 3.0f));
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-J * y, y * y, 1.0);
    y = fma(y * (1.0 / 3.0), e, y);
  }
  return y;
}
__device__ __forceinline__ float icbrt(float J) {
  float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(J) * (-1.0f / 3.0f));
  const float e = fmaf(-J * y, y * y, 1.0f);
  return fmaf(y * (1.0f / 3.0f), e, y);
}

// Primitive variables (as prim_from_q) with the short reciprocal.
template <class T>
__device__ __forceinline__ void prim_from_q_fast(T q0, T q1, T q2, T q3, T q4, const Phys& P, T& u, T& v, T& w,
                                                 T& p, T& tem) {
  T ir = rcp_nr(q0);
  u = q1 * ir;
  v = q2 * ir;
  w = q3 * ir;
  p = T(P.gm1) * (q4 - T(0.5) * q0 * (u * u + v * v + w * w));
  tem = p * ir * T(P.inv_R);
}

// Sutherland's law (as sutherland) with the short sequences.
template <class T>
__device__ __forceinline__ T sutherland_fast(T tem, const Phys& P) {
  T th = tem * T(P.inv_Tref);
  return T(P.mu_ref * P.one_plus_S) * th * sqrt_pos(th) * rcp_nr(th + T(P.S));
}

// Local CFL bound of one node (FP64, with the short reciprocal and square
// root): the inverse of
//   sum_d (|U_d| + c |grad d|) + 2 max(4/3, gamma/Pr) (mu/rho) sum_d |grad d|^2
// with the physical metrics grad d = J (d_x/J, d_y/J, d_z/J) (m9 = the nine
// metric terms over J, row by row) and the molecular viscosity of Eq. 6;
// dt = cfl * min over the interior.  NaN for a state with non-positive
// density or pressure, so that the minimum reports it (the short sequences
// may return anything there; the test below overrides it).
__device__ inline double cfl_local(double q0, double q1, double q2, double q3, double q4, double J,
                                   const double m9[9], const Phys& P) {
  double u, v, w, p, tem;
  prim_from_q_fast(q0, q1, q2, q3, q4, P, u, v, w, p, tem);
  const double ir = rcp_nr(q0);
  const double c = sqrt_pos(P.gamma * p * ir);
  const double nuv = P.nu_fac * sutherland_fast(tem, P) * ir;
  double lam = 0.0, g2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double gx = J * m9[3 * d], gy = J * m9[3 * d + 1], gz = J * m9[3 * d + 2];
    const double U = gx * u + gy * v + gz * w;
    const double gg = gx * gx + gy * gy + gz * gz;
    lam += fabs(U) + c * sqrt_pos(gg);
    g2 += gg;
  }
  double l = rcp_nr(lam + 2.0 * nuv * g2);
  if (!(l > 0.0) || !(q0 > 0.0) || !(p > 0.0)) l = __builtin_nan("");
  return l;
}

// min(a, b) in which a NaN wins (a non-physical state is reported)
__device__ __forceinline__ double min_nan(double a, double b) { return (b < a || b != b) ? b : a; }

// ---------------------------------------------------------------------------
// Wavefront / block reductions (64-lane wavefronts).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_down(v, off, 64);
    v = (o > v || o != o) ? o : v;  // NaN wins so that it is reported
  }
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_down(v, off, 64);
    v = (o < v || o != o) ? o : v;
  }
  return v;
}

}  // namespace les
