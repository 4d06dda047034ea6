// les_faces.hpp -- boundary faces of a Dirichlet direction (Sec. 3: entrance,
// far field and exit of the jet domain), shared by the ghost fill (forward)
// and the adjoint (its Jacobian, by forward-mode dual numbers).
#pragma once
#include "les_common.hpp"

namespace les {

// Faces in the order i-lo, i-hi, j-lo, j-hi, k-lo, k-hi (les_set_face):
// 0 = frozen ghosts, 1 = characteristic entrance, 2 = subsonic exit with
// imposed pressure, 3 = far field.
struct Faces {
  int type[6];
  double p_exit[6];
  const double* outside;  // [5][fe] outside state at the ghost nodes (characteristic and far-field faces)
  const double* M;        // metrics [10][fe] (face normals)
  double gamma;
  int any;                // some face is not frozen
  int axis;               // j = 0 is the polar axis (face normals there, see face_normal)
};

// A value with one derivative (forward mode), enough for the face rule.
struct DualD {
  double v, d;
  __host__ __device__ DualD() : v(0.0), d(0.0) {}
  __host__ __device__ DualD(double a) : v(a), d(0.0) {}
  __host__ __device__ DualD(double a, double b) : v(a), d(b) {}
};
__host__ __device__ inline DualD operator+(DualD a, DualD b) { return DualD(a.v + b.v, a.d + b.d); }
__host__ __device__ inline DualD operator-(DualD a, DualD b) { return DualD(a.v - b.v, a.d - b.d); }
__host__ __device__ inline DualD operator*(DualD a, DualD b) { return DualD(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ inline DualD operator/(DualD a, DualD b) {
  return DualD(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
__host__ __device__ inline double fval(double a) { return a; }
__host__ __device__ inline double fval(DualD a) { return a.v; }
__device__ inline double fsqrt(double a) { return sqrt(a); }
__device__ inline DualD fsqrt(DualD a) {
  const double s = sqrt(a.v);
  return DualD(s, a.d / (2.0 * s));
}
__device__ inline double fpow(double a, double e) { return pow(a, e); }
__device__ inline DualD fpow(DualD a, double e) {
  const double p = pow(a.v, e);
  return DualD(p, e * p / a.v * a.d);
}

// Ghost state of a boundary face from the boundary node's conserved state
// qr, the outside state qo and the outward unit normal nv:
//   exit (type 2, subsonic, imposed pressure pe): velocity and internal
//     energy per unit mass p / ((gamma - 1) rho) of the boundary node are
//     kept, p = pe, so rho = rho_r pe / p_r and e = pe / (gamma - 1) +
//     rho |u|^2 / 2;
//   far field (type 3; Sec. 3: Riemann invariants, normal velocity
//     extrapolated at zero order, fixed flow angle, the rest from the jet
//     Mach number carried by the outside state): u.n of the boundary node;
//     tangential velocity of the outside state; the outside state's incoming
//     invariant u.n - 2c/(gamma-1) gives c; entropy p / rho^gamma from
//     outside when u.n < 0, from the boundary node otherwise;
//   characteristic (type 1, the entrance; locally one-dimensional along nv): supersonic
//     outflow at the boundary node keeps its state, supersonic inflow from
//     outside takes the outside state; otherwise the outgoing Riemann
//     invariant u.n + 2c/(gamma-1) comes from the boundary node and the
//     incoming one u.n - 2c/(gamma-1) from outside, and the entropy
//     p / rho^gamma and the tangential velocity from the boundary node
//     (outflow, u.n >= 0) or from outside.
// T = double (the ghost fill) or DualD (its derivative along a direction of
// qr; branches follow the values).
template <class T>
__device__ void face_value(int type, double gamma, double pe, const double nv[3], const T qr[5],
                           const double qo[5], T out[5]) {
  const double gm1 = gamma - 1.0;
  const T rr = qr[0];
  const T ur[3] = {qr[1] / rr, qr[2] / rr, qr[3] / rr};
  const T kr = ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2];
  const T pr = T(gm1) * (qr[4] - T(0.5) * rr * kr);
  if (type == 2) {
    const T rho = rr * T(pe) / pr;
    out[0] = rho;
    for (int a = 0; a < 3; ++a) out[1 + a] = rho * ur[a];
    out[4] = T(pe / gm1) + T(0.5) * rho * kr;
    return;
  }
  const double ro = qo[0];
  const double uo[3] = {qo[1] / ro, qo[2] / ro, qo[3] / ro};
  const double po = gm1 * (qo[4] - 0.5 * ro * (uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2]));
  const T cr = fsqrt(T(gamma) * pr / rr);
  const double co = sqrt(gamma * po / ro);
  const T unr = ur[0] * T(nv[0]) + ur[1] * T(nv[1]) + ur[2] * T(nv[2]);
  const double uno = uo[0] * nv[0] + uo[1] * nv[1] + uo[2] * nv[2];
  if (type == 3) {
    // far field: u.n kept from the boundary node, tangential velocity (the
    // fixed flow angle) and incoming invariant u.n - 2c/(gamma-1) from
    // outside, entropy from outside on inflow and from the node otherwise
    const double rm = uno - 2.0 * co / gm1;
    const T c = T(0.5 * gm1) * (unr - T(rm));
    const T ent = fval(unr) >= 0.0 ? pr / fpow(rr, gamma) : T(po / pow(ro, gamma));
    const T rho = fpow(c * c / (T(gamma) * ent), 1.0 / gm1);
    const T p = rho * c * c / T(gamma);
    T k = T(0.0);
    out[0] = rho;
    for (int a = 0; a < 3; ++a) {
      const T ub = T(uo[a] - uno * nv[a]) + unr * T(nv[a]);
      out[1 + a] = rho * ub;
      k = k + ub * ub;
    }
    out[4] = p / T(gm1) + T(0.5) * rho * k;
    return;
  }
  if (fval(unr) >= fval(cr)) {  // supersonic outflow
    for (int c = 0; c < 5; ++c) out[c] = qr[c];
    return;
  }
  if (uno <= -co) {  // supersonic inflow
    for (int c = 0; c < 5; ++c) out[c] = T(qo[c]);
    return;
  }
  const T rplus = unr + T(2.0) * cr / T(gm1);  // outgoing, from inside
  const double rminus = uno - 2.0 * co / gm1;  // incoming, from outside
  const T un = T(0.5) * (rplus + T(rminus));
  const T c = T(0.25 * gm1) * (rplus - T(rminus));
  const bool from_r = fval(un) >= 0.0;
  const T ent = from_r ? pr / fpow(rr, gamma) : T(po / pow(ro, gamma));
  T us[3], uns;
  if (from_r) {
    for (int a = 0; a < 3; ++a) us[a] = ur[a];
    uns = unr;
  } else {
    for (int a = 0; a < 3; ++a) us[a] = T(uo[a]);
    uns = T(uno);
  }
  const T rho = fpow(c * c / (T(gamma) * ent), 1.0 / gm1);
  const T p = rho * c * c / T(gamma);
  T k = T(0.0);
  out[0] = rho;
  for (int a = 0; a < 3; ++a) {
    const T ub = us[a] - uns * T(nv[a]) + un * T(nv[a]);
    out[1 + a] = rho * ub;
    k = k + ub * ub;
  }
  out[4] = p / T(gm1) + T(0.5) * rho * k;
}

// Outward unit normal of face (d, hi) at node rn from grad(xi_d) = J (xi_d/J).
__device__ inline void face_normal(const Layout& L, const Faces& F, int d, int hi, int i, int j, int k,
                                   double nv[3]) {
  const double* __restrict__ M = F.M;
  if (F.axis && j == 0 && d != 1) {
    // on the polar axis every azimuth meets and the metric row of d
    // vanishes: the normal is the azimuthal mean of the unit normals of the
    // ring j = 1 (k' = 0 .. nk - 2, ascending), normalised
    double sm[3] = {0.0, 0.0, 0.0};
    for (int kk = 0; kk < L.nk - 1; ++kk) {
      const long long rr = L.at(i, 1, kk);
      const double J = M[9 * L.fe + rr];
      double u[3], nrm = 0.0;
      for (int x = 0; x < 3; ++x) {
        u[x] = J * M[(3 * d + x) * L.fe + rr];
        nrm += u[x] * u[x];
      }
      const double inv = 1.0 / sqrt(nrm);
      for (int x = 0; x < 3; ++x) sm[x] += u[x] * inv;
    }
    const double sg = (hi ? 1.0 : -1.0) / sqrt(sm[0] * sm[0] + sm[1] * sm[1] + sm[2] * sm[2]);
    for (int x = 0; x < 3; ++x) nv[x] = sm[x] * sg;
    return;
  }
  const long long rn = L.at(i, j, k);
  const double J = M[9 * L.fe + rn];
  double nrm = 0.0;
  for (int x = 0; x < 3; ++x) {
    nv[x] = J * M[(3 * d + x) * L.fe + rn];
    nrm += nv[x] * nv[x];
  }
  const double sg = (hi ? 1.0 : -1.0) / sqrt(nrm);
  for (int x = 0; x < 3; ++x) nv[x] *= sg;
}

}  // namespace les
