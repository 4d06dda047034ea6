// les_adjoint.hip -- reverse mode (adjoint) of the residual and of one
// Runge-Kutta step, written as gather kernels.
//
// For a residual weight Rbar on the interior, Qbar = (dR/dQ)^T Rbar is the
// reverse of the residual's composition (Eq. 12-15 with the Turkel-Vatsa
// dissipation): node primitives -> node gradients -> stress / heat flux /
// eddy viscosity -> node fluxes and spectral radii / sensors -> face fluxes
// -> residual.  Every backward step that would scatter is written as a
// gather over stored per-node weights, so no atomics are needed:
//   pass 1 (node, nodes with indices in [-1, n]): with W = J Rbar (zero off
//      the interior) the node flux adjoint is Hbar_d(n) = (W(n-e_d) -
//      W(n+e_d))/2; the thread reverses its node flux, viscous stress, heat
//      flux, Smagorinsky and Sutherland viscosity and its share of the two
//      dissipation faces on each side, and stores: the adjoint in primitive
//      variables (rho, u, v, w, p, T), the direct Q adjoint of the fluxes,
//      the gradient-stencil weights a_{q,d} = J m_d . gbar_q, the sensor
//      weights for p at n +- e_d, and the face coefficients
//      Lambda eps2, Lambda eps4 of the face (n, n + e_d);
//   pass 2 (gather, interior nodes and their periodic ghost images):
//      collects the gradient and sensor weights of its neighbours and the
//      dissipation faces whose five-point stencil contains it, and maps the
//      primitive adjoint back to conserved variables;
//   pass 3 (fold, interior nodes with ghost images): adds the adjoint of
//      every periodic ghost image to its interior node and pulls the
//      adjoint of a boundary face's ghosts back to the face's boundary node
//      through the face rule's Jacobian (frozen Dirichlet ghosts carry no
//      dependence).
// Non-smooth points take the derivative of the active branch: d|x|/dx =
// sign(x) with 0 at 0, max(a, b) follows a when a >= b, and the eddy
// viscosity's |S| has derivative 0 at |S| = 0.
//
// les_adjoint_step applies it stage by stage in reverse from the stage
// inputs saved by les_rk_step: for l = 5..1, acc += qbar, fbar += alpha_l dt
// qbar on the source plane, qbar = (dR/dQ|Q^(l-1))^T (-alpha_l dt qbar);
// finally Qbar = acc + qbar.  The accumulation, the fbar update and the
// final sum run inside passes 2 and 3 of the next (or last) stage.
#include "les_adjoint.hpp"

namespace les {

namespace {

// Work-array field indices (library layout, one field each).
enum {
  W_PRHO = 0, W_PU, W_PV, W_PW, W_PP, W_PT,  // primitive-variable adjoint (local part)
  W_QD1, W_QD2, W_QD3, W_QD4,                 // direct Q adjoint of the node fluxes
  W_A = 10,                                   // a_{q,d}: 12 fields, index W_A + 3 q + d
  W_CP = 22,                                  // sensor weights for p(n +- e_d): 3 fields
  W_A2 = 25,                                  // Lambda eps2 of face (n, n+e_d): 3 fields
  W_A4 = 28,                                  // Lambda eps4 of face (n, n+e_d): 3 fields
  W_LAM = 31,                                 // Lambda_d at the node: 3 fields
  W_NU = 34,                                  // signed sensor (p+ - 2p + p-) / Sigma: 3 fields
  W_LH = 37,                                  // half the face-mean adjoint of face (n, n+e_d): 3
  W_NUA = 40,                                 // sensor adjoint of face (n, n+e_d) for node n: 3
  W_NUB = 43,                                 // ... for node n + e_d: 3
  W_Q1 = 46,                                  // stage adjoint ping-pong: 5 + 5 fields
  W_ACC = 56,                                 // accumulated adjoint of Q^(0): 5 fields
  W_DB = 61,                                  // Dbar = W(n+e_d) - W(n) of face (n, n+e_d): 15
  W_IS = 76,                                  // 1 / Sigma of the sensor, Sigma = p+ + 2p + p-: 3
  W_GG = 79,                                  // gather result at periodic ghost images: 5
  W_NF = 84
};

struct Prim {
  double rho, u, v, w, p, T;
};

__device__ __forceinline__ Prim prim_at(const double* __restrict__ Q, long long fe, long long n, const Phys& P) {
  Prim r;
  r.rho = Q[n];
  prim_from_q_fast(r.rho, Q[fe + n], Q[2 * fe + n], Q[3 * fe + n], Q[4 * fe + n], P, r.u, r.v, r.w, r.p, r.T);
  return r;
}

__device__ __forceinline__ long long dstr(const Layout& L, int d) { return d == 0 ? 1LL : (d == 1 ? L.sj : L.sk); }

__device__ __forceinline__ bool interior(const Layout& L, int i, int j, int k) {
  return i >= 0 && i < L.ni && j >= 0 && j < L.nj && k >= 0 && k < L.nk;
}

// Does the face (a, a + e_d) exist, i.e. is it used by an interior residual?
__device__ __forceinline__ bool face_ok(const Layout& L, int d, int i, int j, int k) {
  const int id[3] = {i, j, k};
  const int nn[3] = {L.ni, L.nj, L.nk};
  for (int e = 0; e < 3; ++e) {
    if (e == d) {
      if (id[e] < -1 || id[e] > nn[e] - 1) return false;
    } else if (id[e] < 0 || id[e] >= nn[e]) {
      return false;
    }
  }
  return true;
}

// W = coef * J * qbar on the interior, zero elsewhere and on the polar axis
// (whose nodes the residual does not advance; J is infinite there).
__device__ __forceinline__ void Wat(const Layout& L, const double* __restrict__ M, const double* __restrict__ qb,
                                    double coef, int i, int j, int k, double W[5], bool axis) {
  if (!interior(L, i, j, k) || (axis && j == 0)) {
    for (int c = 0; c < 5; ++c) W[c] = 0.0;
    return;
  }
  const long long n = L.at(i, j, k);
  const double s = coef * M[9 * L.fe + n];
  for (int c = 0; c < 5; ++c) W[c] = s * qb[c * L.fe + n];
}

// Spectral radii and their ingredients at node n.
struct Radii {
  double lam[3], U[3], nrm[3], c;
};

__device__ __forceinline__ Radii radii_at(const double* __restrict__ M, long long fe, long long n, const Prim& q,
                                          const Phys& P) {
  Radii r;
  r.c = sqrt_pos(P.gamma_R * q.T);  // c^2 = gamma p / rho = gamma R T
  for (int e = 0; e < 3; ++e) {
    const double mx = M[(3 * e) * fe + n], my = M[(3 * e + 1) * fe + n], mz = M[(3 * e + 2) * fe + n];
    r.U[e] = mx * q.u + my * q.v + mz * q.w;
    r.nrm[e] = sqrt_pos(mx * mx + my * my + mz * mz);
    r.lam[e] = fabs(r.U[e]) + r.c * r.nrm[e];
  }
  return r;
}

// Anisotropic scaling Lam_d and its partial derivatives w.r.t. (lam_d, lam_e, lam_f).
__device__ __forceinline__ double aniso_d(double ld, double le, double lf, const Phys& P, double& dd, double& de,
                                          double& df) {
  if (P.alpha_half) {
    // Lam = ld + sqrt(ld) (sqrt(le) + sqrt(lf))
    const double sd = sqrt_pos(ld), se = sqrt_pos(le), sf = sqrt_pos(lf);
    dd = 1.0 + 0.5 * (se + sf) * rcp_nr(sd);
    de = 0.5 * sd * rcp_nr(se);
    df = 0.5 * sd * rcp_nr(sf);
    return ld + sd * (se + sf);
  }
  const double a = P.alpha;
  const double re = pow(le / ld, a), rf = pow(lf / ld, a);
  dd = 1.0 + (1.0 - a) * (re + rf);
  de = a * re * ld / le;
  df = a * rf * ld / lf;
  return ld * (1.0 + re + rf);
}

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

struct AdjK {
  Layout L;
  Phys P;
  const double* M;
  int bc0, bc1, bc2;
  int per[3];          // period of each axis: n (periodic), n - 1 (superposed), 0 (Dirichlet)
  int lo[3], hi[3];    // pass-2 box: ghost layers of periodic axes and of active faces included
  Faces F;             // boundary faces
  int general;         // a superposed axis, the polar axis or an active face: pass 3 visits every interior node
  int axis;            // j = 0 is the polar axis (bc1 == 3)
};

AdjK make_adjk(const AdjArgs& a) {
  AdjK A;
  A.L = a.L;
  A.P = a.P;
  A.M = a.M;
  A.bc0 = a.bc0;
  A.bc1 = a.bc1;
  A.bc2 = a.bc2;
  A.F = a.F;
  A.general = 0;
  A.axis = a.axis;
  const int bc[3] = {a.bc0, a.bc1, a.bc2}, nn[3] = {a.L.ni, a.L.nj, a.L.nk};
  for (int d = 0; d < 3; ++d) {
    // bc 3 (polar axis, j only): its lo side is the axis, whose cross-axis
    // ghosts are images of interior nodes; its hi side is Dirichlet
    const bool per_like_lo = bc[d] == 0 || bc[d] == 2 || bc[d] == 3;
    const bool per_like_hi = bc[d] == 0 || bc[d] == 2;
    A.per[d] = bc[d] == 0 ? nn[d] : (bc[d] == 2 ? nn[d] - 1 : 0);
    const bool flo = bc[d] == 1 && a.F.type[2 * d] != 0;
    const bool fhi = (bc[d] == 1 || bc[d] == 3) && a.F.type[2 * d + 1] != 0;
    A.lo[d] = (per_like_lo || flo) ? -2 : 0;
    A.hi[d] = (per_like_hi || fhi) ? nn[d] + 1 : nn[d] - 1;
    if (bc[d] == 2 || bc[d] == 3 || flo || fhi) A.general = 1;
  }
  return A;
}

// ---------------------------------------------------------------------------
// Pass 1
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adj_flux(AdjK A, const double* __restrict__ Q, const double* __restrict__ qb,
                                                  double coef, double* __restrict__ Wk) {
  const Layout& L = A.L;
  const Phys& P = A.P;
  const long long fe = L.fe;
  const double* __restrict__ M = A.M;
  // (the adjoint entry points refuse blocks of 2^30 padded nodes or more: 32-bit index math)
  const unsigned ext_i = L.ni + 2, ext_j = L.nj + 2;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ext_i * ext_j * (unsigned)(L.nk + 2)) return;
  const int i = (int)(t % ext_i) - 1;
  const int j = (int)((t / ext_i) % ext_j) - 1;
  const int k = (int)(t / (ext_i * ext_j)) - 1;
  const long long n = L.at(i, j, k);

  const Prim q = prim_at(Q, fe, n, P);
  double m[9];
  for (int c = 0; c < 9; ++c) m[c] = M[c * fe + n];
  const double J = M[9 * fe + n];

  // ---- forward recomputation at the node ----
  double g[4][3];
  {
    double dd[3][4];
    for (int d = 0; d < 3; ++d) {
      const long long s = dstr(L, d);
      const Prim a = prim_at(Q, fe, n + s, P), b = prim_at(Q, fe, n - s, P);
      dd[d][0] = 0.5 * (a.u - b.u);
      dd[d][1] = 0.5 * (a.v - b.v);
      dd[d][2] = 0.5 * (a.w - b.w);
      dd[d][3] = 0.5 * (a.T - b.T);
      // for the dissipation adjoint: signed sensor (p+ - 2p + p-) / Sigma and 1 / Sigma
      const double iS = rcp_nr(a.p + 2.0 * q.p + b.p);
      Wk[(W_NU + d) * fe + n] = (a.p - 2.0 * q.p + b.p) * iS;
      Wk[(W_IS + d) * fe + n] = iS;
    }
    for (int qq = 0; qq < 4; ++qq)
      for (int x = 0; x < 3; ++x) g[qq][x] = J * (m[x] * dd[0][qq] + m[3 + x] * dd[1][qq] + m[6 + x] * dd[2][qq]);
  }
  if (A.axis && j <= 0) {
    // polar axis: its residual is not formed (W = 0 around it along xi and
    // zeta) and its eta node flux and spectral radius are the constant 0;
    // the row below it (a ghost across the axis, where J < 0) serves only
    // the axis residual.  Nothing but the pressure sensors (kept above)
    // depends on them here
    for (int d = 0; d < 3; ++d) Wk[(W_LAM + d) * fe + n] = 0.0;
    for (int c = 0; c < 12; ++c) Wk[(W_A + c) * fe + n] = 0.0;
    for (int c = W_PRHO; c <= W_PT; ++c) Wk[c * fe + n] = 0.0;
    for (int a = 0; a < 4; ++a) Wk[(W_QD1 + a) * fe + n] = 0.0;
    return;
  }
  {
    // for the dissipation adjoint: Lambda_d at the node
    const Radii r = radii_at(M, fe, n, q, P);
    for (int d = 0; d < 3; ++d) {
      double dd0, de0, df0;
      Wk[(W_LAM + d) * fe + n] = aniso_d(r.lam[d], r.lam[(d + 1) % 3], r.lam[(d + 2) % 3], P, dd0, de0, df0);
    }
  }
  const double S11 = g[0][0], S22 = g[1][1], S33 = g[2][2];
  const double S12 = 0.5 * (g[0][1] + g[1][0]), S13 = 0.5 * (g[0][2] + g[2][0]), S23 = 0.5 * (g[1][2] + g[2][1]);
  const double skk3 = (S11 + S22 + S33) * (1.0 / 3.0);
  const double th = q.T * P.inv_Tref;
  const double ithS = rcp_nr(th + P.S);
  const double mu = P.mu_ref * P.one_plus_S * th * sqrt_pos(th) * ithS;
  double mus = 0.0, Smag = 0.0, cd2 = 0.0, ss = 0.0, cid2 = 0.0, pis = 0.0;
  if (P.sgs) {
    ss = S11 * S11 + S22 * S22 + S33 * S33 + 2.0 * (S12 * S12 + S13 * S13 + S23 * S23);
    Smag = sqrt_nn(2.0 * ss);
    double d2 = icbrt(J);  // (1/J)^(1/3)
    cd2 = P.Cs2 * d2 * d2;
    mus = q.rho * cd2 * Smag;
    // isotropic SGS stress: sigma_kk / 3 = CI43 rho D^2 S:S, added to the
    // pressure of the momentum and energy fluxes (not to the sensor or the
    // spectral radii)
    cid2 = P.CI43 * d2 * d2;
    pis = q.rho * cid2 * ss;
  }
  const double pe = q.p + pis;
  const double mt = mu + mus;
  const double mt2 = 2.0 * mt;
  const double tau[3][3] = {{mt2 * (S11 - skk3), mt2 * S12, mt2 * S13},
                            {mt2 * S12, mt2 * (S22 - skk3), mt2 * S23},
                            {mt2 * S13, mt2 * S23, mt2 * (S33 - skk3)}};
  const double kap = mu * P.Cp_over_Pr + mus * P.Cp_over_Prsgs;
  const double uu[3] = {q.u, q.v, q.w};

  // ---- adjoint accumulators ----
  double rb = 0, ub[3] = {0, 0, 0}, pb = 0, Tb = 0;  // primitive adjoint
  double qd[4] = {0, 0, 0, 0};                        // direct Q1..Q4 adjoint
  double tb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // tau adjoint (full, symmetrised below)
  double thb[3] = {0, 0, 0};                          // Theta adjoint
  const double Qv[5] = {q.rho, Q[fe + n], Q[2 * fe + n], Q[3 * fe + n], Q[4 * fe + n]};

  // ---- node flux adjoints Hbar_d = (W(n-e) - W(n+e)) / 2 ----
  for (int d = 0; d < 3; ++d) {
    const int di = d == 0, dj = d == 1, dk = d == 2;
    double Wm[5], Wp[5];
    Wat(L, M, qb, coef, i - di, j - dj, k - dk, Wm, A.axis);
    Wat(L, M, qb, coef, i + di, j + dj, k + dk, Wp, A.axis);
    double Hb[5];
    bool any = false;
    for (int c = 0; c < 5; ++c) {
      Hb[c] = 0.5 * (Wm[c] - Wp[c]);
      any = any || Hb[c] != 0.0;
    }
    if (!any) continue;
    const double mx = m[3 * d], my = m[3 * d + 1], mz = m[3 * d + 2];
    const double mm[3] = {mx, my, mz};
    const double U = mx * q.u + my * q.v + mz * q.w;
    double Ub = 0.0;
    // H0 = rho U
    rb += Hb[0] * U;
    Ub += Hb[0] * q.rho;
    // H_{1+a} = Q_{1+a} U + m_a p - m . tau_a
    for (int a = 0; a < 3; ++a) {
      qd[a] += Hb[1 + a] * U;
      Ub += Hb[1 + a] * Qv[1 + a];
      pb += Hb[1 + a] * mm[a];
      for (int x = 0; x < 3; ++x) tb[a][x] -= Hb[1 + a] * mm[x];
    }
    // H4 = (e + p) U - m . Theta
    qd[3] += Hb[4] * U;
    pb += Hb[4] * U;
    Ub += Hb[4] * (Qv[4] + pe);
    for (int x = 0; x < 3; ++x) thb[x] -= Hb[4] * mm[x];
    ub[0] += Ub * mx;
    ub[1] += Ub * my;
    ub[2] += Ub * mz;
  }
  // so far pb is the adjoint of the flux pressure p + sigma_kk / 3
  const double peb = pb;
  // ---- Theta_x = u_a tau_ax + kappa dT/dx ----
  double kapb = 0.0;
  double gb[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int x = 0; x < 3; ++x) {
    for (int a = 0; a < 3; ++a) {
      ub[a] += thb[x] * tau[a][x];
      tb[a][x] += uu[a] * thb[x];
    }
    kapb += thb[x] * g[3][x];
    gb[3][x] += kap * thb[x];
  }
  // ---- tau = 2 mt (S - delta skk/3), symmetric ----
  const double t11 = tb[0][0], t22 = tb[1][1], t33 = tb[2][2];
  const double t12 = tb[0][1] + tb[1][0], t13 = tb[0][2] + tb[2][0], t23 = tb[1][2] + tb[2][1];
  const double mtb = 2.0 * ((S11 - skk3) * t11 + (S22 - skk3) * t22 + (S33 - skk3) * t33 + S12 * t12 + S13 * t13 +
                            S23 * t23);
  const double tr = (t11 + t22 + t33) * (1.0 / 3.0);
  double Sb11 = mt2 * (t11 - tr), Sb22 = mt2 * (t22 - tr), Sb33 = mt2 * (t33 - tr);
  double Sb12 = mt2 * t12, Sb13 = mt2 * t13, Sb23 = mt2 * t23;
  // ---- viscosities ----
  const double mub = mtb + kapb * P.Cp_over_Pr;
  if (P.sgs) {
    const double musb = mtb + kapb * P.Cp_over_Prsgs;
    rb += musb * cd2 * Smag;
    if (Smag > 0.0) {
      const double sb = musb * q.rho * cd2 * rcp_nr(Smag);
      Sb11 += 2.0 * S11 * sb;
      Sb22 += 2.0 * S22 * sb;
      Sb33 += 2.0 * S33 * sb;
      Sb12 += 4.0 * S12 * sb;
      Sb13 += 4.0 * S13 * sb;
      Sb23 += 4.0 * S23 * sb;
    }
  }
  if (cid2 != 0.0) {
    // sigma_kk / 3 = CI43 rho D^2 S:S -> rho and S
    rb += peb * cid2 * ss;
    const double ssb = peb * q.rho * cid2;
    Sb11 += 2.0 * S11 * ssb;
    Sb22 += 2.0 * S22 * ssb;
    Sb33 += 2.0 * S33 * ssb;
    Sb12 += 4.0 * S12 * ssb;
    Sb13 += 4.0 * S13 * ssb;
    Sb23 += 4.0 * S23 * ssb;
  }
  // Sutherland: dmu/dT = mu (3/(2 th) - 1/(th + S)) / T_ref
  Tb += mub * mu * (1.5 * rcp_nr(th) - ithS) * P.inv_Tref;
  // ---- S from the velocity gradient ----
  gb[0][0] += Sb11;
  gb[1][1] += Sb22;
  gb[2][2] += Sb33;
  gb[0][1] += 0.5 * Sb12;
  gb[1][0] += 0.5 * Sb12;
  gb[0][2] += 0.5 * Sb13;
  gb[2][0] += 0.5 * Sb13;
  gb[1][2] += 0.5 * Sb23;
  gb[2][1] += 0.5 * Sb23;
  // gradient-stencil weights a_{q,d} = J m_d . gbar_q
  for (int qq = 0; qq < 4; ++qq)
    for (int d = 0; d < 3; ++d)
      Wk[(W_A + 3 * qq + d) * fe + n] = J * (m[3 * d] * gb[qq][0] + m[3 * d + 1] * gb[qq][1] + m[3 * d + 2] * gb[qq][2]);

  Wk[W_PRHO * fe + n] = rb;
  Wk[W_PU * fe + n] = ub[0];
  Wk[W_PV * fe + n] = ub[1];
  Wk[W_PW * fe + n] = ub[2];
  Wk[W_PP * fe + n] = pb;
  Wk[W_PT * fe + n] = Tb;
  for (int a = 0; a < 4; ++a) Wk[(W_QD1 + a) * fe + n] = qd[a];
}

// ---- dissipation adjoint, face by face (pass 1a also stores, per node and
// direction, Lambda_d, the signed pressure sensor (p+ - 2p + p-) / Sigma and
// 1 / Sigma) ----
// Pass 1c (one thread per face (a, b = a + e_d) used by an interior
// residual): the face's dissipation D = Lf (eps2 dQ - eps4 d3Q) reversed
// with Dbar = W(b) - W(a).  Stores the face coefficients Lambda eps2,
// Lambda eps4 (for the gather), half the adjoint of the face mean Lf (one
// share per end node) and the sensor adjoint k2 eps2bar, given to the end
// node whose sensor wins max(nu_a, nu_b) (a on ties).
__global__ void __launch_bounds__(256) k_adj_face(AdjK A, const double* __restrict__ Q, const double* __restrict__ qb,
                                                  double coef, double* __restrict__ Wk) {
  const Layout& L = A.L;
  const Phys& P = A.P;
  const long long fe = L.fe;
  const unsigned ni = L.ni, nj = L.nj, nk = L.nk;
  const unsigned F0 = (ni + 1) * nj * nk, F1 = ni * (nj + 1) * nk, F2 = ni * nj * (nk + 1);
  unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= F0 + F1 + F2) return;
  int d, ai, aj, ak;
  if (t < F0) {
    d = 0;
    ai = (int)(t % (ni + 1)) - 1; aj = (int)((t / (ni + 1)) % nj); ak = (int)(t / ((ni + 1) * nj));
  } else if (t < F0 + F1) {
    t -= F0;
    d = 1;
    ai = (int)(t % ni); aj = (int)((t / ni) % (nj + 1)) - 1; ak = (int)(t / (ni * (nj + 1)));
  } else {
    t -= F0 + F1;
    d = 2;
    ai = (int)(t % ni); aj = (int)((t / ni) % nj); ak = (int)(t / (ni * nj)) - 1;
  }
  const int di = d == 0, dj = d == 1, dk = d == 2;
  const long long s = dstr(L, d);
  const long long an = L.at(ai, aj, ak), bn = an + s;
  const bool axis_face = A.axis && d == 1 && aj == 0;
  const double La = Wk[(W_LAM + d) * fe + an], Lb = Wk[(W_LAM + d) * fe + bn];
  const double na = fabs(Wk[(W_NU + d) * fe + an]), nb = fabs(Wk[(W_NU + d) * fe + bn]);
  const double e2 = P.k2 * (na >= nb ? na : nb);
  const double e4raw = P.k4 - e2;
  const bool e4_active = !(0.0 >= e4raw);  // max(0, x) follows 0 on ties
  const double e4 = e4_active ? e4raw : 0.0;
  const double Lf = 0.5 * (La + Lb);
  double Wa[5], Wb[5];
  Wat(L, A.M, qb, coef, ai, aj, ak, Wa, A.axis);
  Wat(L, A.M, qb, coef, ai + di, aj + dj, ak + dk, Wb, A.axis);
  double Lfb = 0.0, e2b = 0.0, e4b = 0.0;
  for (int c = 0; c < 5; ++c) {
    const double Db = Wb[c] - Wa[c];
    Wk[(W_DB + 5 * d + c) * fe + an] = Db;
    const double* Qc = Q + c * fe;
    const double d1 = Qc[bn] - Qc[an];
    // the face between the axis and j = 1 takes the cross-axis value by
    // linear extrapolation, Q(-1) = 2 Q(0) - Q(1): d3 = Q(2) - 2 Q(1) + Q(0)
    const double qam = axis_face ? 2.0 * Qc[an] - Qc[bn] : Qc[an - s];
    const double d3 = Qc[bn + s] - 3.0 * Qc[bn] + 3.0 * Qc[an] - qam;
    Lfb += Db * (e2 * d1 - e4 * d3);
    e2b += Db * Lf * d1;
    e4b -= Db * Lf * d3;
  }
  if (e4_active) e2b -= e4b;
  const bool a_wins = na >= nb;
  Wk[(W_A2 + d) * fe + an] = Lf * e2;
  Wk[(W_A4 + d) * fe + an] = Lf * e4;
  Wk[(W_LH + d) * fe + an] = 0.5 * Lfb;
  Wk[(W_NUA + d) * fe + an] = a_wins ? P.k2 * e2b : 0.0;
  Wk[(W_NUB + d) * fe + an] = a_wins ? 0.0 : P.k2 * e2b;
}

// Pass 1d (nodes in [-1, n]^3): the node's shares of its two faces per
// direction, back through Lambda_d(lam_d, lam_e, lam_f), lam = |U| + c|m|
// and nu_d(p(n-e), p, p(n+e)) to the primitive variables (added to pass 1a's
// part); stores the sensor weight of p(n +- e) for the gather.
__global__ void __launch_bounds__(256) k_adj_dnode(AdjK A, const double* __restrict__ Q, double* __restrict__ Wk) {
  const Layout& L = A.L;
  const Phys& P = A.P;
  const long long fe = L.fe;
  const double* __restrict__ M = A.M;
  const unsigned ext_i = L.ni + 2, ext_j = L.nj + 2;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ext_i * ext_j * (unsigned)(L.nk + 2)) return;
  const int i = (int)(t % ext_i) - 1;
  const int j = (int)((t / ext_i) % ext_j) - 1;
  const int k = (int)(t / (ext_i * ext_j)) - 1;
  const long long n = L.at(i, j, k);

  double rb = 0, ub[3] = {0, 0, 0}, pb = 0;
  double lamb[3] = {0, 0, 0};
  bool any = false;
  // on the polar axis the spectral radii are constants (0 along eta; the
  // others serve only faces between axis nodes, whose adjoint is 0): only
  // the pressure sensors depend on the state there
  const bool on_axis = A.axis && j == 0;
  Prim q;
  Radii r0;
  for (int d = 0; d < 3; ++d) {
    const long long s = dstr(L, d);
    const int di = d == 0, dj = d == 1, dk = d == 2;
    const bool f_lo = face_ok(L, d, i - di, j - dj, k - dk);  // face (n-e, n): node is b
    const bool f_hi = face_ok(L, d, i, j, k);                 // face (n, n+e): node is a
    double cpw = 0.0;
    if (f_lo || f_hi) {
      if (!any && !on_axis) {
        q = prim_at(Q, fe, n, P);
        r0 = radii_at(M, fe, n, q, P);
        any = true;
      }
      const double nub = (f_lo ? Wk[(W_NUB + d) * fe + n - s] : 0.0) + (f_hi ? Wk[(W_NUA + d) * fe + n] : 0.0);
      if (!on_axis) {
        const double Lamb = (f_lo ? Wk[(W_LH + d) * fe + n - s] : 0.0) + (f_hi ? Wk[(W_LH + d) * fe + n] : 0.0);
        // Lambda_d(n) -> lam_d, lam_e, lam_f
        double dd0, de0, df0;
        aniso_d(r0.lam[d], r0.lam[(d + 1) % 3], r0.lam[(d + 2) % 3], P, dd0, de0, df0);
        lamb[d] += Lamb * dd0;
        lamb[(d + 1) % 3] += Lamb * de0;
        lamb[(d + 2) % 3] += Lamb * df0;
      }
      // nu_d(n) = |Delta2| / Sigma with p(n-e), p(n), p(n+e): from the
      // pre-pass, Delta2 / Sigma (signed) and 1 / Sigma
      const double ns = Wk[(W_NU + d) * fe + n], iSg = Wk[(W_IS + d) * fe + n];
      const double sd = sgn(ns) * iSg, sv = fabs(ns) * iSg;
      pb += nub * (-2.0 * sd - 2.0 * sv);
      cpw = nub * (sd - sv);  // weight of p(n - e) and p(n + e)
    }
    Wk[(W_CP + d) * fe + n] = cpw;
  }
  if (on_axis) {
    Wk[W_PP * fe + n] += pb;
    return;
  }
  if (!any) return;
  // lam_e = |U_e| + c |m_e|
  double cb = 0.0;
  for (int e = 0; e < 3; ++e) {
    if (lamb[e] == 0.0) continue;
    const double Ueb = sgn(r0.U[e]) * lamb[e];
    cb += r0.nrm[e] * lamb[e];
    ub[0] += Ueb * M[(3 * e) * fe + n];
    ub[1] += Ueb * M[(3 * e + 1) * fe + n];
    ub[2] += Ueb * M[(3 * e + 2) * fe + n];
  }
  // c = sqrt(gamma p / rho)
  if (cb != 0.0) {
    const double ir2 = rcp_nr(2.0 * q.rho);
    pb += cb * P.gamma * rcp_nr(r0.c) * ir2;
    rb -= cb * r0.c * ir2;
  }
  Wk[W_PRHO * fe + n] += rb;
  Wk[W_PU * fe + n] += ub[0];
  Wk[W_PV * fe + n] += ub[1];
  Wk[W_PW * fe + n] += ub[2];
  Wk[W_PP * fe + n] += pb;
}

// ---------------------------------------------------------------------------
// Pass 2
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool in_b1(const Layout& L, int i, int j, int k) {
  return i >= -1 && i <= L.ni && j >= -1 && j <= L.nj && k >= -1 && k <= L.nk;
}

// Does interior node (i, j, k) have ghost images: a periodic image along an
// axis of period p (x + p in [n, n + 1] or x - p in [-2, -1]), or face ghosts
// (x at an active boundary face of a Dirichlet axis)?
__device__ __forceinline__ bool has_images(const AdjK& A, int i, int j, int k) {
  const int id[3] = {i, j, k}, nn[3] = {A.L.ni, A.L.nj, A.L.nk}, bc[3] = {A.bc0, A.bc1, A.bc2};
  // rings j = 1, 2 are the images of the ghosts across the polar axis
  if (A.axis && (j == 1 || j == 2)) return true;
  for (int d = 0; d < 3; ++d) {
    const int p = A.per[d];
    if (p) {
      if ((id[d] + p >= nn[d] && id[d] + p <= nn[d] + 1) || (id[d] - p <= -1 && id[d] - p >= -2)) return true;
    } else if (bc[d] == 1 || bc[d] == 3) {
      if ((id[d] == 0 && bc[d] == 1 && A.F.type[2 * d] != 0) || (id[d] == nn[d] - 1 && A.F.type[2 * d + 1] != 0))
        return true;
    }
  }
  return false;
}

// Last steps at an interior node whose adjoint q is complete: in the
// Runge-Kutta reverse, fbar[c][k][j] += fw q_c on the source plane (fbar
// non-null, on_f) and, after the last stage, qfin = acc + q (qfin non-null).
__device__ __forceinline__ void finish_node(const Layout& L, long long n, int j, int k, const double q[5],
                                            const double* __restrict__ acc, double* __restrict__ fbar, bool on_f,
                                            double fw, double* __restrict__ qfin, int c0 = 0, int c1 = 5) {
  if (fbar && on_f)
    for (int c = c0; c < c1; ++c) fbar[((long long)c * L.nk + k) * L.nj + j] += fw * q[c];
  if (qfin)
    for (int c = c0; c < c1; ++c) qfin[c * L.fe + n] = acc[c * L.fe + n] + q[c];
}

// Pass 2 runs over B = R_i x R_j x R_k, R_d = [lo_d, hi_d]: the ghost layers
// are included along a periodic axis and on the active faces of a Dirichlet
// axis (frozen Dirichlet ghosts carry no dependence).  An interior node
// writes its gather to qout (and, in the Runge-Kutta reverse, does
// acc += accsrc); a ghost node -- a periodic image or a face ghost of an
// interior node -- writes it to W_GG for pass 3.
__global__ void __launch_bounds__(256) k_adj_gather(AdjK A, const double* __restrict__ Q, double* __restrict__ Wk,
                                                    double* __restrict__ qout, double* __restrict__ acc,
                                                    const double* __restrict__ accsrc, double* __restrict__ fbar,
                                                    int i_f, double fw, double* __restrict__ qfin) {
  const Layout& L = A.L;
  const Phys& P = A.P;
  const long long fe = L.fe;
  const unsigned ri = A.hi[0] - A.lo[0] + 1, rj = A.hi[1] - A.lo[1] + 1, rk = A.hi[2] - A.lo[2] + 1;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ri * rj * rk) return;
  const int i = (int)(t % ri) + A.lo[0];
  const int j = (int)((t / ri) % rj) + A.lo[1];
  const int k = (int)(t / (ri * rj)) + A.lo[2];
  const long long n = L.at(i, j, k);
  const bool b1 = in_b1(L, i, j, k);

  double rb = 0, ub[3] = {0, 0, 0}, pb = 0, Tb = 0;
  double out[5] = {0, 0, 0, 0, 0};
  if (b1) {
    rb = Wk[W_PRHO * fe + n];
    ub[0] = Wk[W_PU * fe + n];
    ub[1] = Wk[W_PV * fe + n];
    ub[2] = Wk[W_PW * fe + n];
    pb = Wk[W_PP * fe + n];
    Tb = Wk[W_PT * fe + n];
    for (int a = 0; a < 4; ++a) out[1 + a] += Wk[(W_QD1 + a) * fe + n];
  }
  // gradient-stencil and sensor weights of the neighbours
  for (int d = 0; d < 3; ++d) {
    const int di = d == 0, dj = d == 1, dk = d == 2;
    const long long s = dstr(L, d);
    const bool lo = in_b1(L, i - di, j - dj, k - dk), hi = in_b1(L, i + di, j + dj, k + dk);
    double phib[4] = {0, 0, 0, 0};
    for (int qq = 0; qq < 4; ++qq) {
      const double* a = Wk + (W_A + 3 * qq + d) * fe;
      phib[qq] = 0.5 * ((lo ? a[n - s] : 0.0) - (hi ? a[n + s] : 0.0));
    }
    ub[0] += phib[0];
    ub[1] += phib[1];
    ub[2] += phib[2];
    Tb += phib[3];
    const double* cp = Wk + (W_CP + d) * fe;
    pb += (lo ? cp[n - s] : 0.0) + (hi ? cp[n + s] : 0.0);
  }
  // primitive adjoint -> conserved variables (nodes without any adjoint skip
  // the map, so unused ghost corners are never read)
  if (rb != 0.0 || ub[0] != 0.0 || ub[1] != 0.0 || ub[2] != 0.0 || pb != 0.0 || Tb != 0.0) {
  const Prim q = prim_at(Q, fe, n, P);
  const double ir = rcp_nr(q.rho);
  pb += Tb * P.inv_R * ir;
  rb -= Tb * q.T * ir;
  out[4] += P.gm1 * pb;
  out[1] -= P.gm1 * q.u * pb;
  out[2] -= P.gm1 * q.v * pb;
  out[3] -= P.gm1 * q.w * pb;
  out[0] += P.gm1 * 0.5 * (q.u * q.u + q.v * q.v + q.w * q.w) * pb;
  out[1] += ub[0] * ir;
  out[2] += ub[1] * ir;
  out[3] += ub[2] * ir;
  out[0] -= (ub[0] * q.u + ub[1] * q.v + ub[2] * q.w) * ir;
  out[0] += rb;
  }
  // dissipation faces whose five-point stencil contains this node:
  //   face a = n-e (node is b):    +(A2 + 3 A4) Dbar
  //   face a = n   (node is a):    -(A2 + 3 A4) Dbar
  //   face a = n-2e (node is b+e): -A4 Dbar
  //   face a = n+e (node is a-e):  +A4 Dbar
  for (int d = 0; d < 3; ++d) {
    const int di = d == 0, dj = d == 1, dk = d == 2;
    const long long s = dstr(L, d);
    const int off[4] = {-1, 0, -2, 1};
    for (int r = 0; r < 4; ++r) {
      const int ai = i + off[r] * di, aj = j + off[r] * dj, ak = k + off[r] * dk;
      if (!face_ok(L, d, ai, aj, ak)) continue;
      const long long an = n + off[r] * s;
      const double A2 = Wk[(W_A2 + d) * fe + an], A4 = Wk[(W_A4 + d) * fe + an];
      double w = r == 0 ? (A2 + 3.0 * A4) : (r == 1 ? -(A2 + 3.0 * A4) : (r == 2 ? -A4 : A4));
      if (A.axis && d == 1 && aj == 0) {
        // the face between the axis and j = 1: d3 = Q(2) - 2 Q(1) + Q(0)
        // (the cross-axis value linearly extrapolated), so the axis node
        // takes -(A2 + A4), node j = 1 takes A2 + 2 A4 and the ghost below
        // the axis nothing
        w = r == 0 ? (A2 + 2.0 * A4) : (r == 1 ? -(A2 + A4) : (r == 2 ? -A4 : 0.0));
      }
      if (w == 0.0) continue;
      // Dbar of the face, stored by the face pass
      for (int c = 0; c < 5; ++c) out[c] += w * Wk[(W_DB + 5 * d + c) * fe + an];
    }
  }
  if (interior(L, i, j, k)) {
    for (int c = 0; c < 5; ++c) qout[c * fe + n] = out[c];
    if (acc)
      for (int c = 0; c < 5; ++c) acc[c * fe + n] += accsrc[c * fe + n];
    // nodes without periodic images are final here; pass 3 finishes the rest
    if (!has_images(A, i, j, k)) finish_node(L, n, j, k, out, acc, fbar, i == i_f, fw, qfin);
  } else {
    for (int c = 0; c < 5; ++c) Wk[(W_GG + c) * fe + n] = out[c];
  }
}

// ---------------------------------------------------------------------------
// Pass 3: add the periodic ghost images' gathers to their interior nodes:
// qout(n) += W_GG over the images of n (at x + n_d for x <= 1 and at x - n_d
// for x >= n_d - 2 along each periodic axis, all combinations, in a fixed
// order).  Only nodes in the band {x <= 1 or x >= n_d - 2} of some periodic
// axis have images; threads enumerate the band as three disjoint slabs
// (band of k; core of k x band of j; core of k and j x band of i; the core
// of an axis is [2, n_d - 2), all of [0, n_d) along a non-periodic axis).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int band_coord(unsigned u, int n) { return n <= 4 ? (int)u : (u < 2 ? (int)u : n - 4 + (int)u); }

__global__ void __launch_bounds__(256) k_adj_fold(AdjK A, const double* __restrict__ Wk, double* __restrict__ qout,
                                                  const double* __restrict__ acc, double* __restrict__ fbar, int i_f,
                                                  double fw, double* __restrict__ qfin) {
  const Layout& L = A.L;
  const int nn[3] = {L.ni, L.nj, L.nk};
  const int bc[3] = {A.bc0, A.bc1, A.bc2};
  unsigned bs[3], cs[3];  // band and core sizes
  int c0[3];              // first core coordinate
  for (int d = 0; d < 3; ++d) {
    if (bc[d] == 0) {
      bs[d] = nn[d] < 4 ? nn[d] : 4;
      cs[d] = nn[d] > 4 ? nn[d] - 4 : 0;
      c0[d] = 2;
    } else {
      bs[d] = 0;
      cs[d] = nn[d];
      c0[d] = 0;
    }
  }
  const unsigned ni = nn[0], nj = nn[1];
  const unsigned S2 = bs[2] * nj * ni, S1 = cs[2] * bs[1] * ni, S0 = cs[2] * cs[1] * bs[0];
  unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S2 + S1 + S0) return;
  int i, j, k;
  if (t < S2) {
    i = (int)(t % ni);
    j = (int)((t / ni) % nj);
    k = band_coord(t / (ni * nj), nn[2]);
  } else if (t < S2 + S1) {
    t -= S2;
    i = (int)(t % ni);
    j = band_coord((t / ni) % bs[1], nn[1]);
    k = c0[2] + (int)(t / (ni * bs[1]));
  } else {
    t -= S2 + S1;
    i = band_coord(t % bs[0], nn[0]);
    j = c0[1] + (int)((t / bs[0]) % cs[1]);
    k = c0[2] + (int)(t / (bs[0] * cs[1]));
  }
  const int id[3] = {i, j, k};
  int cand[3][3], nc[3];
  for (int d = 0; d < 3; ++d) {
    nc[d] = 0;
    cand[d][nc[d]++] = id[d];
    if (bc[d] == 0) {
      if (id[d] + nn[d] <= nn[d] + 1) cand[d][nc[d]++] = id[d] + nn[d];
      if (id[d] - nn[d] >= -2) cand[d][nc[d]++] = id[d] - nn[d];
    }
  }
  const long long n0 = L.at(i, j, k);
  const double* G = Wk + (long long)W_GG * L.fe;
  double q[5];
  for (int c = 0; c < 5; ++c) {
    double s = qout[c * L.fe + n0];
    for (int a = 0; a < nc[0]; ++a)
      for (int b = 0; b < nc[1]; ++b)
        for (int e = 0; e < nc[2]; ++e)
          if (a | b | e) s += G[c * L.fe + L.at(cand[0][a], cand[1][b], cand[2][e])];
    qout[c * L.fe + n0] = s;
    q[c] = s;
  }
  finish_node(L, n0, j, k, q, acc, fbar, i == i_f, fw, qfin);
}

// Pass 3 when an axis is superposed or a boundary face is active: every
// interior node with images adds, in a fixed order, the gathers of its
// periodic images (period p along each periodic axis) and pulls back those
// of its face ghosts through the face rule: qbar(r) += (dG/dq_r)^T Gbar for
// each face ghost G = face_value(q_r) (both layers, and their periodic
// images), the Jacobian column by column from forward-mode dual numbers.
// Ghosts of two Dirichlet directions are frozen and carry nothing.
// Is interior node (i, j, k) the boundary node of an active face (so that
// its face ghosts depend on it through the face rule)?
__device__ __forceinline__ bool at_active_face(const AdjK& A, int i, int j, int k) {
  const int id[3] = {i, j, k}, nn[3] = {A.L.ni, A.L.nj, A.L.nk}, bc[3] = {A.bc0, A.bc1, A.bc2};
  for (int d = 0; d < 3; ++d) {
    if (bc[d] == 1 && id[d] == 0 && A.F.type[2 * d] != 0) return true;
    if ((bc[d] == 1 || bc[d] == 3) && id[d] == nn[d] - 1 && A.F.type[2 * d + 1] != 0) return true;
  }
  return false;
}

// Boundary nodes of the active faces, listed face by face (face f = 2 d +
// hi, the plane id[d] = 0 or n_d - 1 with the other two indices in row
// order); a node on several active faces is listed under the first.
__host__ __device__ inline long long face_plane(const int nn[3], int f) {
  const int d = f / 2;
  return (long long)nn[(d + 1) % 3] * nn[(d + 2) % 3];
}
inline long long face_node_slots(const AdjK& A) {
  const int nn[3] = {A.L.ni, A.L.nj, A.L.nk};
  long long n = 0;
  for (int f = 0; f < 6; ++f)
    if (A.F.type[f] != 0) n += face_plane(nn, f);
  return n;
}
// node of slot x of that list, or false when the slot is a repeat
__device__ inline bool face_node(const AdjK& A, long long x, int id[3]) {
  const int nn[3] = {A.L.ni, A.L.nj, A.L.nk};
  for (int f = 0; f < 6; ++f) {
    if (A.F.type[f] == 0) continue;
    const long long np = face_plane(nn, f);
    if (x >= np) {
      x -= np;
      continue;
    }
    const int d = f / 2, e1 = (d + 1) % 3, e2 = (d + 2) % 3;
    id[d] = (f & 1) ? nn[d] - 1 : 0;
    id[e1] = (int)(x % nn[e1]);
    id[e2] = (int)(x / nn[e1]);
    for (int g = 0; g < f; ++g) {  // listed under an earlier face?
      if (A.F.type[g] == 0) continue;
      const int dg = g / 2;
      if (id[dg] == ((g & 1) ? nn[dg] - 1 : 0)) return false;
    }
    return true;
  }
  return false;
}

// FACES = false: the nodes with images that are not at an active face (no
// face-rule Jacobian, so the kernel stays light), one thread per node;
// FACES = true: the boundary nodes of the active faces, one thread per
// (component, listed node), each taking one column of the face rule's
// Jacobian.  Together they visit each node with images once; each
// component's sum is formed in the same order either way.
template <bool FACES>
__global__ void __launch_bounds__(256) k_adj_fold_general(AdjK A, const double* __restrict__ Q,
                                                          const double* __restrict__ Wk, double* __restrict__ qout,
                                                          const double* __restrict__ acc, double* __restrict__ fbar,
                                                          int i_f, double fw, double* __restrict__ qfin,
                                                          long long slots) {
  const Layout& L = A.L;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int c0 = 0, c1 = 5, i, j, k;
  if (FACES) {
    if (t >= 5 * slots) return;
    c0 = (int)(t / slots);
    c1 = c0 + 1;
    int id3[3];
    if (!face_node(A, t % slots, id3)) return;
    i = id3[0];
    j = id3[1];
    k = id3[2];
  } else {
    const unsigned ni = L.ni, nij = (unsigned)L.ni * L.nj;
    if (t >= (long long)nij * L.nk) return;
    i = (int)(t % ni);
    j = (int)((t % nij) / ni);
    k = (int)(t / nij);
    if (!has_images(A, i, j, k) || at_active_face(A, i, j, k)) return;
  }
  const int id[3] = {i, j, k}, nn[3] = {L.ni, L.nj, L.nk}, bc[3] = {A.bc0, A.bc1, A.bc2};
  int cand[3][3], kind[3][3], nc[3];  // kind: 0 own / periodic image, 1 lo-face ghost, 2 hi-face ghost
  for (int d = 0; d < 3; ++d) {
    nc[d] = 1;
    cand[d][0] = id[d];
    kind[d][0] = 0;
    const int p = A.per[d];
    if (p) {
      if (id[d] + p >= nn[d] && id[d] + p <= nn[d] + 1) {
        cand[d][nc[d]] = id[d] + p;
        kind[d][nc[d]++] = 0;
      }
      if (id[d] - p <= -1 && id[d] - p >= -2) {
        cand[d][nc[d]] = id[d] - p;
        kind[d][nc[d]++] = 0;
      }
    } else if (bc[d] == 1 || bc[d] == 3) {
      if (id[d] == 0 && bc[d] == 1 && A.F.type[2 * d] != 0) {
        cand[d][nc[d]] = -1;
        kind[d][nc[d]++] = 1;
        cand[d][nc[d]] = -2;
        kind[d][nc[d]++] = 1;
      } else if (id[d] == nn[d] - 1 && A.F.type[2 * d + 1] != 0) {
        cand[d][nc[d]] = nn[d];
        kind[d][nc[d]++] = 2;
        cand[d][nc[d]] = nn[d] + 1;
        kind[d][nc[d]++] = 2;
      }
    }
  }
  const long long fe = L.fe, n0 = L.at(i, j, k);
  const double* G = Wk + (long long)W_GG * fe;
  double s[5], qr[5];
  for (int c = c0; c < c1; ++c) s[c] = qout[c * fe + n0];
  if (FACES)
    for (int c = 0; c < 5; ++c) qr[c] = Q[c * fe + n0];
  for (int a = 0; a < nc[0]; ++a)
    for (int b = 0; b < nc[1]; ++b)
      for (int e = 0; e < nc[2]; ++e) {
        if (!(a | b | e)) continue;
        const int kd[3] = {kind[0][a], kind[1][b], kind[2][e]};
        const int nface = (kd[0] != 0) + (kd[1] != 0) + (kd[2] != 0);
        if (nface > 1) continue;  // edge ghost: frozen
        const long long g = L.at(cand[0][a], cand[1][b], cand[2][e]);
        if (nface == 0) {
          for (int c = c0; c < c1; ++c) s[c] += G[c * fe + g];
          continue;
        }
        if (!FACES) continue;  // (not reached: face ghosts exist at active faces only)
        double gb[5];
        for (int c = 0; c < 5; ++c) gb[c] = G[c * fe + g];
        const int d = kd[0] ? 0 : (kd[1] ? 1 : 2), hi = kd[d] == 2;
        const int type = A.F.type[2 * d + hi];
        double nv[3], qo[5] = {0, 0, 0, 0, 0};
        {
          int r[3] = {i, j, k};
          r[d] = hi ? nn[d] - 1 : 0;
          face_normal(L, A.F, d, hi, r[0], r[1], r[2], nv);
        }
        if (A.F.outside)
          for (int c = 0; c < 5; ++c) qo[c] = A.F.outside[c * fe + g];
        for (int c = c0; c < c1; ++c) {  // column c of the face rule's Jacobian
          DualD qd[5], od[5];
          for (int m = 0; m < 5; ++m) qd[m] = DualD(qr[m], m == c ? 1.0 : 0.0);
          face_value<DualD>(type, A.F.gamma, A.F.p_exit[2 * d + hi], nv, qd, qo, od);
          double dot = 0.0;
          for (int m = 0; m < 5; ++m) dot += od[m].d * gb[m];
          s[c] += dot;
        }
      }
  if (A.axis && (j == 1 || j == 2)) {
    // ghosts (i', -j, k') across the polar axis copy node (w(i'), j,
    // (w(k') + (nk - 1)/2) mod (nk - 1)), w wrapping a ghost index (i' a
    // periodic image of i; ghosts of a Dirichlet i side below the axis are
    // edges and keep their values)
    // the ghost azimuths kk in [-2, nk + 1] with ((w(kk) + half) mod p) = k,
    // w(kk) = kk on [0, nk) and (kk + p) mod p outside, in ascending kk:
    // -2, -1, t0, t0 + p (when t0 = 0), nk, nk + 1 with t0 = (k - half) mod p
    const int p = L.nk - 1, half = p / 2;
    const int t0 = ((k - half) % p + p) % p;
    const int kks[6] = {-2, -1, t0, t0 + p, L.nk, L.nk + 1};
    for (int a = 0; a < nc[0]; ++a) {
      if (kind[0][a] != 0) continue;
      for (int q = 0; q < 6; ++q) {
        const int kk = kks[q];
        if (q == 3 && kk >= L.nk) continue;  // t0 + p lies in [0, nk) only for t0 = 0
        const int w2 = (kk >= 0 && kk < L.nk) ? kk : (kk + p) % p;
        if ((w2 + half) % p != k) continue;
        const long long g = L.at(cand[0][a], -j, kk);
        for (int c = c0; c < c1; ++c) s[c] += G[c * fe + g];
      }
    }
  }
  for (int c = c0; c < c1; ++c) qout[c * fe + n0] = s[c];
  finish_node(L, n0, j, k, s, acc, fbar, i == i_f, fw, qfin, c0, c1);
}

// Start of the Runge-Kutta reverse (interior): qcur = Qbar, acc = 0, and
// fbar[c][k][j] += w Qbar_c on the source plane (fbar non-null).
__global__ void __launch_bounds__(256) k_adj_init(Layout L, const double* __restrict__ Qbar, double* __restrict__ qcur,
                                                  double* __restrict__ acc, double* __restrict__ fbar, int i_f,
                                                  double w) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned ni = L.ni, nij = (unsigned)L.ni * L.nj;
  if (t >= nij * (unsigned)L.nk) return;
  const int i = (int)(t % ni);
  const int j = (int)((t % nij) / ni);
  const int k = (int)(t / nij);
  const long long n = L.at(i, j, k);
  for (int c = 0; c < 5; ++c) {
    const double q = Qbar[c * L.fe + n];
    qcur[c * L.fe + n] = q;
    acc[c * L.fe + n] = 0.0;
    if (fbar && i == i_f) fbar[((long long)c * L.nk + k) * L.nj + j] += w * q;
  }
}

// Reverse of the centerline condition, one wave per (i, variable): the
// forward writes the mean of the ring (i, 1, k'), k' = 0 .. nk - 2, to every
// axis node (i, 0, k), k = 0 .. nk - 1; so every ring node receives the sum
// of the axis adjoints over k divided by nk - 1, and the axis adjoints are
// consumed (set to 0).  Lane l sums k = l, l + 64, ... ascending, and the
// partial sums are added by a fixed shuffle tree.
__global__ void __launch_bounds__(64) k_axis_avg_adj(Layout L, double* __restrict__ q) {
  const int f = blockIdx.x / L.ni, i = blockIdx.x % L.ni;
  double* a = q + f * L.fe;
  double sum = 0.0;
  for (int k = threadIdx.x; k < L.nk; k += 64) {
    const long long n = L.at(i, 0, k);
    sum += a[n];
    a[n] = 0.0;
  }
  sum = __shfl(wave_sum(sum), 0, 64);
  const double share = sum / (double)(L.nk - 1);
  for (int k = threadIdx.x; k < L.nk - 1; k += 64) a[L.at(i, 1, k)] += share;
}

// fbar[c][k][j] += w q_c on the source plane i_f (interior nodes).
__global__ void __launch_bounds__(256) k_adj_source(Layout L, const double* __restrict__ q, double* __restrict__ fbar,
                                                    int i_f, double w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.nj * L.nk) return;
  const int j = t % L.nj, k = t / L.nj;
  const long long n = L.at(i_f, j, k);
  for (int c = 0; c < 5; ++c) fbar[((long long)c * L.nk + k) * L.nj + j] += w * q[c * L.fe + n];
}

inline unsigned nb(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// qout = (dR/dQ|Q)^T (coef * qb) on the interior; with acc non-null also
// acc += qb (the gather pass is the last one that reads qb); fbar, qfin: see
// finish_node.
hipError_t residual_vjp(hipStream_t s, const AdjK& A, const double* Q, const double* qb, double coef, double* Wk,
                        double* qout, double* acc = nullptr, double* fbar = nullptr, int i_f = -1, double fw = 0.0,
                        double* qfin = nullptr) {
  const Layout& L = A.L;
  const long long nB1 = (long long)(L.ni + 2) * (L.nj + 2) * (L.nk + 2);
  const long long nFace = (long long)(L.ni + 1) * L.nj * L.nk + (long long)L.ni * (L.nj + 1) * L.nk +
                         (long long)L.ni * L.nj * (L.nk + 1);
  const long long nB = (long long)(A.hi[0] - A.lo[0] + 1) * (A.hi[1] - A.lo[1] + 1) * (A.hi[2] - A.lo[2] + 1);
  const long long nIn = (long long)L.ni * L.nj * L.nk;
  long long nBand = 0;
  {
    const long long nn[3] = {L.ni, L.nj, L.nk};
    const int bc[3] = {A.bc0, A.bc1, A.bc2};
    long long bs[3], cs[3];
    for (int d = 0; d < 3; ++d) {
      bs[d] = bc[d] == 0 ? (nn[d] < 4 ? nn[d] : 4) : 0;
      cs[d] = bc[d] == 0 ? (nn[d] > 4 ? nn[d] - 4 : 0) : nn[d];
    }
    nBand = bs[2] * nn[1] * nn[0] + cs[2] * bs[1] * nn[0] + cs[2] * cs[1] * bs[0];
  }
  k_adj_flux<<<nb(nB1, 256), 256, 0, s>>>(A, Q, qb, coef, Wk);
  k_adj_face<<<nb(nFace, 256), 256, 0, s>>>(A, Q, qb, coef, Wk);
  k_adj_dnode<<<nb(nB1, 256), 256, 0, s>>>(A, Q, Wk);
  k_adj_gather<<<nb(nB, 256), 256, 0, s>>>(A, Q, Wk, qout, acc, qb, fbar, i_f, fw, qfin);
  if (A.general)
  {
    k_adj_fold_general<false><<<nb(nIn, 256), 256, 0, s>>>(A, Q, Wk, qout, acc, fbar, i_f, fw, qfin, 0);
    const long long slots = face_node_slots(A);
    if (slots > 0)
      k_adj_fold_general<true><<<nb(5 * slots, 256), 256, 0, s>>>(A, Q, Wk, qout, acc, fbar, i_f, fw, qfin, slots);
  }
  else if (nBand > 0)
    k_adj_fold<<<nb(nBand, 256), 256, 0, s>>>(A, Wk, qout, acc, fbar, i_f, fw, qfin);
  return hipGetLastError();
}

}  // namespace

size_t adjoint_work_elems(const Layout& L) { return (size_t)W_NF * (size_t)L.fe; }

hipError_t launch_axis_avg_adjoint(hipStream_t s, const Layout& L, double* qbar) {
  k_axis_avg_adj<<<(unsigned)(5LL * L.ni), 64, 0, s>>>(L, qbar);
  return hipGetLastError();
}

hipError_t run_residual_vjp(hipStream_t s, const AdjArgs& a, const double* Q, const double* Rbar, double* Qbar,
                            double* work) {
  const AdjK A = make_adjk(a);
  hipError_t e = residual_vjp(s, A, Q, Rbar, 1.0, work, Qbar);
  // the residual reads the state after the centerline condition
  if (e == hipSuccess && A.axis) e = launch_axis_avg_adjoint(s, a.L, Qbar);
  return e;
}

hipError_t run_adjoint_step(hipStream_t s, const AdjArgs& a, const double* ckpt, double dt, double* Qbar,
                            double* fbar, double* work) {
  const AdjK A = make_adjk(a);
  const Layout& L = a.L;
  const long long fe = L.fe;
  const long long nIn = (long long)L.ni * L.nj * L.nk;
  double* qcur = work + (long long)W_Q1 * fe;
  double* qnext = work + (long long)(W_Q1 + 5) * fe;
  double* acc = work + (long long)W_ACC * fe;
  // With the polar axis every stage input and the step's result pass
  // through the centerline condition C (linear): Q^{n+1} = C(Z_5) and the
  // stage input of stage l > 1 is C(Z_l) for the raw stage output Z_l, so
  // the reverse applies C^T to Qbar first, to each stage's result before it
  // is used, and to the final sum (the step's input was C(Q^n)).  The
  // source-plane update then takes the transformed adjoint, in a pass of its
  // own.
  const bool want_f = fbar && a.i_f >= 0;
  hipError_t e = hipSuccess;
  if (A.axis && (e = launch_axis_avg_adjoint(s, L, Qbar)) != hipSuccess) return e;
  // qcur = Qbar, acc = 0, fbar += alpha_5 dt Qbar (interior)
  k_adj_init<<<nb(nIn, 256), 256, 0, s>>>(L, Qbar, qcur, acc, want_f ? fbar : nullptr, a.i_f, rk_alpha(4) * dt);
  for (int l = 4; l >= 0; --l) {
    const double al = rk_alpha(l) * dt;
    // qbar_{l-1} = (dR/dQ|Q^(l-1))^T (-alpha_l dt qbar_l), acc += qbar_l,
    // fbar += alpha_{l-1} dt qbar_{l-1}; after the last stage Qbar = acc +
    // qbar_0
    const double* Ql = ckpt + (long long)l * 5 * fe;
    const bool f_next = want_f && l > 0;
    const bool f_here = f_next && !A.axis;
    e = residual_vjp(s, A, Ql, qcur, -al, work, qnext, acc, f_here ? fbar : nullptr, a.i_f,
                     f_here ? rk_alpha(l - 1) * dt : 0.0, l == 0 ? Qbar : nullptr);
    if (e != hipSuccess) return e;
    if (A.axis) {
      e = launch_axis_avg_adjoint(s, L, l == 0 ? Qbar : qnext);
      if (e != hipSuccess) return e;
      if (f_next) k_adj_source<<<nb((long long)L.nj * L.nk, 256), 256, 0, s>>>(L, qnext, fbar, a.i_f,
                                                                                rk_alpha(l - 1) * dt);
    }
    double* tmp = qcur;
    qcur = qnext;
    qnext = tmp;
  }
  return hipGetLastError();
}

}  // namespace les
