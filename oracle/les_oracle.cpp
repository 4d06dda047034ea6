// les_oracle.cpp -- plain, slow FP64 CPU oracle of the LES residual and the
// five-stage Runge-Kutta step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no source with the GPU path.
//
// What it computes (paper: "Strong Scaling of Numerical Solver for Supersonic
// Jet Flow Configurations", arXiv 2003.08746):
//   * Sec. 3, Eq. (1)-(15): filtered compressible Navier-Stokes written as
//     dQ/dt = -RHS with Q = [rho, rho u_i, e]; e = p/(gamma-1) + rho u_i u_i/2
//     (Eq. 2); p = rho R T (Eq. 7); Sutherland viscosity (Eq. 6); Fourier heat
//     flux with kappa = mu Cp / Pr (Eq. 3-4) and kappa_sgs = mu_sgs Cp/Pr_sgs
//     (Eq. 5); stress tau_ij = 2(mu+mu_sgs)(S_ij - S_kk delta_ij/3) (Eq. 9-10).
//   * Sec. 3 (end) and Sec. 4: centred finite differences in general
//     curvilinear coordinates, Turkel-Vatsa anisotropic scalar artificial
//     dissipation, Jameson's explicit 5-stage 2nd-order Runge-Kutta scheme.
//   * Sec. 4, Alg. 2: each stage re-evaluates inviscid flux, artificial
//     dissipation, viscous flux and the RHS at every point, then updates the
//     conserved vector with coefficient alpha_l; boundary (ghost) values and
//     the viscosity are refreshed between stages; two ghost layers (Sec. 4,
//     Fig. 3) because the dissipation uses a five-point stencil.
//
// The paper defers the discrete details to other works, so the following
// readings are fixed here (each one marked where it is used):
//   R1  strong-conservation form on a stationary grid, index spacing 1, the
//       state is Q itself and R = J * sum_d d/dxi_d (contravariant flux).
//   R2  metrics by the conservative (Thomas-Lombard) form with the same
//       central difference, J from the central-difference determinant; in a
//       periodic direction the ghost-layer metrics are copies of the interior
//       metrics at the wrapped index.
//   R3  node gradients by central differences + chain rule; node fluxes;
//       face flux = average of the two node fluxes.
//   R4  heat flux enters the energy flux as +(kappa+kappa_sgs) dT/dx_j
//       (physical Fourier conduction; the printed sign is inconsistent).
//   R5  Sutherland: mu = mu_ref (T/T_ref)^(3/2) (1+S)/(T/T_ref+S), S=S1/T_ref.
//   R6  static Smagorinsky eddy viscosity mu_sgs = rho (Cs D)^2 |S|,
//       |S| = sqrt(2 S_ij S_ij), D = (1/J)^(1/3), sigma_kk = 0.
//   R7  Turkel-Vatsa: pressure sensor nu = |p+ - 2p + p-|/(p+ + 2p + p-);
//       eps2 = k2 max(nu_i, nu_i+1); eps4 = max(0, k4 - eps2);
//       lambda_d = |U~_d| + c |grad d / J|;
//       Lambda_d = lambda_d [1 + sum_{e!=d} (lambda_e/lambda_d)^alpha];
//       face Lambda = mean of the node values; D = Lambda (eps2 dQ - eps4 d3Q).
//   R8  RK coefficients alpha = (1/4, 1/6, 3/8, 1/2, 1); the full residual is
//       re-evaluated at every stage.
//   R9  CFL time step: dt = cfl * min 1/(sum_d lam^_d + 2 nu_v sum_d |grad d|^2),
//       lam^_d = |U_d| + c |grad d| with physical metrics,
//       nu_v = max(4/3, gamma/Pr) mu/rho; one global min per step from Q^n.
//   R10 ghost nodes: a node that is a ghost in a Dirichlet direction keeps its
//       given (frozen) value; every other ghost node takes the value of the
//       node whose periodic indices are wrapped into the interior.
//   R11 non-smooth derivatives (dual numbers): d|x|/dx = sign(x), 0 at 0;
//       max(a, b) follows a when a >= b; d sqrt(x)/dx = 0 at x = 0.
//   R12 an optional constant source f on the plane i = i_f: dQ/dt = -R + f.
//   R13, R14, R16 boundary faces of a Dirichlet direction: see fill_faces.
//   R17 dynamic SGS closure (sgs = 2; the paper fixes Pr_sgs = 0.9 only for
//       static closures): the coefficients of mu_sgs = C rho D^2 |S| and
//       kappa_sgs = Cp D_T rho D^2 |S| (D_T = C / Pr_sgs) come from Germano's
//       identity between the grid filter and a test filter of width 2D, in
//       the compressible (Favre) form of Moin, Squires, Cabot and Lee (1991),
//       by Lilly's least squares averaged over the periodic k direction:
//         C(i,j) = max(0, <L^d : M> / <M : M>),  D_T(i,j) = max(0, <K . N> / <N . N>),
//       with <.> the sum over the distinct interior k (nk - 1 of them along a
//       superposed direction, R15) and, at one node (^ = test filter,
//       the index-space tensor product of the weights (1/4, 1/2, 1/4)):
//         L_ij = (rho u_i u_j)^ - (rho u_i)^ (rho u_j)^ / rho^,
//         M_ij = 2 (D^2 rho |S| S^d_ij)^ - 2 (2D)^2 rho^ |S~| S~^d_ij,
//         K_j  = (rho u_j T)^ - (rho u_j)^ (rho T)^ / rho^,
//         N_j  = (D^2 rho |S| dT/dx_j)^ - (2D)^2 rho^ |S~| dT~/dx_j,
//       where S~ and T~ are the strain rate and gradient (central
//       differences, chain rule) of u~ = (rho u)^ / rho^ and T~ = (rho T)^ /
//       rho^, D = (1/J)^(1/3) at the node.  Ghost columns take the wrapped
//       (periodic) or nearest interior (Dirichlet) column's coefficients.
//       Re-evaluated with every residual, as the viscosity is.
//   R18 isotropic part of the SGS stress (Eq. 11), Yoshizawa's model:
//       sigma_kk = 2 CI rho D^2 |S|^2 (sgs >= 1).  By Eq. 1 it acts as an
//       added pressure sigma_kk / 3 in the momentum and energy fluxes.
//   R19 centerline of the O-grid (Sec. 3: a singularity of the coordinate
//       transformation), bc[1] = 3: node j = 0 lies on the polar axis (every
//       k there is the same point); the j-hi side is Dirichlet.  k must be
//       superposed periodic with nk - 1 even.  Ghost (i, -m, k) is the node
//       across the axis, (i, m, k + (nk - 1)/2) (frozen where i is a ghost of
//       a Dirichlet side, like other edges).  The axis nodes are not
//       advanced by the residual (R = 0 there): before every residual
//       evaluation and after every stage update each takes the conserved
//       variables of the adjacent ring j = 1 extrapolated at zero order and
//       averaged over the nk - 1 distinct azimuths.  The metrics give
//       xi/J = eta/J = 0 on the axis, so the eta node flux and the eta
//       spectral radius there are 0 (their limits; J itself is infinite).
//       The fourth difference of the face between the axis and j = 1 takes
//       the cross-axis value by linear extrapolation, Q(-1) = 2 Q(0) - Q(1),
//       i.e. d3 = Q(2) - 2 Q(1) + Q(0), so no five-point stencil reaches
//       across the axis (the pressure sensor, a three-point stencil, keeps
//       its cross-axis neighbour).  The CFL bound skips the axis nodes.
//   R20 the face normal of an entrance, exit or far-field face at an axis
//       node (where the metric row of that direction vanishes): the
//       normalised azimuthal mean of the unit normals of the ring j = 1.
//   R21 the dynamic closure (R17) with the polar axis: an axis node's control
//       volume vanishes (1/J = 0, so D = 0) and its strain is 0/0, so its
//       grid-level products D^2 rho |S| S^d and D^2 rho |S| grad T are 0, the
//       contractions are summed over the off-axis rings only, the axis
//       column takes the ring j = 1's coefficients, and ghost column (i, -m)
//       across the axis takes column (i, m) (its azimuthal sums run over the
//       same points).  (Only the axis nodes' own residual, which is not
//       formed, reads the axis column.)
//   R15 superposed periodic direction (Sec. 3: the first and last azimuthal
//       points coincide): bc = 2, period n - 1; node n - 1 is node 0 again
//       (it takes node 0's metrics), ghosts wrap with period n - 1.  A ghost
//       takes the node reached by wrapping its ghost coordinates only; its
//       interior coordinates are kept (a ghost next to node n - 1 is the
//       image of a node of that plane, not of plane 0).
//
// Data layout (all arrays): padded box [nk+4][nj+4][ni+4], i fastest, two
// ghost layers per side; interior index 0..n-1 is stored at n+2.  Multi-field
// arrays are [field][box].
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -fPIC -shared.
// OpenMP only splits loops whose iterations are independent (pointwise work);
// every reduction is a serial loop.

#include <cmath>
#include <cstdio>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <vector>
#include <algorithm>

// ---------------------------------------------------------------------------
// Scalar types: double, and a forward-mode dual number for exact tangents.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
static inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
static inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
static inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
static inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
static inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
static inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
static inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
static inline Dual operator/(double a, Dual b) { return Dual(a / b.v, -a * b.d / (b.v * b.v)); }

static inline double val(double a) { return a; }
static inline double val(const Dual& a) { return a.v; }

static inline double s_sqrt(double a) { return std::sqrt(a); }
// R11: sqrt has derivative 0 at 0 (the eddy viscosity's |S| at rest).
static inline Dual s_sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0.0 ? a.d / (2.0 * s) : 0.0);
}
static inline double s_pow(double a, double e) { return std::pow(a, e); }
static inline Dual s_pow(Dual a, double e) {
  return Dual(std::pow(a.v, e), e * std::pow(a.v, e - 1.0) * a.d);
}
// R11: d|x|/dx = sign(x), and 0 at x = 0.
static inline double s_abs(double a) { return std::fabs(a); }
static inline Dual s_abs(Dual a) {
  if (a.v > 0.0) return a;
  if (a.v < 0.0) return -a;
  return Dual(0.0, 0.0);
}
// R11: max(a, b) follows a when a >= b.
static inline double s_max(double a, double b) { return a >= b ? a : b; }
static inline Dual s_max(Dual a, Dual b) { return a.v >= b.v ? a : b; }

// ---------------------------------------------------------------------------
// Problem description (mirrored by the Python wrapper with ctypes).
// ---------------------------------------------------------------------------
extern "C" {
typedef struct {
  int ni, nj, nk;  // interior points per direction
  int bc[3];       // per direction i, j, k: 0 = periodic, 1 = frozen Dirichlet ghosts,
                   // 2 = periodic with superposed first and last nodes (R15),
                   // 3 (j only) = polar axis at j = 0, Dirichlet at j-hi (R19)
  // Boundary faces of a Dirichlet direction (R13, R14, R16), in the order i-lo,
  // i-hi, j-lo, j-hi, k-lo, k-hi: 0 = frozen ghosts, 1 = characteristic
  // entrance (R13), 2 = subsonic exit with imposed pressure p_exit (R14),
  // 3 = far field (R16).  outside: padded [5][N] state whose ghost-node
  // values are the outside state of the characteristic and far-field faces
  // (NULL when no face needs it).
  int face[6];
  double p_exit[6];
  const double* outside;
} orc_dims;

typedef struct {
  double gamma;   // ratio of specific heats
  double Pr;      // molecular Prandtl number (Eq. 4)
  double Pr_sgs;  // SGS Prandtl number (Eq. 5)
  double mu_ref;  // Sutherland reference viscosity at T_ref (Eq. 6)
  double T_ref;   // Sutherland reference temperature (nondimensional)
  double S_suth;  // S1 / T_ref (Eq. 6, reading R5)
  double R_gas;   // gas constant (Eq. 7-8)
  int sgs;        // 0: mu_sgs = 0 (the paper's runs), 1: static Smagorinsky (R6),
                  // 2: dynamic closure (R17)
  double Cs;      // Smagorinsky constant
  double k2, k4, alpha;  // Turkel-Vatsa constants (R7)
  double cfl;     // CFL number (R9)
  double CI;      // isotropic SGS constant of the sigma_kk model (R18); 0 = sigma_kk off
} orc_params;
}

namespace {

const int G = 2;  // ghost layers per side

struct Box {
  int ni, nj, nk, bc[3];
  int pi, pj, pk;  // padded extents
  size_t N;        // padded node count
  int face[6];     // boundary-face types (orc_dims.face)
  double p_exit[6];
  const double* outside;
  const double* m = nullptr;  // metrics, for the face normals (set where faces are applied)
  double gamma = 0.0;
  bool axis = false;          // R19: j = 0 is the polar axis
  explicit Box(const orc_dims& d) {
    ni = d.ni; nj = d.nj; nk = d.nk;
    bc[0] = d.bc[0]; bc[1] = d.bc[1]; bc[2] = d.bc[2];
    pi = ni + 2 * G; pj = nj + 2 * G; pk = nk + 2 * G;
    N = (size_t)pi * pj * pk;
    for (int f = 0; f < 6; ++f) {
      face[f] = d.face[f];
      p_exit[f] = d.p_exit[f];
    }
    outside = d.outside;
    axis = bc[1] == 3;
    if (bc[0] == 3 || bc[2] == 3 || (axis && (bc[2] != 2 || (nk - 1) % 2 != 0))) {
      std::fprintf(stderr, "oracle: the axis (bc 3) is for j only, with k superposed periodic and nk - 1 even\n");
      std::abort();
    }
  }
  // ghost index x along d lies on a Dirichlet side (frozen, or a face rule)
  bool dirichlet_side(int d, int x) const { return bc[d] == 1 || (bc[d] == 3 && x >= n(d)); }
  bool any_face() const {
    for (int f = 0; f < 6; ++f)
      if (face[f] != 0) return true;
    return false;
  }
  // index of node (i, j, k) with interior range 0..n-1 and ghosts -2, -1, n, n+1
  size_t at(int i, int j, int k) const {
    return ((size_t)(k + G) * pj + (size_t)(j + G)) * pi + (size_t)(i + G);
  }
  int n(int d) const { return d == 0 ? ni : (d == 1 ? nj : nk); }
};

// offset of the unit step in direction d
static inline void step(int d, int& di, int& dj, int& dk) {
  di = (d == 0); dj = (d == 1); dk = (d == 2);
}

// Interior index of a periodic image: period n, or n - 1 when the first and
// last nodes are superposed (R15).
static inline int wrap(int x, int n, int bc) {
  const int p = bc == 2 ? n - 1 : n;
  return ((x % p) + p) % p;
}

// ---------------------------------------------------------------------------
// R13, R14, R16: boundary faces of a Dirichlet direction (Sec. 3: entrance, far
// field and exit conditions).  A ghost node that lies outside the interior
// along exactly one Dirichlet direction d, on a face of type 1, 2 or 3, takes a
// state built from the boundary node r (the interior node next to the face
// on the same line along d, periodic indices wrapped: zero-order
// extrapolation for both ghost layers) and, for types 1 and 3, the outside
// state at the ghost node.  Edge and corner ghosts of two Dirichlet directions stay
// frozen.
//   R14 exit (subsonic, imposed pressure): velocity and internal energy per
//       unit mass eps = p / ((gamma - 1) rho) from r, p = p_exit, hence
//       rho = p_exit / ((gamma - 1) eps) and e from Eq. 2.
//   R13 characteristic (entrance, locally one-dimensional along
//       the outward unit normal n = -+grad(xi_d) / |grad(xi_d)| at r):
//       supersonic outflow (u.n >= c at r): the state of r;
//       supersonic inflow (u.n <= -c outside): the outside state;
//       otherwise R+ = u.n + 2c/(gamma-1) from r, R- = u.n - 2c/(gamma-1)
//       from outside, u.n = (R+ + R-)/2, c = (gamma-1)(R+ - R-)/4, entropy
//       p/rho^gamma and the tangential velocity from r when u.n >= 0, else
//       from outside; rho = (c^2/(gamma s))^(1/(gamma-1)), p = rho c^2/gamma.
//       This rule serves the entrance (the flat-hat profile is the outside
//       state).
//   R16 far field (Sec. 3: Riemann invariants, normal velocity extrapolated
//       at zero order from inside, flow angle fixed, the rest from the jet
//       Mach number through the outside state): u.n = u_r.n; tangential
//       velocity = the outside state's (its direction, the flow angle, does
//       not follow the interior); the incoming invariant
//       R- = u_o.n - 2c_o/(gamma-1) of the outside state is kept, so
//       c = (gamma-1)(u.n - R-)/2; entropy p/rho^gamma from outside when
//       u.n < 0 (inflow), from r otherwise; rho and p from c and entropy.
//       The outside state carries the jet-Mach-number-dependent far-field
//       values (ambient density and pressure, co-flow velocity).
// ---------------------------------------------------------------------------
template <class S>
void face_state(int type, double gamma, double p_exit, const double nrm[3], const S qr[5], const double qo[5],
                S out[5]) {
  const double gm1 = gamma - 1.0;
  const S rho = qr[0];
  const S u[3] = {qr[1] / rho, qr[2] / rho, qr[3] / rho};
  const S uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const S p = gm1 * (qr[4] - 0.5 * rho * uu);
  if (type == 2) {
    const S rg = rho * p_exit / p;
    out[0] = rg;
    for (int a = 0; a < 3; ++a) out[1 + a] = rg * u[a];
    out[4] = p_exit / gm1 + 0.5 * rg * uu;
    return;
  }
  const double ro = qo[0];
  const double uo[3] = {qo[1] / ro, qo[2] / ro, qo[3] / ro};
  const double po = gm1 * (qo[4] - 0.5 * ro * (uo[0] * uo[0] + uo[1] * uo[1] + uo[2] * uo[2]));
  const S cr = s_sqrt(gamma * p / rho);
  const double co = std::sqrt(gamma * po / ro);
  const S unr = u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2];
  const double uno = uo[0] * nrm[0] + uo[1] * nrm[1] + uo[2] * nrm[2];
  if (type == 3) {
    // R16 far field, in the order of the Sec. 3 sentence: normal velocity
    // from r (zero order); tangential velocity of the outside state (the
    // fixed flow angle); the incoming Riemann invariant of the outside
    // state at that normal velocity gives c; entropy from outside on
    // inflow (u.n < 0), from r otherwise.
    const S un = unr;
    const double Rm = uno - 2.0 * co / gm1;
    const S cb = 0.5 * gm1 * (un - Rm);
    const S ent = val(un) >= 0.0 ? p / s_pow(rho, gamma) : S(po / std::pow(ro, gamma));
    const S rb = s_pow(cb * cb / (gamma * ent), 1.0 / gm1);
    const S pb = rb * cb * cb / gamma;
    S ubb = S(0.0);
    out[0] = rb;
    for (int a = 0; a < 3; ++a) {
      const S ub = (uo[a] - uno * nrm[a]) + un * nrm[a];
      out[1 + a] = rb * ub;
      ubb = ubb + ub * ub;
    }
    out[4] = pb / gm1 + 0.5 * rb * ubb;
    return;
  }
  if (val(unr) >= val(cr)) {
    for (int c = 0; c < 5; ++c) out[c] = qr[c];
    return;
  }
  if (uno <= -co) {
    for (int c = 0; c < 5; ++c) out[c] = S(qo[c]);
    return;
  }
  const S Rp = unr + 2.0 * cr / gm1;
  const S Rm = S(uno - 2.0 * co / gm1);
  const S un = 0.5 * (Rp + Rm);
  const S cb = 0.25 * gm1 * (Rp - Rm);
  S ent, ut[3];
  if (val(un) >= 0.0) {
    ent = p / s_pow(rho, gamma);
    for (int a = 0; a < 3; ++a) ut[a] = u[a] - unr * nrm[a];
  } else {
    ent = S(po / std::pow(ro, gamma));
    for (int a = 0; a < 3; ++a) ut[a] = S(uo[a] - uno * nrm[a]);
  }
  const S rb = s_pow(cb * cb / (gamma * ent), 1.0 / gm1);
  const S pb = rb * cb * cb / gamma;
  S ub[3], ubb = S(0.0);
  for (int a = 0; a < 3; ++a) {
    ub[a] = ut[a] + un * nrm[a];
    ubb = ubb + ub[a] * ub[a];
  }
  out[0] = rb;
  for (int a = 0; a < 3; ++a) out[1 + a] = rb * ub[a];
  out[4] = pb / gm1 + 0.5 * rb * ubb;
}

template <class S>
void fill_faces(const Box& b, S* a) {
  if (!b.m) {
    std::fprintf(stderr, "oracle: boundary faces need the metrics (call through an entry point that has them)\n");
    std::abort();
  }
  for (int k = -G; k < b.nk + G; ++k)
    for (int j = -G; j < b.nj + G; ++j)
      for (int i = -G; i < b.ni + G; ++i) {
        const int idx[3] = {i, j, k};
        if (b.axis && j < 0) continue;  // across the axis: filled from its image (R19)
        int nd = 0, d = -1, w[3];
        for (int e = 0; e < 3; ++e) {
          const int n = b.n(e);
          const bool g = idx[e] < 0 || idx[e] >= n;
          if (g && b.dirichlet_side(e, idx[e])) {
            ++nd;
            d = e;
          }
          w[e] = g ? wrap(idx[e], n, b.bc[e]) : idx[e];  // R15: only ghost coordinates wrap
        }
        if (nd != 1) continue;
        const int hi = idx[d] >= b.n(d) ? 1 : 0;
        const int f = 2 * d + hi;
        if (b.face[f] == 0) continue;
        w[d] = hi ? b.n(d) - 1 : 0;  // boundary node r
        const size_t r = b.at(w[0], w[1], w[2]), g = b.at(i, j, k);
        // outward unit normal from grad(xi_d) = J (xi_d/J)_x,y,z at r
        double nrm[3], nn = 0.0;
        if (b.axis && w[1] == 0 && d != 1) {
          // R20: at a node on the polar axis every azimuth meets and the
          // metric row vanishes; the normal is the mean over the ring j = 1
          // (k' = 0 .. nk - 2) of its unit normals, normalised
          double sum[3] = {0.0, 0.0, 0.0};
          for (int kk = 0; kk < b.nk - 1; ++kk) {
            int rw[3] = {w[0], 1, kk};
            rw[d] = hi ? b.n(d) - 1 : 0;
            const size_t rr = b.at(rw[0], rw[1], rw[2]);
            const double Jr = b.m[9 * b.N + rr];
            double u[3], un = 0.0;
            for (int x = 0; x < 3; ++x) {
              u[x] = Jr * b.m[(size_t)(3 * d + x) * b.N + rr];
              un += u[x] * u[x];
            }
            un = std::sqrt(un);
            for (int x = 0; x < 3; ++x) sum[x] += u[x] / un;
          }
          for (int x = 0; x < 3; ++x) {
            nrm[x] = sum[x];
            nn += nrm[x] * nrm[x];
          }
        } else {
          const double J = b.m[9 * b.N + r];
          for (int x = 0; x < 3; ++x) {
            nrm[x] = J * b.m[(size_t)(3 * d + x) * b.N + r];
            nn += nrm[x] * nrm[x];
          }
        }
        nn = std::sqrt(nn);
        for (int x = 0; x < 3; ++x) nrm[x] = (hi ? 1.0 : -1.0) * nrm[x] / nn;
        S qr[5], out[5];
        double qo[5] = {0, 0, 0, 0, 0};
        for (int c = 0; c < 5; ++c) {
          qr[c] = a[(size_t)c * b.N + r];
          if (b.outside) qo[c] = b.outside[(size_t)c * b.N + g];
        }
        face_state(b.face[f], b.gamma, b.p_exit[f], nrm, qr, qo, out);
        for (int c = 0; c < 5; ++c) a[(size_t)c * b.N + g] = out[c];
      }
}

// ---------------------------------------------------------------------------
// R10: ghost fill.
// ---------------------------------------------------------------------------
template <class S>
void fill_ghosts(const Box& b, S* a, int nfields) {
  for (int f = 0; f < nfields; ++f) {
    S* q = a + (size_t)f * b.N;
    for (int k = -G; k < b.nk + G; ++k)
      for (int j = -G; j < b.nj + G; ++j)
        for (int i = -G; i < b.ni + G; ++i) {
          int idx[3] = {i, j, k};
          bool ghost = false, dirichlet = false;
          int w[3];
          for (int d = 0; d < 3; ++d) {
            int n = b.n(d);
            bool g = idx[d] < 0 || idx[d] >= n;
            if (g) {
              ghost = true;
              if (b.dirichlet_side(d, idx[d])) dirichlet = true;
            }
            w[d] = g ? wrap(idx[d], n, b.bc[d]) : idx[d];  // R15: only ghost coordinates wrap
          }
          if (!ghost || dirichlet || (b.axis && j < 0)) continue;
          q[b.at(i, j, k)] = q[b.at(w[0], w[1], w[2])];
        }
  }
  if (nfields == 5 && b.any_face()) fill_faces(b, a);
  // R19: a ghost across the axis is the node diametrically opposite (one that
  // is also a ghost of a Dirichlet i side keeps its given value, like the
  // other edges of two boundary directions)
  if (b.axis) {
    const int half = (b.nk - 1) / 2;
    for (int f = 0; f < nfields; ++f) {
      S* q = a + (size_t)f * b.N;
      for (int k = -G; k < b.nk + G; ++k)
        for (int j = -G; j < 0; ++j)
          for (int i = -G; i < b.ni + G; ++i) {
            if ((i < 0 || i >= b.ni) && b.bc[0] == 1) continue;
            q[b.at(i, j, k)] = q[b.at(i, -j, wrap(k + half, b.nk, 2))];
          }
    }
  }
}

// R19: centerline condition on the axis nodes of the interior columns: the
// azimuthal mean of the adjacent ring j = 1 (zero-order extrapolation, then
// the average over the nk - 1 distinct azimuths), for every k.
template <class S>
void apply_axis(const Box& b, S* a) {
  if (!b.axis) return;
  for (int f = 0; f < 5; ++f) {
    S* q = a + (size_t)f * b.N;
    for (int i = 0; i < b.ni; ++i) {
      S sum = 0.0;
      for (int k = 0; k < b.nk - 1; ++k) sum = sum + q[b.at(i, 1, k)];
      const S mean = sum / double(b.nk - 1);
      for (int k = 0; k < b.nk; ++k) q[b.at(i, 0, k)] = mean;
    }
  }
}

// ---------------------------------------------------------------------------
// R2: metrics.  m[0..8] = xi_x/J, xi_y/J, xi_z/J, eta_x/J, ..., zeta_z/J;
// m[9] = J.  Defined on every node with all indices in [-1, n]; NaN elsewhere.
// ---------------------------------------------------------------------------
void metrics(const Box& b, const double* xyz, double* m) {
  const double* X[3] = {xyz, xyz + b.N, xyz + 2 * b.N};
  const double nan = std::nan("");
  for (int c = 0; c < 10; ++c)
    for (size_t n = 0; n < b.N; ++n) m[(size_t)c * b.N + n] = nan;

  // first derivatives of the coordinates, dX[c][d] = delta_d x_c, on [-2+1, n+1-1]
  // along d and on the full padded range in the other directions.
  std::vector<double> dX(9 * b.N, nan);
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) {
      int di, dj, dk;
      step(d, di, dj, dk);
      double* out = &dX[(size_t)(3 * c + d) * b.N];
      for (int k = -G; k < b.nk + G; ++k)
        for (int j = -G; j < b.nj + G; ++j)
          for (int i = -G; i < b.ni + G; ++i) {
            int id[3] = {i, j, k};
            if (id[d] - 1 < -G || id[d] + 1 >= b.n(d) + G) continue;
            out[b.at(i, j, k)] =
                0.5 * (X[c][b.at(i + di, j + dj, k + dk)] - X[c][b.at(i - di, j - dj, k - dk)]);
          }
    }
  auto dx = [&](int c, int d, int i, int j, int k) { return dX[(size_t)(3 * c + d) * b.N + b.at(i, j, k)]; };

  // Conservative form: the metric row of direction a (cyclic a, b=a+1, c=a+2)
  // component x_l (with cyclic l, l+1, l+2 as x, y, z):
  //   (a_{x_l}) / J = delta_c[(delta_b y_{l+1}) y_{l+2}] - delta_b[(delta_c y_{l+1}) y_{l+2}]
  // e.g. xi_x/J = delta_zeta[(delta_eta y) z] - delta_eta[(delta_zeta y) z].
  for (int a = 0; a < 3; ++a) {
    int bd = (a + 1) % 3, cd = (a + 2) % 3;
    int bi, bj, bk, ci, cj, ck;
    step(bd, bi, bj, bk);
    step(cd, ci, cj, ck);
    for (int l = 0; l < 3; ++l) {
      int l1 = (l + 1) % 3, l2 = (l + 2) % 3;
      double* out = m + (size_t)(3 * a + l) * b.N;
      for (int k = -1; k <= b.nk; ++k)
        for (int j = -1; j <= b.nj; ++j)
          for (int i = -1; i <= b.ni; ++i) {
            // delta_c [ (delta_b x_l1) x_l2 ]
            double t1 = 0.5 * (dx(l1, bd, i + ci, j + cj, k + ck) * X[l2][b.at(i + ci, j + cj, k + ck)] -
                               dx(l1, bd, i - ci, j - cj, k - ck) * X[l2][b.at(i - ci, j - cj, k - ck)]);
            // delta_b [ (delta_c x_l1) x_l2 ]
            double t2 = 0.5 * (dx(l1, cd, i + bi, j + bj, k + bk) * X[l2][b.at(i + bi, j + bj, k + bk)] -
                               dx(l1, cd, i - bi, j - bj, k - bk) * X[l2][b.at(i - bi, j - bj, k - bk)]);
            out[b.at(i, j, k)] = t1 - t2;
          }
    }
  }
  // 1/J = det d(x,y,z)/d(xi,eta,zeta) with central differences; J = 1/(1/J).
  double* Jout = m + (size_t)9 * b.N;
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        double a11 = dx(0, 0, i, j, k), a12 = dx(0, 1, i, j, k), a13 = dx(0, 2, i, j, k);
        double a21 = dx(1, 0, i, j, k), a22 = dx(1, 1, i, j, k), a23 = dx(1, 2, i, j, k);
        double a31 = dx(2, 0, i, j, k), a32 = dx(2, 1, i, j, k), a33 = dx(2, 2, i, j, k);
        double vol = a11 * (a22 * a33 - a23 * a32) - a12 * (a21 * a33 - a23 * a31) + a13 * (a21 * a32 - a22 * a31);
        Jout[b.at(i, j, k)] = 1.0 / vol;
      }
  // R2: periodic directions take wrapped interior metrics in their ghost
  // layer; R15: along a superposed direction node n - 1 takes node 0's.
  for (int c = 0; c < 10; ++c) {
    double* q = m + (size_t)c * b.N;
    for (int k = -1; k <= b.nk; ++k)
      for (int j = -1; j <= b.nj; ++j)
        for (int i = -1; i <= b.ni; ++i) {
          int id[3] = {i, j, k}, w[3];
          bool any = false;
          for (int d = 0; d < 3; ++d) {
            int n = b.n(d);
            w[d] = id[d];
            const int top = b.bc[d] == 2 ? n - 1 : n;  // first index that is an image
            if (b.bc[d] != 1 && b.bc[d] != 3 && (id[d] < 0 || id[d] >= top)) {
              w[d] = wrap(id[d], n, b.bc[d]);
              any = true;
            }
          }
          if (any) q[b.at(i, j, k)] = q[b.at(w[0], w[1], w[2])];
        }
  }
}

// ---------------------------------------------------------------------------
// R17: dynamic coefficients C(i,j), D_T(i,j) on every padded column
// (index (j + G) * pi + (i + G)), from Q with its ghosts filled.
// ---------------------------------------------------------------------------
template <class S>
void dynamic_coefficients(const Box& b, const orc_params& P, const double* m, const S* Q, std::vector<S>& Cc,
                          std::vector<S>& Dc) {
  const size_t N = b.N;
  const double g = P.gamma;
  const S* Qv[5] = {Q, Q + N, Q + 2 * N, Q + 3 * N, Q + 4 * N};
  const double* M[10];
  for (int c = 0; c < 10; ++c) M[c] = m + (size_t)c * N;
  // primitives on the padded box
  std::vector<S> u(3 * N), T(N);
  for (size_t n = 0; n < N; ++n) {
    for (int a = 0; a < 3; ++a) u[(size_t)a * N + n] = Qv[1 + a][n] / Qv[0][n];
    S uu = u[n] * u[n] + u[N + n] * u[N + n] + u[2 * N + n] * u[2 * N + n];
    S p = (g - 1.0) * (Qv[4][n] - 0.5 * Qv[0][n] * uu);
    T[n] = p / (Qv[0][n] * P.R_gas);
  }
  // gradient (central differences, chain rule) of field F at node (i,j,k)
  auto gradient = [&](const S* F, int i, int j, int k, S out[3]) {
    const size_t n = b.at(i, j, k);
    const double Jn = M[9][n];
    S dxi = 0.5 * (F[b.at(i + 1, j, k)] - F[b.at(i - 1, j, k)]);
    S deta = 0.5 * (F[b.at(i, j + 1, k)] - F[b.at(i, j - 1, k)]);
    S dzeta = 0.5 * (F[b.at(i, j, k + 1)] - F[b.at(i, j, k - 1)]);
    for (int x = 0; x < 3; ++x) out[x] = Jn * (M[0 + x][n] * dxi + M[3 + x][n] * deta + M[6 + x][n] * dzeta);
  };
  // strain rate, its deviatoric part and |S| = sqrt(2 S:S) from the
  // velocity gradient du[a][x]
  auto strain = [&](S du[3][3], S Sd[3][3], S& mag) {
    S Sij[3][3], SS = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int x = 0; x < 3; ++x) {
        Sij[a][x] = 0.5 * (du[a][x] + du[x][a]);
        SS = SS + Sij[a][x] * Sij[a][x];
      }
    S tr = (Sij[0][0] + Sij[1][1] + Sij[2][2]) / 3.0;
    for (int a = 0; a < 3; ++a)
      for (int x = 0; x < 3; ++x) Sd[a][x] = Sij[a][x] - (a == x ? tr : S(0.0));
    mag = s_sqrt(2.0 * SS);
  };
  // grid-level fields: F0 = rho, F1..3 = rho u_a, F4 = rho T, F5..10 = rho u_i u_j
  // (i <= j), F11..13 = rho u_j T (whole box); F14..19 = D^2 rho |S| S^d_ij
  // (i <= j), F20..22 = D^2 rho |S| dT/dx_j (on [-1, n]^3)
  const int NF = 23;
  const int pair[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
  std::vector<S> F((size_t)NF * N, S(0.0));
  for (size_t n = 0; n < N; ++n) {
    const S r = Qv[0][n];
    F[n] = r;
    for (int a = 0; a < 3; ++a) F[(size_t)(1 + a) * N + n] = Qv[1 + a][n];
    F[4 * N + n] = r * T[n];
    for (int q = 0; q < 6; ++q) F[(size_t)(5 + q) * N + n] = r * u[(size_t)pair[q][0] * N + n] * u[(size_t)pair[q][1] * N + n];
    for (int a = 0; a < 3; ++a) F[(size_t)(11 + a) * N + n] = r * u[(size_t)a * N + n] * T[n];
  }
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        // R21: on the polar axis the node's control volume vanishes (1/J = 0,
        // so D = 0) and its strain is 0/0: the products are 0 there
        if (b.axis && j == 0) continue;
        const size_t n = b.at(i, j, k);
        S du[3][3], dT[3], Sd[3][3], mag;
        for (int a = 0; a < 3; ++a) gradient(&u[(size_t)a * N], i, j, k, du[a]);
        gradient(T.data(), i, j, k, dT);
        strain(du, Sd, mag);
        const double D2 = std::pow(std::cbrt(1.0 / M[9][n]), 2);
        const S w = D2 * Qv[0][n] * mag;
        for (int q = 0; q < 6; ++q) F[(size_t)(14 + q) * N + n] = w * Sd[pair[q][0]][pair[q][1]];
        for (int a = 0; a < 3; ++a) F[(size_t)(20 + a) * N + n] = w * dT[a];
      }
  // test filter at node (i,j,k): weights (1/4, 1/2, 1/4) along each index
  const double wt[3] = {0.25, 0.5, 0.25};
  auto filt = [&](int f, int i, int j, int k) {
    S acc = 0.0;
    for (int c = -1; c <= 1; ++c)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a)
          acc = acc + (wt[a + 1] * wt[bb + 1] * wt[c + 1]) * F[(size_t)f * N + b.at(i + a, j + bb, k + c)];
    return acc;
  };
  // test-filtered velocity and temperature on [-1, n]^3
  std::vector<S> ut(3 * N, S(0.0)), Tt(N, S(0.0));
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        const size_t n = b.at(i, j, k);
        const S rh = filt(0, i, j, k);
        for (int a = 0; a < 3; ++a) ut[(size_t)a * N + n] = filt(1 + a, i, j, k) / rh;
        Tt[n] = filt(4, i, j, k) / rh;
      }
  // per-column sums over the distinct interior k (ascending; a superposed k
  // direction's last plane is its first one's place) of L^d:M, M:M, K.N,
  // N.N; none on the polar axis (R21)
  const size_t cols = (size_t)b.pj * b.pi;
  const int nks = b.bc[2] == 2 ? b.nk - 1 : b.nk;
  std::vector<S> nC(cols, S(0.0)), dC(cols, S(0.0)), nD(cols, S(0.0)), dD(cols, S(0.0));
  for (int j = b.axis ? 1 : 0; j < b.nj; ++j)
    for (int i = 0; i < b.ni; ++i) {
      const size_t col = (size_t)(j + G) * b.pi + (size_t)(i + G);
      for (int k = 0; k < nks; ++k) {
        const size_t n = b.at(i, j, k);
        S fv[NF];
        for (int f = 0; f < NF; ++f) fv[f] = filt(f, i, j, k);
        S du[3][3], dT[3], Sd[3][3], mag;
        for (int a = 0; a < 3; ++a) gradient(&ut[(size_t)a * N], i, j, k, du[a]);
        gradient(Tt.data(), i, j, k, dT);
        strain(du, Sd, mag);
        const double Dt2 = 4.0 * std::pow(std::cbrt(1.0 / M[9][n]), 2);  // (2 D)^2
        S L[3][3], Mm[3][3];
        for (int q = 0; q < 6; ++q) {
          const int a = pair[q][0], c = pair[q][1];
          L[a][c] = L[c][a] = fv[5 + q] - fv[1 + a] * fv[1 + c] / fv[0];
          Mm[a][c] = Mm[c][a] = 2.0 * fv[14 + q] - 2.0 * Dt2 * fv[0] * mag * Sd[a][c];
        }
        const S tr = (L[0][0] + L[1][1] + L[2][2]) / 3.0;
        for (int a = 0; a < 3; ++a) L[a][a] = L[a][a] - tr;
        S lm = 0.0, mm = 0.0, kn = 0.0, nn = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) {
            lm = lm + L[a][c] * Mm[a][c];
            mm = mm + Mm[a][c] * Mm[a][c];
          }
        for (int a = 0; a < 3; ++a) {
          const S K = fv[11 + a] - fv[1 + a] * fv[4] / fv[0];
          const S Nj = fv[20 + a] - Dt2 * fv[0] * mag * dT[a];
          kn = kn + K * Nj;
          nn = nn + Nj * Nj;
        }
        nC[col] = nC[col] + lm;
        dC[col] = dC[col] + mm;
        nD[col] = nD[col] + kn;
        dD[col] = dD[col] + nn;
      }
    }
  Cc.assign(cols, S(0.0));
  Dc.assign(cols, S(0.0));
  for (int j = -G; j < b.nj + G; ++j)
    for (int i = -G; i < b.ni + G; ++i) {
      // ghost columns: wrapped (periodic) or nearest interior (Dirichlet)
      // column; across the polar axis column (i, -m) is the ring column
      // (i, m) (its azimuthal sums run over the same points), and the axis
      // column takes the ring j = 1's coefficients (R21)
      int ii = i, jj = j;
      if (i < 0 || i >= b.ni) ii = b.bc[0] == 1 ? std::min(std::max(i, 0), b.ni - 1) : wrap(i, b.ni, b.bc[0]);
      if (b.axis) {
        jj = j < 0 ? -j : std::min(j, b.nj - 1);
        if (jj == 0) jj = 1;
      } else if (j < 0 || j >= b.nj) {
        jj = b.bc[1] == 1 ? std::min(std::max(j, 0), b.nj - 1) : wrap(j, b.nj, b.bc[1]);
      }
      const size_t src = (size_t)(jj + G) * b.pi + (size_t)(ii + G), dst = (size_t)(j + G) * b.pi + (size_t)(i + G);
      Cc[dst] = val(dC[src]) > 0.0 ? s_max(S(0.0), nC[src] / dC[src]) : S(0.0);
      Dc[dst] = val(dD[src]) > 0.0 ? s_max(S(0.0), nD[src] / dD[src]) : S(0.0);
    }
}

// ---------------------------------------------------------------------------
// Residual R(Q) at interior nodes (R1-R7, R12).  Q must have its ghosts
// filled.  Everything is computed on the box B1 = [-1, n]^3 with separate
// arrays for every intermediate.
// ---------------------------------------------------------------------------
template <class S>
void residual(const Box& b, const orc_params& P, const double* m, const S* Q, const S* f, int i_f, S* R) {
  const size_t N = b.N;
  const double g = P.gamma;
  const double Cp = g * P.R_gas / (g - 1.0);
  const S* Qv[5] = {Q, Q + N, Q + 2 * N, Q + 3 * N, Q + 4 * N};
  const double* M[10];
  for (int c = 0; c < 10; ++c) M[c] = m + (size_t)c * N;

  // --- node primitives on the full padded box (Eq. 2, 6, 7) ---
  std::vector<S> rho(N), u(N), v(N), w(N), p(N), T(N), c(N), mu(N);
#pragma omp parallel for
  for (int k = -G; k < b.nk + G; ++k)
    for (int j = -G; j < b.nj + G; ++j)
      for (int i = -G; i < b.ni + G; ++i) {
        size_t n = b.at(i, j, k);
        rho[n] = Qv[0][n];
        u[n] = Qv[1][n] / rho[n];
        v[n] = Qv[2][n] / rho[n];
        w[n] = Qv[3][n] / rho[n];
        p[n] = (g - 1.0) * (Qv[4][n] - 0.5 * rho[n] * (u[n] * u[n] + v[n] * v[n] + w[n] * w[n]));
        T[n] = p[n] / (rho[n] * P.R_gas);
        c[n] = s_sqrt(g * p[n] / rho[n]);
        S th = T[n] / P.T_ref;
        mu[n] = P.mu_ref * s_pow(th, 1.5) * (1.0 + P.S_suth) / (th + P.S_suth);
      }

  // --- node gradients of u, v, w, T on B1 (R3): grad[q][x] ---
  // q = 0..3 for u, v, w, T;  x = 0..2 for d/dx, d/dy, d/dz.
  std::vector<S> grad(12 * N);
  const std::vector<S>* phi[4] = {&u, &v, &w, &T};
#pragma omp parallel for
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        size_t n = b.at(i, j, k);
        double Jn = M[9][n];
        for (int q = 0; q < 4; ++q) {
          const std::vector<S>& F = *phi[q];
          S dxi = 0.5 * (F[b.at(i + 1, j, k)] - F[b.at(i - 1, j, k)]);
          S deta = 0.5 * (F[b.at(i, j + 1, k)] - F[b.at(i, j - 1, k)]);
          S dzeta = 0.5 * (F[b.at(i, j, k + 1)] - F[b.at(i, j, k - 1)]);
          for (int x = 0; x < 3; ++x)
            grad[(size_t)(3 * q + x) * N + n] = Jn * (M[0 + x][n] * dxi + M[3 + x][n] * deta + M[6 + x][n] * dzeta);
        }
      }

  // --- stress, SGS viscosity and the energy-flux vector Theta on B1 ---
  // tau[3*a+b] (symmetric), Theta[x] = u_i tau_ix + (kappa + kappa_sgs) dT/dx,
  // pis = sigma_kk / 3 (R18)
  std::vector<S> Cdyn, Ddyn;
  if (P.sgs == 2) dynamic_coefficients(b, P, m, Q, Cdyn, Ddyn);
  std::vector<S> tau(9 * N), Theta(3 * N), pis(N, S(0.0));
#pragma omp parallel for
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        size_t n = b.at(i, j, k);
        S du[3][3];  // du[a][x] = d u_a / d x
        for (int a = 0; a < 3; ++a)
          for (int x = 0; x < 3; ++x) du[a][x] = grad[(size_t)(3 * a + x) * N + n];
        S Sij[3][3];
        for (int a = 0; a < 3; ++a)
          for (int x = 0; x < 3; ++x) Sij[a][x] = 0.5 * (du[a][x] + du[x][a]);
        S Skk = Sij[0][0] + Sij[1][1] + Sij[2][2];
        S mu_sgs = 0.0, kap_sgs = 0.0;
        if (P.sgs) {
          S SS = 0.0;
          for (int a = 0; a < 3; ++a)
            for (int x = 0; x < 3; ++x) SS = SS + Sij[a][x] * Sij[a][x];
          S Smag = s_sqrt(2.0 * SS);
          double Delta = std::cbrt(1.0 / M[9][n]);
          if (P.sgs == 1) {
            mu_sgs = rho[n] * (P.Cs * Delta) * (P.Cs * Delta) * Smag;
            kap_sgs = mu_sgs * Cp / P.Pr_sgs;
          } else {  // R17
            const size_t col = (size_t)(j + G) * b.pi + (size_t)(i + G);
            mu_sgs = Cdyn[col] * rho[n] * (Delta * Delta) * Smag;
            kap_sgs = Cp * Ddyn[col] * rho[n] * (Delta * Delta) * Smag;
          }
          // R18: sigma_kk / 3 = (2/3) CI rho D^2 |S|^2, |S|^2 = 2 S:S
          if (P.CI > 0.0) pis[n] = (2.0 / 3.0) * P.CI * rho[n] * (Delta * Delta) * (2.0 * SS);
        }
        S mut = mu[n] + mu_sgs;
        for (int a = 0; a < 3; ++a)
          for (int x = 0; x < 3; ++x)
            tau[(size_t)(3 * a + x) * N + n] = 2.0 * mut * (Sij[a][x] - (a == x ? Skk / 3.0 : S(0.0)));
        S kap = mu[n] * Cp / P.Pr + kap_sgs;
        S uu[3] = {u[n], v[n], w[n]};
        for (int x = 0; x < 3; ++x) {
          S t = 0.0;
          for (int a = 0; a < 3; ++a) t = t + uu[a] * tau[(size_t)(3 * a + x) * N + n];
          Theta[(size_t)x * N + n] = t + kap * grad[(size_t)(9 + x) * N + n];  // R4
        }
      }

  // --- node fluxes H_d = E^_d - Ev^_d on B1, d = xi, eta, zeta (Eq. 15) ---
  std::vector<S> H(15 * N);
#pragma omp parallel for
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        size_t n = b.at(i, j, k);
        for (int d = 0; d < 3; ++d) {
          double mx = M[3 * d][n], my = M[3 * d + 1][n], mz = M[3 * d + 2][n];
          S U = mx * u[n] + my * v[n] + mz * w[n];
          // the isotropic SGS stress enters like a pressure (Eq. 1, R18)
          const S pe = p[n] + pis[n];
          S E[5];
          E[0] = rho[n] * U;
          E[1] = rho[n] * u[n] * U + mx * pe;
          E[2] = rho[n] * v[n] * U + my * pe;
          E[3] = rho[n] * w[n] * U + mz * pe;
          E[4] = (Qv[4][n] + pe) * U;
          S Ev[5];
          Ev[0] = 0.0;
          for (int a = 0; a < 3; ++a)
            Ev[1 + a] = mx * tau[(size_t)(3 * a + 0) * N + n] + my * tau[(size_t)(3 * a + 1) * N + n] +
                        mz * tau[(size_t)(3 * a + 2) * N + n];
          Ev[4] = mx * Theta[n] + my * Theta[N + n] + mz * Theta[2 * N + n];
          for (int q = 0; q < 5; ++q) H[(size_t)(5 * d + q) * N + n] = E[q] - Ev[q];
          // R19: on the axis xi/J = eta/J = 0 and J is infinite; the node
          // fluxes are taken as their limits there (0 for eta, the only one an
          // off-axis residual uses)
          if (b.axis && j == 0)
            for (int q = 0; q < 5; ++q) H[(size_t)(5 * d + q) * N + n] = 0.0;
        }
      }

  // --- spectral radii, anisotropic scaling and pressure sensor on B1 (R7) ---
  std::vector<S> lam(3 * N), Lam(3 * N), nu(3 * N);
#pragma omp parallel for
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        size_t n = b.at(i, j, k);
        for (int d = 0; d < 3; ++d) {
          double mx = M[3 * d][n], my = M[3 * d + 1][n], mz = M[3 * d + 2][n];
          S U = mx * u[n] + my * v[n] + mz * w[n];
          lam[(size_t)d * N + n] = s_abs(U) + c[n] * std::sqrt(mx * mx + my * my + mz * mz);
        }
      }
#pragma omp parallel for
  for (int k = -1; k <= b.nk; ++k)
    for (int j = -1; j <= b.nj; ++j)
      for (int i = -1; i <= b.ni; ++i) {
        size_t n = b.at(i, j, k);
        for (int d = 0; d < 3; ++d) {
          S ld = lam[(size_t)d * N + n];
          S le = lam[(size_t)((d + 1) % 3) * N + n];
          S lf = lam[(size_t)((d + 2) % 3) * N + n];
          Lam[(size_t)d * N + n] = ld * (1.0 + s_pow(le / ld, P.alpha) + s_pow(lf / ld, P.alpha));
          if (b.axis && j == 0) Lam[(size_t)d * N + n] = 0.0;  // R19: lam_eta = 0 on the axis
          int di, dj, dk;
          step(d, di, dj, dk);
          S pp = p[b.at(i + di, j + dj, k + dk)], pm = p[b.at(i - di, j - dj, k - dk)];
          nu[(size_t)d * N + n] = s_abs(pp - 2.0 * p[n] + pm) / (pp + 2.0 * p[n] + pm);
        }
      }

  // --- face fluxes F = (H_a + H_b)/2 - D, stored at the lower node a ---
  // faces exist for a = -1..n-1 along d, interior in the other directions.
  std::vector<S> F(15 * N);
  for (int d = 0; d < 3; ++d) {
    int di, dj, dk;
    step(d, di, dj, dk);
#pragma omp parallel for
    for (int k = -1; k < b.nk; ++k)
      for (int j = -1; j < b.nj; ++j)
        for (int i = -1; i < b.ni; ++i) {
          int id[3] = {i, j, k};
          bool ok = true;
          for (int e = 0; e < 3; ++e)
            if (e != d && id[e] < 0) ok = false;
          if (!ok) continue;
          size_t a = b.at(i, j, k);
          size_t bb = b.at(i + di, j + dj, k + dk);
          size_t am = b.at(i - di, j - dj, k - dk);
          size_t bp = b.at(i + 2 * di, j + 2 * dj, k + 2 * dk);
          S eps2 = P.k2 * s_max(nu[(size_t)d * N + a], nu[(size_t)d * N + bb]);
          S eps4 = s_max(S(0.0), P.k4 - eps2);
          S Lf = 0.5 * (Lam[(size_t)d * N + a] + Lam[(size_t)d * N + bb]);
          // R19: the face between the axis and j = 1 takes the cross-axis value
          // by linear extrapolation (no five-point stencil across the axis)
          const bool axis_face = b.axis && d == 1 && j == 0;
          for (int q = 0; q < 5; ++q) {
            S d1 = Qv[q][bb] - Qv[q][a];
            S d3 = axis_face ? Qv[q][bp] - 2.0 * Qv[q][bb] + Qv[q][a]
                             : Qv[q][bp] - 3.0 * Qv[q][bb] + 3.0 * Qv[q][a] - Qv[q][am];
            S D = Lf * (eps2 * d1 - eps4 * d3);
            F[(size_t)(5 * d + q) * N + a] = 0.5 * (H[(size_t)(5 * d + q) * N + a] + H[(size_t)(5 * d + q) * N + bb]) - D;
          }
        }
  }

  // --- residual at interior nodes (R1, R12) ---
  for (size_t n = 0; n < 5 * N; ++n) R[n] = 0.0;
#pragma omp parallel for
  for (int k = 0; k < b.nk; ++k)
    for (int j = 0; j < b.nj; ++j)
      for (int i = 0; i < b.ni; ++i) {
        size_t n = b.at(i, j, k);
        for (int q = 0; q < 5; ++q) {
          S s = 0.0;
          s = s + (F[(size_t)(0 + q) * N + n] - F[(size_t)(0 + q) * N + b.at(i - 1, j, k)]);
          s = s + (F[(size_t)(5 + q) * N + n] - F[(size_t)(5 + q) * N + b.at(i, j - 1, k)]);
          s = s + (F[(size_t)(10 + q) * N + n] - F[(size_t)(10 + q) * N + b.at(i, j, k - 1)]);
          S r = M[9][n] * s;
          if (f && i == i_f) r = r - f[((size_t)q * b.nk + k) * b.nj + j];
          if (b.axis && j == 0) r = 0.0;  // R19: the axis follows the centerline condition
          R[(size_t)q * N + n] = r;
        }
      }
}

// ---------------------------------------------------------------------------
// R9: CFL time step from the interior of Q (no ghosts needed).
// ---------------------------------------------------------------------------
double cfl_dt(const Box& b, const orc_params& P, const double* m, const double* Q) {
  const size_t N = b.N;
  const double g = P.gamma;
  double best = INFINITY;
  for (int k = 0; k < b.nk; ++k)
    for (int j = b.axis ? 1 : 0; j < b.nj; ++j)  // R19: not on the axis
      for (int i = 0; i < b.ni; ++i) {
        size_t n = b.at(i, j, k);
        double rho = Q[n], u = Q[N + n] / rho, v = Q[2 * N + n] / rho, w = Q[3 * N + n] / rho;
        double p = (g - 1.0) * (Q[4 * N + n] - 0.5 * rho * (u * u + v * v + w * w));
        double T = p / (rho * P.R_gas);
        double c = std::sqrt(g * p / rho);
        double th = T / P.T_ref;
        double mu = P.mu_ref * std::pow(th, 1.5) * (1.0 + P.S_suth) / (th + P.S_suth);
        double nuv = std::max(4.0 / 3.0, g / P.Pr) * mu / rho;
        double J = m[9 * N + n];
        double lam = 0.0, g2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          double gx = J * m[(3 * d) * N + n], gy = J * m[(3 * d + 1) * N + n], gz = J * m[(3 * d + 2) * N + n];
          double U = gx * u + gy * v + gz * w;
          double gg = gx * gx + gy * gy + gz * gz;
          lam += std::fabs(U) + c * std::sqrt(gg);
          g2 += gg;
        }
        double loc = 1.0 / (lam + 2.0 * nuv * g2);
        if (loc < best) best = loc;
      }
  return P.cfl * best;
}

const double RK_ALPHA[5] = {0.25, 1.0 / 6.0, 0.375, 0.5, 1.0};

// ---------------------------------------------------------------------------
// One RK step (R8).  Q: padded [5][N], in/out (interior = Q^{n+1} on return;
// ghosts = the filled ghosts of Q^n).  stages (optional): [5][5][N] receives
// the stage inputs Q^(0..4) with their ghosts filled.  norms (optional):
// L2 (RMS) then Linf of R(Q^n) per variable.
// ---------------------------------------------------------------------------
template <class S>
void rk_step(const Box& b, const orc_params& P, const double* m, S* Q, double dt, const S* f, int i_f,
             double* norms, S* stages) {
  const size_t N = b.N;
  apply_axis(b, Q);
  fill_ghosts(b, Q, 5);
  std::vector<S> Q0(Q, Q + 5 * N), cur(Q, Q + 5 * N), R(5 * N);
  for (int l = 0; l < 5; ++l) {
    apply_axis(b, cur.data());
    fill_ghosts(b, cur.data(), 5);
    if (stages) std::copy(cur.begin(), cur.end(), stages + (size_t)l * 5 * N);
    residual(b, P, m, cur.data(), f, i_f, R.data());
    if (l == 0 && norms) {
      size_t cnt = (size_t)b.ni * b.nj * b.nk;
      for (int q = 0; q < 5; ++q) {
        double s2 = 0.0, mx = 0.0;
        for (int k = 0; k < b.nk; ++k)
          for (int j = 0; j < b.nj; ++j)
            for (int i = 0; i < b.ni; ++i) {
              double r = val(R[(size_t)q * N + b.at(i, j, k)]);
              s2 += r * r;
              if (std::fabs(r) > mx || std::isnan(r)) mx = std::isnan(r) ? r : std::fabs(r);
            }
        norms[q] = std::sqrt(s2 / (double)cnt);
        norms[5 + q] = mx;
      }
    }
    std::vector<S> nxt(Q0);
#pragma omp parallel for
    for (int k = 0; k < b.nk; ++k)
      for (int j = 0; j < b.nj; ++j)
        for (int i = 0; i < b.ni; ++i) {
          size_t n = b.at(i, j, k);
          for (int q = 0; q < 5; ++q)
            nxt[(size_t)q * N + n] = Q0[(size_t)q * N + n] - (RK_ALPHA[l] * dt) * R[(size_t)q * N + n];
        }
    apply_axis(b, nxt.data());  // boundary update after the stage (Alg. 2)
    cur.swap(nxt);
  }
  for (int k = 0; k < b.nk; ++k)
    for (int j = 0; j < b.nj; ++j)
      for (int i = 0; i < b.ni; ++i) {
        size_t n = b.at(i, j, k);
        for (int q = 0; q < 5; ++q) Q[(size_t)q * N + n] = cur[(size_t)q * N + n];
      }
}

template <class S>
S probe_pressure_sq(const Box& b, const orc_params& P, const S* Q, int i_p, double p_inf) {
  const size_t N = b.N;
  const double g = P.gamma;
  S acc = 0.0;
  // over the distinct k planes (a superposed direction's last plane is its
  // first one's place)
  const int nks = b.bc[2] == 2 ? b.nk - 1 : b.nk;
  for (int k = 0; k < nks; ++k)
    for (int j = 0; j < b.nj; ++j) {
      size_t n = b.at(i_p, j, k);
      S rho = Q[n], u = Q[N + n] / rho, v = Q[2 * N + n] / rho, w = Q[3 * N + n] / rho;
      S p = (g - 1.0) * (Q[4 * N + n] - 0.5 * rho * (u * u + v * v + w * w));
      S dp = p - p_inf;
      acc = acc + dp * dp;
    }
  return acc;
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

size_t orc_box_nodes(const orc_dims* d) { return Box(*d).N; }

// Threads of the OpenMP loops (n <= 0: leave unchanged); returns the number
// the next parallel loop will use (1 without OpenMP).
int orc_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void orc_metrics(const orc_dims* d, const double* xyz, double* m) { metrics(Box(*d), xyz, m); }

void orc_fill_ghosts(const orc_dims* d, double* a, int nfields) { fill_ghosts(Box(*d), a, nfields); }

// Ghost fill of a state including the boundary faces of d (R13, R14, R16).
void orc_fill_ghosts_faces(const orc_dims* d, const orc_params* P, const double* m, double* Q) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  apply_axis(b, Q);
  fill_ghosts(b, Q, 5);
}

// The residual of a state whose ghost layers (and axis nodes) are taken as
// given, without the ghost fill: for tests of what a stencil reads.
void orc_residual_nofill(const orc_dims* d, const orc_params* P, const double* m, const double* Q, double* R) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  residual(b, *P, m, Q, (const double*)nullptr, -1, R);
}

// R of a state (ghosts of a copy are filled first).  f: [5][nk][nj] or NULL.
void orc_residual(const orc_dims* d, const orc_params* P, const double* m, const double* Q, const double* f, int i_f,
                  double* R) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  std::vector<double> q(Q, Q + 5 * b.N);
  apply_axis(b, q.data());
  fill_ghosts(b, q.data(), 5);
  residual(b, *P, m, q.data(), f, i_f, R);
}

// Tangent of the residual: dR = (dR/dQ) dQ + (dR/df) df (ghosts of copies filled).
void orc_residual_tangent(const orc_dims* d, const orc_params* P, const double* m, const double* Q, const double* dQ,
                          const double* f, const double* df, int i_f, double* R, double* dR) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  std::vector<Dual> q(5 * b.N), r(5 * b.N);
  for (size_t n = 0; n < 5 * b.N; ++n) q[n] = Dual(Q[n], dQ ? dQ[n] : 0.0);
  apply_axis(b, q.data());
  fill_ghosts(b, q.data(), 5);
  std::vector<Dual> fd;
  if (f) {
    size_t nf = (size_t)5 * b.nk * b.nj;
    fd.resize(nf);
    for (size_t n = 0; n < nf; ++n) fd[n] = Dual(f[n], df ? df[n] : 0.0);
  }
  residual(b, *P, m, q.data(), f ? fd.data() : nullptr, i_f, r.data());
  for (size_t n = 0; n < 5 * b.N; ++n) {
    R[n] = r[n].v;
    dR[n] = r[n].d;
  }
}

// R17: dynamic coefficients of a state (ghosts of a copy filled first);
// C, D: [(nj+4)(ni+4)] per padded column (i fastest).
void orc_dynamic_coefficients(const orc_dims* d, const orc_params* P, const double* m, const double* Q, double* C,
                              double* D) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  std::vector<double> q(Q, Q + 5 * b.N);
  fill_ghosts(b, q.data(), 5);
  std::vector<double> Cc, Dc;
  dynamic_coefficients(b, *P, m, q.data(), Cc, Dc);
  std::copy(Cc.begin(), Cc.end(), C);
  std::copy(Dc.begin(), Dc.end(), D);
}

double orc_cfl_dt(const orc_dims* d, const orc_params* P, const double* m, const double* Q) {
  return cfl_dt(Box(*d), *P, m, Q);
}

// One RK step.  dt <= 0 selects the CFL time step from Q^n.  Returns the dt used.
double orc_rk_step(const orc_dims* d, const orc_params* P, const double* m, double* Q, double dt, const double* f,
                   int i_f, double* norms, double* stages) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  if (!(dt > 0.0)) dt = cfl_dt(b, *P, m, Q);
  rk_step(b, *P, m, Q, dt, f, i_f, norms, stages);
  return dt;
}

// Tangent of one RK step at fixed dt: (Q, dQ) -> (Q^{n+1}, dQ^{n+1}) for the
// perturbation (dQ, df) of the state and of the source f on plane i_f.
void orc_rk_step_tangent(const orc_dims* d, const orc_params* P, const double* m, double* Q, double* dQ, double dt,
                         const double* f, const double* df, int i_f) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  std::vector<Dual> q(5 * b.N);
  for (size_t n = 0; n < 5 * b.N; ++n) q[n] = Dual(Q[n], dQ[n]);
  std::vector<Dual> fd;
  if (f) {
    size_t nf = (size_t)5 * b.nk * b.nj;
    fd.resize(nf);
    for (size_t n = 0; n < nf; ++n) fd[n] = Dual(f[n], df ? df[n] : 0.0);
  }
  rk_step(b, *P, m, q.data(), dt, f ? fd.data() : nullptr, i_f, nullptr, (Dual*)nullptr);
  for (size_t n = 0; n < 5 * b.N; ++n) {
    Q[n] = q[n].v;
    dQ[n] = q[n].d;
  }
}

// Objective of the differentiation workload: run nsteps RK steps at fixed dt
// from Q0 with source f on plane i_f, and return
//   J = sum_{n=1..nsteps} dt * sum_{j,k} (p(Q^n)_{i_p,j,k} - p_inf)^2
// together with its directional derivative along (dQ0, df) in *dJ.
// Q0 is overwritten with Q^nsteps.
double orc_objective_rollout(const orc_dims* d, const orc_params* P, const double* m, double* Q0, const double* dQ0,
                             const double* f, const double* df, int i_f, int i_p, double p_inf, int nsteps, double dt,
                             double* dJ) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  std::vector<Dual> q(5 * b.N);
  for (size_t n = 0; n < 5 * b.N; ++n) q[n] = Dual(Q0[n], dQ0 ? dQ0[n] : 0.0);
  size_t nf = (size_t)5 * b.nk * b.nj;
  std::vector<Dual> fd(nf);
  for (size_t n = 0; n < nf; ++n) fd[n] = Dual(f ? f[n] : 0.0, df ? df[n] : 0.0);
  Dual J = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    rk_step(b, *P, m, q.data(), dt, fd.data(), i_f, nullptr, (Dual*)nullptr);
    J = J + dt * probe_pressure_sq(b, *P, q.data(), i_p, p_inf);
  }
  for (size_t n = 0; n < 5 * b.N; ++n) Q0[n] = q[n].v;
  if (dJ) *dJ = J.d;
  return J.v;
}

// Plain-double objective (same definition) for finite differences.
double orc_objective(const orc_dims* d, const orc_params* P, const double* m, double* Q0, const double* f, int i_f,
                     int i_p, double p_inf, int nsteps, double dt) {
  Box b(*d);
  b.m = m;
  b.gamma = P->gamma;
  double J = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    rk_step(b, *P, m, Q0, dt, f, i_f, nullptr, (double*)nullptr);
    J += dt * probe_pressure_sq(b, *P, Q0, i_p, p_inf);
  }
  return J;
}

// Running flow statistics (the time- and azimuth-averaged mean-flow and RMS
// profiles of Sec. 6; the averaged periodic direction is k):
//   acc[s][j][i] += sum over the distinct azimuths k = 0..nk_s-1 of phi_s(i, j, k),
//   phi = (rho, u, v, w, p, uu, vv, ww, uv, uw, vw, pp),
// with the primitives of Eq. 2: u_a = (rho u_a) / rho,
// p = (gamma - 1)(e - rho (u^2 + v^2 + w^2) / 2).  acc: dense [12][nj][ni].
// nk_s = nk, or nk - 1 when k is superposed periodic (Sec. 3: the first and
// last points are the same place, which the average counts once).
void orc_stats(const orc_dims* d, const orc_params* P, const double* Q, double* acc) {
  Box b(*d);
  const size_t plane = (size_t)b.ni * b.nj;
  const int nks = b.bc[2] == 2 ? b.nk - 1 : b.nk;
  for (int j = 0; j < b.nj; ++j)
    for (int i = 0; i < b.ni; ++i)
      for (int k = 0; k < nks; ++k) {
        const size_t n = b.at(i, j, k);
        const double rho = Q[n];
        const double u = Q[b.N + n] / rho, v = Q[2 * b.N + n] / rho, w = Q[3 * b.N + n] / rho;
        const double p = (P->gamma - 1.0) * (Q[4 * b.N + n] - 0.5 * rho * (u * u + v * v + w * w));
        const double phi[12] = {rho, u, v, w, p, u * u, v * v, w * w, u * v, u * w, v * w, p * p};
        for (int s = 0; s < 12; ++s) acc[s * plane + (size_t)j * b.ni + i] += phi[s];
      }
}

// Profiles of Sec. 6 from those sums after `samples` terms per entry: the
// Reynolds means <phi> = acc / samples of rho, u, v, w, p, the RMS
// fluctuations a_rms = sqrt(<a a> - <a>^2) of u, v, w, p (0 where rounding
// makes the difference negative) and the covariance <u'v'> = <u v> - <u><v>:
// prof = dense [10][nj][ni].  The potential core (Sec. 6) is where the mean
// axial velocity <u> reaches core_frac times the jet velocity u_jet:
// core[j][i] = 1 there, else 0 (core may be null).
void orc_stats_profiles(int ni, int nj, const double* acc, double samples, double u_jet, double core_frac,
                        double* prof, unsigned char* core) {
  const size_t plane = (size_t)ni * nj;
  for (size_t n = 0; n < plane; ++n) {
    double mean[12];
    for (int s = 0; s < 12; ++s) mean[s] = acc[s * plane + n] / samples;
    const double rho = mean[0], u = mean[1], v = mean[2], w = mean[3], p = mean[4];
    const double uu = mean[5], vv = mean[6], ww = mean[7], uv = mean[8], pp = mean[11];
    prof[0 * plane + n] = rho;
    prof[1 * plane + n] = u;
    prof[2 * plane + n] = v;
    prof[3 * plane + n] = w;
    prof[4 * plane + n] = p;
    prof[5 * plane + n] = std::sqrt(std::max(0.0, uu - u * u));
    prof[6 * plane + n] = std::sqrt(std::max(0.0, vv - v * v));
    prof[7 * plane + n] = std::sqrt(std::max(0.0, ww - w * w));
    prof[8 * plane + n] = std::sqrt(std::max(0.0, pp - p * p));
    prof[9 * plane + n] = uv - u * v;
    if (core) core[n] = u >= core_frac * u_jet ? 1 : 0;
  }
}

// Test hook for the scalar rules R11 and the RK driver on y' = lambda y
// (complex lambda), used to check the amplification polynomial.
void orc_rk_scalar(double lr, double li, double dt, double* yr, double* yi) {
  double y0r = *yr, y0i = *yi, cr = y0r, ci = y0i;
  for (int l = 0; l < 5; ++l) {
    // R(y) = -lambda y  (dy/dt = -R)
    double Rr = -(lr * cr - li * ci), Ri = -(lr * ci + li * cr);
    cr = y0r - RK_ALPHA[l] * dt * Rr;
    ci = y0i - RK_ALPHA[l] * dt * Ri;
  }
  *yr = cr;
  *yi = ci;
}

}  // extern "C"
