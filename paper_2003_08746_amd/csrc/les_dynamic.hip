// les_dynamic.hip -- dynamic SGS closure for gfx950: the per-column
// coefficients of mu_sgs = C rho D^2 |S| and kappa_sgs = Cp D_T rho D^2 |S|
// (the paper fixes Pr_sgs = 0.9 for static closures only, Sec. 3, Eq. 5).
//
// Germano's identity between the grid filter and a test filter of twice its
// width, in the Favre form of Moin, Squires, Cabot and Lee (1991), with
// Lilly's least squares summed over the periodic k direction:
//   C   = max(0, <L^d : M> / <M : M>),   D_T = max(0, <K . N> / <N . N>),
//   L_ij = (rho u_i u_j)^ - (rho u_i)^ (rho u_j)^ / rho^,
//   M_ij = 2 (D^2 rho |S| S^d_ij)^ - 2 (2D)^2 rho^ |S~| S~^d_ij,
//   K_j  = (rho u_j T)^ - (rho u_j)^ (rho T)^ / rho^,
//   N_j  = (D^2 rho |S| dT/dx_j)^ - (2D)^2 rho^ |S~| dT~/dx_j,
// ^ the test filter (weights 1/4, 1/2, 1/4 along each index), u~ and T~ the
// test-filtered Favre velocity and temperature, D = (1/J)^(1/3).
//
// Five launches per evaluation, all streaming one node per thread:
//   k_dyn_raw     the 23 grid-level fields (rho, rho u, rho T, rho u u,
//                 rho u T on the whole padded box; the 9 strain and
//                 temperature-gradient products on [-1, n]^3);
//   k_dyn_filter  three separable passes of the test filter (i, j, k);
//   k_dyn_node    the four contractions at every interior node;
//   k_dyn_coef    per padded column: the sums over interior k (ascending,
//                 one thread per column, so the order is fixed) and the
//                 clipped ratios; ghost columns take the wrapped (periodic)
//                 or nearest interior (Dirichlet) column.
// This is an optional model: the streaming passes cost about 1 KB of HBM
// traffic per point and evaluation (23 fields, three filter passes).
#include "les_dynamic.hpp"

namespace les {

namespace {

constexpr int NRAW = 23;
// symmetric index pairs (a <= b) in the order of the raw fields
__constant__ int kPair[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};

__device__ inline bool in_box(const Layout& L, int i, int j, int k) {
  return i >= -2 && j >= -2 && k >= -2 && i <= L.ni + 1 && j <= L.nj + 1 && k <= L.nk + 1;
}

// node index (i, j, k) in [-2, n+1]^3 of a linear thread index over the padded box
__device__ inline void padded_node(const Layout& L, long long t, int& i, int& j, int& k) {
  const int pi = L.ni + 4, pj = L.nj + 4;
  i = (int)(t % pi) - 2;
  j = (int)((t / pi) % pj) - 2;
  k = (int)(t / ((long long)pi * pj)) - 2;
}

// primitives (u, v, w, T) of a state node, in FP64
template <class QI>
__device__ inline void dyn_prims(const QI* Q, long long fe, long long n, const Phys& P, double& rho, double u[3],
                                 double& T) {
  rho = (double)Q[n];
  for (int a = 0; a < 3; ++a) u[a] = (double)Q[(1 + a) * fe + n] / rho;
  const double p = P.gm1 * ((double)Q[4 * fe + n] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  T = p / rho * P.inv_R;
}

// strain rate's deviatoric part and |S| = sqrt(2 S:S) from du[a][x]
__device__ inline void dyn_strain(const double du[3][3], double Sd[3][3], double& mag) {
  double S[3][3], ss = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int x = 0; x < 3; ++x) {
      S[a][x] = 0.5 * (du[a][x] + du[x][a]);
      ss += S[a][x] * S[a][x];
    }
  const double tr = (S[0][0] + S[1][1] + S[2][2]) / 3.0;
  for (int a = 0; a < 3; ++a)
    for (int x = 0; x < 3; ++x) Sd[a][x] = S[a][x] - (a == x ? tr : 0.0);
  mag = sqrt(2.0 * ss);
}

// chain rule: physical gradient from index-space differences d[e] (e = xi,
// eta, zeta) and the node's metrics over J
__device__ inline void dyn_chain(const double* M, long long fe, long long n, const double d[3], double g[3]) {
  const double J = M[9 * fe + n];
  for (int x = 0; x < 3; ++x) g[x] = J * (M[x * fe + n] * d[0] + M[(3 + x) * fe + n] * d[1] + M[(6 + x) * fe + n] * d[2]);
}

template <class QI>
__global__ void __launch_bounds__(256) k_dyn_raw(Layout L, Phys P, const double* __restrict__ M,
                                                 const QI* __restrict__ Q, double* __restrict__ W) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)(L.ni + 4) * (L.nj + 4) * (L.nk + 4);
  if (t >= tot) return;
  int i, j, k;
  padded_node(L, t, i, j, k);
  const long long fe = L.fe, n = L.at(i, j, k);
  double rho, u[3], T;
  dyn_prims(Q, fe, n, P, rho, u, T);
  double F[NRAW];
  F[0] = rho;
  for (int a = 0; a < 3; ++a) F[1 + a] = rho * u[a];
  F[4] = rho * T;
  for (int q = 0; q < 6; ++q) F[5 + q] = rho * u[kPair[q][0]] * u[kPair[q][1]];
  for (int a = 0; a < 3; ++a) F[11 + a] = rho * u[a] * T;
  for (int q = 14; q < NRAW; ++q) F[q] = 0.0;
  if (i >= -1 && j >= -1 && k >= -1 && i <= L.ni && j <= L.nj && k <= L.nk) {
    // node gradients of u, v, w, T (central differences, chain rule)
    double dd[4][3];
    const long long st[3] = {1, L.sj, L.sk};
    for (int e = 0; e < 3; ++e) {
      double r1, u1[3], T1, r0, u0[3], T0;
      dyn_prims(Q, fe, n + st[e], P, r1, u1, T1);
      dyn_prims(Q, fe, n - st[e], P, r0, u0, T0);
      for (int a = 0; a < 3; ++a) dd[a][e] = 0.5 * (u1[a] - u0[a]);
      dd[3][e] = 0.5 * (T1 - T0);
    }
    double du[3][3], dT[3], Sd[3][3], mag;
    for (int a = 0; a < 3; ++a) dyn_chain(M, fe, n, dd[a], du[a]);
    dyn_chain(M, fe, n, dd[3], dT);
    dyn_strain(du, Sd, mag);
    const double D = cbrt(1.0 / M[9 * fe + n]);
    const double w = D * D * rho * mag;
    for (int q = 0; q < 6; ++q) F[14 + q] = w * Sd[kPair[q][0]][kPair[q][1]];
    for (int a = 0; a < 3; ++a) F[20 + a] = w * dT[a];
  }
  for (int q = 0; q < NRAW; ++q) W[q * fe + n] = F[q];
}

// out = test filter of in along direction d at nodes whose d index is in
// [-1, n] (every other index over the padded box)
__global__ void __launch_bounds__(256) k_dyn_filter(Layout L, int d, const double* __restrict__ in,
                                                    double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)(L.ni + 4) * (L.nj + 4) * (L.nk + 4);
  if (t >= tot) return;
  int i, j, k;
  padded_node(L, t, i, j, k);
  const int id[3] = {i, j, k}, nn[3] = {L.ni, L.nj, L.nk};
  if (id[d] < -1 || id[d] > nn[d]) return;
  const long long n = L.at(i, j, k), s = d == 0 ? 1 : (d == 1 ? L.sj : L.sk);
  for (int q = 0; q < NRAW; ++q) {
    const double* a = in + q * L.fe;
    out[q * L.fe + n] = 0.25 * a[n - s] + 0.5 * a[n] + 0.25 * a[n + s];
  }
}

// X[0..3][n] = L^d:M, M:M, K.N, N.N at interior nodes from the filtered
// fields F (valid on [-1, n]^3 for rho^, (rho u)^, (rho T)^; on the
// interior for the rest)
__global__ void __launch_bounds__(256) k_dyn_node(Layout L, const double* __restrict__ M,
                                                  const double* __restrict__ F, double* __restrict__ X) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)L.ni * L.nj * L.nk;
  if (t >= tot) return;
  const int i = (int)(t % L.ni), j = (int)((t / L.ni) % L.nj), k = (int)(t / ((long long)L.ni * L.nj));
  const long long fe = L.fe, n = L.at(i, j, k);
  const long long st[3] = {1, L.sj, L.sk};
  // test-filtered velocity and temperature at the axis neighbours
  double dd[4][3];
  for (int e = 0; e < 3; ++e) {
    const long long p1 = n + st[e], p0 = n - st[e];
    const double r1 = F[p1], r0 = F[p0];
    for (int a = 0; a < 3; ++a) dd[a][e] = 0.5 * (F[(1 + a) * fe + p1] / r1 - F[(1 + a) * fe + p0] / r0);
    dd[3][e] = 0.5 * (F[4 * fe + p1] / r1 - F[4 * fe + p0] / r0);
  }
  double du[3][3], dT[3], Sd[3][3], mag;
  for (int a = 0; a < 3; ++a) dyn_chain(M, fe, n, dd[a], du[a]);
  dyn_chain(M, fe, n, dd[3], dT);
  dyn_strain(du, Sd, mag);
  const double D = cbrt(1.0 / M[9 * fe + n]);
  const double Dt2 = 4.0 * D * D;  // (2 D)^2
  double fv[NRAW];
  for (int q = 0; q < NRAW; ++q) fv[q] = F[q * fe + n];
  double Lm[3][3], Mm[3][3];
  for (int q = 0; q < 6; ++q) {
    const int a = kPair[q][0], c = kPair[q][1];
    Lm[a][c] = Lm[c][a] = fv[5 + q] - fv[1 + a] * fv[1 + c] / fv[0];
    Mm[a][c] = Mm[c][a] = 2.0 * fv[14 + q] - 2.0 * Dt2 * fv[0] * mag * Sd[a][c];
  }
  const double tr = (Lm[0][0] + Lm[1][1] + Lm[2][2]) / 3.0;
  for (int a = 0; a < 3; ++a) Lm[a][a] -= tr;
  double lm = 0.0, mm = 0.0, kn = 0.0, nn = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      lm += Lm[a][c] * Mm[a][c];
      mm += Mm[a][c] * Mm[a][c];
    }
  for (int a = 0; a < 3; ++a) {
    const double K = fv[11 + a] - fv[1 + a] * fv[4] / fv[0];
    const double N = fv[20 + a] - Dt2 * fv[0] * mag * dT[a];
    kn += K * N;
    nn += N * N;
  }
  X[n] = lm;
  X[fe + n] = mm;
  X[2 * fe + n] = kn;
  X[3 * fe + n] = nn;
}

__device__ inline int dyn_src(int x, int n, int bc) {
  if (x >= 0 && x < n) return x;
  if (bc == 1) return x < 0 ? 0 : n - 1;  // Dirichlet: nearest interior column
  const int p = bc == 2 ? n - 1 : n;      // periodic (superposed: period n - 1)
  return ((x % p) + p) % p;
}

__global__ void __launch_bounds__(256) k_dyn_coef(Layout L, int bc0, int bc1, const double* __restrict__ X,
                                                  double* __restrict__ dyn) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncol = dyn_ncol(L);
  if (c >= ncol) return;
  const int i = (int)(c % (L.ni + 4)) - 2, j = (int)(c / (L.ni + 4)) - 2;
  const int is = dyn_src(i, L.ni, bc0), js = dyn_src(j, L.nj, bc1);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < L.nk; ++k) {
    const long long n = L.at(is, js, k);
    for (int q = 0; q < 4; ++q) s[q] += X[q * L.fe + n];
  }
  dyn[c] = s[1] > 0.0 ? fmax(0.0, s[0] / s[1]) : 0.0;
  dyn[ncol + c] = s[3] > 0.0 ? fmax(0.0, s[2] / s[3]) : 0.0;
}

inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

template <class QI>
hipError_t run(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M, const QI* Q,
               double* work, double* dyn) {
  const long long fe = L.fe;
  double* W = work;
  double* V = work + NRAW * fe;
  double* X = work + 2 * NRAW * fe;
  const long long tot = (long long)(L.ni + 4) * (L.nj + 4) * (L.nk + 4);
  k_dyn_raw<QI><<<nblk(tot, 256), 256, 0, s>>>(L, P, M, Q, W);
  k_dyn_filter<<<nblk(tot, 256), 256, 0, s>>>(L, 0, W, V);
  k_dyn_filter<<<nblk(tot, 256), 256, 0, s>>>(L, 1, V, W);
  k_dyn_filter<<<nblk(tot, 256), 256, 0, s>>>(L, 2, W, V);
  k_dyn_node<<<nblk((long long)L.ni * L.nj * L.nk, 256), 256, 0, s>>>(L, M, V, X);
  k_dyn_coef<<<nblk(dyn_ncol(L), 256), 256, 0, s>>>(L, bc[0], bc[1], X, dyn);
  return hipGetLastError();
}

}  // namespace

long long dynamic_work_elems(const Layout& L) { return (2LL * NRAW + 4) * L.fe; }

hipError_t launch_dynamic(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M,
                          const double* Q, double* work, double* dyn) {
  return run<double>(s, L, bc, P, M, Q, work, dyn);
}

hipError_t launch_dynamic_f32(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M,
                              const float* Q, double* work, double* dyn) {
  return run<float>(s, L, bc, P, M, Q, work, dyn);
}

}  // namespace les
