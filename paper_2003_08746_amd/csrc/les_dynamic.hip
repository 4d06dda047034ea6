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
// Three launches per evaluation:
//   k_dyn_plane   per (i, j) tile and segment of k planes, marching in k:
//                 the 23 grid-level fields of each plane (rho, rho u,
//                 rho T, rho u u, rho u T on the whole padded box; the 9
//                 strain and temperature-gradient products on [-1, n]^3)
//                 computed into LDS and filtered along i and j there, then
//                 along k in registers; written on [-1, n]^3;
//   k_dyn_node    per interior column and segment of k: the test-filtered
//                 Favre velocity and temperature gradients and the four
//                 contractions at each node, summed over the segment's k
//                 in ascending order;
//   k_dyn_coef    per padded column: the segment sums added in ascending
//                 order (a fixed order) and the clipped ratios; ghost
//                 columns take the wrapped (periodic) or nearest interior
//                 (Dirichlet) column, across the polar axis the ring column
//                 of the same radius; the axis column takes ring 1's.
// The sums over k run over the distinct planes (nk - 1 along a superposed
// direction).  On the polar axis (a node of zero volume) the strain and
// temperature-gradient products are 0 and no contractions are formed.
// The filter is separable and applied along i, then j, then k, each a
// three-point sum evaluated left to right.  This is an optional model: its
// passes move about 0.45 KB of HBM traffic per point and evaluation (the 23
// filtered fields written once and read once).

#include "les_dynamic.hpp"

namespace les {

namespace {

constexpr int NRAW = 23;
// symmetric index pairs (a <= b) in the order of the raw fields
__constant__ int kPair[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};

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

// Tile of k_dyn_plane: DPX x DPY threads hold the raw fields of the output
// tile (DPX - 2) x (DPY - 2) and its one-node ring; a block marches DPK
// output planes in k.  The primitives are formed once per node and plane on
// the thread tile and one more ring (PPX x PPY) and shared through LDS.
constexpr int DPX = 32, DPY = 16, DPK = 16;
constexpr int DPTI = DPX - 2, DPTJ = DPY - 2;
constexpr int PPX = DPX + 2, PPY = DPY + 2;

__host__ __device__ inline long long dyn_plane_tiles(const Layout& L) {
  return (long long)((L.ni + 2 + DPTI - 1) / DPTI) * ((L.nj + 2 + DPTJ - 1) / DPTJ);
}
inline long long dyn_plane_blocks(const Layout& L) { return dyn_plane_tiles(L) * ((L.nk + 2 + DPK - 1) / DPK); }

// the primitives (rho, u, v, w, T) of node (i, j, k), zero off the padded box
template <class QI>
__device__ inline void dyn_prims_at(const Layout& L, const Phys& P, const QI* __restrict__ Q, int i, int j, int k,
                                    double pr[5]) {
  for (int c = 0; c < 5; ++c) pr[c] = 0.0;
  if (i >= -2 && j >= -2 && k >= -2 && i <= L.ni + 1 && j <= L.nj + 1 && k <= L.nk + 1)
    dyn_prims(Q, L.fe, L.at(i, j, k), P, pr[0], &pr[1], pr[4]);
}

// A double from the neighbouring lane of the wave (DPP wave shifts by one
// lane): lane l reads lane l - 1 (shr) or l + 1 (shl); the end lanes read 0.
__device__ inline double lane_prev(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double lane_next(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// V[q] = the test filter of raw field q (along i, then j, then k) at every
// node of [-1, n]^3.  Each block owns a tile and a segment of DPK output
// planes.  Per plane k of its march: the primitives of plane k + 1 into LDS,
// the raw fields of plane k in registers (in-plane neighbours' primitives
// from LDS, those of planes k -+ 1 of the thread's own column from registers
// and LDS), the filter along i across lanes into LDS, along j from LDS, and
// along k in
// registers: out(k) = (0.25 G(k-1) + 0.5 G(k)) + 0.25 G(k+1), carried as the
// pending sum of the two earlier planes and a quarter of the last.
template <class QI>
__global__ void __launch_bounds__(DPX * DPY) k_dyn_plane(Layout L, Phys P, int axis, const double* __restrict__ M,
                                                         const QI* __restrict__ Q, double* __restrict__ V) {
  __shared__ double sF[NRAW][DPY][DPX];
  __shared__ double sP[2][5][PPY][PPX];
  const long long fe = L.fe;
  const int tiles_i = (L.ni + 2 + DPTI - 1) / DPTI;
  const long long tiles = dyn_plane_tiles(L);
  const long long b = blockIdx.x;
  const long long tb = b % tiles;
  const int ka = -1 + (int)(b / tiles) * DPK;                // first output plane
  const int kb = ka + DPK < L.nk + 1 ? ka + DPK : L.nk + 1;  // one past the last
  const int tx = threadIdx.x % DPX, ty = threadIdx.x / DPX;
  const int i0 = -1 + (int)(tb % tiles_i) * DPTI, j0 = -1 + (int)(tb / tiles_i) * DPTJ;
  const int i = i0 - 1 + tx, j = j0 - 1 + ty;  // this thread's node; the LDS tiles start at (i0 - 2, j0 - 2)
  const bool in_box = i <= L.ni + 1 && j <= L.nj + 1;
  // the strain and temperature-gradient products on [-1, n]^3, except on the
  // polar axis (a node of zero volume, D = 0, whose strain is 0/0: 0 there)
  const bool grad_ij = i >= -1 && j >= -1 && i <= L.ni && j <= L.nj && !(axis && j == 0);
  const bool out_node = tx >= 1 && tx < DPX - 1 && ty >= 1 && ty < DPY - 1 && i <= L.ni && j <= L.nj;

  // primitives of plane kp on the LDS tile, into buffer kp & 1
  auto prims_plane = [&](int kp) {
    for (int t = threadIdx.x; t < PPX * PPY; t += DPX * DPY) {
      const int x = t % PPX, y = t / PPX;
      double pr[5];
      dyn_prims_at(L, P, Q, i0 - 2 + x, j0 - 2 + y, kp, pr);
      for (int c = 0; c < 5; ++c) sP[kp & 1][c][y][x] = pr[c];
    }
  };
  double pm[5];  // primitives of plane k - 1 at this node
  dyn_prims_at(L, P, Q, i, j, ka - 2, pm);
  prims_plane(ka - 1);
  double pend[NRAW], quarter[NRAW];
  for (int q = 0; q < NRAW; ++q) pend[q] = quarter[q] = 0.0;
  for (int k = ka - 1; k <= kb; ++k) {
    // (the previous plane's readers of buffer (k + 1) & 1 and of sF passed
    // the barrier before its filter)
    prims_plane(k + 1);
    __syncthreads();
    const int bc = k & 1, bn = (k + 1) & 1;
    double pc[5];
    for (int c = 0; c < 5; ++c) pc[c] = sP[bc][c][ty + 1][tx + 1];
    double F[NRAW];
    for (int q = 0; q < NRAW; ++q) F[q] = 0.0;
    if (in_box) {
      const double rho = pc[0], u[3] = {pc[1], pc[2], pc[3]}, T = pc[4];
      F[0] = rho;
      for (int a = 0; a < 3; ++a) F[1 + a] = rho * u[a];
      F[4] = rho * T;
      for (int q = 0; q < 6; ++q) F[5 + q] = rho * u[kPair[q][0]] * u[kPair[q][1]];
      for (int a = 0; a < 3; ++a) F[11 + a] = rho * u[a] * T;
      if (grad_ij && k >= -1 && k <= L.nk) {
        // node gradients of u, v, w, T (central differences, chain rule)
        double dd[4][3];
        for (int a = 0; a < 4; ++a) {
          dd[a][0] = 0.5 * (sP[bc][1 + a][ty + 1][tx + 2] - sP[bc][1 + a][ty + 1][tx]);
          dd[a][1] = 0.5 * (sP[bc][1 + a][ty + 2][tx + 1] - sP[bc][1 + a][ty][tx + 1]);
          dd[a][2] = 0.5 * (sP[bn][1 + a][ty + 1][tx + 1] - pm[1 + a]);
        }
        const long long n = L.at(i, j, k);
        double du[3][3], dT[3], Sd[3][3], mag;
        for (int a = 0; a < 3; ++a) dyn_chain(M, fe, n, dd[a], du[a]);
        dyn_chain(M, fe, n, dd[3], dT);
        dyn_strain(du, Sd, mag);
        const double D = cbrt(1.0 / M[9 * fe + n]);
        const double w = D * D * rho * mag;
        for (int q = 0; q < 6; ++q) F[14 + q] = w * Sd[kPair[q][0]][kPair[q][1]];
        for (int a = 0; a < 3; ++a) F[20 + a] = w * dT[a];
      }
    }
    for (int c = 0; c < 5; ++c) pm[c] = pc[c];
    // along i: the row's neighbours are the adjacent lanes (a row of the
    // tile is 32 consecutive lanes of one wave; only interior columns are
    // used below)
    for (int q = 0; q < NRAW; ++q) sF[q][ty][tx] = 0.25 * lane_prev(F[q]) + 0.5 * F[q] + 0.25 * lane_next(F[q]);
    __syncthreads();
    // along j, then along k
    if (out_node) {
      const long long n = L.at(i, j, k - 1);
      for (int q = 0; q < NRAW; ++q) {
        const double g = 0.25 * sF[q][ty - 1][tx] + 0.5 * sF[q][ty][tx] + 0.25 * sF[q][ty + 1][tx];
        if (k - 1 >= ka) V[q * fe + n] = pend[q] + 0.25 * g;
        pend[q] = quarter[q] + 0.5 * g;
        quarter[q] = 0.25 * g;
      }
    }
  }
}

// x[0..3] = L^d:M, M:M, K.N, N.N at interior node (i, j, k) from the
// filtered fields V (rho^, (rho u)^, (rho T)^ are also read at the six
// axis neighbours)
__device__ inline void dyn_contract(const Layout& L, const double* __restrict__ M, const double* __restrict__ V,
                                    int i, int j, int k, double x[4]) {
  const long long fe = L.fe, n = L.at(i, j, k);
  const long long st[3] = {1, L.sj, L.sk};
  // test-filtered velocity and temperature at the axis neighbours
  double dd[4][3];
  for (int e = 0; e < 3; ++e) {
    const long long p1 = n + st[e], p0 = n - st[e];
    const double r1 = V[p1], r0 = V[p0];
    for (int a = 0; a < 3; ++a) dd[a][e] = 0.5 * (V[(1 + a) * fe + p1] / r1 - V[(1 + a) * fe + p0] / r0);
    dd[3][e] = 0.5 * (V[4 * fe + p1] / r1 - V[4 * fe + p0] / r0);
  }
  double du[3][3], dT[3], Sd[3][3], mag;
  for (int a = 0; a < 3; ++a) dyn_chain(M, fe, n, dd[a], du[a]);
  dyn_chain(M, fe, n, dd[3], dT);
  dyn_strain(du, Sd, mag);
  const double D = cbrt(1.0 / M[9 * fe + n]);
  const double Dt2 = 4.0 * D * D;  // (2 D)^2
  double fv[NRAW];
  for (int q = 0; q < NRAW; ++q) fv[q] = V[q * fe + n];
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
  x[0] = lm;
  x[1] = mm;
  x[2] = kn;
  x[3] = nn;
}

// Column segments of the k sums: DNK planes per thread, over the nks
// distinct planes (nk - 1 along a superposed k direction, whose last plane
// is its first one's place).
constexpr int DNK = 16;
inline int dyn_nseg(int nks) { return (nks + DNK - 1) / DNK; }

// Xp[q][seg][j][i] = sum over k of segment seg (ascending) of contraction q
// at the interior nodes of column (i, j).
__global__ void __launch_bounds__(256) k_dyn_node(Layout L, int nks, int nseg, int axis, const double* __restrict__ M,
                                                  const double* __restrict__ V, double* __restrict__ Xp) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncoli = (long long)L.ni * L.nj;
  if (t >= ncoli * nseg) return;
  const long long col = t % ncoli;
  const int seg = (int)(t / ncoli);
  const int i = (int)(col % L.ni), j = (int)(col / L.ni);
  // (no contractions on the polar axis: its column takes the ring j = 1's)
  const int k1 = (axis && j == 0) ? 0 : ((seg + 1) * DNK < nks ? (seg + 1) * DNK : nks);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = seg * DNK; k < k1; ++k) {
    double x[4];
    dyn_contract(L, M, V, i, j, k, x);
    for (int q = 0; q < 4; ++q) s[q] += x[q];
  }
  for (int q = 0; q < 4; ++q) Xp[((long long)q * nseg + seg) * ncoli + col] = s[q];
}

__device__ inline int dyn_src(int x, int n, int bc) {
  if (bc == 3) {
    // polar axis (j): column -m across the axis is ring column m, the axis
    // column takes ring 1's, the far side is Dirichlet
    const int y = x < 0 ? -x : (x < n ? x : n - 1);
    return y == 0 ? 1 : y;
  }
  if (x >= 0 && x < n) return x;
  if (bc == 1) return x < 0 ? 0 : n - 1;  // Dirichlet: nearest interior column
  const int p = bc == 2 ? n - 1 : n;      // periodic (superposed: period n - 1)
  return ((x % p) + p) % p;
}

// per padded column: the segment sums of its source column added in
// ascending segment order, then the clipped ratios
__global__ void __launch_bounds__(256) k_dyn_coef(Layout L, int bc0, int bc1, int nseg, const double* __restrict__ Xp,
                                                  double* __restrict__ dyn) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ncol = dyn_ncol(L);
  if (c >= ncol) return;
  const int i = (int)(c % (L.ni + 4)) - 2, j = (int)(c / (L.ni + 4)) - 2;
  const int is = dyn_src(i, L.ni, bc0), js = dyn_src(j, L.nj, bc1);
  const long long ncoli = (long long)L.ni * L.nj, col = (long long)js * L.ni + is;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = 0; g < nseg; ++g)
    for (int q = 0; q < 4; ++q) s[q] += Xp[((long long)q * nseg + g) * ncoli + col];
  dyn[c] = s[1] > 0.0 ? fmax(0.0, s[0] / s[1]) : 0.0;
  dyn[ncol + c] = s[3] > 0.0 ? fmax(0.0, s[2] / s[3]) : 0.0;
}

inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

template <class QI>
hipError_t run(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M, const QI* Q,
               double* work, double* dyn) {
  double* V = work;
  double* X = work + (long long)NRAW * L.fe;
  const int axis = bc[1] == 3;
  const int nks = bc[2] == 2 ? L.nk - 1 : L.nk;
  k_dyn_plane<QI><<<(unsigned)dyn_plane_blocks(L), DPX * DPY, 0, s>>>(L, P, axis, M, Q, V);
  const int nseg = dyn_nseg(nks);
  k_dyn_node<<<nblk((long long)L.ni * L.nj * nseg, 256), 256, 0, s>>>(L, nks, nseg, axis, M, V, X);
  k_dyn_coef<<<nblk(dyn_ncol(L), 256), 256, 0, s>>>(L, bc[0], bc[1], nseg, X, dyn);
  return hipGetLastError();
}

}  // namespace

long long dynamic_work_elems(const Layout& L) { return (NRAW + 4LL) * L.fe; }

hipError_t launch_dynamic(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M,
                          const double* Q, double* work, double* dyn) {
  return run<double>(s, L, bc, P, M, Q, work, dyn);
}

hipError_t launch_dynamic_f32(hipStream_t s, const Layout& L, const int bc[3], const Phys& P, const double* M,
                              const float* Q, double* work, double* dyn) {
  return run<float>(s, L, bc, P, M, Q, work, dyn);
}

}  // namespace les
