// les_kernels.hip -- setup, boundary, reduction and reference-residual kernels.
//
// * k_metrics: Jacobian and metric terms (Alg. 2, "Calc(Jacob., Metric)")
//   in the conservative central-difference form.
// * k_ghost_fill: two ghost layers (Sec. 4, Fig. 3): periodic wrap (Sec. 3,
//   azimuthal periodicity; period n - 1 where the first and last nodes are
//   superposed), frozen Dirichlet values, or the entrance / far field / exit
//   conditions of a boundary face (Sec. 3).
// * k_cfl_partial / k_cfl_final: global CFL time step (FP64 min reduction).
// * k_residual_ref / k_stage_ref: one thread per interior node evaluating the
//   residual (Eq. 12-15 with Turkel-Vatsa dissipation) directly from global
//   memory, recomputing every neighbour quantity.  It is the simple,
//   structure-independent GPU formulation used by les_residual and to
//   cross-check the fused stage kernel.
// * k_norm_final: RMS / max norms of R from per-block partials (FP64).
// * k_probe: pressure-fluctuation objective on a plane and its gradient.
// * k_stats: running sums of the primitives and their second moments over
//   the periodic k direction (mean-flow and RMS profiles).
#include "les_common.hpp"
#include "les_launch.hpp"

namespace les {

// ---------------------------------------------------------------------------
// Metrics: m[0..8] = xi_x/J .. zeta_z/J, m[9] = J on nodes in [-1, n]^3.
// ---------------------------------------------------------------------------
__global__ void k_metrics(Layout L, Dense D, int bc0, int bc1, int bc2, const double* __restrict__ xyz,
                          double* __restrict__ M) {
  const int ext_i = L.ni + 2, ext_j = L.nj + 2;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = (long long)ext_i * ext_j * (L.nk + 2);
  if (t >= tot) return;
  int i = (int)(t % ext_i) - 1;
  int j = (int)((t / ext_i) % ext_j) - 1;
  int k = (int)(t / ((long long)ext_i * ext_j)) - 1;
  // a periodic ghost takes the metrics of its wrapped interior node; along a
  // superposed direction (period n - 1) node n - 1 takes node 0's
  int id[3] = {i, j, k};
  const int nn[3] = {L.ni, L.nj, L.nk};
  const int bc[3] = {bc0, bc1, bc2};
  for (int d = 0; d < 3; ++d) {
    if (bc[d] == 0) id[d] = (id[d] + nn[d]) % nn[d];
    if (bc[d] == 2) id[d] = (id[d] + nn[d] - 1) % (nn[d] - 1);
  }
  const long long N = D.n();
  auto X = [&](int c, int a, int b, int e) { return xyz[c * N + D.at(a, b, e)]; };
  // central difference of coordinate c along direction d at node (a, b, e)
  auto dX = [&](int c, int d, int a, int b, int e) {
    int da = d == 0, db = d == 1, de = d == 2;
    return 0.5 * (X(c, a + da, b + db, e + de) - X(c, a - da, b - db, e - de));
  };
  const long long out = L.at(i, j, k);
  for (int a = 0; a < 3; ++a) {
    int bd = (a + 1) % 3, cd = (a + 2) % 3;
    int bi = bd == 0, bj = bd == 1, bk = bd == 2;
    int ci = cd == 0, cj = cd == 1, ck = cd == 2;
    for (int l = 0; l < 3; ++l) {
      int l1 = (l + 1) % 3, l2 = (l + 2) % 3;
      double t1 = 0.5 * (dX(l1, bd, id[0] + ci, id[1] + cj, id[2] + ck) * X(l2, id[0] + ci, id[1] + cj, id[2] + ck) -
                         dX(l1, bd, id[0] - ci, id[1] - cj, id[2] - ck) * X(l2, id[0] - ci, id[1] - cj, id[2] - ck));
      double t2 = 0.5 * (dX(l1, cd, id[0] + bi, id[1] + bj, id[2] + bk) * X(l2, id[0] + bi, id[1] + bj, id[2] + bk) -
                         dX(l1, cd, id[0] - bi, id[1] - bj, id[2] - bk) * X(l2, id[0] - bi, id[1] - bj, id[2] - bk));
      M[(3 * a + l) * L.fe + out] = t1 - t2;
    }
  }
  double a11 = dX(0, 0, id[0], id[1], id[2]), a12 = dX(0, 1, id[0], id[1], id[2]), a13 = dX(0, 2, id[0], id[1], id[2]);
  double a21 = dX(1, 0, id[0], id[1], id[2]), a22 = dX(1, 1, id[0], id[1], id[2]), a23 = dX(1, 2, id[0], id[1], id[2]);
  double a31 = dX(2, 0, id[0], id[1], id[2]), a32 = dX(2, 1, id[0], id[1], id[2]), a33 = dX(2, 2, id[0], id[1], id[2]);
  double vol = a11 * (a22 * a33 - a23 * a32) - a12 * (a21 * a33 - a23 * a31) + a13 * (a21 * a32 - a22 * a31);
  M[9 * L.fe + out] = 1.0 / vol;
}

// Copy caller metrics (dense) into the library layout on [-1, n]^3.
__global__ void k_metrics_copy(Layout L, Dense D, const double* __restrict__ src, double* __restrict__ M) {
  const int ext_i = L.ni + 2, ext_j = L.nj + 2;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = (long long)ext_i * ext_j * (L.nk + 2);
  if (t >= tot) return;
  int i = (int)(t % ext_i) - 1;
  int j = (int)((t / ext_i) % ext_j) - 1;
  int k = (int)(t / ((long long)ext_i * ext_j)) - 1;
  for (int c = 0; c < 10; ++c) M[c * L.fe + L.at(i, j, k)] = src[c * D.n() + D.at(i, j, k)];
}

// Library metrics -> dense array (nodes outside [-1, n]^3 are zero).
__global__ void k_metrics_export(Layout L, Dense D, const double* __restrict__ M, double* __restrict__ dst) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= D.n()) return;
  int pi = L.ni + 4, pj = L.nj + 4;
  int i = (int)(t % pi) - 2;
  int j = (int)((t / pi) % pj) - 2;
  int k = (int)(t / ((long long)pi * pj)) - 2;
  bool ok = i >= -1 && i <= L.ni && j >= -1 && j <= L.nj && k >= -1 && k <= L.nk;
  for (int c = 0; c < 10; ++c) dst[c * D.n() + t] = ok ? M[c * L.fe + L.at(i, j, k)] : 0.0;
}

// ---------------------------------------------------------------------------
// Boundary faces (Sec. 3: entrance, far field and exit of the jet domain).
// A ghost node outside the interior along exactly one Dirichlet direction
// d, on a face whose type is not frozen, takes face_value (les_faces.hpp) of
// the boundary node r next to the face on its line along d (periodic indices
// wrapped; the same r for both ghost layers: zero-order extrapolation) and,
// for the characteristic type, of the outside state stored at the ghost
// node.  Ghosts of two Dirichlet directions (edges) stay frozen.  Computed
// in FP64 whatever the storage type of the state.
// ---------------------------------------------------------------------------
// The face rule at ghost node dst of the state q (storage type T).  Returns
// false when the node is not a face ghost (ghost along zero or several
// Dirichlet directions, or a frozen face).
template <class T>
__device__ bool face_ghost(const Layout& L, const Faces& F, const int bc[3], const int id[3], const int w[3],
                           long long dst, T* q) {
  const int nn[3] = {L.ni, L.nj, L.nk};
  // below the polar axis a ghost of a Dirichlet i side is an edge of two
  // boundary directions: it keeps its given value
  if (bc[1] == 3 && id[1] < 0) return false;
  int nd = 0, d = 0;
  for (int e = 0; e < 3; ++e)
    if ((bc[e] == 1 && (id[e] < 0 || id[e] >= nn[e])) || (bc[e] == 3 && id[e] >= nn[e])) {
      ++nd;
      d = e;
    }
  if (nd != 1) return false;
  const int hi = id[d] >= nn[d] ? 1 : 0;
  const int type = F.type[2 * d + hi];
  if (type == 0) return false;
  int r[3] = {w[0], w[1], w[2]};
  r[d] = hi ? nn[d] - 1 : 0;
  const long long rn = L.at(r[0], r[1], r[2]);
  double nv[3];
  face_normal(L, F, d, hi, r[0], r[1], r[2], nv);
  double qr[5], qo[5] = {0, 0, 0, 0, 0}, out[5];
  for (int c = 0; c < 5; ++c) {
    qr[c] = (double)q[c * L.fe + rn];
    if (F.outside) qo[c] = F.outside[c * L.fe + dst];
  }
  face_value<double>(type, F.gamma, F.p_exit[2 * d + hi], nv, qr, qo, out);
  for (int c = 0; c < 5; ++c) q[c * L.fe + dst] = (T)out[c];
  return true;
}

// Source of ghost node id: dir = true for a node outside a Dirichlet side
// (frozen or a face rule; bc 3 is Dirichlet at j-hi); otherwise w = the node
// whose value it copies: periodic indices wrapped (period n, or n - 1 when
// superposed), and across the polar axis (bc 3 at j-lo) the node
// diametrically opposite, (i, -j, k + (nk - 1)/2), with i and k wrapped into
// the interior (so the source is never a node the fill writes).
__device__ inline void ghost_source(const int nn[3], const int bc[3], const int id[3], int w[3], bool& dir) {
  dir = false;
  for (int d = 0; d < 3; ++d) {
    const bool g = id[d] < 0 || id[d] >= nn[d];
    if (g && (bc[d] == 1 || (bc[d] == 3 && id[d] >= nn[d]))) dir = true;
    w[d] = (g && bc[d] == 0) ? (id[d] + nn[d]) % nn[d]
         : (g && bc[d] == 2) ? (id[d] + nn[d] - 1) % (nn[d] - 1) : id[d];
  }
  if (bc[1] == 3 && id[1] < 0 && !dir) {
    const int p = nn[2] - 1;
    w[1] = -id[1];
    w[2] = (w[2] + p / 2) % p;
  }
}

// ---------------------------------------------------------------------------
// Ghost fill.  Threads enumerate only the ghost shell: the k-ghost slabs
// (full i, j extent), then the j-ghost slabs inside interior k, then the
// i-ghost columns inside interior j, k.  A node that is a ghost in a
// Dirichlet direction copies its frozen value from `frozen` (nothing to do
// when frozen == q); any other ghost copies the interior node obtained by
// wrapping its periodic indices.  Sources are always interior nodes or the
// frozen array, never a node this kernel writes.
// ---------------------------------------------------------------------------
__global__ void k_ghost_fill(Layout L, int bc0, int bc1, int bc2, double* q, const double* frozen, int nf, Faces F) {
  const int PI = L.ni + 4, PJ = L.nj + 4;
  const long long cA = 4LL * PJ * PI;
  const long long cB = (long long)L.nk * 4 * PI;
  const long long cC = (long long)L.nk * L.nj * 4;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t < cA) {
    int kk = (int)(t / ((long long)PJ * PI));
    long long r = t % ((long long)PJ * PI);
    k = kk < 2 ? kk - 2 : L.nk + kk - 2;
    j = (int)(r / PI) - 2;
    i = (int)(r % PI) - 2;
  } else if (t < cA + cB) {
    long long u = t - cA;
    k = (int)(u / (4LL * PI));
    long long r = u % (4LL * PI);
    int jj = (int)(r / PI);
    j = jj < 2 ? jj - 2 : L.nj + jj - 2;
    i = (int)(r % PI) - 2;
  } else if (t < cA + cB + cC) {
    long long u = t - cA - cB;
    k = (int)(u / (4LL * L.nj));
    long long r = u % (4LL * L.nj);
    j = (int)(r / 4);
    int ii = (int)(r % 4);
    i = ii < 2 ? ii - 2 : L.ni + ii - 2;
  } else {
    return;
  }
  const int id[3] = {i, j, k};
  const int nn[3] = {L.ni, L.nj, L.nk};
  const int bc[3] = {bc0, bc1, bc2};
  bool dir;
  int w[3];
  ghost_source(nn, bc, id, w, dir);
  const long long dst = L.at(i, j, k);
  if (dir) {
    if (F.any && nf == 5 && face_ghost(L, F, bc, id, w, dst, q)) return;
    if (frozen != q)
      for (int f = 0; f < nf; ++f) q[f * L.fe + dst] = frozen[f * L.fe + dst];
    return;
  }
  const long long src = L.at(w[0], w[1], w[2]);
  for (int f = 0; f < nf; ++f) q[f * L.fe + dst] = q[f * L.fe + src];
}

// FP32 stage state: same shell enumeration; Dirichlet ghosts take the
// rounded frozen FP64 values, periodic ghosts wrap.
__global__ void k_ghost_fill_f32(Layout L, int bc0, int bc1, int bc2, float* __restrict__ q,
                                 const double* __restrict__ frozen, Faces F) {
  const int PI = L.ni + 4, PJ = L.nj + 4;
  const long long cA = 4LL * PJ * PI;
  const long long cB = (long long)L.nk * 4 * PI;
  const long long cC = (long long)L.nk * L.nj * 4;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (t < cA) {
    int kk = (int)(t / ((long long)PJ * PI));
    long long r = t % ((long long)PJ * PI);
    k = kk < 2 ? kk - 2 : L.nk + kk - 2;
    j = (int)(r / PI) - 2;
    i = (int)(r % PI) - 2;
  } else if (t < cA + cB) {
    long long u = t - cA;
    k = (int)(u / (4LL * PI));
    long long r = u % (4LL * PI);
    int jj = (int)(r / PI);
    j = jj < 2 ? jj - 2 : L.nj + jj - 2;
    i = (int)(r % PI) - 2;
  } else if (t < cA + cB + cC) {
    long long u = t - cA - cB;
    k = (int)(u / (4LL * L.nj));
    long long r = u % (4LL * L.nj);
    j = (int)(r / 4);
    int ii = (int)(r % 4);
    i = ii < 2 ? ii - 2 : L.ni + ii - 2;
  } else {
    return;
  }
  const int id[3] = {i, j, k};
  const int nn[3] = {L.ni, L.nj, L.nk};
  const int bc[3] = {bc0, bc1, bc2};
  bool dir;
  int w[3];
  ghost_source(nn, bc, id, w, dir);
  const long long dst = L.at(i, j, k);
  if (dir) {
    if (F.any && face_ghost(L, F, bc, id, w, dst, q)) return;
    for (int f = 0; f < 5; ++f) q[f * L.fe + dst] = (float)frozen[f * L.fe + dst];
    return;
  }
  const long long src = L.at(w[0], w[1], w[2]);
  for (int f = 0; f < 5; ++f) q[f * L.fe + dst] = q[f * L.fe + src];
}

// ---------------------------------------------------------------------------
// Centerline of the O-grid (Sec. 3): every axis node (i, 0, k) takes, per
// conserved variable, the mean of the ring (i, 1, k'), k' = 0 .. nk - 2 (the
// distinct azimuths; zero-order extrapolation from the adjacent ring, then
// the azimuthal average).  One wave per (i, variable): lane l sums k' = l,
// l + 64, ... in ascending order in FP64, the 64 partial sums are added by a
// fixed shuffle tree, and the lanes write the axis nodes.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(64) k_axis_avg(Layout L, T* __restrict__ q) {
  const int f = blockIdx.x / L.ni, i = blockIdx.x % L.ni;
  T* a = q + f * L.fe;
  double sum = 0.0;
  for (int k = threadIdx.x; k < L.nk - 1; k += 64) sum += (double)a[L.at(i, 1, k)];
  sum = __shfl(wave_sum(sum), 0, 64);
  const T mean = (T)(sum / (double)(L.nk - 1));
  for (int k = threadIdx.x; k < L.nk; k += 64) a[L.at(i, 0, k)] = mean;
}

// ---------------------------------------------------------------------------
// CFL time step: per-block minima, then one block of 1024 threads for the
// global minimum.  A block covers 64 columns of 4 rows in kc consecutive
// planes.  Its columns are a 64-element chunk of the row storage (chunks
// start at the 128-byte-aligned row start, so node i sits in column
// i + LEAD): every row segment is four whole 128-byte lines.  kc = 1 (many
// small blocks keep the most loads in flight) unless that would leave more
// than CFL_PARTS partials for the final block.  NaN wins every comparison,
// so that a non-physical state is reported.
// ---------------------------------------------------------------------------
constexpr long long CFL_PARTS = 65536;

__global__ void __launch_bounds__(256) k_cfl_partial(Layout L, Phys P, const double* __restrict__ M,
                                                     const double* __restrict__ Q, int kc, int jlo,
                                                     double* __restrict__ part) {
  __shared__ double red[4];
  const int i = blockIdx.x * 64 + threadIdx.x - LEAD;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k0 = blockIdx.z * kc, k1 = min(L.nk, k0 + kc);
  double loc = INFINITY;
  // (rows j < jlo are skipped: the polar axis, whose nodes the residual does not advance)
  for (int k = k0; k < k1 && i >= 0 && i < L.ni && j >= jlo && j < L.nj; ++k) {
    long long n = L.at(i, j, k);
    double m9[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) m9[c] = M[c * L.fe + n];
    loc = min_nan(loc, cfl_local(Q[n], Q[L.fe + n], Q[2 * L.fe + n], Q[3 * L.fe + n], Q[4 * L.fe + n],
                                 M[9 * L.fe + n], m9, P));
  }
  loc = wave_min(loc);
  const int tid = threadIdx.y * 64 + threadIdx.x;
  if ((tid & 63) == 0) red[tid >> 6] = loc;
  __syncthreads();
  if (tid == 0) {
    double m = red[0];
    for (int a = 1; a < 4; ++a) m = min_nan(m, red[a]);
    part[((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = m;
  }
}

// *dt_out = dt (and *also = dt when also is not null); flag |= 1 when the
// minimum is not a positive finite number.
__global__ void __launch_bounds__(1024) k_cfl_final(const double* __restrict__ part, long long np, double cfl,
                                                    double* __restrict__ dt_out, double* __restrict__ also,
                                                    int* __restrict__ flag) {
  __shared__ double red[16];
  double m = INFINITY;
#pragma unroll 8
  for (long long b = threadIdx.x; b < np; b += 1024) m = min_nan(m, part[b]);
  m = wave_min(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int a = 1; a < 16; ++a) r = min_nan(r, red[a]);
    double dt = cfl * r;
    if (!(dt > 0.0) || !(dt < INFINITY)) *flag |= 1;
    *dt_out = dt;
    if (also) *also = dt;
  }
}

// ---------------------------------------------------------------------------
// Reference residual: one thread per interior node, every neighbour
// quantity recomputed from global memory.
// ---------------------------------------------------------------------------
struct RefArgs {
  Layout L;
  Phys P;
  const double* M;
  const double* Q;
  const double* dyn;  // per-column dynamic SGS coefficients (P.sgs == 2)
  int axis;           // j = 0 is the polar axis
};

// j index of a node given by its element offset
__device__ inline int ref_j(const Layout& L, long long n) {
  const long long t = n - L.at(-2, -2, -2);
  return (int)((t % L.sk) / L.sj) - 2;
}

// dynamic-coefficient column (dyn_col) of a node given by its element offset
__device__ inline long long ref_col(const Layout& L, long long n) {
  const long long t = n - L.at(-2, -2, -2);
  const long long r = t % L.sk;
  return (r / L.sj) * (L.ni + 4) + (r % L.sj);
}

__device__ inline void ref_prim(const RefArgs& A, long long n, double& rho, double& u, double& v, double& w,
                                double& p, double& tem) {
  const long long fe = A.L.fe;
  rho = A.Q[n];
  prim_from_q(rho, A.Q[fe + n], A.Q[2 * fe + n], A.Q[3 * fe + n], A.Q[4 * fe + n], A.P, u, v, w, p, tem);
}

__device__ inline long long dstride(const Layout& L, int d) { return d == 0 ? 1LL : (d == 1 ? L.sj : L.sk); }

// Node flux H_d = inviscid - viscous (Eq. 15) at node n.
__device__ void ref_node_flux(const RefArgs& A, int d, long long n, double H[5]) {
  const Layout& L = A.L;
  if (A.axis && ref_j(L, n) == 0) {  // on the axis: the limit (xi/J = eta/J = 0)
    for (int q = 0; q < 5; ++q) H[q] = 0.0;
    return;
  }
  const Phys& P = A.P;
  const long long fe = L.fe;
  double rho, u, v, w, p, tem;
  ref_prim(A, n, rho, u, v, w, p, tem);
  // gradients of u, v, w, T along the index directions
  double dd[3][4];
  for (int e = 0; e < 3; ++e) {
    long long s = dstride(L, e);
    double r1, u1, v1, w1, p1, t1, r0, u0, v0, w0, p0, t0;
    ref_prim(A, n + s, r1, u1, v1, w1, p1, t1);
    ref_prim(A, n - s, r0, u0, v0, w0, p0, t0);
    dd[e][0] = 0.5 * (u1 - u0);
    dd[e][1] = 0.5 * (v1 - v0);
    dd[e][2] = 0.5 * (w1 - w0);
    dd[e][3] = 0.5 * (t1 - t0);
  }
  const double J = A.M[9 * fe + n];
  double m[9];
  for (int c = 0; c < 9; ++c) m[c] = A.M[c * fe + n];
  double g[4][3];  // g[q][x] = d phi_q / d x
  for (int q = 0; q < 4; ++q)
    for (int x = 0; x < 3; ++x) g[q][x] = J * (m[x] * dd[0][q] + m[3 + x] * dd[1][q] + m[6 + x] * dd[2][q]);
  double S[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S[a][b] = 0.5 * (g[a][b] + g[b][a]);
  double skk = S[0][0] + S[1][1] + S[2][2];
  double mu = sutherland(tem, P);
  double mus = 0.0, kaps = 0.0, pis = 0.0;
  if (P.sgs) {
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) ss += S[a][b] * S[a][b];
    double delta2 = cbrt(1.0 / J);
    delta2 *= delta2;
    const double rd = rho * delta2 * sqrt(2.0 * ss);
    if (P.sgs == 1) {
      mus = P.Cs2 * rd;
      kaps = mus * P.Cp_over_Prsgs;
    } else {
      const long long c = ref_col(L, n);
      mus = A.dyn[c] * rd;
      kaps = P.Cp * A.dyn[dyn_ncol(L) + c] * rd;
    }
    pis = P.CI43 * rho * delta2 * ss;  // sigma_kk / 3
  }
  const double mt2 = 2.0 * (mu + mus);
  double tau[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) tau[a][b] = mt2 * (S[a][b] - (a == b ? skk / 3.0 : 0.0));
  const double kap = mu * P.Cp_over_Pr + kaps;
  const double uu[3] = {u, v, w};
  double th[3];
  for (int x = 0; x < 3; ++x) th[x] = uu[0] * tau[0][x] + uu[1] * tau[1][x] + uu[2] * tau[2][x] + kap * g[3][x];
  const double mx = m[3 * d], my = m[3 * d + 1], mz = m[3 * d + 2];
  const double U = mx * u + my * v + mz * w;
  const double pe = p + pis;  // the isotropic SGS stress enters like a pressure
  H[0] = rho * U;
  H[1] = rho * u * U + mx * pe - (mx * tau[0][0] + my * tau[0][1] + mz * tau[0][2]);
  H[2] = rho * v * U + my * pe - (mx * tau[1][0] + my * tau[1][1] + mz * tau[1][2]);
  H[3] = rho * w * U + mz * pe - (mx * tau[2][0] + my * tau[2][1] + mz * tau[2][2]);
  H[4] = (A.Q[4 * fe + n] + pe) * U - (mx * th[0] + my * th[1] + mz * th[2]);
}

// Lambda_d (anisotropic spectral radius) and pressure at node n.
__device__ double ref_Lambda(const RefArgs& A, int d, long long n) {
  const long long fe = A.L.fe;
  if (A.axis && ref_j(A.L, n) == 0) return 0.0;  // lam_eta = 0 on the axis
  double rho, u, v, w, p, tem;
  ref_prim(A, n, rho, u, v, w, p, tem);
  double c = sqrt(A.P.gamma * p / rho);
  double lam[3];
  for (int e = 0; e < 3; ++e) {
    double mx = A.M[(3 * e) * fe + n], my = A.M[(3 * e + 1) * fe + n], mz = A.M[(3 * e + 2) * fe + n];
    lam[e] = fabs(mx * u + my * v + mz * w) + c * sqrt(mx * mx + my * my + mz * mz);
  }
  return aniso(lam[d], lam[(d + 1) % 3], lam[(d + 2) % 3], A.P);
}

__device__ inline double ref_p(const RefArgs& A, long long n) {
  double rho, u, v, w, p, tem;
  ref_prim(A, n, rho, u, v, w, p, tem);
  return p;
}

// Dissipation flux at the face between a and a + e_d.
__device__ void ref_face_diss(const RefArgs& A, int d, long long a, double D[5]) {
  const long long s = dstride(A.L, d), fe = A.L.fe;
  const double pm = ref_p(A, a - s), p0 = ref_p(A, a), p1 = ref_p(A, a + s), p2 = ref_p(A, a + 2 * s);
  const double nua = fabs(p1 - 2.0 * p0 + pm) / (p1 + 2.0 * p0 + pm);
  const double nub = fabs(p2 - 2.0 * p1 + p0) / (p2 + 2.0 * p1 + p0);
  const double e2 = A.P.k2 * tmax(nua, nub);
  const double e4 = tmax(0.0, A.P.k4 - e2);
  const double Lf = 0.5 * (ref_Lambda(A, d, a) + ref_Lambda(A, d, a + s));
  // the face between the axis and j = 1: cross-axis value by linear extrapolation
  const bool axf = A.axis && d == 1 && ref_j(A.L, a) == 0;
  for (int q = 0; q < 5; ++q) {
    const double* Qq = A.Q + q * fe;
    double d1 = Qq[a + s] - Qq[a];
    double d3 = axf ? Qq[a + 2 * s] - 2.0 * Qq[a + s] + Qq[a]
                    : Qq[a + 2 * s] - 3.0 * Qq[a + s] + 3.0 * Qq[a] - Qq[a - s];
    D[q] = Lf * (e2 * d1 - e4 * d3);
  }
}

__device__ void ref_residual(const RefArgs& A, int i, int j, int k, const double* f, int i_f, double R[5]) {
  const long long n = A.L.at(i, j, k);
  if (A.axis && j == 0) {  // the axis follows the centerline condition
    for (int q = 0; q < 5; ++q) R[q] = 0.0;
    return;
  }
  double acc[5] = {0, 0, 0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    const long long s = dstride(A.L, d);
    double Hp[5], Hm[5], Dp[5], Dm[5];
    ref_node_flux(A, d, n + s, Hp);
    ref_node_flux(A, d, n - s, Hm);
    ref_face_diss(A, d, n, Dp);
    ref_face_diss(A, d, n - s, Dm);
    for (int q = 0; q < 5; ++q) acc[q] += 0.5 * (Hp[q] - Hm[q]) - (Dp[q] - Dm[q]);
  }
  const double J = A.M[9 * A.L.fe + n];
  for (int q = 0; q < 5; ++q) {
    R[q] = J * acc[q];
    if (f && i == i_f) R[q] -= f[((long long)q * A.L.nk + k) * A.L.nj + j];
  }
}

// Per-block partial norms: part[b*10 + q] = sum R_q^2, part[b*10 + 5 + q] = max |R_q|.
__device__ inline void block_norms(const double R[5], bool active, double* part, long long bid) {
  __shared__ double red[4][10];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  for (int q = 0; q < 5; ++q) {
    double s = active ? R[q] * R[q] : 0.0;
    double m = active ? fabs(R[q]) : 0.0;
    s = wave_sum(s);
    m = wave_max(m);
    if ((tid & 63) == 0) {
      red[tid >> 6][q] = s;
      red[tid >> 6][5 + q] = m;
    }
  }
  __syncthreads();
  if (tid < 10) {
    double v = red[0][tid];
    const int nw = (blockDim.x * blockDim.y) >> 6;
    for (int a = 1; a < nw; ++a) {
      double o = red[a][tid];
      v = tid < 5 ? v + o : ((o > v || o != o) ? o : v);
    }
    part[bid * 10 + tid] = v;
  }
}

__global__ void __launch_bounds__(256) k_residual_ref(RefArgs A, const double* __restrict__ f, int i_f,
                                                      double* __restrict__ R, double* __restrict__ part) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  const bool active = i < A.L.ni && j < A.L.nj;
  double r[5] = {0, 0, 0, 0, 0};
  if (active) {
    ref_residual(A, i, j, k, f, i_f, r);
    const long long n = A.L.at(i, j, k);
    for (int q = 0; q < 5; ++q) R[q * A.L.fe + n] = r[q];
  }
  if (part) block_norms(r, active, part, ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
}

// Q_out = Q0 - alpha dt R(Q_in) on the interior.
// Q0 and Qout may be the same array (last stage): each thread reads Q0 at
// its own node before writing Qout there, and the stencil reads only A.Q.
__global__ void __launch_bounds__(256) k_stage_ref(RefArgs A, const double* Q0, double* Qout,
                                                   const double* __restrict__ dtp, double dt_host, double alpha, const double* __restrict__ f, int i_f,
                                                   double* __restrict__ part) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  const bool active = i < A.L.ni && j < A.L.nj;
  double r[5] = {0, 0, 0, 0, 0};
  if (active) {
    ref_residual(A, i, j, k, f, i_f, r);
    const long long n = A.L.at(i, j, k);
    const double c = alpha * (dtp ? dtp[0] : dt_host);
    for (int q = 0; q < 5; ++q) Qout[q * A.L.fe + n] = Q0[q * A.L.fe + n] - c * r[q];
  }
  if (part) block_norms(r, active, part, ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
}

// norms[q] = sqrt(sum/N), norms[5+q] = max; flag |= 2 if any is not finite.
__global__ void __launch_bounds__(256) k_norm_final(const double* __restrict__ part, long long np, double count,
                                                    double* __restrict__ norms, int* __restrict__ flag) {
  __shared__ double red[4][10];
  double acc[10];
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (long long b = threadIdx.x; b < np; b += 256)
    for (int q = 0; q < 10; ++q) {
      double v = part[b * 10 + q];
      acc[q] = q < 5 ? acc[q] + v : ((v > acc[q] || v != v) ? v : acc[q]);
    }
  for (int q = 0; q < 10; ++q) {
    double v = q < 5 ? wave_sum(acc[q]) : wave_max(acc[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int q = threadIdx.x;
    double v = red[0][q];
    for (int a = 1; a < 4; ++a) v = q < 5 ? v + red[a][q] : ((red[a][q] > v || red[a][q] != red[a][q]) ? red[a][q] : v);
    double out = q < 5 ? sqrt(v / count) : v;
    norms[q] = out;
    if (!(out < INFINITY)) atomicOr(flag, 2);
  }
}

// ---------------------------------------------------------------------------
// Probe objective on plane i_p: one block; J += w sum (p - p_inf)^2 and
// Qbar += w 2 (p - p_inf) dp/dQ.
// ---------------------------------------------------------------------------
// Pass 1: every block sums its share of the plane into part[blockIdx.x]
// (and adds the objective's Q adjoint, node by node); pass 2 adds the block
// sums in a fixed order, so that the objective does not depend on timing.
__global__ void __launch_bounds__(256) k_probe(Layout L, Phys P, int nks, const double* __restrict__ Q, int i_p,
                                               double p_inf, double weight, double* __restrict__ part,
                                               double* __restrict__ Qbar) {
  __shared__ double red[4];
  double s = 0.0;
  const long long cnt = (long long)L.nj * nks;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < cnt; t += (long long)gridDim.x * 256) {
    int j = (int)(t % L.nj), k = (int)(t / L.nj);
    long long n = L.at(i_p, j, k);
    double rho = Q[n], m1 = Q[L.fe + n], m2 = Q[2 * L.fe + n], m3 = Q[3 * L.fe + n], e = Q[4 * L.fe + n];
    double u = m1 / rho, v = m2 / rho, w = m3 / rho;
    double p = P.gm1 * (e - 0.5 * rho * (u * u + v * v + w * w));
    double dp = p - p_inf;
    s += dp * dp;
    if (Qbar) {
      double g = weight * 2.0 * dp * P.gm1;
      Qbar[n] += g * 0.5 * (u * u + v * v + w * w);
      Qbar[L.fe + n] -= g * u;
      Qbar[2 * L.fe + n] -= g * v;
      Qbar[3 * L.fe + n] -= g * w;
      Qbar[4 * L.fe + n] += g;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(64) k_probe_final(const double* __restrict__ part, int nparts, double weight,
                                                    double* __restrict__ Jacc) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 64) s += part[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) Jacc[0] += weight * s;
}

}  // namespace les

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace les {

// ---------------------------------------------------------------------------
// Running flow statistics (Sec. 6: time- and azimuth-averaged mean-flow and
// RMS profiles; the periodic k direction is the averaged one):
//   acc[s][j][i] += sum over k = 0..nks-1 of phi_s(i, j, k),
//   phi = (rho, u, v, w, p, uu, vv, ww, uv, uw, vw, pp),
// nks = the distinct k planes (nk, or nk - 1 along a superposed direction).
// A block of 64 x 4 threads covers 64 nodes of one row j; thread (x, y) sums
// the y-th of four contiguous k ranges in ascending k, and the four partial
// sums are added in a fixed order, so repeated runs give identical sums.
// ---------------------------------------------------------------------------
constexpr int STATS_NF = 12;

__global__ void __launch_bounds__(256) k_stats(Layout L, Phys P, int nks, const double* __restrict__ Q,
                                               double* __restrict__ acc) {
  __shared__ double red[3][STATS_NF][64];
  const int x = threadIdx.x, y = threadIdx.y;
  const int i = blockIdx.x * 64 + x, j = blockIdx.y;
  const int kper = (nks + 3) / 4;
  const int k0 = y * kper, k1 = min(nks, k0 + kper);
  double s[STATS_NF];
#pragma unroll
  for (int f = 0; f < STATS_NF; ++f) s[f] = 0.0;
  if (i < L.ni) {
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
      const long long n = L.at(i, j, k);
      const double rho = Q[n];
      double u, v, w, p, tem;
      prim_from_q(rho, Q[L.fe + n], Q[2 * L.fe + n], Q[3 * L.fe + n], Q[4 * L.fe + n], P, u, v, w, p, tem);
      s[0] += rho;
      s[1] += u;
      s[2] += v;
      s[3] += w;
      s[4] += p;
      s[5] += u * u;
      s[6] += v * v;
      s[7] += w * w;
      s[8] += u * v;
      s[9] += u * w;
      s[10] += v * w;
      s[11] += p * p;
    }
  }
  if (y > 0)
#pragma unroll
    for (int f = 0; f < STATS_NF; ++f) red[y - 1][f][x] = s[f];
  __syncthreads();
  if (y == 0 && i < L.ni) {
    const long long plane = (long long)L.ni * L.nj;
#pragma unroll
    for (int f = 0; f < STATS_NF; ++f)
      acc[f * plane + (long long)j * L.ni + i] += ((s[f] + red[0][f][x]) + red[1][f][x]) + red[2][f][x];
  }
}

// Mean-flow and RMS profiles from the running sums: one thread per (i, j).
// prof = (<rho>, <u>, <v>, <w>, <p>, u_rms, v_rms, w_rms, p_rms, <u'v'>) with
// <phi> = acc / samples and rms = sqrt(max(0, <phi phi> - <phi>^2)); core
// (if not null) marks <u> >= core_u.
// The means are IEEE quotients, so a core decision on <u> is the one an FP64
// host computation of acc / samples takes.
__global__ void __launch_bounds__(256) k_stats_profiles(int nij, const double* __restrict__ acc, double samples,
                                                        double core_u, double* __restrict__ prof,
                                                        unsigned char* __restrict__ core) {
  const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
  if (n >= nij) return;
  double m[STATS_NF];
#pragma unroll
  for (int f = 0; f < STATS_NF; ++f) m[f] = acc[f * (long long)nij + n] / samples;
#pragma unroll
  for (int f = 0; f < 5; ++f) prof[f * (long long)nij + n] = m[f];
  // second moments uu, vv, ww of fields 5..7, pp of field 11
  prof[5 * (long long)nij + n] = sqrt(fmax(0.0, m[5] - m[1] * m[1]));
  prof[6 * (long long)nij + n] = sqrt(fmax(0.0, m[6] - m[2] * m[2]));
  prof[7 * (long long)nij + n] = sqrt(fmax(0.0, m[7] - m[3] * m[3]));
  prof[8 * (long long)nij + n] = sqrt(fmax(0.0, m[11] - m[4] * m[4]));
  prof[9 * (long long)nij + n] = m[8] - m[1] * m[2];
  if (core) core[n] = m[1] >= core_u ? 1 : 0;
}

static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_stats_profiles(hipStream_t s, const Layout& L, const double* acc, double samples, double core_u,
                                 double* prof, unsigned char* core) {
  const long long nij = (long long)L.ni * L.nj;
  k_stats_profiles<<<nblk(nij, 256), 256, 0, s>>>((int)nij, acc, samples, core_u, prof, core);
  return hipGetLastError();
}

hipError_t launch_metrics(hipStream_t s, const Layout& L, const int bc[3], const double* xyz, double* M) {
  Dense D{L.ni, L.nj, L.nk};
  long long tot = (long long)(L.ni + 2) * (L.nj + 2) * (L.nk + 2);
  k_metrics<<<nblk(tot, 256), 256, 0, s>>>(L, D, bc[0], bc[1], bc[2], xyz, M);
  return hipGetLastError();
}

hipError_t launch_metrics_copy(hipStream_t s, const Layout& L, const double* src, double* M) {
  Dense D{L.ni, L.nj, L.nk};
  long long tot = (long long)(L.ni + 2) * (L.nj + 2) * (L.nk + 2);
  k_metrics_copy<<<nblk(tot, 256), 256, 0, s>>>(L, D, src, M);
  return hipGetLastError();
}

hipError_t launch_metrics_export(hipStream_t s, const Layout& L, const double* M, double* dst) {
  Dense D{L.ni, L.nj, L.nk};
  k_metrics_export<<<nblk(D.n(), 256), 256, 0, s>>>(L, D, M, dst);
  return hipGetLastError();
}

long long ghost_count(const Layout& L) {
  return 4LL * (L.nj + 4) * (L.ni + 4) + (long long)L.nk * 4 * (L.ni + 4) + (long long)L.nk * L.nj * 4;
}

hipError_t launch_ghost_fill(hipStream_t s, const Layout& L, const int bc[3], double* q, const double* frozen, int nf,
                             const Faces& F) {
  k_ghost_fill<<<nblk(ghost_count(L), 256), 256, 0, s>>>(L, bc[0], bc[1], bc[2], q, frozen, nf, F);
  return hipGetLastError();
}

hipError_t launch_ghost_fill_f32(hipStream_t s, const Layout& L, const int bc[3], float* q, const double* frozen,
                                 const Faces& F) {
  k_ghost_fill_f32<<<nblk(ghost_count(L), 256), 256, 0, s>>>(L, bc[0], bc[1], bc[2], q, frozen, F);
  return hipGetLastError();
}

// p[0 .. n) = 0 (a kernel, not a memset, so that a captured call records
// only kernel nodes).
__global__ void __launch_bounds__(256) k_zero(double* __restrict__ p, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

hipError_t launch_zero(hipStream_t s, double* p, long long n) {
  k_zero<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

// Stream copy (instrumentation): the bandwidth a plain, coalesced copy
// reaches, as the achievable counterpart of the HBM peak.  Each thread
// moves four 16-byte words, 256 words apart, loaded before any is stored.
__global__ void __launch_bounds__(256) k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     long long n16) {
  const long long i = (long long)blockIdx.x * 1024 + threadIdx.x;
  uint4 v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (i + 256 * u < n16) v[u] = src[i + 256 * u];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (i + 256 * u < n16) dst[i + 256 * u] = v[u];
}

hipError_t launch_stream_copy(hipStream_t s, const void* src, void* dst, long long n16) {
  const long long blocks = (n16 + 1023) / 1024;
  k_stream_copy<<<(unsigned)blocks, 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_stats(hipStream_t s, const Layout& L, const Phys& P, int nks, const double* Q, double* acc) {
  dim3 g(nblk(L.ni, 64), L.nj), b(64, 4);
  k_stats<<<g, b, 0, s>>>(L, P, nks, Q, acc);
  return hipGetLastError();
}

long long ref_blocks(const Layout& L) { return (long long)nblk(L.ni, 64) * nblk(L.nj, 4) * L.nk; }

// planes per CFL block
static int cfl_kc(const Layout& L) {
  const long long plane = (long long)nblk(L.ni + LEAD, 64) * nblk(L.nj, 4);
  long long kc = (plane * L.nk + CFL_PARTS - 1) / CFL_PARTS;
  return (int)(kc < 1 ? 1 : (kc > L.nk ? L.nk : kc));
}

long long cfl_blocks(const Layout& L) {
  return (long long)nblk(L.ni + LEAD, 64) * nblk(L.nj, 4) * nblk(L.nk, cfl_kc(L));
}

hipError_t launch_cfl(hipStream_t s, const Layout& L, const Phys& P, const double* M, const double* Q, double* part,
                      double* dt_out, int* flag, double* also, int axis) {
  const int kc = cfl_kc(L);
  dim3 g(nblk(L.ni + LEAD, 64), nblk(L.nj, 4), nblk(L.nk, kc)), b(64, 4);
  k_cfl_partial<<<g, b, 0, s>>>(L, P, M, Q, kc, axis ? 1 : 0, part);
  k_cfl_final<<<1, 1024, 0, s>>>(part, cfl_blocks(L), P.cfl, dt_out, also, flag);
  return hipGetLastError();
}

hipError_t launch_axis_avg(hipStream_t s, const Layout& L, double* q) {
  k_axis_avg<double><<<(unsigned)(5LL * L.ni), 64, 0, s>>>(L, q);
  return hipGetLastError();
}

hipError_t launch_axis_avg_f32(hipStream_t s, const Layout& L, float* q) {
  k_axis_avg<float><<<(unsigned)(5LL * L.ni), 64, 0, s>>>(L, q);
  return hipGetLastError();
}

hipError_t launch_cfl_final(hipStream_t s, const double* part, long long np, double cfl, double* dt_out,
                            double* also, int* flag) {
  k_cfl_final<<<1, 1024, 0, s>>>(part, np, cfl, dt_out, also, flag);
  return hipGetLastError();
}

hipError_t launch_residual_ref(hipStream_t s, const Layout& L, const Phys& P, const double* M, const double* Q,
                               const double* f, int i_f, double* R, double* part, const double* dyn, int axis) {
  dim3 g(nblk(L.ni, 64), nblk(L.nj, 4), L.nk), b(64, 4);
  RefArgs A{L, P, M, Q, dyn, axis};
  k_residual_ref<<<g, b, 0, s>>>(A, f, i_f, R, part);
  return hipGetLastError();
}

hipError_t launch_stage_ref(hipStream_t s, const Layout& L, const Phys& P, const double* M, const double* Qin,
                            const double* Q0, double* Qout, const double* dtp, double dt, double alpha,
                            const double* f, int i_f, double* part, const double* dyn, int axis) {
  dim3 g(nblk(L.ni, 64), nblk(L.nj, 4), L.nk), b(64, 4);
  RefArgs A{L, P, M, Qin, dyn, axis};
  k_stage_ref<<<g, b, 0, s>>>(A, Q0, Qout, dtp, dt, alpha, f, i_f, part);
  return hipGetLastError();
}

hipError_t launch_norm_final(hipStream_t s, const double* part, long long np, double count, double* norms, int* flag) {
  k_norm_final<<<1, 256, 0, s>>>(part, np, count, norms, flag);
  return hipGetLastError();
}

hipError_t launch_probe(hipStream_t s, const Layout& L, const Phys& P, int nks, const double* Q, int i_p,
                        double p_inf, double weight, double* Jacc, double* Qbar, double* part) {
  // up to 64 blocks (part holds at least that many doubles)
  const unsigned nb = min(64u, nblk((long long)L.nj * nks, 256));
  k_probe<<<nb, 256, 0, s>>>(L, P, nks, Q, i_p, p_inf, weight, part, Qbar);
  k_probe_final<<<1, 64, 0, s>>>(part, (int)nb, weight, Jacc);
  return hipGetLastError();
}

}  // namespace les
