// les_stage.hip -- fused residual + Runge-Kutta stage kernel for gfx950.
//
// One launch evaluates R(Q^(l-1)) at every interior node and writes
// Q^(l) = Q^(0) - alpha_l dt R (Sec. 4, Alg. 2: inviscid flux, artificial
// dissipation, viscous flux, RHS and the stage update of one RK stage,
// fused), plus per-block partial norms of R.
//
// Decomposition.  A block of 32 x 16 threads owns the nodes of a 32 x 16
// patch of one k-plane: the 30 x 14 output tile and a one-node halo ring.
// It marches along k over a chunk of planes.  Each thread keeps the
// k-direction stencil of its own column in registers (primitives at
// t-1, t, t+1, conserved variables at t-2..t+1, the zeta node flux, the
// zeta face flux and the partial residual of the previous plane), so the
// zeta direction needs no LDS.  The in-plane (xi, eta) stencil goes through
// LDS in three phases per plane, separated by barriers:
//   B  fill:   every node of the patch (and a second halo ring along the
//              axes, loaded by helper threads) stores Q, p, u, v, w, T;
//   C  node:   every non-corner node of the patch computes its velocity /
//              temperature gradient (chain rule through its metrics), the
//              viscous stress with Sutherland and Smagorinsky viscosity,
//              the node fluxes it is responsible for, the Turkel-Vatsa
//              anisotropic spectral radii and pressure sensors;
//   E  face:   tile nodes difference the node fluxes, build the four
//              in-plane dissipation faces from LDS and the zeta face from
//              registers, and finish the residual of the plane below.
// Each node quantity is computed once per patch (the halo ring costs 22%
// extra node work); every HBM array is read once per stage apart from the
// halo overlap between neighbouring patches, which L2 serves.
//
// Work per thread is independent of the floating-point type T (double for
// the FP64 path, float for the mixed path); Q^(0), the stage update, J and
// all reductions stay in FP64.
#include <stdlib.h>

#include "les_stage.hpp"
#include "les_launch.hpp"

namespace les {

namespace {

constexpr int BX = 32, BY = 16, NT = BX * BY;  // patch (threads)
constexpr int TX = BX - 2, TY = BY - 2;        // output tile
constexpr int EX = BX + 2, EY = BY + 2;        // patch + axis halo (LDS planes)
constexpr int NH2 = 2 * TY + 2 * TX;           // second-ring helper nodes

struct KArgs {
  Layout L;
  Phys P;
  const double* M;
  const double* f;
  int i_f;
  int kchunk;     // planes per block
  int ntx, nty;   // tiles in i, j
  int nkc;        // k chunks
  int nblocks;    // real blocks (grid may be padded to a multiple of 8)
  int per_xcd;    // blocks per XCD in the remapped order
};

template <class T>
struct Smem {
  T q[5][EY][EX];
  T p[EY][EX];
  T u[EY][EX], v[EY][EX], w[EY][EX], tem[EY][EX];
  T hx[5][BY][BX];
  T hy[5][BY][BX];
  T lx[BY][BX], ly[BY][BX];
  T nx[BY][BX], ny[BY][BX];
};

// Global accesses use a uniform (scalar) base per field plus a 32-bit
// per-thread byte offset, so that each access needs one VGPR for its address.
template <class X>
__device__ __forceinline__ X ldo(const X* base, unsigned off) {
  return *(const X*)((const char*)base + (size_t)(off * (unsigned)sizeof(X)));
}
template <class X>
__device__ __forceinline__ void sto(X* base, unsigned off, X v) {
  *(X*)((char*)base + (size_t)(off * (unsigned)sizeof(X))) = v;
}

template <class T, class QI>
__device__ __forceinline__ void load_q(const QI* __restrict__ Q, long long fe, unsigned off, T q[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) q[c] = (T)ldo(Q + c * fe, off);
}

// Dissipation flux of the face between nodes a and b = a + 1 along a line
// (am = a - 1, bp = b + 1), given the node spectral radii and sensors.
template <class T>
__device__ __forceinline__ void face_diss(const Phys& P, T La, T Lb, T na, T nb, const T qam[5], const T qa[5],
                                          const T qb[5], const T qbp[5], T D[5]) {
  const T e2 = T(P.k2) * tmax(na, nb);
  const T e4 = tmax(T(0), T(P.k4) - e2);
  const T Lf = T(0.5) * (La + Lb);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const T d1 = qb[c] - qa[c];
    const T d3 = qbp[c] - T(3) * qb[c] + T(3) * qa[c] - qam[c];
    D[c] = Lf * (e2 * d1 - e4 * d3);
  }
}

// Per-wave reduction of one plane's R^2 sums and |R| maxima, accumulated in
// the wave's row of `red` (all lanes of the wave must call it).
__device__ __forceinline__ void norm_accumulate(const double s2[5], const double sm[5], double (*red)[10], int tid) {
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double sum = wave_sum(s2[c]);
    const double mx = wave_max(sm[c]);
    if ((tid & 63) == 0) {
      red[tid >> 6][c] += sum;
      const double o = red[tid >> 6][5 + c];
      red[tid >> 6][5 + c] = (mx > o || mx != mx) ? mx : o;
    }
  }
}

template <class T, class QI, bool NORM>
__global__ void __launch_bounds__(NT) k_stage(KArgs a, const QI* __restrict__ Qin, const double* Q0, double* Qout,
                                              float* Qsh, const double* __restrict__ dtp, double dt_host,
                                              double alpha, double* __restrict__ part) {
  __shared__ Smem<T> s;
  __shared__ double red[NT / 64][10];  // per-wave norm partials (NORM only)
  const Layout& L = a.L;
  const Phys& P = a.P;
  const long long fe = L.fe;

  // XCD-aware block order: consecutive virtual blocks land on one XCD.
  const int b = blockIdx.x;
  const int v = (b & 7) * a.per_xcd + (b >> 3);
  if (v >= a.nblocks) return;
  const int kci = v % a.nkc;
  const int tile = v / a.nkc;
  const int tix = tile % a.ntx, tiy = tile / a.ntx;
  const int i0 = tix * TX, j0 = tiy * TY;
  const int kb = kci * a.kchunk;
  const int ke = min(kb + a.kchunk, L.nk);

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int ex = tx + 1, ey = ty + 1;
  const int i = i0 - 1 + tx, j = j0 - 1 + ty;
  const bool xh = (tx == 0 || tx == BX - 1), yh = (ty == 0 || ty == BY - 1);
  const bool load_ok = i <= L.ni + 1 && j <= L.nj + 1;
  const bool node_ok = load_ok && i <= L.ni && j <= L.nj && !(xh && yh);
  const bool need_x = node_ok && !yh;  // xi node flux / sensor needed here
  const bool need_y = node_ok && !xh;  // eta node flux / sensor needed here
  const bool out_ok = !xh && !yh && i < L.ni && j < L.nj;

  // second halo ring along the axes (helper thread h < NH2)
  int hx2 = 0, hy2 = 0, hi = 0, hj = 0;
  bool h_ok = false;
  if (tid < NH2) {
    int h = tid;
    if (h < TY) { hx2 = 0; hy2 = 2 + h; }
    else if (h < 2 * TY) { hx2 = EX - 1; hy2 = 2 + h - TY; }
    else if (h < 2 * TY + TX) { hy2 = 0; hx2 = 2 + h - 2 * TY; }
    else { hy2 = EY - 1; hx2 = 2 + h - 2 * TY - TX; }
    hi = i0 - 2 + hx2;
    hj = j0 - 2 + hy2;
    h_ok = hi <= L.ni + 1 && hj <= L.nj + 1;
  }
  if (NORM && tid < NT / 64 * 10) red[tid / 10][tid % 10] = 0.0;

  // element offsets of nodes (i, j, 0) and (hi, hj, 0); every node of the
  // padded box lies below 2^29 elements per field (checked at creation)
  const unsigned col = (unsigned)((long long)i + (long long)j * L.sj + L.o);
  const unsigned hcol = (unsigned)((long long)hi + (long long)hj * L.sj + L.o);
  const unsigned sk = (unsigned)L.sk;
  const double dt = dtp ? dtp[0] : dt_host;
  const double adt = alpha * dt;

  // ---- column queues (own node); plane-t values live in LDS ----
  T qm1[5], qp1[5];   // Q at t-1 and t+1
  T um1[4], up1[4];   // u, v, w, T at t-1 and t+1
  T pm1 = 0, pp1 = 0; // p at t-1 and t+1
  T hz_prev[5];       // zeta node flux at t-1
  T racc[5];          // partial residual of plane t-1: in-plane part - zeta face (t-3/2)
  T lz_prev = 0, nz_prev = 0;
  double J_prev = 0.0;
#pragma unroll
  for (int c = 0; c < 5; ++c) qm1[c] = qp1[c] = hz_prev[c] = racc[c] = T(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) um1[c] = up1[c] = T(0);

  auto prims = [&](const T q[5], T uu[4], T& pp) {
    T u, vv, w, p, tem;
    prim_from_q(q[0], q[1], q[2], q[3], q[4], P, u, vv, w, p, tem);
    uu[0] = u; uu[1] = vv; uu[2] = w; uu[3] = tem;
    pp = p;
  };

  // prime: plane kb-2 -> t-1 slot, plane kb-1 -> the slot written to LDS at t = kb-1
  if (load_ok) {
    load_q<T>(Qin, fe, col + (unsigned)(kb - 2) * sk, qm1);
    prims(qm1, um1, pm1);
    load_q<T>(Qin, fe, col + (unsigned)(kb - 1) * sk, qp1);
  }

  for (int t = kb - 1; t <= ke; ++t) {
    const unsigned nt = col + (unsigned)t * sk;
    // the first and last plane of a chunk only provide zeta quantities of
    // the tile columns; their in-plane fluxes and residual are not needed
    const bool inner = t >= kb && t < ke;
    const bool nx_t = need_x && inner, ny_t = need_y && inner;
    const bool node_t = inner ? node_ok : out_ok;

    // ---- B: fill LDS plane t (own node from the queue, second ring by helpers) ----
    if (load_ok) {
      T u4[4], pc;
      prims(qp1, u4, pc);
#pragma unroll
      for (int c = 0; c < 5; ++c) s.q[c][ey][ex] = qp1[c];
      s.p[ey][ex] = pc;
      s.u[ey][ex] = u4[0]; s.v[ey][ex] = u4[1]; s.w[ey][ex] = u4[2]; s.tem[ey][ex] = u4[3];
      // ---- A: load plane t+1 of the own column ----
      load_q<T>(Qin, fe, nt + sk, qp1);
      prims(qp1, up1, pp1);
    }
    if (h_ok) {
      T hq[5], hu[4], hp;
      load_q<T>(Qin, fe, hcol + (unsigned)t * sk, hq);
      prims(hq, hu, hp);
#pragma unroll
      for (int c = 0; c < 5; ++c) s.q[c][hy2][hx2] = hq[c];
      s.p[hy2][hx2] = hp;
      s.u[hy2][hx2] = hu[0]; s.v[hy2][hx2] = hu[1]; s.w[hy2][hx2] = hu[2]; s.tem[hy2][hx2] = hu[3];
    }
    __syncthreads();

    // ---- C: node work at plane t ----
    T hz[5] = {0, 0, 0, 0, 0};
    T lz = 0, nz = 0;
    double Jn = 0.0;
    if (node_t) {
      double m[10];
#pragma unroll
      for (int c = 0; c < 10; ++c) m[c] = ldo(a.M + c * fe, nt);
      Jn = m[9];
      T mt[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) mt[c] = (T)m[c];
      const T Jt = (T)Jn;
      T g[4][3];
      {
        // derivatives along xi, eta (LDS) and zeta (registers), chain rule
        const T (*F[4])[EX] = {s.u, s.v, s.w, s.tem};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T dx = T(0.5) * (F[q][ey][ex + 1] - F[q][ey][ex - 1]);
          const T dy = T(0.5) * (F[q][ey + 1][ex] - F[q][ey - 1][ex]);
          const T dz = T(0.5) * (up1[q] - um1[q]);
#pragma unroll
          for (int x = 0; x < 3; ++x) g[q][x] = Jt * (mt[x] * dx + mt[3 + x] * dy + mt[6 + x] * dz);
        }
      }
      const T s11 = g[0][0], s22 = g[1][1], s33 = g[2][2];
      const T s12 = T(0.5) * (g[0][1] + g[1][0]);
      const T s13 = T(0.5) * (g[0][2] + g[2][0]);
      const T s23 = T(0.5) * (g[1][2] + g[2][1]);
      const T skk3 = (s11 + s22 + s33) / T(3);
      const T rho = s.q[0][ey][ex];
      const T u = s.u[ey][ex], vv = s.v[ey][ex], w = s.w[ey][ex];
      const T mu = sutherland(s.tem[ey][ex], P);
      T mus = T(0);
      if (P.sgs) {
        const T ss = s11 * s11 + s22 * s22 + s33 * s33 + T(2) * (s12 * s12 + s13 * s13 + s23 * s23);
        T d2 = (T)cbrt(1.0 / Jn);
        d2 *= d2;
        mus = rho * T(P.Cs2) * d2 * sqrt(T(2) * ss);
      }
      const T mt2 = T(2) * (mu + mus);
      const T t11 = mt2 * (s11 - skk3), t22 = mt2 * (s22 - skk3), t33 = mt2 * (s33 - skk3);
      const T t12 = mt2 * s12, t13 = mt2 * s13, t23 = mt2 * s23;
      const T kap = mu * T(P.Cp_over_Pr) + mus * T(P.Cp_over_Prsgs);
      const T th0 = u * t11 + vv * t12 + w * t13 + kap * g[3][0];
      const T th1 = u * t12 + vv * t22 + w * t23 + kap * g[3][1];
      const T th2 = u * t13 + vv * t23 + w * t33 + kap * g[3][2];
      const T p = s.p[ey][ex];
      const T c = sqrt(T(P.gamma) * p / rho);
      // spectral radii of the three directions
      T lam[3], U[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const T mx = mt[3 * e], my = mt[3 * e + 1], mz = mt[3 * e + 2];
        U[e] = mx * u + my * vv + mz * w;
        lam[e] = fabs(U[e]) + c * sqrt(mx * mx + my * my + mz * mz);
      }
      auto node_flux = [&](int e, T H[5]) {
        const T mx = mt[3 * e], my = mt[3 * e + 1], mz = mt[3 * e + 2];
        const T Ue = U[e];
        H[0] = rho * Ue;
        H[1] = s.q[1][ey][ex] * Ue + mx * p - (mx * t11 + my * t12 + mz * t13);
        H[2] = s.q[2][ey][ex] * Ue + my * p - (mx * t12 + my * t22 + mz * t23);
        H[3] = s.q[3][ey][ex] * Ue + mz * p - (mx * t13 + my * t23 + mz * t33);
        H[4] = (s.q[4][ey][ex] + p) * Ue - (mx * th0 + my * th1 + mz * th2);
      };
      if (nx_t) {
        T H[5];
        node_flux(0, H);
#pragma unroll
        for (int q = 0; q < 5; ++q) s.hx[q][ty][tx] = H[q];
        s.lx[ty][tx] = aniso(lam[0], lam[1], lam[2], P);
        const T pa = s.p[ey][ex + 1], pb = s.p[ey][ex - 1];
        s.nx[ty][tx] = fabs(pa - T(2) * p + pb) / (pa + T(2) * p + pb);
      }
      if (ny_t) {
        T H[5];
        node_flux(1, H);
#pragma unroll
        for (int q = 0; q < 5; ++q) s.hy[q][ty][tx] = H[q];
        s.ly[ty][tx] = aniso(lam[1], lam[2], lam[0], P);
        const T pa = s.p[ey + 1][ex], pb = s.p[ey - 1][ex];
        s.ny[ty][tx] = fabs(pa - T(2) * p + pb) / (pa + T(2) * p + pb);
      }
      if (out_ok) {
        node_flux(2, hz);
        lz = aniso(lam[2], lam[0], lam[1], P);
        nz = fabs(pp1 - T(2) * p + pm1) / (pp1 + T(2) * p + pm1);
      }
    }
    __syncthreads();

    // ---- E: residual (tile nodes) ----
    double s2[5] = {0, 0, 0, 0, 0}, sm[5] = {0, 0, 0, 0, 0};
    if (out_ok) {
      T r[5] = {0, 0, 0, 0, 0};
      if (inner) {
        // central differences of the in-plane node fluxes
#pragma unroll
        for (int q = 0; q < 5; ++q)
          r[q] = T(0.5) * (s.hx[q][ty][tx + 1] - s.hx[q][ty][tx - 1]) +
                 T(0.5) * (s.hy[q][ty + 1][tx] - s.hy[q][ty - 1][tx]);
        // in-plane dissipation faces
        T qa[5], qb[5], qc[5], qd[5], qe[5], D1[5], D0[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          qa[c] = s.q[c][ey][ex - 2]; qb[c] = s.q[c][ey][ex - 1]; qc[c] = s.q[c][ey][ex];
          qd[c] = s.q[c][ey][ex + 1]; qe[c] = s.q[c][ey][ex + 2];
        }
        face_diss(P, s.lx[ty][tx], s.lx[ty][tx + 1], s.nx[ty][tx], s.nx[ty][tx + 1], qb, qc, qd, qe, D1);
        face_diss(P, s.lx[ty][tx - 1], s.lx[ty][tx], s.nx[ty][tx - 1], s.nx[ty][tx], qa, qb, qc, qd, D0);
#pragma unroll
        for (int c = 0; c < 5; ++c) r[c] -= D1[c] - D0[c];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          qa[c] = s.q[c][ey - 2][ex]; qb[c] = s.q[c][ey - 1][ex];
          qd[c] = s.q[c][ey + 1][ex]; qe[c] = s.q[c][ey + 2][ex];
        }
        face_diss(P, s.ly[ty][tx], s.ly[ty + 1][tx], s.ny[ty][tx], s.ny[ty + 1][tx], qb, qc, qd, qe, D1);
        face_diss(P, s.ly[ty - 1][tx], s.ly[ty][tx], s.ny[ty - 1][tx], s.ny[ty][tx], qa, qb, qc, qd, D0);
#pragma unroll
        for (int c = 0; c < 5; ++c) r[c] -= D1[c] - D0[c];
      }
      if (t >= kb) {
        // zeta face t - 1/2 between plane t-1 and plane t (Q at t-2 re-read; L2 hit)
        T qm2[5], qc[5], D[5];
        load_q<T>(Qin, fe, nt - 2 * sk, qm2);
#pragma unroll
        for (int c = 0; c < 5; ++c) qc[c] = s.q[c][ey][ex];
        face_diss(P, lz_prev, lz, nz_prev, nz, qm2, qm1, qc, qp1, D);
        T fz[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) fz[c] = T(0.5) * (hz_prev[c] + hz[c]) - D[c];
        if (t > kb) {
          // residual of plane t-1 and its stage update
          const int k = t - 1;
          const unsigned n = nt - sk;
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            double R = J_prev * (double)(racc[c] + fz[c]);
            if (a.f && i == a.i_f) R -= a.f[((long long)c * L.nk + k) * L.nj + j];
            const double qn = ldo(Q0 + c * fe, n) - adt * R;
            if (Qout) sto(Qout + c * fe, n, qn);
            if (Qsh) sto(Qsh + c * fe, n, (float)qn);
            if (NORM) {
              s2[c] = R * R;
              sm[c] = fabs(R);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) racc[c] = r[c] - fz[c];
      } else {
#pragma unroll
        for (int c = 0; c < 5; ++c) racc[c] = r[c];
      }
#pragma unroll
      for (int c = 0; c < 5; ++c) hz_prev[c] = hz[c];
      lz_prev = lz;
      nz_prev = nz;
      J_prev = Jn;
    }
    if (NORM && t > kb) norm_accumulate(s2, sm, red, tid);
    // ---- shift the column queues (plane t values from LDS) ----
    if (load_ok) {
#pragma unroll
      for (int c = 0; c < 5; ++c) qm1[c] = s.q[c][ey][ex];
      um1[0] = s.u[ey][ex]; um1[1] = s.v[ey][ex]; um1[2] = s.w[ey][ex]; um1[3] = s.tem[ey][ex];
      pm1 = s.p[ey][ex];
    }
    __syncthreads();
  }

  // ---- block partial norms ----
  if (NORM) {
    __syncthreads();
    if (tid < 10) {
      double r = red[0][tid];
      for (int w = 1; w < NT / 64; ++w) {
        const double o = red[w][tid];
        r = tid < 5 ? r + o : ((o > r || o != o) ? o : r);
      }
      part[(long long)v * 10 + tid] = r;
    }
  }
}

// Stage kernel configuration for a layout.
struct Config {
  int ntx, nty, nkc, kchunk, nblocks, grid, per_xcd;
};

int auto_kchunk(const Layout& L) {
  const long long tiles = (long long)((L.ni + TX - 1) / TX) * ((L.nj + TY - 1) / TY);
  // enough blocks to fill the 256 CUs at least twice, chunks of >= 8 planes
  int chunk = L.nk;
  while (chunk > 8 && tiles * ((L.nk + chunk - 1) / chunk) < 2 * 256) chunk = (chunk + 1) / 2;
  return chunk;
}

Config config(const Layout& L, int kchunk) {
  Config c;
  c.ntx = (L.ni + TX - 1) / TX;
  c.nty = (L.nj + TY - 1) / TY;
  c.kchunk = kchunk < 1 ? 1 : (kchunk > L.nk ? L.nk : kchunk);
  c.nkc = (L.nk + c.kchunk - 1) / c.kchunk;
  c.nblocks = c.ntx * c.nty * c.nkc;
  c.per_xcd = (c.nblocks + 7) / 8;
  c.grid = c.per_xcd * 8;
  return c;
}

template <class T, class QI>
hipError_t launch(hipStream_t st, const StageArgs& sa, const QI* Qin, const double* Q0, double* Qout, float* Qsh,
                  const double* dtp, double dt, double alpha, double* part) {
  Config c = config(sa.L, sa.kchunk);
  KArgs a{sa.L, sa.P, sa.M, sa.f, sa.i_f, c.kchunk, c.ntx, c.nty, c.nkc, c.nblocks, c.per_xcd};
  if (part)
    k_stage<T, QI, true><<<c.grid, NT, 0, st>>>(a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part);
  else
    k_stage<T, QI, false><<<c.grid, NT, 0, st>>>(a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part);
  return hipGetLastError();
}

}  // namespace

int stage_kchunk(const Layout& L) {
  const char* env = getenv("LES_KCHUNK");
  if (env && atoi(env) > 0) return atoi(env) < L.nk ? atoi(env) : L.nk;
  return auto_kchunk(L);
}

long long stage_blocks(const Layout& L, int kchunk) { return config(L, kchunk).nblocks; }

hipError_t launch_stage_fp64(hipStream_t s, const StageArgs& a, const double* Qin, const double* Q0, double* Qout,
                             const double* dtp, double dt, double alpha, double* part) {
  return launch<double, double>(s, a, Qin, Q0, Qout, nullptr, dtp, dt, alpha, part);
}

hipError_t launch_stage_mixed(hipStream_t s, const StageArgs& a, const double* Qin64, const float* Qin32,
                              const double* Q0, double* Qout, float* Qsh, const double* dtp, double dt, double alpha,
                              double* part) {
  if (Qin64) return launch<float, double>(s, a, Qin64, Q0, Qout, Qsh, dtp, dt, alpha, part);
  return launch<float, float>(s, a, Qin32, Q0, Qout, Qsh, dtp, dt, alpha, part);
}

}  // namespace les
