// les_stage.hip -- fused residual + Runge-Kutta stage kernel for gfx950.
//
// One launch evaluates R(Q^(l-1)) at every interior node and writes
// Q^(l) = Q^(0) - alpha_l dt R (Sec. 4, Alg. 2: inviscid flux, artificial
// dissipation, viscous flux, RHS and the stage update of one RK stage,
// fused), plus per-block partial norms of R (first stage) or per-block
// minima of the local CFL bound of the updated state (last stage: the time
// step of the next step is pointwise in Q^{n+1}, so it is reduced while the
// state is in registers instead of by a pass of its own).
//
// Decomposition.  A block of 32 x 16 threads owns the nodes of a 32 x 16
// patch of one k-plane: the 30 x 14 output tile and a one-node halo ring.
// Blocks are persistent (one per CU of the device): block v marches a contiguous range of
// (tile, k) planes in chunk-major order (k chunks as long as one block's
// range, tiles within a chunk, planes within a tile), so the blocks that
// run together on one XCD start on neighbouring tiles at the same plane and
// read the halo lines they share while those are still in the XCD's L2, and
// the per-tile start-up cost (two extra planes) is paid about once per
// block.  Each thread keeps the k-direction stencil of its own column in
// registers (conserved variables at t-2 .. t+1, primitives at t-1 and t+1,
// the zeta node flux and the partial residual of the plane below), so the
// zeta direction needs no LDS.  The in-plane (xi, eta) stencil goes
// through LDS in three phases per plane, separated by barriers (a third
// barrier closes the plane in the FP64 path; the FP32 path double-buffers
// the LDS Q plane instead, see below):
//   B  fill:  every node of the patch (and a second halo ring along the
//             axes, written by helper threads) stores Q, p, u, v, w, T;
//   C  node:  every non-corner node of the patch computes its velocity and
//             temperature gradient (chain rule through its metrics), the
//             viscous stress with Sutherland and Smagorinsky viscosity, the
//             node fluxes it is responsible for, the Turkel-Vatsa
//             anisotropic spectral radii and the pressure sensors;
//   E  face:  tile nodes difference the node fluxes, build the four in-plane
//             dissipation faces from LDS and the zeta face from registers,
//             and finish the residual and stage update of the plane below
//             (stage 1 also accumulates R^2 and max |R| per thread; the
//             block reduces them once, after its last plane).
// Memory.  Wave w owns patch rows 2w and 2w+1 (rows 4w .. 4w+3 with the
// 16-wide patch the shape constants also allow).  The ten metric fields and
// Q^(0) of those rows are wave-private, so they travel as asynchronous
// global->LDS copies (16 bytes per lane) into per-wave LDS blocks with no
// barrier: Q^(0) of the plane being finished is issued at the start of C
// and read at the start of E; the next plane's metrics are issued right
// after that read and land during E (E stores nothing to LDS, so no LDS
// store has to wait for them).  The block barriers order LDS data only:
// a full __syncthreads would also drain every outstanding global load,
// store and copy of the wave, so each barrier would wait out the latency of
// what was just issued.  Reads of copied blocks are preceded by counted
// vmcnt waits instead.  The own-column loads are branch-free (threads past
// the padded box load a clamped node), which lets the compiler see that
// they have completed and keeps it from adding full vmcnt waits of its own.
// The flow constants are read from the kernel-argument segment where they
// are used, instead of occupying scalar registers across the loop.  Divisions and square roots
// use short Newton-refined sequences (valid for the positive, normal
// arguments met here).  Scheduling fences split phases C and E into short
// regions (gradient / stress / spectral radii / each node flux; each
// dissipation direction / zeta face / residual): without them the scheduler
// hoists LDS reads of later regions over the FP64 work of earlier ones and
// the live ranges exceed the 256 registers of a two-wave-per-SIMD launch.
//
// Work per thread is independent of the floating-point type T (double for
// the FP64 path, float for the mixed path); metrics, Q^(0), the stage
// update, J and all reductions stay in FP64.  The FP32 path has registers
// and LDS to spare, and spends them on latency: it loads the helper ring one
// plane ahead and its own column two planes ahead (in phase E, consumed in C
// of the next plane), and it keeps two LDS Q planes, written at B of
// alternate planes.  Phase E reads no other LDS array of the current plane
// at other threads' nodes (p, u, v, w, T are read at neighbours only in C;
// the node fluxes, radii and sensors are next written in C, after the next
// plane's first barrier), so the barrier at the end of a plane is not needed
// there.  The FP64 path has neither the registers nor the 24 KB of LDS.
#include <stdlib.h>

#include "les_stage.hpp"
#include "les_launch.hpp"

namespace les {

namespace {

#ifndef LES_STAGE_BX
#define LES_STAGE_BX 32
#endif
#ifndef LES_STAGE_BY
#define LES_STAGE_BY 16
#endif
constexpr int BX = LES_STAGE_BX, BY = LES_STAGE_BY, NT = BX * BY;  // patch (threads)
constexpr int TX = BX - 2, TY = BY - 2;        // output tile
constexpr int EX = BX + 2, EY = BY + 2;        // patch + axis halo (LDS planes)
constexpr int NH2 = 2 * TY + 2 * TX;           // second-ring helper nodes
constexpr int NW = NT / 64;                    // waves per block
constexpr int RPW = 64 / BX;                   // patch rows per wave
constexpr int LPR = BX / 2;                    // lanes per row of a 16-byte row copy
constexpr int BPC = 512 / NT;                  // resident blocks per CU (two waves per SIMD)
static_assert(BX == 16 || BX == 32, "a wave covers whole patch rows");
static_assert(BY % RPW == 0 && NT % 64 == 0 && NH2 <= NT && BPC >= 1, "tile shape");

struct KArgs {
  Layout L;
  Phys P;
  const double* M;
  const double* f;
  const double* dyn;    // per-column dynamic SGS coefficients (P.sgs == 2)
  int axis;             // j = 0 is the polar axis
  int i_f;
  int ntx, nty;         // tiles in i, j
  long long total;      // tile-planes = ntx * nty * nk
  long long per_block;  // tile-planes per block (contiguous range)
  int kc;               // planes per k chunk of the chunk-major order
  int rr;               // 1: blocks take (chunk, tile) segments round robin
  long long nseg;       // segments in round-robin mode
  int nblocks;          // blocks with work
  int per_xcd;          // blocks per XCD in the remapped order
  int nxcd;             // XCDs of the device
};

// The FP32 path has the LDS for two Q planes (written at B of alternate
// planes), which removes the barrier at the end of a plane: the only LDS
// values that E reads at other threads' nodes are Q.
template <class T>
constexpr int kQBuf = sizeof(T) == 4 ? 2 : 1;
template <class T>
struct Smem {
  T q[kQBuf<T>][5][EY][EX];
  T p[EY][EX];
  T u[EY][EX], v[EY][EX], w[EY][EX], tem[EY][EX];
  T hx[5][TY][BX];  // xi node flux, patch rows 1..TY
  T hy[5][BY][TX];  // eta node flux, patch columns 1..TX
  T lx[TY][BX], nx[TY][BX];
  T ly[BY][TX], ny[BY][TX];
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

// Per-wave reduction of the threads' R^2 sums and |R| maxima into the ten
// doubles at red (all lanes of the wave must call it; lane 0 writes).
__device__ __forceinline__ void norm_wave(const double s2[5], const double sm[5], double* red, int lane) {
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double sum = wave_sum(s2[c]);
    const double mx = wave_max(sm[c]);
    if (lane == 0) {
      red[c] = sum;
      red[5 + c] = mx;
    }
  }
}

// Per-wave row staging.  Wave w owns patch rows RPW w .. RPW w + RPW - 1 (the
// rows of its own threads: two rows of 32 or four rows of 16), so the
// metrics and Q^(0) of those rows can be copied into a wave-private LDS block
// with no barrier.  One asynchronous global->LDS copy moves 16 bytes (two
// doubles) per lane: lanes 0-31 the 64 nodes of field f (row after row),
// lanes 32-63 the same for field f+1; they land contiguously at [f][r][col]
// of the block.  src is the lane's
// byte address for field (lane >> 5); fstep2 is two fields in bytes.  With
// an odd field count the last copy uses lanes 0-31 only.
template <int NF>
__device__ __forceinline__ void dma_rows(const char* src, long long fstep2, double* dst, int lane) {
#pragma unroll
  for (int q = 0; q < NF / 2; ++q)
    __builtin_amdgcn_global_load_lds((const void*)(src + q * fstep2),
                                     (__attribute__((address_space(3))) void*)(dst + q * 128), 16, 0, 0);
  if (NF & 1) {
    if (lane < 32)
      __builtin_amdgcn_global_load_lds((const void*)(src + (NF / 2) * fstep2),
                                       (__attribute__((address_space(3))) void*)(dst + (NF / 2) * 128), 16, 0, 0);
  }
}

// s_waitcnt vmcnt(N): all but the N most recent vector memory operations of
// this wave have completed (expcnt and lgkmcnt left unconstrained)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}
// s_waitcnt lgkmcnt(0): this wave's LDS reads have returned
__device__ __forceinline__ void wait_lgkm_all() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Block barrier for LDS data only: release/acquire at workgroup scope for
// the local address space, so the wave waits for its own LDS operations but
// not for outstanding global loads, stores or global->LDS copies (which a
// full __syncthreads drains).
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Optional paths of the stage kernel (template bit mask EXT)
constexpr int kExtSgs = 1;   // dynamic closure coefficients, isotropic SGS stress
constexpr int kExtAxis = 2;  // the O-grid's polar axis at j = 0

template <class T, class QI, bool NORM, bool CFL, int EXT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2, 2))) k_stage(KArgs a, const QI* __restrict__ Qin, const double* Q0, double* Qout,
                                              float* Qsh, const double* __restrict__ dtp, double dt_host,
                                              double alpha, double* __restrict__ part, double* __restrict__ cpart) {
  // the FP32 path has the registers to prefetch the helper ring one plane
  // ahead; the FP64 path loads it at phase B (holding it would spill)
  constexpr bool kPrefetchRing = sizeof(T) == 4;
  // the FP32 path also loads the own column two planes ahead (in E)
  constexpr bool kPrefetchQ = sizeof(T) == 4;
  constexpr bool kQ2 = kQBuf<T> == 2;
  __shared__ Smem<T> s;
  __shared__ double mbw[NW][10][RPW][BX];  // per-wave metrics rows of the current plane
  __shared__ double q0w[NW][5][RPW][BX];   // per-wave Q^(0) rows of the plane being finished
  static_assert(sizeof(Smem<T>) + sizeof(mbw) + sizeof(q0w) <= 163840 / BPC, "LDS of BPC blocks per CU");
  const Layout& L = a.L;
  // a (the first kernel argument) sits at the start of the kernel-argument
  // segment; the loop re-reads the flow constants through this pointer
  // (scalar loads) where they are used, so that they do not hold scalar
  // registers across the loop
  typedef __attribute__((address_space(4))) const KArgs CKArgs;
  CKArgs* const ka = (CKArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  const long long fe = L.fe;

  // XCD-aware order: consecutive virtual blocks land on one XCD.
  const int hb = blockIdx.x;
  const int v = (hb % a.nxcd) * a.per_xcd + hb / a.nxcd;
  if (v >= a.nblocks) return;
  // contiguous mode: tile-planes [w_begin, w_end) of the chunk-major order;
  // round-robin mode: segments v, v + nblocks, v + 2 nblocks, ...
  const long long w_begin = a.rr ? (long long)v : (long long)v * a.per_block;
  const long long w_end = a.rr ? a.nseg : min(a.total, w_begin + a.per_block);

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int ex = tx + 1, ey = ty + 1;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int fsel = lane >> 5, rsel = (lane / LPR) % RPW, pr = lane % LPR;  // row-copy lane geometry
  const int ty1 = ty % RPW;                                                // own row within the wave's rows
  const bool xh = (tx == 0 || tx == BX - 1), yh = (ty == 0 || ty == BY - 1);
  const unsigned sk = (unsigned)L.sk;
  const double adt = alpha * (dtp ? dtp[0] : dt_host);

  // second halo ring along the axes: helper thread h < NH2 owns LDS slot (hy2, hx2)
  int hx2 = 0, hy2 = 0;
  if (tid < NH2) {
    const int h = tid;
    if (h < TY) { hx2 = 0; hy2 = 2 + h; }
    else if (h < 2 * TY) { hx2 = EX - 1; hy2 = 2 + h - TY; }
    else if (h < 2 * TY + TX) { hy2 = 0; hx2 = 2 + h - 2 * TY; }
    else { hy2 = EY - 1; hx2 = 2 + h - 2 * TY - TX; }
  }

  auto prims = [&](const Phys& P, const T q[5], T uu[4], T& pp) {
    T u, vv, w, p, tem;
    prim_from_q_fast(q[0], q[1], q[2], q[3], q[4], P, u, vv, w, p, tem);
    uu[0] = u; uu[1] = vv; uu[2] = w; uu[3] = tem;
    pp = p;
  };

  // residual norms: per-thread running sums of R^2 and maxima of |R| over
  // all planes of the block (NORM only), reduced once at the end
  double n2[5] = {0, 0, 0, 0, 0}, nm[5] = {0, 0, 0, 0, 0};
  // CFL only (the last stage): running minimum of the local CFL bound of the
  // updated state Q^(l) = Q^{n+1} over the block's nodes
  double cmin = INFINITY;
  int qbuf = 0;  // LDS Q plane written at the next B (alternates every plane)
  for (long long wq = w_begin; wq < w_end;) {
    // ---- one segment: planes [kb, ke) of one tile ----
    // tile-planes are ordered k chunk by k chunk (kc planes; the last chunk
    // may be shorter), tile by tile within a chunk, plane by plane within a
    // tile: the blocks that run at the same time on one XCD start on
    // neighbouring tiles at the same plane, so the halo lines they share
    // are read while they are still in that XCD's L2.  A block takes a
    // contiguous range of that order when its share is at most one chunk;
    // with larger shares it takes whole (chunk, tile) segments round robin,
    // which keeps the blocks of an XCD on neighbouring tiles throughout.
    int tile, kb, ke;
    if (a.rr) {
      const long long ntiles = (long long)a.ntx * a.nty;
      const int ch = (int)(wq / ntiles);
      tile = (int)(wq % ntiles);
      kb = ch * a.kc;
      ke = min(L.nk, kb + a.kc);
      wq += a.nblocks;
    } else {
      const long long cfull = (long long)a.ntx * a.nty * a.kc;
      const int ch = (int)(wq / cfull);
      const int k0 = ch * a.kc;
      const int kcc = min(a.kc, L.nk - k0);
      const long long rr = wq - (long long)ch * cfull;
      tile = (int)(rr / kcc);
      kb = k0 + (int)(rr % kcc);
      ke = (int)min((long long)(k0 + kcc), (long long)kb + (w_end - wq));
      wq += ke - kb;
    }
    // segment base: plane kb - 2, the first the segment reads.  Per-thread
    // element offsets are taken from there, so they stay below 2^29 for any
    // block whose planes are small enough that kc + 6 of them are (the
    // schedule bounds kc accordingly); field and segment bases are 64-bit.
    const int kr = kb - 2;
    const long long sb = (long long)kr * L.sk;
    const QI* const Qs = Qin + sb;
    const int tix = tile % a.ntx, tiy = tile / a.ntx;
    const int i0 = tix * TX, j0 = tiy * TY;
    const int i = i0 - 1 + tx, j = j0 - 1 + ty;
    const bool load_ok = i <= L.ni + 1 && j <= L.nj + 1;
    const bool node_ok = load_ok && i <= L.ni && j <= L.nj && !(xh && yh);
    const bool need_x = node_ok && !yh;  // xi node flux / sensor needed here
    const bool need_y = node_ok && !xh;  // eta node flux / sensor needed here
    const bool out_ok = !xh && !yh && i < L.ni && j < L.nj;
    const int hi = i0 - 2 + hx2, hj = j0 - 2 + hy2;
    const bool h_ok = tid < NH2 && hi <= L.ni + 1 && hj <= L.nj + 1;
    // element offsets of nodes (i, j, kr) and (hi, hj, kr) from the segment
    // base
    const unsigned col = (unsigned)((long long)i + (long long)j * L.sj + L.o);
    const unsigned hcol = (unsigned)((long long)hi + (long long)hj * L.sj + L.o);
    // own-column loads use the node clamped into the padded box, so that they
    // and their uses need no branch (threads past the box load, and never
    // publish, a copy of the box's edge node)
    const unsigned qcol =
        (unsigned)((long long)min(i, L.ni + 1) + (long long)min(j, L.nj + 1) * L.sj + L.o);

    // ---- column queues (own node) ----
    T qw[5], qa[5], qn[5];  // Q at t (written at B), t+1 and t+2 (prefetch)
    T qm1[5], qm2[5];       // Q at t-1, t-2
    T um1[4], up1[4];       // u, v, w, T at t-1; at t+1 (at B: plane t)
    T pm1 = 0, pp1 = 0;
    T hq[5];                // helper node, next plane
    T hz_prev[5], racc[5];  // zeta node flux at t-1; partial residual of t-1
    T lz_prev = 0, nz_prev = 0;
    double J_prev = 0.0;
#pragma unroll
    for (int c = 0; c < 5; ++c) qw[c] = qa[c] = qn[c] = qm1[c] = qm2[c] = hq[c] = hz_prev[c] = racc[c] = T(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) um1[c] = up1[c] = T(0);

    // (the empty asm hides the pointer's origin, so the loads below are not
    // hoisted out of the loop)
    CKArgs* kp4 = ka;
    asm volatile("" : "+s"(kp4));
    const KArgs* kp = (const KArgs*)kp4;
    // prime for t = kb-1: metrics(kb-1) -> LDS; Q(kb-2), Q(kb-1) of the own
    // column; helper Q(kb-1)
    //
    // element offset (plane 0) of this lane's row copy: field fsel, row
    // RPW wave + rsel, column pair starting at i0-1+2pr (16-byte aligned);
    // pairs past i = ni (ragged last tile) re-read the last pair within the row
    int icp = i0 - 1 + 2 * pr;
    if (icp > L.ni) icp = L.ni - ((LEAD + L.ni) & 1);
    const int jcp = min(j0 - 1 + RPW * wave + rsel, L.nj);
    const long long lane_el = (long long)fsel * fe + L.o + icp + (long long)jcp * L.sj;
    const long long fstep2 = 2 * fe * (long long)sizeof(double);
    dma_rows<10>((const char*)(kp->M + lane_el + (long long)(kb - 1) * L.sk), fstep2, &mbw[wave][0][0][0], lane);
    load_q<T>(Qs, fe, qcol, qm1);
    load_q<T>(Qs, fe, qcol + sk, qw);
    if (kPrefetchQ) load_q<T>(Qs, fe, qcol + 2 * sk, qa);
    prims(kp->P, qm1, um1, pm1);
    prims(kp->P, qw, up1, pp1);  // plane kb-1, written at the first B
    if (kPrefetchRing && h_ok) load_q<T>(Qs, fe, hcol + sk, hq);

    for (int t = kb - 1; t <= ke; ++t) {
      const unsigned nt = col + (unsigned)(t - kr) * sk;
      CKArgs* kq4 = ka;
      asm volatile("" : "+s"(kq4));
      const KArgs* kq = (const KArgs*)kq4;
      const Phys& P = kq->P;
      // the first and last plane of a segment only provide zeta quantities
      // of the tile columns; their in-plane fluxes and residual are not needed
      const bool inner = t >= kb && t < ke;
      const bool nx_t = need_x && inner, ny_t = need_y && inner;
      const bool node_t = inner ? node_ok : out_ok;
      T(*const sq)[EY][EX] = s.q[kQ2 ? qbuf : 0];
      if (kQ2) qbuf ^= 1;

      // ---- B: fill LDS plane t ----
      if (load_ok) {
#pragma unroll
        for (int c = 0; c < 5; ++c) sq[c][ey][ex] = qw[c];
        s.p[ey][ex] = pp1;
        s.u[ey][ex] = up1[0]; s.v[ey][ex] = up1[1]; s.w[ey][ex] = up1[2]; s.tem[ey][ex] = up1[3];
      }
      if (!kPrefetchQ) load_q<T>(Qs, fe, qcol + (unsigned)(t + 1 - kr) * sk, qa);  // plane t+1 of the own column
      if (h_ok) {
        T hu[4], hp;
        if (!kPrefetchRing) load_q<T>(Qs, fe, hcol + (unsigned)(t - kr) * sk, hq);
        prims(P, hq, hu, hp);
#pragma unroll
        for (int c = 0; c < 5; ++c) sq[c][hy2][hx2] = hq[c];
        s.p[hy2][hx2] = hp;
        s.u[hy2][hx2] = hu[0]; s.v[hy2][hx2] = hu[1]; s.w[hy2][hx2] = hu[2]; s.tem[hy2][hx2] = hu[3];
      }
      wait_vm<0>();  // metrics of plane t, helper ring, plane t+1 of the own column
      lds_barrier();

      // ---- C: node work at plane t ----
      // the face between the axis and j = 1 takes the cross-axis value by
      // linear extrapolation (no five-point stencil across the axis): the
      // halo row below the axis holds 2 Q(0) - Q(1) for the dissipation of
      // phase E (its pressure, velocity and temperature keep the cross-axis
      // values for the sensor and the gradients; the row's own fluxes serve
      // only the axis, whose residual is not formed)
      if ((EXT & kExtAxis) && j == -1 && load_ok && kq->axis) {
#pragma unroll
        for (int c = 0; c < 5; ++c) sq[c][ey][ex] = T(2) * sq[c][ey + 1][ex] - sq[c][ey + 2][ex];
      }
      prims(P, qa, up1, pp1);  // plane t+1 of the own column
      // Q^(0) rows of the plane finished in this iteration (t-1), needed in E
      if (t > kb)
        dma_rows<5>((const char*)(Q0 + lane_el + (long long)(t - 1) * L.sk), fstep2, &q0w[wave][0][0][0], lane);
      T hz[5] = {0, 0, 0, 0, 0};
      T lz = 0, nz = 0;
      double Jn = 0.0;
      T mt[9];
      Jn = mbw[wave][9][ty1][tx];
#pragma unroll
      for (int c = 0; c < 9; ++c) mt[c] = (T)mbw[wave][c][ty1][tx];
      wait_lgkm_all();  // the wave's metric reads are done before its copies overwrite them
      // issue the next plane's loads now so that they land during C and E:
      // helper ring (FP32 path), then the wave's metric rows (five copies)
      if (kPrefetchRing && h_ok && t < ke) load_q<T>(Qs, fe, hcol + (unsigned)(t + 1 - kr) * sk, hq);
      if (node_t) {
        const T Jt = (T)Jn;
        T g[4][3];
        {
          // derivatives along xi, eta (LDS) and zeta (registers), chain rule
          const T(*F[4])[EX] = {s.u, s.v, s.w, s.tem};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const T dx = T(0.5) * (F[q][ey][ex + 1] - F[q][ey][ex - 1]);
            const T dy = T(0.5) * (F[q][ey + 1][ex] - F[q][ey - 1][ex]);
            const T dz = T(0.5) * (up1[q] - um1[q]);
#pragma unroll
            for (int x = 0; x < 3; ++x) g[q][x] = Jt * (mt[x] * dx + mt[3 + x] * dy + mt[6 + x] * dz);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
        const T s11 = g[0][0], s22 = g[1][1], s33 = g[2][2];
        const T s12 = T(0.5) * (g[0][1] + g[1][0]);
        const T s13 = T(0.5) * (g[0][2] + g[2][0]);
        const T s23 = T(0.5) * (g[1][2] + g[2][1]);
        const T skk3 = (s11 + s22 + s33) * T(1.0 / 3.0);
        const T rho = sq[0][ey][ex];
        const T u = s.u[ey][ex], vv = s.v[ey][ex], w = s.w[ey][ex];
        const T tn = s.tem[ey][ex];
        const T mu = sutherland_fast(tn, P);
        T mus = T(0), kaps = T(0), pis = T(0);
        if (P.sgs) {
          const T ss = s11 * s11 + s22 * s22 + s33 * s33 + T(2) * (s12 * s12 + s13 * s13 + s23 * s23);
          T d2 = (T)icbrt(Jn);  // (1/J)^(1/3)
          d2 *= d2;
          const T rd = rho * d2 * sqrt_nn(T(2) * ss);
          if (!(EXT & kExtSgs) || P.sgs == 1) {
            mus = T(P.Cs2) * rd;
            kaps = mus * T(P.Cp_over_Prsgs);
          } else {  // dynamic coefficients of this column
            const long long cc = dyn_col(kq->L, i, j);
            mus = T(kq->dyn[cc]) * rd;
            kaps = T(P.Cp) * T(kq->dyn[dyn_ncol(kq->L) + cc]) * rd;
          }
          // isotropic SGS stress: sigma_kk / 3, added to the pressure of the fluxes
          if ((EXT & kExtSgs) && P.CI43 != 0.0) pis = T(P.CI43) * rho * d2 * ss;
        }
        const T mt2 = T(2) * (mu + mus);
        const T t11 = mt2 * (s11 - skk3), t22 = mt2 * (s22 - skk3), t33 = mt2 * (s33 - skk3);
        const T t12 = mt2 * s12, t13 = mt2 * s13, t23 = mt2 * s23;
        const T kap = mu * T(P.Cp_over_Pr) + kaps;
        const T th0 = u * t11 + vv * t12 + w * t13 + kap * g[3][0];
        const T th1 = u * t12 + vv * t22 + w * t23 + kap * g[3][1];
        const T th2 = u * t13 + vv * t23 + w * t33 + kap * g[3][2];
        __builtin_amdgcn_sched_barrier(0);
        const T p = s.p[ey][ex];
        const T pe = (EXT & kExtSgs) ? p + pis : p;  // pressure of the fluxes
        const T c2 = T(P.gamma_R) * tn;  // c^2 = gamma p / rho = gamma R T
        // spectral radii of the three directions and their square roots
        T lam[3], U[3], sl[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const T mx = mt[3 * e], my = mt[3 * e + 1], mz = mt[3 * e + 2];
          U[e] = mx * u + my * vv + mz * w;
          lam[e] = fabs(U[e]) + sqrt_pos(c2 * (mx * mx + my * my + mz * mz));
          sl[e] = sqrt_pos(lam[e]);
        }
        // anisotropic scaling Lam_d = lam_d [1 + sum_e (lam_e / lam_d)^alpha]
        auto aniso_n = [&](int d, int e, int f) -> T {
          if (P.alpha_half) return lam[d] + sl[d] * (sl[e] + sl[f]);
          return aniso(lam[d], lam[e], lam[f], P);
        };
        auto node_flux = [&](int e, T H[5]) {
          const T mx = mt[3 * e], my = mt[3 * e + 1], mz = mt[3 * e + 2];
          const T Ue = U[e];
          H[0] = rho * Ue;
          H[1] = sq[1][ey][ex] * Ue + mx * pe - (mx * t11 + my * t12 + mz * t13);
          H[2] = sq[2][ey][ex] * Ue + my * pe - (mx * t12 + my * t22 + mz * t23);
          H[3] = sq[3][ey][ex] * Ue + mz * pe - (mx * t13 + my * t23 + mz * t33);
          H[4] = (sq[4][ey][ex] + pe) * Ue - (mx * th0 + my * th1 + mz * th2);
        };
        __builtin_amdgcn_sched_barrier(0);
        if (nx_t) {
          T H[5];
          node_flux(0, H);
#pragma unroll
          for (int q = 0; q < 5; ++q) s.hx[q][ty - 1][tx] = H[q];
          s.lx[ty - 1][tx] = aniso_n(0, 1, 2);
          const T pa = s.p[ey][ex + 1], pb = s.p[ey][ex - 1];
          s.nx[ty - 1][tx] = fabs(pa - T(2) * p + pb) * rcp_nr(pa + T(2) * p + pb);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ny_t) {
          T H[5];
          node_flux(1, H);
          // on the polar axis eta/J = 0: the eta node flux and radius take
          // their limit 0 (J is infinite there)
          const bool on_axis = (EXT & kExtAxis) && kq->axis && j == 0;
#pragma unroll
          for (int q = 0; q < 5; ++q) s.hy[q][ty][tx - 1] = on_axis ? T(0) : H[q];
          s.ly[ty][tx - 1] = on_axis ? T(0) : aniso_n(1, 2, 0);
          const T pa = s.p[ey + 1][ex], pb = s.p[ey - 1][ex];
          s.ny[ty][tx - 1] = fabs(pa - T(2) * p + pb) * rcp_nr(pa + T(2) * p + pb);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (out_ok) {
          node_flux(2, hz);
          lz = aniso_n(2, 0, 1);
          nz = fabs(pp1 - T(2) * p + pm1) * rcp_nr(pp1 + T(2) * p + pm1);
        }
      }
      lds_barrier();

      double q0v[5] = {0, 0, 0, 0, 0};
      if (t > kb) {
        wait_vm<0>();  // the Q^(0) copies (issued in C)
#pragma unroll
        for (int c = 0; c < 5; ++c) q0v[c] = q0w[wave][c][ty1][tx];
      }
      // the wave's metric rows of the next plane, landing during E (which
      // stores nothing to LDS); read at C of the next plane
      if (t < ke)
        dma_rows<10>((const char*)(kq->M + lane_el + (long long)(t + 1) * L.sk), fstep2, &mbw[wave][0][0][0], lane);
      if (kPrefetchQ && t < ke) load_q<T>(Qs, fe, qcol + (unsigned)(t + 2 - kr) * sk, qn);  // consumed at C of t+1

      // ---- E: residual (tile nodes) ----
      if (out_ok) {
        const int cx = tx - 1, cy = ty - 1;  // tile-local column / row
        T r[5] = {0, 0, 0, 0, 0};
        if (inner) {
          // central differences of the in-plane node fluxes
#pragma unroll
          for (int q = 0; q < 5; ++q)
            r[q] = T(0.5) * (s.hx[q][cy][tx + 1] - s.hx[q][cy][tx - 1]) +
                   T(0.5) * (s.hy[q][ty + 1][cx] - s.hy[q][ty - 1][cx]);
          // in-plane dissipation faces
          T q_a[5], q_b[5], q_c[5], q_d[5], q_e[5], D1[5], D0[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            q_a[c] = sq[c][ey][ex - 2]; q_b[c] = sq[c][ey][ex - 1]; q_c[c] = sq[c][ey][ex];
            q_d[c] = sq[c][ey][ex + 1]; q_e[c] = sq[c][ey][ex + 2];
          }
          face_diss(P, s.lx[cy][tx], s.lx[cy][tx + 1], s.nx[cy][tx], s.nx[cy][tx + 1], q_b, q_c, q_d, q_e, D1);
          face_diss(P, s.lx[cy][tx - 1], s.lx[cy][tx], s.nx[cy][tx - 1], s.nx[cy][tx], q_a, q_b, q_c, q_d, D0);
#pragma unroll
          for (int c = 0; c < 5; ++c) r[c] -= D1[c] - D0[c];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            q_a[c] = sq[c][ey - 2][ex]; q_b[c] = sq[c][ey - 1][ex];
            q_d[c] = sq[c][ey + 1][ex]; q_e[c] = sq[c][ey + 2][ex];
          }
          face_diss(P, s.ly[ty][cx], s.ly[ty + 1][cx], s.ny[ty][cx], s.ny[ty + 1][cx], q_b, q_c, q_d, q_e, D1);
          face_diss(P, s.ly[ty - 1][cx], s.ly[ty][cx], s.ny[ty - 1][cx], s.ny[ty][cx], q_a, q_b, q_c, q_d, D0);
#pragma unroll
          for (int c = 0; c < 5; ++c) r[c] -= D1[c] - D0[c];
        }
        __builtin_amdgcn_sched_barrier(0);
        // CFL only: the nine metric terms of the node finished in this
        // iteration (plane t-1), read back through the caches (they were
        // copied to LDS two planes ago); consumed after the update
        double cm[9];
        if (CFL) {
          const unsigned n = (out_ok && t > kb) ? nt - sk : qcol;
#pragma unroll
          for (int c = 0; c < 9; ++c) cm[c] = ldo(kq->M + sb + c * fe, n);
        }
        if (t >= kb) {
          // zeta face t - 1/2 between plane t-1 and plane t
          T qc[5], D[5], fz[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) qc[c] = sq[c][ey][ex];
          face_diss(P, lz_prev, lz, nz_prev, nz, qm2, qm1, qc, qa, D);
#pragma unroll
          for (int c = 0; c < 5; ++c) fz[c] = T(0.5) * (hz_prev[c] + hz[c]) - D[c];
          __builtin_amdgcn_sched_barrier(0);
          if (t > kb) {
            // residual of plane t-1 and its stage update
            const int k = t - 1;
            const unsigned n = nt - sk;
            double qnv[5];
            const bool on_axis = (EXT & kExtAxis) && kq->axis && j == 0;  // advanced by the centerline condition
#pragma unroll
            for (int c = 0; c < 5; ++c) {
              double R = J_prev * (double)(racc[c] + fz[c]);
              if (kq->f && i == kq->i_f) R -= kq->f[((long long)c * kq->L.nk + k) * kq->L.nj + j];
              if (on_axis) R = 0.0;
              const double qn = q0v[c] - adt * R;
              qnv[c] = qn;
              if (Qout) sto(Qout + sb + c * fe, n, qn);
              if (Qsh) sto(Qsh + sb + c * fe, n, (float)qn);
              if (NORM) {
                n2[c] += R * R;
                const double a = fabs(R);
                nm[c] = (a > nm[c] || a != a) ? a : nm[c];  // NaN wins so that it is reported
              }
            }
            if (CFL && !on_axis) cmin = min_nan(cmin, cfl_local(qnv[0], qnv[1], qnv[2], qnv[3], qnv[4], J_prev, cm, kq->P));
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
      // ---- shift the column queues (plane t values from LDS) ----
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        qm2[c] = qm1[c];
        qm1[c] = sq[c][ey][ex];
        qw[c] = qa[c];
        if (kPrefetchQ) qa[c] = qn[c];
      }
      um1[0] = s.u[ey][ex]; um1[1] = s.v[ey][ex]; um1[2] = s.w[ey][ex]; um1[3] = s.tem[ey][ex];
      pm1 = s.p[ey][ex];
      if (!kQ2) lds_barrier();
    }
  }

  // ---- block partial norms ----
  // (the wave's Q^(0) block is free: its last copy was waited for and read)
  if (NORM) {
    constexpr int QW = 5 * RPW * BX;  // doubles per wave in q0w
    norm_wave(n2, nm, &q0w[wave][0][0][0], lane);
    __syncthreads();
    if (tid < 10) {
      const double* red = &q0w[0][0][0][0];
      double r = red[tid];
      for (int w = 1; w < NW; ++w) {
        const double o = red[w * QW + tid];
        r = tid < 5 ? r + o : ((o > r || o != o) ? o : r);
      }
      part[(long long)v * 10 + tid] = r;
    }
  }
  // ---- block partial of the CFL bound (CFL only) ----
  if (CFL) {
    const double m = wave_min(cmin);
    double* red = &q0w[0][0][0][0];
    __syncthreads();  // every wave is past its last read of q0w
    if (lane == 0) red[wave] = m;
    __syncthreads();
    if (tid == 0) {
      double r = red[0];
      for (int w = 1; w < NW; ++w) r = min_nan(r, red[w]);
      cpart[v] = r;
    }
  }
}

}  // namespace

// The most planes one segment may march: its per-thread element offsets,
// taken from plane kb - 2, reach kc + 6 planes and must stay below 2^29
// (32-bit byte offsets of doubles).  0 when even one plane is too large.
int stage_kmax(const Layout& L) {
  const long long k = (1LL << 29) / L.sk - 6;
  return k < 1 ? 0 : (k > (1 << 30) ? (1 << 30) : (int)k);
}

namespace {

// Stage kernel configuration for a layout.
struct Config {
  int ntx, nty, nblocks, grid, per_xcd, kc, rr, nxcd;
  long long total, per_block, nseg;
};

long long auto_per_block(const Layout& L, const Machine& m) {
  const long long tiles = (long long)((L.ni + TX - 1) / TX) * ((L.nj + TY - 1) / TY);
  const long long total = tiles * L.nk;
  // one persistent block per resident slot (BPC per CU), at least 8 planes each
  const long long slots = (long long)m.cus * BPC;
  long long pb = (total + slots - 1) / slots;
  return pb < 8 ? 8 : pb;
}

Config config(const Layout& L, long long per_block, const Machine& m) {
  Config c;
  c.ntx = (L.ni + TX - 1) / TX;
  c.nty = (L.nj + TY - 1) / TY;
  c.total = (long long)c.ntx * c.nty * L.nk;
  c.per_block = per_block < 1 ? 1 : per_block;
  c.rr = c.per_block > L.nk;
  c.nseg = 0;
  const int kmax = stage_kmax(L);
  if (!c.rr) {
    c.kc = (int)(c.per_block < kmax ? c.per_block : kmax);
    c.nblocks = (int)((c.total + c.per_block - 1) / c.per_block);
  } else {
    // the number of k chunks (from the fewest whose chunks fit the 32-bit
    // offsets, at most 16 more, chunks of at least 32 planes when nk allows)
    // that best fills whole rounds of the blocks there are slots for; fewer
    // chunks on ties (fewer segment start-ups)
    const long long ntiles = (long long)c.ntx * c.nty;
    const long long slots = (c.total + c.per_block - 1) / c.per_block;
    const int n0 = (L.nk + kmax - 1) / kmax;
    double best = -1.0;
    for (int n = n0; n <= n0 + 15; ++n) {
      const int kc = (L.nk + n - 1) / n;
      if (n > n0 && kc < 32) break;
      const long long nseg = ntiles * ((L.nk + kc - 1) / kc);
      const long long nb = nseg < slots ? nseg : slots;
      const long long rounds = (nseg + nb - 1) / nb;
      const double eff = (double)nseg / (double)(rounds * nb);
      if (eff > best + 1e-9) {
        best = eff;
        c.kc = kc;
        c.nseg = nseg;
        c.nblocks = (int)nb;
      }
    }
  }
  // hardware block b runs on XCD b mod xcds: virtual block (b mod xcds)
  // per_xcd + b / xcds, so consecutive virtual blocks share an XCD
  c.nxcd = m.xcds;
  c.per_xcd = (c.nblocks + c.nxcd - 1) / c.nxcd;
  c.grid = c.per_xcd * c.nxcd;
  return c;
}

template <class T, class QI, int EXT>
hipError_t launch_x(hipStream_t st, const Config& c, const KArgs& a, const QI* Qin, const double* Q0, double* Qout,
                    float* Qsh, const double* dtp, double dt, double alpha, double* part, double* cpart) {
  if (part)
    k_stage<T, QI, true, false, EXT><<<c.grid, NT, 0, st>>>(a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
  else if (cpart)
    k_stage<T, QI, false, true, EXT><<<c.grid, NT, 0, st>>>(a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
  else
    k_stage<T, QI, false, false, EXT><<<c.grid, NT, 0, st>>>(a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
  return hipGetLastError();
}

template <class T, class QI>
hipError_t launch(hipStream_t st, const StageArgs& sa, const QI* Qin, const double* Q0, double* Qout, float* Qsh,
                  const double* dtp, double dt, double alpha, double* part, double* cpart) {
  if (part && cpart) return hipErrorInvalidValue;  // norms belong to stage 1, the CFL bound to stage 5
  Config c = config(sa.L, sa.kchunk, sa.mach);
  KArgs a{sa.L,        sa.P,   sa.M,   sa.f,   sa.dyn,  sa.axis,  sa.i_f,    c.ntx,    c.nty,
          c.total,     c.per_block, c.kc, c.rr, c.nseg, c.nblocks, c.per_xcd, c.nxcd};
  // the optional SGS models (dynamic closure, isotropic SGS stress) and the
  // polar axis run in instantiations of their own, so that each path keeps
  // only the registers it needs
  const int x = ((sa.P.sgs == 2 || sa.P.CI43 != 0.0) ? kExtSgs : 0) | (sa.axis ? kExtAxis : 0);
  if ((x & kExtSgs) && sa.P.sgs == 2 && !sa.dyn) return hipErrorInvalidValue;
  switch (x) {
    case 0: return launch_x<T, QI, 0>(st, c, a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
    case kExtSgs: return launch_x<T, QI, kExtSgs>(st, c, a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
    case kExtAxis: return launch_x<T, QI, kExtAxis>(st, c, a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
    default:
      return launch_x<T, QI, kExtSgs | kExtAxis>(st, c, a, Qin, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
  }
}

}  // namespace

int stage_kchunk(const Layout& L, const Machine& m) {
  const char* env = getenv("LES_SEG");
  if (env && atoi(env) > 0) return atoi(env);
  return (int)auto_per_block(L, m);
}

long long stage_blocks(const Layout& L, int kchunk, const Machine& m) { return config(L, kchunk, m).nblocks; }

hipError_t launch_stage_fp64(hipStream_t s, const StageArgs& a, const double* Qin, const double* Q0, double* Qout,
                             const double* dtp, double dt, double alpha, double* part, double* cpart) {
  return launch<double, double>(s, a, Qin, Q0, Qout, nullptr, dtp, dt, alpha, part, cpart);
}

hipError_t launch_stage_mixed(hipStream_t s, const StageArgs& a, const double* Qin64, const float* Qin32,
                              const double* Q0, double* Qout, float* Qsh, const double* dtp, double dt, double alpha,
                              double* part, double* cpart) {
  if (Qin64) return launch<float, double>(s, a, Qin64, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
  return launch<float, float>(s, a, Qin32, Q0, Qout, Qsh, dtp, dt, alpha, part, cpart);
}

}  // namespace les
