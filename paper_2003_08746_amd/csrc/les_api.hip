// les_api.hip -- implementation of the C ABI declared in include/les.h.
//
// Host code only: argument checks, device allocations owned by the context,
// and the launch sequence of one residual evaluation / one five-stage
// Runge-Kutta step (Sec. 4, Alg. 2) on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "les.h"
#include "les_debug.h"
#include "les_launch.hpp"
#include "les_stage.hpp"
#include "les_adjoint.hpp"
#include "les_dynamic.hpp"

// Scratch of les_residual_noalloc: LES_NOALLOC_BLOCKS per-block norm
// partials (10 doubles each) and one flag word.  One copy per GPU, held
// until the process ends.  Host code never uses this name as an address: the
// per-device address comes from hipGetSymbolAddress (scratch_on) and is
// what the kernels get.
constexpr long long kScratchDoubles = 10LL * LES_NOALLOC_BLOCKS + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static double* g_scratch_at[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of this device's scratch (the device must be current);
// resolved once per device.
static hipError_t scratch_on(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_at[device] = (double*)p;
  }
  *out = g_scratch_at[device];
  return hipSuccess;
}

struct les_ctx {
  les::Layout L;
  les::Phys P;
  int bc[3];
  int prec;
  hipStream_t s;
  int device;
  double* M = nullptr;               // metrics [10][fe]
  double* S[2] = {nullptr, nullptr}; // FP64 stage buffers [5][fe]
  float* Sf[2] = {nullptr, nullptr}; // FP32 stage buffers [5][fe] (mixed precision)
  double* f = nullptr;               // source [5][nk][nj]
  int i_f = -1;
  double* part = nullptr;            // per-block reduction partials
  long long part_n = 0;              // capacity in blocks (10 doubles each)
  double* cpart = nullptr;           // per-block CFL bounds from the last stage (stage_blocks doubles)
  double* dthist = nullptr;          // time steps of one les_advance call (LES_ADVANCE_DT_MAX doubles)
  double* scal = nullptr;            // [0] dt, [1..10] norms, [12] dt of the next step (les_advance)
  int* flag = nullptr;               // bit 0: bad dt, bit 1: non-finite norm
  double* dyn = nullptr;             // dynamic SGS coefficients per column [2][ncol] (sgs == 2)
  double* dynw = nullptr;            // work arrays of the dynamic closure
  double* adj = nullptr;             // adjoint work arrays
  long long adj_n = 0;
  int face[6] = {0, 0, 0, 0, 0, 0};  // boundary-face types (les_set_face)
  double p_exit[6] = {0, 0, 0, 0, 0, 0};
  double* outside = nullptr;         // [5][fe] outside state of characteristic faces
  int axis = 0;                      // j = 0 is the polar axis of an O-grid (bc[1] == LES_BC_AXIS)
  int use_ref = 0;                   // 1: stage through the reference kernel
  int kchunk = 0;                    // k planes per block of the fused kernel
  les::Machine mach;                 // CU and XCD counts of the device
  double* scratch = nullptr;         // this device's les_residual_noalloc scratch
  // optional HIP-event timing of every stage-kernel launch
  int timing = 0;
  static const int TMAX = 4096;
  hipEvent_t ev[2 * 4096];
  int nev = 0;                       // events created
  int nrec = 0;                      // launches recorded since the last read
  double t_ms = 0.0;                 // resolved total
  long long t_cnt = 0;
  char err[512];
};

static thread_local char g_create_err[512] = "";

static les::Faces faces_of(const les_ctx* c) {
  les::Faces F;
  F.any = 0;
  for (int f = 0; f < 6; ++f) {
    F.type[f] = c->face[f];
    F.p_exit[f] = c->p_exit[f];
    if (c->face[f] != LES_FACE_FROZEN) F.any = 1;
  }
  F.outside = c->outside;
  F.M = c->M;
  F.gamma = c->P.gamma;
  F.axis = c->axis;
  return F;
}

static int fail(les_ctx* c, int code, const char* fmt, ...) {
  char* buf = c ? c->err : g_create_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(ctx, call)                                                                        \
  do {                                                                                           \
    hipError_t e_ = (call);                                                                      \
    if (e_ != hipSuccess) return fail((ctx), LES_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static void free_all(les_ctx* c) {
  if (!c) return;
  for (int e = 0; e < c->nev; ++e) (void)hipEventDestroy(c->ev[e]);
  c->nev = 0;
  (void)hipFree(c->M);
  (void)hipFree(c->S[0]);
  (void)hipFree(c->S[1]);
  (void)hipFree(c->Sf[0]);
  (void)hipFree(c->Sf[1]);
  (void)hipFree(c->f);
  (void)hipFree(c->part);
  (void)hipFree(c->cpart);
  (void)hipFree(c->dthist);
  (void)hipFree(c->outside);
  (void)hipFree(c->scal);
  (void)hipFree(c->flag);
  (void)hipFree(c->adj);
  (void)hipFree(c->dyn);
  (void)hipFree(c->dynw);
}

// Boundary update of an FP64 state before a residual evaluation: the
// centerline condition on the axis nodes (O-grid), then the ghost layers.
static hipError_t bc_fill(les_ctx* c, double* Q) {
  if (c->axis) {
    hipError_t e = les::launch_axis_avg(c->s, c->L, Q);
    if (e != hipSuccess) return e;
  }
  return les::launch_ghost_fill(c->s, c->L, c->bc, Q, Q, 5, faces_of(c));
}

// Dynamic SGS coefficients of the state about to be differenced (its
// ghosts filled), when the context uses the dynamic closure.
static hipError_t dyn_update(les_ctx* c, const double* Q64, const float* Q32) {
  if (c->P.sgs != 2) return hipSuccess;
  return Q32 ? les::launch_dynamic_f32(c->s, c->L, c->bc, c->P, c->M, Q32, c->dynw, c->dyn)
             : les::launch_dynamic(c->s, c->L, c->bc, c->P, c->M, Q64, c->dynw, c->dyn);
}

// Resolve recorded event pairs into the running total (synchronises).
static int resolve_timing(les_ctx* c) {
  if (c->nrec == 0) return LES_OK;
  HIPCHK(c, hipEventSynchronize(c->ev[2 * c->nrec - 1]));
  for (int r = 0; r < c->nrec; ++r) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * r], c->ev[2 * r + 1]));
    c->t_ms += ms;
  }
  c->t_cnt += c->nrec;
  c->nrec = 0;
  return LES_OK;
}

static int timing_begin(les_ctx* c) {
  if (!c->timing) return LES_OK;
  if (c->nrec == les_ctx::TMAX) {
    int rc = resolve_timing(c);
    if (rc != LES_OK) return rc;
  }
  while (c->nev < 2 * (c->nrec + 1)) {
    HIPCHK(c, hipEventCreate(&c->ev[c->nev]));
    c->nev++;
  }
  HIPCHK(c, hipEventRecord(c->ev[2 * c->nrec], c->s));
  return LES_OK;
}

static int timing_end(les_ctx* c) {
  if (!c->timing) return LES_OK;
  HIPCHK(c, hipEventRecord(c->ev[2 * c->nrec + 1], c->s));
  c->nrec++;
  return LES_OK;
}

// Adjoint work arrays are allocated on first use and kept by the context.
static int ensure_adj_work(les_ctx* c) {
  // the adjoint passes index nodes and faces (about three per node) with
  // 32-bit integers (their work arrays limit the block far below that anyway)
  const long long box = (long long)(c->L.ni + 4) * (c->L.nj + 4) * (c->L.nk + 4);
  if (box >= (1LL << 30))
    return fail(c, LES_ERR_STATE, "adjoint: block too large (%lld padded nodes, limit 2^30)", box);
  const size_t need = les::adjoint_work_elems(c->L);
  if ((long long)need <= c->adj_n) return LES_OK;
  (void)hipFree(c->adj);
  c->adj = nullptr;
  c->adj_n = 0;
  if (hipMalloc(&c->adj, need * sizeof(double)) != hipSuccess)
    return fail(c, LES_ERR_NOMEM, "adjoint work allocation (%zu bytes)", need * sizeof(double));
  c->adj_n = (long long)need;
  return LES_OK;
}

extern "C" {

const char* les_last_create_error(void) { return g_create_err; }

const char* les_last_error(const les_ctx* ctx) { return ctx ? ctx->err : g_create_err; }

int les_layout_for(int ni, int nj, int nk, long long strides[3], long long* origin, long long* field_elems,
                   int* ghost) {
  if (ni < 5 || nj < 5 || nk < 5) return fail(nullptr, LES_ERR_ARG, "les_layout_for: sizes must be >= 5");
  les::Layout L = les::make_layout(ni, nj, nk);
  if (strides) {
    strides[0] = 1;
    strides[1] = L.sj;
    strides[2] = L.sk;
  }
  if (origin) *origin = L.o;
  if (field_elems) *field_elems = L.fe;
  if (ghost) *ghost = les::GH;
  return LES_OK;
}

int les_layout(const les_ctx* ctx, long long strides[3], long long* origin, long long* field_elems, int* ghost) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_layout: null context");
  if (strides) {
    strides[0] = 1;
    strides[1] = ctx->L.sj;
    strides[2] = ctx->L.sk;
  }
  if (origin) *origin = ctx->L.o;
  if (field_elems) *field_elems = ctx->L.fe;
  if (ghost) *ghost = les::GH;
  return LES_OK;
}

int les_create(les_ctx** out, const les_grid* grid, const les_metrics* metrics, const les_flow_params* prm,
               void* hip_stream) {
  const double* metrics_dense = metrics ? metrics->m : nullptr;
  if (!out) return fail(nullptr, LES_ERR_ARG, "les_create: out is NULL");
  *out = nullptr;
  if (!grid || !prm) return fail(nullptr, LES_ERR_ARG, "les_create: grid or params is NULL");
  if (grid->ni < 5 || grid->nj < 5 || grid->nk < 5)
    return fail(nullptr, LES_ERR_ARG, "les_create: every interior size must be >= 5 (got %d x %d x %d)", grid->ni,
                grid->nj, grid->nk);
  {
    // the stage kernel takes 32-bit per-thread offsets from a 64-bit base
    // per segment of k planes: a segment of a few planes must fit them
    les::Layout Lc = les::make_layout(grid->ni, grid->nj, grid->nk);
    if (les::stage_kmax(Lc) < 1)
      return fail(nullptr, LES_ERR_ARG,
                  "les_create: k plane too large (%lld elements with padding; 7 planes must stay below 2^29)", Lc.sk);
  }
  for (int d = 0; d < 3; ++d)
    if (grid->bc[d] != LES_BC_PERIODIC && grid->bc[d] != LES_BC_DIRICHLET && grid->bc[d] != LES_BC_PERIODIC_SUPERPOSED &&
        !(d == 1 && grid->bc[d] == LES_BC_AXIS))
      return fail(nullptr, LES_ERR_ARG, "les_create: bc[%d] = %d is not a known boundary type for that direction", d,
                  grid->bc[d]);
  if (grid->bc[1] == LES_BC_AXIS && (grid->bc[2] != LES_BC_PERIODIC_SUPERPOSED || (grid->nk - 1) % 2 != 0))
    return fail(nullptr, LES_ERR_ARG, "les_create: the axis needs a superposed periodic k direction with nk - 1 even");
  if (!metrics_dense && !grid->xyz) return fail(nullptr, LES_ERR_ARG, "les_create: need xyz or metrics");
  if (!(prm->gamma > 1.0) || !(prm->R_gas > 0.0) || !(prm->Pr > 0.0) || !(prm->Pr_sgs > 0.0) ||
      !(prm->mu_ref >= 0.0) || !(prm->T_ref > 0.0) || !(prm->S_suth >= 0.0) || !(prm->k2 >= 0.0) ||
      !(prm->k4 >= 0.0) || !(prm->alpha > 0.0) || !(prm->cfl > 0.0) || !(prm->Cs >= 0.0) ||
      (prm->sgs != 0 && prm->sgs != 1 && prm->sgs != 2) || !(prm->CI >= 0.0))
    return fail(nullptr, LES_ERR_ARG, "les_create: a flow parameter is out of range");
  if (prm->prec != LES_FP64 && prm->prec != LES_MIXED)
    return fail(nullptr, LES_ERR_ARG, "les_create: unknown precision %d", prm->prec);

  les_ctx* c = new les_ctx();
  c->err[0] = 0;
  c->L = les::make_layout(grid->ni, grid->nj, grid->nk);
  for (int d = 0; d < 3; ++d) c->bc[d] = grid->bc[d];
  c->axis = grid->bc[1] == LES_BC_AXIS;
  c->prec = prm->prec;
  c->s = (hipStream_t)hip_stream;
  les::Phys& P = c->P;
  P.gamma = prm->gamma;
  P.gm1 = prm->gamma - 1.0;
  P.inv_R = 1.0 / prm->R_gas;
  const double Cp = prm->gamma * prm->R_gas / (prm->gamma - 1.0);
  P.Cp_over_Pr = Cp / prm->Pr;
  P.Cp_over_Prsgs = Cp / prm->Pr_sgs;
  P.mu_ref = prm->mu_ref;
  P.inv_Tref = 1.0 / prm->T_ref;
  P.S = prm->S_suth;
  P.one_plus_S = 1.0 + prm->S_suth;
  P.Cs2 = prm->Cs * prm->Cs;
  P.k2 = prm->k2;
  P.k4 = prm->k4;
  P.alpha = prm->alpha;
  P.alpha_half = prm->alpha == 0.5;
  P.gamma_R = prm->gamma * prm->R_gas;
  P.cfl = prm->cfl;
  P.nu_fac = fmax(4.0 / 3.0, prm->gamma / prm->Pr);
  P.sgs = prm->sgs;
  P.CI43 = prm->sgs ? 4.0 / 3.0 * prm->CI : 0.0;
  P.Cp = Cp;

  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, LES_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  e = scratch_on(c->device, &c->scratch);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, LES_ERR_HIP, "les_create: scratch address on device %d: %s", c->device,
                hipGetErrorString(e));
  }
  const size_t fe = (size_t)c->L.fe;
  {
    int cus = 0, xcds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
      c->mach.cus = cus;
    if (hipDeviceGetAttribute(&xcds, hipDeviceAttributeNumberOfXccs, c->device) == hipSuccess && xcds > 0)
      c->mach.xcds = xcds;
    else
      c->mach.xcds = 1;
  }
  c->kchunk = les::stage_kchunk(c->L, c->mach);
  // partials of the reference kernel, the fused kernel and the CFL kernel
  c->part_n = les::ref_blocks(c->L);
  const long long sb = les::stage_blocks(c->L, c->kchunk, c->mach), cb = les::cfl_blocks(c->L);
  if (sb > c->part_n) c->part_n = sb;
  if (cb > c->part_n) c->part_n = cb;
  bool ok = hipMalloc(&c->M, 10 * fe * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->S[0], 5 * fe * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->S[1], 5 * fe * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->part, (size_t)c->part_n * 10 * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->cpart, (size_t)sb * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->dthist, (size_t)LES_ADVANCE_DT_MAX * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->scal, 16 * sizeof(double)) == hipSuccess && hipMalloc(&c->flag, sizeof(int)) == hipSuccess;
  if (ok && c->prec == LES_MIXED)
    ok = hipMalloc(&c->Sf[0], 5 * fe * sizeof(float)) == hipSuccess &&
         hipMalloc(&c->Sf[1], 5 * fe * sizeof(float)) == hipSuccess;
  if (ok && prm->sgs == 2)
    ok = hipMalloc(&c->dyn, 2 * les::dyn_ncol(c->L) * sizeof(double)) == hipSuccess &&
         hipMalloc(&c->dynw, les::dynamic_work_elems(c->L) * sizeof(double)) == hipSuccess;
  if (!ok) {
    free_all(c);
    delete c;
    return fail(nullptr, LES_ERR_NOMEM, "les_create: device allocation failed (%zu bytes per field)",
                fe * sizeof(double));
  }
  int rc = LES_OK;
  do {
    if (hipMemsetAsync(c->M, 0, 10 * fe * sizeof(double), c->s) != hipSuccess ||
        hipMemsetAsync(c->S[0], 0, 5 * fe * sizeof(double), c->s) != hipSuccess ||
        hipMemsetAsync(c->S[1], 0, 5 * fe * sizeof(double), c->s) != hipSuccess ||
        hipMemsetAsync(c->scal, 0, 16 * sizeof(double), c->s) != hipSuccess ||
        hipMemsetAsync(c->flag, 0, sizeof(int), c->s) != hipSuccess) {
      rc = fail(nullptr, LES_ERR_HIP, "les_create: hipMemsetAsync failed");
      break;
    }
    if (c->dynw && (hipMemsetAsync(c->dynw, 0, les::dynamic_work_elems(c->L) * sizeof(double), c->s) != hipSuccess ||
                    hipMemsetAsync(c->dyn, 0, 2 * les::dyn_ncol(c->L) * sizeof(double), c->s) != hipSuccess)) {
      rc = fail(nullptr, LES_ERR_HIP, "les_create: hipMemsetAsync failed");
      break;
    }
    if (c->Sf[0] && (hipMemsetAsync(c->Sf[0], 0, 5 * fe * sizeof(float), c->s) != hipSuccess ||
                     hipMemsetAsync(c->Sf[1], 0, 5 * fe * sizeof(float), c->s) != hipSuccess)) {
      rc = fail(nullptr, LES_ERR_HIP, "les_create: hipMemsetAsync failed");
      break;
    }
    e = metrics_dense ? les::launch_metrics_copy(c->s, c->L, metrics_dense, c->M)
                      : les::launch_metrics(c->s, c->L, c->bc, grid->xyz, c->M);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (e != hipSuccess) {
      rc = fail(nullptr, LES_ERR_HIP, "les_create: metrics: %s", hipGetErrorString(e));
      break;
    }
  } while (0);
  if (rc != LES_OK) {
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return LES_OK;
}

void les_destroy(les_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->s);
  free_all(ctx);
  delete ctx;
}

int les_get_metrics(les_ctx* ctx, double* dense_out) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_get_metrics: null context");
  if (!dense_out) return fail(ctx, LES_ERR_ARG, "les_get_metrics: null output");
  HIPCHK(ctx, les::launch_metrics_export(ctx->s, ctx->L, ctx->M, dense_out));
  HIPCHK(ctx, hipStreamSynchronize(ctx->s));
  return LES_OK;
}

// Read back the host outputs and the non-finite flag (synchronises).
static int sync_outputs(les_ctx* c, double* dt_out, double* norms) {
  double host[16];
  int flag = 0;
  HIPCHK(c, hipMemcpyAsync(host, c->scal, 16 * sizeof(double), hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->s));
  HIPCHK(c, hipStreamSynchronize(c->s));
  if (dt_out) *dt_out = host[0];
  if (norms)
    for (int q = 0; q < 10; ++q) norms[q] = host[1 + q];
  if (flag) {
    HIPCHK(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->s));
    return fail(c, LES_ERR_NONFINITE, "non-finite value detected (flag %d): %s", flag,
                (flag & 1) ? "time step (density/pressure not positive or NaN)" : "residual norm");
  }
  return LES_OK;
}

int les_residual(les_ctx* ctx, double* Q, double* R, double* norms) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_residual: null context");
  if (!Q || !R) return fail(ctx, LES_ERR_ARG, "les_residual: Q and R must be device pointers");
  if (Q == R) return fail(ctx, LES_ERR_ARG, "les_residual: Q and R must not alias");
  HIPCHK(ctx, bc_fill(ctx, Q));
  const double* f = ctx->i_f >= 0 ? ctx->f : nullptr;
  double* part = norms ? ctx->part : nullptr;
  long long nb;
  if (!ctx->use_ref && !(((uintptr_t)R) & 15)) {
    // the fused stage kernel with Q^(0) = R = 0 and alpha dt = -1 writes
    // 0 + R(Q) at every interior node (and reduces the norms of R)
    const les::Layout& L = ctx->L;
    HIPCHK(ctx, les::launch_zero(ctx->s, R, 5 * L.fe));
    HIPCHK(ctx, dyn_update(ctx, Q, nullptr));
    const les::StageArgs a{L, ctx->P, ctx->M, f, ctx->i_f, ctx->kchunk, ctx->dyn, ctx->axis, ctx->mach};
    HIPCHK(ctx, les::launch_stage_fp64(ctx->s, a, Q, R, R, nullptr, 1.0, -1.0, part, nullptr));
    nb = les::stage_blocks(L, ctx->kchunk, ctx->mach);
  } else {
    HIPCHK(ctx, dyn_update(ctx, Q, nullptr));
    HIPCHK(ctx, les::launch_residual_ref(ctx->s, ctx->L, ctx->P, ctx->M, Q, ctx->f, ctx->i_f, R, part, ctx->dyn,
                                         ctx->axis));
    nb = les::ref_blocks(ctx->L);
  }
  if (!norms) return LES_OK;
  const double cnt = (double)ctx->L.ni * ctx->L.nj * ctx->L.nk;
  HIPCHK(ctx, les::launch_norm_final(ctx->s, ctx->part, nb, cnt, ctx->scal + 1, ctx->flag));
  return sync_outputs(ctx, nullptr, norms);
}

int les_residual_noalloc(les_ctx* ctx, double* Q, double* R, double* norms_dev) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_residual_noalloc: null context");
  if (!Q || !R) return fail(ctx, LES_ERR_ARG, "les_residual_noalloc: Q and R must be device pointers");
  if (Q == R) return fail(ctx, LES_ERR_ARG, "les_residual_noalloc: Q and R must not alias");
  if (((uintptr_t)R) & 15) return fail(ctx, LES_ERR_ARG, "les_residual_noalloc: R must be 16-byte aligned");
  if (!ctx->scratch) return fail(ctx, LES_ERR_STATE, "les_residual_noalloc: no scratch on this device");
  const les::Layout& L = ctx->L;
  const long long nb = les::stage_blocks(L, ctx->kchunk, ctx->mach);
  if (nb > LES_NOALLOC_BLOCKS)
    return fail(ctx, LES_ERR_ARG, "les_residual_noalloc: %lld kernel blocks exceed the scratch's %d", nb,
                LES_NOALLOC_BLOCKS);
  HIPCHK(ctx, bc_fill(ctx, Q));
  HIPCHK(ctx, les::launch_zero(ctx->s, R, 5 * L.fe));
  const double* f = ctx->i_f >= 0 ? ctx->f : nullptr;
  HIPCHK(ctx, dyn_update(ctx, Q, nullptr));
  const les::StageArgs a{L, ctx->P, ctx->M, f, ctx->i_f, ctx->kchunk, ctx->dyn, ctx->axis, ctx->mach};
  double* part = norms_dev ? ctx->scratch : nullptr;
  HIPCHK(ctx, les::launch_stage_fp64(ctx->s, a, Q, R, R, nullptr, 1.0, -1.0, part, nullptr));
  if (norms_dev) {
    // the flag word after the partials is written but never read: a
    // non-finite residual shows as NaN in the norms
    int* flag = (int*)(ctx->scratch + 10LL * LES_NOALLOC_BLOCKS);
    const double cnt = (double)L.ni * L.nj * L.nk;
    HIPCHK(ctx, les::launch_norm_final(ctx->s, part, nb, cnt, norms_dev, flag));
  }
  return LES_OK;
}

int les_cfl_dt(les_ctx* ctx, const double* Q, double* dt_out) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_cfl_dt: null context");
  if (!Q || !dt_out) return fail(ctx, LES_ERR_ARG, "les_cfl_dt: null pointer");
  HIPCHK(ctx, les::launch_cfl(ctx->s, ctx->L, ctx->P, ctx->M, Q, ctx->part, ctx->scal, ctx->flag, nullptr,
                              ctx->axis));
  return sync_outputs(ctx, dt_out, nullptr);
}

int les_set_forcing(les_ctx* ctx, const double* f, int i_f) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_set_forcing: null context");
  if (!f) {
    ctx->i_f = -1;
    return LES_OK;
  }
  if (i_f < 0 || i_f >= ctx->L.ni) return fail(ctx, LES_ERR_ARG, "les_set_forcing: plane %d outside [0, %d)", i_f, ctx->L.ni);
  const size_t bytes = (size_t)5 * ctx->L.nk * ctx->L.nj * sizeof(double);
  if (!ctx->f && hipMalloc(&ctx->f, bytes) != hipSuccess) return fail(ctx, LES_ERR_NOMEM, "les_set_forcing: allocation");
  HIPCHK(ctx, hipMemcpyAsync(ctx->f, f, bytes, hipMemcpyDeviceToDevice, ctx->s));
  ctx->i_f = i_f;
  return LES_OK;
}

// One Runge-Kutta step on the context's stream: ghost fill of Q^n, five
// stages (time step read from dtp on the device when not null, else dt),
// norm reduction of R(Q^n).  cpart (or null): the last stage also reduces
// the per-block CFL bounds of Q^{n+1} into it (fused kernel only).
// One Runge-Kutta step of Q.  with_norms: stage 1 reduces the residual norms
// of R(Q^n) (and their non-finite flag); les_advance leaves them out of every
// step but its last, whose non-finite states the next step's dt reduction
// reports instead.
//
// Mixed precision: stage l writes its FP32 state to Sf[(l + par) & 1] and
// stage l + 1 reads it.  shadow_out: the last stage also writes the FP32
// copy of Q^{n+1} (to Sf[par]); shadow_in: stage 1 reads that copy (written
// by the step before, with the other par) for its stencil instead of
// converting the FP64 Q^n as it loads it -- the same FP32 values.
static int step_core(les_ctx* ctx, double* Q, const double* dtp, double dt, double* stage_ckpt, double* cpart,
                     bool with_norms = true, int par = 0, bool shadow_in = false, bool shadow_out = false) {
  les::Layout& L = ctx->L;
  const size_t fe = (size_t)L.fe;
  const double* f = ctx->i_f >= 0 ? ctx->f : nullptr;
  const double cnt = (double)L.ni * L.nj * L.nk;
  if (ctx->prec == LES_MIXED) {
    les::StageArgs a{L, ctx->P, ctx->M, f, ctx->i_f, ctx->kchunk, ctx->dyn, ctx->axis, ctx->mach};
    for (int l = 0; l < 5; ++l) {
      const float* in32 = (l == 0 && !shadow_in) ? nullptr : ctx->Sf[(l + 1 + par) & 1];
      float* out32 = (l < 4 || shadow_out) ? ctx->Sf[(l + par) & 1] : nullptr;
      if (l > 0 && ctx->axis) HIPCHK(ctx, les::launch_axis_avg_f32(ctx->s, L, (float*)in32));
      if (in32) HIPCHK(ctx, les::launch_ghost_fill_f32(ctx->s, L, ctx->bc, (float*)in32, Q, faces_of(ctx)));
      HIPCHK(ctx, dyn_update(ctx, in32 ? nullptr : Q, in32));
      int trc = timing_begin(ctx);
      if (trc != LES_OK) return trc;
      HIPCHK(ctx, les::launch_stage_mixed(ctx->s, a, in32 ? nullptr : Q, in32, Q, l == 4 ? Q : nullptr, out32, dtp,
                                          dt, les::rk_alpha(l), (l == 0 && with_norms) ? ctx->part : nullptr,
                                          l == 4 ? cpart : nullptr));
      trc = timing_end(ctx);
      if (trc != LES_OK) return trc;
    }
    if (ctx->axis) HIPCHK(ctx, les::launch_axis_avg(ctx->s, L, Q));
    if (with_norms)
      HIPCHK(ctx, les::launch_norm_final(ctx->s, ctx->part, les::stage_blocks(L, ctx->kchunk, ctx->mach), cnt,
                                         ctx->scal + 1, ctx->flag));
  } else {
    if (stage_ckpt) HIPCHK(ctx, hipMemcpyAsync(stage_ckpt, Q, 5 * fe * sizeof(double), hipMemcpyDeviceToDevice, ctx->s));
    const double* in = stage_ckpt ? stage_ckpt : Q;
    for (int l = 0; l < 5; ++l) {
      double* out = l == 4 ? Q : (stage_ckpt ? stage_ckpt + (size_t)(l + 1) * 5 * fe : ctx->S[l & 1]);
      if (l > 0 && ctx->axis) HIPCHK(ctx, les::launch_axis_avg(ctx->s, L, (double*)in));
      if (l > 0 || stage_ckpt) HIPCHK(ctx, les::launch_ghost_fill(ctx->s, L, ctx->bc, (double*)in, Q, 5, faces_of(ctx)));
      // the residual norms of R(Q^n) are reduced on the device (fused into
      // stage 1) whenever with_norms; only their copy to the host is optional
      double* part = (l == 0 && with_norms) ? ctx->part : nullptr;
      HIPCHK(ctx, dyn_update(ctx, in, nullptr));
      int trc = timing_begin(ctx);
      if (trc != LES_OK) return trc;
      if (ctx->use_ref) {
        HIPCHK(ctx, les::launch_stage_ref(ctx->s, L, ctx->P, ctx->M, in, Q, out, dtp, dt, les::rk_alpha(l), f,
                                          ctx->i_f, part, ctx->dyn, ctx->axis));
      } else {
        les::StageArgs a{L, ctx->P, ctx->M, f, ctx->i_f, ctx->kchunk, ctx->dyn, ctx->axis, ctx->mach};
        HIPCHK(ctx, les::launch_stage_fp64(ctx->s, a, in, Q, out, dtp, dt, les::rk_alpha(l), part,
                                           l == 4 ? cpart : nullptr));
      }
      trc = timing_end(ctx);
      if (trc != LES_OK) return trc;
      in = out;
    }
    if (ctx->axis) HIPCHK(ctx, les::launch_axis_avg(ctx->s, L, Q));
    long long nb = ctx->use_ref ? les::ref_blocks(L) : les::stage_blocks(L, ctx->kchunk, ctx->mach);
    if (with_norms) HIPCHK(ctx, les::launch_norm_final(ctx->s, ctx->part, nb, cnt, ctx->scal + 1, ctx->flag));
  }
  return LES_OK;
}

int les_rk_step(les_ctx* ctx, double* Q, double dt, double* dt_out, double* norms, double* stage_ckpt) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_rk_step: null context");
  if (!Q) return fail(ctx, LES_ERR_ARG, "les_rk_step: Q is NULL");
  if (((uintptr_t)Q) & 15) return fail(ctx, LES_ERR_ARG, "les_rk_step: Q must be 16-byte aligned");
  if (dt != dt) return fail(ctx, LES_ERR_ARG, "les_rk_step: dt is NaN");
  if (stage_ckpt && ctx->prec != LES_FP64)
    return fail(ctx, LES_ERR_STATE, "les_rk_step: stage checkpoints need an FP64 context");
  les::Layout& L = ctx->L;
  HIPCHK(ctx, bc_fill(ctx, Q));
  const double* dtp = nullptr;
  if (!(dt > 0.0)) {
    HIPCHK(ctx, les::launch_cfl(ctx->s, L, ctx->P, ctx->M, Q, ctx->part, ctx->scal, ctx->flag, nullptr, ctx->axis));
    dtp = ctx->scal;
  }
  int rc = step_core(ctx, Q, dtp, dt, stage_ckpt, nullptr);
  if (rc != LES_OK) return rc;
  if (!dt_out && !norms) return LES_OK;
  rc = sync_outputs(ctx, dt_out, norms);
  if (dt_out && dtp == nullptr) *dt_out = dt;
  return rc;
}

int les_advance(les_ctx* ctx, double* Q, int nsteps, double* dt_out, double* norms) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_advance: null context");
  if (!Q) return fail(ctx, LES_ERR_ARG, "les_advance: Q is NULL");
  if (((uintptr_t)Q) & 15) return fail(ctx, LES_ERR_ARG, "les_advance: Q must be 16-byte aligned");
  if (nsteps < 1) return fail(ctx, LES_ERR_ARG, "les_advance: nsteps must be >= 1 (got %d)", nsteps);
  if (dt_out && nsteps > LES_ADVANCE_DT_MAX)
    return fail(ctx, LES_ERR_ARG, "les_advance: dt_out holds at most %d steps (got %d)", LES_ADVANCE_DT_MAX, nsteps);
  les::Layout& L = ctx->L;
  const long long nb = les::stage_blocks(L, ctx->kchunk, ctx->mach);
  // the first step's dt by a pass of its own; each later one was reduced by
  // the last stage of the step before (the state it reads is that stage's
  // output, untouched since)
  HIPCHK(ctx, bc_fill(ctx, Q));
  HIPCHK(ctx, les::launch_cfl(ctx->s, L, ctx->P, ctx->M, Q, ctx->part, ctx->scal, ctx->flag,
                              dt_out ? ctx->dthist : nullptr, ctx->axis));
  // Mixed precision: each step after the first takes the FP32 copy of its
  // Q^n from the step before, where its ghost layers are plain copies or
  // frozen values (no face rules, polar axis or dynamic closure, which would
  // then work on FP32 values): the same stencil values, one FP64 read less.
  const bool shadow = ctx->prec == LES_MIXED && !ctx->axis && ctx->P.sgs != 2 && !faces_of(ctx).any;
  for (int n = 0; n < nsteps; ++n) {
    double* dtp = ctx->scal + ((n & 1) ? 12 : 0);
    double* dnext = ctx->scal + ((n & 1) ? 0 : 12);
    const bool more = n + 1 < nsteps;
    if (n > 0) HIPCHK(ctx, bc_fill(ctx, Q));
    int rc = step_core(ctx, Q, dtp, 0.0, nullptr, (more && !ctx->use_ref) ? ctx->cpart : nullptr, !more, n & 1,
                       shadow && n > 0, shadow && more);
    if (rc != LES_OK) return rc;
    if (!more) break;
    double* rec = dt_out ? ctx->dthist + n + 1 : nullptr;
    if (ctx->use_ref)
      HIPCHK(ctx, les::launch_cfl(ctx->s, L, ctx->P, ctx->M, Q, ctx->part, dnext, ctx->flag, rec, ctx->axis));
    else
      HIPCHK(ctx, les::launch_cfl_final(ctx->s, ctx->cpart, nb, ctx->P.cfl, dnext, rec, ctx->flag));
  }
  if (!dt_out && !norms) return LES_OK;
  if (dt_out) HIPCHK(ctx, hipMemcpyAsync(dt_out, ctx->dthist, (size_t)nsteps * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  return sync_outputs(ctx, nullptr, norms);
}

int les_adjoint_step(les_ctx* ctx, const double* stage_ckpt, double dt, double* Qbar, double* fbar) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_adjoint_step: null context");
  if (!stage_ckpt || !Qbar) return fail(ctx, LES_ERR_ARG, "les_adjoint_step: stage_ckpt and Qbar are required");
  if (!(dt > 0.0)) return fail(ctx, LES_ERR_ARG, "les_adjoint_step: dt must be > 0 (the step's fixed dt)");
  if (ctx->prec != LES_FP64) return fail(ctx, LES_ERR_STATE, "les_adjoint_step: needs an FP64 context");
  if (ctx->P.sgs == 2)
    return fail(ctx, LES_ERR_STATE, "les_adjoint_step: the adjoint covers the static Smagorinsky model "
                                    "(sgs <= 1, with or without the isotropic SGS stress)");
  int rc = ensure_adj_work(ctx);
  if (rc != LES_OK) return rc;
  les::AdjArgs a{ctx->L, ctx->P, ctx->M, ctx->bc[0], ctx->bc[1], ctx->bc[2], ctx->i_f, faces_of(ctx), ctx->axis};
  HIPCHK(ctx, les::run_adjoint_step(ctx->s, a, stage_ckpt, dt, Qbar, ctx->i_f >= 0 ? fbar : nullptr, ctx->adj));
  return LES_OK;
}

int les_set_face(les_ctx* ctx, int face, int type, const double* Q_outside, double p_exit) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_set_face: null context");
  if (face < 0 || face > 5) return fail(ctx, LES_ERR_ARG, "les_set_face: face %d outside [0, 6)", face);
  if (ctx->bc[face / 2] != LES_BC_DIRICHLET && !(face == 3 && ctx->bc[1] == LES_BC_AXIS))
    return fail(ctx, LES_ERR_ARG, "les_set_face: face %d is not on a Dirichlet side", face);
  if (type != LES_FACE_FROZEN && type != LES_FACE_CHARACTERISTIC && type != LES_FACE_EXIT &&
      type != LES_FACE_FARFIELD)
    return fail(ctx, LES_ERR_ARG, "les_set_face: unknown face type %d", type);
  if (type == LES_FACE_EXIT && !(p_exit > 0.0 && p_exit < INFINITY))
    return fail(ctx, LES_ERR_ARG, "les_set_face: the exit pressure must be positive and finite");
  if ((type == LES_FACE_CHARACTERISTIC || type == LES_FACE_FARFIELD) && !Q_outside && !ctx->outside)
    return fail(ctx, LES_ERR_ARG, "les_set_face: a characteristic or far-field face needs an outside state");
  if (Q_outside) {
    const size_t bytes = (size_t)5 * ctx->L.fe * sizeof(double);
    if (!ctx->outside && hipMalloc(&ctx->outside, bytes) != hipSuccess) {
      ctx->outside = nullptr;
      return fail(ctx, LES_ERR_NOMEM, "les_set_face: cannot allocate the outside state");
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->outside, Q_outside, bytes, hipMemcpyDeviceToDevice, ctx->s));
  }
  ctx->face[face] = type;
  ctx->p_exit[face] = type == LES_FACE_EXIT ? p_exit : 0.0;
  return LES_OK;
}

int les_stats_accumulate(les_ctx* ctx, const double* Q, double* acc) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_stats_accumulate: null context");
  if (!Q || !acc) return fail(ctx, LES_ERR_ARG, "les_stats_accumulate: Q and acc are required");
  // a superposed k direction repeats plane 0 as plane nk - 1: counted once
  const int nks = ctx->bc[2] == 2 ? ctx->L.nk - 1 : ctx->L.nk;
  HIPCHK(ctx, les::launch_stats(ctx->s, ctx->L, ctx->P, nks, Q, acc));
  return LES_OK;
}

int les_stats_profiles(les_ctx* ctx, const double* acc, double samples, double u_jet, double core_frac,
                       double* prof, unsigned char* core) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_stats_profiles: null context");
  if (!acc || !prof) return fail(ctx, LES_ERR_ARG, "les_stats_profiles: acc and prof are required");
  if (!(samples > 0.0) || !isfinite(samples))
    return fail(ctx, LES_ERR_ARG, "les_stats_profiles: samples must be positive (got %g)", samples);
  if (core && (!(u_jet > 0.0) || !isfinite(u_jet) || !(core_frac > 0.0 && core_frac <= 1.0)))
    return fail(ctx, LES_ERR_ARG, "les_stats_profiles: the core needs u_jet > 0 and 0 < core_frac <= 1");
  HIPCHK(ctx, les::launch_stats_profiles(ctx->s, ctx->L, acc, samples, core ? core_frac * u_jet : 0.0, prof, core));
  return LES_OK;
}

int les_residual_adjoint(les_ctx* ctx, double* Q, const double* Rbar, double* Qbar) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_residual_adjoint: null context");
  if (!Q || !Rbar || !Qbar) return fail(ctx, LES_ERR_ARG, "les_residual_adjoint: Q, Rbar and Qbar are required");
  if (Qbar == Q || Qbar == Rbar) return fail(ctx, LES_ERR_ARG, "les_residual_adjoint: Qbar must not alias Q or Rbar");
  if (ctx->P.sgs == 2)
    return fail(ctx, LES_ERR_STATE, "les_residual_adjoint: the adjoint covers the static Smagorinsky model "
                                    "(sgs <= 1, with or without the isotropic SGS stress)");
  int rc = ensure_adj_work(ctx);
  if (rc != LES_OK) return rc;
  HIPCHK(ctx, bc_fill(ctx, Q));
  les::AdjArgs a{ctx->L, ctx->P, ctx->M, ctx->bc[0], ctx->bc[1], ctx->bc[2], ctx->i_f, faces_of(ctx), ctx->axis};
  HIPCHK(ctx, les::run_residual_vjp(ctx->s, a, Q, Rbar, Qbar, ctx->adj));
  return LES_OK;
}

int les_probe_objective(les_ctx* ctx, const double* Q, int i_p, double p_inf, double weight, double* J_accum,
                        double* Qbar) {
  if (!ctx) return fail(nullptr, LES_ERR_ARG, "les_probe_objective: null context");
  if (!Q || !J_accum) return fail(ctx, LES_ERR_ARG, "les_probe_objective: Q and J_accum are required");
  if (i_p < 0 || i_p >= ctx->L.ni) return fail(ctx, LES_ERR_ARG, "les_probe_objective: plane %d outside [0, %d)", i_p, ctx->L.ni);
  // over the distinct k planes (a superposed direction's last plane repeats its first)
  const int nks = ctx->bc[2] == 2 ? ctx->L.nk - 1 : ctx->L.nk;
  HIPCHK(ctx, les::launch_probe(ctx->s, ctx->L, ctx->P, nks, Q, i_p, p_inf, weight, J_accum, Qbar, ctx->part));
  return LES_OK;
}

// Instrumentation (les_debug.h).  Select the stage kernel: 0 = fused tiled
// kernel (default), 1 = reference kernel; a testing switch used to
// cross-check the two formulations.
int les_debug_use_reference(les_ctx* ctx, int on) {
  if (!ctx) return LES_ERR_ARG;
  ctx->use_ref = on ? 1 : 0;
  return LES_OK;
}

// Stage-kernel timing (les_debug.h; used by the benchmark):
// on != 0 starts recording a HIP event pair around every stage-kernel
// launch on the context's stream; les_debug_stage_time synchronises and
// returns the summed elapsed milliseconds and the launch count since
// timing was switched on, then resets them.
int les_debug_stage_timing(les_ctx* ctx, int on) {
  if (!ctx) return LES_ERR_ARG;
  int rc = resolve_timing(ctx);
  ctx->timing = on ? 1 : 0;
  ctx->t_ms = 0.0;
  ctx->t_cnt = 0;
  return rc;
}

int les_debug_stage_time(les_ctx* ctx, double* total_ms, long long* launches) {
  if (!ctx || !total_ms || !launches) return LES_ERR_ARG;
  int rc = resolve_timing(ctx);
  *total_ms = ctx->t_ms;
  *launches = ctx->t_cnt;
  ctx->t_ms = 0.0;
  ctx->t_cnt = 0;
  return rc;
}

int les_debug_dynamic_coefficients(les_ctx* ctx, double* Q, double* out) {
  if (!ctx) return LES_ERR_ARG;
  if (!Q || !out) return fail(ctx, LES_ERR_ARG, "les_debug_dynamic_coefficients: null pointer");
  if (ctx->P.sgs != 2) return fail(ctx, LES_ERR_STATE, "les_debug_dynamic_coefficients: sgs is not 2");
  HIPCHK(ctx, les::launch_ghost_fill(ctx->s, ctx->L, ctx->bc, Q, Q, 5, faces_of(ctx)));
  HIPCHK(ctx, dyn_update(ctx, Q, nullptr));
  HIPCHK(ctx, hipMemcpyAsync(out, ctx->dyn, 2 * les::dyn_ncol(ctx->L) * sizeof(double), hipMemcpyDeviceToDevice,
                             ctx->s));
  HIPCHK(ctx, hipStreamSynchronize(ctx->s));
  return LES_OK;
}

// Plain device copy of nbytes (a multiple of 16, both pointers 16-byte
// aligned) on the given HIP stream (les_debug.h; the benchmark's achievable
// stream bandwidth).
int les_debug_stream_copy(const void* src, void* dst, long long nbytes, void* hip_stream) {
  if (!src || !dst || nbytes <= 0 || (nbytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15))
    return LES_ERR_ARG;
  if (les::launch_stream_copy((hipStream_t)hip_stream, src, dst, nbytes / 16) != hipSuccess) return LES_ERR_HIP;
  return LES_OK;
}

}  // extern "C"
