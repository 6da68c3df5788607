// Host side of libelh: handle and hierarchy, C-ABI entry points, the
// multigrid cycle driver and the batched flexible GMRES driver.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include <atomic>
#include <chrono>
#include <complex>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/elh.h"
#include "elh_internal.h"

using namespace elh;
typedef std::complex<double> zd;

std::atomic<unsigned long long> elh::g_kernels{0};

static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHK(call)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail(ELH_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)
#define CHK(call)                    \
  do {                               \
    int r_ = (call);                 \
    if (r_ != 0) {                   \
      if (r_ > 0) r_ = fail(ELH_ERR_HIP, "kernel launch failed: %s (%s)", hipGetErrorString((hipError_t)r_), #call); \
      return r_;                     \
    }                                \
  } while (0)

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// bumped on every (re)allocation: captured graphs embed buffer addresses
static std::atomic<uint64_t> g_alloc_gen{1};

static int ensure(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return 0;
  ++g_alloc_gen;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  size_t want = (bytes + 255) & ~(size_t)255;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ELH_ERR_OOM, "device allocation of %zu bytes failed", want);
  }
  b.bytes = want;
  return 0;
}
static void release(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

struct LevelData {
  int n[3];
  double h;
  int64_t fs, vs;
  DevBuf lam, mu, rho, kap, mu32, rho32, kap32;
  DevBuf b[2], x[2], r[2];  // cycle work per precision (0: f64, 1: f32)
  DevBuf kw[2];             // K-cycle work on this (coarse) level: E1, V1, R1, V2, E2
  DevBuf ablz[2];           // absorbing-layer term along x_3 per plane (centres, faces), f64 / f32
  DevBuf kc;                // K-cycle dots / coefficients / state of the step into this level
};

// Krylov workspace for one (level, precision, Z precision) combination.
struct KrylovWS {
  DevBuf V, Z, w, t;
  DevBuf B, X;  // outer solve: right-hand sides and iterates of the packed (still active) rhs
};

// Hybrid Kaczmarz coarsest solve: rows of the Schur complement in the slot
// pattern, sub-region gather lists and work buffers.
struct KaczData {
  int ns = 0, box = 0, nreg = 0, ls = 0;
  int E[3] = {1, 1, 1}, nb[3] = {1, 1, 1};
  DevBuf val[2][2], inv[2][2];             // [adjoint][precision]
  DevBuf tab[2], dl[2], gptr[2], gent[2];  // [adjoint]
  DevBuf app[2];                           // A_pp per cell, [precision]
  DevBuf scr, t, y, bs;                    // solve work
};

struct GraphEntry {
  int kind = 0, step = 0;  // 0: preconditioner cycle; 1: outer Gram-Schmidt step `step`
  int prec, adj, nrhs;
  const void* in;
  void* out;
  uint64_t gen;
  unsigned long long nkern = 0;  // kernel nodes
  hipGraphExec_t exec;
};

struct elh_handle {
  elh_desc d;
  hipStream_t st;
  int nlev;
  LevelData lv[8];
  KrylovWS kout[2], kin[2];  // outer (level 0, f64; Z f64/f32), inner (coarsest; f64/f32)
  DevBuf part, dots, coef, tmpvec;
  DevBuf gstate, gpart, gdots, gnrm, gcoef, gscale, ones;  // device-resident GMRES (coarsest level)
  DevBuf ostate, opart, odots, ocoef, ostat, opar;           // device-resident outer FGMRES
  double* hstat = nullptr;  // pinned host copy of ostat
  double* hpar = nullptr;   // pinned staging of opar
  DevBuf dq64, dq32;                                        // dense coarsest inverse (Q = inv(H_s^T))
  KaczData kz;                                              // hybrid Kaczmarz coarsest solve
  int64_t dn = 0;
  hipStream_t cap = nullptr;                               // stream used only to record graphs
  std::vector<GraphEntry> graphs;
  int use_graphs = 1;                                      // ELH_GRAPHS=0 disables capture
  double* hdots = nullptr;  // pinned host mirror
  double* hcoef = nullptr;
  int zchunk = 32;          // default x_3 planes per workgroup of the wavefront march (ELH_ZCHUNK)
  // stencil autotuner: chosen x_3 chunk of the wavefront march per (level,
  // precision, input precision, residual, adjoint, nrhs); ELH_TUNE=0 keeps
  // the default heuristic,
  // ELH_TUNE_CACHE=path persists the choices across processes
  int tune = 1;
  std::map<int, int> tuned;
  hipEvent_t tev[2] = {nullptr, nullptr};
  std::string tune_path;
  void* scratch = nullptr;  // this device's address of the allocation-free relaxation's work array
  int ok = 0;
};

static size_t csz(int prec) { return prec == 0 ? 16 : 8; }  // bytes per complex entry
static int prec_of(int dtype) { return dtype == ELH_C64 ? 1 : 0; }

template <typename T>
static LevelArgs<T> largs(const elh_handle* H, int l, bool shifted) {
  const LevelData& L = H->lv[l];
  LevelArgs<T> a;
  a.n[0] = L.n[0];
  a.n[1] = L.n[1];
  a.n[2] = L.n[2];
  a.fs = L.fs;
  a.vs = L.vs;
  a.h = (T)L.h;
  a.ih = (T)(1.0 / L.h);
  a.beta = (T)H->d.beta;
  a.omega2 = (T)(H->d.omega * H->d.omega);
  a.gam = (T)(H->d.gamma + (shifted ? H->d.alpha : 0.0));
  a.abl_w = (T)H->d.abl_width;
  a.abl_amp = (T)H->d.abl_amp;
  a.abl_iw = H->d.abl_width > 0 ? (T)(1.0 / H->d.abl_width) : (T)0;
  if (sizeof(T) == 8) {
    a.mu = (const T*)L.mu.p;
    a.rho = (const T*)L.rho.p;
    a.kap = (const T*)L.kap.p;
    a.ablz = (const T*)L.ablz[0].p;
  } else {
    a.mu = (const T*)L.mu32.p;
    a.rho = (const T*)L.rho32.p;
    a.kap = (const T*)L.kap32.p;
    a.ablz = (const T*)L.ablz[1].p;
  }
  return a;
}

static int check_desc(const elh_desc* d) {
  if (!d) return fail(ELH_ERR_ARG, "desc is NULL");
  if (d->dim != 2 && d->dim != 3) return fail(ELH_ERR_ARG, "dim must be 2 or 3");
  if (d->levels < 1 || d->levels > 8) return fail(ELH_ERR_ARG, "levels must be in 1..8");
  for (int a = 0; a < d->dim; ++a) {
    if (d->n[a] < 2) return fail(ELH_ERR_ARG, "n[%d] must be >= 2", a);
    int div = 1 << (d->levels - 1);
    if (d->n[a] % div != 0 || d->n[a] / div < 2)
      return fail(ELH_ERR_ARG, "n[%d]=%d not divisible by 2^(levels-1) with >= 2 coarse cells", a, d->n[a]);
  }
  if (d->dim == 2 && d->n[2] != 1) return fail(ELH_ERR_ARG, "n[2] must be 1 in 2D");
  if (!(d->h > 0)) return fail(ELH_ERR_ARG, "h must be positive");
  if (!(d->beta > 0 && d->beta <= 1)) return fail(ELH_ERR_ARG, "beta must be in (0,1]");
  if (d->nu1 < 0 || d->nu2 < 0) return fail(ELH_ERR_ARG, "nu1/nu2 must be >= 0");
  if (d->cycle_calls < 1 || d->cycle_calls > 3)
    return fail(ELH_ERR_ARG, "cycle_calls must be 1 (V), 2 (W) or 3 (K)");
  if (d->coarse_mode < 0 || d->coarse_mode > 3) return fail(ELH_ERR_ARG, "bad coarse_mode");
  if (d->coarse_mode != ELH_COARSE_DENSE && d->coarse_sweeps < 1) return fail(ELH_ERR_ARG, "coarse_sweeps must be >= 1");
  if ((d->coarse_mode == ELH_COARSE_KRYLOV || d->coarse_mode == ELH_COARSE_KACZMARZ) &&
      (d->coarse_restart < 1 || d->coarse_maxit < 1))
    return fail(ELH_ERR_ARG, "coarse_restart/coarse_maxit must be >= 1");
  if (d->coarse_mode == ELH_COARSE_KACZMARZ) {
    if (d->kacz_box < 0) return fail(ELH_ERR_ARG, "kacz_box must be >= 0");
    const int box = d->kacz_box > 0 ? d->kacz_box : 4;
    int64_t ls = d->dim;
    for (int a = 0; a < d->dim; ++a) ls *= box + 4;
    if (ls * 16 > (int64_t)KACZ_MAX_LDS)
      return fail(ELH_ERR_ARG, "kacz_box %d: the private copy of a sub-region exceeds %zu bytes of LDS", box,
                  KACZ_MAX_LDS);
    int64_t fs = 1;
    for (int a = 0; a < d->dim; ++a) fs *= d->n[a] >> (d->levels - 1);
    if (fs > 64 * 64 * 64) return fail(ELH_ERR_ARG, "Kaczmarz coarsest solve needs at most 64^3 coarsest cells");
  }
  if (d->coarse_restart + 1 > MAXDOT) return fail(ELH_ERR_ARG, "coarse_restart too large");
  if (d->precond_dtype != ELH_C64 && d->precond_dtype != ELH_C128) return fail(ELH_ERR_ARG, "bad precond_dtype");
  if (d->abl_width < 0) return fail(ELH_ERR_ARG, "abl_width must be >= 0");
  if (!(d->gamma >= 0) || !(d->alpha >= 0) || !(d->gamma + d->alpha > 0))
    return fail(ELH_ERR_ARG, "gamma and alpha must be >= 0 with gamma + alpha > 0");
  if (!(d->omega > 0) || !isfinite(d->omega)) return fail(ELH_ERR_ARG, "omega must be positive and finite");
  return 0;
}

static int build_hierarchy(elh_handle* H, const double* lam, const double* mu, const double* rho) {
  hipStream_t st = H->st;
  LevelData& L0 = H->lv[0];
  HIPCHK(hipMemcpyAsync(L0.lam.p, lam, L0.fs * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(L0.mu.p, mu, L0.fs * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(L0.rho.p, rho, L0.fs * 8, hipMemcpyDeviceToDevice, st));
  for (int l = 1; l < H->nlev; ++l) {
    LevelData& F = H->lv[l - 1];
    LevelData& C = H->lv[l];
    CHK(launch_coarsen_media(H->d.dim, F.n, (const double*)F.lam.p, (double*)C.lam.p, st));
    CHK(launch_coarsen_media(H->d.dim, F.n, (const double*)F.mu.p, (double*)C.mu.p, st));
    CHK(launch_coarsen_media(H->d.dim, F.n, (const double*)F.rho.p, (double*)C.rho.p, st));
  }
  for (int l = 0; l < H->nlev; ++l) {
    LevelData& L = H->lv[l];
    CHK(launch_media_finish(L.fs, (const double*)L.lam.p, (const double*)L.mu.p, (const double*)L.rho.p,
                            (double*)L.kap.p, (float*)L.mu32.p, (float*)L.rho32.p, (float*)L.kap32.p, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}

// Dense coarsest-level inverse (ELH_COARSE_DENSE): columns of H_s from
// applying it to unit vectors (boundary-face unknowns made identity), then
// Gauss-Jordan inversion of H_s^T on the device.
static constexpr int64_t DENSE_MAX = 8192;
static int build_dense(elh_handle* H);
static int build_kaczmarz(elh_handle* H);

static void tune_load(elh_handle* H);
static int tune_key(int l, int prec, int iprec, int kind, bool adj, int nrhs);

// Work array of the allocation-free relaxation (elh_relax_noalloc): a
// file-scope device array, so the loaded code object gives every GPU its own
// copy, held until the process ends.  Host code never uses the array's name
// as an address: each device's address comes from hipGetSymbolAddress, once
// per device, at elh_create (with that device current), and is kept here.
static __device__ __align__(256) unsigned char scratch[ELH_NOALLOC_SCRATCH_BYTES];
static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

static int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(ELH_ERR_HIP, "no usable current device for the relaxation work array");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ELH_ERR_HIP, "hipGetSymbolAddress of the relaxation work array failed: %s", hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return 0;
}

extern "C" int elh_create(const elh_desc* desc, const double* lam, const double* mu, const double* rho,
                          void* stream, elh_handle** out) {
  if (!out) return fail(ELH_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_desc(desc);
  if (rc) return rc;
  if (!lam || !mu || !rho) return fail(ELH_ERR_ARG, "media pointers must be non-NULL device pointers");
  elh_handle* H = new elh_handle();
  H->d = *desc;
  {
    const char* z = getenv("ELH_ZCHUNK");  // > 0: default chunk (shortened on small grids); < 0: exactly -z
    if (z && atoi(z) != 0) H->zchunk = atoi(z);
    const char* g = getenv("ELH_GRAPHS");
    if (g && strcmp(g, "0") == 0) H->use_graphs = 0;
    const char* tu = getenv("ELH_TUNE");
    if (tu && strcmp(tu, "0") == 0) H->tune = 0;
    const char* tc = getenv("ELH_TUNE_CACHE");
    if (tc && *tc) H->tune_path = tc;
  }
  H->st = (hipStream_t)stream;
  H->nlev = desc->levels;
  for (int l = 0; l < H->nlev; ++l) {
    LevelData& L = H->lv[l];
    for (int a = 0; a < 3; ++a) L.n[a] = (a < desc->dim) ? (desc->n[a] >> l) : 1;
    L.h = desc->h * (double)(1 << l);
    L.fs = (int64_t)L.n[0] * L.n[1] * L.n[2];
    L.vs = (int64_t)(desc->dim + 1) * L.fs;
    int e = 0;
    e |= ensure(L.lam, L.fs * 8);
    e |= ensure(L.mu, L.fs * 8);
    e |= ensure(L.rho, L.fs * 8);
    e |= ensure(L.kap, L.fs * 8);
    e |= ensure(L.mu32, L.fs * 4);
    e |= ensure(L.rho32, L.fs * 4);
    e |= ensure(L.kap32, L.fs * 4);
    e |= ensure(L.ablz[0], (size_t)2 * L.n[2] * 8);
    e |= ensure(L.ablz[1], (size_t)2 * L.n[2] * 4);
    if (!e) {
      // amp * (delta/width)^2 along x_3 at plane centres (t + 1/2) h and
      // lower faces t h, delta the distance into the layer (physical width)
      std::vector<double> t64(2 * L.n[2]);
      std::vector<float> t32(2 * L.n[2]);
      const double w = desc->abl_width, len = L.n[2] * L.h;
      for (int t = 0; t < L.n[2]; ++t)
        for (int f = 0; f < 2; ++f) {
          const double xp = (f == 0 ? t + 0.5 : (double)t) * L.h;
          double v = 0;
          if (w > 0 && desc->abl_amp != 0) {
            const double d = (w - xp > 0 ? w - xp : 0) + (xp - (len - w) > 0 ? xp - (len - w) : 0);
            v = desc->abl_amp * (d / w) * (d / w);
          }
          t64[f * L.n[2] + t] = v;
          t32[f * L.n[2] + t] = (float)v;
        }
      e |= hipMemcpy(L.ablz[0].p, t64.data(), t64.size() * 8, hipMemcpyHostToDevice) != hipSuccess;
      e |= hipMemcpy(L.ablz[1].p, t32.data(), t32.size() * 4, hipMemcpyHostToDevice) != hipSuccess;
    }
    if (e) {
      elh_destroy(H);
      return ELH_ERR_OOM;
    }
  }
  if (ensure(H->part, (size_t)MAXRHS_KRYLOV * 512 * MAXDOT * 2 * 8) ||
      ensure(H->dots, MAXRHS_KRYLOV * MAXDOT * 16) || ensure(H->coef, MAXRHS_KRYLOV * MAXDOT * 16)) {
    elh_destroy(H);
    return ELH_ERR_OOM;
  }
  if (ensure(H->gstate, (size_t)MAXRHS_KRYLOV * GM_STRIDE * 8) ||
      ensure(H->gpart, (size_t)MAXRHS_KRYLOV * 512 * MAXDOT * 2 * 8) ||
      ensure(H->gdots, MAXRHS_KRYLOV * MAXDOT * 16) || ensure(H->gnrm, MAXRHS_KRYLOV * 16) ||
      ensure(H->gcoef, MAXRHS_KRYLOV * MAXDOT * 16) || ensure(H->gscale, MAXRHS_KRYLOV * 16)) {
    elh_destroy(H);
    return ELH_ERR_OOM;
  }
  if (hipStreamCreateWithFlags(&H->cap, hipStreamNonBlocking) != hipSuccess) {
    elh_destroy(H);
    return fail(ELH_ERR_HIP, "stream creation failed");
  }
  if (ensure(H->ostate, (size_t)MAXRHS_KRYLOV * GO_STRIDE * 8) ||
      ensure(H->opart, (size_t)MAXRHS_KRYLOV * 512 * MAXDOT * 2 * 8) || ensure(H->odots, MAXRHS_KRYLOV * MAXDOT * 16) ||
      ensure(H->ocoef, MAXRHS_KRYLOV * MAXDOT * 16) || ensure(H->ostat, MAXRHS_KRYLOV * 4 * 8) ||
      ensure(H->opar, MAXRHS_KRYLOV * 4 * 8)) {
    elh_destroy(H);
    return ELH_ERR_OOM;
  }
  if (hipHostMalloc((void**)&H->hdots, MAXRHS_KRYLOV * MAXDOT * 16, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&H->hcoef, MAXRHS_KRYLOV * MAXDOT * 16, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&H->hstat, MAXRHS_KRYLOV * 4 * 8, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&H->hpar, MAXRHS_KRYLOV * 4 * 8, hipHostMallocDefault) != hipSuccess) {
    elh_destroy(H);
    return fail(ELH_ERR_OOM, "pinned host allocation failed");
  }
  rc = scratch_address(&H->scratch);
  if (!rc) rc = build_hierarchy(H, lam, mu, rho);
  if (!rc && desc->coarse_mode == ELH_COARSE_DENSE) rc = build_dense(H);
  if (!rc && desc->coarse_mode == ELH_COARSE_KACZMARZ) rc = build_kaczmarz(H);
  if (rc) {
    elh_destroy(H);
    return rc;
  }
  tune_load(H);
  H->ok = 1;
  *out = H;
  return 0;
}

extern "C" int elh_set_media(elh_handle* H, const double* lam, const double* mu, const double* rho) {
  if (!H || !H->ok) return fail(ELH_ERR_STATE, "invalid handle");
  if (!lam || !mu || !rho) return fail(ELH_ERR_ARG, "media pointers must be non-NULL");
  int rc = build_hierarchy(H, lam, mu, rho);
  if (!rc && H->d.coarse_mode == ELH_COARSE_DENSE) rc = build_dense(H);
  if (!rc && H->d.coarse_mode == ELH_COARSE_KACZMARZ) rc = build_kaczmarz(H);
  return rc;
}

extern "C" int elh_destroy(elh_handle* H) {
  if (!H) return 0;
  if (H->st) (void)hipStreamSynchronize(H->st);
  else (void)hipDeviceSynchronize();
  for (int l = 0; l < 8; ++l) {
    LevelData& L = H->lv[l];
    release(L.lam); release(L.mu); release(L.rho); release(L.kap);
    release(L.mu32); release(L.rho32); release(L.kap32);
    for (int p = 0; p < 2; ++p) {
      release(L.b[p]); release(L.x[p]); release(L.r[p]); release(L.kw[p]); release(L.ablz[p]);
    }
    release(L.kc);
  }
  for (int p = 0; p < 2; ++p) {
    KrylovWS* ws[2] = {&H->kout[p], &H->kin[p]};
    for (auto* w : ws) { release(w->V); release(w->Z); release(w->w); release(w->t); release(w->B); release(w->X); }
  }
  release(H->part); release(H->dots); release(H->coef); release(H->tmpvec);
  release(H->gstate); release(H->gpart); release(H->gdots); release(H->gnrm); release(H->gcoef);
  release(H->gscale); release(H->ones); release(H->dq64); release(H->dq32);
  release(H->ostate); release(H->opart); release(H->odots); release(H->ocoef); release(H->ostat); release(H->opar);
  for (int a = 0; a < 2; ++a) {
    for (int p = 0; p < 2; ++p) { release(H->kz.val[a][p]); release(H->kz.inv[a][p]); }
    release(H->kz.tab[a]); release(H->kz.dl[a]); release(H->kz.gptr[a]); release(H->kz.gent[a]);
    release(H->kz.app[a]);
  }
  release(H->kz.scr); release(H->kz.t); release(H->kz.y); release(H->kz.bs);
  for (auto& g : H->graphs) (void)hipGraphExecDestroy(g.exec);
  H->graphs.clear();
  if (H->cap) (void)hipStreamDestroy(H->cap);
  for (auto& e : H->tev)
    if (e) (void)hipEventDestroy(e);
  if (H->hdots) (void)hipHostFree(H->hdots);
  if (H->hcoef) (void)hipHostFree(H->hcoef);
  if (H->hstat) (void)hipHostFree(H->hstat);
  if (H->hpar) (void)hipHostFree(H->hpar);
  delete H;
  return 0;
}

extern "C" int elh_stencil_choice(elh_handle* H, int level, int dtype, int flags, int residual, int nrhs,
                                  int* choice) {
  if (!H || !H->ok) return fail(ELH_ERR_STATE, "invalid handle");
  if (level < 0 || level >= H->nlev) return fail(ELH_ERR_ARG, "level %d out of range", level);
  if (dtype != ELH_C64 && dtype != ELH_C128) return fail(ELH_ERR_ARG, "dtype must be ELH_C64 or ELH_C128");
  if (!choice || nrhs < 1) return fail(ELH_ERR_ARG, "choice must be non-NULL and nrhs >= 1");
  const int prec = prec_of(dtype);
  if (residual < 0 || residual > 2) return fail(ELH_ERR_ARG, "residual must be 0, 1 or 2");
  auto it = H->tuned.find(tune_key(level, prec, prec, residual, (flags & ELH_ADJOINT) != 0, nrhs));
  *choice = it == H->tuned.end() ? -1 : it->second;
  return 0;
}

extern "C" int elh_level_info(elh_handle* H, int level, int* n3, double* hl) {
  if (!H || !H->ok) return fail(ELH_ERR_STATE, "invalid handle");
  if (level < 0 || level >= H->nlev) return fail(ELH_ERR_ARG, "level out of range");
  if (n3) for (int a = 0; a < 3; ++a) n3[a] = H->lv[level].n[a];
  if (hl) *hl = H->lv[level].h;
  return H->nlev;
}

static int check_common(elh_handle* H, int level, int dtype, int nrhs) {
  if (!H || !H->ok) return fail(ELH_ERR_STATE, "invalid handle");
  if (level < 0 || level >= H->nlev) return fail(ELH_ERR_ARG, "level %d out of range", level);
  if (dtype != ELH_C64 && dtype != ELH_C128) return fail(ELH_ERR_ARG, "dtype must be ELH_C64 or ELH_C128");
  if (nrhs < 1 || nrhs > 65535) return fail(ELH_ERR_ARG, "nrhs must be in 1..65535");
  return 0;
}

static int ensure_cycle_bufs(elh_handle* H, int prec, int nrhs) {
  if (H->d.cycle_calls == 2 && H->ones.bytes < (size_t)nrhs * 16) {
    // W-cycle: coefficient 1 per rhs for adding the second coarse correction
    if (ensure(H->ones, (size_t)nrhs * 16)) return ELH_ERR_OOM;
    std::vector<double> one(H->ones.bytes / 8, 0.0);
    for (size_t i = 0; i < one.size(); i += 2) one[i] = 1.0;
    if (hipMemcpy(H->ones.p, one.data(), one.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return fail(ELH_ERR_HIP, "upload of the W-cycle coefficients failed");
  }
  for (int l = 0; l < H->nlev; ++l) {
    LevelData& L = H->lv[l];
    size_t bytes = (size_t)nrhs * L.vs * csz(prec);
    if (ensure(L.b[prec], bytes) || ensure(L.x[prec], bytes) || ensure(L.r[prec], bytes)) return ELH_ERR_OOM;
    if (H->d.cycle_calls == 3 && l > 0) {
      if (ensure(L.kw[prec], 5 * bytes) || ensure(L.kc, (size_t)MAXRHS_KRYLOV * 20 * 8)) return ELH_ERR_OOM;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// level operations (precision T)
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// stencil autotuner
// ---------------------------------------------------------------------------
static std::mutex g_tune_file_mu;

// kind: 0 apply, 1 residual, 2 residual restricted to the next level
static int tune_key(int l, int prec, int iprec, int kind, bool adj, int nrhs) {
  return (((((l * 2 + prec) * 2 + iprec) * 3 + kind) * 2 + (adj ? 1 : 0)) << 8) | (nrhs & 0xff);
}

// choices persisted by earlier processes for this handle's grids
static void tune_load(elh_handle* H) {
  if (H->tune_path.empty()) return;
  std::lock_guard<std::mutex> lk(g_tune_file_mu);
  FILE* f = fopen(H->tune_path.c_str(), "r");
  if (!f) return;
  int n1, n2, n3, prec, iprec, resid, adj, nrhs, choice;
  while (fscanf(f, "%d %d %d %d %d %d %d %d %d", &n1, &n2, &n3, &prec, &iprec, &resid, &adj, &nrhs, &choice) == 9) {
    for (int l = 0; l < H->nlev; ++l)
      if (H->lv[l].n[0] == n1 && H->lv[l].n[1] == n2 && H->lv[l].n[2] == n3)
        if (resid >= 0 && resid <= 2) H->tuned[tune_key(l, prec, iprec, resid, adj != 0, nrhs)] = choice;
  }
  fclose(f);
}

static void tune_store(elh_handle* H, int l, int prec, int iprec, int kind, bool adj, int nrhs, int choice) {
  if (H->tune_path.empty()) return;
  std::lock_guard<std::mutex> lk(g_tune_file_mu);
  FILE* f = fopen(H->tune_path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%d %d %d %d %d %d %d %d %d\n", H->lv[l].n[0], H->lv[l].n[1], H->lv[l].n[2], prec, iprec, kind,
          adj ? 1 : 0, nrhs, choice);
  fclose(f);
}

// One 3D apply / residual with input precision TI (float or T): x_3 chunk
// `choice` (> 0) of the wavefront march (0: the point-wise kernel).
template <typename T, typename TI>
static int launch_choice(elh_handle* H, int l, bool shifted, bool adj, const void* x, const void* b, void* y,
                         int nrhs, int choice) {
  const LevelArgs<T> a = largs<T>(H, l, shifted);
  if (adj && sizeof(TI) != sizeof(T)) return (int)hipErrorInvalidValue;  // adjoint reads T input only
  if (choice > 0) {
    if (adj) return launch_apply3d_w3_adj<T>(a, x, b, y, nrhs, -choice, H->st);
    return launch_apply3d_w3<T, TI>(a, x, b, y, nrhs, -choice, H->st);
  }
  if (sizeof(TI) != sizeof(T)) return (int)hipErrorInvalidValue;  // point-wise needs T input
  return launch_apply<T>(a, H->d.dim, adj, x, b, y, nrhs, H->st);
}

// x_3 chunk for this call: the tuned choice if there is one; else,
// when tuning is allowed here, time the candidates on the call's own
// buffers (the operation is idempotent when its output aliases no input)
// with HIP events on the library's stream and keep the fastest.  The chunk
// only changes which workgroup marches which planes, not any output's
// arithmetic, so every choice gives bitwise the same result.  Never tunes
// while the stream is being captured into a graph.  n3: planes of the
// marched column in the chunk's unit; launch(c) runs the kernel with chunk c.
static constexpr int CHUNK_DEFAULT = 0x7fffffff;  // the launcher's heuristic

template <typename Launch>
static int tune_chunk(elh_handle* H, int l, int prec, int iprec, int kind, bool adj, int nrhs, int n3,
                      bool may_tune, Launch launch) {
  const int key = tune_key(l, prec, iprec, kind, adj, nrhs);
  auto it = H->tuned.find(key);
  if (it != H->tuned.end()) return it->second;
  const int dflt = CHUNK_DEFAULT;
  if (!H->tune || !may_tune || nrhs > 255) return dflt;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(H->st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return dflt;
  if (!H->tev[0]) {
    if (hipEventCreate(&H->tev[0]) != hipSuccess || hipEventCreate(&H->tev[1]) != hipSuccess) return dflt;
  }
  std::vector<int> cand;
  for (int zc : {1, 2, 4, 8, 16, 32, 64})
    if (zc < n3 && (zc >= 4 || n3 <= 64)) cand.push_back(zc);  // 1, 2 only on short columns
  if (n3 <= 64) cand.push_back(n3);  // the whole column in one chunk
  int best = dflt;
  float tbest = 0;
  for (int c : cand) {
    if (launch(c)) return dflt;  // warm-up
    if (hipEventRecord(H->tev[0], H->st) != hipSuccess) return dflt;
    for (int r = 0; r < 3; ++r)
      if (launch(c)) return dflt;
    if (hipEventRecord(H->tev[1], H->st) != hipSuccess) return dflt;
    float ms = 0;
    if (hipEventSynchronize(H->tev[1]) != hipSuccess || hipEventElapsedTime(&ms, H->tev[0], H->tev[1]) != hipSuccess)
      return dflt;
    if (best == dflt || ms < tbest) {
      best = c;
      tbest = ms;
    }
  }
  H->tuned[key] = best;
  tune_store(H, l, prec, iprec, kind, adj, nrhs, best);
  return best;
}

template <typename T, typename TI>
static int stencil_choice(elh_handle* H, int l, bool shifted, bool adj, const void* x, const void* b, void* y,
                          int nrhs, bool may_tune = true) {
  const int prec = sizeof(T) == 8 ? 0 : 1, iprec = sizeof(TI) == 8 ? 0 : 1;
  return tune_chunk(H, l, prec, iprec, b != nullptr ? 1 : 0, adj, nrhs, H->lv[l].n[2],
                    may_tune && y != x && y != b,
                    [&](int c) { return launch_choice<T, TI>(H, l, shifted, adj, x, b, y, nrhs, c); });
}

// 3D levels from 16^3 whose fields fit 32-bit byte offsets take the
// wavefront march (x_3 chunk from the autotuner); 2D and smaller levels the
// point-wise kernel.
static bool marches(const elh_handle* H, int l, size_t entry_bytes) {
  return H->d.dim == 3 && H->lv[l].fs * (int64_t)entry_bytes <= (int64_t)0x7fffffff && H->lv[l].fs >= 16 * 16 * 16;
}

template <typename T>
static int op_apply(elh_handle* H, int l, bool shifted, bool adj, const void* x, const void* b, void* y, int nrhs,
                    bool may_tune = true) {
  if (marches(H, l, sizeof(cx<T>))) {
    const int c = stencil_choice<T, T>(H, l, shifted, adj, x, b, y, nrhs, may_tune);
    if (c == CHUNK_DEFAULT) {
      if (adj) return launch_apply3d_w3_adj<T>(largs<T>(H, l, shifted), x, b, y, nrhs, H->zchunk, H->st);
      return launch_apply3d_w3<T>(largs<T>(H, l, shifted), x, b, y, nrhs, H->zchunk, H->st);
    }
    return launch_choice<T, T>(H, l, shifted, adj, x, b, y, nrhs, c);
  }
  return launch_apply<T>(largs<T>(H, l, shifted), H->d.dim, adj, x, b, y, nrhs, H->st);
}

// rc = R (b - H_s x) from level l to l+1 (x == nullptr: x = 0, rc = R b):
// one launch, the fine residual is never stored; the march form (x_3 chunk
// in coarse planes from the autotuner) on march levels, the point-wise form
// otherwise.
template <typename T>
static int op_restrict_residual(elh_handle* H, int l, bool adj, const void* x, const void* b, void* rc, int nrhs,
                                bool may_tune = true) {
  const LevelArgs<T> F = largs<T>(H, l, true), Cl = largs<T>(H, l + 1, true);
  if (!x) return launch_restrict<T>(F, Cl, H->d.dim, b, rc, nrhs, H->st);
  if (marches(H, l, sizeof(cx<T>))) {
    const int prec = sizeof(T) == 8 ? 0 : 1;
    const int c = tune_chunk(H, l, prec, prec, 2, adj, nrhs, H->lv[l + 1].n[2], may_tune && rc != x && rc != b,
                             [&](int zc) {
                               return launch_restrict_resid3d_w3<T>(F, Cl, adj, x, b, rc, nrhs, -zc, H->st);
                             });
    // default: half the fine default in coarse planes; ELH_ZCHUNK < 0 forces exactly -ELH_ZCHUNK coarse planes
    const int dz = H->zchunk > 0 ? (H->zchunk / 2 > 0 ? H->zchunk / 2 : 1) : H->zchunk;
    return launch_restrict_resid3d_w3<T>(F, Cl, adj, x, b, rc, nrhs, c == CHUNK_DEFAULT ? dz : -c, H->st);
  }
  return launch_restrict_resid<T>(F, Cl, H->d.dim, adj, x, b, rc, nrhs, H->st);
}

// outer operator on float32 input (level 0, float64 arithmetic and output)
static int op_apply_f32in(elh_handle* H, bool adj, const void* x, void* y, int nrhs) {
  const int c = stencil_choice<double, float>(H, 0, false, adj, x, nullptr, y, nrhs);
  if (c == CHUNK_DEFAULT || c == 0)
    return launch_apply3d_w3<double, float>(largs<double>(H, 0, false), x, nullptr, y, nrhs, H->zchunk, H->st);
  return launch_choice<double, float>(H, 0, false, adj, x, nullptr, y, nrhs, c);
}

static double level_damping(const elh_handle* H, int l) {
  if (l == H->nlev - 1 && H->d.coarse_damping > 0) return H->d.coarse_damping;
  return H->d.damping[l < 8 ? l : 7];
}

// one colour of red-black Vanka; x_is_zero lets the residual be b itself
template <typename T>
// x_is_zero: the iterate is zero and x holds nothing yet (the residual is b;
// in 3D the half-sweep writes every entry of x, in 2D x is cleared first)
static int op_relax(elh_handle* H, int l, bool adj, int colour, const void* b, void* x, int nrhs, bool x_is_zero) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  LevelData& L = H->lv[l];
  const void* r = b;
  if (!x_is_zero) {
    CHK(op_apply<T>(H, l, true, adj, x, b, L.r[prec].p, nrhs));
    r = L.r[prec].p;
  } else if (H->d.dim != 3) {
    CHK(launch_zero(x, (int64_t)nrhs * L.vs * csz(prec), H->st));
  }
  return launch_vanka<T>(largs<T>(H, l, true), H->d.dim, adj, r, x, colour, level_damping(H, l), nrhs, H->st,
                         x_is_zero && H->d.dim == 3);
}

// one colour of red-black Vanka with the residual in the caller's work
// buffer r; the stencil chunk is the autotuner's earlier choice or the
// default (no tuning: nothing is timed or allocated)
template <typename T>
static int op_relax_with(elh_handle* H, int l, bool adj, int colour, const void* b, void* x, void* r, int nrhs) {
  CHK(op_apply<T>(H, l, true, adj, x, b, r, nrhs, false));
  return launch_vanka<T>(largs<T>(H, l, true), H->d.dim, adj, r, x, colour, level_damping(H, l), nrhs, H->st, false);
}

template <typename T>
static int op_sweeps_from_zero(elh_handle* H, int l, bool adj, const void* b, void* x, int nrhs, int sweeps) {
  for (int s = 0; s < sweeps; ++s) {
    CHK(op_relax<T>(H, l, adj, 0, b, x, nrhs, s == 0));
    CHK(op_relax<T>(H, l, adj, 1, b, x, nrhs, false));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// batched restarted (flexible) GMRES, right preconditioned
// ---------------------------------------------------------------------------
struct GmresStats {
  std::vector<int> iters, restarts, status;
  std::vector<double> relres;
  std::vector<std::vector<double>> history;  // per rhs: residual estimate after each iteration
  bool timing = false;                        // record the time split below (events on the stream)
  double t_precond = 0, t_apply = 0, t_orth = 0;  // ms
};

// GPU-time accounting of one solve: events recorded between the phases of
// an iteration, read after the host synchronisation that follows them.
struct PhaseTimer {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  explicit PhaseTimer(bool want) {
    if (!want) return;
    on = true;
    for (auto& x : e)
      if (hipEventCreate(&x) != hipSuccess) on = false;
  }
  ~PhaseTimer() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  void mark(int i, hipStream_t st) {
    if (on && hipEventRecord(e[i], st) != hipSuccess) on = false;
  }
  double span(int a, int b) {
    float ms = 0;
    if (!on || hipEventElapsedTime(&ms, e[a], e[b]) != hipSuccess) return 0.0;
    return ms;
  }
};

// dots[s][i] for i < m, from the device buffer (synchronises)
static int fetch_dots(elh_handle* H, int nrhs, int m, std::vector<zd>& out) {
  HIPCHK(hipMemcpyAsync(H->hdots, H->dots.p, (size_t)nrhs * m * 16, hipMemcpyDeviceToHost, H->st));
  HIPCHK(hipStreamSynchronize(H->st));
  out.resize((size_t)nrhs * m);
  for (int i = 0; i < nrhs * m; ++i) out[i] = zd(H->hdots[2 * i], H->hdots[2 * i + 1]);
  return 0;
}

static int push_coef(elh_handle* H, const std::vector<zd>& c) {
  for (size_t i = 0; i < c.size(); ++i) {
    H->hcoef[2 * i] = c[i].real();
    H->hcoef[2 * i + 1] = c[i].imag();
  }
  HIPCHK(hipMemcpyAsync(H->coef.p, H->hcoef, c.size() * 16, hipMemcpyHostToDevice, H->st));
  // the pinned staging buffer is reused by the next push: wait for the copy
  HIPCHK(hipStreamSynchronize(H->st));
  return 0;
}

template <typename TX, typename TY>
static int scale_copy(elh_handle* H, const std::vector<zd>* a, const void* x, int64_t xs, void* y, int64_t ys,
                      int64_t len, int nrhs) {
  const double* dev = nullptr;
  if (a) {
    CHK(push_coef(H, *a));
    dev = (const double*)H->coef.p;
  }
  return launch_scale_copy<TX, TY>(dev, x, xs, y, ys, len, nrhs, H->st);
}


// AZ: w = A z (z in TZ, w in T); AR: r = b - A x (T vectors);
// M: z = M v (v in TZ, z in TZ).  Right-preconditioned flexible GMRES(m),
// zero initial guess, classical Gram-Schmidt, complex Givens rotations.
//
// The basis is kept unnormalised: V_i holds v_i / sig_i (sig_i = 1/||V_i||
// kept per rhs on the host) and Z_i = M V_i, so that
//   A M v_j = sig_j A Z_j,  h_ij = sig_i sig_j <V_i, A Z_j>,
//   V_{j+1} = A Z_j - sum_i sig_i^2 <V_i, A Z_j> V_i,
//   h_{j+1,j} = sig_j ||V_{j+1}||,  x += sum_j (y_j sig_j) Z_j.
// A Z_j is written straight into V_{j+1}; the Gram-Schmidt update, its
// norm and (when TZ != T) the TZ copy that feeds the next preconditioner
// application (cyc_in) come out of one pass.  No vector is rescaled.
//
// x0: x holds the initial guess (the first basis vector is the true
// residual b - A x); otherwise x starts at zero and the first basis vector
// is b.
template <typename T, typename TZ, typename OpAZ, typename OpAR, typename OpM>
static int gmres(elh_handle* H, KrylovWS& ws, int64_t len, int nrhs, OpAZ AZ, OpAR AR, OpM M, const void* b,
                 void* x, int restart, int maxit, double rtol, GmresStats& st_out, void* cyc_in, bool x0 = false) {
  typedef cx<T> CT;
  typedef cx<TZ> CZ;
  const bool cast_in = sizeof(TZ) != sizeof(T);
  if (cast_in && !cyc_in) return fail(ELH_ERR_STATE, "mixed-precision GMRES needs a preconditioner input buffer");
  const int m = restart;
  const size_t vbytes = (size_t)nrhs * len * sizeof(CT);
  const size_t zbytes = (size_t)nrhs * len * sizeof(CZ);
  if (ensure(ws.V, vbytes * (m + 1)) || ensure(ws.Z, zbytes * m)) return ELH_ERR_OOM;
  CT* V = (CT*)ws.V.p;
  CZ* Z = (CZ*)ws.Z.p;
  const int64_t vstr = (int64_t)nrhs * len;  // stride between basis vectors
  hipStream_t st = H->st;
  std::vector<zd> dots;
  // ||b||
  CHK((launch_multidot<CT, CT>(1, b, 0, len, b, len, len, nrhs, (double*)H->part.p, (double*)H->dots.p, st)));
  CHK(fetch_dots(H, nrhs, 1, dots));
  std::vector<double> nb(nrhs), beta(nrhs);
  for (int s = 0; s < nrhs; ++s) nb[s] = sqrt(dots[s].real());
  if (x0) {
    // V_0 = r = b - A x
    CHK(AR((const void*)x, b, (void*)V));
    CHK((launch_multidot<CT, CT>(1, V, 0, len, V, len, len, nrhs, (double*)H->part.p, (double*)H->dots.p, st)));
    CHK(fetch_dots(H, nrhs, 1, dots));
    for (int s = 0; s < nrhs; ++s) beta[s] = sqrt(dots[s].real());
  } else {
    // x = 0, V_0 = r = b
    CHK(launch_zero(x, vbytes, st));
    HIPCHK(hipMemcpyAsync(V, b, vbytes, hipMemcpyDeviceToDevice, st));
    for (int s = 0; s < nrhs; ++s) beta[s] = nb[s];
  }
  st_out.iters.assign(nrhs, 0);
  st_out.restarts.assign(nrhs, 0);
  st_out.status.assign(nrhs, ELH_NOT_CONVERGED);
  st_out.relres.assign(nrhs, 1.0);
  st_out.history.assign(nrhs, std::vector<double>());
  PhaseTimer tm(st_out.timing);
  std::vector<char> active(nrhs);
  int nact = 0;
  for (int s = 0; s < nrhs; ++s) {
    if (!isfinite(nb[s]) || !isfinite(beta[s])) return fail(ELH_ERR_NUMERIC, "non-finite initial residual (rhs %d)", s);
    if (!(nb[s] > 0)) {
      // q = 0: the solution is 0 (an initial guess is discarded)
      active[s] = 0;
      st_out.status[s] = ELH_OK;
      st_out.relres[s] = 0.0;
      if (x0) CHK(launch_zero((CT*)x + (int64_t)s * len, len * (int64_t)sizeof(CT), st));
    } else {
      st_out.relres[s] = beta[s] / nb[s];
      active[s] = st_out.relres[s] > rtol && beta[s] > 0;
      if (!active[s]) st_out.status[s] = ELH_OK;
    }
    nact += active[s];
  }
  int iters = 0;
  std::vector<zd> Hm((size_t)nrhs * (m + 1) * m), g((size_t)nrhs * (m + 1)), sn((size_t)nrhs * m), coef;
  std::vector<double> cs((size_t)nrhs * m), sig((size_t)nrhs * (m + 1));
  std::vector<int> jend(nrhs);
  std::vector<char> live(nrhs);
  while (nact > 0 && iters < maxit) {
    for (int s = 0; s < nrhs; ++s) {
      sig[(size_t)s * (m + 1)] = active[s] ? 1.0 / beta[s] : 0.0;
      for (int i = 0; i <= m; ++i) g[s * (m + 1) + i] = 0;
      g[s * (m + 1)] = beta[s];
      jend[s] = -1;
      live[s] = active[s];
    }
    if (cast_in) CHK((launch_scale_copy<CT, CZ>(nullptr, V, len, cyc_in, len, len, nrhs, st)));
    int j;
    for (j = 0; j < m; ++j) {
      tm.mark(0, st);
      CHK(M(cast_in ? (const void*)cyc_in : (const void*)(V + j * vstr), (void*)(Z + j * vstr)));
      tm.mark(1, st);
      CT* W = V + (j + 1) * vstr;
      CHK(AZ((const void*)(Z + j * vstr), (void*)W));
      tm.mark(2, st);
      ++iters;
      // classical Gram-Schmidt on the unnormalised basis
      CHK((launch_multidot<CT, CT>(j + 1, V, vstr, len, W, len, len, nrhs, (double*)H->part.p, (double*)H->dots.p,
                                   st)));
      CHK(fetch_dots(H, nrhs, j + 1, dots));
      coef.assign((size_t)nrhs * (j + 1), zd(0, 0));
      for (int s = 0; s < nrhs; ++s)
        for (int i = 0; i <= j; ++i) {
          const double si = sig[(size_t)s * (m + 1) + i];
          coef[s * (j + 1) + i] = -(si * si) * dots[s * (j + 1) + i];
        }
      CHK(push_coef(H, coef));
      std::vector<zd> d = dots;
      CHK((launch_axpy_norm<CT, CZ>(j + 1, (const double*)H->coef.p, V, vstr, len, W, len,
                                    cast_in ? cyc_in : nullptr, len, len, nrhs, (double*)H->part.p,
                                    (double*)H->dots.p, st)));
      tm.mark(3, st);
      CHK(fetch_dots(H, nrhs, 1, dots));
      st_out.t_precond += tm.span(0, 1);
      st_out.t_apply += tm.span(1, 2);
      st_out.t_orth += tm.span(2, 3);
      bool any_live = false;
      for (int s = 0; s < nrhs; ++s) {
        const double sj = sig[(size_t)s * (m + 1) + j];
        const double wn = sqrt(dots[s].real());
        sig[(size_t)s * (m + 1) + j + 1] = wn > 0 ? 1.0 / wn : 0.0;
        if (!live[s]) continue;
        st_out.iters[s]++;
        double hn = sj * wn;
        if (!isfinite(hn)) return fail(ELH_ERR_NUMERIC, "non-finite norm in GMRES (rhs %d)", s);
        zd* hc = &Hm[(size_t)s * (m + 1) * m];
        for (int i = 0; i <= j; ++i) hc[i * m + j] = (sig[(size_t)s * (m + 1) + i] * sj) * d[s * (j + 1) + i];
        hc[(j + 1) * m + j] = hn;
        // apply previous rotations
        for (int i = 0; i < j; ++i) {
          zd a = hc[i * m + j], bb = hc[(i + 1) * m + j];
          double c = cs[s * m + i];
          zd sgn = sn[s * m + i];
          hc[i * m + j] = c * a + sgn * bb;
          hc[(i + 1) * m + j] = -std::conj(sgn) * a + c * bb;
        }
        zd a = hc[j * m + j], bb = hc[(j + 1) * m + j];
        double c;
        zd sgn;
        if (std::abs(bb) == 0) {
          c = 1;
          sgn = 0;
        } else if (std::abs(a) == 0) {
          c = 0;
          sgn = std::conj(bb) / std::abs(bb);
        } else {
          double den = hypot(std::abs(a), std::abs(bb));
          c = std::abs(a) / den;
          sgn = (a / std::abs(a)) * std::conj(bb) / den;
        }
        cs[s * m + j] = c;
        sn[s * m + j] = sgn;
        hc[j * m + j] = c * a + sgn * bb;
        hc[(j + 1) * m + j] = 0;
        zd* gs = &g[(size_t)s * (m + 1)];
        gs[j + 1] = -std::conj(sgn) * gs[j];
        gs[j] = c * gs[j];
        jend[s] = j;
        double res = std::abs(gs[j + 1]) / nb[s];
        st_out.history[s].push_back(res);
        if (res <= rtol || hn == 0) live[s] = 0;
        if (live[s]) any_live = true;
      }
      if (!any_live || iters >= maxit) {
        ++j;
        break;
      }
    }
    // y = H^{-1} g per rhs, then x += sum_j (y_j sig_j) Z_j
    int kmax = j;
    coef.assign((size_t)nrhs * kmax, zd(0, 0));
    for (int s = 0; s < nrhs; ++s) {
      if (!active[s]) continue;
      int k = jend[s] + 1;
      const zd* hc = &Hm[(size_t)s * (m + 1) * m];
      const zd* gs = &g[(size_t)s * (m + 1)];
      std::vector<zd> y(k);
      for (int i = k - 1; i >= 0; --i) {
        zd acc = gs[i];
        for (int q = i + 1; q < k; ++q) acc -= hc[i * m + q] * y[q];
        y[i] = acc / hc[i * m + i];
      }
      for (int i = 0; i < k; ++i) coef[(size_t)s * kmax + i] = y[i] * sig[(size_t)s * (m + 1) + i];
    }
    CHK(push_coef(H, coef));
    CHK((launch_multiaxpy<CZ, CT>(kmax, (const double*)H->coef.p, Z, vstr, len, x, len, len, nrhs, st)));
    // true residual r = b - A x, the next V_0
    CHK(AR((const void*)x, b, (void*)V));
    CHK((launch_multidot<CT, CT>(1, V, 0, len, V, len, len, nrhs, (double*)H->part.p, (double*)H->dots.p, st)));
    CHK(fetch_dots(H, nrhs, 1, dots));
    nact = 0;
    for (int s = 0; s < nrhs; ++s) {
      if (!active[s]) continue;
      st_out.restarts[s]++;
      beta[s] = sqrt(dots[s].real());
      if (!isfinite(beta[s])) return fail(ELH_ERR_NUMERIC, "non-finite residual (rhs %d)", s);
      st_out.relres[s] = beta[s] / nb[s];
      if (st_out.relres[s] <= rtol) {
        active[s] = 0;
        st_out.status[s] = ELH_OK;
      } else if (beta[s] == 0) {
        active[s] = 0;
        st_out.status[s] = ELH_OK;
      }
      nact += active[s];
    }
  }
  return 0;
}

static int build_dense(elh_handle* H) {
  const int l = H->nlev - 1;
  LevelData& L = H->lv[l];
  const int64_t N = L.vs;
  if (N > DENSE_MAX) return fail(ELH_ERR_ARG, "dense coarsest solve needs <= %lld unknowns, level %d has %lld",
                                 (long long)DENSE_MAX, l, (long long)N);
  DevBuf E, A, col, piv, isb;
  int rc = 0;
  const size_t mat = (size_t)N * N * 16;
  if (ensure(E, mat) || ensure(A, mat) || ensure(col, (N + 1) * 16) || ensure(piv, 64) || ensure(isb, N * 4) ||
      ensure(H->dq64, mat) || ensure(H->dq32, mat / 2)) {
    release(E); release(A); release(col); release(piv); release(isb);
    return ELH_ERR_OOM;
  }
  std::vector<int> hb(N, 0);
  for (int f = 0; f < H->d.dim; ++f)
    for (int64_t c = 0; c < L.fs; ++c) {
      int idx[3] = {(int)(c % L.n[0]), (int)((c / L.n[0]) % L.n[1]), (int)(c / ((int64_t)L.n[0] * L.n[1]))};
      if (idx[f] == 0) hb[f * L.fs + c] = 1;
    }
  hipStream_t st = H->st;
  if (hipMemcpy(isb.p, hb.data(), N * 4, hipMemcpyHostToDevice) != hipSuccess) rc = fail(ELH_ERR_HIP, "upload failed");
  if (!rc) rc = launch_dense_assemble_prep(N, E.p, st);
  // A[j] = H_s e_j  (row-major A = H_s^T); batched apply over the N unit vectors
  if (!rc) rc = launch_apply<double>(largs<double>(H, l, true), H->d.dim, false, E.p, nullptr, A.p, (int)N, st);
  if (!rc) rc = launch_dense_fix(N, (const int*)isb.p, A.p, st);
  if (!rc) rc = launch_dense_invert(N, A.p, H->dq64.p, col.p, (int*)piv.p, st);
  if (!rc) rc = launch_scale_copy<cx<double>, cx<float>>(nullptr, H->dq64.p, 0, H->dq32.p, 0, N * N, 1, st);
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(ELH_ERR_HIP, "dense coarse setup failed");
  if (rc > 0) rc = fail(ELH_ERR_HIP, "dense coarse setup launch failed");
  release(E); release(A); release(col); release(piv); release(isb);
  H->dn = N;
  return rc;
}

// Hybrid Kaczmarz coarsest solve, setup.  The entries of A = H_s on the
// coarsest level come from applying it (float64 point-wise kernel) to
// (dim+1)*3^dim probe vectors: probe (f, r) holds ones on the unknowns of
// field f whose storage index is congruent to r modulo 3 on every axis.
// Every column of A reaches rows within one cell of it, so the entry of
// row i and column j (|i - j| <= 1 cell per axis) is the value of row i
// in the probe that holds j.  From those, per displacement row and slot of
// the pattern,
//   S_ij = [A_uu]_ij - sum_m [A_up]_im [A_pu]_mj / [A_pp]_mm,
// the adjoint rows being conj(S_ji).  Slot pattern of the row of u_k
// towards u_l (offsets of the column's storage index): the 3^dim box when
// l = k; otherwise o_l in {0, 1}, o_k in {-2..1}, the remaining axis in
// {-1, 0, 1}; adjoint rows take the negated pattern of u_l towards u_k.
static void kacz_slots(int dim, int k, bool adj, std::vector<int>& tab) {
  for (int l = 0; l < dim; ++l) {
    const int kk = adj ? l : k, ll = adj ? k : l;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      if (kk == ll) { lo[a] = -1; hi[a] = 1; }
      else if (a == ll) { lo[a] = 0; hi[a] = 1; }
      else if (a == kk) { lo[a] = -2; hi[a] = 1; }
      else { lo[a] = -1; hi[a] = 1; }
    }
    const int sg = adj ? -1 : 1;
    for (int o2 = lo[2]; o2 <= hi[2]; ++o2)
      for (int o1 = lo[1]; o1 <= hi[1]; ++o1)
        for (int o0 = lo[0]; o0 <= hi[0]; ++o0) {
          tab.push_back(l);
          tab.push_back(sg * o0);
          tab.push_back(sg * o1);
          tab.push_back(sg * o2);
        }
  }
}

static int build_kaczmarz(elh_handle* H) {
  const int l = H->nlev - 1;
  const LevelData& L = H->lv[l];
  const int dim = H->d.dim;
  const int64_t fs = L.fs, vs = L.vs, nu = (int64_t)dim * fs;
  const int n0 = L.n[0], n1 = L.n[1], n2 = L.n[2];
  KaczData& K = H->kz;
  K.box = H->d.kacz_box > 0 ? H->d.kacz_box : 4;
  const int P = dim == 3 ? 27 : 9;
  const int np = (dim + 1) * P;
  auto lin = [&](int x, int y, int z) { return ((int64_t)z * n1 + y) * n0 + x; };
  auto res3 = [&](int x, int y, int z) { return x % 3 + 3 * (y % 3) + 9 * (z % 3); };
  // probes and their images
  std::vector<double> he((size_t)np * vs * 2, 0.0);
  for (int f = 0; f <= dim; ++f)
    for (int z = 0; z < n2; ++z)
      for (int y = 0; y < n1; ++y)
        for (int x = 0; x < n0; ++x) {
          const int c[3] = {x, y, z};
          if (f < dim && c[f] == 0) continue;
          const int64_t p = (int64_t)f * P + res3(x, y, z);
          he[2 * ((size_t)p * vs + f * fs + lin(x, y, z))] = 1.0;
        }
  DevBuf E, Y;
  int rc = 0;
  if (ensure(E, he.size() * 8) || ensure(Y, he.size() * 8)) {
    release(E); release(Y);
    return ELH_ERR_OOM;
  }
  hipStream_t st = H->st;
  if (hipMemcpy(E.p, he.data(), he.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
    rc = fail(ELH_ERR_HIP, "probe upload failed");
  if (!rc) rc = launch_apply<double>(largs<double>(H, l, true), dim, false, E.p, nullptr, Y.p, np, st);
  if (rc > 0) rc = fail(ELH_ERR_HIP, "probe apply failed");
  std::vector<double> hy(he.size());
  if (!rc && (hipStreamSynchronize(st) != hipSuccess ||
              hipMemcpy(hy.data(), Y.p, hy.size() * 8, hipMemcpyDeviceToHost) != hipSuccess))
    rc = fail(ELH_ERR_HIP, "probe download failed");
  release(E); release(Y);
  if (rc) return rc;
  // A(F, c; f, c'), |c - c'| <= 1 cell per axis
  auto A = [&](int F, const int* c, int f, const int* cp) {
    const size_t p = (size_t)f * P + res3(cp[0], cp[1], cp[2]);
    const size_t i = p * vs + F * fs + lin(c[0], c[1], c[2]);
    return zd(hy[2 * i], hy[2 * i + 1]);
  };
  auto inside = [&](const int* c) {
    return c[0] >= 0 && c[0] < n0 && c[1] >= 0 && c[1] < n1 && c[2] >= 0 && c[2] < n2;
  };
  auto cheb1 = [&](const int* a, const int* b) {
    return abs(a[0] - b[0]) <= 1 && abs(a[1] - b[1]) <= 1 && abs(a[2] - b[2]) <= 1;
  };
  const int rz = dim == 3 ? 1 : 0;
  // A_pp per cell
  std::vector<zd> app(fs);
  for (int z = 0; z < n2; ++z)
    for (int y = 0; y < n1; ++y)
      for (int x = 0; x < n0; ++x) {
        const int c[3] = {x, y, z};
        app[lin(x, y, z)] = A(dim, c, dim, c);
        if (app[lin(x, y, z)] == zd(0, 0)) return fail(ELH_ERR_NUMERIC, "zero pressure diagonal");
      }
  // nonzero A_up couplings of every displacement row: (cell, value)
  std::vector<std::vector<std::pair<int64_t, zd>>> up(nu);
  for (int k = 0; k < dim; ++k)
    for (int z = 0; z < n2; ++z)
      for (int y = 0; y < n1; ++y)
        for (int x = 0; x < n0; ++x) {
          const int c[3] = {x, y, z};
          if (c[k] == 0) continue;
          auto& lst = up[k * fs + lin(x, y, z)];
          for (int dz = -rz; dz <= rz; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                const int m[3] = {x + dx, y + dy, z + dz};
                if (!inside(m)) continue;
                const zd a = A(k, c, dim, m);
                if (a != zd(0, 0)) lst.push_back({lin(m[0], m[1], m[2]), a});
              }
        }
  // forward Schur entry of row (kr, cr), column (kc, cc)
  auto Sf = [&](int kr, const int* cr, int kc, const int* cc) {
    zd v(0, 0);
    if (kr == kc && cheb1(cr, cc)) v = A(kr, cr, kc, cc);
    for (const auto& e : up[kr * fs + lin(cr[0], cr[1], cr[2])]) {
      const int64_t mc = e.first;
      const int m[3] = {(int)(mc % n0), (int)((mc / n0) % n1), (int)(mc / ((int64_t)n0 * n1))};
      if (!cheb1(m, cc)) continue;
      v -= e.second * A(dim, m, kc, cc) / app[mc];
    }
    return v;
  };
  // sub-regions and private copies
  int64_t nreg = 1, ee = 1;
  for (int a = 0; a < 3; ++a) {
    K.nb[a] = a < dim ? (L.n[a] + K.box - 1) / K.box : 1;
    K.E[a] = a < dim ? K.box + 4 : 1;
    nreg *= K.nb[a];
    ee *= K.E[a];
  }
  K.nreg = (int)nreg;
  K.ls = (int)(dim * ee);
  for (int adj = 0; adj < 2; ++adj) {
    std::vector<int> tab;
    for (int k = 0; k < dim; ++k) kacz_slots(dim, k, adj != 0, tab);
    const int ns = (int)(tab.size() / 4 / dim);
    K.ns = ns;
    std::vector<int> dl((size_t)dim * ns);
    for (int k = 0; k < dim; ++k)
      for (int q = 0; q < ns; ++q) {
        const int* t = &tab[(size_t)(k * ns + q) * 4];
        dl[(size_t)k * ns + q] = (int)(t[0] * ee + (t[3] * K.E[1] + t[2]) * K.E[0] + t[1]);
      }
    // rows
    // 128 zero slots of padding after the last row: the sweep's lanes load
    // slots lane and lane + 64 of every row unconditionally
    std::vector<double> v64(((size_t)nu * ns + 128) * 2, 0.0), i64(nu, 0.0);
    std::vector<float> v32(((size_t)nu * ns + 128) * 2, 0.0f), i32(nu, 0.0f);
    for (int k = 0; k < dim; ++k)
      for (int z = 0; z < n2; ++z)
        for (int y = 0; y < n1; ++y)
          for (int x = 0; x < n0; ++x) {
            const int c[3] = {x, y, z};
            if (c[k] == 0) continue;
            const int64_t row = k * fs + lin(x, y, z);
            double nrm = 0;
            for (int q = 0; q < ns; ++q) {
              const int* t = &tab[(size_t)(k * ns + q) * 4];
              const int lc = t[0];
              const int cc[3] = {x + t[1], y + t[2], z + t[3]};
              if (!inside(cc) || cc[lc] == 0) continue;
              const zd v = adj ? std::conj(Sf(lc, cc, k, c)) : Sf(k, c, lc, cc);
              const size_t o = ((size_t)row * ns + q) * 2;
              v64[o] = v.real();
              v64[o + 1] = v.imag();
              v32[o] = (float)v.real();
              v32[o + 1] = (float)v.imag();
              nrm += std::norm(v);
            }
            i64[row] = nrm > 0 ? 1.0 / nrm : 0.0;
            i32[row] = (float)i64[row];
          }
    // gather lists: for each unknown, the (sub-region, private index) pairs
    // of the sub-regions whose rows reach it, sub-regions ascending
    std::vector<std::vector<std::pair<int, int>>> lists(nu);
    std::vector<char> mark(K.ls);
    for (int r = 0; r < K.nreg; ++r) {
      const int br[3] = {r % K.nb[0], (r / K.nb[0]) % K.nb[1], r / (K.nb[0] * K.nb[1])};
      int lo[3], c0[3], c1[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = a < dim ? br[a] * K.box - 2 : 0;
        c0[a] = a < dim ? br[a] * K.box : 0;
        c1[a] = a < dim ? std::min(c0[a] + K.box, L.n[a]) : 1;
      }
      std::fill(mark.begin(), mark.end(), 0);
      for (int k = 0; k < dim; ++k)
        for (int z = c0[2]; z < c1[2]; ++z)
          for (int y = c0[1]; y < c1[1]; ++y)
            for (int x = c0[0]; x < c1[0]; ++x) {
              const int c[3] = {x, y, z};
              if (c[k] == 0) continue;
              for (int q = 0; q < ns; ++q) {
                const int* t = &tab[(size_t)(k * ns + q) * 4];
                const int lc = t[0];
                const int cc[3] = {x + t[1], y + t[2], z + t[3]};
                if (!inside(cc) || cc[lc] == 0) continue;
                const int li = (int)(lc * ee + ((cc[2] - lo[2]) * K.E[1] + (cc[1] - lo[1])) * K.E[0] + (cc[0] - lo[0]));
                if (mark[li]) continue;
                mark[li] = 1;
                lists[lc * fs + lin(cc[0], cc[1], cc[2])].push_back({r, li});
              }
            }
    }
    std::vector<int> gptr(nu + 1, 0), gent;
    for (int64_t j = 0; j < nu; ++j) {
      gptr[j + 1] = gptr[j] + (int)lists[j].size();
      for (const auto& e : lists[j]) {
        gent.push_back(e.first);
        gent.push_back(e.second);
      }
    }
    if (gent.empty()) gent.push_back(0);
    if (ensure(K.val[adj][0], v64.size() * 8) || ensure(K.val[adj][1], v32.size() * 4) ||
        ensure(K.inv[adj][0], i64.size() * 8) || ensure(K.inv[adj][1], i32.size() * 4) ||
        ensure(K.tab[adj], tab.size() * 4) || ensure(K.dl[adj], dl.size() * 4) ||
        ensure(K.gptr[adj], gptr.size() * 4) || ensure(K.gent[adj], gent.size() * 4))
      return ELH_ERR_OOM;
    if (hipMemcpy(K.val[adj][0].p, v64.data(), v64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.val[adj][1].p, v32.data(), v32.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.inv[adj][0].p, i64.data(), i64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.inv[adj][1].p, i32.data(), i32.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.tab[adj].p, tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.dl[adj].p, dl.data(), dl.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.gptr[adj].p, gptr.data(), gptr.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(K.gent[adj].p, gent.data(), gent.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      return fail(ELH_ERR_HIP, "upload of the Kaczmarz rows failed");
  }
  std::vector<double> a64(2 * fs);
  std::vector<float> a32(2 * fs);
  for (int64_t c = 0; c < fs; ++c) {
    a64[2 * c] = app[c].real();
    a64[2 * c + 1] = app[c].imag();
    a32[2 * c] = (float)app[c].real();
    a32[2 * c + 1] = (float)app[c].imag();
  }
  if (ensure(K.app[0], a64.size() * 8) || ensure(K.app[1], a32.size() * 4)) return ELH_ERR_OOM;
  if (hipMemcpy(K.app[0].p, a64.data(), a64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(K.app[1].p, a32.data(), a32.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(ELH_ERR_HIP, "upload of the pressure diagonal failed");
  return 0;
}

// Fixed-budget restarted GMRES with all bookkeeping on the device (no host
// synchronisation, graph-capturable).  Same algorithm as gmres() with
// rtol = 0: classical Gram-Schmidt, complex Givens, restart every m steps,
// exactly `maxit` preconditioner applications.
template <typename T, typename OpAZ, typename OpAR, typename OpM>
static int gmres_device(elh_handle* H, KrylovWS& ws, int64_t len, int nrhs, OpAZ AZ, OpAR AR, OpM M, const void* b,
                        void* x, int restart, int maxit) {
  typedef cx<T> CT;
  const int m = restart;
  const size_t vbytes = (size_t)nrhs * len * sizeof(CT);
  if (ensure(ws.V, vbytes * (m + 1)) || ensure(ws.Z, vbytes * m) || ensure(ws.w, vbytes)) return ELH_ERR_OOM;
  CT* V = (CT*)ws.V.p;
  CT* Z = (CT*)ws.Z.p;
  CT* w = (CT*)ws.w.p;
  const int64_t vstr = (int64_t)nrhs * len;
  hipStream_t st = H->st;
  double* gst = (double*)H->gstate.p;
  double* gpart = (double*)H->gpart.p;
  double* gdots = (double*)H->gdots.p;
  double* gnrm = (double*)H->gnrm.p;
  double* gcoef = (double*)H->gcoef.p;
  double* gscale = (double*)H->gscale.p;
  // x0 = 0: the first residual is b itself, and the first solution update
  // writes x instead of adding to it
  int done = 0;
  const CT* r0 = (const CT*)b;
  while (done < maxit) {
    // small reductions are finished by their consumer (no separate launch)
    const bool fn = nrhs * 2 <= FUSE_VALS;
    const int nbn = norm_blocks(len, FUSE_BLOCKS);
    CHK((launch_multidot<CT, CT>(1, r0, 0, len, r0, len, len, nrhs, gpart, fn ? nullptr : gnrm, st)));
    // with the small reductions, the start and each rotation but the last
    // run in the scaled copy that follows them, and the last rotation does
    // the back substitution (one launch each instead of two)
    if (fn) {
      CHK(launch_gm_step_copy<T>(nrhs, -1, gpart, multidot_blocks(1, len, FUSE_BLOCKS), gst, gscale, r0, V, len, st));
    } else {
      CHK(launch_gm_start(nrhs, gnrm, nullptr, 0, gst, gscale, st));
      CHK((launch_scale_copy<CT, CT>(gscale, r0, len, V, len, len, nrhs, st)));
    }
    const int k = (maxit - done) < m ? (maxit - done) : m;
    for (int j = 0; j < k; ++j) {
      CHK(M((const void*)(V + j * vstr), (void*)(Z + j * vstr)));
      CHK(AZ((const void*)(Z + j * vstr), (void*)w));
      const bool fd = nrhs * 2 * (j + 1) <= FUSE_VALS;
      CHK((launch_multidot<CT, CT>(j + 1, V, vstr, len, w, len, len, nrhs, gpart, fd ? nullptr : gdots, st)));
      CHK(launch_gm_hcol(nrhs, j, fd ? nullptr : gdots, fd ? gpart : nullptr, multidot_blocks(j + 1, len, FUSE_BLOCKS), gst, gcoef,
                         st));
      // Gram-Schmidt update and its norm in one pass
      CHK((launch_axpy_norm<CT, CT>(j + 1, gcoef, V, vstr, len, w, len, nullptr, len, len, nrhs, gpart,
                                    fn ? nullptr : gnrm, st)));
      const bool last = j + 1 == k;
      if (fn && !last) {
        CHK(launch_gm_step_copy<T>(nrhs, j, gpart, nbn, gst, gscale, w, V + (j + 1) * vstr, len, st));
      } else {
        CHK(launch_gm_rotate(nrhs, j, fn ? nullptr : gnrm, fn ? gpart : nullptr, nbn, gst, gscale, st, last ? k : 0,
                             gcoef));
        if (!last) CHK((launch_scale_copy<CT, CT>(gscale, w, len, V + (j + 1) * vstr, len, len, nrhs, st)));
      }
    }
    CHK((launch_multiaxpy<CT, CT>(k, gcoef, Z, vstr, len, x, len, len, nrhs, st, done == 0)));
    done += k;
    if (done < maxit) {
      CHK(AR((const void*)x, b, (void*)w));
      r0 = w;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// hybrid Kaczmarz coarsest solve
// ---------------------------------------------------------------------------
template <typename T>
static KaczArgs<T> kacz_args(const elh_handle* H, bool adj) {
  const KaczData& K = H->kz;
  const LevelData& L = H->lv[H->nlev - 1];
  const int p = sizeof(T) == 8 ? 0 : 1, a = adj ? 1 : 0;
  KaczArgs<T> k;
  k.dim = H->d.dim;
  for (int i = 0; i < 3; ++i) {
    k.n[i] = L.n[i];
    k.nb[i] = K.nb[i];
    k.E[i] = K.E[i];
  }
  k.fs = L.fs;
  k.vs = L.vs;
  k.ns = K.ns;
  k.box = K.box;
  k.ls = K.ls;
  k.nreg = K.nreg;
  k.val = (const cx<T>*)K.val[a][p].p;
  k.inv = (const T*)K.inv[a][p].p;
  k.tab = (const int*)K.tab[a].p;
  k.dl = (const int*)K.dl[a].p;
  k.gptr = (const int*)K.gptr[a].p;
  k.gent = (const int*)K.gent[a].p;
  k.omega = (T)(H->d.coarse_damping > 0 ? H->d.coarse_damping : 0.8);
  return k;
}

// z = `sweeps` hybrid Kaczmarz sweeps from zero on S z_u = v_u (z_p = 0)
template <typename T>
static int kacz_apply(elh_handle* H, bool adj, const void* v, void* z, int nrhs, int sweeps) {
  const LevelData& L = H->lv[H->nlev - 1];
  KaczData& K = H->kz;
  if (ensure(K.scr, (size_t)nrhs * K.nreg * K.ls * sizeof(cx<T>))) return ELH_ERR_OOM;
  const KaczArgs<T> k = kacz_args<T>(H, adj);
  CHK(launch_zero(z, (int64_t)nrhs * L.vs * (int64_t)sizeof(cx<T>), H->st));
  for (int s = 0; s < sweeps; ++s) {
    CHK(launch_kacz_sweep<T>(k, v, s == 0 ? nullptr : z, K.scr.p, nrhs, H->st));
    CHK(launch_kacz_avg<T>(k, K.scr.p, z, nrhs, H->st));
  }
  return 0;
}

// x = FGMRES on the Schur complement (preconditioned by kacz_apply), then
// the pressure by back-substitution
template <typename T>
static int kacz_coarse_solve(elh_handle* H, bool adj, const void* b, void* x, int nrhs) {
  const int l = H->nlev - 1;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const elh_desc& d = H->d;
  const LevelData& L = H->lv[l];
  KaczData& K = H->kz;
  const size_t vb = (size_t)nrhs * L.vs * sizeof(cx<T>);
  if (ensure(K.t, vb) || ensure(K.y, vb) || ensure(K.bs, vb)) return ELH_ERR_OOM;
  const KaczArgs<T> k = kacz_args<T>(H, adj);
  const void* app = K.app[prec].p;
  hipStream_t st = H->st;
  // Schur right-hand side b_u - A_up A_pp^-1 b_p (p entries zero)
  CHK(launch_kacz_elem<T>(0, d.dim, L.fs, L.vs, nrhs, app, adj ? 1 : 0, b, nullptr, K.t.p, st));
  CHK(op_apply<T>(H, l, true, adj, K.t.p, nullptr, K.y.p, nrhs));
  CHK(launch_kacz_elem<T>(1, d.dim, L.fs, L.vs, nrhs, app, adj ? 1 : 0, b, K.y.p, K.bs.p, st));
  auto AZ = [&](const void* zi, void* wo) { return launch_kacz_spmv<T>(k, zi, nullptr, wo, nrhs, st); };
  auto AR = [&](const void* xi, const void* bi, void* ro) { return launch_kacz_spmv<T>(k, xi, bi, ro, nrhs, st); };
  auto M = [&](const void* v, void* z) { return kacz_apply<T>(H, adj, v, z, nrhs, d.coarse_sweeps); };
  if (d.coarse_rtol <= 0) {
    CHK(gmres_device<T>(H, H->kin[prec], L.vs, nrhs, AZ, AR, M, K.bs.p, x, d.coarse_restart, d.coarse_maxit));
  } else {
    GmresStats gs;
    int rc = gmres<T, T>(H, H->kin[prec], L.vs, nrhs, AZ, AR, M, K.bs.p, x, d.coarse_restart, d.coarse_maxit,
                         d.coarse_rtol, gs, nullptr);
    if (rc < 0) return rc;
  }
  // p = A_pp^-1 (b_p - A_pu u); the pressure entries of x are zero here
  CHK(op_apply<T>(H, l, true, adj, x, nullptr, K.y.p, nrhs));
  CHK(launch_kacz_elem<T>(2, d.dim, L.fs, L.vs, nrhs, app, adj ? 1 : 0, b, K.y.p, x, st));
  return 0;
}

// ---------------------------------------------------------------------------
// coarsest solve and cycle
// ---------------------------------------------------------------------------
template <typename T>
static int coarse_solve(elh_handle* H, bool adj, const void* b, void* x, int nrhs) {
  const int l = H->nlev - 1;
  const int prec = sizeof(T) == 8 ? 0 : 1;
  const elh_desc& d = H->d;
  if (d.coarse_mode == ELH_COARSE_RELAX) return op_sweeps_from_zero<T>(H, l, adj, b, x, nrhs, d.coarse_sweeps);
  if (d.coarse_mode == ELH_COARSE_KACZMARZ) {
    if (nrhs > MAXRHS_KRYLOV) return fail(ELH_ERR_ARG, "at most %d right-hand sides with the Kaczmarz coarse solve", MAXRHS_KRYLOV);
    return kacz_coarse_solve<T>(H, adj, b, x, nrhs);
  }
  if (d.coarse_mode == ELH_COARSE_DENSE) {
    // Q = inv(H_s^T):  H_s^{-1} b = Q^T b,  (H_s^H)^{-1} b = conj(Q) b
    const void* Q = prec == 0 ? H->dq64.p : H->dq32.p;
    return launch_dense_mv<T>(H->dn, Q, adj ? 0 : 1, adj ? 1 : 0, b, x, nrhs, H->st);
  }
  if (nrhs > MAXRHS_KRYLOV) return fail(ELH_ERR_ARG, "at most %d right-hand sides with the Krylov coarse solve", MAXRHS_KRYLOV);
  // ELH_COARSE_KRYLOV: GMRES on H_s preconditioned by Vanka sweeps
  LevelData& L = H->lv[l];
  auto AZ = [&](const void* zi, void* wo) { return op_apply<T>(H, l, true, adj, zi, nullptr, wo, nrhs); };
  auto AR = [&](const void* xi, const void* bi, void* ro) { return op_apply<T>(H, l, true, adj, xi, bi, ro, nrhs); };
  auto M = [&](const void* v, void* z) { return op_sweeps_from_zero<T>(H, l, adj, v, z, nrhs, d.coarse_sweeps); };
  if (d.coarse_rtol <= 0)
    return gmres_device<T>(H, H->kin[prec], L.vs, nrhs, AZ, AR, M, b, x, d.coarse_restart, d.coarse_maxit);
  GmresStats gs;
  int rc = gmres<T, T>(H, H->kin[prec], L.vs, nrhs, AZ, AR, M, b, x, d.coarse_restart, d.coarse_maxit,
                       d.coarse_rtol, gs, nullptr);
  return rc < 0 ? rc : 0;
}

template <typename T>
static int cycle(elh_handle* H, int l, bool adj, const void* b, void* x, int nrhs) {
  const int prec = sizeof(T) == 8 ? 0 : 1;
  if (l == H->nlev - 1) return coarse_solve<T>(H, adj, b, x, nrhs);
  LevelData& L = H->lv[l];
  LevelData& C = H->lv[l + 1];
  // with pre-smoothing the first half-sweep defines every entry of x
  if (H->d.nu1 == 0) CHK(launch_zero(x, (int64_t)nrhs * L.vs * csz(prec), H->st));
  bool zero = true;
  for (int s = 0; s < H->d.nu1; ++s) {
    CHK(op_relax<T>(H, l, adj, 0, b, x, nrhs, zero));
    zero = false;
    CHK(op_relax<T>(H, l, adj, 1, b, x, nrhs, false));
  }
  // coarse right-hand side R (b - H_s x), one fused launch
  const void* xr = zero ? nullptr : x;
  if (H->d.cycle_calls == 3) {
    // K-cycle: the coarse correction from two steps of flexible GCR on the
    // coarse system, each preconditioned by the coarse cycle (or the
    // coarsest solve); workspace E1, V1, R1, V2, E2 on the coarse level
    typedef cx<T> CT;
    const int64_t vec = (int64_t)nrhs * C.vs;
    CT* E1 = (CT*)C.kw[prec].p;
    CT* V1 = E1 + vec;
    CT* R1 = E1 + 2 * vec;
    CT* V2 = E1 + 3 * vec;
    CT* E2 = E1 + 4 * vec;
    double* kd = (double*)C.kc.p;                     // dots: 6 doubles per rhs
    double* kc1 = kd + 6 * MAXRHS_KRYLOV;             // stage-1 coefficients: 2 per rhs
    double* kc2 = kc1 + 2 * MAXRHS_KRYLOV;            // stage-2 coefficients: 4 per rhs
    double* ks = kc2 + 4 * MAXRHS_KRYLOV;             // state: 4 per rhs
    CHK(op_restrict_residual<T>(H, l, adj, xr, b, R1, nrhs));
    CHK(cycle<T>(H, l + 1, adj, R1, E1, nrhs));
    CHK(op_apply<T>(H, l + 1, true, adj, E1, nullptr, V1, nrhs));
    // the coefficient kernels finish small reductions themselves
    double* kp = (double*)H->part.p;
    const bool f1 = nrhs * 4 <= FUSE_VALS, f2 = nrhs * 6 <= FUSE_VALS;
    CHK((launch_multidot<CT, CT>(2, V1, vec, C.vs, V1, C.vs, C.vs, nrhs, kp, f1 ? nullptr : kd, H->st)));
    CHK(launch_kcycle_coef(1, f1 ? nullptr : kd, f1 ? kp : nullptr, multidot_blocks(2, C.vs, FUSE_BLOCKS), kc1, ks, nrhs,
                              H->st));
    CHK((launch_multiaxpy<CT, CT>(1, kc1, V1, 0, C.vs, R1, C.vs, C.vs, nrhs, H->st)));
    CHK(cycle<T>(H, l + 1, adj, R1, E2, nrhs));
    CHK(op_apply<T>(H, l + 1, true, adj, E2, nullptr, V2, nrhs));
    CHK((launch_multidot<CT, CT>(3, V1, vec, C.vs, V2, C.vs, C.vs, nrhs, kp, f2 ? nullptr : kd, H->st)));
    CHK(launch_kcycle_coef(2, f2 ? nullptr : kd, f2 ? kp : nullptr, multidot_blocks(3, C.vs, FUSE_BLOCKS), kc2, ks, nrhs,
                              H->st));
    // e = coef0 E1 + coef1 E2 written, not added (E2 = E1 + 4 vec)
    CHK((launch_multiaxpy<CT, CT>(2, kc2, E1, 4 * vec, C.vs, C.x[prec].p, C.vs, C.vs, nrhs, H->st, true)));
  } else {
    CHK(op_restrict_residual<T>(H, l, adj, xr, b, C.b[prec].p, nrhs));
    CHK(cycle<T>(H, l + 1, adj, C.b[prec].p, C.x[prec].p, nrhs));
  }
  if (H->d.cycle_calls == 2) {
    // W-cycle: second coarse cycle on the coarse residual, added to the
    // first (on every level: above the coarsest level these are two
    // coarsest solves, the second on the residual the first leaves)
    CHK(op_apply<T>(H, l + 1, true, adj, C.x[prec].p, C.b[prec].p, C.r[prec].p, nrhs));
    CHK((launch_scale_copy<cx<T>, cx<T>>(nullptr, C.r[prec].p, C.vs, C.b[prec].p, C.vs, C.vs, nrhs, H->st)));
    CHK((launch_scale_copy<cx<T>, cx<T>>(nullptr, C.x[prec].p, C.vs, L.r[prec].p, C.vs, C.vs, nrhs, H->st)));
    CHK(cycle<T>(H, l + 1, adj, C.b[prec].p, C.x[prec].p, nrhs));
    CHK((launch_multiaxpy<cx<T>, cx<T>>(1, (const double*)H->ones.p, L.r[prec].p, 0, C.vs, C.x[prec].p, C.vs, C.vs,
                                        nrhs, H->st)));
  }
  CHK(launch_prolong_add<T>(largs<T>(H, l, true), largs<T>(H, l + 1, true), H->d.dim, C.x[prec].p, x, nrhs, H->st));
  for (int s = 0; s < H->d.nu2; ++s) {
    CHK(op_relax<T>(H, l, adj, 0, b, x, nrhs, false));
    CHK(op_relax<T>(H, l, adj, 1, b, x, nrhs, false));
  }
  return 0;
}

// Run `fn` (which enqueues on H->st) through a cached hipGraph: recorded
// once on a private stream, then replayed on the handle's stream.  Only
// sequences with no host synchronisation are captured (the cycle with a
// fixed-budget coarse solve).
template <typename Fn>
static int run_graph(elh_handle* H, int prec, int adj, int nrhs, const void* in, void* out, Fn fn, int kind = 0,
                     int step = 0) {
  for (size_t i = 0; i < H->graphs.size(); ++i) {
    GraphEntry& g = H->graphs[i];
    if (g.kind == kind && g.step == step && g.prec == prec && g.adj == adj && g.nrhs == nrhs && g.in == in &&
        g.out == out) {
      if (g.gen == g_alloc_gen) {
        HIPCHK(hipGraphLaunch(g.exec, H->st));
        g_kernels.fetch_add(g.nkern, std::memory_order_relaxed);
        return 0;
      }
      (void)hipGraphExecDestroy(g.exec);
      H->graphs.erase(H->graphs.begin() + i);
      break;
    }
  }
  // the first (eager) run also performs any lazy allocation, so the recorded
  // addresses are final
  CHK(fn());
  const uint64_t gen = g_alloc_gen;
  hipStream_t saved = H->st;
  H->st = H->cap;
  hipError_t e = hipStreamBeginCapture(H->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    H->st = saved;
    return fail(ELH_ERR_HIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
  }
  int rc = fn();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(H->cap, &graph);
  H->st = saved;
  // the recorded launches did not run: take them off the count
  unsigned long long nkern = 0;
  if (graph) {
    size_t nn = 0;
    std::vector<hipGraphNode_t> nodes;
    if (hipGraphGetNodes(graph, nullptr, &nn) == hipSuccess && nn > 0) {
      nodes.resize(nn);
      if (hipGraphGetNodes(graph, nodes.data(), &nn) == hipSuccess)
        for (size_t i = 0; i < nn; ++i) {
          hipGraphNodeType t;
          if (hipGraphNodeGetType(nodes[i], &t) == hipSuccess && t == hipGraphNodeTypeKernel) ++nkern;
        }
    }
    g_kernels.fetch_sub(nkern, std::memory_order_relaxed);
  }
  if (rc != 0 || e != hipSuccess || gen != g_alloc_gen) {
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != 0) return rc > 0 ? fail(ELH_ERR_HIP, "launch failed during graph capture") : rc;
    if (e != hipSuccess) return fail(ELH_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    return 0;  // allocation changed while recording: keep running eagerly
  }
  GraphEntry g;
  g.kind = kind; g.step = step;
  g.prec = prec; g.adj = adj; g.nrhs = nrhs; g.in = in; g.out = out; g.gen = gen;
  g.nkern = nkern;
  e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ELH_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  H->graphs.push_back(g);
  return 0;
}

static bool graphs_ok(const elh_handle* H) {
  return H->use_graphs && !((H->d.coarse_mode == ELH_COARSE_KRYLOV || H->d.coarse_mode == ELH_COARSE_KACZMARZ) &&
                             H->d.coarse_rtol > 0);
}

// ---------------------------------------------------------------------------
// Outer flexible GMRES with its bookkeeping on the device (the solve entry
// points).  Right-preconditioned FGMRES(m) from x0 (zero or the caller's),
// relative-residual stop per rhs, classical Gram-Schmidt on the unnormalised
// basis (see gmres() above for the scaling), complex Givens rotations.  One
// iteration is three submissions with no host work between them -- the
// preconditioner cycle (a replayed hipGraph), the outer operator, and the
// Gram-Schmidt step (dots, Hessenberg column, update and norm, rotation and
// stop test, copy of the per-rhs status to the host; a replayed hipGraph per
// step index) -- and the host waits once per iteration, for the status.  At a
// restart the right-hand sides that have converged leave: the rest are packed
// into leading slots, so later cycles and operator applies skip them.  The
// solve is a resumable state machine, so that one host thread can drive
// several problems side by side (elh_solve_batch).
// ---------------------------------------------------------------------------
struct OuterOps {
  std::function<int(const void* v, void* z, int n)> M;                  // z = M v
  std::function<int(const void* z, void* w, int n)> AZ;                 // w = A z
  std::function<int(const void* x, const void* b, void* r, int n)> AR;  // r = b - A x
};

struct OuterSolve {
  elh_handle* H = nullptr;
  int nrhs = 0, m = 5, maxit = 1;
  double rtol = 0;
  bool x0 = false, z32 = false;
  int64_t len = 0;
  const cx<double>* q = nullptr;
  cx<double>* u = nullptr;
  OuterOps ops;
  KrylovWS* ws = nullptr;
  void* cyc_in = nullptr;  // float32 copy of v_j when the cycle reads float32 (z32)
  // packed rhs: slot i holds rhs map[i] (b, x in bp / xp, stride len)
  int np = 0;
  std::vector<int> map;
  const cx<double>* bp = nullptr;
  cx<double>* xp = nullptr;
  bool own = false;
  std::vector<double> nb, beta;
  std::vector<char> active, live;  // active: per rhs; live: per slot in the current restart
  GmresStats gs;
  std::unique_ptr<PhaseTimer> tm;
  int iters = 0, j = 0;
  bool in_restart = false, done = false;
  // basis vectors sit 1 MiB + 8 KiB (complex128) apart beyond their packed
  // length: at power-of-two strides the Gram-Schmidt kernels' streams (one
  // per basis vector, same offsets) lose 5-10 % of their bandwidth
  static constexpr int64_t kPad = 66048;
  int64_t vstr() const { return (int64_t)np * len + kPad; }
  cx<double>* V(int i) const { return (cx<double>*)ws->V.p + i * vstr(); }
  void* Z(int i) const { return (char*)ws->Z.p + i * vstr() * (z32 ? 8 : 16); }
};

// ||V_0||^2 (or ||q||^2) per packed slot -> host (synchronises)
static int os_norms(OuterSolve& S, const void* v, int n, std::vector<double>& out) {
  elh_handle* H = S.H;
  std::vector<zd> d;
  CHK((launch_multidot<cx<double>, cx<double>>(1, v, 0, S.len, v, S.len, S.len, n, (double*)H->part.p,
                                               (double*)H->dots.p, H->st)));
  CHK(fetch_dots(H, n, 1, d));
  out.resize(n);
  for (int i = 0; i < n; ++i) out[i] = sqrt(d[i].real());
  return 0;
}

static int os_begin(OuterSolve& S) {
  elh_handle* H = S.H;
  const int n = S.nrhs;
  const size_t vb = (size_t)n * S.len * 16;
  const size_t vpad = (size_t)OuterSolve::kPad;
  if (ensure(S.ws->V, (vb + vpad * 16) * (S.m + 1)) ||
      ensure(S.ws->Z, ((size_t)n * S.len + vpad) * (S.z32 ? 8 : 16) * S.m))
    return ELH_ERR_OOM;
  S.np = n;
  S.map.resize(n);
  for (int i = 0; i < n; ++i) S.map[i] = i;
  S.bp = S.q;
  S.xp = S.u;
  S.own = false;
  CHK(os_norms(S, S.q, n, S.nb));
  if (S.x0) {
    CHK(S.ops.AR(S.u, S.q, S.V(0), n));
    CHK(os_norms(S, S.V(0), n, S.beta));
  } else {
    CHK(launch_zero(S.u, vb, H->st));
    HIPCHK(hipMemcpyAsync(S.V(0), S.q, vb, hipMemcpyDeviceToDevice, H->st));
    S.beta = S.nb;
  }
  S.gs.iters.assign(n, 0);
  S.gs.restarts.assign(n, 0);
  S.gs.status.assign(n, ELH_NOT_CONVERGED);
  S.gs.relres.assign(n, 1.0);
  S.gs.history.assign(n, std::vector<double>());
  S.tm.reset(new PhaseTimer(S.gs.timing));
  S.active.assign(n, 0);
  int nact = 0;
  for (int s = 0; s < n; ++s) {
    if (!isfinite(S.nb[s]) || !isfinite(S.beta[s])) return fail(ELH_ERR_NUMERIC, "non-finite initial residual (rhs %d)", s);
    if (!(S.nb[s] > 0)) {
      // q = 0: the solution is 0 (an initial guess is discarded)
      S.gs.status[s] = ELH_OK;
      S.gs.relres[s] = 0.0;
      if (S.x0) CHK(launch_zero(S.u + (int64_t)s * S.len, S.len * 16, H->st));
    } else {
      S.gs.relres[s] = S.beta[s] / S.nb[s];
      S.active[s] = S.gs.relres[s] > S.rtol && S.beta[s] > 0;
      if (!S.active[s]) S.gs.status[s] = ELH_OK;
    }
    nact += S.active[s];
  }
  S.iters = 0;
  S.done = nact == 0;
  S.in_restart = false;
  return 0;
}

// pack the active rhs into the leading slots (b, x and the restart's first
// basis vector); rhs that leave have their iterate written back to u
static int os_compact(OuterSolve& S) {
  elh_handle* H = S.H;
  std::vector<int> keep;
  for (int i = 0; i < S.np; ++i)
    if (S.active[S.map[i]]) keep.push_back(i);
  if ((int)keep.size() == S.np) return 0;
  const size_t vb1 = (size_t)S.len * 16;
  if (!S.own) {
    if (ensure(S.ws->B, vb1 * S.nrhs) || ensure(S.ws->X, vb1 * S.nrhs)) return ELH_ERR_OOM;
    cx<double>* B = (cx<double>*)S.ws->B.p;
    cx<double>* X = (cx<double>*)S.ws->X.p;
    for (size_t k = 0; k < keep.size(); ++k) {
      const int i = keep[k], s = S.map[i];
      HIPCHK(hipMemcpyAsync(B + k * S.len, S.q + (int64_t)s * S.len, vb1, hipMemcpyDeviceToDevice, H->st));
      HIPCHK(hipMemcpyAsync(X + k * S.len, S.u + (int64_t)s * S.len, vb1, hipMemcpyDeviceToDevice, H->st));
    }
    S.bp = B;
    S.xp = X;
    S.own = true;
  } else {
    cx<double>* B = (cx<double>*)S.ws->B.p;
    cx<double>* X = (cx<double>*)S.ws->X.p;
    for (int i = 0; i < S.np; ++i)
      if (!S.active[S.map[i]])
        HIPCHK(hipMemcpyAsync(S.u + (int64_t)S.map[i] * S.len, X + (int64_t)i * S.len, vb1, hipMemcpyDeviceToDevice,
                              H->st));
    for (size_t k = 0; k < keep.size(); ++k)
      if ((int)k != keep[k]) {
        HIPCHK(hipMemcpyAsync(B + k * S.len, B + keep[k] * S.len, vb1, hipMemcpyDeviceToDevice, H->st));
        HIPCHK(hipMemcpyAsync(X + k * S.len, X + keep[k] * S.len, vb1, hipMemcpyDeviceToDevice, H->st));
      }
  }
  // the first basis vector (true residual of the last restart), slot stride len
  cx<double>* V0 = (cx<double>*)S.ws->V.p;
  for (size_t k = 0; k < keep.size(); ++k)
    if ((int)k != keep[k])
      HIPCHK(hipMemcpyAsync(V0 + k * S.len, V0 + keep[k] * S.len, vb1, hipMemcpyDeviceToDevice, H->st));
  std::vector<int> nm;
  for (int i : keep) nm.push_back(S.map[i]);
  S.map = nm;
  S.np = (int)keep.size();
  return 0;
}

static int os_restart_begin(OuterSolve& S) {
  elh_handle* H = S.H;
  CHK(os_compact(S));
  const int n = S.np;
  for (int i = 0; i < n; ++i) {
    const int s = S.map[i];
    H->hpar[4 * i] = S.active[s] ? 1.0 : 0.0;
    H->hpar[4 * i + 1] = S.nb[s];
    H->hpar[4 * i + 2] = S.rtol;
    H->hpar[4 * i + 3] = 0.0;
  }
  HIPCHK(hipMemcpyAsync(H->opar.p, H->hpar, (size_t)n * 32, hipMemcpyHostToDevice, H->st));
  double* part = (double*)H->opart.p;
  const bool fn = n * 2 <= FUSE_VALS;
  CHK((launch_multidot<cx<double>, cx<double>>(1, S.V(0), 0, S.len, S.V(0), S.len, S.len, n, part,
                                               fn ? nullptr : (double*)H->odots.p, H->st)));
  CHK(launch_go_start(n, fn ? nullptr : (double*)H->odots.p, fn ? part : nullptr,
                      multidot_blocks(1, S.len, FUSE_BLOCKS), (const double*)H->opar.p, (double*)H->ostate.p,
                      (double*)H->ostat.p, H->st));
  if (S.z32) CHK((launch_scale_copy<cx<double>, cx<float>>(nullptr, S.V(0), S.len, S.cyc_in, S.len, S.len, n, H->st)));
  S.live.assign(n, 0);
  for (int i = 0; i < n; ++i) S.live[i] = S.active[S.map[i]] && S.beta[S.map[i]] > 0;
  S.j = 0;
  S.in_restart = true;
  // the pinned parameter block is rewritten at the next restart, after the
  // synchronisation that ends this one
  return 0;
}

// the Gram-Schmidt step j: dots, Hessenberg column, update with its norm
// (and the float32 copy feeding the next cycle), rotation and stop test,
// status to the host
static int os_gs_step(OuterSolve& S) {
  elh_handle* H = S.H;
  const int n = S.np, j = S.j;
  const int64_t vs = S.vstr();
  cx<double>* W = S.V(j + 1);
  double* part = (double*)H->opart.p;
  const bool fd = n * 2 * (j + 1) <= FUSE_VALS, fn = n * 2 <= FUSE_VALS;
  CHK((launch_multidot<cx<double>, cx<double>>(j + 1, S.V(0), vs, S.len, W, S.len, S.len, n, part,
                                               fd ? nullptr : (double*)H->odots.p, H->st)));
  CHK(launch_go_hcol(n, j, fd ? nullptr : (double*)H->odots.p, fd ? part : nullptr,
                     multidot_blocks(j + 1, S.len, FUSE_BLOCKS), (double*)H->ostate.p, (double*)H->ocoef.p, H->st));
  if (S.z32)
    CHK((launch_axpy_norm<cx<double>, cx<float>>(j + 1, (const double*)H->ocoef.p, S.V(0), vs, S.len, W, S.len,
                                                 S.cyc_in, S.len, S.len, n, part,
                                                 fn ? nullptr : (double*)H->odots.p, H->st)));
  else
    CHK((launch_axpy_norm<cx<double>, cx<double>>(j + 1, (const double*)H->ocoef.p, S.V(0), vs, S.len, W, S.len,
                                                  nullptr, S.len, S.len, n, part,
                                                  fn ? nullptr : (double*)H->odots.p, H->st)));
  CHK(launch_go_rotate(n, j, fn ? nullptr : (double*)H->odots.p, fn ? part : nullptr, norm_blocks(S.len, FUSE_BLOCKS),
                       (double*)H->ostate.p, (double*)H->ostat.p, H->st));
  HIPCHK(hipMemcpyAsync(H->hstat, H->ostat.p, (size_t)n * 32, hipMemcpyDeviceToHost, H->st));
  return 0;
}

// enqueue iteration j of the current restart (no host synchronisation)
static int os_iter_enqueue(OuterSolve& S) {
  elh_handle* H = S.H;
  PhaseTimer& tm = *S.tm;
  const int n = S.np, j = S.j;
  tm.mark(0, H->st);
  CHK(S.ops.M(S.z32 ? (const void*)S.cyc_in : (const void*)S.V(j), S.Z(j), n));
  tm.mark(1, H->st);
  CHK(S.ops.AZ(S.Z(j), S.V(j + 1), n));
  tm.mark(2, H->st);
  auto step = [&]() { return os_gs_step(S); };
  CHK(H->use_graphs ? run_graph(H, S.z32 ? 1 : 0, 0, n, S.Z(0), S.V(0), step, 1, j) : step());
  tm.mark(3, H->st);
  return 0;
}

// wait for iteration j's status; ends the restart when every packed rhs has
// stopped, the budget is spent or the basis is full
static int os_restart_end(OuterSolve& S);
static int os_iter_finish(OuterSolve& S) {
  elh_handle* H = S.H;
  HIPCHK(hipStreamSynchronize(H->st));
  S.gs.t_precond += S.tm->span(0, 1);
  S.gs.t_apply += S.tm->span(1, 2);
  S.gs.t_orth += S.tm->span(2, 3);
  ++S.iters;
  bool any = false;
  for (int i = 0; i < S.np; ++i) {
    const double* st = H->hstat + 4 * i;
    const int s = S.map[i];
    if (st[3] != 0.0) return fail(ELH_ERR_NUMERIC, "non-finite norm in GMRES (rhs %d)", s);
    if (!S.live[i]) continue;
    S.gs.iters[s]++;
    S.gs.history[s].push_back(st[2]);
    S.live[i] = st[0] != 0.0;
    any = any || S.live[i];
  }
  ++S.j;
  if (!any || S.iters >= S.maxit || S.j == S.m) return os_restart_end(S);
  return 0;
}

// x += Z y per rhs, then the true residual (the next restart's first basis
// vector), its norm (synchronises) and the stop test
static int os_restart_end(OuterSolve& S) {
  elh_handle* H = S.H;
  const int n = S.np, k = S.j;
  CHK(launch_go_update(n, k, (const double*)H->ostate.p, (double*)H->ocoef.p, H->st));
  if (S.z32)
    CHK((launch_multiaxpy<cx<float>, cx<double>>(k, (const double*)H->ocoef.p, S.Z(0), S.vstr(), S.len, S.xp, S.len,
                                                 S.len, n, H->st)));
  else
    CHK((launch_multiaxpy<cx<double>, cx<double>>(k, (const double*)H->ocoef.p, S.Z(0), S.vstr(), S.len, S.xp,
                                                  S.len, S.len, n, H->st)));
  CHK(S.ops.AR(S.xp, S.bp, S.V(0), n));
  std::vector<double> bn;
  CHK(os_norms(S, S.V(0), n, bn));
  int nact = 0;
  for (int i = 0; i < n; ++i) {
    const int s = S.map[i];
    if (!S.active[s]) continue;
    S.gs.restarts[s]++;
    S.beta[s] = bn[i];
    if (!isfinite(bn[i])) return fail(ELH_ERR_NUMERIC, "non-finite residual (rhs %d)", s);
    S.gs.relres[s] = bn[i] / S.nb[s];
    if (S.gs.relres[s] <= S.rtol || bn[i] == 0) {
      S.active[s] = 0;
      S.gs.status[s] = ELH_OK;
    }
    nact += S.active[s];
  }
  S.in_restart = false;
  S.done = nact == 0 || S.iters >= S.maxit;
  return 0;
}

// write the packed iterates back to u
static int os_finish(OuterSolve& S) {
  if (!S.own) return 0;
  const cx<double>* X = (const cx<double>*)S.ws->X.p;
  for (int i = 0; i < S.np; ++i)
    HIPCHK(hipMemcpyAsync(S.u + (int64_t)S.map[i] * S.len, X + (int64_t)i * S.len, (size_t)S.len * 16,
                          hipMemcpyDeviceToDevice, S.H->st));
  return 0;
}

static int os_run(OuterSolve& S) {
  CHK(os_begin(S));
  while (!S.done) {
    if (!S.in_restart) CHK(os_restart_begin(S));
    CHK(os_iter_enqueue(S));
    CHK(os_iter_finish(S));
  }
  return os_finish(S);
}

// ---------------------------------------------------------------------------
// C ABI: level operations
// ---------------------------------------------------------------------------
extern "C" int elh_apply(elh_handle* H, int level, int flags, int dtype, int nrhs, const void* x, void* y) {
  int rc = check_common(H, level, dtype, nrhs);
  if (rc) return rc;
  if (!x || !y || x == y) return fail(ELH_ERR_ARG, "x and y must be distinct non-NULL pointers");
  bool sh = flags & ELH_SHIFTED, adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(op_apply<double>(H, level, sh, adj, x, nullptr, y, nrhs));
  else CHK(op_apply<float>(H, level, sh, adj, x, nullptr, y, nrhs));
  return 0;
}

extern "C" int elh_apply_f32in(elh_handle* H, int flags, int nrhs, const void* x, void* y) {
  int rc = check_common(H, 0, ELH_C128, nrhs);
  if (rc) return rc;
  if (!x || !y || x == y) return fail(ELH_ERR_ARG, "x and y must be distinct non-NULL pointers");
  if (flags & ELH_SHIFTED) return fail(ELH_ERR_ARG, "the outer operator is unshifted");
  const bool adj = flags & ELH_ADJOINT;
  const LevelData& L0 = H->lv[0];
  const bool direct = H->d.dim == 3 && !adj && L0.fs >= 16 * 16 * 16 &&
                      L0.fs * 16 <= (int64_t)0x7fffffff;
  if (direct) {
    CHK(op_apply_f32in(H, adj, x, y, nrhs));
    return 0;
  }
  // other layouts: widen to float64 first (as the solve does)
  if (ensure(H->tmpvec, (size_t)nrhs * L0.vs * 16)) return ELH_ERR_OOM;
  CHK((launch_scale_copy<cx<float>, cx<double>>(nullptr, x, L0.vs, H->tmpvec.p, L0.vs, L0.vs, nrhs, H->st)));
  CHK(op_apply<double>(H, 0, false, adj, H->tmpvec.p, nullptr, y, nrhs));
  return 0;
}

extern "C" int elh_residual(elh_handle* H, int level, int flags, int dtype, int nrhs, const void* b, const void* x,
                            void* r) {
  int rc = check_common(H, level, dtype, nrhs);
  if (rc) return rc;
  if (!x || !b || !r || x == r) return fail(ELH_ERR_ARG, "b, x, r must be non-NULL and r != x");
  bool sh = flags & ELH_SHIFTED, adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(op_apply<double>(H, level, sh, adj, x, b, r, nrhs));
  else CHK(op_apply<float>(H, level, sh, adj, x, b, r, nrhs));
  return 0;
}

extern "C" int elh_restrict_residual(elh_handle* H, int level, int flags, int dtype, int nrhs, const void* b,
                                     const void* x, void* rc_out) {
  int rc = check_common(H, level, dtype, nrhs);
  if (rc) return rc;
  if (level >= H->nlev - 1) return fail(ELH_ERR_ARG, "no coarser level below %d", level);
  if (!b || !rc_out) return fail(ELH_ERR_ARG, "b and rc must be non-NULL");
  bool adj = flags & ELH_ADJOINT;
  if (rc_out == b || (x && rc_out == x)) return fail(ELH_ERR_ARG, "rc must not alias b or x");
  if (dtype == ELH_C128) CHK(op_restrict_residual<double>(H, level, adj, x, b, rc_out, nrhs));
  else CHK(op_restrict_residual<float>(H, level, adj, x, b, rc_out, nrhs));
  return 0;
}

extern "C" int elh_prolong_add(elh_handle* H, int level, int dtype, int nrhs, const void* e, void* x) {
  int rc = check_common(H, level, dtype, nrhs);
  if (rc) return rc;
  if (level >= H->nlev - 1) return fail(ELH_ERR_ARG, "no coarser level below %d", level);
  if (!e || !x) return fail(ELH_ERR_ARG, "e and x must be non-NULL");
  if (dtype == ELH_C128)
    CHK(launch_prolong_add<double>(largs<double>(H, level, true), largs<double>(H, level + 1, true), H->d.dim, e, x,
                                   nrhs, H->st));
  else
    CHK(launch_prolong_add<float>(largs<float>(H, level, true), largs<float>(H, level + 1, true), H->d.dim, e, x,
                                  nrhs, H->st));
  return 0;
}

extern "C" int elh_relax(elh_handle* H, int level, int flags, int dtype, int nrhs, int colour, const void* b,
                         void* x) {
  int rc = check_common(H, level, dtype, nrhs);
  if (rc) return rc;
  if (colour != 0 && colour != 1) return fail(ELH_ERR_ARG, "colour must be 0 or 1");
  if (!b || !x || b == x) return fail(ELH_ERR_ARG, "b and x must be distinct non-NULL pointers");
  const int prec = prec_of(dtype);
  if (ensure_cycle_bufs(H, prec, nrhs)) return ELH_ERR_OOM;
  bool adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(op_relax<double>(H, level, adj, colour, b, x, nrhs, false));
  else CHK(op_relax<float>(H, level, adj, colour, b, x, nrhs, false));
  return 0;
}

extern "C" int elh_relax_noalloc(elh_handle* H, int level, int flags, int dtype, int nrhs, int colour,
                                 const void* b, void* x) {
  int rc = check_common(H, level, dtype, nrhs);
  if (rc) return rc;
  if (colour != 0 && colour != 1) return fail(ELH_ERR_ARG, "colour must be 0 or 1");
  if (!b || !x || b == x) return fail(ELH_ERR_ARG, "b and x must be distinct non-NULL pointers");
  const size_t need = (size_t)nrhs * (size_t)H->lv[level].vs * csz(prec_of(dtype));
  if (need > (size_t)ELH_NOALLOC_SCRATCH_BYTES)
    return fail(ELH_ERR_ARG, "the residual of %d right-hand side(s) on level %d needs %zu bytes; the allocation-free "
                "relaxation holds at most %zu", nrhs, level, need, (size_t)ELH_NOALLOC_SCRATCH_BYTES);
  if (!H->scratch) return fail(ELH_ERR_STATE, "the relaxation work array has no device address");
  const bool adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(op_relax_with<double>(H, level, adj, colour, b, x, H->scratch, nrhs));
  else CHK(op_relax_with<float>(H, level, adj, colour, b, x, H->scratch, nrhs));
  return 0;
}

extern "C" int elh_coarse_solve(elh_handle* H, int flags, int dtype, int nrhs, const void* b, void* x) {
  int rc = check_common(H, H ? H->nlev - 1 : 0, dtype, nrhs);
  if (rc) return rc;
  if (!b || !x || b == x) return fail(ELH_ERR_ARG, "b and x must be distinct non-NULL pointers");
  const int prec = prec_of(dtype);
  if (ensure_cycle_bufs(H, prec, nrhs)) return ELH_ERR_OOM;
  bool adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(coarse_solve<double>(H, adj, b, x, nrhs));
  else CHK(coarse_solve<float>(H, adj, b, x, nrhs));
  return 0;
}

extern "C" int elh_kaczmarz(elh_handle* H, int flags, int dtype, int nrhs, int sweeps, const void* b, void* x) {
  int rc = check_common(H, H ? H->nlev - 1 : 0, dtype, nrhs);
  if (rc) return rc;
  if (H->d.coarse_mode != ELH_COARSE_KACZMARZ) return fail(ELH_ERR_ARG, "handle was not created with ELH_COARSE_KACZMARZ");
  if (!b || !x || b == x) return fail(ELH_ERR_ARG, "b and x must be distinct non-NULL pointers");
  if (sweeps < 1) return fail(ELH_ERR_ARG, "sweeps must be >= 1");
  if (nrhs > MAXRHS_KRYLOV) return fail(ELH_ERR_ARG, "at most %d right-hand sides", MAXRHS_KRYLOV);
  const bool adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(kacz_apply<double>(H, adj, b, x, nrhs, sweeps));
  else CHK(kacz_apply<float>(H, adj, b, x, nrhs, sweeps));
  return 0;
}

// The K-cycle and the Krylov / Kaczmarz coarsest solves keep per-rhs
// coefficients and reductions in buffers of MAXRHS_KRYLOV entries.
static int check_cycle_nrhs(const elh_handle* H, int nrhs) {
  if (nrhs <= MAXRHS_KRYLOV) return 0;
  if (H->d.cycle_calls == 3) return fail(ELH_ERR_ARG, "at most %d right-hand sides with the K-cycle", MAXRHS_KRYLOV);
  if (H->nlev >= 1 && (H->d.coarse_mode == ELH_COARSE_KRYLOV || H->d.coarse_mode == ELH_COARSE_KACZMARZ))
    return fail(ELH_ERR_ARG, "at most %d right-hand sides with the Krylov / Kaczmarz coarsest solve", MAXRHS_KRYLOV);
  return 0;
}

extern "C" int elh_vcycle(elh_handle* H, int flags, int dtype, int nrhs, const void* b, void* x) {
  int rc = check_common(H, 0, dtype, nrhs);
  if (rc) return rc;
  if (!b || !x || b == x) return fail(ELH_ERR_ARG, "b and x must be distinct non-NULL pointers");
  rc = check_cycle_nrhs(H, nrhs);
  if (rc) return rc;
  const int prec = prec_of(dtype);
  if (ensure_cycle_bufs(H, prec, nrhs)) return ELH_ERR_OOM;
  bool adj = flags & ELH_ADJOINT;
  if (dtype == ELH_C128) CHK(cycle<double>(H, 0, adj, b, x, nrhs));
  else CHK(cycle<float>(H, 0, adj, b, x, nrhs));
  return 0;
}

// ---------------------------------------------------------------------------
// C ABI: solves
// ---------------------------------------------------------------------------
// Validate a solve and set up its state (operators of the problem's
// precision mode, workspaces); nothing is launched.
static int os_setup(elh_handle* H, bool adj, int nrhs, const void* q, void* u, const elh_solve_opts* opts, bool timing,
                    OuterSolve& S) {
  int rc = check_common(H, 0, ELH_C128, nrhs);
  if (rc) return rc;
  if (!q || !u || q == u) return fail(ELH_ERR_ARG, "q and u must be distinct non-NULL pointers");
  if (!opts) return fail(ELH_ERR_ARG, "opts is NULL");
  if (opts->restart < 1 || opts->restart + 1 > MAXDOT) return fail(ELH_ERR_ARG, "restart must be in 1..%d", MAXDOT - 1);
  if (opts->maxit < 1) return fail(ELH_ERR_ARG, "maxit must be >= 1");
  if (nrhs > MAXRHS_KRYLOV) return fail(ELH_ERR_ARG, "at most %d right-hand sides per solve", MAXRHS_KRYLOV);
  if (!(opts->rtol >= 0)) return fail(ELH_ERR_ARG, "rtol must be >= 0");
  if (opts->zero_x0 != 0 && opts->zero_x0 != 1) return fail(ELH_ERR_ARG, "zero_x0 must be 0 or 1");
  if (opts->store_z_fp32 != 0 && opts->store_z_fp32 != 1) return fail(ELH_ERR_ARG, "store_z_fp32 must be 0 or 1");
  if (opts->store_z_fp32 && H->d.precond_dtype != ELH_C64)
    return fail(ELH_ERR_ARG, "store_z_fp32 needs the float32 cycle (precond_dtype ELH_C64)");
  const int pprec = prec_of(H->d.precond_dtype);
  if (ensure_cycle_bufs(H, pprec, nrhs)) return ELH_ERR_OOM;
  LevelData& L0 = H->lv[0];
  const int64_t len = L0.vs;
  S.H = H;
  S.nrhs = nrhs;
  S.m = opts->restart;
  S.maxit = opts->maxit;
  S.rtol = opts->rtol;
  S.x0 = opts->zero_x0 == 0;
  S.len = len;
  S.q = (const cx<double>*)q;
  S.u = (cx<double>*)u;
  S.gs.timing = timing;
  S.ops.AR = [H, adj](const void* xi, const void* bi, void* ro, int n) {
    return op_apply<double>(H, 0, false, adj, xi, bi, ro, n);
  };
  if (pprec == 0) {
    S.ws = &H->kout[0];
    S.ops.AZ = [H, adj](const void* zi, void* wo, int n) { return op_apply<double>(H, 0, false, adj, zi, nullptr, wo, n); };
    S.ops.M = [H, adj](const void* v, void* z, int n) {
      auto fn = [&]() { return cycle<double>(H, 0, adj, v, z, n); };
      return graphs_ok(H) ? run_graph(H, 0, adj, n, v, z, fn) : fn();
    };
  } else if (!opts->store_z_fp32) {
    // float32 cycle, z_j widened to complex128: the cycle reads a float32
    // copy of v_j and writes float32 into a level-0 work buffer, which is
    // widened into Z (exact); everything else is the float64 solve
    S.ws = &H->kout[0];
    LevelData* W = &H->lv[0];
    S.ops.M = [H, adj, W, len](const void* v, void* z, int n) {
      CHK((launch_scale_copy<cx<double>, cx<float>>(nullptr, v, len, W->b[1].p, len, len, n, H->st)));
      auto fn = [&]() { return cycle<float>(H, 0, adj, W->b[1].p, W->x[1].p, n); };
      CHK(graphs_ok(H) ? run_graph(H, 1, adj, n, W->b[1].p, W->x[1].p, fn) : fn());
      return launch_scale_copy<cx<float>, cx<double>>(nullptr, W->x[1].p, len, z, len, len, n, H->st);
    };
    S.ops.AZ = [H, adj](const void* zi, void* wo, int n) { return op_apply<double>(H, 0, false, adj, zi, nullptr, wo, n); };
  } else {
    // float32 cycle (Section 5.3 mixed precision): the cycle reads a
    // float32 copy of the basis vector (written by the Gram-Schmidt pass)
    // and writes z_j in float32; the outer operator reads z_j in float32
    // and computes in float64; all Krylov state stays float64.
    KrylovWS* ws = &H->kout[1];
    S.ws = ws;
    S.z32 = true;
    S.cyc_in = L0.b[1].p;
    S.ops.M = [H, adj](const void* v, void* z, int n) {
      auto fn = [&]() { return cycle<float>(H, 0, adj, v, z, n); };
      return graphs_ok(H) ? run_graph(H, 1, adj, n, v, z, fn) : fn();
    };
    const bool direct = H->d.dim == 3 && !adj && L0.fs >= 16 * 16 * 16 && L0.fs * 16 <= (int64_t)0x7fffffff;
    if (!direct && ensure(ws->t, (size_t)nrhs * len * 16)) return ELH_ERR_OOM;
    S.ops.AZ = [H, adj, direct, ws, len](const void* zi, void* wo, int n) {
      if (direct) return op_apply_f32in(H, adj, zi, wo, n);
      CHK((launch_scale_copy<cx<float>, cx<double>>(nullptr, zi, len, ws->t.p, len, len, n, H->st)));
      return op_apply<double>(H, 0, false, adj, ws->t.p, nullptr, wo, n);
    };
  }
  return 0;
}

// statistics of a finished solve; returns the most severe per-rhs status
static int os_report(const OuterSolve& S, double wall, unsigned long long kernels, elh_solve_stats* stats) {
  int worst = ELH_OK;
  const GmresStats& gs = S.gs;
  for (int s = 0; s < S.nrhs; ++s) {
    if (stats) {
      stats[s].iters = gs.iters[s];
      stats[s].restarts = gs.restarts[s];
      stats[s].status = gs.status[s];
      stats[s].relres = gs.relres[s];
      const int nh = (int)gs.history[s].size();
      const int cap = stats[s].history && stats[s].history_cap > 0 ? stats[s].history_cap : 0;
      stats[s].history_len = nh < cap ? nh : cap;
      for (int i = 0; i < stats[s].history_len; ++i) stats[s].history[i] = gs.history[s][i];
      stats[s].t_total_ms = wall;
      stats[s].t_precond_ms = gs.t_precond;
      stats[s].t_apply_ms = gs.t_apply;
      stats[s].t_orth_ms = gs.t_orth;
      stats[s].kernels = kernels;
    }
    if (gs.status[s] != ELH_OK) worst = gs.status[s];
  }
  return worst;
}

static int solve_impl(elh_handle* H, bool adj, int nrhs, const void* q, void* u, const elh_solve_opts* opts,
                      elh_solve_stats* stats) {
  const auto wall0 = std::chrono::steady_clock::now();
  const unsigned long long k0 = g_kernels.load();
  OuterSolve S;
  int rc = os_setup(H, adj, nrhs, q, u, opts, stats != nullptr, S);
  if (rc) return rc;
  rc = os_run(S);
  if (rc < 0) return rc;
  const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
  return os_report(S, wall, g_kernels.load() - k0, stats);
}

extern "C" int elh_solve(elh_handle* H, int nrhs, const void* q, void* u, const elh_solve_opts* opts,
                         elh_solve_stats* stats) {
  return solve_impl(H, false, nrhs, q, u, opts, stats);
}

extern "C" int elh_solve_adjoint(elh_handle* H, int nrhs, const void* r, void* v, const elh_solve_opts* opts,
                                 elh_solve_stats* stats) {
  return solve_impl(H, true, nrhs, r, v, opts, stats);
}

// Several problems from one host thread: each unfinished problem has one
// iteration (cycle, operator and Gram-Schmidt step) in flight on its own
// stream, and the host polls the streams, finishing and re-enqueueing each
// problem as its status arrives, so the problems' kernels run side by side
// on the GPU; a problem leaves when its rhs have converged.
static int batch_drive(int nprob, elh_handle* const* hs, const int* nrhs, const void* const* q, void* const* u,
                       const elh_solve_opts* opts, elh_solve_stats* stats) {
  if (nprob < 1 || !hs || !nrhs || !q || !u || !opts) return fail(ELH_ERR_ARG, "invalid batch arguments");
  std::vector<int> off(nprob + 1, 0);
  for (int i = 0; i < nprob; ++i) {
    if (!hs[i] || !hs[i]->ok) return fail(ELH_ERR_STATE, "invalid handle %d", i);
    if (nrhs[i] < 1) return fail(ELH_ERR_ARG, "nrhs[%d] must be >= 1", i);
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(ELH_ERR_ARG, "handle %d appears twice", i);
    off[i + 1] = off[i] + nrhs[i];
  }
  const auto wall0 = std::chrono::steady_clock::now();
  const unsigned long long k0 = g_kernels.load();
  std::vector<OuterSolve> S(nprob);
  std::vector<int> rcs(nprob, 0);
  std::vector<std::string> errs(nprob);
  auto failed = [&](int i, int rc) {
    if (rc < 0) {
      rcs[i] = rc;
      errs[i] = g_err;
      S[i].done = true;
    }
    return rc < 0;
  };
  for (int i = 0; i < nprob; ++i) {
    int rc = os_setup(hs[i], false, nrhs[i], q[i], u[i], opts, stats != nullptr, S[i]);
    if (rc > 0) rc = fail(ELH_ERR_HIP, "launch failed");
    if (failed(i, rc)) continue;
    failed(i, os_begin(S[i]));
  }
  // each problem's next iteration is enqueued as soon as its own status
  // has arrived (its stream is idle), not when the whole round has: the
  // small problems do not wait for the largest one's iterations
  std::vector<char> queued(nprob, 0);
  auto enqueue = [&](int i) {
    int rc = S[i].in_restart ? 0 : os_restart_begin(S[i]);
    if (!rc) rc = os_iter_enqueue(S[i]);
    if (rc > 0) rc = fail(ELH_ERR_HIP, "launch failed");
    if (!failed(i, rc)) queued[i] = 1;
  };
  for (int i = 0; i < nprob; ++i)
    if (!S[i].done) enqueue(i);
  for (;;) {
    bool pending = false, progressed = false;
    for (int i = 0; i < nprob; ++i) {
      if (S[i].done || !queued[i]) continue;
      pending = true;
      // not ready yet: look again later; any other answer (done, or an
      // error, which the synchronisation in os_iter_finish reports) ends
      // this iteration
      if (hipStreamQuery(S[i].H->st) == hipErrorNotReady) continue;
      queued[i] = 0;
      progressed = true;
      int rc = os_iter_finish(S[i]);
      if (rc > 0) rc = fail(ELH_ERR_HIP, "launch failed");
      if (failed(i, rc) || S[i].done) continue;
      enqueue(i);
    }
    if (!pending) break;
    if (!progressed) std::this_thread::yield();
  }
  for (int i = 0; i < nprob; ++i)
    if (!rcs[i]) {
      int rc = os_finish(S[i]);
      if (rc > 0) rc = fail(ELH_ERR_HIP, "copy failed");
      failed(i, rc);
    }
  const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
  int worst = ELH_OK;
  for (int i = 0; i < nprob; ++i) {
    if (rcs[i] < 0) {
      if (worst >= 0 || rcs[i] < worst) {
        worst = rcs[i];
        snprintf(g_err, sizeof(g_err), "problem %d: %s", i, errs[i].c_str());
      }
      continue;
    }
    const int r = os_report(S[i], wall, g_kernels.load() - k0, stats ? stats + off[i] : nullptr);
    if (r > 0 && worst == ELH_OK) worst = r;
  }
  return worst;
}

extern "C" int elh_solve_batch(int nprob, elh_handle* const* hs, const int* nrhs, const void* const* q,
                               void* const* u, const elh_solve_opts* opts, elh_solve_stats* stats) {
  return batch_drive(nprob, hs, nrhs, q, u, opts, stats);
}

// uneven-grid batch handle: problem handles on library-owned streams
struct elh_batch {
  std::vector<elh_handle*> h;
  std::vector<hipStream_t> st;
  std::vector<hipEvent_t> ev;
  hipStream_t caller = nullptr;
  hipEvent_t cev = nullptr;
};

extern "C" int elh_batch_destroy(elh_batch* B) {
  if (!B) return 0;
  for (auto* h : B->h) elh_destroy(h);
  for (auto s : B->st) (void)hipStreamDestroy(s);
  for (auto e : B->ev) (void)hipEventDestroy(e);
  if (B->cev) (void)hipEventDestroy(B->cev);
  delete B;
  return 0;
}

extern "C" int elh_batch_create(int nprob, const elh_desc* descs, const double* const* lam, const double* const* mu,
                                const double* const* rho, void* stream, elh_batch** out) {
  if (!out) return fail(ELH_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (nprob < 1 || nprob > 4096 || !descs || !lam || !mu || !rho) return fail(ELH_ERR_ARG, "invalid batch arguments");
  for (int i = 0; i < nprob; ++i) {
    const int rc = check_desc(&descs[i]);
    if (rc) return fail(rc, "problem %d: %s", i, std::string(g_err).c_str());
  }
  elh_batch* B = new elh_batch();
  B->caller = (hipStream_t)stream;
  if (hipEventCreateWithFlags(&B->cev, hipEventDisableTiming) != hipSuccess) {
    elh_batch_destroy(B);
    return fail(ELH_ERR_HIP, "event creation failed");
  }
  // the media were written on the caller's stream
  if (hipEventRecord(B->cev, B->caller) != hipSuccess) {
    elh_batch_destroy(B);
    return fail(ELH_ERR_HIP, "event record failed");
  }
  for (int i = 0; i < nprob; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      if (s) (void)hipStreamDestroy(s);
      elh_batch_destroy(B);
      return fail(ELH_ERR_HIP, "stream creation failed");
    }
    B->st.push_back(s);
    B->ev.push_back(e);
    if (hipStreamWaitEvent(s, B->cev, 0) != hipSuccess) {
      elh_batch_destroy(B);
      return fail(ELH_ERR_HIP, "stream wait failed");
    }
    elh_handle* h = nullptr;
    const int rc = elh_create(&descs[i], lam[i], mu[i], rho[i], s, &h);
    if (rc) {
      const std::string msg = g_err;
      elh_batch_destroy(B);
      return fail(rc, "problem %d: %s", i, msg.c_str());
    }
    B->h.push_back(h);
  }
  *out = B;
  return 0;
}

extern "C" int elh_batch_size(const elh_batch* B) { return B ? (int)B->h.size() : ELH_ERR_ARG; }

extern "C" int elh_batch_handle(elh_batch* B, int i, elh_handle** h) {
  if (!B || !h || i < 0 || i >= (int)B->h.size()) return fail(ELH_ERR_ARG, "invalid batch or index");
  *h = B->h[i];
  return 0;
}

extern "C" int elh_batch_solve(elh_batch* B, const int* nrhs, const void* const* q, void* const* u,
                               const elh_solve_opts* opts, elh_solve_stats* stats) {
  if (!B) return fail(ELH_ERR_ARG, "batch is NULL");
  const int n = (int)B->h.size();
  // inputs were written on the caller's stream; outputs are ready on it
  // when the call returns (after its own synchronisation)
  HIPCHK(hipEventRecord(B->cev, B->caller));
  for (int i = 0; i < n; ++i) HIPCHK(hipStreamWaitEvent(B->st[i], B->cev, 0));
  const int rc = batch_drive(n, B->h.data(), nrhs, q, u, opts, stats);
  for (int i = 0; i < n; ++i) {
    if (hipEventRecord(B->ev[i], B->st[i]) != hipSuccess || hipStreamWaitEvent(B->caller, B->ev[i], 0) != hipSuccess)
      return rc < 0 ? rc : fail(ELH_ERR_HIP, "stream join failed");
  }
  return rc;
}

extern "C" int elh_gradient(elh_handle* H, int nrhs, const void* u, const void* v, double* g_lam, double* g_mu,
                            double* g_rho) {
  int rc = check_common(H, 0, ELH_C128, nrhs);
  if (rc) return rc;
  if (!u || !v || !g_lam || !g_mu || !g_rho) return fail(ELH_ERR_ARG, "u, v and the gradients must be non-NULL");
  // the gradient is of the unshifted forward operator
  CHK(launch_gradient(largs<double>(H, 0, false), H->d.dim, nrhs, u, v, g_lam, g_mu, g_rho, H->st));
  return 0;
}

extern "C" int elh_receivers(elh_handle* H, int nrhs, const void* u, int nrec, const int64_t* idx, const void* dobs,
                             void* d, double* phi) {
  int rc = check_common(H, 0, ELH_C128, nrhs);
  if (rc) return rc;
  if (nrec < 1 || !u || !idx || !d) return fail(ELH_ERR_ARG, "u, idx and d must be non-NULL and nrec >= 1");
  if (d == u || (const void*)d == (const void*)idx) return fail(ELH_ERR_ARG, "d must not alias u or idx");
  CHK(launch_rec_sample(H->lv[0].vs, nrec, idx, u, dobs, d, phi, nrhs, H->st));
  return 0;
}

extern "C" int elh_inject(elh_handle* H, int nrhs, int nrec, const int64_t* idx, const void* r, double scale,
                          void* v) {
  int rc = check_common(H, 0, ELH_C128, nrhs);
  if (rc) return rc;
  if (nrec < 1 || !idx || !r || !v) return fail(ELH_ERR_ARG, "idx, r and v must be non-NULL and nrec >= 1");
  if (v == r || (const void*)v == (const void*)idx) return fail(ELH_ERR_ARG, "v must not alias r or idx");
  if (nrhs > 65535) return fail(ELH_ERR_ARG, "at most 65535 right-hand sides");
  if (!std::isfinite(scale)) return fail(ELH_ERR_ARG, "scale must be finite");
  CHK(launch_zero(v, (int64_t)nrhs * H->lv[0].vs * 16, H->st));
  CHK(launch_rec_inject(H->lv[0].vs, nrec, idx, r, scale, v, nrhs, H->st));
  return 0;
}

extern "C" const char* elh_status_string(int s) {
  switch (s) {
    case ELH_OK: return "ok";
    case ELH_NOT_CONVERGED: return "not converged";
    case ELH_ERR_ARG: return "invalid argument";
    case ELH_ERR_HIP: return "HIP runtime error";
    case ELH_ERR_NUMERIC: return "numerical breakdown";
    case ELH_ERR_OOM: return "out of device memory";
    case ELH_ERR_STATE: return "invalid state";
    default: return "unknown status";
  }
}

extern "C" const char* elh_last_error(void) { return g_err; }
