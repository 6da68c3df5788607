// Internal declarations shared by the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "elh_device.h"

#include <atomic>

namespace elh {

// kernels this library has had executed: eager launches plus the kernel
// nodes of replayed graphs (solve statistics, launches per iteration)
extern std::atomic<unsigned long long> g_kernels;
#define ELH_LAUNCH(...)                                                \
  do {                                                                 \
    ::elh::g_kernels.fetch_add(1, std::memory_order_relaxed);          \
    hipLaunchKernelGGL(__VA_ARGS__);                                   \
  } while (0)

constexpr int MAXDOT = 16;         // most vectors in one fused multi-dot
constexpr int MAXRHS_KRYLOV = 64;  // right-hand sides per Krylov solve (reduction buffers)
// per-rhs device GMRES state in doubles: H (MAXDOT x MAXDOT complex), g and
// sines (MAXDOT complex each), cosines (MAXDOT)
constexpr int GM_STRIDE = 2 * MAXDOT * MAXDOT + 2 * MAXDOT + 2 * MAXDOT + MAXDOT;

template <typename T>
int launch_apply(const LevelArgs<T>& L, int dim, bool adj, const void* x, const void* b, void* y, int nrhs,
                 hipStream_t st);
template <typename T>
int launch_vanka(const LevelArgs<T>& L, int dim, bool adj, const void* r, void* x, int colour, double w, int nrhs,
                 hipStream_t st, bool write = false);  // write: 3D first half-sweep, x not yet set
template <typename T>
int launch_restrict(const LevelArgs<T>& F, const LevelArgs<T>& C, int dim, const void* r, void* rc, int nrhs,
                    hipStream_t st);
template <typename T>
int launch_prolong_add(const LevelArgs<T>& F, const LevelArgs<T>& C, int dim, const void* e, void* x, int nrhs,
                       hipStream_t st);
// rc = R (b - H_s x) in one point-wise launch (one thread per coarse cell)
template <typename T>
int launch_restrict_resid(const LevelArgs<T>& F, const LevelArgs<T>& C, int dim, bool adj, const void* x,
                          const void* b, void* rc, int nrhs, hipStream_t st);

// 3D forward apply / residual, component-split wavefront march: three
// wavefronts per x_2 row (one per displacement component) marching along
// x_3, DPP for x_1 neighbours, one LDS hand-off per plane for the p row.
// x holds complex TI (TI = T, or float with T = double); b, y complex T.
template <typename T, typename TI = T>
int launch_apply3d_w3(const LevelArgs<T>& L, const void* x, const void* b, void* y, int nrhs, int zc,
                      hipStream_t st);
// Same march for the adjoint H^H.
template <typename T>
int launch_apply3d_w3_adj(const LevelArgs<T>& L, const void* x, const void* b, void* y, int nrhs, int zc,
                          hipStream_t st);
// rc = R (b - H_s x) (adj: H_s^H) fused into the march: a workgroup of
// seven wavefronts computes the residual rows of fine rows 2J and 2J+1 (and
// the u_2 rows of row 2J-1) and restricts them to coarse row J; the fine
// residual is never stored.  zc: x_3 chunk in coarse planes (< 0: exactly
// -zc).  F must have even n (it has a coarser level).
template <typename T>
int launch_restrict_resid3d_w3(const LevelArgs<T>& F, const LevelArgs<T>& C, bool adj, const void* x,
                               const void* b, void* rc, int nrhs, int zc, hipStream_t st);
int launch_coarsen_media(int dim, const int* nf, const double* a, double* out, hipStream_t st);
int launch_media_finish(int64_t n, const double* lam, const double* mu, const double* rho, double* kap, float* mu32,
                        float* rho32, float* kap32, hipStream_t st);
template <typename TV, typename TW>
int launch_multidot(int m, const void* V, int64_t vstride_vec, int64_t vstride_rhs, const void* w,
                    int64_t wstride_rhs, int64_t len, int nrhs, double* part, double* out, hipStream_t st);
template <typename TV, typename TW>
int launch_multiaxpy(int m, const double* coef, const void* V, int64_t vstride_vec, int64_t vstride_rhs, void* w,
                     int64_t wstride_rhs, int64_t len, int nrhs, hipStream_t st, bool set = false);  // set: w = sum
// w += sum_i coef_i V_i in place with ||w||^2 per rhs into out[2s] (part:
// scratch of 512*MAXDOT*2 doubles per rhs); f (optional) receives w in TF.
template <typename TV, typename TF>
int launch_axpy_norm(int m, const double* coef, const void* V, int64_t vstride_vec, int64_t vstride_rhs, void* w,
                     int64_t wstride_rhs, void* f, int64_t fstride_rhs, int64_t len, int nrhs, double* part,
                     double* out, hipStream_t st);
// Reductions: launch_multidot / launch_axpy_norm leave per-block partials in
// `part` and, unless `out` is null, reduce them into `out`.  With `out` null
// they use at most FUSE_BLOCKS blocks per rhs (multidot_blocks(m, len,
// FUSE_BLOCKS) / norm_blocks(len, FUSE_BLOCKS)), and the consumer below,
// given the partials instead of `out`, finishes the reduction; this is for
// reductions of at most FUSE_VALS values (nrhs * 2m).
constexpr int FUSE_VALS = 16;
constexpr int FUSE_BLOCKS = 1024;
int multidot_blocks(int m, int64_t len, int cap);
int norm_blocks(int64_t len, int cap);
// K-cycle step coefficients from the dots (stage 1: m = 2, stage 2: m = 3).
int launch_kcycle_coef(int stage, const double* dots, const double* part, int nb, double* coef, double* state,
                       int nrhs, hipStream_t st);
template <typename TX, typename TY>
int launch_scale_copy(const double* a, const void* x, int64_t xstride, void* y, int64_t ystride, int64_t len,
                      int nrhs, hipStream_t st);
int launch_zero(void* p, int64_t bytes, hipStream_t st);
int launch_dense_assemble_prep(int64_t N, void* E, hipStream_t st);
int launch_dense_fix(int64_t N, const int* isb, void* A, hipStream_t st);
int launch_dense_invert(int64_t N, void* A, void* B, void* col, int* piv, hipStream_t st);
template <typename T>
int launch_dense_mv(int64_t N, const void* Q, int transposed, int cj, const void* b, void* x, int nrhs,
                    hipStream_t st);
// receivers: d = P_r u (- dobs), phi = 1/2 |d|^2 per rhs and their total (optional); v[idx] = scale r
int launch_rec_sample(int64_t vs, int nrec, const int64_t* idx, const void* u, const void* dobs, void* d, double* phi,
                      int nrhs, hipStream_t st);
int launch_rec_inject(int64_t vs, int nrec, const int64_t* idx, const void* r, double scale, void* v, int nrhs,
                      hipStream_t st);
int launch_gradient(const LevelArgs<double>& L, int dim, int nrhs, const void* u, const void* v, double* gl,
                    double* gm, double* gr, hipStream_t st);
// Hybrid Kaczmarz on the Schur complement of the pressure at the coarsest
// level (rows of S in a fixed per-field slot pattern, built on the host).
constexpr size_t KACZ_MAX_LDS = 65536;  // private copy of one sub-region
template <typename T> struct KaczArgs {
  int dim;
  int n[3];
  int64_t fs, vs;    // cells per field, entries per vector
  int ns;            // slots per row
  int box;           // sub-region edge in cells
  int nb[3];         // sub-regions per axis (1 beyond dim)
  int E[3];          // private-copy extent per axis: box + 4 (1 beyond dim)
  int ls;            // private-copy entries: dim * E[0]*E[1]*E[2]
  int nreg;          // sub-regions
  const cx<T>* val;  // [dim*fs][ns] row entries (zero where the column is not an unknown)
  const T* inv;      // [dim*fs] 1/||row||^2, 0 for rows that are not unknowns
  const int* tab;    // [dim][ns][4] column field and x_1, x_2, x_3 offsets of each slot
  const int* dl;     // [dim][ns] the slot's offset inside the private copy
  const int* gptr;   // [dim*fs + 1] gather list of each unknown: entries gptr[j]..gptr[j+1]-1
  const int* gent;   // [entries][2] (sub-region, private-copy index)
  T omega;           // relaxation
};
template <typename T>
int launch_kacz_sweep(const KaczArgs<T>& K, const void* b, const void* xin, void* scr, int nrhs, hipStream_t st);
template <typename T>
int launch_kacz_avg(const KaczArgs<T>& K, const void* scr, void* x, int nrhs, hipStream_t st);
template <typename T>
int launch_kacz_spmv(const KaczArgs<T>& K, const void* x, const void* b, void* y, int nrhs, hipStream_t st);
template <typename T>
int launch_kacz_elem(int mode, int dim, int64_t fs, int64_t vs, int nrhs, const void* app, int cj, const void* b,
                     const void* y, void* out, hipStream_t st);
int launch_gm_start(int nrhs, const double* nrm2, const double* part, int nb, double* st, double* scale,
                    hipStream_t s);
int launch_gm_hcol(int nrhs, int j, const double* dots, const double* part, int nb, double* st, double* coef,
                   hipStream_t s);
// bk > 0: also the back substitution over bk columns into coef (the last step)
int launch_gm_rotate(int nrhs, int j, const double* nrm2, const double* part, int nb, double* st, double* scale,
                     hipStream_t s, int bk = 0, double* coef = nullptr);
// the start (rotation < 0) or rotation j fused with the scaled copy y = x / ||x||
// that follows it (small-reduction path only: part set, nrhs * 2 <= FUSE_VALS)
template <typename T>
int launch_gm_step_copy(int nrhs, int rotation, const double* part, int nb, double* st, double* scale, const void* x,
                        void* y, int64_t len, hipStream_t s);
// Outer flexible GMRES bookkeeping on the device (per-rhs record of
// GO_STRIDE doubles; stat: 4 doubles per rhs: live, jend, residual
// estimate, non-finite flag).  par: 4 doubles per rhs: active, ||b||, rtol.
constexpr int GO_STRIDE = GM_STRIDE + MAXDOT + 8;
int launch_go_start(int nrhs, const double* nrm2, const double* part, int nb, const double* par, double* st,
                    double* stat, hipStream_t s);
int launch_go_hcol(int nrhs, int j, const double* dots, const double* part, int nb, double* st, double* coef,
                   hipStream_t s);
int launch_go_rotate(int nrhs, int j, const double* nrm2, const double* part, int nb, double* st, double* stat,
                     hipStream_t s);
int launch_go_update(int nrhs, int k, const double* st, double* coef, hipStream_t s);

}  // namespace elh
