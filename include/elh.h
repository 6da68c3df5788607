/*
 * elh.h -- C ABI of the MI355X library for the matrix-free elastic
 * Helmholtz multigrid solver of Yovel & Treister, "LFA-tuned matrix-free
 * multigrid method for the elastic Helmholtz equation".
 *
 * Problem (Section 2.2, eq. linsys; Section 3.1, eq. mixed-discretized):
 * solve  H^beta u = q  where H^beta is the beta-spread MAC discretisation
 * of the mixed displacement/pressure elastic Helmholtz system (eq.
 * elasticMixed) with heterogeneous lam, mu, rho and attenuation gamma.
 * The preconditioner is a multigrid cycle (Algorithm 1, applied
 * recursively) on the shifted operator H^beta_s (gamma -> gamma + alpha,
 * Section 2.2, eq. shift), used on the right of restarted flexible GMRES
 * (Section 5: FGMRES(5), zero initial guess, relative-residual stop).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Pointers: unless stated otherwise every array pointer is a DEVICE
 *   pointer on the GPU the handle was created on; host pointers are marked
 *   "(host)".  The caller owns all buffers it passes; the handle owns its
 *   media copies, hierarchy and workspaces.
 * Grid: n[0..2] = cells along x_1, x_2, x_3 (n[2] = 1 in 2D); spacing h.
 * Media (lam, mu, rho): real float64 arrays of n[dim-1]*...*n[0] cells,
 *   C order with x_1 fastest (numpy shape (n_d, ..., n_1)).
 * Vectors: complex, interleaved (re, im), float64 (ELH_C128) or float32
 *   (ELH_C64).  One vector = d+1 fields u_1..u_d, p, each of n cells in the
 *   media order; a batch of nrhs vectors is contiguous:
 *   (nrhs, d+1, n_d, ..., n_1).  Field u_k lives on the faces normal to
 *   x_k (MAC grid, Section 2.3, Figure 1a): its entry with index i along
 *   x_k is the face between cells i-1 and i, so index 0 is the domain
 *   boundary face.  Boundary faces are not unknowns: they are ignored on
 *   input and written as 0 on output.
 * Levels: level 0 is the finest; level l has n/2^l cells and spacing
 *   2^l h; coarse media are the means of the 2^d child cells.
 * Streams: all work is enqueued on the stream given to elh_create; calls
 *   returning vectors are asynchronous except elh_solve* (which wait for
 *   their statistics).  Calls on one handle must not overlap.
 * Errors: 0 = success; ELH_NOT_CONVERGED (> 0) still writes the best
 *   iterate and statistics; negative codes leave outputs unspecified.
 *   elh_last_error() returns a thread-local message for the last failure.
 */
#ifndef ELH_H
#define ELH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ELH_OK = 0,
  ELH_NOT_CONVERGED = 1,
  ELH_ERR_ARG = -1,      /* invalid argument (sizes, pointers, parameters)  */
  ELH_ERR_HIP = -2,      /* a HIP runtime call failed                        */
  ELH_ERR_NUMERIC = -3,  /* NaN/Inf in a norm, or a Krylov breakdown         */
  ELH_ERR_OOM = -4,      /* device allocation failed                         */
  ELH_ERR_STATE = -5     /* handle not usable (e.g. setup failed)            */
} elh_status;

typedef enum { ELH_C64 = 1, ELH_C128 = 2 } elh_dtype;

/* elh_apply / elh_residual / elh_relax / elh_vcycle flags */
enum { ELH_SHIFTED = 1,  /* use H^beta_s (alpha added to gamma), eq. shift */
       ELH_ADJOINT = 2   /* use the conjugate transpose                     */ };

/* coarsest-level solver (Section 3.2, "Coarsest grid solution") */
enum { ELH_COARSE_KRYLOV = 0,  /* restarted GMRES preconditioned by red-black
                                  Vanka sweeps, fixed budget / residual drop */
       ELH_COARSE_DENSE = 1,   /* exact solve (dense inverse built at setup;
                                  the paper's LU choice for 2D)             */
       ELH_COARSE_RELAX = 2,   /* fixed number of red-black Vanka sweeps    */
       ELH_COARSE_KACZMARZ = 3 /* the paper's 3D choice: p eliminated through
                                  its diagonal block, FGMRES on the Schur
                                  complement preconditioned by hybrid
                                  Kaczmarz sweeps (see elh_kaczmarz)        */ };

typedef struct {
  int dim;              /* 2 or 3                                              */
  int n[3];             /* cells along x_1, x_2, x_3; each divisible by
                           2^(levels-1)                                       */
  double h;             /* grid spacing of level 0                            */
  double omega;         /* angular frequency (eq. elasticHelm)                */
  double gamma;         /* physical attenuation (eq. elasticHelm), >= 0       */
  double alpha;         /* preconditioner shift added to gamma (eq. shift),
                           >= 0; gamma + alpha > 0 keeps the shifted operator
                           nonsingular (elh_create: ELH_ERR_ARG otherwise)    */
  double beta;          /* spread weight of the compact stencils, (0,1];
                           2/3 is the LFA-tuned value (Section 4.3)           */
  double abl_width;     /* absorbing-layer width, PHYSICAL units (0 = none)   */
  double abl_amp;       /* absorbing-layer peak attenuation: the layer adds
                           abl_amp * sum_k (delta_k/abl_width)^2 to gamma,
                           delta_k = distance into the layer along x_k        */
  int levels;           /* multigrid levels, 1..8 (1 = coarsest solve only)   */
  int nu1, nu2;         /* pre/post red-black Vanka sweeps (Section 3.2)      */
  int cycle_calls;      /* recursive calls per level: 1 = V-cycle, 2 = W-cycle,
                           3 = K-cycle: the two calls precondition two steps
                           of flexible GCR on the coarse system (Section 2.2,
                           below Algorithm 1)                                 */
  double damping[8];    /* Vanka damping w per level (Section 5.2)            */
  int coarse_mode;      /* ELH_COARSE_*                                       */
  int coarse_sweeps;    /* Vanka sweeps per coarse relaxation/preconditioning;
                           KACZMARZ: hybrid Kaczmarz sweeps per
                           preconditioning (paper: 10)                        */
  int coarse_restart;   /* inner GMRES restart length (KRYLOV, KACZMARZ;
                           paper: 5)                                          */
  int coarse_maxit;     /* inner GMRES iterations budget (KRYLOV, KACZMARZ;
                           paper: 25, i.e. at most 250 Kaczmarz sweeps)      */
  double coarse_rtol;   /* inner residual-drop stop, 0 = always full budget
                           (paper, KACZMARZ: 0.1)                             */
  double coarse_damping;/* Vanka damping on the coarsest level (<=0: use
                           damping[levels-1]); KACZMARZ: the relaxation of
                           the row projections (<=0: 0.8, the paper's)        */
  int precond_dtype;    /* ELH_C128: float64 cycle; ELH_C64: float32 cycle
                           inside the float64 Krylov solve (Section 5.3)      */
  int kacz_box;         /* KACZMARZ: sub-regions are boxes of kacz_box^dim
                           cells (<= 0: 4); the private copy of a sub-region,
                           dim*(kacz_box+4)^dim complex float64, must fit in
                           64 KiB of LDS (3D: kacz_box <= 7)                  */
} elh_desc;

typedef struct {
  int restart;          /* FGMRES restart length m (paper: 5)                 */
  int maxit;            /* maximum preconditioner applications                */
  double rtol;          /* stop at ||q - H u|| <= rtol ||q|| (per RHS)        */
  int zero_x0;          /* 1: start from u = 0 (the paper's choice, Section
                           5); 0: u holds the initial guess on entry, e.g.
                           the iterate an earlier call returned with
                           ELH_NOT_CONVERGED (resume).  The stop stays
                           relative to ||q||, and a resumed solve continues
                           the iterates of the interrupted one exactly when
                           it was cut at a restart boundary (maxit a
                           multiple of restart)                               */
  int store_z_fp32;     /* with precond_dtype ELH_C64: 1 keeps the
                           preconditioned vectors z_j in complex64 (exact,
                           since the cycle produces them in float32; half
                           the memory and traffic), 0 widens them to
                           complex128; must be 0 with ELH_C128            */
} elh_solve_opts;

typedef struct {        /* (host) one record per right-hand side              */
  int iters;            /* preconditioner applications (Section 5 counts)     */
  int restarts;
  int status;           /* ELH_OK / ELH_NOT_CONVERGED / ELH_ERR_NUMERIC       */
  double relres;        /* final true relative residual, float64              */
  double* history;      /* in: NULL, or a host array of history_cap doubles   */
  int history_cap;      /*   that receives the FGMRES estimate of the         */
  int history_len;      /*   relative residual after each iteration; out:     */
                        /*   entries written (min(iters, history_cap))        */
  double t_total_ms;    /* out: wall time of the call (same for every rhs)    */
  double t_precond_ms;  /* out: GPU time in the preconditioner cycles         */
  double t_apply_ms;    /* out: GPU time in the outer operator A z            */
  double t_orth_ms;     /* out: Gram-Schmidt passes, reductions and their     */
                        /*   host round trips                                 */
  unsigned long long kernels; /* out: kernels the call had executed (eager
                           launches and kernel nodes of replayed graphs; for
                           elh_solve_batch / elh_batch_solve, all problems)   */
} elh_solve_stats;

typedef struct elh_handle elh_handle;

/* Create a handle: copies the media (device float64 arrays), builds the
 * coarse hierarchy (media means, kappa = 1/(lam+mu), float32 copies) and,
 * for ELH_COARSE_DENSE, the coarsest-level inverse.  stream: hipStream_t
 * (NULL = default stream).  Section 3.1 (operator), Section 3.2 (hierarchy
 * by re-discretisation).
 * Environment, read here: ELH_GRAPHS=0 runs the cycles and Gram-Schmidt
 * steps eagerly instead of as replayed hipGraphs; ELH_ZCHUNK=c sets the
 * marching kernels' default x_3 chunk (c > 0, shortened on small grids) or
 * forces exactly -c planes (c < 0); ELH_TUNE / ELH_TUNE_CACHE: see
 * elh_stencil_choice.  None of them changes results. */
int elh_create(const elh_desc* desc, const double* lam, const double* mu,
               const double* rho, void* stream, elh_handle** out);

/* Replace the media of an existing handle (same sizes); rebuilds the
 * hierarchy in place without reallocating. */
int elh_set_media(elh_handle* h, const double* lam, const double* mu,
                  const double* rho);

int elh_destroy(elh_handle* h);

/* y = H x on `level` (eq. mixed-discretized; ELH_SHIFTED: H_s; ELH_ADJOINT:
 * H^H).  x and y: nrhs vectors of that level, dtype `dtype`; x != y. */
int elh_apply(elh_handle* h, int level, int flags, int dtype, int nrhs,
              const void* x, void* y);

/* y = H x on level 0 with x in complex64 and float64 arithmetic and output:
 * the outer operator of the mixed-precision solve (Section 5.3), applied to
 * the float32 preconditioned vectors.  x: (nrhs, dim+1, n_d..n_1) complex64,
 * y: same shape complex128, distinct buffers.  flags: ELH_ADJOINT (H^H);
 * ELH_SHIFTED is rejected (ELH_ERR_ARG).  Errors as elh_apply. */
int elh_apply_f32in(elh_handle* h, int flags, int nrhs, const void* x, void* y);

/* r = b - H x  (same operator selection as elh_apply); r may alias b. */
int elh_residual(elh_handle* h, int level, int flags, int dtype, int nrhs,
                 const void* b, const void* x, void* r);

/* rc = R (b - H_s x): residual of the shifted operator on `level` followed
 * by the MAC restriction of Section 2.3 (eqs. pIntergrid, u2Intergrid and
 * their 3D tensor-product form) to level+1.  x == NULL means x = 0.
 * flags: ELH_ADJOINT selects H_s^H. */
int elh_restrict_residual(elh_handle* h, int level, int flags, int dtype,
                          int nrhs, const void* b, const void* x, void* rc);

/* x += P e: MAC prolongation (Section 2.3) from level+1 to `level`. */
int elh_prolong_add(elh_handle* h, int level, int dtype, int nrhs,
                    const void* e, void* x);

/* One colour of red-black full-Vanka relaxation of H_s x = b on `level`
 * (Section 2.3 Vanka smoother, Section 3.2 red-black order): with the
 * residual r = b - H_s x, every cell of colour `colour` ((i_1+..+i_d) mod
 * 2) solves its (2d+1)x(2d+1) block (its unknown faces and its pressure)
 * and adds w * correction; w = damping[level] (coarse_damping on the
 * coarsest level).  x is updated in place.  flags: ELH_ADJOINT. */
int elh_relax(elh_handle* h, int level, int flags, int dtype, int nrhs,
              int colour, const void* b, void* x);

/* Allocation-free form of elh_relax, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same operation, arguments, results and
 * errors as elh_relax, bitwise.  The residual work lives in one static
 * device array per GPU of ELH_NOALLOC_SCRATCH_BYTES (64 MiB), which the
 * library holds from its first elh_create on that GPU until the process
 * ends; nrhs * (dim+1) * (cells of the level) * (8 for ELH_C64, 16 for
 * ELH_C128) bytes must fit, else ELH_ERR_ARG before anything is launched
 * (e.g. one complex64 right-hand side on up to 128^3 cells).  Calls no
 * allocator and never runs the stencil autotuner (it uses a chunk the tuner
 * chose earlier, else the default; the results are the same).  Every call on
 * one GPU shares that array: calls that overlap in time on one GPU (other
 * streams, other threads, other handles) race and give wrong results; calls
 * ordered on one stream are safe. */
#define ELH_NOALLOC_SCRATCH_BYTES (64u << 20)
int elh_relax_noalloc(elh_handle* h, int level, int flags, int dtype, int nrhs,
                      int colour, const void* b, void* x);

/* x = coarsest-level solve of H_s x = b (mode desc->coarse_mode) on level
 * levels-1. */
int elh_coarse_solve(elh_handle* h, int flags, int dtype, int nrhs,
                     const void* b, void* x);

/* The preconditioner of the ELH_COARSE_KACZMARZ coarsest solve (Section
 * 3.2, "Coarsest grid solution"; parameters in Section 5.3), on level
 * levels-1, for a handle created with that mode: x = `sweeps` hybrid
 * Kaczmarz sweeps from x = 0 on S x_u = b_u, where
 * S = A_uu - A_up diag(A_pp)^-1 A_pu is the Schur complement of the
 * pressure of A = H_s (ELH_ADJOINT: of H_s^H, i.e. S^H).  One sweep: every
 * sub-region (a box of kacz_box^dim cells; a displacement unknown belongs
 * to the box holding its storage index) starts from the current iterate
 * and projects it, row by row in ascending storage order over its own rows
 * a_i, onto  x <- x + w (b_i - a_i x) / ||a_i||^2 conj(a_i)  (w =
 * coarse_damping, or 0.8); each unknown then takes the mean of the copies of
 * the sub-regions whose rows reach it through the stencil pattern of S.
 * b, x: device vectors in storage layout (nrhs, dim+1, n_d..n_1) of the
 * coarsest level in dtype; the pressure entries of b are ignored, those of
 * x are set to zero.  nrhs <= 64.  Errors: ELH_ERR_ARG (mode, sizes),
 * ELH_ERR_OOM (work buffers), ELH_ERR_HIP (launch). */
int elh_kaczmarz(elh_handle* h, int flags, int dtype, int nrhs, int sweeps,
                 const void* b, void* x);

/* x = V(nu1,nu2)-cycle (cycle_calls = 1), W-cycle (2) or K-cycle (3)
 * approximation of H_s^{-1} b on level 0 from a zero initial guess
 * (Algorithm 1 applied recursively).  In the K-cycle the coarse correction
 * of every level minimises the coarse residual over the span of the two
 * preconditioned directions.  flags: ELH_ADJOINT for the cycle on H_s^H. */
int elh_vcycle(elh_handle* h, int flags, int dtype, int nrhs, const void* b,
               void* x);

/* Solve H u = q for nrhs right-hand sides (float64 q, u on level 0) by
 * FGMRES(opts->restart) right-preconditioned with the cycle in
 * desc->precond_dtype (Section 5: restarted flexible GMRES, relative-
 * residual stop).  The Krylov bookkeeping (Hessenberg columns, Givens
 * rotations, stop test per rhs) runs on the device; an iteration is three
 * submissions (cycle graph, outer operator, Gram-Schmidt graph) and one wait
 * for a small status copy.  At each restart the right-hand sides that have
 * converged are dropped from the batch, so later cycles skip them.  u is overwritten; it is read first as the initial guess
 * when opts->zero_x0 == 0.  stats: (host) array of nrhs records, may be
 * NULL.  Returns ELH_OK when every right-hand side met rtol,
 * ELH_NOT_CONVERGED when one did not within maxit (u then holds the last
 * iterate and the stats its true residual: a later call with zero_x0 = 0
 * resumes from it), ELH_ERR_NUMERIC on a NaN/Inf norm (e.g. non-finite
 * media or right-hand side), ELH_ERR_ARG on invalid options. */
int elh_solve(elh_handle* h, int nrhs, const void* q, void* u,
              const elh_solve_opts* opts, elh_solve_stats* stats);

/* Same for the adjoint system H^H v = r (preconditioned by the cycle on
 * H_s^H). */
int elh_solve_adjoint(elh_handle* h, int nrhs, const void* r, void* v,
                      const elh_solve_opts* opts, elh_solve_stats* stats);

/* Solve several independent problems together: problem i (handle h[i],
 * any grid size) solves nrhs[i] right-hand sides q[i] -> u[i] exactly as
 * elh_solve would (same iterates, bitwise).  The calling thread drives all
 * problems: each unfinished problem has one FGMRES iteration (cycle, outer
 * operator, Gram-Schmidt step) in flight on its handle's stream, and the
 * thread polls the streams, enqueueing a problem's next iteration as soon as
 * its status has arrived, so the kernels of problems created on different
 * streams overlap on the GPU; a problem leaves when its right-hand sides
 * have converged.  stats: (host) sum(nrhs) records in
 * problem order, may be NULL.  Returns the most severe status of all
 * problems (a negative one names its problem in elh_last_error). */
int elh_solve_batch(int nprob, elh_handle* const* h, const int* nrhs,
                    const void* const* q, void* const* u,
                    const elh_solve_opts* opts, elh_solve_stats* stats);

/* Batch of problems of uneven grid sizes (the batching form of the solver;
 * the paper solves one right-hand side of one problem at a time, Section
 * 5).  elh_batch_create builds one problem handle per desc[i] (copying
 * lam[i], mu[i], rho[i], device float64, as elh_create does) on a stream of
 * its own that the library creates, after the work already enqueued on
 * `stream` (the caller's; NULL = default stream).  elh_batch_solve solves
 * problem i's nrhs[i] right-hand sides q[i] -> u[i] as elh_solve_batch
 * does; it waits for the caller's stream first, and later work on the
 * caller's stream is ordered after its outputs.  elh_batch_handle returns
 * problem i's handle (owned by the batch, valid until elh_batch_destroy)
 * for the other entry points; elh_batch_size the number of problems.
 * Errors: ELH_ERR_ARG (arguments; a bad desc names its problem),
 * ELH_ERR_OOM, ELH_ERR_HIP; a failed create leaves nothing allocated. */
typedef struct elh_batch elh_batch;
int elh_batch_create(int nprob, const elh_desc* descs, const double* const* lam,
                     const double* const* mu, const double* const* rho,
                     void* stream, elh_batch** out);
int elh_batch_size(const elh_batch* b);
int elh_batch_handle(elh_batch* b, int i, elh_handle** h);
int elh_batch_solve(elh_batch* b, const int* nrhs, const void* const* q,
                    void* const* u, const elh_solve_opts* opts,
                    elh_solve_stats* stats);
int elh_batch_destroy(elh_batch* b);

/* Parameter gradient of an FWI misfit by the adjoint state:
 *   g_m(c) = - Re sum_s v_s^H (dH/dm_c) u_s,  m in {lam, mu, rho},
 * for forward fields u and adjoint fields v (float64, nrhs each, level 0).
 * g_lam, g_mu, g_rho: float64 arrays of n cells (overwritten). */
int elh_gradient(elh_handle* h, int nrhs, const void* u, const void* v,
                 double* g_lam, double* g_mu, double* g_rho);

/* Receivers of an FWI misfit (the adjoint-state setting that motivates the
 * solver, Section 1).  A receiver samples one unknown of the level-0 vector;
 * idx: (device) int64 storage indices into one vector of (dim+1)*n cells,
 * distinct; an index outside the vector samples zero and is skipped by the
 * injection.
 * elh_receivers: d[s][i] = u[s][idx[i]] - dobs[s][i] (P_r u - d_obs; dobs
 *   may be NULL for plain sampling), u: nrhs complex128 vectors, dobs and d:
 *   (nrhs, nrec) complex128; phi (device, may be NULL): nrhs + 1 doubles,
 *   phi[s] = 1/2 sum_i |d[s][i]|^2 (the misfit of source s, fixed-order
 *   reduction) and phi[nrhs] = sum_s phi[s] (the total misfit).
 * elh_inject: v = scale P_r^T r, i.e. v[s] = 0 except v[s][idx[i]] =
 *   scale r[s][i] (the adjoint source); r: (nrhs, nrec), v: nrhs complex128
 *   vectors (overwritten).
 * Both run on the handle's stream and return without synchronising.  The
 * output must not overlap the inputs (d = u or v = r is rejected).
 * Errors: ELH_ERR_ARG on sizes, NULL pointers, aliased outputs or a
 * non-finite scale. */
int elh_receivers(elh_handle* h, int nrhs, const void* u, int nrec,
                  const int64_t* idx, const void* dobs, void* d, double* phi);
int elh_inject(elh_handle* h, int nrhs, int nrec, const int64_t* idx,
               const void* r, double scale, void* v);

/* Number of levels, cells per axis (x-order) and spacing of `level`. *//* Number of levels, cells per axis (x-order) and spacing of `level`. */
int elh_level_info(elh_handle* h, int level, int* n3, double* hl);

/* Stencil autotuner (batching / set-up row of the hot path).  On its first
 * use outside graph capture, each kind of 3D march (level, precision, input
 * precision, kind: 0 apply, 1 residual, 2 residual restricted to the next
 * level; adjoint or not; nrhs) times its candidate x_3 chunks of the
 * wavefront march (4, 8, 16, 32, 64 planes per workgroup; on columns of at
 * most 64 planes also 1, 2 and the whole column; coarse planes for kind 2)
 * on the call's own buffers with HIP events on the handle's stream and keeps
 * the fastest for the handle's lifetime.  The chunk never changes an
 * output's arithmetic, so tuned and untuned results are bitwise equal.
 * Environment: ELH_TUNE=0 (read at elh_create) keeps the default chunk
 * heuristic; ELH_TUNE_CACHE=path loads earlier choices for the handle's
 * grids at elh_create and appends new ones (one text line each).
 * elh_stencil_choice reports the choice for one kind of call: *choice (host)
 * = the chunk (> 0), or -1 when none has been made.  flags: ELH_ADJOINT
 * selects the adjoint; residual: the kind (0, 1, 2).
 * Returns ELH_ERR_STATE / ELH_ERR_ARG on an invalid handle, level, dtype,
 * kind or NULL choice. */
int elh_stencil_choice(elh_handle* h, int level, int dtype, int flags,
                       int residual, int nrhs, int* choice);

const char* elh_status_string(int status);
const char* elh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ELH_H */
