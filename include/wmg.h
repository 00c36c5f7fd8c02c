/*
 * wmg.h -- C ABI of the MI355X (gfx950) adaptive-multigrid solver for the
 * Wilson-Dirac operator, after Babich, Brannick, Brower, Clark, Cohen,
 * Osborn, Rebbi, "The role of multigrid algorithms for LQCD"
 * (arXiv:0912.2186).
 *
 * Problem (Sec. 2, Eq. 2.1):  D(U) psi = b  on an L0 x L1 x L2 x L3 lattice,
 * D the Wilson operator of Eq. 2.2 (read in its gauge-covariant form):
 *   (D psi)(x) = (4+m) psi(x) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x) psi(x+mu)
 *                                         + (1+gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * with periodic boundaries and the chiral gamma basis
 *   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = 1,2,3),
 *   gamma_4 = [[0, 1], [1, 0]],  gamma_5 = diag(1, 1, -1, -1).
 *
 * Canonical layouts (all fields complex128, interleaved re/im):
 *   site      s = x + L0*(y + L1*(z + L2*t))
 *   U         [V][4][3][3]   U[s][mu][a][b]: link s -> s+mu, row a, column b
 *   spinor    [nrhs][V][12]  component spin*3 + colour
 *   coarse    [nrhs][Vc][n]  n = 2*Nv, dof ordered (chirality, vector); with
 *                            WMG_SPIN_SPLIT n = 4*Nv on the first coarse level,
 *                            ordered (spin, vector)
 *   links     [Vc][9][n][n]  block d = 0 local, 1+mu forward, 5+mu backward
 *   vectors   [Nv][V][dof]   null vectors / prolongator columns (dof = 12 on
 *                            the fine lattice, n of the finer level otherwise)
 *
 * Every field pointer is a DEVICE pointer (hipMalloc'd memory, e.g. a torch
 * CUDA tensor's data_ptr()).  The caller owns U, b, x and every array it
 * passes; the library copies what it keeps, so U may be freed after
 * mg_setup returns.  A context owns all its internal buffers until
 * mg_destroy.  A context is not thread safe; its work runs on its own
 * non-blocking HIP stream (no implicit ordering with the default stream) and
 * every call returns only after that work has finished.  Device inputs must
 * be complete when a call starts (e.g. the device synchronised after the
 * kernels that wrote them).
 *
 * Return codes: 0 success, WMG_ENOTCONV (1) = not converged (x holds the
 * last iterate, stats filled), negative = error, message via wmg_strerror().
 */
#ifndef WMG_H
#define WMG_H

#ifdef __cplusplus
extern "C" {
#endif

#define WMG_OK 0
#define WMG_ENOTCONV 1
#define WMG_EINVAL (-1)      /* bad argument: null pointer, size, divisibility */
#define WMG_ENOMEM (-2)      /* device allocation failed */
#define WMG_EHIP (-3)        /* HIP runtime error */
#define WMG_ERANK (-4)       /* block Gram-Schmidt breakdown (dependent null vectors) */
#define WMG_EBREAKDOWN (-5)  /* NaN/Inf or Krylov breakdown */

#define WMG_FP64 0   /* every step in double precision */
#define WMG_MIXED 1  /* FP64 outer GCR + reliable updates, FP32 cycle on FP16-stored links/null vectors */

#define WMG_VCYCLE 0
#define WMG_WCYCLE 1

#define WMG_X0_GIVEN 1 /* flags: x holds the initial guess on entry to mg_solve */
#define WMG_COARSE_FP32 2 /* flags: mixed precision keeps FP32 coarse links in the cycle
                             (default: FP16 with one FP32 scale per site and direction) */
#define WMG_EO_SMOOTHER 8 /* flags: the fine-level post-smoother runs its MR steps on the
                             red/black (even-odd) Schur complement S = D_ee - D_eo D_oo^-1 D_oe
                             and solves the odd sites exactly (Sec. 3, MG combined with
                             red/black preconditioning); every extent must be even */
#define WMG_GRAPHS 16     /* flags: the coarsest CGNR runs its iterations as captured HIP
                             graphs of 4 iterations (same launches, same results; captured
                             at the second solve of a buffer set, not while profiling;
                             ignored by mg_setup_batch, whose instances run on concurrent
                             host threads) */
#define WMG_COARSE_B32 64 /* flags: the mixed cycle's matrix-core coarse stencil (FP16 links)
                             and fine-level restriction and prolongation multiply FP32
                             vectors (default: the vectors rounded to FP16 with one
                             power-of-two scale per rhs, FP16 products, FP32 accumulation;
                             stencil for 32, 48 or 64 coarse dof, prolongation for Nv a
                             multiple of 8, <= 64 rhs) */
#define WMG_Z32 128        /* flags: the mixed solve stores the cycle's output z in FP32 (default
                             with WMG_EO_SMOOTHER, FP16 prolongation and <= 64 rhs: FP16, the
                             flexible GCR taking any preconditioner output; A z and the
                             solution update read the same FP16 values) */
#define WMG_SPIN_SPLIT 32 /* flags: the fine level's blocking splits each null vector into its
                             four Dirac spins instead of its two chiralities (Sec. 3, exposing
                             the full spin structure on the coarse blocks): 4 Nv coarse dof per
                             block, ordered (spin, vector); coarser levels split by chirality */
#define WMG_LINKS18 4     /* flags: the fine operator reads whole 3x3 links (18 reals); by
                             default it reads the first two rows (12 reals, Table 2) and
                             rebuilds the third as conj(row0 x row1) when every link of U
                             satisfies that identity to 1e-12 (U in SU(3)) */

typedef struct wmg_ctx wmg_ctx;

typedef struct {
  int L[4]; /* lattice extents, x fastest */
} wmg_geom;

/* Solver parameters.  Defaults (wmg_default_params) follow Sec. 3 of the
 * paper: 4^4 aggregates, chirality split, 4 post-smoothing steps, GCR(8)
 * outer solver, CG on the normal equations at the coarsest level, W-cycle
 * when three levels are used. */
typedef struct {
  int levels;             /* 2 or 3 */
  int block[2][4];        /* aggregate of level l -> l+1 (block[0] is overridden by mg_setup's block) */
  int nvec[2];            /* null vectors of level l (nvec[0] is overridden by mg_setup's Nv) */
  int setup_iters;        /* GCR iterations per null vector in the adaptive setup */
  int post_smooth;        /* MR post-smoothing steps per level */
  int gcr_restart;        /* outer GCR restart length (<= 16) */
  int cycle;              /* WMG_VCYCLE or WMG_WCYCLE */
  int precision;          /* WMG_FP64 or WMG_MIXED */
  int nrhs_max;           /* largest nrhs accepted by mg_solve */
  double coarse_tol;      /* coarsest CGNR: relative residual */
  int coarse_maxiter;     /* coarsest CGNR: iteration cap */
  double reliable_delta;  /* mixed: restart in FP64 when |r_inner| < delta * |r_last_update| (default 1e-3) */
  int maxiter;            /* outer GCR iteration cap */
  unsigned long long seed;/* Philox key of the setup's random start vectors */
  int flags;              /* WMG_* flags above */
} wmg_params;

typedef struct {
  int outer_iters;        /* outer GCR iterations (max over right-hand sides) */
  int fine_matvecs;       /* fine-operator applications (any precision, per rhs block) */
  int fine_matvecs_fp64;  /* of which FP64 (true residuals / reliable updates) */
  int coarse_iters;       /* CGNR iterations summed over all coarse solves */
  int reliable_updates;   /* FP64 residual recomputations */
  int converged;          /* 1 if every rhs reached tol */
  double true_relres;     /* max over rhs of |b - D x| / |b| in FP64 */
  double setup_s;         /* wall time of mg_setup */
  double solve_s;         /* wall time of this solve */
} wmg_stats;

/* Fill p with the defaults above.  Returns 0. */
int wmg_default_params(wmg_params *p);

/* Eq. 2.2: out = D(U) in, FP64, canonical layouts, one right-hand side.
 * U: [V][4][3][3], in/out: [V][12] device pointers; in and out must not
 * alias.  Runs on hip_stream (NULL = default stream) and returns without
 * synchronising.  EINVAL on a null pointer or a non-positive extent. */
int wilson_apply(const wmg_geom *g, const double *U, double m, const double *in, double *out, void *hip_stream);

/* Adaptive setup (Sec. 2, Eqs. 2.6-2.7; Sec. 3): builds Nv near-null
 * vectors by the sequential adaptive procedure, the chirality-split block
 * orthonormal prolongator P (sigma_3 P = P gamma_5) and the Galerkin coarse
 * operator P^dag D P, recursively for `levels` levels, at mass m.
 * block[4] must divide the lattice; 1 <= Nv <= 6*|block|.  p may be NULL
 * (defaults).  On success *out receives a new context.  With the environment
 * variable WMG_VERBOSE set (not "0") the setup prints one line per finished
 * null vector to stderr. */
int mg_setup(const wmg_geom *g, const double *U, double m, int Nv, const int block[4], const wmg_params *p,
             wmg_ctx **out);

/* MG-preconditioned flexible GCR solve of D x = b (Sec. 3) for nrhs
 * right-hand sides b[nrhs][V][12] -> x[nrhs][V][12], each to
 * |b - D x| / |b| <= tol in FP64.  x is output only unless
 * params.flags & WMG_X0_GIVEN.  st may be NULL. */
int mg_solve(wmg_ctx *ctx, const double *b, double *x, double tol, int nrhs, wmg_stats *st);

/* ---- setup reuse (Sec. 4: amortise the setup as U evolves) ---------- */
/* Write the context's setup -- lattice, parameters, mass and the null
 * vectors of every level (canonical [Nv][V][dof], complex128) -- to the
 * file `path`, followed by a checksum.  EINVAL if the file cannot be
 * written; a batch context is rejected. */
int mg_save(wmg_ctx *ctx, const char *path);
/* New context from a saved setup for links U at mass m: P and the Galerkin
 * operators are rebuilt from the saved vectors for these links (no adaptive
 * iterations).  The lattice must be the file's; p (NULL = the saved
 * parameters) may change solver settings (precision, tolerances, nrhs_max,
 * flags) but not the hierarchy (levels, Nv, coarser aggregates).  EINVAL
 * for a missing, truncated, foreign or corrupted file (checked before any
 * device work) or a mismatch. */
int mg_load(const char *path, const wmg_geom *g, const double *U, double m, const wmg_params *p, wmg_ctx **out);
/* Adapt a context to new links U (e.g. the next configuration of a Monte
 * Carlo chain): rebuild the hierarchy from the old null vectors for U, relax
 * each vector by `iters` steps of GCR on D(U) x = 0 preconditioned with that
 * hierarchy (starting from the vector itself), normalise, and rebuild;
 * level by level for three levels.  iters = 0 only rebuilds.  The cost is
 * two Galerkin builds per level against one per vector in mg_setup. */
int mg_refresh(wmg_ctx *ctx, const double *U, int iters);

/* Change the quark mass without a new setup: D_hat(m) = D_hat(m0) + (m-m0) 1
 * exactly, since P^dag P = 1 and D(m) = D(0) + m. */
int mg_set_mass(wmg_ctx *ctx, double m);

/* Switch the solve precision (WMG_FP64 / WMG_MIXED) of a context without
 * a new setup; the hierarchy is always built in FP64. */
int mg_set_precision(wmg_ctx *ctx, int precision);

/* Reals per link the fine operator of the context reads: 12 (two rows,
 * third rebuilt; SU(3) field) or 18 (whole links). */
int mg_link_reals(wmg_ctx *ctx);

/* Release the context and all its device memory. */
int mg_destroy(wmg_ctx *ctx);

/* Message of the last error (thread-local), or a description of `code`. */
const char *wmg_strerror(int code);

/* Unpreconditioned BiCGStab on D x = b from x = 0 (the unigrid baseline),
 * FP64, one rhs, canonical layouts; st->outer_iters = iterations (two
 * operator applications each). */
int bicgstab_solve(const wmg_geom *g, const double *U, double m, const double *b, double *x, double tol, int maxiter,
                   wmg_stats *st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * BiCGStab solve as bicgstab_solve, with every work buffer (SoA links, eight
 * fine vectors, device scalars, reduction partials) placed in one fixed
 * device array of WMG_NOALLOC_SCRATCH_BYTES inside the library, one copy per
 * GPU, held until the process ends.  Needs about 2112 * (V + 384) + 262656
 * bytes, so lattices up to about 15,400 sites fit (8^4, 8^3 x 16, 12^3 x 8);
 * larger ones return WMG_EINVAL with the sizes in the message.  It calls no
 * hipMalloc, hipFree or host-pinning routine.  Work runs on hip_stream (NULL
 * = the default stream), which the call synchronises at every scalar
 * read-back and before it returns.  All calls on one GPU share that GPU's
 * array: calls that overlap in time on the same GPU (from several host
 * threads, or on several streams) race and give wrong results.  The array
 * keeps the previous call's contents; the call clears what it needs with a
 * fill kernel first. */
#define WMG_NOALLOC_SCRATCH_BYTES (32u << 20)
int bicgstab_solve_noalloc(const wmg_geom *g, const double *U, double m, const double *b, double *x, double tol,
                           int maxiter, wmg_stats *st, void *hip_stream);

/* ---- uneven batch (Sec. 4: one API over several lattices) ------------ */
/* n (1..256) independent instances with their own lattice, links and mass,
 * the same Nv/block/params.  Each instance gets its own context (own HIP
 * stream and buffers); mg_setup_batch and mg_solve_batch drive the
 * instances from one host thread each, so their kernels run concurrently on
 * the device.  mg_solve_batch takes one rhs per instance (b[i], x[i] device
 * pointers of instance i's size) and fills st[i] (st may be NULL); it
 * returns the first negative error of any instance, else WMG_ENOTCONV if
 * any instance did not converge, else 0. */
int mg_setup_batch(int n, const wmg_geom *g, const double *const *U, const double *m, int Nv, const int block[4],
                   const wmg_params *p, wmg_ctx **out);
int mg_solve_batch(wmg_ctx *ctx, const double *const *b, double *const *x, double tol, wmg_stats *st);

/* ---- test hooks (exported for parity tests; not needed by solvers) ---- */
/* level info: lattice extents, per-site dof, null vectors to the next level */
int mg_level_info(wmg_ctx *ctx, int level, int L[4], int *dof, int *nv);
/* Replace level `level`'s null vectors (canonical [Nv][V][dof]) and rebuild
 * P and every coarser operator from them (no adaptive iteration). */
int mg_set_null_vectors(wmg_ctx *ctx, int level, const double *vecs);
/* Copy out the null vectors (before orthonormalisation) / the block
 * orthonormal prolongator, canonical [Nv][V][dof]. */
int mg_get_null_vectors(wmg_ctx *ctx, int level, double *vecs);
int mg_get_prolongator(wmg_ctx *ctx, int level, double *P);
/* Coarse links of level `level` (>= 1), canonical [Vc][9][n][n]. */
int mg_get_coarse_links(wmg_ctx *ctx, int level, double *links);
/* FP64 restriction / prolongation between level and level+1. */
int mg_restrict(wmg_ctx *ctx, int level, const double *fine, double *coarse, int nrhs);
int mg_prolong(wmg_ctx *ctx, int level, const double *coarse, double *fine, int nrhs);
/* FP64 coarse operator (or its adjoint) at level >= 1. */
int mg_coarse_apply(wmg_ctx *ctx, int level, const double *in, double *out, int dagger, int nrhs);
/* Restriction / prolongation through the FP32 vectors and the FP16-stored
 * prolongator of a mixed-precision context, as the mixed cycle runs them
 * (on the fine level with FP16 products unless WMG_COARSE_B32); canonical
 * FP64 in/out. */
int mg_restrict_f32(wmg_ctx *ctx, int level, const double *fine, double *coarse, int nrhs);
int mg_prolong_f32(wmg_ctx *ctx, int level, const double *coarse, double *fine, int nrhs);
/* The same through the FP32 coarse operator of a mixed-precision context
 * (matrix-core kernel for n <= 64); canonical FP64 in/out. */
int mg_coarse_apply_f32(wmg_ctx *ctx, int level, const double *in, double *out, int dagger, int nrhs);
/* Fine operator through the internal kernels: prec 0 FP64, 1 FP32 links and
 * spinors, 2 FP16 links with FP32 spinors, 3 the smoother's MR-step form
 * (in/|in| per rhs stored in FP16 by the smoother's residual kernel, FP16
 * links on FP16 spinors, FP16 output, returned times |in|), 4 the inner
 * GCR's operator on the FP16-stored preconditioner output (in rounded to
 * FP16, FP32 links and arithmetic, FP32 output); canonical FP64 in/out,
 * nrhs <= 64. */
int mg_apply_fine(wmg_ctx *ctx, int prec, const double *in, double *out, int nrhs);
/* The mixed cycle's smoother residual kernel: out = r/|r| - D e per rhs,
 * r rounded to FP32 and e to FP32 (or, in a mixed context with
 * WMG_EO_SMOOTHER whose prolongation writes FP16, to FP16, the output in
 * the two half-lattice arrays as the red/black smoother reads it), FP16
 * links, the result stored in FP16 and returned as FP64 (canonical layouts,
 * nrhs <= 64). */
int mg_smoother_residual(wmg_ctx *ctx, const double *r, const double *e, double *out, int nrhs);
/* One red/black hopping kernel of the smoother's Schur complement (Sec. 3,
 * red/black preconditioning): out = a diag + b H_par(hop) on the sites of
 * parity par = (x+y+z+t) mod 2, where H_par(v) is the hopping sum of Eq. 2.2
 * at those sites from v on the other parity (D_{par,1-par} = -H_par / 2).
 * diag (read at parity par; NULL allowed when a == 0), hop (read at the other
 * parity) and out (zero at the other parity) are canonical FP64 full-lattice
 * vectors.  prec 0: FP64 links and vectors; 3: FP16 links and FP16 vectors
 * (the MR steps: projection and SU(3) products in packed FP16 arithmetic,
 * the eight directions summed in FP32); 4: FP16 links and diag, FP32 hop
 * input and output (the odd correction); 5: FP16 links, diag and hop input
 * with FP32 output, the smoother's fused last step (par must be 1), which
 * also returns hop's values at the even sites; 6: as 5 with the output
 * stored in FP16.  Needs every extent even; nrhs <= 64. */
int mg_hop_eo(wmg_ctx *ctx, int prec, int par, double a, double b, const double *diag, const double *hop,
              double *out, int nrhs);
/* One application of the FP64 preconditioner z = M r (one MG cycle). */
int mg_cycle(wmg_ctx *ctx, const double *r, double *z);
/* Per-rhs outer iteration counts of the last solve (array of nrhs ints,
 * host memory). */
int mg_last_iters(wmg_ctx *ctx, int *iters, int nrhs);
/* Time (ms) of `reps` back-to-back fine-operator applications on internal
 * layouts, measured with HIP events on the context stream (Dslash
 * bandwidth measurement).  prec as in mg_apply_fine. */
int mg_time_dslash(wmg_ctx *ctx, int prec, int nrhs, int reps, double *ms);

/* Test hook of the launch-shape autotuner (process-wide): choice >= 0 makes
 * every tuned launch run candidate `choice` (candidate 0, the default, where
 * a launch has fewer) with no search and nothing recorded; choice < 0
 * restores normal tuning.  Returns the previous setting (-1 when off). */
int wmg_tune_force(int choice);

/* ---- measurement hooks --------------------------------------------- */
/* Kernel classes timed by mg_profile. */
#define WMG_K_DSLASH_CYCLE 0   /* fine operator of the cycle's MR steps (FP16 links, FP32 spinors) */
#define WMG_K_DSLASH_OUTER32 1 /* fine operator of the inner GCR (FP32) */
#define WMG_K_DSLASH_64 2      /* fine operator in FP64 */
#define WMG_K_COARSE32 3       /* coarse stencil, FP32 */
#define WMG_K_COARSE64 4       /* coarse stencil, FP64 */
#define WMG_K_RESTRICT 5       /* fine -> first coarse level */
#define WMG_K_PROLONG 6        /* first coarse level -> fine */
#define WMG_K_DSLASH_RES 7     /* smoother residual r - A e in the cycle (FP16 links, FP32 spinors) */
/* enable != 0: from now on record a HIP event pair on the context stream
 * around every launch of the classes above; resets the accumulators. */
int mg_profile(wmg_ctx *ctx, int enable);
/* Launch count, summed event time (ms) and summed algorithmic bytes of one
 * class since the last mg_profile call. */
int mg_profile_get(wmg_ctx *ctx, int kind, int *launches, double *total_ms, double *total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* WMG_H */
