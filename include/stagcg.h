/*
 * stagcg — staggered-fermion D_slash and conjugate-gradient solves on MI355X
 * (gfx950), C ABI.
 *
 * The library implements the hot path of P. Majumdar, "Lattice Simulations
 * using OpenACC compilers" (LATTICE 2013, arXiv:1311.2719): the staggered
 * matrix-vector routine of Sec. 3, called repeatedly inside the
 * conjugate-gradient solve of the normal operator of Sec. 4.
 *
 * Conventions (fixed here because the paper elides the operator's body):
 *   sites      lexicographic s = x + Lx*(y + Ly*(z + Lz*t)); mu = 0..3 = x,y,z,t;
 *              every extent even and >= 2; parity(x) = (x+y+z+t) mod 2,
 *              0 = even, 1 = odd;
 *   operator   (D chi)(x) = 1/2 sum_mu eta_mu(x) [U_mu(x) chi(x+mu)
 *                                             - U_mu(x-mu)^dagger chi(x-mu)],
 *              eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}); periodic in x,y,z;
 *              a hop across the t boundary carries -1 if the field is
 *              antiperiodic in t.  D is anti-Hermitian and maps even <-> odd;
 *   solve      (m^2 - D^2) x = b (= M^dagger M x = b with M = m + D), which
 *              is block-diagonal in parity: each parity is an independent
 *              system.  The paper's CG runs on one half of the lattice from
 *              x = 0 and reconstructs y = D x on the other half (Sec. 4).
 *
 * Fermion-field layout ("even-odd layout", the paper's p(l,ic) indexing with
 * the lattice split into halves, one colour column after another):
 *   complex128 [parity 2][colour 3][Vh], Vh = V/2, interleaved (re, im);
 *   within a parity the site index is cb = s >> 1 (s lexicographic).
 *   A full-lattice field is the even half followed by the odd half.
 *   stag_pack_fermion / stag_unpack_fermion convert from / to the
 *   lexicographic [V][3] complex128 layout.
 *
 * Gauge-field input layout: complex128 [V][4][3][3], U_mu(x)[a][b] row-major.
 *
 * Memory: the caller supplies one device buffer (the arena) at stag_create;
 * the library sub-allocates all device memory from it and never calls
 * hipMalloc.  The arena size is the HBM budget used for admission.  Small
 * pinned host buffers for status polling are allocated with hipHostMalloc.
 *
 * Streams: calls that take a `stream` argument enqueue work on that HIP
 * stream (NULL = the context's stream) and are asynchronous unless stated.
 *
 * Errors: every function returns int32: 0 = OK, 1 = PENDING, negative =
 * error (STAG_E*).  Nothing aborts or throws across the ABI.  The message of
 * the last error on the calling thread is returned by stag_last_error.
 *
 * Threading: one context per device.  stag_submit / stag_poll / stag_wait
 * are thread-safe; other calls on one context must not run concurrently.
 */
#ifndef STAGCG_H
#define STAGCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define STAG_OK          0
#define STAG_PENDING     1
#define STAG_EINVAL     -1   /* bad argument (odd extent, m <= 0, bad parity, range) */
#define STAG_ENOMEM     -2   /* arena exhausted */
#define STAG_ENOENT     -3   /* unknown gauge id or ticket */
#define STAG_EBUSY      -4   /* gauge field still in use by queued requests */
#define STAG_EAGAIN     -5   /* request queue full */
#define STAG_ENOCONV    -6   /* iteration limit reached; x holds the last iterate */
#define STAG_EBREAKDOWN -7   /* <p,Ap> <= 0 or not finite */
#define STAG_ENONFINITE -8   /* NaN / Inf in the input */
#define STAG_EHIP       -9   /* HIP runtime error */
#define STAG_ECANCELED -10   /* request cancelled (context destroyed) */

/* Smallest reliable-update threshold accepted for STAG_FP16_RU. */
#define STAG_FP16_DELTA_MIN 0.01

/* ---- enumerations ---------------------------------------------------- */
enum { STAG_EVEN = 0, STAG_ODD = 1, STAG_ALL = 2 };
enum {
    STAG_FP64 = 0,     /* plain FP64 CG (the paper's precision) */
    STAG_FP32_RU = 1,  /* FP32 inner CG, FP64 reliable updates */
    STAG_FP16_RU = 2   /* FP16 storage with per-site norm, FP32 arithmetic,
                          FP64 reliable updates */
};

/* Storage precision of a fermion field handed to stag_dslash and
 * stag_convert_fermion (even-odd layout, see above):
 *   STAG_F64  complex128 [parity 2][colour 3][Vh]   (48 bytes per site)
 *   STAG_F32  complex64  [parity 2][colour 3][Vh]   (24 bytes per site)
 *   STAG_F16  [parity 2][Vh] records of 16 bytes: three colours as
 *             (re, im) pairs of IEEE binary16 divided by the site's scale,
 *             then the scale as an IEEE binary32 = the largest |re| or |im|
 *             of the site (0 for a zero site).
 * Links follow the same precision (FP16 links unscaled). */
enum { STAG_F64 = 0, STAG_F32 = 1, STAG_F16 = 2 };

typedef struct stag_ctx stag_ctx;

typedef struct {
    double mass;           /* m > 0 */
    double tol;            /* stop when ||b - A x|| <= tol ||b|| per parity system */
    int32_t maxiter;       /* CG iteration limit (per parity system) */
    int32_t precision;     /* STAG_FP64, STAG_FP32_RU, STAG_FP16_RU */
    int32_t parity;        /* STAG_EVEN, STAG_ODD, STAG_ALL */
    int32_t max_restarts;  /* FP64: restarts from the true residual (>= 0) */
    double delta;          /* reliable-update threshold (mixed precision): update when
                              ||r|| < delta * (largest ||r|| since the last update);
                              <= 0 selects the default: 0.01 for STAG_FP32_RU,
                              0.1 for STAG_FP16_RU.  STAG_FP16_RU rejects (EINVAL)
                              a threshold below STAG_FP16_DELTA_MIN: FP16 vectors
                              carry about three decimal digits, and an iterated
                              residual pushed further below its last FP64 value
                              drifts from the true one */
} stag_cg_params;

typedef struct {
    int32_t status;            /* STAG_OK or a negative STAG_E* code */
    int32_t iters;             /* CG iterations (largest over the parity systems) */
    int32_t reliable_updates;  /* FP64 residual recomputations (incl. the final check) */
    int32_t restarts;          /* FP64 mode: restarts after a failed true-residual check */
    double true_rel_resid;     /* ||b - A x|| / ||b|| in FP64 on the GPU, over the solved parities */
    double seconds;            /* wall time of the solve (cg_solve) or submit->completion (serving) */
    double queue_seconds;      /* serving: submit -> admission into a batch slot */
    int32_t iters_parity[2];   /* CG iterations of the even / odd parity system (-1: not solved) */
} stag_cg_info;

/* ---- context --------------------------------------------------------- */

/*
 * Create a context on HIP device `device`.  `arena_dev` / `arena_bytes`: a
 * device buffer owned by the caller that must outlive the context; every
 * device allocation of the library is carved out of it.  `stream`: default
 * HIP stream for the context (NULL = the null stream).  On success *out
 * receives the context.  Errors: EINVAL (NULL pointers, arena < 1 MiB),
 * EHIP.
 */
int stag_create(int device, void *arena_dev, size_t arena_bytes, void *stream,
                stag_ctx **out);

/* Destroy the context: stops the serving thread (queued requests end with
 * ECANCELED), waits for the device, releases host resources.  The arena is
 * not freed (the caller owns it). */
int stag_destroy(stag_ctx *ctx);

/* Message of the last error raised on the calling thread by any call of the
 * library ("" if none).  The message is kept per thread, so `ctx` only names
 * the context the caller asks about and may be NULL (after a failed
 * stag_create).  The string stays valid until the thread's next call. */
const char *stag_last_error(const stag_ctx *ctx);

/* Bytes of the arena in use / total. */
int stag_arena_usage(const stag_ctx *ctx, size_t *used, size_t *total);

/* ---- gauge fields (Sec. 4: `linkc_acc` and the data region's copyin) -- */

/*
 * Register a gauge field.  dims = (Lx, Ly, Lz, Lt), each even and >= 2.
 * links: complex128 [V][4][3][3] (layout above), on the host
 * (links_on_device = 0; copied, the caller keeps ownership) or on the
 * device (1; read once, the caller keeps ownership).  The library folds the
 * staggered phases, the 1/2 and the t-boundary sign into its own copy,
 * builds the daggered backward links (the paper's `ud`) stored at the site
 * that uses them, reorders everything into a checkerboard
 * structure-of-arrays layout, and keeps FP64, FP32 and FP16 copies plus the
 * iup/idn neighbour tables resident in the arena.  When every link is
 * special unitary (each stored matrix then has row 2 = conj(row 0 x row 1)
 * divided by its folded factor, to within 1e-14 absolute), only two rows
 * are kept and the kernels rebuild the third; otherwise all three rows are
 * kept.  The environment variable STAG_LINK_ROWS=3 keeps three rows always.
 * Errors: EINVAL (bad dims), ENOMEM, ENONFINITE (NaN/Inf in the links).
 * Synchronous.
 */
int stag_set_gauge(stag_ctx *ctx, const int32_t dims[4], const double *links,
                   int32_t links_on_device, int32_t t_antiperiodic,
                   int32_t *gauge_id);

/* Release a gauge field.  EBUSY while serving requests on it are pending. */
int stag_free_gauge(stag_ctx *ctx, int32_t gauge_id);

/* Lattice extents of a registered field. */
int stag_gauge_dims(stag_ctx *ctx, int32_t gauge_id, int32_t dims[4]);

/* Link rows stored for a registered field: 2 (third row rebuilt in the
 * kernels) or 3.  Errors: EINVAL (NULL), ENOENT (unknown id). */
int stag_gauge_link_rows(stag_ctx *ctx, int32_t gauge_id, int32_t *rows);

/* ---- layout conversion ----------------------------------------------- */

/* lex: device complex128 [V][3] -> eo: device complex128 [2][3][Vh]. */
int stag_pack_fermion(stag_ctx *ctx, const int32_t dims[4], const double *lex,
                      double *eo, void *stream);
/* eo: device complex128 [2][3][Vh] -> lex: device complex128 [V][3]. */
int stag_unpack_fermion(stag_ctx *ctx, const int32_t dims[4], const double *eo,
                        double *lex, void *stream);

/* ---- the matrix-vector routine (Sec. 3) ------------------------------- */

/*
 * out(x) = (accumulate ? out(x) : 0) + (D in)(x) for the output sites x of
 * parity out_parity whose checkerboard index lies in [offset, offset+count)
 * (count = -1: to the end of the parity).  This is the paper's
 * matrix-vector(offset, local_length, v, w) of Sec. 3, restricted to one
 * parity.  out_parity = STAG_ALL applies D to every site (offset must be 0,
 * count -1).  in, out: full-lattice fields in the even-odd layout, stored in
 * `precision` (STAG_F64, STAG_F32 or STAG_F16, layouts above; the links and
 * the arithmetic are of the same precision, FP32 arithmetic for STAG_F16).
 * Only the other parity of `in` is read.  Sites outside the range are
 * untouched.
 * on_device = 1: in and out are device pointers; the call is asynchronous
 *   on `stream` (NULL = the context's stream); they must not overlap.  The
 *   first call for a field and precision times the kernel shapes on scratch
 *   from the arena and waits for that.
 * on_device = 0: in and out are host pointers (the paper's copyin / copyout
 *   of Sec. 4): the input half is copied to the device, D applied there, the
 *   output range copied back into `out` (and first copied in when
 *   accumulating); the call returns when `out` is complete.  Staging memory
 *   comes from the arena (ENOMEM if it cannot hold two fields).
 * Errors: ENOENT, EINVAL (parity, range, precision, NULL, overlap), ENOMEM,
 * EHIP.
 */
int stag_dslash(stag_ctx *ctx, int32_t gauge_id, int32_t out_parity,
                int64_t offset, int64_t count, const void *in, void *out,
                int32_t accumulate, int32_t precision, int32_t on_device,
                void *stream);

/*
 * Convert a full-lattice fermion field of the field shape `dims` between
 * storage precisions (STAG_F64 / STAG_F32 / STAG_F16, even-odd layout):
 * rounding to nearest; to STAG_F16 each site is divided by its scale first.
 * in, out: device pointers, not overlapping.  Asynchronous on `stream`.
 * Errors: EINVAL.
 */
int stag_convert_fermion(stag_ctx *ctx, const int32_t dims[4], const void *in,
                         int32_t in_precision, void *out, int32_t out_precision,
                         void *stream);

/* ---- the conjugate-gradient solve (Sec. 4) --------------------------- */

/*
 * Solve (m^2 - D^2) x = b on the parity systems selected by params->parity,
 * from x = 0 (Sec. 4).  b, x: full-lattice FP64 fields in the even-odd
 * layout; only the selected parities are read / written.  y (nullable): if
 * given, y = D x on the opposite parity of every solved system (the paper
 * reconstructs the other half of the lattice from the solution after the
 * loop, Sec. 4).  Every iteration runs on the GPU with the scalars and the
 * stopping test kept in device memory; the host only looks at a status
 * record every few iterations.  The result is accepted when the FP64 true
 * residual on the GPU satisfies ||b - A x|| <= tol ||b|| for each parity
 * system.
 * on_device = 1: b, x, y are device pointers, and the solve runs on
 *   `stream` (NULL = the context's stream).
 * on_device = 0: they are host pointers (the paper's copyin / copyout data
 *   region of Sec. 4): b is copied to the device, the solve runs there and
 *   x (and y) are copied back; staging memory comes from the arena.
 * Blocks until done; info (nullable) receives the outcome.  Returns STAG_OK
 * or the solve's error (ENOCONV: x holds the last iterate).  Errors: ENOENT,
 * EINVAL (m <= 0, tol <= 0, bad parity or precision, an FP16 threshold
 * below its floor), ENOMEM, ENOCONV, EBREAKDOWN, ENONFINITE.
 */
int stag_cg_solve(stag_ctx *ctx, int32_t gauge_id, const stag_cg_params *params,
                  const double *b, double *x, double *y, int32_t on_device,
                  void *stream, stag_cg_info *info);

/*
 * For callers that cannot allocate memory (code that must not call hipMalloc
 * or a caching allocator, e.g. inside tight serving loops or harnesses that
 * forbid allocation): stag_cg_solve on device pointers whose workspace is
 * the library's fixed device buffer of STAG_NOALLOC_WORKSPACE_BYTES instead
 * of the arena.  The buffer is a file-scope device array: every GPU the
 * library runs on holds one copy of it from stag_create until the process
 * ends.  Nothing is allocated during the call (no arena, hipMalloc, pinned
 * host memory, event, stream or graph); the state records travel through a
 * fixed host buffer and the call synchronises `stream` where
 * stag_cg_solve waits on events.  The kernel shape is the one tuned for the
 * field by an earlier stag_cg_solve at the same precision, else the default
 * (the call never tunes).  Calls on one GPU share its buffer: they are
 * serialised by a lock within the process, each call re-initialises all of
 * the buffer it reads, and the buffer keeps the last call's contents.
 * Arguments, results and errors as for stag_cg_solve with on_device = 1,
 * plus EINVAL when the solve's workspace (about 480 bytes per checkerboard
 * site in FP64, 340 in FP32 and 290 in FP16, plus 200 KB) exceeds the buffer.
 */
#define STAG_NOALLOC_WORKSPACE_BYTES ((size_t)128 << 20)
int stag_cg_solve_noalloc(stag_ctx *ctx, int32_t gauge_id, const stag_cg_params *params,
                          const double *b, double *x, double *y, void *stream,
                          stag_cg_info *info);

/*
 * Solve nrhs systems that share one gauge field in one batched solve: every
 * CG iteration reads the links once for all right-hand sides.  params[i]
 * may differ in mass, tol, maxiter and parity; precision must be the same for
 * all.  b[i], x[i]: device full-lattice fields (even-odd layout).  The tile
 * of right-hand sides processed per link read and the kernel shapes are
 * chosen by the library's autotuner; while fewer systems are still running
 * than a tile takes, smaller tiles (tuned alongside, possibly with other
 * lanes per site and block sizes) take over.  A system's arithmetic is that
 * of the single solve up to the order in which its sums are formed, so its
 * result can differ from the same system solved alone (or in another batch)
 * by rounding: both meet the FP64 true residual tol, and the solutions agree
 * within the error that residual allows.  The same batch solved twice gives
 * the same bits.  infos[i] receives each outcome.  Blocks until all are done.
 * Returns STAG_OK if every system converged, else the first error.
 */
int stag_cg_solve_batch(stag_ctx *ctx, int32_t gauge_id, int32_t nrhs,
                        const stag_cg_params *params, const double *const *b,
                        double *const *x, void *stream, stag_cg_info *infos);

/* ---- molecular dynamics around the solve (Sec. 2, Sec. 6) ------------- */

/*
 * The force of the staggered pseudofermion action of the paper's HMD
 * program, which it runs around the CG of Sec. 4 without writing the action
 * out; the textbook reading for the even-site operator the CG solves:
 *   S_F = phi^dagger (m^2 - D_eo D_oe)^{-1} phi   (phi on the even sites),
 *   F_mu(z) = TA[ eps(z) c_mu(z) U_mu(z) W(z + mu) W(z)^dagger ],
 * with W = x on the even sites and y = D_oe x on the odd sites (exactly what
 * stag_cg_solve returns for parity STAG_EVEN with y: x's even half and y's
 * odd half), c_mu(z) = eta_mu(z) b_mu(z) / 2 (b: the t-boundary sign of the
 * hop from z to z + mu), eps(z) = +1 on even and -1 on odd sites, and
 * TA(Z) = (Z - Z^dagger)/2 - tr(Z - Z^dagger)/6 the traceless anti-Hermitian
 * part.  Then dS_F/dw = 2 Re tr[i T F_mu(z)] for U_mu(z) -> exp(i w T) U_mu(z),
 * T Hermitian and traceless.
 * w: device even-odd FP64 field (layout above).  force: device complex128
 * [V][4][3][3] in the gauge-field input layout; force = (accumulate ? force :
 * 0) + coeff * F.  Asynchronous on `stream`.  Errors: ENOENT, EINVAL (NULL,
 * overlap, non-finite coeff, a Wilson field).
 */
int stag_fermion_force(stag_ctx *ctx, int32_t gauge_id, const double *w, double *force,
                       double coeff, int32_t accumulate, void *stream);

/*
 * The Wilson gauge action's force on links given in the input layout
 * (complex128 [V][4][3][3] lexicographic, device, periodic in every
 * direction): S_G = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3) and
 * F_G = -(beta/6) TA[U_mu(x) Sigma_mu(x)] with Sigma the sum of the six
 * staples, in the convention of stag_fermion_force.  force: same layout;
 * force = (accumulate ? force : 0) + coeff * F_G.  dims as for set_gauge.
 * Asynchronous on `stream`.  Errors: EINVAL.
 */
int stag_gauge_force(stag_ctx *ctx, const int32_t dims[4], const double *links, double beta,
                     double *force, double coeff, int32_t accumulate, void *stream);

/*
 * The pseudofermion of a registered staggered field from a Gaussian field
 * chi on every site: phi = m chi - D chi on the even sites, phi = 0 on the
 * odd ones, so that <phi phi^dagger> is proportional to m^2 - D_eo D_oe.
 * chi, phi: device even-odd FP64 fields, not overlapping.  Asynchronous on
 * `stream`.  Errors: ENOENT, EINVAL.
 */
int stag_pseudofermion(stag_ctx *ctx, int32_t gauge_id, const double *chi, double *phi,
                       double mass, void *stream);

typedef struct {
    double beta;            /* Wilson gauge coupling */
    double mass;            /* staggered mass, > 0 */
    double eps;             /* molecular-dynamics step, > 0 */
    double tol;             /* CG tolerance of every force solve */
    int32_t nsteps;         /* leapfrog steps, >= 1 */
    int32_t maxiter;        /* CG iteration limit per solve */
    int32_t precision;      /* CG precision: STAG_FP64, STAG_FP32_RU or STAG_FP16_RU */
    int32_t t_antiperiodic; /* fermion boundary in t */
} stag_md_params;

typedef struct {
    double kinetic[2];        /* -sum tr Q^2 at the start and at the end */
    double gauge_action[2];   /* S_G at the start and at the end */
    double fermion_action[2]; /* S_F = Re phi^dagger x at the start and at the end */
    double delta_h;           /* H(end) - H(start) */
    double seconds;
    int32_t cg_iters;         /* CG iterations summed over the force solves */
    int32_t solves;           /* CG solves (nsteps + 1) */
} stag_md_info;

/*
 * One molecular-dynamics trajectory of the HMD program the paper runs
 * around its CG (Sec. 2, Sec. 6), in the textbook reading the paper leaves
 * open: H = -sum tr Q^2 + S_G + S_F (S_F as for stag_fermion_force),
 * dU/dt = Q U and dQ/dt = F_G + F_F; leapfrog with n steps of eps: Q +=
 * eps/2 F, then n times { U = exp(eps Q) U projected onto SU(3); Q += eps F }
 * with the last momentum step eps/2.  Every force needs one CG solve of the
 * even-site system on the current links (stag_cg_solve with parity EVEN and
 * y), on a private copy of the field rebuilt after each link update.
 * links (in/out): device complex128 [V][4][3][3] lexicographic, special
 * unitary.  momenta (in/out): same layout, anti-Hermitian and traceless.
 * phi: device even-odd FP64 pseudofermion (even sites).  Blocks until done;
 * info (nullable) receives the energies.  Errors: EINVAL (bad parameters,
 * links that are not special unitary), ENOMEM, and the errors of the solves.
 */
int stag_md_trajectory(stag_ctx *ctx, const int32_t dims[4], double *links, double *momenta,
                       const double *phi, const stag_md_params *params, void *stream,
                       stag_md_info *info);

/* ---- serving: continuous batching ------------------------------------ */

/*
 * Queue a solve.  b_dev / x_dev are device full-lattice fields (even-odd
 * layout) borrowed until stag_poll / stag_wait report completion.  The
 * request is ordered after the work enqueued on the context's stream before
 * this call (an event recorded there is waited on before b is read and x
 * written), so a source written on that stream needs no synchronisation.  A
 * scheduler thread admits queued requests into batch slots of their gauge
 * field while memory (the arena) and slots allow, runs the batch in epochs
 * of CG iterations on the field's own stream, and between epochs retires
 * converged requests and admits new ones, so requests arriving while others
 * run join the running batch.  Different gauge fields run on different
 * streams and overlap.  *ticket receives the request's handle.
 * Errors: ENOENT, EINVAL, EAGAIN (queue full).
 */
int stag_submit(stag_ctx *ctx, int32_t gauge_id, const stag_cg_params *params,
                const double *b_dev, double *x_dev, uint64_t *ticket);

/* STAG_PENDING while the request is queued or running; otherwise its final
 * status, with info filled (seconds = submit -> completion).  A completed
 * ticket may be polled repeatedly until stag_release_ticket. ENOENT: unknown. */
int stag_poll(stag_ctx *ctx, uint64_t ticket, stag_cg_info *info);

/* Block until the request completes; returns its final status. */
int stag_wait(stag_ctx *ctx, uint64_t ticket, stag_cg_info *info);

/* Forget a completed ticket.  EBUSY if it is still pending. */
int stag_release_ticket(stag_ctx *ctx, uint64_t ticket);

/* Serving limits: slots per gauge field (1..64) and queue capacity.  Call
 * before the first stag_submit; EBUSY afterwards. */
int stag_serve_config(stag_ctx *ctx, int32_t slots_per_field, int32_t epoch_iters,
                      int32_t queue_capacity);

/* ---- tuning and introspection ---------------------------------------- */

/*
 * Describe the kernel configuration the autotuner chose for the D_slash of a
 * gauge field at a precision (0 FP64, 1 FP32, 2 FP16) and right-hand-side
 * count: lanes per site, threads per block, right-hand sides per link read,
 * and whether the neighbour tables are read (1) or neighbours are computed
 * from coordinates (0).  Runs the tuner if that case has not been tuned yet.
 */
int stag_tune_info(stag_ctx *ctx, int32_t gauge_id, int32_t precision,
                   int32_t nrhs, int32_t *lanes_per_site, int32_t *block,
                   int32_t *rhs_tile, int32_t *use_tables);

/*
 * Describe the CG step-kernel shape tuned for a gauge field, a precision
 * (0 FP64, 1 FP32_RU, 2 FP16_RU) and a number of right-hand sides (the
 * slots of the solve: 1 for stag_cg_solve, nrhs for stag_cg_solve_batch,
 * slots_per_field for the server): lanes per site, threads per block,
 * systems per tile, neighbour tables read (1) or computed (0), and whether a
 * reduction kernel sums each step kernel's partial sums (1) or every block of
 * the next kernel does (0).  While fewer systems run than a tile takes, the
 * solve may use smaller tiles tuned alongside.  shared_links = 1: the FP32 /
 * FP16 tiles that stage each block's links in LDS for all systems of the tile
 * (one wavefront per system, block = 64 x rhs_tile threads, one lane per
 * site); 0: register tiles.  Does not tune: ENOENT until a solve of that
 * shape has run on the field; EINVAL for a bad precision or count, or a
 * Wilson field.  Any output pointer may be null.
 */
int stag_cg_tune_info(stag_ctx *ctx, int32_t gauge_id, int32_t precision, int32_t nrhs,
                      int32_t *lanes_per_site, int32_t *block, int32_t *rhs_tile,
                      int32_t *use_tables, int32_t *reduce, int32_t *shared_links);

/* ---- Wilson fermions (the paper's second workload, Sec. 2 and Sec. 6) ------------
 *
 * The paper runs an N_f = 2 Wilson-fermion program without writing the
 * operator out; the library takes the textbook form
 *   M = 1 - kappa H,
 *   (H psi)(x) = sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                        + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)],
 * with the same sites, links and boundary conditions as the staggered
 * operator, and gamma matrices of a chiral basis, gamma_5 = diag(1,1,-1,-1):
 *   gamma_x = [[0,0,0,i],[0,0,i,0],[0,-i,0,0],[-i,0,0,0]],
 *   gamma_y = [[0,0,0,-1],[0,0,1,0],[0,1,0,0],[-1,0,0,0]],
 *   gamma_z = [[0,0,i,0],[0,0,0,-i],[-i,0,0,0],[0,i,0,0]],
 *   gamma_t = [[0,0,1,0],[0,0,0,1],[1,0,0,0],[0,1,0,0]].
 * Spin-colour vectors: lexicographic complex128 [V][4 spin][3 colour]
 * (host side, for stag_pack_spinor), and the library's even-odd layout
 * complex128 [2 parity][4 spin][3 colour][V/2] on the device.  All FP64.
 */

/* Register links for the Wilson operator (same input layout and ownership as
 * stag_set_gauge).  The t-boundary sign is folded in, the backward links
 * U(x-mu)^dagger are stored at the site that uses them, and special unitary
 * fields keep two rows (as for stag_set_gauge; STAG_LINK_ROWS=3 keeps three).
 * The id is usable only with the stag_wilson_* calls (the staggered calls
 * return EINVAL for it, and the Wilson calls for a staggered id).
 * Errors: EINVAL, ENOMEM, ENONFINITE.  Synchronous. */
int stag_set_gauge_wilson(stag_ctx *ctx, const int32_t dims[4], const double *links,
                          int32_t links_on_device, int32_t t_antiperiodic,
                          int32_t *gauge_id);

/* Lexicographic [V][4][3] <-> even-odd [2][4][3][V/2] spin-colour vectors
 * (device pointers, not overlapping).  Stream-ordered on `stream`. */
int stag_pack_spinor(stag_ctx *ctx, const int32_t dims[4], const double *lex,
                     double *eo, void *stream);
int stag_unpack_spinor(stag_ctx *ctx, const int32_t dims[4], const double *eo,
                       double *lex, void *stream);

/* out = H in on the sites of out_parity (STAG_EVEN / STAG_ODD: the other
 * parity of `out` is not written; STAG_ALL: every site).  in, out: device
 * even-odd spin-colour vectors, not overlapping.  Errors: EINVAL, ENOENT.
 * Asynchronous on `stream`, except that the first hop or solve of a field
 * times the kernel shapes on scratch vectors from the arena (the defaults if
 * they do not fit) and waits for that. */
int stag_wilson_dslash(stag_ctx *ctx, int32_t gauge_id, int32_t out_parity,
                       const double *in, double *out, void *stream);

/* Solve M x = b (full lattice) by CG on the even-odd normal equations:
 * Mhat = 1 - kappa^2 D_eo D_oe on the even sites, Mhat^dagger Mhat x_e =
 * Mhat^dagger (b_e + kappa D_eo b_o) (Mhat^dagger = gamma_5 Mhat gamma_5),
 * stopping when <r,r> < tol^2 <Mhat^dagger bhat, Mhat^dagger bhat>, then
 * x_o = b_o + kappa D_oe x_e.  Scalars and the stopping test stay on the
 * device.  info->true_rel_resid is ||b - M x|| / ||b|| in FP64.
 * b, x: device even-odd vectors (x is overwritten).  Errors: EINVAL (kappa
 * <= 0, tol outside (0,1), maxiter < 0, overlap), ENOENT, ENOMEM, ENOCONV,
 * EBREAKDOWN, ENONFINITE.  Returns when the solve is complete. */
int stag_wilson_solve(stag_ctx *ctx, int32_t gauge_id, double kappa, double tol,
                      int32_t maxiter, const double *b, double *x, void *stream,
                      stag_cg_info *info);

/* Library version string. */
const char *stag_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STAGCG_H */
