/* voxcap.h -- C ABI of the MI355X FFT-accelerated capacitance solver for voxelized
 * conductor / dielectric structures (VoxCap, Wang, Qian, White, Yucel).
 *
 * Problem statement (Sec. II.A): a box of nx*ny*nz cubic voxels of edge dv holds
 * conductors (dense ids 0..m-1) and non-conductor voxels of relative permittivity
 * eps_r; outside the box is a background of relative permittivity eps_background.
 * Charges live on piecewise-constant panels (eq. 3): every voxel face between a
 * conductor and a non-conductor, and every face between two non-conductors of
 * different permittivity.  The Galerkin system of eq. (4) -- potentials on conductor
 * panels (eq. 5), normal-field continuity with the jump term on dielectric panels
 * (eq. 6, eq. 7) -- is solved once per conductor held at unit potential (text after
 * eq. 7), and the capacitance matrix follows from eq. (8) with the free-charge
 * scaling of Sec. II.A.
 *
 * Conventions used by every call:
 *  - Arrays of voxels are C ordered, x slowest: index (i*ny + j)*nz + k.
 *  - Dimensionless form: voxel edge 1 and 4*pi*eps0 = 1.  The operator A applied by
 *    vc_apply is the matrix of eq. (4) in that form, in the library's panel order,
 *    with dielectric rows written for the +axis normal: its diagonal is
 *    2*pi*(eps_lo+eps_hi)/(eps_lo-eps_hi) and its field integral is taken along
 *    +axis (this is the paper's row multiplied by +-1, Sec. II.B note 3; the
 *    solution is the same).  The right-hand side of conductor i is 1 on the panels
 *    of conductor i and 0 elsewhere.  C_ij = 4*pi*eps0*dv * sum_{k in i} eps_adj(k) *
 *    rho_k^(j) in farads.
 *  - Panel order: sorted by (normal axis, i, j, k).
 *  - "_dev" pointers are device pointers on the problem's device; the caller owns
 *    them and keeps them alive until the given stream has finished with them.
 *    "hip_stream" is a hipStream_t (NULL = the null stream).
 *  - Every call returns a vc_status; on failure vc_last_error() gives a message
 *    (thread local).  A VC_ERR_HIP failure leaves the problem unusable.
 *  - One vc_problem must not be used from two threads at once.
 */
#ifndef VOXCAP_H
#define VOXCAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VC_OK = 0,
  VC_ERR_ARG = -1,           /* bad argument or size                                    */
  VC_ERR_GEOMETRY = -2,      /* touching conductors, eps <= 0, no conductor, bad ids     */
  VC_ERR_HIP = -3,           /* HIP runtime error (sticky for the problem)               */
  VC_ERR_OOM = -4,           /* device or host allocation failed                         */
  VC_ERR_NOT_CONVERGED = -5, /* iteration limit hit; outputs hold the last iterate       */
  VC_ERR_NUMERIC = -6,       /* NaN/Inf or breakdown in the iteration                    */
  VC_ERR_STATE = -7          /* call order violated (e.g. apply before setup)            */
} vc_status;

typedef enum {
  VC_FP64 = 0,   /* FFT, block multiply and kernel spectra in double                      */
  VC_FP32 = 1,   /* FFT and block multiply in float, FP64 in/out and FP64 diagonal term    */
  VC_MIXED = 2   /* solves only: FP32 inner GMRES inside FP64 iterative refinement        */
} vc_precision;

typedef struct vc_problem vc_problem;

/* Voxel geometry.  cond_id: nx*ny*nz ids, -1 = not a conductor, else 0..m-1 (every id
 * used).  eps_r: nx*ny*nz relative permittivities (> 0) of non-conductor voxels (read
 * only where cond_id == -1).  dv: voxel edge in metres (> 0). */
typedef struct {
  int32_t nx, ny, nz;
  double dv;
  const int32_t *cond_id;
  const double *eps_r;
  double eps_background;
} vc_geometry;

/* One panel (Sec. II.A eq. 3).  The face lies at coordinate i (dir 0), j (dir 1) or
 * k (dir 2) along its normal axis and spans [idx, idx+1] along the other two.
 * kind 0 = conductor (cond = id, eps_adj = permittivity of the non-conductor side),
 * kind 1 = dielectric (cond = -1, eps_adj = 0).  eps_lo / eps_hi: permittivity on the
 * -axis / +axis side (0 on a conductor side). */
typedef struct {
  int32_t i, j, k;
  int8_t dir, kind;
  int16_t pad;
  int32_t cond;
  double eps_lo, eps_hi, eps_adj;
} vc_panel;

/* Setup options.  fft_size[a] = 0 chooses the smallest even 7-smooth size >= 2*n_a+1
 * (any size >= 2*n_a+1 gives the same product, the paper uses 2*(n_a+1), Sec. II.B).
 * nv[a] = voxels per preconditioner box along a (Sec. II.D; 0 = 8).  tucker_tol > 0
 * compresses the kernel spectra (eq. 13) and rebuilds them for each product;
 * 0 keeps them uncompressed.  precisions: bit mask of (1<<VC_FP64)|(1<<VC_FP32)
 * spectra to keep (0 = both). */
typedef struct {
  int32_t fft_size[3];
  int32_t nv[3];
  double tucker_tol;
  int32_t precisions;
  int32_t max_rhs;     /* largest nrhs later passed to vc_apply (0 = m)              */
  int32_t autotune;    /* 1: the first product of each (precision, direction, nrhs)
                          times every launch configuration of the x pass (radix plan x
                          column tile) and keeps the fastest; 0: a fixed heuristic.
                          Tuning synchronizes the stream once and is skipped while the
                          stream is being captured into a graph.                    */
  const char *tune_cache; /* optional tuning cache file (NULL: none): its matching
                          entries are loaded at setup (as vc_tuning_load; a missing
                          file loads nothing), and every x- and y-pass choice the
                          autotuner makes afterwards is merged into it (as
                          vc_tuning_save).  The string is copied.                    */
} vc_setup_opts;

/* Solve options.  GMRES(restart) with the block-diagonal-diagonal preconditioner
 * (Sec. II.D) applied on the right; stops when ||b - A x|| <= rtol ||b|| per column.
 * VC_MIXED has two forms (mixed_form):
 *   refinement: FP32 inner GMRES inside FP64 refinement (ir_max outer steps): each
 *     inner solve stops at max(inner_rtol, rtol / (2 x the largest outer relative
 *     residual still above rtol)), i.e. when the step has done what the outer tolerance
 *     needs or FP32 products can do (inner_rtol), and after at most 4 restart cycles;
 *   relaxed: one GMRES on the FP64 system whose restarts start from the FP64 residual,
 *     and whose Arnoldi products are FP64 until every iterating column's residual
 *     estimate is at most rtol / inner_rtol, FP32 after that (the product error a
 *     step can afford grows as the residual shrinks); a cycle that starts in FP32 and
 *     does not halve the true residual sends the rest of the solve back to FP64.
 * 0 picks defaults (rtol 1e-12, restart 35, max_iter 2000, inner_rtol 1e-6, ir_max 20,
 * mixed_form automatic). */
typedef struct {
  vc_precision prec;
  double rtol;
  int32_t restart, max_iter;
  double inner_rtol;
  int32_t ir_max;
  int32_t use_precond;   /* 1 = block-diagonal-diagonal (default), 0 = none, 2 = diagonal only,
                            3 = conventional block-diagonal over all panels (built on first
                            use; not for packed sets) */
  int32_t graph;         /* 0: each restart cycle runs on the device without host round trips
                            and, after the first, is replayed as one captured hipGraph
                            (default); 1: the same kernels issued one by one             */
  int32_t mixed_form;    /* VC_MIXED only: 0 automatic (relaxed when one FP64 product's
                            algorithmic bytes, vc_stats.bytes_model at FP64, are at most
                            VC_MIXED_RELAXED_MAX_BYTES: products that small are bound by
                            latency and cache, so FP64 steps cost about as much as FP32
                            ones, and refinement's restart would cost more; refinement
                            otherwise), 1 refinement, 2 relaxed                          */
} vc_solve_opts;

#define VC_MIXED_REFINEMENT 1
#define VC_MIXED_RELAXED 2
#define VC_MIXED_RELAXED_MAX_BYTES (256.0 * 1024 * 1024)

typedef struct {
  int32_t iters[64];          /* GMRES iterations per right-hand side (first 64)   */
  double final_rre[64];       /* true relative residual per right-hand side        */
  int32_t ir_steps;           /* refinement steps (VC_MIXED)                        */
  int32_t mvp_count;          /* batched operator applications                      */
  double t_setup_s, t_solve_s;
  double spectra_bytes;       /* device bytes held by the kernel spectra            */
  int32_t tucker_rank_max;
  double bytes_model;         /* algorithmic HBM bytes of one product of the solve's
                                 right-hand sides (every pass, the model of
                                 vc_pass_times), in the inner product's precision   */
  int32_t mixed_form;         /* VC_MIXED: the form that ran (VC_MIXED_REFINEMENT or
                                 VC_MIXED_RELAXED); 0 otherwise                      */
  int32_t steps_fp32;         /* Arnoldi steps taken with FP32 products (the largest
                                 over right-hand sides, summed over segments)       */
} vc_stats;

/* Copy the geometry, extract the panels and validate (host only, no GPU work).
 * device: HIP device ordinal used by later calls. */
vc_status vc_problem_create(const vc_geometry *geom, int device, vc_problem **out);
vc_status vc_problem_destroy(vc_problem *p);
vc_status vc_panel_counts(const vc_problem *p, int64_t *n_cond, int64_t *n_diel, int32_t *m);
/* out: caller-allocated host array of n_cond + n_diel panels, library order. */
vc_status vc_panels(const vc_problem *p, vc_panel *out);
/* FFT grid sizes chosen by vc_setup (or the ones it will choose). */
vc_status vc_fft_size(const vc_problem *p, int32_t out_m[3]);

/* Build the kernel spectra (App. B tensors, FFT'ed; Sec. II.B), the optional Tucker
 * compression (Sec. II.C) and the preconditioner blocks (Sec. II.D) on the device. */
vc_status vc_setup(vc_problem *p, const vc_setup_opts *opts, void *hip_stream);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), eq. (4) via eq. (11).
 * x_dev, y_dev: N x nrhs doubles, column-major (column r at offset r*N), N = panels.
 * prec: VC_FP64 or VC_FP32 arithmetic inside the FFT product. */
vc_status vc_apply(vc_problem *p, int transpose, vc_precision prec, const double *x_dev,
                   double *y_dev, int32_t nrhs, void *hip_stream);

/* y = R x with the block-diagonal-diagonal preconditioner R of eq. (14)
 * (R^T when transpose = 1; the blocks are symmetric).  x_dev, y_dev: N x nrhs doubles as
 * in vc_apply, distinct arrays; 1 <= nrhs <= max_rhs of vc_setup, else VC_ERR_ARG. */
vc_status vc_apply_precond(vc_problem *p, int transpose, const double *x_dev, double *y_dev,
                           int32_t nrhs, void *hip_stream);

/* y = R x (R^T x when transpose = 1) with one of the preconditioners compared in
 * Sec. III.A.  kind: 1 = block-diagonal-diagonal of eq. (14); 2 = diagonal (the eq. (7)
 * diagonal on dielectric rows, the eq. (5) self term on conductor rows); 3 = the
 * conventional block-diagonal preconditioner: every panel (conductor and dielectric)
 * joins one nv box and each box's block of the full eq. (4) matrix is inverted (LU, FP64,
 * identical boxes sharing one inverse).  Kind 3 is built on first use (host work, then
 * device upload; not allowed during stream capture).  x_dev, y_dev: nrhs x N row-major
 * device arrays, distinct, 1 <= nrhs <= max_rhs.  Errors: VC_ERR_STATE before setup, VC_ERR_ARG for a
 * bad kind, nrhs or a packed set, VC_ERR_NUMERIC for a singular block. */
vc_status vc_apply_precond_kind(vc_problem *p, int32_t kind, int transpose, const double *x_dev,
                                double *y_dev, int32_t nrhs, void *hip_stream);

/* Storage of preconditioner kind 1 or 3 (kind 3 is built if needed): boxes, distinct
 * inverse blocks, and bytes of the distinct inverses plus the per-panel index and
 * diagonal arrays the apply reads.  Any output pointer may be null. */
vc_status vc_precond_info(vc_problem *p, int32_t kind, int64_t *nbox, int64_t *nblock, int64_t *bytes);

/* Capacitance matrix C (m x m, row-major, farads) by one solve per conductor, all m
 * right-hand sides advancing together.  rho_dev: optional N x m device output of the
 * dimensionless charges.  stats: optional. */
vc_status vc_capacitance(vc_problem *p, const vc_solve_opts *opts, double *C, double *rho_dev,
                         vc_stats *stats);

/* vc_capacitance for callers that cannot allocate device memory (code next to graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve and
 * kernels, with every device array of the solve (Krylov basis, vectors, Gram-Schmidt
 * partials and completion counters, cycle state, the m x m result) taken from one
 * static device array of VC_STATIC_SCRATCH_BYTES per GPU, held until the process ends.
 * It calls no hipMalloc / hipFree; the problem must have been set up (vc_setup
 * allocates its spectra, work arrays and preconditioner).  Restart cycles are issued
 * kernel by kernel on hip_stream (NULL = the null stream; opts->graph is ignored: no
 * graph is captured), and the call returns after C is on the host.  The first product
 * of a (precision, direction, nrhs) key still runs the x-pass autotuner when the
 * problem was set up with autotune = 1 (HIP events, no device memory).
 * Errors: VC_ERR_ARG when the solve needs more than VC_STATIC_SCRATCH_BYTES (about
 * 8 (N m (restart + 10)) bytes) or use_precond is 3 (its blocks are built on first
 * use); otherwise as vc_capacitance.  Every call on one GPU shares that GPU's array
 * and leaves its contents behind: calls that overlap on one GPU (several host threads,
 * or streams that run concurrently) race and give wrong results. */
#define VC_STATIC_SCRATCH_BYTES (64u << 20)
vc_status vc_capacitance_static(vc_problem *p, const vc_solve_opts *opts, double *C, double *rho_dev,
                                vc_stats *stats, void *hip_stream);

/* ---- Packed sets: many independent problems of different sizes solved as one
 * (eq. (8) per member; the product of eq. (11) and preconditioner of eq. (14) of every
 * member in the same launches).  The members' conductor right-hand sides become the
 * columns of one block whose rows are the largest member's panel count (zero past each
 * member's own panels); one GMRES runs over all columns, each column stopping at its
 * own tolerance, and every restart cycle of the whole set is one graph launch in which
 * each pass of the product is ONE kernel launch over all members (the x pass: one per
 * distinct compiled radix).
 * vc_pack_create: problems[0..n) after vc_setup (uncompressed spectra, max_rhs >= m,
 * one device, at most 256 conductors in total).  The set keeps pointers into the
 * members' device tables and work arrays: the members must outlive it and must not be
 * set up again or solved concurrently with it.  Errors: VC_ERR_ARG / VC_ERR_STATE with
 * vc_last_error; *out stays NULL. */
typedef struct vc_pack vc_pack;
vc_status vc_pack_create(vc_problem *const *problems, int32_t n, vc_pack **out);
vc_status vc_pack_destroy(vc_pack *pk);
/* out[0] members, out[1] columns, out[2] rows, out[3] / out[4] kernel launches per
 * FP64 / FP32 product, out[5] launches per preconditioner application. */
vc_status vc_pack_info(const vc_pack *pk, int32_t out[6]);
/* The product of every member at once: x_dev / y_dev hold out[1] columns of out[2]
 * rows (column-major device doubles); member k's columns (one per conductor, members in
 * order) carry its panel vector in their first N_k rows.  Rows past N_k of y are left
 * as they are.  Same per-member arithmetic as vc_apply (transpose 0); stream as in
 * vc_apply. */
vc_status vc_pack_apply(vc_pack *pk, vc_precision prec, const double *x_dev, double *y_dev, void *hip_stream);
/* Capacitance matrices of every member: C_out[k] m_k x m_k host doubles (row-major),
 * stats: optional array of n (iterations and final relative residual per column; solve
 * time and product count are the whole set's).  The first call for a given (precision,
 * restart) captures the cycle graphs; later calls replay them. */
vc_status vc_pack_capacitance(vc_pack *pk, const vc_solve_opts *opts, double *const *C_out, vc_stats *stats);

/* One-shot form: vc_pack_create + vc_pack_capacitance + vc_pack_destroy, under two
 * names (vc_batch_capacitance is the name of the batched call in the problem
 * statement's interface; both behave identically). */
vc_status vc_batch_capacitance(vc_problem *const *problems, int32_t n, const vc_solve_opts *opts,
                               double *const *C_out, vc_stats *stats);
vc_status vc_capacitance_batch(vc_problem *const *problems, int32_t n, const vc_solve_opts *opts,
                               double *const *C_out, vc_stats *stats);

/* dC/d(eps_r of block b) for every block (nblocks x m x m, row-major, farads per unit
 * relative permittivity) by one adjoint solve per conductor (A^T lambda_i = w_i).
 * block_of_voxel: nx*ny*nz host ids in [-1, nblocks).  C_out: optional m x m. */
vc_status vc_capacitance_grad_eps(vc_problem *p, const vc_solve_opts *opts,
                                  const int32_t *block_of_voxel, int32_t nblocks,
                                  double *dC, double *C_out, vc_stats *stats);

/* New relative permittivities for a set-up problem without a new setup (eq. 7, eq. 8):
 * the operator depends on them only through the jump term of eq. (7) on dielectric
 * panels, and C through the free-charge weights of eq. (8); the kernel spectra (and
 * their Tucker form), the Toeplitz tensors and the eq. (14) conductor blocks do not, so
 * only those per-panel arrays and the preconditioner's dielectric diagonal are
 * rewritten (in place: graphs captured by earlier solves stay valid).
 * eps_r: nx*ny*nz host doubles, C order, read where cond_id == -1 (> 0, finite);
 * eps_background: the new background permittivity (> 0).  The panel list must not
 * change: every dielectric face keeps different permittivities on its two sides and
 * no new one appears, else VC_ERR_ARG and nothing is changed (VC_ERR_GEOMETRY for an
 * invalid value).  Synchronizes hip_stream before and after the update.  The
 * comparison preconditioner of use_precond 3, if built, is dropped and rebuilt at its
 * next use.  A packed set created from p earlier keeps the old values: create packs
 * after the update.  VC_ERR_STATE before vc_setup, VC_ERR_ARG on a packed set. */
vc_status vc_update_eps(vc_problem *p, const double *eps_r, double eps_background, void *hip_stream);

/* Per-pass timing of the product (measurement only).  At level 1, vc_apply records HIP
 * events on its stream around each of its passes (and the Tucker rebuild):
 *   0 scatter + z transform, 1 y transform, 2 x transform + block multiply + inverse x,
 *   3 inverse y transform, 4 inverse z transform + gather.
 * At level 2 it brackets pass 2 only (two events per product instead of six: each
 * event adds a few microseconds between the launches it separates); the other passes
 * then report zero launches.  Level 0 records nothing.  No events are recorded while
 * the stream is being captured.
 * vc_pass_times waits for the recorded events and returns, per pass, the summed
 * milliseconds, the number of launches, and the algorithmic bytes of ONE launch of the
 * most recent vc_apply (compulsory reads + writes of the pruned pass, counting the
 * kernel spectra once per launch); it then clears the accumulators. */
/* The reduction of eq. (8) as a map of given charges: C_dev[i*nrhs + j] =
 * 4 pi eps0 dv sum over the panels k of conductor i of eps_adj(k) rho[j*N + k].
 * rho_dev: N x nrhs device doubles, column-major; C_dev: m x nrhs device doubles. */
vc_status vc_charges_to_capacitance(vc_problem *p, const double *rho_dev, int32_t nrhs, double *C_dev,
                                    void *hip_stream);

/* Its adjoint (dC/d(charges) applied to a cotangent): grho_dev[j*N + k] =
 * 4 pi eps0 dv eps_adj(k) gC_dev[cond(k)*nrhs + j] on conductor panels, 0 on dielectric. */
vc_status vc_charges_to_capacitance_adjoint(vc_problem *p, const double *gC_dev, int32_t nrhs,
                                            double *grho_dev, void *hip_stream);

/* Tucker form of the stored spectra (vc_setup with tucker_tol > 0; eq. 13, Sec. II.C):
 * number of stored pairs, their multilinear ranks (rows of 3 in ranks[0..44], pair order
 * P xx yy zz xy xz yz then E xx xy xz yx yy yz zx zy zz), numbers kept compressed
 * (r1 r2 r3 + sum D_i r_i) and uncompressed (D1 D2 D3 per pair), and the summed time and
 * count of the rebuilds recorded while profiling was enabled.  Zeros without Tucker. */
vc_status vc_tucker_info(vc_problem *p, int32_t *npairs, int32_t ranks[45], double *stored_numbers,
                         double *full_numbers, double *rebuild_ms, int32_t *rebuilds);

/* enable: the profiling level 0, 1 or 2 above; VC_ERR_ARG otherwise. */
vc_status vc_profile_enable(vc_problem *p, int enable);

/* Text report of the x-pass launch configurations in use, one line per
 * (precision, direction, nrhs): radices, columns per workgroup, threads, and whether
 * the autotuner timed it (with the time of the chosen and of the default
 * configuration).  Writes at most len bytes including the terminating zero. */
vc_status vc_tuning_report(vc_problem *p, char *buf, int32_t len);

/* Launch configurations of the x pass available for a precision and direction, as
 * rows of 8 int32: {nst, r_0, ..., r_5, cols} (radices r_0 >= ... >= r_{nst-1}, unused
 * ones 0; cols = columns per workgroup).  With stored (uncompressed) spectra, cols < 0
 * is the staged form of |cols| columns: one workgroup per column tile copies the tile's
 * stored spectra into LDS once and runs every right-hand side against them (cols > 0:
 * one workgroup per tile and right-hand side, spectra read from memory).  Writes at
 * most max_rows rows to out and the number available to *n_rows.  Requires vc_setup. */
vc_status vc_xpass_candidates(vc_problem *p, vc_precision prec, int transpose, int32_t *out,
                              int32_t max_rows, int32_t *n_rows);

/* Pins the x-pass configuration (a row as returned above) for products with this
 * precision, direction and nrhs; it replaces what the heuristic or the autotuner chose
 * and is kept until the next vc_setup.  VC_ERR_ARG if the row is not a valid
 * configuration for this problem. */
vc_status vc_xpass_set(vc_problem *p, vc_precision prec, int transpose, int32_t nrhs,
                       const int32_t cfg[8]);
vc_status vc_pass_times(vc_problem *p, double ms[5], int32_t launches[5], double bytes[5]);

/* Pins the y-pass kernel for products with this precision, direction (transpose),
 * transform direction (inverse = 0 after the z pass, 1 before it) and nrhs: kernel 0 =
 * LDS ping-pong tiles, 1 = register-edge stages with `cols` columns per workgroup
 * (0 = the heuristic's width; a width whose tile does not fit runs at that width) and
 * xcd_group = 1, 2 or 4 consecutive column tiles of a row per XCD, or -1 for all of a
 * row's tiles.  Kept until the next vc_setup.  VC_ERR_ARG on a value outside those
 * ranges. */
vc_status vc_ypass_set(vc_problem *p, vc_precision prec, int transpose, int inverse, int32_t nrhs,
                       int32_t kernel, int32_t cols, int32_t xcd_group);

/* Tuning cache file (text, one line per choice).  vc_tuning_save merges this problem's
 * timed x-pass and y-pass choices into `path` (replacing entries of the same shape,
 * precision, direction, nrhs and GPU architecture; written to path.tmp, then renamed)
 * and reports how many it wrote.  vc_tuning_load adopts every entry of `path` that
 * matches this problem's shape and architecture (an x-pass entry only if it is one of
 * this problem's own candidates), as if pinned by vc_xpass_set / vc_ypass_set, so those
 * passes skip the timing and a problem of the same shape computes bitwise the same
 * products; it reports how many it adopted, and a missing file loads nothing.  Both
 * require vc_setup; a later vc_setup forgets what was loaded. */
vc_status vc_tuning_save(vc_problem *p, const char *path, int32_t *n_saved);
vc_status vc_tuning_load(vc_problem *p, const char *path, int32_t *n_loaded);

/* ---- Toeplitz setup path (Sec. II.C, Tab. I) ----
 * The block Toeplitz tensors of App. B are computed once over a largest grid of
 * nmax[0] x nmax[1] x nmax[2] voxels, Tucker-compressed (eq. 13) and kept (in memory, or
 * on disk through save / load); a problem's setup can then restore them cropped to its
 * own grid and embed them in its circulants instead of evaluating the panel integrals.
 *
 * Pairs are numbered as in vc_tucker_info: 0..5 = eq. (5) xx yy zz xy xz yz, 6 + 3a + b
 * = eq. (6) with observer normal a and source normal b.  Pair q is stored as its octant
 * T_q[t0][t1][t2] = K_q(d) at the non-negative centre offsets d_a = t_a + h_a,
 * t_a = 0..n_a, where h_a = 1/2 on the two normal axes of an orthogonal pair and 0
 * otherwise (row-major, t2 fastest; (n0+1)(n1+1)(n2+1) doubles).  Eq. (5) is even in
 * every offset component and eq. (6) odd in d_a and even in the rest, so the octant
 * gives every lag of a grid of n voxels.  A grid of n <= nmax voxels uses the leading
 * n_a + 1 rows of each Tucker factor, so its restored tensor carries no error beyond
 * the compression's: ||T - T_restored||_F <= tol ||T over nmax||_F per pair.  Values
 * are dimensionless (voxel edge 1), so one cache serves every voxel size. */
typedef struct vc_toeplitz_cache vc_toeplitz_cache;

/* Fills the 15 octants over nmax (1..4096 per axis, (nmax0+1)(nmax1+1)(nmax2+1) < 2^31) on
 * `device` and compresses each with
 * relative tolerance tol in (0, 1) (FP64, sequentially truncated HOSVD).  Synchronizes
 * hip_stream.  *out is owned by the caller (vc_toeplitz_cache_destroy). */
vc_status vc_toeplitz_cache_build(const int32_t nmax[3], double tol, int device, void *hip_stream,
                                  vc_toeplitz_cache **out);
vc_status vc_toeplitz_cache_destroy(vc_toeplitz_cache *c);
/* Binary file: 8-byte tag, nmax, pair count, tol, then per pair its ranks, core and the
 * three factors as host-order doubles.  load checks the tag, sizes and ranks
 * (VC_ERR_ARG on any mismatch or a truncated file) and uploads to `device`. */
vc_status vc_toeplitz_cache_save(const vc_toeplitz_cache *c, const char *path);
vc_status vc_toeplitz_cache_load(const char *path, int device, vc_toeplitz_cache **out);
/* Any output may be NULL.  ranks: 3 per pair; stored_numbers: sum of core and factor
 * sizes; seconds: wall time of the build (fill and compression) or of the load. */
vc_status vc_toeplitz_cache_info(const vc_toeplitz_cache *c, int32_t nmax[3], double *tol,
                                 int32_t ranks[45], double *stored_numbers, double *seconds);
/* out_dev: (n0+1)(n1+1)(n2+1) doubles on the cache's device, the restored octant of pair
 * `pair` for a grid of n voxels (1 <= n_a <= nmax_a, else VC_ERR_ARG).  Synchronizes. */
vc_status vc_toeplitz_cache_restore(const vc_toeplitz_cache *c, int32_t pair, const int32_t n[3],
                                    double *out_dev, void *hip_stream);
/* The same octant evaluated from the panel integrals (no cache), for comparison. */
vc_status vc_toeplitz_octant(int32_t pair, const int32_t n[3], int device, double *out_dev,
                             void *hip_stream);
/* Later vc_setup calls on p take the Toeplitz tensors from c (NULL: the panel integrals,
 * the default).  c must cover p's grid and live on p's device, and must stay alive until
 * those vc_setup calls have returned.  The eq. (14) preconditioner blocks that vc_setup
 * builds are read from the cache too; the comparison preconditioner of use_precond 3,
 * built at its first use, evaluates the panel integrals. */
vc_status vc_setup_toeplitz_source(vc_problem *p, const vc_toeplitz_cache *c);
/* Wall time of the last vc_setup, and the part of it spent producing the Toeplitz
 * tensors in circulant form (the integrals, or restore + crop + embed). */
vc_status vc_setup_time(const vc_problem *p, double *total_s, double *toeplitz_s);
/* Device bytes the problem holds after vc_setup (Sec. II.C is about this memory):
 * spectra_bytes: the kernel spectra as stored, uncompressed (6 or 15 real octants per
 * kept precision) or in the Tucker form (cores and factors in FP64 and FP32, plus the
 * strips T1 and T2 each product rebuilds; the spectra themselves are never stored);
 * work_bytes: the product's spectral work arrays and the solver workspace allocated so
 * far.  Any output pointer may be null. */
vc_status vc_memory_info(const vc_problem *p, double *spectra_bytes, double *work_bytes);

const char *vc_status_string(vc_status s);
const char *vc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VOXCAP_H */
