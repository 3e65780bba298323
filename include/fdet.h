/*
 * fdet.h -- C ABI of libfdet, a gfx950 (MI355X) implementation of the dense
 * stabilised fermion determinant.
 *
 * Problem (paper Sec. 2, "The sausage"): V = N lattice sites, N_t time
 * slices, slice matrices B_t = exp(dk K) diag(exp(i phi_t)), t = 1..N_t, and
 *     M = 1 + B_{N_t} ... B_1          (later slices to the left).
 * det M equals the determinant of the full (N N_t)^2 block fermion matrix
 * (Sec. 2), M^{-1} is the equal-time Green's function, and the HMC action
 * carries -log det M (eq. hamiltonian_alg), so its force is built from
 * d log det M / d phi_{t,x} (Sec. 3.1, Sec. 4 response formula).
 *
 * Method (Sec. 7, with the sporadic stabilisation of Sec. 9): the product is
 * kept as X D Y^{-1} (eq. def_matrix_as_product), re-decomposed by a pivoted
 * Householder QR every s slices (eqs. prod_2_mat_stab .. res_2_mat_stab) and
 * closed by one more QR (Sec. 7 steps 4-6).
 *
 * Conventions for every entry point
 *   - Matrix and field arrays are DEVICE pointers; descriptors and option
 *     structs are host memory.  Real matrices are N*N doubles; complex
 *     matrices are N*N interleaved {re, im} doubles; all row-major.
 *   - phi is N_t*N doubles, row t-1 holding phi_t (B_1, row 0, acts first).
 *   - logdet is 2 doubles {Re, Im}, Im wrapped into (-pi, pi].
 *   - The caller owns every buffer, including the workspace, whose size comes
 *     from fd_workspace_bytes for the same problems, options and `what`.  The
 *     library never frees caller memory and allocates no device memory in
 *     these calls.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  The return code reports argument and launch errors found
 *     before or while enqueueing.  Numerical outcomes are written to the
 *     device `status` word(s) (one int32 per problem): FD_OK,
 *     FD_WARN_ILLCOND (results returned, M nearly singular),
 *     FD_ERR_SINGULAR (a pivot of the close was zero or non-finite),
 *     FD_ERR_NONFINITE (non-finite input or intermediate).
 *   - Thread-safe; calls on different streams must use different workspaces.
 */
#ifndef FDET_H
#define FDET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FD_MAX_N 512          /* largest supported number of sites            */

/* return and status codes */
enum {
  FD_OK = 0,
  FD_WARN_ILLCOND = 1,
  FD_ERR_INVALID_ARG = -1,
  FD_ERR_WORKSPACE = -2,
  FD_ERR_SINGULAR = -3,
  FD_ERR_NONFINITE = -4,
  FD_ERR_HIP = -5,
  FD_ERR_UNSUPPORTED = -6
};

/* what a workspace is sized for */
enum { FD_WHAT_LOGDET = 0, FD_WHAT_GREENS = 1, FD_WHAT_FORCE = 2, FD_WHAT_UDV = 3,
       FD_WHAT_HMC = 4 };

/* option flags */
#define FD_REUSE_E 0x1   /* exp(+-dk K) already in this workspace from an earlier
                            call on the same problems: skip recomputing it     */
#define FD_SINGLE_LAUNCH 0x4 /* the whole call as one persistent launch whose
                            workgroups claim work items in a precomputed order
                            and wait on per-item completion flags, instead of
                            one launch per phase.  Currently switched off: every
                            call with this flag returns FD_ERR_UNSUPPORTED (one
                            run did not finish; its cause is not known)        */
#define FD_KEEP_CHECKPOINTS 0x8 /* log det / G leave the UDV checkpoints (the
                            products of every checkpoint interval and the
                            prefix / suffix or window products built from
                            them) in the workspace, which is then sized and
                            laid out as for FD_WHAT_FORCE; fd_force with this
                            flag on the same problems, options and workspace
                            runs only the checkpoint items on them: G~ at each
                            checkpoint and the carried slices (the autograd
                            forward / backward pair).  Nothing may use the
                            workspace in between.  segments are not used (the
                            checkpoint intervals take their place); not for
                            fd_udv.                                            */
#define FD_FORCE_SCANS 0x2 /* force: build the checkpoint products by prefix /
                            suffix scans even where cyclic windows would take
                            fewer rounds (fd_force)                           */

typedef struct {
  int32_t N;            /* sites V, 1 <= N <= FD_MAX_N                        */
  int32_t Nt;           /* time slices, >= 1                                   */
  double dk;            /* delta * kappa: the exponent of a slice is dk*K      */
  const double *K;      /* device, N*N real symmetric hopping matrix           */
  const double *phi;    /* device, Nt*N auxiliary field                        */
} fd_problem;

typedef struct {
  int32_t s;            /* QR every s slices (Sec. 9 sporadic stabilisation);
                           0 = the tuned value for this shape (fd_autotune),
                           else 8.  Keep s*dk*spectral_radius(K) <= 6.         */
  int32_t checkpoint;   /* force: UDV checkpoint interval c (0 = 16).  G~ is
                           carried across c slices, which amplifies rounding
                           like cond(B)^c: keep c*dk*spectral_radius(K) <= 6. */
  int32_t segments;     /* det/G: independent time segments per problem that
                           are combined by stabilised products.  0 = the tuned
                           value for this shape; else, for one problem, a
                           power of two near Nt/8 (at most 32), and for a
                           batch, per problem in proportion to its chain work
                           max(N,32)^2 Nt, so that the batch's chains fill the
                           compute units about once (at most min(32, Nt/4))  */
  int32_t flags;        /* FD_REUSE_E | FD_FORCE_SCANS | FD_KEEP_CHECKPOINTS
                           (FD_SINGLE_LAUNCH: switched off)                    */
} fd_options;

/* Bytes of workspace needed for `nprob` problems and the given entry point
 * (`what` = FD_WHAT_*).  Returns 0 on invalid arguments (see fd_last_error).
 * The workspace must be 256-byte aligned.                                    */
size_t fd_workspace_bytes(const fd_problem *p, int32_t nprob, const fd_options *o,
                          int32_t what);

/* E = exp(dk K) (Sec. 6 steps 1-2; Sec. 8 notes that a truncated polynomial
 * serves equally).  E is N*N row-major real; ws as for FD_WHAT_LOGDET.       */
int fd_slice_exponential(const fd_problem *p, double *E, void *ws, size_t ws_bytes,
                         void *stream);

/* log det M (Sec. 7 steps 1-5).  logdet: device, 2 doubles.                  */
int fd_logdet(const fd_problem *p, const fd_options *o, double *logdet, void *ws,
              size_t ws_bytes, int32_t *status, void *stream);

/* log det M and G = M^{-1} (Sec. 7 steps 1-6).  logdet may be NULL.
 * G: device, N*N complex (interleaved), row-major.                           */
int fd_greens(const fd_problem *p, const fd_options *o, double *logdet, double *G,
              void *ws, size_t ws_bytes, int32_t *status, void *stream);

/* Force F_{t,x} = d log det M / d phi_{t,x} = i (1 - G~_t)_{xx} with
 * G~_t = (1 + B_{t-1}...B_1 B_{N_t}...B_t)^{-1} (Sec. 4 response formula;
 * phi_{t,x} enters only the right-most factor of B_t, so the derivative is
 * exact).  The G~_t come from UDV checkpoints every c slices of the prefix and
 * suffix products (Sec. 5, stabilised dense pre- and suffix) and are carried
 * between checkpoints by G~_{t+1} = B_t G~_t B_t^{-1}.  The checkpoint
 * intervals (nc = ceil(N_t/c)) are multiplied out in parallel; the two
 * factors of each checkpoint's cyclic product then follow from rounds of
 * stabilised products (eq. prod_2_mat_stab is associative up to rounding):
 * either cyclic windows of P and nc - P consecutive intervals (P the smallest
 * power of two with 2P >= nc; log2(P) rounds of nc products) or prefix and
 * suffix scans (grouped, about 2 nc products per direction), whichever takes
 * fewer rounds of one workgroup per compute unit for the whole call
 * (FD_FORCE_SCANS: scans).  Checkpoint 0 gives log det M and G.
 * force: device, Nt*N doubles, Re F (row t-1 = slice t).
 * force_im: NULL or Nt*N doubles, Im F.  logdet: NULL or 2 doubles.          */
int fd_force(const fd_problem *p, const fd_options *o, double *logdet, double *force,
             double *force_im, void *ws, size_t ws_bytes, int32_t *status, void *stream);

/* The stabilised factorisation B_{N_t}...B_1 = X diag(D) T (eq.
 * def_matrix_as_product with T = Y^{-1}): X unitary, D >= 0 in decreasing
 * order up to the conditioning of one stabilisation interval (the pivot order
 * of each QR is refreshed every 16 columns), |det T| = 1.  X, T: N*N complex row-major;
 * D: N doubles.                                                              */
int fd_udv(const fd_problem *p, const fd_options *o, double *X, double *D, double *T,
           void *ws, size_t ws_bytes, int32_t *status, void *stream);

/* Time-displaced Green's functions G(t, t0) = block (t, t0) of the inverse of
 * the (N N_t)^2 block fermion matrix (Sec. 4, matrix element derivatives,
 * eq. sausage_all_in_denominator), 1-based slice labels t, t0 in [1, N_t],
 * G(1, 1) = G = M^{-1}.  For each pair, P = the slices from t up to t0 - 1
 * (cyclically; all of them when t = t0) and Q = the remaining ones; then
 * G(t, t0) = (P + Q^{-1})^{-1} for t >= t0 and -(P + Q^{-1})^{-1} for t < t0,
 * evaluated without forming either product: P and Q^{-H} (the slices
 * exp(-dk K) diag(e^{i phi_t})) as stabilised UDV chains (QR every s
 * slices), and P + Q^{-1} = Xp [Dp (Tp Xq) + (Xp^H Tq^H) Dq] Xq^H inverted
 * through one pivoted QR of its scale-split bracket (Sec. 7 steps 7-9).
 * t, t0: host arrays of npairs int32.  G: device, npairs N*N complex
 * (interleaved, row-major), pair k at offset 2*N*N*k doubles.  Workspace from
 * fd_displaced_workspace_bytes (0 on invalid arguments).  One problem;
 * options: s and FD_REUSE_E.                                               */
size_t fd_displaced_workspace_bytes(const fd_problem *p, const fd_options *o, int32_t npairs);
int fd_greens_displaced(const fd_problem *p, const fd_options *o, int32_t npairs,
                        const int32_t *t, const int32_t *t0, double *G, void *ws,
                        size_t ws_bytes, int32_t *status, void *stream);

/* Batched forms: `p` is a host array of nprob descriptors (sizes may differ).
 * logdet: 2*nprob doubles.  G: one device buffer, problem i at offset
 * 2*sum_{j<i} N_j^2 doubles.  force / force_im: problem i at offset
 * sum_{j<i} Nt_j*N_j doubles.  status: nprob int32.  All problems run in the
 * same kernel launches.                                                      */
int fd_logdet_batched(const fd_problem *p, int32_t nprob, const fd_options *o,
                      double *logdet, void *ws, size_t ws_bytes, int32_t *status,
                      void *stream);
int fd_greens_batched(const fd_problem *p, int32_t nprob, const fd_options *o,
                      double *logdet, double *G, void *ws, size_t ws_bytes,
                      int32_t *status, void *stream);
int fd_force_batched(const fd_problem *p, int32_t nprob, const fd_options *o,
                     double *logdet, double *force, double *force_im, void *ws,
                     size_t ws_bytes, int32_t *status, void *stream);

/* Prepared calls.  A plan fixes one call of kind `what` (FD_WHAT_LOGDET,
 * FD_WHAT_GREENS or FD_WHAT_FORCE) on fixed problems, outputs and workspace,
 * and uploads its work descriptors into the head of the workspace once
 * (synchronously on `stream`; not allowed while `stream` is capturing).
 * fd_plan_launch then only enqueues kernels (no copies, no fills), so it may
 * be captured into a HIP graph and replayed; it reads K and phi at launch
 * time, so the caller updates phi in place between launches (the molecular
 * dynamics steps of HMC, Sec. 3.1).  Outputs as for the matching entry
 * point; force is ignored unless what = FD_WHAT_FORCE and may then be NULL.
 * With FD_WHAT_FORCE, a non-NULL G (layout as for fd_greens_batched)
 * receives G = M^{-1} = G~_1, which the force computes at its first
 * checkpoint anyway; FD_WHAT_LOGDET ignores G.
 * The workspace must not be used by any other call while the plan is alive;
 * with FD_REUSE_E, exp(+-dk K) must already be in it from a call of the same
 * kind and options.  fd_plan_destroy frees host memory only.               */
typedef struct fd_plan fd_plan;
int fd_plan_create(int32_t what, const fd_problem *p, int32_t nprob, const fd_options *o,
                   double *logdet, double *G, double *force, double *force_im, void *ws,
                   size_t ws_bytes, int32_t *status, void *stream, fd_plan **plan);
int fd_plan_launch(const fd_plan *plan, void *stream);
void fd_plan_destroy(fd_plan *plan);
/* Work units a plan gave each problem: for FD_WHAT_LOGDET / _GREENS the time
 * segments (independent slice ranges combined by stabilised products), for
 * FD_WHAT_FORCE the checkpoint intervals.  Writes min(n, nprob) int32 to the
 * host array seg (may be NULL) and returns nprob, or FD_ERR_INVALID_ARG for a
 * NULL plan.  A single call with options.segments set to a problem's value
 * repeats that problem's part of a batched plan work item for work item.    */
int fd_plan_segments(const fd_plan *plan, int32_t *seg, int32_t n);

/* fd_greens without a caller workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a fixed array of
 * FD_NOALLOC_MAX_BYTES inside the library, one per GPU, held until the
 * process ends; the call allocates nothing (no hipMalloc / hipFree).  Same
 * arguments and results as fd_greens for one problem, bit for bit, on the
 * same options.  FD_ERR_WORKSPACE if the call would need more than the
 * fixed size (fd_workspace_bytes with FD_WHAT_GREENS; fewer segments need
 * less).  All calls on one GPU share its array: calls that overlap in time
 * on one GPU (other streams, other threads) race and must be serialised by
 * the caller.                                                              */
#define FD_NOALLOC_MAX_BYTES (64u << 20)
int fd_greens_noalloc(const fd_problem *p, const fd_options *o, double *logdet, double *G,
                      int32_t *status, void *stream);

/* Autotuning of the stabilisation interval s (Sec. 9 leaves its choice to
 * the conditioning: candidates 4, 8, 16 within s*dk*radius(K) <= 6, radius
 * bounded by the largest absolute row sum of K) and of the time segments
 * (1, 2, 4, ..., 64) for these problems and `what` (LOGDET, GREENS or FORCE;
 * FORCE tunes s only).  Fields of `o` that are nonzero are kept fixed.  Each
 * candidate runs once untimed and three times timed on `stream`; the median
 * decides, candidates whose status is an error are skipped.  The winner is
 * stored in the process-wide table that fields left at 0 consult (key: what,
 * largest N, largest Nt, nprob, dk) and returned in *best / *best_ms (either
 * may be NULL).  Synchronous; allocates and frees its own device memory, so
 * it is a set-up call, never one for graph capture.
 * fd_tune_save / fd_tune_load write / merge the table as text ("fdet-tune 1"
 * and one line per entry); load returns the number of entries read or an
 * error code.  fd_tune_clear empties the table.                             */
int fd_autotune(int32_t what, const fd_problem *p, int32_t nprob, const fd_options *o,
                void *stream, fd_options *best, float *best_ms);
int fd_tune_save(const char *path);
int fd_tune_load(const char *path);
int fd_tune_clear(void);

/* Molecular dynamics of HMC (Sec. 3.1): one leapfrog trajectory of `nsteps`
 * steps of size `eps` for each of `nprob` fields, with unit-mass momenta,
 * two fermion flavours whose determinants are complex conjugates and the
 * Gaussian weight of the auxiliary field:
 *     H = 1/2 sum pi^2 + sum phi^2 / (2 dU) - 2 Re log det M(phi),
 *     dH/dphi_{t,x} = phi_{t,x} / dU - 2 Re F_{t,x}   (F as for fd_force).
 * Half kick, then nsteps x (drift, force, kick), the last kick a half one:
 * nsteps + 1 force evaluations, each a prepared fd_force call.
 *   p[i].phi  device, N_t*N: advanced IN PLACE to the end of the trajectory
 *   pi        device, momenta of every field, concatenated in the layout of
 *             fd_force_batched's force (the caller draws them); advanced in place
 *   dH        device, nprob doubles: H at the end minus H at the start (the
 *             caller accepts with probability min(1, exp(-dH)) and otherwise
 *             restores its copy of phi)
 *   dU        delta * U > 0, the variance of the auxiliary field's weight
 *   ws        fd_workspace_bytes(p, nprob, o, FD_WHAT_HMC) bytes, 256-aligned
 *   status    device, nprob int32: the worst status of all force evaluations
 * o as for fd_force (FD_REUSE_E is ignored: the first evaluation computes
 * exp(+-dk K), the rest reuse it).  Prepares plans (a synchronous descriptor
 * upload), so it is not for stream capture; FD_ERR_INVALID_ARG for bad
 * arguments, FD_ERR_WORKSPACE for a short workspace, FD_ERR_HIP on launch
 * errors.                                                                   */
int fd_hmc_leapfrog(const fd_problem *p, int32_t nprob, const fd_options *o, double dU, double eps,
                    int32_t nsteps, double *pi, double *dH, void *ws, size_t ws_bytes,
                    int32_t *status, void *stream);

/* A prepared trajectory: fd_hmc_leapfrog's arguments fixed once.  Creation
 * (outside stream capture, synchronous) uploads the field descriptors and
 * runs one full force call so that exp(+-dk K) sits in the workspace; K and
 * dk must then stay fixed.  fd_hmc_plan_launch enqueues kernels only (every
 * force evaluation of the trajectory reuses the exponential), so it may be
 * captured into a HIP graph and replayed; it reads phi and pi at launch time
 * and advances both in place, as fd_hmc_leapfrog does, with the same
 * results.  The workspace (FD_WHAT_HMC size) belongs to the plan while it
 * lives.  fd_hmc_plan_destroy frees host memory only.                      */
typedef struct fd_hmc_plan fd_hmc_plan;
int fd_hmc_plan_create(const fd_problem *p, int32_t nprob, const fd_options *o, double dU,
                       double eps, int32_t nsteps, double *pi, double *dH, void *ws,
                       size_t ws_bytes, int32_t *status, void *stream, fd_hmc_plan **plan);
int fd_hmc_plan_launch(const fd_hmc_plan *plan, void *stream);
void fd_hmc_plan_destroy(fd_hmc_plan *plan);

/* Equal-time response trace (Sec. 4, shortcut for simple operators): the
 * expectation value of an operator A from one Green's function G = M^{-1},
 *     out = tr((1 - G) A) = tr A - sum_ij G_ij A_ji,
 * the trace of A against M^{-1} P at the slice where the partial products of
 * the response formula are empty.  A == NULL stands for A = 1 / N, giving the
 * fermion number n = 1 - tr G / N (eq. fermion_number).
 *   G    device, N*N complex (interleaved, row-major, as fd_greens writes it)
 *   A    device, N*N complex in the same layout, or NULL
 *   out  device, 2 doubles {Re, Im}
 *   ws   device workspace of fd_response_trace_workspace_bytes(N) bytes,
 *        256-byte aligned (per-tile partial sums)
 * 1 <= N <= FD_MAX_N.  Asynchronous on `stream`; the result does not depend
 * on scheduling (partials are added in a fixed order).  Returns
 * FD_ERR_INVALID_ARG for a bad N or a NULL G / out, FD_ERR_WORKSPACE for a
 * missing, misaligned or short workspace, FD_ERR_HIP for a launch error.
 * fd_response_trace_workspace_bytes returns 0 for a bad N.                   */
size_t fd_response_trace_workspace_bytes(int32_t N);
int fd_response_trace(int32_t N, const double *G, const double *A, double *out, void *ws,
                      size_t ws_bytes, void *stream);

/* Average over all slices of the response to a diagonal operator diag(a)
 * (the shortcut of Sec. 4 summed over every slice, which for a
 * non-constant a differs from the single-slice trace above):
 *     out = (1 / N_t) sum_t sum_x a_x (1 - G~_t)_xx,
 * read off the force sweep's output, (1 - G~_t)_xx = Im F_{t,x} - i Re F_{t,x}.
 *   force, force_im  device, N_t*N: Re F and Im F as fd_force writes them
 *                    (force_im must have been requested)
 *   a                device, N doubles, or NULL for a_x = 1 / N (the
 *                    fermion number)
 *   out              device, 2 doubles {Re, Im}
 * One workgroup, fixed summation order; no workspace.  FD_ERR_INVALID_ARG
 * for bad sizes or NULL pointers, FD_ERR_HIP on a launch error.            */
int fd_diag_response(int32_t Nt, int32_t N, const double *force, const double *force_im,
                     const double *a, double *out, void *stream);

/* The force sweep with, in addition, the per-slice response to a general
 * operator A (Sec. 4, shortcut for simple operators: the trace inside
 * eq. response_simple, before its average over the slices):
 *     trace[t-1] = tr((1 - G~_t) A) = tr A - sum_xy (G~_t)_xy A_yx,
 * taken on each G~_t as the sweep forms it (checkpoints and carried rows),
 * so it costs N^2 per slice beside the 8 N^3 of each carry.  The mean of the
 * N_t traces is the slice-averaged response; A = diag(a) reproduces
 * fd_diag_response slice by slice.
 *   A      device, N*N complex (interleaved, row-major), shared by all slices
 *   trace  device, N_t complex (interleaved): row t-1 = slice t
 * The other arguments, the workspace and the options are those of fd_force
 * (FD_KEEP_CHECKPOINTS included).  Batched: A of problem i at offset
 * 2*sum_{j<i} N_j^2 doubles, trace at 2*sum_{j<i} Nt_j doubles.
 * FD_ERR_INVALID_ARG for a NULL A, trace, force or status.
 * FD_ERR_UNSUPPORTED for any problem with N > 128: the trace is switched off
 * in the blocked class (one run there returned wrong traces and the next
 * faulted; the cause is not known).                                        */
int fd_force_response(const fd_problem *p, const fd_options *o, const double *A,
                      double *trace, double *logdet, double *force, double *force_im,
                      void *ws, size_t ws_bytes, int32_t *status, void *stream);
int fd_force_response_batched(const fd_problem *p, int32_t nprob, const fd_options *o,
                              const double *A, double *trace, double *logdet, double *force,
                              double *force_im, void *ws, size_t ws_bytes, int32_t *status,
                              void *stream);

/* Intermediate volume, low temperature (Sec. 9, with the slices of Sec. 8):
 * log det and G of M~ = 1 + B~_{N_t} ... B~_1 where each slice
 * B~_t = [prod_{k=1}^{n} (1 + gamma_k dk K)] diag(e^{i phi_t}) replaces
 * exp(dk K) by its degree-n Taylor polynomial in product form (the gamma_k
 * are -1 / the roots of that polynomial, computed by the library) and is
 * never formed: every slice is applied to the stabilised product's unitary
 * factor as a field phase and n stencil steps x <- x + gamma_k dk K x over
 * the nonzeros of K, and the product is re-decomposed by a pivoted QR every
 * s slices (the sporadic stabilisation).  The truncation changes the result
 * at O((dk |K|)^{n+1}) per slice: this is a different slice matrix from the
 * exact one of fd_greens, not an approximation of its output.
 * K by its nonzeros (ELL form): row i has q entries, neighbours col[i*q + j]
 * in [0, N) with weights val[i*q + j]; pad short rows with weight 0.        */
typedef struct {
  int32_t q;            /* entries per row, 1 <= q <= 64                      */
  const int32_t *col;   /* device, N*q                                         */
  const double *val;    /* device, N*q                                         */
} fd_ell;
/* fd_problem.K is not read (may be NULL).  taylor_n in [1, 8] (the paper
 * takes 4).  Options: s <= 16 and segments as for fd_greens; no flags.
 * G == NULL: log det only.  Batched: hop and p are host arrays of nprob
 * entries; outputs laid out as for fd_greens_batched.  Workspace from
 * fd_sparse_workspace_bytes (what = FD_WHAT_LOGDET or FD_WHAT_GREENS; 0 on
 * invalid arguments).                                                       */
size_t fd_sparse_workspace_bytes(const fd_problem *p, int32_t nprob, const fd_options *o,
                                 int32_t what);
int fd_sparse_greens(const fd_problem *p, const fd_ell *hop, int32_t taylor_n,
                     const fd_options *o, double *logdet, double *G, void *ws, size_t ws_bytes,
                     int32_t *status, void *stream);
int fd_sparse_greens_batched(const fd_problem *p, int32_t nprob, const fd_ell *hop,
                             int32_t taylor_n, const fd_options *o, double *logdet, double *G,
                             void *ws, size_t ws_bytes, int32_t *status, void *stream);

/* Text for a return/status code; the last error message of this thread.      */
const char *fd_strerror(int code);
const char *fd_last_error(void);
/* Library version string: "fdet <version> (gfx950) src <digest>", the digest
 * being the first 16 hex digits of a sha256 over the library's source files
 * (the binding compares it with the sources it ships beside).               */
const char *fd_version(void);

/* Diagnostics: after fd_profile_start, every kernel phase launched by this
 * thread is bracketed by HIP events recorded on the call's stream.
 * fd_profile_stop waits for those events, writes up to `max` records (phase
 * kind: 0 exponential, 1 chain, 2 combine, 3 close, 4 force, 5 export, -1 a
 * single launch of a whole call (see FD_SINGLE_LAUNCH); work
 * items in the launch; milliseconds) and returns the number of phases seen.
 * Any output pointer may be NULL.                                            */
int fd_profile_start(void);
int fd_profile_stop(int32_t max, int32_t *kinds, int32_t *nitems, float *ms);

#ifdef __cplusplus
}
#endif
#endif /* FDET_H */
