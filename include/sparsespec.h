/*
 * sparsespec -- sparse spectral Galerkin solver for -div(a grad u) = f on the
 * d-torus, MI355X (gfx950) native.  C ABI.
 *
 * Mathematical objects (Gross & Iwen, "Sparse spectral methods for solving
 * high-dimensional and multiscale elliptic PDEs"):
 *   - Fourier convention e_k(x) = exp(2 pi i k.x), u_k = <u, e_k> (Sec. 3).
 *   - Stamping set S^N[a](F): S^0 = F, S^n = S^{n-1} + supp(a), Minkowski sum
 *     (Sec. 6, Eq. StampSet).  The level of k is the first n with k in S^n.
 *   - Truncated Galerkin operator (Sec. 9, Eq. FiniteGalerkinOperator):
 *       (L_N u)_k = sum_{l in S^N} 4 pi^2 (l . k) a_{k-l} u_l,   k in S^N.
 *   - The solve replaces the dense direct solve of Alg. 1 (step 5) by
 *     Jacobi-preconditioned conjugate gradients; the Jacobi diagonal
 *     4 pi^2 |k|^2 a_0 is the denominator of the recurrence in the proof of
 *     Prop. SolutionSupport.  The solution is the unique mean-zero one
 *     (u_0 = 0; Prop. ExistenceUniquenessStability needs f_0 = 0).
 *
 * Conventions for every call:
 *   - Every function returns ss_status and never aborts.  ss_last_error()
 *     returns a thread-local description of the last failure.
 *   - Frequencies are int16, row-major [count x d].  Complex numbers are
 *     interleaved (re, im) doubles (complex128) or floats (complex64).
 *   - "host" pointers are borrowed for the duration of the call only.
 *     "device" pointers are caller-owned device memory (e.g. a torch
 *     tensor's data_ptr()) on the current HIP device.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls that return
 *     host data synchronise that stream; calls that only write device data
 *     are asynchronous on it.
 *   - Handles are not thread-safe; distinct handles may be used from
 *     distinct threads.
 *   - Slot order: the keys of one problem are numbered in ascending
 *     lexicographic order of their signed coordinates, coordinate 0 most
 *     significant ("canonical order").  A batch numbers problem after
 *     problem.
 *   - Limits: 1 <= d <= 1024; |supp a| (after closing under negation) <= 127;
 *     every key coordinate must fit int16 (else SS_ERANGE); at most 16383
 *     problems per batch and 4194303 keys per problem.
 */
#ifndef SPARSESPEC_H
#define SPARSESPEC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SS_OK = 0,
  SS_EINVAL = 1,      /* malformed argument (shape, duplicate, non-conjugate pair, f_0 != 0, ...) */
  SS_ENOMEM = 2,      /* device or host allocation failed                              */
  SS_ERANGE = 3,      /* a key coordinate leaves int16, or a size limit is exceeded    */
  SS_ENOTPD = 4,      /* l1 positivity certificate a_0 > sum_{w != 0} |a_w| failed      */
  SS_ENOCONV = 5,     /* iteration limit reached; best iterate returned, info filled   */
  SS_EBREAKDOWN = 6,  /* <p, L p> <= 0 or not finite during CG                        */
  SS_EDEVICE = 7      /* a HIP runtime call failed                                    */
} ss_status;

typedef enum { SS_FP64 = 0, SS_FP32_REFINE = 1 } ss_precision;

/* ss_build_op flags */
#define SS_SKIP_L1_CHECK 1u   /* accept a whose l1 certificate fails (e.g. product coefficients) */
#define SS_EXACT_LOOKUP 2u    /* neighbour lookups compare keys, not rank-1 lattice values (see ss_build_op) */

typedef struct ss_stamp ss_stamp;  /* device-resident stamping sets of a batch of problems       */
typedef struct ss_op ss_op;        /* device-resident operator(s) L_N built on an ss_stamp        */
typedef struct ss_batch ss_batch;  /* device-resident solutions of a batch solve                  */

typedef struct {
  int32_t iters;          /* CG iterations (summed over refinement steps for FP32_REFINE)     */
  int32_t outer_steps;    /* refinement steps (FP32_REFINE), else 0                           */
  double rel_residual;    /* |f - L_N u|_2 / |f|_2 in FP64 at return                           */
  int64_t n;              /* |S^N|                                                             */
  int64_t nnz;            /* stored neighbour pairs (k, k - w) with both in S^N                */
  int32_t n_components;   /* independent classes (Sec. 6, proof of Prop. SolutionSupport)      */
  int32_t status;         /* ss_status of this problem                                         */
  double t_build_ms;      /* wall time of stamp + operator build (ss_solve only)               */
  double t_solve_ms;      /* wall time of the iteration                                        */
} ss_solve_info;

/* ---------------------------------------------------------------- stamp sets
 * ss_build_stamp_batch -- build S^{level[p]}[a_p](F_p) for n_prob problems of
 * the same dimension d (Sec. 6, Eq. StampSet; Alg. 1, step 3).
 *   n_a[p], a_freqs: supp(a_p) as n_a[p] frequencies, all problems
 *     concatenated (host).  A half list is completed by negation; 0 must be
 *     present.  Duplicates -> SS_EINVAL.
 *   n_f[p], f_freqs: F_p = supp(f_p), concatenated (host).  Duplicates within
 *     a problem -> SS_EINVAL.
 *   level[p] >= 0: the stamping level N (host).
 * On success *out owns the keys (canonical order), their levels, |k|^2 and a
 * device hash index; free with ss_free_stamp.
 */
ss_status ss_build_stamp_batch(int32_t n_prob, int32_t d, const int32_t* n_a,
                               const int16_t* a_freqs, const int32_t* n_f,
                               const int16_t* f_freqs, const int32_t* level,
                               void* stream, ss_stamp** out);

/* single-problem form of ss_build_stamp_batch */
ss_status ss_build_stamp(int32_t d, int32_t n_a, const int16_t* a_freqs, int32_t n_f,
                         const int16_t* f_freqs, int32_t level, void* stream,
                         ss_stamp** out);

/* total keys and number of problems; offsets (host, n_prob+1 entries,
 * nullable) receive each problem's first canonical slot. */
ss_status ss_stamp_size(const ss_stamp* st, int64_t* n_total, int32_t* n_prob,
                        int64_t* offsets);

/* copy keys [n_total x d] int16 (host, canonical order) and levels (host,
 * nullable) out.  Synchronises. */
ss_status ss_stamp_keys(const ss_stamp* st, int16_t* keys_out, uint8_t* level_out);

/* hash lookup of nq query keys [nq x d] (host) of problem `prob`: slot_out[i]
 * (host) = canonical slot within that problem, or -1 if absent.  Synchronises. */
ss_status ss_stamp_lookup(const ss_stamp* st, int32_t prob, int64_t nq,
                          const int16_t* q, int64_t* slot_out);

/* batched form: query i belongs to problem prob[i] (host); slot_out[i] (host)
 * = global canonical slot (problem offset included), or -1.  Synchronises. */
ss_status ss_stamp_lookup_batch(const ss_stamp* st, int64_t nq, const int32_t* prob,
                                const int16_t* q, int64_t* slot_out);

/* the right-hand side of the Galerkin system (Sec. 9, Eq. FiniteGalerkinOperator
 * applied to u_N = f restricted to S^N; Alg. 1, step 4): f (device, complex128,
 * n_total entries, canonical order) is set to f_hat[i] at the slot of the i-th
 * forcing frequency given to the build and to 0 elsewhere.  f_hat (host,
 * complex128) lists one coefficient per forcing frequency, in the order they
 * were given (all problems concatenated).  F_p is contained in S^N, so every
 * coefficient has a slot.  Synchronises `stream`. */
ss_status ss_stamp_forcing(const ss_stamp* st, const double* f_hat, void* f, void* stream);

/* ---------------------------------------------------------------- rank-1 lattices
 * Random rank-1 lattices Lambda(z, M) on the stamping sets (Sec. 8, Definition of a
 * reconstructing rank-1 lattice, Lemma RandomRank1Lattice).  The lattice gives frequency k
 * the index k . z mod M; it reconstructs a set when distinct frequencies get distinct indices.
 *
 * ss_lattice_modulus -- the Lemma's modulus: *M (host) = the smallest prime greater than
 *   max(expansion, n^2 / sigma), where expansion is K of the Lemma (side of the smallest cube
 *   holding the set) and n the set's size; a z drawn uniformly from {1..M-1}^d then
 *   reconstructs the set with probability at least 1 - sigma.  The threshold is formed in
 *   double precision.  sigma outside (0, 1] or negative sizes -> SS_EINVAL; a modulus above
 *   2^40 -> SS_ERANGE.  Host only, no device work.
 */
ss_status ss_lattice_modulus(int64_t expansion, int64_t n, double sigma, int64_t* M);

/* ss_stamp_lattice -- lattice indices of every key of st and, per problem, whether the
 * lattice reconstructs that problem's stamping set.
 *   z: d generating-vector entries (host, borrowed for the call), each in [1, M-1].
 *   M: the lattice size, 2 <= M <= 2^40 (need not be prime).
 *   values: device, int64 [n_total] in canonical order, receives k . z mod M in [0, M);
 *     nullable (only the check).
 *   reconstructing: host, int32 [n_prob]: 1 if the indices of the problem's keys are distinct.
 * Argument errors -> SS_EINVAL (nothing written).  Synchronises `stream`.
 */
ss_status ss_stamp_lattice(const ss_stamp* st, const int64_t* z, int64_t M, void* values,
                           int32_t* reconstructing, void* stream);

void ss_free_stamp(ss_stamp* st);

/* ---------------------------------------------------------------- operator
 * ss_build_op -- the truncated Galerkin operator L_N on every problem of st
 * (Sec. 9, Eq. FiniteGalerkinOperator; replaces the dense assembly of Alg. 1,
 * step 4 by a matrix-free neighbour map).
 *   n_a, a_freqs, a_hat: the diffusion coefficients, concatenated per
 *     problem (host; a_hat interleaved complex128).  After completing -w by
 *     conjugation the support must equal the one st was built with.  Present
 *     +-w pairs must be conjugate to 1e-14 max|a| (else SS_EINVAL); a_0 must
 *     be real and positive; unless SS_SKIP_L1_CHECK, a_0 > sum_{w!=0} |a_w|
 *     (the positivity check after Cor. SpectralConvergenceNoSFT) else SS_ENOTPD.
 * The operator copies what it needs; st may be freed afterwards.
 */
ss_status ss_build_op(const ss_stamp* st, const int32_t* n_a, const int16_t* a_freqs,
                      const double* a_hat, uint32_t flags, void* stream, ss_op** out);
/* Neighbour lookups.  By default the map finds l = k - w_j in S^N by the rank-1 lattice value
 * lat(k) = k . z mod M (Sec. 8, Definition of a reconstructing rank-1 lattice; M = 2^61 - 1 prime,
 * z drawn once from [1, M - 1]^d by a fixed seeded generator): the map is linear, so
 * lat(k - w_j) = lat(k) - lat(w_j) mod M comes from two stored values, and a hash-table slot whose
 * 31-bit fingerprint matches is accepted when its key's stored lattice value equals it -- no key
 * (2d bytes) is read.  The result is exact whenever the lattice separates S^N from the looked-up
 * differences (the reconstructing property of Lemma RandomRank1Lattice on that set); a false
 * match needs a distinct key with the same fingerprint and the same lattice value, probability at
 * most 1/M per compared pair over z, below |S^N|^2 s / M (about 1e-8 at |S| = 3e4, s = 21) per
 * problem even ignoring the fingerprint.  SS_EXACT_LOOKUP confirms every match by comparing the
 * keys instead (deterministic, slower for large d). */

/* sizes: n_total keys, n_exec rows of the execution layout (>= n_total), nnz,
 * number of independent classes summed over problems (all nullable). */
ss_status ss_op_info(const ss_op* op, int64_t* n_total, int64_t* n_exec, int64_t* nnz,
                     int64_t* n_components);

/* canonical neighbour map (host outputs, synchronises): row_ptr [n_total+1]
 * (global offsets), cols [nnz] (canonical slot within the row's problem),
 * js [nnz] (index into the problem's lexicographically sorted a-table),
 * component [n_total] (smallest canonical slot of the row's class; nullable). */
ss_status ss_op_csr(const ss_op* op, int64_t* row_ptr, int32_t* cols, int32_t* js,
                    int32_t* component);

/* execution order (host output, synchronises): exec_to_canon[e] for
 * e < n_exec is the global canonical slot held in execution row e, or -1 for a
 * padding row.  Execution order groups rows by problem, then by class. */
ss_status ss_op_exec_map(const ss_op* op, int64_t* exec_to_canon);

/* y = L_N x for every problem at once (Sec. 9, Eq. FiniteGalerkinOperator).
 * x_dev, y_dev: device vectors of n_exec entries in execution order,
 * complex128 for SS_FP64 and complex64 for SS_FP32_REFINE (which applies the
 * FP32 operator).  Padding entries of y are written as 0.  Asynchronous. */
ss_status ss_apply(const ss_op* op, ss_precision prec, const void* x_dev, void* y_dev,
                   void* stream);

/* Solve L_N u = f for every problem of op (Alg. 1, step 5, by PCG).
 *   f_dev: device, n_total complex128 in canonical order; f at k = 0 must be 0.
 *   u_dev: device, n_total complex128 in canonical order; in: initial guess
 *          (zeros for none); out: solution with u_0 = 0.
 *   tol:   stop when |f - L_N u|_2 <= tol |f|_2 per problem (FP64 residual).
 *   prec:  SS_FP64 -- FP64 PCG;  SS_FP32_REFINE -- FP32 PCG inside FP64
 *          iterative refinement (residual and update in FP64).
 *   max_iter: CG iteration limit per problem (per refinement step for FP32).
 *   info:  host, n_prob entries (nullable).
 * Returns SS_ENOCONV if any problem missed tol (u holds its last iterate).
 * Synchronises the stream. */
ss_status ss_solve_op(const ss_op* op, const void* f_dev, void* u_dev, double tol,
                      ss_precision prec, int32_t max_iter, void* stream,
                      ss_solve_info* info);

/* ss_solve_op_noalloc -- ss_solve_op for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It allocates no device
 * or pinned host memory: the class-resident CG's tables (problem descriptors, unit lists) and its
 * per-unit results live in one fixed device array of SS_NOALLOC_SCRATCH_BYTES per GPU, held by
 * the library until the process ends.
 *   Arguments, layouts, tolerance, precision, result and info: as for ss_solve_op (the results
 *   are bitwise those of ss_solve_op on the same operator).
 *   Only operators whose every class has at most 2048 rows are served (their problems run the
 *   class-resident CG); a larger class needs ss_solve_op's per-problem workspace -> SS_EINVAL.
 *   The tables take about 100 bytes per problem and 60 per solve unit (a run of whole classes of
 *   at most 2048 rows); more than SS_NOALLOC_SCRATCH_BYTES in all -> SS_ERANGE, nothing launched.
 *   An operator built on another device -> SS_EINVAL.
 * Calls that overlap on one GPU share its array and race: serialise them.  Synchronises `stream`. */
#define SS_NOALLOC_SCRATCH_BYTES (2u << 20)
ss_status ss_solve_op_noalloc(const ss_op* op, const void* f_dev, void* u_dev, double tol,
                              ss_precision prec, int32_t max_iter, void* stream, ss_solve_info* info);

/* Exact proxy error of Sec. 10.1 (Lemma ProxyError) for every problem of a batch:
 * err_out[p] = |f - L u^N|_2 / |f|_2 with L the untruncated operator, u^N the
 * level-N solution extended by zero.  L u^N is supported on S^{N+1} (Prop.
 * LExpansion), so the norm is taken exactly there, by one FP64 matvec of the
 * level-(N+1) operator.
 *   st_next, op_next: stamping sets and operator built on the same problems
 *          (same a, same F in the same order) at level N_p + 1 each; every
 *          level must be >= 1.  Their keys of first-appearance level <= N_p
 *          are S^{N_p}, in the same canonical order.
 *   u_dev, n_u: device complex128, the level-N solutions in the canonical order
 *          of the level-N stamp (n_u = sum over p of |S^{N_p}| entries; read
 *          only).
 *   f_hat: host complex128 forcing coefficients, as for ss_stamp_forcing.
 *   err_out: host double [n_prob]; 0 for a problem with f = 0.
 * Errors: SS_EINVAL (null argument, op_next not built on st_next, a level 0,
 * n_u not the number of keys of level <= N_p).  Synchronises `stream`. */
ss_status ss_proxy_error(const ss_stamp* st_next, const ss_op* op_next, const void* u_dev,
                         int64_t n_u, const double* f_hat, double* err_out, void* stream);

/* ss_solve_direct -- the paper's own solver (Alg. 1, steps 4-5: dense assembly of L_N and a
 * direct solve), run per connected class (Sec. 6; the system is block diagonal over classes, proof
 * of Prop. SolutionSupport).  Each class block is assembled densely (entries formed in FP64) and
 * factored as L L^H (Cholesky; the block is Hermitian positive definite on k != 0 by Prop.
 * ExistenceUniquenessStability), then L y = f, L^H u = y.  The zero frequency gets u_0 = 0.
 *   prec: SS_FP64 -- factor and substitutions in FP64;  SS_FP32_REFINE -- factor and substitutions
 *         in FP32, wrapped in iterative refinement with the FP64 residual f - L u and update.
 *   tol:  > 0: refinement steps until every class has |f_c - L u_c|_2 <= tol |f_c|_2 (at most 30);
 *         <= 0: one solve, no refinement.
 *   f_dev: device, n_total complex128 in canonical order (as for ss_solve_op; f_0 is ignored).
 *   u_dev: device, n_total complex128 in canonical order; out only.
 *   info (host, nullable): factorisation time and size, steps and residual, see ss_direct_info.
 * Memory: the lower triangle of every class block, in chunks of consecutive classes of about equal
 * size and at most 16 GiB (one class per chunk at least), plus four FP64 vectors of n_exec.
 * Errors: SS_ERANGE (a class of more than 32768 rows), SS_ENOTPD (a non-positive pivot: u is then
 * not a solution), SS_ENOCONV (tol > 0 not reached), SS_ENOMEM, SS_EDEVICE.  Synchronises `stream`. */
typedef struct {
  double factor_ms;       /* device time of the factorisation kernels, summed over chunks       */
  int64_t tiles;          /* 32 x 32 complex tiles of the lower triangles factored               */
  int32_t chunks;         /* chunks the classes were factored in                                 */
  int32_t refine_steps;   /* substitution steps (1 without refinement), most over the chunks     */
  double rel_residual;    /* max over classes of |f_c - L_N u_c|_2 / |f_c|_2, in FP64            */
} ss_direct_info;
ss_status ss_solve_direct(const ss_op* op, const void* f_dev, void* u_dev, ss_precision prec, double tol,
                          void* stream, ss_direct_info* info);

/* rows of every connected class of op (Sec. 6), in execution order (problem by problem).
 *   sizes (host, nullable): cap entries; n_out: the number of classes.  cap smaller than the
 *   number of classes with sizes != NULL -> SS_EINVAL. */
ss_status ss_op_class_sizes(const ss_op* op, int64_t cap, int64_t* sizes, int64_t* n_out);

/* ---------------------------------------------------------------- advection-diffusion-reaction
 * -div(a grad u) + b . grad u + c u = f (Remark ADR, Eq. ADR).  With grad e_l = 2 pi i l e_l the
 * operator's entry at (k, l) is 4 pi^2 (k . l) a_{k-l} + 2 pi i (l . b_{k-l}) + c_{k-l}.  Build the
 * stamp and the operator with the diffusion calls on the union W = supp(a) u supp(b) u supp(c)
 * (with 0 and closed under negation): pass W as the stamp's support, and to ss_build_op W with
 * a's coefficients (0 where a has none).  One level adds W once (reading of the Remark's stamp:
 * each application of the operator shifts a frequency by one element of one support).
 *
 * ss_build_adr adds the advection and reaction terms to op (which must outlive the handle).
 *   n_b[p], b_freqs (host int16 [sum n_b x d]), b_hat (host complex128 [sum n_b x d]): for each
 *     frequency w of problem p, the d components' coefficients (b_{1,w}, ..., b_{d,w}); list w and
 *     -w (conjugate coefficients for a real field).
 *   n_c[p], c_freqs, c_hat (complex128 [sum n_c]): c the same way; c_0 must be real and positive
 *     (then the zero frequency is an ordinary unknown).
 * Errors: SS_EINVAL (a frequency outside op's support, c_0 missing or not positive, not finite).
 * Synchronises `stream`. */
typedef struct ss_adr ss_adr;
ss_status ss_build_adr(const ss_stamp* st, const ss_op* op, const int32_t* n_b, const int16_t* b_freqs,
                       const double* b_hat, const int32_t* n_c, const int16_t* c_freqs, const double* c_hat,
                       void* stream, ss_adr** out);

/* y = L x with the advection and reaction terms, FP64; x_dev, y_dev: device complex128 [n_exec]
 * in execution order (as ss_apply).  Asynchronous. */
ss_status ss_adr_apply(const ss_adr* adr, const void* x_dev, void* y_dev, void* stream);

/* Solve L u = f for every problem: Jacobi-preconditioned BiCGSTAB in FP64 (the operator is not
 * Hermitian), per-problem scalars, stop when the true residual |f - L u|_2 <= tol |f|_2 (the
 * recursively updated residual triggers the check; up to 3 restarts from the true residual).
 *   f_dev, u_dev: device complex128 [n_total], canonical order; u is out only (start from 0).
 *   max_iter: BiCGSTAB iterations (two matvecs each) over all restarts.
 *   info (host, nullable): n_prob entries.
 * Returns SS_ENOCONV / SS_EBREAKDOWN when a problem missed tol (u holds its last iterate).
 * Synchronises `stream`. */
ss_status ss_adr_solve(const ss_adr* adr, const void* f_dev, void* u_dev, double tol, int32_t max_iter,
                       void* stream, ss_solve_info* info);

void ss_free_adr(ss_adr* adr);

void ss_free_op(ss_op* op);

/* device bytes held by op, including its solver workspace once a solve ran */
ss_status ss_op_bytes(const ss_op* op, int64_t* bytes);

/* ---------------------------------------------------------------- serving engine
 * Continuous batching of solves (no passage of the paper; the request-level
 * pattern on top of Alg. 1 steps 3-5).  An engine holds a changing set of
 * admitted problems -- possibly of different operators, dimensions, sizes and
 * precisions -- and advances all of them with the same launches: each tick
 * runs the pending admissions and refinement transitions, then `iters` PCG
 * iterations over every active problem, then retires problems that
 * finished.  Per-problem reductions have a fixed order, so a problem's result
 * is bitwise the same alone and in any mix.
 *
 * ss_engine_create: hbm_budget_bytes (0 = unlimited) bounds the device bytes
 *   of admitted operators plus their solver workspaces (a request larger than
 *   the whole budget is admitted only when the engine holds no other); max_slots
 *   (0 = unlimited) bounds the admitted requests.  stream: the engine's stream.
 * ss_engine_submit: admits every problem of op as one request.  f_dev, u_dev:
 *   device complex128 vectors of op's n_total entries in canonical order
 *   (u_dev: initial guess in, solution out); op, f_dev and u_dev must stay
 *   valid until every problem of the request has been polled.  Returns
 *   SS_ENOMEM -- and admits nothing -- when the budget or the slots would be
 *   exceeded (the caller keeps the request queued), SS_EINVAL if op already
 *   has a solve in flight.
 * ss_engine_step: one tick; *n_active = problems still active.  Synchronises.
 * ss_engine_poll: moves up to cap finished problems out: tags[i] (request tag),
 *   probs[i] (problem index within the request's op), info[i].  Host arrays,
 *   each nullable except n_out.
 * ss_engine_usage: admitted requests and the bytes they hold.
 */
typedef struct ss_engine ss_engine;
ss_status ss_engine_create(int64_t hbm_budget_bytes, int32_t max_slots, void* stream, ss_engine** out);
ss_status ss_engine_submit(ss_engine* e, ss_op* op, const void* f_dev, void* u_dev, double tol,
                           ss_precision prec, int32_t max_iter, int64_t tag);
ss_status ss_engine_step(ss_engine* e, int32_t iters, int32_t* n_active);
ss_status ss_engine_poll(ss_engine* e, int32_t cap, int64_t* tags, int32_t* probs,
                         ss_solve_info* info, int32_t* n_out);
ss_status ss_engine_usage(const ss_engine* e, int32_t* n_active_requests, int64_t* bytes);
void ss_engine_free(ss_engine* e);

/* ss_solve_batch -- Alg. 1, steps 3-5, for n_prob problems of one dimension d from host data:
 * stamping sets (Sec. 6, Eq. StampSet), operators (Sec. 9, Eq. FiniteGalerkinOperator), right-hand
 * sides and solves, with the problems split into n_parts contiguous parts (at most n_prob) that are
 * built and solved concurrently, each by its own host thread on its own stream.
 *   n_a, a_freqs, a_hat: supp(a_p) and its coefficients, all problems concatenated (host), as for
 *     ss_build_stamp_batch and ss_build_op (a_hat interleaved complex128).
 *   n_f, f_freqs, f_hat: F_p and f_hat on it, concatenated (host; f_hat complex128), as for
 *     ss_build_stamp_batch and ss_stamp_forcing; f_0 must not be listed.
 *   level[p], tol, prec, max_iter, flags: as for ss_build_stamp_batch, ss_solve_op and ss_build_op.
 *   info (host, nullable): n_prob entries, filled for every problem that was solved.
 * On SS_OK, and on SS_ENOCONV / SS_EBREAKDOWN (best iterates kept), *out holds every problem's
 * u in canonical order; read it with ss_batch_size / ss_batch_solution and free it with
 * ss_free_batch.  On any other error *out is NULL.  Each problem's u is bitwise the one it gets
 * when solved alone.  Synchronous. */
ss_status ss_solve_batch(int32_t n_prob, int32_t d, const int32_t* n_a, const int16_t* a_freqs,
                         const double* a_hat, const int32_t* n_f, const int16_t* f_freqs,
                         const double* f_hat, const int32_t* level, double tol, ss_precision prec,
                         int32_t max_iter, uint32_t flags, int32_t n_parts, ss_batch** out,
                         ss_solve_info* info);

/* total rows of a batch solution and (host, nullable, n_prob+1 entries) each problem's first row */
ss_status ss_batch_size(const ss_batch* b, int64_t* n_total, int64_t* offsets);

/* copy the batch solution, all problems concatenated in canonical order, into u (device,
 * complex128, n_total entries); asynchronous on `stream` */
ss_status ss_batch_solution(const ss_batch* b, void* u, void* stream);

void ss_free_batch(ss_batch* b);

/* ---------------------------------------------------------------- one shot
 * ss_solve -- Alg. 1 steps 3-5 for one problem from host data.
 *   a: n_a frequencies/coefficients (exact zeros dropped, -w completed);
 *   f: n_f frequencies/coefficients (host);
 *   tol, prec, max_iter, flags: as for ss_solve_op and ss_build_op.
 *   x0 (host, nullable): initial guess, |S^N| complex128 in canonical order (query the size
 *   first); NULL starts from 0.
 *   u_cap: complex entries available in u_hat_out.  u_hat_out == NULL is a
 *   size query: *n_out = |S^N| and SS_OK.  u_cap < |S^N| -> SS_EINVAL.
 *   keys_out (nullable): [|S^N| x d] canonical keys.
 */
ss_status ss_solve(int32_t d, int32_t n_a, const int16_t* a_freqs, const double* a_hat,
                   int32_t n_f, const int16_t* f_freqs, const double* f_hat, int32_t level,
                   double tol, ss_precision prec, int32_t max_iter, uint32_t flags,
                   const double* x0, int64_t u_cap, int64_t* n_out, double* u_hat_out,
                   int16_t* keys_out, ss_solve_info* info);

/* ---------------------------------------------------------------- device memory
 * ss_memory_stats -- the library's caching allocator (not a passage of the paper: accounting for
 *   callers that budget device memory, e.g. a serving loop).  Every device block the library uses
 *   comes from it; a released block is kept for reuse and returned to the driver only when an
 *   allocation would otherwise fail.
 *   live_bytes: bytes in blocks currently held by stamps, operators, engines and calls in flight;
 *   cached_bytes: bytes in released blocks kept for reuse;
 *   driver_allocs: number of blocks taken from the driver since the process started.
 *   All three are totals over every device, written to host memory the caller owns.  Needs no
 *   device (all zero before the first allocation).  Null argument -> SS_EINVAL.
 */
ss_status ss_memory_stats(int64_t* live_bytes, int64_t* cached_bytes, int64_t* driver_allocs);

const char* ss_last_error(void);
const char* ss_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPARSESPEC_H */
