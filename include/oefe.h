/*
 * oefe.h -- C ABI of the MI355X library for the Chebyshev-filtered subspace
 * iteration (ChFSI) on the orthogonalized-enriched finite-element (OEFE)
 * Kohn-Sham operator (Rufus, Kanungo, Gavini, arXiv 2010.09701).
 *
 * Operator.  The discrete generalized problem H u = eps M u (eqnKSEigGenDiscrete)
 * with block-diagonal overlap M = diag(M^cc, M^oo) (eqnMOEFE, eqnMOEFEInv) is
 * used in the symmetric standard form
 *
 *     Ht = M^-1/2 H M^-1/2,   M^-1/2 = diag(m^-1/2) (+) S,  S = (M^oo)^-1/2,
 *
 * which has the eigenvalues of (M^O)^-1 H^O (eqnKSEignStandDiscrete).  H is
 * 1/2 int grad N* . grad N + int V N* N (eqnHOEFEelelements) over the basis of
 * spectral (GLL) Lagrange elements plus orthogonalized enrichment functions
 * N^O = N^A - N^B (eqnUOEFESplit, eqnUOEFEAtomic, eqnKSAtomicTrunc,
 * eqnorthCGLL).  At a Bloch wavevector k the basis functions carry the Bloch
 * phase (the FE gather is phase-twisted) and the operator is Hermitian.
 *
 * Conventions (all entry points):
 *  - Return value: OEFE_OK (0) or a negative oefe_status.  Argument checks are
 *    synchronous; oefe_last_error() gives a message for the last failure on the
 *    calling thread.
 *  - Vectors are row-major blocks [n_tot x ld] of device memory, ld >= nv,
 *    FE rows first (global FE index g = i + n j + n^2 k, n = nc p), then the
 *    enrichment rows in the order of the enrichment list.  Complex blocks are
 *    interleaved (re, im); ld and nv count complex elements.
 *  - Device buffers (vectors, `work`, outputs marked "device") are owned by the
 *    caller; the library never allocates in the compute calls.  `work` must hold
 *    at least oefe_work_size(op, prec, nv) bytes, 256-byte aligned.
 *  - All compute calls are ordered on the caller's HIP stream; calls that
 *    return host values (lanczos_bounds, cholgs) synchronize that stream.
 *  - An oefe_op handle is not thread-safe; one handle per device.
 */
#ifndef OEFE_H
#define OEFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* oefe_stream; /* a hipStream_t (NULL = default stream) */

typedef enum {
  OEFE_OK = 0,
  OEFE_EINVAL = -1,       /* bad shape, pointer, leading dimension or precision */
  OEFE_ENOMEM = -2,       /* device allocation failed in oefe_op_create */
  OEFE_EDEVICE = -3,      /* HIP runtime error (message via oefe_last_error) */
  OEFE_ENOTSPD = -4,      /* Cholesky breakdown: Gram matrix not positive definite */
  OEFE_ENOCONV = -5,      /* dense eigensolver or Poisson CG did not converge */
  OEFE_EUNSUPPORTED = -6  /* precision / degree / operator kind not supported */
} oefe_status;

/* Element type and arithmetic of the vector block.
 *  F64   real float64 (Gamma-point operator)
 *  F32   real float32 vectors and float32 arithmetic in the filter / H apply
 *  BF16  real float32 vectors; the cell-level contractions take bfloat16
 *        operands (round-to-nearest-even) with float32 accumulation
 *  C128  complex128 (Bloch operator)
 *  C64   complex64 (Bloch operator, float32 arithmetic)
 * cholgs / rayleigh_ritz / lanczos_bounds run in float64 (F64 or C128). */
typedef enum { OEFE_F64 = 0, OEFE_F32 = 1, OEFE_BF16 = 2, OEFE_C128 = 3, OEFE_C64 = 4 } oefe_prec;

/* System description (host memory; copied by oefe_op_create).
 * Periodic cube [0, L)^3 with nc^3 hex cells of degree p (p + 1 GLL nodes per
 * edge; p in {2, 3, 4}).  Atoms at pos[3*I .. 3*I+2] with charge Z[I]; the
 * potential at the Gauss points is V = sum_I -Z_I erf(r_I / sigma) / r_I with
 * r_I the nearest-image distance (replace it with oefe_op_set_potential).
 * Enrichment function nu: atom enr_atom[nu], radial factor
 * r^enr_power[nu] exp(-enr_zeta[nu] r), times d_x/d_y/d_z if enr_axis[nu] is
 * 0/1/2 (-1: none), times the smooth cutoff h(r) = 1 (r <= r0), 0 (r >= r1),
 * 1 / (1 + exp(1/x - 1/(1-x))), x = (r1 - r)/(r1 - r0) in between
 * (eqnKSAtomicTrunc, eqnCutoffProperties); requires r1 < L / 2.
 * kvec: NULL for the real Gamma-point operator, else the Bloch wavevector [3]. */
typedef struct {
  double L;
  int32_t nc, p;
  int32_t n_atoms;
  const double* pos;
  const double* Z;
  double sigma, r0, r1;
  int32_t n_enr;
  const int32_t* enr_atom;
  const int32_t* enr_power;
  const double* enr_zeta;
  const int32_t* enr_axis;
  const double* kvec;
} oefe_system_desc;

typedef struct oefe_op_s* oefe_op;

/* Build the operator on the current HIP device: quadrature rules, lumped GLL
 * mass (eqnMcc), potential, orthogonalized enrichment (eqnorthC, eqnorthCGLL),
 * blocks M^oo (eqnMoo), H^co, H^oo, S = (M^oo)^-1/2; uploads device data.
 * The FE rows are grouped into coupling tiles of 64 rows: 64 consecutive rows, or blocks
 * of 16 x 2 x 2 FE nodes where those couple to clearly fewer enrichment functions in all
 * (the operator's choice, made here).
 * Errors: EINVAL (bad description, or more than 144 enrichment functions coupling
 * to one coupling tile), EUNSUPPORTED (p), ENOMEM, EDEVICE. */
int oefe_op_create(const oefe_system_desc* desc, oefe_op* out);

/* The k-point operator in the periodic-function form (Sec. II eqnksdftu; Sec. III.A
 * eqnUOEFEAtomic, eqnHOEFEelelements): u = exp(-i k.x) psi in periodic FE functions (no
 * Bloch phase) plus orthogonalized enrichment functions with the atomic part
 * exp(-i k.(x - R^x)) psi~(x - R^x), and H = 1/2 grad . grad - i k . grad + |k|^2/2 + V
 * (the enrichment blocks' first-derivative term in its Hermitian form
 * -i/2 k . int (N_m^* grad N_n - grad N_m^* N_n), equal to the written one where the Gauss
 * rule integrates grad (N_m^* N_n) exactly).  desc->kvec is required.  The handle is used
 * like one of oefe_op_create with a wavevector (complex blocks, C128 / C64; batches of
 * this form only); oefe_op_set_potential and oefe_op_get_potential take and return V
 * without the |k|^2/2.  Errors as oefe_op_create; EUNSUPPORTED from a step on a mesh whose
 * n^2 ld or (nc (p+1))^2 ld reach 2^31 elements. */
int oefe_op_create_uform(const oefe_system_desc* desc, oefe_op* out);

/* The operator of oefe_op_create (Gamma point, or the Bloch-function form with desc->kvec)
 * with the integrals of the enrichment functions on an adaptive quadrature (Sec. III.B: each
 * finite element of an enrichment support is divided recursively until trial integrals of the
 * enrichment functions converge).  Rule: a box carries the tensor Gauss rule of p + 1 points
 * per direction; the trial integrals of a box are int psi~^2 and int |grad psi~|^2 of every
 * atomic function (no phase) whose atom's support holds the cell; a box is kept when its rule
 * and the sum of its 8 half-size children's rules differ by at most tol times the function's
 * whole-space integral (radial integrals), else its children are refined (order
 * cx + 2 cy + 4 cz, depth first) down to max_depth levels.  The rule covers the union of the
 * supports (cells ascending); the orthogonalization numerator (eqnorthC), M^oo, H^oo and H^co
 * use it, H^cc keeps the Gauss rule.  V at the rule's points is the nuclear potential of desc
 * at creation; oefe_op_set_potential_adaptive replaces it.  0 < tol < 1, 0 <= max_depth <= 5,
 * desc->n_enr >= 1.  Errors as oefe_op_create.  The periodic-function k-point form:
 * oefe_op_create_uform_adaptive. */
int oefe_op_create_adaptive(const oefe_system_desc* desc, double tol, int32_t max_depth, oefe_op* out);

/* The k-point operator in the periodic-function form (as oefe_op_create_uform: Sec. II
 * eqnksdftu; Sec. III.A eqnUOEFEAtomic, eqnHOEFEelelements) with its enrichment integrals on
 * the adaptive rule of oefe_op_create_adaptive (Sec. III.B; the rule is built from the atomic
 * functions without phase, the same for every k): exp(-i k.(x - R^x)) psi~ at the rule's
 * points, the first-derivative terms and |k|^2/2 on the rule.  oefe_op_set_potential_adaptive
 * takes both potentials without the |k|^2/2.  desc->kvec is required.  Errors as
 * oefe_op_create_adaptive. */
int oefe_op_create_uform_adaptive(const oefe_system_desc* desc, double tol, int32_t max_depth, oefe_op* out);

/* The points of the adaptive rule of an operator from oefe_op_create_adaptive: *n_points, and
 * (host, either may be NULL) xyz [n_points x 3] and weights [n_points], in rule order (cells
 * ascending, leaves depth first, points qx + (p+1) qy + (p+1)^2 qz within a leaf).
 * Errors: EINVAL (not an adaptive-rule operator). */
int oefe_op_adaptive_points(oefe_op op, int64_t* n_points, double* xyz_host, double* w_host);

/* oefe_op_set_potential for an operator with the adaptive rule: V at the Gauss points (device
 * [n_cells * nq], for H^cc) and V_adapt at the rule's points (device [n_points], rule order,
 * for the enrichment blocks), read in stream order; H^co and H^oo are rebuilt on the device
 * (eqnHOEFEelelements with the adaptive rule), queued on `stream`.  oefe_op_set_potential
 * refuses such an operator.  Errors: EINVAL, EDEVICE. */
int oefe_op_set_potential_adaptive(oefe_op op, const double* V, const double* V_adapt, oefe_stream stream);

/* Test operator Ht = diag(lambda) (n real entries, host memory), no mesh. */
int oefe_op_create_diagonal(const double* lambda, int64_t n, oefe_op* out);

int oefe_op_destroy(oefe_op op);

/* dims[0..10] = n_fe, n_enr, n_tot, n_cells, nq, nc, p, is_complex,
 * coupling-tile slots (sum over the coupling tiles of the number of enrichment
 * functions each couples to, padded to 4), tile_rows (64),
 * nonzeros of H^co (FE row, enrichment function pairs whose supports overlap).
 * dims must hold 11 entries. */
int oefe_op_dims(oefe_op op, int64_t* dims);

/* Replace the potential at the quadrature points: V device float64 [n_cells * nq]
 * (cell-major, point index qx + (p+1) qy + (p+1)^2 qz), read in stream order.
 * Rebuilds on the device, queued on `stream` without a host wait, the potential
 * parts of the operator (eqnHOEFEelelements): W V at the quadrature points for the
 * H^cc cell stage, H^co = kinetic part + sum over the cells of a row's node of
 * B^T diag(W V) N^O (pre-scaled by m^-1/2, in every layout the kernels read) and
 * H^oo = kinetic part + sum W V conj(N^O) N^O; the overlap and S do not depend on
 * V.  Compute calls on other streams must be ordered after it by the caller.
 * Errors: EINVAL (null V, diagonal operator, an operator with the adaptive rule), EDEVICE. */
int oefe_op_set_potential(oefe_op op, const double* V, oefe_stream stream);

/* Copy the current potential and the quadrature weights W_{e,q} to host
 * arrays of n_cells * nq doubles (either pointer may be NULL).  Waits for the
 * device (so a queued oefe_op_set_potential is included). */
int oefe_op_get_potential(oefe_op op, double* V_host, double* W_host);

/* Copy S = (M^oo)^-1/2 (n_enr^2, row-major; complex interleaved) and the
 * eigenvalues of M^oo (n_enr) to host (either may be NULL). */
int oefe_op_get_enrichment(oefe_op op, double* S_host, double* Moo_eigs_host);

/* Bytes of `work` needed by the compute calls below for a block of nv vectors. */
size_t oefe_work_size(oefe_op op, oefe_prec prec, int32_t nv);

/* Y = Ht X: one application of the symmetrized operator M^-1/2 H M^-1/2 of the
 * generalized problem H u = eps M u (eqnKSEigGenDiscrete, eqnHOEFEelelements), with
 * the block-diagonal overlap inverse (eqnMOEFEInv: diagonal GLL mass on the FE rows,
 * dense (M^oo)^-1/2 on the enrichment rows) applied as a scaling on both sides; same
 * eigenvalues as the standard form of eqnKSEignStandDiscrete.  X, Y device
 * [n_tot x ld], must not overlap.  prec: F64/F32/BF16 for a real operator, C128/C64
 * for a Bloch operator. */
int ham_apply(oefe_op op, oefe_prec prec, const void* X, void* Y, int64_t ld, int32_t nv,
              void* work, oefe_stream stream);

/* In place X <- T_m(tau(Ht)) X / T_m(tau(a0)), tau(t) = (t - c)/e, e = (b - a)/2,
 * c = (b + a)/2, by the scaled three-term Chebyshev recurrence (Sec. IV: the
 * filter maps the unwanted spectrum [a, b] to [-1, 1]).  m >= 1 applications of
 * Ht; the recurrence scalars are computed in float64.  Requires a < b, a0 < a. */
int chebyshev_filter(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t m,
                     double a, double b, double a0, void* work, oefe_stream stream);

/* The same filter with its bounds in device memory: bounds = {a, b, a0} (device
 * float64[3], read in stream order, e.g. written there from the previous
 * Rayleigh-Ritz values), so that a pipeline queues the filter without waiting
 * for them.  The recurrence scalars are computed on the device with the same
 * float64 arithmetic (same results as chebyshev_filter).  Bounds that violate
 * a0 < a < b are reported in dev_status (device int32[2], optional) as
 * {OEFE_EINVAL, 0}, and the filter then writes zeros; {0, -1} otherwise.
 * 1 <= m <= 160; finite-element operators only. */
int chebyshev_filter_dev(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t m,
                         const double* bounds, void* work, int32_t* dev_status, oefe_stream stream);

/* Mixed-precision filter on a float64 block: X (F64 or C128 layout, device) is
 * rounded to float32 (round-to-nearest-even), filtered with prec_filter (F32 or
 * BF16 for a real operator, C64 for a Bloch operator) as in chebyshev_filter,
 * and widened back into X.  Same requirements and `work` size rule
 * (oefe_work_size(op, prec_filter, nv)). */
int chebyshev_filter_mixed(oefe_op op, oefe_prec prec_filter, void* X, int64_t ld, int32_t nv, int32_t m, double a,
                           double b, double a0, void* work, oefe_stream stream);

/* Chebyshev filters of nk operators sharing one mesh and enrichment layout (the
 * Bloch k-points of one system), advanced in lockstep: each stage of each degree
 * is a single launch covering all operators, so uneven blocks (different nv[q])
 * fill the device together.  Operator q filters X[q] (device [n_tot x ld[q]],
 * nv[q] vectors, in place) with its own bounds abc[3q], abc[3q+1], abc[3q+2] =
 * (a, b, a0) as in chebyshev_filter; all use degree m.  prec as for
 * chebyshev_filter (C128/C64 for Bloch operators).  work: at least
 * oefe_batched_work_size(nk, ops, prec, nv) bytes.  Errors: EINVAL when the
 * operators do not share the mesh / enrichment layout. */
int chebyshev_filter_batched(int32_t nk, const oefe_op* ops, oefe_prec prec, void* const* X, const int64_t* ld,
                             const int32_t* nv, int32_t m, const double* abc, void* work, oefe_stream stream);
size_t oefe_batched_work_size(int32_t nk, const oefe_op* ops, oefe_prec prec, const int32_t* nv);

/* Launch shape of the operator stages.  cw selects the cell-stage tiling:
 * 0 (built-in) puts the (p+1) planes of a cell tensor in the lanes of one wave
 * (64/(p+1) columns, rounded down to even, per wave); 8, 16, 32 or 64 put one
 * plane per wave with cw real columns per cell in a 64-lane tile (64/cw cells).
 * cb (a multiple of 16 up to 128; 0 = built-in) is the real-column width of one
 * unit of the node stage: the workgroup of the fused node kernel of a real
 * operator (at most 80 columns are used: built-in, all columns up to 80, else
 * near-equal blocks), or one
 * wave of the coupling kernel (the H^co products) of a Bloch operator, where 16
 * and 32 are used (larger values act as 32; built-in 16).  Results do not depend
 * on the shape. */
int oefe_set_launch_shape(oefe_op op, int32_t cw, int32_t cb);

/* Autotuner of the launch shape for a batch of operators (nk >= 1, same rules
 * as chebyshev_filter_batched).  Times `reps` batched recurrence steps on
 * copies of the blocks X[q] for each cw in {0, 8, 16, 32, 64} and cb in
 * {16, 32, 64, 128}, with HIP events on `stream`, and sets the fastest shape on
 * every operator.  X is not modified.  work: oefe_batched_work_size(nk, ops,
 * prec, nv) bytes.  Outputs (host, may be NULL): the chosen cw, cb and the
 * time of one batched step in ms.  Synchronizes the stream. */
int oefe_autotune(int32_t nk, const oefe_op* ops, oefe_prec prec, void* const* X, const int64_t* ld,
                  const int32_t* nv, int32_t reps, void* work, int32_t* cw_out, int32_t* cb_out,
                  double* ms_per_step, oefe_stream stream);

/* Spectrum bounds of the filter (Sec. IV: the filter maps the unwanted part of the
 * spectrum, [a, b], linearly onto [-1, 1], so it needs an upper bound b of the
 * spectrum and an estimate a0 of its lower end): k-step Lanczos with full
 * reorthogonalization (twice) from v0 (device, n_tot real, or complex interleaved for
 * a Bloch operator) in float64.  out (host double[3]): out[0] = a0 = smallest Ritz
 * value of T_k, out[1] = b = largest + beta_k, out[2] = the first pass's cut
 * a = (a0 + b) / 2 (later passes take a0 = theta_1 and a = theta_nv of the previous
 * Rayleigh-Ritz, see rayleigh_ritz).  dev_bounds (device double[3], optional)
 * receives {a, b, a0} in the order chebyshev_filter_dev reads.  Synchronizes
 * `stream`.  1 <= k <= 64.  Errors: EINVAL; ENOCONV if the eigensolver of T_k hit
 * its sweep limit. */
int lanczos_bounds(oefe_op op, int32_t k, const double* v0, double* out, void* work, double* dev_bounds,
                   oefe_stream stream);

/* Orthonormalization of the filtered block (Sec. IV: the filtered vectors are
 * orthonormalized before the Rayleigh-Ritz step; the paper uses a QR factorization)
 * by Cholesky-Gram-Schmidt in float64: G = X^* X, G = L L^* (from the Jacobi-scaled
 * G), X <- X L^-* (the Q of a QR factorization with positive diagonal R), repeated
 * once when max|Q^* Q - I| > 1e-12.  prec F64 or C128.  On breakdown (a squared pivot
 * of the unit-diagonal scaled Gram matrix at or below nv 2^-52) returns
 * OEFE_ENOTSPD and, if dev_status (device int32[2]) is given, writes
 * {OEFE_ENOTSPD, column}.  Synchronizes `stream`. */
int cholgs(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, void* work, int32_t* dev_status,
           oefe_stream stream);

/* The same CholGS without waiting on the stream, for pipelines that queue the
 * next step (Rayleigh-Ritz) at once: dev_status (device int32[2], required)
 * receives {0, -1} or {OEFE_ENOTSPD, column} in stream order, and the caller
 * reads it after a later synchronization.  A failed factorization leaves X
 * unchanged, as does the repeated pass when its factorization fails.  Argument
 * errors return at once.  Blocks whose CholGS needs host decisions (complex,
 * more than 80 columns, or a Gram matrix too large for one workgroup's LDS)
 * take the synchronous path of cholgs, which also fills dev_status. */
int cholgs_async(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, void* work, int32_t* dev_status,
                 oefe_stream stream);

/* cholgs_async without a `work` buffer, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Its scratch (Gram matrix, factor inverse, Gram chunk partials,
 * flags; at most 14 MiB) lives in a device array of the library, one per GPU, held
 * until the process ends; the call itself allocates nothing.  Real float64 blocks
 * (F64) of 1..80 columns of a finite-element operator; otherwise EUNSUPPORTED, and
 * EINVAL for a block whose scratch would exceed 14 MiB.  Same results, status and
 * stream ordering as cholgs_async.  Every call on one GPU shares that scratch:
 * calls that overlap on one GPU (several streams or host threads) race. */
int cholgs_noalloc(oefe_op op, oefe_prec prec, void* X, int64_t ld, int32_t nv, int32_t* dev_status,
                   oefe_stream stream);

/* Rayleigh-Ritz (eqnProjKS in symmetric form, Q^* Q = I): W = Ht Q,
 * Hq = Q^* W (Hermitian part), Hq = U diag(theta) U^* (float64 cyclic Jacobi),
 * Q <- Q U.  eigvals: device float64 [nv], ascending.  prec F64 or C128.
 * Queued on `stream` without a host wait.  dev_status (device int32[2], optional)
 * receives {0, sweeps} or {OEFE_ENOCONV, sweeps} when the eigensolver reached its
 * sweep limit before the off-diagonal part fell to rounding (the values and vectors
 * are then those of the last sweep).  next_bounds (device double[3], optional)
 * receives the next pass's filter bounds in chebyshev_filter_dev's order:
 * next_bounds[0] = a = theta_nv, next_bounds[2] = a0 = theta_1 (next_bounds[1] = b
 * is left as it is). */
int rayleigh_ritz(oefe_op op, oefe_prec prec, void* Q, int64_t ld, int32_t nv, double* eigvals, void* work,
                  int32_t* dev_status, double* next_bounds, oefe_stream stream);

/* Sweep limit of the dense Hermitian eigensolver used by rayleigh_ritz and
 * lanczos_bounds on this operator (0 restores the built-in limit of 40 sweeps for
 * matrices held in LDS, 60 otherwise).  Lets a caller bound the eigensolver's time;
 * reaching the limit is reported as OEFE_ENOCONV. */
int oefe_set_eig_sweep_limit(oefe_op op, int32_t sweeps);

/* Band energy E = sum_i f_i x_i^* Ht x_i (device scalar, float64) and its
 * gradients: dE_dV[e,q] = W_{e,q} sum_i f_i |psi_i(x_{e,q})|^2 (device float64
 * [n_cells * nq]; psi_i the field of M^-1/2 x_i, the density of eqnrho times W),
 * dE_dX = 2 Ht X diag(f) (device, layout of X).  f: device float64 [nv].
 * dE_dV / dE_dX may be NULL.  prec F64/F32 (real) or C128/C64 (Bloch).  dE_dV of an
 * operator with the adaptive rule (oefe_op_create_adaptive) is EUNSUPPORTED: V enters its
 * enrichment blocks at the rule's points as well. */
int band_energy_grad(oefe_op op, oefe_prec prec, const void* X, int64_t ld, int32_t nv, const double* f,
                     double* E, double* dE_dV, void* dE_dX, void* work, oefe_stream stream);

/* Occupations from Ritz values (Sec. II): Fermi-Dirac f = 1 / (1 + exp((theta - mu)
 * / kT)) (eqnfd) with the Fermi level mu fixed by the electron count
 * 2 sum_k w_k sum_alpha f = n_elec (eqnne), found by bisection in float64 (the paper
 * does not say how; see the oracle), and the band energy 2 sum_k w_k sum_alpha f theta.
 * nk k-points (1..64): nv[k] values each (host), weights wk[k] (host); theta: device
 * float64, the nk blocks of Ritz values concatenated.  Outputs (device): f [sum nv]
 * (occupations in [0, 1], same layout), out[3] = {mu, E_band, electron count at mu};
 * dev_status int32[2] = {0, halvings} or {OEFE_EINVAL, 0} when n_elec is not between 0
 * and twice the weighted number of states.  kT > 0 (Hartree).  One workgroup, queued on
 * `stream`. */
int oefe_fermi_occupations(int32_t nk, const int32_t* nv, const double* wk, const double* theta, double n_elec,
                           double kT, double* f, double* out, int32_t* dev_status, oefe_stream stream);

/* Electron density at the quadrature points from a block of Ritz vectors (eqnrho):
 * rho[e * nq + q] (+)= sum_i weights[i] |psi_i(x_{e,q})|^2, psi_i the field of
 * M^-1/2 x_i (|u| = |psi| for the Bloch functions of a phase-twisted basis); with
 * weights = 2 w_k f this is one k-point's term of eqnrho, and accumulate != 0 adds it
 * to rho (k-points summed in call order).  weights: device float64 [nv]; rho: device
 * float64 [n_cells * nq].  prec as for band_energy_grad; work: oefe_work_size(op,
 * prec, nv) bytes. */
int oefe_density(oefe_op op, oefe_prec prec, const void* X, int64_t ld, int32_t nv, const double* weights, double* rho,
                 int32_t accumulate, void* work, oefe_stream stream);

/* Operator of the discrete Poisson problem for the auxiliary electrostatic potential
 * (Sec. II eqnpoissonaux; Sec. III.A eqnPhiOEFE, eqnpoissX, eqnDiscLaplace) on the mesh
 * and atoms of desc: the FE functions plus one orthogonalized enrichment function per
 * atom (eqnOrthoEnrichedPhiAux), whose atomic part is (V_H - Z v_g(r, rc)) h(r)
 * (eqnPhiAuxAtomic, eqnEnrichedPhiAux, eqnnucsmear, eqnvg) with the cutoff h of
 * desc (r0, r1), rc half the distance to the nearest other atom or periodic image, and
 * V_H the Hartree potential of the model atom density Z alpha^3/(8 pi) exp(-alpha r),
 * alpha = 2 Z^(1/3) (an atomic solver's radial Hartree potential stands there in the
 * paper).  desc's enrichment list and sigma are not used.  The handle applies
 * At = P^T A P, P = diag(m^-1/2, S), S = (A^oo)^-1/2, through ham_apply (F64) and
 * solves with oefe_poisson_solve; dims (oefe_op_dims) count one enrichment function per
 * atom.  Errors: EINVAL (no atoms, Z <= 0, kvec set, bad cutoff), EUNSUPPORTED (p),
 * ENOMEM, EDEVICE. */
int oefe_poisson_create(const oefe_system_desc* desc, oefe_op* out);

/* The operator of oefe_poisson_create with the integrals of its enrichment functions on an
 * adaptive rule (Sec. III.B; as oefe_op_create_adaptive, the trial functions being the phi
 * enrichment's atomic parts (V_H - Z v_g) h): the orthogonalization numerator, A^co and A^oo on
 * the rule, A^cc on the Gauss rule; solved with oefe_poisson_solve_adaptive.  Errors as
 * oefe_poisson_create, EINVAL for tol outside (0, 1) or max_depth outside [0, 5]. */
int oefe_poisson_create_adaptive(const oefe_system_desc* desc, double tol, int32_t max_depth, oefe_op* out);

/* Work bytes of oefe_poisson_solve (0 for other operators). */
size_t oefe_poisson_work_size(oefe_op pop);

/* phi with A phi = c (eqnpoissX): A_mn = 1/(4 pi) int grad N_m . grad N_n
 * (eqnDiscLaplace), c_m = int (b + rho - background) N_m (eqnDiscForceVec) with b the
 * smeared nuclear charge -sum_I Z_I g(|x - R_I|, rc_I) (eqnsmeared, eqngr, nearest
 * image) and the background the quadrature mean of b + rho (so that the periodic
 * problem is consistent).  rho: device float64 [n_cells * nq] (cell-major, as
 * oefe_density writes it).  phi: device float64 [n_fe + n_atoms], the FE coefficients
 * (GLL-mass-weighted mean zero) then the enrichment coefficients.  Conjugate gradients on
 * At (the GLL mass and A^oo as preconditioner) from zero, stopping when the residual
 * norm falls below tol times its starting value (tested every 8 iterations) or after
 * max_iter iterations; info (host double[2]) = {iterations, relative residual}.  Queued
 * on `stream`, with one host wait per 8 iterations.  Errors: EINVAL (bad arguments, not
 * a Poisson operator), ENOCONV (tolerance not met: phi holds the last iterate), EDEVICE. */
int oefe_poisson_solve(oefe_op pop, const double* rho, double* phi, double tol, int32_t max_iter, double* info,
                       void* work, oefe_stream stream);

/* oefe_poisson_solve for an operator of oefe_poisson_create_adaptive: rho at the Gauss points
 * (the FE rows of the force vector and the background, as in oefe_poisson_solve) and rho_adapt at
 * the rule's points (device float64 [n_points], rule order: oefe_op_adaptive_points) for the
 * enrichment rows, c_I = int (b + rho - background) N^O_I on the rule with the smeared charge b
 * evaluated at its points.  oefe_poisson_solve refuses such an operator.  Same results and
 * errors otherwise. */
int oefe_poisson_solve_adaptive(oefe_op pop, const double* rho, const double* rho_adapt, double* phi, double tol,
                                int32_t max_iter, double* info, void* work, oefe_stream stream);

/* Instrumentation.  While a kernel is selected, each of its launches inside
 * ham_apply / chebyshev_filter* is bracketed by HIP events on the stream it is
 * launched on.  which: OEFE_TIMER_OFF, OEFE_TIMER_CELL (the sum-factorized
 * H^cc cell stage), OEFE_TIMER_NODE (the node stage on the main stream: for a
 * real operator the fused kernel with the slot gather, the H^co products and the
 * recurrence epilogue; for a Bloch operator the node assembly, slot gather and
 * epilogue) or OEFE_TIMER_COUPLING (the H^co products of a Bloch operator, on
 * the filter's side stream).  oefe_kernel_timer_read
 * synchronizes, returns the number of bracketed launches and their summed
 * duration (ms), and clears the record.  Selecting a kernel discards events not
 * yet read. */
typedef enum {
  OEFE_TIMER_OFF = 0,
  OEFE_TIMER_CELL = 1,
  OEFE_TIMER_NODE = 2,
  OEFE_TIMER_COUPLING = 3
} oefe_timer_kind;
int oefe_kernel_timer(oefe_op op, int which);
int oefe_kernel_timer_read(oefe_op op, int64_t* launches, double* total_ms);

/* Measurement aid (not part of the method): the achievable device-memory rate of
 * this GPU, from a hand-written grid-stride copy of `bytes` bytes from src to dst
 * (device, 16-byte aligned, non-overlapping, caller-owned; bytes a positive
 * multiple of 16).  One untimed copy, then `reps` >= 1 copies each bracketed by
 * HIP events on `stream`; *gbs = 2 bytes / median time (read + write, GB/s).
 * Synchronizes the stream; allocates no device memory.  Errors: EINVAL. */
int oefe_copy_rate(const void* src, void* dst, size_t bytes, int32_t reps, double* gbs, oefe_stream stream);

const char* oefe_strerror(int code);
const char* oefe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OEFE_H */
