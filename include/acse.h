/*
 * acse.h -- C ABI of the MI355X (gfx950) ACSE residual library, libacse.so.
 *
 * The library evaluates the hot path of the anti-Hermitian contracted
 * Schroedinger equation (ACSE, arXiv 2604.02550) for singlet-type states:
 *
 *   residual  R^{ij}_{kl} = <psi| [a+_i a+_j a_l a_k, H] |psi>        (Eq. (4))
 *             with the 3-RDM rebuilt by Valdemoro cumulant reconstruction
 *             (Eq. (7) with 3Delta = 0; App. C, Eq. (C5)) or, as an option,
 *             by the Nakatsuji-Yasuda one (Eq. (8)), and never stored,
 *   update    U = 1/2 <[a+a+aa, A]>, A = sum R_m a+a+aa,  2D <- 2D + eps U  (Eq. (9)),
 *   energy    E = Tr(K 2D) with the reduced Hamiltonian K of Eq. (2).
 *
 * Conventions (all arrays row-major, FP64, caller-owned):
 *   r          number of spatial orbitals; indices p,q,r,s in [0, r).
 *   h[r*r]     one-electron integrals 1K (symmetric).
 *   V[r^4]     two-electron integrals in chemists' notation V[p,q,r,s] = (pq|rs)
 *              (8-fold symmetric).  The reduced Hamiltonian of Eq. (2) is
 *              K^{pq}_{rs} = (pr|qs) + (h_pr d_qs + h_qs d_pr)/(N-1) on every
 *              spin block, so that H = 1/2 sum K a+_p a+_q a_s a_r and E = Tr(K 2D).
 *   d1[r*r]    alpha 1-RDM  1D[p,r] = <a+_pa a_ra>  (beta is equal).
 *   d2aa[r^4]  2D(pa qa | ra sa) = 1/2 <a+_pa a+_qa a_sa a_ra>     (Eq. (6))
 *   d2ab[r^4]  2D(pa qb | ra sb) = 1/2 <a+_pa a+_qb a_sb a_ra>
 *              (the beta-beta block equals alpha-alpha; App. A traces
 *              Tr d2aa = Na(Na-1)/2, Tr d2ab = Na Nb/2).
 *              Required symmetries (those of singlet RDMs, which the spin
 *              blocks encode): d2aa antisymmetric within (p,q) and within
 *              (r,s); d2ab[p,q,r,s] = d2ab[q,p,s,r] (the beta-alpha block is
 *              the pair-exchanged alpha-beta block).  The contractions exploit
 *              them and do not check them unless the options carry
 *              ACSE_FLAG_CHECK_INPUTS: other inputs give results that match
 *              no residual, with no error reported.
 *   R_aa, R_ab the residual blocks R(ia ja | ka la), R(ia jb | ka lb), same layout.
 *   ||R||^2    the squared Frobenius norm over all spin-orbital elements,
 *              2 ||R_aa||^2 + 4 ||R_ab||^2, taken before the active mask.
 *
 * Sign: Eq. (4) is followed (R = +<[O,H]>); Eq. (5) as printed gives -R.  The
 * update U is even in this sign.
 *
 * Memory: h, V, d1, d2aa, d2ab and all outputs are DEVICE pointers on the
 * context's device, 16-byte aligned, owned by the caller.  Outputs ending in
 * _host are host pointers.  The library owns only its workspace, allocated in
 * acse_create for a maximum size r_max (the adjoint, the Euler driver, the
 * batched residual and the Nakatsuji-Yasuda reconstruction add their own on
 * their first call, also sized for r_max or the batch) and released in
 * acse_destroy; it keeps no caller pointer after a call returns.
 *
 * Streams: every call is ordered on the context's HIP stream.  Calls that
 * return a host scalar synchronise that stream before returning; the others
 * return as soon as the work is enqueued.
 *
 * Errors: every call returns an acse_status; no C++ exception crosses the ABI.
 * acse_last_error() gives a human-readable detail for the last failing call
 * on a context.  A failing call leaves caller outputs unspecified and the
 * inputs unchanged (acse_step validates before it writes).
 */
#ifndef ACSE_H
#define ACSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct acse_ctx_s *acse_ctx;

typedef enum {
  ACSE_OK = 0,
  ACSE_ERR_ARG = 1,         /* null pointer, bad enum value, non-finite eps */
  ACSE_ERR_SHAPE = 2,       /* r < 2, r > r_max, N < 2 or N > 2r */
  ACSE_ERR_ALIGN = 3,       /* a device pointer is not 16-byte aligned */
  ACSE_ERR_UNSUPPORTED = 4, /* n_alpha != n_beta in the singlet calls (use the _spin calls),
                               a combination of options that is not built */
  ACSE_ERR_NOMEM = 5,       /* workspace allocation failed */
  ACSE_ERR_HIP = 6,         /* a HIP runtime call failed */
  ACSE_ERR_NONFINITE = 7    /* ||R||^2 or E came out non-finite */
} acse_status;

/* Arithmetic of the O(r^6) contractions.  Everything else (folds, the
 * residual norm, the step, trace restoration, the 1-RDM contraction and the
 * energy) is FP64 in every mode. */
typedef enum {
  ACSE_FP64 = 0,   /* FP64 MFMA (v_mfma_f64_16x16x4) */
  ACSE_FP32 = 1,   /* FP32 operands, FP32 MFMA accumulation */
  ACSE_BF16X3 = 2, /* split-BF16 products a_hi b_hi + a_hi b_lo + a_lo b_hi, FP32 accumulation */
  ACSE_INT8CRT = 3 /* exact accumulation on the int8 MFMA: each operand row is scaled by a
                      power of two to integers of k bits (the largest k with
                      K 2^(2k) < M/4; k = 44 for 13 moduli at K = 2500), the integers are
                      split into their residues modulo `moduli` pairwise coprime moduli
                      <= 256, each modulus runs one int8 product with exact int32
                      accumulation (v_mfma_i32_32x32x32_i8), and the exact integer
                      product is rebuilt by the Chinese remainder theorem in FP64.  The
                      only rounding is that of the operands to k bits relative to their
                      row's largest magnitude.  Residual, update map, step, autotune
                      and the Euler iteration (every control; the quadratic one through
                      the adjoint), with the Valdemoro or the NY reconstruction, the
                      residual adjoint (Valdemoro), the spin-block calls and the batched
                      residual on its lanes (one residue workspace per lane, allocated
                      by the first such batch); the persistent batch and
                      acse_residual_noalloc are ACSE_ERR_UNSUPPORTED with it.  The first
                      call allocates residue buffers for r_max: 12 x (15 x op_rows x
                      round_up(r_max^2, 256) + 4 op_rows) bytes for the operands
                      (op_rows = r_max^2 rounded up to 256) and 15 x about 4.5 r_max^4
                      bytes for the products' residues (1.6 GB in all at r_max = 50);
                      the first NY call in this mode adds the residues of the NY
                      operand buffers and of six block products (about 0.1 GB per
                      operand buffer and 0.6 GB at r_max = 50). */
} acse_precision;

typedef struct {
  int32_t r;          /* spatial orbitals, 2 <= r <= r_max */
  int32_t n_alpha;    /* alpha electrons */
  int32_t n_beta;     /* beta electrons; must equal n_alpha (singlet blocks) */
  const double *h;    /* device [r*r] */
  const double *V;    /* device [r^4]  */
  double *d1;         /* device [r*r]  alpha 1-RDM (acse_step overwrites it) */
  double *d2aa;       /* device [r^4]  (acse_step overwrites it) */
  double *d2ab;       /* device [r^4]  (acse_step overwrites it) */
} acse_problem;

typedef struct {
  int32_t precision;      /* acse_precision */
  const uint8_t *active;  /* HOST [r]: nonzero = active orbital, or NULL for no mask.
                             A residual element is zeroed before the update iff all
                             four of its spatial indices are active (the "all active"
                             option of the method section); the norm is taken first. */
  int32_t tile;           /* GEMM tile configuration, -1 = autotuned default */
  int32_t flags;          /* bitwise OR of ACSE_FLAG_* (0 = none) */
  int32_t reconstruction; /* acse_reconstruction of the 3-RDM (0 = Valdemoro); other values
                             are an ACSE_ERR_ARG */
  const int8_t *ny_sigma; /* HOST [r] or NULL, ACSE_RECON_NY only: +1 for an orbital occupied
                             in the Hartree-Fock reference, -1 for an unoccupied one;
                             NULL = orbitals 0 .. n_alpha-1 occupied.  The _spin calls
                             take HOST [2r], one per spin orbital, alpha orbitals first
                             (NULL = alpha orbitals below n_alpha and beta orbitals below
                             n_beta occupied).  Other values are an ACSE_ERR_ARG. */
  int32_t moduli;         /* ACSE_INT8CRT: number of moduli, 8..15 (0 = 13); more moduli
                             give more bits k per operand (k = 40 / 44 / 48 at
                             K = 2500 for 12 / 13 / 14) and one more int8 product
                             each.  Ignored by the other precisions (0 or 8..15). */
} acse_options;

/* 3-RDM reconstruction of the residual map (Eq. (7)).
 *   ACSE_RECON_V   Valdemoro: the 3-cumulant is dropped (App. C, Eq. (C5)).
 *   ACSE_RECON_NY  Nakatsuji-Yasuda: the 3-cumulant is approximated by the
 *                  sigma-weighted, antisymmetrised product of two 2-cumulants
 *                  of Eq. (8) (App. D, NY part), never formed.  Both maps of
 *                  a step use it.  Its share runs as 18 spatial-block GEMMs
 *                  of r^2 x r^2 x r^2 per map (one with K packed to r(r-1)/2;
 *                  a spin-orbital contraction split over the spins of its
 *                  internal indices) in the call's precision; its combination into the map is FP64.  The
 *                  first NY call allocates its workspace for r_max (about
 *                  (19 r^4 + 44 r^4-sized operand buffers) x 8 bytes: 3.3 GB at
 *                  r_max = 50; ACSE_ERR_NOMEM if that fails).  In the
 *                  batched residual each instance takes its reference
 *                  occupations from its n_alpha (ny_sigma must be NULL) and
 *                  the NY shares run in order on the context's stream.  The
 *                  adjoint (acse_residual_vjp) and the quadratic step control
 *                  of acse_solve (which needs it) take the NY share's adjoint
 *                  for r <= 64 (ACSE_ERR_UNSUPPORTED above): over
 *                  spin-orbital tensors (n = 2r) as 15 pairwise contractions,
 *                  each run as the 10 of its 64 r^2 x r^2 x r^2 spin-block
 *                  products whose operand blocks conserve spin (FP64, or int8
 *                  exact-accumulation products under ACSE_INT8CRT; the rest
 *                  FP64); its first call allocating 12 n^4 doubles and two
 *                  operand buffers of 16 round_up(r^2, 256) round_up(r^2, 64)
 *                  doubles for its r (1.9 GB at r = 32, 11.3 GB at r = 50),
 *                  its first ACSE_INT8CRT call the residues of the 32 operand
 *                  sub-blocks and of one launch's six products (3.7 GB at
 *                  r = 50), reallocated when a larger r comes, kept until
 *                  acse_destroy. */
typedef enum { ACSE_RECON_V = 0, ACSE_RECON_NY = 1 } acse_reconstruction;

/* acse_options.flags: run the general-size kernels at every r (the one-index
 * transforms for the ph A operands (otherwise r > 56); the G2 kernel that
 * stores G2, followed by two one-index transforms for the g G2 g product
 * (otherwise r > 52), without its mirrored-row staging (otherwise r > 82) and
 * without its pair-index tables (otherwise r in 80..82 and r > 94); the
 * row-chunked assembly (otherwise r > 81); the mode-product kernel in its
 * r > 64 shape and the Gram kernel in its r > 80 shape; in the adjoint, the
 * alpha-beta pp products packed over the pair-exchange symmetry (otherwise
 * r >= 40)).  Same results up to
 * rounding order; meant for verifying those kernels at small r.  Other bits
 * are an ACSE_ERR_ARG. */
#define ACSE_FLAG_GENERAL_KERNELS 1

/* acse_options.flags: before computing, check on the device that the inputs
 * have the symmetries the method requires of them (h and d1 symmetric; V
 * invariant under p<->q, r<->s and (pq)<->(rs); d2aa antisymmetric under i<->j
 * and k<->l and Hermitian; d2ab Hermitian and invariant under
 * (ij)(kl) -> (ji)(lk)).  A largest violation above 1e-12 times the array's
 * largest magnitude (or a non-finite value) returns ACSE_ERR_ARG naming the
 * array; otherwise the call proceeds as without the flag.  Synchronises the
 * stream.  Without the flag the symmetries are assumed, not checked: other
 * inputs give results that are no residual of any state. */
#define ACSE_FLAG_CHECK_INPUTS 2

/* acse_options.flags, acse_residual_batched and acse_autotune_batched only
 * (ignored by the other calls): run the pair-index products of all instances
 * as one persistent launch between the per-instance stages instead of each
 * instance's own grouped launch on its side stream. */
#define ACSE_FLAG_BATCH_PERSISTENT 4

/* Creates a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t; NULL = the default stream), with workspace for problems up
 * to r_max spatial orbitals.  Returns ACSE_ERR_NOMEM if the workspace does
 * not fit. */
acse_status acse_create(acse_ctx *out, int device, void *hip_stream, int32_t r_max);

/* Frees the workspace (after synchronising the stream) and the context. */
acse_status acse_destroy(acse_ctx ctx);

/* Replaces the stream later calls are ordered on. */
acse_status acse_set_stream(acse_ctx ctx, void *hip_stream);

/* Residual of Eq. (4) (Valdemoro 3-RDM, never stored).  Writes R_aa, R_ab
 * (device [r^4] each, may not alias inputs) and, if norm2_host is not NULL,
 * ||R||^2 (synchronises).  The active mask in opts is ignored here. */
acse_status acse_residual(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                          double *R_aa, double *R_ab, double *norm2_host);

/* Update map of Eq. (9) for a given anti-Hermitian two-body tensor X (blocks
 * X_aa, X_ab in the layout of R): U = 1/2 <[a+a+aa, sum X a+a+aa]> with the
 * Valdemoro 3-RDM of the problem's RDMs.  With X = the masked residual this
 * is the 2-RDM update direction.  Writes U_aa, U_ab (device [r^4]). */
acse_status acse_update_map(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                            const double *X_aa, const double *X_ab, double *U_aa, double *U_ab);

/* Energy E = Tr(K 2D) = 2<K_s, d2aa> + 2<K_s, d2ab> (Eq. (2), Eq. (6)), FP64.
 * Synchronises. */
acse_status acse_energy(acse_ctx ctx, const acse_problem *prob, double *E_host);

/* One Euler step of Eq. (9): R = residual, R_m = mask(R), U = update_map(R_m),
 * 2D <- 2D + eps U, each 2-RDM block rescaled to its input trace (FP64),
 * 1D <- 2/(N-1) sum_q 2D[p,q,r,q] (alpha block), and E = Tr(K 2D) of the new 2D.
 * Overwrites prob->d1, d2aa, d2ab.  R_aa/R_ab/U_aa/U_ab (device [r^4] each)
 * receive R and U if not NULL.  E_host and norm2_host (||R||^2 of the input
 * state, before masking) may be NULL.  Synchronises if either is not NULL. */
acse_status acse_step(acse_ctx ctx, acse_problem *prob, double eps, const acse_options *opts,
                      double *R_aa, double *R_ab, double *U_aa, double *U_ab,
                      double *E_host, double *norm2_host);

/* The Euler iteration of Eq. (9) with the stopping rules of the method
 * section (fixed eps; stop when E or ||R|| rises, or when |dE| < 1e-6 Eh),
 * driven on the host with every step on the device.
 *
 * Step n starts from the state 2D_n (with 1D_n, E_n, ||R_n||^2) and its update
 * direction U_n = update_map(mask(R_n)).  A trial with step size x is
 * 2D' = (2D_n + x U_n) rescaled per block to the trace of 2D_n, 1D' its
 * contraction and E', ||R(2D')||^2 (before masking) its scalars.  A trial is
 * acceptable iff E' <= E_n and ||R'||^2 <= ||R_n||^2.  Step-size control:
 *   ACSE_EULER_FIXED      the method section's loop: the trial at eps is the
 *                         step; a rise ends the iteration and the state before
 *                         it is kept.
 *   ACSE_EULER_BACKTRACK  a rise halves the step size (same U_n, new trial from
 *                         2D_n) up to max_halvings times before ending; the step
 *                         size of an accepted step carries over.
 *   ACSE_EULER_QUADRATIC  Newton-like control from the adjoint: the slope
 *                         f'(0) of f(x) = ||R(2D_n + x U_n)||^2 comes from
 *                         acse_residual_vjp with the cotangent (4 R_aa, 8 R_ab)
 *                         (the 1-RDM's dependence on 2D included); after the
 *                         first trial at x = eps, if f'(0) < 0 the minimiser of
 *                         f(0) + f'(0) x + c x^2 through f(eps) (4 eps if c <= 0),
 *                         clamped to [eps/4, min(4 eps, eps_max)], is tried too
 *                         unless within 5% of eps; the acceptable trial with the
 *                         smaller ||R||^2 is taken (the first on a tie), else
 *                         halving continues from the smaller step size.  Its
 *                         step size carries over.  With the NY reconstruction
 *                         the slope is the NY residual's (r <= 64).
 * After an accepted step, |E_{n+1} - E_n| < de_tol ends the iteration.
 * Inputs whose 1D is not the contraction of 2D have it replaced by the
 * contraction at the first accepted step (as in acse_step).
 */
typedef enum {
  ACSE_EULER_FIXED = 0,
  ACSE_EULER_BACKTRACK = 1,
  ACSE_EULER_QUADRATIC = 2
} acse_step_control;

typedef enum {
  ACSE_STOP_MAX_ITER = 0,     /* max_iter accepted steps taken */
  ACSE_STOP_CONVERGED = 1,    /* the last accepted step changed E by less than de_tol */
  ACSE_STOP_ENERGY_ROSE = 2,  /* the last trial raised E; the state before it is returned */
  ACSE_STOP_NORM_ROSE = 3     /* the last trial raised ||R||; the state before it is returned */
} acse_stop_reason;

typedef struct {
  double eps;            /* first step size (the method section uses 1e-3); finite, nonzero;
                            > 0 for ACSE_EULER_QUADRATIC (a negative eps moves uphill) */
  double de_tol;         /* energy-change threshold in Eh (the method section: 1e-6); >= 0 */
  double eps_max;        /* ACSE_EULER_QUADRATIC: largest step size; 0 = 16 eps */
  int32_t max_iter;      /* most accepted steps, >= 0 */
  int32_t control;       /* acse_step_control */
  int32_t max_halvings;  /* BACKTRACK, QUADRATIC: most halvings within one step, 0..60 */
  int32_t reserved;      /* must be 0 */
} acse_solve_options;

typedef struct {
  double eps;         /* step size of the trial */
  double energy;      /* E of the trial 2-RDM */
  double norm2;       /* ||R||^2 of the trial 2-RDM (before masking) */
  int32_t step;       /* index n of the step the trial belongs to */
  int32_t accepted;   /* 1 if the trial became 2D_{n+1} */
} acse_trial;

typedef struct {
  double energy0, norm2_0;  /* E and ||R||^2 of the input state */
  double energy, norm2;     /* of the returned state */
  double eps;               /* step size of the last accepted step (0 if none) */
  int32_t iterations;       /* accepted steps */
  int32_t trials;           /* trials evaluated (all of them, also beyond the history capacity) */
  int32_t maps;             /* residual maps F evaluated (residuals and update directions) */
  int32_t stop;             /* acse_stop_reason */
} acse_solve_result;

/* Runs the iteration above on prob (1D, d2aa, d2ab overwritten with the
 * returned state).  opts as for acse_step (precision of the contractions,
 * active mask, tile, flags).  result (host) receives the summary; history
 * (host, capacity entries, may be NULL if capacity is 0) receives the trials in
 * order.  The first call allocates a driver workspace (2 r_max^2 + 1032
 * doubles; 5 r_max^4 + 2 r_max^2 more for ACSE_EULER_QUADRATIC, which also
 * allocates the adjoint workspace), kept until acse_destroy.  The state 2D_n is
 * kept in the context's workspace while trials run.  Synchronises once per trial.  Errors as
 * acse_step; bad solve options are ACSE_ERR_ARG; on an error mid-run the
 * problem arrays hold the last accepted or trial state. */
acse_status acse_solve(acse_ctx ctx, acse_problem *prob, const acse_options *opts,
                       const acse_solve_options *sopts, acse_solve_result *result,
                       acse_trial *history, int32_t capacity);

/* Hand-written adjoint (vector-Jacobian product) of the residual of Eq. (4):
 * given a cotangent (Rbar_aa, Rbar_ab) on (R_aa, R_ab), writes the gradients of
 * L = <Rbar_aa, R_aa> + <Rbar_ab, R_ab> with respect to h, V, d1, d2aa and
 * d2ab (device arrays of the same shapes).  The forward intermediates are
 * recomputed, not stored.  Each gradient is projected onto the symmetry
 * subspace of its input (h, d1 symmetric; V 8-fold symmetric; d2aa
 * antisymmetric in both pairs and Hermitian; d2ab Hermitian and symmetric
 * under (pq)(rs) -> (qp)(sr)), which is what finite differences along
 * symmetry-respecting directions measure.  The contractions run in
 * opts->precision (with ACSE_INT8CRT the adjoint products are int8
 * exact-accumulation products of FP64 operands, as in the forward map);
 * accumulation of the gradients is FP64.  The first call allocates the
 * adjoint workspace (36 r_max^4 doubles plus 12 pair-index operand buffers),
 * the first ACSE_INT8CRT call the residues of those 12 buffers and of one
 * launch's products; both are kept until acse_destroy.  With the NY
 * reconstruction (r <= 64, otherwise ACSE_ERR_UNSUPPORTED) the NY share's
 * adjoint joins, in FP64 whatever the precision (see ACSE_RECON_NY).  Errors
 * as acse_residual. */
acse_status acse_residual_vjp(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                              const double *Rbar_aa, const double *Rbar_ab, double *h_bar,
                              double *V_bar, double *d1_bar, double *d2aa_bar, double *d2ab_bar);

/* Adjoint of the energy E = Tr(K 2D): gradients of Ebar * E with respect to
 * h, V, d2aa, d2ab (projected as above).  d1 does not enter E. */
acse_status acse_energy_vjp(acse_ctx ctx, const acse_problem *prob, double Ebar, double *h_bar,
                            double *V_bar, double *d2aa_bar, double *d2ab_bar);

/* Stage timing with HIP events recorded on the context's stream.  Stages:
 *   0  RDM-side operands (W = Gamma2 - 2/3 Gamma1^Gamma1 and its layouts;
 *      with ACSE_INT8CRT also their residues)
 *   1  fold of the reduced Hamiltonian (Eq. (2))
 *   2  O(r^4)/O(r^5) transforms feeding the contractions (with
 *      ACSE_INT8CRT also the X-side residues)
 *   3  grouped pair-index GEMM (the six O(r^6) contractions of one map; with
 *      ACSE_INT8CRT the modular int8 products alone; on the spin-block path
 *      its 17 block products)
 *   4  assembly, (ij)<->(kl) exchange and the FP64 norm (with ACSE_INT8CRT
 *      also the reconstruction of the products from their residues)
 *   5  step tail: axpy, trace restoration, 1-RDM contraction, energy
 *   6  Nakatsuji-Yasuda share, whole (cumulant blocks, operand builds, its
 *      block GEMMs, unscrambling and the combination into the map;
 *      ACSE_RECON_NY only)
 *   7  the block GEMMs of the Nakatsuji-Yasuda share alone (inside stage 6)
 * acse_profile_enable(ctx, 1) clears the totals and starts recording;
 * acse_profile_read synchronises the stream and returns the totals (ms and
 * number of timed intervals per stage) since the last enable. */
#define ACSE_NUM_STAGES 8
typedef struct {
  double ms[ACSE_NUM_STAGES];
  int64_t count[ACSE_NUM_STAGES];
} acse_profile_data;
acse_status acse_profile_enable(acse_ctx ctx, int32_t enable);
acse_status acse_profile_read(acse_ctx ctx, acse_profile_data *out);

/* Autotuner: times the grouped GEMM of one residual map per tile
 * configuration on this problem (one warm-up, then the fastest of five runs)
 * and caches the fastest configuration for (r, precision) (the size default
 * is kept unless another configuration is at least 3% faster); later calls with
 * opts->tile = -1 use it.  Writes the chosen configuration index to
 * *best_tile and, if times_ms is not NULL, the time of every configuration
 * (times_ms[0..n-1], n = ACSE_NUM_TILE_CONFIGS).  Synchronises. */
#define ACSE_NUM_TILE_CONFIGS 3
acse_status acse_autotune(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                          int32_t *best_tile, double *times_ms);

/* Batched residual of Eq. (4) over `count` independent instances (1 <= count
 * <= 4096) of possibly different r, each r <= r_max: ground and excited
 * states, several molecules.  Each instance runs the launches of its own
 * acse_residual call (RDM operands, fold, transforms, its grouped product
 * launch, assembly) in order on one of four side streams (largest instances
 * first, each to the least loaded stream), so one instance's memory-bound
 * stages overlap another's products; the context's stream waits for all of
 * them.  With ACSE_FLAG_BATCH_PERSISTENT (and always with the
 * Nakatsuji-Yasuda reconstruction) the per-instance stages before and after
 * the products run on the side streams and the six pair-index products of
 * all instances run in between as one persistent launch: a grid sized to the
 * resident capacity walks one tile list ordered by decreasing K.
 *   probs       host array [count]
 *   R_aa, R_ab  host arrays [count] of device pointers, [r_i^4] each
 *   norm2_host  host [count] (||R_i||^2 as in acse_residual) or NULL;
 *               if not NULL the call synchronises
 *   opts        apply to every instance.  tile = -1: per instance the
 *               configuration a single call of that r takes (acse_autotune's
 *               choice for (r, precision), else the size default); with
 *               ACSE_FLAG_BATCH_PERSISTENT the one acse_autotune_batched
 *               chose for this (precision, list of r), else the size default.
 * The first call (and any call that needs more room) allocates a batch
 * workspace kept until acse_destroy.  Errors are as for acse_residual; the
 * detail names the failing instance. */
acse_status acse_residual_batched(acse_ctx ctx, int32_t count, const acse_problem *probs,
                                  const acse_options *opts, double *const *R_aa,
                                  double *const *R_ab, double *norm2_host);

/* Autotuner of the batched call.  Default: runs acse_autotune on one instance
 * of each distinct r (each choice cached for (r, precision), as the batched
 * call takes them) and reports the outputs of the largest r.  With
 * ACSE_FLAG_BATCH_PERSISTENT: times the persistent product launch of this
 * batch under every tile configuration and caches the fastest for
 * (precision, list of r).  Outputs as for acse_autotune.  Synchronises. */
acse_status acse_autotune_batched(acse_ctx ctx, int32_t count, const acse_problem *probs,
                                  const acse_options *opts, int32_t *best_tile, double *times_ms);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, allocation-free serving loops, harnesses that forbid hipMalloc):
 * the residual of acse_residual with no context and no allocation of any kind.
 * The workspace of the call lives in a device array of the library, 24 MiB,
 * one copy per GPU it runs on, held until the process ends; it covers
 * r <= 16 (r > 16 is ACSE_ERR_SHAPE; the Nakatsuji-Yasuda reconstruction,
 * whose workspace is larger, is ACSE_ERR_UNSUPPORTED).
 *   hip_stream  the hipStream_t the work is ordered on (NULL = default stream)
 *               on the current HIP device
 *   prob, opts  as for acse_residual (tile -1 takes the size default; with
 *               ACSE_FLAG_CHECK_INPUTS the call synchronises the stream)
 *   R_aa, R_ab  device [r^4] outputs
 *   norm2_dev   device double receiving ||R||^2, or NULL; the call never
 *               synchronises or copies to the host otherwise
 * Calls on one GPU share its array: calls whose work overlaps in time on one
 * GPU (other streams, other host threads) race and must be serialised by the
 * caller; calls ordered on one stream are safe.  Every buffer a call reads is
 * written earlier in the same call.  The first call on a device looks up the
 * array's address there (hipGetSymbolAddress).  On an error nothing is
 * enqueued and acse_last_error(NULL) gives the detail (per host thread). */
acse_status acse_residual_noalloc(void *hip_stream, const acse_problem *prob, const acse_options *opts,
                                  double *R_aa, double *R_ab, double *norm2_dev);

/* States of any S_z (N_alpha != N_beta; the Theory section's fixed-spin
 * blocks): the three unique 2-RDM blocks and one 1-RDM per spin.
 *   d1a, d1b   device [r*r]  1D(pa|ra), 1D(pb|rb)
 *   d2aa, d2bb device [r^4]  2D(pa qa|ra sa), 2D(pb qb|rb sb), antisymmetric in
 *              each pair and Hermitian (App. A traces N_a(N_a-1)/2, N_b(N_b-1)/2)
 *   d2ab       device [r^4]  2D(pa qb|ra sb), Hermitian (trace N_a N_b / 2); no
 *              pair-exchange symmetry is assumed.  The other mixed blocks follow
 *              from the antisymmetry: 2D(pb qa|rb sa) = d2ab[q,p,s,r],
 *              2D(pa qb|rb sa) = -d2ab[p,q,s,r].
 * The residual and update come in the same three blocks (R_aa, R_bb, R_ab with
 * R_ab = R(ia jb|ka lb)); ||R||^2 = ||R_aa||^2 + ||R_bb||^2 + 4 ||R_ab||^2 over
 * spin orbitals.  These calls run the spin-orbital map over spatial spin
 * blocks: 17 r^2 x r^2 x r^2 products per map, in FP64 or (with precision
 * ACSE_INT8CRT, moduli as for the singlet calls) as int8 exact-accumulation
 * products of FP64 accuracy.  Options: precision ACSE_FP64 or ACSE_INT8CRT,
 * ACSE_FLAG_GENERAL_KERNELS allowed (ACSE_FLAG_CHECK_INPUTS and the other
 * precisions are ACSE_ERR_UNSUPPORTED); tile as for acse_residual (FP64);
 * either reconstruction.  With ACSE_RECON_NY (r <= 64, otherwise
 * ACSE_ERR_UNSUPPORTED) the NY 3-cumulant of Eq. (8) joins both maps of a
 * step: its share runs over spin-orbital tensors (n = 2r spin orbitals; six
 * pairwise contractions per map, each run as the 10 of its 64 r^2 x r^2 x r^2
 * spin-block products whose operand blocks conserve spin), the block
 * products in FP64, or under ACSE_INT8CRT as int8 exact-accumulation
 * products; its first call allocates 6 n^4 doubles and two operand buffers
 * of 16 round_up(r^2, 256) round_up(r^2, 64) doubles for its r (1.1 GB at
 * r = 32, 6.5 GB at r = 50), its first ACSE_INT8CRT call the residues of
 * the 32 operand sub-blocks and of one launch's six products (3.7 GB at
 * r = 50), reallocated when a larger r comes and kept until acse_destroy.  The first call allocates a workspace for
 * r_max: 48 r_max^4 doubles and 25 GEMM operand buffers (about 3.7 GB at
 * r_max = 50), kept until acse_destroy; the first ACSE_INT8CRT call adds the
 * residues of those buffers and of one launch's products (about 3.0 GB at
 * r_max = 50).  A singlet state given in this form
 * (d1b = d1a, d2bb = d2aa, d2ab pair-exchange symmetric) gives the singlet
 * calls' results. */
typedef struct {
  int32_t r;          /* spatial orbitals, 2 <= r <= r_max */
  int32_t n_alpha;    /* alpha electrons, <= r */
  int32_t n_beta;     /* beta electrons, <= r; n_alpha + n_beta >= 2 */
  const double *h;    /* device [r*r] */
  const double *V;    /* device [r^4] */
  double *d1a;        /* device [r*r] (acse_step_spin overwrites it) */
  double *d1b;        /* device [r*r] (acse_step_spin overwrites it) */
  double *d2aa;       /* device [r^4] (acse_step_spin overwrites it) */
  double *d2bb;       /* device [r^4] (acse_step_spin overwrites it) */
  double *d2ab;       /* device [r^4] (acse_step_spin overwrites it) */
} acse_problem_spin;

/* Residual of Eq. (4) for a state of any S_z: R_aa, R_bb, R_ab (device [r^4]
 * each) and, if norm2_host is not NULL, ||R||^2 (synchronises). */
acse_status acse_residual_spin(acse_ctx ctx, const acse_problem_spin *prob, const acse_options *opts,
                               double *R_aa, double *R_bb, double *R_ab, double *norm2_host);

/* One Euler step of Eq. (9) for a state of any S_z: R, R_m = mask(R),
 * U = F(R_m), each 2-RDM block <- (block + eps U) rescaled to its input trace
 * (a block with zero input trace, i.e. fewer than two electrons of its kind, is
 * set to zero),
 * 1D per spin <- 2/(N-1) times the partial trace of the new 2-RDM (alpha:
 * Tr_2 d2aa + Tr_2 d2ab; beta: Tr_2 d2bb + Tr_1 d2ab), E of the new 2-RDM.
 * Outputs as for acse_step (NULL output arrays are allowed). */
acse_status acse_step_spin(acse_ctx ctx, acse_problem_spin *prob, double eps, const acse_options *opts,
                           double *R_aa, double *R_bb, double *R_ab, double *U_aa, double *U_bb, double *U_ab,
                           double *E_host, double *norm2_host);

/* The Euler iteration of acse_solve (Eq. (9), the method section's stopping
 * rules) for a state of any S_z: each trial is the step of acse_step_spin at
 * its step size from the kept state 2D_n (every block at 2D_n's block trace,
 * both 1-RDMs contracted from the new 2-RDM), its E and ||R||^2 as for
 * acse_residual_spin.  The three controls of acse_solve; for
 * ACSE_EULER_QUADRATIC the slope f'(0) of ||R||^2 along the step comes from
 * the residual's derivative along the straight line (2D_n + x U_n, 1D_n + x dD),
 * dD the 1-RDMs contracted from U_n: R is a polynomial of degree at most 4 in
 * x there (the 3-RDM of either reconstruction is at most quartic in the
 * RDMs), so the five-point central difference at x = +-eps, +-2eps is exact up
 * to rounding (four more residual maps per step, counted in result->maps;
 * the trace restoration leaves the slope unchanged since Tr U_n = 0 per
 * block).  prob's d1a, d1b, d2aa, d2bb and d2ab are overwritten with the
 * returned state; a rise returns the state before it.  opts, result, history
 * and capacity as for acse_solve and acse_step_spin (ACSE_FP64 or
 * ACSE_INT8CRT, either reconstruction).  The first call allocates
 * 3 r_max^4 + 2 r_max^2 doubles more (the kept state), the first quadratic
 * one 6 r_max^4 + 2 r_max^2 more, kept until acse_destroy.  Synchronises once
 * per trial and once per slope.
 * On an error mid-run the problem arrays hold the last accepted or trial
 * state. */
acse_status acse_solve_spin(acse_ctx ctx, acse_problem_spin *prob, const acse_options *opts,
                            const acse_solve_options *sopts, acse_solve_result *result,
                            acse_trial *history, int32_t capacity);

/* Energy Tr(K 2D) = <K_s, d2aa> + <K_s, d2bb> + 2 <K_s, d2ab> (Eq. (2), Eq. (6)); the
 * 1-RDM pointers may be NULL.  Synchronises. */
acse_status acse_energy_spin(acse_ctx ctx, const acse_problem_spin *prob, double *E_host);

/* Human-readable name of a status code (static storage). */
const char *acse_status_str(acse_status s);

/* Detail of the last failing call on ctx (valid until the next call); with
 * ctx = NULL, of the last failing context-free call on this host thread. */
const char *acse_last_error(acse_ctx ctx);

/* Number of bytes of device workspace the context holds. */
int64_t acse_workspace_bytes(acse_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* ACSE_H */
