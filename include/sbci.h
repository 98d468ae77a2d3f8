/*
 * sbci.h -- C ABI of libsbci.so: the FCI sigma build and the SBCI1 solver of
 * "Quantum chemistry based on classical mechanics inspired by simulated
 * bifurcation" (Aiga & Goto), on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Results, "SBCI1 algorithm"): the lowest n eigenpairs of the
 * electronic Hamiltonian H in the Slater-determinant basis of norb spatial
 * orbitals with n_alpha / n_beta electrons:
 *   H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps),
 *   E_pq = sum over spins of a+_p a_q.
 * Determinants are pairs of occupation strings (Ia, Ib); a string is an
 * m-subset of orbitals, strings are ordered by ascending bit mask and the
 * determinant index is Ia * N_beta + Ib (CI vectors are row-major [Ia][Ib]).
 * Energies are electronic (no constant term).
 *
 * Conventions for every function:
 *   - return value: SBCI_OK (0) or a negative sbci_status; the message of
 *     the last failure on the calling thread is sbci_last_error();
 *   - "dev" pointers are device (HIP) memory on the context's device,
 *     "host" pointers are host memory; the caller owns every pointer it passes;
 *   - the context owns everything it allocates and frees it in sbci_destroy;
 *   - one context is driven by one host thread at a time; all GPU work is
 *     enqueued on the context's stream (sbci_set_stream), sbci_sigma is
 *     asynchronous, the solvers return after synchronising that stream;
 *   - on error the outputs are unspecified and the context stays usable.
 */
#ifndef SBCI_H
#define SBCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sbci_status {
  SBCI_OK = 0,
  SBCI_EINVAL = -1,   /* bad argument: sizes, null pointers, aliasing, unknown dtype */
  SBCI_ENOMEM = -2,   /* device allocation failed */
  SBCI_EDEVICE = -3,  /* a HIP call or kernel launch failed */
  SBCI_ENOCONV = -4,  /* step cap reached; outputs hold the last iterate */
  SBCI_ENUMERIC = -5  /* NaN/Inf in a reduction or an unrecoverable subspace */
} sbci_status;

typedef enum sbci_dtype {
  SBCI_F64 = 0,   /* FP64 vectors, FP64 sigma (reference form)                     */
  SBCI_F32 = 1,   /* FP32 vectors, FP32 sigma (FP32 MFMA for the opposite-spin part) */
  SBCI_BF16 = 2   /* FP32 vectors; opposite-spin part on BF16 MFMA with FP32
                     accumulation, one-electron and same-spin parts in FP32         */
} sbci_dtype;

/* Form of the opposite-spin contraction sum (kl|k'l') E^alpha_kl E^beta_k'l'
 * (the two-electron part between the spins of the Hamiltonian of the
 * Results section): SBCI_OPP_PAIR contracts over every unordered orbital
 * pair {k'l'} per beta string, the cheaper form near half filling;
 * SBCI_OPP_ORBITAL groups beta strings by the orbital q that E_pq empties,
 * the cheaper form when few electrons occupy many orbitals; SBCI_OPP_AUTO
 * picks one per sigma dtype from the sizes.  When a row of sigma (one alpha
 * string, all beta strings) does not fit in LDS, the orbital form splits it
 * into windows of beta strings, each recomputing the contraction (more
 * MFMA work, no size limit); SBCI_OPP_ORBITAL_WINDOWED forces at least two
 * windows.  sbci_get_opp_form reports either orbital variant as
 * SBCI_OPP_ORBITAL. */
typedef enum sbci_opp_form {
  SBCI_OPP_AUTO = 0,
  SBCI_OPP_PAIR = 1,
  SBCI_OPP_ORBITAL = 2,
  SBCI_OPP_ORBITAL_WINDOWED = 3,
  SBCI_OPP_CLASS_MFMA = 4  /* symmetry-blocked contexts only: see sbci_create_sym */
} sbci_opp_form;

/* Form of the one-electron and same-spin parts H_alpha + H_beta:
 * SBCI_SAME_LISTS applies each spin's operator from its Slater-Condon lists
 * (one entry per connected string); SBCI_SAME_DENSE multiplies by the dense
 * operator on MFMA, the cheaper form when the lists cover a sizeable
 * fraction of each row (few electrons in many orbitals); SBCI_SAME_AUTO
 * picks per spin from the sizes. */
typedef enum sbci_same_form {
  SBCI_SAME_AUTO = 0,
  SBCI_SAME_LISTS = 1,
  SBCI_SAME_DENSE = 2
} sbci_same_form;

typedef struct sbci_ctx sbci_ctx;

/* Thresholds and policies.  Defaults (sbci_default_opts) are the paper's
 * values: eps0 = 1e-10 Eh, r0 = 1e-5 (Sections S1.2/S1.3, frozen core = No),
 * b_th = 1e-2, eps1 = 1e-7, x_th1 = 0.1, x_th2 = 1.2, r1 = 1, max_cycle = 20
 * (Section S1.5). */
typedef struct sbci_opts {
  double eps0, r0;            /* convergence: dE < eps0 and |z'| < r0 (Eqs. S30, S61) */
  double b_th, eps1;          /* restart S62a: alpha > 0, |b| < b_th, dE < eps1        */
  double x_th1, x_th2;        /* restart S62b: |x| < x_th1 or |x| > x_th2              */
  double r1;                  /* restart S62c: |z'| > r1 and t > 0                     */
  int max_cycle;              /* steps per segment before a forced restart             */
  int max_steps;              /* sigma builds per root before SBCI_ENOCONV             */
  int precision;              /* first phase: SBCI_F64 (FP64 only), SBCI_F32 (FP32 then
                                 FP64) or SBCI_BF16 (BF16, FP32, then FP64)           */
  double mix_eps0, mix_r0;    /* low-precision phase ends at dE < mix_eps0 and |z'| < mix_r0 */
  int mix_stall;              /* ... or after this many steps without an energy decrease */
  double precond_floor;       /* |D - E0| is floored at this value (default 1e-8)      */
  double lindep;              /* Gram-Schmidt radicand / Ritz coefficient guard (1e-14) */
  int max_space;              /* Davidson subspace cap (default 12 + nroots if <= 0)    */
  const double *x0;           /* host [ndet] start vector for root 0, or NULL for the
                                 Section S1.1 start from the lowest diagonal elements */
  double bf16_eps0, bf16_r0;  /* SBCI_BF16: BF16 phase hands over to FP32 at these   */
  int max_cycle2;             /* SBCI2 steps per segment before a forced restart (10,
                                 Section S2.5)                                          */
  int s78_printed;            /* SBCI2: 1 projects the images off the converged roots
                                 with E_c x_c, as Eq. S78 is printed; 0 (default) with
                                 the image H x_c carried to each root's acceptance
                                 (an accepted x_c keeps a residual, which E_c x_c
                                 would leave in the images)                             */
  /* Resume (sbci_solve and sbci_begin only; SBCI2, Davidson and the batch
   * form refuse nconv0 != 0).  The solver's state between roots is the set
   * {x_c, E_c} of converged roots (Algorithm 1 deflates against nothing
   * else), so a solve stopped after k roots continues from them: pass the
   * k vectors (e.g. rows of an earlier dev_vecs, copied to the host) and
   * optionally their energies, and root k starts from x0 when given (an
   * earlier iterate) or else from the Section S1.1 start block's vector k,
   * projected off the given roots (Eqs. S4-S5).  The given vectors are
   * orthonormalised in order (Gram-Schmidt, FP64); SBCI_EINVAL if one is
   * zero, not finite or (to lindep) dependent on the earlier ones.
   * energies / dev_vecs / the report count the given roots as roots 0..k-1
   * (their t_converged and resid read 0). */
  int nconv0;                 /* roots already converged, in [0, nroots); 0 = none      */
  const double *xc0;          /* host [nconv0][N_det] FP64 converged vectors, row-major */
  const double *ec0;          /* host [nconv0] their energies, or NULL: the Rayleigh
                                 quotients x_c^T H x_c (one FP64 sigma each)            */
} sbci_opts;

typedef struct sbci_report {
  int nroots_converged;
  int nsteps;                 /* SBCI steps (or Davidson iterations) over all roots    */
  int nrestarts;
  int64_t nsigma_f64;         /* sigma vector applications in FP64                     */
  int64_t nsigma_low;         /* ... in the low-precision form                          */
  double seconds;             /* wall time of the solve, seconds                        */
  double t_converged[16];     /* seconds from solve start until root i converged        */
  double resid[16];           /* final |z'| (SBCI) or |r| (Davidson) of root i          */
  int64_t peak_vector_bytes;  /* device bytes of solver vectors at the peak             */
  int64_t nsigma_bf16;        /* of nsigma_low, those with the BF16-MFMA contraction    */
} sbci_report;

/* One record per SBCI step (filled when tracing is on, sbci_set_trace). */
typedef struct sbci_step_info {
  int root, segment, t;
  int precision;              /* sbci_dtype of the sigma used in this step             */
  double E, dE, dz, b, c, k, xnorm;
  double seconds;             /* since the solve started                                */
  int reason;                 /* 0 none, 1 converged, 2 S62a, 3 S62b, 4 S62c,
                                 5 max_cycle, 6 rank guard, 7 coefficient guard,
                                 8 hand-over to the next precision (FP64 refinement),
                                 9 hand-over before a low-precision step whose new
                                   iterate would have norm |k| < x_th1               */
} sbci_step_info;

void sbci_default_opts(sbci_opts *opt);
const char *sbci_last_error(void);

/* Build a context: validates the integrals, uploads them and builds on the
 * device the alpha/beta strings, single-excitation tables, same-spin
 * Hamiltonian lists, pair-scatter tables and the diagonal D.
 *   norb in [1, 63]; 0 <= nalpha, nbeta <= norb;
 *   h1  host [norb][norb] row-major, symmetric to 1e-12 * max|h|;
 *   eri host [norb]^4 chemists' (pq|rs), 8-fold symmetric to 1e-12 * max|eri|.
 * Errors: SBCI_EINVAL (sizes, symmetry, NULL), SBCI_ENOMEM, SBCI_EDEVICE. */
int sbci_create(int norb, int nalpha, int nbeta, const double *h1, const double *eri,
                sbci_ctx **out);
int sbci_destroy(sbci_ctx *ctx);

/* A context restricted to the determinants of one irreducible representation
 * of an abelian point group with irreps 0..7 multiplying by XOR (D2h and its
 * subgroups).  Every instance of the paper is solved inside one irrep (the
 * IRep column of the Section S3.1 table); the determinant counts printed
 * there are the full C(norb, nalpha) * C(norb, nbeta) products, not the
 * size of that irrep's block.
 *   orbsym host [norb], irrep label 0..7 of each orbital;
 *   irrep  0..7, the irrep of the states sought.
 * A string's irrep is the XOR of its occupied orbitals' labels and |Ia, Ib>
 * has irrep irr(Ia) ^ irr(Ib).  Vectors of this context (sigma's c and
 * sigma, the solvers' vectors, sbci_hdiag) hold only the N_det =
 * sum_a n_alpha(a) * n_beta(a ^ irrep) determinants of the irrep, as blocks
 * a = 0..7 of [alpha strings of irrep a] x [beta strings of irrep a ^ irrep]
 * (row-major, strings in ascending mask order inside their irrep), one
 * block after another; sbci_sym_blocks reports the block shapes.  The
 * integrals must be totally symmetric: entries that break the symmetry must
 * be below 1e-10 of the largest entry (they are left out).  sigma runs in
 * FP64, FP32 and BF16.  The opposite-spin part contracts per class of
 * orbital pairs (the irrep of E_pq).  SBCI_OPP_AUTO picks the vector pair
 * form in FP64 and FP32, the faster one at these class sizes, and the MFMA
 * form in BF16.  SBCI_OPP_PAIR forces the vector form (FP64 and FP32), and
 * SBCI_OPP_CLASS_MFMA forces the MFMA form (all three dtypes).  The MFMA
 * form needs every class to hold at most 64 pairs, otherwise SBCI_EINVAL
 * (and with it no BF16 precision form).  The orbital forms are refused by
 * sbci_set_opp_form.  The caller keeps ownership of every host array.
 * Errors: as sbci_create, plus SBCI_EINVAL for labels out of range,
 * integrals that are not totally symmetric, or an irrep with no
 * determinant. */
int sbci_create_sym(int norb, int nalpha, int nbeta, const double *h1, const double *eri,
                    const int *orbsym, int irrep, sbci_ctx **out);

/* Block shapes of a symmetry-blocked context: out[0..7] alpha strings of
 * irrep a, out[8..15] beta strings of irrep a ^ irrep, out[16..23] block
 * offsets.  SBCI_EINVAL for a context without symmetry blocking. */
int sbci_sym_blocks(const sbci_ctx *ctx, int64_t *out /* host [24] */);

/* Use this HIP stream (hipStream_t passed as void*) for all later work; NULL
 * selects the null (legacy default) stream.  A new context uses a
 * non-blocking stream of its own until this is called. */
int sbci_set_stream(sbci_ctx *ctx, void *hip_stream);

/* Sizes: N_det = C(norb, nalpha) * C(norb, nbeta) (the blocked count for a
 * symmetry-blocked context) and the string counts. */
int64_t sbci_ndet(const sbci_ctx *ctx);
int64_t sbci_nstrings(const sbci_ctx *ctx, int spin /* 0 alpha, 1 beta */);

/* Copy a device table into dev_out (which = 0/1: alpha/beta strings as
 * uint64 masks [N_s]; 2/3: alpha/beta single-excitation tables as 8-byte
 * records {int32 J; uint8 p; uint8 q; int8 sign; uint8 0} [N_s][s] with
 * s = m (norb - m + 1): E_pq |I> = sign |J>; per string the m diagonal
 * entries (p = q ascending) come first, then q occupied ascending x p empty
 * ascending).  *bytes receives the size; dev_out may be NULL to query it. */
int sbci_tables(sbci_ctx *ctx, int which, void *dev_out, int64_t *bytes);

/* D[Ia, Ib] = <Ia Ib|H|Ia Ib> into dev_out [N_det] FP64 (the diagonal used by
 * the preconditioner (D - E0 I)^-1 of Eq. 7). */
int sbci_hdiag(sbci_ctx *ctx, double *dev_out);

/* sigma = H c for nvec vectors (the matrix-vector product every SBCI step
 * needs once, Eq. S32).  dev_c, dev_sigma: [nvec][N_det] contiguous, element
 * type double (SBCI_F64) or float (SBCI_F32, SBCI_BF16); they must not
 * overlap.  Asynchronous on the context stream. */
int sbci_sigma(sbci_ctx *ctx, const void *dev_c, void *dev_sigma, int nvec, int dtype);

/* FP64 sigma reproducibility.  on = 1 (the default): the FP64 opposite-spin
 * part accumulates each row of sigma in 64-bit fixed point with integer
 * atomics, under a power-of-two scale set per row from a bound on its
 * partial sums (max |C| over the rows it reads times s_beta times the
 * largest row sum of |(kl|k'l')|), so an FP64 sigma is the same to the last
 * bit on every call; every other part sums in a fixed order.  This holds for
 * unblocked and point-group blocked contexts, in every opposite-spin form.
 * A row whose scale bound is not finite (a NaN or Inf in a row of c it
 * reads) becomes NaN.  on = 0: FP64 atomics (the order of additions varies;
 * about 10% faster unblocked, 2-3% blocked).  FP32 and BF16 sigma are not
 * covered.  SBCI_EINVAL unless on is 0 or 1. */
int sbci_set_deterministic(sbci_ctx *ctx, int on);

/* sbci_sigma for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result, with the beta part's transposed operand and result in a
 * 64 MiB device array inside the library (one per device, held until the
 * process ends) instead of workspaces allocated on first use.  This call
 * makes no hipMalloc, hipFree or other allocating call.  Limits, refused
 * with SBCI_EINVAL before any launch: dtype SBCI_F64 or SBCI_F32;
 * 2 * nvec * N_det * element size (plus, in FP64, 8 * nvec * N_alpha bytes
 * of row maxima; each part rounded up to 256 bytes) at most 64 MiB, so
 * nvec * N_det * element size up to just under 32 MiB; the list same-spin form and
 * the pair opposite-spin form (no dense or orbital forms, whose operands are
 * built on first use); no symmetry blocking.  Every call on a device shares
 * that device's array: calls that overlap on one device (several contexts or
 * streams at once) race.  Asynchronous on the context stream. */
int sbci_sigma_noalloc(sbci_ctx *ctx, const void *dev_c, void *dev_sigma, int nvec, int dtype);

/* The same sigma, synchronously, with HIP events recorded on the context
 * stream around its five kernels; ms_parts (host [5]) receives the elapsed
 * milliseconds of: same-spin alpha lists, opposite-spin MFMA contraction,
 * transpose of c, same-spin beta lists on the transpose, transposed add. */
int sbci_sigma_timed(sbci_ctx *ctx, const void *dev_c, void *dev_sigma, int nvec, int dtype,
                     float *ms_parts);

/* Force the opposite-spin form of later sigma calls (sbci_opp_form value),
 * or SBCI_OPP_AUTO (the default).  A forced form that does not fit this
 * context makes the sigma call fail with SBCI_EINVAL.  Both forms compute
 * the same sigma up to rounding order. */
int sbci_set_opp_form(sbci_ctx *ctx, int form);

/* The opposite-spin form sigma calls of this dtype use (SBCI_OPP_PAIR or
 * SBCI_OPP_ORBITAL) into *form; SBCI_EINVAL if no form fits. */
int sbci_get_opp_form(sbci_ctx *ctx, int dtype, int *form);

/* Force the same-spin form of later sigma calls (sbci_same_form value), or
 * SBCI_SAME_AUTO (the default).  The dense form keeps an N_s x N_s operator
 * per spin and precision (built on first use) and is limited to N_s <= 32768
 * strings; beyond that a forced dense form makes sigma fail with
 * SBCI_EINVAL.  For the SBCI_BF16 sigma the dense form runs on BF16 MFMA
 * with FP32 accumulation (the operator's diagonal stays FP32) and is the
 * automatic choice from 1024 to 32768 strings. */
int sbci_set_same_form(sbci_ctx *ctx, int form);

/* The same-spin form (SBCI_SAME_LISTS or SBCI_SAME_DENSE) sigma calls of
 * this dtype use for spin 0 (alpha) or 1 (beta), into *form. */
int sbci_get_same_form(sbci_ctx *ctx, int spin, int dtype, int *form);

/* SBCI1 (Algorithm 1 with Sections S1.1-S1.5) for the lowest nroots states.
 * tol > 0 overrides opt: eps0 = tol, r0 = sqrt(tol) (the paper's two pairs,
 * 1e-10/1e-5 and 1e-8/1e-4, both have r0 = sqrt(eps0)); tol <= 0 keeps opt.
 * opt may be NULL (defaults).  energies: host [nroots]; dev_vecs: device
 * [nroots][N_det] FP64 normalised eigenvectors, or NULL; rep may be NULL.
 * Returns SBCI_ENOCONV if a root hits max_steps (outputs hold the last
 * iterates). */
int sbci_solve(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt,
               double *energies, double *dev_vecs, sbci_report *rep);

/* Step-level interface to the same solver: sbci_begin prepares root 0,
 * each sbci_step performs one SBCI step (one sigma build) and fills *info;
 * *done becomes 1 once all roots have converged.  sbci_finish copies the
 * results like sbci_solve. */
int sbci_begin(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt);
int sbci_step(sbci_ctx *ctx, sbci_step_info *info, int *done);
int sbci_finish(sbci_ctx *ctx, double *energies, double *dev_vecs, sbci_report *rep);

/* Checkpoint of a step-level solve: the current iterate x of the root being
 * solved (root index = roots converged so far), unnormalised, as FP64 into
 * dev_x (device [N_det]); from the running precision's copy in a
 * low-precision phase.  At a step boundary the solver's state is x (X = H x
 * is recomputed, Eq. S32) and the converged pairs {x_c, E_c}
 * (sbci_finish mid-solve writes those and returns SBCI_ENOCONV; stepping
 * can go on after it).  A new solve with opts x0 = x and nconv0 / xc0 / ec0
 * = the pairs continues from that point.  Synchronous.  SBCI_EINVAL if no
 * SBCI1 solve was begun on ctx (sbci_begin or sbci_solve), after
 * sbci_solve2 or sbci_davidson, or once every root has converged. */
int sbci_iterate(sbci_ctx *ctx, double *dev_x);

/* Per-step trace of the last solve (tracing on by default): copies up to
 * max records into out (host) and returns the number copied (>= 0). */
int sbci_set_trace(sbci_ctx *ctx, int on);
int sbci_trace(sbci_ctx *ctx, sbci_step_info *out, int max);

/* Progress of long solves: fn(info, user) is called on the host thread that
 * runs the solve, after every step of sbci_solve / sbci_step / sbci_solve2
 * (the record the trace would hold, whether or not tracing is on) and after
 * every iteration of sbci_davidson (root = lowest unconverged root, t = the
 * iteration, E its Ritz value, dE its change, dz its residual norm, reason 1
 * once every root has converged).  fn = NULL removes it.  The callback must
 * not call into the library with this context. */
typedef void (*sbci_progress_fn)(const sbci_step_info *info, void *user);
int sbci_set_progress(sbci_ctx *ctx, sbci_progress_fn fn, void *user);

/* Block Davidson-Liu on the same sigma (the paper's baseline method):
 * block = nroots, preconditioner (D - theta_k)^-1, subspace cap max_space
 * (12 + nroots by default), collapse to the Ritz vectors.  Same outputs and
 * thresholds as sbci_solve; always FP64. */
int sbci_davidson(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt,
                  double *energies, double *dev_vecs, sbci_report *rep);

/* SBCI2 (Algorithm 2; Supplementary Sections S2.1-S2.5): the states of a
 * pair (alpha, alpha + 1) are updated together, a 6 x 6 Rayleigh-Ritz problem
 * in the canonically orthonormalised span of x, y, z of both states per step
 * (two sigma applications); state alpha is accepted on Eq. S127, restarts
 * follow Eqs. S130a-c and max_cycle2; the highest state is finished by SBCI1
 * (Fig. 1B).  Start vectors: Section S2.2.  Arguments, outputs, errors and
 * the trace as for sbci_solve; opt->x0 is ignored.  opt->precision selects
 * the precision form: each pair starts on the BF16-MFMA or FP32 sigma (its
 * vectors and reductions stay FP64), hands over at the thresholds of
 * sbci_opts with X recomputed (trace reason 8), and a state is accepted only
 * in FP64; the highest state runs SBCI1's ladder.  energies[i] / dev_vecs
 * row i are state i. */
int sbci_solve2(sbci_ctx *ctx, int nroots, double tol, const sbci_opts *opt,
                double *energies, double *dev_vecs, sbci_report *rep);


/* ------------------------------------------------------------------------
 * Batching form: many independent instances (each its own norb, n_alpha,
 * n_beta, integrals and number of roots) solved by SBCI1 in one
 * persistent-kernel launch captured in a hipGraph.  One workgroup runs the
 * whole SBCI1 state machine of one instance (Algorithm 1 with Sections
 * S1.1-S1.5: start vectors, steps, restarts, deflation against the lower
 * roots, the precision hand-overs of sbci_solve); workgroups take instances
 * from a device queue.  An instance whose estimated work exceeds the
 * balanced share of one workgroup runs on a team of up to max_team
 * co-resident workgroups that split its rows and meet at bounded barriers
 * (the device should not be shared with other work during the solve: a team
 * that waits longer than config.team_wait_us, one second by default, ends its
 * instance with SBCI_EDEVICE).
 * Limits per instance: 1 <= norb <= 10 (at most 252 strings per spin),
 * 1 <= nroots <= min(4, N_det).
 */
typedef struct sbci_batch sbci_batch;

/* Launch shape of the persistent kernel (chosen by sbci_batch_tune). */
typedef struct sbci_batch_config {
  int threads;    /* workgroup size: 256, 512 or 1024                          */
  int wg_per_cu;  /* persistent workgroups per compute unit: 1..4              */
  int order;      /* queue order: 0 = largest estimated work first, 1 = input  */
  int k_panel;    /* K panel of the same-spin MFMA products in LDS: 8 or 16    */
  int max_team;   /* workgroups per instance at most: 1 (no teams) .. 4; 0 = 4 */
  int team_wait_us; /* bound of a team barrier wait in microseconds; 0 = 1 s.
                       A team whose wait exceeds it ends its instance with
                       SBCI_EDEVICE                                             */
  int queue_reserve; /* teams take at most slots - slots / queue_reserve of the
                        resident workgroup slots, the rest start on the queue:
                        2..64; 0 = 16                                           */
} sbci_batch_config;

typedef struct sbci_batch_report {
  double seconds;            /* device time of the graph launch (HIP events)    */
  double span_seconds;       /* first instance start to last instance end,
                                from the device real-time counter              */
  int64_t nsigma_f64;        /* sigma applications, summed over instances       */
  int64_t nsigma_low;
  int64_t det_sigma;         /* sum over instances of N_det x sigma applications */
  int64_t nsteps, nrestarts; /* summed over instances                           */
  int ninst_converged;       /* instances with status SBCI_OK                   */
  int threads, wg_per_cu, order, k_panel, max_team, team_wait_us;  /* the shape used */
  int nteams;                /* instances run by a team of workgroups          */
  int team_workgroups;       /* workgroups in those teams                       */
  int team_timeouts;         /* team instances ended by the wait bound
                                (status SBCI_EDEVICE; the call then returns
                                SBCI_EDEVICE with every output written)         */
  int queue_reserve;         /* the shape used (continued)                      */
} sbci_batch_report;

/* Per-instance outcome of a batch solve (times from the device real-time
 * counter, relative to the earliest instance start). */
typedef struct sbci_batch_inst {
  int status;                /* sbci_status of this instance                    */
  int nroots_converged;
  int nsteps, nrestarts, nsigma_f64, nsigma_low;
  double t_start, t_end;     /* seconds                                         */
  double resid[4];           /* |z'| at convergence of each root (NaN if none)   */
  double t_same, t_opp;      /* seconds in sigma: one-electron + same-spin part,
                                opposite-spin part                              */
} sbci_batch_inst;

/* Builds every instance's tables (as sbci_create does for one) on the
 * current device.  norb, nalpha, nbeta: host [ninst]; h1[i], eri[i]: host
 * pointers to instance i's integrals in the layout of sbci_create (read
 * during the call only).  EINVAL for a NULL argument, ninst < 1 or an
 * instance outside the limits above. */
int sbci_batch_create(int ninst, const int *norb, const int *nalpha, const int *nbeta,
                      const double *const *h1, const double *const *eri, sbci_batch **out);
int sbci_batch_destroy(sbci_batch *b);
int64_t sbci_batch_ndet(const sbci_batch *b, int inst);   /* -1 for a bad index */

/* Solves every instance: nroots host [ninst]; tol, opt as for sbci_solve
 * (opt->x0 must be NULL; opt->precision selects the FP64 or mixed form);
 * cfg NULL = the last tuned shape, else a default shape.  energies: host,
 * the roots of instance 0, then instance 1, ... (sum of nroots entries; NaN
 * for a root that was not reached); info: host [ninst] per-instance
 * outcome, or NULL.  Returns SBCI_ENOCONV / SBCI_ENUMERIC if any
 * instance ended so (the outputs are still written). */
int sbci_batch_solve(sbci_batch *b, const int *nroots, double tol, const sbci_opts *opt,
                     const sbci_batch_config *cfg, double *energies, sbci_batch_inst *info,
                     sbci_batch_report *rep);

/* Autotuner: times full batch solves over a candidate set of launch shapes
 * (workgroup size x residency, then queue order and K panel around the
 * best) with HIP events, keeps the fastest for later sbci_batch_solve calls
 * and writes it to best.  ms, cand: host arrays of capacity *ncand (or
 * NULL) receive each candidate's time and shape; *ncand returns the number
 * of candidates tried. */
int sbci_batch_tune(sbci_batch *b, const int *nroots, double tol, const sbci_opts *opt,
                    sbci_batch_config *best, double *ms, sbci_batch_config *cand, int *ncand);

/* Copies the converged FP64 vectors of instance inst from the last solve to
 * dev_out ([nconv][N_det], nconv = roots reached). */
int sbci_batch_vectors(sbci_batch *b, int inst, double *dev_out);

#ifdef __cplusplus
}
#endif
#endif /* SBCI_H */
