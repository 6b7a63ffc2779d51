/*
 * mahi.h - C ABI of the MI355X MAHI library (libmahi.so).
 *
 * Multipole-Accelerated Hamiltonian Interpolation (Kohnke, Briand, Kutzner,
 * Grubmueller, arXiv 2410.01754): one fast-multipole Coulomb evaluation of the
 * lambda-tilde scaled charges in a cubic box, followed by a per-site correction
 * that turns the charge-scaled result into the exact Hamiltonian-interpolation
 * (HI) energy, atom forces and per-form derivatives dE/dlambda-tilde.
 *
 * Problem statement (paper, Theory):
 *   - N point charges in a cube of edge L, periodic in all three directions
 *     (eq nbody_periodic) or with open boundaries;
 *   - M titratable sites; site s owns n_s atoms and f_s forms, form r giving
 *     those atoms the charges q^(s,r) (section "Hamiltonian Interpolation
 *     Formulation");
 *   - per-form weights lambda-tilde (eq lambda_tilde, constraint eq
 *     constraint); site-atom charges become qt = sum_r lt_r q^(s,r);
 *   - outputs: the HI energy of the general formulation (eq iter_ham_lambda),
 *     forces F = -dE/dx and dE/dlambda-tilde per form (the per-form part of the
 *     mapping K of section "Calculation of Forces on lambda Particles").
 * Periodic energies are Ewald energies with tin-foil boundaries (section
 * "Multipole-Accelerated Hamiltonian Interpolation", eq approx_nbody_periodic)
 * and, for a charged cell, a uniform neutralising background.
 *
 * Conventions
 *   Units: nm and elementary charges; energies are scaled by coulomb_k
 *     (default 138.9354576 kJ mol^-1 nm e^-2).
 *   Ownership: the caller owns every array it passes.  mahi_create copies the
 *     charges and site tables; no call keeps a pointer after it returns.  The
 *     context owns all device memory (allocated once, in mahi_create).
 *   Errors: every call returns a mahi_status.  Argument checks run before any
 *     device work, so invalid input never reaches the GPU; on error no output
 *     is written.  mahi_last_error() gives a message for the last failure on a
 *     context.  No call aborts the process.
 *   Threads: one context may be used by one host thread at a time.
 *   Determinism: identical inputs give bit-identical outputs (no floating-point
 *     atomics; all reductions run in a fixed order).
 */
#ifndef MAHI_H
#define MAHI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mahi_ctx mahi_ctx; /* opaque; owned by the library */

typedef enum {
  MAHI_OK = 0,
  MAHI_EINVAL = -1,        /* bad argument (null pointer, size, non-finite value, bad site table) */
  MAHI_ENOMEM = -2,        /* host or device allocation failed */
  MAHI_EDEVICE = -3,       /* HIP runtime error or no usable gfx950 device */
  MAHI_ERANGE = -4,        /* value outside the supported range (order, depth, forms, atoms per site) */
  MAHI_ESTATE = -5,        /* call out of order (mahi_eval before mahi_set_lambda) */
  MAHI_EUNSUPPORTED = -6   /* feature not available in this build */
} mahi_status;

/* Simulation cell: a cube (the paper's method supports cubic boxes only). */
typedef struct {
  double edge;   /* periodic: cube edge L > 0 (nm).  open: ignored; the root
                    cube of the octree is the bounding cube of each call's
                    coordinates */
  int periodic;  /* 1: periodic in x, y, z;  0: open boundaries */
} mahi_box;

/* Titratable sites.  Site s owns atoms_per_site[s] atoms (indices into the
 * N atoms, pairwise disjoint over all sites) and forms_per_site[s] forms.
 * form_charges holds, site after site, the charges of form 0 for every atom
 * of the site, then form 1, ... (form-major, atom-minor), in e.            */
typedef struct {
  int32_t n_sites;                /* M >= 0 */
  const int32_t *forms_per_site;  /* [M], each in 1..16 */
  const int32_t *atoms_per_site;  /* [M], each in 1..32 */
  const int32_t *site_atoms;      /* [sum atoms_per_site] */
  const double *form_charges;     /* [sum forms_per_site * atoms_per_site] */
} mahi_sites;

typedef struct {
  int order;         /* multipole order p: degrees 0..p, (p+1)^2 real coefficients; 1..20 */
  int depth;         /* octree depth d (8^d leaves); 0..7 */
  int precision;     /* 32: float32 arithmetic in the bulk FMM (lattice, site
                        correction and reductions stay float64);
                        64: float64 everywhere */
  double coulomb_k;  /* energy scale; <= 0 selects 138.9354576 */
  void *hip_stream;  /* hipStream_t to run on; NULL = a stream created by the context */
} mahi_opts;

/* mahi_eval flags */
#define MAHI_DEVICE_IO 1u /* every pointer in mahi_eval_args is device memory and the
                             call returns without waiting for the GPU (the caller
                             synchronises the stream) */

typedef struct {
  const void *xyz;    /* [N][3] positions (nm); float when precision = 32, double when 64.
                         periodic: any finite values (wrapped into the cell);
                         open: any finite values */
  double *energy;     /* [1] HI energy; may be NULL */
  void *forces;       /* [N][3] F = -dE/dx, same type as xyz; may be NULL */
  double *dvdl;       /* [sum forms] dE/dlambda-tilde per form, site-major; may be NULL */
  void *potential;    /* [N] coulomb_k * charge-scaled potential at each atom (the
                         potential of the charge-scaled Hamiltonian, including
                         the atom's own periodic images), same type as xyz; may be NULL */
  uint32_t flags;     /* 0 or MAHI_DEVICE_IO */
  /* Derivatives for fitting and for charge interpolation (all may be NULL):  */
  double *dedq;       /* [sum forms * atoms] dE/dq^(s,r)_i for every form charge, in the
                         layout of mahi_sites.form_charges.  Every weight and form
                         charge is an independent variable of the general
                         formulation (eq iter_ham_lambda):
                         dE/dq^(s,r)_i = coulomb_k lt_r (V_i + sum_{j in s} Phi_ij (q^(s,r)_j - qt_j)) */
  double *energy_qi;  /* [1] charge-interpolated (QI) energy coulomb_k/2 qt.Phi.qt: the
                         energy of the scaled charges alone, before the site
                         correction (section "Differences Between Hamiltonian and
                         Charge Interpolation") */
  double *dvdl_qi;    /* [sum forms] dE_QI/dlambda-tilde = coulomb_k sum_{i in s} q^(s,r)_i V_i */
} mahi_eval_args;

/* Create a context for N point charges in a cube (periodic: eq nbody_periodic;
 * open: the plain Coulomb sum) with M titratable sites whose forms give their
 * atoms different charges (section "Hamiltonian Interpolation Formulation").
 * Validates everything, chooses no parameters on its own, generates the
 * translation and lattice tables in float64 on the host, and allocates all
 * device buffers.  charges[N] are the environment charges; entries at site
 * atoms are ignored.  sites may be NULL (plain FMM).  Errors: MAHI_EINVAL for
 * NULL pointers, non-finite values or a bad site table (atom index out of
 * range, atoms shared by two sites); MAHI_ERANGE for sizes outside the limits
 * of mahi_opts and mahi_sites; MAHI_EDEVICE without a gfx950 device;
 * MAHI_ENOMEM when an allocation fails.  *out is NULL on error.            */
mahi_status mahi_create(mahi_ctx **out, const mahi_box *box, int64_t n_atoms, const double *charges,
                        const mahi_sites *sites, const mahi_opts *opts);

/* Set the per-form weights lambda-tilde[sum forms] (site-major, then form;
 * eq lambda_tilde, whose sum over the forms of a site is 1 by eq constraint).
 * Values are used as given (no renormalisation; the general formulation, eq
 * iter_ham_lambda, stays exact off the simplex).  Non-finite values give
 * MAHI_EINVAL and leave the context unchanged.  Runs the charge scaling
 * qt = sum_r lt_r q^(s,r) at the site atoms on the device and waits for it.  */
mahi_status mahi_set_lambda(mahi_ctx *ctx, const double *lambda_tilde);

/* One evaluation: octree build, P2M, M2M, periodic lattice, M2L, L2L, L2P and
 * P2P on the scaled charges (the work of the upper tree levels, M2M included,
 * on a second stream of the context, beside the M2L of the two deepest levels),
 * then the per-site correction (paper, section "Multipole-Accelerated
 * Hamiltonian Interpolation": eqs correction_scheme to C_B and the execution
 * order of section "Execution of MAHI").
 * With forces = NULL only the potential is formed (the near field and the
 * local expansions without their gradients): the energy, dvdl, dedq and the
 * charge-interpolation outputs need nothing else.
 * Without MAHI_DEVICE_IO the call copies host inputs and outputs and waits
 * for the GPU.  Errors: MAHI_EINVAL (NULL args or xyz, unknown flags,
 * non-finite host coordinates), MAHI_ESTATE before mahi_set_lambda (nothing is
 * written), MAHI_EDEVICE for a HIP error.                                   */
mahi_status mahi_eval(mahi_ctx *ctx, const mahi_eval_args *args);

/* Replace the charges of every form of every site (same layout and checks as
 * mahi_sites.form_charges at creation; the site atoms and form counts stay).
 * The scaled charges are formed again from the current lambda-tilde (when
 * one has been set).  For fitting form charges with dedq.  Non-finite values
 * give MAHI_EINVAL and leave the context unchanged.                        */
mahi_status mahi_set_form_charges(mahi_ctx *ctx, const double *form_charges);

/* Solver-agnostic site correction (paper, section "GROMACS performance with
 * FMM and constant pH": the corrections act on a charge-scaled potential V computed by
 * any method that is accurate enough, e.g. particle-mesh Ewald).  Given V at
 * every atom from another solver, this runs only the per-site correction of
 * mahi_eval (eqs correction_scheme to C_B) on the context's sites:
 *   E_HI  = E_QI + *energy,   F_HI = F_QI + (the correction added to forces),
 *   dvdl, dedq as in mahi_eval (they need V at the site atoms only).
 * The site kernel is the one mahi_eval uses: periodic pairs take the 27
 * nearest images plus the lattice remainder of order `order` (with the r^2
 * term of a tin-foil, neutralised cell), i.e. the Ewald pair potential.
 * No octree work is done; the context's depth is irrelevant here.           */
typedef struct {
  const void *xyz;        /* [N][3] positions (nm), type as mahi_eval; only site atoms are read */
  const void *potential;  /* [N] coulomb_k * V_i (the charge-scaled potential at each atom,
                             including the atom's own periodic images, in the form of
                             mahi_eval's potential output); only site atoms are read */
  double *energy;         /* [1] E_HI - E_QI; may be NULL */
  void *forces;           /* [N][3] F_HI - F_QI is ADDED at site atoms (other entries are
                             not touched); may be NULL */
  double *dvdl;           /* [sum forms] dE_HI/dlambda-tilde; may be NULL */
  double *dedq;           /* [sum forms * atoms] dE_HI/dq^(s,r)_i; may be NULL */
  uint32_t flags;         /* 0 or MAHI_DEVICE_IO */
} mahi_correct_args;
mahi_status mahi_correct(mahi_ctx *ctx, const mahi_correct_args *args);

/* mahi_correct without any allocation and without the context's scratch, for
 * callers that cannot allocate device memory at the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same operation, kernels and results as mahi_correct; args->flags must be
 * MAHI_DEVICE_IO (device pointers only; the call never waits for the GPU).
 * Its scratch (per-site energies, plus the site pass's work arrays when a
 * site exceeds local memory: 8 doubles per site rounded up to 256 bytes, plus
 * 8 * (4 maxa^2 + maxa K + 5 maxf K) bytes per site in that case, K =
 * (order+1)^2) lives in a static device array of 8 MiB that every device
 * holds for the life of the process; calls needing more return MAHI_ERANGE
 * and do nothing.  All calls on one device share that array, so calls that
 * overlap on one device (other threads, other streams) race; calls ordered on
 * one stream do not.  Nothing in it needs to start at zero: every call writes
 * what it reads.  MAHI_EINVAL for NULL args, xyz or potential and for flags
 * other than MAHI_DEVICE_IO; MAHI_ESTATE before mahi_set_lambda.            */
mahi_status mahi_correct_noalloc(mahi_ctx *ctx, const mahi_correct_args *args);

/* Binary multi-form sites (paper, appendix: eqs lambda_list and
 * one_site_lambda and the mapping of derivatives that follows them; section
 * "Calculation of Forces on lambda Particles").  A site with 2^L forms is
 * driven by L original lambdas; form r gets
 *   lt_r = prod_k (lambda_k if bit k of r is set, else 1 - lambda_k)
 * (least significant bit = lambda_0), and
 *   dE/dlambda_k = sum_r s(r,k) f(r,k) dE/dlt_r
 * with s = +1 when bit k of r is set, -1 otherwise, and f the product of the
 * other L-1 factors of lt_r.  Host only; n_lambda in 1..4 (2..16 forms);
 * MAHI_EINVAL for NULL pointers or non-finite values.                       */
mahi_status mahi_lambda_tilde(int n_lambda, const double *lambda, double *lambda_tilde /* [2^n_lambda] */);
mahi_status mahi_dlambda(int n_lambda, const double *lambda, const double *dvdl /* [2^n_lambda] */,
                         double *dlambda /* [n_lambda] */);

/* Batched evaluation of many systems (small systems leave most of the GPU
 * idle in a single evaluation; the paper's small-system regime, sections
 * "Scaling with Number of Particles" and "Performance").  A batch holds n
 * distinct contexts of one device and evaluates them together; later work on
 * `hip_stream` (the batch's origin stream, NULL = a stream the batch creates)
 * sees every output.  flags:
 *   0: every call forks from the origin stream, runs each context's own
 *      evaluation on that context's streams and joins back (outputs identical
 *      to evaluating each context alone);
 *   MAHI_BATCH_PACKED: every stage of the evaluation is one launch over all
 *      systems (octree build over the concatenated atoms, M2L of every level
 *      of every system together, ...), on the origin stream only; the batch
 *      owns the evaluation buffers (the contexts give their tables, charges,
 *      sites and geometry).  Needs float32 periodic contexts of one order
 *      whose sites fit in local memory (else MAHI_EUNSUPPORTED).  Above order
 *      8 the near field uses the leading part of the leaf-local coordinates
 *      only (no rounding residuals: for orders of production accuracy).
 *      Results agree with single evaluations up to the summation order of
 *      the M2L operator ranges;
 *   MAHI_BATCH_PACKED | MAHI_BATCH_GRAPH: the packed launches are captured once
 *      into a HIP graph and replayed (captured again when a pointer in args
 *      changes; new weights or form charges need no new capture).
 *   MAHI_BATCH_GRAPH alone returns MAHI_EUNSUPPORTED.
 * The contexts stay owned by the caller and must outlive the batch; while in
 * a batch they may still be used alone, but not concurrently with it.      */
#define MAHI_BATCH_GRAPH 1u
#define MAHI_BATCH_PACKED 2u
typedef struct mahi_batch mahi_batch;
mahi_status mahi_batch_create(mahi_batch **out, mahi_ctx *const *ctxs, int n_ctx, int flags, void *hip_stream);
/* args[n_ctx], each with MAHI_DEVICE_IO (device pointers; the call returns
 * without waiting).  Every context must have its lambda-tilde set and no stage
 * profiling open.  MAHI_EINVAL for host-memory arguments.                   */
mahi_status mahi_batch_eval(mahi_batch *b, const mahi_eval_args *args);
void mahi_batch_destroy(mahi_batch *b);
const char *mahi_batch_last_error(const mahi_batch *b);

/* Parameter choice for one system (host only, no device work).  order: the
 * smallest p whose modelled relative RMS error of forces and dE/dlambda-tilde
 * is at most target_rel_err:
 *   err(p) = 1.75e-4 * 0.41^(p-8)  sites of extent <= 1 nm,
 *   err(p) = 5.0e-4  * 0.40^(p-8)  larger or unknown (site_extent < 0) extent,
 * envelopes with a margin of order sweeps of this library against Ewald sums
 * on water boxes of 900..60,000 atoms with clustered and spread sites (a
 * spread site's intra-site pairs lie in the far field).  The per-site
 * tangent dE/dlambda-tilde_r - dE/dlambda-tilde_0 (the lambda forces) of
 * systems with a few sites scatters up to twice these values.  site_extent: the largest
 * distance between two atoms of one site (nm).  depth: the d in 0..7 that
 * minimises a cost model of one evaluation (near-field pairs, the serial near
 * field of one crowded leaf, M2L translations scaled by (p+1)^4, and a
 * per-level latency; constants measured on MI355X) for n_atoms spread evenly
 * in the cube.  precision 32 cannot reach targets below 2e-5 (float32
 * rounding), 64 not below 2e-8 (order 20): MAHI_ERANGE.                     */
mahi_status mahi_autotune(int periodic, double edge, int64_t n_atoms, int precision, double target_rel_err,
                          double site_extent, int *order, int *depth);

/* Measured choice of the launch shapes of one context (device work; blocks
 * until done).  Times `reps` evaluations (after one warm-up each) of the
 * positions `xyz` (device memory, the context's precision, [n_atoms][3], as
 * with MAHI_DEVICE_IO) for each candidate and keeps the fastest:
 *   - float32 contexts: the number of operator ranges of the main M2L launch
 *     (1, 2, 3, 4, 5, 6 or 8; the default comes from a makespan model),
 *   - the most near-field targets per lane (1, 2 or 3; default 3; each leaf
 *     still picks its own count up to this cap by lane utilisation).
 * Later evaluations of the context use the choices, which change results only
 * by rounding (another grouping of the same sums).  Writes the choices to
 * *m2l_ranges (0 for float64) and *p2p_targets when those are not NULL.
 * The evaluations write the context's own buffers, not the caller's.
 * Errors: MAHI_EINVAL (NULL ctx or xyz), MAHI_ERANGE (reps outside 1..1000),
 * MAHI_ESTATE (lambda-tilde not set, or stage profiling open), MAHI_EDEVICE;
 * on an error the context keeps its previous choices.                        */
mahi_status mahi_tune(mahi_ctx *ctx, const void *xyz, int reps, int *m2l_ranges, int *p2p_targets);

/* Release every host and device resource of the context (NULL is allowed). */
void mahi_destroy(mahi_ctx *ctx);

const char *mahi_strerror(mahi_status s);
const char *mahi_last_error(const mahi_ctx *ctx);

/* The hipStream_t the context's evaluations run on (mahi_opts.hip_stream, or
 * the stream the context created when that was NULL), for callers that order
 * their own work with MAHI_DEVICE_IO evaluations through events.            */
mahi_status mahi_get_stream(const mahi_ctx *ctx, void **stream);

/* Sizes a context was created with: n_atoms, n_sites, total forms, order,
 * depth, precision (NULL pointers are skipped).                              */
mahi_status mahi_info(const mahi_ctx *ctx, int64_t *n_atoms, int32_t *n_sites, int32_t *n_forms, int *order,
                      int *depth, int *precision);

/* Host-only checks of the float64 operator tables against direct sums
 * (translations, lattice coefficients); no device is touched.  Writes the
 * largest relative deviation found to *max_rel_err.                         */
mahi_status mahi_host_selftest(int order, double *max_rel_err);

/* Device check of the matrix-core tile layouts used by the translation
 * kernels: multiplies random matrices with each kernel's tile code (float32:
 * the 32x32x2 tile and the 16x16x4 tile of the M2L kernel for orders up to 8;
 * float64: the 16x16x4 tile) and compares with a host product.  precision 32
 * or 64.  Writes the largest relative error.                               */
mahi_status mahi_device_selftest(int precision, double *max_rel_err);

/* Stage timing.  Between mahi_profile_begin and mahi_profile_end the library
 * records HIP events on its stream at every stage boundary of up to max_evals
 * evaluations (no extra synchronisation).  mahi_profile_end waits for the
 * stream and writes the mean duration in ms of each stage over the recorded
 * evaluations to stage_ms[MAHI_N_STAGES] and their number to *n_evals.
 * Stages: 0 octree build, 1 P2M, 2 M2M into level d-1, 3 upper levels, 4 M2L
 * of the two deepest levels, 5 L2L into the two deepest levels (after joining
 * stage 3), 6 P2P + L2P + outputs, 7 site correction, 8 energy reduction.
 * Stage 3 (lattice charge moments, M2M into levels d-2..0, M2L of the upper
 * levels, the periodic lattice and L2L into the upper levels) runs on a
 * second stream of the context concurrently with stage 4, so the stages add
 * up to more than the evaluation.                                           */
#define MAHI_N_STAGES 9
mahi_status mahi_profile_begin(mahi_ctx *ctx, int max_evals);
mahi_status mahi_profile_end(mahi_ctx *ctx, double *stage_ms, int *n_evals);
const char *mahi_stage_name(int stage);
/* Per-evaluation durations (ms, first to last stage boundary on the context's
 * stream) of the evaluations recorded by the last mahi_profile_begin /
 * mahi_profile_end pair, in order: min(max, recorded) values are written to
 * eval_ms and their number to *n.  MAHI_ESTATE before any profile has ended. */
mahi_status mahi_profile_eval_times(const mahi_ctx *ctx, double *eval_ms, int max, int *n);

/* Test hook: copy an internal buffer of the last evaluation to host memory.
 * which: 0 multipoles (all levels, level 0 first, boxes in Morton order,
 *          (order+1)^2 coefficients each), 1 local expansions (same layout),
 *        2 leaf start offsets (int32, 8^depth + 1), 3 sorted-to-user atom
 *          permutation (int32, N), 4 sorted atoms (leaf-local x, y, z and
 *          scaled charge per atom).
 * Elements are float or double as the context's precision (ints for 2, 3).
 * count is the number of elements to copy; MAHI_ERANGE if it exceeds the
 * buffer.  Waits for the context's stream.                                  */
mahi_status mahi_debug_copy(mahi_ctx *ctx, int which, void *host_out, int64_t count);

#ifdef __cplusplus
}
#endif

#endif /* MAHI_H */
