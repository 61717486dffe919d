/*
 * hfgpe.h -- C ABI of the MI355X Hermite-Fourier GPE time-stepping library.
 *
 * Method: P. Bader and S. Blanes, "Fourier methods for the perturbed harmonic
 * oscillator in linear and nonlinear Schroedinger equations" (arXiv:1007.3470).
 *
 * The library advances, on one AMD Instinct MI355X (gfx950), a batch of
 * independent solutions of the Gross-Pitaevskii equation (Sec. 1)
 *
 *   i psi_t = ( p^2/(2 mu) + sum_j mu omega_j(t)^2 x_j^2 / 2
 *               + eps V_I(x) + sigma(t) |psi|^2 ) psi,      x in R^d, d <= 3,
 *
 * with the Hermite-Fourier splitting methods of Sec. 3: the harmonic part
 * H0(t) (Eq. GP1b) is propagated exactly (Lemma 2) or through the
 * commutator-free / sixth-order Magnus approximations (Eq. CommutatorFree,
 * Sec. 4.2) factored into a chirp, a kinetic phase in Fourier space and a
 * chirp (Theorems 1 and 2); the rest, eps V_I + sigma |psi|^2, is a pointwise
 * phase (Lemma 1).  A step of an m-stage composition (Eq. prod-gen with time
 * frozen in B as in Table "algorithm") costs m FFT pairs because adjacent
 * x-space phases are merged (Eq. leapfrogHF, Eq. prod-genHarmOsc).
 *
 * Conventions
 *   - Grid (Eq. GP1ODE): x_{j,i} = lo_j + i (hi_j - lo_j)/n_j, i = 0..n_j-1,
 *     periodic; n_j a power of two.
 *   - Data: one packed device buffer of interleaved complex values
 *     (float2 for HFGPE_C64, double2 for HFGPE_C128).  Instance k occupies
 *     complex elements [off[k], off[k+1]) (see hfgpe_instance_offsets) in
 *     row-major order with x fastest: element (ix, iy, iz) of instance k is
 *     at off[k] + (iz * n_y + iy) * n_x + ix.  The buffer must be aligned to
 *     its element size (8 bytes for c64, 16 for c128): hfgpe_evolve,
 *     hfgpe_norm and hfgpe_energy return INVALID_ARG otherwise.
 *   - Kinetic wavenumbers k_q = 2 pi / L * (q < n/2 ? q : q - n).
 *   - Every function returns an int status: HFGPE_OK (0) or a negative code.
 *     No exception crosses the ABI.  hfgpe_status_string() names a code.
 *   - Ownership: the caller owns every buffer it passes; the plan owns its
 *     device workspace and releases it in hfgpe_plan_destroy.
 *   - Streams: a plan is bound to one HIP stream (NULL = the default stream)
 *     and is not thread-safe; calls on one plan must not overlap.
 */
#ifndef HFGPE_H
#define HFGPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HFGPE_VERSION_MAJOR 0
#define HFGPE_VERSION_MINOR 3

/* Status codes. */
#define HFGPE_OK 0
#define HFGPE_E_INVALID_ARG (-1)       /* null pointer, bad count, bad scheme ... */
#define HFGPE_E_UNSUPPORTED_SHAPE (-2) /* n_j not a power of two, or too large  */
#define HFGPE_E_SINGULAR (-3)          /* |a_i dt| reaches the first zero of g  */
#define HFGPE_E_NONPOSITIVE_FREQ (-4)  /* omega <= 0, omega_L^2 <= 0, eta^2 <= 0 */
#define HFGPE_E_ALLOC (-5)             /* device or host allocation failed      */
#define HFGPE_E_HIP (-6)               /* a HIP call failed; hfgpe_last_hip_error */
#define HFGPE_E_NONFINITE (-7)         /* a coefficient came out NaN/Inf        */
#define HFGPE_E_NO_DEVICE (-8)         /* no usable gfx950 device               */
#define HFGPE_E_SCRATCH (-9)           /* the request exceeds the static scratch of an
                                          allocation-free entry point           */

/* Largest grid extent per axis supported by the resident kernels. */
#define HFGPE_MAX_N_1D 4096
#define HFGPE_MAX_N_ND 1024

typedef enum { HFGPE_C64 = 0, HFGPE_C128 = 1 } hfgpe_dtype;

/* Rule for the harmonic-oscillator part of each stage (Sec. 2.2, 4.2). */
typedef enum {
    HFGPE_HO_EXACT_CONST = 0, /* Lemma 2; omega must be constant in time        */
    HFGPE_HO_CF4 = 1,         /* Eq. CommutatorFree + Theorem 2 (order 4)       */
    HFGPE_HO_MAGNUS6 = 2,     /* sixth-order Magnus of Sec. 4.2 + Theorem 1     */
    HFGPE_FSPLIT = 3,         /* the Fourier split (i) of Sec. 2.1, the paper's
                                 comparison method: A = p^2/(2 mu) as an exact
                                 drift, the harmonic potential moved into B */
    HFGPE_HO_FUNDAMENTAL = 4  /* the stage's 2x2 classical fundamental matrix
                                 (Eq. HO(t)sol: the HO flow for any omega(t) is
                                 one exponential of E, F, G) integrated
                                 numerically as a product of ho_substeps
                                 sixth-order Magnus sub-steps of Sec. 4.2, then
                                 factored as K(f) D(g) K(e) (Theorem 1's
                                 decomposition applied to the product) */
} hfgpe_ho_rule;

/* Largest number of sub-steps of the HFGPE_HO_FUNDAMENTAL rule. */
#define HFGPE_MAX_HO_SUBSTEPS 256

/* Uniform periodic grid of one instance: the equidistant nodes
 * x_{j,i} = lo_j + i (hi_j - lo_j)/n_j of the Fourier collocation of
 * Eq. GP1ODE (Sec. 1), on which the state is the vector of point values. */
typedef struct {
    int ndim;      /* 1, 2 or 3 */
    int n[3];      /* points per axis, powers of two; axes >= ndim must be 1 */
    double lo[3];  /* box [lo_j, hi_j) per axis */
    double hi[3];
} hfgpe_grid;

/* Time dependence of omega_j(t) and sigma(t). */
typedef enum {
    HFGPE_TF_SIN = 0,    /* v(t)   = v0 (1 + amp sin(freq t + phase))                  */
    HFGPE_TF_SQ_SIN = 1, /* v(t)^2 = v0 (1 + amp sin(freq t + phase)); frequencies only:
                            the modulated squared trap frequency of Sec. 4.2's first
                            example (phase = pi/2 gives the cosine there)            */
    HFGPE_TF_PULSE = 2   /* v(t)   = v0 (1 + amp t / cosh^2(freq (t - phase))): the
                            short pulse of Sec. 4.2's second example (phase is the
                            pulse centre; freq must be non-zero when amp is)          */
} hfgpe_tf_kind;

/* A time-dependent coefficient; zero-initialised kind is HFGPE_TF_SIN, and
 * amp = 0 makes any kind constant (v0, or sqrt(v0) for HFGPE_TF_SQ_SIN). */
typedef struct {
    double v0, amp, freq, phase;
    int kind; /* hfgpe_tf_kind */
} hfgpe_tfunc;

/* A time modulation factor m(t) (Sec. 1 lets the quadratic part M(t) and the
 * perturbation V_I depend on time):
 *   kind HFGPE_TF_SIN:   m(t) = 1 + amp sin(freq t + phase)
 *   kind HFGPE_TF_PULSE: m(t) = 1 + amp t / cosh^2(freq (t - phase))
 *                        (freq non-zero when amp is)
 * Zero-initialised (amp = 0): m = 1, no time dependence. */
typedef struct {
    double amp, freq, phase;
    int kind; /* HFGPE_TF_SIN or HFGPE_TF_PULSE */
} hfgpe_tmod;

/* One separable factor of the perturbation V_I:
 *   v(x) = (c0 + c2 x^2 + c4 x^4) * exp(-x^2 / gs) * cos(k x + phi),
 * the Gaussian factor being omitted when gs <= 0.  V_I(x) = prod_j v_j(x_j). */
typedef struct {
    double c0, c2, c4, gs, k, phi;
} hfgpe_vfactor;

/* Physical parameters of one instance. */
typedef struct {
    double mu;              /* mass, > 0 */
    hfgpe_tfunc omega[3];   /* trap frequency per axis (Eq. GP1b); must stay > 0 */
    hfgpe_tfunc sigma;      /* mean-field coupling sigma(t) (Sec. 1); v0 may be
                               negative (attractive) or zero (linear problem);
                               kind HFGPE_TF_SIN or HFGPE_TF_PULSE */
    double eps;             /* strength of V_I */
    hfgpe_vfactor v[3];     /* V_I factors; set c0 = 1, rest 0, for "no factor" */
    double wcross[3];       /* coupled trap (d >= 2): off-diagonal entries
                               W_xy, W_xz, W_yz of the squared-frequency matrix W(t)
                               with W_jj = omega_j(t)^2, each times its modulation
                               wmod[k]; the trap is then (mu/2) x^T W(t) x, the
                               general quadratic potential x^T M(t) x of Sec. 1.
                               Zero-initialise for a diagonal trap.  A plan
                               whose instances use it must have it on all of them;
                               rules: EXACT_CONST (omega and W constant; one drift
                               per stage), CF4 (W(t) averaged at its Gauss nodes,
                               cross terms included, and applied as its two
                               exponentials: two drifts per stage) and FSPLIT
                               (W(t) at the B times); W(t) must stay positive
                               definite.  The coupled drift k^T G k / 2 is not
                               separable: a stage costs 2d - 1 axis passes. */
    hfgpe_tmod vmod;        /* time factor of the perturbation:
                               eps V_I(x, t) = m(t) eps V_I(x), for the factor form
                               and for a caller's array (hfgpe_set_potential)
                               alike; evaluated at the B times (Table
                               "algorithm") */
    hfgpe_tmod wmod[3];     /* time factors of W_xy, W_xz, W_yz */
} hfgpe_params;

/* BAB composition of Eq. prod-gen: B(b_0) A(a_0) B(b_1) ... A(a_{m-1}) B(b_m).
 * b_0 = 0 gives an ABA-type scheme.  a_i must be non-zero. */
typedef struct {
    int m;                 /* number of A stages = FFT pairs per step, 1..16 */
    const double *a;       /* m stage fractions, sum 1 */
    const double *b;       /* m+1 B weights, sum 1 */
    hfgpe_ho_rule ho_rule;
    int ho_substeps;       /* HFGPE_HO_FUNDAMENTAL: Magnus sub-steps per stage,
                              1..HFGPE_MAX_HO_SUBSTEPS (0 = 16); ignored otherwise */
} hfgpe_scheme;

/* Optional execution settings (zero-initialise for defaults). */
typedef struct {
    int steps_per_launch;  /* 1-D: time steps per resident launch (0 = all of
                              the evolve call up to an internal cap) */
    int plain;             /* 1 = reference schedule: one launch per step per
                              grid-size group (1-D), pass launches only (d-D:
                              use_graph is ignored) */
    int use_graph;         /* 1 = d-D plans replay blocks of 16 steps from a
                              captured hipGraph (a plan on the legacy default
                              stream then runs on a blocking stream of its own,
                              ordered against the default stream) */
    int profile;           /* 1 = bracket every step-kernel launch with HIP
                              events on the plan's stream (hfgpe_profile);
                              2 = also every coefficient-kernel launch */
    int nd_workgroups;     /* d-D: persistent workgroups per axis pass (0 =
                              per pass, as many as the device holds at once:
                              at most 3 per CU, 2 along x and for strided rows
                              under 64 bytes) */
    int nd_generic;        /* d-D: 1 = every axis pass runs the runtime-shaped
                              FFT (by default separable passes along axes of
                              128 .. 1024 points run fixed-shape instances;
                              both give the same bits) */
    int chunk_steps;       /* most steps per coefficient chunk (0 = as many as
                              256 MB of per-stage records hold, at most 16384);
                              a smaller value bounds the plan's record table.
                              The merged phases carry across chunk boundaries,
                              so results do not depend on it (bitwise for
                              FP64).  Negative: INVALID_ARG */
    int in_kernel_records; /* 1-D: 1 = a plan whose grid sizes all lie in
                              64..2048 evaluates the stage coefficients inside
                              the resident step kernel, per block of steps, with
                              the coefficient kernel's arithmetic (the same bits
                              in FP64): no record table traffic and launches of
                              up to 16384 steps whatever the batch size, but
                              each workgroup waits for its records, so it is
                              slower on batches of many workgroups; 0 (default)
                              = a coefficient kernel writes a record table
                              before each chunk (always so for d-D plans, host
                              callbacks and the plain schedule).  Other values:
                              INVALID_ARG */
} hfgpe_options;

typedef struct hfgpe_plan hfgpe_plan;

/* Create a plan for n_inst independent instances of the problem of Sec. 1
 * (Eq. GP1 with the harmonic part of Eq. GP1b), advanced by the composition
 * of Eq. prod-gen with the HO split (ii) of Sec. 2.1 (n_inst >= 0; 0 gives an
 * empty plan whose calls do nothing).  grids and params are host arrays of
 * n_inst entries, copied into the plan.  All instances share the scheme, the
 * dtype, the step dt (may be negative) and the spatial dimension.
 * opts may be NULL.  hip_stream is a hipStream_t or NULL.
 * Errors: INVALID_ARG, UNSUPPORTED_SHAPE, SINGULAR (a stage |a_i dt| at or
 * beyond the first zero of g for the largest frequency the instance reaches),
 * NONPOSITIVE_FREQ, ALLOC, HIP, NO_DEVICE.  On error *out is NULL. */
int hfgpe_plan_create(hfgpe_plan **out, int n_inst, const hfgpe_grid *grids,
                      const hfgpe_params *params, const hfgpe_scheme *scheme,
                      hfgpe_dtype dtype, double dt, const hfgpe_options *opts,
                      void *hip_stream);

/* Release a plan and its device workspace (NULL is accepted). */
int hfgpe_plan_destroy(hfgpe_plan *plan);

/* off[0..n_inst]: start of each instance in the packed buffer, in complex
 * elements; off[n_inst] is the total the caller must allocate. */
int hfgpe_instance_offsets(const hfgpe_plan *plan, int64_t *off);

/* Advance every instance nsteps steps of size dt from time t0, in place on
 * the device buffer d_psi (layout above).  A step is the composition of
 * Table "algorithm" (time frozen in the B flows at the stage times) with each
 * A stage factored as chirp, kinetic phase, chirp (Lemma 2, Theorems 1 and
 * 2), adjacent x-space phases merged as in Eq. prod-genHarmOsc: m FFT pairs
 * per step (per axis for d-D).  Stream-ordered and asynchronous:
 * the call returns once the work is enqueued.  On return of the enqueued
 * work d_psi holds the state at t0 + nsteps*dt with no pending merged phase.
 * nsteps = 0 does nothing. */
int hfgpe_evolve(hfgpe_plan *plan, void *d_psi, double t0, int64_t nsteps);

/* User-defined harmonic-oscillator stages (the exact flow for an omega(t)
 * known only to the caller, e.g. from a host callback or a numerically
 * integrated fundamental matrix, or a table of coefficients): fn returns, for
 * instance inst and axis, the K(f) D(g) K(e) factorisation of the HO flow of
 * that axis over [t0, t0 + tau] (e acts first; K(c) = exp(-i c x^2/2),
 * D(g) = exp(-i g k^2/2), Sec. 2.2) in fge[0..2] = f, g, e, and 0; any other
 * return value makes hfgpe_evolve fail with INVALID_ARG.  The library merges
 * the chirps and the B weights as for its own rules; the plan's HO rule is
 * then ignored (and no harmonic term enters B).  fn is called on the host, from
 * the thread calling hfgpe_evolve, for every instance, step, stage and axis of
 * each chunk of steps, before the chunk's records are copied (async, on the
 * plan's stream) to the device.  fn = NULL restores the plan's rule.
 * Diagonal traps only (INVALID_ARG for coupled plans). */
typedef int (*hfgpe_stage_fn)(void *user, int inst, int axis, double t0, double tau, double mu,
                              double *fge);
int hfgpe_set_stage_callback(hfgpe_plan *plan, hfgpe_stage_fn fn, void *user);

/* Time dependence given by the caller (Sec. 1: omega(t) and sigma(t) are any
 * functions of time): fn returns, for instance inst, omega_j(t) for which = j
 * (j < ndim) and sigma(t) for which = 3.  The plan's HO rule samples it where
 * the rule needs the frequency: omega at the start of each stage for
 * EXACT_CONST (the caller takes care that it is constant), the Gauss nodes of
 * CF4 and MAGNUS6, the sub-step nodes of FUNDAMENTAL, and omega^2 at the B
 * times for FSPLIT; sigma is sampled at the B times.  The parameters' omega
 * and sigma forms are then ignored.  Like hfgpe_set_stage_callback, fn runs
 * on the host for each chunk of steps, and the two are exclusive: setting
 * one clears the other.  An omega that is not finite and positive makes
 * hfgpe_evolve fail with NONPOSITIVE_FREQ, a stage beyond the rule's
 * singular bound with SINGULAR, a non-finite sigma or coefficient with
 * NONFINITE.  fn = NULL restores the parameters' forms.  Diagonal traps only
 * (INVALID_ARG for coupled plans). */
typedef double (*hfgpe_coef_fn)(void *user, int inst, int which, double t);
int hfgpe_set_coef_callback(hfgpe_plan *plan, hfgpe_coef_fn fn, void *user);

/* Perturbation as a device array (Sec. 1: V_I is any potential; the B flow of
 * Lemma 1 is pointwise): d_vi holds eps V_I(x) in FP64 at every grid point of
 * every instance, in the packed layout of the state (hfgpe_instance_offsets),
 * and replaces the instances' eps and per-axis factors in hfgpe_evolve and
 * hfgpe_energy.  NULL restores the factor form.  The caller owns the buffer
 * and keeps it alive and unchanged while work that uses it may run on the
 * plan's stream.  Costs one extra read of 8 bytes per point wherever the
 * x-space phase is applied (every step of the 1-D kernel reads it once per
 * chunk into LDS).  Errors: INVALID_ARG (plan NULL, or d_vi not aligned to 8
 * bytes). */
int hfgpe_set_potential(hfgpe_plan *plan, const double *d_vi);

/* The same with eps V_I held in FP32 (4 bytes per point: half the extra bytes
 * of the passes that apply the x-space phase).  The values enter the FP64
 * phase as they are, so the potential carries its FP32 rounding (~6e-8
 * relative), which the caller accepts by choosing this form.  Setting either
 * form replaces the other; NULL restores the factor form.  Errors:
 * INVALID_ARG (plan NULL, or d_vi not aligned to 4 bytes). */
int hfgpe_set_potential_f32(hfgpe_plan *plan, const float *d_vi);

/* Discrete squared norm h^d sum |u|^2 of every instance into the host array
 * h_out[n_inst] (FP64, compensated summation): the norm that the GPE and its
 * split flows preserve (Sec. 1; Lemma 1 for the B flow).  Synchronises the
 * stream. */
int hfgpe_norm(hfgpe_plan *plan, const void *d_psi, double *h_out);

/* Bytes of the static device scratch of hfgpe_norm_noalloc. */
#define HFGPE_NOALLOC_SCRATCH_BYTES (1u << 20)

/* Allocation-free variant of hfgpe_norm, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same compensated sums, with the per-block partial sums
 * kept in a file-scope static device array of HFGPE_NOALLOC_SCRATCH_BYTES
 * (one per GPU, held until the process ends) instead of the plan's
 * workspace, and the per-instance results written to the caller's device
 * array d_out[n_inst] (FP64, 8-byte aligned).  Stream-ordered on the plan's
 * stream and asynchronous: nothing is allocated, copied to the host or
 * synchronised.  The plan is used on the device it was created on.
 * Requires n_inst * (partial blocks per instance) * 32 bytes of scratch:
 * HFGPE_E_SCRATCH when that exceeds HFGPE_NOALLOC_SCRATCH_BYTES (nothing is
 * launched).  Every call on a GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (other streams, other threads) race; the array
 * needs no clearing (each call writes every partial it reads).
 * INVALID_ARG for a NULL plan, d_psi or d_out (n_inst > 0) or misaligned
 * buffers. */
int hfgpe_norm_noalloc(hfgpe_plan *plan, const void *d_psi, double *d_out);

/* GPE energy of every instance at time t into h_out[4*n_inst] (Sec. 1 names
 * the energy but prints no functional; this is the standard GPE energy, whose
 * interaction term carries sigma/2 so that its variation gives the equation):
 * (total, kinetic, potential, interaction) per instance, with
 *   kinetic     = h^d / N sum_k |k|^2 / (2 mu) |u^_k|^2,
 *   potential   = h^d sum_x ((mu/2) x^T W(t) x + eps V_I) |u|^2, with
 *                 W_jj = omega_j(t)^2 and the off-diagonal entries wcross,
 *   interaction = h^d sum_x sigma(t)/2 |u|^4.
 * Synchronises the stream. */
int hfgpe_energy(hfgpe_plan *plan, const void *d_psi, double t, double *h_out);

/* Testing hook: (f, g, e) of every stage and axis of the step starting at tn
 * for instance inst, computed by the library's closed forms, into
 * out[(i*ndim + j)*3 + {0,1,2}].  Host only. */
int hfgpe_stage_coeffs(const hfgpe_plan *plan, int inst, double tn, double *out);

/* Host-only variant of hfgpe_stage_coeffs that needs no plan and no device:
 * (f, g, e) for one instance described by params (ndim axes) under the scheme
 * with step dt, for the step starting at tn; same layout as above.  Returns
 * SINGULAR / NONPOSITIVE_FREQ when a stage is outside the closed forms'
 * domain. */
int hfgpe_stage_coeffs_params(const hfgpe_params *params, int ndim, const hfgpe_scheme *scheme,
                              double dt, double tn, double *out);

/* Host-only testing hook for a coupled trap (params->wcross non-zero, ndim 2
 * or 3): the factor triples K(F) D(G) K(E) of the step starting at tn, in the
 * order they act (one per stage for EXACT_CONST and FSPLIT, two per stage for
 * CF4), as out[(k*3 + {0: F, 1: G, 2: E}) * ndim*ndim + row*ndim + col], and
 * their number in *ntriples.  out needs room for 2 * m * 3 * ndim^2 doubles.
 * hfgpe_stage_coeffs returns INVALID_ARG for coupled plans. */
int hfgpe_stage_coeffs_coupled(const hfgpe_params *params, int ndim, const hfgpe_scheme *scheme,
                               double dt, double tn, double *out, int *ntriples);

/* Named compositions: "leapfrog" (Eq. LeapFrogB), "lie", "srkn6_4",
 * "ni4_82", "ni5_84" (Table tab.1).  Writes m into *m and, when a and b are
 * non-NULL, the coefficients (room for 16 and 17 doubles). */
int hfgpe_scheme_preset(const char *name, int *m, double *a, double *b);

/* Pick the plan's schedule by timing candidates with HIP events on its
 * stream (the FFT passes of Sec. 2.1 cost the same arithmetic in every
 * schedule; only how the pencils and steps are shared out changes, so the
 * results do not depend on the choice -- bitwise in FP64).
 *   d-D plans: the pass positions of a stage (the axis passes of
 *     Eq. prod-genHarmOsc's stages, opening pass excluded) are tuned one
 *     after another over the default policy, the persistent workgroups per
 *     compute unit (1 .. 4, capped at what fits) and, for c64 separable
 *     passes along strided axes that allow it, 256- or 512-thread groups;
 *     each candidate is timed on min(trial_steps, 64) whole steps (the
 *     positions tuned so far at their winners) after one untimed step.  The
 *     winners are
 *     kept in the plan (hfgpe_tune_get) and in a process-wide cache keyed by
 *     grid shape, storage type, pass structure and position, from which
 *     later plans of the same key start (hfgpe_tune_save / hfgpe_tune_load
 *     carry it across processes).  nd_workgroups is set aside while tuning;
 *     when non-zero it still overrides the tuned counts.  *choice = the
 *     number of pass positions tuned.
 *   1-D plans: the steps per resident launch (whole chunk, 1024 or 256;
 *     candidates not shorter than trial_steps are skipped), trial_steps
 *     steps each; *choice = the winner (0 = whole chunk).
 * d_scratch is a device buffer of the plan's layout holding representative
 * data (its contents are overwritten).  choice may be NULL.  Synchronises
 * the stream. */
int hfgpe_autotune(hfgpe_plan *plan, void *d_scratch, int64_t trial_steps, int *choice);

/* The plan's launch settings of d-D pass position pass (0 .. *npasses - 1):
 * workgroups per compute unit and threads per group, 0 meaning the default
 * policy.  *npasses (may be NULL) receives the positions per stage (0 for 1-D
 * plans); INVALID_ARG for a position out of range.  Host only. */
int hfgpe_tune_get(const hfgpe_plan *plan, int pass, int *per_cu, int *tpb, int *npasses);

/* Write the process-wide cache of tuned pass settings to a text file, or
 * merge such a file into it (plans created afterwards start from it).  A
 * malformed file is rejected whole (INVALID_ARG), as are unreadable paths.
 * Host only; safe to call from several threads. */
int hfgpe_tune_save(const char *path);
int hfgpe_tune_load(const char *path);

/* Device-side error word raised by the coefficient kernel since the last
 * call (0 or a status code); synchronises and clears it. */
int hfgpe_device_status(hfgpe_plan *plan);

/* With opts.profile set: total milliseconds spent in the step kernels and
 * (profile level 2) in the coefficient kernel, and the number of step-kernel
 * launches, since the last call (synchronises the stream; resets the
 * counters). */
int hfgpe_profile(hfgpe_plan *plan, double *step_ms, double *coeff_ms, int64_t *step_launches);

const char *hfgpe_status_string(int status);
int hfgpe_version(int *major, int *minor);
/* The hipError_t of the last failing HIP call made by the library. */
int hfgpe_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HFGPE_H */
