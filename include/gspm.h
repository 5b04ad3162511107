/*
 * gspm.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of one time step of the Gauss-Seidel projection method (GSPM) for
 * finite-element micromagnetics with magnetostriction (Guan & Renuka
 * Balakrishna, "CuPyMag", arXiv 2510.09812).
 *
 * The problem (Sec. 2.1): a cuboid computational cell Omega_c inside an
 * ellipsoidal body, split into a ferromagnetic host Omega_m and nonmagnetic
 * inclusions; unknowns are the unit magnetisation m = M/Ms and the periodic
 * displacement u.  One call of gspm_step advances Algorithm B.1 (App. B) by
 * n steps: volume averages (Sec. 2.4) feed the far-field demagnetising field
 * -Ms N_d mbar (Sec. 2.1, ellipsoid theorem) and the homogeneous strain;
 * mechanical equilibrium (Eq. elasticity, weak form Eq. weak_elasticity) is
 * solved by unpreconditioned CG with one pinned node (Sec. 2.5; run in the
 * single-reduction form, one fused kernel launch per iteration); the three
 * stages of (1 - eps lap) g = f (Eq. GS, weak form Eq. weak_GS) are solved by
 * unpreconditioned CG; the cross-product update and the unit-length
 * projection close the step.  Optionally (gspm_params.local_demag) each step
 * also solves the local magnetostatic potential U~ of Eq. (demag) in the weak
 * form (weak_demag) by CG and adds its field -grad U~ to the effective field,
 * and (gspm_params.crystal_rot) the cubic crystal may be turned against the
 * sample frame of the mesh as in App. D.
 *
 * Conventions shared by every entry point
 *   - Units are SI (metres, A/m, Pa, J/m^3, seconds).
 *   - Node-indexed arrays are host arrays in the caller's node order, three
 *     doubles per node, row-major (n_nodes x 3).  The library identifies the
 *     max-face copies of periodic nodes with their min-face partners (Sec. 2.5)
 *     and renumbers nodes internally; neither is visible to the caller.  On
 *     input, the copies of one periodic node must carry the same values (to
 *     1e-12 relative) or the call fails with GSPM_E_ARG; on output all copies
 *     receive the value of their node.
 *   - Ownership: the caller owns every host array; the library reads or writes
 *     it only during the call and keeps no pointer.  The context owns all device
 *     memory and releases it in gspm_destroy.
 *   - Errors: every call returns a gspm_status; on failure gspm_last_error()
 *     gives a message.  No call throws or aborts.  A failed call leaves the
 *     state as it was, except gspm_step (see there).
 *   - Call order: create -> upload_mesh -> set_params -> set_field(M) -> step.
 *     Calls out of order return GSPM_E_STATE.
 *   - Threads: one context is used by one host thread at a time.  All device
 *     work runs on the context's stream.
 */
#ifndef GSPM_H
#define GSPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gspm_ctx gspm_ctx;

typedef enum {
    GSPM_OK = 0,
    GSPM_E_ARG = -1,        /* invalid argument (null pointer, size, value) */
    GSPM_E_MESH = -2,       /* degenerate element, unmatched periodic node, bad index */
    GSPM_E_STATE = -3,      /* call out of order */
    GSPM_E_DEVICE = -4,     /* HIP runtime error or no usable gfx950 device */
    GSPM_E_NOCONV = -5,     /* CG reached cg_maxit */
    GSPM_E_NONFINITE = -6,  /* NaN or Inf in the state */
    GSPM_E_OOM = -7         /* device allocation failed */
} gspm_status;

typedef enum { GSPM_FP64 = 0, GSPM_MIXED = 1 } gspm_precision;

typedef enum {
    GSPM_FIELD_M = 0,       /* magnetisation direction m, n_nodes x 3 */
    GSPM_FIELD_U = 1,       /* displacement u~ [m], n_nodes x 3 */
    GSPM_FIELD_UD = 2       /* local magnetostatic potential U~ of Eq. (demag) [A], ONE value per node */
} gspm_field;

/* Operators of Eq. (LHS) and Eq. (RHS_F), Sec. 2.3, for gspm_apply/gspm_solve. */
typedef enum {
    GSPM_OP_LAPLACE = 0,    /* K_ij = int grad phi_i . grad phi_j over magnetic elements, per component */
    GSPM_OP_MASS = 1,       /* M_ij = int phi_i phi_j over magnetic elements (F^GS), per component */
    GSPM_OP_GS = 2,         /* eps K + M: the GSPM operator of Eq. (weak_GS), per component */
    GSPM_OP_ELASTIC = 3,    /* K^mech over all elements; rows of the pinned node are zero */
    GSPM_OP_MS = 4,         /* K^ms: int grad phi_i . grad phi_j over all elements (Eq. weak_demag), rows of
                               the pinned node zero, per component */
    GSPM_OP_PRECOND = 5     /* gspm_apply only: the elastic preconditioner B of elastic_precond = 1 (FP64
                               contexts) */
} gspm_op;

typedef enum {
    GSPM_PRECOND_NONE = 0,  /* the paper's unpreconditioned CG on the pinned system (Sec. 2.5) */
    GSPM_PRECOND_GREEN = 1, /* CG on the periodic system preconditioned by the lattice Green's operator of the
                               stiffness on an auxiliary grid; pinned by a translation afterwards */
    GSPM_PRECOND_JACOBI = 2 /* CG preconditioned by the operator's diagonal */
} gspm_precond;

#define GSPM_PERIODIC 1u

typedef struct {
    int32_t device;         /* HIP device ordinal */
    int32_t precision;      /* GSPM_FP64, or GSPM_MIXED: every CG solve is FP64 iterative
                               refinement (true FP64 residual, same stopping rule)
                               around an inner CG with FP32 vectors and FP32 element
                               arithmetic; state, right-hand sides, dot products,
                               norms and averages stay FP64 */
    int32_t block_nodes;    /* nodes per owner block (power of two, 64..1024), 0 = automatic */
    int32_t profile;        /* nonzero: time every elastic CG iteration launch with HIP events */
    void *stream;           /* hipStream_t to run on, or NULL for a stream owned by the context */
    int32_t reorder;        /* internal node order: GSPM_REORDER_MORTON (default), GSPM_REORDER_NONE (the order
                               in which the caller's nodes first appear), GSPM_REORDER_RCM (reverse
                               Cuthill-McKee on the mesh graph).  Owner blocks are ranges of this order, so
                               it sets the halo sizes; results agree to rounding. */
    /* Optional device allocator (both or neither): every device buffer the context owns comes from
     * dev_alloc(bytes, alloc_user) (device memory of opts->device, 256-byte aligned, NULL on failure)
     * and goes back through dev_free(ptr, alloc_user), for example from PyTorch's caching allocator.
     * NULL: hipMalloc / hipFree. */
    void *(*dev_alloc)(size_t bytes, void *alloc_user);
    void (*dev_free)(void *ptr, void *alloc_user);
    void *alloc_user;
    int32_t deterministic;  /* nonzero: bitwise reproducible steps (same device, mesh, block size and inputs
                               give the same bits, whether run at once or split by a save and restore of M
                               and U).  Every sum is added in a fixed order: workgroup totals go to slots
                               that a follow-up launch adds in a fixed order (no atomic adds), and the
                               element passes gather each owned node's elements in a fixed order (no LDS
                               atomics; each element is evaluated once per owned vertex).  Slower; the
                               learned and extrapolated warm starts and the corrected GS start are not
                               available (GSPM_E_STATE). */
} gspm_create_opts;

typedef enum { GSPM_REORDER_MORTON = 0, GSPM_REORDER_NONE = 1, GSPM_REORDER_RCM = 2 } gspm_reorder;

/* Material and run parameters (App. A notation; SI units). */
typedef struct {
    double Ms;              /* saturation magnetisation m_s [A/m] */
    double A;               /* exchange coefficient [J/m] */
    double K1;              /* cubic anisotropy kappa_1 [J/m^3] */
    double lambda100, lambda111;   /* magnetostriction constants */
    double c11, c12, c44;   /* cubic elastic constants [Pa] */
    double alpha;           /* damping constant */
    double mu0;             /* vacuum permeability [T m/A] */
    double gamma0;          /* gyromagnetic ratio of tau = gamma0 Ms t [m/(A s)] */
    double Nd[9];           /* demagnetisation tensor of the body, row-major */
    double hext[3];         /* applied field H_ext [A/m] */
    double sigma_ext[6];    /* applied stress [Pa], order xx yy zz yz xz xy */
    double cg_tol;          /* CG stops at ||r||_2 <= cg_tol ||b||_2 (Sec. 3.1 criterion) */
    int32_t cg_maxit;       /* CG iteration cap per scalar or vector solve; exceeding it is GSPM_E_NOCONV */
    int32_t precession;     /* 1: full Algorithm B.1; 0: damping stage only (m* = m^n) */
    int32_t local_demag;    /* 1: each step solves K^ms U~ = Ms F^ms m (Eqs. weak_demag, RHS_F, RHS_b) at m^n,
                               pinned at the caller's node 0 and warm-started from the previous U~, and adds
                               the element field -grad U~ / Ms to h on magnetic elements (held for h[m*]);
                               the energy total gains (mu0/2) <|grad U~|^2>.  0: far field only. */
    double crystal_rot[9];  /* crystal orientation of App. D, row-major R with v_sample = R v_crystal (the rows
                               are the sample axes in crystal coordinates; App. D's <111>, <-110>, <11-2> frame
                               is one example).  The stiffness, spontaneous strain, anisotropy and
                               magnetoelastic field are taken in the crystal frame; the mesh, u, hext,
                               sigma_ext and Nd are in the sample frame.  All zeros (or the identity): crystal
                               axes along the sample axes.  Otherwise R must be a proper rotation to 1e-12
                               (GSPM_E_ARG). */
    int32_t elastic_precond; /* GSPM_PRECOND_NONE or GSPM_PRECOND_GREEN: the elastic solves (the step's and
                               gspm_solve's) by CG preconditioned with
                                 B = Q A_g^+ Q^T + (1/2) D^-1,
                               A_g the stiffness on a periodic grid of round(L_a / l) points per axis
                               (l = (V_c / n_unique)^(1/3)) with every cell split into six tetrahedra around
                               its main diagonal, inverted mode by mode by FFT (the translation mode left out),
                               Q the trilinear interpolation from the grid to the nodes, D the diagonal of
                               K^mech.  The solve runs on the periodic system (the right-hand side's mean per
                               component removed, K u = b tested as ||b - K u|| <= cg_tol ||b||) and pins the
                               caller's node 0 by a translation at the end.  Sec. 5.2 names the elastic CG as
                               the cost to cut; the paper does not precondition it. */
    int32_t gs_precond;     /* GSPM_PRECOND_NONE or GSPM_PRECOND_JACOBI: the GS solves of Eq. (weak_GS) (the
                               step's and gspm_solve's) by CG preconditioned with D = diag(eps K + M), the
                               same stopping rule; nodes in the inclusions only keep their identity rows */
    double ms_tol;          /* local_demag: the magnetostatic CG stops at ||r|| <= ms_tol ||b||; 0 selects
                               max(1e-3 cg_tol, 1e-12) (the floor: what FP64 residuals of K^ms can reach).  K^ms (the Laplacian of the whole cell, one pinned node) has a
                               condition number growing as (L/h)^2, so two iterates that both pass a 1e-8
                               test can differ by ~1e-5; the tighter test keeps the potential (and m, u
                               through its field) within 1e-6 whatever precision the solve ran in. */
} gspm_params;

typedef struct {
    int32_t steps_done;     /* steps completed by this call */
    int32_t failed_step;    /* index (within the call) of the step that failed, or -1 */
    int64_t mech_iters;     /* elastic CG iterations (GSPM_MIXED: inner FP32 iterations), summed over the steps */
    int64_t gs_iters;       /* GS CG iterations, summed over all scalar solves and steps */
    int64_t gs_iters_stage[8]; /* per scalar solve: g1 g2 g3, g*1 g*2, m**1 m**2 m**3 */
    double dm_avg;          /* mean |m^{n+1} - m^n| over magnetic nodes, last step (Sec. 3.2) */
    double elapsed_ms;      /* wall time of the call on the device stream */
    double matvec_ms;       /* profile mode: summed kernel duration of the working elastic CG
                               iteration launches (the matvec fused with the CG vector updates, or with
                               elastic_precond the preconditioned iteration's matvec; those issued after
                               convergence, which exit at once, excluded) */
    int64_t matvec_launches;/* profile mode: number of elastic CG iteration launches timed */
    int64_t refinements;    /* GSPM_MIXED: outer FP64 residual evaluations that started an FP32 inner solve */
    int64_t learned_starts; /* steps whose elastic start used the network's increment */
    int64_t minres_starts; /* steps whose elastic start was a minimum-residual step (learned or extrapolated) */
    double warm_coef[2];    /* last minimum-residual start: coefficients of the network increment and of the
                               previous displacement increment (0 if unused) */
    int64_t ms_iters;       /* local_demag: magnetostatic CG iterations (GSPM_MIXED: inner FP32), summed */
    int64_t mech_refinements; /* GSPM_MIXED: the refinements of the elastic solves (part of `refinements`) */
    double gs_matvec_ms;    /* profile mode: summed kernel duration of the working GS CG iteration launches on
                               three components (one fused launch per iteration: the matvec with the CG vector
                               updates; stages 1 and 3; those after convergence excluded) */
    int64_t gs_matvec_launches; /* profile mode: their number */
    double phase_ms[8];     /* profile mode: device time of each phase of Alg. B.1, summed over the steps:
                               [0] averages at m^n, [1] elastic solve (right-hand side, start, CG), [2] local
                               magnetostatic solve, [3] GS stage 1 (field right-hand side, 3 solves), [4] stage 2
                               (m updates, right-hand side, 2 solves), [5] averages at m*, [6] stage 3, [7]
                               projection and commit check */
    double final_residual[5]; /* the last step of the call: the relative residual ||b - A x|| / ||b|| at which
                               each solve stopped (largest over its components; FP64 in both precisions):
                               elastic, GS stage 1, stage 2, stage 3, magnetostatic; 0 for a solve not run */
} gspm_step_stats;

/* Create a context on opts->device (NULL opts: device 0, FP64, own stream).
 * Fails with GSPM_E_DEVICE when no HIP device is usable. */
gspm_status gspm_create(gspm_ctx **out, const gspm_create_opts *opts);
void gspm_destroy(gspm_ctx *ctx);

/* Mesh upload (Sec. 2.1 domain, Sec. 2.5 periodic identification).
 * xyz: n_nodes x 3 coordinates; tets: n_tets x 4 node indices (0-based, either
 * orientation); tags: n_tets bytes, 0 = nonmagnetic inclusion (Omega_d), any
 * other value = magnetic host (Omega_m); lo/hi: the periodic box.  flags must
 * contain GSPM_PERIODIC.  Validates the mesh (GSPM_E_MESH on a degenerate or
 * repeated-node element, a node outside the box, or an unmatched periodic
 * node), renumbers nodes along a Morton curve, builds the element blocks and
 * copies everything to the device once.  Resets all fields to zero. */
gspm_status gspm_upload_mesh(gspm_ctx *ctx, int64_t n_nodes, const double *xyz, int64_t n_tets,
                             const int32_t *tets, const uint8_t *tags, const double lo[3], const double hi[3],
                             uint32_t flags);

/* Set material and run parameters; may be called again between steps (for
 * example to change hext along a hysteresis sweep). */
gspm_status gspm_set_params(gspm_ctx *ctx, const gspm_params *params);

typedef enum {
    GSPM_GS_START_LUMPED = 0,    /* the lumped-mass solution of each GS system (the default) */
    GSPM_GS_START_CORRECTED = 1  /* that start plus the same stage's correction of the previous step */
} gspm_gs_start;

/* Choose the start vector of the Gauss-Seidel solves of Alg. B.1 (steps 1
 * and 3).  Each GS system (eps K + M) g = b starts from the lumped solution
 * g0 = M_L^-1 b' that the right-hand side defines (m + dtau h-terms / w per
 * node); the corrected start adds d = g - g0 of the same stage at the last
 * step, so that a solve whose answer moves little from step to step starts
 * closer to it.  Only the start changes: every solve still stops at cg_tol.
 * The correction is kept per stage from the second step on and dropped by
 * gspm_set_field(M), by a failed solve and by a new mesh.  Not available in
 * deterministic mode (GSPM_E_STATE): a restored state would lack it.  Uses
 * 11 doubles per node of device memory (allocated with the mesh). */
gspm_status gspm_set_gs_start(gspm_ctx *ctx, int32_t mode);

/* Set or read a nodal field (n_nodes x 3, caller's order; GSPM_FIELD_UD:
 * n_nodes values).  Setting M normalises m on magnetic nodes (a vector whose
 * length is 1 to within 1e-14 is kept as given, so a state read with
 * get_field restores bit for bit) and zeroes it on nodes that lie in
 * inclusions only; a zero or non-finite vector on a magnetic node is
 * GSPM_E_ARG.  U is the periodic displacement [m]; UD the
 * local magnetostatic potential [A] (the warm start of the next solve and
 * the potential the energies use). */
gspm_status gspm_set_field(gspm_ctx *ctx, gspm_field which, const double *values, int64_t n_nodes);
gspm_status gspm_get_field(gspm_ctx *ctx, gspm_field which, double *out, int64_t n_nodes);

/* Advance Algorithm B.1 by n_steps steps of dt seconds.  stats may be NULL.
 * On GSPM_E_NOCONV or GSPM_E_NONFINITE the state is that after the last
 * completed step and stats->failed_step names the step that failed. */
gspm_status gspm_step(gspm_ctx *ctx, double dt, int32_t n_steps, gspm_step_stats *stats);

/* Relax at the current applied field and stress (Sec. 3.3): steps of dt
 * seconds until the mean per-node change of m over one step, dm_avg =
 * <|m^n - m^{n-1}|> on the magnetic nodes (Sec. 3.2), falls below dm_tol (the
 * paper uses 5e-10), at most max_steps.  stats (nullable) sums the
 * iterations of the steps taken; steps_done counts them, dm_avg is the last
 * step's.  Returns GSPM_E_NOCONV after max_steps steps without convergence
 * (the state is that after the last step, so the call can be repeated); a
 * failing step returns its status with the state after the step before. */
gspm_status gspm_relax(gspm_ctx *ctx, double dt, double dm_tol, int32_t max_steps, gspm_step_stats *stats);

/* Flags of gspm_sweep. */
#define GSPM_SWEEP_STOP_ON_REVERSAL 1u  /* end after the first point whose mbar has a non-positive component
                                           along the first point's field (the coercive point) */
#define GSPM_SWEEP_CONTINUE 2u          /* a point that does not relax within max_steps keeps its state after
                                           max_steps, records mbar there with converged = 0, and the sweep
                                           goes on (a fixed number of steps per point, as a field loop run
                                           for a set length) */

/* A field (and stress) sweep, as the hysteresis runs of Sec. 3.3 (the field
 * lowered in steps of 20 A/m until the magnetisation reverses; a uniaxial
 * stress as a second parameter): for point k = 0 .. n_points-1 the applied
 * field becomes hext[3k .. 3k+2] and, when sigma_ext is not NULL, the applied
 * stress sigma_ext[6k .. 6k+5] (the other parameters stay as set), the state
 * relaxes as in gspm_relax, and mbar[3k .. 3k+2] receives the cell-averaged
 * magnetisation, steps[k] the steps taken and converged[k] (nullable) 1 if
 * dm_avg fell below dm_tol.  flags: GSPM_SWEEP_STOP_ON_REVERSAL (that first
 * field must be nonzero) and GSPM_SWEEP_CONTINUE, above; any other bit is
 * GSPM_E_ARG.  points_done (nullable) receives the points completed.  Without
 * GSPM_SWEEP_CONTINUE the first point that fails to relax ends the sweep with
 * GSPM_E_NOCONV (steps and converged filled for it, mbar not); a failing step
 * ends it with its status either way.  The parameters keep the last point's
 * field. */
gspm_status gspm_sweep(gspm_ctx *ctx, double dt, double dm_tol, int32_t max_steps, int32_t n_points,
                       const double *hext, const double *sigma_ext, uint32_t flags, double *mbar,
                       int32_t *steps, int32_t *converged, int32_t *points_done);

/* Energy densities of Eq. (MicromagneticsEnergy) averaged over the cell
 * [J/m^3] at the current state: out = {exchange, anisotropy, zeeman,
 * magnetoelastic, stress work, far-field demagnetisation, total}.  With
 * local_demag the total also holds the local magnetostatic energy of the
 * stored U~ (gspm_demag_local_energy). */
gspm_status gspm_energies(gspm_ctx *ctx, double out[7]);

/* The local magnetostatic energy density (mu0 / 2 V_c) int |grad U~|^2 over
 * the cell [J/m^3] of the stored potential U~ (Sec. 2.1; the cross term with
 * the uniform far field vanishes since grad U~ has zero mean).  Needs
 * set_params. */
gspm_status gspm_demag_local_energy(gspm_ctx *ctx, double *e);

/* Volume averages over the cell (Sec. 2.4): mbar[3] and the homogeneous
 * strain ebar[6] (order xx yy zz yz xz xy). */
gspm_status gspm_averages(gspm_ctx *ctx, double mbar[3], double ebar[6]);

/* gspm_averages without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no hipMalloc, hipFree or allocating library call, no
 * host synchronisation.  m_dev: device array of n_nodes x 3 doubles in the
 * caller's node order (row-major), read at the first copy of each periodic
 * node and used as given (not normalised; copies are not compared);
 * out_dev: device array of 9 doubles receiving mbar[3] then ebar[6] (order
 * xx yy zz yz xz xy).  The work is enqueued on the context's stream and the
 * call returns at once: out_dev is valid once that stream has reached it.
 * Partial sums go to a fixed scratch array of the library, one per GPU, held
 * until the process ends (4096 x 9 partial sums plus a few totals, 300 KB):
 * meshes of more than 4,194,304 unique nodes are GSPM_E_ARG.  The partial
 * sums are added in a fixed order, so results repeat bitwise; they agree with
 * gspm_averages to rounding.  Every call on a GPU shares that GPU's scratch
 * and keeps the last call's contents, so calls that overlap on one GPU (on
 * different streams or contexts) race.  Needs upload_mesh and set_params. */
gspm_status gspm_averages_noalloc(gspm_ctx *ctx, const double *m_dev, double *out_dev);

/* Apply one operator of Sec. 2.3 to x (n_nodes x 3, caller's order), writing
 * y = A x (the assembled residual at each node, reported at all its copies).
 * eps is used by GSPM_OP_GS only.  GSPM_OP_ELASTIC needs gspm_set_params;
 * GSPM_OP_PRECOND (y = B x) needs elastic_precond = GSPM_PRECOND_GREEN on an
 * FP64 context (GSPM_E_STATE otherwise). */
gspm_status gspm_apply(gspm_ctx *ctx, gspm_op op, double eps, const double *x, double *y, int64_t n_nodes);

/* Solve A x = b by the library's CG (GSPM_OP_GS per component on the magnetic
 * nodes, GSPM_OP_ELASTIC with the pinned node, or GSPM_OP_MS per component
 * with the pinned node).  x holds the initial guess on entry and the solution
 * on return; iters (nullable) receives the iteration count (summed over
 * components for GSPM_OP_GS and GSPM_OP_MS).  With elastic_precond =
 * GSPM_PRECOND_GREEN, GSPM_OP_ELASTIC solves the periodic system for b with
 * its mean removed (see gspm_params) and pins node 0 afterwards. */
gspm_status gspm_solve(gspm_ctx *ctx, gspm_op op, double eps, const double *b, double *x, int64_t n_nodes,
                       double tol, int32_t maxit, int32_t *iters);

/* Time one operator of Sec. 2.3 on device-resident data: reps launches of the
 * matvec y = A x on internal work vectors (their contents are whatever the
 * last call left; timing does not depend on them), bracketed by HIP events on
 * the context's stream.  *avg_ms receives the mean duration of one launch.
 * GSPM_OP_ELASTIC needs gspm_set_params.  Changes no field. */
gspm_status gspm_time_operator(gspm_ctx *ctx, gspm_op op, double eps, int32_t reps, double *avg_ms);

/* Switch the per-launch timing of the elastic CG iteration (the create option
 * `profile`) on or off for later gspm_step calls.  Each iteration kernel is
 * launched with a start/stop event pair that the runtime records at the
 * kernel's own execution (its duration alone, as a kernel trace reports it);
 * the events add a little host overhead to each CG iteration. */
gspm_status gspm_set_profile(gspm_ctx *ctx, int32_t enable);

/* Mesh facts after upload: unique nodes, tetrahedra, owner blocks, element
 * copies processed per element pass, cell volume [m^3]. Pointers may be NULL. */
gspm_status gspm_mesh_info(gspm_ctx *ctx, int64_t *n_unique, int64_t *n_tets, int64_t *n_blocks,
                           int64_t *n_elem_copies, double *volume);

/* Demagnetisation factors (N_a, N_b, N_c) of an ellipsoid with semi-axes a, b,
 * c along its own axes (the body factor N_d of Sec. 2.1; for a body aligned
 * with the crystal axes pass diag(N) as gspm_params.Nd).  Host only: needs no
 * device and no context.  GSPM_E_ARG unless a, b, c are positive and finite. */
gspm_status gspm_demag_factors(double a, double b, double c, double N[3]);

/* ---------------------------------------------------------------------------
 * Learned warm start of the elastic solve.
 *
 * The paper starts each elastic CG (Sec. 2.5, stopping rule of Sec. 3.1) from
 * the previous step's displacement and names the elastic solve as the cost to
 * reduce (Sec. 5.2); it describes no learned start.  These entry points add
 * one: a message-passing network predicts the displacement increment d from
 * the magnetisation increment m^n - m^{n-1}.  With e = u^{n-1} - u^{n-2} the
 * previous displacement increment (the long-wavelength response a local
 * network cannot see), the solve starts from u^{n-1} + a d + c e with (a, c)
 * the coefficients that minimise the start's residual 2-norm (the quantity
 * the CG stopping test measures) on span{d, e}:
 *   [[Kd.Kd, Kd.Ke], [Ke.Kd, Ke.Ke]] (a, c) = (Kd.r0, Ke.r0),  r0 = b - K u^{n-1},
 * so |b - K u0| <= |r0| whatever the network predicts (nearly parallel K d,
 * K e: the better single-direction step).  CG then runs to the same tolerance, so
 * the solution is that of the plain path within the CG tolerance.
 *
 * Network (hidden width 64, weights and stored activations BF16, FP32
 * arithmetic, MFMA node GEMMs), on the directed edges (i, j) of the mesh
 * (nodes sharing a tetrahedron):
 *   x_i = tag_i [dm_i / s_m, m_i, 1], s_m = sqrt(sum w |dm|^2 / sum w),
 *         tag_i = 1 on magnetic nodes (w = lumped magnetic volume), else 0
 *   h_i = SiLU(W0 x_i + b0)
 *   3 layers: z_ij = Wa h_i + Wb h_j + We e_ij + c, e_ij = nearest-image
 *         (x_j - x_i) / hbar, hbar = (6 V_cell / n_tets)^(1/3);
 *         a_i = mean_j SiLU(z_ij); h_i <- h_i + Wu [h_i ; a_i] + bu
 *   y_i = Wd h_i + bd;  d = lambda100 hbar s_m (y - y_pinned)
 * Parameters: GSPM_MPNN_PARAMS floats, in this order, matrices row-major
 * (out x in): W0[64][7] b0[64], 3 x (Wa[64][64] Wb[64][64] We[64][3] c[64]
 * Wu[64][128] bu[64]), Wd[3][64] bd[3].
 * ------------------------------------------------------------------------- */
#define GSPM_MPNN_PARAMS 50819

typedef enum {
    GSPM_WARM_PREVIOUS = 0,     /* u^{n-1} (the paper's start) */
    GSPM_WARM_LEARNED = 1,      /* u^{n-1} + a d + c e: network increment and previous increment */
    GSPM_WARM_EXTRAPOLATE = 2   /* u^{n-1} + c e: previous increment only (no network) */
} gspm_warm_start;

/* Choose the elastic start of gspm_step.  GSPM_WARM_LEARNED needs
 * gspm_mpnn_set_params.  The network term needs m^{n-1} (from the second
 * step after gspm_set_field(M)); the increment term needs u^{n-2} (from the
 * third step after the last gspm_set_field); before that the missing term is
 * left out. */
gspm_status gspm_set_warm_start(gspm_ctx *ctx, int32_t mode);

/* Load (or replace) the network parameters (count == GSPM_MPNN_PARAMS, all
 * finite) and reset the optimiser moments.  The first call after a mesh
 * upload builds the edge graph and allocates the network's device buffers. */
gspm_status gspm_mpnn_set_params(gspm_ctx *ctx, const float *params, int64_t count);
gspm_status gspm_mpnn_get_params(gspm_ctx *ctx, float *params, int64_t count);

/* Network output y (n_nodes x 3, caller's order) for the inputs (m_prev, m)
 * (n_nodes x 3 each); s_m (nullable) receives the increment scale. */
gspm_status gspm_mpnn_forward(gspm_ctx *ctx, const double *m_prev, const double *m, int64_t n_nodes, double *y,
                              double *s_m);

/* One training step on one sample: forward, loss = mean over nodes and
 * components of ((y - mean y) - (t - mean t))^2 with t = du / (lambda100 hbar
 * s_m), backward, and (update != 0) one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, learning rate lr).  du is the displacement increment
 * u^n - u^{n-1} (n_nodes x 3).  loss and grad (GSPM_MPNN_PARAMS floats, the
 * gradient before the update) are nullable.  Needs gspm_set_params. */
gspm_status gspm_mpnn_train_step(gspm_ctx *ctx, const double *m_prev, const double *m, const double *du,
                                 int64_t n_nodes, float lr, int32_t update, double *loss, float *grad);

/* The learned start for the current state (M and U as set): forms the
 * elastic right-hand side at m, evaluates the network at (m_prev, m) and
 * writes u0 = u + a d + c e (n_nodes x 3) with e = u - u_prev when u_prev is
 * given (else c = 0), and coef = (a, c) (nullable), (a, c) minimising
 * |b - K u0| as above.  Changes no field. */
gspm_status gspm_mpnn_warm_start(gspm_ctx *ctx, const double *m_prev, const double *u_prev, int64_t n_nodes,
                                 double *u0, double coef[2]);

/* Message of the last failure on this context (or of the last failed
 * gspm_create when ctx is NULL).  Never NULL. */
const char *gspm_last_error(const gspm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
