/*
 * GSPM oracle: a plain, slow CPU FP64 reference of one time step of the
 * Gauss-Seidel projection method for finite-element micromagnetics with
 * magnetostriction and ellipsoid-theorem far-field demagnetisation.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers.  The HIP library never
 * includes this header or links this code, and this code knows nothing of it.
 *
 * Units are SI.  Node-indexed arrays passed in or out are in the caller's
 * node order, three values per node (row-major n0 x 3), unless stated.
 */
#ifndef GSPM_ORACLE_H
#define GSPM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_E_ARG = -1, OR_E_MESH = -2, OR_E_STATE = -3, OR_E_NOCONV = -5, OR_E_NONFINITE = -6 };

typedef struct {
    double Ms, A, K1, lambda100, lambda111, c11, c12, c44, alpha, mu0, gamma0;
    double Nd[9];          /* body demagnetisation tensor, row-major */
    double hext[3];        /* applied field [A/m] */
    double sigma_ext[6];   /* applied stress [Pa], order xx yy zz yz xz xy */
    double cg_tol;         /* relative residual ||r|| <= tol ||b|| */
    int32_t cg_maxit;
    int32_t precession;    /* 1: full Algorithm B.1; 0: damping stage only (m* = m^n) */
    int32_t local_demag;   /* 1: solve the local magnetostatic potential U~ each step (periodic meshes only) */
    double crystal_rot[9]; /* R of App. D, row-major: v_sample = R v_crystal; all zeros = identity */
    int32_t elastic_precond; /* 1: elastic solves by CG with the Green's-operator preconditioner (periodic
                                system, pinned by translation afterwards); 0: plain CG on the pinned system */
    int32_t gs_precond;    /* 2: GS solves by CG preconditioned with the operator's diagonal (Jacobi); 0: plain */
    double ms_tol;         /* magnetostatic CG tolerance; 0 selects max(1e-3 cg_tol, 1e-12) */
} or_params;

typedef struct {
    int32_t steps_done;
    int32_t mech_iters;    /* elastic CG iterations summed over the steps */
    int32_t gs_iters[8];   /* per scalar GS solve, summed: g1 g2 g3, g*1 g*2, m**1 m**2 m**3 */
    double dm_avg;         /* mean |m^{n+1} - m^n| over magnetic nodes, last step */
    int32_t ms_iters;      /* magnetostatic CG iterations summed over the steps */
} or_stats;

typedef struct or_sim or_sim;

/* Mesh: xyz n0x3, tets ne x 4 (0-based), tags ne (0 = nonmagnetic).  With
 * periodic != 0 nodes on the max face of the box [lo, hi] are identified with
 * their min-face partners.  Returns OR_E_MESH with a message in err on failure. */
int or_create(or_sim **out, int32_t n0, const double *xyz, int32_t ne, const int32_t *tets,
              const uint8_t *tags, const double lo[3], const double hi[3], int32_t periodic,
              char *err, int32_t errlen);
void or_destroy(or_sim *s);

int32_t or_n_unique(const or_sim *s);
void or_node_map(const or_sim *s, int32_t *map);          /* n0: caller node -> unique node */
void or_geometry(const or_sim *s, double *vol, double *grad); /* ne and ne x 4 x 3 */
double or_total_volume(const or_sim *s);
void or_lumped_weights(const or_sim *s, double *w);       /* unique-node order, n */
int32_t or_pinned_node(const or_sim *s);

int or_set_params(or_sim *s, const or_params *p);
int or_set_m(or_sim *s, const double *m);                 /* n0 x 3 */
int or_set_u(or_sim *s, const double *u);                 /* n0 x 3 */
void or_get_m(const or_sim *s, double *m);
void or_get_u(const or_sim *s, double *u);
int or_set_ud(or_sim *s, const double *ud);               /* n0 values: the potential U~ [A] */
void or_get_ud(const or_sim *s, double *ud);

/* Operators in unique-node order, x and y are n x 3.
 * which: 0 Laplacian K over magnetic elements (per component)
 *        1 mass M over magnetic elements (per component)
 *        2 eps K + M (per component)
 *        3 elastic K^mech over all elements, pinned node rows zeroed
 *        4 Laplacian over all elements (per component)
 *        5 K^ms: Laplacian over all elements, pinned node rows zeroed (per component) */
int or_apply(const or_sim *s, int32_t which, double eps, const double *x, double *y);

/* CG on operator `which` (2, 3 or 5 above), unique-node order; x holds x0 on
 * entry.  Components of the GS and K^ms operators are solved independently.
 * which = 6: the elastic system (3) by Jacobi-preconditioned CG.
 * which = 7: the periodic elastic system (b's mean removed) by CG with the Green's-operator preconditioner,
 *            pinned at p0 by translation afterwards (needs elastic_precond = 1). */
int or_solve(const or_sim *s, int32_t which, double eps, const double *b, double *x, double tol,
             int32_t maxit, int32_t *iters);

int or_step(or_sim *s, double dt, int32_t n, or_stats *st);

/* Energy densities averaged over the computational cell [J/m^3]:
 * out = {exchange, anisotropy, zeeman, magnetoelastic, stress work, far-field demag, total}.
 * With local_demag the total includes the local magnetostatic energy of the stored U~. */
int or_energies(or_sim *s, double out[7]);
/* (mu0 / 2 V_c) int |grad U~|^2 of the stored potential [J/m^3]. */
int or_demag_local_energy(or_sim *s, double *e);
/* mbar[3]; ebar[6] = mean strain, order xx yy zz yz xz xy. */
int or_averages(or_sim *s, double mbar[3], double ebar[6]);

/* Pieces exposed for the pins. */
int or_elastic_rhs(or_sim *s, double *b);                 /* unique order n x 3, at current m */
int or_field_rhs(or_sim *s, double c, double *b, double *ch); /* at current m and u, n x 3 each */
void or_demag_factors(double a, double b, double c, double N[3]);
void or_h_local(const or_params *p, const double m[3], const double E[6], const double mbar[3],
                double h[3]);
double or_energy_density_local(const or_params *p, const double m[3], const double E[6]);
/* The material in the sample frame (App. D): the stiffness as a 6x6 Voigt
 * matrix (order xx yy zz yz xz xy, engineering shear), and the spontaneous
 * strain E0(m) for a sample-frame m (tensor components, same order). */
void or_stiffness_voigt(const or_params *p, double C6[36]);
void or_spont_strain(const or_params *p, const double m[3], double E6[6]);
/* Local magnetostatics (Eq. weak_demag) on explicit arrays in unique-node
 * order, state untouched (need set_params for Ms): the right-hand side b (n)
 * for a field m (n x 3, any values); the CG solve for U~ (n, x0 on entry);
 * the element fields h~_d = -grad U~ / Ms (ne x 3); the energy density. */
int or_ms_rhs_at(or_sim *s, const double *m, double *b);
int or_ms_solve_at(or_sim *s, const double *m, double *U, double tol, int32_t maxit, int32_t *iters);
int or_ms_field(or_sim *s, const double *U, double *hd);
int or_ms_energy(or_sim *s, const double *U, double *e);

/* The elastic preconditioner B of elastic_precond = 1 (unique-node order, n x 3), the points per axis of its
 * grid, and the weight of its diagonal term (1/2 by default; tests may change it). */
int or_precond_apply(or_sim *s, const double *r, double *z);
int or_precond_grid(const or_sim *s, int32_t g[3]);
void or_set_precond_omega(or_sim *s, double omega);

const char *or_last_error(const or_sim *s);
int32_t or_num_threads(void);   /* OpenMP threads the oracle's loops use */
void or_set_num_threads(int32_t k);   /* set them (k > 0) */

#ifdef __cplusplus
}
#endif
#endif
