/*
 * GSPM oracle -- plain CPU FP64 reference.  TEST INFRASTRUCTURE ONLY: only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark call
 * it; the HIP product library shares no code with it.
 *
 * What it computes, and where the paper defines it:
 *   - periodic node identification by wrapping max-face nodes onto their
 *     min-face partners (Sec. 2.5);
 *   - P1 tetrahedral geometry; the global sparse matrices of Eq. (LHS):
 *     Laplacian K, mass M (= F^GS of Eq. (RHS_F)) and the elastic K^mech,
 *     assembled once, as the paper does (Sec. 2.3);
 *   - the right-hand sides of Eq. (RHS_b) by element integration;
 *   - volume averages (Sec. 2.4), the ellipsoid-theorem split and the
 *     far-field demagnetising field -N_d mbar (Sec. 2.1);
 *   - unpreconditioned CG with d pinned DOFs (Sec. 2.5) and the relative
 *     residual criterion of Sec. 3.1;
 *   - optionally the elastic solve preconditioned (Sec. 5.2 names the
 *     elastic CG as the cost to cut) by the Green's operator of the elastic
 *     stiffness on a periodic auxiliary grid, on the periodic system, pinned
 *     afterwards by a translation;
 *   - optionally the local magnetostatic potential of Eq. (demag) in the weak
 *     form (weak_demag), with K^ms and F^ms of Eqs. (LHS), (RHS_F) and
 *     (RHS_b), and its field -grad U~ (Sec. 2.1);
 *   - optionally a rotated crystal frame (App. D): the cubic stiffness, the
 *     spontaneous strain, the anisotropy and the magnetoelastic field taken
 *     in the crystal frame and carried to the sample frame of the mesh;
 *   - one step of the Gauss-Seidel projection method, Algorithm B.1 (App. B),
 *     with the effective field of App. B and the energy of Eq.
 *     (MicromagneticsEnergy), spontaneous strain from App. A.
 * Where the paper is silent the readings are listed in the design notes; the
 * ones this file depends on are named at the point of use.
 */
#include "gspm_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct or_sim {
    int n0, n, ne;
    int *map;            /* n0: caller node -> unique node */
    double *x;           /* n x 3 coordinates of the unique nodes */
    int *tet;            /* ne x 4 unique ids */
    uint8_t *tag;        /* ne */
    int periodic;
    double lo[3], L[3];
    double *vol;         /* ne */
    double *grad;        /* ne x 4 x 3: gradients of the barycentric coordinates */
    double vc;           /* volume of the computational cell */
    double *w;           /* n: sum over magnetic elements of V_e / 4 */
    uint8_t *mag;        /* n: node touched by a magnetic element */
    int *n2e_ptr, *n2e;  /* node -> element incidence */
    int *adj_ptr, *adj;  /* node adjacency (sparsity of the scalar matrices), sorted, with self */
    double *Kmag, *Mmag, *Kall, *Kmech; /* Kmech: 3x3 block per adjacency entry */
    int have_params, have_m;
    or_params p;
    double C[3][3][3][3];
    int p0;
    double *m, *u;       /* n x 3 */
    double *ud;          /* n: local magnetostatic potential U~ */
    struct green_pc *gpc; /* elastic preconditioner (elastic_precond = 1), built by set_params */
    double gpc_omega;    /* weight of its diagonal term (1/2 unless a test changes it) */
    char err[256];
};

struct green_pc;
static void green_free(struct green_pc *g);
static int green_setup(struct or_sim *s);

/* ------------------------------------------------------------------ utils */

static void seterr(or_sim *s, const char *msg) {
    if (s) snprintf(s->err, sizeof s->err, "%s", msg);
}

static double dot(const double *a, const double *b, int n) {
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (int i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

/* Symmetric 3x3 tensor <-> 6 components, order xx yy zz yz xz xy. */
static void sym_from6(const double v[6], double T[3][3]) {
    T[0][0] = v[0]; T[1][1] = v[1]; T[2][2] = v[2];
    T[1][2] = T[2][1] = v[3];
    T[0][2] = T[2][0] = v[4];
    T[0][1] = T[1][0] = v[5];
}
static void sym_to6(double T[3][3], double v[6]) {
    v[0] = T[0][0]; v[1] = T[1][1]; v[2] = T[2][2];
    v[3] = T[1][2]; v[4] = T[0][2]; v[5] = T[0][1];
}

/* Gaussian elimination with partial pivoting on an n x n system (n <= 9),
 * k right-hand sides stored as columns of B (n x k, row-major).  Returns the
 * determinant of A. */
static double gauss_solve(int n, double *A, int k, double *B) {
    double det = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return 0.0;
        if (piv != c) {
            det = -det;
            for (int j = 0; j < n; ++j) { double t = A[c * n + j]; A[c * n + j] = A[piv * n + j]; A[piv * n + j] = t; }
            for (int j = 0; j < k; ++j) { double t = B[c * k + j]; B[c * k + j] = B[piv * k + j]; B[piv * k + j] = t; }
        }
        det *= A[c * n + c];
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            for (int j = 0; j < k; ++j) B[r * k + j] -= f * B[c * k + j];
        }
    }
    for (int c = n - 1; c >= 0; --c)
        for (int j = 0; j < k; ++j) {
            double v = B[c * k + j];
            for (int q = c + 1; q < n; ++q) v -= A[c * n + q] * B[q * k + j];
            B[c * k + j] = v / A[c * n + c];
        }
    return det;
}

/* ------------------------------------------------------------- material */

/* The crystal orientation of App. D: v_sample = R v_crystal (an all-zero
 * matrix means the crystal axes are the sample axes). */
static void crystal_rot(const or_params *p, double R[3][3]) {
    int zero = 1;
    for (int k = 0; k < 9; ++k) zero &= p->crystal_rot[k] == 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = zero ? (i == j) : p->crystal_rot[i * 3 + j];
}

/* Crystal axes along the sample axes (no rotation to apply). */
static int crystal_aligned(const or_params *p) {
    double R[3][3];
    crystal_rot(p, R);
    int ident = 1;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) ident &= R[i][j] == (double)(i == j);
    return ident;
}

/* Cubic stiffness as a full fourth-order tensor in the crystal frame:
 * C_ijkl = c12 d_ij d_kl + c44 (d_ik d_jl + d_il d_jk) + (c11 - c12 - 2 c44) sum_p d_ip d_jp d_kp d_lp,
 * carried to the sample frame as a fourth-order tensor (App. D):
 * C'_ijkl = R_ia R_jb R_kc R_ld C_abcd. */
static void cubic_tensor(const or_params *p, double C[3][3][3][3]) {
    double Cc[3][3][3][3], R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double v = p->c12 * (i == j) * (k == l) + p->c44 * ((i == k) * (j == l) + (i == l) * (j == k));
                    if (i == j && j == k && k == l) v += p->c11 - p->c12 - 2.0 * p->c44;
                    Cc[i][j][k][l] = v;
                }
    crystal_rot(p, R);
    /* one index at a time: T <- R applied to the first, second, third, fourth index */
    double T[3][3][3][3];
    memcpy(C, Cc, sizeof Cc);
    for (int pass = 0; pass < (crystal_aligned(p) ? 0 : 4); ++pass) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) {
                        double v = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            if (pass == 0) v += R[i][a] * C[a][j][k][l];
                            else if (pass == 1) v += R[j][a] * C[i][a][k][l];
                            else if (pass == 2) v += R[k][a] * C[i][j][a][l];
                            else v += R[l][a] * C[i][j][k][a];
                        }
                        T[i][j][k][l] = v;
                    }
        memcpy(C, T, sizeof T);
    }
}

/* m in the crystal frame: m_c = R^T m. */
static void to_crystal(const or_params *p, const double m[3], double mc[3]) {
    double R[3][3];
    crystal_rot(p, R);
    for (int a = 0; a < 3; ++a) mc[a] = R[0][a] * m[0] + R[1][a] * m[1] + R[2][a] * m[2];
}

/* A symmetric tensor from the crystal frame to the sample frame: R T R^T. */
static void tensor_to_sample(const or_params *p, double T[3][3]) {
    double R[3][3], X[3][3];
    if (crystal_aligned(p)) return;
    crystal_rot(p, R);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v += R[i][a] * T[a][b] * R[j][b];
            X[i][j] = v;
        }
    memcpy(T, X, sizeof X);
}

static void contract(double C[3][3][3][3], double E[3][3], double S[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) v += C[i][j][k][l] * E[k][l];
            S[i][j] = v;
        }
}

/* Spontaneous strain of a cubic crystal, App. A, for a sample-frame m: the
 * crystal-frame form at m_c = R^T m, carried to the sample frame (App. D,
 * Step 1). */
static void spont_strain(const or_params *p, const double m[3], double E0[3][3]) {
    double mc[3];
    to_crystal(p, m, mc);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            E0[i][j] = (i == j) ? 1.5 * p->lambda100 * (mc[i] * mc[i] - 1.0 / 3.0)
                                : 1.5 * p->lambda111 * mc[i] * mc[j];
    tensor_to_sample(p, E0);
}

/* d E0_ij / d m_k for the sample-frame m: sum_c R (dE0/dm_c) R^T R_kc. */
static void spont_strain_deriv(const or_params *p, const double m[3], int k, double D[3][3]) {
    double mc[3], R[3][3];
    if (crystal_aligned(p)) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                if (i == j) D[i][j] = (i == k) ? 3.0 * p->lambda100 * m[i] : 0.0;
                else D[i][j] = 1.5 * p->lambda111 * ((i == k) * m[j] + (j == k) * m[i]);
            }
        return;
    }
    to_crystal(p, m, mc);
    crystal_rot(p, R);
    memset(D, 0, sizeof(double) * 9);
    for (int c = 0; c < 3; ++c) {
        double Dc[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                if (i == j) Dc[i][j] = (i == c) ? 3.0 * p->lambda100 * mc[i] : 0.0;
                else Dc[i][j] = 1.5 * p->lambda111 * ((i == c) * mc[j] + (j == c) * mc[i]);
            }
        tensor_to_sample(p, Dc);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) D[i][j] += Dc[i][j] * R[k][c];
    }
}

/* Cubic anisotropy kappa_1 (m1^2 m2^2 + m2^2 m3^2 + m3^2 m1^2) of the
 * crystal-frame components, and its sample-frame gradient R (dpsi/dm_c). */
static double anis_energy(const or_params *p, const double m[3]) {
    double c[3];
    to_crystal(p, m, c);
    return p->K1 * (c[0] * c[0] * c[1] * c[1] + c[1] * c[1] * c[2] * c[2] + c[2] * c[2] * c[0] * c[0]);
}

static void anis_gradient(const or_params *p, const double m[3], double g[3]) {
    double c[3], gc[3], R[3][3];
    to_crystal(p, m, c);
    crystal_rot(p, R);
    for (int k = 0; k < 3; ++k) {
        double others = 0.0;
        for (int l = 0; l < 3; ++l)
            if (l != k) others += c[l] * c[l];
        gc[k] = 2.0 * p->K1 * c[k] * others;
    }
    for (int k = 0; k < 3; ++k) g[k] = R[k][0] * gc[0] + R[k][1] * gc[1] + R[k][2] * gc[2];
}

void or_stiffness_voigt(const or_params *p, double C6[36]) {
    static const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    double C[3][3][3][3];
    cubic_tensor(p, C);
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) C6[r * 6 + c] = C[ij[r][0]][ij[r][1]][ij[c][0]][ij[c][1]];
}

void or_spont_strain(const or_params *p, const double m[3], double E6[6]) {
    double E0[3][3];
    spont_strain(p, m, E0);
    sym_to6(E0, E6);
}

/* Solve C : X = S for symmetric X in the six independent components. */
static void cubic_compliance_apply(double C[3][3][3][3], const double S6[6], double X6[6]) {
    static const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    double A[36], B[6];
    for (int r = 0; r < 6; ++r) {
        for (int c = 0; c < 6; ++c) {
            int k = ij[c][0], l = ij[c][1];
            A[r * 6 + c] = (k == l) ? C[ij[r][0]][ij[r][1]][k][l] : 2.0 * C[ij[r][0]][ij[r][1]][k][l];
        }
        B[r] = S6[r];
    }
    gauss_solve(6, A, 1, B);
    for (int r = 0; r < 6; ++r) X6[r] = B[r];
}

/* The local part of the effective field h(m) of App. B (everything except the
 * exchange term): cubic anisotropy, Zeeman, far-field demagnetisation -N mbar
 * (Sec. 2.1) and magnetoelastic, h = -(1/(mu0 Ms^2)) d psi / d m with psi from
 * Eq. (MicromagneticsEnergy); E is the total strain at the point. */
void or_h_local(const or_params *p, const double m[3], const double E6[6], const double mbar[3], double h[3]) {
    double C[3][3][3][3], E[3][3], E0[3][3], D[3][3], R[3][3], S[3][3];
    cubic_tensor(p, C);
    sym_from6(E6, E);
    spont_strain(p, m, E0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = E[i][j] - E0[i][j];
    contract(C, R, S);
    double scale = 1.0 / (p->mu0 * p->Ms * p->Ms), ga[3];
    anis_gradient(p, m, ga);
    for (int k = 0; k < 3; ++k) {
        double h_anis = -scale * ga[k];
        double h_zee = p->hext[k] / p->Ms;
        double h_dem = 0.0;
        for (int l = 0; l < 3; ++l) h_dem -= p->Nd[k * 3 + l] * mbar[l];
        spont_strain_deriv(p, m, k, D);
        double me = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) me += S[i][j] * D[i][j];
        h[k] = h_anis + h_zee + h_dem + scale * me;
    }
}

/* Local energy density without exchange and demagnetisation: anisotropy,
 * magnetoelastic and Zeeman terms of Eq. (MicromagneticsEnergy). */
double or_energy_density_local(const or_params *p, const double m[3], const double E6[6]) {
    double C[3][3][3][3], E[3][3], E0[3][3], R[3][3], S[3][3];
    cubic_tensor(p, C);
    sym_from6(E6, E);
    spont_strain(p, m, E0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = E[i][j] - E0[i][j];
    contract(C, R, S);
    double el = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) el += 0.5 * R[i][j] * S[i][j];
    double an = anis_energy(p, m);
    double ze = -p->mu0 * p->Ms * (p->hext[0] * m[0] + p->hext[1] * m[1] + p->hext[2] * m[2]);
    return an + el + ze;
}

/* ----------------------------------------------------------------- mesh */

typedef struct { long long q[3]; int node; } keyed;

static int cmp_keyed(const void *a, const void *b) {
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    for (int k = 0; k < 3; ++k) {
        if (x->q[k] < y->q[k]) return -1;
        if (x->q[k] > y->q[k]) return 1;
    }
    return (x->node > y->node) - (x->node < y->node);
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* Periodic identification, Sec. 2.5: a node on the max face in some axis is
 * wrapped onto the min face; nodes with equal wrapped coordinates (quantised
 * to 1e-9 of the box edge) become one unique node. */
static int wrap_nodes(or_sim *s, const double *xyz, const double lo[3], const double hi[3]) {
    int n0 = s->n0;
    keyed *k = (keyed *)malloc(sizeof(keyed) * (size_t)n0);
    unsigned char *onmax = (unsigned char *)calloc((size_t)n0, 1);
    for (int i = 0; i < n0; ++i) {
        for (int a = 0; a < 3; ++a) {
            double L = hi[a] - lo[a], tol = 1e-9 * L, v = xyz[i * 3 + a];
            if (v < lo[a] - tol || v > hi[a] + tol) {
                free(k); free(onmax);
                seterr(s, "node outside the periodic box");
                return OR_E_MESH;
            }
            if (fabs(v - hi[a]) <= tol) { v = lo[a]; onmax[i] = 1; }
            k[i].q[a] = llround((v - lo[a]) / tol);
        }
        k[i].node = i;
    }
    qsort(k, (size_t)n0, sizeof(keyed), cmp_keyed);
    int *rep_of = (int *)malloc(sizeof(int) * (size_t)n0);
    int *reps = (int *)malloc(sizeof(int) * (size_t)n0);
    int ng = 0, g0 = 0;
    while (g0 < n0) {
        int g1 = g0 + 1;
        while (g1 < n0 && k[g1].q[0] == k[g0].q[0] && k[g1].q[1] == k[g0].q[1] && k[g1].q[2] == k[g0].q[2]) ++g1;
        int rep = -1, count = 0;
        for (int t = g0; t < g1; ++t)
            if (!onmax[k[t].node]) { if (rep < 0) rep = k[t].node; ++count; }
        if (rep < 0 || count > 1) {
            free(k); free(onmax); free(rep_of); free(reps);
            seterr(s, rep < 0 ? "unmatched periodic node" : "duplicate node");
            return OR_E_MESH;
        }
        for (int t = g0; t < g1; ++t) rep_of[k[t].node] = rep;
        reps[ng++] = rep;
        g0 = g1;
    }
    /* Unique ids follow the caller's order of the representatives. */
    qsort(reps, (size_t)ng, sizeof(int), cmp_int);
    int *uid = (int *)malloc(sizeof(int) * (size_t)n0);
    for (int i = 0; i < n0; ++i) uid[i] = -1;
    for (int g = 0; g < ng; ++g) uid[reps[g]] = g;
    s->n = ng;
    s->map = (int *)malloc(sizeof(int) * (size_t)n0);
    s->x = (double *)malloc(sizeof(double) * 3 * (size_t)ng);
    for (int i = 0; i < n0; ++i) s->map[i] = uid[rep_of[i]];
    for (int g = 0; g < ng; ++g)
        for (int a = 0; a < 3; ++a) s->x[g * 3 + a] = xyz[reps[g] * 3 + a];
    free(k); free(onmax); free(rep_of); free(reps); free(uid);
    return OR_OK;
}

/* P1 geometry of one element: gradients g_i of the barycentric coordinates
 * from g_i . (x_k - x_0) = delta_ik (k = 1..3), g_0 = -(g_1 + g_2 + g_3), and the
 * volume |det[x1-x0, x2-x0, x3-x0]| / 6.  Edges use the nearest periodic image. */
static int tet_geometry(const or_sim *s, int e, double *vol, double g[4][3]) {
    double X[4][3];
    for (int v = 0; v < 4; ++v)
        for (int a = 0; a < 3; ++a) X[v][a] = s->x[s->tet[e * 4 + v] * 3 + a];
    double A[9], B[9];
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
            double d = X[k + 1][a] - X[0][a];
            if (s->periodic) d -= s->L[a] * round(d / s->L[a]);
            A[k * 3 + a] = d;          /* row k: edge vector k */
        }
    for (int r = 0; r < 9; ++r) B[r] = (r % 4 == 0) ? 1.0 : 0.0;   /* identity: columns are the three RHS */
    double edge = 0.0;
    for (int r = 0; r < 9; ++r) edge += A[r] * A[r];
    edge = sqrt(edge / 3.0);
    double det = gauss_solve(3, A, 3, B);
    *vol = fabs(det) / 6.0;
    if (!(*vol > 1e-9 * edge * edge * edge)) return OR_E_MESH;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) g[i + 1][a] = B[a * 3 + i];
    for (int a = 0; a < 3; ++a) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
    return OR_OK;
}

static int find_col(const or_sim *s, int row, int col) {
    int lo = s->adj_ptr[row], hi = s->adj_ptr[row + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (s->adj[mid] == col) return mid;
        if (s->adj[mid] < col) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

int or_create(or_sim **out, int32_t n0, const double *xyz, int32_t ne, const int32_t *tets, const uint8_t *tags,
              const double lo[3], const double hi[3], int32_t periodic, char *err, int32_t errlen) {
    *out = NULL;
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    s->n0 = n0; s->ne = ne; s->periodic = periodic ? 1 : 0;
    s->gpc_omega = 0.5;
    for (int a = 0; a < 3; ++a) { s->lo[a] = lo[a]; s->L[a] = hi[a] - lo[a]; }
    int rc = OR_OK;
    if (n0 < 4 || ne < 1) { seterr(s, "empty mesh"); rc = OR_E_ARG; goto fail; }
    for (int a = 0; a < 3; ++a)
        if (!(s->L[a] > 0)) { seterr(s, "bad box"); rc = OR_E_ARG; goto fail; }
    if (s->periodic) {
        rc = wrap_nodes(s, xyz, lo, hi);
        if (rc) goto fail;
    } else {
        s->n = n0;
        s->map = (int *)malloc(sizeof(int) * (size_t)n0);
        s->x = (double *)malloc(sizeof(double) * 3 * (size_t)n0);
        for (int i = 0; i < n0; ++i) s->map[i] = i;
        memcpy(s->x, xyz, sizeof(double) * 3 * (size_t)n0);
    }
    int n = s->n;
    s->tet = (int *)malloc(sizeof(int) * 4 * (size_t)ne);
    s->tag = (uint8_t *)malloc((size_t)ne);
    for (int e = 0; e < ne; ++e) {
        for (int v = 0; v < 4; ++v) {
            int t = tets[e * 4 + v];
            if (t < 0 || t >= n0) { seterr(s, "node index out of range"); rc = OR_E_MESH; goto fail; }
            s->tet[e * 4 + v] = s->map[t];
        }
        for (int v = 0; v < 4; ++v)
            for (int w = v + 1; w < 4; ++w)
                if (s->tet[e * 4 + v] == s->tet[e * 4 + w]) { seterr(s, "element with repeated node"); rc = OR_E_MESH; goto fail; }
        s->tag[e] = tags[e];
    }
    s->vol = (double *)malloc(sizeof(double) * (size_t)ne);
    s->grad = (double *)malloc(sizeof(double) * 12 * (size_t)ne);
    s->w = (double *)calloc((size_t)n, sizeof(double));
    s->mag = (uint8_t *)calloc((size_t)n, 1);
    s->vc = 0.0;
    for (int e = 0; e < ne; ++e) {
        double g[4][3];
        if (tet_geometry(s, e, &s->vol[e], g)) { seterr(s, "degenerate element"); rc = OR_E_MESH; goto fail; }
        for (int v = 0; v < 4; ++v)
            for (int a = 0; a < 3; ++a) s->grad[e * 12 + v * 3 + a] = g[v][a];
        s->vc += s->vol[e];
        if (s->tag[e])
            for (int v = 0; v < 4; ++v) { s->w[s->tet[e * 4 + v]] += s->vol[e] / 4.0; s->mag[s->tet[e * 4 + v]] = 1; }
    }
    /* node -> element incidence */
    s->n2e_ptr = (int *)calloc((size_t)n + 1, sizeof(int));
    for (int e = 0; e < ne; ++e)
        for (int v = 0; v < 4; ++v) s->n2e_ptr[s->tet[e * 4 + v] + 1]++;
    for (int i = 0; i < n; ++i) s->n2e_ptr[i + 1] += s->n2e_ptr[i];
    s->n2e = (int *)malloc(sizeof(int) * 4 * (size_t)ne);
    {
        int *fill = (int *)malloc(sizeof(int) * (size_t)n);
        memcpy(fill, s->n2e_ptr, sizeof(int) * (size_t)n);
        for (int e = 0; e < ne; ++e)
            for (int v = 0; v < 4; ++v) s->n2e[fill[s->tet[e * 4 + v]]++] = e;
        free(fill);
    }
    /* adjacency: all nodes sharing an element with node i (self included), sorted */
    s->adj_ptr = (int *)calloc((size_t)n + 1, sizeof(int));
    {
        int *cnt = (int *)calloc((size_t)n, sizeof(int));
#pragma omp parallel for schedule(dynamic, 256)
        for (int i = 0; i < n; ++i) {
            int deg = s->n2e_ptr[i + 1] - s->n2e_ptr[i];
            int *buf = (int *)malloc(sizeof(int) * 4 * (size_t)deg);
            int c = 0;
            for (int t = s->n2e_ptr[i]; t < s->n2e_ptr[i + 1]; ++t)
                for (int v = 0; v < 4; ++v) buf[c++] = s->tet[s->n2e[t] * 4 + v];
            qsort(buf, (size_t)c, sizeof(int), cmp_int);
            int u = 0;
            for (int t = 0; t < c; ++t)
                if (t == 0 || buf[t] != buf[t - 1]) ++u;
            cnt[i] = u;
            free(buf);
        }
        for (int i = 0; i < n; ++i) s->adj_ptr[i + 1] = s->adj_ptr[i] + cnt[i];
        free(cnt);
    }
    s->adj = (int *)malloc(sizeof(int) * (size_t)s->adj_ptr[n]);
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < n; ++i) {
        int deg = s->n2e_ptr[i + 1] - s->n2e_ptr[i];
        int *buf = (int *)malloc(sizeof(int) * 4 * (size_t)deg);
        int c = 0;
        for (int t = s->n2e_ptr[i]; t < s->n2e_ptr[i + 1]; ++t)
            for (int v = 0; v < 4; ++v) buf[c++] = s->tet[s->n2e[t] * 4 + v];
        qsort(buf, (size_t)c, sizeof(int), cmp_int);
        int o = s->adj_ptr[i];
        for (int t = 0; t < c; ++t)
            if (t == 0 || buf[t] != buf[t - 1]) s->adj[o++] = buf[t];
        free(buf);
    }
    /* Scalar matrices of Eq. (LHS) and the mass matrix F^GS of Eq. (RHS_F),
     * assembled row by row from the elements incident to the row's node. */
    {
        size_t nnz = (size_t)s->adj_ptr[n];
        s->Kmag = (double *)calloc(nnz, sizeof(double));
        s->Mmag = (double *)calloc(nnz, sizeof(double));
        s->Kall = (double *)calloc(nnz, sizeof(double));
#pragma omp parallel for schedule(dynamic, 256)
        for (int i = 0; i < n; ++i)
            for (int t = s->n2e_ptr[i]; t < s->n2e_ptr[i + 1]; ++t) {
                int e = s->n2e[t], li = -1;
                for (int v = 0; v < 4; ++v)
                    if (s->tet[e * 4 + v] == i) li = v;
                const double *gi = &s->grad[e * 12 + li * 3];
                double V = s->vol[e];
                for (int lj = 0; lj < 4; ++lj) {
                    const double *gj = &s->grad[e * 12 + lj * 3];
                    int pos = find_col(s, i, s->tet[e * 4 + lj]);
                    double kij = V * (gi[0] * gj[0] + gi[1] * gj[1] + gi[2] * gj[2]);
                    double mij = V * (li == lj ? 2.0 : 1.0) / 20.0;   /* int phi_i phi_j over a tet */
                    s->Kall[pos] += kij;
                    if (s->tag[e]) { s->Kmag[pos] += kij; s->Mmag[pos] += mij; }
                }
            }
    }
    s->p0 = s->map[0];   /* pinned node for the elastic solve: the caller's node 0 */
    *out = s;
    return OR_OK;
fail:
    if (err && errlen > 0) snprintf(err, (size_t)errlen, "%s", s->err);
    or_destroy(s);
    return rc;
}

void or_destroy(or_sim *s) {
    if (!s) return;
    free(s->map); free(s->x); free(s->tet); free(s->tag); free(s->vol); free(s->grad); free(s->w); free(s->mag);
    free(s->n2e_ptr); free(s->n2e); free(s->adj_ptr); free(s->adj);
    free(s->Kmag); free(s->Mmag); free(s->Kall); free(s->Kmech); free(s->m); free(s->u);
    free(s->ud);
    green_free(s->gpc);
    free(s);
}

int32_t or_n_unique(const or_sim *s) { return s->n; }
void or_node_map(const or_sim *s, int32_t *map) { memcpy(map, s->map, sizeof(int) * (size_t)s->n0); }
void or_geometry(const or_sim *s, double *vol, double *grad) {
    memcpy(vol, s->vol, sizeof(double) * (size_t)s->ne);
    memcpy(grad, s->grad, sizeof(double) * 12 * (size_t)s->ne);
}
double or_total_volume(const or_sim *s) { return s->vc; }
void or_lumped_weights(const or_sim *s, double *w) { memcpy(w, s->w, sizeof(double) * (size_t)s->n); }
int32_t or_pinned_node(const or_sim *s) { return s->p0; }
const char *or_last_error(const or_sim *s) { return s ? s->err : "null oracle"; }

int32_t or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the OpenMP loops (the CPU baseline reports a one-thread rate). */
void or_set_num_threads(int32_t k) {
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

/* Elastic stiffness of Eq. (LHS): block (i,j)_ab = int E(phi_j e_b) : C E(phi_i e_a)
 * = V_e sum_qs C_aqbs d_q phi_i d_s phi_j on each element. */
static void assemble_elastic(or_sim *s) {
    int n = s->n;
    size_t nnz = (size_t)s->adj_ptr[n];
    free(s->Kmech);
    s->Kmech = (double *)calloc(nnz * 9, sizeof(double));
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < n; ++i)
        for (int t = s->n2e_ptr[i]; t < s->n2e_ptr[i + 1]; ++t) {
            int e = s->n2e[t], li = -1;
            for (int v = 0; v < 4; ++v)
                if (s->tet[e * 4 + v] == i) li = v;
            const double *gi = &s->grad[e * 12 + li * 3];
            double V = s->vol[e];
            for (int lj = 0; lj < 4; ++lj) {
                const double *gj = &s->grad[e * 12 + lj * 3];
                int pos = find_col(s, i, s->tet[e * 4 + lj]);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double v = 0.0;
                        for (int q = 0; q < 3; ++q)
                            for (int r = 0; r < 3; ++r) v += s->C[a][q][b][r] * gi[q] * gj[r];
                        s->Kmech[pos * 9 + a * 3 + b] += V * v;
                    }
            }
        }
}

int or_set_params(or_sim *s, const or_params *p) {
    if (!(p->Ms > 0 && p->A >= 0 && p->mu0 > 0 && p->gamma0 > 0 && p->alpha >= 0 && p->cg_tol > 0 && p->cg_maxit > 0)) {
        seterr(s, "invalid parameters");
        return OR_E_ARG;
    }
    if (p->local_demag != 0 && p->local_demag != 1) { seterr(s, "local_demag must be 0 or 1"); return OR_E_ARG; }
    {
        /* the crystal orientation must be a proper rotation (or all zeros) */
        double R[3][3], err = 0.0;
        crystal_rot(p, R);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double v = R[i][0] * R[j][0] + R[i][1] * R[j][1] + R[i][2] * R[j][2];
                err = fmax(err, fabs(v - (i == j)));
            }
        double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) - R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                     R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
        if (!(err < 1e-12) || !(det > 0)) { seterr(s, "crystal_rot is not a proper rotation"); return OR_E_ARG; }
    }
    if (p->local_demag && !s->periodic) {
        seterr(s, "the local magnetostatic solve needs a periodic mesh");
        return OR_E_ARG;
    }
    if (p->elastic_precond != 0 && p->elastic_precond != 1) { seterr(s, "elastic_precond must be 0 or 1"); return OR_E_ARG; }
    if (p->gs_precond != 0 && p->gs_precond != 2) { seterr(s, "gs_precond must be 0 or 2"); return OR_E_ARG; }
    if (!(p->ms_tol >= 0.0)) { seterr(s, "ms_tol must be >= 0"); return OR_E_ARG; }
    if (p->elastic_precond && !s->periodic) {
        seterr(s, "the elastic preconditioner needs a periodic mesh");
        return OR_E_ARG;
    }
    s->p = *p;
    cubic_tensor(p, s->C);
    assemble_elastic(s);
    if (p->elastic_precond) {
        green_setup(s);
    } else {
        green_free(s->gpc);
        s->gpc = NULL;
    }
    s->have_params = 1;
    if (!s->u) s->u = (double *)calloc((size_t)s->n * 3, sizeof(double));
    if (!s->ud) s->ud = (double *)calloc((size_t)s->n, sizeof(double));
    return OR_OK;
}

static int set_nodal(or_sim *s, const double *v, double *dst) {
    /* periodic copies must carry the same value */
    unsigned char *seen = (unsigned char *)calloc((size_t)s->n, 1);
    for (int i = 0; i < s->n0; ++i) {
        int g = s->map[i];
        for (int a = 0; a < 3; ++a)
            if (!isfinite(v[i * 3 + a])) { free(seen); seterr(s, "non-finite field value"); return OR_E_ARG; }
        if (seen[g]) {
            for (int a = 0; a < 3; ++a)
                if (fabs(dst[g * 3 + a] - v[i * 3 + a]) > 1e-12 * (1.0 + fabs(dst[g * 3 + a]))) {
                    free(seen); seterr(s, "periodic copies disagree"); return OR_E_ARG;
                }
        } else {
            for (int a = 0; a < 3; ++a) dst[g * 3 + a] = v[i * 3 + a];
            seen[g] = 1;
        }
    }
    free(seen);
    return OR_OK;
}

/* m is normalised on magnetic nodes and zero on nodes of the inclusions only. */
int or_set_m(or_sim *s, const double *m) {
    if (!s->m) s->m = (double *)calloc((size_t)s->n * 3, sizeof(double));
    int rc = set_nodal(s, m, s->m);
    if (rc) return rc;
    for (int g = 0; g < s->n; ++g) {
        double *v = &s->m[g * 3];
        if (!s->mag[g]) { v[0] = v[1] = v[2] = 0.0; continue; }
        double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(r > 0)) { seterr(s, "zero magnetisation on a magnetic node"); return OR_E_ARG; }
        for (int a = 0; a < 3; ++a) v[a] /= r;
    }
    s->have_m = 1;
    return OR_OK;
}

int or_set_u(or_sim *s, const double *u) {
    if (!s->u) s->u = (double *)calloc((size_t)s->n * 3, sizeof(double));
    return set_nodal(s, u, s->u);
}

int or_set_ud(or_sim *s, const double *ud) {
    if (!s->ud) s->ud = (double *)calloc((size_t)s->n, sizeof(double));
    unsigned char *seen = (unsigned char *)calloc((size_t)s->n, 1);
    for (int i = 0; i < s->n0; ++i) {
        int g = s->map[i];
        if (!isfinite(ud[i])) { free(seen); seterr(s, "non-finite field value"); return OR_E_ARG; }
        if (seen[g] && fabs(s->ud[g] - ud[i]) > 1e-12 * (1.0 + fabs(s->ud[g]))) {
            free(seen); seterr(s, "periodic copies disagree"); return OR_E_ARG;
        }
        s->ud[g] = ud[i];
        seen[g] = 1;
    }
    free(seen);
    return OR_OK;
}

void or_get_ud(const or_sim *s, double *ud) {
    for (int i = 0; i < s->n0; ++i) ud[i] = s->ud ? s->ud[s->map[i]] : 0.0;
}

void or_get_m(const or_sim *s, double *m) {
    for (int i = 0; i < s->n0; ++i)
        for (int a = 0; a < 3; ++a) m[i * 3 + a] = s->m ? s->m[s->map[i] * 3 + a] : 0.0;
}
void or_get_u(const or_sim *s, double *u) {
    for (int i = 0; i < s->n0; ++i)
        for (int a = 0; a < 3; ++a) u[i * 3 + a] = s->u ? s->u[s->map[i] * 3 + a] : 0.0;
}

/* ------------------------------------------------------------ operators */

static void spmv_scalar(const or_sim *s, const double *A, const double *x, double *y, int stride, int comp) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i) {
        double v = 0.0;
        for (int t = s->adj_ptr[i]; t < s->adj_ptr[i + 1]; ++t) v += A[t] * x[s->adj[t] * stride + comp];
        y[i * stride + comp] = v;
    }
}

static void spmv_elastic(const or_sim *s, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int t = s->adj_ptr[i]; t < s->adj_ptr[i + 1]; ++t) {
            const double *B = &s->Kmech[(size_t)t * 9];
            const double *xj = &x[s->adj[t] * 3];
            for (int a = 0; a < 3; ++a) v[a] += B[a * 3 + 0] * xj[0] + B[a * 3 + 1] * xj[1] + B[a * 3 + 2] * xj[2];
        }
        for (int a = 0; a < 3; ++a) y[i * 3 + a] = (i == s->p0) ? 0.0 : v[a];
    }
}

/* eps K + M on one scalar component (contiguous length-n vectors). */
static void apply_gs_scalar(const or_sim *s, double eps, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i) {
        double v = 0.0;
        for (int t = s->adj_ptr[i]; t < s->adj_ptr[i + 1]; ++t) v += (eps * s->Kmag[t] + s->Mmag[t]) * x[s->adj[t]];
        y[i] = v;
    }
}

int or_apply(const or_sim *s, int32_t which, double eps, const double *x, double *y) {
    if (which == 3) {
        if (!s->have_params) return OR_E_STATE;
        spmv_elastic(s, x, y);
        return OR_OK;
    }
    for (int c = 0; c < 3; ++c) {
        if (which == 0) spmv_scalar(s, s->Kmag, x, y, 3, c);
        else if (which == 1) spmv_scalar(s, s->Mmag, x, y, 3, c);
        else if (which == 4) spmv_scalar(s, s->Kall, x, y, 3, c);
        else if (which == 5) {
            spmv_scalar(s, s->Kall, x, y, 3, c);
            y[s->p0 * 3 + c] = 0.0;
        }
        else if (which == 2) {
#pragma omp parallel for schedule(static)
            for (int i = 0; i < s->n; ++i) {
                double v = 0.0;
                for (int t = s->adj_ptr[i]; t < s->adj_ptr[i + 1]; ++t)
                    v += (eps * s->Kmag[t] + s->Mmag[t]) * x[s->adj[t] * 3 + c];
                y[i * 3 + c] = v;
            }
        } else return OR_E_ARG;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------- CG */

typedef void (*apply_fn)(const or_sim *s, const void *ctx, const double *x, double *y);

/* Unpreconditioned conjugate gradients on the DOFs not marked fixed (those
 * rows are the identity with zero right-hand side, Sec. 2.5).  Stops when the
 * recurrence residual satisfies ||r|| <= tol ||b||; b = 0 gives x = 0. */
static int cg(const or_sim *s, apply_fn A, const void *ctx, int len, const uint8_t *fixed, const double *b_in,
              double *x, double tol, int maxit, int *iters) {
    double *b = (double *)malloc(sizeof(double) * (size_t)len);
    double *r = (double *)malloc(sizeof(double) * (size_t)len);
    double *p = (double *)malloc(sizeof(double) * (size_t)len);
    double *q = (double *)malloc(sizeof(double) * (size_t)len);
    for (int i = 0; i < len; ++i) {
        b[i] = fixed[i] ? 0.0 : b_in[i];
        if (fixed[i]) x[i] = 0.0;
    }
    int rc = OR_OK, k = 0;
    double bb = dot(b, b, len);
    if (bb == 0.0) {
        for (int i = 0; i < len; ++i) x[i] = 0.0;
        goto done;
    }
    A(s, ctx, x, q);
    for (int i = 0; i < len; ++i) {
        r[i] = fixed[i] ? 0.0 : b[i] - q[i];
        p[i] = r[i];
    }
    double rr = dot(r, r, len), thr = tol * tol * bb;
    while (rr > thr) {
        if (k >= maxit) { rc = OR_E_NOCONV; break; }
        A(s, ctx, p, q);
        for (int i = 0; i < len; ++i)
            if (fixed[i]) q[i] = 0.0;
        double pq = dot(p, q, len);
        double alpha = rr / pq;
        for (int i = 0; i < len; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rr_new = dot(r, r, len);
        ++k;
        if (!isfinite(rr_new)) { rc = OR_E_NONFINITE; break; }
        if (rr_new <= thr) { rr = rr_new; break; }
        double beta = rr_new / rr;
        for (int i = 0; i < len; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
done:
    *iters = k;
    free(b); free(r); free(p); free(q);
    return rc;
}

static void cg_apply_elastic(const or_sim *s, const void *ctx, const double *x, double *y) {
    (void)ctx;
    spmv_elastic(s, x, y);
}
static void cg_apply_gs(const or_sim *s, const void *ctx, const double *x, double *y) {
    apply_gs_scalar(s, *(const double *)ctx, x, y);
}

static void cg_apply_ms(const or_sim *s, const void *ctx, const double *x, double *y) {
    (void)ctx;
    spmv_scalar(s, s->Kall, x, y, 1, 0);
}

/* K^ms U = b (Eq. weak_demag): the Laplacian over the whole cell with the
 * potential pinned to zero at node p0 (d = 1 pinned DOF, Sec. 2.5). */
static int solve_ms(const or_sim *s, const double *b, double *U, double tol, int maxit, int *iters) {
    uint8_t *fixed = (uint8_t *)calloc((size_t)s->n, 1);
    fixed[s->p0] = 1;
    int rc = cg(s, cg_apply_ms, NULL, s->n, fixed, b, U, tol, maxit, iters);
    free(fixed);
    return rc;
}

static int solve_elastic(const or_sim *s, const double *b, double *u, double tol, int maxit, int *iters) {
    int len = 3 * s->n;
    uint8_t *fixed = (uint8_t *)calloc((size_t)len, 1);
    for (int a = 0; a < 3; ++a) fixed[s->p0 * 3 + a] = 1;
    int rc = cg(s, cg_apply_elastic, NULL, len, fixed, b, u, tol, maxit, iters);
    free(fixed);
    return rc;
}

/* Jacobi-preconditioned CG on the elastic system (the preconditioning the
 * paper leaves aside, Sec. 2.5): M^-1 = diag(K^mech)^-1 on the free DOFs, the
 * same recurrence-residual stopping rule ||r|| <= tol ||b|| as plain CG. */
static int solve_elastic_jacobi(const or_sim *s, const double *b_in, double *u, double tol, int maxit, int *iters) {
    int len = 3 * s->n, rc = OR_OK, k = 0;
    double *b = (double *)calloc((size_t)len, sizeof(double)), *r = (double *)malloc(sizeof(double) * (size_t)len);
    double *z = (double *)malloc(sizeof(double) * (size_t)len), *p = (double *)malloc(sizeof(double) * (size_t)len);
    double *q = (double *)malloc(sizeof(double) * (size_t)len), *minv = (double *)calloc((size_t)len, sizeof(double));
    for (int i = 0; i < s->n; ++i) {
        int self = find_col(s, i, i);
        for (int a = 0; a < 3; ++a) {
            int dof = i * 3 + a;
            if (i == s->p0) { u[dof] = 0.0; continue; }
            b[dof] = b_in[dof];
            minv[dof] = 1.0 / s->Kmech[(size_t)self * 9 + a * 3 + a];
        }
    }
    double bb = dot(b, b, len);
    if (bb == 0.0) {
        for (int i = 0; i < len; ++i) u[i] = 0.0;
        goto done;
    }
    spmv_elastic(s, u, q);
    for (int i = 0; i < len; ++i) { r[i] = b[i] - q[i]; z[i] = minv[i] * r[i]; p[i] = z[i]; }
    for (int a = 0; a < 3; ++a) r[s->p0 * 3 + a] = z[s->p0 * 3 + a] = p[s->p0 * 3 + a] = 0.0;
    double rr = dot(r, r, len), rz = dot(r, z, len), thr = tol * tol * bb;
    while (rr > thr) {
        if (k >= maxit) { rc = OR_E_NOCONV; break; }
        spmv_elastic(s, p, q);
        double alpha = rz / dot(p, q, len);
        for (int i = 0; i < len; ++i) { u[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++k;
        rr = dot(r, r, len);
        if (!isfinite(rr)) { rc = OR_E_NONFINITE; break; }
        if (rr <= thr) break;
        for (int i = 0; i < len; ++i) z[i] = minv[i] * r[i];
        double rz_new = dot(r, z, len), beta = rz_new / rz;
        for (int i = 0; i < len; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
done:
    *iters = k;
    free(b); free(r); free(z); free(p); free(q); free(minv);
    return rc;
}

/* ------------------------------------------ Green's-operator preconditioner
 *
 * The paper runs the elastic CG without a preconditioner and names that
 * solve as the cost to cut (Sec. 5.2).  The elastic stiffness is one
 * homogeneous C on a periodic cell, so its inverse is nearly the lattice
 * Green's operator of the same C: this preconditioner is
 *     B = Q A_g^+ Q^T + omega D^-1
 * with
 *   - a periodic auxiliary grid of g_a = round(L_a / l) points per axis,
 *     l = (V_c / n)^(1/3) the mean node spacing (at least 2 points);
 *   - Q: grid -> mesh nodes, trilinear interpolation of grid values at the
 *     node positions (wrapped into the cell), so Q^T spreads nodal values to
 *     the 8 grid points around each node with the same weights;
 *   - A_g: the P1 stiffness of C on the grid cells split into six Kuhn
 *     tetrahedra (each cell around its main diagonal), a block-circulant
 *     operator whose symbol A(k) = sum_o S(o) exp(2 pi i k.o / g) (S(o) the
 *     3 x 3 coupling of a node to the node at offset o) is inverted mode by
 *     mode, the translation mode k = 0 left out (the pseudo-inverse);
 *   - D: the diagonal of K^mech, omega = 1/2.
 * B is symmetric and positive semi-definite.  It acts on the periodic system
 * K u = b (b with its mean removed, the part a periodic u can balance): CG
 * with B runs on that singular but consistent system, with the stopping rule
 * of Sec. 3.1 on its residual, and the solution is then pinned at node p0 by
 * a translation (the pinned system of Sec. 2.5 has the same solution up to
 * that translation).  Transforms here are plain separable DFTs. */

typedef struct green_pc {
    int g[3];
    double h[3];
    double *Ainv;        /* G x 18: A(k)^-1 / G as a complex 3x3, row-major, (re, im) pairs; zero at k = 0 */
    double *dinv;        /* n x 3: 1 / diag(K^mech) */
} green_pc;

static void green_free(green_pc *g) {
    if (!g) return;
    free(g->Ainv); free(g->dinv); free(g);
}

/* Gradients of the barycentric coordinates of a tetrahedron given by its
 * four vertices; returns the volume. */
static double tet_grads(const double X[4][3], double g[4][3]) {
    double A[9], B[9];
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) A[k * 3 + a] = X[k + 1][a] - X[0][a];
    for (int r = 0; r < 9; ++r) B[r] = (r % 4 == 0) ? 1.0 : 0.0;
    double det = gauss_solve(3, A, 3, B);
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) g[i + 1][a] = B[a * 3 + i];
    for (int a = 0; a < 3; ++a) g[0][a] = -(g[1][a] + g[2][a] + g[3][a]);
    return fabs(det) / 6.0;
}

/* Inverse of a complex 3x3 matrix (re, im pairs, row-major) by cofactors. */
static void cinv3(const double M[18], double out[18]) {
#define RE(i, j) M[((i) * 3 + (j)) * 2]
#define IM(i, j) M[((i) * 3 + (j)) * 2 + 1]
    double cof[3][3][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int r0 = (i + 1) % 3, r1 = (i + 2) % 3, c0 = (j + 1) % 3, c1 = (j + 2) % 3;
            double are = RE(r0, c0) * RE(r1, c1) - IM(r0, c0) * IM(r1, c1);
            double aim = RE(r0, c0) * IM(r1, c1) + IM(r0, c0) * RE(r1, c1);
            double bre = RE(r0, c1) * RE(r1, c0) - IM(r0, c1) * IM(r1, c0);
            double bim = RE(r0, c1) * IM(r1, c0) + IM(r0, c1) * RE(r1, c0);
            cof[i][j][0] = are - bre;
            cof[i][j][1] = aim - bim;
        }
    double dre = 0.0, dim = 0.0;
    for (int j = 0; j < 3; ++j) {
        dre += RE(0, j) * cof[0][j][0] - IM(0, j) * cof[0][j][1];
        dim += RE(0, j) * cof[0][j][1] + IM(0, j) * cof[0][j][0];
    }
    double den = dre * dre + dim * dim;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {   /* inverse = adj / det, adj(i,j) = cof(j,i) */
            double cre = cof[j][i][0], cim = cof[j][i][1];
            out[(i * 3 + j) * 2] = (cre * dre + cim * dim) / den;
            out[(i * 3 + j) * 2 + 1] = (cim * dre - cre * dim) / den;
        }
#undef RE
#undef IM
}

static int green_setup(or_sim *s) {
    green_free(s->gpc);
    s->gpc = NULL;
    green_pc *G = (green_pc *)calloc(1, sizeof(green_pc));
    double ell = cbrt(s->vc / s->n);
    for (int a = 0; a < 3; ++a) {
        int ga = (int)floor(s->L[a] / ell + 0.5);
        G->g[a] = ga < 2 ? 2 : ga;
        G->h[a] = s->L[a] / G->g[a];
    }
    /* stencil S(o), o in {-1,0,1}^3, of the Kuhn-split grid cell */
    double S[27][3][3];
    memset(S, 0, sizeof S);
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int t = 0; t < 6; ++t) {
        int off[4][3] = {{0, 0, 0}};
        for (int v = 1; v < 4; ++v) {
            for (int a = 0; a < 3; ++a) off[v][a] = off[v - 1][a];
            off[v][perm[t][v - 1]] += 1;
        }
        double X[4][3], gr[4][3];
        for (int v = 0; v < 4; ++v)
            for (int a = 0; a < 3; ++a) X[v][a] = off[v][a] * G->h[a];
        double V = tet_grads(X, gr);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                int o = 0;
                for (int a = 2; a >= 0; --a) o = o * 3 + (off[j][a] - off[i][a] + 1);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double v = 0.0;
                        for (int q = 0; q < 3; ++q)
                            for (int r = 0; r < 3; ++r) v += s->C[a][q][b][r] * gr[i][q] * gr[j][r];
                        S[o][a][b] += V * v;
                    }
            }
    }
    int gx = G->g[0], gy = G->g[1], gz = G->g[2];
    size_t ng = (size_t)gx * gy * gz;
    G->Ainv = (double *)calloc(ng * 18, sizeof(double));
    for (int kz = 0; kz < gz; ++kz)
        for (int ky = 0; ky < gy; ++ky)
            for (int kx = 0; kx < gx; ++kx) {
                size_t id = ((size_t)kz * gy + ky) * gx + kx;
                if (id == 0) continue;
                double A[18] = {0};
                for (int o = 0; o < 27; ++o) {
                    int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
                    double ph = 2.0 * M_PI * ((double)kx * ox / gx + (double)ky * oy / gy + (double)kz * oz / gz);
                    double c = cos(ph), sn = sin(ph);
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            A[(a * 3 + b) * 2] += S[o][a][b] * c;
                            A[(a * 3 + b) * 2 + 1] += S[o][a][b] * sn;
                        }
                }
                cinv3(A, &G->Ainv[id * 18]);
                for (int q = 0; q < 18; ++q) G->Ainv[id * 18 + q] /= (double)ng;
            }
    G->dinv = (double *)malloc(sizeof(double) * 3 * (size_t)s->n);
    for (int i = 0; i < s->n; ++i) {
        int self = find_col(s, i, i);
        for (int a = 0; a < 3; ++a) G->dinv[i * 3 + a] = 1.0 / s->Kmech[(size_t)self * 9 + a * 3 + a];
    }
    s->gpc = G;
    return OR_OK;
}

/* Trilinear weights of node i on the 8 grid points around it: grid index and
 * weight per corner (corner bits x, y, z). */
static void green_corners(const or_sim *s, const green_pc *G, int i, size_t idx[8], double wt[8]) {
    int i0[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double f = (s->x[i * 3 + a] - s->lo[a]) / G->h[a];
        f -= G->g[a] * floor(f / G->g[a]);
        int k = (int)floor(f);
        if (k >= G->g[a]) k = G->g[a] - 1;
        i0[a] = k;
        t[a] = f - k;
    }
    for (int c = 0; c < 8; ++c) {
        int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
        int ix = (i0[0] + cx) % G->g[0], iy = (i0[1] + cy) % G->g[1], iz = (i0[2] + cz) % G->g[2];
        idx[c] = ((size_t)iz * G->g[1] + iy) * G->g[0] + ix;
        wt[c] = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
    }
}

/* In-place DFT of complex data (re, im pairs) along one axis of the grid,
 * sign -1 (forward) or +1 (inverse, unnormalised). */
static void dft_axis(const green_pc *G, double *d, int axis, int sign) {
    int n = G->g[axis];
    size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)G->g[0] : (size_t)G->g[0] * G->g[1]);
    size_t total = (size_t)G->g[0] * G->g[1] * G->g[2], lines = total / n;
    double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    for (size_t l = 0; l < lines; ++l) {
        /* first element of line l: index with the axis coordinate zero */
        size_t base = (l / stride) * stride * n + (l % stride);
        for (int k = 0; k < n; ++k) {
            double re = 0.0, im = 0.0;
            for (int j = 0; j < n; ++j) {
                double ph = sign * 2.0 * M_PI * (double)((long long)k * j % n) / n;
                double c = cos(ph), sn = sin(ph);
                const double *v = &d[(base + j * stride) * 2];
                re += v[0] * c - v[1] * sn;
                im += v[0] * sn + v[1] * c;
            }
            tmp[2 * k] = re;
            tmp[2 * k + 1] = im;
        }
        for (int k = 0; k < n; ++k) {
            d[(base + k * stride) * 2] = tmp[2 * k];
            d[(base + k * stride) * 2 + 1] = tmp[2 * k + 1];
        }
    }
    free(tmp);
}

/* z = B r on n x 3 vectors (unique-node order). */
static void green_apply(const or_sim *s, const double *r, double *z) {
    const green_pc *G = s->gpc;
    size_t ng = (size_t)G->g[0] * G->g[1] * G->g[2];
    double *grid = (double *)calloc(ng * 2 * 3, sizeof(double));   /* [comp][point] complex */
    for (int i = 0; i < s->n; ++i) {
        size_t idx[8];
        double wt[8];
        green_corners(s, G, i, idx, wt);
        for (int c = 0; c < 8; ++c)
            for (int a = 0; a < 3; ++a) grid[((size_t)a * ng + idx[c]) * 2] += wt[c] * r[i * 3 + a];
    }
    for (int a = 0; a < 3; ++a)
        for (int ax = 0; ax < 3; ++ax) dft_axis(G, grid + (size_t)a * ng * 2, ax, -1);
    for (size_t k = 0; k < ng; ++k) {
        const double *M = &G->Ainv[k * 18];
        double in[3][2], out[3][2];
        for (int a = 0; a < 3; ++a) { in[a][0] = grid[((size_t)a * ng + k) * 2]; in[a][1] = grid[((size_t)a * ng + k) * 2 + 1]; }
        for (int a = 0; a < 3; ++a) {
            out[a][0] = out[a][1] = 0.0;
            for (int b = 0; b < 3; ++b) {
                double mre = M[(a * 3 + b) * 2], mim = M[(a * 3 + b) * 2 + 1];
                out[a][0] += mre * in[b][0] - mim * in[b][1];
                out[a][1] += mre * in[b][1] + mim * in[b][0];
            }
        }
        for (int a = 0; a < 3; ++a) { grid[((size_t)a * ng + k) * 2] = out[a][0]; grid[((size_t)a * ng + k) * 2 + 1] = out[a][1]; }
    }
    for (int a = 0; a < 3; ++a)
        for (int ax = 0; ax < 3; ++ax) dft_axis(G, grid + (size_t)a * ng * 2, ax, +1);
    for (int i = 0; i < s->n; ++i) {
        size_t idx[8];
        double wt[8];
        green_corners(s, G, i, idx, wt);
        for (int a = 0; a < 3; ++a) {
            double v = s->gpc_omega * G->dinv[i * 3 + a] * r[i * 3 + a];
            for (int c = 0; c < 8; ++c) v += wt[c] * grid[((size_t)a * ng + idx[c]) * 2];
            z[i * 3 + a] = v;
        }
    }
    free(grid);
}

/* K^mech without the pinned rows: the periodic operator. */
static void spmv_elastic_periodic(const or_sim *s, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < s->n; ++i) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int t = s->adj_ptr[i]; t < s->adj_ptr[i + 1]; ++t) {
            const double *B = &s->Kmech[(size_t)t * 9];
            const double *xj = &x[s->adj[t] * 3];
            for (int a = 0; a < 3; ++a) v[a] += B[a * 3 + 0] * xj[0] + B[a * 3 + 1] * xj[1] + B[a * 3 + 2] * xj[2];
        }
        for (int a = 0; a < 3; ++a) y[i * 3 + a] = v[a];
    }
}

/* CG preconditioned by B on the periodic elastic system: b's mean removed,
 * ||r|| <= tol ||b|| on the periodic residual, then u(p0) = 0 by translation. */
static int solve_elastic_green(const or_sim *s, const double *b_in, double *u, double tol, int maxit, int *iters) {
    int len = 3 * s->n, rc = OR_OK, k = 0;
    double *b = (double *)malloc(sizeof(double) * (size_t)len), *r = (double *)malloc(sizeof(double) * (size_t)len);
    double *z = (double *)malloc(sizeof(double) * (size_t)len), *p = (double *)malloc(sizeof(double) * (size_t)len);
    double *q = (double *)malloc(sizeof(double) * (size_t)len);
    double mean[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < 3; ++a) mean[a] += b_in[i * 3 + a];
    for (int i = 0; i < s->n; ++i)
        for (int a = 0; a < 3; ++a) b[i * 3 + a] = b_in[i * 3 + a] - mean[a] / s->n;
    double bb = dot(b, b, len);
    if (bb == 0.0) {
        for (int i = 0; i < len; ++i) u[i] = 0.0;
        goto done;
    }
    spmv_elastic_periodic(s, u, q);
    for (int i = 0; i < len; ++i) r[i] = b[i] - q[i];
    double rr = dot(r, r, len), thr = tol * tol * bb;
    if (rr > thr) {
        green_apply(s, r, z);
        for (int i = 0; i < len; ++i) p[i] = z[i];
    }
    double rz = dot(r, z, len);
    while (rr > thr) {
        if (k >= maxit) { rc = OR_E_NOCONV; break; }
        spmv_elastic_periodic(s, p, q);
        double alpha = rz / dot(p, q, len);
        for (int i = 0; i < len; ++i) { u[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++k;
        rr = dot(r, r, len);
        if (!isfinite(rr)) { rc = OR_E_NONFINITE; break; }
        if (rr <= thr) break;
        green_apply(s, r, z);
        double rz_new = dot(r, z, len), beta = rz_new / rz;
        for (int i = 0; i < len; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
    {
        double sh[3] = {u[s->p0 * 3], u[s->p0 * 3 + 1], u[s->p0 * 3 + 2]};
        for (int i = 0; i < s->n; ++i)
            for (int a = 0; a < 3; ++a) u[i * 3 + a] -= sh[a];
    }
done:
    *iters = k;
    free(b); free(r); free(z); free(p); free(q);
    return rc;
}

int or_precond_apply(or_sim *s, const double *r, double *z) {
    if (!s->have_params || !s->gpc) return OR_E_STATE;
    green_apply(s, r, z);
    return OR_OK;
}

int or_precond_grid(const or_sim *s, int32_t g[3]) {
    if (!s->gpc) return OR_E_STATE;
    for (int a = 0; a < 3; ++a) g[a] = s->gpc->g[a];
    return OR_OK;
}

void or_set_precond_omega(or_sim *s, double omega) { s->gpc_omega = omega; }

/* CG preconditioned by the inverse diagonal dinv on the DOFs not marked
 * fixed (identity rows, zero right-hand side), with the recurrence-residual
 * stopping rule ||r|| <= tol ||b|| of plain CG. */
static int pcg_diag(const or_sim *s, apply_fn A, const void *ctx, int len, const uint8_t *fixed, const double *dinv,
                    const double *b_in, double *x, double tol, int maxit, int *iters) {
    double *b = (double *)malloc(sizeof(double) * (size_t)len), *r = (double *)malloc(sizeof(double) * (size_t)len);
    double *z = (double *)malloc(sizeof(double) * (size_t)len), *p = (double *)malloc(sizeof(double) * (size_t)len);
    double *q = (double *)malloc(sizeof(double) * (size_t)len);
    for (int i = 0; i < len; ++i) {
        b[i] = fixed[i] ? 0.0 : b_in[i];
        if (fixed[i]) x[i] = 0.0;
    }
    int rc = OR_OK, k = 0;
    double bb = dot(b, b, len);
    if (bb == 0.0) {
        for (int i = 0; i < len; ++i) x[i] = 0.0;
        goto done;
    }
    A(s, ctx, x, q);
    for (int i = 0; i < len; ++i) {
        r[i] = fixed[i] ? 0.0 : b[i] - q[i];
        z[i] = fixed[i] ? 0.0 : dinv[i] * r[i];
        p[i] = z[i];
    }
    double rr = dot(r, r, len), rz = dot(r, z, len), thr = tol * tol * bb;
    while (rr > thr) {
        if (k >= maxit) { rc = OR_E_NOCONV; break; }
        A(s, ctx, p, q);
        for (int i = 0; i < len; ++i)
            if (fixed[i]) q[i] = 0.0;
        double alpha = rz / dot(p, q, len);
        for (int i = 0; i < len; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        ++k;
        rr = dot(r, r, len);
        if (!isfinite(rr)) { rc = OR_E_NONFINITE; break; }
        if (rr <= thr) break;
        for (int i = 0; i < len; ++i) z[i] = fixed[i] ? 0.0 : dinv[i] * r[i];
        double rz_new = dot(r, z, len), beta = rz_new / rz;
        for (int i = 0; i < len; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
done:
    *iters = k;
    free(b); free(r); free(z); free(p); free(q);
    return rc;
}

/* One scalar GS solve (eps K + M) x = b on the magnetic nodes (Eq. weak_GS);
 * with gs_precond = 2, CG preconditioned by the inverse of the operator's
 * diagonal (Jacobi), the same stopping rule. */
static int solve_gs(const or_sim *s, double eps, const double *b, double *x, double tol, int maxit, int *iters) {
    uint8_t *fixed = (uint8_t *)malloc((size_t)s->n);
    for (int i = 0; i < s->n; ++i) fixed[i] = !s->mag[i];
    int rc;
    if (s->p.gs_precond == 2) {
        double *dinv = (double *)malloc(sizeof(double) * (size_t)s->n);
        for (int i = 0; i < s->n; ++i) {
            int self = find_col(s, i, i);
            double d = eps * s->Kmag[self] + s->Mmag[self];
            dinv[i] = fixed[i] ? 0.0 : 1.0 / d;
        }
        rc = pcg_diag(s, cg_apply_gs, &eps, s->n, fixed, dinv, b, x, tol, maxit, iters);
        free(dinv);
    } else {
        rc = cg(s, cg_apply_gs, &eps, s->n, fixed, b, x, tol, maxit, iters);
    }
    free(fixed);
    return rc;
}

int or_solve(const or_sim *s, int32_t which, double eps, const double *b, double *x, double tol, int32_t maxit,
             int32_t *iters) {
    if (which == 3 || which == 6 || which == 7) {
        if (!s->have_params) return OR_E_STATE;
        if (which == 7 && !s->gpc) return OR_E_STATE;
        int it = 0, rc = which == 3 ? solve_elastic(s, b, x, tol, maxit, &it)
                                    : (which == 6 ? solve_elastic_jacobi(s, b, x, tol, maxit, &it)
                                                  : solve_elastic_green(s, b, x, tol, maxit, &it));
        *iters = it;
        return rc;
    }
    if (which != 2 && which != 5) return OR_E_ARG;
    int n = s->n, total = 0, rc = OR_OK;
    double *bc = (double *)malloc(sizeof(double) * (size_t)n), *xc = (double *)malloc(sizeof(double) * (size_t)n);
    for (int c = 0; c < 3 && rc == OR_OK; ++c) {
        for (int i = 0; i < n; ++i) { bc[i] = b[i * 3 + c]; xc[i] = x[i * 3 + c]; }
        int it = 0;
        rc = which == 2 ? solve_gs(s, eps, bc, xc, tol, maxit, &it) : solve_ms(s, bc, xc, tol, maxit, &it);
        total += it;
        for (int i = 0; i < n; ++i) x[i * 3 + c] = xc[i];
    }
    free(bc); free(xc);
    *iters = total;
    return rc;
}

/* --------------------------------------------------- averages and RHS */

/* Volume averages over the computational cell (Sec. 2.4).  For a P1 field the
 * element integral is V_e times the vertex mean, so any quadrature rule of
 * degree >= 1 gives sum_j w_j g_j / V_c with w_j the magnetic lumped weights;
 * m and E0(m) vanish in the inclusions.  Ebar = <E0(m)> + C^-1 sigma_ext
 * minimises Eq. (MicromagneticsEnergy) over the homogeneous strain when the
 * heterogeneous strain has zero mean. */
static void averages_at(const or_sim *s, const double *m, double mbar[3], double ebar[6]) {
    double sm[3] = {0, 0, 0}, se[3][3] = {{0}};
    for (int i = 0; i < s->n; ++i) {
        if (!s->mag[i]) continue;
        double E0[3][3];
        spont_strain(&s->p, &m[i * 3], E0);
        for (int a = 0; a < 3; ++a) {
            sm[a] += s->w[i] * m[i * 3 + a];
            for (int b = 0; b < 3; ++b) se[a][b] += s->w[i] * E0[a][b];
        }
    }
    double e6[6], c6[6], C[3][3][3][3];
    for (int a = 0; a < 3; ++a) {
        mbar[a] = sm[a] / s->vc;
        for (int b = 0; b < 3; ++b) se[a][b] /= s->vc;
    }
    sym_to6(se, e6);
    memcpy(C, s->C, sizeof C);
    cubic_compliance_apply(C, s->p.sigma_ext, c6);
    for (int k = 0; k < 6; ++k) ebar[k] = e6[k] + c6[k];
}

/* Elastic right-hand side of Eq. (RHS_b): b_(i,a) = int E(phi_i e_a) : C E0_h with
 * E0_h the P1 interpolant of E0(m) on magnetic elements and zero in the
 * inclusions; the pinned node's rows are zero. */
static void elastic_rhs_full_at(const or_sim *s, const double *m, double *b);

static void elastic_rhs_at(const or_sim *s, const double *m, double *b) {
    elastic_rhs_full_at(s, m, b);
    for (int a = 0; a < 3; ++a) b[s->p0 * 3 + a] = 0.0;
}

/* The same before pinning: the right-hand side of the periodic system. */
static void elastic_rhs_full_at(const or_sim *s, const double *m, double *b) {
    memset(b, 0, sizeof(double) * 3 * (size_t)s->n);
    for (int e = 0; e < s->ne; ++e) {
        if (!s->tag[e]) continue;
        double E0m[3][3] = {{0}}, S[3][3], C[3][3][3][3];
        for (int v = 0; v < 4; ++v) {
            double E0[3][3];
            spont_strain(&s->p, &m[s->tet[e * 4 + v] * 3], E0);
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) E0m[a][c] += 0.25 * E0[a][c];
        }
        memcpy(C, s->C, sizeof C);
        contract(C, E0m, S);
        for (int v = 0; v < 4; ++v) {
            const double *g = &s->grad[e * 12 + v * 3];
            int node = s->tet[e * 4 + v];
            for (int a = 0; a < 3; ++a)
                b[node * 3 + a] += s->vol[e] * (S[a][0] * g[0] + S[a][1] * g[1] + S[a][2] * g[2]);
        }
    }
}

/* ------------------------------------------------ local magnetostatics */

/* Right-hand side of Eq. (weak_demag) as assembled in Eqs. (RHS_F) and
 * (RHS_b): b_i = Ms F^ms_{ij,a} m_{j,a} with F^ms_{ij,a} = -int phi_i d_a phi_j
 * over the whole cell, i.e. b_i = -Ms int phi_i div(m_h).  On a tetrahedron
 * div(m_h) = sum_j m_j . grad(lambda_j) is constant and int phi_i = V_e / 4.
 * m is the nodal field (zero at nodes inside the inclusions only); the mean
 * mbar drops out (its divergence is zero), so this is the right-hand side for
 * m~ as well.  The pinned node's row is zero. */
static void ms_rhs_at(const or_sim *s, const double *m, double *b) {
    memset(b, 0, sizeof(double) * (size_t)s->n);
    for (int e = 0; e < s->ne; ++e) {
        double div = 0.0;
        for (int v = 0; v < 4; ++v) {
            const double *g = &s->grad[e * 12 + v * 3];
            const double *mv = &m[s->tet[e * 4 + v] * 3];
            div += mv[0] * g[0] + mv[1] * g[1] + mv[2] * g[2];
        }
        for (int v = 0; v < 4; ++v) b[s->tet[e * 4 + v]] += -s->p.Ms * 0.25 * s->vol[e] * div;
    }
    b[s->p0] = 0.0;
}

/* The local demagnetising field of element e in units of Ms (Sec. 2.1):
 * h~_d = H~_d / Ms = -grad(U~) / Ms, constant on a P1 element. */
static void ms_field_elem(const or_sim *s, const double *U, int e, double hd[3]) {
    hd[0] = hd[1] = hd[2] = 0.0;
    for (int v = 0; v < 4; ++v) {
        const double *g = &s->grad[e * 12 + v * 3];
        const double uv = U[s->tet[e * 4 + v]];
        for (int a = 0; a < 3; ++a) hd[a] -= uv * g[a] / s->p.Ms;
    }
}

/* (mu0 / 2) int |H~_d|^2 over the cell, averaged over V_c: the local part of
 * the magnetostatic energy of Eq. (MicromagneticsEnergy) (the cross term with
 * the uniform far field vanishes because grad U~ has zero mean). */
static double ms_energy(const or_sim *s, const double *U) {
    double acc = 0.0;
    for (int e = 0; e < s->ne; ++e) {
        double hd[3];
        ms_field_elem(s, U, e, hd);
        acc += s->vol[e] * (hd[0] * hd[0] + hd[1] * hd[1] + hd[2] * hd[2]);
    }
    return 0.5 * s->p.mu0 * s->p.Ms * s->p.Ms * acc / s->vc;
}

int or_ms_rhs_at(or_sim *s, const double *m, double *b) {
    if (!s->have_params) return OR_E_STATE;
    ms_rhs_at(s, m, b);
    return OR_OK;
}

int or_ms_solve_at(or_sim *s, const double *m, double *U, double tol, int32_t maxit, int32_t *iters) {
    if (!s->have_params) return OR_E_STATE;
    double *b = (double *)malloc(sizeof(double) * (size_t)s->n);
    ms_rhs_at(s, m, b);
    int it = 0, rc = solve_ms(s, b, U, tol, maxit, &it);
    *iters = it;
    free(b);
    return rc;
}

int or_ms_field(or_sim *s, const double *U, double *hd) {
    if (!s->have_params) return OR_E_STATE;
    for (int e = 0; e < s->ne; ++e) ms_field_elem(s, U, e, &hd[e * 3]);
    return OR_OK;
}

int or_ms_energy(or_sim *s, const double *U, double *e) {
    if (!s->have_params) return OR_E_STATE;
    *e = ms_energy(s, U);
    return OR_OK;
}

/* Right-hand side of Eq. (RHS_b) for the GS equation (Eq. weak_GS) with
 * f = y + c h: b = M y + ch, ch = sum_e M^e (c h^e) over magnetic elements.
 * h^e at vertex j uses m_j and the element's total strain Ebar + sym grad u
 * (constant on a P1 element); with a potential U (local magnetostatics on)
 * it also holds the element's local demagnetising field -grad U / Ms. */
static void field_rhs_at(const or_sim *s, const double *m, const double *y, const double *u, const double *U,
                         const double ebar[6], const double mbar[3], double c, double *b, double *ch) {
    memset(ch, 0, sizeof(double) * 3 * (size_t)s->n);
    for (int e = 0; e < s->ne; ++e) {
        if (!s->tag[e]) continue;
        double H[3][3] = {{0}}, E[3][3], E6[6], Eb[3][3];
        for (int v = 0; v < 4; ++v) {
            const double *g = &s->grad[e * 12 + v * 3];
            const double *uv = &u[s->tet[e * 4 + v] * 3];
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) H[a][d] += uv[a] * g[d];
        }
        sym_from6(ebar, Eb);
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) E[a][d] = Eb[a][d] + 0.5 * (H[a][d] + H[d][a]);
        sym_to6(E, E6);
        double f[4][3], hd[3] = {0.0, 0.0, 0.0};
        if (U) ms_field_elem(s, U, e, hd);
        for (int v = 0; v < 4; ++v) {
            double h[3];
            or_h_local(&s->p, &m[s->tet[e * 4 + v] * 3], E6, mbar, h);
            for (int a = 0; a < 3; ++a) f[v][a] = c * (h[a] + hd[a]);
        }
        for (int i = 0; i < 4; ++i) {
            int node = s->tet[e * 4 + i];
            for (int j = 0; j < 4; ++j) {
                double mij = s->vol[e] * (i == j ? 2.0 : 1.0) / 20.0;
                for (int a = 0; a < 3; ++a) ch[node * 3 + a] += mij * f[j][a];
            }
        }
    }
    for (int comp = 0; comp < 3; ++comp) spmv_scalar(s, s->Mmag, y, b, 3, comp);
    for (int i = 0; i < 3 * s->n; ++i) b[i] += ch[i];
}

int or_elastic_rhs(or_sim *s, double *b) {
    if (!s->have_params || !s->have_m) return OR_E_STATE;
    elastic_rhs_at(s, s->m, b);
    return OR_OK;
}

int or_field_rhs(or_sim *s, double c, double *b, double *ch) {
    if (!s->have_params || !s->have_m) return OR_E_STATE;
    double mbar[3], ebar[6];
    averages_at(s, s->m, mbar, ebar);
    field_rhs_at(s, s->m, s->m, s->u, s->p.local_demag ? s->ud : NULL, ebar, mbar, c, b, ch);
    return OR_OK;
}

int or_averages(or_sim *s, double mbar[3], double ebar[6]) {
    if (!s->have_params || !s->have_m) return OR_E_STATE;
    averages_at(s, s->m, mbar, ebar);
    return OR_OK;
}

/* ------------------------------------------------------------ the step */

/* GS initial guess: the lumped estimate y + ch / w of f (the solution is close
 * to f when eps is small, Sec. 2.1); zero off the magnetic nodes. */
static void gs_guess(const or_sim *s, const double *y, const double *ch, int comp, double *x) {
    for (int i = 0; i < s->n; ++i) x[i] = s->mag[i] ? y[i * 3 + comp] + ch[i * 3 + comp] / s->w[i] : 0.0;
}

static int gs_component(const or_sim *s, double eps, const double *b, const double *y, const double *ch, int comp,
                        double *out, int *iters) {
    int n = s->n;
    double *bc = (double *)calloc((size_t)n, sizeof(double)), *xc = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) bc[i] = b[i * 3 + comp];
    gs_guess(s, y, ch, comp, xc);
    int rc = solve_gs(s, eps, bc, xc, s->p.cg_tol, s->p.cg_maxit, iters);
    for (int i = 0; i < n; ++i) out[i * 3 + comp] = xc[i];
    free(bc); free(xc);
    return rc;
}

/* Algorithm B.1 (App. B) in the finite-element form of Eq. (weak_GS):
 * (1 - eps lap)^-1 [y + c h] is the solution g of (eps K + M) g = M y + c M h,
 * with eps = A* dtau = l_ex^2 dtau (SI lengths), dtau = gamma0 Ms dt.
 * The updates of Step 2 use the values printed in the algorithm: rows 1 and 2
 * take m^n and g^n, row 3 takes m* and g*; g* uses h[m^n].  Elasticity is
 * solved once per step at m^n and its displacement is held for h[m*]. */
int or_step(or_sim *s, double dt, int32_t nsteps, or_stats *st) {
    if (!s->have_params || !s->have_m) { seterr(s, "step before params and m"); return OR_E_STATE; }
    if (!(dt > 0) || nsteps < 0) { seterr(s, "bad dt or step count"); return OR_E_ARG; }
    const or_params *p = &s->p;
    int n = s->n;
    size_t sz = sizeof(double) * 3 * (size_t)n;
    double *b = (double *)malloc(sz), *ch = (double *)malloc(sz), *g = (double *)malloc(sz);
    double *ms = (double *)malloc(sz), *gs = (double *)malloc(sz), *mss = (double *)malloc(sz);
    double *u = (double *)malloc(sz), *bm = (double *)malloc(sz);
    double *U = p->local_demag ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
    double dtau = p->gamma0 * p->Ms * dt;
    double lex2 = 2.0 * p->A / (p->mu0 * p->Ms * p->Ms);
    double eps1 = lex2 * dtau, eps3 = p->alpha * eps1;
    int rc = OR_OK;
    if (st) memset(st, 0, sizeof *st);
    for (int step = 0; step < nsteps; ++step) {
        const double *m = s->m;
        double mbar[3], ebar[6];
        int it;
        /* averages at m^n feed the far field and the homogeneous strain */
        averages_at(s, m, mbar, ebar);
        /* mechanical equilibrium, Eq. (weak_elasticity), warm start u^{n-1} */
        memcpy(u, s->u, sz);
        if (p->elastic_precond) {
            elastic_rhs_full_at(s, m, bm);
            rc = solve_elastic_green(s, bm, u, p->cg_tol, p->cg_maxit, &it);
        } else {
            elastic_rhs_at(s, m, bm);
            rc = solve_elastic(s, bm, u, p->cg_tol, p->cg_maxit, &it);
        }
        if (st) st->mech_iters += it;
        if (rc) break;
        /* local magnetostatics, Eq. (weak_demag), at m^n, warm start U~^{n-1};
         * held for h[m*] like the displacement */
        if (U) {
            ms_rhs_at(s, m, bm);
            memcpy(U, s->ud, sizeof(double) * (size_t)n);
            /* reading: the magnetostatic stopping test is tighter than the others (ms_tol,
             * 1e-3 cg_tol by default, not below 1e-12) since K^ms's conditioning grows as (L/h)^2 */
            rc = solve_ms(s, bm, U, p->ms_tol > 0.0 ? p->ms_tol : fmax(1e-3 * p->cg_tol, 1e-12), p->cg_maxit, &it);
            if (st) st->ms_iters += it;
            if (rc) break;
        }
        if (p->precession) {
            /* Step 1: g^n for all three components */
            field_rhs_at(s, m, m, u, U, ebar, mbar, dtau, b, ch);
            for (int c = 0; c < 3 && !rc; ++c) {
                rc = gs_component(s, eps1, b, m, ch, c, g, &it);
                if (st) st->gs_iters[c] += it;
            }
            if (rc) break;
            /* Step 2, rows 1 and 2 */
            for (int i = 0; i < n; ++i) {
                const double *mi = &m[i * 3], *gi = &g[i * 3];
                ms[i * 3 + 0] = mi[0] + (gi[1] * mi[2] - gi[2] * mi[1]);
                ms[i * 3 + 1] = mi[1] + (gi[2] * mi[0] - gi[0] * mi[2]);
                ms[i * 3 + 2] = mi[2];
            }
            /* Step 1, g* for components 1 and 2 with h[m^n] */
            for (int c = 0; c < 2; ++c) spmv_scalar(s, s->Mmag, ms, b, 3, c);
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < 2; ++c) b[i * 3 + c] += ch[i * 3 + c];
            for (int c = 0; c < 2 && !rc; ++c) {
                rc = gs_component(s, eps1, b, ms, ch, c, gs, &it);
                if (st) st->gs_iters[3 + c] += it;
            }
            if (rc) break;
            /* Step 2, row 3 */
            for (int i = 0; i < n; ++i)
                ms[i * 3 + 2] = m[i * 3 + 2] + (gs[i * 3 + 0] * ms[i * 3 + 1] - gs[i * 3 + 1] * ms[i * 3 + 0]);
        } else {
            memcpy(ms, m, sz);
        }
        /* Step 3: damped solve with h[m*] (averages re-evaluated at m*) */
        {
            double mbar2[3], ebar2[6];
            averages_at(s, ms, mbar2, ebar2);
            field_rhs_at(s, ms, ms, u, U, ebar2, mbar2, p->alpha * dtau, b, ch);
            for (int c = 0; c < 3 && !rc; ++c) {
                rc = gs_component(s, eps3, b, ms, ch, c, mss, &it);
                if (st) st->gs_iters[5 + c] += it;
            }
            if (rc) break;
        }
        /* Step 4: unit length on the magnetic nodes */
        double dsum = 0.0;
        int nmag = 0, bad = 0;
        for (int i = 0; i < n; ++i) {
            double *v = &mss[i * 3];
            if (!s->mag[i]) { v[0] = v[1] = v[2] = 0.0; continue; }
            double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(r > 0) || !isfinite(r)) { bad = 1; break; }
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                v[a] /= r;
                d2 += (v[a] - m[i * 3 + a]) * (v[a] - m[i * 3 + a]);
            }
            dsum += sqrt(d2);
            ++nmag;
        }
        if (bad) { rc = OR_E_NONFINITE; seterr(s, "non-finite magnetisation"); break; }
        memcpy(s->m, mss, sz);
        memcpy(s->u, u, sz);
        if (U) memcpy(s->ud, U, sizeof(double) * (size_t)n);
        if (st) { st->steps_done = step + 1; st->dm_avg = nmag ? dsum / nmag : 0.0; }
    }
    if (rc == OR_E_NOCONV) seterr(s, "CG did not converge");
    free(b); free(ch); free(g); free(ms); free(gs); free(mss); free(u); free(bm); free(U);
    return rc;
}

/* --------------------------------------------------------------- energy */

/* Energy densities of Eq. (MicromagneticsEnergy) averaged over the cell:
 * exchange A |grad m|^2 exact for P1; anisotropy, Zeeman and magnetoelastic
 * by the vertex rule (V_e / 4 per vertex); stress work -sigma_ext : Ebar (the
 * heterogeneous strain has zero mean); far-field demagnetisation
 * (mu0 Ms^2 / 2) mbar . N mbar. */
int or_energies(or_sim *s, double out[7]) {
    if (!s->have_params || !s->have_m) return OR_E_STATE;
    const or_params *p = &s->p;
    double mbar[3], ebar[6], Eb[3][3], C[3][3][3][3];
    averages_at(s, s->m, mbar, ebar);
    sym_from6(ebar, Eb);
    memcpy(C, s->C, sizeof C);
    double ex = 0, an = 0, ze = 0, me = 0;
    for (int e = 0; e < s->ne; ++e) {
        double V = s->vol[e], H[3][3] = {{0}}, Gm[3][3] = {{0}};
        for (int v = 0; v < 4; ++v) {
            const double *g = &s->grad[e * 12 + v * 3];
            const double *uv = &s->u[s->tet[e * 4 + v] * 3], *mv = &s->m[s->tet[e * 4 + v] * 3];
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) { H[a][d] += uv[a] * g[d]; Gm[a][d] += mv[a] * g[d]; }
        }
        double E[3][3];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) E[a][d] = Eb[a][d] + 0.5 * (H[a][d] + H[d][a]);
        if (s->tag[e])
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) ex += p->A * V * Gm[a][d] * Gm[a][d];
        for (int v = 0; v < 4; ++v) {
            const double *mv = &s->m[s->tet[e * 4 + v] * 3];
            double E0[3][3] = {{0}}, R[3][3], S[3][3];
            if (s->tag[e]) {
                spont_strain(p, mv, E0);
                an += 0.25 * V * anis_energy(p, mv);
                ze += -0.25 * V * p->mu0 * p->Ms * (p->hext[0] * mv[0] + p->hext[1] * mv[1] + p->hext[2] * mv[2]);
            }
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) R[a][d] = E[a][d] - E0[a][d];
            contract(C, R, S);
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) me += 0.25 * V * 0.5 * R[a][d] * S[a][d];
        }
    }
    double sg[3][3], work = 0.0;
    sym_from6(p->sigma_ext, sg);
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) work -= sg[a][d] * Eb[a][d];
    double dem = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) dem += mbar[a] * p->Nd[a * 3 + d] * mbar[d];
    dem *= 0.5 * p->mu0 * p->Ms * p->Ms;
    out[0] = ex / s->vc; out[1] = an / s->vc; out[2] = ze / s->vc; out[3] = me / s->vc;
    out[4] = work; out[5] = dem;
    out[6] = out[0] + out[1] + out[2] + out[3] + out[4] + out[5];
    if (p->local_demag) out[6] += ms_energy(s, s->ud);
    return OR_OK;
}

int or_demag_local_energy(or_sim *s, double *e) {
    if (!s->have_params) return OR_E_STATE;
    *e = ms_energy(s, s->ud);
    return OR_OK;
}

/* ---------------------------------------------------------------- demag */

/* Demagnetisation factors of an ellipsoid with semi-axes a, b, c:
 * N_a = (abc/2) int_0^inf ds / ((a^2+s) sqrt((a^2+s)(b^2+s)(c^2+s))),
 * evaluated by composite Simpson quadrature in t = ln s. */
void or_demag_factors(double a, double b, double c, double N[3]) {
    double ax[3] = {a, b, c};
    double smin = fmin(a, fmin(b, c)), smax = fmax(a, fmax(b, c));
    double t0 = log(smin * smin) - 45.0, t1 = log(smax * smax) + 80.0;
    int steps = 200000;
    double h = (t1 - t0) / steps;
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int i = 0; i <= steps; ++i) {
            double t = t0 + h * i, s = exp(t);
            double f = s / ((ax[k] * ax[k] + s) * sqrt((a * a + s) * (b * b + s) * (c * c + s)));
            double wgt = (i == 0 || i == steps) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
            acc += wgt * f;
        }
        N[k] = 0.5 * a * b * c * acc * h / 3.0;
    }
}
