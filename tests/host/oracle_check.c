/* Host driver of the oracle for sanitizer builds: reads a mesh dump (the
 * format of strip_check.cpp), runs two plain steps, one with both
 * preconditioners and one with the local magnetostatic potential, and checks
 * that every result is finite and |m| = 1 on magnetic nodes.
 * Usage: oracle_check <mesh.bin>; exit 0 if every call succeeded. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gspm_oracle.h"

static int fail(const char *what, const or_sim *s) {
    printf("%s failed: %s\n", what, s ? or_last_error(s) : "");
    return 1;
}

int main(int argc, char **argv) {
    setvbuf(stdout, NULL, _IONBF, 0);   /* the sanitizers end the process without flushing stdio */
    if (argc < 2) return 2;
    FILE *fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int64_t n0, ne;
    double lo[3], hi[3];
    size_t got = 0;
    got += fread(&n0, 8, 1, fp);
    got += fread(&ne, 8, 1, fp);
    got += fread(lo, 8, 3, fp);
    got += fread(hi, 8, 3, fp);
    double *xyz = malloc(sizeof(double) * 3 * (size_t)n0);
    int32_t *tets = malloc(sizeof(int32_t) * 4 * (size_t)ne);
    uint8_t *tags = malloc((size_t)ne);
    got += fread(xyz, 8, 3 * (size_t)n0, fp);
    got += fread(tets, 4, 4 * (size_t)ne, fp);
    got += fread(tags, 1, (size_t)ne, fp);
    fclose(fp);
    if (got != (size_t)(8 + 3 * n0 + 4 * ne + ne)) return 2;
    char err[256];
    or_sim *s = NULL;
    if (or_create(&s, (int32_t)n0, xyz, (int32_t)ne, tets, tags, lo, hi, 1, err, sizeof err) != OR_OK) {
        printf("or_create failed: %s\n", err);
        return 1;
    }
    or_params p;
    memset(&p, 0, sizeof p);
    p.Ms = 1.36e6; p.A = 1.5e-11; p.K1 = 1.3e4; p.lambda100 = 2e-4; p.lambda111 = -2e-5;
    p.c11 = 196e9; p.c12 = 156e9; p.c44 = 123e9; p.alpha = 0.5; p.mu0 = 4e-7 * M_PI; p.gamma0 = 2.211e5;
    p.Nd[0] = p.Nd[4] = p.Nd[8] = 1.0 / 3.0;
    p.hext[0] = -0.3 * p.Ms;
    p.sigma_ext[0] = 2e6;
    p.cg_tol = 1e-8;
    p.cg_maxit = 20000;
    p.precession = 1;
    /* a deterministic random start per unique node (xorshift64), copied to its periodic copies */
    const int32_t nu = or_n_unique(s);
    int32_t *map = malloc(sizeof(int32_t) * (size_t)n0);
    double *mu = malloc(sizeof(double) * 3 * (size_t)nu);
    double *m = malloc(sizeof(double) * 3 * (size_t)n0);
    or_node_map(s, map);
    uint64_t st = 88172645463325252ull;
    for (int64_t i = 0; i < 3 * (int64_t)nu; ++i) {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        mu[i] = (double)(st >> 11) / 9007199254740992.0 - 0.5;
    }
    for (int32_t i = 0; i < nu; ++i) {
        mu[3 * i] += 1.0;
        const double r = sqrt(mu[3 * i] * mu[3 * i] + mu[3 * i + 1] * mu[3 * i + 1] + mu[3 * i + 2] * mu[3 * i + 2]);
        for (int a = 0; a < 3; ++a) mu[3 * i + a] /= r;
    }
    for (int64_t i = 0; i < n0; ++i)
        for (int a = 0; a < 3; ++a) m[3 * i + a] = mu[3 * (int64_t)map[i] + a];
    int bad = 0;
    or_stats stats;
    const double dt = 5e-12;
    struct { int elastic_precond, gs_precond, local_demag, steps; } runs[3] = {{0, 0, 0, 2}, {1, 2, 0, 1}, {0, 0, 1, 1}};
    for (int k = 0; k < 3; ++k) {
        p.elastic_precond = runs[k].elastic_precond;
        p.gs_precond = runs[k].gs_precond;
        p.local_demag = runs[k].local_demag;
        if (or_set_params(s, &p) != OR_OK) return fail("or_set_params", s);
        if (k == 0 && or_set_m(s, m) != OR_OK) return fail("or_set_m", s);
        if (or_step(s, dt, runs[k].steps, &stats) != OR_OK) return fail("or_step", s);
        double e[7], mbar[3], ebar[6];
        if (or_energies(s, e) != OR_OK) return fail("or_energies", s);
        if (or_averages(s, mbar, ebar) != OR_OK) return fail("or_averages", s);
        for (int q = 0; q < 7; ++q) bad += !isfinite(e[q]);
        for (int q = 0; q < 3; ++q) bad += !isfinite(mbar[q]);
        printf("run %d: %d steps, elastic %d, GS %d, magnetostatic %d iterations, dm_avg %.3e, total energy %.6e\n", k,
               stats.steps_done, stats.mech_iters, stats.gs_iters[0] + stats.gs_iters[1] + stats.gs_iters[2],
               stats.ms_iters, stats.dm_avg, e[6]);
    }
    or_get_m(s, m);
    double worst = 0.0;
    for (int64_t i = 0; i < n0; ++i) {
        const double r = sqrt(m[3 * i] * m[3 * i] + m[3 * i + 1] * m[3 * i + 1] + m[3 * i + 2] * m[3 * i + 2]);
        if (r > 0.0) worst = fmax(worst, fabs(r - 1.0));
    }
    printf("max ||m| - 1| %.2e\n", worst);
    bad += !(worst < 1e-12);
    or_destroy(s);
    free(map);
    free(mu);
    free(m);
    free(xyz);
    free(tets);
    free(tags);
    return bad ? 1 : 0;
}
