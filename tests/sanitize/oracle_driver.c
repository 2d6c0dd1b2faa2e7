/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: for every stack of
 * the list, Step 0, three forward-Euler steps, two predictor-corrector steps, the
 * residual norms, the Poisson parts and Q-V, on odd and degenerate shapes.  Prints one
 * line per stack (the final relative residual); any sanitizer report fails the run. */
#include "../../oracle/ferro_oracle.c"
#include "stacks.h"

int main(int argc, char **argv) {
    san_stack *v;
    const int n = argc > 1 ? san_read(argv[1], &v) : -1;
    if (n <= 0) { fprintf(stderr, "no stacks\n"); return 2; }
    for (int i = 0; i < n; ++i) {
        const san_stack *s = &v[i];
        orc_desc d = {s->nx, s->ny, s->nz, s->h, s->mat, s->eps, s->Na, s->Nd, -2.5e9, 6e10, 1.5e11, 1e-10, 1e-10,
                      100.0, s->pbc, s->lambda, s->ni, s->T, 0.0, s->v_top, s->carriers, 1.08, 0.81, 1.12};
        const size_t nc = (size_t)s->nx * s->ny * s->nz;
        double *P = (double *)calloc(nc, sizeof(double)), *phi = (double *)calloc(nc, sizeof(double));
        double *f = (double *)calloc(nc, sizeof(double)), *N = (double *)calloc(nc, sizeof(double));
        double *rho = (double *)calloc(nc, sizeof(double)), *sig = (double *)calloc(nc, sizeof(double));
        unsigned r = 12345u + (unsigned)i;
        for (size_t c = 0; c < nc; ++c) {
            r = r * 1664525u + 1013904223u;
            const int k = (int)(c / ((size_t)s->nx * s->ny));
            P[c] = s->mat[k] == 1 ? 0.02 * ((double)(r >> 8) / 16777216.0 - 0.5) : 0.0;
        }
        orc_info info;
        int st = orc_solve(&d, P, phi, 1e-12, 200, &info);
        if (!st) st = orc_run(&d, P, phi, 3, 1e-13, NULL, 1e-12, 200, &info);
        if (!st) st = orc_run_pc(&d, P, phi, 2, 1e-13, NULL, 1e-12, 200, &info);
        double rn = 0, fn = 0, Q = 0, V = 0;
        if (!st) st = orc_residual_norms(&d, P, phi, &rn, &fn);
        if (!st) st = orc_poisson_parts(&d, P, phi, f, N, rho, sig);
        const int qv = orc_qv(&d, P, phi, &Q, &V);
        printf("stack %d %dx%dx%d: status %d |r|/|f| %.3e qv %d\n", i, s->nx, s->ny, s->nz, st,
               fn > 0 ? rn / fn : 0.0, qv);
        free(P); free(phi); free(f); free(N); free(rho); free(sig);
        if (st) { san_free(v, n); return 1; }
    }
    san_free(v, n);
    return 0;
}
