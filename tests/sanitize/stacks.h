/* Reader of the stack list the sanitizer test writes (one stack per block):
 *   nx ny nz h pbc lambda ni T v_top carriers
 *   then nz lines: material eps_r Na Nd
 * Shared by the two sanitizer drivers (test infrastructure). */
#ifndef SANITIZE_STACKS_H
#define SANITIZE_STACKS_H
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int nx, ny, nz, pbc, carriers;
    double h, lambda, ni, T, v_top;
    int *mat;
    double *eps, *Na, *Nd;
} san_stack;

static int san_read(const char *path, san_stack **out) {
    FILE *f = fopen(path, "r");
    if (!f) return -1;
    int n = 0, cap = 0;
    san_stack *v = NULL;
    san_stack s;
    while (fscanf(f, "%d %d %d %lf %d %lf %lf %lf %lf %d", &s.nx, &s.ny, &s.nz, &s.h, &s.pbc, &s.lambda, &s.ni, &s.T,
                  &s.v_top, &s.carriers) == 10) {
        s.mat = (int *)malloc(sizeof(int) * s.nz);
        s.eps = (double *)malloc(sizeof(double) * s.nz);
        s.Na = (double *)malloc(sizeof(double) * s.nz);
        s.Nd = (double *)malloc(sizeof(double) * s.nz);
        for (int k = 0; k < s.nz; ++k)
            if (fscanf(f, "%d %lf %lf %lf", &s.mat[k], &s.eps[k], &s.Na[k], &s.Nd[k]) != 4) { fclose(f); return -1; }
        if (n == cap) {
            cap = cap ? 2 * cap : 16;
            v = (san_stack *)realloc(v, sizeof(san_stack) * cap);
        }
        v[n++] = s;
    }
    fclose(f);
    *out = v;
    return n;
}

static void san_free(san_stack *v, int n) {
    for (int i = 0; i < n; ++i) { free(v[i].mat); free(v[i].eps); free(v[i].Na); free(v[i].Nd); }
    free(v);
}
#endif
