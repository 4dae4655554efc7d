/* Sanitizer driver for the oracle's C part (AddressSanitizer and
 * UndefinedBehaviorSanitizer): every exported routine on a small mesh pair
 * read from text files "nv nt / xyz rows / tri rows" (argv: ext, int).
 * Exit 0 when every call returns normally; a sanitizer report aborts. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_assemble_rows(int64_t nv, const double *xyz, int64_t nt, const int32_t *tri, double kre, double kim, int ng,
                      int which, int64_t nrows, const int64_t *rows, double *Vo, double *Ko, double *To, double *Do);
int orc_mortar_rows(int64_t nvi, const double *xi, int64_t nti, const int32_t *ti, int64_t nve, const double *xe,
                    int64_t nte, const int32_t *te, int mode, const double *centre, int64_t nrows, const int64_t *rows,
                    double *P);
int orc_plane_wave_rhs(int64_t nv, const double *xyz, int64_t nt, const int32_t *tri, double kre, double kim,
                       const double *d, double *f, double *g);
void orc_pair_blocks(const double *xyz, const int32_t *tri, int64_t t, int64_t s, double kre, double kim, int ng,
                     double *out);
void orc_gauss01(int n, double *x, double *w);
double orc_ss_poly(int kind, int ng, int a, int b, int c, int d);
void orc_set_threads(int n);

static int read_mesh(const char *path, int64_t *nv, int64_t *nt, double **xyz, int32_t **tri)
{
    FILE *f = fopen(path, "r");
    if (!f) return 1;
    long a, b;
    if (fscanf(f, "%ld %ld", &a, &b) != 2) return 1;
    *nv = a;
    *nt = b;
    *xyz = malloc(sizeof(double) * 3 * a);
    *tri = malloc(sizeof(int32_t) * 3 * b);
    for (long i = 0; i < 3 * a; ++i)
        if (fscanf(f, "%lf", *xyz + i) != 1) return 1;
    for (long i = 0; i < 3 * b; ++i)
        if (fscanf(f, "%d", *tri + i) != 1) return 1;
    fclose(f);
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    int64_t nve, nte, nvi, nti;
    double *xe, *xi;
    int32_t *te, *ti;
    if (read_mesh(argv[1], &nve, &nte, &xe, &te) || read_mesh(argv[2], &nvi, &nti, &xi, &ti)) return 3;
    orc_set_threads(4);
    int64_t *rows = malloc(sizeof(int64_t) * nve);
    for (int64_t i = 0; i < nve; ++i) rows[i] = i;
    double complex *V = calloc((size_t)nve * nve, sizeof(double complex));
    double complex *K = calloc((size_t)nve * nve, sizeof(double complex));
    double complex *T = calloc((size_t)nve * nve, sizeof(double complex));
    double complex *D = calloc((size_t)nve * nve, sizeof(double complex));
    for (int which = 1; which <= 3; ++which)
        if (orc_assemble_rows(nve, xe, nte, te, 2.0, which == 3 ? 0.3 : 0.0, 4, which, nve, rows, (double *)V,
                              (double *)K, (double *)T, (double *)D))
            return 4;
    double *P = calloc((size_t)nvi * nve, sizeof(double));
    const double c0[3] = {0, 0, 0};
    int64_t *ri = malloc(sizeof(int64_t) * nvi);
    for (int64_t i = 0; i < nvi; ++i) ri[i] = i;
    if (orc_mortar_rows(nvi, xi, nti, ti, nve, xe, nte, te, 0, c0, nvi, ri, P)) return 5;
    const double d[3] = {0.0, 0.6, 0.8};
    double complex *f = calloc(nve, sizeof(double complex)), *g = calloc(nve, sizeof(double complex));
    if (orc_plane_wave_rhs(nve, xe, nte, te, 3.0, 0.0, d, (double *)f, (double *)g)) return 6;
    double complex blk[36];
    for (int64_t t = 0; t < 4; ++t)
        for (int64_t s = 0; s < nte; s += 7) orc_pair_blocks(xe, te, t, s, 2.0, 0.1, 4, (double *)blk);
    double gx[16], gw[16];
    orc_gauss01(16, gx, gw);
    double sum = 0;
    for (int k = 1; k <= 3; ++k) sum += orc_ss_poly(k, 4, 1, 2, 0, 1);
    printf("oracle driver ok (%g)\n", sum + creal(V[1]) + P[0] + creal(f[0]));
    free(V); free(K); free(T); free(D); free(P); free(f); free(g); free(rows); free(ri);
    free(xe); free(xi); free(te); free(ti);
    return 0;
}
