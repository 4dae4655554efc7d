/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 reference for the dense Galerkin P1
 * boundary integral operators of the Helmholtz equation and for the L2 mortar
 * matrix between two independent triangle meshes of one closed surface, as
 * defined in van 't Wout, "The Boundary Element Method for Acoustic
 * Transmission with Nonconforming Grids" (J. Comput. Appl. Math. 2024):
 *
 *   Green's function G(x,y) = exp(i k |x-y|) / (4 pi |x-y|)    (Sec. 2.1)
 *   V: kernel G;  K: dG/dn(y);  T: dG/dn(x);  D: -d/dn(x) d/dn(y) G
 *                                                             (Sec. 2.1)
 *   Continuous P1 Lagrange test and trial functions           (Sec. 2.4)
 *   Regular pairs: quadrature of order four; pairs that share a vertex:
 *   the semi-analytical (Sauter-Schwab) transformations       (Sec. 5.1)
 *   Mortar matrix P_int,ext[i][j] = <theta_i^int, phi_j^ext>_L2 (Sec. 3.1)
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file.  It shares no code, header, table or constant
 * generator with the GPU library.  Every loop runs over ORDERED triangle
 * pairs; every matrix entry is the plain sum of its element contributions.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - "order four" = the 6-point degree-4 triangle rule (Strang-Fix /
 *    Dunavant) used on every pair that shares no vertex, no near-field
 *    refinement;
 *  - singular rule = Sauter-Schwab regularising maps of [0,1]^4 (6 regions for
 *    coincident, 5 for edge-adjacent, 2 for vertex-adjacent pairs) with an
 *    n-point Gauss-Legendre rule per coordinate (n = 4 by default);
 *  - D in the integration-by-parts (Maue) form
 *      <D u, v> = int int G [curl v(x) . curl u(y) - k^2 n_x.n_y v(x) u(y)];
 *  - curved surfaces: interior functions are carried to the exterior facets
 *    by central projection of interior vertices from a centre point (or by
 *    orthogonal projection onto the facet plane for flat meshes), then
 *    interpolated linearly on the projected triangle.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ---------------------------------------------------------------- rules */

/* 6-point degree-4 rule on a triangle, as barycentric coordinates and
 * weights summing to one (multiply by the area).  Two orbits of type
 * (a, a, 1-2a). */
static void rule6(double bary[6][3], double w[6])
{
    const double a1 = 0.445948490915964886318329253883;
    const double w1 = 0.223381589678011465944827736698;
    const double a2 = 0.091576213509770743459571463402;
    const double w2 = 0.109951743655321867388505596635;
    const double a[2] = {a1, a2}, ww[2] = {w1, w2};
    int q = 0;
    for (int o = 0; o < 2; ++o) {
        double s = a[o], t = 1.0 - 2.0 * a[o];
        double pts[3][3] = {{t, s, s}, {s, t, s}, {s, s, t}};
        for (int r = 0; r < 3; ++r, ++q) {
            for (int c = 0; c < 3; ++c) bary[q][c] = pts[r][c];
            w[q] = ww[o];
        }
    }
}

/* n-point Gauss-Legendre rule on [0,1]: Newton iteration on P_n. */
static void gauss01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {   /* final derivative at the converged root */
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* exported for the quadrature pins */
void orc_rule6(double *bary18, double *w6)
{
    double b[6][3];
    rule6(b, w6);
    memcpy(bary18, b, sizeof b);
}

void orc_gauss01(int n, double *x, double *w) { gauss01(n, x, w); }

/* Thread count of the OpenMP loops (the CPU timing runs one thread and all). */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* --------------------------------------------------------------- geometry */

typedef struct {
    double p[3][3];    /* vertices, CCW seen from outside */
    double n[3];       /* unit normal (p1-p0)x(p2-p0) normalised */
    double area;
    double curl[3][3]; /* surface curl of the barycentric function of vertex a */
} tri_geo;

static void sub3(const double *a, const double *b, double *c) { c[0]=a[0]-b[0]; c[1]=a[1]-b[1]; c[2]=a[2]-b[2]; }
static double dot3(const double *a, const double *b) { return a[0]*b[0]+a[1]*b[1]+a[2]*b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1]*b[2] - a[2]*b[1];
    c[1] = a[2]*b[0] - a[0]*b[2];
    c[2] = a[0]*b[1] - a[1]*b[0];
}

static void make_geo(const double *xyz, const int32_t *t, tri_geo *g)
{
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) g->p[a][c] = xyz[3 * (int64_t)t[a] + c];
    double e1[3], e2[3], cr[3];
    sub3(g->p[1], g->p[0], e1);
    sub3(g->p[2], g->p[0], e2);
    cross3(e1, e2, cr);
    double len = sqrt(dot3(cr, cr));
    g->area = 0.5 * len;
    for (int c = 0; c < 3; ++c) g->n[c] = cr[c] / len;
    /* grad lambda_a = n x (p_{a+2} - p_{a+1}) / (2A); curl lambda_a = n x grad lambda_a
     * = (p_{a+1} - p_{a+2}) / (2A). */
    for (int a = 0; a < 3; ++a) {
        const double *pa1 = g->p[(a + 1) % 3], *pa2 = g->p[(a + 2) % 3];
        for (int c = 0; c < 3; ++c) g->curl[a][c] = (pa1[c] - pa2[c]) / (2.0 * g->area);
    }
}

/* ---------------------------------------------------------------- kernels */

/* G, dG/dn_y and dG/dn_x at one point pair. */
static void kernels(cplx k, const double *x, const double *y, const double *nx, const double *ny,
                    cplx *g, cplx *gk, cplx *gt)
{
    double d[3];
    sub3(x, y, d);
    double r = sqrt(dot3(d, d));
    cplx G = cexp(I * k * r) / (4.0 * M_PI * r);
    cplx f = G * (I * k * r - 1.0) / (r * r);     /* dG/dr / r */
    *g = G;
    *gk = f * (-dot3(d, ny));                      /* (y - x).n_y */
    *gt = f * dot3(d, nx);                         /* (x - y).n_x */
}

/* Local 3x3 blocks, index [op][a][b] with op = V,K,T,D, a = test vertex of
 * tau (x), b = trial vertex of sigma (y), in the triangles' own vertex order. */
typedef struct { cplx m[4][3][3]; } local_blocks;

static void accumulate(local_blocks *L, cplx k, double wgt, const tri_geo *tx, const tri_geo *ty,
                       const double *x, const double *y, const double *phx, const double *phy)
{
    cplx g, gk, gt;
    kernels(k, x, y, tx->n, ty->n, &g, &gk, &gt);
    double nn = dot3(tx->n, ty->n);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double ph = phx[a] * phy[b];
            L->m[0][a][b] += wgt * g * ph;
            L->m[1][a][b] += wgt * gk * ph;
            L->m[2][a][b] += wgt * gt * ph;
            L->m[3][a][b] += wgt * g * (dot3(tx->curl[a], ty->curl[b]) - k * k * nn * ph);
        }
}

static void pair_regular(cplx k, const tri_geo *tx, const tri_geo *ty, local_blocks *L)
{
    double b[6][3], w[6];
    rule6(b, w);
    memset(L, 0, sizeof *L);
    for (int p = 0; p < 6; ++p) {
        double x[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c)
            for (int v = 0; v < 3; ++v) x[c] += b[p][v] * tx->p[v][c];
        for (int q = 0; q < 6; ++q) {
            double y[3] = {0, 0, 0};
            for (int c = 0; c < 3; ++c)
                for (int v = 0; v < 3; ++v) y[c] += b[q][v] * ty->p[v][c];
            accumulate(L, k, w[p] * w[q] * tx->area * ty->area, tx, ty, x, y, b[p], b[q]);
        }
    }
}

/* Sauter-Schwab regions.  Reference triangle {0 <= s2 <= s1 <= 1} with
 * vertices (0,0), (1,0), (1,1); map  chi(s) = Q0 + s1 (Q1-Q0) + s2 (Q2-Q1);
 * P1 shape functions (1-s1, s1-s2, s2).  For the edge case the shared edge is
 * Q0 Q1 in both triangles; for the vertex case the shared vertex is Q0. */
enum { SS_COINC = 3, SS_EDGE = 2, SS_VERT = 1 };

static int ss_region(int kind, int r, double xi, double e1, double e2, double e3,
                     double *xs, double *ys, double *jac)
{
    if (kind == SS_COINC) {
        *jac = xi * xi * xi * e1 * e1 * e2;
        switch (r) {
        case 0: xs[0]=xi; xs[1]=xi*(1-e1+e1*e2); ys[0]=xi*(1-e1*e2*e3); ys[1]=xi*(1-e1); break;
        case 1: ys[0]=xi; ys[1]=xi*(1-e1+e1*e2); xs[0]=xi*(1-e1*e2*e3); xs[1]=xi*(1-e1); break;
        case 2: xs[0]=xi; xs[1]=xi*e1*(1-e2+e2*e3); ys[0]=xi*(1-e1*e2); ys[1]=xi*e1*(1-e2); break;
        case 3: ys[0]=xi; ys[1]=xi*e1*(1-e2+e2*e3); xs[0]=xi*(1-e1*e2); xs[1]=xi*e1*(1-e2); break;
        case 4: xs[0]=xi*(1-e1*e2*e3); xs[1]=xi*e1*(1-e2*e3); ys[0]=xi; ys[1]=xi*e1*(1-e2); break;
        case 5: ys[0]=xi*(1-e1*e2*e3); ys[1]=xi*e1*(1-e2*e3); xs[0]=xi; xs[1]=xi*e1*(1-e2); break;
        default: return 0;
        }
        return 1;
    }
    if (kind == SS_EDGE) {
        *jac = xi * xi * xi * e1 * e1 * (r == 0 ? 1.0 : e2);
        switch (r) {
        case 0: xs[0]=xi; xs[1]=xi*e1*e3; ys[0]=xi*(1-e1*e2); ys[1]=xi*e1*(1-e2); break;
        case 1: xs[0]=xi; xs[1]=xi*e1; ys[0]=xi*(1-e1*e2*e3); ys[1]=xi*e1*e2*(1-e3); break;
        case 2: xs[0]=xi*(1-e1*e2); xs[1]=xi*e1*(1-e2); ys[0]=xi; ys[1]=xi*e1*e2*e3; break;
        case 3: xs[0]=xi*(1-e1*e2*e3); xs[1]=xi*e1*e2*(1-e3); ys[0]=xi; ys[1]=xi*e1; break;
        case 4: xs[0]=xi*(1-e1*e2*e3); xs[1]=xi*e1*(1-e2*e3); ys[0]=xi; ys[1]=xi*e1*e2; break;
        default: return 0;
        }
        return 1;
    }
    if (kind == SS_VERT) {
        *jac = xi * xi * xi * e2;
        switch (r) {
        case 0: xs[0]=xi; xs[1]=xi*e1; ys[0]=xi*e2; ys[1]=xi*e2*e3; break;
        case 1: ys[0]=xi; ys[1]=xi*e1; xs[0]=xi*e2; xs[1]=xi*e2*e3; break;
        default: return 0;
        }
        return 1;
    }
    return 0;
}

/* kind = number of shared vertices; perm_x/perm_y give, for each reference
 * vertex, the triangle's own local vertex index. */
static void pair_singular(cplx k, int kind, int ng, const tri_geo *tx, const tri_geo *ty,
                          const int *perm_x, const int *perm_y, local_blocks *L)
{
    double gx[64], gw[64];
    gauss01(ng, gx, gw);
    memset(L, 0, sizeof *L);
    int nreg = kind == SS_COINC ? 6 : (kind == SS_EDGE ? 5 : 2);
    double Qx[3][3], Qy[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) { Qx[r][c] = tx->p[perm_x[r]][c]; Qy[r][c] = ty->p[perm_y[r]][c]; }
    double scale = 4.0 * tx->area * ty->area;
    for (int reg = 0; reg < nreg; ++reg)
        for (int i0 = 0; i0 < ng; ++i0)
            for (int i1 = 0; i1 < ng; ++i1)
                for (int i2 = 0; i2 < ng; ++i2)
                    for (int i3 = 0; i3 < ng; ++i3) {
                        double xs[2], ys[2], jac;
                        ss_region(kind, reg, gx[i0], gx[i1], gx[i2], gx[i3], xs, ys, &jac);
                        double wgt = gw[i0] * gw[i1] * gw[i2] * gw[i3] * jac * scale;
                        double x[3], y[3];
                        for (int c = 0; c < 3; ++c) {
                            x[c] = Qx[0][c] + xs[0] * (Qx[1][c] - Qx[0][c]) + xs[1] * (Qx[2][c] - Qx[1][c]);
                            y[c] = Qy[0][c] + ys[0] * (Qy[1][c] - Qy[0][c]) + ys[1] * (Qy[2][c] - Qy[1][c]);
                        }
                        double shx[3] = {1.0 - xs[0], xs[0] - xs[1], xs[1]};
                        double shy[3] = {1.0 - ys[0], ys[0] - ys[1], ys[1]};
                        double phx[3], phy[3];
                        for (int r = 0; r < 3; ++r) { phx[perm_x[r]] = shx[r]; phy[perm_y[r]] = shy[r]; }
                        accumulate(L, k, wgt, tx, ty, x, y, phx, phy);
                    }
}


/* Integral of x1^a x2^b y1^c y2^d over the reference pair domain computed
 * through the regularising regions of one singular case (kind = number of
 * shared vertices) -- exposes the region maps and Jacobians to the pins. */
double orc_ss_poly(int kind, int ng, int a, int b, int c, int d)
{
    double gx[64], gw[64];
    if (ng < 1 || ng > 64) return NAN;
    gauss01(ng, gx, gw);
    int nreg = kind == SS_COINC ? 6 : (kind == SS_EDGE ? 5 : 2);
    double s = 0.0;
    for (int reg = 0; reg < nreg; ++reg)
        for (int i0 = 0; i0 < ng; ++i0)
            for (int i1 = 0; i1 < ng; ++i1)
                for (int i2 = 0; i2 < ng; ++i2)
                    for (int i3 = 0; i3 < ng; ++i3) {
                        double xs[2], ys[2], jac;
                        ss_region(kind, reg, gx[i0], gx[i1], gx[i2], gx[i3], xs, ys, &jac);
                        s += gw[i0] * gw[i1] * gw[i2] * gw[i3] * jac *
                             pow(xs[0], a) * pow(xs[1], b) * pow(ys[0], c) * pow(ys[1], d);
                    }
    return s;
}

/* Number of shared vertices between two triangles and the reference-vertex
 * permutations that put the shared vertices first in the same order. */
static int classify(const int32_t *tx, const int32_t *ty, int *px, int *py)
{
    int sx[3], sy[3], ns = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (tx[a] == ty[b]) { sx[ns] = a; sy[ns] = b; ++ns; }
    if (ns == 3) {
        for (int r = 0; r < 3; ++r) { px[r] = r; py[r] = r; }
    } else if (ns == 2) {
        px[0] = sx[0]; px[1] = sx[1]; px[2] = 3 - sx[0] - sx[1];
        py[0] = sy[0]; py[1] = sy[1]; py[2] = 3 - sy[0] - sy[1];
    } else if (ns == 1) {
        for (int r = 0; r < 3; ++r) { px[r] = (sx[0] + r) % 3; py[r] = (sy[0] + r) % 3; }
    }
    return ns;
}

/* Element blocks of one ordered pair, exported for the element-level pins.
 * which: bit 0 = regular pairs, bit 1 = singular pairs (others give zero). */
static void pair_blocks(cplx k, int ng, int which, const double *xyz, const int32_t *tri,
                        int64_t t, int64_t s, local_blocks *L)
{
    tri_geo gx, gy;
    make_geo(xyz, tri + 3 * t, &gx);
    make_geo(xyz, tri + 3 * s, &gy);
    int px[3], py[3];
    int ns = classify(tri + 3 * t, tri + 3 * s, px, py);
    if (ns == 0) {
        if (which & 1) pair_regular(k, &gx, &gy, L);
        else memset(L, 0, sizeof *L);
    } else {
        if (which & 2) pair_singular(k, ns, ng, &gx, &gy, px, py, L);
        else memset(L, 0, sizeof *L);
    }
}

void orc_pair_blocks(const double *xyz, const int32_t *tri, int64_t t, int64_t s,
                     double kre, double kim, int ng, double *out /* [4][3][3] complex */)
{
    local_blocks L;
    pair_blocks(kre + I * kim, ng, 3, xyz, tri, t, s, &L);
    memcpy(out, L.m, sizeof L.m);
}

/* ------------------------------------------------------------- assembly */

/* vertex -> triangles adjacency (CSR) */
static void vertex_star(int64_t nv, int64_t nt, const int32_t *tri, int64_t **ptr_out, int64_t **idx_out)
{
    int64_t *ptr = calloc(nv + 1, sizeof *ptr), *idx = malloc(3 * nt * sizeof *idx), *fill;
    for (int64_t t = 0; t < 3 * nt; ++t) ptr[tri[t] + 1]++;
    for (int64_t v = 0; v < nv; ++v) ptr[v + 1] += ptr[v];
    fill = malloc(nv * sizeof *fill);
    memcpy(fill, ptr, nv * sizeof *fill);
    for (int64_t t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a) idx[fill[tri[3 * t + a]]++] = t;
    free(fill);
    *ptr_out = ptr; *idx_out = idx;
}

/*
 * Rows of the four dense Galerkin matrices (row = test vertex i, column =
 * trial vertex j):  X[i][j] = sum over triangles tau containing i and sigma
 * containing j of the local element entry.  Outputs are row-major complex
 * [nrows][nv], any may be NULL.  which: 1 regular only, 2 singular only,
 * 3 both.  ng: Gauss points per coordinate of the singular rule.
 * Returns 0, or -1 on an invalid argument.
 */
int orc_assemble_rows(int64_t nv, const double *xyz, int64_t nt, const int32_t *tri,
                      double kre, double kim, int ng, int which,
                      int64_t nrows, const int64_t *rows,
                      double *Vo, double *Ko, double *To, double *Do)
{
    if (nv <= 0 || nt <= 0 || ng < 1 || ng > 64) return -1;
    for (int64_t r = 0; r < nrows; ++r) if (rows[r] < 0 || rows[r] >= nv) return -1;
    cplx k = kre + I * kim;
    cplx *out[4] = {(cplx *)Vo, (cplx *)Ko, (cplx *)To, (cplx *)Do};
    for (int op = 0; op < 4; ++op)
        if (out[op]) memset(out[op], 0, (size_t)nrows * nv * sizeof(cplx));
    int64_t *sptr, *sidx;
    vertex_star(nv, nt, tri, &sptr, &sidx);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        for (int64_t e = sptr[i]; e < sptr[i + 1]; ++e) {
            int64_t t = sidx[e];
            int a = 0;
            while (tri[3 * t + a] != i) ++a;
            for (int64_t s = 0; s < nt; ++s) {
                local_blocks L;
                pair_blocks(k, ng, which, xyz, tri, t, s, &L);
                for (int b = 0; b < 3; ++b) {
                    int64_t j = tri[3 * s + b];
                    for (int op = 0; op < 4; ++op)
                        if (out[op]) out[op][r * nv + j] += L.m[op][a][b];
                }
            }
        }
    }
    free(sptr); free(sidx);
    return 0;
}

/* ---------------------------------------------------------------- mortar */

typedef struct { double u, v; } pt2;

static double cross2(pt2 a, pt2 b, pt2 c) { return (b.u - a.u) * (c.v - a.v) - (b.v - a.v) * (c.u - a.u); }

/* Clip the convex polygon poly (n points) by the half-plane left of a->b
 * (points on the line count as inside).  Returns the new size. */
static int clip_halfplane(const pt2 *poly, int n, pt2 a, pt2 b, double tol, pt2 *out)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        pt2 p = poly[i], q = poly[(i + 1) % n];
        double dp = cross2(a, b, p), dq = cross2(a, b, q);
        int ip = dp >= -tol, iq = dq >= -tol;
        if (ip) out[m++] = p;
        if (ip != iq) {
            double t = dp / (dp - dq);
            pt2 z = {p.u + t * (q.u - p.u), p.v + t * (q.v - p.v)};
            out[m++] = z;
        }
    }
    return m;
}

static void bary2(pt2 A, pt2 B, pt2 C, pt2 q, double *l)
{
    double det = cross2(A, B, C);
    l[0] = cross2(q, B, C) / det;
    l[1] = cross2(A, q, C) / det;
    l[2] = cross2(A, B, q) / det;
}

/* Contribution of one (interior triangle ti, exterior triangle te) pair:
 * out[a][b] = int over te of lambda_a^proj(ti) * phi_b(te).  mode 0: central
 * projection of the interior vertices from `centre` onto the plane of te;
 * mode 1: orthogonal projection onto that plane. */
static int mortar_pair(const tri_geo *gi, const tri_geo *ge, int mode, const double *centre,
                       double out[3][3])
{
    memset(out, 0, 9 * sizeof(double));
    double e1[3], e2[3], len;
    sub3(ge->p[1], ge->p[0], e1);
    len = sqrt(dot3(e1, e1));
    for (int c = 0; c < 3; ++c) e1[c] /= len;
    cross3(ge->n, e1, e2);
    pt2 E[3], S[3];
    for (int a = 0; a < 3; ++a) {
        double d[3];
        sub3(ge->p[a], ge->p[0], d);
        E[a].u = dot3(d, e1); E[a].v = dot3(d, e2);
    }
    for (int a = 0; a < 3; ++a) {
        double q[3];
        if (mode == 0) {
            double v[3], off[3];
            sub3(gi->p[a], centre, v);
            sub3(ge->p[0], centre, off);
            double den = dot3(ge->n, v);
            if (den <= 0.0) return 0;
            double t = dot3(ge->n, off) / den;
            for (int c = 0; c < 3; ++c) q[c] = centre[c] + t * v[c];
        } else {
            double d[3];
            sub3(gi->p[a], ge->p[0], d);
            double h = dot3(d, ge->n);
            for (int c = 0; c < 3; ++c) q[c] = gi->p[a][c] - h * ge->n[c];
        }
        double d[3];
        sub3(q, ge->p[0], d);
        S[a].u = dot3(d, e1); S[a].v = dot3(d, e2);
    }
    /* bounding-box reject */
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    double smin_u = 1e300, smax_u = -1e300, smin_v = 1e300, smax_v = -1e300;
    for (int a = 0; a < 3; ++a) {
        umin = fmin(umin, E[a].u); umax = fmax(umax, E[a].u);
        vmin = fmin(vmin, E[a].v); vmax = fmax(vmax, E[a].v);
        smin_u = fmin(smin_u, S[a].u); smax_u = fmax(smax_u, S[a].u);
        smin_v = fmin(smin_v, S[a].v); smax_v = fmax(smax_v, S[a].v);
    }
    double h = umax - umin + vmax - vmin;
    if (smin_u > umax + 1e-12 * h || smax_u < umin - 1e-12 * h ||
        smin_v > vmax + 1e-12 * h || smax_v < vmin - 1e-12 * h) return 0;
    if (cross2(S[0], S[1], S[2]) <= 0.0) return 0;   /* folded projection */
    pt2 poly[16], tmp[16];
    int n = 3;
    for (int a = 0; a < 3; ++a) poly[a] = S[a];
    double tol = 1e-12 * h * h;
    for (int a = 0; a < 3 && n > 0; ++a) {
        n = clip_halfplane(poly, n, E[a], E[(a + 1) % 3], tol, tmp);
        memcpy(poly, tmp, n * sizeof(pt2));
    }
    if (n < 3) return 0;
    double area = 0.0;
    for (int i = 1; i + 1 < n; ++i) area += 0.5 * cross2(poly[0], poly[i], poly[i + 1]);
    double area_e = 0.5 * cross2(E[0], E[1], E[2]);
    if (area < 1e-14 * area_e) return 0;
    /* fan triangulation, 3-point edge-midpoint rule (exact for degree 2) */
    for (int i = 1; i + 1 < n; ++i) {
        pt2 A = poly[0], B = poly[i], C = poly[i + 1];
        double at = 0.5 * cross2(A, B, C);
        pt2 mids[3] = {{0.5 * (A.u + B.u), 0.5 * (A.v + B.v)},
                       {0.5 * (B.u + C.u), 0.5 * (B.v + C.v)},
                       {0.5 * (C.u + A.u), 0.5 * (C.v + A.v)}};
        for (int m = 0; m < 3; ++m) {
            double li[3], le[3];
            bary2(S[0], S[1], S[2], mids[m], li);
            bary2(E[0], E[1], E[2], mids[m], le);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) out[a][b] += at / 3.0 * li[a] * le[b];
        }
    }
    return 1;
}

/*
 * Rows of the mortar matrix P_int,ext (N_int x N_ext), row-major doubles
 * [nrows][nve]:  P[i][j] = sum over interior triangles ti containing i and
 * exterior triangles te containing j of  int_te lambda_i^proj phi_j  dA.
 * mode 0 = central projection from centre[3]; mode 1 = orthogonal.
 */
int orc_mortar_rows(int64_t nvi, const double *xi, int64_t nti, const int32_t *ti,
                    int64_t nve, const double *xe, int64_t nte, const int32_t *te,
                    int mode, const double *centre, int64_t nrows, const int64_t *rows, double *P)
{
    if (nvi <= 0 || nve <= 0) return -1;
    for (int64_t r = 0; r < nrows; ++r) if (rows[r] < 0 || rows[r] >= nvi) return -1;
    memset(P, 0, (size_t)nrows * nve * sizeof(double));
    int64_t *sptr, *sidx;
    vertex_star(nvi, nti, ti, &sptr, &sidx);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        for (int64_t e = sptr[i]; e < sptr[i + 1]; ++e) {
            int64_t t = sidx[e];
            int a = 0;
            while (ti[3 * t + a] != i) ++a;
            tri_geo gi;
            make_geo(xi, ti + 3 * t, &gi);
            for (int64_t s = 0; s < nte; ++s) {
                tri_geo ge;
                make_geo(xe, te + 3 * s, &ge);
                double blk[3][3];
                if (!mortar_pair(&gi, &ge, mode, centre, blk)) continue;
                for (int b = 0; b < 3; ++b) P[r * nve + te[3 * s + b]] += blk[a][b];
            }
        }
    }
    free(sptr); free(sidx);
    return 0;
}

/* Plane-wave load vectors on a mesh (row j = vertex j):
 *   f_j = int phi_j exp(i k d.x),  g_j = int phi_j i k (d.n) exp(i k d.x)
 * with the same 6-point rule; outputs complex [nv]. */
int orc_plane_wave_rhs(int64_t nv, const double *xyz, int64_t nt, const int32_t *tri,
                       double kre, double kim, const double *d, double *fo, double *go)
{
    if (nv <= 0 || nt <= 0) return -1;
    cplx k = kre + I * kim;
    cplx *f = (cplx *)fo, *g = (cplx *)go;
    memset(f, 0, nv * sizeof(cplx));
    memset(g, 0, nv * sizeof(cplx));
    double b[6][3], w[6];
    rule6(b, w);
    for (int64_t t = 0; t < nt; ++t) {
        tri_geo gt;
        make_geo(xyz, tri + 3 * t, &gt);
        double dn = dot3(d, gt.n);
        for (int q = 0; q < 6; ++q) {
            double x[3] = {0, 0, 0};
            for (int c = 0; c < 3; ++c)
                for (int v = 0; v < 3; ++v) x[c] += b[q][v] * gt.p[v][c];
            cplx u = cexp(I * k * dot3(d, x));
            for (int a = 0; a < 3; ++a) {
                double wq = w[q] * gt.area * b[q][a];
                f[tri[3 * t + a]] += wq * u;
                g[tri[3 * t + a]] += wq * I * k * dn * u;
            }
        }
    }
    return 0;
}
