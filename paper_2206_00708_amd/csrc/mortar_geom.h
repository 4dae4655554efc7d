// Geometry of one (exterior facet, interior triangle) pair of the L2 mortar
// matrix (Sec. 3.1), shared by the host and device assemblies so that both
// take the same steps: the interior triangle is carried onto the facet's
// plane by central projection of its vertices from the origin, the facet is
// clipped by the three edges of the projected triangle (convex polygons),
// and the product of the two P1 bases is integrated over the intersection
// with a 3-point rule per fan triangle (exact for quadratics, so exact here).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace bemtx {
namespace mgeo {

struct V2 { double x, y; };

__host__ __device__ inline double orient(V2 a, V2 b, V2 c) { return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x); }
__host__ __device__ inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

constexpr int kPolyMax = 16;   // clipped polygons hold at most 6 vertices in exact arithmetic

// Keep the part of convex polygon `in` on the left of the directed line a->b;
// boundary points (within tol) are kept.  Returns the vertex count, or -1 if
// rounding would produce more than kPolyMax vertices.
__host__ __device__ inline int keep_left(const V2 *in, int n, V2 a, V2 b, double tol, V2 *out)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const V2 cur = in[i], nxt = in[i + 1 < n ? i + 1 : 0];
        const double sc = orient(a, b, cur), sn = orient(a, b, nxt);
        const bool ic = sc >= -tol, inn = sn >= -tol;
        if (ic) {
            if (m >= kPolyMax) return -1;
            out[m++] = cur;
        }
        if (ic != inn) {
            if (m >= kPolyMax) return -1;
            const double s = sc / (sc - sn);
            out[m++] = V2{cur.x + s * (nxt.x - cur.x), cur.y + s * (nxt.y - cur.y)};
        }
    }
    return m;
}

struct Facet {
    double o[3], e1[3], e2[3], n[3];
    V2 v[3];
    double area, plane, tol;
};

__host__ __device__ inline Facet make_facet(const double *p0, const double *p1, const double *p2)
{
    Facet f;
    double a[3], b[3];
    for (int c = 0; c < 3; ++c) { a[c] = p1[c] - p0[c]; b[c] = p2[c] - p0[c]; f.o[c] = p0[c]; }
    const double nn[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double ln = sqrt(dot3(nn, nn)), la = sqrt(dot3(a, a));
    for (int c = 0; c < 3; ++c) { f.n[c] = nn[c] / ln; f.e1[c] = a[c] / la; }
    f.e2[0] = f.n[1] * f.e1[2] - f.n[2] * f.e1[1];
    f.e2[1] = f.n[2] * f.e1[0] - f.n[0] * f.e1[2];
    f.e2[2] = f.n[0] * f.e1[1] - f.n[1] * f.e1[0];
    f.area = 0.5 * ln;
    const double *P[3] = {p0, p1, p2};
    for (int k = 0; k < 3; ++k) {
        const double d[3] = {P[k][0] - p0[0], P[k][1] - p0[1], P[k][2] - p0[2]};
        f.v[k] = V2{dot3(d, f.e1), dot3(d, f.e2)};
    }
    const double scale = fabs(f.v[1].x) + fabs(f.v[2].x) + fabs(f.v[2].y);
    f.tol = 1e-12 * scale * scale;
    f.plane = dot3(f.n, f.o);
    return f;
}

// barycentric coordinates of q in triangle (a, b, c)
__host__ __device__ inline void bary(V2 a, V2 b, V2 c, V2 q, double *l)
{
    const double det = orient(a, b, c);
    l[1] = orient(a, q, c) / det;
    l[2] = orient(a, b, q) / det;
    l[0] = 1.0 - l[1] - l[2];
}

// unit direction of the centre of a triangle's cone seen from the origin and
// the cone's chord radius
__host__ __device__ inline void cone(const double *p0, const double *p1, const double *p2, double *c, double *r)
{
    const double *P[3] = {p0, p1, p2};
    double u[3][3], s[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        const double l = sqrt(dot3(P[a], P[a]));
        for (int k = 0; k < 3; ++k) { u[a][k] = P[a][k] / l; s[k] += u[a][k]; }
    }
    const double ls = sqrt(dot3(s, s));
    for (int k = 0; k < 3; ++k) c[k] = s[k] / ls;
    *r = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d2 = 0;
        for (int k = 0; k < 3; ++k) d2 += (u[a][k] - c[k]) * (u[a][k] - c[k]);
        *r = fmax(*r, sqrt(d2));
    }
}

// cones that may overlap
__host__ __device__ inline bool cones_meet(const double *ci, double ri, const double *ce, double re)
{
    double d2 = 0;
    for (int k = 0; k < 3; ++k) d2 += (ci[k] - ce[k]) * (ci[k] - ce[k]);
    return !(sqrt(d2) > (ri + re) * 1.0001 + 1e-12);
}

// Contribution of interior triangle (q0, q1, q2) to the facet: blk[a][b] =
// int theta_a phi_b over the intersection, *apoly its area.  Returns 1 if the
// pair contributes, 0 if not, -1 if clipping overflowed (degenerate input).
__host__ __device__ inline int pair_block(const Facet &F, const double *q0, const double *q1, const double *q2,
                                          double (&blk)[3][3], double *apoly)
{
    const double *Q[3] = {q0, q1, q2};
    V2 S[3];
    for (int a = 0; a < 3; ++a) {
        const double den = dot3(F.n, Q[a]);
        if (!(den > 0.0)) return 0;
        const double sc = F.plane / den;
        const double q[3] = {sc * Q[a][0] - F.o[0], sc * Q[a][1] - F.o[1], sc * Q[a][2] - F.o[2]};
        S[a] = V2{dot3(q, F.e1), dot3(q, F.e2)};
    }
    if (orient(S[0], S[1], S[2]) <= 0.0) return 0;
    V2 poly[kPolyMax], tmp[kPolyMax];
    int n = 3;
    for (int a = 0; a < 3; ++a) poly[a] = F.v[a];
    for (int a = 0; a < 3 && n >= 3; ++a) {
        n = keep_left(poly, n, S[a], S[a < 2 ? a + 1 : 0], F.tol, tmp);
        if (n < 0) return -1;
        for (int k = 0; k < n; ++k) poly[k] = tmp[k];
    }
    if (n < 3) return 0;
    double ap = 0.0;
    for (int k = 1; k + 1 < n; ++k) ap += 0.5 * orient(poly[0], poly[k], poly[k + 1]);
    if (ap < 1e-14 * F.area) return 0;
    *apoly = ap;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) blk[a][b] = 0.0;
    const double w1 = 2.0 / 3.0, w2 = 1.0 / 6.0;
    for (int k = 1; k + 1 < n; ++k) {
        const V2 A = poly[0], B = poly[k], C = poly[k + 1];
        const double at = 0.5 * orient(A, B, C);
        for (int g = 0; g < 3; ++g) {
            const double l0 = g == 0 ? w1 : w2, l1 = g == 1 ? w1 : w2, l2 = g == 2 ? w1 : w2;
            const V2 q = V2{l0 * A.x + l1 * B.x + l2 * C.x, l0 * A.y + l1 * B.y + l2 * C.y};
            double li[3], le[3];
            bary(S[0], S[1], S[2], q, li);
            bary(F.v[0], F.v[1], F.v[2], q, le);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) blk[a][b] += at / 3.0 * li[a] * le[b];
        }
    }
    return 1;
}

// cell index of a cone centre coordinate on the [-1, 1]^3 candidate grid
__host__ __device__ inline int cell_of(double x, int ncell, double h)
{
    const int c = (int)floor((x + 1.0) / h);
    return c < 0 ? 0 : (c > ncell - 1 ? ncell - 1 : c);
}

}  // namespace mgeo
}  // namespace bemtx
