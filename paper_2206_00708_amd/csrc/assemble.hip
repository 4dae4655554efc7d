// Galerkin P1 assembly of the Helmholtz boundary integral operators
// V (kernel G), K (dG/dn_y), T (dG/dn_x) and D (hypersingular, integrated by
// parts) on one triangle mesh, G(x,y) = exp(i k |x-y|) / (4 pi |x-y|)
// (Sec. 2.1, Sec. 2.4), in FP64 on gfx950.
//
//   geometry_kernel   per-triangle table: vertices, unit normal, area, the
//                     six points of the order-four rule, P1 surface curls.
//   regular_tiles     triangle pairs that share no vertex, order-four rule
//                     (6 x 6 points, Sec. 5.1).  One workgroup per unordered
//                     pair of locality blocks (16 x 16 triangles), one
//                     triangle pair per thread; V, K, T and the scalar sum of
//                     G are reduced in registers, D follows from them
//                     (curl.curl S - k^2 n.n V).  The 9 entries of each pair
//                     are summed per vertex slot through LDS in a fixed order
//                     (runs of slot-sorted corners) and the block-pair tile
//                     is written once.  Because the
//                     regular rule is symmetric in (x, y), the tile of
//                     (b1, b2) also provides (b2, b1): V, D transpose to
//                     themselves and K, T into each other.
//   gather_tiles      dense entries (i, j) and (j, i) = one fixed-order sum
//                     of the tile entries of the blocks containing i and j.
//   singular_pairs    ordered pairs sharing 3 / 2 / 1 vertices: Sauter-Schwab
//                     regularising maps of [0,1]^4 with ng^4 Gauss points per
//                     region (6 / 5 / 2 regions); 16 lanes per pair.
//   near_scatter      adds the singular contributions of each touched entry
//                     in a fixed order.
// Every entry is produced by a fixed sequence of additions, so the result is
// bitwise reproducible run to run.
#include <cmath>

#include "internal.h"
#include "phase.h"
#include "rule6.h"

namespace bemtx {

namespace {


__device__ inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

}  // namespace

__global__ void geometry_kernel(const double *__restrict__ xyz, const int32_t *__restrict__ tri, int nt,
                                TriGeo *__restrict__ geo, TriGeoF *__restrict__ geof)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    TriGeo g;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) g.p[a][c] = xyz[3 * (int64_t)tri[3 * t + a] + c];
    double e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = g.p[1][c] - g.p[0][c]; e2[c] = g.p[2][c] - g.p[0][c]; }
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double len = sqrt(dot3(cr, cr));
    g.area = 0.5 * len;
    for (int c = 0; c < 3; ++c) g.n[c] = cr[c] / len;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) g.curl[a][c] = (g.p[(a + 1) % 3][c] - g.p[(a + 2) % 3][c]) / len;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        for (int c = 0; c < 3; ++c)
            g.qp[q][c] = r6_bary(q, 0) * g.p[0][c] + r6_bary(q, 1) * g.p[1][c] + r6_bary(q, 2) * g.p[2][c];
    for (int c = 0; c < 3; ++c) g.c[c] = (g.p[0][c] + g.p[1][c] + g.p[2][c]) / 3.0;
    g.rho = 0.0;
    for (int q = 0; q < 6; ++q) {
        const double e[3] = {g.qp[q][0] - g.c[0], g.qp[q][1] - g.c[1], g.qp[q][2] - g.c[2]};
        g.rho = fmax(g.rho, sqrt(dot3(e, e)));
    }
    geo[t] = g;
    TriGeoF f;
    for (int c = 0; c < 3; ++c) f.c[c] = (g.p[0][c] + g.p[1][c] + g.p[2][c]) / 3.0;
    for (int q = 0; q < 6; ++q)
        for (int c = 0; c < 3; ++c) f.dq[q][c] = (float)(g.qp[q][c] - f.c[c]);
    for (int c = 0; c < 3; ++c) f.n[c] = (float)g.n[c];
    f.area = (float)g.area;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) f.curl[a][c] = (float)g.curl[a][c];
    f.pad = 0.f;
    geof[t] = f;
}

// ------------------------------------------------------------ regular pairs

struct TileArgs {
    const TriGeo *geo;
    const int32_t *tri;
    const int32_t *blk_start;
    const int32_t *blk_nslot;
    const uint8_t *slot_off;    // [nb][SLOT_OFF_LD] first slot-major rank of each slot
    const uint8_t *slot_rank;   // [nb][3 * BT] slot-major rank of each corner
    int32_t nb;
    double k;
    double kim;            // imaginary part of the wavenumber (read by the absorbing instantiation only)
    double2 *scratch;      // [tile - tile_base][SMAX*SMAX][op]
    int64_t tile_base;     // first tile of the strip the scratch holds
};

// tiles of assembly strip s: rows b in [strip_b[s], strip_b[s + 1]), nb - b each
inline int64_t strip_tiles(const MeshData &h, int s)
{
    int64_t n = 0;
    for (int b = h.strip_b[s]; b < h.strip_b[s + 1]; ++b) n += h.nb - b;
    return n;
}

__device__ inline void tile_of(int64_t t, int nb, int &b1, int &b2)
{
    // tiles enumerate (b1, b2), b1 <= b2, row by row; offset(b) = b*nb - b*(b-1)/2
    double B = 2.0 * nb + 1.0;
    int b = (int)floor(0.5 * (B - sqrt(B * B - 8.0 * (double)t)));
    if (b < 0) b = 0;
    if (b > nb - 1) b = nb - 1;
    while (b > 0 && (int64_t)b * nb - (int64_t)b * (b - 1) / 2 > t) --b;
    while (b + 1 < nb && (int64_t)(b + 1) * nb - (int64_t)(b + 1) * b / 2 <= t) ++b;
    b1 = b;
    b2 = b + (int)(t - ((int64_t)b * nb - (int64_t)b * (b - 1) / 2));
}

// Per-slot sums of the 9 entries of every triangle pair of the tile:
// entry (q1, q2) adds the entries (a, b) of every pair whose test triangle
// has slot q1 at corner a and trial triangle slot q2 at corner b.  The
// corners of each block are ranked in slot-major order (the order of the
// block's slot lists, built on the host), so that the corners of a slot
// form a run of consecutive ranks.  The sum separates over the two blocks
// and runs in two stages, each a set of independent items spread over the
// workgroup's threads:
//   1. item (u, q2): P[rank1(u)][q2] = sum over the run of trial slot q2 of
//      the staged row of test corner u = (t1, a);
//   2. item (q1, q2): entry (q1, q2) = sum over the run of test slot q1 of
//      the P rows, written to out[4 * e + op] (tile layout [entry][op]).
// Both stages add in run order, i.e. in slot-list order.  Each item loads
// the first 4 (then, for longer runs, 4 more) entries of its run at once;
// the loads past a run's end fall in the padding or the next run and are
// not added.  Staged entries: st[u * SROW + rank2(t2, b)].
constexpr int SROW = 3 * BT + 1;    // staged row: one entry per trial corner (+1: distinct LDS banks per lane)
constexpr int PROW = SMAX + 1;      // partial-sum row: one entry per trial slot (+1 likewise)
constexpr int ST_LEN = 3 * BT * SROW + 8;
constexpr int P_LEN = (3 * BT + 8) * PROW;
constexpr int SLOT_IT1 = (3 * BT * SMAX + 255) / 256;   // stage-1 items per thread
constexpr int SLOT_IT2 = (SMAX * SMAX + 255) / 256;     // stage-2 items per thread

// sum of x[0 .. m) with x[v] = src[v * stride], in order; m <= LMAX
template <class C2>
__device__ inline C2 run_sum(const C2 *src, int stride, int m)
{
    using R = decltype(C2::x);
    const C2 x0 = src[0], x1 = src[stride], x2 = src[2 * stride], x3 = src[3 * stride];
    R re = x0.x, im = x0.y;
    if (m > 1) { re += x1.x; im += x1.y; }
    if (m > 2) { re += x2.x; im += x2.y; }
    if (m > 3) { re += x3.x; im += x3.y; }
    if (m > 4) {
        const C2 y0 = src[4 * stride], y1 = src[5 * stride], y2 = src[6 * stride], y3 = src[7 * stride];
        re += y0.x; im += y0.y;
        if (m > 5) { re += y1.x; im += y1.y; }
        if (m > 6) { re += y2.x; im += y2.y; }
        if (m > 7) { re += y3.x; im += y3.y; }
        for (int v = 8; v < m; ++v) { re += src[v * stride].x; im += src[v * stride].y; }
    }
    return C2{re, im};
}

// stage 1 (every run has at least one corner, so m >= 1)
template <class C2>
__device__ inline void slot_sums_trial(int tid, int nc1, int ns2, const uint8_t *o2, const uint8_t *r1, const C2 *st,
                                       C2 *P)
{
#pragma unroll
    for (int j = 0; j < SLOT_IT1; ++j) {
        const int it = tid + 256 * j, q2 = it / (3 * BT), u = it - q2 * (3 * BT);
        if (q2 < ns2 && u < nc1) {
            const int s0 = o2[q2];
            P[r1[u] * PROW + q2] = run_sum(st + u * SROW + s0, 1, o2[q2 + 1] - s0);
        }
    }
}

// stage 2
template <class C2>
__device__ inline void slot_sums_test(int tid, int op, int ns1, int ns2, const uint8_t *o1, const C2 *P, C2 *out)
{
#pragma unroll
    for (int j = 0; j < SLOT_IT2; ++j) {
        const int it = tid + 256 * j, q1 = it / SMAX, q2 = it - q1 * SMAX;
        if (q1 < ns1 && q2 < ns2) {
            const int s0 = o1[q1];
            out[4 * it + op] = run_sum(P + s0 * PROW + q2, PROW, o1[q1 + 1] - s0);
        }
    }
}

// sin and cos of a small angle t, |t| <= 1: Taylor polynomials of sin
// through t^17 and of cos through t^18 (the first omitted terms are below
// 1e-17 and 5e-19); the coefficients are 1/n!.
__device__ inline void small_sincos(double t, double &s, double &c)
{
    const double z = t * t;
    double ps = 2.8114572543455206e-15;            //  1/17!
    ps = fma(ps, z, -7.647163731819816e-13);       // -1/15!
    ps = fma(ps, z, 1.6059043836821613e-10);       //  1/13!
    ps = fma(ps, z, -2.505210838544172e-08);       // -1/11!
    ps = fma(ps, z, 2.7557319223985893e-06);       //  1/9!
    ps = fma(ps, z, -0.0001984126984126984);       // -1/7!
    ps = fma(ps, z, 0.008333333333333333);         //  1/5!
    ps = fma(ps, z, -0.16666666666666666);         // -1/3!
    s = fma(t * z, ps, t);
    double pc = -1.5619206968586225e-16;           // -1/18!
    pc = fma(pc, z, 4.779477332387385e-14);        //  1/16!
    pc = fma(pc, z, -1.1470745597729725e-11);      // -1/14!
    pc = fma(pc, z, 2.08767569878681e-09);         //  1/12!
    pc = fma(pc, z, -2.755731922398589e-07);       // -1/10!
    pc = fma(pc, z, 2.48015873015873e-05);         //  1/8!
    pc = fma(pc, z, -0.001388888888888889);        // -1/6!
    pc = fma(pc, z, 0.041666666666666664);         //  1/4!
    pc = fma(pc, z, -0.5);                         // -1/2!
    c = fma(z, pc, 1.0);
}

// 6 x 6 point pairs of one regular triangle pair (x on X, y on Y): the 3 x 3
// element sums of V (kernel G), K (dG/dn_y), T (dG/dn_x) and the scalar sum
// of G, unscaled (times area_X area_Y / (4 pi) later).  K uses that
// (y - x).n_y is the same for every y on the plane of Y, so its factor is
// applied once per test point.  BASE: phase from the per-pair base (see the
// caller).  CK: complex wavenumber k + i kim.
template <bool CK, bool BASE>
__device__ inline void pair_quadrature(const TriGeo &X, const TriGeo &Y, double k, double kim, double (&vr)[9],
                                       double (&vi)[9], double (&kr)[9], double (&ki)[9], double (&tr)[9],
                                       double (&ti)[9], double &sr, double &si)
{
    const double nx0 = X.n[0], nx1 = X.n[1], nx2 = X.n[2];
    const double ny0 = Y.n[0], ny1 = Y.n[1], ny2 = Y.n[2];
    const double ey0 = ny0 * Y.p[0][0] + ny1 * Y.p[0][1] + ny2 * Y.p[0][2];   // n_y . (a vertex of Y)
    double e0r = 1.0, e0i = 0.0, kr0 = 0.0;
    if constexpr (BASE) {
        const double c0 = X.c[0] - Y.c[0], c1 = X.c[1] - Y.c[1], c2 = X.c[2] - Y.c[2];
        kr0 = k * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        phase_sincos(kr0, &e0i, &e0r);
    }
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const double x0 = X.qp[p][0], x1 = X.qp[p][1], x2 = X.qp[p][2];
        const double dkp = ey0 - (ny0 * x0 + ny1 * x1 + ny2 * x2);   // (y - x).n_y
        double hvr[3] = {0, 0, 0}, hvi[3] = {0, 0, 0}, hkr[3] = {0, 0, 0}, hki[3] = {0, 0, 0};
        double htr[3] = {0, 0, 0}, hti[3] = {0, 0, 0};
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double d0 = x0 - Y.qp[q][0], d1 = x1 - Y.qp[q][1], d2 = x2 - Y.qp[q][2];
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double rinv = rsqrt(r2);
            const double r = r2 * rinv;
            const double kr_ = k * r;
            double sn, cs;
            if constexpr (BASE) {
                double sd, cd;
                small_sincos(fma(k, r, -kr0), sd, cd);
                cs = e0r * cd - e0i * sd;
                sn = e0r * sd + e0i * cd;
            } else {
                phase_sincos(kr_, &sn, &cs);
            }
            double gr = cs * rinv, gi = sn * rinv;                 // exp(ikr)/r
            const double rinv2 = rinv * rinv;
            double fr, fi;                                         // exp(ikr)(ikr-1)/r^3
            if constexpr (CK) {
                const double dmp = exp(-kim * r), am = -1.0 - kim * r;
                gr *= dmp; gi *= dmp;
                fr = (gr * am - gi * kr_) * rinv2;
                fi = (gr * kr_ + gi * am) * rinv2;
            } else {
                fr = (-gr - gi * kr_) * rinv2;
                fi = (gr * kr_ - gi) * rinv2;
            }
            const double dt = d0 * nx0 + d1 * nx1 + d2 * nx2;     // (x-y).n_x
            const double gtr = fr * dt, gti = fi * dt;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double W = r6_w(q) * r6_bary(q, b);
                hvr[b] += W * gr; hvi[b] += W * gi;
                hkr[b] += W * fr; hki[b] += W * fi;
                htr[b] += W * gtr; hti[b] += W * gti;
            }
        }
        const double wp = p < 3 ? kW1 : kW2;
        const double ap = p < 3 ? kA1 : kA2;
        const int pc = p < 3 ? p : p - 3;            // corner carrying 1 - 2a
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double W = wp * (a == pc ? 1.0 - 2.0 * ap : ap);
            const double Wk = W * dkp;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                vr[3 * a + b] += W * hvr[b]; vi[3 * a + b] += W * hvi[b];
                kr[3 * a + b] += Wk * hkr[b]; ki[3 * a + b] += Wk * hki[b];
                tr[3 * a + b] += W * htr[b]; ti[3 * a + b] += W * hti[b];
            }
        }
    }
    const double scale = X.area * Y.area * kInv4Pi;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        vr[e] *= scale; vi[e] *= scale; kr[e] *= scale; ki[e] *= scale; tr[e] *= scale; ti[e] *= scale;
    }
    // sum G over the point pairs: the P1 functions sum to one at every point,
    // so the sum over a, b of the V entries is that sum
    sr = 0.0;
    si = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) { sr += vr[e]; si += vi[e]; }
}

// A triangle's table in LDS, padded to an odd number of 16-byte units (23):
// the 16 trial triangles a wave reads at once then fall on distinct LDS banks
// (the unpadded 22 units put triangles t and t + 8 on the same banks).
struct alignas(16) TriGeoLds {
    TriGeo g;
    double pad[2];
};
static_assert(sizeof(TriGeoLds) % 32 == 16, "LDS stride of the triangle tables must be an odd number of 16-byte units");

struct TileArgsF {
    const TriGeoF *geof;
    const int32_t *tri;
    const int32_t *blk_start;
    const int32_t *blk_nslot;
    const uint8_t *slot_off;    // [nb][SLOT_OFF_LD] first slot-major rank of each slot
    const uint8_t *slot_rank;   // [nb][3 * BT] slot-major rank of each corner
    int32_t nb;
    double k;
    double kim;            // imaginary part of the wavenumber (read by the absorbing instantiation only)
    float2 *scratch;       // [tile - tile_base][SMAX*SMAX][op]
    int64_t tile_base;
};

// CK: complex wavenumber k + i kim (an absorbing medium), G = exp(i k r - kim r) / (4 pi r);
// the real-k instantiation is the one the benchmarks time.
template <bool CK>
__global__ __launch_bounds__(256, 2) void regular_tiles_kernel(TileArgs A, int64_t tile0)
{
    __shared__ TriGeoLds gX[BT], gY[BT];
    __shared__ int32_t vX[BT * 3], vY[BT * 3];
    __shared__ uint8_t o1[SLOT_OFF_LD], o2[SLOT_OFF_LD];   // first slot-major rank of each slot
    __shared__ uint8_t r1[3 * BT], r2[3 * BT];             // slot-major rank of each corner
    __shared__ double2 st[ST_LEN];   // the 9 entries of every thread's pair, one operator at a time
    __shared__ double2 P[P_LEN];     // test-corner rank x trial slot partial sums

    const int64_t tile = tile0 + blockIdx.x;
    int b1, b2;
    tile_of(tile, A.nb, b1, b2);
    const int s1 = A.blk_start[b1], n1 = A.blk_start[b1 + 1] - s1;
    const int s2 = A.blk_start[b2], n2 = A.blk_start[b2 + 1] - s2;
    const int ns1 = A.blk_nslot[b1], ns2 = A.blk_nslot[b2];
    const int tid = threadIdx.x;
    {
        const double *src1 = reinterpret_cast<const double *>(A.geo + s1);
        const double *src2 = reinterpret_cast<const double *>(A.geo + s2);
        double *d1 = reinterpret_cast<double *>(gX), *d2 = reinterpret_cast<double *>(gY);
        constexpr int w = sizeof(TriGeo) / sizeof(double), wl = sizeof(TriGeoLds) / sizeof(double);
        for (int q = tid; q < n1 * w; q += 256) d1[(q / w) * wl + q % w] = src1[q];
        for (int q = tid; q < n2 * w; q += 256) d2[(q / w) * wl + q % w] = src2[q];
        if (tid < n1 * 3) vX[tid] = A.tri[3 * s1 + tid];
        if (tid < n2 * 3) vY[tid] = A.tri[3 * s2 + tid];
        if (tid < SLOT_OFF_LD) {
            o1[tid] = A.slot_off[(size_t)b1 * SLOT_OFF_LD + tid];
            o2[tid] = A.slot_off[(size_t)b2 * SLOT_OFF_LD + tid];
        } else if (tid >= 64 && tid < 64 + 3 * BT) {
            r1[tid - 64] = A.slot_rank[(size_t)b1 * 3 * BT + tid - 64];
            r2[tid - 64] = A.slot_rank[(size_t)b2 * 3 * BT + tid - 64];
        }
    }
    __syncthreads();

    const int t1 = tid >> 4, t2 = tid & 15, sbase = 3 * t1 * SROW;
    const bool staged = t1 < n1 && t2 < n2;   // the pair's entries have a place in the staged rows
    const int rk0 = staged ? r2[3 * t2] : 0, rk1 = staged ? r2[3 * t2 + 1] : 0, rk2 = staged ? r2[3 * t2 + 2] : 0;
    bool active = staged;
    if (active) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) active = active && (vX[3 * t1 + a] != vY[3 * t2 + b]);
    }
    double vr[9], vi[9], kr[9], ki[9], tr[9], ti[9], sr = 0.0, si = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) { vr[e] = vi[e] = kr[e] = ki[e] = tr[e] = ti[e] = 0.0; }
    const double k = A.k;
    if (active) {
        const TriGeo &X = gX[t1].g;
        const TriGeo &Y = gY[t2].g;
        // Phase by a per-pair base when k (rho_X + rho_Y) <= 1: with r0 the
        // centroid distance, |k (r - r0)| <= 1 for every point pair, so
        // exp(i k r) = exp(i k r0) exp(i k (r - r0)) takes one reduced
        // sin/cos per pair and short polynomials per point pair.
        if (!CK && k * (X.rho + Y.rho) <= 1.0)
            pair_quadrature<CK, true>(X, Y, k, A.kim, vr, vi, kr, ki, tr, ti, sr, si);
        else
            pair_quadrature<CK, false>(X, Y, k, A.kim, vr, vi, kr, ki, tr, ti, sr, si);
    }

    // ---- per-slot reduction through LDS, one operator at a time (two barriers per operator)
    double2 *out = A.scratch + (tile - A.tile_base) * (4 * SMAX * SMAX);
#pragma unroll 1
    for (int op = 0; op < 4; ++op) {
        if (op == 3 && active) {
            const TriGeo &X = gX[t1].g;
            const TriGeo &Y = gY[t2].g;
            const double nn = X.n[0] * Y.n[0] + X.n[1] * Y.n[1] + X.n[2] * Y.n[2];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double cc = X.curl[a][0] * Y.curl[b][0] + X.curl[a][1] * Y.curl[b][1] + X.curl[a][2] * Y.curl[b][2];
                    if constexpr (CK) {   // complex k^2
                        const double k2r = k * k - A.kim * A.kim, k2i = 2.0 * k * A.kim;
                        const double v_r = vr[3 * a + b], v_i = vi[3 * a + b];
                        st[sbase + a * SROW + (b == 0 ? rk0 : (b == 1 ? rk1 : rk2))] = make_double2(cc * sr - nn * (k2r * v_r - k2i * v_i),
                                                               cc * si - nn * (k2r * v_i + k2i * v_r));
                    } else {
                        st[sbase + a * SROW + (b == 0 ? rk0 : (b == 1 ? rk1 : rk2))] = make_double2(cc * sr - k * k * nn * vr[3 * a + b],
                                                               cc * si - k * k * nn * vi[3 * a + b]);
                    }
                }
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                double re = op == 0 ? vr[e] : (op == 1 ? kr[e] : (op == 2 ? tr[e] : 0.0));
                double im = op == 0 ? vi[e] : (op == 1 ? ki[e] : (op == 2 ? ti[e] : 0.0));
                if (staged)
                    st[sbase + (e / 3) * SROW + (e % 3 == 0 ? rk0 : (e % 3 == 1 ? rk1 : rk2))] =
                        active ? make_double2(re, im) : make_double2(0.0, 0.0);
            }
        }
        __syncthreads();   // st holds this operator; the previous operator's stage 2 is done with P
        slot_sums_trial(tid, 3 * n1, ns2, o2, r1, st, P);
        __syncthreads();   // P complete; st free for the next operator
        slot_sums_test(tid, op, ns1, ns2, o1, P, out);
    }
}

// Mixed-precision form of the regular-pair tile (FP32 arithmetic, complex64
// tiles).  The phase k|x - y| is split per triangle pair: with d0 the FP64
// centroid difference and r0 = |d0|, exp(i k r) = exp(i k r0) exp(i k D)
// where exp(i k r0) is evaluated once in FP64 and D = r - r0 =
// (2 d0.e + |e|^2) / (r + r0), e = (x - c_x) - (y - c_y), is small and
// accurate in FP32; FP32 alone would lose about k r * 6e-8 of phase.
// CK as in the FP64 kernel: the damping exp(-kim r) splits like the phase,
// exp(-kim r0) in FP64 per pair and exp(-kim D) in FP32 per point.
template <bool CK>
__global__ __launch_bounds__(256, 3) void regular_tiles_f32_kernel(TileArgsF A, int64_t tile0)
{
    __shared__ TriGeoF gX[BT], gY[BT];
    __shared__ int32_t vX[BT * 3], vY[BT * 3];
    __shared__ uint8_t o1[SLOT_OFF_LD], o2[SLOT_OFF_LD];   // first slot-major rank of each slot
    __shared__ uint8_t r1[3 * BT], r2[3 * BT];             // slot-major rank of each corner
    __shared__ float2 st[ST_LEN];
    __shared__ float2 P[P_LEN];

    const int64_t tile = tile0 + blockIdx.x;
    int b1, b2;
    tile_of(tile, A.nb, b1, b2);
    const int s1 = A.blk_start[b1], n1 = A.blk_start[b1 + 1] - s1;
    const int s2 = A.blk_start[b2], n2 = A.blk_start[b2 + 1] - s2;
    const int ns1 = A.blk_nslot[b1], ns2 = A.blk_nslot[b2];
    const int tid = threadIdx.x;
    {
        const double *src1 = reinterpret_cast<const double *>(A.geof + s1);
        const double *src2 = reinterpret_cast<const double *>(A.geof + s2);
        double *d1 = reinterpret_cast<double *>(gX), *d2 = reinterpret_cast<double *>(gY);
        const int w = sizeof(TriGeoF) / sizeof(double);
        for (int q = tid; q < n1 * w; q += 256) d1[q] = src1[q];
        for (int q = tid; q < n2 * w; q += 256) d2[q] = src2[q];
        if (tid < n1 * 3) vX[tid] = A.tri[3 * s1 + tid];
        if (tid < n2 * 3) vY[tid] = A.tri[3 * s2 + tid];
        if (tid < SLOT_OFF_LD) {
            o1[tid] = A.slot_off[(size_t)b1 * SLOT_OFF_LD + tid];
            o2[tid] = A.slot_off[(size_t)b2 * SLOT_OFF_LD + tid];
        } else if (tid >= 64 && tid < 64 + 3 * BT) {
            r1[tid - 64] = A.slot_rank[(size_t)b1 * 3 * BT + tid - 64];
            r2[tid - 64] = A.slot_rank[(size_t)b2 * 3 * BT + tid - 64];
        }
    }
    __syncthreads();

    const int t1 = tid >> 4, t2 = tid & 15, sbase = 3 * t1 * SROW;
    const bool staged = t1 < n1 && t2 < n2;   // the pair's entries have a place in the staged rows
    const int rk0 = staged ? r2[3 * t2] : 0, rk1 = staged ? r2[3 * t2 + 1] : 0, rk2 = staged ? r2[3 * t2 + 2] : 0;
    bool active = staged;
    if (active) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) active = active && (vX[3 * t1 + a] != vY[3 * t2 + b]);
    }
    float vr[9], vi[9], kr[9], ki[9], tr[9], ti[9], sr = 0.f, si = 0.f;
#pragma unroll
    for (int e = 0; e < 9; ++e) { vr[e] = vi[e] = kr[e] = ki[e] = tr[e] = ti[e] = 0.f; }
    const float kf = (float)A.k;
    if (active) {
        const TriGeoF &X = gX[t1];
        const TriGeoF &Y = gY[t2];
        const double d00 = X.c[0] - Y.c[0], d01 = X.c[1] - Y.c[1], d02 = X.c[2] - Y.c[2];
        const double r0 = sqrt(d00 * d00 + d01 * d01 + d02 * d02);
        double s0, c0;
        phase_sincos(A.k * r0, &s0, &c0);
        if constexpr (CK) {
            const double dm0 = exp(-A.kim * r0);
            s0 *= dm0;
            c0 *= dm0;
        }
        const float e0r = (float)c0, e0i = (float)s0;
        const float f00 = (float)d00, f01 = (float)d01, f02 = (float)d02, r0f = (float)r0;
        const float nx0 = X.n[0], nx1 = X.n[1], nx2 = X.n[2];
        const float ny0 = Y.n[0], ny1 = Y.n[1], ny2 = Y.n[2];
#pragma unroll 1
        for (int p = 0; p < 6; ++p) {
            const float x0 = X.dq[p][0], x1 = X.dq[p][1], x2 = X.dq[p][2];
            float hvr[3] = {0, 0, 0}, hvi[3] = {0, 0, 0}, hkr[3] = {0, 0, 0}, hki[3] = {0, 0, 0};
            float htr[3] = {0, 0, 0}, hti[3] = {0, 0, 0};
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const float q0 = x0 - Y.dq[q][0], q1 = x1 - Y.dq[q][1], q2 = x2 - Y.dq[q][2];   // e
                const float d0 = f00 + q0, d1 = f01 + q1, d2 = f02 + q2;                         // x - y
                const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const float rinv = __frsqrt_rn(r2);
                const float r = r2 * rinv;
                const float num = 2.f * (f00 * q0 + f01 * q1 + f02 * q2) + (q0 * q0 + q1 * q1 + q2 * q2);
                const float dr = num / (r + r0f);
                float sd, cd;
                sincosf(kf * dr, &sd, &cd);
                float er = e0r * cd - e0i * sd, ei = e0r * sd + e0i * cd;   // exp(ikr)
                const float kr_ = kf * r, rinv2 = rinv * rinv;
                float fr, fi;
                if constexpr (CK) {
                    const float dd = expf(-(float)A.kim * dr), am = -1.f - (float)A.kim * r;
                    er *= dd;
                    ei *= dd;
                    const float gr = er * rinv, gi = ei * rinv;
                    fr = (gr * am - gi * kr_) * rinv2;
                    fi = (gr * kr_ + gi * am) * rinv2;
                } else {
                    const float gr = er * rinv, gi = ei * rinv;
                    fr = (-gr - gi * kr_) * rinv2;
                    fi = (gr * kr_ - gi) * rinv2;
                }
                const float gr = er * rinv, gi = ei * rinv;
                const float dk = -(d0 * ny0 + d1 * ny1 + d2 * ny2);
                const float dt = d0 * nx0 + d1 * nx1 + d2 * nx2;
                const float gkr = fr * dk, gki = fi * dk, gtr = fr * dt, gti = fi * dt;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const float W = (float)(r6_w(q) * r6_bary(q, b));
                    hvr[b] += W * gr; hvi[b] += W * gi;
                    hkr[b] += W * gkr; hki[b] += W * gki;
                    htr[b] += W * gtr; hti[b] += W * gti;
                }
            }
            const float wp = p < 3 ? (float)kW1 : (float)kW2;
            const float ap = p < 3 ? (float)kA1 : (float)kA2;
            const float am = p < 3 ? (float)(1.0 - 2.0 * kA1) : (float)(1.0 - 2.0 * kA2);
            const int pc = p < 3 ? p : p - 3;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float W = wp * (a == pc ? am : ap);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    vr[3 * a + b] += W * hvr[b]; vi[3 * a + b] += W * hvi[b];
                    kr[3 * a + b] += W * hkr[b]; ki[3 * a + b] += W * hki[b];
                    tr[3 * a + b] += W * htr[b]; ti[3 * a + b] += W * hti[b];
                }
            }
        }
        const float scale = X.area * Y.area * (float)kInv4Pi;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            vr[e] *= scale; vi[e] *= scale; kr[e] *= scale; ki[e] *= scale; tr[e] *= scale; ti[e] *= scale;
        }
        // the sum of G over the point pairs is the sum of the V entries (the P1 functions sum to one)
#pragma unroll
        for (int e = 0; e < 9; ++e) { sr += vr[e]; si += vi[e]; }
    }
    float2 *out = A.scratch + (tile - A.tile_base) * (4 * SMAX * SMAX);
#pragma unroll 1
    for (int op = 0; op < 4; ++op) {
        if (op == 3 && active) {
            const TriGeoF &X = gX[t1];
            const TriGeoF &Y = gY[t2];
            const float nn = X.n[0] * Y.n[0] + X.n[1] * Y.n[1] + X.n[2] * Y.n[2];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const float cc = X.curl[a][0] * Y.curl[b][0] + X.curl[a][1] * Y.curl[b][1] + X.curl[a][2] * Y.curl[b][2];
                    if constexpr (CK) {   // complex k^2
                        const float k2r = (float)(A.k * A.k - A.kim * A.kim), k2i = (float)(2.0 * A.k * A.kim);
                        const float v_r = vr[3 * a + b], v_i = vi[3 * a + b];
                        st[sbase + a * SROW + (b == 0 ? rk0 : (b == 1 ? rk1 : rk2))] = make_float2(cc * sr - nn * (k2r * v_r - k2i * v_i),
                                                              cc * si - nn * (k2r * v_i + k2i * v_r));
                    } else {
                        st[sbase + a * SROW + (b == 0 ? rk0 : (b == 1 ? rk1 : rk2))] = make_float2(cc * sr - kf * kf * nn * vr[3 * a + b],
                                                              cc * si - kf * kf * nn * vi[3 * a + b]);
                    }
                }
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                float re = op == 0 ? vr[e] : (op == 1 ? kr[e] : (op == 2 ? tr[e] : 0.f));
                float im = op == 0 ? vi[e] : (op == 1 ? ki[e] : (op == 2 ? ti[e] : 0.f));
                if (staged)
                    st[sbase + (e / 3) * SROW + (e % 3 == 0 ? rk0 : (e % 3 == 1 ? rk1 : rk2))] =
                        active ? make_float2(re, im) : make_float2(0.f, 0.f);
            }
        }
        __syncthreads();   // st holds this operator; the previous operator's stage 2 is done with P
        slot_sums_trial(tid, 3 * n1, ns2, o2, r1, st, P);
        __syncthreads();   // P complete; st free for the next operator
        slot_sums_test(tid, op, ns1, ns2, o1, P, out);
    }
}

// The contributions to dense entry (i, j) of the tiles of one strip (tile
// rows [b0, b1), tile t at (t - tile_base) in the scratch): every tile
// (min(bi, bj), max(bi, bj)) of the blocks bi, bj containing i and j whose
// first block lies in the strip, in membership order (memberships of i,
// then of j).  The same terms with the roles of i and j exchanged make up
// entry (j, i): V and D are the same numbers, K and T exchange (the tile of
// (bj, bi) read from the other side).  So one sum gives both entries, and a
// strip reads each tile entry once.  The strip of the smallest membership
// of i and j is the first to reach (i, j) and writes it; later strips add
// their share (strips run in order on one stream).
//
// Entries a strip reaches have i or j in its row list R (the vertices with a
// membership in its blocks) and both at or after lo (the first vertex with a
// membership at or after b0).  Two launches cover them as unordered pairs:
//   RR: i = R[a], j = R[b] for a <= b (16 x 16 chunks of R; workgroups whose
//       row chunk comes after their column chunk return at once);
//   RO: i in R, j in [lo, nv) outside R (16 rows of R x 16 columns).
// A workgroup of 256 threads holds a 16 x 16 block: it writes (i, j) along
// rows (consecutive j), stages the sums in LDS and writes (j, i) along rows
// j (consecutive i of R).
template <class C2>
__device__ inline bool strip_sum(int i, int j, int nb, int b0, int b1, int64_t tile_base, const int32_t *memb_ptr,
                                 const int32_t *memb, const C2 *scratch, C2 (&acc)[4], bool &first)
{
    using R = decltype(C2::x);
    const int pi0 = memb_ptr[i], pi1 = memb_ptr[i + 1];
    const int pj0 = memb_ptr[j], pj1 = memb_ptr[j + 1];
    R vx = 0, vy = 0, kx = 0, ky = 0, tx = 0, ty = 0, dx = 0, dy = 0;
    bool any = false;
    for (int p = pi0; p < pi1; ++p) {
        const int mi = memb[p], bi = mi >> 8, si = mi & 255;
        for (int q = pj0; q < pj1; ++q) {
            const int mj = memb[q], bj = mj >> 8, sj = mj & 255;
            const int lo_b = bi < bj ? bi : bj, hi_b = bi < bj ? bj : bi;
            if (lo_b < b0 || lo_b >= b1) continue;
            any = true;
            const int64_t tile = (int64_t)lo_b * nb - (int64_t)lo_b * (lo_b - 1) / 2 + (hi_b - lo_b) - tile_base;
            const C2 *tl = scratch + tile * (4 * SMAX * SMAX);
            if (bi <= bj) {
                const int e = si * SMAX + sj;
                const C2 a0 = tl[4 * e], a1 = tl[4 * e + 1], a2 = tl[4 * e + 2], a3 = tl[4 * e + 3];
                vx += a0.x; vy += a0.y; kx += a1.x; ky += a1.y;
                tx += a2.x; ty += a2.y; dx += a3.x; dy += a3.y;
            } else {
                // tile of (bj, bi): test side is j; K and T swap under transposition
                const int e = sj * SMAX + si;
                const C2 a0 = tl[4 * e], a1 = tl[4 * e + 1], a2 = tl[4 * e + 2], a3 = tl[4 * e + 3];
                vx += a0.x; vy += a0.y; kx += a2.x; ky += a2.y;
                tx += a1.x; ty += a1.y; dx += a3.x; dy += a3.y;
            }
        }
    }
    acc[0] = C2{vx, vy};
    acc[1] = C2{kx, ky};
    acc[2] = C2{tx, ty};
    acc[3] = C2{dx, dy};
    first = min(memb[pi0] >> 8, memb[pj0] >> 8) >= b0;   // lists ascend by block
    return any;
}

// (i, j) of the four operators: written by the first strip to reach it, added to by later ones
template <class C2>
__device__ inline void strip_put(C2 *const (&op)[4], int64_t o, const C2 (&v)[4], bool first)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (first) {
            op[k][o] = v[k];
        } else {
            const C2 x = op[k][o];
            op[k][o] = C2{x.x + v[k].x, x.y + v[k].y};
        }
    }
}

template <class C2, bool RR>
__global__ __launch_bounds__(256) void gather_strip_kernel(int nv, int nb, int b0, int b1, int64_t tile_base, int lo,
                                                           const int32_t *__restrict__ rows, int nrows,
                                                           const int32_t *__restrict__ memb_ptr,
                                                           const int32_t *__restrict__ memb,
                                                           const C2 *__restrict__ scratch, C2 *__restrict__ V,
                                                           C2 *__restrict__ K, C2 *__restrict__ T, C2 *__restrict__ D)
{
    __shared__ C2 sv[4][16][17];
    __shared__ uint8_t sflag[16][17];   // bit 0: a contribution, bit 1: first strip to reach the entry
    if (RR && blockIdx.x > blockIdx.y) return;
    C2 *const op[4] = {V, K, T, D};
    const int64_t ld = op_ld(nv);
    const int tid = threadIdx.x, ra = tid >> 4, cb = tid & 15;
    // (i, j): i = R[16 blockIdx.x + ra], j = R[16 blockIdx.y + cb] (RR) or lo + 16 blockIdx.y + cb (RO)
    const int ai = 16 * (int)blockIdx.x + ra, aj = 16 * (int)blockIdx.y + cb;
    bool ok = ai < nrows && (RR ? (aj < nrows && (blockIdx.x < blockIdx.y || ra <= cb)) : lo + aj < nv);
    int i = 0, j = 0;
    if (ok) {
        i = rows[ai];
        j = RR ? rows[aj] : lo + aj;
        if (!RR)   // columns in R are the RR launch's
            for (int p = memb_ptr[j]; p < memb_ptr[j + 1] && ok; ++p) {
                const int bj = memb[p] >> 8;
                ok = bj < b0 || bj >= b1;
            }
    }
    C2 acc[4];
    bool first = false, any = false;
    if (ok) {
        any = strip_sum(i, j, nb, b0, b1, tile_base, memb_ptr, memb, scratch, acc, first);
        if (first || any) strip_put(op, (int64_t)i * ld + j, acc, first);
    }
    // (j, i) from the same sums, through LDS: V, D as they are, K and T exchanged
#pragma unroll
    for (int k = 0; k < 4; ++k) sv[k][ra][cb] = acc[k];
    sflag[ra][cb] = (uint8_t)((ok && any ? 1 : 0) | (ok && first && i != j ? 2 : 0) | (ok && i != j ? 4 : 0));
    __syncthreads();
    const int rb = tid >> 4, ca = tid & 15;   // row j of column block rb, column i of row block ca
    const int f = sflag[ca][rb];
    if (f & 4) {
        const int aj2 = 16 * (int)blockIdx.y + rb, ai2 = 16 * (int)blockIdx.x + ca;
        const int jj = RR ? rows[aj2] : lo + aj2, ii = rows[ai2];
        if (f & 3) {
            const C2 w[4] = {sv[0][ca][rb], sv[2][ca][rb], sv[1][ca][rb], sv[3][ca][rb]};
            strip_put(op, (int64_t)jj * ld + ii, w, (f & 2) != 0);
        }
    }
}

// the padding columns [nv, op_ld(nv)) of every row of the four operators: zero
template <class C2>
__global__ void zero_padding_kernel(int nv, C2 *__restrict__ V, C2 *__restrict__ K, C2 *__restrict__ T, C2 *__restrict__ D)
{
    const int pad = (int)(op_ld(nv) - nv);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pad == 0 || t >= (int64_t)nv * pad) return;
    const int64_t o = (t / pad) * op_ld(nv) + nv + t % pad;
    V[o] = C2{0, 0};
    K[o] = C2{0, 0};
    T[o] = C2{0, 0};
    D[o] = C2{0, 0};
}

// ----------------------------------------------------------- singular pairs

struct GLTab {
    double x[NG_MAX], w[NG_MAX];
};

// Sauter-Schwab regions on the reference triangle {0 <= s2 <= s1 <= 1}.
__device__ inline void ss_map(int kind, int reg, double xi, double e1, double e2, double e3, double &x0, double &x1,
                              double &y0, double &y1, double &jac)
{
    const double xi3 = xi * xi * xi;
    if (kind == 3) {
        jac = xi3 * e1 * e1 * e2;
        const double a = xi, b = xi * (1.0 - e1 + e1 * e2), c = xi * (1.0 - e1 * e2 * e3), d = xi * (1.0 - e1);
        const double f = xi * e1 * (1.0 - e2 + e2 * e3), g = xi * (1.0 - e1 * e2), h = xi * e1 * (1.0 - e2);
        const double m = xi * e1 * (1.0 - e2 * e3);
        switch (reg) {
        case 0: x0 = a; x1 = b; y0 = c; y1 = d; break;
        case 1: x0 = c; x1 = d; y0 = a; y1 = b; break;
        case 2: x0 = a; x1 = f; y0 = g; y1 = h; break;
        case 3: x0 = g; x1 = h; y0 = a; y1 = f; break;
        case 4: x0 = c; x1 = m; y0 = a; y1 = h; break;
        default: x0 = a; x1 = h; y0 = c; y1 = m; break;
        }
    } else if (kind == 2) {
        jac = xi3 * e1 * e1 * (reg == 0 ? 1.0 : e2);
        switch (reg) {
        case 0: x0 = xi; x1 = xi * e1 * e3; y0 = xi * (1.0 - e1 * e2); y1 = xi * e1 * (1.0 - e2); break;
        case 1: x0 = xi; x1 = xi * e1; y0 = xi * (1.0 - e1 * e2 * e3); y1 = xi * e1 * e2 * (1.0 - e3); break;
        case 2: x0 = xi * (1.0 - e1 * e2); x1 = xi * e1 * (1.0 - e2); y0 = xi; y1 = xi * e1 * e2 * e3; break;
        case 3: x0 = xi * (1.0 - e1 * e2 * e3); x1 = xi * e1 * e2 * (1.0 - e3); y0 = xi; y1 = xi * e1; break;
        default: x0 = xi * (1.0 - e1 * e2 * e3); x1 = xi * e1 * (1.0 - e2 * e3); y0 = xi; y1 = xi * e1 * e2; break;
        }
    } else {
        jac = xi3 * e2;
        if (reg == 0) { x0 = xi; x1 = xi * e1; y0 = xi * e2; y1 = xi * e2 * e3; }
        else { x0 = xi * e2; x1 = xi * e2 * e3; y0 = xi; y1 = xi * e1; }
    }
}

template <bool CK>
__global__ __launch_bounds__(256, 2) void singular_pairs_kernel(const TriGeo *__restrict__ geo,
                                                             const SingPair *__restrict__ pairs, int npairs, int ng,
                                                             GLTab gl, double k, double kim, double2 *__restrict__ out)
{
    const int grp = threadIdx.x >> 4, lane = threadIdx.x & 15;
    const int pid = blockIdx.x * 16 + grp;
    if (pid >= npairs) return;
    const SingPair sp = pairs[pid];
    const TriGeo &X = geo[sp.tau];
    const TriGeo &Y = geo[sp.sig];
    int px[3], py[3];
    for (int r = 0; r < 3; ++r) { px[r] = (sp.perm >> (2 * r)) & 3; py[r] = (sp.perm >> (6 + 2 * r)) & 3; }
    double Qx[3][3], Qy[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) { Qx[r][c] = X.p[px[r]][c]; Qy[r][c] = Y.p[py[r]][c]; }
    double ax[2][3], ay[2][3];
    for (int c = 0; c < 3; ++c) {
        ax[0][c] = Qx[1][c] - Qx[0][c]; ax[1][c] = Qx[2][c] - Qx[1][c];
        ay[0][c] = Qy[1][c] - Qy[0][c]; ay[1][c] = Qy[2][c] - Qy[1][c];
    }
    const double nx[3] = {X.n[0], X.n[1], X.n[2]}, ny[3] = {Y.n[0], Y.n[1], Y.n[2]};
    const int kind = sp.kind;
    const int nreg = kind == 3 ? 6 : (kind == 2 ? 5 : 2);
    double vr[9], vi[9], kr[9], ki[9], tr[9], ti[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) { vr[e] = vi[e] = kr[e] = ki[e] = tr[e] = ti[e] = 0.0; }
    const int ng2 = ng * ng;
    for (int inner = lane; inner < ng2; inner += 16) {
        const int i2 = inner / ng, i3 = inner - i2 * ng;
        const double e2 = gl.x[i2], e3 = gl.x[i3], w23 = gl.w[i2] * gl.w[i3];
        for (int reg = 0; reg < nreg; ++reg)
            for (int i0 = 0; i0 < ng; ++i0)
                for (int i1 = 0; i1 < ng; ++i1) {
                    const double xi = gl.x[i0], e1 = gl.x[i1];
                    double xs0, xs1, ys0, ys1, jac;
                    ss_map(kind, reg, xi, e1, e2, e3, xs0, xs1, ys0, ys1, jac);
                    const double wt = gl.w[i0] * gl.w[i1] * w23 * jac;
                    double d[3];
                    for (int c = 0; c < 3; ++c)
                        d[c] = (Qx[0][c] + xs0 * ax[0][c] + xs1 * ax[1][c]) - (Qy[0][c] + ys0 * ay[0][c] + ys1 * ay[1][c]);
                    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    const double rinv = rsqrt(r2);
                    const double r = r2 * rinv, kr_ = k * r;
                    double sn, cs;
                    phase_sincos(kr_, &sn, &cs);
                    double gr = cs * rinv * wt, gi = sn * rinv * wt;
                    const double rinv2 = rinv * rinv;
                    double fr, fi;
                    if constexpr (CK) {
                        const double dmp = exp(-kim * r), am = -1.0 - kim * r;
                        gr *= dmp; gi *= dmp;
                        fr = (gr * am - gi * kr_) * rinv2;
                        fi = (gr * kr_ + gi * am) * rinv2;
                    } else {
                        fr = (-gr - gi * kr_) * rinv2;
                        fi = (gr * kr_ - gi) * rinv2;
                    }
                    const double dk = -(d[0] * ny[0] + d[1] * ny[1] + d[2] * ny[2]);
                    const double dt = d[0] * nx[0] + d[1] * nx[1] + d[2] * nx[2];
                    const double gkr = fr * dk, gki = fi * dk, gtr = fr * dt, gti = fi * dt;
                    const double phx[3] = {1.0 - xs0, xs0 - xs1, xs1}, phy[3] = {1.0 - ys0, ys0 - ys1, ys1};
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            const double ph = phx[a] * phy[b];
                            vr[3 * a + b] += ph * gr; vi[3 * a + b] += ph * gi;
                            kr[3 * a + b] += ph * gkr; ki[3 * a + b] += ph * gki;
                            tr[3 * a + b] += ph * gtr; ti[3 * a + b] += ph * gti;
                        }
                }
    }
    // the sum of G over the points: the P1 functions of each side sum to one
    // at every point, so it is the sum of the nine V entries
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) { sr += vr[e]; si += vi[e]; }
    // reduce over the 16 lanes of the group
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            vr[e] += __shfl_xor(vr[e], off, 16); vi[e] += __shfl_xor(vi[e], off, 16);
            kr[e] += __shfl_xor(kr[e], off, 16); ki[e] += __shfl_xor(ki[e], off, 16);
            tr[e] += __shfl_xor(tr[e], off, 16); ti[e] += __shfl_xor(ti[e], off, 16);
        }
        sr += __shfl_xor(sr, off, 16);
        si += __shfl_xor(si, off, 16);
    }
    if (lane != 0) return;
    const double scale = 4.0 * X.area * Y.area * kInv4Pi;
    const double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
    double2 *o = out + (int64_t)pid * 36;
    for (int ra = 0; ra < 3; ++ra)
        for (int rb = 0; rb < 3; ++rb) {
            const int a = px[ra], b = py[rb];        // own corners
            const int e = 3 * a + b, re = 3 * ra + rb;
            const double cc = X.curl[a][0] * Y.curl[b][0] + X.curl[a][1] * Y.curl[b][1] + X.curl[a][2] * Y.curl[b][2];
            const double Vr = vr[re] * scale, Vi = vi[re] * scale;
            o[e] = make_double2(Vr, Vi);
            o[9 + e] = make_double2(kr[re] * scale, ki[re] * scale);
            o[18 + e] = make_double2(tr[re] * scale, ti[re] * scale);
            if constexpr (CK) {
                const double k2r = k * k - kim * kim, k2i = 2.0 * k * kim;
                o[27 + e] = make_double2(cc * sr * scale - nn * (k2r * Vr - k2i * Vi),
                                         cc * si * scale - nn * (k2r * Vi + k2i * Vr));
            } else {
                o[27 + e] = make_double2(cc * sr * scale - k * k * nn * Vr, cc * si * scale - k * k * nn * Vi);
            }
        }
}

// add the singular contributions (FP64) to their dense entries (fixed order)
template <class C2>
__global__ void near_scatter_kernel(int nv, int nnear, const int32_t *__restrict__ ni, const int32_t *__restrict__ nj,
                                    const int32_t *__restrict__ nptr, const int32_t *__restrict__ nsrc,
                                    const double2 *__restrict__ contrib, C2 *__restrict__ V, C2 *__restrict__ K,
                                    C2 *__restrict__ T, C2 *__restrict__ D)
{
    using R = decltype(C2::x);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnear) return;
    double2 s[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    for (int q = nptr[e]; q < nptr[e + 1]; ++q) {
        const int src = nsrc[q], pid = src / 9, ab = src - 9 * pid;
        const double2 *c = contrib + (int64_t)pid * 36 + ab;
        for (int op = 0; op < 4; ++op) { s[op].x += c[9 * op].x; s[op].y += c[9 * op].y; }
    }
    const int64_t o = (int64_t)ni[e] * op_ld(nv) + nj[e];
    C2 *dst[4] = {V, K, T, D};
    for (int op = 0; op < 4; ++op) {
        const C2 x = dst[op][o];
        dst[op][o] = C2{(R)((double)x.x + s[op].x), (R)((double)x.y + s[op].y)};
    }
}

// ------------------------------------------------------------- launchers

bem_status launch_geometry(const bem_mesh *m, hipStream_t st)
{
    const int nt = (int)m->h.nt;
    hipLaunchKernelGGL(geometry_kernel, dim3((nt + 255) / 256), dim3(256), 0, st, m->d.xyz.as<double>(),
                       m->d.tri.as<int32_t>(), nt, m->d.geo.as<TriGeo>(), m->d.geof.as<TriGeoF>());
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

// tile scratch of one mesh: two strips' tiles (or one when the mesh has a
// single strip); entry size 16 B (complex128) or 8 B (complex64)
size_t tile_scratch_bytes(const bem_mesh *m, size_t entry_bytes)
{
    const MeshData &h = m->h;
    const int ns = (int)h.strip_b.size() - 1;
    int64_t most = 0;
    for (int s = 0; s < ns; ++s) most = std::max(most, strip_tiles(h, s));
    return (size_t)(ns > 1 ? 2 : 1) * (size_t)most * 4 * SMAX * SMAX * entry_bytes;
}

// Regular-pair assembly strip by strip: the tiles of strip s into half s % 2
// of the scratch on the main stream; its gather into the operators on the
// context's gather stream, which overlaps the next strip's tiles.  The main
// stream reuses a half once the gather of two strips before is done, and
// waits for the last gather before returning.
bem_status launch_regular(const bem_mesh *m, double k, double kim, bool fp32, void *scratch, void *ops[4], hipStream_t st)
{
    bem_ctx *ctx = m->ctx;
    const MeshData &h = m->h;
    const int64_t nb = h.nb;
    const int nv = (int)h.nv;
    const int ns = (int)h.strip_b.size() - 1;
    const size_t eb = fp32 ? sizeof(float2) : sizeof(double2);
    int64_t most = 0;
    for (int s = 0; s < ns; ++s) most = std::max(most, strip_tiles(h, s));
    const size_t half = (size_t)most * 4 * SMAX * SMAX * eb;
    if (!ctx->gather) BEM_HIP(hipStreamCreateWithFlags(&ctx->gather, hipStreamNonBlocking));
    hipStream_t gs = ctx->gather;
    // events (kept by the context, so that no event is destroyed while a wait on it is queued): [0] main-stream
    // work before the assembly, [1 + b] tiles of half b done, [3 + b] its gather done
    hipEvent_t *ev = ctx->strip_ev;
    for (int q = 0; q < 5; ++q)
        if (!ev[q]) BEM_HIP(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming));
    BEM_HIP(hipEventRecord(ev[0], st));
    BEM_HIP(hipStreamWaitEvent(gs, ev[0], 0));   // the operator blocks may have served earlier main-stream work
    if ((int64_t)op_ld(nv) > nv) {
        const int64_t npad = (int64_t)nv * (op_ld(nv) - nv);
        const dim3 gz((unsigned)((npad + 255) / 256));
        if (!fp32)
            hipLaunchKernelGGL(zero_padding_kernel<double2>, gz, dim3(256), 0, gs, nv, static_cast<double2 *>(ops[0]),
                               static_cast<double2 *>(ops[1]), static_cast<double2 *>(ops[2]), static_cast<double2 *>(ops[3]));
        else
            hipLaunchKernelGGL(zero_padding_kernel<float2>, gz, dim3(256), 0, gs, nv, static_cast<float2 *>(ops[0]),
                               static_cast<float2 *>(ops[1]), static_cast<float2 *>(ops[2]), static_cast<float2 *>(ops[3]));
        BEM_HIP(hipGetLastError());
    }
    for (int s = 0; s < ns; ++s) {
        const int b0 = h.strip_b[s], b1 = h.strip_b[s + 1], hb = s % 2;
        const int64_t t0 = b0 * nb - (int64_t)b0 * (b0 - 1) / 2, n = strip_tiles(h, s);
        char *buf = static_cast<char *>(scratch) + hb * half;
        if (s >= 2) BEM_HIP(hipStreamWaitEvent(st, ev[3 + hb], 0));
        {
            KTimer kt(ctx, K_REGULAR);
            if (!fp32) {
                TileArgs A;
                A.geo = m->d.geo.as<TriGeo>();
                A.tri = m->d.tri.as<int32_t>();
                A.blk_start = m->d.blk_start.as<int32_t>();
                A.blk_nslot = m->d.blk_nslot.as<int32_t>();
                A.slot_off = m->d.slot_off.as<uint8_t>();
                A.slot_rank = m->d.slot_rank.as<uint8_t>();
                A.nb = (int32_t)nb;
                A.k = k;
                A.kim = kim;
                A.scratch = reinterpret_cast<double2 *>(buf);
                A.tile_base = t0;
                if (kim != 0.0)
                    launch_k(kt, regular_tiles_kernel<true>, dim3((unsigned)n), dim3(256), 0, st, A, t0);
                else
                    launch_k(kt, regular_tiles_kernel<false>, dim3((unsigned)n), dim3(256), 0, st, A, t0);
            } else {
                TileArgsF A;
                A.geof = m->d.geof.as<TriGeoF>();
                A.tri = m->d.tri.as<int32_t>();
                A.blk_start = m->d.blk_start.as<int32_t>();
                A.blk_nslot = m->d.blk_nslot.as<int32_t>();
                A.slot_off = m->d.slot_off.as<uint8_t>();
                A.slot_rank = m->d.slot_rank.as<uint8_t>();
                A.nb = (int32_t)nb;
                A.k = k;
                A.kim = kim;
                A.scratch = reinterpret_cast<float2 *>(buf);
                A.tile_base = t0;
                if (kim != 0.0)
                    launch_k(kt, regular_tiles_f32_kernel<true>, dim3((unsigned)n), dim3(256), 0, st, A, t0);
                else
                    launch_k(kt, regular_tiles_f32_kernel<false>, dim3((unsigned)n), dim3(256), 0, st, A, t0);
            }
        }
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipEventRecord(ev[1 + hb], st));
        BEM_HIP(hipStreamWaitEvent(gs, ev[1 + hb], 0));
        const int r0 = h.strip_rptr[s], nr = h.strip_rptr[s + 1] - r0, lo = h.strip_lo[s];
        const int32_t *rows = m->d.strip_rows.as<int32_t>() + r0;
        const unsigned cr = (unsigned)((nr + 15) / 16);
        const dim3 ga(cr, cr), gb(cr, (unsigned)((nv - lo + 15) / 16));
#define GATHER_ARGS(C2)                                                                                              \
    nv, (int)nb, b0, b1, t0, lo, rows, nr, m->d.memb_ptr.as<int32_t>(), m->d.memb.as<int32_t>(),                    \
        reinterpret_cast<const C2 *>(buf), static_cast<C2 *>(ops[0]), static_cast<C2 *>(ops[1]),                     \
        static_cast<C2 *>(ops[2]), static_cast<C2 *>(ops[3])
        if (nr > 0) {   // (every strip has rows: its blocks have vertices)
            KTimer kt(ctx, K_GATHER);
            if (!fp32) {
                launch_k(kt, gather_strip_kernel<double2, true>, ga, dim3(256), 0, gs, GATHER_ARGS(double2));
                KTimer kt2(ctx, K_GATHER);
                launch_k(kt2, gather_strip_kernel<double2, false>, gb, dim3(256), 0, gs, GATHER_ARGS(double2));
            } else {
                launch_k(kt, gather_strip_kernel<float2, true>, ga, dim3(256), 0, gs, GATHER_ARGS(float2));
                KTimer kt2(ctx, K_GATHER);
                launch_k(kt2, gather_strip_kernel<float2, false>, gb, dim3(256), 0, gs, GATHER_ARGS(float2));
            }
        }
#undef GATHER_ARGS
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipEventRecord(ev[3 + hb], gs));
    }
    BEM_HIP(hipStreamWaitEvent(st, ev[3 + (ns - 1) % 2], 0));   // gathers run in order: the last covers all
    return BEM_OK;
}

bem_status launch_singular(const bem_mesh *m, double k, double kim, int ng, const double *glx, const double *glw, bool fp32,
                           double2 *contrib, void *ops[4], hipStream_t st)
{
    GLTab gl;
    for (int i = 0; i < NG_MAX; ++i) { gl.x[i] = i < ng ? glx[i] : 0.0; gl.w[i] = i < ng ? glw[i] : 0.0; }
    const int np = (int)m->h.sing.size();
    if (np > 0) {
        KTimer kt(m->ctx, K_SINGULAR);
        if (kim != 0.0)
            launch_k(kt, singular_pairs_kernel<true>, dim3((np + 15) / 16), dim3(256), 0, st, m->d.geo.as<TriGeo>(),
                     m->d.sing.as<SingPair>(), np, ng, gl, k, kim, contrib);
        else
            launch_k(kt, singular_pairs_kernel<false>, dim3((np + 15) / 16), dim3(256), 0, st, m->d.geo.as<TriGeo>(),
                     m->d.sing.as<SingPair>(), np, ng, gl, k, kim, contrib);
        BEM_HIP(hipGetLastError());
    }
    const int nn = (int)m->h.near_i.size();
    if (nn > 0) {
        KTimer kt(m->ctx, K_NEAR);
        const int nv = (int)m->h.nv;
        if (!fp32)
            launch_k(kt, near_scatter_kernel<double2>, dim3((nn + 255) / 256), dim3(256), 0, st, nv, nn,
                     m->d.near_i.as<int32_t>(), m->d.near_j.as<int32_t>(), m->d.near_ptr.as<int32_t>(),
                     m->d.near_src.as<int32_t>(), (const double2 *)contrib, static_cast<double2 *>(ops[0]),
                     static_cast<double2 *>(ops[1]), static_cast<double2 *>(ops[2]), static_cast<double2 *>(ops[3]));
        else
            launch_k(kt, near_scatter_kernel<float2>, dim3((nn + 255) / 256), dim3(256), 0, st, nv, nn,
                     m->d.near_i.as<int32_t>(), m->d.near_j.as<int32_t>(), m->d.near_ptr.as<int32_t>(),
                     m->d.near_src.as<int32_t>(), (const double2 *)contrib, static_cast<float2 *>(ops[0]),
                     static_cast<float2 *>(ops[1]), static_cast<float2 *>(ops[2]), static_cast<float2 *>(ops[3]));
        BEM_HIP(hipGetLastError());
    }
    return BEM_OK;
}

}  // namespace bemtx
