// Mass matrices, the L2 mortar matrix between the two meshes (Sec. 3.1), and
// the Gauss-Legendre rule of the singular quadrature.  Host code: integer
// connectivity, clipping and O(N) sparse work that the paper reports at a few
// percent of the assembly time (Sec. 5.4).
//
// Mortar matrix: P_int,ext[i][j] = <theta_i, phi_j>_L2 with theta_i the P1
// function of interior vertex i and phi_j that of exterior vertex j.  For the
// curved (star-shaped) surfaces used here the two polyhedra differ; an
// interior triangle is carried onto the plane of an exterior facet by central
// projection of its vertices from the origin, theta_i is interpolated
// linearly on the projected triangle, and the product is integrated exactly
// over the convex intersection polygon.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "mortar_geom.h"

namespace bemtx {

// CSR from row-grouped entries: ent[ptr[i], ptr[i + 1]) are the entries of
// row i in generation order.  Duplicate columns are summed in that order
// (first occurrence first), then the distinct columns of a row are sorted.
// Rows are independent and split over the host workers.
template <class PtrVec, class EntVec>
static void rows_to_csr(int64_t nrows, int64_t ncols, const PtrVec &ptr, EntVec &ent, Csr &A)
{
    std::vector<int32_t> ucnt(nrows, 0);
    parallel_for(nrows, 64, [&](int64_t r0, int64_t r1) {
        std::vector<int32_t> mark(ncols, -1), pos(ncols, 0);
        for (int64_t i = r0; i < r1; ++i) {
            auto *e = ent.data() + ptr[i];
            const int32_t n = ptr[i + 1] - ptr[i];
            int32_t m = 0;
            for (int32_t q = 0; q < n; ++q) {
                const int32_t c = e[q].first;
                if (mark[c] != (int32_t)i) {
                    mark[c] = (int32_t)i;
                    pos[c] = m;
                    e[m++] = e[q];
                } else {
                    e[pos[c]].second += e[q].second;
                }
            }
            std::sort(e, e + m, [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                return x.first < y.first;
            });
            ucnt[i] = m;
        }
    });
    A.nrows = nrows;
    A.ncols = ncols;
    A.ptr.assign(nrows + 1, 0);
    for (int64_t i = 0; i < nrows; ++i) A.ptr[i + 1] = A.ptr[i] + ucnt[i];
    A.col.resize(A.ptr[nrows]);
    A.val.resize(A.ptr[nrows]);
    parallel_for(nrows, 256, [&](int64_t r0, int64_t r1) {
        for (int64_t i = r0; i < r1; ++i)
            for (int32_t q = 0; q < ucnt[i]; ++q) {
                A.col[A.ptr[i] + q] = ent[ptr[i] + q].first;
                A.val[A.ptr[i] + q] = ent[ptr[i] + q].second;
            }
    });
}

void mass_csr(const MeshData &m, Csr &M)
{
    const int64_t nv = m.nv, nt = m.nt;
    // entries of row v[i] in triangle order: (v[j], |t| (1 + [i == j]) / 12)
    std::vector<int32_t> ptr(nv + 1, 0);
    for (int64_t t = 0; t < nt; ++t)
        for (int i = 0; i < 3; ++i) ptr[m.tri[3 * t + i] + 1] += 3;
    for (int64_t i = 0; i < nv; ++i) ptr[i + 1] += ptr[i];
    std::vector<std::pair<int32_t, double>> ent(ptr[nv]);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *v = &m.tri[3 * t];
        const double *p0 = &m.xyz[3 * v[0]], *p1 = &m.xyz[3 * v[1]], *p2 = &m.xyz[3 * v[2]];
        double a[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        double b[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        double area = 0.5 * std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) ent[fill[v[i]]++] = {v[j], area * (i == j ? 2.0 : 1.0) / 12.0};
    }
    rows_to_csr(nv, nv, ptr, ent, M);
}

void transpose_csr(const Csr &A, Csr &At)
{
    At.nrows = A.ncols;
    At.ncols = A.nrows;
    At.ptr.assign(At.nrows + 1, 0);
    for (int32_t c : A.col) At.ptr[c + 1]++;
    for (int64_t i = 0; i < At.nrows; ++i) At.ptr[i + 1] += At.ptr[i];
    At.col.assign(A.col.size(), 0);
    At.val.assign(A.val.size(), 0.0);
    std::vector<int32_t> fill(At.ptr.begin(), At.ptr.end() - 1);
    for (int64_t r = 0; r < A.nrows; ++r)
        for (int32_t q = A.ptr[r]; q < A.ptr[r + 1]; ++q) {
            int32_t d = fill[A.col[q]]++;
            At.col[d] = (int32_t)r;
            At.val[d] = A.val[q];
        }
}

void mortar_grid(const MeshData &mi, const MeshData &me, MortarGrid &g)
{
    auto cones = [](const MeshData &m, std::vector<double> &c, std::vector<double> &r) {
        c.assign(3 * m.nt, 0.0);
        r.assign(m.nt, 0.0);
        for (int64_t t = 0; t < m.nt; ++t) {
            const int32_t *v = &m.tri[3 * t];
            mgeo::cone(&m.xyz[3 * v[0]], &m.xyz[3 * v[1]], &m.xyz[3 * v[2]], &c[3 * t], &r[t]);
        }
    };
    cones(mi, g.ci, g.ri);
    cones(me, g.ce, g.re);
    const double rmax_i = *std::max_element(g.ri.begin(), g.ri.end()), rmax_e = *std::max_element(g.re.begin(), g.re.end());
    const double cell = 1.05 * (rmax_i + rmax_e) + 1e-12;
    g.ncell = std::max(1, std::min(256, (int)std::floor(2.0 / cell)));
    g.h = 2.0 / g.ncell;
    const int64_t nc = (int64_t)g.ncell * g.ncell * g.ncell;
    std::vector<int32_t> cid(mi.nt);
    g.cell_ptr.assign(nc + 1, 0);
    for (int64_t t = 0; t < mi.nt; ++t) {
        cid[t] = (int32_t)(((int64_t)mgeo::cell_of(g.ci[3 * t], g.ncell, g.h) * g.ncell +
                            mgeo::cell_of(g.ci[3 * t + 1], g.ncell, g.h)) * g.ncell +
                           mgeo::cell_of(g.ci[3 * t + 2], g.ncell, g.h));
        g.cell_ptr[cid[t] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) g.cell_ptr[c + 1] += g.cell_ptr[c];
    g.cell_tri.resize(mi.nt);
    std::vector<int32_t> fill(g.cell_ptr.begin(), g.cell_ptr.end() - 1);
    for (int64_t t = 0; t < mi.nt; ++t) g.cell_tri[fill[cid[t]]++] = (int32_t)t;   // ascending within a cell
}

bem_status mortar_csr(const MeshData &mi, const MeshData &me, Csr &P, double *coverage_defect)
{
    const int64_t nte = me.nt;
    MortarGrid g;
    mortar_grid(mi, me, g);
    // per exterior facet: (interior triangle, 3x3 block) contributions, facets split over host threads
    // (contiguous facet chunks, so the concatenation of the chunk lists is in facet order)
    struct Chunk { std::vector<int32_t> ti, te; std::vector<double> blk; int overflow = 0; };
    const int64_t nchunk = std::min<int64_t>(nte, 256);
    std::vector<Chunk> per_chunk(nchunk);
    std::vector<double> defect(nte, 0.0);
    auto work = [&](int64_t c0, int64_t c1) {
        for (int64_t ch = c0; ch < c1; ++ch) {
            Chunk &out = per_chunk[ch];
            for (int64_t te = nte * ch / nchunk; te < nte * (ch + 1) / nchunk; ++te) {
                const int32_t *ve = &me.tri[3 * te];
                const mgeo::Facet F = mgeo::make_facet(&me.xyz[3 * ve[0]], &me.xyz[3 * ve[1]], &me.xyz[3 * ve[2]]);
                double covered = 0.0;
                const int gx = mgeo::cell_of(g.ce[3 * te], g.ncell, g.h), gy = mgeo::cell_of(g.ce[3 * te + 1], g.ncell, g.h),
                          gz = mgeo::cell_of(g.ce[3 * te + 2], g.ncell, g.h);
                for (int dx = -1; dx <= 1; ++dx)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dz = -1; dz <= 1; ++dz) {
                            const int x = gx + dx, y = gy + dy, z = gz + dz;
                            if (x < 0 || y < 0 || z < 0 || x >= g.ncell || y >= g.ncell || z >= g.ncell) continue;
                            const int64_t c = ((int64_t)x * g.ncell + y) * g.ncell + z;
                            for (int32_t q = g.cell_ptr[c]; q < g.cell_ptr[c + 1]; ++q) {
                                const int32_t ti = g.cell_tri[q];
                                if (!mgeo::cones_meet(&g.ci[3 * ti], g.ri[ti], &g.ce[3 * te], g.re[te])) continue;
                                const int32_t *vi = &mi.tri[3 * ti];
                                double blk[3][3], ap = 0.0;
                                const int r = mgeo::pair_block(F, &mi.xyz[3 * vi[0]], &mi.xyz[3 * vi[1]], &mi.xyz[3 * vi[2]], blk, &ap);
                                if (r < 0) out.overflow = 1;
                                if (r <= 0) continue;
                                covered += ap;
                                out.ti.push_back(ti);
                                out.te.push_back((int32_t)te);
                                for (int a = 0; a < 3; ++a)
                                    for (int b = 0; b < 3; ++b) out.blk.push_back(blk[a][b]);
                            }
                        }
                defect[te] = std::fabs(covered - F.area) / F.area;
            }
        }
    };
    parallel_for(nchunk, 1, work);
    double worst = 0.0;
    for (double d : defect) worst = std::max(worst, d);
    if (coverage_defect) *coverage_defect = worst;
    // one array in facet order: chunk offsets, then the chunks copied in parallel
    std::vector<int64_t> coff(nchunk + 1, 0);
    for (int64_t ch = 0; ch < nchunk; ++ch) {
        if (per_chunk[ch].overflow) return set_error(BEM_E_MESH, "degenerate facet intersection in the mortar projection");
        coff[ch + 1] = coff[ch] + (int64_t)per_chunk[ch].ti.size();
    }
    const int64_t ncon = coff[nchunk];
    HVec<int32_t> ti(ncon), te(ncon);
    HVec<double> blk(9 * ncon);
    parallel_for(nchunk, 1, [&](int64_t c0, int64_t c1) {
        for (int64_t ch = c0; ch < c1; ++ch) {
            const Chunk &c = per_chunk[ch];
            std::copy(c.ti.begin(), c.ti.end(), ti.begin() + coff[ch]);
            std::copy(c.te.begin(), c.te.end(), te.begin() + coff[ch]);
            std::copy(c.blk.begin(), c.blk.end(), blk.begin() + 9 * coff[ch]);
        }
    });
    return mortar_from_contribs(mi, me, ncon, ti.data(), te.data(), blk.data(), worst, P);
}

bem_status mortar_from_contribs(const MeshData &mi, const MeshData &me, int64_t ncon, const int32_t *cti,
                                const int32_t *cte, const double *cblk, double worst, Csr &P)
{
    const int64_t nti = mi.nt;
    // entries grouped by interior row, each row in facet order, then CSR.
    // Contributions are numbered in facet order and listed per interior
    // triangle; a row gathers the lists of the triangles around its vertex and
    // sorts them by that number, so rows fill independently.
    HVec<int32_t> tptr(nti + 1, 0), tcon(ncon);
    for (int64_t k = 0; k < ncon; ++k) tptr[cti[k] + 1]++;
    for (int64_t t = 0; t < nti; ++t) tptr[t + 1] += tptr[t];
    {
        std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
        for (int64_t k = 0; k < ncon; ++k) tcon[fill[cti[k]]++] = (int32_t)k;
    }
    // triangles around each interior vertex
    HVec<int32_t> vptr(mi.nv + 1, 0), vtri(3 * nti);
    for (int64_t t = 0; t < nti; ++t)
        for (int a = 0; a < 3; ++a) vptr[mi.tri[3 * t + a] + 1]++;
    for (int64_t i = 0; i < mi.nv; ++i) vptr[i + 1] += vptr[i];
    {
        std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t t = 0; t < nti; ++t)
            for (int a = 0; a < 3; ++a) vtri[fill[mi.tri[3 * t + a]]++] = (int32_t)t;
    }
    HVec<int32_t> cnt(mi.nv + 1, 0);
    for (int64_t i = 0; i < mi.nv; ++i) {
        int32_t n = 0;
        for (int32_t q = vptr[i]; q < vptr[i + 1]; ++q) n += tptr[vtri[q] + 1] - tptr[vtri[q]];
        cnt[i + 1] = cnt[i] + 3 * n;
    }
    HVec<std::pair<int32_t, double>> ent(cnt[mi.nv]);
    parallel_for(mi.nv, 64, [&](int64_t r0, int64_t r1) {
        std::vector<int32_t> ks;
        for (int64_t i = r0; i < r1; ++i) {
            ks.clear();
            for (int32_t q = vptr[i]; q < vptr[i + 1]; ++q)
                for (int32_t u = tptr[vtri[q]]; u < tptr[vtri[q] + 1]; ++u) ks.push_back(tcon[u]);
            std::sort(ks.begin(), ks.end());
            int32_t w = cnt[i];
            for (int32_t k : ks) {
                const int32_t t = cti[k];
                const int a = mi.tri[3 * t] == i ? 0 : mi.tri[3 * t + 1] == i ? 1 : 2;
                for (int b = 0; b < 3; ++b) ent[w++] = {me.tri[3 * cte[k] + b], cblk[9 * (int64_t)k + 3 * a + b]};
            }
        }
    });
    rows_to_csr(mi.nv, me.nv, cnt, ent, P);
    if (worst > 1e-6)
        return set_error(BEM_E_MESH_MISMATCH, "projected interior mesh leaves an exterior facet uncovered (relative defect " +
                                                  std::to_string(worst) + ")");
    return BEM_OK;
}

// Gauss-Legendre nodes and weights on [0,1] from the eigen-decomposition of
// the symmetric tridiagonal Jacobi matrix of the Legendre recurrence
// (Golub-Welsch), computed with cyclic Jacobi rotations.
void gauss_legendre01(int n, double *x, double *w)
{
    std::vector<double> A((size_t)n * n, 0.0), Q((size_t)n * n, 0.0);
    for (int k = 1; k < n; ++k) {
        double b = k / std::sqrt(4.0 * k * k - 1.0);
        A[(size_t)(k - 1) * n + k] = A[(size_t)k * n + k - 1] = b;
    }
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (off < 1e-34) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
                    Q[(size_t)k * n + p] = c * qkp - s * qkq;
                    Q[(size_t)k * n + q] = s * qkp + c * qkq;
                }
            }
    }
    std::vector<std::pair<double, double>> nw(n);
    for (int i = 0; i < n; ++i) nw[i] = {A[(size_t)i * n + i], Q[i] * Q[i]};   // first component of eigenvector i
    std::sort(nw.begin(), nw.end());
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (nw[i].first + 1.0);
        w[i] = nw[i].second;     // (2 * q0^2) on [-1,1], halved on [0,1]
    }
}

}  // namespace bemtx
