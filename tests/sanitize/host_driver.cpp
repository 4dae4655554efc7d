// Sanitizer driver for the library's host code (built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host pass only, no device code):
// mesh checks and tables (mesh_prep.cpp, its thread pool), the mass and
// mortar matrices (mortar.cpp), the inverse-mass patch tables
// (mass_cheb.cpp) and the host-only C-ABI calls.  Meshes come from text
// files "nv nt / xyz rows / tri rows"; argv: int mesh, ext mesh, a broken
// mesh.  Exit 0 when every call behaves; any sanitizer report aborts.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <vector>

#include "../../paper_2206_00708_amd/csrc/internal.h"

using namespace bemtx;

struct Mesh {
    std::vector<double> xyz;
    std::vector<int32_t> tri;
    int64_t nv = 0, nt = 0;
};

static bool read_mesh(const char *path, Mesh &m)
{
    std::ifstream f(path);
    if (!(f >> m.nv >> m.nt)) return false;
    m.xyz.resize(3 * m.nv);
    m.tri.resize(3 * m.nt);
    for (auto &x : m.xyz) f >> x;
    for (auto &t : m.tri) f >> t;
    return (bool)f;
}

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                              \
        }                                                          \
    } while (0)

// The slot-major corner ranks of every block: the corners of a block's
// triangles get the ranks 0 .. 3n - 1 once each; slot q holds the run
// [off[q], off[q + 1]) of length cnt[q], its corners ranked in the order of
// its list, and every corner of the run is at slot q's vertex.
static int check_slot_ranks(const MeshData &m)
{
    for (int b = 0; b < m.nb; ++b) {
        const int n = m.blk_start[b + 1] - m.blk_start[b], ns = m.blk_nslot[b];
        const uint8_t *off = &m.slot_off[(size_t)b * SLOT_OFF_LD], *rank = &m.slot_rank[(size_t)b * 3 * BT];
        CHECK(off[0] == 0 && off[ns] == 3 * n);
        std::vector<int> seen(3 * n, 0);
        for (int q = 0; q < ns; ++q) {
            const int cnt = m.slot_cnt[(size_t)b * SMAX + q];
            CHECK(cnt >= 1 && off[q + 1] - off[q] == cnt);
            for (int v = 0; v < cnt; ++v) {
                const int c = m.slot_ent[((size_t)b * SMAX + q) * LMAX + v];
                CHECK(c < 3 * n && rank[c] == off[q] + v);
                CHECK(m.tri[3 * (m.blk_start[b] + c / 3) + c % 3] == m.blk_slots[(size_t)b * SMAX + q]);
                seen[rank[c]]++;
            }
        }
        for (int r = 0; r < 3 * n; ++r) CHECK(seen[r] == 1);
    }
    return 0;
}

// The assembly strips of a prepared mesh: block ranges within the tile
// budget, the row list of each strip (the vertices with a membership in its
// blocks), its first reachable vertex, and the gather's coverage: over all
// strips, every dense entry (i, j) is visited where a strip holds one of its
// tiles (rows of the list against columns from the first reachable vertex,
// and rows outside the list from there against columns of the list),
// receives each membership pair's tile exactly once, and is written first
// by the strip of its smallest membership.
static int check_strips(const MeshData &m, int64_t cap)
{
    const int nv = (int)m.nv, nb = m.nb, ns = (int)m.strip_b.size() - 1;
    CHECK(ns >= 1 && m.strip_b[0] == 0 && m.strip_b[ns] == nb);
    CHECK((int)m.strip_rptr.size() == ns + 1 && (int)m.strip_lo.size() == ns);
    auto off = [&](int64_t b) { return b * nb - b * (b - 1) / 2; };
    std::vector<int> minb(nv), maxb(nv);
    for (int v = 0; v < nv; ++v) {
        CHECK(m.memb_ptr[v + 1] > m.memb_ptr[v]);
        minb[v] = m.memb[m.memb_ptr[v]] >> 8;
        maxb[v] = m.memb[m.memb_ptr[v + 1] - 1] >> 8;
    }
    std::vector<long> count((size_t)nv * nv, 0);
    std::vector<char> written((size_t)nv * nv, 0);
    for (int s = 0; s < ns; ++s) {
        const int b0 = m.strip_b[s], b1 = m.strip_b[s + 1];
        CHECK(b1 > b0);
        CHECK(b1 == b0 + 1 || off(b1) - off(b0) <= cap);
        std::vector<char> in(nv, 0);
        for (int q = m.strip_rptr[s]; q < m.strip_rptr[s + 1]; ++q) {
            CHECK(q == m.strip_rptr[s] || m.strip_rows[q] > m.strip_rows[q - 1]);
            in[m.strip_rows[q]] = 1;
        }
        int lo = nv;
        for (int v = 0; v < nv; ++v) {
            bool has = false;
            for (int p = m.memb_ptr[v]; p < m.memb_ptr[v + 1]; ++p) has |= (m.memb[p] >> 8) >= b0 && (m.memb[p] >> 8) < b1;
            CHECK(has == (in[v] != 0));
            if (maxb[v] >= b0 && v < lo) lo = v;
        }
        CHECK(m.strip_lo[s] == lo);
        auto visit = [&](int i, int j) -> bool {
            bool any = false;
            for (int p = m.memb_ptr[i]; p < m.memb_ptr[i + 1]; ++p)
                for (int q = m.memb_ptr[j]; q < m.memb_ptr[j + 1]; ++q) {
                    const int lb = std::min(m.memb[p] >> 8, m.memb[q] >> 8), hb = std::max(m.memb[p] >> 8, m.memb[q] >> 8);
                    if (lb < b0 || lb >= b1) continue;
                    const int64_t t = off(lb) + (hb - lb) - off(b0);
                    if (t < 0 || t >= off(b1) - off(b0)) return false;
                    any = true;
                    ++count[(size_t)i * nv + j];
                }
            const size_t o = (size_t)i * nv + j;
            if (std::min(minb[i], minb[j]) >= b0) {
                if (!any || written[o]) return false;
                written[o] = 1;
            } else if (any && !written[o]) {
                return false;
            }
            return true;
        };
        for (int i = 0; i < nv; ++i)
            for (int j = lo; j < nv; ++j)
                if (in[i]) CHECK(visit(i, j));
        for (int i = lo; i < nv; ++i)
            for (int j = 0; j < nv; ++j)
                if (!in[i] && in[j]) CHECK(visit(i, j));
    }
    for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
            const size_t o = (size_t)i * nv + j;
            CHECK(written[o]);
            CHECK(count[o] == (long)(m.memb_ptr[i + 1] - m.memb_ptr[i]) * (m.memb_ptr[j + 1] - m.memb_ptr[j]));
        }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 4) return 2;
    Mesh mi, me, bad;
    CHECK(read_mesh(argv[1], mi) && read_mesh(argv[2], me) && read_mesh(argv[3], bad));
    CHECK(bem_check_mesh(mi.xyz.data(), mi.nv, mi.tri.data(), mi.nt) == BEM_OK);
    CHECK(bem_check_mesh(me.xyz.data(), me.nv, me.tri.data(), me.nt) == BEM_OK);
    CHECK(bem_check_mesh(bad.xyz.data(), bad.nv, bad.tri.data(), bad.nt) == BEM_E_MESH);
    // host mortar: size query, then the matrix
    int64_t nnz = 0;
    double defect = 0;
    CHECK(bem_host_mortar(mi.xyz.data(), mi.nv, mi.tri.data(), mi.nt, me.xyz.data(), me.nv, me.tri.data(), me.nt,
                          nullptr, nullptr, nullptr, &nnz, &defect) == BEM_OK);
    std::vector<int64_t> rp(mi.nv + 1);
    std::vector<int32_t> col(nnz);
    std::vector<double> val(nnz);
    CHECK(bem_host_mortar(mi.xyz.data(), mi.nv, mi.tri.data(), mi.nt, me.xyz.data(), me.nv, me.tri.data(), me.nt,
                          rp.data(), col.data(), val.data(), &nnz, &defect) == BEM_OK);
    double total = 0;
    for (double v : val) total += v;
    CHECK(total > 0);
    // mesh tables, mass matrices and the inverse-mass patch tables of both meshes
    MeshData md[2];
    const Mesh *ms[2] = {&me, &mi};
    Csr M[2];
    for (int m = 0; m < 2; ++m) {
        md[m].nv = ms[m]->nv;
        md[m].nt = ms[m]->nt;
        md[m].xyz_user.assign(ms[m]->xyz.begin(), ms[m]->xyz.end());
        md[m].tri_user.assign(ms[m]->tri.begin(), ms[m]->tri.end());
        CHECK(mesh_prepare(md[m]) == BEM_OK);
        CHECK(check_strips(md[m], ASM_STRIP_TILES) == 0);
        CHECK(check_slot_ranks(md[m]) == 0);
        for (int64_t cap : {1, 37, 400}) {   // small strips: many strips, entries fed by several
            MeshData t;
            t.nv = md[m].nv;
            t.nt = md[m].nt;
            t.xyz_user = md[m].xyz_user;
            t.tri_user = md[m].tri_user;
            CHECK(mesh_prepare(t, cap) == BEM_OK);
            CHECK(check_strips(t, cap) == 0);
        }
        mass_csr(md[m], M[m]);
    }
    Csr P, Pt;
    CHECK(mortar_csr(md[1], md[0], P, &defect) == BEM_OK);
    transpose_csr(P, Pt);
    ChebTables T;
    CHECK(cheb_tables(M, CHEB_S, T) == BEM_OK);
    CHECK(T.lmax <= CHEB_LMAX && (int)T.vbeg.size() == T.nparts[0] + T.nparts[1] + 1);
    // host helpers
    double x[16], w[16];
    CHECK(bem_host_gauss_legendre(16, x, w) == BEM_OK);
    CHECK(bem_host_gauss_legendre(17, x, w) != BEM_OK);
    std::vector<double> ph(1000), s(1000), c(1000);
    for (int i = 0; i < 1000; ++i) ph[i] = 0.37 * i - 100.0;
    CHECK(bem_host_phase_sincos(1000, ph.data(), s.data(), c.data()) == BEM_OK);
    for (int i = 0; i < 1000; ++i) CHECK(std::fabs(s[i] * s[i] + c[i] * c[i] - 1.0) < 1e-14);
    std::printf("host driver ok: mortar nnz %ld, patches %d + %d\n", (long)nnz, T.nparts[0], T.nparts[1]);
    return 0;
}
