// Sanitizer driver for the library's host code (built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host pass only, no device code):
// mesh checks and tables (mesh_prep.cpp, its thread pool), the mass and
// mortar matrices (mortar.cpp), the inverse-mass patch tables
// (mass_cheb.cpp) and the host-only C-ABI calls.  Meshes come from text
// files "nv nt / xyz rows / tri rows"; argv: int mesh, ext mesh, a broken
// mesh.  Exit 0 when every call behaves; any sanitizer report aborts.
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
