// Tables of the sparse inverse-mass apply (the mass-matrix preconditioner of
// Sec. 3.3 applied without forming M^-1).
//
// z = M^-1 y is computed by Chebyshev iteration on the Jacobi-scaled P1 mass
// matrix: every eigenvalue of diag(M)^-1 M lies in [1/2, 2] (each element
// matrix (A/12)[[2,1,1],[1,2,1],[1,1,2]] scaled by its diagonal has the
// eigenvalues 2, 1/2, 1/2, and the Rayleigh quotient of the sum lies between
// those of its terms), so k steps reduce the error by 4 3^-k on any mesh.
// One kernel launch takes s steps on overlapping patches: a patch owns a
// compact cluster of vertices and holds every vertex within s edges of them; after t steps the iterate is exact (to rounding) on the
// vertices within s - t edges, so after s steps on the owned ones.  The
// patch's vertices are listed by distance from the owned range, so that the
// rows updated at step t are a prefix of the list.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace bemtx {

namespace {

// one patch: its owned vertices and every vertex within s edges of them
struct Patch {
    std::vector<int32_t> vert, cnt, rptr, col;
    std::vector<double> dinv, val;
};

// Owned sets: compact clusters of at most `own` vertices, grown breadth-first
// from the lowest unassigned vertex over unassigned neighbours (a compact
// set has the shortest rings around it).  Deterministic.
std::vector<std::vector<int32_t>> clusters(const Csr &M, int own)
{
    const int32_t nv = (int32_t)M.nrows;
    std::vector<char> taken(nv, 0);
    std::vector<std::vector<int32_t>> out;
    for (int32_t seed = 0; seed < nv; ++seed) {
        if (taken[seed]) continue;
        std::vector<int32_t> c{seed};
        taken[seed] = 1;
        for (size_t q = 0; q < c.size() && (int)c.size() < own; ++q)
            for (int32_t e = M.ptr[c[q]]; e < M.ptr[c[q] + 1] && (int)c.size() < own; ++e) {
                const int32_t u = M.col[e];
                if (!taken[u]) {
                    taken[u] = 1;
                    c.push_back(u);
                }
            }
        std::sort(c.begin(), c.end());
        out.push_back(std::move(c));
    }
    return out;
}

void build_patch(const Csr &M, const std::vector<int32_t> &owned, int s, std::vector<int32_t> &dist,
                 std::vector<int32_t> &loc, Patch &P)
{
    P.vert.clear();
    for (int32_t v : owned) {
        dist[v] = 0;
        P.vert.push_back(v);
    }
    size_t front = 0;
    for (int d = 1; d <= s; ++d) {   // breadth-first rings; each ring in ascending vertex order
        const size_t end = P.vert.size();
        std::vector<int32_t> ring;
        for (size_t q = front; q < end; ++q) {
            const int32_t v = P.vert[q];
            for (int32_t e = M.ptr[v]; e < M.ptr[v + 1]; ++e) {
                const int32_t u = M.col[e];
                if (dist[u] < 0) {
                    dist[u] = d;
                    ring.push_back(u);
                }
            }
        }
        std::sort(ring.begin(), ring.end());
        P.vert.insert(P.vert.end(), ring.begin(), ring.end());
        front = end;
    }
    const int32_t L = (int32_t)P.vert.size();
    for (int32_t l = 0; l < L; ++l) loc[P.vert[l]] = l;
    P.cnt.assign(s + 1, 0);
    for (int32_t l = 0; l < L; ++l) P.cnt[dist[P.vert[l]]]++;
    for (int d = 1; d <= s; ++d) P.cnt[d] += P.cnt[d - 1];   // cnt[d] = vertices within d edges
    P.dinv.assign(L, 0.0);
    P.rptr.assign(L + 1, 0);
    P.col.clear();
    P.val.clear();
    for (int32_t l = 0; l < L; ++l) {
        const int32_t v = P.vert[l];
        double diag = 0.0;
        for (int32_t e = M.ptr[v]; e < M.ptr[v + 1]; ++e)
            if (M.col[e] == v) diag += M.val[e];
        P.dinv[l] = 1.0 / diag;
        if (dist[v] < s)   // rows read only at the steps that update them
            for (int32_t e = M.ptr[v]; e < M.ptr[v + 1]; ++e) {
                P.col.push_back(loc[M.col[e]]);
                P.val.push_back(M.val[e]);
            }
        P.rptr[l + 1] = (int32_t)P.col.size();
    }
    for (int32_t v : P.vert) {
        dist[v] = -1;
        loc[v] = -1;
    }
}

}  // namespace

bem_status cheb_tables(const Csr M[2], int s, ChebTables &T)
{
    T.s = s;
    // owned range per patch: halved until the largest patch fits the kernel's register and LDS budget
    for (int own = CHEB_OWN_MAX; own >= 32; own /= 2) {
        std::vector<Patch> patches;
        std::vector<int32_t> pm;
        for (int m = 0; m < 2; ++m) {
            const int32_t nv = (int32_t)M[m].nrows;
            const std::vector<std::vector<int32_t>> cl = clusters(M[m], own);
            const int32_t np = (int32_t)cl.size();
            T.nparts[m] = np;
            const size_t first = patches.size();
            patches.resize(first + np);
            pm.insert(pm.end(), np, m);
            parallel_for(np, 1, [&](int64_t a, int64_t b) {
                std::vector<int32_t> dist(nv, -1), loc(nv, -1);
                for (int64_t q = a; q < b; ++q) build_patch(M[m], cl[q], s, dist, loc, patches[first + q]);
            });
        }
        int lmax = 0;
        for (const Patch &P : patches) lmax = std::max(lmax, (int)P.vert.size());
        int wmax = 1;
        for (const Patch &P : patches)
            for (size_t l = 0; l + 1 < P.rptr.size(); ++l) wmax = std::max(wmax, P.rptr[l + 1] - P.rptr[l]);
        if (wmax > CHEB_WMAX) return set_error(BEM_E_MESH, "inverse-mass rows wider than the kernel's limit "
                                                           "(a vertex with more than 15 neighbours)");
        if (lmax > CHEB_LMAX && own > 32) continue;
        if (lmax > CHEB_LMAX) return set_error(BEM_E_MESH, "inverse-mass patches exceed the kernel's limit");
        T.own = own;
        T.lmax = lmax;
        T.pmesh.assign(pm.begin(), pm.end());
        T.vbeg.assign(1, 0);
        T.cnt.clear();
        T.vert.clear();
        T.dinv.clear();
        T.rptr.clear();
        T.col.clear();
        T.val.clear();
        for (const Patch &P : patches) {
            const int32_t coff = (int32_t)T.col.size();
            T.vert.insert(T.vert.end(), P.vert.begin(), P.vert.end());
            T.dinv.insert(T.dinv.end(), P.dinv.begin(), P.dinv.end());
            T.cnt.insert(T.cnt.end(), P.cnt.begin(), P.cnt.end());
            for (size_t l = 0; l + 1 < P.rptr.size(); ++l) T.rptr.push_back(coff + P.rptr[l]);
            T.col.insert(T.col.end(), P.col.begin(), P.col.end());
            T.val.insert(T.val.end(), P.val.begin(), P.val.end());
            T.vbeg.push_back((int32_t)T.vert.size());
        }
        T.rptr.push_back((int32_t)T.col.size());
        // the same rows as ELL blocks of width w per patch, [q][local row], padded with zero entries on the
        // row's own vertex: the kernel keeps a row's entries in registers for all steps of a launch
        int w = 1;
        for (size_t l = 0; l + 1 < T.rptr.size(); ++l) w = std::max(w, T.rptr[l + 1] - T.rptr[l]);
        T.ell_w = w;
        T.ecol.assign((size_t)w * T.vert.size(), 0);
        T.eval.assign((size_t)w * T.vert.size(), 0.0);
        for (size_t q = 0; q + 1 < T.vbeg.size(); ++q) {
            const int32_t vb = T.vbeg[q], L = T.vbeg[q + 1] - vb;
            for (int32_t l = 0; l < L; ++l) {
                int e = 0;
                for (int32_t k = T.rptr[vb + l]; k < T.rptr[vb + l + 1]; ++k, ++e) {
                    T.ecol[(size_t)w * vb + (size_t)e * L + l] = (uint16_t)T.col[k];
                    T.eval[(size_t)w * vb + (size_t)e * L + l] = T.val[k];
                }
                for (; e < w; ++e) T.ecol[(size_t)w * vb + (size_t)e * L + l] = (uint16_t)l;
            }
        }
        return BEM_OK;
    }
    return set_error(BEM_E_MESH, "inverse-mass patches exceed the kernel's limit");
}

}  // namespace bemtx
