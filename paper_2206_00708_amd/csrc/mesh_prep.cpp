// Mesh validation and connectivity tables (host side of the geometry step).
//
// A mesh Gamma_int or Gamma_ext is a conforming triangulation of the closed
// surface (Sec. 3).  This file checks that, renumbers triangles and vertices
// for locality, and builds the integer tables the kernels need:
//   * locality blocks of <= BT triangles / <= SMAX vertices and, per block,
//     the (triangle, corner) list of every vertex slot;
//   * vertex -> (block, slot) memberships for the deterministic gather of
//     the dense operator entries;
//   * the ordered triangle pairs sharing 1, 2 or 3 vertices, which take the
//     Sauter-Schwab rules (Sec. 5.1), with the corner permutations that put
//     the shared vertices first; and the list of dense entries they touch;
//   * the vertex star (triangle, corner) lists for load-vector gathers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "internal.h"

namespace bemtx {

static uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &f)
{
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nth = std::max<int64_t>(1, std::min<int64_t>(16, hw ? hw : 1));
    nth = std::min<int64_t>(nth, std::max<int64_t>(1, n / std::max<int64_t>(1, grain)));
    if (nth <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nth; ++t) pool.emplace_back(f, n * t / nth, n * (t + 1) / nth);
    for (auto &th : pool) th.join();
}

bem_status mesh_prepare(MeshData &m)
{
    const int64_t nv = m.nv, nt = m.nt;
    const double *X = m.xyz_user.data();
    const int32_t *T = m.tri_user.data();
    if (nv < 4 || nt < 4) return set_error(BEM_E_MESH, "mesh needs at least 4 vertices and 4 triangles");
    if (nv > (1 << 30) || nt > (1 << 30)) return set_error(BEM_E_ARG, "mesh too large");
    std::vector<int32_t> used(nv, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) {
        if (T[i] < 0 || T[i] >= nv) return set_error(BEM_E_MESH, "triangle index out of range");
        used[T[i]] = 1;
    }
    for (int64_t v = 0; v < nv; ++v)
        if (!used[v]) return set_error(BEM_E_MESH, "unused vertex " + std::to_string(v));
    // closed, consistently oriented: every directed edge once, its reverse present
    {
        std::vector<uint64_t> e(3 * nt), r(3 * nt);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a) {
                uint64_t u = (uint32_t)T[3 * t + a], w = (uint32_t)T[3 * t + (a + 1) % 3];
                if (u == w) return set_error(BEM_E_MESH, "repeated vertex in a triangle");
                e[3 * t + a] = u << 32 | w;
                r[3 * t + a] = w << 32 | u;
            }
        std::sort(e.begin(), e.end());
        if (std::adjacent_find(e.begin(), e.end()) != e.end())
            return set_error(BEM_E_MESH, "edge used twice with the same orientation (non-manifold or flipped)");
        std::sort(r.begin(), r.end());
        if (e != r) return set_error(BEM_E_MESH, "mesh is not closed or not consistently oriented");
    }
    double vol = 0.0, amax = 0.0, amin = 1e300;
    m.area_total = 0.0;
    for (int64_t t = 0; t < nt; ++t) {
        const double *p0 = X + 3 * T[3 * t], *p1 = X + 3 * T[3 * t + 1], *p2 = X + 3 * T[3 * t + 2];
        double a[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        double b[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        double ar = 0.5 * std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        amax = std::max(amax, ar);
        amin = std::min(amin, ar);
        m.area_total += ar;
        vol += (p0[0] * (p1[1] * p2[2] - p1[2] * p2[1]) - p0[1] * (p1[0] * p2[2] - p1[2] * p2[0]) +
                p0[2] * (p1[0] * p2[1] - p1[1] * p2[0])) / 6.0;
    }
    if (!(amin > 1e-12 * amax)) return set_error(BEM_E_MESH, "degenerate triangle");
    if (!(vol > 0)) return set_error(BEM_E_MESH, "triangles are oriented inwards (negative enclosed volume)");

    // ---- Morton order of triangle centroids
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < nv; ++v)
        for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], X[3 * v + c]); hi[c] = std::max(hi[c], X[3 * v + c]); }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    std::vector<std::pair<uint64_t, int32_t>> key(nt);
    for (int64_t t = 0; t < nt; ++t) {
        uint64_t code = 0;
        for (int c = 0; c < 3; ++c) {
            double g = (X[3 * T[3 * t] + c] + X[3 * T[3 * t + 1] + c] + X[3 * T[3 * t + 2] + c]) / 3.0;
            uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, (g - lo[c]) / ext * 2097151.0));
            code |= spread3(q) << c;
        }
        key[t] = {code, (int32_t)t};
    }
    std::sort(key.begin(), key.end());

    // ---- blocks (<= BT triangles, <= SMAX vertices) and internal vertex numbering
    m.int_of_v.assign(nv, -1);
    m.v_of_int.clear();
    m.v_of_int.reserve(nv);
    m.tri.assign(3 * nt, 0);
    m.blk_start.clear();
    int32_t cur_n = 0;
    std::vector<int32_t> cur_verts;
    for (int64_t s = 0; s < nt; ++s) {
        int32_t t = key[s].second;
        int newv = 0;
        for (int a = 0; a < 3; ++a) {
            int32_t u = T[3 * t + a];
            if (std::find(cur_verts.begin(), cur_verts.end(), u) == cur_verts.end()) ++newv;
        }
        if (cur_n == 0 || cur_n == BT || (int)cur_verts.size() + newv > SMAX) {
            m.blk_start.push_back((int32_t)s);
            cur_n = 0;
            cur_verts.clear();
        }
        for (int a = 0; a < 3; ++a) {
            int32_t u = T[3 * t + a];
            if (std::find(cur_verts.begin(), cur_verts.end(), u) == cur_verts.end()) cur_verts.push_back(u);
            if (m.int_of_v[u] < 0) {
                m.int_of_v[u] = (int32_t)m.v_of_int.size();
                m.v_of_int.push_back(u);
            }
        }
        ++cur_n;
    }
    m.blk_start.push_back((int32_t)nt);
    m.nb = (int32_t)m.blk_start.size() - 1;
    for (int64_t s = 0; s < nt; ++s)
        for (int a = 0; a < 3; ++a) m.tri[3 * s + a] = m.int_of_v[T[3 * key[s].second + a]];
    m.xyz.assign(3 * nv, 0.0);
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) m.xyz[3 * i + c] = X[3 * m.v_of_int[i] + c];

    // ---- per-block slots and (triangle, corner) lists
    const int nb = m.nb;
    m.blk_nslot.assign(nb, 0);
    m.blk_slots.assign((size_t)nb * SMAX, -1);
    m.slot_cnt.assign((size_t)nb * SMAX, 0);
    m.slot_ent.assign((size_t)nb * SMAX * LMAX, 0);
    std::vector<std::vector<int32_t>> memb_lists(nv);
    for (int b = 0; b < nb; ++b) {
        std::vector<int32_t> vs;
        for (int32_t t = m.blk_start[b]; t < m.blk_start[b + 1]; ++t)
            for (int a = 0; a < 3; ++a) vs.push_back(m.tri[3 * t + a]);
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        if ((int)vs.size() > SMAX) return set_error(BEM_E_MESH, "internal: block vertex overflow");
        m.blk_nslot[b] = (int32_t)vs.size();
        for (size_t s = 0; s < vs.size(); ++s) {
            m.blk_slots[(size_t)b * SMAX + s] = vs[s];
            memb_lists[vs[s]].push_back(b << 8 | (int32_t)s);
        }
        for (int32_t t = m.blk_start[b]; t < m.blk_start[b + 1]; ++t)
            for (int a = 0; a < 3; ++a) {
                int s = (int)(std::lower_bound(vs.begin(), vs.end(), m.tri[3 * t + a]) - vs.begin());
                uint8_t &cnt = m.slot_cnt[(size_t)b * SMAX + s];
                if (cnt >= LMAX) return set_error(BEM_E_MESH, "vertex valence too high (> 12 corners in one block)");
                m.slot_ent[((size_t)b * SMAX + s) * LMAX + cnt] = (uint8_t)((t - m.blk_start[b]) * 3 + a);
                ++cnt;
            }
    }
    m.memb_ptr.assign(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) m.memb_ptr[v + 1] = m.memb_ptr[v] + (int32_t)memb_lists[v].size();
    m.memb.resize(m.memb_ptr[nv]);
    for (int64_t v = 0; v < nv; ++v)
        std::copy(memb_lists[v].begin(), memb_lists[v].end(), m.memb.begin() + m.memb_ptr[v]);

    // ---- vertex stars (internal numbering)
    m.star_ptr.assign(nv + 1, 0);
    for (int64_t i = 0; i < 3 * nt; ++i) m.star_ptr[m.tri[i] + 1]++;
    for (int64_t v = 0; v < nv; ++v) m.star_ptr[v + 1] += m.star_ptr[v];
    m.star_ent.assign(3 * nt, 0);
    {
        std::vector<int32_t> fill(m.star_ptr.begin(), m.star_ptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a) m.star_ent[fill[m.tri[3 * t + a]]++] = (int32_t)(3 * t + a);
    }

    // ---- ordered singular pairs, kinds 3 / 2 / 1, corner permutations
    std::vector<SingPair> by_kind[4];
    for (int k = 1; k <= 3; ++k) by_kind[k].reserve(k == 1 ? 10 * nt : (k == 2 ? 3 * nt : nt));
    std::vector<int64_t> seen_by(nt, -1);
    for (int64_t t = 0; t < nt; ++t) {
        for (int a = 0; a < 3; ++a) {
            int32_t v = m.tri[3 * t + a];
            for (int32_t e = m.star_ptr[v]; e < m.star_ptr[v + 1]; ++e) {
                int32_t s = m.star_ent[e] / 3;
                if (seen_by[s] == t) continue;
                seen_by[s] = t;
                int sx[3], sy[3], ns = 0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        if (m.tri[3 * t + i] == m.tri[3 * s + j]) { sx[ns] = i; sy[ns] = j; ++ns; }
                int px[3], py[3];
                if (ns == 3) {
                    for (int r = 0; r < 3; ++r) { px[r] = r; py[r] = r; }
                } else if (ns == 2) {
                    px[0] = sx[0]; px[1] = sx[1]; px[2] = 3 - sx[0] - sx[1];
                    py[0] = sy[0]; py[1] = sy[1]; py[2] = 3 - sy[0] - sy[1];
                } else {
                    for (int r = 0; r < 3; ++r) { px[r] = (sx[0] + r) % 3; py[r] = (sy[0] + r) % 3; }
                }
                SingPair sp;
                sp.tau = (int32_t)t;
                sp.sig = s;
                sp.kind = ns;
                sp.perm = px[0] | px[1] << 2 | px[2] << 4 | py[0] << 6 | py[1] << 8 | py[2] << 10;
                by_kind[ns].push_back(sp);
            }
        }
    }
    m.sing.clear();
    for (int kind = 3; kind >= 1; --kind) {
        m.nsing_kind[kind] = (int32_t)by_kind[kind].size();
        m.sing.insert(m.sing.end(), by_kind[kind].begin(), by_kind[kind].end());
    }

    // ---- near entries: unique (i, j) touched by singular pairs, contributions in pair order
    {
        const size_t nc = m.sing.size() * 9;
        std::vector<int32_t> row_cnt(nv + 1, 0);
        for (size_t p = 0; p < m.sing.size(); ++p)
            for (int a = 0; a < 3; ++a) row_cnt[m.tri[3 * m.sing[p].tau + a] + 1] += 3;
        for (int64_t v = 0; v < nv; ++v) row_cnt[v + 1] += row_cnt[v];
        std::vector<int32_t> fill(row_cnt.begin(), row_cnt.end() - 1);
        std::vector<std::pair<int32_t, int32_t>> byrow(nc);   // (j, src), grouped by i, src ascending
        for (size_t p = 0; p < m.sing.size(); ++p)
            for (int a = 0; a < 3; ++a) {
                const int32_t i = m.tri[3 * m.sing[p].tau + a];
                for (int b = 0; b < 3; ++b)
                    byrow[fill[i]++] = {m.tri[3 * m.sing[p].sig + b], (int32_t)(p * 9 + a * 3 + b)};
            }
        // group each row's contributions by column j in order of first appearance
        // (deterministic; contributions keep their pair order within an entry);
        // rows in parallel: count distinct columns, prefix, then fill
        std::vector<int32_t> nuniq(nv + 1, 0);
        auto group_rows = [&](int64_t r0, int64_t r1, bool fill) {
            std::vector<int32_t> mark(nv, -1), slot_of(nv, 0), ucol, ucnt, off;
            for (int64_t i = r0; i < r1; ++i) {
                ucol.clear();
                ucnt.clear();
                for (int32_t e = row_cnt[i]; e < row_cnt[i + 1]; ++e) {
                    const int32_t j = byrow[e].first;
                    if (mark[j] != (int32_t)i) {
                        mark[j] = (int32_t)i;
                        slot_of[j] = (int32_t)ucol.size();
                        ucol.push_back(j);
                        ucnt.push_back(0);
                    }
                    ucnt[slot_of[j]]++;
                }
                if (!fill) {
                    nuniq[i + 1] = (int32_t)ucol.size();
                    continue;
                }
                off.resize(ucol.size());
                int32_t acc = row_cnt[i];
                for (size_t u = 0; u < ucol.size(); ++u) {
                    const size_t k = (size_t)nuniq[i] + u;
                    m.near_ptr[k] = acc;
                    m.near_i[k] = (int32_t)i;
                    m.near_j[k] = ucol[u];
                    off[u] = acc;
                    acc += ucnt[u];
                }
                for (int32_t e = row_cnt[i]; e < row_cnt[i + 1]; ++e)
                    m.near_src[off[slot_of[byrow[e].first]]++] = byrow[e].second;
            }
        };
        parallel_for(nv, 256, [&](int64_t a, int64_t b) { group_rows(a, b, false); });
        for (int64_t i = 0; i < nv; ++i) nuniq[i + 1] += nuniq[i];
        m.near_i.assign(nuniq[nv], 0);
        m.near_j.assign(nuniq[nv], 0);
        m.near_ptr.assign(nuniq[nv], 0);
        m.near_src.assign(nc, 0);
        parallel_for(nv, 256, [&](int64_t a, int64_t b) { group_rows(a, b, true); });
        m.near_ptr.push_back((int32_t)nc);
    }
    return BEM_OK;
}

}  // namespace bemtx
