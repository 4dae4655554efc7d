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
#include <functional>
#include <numeric>
#include <atomic>
#include <condition_variable>
#include <map>
#include <mutex>
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

// Persistent worker threads for parallel_for (host table building and the
// mortar).  One parallel_for owns the pool at a time; a call that finds it
// busy (another thread of the caller inside the library) runs its range
// inline, so concurrent callers never wait on each other.
namespace {
class Pool {
  public:
    static Pool &get()
    {
        // never destroyed: the workers wait on its condition variable until the process ends
        static Pool *pool = new Pool;
        return *pool;
    }
    int size() const { return (int)workers_.size() + 1; }
    std::mutex owner;   // held for the duration of one parallel_for

    // run f(part) for part in [0, nparts) on the workers and the caller
    void run(int nparts, const std::function<void(int)> &f)
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            job_ = &f;
            nparts_ = nparts;
            next_ = 1;   // the caller takes part 0
            done_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        f(0);
        int mine;
        while ((mine = take()) >= 0) { f(mine); finish(); }
        std::unique_lock<std::mutex> lk(m_);
        cv_done_.wait(lk, [&] { return done_ == nparts_ - 1; });
        job_ = nullptr;
    }

  private:
    Pool()
    {
        unsigned hw = std::thread::hardware_concurrency();
        const int nw = (int)std::max(0u, std::min(16u, hw ? hw : 1u) - 1u);
        for (int i = 0; i < nw; ++i) workers_.emplace_back([this] { loop(); });
        for (auto &w : workers_) w.detach();   // live until the process ends
    }
    int take()
    {
        std::lock_guard<std::mutex> lk(m_);
        if (!job_ || next_ >= nparts_) return -1;
        return next_++;
    }
    void finish()
    {
        std::lock_guard<std::mutex> lk(m_);
        if (++done_ == nparts_ - 1) cv_done_.notify_all();
    }
    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *job;
            int part;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return gen_ != seen && job_ && next_ < nparts_; });
                seen = gen_;
                job = job_;
                part = next_++;
            }
            (*job)(part);
            finish();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex m_;
    std::condition_variable cv_, cv_done_;
    const std::function<void(int)> *job_ = nullptr;
    int nparts_ = 0, next_ = 0, done_ = 0;
    uint64_t gen_ = 0;
};
}  // namespace

namespace {
struct HostBlocks {
    std::mutex mu;
    std::multimap<size_t, void *> free_blocks;   // exact (rounded) size -> block
    size_t cached = 0;
    static HostBlocks &get()
    {
        static HostBlocks *h = new HostBlocks;   // never destroyed: blocks may come back during exit
        return *h;
    }
};
constexpr size_t kHostCacheMax = size_t(256) << 20;
}  // namespace

void *host_block_get(size_t bytes)
{
    HostBlocks &h = HostBlocks::get();
    {
        std::lock_guard<std::mutex> lk(h.mu);
        auto it = h.free_blocks.find(bytes);
        if (it != h.free_blocks.end()) {
            void *p = it->second;
            h.free_blocks.erase(it);
            h.cached -= bytes;
            return p;
        }
    }
    void *p = std::malloc(bytes);
    if (!p) throw std::bad_alloc();
    return p;
}

void host_block_put(void *p, size_t bytes)
{
    HostBlocks &h = HostBlocks::get();
    {
        std::lock_guard<std::mutex> lk(h.mu);
        if (h.cached + bytes <= kHostCacheMax) {
            h.free_blocks.emplace(bytes, p);
            h.cached += bytes;
            return;
        }
    }
    std::free(p);
}

void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &f)
{
    Pool &pool = Pool::get();
    int64_t nth = std::min<int64_t>(pool.size(), std::max<int64_t>(1, n / std::max<int64_t>(1, grain)));
    if (nth <= 1) {
        f(0, n);
        return;
    }
    std::unique_lock<std::mutex> own(pool.owner, std::try_to_lock);
    if (!own.owns_lock()) {   // pool in use by another caller: run inline
        f(0, n);
        return;
    }
    pool.run((int)nth, [&](int part) { f(n * part / nth, n * (part + 1) / nth); });
}

bem_status mesh_prepare(MeshData &m, int64_t strip_tiles)
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
    // closed, consistently oriented: every directed edge once, its reverse
    // present.  Directed edges are listed per start vertex (counting sort);
    // both conditions are checked inside the short lists of the two ends.
    {
        std::vector<int32_t> optr(nv + 1, 0), oto(3 * nt);
        for (int64_t t = 0; t < nt; ++t)
            for (int a = 0; a < 3; ++a) {
                if (T[3 * t + a] == T[3 * t + (a + 1) % 3])
                    return set_error(BEM_E_MESH, "repeated vertex in a triangle");
                optr[T[3 * t + a] + 1]++;
            }
        for (int64_t v = 0; v < nv; ++v) optr[v + 1] += optr[v];
        {
            std::vector<int32_t> fill(optr.begin(), optr.end() - 1);
            for (int64_t t = 0; t < nt; ++t)
                for (int a = 0; a < 3; ++a) oto[fill[T[3 * t + a]]++] = T[3 * t + (a + 1) % 3];
        }
        bool dup = false, open = false;
        for (int64_t u = 0; u < nv && !dup; ++u)
            for (int32_t q = optr[u]; q < optr[u + 1]; ++q) {
                const int32_t w = oto[q];
                for (int32_t q2 = optr[u]; q2 < q; ++q2) dup = dup || oto[q2] == w;
                bool back = false;
                for (int32_t q2 = optr[w]; q2 < optr[w + 1]; ++q2) back = back || oto[q2] == (int32_t)u;
                open = open || !back;
            }
        if (dup) return set_error(BEM_E_MESH, "edge used twice with the same orientation (non-manifold or flipped)");
        if (open) return set_error(BEM_E_MESH, "mesh is not closed or not consistently oriented");
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
    // by code, equal codes by triangle: a stable LSD radix sort of the
    // 63-bit codes (7 passes of 9 bits) over the triangles in index order
    {
        std::vector<std::pair<uint64_t, int32_t>> tmp(nt);
        std::vector<int64_t> cnt(513);
        for (int shift = 0; shift < 63; shift += 9) {
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t t = 0; t < nt; ++t) cnt[((key[t].first >> shift) & 511) + 1]++;
            if (cnt[1 + ((key[0].first >> shift) & 511)] == nt) continue;   // one digit value: order unchanged
            for (int d = 0; d < 512; ++d) cnt[d + 1] += cnt[d];
            for (int64_t t = 0; t < nt; ++t) tmp[cnt[(key[t].first >> shift) & 511]++] = key[t];
            key.swap(tmp);
        }
    }

    // ---- blocks (<= BT triangles, <= SMAX vertices) and internal vertex numbering
    m.int_of_v.assign(nv, -1);
    m.v_of_int.clear();
    m.v_of_int.reserve(nv);
    m.tri.assign(3 * nt, 0);
    m.blk_start.clear();
    int32_t cur_n = 0, cur_nv = 0, blk = -1;
    std::vector<int32_t> in_blk(nv, -1);   // the last block a vertex was counted in
    for (int64_t s = 0; s < nt; ++s) {
        int32_t t = key[s].second;
        int newv = 0;   // vertices of t not yet in the current block (a triangle's three are distinct)
        for (int a = 0; a < 3; ++a) newv += in_blk[T[3 * t + a]] != blk;
        if (cur_n == 0 || cur_n == BT || cur_nv + newv > SMAX) {
            m.blk_start.push_back((int32_t)s);
            cur_n = 0;
            cur_nv = 0;
            ++blk;
        }
        for (int a = 0; a < 3; ++a) {
            int32_t u = T[3 * t + a];
            if (in_blk[u] != blk) { in_blk[u] = blk; ++cur_nv; }
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
    m.slot_off.assign((size_t)nb * SLOT_OFF_LD, 0);
    m.slot_rank.assign((size_t)nb * 3 * BT, 0);
    m.memb_ptr.assign(nv + 1, 0);
    // blocks are independent (each writes only its own slot tables): in parallel
    std::atomic<int> slot_err{0};   // 1: vertex overflow, 2: valence
    parallel_for(nb, 16, [&](int64_t b0, int64_t b1) {
        int32_t vs[3 * BT];
        for (int64_t b = b0; b < b1; ++b) {
            int nvs = 0;
            for (int32_t t = m.blk_start[b]; t < m.blk_start[b + 1]; ++t)
                for (int a = 0; a < 3; ++a) vs[nvs++] = m.tri[3 * t + a];
            std::sort(vs, vs + nvs);
            nvs = (int)(std::unique(vs, vs + nvs) - vs);
            if (nvs > SMAX) { slot_err = 1; return; }
            m.blk_nslot[b] = nvs;
            for (int q = 0; q < nvs; ++q) m.blk_slots[(size_t)b * SMAX + q] = vs[q];
            for (int32_t t = m.blk_start[b]; t < m.blk_start[b + 1]; ++t)
                for (int a = 0; a < 3; ++a) {
                    const int q = (int)(std::lower_bound(vs, vs + nvs, m.tri[3 * t + a]) - vs);
                    uint8_t &cnt = m.slot_cnt[(size_t)b * SMAX + q];
                    if (cnt >= LMAX) { slot_err = 2; return; }
                    m.slot_ent[((size_t)b * SMAX + q) * LMAX + cnt] = (uint8_t)((t - m.blk_start[b]) * 3 + a);
                    ++cnt;
                }
            int off = 0;
            for (int q = 0; q < nvs; ++q) {
                m.slot_off[(size_t)b * SLOT_OFF_LD + q] = (uint8_t)off;
                for (int v = 0; v < m.slot_cnt[(size_t)b * SMAX + q]; ++v)
                    m.slot_rank[(size_t)b * 3 * BT + m.slot_ent[((size_t)b * SMAX + q) * LMAX + v]] = (uint8_t)(off + v);
                off += m.slot_cnt[(size_t)b * SMAX + q];
            }
            m.slot_off[(size_t)b * SLOT_OFF_LD + nvs] = (uint8_t)off;
        }
    });
    if (slot_err == 1) return set_error(BEM_E_MESH, "internal: block vertex overflow");
    if (slot_err == 2) return set_error(BEM_E_MESH, "vertex valence too high (> 12 corners in one block)");
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < m.blk_nslot[b]; ++q) m.memb_ptr[m.blk_slots[(size_t)b * SMAX + q] + 1]++;
    // vertex -> (block, slot) memberships, blocks ascending
    for (int64_t v = 0; v < nv; ++v) m.memb_ptr[v + 1] += m.memb_ptr[v];
    m.memb.resize(m.memb_ptr[nv]);
    {
        std::vector<int32_t> mfill(m.memb_ptr.begin(), m.memb_ptr.end() - 1);
        for (int b = 0; b < nb; ++b)
            for (int s = 0; s < m.blk_nslot[b]; ++s) m.memb[mfill[m.blk_slots[(size_t)b * SMAX + s]]++] = b << 8 | s;
    }

    // ---- assembly strips: consecutive tile rows b (tiles (b, b2), b2 >= b: nb - b of them) up to
    // strip_tiles tiles, the vertices each strip's tiles reach as rows, and the first vertex that
    // can receive a contribution from the strip (its last membership at or after the strip's first block)
    m.strip_b.assign(1, 0);
    for (int b = 0; b < nb;) {
        int64_t tiles = 0;
        int e = b;
        while (e < nb && (e == b || tiles + (nb - e) <= strip_tiles)) tiles += nb - e++;
        m.strip_b.push_back(e);
        b = e;
    }
    const int ns = (int)m.strip_b.size() - 1;
    m.strip_rptr.assign(1, 0);
    m.strip_rows.clear();
    m.strip_lo.assign(ns, (int32_t)nv);
    {
        // each strip's rows ascending: stamp the slots of its blocks, then scan the stamped range
        std::vector<int32_t> stamp(nv, -1);
        for (int s = 0; s < ns; ++s) {
            int32_t vlo = (int32_t)nv, vhi = -1;
            for (int b = m.strip_b[s]; b < m.strip_b[s + 1]; ++b)
                for (int q = 0; q < m.blk_nslot[b]; ++q) {
                    const int32_t v = m.blk_slots[(size_t)b * SMAX + q];
                    stamp[v] = s;
                    vlo = std::min(vlo, v);
                    vhi = std::max(vhi, v);
                }
            for (int32_t v = vlo; v <= vhi; ++v)
                if (stamp[v] == s) m.strip_rows.push_back(v);
            m.strip_rptr.push_back((int32_t)m.strip_rows.size());
        }
        // strip_lo: strips in ascending first block, so one pass per vertex over the strips it reaches
        for (int64_t v = 0; v < nv; ++v) {
            const int maxb = m.memb[m.memb_ptr[v + 1] - 1] >> 8;
            for (int s = 0; s < ns && m.strip_b[s] <= maxb; ++s)
                if (m.strip_lo[s] > v) m.strip_lo[s] = (int32_t)v;
        }
    }

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

    // ---- ordered singular pairs, kinds 3 / 2 / 1, corner permutations.
    // Kind-major order, within a kind by test triangle t, for each t in the
    // order its vertex stars list the trial triangles.  Chunks of t in
    // parallel, concatenated in t order.
    std::vector<int32_t> pcnt[4];   // pcnt[k][t]: first pair of kind k and test triangle t, within kind k
    for (int k = 1; k <= 3; ++k) pcnt[k].assign(nt + 1, 0);
    auto pairs_of = [&](int64_t t, std::vector<int64_t> &seen_by, auto &&emit) {
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
                emit(ns, sp);
            }
        }
    };
    // two passes over chunks of test triangles in parallel: count the pairs of
    // each (kind, t), then write them at their final places (no staging lists)
    const int64_t nchunk_t = std::min<int64_t>(nt, 128);
    parallel_for(nchunk_t, 1, [&](int64_t c0, int64_t c1) {
        std::vector<int64_t> seen_by(nt, -1);
        for (int64_t c = c0; c < c1; ++c)
            for (int64_t t = nt * c / nchunk_t; t < nt * (c + 1) / nchunk_t; ++t)
                pairs_of(t, seen_by, [&](int k, const SingPair &) { pcnt[k][t + 1]++; });
    });
    int64_t kbase[4] = {0, 0, 0, 0};
    {
        int64_t acc = 0;
        for (int k = 3; k >= 1; --k) {
            for (int64_t t = 0; t < nt; ++t) pcnt[k][t + 1] += pcnt[k][t];
            kbase[k] = acc;
            m.nsing_kind[k] = pcnt[k][nt];
            acc += pcnt[k][nt];
        }
        m.sing.resize((size_t)acc);
    }
    parallel_for(nchunk_t, 1, [&](int64_t c0, int64_t c1) {
        std::vector<int64_t> seen_by(nt, -1);
        for (int64_t c = c0; c < c1; ++c)
            for (int64_t t = nt * c / nchunk_t; t < nt * (c + 1) / nchunk_t; ++t) {
                int64_t at[4] = {0, kbase[1] + pcnt[1][t], kbase[2] + pcnt[2][t], kbase[3] + pcnt[3][t]};
                pairs_of(t, seen_by, [&](int k, const SingPair &sp) { m.sing[at[k]++] = sp; });
            }
    });

    // ---- near entries: unique (i, j) touched by singular pairs, contributions in pair order.
    // Row i collects, kind by kind and triangle by triangle of its star (the
    // global pair order restricted to the row), the 3 entries (i, j) of every
    // pair whose test triangle holds i; columns are numbered by first
    // appearance.  Two parallel passes over the rows: count each row's
    // columns and contributions, then write them at their final places.
    {
        const size_t nc = m.sing.size() * 9;
        auto row_entries = [&](int64_t i, std::vector<std::pair<int32_t, int32_t>> &out) {
            out.clear();
            for (int k = 3; k >= 1; --k)
                for (int32_t e = m.star_ptr[i]; e < m.star_ptr[i + 1]; ++e) {
                    const int32_t t = m.star_ent[e] / 3, a = m.star_ent[e] - 3 * (m.star_ent[e] / 3);
                    for (int64_t p = kbase[k] + pcnt[k][t]; p < kbase[k] + pcnt[k][t + 1]; ++p)
                        for (int b = 0; b < 3; ++b)
                            out.push_back({m.tri[3 * m.sing[p].sig + b], (int32_t)(p * 9 + a * 3 + b)});
                }
        };
        std::vector<int64_t> src_row(nv + 1, 0);   // first contribution of each row
        m.near_row.assign(nv + 1, 0);
        parallel_for(nv, 256, [&](int64_t r0, int64_t r1) {
            std::vector<int32_t> mark(nv, -1);
            std::vector<std::pair<int32_t, int32_t>> ent;
            for (int64_t i = r0; i < r1; ++i) {
                row_entries(i, ent);
                int32_t u = 0;
                for (const auto &e : ent)
                    if (mark[e.first] != (int32_t)i) { mark[e.first] = (int32_t)i; ++u; }
                m.near_row[i + 1] = u;
                src_row[i + 1] = (int64_t)ent.size();
            }
        });
        for (int64_t v = 0; v < nv; ++v) {
            m.near_row[v + 1] += m.near_row[v];
            src_row[v + 1] += src_row[v];
        }
        if ((size_t)src_row[nv] != nc) return set_error(BEM_E_MESH, "internal: singular contribution count");
        const size_t nent = (size_t)m.near_row[nv];
        m.near_i.resize(nent);
        m.near_j.resize(nent);
        m.near_ptr.resize(nent + 1);
        m.near_src.resize(nc);
        parallel_for(nv, 256, [&](int64_t r0, int64_t r1) {
            std::vector<int32_t> mark(nv, -1), slot_of(nv, 0), off;
            std::vector<std::pair<int32_t, int32_t>> ent;
            for (int64_t i = r0; i < r1; ++i) {
                row_entries(i, ent);
                const int64_t e0 = m.near_row[i];
                int32_t u = 0;
                for (const auto &e : ent) {   // columns by first appearance, with their contribution counts
                    const int32_t j = e.first;
                    if (mark[j] != (int32_t)i) {
                        mark[j] = (int32_t)i;
                        slot_of[j] = u;
                        m.near_i[e0 + u] = (int32_t)i;
                        m.near_j[e0 + u] = j;
                        m.near_ptr[e0 + u] = 0;
                        ++u;
                    }
                    m.near_ptr[e0 + slot_of[j]]++;
                }
                off.resize(u);
                int32_t acc = (int32_t)src_row[i];
                for (int32_t q = 0; q < u; ++q) {
                    const int32_t c = m.near_ptr[e0 + q];
                    m.near_ptr[e0 + q] = acc;
                    off[q] = acc;
                    acc += c;
                }
                for (const auto &e : ent) m.near_src[off[slot_of[e.first]]++] = e.second;
            }
        });
        m.near_ptr[nent] = (int32_t)nc;
    }
    return BEM_OK;
}

}  // namespace bemtx
