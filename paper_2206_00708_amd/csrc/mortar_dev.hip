// The L2 mortar matrix P_int,ext (Sec. 3.1) on the device: the central
// projection, clipping and quadrature of every candidate (exterior facet,
// interior triangle) pair run in kernels with the steps of the host assembly
// (mortar_geom.h), the contributions are numbered in the host's facet order,
// and the CSR rows are formed in a kernel with the host grouping's steps and
// summation order, so the matrix is the host assembly's up to the rounding of
// the pair integrals.  The host keeps the candidate grid and the listing of
// the contributions per interior triangle (integer work, O(n)).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "mortar_geom.h"

namespace bemtx {
namespace {

struct MortarDevArgs {
    const double *xi, *xe;          // vertex coordinates [nv][3] of the interior / exterior mesh
    const int32_t *tri_i, *tri_e;   // triangles [nt][3]
    const double *ci, *ri, *ce, *re;
    const int32_t *cell_ptr, *cell_tri;
    int ncell;
    double h;
    int nte;
};

// One wave per exterior facet.  Its candidates are the interior triangles of
// the 27 cells around the facet's cone centre, in the host's order (cells by
// dx, then dy, then dz; ascending triangles within a cell).  The wave walks
// them 64 at a time and keeps the contributing ones in that order (prefix
// counts of a ballot), so no atomics are needed and the output is
// deterministic.  Pass 0 counts the contributions and the coverage defect of
// each facet; pass 1 writes them from the facet's offset.
template <bool FILL>
__global__ __launch_bounds__(256) void mortar_facet_kernel(MortarDevArgs A, int32_t *__restrict__ count,
                                                           const int64_t *__restrict__ offset,
                                                           int32_t *__restrict__ con_ti, double *__restrict__ con_blk,
                                                           double *__restrict__ defect, int32_t *__restrict__ overflow)
{
    const int lane = threadIdx.x & 63;
    const int te = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (te >= A.nte) return;   // whole waves leave; the kernel has no barrier
    const int32_t *ve = A.tri_e + 3 * te;
    const mgeo::Facet F = mgeo::make_facet(A.xe + 3 * ve[0], A.xe + 3 * ve[1], A.xe + 3 * ve[2]);
    const double *cte = A.ce + 3 * te;
    const double rte = A.re[te];
    // lane c < 27 holds cell (dx, dy, dz) = (c / 9, c / 3 % 3, c % 3) - 1
    int cstart = 0, csize = 0;
    if (lane < 27) {
        const int x = mgeo::cell_of(cte[0], A.ncell, A.h) + lane / 9 - 1;
        const int y = mgeo::cell_of(cte[1], A.ncell, A.h) + (lane / 3) % 3 - 1;
        const int z = mgeo::cell_of(cte[2], A.ncell, A.h) + lane % 3 - 1;
        if (x >= 0 && y >= 0 && z >= 0 && x < A.ncell && y < A.ncell && z < A.ncell) {
            const int64_t c = ((int64_t)x * A.ncell + y) * A.ncell + z;
            cstart = A.cell_ptr[c];
            csize = A.cell_ptr[c + 1] - cstart;
        }
    }
    int incl = csize;   // inclusive scan of the cell sizes over lanes 0..31
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    const int excl = incl - csize;
    const int total = __shfl(incl, 26, 64);
    int64_t run = FILL ? offset[te] : 0;
    const int64_t kend = FILL ? offset[te + 1] : 0;   // the count pass's end of this facet
    double covered = 0.0;
    int ovf = 0;
    for (int base = 0; base < total; base += 64) {
        const int f = base + lane;
        // the cell of candidate f: the last cell whose first candidate is at or before f
        int cc = 0;
        for (int c = 1; c < 27; ++c)
            if (f >= __shfl(excl, c, 64)) cc = c;
        const int st = __shfl(cstart, cc, 64), ex = __shfl(excl, cc, 64);
        int ok = 0;
        int32_t ti = -1;
        double blk[3][3], ap = 0.0;
        if (f < total) {
            ti = A.cell_tri[st + (f - ex)];
            if (mgeo::cones_meet(A.ci + 3 * ti, A.ri[ti], cte, rte)) {
                const int32_t *vi = A.tri_i + 3 * ti;
                const int r = mgeo::pair_block(F, A.xi + 3 * vi[0], A.xi + 3 * vi[1], A.xi + 3 * vi[2], blk, &ap);
                if (r < 0) ovf = 1;
                ok = r > 0;
            }
        }
        const uint64_t bal = __ballot(ok);
        if (FILL && ok) {
            const int64_t k = run + __popcll(bal & ((1ull << lane) - 1ull));
            if (k < kend) {   // the two passes take the same decisions; never write past the facet
                con_ti[k] = ti;
#pragma unroll
                for (int e = 0; e < 9; ++e) con_blk[9 * k + e] = blk[e / 3][e % 3];
            }
        }
        run += __popcll(bal);
        if (ok) covered += ap;
    }
    if (FILL) {
        if (lane == 0 && run != kend) overflow[0] = 2;   // the passes disagree: reported, never used
        return;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) covered += __shfl_xor(covered, off, 64);
    const uint64_t anyovf = __ballot(ovf);
    if (lane == 0) {
        count[te] = (int32_t)run;
        defect[te] = fabs(covered - F.area) / F.area;
        if (anyovf) overflow[0] = 1;
    }
}

constexpr int kRowStar = 16;   // triangles around a vertex held by the row kernel
constexpr int kRowCols = 64;   // distinct columns of a row held by the row kernel

// One thread per interior vertex i, a row of P_int,ext, with the steps of the
// host grouping: the contributions of the triangles around i, merged in
// contribution order (each triangle's list is ascending), give 3 entries each
// (the facet's vertices b, the block's row of i's corner a); duplicate columns
// are summed in that order, then the distinct columns are sorted.  Pass 0
// counts the columns, pass 1 writes them at rowptr[i].  A row beyond the
// local buffers sets *flag = 1 (the host then groups the matrix itself); a
// pass 1 that disagrees with pass 0 sets 2 and writes nothing past its row.
constexpr int kRowBlock = 64;   // one wave per workgroup: the few row waves spread over the compute units
template <bool WRITE>
__global__ __launch_bounds__(kRowBlock) void mortar_rows_kernel(int nv, const int32_t *__restrict__ star_ptr,
                                                          const int32_t *__restrict__ star_ent,
                                                          const int32_t *__restrict__ tptr, const int32_t *__restrict__ tcon,
                                                          const int32_t *__restrict__ con_te,
                                                          const int32_t *__restrict__ tri_e,
                                                          const double *__restrict__ con_blk, int32_t *__restrict__ count,
                                                          const int64_t *__restrict__ rowptr, int32_t *__restrict__ col,
                                                          double *__restrict__ val, int32_t *__restrict__ flag)
{
    const int i = blockIdx.x * kRowBlock + threadIdx.x;
    if (i >= nv) return;
    const int s0 = star_ptr[i], ns = star_ptr[i + 1] - s0;
    if (ns > kRowStar) {
        flag[0] = 1;
        return;
    }
    int cur[kRowStar], end[kRowStar], cor[kRowStar];
    for (int q = 0; q < ns; ++q) {
        const int e = star_ent[s0 + q], t = e / 3;
        cor[q] = e - 3 * t;
        cur[q] = tptr[t];
        end[q] = tptr[t + 1];
    }
    int cols[kRowCols];
    double vals[kRowCols];
    int m = 0;
    for (;;) {
        int best = -1, bk = 0x7fffffff;
        for (int q = 0; q < ns; ++q)
            if (cur[q] < end[q]) {
                const int k = tcon[cur[q]];
                if (k < bk) { bk = k; best = q; }
            }
        if (best < 0) break;
        ++cur[best];
        const int te = con_te[bk], a = cor[best];
        for (int b = 0; b < 3; ++b) {
            const int c = tri_e[3 * te + b];
            const double v = con_blk[9 * (int64_t)bk + 3 * a + b];
            int p = -1;
            for (int r = 0; r < m; ++r)
                if (cols[r] == c) { p = r; break; }
            if (p >= 0) {
                vals[p] += v;
            } else {
                if (m >= kRowCols) {
                    flag[0] = 1;
                    return;
                }
                cols[m] = c;
                vals[m] = v;
                ++m;
            }
        }
    }
    for (int r = 1; r < m; ++r) {   // distinct columns, ascending
        const int c = cols[r];
        const double v = vals[r];
        int q = r - 1;
        while (q >= 0 && cols[q] > c) { cols[q + 1] = cols[q]; vals[q + 1] = vals[q]; --q; }
        cols[q + 1] = c;
        vals[q + 1] = v;
    }
    if (!WRITE) {
        count[i] = m;
        return;
    }
    const int64_t o = rowptr[i];
    if (rowptr[i + 1] - o != m) {
        flag[0] = 2;
        return;
    }
    for (int r = 0; r < m; ++r) { col[o + r] = cols[r]; val[o + r] = vals[r]; }
}

template <class V>
bem_status upload_vec(bem_ctx *ctx, DevMem &m, const V &v, hipStream_t st)
{
    using T = typename V::value_type;
    bem_status s = dev_alloc(ctx, m, std::max<size_t>(1, v.size()) * sizeof(T), st);
    if (s) return s;
    if (!v.empty()) BEM_HIP(hipMemcpyAsync(m.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return BEM_OK;
}

}  // namespace

bem_status mortar_csr_device(bem_ctx *ctx, const bem_mesh *mi, const bem_mesh *me, hipStream_t st, Csr &P,
                             double *coverage_defect)
{
    MortarGrid g;
    mortar_grid(mi->h, me->h, g);
    const int nte = (int)me->h.nt;
    DevMem d_ci, d_ri, d_ce, d_re, d_cptr, d_ctri, d_count, d_off, d_def, d_ovf, d_ti, d_blk;
    bem_status s = upload_vec(ctx, d_ci, g.ci, st);
    if (!s) s = upload_vec(ctx, d_ri, g.ri, st);
    if (!s) s = upload_vec(ctx, d_ce, g.ce, st);
    if (!s) s = upload_vec(ctx, d_re, g.re, st);
    if (!s) s = upload_vec(ctx, d_cptr, g.cell_ptr, st);
    if (!s) s = upload_vec(ctx, d_ctri, g.cell_tri, st);
    if (!s) s = dev_alloc(ctx, d_count, (size_t)nte * sizeof(int32_t), st);
    if (!s) s = dev_alloc(ctx, d_def, (size_t)nte * sizeof(double), st);
    if (!s) s = dev_alloc(ctx, d_ovf, sizeof(int32_t), st);
    if (!s) s = dev_alloc(ctx, d_off, ((size_t)nte + 1) * sizeof(int64_t), st);
    if (s) return s;
    MortarDevArgs A;
    A.xi = mi->d.xyz.as<double>();
    A.xe = me->d.xyz.as<double>();
    A.tri_i = mi->d.tri.as<int32_t>();
    A.tri_e = me->d.tri.as<int32_t>();
    A.ci = d_ci.as<double>();
    A.ri = d_ri.as<double>();
    A.ce = d_ce.as<double>();
    A.re = d_re.as<double>();
    A.cell_ptr = d_cptr.as<int32_t>();
    A.cell_tri = d_ctri.as<int32_t>();
    A.ncell = g.ncell;
    A.h = g.h;
    A.nte = nte;
    const dim3 grid((unsigned)((nte + 3) / 4));
    // the overflow flag is cleared by a copy (no memset node in code a caller may capture)
    const int32_t zero = 0;
    BEM_HIP(hipMemcpyAsync(d_ovf.ptr, &zero, sizeof zero, hipMemcpyHostToDevice, st));
    {
        KTimer kt(ctx, K_MORTAR);
        launch_k(kt, mortar_facet_kernel<false>, grid, dim3(256), 0, st, A, d_count.as<int32_t>(),
                 (const int64_t *)nullptr, (int32_t *)nullptr, (double *)nullptr, d_def.as<double>(), d_ovf.as<int32_t>());
        BEM_HIP(hipGetLastError());
    }
    std::vector<int32_t> cnt(nte);
    std::vector<double> def(nte);
    int32_t ovf = 0;
    BEM_HIP(hipMemcpyAsync(cnt.data(), d_count.ptr, (size_t)nte * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BEM_HIP(hipMemcpyAsync(def.data(), d_def.ptr, (size_t)nte * sizeof(double), hipMemcpyDeviceToHost, st));
    BEM_HIP(hipMemcpyAsync(&ovf, d_ovf.ptr, sizeof ovf, hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    if (ovf) return set_error(BEM_E_MESH, "degenerate facet intersection in the mortar projection");
    std::vector<int64_t> off(nte + 1, 0);
    for (int t = 0; t < nte; ++t) off[t + 1] = off[t] + cnt[t];
    const int64_t ncon = off[nte];
    if (ncon > INT32_MAX) return set_error(BEM_E_UNSUPPORTED, "too many mortar contributions");
    HVec<int32_t> ti(ncon), te(ncon);
    if (ncon > 0) {
        s = upload_vec(ctx, d_off, off, st);
        if (!s) s = dev_alloc(ctx, d_ti, (size_t)ncon * sizeof(int32_t), st);
        if (!s) s = dev_alloc(ctx, d_blk, (size_t)ncon * 9 * sizeof(double), st);
        if (s) return s;
        {
            KTimer kt(ctx, K_MORTAR);
            launch_k(kt, mortar_facet_kernel<true>, grid, dim3(256), 0, st, A, (int32_t *)nullptr,
                     d_off.as<int64_t>(), d_ti.as<int32_t>(), d_blk.as<double>(), (double *)nullptr, d_ovf.as<int32_t>());
            BEM_HIP(hipGetLastError());
        }
        BEM_HIP(hipMemcpyAsync(ti.data(), d_ti.ptr, (size_t)ncon * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        BEM_HIP(hipMemcpyAsync(&ovf, d_ovf.ptr, sizeof ovf, hipMemcpyDeviceToHost, st));
        BEM_HIP(hipStreamSynchronize(st));
        if (ovf) return set_error(BEM_E_DEVICE, "mortar passes disagree on the contributions");
    }
    for (int t = 0; t < nte; ++t)
        for (int64_t k = off[t]; k < off[t + 1]; ++k) te[k] = t;
    double worst = 0.0;
    for (double d : def) worst = std::max(worst, d);
    if (coverage_defect) *coverage_defect = worst;
    if (worst > 1e-6)
        return set_error(BEM_E_MESH_MISMATCH, "projected interior mesh leaves an exterior facet uncovered (relative defect " +
                                                  std::to_string(worst) + ")");
    // rows on the device: the contributions listed per interior triangle (a
    // counting sort on the host, O(contributions)), then the row kernel
    const int64_t nti = mi->h.nt, nvi = mi->h.nv;
    HVec<int32_t> tptr(nti + 1, 0), tcon(std::max<int64_t>(1, ncon));
    for (int64_t k = 0; k < ncon; ++k) tptr[ti[k] + 1]++;
    for (int64_t t = 0; t < nti; ++t) tptr[t + 1] += tptr[t];
    {
        std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
        for (int64_t k = 0; k < ncon; ++k) tcon[fill[ti[k]]++] = (int32_t)k;
    }
    DevMem d_te, d_tptr, d_tcon, d_rcnt, d_rptr, d_col, d_val;
    s = upload_vec(ctx, d_te, te, st);
    if (!s) s = upload_vec(ctx, d_tptr, tptr, st);
    if (!s) s = upload_vec(ctx, d_tcon, tcon, st);
    if (!s) s = dev_alloc(ctx, d_rcnt, (size_t)nvi * sizeof(int32_t), st);
    if (s) return s;
    const double *blk_dev = ncon > 0 ? d_blk.as<double>() : nullptr;
    const dim3 rgrid((unsigned)((nvi + kRowBlock - 1) / kRowBlock));
    {
        KTimer kt(ctx, K_MORTAR);
        launch_k(kt, mortar_rows_kernel<false>, rgrid, dim3(kRowBlock), 0, st, (int)nvi, mi->d.star_ptr.as<int32_t>(),
                 mi->d.star_ent.as<int32_t>(), d_tptr.as<int32_t>(), d_tcon.as<int32_t>(), d_te.as<int32_t>(),
                 me->d.tri.as<int32_t>(), blk_dev, d_rcnt.as<int32_t>(), (const int64_t *)nullptr, (int32_t *)nullptr,
                 (double *)nullptr, d_ovf.as<int32_t>());
        BEM_HIP(hipGetLastError());
    }
    std::vector<int32_t> rcnt(nvi);
    BEM_HIP(hipMemcpyAsync(rcnt.data(), d_rcnt.ptr, (size_t)nvi * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BEM_HIP(hipMemcpyAsync(&ovf, d_ovf.ptr, sizeof ovf, hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    if (ovf) {   // a row beyond the kernel's buffers: the host groups the contributions
        HVec<double> blk(9 * ncon);
        if (ncon > 0) {
            BEM_HIP(hipMemcpyAsync(blk.data(), d_blk.ptr, (size_t)ncon * 9 * sizeof(double), hipMemcpyDeviceToHost, st));
            BEM_HIP(hipStreamSynchronize(st));
        }
        return mortar_from_contribs(mi->h, me->h, ncon, ti.data(), te.data(), blk.data(), worst, P);
    }
    std::vector<int64_t> rptr(nvi + 1, 0);
    for (int64_t r = 0; r < nvi; ++r) rptr[r + 1] = rptr[r] + rcnt[r];
    const int64_t nnz = rptr[nvi];
    if (nnz > INT32_MAX) return set_error(BEM_E_UNSUPPORTED, "too many mortar nonzeros");
    s = upload_vec(ctx, d_rptr, rptr, st);
    if (!s) s = dev_alloc(ctx, d_col, std::max<int64_t>(1, nnz) * sizeof(int32_t), st);
    if (!s) s = dev_alloc(ctx, d_val, std::max<int64_t>(1, nnz) * sizeof(double), st);
    if (s) return s;
    {
        KTimer kt(ctx, K_MORTAR);
        launch_k(kt, mortar_rows_kernel<true>, rgrid, dim3(kRowBlock), 0, st, (int)nvi, mi->d.star_ptr.as<int32_t>(),
                 mi->d.star_ent.as<int32_t>(), d_tptr.as<int32_t>(), d_tcon.as<int32_t>(), d_te.as<int32_t>(),
                 me->d.tri.as<int32_t>(), blk_dev, (int32_t *)nullptr, d_rptr.as<int64_t>(), d_col.as<int32_t>(),
                 d_val.as<double>(), d_ovf.as<int32_t>());
        BEM_HIP(hipGetLastError());
    }
    P.nrows = nvi;
    P.ncols = me->h.nv;
    P.ptr.resize(nvi + 1);
    for (int64_t r = 0; r <= nvi; ++r) P.ptr[r] = (int32_t)rptr[r];
    P.col.resize(nnz);
    P.val.resize(nnz);
    if (nnz > 0) {
        BEM_HIP(hipMemcpyAsync(P.col.data(), d_col.ptr, (size_t)nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        BEM_HIP(hipMemcpyAsync(P.val.data(), d_val.ptr, (size_t)nnz * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    BEM_HIP(hipMemcpyAsync(&ovf, d_ovf.ptr, sizeof ovf, hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    if (ovf) return set_error(BEM_E_DEVICE, "mortar row passes disagree");
    return BEM_OK;
}

}  // namespace bemtx
