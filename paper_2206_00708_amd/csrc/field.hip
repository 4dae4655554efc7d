// Field off the surface and winding numbers of a mesh.
//
// Field (Sec. 2, Eq. "representation"): outside the body the total field is
// the incident plane wave plus [SLP_ext psi_ext - DLP_ext phi_ext](x), inside
// it is [SLP_int psi_int - DLP_int phi_int](x), with
//   [SLP psi](x) = int G(x, y) psi(y) dy,  [DLP phi](x) = int dG/dn(y) phi(y) dy,
//   G = exp(i k r) / (4 pi r),  dG/dn(y) = exp(i k r) (i k r - 1) ((y - x).n_y) / (4 pi r^3).
// The potentials are the P1 functions of the solve's unknowns: with the
// multiple-traces system as printed (Sec. 3.3) p = -v and dp/dn = -w on each
// mesh, so phi_ext = v_ext, psi_ext = w_ext (phi_ext = -gamma_D p,
// psi_ext = -gamma_N p, Eq. "potentials:traces") and phi_int = -v_int,
// psi_int = -w_int.  Each triangle integral is the 6-point rule of the
// regular assembly; points near a mesh get that rule's nearly-singular error.
//
//   field_density_kernel   per triangle: area * weight * density at the six
//                          quadrature points (P1 interpolation), both
//                          potentials, with their signs.
//   field_partial_kernel   one thread per point (sorted by region), one
//                          workgroup per (256 points, chunk of triangles);
//                          triangles staged in LDS 128 at a time and read by
//                          every lane at once (broadcast); FP64 throughout;
//                          per-chunk partial sums.
//   field_combine_kernel   fixed-order sum of the chunk partials, 1 / (4 pi),
//                          the incident wave for exterior points, written at
//                          the point's place in the caller's order.
//   winding kernels        sum over triangles of the signed solid angle
//                          (Van Oosterom and Strackee, 1983) over 4 pi, the
//                          same chunked structure: 1 inside a closed outward
//                          mesh, 0 outside.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "phase.h"
#include "rule6.h"

namespace bemtx {

namespace {

constexpr int FLD_PB = 256;   // points per workgroup
constexpr int FLD_TS = 128;   // triangles staged in LDS at a time
constexpr int FLD_WG = 2048;  // target workgroups per launch (points x triangle chunks)

struct alignas(16) FieldTri {
    double y[6][3];     // quadrature points
    double n[3];        // unit normal
    double pad;
    double2 phi[6];     // area * w_q * phi(y_q) (sign folded in)
    double2 psi[6];     // area * w_q * psi(y_q)
};
static_assert(sizeof(FieldTri) % 16 == 0, "FieldTri stages as 16-byte words");

__global__ __launch_bounds__(256) void field_permute_kernel(int nv, const int32_t *__restrict__ perm,
                                                            const double2 *__restrict__ src, double2 *__restrict__ dst)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;   // caller vertex
    if (c < nv) dst[perm[c]] = src[c];
}

__global__ __launch_bounds__(256) void field_density_kernel(int nt, const TriGeo *__restrict__ geo,
                                                            const int32_t *__restrict__ tri,
                                                            const double2 *__restrict__ phi,
                                                            const double2 *__restrict__ psi, double sgn,
                                                            FieldTri *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const TriGeo &g = geo[t];
    FieldTri f;
    double2 ph[3], ps[3];
    for (int a = 0; a < 3; ++a) {
        ph[a] = phi[tri[3 * t + a]];
        ps[a] = psi[tri[3 * t + a]];
    }
    for (int q = 0; q < 6; ++q) {
        for (int c = 0; c < 3; ++c) f.y[q][c] = g.qp[q][c];
        const double W = sgn * g.area * r6_w(q);
        double pr = 0, pi = 0, sr = 0, si = 0;
        for (int a = 0; a < 3; ++a) {
            const double b = r6_bary(q, a);
            pr += b * ph[a].x; pi += b * ph[a].y;
            sr += b * ps[a].x; si += b * ps[a].y;
        }
        f.phi[q] = make_double2(W * pr, W * pi);
        f.psi[q] = make_double2(W * sr, W * si);
    }
    for (int c = 0; c < 3; ++c) f.n[c] = g.n[c];
    f.pad = 0.0;
    out[t] = f;
}

// part[chunk][i] = sum over the chunk's triangles and quadrature points of
// G psi - dG/dn phi at point i, times 4 pi (the factor is applied once in
// the combine).
// CK: complex wavenumber k + i kim (absorbing medium), G = exp(i k r - kim r) / (4 pi r).
template <bool CK>
__global__ __launch_bounds__(FLD_PB) void field_partial_kernel(int np, const double *__restrict__ pts, int nt, int tpc,
                                                               const FieldTri *__restrict__ ft, double k, double kim,
                                                               double2 *__restrict__ part)
{
    __shared__ FieldTri sh[FLD_TS];
    const int chunk = blockIdx.y;
    const int t0 = chunk * tpc, t1 = min(nt, t0 + tpc);
    const int i = blockIdx.x * FLD_PB + threadIdx.x;
    const bool live = i < np;
    const double x0 = live ? pts[3 * i] : 0.0, x1 = live ? pts[3 * i + 1] : 0.0, x2 = live ? pts[3 * i + 2] : 0.0;
    double ar = 0.0, ai = 0.0;
    for (int s0 = t0; s0 < t1; s0 += FLD_TS) {
        const int ns = min(FLD_TS, t1 - s0);
        __syncthreads();   // the previous batch is no longer read
        {
            const double2 *src = reinterpret_cast<const double2 *>(ft + s0);
            double2 *dst = reinterpret_cast<double2 *>(sh);
            const int words = ns * (int)(sizeof(FieldTri) / sizeof(double2));
            for (int w = threadIdx.x; w < words; w += FLD_PB) dst[w] = src[w];
        }
        __syncthreads();
        if (live)
            for (int t = 0; t < ns; ++t) {
                const FieldTri &f = sh[t];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const double d0 = f.y[q][0] - x0, d1 = f.y[q][1] - x1, d2 = f.y[q][2] - x2;   // y - x
                    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    const double rinv = rsqrt(r2);
                    const double kr = k * (r2 * rinv);
                    double sn, cs;
                    phase_sincos(kr, &sn, &cs);
                    double gr = cs * rinv, gi = sn * rinv;                           // exp(ikr) / r
                    const double s = (d0 * f.n[0] + d1 * f.n[1] + d2 * f.n[2]) * rinv * rinv;
                    double fr, fi;                                                   // exp(ikr)(ikr - 1)(y-x).n / r^3
                    if constexpr (CK) {
                        const double r = r2 * rinv, dmp = exp(-kim * r), am = -1.0 - kim * r;
                        gr *= dmp; gi *= dmp;
                        fr = (gr * am - gi * kr) * s;
                        fi = (gr * kr + gi * am) * s;
                    } else {
                        fr = (-gr - gi * kr) * s;
                        fi = (gr * kr - gi) * s;
                    }
                    const double2 ps = f.psi[q], ph = f.phi[q];
                    ar += gr * ps.x - gi * ps.y - (fr * ph.x - fi * ph.y);
                    ai += gr * ps.y + gi * ps.x - (fr * ph.y + fi * ph.x);
                }
            }
    }
    if (live) part[(int64_t)chunk * np + i] = make_double2(ar, ai);
}

__global__ __launch_bounds__(256) void field_combine_kernel(int np, int nchunk, const double2 *__restrict__ part,
                                                            const double *__restrict__ pts,
                                                            const int32_t *__restrict__ dst_index, int add_incident,
                                                            int kind, double k, double d0, double d1, double d2,
                                                            double2 *__restrict__ field)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        const double2 v = part[(int64_t)c * np + i];
        sr += v.x;
        si += v.y;
    }
    sr *= kInv4Pi;
    si *= kInv4Pi;
    if (add_incident && kind == 0) {   // plane wave exp(i k d.x)
        double sn, cs;
        phase_sincos(k * (d0 * pts[3 * i] + d1 * pts[3 * i + 1] + d2 * pts[3 * i + 2]), &sn, &cs);
        sr += cs;
        si += sn;
    } else if (add_incident) {         // point source exp(i k r) / (4 pi r), r = |x - x0|
        const double R0 = pts[3 * i] - d0, R1 = pts[3 * i + 1] - d1, R2 = pts[3 * i + 2] - d2;
        const double r = sqrt(R0 * R0 + R1 * R1 + R2 * R2);
        double sn, cs;
        phase_sincos(k * r, &sn, &cs);
        sr += cs * kInv4Pi / r;
        si += sn * kInv4Pi / r;
    }
    field[dst_index[i]] = make_double2(sr, si);
}

__global__ __launch_bounds__(FLD_PB) void winding_partial_kernel(int np, const double *__restrict__ pts, int nt,
                                                                 int tpc, const TriGeo *__restrict__ geo,
                                                                 double *__restrict__ part)
{
    __shared__ double sv[FLD_TS][9];
    const int chunk = blockIdx.y;
    const int t0 = chunk * tpc, t1 = min(nt, t0 + tpc);
    const int i = blockIdx.x * FLD_PB + threadIdx.x;
    const bool live = i < np;
    const double x0 = live ? pts[3 * i] : 0.0, x1 = live ? pts[3 * i + 1] : 0.0, x2 = live ? pts[3 * i + 2] : 0.0;
    double acc = 0.0;
    for (int s0 = t0; s0 < t1; s0 += FLD_TS) {
        const int ns = min(FLD_TS, t1 - s0);
        __syncthreads();
        for (int w = threadIdx.x; w < ns * 9; w += FLD_PB) sv[w / 9][w % 9] = geo[s0 + w / 9].p[(w % 9) / 3][w % 3];
        __syncthreads();
        if (live)
            for (int t = 0; t < ns; ++t) {
                const double *v = sv[t];
                const double a0 = v[0] - x0, a1 = v[1] - x1, a2 = v[2] - x2;
                const double b0 = v[3] - x0, b1 = v[4] - x1, b2 = v[5] - x2;
                const double c0 = v[6] - x0, c1 = v[7] - x1, c2 = v[8] - x2;
                const double la = sqrt(a0 * a0 + a1 * a1 + a2 * a2), lb = sqrt(b0 * b0 + b1 * b1 + b2 * b2),
                             lc = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
                const double num = a0 * (b1 * c2 - b2 * c1) + a1 * (b2 * c0 - b0 * c2) + a2 * (b0 * c1 - b1 * c0);
                const double den = la * lb * lc + (a0 * b0 + a1 * b1 + a2 * b2) * lc + (a0 * c0 + a1 * c1 + a2 * c2) * lb +
                                   (b0 * c0 + b1 * c1 + b2 * c2) * la;
                acc += 2.0 * atan2(num, den);
            }
    }
    if (live) part[(int64_t)chunk * np + i] = acc;
}

__global__ __launch_bounds__(256) void winding_combine_kernel(int np, int nchunk, const double *__restrict__ part,
                                                              double *__restrict__ w)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * np + i];
    w[i] = s * kInv4Pi;
}

// triangle chunks for np points: about FLD_WG workgroups, at least FLD_TS
// triangles per chunk
void chunking(int64_t np, int nt, int &nchunk, int &tpc)
{
    const int64_t pblocks = (np + FLD_PB - 1) / FLD_PB;
    const int64_t maxc = std::max<int64_t>(1, (nt + FLD_TS - 1) / FLD_TS);
    nchunk = (int)std::min<int64_t>(maxc, std::max<int64_t>(1, FLD_WG / std::max<int64_t>(1, pblocks)));
    tpc = (nt + nchunk - 1) / nchunk;
    nchunk = (nt + tpc - 1) / tpc;
}

}  // namespace

size_t field_scratch_bytes(int64_t np, int nt)
{
    int nchunk, tpc;
    chunking(np, nt, nchunk, tpc);
    return (size_t)nchunk * (size_t)np * sizeof(double2);
}

// Field of one right-hand side at np points of one region (points [np][3]
// and dst_index on the device, sorted by region); x: the unknowns of the
// right-hand side in internal numbering (device).
bem_status launch_field_region(bem_problem *p, int region, int np, const double *pts, const int32_t *dst_index,
                               const double2 *x_int, const double *dir, double2 *field, DevMem &dens, DevMem &part,
                               hipStream_t st)
{
    if (np == 0) return BEM_OK;
    const bem_mesh *m = region == 0 ? p->ext : p->inte;
    const int nt = (int)m->h.nt, ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    const double k = region == 0 ? p->k_ext : p->k_int, kim = region == 0 ? 0.0 : p->k_int_im;
    const double2 *phi = region == 0 ? x_int : x_int + 2 * ne;
    const double2 *psi = region == 0 ? x_int + ne : x_int + 2 * ne + ni;
    bem_status s = dev_alloc(p->ctx, dens, (size_t)nt * sizeof(FieldTri));
    if (s) return s;
    int nchunk, tpc;
    chunking(np, nt, nchunk, tpc);
    s = dev_alloc(p->ctx, part, (size_t)nchunk * np * sizeof(double2));
    if (s) return s;
    hipLaunchKernelGGL(field_density_kernel, dim3((nt + 255) / 256), dim3(256), 0, st, nt, m->d.geo.as<TriGeo>(),
                       m->d.tri.as<int32_t>(), phi, psi, region == 0 ? 1.0 : -1.0, dens.as<FieldTri>());
    BEM_HIP(hipGetLastError());
    {
        KTimer kt(p->ctx, K_FIELD);
        if (kim != 0.0)
            launch_k(kt, field_partial_kernel<true>, dim3((np + FLD_PB - 1) / FLD_PB, nchunk), dim3(FLD_PB), 0, st, np,
                     pts, nt, tpc, dens.as<FieldTri>(), k, kim, part.as<double2>());
        else
            launch_k(kt, field_partial_kernel<false>, dim3((np + FLD_PB - 1) / FLD_PB, nchunk), dim3(FLD_PB), 0, st, np,
                     pts, nt, tpc, dens.as<FieldTri>(), k, kim, part.as<double2>());
        BEM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(field_combine_kernel, dim3((np + 255) / 256), dim3(256), 0, st, np, nchunk,
                       part.as<double2>(), pts, dst_index, region == 0 ? 1 : 0, p->incident, p->k_ext, dir[0], dir[1],
                       dir[2],
                       field);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

bem_status launch_field_permute(bem_problem *p, const double2 *x_caller, double2 *x_int, hipStream_t st)
{
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    const int32_t *pe = p->ext->d.perm.as<int32_t>(), *pi = p->inte->d.perm.as<int32_t>();
    const int nvs[4] = {ne, ne, ni, ni};
    const int32_t *perms[4] = {pe, pe, pi, pi};
    int off = 0;
    for (int b = 0; b < 4; ++b) {
        hipLaunchKernelGGL(field_permute_kernel, dim3((nvs[b] + 255) / 256), dim3(256), 0, st, nvs[b], perms[b],
                           x_caller + off, x_int + off);
        off += nvs[b];
    }
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

bem_status launch_winding(const bem_mesh *m, int np, const double *pts, double *w, DevMem &part, hipStream_t st)
{
    if (np == 0) return BEM_OK;
    const int nt = (int)m->h.nt;
    int nchunk, tpc;
    chunking(np, nt, nchunk, tpc);
    bem_status s = dev_alloc(m->ctx, part, (size_t)nchunk * np * sizeof(double));
    if (s) return s;
    hipLaunchKernelGGL(winding_partial_kernel, dim3((np + FLD_PB - 1) / FLD_PB, nchunk), dim3(FLD_PB), 0, st, np, pts,
                       nt, tpc, m->d.geo.as<TriGeo>(), part.as<double>());
    BEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(winding_combine_kernel, dim3((np + 255) / 256), dim3(256), 0, st, np, nchunk,
                       part.as<double>(), w);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

}  // namespace bemtx
