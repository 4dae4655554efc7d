// Multiple-traces system (Sec. 3.3, Eq. "mtf:discrete") on the device, FP64:
//
//   [ -K_e   V_e    1/2 P_ei              0               ] [v_e]   [-f]
//   [  D_e   T_e    0                    1/2 (re/ri) P_ei ] [w_e] = [-g]
//   [ -1/2 P_ie     0      -K_i          V_i              ] [v_i]   [ 0]
//   [  0  -1/2 (ri/re) P_ie  D_i         T_i              ] [w_i]   [ 0]
//
// with mass-matrix (strong-form) preconditioning blockdiag(M_e, M_e, M_i,
// M_i)^-1 (Sec. 3.3) and GMRES without restart (Sec. 5.1).
//
//   mass_inverse_kernel  dense M^-1 by Chebyshev iteration on Jacobi-scaled M
//                        (the spectrum of diag(M)^-1 M of P1 triangles lies
//                        in [1/2, 2], so 40 steps reach rounding level);
//                        search directions live in LDS, one workgroup per
//                        group of columns.
//   mtf_dense_kernel     one wave per row, streams the four dense rows of the
//                        row's mesh once (complex128, 16 B per lane, coalesced)
//                        and adds the mortar coupling of that row (CSR).
//   mass_apply_kernel    z = M^-1 y for the two vectors of one mesh at once.
//   cgs_dots / cgs_update / norm kernels: classical Gram-Schmidt with one
//                        re-orthogonalisation in FP64, reductions in a fixed
//                        order (deterministic).
//   Givens rotations and the convergence test run on the host from the
//   (j+2) Hessenberg entries copied back each step.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "internal.h"

namespace bemtx {

namespace {

constexpr double kA1 = 0.445948490915964886318329253883;
constexpr double kW1 = 0.223381589678011465944827736698;
constexpr double kA2 = 0.091576213509770743459571463402;
constexpr double kW2 = 0.109951743655321867388505596635;

__host__ __device__ constexpr double q6_bary(int q, int c)
{
    return q < 3 ? (c == q ? 1.0 - 2.0 * kA1 : kA1) : (c == q - 3 ? 1.0 - 2.0 * kA2 : kA2);
}
__host__ __device__ constexpr double q6_w(int q) { return q < 3 ? kW1 : kW2; }

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

typedef double v2d __attribute__((ext_vector_type(2)));

// streaming load of a complex128 matrix entry (read once, do not keep in cache)
__device__ inline double2 ld_stream(const double2 *p)
{
    const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p));
    return make_double2(v.x, v.y);
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

// ----------------------------------------------------------------- loads

// b = [-f, -g, 0, 0] in internal numbering for one direction d:
// f_j = sum over triangles t at j of A_t sum_q w_q lambda_j(q) exp(i k d.x_q),
// g_j = the same with the factor i k (d.n_t).
__global__ void rhs_kernel(int ne, int ni, const int32_t *__restrict__ star_ptr, const int32_t *__restrict__ star_ent,
                           const TriGeo *__restrict__ geo, double k, double d0, double d1, double d2,
                           double2 *__restrict__ b)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 2 * ne + 2 * ni;
    if (j >= n) return;
    if (j >= 2 * ne) { b[j] = make_double2(0, 0); return; }
    const int v = j < ne ? j : j - ne;
    const bool is_g = j >= ne;
    double re = 0.0, im = 0.0;
    for (int e = star_ptr[v]; e < star_ptr[v + 1]; ++e) {
        const int t = star_ent[e] / 3, a = star_ent[e] - 3 * (star_ent[e] / 3);
        const TriGeo &g = geo[t];
        const double dn = d0 * g.n[0] + d1 * g.n[1] + d2 * g.n[2];
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < 6; ++q) {
            const double ph = k * (d0 * g.qp[q][0] + d1 * g.qp[q][1] + d2 * g.qp[q][2]);
            double s, c;
            sincos(ph, &s, &c);
            const double w = q6_w(q) * q6_bary(q, a);
            sr += w * c;
            si += w * s;
        }
        sr *= g.area;
        si *= g.area;
        if (is_g) {   // i k dn (sr + i si)
            re += -k * dn * si;
            im += k * dn * sr;
        } else {
            re += sr;
            im += si;
        }
    }
    b[j] = make_double2(-re, -im);
}

// --------------------------------------------------------- mass inverse

// Column c = blockIdx.x of M^-1 (= row c, M is symmetric), blockDim 1024,
// R rows per thread kept in registers; the search direction lives in LDS.
template <int R>
__global__ __launch_bounds__(1024) void mass_inverse_kernel(int nv, const int32_t *__restrict__ mp,
                                                             const int32_t *__restrict__ mc,
                                                             const double *__restrict__ mv, double *__restrict__ Minv)
{
    extern __shared__ double dsh[];   // [nv]
    const int col = blockIdx.x;
    const int tid = threadIdx.x;
    const double lmin = 0.5, lmax = 2.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma1 = theta / delta;
    double x[R], r[R], dg[R], ad[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int row = tid + 1024 * k;
        x[k] = 0.0;
        r[k] = 0.0;
        dg[k] = 0.0;
        if (row < nv) {
            double diag = 0.0;
            for (int q = mp[row]; q < mp[row + 1]; ++q)
                if (mc[q] == row) diag = mv[q];
            dg[k] = 1.0 / diag;
            r[k] = row == col ? 1.0 : 0.0;
            dsh[row] = dg[k] * r[k] / theta;
        }
    }
    double rho = 1.0 / sigma1;
    __syncthreads();
    for (int it = 0; it < 40; ++it) {
        const double rho_new = 1.0 / (2.0 * sigma1 - rho);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int row = tid + 1024 * k;
            double s = 0.0;
            if (row < nv)
                for (int q = mp[row]; q < mp[row + 1]; ++q) s += mv[q] * dsh[mc[q]];
            ad[k] = s;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int row = tid + 1024 * k;
            if (row < nv) {
                const double dold = dsh[row];
                x[k] += dold;
                r[k] -= ad[k];
                dsh[row] = rho_new * rho * dold + (2.0 * rho_new / delta) * dg[k] * r[k];
            }
        }
        rho = rho_new;
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int row = tid + 1024 * k;
        if (row < nv) Minv[(int64_t)col * nv + row] = x[k];
    }
}

template <int R>
static bem_status launch_minv_r(bem_problem *p, int nv, int mesh)
{
    const size_t lds = (size_t)nv * sizeof(double);
    BEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&mass_inverse_kernel<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(mass_inverse_kernel<R>, dim3(nv), dim3(1024), lds, p->ctx->stream, nv,
                       p->M_ptr[mesh].as<int32_t>(), p->M_col[mesh].as<int32_t>(), p->M_val[mesh].as<double>(),
                       p->Minv[mesh].as<double>());
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

bem_status launch_mass_inverse(bem_problem *p, int mesh)
{
    const bem_mesh *m = mesh == 0 ? p->ext : p->inte;
    const int nv = (int)m->h.nv;
    if (nv > 16 * 1024) return set_error(BEM_E_UNSUPPORTED, "mass inverse: more than 16384 vertices on one mesh");
    bem_status s = dev_alloc(p->ctx, p->Minv[mesh], (size_t)nv * nv * sizeof(double));
    if (s) return s;
    const int R = (nv + 1023) / 1024;
    switch (R) {
    case 1: return launch_minv_r<1>(p, nv, mesh);
    case 2: return launch_minv_r<2>(p, nv, mesh);
    case 3: return launch_minv_r<3>(p, nv, mesh);
    case 4: return launch_minv_r<4>(p, nv, mesh);
    case 5: case 6: return launch_minv_r<6>(p, nv, mesh);
    case 7: case 8: return launch_minv_r<8>(p, nv, mesh);
    case 9: case 10: case 11: case 12: return launch_minv_r<12>(p, nv, mesh);
    default: return launch_minv_r<16>(p, nv, mesh);
    }
}

// --------------------------------------------------------------- mat-vec

struct MtfArgs {
    int ne, ni;
    const double2 *Ve, *Ke, *Te, *De, *Vi, *Ki, *Ti, *Di;
    const int32_t *pie_ptr, *pie_col, *pei_ptr, *pei_col;
    const double *pie_val, *pei_val;
    double c_ext_v, c_ext_w, c_int_v, c_int_w;   // 1/2, 1/2 re/ri, -1/2, -1/2 ri/re
};

// y = A x (weak form), one wave per row of [ext rows ; int rows]
__global__ __launch_bounds__(256) void mtf_dense_kernel(MtfArgs A, const double2 *__restrict__ x, double2 *__restrict__ y)
{
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= A.ne + A.ni) return;
    const bool ext = wave < A.ne;
    const int i = ext ? wave : wave - A.ne;
    const int nv = ext ? A.ne : A.ni;
    const double2 *Km = ext ? A.Ke : A.Ki, *Vm = ext ? A.Ve : A.Vi, *Dm = ext ? A.De : A.Di, *Tm = ext ? A.Te : A.Ti;
    const double2 *xv = ext ? x : x + 2 * A.ne;
    const double2 *xw = xv + nv;
    const int64_t o = (int64_t)i * nv;
    double ar = 0, ai = 0, br = 0, bi = 0;   // row of [-K V] and of [D T]
    int j = lane;
    for (; j + 64 < nv; j += 128) {
        const double2 k0 = ld_stream(&Km[o + j]), k1 = ld_stream(&Km[o + j + 64]);
        const double2 v0 = ld_stream(&Vm[o + j]), v1 = ld_stream(&Vm[o + j + 64]);
        const double2 d0 = ld_stream(&Dm[o + j]), d1 = ld_stream(&Dm[o + j + 64]);
        const double2 t0 = ld_stream(&Tm[o + j]), t1 = ld_stream(&Tm[o + j + 64]);
        const double2 p0 = xv[j], p1 = xv[j + 64], q0 = xw[j], q1 = xw[j + 64];
        ar += -(k0.x * p0.x - k0.y * p0.y) + (v0.x * q0.x - v0.y * q0.y);
        ai += -(k0.x * p0.y + k0.y * p0.x) + (v0.x * q0.y + v0.y * q0.x);
        br += (d0.x * p0.x - d0.y * p0.y) + (t0.x * q0.x - t0.y * q0.y);
        bi += (d0.x * p0.y + d0.y * p0.x) + (t0.x * q0.y + t0.y * q0.x);
        ar += -(k1.x * p1.x - k1.y * p1.y) + (v1.x * q1.x - v1.y * q1.y);
        ai += -(k1.x * p1.y + k1.y * p1.x) + (v1.x * q1.y + v1.y * q1.x);
        br += (d1.x * p1.x - d1.y * p1.y) + (t1.x * q1.x - t1.y * q1.y);
        bi += (d1.x * p1.y + d1.y * p1.x) + (t1.x * q1.y + t1.y * q1.x);
    }
    for (; j < nv; j += 64) {
        const double2 k0 = Km[o + j], v0 = Vm[o + j], d0 = Dm[o + j], t0 = Tm[o + j];
        const double2 p0 = xv[j], q0 = xw[j];
        ar += -(k0.x * p0.x - k0.y * p0.y) + (v0.x * q0.x - v0.y * q0.y);
        ai += -(k0.x * p0.y + k0.y * p0.x) + (v0.x * q0.y + v0.y * q0.x);
        br += (d0.x * p0.x - d0.y * p0.y) + (t0.x * q0.x - t0.y * q0.y);
        bi += (d0.x * p0.y + d0.y * p0.x) + (t0.x * q0.y + t0.y * q0.x);
    }
    // mortar coupling of this row
    const int32_t *pp = ext ? A.pei_ptr : A.pie_ptr;
    const int32_t *pc = ext ? A.pei_col : A.pie_col;
    const double *pv = ext ? A.pei_val : A.pie_val;
    const double2 *cv = ext ? x + 2 * A.ne : x;           // other mesh's v
    const int nother = ext ? A.ni : A.ne;
    const double2 *cw = cv + nother;                        // other mesh's w
    const double fv = ext ? A.c_ext_v : A.c_int_v, fw = ext ? A.c_ext_w : A.c_int_w;
    for (int q = pp[i] + lane; q < pp[i + 1]; q += 64) {
        const double pvq = pv[q];
        const int c = pc[q];
        ar += fv * pvq * cv[c].x;
        ai += fv * pvq * cv[c].y;
        br += fw * pvq * cw[c].x;
        bi += fw * pvq * cw[c].y;
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    br = wave_sum(br);
    bi = wave_sum(bi);
    if (lane == 0) {
        double2 *ya = ext ? y : y + 2 * A.ne;
        ya[i] = make_double2(ar, ai);
        ya[i + nv] = make_double2(br, bi);
    }
}

// z = blockdiag(M_e^-1, M_e^-1, M_i^-1, M_i^-1) y; one wave per (mesh row)
__global__ __launch_bounds__(256) void mass_apply_kernel(int ne, int ni, const double *__restrict__ Me_inv,
                                                         const double *__restrict__ Mi_inv,
                                                         const double2 *__restrict__ y, double2 *__restrict__ z)
{
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= ne + ni) return;
    const bool ext = wave < ne;
    const int i = ext ? wave : wave - ne;
    const int nv = ext ? ne : ni;
    const double *Mr = (ext ? Me_inv : Mi_inv) + (int64_t)i * nv;
    const double2 *ya = ext ? y : y + 2 * ne;
    const double2 *yb = ya + nv;
    double ar = 0, ai = 0, br = 0, bi = 0;
    for (int j = lane; j < nv; j += 64) {
        const double m = __builtin_nontemporal_load(&Mr[j]);
        const double2 a = ya[j], b = yb[j];
        ar += m * a.x; ai += m * a.y; br += m * b.x; bi += m * b.y;
    }
    ar = wave_sum(ar); ai = wave_sum(ai); br = wave_sum(br); bi = wave_sum(bi);
    if (lane == 0) {
        double2 *za = ext ? z : z + 2 * ne;
        za[i] = make_double2(ar, ai);
        za[i + nv] = make_double2(br, bi);
    }
}

// ------------------------------------------------------ Krylov kernels

constexpr int CGS_CHUNK = 4096;   // rows per workgroup of the dot kernel

// partial[blk][c] = sum over the rows of chunk blk of conj(Vb[c][r]) w[r]
__global__ __launch_bounds__(256) void cgs_dots_kernel(int n, int nvec, const double2 *__restrict__ Vb,
                                                       const double2 *__restrict__ w, double2 *__restrict__ partial)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r0 = blockIdx.x * CGS_CHUNK, r1 = min(n, r0 + CGS_CHUNK);
    for (int c = wv; c < nvec; c += 4) {
        const double2 *vc = Vb + (int64_t)c * n;
        double sr = 0, si = 0;
        for (int r = r0 + lane; r < r1; r += 64) {
            const double2 a = vc[r], b = w[r];
            sr += a.x * b.x + a.y * b.y;
            si += a.x * b.y - a.y * b.x;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) partial[(int64_t)blockIdx.x * nvec + c] = make_double2(sr, si);
    }
}

// h = sum of partials (fixed order); w -= Vb h; hsum += h (block 0)
__global__ __launch_bounds__(256) void cgs_update_kernel(int n, int nvec, int nblk, const double2 *__restrict__ Vb,
                                                         const double2 *__restrict__ partial, double2 *__restrict__ w,
                                                         double2 *__restrict__ hsum)
{
    extern __shared__ double2 hs[];
    for (int c = threadIdx.x; c < nvec; c += blockDim.x) {
        double2 s = make_double2(0, 0);
        for (int b = 0; b < nblk; ++b) s = cadd(s, partial[(int64_t)b * nvec + c]);
        hs[c] = s;
        if (blockIdx.x == 0) hsum[c] = cadd(hsum[c], s);
    }
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double2 acc = w[r];
    for (int c = 0; c < nvec; ++c) {
        const double2 v = Vb[(int64_t)c * n + r], h = hs[c];
        acc.x -= v.x * h.x - v.y * h.y;
        acc.y -= v.x * h.y + v.y * h.x;
    }
    w[r] = acc;
}

// partial[blk] = sum |w|^2 over the chunk
__global__ __launch_bounds__(256) void norm_partial_kernel(int n, const double2 *__restrict__ w, double *__restrict__ partial)
{
    __shared__ double red[4];
    const int r0 = blockIdx.x * CGS_CHUNK, r1 = min(n, r0 + CGS_CHUNK);
    double s = 0;
    for (int r = r0 + threadIdx.x; r < r1; r += 256) s += w[r].x * w[r].x + w[r].y * w[r].y;
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// beta = sqrt(sum partial); out = w / beta; beta_out = beta
__global__ __launch_bounds__(256) void normalize_kernel(int n, int nblk, const double *__restrict__ partial,
                                                        const double2 *__restrict__ w, double2 *__restrict__ out,
                                                        double *__restrict__ beta_out)
{
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[b];
    const double beta = sqrt(s);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) *beta_out = beta;
    if (r >= n) return;
    const double inv = beta > 0 ? 1.0 / beta : 0.0;
    out[r] = make_double2(w[r].x * inv, w[r].y * inv);
}

// x = sum_c y[c] Vb[c]
__global__ void combine_kernel(int n, int nvec, const double2 *__restrict__ Vb, const double2 *__restrict__ yc,
                               double2 *__restrict__ x)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double2 acc = make_double2(0, 0);
    for (int c = 0; c < nvec; ++c) acc = cadd(acc, cmul(yc[c], Vb[(int64_t)c * n + r]));
    x[r] = acc;
}

__global__ void axpy_sub_kernel(int n, const double2 *__restrict__ a, const double2 *__restrict__ b, double2 *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = make_double2(a[r].x - b[r].x, a[r].y - b[r].y);
}

// ---------------------------------------------------- numbering changes

// internal -> caller (dir = 0) or caller -> internal (dir = 1) for an MTF vector
__global__ void permute_vec_kernel(int ne, int ni, const int32_t *__restrict__ pe, const int32_t *__restrict__ pi,
                                   const double2 *__restrict__ src, double2 *__restrict__ dst, int dir)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = 2 * ne + 2 * ni;
    if (u >= n) return;
    int base, loc;
    const int32_t *perm;
    if (u < 2 * ne) { base = u < ne ? 0 : ne; loc = u - base; perm = pe; }
    else { base = u < 2 * ne + ni ? 2 * ne : 2 * ne + ni; loc = u - base; perm = pi; }
    const int in = base + perm[loc];
    if (dir == 0) dst[u] = src[in];
    else dst[in] = src[u];
}

__global__ void permute_mat_kernel(int nv, const int32_t *__restrict__ perm, const double2 *__restrict__ src,
                                   double2 *__restrict__ dst)
{
    const int iu = blockIdx.y;
    const int ju = blockIdx.x * blockDim.x + threadIdx.x;
    if (ju >= nv) return;
    dst[(int64_t)iu * nv + ju] = src[(int64_t)perm[iu] * nv + perm[ju]];
}

bem_status permute_matrix_out(const bem_problem *p, int mesh, const double2 *src, double2 *dst)
{
    const bem_mesh *m = mesh == 0 ? p->ext : p->inte;
    const int nv = (int)m->h.nv;
    hipLaunchKernelGGL(permute_mat_kernel, dim3((nv + 255) / 256, nv), dim3(256), 0, p->ctx->stream, nv,
                       m->d.perm.as<int32_t>(), src, dst);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

// ------------------------------------------------------------ host side

namespace {

struct Work {
    DevMem xin, y, z, b, r, Vb, partial, hsum, beta, yc, npart;
};

MtfArgs make_args(const bem_problem *p)
{
    MtfArgs A;
    A.ne = (int)p->ext->h.nv;
    A.ni = (int)p->inte->h.nv;
    A.Ve = p->ops[0][0].as<double2>(); A.Ke = p->ops[0][1].as<double2>();
    A.Te = p->ops[0][2].as<double2>(); A.De = p->ops[0][3].as<double2>();
    A.Vi = p->ops[1][0].as<double2>(); A.Ki = p->ops[1][1].as<double2>();
    A.Ti = p->ops[1][2].as<double2>(); A.Di = p->ops[1][3].as<double2>();
    A.pie_ptr = p->P_ie_ptr.as<int32_t>(); A.pie_col = p->P_ie_col.as<int32_t>(); A.pie_val = p->P_ie_val.as<double>();
    A.pei_ptr = p->P_ei_ptr.as<int32_t>(); A.pei_col = p->P_ei_col.as<int32_t>(); A.pei_val = p->P_ei_val.as<double>();
    A.c_ext_v = 0.5;
    A.c_ext_w = 0.5 * p->rho_ext / p->rho_int;
    A.c_int_v = -0.5;
    A.c_int_w = -0.5 * p->rho_int / p->rho_ext;
    return A;
}

bem_status apply_A(const bem_problem *p, const MtfArgs &A, const double2 *x, double2 *y, double2 *z, bool strong)
{
    hipStream_t st = p->ctx->stream;
    const int rows = A.ne + A.ni;
    hipLaunchKernelGGL(mtf_dense_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, A, x, y);
    BEM_HIP(hipGetLastError());
    if (strong) {
        hipLaunchKernelGGL(mass_apply_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, A.ne, A.ni,
                           p->Minv[0].as<double>(), p->Minv[1].as<double>(), y, z);
        BEM_HIP(hipGetLastError());
    }
    return BEM_OK;
}

}  // namespace

bem_status matvec_impl(bem_problem *p, const void *x, void *y, int strong, bem_memspace space)
{
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    const size_t bytes = (size_t)n * sizeof(double2);
    DevMem xu, xi, yi, zi, yu;
    bem_status s = dev_alloc(ctx, xu, bytes);
    if (!s) s = dev_alloc(ctx, xi, bytes);
    if (!s) s = dev_alloc(ctx, yi, bytes);
    if (!s) s = dev_alloc(ctx, zi, bytes);
    if (!s) s = dev_alloc(ctx, yu, bytes);
    if (s) return s;
    BEM_HIP(hipMemcpyAsync(xu.ptr, x, bytes, space == BEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
    const dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                       p->inte->d.perm.as<int32_t>(), xu.as<double2>(), xi.as<double2>(), 1);
    MtfArgs A = make_args(p);
    s = apply_A(p, A, xi.as<double2>(), yi.as<double2>(), zi.as<double2>(), strong != 0);
    if (s) return s;
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                       p->inte->d.perm.as<int32_t>(), strong ? zi.as<double2>() : yi.as<double2>(), yu.as<double2>(), 0);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipMemcpyAsync(y, yu.ptr, bytes, space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    BEM_HIP(hipStreamSynchronize(st));
    return BEM_OK;
}

static bem_status rhs_internal(bem_problem *p, const double *d, double2 *b)
{
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    hipLaunchKernelGGL(rhs_kernel, dim3((n + 255) / 256), dim3(256), 0, p->ctx->stream, ne, ni,
                       p->ext->d.star_ptr.as<int32_t>(), p->ext->d.star_ent.as<int32_t>(), p->ext->d.geo.as<TriGeo>(),
                       p->k_ext, d[0], d[1], d[2], b);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

bem_status rhs_impl(bem_problem *p, const double *dirs, int nrhs, void *b, bem_memspace space)
{
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    const size_t bytes = (size_t)n * sizeof(double2);
    DevMem bi, bu;
    bem_status s = dev_alloc(ctx, bi, bytes);
    if (!s) s = dev_alloc(ctx, bu, bytes);
    if (s) return s;
    for (int r = 0; r < nrhs; ++r) {
        s = rhs_internal(p, dirs + 3 * r, bi.as<double2>());
        if (s) return s;
        hipLaunchKernelGGL(permute_vec_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, ne, ni,
                           p->ext->d.perm.as<int32_t>(), p->inte->d.perm.as<int32_t>(), bi.as<double2>(),
                           bu.as<double2>(), 0);
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipMemcpyAsync(static_cast<double2 *>(b) + (size_t)r * n, bu.ptr, bytes,
                               space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, ctx->stream));
    }
    BEM_HIP(hipStreamSynchronize(ctx->stream));
    return BEM_OK;
}

bem_status solve_impl(bem_problem *p, const double *dirs, int nrhs, const bem_solver_opts *opts, void *traces,
                      bem_memspace space, bem_stats *stats)
{
    using cd = std::complex<double>;
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    const int m = opts->maxit;
    const size_t vb = (size_t)n * sizeof(double2);
    const int nblk = (n + CGS_CHUNK - 1) / CGS_CHUNK;
    Work W;
    bem_status s = dev_alloc(ctx, W.y, vb);
    if (!s) s = dev_alloc(ctx, W.z, vb);
    if (!s) s = dev_alloc(ctx, W.b, vb);
    if (!s) s = dev_alloc(ctx, W.r, vb);
    if (!s) s = dev_alloc(ctx, W.xin, vb);
    if (!s) s = dev_alloc(ctx, W.Vb, (size_t)(m + 1) * vb);
    if (!s) s = dev_alloc(ctx, W.partial, (size_t)nblk * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.hsum, (size_t)(m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.beta, sizeof(double) * 2);
    if (!s) s = dev_alloc(ctx, W.yc, (size_t)(m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.npart, (size_t)nblk * sizeof(double));
    if (s) return s;
    MtfArgs A = make_args(p);
    double2 *Vb = W.Vb.as<double2>();
    const dim3 gv((n + 255) / 256);
    int total_it = 0;
    double worst_res = 0.0;
    bool all_conv = true;
    auto t0 = std::chrono::steady_clock::now();
    std::vector<cd> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), h(m + 1);
    for (int rhs = 0; rhs < nrhs; ++rhs) {
        s = rhs_internal(p, dirs + 3 * rhs, W.b.as<double2>());
        if (s) return s;
        // r0 = M^-1 b (x0 = 0), v0 = r0 / ||r0||
        hipLaunchKernelGGL(mass_apply_kernel, dim3((ne + ni + 3) / 4), dim3(256), 0, st, ne, ni, p->Minv[0].as<double>(),
                           p->Minv[1].as<double>(), W.b.as<double2>(), W.r.as<double2>());
        hipLaunchKernelGGL(norm_partial_kernel, dim3(nblk), dim3(256), 0, st, n, W.r.as<double2>(), W.npart.as<double>());
        hipLaunchKernelGGL(normalize_kernel, gv, dim3(256), 0, st, n, nblk, W.npart.as<double>(), W.r.as<double2>(), Vb,
                           W.beta.as<double>());
        BEM_HIP(hipGetLastError());
        double beta0 = 0;
        BEM_HIP(hipMemcpyAsync(&beta0, W.beta.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
        BEM_HIP(hipStreamSynchronize(st));
        std::fill(g.begin(), g.end(), cd(0));
        g[0] = beta0;
        int j = 0;
        bool conv = beta0 == 0.0;
        double res = conv ? 0.0 : 1.0;
        for (; j < m && !conv; ++j) {
            const double2 *vj = Vb + (size_t)j * n;
            s = apply_A(p, A, vj, W.y.as<double2>(), W.z.as<double2>(), true);
            if (s) return s;
            BEM_HIP(hipMemsetAsync(W.hsum.ptr, 0, (size_t)(j + 1) * sizeof(double2), st));
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(cgs_dots_kernel, dim3(nblk), dim3(256), 0, st, n, j + 1, Vb, W.z.as<double2>(),
                                   W.partial.as<double2>());
                hipLaunchKernelGGL(cgs_update_kernel, gv, dim3(256), (size_t)(j + 1) * sizeof(double2), st, n, j + 1,
                                   nblk, Vb, W.partial.as<double2>(), W.z.as<double2>(), W.hsum.as<double2>());
            }
            hipLaunchKernelGGL(norm_partial_kernel, dim3(nblk), dim3(256), 0, st, n, W.z.as<double2>(), W.npart.as<double>());
            hipLaunchKernelGGL(normalize_kernel, gv, dim3(256), 0, st, n, nblk, W.npart.as<double>(), W.z.as<double2>(),
                               Vb + (size_t)(j + 1) * n, W.beta.as<double>());
            BEM_HIP(hipGetLastError());
            BEM_HIP(hipMemcpyAsync(h.data(), W.hsum.ptr, (size_t)(j + 1) * sizeof(double2), hipMemcpyDeviceToHost, st));
            double beta = 0;
            BEM_HIP(hipMemcpyAsync(&beta, W.beta.ptr, sizeof(double), hipMemcpyDeviceToHost, st));
            BEM_HIP(hipStreamSynchronize(st));
            // Hessenberg column j, previous rotations, new rotation
            cd *col = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = h[i];
            col[j + 1] = beta;
            for (int i = 0; i < j; ++i) {
                cd a = col[i], b = col[i + 1];
                col[i] = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
                col[i + 1] = -sn[i] * a + cs[i] * b;
            }
            double den = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
            if (den == 0.0) { cs[j] = 1; sn[j] = 0; }
            else { cs[j] = col[j] / den; sn[j] = col[j + 1] / den; }
            col[j] = den;
            col[j + 1] = 0;
            cd gj = g[j];
            g[j] = std::conj(cs[j]) * gj;
            g[j + 1] = -sn[j] * gj;
            res = std::abs(g[j + 1]) / beta0;
            if (res <= opts->tol || beta == 0.0) conv = true;
        }
        const int k = j;
        total_it += k;
        // back substitution R y = g
        std::vector<cd> yv(k);
        for (int i = k - 1; i >= 0; --i) {
            cd sacc = g[i];
            for (int c = i + 1; c < k; ++c) sacc -= H[(size_t)c * (m + 1) + i] * yv[c];
            yv[i] = sacc / H[(size_t)i * (m + 1) + i];
        }
        if (k > 0) BEM_HIP(hipMemcpyAsync(W.yc.ptr, yv.data(), (size_t)k * sizeof(double2), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(combine_kernel, gv, dim3(256), 0, st, n, k, Vb, W.yc.as<double2>(), W.xin.as<double2>());
        BEM_HIP(hipGetLastError());
        // true strong-form residual in FP64: M^-1 (b - A x)
        s = apply_A(p, A, W.xin.as<double2>(), W.y.as<double2>(), W.z.as<double2>(), false);
        if (s) return s;
        hipLaunchKernelGGL(axpy_sub_kernel, gv, dim3(256), 0, st, n, W.b.as<double2>(), W.y.as<double2>(), W.r.as<double2>());
        hipLaunchKernelGGL(mass_apply_kernel, dim3((ne + ni + 3) / 4), dim3(256), 0, st, ne, ni, p->Minv[0].as<double>(),
                           p->Minv[1].as<double>(), W.r.as<double2>(), W.z.as<double2>());
        hipLaunchKernelGGL(norm_partial_kernel, dim3(nblk), dim3(256), 0, st, n, W.z.as<double2>(), W.npart.as<double>());
        hipLaunchKernelGGL(normalize_kernel, gv, dim3(256), 0, st, n, nblk, W.npart.as<double>(), W.z.as<double2>(),
                           W.r.as<double2>(), W.beta.as<double>() + 1);
        BEM_HIP(hipGetLastError());
        double rn = 0;
        BEM_HIP(hipMemcpyAsync(&rn, W.beta.as<double>() + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        // traces in caller numbering
        hipLaunchKernelGGL(permute_vec_kernel, gv, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                           p->inte->d.perm.as<int32_t>(), W.xin.as<double2>(), W.y.as<double2>(), 0);
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipMemcpyAsync(static_cast<double2 *>(traces) + (size_t)rhs * n, W.y.ptr, vb,
                               space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
        BEM_HIP(hipStreamSynchronize(st));
        const double rel = beta0 > 0 ? rn / beta0 : 0.0;
        worst_res = std::max(worst_res, rel);
        if (!(res <= opts->tol)) all_conv = false;
    }
    const double t_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->iterations = total_it;
        stats->rel_residual = worst_res;
        stats->t_geometry_ms = p->t_geometry_ms;
        stats->t_regular_ms = p->t_regular_ms;
        stats->t_singular_ms = p->t_singular_ms;
        stats->t_projection_ms = p->t_projection_ms;
        stats->t_matrix_ms = p->t_regular_ms + p->t_singular_ms + p->t_projection_ms;
        stats->t_solve_ms = t_solve;
        stats->t_iter_ms = total_it > 0 ? t_solve / total_it : 0.0;
    }
    return all_conv ? BEM_OK : set_error(BEM_W_NOCONV, "GMRES reached maxit before the tolerance");
}

}  // namespace bemtx
