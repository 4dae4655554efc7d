// Multiple-traces system (Sec. 3.3, Eq. "mtf:discrete") on the device:
//
//   [ -K_e   V_e    1/2 P_ei              0               ] [v_e]   [-f]
//   [  D_e   T_e    0                    1/2 (re/ri) P_ei ] [w_e] = [-g]
//   [ -1/2 P_ie     0      -K_i          V_i              ] [v_i]   [ 0]
//   [  0  -1/2 (ri/re) P_ie  D_i         T_i              ] [w_i]   [ 0]
//
// with mass-matrix (strong-form) preconditioning blockdiag(M_e, M_e, M_i,
// M_i)^-1 (Sec. 3.3) and GMRES without restart (Sec. 5.1).
//
//   mass_inverse kernels   dense M^-1 by Chebyshev iteration on Jacobi-scaled
//                          M (the spectrum of diag(M)^-1 M of P1 triangles
//                          lies in [1/2, 2], so 36 steps reach FP64 rounding
//                          level); search directions live in LDS, several
//                          columns per workgroup.
//   mtf_sym_tile           one product with the dense blocks of both meshes,
//                          K read in full, V and D only on and above the
//                          diagonal, T = K^T (128 x 128 tiles,
//                          16-byte non-temporal loads; row sums reduced with
//                          DPP, column sums per lane); per-tile partials.
//   mtf_sym_combine        fixed-order sum of the tile partials, the
//                          near-entry corrections of the parts that are not
//                          symmetric, and the mortar coupling of the row.
//   mass_apply_part/combine  z = M^-1 y, split-column scheme: a chunk of y
//                          staged in LDS, several rows per wave.
//   block products         R Krylov vectors at once on the matrix cores
//                          (gemm.hip) for batched right-hand sides.
//   cgs_dots / cgs_update / arnoldi_finish   classical Gram-Schmidt with one
//                          re-orthogonalisation in FP64 and the Givens
//                          rotations of the new Hessenberg column on the
//                          device; reductions in a fixed order
//                          (deterministic).
//   The host issues steps ahead and polls a small state record; it learns of
//   convergence without stalling the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "phase.h"

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

// row stride of the dense inverse mass matrices: rows start on 16-byte
// boundaries (even for FP64 storage; a multiple of 32 for FP32, the k step of
// the matrix-core product)
__host__ __device__ inline int minv_ld(int nv, bool f32) { return f32 ? (nv + 31) & ~31 : (nv + 1) & ~1; }

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
// incident field: kind 0 the plane wave exp(i k d.x) (Sec. 5.3), kind 1 the
// point source exp(i k |x - x0|) / (4 pi |x - x0|) at x0 = (d0, d1, d2) (Sec. 5.7)
__global__ void rhs_kernel(int ne, int ni, const int32_t *__restrict__ star_ptr, const int32_t *__restrict__ star_ent,
                           const TriGeo *__restrict__ geo, double k, int kind, double d0, double d1, double d2,
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
        if (kind == 0) {
            for (int q = 0; q < 6; ++q) {
                const double ph = k * (d0 * g.qp[q][0] + d1 * g.qp[q][1] + d2 * g.qp[q][2]);
                double s, c;
                phase_sincos(ph, &s, &c);
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
        } else {
            for (int q = 0; q < 6; ++q) {
                const double R0 = g.qp[q][0] - d0, R1 = g.qp[q][1] - d1, R2 = g.qp[q][2] - d2;   // y - x0
                const double r = sqrt(R0 * R0 + R1 * R1 + R2 * R2), inv = 0.0795774715459476678844418816863 / r;
                double s, c;
                phase_sincos(k * r, &s, &c);
                const double w = q6_w(q) * q6_bary(q, a);
                if (is_g) {   // exp(ikr)(ikr - 1)((y - x0).n) / (4 pi r^3)
                    const double f = (R0 * g.n[0] + R1 * g.n[1] + R2 * g.n[2]) / (r * r) * inv;
                    sr += w * (-c - s * k * r) * f;
                    si += w * (c * k * r - s) * f;
                } else {
                    sr += w * c * inv;
                    si += w * s * inv;
                }
            }
            re += sr * g.area;
            im += si * g.area;
        }
    }
    b[j] = make_double2(-re, -im);
}

// --------------------------------------------------------- mass inverse


// Column c = blockIdx.x of M^-1 (= row c, M is symmetric), blockDim 1024,
// R rows per thread kept in registers; the search direction lives in LDS;
// nsteps Chebyshev steps.
template <int R, class TOut>
__global__ __launch_bounds__(1024) void mass_inverse_kernel(int nv, int ldm, int nsteps, const int32_t *__restrict__ mp,
                                                             const int32_t *__restrict__ mc,
                                                             const double *__restrict__ mv, TOut *__restrict__ Minv)
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
    for (int it = 0; it < nsteps; ++it) {
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
        if (row < nv) Minv[(int64_t)col * ldm + row] = (TOut)x[k];
    }
}

// Same iteration for C columns per workgroup: M in ELL form (width W, layout
// [q][row] so that loads are coalesced, padding = zero entries on the
// diagonal) read from L2 once per step for all C columns, and the search
// directions double-buffered in LDS so that one barrier per step suffices
// (DB), or single-buffered with a second barrier when two copies do not fit.
template <int R, int C, class TOut, bool DB>
__global__ __launch_bounds__(1024) void mass_inverse_ell_kernel(int nv, int ldm, int W, int nsteps,
                                                                 const int32_t *__restrict__ ell_col,
                                                                 const double *__restrict__ ell_val,
                                                                 TOut *__restrict__ Minv)
{
    extern __shared__ double dsh[];   // [2][C][nv] (double-buffered) or [C][nv]
    const int c0 = blockIdx.x * C;
    const int tid = threadIdx.x;
    const double lmin = 0.5, lmax = 2.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma1 = theta / delta;
    double dg[R], x[R][C], r[R][C];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int row = tid + 1024 * k;
        const bool ok = row < nv;
        double dsum = 0.0;
        if (ok)
            for (int q = 0; q < W; ++q)
                if (ell_col[(int64_t)q * nv + row] == row) dsum += ell_val[(int64_t)q * nv + row];
        dg[k] = ok ? 1.0 / dsum : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            x[k][c] = 0.0;
            r[k][c] = (ok && row == c0 + c) ? 1.0 : 0.0;
            if (ok) dsh[c * nv + row] = dg[k] * r[k][c] / theta;
        }
    }
    double rho = 1.0 / sigma1;
    int cur = 0;
    __syncthreads();
    for (int it = 0; it < nsteps; ++it) {
        const double rho_new = 1.0 / (2.0 * sigma1 - rho);
        const double *dold = dsh + (DB ? cur * C * nv : 0);
        double *dnew = dsh + (DB ? (cur ^ 1) * C * nv : 0);
        double dk[R][C];   // single buffer: directions kept until every product of the step is done
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int row = tid + 1024 * k;
            if (row >= nv) continue;
            double ad[C];
#pragma unroll
            for (int c = 0; c < C; ++c) ad[c] = 0.0;
            for (int q = 0; q < W; ++q) {
                const int col = ell_col[(int64_t)q * nv + row];
                const double v = ell_val[(int64_t)q * nv + row];
#pragma unroll
                for (int c = 0; c < C; ++c) ad[c] += v * dold[c * nv + col];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double d = dold[c * nv + row];
                x[k][c] += d;
                r[k][c] -= ad[c];
                dk[k][c] = rho_new * rho * d + (2.0 * rho_new / delta) * dg[k] * r[k][c];
                if (DB) dnew[c * nv + row] = dk[k][c];
            }
        }
        if (!DB) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int row = tid + 1024 * k;
                if (row < nv)
#pragma unroll
                    for (int c = 0; c < C; ++c) dnew[c * nv + row] = dk[k][c];
            }
        }
        rho = rho_new;
        cur ^= 1;
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int row = tid + 1024 * k;
        if (row < nv)
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (c0 + c < nv) Minv[(int64_t)(c0 + c) * ldm + row] = (TOut)x[k][c];
    }
}

// Chebyshev steps for the stored precision: the error falls by 1/3 per step
// on a spectrum inside [1/2, 2] (bound 2 (1/3)^k), so 36 steps reach 1e-17
// (FP64 storage) and 18 steps 5e-9 (FP32 storage, below its rounding).
template <class TOut> constexpr int chebyshev_steps() { return sizeof(TOut) == 4 ? 18 : 36; }

template <int R, class TOut>
static bem_status launch_minv_r(bem_problem *p, int nv, int mesh, hipStream_t st)
{
    const size_t lds = (size_t)nv * sizeof(double);
    BEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&mass_inverse_kernel<R, TOut>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    KTimer kt(p->ctx, K_MASS_INVERSE);
    launch_k(kt, mass_inverse_kernel<R, TOut>, dim3(nv), dim3(1024), lds, st, nv,
             minv_ld(nv, sizeof(TOut) == 4), chebyshev_steps<TOut>(), p->M_ptr[mesh].as<int32_t>(),
             p->M_col[mesh].as<int32_t>(),
             p->M_val[mesh].as<double>(), p->Minv[mesh].as<TOut>());
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

template <int R, int C, class TOut, bool DB>
static bem_status launch_minv_ell(bem_problem *p, int nv, int W, int mesh, const int32_t *ec, const double *ev,
                                  hipStream_t st)
{
    const size_t lds = (size_t)(DB ? 2 : 1) * C * nv * sizeof(double);
    BEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&mass_inverse_ell_kernel<R, C, TOut, DB>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    KTimer kt(p->ctx, K_MASS_INVERSE);
    launch_k(kt, mass_inverse_ell_kernel<R, C, TOut, DB>, dim3((nv + C - 1) / C), dim3(1024), lds, st,
             nv, minv_ld(nv, sizeof(TOut) == 4), W, chebyshev_steps<TOut>(), ec, ev, p->Minv[mesh].as<TOut>());
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

template <int R, class TOut>
static bem_status launch_minv_ell_r(bem_problem *p, int nv, int W, int mesh, const int32_t *ec, const double *ev,
                                    hipStream_t st)
{
    // columns per workgroup: as many double-buffered directions as fit in 160 KiB of LDS
    const int cfit = (int)(163840 / (2 * (size_t)nv * sizeof(double)));
    if (cfit >= 8) return launch_minv_ell<R, 8, TOut, true>(p, nv, W, mesh, ec, ev, st);
    if (cfit >= 4) return launch_minv_ell<R, 4, TOut, true>(p, nv, W, mesh, ec, ev, st);
    if (cfit >= 3) return launch_minv_ell<R, 3, TOut, true>(p, nv, W, mesh, ec, ev, st);
    if (cfit >= 2) return launch_minv_ell<R, 2, TOut, true>(p, nv, W, mesh, ec, ev, st);
    if (cfit >= 1) return launch_minv_ell<R, 1, TOut, true>(p, nv, W, mesh, ec, ev, st);
    return launch_minv_ell<R, 1, TOut, false>(p, nv, W, mesh, ec, ev, st);
}

template <class TOut>
static bem_status launch_minv_ell_any(bem_problem *p, int nv, int W, int mesh, const int32_t *dc, const double *dv,
                                      hipStream_t st)
{
    switch ((nv + 1023) / 1024) {
    case 1: return launch_minv_ell_r<1, TOut>(p, nv, W, mesh, dc, dv, st);
    case 2: return launch_minv_ell_r<2, TOut>(p, nv, W, mesh, dc, dv, st);
    case 3: return launch_minv_ell_r<3, TOut>(p, nv, W, mesh, dc, dv, st);
    case 4: return launch_minv_ell_r<4, TOut>(p, nv, W, mesh, dc, dv, st);
    case 5: case 6: return launch_minv_ell_r<6, TOut>(p, nv, W, mesh, dc, dv, st);
    case 7: case 8: return launch_minv_ell_r<8, TOut>(p, nv, W, mesh, dc, dv, st);
    case 9: case 10: return launch_minv_ell_r<10, TOut>(p, nv, W, mesh, dc, dv, st);
    case 11: case 12: return launch_minv_ell_r<12, TOut>(p, nv, W, mesh, dc, dv, st);
    case 13: case 14: case 15: case 16: return launch_minv_ell_r<16, TOut>(p, nv, W, mesh, dc, dv, st);
    default: return launch_minv_ell_r<20, TOut>(p, nv, W, mesh, dc, dv, st);
    }
}

template <class TOut>
static bem_status launch_minv_csr_any(bem_problem *p, int nv, int mesh, hipStream_t st)
{
    switch ((nv + 1023) / 1024) {
    case 1: return launch_minv_r<1, TOut>(p, nv, mesh, st);
    case 2: return launch_minv_r<2, TOut>(p, nv, mesh, st);
    case 3: return launch_minv_r<3, TOut>(p, nv, mesh, st);
    case 4: return launch_minv_r<4, TOut>(p, nv, mesh, st);
    case 5: case 6: return launch_minv_r<6, TOut>(p, nv, mesh, st);
    case 7: case 8: return launch_minv_r<8, TOut>(p, nv, mesh, st);
    case 9: case 10: case 11: case 12: return launch_minv_r<12, TOut>(p, nv, mesh, st);
    default: return launch_minv_r<16, TOut>(p, nv, mesh, st);
    }
}

bem_status launch_mass_inverse(bem_problem *p, int mesh, hipStream_t st)
{
    const bem_mesh *m = mesh == 0 ? p->ext : p->inte;
    const int nv = (int)m->h.nv;
    if (nv > 16 * 1024) return set_error(BEM_E_UNSUPPORTED, "mass inverse: more than 16384 vertices on one mesh");
    const bool f32 = p->prec == BEM_C64_MIXED;
    const size_t bytes = (size_t)nv * minv_ld(nv, f32) * (f32 ? sizeof(float) : sizeof(double));
    bem_status s = dev_alloc(p->ctx, p->Minv[mesh], bytes, st);
    if (s) return s;
    // padding columns must read as zero (vector loads cover them)
    BEM_HIP(hipMemsetAsync(p->Minv[mesh].ptr, 0, bytes, st));
    const Csr &M = p->M[mesh];
    int W = 0;
    for (int64_t i = 0; i < M.nrows; ++i) W = std::max(W, M.ptr[i + 1] - M.ptr[i]);
    if ((size_t)nv * sizeof(double) <= 163840) {
        // ELL, [q][row], padded with zeros on the diagonal
        auto &ec = p->ell_col_h[mesh];
        auto &ev = p->ell_val_h[mesh];
        ec.assign((size_t)nv * W, 0);
        ev.assign((size_t)nv * W, 0.0);
        for (int i = 0; i < nv; ++i) {
            int q = 0;
            for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k, ++q) {
                ec[(size_t)q * nv + i] = M.col[k];
                ev[(size_t)q * nv + i] = M.val[k];
            }
            for (; q < W; ++q) ec[(size_t)q * nv + i] = i;
        }
        s = dev_alloc(p->ctx, p->M_ell_col[mesh], ec.size() * sizeof(int32_t), st);
        if (!s) s = dev_alloc(p->ctx, p->M_ell_val[mesh], ev.size() * sizeof(double), st);
        if (s) return s;
        BEM_HIP(hipMemcpyAsync(p->M_ell_col[mesh].ptr, ec.data(), ec.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               st));
        BEM_HIP(hipMemcpyAsync(p->M_ell_val[mesh].ptr, ev.data(), ev.size() * sizeof(double), hipMemcpyHostToDevice,
                               st));
        const int32_t *dc = p->M_ell_col[mesh].as<int32_t>();
        const double *dv = p->M_ell_val[mesh].as<double>();
        return f32 ? launch_minv_ell_any<float>(p, nv, W, mesh, dc, dv, st)
                   : launch_minv_ell_any<double>(p, nv, W, mesh, dc, dv, st);
    }
    return f32 ? launch_minv_csr_any<float>(p, nv, mesh, st) : launch_minv_csr_any<double>(p, nv, mesh, st);
}

// --------------------------------------------------------------- mat-vec

struct KrylovState {
    int done;       // 1 once the residual estimate met tol (or the step limit was reached)
    int iters;      // Arnoldi steps taken
    double resid;   // |g_{j+1}| / beta0
    double beta0;
    double tol;     // relative residual target of this run
};

// Element strides between the work arrays of independent GMRES runs that
// advance together (run r = a grid index); all zero for a single run.
struct KBatch {
    int64_t basis;     // Krylov basis: (m + 1) n
    int64_t vec;       // work vector: n
    int64_t partial;   // partial dot products: nchunk 2 (m + 1)
    int64_t small;     // pending Hessenberg column and g: m + 1
    int64_t npart;     // norm partials: row blocks
    int64_t hess;      // triangular factor, and the Hessenberg matrix: m (m + 1)
    int64_t rot;       // Givens cosines and sines: m
    int64_t coef;      // Gram-Schmidt coefficients of the step: 2 m + 4
};


struct MtfArgs {
    int ne, ni;
    const void *op[2][4];    // [mesh][V, K, T, D], row stride op_ld(nv), complex128 or complex64
    const int32_t *pie_ptr, *pie_col, *pei_ptr, *pei_col;
    const double *pie_val, *pei_val;
    double c_ext_v, c_ext_w, c_int_v, c_int_w;   // 1/2, 1/2 re/ri, -1/2, -1/2 ri/re
    const int32_t *near_row[2], *near_j[2];      // near entries of each mesh, by row
    const double2 *corr[2];                      // [near entry][3]: V_ij - V_ji, D_ij - D_ji (j < i), T_ij - K_ji
    int sym_ts;                                  // tile edge of the symmetric tile form
    int no_mortar;                               // 1: no mortar terms (the combine skips them)
};

// ---- split-column form of the inverse-mass apply: a chunk of the vectors
// staged in LDS, per-chunk partial sums, fixed-order combine.  Rows of the
// two meshes form one grid; chunk widths are multiples of 64 chosen per mesh.

constexpr int MASS_CW_MAX = 1024;   // columns per chunk of the inverse-mass apply (upper bound)
constexpr int SPLIT_ROWS = 4;       // waves per workgroup
constexpr int MASS_RW64 = 4;        // rows per wave of the FP64 inverse-mass apply
constexpr int MASS_RW32 = 8;        // the same, FP32 storage

__host__ __device__ inline int split_nchunk(int nv, int cwmax) { return (nv + cwmax - 1) / cwmax; }
__host__ __device__ inline int split_cw(int nv, int cwmax)
{
    const int nc = split_nchunk(nv, cwmax);
    return ((nv + nc - 1) / nc + 63) / 64 * 64;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// streaming load of two adjacent complex64 entries (16 bytes)
__device__ inline float4 ld_stream2c(const float2 *p)
{
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

template <class R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

// ---- symmetric tile form: K is read in full and V, D only on and above the
// diagonal; T = K^T.  Exact up to rounding for the regular-pair part, whose
// element blocks are computed once per unordered pair and give V_ij = V_ji,
// D_ij = D_ji, T_ij = K_ji; the singular rule is applied to both orders of a
// vertex-sharing pair and is not symmetric to rounding, so the differences
// on those entries (the near entries) are added by the combine kernel.  One
// workgroup per pair of 128 x 128 tiles (a <= b): the tiles (a, b) of K, V, D
// and (b, a) of K are streamed once; products along rows reduce across the
// wave (DPP), products down columns accumulate per lane.  The partial sums of row
// tile R with column tile Cc go to part[Cc][row] (each written by exactly one
// workgroup) and are summed in a fixed order.

// Tile edge 128, two columns per lane: for complex128 the columns lane and
// lane + 64 (every 16-byte load of a wave covers 1 KB of a row, the two
// together the row's 2 KB), for complex64 two adjacent columns (one 16-byte
// load).  The wider rows of the tile keep DRAM accesses in longer runs than
// 64-column tiles do.
template <class E> constexpr int sym_tile() { return 128; }
constexpr int SYM_TS_MIN = 64;   // the smaller tile edge the tuner may pick (sizes the partial sums)
__host__ __device__ inline int sym_ntile(int nv, int ts) { return (nv + ts - 1) / ts; }

// task t -> tile pair (a, b), a <= b, in row-major order of the upper triangle
__device__ inline void sym_pair(int64_t t, int nt, int &a, int &b)
{
    int lo = 0, hi = nt - 1;
    while (lo < hi) {   // largest a with first(a) <= t, first(a) = a nt - a (a - 1) / 2
        const int mid = (lo + hi + 1) / 2;
        if ((int64_t)mid * nt - (int64_t)mid * (mid - 1) / 2 <= t) lo = mid; else hi = mid - 1;
    }
    a = lo;
    b = a + (int)(t - ((int64_t)a * nt - (int64_t)a * (a - 1) / 2));
}

__device__ inline double2 ld_entry(const double2 *p) { return ld_stream(p); }
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ inline float2 ld_entry(const float2 *p)   // one complex64 entry, streaming
{
    const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f *>(p));
    return make_float2(v.x, v.y);
}
__device__ inline float4 ld_entry2(const float2 *p) { return ld_stream2c(p); }   // two adjacent complex64

// Sum over the 64 lanes of a wave with DPP moves (row shifts within each row
// of 16 lanes, then row broadcasts 15 and 31); the total lands in lane 63.
template <int CTRL, int RM = 0xF> __device__ inline float dpp_mov(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, RM, 0xF, true));
}
template <int CTRL, int RM = 0xF> __device__ inline double dpp_mov(double v)
{
    int2 q = __builtin_bit_cast(int2, v);
    q.x = __builtin_amdgcn_update_dpp(0, q.x, CTRL, RM, 0xF, true);
    q.y = __builtin_amdgcn_update_dpp(0, q.y, CTRL, RM, 0xF, true);
    return __builtin_bit_cast(double, q);
}
template <class R> __device__ inline R wsum63(R v)
{
    v += dpp_mov<0x111>(v);        // row_shr:1
    v += dpp_mov<0x112>(v);        // row_shr:2
    v += dpp_mov<0x114>(v);        // row_shr:4
    v += dpp_mov<0x118>(v);        // row_shr:8  (lane 15 of each row: the row's sum)
    v += dpp_mov<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_mov<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}

template <class R> struct CAcc {   // complex accumulator in the arithmetic type R
    R x = 0, y = 0;
    template <class A, class B> __device__ void mac(const A &a, const B &b)
    {
        x += (R)a.x * b.x - (R)a.y * b.y;
        y += (R)a.x * b.y + (R)a.y * b.x;
    }
    template <class A, class B> __device__ void msub(const A &a, const B &b)
    {
        x -= (R)a.x * b.x - (R)a.y * b.y;
        y -= (R)a.x * b.y + (R)a.y * b.x;
    }
};

// entries (row, col0 .. col0 + CPL - 1) of one operator, zero outside nv x nv.
// Branch-free: an entry outside the matrix is loaded from a valid address
// (row and column clamped) and replaced by zero, so the loads of a row issue
// back to back and the compiler can count them in flight.
template <class E, class C, int CPL>
__device__ inline void ld_cols(const E *M, int64_t ld, int row, int col0, int nv, C (&out)[CPL])
{
    using R = decltype(C::x);
    const bool ok = row < nv && col0 < nv;
    const E *p = M + (int64_t)min(row, nv - 1) * ld + (col0 < nv ? col0 : 0);
    if constexpr (sizeof(E) == 16 && CPL == 2) {   // columns col0 and col0 + 64
        const E e0 = ld_entry(p);
        out[0] = ok ? C{(R)e0.x, (R)e0.y} : C{0, 0};
        const bool ok1 = row < nv && col0 + 64 < nv;
        const E *p1 = M + (int64_t)min(row, nv - 1) * ld + (col0 + 64 < nv ? col0 + 64 : 0);
        const E e1 = ld_entry(p1);
        out[1] = ok1 ? C{(R)e1.x, (R)e1.y} : C{0, 0};
    } else if constexpr (CPL == 1) {
        const E e = ld_entry(p);
        out[0] = ok ? C{(R)e.x, (R)e.y} : C{0, 0};
    } else {   // col0 even and the row stride a multiple of 16: the pair is in the row
        const float4 e = ld_entry2(p);
        out[0] = ok ? C{(R)e.x, (R)e.y} : C{0, 0};
        out[1] = ok && col0 + 1 < nv ? C{(R)e.z, (R)e.w} : C{0, 0};
    }
}

// Tile partials are written with non-temporal stores: the combine kernel reads
// them once, and stores that allocate in L2 slowed the operator stream that
// shares the memory channels (C3 FP64: 927 -> 891 us per product, the same bits).
typedef double v4d_nt __attribute__((ext_vector_type(4)));
__device__ inline void st_part(double4 *p, double a, double b, double c, double d)
{
    __builtin_nontemporal_store(v4d_nt{a, b, c, d}, reinterpret_cast<v4d_nt *>(p));
}

template <class E, class R, int TS>
__global__ __launch_bounds__(256) void mtf_sym_tile_kernel(MtfArgs A, const double2 *__restrict__ x,
                                                           double4 *__restrict__ part,
                                                           const KrylovState *__restrict__ st)
{
    using C = typename Cx<R>::T;
    constexpr int CPL = TS / 64, RPW = TS / 4;   // columns per lane, rows per wave
    if (st && st->done) return;
    __shared__ C sva[TS], swa[TS], svb[TS], swb[TS];
    __shared__ C rowres[3][TS];
    __shared__ C colres[4][3][TS];
    int64_t t = blockIdx.x;
    const int nte = sym_ntile(A.ne, TS), nti = sym_ntile(A.ni, TS);
    const int64_t te = (int64_t)nte * (nte + 1) / 2;
    const bool ext = t < te;
    if (!ext) t -= te;
    const int nt = ext ? nte : nti;
    int a, b;
    sym_pair(t, nt, a, b);
    const int nv = ext ? A.ne : A.ni;
    const int mi = ext ? 0 : 1;
    const E *Vm = static_cast<const E *>(A.op[mi][0]), *Km = static_cast<const E *>(A.op[mi][1]);
    const E *Dm = static_cast<const E *>(A.op[mi][3]);
    const int64_t ld = op_ld(nv);
    const double2 *xv = ext ? x : x + 2 * A.ne, *xw = xv + nv;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const C zero{0, 0};
    for (int q = tid; q < TS; q += 256) {
        const int ia = a * TS + q, ib = b * TS + q;
        sva[q] = ia < nv ? C{(R)xv[ia].x, (R)xv[ia].y} : zero;
        swa[q] = ia < nv ? C{(R)xw[ia].x, (R)xw[ia].y} : zero;
        svb[q] = ib < nv ? C{(R)xv[ib].x, (R)xv[ib].y} : zero;
        swb[q] = ib < nv ? C{(R)xw[ib].x, (R)xw[ib].y} : zero;
    }
    __syncthreads();
    const bool diag = a == b;
    constexpr bool split = sizeof(E) == 16;    // complex128: columns lane + 64 u, else adjacent pairs
    const int c0 = split ? lane : lane * CPL;  // this lane's first column inside the tile
    const int j0 = b * TS + c0, ja0 = a * TS + c0;
    auto colof = [&](int u) { return split ? c0 + 64 * u : c0 + u; };
    C vb[CPL], wb[CPL], va[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) { vb[u] = svb[colof(u)]; wb[u] = swb[colof(u)]; va[u] = sva[colof(u)]; }
    CAcc<R> c1b[CPL], c2b[CPL], c2a[CPL];
#pragma unroll 1
    for (int rr = 0; rr < RPW; ++rr) {
        const int r = wave * RPW + rr;
        const int i = a * TS + r, ib = b * TS + r;
        C kab[CPL], vab[CPL], dab[CPL], kba[CPL];
        ld_cols<E, C, CPL>(Km, ld, i, j0, nv, kab);
        ld_cols<E, C, CPL>(Vm, ld, i, j0, nv, vab);
        ld_cols<E, C, CPL>(Dm, ld, i, j0, nv, dab);
        if (!diag) ld_cols<E, C, CPL>(Km, ld, ib, ja0, nv, kba);
        else
#pragma unroll
            for (int u = 0; u < CPL; ++u) kba[u] = zero;
        const C wi = swa[r], vi = sva[r], wbr = swb[r];
        CAcc<R> y1, y2, y1b;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int c = colof(u);
            // rows of tile a: y1 -= K v, y1 += V w, y2 += D v (V, D on and above the diagonal)
            y1.msub(kab[u], vb[u]);
            if (!diag || c >= r) {
                y1.mac(vab[u], wb[u]);
                y2.mac(dab[u], vb[u]);
            }
            // rows of tile b (column c): y2 += K^T w; y1 += V^T w, y2 += D^T v strictly above the diagonal
            c2b[u].mac(kab[u], wi);
            if (!diag || c > r) {
                c1b[u].mac(vab[u], wi);
                c2b[u].mac(dab[u], vi);
            }
            // tile (b, a) of K: rows of b: y1 -= K v_a; rows of a (column c): y2 += K^T w_b
            y1b.msub(kba[u], va[u]);
            c2a[u].mac(kba[u], wbr);
        }
        const R s0 = wsum63(y1.x), s1 = wsum63(y1.y), s2 = wsum63(y2.x), s3 = wsum63(y2.y), s4 = wsum63(y1b.x),
                s5 = wsum63(y1b.y);
        if (lane == 63) {
            rowres[0][r] = C{s0, s1};
            rowres[1][r] = C{s2, s3};
            rowres[2][r] = C{s4, s5};
        }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        colres[wave][0][colof(u)] = C{c1b[u].x, c1b[u].y};
        colres[wave][1][colof(u)] = C{c2b[u].x, c2b[u].y};
        colres[wave][2][colof(u)] = C{c2a[u].x, c2a[u].y};
    }
    __syncthreads();
    for (int r = tid; r < TS; r += 256) {
        double c1x = 0, c1y = 0, c2x = 0, c2y = 0, c3x = 0, c3y = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            c1x += (double)colres[w][0][r].x; c1y += (double)colres[w][0][r].y;
            c2x += (double)colres[w][1][r].x; c2y += (double)colres[w][1][r].y;
            c3x += (double)colres[w][2][r].x; c3y += (double)colres[w][2][r].y;
        }
        const int64_t stride = (int64_t)A.ne + A.ni;
        const int off = ext ? 0 : A.ne;
        const int i = a * TS + r, ib = b * TS + r;
        if (diag) {
            if (i < nv)
                st_part(part + (int64_t)a * stride + off + i, (double)rowres[0][r].x + c1x, (double)rowres[0][r].y + c1y,
                                                                   (double)rowres[1][r].x + c2x, (double)rowres[1][r].y + c2y);
        } else {
            if (i < nv)
                st_part(part + (int64_t)b * stride + off + i, (double)rowres[0][r].x, (double)rowres[0][r].y,
                                                                   (double)rowres[1][r].x + c3x, (double)rowres[1][r].y + c3y);
            if (ib < nv)
                st_part(part + (int64_t)a * stride + off + ib, (double)rowres[2][r].x + c1x, (double)rowres[2][r].y + c1y,
                                                                    c2x, c2y);
        }
    }
}

// y rows = sum of the tile partials of the row + the near-entry corrections
// + mortar coupling.  16 lanes per row (one DPP row): each lane takes every
// 16th term of the three sums, and a fixed reduction tree within the row
// finishes them (deterministic).
template <class R> __device__ inline R rsum15(R v)   // sum over the 16 lanes of a DPP row, in lane 15
{
    v += dpp_mov<0x111>(v);
    v += dpp_mov<0x112>(v);
    v += dpp_mov<0x114>(v);
    v += dpp_mov<0x118>(v);
    return v;
}

__global__ __launch_bounds__(256) void mtf_sym_combine_kernel(MtfArgs A, const double2 *__restrict__ x,
                                                              const double4 *__restrict__ part,
                                                              double2 *__restrict__ y,
                                                              const KrylovState *__restrict__ st)
{
    if (st && st->done) return;
    const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int l16 = threadIdx.x & 15;
    const bool live = row < A.ne + A.ni;   // whole DPP rows are live or not: no divergence inside a reduction
    const bool ext = row < A.ne;
    const int mi = ext ? 0 : 1;
    const int i = live ? (ext ? row : row - A.ne) : 0;
    const int nv = ext ? A.ne : A.ni;
    double ar = 0, ai = 0, br = 0, bi = 0, sr = 0, si = 0, tr = 0, ti = 0;
    if (live) {
        const int nt = sym_ntile(nv, A.sym_ts);
        const int64_t pstride = (int64_t)A.ne + A.ni;
        for (int c = l16; c < nt; c += 16) {
            const double4 q = part[(int64_t)c * pstride + row];
            ar += q.x; ai += q.y; br += q.z; bi += q.w;
        }
        const double2 *xm = ext ? x : x + 2 * A.ne;   // this mesh's [v; w]
        for (int e = A.near_row[mi][i] + l16; e < A.near_row[mi][i + 1]; e += 16) {
            const int jn = A.near_j[mi][e];
            const double2 cv = A.corr[mi][3 * e], cd = A.corr[mi][3 * e + 1], ct = A.corr[mi][3 * e + 2];
            const double2 vj = xm[jn], wj = xm[nv + jn];
            ar += cv.x * wj.x - cv.y * wj.y; ai += cv.x * wj.y + cv.y * wj.x;
            br += cd.x * vj.x - cd.y * vj.y + ct.x * wj.x - ct.y * wj.y;
            bi += cd.x * vj.y + cd.y * vj.x + ct.x * wj.y + ct.y * wj.x;
        }
        if (!A.no_mortar) {
            const int32_t *pp = ext ? A.pei_ptr : A.pie_ptr;
            const int32_t *pc = ext ? A.pei_col : A.pie_col;
            const double *pv = ext ? A.pei_val : A.pie_val;
            const double2 *cvx = ext ? x + 2 * A.ne : x;
            const int nother = ext ? A.ni : A.ne;
            const double2 *cwx = cvx + nother;
            for (int q = pp[i] + l16; q < pp[i + 1]; q += 16) {
                const double pvq = pv[q];
                const double2 av = cvx[pc[q]], bw = cwx[pc[q]];
                sr += pvq * av.x; si += pvq * av.y; tr += pvq * bw.x; ti += pvq * bw.y;
            }
        }
    }
    ar = rsum15(ar); ai = rsum15(ai); br = rsum15(br); bi = rsum15(bi);
    sr = rsum15(sr); si = rsum15(si); tr = rsum15(tr); ti = rsum15(ti);
    if (live && l16 == 15) {
        const double fv = ext ? A.c_ext_v : A.c_int_v, fw = ext ? A.c_ext_w : A.c_int_w;
        double2 *ya = ext ? y : y + 2 * A.ne;
        ya[i] = make_double2(ar + fv * sr, ai + fv * si);
        ya[i + nv] = make_double2(br + fw * tr, bi + fw * ti);
    }
}

// corr[e] of every near entry (i, j) of one mesh from the stored operators
template <class E>
__global__ void sym_corr_kernel(int nv, int nn, const int32_t *__restrict__ ni_, const int32_t *__restrict__ nj_,
                                const E *__restrict__ V, const E *__restrict__ K, const E *__restrict__ T,
                                const E *__restrict__ D, double2 *__restrict__ corr)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    const int64_t ld = op_ld(nv);
    const int i = ni_[e], jn = nj_[e];
    const int64_t o = i * ld + jn, ot = jn * ld + i;
    double2 cv = make_double2(0, 0), cd = cv;
    if (jn < i) {
        cv = make_double2((double)V[o].x - (double)V[ot].x, (double)V[o].y - (double)V[ot].y);
        cd = make_double2((double)D[o].x - (double)D[ot].x, (double)D[o].y - (double)D[ot].y);
    }
    const double2 ct = make_double2((double)T[o].x - (double)K[ot].x, (double)T[o].y - (double)K[ot].y);
    corr[3 * (int64_t)e] = cv;
    corr[3 * (int64_t)e + 1] = cd;
    corr[3 * (int64_t)e + 2] = ct;
}

bem_status launch_sym_corrections(bem_problem *p, int mesh, hipStream_t st)
{
    const bem_mesh *m = mesh == 0 ? p->ext : p->inte;
    const int nv = (int)m->h.nv, nn = (int)m->h.near_i.size();
    bem_status s = dev_alloc(p->ctx, p->corr[mesh], (size_t)std::max(nn, 1) * 3 * sizeof(double2));
    if (s) return s;
    if (nn == 0) return BEM_OK;
    const dim3 g((nn + 255) / 256);
    if (p->prec == BEM_C128)
        hipLaunchKernelGGL(sym_corr_kernel<double2>, g, dim3(256), 0, st, nv, nn, m->d.near_i.as<int32_t>(),
                           m->d.near_j.as<int32_t>(), p->ops[mesh][0].as<double2>(), p->ops[mesh][1].as<double2>(),
                           p->ops[mesh][2].as<double2>(), p->ops[mesh][3].as<double2>(), p->corr[mesh].as<double2>());
    else
        hipLaunchKernelGGL(sym_corr_kernel<float2>, g, dim3(256), 0, st, nv, nn, m->d.near_i.as<int32_t>(),
                           m->d.near_j.as<int32_t>(), p->ops[mesh][0].as<float2>(), p->ops[mesh][1].as<float2>(),
                           p->ops[mesh][2].as<float2>(), p->ops[mesh][3].as<float2>(), p->corr[mesh].as<double2>());
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

// part[chunk][row] = M^-1 row chunk applied to the mesh's two vectors; the
// inverse is stored in FP64 (pairs of entries per lane) or FP32 (quads),
// accumulation in FP64 either way.  Each wave applies RW rows, so that the
// staged vector entries read from LDS serve RW rows of M^-1 (LDS traffic
// per HBM byte falls by RW).  Padding columns of M^-1 are zero and the
// staged vectors are zero past the chunk's end.
template <class MT, int RW>
__global__ __launch_bounds__(256) void mass_apply_part_kernel(int ne, int ni, const MT *__restrict__ Me_inv,
                                                              const MT *__restrict__ Mi_inv,
                                                              const double2 *__restrict__ y, double4 *__restrict__ part,
                                                              const KrylovState *__restrict__ st)
{
    constexpr bool f32 = sizeof(MT) == 4;
    constexpr int VW = f32 ? 4 : 2;   // entries per lane load (16 bytes)
    constexpr int ROWS = SPLIT_ROWS * RW;
    if (st && st->done) return;
    __shared__ double2 ys[2 * MASS_CW_MAX];
    const int te = (ne + ROWS - 1) / ROWS;
    const bool ext = (int)blockIdx.x < te;
    const int nv = ext ? ne : ni;
    const int chunk = blockIdx.y;
    if (chunk >= split_nchunk(nv, MASS_CW_MAX)) return;
    const int cw = split_cw(nv, MASS_CW_MAX);
    const int c0 = chunk * cw, c1 = min(nv, c0 + cw), ncol = c1 - c0;
    const double2 *ya = ext ? y : y + 2 * ne;
    const double2 *yb = ya + nv;
    for (int t = threadIdx.x; t < cw; t += blockDim.x) {
        ys[t] = t < ncol ? ya[c0 + t] : make_double2(0, 0);
        ys[MASS_CW_MAX + t] = t < ncol ? yb[c0 + t] : make_double2(0, 0);
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = (ext ? blockIdx.x : blockIdx.x - te) * ROWS + wave * RW;
    if (i0 >= nv) return;
    const int ld = minv_ld(nv, f32);
    const MT *Mbase = (ext ? Me_inv : Mi_inv) + c0;   // c0: multiple of 64
    const MT *Mr[RW];
#pragma unroll
    for (int u = 0; u < RW; ++u) Mr[u] = Mbase + (int64_t)min(i0 + u, nv - 1) * ld;   // rows past nv: unused
    double ar[RW], ai[RW], br[RW], bi[RW];
#pragma unroll
    for (int u = 0; u < RW; ++u) ar[u] = ai[u] = br[u] = bi[u] = 0.0;
    constexpr int UNR = f32 ? 1 : 2;   // two column steps in flight for FP64 rows (measured: FP32 prefers one)
#pragma unroll UNR
    for (int j = VW * lane; j < ncol; j += VW * 64) {
        double m[RW][VW];
#pragma unroll
        for (int u = 0; u < RW; ++u) {
            if constexpr (f32) {
                const v4f q = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(Mr[u] + j));
                m[u][0] = q.x; m[u][1] = q.y; m[u][2] = q.z; m[u][3] = q.w;
            } else {
                const v2d q = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(Mr[u] + j));
                m[u][0] = q.x; m[u][1] = q.y;
            }
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const double2 a = ys[j + e], b = ys[MASS_CW_MAX + j + e];
#pragma unroll
            for (int u = 0; u < RW; ++u) {
                ar[u] += m[u][e] * a.x; ai[u] += m[u][e] * a.y; br[u] += m[u][e] * b.x; bi[u] += m[u][e] * b.y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RW; ++u) {
        const double sar = wave_sum(ar[u]), sai = wave_sum(ai[u]), sbr = wave_sum(br[u]), sbi = wave_sum(bi[u]);
        if (lane == 0 && i0 + u < nv) {
            const int row = ext ? i0 + u : ne + i0 + u;
            part[(int64_t)chunk * (ne + ni) + row] = make_double4(sar, sai, sbr, sbi);
        }
    }
}

__global__ __launch_bounds__(256) void mass_combine_kernel(int ne, int ni, const double4 *__restrict__ part,
                                                           double2 *__restrict__ z, const KrylovState *__restrict__ st)
{
    if (st && st->done) return;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= ne + ni) return;
    const bool ext = row < ne;
    const int i = ext ? row : row - ne;
    const int nv = ext ? ne : ni;
    double ar = 0, ai = 0, br = 0, bi = 0;
    const int nch = split_nchunk(nv, MASS_CW_MAX);
    for (int c = 0; c < nch; ++c) {
        const double4 q = part[(int64_t)c * (ne + ni) + row];
        ar += q.x; ai += q.y; br += q.z; bi += q.w;
    }
    double2 *za = ext ? z : z + 2 * ne;
    za[i] = make_double2(ar, ai);
    za[i + nv] = make_double2(br, bi);
}

// ---- sparse inverse-mass apply: Chebyshev iteration on diag(M)^-1 M, whose
// spectrum lies in [1/2, 2] on every P1 mesh (error 4 3^-k after k steps),
// s steps per launch on the overlapping patches of ChebTables: a workgroup
// loads its patch's iterate x, residual r and direction d (from y in the
// first launch), keeps x, r and its rows of M (ELL, up to W entries) in
// registers and d in LDS, and at step t updates the vertices within s - t
// edges of its owned range, which read only vertices updated at step t - 1.
// The owned range's state goes to the other work set (launches alternate
// between two, so that no patch reads what another writes in the same
// launch), and in the last launch x goes to z.  Fixed summation order:
// deterministic.
struct ChebArgs {
    const int32_t *pmesh, *vbeg, *cnt, *vert;
    const uint16_t *ecol;
    const double *dinv, *eval;
    int s, w;           // steps per launch, ELL width
    int nvm[2];         // vertices of each mesh
    int64_t base[2];    // offset of each mesh's first vector in y, z and the work vectors
    int64_t wn;         // length of one work vector
};

constexpr double CHEB_THETA = 1.25, CHEB_DELTA = 0.75;   // centre and half-width of [1/2, 2]

template <int RPT, int W>
__global__ __launch_bounds__(1024) void mass_cheb_kernel(ChebArgs A, int part0, int first, int last, int nsteps,
                                                          double rho0, const double2 *__restrict__ y, int64_t ystride,
                                                          double2 *__restrict__ z, int64_t zstride,
                                                          const double2 *__restrict__ win, double2 *__restrict__ wout,
                                                          int64_t wstride, const KrylovState *__restrict__ st)
{
    __shared__ double2 dsh[CHEB_LMAX];
    const int run = blockIdx.z;
    if (st && st[run].done) return;
    const int p = part0 + (int)blockIdx.x, vec = blockIdx.y;
    const int m = A.pmesh[p];
    const int64_t off = A.base[m] + (int64_t)vec * A.nvm[m];
    const int vb = A.vbeg[p], L = A.vbeg[p + 1] - vb;
    const int32_t *cnt = A.cnt + (int64_t)p * (A.s + 1);
    const int rows = cnt[A.s - 1];   // rows with entries: within s - 1 edges
    const uint16_t *ec = A.ecol + (int64_t)A.w * vb;
    const double *ev = A.eval + (int64_t)A.w * vb;
    const double2 *Xi = win + run * wstride, *Ri = Xi + A.wn, *Di = Ri + A.wn;
    const double2 *yr = y + run * ystride;
    const int tid = threadIdx.x;
    double xr[RPT], xi[RPT], rr[RPT], ri[RPT], dr[RPT], di[RPT], dg[RPT];
    int cc[RPT][W];
    double vv[RPT][W];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int l = tid + 1024 * k;
        xr[k] = xi[k] = rr[k] = ri[k] = dr[k] = di[k] = dg[k] = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const bool has = l < rows && q < A.w;
            cc[k][q] = has ? (int)ec[(int64_t)q * L + l] : 0;
            vv[k][q] = has ? ev[(int64_t)q * L + l] : 0.0;
        }
        if (l < L) {
            const int64_t g = off + A.vert[vb + l];
            dg[k] = A.dinv[vb + l];
            if (first) {
                const double2 yy = yr[g];
                rr[k] = yy.x;
                ri[k] = yy.y;
                dr[k] = dg[k] * yy.x / CHEB_THETA;
                di[k] = dg[k] * yy.y / CHEB_THETA;
            } else {
                const double2 a = Xi[g], b = Ri[g], c = Di[g];
                xr[k] = a.x; xi[k] = a.y; rr[k] = b.x; ri[k] = b.y; dr[k] = c.x; di[k] = c.y;
            }
            dsh[l] = make_double2(dr[k], di[k]);
        }
    }
    const double sigma1 = CHEB_THETA / CHEB_DELTA;
    double rho = rho0;
    __syncthreads();
    for (int t = 1; t <= nsteps; ++t) {
        const int act = cnt[A.s - t];
        double ar[RPT], ai[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            ar[k] = ai[k] = 0.0;
            if (tid + 1024 * k < act)
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const double2 dd = dsh[cc[k][q]];
                    ar[k] += vv[k][q] * dd.x;
                    ai[k] += vv[k][q] * dd.y;
                }
        }
        __syncthreads();
        const double rho_new = 1.0 / (2.0 * sigma1 - rho);
        const double c1 = rho_new * rho, c2 = 2.0 * rho_new / CHEB_DELTA;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int l = tid + 1024 * k;
            if (l < act) {
                xr[k] += dr[k];
                xi[k] += di[k];
                rr[k] -= ar[k];
                ri[k] -= ai[k];
                dr[k] = c1 * dr[k] + c2 * dg[k] * rr[k];
                di[k] = c1 * di[k] + c2 * dg[k] * ri[k];
                dsh[l] = make_double2(dr[k], di[k]);
            }
        }
        rho = rho_new;
        __syncthreads();
    }
    const int own = cnt[0];
    double2 *Xo = wout + run * wstride, *Ro = Xo + A.wn, *Do = Ro + A.wn;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int l = tid + 1024 * k;
        if (l < own) {
            const int64_t g = off + A.vert[vb + l];
            if (last) {
                z[run * zstride + g] = make_double2(xr[k], xi[k]);
            } else {
                Xo[g] = make_double2(xr[k], xi[k]);
                Ro[g] = make_double2(rr[k], ri[k]);
                Do[g] = make_double2(dr[k], di[k]);
            }
        }
    }
}

static inline dim3 split_grid(int ne, int ni, int cwmax, int rw = 1)
{
    const int rows = SPLIT_ROWS * rw;
    const int tiles = (ne + rows - 1) / rows + (ni + rows - 1) / rows;
    return dim3(tiles, std::max(split_nchunk(ne, cwmax), split_nchunk(ni, cwmax)));
}

// ------------------------------------------------------ Krylov kernels
//
// Arnoldi (Sec. 5.1: GMRES without restart) with classical Gram-Schmidt and
// a re-orthogonalisation delayed by one step (the DCGS2 scheme of
// Swirydowicz et al., 2021, and Bielich et al., 2022): every new vector is
// orthogonalised twice, as in CGS2, but the second pass of step j shares
// its sweeps over the basis with the first pass of step j + 1, so a step
// reads the basis twice instead of four times.  Step j, V = v_0 .. v_{j-1}:
//   slot j of the basis holds u_j (one Gram-Schmidt pass, unit norm) and
//   w = M^-1 A u_j;
//   dots:      a = V^H u_j, alpha = |u_j|^2, b = V^H w, gamma = u_j^H w;
//   hess:      nu = sqrt(alpha - |a|^2), so that v_j = (u_j - V a) / nu;
//              the pending column j-1 of the Hessenberg matrix becomes
//              h_{j-1} + beta_{j-1} a over the subdiagonal beta_{j-1} nu
//              (because u_j = nu v_j + V a), then its Givens rotation and the
//              residual estimate of the j-dimensional space;
//              c_j = (gamma - a^H b) / nu = v_j^H w;
//   update:    v_j into slot j and y = w - V b - v_j c_j into slot j+1;
//              since w = nu M^-1 A v_j + M^-1 A V a and M^-1 A V = [V v_j] Hbar,
//              M^-1 A v_j = [V v_j] h_j + y / nu with the pending column
//              h_j = ([b; c_j] - Hbar a) / nu, formed by extra waves;
//   normalise: u_{j+1} = y / |y| and beta_j = |y| / nu.
// The residual estimate of dimension j appears in step j (one operator
// product after the one that made the space).  Sums run in a fixed order;
// every kernel returns at once when the state says the run has converged, so
// steps issued ahead of the host's convergence check cost only their launch.

// Rows per partial dot product: n / 8 rounded up to 256, between 1024 and
// 4096 (at most about 9 partials per coefficient at large n, where the
// Givens kernel sums them; at small n more, shorter chunks, so that more
// waves share the sweep).
__host__ __device__ inline int cgs_chunk(int n)
{
    const int c = ((n + 7) / 8 + 255) / 256 * 256;
    return c < 1024 ? 1024 : (c > 4096 ? 4096 : c);
}
constexpr int UPD_ROWS = 64;      // rows per workgroup of the update sweep
constexpr int MAXIT_CAP = 3000;   // Hessenberg column, rotations and g staged in LDS

// partial[chunk][c] = sum over the chunk's rows of conj(V_c) u_j and
// partial[chunk][j + 1 + c] = that of conj(V_c) w, for c = 0..j (slot j is
// u_j itself: alpha and gamma).  One wave per (chunk, CPW consecutive
// columns): with CPW = 2 the wave reads the chunks of u_j and w once for
// both columns; each column's sum runs over the same rows in the same order
// either way.  Grid (nchunk, ceil((j + 1) / (4 CPW)), runs), or larger (the
// extra waves return).
template <int CPW>
__global__ __launch_bounds__(256) void dgs_dots_kernel(int n, int j, const int *__restrict__ jb,
                                                       const double2 *__restrict__ Vb, const double2 *__restrict__ w,
                                                       double2 *__restrict__ partial,
                                                       const KrylovState *__restrict__ st, KBatch B)
{
    const int run = blockIdx.z;
    if (st[run].done) return;
    if (jb) j += *jb;
    Vb += run * B.basis;
    w += run * B.vec;
    partial += run * B.partial;
    const int lane = threadIdx.x & 63;
    const int c = CPW * (blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));   // wave-uniform
    if (c > j) return;
    const int nc = min(CPW, j + 1 - c);   // columns of this wave
    const int chunk = cgs_chunk(n);
    const int r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
    const double2 *u = Vb + (int64_t)j * n;
    const double2 *vc[CPW];
#pragma unroll
    for (int q = 0; q < CPW; ++q) vc[q] = Vb + (int64_t)min(c + q, j) * n;   // a missing second column repeats u_j, unused
    double ur[CPW], ui[CPW], wr[CPW], wi[CPW];
#pragma unroll
    for (int q = 0; q < CPW; ++q) ur[q] = ui[q] = wr[q] = wi[q] = 0;
#pragma unroll 4
    for (int r = r0 + lane; r < r1; r += 64) {
        double2 av[CPW];
#pragma unroll
        for (int q = 0; q < CPW; ++q) av[q] = vc[q][r];
        const double2 x = u[r], y = w[r];
#pragma unroll
        for (int q = 0; q < CPW; ++q) {
            const double2 a = av[q];
            ur[q] += a.x * x.x + a.y * x.y;
            ui[q] += a.x * x.y - a.y * x.x;
            wr[q] += a.x * y.x + a.y * y.y;
            wi[q] += a.x * y.y - a.y * y.x;
        }
    }
    double2 *pc = partial + (int64_t)blockIdx.x * 2 * (j + 1);
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
        const double sur = wave_sum(ur[q]), sui = wave_sum(ui[q]), swr = wave_sum(wr[q]), swi = wave_sum(wi[q]);
        if (lane == 0 && q < nc) {
            pc[c + q] = make_double2(sur, sui);
            pc[j + 1 + c + q] = make_double2(swr, swi);
        }
    }
}

__device__ inline double2 cconj_mul(double2 a, double2 b)   // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Sums of the partials into coef ([0, j) a, [j] alpha, [j + 1, 2j + 1) b,
// [2j + 1] gamma); nu; the final column j - 1 of the Hessenberg matrix
// (kept row-major in H, row stride m) and, by the first wave, its Givens rotation
// (the earlier rotations as a scanned affine recurrence),
// g and the residual estimate; then coef[j] = (1 / nu, nu) and coef[2j + 1] =
// c_j for the update.  coef[2m + 3] holds beta_{j-1}.  One workgroup per run;
// dynamic LDS for at least 3 j + 1 complex values.
__global__ __launch_bounds__(256) void dgs_hess_kernel(int j, const int *__restrict__ jb, int m, int nchunk,
                                                       const double2 *__restrict__ partial,
                                                       double2 *__restrict__ coef, const double2 *__restrict__ hsum,
                                                       double2 *__restrict__ H, double2 *__restrict__ R,
                                                       double2 *__restrict__ g, double2 *__restrict__ cs,
                                                       double2 *__restrict__ sn, KrylovState *__restrict__ st, KBatch B)
{
    const int run = blockIdx.x;
    st += run;
    if (st->done) return;
    if (jb) j += *jb;
    partial += run * B.partial;
    coef += run * B.coef;
    hsum += run * B.small;
    H += run * B.hess;
    R += run * B.hess;
    g += run * B.small;
    cs += run * B.rot;
    sn += run * B.rot;
    const int tid = threadIdx.x, nk = 2 * (j + 1);
    for (int k = tid; k < nk; k += 256) {
        double2 sum = make_double2(0, 0);
#pragma unroll 8
        for (int c = 0; c < nchunk; ++c) sum = cadd(sum, partial[(int64_t)c * nk + k]);
        coef[k] = sum;
    }
    __syncthreads();
    __shared__ double red[3][4];
    double aa = 0, abr = 0, abi = 0;
    for (int k = tid; k < j; k += 256) {
        const double2 a = coef[k], b = coef[j + 1 + k];
        aa += a.x * a.x + a.y * a.y;
        abr += a.x * b.x + a.y * b.y;
        abi += a.x * b.y - a.y * b.x;
    }
    aa = wave_sum(aa);
    abr = wave_sum(abr);
    abi = wave_sum(abi);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = aa;
        red[1][tid >> 6] = abr;
        red[2][tid >> 6] = abi;
    }
    __syncthreads();
    aa = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    abr = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    abi = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    const double nu2 = coef[j].x - aa;
    const double nu = nu2 > 0 ? sqrt(nu2) : 0.0;
    const double2 gamma = coef[2 * j + 1];
    const double beta_prev = coef[2 * m + 3].x;
    extern __shared__ double2 sh[];   // [h: j + 1][cs: j][sn: j]
    double2 *hl = sh, *csl = sh + (j + 1), *snl = csl + j;
    // final column j - 1: rows 0..j-1 h_{j-1} + beta_{j-1} a, row j beta_{j-1} nu
    const double sub = beta_prev * nu;
    if (j > 0) {
        for (int i = tid; i < j; i += 256) {
            const double2 a = coef[i], h = hsum[i];
            const double2 v = make_double2(h.x + beta_prev * a.x, h.y + beta_prev * a.y);
            hl[i] = v;
            H[(int64_t)i * m + (j - 1)] = v;
        }
        if (tid == 0) H[(int64_t)j * m + (j - 1)] = make_double2(sub, 0.0);
        for (int i = tid; i < j - 1; i += 256) { csl[i] = cs[i]; snl[i] = sn[i]; }
    }
    __syncthreads();   // every thread has read coef before thread 0 rewrites it
    if (tid >= 64) return;
    const int lane = tid;
    bool done = false;
    if (j > 0) {
        // Givens rotations 0 .. jc-1 applied to column jc = j - 1.  With s_i
        // real they form the affine recurrence t_{i+1} = -s_i t_i + c_i h_{i+1}
        // (t_0 = h_0; entry i of the rotated column is conj(c_i) t_i + s_i h_{i+1}),
        // so one wave takes it in segments: each lane composes the maps of its
        // steps, the composites are scanned across the wave, and each lane
        // replays its steps from its start value.
        const int jc = j - 1;
        double2 *col = R + (int64_t)jc * (m + 1);
        const int L = (jc + 63) / 64;
        const int i0 = min(jc, lane * L), i1 = min(jc, i0 + L);
        double P = 1.0, Qx = 0.0, Qy = 0.0;   // t_end = P t_start + Q over the lane's steps
        for (int i = i0; i < i1; ++i) {
            const double a = -snl[i].x;
            const double2 cb = cmul(csl[i], hl[i + 1]);
            P *= a;
            Qx = a * Qx + cb.x;
            Qy = a * Qy + cb.y;
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {   // inclusive scan: the maps of lanes 0..lane, later after earlier
            const double Pp = __shfl_up(P, off, 64), Qpx = __shfl_up(Qx, off, 64), Qpy = __shfl_up(Qy, off, 64);
            if (lane >= off) {
                Qx = P * Qpx + Qx;
                Qy = P * Qpy + Qy;
                P *= Pp;
            }
        }
        const double Pe = __shfl_up(P, 1, 64), Qex = __shfl_up(Qx, 1, 64), Qey = __shfl_up(Qy, 1, 64);
        const double2 h0 = hl[0];
        double2 t = lane == 0 ? h0 : make_double2(Pe * h0.x + Qex, Pe * h0.y + Qey);
        for (int i = i0; i < i1; ++i) {
            const double2 b = hl[i + 1], c = csl[i];
            const double sv = snl[i].x;
            const double2 ca = cconj_mul(c, t), cb = cmul(c, b);
            col[i] = make_double2(ca.x + sv * b.x, ca.y + sv * b.y);
            t = make_double2(cb.x - sv * t.x, cb.y - sv * t.y);
        }
        // lanes past the last step hold t_jc unchanged; lane 63 always does
        t.x = __shfl(t.x, 63, 64);
        t.y = __shfl(t.y, 63, 64);
        if (lane == 0) {
            const double den = sqrt(t.x * t.x + t.y * t.y + sub * sub);
            double2 c = make_double2(1, 0), sv = make_double2(0, 0);
            if (den > 0) { c = make_double2(t.x / den, t.y / den); sv = make_double2(sub / den, 0.0); }
            cs[jc] = c;
            sn[jc] = sv;
            col[jc] = make_double2(den, 0.0);
            const double2 gj = g[jc];
            g[jc] = cconj_mul(c, gj);
            const double2 sg = cmul(sv, gj);
            g[jc + 1] = make_double2(-sg.x, -sg.y);
            const double res = sqrt(sg.x * sg.x + sg.y * sg.y) / st->beta0;
            st->resid = res;
            st->iters = j;
            done = res <= st->tol || sub == 0.0 || j >= m;
        }
    }
    if (lane != 0) return;
    if (!(nu > 0)) done = true;   // u_j in the span of V: the space is invariant
    if (done) {
        st->done = 1;
        return;
    }
    const double inv = 1.0 / nu;
    coef[j] = make_double2(inv, nu);
    coef[2 * j + 1] = make_double2((gamma.x - abr) * inv, (gamma.y - abi) * inv);
}

// Blocks [0, nupd): 64 rows each (four waves split the basis columns, summed
// in LDS in a fixed order); v_j = (u_j - V a) / nu into slot j, y = w - V b -
// v_j c_j into slot j + 1, partial |y|^2 per block.  Blocks from nupd on: one
// wave per row r <= j of the pending column, h_j[r] = ([b; c_j][r] -
// sum over i >= r - 1 of H[r][i] a_i) / nu.  Grid (nupd + ceil((j + 1) / 4), runs),
// or larger (the extra waves return).
__global__ __launch_bounds__(256) void dgs_update_kernel(int n, int j, const int *__restrict__ jb, int m, int nupd,
                                                         double2 *__restrict__ Vb,
                                                         const double2 *__restrict__ w, const double2 *__restrict__ coef,
                                                         const double2 *__restrict__ H, double2 *__restrict__ hsum,
                                                         double *__restrict__ npart, const KrylovState *__restrict__ st,
                                                         KBatch B)
{
    const int run = blockIdx.y;
    if (st[run].done) return;
    if (jb) j += *jb;
    Vb += run * B.basis;
    w += run * B.vec;
    coef += run * B.coef;
    H += run * B.hess;
    hsum += run * B.small;
    npart += run * B.npart;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the coefficients go through scalar loads
    const double inv_nu = coef[j].x;
    if ((int)blockIdx.x >= nupd) {
        const int r = ((int)blockIdx.x - nupd) * 4 + wave;
        if (r > j) return;
        const double2 *hrow = H + (int64_t)r * m;
        double sr = 0, si = 0;
        for (int i = max(r - 1, 0) + lane; i < j; i += 64) {
            const double2 h = hrow[i], a = coef[i];
            sr += h.x * a.x - h.y * a.y;
            si += h.x * a.y + h.y * a.x;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) {
            const double2 bb = coef[j + 1 + r];
            hsum[r] = make_double2((bb.x - sr) * inv_nu, (bb.y - si) * inv_nu);
        }
        return;
    }
    const int row = blockIdx.x * UPD_ROWS + lane;
    const bool live = row < n;
    double ur = 0, ui = 0, wr = 0, wi = 0;
    if (live)
#pragma unroll 4
        for (int c = wave; c < j; c += 4) {
            const double2 v = Vb[(int64_t)c * n + row], a = coef[c], b = coef[j + 1 + c];
            ur += v.x * a.x - v.y * a.y;
            ui += v.x * a.y + v.y * a.x;
            wr += v.x * b.x - v.y * b.y;
            wi += v.x * b.y + v.y * b.x;
        }
    __shared__ double4 acc[3][UPD_ROWS];
    if (wave > 0) acc[wave - 1][lane] = make_double4(ur, ui, wr, wi);
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double4 t = acc[q][lane];
        ur += t.x; ui += t.y; wr += t.z; wi += t.w;
    }
    double nrm = 0.0;
    if (live) {
        const double2 u = Vb[(int64_t)j * n + row], x = w[row], cj = coef[2 * j + 1];
        const double2 v = make_double2((u.x - ur) * inv_nu, (u.y - ui) * inv_nu);
        const double2 y = make_double2(x.x - wr - (v.x * cj.x - v.y * cj.y), x.y - wi - (v.x * cj.y + v.y * cj.x));
        Vb[(int64_t)j * n + row] = v;
        Vb[(int64_t)(j + 1) * n + row] = y;
        nrm = y.x * y.x + y.y * y.y;
    }
    nrm = wave_sum(nrm);
    if (lane == 0) npart[blockIdx.x] = nrm;
}

// u_{j+1} = y / |y| in place in slot j + 1 (|y|^2 from the nupd partials, summed
// in the same order by every block); block 0 stores beta_j = |y| / nu.  With
// u_out, u_{j+1} also goes there (run stride B.vec): the fixed operand of the
// next operator product.  Grid (ceil(n / 256), runs).
__global__ __launch_bounds__(256) void dgs_normalize_kernel(int n, int j, const int *__restrict__ jb, int m, int nupd,
                                                            const double *__restrict__ npart, double2 *__restrict__ Vb,
                                                            double2 *__restrict__ coef, double2 *__restrict__ u_out,
                                                            const KrylovState *__restrict__ st, KBatch B)
{
    const int run = blockIdx.y;
    if (st[run].done) return;
    if (jb) j += *jb;
    npart += run * B.npart;
    Vb += run * B.basis;
    coef += run * B.coef;
    __shared__ double red[4];
    double s2 = 0;
    for (int b = threadIdx.x; b < nupd; b += 256) s2 += npart[b];
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
    __syncthreads();
    const double yn = sqrt(red[0] + red[1] + red[2] + red[3]);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double2 *y = Vb + (int64_t)(j + 1) * n;
    if (r < n) {
        const double inv = yn > 0 ? 1.0 / yn : 0.0;
        const double2 u = make_double2(y[r].x * inv, y[r].y * inv);
        y[r] = u;
        if (u_out) u_out[run * B.vec + r] = u;
    }
    if (r == 0) coef[2 * m + 3] = make_double2(yn / coef[j].y, 0.0);
}

// partial[blk] = sum |w|^2 over 256-row blocks; grid (row blocks, runs)
__global__ __launch_bounds__(256) void norm_partial_kernel(int n, const double2 *__restrict__ w, int64_t wstride,
                                                           double *__restrict__ partial, int64_t pstride)
{
    w += blockIdx.y * wstride;
    partial += blockIdx.y * pstride;
    __shared__ double red[4];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double s = r < n ? w[r].x * w[r].x + w[r].y * w[r].y : 0.0;
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// beta = sqrt(sum partial); out = w / beta; beta_out = beta; grid (row blocks, runs)
__global__ __launch_bounds__(256) void normalize_kernel(int n, int nblk, const double *__restrict__ partial,
                                                        int64_t pstride, const double2 *__restrict__ w, int64_t wstride,
                                                        double2 *__restrict__ out, int64_t ostride,
                                                        double *__restrict__ beta_out)
{
    partial += blockIdx.y * pstride;
    w += blockIdx.y * wstride;
    out += blockIdx.y * ostride;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[b];
    const double beta = sqrt(s);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) beta_out[blockIdx.y] = beta;
    if (r >= n) return;
    const double inv = beta > 0 ? 1.0 / beta : 0.0;
    out[r] = make_double2(w[r].x * inv, w[r].y * inv);
}

// g = [beta0, 0, ...] and the state of each run; grid (ceil((m + 1) / 256), runs)
__global__ void krylov_init_kernel(int m, const double *__restrict__ beta0, const double *__restrict__ tol,
                                   double2 *__restrict__ g, KrylovState *__restrict__ st, KBatch B)
{
    const int run = blockIdx.y;
    g += run * B.small;
    st += run;
    const double b0 = beta0[run];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= m) g[i] = make_double2(i == 0 ? b0 : 0.0, 0.0);
    if (i == 0) {
        st->beta0 = b0;
        st->tol = tol[run];
        st->done = b0 == 0.0 ? 1 : 0;
        st->iters = 0;
        st->resid = b0 == 0.0 ? 0.0 : 1.0;
    }
}

// Back substitution R y = g of every run (k = its Arnoldi steps; R upper
// triangular, column c at offset c (m + 1)), column by column: y_i = g_i /
// R_ii, then g_r -= R_ri y_i for r < i.  One workgroup per run, g staged in
// LDS (dynamic, at least k complex); y of run r at y + r (m + 1).  The next
// column's entries are loaded before the current column's update, since
// only y_i depends on the previous step.
__global__ __launch_bounds__(256) void backsub_kernel(int m, const double2 *__restrict__ Rm,
                                                      const double2 *__restrict__ g,
                                                      const KrylovState *__restrict__ st, KBatch B,
                                                      double2 *__restrict__ y)
{
    constexpr int PER = 12;   // column entries per thread held in registers (k <= 3072)
    const int run = blockIdx.x;
    const int k = st[run].iters;
    Rm += run * B.hess;
    g += run * B.small;
    y += (int64_t)run * (m + 1);
    extern __shared__ double2 gs[];
    const int tid = threadIdx.x;
    for (int i = tid; i < k; i += 256) gs[i] = g[i];
    double2 cur[PER];
    if (k > 0) {
        const double2 *col = Rm + (int64_t)(k - 1) * (m + 1);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int r = tid + 256 * q;
            cur[q] = r < k ? col[r] : make_double2(0, 0);
        }
    }
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        double2 nxt[PER];
        if (i > 0) {
            const double2 *col = Rm + (int64_t)(i - 1) * (m + 1);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int r = tid + 256 * q;
                nxt[q] = r < i ? col[r] : make_double2(0, 0);
            }
        }
        const double2 gi = gs[i], d = Rm[(int64_t)i * (m + 1) + i];
        const double den = d.x * d.x + d.y * d.y;
        const double2 yi = make_double2((gi.x * d.x + gi.y * d.y) / den, (gi.y * d.x - gi.x * d.y) / den);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int r = tid + 256 * q;
            if (r < i) {
                const double2 a = cur[q];
                gs[r] = make_double2(gs[r].x - (a.x * yi.x - a.y * yi.y), gs[r].y - (a.x * yi.y + a.y * yi.x));
            }
        }
        if (tid == 0) y[i] = yi;
#pragma unroll
        for (int q = 0; q < PER; ++q) cur[q] = nxt[q];
        __syncthreads();
    }
}

// x_r = sum_{c < k_r} y_r[c] Vb_r[c] for every run r (grid (row blocks, runs))
__global__ void combine_kernel(int n, int m, const double2 *__restrict__ Vb, int64_t basis_stride,
                               const double2 *__restrict__ yc, double2 *__restrict__ x, int64_t x_stride,
                               const KrylovState *__restrict__ st)
{
    const int run = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int nvec = st[run].iters;
    Vb += run * basis_stride;
    yc += (int64_t)run * (m + 1);
    double2 acc = make_double2(0, 0);
    for (int c = 0; c < nvec; ++c) acc = cadd(acc, cmul(yc[c], Vb[(int64_t)c * n + r]));
    x[run * x_stride + r] = acc;
}

__global__ void axpy_sub_kernel(int n, const double2 *__restrict__ a, const double2 *__restrict__ b, double2 *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = make_double2(a[r].x - b[r].x, a[r].y - b[r].y);
}

// ------------------------------------------- multi-RHS (block) products
//
// R Krylov vectors (one per independent GMRES run) go through the dense
// blocks together on the matrix cores (gemm.hip).  The right-hand matrices
// are built from the FP64 vectors in FP32: for complex operators each
// complex entry x = (a, b) of run r becomes Bt[2r][2j] = a,
// Bt[2r][2j + 1] = -b, Bt[2r + 1][2j] = b, Bt[2r + 1][2j + 1] = a, so the
// real product of an interleaved complex row gives (re, im) of the complex
// product in columns 2r, 2r + 1.  Runs that have converged, runs past R and
// padding rows contribute zeros.

constexpr int BLOCK_RHS = 64;   // runs per block product (128 real columns)

__device__ inline bool run_active(const KrylovState *st, int r, int R)
{
    return r < R && !(st && st[r].done);
}

// Bt_v, Bt_w [128][kld] of one mesh from its [v; w] part of every run;
// grid (ceil(op_ld(nv) / 256), BLOCK_RHS)
__global__ __launch_bounds__(256) void pack_ops_kernel(int nv, int kld, int R, const double2 *__restrict__ X,
                                                       int64_t xstride, int voff, const KrylovState *__restrict__ st,
                                                       float *__restrict__ Btv, float *__restrict__ Btw)
{
    const int r = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * j >= kld) return;
    double2 v = make_double2(0, 0), w = v;
    if (j < nv && run_active(st, r, R)) {
        const double2 *x = X + r * xstride + voff;
        v = x[j];
        w = x[nv + j];
    }
    float *a0 = Btv + (int64_t)(2 * r) * kld + 2 * j, *a1 = a0 + kld;
    float *b0 = Btw + (int64_t)(2 * r) * kld + 2 * j, *b1 = b0 + kld;
    *reinterpret_cast<float2 *>(a0) = make_float2((float)v.x, -(float)v.y);
    *reinterpret_cast<float2 *>(a1) = make_float2((float)v.y, (float)v.x);
    *reinterpret_cast<float2 *>(b0) = make_float2((float)w.x, -(float)w.y);
    *reinterpret_cast<float2 *>(b1) = make_float2((float)w.y, (float)w.x);
}

// Partial products of the eight dense blocks: C[mesh][op] is [nk][128][N]
// (column-major tiles of the GEMM output), op order V, K, T, D.
struct BlockC {
    const float *C[2][4];
    int nk[2];
};

// y rows of every run = sums of the K-chunk partials (fixed order) with the
// block signs of Eq. "mtf:discrete" plus the mortar coupling in FP64;
// grid (ceil((ne + ni) / 256), R), one thread per row and run.
__global__ __launch_bounds__(256) void block_combine_kernel(MtfArgs A, BlockC bc, int R, const double2 *__restrict__ X,
                                                            int64_t xstride, double2 *__restrict__ Y, int64_t ystride,
                                                            const KrylovState *__restrict__ st)
{
    const int r = blockIdx.y;
    if (!run_active(st, r, R)) return;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= A.ne + A.ni) return;
    const bool ext = row < A.ne;
    const int mi = ext ? 0 : 1;
    const int i = ext ? row : row - A.ne;
    const int nv = ext ? A.ne : A.ni;
    double ar = 0, ai = 0, br = 0, bi = 0;
    for (int kc = 0; kc < bc.nk[mi]; ++kc) {
        const int64_t o0 = ((int64_t)kc * 128 + 2 * r) * nv + i, o1 = o0 + nv;
        ar += (double)bc.C[mi][0][o0] - (double)bc.C[mi][1][o0];
        ai += (double)bc.C[mi][0][o1] - (double)bc.C[mi][1][o1];
        br += (double)bc.C[mi][3][o0] + (double)bc.C[mi][2][o0];
        bi += (double)bc.C[mi][3][o1] + (double)bc.C[mi][2][o1];
    }
    const double2 *x = X + r * xstride;
    const int32_t *pp = ext ? A.pei_ptr : A.pie_ptr;
    const int32_t *pc = ext ? A.pei_col : A.pie_col;
    const double *pv = ext ? A.pei_val : A.pie_val;
    const double2 *cv = ext ? x + 2 * A.ne : x;
    const int nother = ext ? A.ni : A.ne;
    const double2 *cwp = cv + nother;
    const double fv = ext ? A.c_ext_v : A.c_int_v, fw = ext ? A.c_ext_w : A.c_int_w;
    double sr = 0, si = 0, tr = 0, ti = 0;
    for (int q = pp[i]; q < pp[i + 1]; ++q) {
        const double pvq = pv[q];
        const double2 a = cv[pc[q]], b = cwp[pc[q]];
        sr += pvq * a.x; si += pvq * a.y; tr += pvq * b.x; ti += pvq * b.y;
    }
    double2 *y = Y + r * ystride + (ext ? 0 : 2 * A.ne);
    y[i] = make_double2(ar + fv * sr, ai + fv * si);
    y[i + nv] = make_double2(br + fw * tr, bi + fw * ti);
}

// Bt [4 BLOCK_RHS][kld] of one mesh for the inverse-mass product: column
// 4r + q = Re y1, Im y1, Re y2, Im y2 of run r; grid (ceil(kld / 256), 4 BLOCK_RHS)
__global__ __launch_bounds__(256) void pack_mass_kernel(int nv, int kld, int R, const double2 *__restrict__ Y,
                                                        int64_t ystride, int yoff, const KrylovState *__restrict__ st,
                                                        float *__restrict__ Bt)
{
    const int c = blockIdx.y, r = c >> 2, q = c & 3;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kld) return;
    float val = 0.f;
    if (k < nv && run_active(st, r, R)) {
        const double2 y = Y[r * ystride + yoff + (q >= 2 ? nv : 0) + k];
        val = (float)((q & 1) ? y.y : y.x);
    }
    Bt[(int64_t)c * kld + k] = val;
}

// z rows of every run from the inverse-mass partials [nk][ccols][N] of each mesh;
// grid (ceil((ne + ni) / 256), R)
__global__ __launch_bounds__(256) void mass_reduce_kernel(int ne, int ni, const float *__restrict__ Ce,
                                                          const float *__restrict__ Ci, int nke, int nki, int ccols,
                                                          int R, double2 *__restrict__ Z, int64_t zstride,
                                                          const KrylovState *__restrict__ st)
{
    const int r = blockIdx.y;
    if (!run_active(st, r, R)) return;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= ne + ni) return;
    const bool ext = row < ne;
    const int i = ext ? row : row - ne;
    const int nv = ext ? ne : ni;
    const float *C = ext ? Ce : Ci;
    const int nk = ext ? nke : nki;
    double s[4] = {0, 0, 0, 0};
    for (int kc = 0; kc < nk; ++kc)
        for (int q = 0; q < 4; ++q) s[q] += (double)C[((int64_t)kc * ccols + 4 * r + q) * nv + i];
    double2 *z = Z + r * zstride + (ext ? 0 : 2 * ne);
    z[i] = make_double2(s[0], s[1]);
    z[i + nv] = make_double2(s[2], s[3]);
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

template <class C2>
__global__ void permute_mat_kernel(int nv, const int32_t *__restrict__ perm, const C2 *__restrict__ src,
                                   C2 *__restrict__ dst)
{
    const int iu = blockIdx.y;
    const int ju = blockIdx.x * blockDim.x + threadIdx.x;
    if (ju >= nv) return;
    dst[(int64_t)iu * nv + ju] = src[(int64_t)perm[iu] * op_ld(nv) + perm[ju]];
}

bem_status resolve_assembly_timing(bem_problem *p);

// operator in caller numbering, dense nv x nv (complex128 or complex64 as stored)
bem_status permute_matrix_out(const bem_problem *p, int mesh, const void *src, void *dst)
{
    const bem_mesh *m = mesh == 0 ? p->ext : p->inte;
    const int nv = (int)m->h.nv;
    const dim3 grid((nv + 255) / 256, nv);
    if (p->prec == BEM_C128)
        hipLaunchKernelGGL(permute_mat_kernel<double2>, grid, dim3(256), 0, p->ctx->stream, nv,
                           m->d.perm.as<int32_t>(), static_cast<const double2 *>(src), static_cast<double2 *>(dst));
    else
        hipLaunchKernelGGL(permute_mat_kernel<float2>, grid, dim3(256), 0, p->ctx->stream, nv,
                           m->d.perm.as<int32_t>(), static_cast<const float2 *>(src), static_cast<float2 *>(dst));
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

// ------------------------------------------------------------ host side

namespace {

struct Work {
    DevMem xin, d, y, z, b, r, Vb, partial, hsum, beta, tolv, yc, npart, R, H, coef, g, cs, sn, state, part;
    DevMem u, jb;   // captured steps: the operand u_j of each run, and the device step base
};

// Buffers of the multi-RHS products (one set per solve or batched mat-vec).
struct BlockBufs {
    DevMem btv[2], btw[2], cop, btm[2], cm;
    DevMem chw;    // sparse inverse-mass apply: two sets of (x, r, d) per run
    int64_t cop_off[2][4], cm_off[2];
};

MtfArgs make_args(const bem_problem *p)
{
    MtfArgs A;
    A.ne = (int)p->ext->h.nv;
    A.ni = (int)p->inte->h.nv;
    for (int m = 0; m < 2; ++m)
        for (int o = 0; o < 4; ++o) A.op[m][o] = p->ops[m][o].ptr;
    A.pie_ptr = p->P_ie_ptr.as<int32_t>(); A.pie_col = p->P_ie_col.as<int32_t>(); A.pie_val = p->P_ie_val.as<double>();
    A.pei_ptr = p->P_ei_ptr.as<int32_t>(); A.pei_col = p->P_ei_col.as<int32_t>(); A.pei_val = p->P_ei_val.as<double>();
    A.c_ext_v = 0.5;
    A.c_ext_w = 0.5 * p->rho_ext / p->rho_int;
    A.c_int_v = -0.5;
    A.c_int_w = -0.5 * p->rho_int / p->rho_ext;
    A.sym_ts = p->mtf_ts ? p->mtf_ts : (p->prec == BEM_C128 ? sym_tile<double2>() : sym_tile<float2>());
    A.no_mortar = 0;
    const bem_mesh *ms[2] = {p->ext, p->inte};
    for (int m = 0; m < 2; ++m) {
        A.near_row[m] = ms[m]->d.near_row.as<int32_t>();
        A.near_j[m] = ms[m]->d.near_j.as<int32_t>();
        A.corr[m] = p->corr[m].as<double2>();
    }
    return A;
}

size_t split_part_bytes(int ne, int ni)
{
    const int nchunk = std::max({split_nchunk(ne, MASS_CW_MAX), split_nchunk(ni, MASS_CW_MAX), sym_ntile(ne, SYM_TS_MIN),
                                 sym_ntile(ni, SYM_TS_MIN)});
    // the sparse inverse-mass apply of one run uses the same buffer for its two work sets (6 n complex)
    return std::max((size_t)nchunk * (ne + ni) * sizeof(double4), (size_t)6 * (2 * ne + 2 * ni) * sizeof(double2));
}

// Chebyshev steps of the sparse inverse-mass apply: M^-1 to FP64 rounding
// (36 steps, error 4 3^-36) in the FP64 form and to 1.4e-11 (24 steps) in the
// mixed form, for the operator products of the C ABI and wherever M^-1 is
// part of an operator (the exterior formulations).
int cheb_steps(const bem_problem *p) { return p->prec == BEM_C128 ? 36 : 24; }
// Inside GMRES on the multiple-traces system, M^-1 only preconditions: a
// fixed number k of Chebyshev steps from zero is a fixed polynomial p(M)
// with error 4 3^-k against M^-1 (7.5e-6 for k = 12, one launch), so
// GMRES on p(M) A x = p(M) b converges to the solution of A x = b, with the
// residual norms of p(M) within 1.5e-5 of those of M^-1.
constexpr int CHEB_PRECOND_STEPS = 12;
int cheb_precond_steps(const bem_problem *p) { return std::min(CHEB_PRECOND_STEPS, cheb_steps(p)); }

template <int RPT, int W>
void launch_cheb(const bem_problem *p, dim3 grid, hipStream_t st, const ChebArgs &A, int part0, int first, int last,
                 int nsteps, double rho, const double2 *y, int64_t ystride, double2 *z, int64_t zstride,
                 const double2 *win, double2 *wout, int64_t wstride, const KrylovState *kst)
{
    KTimer kt(p->ctx, K_MASS_APPLY);
    launch_k(kt, mass_cheb_kernel<RPT, W>, grid, dim3(1024), 0, st, A, part0, first, last, nsteps, rho, y, ystride, z,
             zstride, win, wout, wstride, kst);
}

// z = M^-1 y by K steps of the sparse Chebyshev apply on the patches
// [part0, part0 + np) for R runs.  Mesh m's two vectors start at base[m] in y, z and the work
// vectors (length wn); work holds two sets of (x, r, d), 6 wn complex per
// run, wstride apart.
bem_status cheb_apply(const bem_problem *p, int part0, int np, int64_t base0, int64_t base1, int64_t wn,
                      const double2 *y, int64_t ystride, double2 *z, int64_t zstride, double2 *work, int64_t wstride,
                      int R, const KrylovState *kst, int K)
{
    const ChebTables &T = p->cheb;
    ChebArgs A;
    A.pmesh = p->cheb_pmesh.as<int32_t>();
    A.vbeg = p->cheb_vbeg.as<int32_t>();
    A.cnt = p->cheb_cnt.as<int32_t>();
    A.vert = p->cheb_vert.as<int32_t>();
    A.ecol = p->cheb_ecol.as<uint16_t>();
    A.dinv = p->cheb_dinv.as<double>();
    A.eval = p->cheb_eval.as<double>();
    A.s = T.s;
    A.w = T.ell_w;
    A.nvm[0] = (int)p->ext->h.nv;
    A.nvm[1] = (int)p->inte->h.nv;
    A.base[0] = base0;
    A.base[1] = base1;
    A.wn = wn;
    const int nl = (K + T.s - 1) / T.s;
    const double sigma1 = CHEB_THETA / CHEB_DELTA;
    double rho = 1.0 / sigma1;
    const int rpt = (T.lmax + 1023) / 1024;
    const dim3 grid(np, 2, R);
    hipStream_t st = p->ctx->stream;
    for (int j = 0; j < nl; ++j) {
        const int steps = std::min(T.s, K - j * T.s);
        const double2 *win = work + (j % 2) * 3 * wn;
        double2 *wout = work + ((j + 1) % 2) * 3 * wn;
        const int first = j == 0, last = j == nl - 1;
#define CHEB_ARGS p, grid, st, A, part0, first, last, steps, rho, y, ystride, z, zstride, win, wout, wstride, kst
        if (rpt <= 1) {
            if (T.ell_w <= 8) launch_cheb<1, 8>(CHEB_ARGS);
            else if (T.ell_w <= 12) launch_cheb<1, 12>(CHEB_ARGS);
            else launch_cheb<1, 16>(CHEB_ARGS);
        } else {
            if (T.ell_w <= 8) launch_cheb<2, 8>(CHEB_ARGS);
            else if (T.ell_w <= 12) launch_cheb<2, 12>(CHEB_ARGS);
            else launch_cheb<2, 16>(CHEB_ARGS);
        }
#undef CHEB_ARGS
        BEM_HIP(hipGetLastError());
        for (int t = 0; t < steps; ++t) rho = 1.0 / (2.0 * sigma1 - rho);
    }
    return BEM_OK;
}

// z = blockdiag(M_e, M_e, M_i, M_i)^-1 y; K: Chebyshev steps of the sparse
// form (0: cheb_steps)
bem_status apply_Minv(const bem_problem *p, const double2 *y, double2 *z, double4 *part, const KrylovState *kst,
                      int K = 0)
{
    hipStream_t st = p->ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    if (p->mass_sparse) {
        const int64_t n = 2 * ne + 2 * ni;
        return cheb_apply(p, 0, p->cheb.nparts[0] + p->cheb.nparts[1], 0, 2 * ne, n, y, 0, z, 0,
                          reinterpret_cast<double2 *>(part), 6 * n, 1, kst, K > 0 ? K : cheb_steps(p));
    }
    {
        KTimer kt(p->ctx, K_MASS_APPLY);
        if (p->prec == BEM_C128)
            launch_k(kt, mass_apply_part_kernel<double, MASS_RW64>, split_grid(ne, ni, MASS_CW_MAX, MASS_RW64),
                     dim3(256), 0, st, ne, ni, p->Minv[0].as<double>(), p->Minv[1].as<double>(), y, part, kst);
        else
            launch_k(kt, mass_apply_part_kernel<float, MASS_RW32>, split_grid(ne, ni, MASS_CW_MAX, MASS_RW32),
                     dim3(256), 0, st, ne, ni, p->Minv[0].as<float>(), p->Minv[1].as<float>(), y, part, kst);
    }
    hipLaunchKernelGGL(mass_combine_kernel, dim3((ne + ni + 255) / 256), dim3(256), 0, st, ne, ni, part, z, kst);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

// y = A x (weak form); z = M^-1 y when `strong`.  Complex64 operators are
// applied with FP32 accumulation, or FP64 when `acc64` (refinement residual).
bem_status apply_A(const bem_problem *p, const MtfArgs &A, const double2 *x, double2 *y, double2 *z, bool strong,
                   const KrylovState *kst, double4 *part, bool acc64 = false, int K = 0)
{
    hipStream_t st = p->ctx->stream;
    const int rows = A.ne + A.ni;
    const int nte = sym_ntile(A.ne, A.sym_ts), nti = sym_ntile(A.ni, A.sym_ts);
    const dim3 g((unsigned)((int64_t)nte * (nte + 1) / 2 + (int64_t)nti * (nti + 1) / 2));
    {
        KTimer kt(p->ctx, K_MTF_DENSE);
        if (A.sym_ts == 64) {
            if (p->prec == BEM_C128)
                launch_k(kt, mtf_sym_tile_kernel<double2, double, 64>, g, dim3(256), 0, st, A, x, part, kst);
            else if (acc64)
                launch_k(kt, mtf_sym_tile_kernel<float2, double, 64>, g, dim3(256), 0, st, A, x, part, kst);
            else
                launch_k(kt, mtf_sym_tile_kernel<float2, float, 64>, g, dim3(256), 0, st, A, x, part, kst);
        } else {
            if (p->prec == BEM_C128)
                launch_k(kt, mtf_sym_tile_kernel<double2, double, 128>, g, dim3(256), 0, st, A, x, part, kst);
            else if (acc64)
                launch_k(kt, mtf_sym_tile_kernel<float2, double, 128>, g, dim3(256), 0, st, A, x, part, kst);
            else
                launch_k(kt, mtf_sym_tile_kernel<float2, float, 128>, g, dim3(256), 0, st, A, x, part, kst);
        }
    }
    hipLaunchKernelGGL(mtf_sym_combine_kernel, dim3((rows + 15) / 16), dim3(256), 0, st, A, x, part, y, kst);
    BEM_HIP(hipGetLastError());
    if (strong) return apply_Minv(p, y, z, part, kst, K);
    return BEM_OK;
}

// Tile edge of the symmetric mat-vec (64 or 128) by timing both on the
// problem's operators once per size class and precision (tuning table).
// x: any n-vector; y, part: work buffers.
bem_status mtf_tune(bem_problem *p, const double2 *x, double2 *y, double4 *part)
{
    if (p->mtf_ts) return BEM_OK;
    const std::string key = std::string(p->prec == BEM_C128 ? "mtf-c128" : "mtf-c64") + ":e" +
                            std::to_string(tune_class(p->ext->h.nv)) + ":i" + std::to_string(tune_class(p->inte->h.nv));
    hipStream_t st = p->ctx->stream;
    std::vector<int> v;
    bem_status s = tuned(key, v, [&](std::vector<int> &out) -> bem_status {
        hipEvent_t e0, e1;
        BEM_HIP(hipEventCreate(&e0));
        BEM_HIP(hipEventCreate(&e1));
        struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } g{e0, e1};
        float best = 1e30f;
        int pick = 128;
        for (int ts : {64, 128}) {
            MtfArgs A = make_args(p);
            A.sym_ts = ts;
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                BEM_HIP(hipEventRecord(e0, st));
                bem_status q = apply_A(p, A, x, y, nullptr, false, nullptr, part);
                if (q) return q;
                BEM_HIP(hipEventRecord(e1, st));
                BEM_HIP(hipEventSynchronize(e1));
                float ms = 0;
                BEM_HIP(hipEventElapsedTime(&ms, e0, e1));
                tmin = std::min(tmin, ms);
            }
            if (tmin < best) { best = tmin; pick = ts; }
        }
        out = {pick};
        return BEM_OK;
    });
    if (s) return s;
    p->mtf_ts = v.size() == 1 && (v[0] == 64 || v[0] == 128) ? v[0] : 128;
    return BEM_OK;
}

// ---- exterior PMCHWT (Sec. 3.3, Eq. "pmchwt:discrete"): with x = [v; w] on
// the exterior mesh, A x = C_ext x + P_ei M_i^-1 C_int M_i^-1 P_ie x, where
// C_ext = [-K_e V_e; D_e T_e] and C_int = [-K_i a V_i; D_i / a T_i],
// a = rho_int / rho_ext (the scaled interior Calderon operator of the
// single-trace system, Sec. 2.2).  With u = M_i^-1 P_ie x, one pass of the
// multiple-traces tile products over [v; w; u_a; a u_b] (mortar terms off)
// gives C_ext x on the exterior rows and, on the interior rows,
// [-K_i u_a + a V_i u_b; D_i u_a + a T_i u_b], whose second row times 1/a is
// the second row of C_int u.

// X[0, 2 ne) = x; T = [P_ie v; a P_ie w] (interior layout)
__global__ __launch_bounds__(256) void pmchwt_project_kernel(int ne, int ni, const int32_t *__restrict__ ptr,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val, double a,
                                                             const double2 *__restrict__ x, double2 *__restrict__ X,
                                                             double2 *__restrict__ T, const KrylovState *__restrict__ st)
{
    if (st && st->done) return;
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < 2 * ne) {
        X[u] = x[u];
        return;
    }
    const int i = u - 2 * ne;
    if (i >= ni) return;
    double vr = 0, vi = 0, wr = 0, wi = 0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
        const double pv = val[k];
        const double2 v = x[col[k]], w = x[ne + col[k]];
        vr += pv * v.x; vi += pv * v.y; wr += pv * w.x; wi += pv * w.y;
    }
    T[i] = make_double2(vr, vi);
    T[ni + i] = make_double2(a * wr, a * wi);
}

// Rr = Y[0, 2 ne) + [P_ei Q_a; b P_ei Q_b]
__global__ __launch_bounds__(256) void pmchwt_lift_kernel(int ne, int ni, const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ val, double b,
                                                          const double2 *__restrict__ Y, const double2 *__restrict__ Q,
                                                          double2 *__restrict__ Rr, const KrylovState *__restrict__ st)
{
    if (st && st->done) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ne) return;
    double ar = 0, ai = 0, br = 0, bi = 0;
    for (int k = ptr[j]; k < ptr[j + 1]; ++k) {
        const double pv = val[k];
        const double2 qa = Q[col[k]], qb = Q[ni + col[k]];
        ar += pv * qa.x; ai += pv * qa.y; br += pv * qb.x; bi += pv * qb.y;
    }
    const double2 ya = Y[j], yb = Y[ne + j];
    Rr[j] = make_double2(ya.x + ar, ya.y + ai);
    Rr[ne + j] = make_double2(yb.x + b * br, yb.y + b * bi);
}

// z = blockdiag(M, M)^-1 y on one mesh (y, z: that mesh's two vectors)
bem_status apply_Minv_mesh(const bem_problem *p, int mesh, const double2 *y, double2 *z, double4 *part,
                           const KrylovState *kst)
{
    hipStream_t st = p->ctx->stream;
    const int ne = mesh == 0 ? (int)p->ext->h.nv : 0, ni = mesh == 1 ? (int)p->inte->h.nv : 0;
    if (p->mass_sparse) {   // y, z: this mesh's two vectors
        const int64_t wn = 2 * (int64_t)(ne + ni);
        return cheb_apply(p, mesh == 0 ? 0 : p->cheb.nparts[0], p->cheb.nparts[mesh], 0, 0, wn, y, 0, z, 0,
                          reinterpret_cast<double2 *>(part), 6 * wn, 1, kst, cheb_steps(p));
    }
    {
        KTimer kt(p->ctx, K_MASS_APPLY);
        launch_k(kt, mass_apply_part_kernel<double, MASS_RW64>, split_grid(ne, ni, MASS_CW_MAX, MASS_RW64), dim3(256),
                 0, st, ne, ni, p->Minv[0].as<double>(), p->Minv[1].as<double>(), y, part, kst);
    }
    hipLaunchKernelGGL(mass_combine_kernel, dim3((ne + ni + 255) / 256), dim3(256), 0, st, ne, ni, part, z, kst);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

enum ExtForm { FORM_PMCHWT = 1, FORM_HCN = 2 };   // exterior formulations on [v; w] of the exterior mesh

struct PmchwtBufs {
    int form = FORM_PMCHWT;
    MtfArgs A0;            // the multiple-traces arguments with the mortar terms off
    MtfArgs Ai;            // the same on the interior mesh alone
    DevMem X, Y, T, Q, Rr; // [2 ne + 2 ni] x2, [2 ni] x2, [2 ne]
    DevMem X2, Y2, S, W2;  // high-contrast Neumann: [2 ni], [2 ni], [2 ne], [2 ni]
};

bem_status pmchwt_alloc(bem_problem *p, PmchwtBufs &pb)
{
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    const size_t nm = (size_t)(2 * ne + 2 * ni) * sizeof(double2);
    pb.A0 = make_args(p);
    pb.A0.c_ext_v = pb.A0.c_ext_w = pb.A0.c_int_v = pb.A0.c_int_w = 0.0;
    pb.A0.no_mortar = 1;
    pb.Ai = pb.A0;
    pb.Ai.ne = 0;   // tiles, rows and partials of the interior mesh only
    bem_status s = dev_alloc(p->ctx, pb.X, nm);
    if (!s) s = dev_alloc(p->ctx, pb.Y, nm);
    if (!s) s = dev_alloc(p->ctx, pb.T, (size_t)2 * ni * sizeof(double2));
    if (!s) s = dev_alloc(p->ctx, pb.Q, (size_t)2 * ni * sizeof(double2));
    if (!s) s = dev_alloc(p->ctx, pb.Rr, (size_t)2 * ne * sizeof(double2));
    if (!s && pb.form == FORM_HCN) {
        s = dev_alloc(p->ctx, pb.X2, (size_t)2 * ni * sizeof(double2));
        if (!s) s = dev_alloc(p->ctx, pb.Y2, (size_t)2 * ni * sizeof(double2));
        if (!s) s = dev_alloc(p->ctx, pb.S, (size_t)2 * ne * sizeof(double2));
        if (!s) s = dev_alloc(p->ctx, pb.W2, (size_t)2 * ni * sizeof(double2));
    }
    return s;
}

// y = A x (weak form, 2 ne, internal numbering); with `strong`, z = M_e^-1 y
bem_status apply_pmchwt(const bem_problem *p, const PmchwtBufs &pb, const double2 *x, double2 *y, double2 *z,
                        bool strong, const KrylovState *kst, double4 *part)
{
    hipStream_t st = p->ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    const double a = p->rho_int / p->rho_ext;
    double2 *X = pb.X.as<double2>(), *Y = pb.Y.as<double2>(), *T = pb.T.as<double2>(), *Q = pb.Q.as<double2>();
    hipLaunchKernelGGL(pmchwt_project_kernel, dim3((2 * ne + ni + 255) / 256), dim3(256), 0, st, ne, ni,
                       p->P_ie_ptr.as<int32_t>(), p->P_ie_col.as<int32_t>(), p->P_ie_val.as<double>(), a, x, X, T, kst);
    BEM_HIP(hipGetLastError());
    bem_status s = apply_Minv_mesh(p, 1, T, X + 2 * ne, part, kst);
    if (!s) s = apply_A(p, pb.A0, X, Y, nullptr, false, kst, part);
    if (!s) s = apply_Minv_mesh(p, 1, Y + 2 * ne, Q, part, kst);
    if (s) return s;
    double2 *out = strong ? pb.Rr.as<double2>() : y;
    hipLaunchKernelGGL(pmchwt_lift_kernel, dim3((ne + 255) / 256), dim3(256), 0, st, ne, ni,
                       p->P_ei_ptr.as<int32_t>(), p->P_ei_col.as<int32_t>(), p->P_ei_val.as<double>(), 1.0 / a, Y, Q,
                       out, kst);
    BEM_HIP(hipGetLastError());
    if (strong) return apply_Minv_mesh(p, 0, out, z, part, kst);
    return BEM_OK;
}

// ---- exterior high-contrast Neumann (discrete form of Eq.
// "highcontrast:ext:neu", Sec. 3.3), unknowns [a; b] = [gamma_N p; mu]:
//   row 1: 1/2 M_e a - hat(T_i) a - c hat(D_i) M_e^-1 V_e b,   c = rho_ext / rho_int
//   row 2: M_e a + 1/2 M_e b - T_e b
// with hat(X) = P_ei M_i^-1 X M_i^-1 P_ie.  With u_b = M_i^-1 P_ie a and
// u_a = c M_i^-1 P_ie M_e^-1 V_e b, the hatted terms of row 1 are
// P_ei M_i^-1 (T_i u_b + D_i u_a): one tile pass over [0; b; 0; u_b] gives
// V_e b, T_e b and T_i u_b, one interior pass over [u_a; 0] gives D_i u_a.

// out_a = s P x (+ add), out_b = 0, over the rows of the CSR matrix (ptr null: out_a = x (+ add))
__global__ __launch_bounds__(256) void hcn_spmv_kernel(int nrows, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ col, const double *__restrict__ val,
                                                       const double2 *__restrict__ x, double sc,
                                                       const double2 *__restrict__ add, double2 *__restrict__ out_a,
                                                       double2 *__restrict__ out_b, const KrylovState *__restrict__ st)
{
    if (st && st->done) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    double r = 0, im = 0;
    if (ptr) {
        for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
            const double pv = val[k];
            const double2 v = x[col[k]];
            r += pv * v.x; im += pv * v.y;
        }
        r *= sc; im *= sc;
    } else {
        r = x[i].x; im = x[i].y;
    }
    if (add) { r += add[i].x; im += add[i].y; }
    out_a[i] = make_double2(r, im);
    if (out_b) out_b[i] = make_double2(0.0, 0.0);
}

// rows of the high-contrast product: out[j] = 1/2 (M_e a)_j - (P_ei q)_j,
// out[ne + j] = (M_e a)_j + 1/2 (M_e b)_j - (T_e b)_j
__global__ __launch_bounds__(256) void hcn_rows_kernel(int ne, const int32_t *__restrict__ mptr,
                                                       const int32_t *__restrict__ mcol, const double *__restrict__ mval,
                                                       const int32_t *__restrict__ pptr, const int32_t *__restrict__ pcol,
                                                       const double *__restrict__ pval, const double2 *__restrict__ x,
                                                       const double2 *__restrict__ q, const double2 *__restrict__ Teb,
                                                       double2 *__restrict__ out, const KrylovState *__restrict__ st)
{
    if (st && st->done) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ne) return;
    double ar = 0, ai = 0, br = 0, bi = 0, qr = 0, qi = 0;
    for (int k = mptr[j]; k < mptr[j + 1]; ++k) {
        const double mv = mval[k];
        const double2 a = x[mcol[k]], b = x[ne + mcol[k]];
        ar += mv * a.x; ai += mv * a.y; br += mv * b.x; bi += mv * b.y;
    }
    for (int k = pptr[j]; k < pptr[j + 1]; ++k) {
        const double pv = pval[k];
        const double2 v = q[pcol[k]];
        qr += pv * v.x; qi += pv * v.y;
    }
    out[j] = make_double2(0.5 * ar - qr, 0.5 * ai - qi);
    out[ne + j] = make_double2(ar + 0.5 * br - Teb[j].x, ai + 0.5 * bi - Teb[j].y);
}

// X2 = [c M_i^-1 P_ie M_e^-1 v; 0] for an exterior vector v (through pb.T); returns in pb.X2
bem_status hcn_to_interior(const bem_problem *p, const PmchwtBufs &pb, const double2 *v_ext_minv, double c,
                           const KrylovState *kst, double4 *part)
{
    hipStream_t st = p->ctx->stream;
    const int ni = (int)p->inte->h.nv;
    double2 *T = pb.T.as<double2>();
    hipLaunchKernelGGL(hcn_spmv_kernel, dim3((ni + 255) / 256), dim3(256), 0, st, ni, p->P_ie_ptr.as<int32_t>(),
                       p->P_ie_col.as<int32_t>(), p->P_ie_val.as<double>(), v_ext_minv, c, nullptr, T, T + ni, kst);
    BEM_HIP(hipGetLastError());
    return apply_Minv_mesh(p, 1, T, pb.X2.as<double2>(), part, kst);
}

bem_status apply_hcn(const bem_problem *p, const PmchwtBufs &pb, const double2 *x, double2 *y, double2 *z,
                     bool strong, const KrylovState *kst, double4 *part)
{
    hipStream_t st = p->ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    const double c = p->rho_ext / p->rho_int;
    double2 *X = pb.X.as<double2>(), *Y = pb.Y.as<double2>(), *T = pb.T.as<double2>(), *Q = pb.Q.as<double2>();
    double2 *S = pb.S.as<double2>(), *Y2 = pb.Y2.as<double2>(), *W2 = pb.W2.as<double2>();
    const dim3 ge((ne + 255) / 256), gi((ni + 255) / 256);
    // X = [0; b; M_i^-1 [0; P_ie a]] = [0; b; 0; u_b]
    hipLaunchKernelGGL(hcn_spmv_kernel, ge, dim3(256), 0, st, ne, nullptr, nullptr, nullptr, x + ne, 1.0, nullptr,
                       X + ne, X, kst);
    hipLaunchKernelGGL(hcn_spmv_kernel, gi, dim3(256), 0, st, ni, p->P_ie_ptr.as<int32_t>(), p->P_ie_col.as<int32_t>(),
                       p->P_ie_val.as<double>(), x, 1.0, nullptr, T + ni, T, kst);
    BEM_HIP(hipGetLastError());
    bem_status s = apply_Minv_mesh(p, 1, T, X + 2 * ne, part, kst);
    // Y = [V_e b; T_e b; V_i u_b; T_i u_b]
    if (!s) s = apply_A(p, pb.A0, X, Y, nullptr, false, kst, part);
    // S = M_e^-1 [V_e b; T_e b]; X2 = [u_a; 0]; Y2 = [-K_i u_a; D_i u_a]
    if (!s) s = apply_Minv_mesh(p, 0, Y, S, part, kst);
    if (!s) s = hcn_to_interior(p, pb, S, c, kst, part);
    if (!s) s = apply_A(p, pb.Ai, pb.X2.as<double2>(), Y2, nullptr, false, kst, part);
    if (s) return s;
    // Q = M_i^-1 [T_i u_b + D_i u_a; 0]
    hipLaunchKernelGGL(hcn_spmv_kernel, gi, dim3(256), 0, st, ni, nullptr, nullptr, nullptr, Y + 2 * ne + ni, 1.0,
                       Y2 + ni, W2, W2 + ni, kst);
    BEM_HIP(hipGetLastError());
    s = apply_Minv_mesh(p, 1, W2, Q, part, kst);
    if (s) return s;
    double2 *out = strong ? pb.Rr.as<double2>() : y;
    hipLaunchKernelGGL(hcn_rows_kernel, ge, dim3(256), 0, st, ne, p->M_ptr[0].as<int32_t>(), p->M_col[0].as<int32_t>(),
                       p->M_val[0].as<double>(), p->P_ei_ptr.as<int32_t>(), p->P_ei_col.as<int32_t>(),
                       p->P_ei_val.as<double>(), x, Q, Y + ne, out, kst);
    BEM_HIP(hipGetLastError());
    (void)T;
    if (strong) return apply_Minv_mesh(p, 0, out, z, part, kst);
    return BEM_OK;
}

// right-hand side [c hat(D_i) M_e^-1 f; g] from [f; g]
bem_status hcn_rhs(const bem_problem *p, const PmchwtBufs &pb, const double2 *fg, double2 *b, double4 *part)
{
    hipStream_t st = p->ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv;
    const double c = p->rho_ext / p->rho_int;
    double2 *S = pb.S.as<double2>(), *Y2 = pb.Y2.as<double2>(), *W2 = pb.W2.as<double2>(), *Q = pb.Q.as<double2>();
    const dim3 ge((ne + 255) / 256), gi((ni + 255) / 256);
    bem_status s = apply_Minv_mesh(p, 0, fg, S, part, nullptr);
    if (!s) s = hcn_to_interior(p, pb, S, c, nullptr, part);
    if (!s) s = apply_A(p, pb.Ai, pb.X2.as<double2>(), Y2, nullptr, false, nullptr, part);
    if (s) return s;
    hipLaunchKernelGGL(hcn_spmv_kernel, gi, dim3(256), 0, st, ni, nullptr, nullptr, nullptr, Y2 + ni, 1.0, nullptr,
                       W2, W2 + ni, nullptr);
    BEM_HIP(hipGetLastError());
    s = apply_Minv_mesh(p, 1, W2, Q, part, nullptr);
    if (s) return s;
    hipLaunchKernelGGL(hcn_spmv_kernel, ge, dim3(256), 0, st, ne, p->P_ei_ptr.as<int32_t>(), p->P_ei_col.as<int32_t>(),
                       p->P_ei_val.as<double>(), Q, 1.0, nullptr, b, nullptr, nullptr);
    hipLaunchKernelGGL(hcn_spmv_kernel, ge, dim3(256), 0, st, ne, nullptr, nullptr, nullptr, fg + ne, 1.0, nullptr,
                       b + ne, nullptr, nullptr);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

bem_status apply_ext_form(const bem_problem *p, const PmchwtBufs &pb, const double2 *x, double2 *y, double2 *z,
                          bool strong, const KrylovState *kst, double4 *part)
{
    return pb.form == FORM_HCN ? apply_hcn(p, pb, x, y, z, strong, kst, part)
                               : apply_pmchwt(p, pb, x, y, z, strong, kst, part);
}

// ||w|| on the device: into *out (device double)
bem_status norm_to(const bem_problem *p, int n, const double2 *w, double *npart, double2 *scratch_vec, double *out)
{
    hipStream_t st = p->ctx->stream;
    const int nblk = (n + 255) / 256;
    hipLaunchKernelGGL(norm_partial_kernel, dim3(nblk), dim3(256), 0, st, n, w, (int64_t)0, npart, (int64_t)0);
    hipLaunchKernelGGL(normalize_kernel, dim3(nblk), dim3(256), 0, st, n, nblk, npart, (int64_t)0, w, (int64_t)0,
                       scratch_vec, (int64_t)0, out);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

constexpr int GEMM_MAX_SPLIT = 8;   // K chunks per GEMM segment, at most
int kchunk_for(int K, int nk, int kst = 32) { return ((K + nk - 1) / nk + kst - 1) / kst * kst; }
int nchunks(int K, int kc) { return (K + kc - 1) / kc; }

bem_status block_alloc(bem_problem *p, BlockBufs &bb)
{
    bem_ctx *ctx = p->ctx;
    const int nv[2] = {(int)p->ext->h.nv, (int)p->inte->h.nv};
    size_t cop = 0, cm = 0;
    for (int m = 0; m < 2; ++m) {
        const int kop = 2 * (int)op_ld(nv[m]), km = minv_ld(nv[m], true);
        bem_status s = dev_alloc(ctx, bb.btv[m], (size_t)2 * BLOCK_RHS * kop * sizeof(float));
        if (!s) s = dev_alloc(ctx, bb.btw[m], (size_t)2 * BLOCK_RHS * kop * sizeof(float));
        if (!s) s = dev_alloc(ctx, bb.btm[m], (size_t)4 * BLOCK_RHS * km * sizeof(float));
        if (s) return s;
        // partial outputs sized for the largest chunk count the tuner tries
        for (int o = 0; o < 4; ++o) {
            bb.cop_off[m][o] = (int64_t)cop;
            cop += (size_t)nchunks(kop, kchunk_for(kop, GEMM_MAX_SPLIT)) * 2 * BLOCK_RHS * nv[m];
        }
        bb.cm_off[m] = (int64_t)cm;
        cm += (size_t)nchunks(km, kchunk_for(km, GEMM_MAX_SPLIT)) * 4 * BLOCK_RHS * nv[m];
    }
    bem_status s = dev_alloc(ctx, bb.cop, cop * sizeof(float));
    if (!s) s = dev_alloc(ctx, bb.cm, cm * sizeof(float));
    if (!s && p->mass_sparse && !p->mass_dense)
        s = dev_alloc(ctx, bb.chw, (size_t)6 * BLOCK_RHS * (2 * nv[0] + 2 * nv[1]) * sizeof(double2));
    return s;
}

// tile width (in 32-column units) and 128-column blocks for `cols` right-hand columns
void gemm_width(int cols, int &nt, int &ncb)
{
    ncb = (cols + 127) / 128;
    nt = cols <= 32 ? 1 : cols <= 64 ? 2 : 4;
    if (ncb > 1) nt = 4;
}
int nt_index(int nt) { return nt == 1 ? 0 : nt == 2 ? 1 : 2; }

GemmArgs ops_gemm_args(const bem_problem *p, BlockBufs &bb, const int nk[2], int R, const KrylovState *st, int kst = 32)
{
    GemmArgs G{};
    G.kst = kst;
    int nt, ncb;
    gemm_width(2 * R, nt, ncb);
    G.nt = nt;
    const int nv[2] = {(int)p->ext->h.nv, (int)p->inte->h.nv};
    int q = 0;
    for (int m = 0; m < 2; ++m) {
        const int kop = 2 * (int)op_ld(nv[m]);
        for (int o = 0; o < 4; ++o) {
            GemmSeg &S = G.seg[q++];
            S.A = p->ops[m][o].as<float>();
            S.lda = kop;
            S.Bt = (o == 1 || o == 3) ? bb.btv[m].as<float>() : bb.btw[m].as<float>();   // K, D act on v; V, T on w
            S.ldb = kop;
            S.C = bb.cop.as<float>() + bb.cop_off[m][o];
            S.M = nv[m];
            S.K = kop;
            S.kchunk = kchunk_for(kop, nk[m], kst);
            S.ncb = 1;
        }
    }
    G.nseg = q;
    G.done = st ? &st[0].done : nullptr;
    G.done_stride = (int)(sizeof(KrylovState) / sizeof(int));
    G.nrun = R;
    return G;
}

GemmArgs mass_gemm_args(const bem_problem *p, BlockBufs &bb, const int nk[2], int R, const KrylovState *st)
{
    GemmArgs G{};
    G.kst = 32;
    int nt, ncb;
    gemm_width(4 * R, nt, ncb);
    G.nt = nt;
    const int nv[2] = {(int)p->ext->h.nv, (int)p->inte->h.nv};
    for (int m = 0; m < 2; ++m) {
        const int km = minv_ld(nv[m], true);
        GemmSeg &S = G.seg[m];
        S.A = p->Minv[m].as<float>();
        S.lda = km;
        S.Bt = bb.btm[m].as<float>();
        S.ldb = km;
        S.C = bb.cm.as<float>() + bb.cm_off[m];
        S.M = nv[m];
        S.K = km;
        S.kchunk = kchunk_for(km, nk[m]);
        S.ncb = ncb;
    }
    G.nseg = 2;
    G.done = st ? &st[0].done : nullptr;
    G.done_stride = (int)(sizeof(KrylovState) / sizeof(int));
    G.nrun = R;
    return G;
}

// Modelled duration of one GEMM launch, in units of 32 k: the workgroups
// go to the 8 XCDs in turn, in launch order, and each XCD starts the next
// of its workgroups on the first slot that frees up (slots: workgroups per
// compute unit times compute units per XCD).  A workgroup costs its k range
// plus a fixed share for the fill of its first stage and the store of its
// tile.  Used to rank the K splits worth timing: with few workgroups per
// slot the last wave of workgroups leaves most slots idle.
double gemm_model_time(const GemmArgs &G, int slots_per_xcd)
{
    constexpr int kXcd = 8;
    constexpr double kFixed = 4.0;
    std::vector<std::vector<double>> free_at(kXcd, std::vector<double>(slots_per_xcd, 0.0));   // min-heaps
    int64_t wg = 0;
    double end = 0.0;
    for (int s = 0; s < G.nseg; ++s) {
        const GemmSeg &S = G.seg[s];
        const int nrt = (S.M + 127) / 128, nk = nchunks(S.K, S.kchunk);
        for (int kc = 0; kc < nk; ++kc) {   // launch order: chunk, column block, row tile
            const double cost = (std::min(S.K, (kc + 1) * S.kchunk) - kc * S.kchunk) / 32.0 + kFixed;
            for (int64_t c = 0; c < (int64_t)S.ncb * nrt; ++c) {
                std::vector<double> &h = free_at[wg++ % kXcd];
                std::pop_heap(h.begin(), h.end(), std::greater<double>());
                h.back() += cost;
                end = std::max(end, h.back());
                std::push_heap(h.begin(), h.end(), std::greater<double>());
            }
        }
    }
    return end;
}

// K split of one GEMM (which = 0 operators, 1 inverse masses) for R runs:
// chunk counts for the exterior and interior segments and, for the operator
// product, k per LDS stage.  The splits of 1 to 8 chunks per mesh are ranked
// by the scheduling model above; the best three of each stage depth and the
// even splits 4/4 and 8/8 are timed (best of three launches each)
// on the problem's own matrices (right-hand buffers zeroed first) once per
// size class, and the choice is kept in the process-wide tuning table (and
// its file), so every problem and context of the class uses the same shapes.
bem_status block_tune(bem_problem *p, BlockBufs &bb, int which, int R, int nk[2], int &kst)
{
    int nt, ncb;
    gemm_width(which == 0 ? 2 * R : 4 * R, nt, ncb);
    int *slot = p->gemm_nk[which][nt_index(nt)];
    int &slot_kst = p->gemm_kst[which][nt_index(nt)];
    if (slot[0] > 0) { nk[0] = slot[0]; nk[1] = slot[1]; kst = slot_kst; return BEM_OK; }
    bem_ctx *ctx = p->ctx;
    hipStream_t st = ctx->stream;
    const std::string key = std::string(which == 0 ? "gemm-ops" : "gemm-mass") + ":c" + std::to_string(32 * nt * ncb) +
                            ":e" + std::to_string(tune_class(p->ext->h.nv)) + ":i" +
                            std::to_string(tune_class(p->inte->h.nv));
    auto valid = [&](const std::vector<int> &v) {
        return v.size() == 3 && v[0] >= 1 && v[0] <= GEMM_MAX_SPLIT && v[1] >= 1 && v[1] <= GEMM_MAX_SPLIT &&
               (v[2] == 32 || (v[2] == 64 && which == 0));
    };
    std::vector<int> v;
    bem_status s = tuned(key, v, [&](std::vector<int> &out) -> bem_status {
        for (int m = 0; m < 2; ++m) {   // defined right-hand inputs for the timing runs
            BEM_HIP(hipMemsetAsync(bb.btv[m].ptr, 0, bb.btv[m].bytes, st));
            BEM_HIP(hipMemsetAsync(bb.btw[m].ptr, 0, bb.btw[m].bytes, st));
            BEM_HIP(hipMemsetAsync(bb.btm[m].ptr, 0, bb.btm[m].bytes, st));
        }
        int ncu = 0;
        BEM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
        struct Cand { int nk[2], kst; double model; };
        std::vector<Cand> timed;
        for (int ks : {32, 64}) {
            if (which == 1 && ks != 32) continue;   // inverse-mass rows: multiples of 32 only
            std::vector<Cand> all;
            for (int a = 1; a <= GEMM_MAX_SPLIT; ++a)
                for (int b = 1; b <= GEMM_MAX_SPLIT; ++b) {
                    const int c[2] = {a, b};
                    GemmArgs G = which == 0 ? ops_gemm_args(p, bb, c, R, nullptr, ks) : mass_gemm_args(p, bb, c, R, nullptr);
                    all.push_back({{a, b}, ks, gemm_model_time(G, std::max(1, ncu / 8) * (ks == 32 ? 2 : 1))});
                }
            std::stable_sort(all.begin(), all.end(), [](const Cand &x, const Cand &y) { return x.model < y.model; });
            // the model's best three, and the even splits 4/4 and 8/8 (the model misses part of what the
            // hardware does: in measurements the ranked and the even splits come within a few percent)
            for (size_t q = 0; q < all.size() && q < 3; ++q) timed.push_back(all[q]);
            for (int e : {4, 8}) {
                bool have = false;
                for (const Cand &c : timed) have = have || (c.kst == ks && c.nk[0] == e && c.nk[1] == e);
                if (!have) timed.push_back({{e, e}, ks, 0.0});
            }
        }
        hipEvent_t e0, e1;
        BEM_HIP(hipEventCreate(&e0));
        BEM_HIP(hipEventCreate(&e1));
        struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } g{e0, e1};
        float best = 1e30f;
        Cand pick = timed.front();
        for (const Cand &c : timed) {
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                GemmArgs G = which == 0 ? ops_gemm_args(p, bb, c.nk, R, nullptr, c.kst) : mass_gemm_args(p, bb, c.nk, R, nullptr);
                BEM_HIP(hipEventRecord(e0, st));
                bem_status q = launch_gemm_f32(ctx, G, st, which == 0 ? K_BLOCK_GEMM : K_MASS_GEMM);
                if (q) return q;
                BEM_HIP(hipEventRecord(e1, st));
                BEM_HIP(hipEventSynchronize(e1));
                float ms = 0;
                BEM_HIP(hipEventElapsedTime(&ms, e0, e1));
                tmin = std::min(tmin, ms);
            }
            if (tmin < best) { best = tmin; pick = c; }
        }
        out = {pick.nk[0], pick.nk[1], pick.kst};
        return BEM_OK;
    }, valid);
    if (s) return s;
    const bool ok = valid(v);
    slot[0] = nk[0] = ok ? v[0] : 4;
    slot[1] = nk[1] = ok ? v[1] : 4;
    slot_kst = kst = ok ? v[2] : 32;
    return BEM_OK;
}

// Y = A X (weak form) for R <= 64 runs through the matrix cores, and Z =
// M^-1 Y when `strong`; run r reads X + r xstride and writes Y + r ystride,
// Z + r zstride.  st (nullable) marks converged runs, which are skipped.
bem_status block_apply(bem_problem *p, const MtfArgs &A, BlockBufs &bb, int R, const double2 *X, int64_t xstride,
                       double2 *Y, int64_t ystride, double2 *Z, int64_t zstride, bool strong, const KrylovState *kst)
{
    hipStream_t st = p->ctx->stream;
    const int nv[2] = {A.ne, A.ni};
    int nk_ops[2] = {0, 0}, nk_mass[2] = {0, 0}, kst_ops = 32, kst_mass = 32;   // (tuning zeroes the right-hand buffers: before packing)
    bem_status s = block_tune(p, bb, 0, R, nk_ops, kst_ops);
    if (!s && strong && p->mass_dense) s = block_tune(p, bb, 1, R, nk_mass, kst_mass);
    if (s) return s;
    for (int m = 0; m < 2; ++m) {
        const int kop = 2 * (int)op_ld(nv[m]);
        hipLaunchKernelGGL(pack_ops_kernel, dim3((int)((op_ld(nv[m]) + 255) / 256), BLOCK_RHS), dim3(256), 0, st, nv[m],
                           kop, R, X, xstride, m == 0 ? 0 : 2 * A.ne, kst, bb.btv[m].as<float>(), bb.btw[m].as<float>());
    }
    BEM_HIP(hipGetLastError());
    GemmArgs G = ops_gemm_args(p, bb, nk_ops, R, kst, kst_ops);
    s = launch_gemm_f32(p->ctx, G, st, K_BLOCK_GEMM);
    if (s) return s;
    BlockC bc;
    for (int m = 0; m < 2; ++m) {
        for (int o = 0; o < 4; ++o) bc.C[m][o] = G.seg[4 * m + o].C;
        bc.nk[m] = nchunks(G.seg[4 * m].K, G.seg[4 * m].kchunk);
    }
    hipLaunchKernelGGL(block_combine_kernel, dim3((A.ne + A.ni + 255) / 256, R), dim3(256), 0, st, A, bc, R, X, xstride,
                       Y, ystride, kst);
    BEM_HIP(hipGetLastError());
    if (!strong) return BEM_OK;
    if (!p->mass_dense) {
        const int64_t n = 2 * A.ne + 2 * A.ni;
        return cheb_apply(p, 0, p->cheb.nparts[0] + p->cheb.nparts[1], 0, 2 * A.ne, n, Y, ystride, Z, zstride,
                          bb.chw.as<double2>(), 6 * n, R, kst, cheb_precond_steps(p));
    }
    for (int m = 0; m < 2; ++m) {
        const int km = minv_ld(nv[m], true);
        hipLaunchKernelGGL(pack_mass_kernel, dim3((km + 255) / 256, 4 * BLOCK_RHS), dim3(256), 0, st, nv[m], km, R,
                           (const double2 *)Y, ystride, m == 0 ? 0 : 2 * A.ne, kst, bb.btm[m].as<float>());
    }
    BEM_HIP(hipGetLastError());
    GemmArgs Gm = mass_gemm_args(p, bb, nk_mass, R, kst);
    s = launch_gemm_f32(p->ctx, Gm, st, K_MASS_GEMM);
    if (s) return s;
    hipLaunchKernelGGL(mass_reduce_kernel, dim3((A.ne + A.ni + 255) / 256, R), dim3(256), 0, st, A.ne, A.ni, Gm.seg[0].C,
                       Gm.seg[1].C, nchunks(Gm.seg[0].K, Gm.seg[0].kchunk), nchunks(Gm.seg[1].K, Gm.seg[1].kchunk),
                       128 * Gm.seg[0].ncb, R, Z, zstride, kst);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

__global__ void set_step_kernel(int *__restrict__ jb, int j0)
{
    if (threadIdx.x == 0) *jb = j0;
}

// Executable graphs of one GMRES run, by step range; destroyed after the
// stream has drained.
struct GraphCache {
    hipStream_t st = nullptr;
    std::map<int, hipGraphExec_t> exec;
    ~GraphCache()
    {
        if (exec.empty()) return;
        (void)hipStreamSynchronize(st);
        for (auto &e : exec) (void)hipGraphExecDestroy(e.second);
    }
};

constexpr int GRAPH_SPAN = 64;   // step indices served by one captured graph (grids sized for the range's end)

struct Gmres {
    bem_problem *p;
    const MtfArgs &A;
    Work &W;
    BlockBufs *bb;         // multi-RHS products (null: one run, split-column kernels)
    KrylovState *hstate;   // pinned: two snapshots of R states, polled alternately
    hipEvent_t *ev;
    int n, nchunk, nrow_blk, nupd, m, R;
    KBatch B;
    double acc64_above = 0.0;   // single run, complex64: FP64 accumulation while the residual estimate exceeds this
    const PmchwtBufs *pm = nullptr;   // exterior PMCHWT system (one run, FP64) instead of the multiple-traces one
    int graph_steps = 0;              // steps issued through captured graphs (all runs of this object)

    // The launches of step j: the operator on u_j (vj, run stride vstride),
    // then the Gram-Schmidt kernels.  With jb the kernels take their step
    // index as j + *jb (device memory) and their grids are sized for steps up
    // to jcap; u_out: where the normalisation also writes u_{j+1}.
    bem_status step(int j, const int *jb, int jcap, int maxit, const double2 *vj, int64_t vstride, double2 *u_out,
                    bool acc64)
    {
        bem_ctx *ctx = p->ctx;
        hipStream_t st = ctx->stream;
        double2 *Vb = W.Vb.as<double2>();
        KrylovState *dst = W.state.as<KrylovState>();
        const dim3 gv(nrow_blk, R);
        bem_status s;
        if (pm)
            s = apply_ext_form(p, *pm, vj, W.y.as<double2>(), W.z.as<double2>(), true, dst, W.part.as<double4>());
        else if (bb)
            s = block_apply(p, A, *bb, R, vj, vstride, W.y.as<double2>(), B.vec, W.z.as<double2>(), B.vec, true, dst);
        else
            s = apply_A(p, A, vj, W.y.as<double2>(), W.z.as<double2>(), true, dst, W.part.as<double4>(), acc64,
                        cheb_precond_steps(p));
        if (s) return s;
        {
            KTimer kt(ctx, K_CGS_DOTS);
            // two columns per wave once one-column waves would exceed about two per SIMD: sharing the
            // reads of u_j and w then pays; below that the halved wave count costs more
            if ((int64_t)nchunk * (jcap + 1) * R >= 2048)
                launch_k(kt, dgs_dots_kernel<2>, dim3(nchunk, (jcap + 1 + 7) / 8, R), dim3(256), 0, st, n, j, jb, Vb,
                         W.z.as<double2>(), W.partial.as<double2>(), dst, B);
            else
                launch_k(kt, dgs_dots_kernel<1>, dim3(nchunk, (jcap + 1 + 3) / 4, R), dim3(256), 0, st, n, j, jb, Vb,
                         W.z.as<double2>(), W.partial.as<double2>(), dst, B);
        }
        {
            KTimer kt(ctx, K_ARNOLDI_FINISH);
            launch_k(kt, dgs_hess_kernel, dim3(R), dim3(256), (size_t)(3 * jcap + 1) * sizeof(double2), st, j, jb,
                     maxit, nchunk, W.partial.as<double2>(), W.coef.as<double2>(), W.hsum.as<double2>(),
                     W.H.as<double2>(), W.R.as<double2>(), W.g.as<double2>(), W.cs.as<double2>(), W.sn.as<double2>(),
                     dst, B);
        }
        if (jb || j < maxit) {
            {
                KTimer kt(ctx, K_CGS_UPDATE);
                launch_k(kt, dgs_update_kernel, dim3(nupd + (jcap + 1 + 3) / 4, R), dim3(256), 0, st, n, j, jb, maxit,
                         nupd, Vb, W.z.as<double2>(), W.coef.as<double2>(), W.H.as<double2>(), W.hsum.as<double2>(),
                         W.npart.as<double>(), dst, B);
            }
            KTimer kt(ctx, K_KRYLOV_NORM);
            launch_k(kt, dgs_normalize_kernel, gv, dim3(256), 0, st, n, j, jb, maxit, nupd, W.npart.as<double>(), Vb,
                     W.coef.as<double2>(), u_out, dst, B);
        }
        BEM_HIP(hipGetLastError());
        return BEM_OK;
    }

    // Steps j0 .. j0 + BATCH - 1 (all below maxit) as one graph launch.  The
    // graph of j0's range is captured on first use: BATCH steps whose kernels
    // add the device step base W.jb to their step offset, the operator read
    // from the fixed operand W.u.  The base is set by a one-thread kernel
    // before each launch.  Capture runs on the context's capture stream (the
    // library's launches follow ctx->stream, swapped for the capture), so the
    // main stream may be the null stream.  Per-kernel event timing is off
    // inside graphs.
    bem_status graph_batch(GraphCache &gc, int j0, int maxit, bool acc64, int batch)
    {
        bem_ctx *ctx = p->ctx;
        hipStream_t st = ctx->stream;
        gc.st = st;
        const int range = j0 / GRAPH_SPAN;
        const int key = 2 * range + (acc64 ? 1 : 0);
        auto it = gc.exec.find(key);
        if (it == gc.exec.end()) {
            const int jcap = std::min((range + 1) * GRAPH_SPAN - 1, maxit - 1);
            const int64_t ustride = R > 1 ? (int64_t)n : 0;
            if (!ctx->capture) BEM_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
            hipStream_t cs = ctx->capture;
            hipGraph_t g = nullptr;
            BEM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            bem_status s = BEM_OK;
            ctx->stream = cs;
            {
                NoTiming nt;
                for (int q = 0; q < batch && !s; ++q)
                    s = step(q, W.jb.as<int>(), jcap, maxit, W.u.as<double2>(), ustride, W.u.as<double2>(), acc64);
            }
            ctx->stream = st;
            const hipError_t e = hipStreamEndCapture(cs, &g);
            if (s) {
                if (e == hipSuccess && g) (void)hipGraphDestroy(g);
                return s;
            }
            BEM_HIP(e);
            hipGraphExec_t x = nullptr;
            const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            BEM_HIP(ei);
            it = gc.exec.emplace(key, x).first;
        }
        hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, W.jb.as<int>(), j0);
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipGraphLaunch(it->second, st));
        return BEM_OK;
    }

    // R independent GMRES runs without restart on M^-1 A x = r0 (r0 already
    // preconditioned; run r's start vector at r0 + r r0stride), x0 = 0,
    // Arnoldi (Gram-Schmidt with delayed re-orthogonalisation) and Givens
    // rotations in FP64 on the device; Krylov spaces of dimension at most
    // `maxit`; run r stops at relative residual tol[r].  Writes x + r B.vec
    // and the final states.
    bem_status run(const double2 *r0, int64_t r0stride, const double *tol, int maxit, double2 *x, KrylovState *fin)
    {
        bem_ctx *ctx = p->ctx;
        hipStream_t st = ctx->stream;
        double2 *Vb = W.Vb.as<double2>();
        KrylovState *dst = W.state.as<KrylovState>();
        const int BATCH = 8;
        const dim3 gv(nrow_blk, R);
        BEM_HIP(hipMemcpyAsync(W.tolv.ptr, tol, (size_t)R * sizeof(double), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(norm_partial_kernel, gv, dim3(256), 0, st, n, r0, r0stride, W.npart.as<double>(), B.npart);
        hipLaunchKernelGGL(normalize_kernel, gv, dim3(256), 0, st, n, nrow_blk, W.npart.as<double>(), B.npart, r0,
                           r0stride, Vb, B.basis, W.beta.as<double>());
        hipLaunchKernelGGL(krylov_init_kernel, dim3((maxit + 256) / 256, R), dim3(256), 0, st, maxit,
                           W.beta.as<double>(), W.tolv.as<double>(), W.g.as<double2>(), dst, B);
        BEM_HIP(hipGetLastError());
        // Issue policy: steps go out in batches of BATCH while the host checks
        // the state snapshot of the previous batch (the device never waits on
        // the host).  Once the observed convergence rate of the slowest run
        // predicts the end within the steps already queued plus two batches,
        // each step is followed by a synchronous check, so no step is issued
        // after the one that completes the last run.
        const size_t sb = (size_t)R * sizeof(KrylovState);
        std::vector<int> last_j(R, 0);
        std::vector<double> last_res(R, 1.0);
        int slot = 0, pending = -1;
        bool sync_mode = false, stop = false;
        bool acc64 = acc64_above > 0.0;   // switched off once a polled estimate falls below acc64_above
        auto all_done = [&](const KrylovState *k) {
            for (int r = 0; r < R; ++r)
                if (!k[r].done) return false;
            return true;
        };
        // step j applies the operator to u_j and completes dimension j (j = maxit: completion only).
        // Whole batches of BATCH full steps after the first go out as one captured HIP graph per
        // range of GRAPH_SPAN step indices (device step base, grids sized for the range's end).
        const bool graphs = p->graphs && maxit >= 2 * BATCH;
        if (graphs) {
            bem_status q = dev_alloc(ctx, W.u, (size_t)std::max(R, 1) * n * sizeof(double2));
            if (!q) q = dev_alloc(ctx, W.jb, sizeof(int));
            if (q) return q;
            BEM_HIP(hipMemcpy2DAsync(W.u.ptr, (size_t)n * sizeof(double2), Vb,
                                     (size_t)(R > 1 ? B.basis : n) * sizeof(double2), (size_t)n * sizeof(double2),
                                     R, hipMemcpyDeviceToDevice, st));
        }
        GraphCache gc;
        for (int j = 0; j <= maxit && !stop;) {
            bem_status s;
            if (graphs && !sync_mode && j >= BATCH && j % BATCH == 0 && j + BATCH <= maxit) {
                s = graph_batch(gc, j, maxit, acc64, BATCH);
                if (s) return s;
                j += BATCH;
                graph_steps += BATCH;
            } else {
                s = step(j, nullptr, j, maxit, Vb + (size_t)j * n, B.basis, graphs ? W.u.as<double2>() : nullptr,
                         acc64);
                if (s) return s;
                ++j;
            }
            const int issued = j;
            KrylovState *hs = hstate + (size_t)slot * R;
            if (sync_mode) {
                BEM_HIP(hipMemcpyAsync(hs, dst, sb, hipMemcpyDeviceToHost, st));
                BEM_HIP(hipStreamSynchronize(st));
                stop = all_done(hs);
                if (acc64 && hs[0].resid < acc64_above) acc64 = false;
                continue;
            }
            if (issued % BATCH != 0) continue;
            BEM_HIP(hipMemcpyAsync(hs, dst, sb, hipMemcpyDeviceToHost, st));
            BEM_HIP(hipEventRecord(ev[slot], st));
            if (pending >= 0) {
                BEM_HIP(hipEventSynchronize(ev[pending]));
                const KrylovState *k = hstate + (size_t)pending * R;
                if (all_done(k)) { stop = true; break; }
                if (acc64 && k[0].resid < acc64_above) acc64 = false;
                // steps still to go at the observed geometric rate of the slowest run
                double togo = 0.0;
                int seen = issued;
                for (int r = 0; r < R; ++r) {
                    if (k[r].done) continue;
                    seen = std::min(seen, k[r].iters);
                    if (last_j[r] > 0 && k[r].iters > last_j[r] && k[r].resid > 0 && last_res[r] > 0) {
                        const double rate = std::pow(k[r].resid / last_res[r], 1.0 / (k[r].iters - last_j[r]));
                        togo = std::max(togo, rate < 1.0 ? std::log(tol[r] / k[r].resid) / std::log(rate) : 1e30);
                    } else {
                        togo = 1e30;
                    }
                    last_j[r] = k[r].iters;
                    last_res[r] = k[r].resid;
                }
                if (togo <= (issued - seen) + 2 * BATCH) sync_mode = true;
            }
            pending = slot;
            slot ^= 1;
        }
        KrylovState *hs = hstate + (size_t)slot * R;
        BEM_HIP(hipMemcpyAsync(hs, dst, sb, hipMemcpyDeviceToHost, st));
        BEM_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < R; ++r) fin[r] = hs[r];
        // back substitution of every run and x = V y on the device (y in W.yc, [R][maxit + 1])
        if (maxit + 1 > 12 * 256) return set_error(BEM_E_ARG, "internal: back substitution size");
        hipLaunchKernelGGL(backsub_kernel, dim3(R), dim3(256), (size_t)(maxit + 1) * sizeof(double2), st, maxit,
                           W.R.as<double2>(), W.g.as<double2>(), dst, B, W.yc.as<double2>());
        hipLaunchKernelGGL(combine_kernel, dim3(nrow_blk, R), dim3(256), 0, st, n, maxit, Vb, B.basis,
                           W.yc.as<double2>(), x, B.vec, dst);
        BEM_HIP(hipGetLastError());
        return BEM_OK;
    }
};

__global__ void axpy_add_kernel(int n, const double2 *__restrict__ d, double2 *__restrict__ x)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) x[r] = make_double2(x[r].x + d[r].x, x[r].y + d[r].y);
}

__global__ void zero_kernel(int64_t n, double2 *__restrict__ x)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) x[r] = make_double2(0, 0);
}

}  // namespace

bem_status matvec_impl(bem_problem *p, const void *x, void *y, int strong, bem_memspace space)
{
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    const size_t bytes = (size_t)n * sizeof(double2);
    DevMem xu, xi, yi, zi, yu, part;
    bem_status s = dev_alloc(ctx, xu, bytes);
    if (!s) s = dev_alloc(ctx, part, split_part_bytes(ne, ni));
    if (!s) s = dev_alloc(ctx, xi, bytes);
    if (!s) s = dev_alloc(ctx, yi, bytes);
    if (!s) s = dev_alloc(ctx, zi, bytes);
    if (!s) s = dev_alloc(ctx, yu, bytes);
    if (s) return s;
    BEM_HIP(hipMemcpyAsync(xu.ptr, x, bytes, space == BEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
    const dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                       p->inte->d.perm.as<int32_t>(), xu.as<double2>(), xi.as<double2>(), 1);
    s = mtf_tune(p, xi.as<double2>(), yi.as<double2>(), part.as<double4>());
    if (s) return s;
    MtfArgs A = make_args(p);
    s = apply_A(p, A, xi.as<double2>(), yi.as<double2>(), zi.as<double2>(), strong != 0, nullptr, part.as<double4>());
    if (s) return s;
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                       p->inte->d.perm.as<int32_t>(), strong ? zi.as<double2>() : yi.as<double2>(), yu.as<double2>(), 0);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipMemcpyAsync(y, yu.ptr, bytes, space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    BEM_HIP(hipStreamSynchronize(st));
    return BEM_OK;
}

// ---- the product without allocations: work buffers in one static device
// array per GPU, for callers that cannot allocate (graph capture, tight
// serving loops).  Host code never passes the array's name to a kernel (in
// host code it is a stand-in, not a device address): its address on each
// device is looked up once, at context creation with that device current,
// and kept per device.

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;   // device -> address of that device's copy of `scratch`
}  // namespace

bem_status noalloc_scratch_init(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return BEM_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_error(BEM_E_DEVICE, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[device] = ptr;
    return BEM_OK;
}

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

// Work buffers of one product carved from the static array: the permuted
// input, the weak and strong results (n complex128 each) and the partial
// sums of the tile and inverse-mass kernels.
static size_t noalloc_need(int ne, int ni, size_t off[4])
{
    const size_t vb = ((size_t)(2 * ne + 2 * ni) * sizeof(double2) + 255) & ~size_t(255);
    off[0] = 0;
    off[1] = vb;
    off[2] = 2 * vb;
    off[3] = 3 * vb;
    return 3 * vb + split_part_bytes(ne, ni);
}

bem_status matvec_noalloc_impl(bem_problem *p, const void *x, void *y, int strong)
{
    bem_ctx *ctx = p->ctx;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    size_t off[4];
    const size_t need = noalloc_need(ne, ni, off);
    if (need > NOALLOC_SCRATCH_BYTES)
        return set_error(BEM_E_UNSUPPORTED, "bem_mtf_matvec_noalloc: the product needs " + std::to_string(need) +
                                                " bytes of work space, more than the static " +
                                                std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte array");
    if (!p->ops_ready || !p->proj_ready) return set_error(BEM_E_STATE, "assemble operators and projection first");
    BEM_HIP(hipSetDevice(ctx->device));
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch_ptr.find(ctx->device);
        if (it == g_scratch_ptr.end()) return set_error(BEM_E_STATE, "static work array not set up on this device");
        base = static_cast<unsigned char *>(it->second);
    }
    double2 *xi = reinterpret_cast<double2 *>(base + off[0]);
    double2 *yi = reinterpret_cast<double2 *>(base + off[1]);
    double2 *zi = reinterpret_cast<double2 *>(base + off[2]);
    double4 *part = reinterpret_cast<double4 *>(base + off[3]);
    hipStream_t st = ctx->stream;
    NoTiming nt;   // per-kernel timing would take events from the context's pool
    const dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                       p->inte->d.perm.as<int32_t>(), static_cast<const double2 *>(x), xi, 1);
    MtfArgs A = make_args(p);
    bem_status s = apply_A(p, A, xi, yi, zi, strong != 0, nullptr, part);
    if (s) return s;
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                       p->inte->d.perm.as<int32_t>(), strong ? zi : yi, static_cast<double2 *>(y), 0);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

bem_status matvec_batch_impl(bem_problem *p, const void *x, void *y, int nrhs, int strong, bem_memspace space)
{
    bem_ctx *ctx = p->ctx;
    if (p->prec != BEM_C64_MIXED) {
        const size_t nb = (size_t)(2 * p->ext->h.nv + 2 * p->inte->h.nv) * sizeof(double2);
        for (int r = 0; r < nrhs; ++r) {
            bem_status s = matvec_impl(p, static_cast<const char *>(x) + r * nb, static_cast<char *>(y) + r * nb,
                                       strong, space);
            if (s) return s;
        }
        return BEM_OK;
    }
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    const int R = std::min(nrhs, BLOCK_RHS);
    const size_t vb = (size_t)n * sizeof(double2);
    DevMem xu, xi, yi, zi;
    BlockBufs bb;
    bem_status s = dev_alloc(ctx, xu, R * vb);
    if (!s) s = dev_alloc(ctx, xi, R * vb);
    if (!s) s = dev_alloc(ctx, yi, R * vb);
    if (!s) s = dev_alloc(ctx, zi, R * vb);
    if (!s) s = block_alloc(p, bb);
    if (s) return s;
    const MtfArgs A = make_args(p);
    const dim3 g((n + 255) / 256);
    for (int r0 = 0; r0 < nrhs; r0 += R) {
        const int Rc = std::min(R, nrhs - r0);
        BEM_HIP(hipMemcpyAsync(xu.ptr, static_cast<const char *>(x) + r0 * vb, Rc * vb,
                               space == BEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
        for (int r = 0; r < Rc; ++r)
            hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                               p->inte->d.perm.as<int32_t>(), xu.as<double2>() + (size_t)r * n,
                               xi.as<double2>() + (size_t)r * n, 1);
        s = block_apply(p, A, bb, Rc, xi.as<double2>(), n, yi.as<double2>(), n, zi.as<double2>(), n, strong != 0,
                        nullptr);
        if (s) return s;
        for (int r = 0; r < Rc; ++r)
            hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                               p->inte->d.perm.as<int32_t>(), (strong ? zi : yi).as<double2>() + (size_t)r * n,
                               xu.as<double2>() + (size_t)r * n, 0);
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipMemcpyAsync(static_cast<char *>(y) + r0 * vb, xu.ptr, Rc * vb,
                               space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
        BEM_HIP(hipStreamSynchronize(st));
    }
    return BEM_OK;
}

static bem_status rhs_internal(bem_problem *p, const double *d, double2 *b)
{
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    hipLaunchKernelGGL(rhs_kernel, dim3((n + 255) / 256), dim3(256), 0, p->ctx->stream, ne, ni,
                       p->ext->d.star_ptr.as<int32_t>(), p->ext->d.star_ent.as<int32_t>(), p->ext->d.geo.as<TriGeo>(),
                       p->k_ext, p->incident, d[0], d[1], d[2], b);
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

int solve_runs(const bem_problem *p, const bem_solver_opts *opts)
{
    return (p->prec == BEM_C64_MIXED && opts->batch > 1) ? std::min(opts->batch, BLOCK_RHS) : 1;
}

bem_status solve_impl(bem_problem *p, const double *dirs, int nrhs, const bem_solver_opts *opts, void *traces,
                      bem_memspace space, bem_stats *stats)
{
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    const int m = opts->maxit;
    if (m > MAXIT_CAP) return set_error(BEM_E_ARG, "maxit above 3000");
    const bool mixed = p->prec == BEM_C64_MIXED;
    const int ir_max = opts->ir_max > 0 ? opts->ir_max : 10;
    const int R = std::min(solve_runs(p, opts), nrhs);   // runs advancing together
    const size_t vb = (size_t)n * sizeof(double2);
    const int nchunk = (n + cgs_chunk(n) - 1) / cgs_chunk(n);
    const int nrow_blk = (n + 255) / 256, nupd = (n + UPD_ROWS - 1) / UPD_ROWS;
    Work W;
    bem_status s = dev_alloc(ctx, W.y, R * vb);
    if (!s) s = dev_alloc(ctx, W.z, R * vb);
    if (!s) s = dev_alloc(ctx, W.b, R * vb);
    if (!s) s = dev_alloc(ctx, W.r, R * vb);
    if (!s) s = dev_alloc(ctx, W.xin, R * vb);
    if (!s) s = dev_alloc(ctx, W.d, R * vb);   // refinement corrections (mixed) or the restart correction (FP64)
    if (!s) s = dev_alloc(ctx, W.Vb, (size_t)R * (m + 1) * vb);
    if (!s) s = dev_alloc(ctx, W.partial, (size_t)R * nchunk * 2 * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.hsum, (size_t)R * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.beta, sizeof(double) * (R + 1));
    if (!s) s = dev_alloc(ctx, W.tolv, sizeof(double) * R);
    if (!s) s = dev_alloc(ctx, W.yc, (size_t)R * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.npart, (size_t)R * std::max(nrow_blk, nupd) * sizeof(double));
    if (!s) s = dev_alloc(ctx, W.R, (size_t)R * m * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.H, (size_t)R * m * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.coef, (size_t)R * (2 * m + 4) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.g, (size_t)R * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.cs, (size_t)R * m * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.sn, (size_t)R * m * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.state, R * sizeof(KrylovState));
    if (!s) s = dev_alloc(ctx, W.part, split_part_bytes(ne, ni));
    if (s) return s;
    BlockBufs bb;
    if (R > 1) {
        if (!p->mass_dense && p->mass_sparse && block_dense_mass(p, R)) {   // the block product's inverse masses
            for (int m = 0; m < 2 && !s; ++m) s = launch_mass_inverse(p, m, st);
            if (s) return s;
            p->mass_dense = true;
        }
        s = block_alloc(p, bb);
        if (s) return s;
    }
    // M^-1 of the right-hand sides and residuals: the same operator as in the GMRES steps (the block
    // product applies the dense inverses when they are present, else both take the preconditioner's
    // Chebyshev steps)
    const int kpre = R > 1 && p->mass_dense ? cheb_steps(p) : cheb_precond_steps(p);
    KrylovState *hstate = nullptr;   // two pinned snapshots of the R states
    BEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&hstate), 2 * R * sizeof(KrylovState), hipHostMallocDefault));
    struct PinGuard { KrylovState *p; ~PinGuard() { if (p) (void)hipHostFree(p); } } guard{hstate};
    hipEvent_t ev[2];
    BEM_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    BEM_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    struct EvGuard { hipEvent_t *e; ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); } } eguard{ev};
    s = mtf_tune(p, W.xin.as<double2>(), W.y.as<double2>(), W.part.as<double4>());
    if (s) return s;
    const MtfArgs A = make_args(p);
    const size_t finish_lds = (size_t)(3 * m + 1) * sizeof(double2);
    BEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&dgs_hess_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)finish_lds));
    KBatch B{};
    if (R > 1) {
        B.basis = (int64_t)(m + 1) * n;
        B.vec = n;
        B.partial = (int64_t)nchunk * 2 * (m + 1);
        B.small = m + 1;
        B.npart = std::max(nrow_blk, nupd);
        B.hess = (int64_t)m * (m + 1);
        B.rot = m;
        B.coef = 2 * m + 4;
    }
    Gmres gm{p, A, W, R > 1 ? &bb : nullptr, hstate, ev, n, nchunk, nrow_blk, nupd, m, R, B};
    const dim3 gv(nrow_blk);
    double *beta = W.beta.as<double>();   // [0, R) ||M^-1 b|| of each run; [R] residual norm
    int total_it = 0, total_ir = 0;
    double worst_res = 0.0;
    bool all_conv = true;
    auto t0 = std::chrono::steady_clock::now();
    // true strong-form residual of run r in FP64 arithmetic: W.z_r = M^-1 (b_r - A x_r), its norm into beta[R]
    auto residual = [&](int r) -> bem_status {
        double2 *yr = W.y.as<double2>() + (size_t)r * n, *rr = W.r.as<double2>() + (size_t)r * n;
        double2 *zr = W.z.as<double2>() + (size_t)r * n;
        bem_status q = apply_A(p, A, W.xin.as<double2>() + (size_t)r * n, yr, zr, false, nullptr, W.part.as<double4>(),
                               true);
        if (q) return q;
        hipLaunchKernelGGL(axpy_sub_kernel, gv, dim3(256), 0, st, n, W.b.as<double2>() + (size_t)r * n, yr, rr);
        q = apply_Minv(p, rr, zr, W.part.as<double4>(), nullptr, kpre);
        if (q) return q;
        return norm_to(p, n, zr, W.npart.as<double>(), yr, beta + R);
    };
    std::vector<KrylovState> fin(R);
    std::vector<double> b0(R), rel(R), tolr(R);
    for (int g0 = 0; g0 < nrhs; g0 += R) {
        const int Rg = std::min(R, nrhs - g0);
        // b and r0 = M^-1 b (x0 = 0) of every run; runs past Rg start from zero
        for (int r = 0; r < R; ++r) {
            double2 *br = W.b.as<double2>() + (size_t)r * n, *rr = W.r.as<double2>() + (size_t)r * n;
            if (r < Rg) {
                s = rhs_internal(p, dirs + 3 * (g0 + r), br);
                if (!s) s = apply_Minv(p, br, rr, W.part.as<double4>(), nullptr, kpre);
                if (s) return s;
            } else {
                hipLaunchKernelGGL(zero_kernel, gv, dim3(256), 0, st, (int64_t)n, br);
                hipLaunchKernelGGL(zero_kernel, gv, dim3(256), 0, st, (int64_t)n, rr);
            }
        }
        std::vector<double> rn(R, 0.0);
        if (!mixed) {
            tolr.assign(R, opts->tol);
            s = gm.run(W.r.as<double2>(), n, tolr.data(), m, W.xin.as<double2>(), fin.data());
            if (s) return s;
            for (int r = 0; r < Rg; ++r) {
                total_it += fin[r].iters;
                b0[r] = fin[r].beta0;
                s = residual(r);
                if (s) return s;
                BEM_HIP(hipMemcpyAsync(&rn[r], beta + R, sizeof(double), hipMemcpyDeviceToHost, st));
                BEM_HIP(hipStreamSynchronize(st));
            }
            // Success is decided on the true residual.  The Arnoldi estimate
            // can drift from it (its norm update subtracts squares); when the
            // estimate met the tolerance and the true residual did not, one
            // restart solves for the correction from the true residual
            // M^-1 (b - A x) (in W.z) with the remaining steps.
            if (R == 1 && Rg == 1 && b0[0] > 0.0 && rn[0] / b0[0] > opts->tol && fin[0].resid <= opts->tol &&
                fin[0].iters < m) {
                double tr = opts->tol * b0[0] / rn[0];
                KrylovState fin2;
                s = gm.run(W.z.as<double2>(), n, &tr, m - fin[0].iters, W.d.as<double2>(), &fin2);
                if (s) return s;
                total_it += fin2.iters;
                hipLaunchKernelGGL(axpy_add_kernel, gv, dim3(256), 0, st, n, W.d.as<double2>(), W.xin.as<double2>());
                s = residual(0);
                if (s) return s;
                BEM_HIP(hipMemcpyAsync(&rn[0], beta + R, sizeof(double), hipMemcpyDeviceToHost, st));
                BEM_HIP(hipStreamSynchronize(st));
                ++total_ir;
            }
            for (int r = 0; r < Rg; ++r)
                if (!(b0[r] > 0.0 ? rn[r] / b0[r] <= opts->tol : true)) all_conv = false;
        } else {
            // Iterative refinement: x += d where d solves the FP32-product
            // system M^-1 A d = M^-1 (b - A x) to a relative tolerance that
            // aims at the outer target; the residual of every step is
            // recomputed with FP64 arithmetic.  Runs that have met the
            // target start the next step from zero (and so sit it out).
            hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((R * (int64_t)n + 255) / 256)), dim3(256), 0, st,
                               (int64_t)R * n, W.xin.as<double2>());
            hipLaunchKernelGGL(norm_partial_kernel, dim3(nrow_blk, R), dim3(256), 0, st, n, W.r.as<double2>(),
                               (int64_t)n, W.npart.as<double>(), (int64_t)nrow_blk);
            hipLaunchKernelGGL(normalize_kernel, dim3(nrow_blk, R), dim3(256), 0, st, n, nrow_blk, W.npart.as<double>(),
                               (int64_t)nrow_blk, W.r.as<double2>(), (int64_t)n, W.z.as<double2>(), (int64_t)n, beta);
            BEM_HIP(hipGetLastError());
            BEM_HIP(hipMemcpyAsync(b0.data(), beta, R * sizeof(double), hipMemcpyDeviceToHost, st));
            BEM_HIP(hipStreamSynchronize(st));
            const double2 *rhs_s = W.r.as<double2>();   // preconditioned residuals of the current x
            for (int r = 0; r < R; ++r) rel[r] = b0[r] > 0.0 ? 1.0 : 0.0;
            int used = 0, steps = 0;
            auto active = [&](int r) { return r < Rg && rel[r] > opts->tol; };
            for (;;) {
                bool any = false;
                for (int r = 0; r < R; ++r) any = any || active(r);
                if (!any || steps >= ir_max || used >= m) break;
                for (int r = 0; r < R; ++r) {
                    tolr[r] = opts->ir_inner_tol > 0 ? opts->ir_inner_tol : std::max(0.5 * opts->tol / rel[r], 1e-7);
                    if (!active(r))   // start vector zero: the run is done at once
                        hipLaunchKernelGGL(zero_kernel, gv, dim3(256), 0, st, (int64_t)n,
                                           const_cast<double2 *>(rhs_s) + (size_t)r * n);
                }
                // Inexact Krylov: the product error a GMRES step tolerates grows as
                // the residual falls (relative to the target), so the single-run
                // inner solve accumulates the complex64 products in FP64 while
                // its residual estimate is above 2e4 times its tolerance and in
                // FP32 after that; the early FP32 errors would otherwise leave a
                // gap between the estimate and the true residual that costs a
                // restarted refinement step.  (Block runs: FP32 matrix cores.)
                gm.acc64_above = R == 1 ? std::min(1.0, 2e4 * tolr[0]) : 0.0;
                s = gm.run(rhs_s, n, tolr.data(), m - used, W.d.as<double2>(), fin.data());
                if (s) return s;
                int most = 0;
                for (int r = 0; r < R; ++r) {
                    most = std::max(most, fin[r].iters);
                    if (r < Rg) total_it += fin[r].iters;
                }
                used += most;
                ++steps;
                for (int r = 0; r < Rg; ++r) {
                    if (!active(r)) continue;
                    hipLaunchKernelGGL(axpy_add_kernel, gv, dim3(256), 0, st, n, W.d.as<double2>() + (size_t)r * n,
                                       W.xin.as<double2>() + (size_t)r * n);
                    s = residual(r);
                    if (s) return s;
                    BEM_HIP(hipMemcpyAsync(&rn[r], beta + R, sizeof(double), hipMemcpyDeviceToHost, st));
                    BEM_HIP(hipStreamSynchronize(st));
                    rel[r] = rn[r] / b0[r];
                }
                rhs_s = W.z.as<double2>();
                if (most == 0) break;   // no progress possible
            }
            total_ir += steps;
            for (int r = 0; r < Rg; ++r) {
                rn[r] = rel[r] * b0[r];
                if (!(rel[r] <= opts->tol)) all_conv = false;
            }
        }
        // traces in caller numbering
        for (int r = 0; r < Rg; ++r) {
            hipLaunchKernelGGL(permute_vec_kernel, gv, dim3(256), 0, st, ne, ni, p->ext->d.perm.as<int32_t>(),
                               p->inte->d.perm.as<int32_t>(), W.xin.as<double2>() + (size_t)r * n,
                               W.y.as<double2>() + (size_t)r * n, 0);
            BEM_HIP(hipGetLastError());
            worst_res = std::max(worst_res, b0[r] > 0 ? rn[r] / b0[r] : 0.0);
        }
        BEM_HIP(hipMemcpyAsync(static_cast<double2 *>(traces) + (size_t)g0 * n, W.y.ptr, Rg * vb,
                               space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
        BEM_HIP(hipStreamSynchronize(st));
    }
    const double t_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    s = resolve_assembly_timing(p);
    if (s) return s;
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->iterations = total_it;
        stats->ir_steps = total_ir;
        stats->rel_residual = worst_res;
        stats->t_geometry_ms = p->t_geometry_ms;
        stats->t_regular_ms = p->t_regular_ms;
        stats->t_singular_ms = p->t_singular_ms;
        stats->t_projection_ms = p->t_projection_ms;
        stats->t_matrix_ms = p->t_assembly_ms + p->t_projection_ms;
        stats->t_assembly_ms = p->t_assembly_ms;
        stats->t_solve_ms = t_solve;
        stats->t_iter_ms = total_it > 0 ? t_solve / total_it : 0.0;
        stats->graph_steps = gm.graph_steps;
    }
    return all_conv ? BEM_OK : set_error(BEM_W_NOCONV, "GMRES reached maxit before the tolerance");
}

// [f; g] of the PMCHWT system from the multiple-traces right-hand side [-f; -g; 0; 0]
__global__ void pmchwt_rhs_kernel(int n, const double2 *__restrict__ b_mtf, double2 *__restrict__ b)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) b[r] = make_double2(-b_mtf[r].x, -b_mtf[r].y);
}

// Exterior formulations (Sec. 3.3): PMCHWT (Eq. "pmchwt:discrete", unknowns
// [gamma_D p, gamma_N p], right-hand side [f; g]) or high-contrast Neumann
// (Eq. "highcontrast:ext:neu", unknowns [gamma_N p, mu], right-hand side
// [c hat(D_i) M_e^-1 f; g]); GMRES without restart on the mass-preconditioned
// form M_e^-1 A x = M_e^-1 rhs, one right-hand side at a time, FP64
// throughout.
bem_status ext_form_solve_impl(bem_problem *p, int form, const double *dirs, int nrhs, const bem_solver_opts *opts,
                               void *traces, bem_memspace space, bem_stats *stats)
{
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (p->prec != BEM_C128) return set_error(BEM_E_UNSUPPORTED, "exterior formulations: complex128 problems only");
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne, nm = 2 * ne + 2 * ni;
    const int m = opts->maxit;
    const int R = 1;
    const size_t vb = (size_t)n * sizeof(double2);
    const int nchunk = (n + cgs_chunk(n) - 1) / cgs_chunk(n);
    const int nrow_blk = (n + 255) / 256, nupd = (n + UPD_ROWS - 1) / UPD_ROWS;
    Work W;
    bem_status s = dev_alloc(ctx, W.y, vb);
    if (!s) s = dev_alloc(ctx, W.z, vb);
    if (!s) s = dev_alloc(ctx, W.b, (size_t)nm * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.d, vb);
    if (!s) s = dev_alloc(ctx, W.r, vb);
    if (!s) s = dev_alloc(ctx, W.xin, vb);
    if (!s) s = dev_alloc(ctx, W.Vb, (size_t)(m + 1) * vb);
    if (!s) s = dev_alloc(ctx, W.partial, (size_t)nchunk * 2 * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.hsum, (size_t)(m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.beta, sizeof(double) * (R + 1));
    if (!s) s = dev_alloc(ctx, W.tolv, sizeof(double) * R);
    if (!s) s = dev_alloc(ctx, W.yc, (size_t)R * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.npart, (size_t)std::max(nrow_blk, nupd) * sizeof(double));
    if (!s) s = dev_alloc(ctx, W.R, (size_t)m * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.H, (size_t)m * (m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.coef, (size_t)(2 * m + 4) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.g, (size_t)(m + 1) * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.cs, (size_t)m * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.sn, (size_t)m * sizeof(double2));
    if (!s) s = dev_alloc(ctx, W.state, sizeof(KrylovState));
    if (!s) s = dev_alloc(ctx, W.part, split_part_bytes(ne, ni));
    PmchwtBufs pb;
    pb.form = form;
    if (!s) s = pmchwt_alloc(p, pb);
    if (s) return s;
    KrylovState *hstate = nullptr;
    BEM_HIP(hipHostMalloc(reinterpret_cast<void **>(&hstate), 2 * R * sizeof(KrylovState), hipHostMallocDefault));
    struct PinGuard { KrylovState *p; ~PinGuard() { if (p) (void)hipHostFree(p); } } guard{hstate};
    hipEvent_t ev[2];
    BEM_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    BEM_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    struct EvGuard { hipEvent_t *e; ~EvGuard() { (void)hipEventDestroy(e[0]); (void)hipEventDestroy(e[1]); } } eguard{ev};
    const size_t finish_lds = (size_t)(3 * m + 1) * sizeof(double2);
    BEM_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&dgs_hess_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)finish_lds));
    KBatch B{};
    Gmres gm{p, pb.A0, W, nullptr, hstate, ev, n, nchunk, nrow_blk, nupd, m, R, B};
    gm.pm = &pb;
    const dim3 gv(nrow_blk);
    double *beta = W.beta.as<double>();
    double2 *bp = W.d.as<double2>();
    int total_it = 0;
    double worst_res = 0.0;
    bool all_conv = true;
    auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < nrhs; ++r) {
        s = rhs_internal(p, dirs + 3 * r, W.b.as<double2>());
        if (s) return s;
        if (form == FORM_HCN) {
            hipLaunchKernelGGL(pmchwt_rhs_kernel, gv, dim3(256), 0, st, n, W.b.as<double2>(), W.z.as<double2>());
            s = hcn_rhs(p, pb, W.z.as<double2>(), bp, W.part.as<double4>());
            if (s) return s;
        } else {
            hipLaunchKernelGGL(pmchwt_rhs_kernel, gv, dim3(256), 0, st, n, W.b.as<double2>(), bp);
        }
        s = apply_Minv_mesh(p, 0, bp, W.r.as<double2>(), W.part.as<double4>(), nullptr);
        if (s) return s;
        KrylovState fin;
        const double tol = opts->tol;
        s = gm.run(W.r.as<double2>(), n, &tol, m, W.xin.as<double2>(), &fin);
        if (s) return s;
        total_it += fin.iters;
        // true strong-form residual M_e^-1 (b - A x), FP64 (left in W.z, its norm in rn)
        double rn = 0.0;
        auto residual = [&]() -> bem_status {
            bem_status q = apply_ext_form(p, pb, W.xin.as<double2>(), W.y.as<double2>(), nullptr, false, nullptr,
                                          W.part.as<double4>());
            if (q) return q;
            hipLaunchKernelGGL(axpy_sub_kernel, gv, dim3(256), 0, st, n, bp, W.y.as<double2>(), W.r.as<double2>());
            q = apply_Minv_mesh(p, 0, W.r.as<double2>(), W.z.as<double2>(), W.part.as<double4>(), nullptr);
            if (!q) q = norm_to(p, n, W.z.as<double2>(), W.npart.as<double>(), W.y.as<double2>(), beta + R);
            if (q) return q;
            BEM_HIP(hipMemcpyAsync(&rn, beta + R, sizeof(double), hipMemcpyDeviceToHost, st));
            BEM_HIP(hipStreamSynchronize(st));
            return BEM_OK;
        };
        s = residual();
        if (s) return s;
        // Success is decided on the true residual, as for the multiple-traces
        // system: when the Arnoldi estimate met the tolerance and the true
        // residual did not, one restart solves for the correction from
        // M_e^-1 (b - A x) with the remaining steps (W.r is free here).
        if (fin.beta0 > 0 && rn / fin.beta0 > opts->tol && fin.resid <= opts->tol && fin.iters < m) {
            const double tr = opts->tol * fin.beta0 / rn;
            KrylovState fin2;
            s = gm.run(W.z.as<double2>(), n, &tr, m - fin.iters, W.r.as<double2>(), &fin2);
            if (s) return s;
            total_it += fin2.iters;
            hipLaunchKernelGGL(axpy_add_kernel, gv, dim3(256), 0, st, n, W.r.as<double2>(), W.xin.as<double2>());
            s = residual();
            if (s) return s;
        }
        const double rel = fin.beta0 > 0 ? rn / fin.beta0 : 0.0;
        worst_res = std::max(worst_res, rel);
        if (!(rel <= opts->tol)) all_conv = false;
        hipLaunchKernelGGL(permute_vec_kernel, gv, dim3(256), 0, st, ne, 0, p->ext->d.perm.as<int32_t>(),
                           p->ext->d.perm.as<int32_t>(), W.xin.as<double2>(), W.y.as<double2>(), 0);
        BEM_HIP(hipGetLastError());
        BEM_HIP(hipMemcpyAsync(static_cast<double2 *>(traces) + (size_t)r * n, W.y.ptr, vb,
                               space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
        BEM_HIP(hipStreamSynchronize(st));
    }
    const double t_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    s = resolve_assembly_timing(p);
    if (s) return s;
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->iterations = total_it;
        stats->rel_residual = worst_res;
        stats->t_geometry_ms = p->t_geometry_ms;
        stats->t_regular_ms = p->t_regular_ms;
        stats->t_singular_ms = p->t_singular_ms;
        stats->t_projection_ms = p->t_projection_ms;
        stats->t_matrix_ms = p->t_assembly_ms + p->t_projection_ms;
        stats->t_assembly_ms = p->t_assembly_ms;
        stats->t_solve_ms = t_solve;
        stats->t_iter_ms = total_it > 0 ? t_solve / total_it : 0.0;
        stats->graph_steps = gm.graph_steps;
    }
    return all_conv ? BEM_OK : set_error(BEM_W_NOCONV, "GMRES reached maxit before the tolerance");
}

// y = A x or M_e^-1 A x of an exterior formulation; x, y: [2 N_ext] caller numbering
bem_status ext_form_matvec_impl(bem_problem *p, int form, const void *x, void *y, int strong, bem_memspace space)
{
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (p->prec != BEM_C128) return set_error(BEM_E_UNSUPPORTED, "exterior formulations: complex128 problems only");
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne;
    const size_t bytes = (size_t)n * sizeof(double2);
    DevMem xu, xi, yi, zi, yu, part;
    PmchwtBufs pb;
    pb.form = form;
    bem_status s = dev_alloc(ctx, xu, bytes);
    if (!s) s = dev_alloc(ctx, xi, bytes);
    if (!s) s = dev_alloc(ctx, yi, bytes);
    if (!s) s = dev_alloc(ctx, zi, bytes);
    if (!s) s = dev_alloc(ctx, yu, bytes);
    if (!s) s = dev_alloc(ctx, part, split_part_bytes(ne, ni));
    if (!s) s = pmchwt_alloc(p, pb);
    if (s) return s;
    BEM_HIP(hipMemcpyAsync(xu.ptr, x, bytes, space == BEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
    const dim3 g((n + 255) / 256);
    const int32_t *pe = p->ext->d.perm.as<int32_t>();
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, 0, pe, pe, xu.as<double2>(), xi.as<double2>(), 1);
    s = apply_ext_form(p, pb, xi.as<double2>(), yi.as<double2>(), zi.as<double2>(), strong != 0, nullptr,
                       part.as<double4>());
    if (s) return s;
    hipLaunchKernelGGL(permute_vec_kernel, g, dim3(256), 0, st, ne, 0, pe, pe,
                       strong ? zi.as<double2>() : yi.as<double2>(), yu.as<double2>(), 0);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipMemcpyAsync(y, yu.ptr, bytes, space == BEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    BEM_HIP(hipStreamSynchronize(st));
    return BEM_OK;
}

}  // namespace bemtx
