// C-ABI entry points: contexts, meshes, problems, assembly orchestration and
// copies out.  Kernels live in assemble.hip and solve.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"
#include "phase.h"

namespace bemtx {

static thread_local std::string g_last_error = "no error";

bem_status set_error(bem_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

bem_status hip_error(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return set_error(BEM_E_OOM, std::string("device allocation failed in ") + what);
    return set_error(BEM_E_DEVICE, std::string(hipGetErrorString(e)) + " in " + what);
}

// Released blocks go to the context's reuse cache (size classes: powers of
// two up to 1 MiB, then multiples of 2 MiB), so repeated solves and meshes of
// the same sizes allocate without hipMalloc / hipFree.
static size_t size_class(size_t bytes)
{
    if (bytes <= 256) return 256;
    if (bytes <= (size_t(1) << 20)) {
        size_t c = 512;
        while (c < bytes) c <<= 1;
        return c;
    }
    const size_t g = size_t(2) << 20;
    return (bytes + g - 1) / g * g;
}

// free cached blocks (largest first) until `need` more bytes fit the budget, or all of them
static void drop_cached(bem_ctx *ctx, size_t need)
{
    while (!ctx->free_blocks.empty() && (need == 0 || ctx->in_use + need > ctx->budget)) {
        auto it = std::prev(ctx->free_blocks.end());
        (void)hipFree(it->second);
        ctx->in_use -= it->first;
        ctx->cached_bytes -= it->first;
        ctx->free_blocks.erase(it);
    }
}

void DevMem::release()
{
    if (ptr) {
        if (ctx) {
            std::lock_guard<std::mutex> lk(ctx->mem_mu);
            ctx->free_blocks.emplace(bytes, ptr);
            ctx->cached_bytes += bytes;
            // marks the main-stream work that may still use the block (see dev_alloc)
            if (!ctx->release_ev && hipSetDevice(ctx->device) == hipSuccess)
                (void)hipEventCreateWithFlags(&ctx->release_ev, hipEventDisableTiming);
            if (ctx->release_ev) (void)hipEventRecord(ctx->release_ev, ctx->stream);
        } else {
            (void)hipFree(ptr);
        }
    }
    ptr = nullptr;
    bytes = 0;
}

DevMem::~DevMem() { release(); }

bem_status dev_alloc(bem_ctx *ctx, DevMem &m, size_t bytes, hipStream_t use)
{
    if (m.ptr && m.bytes >= bytes) return BEM_OK;
    m.release();
    const size_t cls = size_class(bytes);
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    // a cached block of this class (or at most a quarter larger)
    auto it = ctx->free_blocks.lower_bound(cls);
    if (it != ctx->free_blocks.end() && it->first <= cls + cls / 4) {
        m.ptr = it->second;
        m.bytes = it->first;
        m.ctx = ctx;
        ctx->cached_bytes -= it->first;
        ctx->free_blocks.erase(it);
        // another stream: wait for the main-stream work queued up to the latest release
        if (use && use != ctx->stream && ctx->release_ev) BEM_HIP(hipStreamWaitEvent(use, ctx->release_ev, 0));
        return BEM_OK;
    }
    if (ctx->budget && ctx->in_use + cls > ctx->budget) drop_cached(ctx, cls);
    if (ctx->budget && ctx->in_use + cls > ctx->budget)
        return set_error(BEM_E_OOM, "context HBM budget exceeded (" + std::to_string(ctx->in_use + cls) + " > " +
                                        std::to_string(ctx->budget) + " bytes)");
    BEM_HIP(hipSetDevice(ctx->device));
    hipError_t e = hipMalloc(&m.ptr, cls);
    if (e == hipErrorOutOfMemory && !ctx->free_blocks.empty()) {   // return the cache to the device and retry
        (void)hipGetLastError();
        drop_cached(ctx, 0);
        e = hipMalloc(&m.ptr, cls);
    }
    if (e != hipSuccess) {
        m.ptr = nullptr;
        return hip_error(e, "hipMalloc");
    }
    m.bytes = cls;
    m.ctx = ctx;
    ctx->in_use += cls;
    return BEM_OK;
}

template <class T, class A>
static bem_status upload(bem_ctx *ctx, DevMem &m, const std::vector<T, A> &v, hipStream_t st = nullptr)
{
    bem_status s = dev_alloc(ctx, m, v.size() * sizeof(T), st);
    if (s) return s;
    if (!v.empty())
        BEM_HIP(hipMemcpyAsync(m.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st ? st : ctx->stream));
    return BEM_OK;
}

// kernels (assemble.hip, solve.hip)
bem_status launch_geometry(const bem_mesh *m, hipStream_t st);
size_t tile_scratch_bytes(const bem_mesh *m, size_t entry_bytes);
bem_status launch_regular(const bem_mesh *m, double k, double kim, bool fp32, void *scratch, void *ops[4], hipStream_t st);
bem_status launch_singular(const bem_mesh *m, double k, double kim, int ng, const double *glx, const double *glw, bool fp32,
                           double2 *contrib, void *ops[4], hipStream_t st);
bem_status launch_mass_inverse(bem_problem *p, int mesh, hipStream_t st);
bem_status launch_sym_corrections(bem_problem *p, int mesh, hipStream_t st);
bem_status ext_form_solve_impl(bem_problem *p, int form, const double *dirs, int nrhs, const bem_solver_opts *opts,
                               void *traces, bem_memspace space, bem_stats *stats);
bem_status ext_form_matvec_impl(bem_problem *p, int form, const void *x, void *y, int strong, bem_memspace space);
bem_status launch_field_region(bem_problem *p, int region, int np, const double *pts, const int32_t *dst_index,
                               const double2 *x_int, const double *dir, double2 *field, DevMem &dens, DevMem &part,
                               hipStream_t st);
bem_status launch_field_permute(bem_problem *p, const double2 *x_caller, double2 *x_int, hipStream_t st);
bem_status launch_winding(const bem_mesh *m, int np, const double *pts, double *w, DevMem &part, hipStream_t st);
bem_status solve_impl(bem_problem *p, const double *dirs, int nrhs, const bem_solver_opts *opts, void *traces,
                      bem_memspace space, bem_stats *stats);
bem_status matvec_impl(bem_problem *p, const void *x, void *y, int strong, bem_memspace space);
bem_status matvec_noalloc_impl(bem_problem *p, const void *x, void *y, int strong);
bem_status noalloc_scratch_init(int device);
bem_status matvec_batch_impl(bem_problem *p, const void *x, void *y, int nrhs, int strong, bem_memspace space);
bem_status rhs_impl(bem_problem *p, const double *dirs, int nrhs, void *b, bem_memspace space);
bem_status permute_matrix_out(const bem_problem *p, int mesh, const void *src, void *dst);

const char *const kKernelNames[K_COUNT] = {"regular_tiles", "gather_tiles", "singular_pairs", "near_scatter",
                                           "mtf_dense", "mass_apply", "cgs_dots", "cgs_update", "arnoldi_finish",
                                           "mass_inverse", "block_gemm", "mass_gemm", "krylov_normalize", "field", "mortar"};

static hipEvent_t take_event(bem_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static thread_local bool t_no_timing = false;
NoTiming::NoTiming() : prev(t_no_timing) { t_no_timing = true; }
NoTiming::~NoTiming() { t_no_timing = prev; }

KTimer::KTimer(bem_ctx *ctx, int kid) : c(ctx), id(kid)
{
    if (!c || t_no_timing || !(c->ktiming >> kid & 1u)) return;
    a = take_event(c);
    b = take_event(c);
    if (!a || !b) {
        if (a) c->pool.push_back(a);
        if (b) c->pool.push_back(b);
        a = b = nullptr;
    }
}

KTimer::~KTimer()
{
    if (!a || !b) return;
    c->pending.push_back({id, a, b});
}

void flush_kernel_timing(bem_ctx *c)
{
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->ktotal_ms[p.id] += ms;
            c->kcount[p.id] += 1;
        }
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
}

// Read the assembly timings once the queued assembly has finished.
bem_status resolve_assembly_timing(bem_problem *p)
{
    if (!p->asm_timing_pending) return BEM_OK;
    BEM_HIP(hipEventSynchronize(p->asm_ev[1][2]));
    float span = 0;
    BEM_HIP(hipEventElapsedTime(&span, p->asm_ev[0][0], p->asm_ev[1][2]));
    double t_reg = 0, t_sing = 0;
    for (int m = 0; m < 2; ++m) {
        float a = 0, b = 0;
        BEM_HIP(hipEventElapsedTime(&a, p->asm_ev[m][0], p->asm_ev[m][1]));
        BEM_HIP(hipEventElapsedTime(&b, p->asm_ev[m][1], p->asm_ev[m][2]));
        t_reg += a;
        t_sing += b;
    }
    p->t_regular_ms = t_reg;
    p->t_singular_ms = t_sing;
    p->t_assembly_ms = span;
    p->asm_timing_pending = false;
    return BEM_OK;
}

static double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// A block solve of R runs with the matrix cores takes the dense inverses as a
// second matrix-core product when the choice is by size, R is at least 32
// and the complex64 inverses take at most 1 GB: there the product of all
// runs costs less than R Chebyshev applies (C4, 64 runs: 0.8 against 1.1 ms
// per step).  Built at the first such solve, beside the sparse tables.
bool block_dense_mass(const bem_problem *p, int R)
{
    const size_t ne = p->ext->h.nv, ni = p->inte->h.nv;
    return p->mass_mode == 0 && p->prec == BEM_C64_MIXED && R >= 32 && std::max(ne, ni) <= 16384 &&
           (ne * ne + ni * ni) * sizeof(float) <= (size_t(1) << 30);
}

}  // namespace bemtx

using namespace bemtx;

extern "C" {

const char *bem_last_error(void) { return g_last_error.c_str(); }

bem_status bem_ctx_create(int32_t device, void *hip_stream, size_t hbm_budget_bytes, bem_ctx **out)
{
    if (!out) return set_error(BEM_E_ARG, "out is NULL");
    int n = 0;
    BEM_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return set_error(BEM_E_ARG, "device index out of range");
    BEM_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    BEM_HIP(hipGetDeviceProperties(&prop, device));
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
        return set_error(BEM_E_UNSUPPORTED, std::string("built for gfx950, device is ") + prop.gcnArchName);
    // the static work array of bem_mtf_matvec_noalloc: its address on this device
    const bem_status ss = noalloc_scratch_init(device);
    if (ss) return ss;
    bem_ctx *c = new bem_ctx;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->budget = hbm_budget_bytes;
    *out = c;
    return BEM_OK;
}

void bem_ctx_destroy(bem_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->gather) {
        (void)hipStreamSynchronize(ctx->gather);
        (void)hipStreamDestroy(ctx->gather);
    }
    for (hipEvent_t e : ctx->strip_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    if (ctx->release_ev) (void)hipEventDestroy(ctx->release_ev);
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    {
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        drop_cached(ctx, 0);
    }
    delete ctx;
}

bem_status bem_ctx_trim(bem_ctx *ctx)
{
    if (!ctx) return set_error(BEM_E_ARG, "null context");
    BEM_HIP(hipSetDevice(ctx->device));
    BEM_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->scratch) {
        BEM_HIP(hipFree(ctx->scratch));
        ctx->in_use -= ctx->scratch_bytes;
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    drop_cached(ctx, 0);
    return BEM_OK;
}

bem_status bem_ctx_set_strip_tiles(bem_ctx *ctx, int64_t tiles)
{
    if (!ctx) return set_error(BEM_E_ARG, "null context");
    if (tiles < 0) return set_error(BEM_E_ARG, "strip tiles must be >= 0");
    ctx->strip_tiles = tiles == 0 ? ASM_STRIP_TILES : tiles;
    return BEM_OK;
}

bem_status bem_ctx_set_kernel_timing(bem_ctx *ctx, uint32_t kernel_mask)
{
    if (!ctx) return set_error(BEM_E_ARG, "null context");
    BEM_HIP(hipStreamSynchronize(ctx->stream));
    flush_kernel_timing(ctx);
    ctx->ktiming = kernel_mask & ((1u << K_COUNT) - 1u);
    for (int k = 0; k < K_COUNT; ++k) { ctx->ktotal_ms[k] = 0.0; ctx->kcount[k] = 0; }
    return BEM_OK;
}

bem_status bem_ctx_kernel_time(bem_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches)
{
    if (!ctx || !kernel || !total_ms || !launches) return set_error(BEM_E_ARG, "null argument");
    BEM_HIP(hipStreamSynchronize(ctx->stream));
    flush_kernel_timing(ctx);
    for (int k = 0; k < K_COUNT; ++k)
        if (std::strcmp(kernel, kKernelNames[k]) == 0) {
            *total_ms = ctx->ktotal_ms[k];
            *launches = ctx->kcount[k];
            return BEM_OK;
        }
    return set_error(BEM_E_ARG, std::string("unknown kernel name ") + kernel);
}

size_t bem_ctx_bytes_in_use(const bem_ctx *ctx) { return ctx ? ctx->in_use : 0; }

bem_status bem_mesh_create(bem_ctx *ctx, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt,
                           bem_mesh **out)
{
    if (!ctx || !xyz || !tri || !out) return set_error(BEM_E_ARG, "null argument");
    if (nv <= 0 || nt <= 0) return set_error(BEM_E_ARG, "empty mesh");
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) return set_error(BEM_E_MESH, "non-finite vertex coordinate");
    bem_mesh *m = new bem_mesh;
    m->ctx = ctx;
    m->h.nv = nv;
    m->h.nt = nt;
    m->h.xyz_user.assign(xyz, xyz + 3 * nv);
    m->h.tri_user.assign(tri, tri + 3 * nt);
    bem_status s = mesh_prepare(m->h, ctx->strip_tiles);
    if (s == BEM_OK) s = upload(ctx, m->d.perm, m->h.int_of_v);
    if (s == BEM_OK) s = upload(ctx, m->d.xyz, m->h.xyz);
    if (s == BEM_OK) s = upload(ctx, m->d.tri, m->h.tri);
    if (s == BEM_OK) s = upload(ctx, m->d.blk_start, m->h.blk_start);
    if (s == BEM_OK) s = upload(ctx, m->d.blk_nslot, m->h.blk_nslot);
    if (s == BEM_OK) s = upload(ctx, m->d.slot_off, m->h.slot_off);
    if (s == BEM_OK) s = upload(ctx, m->d.slot_rank, m->h.slot_rank);
    if (s == BEM_OK) s = upload(ctx, m->d.memb_ptr, m->h.memb_ptr);
    if (s == BEM_OK) s = upload(ctx, m->d.memb, m->h.memb);
    if (s == BEM_OK) s = upload(ctx, m->d.strip_rows, m->h.strip_rows);
    if (s == BEM_OK) s = upload(ctx, m->d.sing, m->h.sing);
    if (s == BEM_OK) s = upload(ctx, m->d.near_i, m->h.near_i);
    if (s == BEM_OK) s = upload(ctx, m->d.near_j, m->h.near_j);
    if (s == BEM_OK) s = upload(ctx, m->d.near_ptr, m->h.near_ptr);
    if (s == BEM_OK) s = upload(ctx, m->d.near_src, m->h.near_src);
    if (s == BEM_OK) s = upload(ctx, m->d.near_row, m->h.near_row);
    if (s == BEM_OK) s = upload(ctx, m->d.star_ptr, m->h.star_ptr);
    if (s == BEM_OK) s = upload(ctx, m->d.star_ent, m->h.star_ent);
    if (s == BEM_OK) s = dev_alloc(ctx, m->d.geo, (size_t)nt * sizeof(TriGeo));
    if (s == BEM_OK) s = dev_alloc(ctx, m->d.geof, (size_t)nt * sizeof(TriGeoF));
    if (s == BEM_OK) s = launch_geometry(m, ctx->stream);
    if (s == BEM_OK) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) s = hip_error(e, "hipStreamSynchronize");
    }
    if (s != BEM_OK) {
        delete m;
        return s;
    }
    *out = m;
    return BEM_OK;
}

void bem_mesh_destroy(bem_mesh *mesh) { delete mesh; }

int64_t bem_mesh_num_vertices(const bem_mesh *mesh) { return mesh ? mesh->h.nv : 0; }

bem_status bem_problem_create(bem_ctx *ctx, const bem_mesh *ext, const bem_mesh *inte, double k_ext, double k_int,
                              double rho_ext, double rho_int, bem_precision precision, const bem_quad_opts *quad,
                              bem_problem **out)
{
    if (!ctx || !ext || !inte || !out) return set_error(BEM_E_ARG, "null argument");
    if (ext->ctx != ctx || inte->ctx != ctx) return set_error(BEM_E_ARG, "meshes belong to another context");
    if (!(k_ext > 0) || !(k_int > 0) || !(rho_ext > 0) || !(rho_int > 0) || !std::isfinite(k_ext) ||
        !std::isfinite(k_int) || !std::isfinite(rho_ext) || !std::isfinite(rho_int))
        return set_error(BEM_E_ARG, "wavenumbers and densities must be positive and finite");
    if (precision != BEM_C128 && precision != BEM_C64_MIXED) return set_error(BEM_E_ARG, "unknown precision");
    for (int m = 0; m < 2; ++m) {
        const bemtx::MeshData &h = m == 0 ? ext->h : inte->h;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < h.nv; ++v)
            for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], h.xyz[3 * v + c]); hi[c] = std::max(hi[c], h.xyz[3 * v + c]); }
        const double diam = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                      (hi[2] - lo[2]) * (hi[2] - lo[2]));
        const double k = m == 0 ? k_ext : k_int;
        if (!(k * diam < 0.5 * kPhaseMax))
            return set_error(BEM_E_UNSUPPORTED, "k * diameter too large for the FP64 phase reduction (>= 5e4)");
    }
    int ng = quad ? quad->singular_gauss : 4;
    if (ng < 1 || ng > NG_MAX) return set_error(BEM_E_ARG, "singular_gauss must be in 1..16");
    bem_problem *p = new bem_problem;
    p->ctx = ctx;
    p->ext = ext;
    p->inte = inte;
    p->k_ext = k_ext;
    p->k_int = k_int;
    p->rho_ext = rho_ext;
    p->rho_int = rho_int;
    p->prec = precision;
    p->ng = ng;
    gauss_legendre01(ng, p->gl_x, p->gl_w);
    *out = p;
    return BEM_OK;
}

void bem_problem_destroy(bem_problem *p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->ctx->stream);
    if (p->ctx->aux) (void)hipStreamSynchronize(p->ctx->aux);
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 3; ++q)
            if (p->asm_ev[m][q]) (void)hipEventDestroy(p->asm_ev[m][q]);
    if (p->ev_pre_asm) (void)hipEventDestroy(p->ev_pre_asm);
    if (p->ev_proj) (void)hipEventDestroy(p->ev_proj);
    delete p;
}

// Dense inverse masses stream (N_e^2 + N_i^2) entries per apply; above this
// many bytes the sparse Chebyshev apply (three or two launches on the
// patches, tens of microseconds together) is the faster one, and above
// 16,384 vertices on a mesh the dense inverse is not built at all.
constexpr size_t kMassDenseMaxBytes = size_t(256) << 20;

static bool pick_mass_sparse(const bem_problem *p)
{
    const size_t ne = p->ext->h.nv, ni = p->inte->h.nv;
    if (p->mass_mode == 2) return true;
    if (p->mass_mode == 1) return false;
    if (std::max(ne, ni) > 16384) return true;
    return (ne * ne + ni * ni) * (p->prec == BEM_C128 ? sizeof(double) : sizeof(float)) > kMassDenseMaxBytes;
}

bem_status bem_problem_set_mass_apply(bem_problem *p, int32_t mode)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    if (mode < 0 || mode > 2) return set_error(BEM_E_ARG, "mass apply mode must be 0 (by size), 1 (dense) or 2 (sparse)");
    if (mode != p->mass_mode) p->proj_ready = false;   // takes effect at the next projection set-up
    p->mass_mode = mode;
    return BEM_OK;
}

bem_status bem_problem_set_graphs(bem_problem *p, int32_t on)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    if (on != 0 && on != 1) return set_error(BEM_E_ARG, "graphs must be 0 (off) or 1 (on)");
    p->graphs = on;
    return BEM_OK;
}

bem_status bem_problem_mass_apply(const bem_problem *p, int32_t *sparse)
{
    if (!p || !sparse) return set_error(BEM_E_ARG, "null argument");
    if (!p->proj_ready) return set_error(BEM_E_STATE, "assemble the projection first");
    *sparse = p->mass_sparse ? 1 : 0;
    return BEM_OK;
}

bem_status bem_problem_footprint(const bem_problem *p, int32_t nrhs, int32_t maxit, size_t *bytes)
{
    if (!p || !bytes || nrhs < 1 || maxit < 1) return set_error(BEM_E_ARG, "bad argument");
    const size_t ne = p->ext->h.nv, ni = p->inte->h.nv, n = 2 * ne + 2 * ni;
    const size_t eb = p->prec == BEM_C128 ? sizeof(double2) : sizeof(float2);
    size_t b = 4 * (ne * op_ld(ne) + ni * op_ld(ni)) * eb;         // dense operators
    const bool sparse_mass = pick_mass_sparse(p);
    if (sparse_mass)   // patch tables: at most 8 patch copies of each vertex with its row (bound)
        b += 8 * (ne + ni) * (3 * sizeof(int32_t) + sizeof(double) + 14 * (sizeof(int32_t) + sizeof(double)));
    if (!sparse_mass || block_dense_mass(p, p->prec == BEM_C64_MIXED ? std::min(nrhs, 64) : 1))
        b += (ne * ne + ni * ni) * (p->prec == BEM_C128 ? sizeof(double) : sizeof(float));   // dense inverse masses
    size_t scratch = std::max(tile_scratch_bytes(p->ext, eb), tile_scratch_bytes(p->inte, eb));
    scratch = std::max(scratch, std::max(p->ext->h.sing.size(), p->inte->h.sing.size()) * 36 * sizeof(double2));
    b += scratch;
    // runs that advance together: every right-hand side of a complex64 problem (up to 64 per block), else one
    const size_t R = p->prec == BEM_C64_MIXED ? (size_t)std::min(nrhs, 64) : 1;
    b += R * ((size_t)(maxit + 1) * n + 8 * n) * sizeof(double2);                 // Krylov bases + work vectors
    b += 2 * R * (size_t)maxit * (maxit + 1) * sizeof(double2);                   // Hessenberg matrices, triangular factors
    b += R * ((n + 1023) / 1024) * 2 * (size_t)(maxit + 1) * sizeof(double2);     // Gram-Schmidt partial dot products
    if (R > 1) {   // right-hand matrices and K-chunk partials of the matrix-core products
        const size_t kop = 2 * (op_ld(ne) + op_ld(ni)), km = ((ne + 31) & ~size_t(31)) + ((ni + 31) & ~size_t(31));
        b += (2 * 128 * kop + 256 * km) * sizeof(float);
        b += (8 * 128 * 4 + 8 * 256) * (ne + ni) * sizeof(float);
        if (sparse_mass) b += 6 * 64 * n * sizeof(double2);   // Chebyshev work sets of the block apply
    }
    b += 64 * (ne + ni) * sizeof(double);                          // sparse couplings (bound)
    *bytes = b;
    return BEM_OK;
}

bem_status bem_assemble_operators(bem_problem *p, int32_t parts)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    if (parts < 0 || parts > 3) return set_error(BEM_E_ARG, "parts must be 0..3");
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // the projection set-up on the auxiliary stream may start once the work queued before this point is done
    if (!p->ev_pre_asm) BEM_HIP(hipEventCreateWithFlags(&p->ev_pre_asm, hipEventDisableTiming));
    BEM_HIP(hipEventRecord(p->ev_pre_asm, st));
    const bem_mesh *meshes[2] = {p->ext, p->inte};
    const double ks[2] = {p->k_ext, p->k_int};
    const double kims[2] = {0.0, p->k_int_im};
    const bool fp32 = p->prec == BEM_C64_MIXED;
    const size_t eb = fp32 ? sizeof(float2) : sizeof(double2);
    size_t scratch_bytes = 16;
    for (int m = 0; m < 2; ++m) {
        scratch_bytes = std::max(scratch_bytes, tile_scratch_bytes(meshes[m], eb));
        scratch_bytes = std::max(scratch_bytes, meshes[m]->h.sing.size() * 36 * sizeof(double2));
    }
    for (int m = 0; m < 2; ++m) {
        const size_t nv = meshes[m]->h.nv;
        for (int op = 0; op < 4; ++op) {
            bem_status s = dev_alloc(ctx, p->ops[m][op], nv * op_ld(nv) * eb);
            if (s) return s;
        }
    }
    if (ctx->scratch_bytes < scratch_bytes) {
        if (ctx->scratch) {
            BEM_HIP(hipStreamSynchronize(st));
            (void)hipFree(ctx->scratch);
            ctx->in_use -= ctx->scratch_bytes;
            ctx->scratch = nullptr;
            ctx->scratch_bytes = 0;
        }
        std::lock_guard<std::mutex> lk(ctx->mem_mu);
        if (ctx->budget && ctx->in_use + scratch_bytes > ctx->budget) drop_cached(ctx, scratch_bytes);
        if (ctx->budget && ctx->in_use + scratch_bytes > ctx->budget)
            return set_error(BEM_E_OOM, "context HBM budget exceeded by the assembly scratch");
        hipError_t e = hipMalloc(&ctx->scratch, scratch_bytes);
        if (e == hipErrorOutOfMemory && !ctx->free_blocks.empty()) {
            (void)hipGetLastError();
            drop_cached(ctx, 0);
            e = hipMalloc(&ctx->scratch, scratch_bytes);
        }
        if (e != hipSuccess) { ctx->scratch = nullptr; return hip_error(e, "hipMalloc(scratch)"); }
        ctx->scratch_bytes = scratch_bytes;
        ctx->in_use += scratch_bytes;
    }
    void *scratch = ctx->scratch;
    // events: [mesh][0] before regular, [1] before singular, [2] after; resolved lazily
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 3; ++q)
            if (!p->asm_ev[m][q]) BEM_HIP(hipEventCreate(&p->asm_ev[m][q]));
    for (int m = 0; m < 2; ++m) {
        void *ops[4];
        for (int op = 0; op < 4; ++op) ops[op] = p->ops[m][op].ptr;
        const size_t nv = meshes[m]->h.nv;
        BEM_HIP(hipEventRecord(p->asm_ev[m][0], st));
        if (parts & 1) {
            bem_status s = launch_regular(meshes[m], ks[m], kims[m], fp32, scratch, ops, st);
            if (s) return s;
        } else {
            for (int op = 0; op < 4; ++op) BEM_HIP(hipMemsetAsync(ops[op], 0, nv * op_ld(nv) * eb, st));
        }
        BEM_HIP(hipEventRecord(p->asm_ev[m][1], st));
        if (parts & 2) {
            bem_status s = launch_singular(meshes[m], ks[m], kims[m], p->ng, p->gl_x, p->gl_w, fp32,
                                           static_cast<double2 *>(scratch), ops, st);
            if (s) return s;
        }
        BEM_HIP(hipEventRecord(p->asm_ev[m][2], st));
        bem_status s = launch_sym_corrections(p, m, st);
        if (s) return s;
    }
    p->asm_timing_pending = true;
    p->ops_ready = true;
    return BEM_OK;
}


bem_status bem_assemble_projection(bem_problem *p)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    auto t0 = std::chrono::steady_clock::now();
    mass_csr(p->ext->h, p->M[0]);
    mass_csr(p->inte->h, p->M[1]);
    // uploads and inverse masses on the auxiliary stream, after the work queued
    // on the main stream before the operator assembly (or before this call),
    // so that they overlap the assembly; the inverse masses are queued before
    // the host builds the mortar projection, which then overlaps them too; the
    // main stream waits for all of it
    if (!ctx->aux) BEM_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    hipStream_t ax = ctx->aux;
    if (!p->ev_pre_asm) {
        BEM_HIP(hipEventCreateWithFlags(&p->ev_pre_asm, hipEventDisableTiming));
        BEM_HIP(hipEventRecord(p->ev_pre_asm, ctx->stream));
    }
    if (!p->ev_proj) BEM_HIP(hipEventCreateWithFlags(&p->ev_proj, hipEventDisableTiming));
    BEM_HIP(hipStreamWaitEvent(ax, p->ev_pre_asm, 0));
    if (p->proj_ready) {
        // a second set-up rewrites this problem's tables in place: first let the main-stream work that may
        // read them (an asynchronous product) finish
        BEM_HIP(hipEventRecord(p->ev_proj, ctx->stream));
        BEM_HIP(hipStreamWaitEvent(ax, p->ev_proj, 0));
    }
    p->proj_ready = false;
    bem_status s = BEM_OK;
    double defect = 0;
    if (p->mortar_dev) {   // geometry on the device, on the auxiliary stream before the inverse masses
        const auto tm = std::chrono::steady_clock::now();
        s = mortar_csr_device(ctx, p->inte, p->ext, ax, p->P_ie, &defect);
        if (s) return s;
        p->t_mortar_ms = ms_since(tm);
    }
    for (int m = 0; m < 2 && !s; ++m) {
        s = upload(ctx, p->M_ptr[m], p->M[m].ptr, ax);
        if (!s) s = upload(ctx, p->M_col[m], p->M[m].col, ax);
        if (!s) s = upload(ctx, p->M_val[m], p->M[m].val, ax);
    }
    if (s) return s;
    p->mass_sparse = pick_mass_sparse(p);
    p->mass_dense = !p->mass_sparse;
    if (p->mass_sparse) {   // patch tables of the sparse apply (host), no dense inverse
        for (int m = 0; m < 2; ++m) p->Minv[m].release();
        s = cheb_tables(p->M, CHEB_S, p->cheb);
        if (!s) s = upload(ctx, p->cheb_pmesh, p->cheb.pmesh, ax);
        if (!s) s = upload(ctx, p->cheb_vbeg, p->cheb.vbeg, ax);
        if (!s) s = upload(ctx, p->cheb_cnt, p->cheb.cnt, ax);
        if (!s) s = upload(ctx, p->cheb_vert, p->cheb.vert, ax);
        if (!s) s = upload(ctx, p->cheb_dinv, p->cheb.dinv, ax);
        if (!s) s = upload(ctx, p->cheb_ecol, p->cheb.ecol, ax);
        if (!s) s = upload(ctx, p->cheb_eval, p->cheb.eval, ax);
    } else {
        for (int m = 0; m < 2 && !s; ++m) s = launch_mass_inverse(p, m, ax);
    }
    if (s) return s;
    if (!p->mortar_dev) {
        const auto tm = std::chrono::steady_clock::now();
        s = mortar_csr(p->inte->h, p->ext->h, p->P_ie, &defect);
        if (s) return s;
        p->t_mortar_ms = ms_since(tm);
    }
    transpose_csr(p->P_ie, p->P_ei);
    s = upload(ctx, p->P_ie_ptr, p->P_ie.ptr, ax);
    if (!s) s = upload(ctx, p->P_ie_col, p->P_ie.col, ax);
    if (!s) s = upload(ctx, p->P_ie_val, p->P_ie.val, ax);
    if (!s) s = upload(ctx, p->P_ei_ptr, p->P_ei.ptr, ax);
    if (!s) s = upload(ctx, p->P_ei_col, p->P_ei.col, ax);
    if (!s) s = upload(ctx, p->P_ei_val, p->P_ei.val, ax);
    if (s) return s;
    BEM_HIP(hipEventRecord(p->ev_proj, ax));
    BEM_HIP(hipStreamWaitEvent(ctx->stream, p->ev_proj, 0));
    BEM_HIP(hipStreamSynchronize(ax));
    p->t_projection_ms = ms_since(t0);
    p->proj_ready = true;
    return BEM_OK;
}

bem_status bem_mtf_matvec(bem_problem *p, const void *x, void *y, int32_t strong, bem_memspace space)
{
    if (!p || !x || !y) return set_error(BEM_E_ARG, "null argument");
    if (!p->ops_ready || !p->proj_ready) return set_error(BEM_E_STATE, "assemble operators and projection first");
    return matvec_impl(p, x, y, strong, space);
}

bem_status bem_tune_table(char *buf, size_t cap, size_t *len)
{
    if (!len) return set_error(BEM_E_ARG, "len is NULL");
    const std::string t = tune_table_text();
    *len = t.size();
    if (buf && cap > 0) {
        const size_t n = std::min(cap - 1, t.size());
        std::memcpy(buf, t.data(), n);
        buf[n] = '\0';
    }
    return BEM_OK;
}

bem_status bem_mtf_matvec_noalloc(bem_problem *p, const void *x, void *y, int32_t strong)
{
    if (!p || !x || !y) return set_error(BEM_E_ARG, "null argument");
    return matvec_noalloc_impl(p, x, y, strong);   // size check first, then the assembly state
}

bem_status bem_mtf_matvec_batch(bem_problem *p, const void *x, void *y, int32_t nrhs, int32_t strong,
                                bem_memspace space)
{
    if (!p || !x || !y || nrhs < 1) return set_error(BEM_E_ARG, "bad argument");
    if (!p->ops_ready || !p->proj_ready) return set_error(BEM_E_STATE, "assemble operators and projection first");
    return matvec_batch_impl(p, x, y, nrhs, strong, space);
}

// the incident fields of a call: unit directions (plane waves) or finite
// positions (point sources), by the problem's setting
static bem_status check_sources(const bem_problem *p, const double *dirs, int32_t nrhs)
{
    for (int r = 0; r < nrhs; ++r) {
        const double *d = dirs + 3 * r;
        if (p->incident == 1) {
            if (!(std::isfinite(d[0]) && std::isfinite(d[1]) && std::isfinite(d[2])))
                return set_error(BEM_E_ARG, "point-source positions must be finite");
        } else {
            const double l = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(std::fabs(l - 1.0) < 1e-6)) return set_error(BEM_E_ARG, "directions must be unit vectors");
        }
    }
    return BEM_OK;
}

bem_status bem_problem_set_incident(bem_problem *p, int32_t kind)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    if (kind != 0 && kind != 1) return set_error(BEM_E_ARG, "incident kind must be 0 (plane waves) or 1 (point sources)");
    p->incident = kind;
    return BEM_OK;
}

bem_status bem_problem_set_mortar(bem_problem *p, int32_t on_device)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    if (on_device != 0 && on_device != 1) return set_error(BEM_E_ARG, "on_device must be 0 or 1");
    p->mortar_dev = on_device;
    return BEM_OK;
}

bem_status bem_problem_mortar_ms(const bem_problem *p, double *ms)
{
    if (!p || !ms) return set_error(BEM_E_ARG, "null argument");
    if (!p->proj_ready) return set_error(BEM_E_STATE, "assemble the projection first");
    *ms = p->t_mortar_ms;
    return BEM_OK;
}

bem_status bem_problem_set_k_int_imag(bem_problem *p, double k_int_imag)
{
    if (!p) return set_error(BEM_E_ARG, "null problem");
    if (!(k_int_imag >= 0) || !std::isfinite(k_int_imag))
        return set_error(BEM_E_ARG, "the imaginary part of the interior wavenumber must be finite and >= 0");
    if (k_int_imag != p->k_int_im) p->ops_ready = false;   // assembled operators belong to the old wavenumber
    p->k_int_im = k_int_imag;
    return BEM_OK;
}

bem_status bem_mtf_rhs(bem_problem *p, const double *dirs, int32_t nrhs, void *b, bem_memspace space)
{
    if (!p || !dirs || !b || nrhs < 1) return set_error(BEM_E_ARG, "bad argument");
    bem_status s = check_sources(p, dirs, nrhs);
    return s ? s : rhs_impl(p, dirs, nrhs, b, space);
}

bem_status bem_solve(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts, void *traces,
                     bem_memspace space, bem_stats *stats)
{
    if (!p || !dirs || !opts || !traces || nrhs < 1) return set_error(BEM_E_ARG, "bad argument");
    if (!(opts->tol > 0) || opts->maxit < 1 || opts->maxit > 3000)
        return set_error(BEM_E_ARG, "tol must be > 0 and 1 <= maxit <= 3000");
    if (opts->batch < 0 || opts->batch > 64) return set_error(BEM_E_ARG, "batch must be 0..64");
    if (!p->ops_ready || !p->proj_ready) return set_error(BEM_E_STATE, "assemble operators and projection first");
    bem_status s = check_sources(p, dirs, nrhs);
    return s ? s : solve_impl(p, dirs, nrhs, opts, traces, space, stats);
}

bem_status bem_copy_operator(const bem_problem *p, int32_t mesh, char op, void *dst, bem_memspace space)
{
    if (!p || !dst) return set_error(BEM_E_ARG, "null argument");
    if (mesh != 0 && mesh != 1) return set_error(BEM_E_ARG, "mesh must be 0 (exterior) or 1 (interior)");
    const char *names = "VKTD";
    const char *f = std::strchr(names, op);
    if (!f || op == 0) return set_error(BEM_E_ARG, "op must be one of V, K, T, D");
    if (!p->ops_ready) return set_error(BEM_E_STATE, "operators not assembled");
    const int o = (int)(f - names);
    const bem_mesh *m = mesh == 0 ? p->ext : p->inte;
    const size_t eb = p->prec == BEM_C128 ? sizeof(double2) : sizeof(float2);
    const size_t nv = m->h.nv, bytes = nv * nv * eb;
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    if (space == BEM_DEVICE) {
        bem_status s = permute_matrix_out(p, mesh, p->ops[mesh][o].ptr, dst);
        if (s) return s;
        BEM_HIP(hipStreamSynchronize(ctx->stream));
        return BEM_OK;
    }
    DevMem tmp;
    bem_status s = dev_alloc(ctx, tmp, bytes);
    if (s) return s;
    s = permute_matrix_out(p, mesh, p->ops[mesh][o].ptr, tmp.ptr);
    if (s) return s;
    BEM_HIP(hipMemcpyAsync(dst, tmp.ptr, bytes, hipMemcpyDeviceToHost, ctx->stream));
    BEM_HIP(hipStreamSynchronize(ctx->stream));
    return BEM_OK;
}

bem_status bem_copy_projection(const bem_problem *p, int64_t *rowptr, int32_t *col, double *val, int64_t *nnz)
{
    if (!p || !nnz) return set_error(BEM_E_ARG, "null argument");
    if (!p->proj_ready) return set_error(BEM_E_STATE, "projection not assembled");
    const MeshData &mi = p->inte->h, &me = p->ext->h;
    const Csr &P = p->P_ie;
    *nnz = (int64_t)P.col.size();
    if (!rowptr) return BEM_OK;
    if (!col || !val) return set_error(BEM_E_ARG, "col and val are required with rowptr");
    // caller numbering: row i_user = v_of_int[i_int], columns mapped and sorted
    int64_t q = 0;
    rowptr[0] = 0;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t iu = 0; iu < mi.nv; ++iu) {
        const int32_t ii = mi.int_of_v[iu];
        row.clear();
        for (int32_t k = P.ptr[ii]; k < P.ptr[ii + 1]; ++k) row.push_back({me.v_of_int[P.col[k]], P.val[k]});
        std::sort(row.begin(), row.end());
        for (auto &e : row) {
            col[q] = e.first;
            val[q] = e.second;
            ++q;
        }
        rowptr[iu + 1] = q;
    }
    return BEM_OK;
}

bem_status bem_check_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt)
{
    if (!xyz || !tri || nv <= 0 || nt <= 0) return set_error(BEM_E_ARG, "bad argument");
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) return set_error(BEM_E_MESH, "non-finite vertex coordinate");
    MeshData m;
    m.nv = nv;
    m.nt = nt;
    m.xyz_user.assign(xyz, xyz + 3 * nv);
    m.tri_user.assign(tri, tri + 3 * nt);
    return mesh_prepare(m);
}

bem_status bem_host_mortar(const double *xyz_int, int64_t nv_int, const int32_t *tri_int, int64_t nt_int,
                           const double *xyz_ext, int64_t nv_ext, const int32_t *tri_ext, int64_t nt_ext,
                           int64_t *rowptr, int32_t *col, double *val, int64_t *nnz, double *coverage_defect)
{
    if (!nnz) return set_error(BEM_E_ARG, "nnz is NULL");
    MeshData mi, me;
    mi.nv = nv_int; mi.nt = nt_int; me.nv = nv_ext; me.nt = nt_ext;
    if (!xyz_int || !tri_int || !xyz_ext || !tri_ext) return set_error(BEM_E_ARG, "null mesh array");
    mi.xyz_user.assign(xyz_int, xyz_int + 3 * nv_int);
    mi.tri_user.assign(tri_int, tri_int + 3 * nt_int);
    me.xyz_user.assign(xyz_ext, xyz_ext + 3 * nv_ext);
    me.tri_user.assign(tri_ext, tri_ext + 3 * nt_ext);
    bem_status s = mesh_prepare(mi);
    if (!s) s = mesh_prepare(me);
    if (s) return s;
    Csr P;
    double defect = 0;
    s = mortar_csr(mi, me, P, &defect);
    if (coverage_defect) *coverage_defect = defect;
    if (s) return s;
    const int64_t total = (int64_t)P.col.size();
    if (!rowptr) {
        *nnz = total;
        return BEM_OK;
    }
    if (!col || !val || *nnz < total) return set_error(BEM_E_ARG, "output arrays missing or too small");
    int64_t q = 0;
    rowptr[0] = 0;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t iu = 0; iu < nv_int; ++iu) {
        const int32_t ii = mi.int_of_v[iu];
        row.clear();
        for (int32_t k = P.ptr[ii]; k < P.ptr[ii + 1]; ++k) row.push_back({me.v_of_int[P.col[k]], P.val[k]});
        std::sort(row.begin(), row.end());
        for (auto &e : row) { col[q] = e.first; val[q] = e.second; ++q; }
        rowptr[iu + 1] = q;
    }
    *nnz = total;
    return BEM_OK;
}

bem_status bem_host_phase_sincos(int64_t n, const double *x, double *s, double *c)
{
    if (n < 0 || (n > 0 && (!x || !s || !c))) return set_error(BEM_E_ARG, "bad argument");
    for (int64_t i = 0; i < n; ++i) phase_sincos(x[i], s + i, c + i);
    return BEM_OK;
}

bem_status bem_host_gauss_legendre(int32_t n, double *x, double *w)
{
    if (n < 1 || n > NG_MAX || !x || !w) return set_error(BEM_E_ARG, "n must be in 1..16");
    gauss_legendre01(n, x, w);
    return BEM_OK;
}


bem_status bem_field(bem_problem *p, const double *dirs, int32_t nrhs, const void *traces, const double *points,
                     const int32_t *region, int64_t npts, void *field, bem_memspace space)
{
    if (!p || !dirs || !traces || nrhs < 1 || npts < 0) return set_error(BEM_E_ARG, "bad argument");
    if (npts > 0 && (!points || !region || !field)) return set_error(BEM_E_ARG, "null points, region or field");
    if (npts > (int64_t)1 << 28) return set_error(BEM_E_ARG, "at most 2^28 points per call");
    if (space != BEM_HOST && space != BEM_DEVICE) return set_error(BEM_E_ARG, "bad memory space");
    {
        bem_status sc = check_sources(p, dirs, nrhs);
        if (sc) return sc;
    }
    if (npts == 0) return BEM_OK;
    bem_ctx *ctx = p->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int np = (int)npts;
    // points and regions on the host, to sort the points by region
    std::vector<double> hp;
    std::vector<int32_t> hr;
    const double *P = points;
    const int32_t *Rg = region;
    if (space == BEM_DEVICE) {
        hp.resize((size_t)3 * np);
        hr.resize(np);
        BEM_HIP(hipMemcpyAsync(hp.data(), points, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        BEM_HIP(hipMemcpyAsync(hr.data(), region, hr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        BEM_HIP(hipStreamSynchronize(st));
        P = hp.data();
        Rg = hr.data();
    }
    std::vector<int32_t> order;
    order.reserve(np);
    int cnt[2] = {0, 0};
    for (int m = 0; m < 2; ++m)
        for (int i = 0; i < np; ++i) {
            if (Rg[i] != 0 && Rg[i] != 1) return set_error(BEM_E_ARG, "region must be 0 (exterior) or 1 (interior)");
            if (Rg[i] == m) { order.push_back(i); ++cnt[m]; }
        }
    std::vector<double> sp((size_t)3 * np);
    for (int o = 0; o < np; ++o)
        for (int c = 0; c < 3; ++c) sp[(size_t)3 * o + c] = P[(size_t)3 * order[o] + c];
    const int ne = (int)p->ext->h.nv, ni = (int)p->inte->h.nv, n = 2 * ne + 2 * ni;
    DevMem dpts, didx, xin, xint, fout, dens, part;
    bem_status s = upload(ctx, dpts, sp);
    if (!s) s = upload(ctx, didx, order);
    if (!s) s = dev_alloc(ctx, xint, (size_t)n * sizeof(double2));
    if (s) return s;
    const double2 *X = static_cast<const double2 *>(traces);
    if (space == BEM_HOST) {
        s = dev_alloc(ctx, xin, (size_t)nrhs * n * sizeof(double2));
        if (!s) s = dev_alloc(ctx, fout, (size_t)nrhs * np * sizeof(double2));
        if (s) return s;
        BEM_HIP(hipMemcpyAsync(xin.ptr, traces, (size_t)nrhs * n * sizeof(double2), hipMemcpyHostToDevice, st));
        X = xin.as<double2>();
    }
    double2 *Fo = space == BEM_HOST ? fout.as<double2>() : static_cast<double2 *>(field);
    for (int r = 0; r < nrhs; ++r) {
        s = launch_field_permute(p, X + (size_t)r * n, xint.as<double2>(), st);
        for (int m = 0, off = 0; m < 2 && !s; off += cnt[m], ++m)
            s = launch_field_region(p, m, cnt[m], dpts.as<double>() + (size_t)3 * off, didx.as<int32_t>() + off,
                                    xint.as<double2>(), dirs + 3 * r, Fo + (size_t)r * np, dens, part, st);
        if (s) return s;
    }
    if (space == BEM_HOST)
        BEM_HIP(hipMemcpyAsync(field, Fo, (size_t)nrhs * np * sizeof(double2), hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    return BEM_OK;
}

bem_status bem_mesh_winding(const bem_mesh *m, const double *points, int64_t npts, double *w, bem_memspace space)
{
    if (!m || npts < 0 || (npts > 0 && (!points || !w))) return set_error(BEM_E_ARG, "bad argument");
    if (npts > (int64_t)1 << 28) return set_error(BEM_E_ARG, "at most 2^28 points per call");
    if (space != BEM_HOST && space != BEM_DEVICE) return set_error(BEM_E_ARG, "bad memory space");
    if (npts == 0) return BEM_OK;
    bem_ctx *ctx = m->ctx;
    BEM_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int np = (int)npts;
    DevMem dpts, dw, part;
    const double *Pd = points;
    double *Wd = w;
    if (space == BEM_HOST) {
        bem_status s = dev_alloc(ctx, dpts, (size_t)3 * np * sizeof(double));
        if (!s) s = dev_alloc(ctx, dw, (size_t)np * sizeof(double));
        if (s) return s;
        BEM_HIP(hipMemcpyAsync(dpts.ptr, points, (size_t)3 * np * sizeof(double), hipMemcpyHostToDevice, st));
        Pd = dpts.as<double>();
        Wd = dw.as<double>();
    }
    bem_status s = launch_winding(m, np, Pd, Wd, part, st);
    if (s) return s;
    if (space == BEM_HOST) BEM_HIP(hipMemcpyAsync(w, Wd, (size_t)np * sizeof(double), hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    return BEM_OK;
}


static bem_status ext_form_check(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts,
                                 void *traces, bem_memspace space)
{
    if (!p || !dirs || !opts || !traces || nrhs < 1) return set_error(BEM_E_ARG, "bad argument");
    if (!(opts->tol > 0) || opts->maxit < 1 || opts->maxit > 3000)
        return set_error(BEM_E_ARG, "tol must be > 0 and 1 <= maxit <= 3000");
    if (space != BEM_HOST && space != BEM_DEVICE) return set_error(BEM_E_ARG, "bad memory space");
    if (!p->ops_ready || !p->proj_ready) return set_error(BEM_E_STATE, "assemble operators and projection first");
    {
        bem_status sc = check_sources(p, dirs, nrhs);
        if (sc) return sc;
    }
    return BEM_OK;
}

static bem_status ext_form_matvec_check(bem_problem *p, const void *x, void *y, bem_memspace space)
{
    if (!p || !x || !y) return set_error(BEM_E_ARG, "null argument");
    if (space != BEM_HOST && space != BEM_DEVICE) return set_error(BEM_E_ARG, "bad memory space");
    if (!p->ops_ready || !p->proj_ready) return set_error(BEM_E_STATE, "assemble operators and projection first");
    return BEM_OK;
}

bem_status bem_solve_pmchwt(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts,
                            void *traces, bem_memspace space, bem_stats *stats)
{
    bem_status s = ext_form_check(p, dirs, nrhs, opts, traces, space);
    return s ? s : ext_form_solve_impl(p, 1, dirs, nrhs, opts, traces, space, stats);
}

bem_status bem_pmchwt_matvec(bem_problem *p, const void *x, void *y, int32_t strong, bem_memspace space)
{
    bem_status s = ext_form_matvec_check(p, x, y, space);
    return s ? s : ext_form_matvec_impl(p, 1, x, y, strong, space);
}

bem_status bem_solve_hc_neumann(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts,
                                void *traces, bem_memspace space, bem_stats *stats)
{
    bem_status s = ext_form_check(p, dirs, nrhs, opts, traces, space);
    return s ? s : ext_form_solve_impl(p, 2, dirs, nrhs, opts, traces, space, stats);
}

bem_status bem_hc_neumann_matvec(bem_problem *p, const void *x, void *y, int32_t strong, bem_memspace space)
{
    bem_status s = ext_form_matvec_check(p, x, y, space);
    return s ? s : ext_form_matvec_impl(p, 2, x, y, strong, space);
}

}  // extern "C"
