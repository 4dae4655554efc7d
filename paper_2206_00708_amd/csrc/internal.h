// Private declarations of the bemtx library (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <utility>
#include <string>
#include <cstdlib>
#include <new>
#include <vector>

#include "../../include/bemtx.h"

namespace bemtx {

// ---------------------------------------------------------------- layout
// Triangles are grouped into locality blocks of at most BT consecutive
// triangles (Morton order of centroids) touching at most SMAX distinct
// vertices; a vertex appears in at most LMAX corners of one block.
constexpr int BT = 16;
constexpr int SMAX = 24;
constexpr int LMAX = 12;
constexpr int SLOT_OFF_LD = 32;   // row length of the per-block slot offsets (SMAX + 1 used)
// block-pair tiles per assembly strip: the tile scratch holds two strips
// (FP64: 2 x 2.4 GB) whatever the mesh size
constexpr int64_t ASM_STRIP_TILES = 65536;
constexpr int NG_MAX = 16;

// Row stride (elements) of the dense operator matrices: a multiple of 32, so
// rows start on 256-byte boundaries and a complex64 row read as floats has a
// length that is a multiple of 64 (the longest k stage of the matrix-core
// product).  Padding columns hold zeros.
__host__ __device__ inline int64_t op_ld(int64_t nv) { return (nv + 31) & ~int64_t(31); }

// Per-triangle geometry table, built on the device (44 doubles, 352 B).
struct alignas(16) TriGeo {
    double p[3][3];     // vertices in the triangle's own corner order
    double qp[6][3];    // points of the 6-point rule
    double n[3];        // unit normal (right-hand rule, outward)
    double area;
    double curl[3][3];  // surface curl of the P1 function of corner a
    double c[3];        // centroid
    double rho;         // largest distance from the centroid to a point of the 6-point rule
};

// Single-precision geometry for the mixed-precision regular kernel: the
// centroid stays FP64 and the quadrature points are stored relative to it,
// so differences of nearby points keep full FP32 accuracy.
struct alignas(8) TriGeoF {
    double c[3];        // centroid
    float dq[6][3];     // quadrature points minus centroid
    float n[3];
    float area;
    float curl[3][3];
    float pad;
};

// Ordered singular pair: x on `tau` (test), y on `sig` (trial); kind = shared
// vertices (3 coincident, 2 edge, 1 vertex); perms map reference vertex r to
// the triangle's own corner.
struct SingPair {
    int32_t tau, sig;
    int32_t kind;
    int32_t perm;   // px0 | px1<<2 | px2<<4 | py0<<6 | py1<<8 | py2<<10
};

// Device allocation tracked against the context budget.
struct DevMem {
    void *ptr = nullptr;
    size_t bytes = 0;
    bem_ctx *ctx = nullptr;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem();
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Host blocks of 128 KB and more (mesh tables, CSR arrays) come from a
// process-wide cache of freed blocks (exact sizes rounded to 64 KB, at most
// 256 MB kept): a mesh built after another of similar size reuses resident
// pages instead of mapping and faulting in fresh ones.
void *host_block_get(size_t bytes);
void host_block_put(void *p, size_t bytes);
constexpr size_t kHostBlockMin = size_t(128) << 10;
inline size_t host_block_round(size_t bytes) { return (bytes + 0xFFFF) & ~size_t(0xFFFF); }

template <class T> struct HostCacheAlloc {
    using value_type = T;
    HostCacheAlloc() = default;
    template <class U> HostCacheAlloc(const HostCacheAlloc<U> &) {}
    T *allocate(size_t n)
    {
        const size_t b = n * sizeof(T);
        if (b < kHostBlockMin) {
            void *p = std::malloc(b ? b : 1);
            if (!p) throw std::bad_alloc();
            return static_cast<T *>(p);
        }
        return static_cast<T *>(host_block_get(host_block_round(b)));
    }
    void deallocate(T *p, size_t n)
    {
        const size_t b = n * sizeof(T);
        if (b < kHostBlockMin) std::free(p);
        else host_block_put(p, host_block_round(b));
    }
    template <class U> bool operator==(const HostCacheAlloc<U> &) const { return true; }
    template <class U> bool operator!=(const HostCacheAlloc<U> &) const { return false; }
};
template <class T> using HVec = std::vector<T, HostCacheAlloc<T>>;

// Host-side mesh tables (internal numbering) and their device copies.
struct MeshData {
    int64_t nv = 0, nt = 0;
    HVec<double> xyz_user;      // caller numbering
    HVec<int32_t> tri_user;
    HVec<int32_t> v_of_int;     // internal vertex -> caller vertex
    HVec<int32_t> int_of_v;     // caller vertex -> internal vertex
    HVec<double> xyz;           // internal numbering [nv][3]
    HVec<int32_t> tri;          // internal triangles, internal vertex ids [nt][3]
    // blocks
    int32_t nb = 0;
    HVec<int32_t> blk_start;    // [nb+1]
    HVec<int32_t> blk_nslot;    // [nb]
    HVec<int32_t> blk_slots;    // [nb][SMAX] internal vertex ids
    HVec<uint8_t> slot_cnt;     // [nb][SMAX]
    HVec<uint8_t> slot_ent;     // [nb][SMAX][LMAX] = tlocal*3 + corner
    // slot-major ranks of a block's corners (the order of its slot lists): slot_off[b][q] the first rank of
    // slot q (slot_off[b][nslot] = number of corners), slot_rank[b][tlocal * 3 + corner] the corner's rank
    HVec<uint8_t> slot_off;     // [nb][SLOT_OFF_LD]
    HVec<uint8_t> slot_rank;    // [nb][3 * BT]
    HVec<int32_t> memb_ptr;     // [nv+1]
    HVec<int32_t> memb;         // block<<8 | slot
    // assembly strips: tile rows (first block of the tile) [strip_b[s], strip_b[s+1]), at most ASM_STRIP_TILES
    // tiles each (one block row at least); strip_rows[strip_rptr[s] ..] the vertices with a membership in the
    // strip's blocks (ascending); strip_lo[s] the first vertex with a membership at or after strip_b[s]
    HVec<int32_t> strip_b, strip_rptr, strip_rows, strip_lo;
    // singular pairs and near-field scatter lists
    HVec<SingPair> sing;        // sorted by kind (3, 2, 1)
    int32_t nsing_kind[4] = {0, 0, 0, 0};
    std::vector<int32_t> near_i, near_j, near_ptr, near_src;   // src = pair*9 + a*3 + b
    std::vector<int32_t> near_row;   // near entries of row i: [near_row[i], near_row[i + 1])
    // vertex star (RHS gather): triangle*3 + corner
    std::vector<int32_t> star_ptr, star_ent;
    double area_total = 0.0;
};

struct MeshDev {
    DevMem perm;   // caller vertex -> internal vertex (int32)
    DevMem geof;   // TriGeoF table
    DevMem xyz, tri, blk_start, blk_nslot, slot_off, slot_rank, memb_ptr, memb, sing, near_i, near_j,
        near_ptr, near_src, near_row, star_ptr, star_ent, geo, strip_rows;
};

// CSR in internal numbering
struct Csr {
    int64_t nrows = 0, ncols = 0;
    HVec<int32_t> ptr, col;
    HVec<double> val;
};

bem_status set_error(bem_status code, const std::string &msg);
bem_status hip_error(hipError_t e, const char *what);
#define BEM_HIP(call)                                                     \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return ::bemtx::hip_error(e_, #call);       \
    } while (0)

// Device memory of at least `bytes` for m, from the context's reuse cache
// when a block fits.  `use`: the stream that will first touch the block; a
// cached block handed to a stream other than the context's main stream
// waits there for the main-stream work queued before the block's release.
bem_status dev_alloc(bem_ctx *ctx, DevMem &m, size_t bytes, hipStream_t use = nullptr);

// Run f(begin, end) over [0, n) split into contiguous ranges on up to 16 host
// threads (serial below `grain` items).  Ranges are fixed by n, so results
// that each range writes to its own slots are independent of scheduling.
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &f);
// validation + tables (host); assembly strips of at most strip_tiles block-pair tiles
bem_status mesh_prepare(MeshData &m, int64_t strip_tiles = ASM_STRIP_TILES);
void mass_csr(const MeshData &m, Csr &M);
bem_status mortar_csr(const MeshData &mi, const MeshData &me, Csr &P, double *coverage_defect);
// candidate search of the mortar assembly: the cones of both meshes'
// triangles seen from the origin, and the interior triangles by cell of a
// [-1, 1]^3 grid of cone centres (CSR, ascending within a cell)
struct MortarGrid {
    std::vector<double> ci, ri, ce, re;
    int ncell = 1;
    double h = 2.0;
    std::vector<int32_t> cell_ptr, cell_tri;
};
void mortar_grid(const MeshData &mi, const MeshData &me, MortarGrid &g);
// P_int,ext from the pair contributions in facet order: interior triangle
// ti[k], exterior facet te[k], block blk[9 k + 3 a + b]
bem_status mortar_csr_device(bem_ctx *ctx, const bem_mesh *mi, const bem_mesh *me, hipStream_t st, Csr &P,
                             double *coverage_defect);
bem_status mortar_from_contribs(const MeshData &mi, const MeshData &me, int64_t ncon, const int32_t *ti,
                                const int32_t *te, const double *blk, double worst, Csr &P);
void transpose_csr(const Csr &A, Csr &At);

// Sparse inverse-mass apply (mass_cheb.cpp): Chebyshev iteration on the
// Jacobi-scaled mass matrix, s steps per launch on overlapping patches of
// vertices (owned range + every vertex within s edges, listed by distance).
constexpr int CHEB_OWN_MAX = 512;    // owned vertices per patch (halved until the patches fit)
constexpr int CHEB_LMAX = 2048;      // vertices per patch: 2 per thread of a 1024-thread workgroup
constexpr int CHEB_WMAX = 16;        // entries per mass-matrix row (the vertex and its neighbours)
constexpr int CHEB_S = 12;           // steps per launch
struct ChebTables {
    int s = 0, own = 0, lmax = 0;
    int nparts[2] = {0, 0};           // patches of each mesh (mesh 0 first)
    HVec<int32_t> pmesh;              // [patch] mesh
    HVec<int32_t> vbeg;               // [patch + 1] offsets of the local vertex lists
    HVec<int32_t> cnt;                // [patch][s + 1] vertices within d edges of the owned range
    HVec<int32_t> vert;               // local vertex -> mesh vertex (internal numbering)
    HVec<double> dinv;                // 1 / M_vv
    HVec<int32_t> rptr;               // [local vertex + 1] row starts into col / val (rows within s - 1 edges)
    HVec<int32_t> col;                // local column index within the patch
    HVec<double> val;
    int ell_w = 0;                    // the rows as ELL blocks: patch p at ell_w vbeg[p], [q][local row]
    HVec<uint16_t> ecol;
    HVec<double> eval;
};
bem_status cheb_tables(const Csr M[2], int s, ChebTables &T);

// dense inverse masses for a matrix-core block solve of R runs (the choice by size; api.cpp)
bool block_dense_mass(const bem_problem *p, int R);

// Kernel-shape tuning table (tune.cpp): process-wide, persisted in a text
// file.  tuned() returns the value of `key`, running `tune` once per key (other
// callers of the same key wait for its result) and recording what it picks;
// a recorded value that `valid` (when given) rejects, such as an entry of an
// older format, is tuned again and replaced.
int tune_class(int64_t n);   // size class: quarter octaves of n
bem_status tuned(const std::string &key, std::vector<int> &value,
                 const std::function<bem_status(std::vector<int> &)> &tune,
                 const std::function<bool(const std::vector<int> &)> &valid = nullptr);
std::string tune_table_text();
void gauss_legendre01(int n, double *x, double *w);      // Jacobi eigenvalue method

}  // namespace bemtx

namespace bemtx {
// kernels timed by the optional per-launch HIP-event timer of a context
enum KernelId { K_REGULAR = 0, K_GATHER, K_SINGULAR, K_NEAR, K_MTF_DENSE, K_MASS_APPLY, K_CGS_DOTS, K_CGS_UPDATE,
                K_ARNOLDI_FINISH, K_MASS_INVERSE, K_BLOCK_GEMM, K_MASS_GEMM, K_KRYLOV_NORM, K_FIELD, K_MORTAR, K_COUNT };
extern const char *const kKernelNames[K_COUNT];
}  // namespace bemtx

struct bem_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // second stream (default priority) for the mass and mortar set-up, so that
    // it overlaps the operator assembly on `stream`; created at first use
    hipStream_t aux = nullptr;
    // stream that GMRES graphs are captured on (capture records, runs nothing;
    // the graphs are launched on `stream`, which may be the null stream)
    hipStream_t capture = nullptr;
    // stream of the assembly's gathers, which overlap the next strip's tiles on `stream`
    hipStream_t gather = nullptr;
    hipEvent_t strip_ev[5] = {};   // the strip assembly's ordering events (created at first use, kept)
    int64_t strip_tiles = bemtx::ASM_STRIP_TILES;   // block-pair tiles per assembly strip of meshes made here
    size_t budget = 0;
    size_t in_use = 0;
    // per-kernel timing (HIP events around each launch on `stream`)
    uint32_t ktiming = 0;   // bit k set: time kernel k
    struct Pending { int id; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double ktotal_ms[bemtx::K_COUNT] = {};
    int64_t kcount[bemtx::K_COUNT] = {};
    // assembly scratch (block-pair tiles, singular contributions), grown on demand
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // Device blocks the library has released, kept for reuse by size class.
    // Main-stream reuse needs no wait (stream order); every release records
    // release_ev on the main stream, and a cached block handed to the
    // auxiliary stream first waits for it.  Work on the auxiliary stream
    // ends before the call that queued it returns.  in_use counts the
    // blocks until bem_ctx_trim, bem_ctx_destroy or a budget shortfall
    // returns them to the device.
    std::multimap<size_t, void *> free_blocks;
    hipEvent_t release_ev = nullptr;
    size_t cached_bytes = 0;
    std::mutex mem_mu;
};

namespace bemtx {
// Timing events for one kernel launch when the context asks for it; the
// events ride on the dispatch itself (hipExtLaunchKernel), so they measure
// the kernel's execution and nothing queued around it.
struct KTimer {
    bem_ctx *c;
    int id;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(bem_ctx *ctx, int kid);
    ~KTimer();
};

// While one of these lives on a thread, KTimer takes no events on that
// thread (calls that must not create events or touch the context's pool).
struct NoTiming {
    bool prev;
    NoTiming();
    ~NoTiming();
};

// Launch `kernel` on `st`, timed by `kt` when it holds events.
template <typename... KArgs, typename... Args>
inline void launch_k(const KTimer &kt, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shmem, hipStream_t st,
                     Args &&...args)
{
    if (kt.a && kt.b)
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shmem, st, kt.a, kt.b, 0, std::forward<Args>(args)...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, std::forward<Args>(args)...);
}

// Resolve finished timings (call after the stream has been synchronised).
void flush_kernel_timing(bem_ctx *ctx);

// Matrix-core FP32 product C[kc][c][row] = sum over the k of chunk kc of
// A[row][k] Bt[c][k] (gemm.hip).  Up to GEMM_MAXSEG independent segments per
// launch; K and kchunk multiples of 32, Bt with 128 * ncb rows.
constexpr int GEMM_MAXSEG = 8;
struct GemmSeg {
    const float *A;     // [M][lda], row-major
    const float *Bt;    // [128 ncb][ldb], k contiguous
    float *C;           // [nk][128 ncb][M], nk = ceil(K / kchunk)
    int64_t lda, ldb;
    int M, K, kchunk, ncb;
    int tile0;          // set by the launcher
};
struct GemmArgs {
    GemmSeg seg[GEMM_MAXSEG];
    int nseg;
    int kst;            // k per LDS stage: 32 or 64
    const int *done;    // optional: nrun flags, done_stride ints apart; all set = skip
    int done_stride, nrun;
    int nt;             // columns computed per 128-column block: 32 nt (nt = 1, 2, 4)
};
bem_status launch_gemm_f32(bem_ctx *ctx, GemmArgs &G, hipStream_t st, int kernel_id);
}  // namespace bemtx

struct bem_mesh {
    bem_ctx *ctx = nullptr;
    bemtx::MeshData h;
    bemtx::MeshDev d;
};

struct bem_problem {
    bem_ctx *ctx = nullptr;
    const bem_mesh *ext = nullptr, *inte = nullptr;
    double k_ext = 0, k_int = 0, rho_ext = 1, rho_int = 1;
    double k_int_im = 0;   // imaginary part of the interior wavenumber (absorbing interior)
    int mortar_dev = 0;        // mortar geometry on the device (1) or the host (0)
    double t_mortar_ms = 0;    // wall time of the mortar step of the last projection set-up
    int incident = 0;   // 0: plane waves (dirs are directions), 1: point sources (dirs are positions)
    bem_precision prec = BEM_C128;
    int ng = 4;
    double gl_x[bemtx::NG_MAX], gl_w[bemtx::NG_MAX];
    bool ops_ready = false, proj_ready = false;
    // dense operators, internal numbering: [mesh][op] N x N complex (op order V, K, T, D)
    bemtx::DevMem ops[2][4];
    // sparse couplings and masses
    bemtx::Csr M[2], P_ie, P_ei;
    bemtx::DevMem P_ie_ptr, P_ie_col, P_ie_val, P_ei_ptr, P_ei_col, P_ei_val;
    bemtx::DevMem Minv[2];          // dense real inverse mass matrices (FP64 or FP32), when mass_sparse is off
    // inverse-mass apply: mass_mode 0 picks by size, 1 dense M^-1, 2 sparse Chebyshev; mass_sparse is the
    // choice of the last projection set-up
    int mass_mode = 0;
    bool mass_sparse = false;
    // dense inverses present (the dense form, or beside the sparse tables for the matrix-core block products
    // of many runs: built at the first such solve when the choice is by size)
    bool mass_dense = false;
    bemtx::ChebTables cheb;
    bemtx::DevMem cheb_pmesh, cheb_vbeg, cheb_cnt, cheb_vert, cheb_dinv, cheb_ecol, cheb_eval;
    // per near entry (i, j) of each mesh: V_ij - V_ji (j < i, else 0), D_ij - D_ji (likewise),
    // T_ij - K_ji, complex128; the mat-vec reads only K and the upper triangles of V and D
    bemtx::DevMem corr[2];
    std::vector<int32_t> ell_col_h[2];   // host staging of the ELL mass rows (kept for async copies)
    std::vector<double> ell_val_h[2];
    bemtx::DevMem M_ptr[2], M_col[2], M_val[2], M_ell_col[2], M_ell_val[2];
    double t_geometry_ms = 0, t_regular_ms = 0, t_singular_ms = 0, t_projection_ms = 0, t_assembly_ms = 0;
    hipEvent_t asm_ev[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    bool asm_timing_pending = false;
    // ordering of the set-up on the auxiliary stream: it starts after the work
    // queued on the main stream before the operator assembly (ev_pre_asm), and
    // the main stream waits for its end (ev_proj)
    hipEvent_t ev_pre_asm = nullptr, ev_proj = nullptr;
    // multi-RHS products: K chunks per GEMM [operators, inverse masses][tile width 32, 64, 128
    // columns][exterior, interior mesh], picked by timing at first use
    int gemm_nk[2][3][2] = {};
    int gemm_kst[2][3] = {{0, 0, 0}, {0, 0, 0}};   // k per LDS stage of those GEMMs (32 or 64)
    int graphs = 1;                                 // GMRES steps in captured HIP graphs (bem_problem_set_graphs)
    int mtf_ts = 0;                                 // tile edge of the symmetric mat-vec (64 or 128; 0: not tuned yet)
};
