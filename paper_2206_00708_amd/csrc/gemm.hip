// Real FP32 GEMM on the matrix cores (v_mfma_f32_32x32x2f32) for the
// multi-right-hand-side products of the multiple-traces system (Sec. 3.3,
// Eq. "mtf:discrete"): one product of a dense block with R Krylov vectors at
// once, so the complex64 operators are read once for all R directions.
//
// A complex block times R complex vectors is one real product: a row of
// complex64 entries, read as 2N interleaved floats (re, im, re, im, ...),
// times a 2N x 2R real matrix holding each complex vector entry x = (a, b)
// as the 2 x 2 block [[a, b], [-b, a]] gives the interleaved (re, im) of
// the complex result.  The inverse mass matrices (real) use the same kernel
// with real and imaginary parts as separate columns.
//
// The right-hand matrix is stored transposed, Bt[c][k] (k contiguous), so
// both operands are read along k.  A workgroup of four waves computes a
// 128-row x 128-column tile over one K chunk: 32-float slices of A (128 rows)
// and Bt (128 columns) are staged in LDS (double-buffered, rows padded to
// 36 floats), each wave owns 32 rows x 128 columns (four 32 x 32
// accumulators) and issues 16 MFMAs per 8 k values; for fewer right-hand
// columns the tile narrows to 32 or 64 columns (one or two accumulators).  Partial tiles of the K
// chunks go to separate output slices; the caller sums them in a fixed
// order (no atomics, deterministic).  The launch returns at once when the
// Krylov runs it serves have all converged.
#include "internal.h"

namespace bemtx {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int GT_M = 128;   // rows per tile
constexpr int GT_N = 128;   // columns per column block of Bt and C

}  // namespace

// One segment: C[kc][cb * 128 + c][row] = sum over the k of chunk kc of A[row][k] Bt[cb * 128 + c][k],
// for the first 32 NT columns c of each 128-column block (NT = 1, 2, 4); KST k
// per LDS stage (32 or 64: a 64-k stage halves the barriers per k and fits
// one workgroup per compute unit).
template <int NT, int KST>
__global__ __launch_bounds__(256, KST == 32 ? 2 : 1) void gemm_f32_kernel(GemmArgs G)
{
    constexpr int GT_K = KST, GT_LD = KST + 4, KH = KST / 32;   // k halves of 32 per stage
    __shared__ float As[2][GT_M * GT_LD];
    __shared__ float Bs[2][32 * NT * GT_LD];
    if (G.done) {   // every run has converged: nothing left to compute
        bool all = true;
        for (int r = 0; r < G.nrun; ++r) all = all && G.done[(int64_t)r * G.done_stride] != 0;
        if (all) return;
    }
    // segment of this workgroup; fields picked by uniform selects (no
    // dynamic indexing of the argument block, which would go through scratch)
    const float *SA = G.seg[0].A, *SB = G.seg[0].Bt;
    float *SC = G.seg[0].C;
    int64_t lda = G.seg[0].lda, ldb = G.seg[0].ldb;
    int M = G.seg[0].M, K = G.seg[0].K, kchunk = G.seg[0].kchunk, ncb = G.seg[0].ncb, tile0 = 0;
#pragma unroll
    for (int s = 1; s < GEMM_MAXSEG; ++s)
        if (s < G.nseg && (int)blockIdx.x >= G.seg[s].tile0) {
            SA = G.seg[s].A; SB = G.seg[s].Bt; SC = G.seg[s].C;
            lda = G.seg[s].lda; ldb = G.seg[s].ldb;
            M = G.seg[s].M; K = G.seg[s].K; kchunk = G.seg[s].kchunk; ncb = G.seg[s].ncb; tile0 = G.seg[s].tile0;
        }
    const int t = blockIdx.x - tile0;
    const int nrt = (M + GT_M - 1) / GT_M;
    const int rt = t % nrt, rest = t / nrt, cb = rest % ncb, kc = rest / ncb;
    const int k0 = kc * kchunk, k1 = min(K, k0 + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // cooperative loads: 1024 float4 per operand per stage, 4 per thread;
    // float4 f = tid + 256 q covers row f / 8 = tid / 8 + 32 q, k offset 4 (tid % 8)
    const int lr = tid >> 3, lc = (tid & 7) * 4;
    const float *ag = SA + (int64_t)min(rt * GT_M + lr, M - 1) * lda + lc;   // rows past M: results not stored
    const float *bg = SB + (int64_t)(cb * GT_N + lr) * ldb + lc;
    const int64_t bstep = (int64_t)32 * ldb;
    // row offsets of the other three loads (rows past M clamp to the last row)
    const int arow0 = min(rt * GT_M + lr, M - 1);
    const int64_t aoff1 = (int64_t)(min(rt * GT_M + lr + 32, M - 1) - arow0) * lda;
    const int64_t aoff2 = (int64_t)(min(rt * GT_M + lr + 64, M - 1) - arow0) * lda;
    const int64_t aoff3 = (int64_t)(min(rt * GT_M + lr + 96, M - 1) - arow0) * lda;
    // staged loads in named registers (arrays of float4 here went to scratch)
    float4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;   // k 0-31 of the stage
    float4 sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3;   // k 32-63 (KST = 64)
    (void)rb1; (void)rb2; (void)rb3; (void)sa0; (void)sa1; (void)sa2; (void)sa3;
    (void)sb0; (void)sb1; (void)sb2; (void)sb3;
#define GEMM_FETCH_HALF(k, A0, A1, A2, A3, B0, B1, B2, B3)                         \
    do {                                                                           \
        A0 = *reinterpret_cast<const float4 *>(ag + (k));                          \
        A1 = *reinterpret_cast<const float4 *>(ag + aoff1 + (k));                  \
        A2 = *reinterpret_cast<const float4 *>(ag + aoff2 + (k));                  \
        A3 = *reinterpret_cast<const float4 *>(ag + aoff3 + (k));                  \
        B0 = *reinterpret_cast<const float4 *>(bg + (k));                          \
        if constexpr (NT > 1) B1 = *reinterpret_cast<const float4 *>(bg + bstep + (k)); \
        if constexpr (NT > 2) {                                                    \
            B2 = *reinterpret_cast<const float4 *>(bg + 2 * bstep + (k));          \
            B3 = *reinterpret_cast<const float4 *>(bg + 3 * bstep + (k));          \
        }                                                                          \
    } while (0)
#define GEMM_STASH_HALF(b, h, A0, A1, A2, A3, B0, B1, B2, B3)                      \
    do {                                                                           \
        float *da = &As[b][lr * GT_LD + lc + 32 * (h)];                            \
        float *db = &Bs[b][lr * GT_LD + lc + 32 * (h)];                            \
        *reinterpret_cast<float4 *>(da) = A0;                                      \
        *reinterpret_cast<float4 *>(da + 32 * GT_LD) = A1;                         \
        *reinterpret_cast<float4 *>(da + 64 * GT_LD) = A2;                         \
        *reinterpret_cast<float4 *>(da + 96 * GT_LD) = A3;                         \
        *reinterpret_cast<float4 *>(db) = B0;                                      \
        if constexpr (NT > 1) *reinterpret_cast<float4 *>(db + 32 * GT_LD) = B1;   \
        if constexpr (NT > 2) {                                                    \
            *reinterpret_cast<float4 *>(db + 64 * GT_LD) = B2;                     \
            *reinterpret_cast<float4 *>(db + 96 * GT_LD) = B3;                     \
        }                                                                          \
    } while (0)
#define GEMM_FETCH(k)                                                              \
    do {                                                                           \
        GEMM_FETCH_HALF(k, ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3);                \
        if constexpr (KH > 1) GEMM_FETCH_HALF((k) + 32, sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3); \
    } while (0)
#define GEMM_STASH(b)                                                              \
    do {                                                                           \
        GEMM_STASH_HALF(b, 0, ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3);             \
        if constexpr (KH > 1) GEMM_STASH_HALF(b, 1, sa0, sa1, sa2, sa3, sb0, sb1, sb2, sb3); \
    } while (0)

    v16f acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[n][v] = 0.f;

    int buf = 0;
    if (k0 < k1) {
        GEMM_FETCH(k0);
        GEMM_STASH(0);
    }
    __syncthreads();
    for (int k = k0; k < k1; k += GT_K) {
        const bool more = k + GT_K < k1;
        if (more) GEMM_FETCH(k + GT_K);   // next stage in flight while this one computes
        const float *as = &As[buf][(wave * 32 + (lane & 31)) * GT_LD + 4 * (lane >> 5)];
        const float *bs = &Bs[buf][(lane & 31) * GT_LD + 4 * (lane >> 5)];
#pragma unroll
        for (int kk = 0; kk < GT_K; kk += 8) {
            const float4 a = *reinterpret_cast<const float4 *>(as + kk);
            float4 b[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) b[n] = *reinterpret_cast<const float4 *>(bs + n * 32 * GT_LD + kk);
            // lanes 0-31 hold k = kk..kk+3, lanes 32-63 k = kk+4..kk+7: MFMA q adds k pair (kk+q, kk+4+q)
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                acc[n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b[n].x, acc[n], 0, 0, 0);
                acc[n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b[n].y, acc[n], 0, 0, 0);
                acc[n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b[n].z, acc[n], 0, 0, 0);
                acc[n] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b[n].w, acc[n], 0, 0, 0);
            }
        }
        if (more) {
            GEMM_STASH(buf ^ 1);
            buf ^= 1;
        }
        __syncthreads();
    }
#undef GEMM_FETCH
#undef GEMM_STASH
#undef GEMM_FETCH_HALF
#undef GEMM_STASH_HALF

    // accumulator v of lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32 of
    // the 32 x 32 tile; the output is column-major per chunk, C[kc][c][row], so the
    // 32 rows of one column that a wave holds form one contiguous 128-byte run
    const int ccols = GT_N * ncb;
    float *Cb = SC + ((int64_t)kc * ccols + cb * GT_N + (lane & 31)) * M;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = rt * GT_M + wave * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row < M)
#pragma unroll
            for (int n = 0; n < NT; ++n) Cb[(int64_t)n * 32 * M + row] = acc[n][v];
    }
}

// Fills tile0 of every segment and launches; K and the K chunks must be
// multiples of 32, lda >= K, ldb >= K, and Bt zero where A has padding.
bem_status launch_gemm_f32(bem_ctx *ctx, GemmArgs &G, hipStream_t st, int kernel_id)
{
    if (G.kst != 32 && G.kst != 64) return set_error(BEM_E_ARG, "internal: GEMM stage depth");
    int tiles = 0;
    for (int s = 0; s < G.nseg; ++s) {
        GemmSeg &S = G.seg[s];
        if (S.K % G.kst || S.kchunk % G.kst || S.kchunk <= 0 || S.lda < S.K || S.ldb < S.K || S.M <= 0 || S.ncb <= 0)
            return set_error(BEM_E_ARG, "internal: GEMM segment shape");
        S.tile0 = tiles;
        const int nk = (S.K + S.kchunk - 1) / S.kchunk;
        tiles += ((S.M + GT_M - 1) / GT_M) * S.ncb * nk;
    }
    if (tiles == 0) return BEM_OK;
    KTimer kt(ctx, kernel_id);
    if (G.kst == 32) {
        if (G.nt == 1) launch_k(kt, gemm_f32_kernel<1, 32>, dim3(tiles), dim3(256), 0, st, G);
        else if (G.nt == 2) launch_k(kt, gemm_f32_kernel<2, 32>, dim3(tiles), dim3(256), 0, st, G);
        else launch_k(kt, gemm_f32_kernel<4, 32>, dim3(tiles), dim3(256), 0, st, G);
    } else {
        if (G.nt == 1) launch_k(kt, gemm_f32_kernel<1, 64>, dim3(tiles), dim3(256), 0, st, G);
        else if (G.nt == 2) launch_k(kt, gemm_f32_kernel<2, 64>, dim3(tiles), dim3(256), 0, st, G);
        else launch_k(kt, gemm_f32_kernel<4, 64>, dim3(tiles), dim3(256), 0, st, G);
    }
    BEM_HIP(hipGetLastError());
    return BEM_OK;
}

}  // namespace bemtx
