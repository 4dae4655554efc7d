/*
 * bemtx -- boundary element method for acoustic transmission on two
 * nonconforming triangle meshes of one closed surface, on one AMD MI355X
 * (gfx950).  C ABI.
 *
 * The problem (van 't Wout, "The Boundary Element Method for Acoustic
 * Transmission with Nonconforming Grids", J. Comput. Appl. Math. 2024):
 * a homogeneous body with surface Gamma in free space; time convention
 * exp(-i omega t); wavenumbers k_ext, k_int; densities rho_ext, rho_int;
 * Helmholtz equation with the transmission conditions of Sec. 2 (Eq.
 * "helmholtz").  The interior operators live on the interior mesh, the
 * exterior operators on the exterior mesh (Sec. 2.1, Sec. 3), and the two
 * are coupled by the L2 mortar matrix P_int,ext and its transpose (Sec. 3.1).
 *
 * Discretisation: continuous P1 Lagrange test and trial functions on both
 * meshes (Sec. 2.4); dense Galerkin matrices of the single-layer V,
 * double-layer K, adjoint double-layer T and hypersingular D operators
 * (Sec. 2.1) with an order-four (6-point) triangle rule on pairs that share
 * no vertex and Sauter-Schwab regularising transformations on pairs that
 * share one, two or three vertices (Sec. 5.1).  The multiple-traces system
 * (Sec. 3.3, Eq. "mtf:discrete"), mass-matrix (strong-form) preconditioning
 * (Sec. 3.3) and GMRES without restart (Sec. 5.1).
 *
 * Conventions common to all entry points
 *  - Meshes: vertices `double[nv][3]`, triangles `int32_t[nt][3]`, 0-based,
 *    counter-clockwise seen from outside.  The P1 degree of freedom j is
 *    vertex j; every matrix and vector crossing this ABI uses the caller's
 *    vertex numbering.  (The library renumbers internally for locality.)
 *  - Complex numbers are interleaved (re, im) pairs of doubles: the layout of
 *    C99 `double complex` and of torch.complex128.
 *  - Matrices are row-major; row = test function, column = trial function.
 *  - Memory spaces: BEM_HOST pointers are ordinary host memory; BEM_DEVICE
 *    pointers are device memory of the context's device (e.g. the
 *    data_ptr() of a torch tensor on that device).  The library never frees
 *    caller memory and copies every input it keeps.
 *  - Streams: all device work is issued on the context's stream.  Entry
 *    points that write into caller buffers return after that work has
 *    completed (they synchronise the stream), so the result may be read at
 *    once from any stream.
 *  - Errors: a negative bem_status; bem_last_error() gives a message for the
 *    last failing call on the calling thread.  On error no output is
 *    written and handles stay valid.
 *  - Thread safety: one handle must not be used from two threads at once.
 */
#ifndef BEMTX_H
#define BEMTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bem_status;
enum {
    BEM_OK = 0,
    BEM_W_NOCONV = 1,          /* warning: GMRES reached maxit; best iterate returned */
    BEM_E_ARG = -1,            /* null pointer, size mismatch, non-positive k/rho/tol, ... */
    BEM_E_MESH = -2,           /* not a closed, consistently oriented, outward 2-manifold,
                                  degenerate triangle or unused vertex */
    BEM_E_MESH_MISMATCH = -3,  /* the two meshes do not cover the same surface */
    BEM_E_STATE = -4,          /* call order violated (e.g. solve before assembly) */
    BEM_E_OOM = -5,            /* device allocation failed or over the context budget */
    BEM_E_DEVICE = -6,         /* HIP runtime error (message carries the HIP error) */
    BEM_E_UNSUPPORTED = -7     /* option not available in this build */
};

typedef enum { BEM_HOST = 0, BEM_DEVICE = 1 } bem_memspace;

/* BEM_C128: complex128 operators, mat-vecs and Krylov vectors.
 * BEM_C64_MIXED: complex64 operators and mat-vecs with FP32 accumulation;
 * singular integrals, Arnoldi and iterative-refinement residuals in FP64. */
typedef enum { BEM_C128 = 0, BEM_C64_MIXED = 1 } bem_precision;

typedef struct {
    int32_t singular_gauss;   /* Gauss-Legendre points per coordinate of the singular rule (1..16; 4) */
} bem_quad_opts;

typedef struct {
    double tol;               /* relative residual of the strong form, ||M^-1(b - A x)|| / ||M^-1 b|| */
    int32_t maxit;            /* Arnoldi steps (no restart, Sec. 5.1), 1..3000 */
    int32_t ir_max;           /* BEM_C64_MIXED: outer refinement steps (0: 10) */
    double ir_inner_tol;      /* BEM_C64_MIXED: inner GMRES tolerance (0: automatic) */
    int32_t batch;            /* BEM_C64_MIXED: right-hand sides solved together through one
                                 matrix-core product per step (2..64; 0 or 1: one at a time) */
} bem_solver_opts;

typedef struct {
    int32_t iterations;       /* total Arnoldi steps over all right-hand sides */
    int32_t ir_steps;
    double rel_residual;      /* worst strong-form relative residual, recomputed in FP64 at exit */
    double t_geometry_ms;
    double t_regular_ms, t_singular_ms;   /* device time of each part, summed over the two meshes */
    double t_projection_ms;   /* host time of bem_assemble_projection */
    double t_matrix_ms;       /* t_assembly_ms + t_projection_ms */
    double t_solve_ms;
    double t_iter_ms;         /* t_solve / iterations */
    double t_assembly_ms;     /* device span of the operator assembly of both meshes */
    int32_t graph_steps;      /* Arnoldi steps issued through captured HIP graphs (bem_problem_set_graphs) */
} bem_stats;

typedef struct bem_ctx bem_ctx;
typedef struct bem_mesh bem_mesh;
typedef struct bem_problem bem_problem;

/* Message of the last failing call on this thread (never NULL). */
const char *bem_last_error(void);

/* Context on HIP device `device`, issuing work on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  hbm_budget_bytes caps the device memory the
 * library allocates for problems of this context (0 = no cap).  Ownership:
 * *out is owned by the caller and freed with bem_ctx_destroy after every
 * problem and mesh of the context. */
bem_status bem_ctx_create(int32_t device, void *hip_stream, size_t hbm_budget_bytes, bem_ctx **out);
void bem_ctx_destroy(bem_ctx *ctx);
/* Device bytes currently held by the context: buffers of its meshes and
 * problems, the assembly scratch, and the blocks the library has released
 * and keeps for reuse (freed by bem_ctx_trim, bem_ctx_destroy, or when an
 * allocation would otherwise exceed hbm_budget_bytes or device memory). */
size_t bem_ctx_bytes_in_use(const bem_ctx *ctx);

/* Free the assembly scratch the context keeps between problems (the
 * block-pair tiles of the regular-pair assembly, grown to the largest mesh
 * assembled so far) and the released blocks kept for reuse; later calls
 * allocate again.  Synchronises the context stream.  For callers that
 * account device memory per request. */
bem_status bem_ctx_trim(bem_ctx *ctx);

/* Per-kernel device time.  Kernels, by bit index: 0 "regular_tiles",
 * 1 "gather_tiles", 2 "singular_pairs", 3 "near_scatter", 4 "mtf_dense",
 * 5 "mass_apply", 6 "cgs_dots" (Gram-Schmidt dot products), 7 "cgs_update"
 * (Gram-Schmidt update), 8 "arnoldi_finish" (Hessenberg column, Givens
 * rotation, residual estimate), 9 "mass_inverse", 10 "block_gemm"
 * (multi-RHS operator product), 11 "mass_gemm" (multi-RHS inverse-mass
 * product), 12 "krylov_normalize" (new Krylov vector scaled to unit norm),
 * 13 "field" (field off the surface, bem_field), 14 "mortar" (the two passes
 * of the device mortar geometry, bem_problem_set_mortar).  Every launch of a kernel whose bit is set in
 * kernel_mask is bracketed by HIP events on the context stream (a few
 * microseconds of overhead per launch); 0 disables.  Setting the mask resets
 * the totals.  bem_ctx_kernel_time synchronises the stream and returns the
 * accumulated milliseconds and launch count of one kernel by name
 * (BEM_E_ARG for an unknown name). */
bem_status bem_ctx_set_kernel_timing(bem_ctx *ctx, uint32_t kernel_mask);
bem_status bem_ctx_kernel_time(bem_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);

/* Size of the assembly strips of the meshes created on this context from
 * now on, in block-pair tiles (0: the default, 65536).  The regular-pair
 * assembly (Sec. 5.1) computes the interactions of every pair of 16-triangle
 * blocks as tiles of per-vertex partial sums, strip by strip over
 * consecutive rows of the block-pair triangle, and gathers each strip into
 * the dense operators while the next strip is computed; the tile scratch
 * holds two strips (each strip at least one row of nb tiles: 2 x 65536 x
 * 36,864 B = 4.8 GB in FP64 at the default, half that in complex64),
 * whatever the mesh size.  Smaller strips need less memory and take a
 * little longer (more launches, each with its ramp and tail).  Entries fed by several strips are summed strip
 * by strip, so the strip size changes the last bits of those entries.
 * BEM_E_ARG for a negative count. */
bem_status bem_ctx_set_strip_tiles(bem_ctx *ctx, int64_t tiles);

/* A triangle mesh Gamma_int or Gamma_ext (Sec. 3): checks that it is a closed,
 * consistently oriented 2-manifold with positive enclosed volume, no
 * degenerate triangle and no unused vertex (BEM_E_MESH otherwise), and builds
 * the connectivity tables (adjacent-pair classes, locality blocks).  xyz and
 * tri are host arrays, copied.  Limits: at most 2^30 vertices and
 * triangles (BEM_E_ARG); a vertex may be a corner of at most 12 of the 16
 * triangles of one locality block (consecutive triangles in Morton order of
 * their centroids; a valence above 12 can exceed it) and, for the sparse
 * inverse-mass apply, have at most 15 neighbours (BEM_E_MESH otherwise). */
bem_status bem_mesh_create(bem_ctx *ctx, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt,
                           bem_mesh **out);
void bem_mesh_destroy(bem_mesh *mesh);
int64_t bem_mesh_num_vertices(const bem_mesh *mesh);

/* Transmission problem (Sec. 2, Eq. "helmholtz") on an exterior and an
 * interior mesh of the same star-shaped surface around the origin (the
 * meshes are related by central projection from the origin), with real
 * wavenumbers k_ext, k_int > 0 and densities rho_ext, rho_int > 0.
 * quad may be NULL (defaults).  The meshes must outlive the problem. */
bem_status bem_problem_create(bem_ctx *ctx, const bem_mesh *ext, const bem_mesh *inte,
                              double k_ext, double k_int, double rho_ext, double rho_int,
                              bem_precision precision, const bem_quad_opts *quad, bem_problem **out);
void bem_problem_destroy(bem_problem *p);

/* Device bytes the problem needs with `nrhs` right-hand sides and `maxit`
 * Krylov steps (operators, projections, Krylov bases, Hessenberg and triangular factors,
 * assembly scratch; for BEM_C64_MIXED problems all nrhs runs advancing
 * together, up to 64, with the buffers of the matrix-core products); for
 * admission control.  May be called before assembly. */
bem_status bem_problem_footprint(const bem_problem *p, int32_t nrhs, int32_t maxit, size_t *bytes);

/* Dense Galerkin matrices V, K, T, D on both meshes (Sec. 2.1, 2.4, 5.1),
 * device-resident.  parts: bit 0 = contributions of triangle pairs that share
 * no vertex, bit 1 = pairs that share a vertex (3 = the full operators; other
 * values exist for testing).  Returns once the work is queued on the context
 * stream (so host work such as bem_assemble_projection overlaps it); every
 * later call on the problem is ordered after it. */
bem_status bem_assemble_operators(bem_problem *p, int32_t parts);

/* Mass matrices M_ext, M_int and the mortar matrix P_int,ext (N_int x N_ext)
 * with P_ext,int = P_int,ext^T (Sec. 3.1), device-resident, plus the dense
 * inverse mass matrices used by the strong form (Sec. 3.3).  The sparse
 * matrices are built on the host; their uploads and the inverse masses run
 * on a second stream of the context, ordered after the work queued before
 * bem_assemble_operators and before every later call on the problem, so
 * that they overlap a queued operator assembly.  Returns when they are done.
 * BEM_E_MESH_MISMATCH if the projected interior mesh leaves part of an
 * exterior facet uncovered (relative area defect above 1e-6). */
bem_status bem_assemble_projection(bem_problem *p);

/* Where the next bem_assemble_projection computes the geometry of the mortar
 * matrix P_int,ext (Sec. 3.1: central projection of every candidate interior
 * triangle onto an exterior facet, clipping of the two, and the exact
 * integral of the product of the P1 bases over the intersection):
 * on_device = 0 on the host threads (the default), 1 in kernels on the
 * context's second stream, one wave per exterior facet, with the same
 * arithmetic steps.  Either way the contributions are listed in exterior
 * facet order and the host forms the CSR from them, so the two settings give
 * the same matrix up to rounding (the device may contract products into
 * fused multiply-adds).  BEM_E_ARG for another value. */
bem_status bem_problem_set_mortar(bem_problem *p, int32_t on_device);

/* How the mass-matrix preconditioner blockdiag(M_e, M_e, M_i, M_i)^-1 of
 * the strong form (Sec. 3.3) is applied: mode 1 through dense inverse mass
 * matrices built once per projection set-up (O(N^2) memory; at most 16,384
 * vertices per mesh, else BEM_E_UNSUPPORTED at the set-up); mode 2 without
 * forming M^-1, by Chebyshev iteration on diag(M)^-1 M (its spectrum lies
 * in [1/2, 2] on every P1 mesh, so k steps reduce the error by 4 3^-k;
 * 36 steps for BEM_C128, 24 for BEM_C64_MIXED), 12 steps per launch on
 * overlapping vertex patches, O(N) memory and no size limit (a vertex may
 * have at most 15 neighbours, else BEM_E_MESH at the set-up); mode 0 (the
 * default) picks mode 2 when the dense inverses would exceed 256 MB or a mesh
 * has more than 16,384 vertices, else mode 1; with mode 0, a BEM_C64_MIXED
 * block solve of 32 or more runs (bem_solver_opts.batch) also builds the
 * complex64-form dense inverses at its start when they take at most 1 GB
 * and applies them to all runs as one matrix-core product (cheaper there
 * than a Chebyshev apply per run), while single solves keep the Chebyshev
 * apply.  Both apply M^-1 to FP64 rounding in the FP64 form (products of
 * bem_mtf_matvec, and M^-1 inside the exterior formulations' operators).
 * Where M^-1 only preconditions GMRES on the multiple-traces system
 * (bem_solve: the Arnoldi products, M^-1 b and the final residual), the
 * Chebyshev form takes 12 steps, one launch: a fixed polynomial p(M) within
 * 7.5e-6 of M^-1, so the solve converges to the same solution of the
 * weak-form system and its residual norms are those of p(M), within 1.5e-5
 * relative of the M^-1 norms (a block solve that applies dense inverses
 * uses them for M^-1 b and the residual as well).  Takes effect at the next
 * bem_assemble_projection (a changed mode marks the projection stale).
 * BEM_E_ARG for another mode. */
bem_status bem_problem_set_mass_apply(bem_problem *p, int32_t mode);

/* The choice of the last projection set-up: *sparse = 1 for the Chebyshev
 * apply, 0 for dense inverses.  BEM_E_STATE before the projection. */
bem_status bem_problem_mass_apply(const bem_problem *p, int32_t *sparse);

/* GMRES of the solves (Sec. 5.1: no restart) in captured HIP graphs (on = 1,
 * the default) or as individual launches (0).  With graphs, every whole
 * batch of eight Arnoldi steps after the first goes out as one graph launch
 * on the context's stream: the operator product (mat-vec or matrix-core
 * block product and the inverse-mass apply) and the Gram-Schmidt and Givens
 * kernels of each step, their step index read from device memory, so one
 * graph serves a range of 64 step indices; graphs are captured on first use
 * within a solve and destroyed at its end.  The kernels, their order and
 * their arithmetic are the same in both modes, so the traces agree bit for
 * bit.  Kernels inside graphs carry no per-kernel timing
 * (bem_ctx_set_kernel_timing times the steps launched individually: the
 * first batch and the last steps).  BEM_E_ARG for other values. */
bem_status bem_problem_set_graphs(bem_problem *p, int32_t on);

/* Wall-clock milliseconds of the mortar step (geometry and CSR) of the last
 * bem_assemble_projection, by the setting above.  BEM_E_STATE before the
 * projection is assembled. */
bem_status bem_problem_mortar_ms(const bem_problem *p, double *ms);

/* Apply the discrete multiple-traces matrix of Sec. 3.3 (Eq.
 * "mtf:discrete") to x: y = A x (strong = 0) or y = blockdiag(M_e, M_e, M_i,
 * M_i)^-1 A x (strong = 1).  x, y: complex128 [2 N_ext + 2 N_int] in the
 * unknown order [v_ext, w_ext, v_int, w_int], caller numbering.  Needs both
 * assemblies.  BEM_C64_MIXED problems apply the complex64 operators with
 * FP32 accumulation (the product GMRES uses). */
bem_status bem_mtf_matvec(bem_problem *p, const void *x, void *y, int32_t strong, bem_memspace space);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of bem_mtf_matvec with its work buffers (the permuted input, the
 * weak and strong results and the kernels' partial sums) taken from one
 * static device array of 128 MiB per GPU instead of allocations.  x, y:
 * device pointers, complex128 [2 N_ext + 2 N_int] as above.  Asynchronous on
 * the context's stream: it calls no hipMalloc, hipFree or other allocating
 * routine, no synchronisation, and records no per-kernel timing.  The work
 * space needed is 3 n 16 bytes (rounded to 256) plus the partial sums,
 * the larger of 32 (N_ext + N_int) max(ceil(N_ext / 64), ceil(N_int / 64))
 * bytes (tile partials at the smaller tile edge the tuner may pick) and
 * 96 n bytes (the two work sets of the sparse inverse-mass apply): about
 * 96 MB for 10,242 + 8,002 vertices; a larger problem returns
 * BEM_E_UNSUPPORTED without launching anything.  All calls on one GPU share
 * that GPU's array: calls that overlap in time on one GPU (other streams or
 * contexts) race and must be ordered by the caller.  Same results as
 * bem_mtf_matvec (the same kernels in the same order). */
bem_status bem_mtf_matvec_noalloc(bem_problem *p, const void *x, void *y, int32_t strong);

/* The same product for nrhs vectors at once: x, y complex128 [nrhs][n].
 * BEM_C64_MIXED problems run it on the matrix cores (FP32 products of the
 * complex64 blocks with up to 64 vectors per pass, the complex product as one
 * real product with 2 x 2 blocks per complex entry; FP64 for the mortar
 * terms and the sums of the K chunks); BEM_C128 problems apply the single
 * product to each vector. */
bem_status bem_mtf_matvec_batch(bem_problem *p, const void *x, void *y, int32_t nrhs, int32_t strong,
                                bem_memspace space);

/* Incident field of the problem's solves, right-hand sides and fields:
 * kind 0 (the default) plane waves exp(i k_ext d.x) (Sec. 5.3), whose `dirs`
 * arguments are unit directions; kind 1 point sources
 * exp(i k_ext |x - x0|) / (4 pi |x - x0|) (Sec. 5.7), whose `dirs` arguments
 * are the source positions x0 (finite; a source on or near the exterior
 * mesh makes the loads' quadrature inaccurate).  BEM_E_ARG for another kind. */
bem_status bem_problem_set_incident(bem_problem *p, int32_t kind);

/* Absorbing interior (the foam model of Sec. 5.7, whose interior wavenumber
 * carries an imaginary part that grows with frequency): the interior
 * wavenumber becomes k_int + i k_int_imag, so that the interior Green's
 * function is exp(i k_int r - k_int_imag r) / (4 pi r) in the assembly of the
 * interior operators (regular and singular pairs, both precisions) and in the
 * interior field of bem_field.  k_int_imag >= 0 and finite, else BEM_E_ARG;
 * 0 (the default) is the lossless medium.  A changed value marks the
 * assembled operators stale: call bem_assemble_operators again before a
 * solve (BEM_E_STATE otherwise). */
bem_status bem_problem_set_k_int_imag(bem_problem *p, double k_int_imag);

/* Right-hand side [-f, -g, 0, 0] of the multiple-traces system for the
 * plane wave exp(i k_ext d.x) (Sec. 5.3, Eq. "planewave"):
 * f_j = <u_inc, phi_j>, g_j = <du_inc/dn, phi_j> on the exterior mesh.
 * dirs: host double[nrhs][3] unit vectors; b: complex128 [nrhs][n]. */
bem_status bem_mtf_rhs(bem_problem *p, const double *dirs, int32_t nrhs, void *b, bem_memspace space);

/* Solve the multiple-traces system for nrhs plane waves with GMRES without
 * restart on the mass-preconditioned form, x0 = 0 (Sec. 3.3, 5.1).
 * traces: complex128 [nrhs][2 N_ext + 2 N_int], the unknowns
 * [v_ext, w_ext, v_int, w_int] of the printed system; with its signs the
 * total field satisfies p = -v_ext, dp/dn+ = -w_ext on Gamma_ext and
 * p = -v_int, dp/dn- = -w_int on Gamma_int.  Returns BEM_W_NOCONV if a
 * right-hand side did not reach opts->tol within opts->maxit (its best
 * iterate is written).  Success is decided on the true residual
 * |M^-1 (b - A x)| / |M^-1 b|, recomputed in FP64 after the GMRES run
 * (stats->rel_residual, the largest over the right-hand sides): when the
 * Arnoldi estimate met the tolerance and the true residual did not, an
 * FP64 run of one right-hand side first restarts once from the true
 * residual with the remaining steps (the mixed form refines instead).
 * stats may be NULL.
 * BEM_C64_MIXED: iterative refinement; each step solves the correction
 * system with GMRES (FP64 Krylov basis) to opts->ir_inner_tol (0: half the
 * remaining reduction, at least 1e-7), its products of the complex64
 * operators accumulated in FP32 once the residual estimate is below 2e4
 * times that tolerance and in FP64 before (single right-hand side; block
 * runs use FP32 throughout), then recomputes M^-1 (b - A x) with FP64
 * arithmetic on the stored operators; at most
 * opts->ir_max steps (0: 10) and opts->maxit Arnoldi steps in total.
 * With opts->batch > 1 up to that many right-hand sides run as independent
 * GMRES instances that share one matrix-core product per step (each run has
 * its own Krylov basis, rotations and stopping test, so each result equals
 * its single solve up to FP32 rounding of the products). */
bem_status bem_solve(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts,
                     void *traces, bem_memspace space, bem_stats *stats);

/* Exterior PMCHWT formulation (Sec. 3.3, Eq. "pmchwt:discrete"): on the
 * exterior mesh, [-K_e - hat(K_i), V_e + a hat(V_i); D_e + hat(D_i) / a,
 * T_e + hat(T_i)] [v; w] = [f; g] with hat(X) = P_ext,int M_int^-1 X
 * M_int^-1 P_int,ext and a = rho_int / rho_ext (the interior operators
 * scaled as in the single-trace Calderon system, Sec. 2.2), f, g as in
 * bem_mtf_rhs.  The unknowns are the traces of the total field on the
 * exterior mesh: v = p, w = dp/dn+.  Uses the operators and projection of
 * the problem (assemble both first; BEM_E_STATE otherwise).
 * bem_solve_pmchwt: GMRES without restart on the mass-preconditioned form
 * M_ext^-1 A x = M_ext^-1 [f; g], x0 = 0, FP64 Arnoldi as in bem_solve, one
 * right-hand side at a time; traces: complex128 [nrhs][2 N_ext] in caller
 * numbering, in `space`; BEM_W_NOCONV as in bem_solve; BEM_E_UNSUPPORTED
 * for BEM_C64_MIXED problems (opts->batch and the refinement fields are
 * not used).
 * bem_pmchwt_matvec: y = A x (strong = 0) or M_ext^-1 A x (strong = 1),
 * x, y: complex128 [2 N_ext] in caller numbering, in `space`; synchronises
 * the context stream. */
bem_status bem_solve_pmchwt(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts,
                            void *traces, bem_memspace space, bem_stats *stats);
bem_status bem_pmchwt_matvec(bem_problem *p, const void *x, void *y, int32_t strong, bem_memspace space);

/* Exterior high-contrast Neumann formulation (Sec. 2.3, Eq.
 * "highcontrast:ext:neu", discrete form of Sec. 3.3): on the exterior mesh,
 *   [1/2 M_e - hat(T_i), -c hat(D_i) M_e^-1 V_e; M_e, 1/2 M_e - T_e] [a; b]
 *     = [c hat(D_i) M_e^-1 f; g],  c = rho_ext / rho_int,
 * hat(X) = P_ext,int M_int^-1 X M_int^-1 P_int,ext; a = dp/dn+ on the
 * exterior mesh and b = mu, the density of the scattered field
 * u_s = [SLP_ext mu] (indirect representation).  The hypersingular term of
 * the right-hand side acts on the P1 coefficients M_e^-1 f of the incident
 * Dirichlet trace.  bem_solve_hc_neumann and bem_hc_neumann_matvec behave as
 * bem_solve_pmchwt and bem_pmchwt_matvec (same arguments, layouts, errors). */
bem_status bem_solve_hc_neumann(bem_problem *p, const double *dirs, int32_t nrhs, const bem_solver_opts *opts,
                                void *traces, bem_memspace space, bem_stats *stats);
bem_status bem_hc_neumann_matvec(bem_problem *p, const void *x, void *y, int32_t strong, bem_memspace space);

/* Total acoustic field at points off the surface, from the unknowns of
 * bem_solve, by the representation formulas (Sec. 2, Eq. "representation"):
 * at an exterior point the incident wave exp(i k_ext d.x) plus
 * [SLP_ext w_ext - DLP_ext v_ext](x), at an interior point
 * [DLP_int v_int - SLP_int w_int](x) (the interior potentials of the
 * printed system are -gamma_D p and -gamma_N p), with
 * [SLP psi](x) = int G psi, [DLP phi](x) = int dG/dn(y) phi,
 * G = exp(i k r) / (4 pi r), outward normals, the P1 functions of the
 * nodal unknowns, and each triangle integral by the 6-point rule of the
 * regular assembly (no near-surface refinement: points close to a mesh get
 * that rule's error; a point on a quadrature point gives a non-finite value).
 * dirs: host double[nrhs][3] unit vectors, the plane waves of the solve;
 * traces: complex128 [nrhs][2 N_ext + 2 N_int] as written by bem_solve;
 * points: double [npts][3]; region: int32 [npts], 0 exterior, 1 interior
 * (bem_mesh_winding of the exterior mesh decides it where the caller has no
 * better rule); field: complex128 [nrhs][npts], caller order.  traces,
 * points, region and field are all in `space`; the call copies the points
 * and regions to the host to sort them by region, and synchronises the
 * context stream.  Errors: BEM_E_ARG (null pointers with npts > 0, a
 * region other than 0 or 1, directions not of unit length, more than 2^28
 * points), BEM_E_OOM, BEM_E_DEVICE.  npts = 0 does nothing. */
bem_status bem_field(bem_problem *p, const double *dirs, int32_t nrhs, const void *traces, const double *points,
                     const int32_t *region, int64_t npts, void *field, bem_memspace space);

/* Winding numbers of a mesh at points: the sum over triangles of the signed
 * solid angle (Van Oosterom and Strackee, 1983) over 4 pi, 1 inside a
 * closed outward-oriented mesh and 0 outside (up to rounding), in between
 * near the surface.  points: double [npts][3]; w: double [npts]; both in
 * `space`.  Synchronises the context stream.  Errors: BEM_E_ARG,
 * BEM_E_OOM, BEM_E_DEVICE. */
bem_status bem_mesh_winding(const bem_mesh *m, const double *points, int64_t npts, double *w, bem_memspace space);

/* The kernel shapes picked by timing so far (the library's tuner): one line
 * per size class, "key value...": "gemm-ops:c<columns>:e<class>:i<class>
 * <K chunks, exterior> <K chunks, interior> <k per LDS stage>" for the
 * multi-right-hand-side operator product (an entry in another format is
 * tuned again), "gemm-mass:..." likewise for the dense inverse-mass product,
 * "mtf-c128:..." / "mtf-c64:... <tile edge>" for the symmetric mat-vec;
 * class = round(4 log2 N) of the exterior and interior vertex counts.  The
 * table is shared by all contexts of the process and kept in the file
 * $BEMTX_TUNE_FILE (else $XDG_CACHE_HOME/bemtx/tune-gfx950.txt, else
 * $HOME/.cache/bemtx/tune-gfx950.txt), so a size class is timed once.
 * Writes at most cap bytes (NUL-terminated) to buf when buf is not NULL;
 * *len receives the text's length without the NUL. */
bem_status bem_tune_table(char *buf, size_t cap, size_t *len);

/* Copy one dense operator: mesh 0 = exterior, 1 = interior; op one of 'V',
 * 'K', 'T', 'D'.  dst: [N][N] in caller numbering, complex128 for BEM_C128
 * problems and complex64 for BEM_C64_MIXED (the stored values). */
bem_status bem_copy_operator(const bem_problem *p, int32_t mesh, char op, void *dst, bem_memspace space);

/* Copy the mortar matrix P_int,ext as CSR in caller numbering (host arrays).
 * With rowptr == NULL only *nnz is returned.  rowptr: int64[N_int + 1],
 * col: int32[nnz], val: double[nnz]; columns sorted within each row. */
bem_status bem_copy_projection(const bem_problem *p, int64_t *rowptr, int32_t *col, double *val, int64_t *nnz);

/* ---- host-only entry points (no device needed) ----------------------- */

/* The mesh checks of bem_mesh_create (closed, oriented outward, no
 * degenerate triangle, no unused vertex) on host arrays. */
bem_status bem_check_mesh(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt);

/* The mortar matrix P_int,ext of bem_assemble_projection computed on host
 * arrays (Sec. 3.1), in caller numbering, CSR with sorted columns.  With
 * rowptr == NULL only *nnz is returned; otherwise rowptr: int64[nv_int + 1],
 * col: int32[*nnz], val: double[*nnz] must hold the size from the first call.
 * coverage_defect (nullable) receives the largest relative area defect of an
 * exterior facet.  Meshes are validated as in bem_mesh_create. */
bem_status bem_host_mortar(const double *xyz_int, int64_t nv_int, const int32_t *tri_int, int64_t nt_int,
                           const double *xyz_ext, int64_t nv_ext, const int32_t *tri_ext, int64_t nt_ext,
                           int64_t *rowptr, int32_t *col, double *val, int64_t *nnz, double *coverage_defect);

/* The FP64 sine and cosine the kernels use for the phase k|x-y| (Cody-Waite
 * reduction by pi/2, Taylor polynomials on [-pi/4, pi/4]), on host arrays of
 * n values; same arithmetic as the device code. */
bem_status bem_host_phase_sincos(int64_t n, const double *x, double *s, double *c);

/* n-point Gauss-Legendre rule on [0,1] used by the singular quadrature
 * (1 <= n <= 16). */
bem_status bem_host_gauss_legendre(int32_t n, double *x, double *w);

#ifdef __cplusplus
}
#endif
#endif
