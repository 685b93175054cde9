/*
 * spx.h - C ABI of an MI355X (gfx950) supernodal sparse Cholesky (and L D L^T) solver.
 *
 * The operation is the one of "Taking advantage of hybrid systems for sparse
 * direct solvers via task-based runtimes" (Lacoste et al.), Section III:
 * solve A x = b for a sparse symmetric positive definite A by
 *   1. an ordering by nested dissection and a symbolic analysis (elimination
 *      tree, predicted nonzero pattern of the factor grouped into column
 *      blocks, amalgamation allowing extra fill, vertical splitting of wide
 *      supernodes)                                   -> spx_analyze
 *   2. the numerical supernodal factorization P A P^T = L L^T (or L D L^T,
 *      SPX_LDLT, the paper's symmetric-indefinite variant): per column
 *      block, dense factorization of the diagonal block, triangular solve of
 *      the off-diagonal rows, and right-looking updates of the facing column
 *      blocks (Section III, the "1D task" and its split into one task per
 *      panel and one per couple of panels)          -> spx_factorize
 *   3. forward and backward triangular solves with the factor, followed by
 *      iterative refinement with an FP64 residual   -> spx_solve
 * Static pivoting (no dynamic pivoting, Section III) makes the structure
 * depend on the pattern only, so one analysis serves many factorizations and
 * one factorization many solves.
 *
 * Conventions.  Indices are 0-based.  A matrix pattern is given in compressed
 * sparse column form: colptr[n+1] (int64, non-decreasing, colptr[0] = 0) and
 * rowind[colptr[n]] (int32, strictly increasing inside a column, in [0, n)).
 * Either the full symmetric pattern or only its lower triangle may be given;
 * the pattern is symmetrized internally.  Values passed to spx_factorize are
 * aligned with that pattern; only entries with row >= column are read.
 *
 * Errors.  Every function returns SPX_OK (0) or a negative code; the text of
 * the last error of a handle is available from spx_last_error.  No function
 * throws.  A handle must not be used by two threads at once.  Calls that take
 * a hip_stream (a hipStream_t, or NULL for the default stream) enqueue their
 * device work on that stream and return when it has finished.
 */
#ifndef SPX_H
#define SPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum spx_status {
    SPX_OK = 0,
    SPX_EINVAL = -1,   /* bad argument, bad pattern (unsorted, out of range, duplicate) */
    SPX_ENOMEM = -2,   /* host or device allocation failed */
    SPX_EDEVICE = -3,  /* a HIP runtime call failed, or the device scheduler stopped early */
    SPX_ESTATE = -4,   /* call out of order (e.g. solve before factorize) */
    SPX_ENOTPD = -5,   /* a pivot was not > 0 (or NaN): matrix not positive definite;
                        * SPX_LDLT: a pivot was zero or not finite */
    SPX_ENOCONV = -6   /* refinement did not reach the tolerance; x is still returned */
};

enum spx_method {
    SPX_LLT = 0,   /* P A P^T = L L^T, A symmetric positive definite */
    SPX_LDLT = 1,  /* P A P^T = L D L^T with unit L and diagonal D, A symmetric with
                    * non-zero pivots in the computed order (static pivoting,
                    * Section III: the structure is the one of L L^T); e.g.
                    * quasi-definite matrices.  All precision modes (the FP32
                    * modes refine in FP64 as for SPX_LLT) */
    SPX_LU = 2     /* P A P^T = L U with unit L, A unsymmetric with a symmetric or
                    * unsymmetric pattern (analysed on the pattern of A + A^T) and
                    * non-zero pivots in the computed order (static pivoting,
                    * Section III: steps 2 and 3 duplicated for L and U).  Values
                    * of both triangles are read.  All precision modes; fuse_small
                    * is ignored (treated as 0); spx_values_grad is not available.
                    * The factor is two panel arrays of the same layout: L (the
                    * square diagonal blocks hold unit L strictly below the
                    * diagonal and U on and above it), then U^T below the
                    * diagonal blocks (row r of column c: u_{c, row r}) */
};

enum spx_precision {
    SPX_FP64 = 0,     /* factor stored and computed in FP64 */
    SPX_FP32_IR = 1,  /* factor stored in FP32, products on the FP32 matrix cores
                       * (the 32x32 diagonal tiles are factored and inverted in
                       * FP64 and rounded); the solve applies the FP32 factor
                       * in FP64 arithmetic and refines with the FP64 residual
                       * until omega <= ir_tol */
    SPX_BF16X3_IR = 2 /* as SPX_FP32_IR, but the update and panel-solve products
                       * split each FP32 operand x into hi = bf16(x) and
                       * lo = bf16(x - hi) and sum hi*hi + hi*lo + lo*hi on the
                       * BF16 matrix cores with FP32 accumulation (about 2^-16
                       * relative per product); refinement as SPX_FP32_IR */
};

typedef struct spx_options {
    int32_t method;           /* enum spx_method (SPX_LLT) */
    int32_t leaf_size;        /* nested dissection stops at components of this size (64) */
    int32_t amalg_pct;        /* extra fill allowed by amalgamation, percent of nnz(L) (12) */
    int32_t split_width;      /* column blocks wider than this are split (256, at most 256) */
    const int32_t* user_perm; /* optional ordering (new -> old) replacing nested dissection */
    int32_t precision;        /* enum spx_precision */
    int32_t ir_max_iter;      /* refinement steps after the first solve; -1 (default):
                               * 2 for SPX_FP64, 10 for the FP32-storage modes */
    double ir_tol;            /* componentwise backward error target (1e-14) */
    int32_t trace;            /* 1: record a per-work-item trace of each factorization (0) */
    int32_t graph;            /* 1: capture the device work of a factorization in a HIP graph
                               * once and replay it for every later factorization (0) */
    int32_t tune;             /* 1: on the first factorization, time one run per work
                               * decomposition (update tile shape, priority policy) and
                               * keep the fastest (0: 256x64 tiles, every chain first) */
    int32_t tile;             /* update tile shape without tuning: 0 = 256 x 64, 1 = 128 x 128 (0) */
    int32_t fuse_small;       /* 1: a column block of width <= 32 with at most 128 panel rows
                               * (and at most 64 update tiles) is factored, solved and
                               * scattered as one work item (1) */
    int32_t merge_split;      /* 1..16: the updates of up to this many consecutive pieces of a
                               * split supernode into a block outside it, or into a piece of it
                               * at least two past the group, are one work item (inner
                               * dimension summed over the pieces, one scatter); 1 = off (4) */
    double static_pivot_eps;  /* SPX_LDLT and SPX_LU (Section III's static pivoting: no row or
                               * column exchange): a pivot p with |p| < eps * max|a_ij| (over
                               * the entries read) is replaced by +eps * max|a_ij| with the sign
                               * of p (+ for p = 0) and counted in spx_info.pivots_replaced;
                               * 0: no replacement (a zero or non-finite pivot is SPX_ENOTPD);
                               * -1 (default): sqrt of the unit roundoff of the factor's
                               * precision (2^-26.5 for SPX_FP64, 2^-12 for the FP32-storage
                               * modes).  A non-finite pivot is never replaced.  Ignored by
                               * SPX_LLT. */
    int32_t deterministic;    /* 1: the updates into one column block are applied in ascending
                               * order of their source block (Section III: the runtimes
                               * serialize the tasks writing one panel; here the order is
                               * fixed), so the factor is the same bit for bit on every run
                               * of one analysis; fused small items are off in this mode.
                               * 0 (default): concurrent updates into one block in any order
                               * (FP64 atomics; factors agree to rounding).  The solve's
                               * scatter is in any order in both modes. */
} spx_options;

typedef struct spx_info {
    int32_t n;
    int32_t ncblk;            /* column blocks after splitting */
    int32_t nblok;            /* blocks, diagonal blocks included */
    int32_t nsnode;           /* supernodes after amalgamation */
    int64_t nnz_a;            /* entries of the input pattern */
    int64_t nnz_l;            /* exact nonzeros of L (column counts summed) */
    int64_t nnz_l_stored;     /* nonzeros of the block structure (after amalgamation) */
    int64_t panel_entries;    /* size of the panel storage (diagonal blocks stored square) */
    double flops_alg;         /* sum of squared exact column counts eta_j (SPX_LU: sum of
                               * 2 (eta_j - 1)^2 + (eta_j - 1)) */
    double flops_exec;        /* the same on the amalgamated structure */
    int64_t ntasks;           /* device scheduler work items per factorization */
    int32_t fail_col;         /* after SPX_ENOTPD: failing column, original numbering */
    int32_t factorized;       /* 1 once a factorization succeeded */
    double logdet;            /* log det A after a factorization (SPX_LDLT, SPX_LU: log |det A|) */
    double factor_kernel_ms;  /* last factorization: scheduler kernel time (HIP events) */
    double assemble_ms;       /* last factorization: assembly kernel time */
    int32_t tile_rows;        /* update tile in use: 256 x 64 or 128 x 128 */
    int32_t tile_cols;
    int32_t hp_policy;        /* 0: every elimination chain first; 1: only the upper levels */
    int32_t nsys;             /* independent systems of the handle (spx_analyze_batch), 1 otherwise */
    int64_t nfused_tiles;     /* update tiles carried out inside fused items (not in ntasks) */
    int32_t nsmall;           /* column blocks handled as one fused item (fuse_small) */
    int32_t nneg;             /* SPX_LDLT: negative pivots (the inertia's negative count;
                               * sign det A = (-1)^nneg); SPX_LU: negative u_jj (sign det
                               * A = (-1)^nneg); 0 for SPX_LLT */
    int32_t pivots_replaced;  /* SPX_LDLT, SPX_LU: pivots replaced by static pivoting in the
                               * last factorization (see static_pivot_eps) */
    int32_t solve_levels;     /* dependency levels of each triangular sweep */
    int32_t solve_pairs;      /* pairs of consecutive pieces of split supernodes solved as one
                               * block in the sweeps (on levels of at most 16 blocks): each
                               * pair's inverse is formed after the factorization */
} spx_info;

typedef struct spx_solve_info {
    int32_t ir_iters;         /* refinement steps taken */
    int32_t converged;        /* omega <= ir_tol */
    double omega;             /* componentwise backward error max_i |b-Ax|_i / (|A||x|+|b|)_i */
    double eta;               /* normwise backward error */
} spx_solve_info;

/* Read-only views of the symbolic structure, valid until spx_destroy.
 * Column blocks ("cblk") are ranges of consecutive columns in the new
 * numbering; each owns a dense column-major panel with leading dimension
 * stride[k]: the w x w diagonal block first, then its off-diagonal blocks. */
typedef struct spx_symbolic_view {
    int32_t n, ncblk, nblok, nsnode, nupd;
    const int32_t* perm;      /* [n] new -> old */
    const int32_t* iperm;     /* [n] old -> new */
    const int32_t* etree;     /* [n] column elimination tree, new numbering, -1 = root */
    const int32_t* snptr;     /* [nsnode+1] first column of every supernode */
    const int32_t* fcol;      /* [ncblk] first column */
    const int32_t* lcol;      /* [ncblk] last column (inclusive) */
    const int32_t* stride;    /* [ncblk] rows of the panel */
    const int64_t* panel_off; /* [ncblk+1] offset of the panel in the factor storage */
    const int32_t* bptr;      /* [ncblk+1] first block of each cblk (its diagonal block) */
    const int32_t* cparent;   /* [ncblk] first facing cblk, -1 if none */
    const int32_t* frow;      /* [nblok] first row */
    const int32_t* lrow;      /* [nblok] last row (inclusive) */
    const int32_t* fcblk;     /* [nblok] facing cblk (whose columns hold these rows) */
    const int32_t* coefind;   /* [nblok] row offset inside the owning panel */
    const int32_t* uptr;      /* [ncblk+1] update targets of cblk k: utgt[uptr[k]..uptr[k+1]) */
    const int32_t* utgt;      /* [nupd] facing cblks, ascending */
    const int32_t* dep;       /* [ncblk] number of cblks updating each cblk */
} spx_symbolic_view;

/* Opaque problem handle: symbolic plan, device task tables, factor. */
typedef struct spx_handle spx_handle;

/* Fill *opt with the defaults listed above. */
void spx_default_options(spx_options* opt);

/* Ordering and symbolic analysis on the host (Section III).  Inputs are host
 * pointers, copied and not retained.  opt may be NULL (defaults).  On success
 * *out owns all host and device memory of the problem (the plan is uploaded
 * to the current HIP device).  Errors: SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE. */
int spx_analyze(int32_t n, const int64_t* colptr, const int32_t* rowind,
                const spx_options* opt, spx_handle** out);

/* Batch of independent systems A_q x_q = b_q (q < nsys, sizes n[q], patterns
 * colptr[q] / rowind[q] as for spx_analyze) analysed as one block-diagonal
 * system: every later call on the handle treats them together, so one
 * factorization launch (one persistent scheduler kernel; with the graph
 * option, one graph replay) factors all of them.  Values and right-hand
 * sides are the systems' arrays concatenated in order (system q's values
 * follow those of systems < q; its unknowns are rows off_q .. off_q + n[q] - 1
 * with off_q = n[0] + ... + n[q-1]).  opt->user_perm must be NULL.
 * Errors: as spx_analyze. */
int spx_analyze_batch(int32_t nsys, const int32_t* n, const int64_t* const* colptr,
                      const int32_t* const* rowind, const spx_options* opt, spx_handle** out);

/* Numerical factorization (Section III and V: diagonal factorization,
 * panel triangular solve, sparse-GEMM updates scattered into the facing
 * panels), scheduled on the GPU by a device-side ready queue.
 * values: colptr[n] doubles aligned with the analysed pattern; a device
 * pointer if values_on_device, else a host pointer; not retained.
 * Errors: SPX_ESTATE (no analysis), SPX_ENOTPD (fail_col in spx_info),
 * SPX_EDEVICE.  May be called again with new values. */
int spx_factorize(spx_handle* h, const double* values, int32_t values_on_device, void* hip_stream);

/* Solve A X = B for nrhs right-hand sides stored column-major with leading
 * dimension ldb >= n; B is overwritten with X.  b is a device pointer if
 * b_on_device, else a host pointer.  Runs the forward and backward sweeps,
 * then FP64 refinement until omega <= ir_tol, ir_max_iter steps, or
 * stagnation (omega above half its previous value in two consecutive steps).
 * info may be NULL.  Errors: SPX_ESTATE, SPX_EINVAL, SPX_ENOCONV, SPX_EDEVICE. */
int spx_solve(spx_handle* h, int32_t nrhs, double* b, int64_t ldb, int32_t b_on_device,
              spx_solve_info* info, void* hip_stream);

/* Allocation-free variant of spx_solve, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same result and refinement as spx_solve; b is a
 * device pointer (n x nrhs, column-major, leading dimension ldb >= n),
 * overwritten with x.  The work vectors live in a fixed array of 64 MiB per
 * device inside the library (set up by spx_analyze on the handle's device and
 * held until the process ends), not in allocations: 7 * n * nrhs doubles
 * (each vector rounded up to 256 bytes) plus 1280 bytes must fit, i.e. n *
 * nrhs up to about 1.19e6; larger calls return SPX_EINVAL before any device
 * work.  The sweeps are launched one by one (no graph).  Every call on a
 * device shares that device's array and leaves its contents behind: calls
 * that overlap on one device (two threads, or two streams not ordered with
 * each other) race and must be serialized by the caller.  The current
 * device must be the handle's.  Errors: as spx_solve. */
int spx_solve_noalloc(spx_handle* h, int32_t nrhs, double* b, int64_t ldb, spx_solve_info* info,
                      void* hip_stream);

/* Adjoint of the solve (x = A^{-1} b): gradient of a loss with respect to
 * the values passed to spx_factorize, given x and db = A^{-T} xbar (for
 * symmetric A, db is spx_solve applied to xbar with the same factor).  The
 * derivative with respect to the matrix is dA = -db x^T summed over the
 * right-hand sides, restricted to the pattern; a stored lower entry a_ij
 * (i > j) stands for both a_ij and a_ji, so
 *   grad[p] = -sum_k (db[i,k] x[j,k] + db[j,k] x[i,k])   for p = (i, j), i > j,
 *   grad[p] = -sum_k db[i,k] x[i,k]                       for i = j,
 *   grad[p] = 0                                           for i < j (not read).
 * x, db: device, n x nrhs column-major with leading dimension ld >= n;
 * grad: device, colptr[n] doubles aligned with the analysed pattern.
 * Errors: SPX_ESTATE (no device plan yet), SPX_EINVAL, SPX_EDEVICE. */
int spx_values_grad(spx_handle* h, int32_t nrhs, const double* x, const double* db, int64_t ld,
                    double* grad, void* hip_stream);

/* Statistics of the analysis and of the last factorization. */
int spx_get_info(const spx_handle* h, spx_info* info);

/* Views of the symbolic arrays (bit-exact comparison with an independent
 * analysis). */
int spx_export_symbolic(const spx_handle* h, spx_symbolic_view* view);

/* Copy the factor panels (panel_entries doubles, layout of the symbolic
 * view; the strict upper triangle of diagonal blocks is zero; SPX_LU:
 * 2 * panel_entries doubles, the L panels then the U^T panels) to dst, a host
 * or device pointer.  An FP32 factor is widened to FP64.  Errors: SPX_ESTATE
 * before a factorization. */
int spx_copy_factor(spx_handle* h, double* dst, int32_t dst_on_device, void* hip_stream);

/* Task trace of the last factorization (trace option on): 4 int64 per work
 * item in dst {claimed, started, finished: device wall-clock ticks; hardware
 * id register of the executing wave}, and, if kinds is not NULL, 4 int32 per
 * item {kind 0 factor / 1 triangular solve / 2 update / 3 fused small block /
 * 4 off-diagonal tiles of a chain block's inverse,
 * source cblk, target cblk, rows*cols of an update tile or rows of a solve
 * tile}.  cap = number of items dst can hold (info.ntasks).  Returns the
 * item count, or a negative status. */
int64_t spx_get_trace(spx_handle* h, int64_t* dst, int64_t cap, int32_t* kinds);

/* Update-kernel microbenchmark (Section V-B's study of the update kernel:
 * C = C - A B^T with B the first k rows of A, into a dense or a gapped
 * target panel, over many calls on one or several streams).  Runs the
 * scheduler's update tiles (the same device code; 256 x 64 tiles, or
 * 128 x 128 with tile = 1) of one synthetic source panel into one target
 * panel, calls times, and returns the elapsed time in *ms (HIP events).
 *   precision: SPX_FP64 (double panels), SPX_FP32_IR (float panels, FP32
 *     products) or SPX_BF16X3_IR (float panels, split-BF16 products);
 *   method: SPX_LLT, or SPX_LDLT (C = C - A D B^T, D the diagonal of the
 *     source panel's diagonal block);
 *   panels: device array of the element type holding the source panel at
 *     offset 0 (column-major, leading dimension n_inner + m, n_inner columns:
 *     an n_inner x n_inner diagonal block, then the m rows of A) and the
 *     target panel at offset (n_inner + m) * n_inner (column-major, leading
 *     dimension ldc >= m, k columns);
 *   rmap: device int32[m], the target row of source row i of A: rmap[i] = i
 *     for i < k (the target's columns), then increasing values in [k, ldc)
 *     (checked; a dense target has rmap[i] = i and ldc = m);
 *   only the lower triangle of the target's k x k diagonal block is
 *     updated (the factorization's symmetric update);
 *   nstreams: 1..3 = one grid per call, the calls round-robin over that many
 *     streams (default priority); 0 = all calls in one grid.
 * The call is synchronous; the target accumulates every call's update.
 * Returns SPX_OK, SPX_EINVAL (the message in spx_last_error(NULL)),
 * SPX_ENOMEM or SPX_EDEVICE. */
int spx_update_bench(int32_t precision, int32_t method, int32_t n_inner, int32_t m, int32_t k, void* panels,
                     const int32_t* rmap, int32_t ldc, int32_t tile, int32_t calls, int32_t nstreams, double* ms);

/* Free everything owned by the handle.  NULL is allowed. */
void spx_destroy(spx_handle* h);

/* Static description of a status code. */
const char* spx_strerror(int status);

/* Text of the last error raised on h ("" if none); valid until the next call.
 * With h == NULL: the message of the last failed spx_analyze or
 * spx_update_bench of this thread. */
const char* spx_last_error(const spx_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H */
