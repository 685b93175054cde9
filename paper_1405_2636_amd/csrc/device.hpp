// Device-side data of the factorization and solve (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace spx {

// Column-block geometry on the device (all arrays indexed by cblk or block).
struct DevPlan {
    int32_t ncblk;
    const int32_t* fcol;
    const int32_t* lcol;
    const int32_t* stride;
    const int64_t* panel_off;
    const int32_t* bptr;
    const int32_t* frow;
    const int32_t* lrow;
    const int32_t* coefind;
    const int64_t* dinv_off;   // offset of the inverted diagonal tiles of each cblk
};

// Work-item kinds of the device scheduler (low byte of the first word; an
// update keeps its merged piece count - 1 in bits 8..11; bit 12 marks a thin
// TRSM or update item of an elimination chain: 16-row wave tiles).
enum ItemKind : int32_t { kFact = 0, kTrsm = 1, kUpdate = 2, kSmall = 3, kInv = 4 };
constexpr int32_t kThinItem = 1 << 12;
constexpr int32_t kSubstItem = 1 << 13;   // TRSM of a chain block: substitution with the diagonal tiles of D

// Two int4 per item: {kind, k, a, b}, {c, d, e, f}
//   kFact:   k
//   kTrsm:   k, row0 = first panel row, nrows (<= 64 * (4 / ceil(w / 64)); thin: 16 * ...)
//   kUpdate: k (source), j (target), row0 (first source panel row);
//            mrows, col0 (first facing panel row), ncols, mbase (row-map base)
//   kSmall:  k; first tile of k in the fused-tile table, tile count, first
//            row-map entry of k, row-map entries of k
//   kInv:    k (the off-diagonal tiles of L_kk^{-1} after a FACT that left them)
// Fused-tile table: three int4 per update tile of a fused block,
//   {j, row0, mrows, col0}, {ncols, mbase, stride of j, 0},
//   {panel offset of j: low word, high word, 0, 0}
struct SchedArgs {
    DevPlan pl;
    void* panels;            // double, or float in the FP32 refinement modes
    void* dinv;              // same element type as the panels
    int32_t split;           // FP32 panels: update and TRSM products as split-BF16 products
    int32_t ldlt;            // L D L^T (FP64): D on the panels' diagonals, inverse D^{-1} L^{-1}
    int64_t upanel;          // L U: elements from the L panels to the U^T panels (same layout)
    int64_t uinv;            // L U: elements from the inverses L_kk^{-1} to U_kk^{-T} (same layout)
    const int4* desc;
    const int32_t* rmap;     // panel row of k -> row inside panel j, per update pair
    const int4* ftab;        // update tiles of fused small blocks
    int32_t hp_total;        // items of the high-priority queue (FACT, TRSM, chain updates)
    int32_t total_normal;    // items of the normal queue (other updates)
    const int32_t* trsm_first;
    const int32_t* trsm_count;
    const int32_t* upd_first;
    const int32_t* upd_hp;   // leading update items of a cblk that go to the high-priority queue
    const int32_t* upd_count;
    const int32_t* hp_cblk;  // 1 if the items of the cblk go to the high-priority queue
    int32_t* fact_dep;
    int32_t* trsm_left;
    int32_t* queue;
    int32_t* qhead;
    int32_t* qtail;
    int32_t* hp_queue;
    int32_t* hp_head;
    int32_t* hp_tail;
    int32_t* status;        // [kStFail] smallest failing column, [kStAbort] abort flag, [kStDone] items done,
                            // [kStReplaced] pivots replaced (static pivoting), [kStAmax] max |a_ij| (2 words)
    double pivot_eps;       // L D L^T, L U: replace pivots below pivot_eps * max |a_ij| (0: off)
    // Deterministic mode (npair > 0): the update items of one (source,
    // target) pair are released when the source's panel solves are done and
    // the previous pair into the same target (ascending source) has finished.
    // Blocks of elimination chains (L L^T): FACT leaves the off-diagonal tiles
    // of the inverse to an INV item, released with the panel solves (which
    // use the diagonal tiles only) and off the chain.
    const int32_t* inv_item;   // INV item of block k, or -1 (FACT computes the whole inverse)
    int32_t npair;          // update pairs (0: any-order mode)
    int32_t ubase;          // id of the first update item
    const int32_t* upair;   // pair of update item ubase + i
    const int32_t* kpair;   // pairs of source k: kpair[k] .. kpair[k + 1] - 1
    const int4* pairs;      // {first item, item count, next pair into the same target (-1: none), high priority}
    const int32_t* pdep0;   // initial pair dependency counts (1, or 2 with a previous pair)
    int32_t* pdep;          // pair dependency counters
    int32_t* pleft;         // unfinished items per pair
    int64_t timeout_ticks;  // wall-clock ticks a worker may wait for work
    int64_t* trace;         // optional: 4 words per item {claimed, started, finished, hw id}
};

// Arguments of the triangular sweeps.
struct SweepArgs {
    DevPlan pl;
    const void* panels;       // double, or float in the FP32 refinement mode
    const void* dinv;
    const void* panels_b;     // backward sweep: L U's U^T panels and U_kk^{-T} (else the same as forward)
    const void* dinv_b;
    int32_t f32;              // 1: panels and inverses are float
    int32_t ldlt;             // 1: L D L^T factor (D on the panel diagonals, inverses D^{-1} L^{-1})
    const int32_t* rowg;      // global row of every off-diagonal panel row
    const int64_t* rowg_off;  // [ncblk] start of cblk k's rows in rowg
    double* y;                // permuted right-hand side, accumulates the forward updates (n x nrhs, ld n)
    double* z;                // forward sweep result L^{-1} P b
    double* x;                // backward sweep result L^{-T} z
    double* tacc;             // backward partial sums
    int32_t n;
    int32_t nrhs;
};

// Work items of the sweeps, built once per analysis.  Each holds everything
// its workgroup needs to address its part of the factor and the vectors,
// so that the loads of the panel, the kept inverse and the vectors go out
// together after one scalar load of the item (instead of behind a chain of
// dependent loads through the plan arrays).
struct DiagItem {          // rows (forward) or columns (backward) r0 .. of the diagonal block of a unit
    int64_t dofs;          // start of the unit's kept inverse (w x w, column-major)
    int64_t pofs;          // start of the (first) block's panel: L D L^T d_c at pofs + c * (ld + 1), c < w1
    int64_t pofs2;         // a pair's second piece's panel: d_c at pofs2 + (c - w1) * (ld2 + 1), c >= w1
    int32_t f, w, r0, ld;  // first column, width, first row of the part, panel stride of the first block
    int32_t w1, ld2;       // width of the first block (w for a single block), panel stride of the second
};
struct OffItem {           // panel rows row0 .. row0 + nr - 1 of k by the columns c0 .. c1 - 1
    int64_t pofs;          // panel element (row0, 0) of k
    int64_t gofs;          // position of panel row row0's global row in the row list
    int32_t ld, f, row0;   // panel stride, first column of k, first panel row
    int32_t cnr;           // c0 | c1 << 9 | nr << 18 (widths are at most 256, nr at most 256)
};

// Two consecutive pieces p, q of a split supernode solved as one block in
// the sweeps: the pair's inverse [[D_p, 0], [X, D_q]] with
// X = -D_q L_qp D_p (the inverse of the block lower-triangular diagonal
// block of the pair; D_p, D_q the pieces' kept inverses, L_qp the rows of
// p's panel that face q), stored column-major with leading dimension
// W = w_p + w_q after the pieces' own inverses.
constexpr int kMaxPairWidth = 512;   // widest diagonal block of the sweeps (a pair of pieces)
struct PairItem {
    int64_t lofs;          // panel element (w_p, 0) of p: L_qp, w_q x w_p, stride ldp
    int64_t dp, dq;        // kept inverses of p and q
    int64_t out;           // the pair's inverse
    int32_t ldp, wp, wq, pad;
};

// Scheduler counters and status words sit 256 bytes apart: every worker
// polls the queue heads and the abort flag, and a shared line would put the
// polls in the way of the claims.
constexpr int kCtrStride = 64;                 // int32 words between counters
constexpr int kStFail = 0, kStAbort = kCtrStride, kStDone = 2 * kCtrStride, kStReplaced = 3 * kCtrStride,
              kStAmax = 4 * kCtrStride;
constexpr int kStatusWords = 5 * kCtrStride;

// Column blocks factored as one fused item: width <= kNB, at most
// kSmallRows panel rows, at most kSmallMaxUpd update tiles and kSmallMap
// row-map entries (bounds of the item's LDS tables).
constexpr int kSmallRows = 128;
constexpr int kSmallMaxUpd = 64;
constexpr int kSmallMap = 2048;

// Residual statistics: one 256-byte line per statistic (five of them),
// filled by a fixed grid of blocks.
constexpr int kStatStride = 32;   // u64 words between statistics
constexpr int kResidualBlocks = 1024;

// Fixed work memory of the allocation-free solve, per device (bytes).
constexpr size_t kScratchBytes = size_t(64) << 20;

constexpr int kThreads = 256;   // 4 waves of 64
constexpr int kTile = 64;       // rows/cols of update, triangular-solve tiles
constexpr int kNB = 32;         // diagonal tile (inverted explicitly)

}  // namespace spx
