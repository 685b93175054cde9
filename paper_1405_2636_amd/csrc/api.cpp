// C ABI of the solver (declared in include/spx.h): handle life cycle, upload
// of the symbolic plan, construction of the device task tables and level
// lists, and the host drivers of factorization, solve and refinement.
#include "../../include/spx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device.hpp"
#include "plan.hpp"

namespace spx {

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_assemble(void* panels, bool f32, const int64_t* amap, const double* values, int64_t nnz,
                           hipStream_t s);
hipError_t launch_widen(double* dst, const float* src, int64_t n, hipStream_t s);
hipError_t launch_gather_diag(double* dst, const void* panels, bool f32, const int64_t* off, int64_t n, hipStream_t s);
hipError_t launch_sched_init(const SchedArgs& a, const int32_t* ready, int32_t nready, int32_t nready_hp,
                             const int32_t* fact_dep0, int32_t ncblk, hipStream_t s);
int sched_blocks_per_cu(bool f32, bool ldlt, bool lu);
hipError_t launch_sched(const SchedArgs& a, bool f32, bool lu, int grid, hipStream_t s);
hipError_t launch_update_bench(const SchedArgs& a, bool f32, bool ldl, const int4* tiles, int ntiles, int mbase,
                               int copies, hipStream_t s);
hipError_t launch_fwd_diag(const SweepArgs& a, const DiagItem* items, int count, int lanes, hipStream_t s);
hipError_t launch_fwd_off(const SweepArgs& a, const OffItem* items, int count, hipStream_t s);
hipError_t launch_bwd_off(const SweepArgs& a, const OffItem* items, int count, bool tall, hipStream_t s);
hipError_t launch_bwd_diag(const SweepArgs& a, const DiagItem* items, int count, int lanes, hipStream_t s);
hipError_t launch_pair_inv(const void* panels, void* dinv, bool f32, bool ldlt, const PairItem* items, int count,
                           int maxnb, hipStream_t s);
hipError_t launch_fwd_small(const SweepArgs& a, const int32_t* cblks, int count, hipStream_t s);
hipError_t launch_bwd_small(const SweepArgs& a, const int32_t* cblks, int count, hipStream_t s);
hipError_t launch_permute_in(double* y, const double* b, int64_t ldb, const int32_t* perm, int32_t n, int32_t nrhs,
                             hipStream_t s);
hipError_t launch_permute_out(double* x, int64_t ldx, const double* y, const int32_t* perm, int32_t n, int32_t nrhs,
                              hipStream_t s);
hipError_t launch_axpy(double* x, const double* d, int64_t n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_values_grad(const int32_t* erow, const int32_t* ecol, int64_t nnz, const double* x, const double* db,
                              int64_t ld, int32_t nrhs, double* grad, hipStream_t s);
hipError_t launch_residual(const int64_t* rptr, const int32_t* rcol, const double* rv, const double* x,
                           const double* b, int64_t ldb, double* r, int32_t n, int32_t nrhs,
                           unsigned long long* stats, hipStream_t s);
hipError_t launch_gather(double* rv, const double* vals, const int64_t* idx, int64_t m, hipStream_t s);
hipError_t launch_absmax(const int64_t* amap, const double* values, int64_t nnz, int32_t* status, hipStream_t s);
hipError_t scratch_region(void** ptr, size_t* bytes);

struct DeviceError : std::runtime_error {
    explicit DeviceError(const std::string& s) : std::runtime_error(s) {}
};
struct StatusError : std::runtime_error {
    int code;
    StatusError(int c, const std::string& s) : std::runtime_error(s), code(c) {}
};

#define HIPCHK(expr)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) throw DeviceError(std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

// Owned device allocation.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count)
    {
        if (count <= n && p) return;
        release();
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (hipMalloc(reinterpret_cast<void**>(&p), bytes) != hipSuccess) {
            p = nullptr;
            throw std::bad_alloc();
        }
        n = count;
    }
    void upload(const std::vector<T>& v)
    {
        alloc(v.size());
        if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
};

struct Level {
    std::vector<int32_t> cptr;   // cblks of level l: cblk[cptr[l]..cptr[l+1])
    std::vector<int32_t> cblk;   // (each level's small blocks first: cblk[cptr[l]..cptr[l]+nsmall[l]))
    std::vector<int32_t> nsmall; // blocks of width <= 32 with at most 128 panel rows, per level
    std::vector<int32_t> dptr;   // diagonal items of level l: ditem[dptr[l]..dptr[l+1])
    std::vector<DiagItem> ditem;
    std::vector<uint8_t> narrow; // level l holds fewer than 64 blocks (its sweep items are cut finer)
    std::vector<uint8_t> dlanes; // lanes per row of level l's diagonal items (4, 16 or 32; 256 / lanes rows each)
    std::vector<int32_t> kptr;   // off-diagonal items of level l: chunk[kptr[l]..kptr[l+1])
    std::vector<OffItem> chunk;
    std::vector<int32_t> kptr1;  // one right-hand side: every chunk cut into 64-column items, chunk1[..]
    std::vector<OffItem> chunk1;
    std::vector<int32_t> bptr;   // narrow levels: the backward sweep's own 256-row items, bchunk[bptr[l]..bptr[l+1])
    std::vector<OffItem> bchunk;
    std::vector<PairItem> pair;  // paired pieces (one unit of the sweeps each)
    int32_t maxnb = 0;           // widest pair in 16-column blocks, plus one
};

}  // namespace spx

using namespace spx;

struct spx_handle {
    Plan plan;
    spx_options opt{};
    std::string err;
    int32_t n = 0;
    int64_t nnz = 0;
    // device plan
    DevBuf<int32_t> fcol, lcol, stride, bptr, frow, lrow, coefind, perm;
    DevBuf<int64_t> panel_off, dinv_off;
    DevBuf<int64_t> diag_off;   // panel offset of the diagonal entry of every column
    DevBuf<int64_t> amap, rptr, rval;
    DevBuf<int32_t> rcol;
    DevBuf<int32_t> erow, ecol;   // row and column of every stored entry (-1: above the diagonal)
    DevBuf<int32_t> rowg;
    DevBuf<int64_t> rowg_off;
    // scheduler tables
    int32_t total = 0, nready = 0, nready_hp = 0, hp_total = 0, total_normal = 0;
    int32_t nsmall = 0, nfused_tiles = 0;   // fused small blocks and their update tiles
    DevBuf<int4> desc;
    DevBuf<int32_t> rmap;
    DevBuf<int32_t> trsm_first, trsm_count, upd_first, upd_hp, upd_count, hp_cblk, fact_dep0, fact_dep, trsm_left,
        queue, hp_queue, ready, qctr, status;
    DevBuf<int4> ftab;
    // deterministic mode: update pairs (see SchedArgs)
    int32_t npair = 0, ubase = 0;
    int32_t ninv = 0;                 // INV items (chain blocks, L L^T)
    DevBuf<int32_t> inv_item;
    DevBuf<int32_t> upair, kpair, pdep0, pdep, pleft;
    DevBuf<int4> pairs;
    DevBuf<int64_t> trace;   // per-item task trace, allocated when the trace option is on
    // levels for the sweeps
    Level lv;
    DevBuf<int32_t> lv_cblk;
    DevBuf<DiagItem> lv_ditem;
    DevBuf<OffItem> lv_chunk, lv_chunk1;
    DevBuf<OffItem> lv_bchunk;
    DevBuf<PairItem> lv_pair;
    // numeric: FP64 panels and inverses, or their FP32 counterparts
    DevBuf<double> panels, dinv, vals, rv;   // rv: values in the order of the residual's row lists
    DevBuf<float> panels_f, dinv_f;
    int64_t dinv_size = 0;
    bool factorized = false;
    int32_t fail_col = -1;
    bool logdet_valid = false;
    double logdet = 0.0;
    int32_t nneg = 0;   // L D L^T: negative pivots
    int32_t nrep = 0;   // L D L^T, L U: pivots replaced by static pivoting (last factorization)
    double factor_ms = 0.0, assemble_ms = 0.0;
    // solve work (internal buffers, n x nrhs_cap) and the captured sweep graph
    DevBuf<double> y, zv, xv, tacc, xw, rw, dw, bw;
    DevBuf<unsigned long long> stats;
    int32_t nrhs_cap = 0;
    int32_t graph_nrhs = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // work decomposition (chosen by the tuner when the tune option is on)
    int32_t tile_rows = 256, tile_cols = 64;   // update tile: 256 x 64, or 128 x 128
    int32_t hp_policy = 0;                     // 0: every chain high priority; 1: only levels of <= 32 blocks
    int32_t nsys = 1;                          // independent systems (spx_analyze_batch)
    bool tuned = false;
    // captured factorization sequence (graph option): assembly + queue set-up,
    // and the scheduler kernel (two graphs, timed by events between them)
    hipGraph_t fgraph[2] = {nullptr, nullptr};
    hipGraphExec_t fgraph_exec[2] = {nullptr, nullptr};
    int device = 0;
    int grid = 0;
    // the fixed work array of the allocation-free solve on this handle's
    // device (device address, from scratch_region at the plan upload)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    int64_t timeout_ticks = 0;
    bool uploaded = false;

    ~spx_handle()
    {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        drop_graph();
        drop_fgraph();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    void drop_fgraph()
    {
        for (int i = 0; i < 2; ++i) {
            if (fgraph_exec[i]) (void)hipGraphExecDestroy(fgraph_exec[i]);
            if (fgraph[i]) (void)hipGraphDestroy(fgraph[i]);
            fgraph_exec[i] = nullptr;
            fgraph[i] = nullptr;
        }
    }

    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_nrhs = 0;
    }

    bool f32() const { return opt.precision != SPX_FP64; }   // FP32 panel storage
    bool ldlt() const { return opt.method == SPX_LDLT; }     // L D L^T (D on the panel diagonals)
    bool lu() const { return opt.method == SPX_LU; }         // L U: L panels, then U^T panels (same layout)
    int64_t panel_count() const { return plan.panel_entries * (lu() ? 2 : 1); }
    int64_t dinv_count() const { return dinv_size * (lu() ? 2 : 1); }
    void* panel_ptr() { return f32() ? static_cast<void*>(panels_f.p) : static_cast<void*>(panels.p); }
    void* dinv_ptr() { return f32() ? static_cast<void*>(dinv_f.p) : static_cast<void*>(dinv.p); }

    DevPlan devplan() const
    {
        DevPlan d;
        d.ncblk = plan.ncblk;
        d.fcol = fcol.p;
        d.lcol = lcol.p;
        d.stride = stride.p;
        d.panel_off = panel_off.p;
        d.bptr = bptr.p;
        d.frow = frow.p;
        d.lrow = lrow.p;
        d.coefind = coefind.p;
        d.dinv_off = dinv_off.p;
        return d;
    }
};

namespace {

thread_local std::string g_analyze_err;   // message of the last failed handle-less call in this thread

int fail(spx_handle* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    return code;
}

template <class F>
int guarded(spx_handle* h, F&& f)
{
    try {
        return f();
    } catch (const InvalidArgument& e) {
        return fail(h, SPX_EINVAL, e.what());
    } catch (const std::bad_alloc&) {
        return fail(h, SPX_ENOMEM, "out of memory");
    } catch (const StatusError& e) {
        return fail(h, e.code, e.what());
    } catch (const DeviceError& e) {
        return fail(h, SPX_EDEVICE, e.what());
    } catch (const std::exception& e) {
        return fail(h, SPX_EDEVICE, e.what());
    } catch (...) {
        return fail(h, SPX_EDEVICE, "unknown error");
    }
}

// Work items of the device scheduler, in id order: FACT(k) = k, then per cblk
// its TRSM row tiles (64 rows), then per cblk its UPDATE tiles.  The update
// tiles of a pair (k, j) are 256 rows by 64 facing columns; tiles entirely
// in the strict upper
// triangle of j's diagonal block are not generated.  The tiles into the
// first facing cblk (the next block of an elimination chain) come first and
// go to the high-priority queue, like FACT and TRSM items.
// rmap holds, per update pair, the row inside panel j of every panel row of
// k from the first facing row on (checked against the target structure).
void build_tasks(spx_handle* h)
{
    const Plan& P = h->plan;
    const int32_t nc = P.ncblk;
    constexpr int kTrsmRows = 64;
    constexpr int kChainLevel = 1;
    // high priority: FACT, the TRSM tiles and the update tiles into the first
    // facing block (the elimination chain) of every block, or (policy 1) of
    // the blocks in dependency levels of at most 32 blocks only; the other
    // update tiles form the bulk in the normal queue
    std::vector<int32_t> hp(nc, 1);
    // dependency levels (level(j) = 1 + max level of the blocks updating j)
    std::vector<int32_t> lvl(nc, 0), per_level(static_cast<size_t>(nc) + 1, 0);
    for (int32_t k = 0; k < nc; ++k)
        for (int32_t q = P.uptr[k]; q < P.uptr[k + 1]; ++q)
            lvl[P.utgt[q]] = std::max(lvl[P.utgt[q]], lvl[k] + 1);
    for (int32_t k = 0; k < nc; ++k) ++per_level[lvl[k]];
    if (h->hp_policy == 1)
        for (int32_t k = 0; k < nc; ++k) hp[k] = per_level[lvl[k]] <= 32 ? 1 : 0;
    // elimination chains: a block of width >= 128 in a level of at most
    // kChainLevel blocks (the top separators' pieces, factored one after the
    // other while most of the GPU waits) takes thin TRSM items and thin
    // update tiles into its first facing block: a quarter of the work per
    // wave, four times as many items side by side, a shorter chain link
    std::vector<char> chain(nc, 0);
    for (int32_t k = 0; k < nc; ++k)
        chain[k] = per_level[lvl[k]] <= kChainLevel && P.lcol[k] - P.fcol[k] + 1 >= 128;
    // L L^T blocks of width >= 128 in levels of at most kInvLevel blocks
    // (high priority): FACT stores L_kk and the diagonal tiles of its inverse
    // only, the panel solves are block substitutions with those tiles (64
    // rows, 16 per wave), and an INV item in the normal queue forms the rest
    // of the inverse (needed by the triangular sweeps only): the chain runs
    // through about half the FACT products and none of the inverse's
    constexpr int kInvLevel = 4;
    std::vector<char> inv(nc, 0);
    for (int32_t k = 0; k < nc; ++k)
        inv[k] = h->opt.method == SPX_LLT && hp[k] && per_level[lvl[k]] <= kInvLevel && P.lcol[k] - P.fcol[k] + 1 >= 128;
    // update tiles of source k into target group [b, b2) (blocks facing one
    // cblk), tr x tcl each
    auto for_tiles = [&](int32_t k, int32_t b, int32_t b2, int32_t tr, int32_t tcl, auto&& fn) {
        const int32_t ld = P.stride[k];
        const int32_t rs = P.coefind[b];
        const int32_t re = P.coefind[b2 - 1] + (P.lrow[b2 - 1] - P.frow[b2 - 1] + 1);
        for (int32_t r0 = rs; r0 < ld; r0 += tr) {
            const int32_t mr = std::min(tr, ld - r0);
            for (int32_t c0 = rs; c0 < re; c0 += tcl) {
                if (r0 + mr - 1 < c0 && !h->lu()) continue;   // strictly above the diagonal of j (L U: whole square)
                fn(r0, mr, c0, std::min(tcl, re - c0));
            }
        }
    };
    // fused small blocks: width <= 32, at most 128 panel rows, tables within
    // the bounds of the item's LDS
    std::vector<char> small(nc, 0);
    int32_t nsmall = 0;
    if (h->opt.fuse_small) {
        for (int32_t k = 0; k < nc; ++k) {
            const int32_t w = P.lcol[k] - P.fcol[k] + 1, ld = P.stride[k];
            if (w > kNB || ld > kSmallRows) continue;
            int64_t ntiles = 0, nmap = 0;
            for (int32_t b = P.bptr[k] + 1; b < P.bptr[k + 1];) {
                int32_t b2 = b;
                while (b2 < P.bptr[k + 1] && P.fcblk[b2] == P.fcblk[b]) ++b2;
                nmap += ld - P.coefind[b];
                for_tiles(k, b, b2, h->tile_rows, h->tile_cols, [&](int32_t, int32_t, int32_t, int32_t) { ++ntiles; });
                b = b2;
            }
            if (ntiles <= kSmallMaxUpd && nmap <= kSmallMap) {
                small[k] = 1;
                ++nsmall;
            }
        }
    }
    // merged updates of split supernodes: the pieces of a supernode are
    // consecutive column blocks sharing the rows below the supernode, and
    // piece p's panel rows are the rows of a later piece k shifted by
    // fcol[k] - fcol[p].  The updates of a group of up to merge_split
    // consecutive pieces into a block outside their supernode, or into a
    // piece at least two past the group, are one item of the group's last
    // piece (the inner dimension spans the group).  The pieces of the group
    // and the next one are updated piece by piece: they are factored one
    // after the other, and the next one's factorization then waits for the
    // last piece's update only.
    std::vector<int32_t> snof(nc), gfirst(nc), glid(nc);
    std::vector<char> glast(nc, 1);
    const int32_t G = std::max(1, h->opt.merge_split);
    for (int32_t k = 0; k < nc; ++k)
        snof[k] = static_cast<int32_t>(std::upper_bound(P.snptr.begin(), P.snptr.end(), P.fcol[k]) - P.snptr.begin()) - 1;
    for (int32_t k0 = 0; k0 < nc;) {
        int32_t k1 = k0;
        while (k1 + 1 < nc && snof[k1 + 1] == snof[k0]) ++k1;
        bool any_small = false;
        for (int32_t k = k0; k <= k1; ++k) any_small = any_small || small[k];
        for (int32_t k = k0; k <= k1; ++k) {
            const bool merge = G > 1 && !any_small;
            gfirst[k] = merge ? k0 + ((k - k0) / G) * G : k;
            glast[k] = merge ? (k == k1 || (k - k0 + 1) % G == 0) : 1;
            glid[k] = merge ? std::min(k1, gfirst[k] + G - 1) : k;
            for (int32_t p = gfirst[k]; p < k && glast[k]; ++p)
                if (P.stride[p] != P.stride[k] + (P.fcol[k] - P.fcol[p]))
                    throw std::runtime_error("split pieces without a common row structure");
        }
        k0 = k1 + 1;
    }
    std::vector<int4> desc;
    desc.reserve(static_cast<size_t>(nc) * 2);
    std::vector<int32_t> tf(nc), tc(nc), uf(nc), uh(nc), ucnt(nc), dep(nc, 0);
    std::vector<int32_t> rmap;
    for (int32_t k = 0; k < nc; ++k) {
        desc.push_back(int4{small[k] ? kSmall : kFact, k, 0, 0});
        desc.push_back(int4{0, 0, 0, 0});
    }
    int32_t id = nc;
    for (int32_t k = 0; k < nc; ++k) {
        const int32_t w = P.lcol[k] - P.fcol[k] + 1, ld = P.stride[k];
        tf[k] = id;
        // 64 rows per wave tile (chains: 16); panels narrower than 256
        // columns stack 4/ceil(w/64) of them
        const int32_t trows = inv[k] ? 64 : (chain[k] ? 16 : kTrsmRows) * (4 / ((w + 63) / 64));
        const int32_t tflag = inv[k] ? kSubstItem : (chain[k] ? kThinItem : 0);
        for (int32_t r = w; r < ld && !small[k]; r += trows) {
            desc.push_back(int4{kTrsm | tflag, k, r, std::min(trows, ld - r)});
            desc.push_back(int4{0, 0, 0, 0});
            ++id;
        }
        tc[k] = id - tf[k];
    }
    int64_t nhp_upd = 0;
    std::vector<int4> ftab;   // update tiles of the fused blocks
    std::vector<int32_t> grow;
    // deterministic mode: the update items of one (source, target) pair are
    // consecutive; pairs into one target are chained in ascending source order
    const bool det = h->opt.deterministic != 0;
    const int32_t ubase = id;
    std::vector<int4> pairs;
    std::vector<int32_t> kpair(static_cast<size_t>(nc) + 1, 0), pdep0, upair, plast(nc, -1);
    for (int32_t k = 0; k < nc; ++k) {
        kpair[k] = static_cast<int32_t>(pairs.size());
        const int32_t ld = P.stride[k];
        // global row of every panel row of k
        grow.assign(static_cast<size_t>(ld), 0);
        for (int32_t b = P.bptr[k]; b < P.bptr[k + 1]; ++b)
            for (int32_t r = P.frow[b]; r <= P.lrow[b]; ++r) grow[P.coefind[b] + (r - P.frow[b])] = r;
        uf[k] = id;
        uh[k] = 0;
        const int64_t mstart = static_cast<int64_t>(rmap.size());
        const int32_t ftile0 = static_cast<int32_t>(ftab.size() / 3);
        bool first_pair = true;
        for (int32_t b = P.bptr[k] + 1; b < P.bptr[k + 1];) {
            const int32_t j = P.fcblk[b];
            int32_t b2 = b;
            while (b2 < P.bptr[k + 1] && P.fcblk[b2] == j) ++b2;
            const bool merged = snof[j] != snof[k] || j > glid[k] + 1;
            if (merged && !glast[k]) {   // carried by the group's last piece
                first_pair = false;
                b = b2;
                continue;
            }
            const int32_t npieces = merged ? k - gfirst[k] + 1 : 1;
            const int32_t rs = P.coefind[b];
            const int32_t re = P.coefind[b2 - 1] + (P.lrow[b2 - 1] - P.frow[b2 - 1] + 1);
            const int64_t moff = static_cast<int64_t>(rmap.size());
            if (moff - rs > INT32_MAX - ld) throw std::runtime_error("row map exceeds 2^31 entries");
            for (int32_t r = rs; r < ld; ++r) {
                const int32_t pos = panel_row(P, j, grow[r]);
                if (pos < 0 || (r < re && pos != grow[r] - P.fcol[j]))
                    throw std::runtime_error("update rows outside the target structure");
                rmap.push_back(pos);
            }
            const int32_t mbase = static_cast<int32_t>(moff - rs);
            const bool thin = chain[k] && first_pair && !small[k];
            const int32_t ttr = thin ? 64 : h->tile_rows, ttc = thin ? 64 : h->tile_cols;
            const int32_t pfirst = id;
            for_tiles(k, b, b2, ttr, ttc, [&](int32_t r0, int32_t mr, int32_t c0, int32_t ncl) {
                ++dep[j];
                if (small[k]) {
                    const int64_t po = P.panel_off[j];
                    ftab.push_back(int4{j, r0, mr, c0});
                    ftab.push_back(int4{ncl, mbase, P.stride[j], 0});
                    ftab.push_back(int4{static_cast<int32_t>(po & 0xffffffff), static_cast<int32_t>(po >> 32), 0, 0});
                    return;
                }
                desc.push_back(int4{kUpdate | ((npieces - 1) << 8) | (thin ? kThinItem : 0), k, j, r0});
                desc.push_back(int4{mr, c0, ncl, mbase});
                ++id;
                if (first_pair && hp[k]) ++uh[k];
            });
            if (det && id > pfirst) {
                const int32_t pi = static_cast<int32_t>(pairs.size());
                pairs.push_back(int4{pfirst, id - pfirst, -1, first_pair && hp[k] ? 1 : 0});
                pdep0.push_back(plast[j] >= 0 ? 2 : 1);
                if (plast[j] >= 0) pairs[static_cast<size_t>(plast[j])].z = pi;
                plast[j] = pi;
                upair.resize(static_cast<size_t>(id - ubase), pi);
            }
            first_pair = false;
            b = b2;
        }
        ucnt[k] = id - uf[k];
        nhp_upd += uh[k];
        if (small[k]) {
            const int32_t nt = static_cast<int32_t>(ftab.size() / 3) - ftile0;
            desc[2 * static_cast<size_t>(k) + 1] =
                int4{ftile0, nt, static_cast<int32_t>(mstart), static_cast<int32_t>(rmap.size() - mstart)};
        }
    }
    kpair[nc] = static_cast<int32_t>(pairs.size());
    const int32_t uend = id;   // end of the update items
    std::vector<int32_t> inv_item(nc, -1);
    for (int32_t k = 0; k < nc; ++k)
        if (inv[k] && !small[k]) {
            desc.push_back(int4{kInv, k, 0, 0});
            desc.push_back(int4{0, 0, 0, 0});
            inv_item[k] = id++;
        }
    h->total = id;
    h->npair = static_cast<int32_t>(pairs.size());
    h->ubase = ubase;
    if (det) {
        if (nsmall > 0) throw std::runtime_error("fused small items in the deterministic mode");
        if (static_cast<int64_t>(upair.size()) != uend - ubase) throw std::runtime_error("update items outside pairs");
        h->pairs.upload(pairs);
        h->kpair.upload(kpair);
        h->pdep0.upload(pdep0);
        h->upair.upload(upair);
        h->pdep.alloc(pairs.size());
        h->pleft.alloc(pairs.size());
    }
    h->nsmall = nsmall;
    h->nfused_tiles = static_cast<int32_t>(ftab.size() / 3);
    int64_t hp_items = nhp_upd;
    for (int32_t k = 0; k < nc; ++k)
        if (hp[k]) hp_items += 1 + tc[k];   // (INV items: normal queue)
    h->hp_total = static_cast<int32_t>(hp_items);
    h->total_normal = h->total - h->hp_total;
    std::vector<int32_t> ready;   // high-priority ones first
    for (int32_t k = 0; k < nc; ++k)
        if (dep[k] == 0 && hp[k]) ready.push_back(k);
    h->nready_hp = static_cast<int32_t>(ready.size());
    for (int32_t k = 0; k < nc; ++k)
        if (dep[k] == 0 && !hp[k]) ready.push_back(k);
    h->nready = static_cast<int32_t>(ready.size());
    h->hp_cblk.upload(hp);
    h->desc.upload(desc);
    if (ftab.empty()) ftab.push_back(int4{0, 0, 0, 0});
    h->ftab.upload(ftab);
    h->rmap.upload(rmap);
    h->ninv = 0;
    for (int32_t k = 0; k < nc; ++k) h->ninv += inv_item[k] >= 0 ? 1 : 0;
    h->inv_item.upload(inv_item);
    h->trsm_first.upload(tf);
    h->trsm_count.upload(tc);
    h->upd_first.upload(uf);
    h->upd_hp.upload(uh);
    h->upd_count.upload(ucnt);
    h->fact_dep0.upload(dep);
    h->fact_dep.alloc(nc);
    h->trsm_left.alloc(nc);
    h->queue.alloc(static_cast<size_t>(h->total_normal));
    h->hp_queue.alloc(static_cast<size_t>(h->hp_total));
    h->ready.upload(ready);
    h->qctr.alloc(4 * kCtrStride);
    h->status.alloc(kStatusWords);
}

// Dependency levels for the sweeps: level(k) = 1 + max level of the cblks
// updating k.  Off-diagonal rows are cut into chunks of 64 rows.
// Pairs: on the narrow levels (at most kPairLevel blocks: the elimination
// chains of the split separators, one piece per level), consecutive pieces
// p, q = p + 1 of a split supernode are solved as one block through the
// pair's inverse (built after each factorization): the chain's levels, each
// a diagonal and an off-diagonal launch bound by latency, are halved.  p's
// rows facing q are then covered by the pair's inverse, so p's off-diagonal
// items start below q's rows.
void build_levels(spx_handle* h, const std::vector<int64_t>& doff, const std::vector<int64_t>& rgo)
{
    const Plan& P = h->plan;
    const int32_t nc = P.ncblk;
    auto width = [&](int32_t k) { return P.lcol[k] - P.fcol[k] + 1; };
    auto small = [&](int32_t k) { return width(k) <= kNB && P.stride[k] <= kSmallRows; };
    // levels over units (a unit: a cblk, or a pair led by its first piece)
    std::vector<int32_t> unit(nc);
    for (int32_t k = 0; k < nc; ++k) unit[k] = k;
    auto levels = [&](std::vector<int32_t>& lvl) {
        lvl.assign(nc, 0);
        int32_t nl = nc > 0 ? 1 : 0;
        for (int32_t k = 0; k < nc; ++k) {
            const int32_t uk = unit[k];
            for (int32_t q = P.uptr[k]; q < P.uptr[k + 1]; ++q) {
                const int32_t uj = unit[P.utgt[q]];
                if (uj != uk) lvl[uj] = std::max(lvl[uj], lvl[uk] + 1);
            }
            nl = std::max(nl, lvl[uk] + 1);
        }
        return nl;
    };
    std::vector<int32_t> lvl;
    int32_t nl = levels(lvl);
    std::vector<int32_t> pairs;   // first pieces of the pairs
    if (nc > 1) {
        constexpr int32_t kPairLevel = 16;
        std::vector<int32_t> pop(nl, 0);
        for (int32_t k = 0; k < nc; ++k) ++pop[lvl[k]];
        std::vector<int32_t> snof(nc);
        for (int32_t k = 0; k < nc; ++k)
            snof[k] = static_cast<int32_t>(std::upper_bound(P.snptr.begin(), P.snptr.end(), P.fcol[k]) -
                                           P.snptr.begin()) - 1;
        for (int32_t k0 = 0; k0 < nc;) {
            int32_t k1 = k0;
            while (k1 + 1 < nc && snof[k1 + 1] == snof[k0]) ++k1;
            bool any_small = false;
            for (int32_t k = k0; k <= k1; ++k) any_small = any_small || small(k);
            for (int32_t k = k0; k + 1 <= k1 && !any_small; k += 2)
                if (pop[lvl[k]] <= kPairLevel && pop[lvl[k + 1]] <= kPairLevel &&
                    width(k) + width(k + 1) <= kMaxPairWidth && P.stride[k] == P.stride[k + 1] + width(k)) {
                    unit[k + 1] = k;
                    pairs.push_back(k);
                }
            k0 = k1 + 1;
        }
        if (!pairs.empty()) nl = levels(lvl);
    }
    // pair inverses after the pieces' own, in each side's inverse region
    Level& L = h->lv;
    L = Level();
    std::vector<int64_t> pofs(nc, -1);
    int64_t dsz = doff[nc];
    for (int32_t p : pairs) {
        const int64_t W = width(p) + width(p + 1);
        pofs[p] = dsz;
        L.pair.push_back(PairItem{P.panel_off[p] + width(p), doff[p], doff[p + 1], dsz, P.stride[p], width(p),
                                  width(p + 1), 0});
        L.maxnb = std::max(L.maxnb, static_cast<int32_t>((W + 15) / 16 + 1));
        dsz += W * W;
    }
    h->dinv_size = dsz;
    L.cptr.assign(nl + 1, 0);
    for (int32_t k = 0; k < nc; ++k)
        if (unit[k] == k) ++L.cptr[lvl[k] + 1];
    for (int32_t l = 0; l < nl; ++l) L.cptr[l + 1] += L.cptr[l];
    L.cblk.resize(L.cptr[nl]);
    // small blocks (one 16-lane group each in the sweeps) first in their level
    L.nsmall.assign(nl, 0);
    std::vector<int32_t> pos(L.cptr.begin(), L.cptr.end() - 1);
    for (int32_t k = 0; k < nc; ++k)
        if (small(k) && unit[k] == k) {
            L.cblk[pos[lvl[k]]++] = k;
            ++L.nsmall[lvl[k]];
        }
    for (int32_t k = 0; k < nc; ++k)
        if (!small(k) && unit[k] == k) L.cblk[pos[lvl[k]]++] = k;
    // diagonal items: 16-row parts on levels with fewer than kNarrowLevel
    // blocks (16 lanes per row: fewer dependent load rounds), else 64-row
    constexpr int32_t kNarrowLevel = 64;
    // (levels holding a pair: 32 lanes, so that a row of the pair's 512-wide
    // inverse takes one round of sixteen loads per lane instead of two)
    L.dptr.assign(nl + 1, 0);
    L.narrow.assign(nl, 0);
    L.dlanes.assign(nl, 4);
    for (int32_t l = 0; l < nl; ++l) {
        const int32_t nb = L.cptr[l + 1] - L.cptr[l] - L.nsmall[l];
        L.narrow[l] = nb < kNarrowLevel ? 1 : 0;
        bool has_pair = false;
        for (int32_t q = L.cptr[l] + L.nsmall[l]; q < L.cptr[l + 1]; ++q) has_pair = has_pair || pofs[L.cblk[q]] >= 0;
        L.dlanes[l] = !L.narrow[l] ? 4 : (has_pair ? 32 : 16);
        const int32_t rows = 256 / L.dlanes[l];
        for (int32_t q = L.cptr[l] + L.nsmall[l]; q < L.cptr[l + 1]; ++q) {
            const int32_t k = L.cblk[q];
            const bool pr = pofs[k] >= 0;
            const int32_t w = pr ? width(k) + width(k + 1) : width(k);
            for (int32_t r0 = 0; r0 < w; r0 += rows)
                L.ditem.push_back(DiagItem{pr ? pofs[k] : doff[k], P.panel_off[k], pr ? P.panel_off[k + 1] : 0,
                                           P.fcol[k], w, r0, P.stride[k], width(k), pr ? P.stride[k + 1] : 0});
        }
        L.dptr[l + 1] = static_cast<int32_t>(L.ditem.size());
    }
    // off-diagonal items: up to 64 rows by a column range.  A level with
    // fewer than kOffTarget 64-row chunks splits the columns of each chunk
    // into 64-column parts (as many as bring the level towards kOffTarget
    // workgroups): the top levels hold one or two column blocks, and one
    // workgroup per 64 rows would leave most compute units idle while each
    // walks its columns serially.  One right-hand side takes its own list,
    // every chunk in 64-column parts (each wave then walks 16 columns, one
    // round of loads: 100^3 solve 3.43 -> 3.38 ms; with 8 right-hand sides,
    // whose items do eight times the work per loaded entry, that list was
    // slower, 6.71 -> 7.04 ms).
    constexpr int64_t kOffTarget = 1024;
    L.kptr.assign(nl + 1, 0);
    L.kptr1.assign(nl + 1, 0);
    L.bptr.assign(nl + 1, 0);
    std::vector<int32_t> members;
    for (int32_t l = 0; l < nl; ++l) {
        // the blocks of the level's units, with the first off-diagonal row of each
        members.clear();
        for (int32_t q = L.cptr[l] + L.nsmall[l]; q < L.cptr[l + 1]; ++q) {
            const int32_t k = L.cblk[q];
            members.push_back(k);
            if (pofs[k] >= 0) members.push_back(k + 1);
        }
        auto first_row = [&](int32_t k) { return pofs[k] >= 0 ? width(k) + width(k + 1) : width(k); };
        int64_t nch = 0;
        for (int32_t k : members) nch += (P.stride[k] - first_row(k) + 63) / 64;
        const int64_t want = nch > 0 ? (kOffTarget + nch - 1) / nch : 1;
        for (int32_t k : members) {
            const int32_t w = width(k);
            const int32_t units = (w + 63) / 64;
            const int32_t parts = static_cast<int32_t>(std::min<int64_t>(units, std::max<int64_t>(1, want)));
            const int32_t pw = 64 * ((units + parts - 1) / parts);
            for (int32_t r = first_row(k); r < P.stride[k]; r += 64) {
                const int32_t nr = std::min(64, P.stride[k] - r);
                for (int32_t c0 = 0; c0 < w; c0 += pw) {
                    const int32_t c1 = std::min(w, c0 + pw);
                    L.chunk.push_back(OffItem{P.panel_off[k] + r, rgo[k] + (r - w), P.stride[k], P.fcol[k], r,
                                              c0 | (c1 << 9) | (nr << 18)});
                }
            }
        }
        L.kptr[l + 1] = static_cast<int32_t>(L.chunk.size());
        for (int32_t k : members) {
            const int32_t w = width(k);
            for (int32_t r = first_row(k); r < P.stride[k]; r += 64) {
                const int32_t nr = std::min(64, P.stride[k] - r);
                for (int32_t c0 = 0; c0 < w; c0 += 64)
                    L.chunk1.push_back(OffItem{P.panel_off[k] + r, rgo[k] + (r - w), P.stride[k], P.fcol[k], r,
                                               c0 | (std::min(w, c0 + 64) << 9) | (nr << 18)});
            }
        }
        L.kptr1[l + 1] = static_cast<int32_t>(L.chunk1.size());
        // the backward sweep on narrow levels: 256 rows by 16 columns
        if (L.narrow[l])
            for (int32_t k : members) {
                const int32_t w = width(k);
                for (int32_t r = first_row(k); r < P.stride[k]; r += 256) {
                    const int32_t nr = std::min(256, P.stride[k] - r);
                    for (int32_t c0 = 0; c0 < w; c0 += 16)
                        L.bchunk.push_back(OffItem{P.panel_off[k] + r, rgo[k] + (r - w), P.stride[k], P.fcol[k], r,
                                                   c0 | (std::min(w, c0 + 16) << 9) | (nr << 18)});
                }
            }
        L.bptr[l + 1] = static_cast<int32_t>(L.bchunk.size());
    }
    h->lv_cblk.upload(L.cblk);
    h->lv_ditem.upload(L.ditem);
    h->lv_chunk.upload(L.chunk);
    h->lv_chunk1.upload(L.chunk1);
    h->lv_bchunk.upload(L.bchunk);
    h->lv_pair.upload(L.pair);
}

void upload_plan(spx_handle* h)
{
    const Plan& P = h->plan;
    h->uploaded = true;
    HIPCHK(hipGetDevice(&h->device));
    h->fcol.upload(P.fcol);
    h->lcol.upload(P.lcol);
    h->stride.upload(P.stride);
    h->bptr.upload(P.bptr);
    h->frow.upload(P.frow);
    h->lrow.upload(P.lrow);
    h->coefind.upload(P.coefind);
    h->perm.upload(P.perm);
    h->panel_off.upload(P.panel_off);
    std::vector<int64_t> doff(static_cast<size_t>(P.ncblk) + 1, 0);
    for (int32_t k = 0; k < P.ncblk; ++k) {
        const int64_t w = P.lcol[k] - P.fcol[k] + 1;
        doff[k + 1] = doff[k] + w * w;
    }
    h->dinv_size = doff[P.ncblk];
    h->dinv_off.upload(doff);
    {
        std::vector<int64_t> dg(static_cast<size_t>(P.n));
        for (int32_t k = 0; k < P.ncblk; ++k)
            for (int32_t c = P.fcol[k]; c <= P.lcol[k]; ++c)
                dg[c] = P.panel_off[k] + static_cast<int64_t>(c - P.fcol[k]) * (P.stride[k] + 1);
        h->diag_off.upload(dg);
    }
    h->amap.upload(P.amap);
    h->rptr.upload(P.rptr);
    h->rcol.upload(P.rcol);
    h->rval.upload(P.rval);
    // global rows of the off-diagonal panel rows
    std::vector<int32_t> rg;
    std::vector<int64_t> rgo(static_cast<size_t>(P.ncblk) + 1, 0);
    for (int32_t k = 0; k < P.ncblk; ++k) {
        rgo[k] = static_cast<int64_t>(rg.size());
        for (int32_t b = P.bptr[k] + 1; b < P.bptr[k + 1]; ++b)
            for (int32_t r = P.frow[b]; r <= P.lrow[b]; ++r) rg.push_back(r);
    }
    rgo[P.ncblk] = static_cast<int64_t>(rg.size());
    h->rowg.upload(rg);
    h->rowg_off.upload(rgo);
    {
        // coordinates of the entries read by the factorization, from the
        // symmetric row lists of the residual (each lower entry appears in
        // row i with column j <= i)
        std::vector<int32_t> er(static_cast<size_t>(h->nnz), -1), ec(static_cast<size_t>(h->nnz), -1);
        for (int32_t i = 0; i < P.n; ++i)
            for (int64_t q = P.rptr[i]; q < P.rptr[i + 1]; ++q)
                if (P.rcol[q] <= i) {
                    er[static_cast<size_t>(P.rval[q])] = i;
                    ec[static_cast<size_t>(P.rval[q])] = P.rcol[q];
                }
        h->erow.upload(er);
        h->ecol.upload(ec);
    }
    build_tasks(h);
    build_levels(h, doff, rgo);
    for (auto& e : h->ev)
        if (!e) HIPCHK(hipEventCreate(&e));
    int ncu = 0, clk_khz = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device));
    if (hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess || clk_khz <= 0)
        clk_khz = 100000;
    h->grid = std::max(1, ncu * sched_blocks_per_cu(h->f32(), h->ldlt(), h->lu()));
    h->timeout_ticks = static_cast<int64_t>(clk_khz) * 1000 * 20;   // 20 s per wait
    HIPCHK(scratch_region(&h->scratch, &h->scratch_bytes));
}

// Vectors of one application of the inverse: y (permuted right-hand side,
// consumed), z (forward result), x (backward result), tacc (backward partial
// sums); n x nrhs each, leading dimension n.
struct SweepBufs {
    double *y, *z, *x, *tacc;
};

// One application of (L L^T)^{-1} to the permuted vectors in w.y (consumed):
// result in w.x.
void sweeps(spx_handle* h, const SweepBufs& w, int32_t nrhs, hipStream_t s)
{
    SweepArgs a;
    a.pl = h->devplan();
    a.panels = h->panel_ptr();
    a.dinv = h->dinv_ptr();
    {
        const size_t esz = h->f32() ? sizeof(float) : sizeof(double);
        const int64_t pu = h->lu() ? h->plan.panel_entries : 0, du = h->lu() ? h->dinv_size : 0;
        a.panels_b = static_cast<const char*>(a.panels) + pu * esz;
        a.dinv_b = static_cast<const char*>(a.dinv) + du * esz;
    }
    a.f32 = h->f32() ? 1 : 0;
    a.ldlt = h->ldlt() ? 1 : 0;
    a.rowg = h->rowg.p;
    a.rowg_off = h->rowg_off.p;
    a.y = w.y;
    a.z = w.z;
    a.x = w.x;
    a.tacc = w.tacc;
    a.n = h->n;
    a.nrhs = nrhs;
    const Level& L = h->lv;
    const int nl = static_cast<int>(L.cptr.size()) - 1;
    for (int l = 0; l < nl; ++l) {
        const int32_t* sm = h->lv_cblk.p + L.cptr[l];
        const int ns = L.nsmall[l];
        HIPCHK(launch_fwd_small(a, sm, ns, s));
        HIPCHK(launch_fwd_diag(a, h->lv_ditem.p + L.dptr[l], L.dptr[l + 1] - L.dptr[l], L.dlanes[l], s));
        if (nrhs == 1) HIPCHK(launch_fwd_off(a, h->lv_chunk1.p + L.kptr1[l], L.kptr1[l + 1] - L.kptr1[l], s));
        else HIPCHK(launch_fwd_off(a, h->lv_chunk.p + L.kptr[l], L.kptr[l + 1] - L.kptr[l], s));
    }
    HIPCHK(launch_fill_f64(w.tacc, static_cast<int64_t>(h->n) * nrhs, 0.0, s));
    for (int l = nl - 1; l >= 0; --l) {
        const int32_t* sm = h->lv_cblk.p + L.cptr[l];
        const int ns = L.nsmall[l];
        // (256-row items for one right-hand side only: with a block of
        // several, gathering a 256-row slice of x per 16 columns costs more
        // than the atomics it saves)
        if (L.narrow[l] && nrhs == 1)
            HIPCHK(launch_bwd_off(a, h->lv_bchunk.p + L.bptr[l], L.bptr[l + 1] - L.bptr[l], true, s));
        else if (nrhs == 1)
            HIPCHK(launch_bwd_off(a, h->lv_chunk1.p + L.kptr1[l], L.kptr1[l + 1] - L.kptr1[l], false, s));
        else HIPCHK(launch_bwd_off(a, h->lv_chunk.p + L.kptr[l], L.kptr[l + 1] - L.kptr[l], false, s));
        HIPCHK(launch_bwd_diag(a, h->lv_ditem.p + L.dptr[l], L.dptr[l + 1] - L.dptr[l], L.dlanes[l], s));
        HIPCHK(launch_bwd_small(a, sm, ns, s));
    }
}

// The device work of one factorization on stream s, in two parts: (0)
// panels zeroed, values assembled (and gathered for the residual), queues
// initialised; (1) the scheduler kernel.
SchedArgs sched_args(spx_handle* h);

void factor_part(spx_handle* h, int part, hipStream_t s)
{
    const Plan& P = h->plan;
    const bool f32 = h->f32();
    const SchedArgs a = sched_args(h);
    if (part == 1) {
        if (h->total > 0) HIPCHK(launch_sched(a, f32, h->lu(), h->grid, s));
        return;
    }
    const int64_t nsym = P.rptr.empty() ? 0 : P.rptr.back();
    if (f32) HIPCHK(launch_fill_f32(h->panels_f.p, h->panel_count(), 0.0f, s));
    else HIPCHK(launch_fill_f64(h->panels.p, h->panel_count(), 0.0, s));
    HIPCHK(launch_assemble(h->panel_ptr(), f32, h->amap.p, h->vals.p, h->nnz, s));
    HIPCHK(launch_gather(h->rv.p, h->vals.p, h->rval.p, nsym, s));
    if (h->opt.method != SPX_LLT) HIPCHK(launch_absmax(h->amap.p, h->vals.p, h->nnz, h->status.p, s));
    HIPCHK(launch_sched_init(a, h->ready.p, h->nready, h->nready_hp, h->fact_dep0.p, P.ncblk, s));
}

SchedArgs sched_args(spx_handle* h)
{
    SchedArgs a;
    a.pl = h->devplan();
    a.panels = h->panel_ptr();
    a.dinv = h->dinv_ptr();
    a.split = h->opt.precision == SPX_BF16X3_IR ? 1 : 0;
    a.ldlt = h->ldlt() ? 1 : 0;
    a.pivot_eps = h->opt.method != SPX_LLT ? h->opt.static_pivot_eps : 0.0;
    a.upanel = h->lu() ? h->plan.panel_entries : 0;
    a.uinv = h->lu() ? h->dinv_size : 0;
    a.desc = h->desc.p;
    a.rmap = h->rmap.p;
    a.ftab = h->ftab.p;
    a.hp_total = h->hp_total;
    a.total_normal = h->total_normal;
    a.trsm_first = h->trsm_first.p;
    a.trsm_count = h->trsm_count.p;
    a.upd_first = h->upd_first.p;
    a.upd_hp = h->upd_hp.p;
    a.upd_count = h->upd_count.p;
    a.hp_cblk = h->hp_cblk.p;
    a.fact_dep = h->fact_dep.p;
    a.trsm_left = h->trsm_left.p;
    a.queue = h->queue.p;
    a.qhead = h->qctr.p;
    a.qtail = h->qctr.p + kCtrStride;
    a.hp_queue = h->hp_queue.p;
    a.hp_head = h->qctr.p + 2 * kCtrStride;
    a.hp_tail = h->qctr.p + 3 * kCtrStride;
    a.status = h->status.p;
    a.timeout_ticks = h->timeout_ticks;
    a.trace = h->opt.trace ? h->trace.p : nullptr;
    a.inv_item = h->ninv > 0 ? h->inv_item.p : nullptr;
    a.npair = h->npair;
    a.ubase = h->ubase;
    a.upair = h->upair.p;
    a.kpair = h->kpair.p;
    a.pairs = h->pairs.p;
    a.pdep0 = h->pdep0.p;
    a.pdep = h->pdep.p;
    a.pleft = h->pleft.p;
    return a;
}

// The inverses of the paired pieces of the sweeps, from the factor (for
// L U also from the U^T panels and U_kk^{-T}, for the backward sweep).
void pair_part(spx_handle* h, hipStream_t s)
{
    const Level& L = h->lv;
    if (L.pair.empty()) return;
    const bool f32 = h->f32();
    const size_t esz = f32 ? sizeof(float) : sizeof(double);
    const int np = static_cast<int>(L.pair.size());
    HIPCHK(launch_pair_inv(h->panel_ptr(), h->dinv_ptr(), f32, h->ldlt(), h->lv_pair.p, np, L.maxnb, s));
    if (h->lu())
        HIPCHK(launch_pair_inv(static_cast<const char*>(h->panel_ptr()) + h->plan.panel_entries * esz,
                               static_cast<char*>(h->dinv_ptr()) + h->dinv_size * esz, f32, false, h->lv_pair.p, np,
                               L.maxnb, s));
}

// One factorization of the values in h->vals: eagerly, or (graph option) by
// replaying the captured sequence (captured on first use and after any
// change of the work decomposition); then the status read-back.
void run_factorization(spx_handle* h, hipStream_t s)
{
    if (h->opt.trace) h->trace.alloc(static_cast<size_t>(h->total) * 4);
    if (h->opt.graph && !h->fgraph_exec[0]) {
        if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        for (int part = 0; part < 2; ++part) {
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            factor_part(h, part, h->cap_stream);
            HIPCHK(hipStreamEndCapture(h->cap_stream, &h->fgraph[part]));
            HIPCHK(hipGraphInstantiate(&h->fgraph_exec[part], h->fgraph[part], nullptr, nullptr, 0));
        }
    }
    for (int part = 0; part < 2; ++part) {
        HIPCHK(hipEventRecord(h->ev[part], s));
        if (h->opt.graph) HIPCHK(hipGraphLaunch(h->fgraph_exec[part], s));
        else factor_part(h, part, s);
    }
    HIPCHK(hipEventRecord(h->ev[2], s));
    pair_part(h, s);
    const Plan& P = h->plan;
    int32_t sw[kStatusWords];
    HIPCHK(hipMemcpyAsync(sw, h->status.p, sizeof sw, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int32_t st[3] = {sw[kStFail], sw[kStAbort], sw[kStDone]};
    h->nrep = sw[kStReplaced];
    float ms0 = 0.f, ms1 = 0.f;
    HIPCHK(hipEventElapsedTime(&ms0, h->ev[0], h->ev[1]));
    HIPCHK(hipEventElapsedTime(&ms1, h->ev[1], h->ev[2]));
    h->assemble_ms = ms0;
    h->factor_ms = ms1;
    if (h->total > 0 && (st[1] != 0 || st[2] != h->total)) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "device scheduler stopped early (%d of %d items, abort=%d)", st[2], h->total,
                      st[1]);
        throw DeviceError(buf);
    }
    if (st[0] != INT_MAX) {
        h->fail_col = (st[0] >= 0 && st[0] < h->n) ? P.perm[st[0]] : st[0];
        throw StatusError(SPX_ENOTPD, std::string(h->opt.method != SPX_LLT ? "zero or non-finite pivot" : "pivot not positive") +
                                          " at column " + std::to_string(h->fail_col));
    }
}

// Refinement shared by the solve entry points (FP64 residual, Section III's
// solve followed by iterative refinement): apply_b() sets xw = A^{-1} b;
// then, until omega <= ir_tol, ir_max_iter steps or stagnation (omega above
// half its previous value twice in a row): r = b - A xw with its statistics
// (stats: 5 lines of kStatStride words), apply_r() sets dw = A^{-1} rw,
// xw += dw.  b is a device array with leading dimension ldb.
template <class FB, class FR>
spx_solve_info refine(spx_handle* h, int32_t nrhs, const double* b, int64_t ldb, double* xw, double* rw,
                      const double* dw, unsigned long long* stats, FB apply_b, FR apply_r, hipStream_t s)
{
    const int32_t n = h->n;
    const size_t tot = static_cast<size_t>(n) * nrhs;
    apply_b();
    int iters = 0, slow = 0;
    double omega = 0.0, eta = 0.0, prev = INFINITY;
    const double tol = h->opt.ir_tol;
    for (;;) {
        HIPCHK(launch_zero_u64(stats, 5 * kStatStride, s));
        HIPCHK(launch_residual(h->rptr.p, h->rcol.p, h->rv.p, xw, b, ldb, rw, n, nrhs, stats, s));
        unsigned long long st[5 * kStatStride];
        HIPCHK(hipMemcpyAsync(st, stats, sizeof st, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double v[5];
        for (int q = 0; q < 5; ++q) std::memcpy(&v[q], &st[q * kStatStride], sizeof(double));
        omega = v[0];
        const double den = v[4] * v[2] + v[3];
        eta = v[1] == 0.0 ? 0.0 : (den == 0.0 ? INFINITY : v[1] / den);
        if (omega <= tol || iters >= h->opt.ir_max_iter) break;
        slow = omega > 0.5 * prev ? slow + 1 : 0;
        if (slow >= 2) break;
        prev = omega;
        apply_r();
        HIPCHK(launch_axpy(xw, dw, static_cast<int64_t>(tot), s));
        ++iters;
    }
    return spx_solve_info{iters, omega <= tol ? 1 : 0, omega, eta};
}

double pairwise_sum(const double* v, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += v[i];
        return s;
    }
    const int64_t m = n / 2;
    return pairwise_sum(v, m) + pairwise_sum(v + m, n - m);
}

}  // namespace

extern "C" {

void spx_default_options(spx_options* o)
{
    if (!o) return;
    o->method = SPX_LLT;
    o->leaf_size = 64;
    o->amalg_pct = 12;
    o->split_width = 256;
    o->user_perm = nullptr;
    o->precision = SPX_FP64;
    o->ir_max_iter = -1;
    o->ir_tol = 1e-14;
    o->trace = 0;
    o->graph = 0;
    o->tune = 0;
    o->tile = 0;
    o->fuse_small = 1;
    o->merge_split = 4;
    o->static_pivot_eps = -1.0;
    o->deterministic = 0;
}

int spx_analyze(int32_t n, const int64_t* colptr, const int32_t* rowind, const spx_options* opt, spx_handle** out)
{
    if (!out) return SPX_EINVAL;
    *out = nullptr;
    if (n < 0 || (n > 0 && (!colptr || !rowind))) return SPX_EINVAL;
    spx_handle* h = nullptr;
    try {
        h = new spx_handle();
    } catch (...) {
        return SPX_ENOMEM;
    }
    if (opt) h->opt = *opt; else spx_default_options(&h->opt);
    int rc = guarded(h, [&]() -> int {
        if (h->opt.method != SPX_LLT && h->opt.method != SPX_LDLT && h->opt.method != SPX_LU)
            throw InvalidArgument("unsupported method");
        if (h->opt.method == SPX_LU) h->opt.fuse_small = 0;   // every column block a FACT / TRSM / UPDATE sequence
        if (h->opt.deterministic != 0 && h->opt.deterministic != 1) throw InvalidArgument("deterministic must be 0 or 1");
        if (h->opt.deterministic) h->opt.fuse_small = 0;   // fused items scatter into several targets at once
        if (h->opt.precision != SPX_FP64 && h->opt.precision != SPX_FP32_IR && h->opt.precision != SPX_BF16X3_IR)
            throw InvalidArgument("unsupported precision");
        if (h->opt.ir_max_iter < -1) throw InvalidArgument("ir_max_iter must be >= 0, or -1 for the default");
        if (h->opt.ir_max_iter == -1) h->opt.ir_max_iter = h->opt.precision == SPX_FP64 ? 2 : 10;
        if (h->opt.tile != 0 && h->opt.tile != 1) throw InvalidArgument("tile must be 0 or 1");
        if (h->opt.merge_split < 1 || h->opt.merge_split > 16) throw InvalidArgument("merge_split must be in 1..16");
        if (!(h->opt.static_pivot_eps >= 0.0 || h->opt.static_pivot_eps == -1.0) || h->opt.static_pivot_eps >= 1.0)
            throw InvalidArgument("static_pivot_eps must be -1 (the default) or in [0, 1)");
        if (h->opt.static_pivot_eps == -1.0)   // sqrt of the unit roundoff of the factor's precision
            h->opt.static_pivot_eps = h->opt.precision == SPX_FP64 ? std::sqrt(std::ldexp(1.0, -53)) : std::ldexp(1.0, -12);
        h->tile_rows = h->opt.tile == 1 ? 128 : 256;
        h->tile_cols = h->opt.tile == 1 ? 128 : 64;
        Options o;
        o.leaf_size = h->opt.leaf_size;
        o.amalg_pct = h->opt.amalg_pct;
        o.split_width = h->opt.split_width;
        o.user_perm = h->opt.user_perm;
        o.lu = h->opt.method == SPX_LU;
        analyze_pattern(n, colptr, rowind, o, h->plan);
        h->n = n;
        h->nnz = n > 0 ? colptr[n] : 0;
        h->opt.user_perm = nullptr;
        // upload now when a device is present; a host-only process (symbolic
        // work only) defers it to the first factorization
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) upload_plan(h);
        return SPX_OK;
    });
    if (rc != SPX_OK) {
        g_analyze_err = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return SPX_OK;
}

int spx_analyze_batch(int32_t nsys, const int32_t* n, const int64_t* const* colptr, const int32_t* const* rowind,
                      const spx_options* opt, spx_handle** out)
{
    if (!out) return SPX_EINVAL;
    *out = nullptr;
    if (nsys <= 0 || !n || !colptr || !rowind || (opt && opt->user_perm)) return SPX_EINVAL;
    // block-diagonal pattern: system s occupies rows and columns
    // [off_s, off_s + n_s) and entries [colptr_all[off_s], ...)
    int64_t ntot = 0, nnz = 0;
    for (int32_t q = 0; q < nsys; ++q) {
        if (n[q] < 0 || (n[q] > 0 && (!colptr[q] || !rowind[q]))) return SPX_EINVAL;
        ntot += n[q];
        nnz += n[q] > 0 ? colptr[q][n[q]] : 0;
    }
    if (ntot > INT32_MAX) return SPX_EINVAL;
    std::vector<int64_t> cp;
    std::vector<int32_t> ri;
    try {
        cp.reserve(static_cast<size_t>(ntot) + 1);
        ri.reserve(static_cast<size_t>(nnz));
    } catch (...) {
        return SPX_ENOMEM;
    }
    cp.push_back(0);
    int32_t off = 0;
    for (int32_t q = 0; q < nsys; ++q) {
        for (int32_t j = 0; j < n[q]; ++j) {
            for (int64_t p = colptr[q][j]; p < colptr[q][j + 1]; ++p) {
                const int32_t r = rowind[q][p];
                if (r < 0 || r >= n[q]) return SPX_EINVAL;
                ri.push_back(off + r);
            }
            cp.push_back(static_cast<int64_t>(ri.size()));
        }
        off += n[q];
    }
    const int rc = spx_analyze(static_cast<int32_t>(ntot), cp.data(), ri.data(), opt, out);
    if (rc == SPX_OK) (*out)->nsys = nsys;
    return rc;
}

int spx_factorize(spx_handle* h, const double* values, int32_t values_on_device, void* hip_stream)
{
    if (!h) return SPX_EINVAL;
    return guarded(h, [&]() -> int {
        if (h->nnz > 0 && !values) throw InvalidArgument("values is NULL");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const Plan& P = h->plan;
        if (!h->uploaded) upload_plan(h);
        h->factorized = false;
        h->logdet_valid = false;
        h->fail_col = -1;
        h->vals.alloc(static_cast<size_t>(h->nnz));
        if (h->nnz > 0)
            HIPCHK(hipMemcpyAsync(h->vals.p, values, h->nnz * sizeof(double),
                                  values_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        const bool f32 = h->f32();
        if (f32) h->panels_f.alloc(static_cast<size_t>(h->panel_count()));
        else h->panels.alloc(static_cast<size_t>(h->panel_count()));
        if (!h->dinv_ptr()) {
            // blocks above the diagonal of each inverse are never written: zero them once
            if (f32) {
                h->dinv_f.alloc(static_cast<size_t>(h->dinv_count()));
                HIPCHK(launch_fill_f32(h->dinv_f.p, h->dinv_count(), 0.0f, s));
            } else {
                h->dinv.alloc(static_cast<size_t>(h->dinv_count()));
                HIPCHK(launch_fill_f64(h->dinv.p, h->dinv_count(), 0.0, s));
            }
        }
        const int64_t nsym = P.rptr.empty() ? 0 : P.rptr.back();
        h->rv.alloc(static_cast<size_t>(nsym));
        if (h->opt.tune && !h->tuned) {
            // autotuner: time one factorization per work decomposition on these
            // values and keep the fastest (update tile shape, priority policy)
            struct Cand {
                int32_t rows, cols, policy;
            };
            const Cand cand[] = {{256, 64, 0}, {128, 128, 0}, {256, 64, 1}, {128, 128, 1}};
            double best = INFINITY;
            Cand pick = cand[0];
            for (const Cand& c : cand) {
                h->tile_rows = c.rows;
                h->tile_cols = c.cols;
                h->hp_policy = c.policy;
                build_tasks(h);
                h->drop_fgraph();
                run_factorization(h, s);   // throws on breakdown, like the real run
                if (h->factor_ms < best) {
                    best = h->factor_ms;
                    pick = c;
                }
            }
            h->tile_rows = pick.rows;
            h->tile_cols = pick.cols;
            h->hp_policy = pick.policy;
            build_tasks(h);
            h->drop_fgraph();
            h->tuned = true;
        }
        run_factorization(h, s);
        h->factorized = true;
        return SPX_OK;
    });
}

int spx_solve(spx_handle* h, int32_t nrhs, double* b, int64_t ldb, int32_t b_on_device, spx_solve_info* info,
              void* hip_stream)
{
    if (!h) return SPX_EINVAL;
    return guarded(h, [&]() -> int {
        if (!h->factorized) throw StatusError(SPX_ESTATE, "solve called without a successful factorization");
        if (nrhs < 0 || ldb < h->n || (nrhs > 0 && h->n > 0 && !b)) throw InvalidArgument("bad right-hand side");
        if (info) *info = spx_solve_info{0, 1, 0.0, 0.0};
        if (nrhs == 0 || h->n == 0) return SPX_OK;
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const int32_t n = h->n;
        const size_t tot = static_cast<size_t>(n) * nrhs;
        if (nrhs > h->nrhs_cap) {
            // new buffers: a graph captured on the old ones is stale
            h->drop_graph();
            const size_t cap = static_cast<size_t>(n) * nrhs;
            for (DevBuf<double>* b : {&h->y, &h->zv, &h->xv, &h->tacc, &h->xw, &h->rw, &h->dw, &h->bw}) {
                b->release();
                b->alloc(cap);
            }
            h->nrhs_cap = nrhs;
        }
        h->stats.alloc(5 * kStatStride);
        if (h->graph_nrhs != nrhs) {
            // one application of A^{-1}: dw = P^T L^{-T} L^{-1} P rw, captured once per nrhs
            h->drop_graph();
            if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            HIPCHK(launch_permute_in(h->y.p, h->rw.p, n, h->perm.p, n, nrhs, h->cap_stream));
            sweeps(h, SweepBufs{h->y.p, h->zv.p, h->xv.p, h->tacc.p}, nrhs, h->cap_stream);
            HIPCHK(launch_permute_out(h->dw.p, n, h->xv.p, h->perm.p, n, nrhs, h->cap_stream));
            HIPCHK(hipStreamEndCapture(h->cap_stream, &h->graph));
            HIPCHK(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
            h->graph_nrhs = nrhs;
        }
        // the right-hand side, packed (leading dimension n)
        HIPCHK(hipMemcpy2DAsync(h->bw.p, n * sizeof(double), b, ldb * sizeof(double), n * sizeof(double), nrhs,
                                b_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        const spx_solve_info si = refine(
            h, nrhs, h->bw.p, n, h->xw.p, h->rw.p, h->dw.p, h->stats.p,
            [&] {   // x0 = A^{-1} b
                HIPCHK(hipMemcpyAsync(h->rw.p, h->bw.p, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipGraphLaunch(h->graph_exec, s));
                HIPCHK(hipMemcpyAsync(h->xw.p, h->dw.p, tot * sizeof(double), hipMemcpyDeviceToDevice, s));
            },
            [&] { HIPCHK(hipGraphLaunch(h->graph_exec, s)); }, s);
        HIPCHK(hipMemcpy2DAsync(b, ldb * sizeof(double), h->xw.p, n * sizeof(double), n * sizeof(double), nrhs,
                                b_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (info) *info = si;
        if (!si.converged) throw StatusError(SPX_ENOCONV, "refinement stopped above the tolerance");
        return SPX_OK;
    });
}

int spx_solve_noalloc(spx_handle* h, int32_t nrhs, double* b, int64_t ldb, spx_solve_info* info, void* hip_stream)
{
    if (!h) return SPX_EINVAL;
    return guarded(h, [&]() -> int {
        if (!h->factorized) throw StatusError(SPX_ESTATE, "solve called without a successful factorization");
        if (nrhs < 0 || ldb < h->n || (nrhs > 0 && h->n > 0 && !b)) throw InvalidArgument("bad right-hand side");
        if (info) *info = spx_solve_info{0, 1, 0.0, 0.0};
        if (nrhs == 0 || h->n == 0) return SPX_OK;
        int dev = -1;
        HIPCHK(hipGetDevice(&dev));
        if (dev != h->device || !h->scratch) throw InvalidArgument("the current device is not the handle's device");
        // work layout in the device's fixed array: the statistics lines, then
        // y, z, x, tacc, xw, rw, dw (n x nrhs doubles each, 256-byte aligned)
        const int32_t n = h->n;
        const size_t tot = static_cast<size_t>(n) * nrhs;
        const size_t vec = (tot * sizeof(double) + 255) / 256 * 256;
        const size_t head = 5 * kStatStride * sizeof(unsigned long long);
        const size_t need = head + 7 * vec;
        if (need > h->scratch_bytes) {
            char buf[200];
            std::snprintf(buf, sizeof buf,
                          "n * nrhs = %zu needs %zu bytes of work memory; the allocation-free solve has %zu "
                          "(at most %zu unknowns times right-hand sides)",
                          tot, need, h->scratch_bytes, (h->scratch_bytes - head) / 7 / sizeof(double));
            throw InvalidArgument(buf);
        }
        char* base = static_cast<char*>(h->scratch);
        unsigned long long* stats = reinterpret_cast<unsigned long long*>(base);
        double* v[7];
        for (int q = 0; q < 7; ++q) v[q] = reinterpret_cast<double*>(base + head + q * vec);
        const SweepBufs w{v[0], v[1], v[2], v[3]};
        double *xw = v[4], *rw = v[5], *dw = v[6];
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const spx_solve_info si = refine(
            h, nrhs, b, ldb, xw, rw, dw, stats,
            [&] {   // x0 = A^{-1} b, read in place
                HIPCHK(launch_permute_in(w.y, b, ldb, h->perm.p, n, nrhs, s));
                sweeps(h, w, nrhs, s);
                HIPCHK(launch_permute_out(xw, n, w.x, h->perm.p, n, nrhs, s));
            },
            [&] {
                HIPCHK(launch_permute_in(w.y, rw, n, h->perm.p, n, nrhs, s));
                sweeps(h, w, nrhs, s);
                HIPCHK(launch_permute_out(dw, n, w.x, h->perm.p, n, nrhs, s));
            },
            s);
        HIPCHK(hipMemcpy2DAsync(b, ldb * sizeof(double), xw, n * sizeof(double), n * sizeof(double), nrhs,
                                hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        if (info) *info = si;
        if (!si.converged) throw StatusError(SPX_ENOCONV, "refinement stopped above the tolerance");
        return SPX_OK;
    });
}

int spx_values_grad(spx_handle* h, int32_t nrhs, const double* x, const double* db, int64_t ld, double* grad,
                    void* hip_stream)
{
    if (!h) return SPX_EINVAL;
    return guarded(h, [&]() -> int {
        if (!h->uploaded) throw StatusError(SPX_ESTATE, "no device plan (no factorization yet)");
        if (nrhs < 0 || (nrhs > 0 && ld < h->n)) throw InvalidArgument("bad vector shape");
        if (h->lu()) throw InvalidArgument("the value gradient needs a symmetric method (SPX_LLT or SPX_LDLT)");
        if (h->nnz > 0 && !grad) throw InvalidArgument("grad is NULL");
        if (nrhs > 0 && h->n > 0 && (!x || !db)) throw InvalidArgument("x or db is NULL");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        HIPCHK(launch_values_grad(h->erow.p, h->ecol.p, h->nnz, x, db, ld, nrhs, grad, s));
        HIPCHK(hipStreamSynchronize(s));
        return SPX_OK;
    });
}

int spx_get_info(const spx_handle* hc, spx_info* info)
{
    if (!hc || !info) return SPX_EINVAL;
    spx_handle* h = const_cast<spx_handle*>(hc);
    return guarded(h, [&]() -> int {
        const Plan& P = h->plan;
        if (h->factorized && !h->logdet_valid) {
            // 2 * sum log l_jj (L D L^T: sum log |d_j| and the count of d_j < 0)
            // with pairwise summation, from the diagonal of each panel
            // one gather kernel into a contiguous FP64 vector, one copy
            std::vector<double> diag(static_cast<size_t>(P.n));
            if (P.n > 0) {
                DevBuf<double> dd;
                dd.alloc(static_cast<size_t>(P.n));
                HIPCHK(launch_gather_diag(dd.p, h->panel_ptr(), h->f32(), h->diag_off.p, P.n, nullptr));
                HIPCHK(hipMemcpy(diag.data(), dd.p, static_cast<size_t>(P.n) * sizeof(double), hipMemcpyDeviceToHost));
            }
            h->nneg = 0;
            if (h->ldlt() || h->lu()) {
                for (auto& d : diag) {
                    h->nneg += d < 0.0;
                    d = std::log(std::fabs(d));
                }
            } else {
                for (auto& d : diag) d = 2.0 * std::log(d);
            }
            h->logdet = pairwise_sum(diag.data(), P.n);
            h->logdet_valid = true;
        }
        spx_info o;
        std::memset(&o, 0, sizeof o);
        o.n = P.n;
        o.ncblk = P.ncblk;
        o.nblok = P.nblok;
        o.nsnode = P.nsnode;
        o.nnz_a = P.nnz_a;
        o.nnz_l = P.nnz_exact;
        o.nnz_l_stored = P.nnz_stored;
        o.panel_entries = P.panel_entries;
        o.flops_alg = h->lu() ? P.flops_alg_lu : P.flops_alg;
        o.flops_exec = h->lu() ? P.flops_exec_lu : P.flops_exec;
        o.ntasks = h->total;
        o.nfused_tiles = h->nfused_tiles;
        o.nsmall = h->nsmall;
        o.fail_col = h->fail_col;
        o.factorized = h->factorized ? 1 : 0;
        o.logdet = h->logdet_valid ? h->logdet : 0.0;
        o.nneg = h->logdet_valid ? h->nneg : 0;
        o.pivots_replaced = h->factorized ? h->nrep : 0;
        o.solve_levels = h->lv.cptr.empty() ? 0 : static_cast<int32_t>(h->lv.cptr.size()) - 1;
        o.solve_pairs = static_cast<int32_t>(h->lv.pair.size());
        o.factor_kernel_ms = h->factor_ms;
        o.assemble_ms = h->assemble_ms;
        o.tile_rows = h->tile_rows;
        o.tile_cols = h->tile_cols;
        o.hp_policy = h->hp_policy;
        o.nsys = h->nsys;
        *info = o;
        return SPX_OK;
    });
}

int spx_export_symbolic(const spx_handle* h, spx_symbolic_view* v)
{
    if (!h || !v) return SPX_EINVAL;
    const Plan& P = h->plan;
    v->n = P.n;
    v->ncblk = P.ncblk;
    v->nblok = P.nblok;
    v->nsnode = P.nsnode;
    v->nupd = static_cast<int32_t>(P.utgt.size());
    v->perm = P.perm.data();
    v->iperm = P.iperm.data();
    v->etree = P.etree.data();
    v->snptr = P.snptr.data();
    v->fcol = P.fcol.data();
    v->lcol = P.lcol.data();
    v->stride = P.stride.data();
    v->panel_off = P.panel_off.data();
    v->bptr = P.bptr.data();
    v->cparent = P.cparent.data();
    v->frow = P.frow.data();
    v->lrow = P.lrow.data();
    v->fcblk = P.fcblk.data();
    v->coefind = P.coefind.data();
    v->uptr = P.uptr.data();
    v->utgt = P.utgt.data();
    v->dep = P.dep.data();
    return SPX_OK;
}

int spx_copy_factor(spx_handle* h, double* dst, int32_t dst_on_device, void* hip_stream)
{
    if (!h) return SPX_EINVAL;
    return guarded(h, [&]() -> int {
        if (!h->factorized) throw StatusError(SPX_ESTATE, "no factorization");
        if (!dst && h->panel_count() > 0) throw InvalidArgument("dst is NULL");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        const int64_t ne = h->panel_count();
        if (ne > 0 && h->f32()) {
            if (dst_on_device) {
                HIPCHK(launch_widen(dst, h->panels_f.p, ne, s));
            } else {
                DevBuf<double> tmp;
                tmp.alloc(static_cast<size_t>(ne));
                HIPCHK(launch_widen(tmp.p, h->panels_f.p, ne, s));
                HIPCHK(hipMemcpyAsync(dst, tmp.p, ne * sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            }
        } else if (ne > 0) {
            HIPCHK(hipMemcpyAsync(dst, h->panels.p, ne * sizeof(double),
                                  dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        return SPX_OK;
    });
}

int64_t spx_get_trace(spx_handle* h, int64_t* dst, int64_t cap, int32_t* kinds)
{
    if (!h) return SPX_EINVAL;
    return guarded(h, [&]() -> int {
        if (!h->opt.trace || !h->trace.p) throw StatusError(SPX_ESTATE, "trace option off or no factorization yet");
        if (cap < h->total) throw InvalidArgument("trace buffer too small");
        HIPCHK(hipMemcpy(dst, h->trace.p, static_cast<size_t>(h->total) * 4 * sizeof(int64_t), hipMemcpyDeviceToHost));
        if (kinds) {
            std::vector<int4> d(static_cast<size_t>(h->total) * 2);
            HIPCHK(hipMemcpy(d.data(), h->desc.p, d.size() * sizeof(int4), hipMemcpyDeviceToHost));
            for (int32_t i = 0; i < h->total; ++i) {
                const int32_t kind = d[2 * i].x & 0xff;
                kinds[4 * i + 0] = kind;         // kind
                kinds[4 * i + 1] = d[2 * i].y;   // source cblk (the last piece of a merged update)
                kinds[4 * i + 2] = kind == kUpdate ? d[2 * i].z : d[2 * i].y;   // target cblk
                kinds[4 * i + 3] = kind == kUpdate ? d[2 * i + 1].x * d[2 * i + 1].z : d[2 * i].w;
            }
        }
        return h->total;
    });
}

int spx_update_bench(int32_t precision, int32_t method, int32_t n_inner, int32_t m, int32_t k, void* panels,
                     const int32_t* rmap, int32_t ldc, int32_t tile, int32_t calls, int32_t nstreams, double* ms)
{
    using namespace spx;
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev;
    auto cleanup = [&]() {
        for (auto e : ev) (void)hipEventDestroy(e);
        for (auto q : st) (void)hipStreamDestroy(q);
    };
    try {
        if (precision != SPX_FP64 && precision != SPX_FP32_IR && precision != SPX_BF16X3_IR)
            throw InvalidArgument("unsupported precision");
        if (method != SPX_LLT && method != SPX_LDLT) throw InvalidArgument("method must be SPX_LLT or SPX_LDLT");
        if (n_inner < 1 || k < 1 || m < k || !panels || !rmap || !ms) throw InvalidArgument("bad sizes or pointers");
        if (ldc < m || tile < 0 || tile > 1 || calls < 1 || nstreams < 0 || nstreams > 3)
            throw InvalidArgument("bad ldc, tile, calls or stream count");
        if (static_cast<int64_t>(n_inner + m) * n_inner + static_cast<int64_t>(ldc) * k > INT32_MAX)
            throw InvalidArgument("panels exceed 2^31 elements");
        // the row map: source row n_inner + i goes to target row rmap[i]; the
        // first k are the target's columns, the others distinct rows below
        std::vector<int32_t> rm(static_cast<size_t>(m));
        HIPCHK(hipMemcpy(rm.data(), rmap, rm.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int32_t i = 0; i < m; ++i)
            if ((i < k && rm[i] != i) || (i >= k && (rm[i] < k || rm[i] >= ldc || (i > k && rm[i] <= rm[i - 1]))))
                throw InvalidArgument("row map: the first k rows must be 0..k-1, the others increasing in [k, ldc)");
        const bool f32 = precision != SPX_FP64;
        const int32_t tr = tile ? 128 : 256, tc = tile ? 128 : 64;
        std::vector<int4> tiles;
        for (int32_t r0 = n_inner; r0 < n_inner + m; r0 += tr)
            for (int32_t c0 = n_inner; c0 < n_inner + k; c0 += tc) {
                const int32_t mr = std::min(tr, n_inner + m - r0);
                if (r0 + mr - 1 < c0) continue;   // strictly above the target's diagonal
                tiles.push_back(int4{r0, mr, c0, std::min(tc, n_inner + k - c0)});
            }
        DevBuf<int32_t> fcol, lcol, stride;
        DevBuf<int64_t> poff;
        DevBuf<int4> dt;
        fcol.upload(std::vector<int32_t>{0, n_inner});
        lcol.upload(std::vector<int32_t>{n_inner - 1, n_inner + k - 1});
        stride.upload(std::vector<int32_t>{n_inner + m, ldc});
        poff.upload(std::vector<int64_t>{0, static_cast<int64_t>(n_inner + m) * n_inner});
        dt.upload(tiles);
        SchedArgs a{};
        a.pl.ncblk = 2;
        a.pl.fcol = fcol.p;
        a.pl.lcol = lcol.p;
        a.pl.stride = stride.p;
        a.pl.panel_off = poff.p;
        a.panels = panels;
        a.rmap = rmap;
        a.split = precision == SPX_BF16X3_IR ? 1 : 0;
        a.ldlt = method == SPX_LDLT ? 1 : 0;
        const int nt = static_cast<int>(tiles.size());
        const int ns = std::max(1, nstreams);
        for (int i = 0; i < ns; ++i) {
            hipStream_t q;
            HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
            st.push_back(q);
        }
        for (int i = 0; i < 2 + ns; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ev.push_back(e);
        }
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipEventRecord(ev[0], st[0]));
        for (int i = 1; i < ns; ++i) HIPCHK(hipStreamWaitEvent(st[i], ev[0], 0));
        if (nstreams == 0) {   // all calls as one grid
            HIPCHK(launch_update_bench(a, f32, method == SPX_LDLT, dt.p, nt, -n_inner, calls, st[0]));
        } else {               // one grid per call, round-robin over the streams
            for (int c = 0; c < calls; ++c)
                HIPCHK(launch_update_bench(a, f32, method == SPX_LDLT, dt.p, nt, -n_inner, 1, st[c % ns]));
        }
        for (int i = 1; i < ns; ++i) {
            HIPCHK(hipEventRecord(ev[2 + i], st[i]));
            HIPCHK(hipStreamWaitEvent(st[0], ev[2 + i], 0));
        }
        HIPCHK(hipEventRecord(ev[1], st[0]));
        HIPCHK(hipEventSynchronize(ev[1]));
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        *ms = t;
        cleanup();
        return SPX_OK;
    } catch (const InvalidArgument& e) {
        cleanup();
        g_analyze_err = e.what();
        return SPX_EINVAL;
    } catch (const std::bad_alloc&) {
        cleanup();
        g_analyze_err = "out of memory";
        return SPX_ENOMEM;
    } catch (const std::exception& e) {
        cleanup();
        g_analyze_err = e.what();
        return SPX_EDEVICE;
    }
}

void spx_destroy(spx_handle* h) { delete h; }

const char* spx_strerror(int status)
{
    switch (status) {
    case SPX_OK: return "success";
    case SPX_EINVAL: return "invalid argument";
    case SPX_ENOMEM: return "out of memory";
    case SPX_EDEVICE: return "device error";
    case SPX_ESTATE: return "call out of order";
    case SPX_ENOTPD: return "matrix is not positive definite (L D L^T: a zero pivot)";
    case SPX_ENOCONV: return "refinement did not converge";
    default: return "unknown status";
    }
}

const char* spx_last_error(const spx_handle* h) { return h ? h->err.c_str() : g_analyze_err.c_str(); }

}  // extern "C"
