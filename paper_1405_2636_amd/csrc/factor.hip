// Numerical supernodal LL^T factorization on one MI355X (gfx950).
//
// The method is the paper's (Section III): for every column block k, (1)
// Cholesky of its diagonal block, (2) triangular solve of its off-diagonal
// rows, (3) right-looking updates C_j -= L_k[rows] L_k[facing j]^T scattered
// into every facing column block j (the sparse GEMM of Section V-B, computed
// directly into the gapped destination panel, without a temporary buffer).
// As in the runtime versions of the paper the 1D task is split: one task
// factors a panel, the updates become separate tasks.  Here they are further
// tiled, and all of them are scheduled by one persistent kernel that pulls
// work items from device-side ready queues:
//   FACT(k)          Cholesky of the diagonal block and its inverse L_kk^{-1}
//   TRSM(k, rows)    64 off-diagonal rows of panel k times L_kk^{-T}
//   UPDATE(k,j,r,c)  a 128x128 (or 256x64) tile of the outer product of panel
//                    k, subtracted into panel j with FP64 atomics
// Dependencies are counters: FACT(j) becomes ready when every UPDATE tile
// into j is done, the TRSM tiles of k when FACT(k) is done, the UPDATE tiles
// of k when its last TRSM tile is done.  FACT, TRSM and the updates into the
// next block of a chain go to a high-priority queue that workers poll first.
// Products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
#include "device.hpp"

namespace spx {

typedef double d4 __attribute__((ext_vector_type(4)));

#define AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// A global operand read through a buffer resource covering one array (a panel
// or an inverse): element (i, p) (i = row or column index of the product, p =
// inner index) is at byte off + i*si + p*sk.  Reads past the end of the array
// return zero (buffer range check), so tiles need no bounds masks: rows or
// columns beyond a tile only feed results that are not stored, and the inner
// ranges either end at the array's end or meet zeros (upper triangle of an
// inverse).
struct GOp {
    __amdgpu_buffer_rsrc_t rs;
    int off, si, sk;
};

// Values the whole wave shares, moved to scalar registers (buffer resources
// must be uniform; the compiler cannot prove it for values read from memory).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ const double* uni(const double* p)
{
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<const double*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ GOp make_gop(const double* base, int64_t count, int64_t off, int64_t si, int64_t sk)
{
    GOp g;
    g.rs = __builtin_amdgcn_make_buffer_rsrc((void*)uni(base), (short)0, uni((int)(count * 8)), 0x00020000);
    g.off = uni((int)(off * 8));
    g.si = uni((int)(si * 8));
    g.sk = uni((int)(sk * 8));
    return g;
}

__device__ __forceinline__ double gload(const GOp& g, int voff)
{
    const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(g.rs, voff, 0, 0);
    return __builtin_bit_cast(double, b);
}

// One wave accumulates a 64 x (16*NB) tile: acc += X Y^T, X(r, p) r < 64,
// Y(c, p) c < 16*NB, p < K (K rounded up to 8 reads zeros or is exact).  The
// whole tile is always computed (no per-block predicates); rows and columns
// beyond the caller's bounds produce results that are not stored.
// The f64 16x16x4 matrix-core lane layout is: operand A lane l holds
// A[l%16][l/16], operand B lane l holds B[l/16][l%16], result slot v of lane
// l holds D[4v + l/16][l%16].  Y feeds operand A and X operand B, so
//   acc[bi][bj][v] = C(16*bj + l%16, 16*bi + 4v + l/16)
// and the 16 lanes of a result slot cover 16 consecutive rows of C.  The
// inner dimension advances 8 at a time through two register buffers: the
// operands of the next 8 are in flight while the products of the current 8
// are issued.
template <int NB>
__device__ __forceinline__ void wave_gemm(d4 (&acc)[NB][4], const GOp& X, const GOp& Y, int K)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nchunks = (K + 7) >> 3;
    if (nchunks <= 0) return;
    int xo[2][4], yo[2][NB];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int b = 0; b < 4; ++b) xo[u][b] = X.off + (16 * b + li) * X.si + (4 * u + lk) * X.sk;
#pragma unroll
        for (int b = 0; b < NB; ++b) yo[u][b] = Y.off + (16 * b + li) * Y.si + (4 * u + lk) * Y.sk;
    }
    const int dx = 8 * X.sk, dy = 8 * Y.sk;
    double xa[2][4], ya[2][NB], xb[2][4], yb[2][NB];
    auto load = [&](double (&xs)[2][4], double (&ys)[2][NB], int ch) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int b = 0; b < 4; ++b) xs[u][b] = gload(X, xo[u][b] + ch * dx);
#pragma unroll
            for (int b = 0; b < NB; ++b) ys[u][b] = gload(Y, yo[u][b] + ch * dy);
        }
    };
    auto mma = [&](const double (&xs)[2][4], const double (&ys)[2][NB]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma_f64(ys[u][bi], xs[u][bj], acc[bi][bj]);
    };
    load(xa, ya, 0);
    int ch = 0;
    for (; ch + 2 <= nchunks; ch += 2) {
        load(xb, yb, ch + 1);
        mma(xa, ya);
        load(xa, ya, min(ch + 2, nchunks - 1));
        mma(xb, yb);
    }
    if (ch < nchunks) mma(xa, ya);
}

// Same product with Y in LDS: Y(c, p) = Y[c*ysc + p*ysp], masked to c < nv, p < K.
template <int NB>
__device__ __forceinline__ void wave_gemm_lds(d4 (&acc)[NB][4], const GOp& X, int nbx, const double* Y, int ysc,
                                              int ysp, int nv, int K)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nby = min(NB, (nv + 15) >> 4);
    if (nbx <= 0 || nby <= 0) return;
    for (int p0 = 0; p0 < K; p0 += 4) {
        const int p = p0 + lk;
        double xs[4], ys[NB];
#pragma unroll
        for (int b = 0; b < 4; ++b) xs[b] = b < nbx ? gload(X, X.off + (16 * b + li) * X.si + p * X.sk) : 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int c = 16 * b + li;
            ys[b] = (c < nv && p < K) ? Y[c * ysc + p * ysp] : 0.0;
        }
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
                if (bi < nby && bj < nbx) acc[bi][bj] = mfma_f64(ys[bi], xs[bj], acc[bi][bj]);
    }
}

template <int NB>
__device__ __forceinline__ void zero_acc(d4 (&acc)[NB][4])
{
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

// epi(r, c, value) over a wave's accumulator, r < mv, c < nv
template <int NB, class Epi>
__device__ __forceinline__ void wave_store(const d4 (&acc)[NB][4], int mv, int nv, Epi epi)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * bj + li, c = 16 * bi + 4 * v + lk;
                if (r < mv && c < nv) epi(r, c, acc[bi][bj][v]);
            }
}

__device__ __forceinline__ int nblk(int n) { return (n + 15) >> 4; }

// ---------------------------------------------------------------- FACT(k)
// Cholesky of one 32x32 tile kept in LDS (Ls, column-major, ld 33), by one
// wave: row r is loaded into registers of lanes r and r+32, columns are
// eliminated one by one with the pivot column broadcast through readlane.
// Rows/columns >= jb must hold the identity.  Pivots that are not > 0 record
// their column with atomicMin and the computation goes on (NaN propagates).
__device__ __noinline__ void tile_potrf(double* Ls, int jb, int col0, int32_t* status)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 31;
    double t[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) t[c] = Ls[r + c * 33];
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const double d = readlane_d(t[c], c);
        if (c < jb && !(d > 0.0) && lane == 0) atomicMin(status, col0 + c);
        const double s = sqrt(d);
        const double inv = 1.0 / s;
        if (r == c) t[c] = s;
        else if (r > c) t[c] *= inv;
#pragma unroll
        for (int c2 = c + 1; c2 < 32; ++c2) {
            const double l2 = readlane_d(t[c], c2);
            if (r >= c2) t[c2] -= t[c] * l2;
        }
    }
    if (lane < 32) {
#pragma unroll
        for (int c = 0; c < 32; ++c) Ls[r + c * 33] = c <= r ? t[c] : 0.0;
    }
}

// Inverse X = L^{-1} of the lower triangular 32x32 tile Ls, by one wave in
// the same row-per-lane layout: column c of L is eliminated from the rows
// below once row c of X is final (row c of X divided by l_cc, then
// x_r -= l_rc x_c for r > c, with x_c broadcast through readlane).  Row r of
// X (r < jb) is stored at D + r, columns strided by ldd.
__device__ __noinline__ void tile_trtri(const double* Ls, double* D, int ldd, int jb)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 31;
    double t[32], x[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        t[c] = Ls[r + c * 33];
        x[c] = (c == r) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const double inv = 1.0 / readlane_d(t[c], c);
#pragma unroll
        for (int q = 0; q <= c; ++q) x[q] = (r == c) ? x[q] * inv : x[q];
#pragma unroll
        for (int q = 0; q <= c; ++q) {
            const double xc = readlane_d(x[q], c);
            if (r > c) x[q] -= t[c] * xc;
        }
    }
    if (lane < jb) {
#pragma unroll
        for (int q = 0; q < 32; ++q)
            if (q < jb) D[r + (int64_t)q * ldd] = q <= r ? x[q] : 0.0;
    }
}

// Left-looking blocked Cholesky of the w x w diagonal block (w <= 256) by one
// workgroup, 32 columns at a time: subtract the products of the factored
// columns (matrix cores), factor and invert the 32x32 diagonal tile in
// registers (wave 0), multiply the rows below by the tile inverse's
// transpose.  Then the blocked inverse D = L_kk^{-1} (lower, w x w,
// column-major; its upper triangle stays zero) is formed block row by block
// row:  D_IJ = -D_II * sum_{J<=K<I} L_IK D_KJ.
__device__ __noinline__ void task_fact(const SchedArgs& a, int k, double* Ls, double* Gs)
{
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k];
    const int w = pl.lcol[k] - f + 1;
    const int64_t ld = pl.stride[k];
    double* A = a.panels + pl.panel_off[k];
    double* D = a.dinv + pl.dinv_off[k];
    const int64_t nA = ld * w, nD = (int64_t)w * w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = (w + kNB - 1) / kNB;
    for (int J = 0; J < w; J += kNB) {
        const int jb = min(kNB, w - J);
        if (J > 0) {
            const int m = w - J, r0 = 64 * wave;
            if (r0 < m) {
                d4 acc[2][4];
                zero_acc(acc);
                wave_gemm<2>(acc, make_gop(A, nA, J + r0, 1, ld), make_gop(A, nA, J, 1, ld), J);
                wave_store(acc, min(64, m - r0), jb, [&](int r, int c, double v) {
                    if (r0 + r >= c) A[(J + r0 + r) + (int64_t)(J + c) * ld] -= v;
                });
            }
            __syncthreads();
        }
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            const int r = idx & 31, c = idx >> 5;
            Ls[r + c * 33] = (r < jb && c < jb) ? (c <= r ? A[(J + r) + (int64_t)(J + c) * ld] : 0.0)
                                                : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        if (wave == 0) {
            tile_potrf(Ls, jb, f + J, a.status);
            tile_trtri(Ls, D + J + (int64_t)J * w, w, jb);
        }
        __syncthreads();
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            const int r = idx & 31, c = idx >> 5;
            if (r < jb && c <= r) A[(J + r) + (int64_t)(J + c) * ld] = Ls[r + c * 33];
        }
        __syncthreads();
        // rows below the tile: B <- B * D_JJ^T  (in place, each wave owns its rows)
        const int m2 = w - J - jb, r0 = 64 * wave;
        if (r0 < m2) {
            d4 acc[2][4];
            zero_acc(acc);
            wave_gemm<2>(acc, make_gop(A, nA, (J + jb + r0) + (int64_t)J * ld, 1, ld),
                         make_gop(D, nD, J + (int64_t)J * w, 1, w), jb);
            double* B = A + (J + jb + r0) + (int64_t)J * ld;
            wave_store(acc, min(64, m2 - r0), jb, [&](int r, int c, double v) { B[r + (int64_t)c * ld] = v; });
        }
        __syncthreads();
    }
    // inverse, block rows I = 1 .. nt-1 (D_II already stored); the ib x I0
    // products are dealt to the waves in 32-column slices
    for (int I = 1; I < nt; ++I) {
        const int I0 = I * kNB, ib = min(kNB, w - I0);
        // rows ib..31 of G stay zero (they meet the padded inner range below)
        for (int idx = tid; idx < kNB * I0; idx += kThreads) {
            const int rr = idx & 31, cc = idx >> 5;
            if (rr >= ib) Gs[rr + cc * 33] = 0.0;
        }
        // G = L[I0:I0+ib, 0:I0] * D[0:I0, 0:I0]   (ib x I0) -> Gs (column-major, ld 33)
        for (int c0 = 32 * wave; c0 < I0; c0 += 128) {
            d4 acc[2][4];
            zero_acc(acc);
            wave_gemm<2>(acc, make_gop(A, nA, I0, 1, ld), make_gop(D, nD, (int64_t)c0 * w, w, 1), I0);
            wave_store(acc, ib, min(32, I0 - c0), [&](int r, int c, double v) { Gs[r + (c0 + c) * 33] = v; });
        }
        __syncthreads();
        // D[I0:I0+ib, 0:I0] = -D_II * G
        for (int c0 = 32 * wave; c0 < I0; c0 += 128) {
            d4 acc[2][4];
            zero_acc(acc);
            wave_gemm_lds<2>(acc, make_gop(D, nD, I0 + (int64_t)I0 * w, 1, w), nblk(ib), Gs + c0 * 33, 33, 1,
                             min(32, I0 - c0), ib);
            wave_store(acc, ib, min(32, I0 - c0),
                       [&](int r, int c, double v) { D[(I0 + r) + (int64_t)(c0 + c) * w] = -v; });
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- TRSM(k, rows)
// Rows [row0, row0+nrows) (nrows <= 64) of panel k below its diagonal block
// are replaced by B L_kk^{-T} = B D^T.  Wave v computes the 64 output columns
// starting at 64v; the inner range stops at the diagonal of the lower
// triangular D.
__device__ __noinline__ void task_trsm(const SchedArgs& a, int k, int row0, int nrows)
{
    const DevPlan& pl = a.pl;
    const int w = pl.lcol[k] - pl.fcol[k] + 1;
    const int64_t ld = pl.stride[k];
    double* P = a.panels + pl.panel_off[k];
    double* B = P + row0;
    const double* D = a.dinv + pl.dinv_off[k];
    const int wave = threadIdx.x >> 6;
    d4 acc[4][4];
    zero_acc(acc);
    const int c0 = 64 * wave;
    const int nv = min(64, w - c0);
    if (nv > 0) wave_gemm<4>(acc, make_gop(P, ld * w, row0, 1, ld), make_gop(D, (int64_t)w * w, c0, 1, w), min(w, c0 + 64));
    __syncthreads();   // every wave has read all of B before any result is written
    if (nv > 0) wave_store(acc, nrows, nv, [&](int r, int c, double v) { B[r + (int64_t)(c0 + c) * ld] = v; });
}

// ---------------------------------------------------------------- UPDATE
// W = L_k[row0 : row0+mrows] * L_k[col0 : col0+ncols]^T (inner dimension =
// width of k), C_j[rmap(row), rmap(col)] -= W on the lower triangle of j.
// rmap (precomputed from the symbolic structure) gives, for every panel row
// of k from the first block facing j on, its row inside panel j; for facing
// rows that is also the column of j.  ncols <= 64, mrows <= 256: the four
// waves cover 64 rows each.
__device__ __noinline__ void task_update(const SchedArgs& a, const int4 d0, const int4 d1, int* rpos, int* cpos)
{
    const DevPlan& pl = a.pl;
    const int k = d0.y, j = d0.z, row0 = d0.w;
    const int mrows = d1.x, col0 = d1.y, ncols = d1.z, mbase = d1.w;
    const int w = pl.lcol[k] - pl.fcol[k] + 1;
    const int64_t ld = pl.stride[k], ldj = pl.stride[j];
    const double* A = a.panels + pl.panel_off[k];
    double* C = a.panels + pl.panel_off[j];
    const int tid = threadIdx.x, wave = tid >> 6;
    if (tid < mrows) rpos[tid] = a.rmap[mbase + row0 + tid];
    if (tid < ncols) cpos[tid] = a.rmap[mbase + col0 + tid];
    __syncthreads();
    const int r0 = 64 * wave;
    const int mv = min(64, mrows - r0);
    if (mv > 0) {
        d4 acc[4][4];
        zero_acc(acc);
        wave_gemm<4>(acc, make_gop(A, ld * w, row0 + r0, 1, ld), make_gop(A, ld * w, col0, 1, ld), w);
        wave_store(acc, mv, ncols, [&](int r, int c, double v) {
            const int tr = rpos[r0 + r], tc = cpos[c];
            if (tr >= tc) unsafeAtomicAdd(C + (int64_t)tc * ldj + tr, -v);
        });
    }
}

// ---------------------------------------------------------------- queues
// Try to take the oldest published item of the high-priority queue.
__device__ __forceinline__ int try_claim_hp(const SchedArgs& a)
{
    for (int tries = 0; tries < 4; ++tries) {
        const int h = __hip_atomic_load(a.hp_head, __ATOMIC_RELAXED, AGENT);
        if (h >= a.hp_total) return -1;
        const int it = __hip_atomic_load(&a.hp_queue[h], __ATOMIC_RELAXED, AGENT);
        if (it < 0) return -1;
        int expected = h;
        if (__hip_atomic_compare_exchange_strong(a.hp_head, &expected, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 AGENT))
            return it;
    }
    return -1;
}

__device__ __forceinline__ void push_items(const SchedArgs& a, bool hp, int base, int first, int count)
{
    int32_t* q = hp ? a.hp_queue : a.queue;
    const int cap = hp ? a.hp_total : a.total_normal;
    for (int i = threadIdx.x; i < count; i += kThreads) {
        if (base + i < cap)
            __hip_atomic_store(&q[base + i], first + i, __ATOMIC_RELAXED, AGENT);
        else
            __hip_atomic_store(&a.status[1], 2, __ATOMIC_RELAXED, AGENT);   // more pushes than slots
    }
}

// ---------------------------------------------------------------- scheduler
__global__ void __launch_bounds__(kThreads, 2) sched_kernel(SchedArgs a)
{
    __shared__ double Ls[kNB * 33 + kNB];
    __shared__ double Gs[kNB * 33 * 7];
    __shared__ int rpos[256], cpos[128];
    __shared__ int s_item;
    __shared__ int s_push[6];   // {hp first, hp count, hp base, normal first, normal count, normal base}
    __shared__ int64_t s_t0, s_t1;
    const int tid = threadIdx.x;
    int my_slot = -1;   // claimed normal-queue slot not yet served (thread 0)
    for (;;) {
        if (tid == 0) {
            int item = -1;
            s_t0 = wall_clock64();
            const int64_t t0 = s_t0;
            for (;;) {
                if (__hip_atomic_load(&a.status[1], __ATOMIC_RELAXED, AGENT) != 0) { item = -1; break; }
                item = try_claim_hp(a);
                if (item >= 0) break;
                if (my_slot < 0) my_slot = __hip_atomic_fetch_add(a.qhead, 1, __ATOMIC_RELAXED, AGENT);
                if (my_slot < a.total_normal) {
                    item = __hip_atomic_load(&a.queue[my_slot], __ATOMIC_RELAXED, AGENT);
                    if (item >= 0) { my_slot = -1; break; }
                } else if (__hip_atomic_load(a.hp_head, __ATOMIC_RELAXED, AGENT) >= a.hp_total) {
                    item = -1;   // both queues exhausted
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > a.timeout_ticks) {
                    __hip_atomic_store(&a.status[1], 1, __ATOMIC_RELAXED, AGENT);
                    item = -1;
                    break;
                }
            }
            s_item = item;
            s_t1 = wall_clock64();
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) break;
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        const int4 d0 = a.desc[2 * item];
        const int4 d1 = a.desc[2 * item + 1];
        if (d0.x == kFact) task_fact(a, d0.y, Ls, Gs);
        else if (d0.x == kTrsm) task_trsm(a, d0.y, d0.z, d0.w);
        else task_update(a, d0, d1, rpos, cpos);
        // every wave's stores and atomics have completed before the barrier
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid < 64 && d0.x != kUpdate) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tid == 0) {
            int hf = 0, hc = 0, nf = 0, nc = 0;
            if (d0.x == kFact) {
                if (a.hp_cblk[d0.y]) {
                    hf = a.trsm_first[d0.y];
                    hc = a.trsm_count[d0.y];
                } else {
                    nf = a.trsm_first[d0.y];
                    nc = a.trsm_count[d0.y];
                }
            } else if (d0.x == kTrsm) {
                if (__hip_atomic_fetch_add(&a.trsm_left[d0.y], -1, __ATOMIC_RELAXED, AGENT) == 1) {
                    hf = a.upd_first[d0.y];
                    hc = a.upd_hp[d0.y];
                    nf = hf + hc;
                    nc = a.upd_count[d0.y] - hc;
                }
            } else {
                if (__hip_atomic_fetch_add(&a.fact_dep[d0.z], -1, __ATOMIC_RELAXED, AGENT) == 1) {
                    if (a.hp_cblk[d0.z]) { hf = d0.z; hc = 1; }
                    else { nf = d0.z; nc = 1; }
                }
            }
            s_push[0] = hf;
            s_push[1] = hc;
            s_push[2] = hc > 0 ? __hip_atomic_fetch_add(a.hp_tail, hc, __ATOMIC_RELAXED, AGENT) : 0;
            s_push[3] = nf;
            s_push[4] = nc;
            s_push[5] = nc > 0 ? __hip_atomic_fetch_add(a.qtail, nc, __ATOMIC_RELAXED, AGENT) : 0;
            __hip_atomic_fetch_add(&a.status[2], 1, __ATOMIC_RELAXED, AGENT);
            if (a.trace) {
                int64_t* t = a.trace + 4 * (int64_t)item;
                t[0] = s_t0;
                t[1] = s_t1;
                t[2] = wall_clock64();
                t[3] = (int64_t)__builtin_amdgcn_s_getreg((31 << 11) | 4);   // HW_ID: wave/simd/cu/se
            }
        }
        __syncthreads();
        if (s_push[1] > 0) push_items(a, true, s_push[2], s_push[0], s_push[1]);
        if (s_push[4] > 0) push_items(a, false, s_push[5], s_push[3], s_push[4]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- set-up kernels
__global__ void fill_f64(double* p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_i32(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// panels[amap[p]] = values[p] for entries read by the factorization
__global__ void assemble_kernel(double* panels, const int64_t* amap, const double* values, int64_t nnz)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = amap[p];
        if (d >= 0) panels[d] = values[p];
    }
}

// queues and counters of one factorization: the ready FACT items are the
// first entries of their queues (ready[0..nready_hp) high priority, the rest
// normal)
__global__ void sched_init(SchedArgs a, const int32_t* ready, int32_t nready, int32_t nready_hp,
                           const int32_t* fact_dep0, int32_t ncblk)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int32_t nready_n = nready - nready_hp;
    for (int64_t i = t; i < a.total_normal; i += stride) a.queue[i] = i < nready_n ? ready[nready_hp + i] : -1;
    for (int64_t i = t; i < a.hp_total; i += stride) a.hp_queue[i] = i < nready_hp ? ready[i] : -1;
    for (int64_t i = t; i < ncblk; i += stride) {
        a.fact_dep[i] = fact_dep0[i];
        a.trsm_left[i] = a.trsm_count[i];
    }
    if (t == 0) {
        *a.qhead = 0;
        *a.qtail = nready_n;
        *a.hp_head = 0;
        *a.hp_tail = nready_hp;
        a.status[0] = 0x7fffffff;
        a.status[1] = 0;
        a.status[2] = 0;
    }
}

// ---------------------------------------------------------------- host launchers
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    fill_f64<<<blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    fill_i32<<<blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_assemble(double* panels, const int64_t* amap, const double* values, int64_t nnz, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    assemble_kernel<<<blocks, 256, 0, s>>>(panels, amap, values, nnz);
    return hipGetLastError();
}

hipError_t launch_sched_init(const SchedArgs& a, const int32_t* ready, int32_t nready, int32_t nready_hp,
                             const int32_t* fact_dep0, int32_t ncblk, hipStream_t s)
{
    const int64_t n = std::max<int64_t>(std::max<int64_t>(a.total_normal, a.hp_total), ncblk);
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    sched_init<<<blocks, 256, 0, s>>>(a, ready, nready, nready_hp, fact_dep0, ncblk);
    return hipGetLastError();
}

int sched_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel, kThreads, 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_sched(const SchedArgs& a, int grid, hipStream_t s)
{
    sched_kernel<<<grid, kThreads, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace spx
