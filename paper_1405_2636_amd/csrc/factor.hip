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
// work items from a device-side ready queue:
//   FACT(k)          diagonal block Cholesky + inverses of its 32x32 tiles
//   TRSM(k, rows)    128 off-diagonal rows of panel k against L_kk^T
//   UPDATE(k,j,r,c)  64x64 tile of the outer product of panel k, subtracted
//                    into panel j with FP64 atomics
// Dependencies are counters: FACT(j) becomes ready when every UPDATE tile
// into j is done, the TRSM tiles of k when FACT(k) is done, the UPDATE tiles
// of k when its last TRSM tile is done.  Products run on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64).
#include "device.hpp"

namespace spx {

typedef double d4 __attribute__((ext_vector_type(4)));

#define AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One wave computes a 32x32 tile C(r, c) = sum_p X[r + p*ldx] * Y[c + p*ldy]
// for r < mv, c < nv, p < K (loads outside those bounds read as zero).
// The matrix-core lane layout of the f64 16x16x4 product is: operand A lane l
// holds A[l%16][l/16], operand B lane l holds B[l/16][l%16], result slot v of
// lane l holds D[4v + l/16][l%16].  Y feeds operand A and X operand B, so
//   acc[bi][bj][v] = C(16*bj + l%16, 16*bi + 4v + l/16)
// and the 16 consecutive lanes of a result slot cover 16 consecutive rows of
// C, i.e. contiguous memory of a column-major destination.
__device__ __forceinline__ void wave_gemm32(d4 (&acc)[2][2], const double* __restrict__ X, int64_t ldx, int mv,
                                            const double* __restrict__ Y, int64_t ldy, int nv, int K)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const bool x0 = li < mv, x1 = li + 16 < mv, y0 = li < nv, y1 = li + 16 < nv;
    const double* xp = X + li;
    const double* yp = Y + li;
    int p0 = 0;
    for (; p0 + 16 <= K; p0 += 16) {
        double xa[4], xb[4], ya[4], yb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t p = p0 + 4 * u + lk;
            xa[u] = x0 ? xp[p * ldx] : 0.0;
            xb[u] = x1 ? xp[16 + p * ldx] : 0.0;
            ya[u] = y0 ? yp[p * ldy] : 0.0;
            yb[u] = y1 ? yp[16 + p * ldy] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc[0][0] = mfma_f64(ya[u], xa[u], acc[0][0]);
            acc[0][1] = mfma_f64(ya[u], xb[u], acc[0][1]);
            acc[1][0] = mfma_f64(yb[u], xa[u], acc[1][0]);
            acc[1][1] = mfma_f64(yb[u], xb[u], acc[1][1]);
        }
    }
    for (; p0 < K; p0 += 4) {
        const int64_t p = p0 + lk;
        const bool pk = p < K;
        const double xa = (x0 && pk) ? xp[p * ldx] : 0.0;
        const double xb = (x1 && pk) ? xp[16 + p * ldx] : 0.0;
        const double ya = (y0 && pk) ? yp[p * ldy] : 0.0;
        const double yb = (y1 && pk) ? yp[16 + p * ldy] : 0.0;
        acc[0][0] = mfma_f64(ya, xa, acc[0][0]);
        acc[0][1] = mfma_f64(ya, xb, acc[0][1]);
        acc[1][0] = mfma_f64(yb, xa, acc[1][0]);
        acc[1][1] = mfma_f64(yb, xb, acc[1][1]);
    }
}

// Workgroup GEMM over 32x32 wave tiles (tiles dealt round-robin to the 4
// waves): for every r < m, c < n: epi(r, c, sum_p X[r + p*ldx] Y[c + p*ldy]).
// A wave tile spans 32 rows and min(32, n) columns; when n <= 32 every wave
// tile covers whole rows, which makes in-place products (X aliasing the
// destination) safe.
template <class Epi>
__device__ __forceinline__ void wg_gemm(int m, int n, int K, const double* X, int64_t ldx, const double* Y, int64_t ldy,
                                        Epi epi)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int ntr = (m + 31) >> 5, ntc = (n + 31) >> 5;
    for (int t = wave; t < ntr * ntc; t += 4) {
        const int r0 = (t % ntr) * 32, c0 = (t / ntr) * 32;
        d4 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        wave_gemm32(acc, X + r0, ldx, min(32, m - r0), Y + c0, ldy, min(32, n - c0), K);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 16 * bj + li, c = c0 + 16 * bi + 4 * v + lk;
                    if (r < m && c < n) epi(r, c, acc[bi][bj][v]);
                }
    }
}

__device__ __forceinline__ int cblk_width(const DevPlan& pl, int k) { return pl.lcol[k] - pl.fcol[k] + 1; }

// ---------------------------------------------------------------- FACT(k)
// Left-looking blocked Cholesky of the w x w diagonal block (w <= 256) by one
// workgroup: for every 32-column tile J, subtract the products of the
// already-factored columns (matrix cores), factor the 32x32 diagonal tile and
// invert it in LDS (one wave), then multiply the rows below by the inverse's
// transpose.  The inverted tiles are kept for the off-diagonal triangular
// solves and for the solve phase.  A pivot that is not > 0 records its column
// with atomicMin and the computation continues (NaN propagates), so the
// smallest failing column in elimination order is reported.
__device__ void task_fact(const SchedArgs& a, int k, double* T, double* Ti)
{
    const DevPlan& pl = a.pl;
    const int w = cblk_width(pl, k);
    const int64_t ld = pl.stride[k];
    double* A = a.panels + pl.panel_off[k];
    double* D = a.dinv + pl.dinv_off[k];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int J = 0; J < w; J += kNB) {
        const int jb = min(kNB, w - J);
        if (J > 0) {
            wg_gemm(w - J, jb, J, A + J, ld, A + J, ld,
                    [&](int r, int c, double v) { if (r >= c) A[(J + r) + (J + c) * ld] -= v; });
            __syncthreads();
        }
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            const int r = idx & 31, c = idx >> 5;
            T[r + c * 33] = (r < jb && c < jb && r >= c) ? A[(J + r) + (J + c) * ld] : 0.0;
        }
        __syncthreads();
        if (wave == 0) {
            // unblocked Cholesky of the tile; one wave, LDS accesses stay in program order
            for (int c = 0; c < jb; ++c) {
                const double d = T[c + c * 33];
                if (!(d > 0.0) && lane == 0) atomicMin(&a.status[0], pl.fcol[k] + J + c);
                const double s = sqrt(d);
                __builtin_amdgcn_wave_barrier();
                if (lane > c && lane < jb) T[lane + c * 33] /= s;
                if (lane == c) T[c + c * 33] = s;
                __builtin_amdgcn_wave_barrier();
                const int r = lane & 31;
                for (int c2 = c + 1 + (lane >> 5); c2 < jb; c2 += 2)
                    if (r >= c2 && r < jb) T[r + c2 * 33] -= T[r + c * 33] * T[c2 + c * 33];
                __builtin_amdgcn_wave_barrier();
            }
            // inverse of the lower triangular tile, one column per lane
            if (lane < kNB) {
                const int c = lane;
                for (int r = 0; r < kNB; ++r) {
                    double x = 0.0;
                    if (c < jb && r < jb && r >= c) {
                        if (r == c) {
                            x = 1.0 / T[c + c * 33];
                        } else {
                            double s = 0.0;
                            for (int p = c; p < r; ++p) s += T[r + p * 33] * Ti[p + c * 33];
                            x = -s / T[r + r * 33];
                        }
                    }
                    Ti[r + c * 33] = x;
                }
            }
        }
        __syncthreads();
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            const int r = idx & 31, c = idx >> 5;
            if (r < jb && c < jb && r >= c) A[(J + r) + (J + c) * ld] = T[r + c * 33];
            D[(J / kNB) * kNB * kNB + r + c * kNB] = Ti[r + c * 33];
        }
        const int m2 = w - J - jb;
        if (m2 > 0)
            wg_gemm(m2, jb, jb, A + (J + jb) + J * ld, ld, Ti, 33,
                    [&](int r, int c, double v) { A[(J + jb + r) + (J + c) * ld] = v; });
        __syncthreads();
    }
}

// ---------------------------------------------------------------- TRSM(k, rows)
// Rows [row0, row0+nrows) of panel k (below its diagonal block) are replaced by
// B L_kk^{-T}, 32 columns at a time: subtract the already solved columns, then
// multiply by the inverted diagonal tile's transpose.
__device__ void task_trsm(const SchedArgs& a, int k, int row0, int nrows)
{
    const DevPlan& pl = a.pl;
    const int w = cblk_width(pl, k);
    const int64_t ld = pl.stride[k];
    double* A = a.panels + pl.panel_off[k];
    const double* D = a.dinv + pl.dinv_off[k];
    double* B = A + row0;
    for (int J = 0; J < w; J += kNB) {
        const int jb = min(kNB, w - J);
        if (J > 0) {
            wg_gemm(nrows, jb, J, B, ld, A + J, ld,
                    [&](int r, int c, double v) { B[r + (J + c) * ld] -= v; });
            __syncthreads();
        }
        wg_gemm(nrows, jb, jb, B + J * ld, ld, D + (J / kNB) * kNB * kNB, kNB,
                [&](int r, int c, double v) { B[r + (J + c) * ld] = v; });
        __syncthreads();
    }
}

// position of panel row r of cblk k: its global row index
__device__ __forceinline__ int global_row(const DevPlan& pl, int k, int r)
{
    const int w = cblk_width(pl, k);
    if (r < w) return pl.fcol[k] + r;
    int lo = pl.bptr[k] + 1, hi = pl.bptr[k + 1] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pl.coefind[mid] <= r) lo = mid; else hi = mid - 1;
    }
    return pl.frow[lo] + (r - pl.coefind[lo]);
}

// position inside panel j of global row g (g belongs to j's structure)
__device__ __forceinline__ int target_row(const DevPlan& pl, int j, int g)
{
    if (g <= pl.lcol[j] || pl.bptr[j + 1] - pl.bptr[j] < 2) return g - pl.fcol[j];
    int lo = pl.bptr[j] + 1, hi = pl.bptr[j + 1] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pl.frow[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return pl.coefind[lo] + (g - pl.frow[lo]);
}

// ---------------------------------------------------------------- UPDATE(k, j, tile)
// W = L_k[row0 : row0+mrows] * L_k[col0 : col0+ncols]^T (K = width of k) and
// C_j[target rows, target cols] -= W, lower triangle of j only.  Row and
// column maps are resolved once per tile into LDS.
__device__ void task_update(const SchedArgs& a, int k, int j, int row0, int col0, int ncols, int mrows,
                            int* rpos, int* rglob, int* cpos, int* cglob)
{
    const DevPlan& pl = a.pl;
    const int w = cblk_width(pl, k);
    const int64_t ld = pl.stride[k];
    const double* A = a.panels + pl.panel_off[k];
    double* C = a.panels + pl.panel_off[j];
    const int64_t ldj = pl.stride[j];
    const int tid = threadIdx.x;
    if (tid < kTile) {
        if (tid < mrows) {
            const int g = global_row(pl, k, row0 + tid);
            rglob[tid] = g;
            rpos[tid] = target_row(pl, j, g);
        }
    } else if (tid < 2 * kTile) {
        const int c = tid - kTile;
        if (c < ncols) {
            const int g = global_row(pl, k, col0 + c);
            cglob[c] = g;
            cpos[c] = g - pl.fcol[j];
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int r0 = 32 * (wave & 1), c0 = 32 * (wave >> 1);
    if (r0 < mrows && c0 < ncols) {
        d4 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[i][q] = d4{0.0, 0.0, 0.0, 0.0};
        wave_gemm32(acc, A + row0 + r0, ld, min(32, mrows - r0), A + col0 + c0, ld, min(32, ncols - c0), w);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = r0 + 16 * bj + li, c = c0 + 16 * bi + 4 * v + lk;
                    if (r < mrows && c < ncols && rglob[r] >= cglob[c])
                        unsafeAtomicAdd(C + cpos[c] * ldj + rpos[r], -acc[bi][bj][v]);
                }
    }
}

// ---------------------------------------------------------------- scheduler
__global__ void __launch_bounds__(kThreads) sched_kernel(SchedArgs a)
{
    __shared__ double T[kNB * 33];
    __shared__ double Ti[kNB * 33];
    __shared__ int rpos[kTile], rglob[kTile], cpos[kTile], cglob[kTile];
    __shared__ int s_item, s_first, s_count, s_base;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            int item = -1;
            if (__hip_atomic_load(&a.status[1], __ATOMIC_RELAXED, AGENT) == 0) {
                const int slot = __hip_atomic_fetch_add(a.qhead, 1, __ATOMIC_RELAXED, AGENT);
                if (slot < a.total) {
                    const int64_t t0 = wall_clock64();
                    for (;;) {
                        item = __hip_atomic_load(&a.queue[slot], __ATOMIC_RELAXED, AGENT);
                        if (item >= 0) break;
                        __builtin_amdgcn_s_sleep(2);
                        if (__hip_atomic_load(&a.status[1], __ATOMIC_RELAXED, AGENT) != 0) break;
                        if (wall_clock64() - t0 > a.timeout_ticks) {
                            __hip_atomic_store(&a.status[1], 1, __ATOMIC_RELAXED, AGENT);
                            break;
                        }
                    }
                }
            }
            s_item = item;
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int4 d0 = a.desc[2 * item];
        const int4 d1 = a.desc[2 * item + 1];
        if (d0.x == kFact) task_fact(a, d0.y, T, Ti);
        else if (d0.x == kTrsm) task_trsm(a, d0.y, d0.z, d0.w);
        else task_update(a, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, rpos, rglob, cpos, cglob);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tid == 0) {
            int first = 0, count = 0;
            if (d0.x == kFact) {
                first = a.trsm_first[d0.y];
                count = a.trsm_count[d0.y];
            } else if (d0.x == kTrsm) {
                if (__hip_atomic_fetch_add(&a.trsm_left[d0.y], -1, __ATOMIC_ACQ_REL, AGENT) == 1) {
                    first = a.upd_first[d0.y];
                    count = a.upd_count[d0.y];
                }
            } else {
                if (__hip_atomic_fetch_add(&a.fact_dep[d0.z], -1, __ATOMIC_ACQ_REL, AGENT) == 1) {
                    first = d0.z;
                    count = 1;
                }
            }
            int base = 0;
            if (count > 0) base = __hip_atomic_fetch_add(a.qtail, count, __ATOMIC_RELAXED, AGENT);
            __hip_atomic_fetch_add(&a.status[2], 1, __ATOMIC_RELAXED, AGENT);
            s_first = first;
            s_count = count;
            s_base = base;
        }
        __syncthreads();
        if (s_count > 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (int i = tid; i < s_count; i += kThreads) {
                if (s_base + i < a.total)
                    __hip_atomic_store(&a.queue[s_base + i], s_first + i, __ATOMIC_RELAXED, AGENT);
                else
                    __hip_atomic_store(&a.status[1], 2, __ATOMIC_RELAXED, AGENT);   // more pushes than items
            }
        }
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

// queue and counters of one factorization
__global__ void sched_init(int32_t* queue, int32_t total, const int32_t* ready, int32_t nready, int32_t* fact_dep,
                           const int32_t* fact_dep0, int32_t* trsm_left, const int32_t* trsm_count, int32_t ncblk,
                           int32_t* qhead, int32_t* qtail, int32_t* status)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += stride)
        queue[i] = i < nready ? ready[i] : -1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ncblk; i += stride) {
        fact_dep[i] = fact_dep0[i];
        trsm_left[i] = trsm_count[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *qhead = 0;
        *qtail = nready;
        status[0] = 0x7fffffff;
        status[1] = 0;
        status[2] = 0;
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

hipError_t launch_sched_init(int32_t* queue, int32_t total, const int32_t* ready, int32_t nready, int32_t* fact_dep,
                             const int32_t* fact_dep0, int32_t* trsm_left, const int32_t* trsm_count, int32_t ncblk,
                             int32_t* qhead, int32_t* qtail, int32_t* status, hipStream_t s)
{
    const int64_t n = std::max<int64_t>(total, ncblk);
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    sched_init<<<blocks, 256, 0, s>>>(queue, total, ready, nready, fact_dep, fact_dep0, trsm_left, trsm_count, ncblk,
                                      qhead, qtail, status);
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
