// Triangular solves with the supernodal factor, FP64 residual and the
// refinement helpers (the solve phase of A x = b; the paper states the
// problem, the sweeps are the standard supernodal ones).
//
// Forward sweep, column blocks in ascending dependency levels:
//   z_k = L_kk^{-1} y_k                   (diagonal rows split over workgroups)
//   y[rows of k] -= L_k,off z_k           (64-row chunks, FP64 atomics)
// Backward sweep, levels descending:
//   t_k  = L_k,off^T x[rows of k]         (64- or 256-row chunks)
//   x_k  = L_kk^{-T} (z_k - t_k)
// Both use the inverse of each diagonal block kept by the factorization.
// On the narrow levels two consecutive pieces p, q of a split supernode are
// one block of the sweeps: the diagonal steps use the pair's inverse
// (pair_inv, formed after each factorization), so p's rows facing q are left
// out of its off-diagonal steps.  Every launch reads its work from a list of
// self-contained items (DiagItem, OffItem) built once per analysis.
// Several right-hand sides are handled in blocks of up to 8 per pass over
// the panels (each loaded entry serves the whole block); with 4 or 8 the
// off-diagonal steps are matrix-core products (fwd_off_mm, bwd_off_mm).
// Column blocks of width <= 32 with at most 128 panel rows take both halves
// of a step in one kernel per level, a group of 16 lanes per block
// (fwd_small, bwd_small).
// Every sweep step writes a different vector than it reads (y -> z -> x), so
// a diagonal block can be spread over several workgroups.  Every dot product
// is split over four lanes (interleaved inner indices) and combined by two
// shuffles: the dependent load rounds per thread are a quarter of a
// one-lane loop.  The sweeps stream the panels once each: they are bound by
// HBM bandwidth and, on the narrow top levels, by load latency.
// The factor is read in its storage type T (double, or float in the FP32
// refinement mode); vectors and arithmetic are FP64 in both cases.
// L U (unit L and U in the square diagonal blocks, L below them, U^T in a
// second panel array of the same layout, kept inverses L_kk^{-1} and
// U_kk^{-T}): the forward sweep reads L and L_kk^{-1}, the backward sweep the
// U^T panels and U_kk^{-T} (x_k = U_kk^{-1} (z_k - t_k), t_k = U_k,off x[rows])
// in the places of L and L_kk^{-1}.
// L D L^T (unit L, d_j on the panel diagonal, kept inverse Y = D^{-1} L^{-1}):
// the same steps give w_k = Y_kk y_k = D_k^{-1} z_k in z, so the forward rows
// below take D_k w_k, and the backward step x_k = L_kk^{-T} (w_k - t_k) is
// Y_kk^T applied to D_k (w_k - t_k); the scaling by d is applied where z_k
// and z_k - t_k are staged.
#include "device.hpp"

namespace spx {

constexpr int kChunk = 64;     // off-diagonal rows per chunk of the level lists

// sum over the LANES consecutive lanes of a group (LANES = 4, 16 or 32)
template <int LANES>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

// Every sweep kernel handles the right-hand sides in blocks of NR (1, 4 or
// 8, the small-block kernels 1 or 2; chosen from nrhs at launch): the panel and inverse entries a thread
// loads serve all NR columns of the block, so a panel is read once per
// block of right-hand sides instead of once per right-hand side.  The
// diagonal and off-diagonal kernels take one block per grid row (a loop
// over the blocks kept the loop-invariant addresses of the hoisted loads
// live: 150-210 registers per lane instead of 85-135, and half the
// resident waves).
// (staged vectors: element c of right-hand side j at [c * NR + j]; a masked
// term is formed as 0 * value, so clamped indices stay inside the staged
// entries: a value read from unwritten LDS may be NaN)

// ---- forward, diagonal block: z_k = D y_k, D = L_kk^{-1} (lower, w x w,
// column-major).  LANES lanes per row, one workgroup per item: the rows
// r0 .. r0 + 256/LANES - 1 of one block; lane q of a row takes the
// columns p = q, q+LANES, ..., sixteen loads at a time (p > row clamped and
// multiplied by zero).  Narrow levels (few blocks) use 16 lanes, or 32 when
// they hold a pair of pieces (a 512-wide inverse): fewer dependent load
// rounds; wide levels 4 (the items of a level are cut to match).
template <class T, int LANES, int NR>
__global__ void __launch_bounds__(256) fwd_diag(SweepArgs a, const DiagItem* items)
{
    __shared__ double ys[kMaxPairWidth * NR];
    const DiagItem it = items[blockIdx.x];
    const int f = it.f, w = it.w, r0 = it.r0;
    const T* D = static_cast<const T*>(a.dinv) + it.dofs;
    const int tid = threadIdx.x, q = tid % LANES, row = min(r0 + tid / LANES, w - 1);
    {   // the grid row's block of right-hand sides
        const int rb = blockIdx.y * NR;
        const int nv = min(NR, a.nrhs - rb);
        T d[16];   // the first sixteen loads are issued before the staging barrier
#pragma unroll
        for (int u = 0; u < 16; ++u) d[u] = D[(uint32_t)(row + min(q + LANES * u, row) * w)];
        for (int idx = tid; idx < w * NR; idx += 256) {
            const int c = idx / NR, j = idx - c * NR;
            ys[idx] = j < nv ? a.y[(int64_t)(rb + j) * a.n + f + c] : 0.0;
        }
        __syncthreads();
        double v[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) v[j] = 0.0;
        for (int pb = 0; pb <= row; pb += 16 * LANES) {
            if (pb != 0) {
#pragma unroll
                for (int u = 0; u < 16; ++u) d[u] = D[(uint32_t)(row + min(pb + q + LANES * u, row) * w)];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int p = pb + q + LANES * u;
                const double dv = p <= row ? (double)d[u] : 0.0;
                const double* yp = ys + min(p, w - 1) * NR;
#pragma unroll
                for (int j = 0; j < NR; ++j) v[j] += dv * yp[j];
            }
        }
#pragma unroll
        for (int j = 0; j < NR; ++j) v[j] = group_sum<LANES>(v[j]);
        if (r0 + tid / LANES < w && q == 0)
            for (int j = 0; j < nv; ++j) a.z[(int64_t)(rb + j) * a.n + f + row] = v[j];
        __syncthreads();
    }
}

// ---- forward, off-diagonal rows: y[g(r)] -= sum_c L[r, c] z_k[c].  One
// workgroup per item: up to 64 panel rows from row0 by the columns
// c0..c1-1 (levels with few row chunks split each chunk's columns over
// several items so that the launch fills the chip; their partial sums meet
// in the atomics).  Lane = row (each load covers 64 consecutive rows of one
// column), wave v = quarter v of the columns, issued 16 at a time, the
// first sixteen before the staging barrier; the four partial sums meet in
// LDS.
template <class T, int NR>
__global__ void __launch_bounds__(256) fwd_off(SweepArgs a, const OffItem* items)
{
    __shared__ double zk[256 * NR];
    __shared__ double part[4 * 64 * NR];
    const OffItem it = items[blockIdx.x];
    const int f = it.f, c0 = it.cnr & 511, c1 = (it.cnr >> 9) & 511, nr = it.cnr >> 18;
    const int64_t ld = it.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = min(lane, nr - 1);
    const int gi = a.rowg[it.gofs + r];   // global row of the lane's panel row (read ahead of the products)
    const int qw = (c1 - c0 + 3) >> 2, cb = c0 + wave * qw, ce = min(c1, cb + qw);
    const T* Lr = static_cast<const T*>(a.panels) + it.pofs + r;
    const T* Pd = static_cast<const T*>(a.panels) + (it.pofs - it.row0);   // d_c at c * (ld + 1) (L D L^T)
    {   // the grid row's block of right-hand sides
        const int rb = blockIdx.y * NR;
        const int nv = min(NR, a.nrhs - rb);
        T l[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) l[u] = Lr[(int64_t)min(cb + u, c1 - 1) * ld];
        for (int idx = tid; idx < (c1 - c0) * NR; idx += 256) {
            const int c = c0 + idx / NR, j = idx % NR;
            zk[idx] = j < nv ? a.z[(int64_t)(rb + j) * a.n + f + c] * (a.ldlt ? (double)Pd[c * (ld + 1)] : 1.0) : 0.0;
        }
        __syncthreads();
        double v[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) v[j] = 0.0;
        for (int c = cb; c < ce; c += 16) {
            if (c != cb) {
#pragma unroll
                for (int u = 0; u < 16; ++u) l[u] = Lr[(int64_t)min(c + u, ce - 1) * ld];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const double lv = c + u < ce ? (double)l[u] : 0.0;
                const double* zc = zk + (min(c + u, ce - 1) - c0) * NR;
#pragma unroll
                for (int j = 0; j < NR; ++j) v[j] += lv * zc[j];
            }
        }
#pragma unroll
        for (int j = 0; j < NR; ++j) part[(wave * 64 + lane) * NR + j] = v[j];
        __syncthreads();
        if (wave == 0 && lane < nr) {
            for (int j = 0; j < nv; ++j) {
                const double sum = (part[lane * NR + j] + part[(64 + lane) * NR + j]) +
                                   (part[(128 + lane) * NR + j] + part[(192 + lane) * NR + j]);
                unsafeAtomicAdd(a.y + (int64_t)(rb + j) * a.n + gi, -sum);
            }
        }
        __syncthreads();
    }
}

// ---- backward, off-diagonal rows: tacc[f + c] += sum_r L[r, c] x[g(r)].
// One workgroup per item: up to 16 LANES panel rows from row0 by the
// columns c0 .. c1 - 1, 256 / LANES columns at a time; LANES lanes per
// column, lane q takes the rows q, q + LANES, ... with all sixteen loads in
// flight (the first block's before the staging barrier).  LANES = 4: 64-row
// items, the forward kernel's (wide levels: many blocks, few rows each);
// LANES = 16: 256-row items of 16 columns (narrow levels with one
// right-hand side; their blocks have thousands of rows: a column of tacc
// then takes one atomic add per 256 rows instead of per 64, and each load
// instruction covers 16 consecutive rows of four columns instead of four
// rows of sixteen).
template <class T, int LANES, int NR>
__global__ void __launch_bounds__(256) bwd_off(SweepArgs a, const OffItem* items)
{
    constexpr int COLS = 256 / LANES, ROWS = 16 * LANES, NST = (ROWS * NR + 255) / 256;
    __shared__ double xr[ROWS * NR];
    const OffItem it = items[blockIdx.x];
    const int f = it.f, c0 = it.cnr & 511, c1 = (it.cnr >> 9) & 511, nr = it.cnr >> 18;
    const int64_t ld = it.ld;
    const int32_t* g = a.rowg + it.gofs;
    const int tid = threadIdx.x, q = tid % LANES, cl = tid / LANES;
    const T* L = static_cast<const T*>(a.panels_b) + it.pofs;
    // global rows of the thread's staged entries (staged entry idx = tid +
    // 256 i holds row idx / NR), loaded ahead of the panel: the gather then
    // waits for them only, not for the panel loads issued after them
    int gv[NST];
#pragma unroll
    for (int i = 0; i < NST; ++i) gv[i] = g[min((tid + 256 * i) / NR, nr - 1)];
    {   // the grid row's block of right-hand sides
        const int rb = blockIdx.y * NR;
        const int nv = min(NR, a.nrhs - rb);
        T l[16];
        {
            const T* Lc = L + (int64_t)min(c0 + cl, c1 - 1) * ld;
#pragma unroll
            for (int u = 0; u < 16; ++u) l[u] = Lc[min(q + LANES * u, nr - 1)];
        }
#pragma unroll
        for (int i = 0; i < NST; ++i) {
            const int idx = tid + 256 * i, j = idx % NR;
            if (idx < nr * NR) xr[idx] = j < nv ? a.x[(int64_t)(rb + j) * a.n + gv[i]] : 0.0;
        }
        __syncthreads();
        for (int cb = c0; cb < c1; cb += COLS) {
            const int c = min(cb + cl, c1 - 1);
            if (cb != c0) {
                const T* Lc = L + (int64_t)c * ld;
#pragma unroll
                for (int u = 0; u < 16; ++u) l[u] = Lc[min(q + LANES * u, nr - 1)];
            }
            double v[NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) v[j] = 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const double lv = q + LANES * u < nr ? (double)l[u] : 0.0;
                const double* xp = xr + min(q + LANES * u, nr - 1) * NR;
#pragma unroll
                for (int j = 0; j < NR; ++j) v[j] += lv * xp[j];
            }
#pragma unroll
            for (int j = 0; j < NR; ++j) v[j] = group_sum<LANES>(v[j]);
            if (cb + cl < c1 && q == 0)
                for (int j = 0; j < nv; ++j) unsafeAtomicAdd(a.tacc + (int64_t)(rb + j) * a.n + f + c, v[j]);
        }
        __syncthreads();
    }
}

// ---- off-diagonal steps for blocks of NR = 4 or 8 right-hand sides, on
// the matrix cores (v_mfma_f64_16x16x4f64: operand A lane l holds
// A[l%16][l/16], operand B lane l holds B[l/16][l%16], result slot v of
// lane l holds D[4v + l/16][l%16]); FP32 panels are converted, so the
// arithmetic stays FP64.  With several right-hand sides the scalar kernels
// spend a product and an LDS read per loaded entry and right-hand side:
// they were bound by that, not by the panel bytes.
typedef double sw_d4 __attribute__((ext_vector_type(4)));

// forward: y[g(r)] -= (L z)[r] over the item's 64 rows and columns c0..c1.
// Wave v takes a quarter of the columns, all four 16-row tiles (A = panel
// rows, B = the staged z, right-hand sides past NR zero); the four waves'
// partial sums meet in LDS.
template <class T, int NR>
__global__ void __launch_bounds__(256) fwd_off_mm(SweepArgs a, const OffItem* items)
{
    __shared__ double zk[256 * NR];
    __shared__ double part[4 * 64 * NR];
    const OffItem it = items[blockIdx.x];
    const int f = it.f, c0 = it.cnr & 511, c1 = (it.cnr >> 9) & 511, nr = it.cnr >> 18;
    const int64_t ld = it.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int rb = blockIdx.y * NR, nv = min(NR, a.nrhs - rb);
    const int qw = (((c1 - c0 + 3) >> 2) + 3) & ~3;   // a wave's columns, a multiple of 4
    const int cb = c0 + wave * qw, ce = min(c1, cb + qw);
    const T* L = static_cast<const T*>(a.panels) + it.pofs;
    const T* Pd = static_cast<const T*>(a.panels) + (it.pofs - it.row0);   // d_c at c * (ld + 1) (L D L^T)
    for (int idx = tid; idx < (c1 - c0) * NR; idx += 256) {
        const int c = c0 + idx / NR, j = idx % NR;
        zk[idx] = j < nv ? a.z[(int64_t)(rb + j) * a.n + f + c] * (a.ldlt ? (double)Pd[c * (ld + 1)] : 1.0) : 0.0;
    }
    __syncthreads();
    sw_d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = sw_d4{0, 0, 0, 0};
    // (columns past ce read a clamped column and meet B = 0; rows past nr
    // read a clamped row whose results are not stored)
    for (int k0 = cb; k0 < ce; k0 += 16) {
        T al[4][4];
        double bz[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int c = k0 + 4 * s + lk;
            const int cc = min(c, ce - 1);
            bz[s] = (c < ce && li < NR) ? zk[(cc - c0) * NR + li] : 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) al[t][s] = L[min(16 * t + li, nr - 1) + (int64_t)cc * ld];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)al[t][s], bz[s], acc[t], 0, 0, 0);
    }
    if (li < NR)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[(wave * 64 + 16 * t + 4 * v + lk) * NR + li] = acc[t][v];
    __syncthreads();
    for (int idx = tid; idx < nr * NR; idx += 256) {
        const int r = idx / NR, j = idx % NR;
        if (j < nv) {
            const double sum = (part[r * NR + j] + part[(64 + r) * NR + j]) +
                               (part[(128 + r) * NR + j] + part[(192 + r) * NR + j]);
            unsafeAtomicAdd(a.y + (int64_t)(rb + j) * a.n + a.rowg[it.gofs + r], -sum);
        }
    }
}

// backward: tacc[f + c] += (L^T x)[c] over the item's rows.  A = the staged
// x (right-hand side by row, rows past nr zero), B = 16 panel columns; wave
// v takes the column tiles c0 + 16 v, c0 + 16 (v + 4), ...
template <class T, int NR>
__global__ void __launch_bounds__(256) bwd_off_mm(SweepArgs a, const OffItem* items)
{
    __shared__ double xr[kChunk * NR];
    const OffItem it = items[blockIdx.x];
    const int f = it.f, c0 = it.cnr & 511, c1 = (it.cnr >> 9) & 511, nr = it.cnr >> 18;
    const int64_t ld = it.ld;
    const int32_t* g = a.rowg + it.gofs;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int rb = blockIdx.y * NR, nv = min(NR, a.nrhs - rb);
    const T* L = static_cast<const T*>(a.panels_b) + it.pofs;
    for (int idx = tid; idx < kChunk * NR; idx += 256) {
        const int r = idx / NR, j = idx % NR;
        xr[idx] = (r < nr && j < nv) ? a.x[(int64_t)(rb + j) * a.n + g[r]] : 0.0;
    }
    __syncthreads();
    double ax[16];   // A[rhs = li][row = 4 s + lk]
#pragma unroll
    for (int s = 0; s < 16; ++s) ax[s] = li < NR ? xr[(4 * s + lk) * NR + li] : 0.0;
    for (int cb = c0 + 16 * wave; cb < c1; cb += 64) {
        const T* Lc = L + (int64_t)min(cb + li, c1 - 1) * ld;
        T bl[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) bl[s] = Lc[min(4 * s + lk, nr - 1)];
        sw_d4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], (double)bl[s], acc, 0, 0, 0);
        if (cb + li < c1)
#pragma unroll
            for (int v = 0; v < NR / 4; ++v)
                if (4 * v + lk < nv) unsafeAtomicAdd(a.tacc + (int64_t)(rb + 4 * v + lk) * a.n + f + cb + li, acc[v]);
    }
}

// ---- backward, diagonal block: x_k = D^T (z_k - t_k); LANES lanes per
// column c of D, lane q takes the rows p = c+q, c+q+LANES, ... (p >= w
// clamped and multiplied by zero); the forward kernel's items, columns
// r0 .. r0 + 256/LANES - 1
template <class T, int LANES, int NR>
__global__ void __launch_bounds__(256) bwd_diag(SweepArgs a, const DiagItem* items)
{
    __shared__ double zs[kMaxPairWidth * NR];
    const DiagItem it = items[blockIdx.x];
    const int f = it.f, w = it.w, c0 = it.r0;
    const T* D = static_cast<const T*>(a.dinv_b) + it.dofs;
    const int tid = threadIdx.x, q = tid % LANES, col = min(c0 + tid / LANES, w - 1);
    const T* Pd = static_cast<const T*>(a.panels) + it.pofs;    // L D L^T: d_c, c < w1, at c * (ld + 1)
    const T* Pd2 = static_cast<const T*>(a.panels) + it.pofs2;  // and c >= w1 at (c - w1) * (ld2 + 1)
    const int64_t ld = it.ld, ld2 = it.ld2;
    const int w1 = it.w1;
    {   // the grid row's block of right-hand sides
        const int rb = blockIdx.y * NR;
        const int nv = min(NR, a.nrhs - rb);
        T d[16];   // the first sixteen loads are issued before the staging barrier
#pragma unroll
        for (int u = 0; u < 16; ++u) d[u] = D[(uint32_t)(col * w + min(col + q + LANES * u, w - 1))];
        for (int idx = tid; idx < w * NR; idx += 256) {
            const int c = idx / NR, j = idx - c * NR;
            const int64_t o = (int64_t)(rb + j) * a.n + f + c;
            const double dc = !a.ldlt ? 1.0 : (double)(c < w1 ? Pd[c * (ld + 1)] : Pd2[(c - w1) * (ld2 + 1)]);
            zs[idx] = j < nv ? (a.z[o] - a.tacc[o]) * dc : 0.0;
        }
        __syncthreads();
        double v[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) v[j] = 0.0;
        for (int pb = col; pb < w; pb += 16 * LANES) {
            if (pb != col) {
#pragma unroll
                for (int u = 0; u < 16; ++u) d[u] = D[(uint32_t)(col * w + min(pb + q + LANES * u, w - 1))];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int p = pb + q + LANES * u;
                const double dv = p < w ? (double)d[u] : 0.0;
                const double* zp = zs + min(p, w - 1) * NR;
#pragma unroll
                for (int j = 0; j < NR; ++j) v[j] += dv * zp[j];
            }
        }
#pragma unroll
        for (int j = 0; j < NR; ++j) v[j] = group_sum<LANES>(v[j]);
        if (c0 + tid / LANES < w && q == 0)
            for (int j = 0; j < nv; ++j) a.x[(int64_t)(rb + j) * a.n + f + col] = v[j];
        __syncthreads();
    }
}

// ---- small blocks (width <= 32, at most 128 panel rows), both halves of a
// sweep step in one kernel per level: a group of 16 lanes per block, 16 blocks per
// workgroup (the bottom levels of small systems hold tens of thousands of
// blocks a few columns wide; one workgroup per block would leave most of
// each workgroup idle and the launch bound by workgroup dispatch).
constexpr int kSG = 16;                    // lanes per small block
constexpr int kSGroups = 256 / kSG;        // small blocks per workgroup

// forward: z_k = D y_k, then y[g(r)] -= L[r, :] z_k for the rows below
constexpr int kMaxPass = (128 + kSG - 1) / kSG;   // rows below per lane, at most

template <class T, int NR>
__global__ void __launch_bounds__(256) fwd_small(SweepArgs a, const int32_t* cblks, int count)
{
    __shared__ double ys[kSGroups][32 * NR];
    __shared__ double zs[kSGroups][32 * NR];
    const int tid = threadIdx.x, g = tid / kSG, l = tid % kSG;
    const int idx = blockIdx.x * kSGroups + g;
    const bool on = idx < count;
    const int k = cblks[on ? idx : count - 1];
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k];
    const int w = on ? pl.lcol[k] - f + 1 : 0;
    const int ld = on ? pl.stride[k] : 0;
    const T* D = static_cast<const T*>(a.dinv) + pl.dinv_off[k];
    const T* L = static_cast<const T*>(a.panels) + pl.panel_off[k];
    const int32_t* rg = a.rowg + a.rowg_off[k] - w;   // rg[r]: global row of panel row r >= w
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        const int nv = min(NR, a.nrhs - rb);
        for (int r = l; r < w; r += kSG)
#pragma unroll
            for (int j = 0; j < NR; ++j) ys[g][r * NR + j] = j < nv ? a.y[(int64_t)(rb + j) * a.n + f + r] : 0.0;
        __syncthreads();
        // (indices past the triangle or the panel are clamped; their terms
        // are multiplied by zero, so the loads of a round are unconditional)
        for (int r = l; r < w; r += kSG) {
            double v[NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) v[j] = 0.0;
#pragma unroll 1
            for (int p0 = 0; p0 <= r; p0 += 8) {
                T d[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) d[u] = D[r + min(p0 + u, r) * w];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double dv = p0 + u <= r ? (double)d[u] : 0.0;
                    const double* yp = &ys[g][min(p0 + u, r) * NR];
#pragma unroll
                    for (int j = 0; j < NR; ++j) v[j] += dv * yp[j];
                }
            }
            const double s = a.ldlt ? (double)L[r * (ld + 1)] : 1.0;
#pragma unroll
            for (int j = 0; j < NR; ++j) zs[g][r * NR + j] = v[j] * s;
            for (int j = 0; j < nv; ++j) a.z[(int64_t)(rb + j) * a.n + f + r] = v[j];
        }
        __syncthreads();
        if (ld > w) {
            double v[kMaxPass][NR];
#pragma unroll
            for (int i = 0; i < kMaxPass; ++i)
#pragma unroll
                for (int j = 0; j < NR; ++j) v[i][j] = 0.0;
#pragma unroll 1
            for (int c0 = 0; c0 < w; c0 += 4) {
                T lv[4][kMaxPass];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int i = 0; i < kMaxPass; ++i)
                        lv[u][i] = L[min(w + l + kSG * i, ld - 1) + (int64_t)min(c0 + u, w - 1) * ld];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool cu = c0 + u < w;
                    const double* zp = &zs[g][min(c0 + u, 31) * NR];
#pragma unroll
                    for (int j = 0; j < NR; ++j) {
                        const double z = cu ? zp[j] : 0.0;
#pragma unroll
                        for (int i = 0; i < kMaxPass; ++i) v[i][j] += (double)lv[u][i] * z;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < kMaxPass; ++i) {
                const int r = w + l + kSG * i;
                if (r < ld)
                    for (int j = 0; j < nv; ++j) unsafeAtomicAdd(a.y + (int64_t)(rb + j) * a.n + rg[r], -v[i][j]);
            }
        }
        __syncthreads();
    }
}

// backward: t = L_off^T x[g(rows below)] (sums over the group's lanes),
// then x_k = D^T (z_k - t)
template <class T, int NR>
__global__ void __launch_bounds__(256) bwd_small(SweepArgs a, const int32_t* cblks, int count)
{
    __shared__ double us[kSGroups][32 * NR];
    const int tid = threadIdx.x, g = tid / kSG, l = tid % kSG;
    const int idx = blockIdx.x * kSGroups + g;
    const bool on = idx < count;
    const int k = cblks[on ? idx : count - 1];
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k];
    const int w = on ? pl.lcol[k] - f + 1 : 0;
    const int ld = on ? pl.stride[k] : 0;
    const T* D = static_cast<const T*>(a.dinv_b) + pl.dinv_off[k];
    const T* L = static_cast<const T*>(a.panels_b) + pl.panel_off[k];
    const int32_t* rg = a.rowg + a.rowg_off[k] - w;
    for (int rb = 0; rb < a.nrhs; rb += NR) {
        const int nv = min(NR, a.nrhs - rb);
        double xr[kMaxPass][NR];
#pragma unroll
        for (int i = 0; i < kMaxPass; ++i) {
            const int r = w + l + kSG * i;
#pragma unroll
            for (int j = 0; j < NR; ++j) xr[i][j] = (r < ld && j < nv) ? a.x[(int64_t)(rb + j) * a.n + rg[r]] : 0.0;
        }
        // (xr is zero for rows past the panel: their clamped loads count zero)
#pragma unroll 1
        for (int c0 = 0; c0 < w; c0 += 4) {
            double v[4][NR];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                T lv[kMaxPass];
#pragma unroll
                for (int i = 0; i < kMaxPass; ++i)
                    lv[i] = L[min(w + l + kSG * i, ld - 1) + (int64_t)min(c0 + u, w - 1) * ld];
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    double t = 0.0;
#pragma unroll
                    for (int i = 0; i < kMaxPass; ++i) t += (double)lv[i] * xr[i][j];
                    v[u][j] = group_sum<kSG>(t);
                }
            }
            if (l < 4 && c0 + l < w) {
                const double s = a.ldlt ? (double)L[(c0 + l) * (ld + 1)] : 1.0;
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    const double t = l == 0 ? v[0][j] : l == 1 ? v[1][j] : l == 2 ? v[2][j] : v[3][j];
                    const double u = j < nv ? a.z[(int64_t)(rb + j) * a.n + f + c0 + l] - t : 0.0;
                    us[g][(c0 + l) * NR + j] = u * s;
                }
            }
        }
        __syncthreads();
        for (int c = l; c < w; c += kSG) {
            double v[NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) v[j] = 0.0;
#pragma unroll 1
            for (int p0 = c; p0 < w; p0 += 8) {
                T d[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) d[u] = D[min(p0 + u, w - 1) + c * w];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double dv = p0 + u < w ? (double)d[u] : 0.0;
                    const double* up = &us[g][min(p0 + u, w - 1) * NR];
#pragma unroll
                    for (int j = 0; j < NR; ++j) v[j] += dv * up[j];
                }
            }
            for (int j = 0; j < nv; ++j) a.x[(int64_t)(rb + j) * a.n + f + c] = v[j];
        }
        __syncthreads();
    }
}

// ---- vector kernels
__global__ void permute_in(double* y, const double* b, int64_t ldb, const int32_t* perm, int32_t n, int32_t nrhs)
{
    const int64_t tot = (int64_t)n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / n, i = t - c * n;
        y[t] = b[c * ldb + perm[i]];
    }
}

__global__ void permute_out(double* x, int64_t ldx, const double* y, const int32_t* perm, int32_t n, int32_t nrhs)
{
    const int64_t tot = (int64_t)n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / n, i = t - c * n;
        x[c * ldx + perm[i]] = y[t];
    }
}

__global__ void zero_u64(unsigned long long* p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

__global__ void axpy_kernel(double* x, const double* d, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += d[i];
}

// order-preserving bits of a non-negative double (NaN is treated as +inf)
__device__ __forceinline__ unsigned long long key_of(double v)
{
    if (v != v) v = __builtin_inf();
    return (unsigned long long)__double_as_longlong(v);
}

__device__ __forceinline__ unsigned long long block_max(unsigned long long v)
{
    __shared__ unsigned long long sm[4];
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    unsigned long long r = sm[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = sm[i] > r ? sm[i] : r;
    __syncthreads();
    return r;
}

// r = b - A x and componentwise / normwise error statistics, in FP64.
// A is read through the symmetric row pattern (rptr, rcol) with its values rv
// in the same order (the input's lower triangle mirrored, gathered once per
// factorization by gather_kernel so that the residual reads them in order).
// stats[0] = max_i |r_i| / (|A||x| + |b|)_i   (0/0 = 0, p/0 = inf)
// stats[1] = max |r_i|, stats[2] = max |x_i|, stats[3] = max |b_i|, stats[4] = max_i sum_j |a_ij|
// (stats[q] at word q * kStatStride: every block adds its maxima by atomics,
// one cache line per statistic; a fixed grid of kResidualBlocks blocks)
__global__ void __launch_bounds__(256) residual_kernel(const int64_t* rptr, const int32_t* rcol, const double* rv,
                                                       const double* x, const double* b,
                                                       int64_t ldb, double* r, int32_t n, int32_t nrhs,
                                                       unsigned long long* stats)
{
    unsigned long long m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
    const int64_t tot = (int64_t)n * nrhs;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = t / n, i = t - c * n;
        const double* xc = x + c * n;
        const double bi = b[c * ldb + i];
        double acc = bi, den = fabs(bi), arow = 0.0;
        for (int64_t q = rptr[i]; q < rptr[i + 1]; ++q) {
            const double av = rv[q];
            const double xv = xc[rcol[q]];
            acc -= av * xv;
            den += fabs(av) * fabs(xv);
            arow += fabs(av);
        }
        r[t] = acc;
        const double ar = fabs(acc);
        const double om = ar == 0.0 ? 0.0 : (den == 0.0 ? __builtin_inf() : ar / den);
        unsigned long long k0 = key_of(om), k1 = key_of(ar), k2 = key_of(fabs(xc[i])), k3 = key_of(fabs(bi)),
                           k4 = key_of(arow);
        m0 = k0 > m0 ? k0 : m0;
        m1 = k1 > m1 ? k1 : m1;
        m2 = k2 > m2 ? k2 : m2;
        m3 = k3 > m3 ? k3 : m3;
        m4 = k4 > m4 ? k4 : m4;
    }
    m0 = block_max(m0);
    m1 = block_max(m1);
    m2 = block_max(m2);
    m3 = block_max(m3);
    m4 = block_max(m4);
    if (threadIdx.x == 0) {
        atomicMax(stats + 0 * kStatStride, m0);
        atomicMax(stats + 1 * kStatStride, m1);
        atomicMax(stats + 2 * kStatStride, m2);
        atomicMax(stats + 3 * kStatStride, m3);
        atomicMax(stats + 4 * kStatStride, m4);
    }
}

// ---- rv[q] = vals[idx[q]]
__global__ void gather_kernel(double* rv, const double* vals, const int64_t* idx, int64_t m)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < m; q += (int64_t)gridDim.x * blockDim.x)
        rv[q] = vals[idx[q]];
}

// ---- value gradient of x = A^{-1} b (adjoint): for a stored entry p = (i, j),
// grad[p] = -sum_k (db[i,k] x[j,k] + db[j,k] x[i,k]) if i > j, -sum_k db[i,k] x[i,k]
// if i == j, and 0 for entries above the diagonal (erow[p] < 0: not read by
// the factorization)
__global__ void values_grad_kernel(const int32_t* erow, const int32_t* ecol, int64_t nnz, const double* x,
                                   const double* db, int64_t ld, int32_t nrhs, double* grad)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = erow[p], j = ecol[p];
        double g = 0.0;
        if (i >= 0) {
            for (int32_t k = 0; k < nrhs; ++k) {
                const double* xk = x + (int64_t)k * ld;
                const double* dk = db + (int64_t)k * ld;
                g -= i == j ? dk[i] * xk[i] : dk[i] * xk[j] + dk[j] * xk[i];
            }
        }
        grad[p] = g;
    }
}

// ---- inverses of paired pieces (built after the factorization): the pair's
// inverse [[D_p, 0], [X, D_q]], X = -D_q (L_qp D_p), on the matrix cores
// (16x16x4 products; operand A lane l holds A[l%16][l/16], operand B lane l
// holds B[l/16][l%16], result slot v of lane l holds D[row(v, l/16)][l%16]).
// Workgroup (pair, jb): for jb < ceil(w_p/16) the columns j0 = 16 jb ..
// j0 + 15 of p: D_p's columns staged in LDS (zero above the diagonal) and
// copied, T = L_qp D_p[:, cols] (inner indices from j0: D_p is lower
// triangular) into LDS, then X[:, cols] = -D_q T (inner indices up to each
// row tile's end: D_q is lower triangular); for the remaining jb the columns
// of q: zeros above, D_q below.  L D L^T (kept inverses Y = D^{-1} L^{-1},
// unit L): X = -Y_q L_qp D_p Y_p, the staged rows of Y_p scaled by p's
// pivots.  Each wave takes the 16-row tiles
// wave, wave + 4, ...; the loads of sixteen inner steps go out together.
template <class T>
struct PairMM;
template <>
struct PairMM<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc mfma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int v, int lk) { return 4 * v + lk; }
};
template <>
struct PairMM<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc mfma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};

constexpr int kPairLd = 17;   // LDS leading dimension of the staged 16-column blocks

template <class T>
__global__ void __launch_bounds__(256) pair_inv(const T* panels, T* dinv, const PairItem* items, int ldlt)
{
    typedef typename PairMM<T>::acc acc;
    __shared__ T dps[256 * kPairLd];   // D_p[kk][n]
    __shared__ T ts[256 * kPairLd];    // T[kk][n]
    const PairItem it = items[blockIdx.x];
    const int wp = it.wp, wq = it.wq, W = wp + wq;
    const int nbp = (wp + 15) / 16, nbq = (wq + 15) / 16;
    const int jb = blockIdx.y;
    if (jb >= nbp + nbq) return;
    T* P = dinv + it.out;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    if (jb >= nbp) {
        const int j0 = 16 * (jb - nbp);
        const T* Dq = dinv + it.dq;
        for (int idx = tid; idx < 16 * W; idx += 256) {
            const int j = j0 + idx / W, r = idx % W;
            if (j < wq) P[(int64_t)(wp + j) * W + r] = (r >= wp + j) ? Dq[(int64_t)j * wq + (r - wp)] : T(0);
        }
        return;
    }
    const int j0 = 16 * jb;
    const T* Dp = dinv + it.dp;
    const T* Pp = panels + (it.lofs - wp);   // p's panel: L D L^T pivot d_r at r * (ldp + 1)
    for (int idx = tid; idx < 16 * wp; idx += 256) {
        const int c = idx / wp, r = idx % wp, j = j0 + c;
        const T v = (j < wp && r >= j) ? Dp[(int64_t)j * wp + r] : T(0);
        dps[r * kPairLd + c] = ldlt ? v * Pp[(int64_t)r * (it.ldp + 1)] : v;
        if (j < wp) P[(int64_t)j * W + r] = v;
    }
    __syncthreads();
    const int ntile = (wq + 15) / 16;
    const T* Lq = panels + it.lofs;   // L_qp[i][kk] at Lq[i + kk * ldp]
    const int64_t ldp = it.ldp;
    for (int t = wave; t < ntile; t += 4) {
        acc c = {0, 0, 0, 0};
        const int i = min(16 * t + li, wq - 1);
        for (int kk0 = j0; kk0 < wp; kk0 += 64) {
            T av[16], bv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int kk = kk0 + 4 * u + lk;
                av[u] = Lq[i + (int64_t)min(kk, wp - 1) * ldp];
                bv[u] = kk < wp ? dps[kk * kPairLd + li] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) c = PairMM<T>::mfma(av[u], bv[u], c);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) ts[(16 * t + PairMM<T>::row(v, lk)) * kPairLd + li] = c[v];
    }
    __syncthreads();
    const T* Dq = dinv + it.dq;   // D_q[i][kk] at Dq[i + kk * wq]
    for (int t = wave; t < ntile; t += 4) {
        acc c = {0, 0, 0, 0};
        const int irow = 16 * t + li, i = min(irow, wq - 1);
        const int kend = min(16 * t + 16, wq);
        for (int kk0 = 0; kk0 < kend; kk0 += 64) {
            T av[16], bv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int kk = kk0 + 4 * u + lk;
                const T d = Dq[i + (int64_t)min(kk, wq - 1) * wq];
                av[u] = kk <= irow ? d : T(0);
                bv[u] = kk < kend ? ts[kk * kPairLd + li] : T(0);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) c = PairMM<T>::mfma(av[u], bv[u], c);
        }
        if (j0 + li < wp)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * t + PairMM<T>::row(v, lk);
                if (r < wq) P[(int64_t)(j0 + li) * W + wp + r] = -c[v];
            }
    }
}

// ---- host launchers
static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

// right-hand sides per pass over a panel: 1, 4 or 8 (16-lane small-block
// kernels, whose lanes each keep up to 8 rows: 1 or 2)
static int nr_block(int nrhs) { return nrhs <= 1 ? 1 : (nrhs <= 4 ? 4 : 8); }

#define SPX_NR_DISPATCH(NRV, CALL) \
    do {                           \
        if ((NRV) == 1) { constexpr int NR = 1; CALL; } \
        else if ((NRV) == 4) { constexpr int NR = 4; CALL; } \
        else { constexpr int NR = 8; CALL; } \
    } while (0)

hipError_t launch_fwd_diag(const SweepArgs& a, const DiagItem* items, int count, int lanes, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int nrv = nr_block(a.nrhs);
    const dim3 grid(count, (a.nrhs + nrv - 1) / nrv);
#define SPX_FD(L) SPX_NR_DISPATCH(nrv, (a.f32 ? fwd_diag<float, L, NR><<<grid, 256, 0, s>>>(a, items) \
                                               : fwd_diag<double, L, NR><<<grid, 256, 0, s>>>(a, items)))
    if (lanes == 32) SPX_FD(32);
    else if (lanes == 16) SPX_FD(16);
    else SPX_FD(4);
#undef SPX_FD
    return hipGetLastError();
}
hipError_t launch_fwd_off(const SweepArgs& a, const OffItem* items, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (a.nrhs > 1) {   // blocks of 4 or 8 right-hand sides: the matrix-core form
        const dim3 grid(count, (a.nrhs + (a.nrhs <= 4 ? 3 : 7)) / (a.nrhs <= 4 ? 4 : 8));
        if (a.nrhs <= 4) {
            if (a.f32) fwd_off_mm<float, 4><<<grid, 256, 0, s>>>(a, items);
            else fwd_off_mm<double, 4><<<grid, 256, 0, s>>>(a, items);
        } else {
            if (a.f32) fwd_off_mm<float, 8><<<grid, 256, 0, s>>>(a, items);
            else fwd_off_mm<double, 8><<<grid, 256, 0, s>>>(a, items);
        }
        return hipGetLastError();
    }
    SPX_NR_DISPATCH(nr_block(a.nrhs), (a.f32 ? fwd_off<float, NR><<<dim3(count, (a.nrhs + NR - 1) / NR), 256, 0, s>>>(a, items)
                                             : fwd_off<double, NR><<<dim3(count, (a.nrhs + NR - 1) / NR), 256, 0, s>>>(a, items)));
    return hipGetLastError();
}
hipError_t launch_bwd_off(const SweepArgs& a, const OffItem* items, int count, bool tall, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (a.nrhs > 1) {   // blocks of 4 or 8 right-hand sides (64-row items): the matrix-core form
        const dim3 grid(count, (a.nrhs + (a.nrhs <= 4 ? 3 : 7)) / (a.nrhs <= 4 ? 4 : 8));
        if (a.nrhs <= 4) {
            if (a.f32) bwd_off_mm<float, 4><<<grid, 256, 0, s>>>(a, items);
            else bwd_off_mm<double, 4><<<grid, 256, 0, s>>>(a, items);
        } else {
            if (a.f32) bwd_off_mm<float, 8><<<grid, 256, 0, s>>>(a, items);
            else bwd_off_mm<double, 8><<<grid, 256, 0, s>>>(a, items);
        }
        return hipGetLastError();
    }
    if (tall) {
        SPX_NR_DISPATCH(nr_block(a.nrhs), (a.f32 ? bwd_off<float, 16, NR><<<dim3(count, (a.nrhs + NR - 1) / NR), 256, 0, s>>>(a, items)
                                                 : bwd_off<double, 16, NR><<<dim3(count, (a.nrhs + NR - 1) / NR), 256, 0, s>>>(a, items)));
    } else {
        SPX_NR_DISPATCH(nr_block(a.nrhs), (a.f32 ? bwd_off<float, 4, NR><<<dim3(count, (a.nrhs + NR - 1) / NR), 256, 0, s>>>(a, items)
                                                 : bwd_off<double, 4, NR><<<dim3(count, (a.nrhs + NR - 1) / NR), 256, 0, s>>>(a, items)));
    }
    return hipGetLastError();
}
hipError_t launch_bwd_diag(const SweepArgs& a, const DiagItem* items, int count, int lanes, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int nrv = nr_block(a.nrhs);
    const dim3 grid(count, (a.nrhs + nrv - 1) / nrv);
#define SPX_BD(L) SPX_NR_DISPATCH(nrv, (a.f32 ? bwd_diag<float, L, NR><<<grid, 256, 0, s>>>(a, items) \
                                               : bwd_diag<double, L, NR><<<grid, 256, 0, s>>>(a, items)))
    if (lanes == 32) SPX_BD(32);
    else if (lanes == 16) SPX_BD(16);
    else SPX_BD(4);
#undef SPX_BD
    return hipGetLastError();
}
hipError_t launch_pair_inv(const void* panels, void* dinv, bool f32, bool ldlt, const PairItem* items, int count,
                          int maxnb, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const dim3 grid(count, maxnb);
    if (f32)
        pair_inv<float><<<grid, 256, 0, s>>>(static_cast<const float*>(panels), static_cast<float*>(dinv), items,
                                             ldlt ? 1 : 0);
    else
        pair_inv<double><<<grid, 256, 0, s>>>(static_cast<const double*>(panels), static_cast<double*>(dinv), items,
                                              ldlt ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_permute_in(double* y, const double* b, int64_t ldb, const int32_t* perm, int32_t n, int32_t nrhs,
                             hipStream_t s)
{
    permute_in<<<grid_for((int64_t)n * nrhs), 256, 0, s>>>(y, b, ldb, perm, n, nrhs);
    return hipGetLastError();
}
hipError_t launch_permute_out(double* x, int64_t ldx, const double* y, const int32_t* perm, int32_t n, int32_t nrhs,
                              hipStream_t s)
{
    permute_out<<<grid_for((int64_t)n * nrhs), 256, 0, s>>>(x, ldx, y, perm, n, nrhs);
    return hipGetLastError();
}
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s)
{
    zero_u64<<<1, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_fwd_small(const SweepArgs& a, const int32_t* cblks, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int blocks = (count + kSGroups - 1) / kSGroups;
    if (a.nrhs <= 1) {
        if (a.f32) fwd_small<float, 1><<<blocks, 256, 0, s>>>(a, cblks, count);
        else fwd_small<double, 1><<<blocks, 256, 0, s>>>(a, cblks, count);
    } else {
        if (a.f32) fwd_small<float, 2><<<blocks, 256, 0, s>>>(a, cblks, count);
        else fwd_small<double, 2><<<blocks, 256, 0, s>>>(a, cblks, count);
    }
    return hipGetLastError();
}

hipError_t launch_bwd_small(const SweepArgs& a, const int32_t* cblks, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int blocks = (count + kSGroups - 1) / kSGroups;
    if (a.nrhs <= 1) {
        if (a.f32) bwd_small<float, 1><<<blocks, 256, 0, s>>>(a, cblks, count);
        else bwd_small<double, 1><<<blocks, 256, 0, s>>>(a, cblks, count);
    } else {
        if (a.f32) bwd_small<float, 2><<<blocks, 256, 0, s>>>(a, cblks, count);
        else bwd_small<double, 2><<<blocks, 256, 0, s>>>(a, cblks, count);
    }
    return hipGetLastError();
}

hipError_t launch_axpy(double* x, const double* d, int64_t n, hipStream_t s)
{
    axpy_kernel<<<grid_for(n), 256, 0, s>>>(x, d, n);
    return hipGetLastError();
}
hipError_t launch_residual(const int64_t* rptr, const int32_t* rcol, const double* rv, const double* x,
                           const double* b, int64_t ldb, double* r, int32_t n, int32_t nrhs,
                           unsigned long long* stats, hipStream_t s)
{
    const int blocks = (int)std::min<int64_t>(kResidualBlocks, std::max<int64_t>(1, ((int64_t)n * nrhs + 255) / 256));
    residual_kernel<<<blocks, 256, 0, s>>>(rptr, rcol, rv, x, b, ldb, r, n, nrhs, stats);
    return hipGetLastError();
}

}  // namespace spx

namespace spx {
hipError_t launch_gather(double* rv, const double* vals, const int64_t* idx, int64_t m, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    gather_kernel<<<grid_for(m), 256, 0, s>>>(rv, vals, idx, m);
    return hipGetLastError();
}
hipError_t launch_values_grad(const int32_t* erow, const int32_t* ecol, int64_t nnz, const double* x, const double* db,
                              int64_t ld, int32_t nrhs, double* grad, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    values_grad_kernel<<<grid_for(nnz), 256, 0, s>>>(erow, ecol, nnz, x, db, ld, nrhs, grad);
    return hipGetLastError();
}
}  // namespace spx
