// Triangular solves with the supernodal factor, FP64 residual and the
// refinement helpers (the solve phase of A x = b; the paper states the
// problem, the sweeps are the standard supernodal ones).
//
// Forward sweep, column blocks in ascending dependency levels:
//   y_k <- L_kk^{-1} y_k                  (one workgroup per block)
//   y[rows of k] -= L_k,off y_k           (row chunks, FP64 atomics)
// Backward sweep, levels descending:
//   t_k  = L_k,off^T x[rows of k]         (row chunks, wave reductions)
//   x_k <- L_kk^{-T} (y_k - t_k)
// Both use the inverse of each diagonal block kept by the factorization.
// The sweeps stream the panels once each: they are bound by HBM bandwidth.
// The factor is read in its storage type T (double, or float in the FP32
// refinement mode); vectors and arithmetic are FP64 in both cases.
#include "device.hpp"

namespace spx {

constexpr int kChunk = 256;   // off-diagonal rows per workgroup

// ---- forward, diagonal block: y_k <- D y_k with D = L_kk^{-1} (lower, w x w,
// column-major, kept by the factorization).  Thread r owns row r; the loads
// D[r + p*w] of one p are contiguous over the threads.
template <class T>
__global__ void __launch_bounds__(256) fwd_diag(SweepArgs a, const int32_t* cblks)
{
    __shared__ double ys[256];
    const int k = cblks[blockIdx.x];
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k], w = pl.lcol[k] - f + 1;
    const T* D = static_cast<const T*>(a.dinv) + pl.dinv_off[k];
    const int tid = threadIdx.x;
    for (int rhs = 0; rhs < a.nrhs; ++rhs) {
        double* y = a.y + (int64_t)rhs * a.n + f;
        if (tid < w) ys[tid] = y[tid];
        __syncthreads();
        if (tid < w) {
            const T* row = D + tid;
            double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int p = 0;
            for (; p + 8 <= tid + 1; p += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] += row[(int64_t)(p + u) * w] * ys[p + u];
            }
            for (; p <= tid; ++p) v[0] += row[(int64_t)p * w] * ys[p];
            y[tid] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        }
        __syncthreads();
    }
}

// ---- forward, off-diagonal rows: y[g(r)] -= sum_c L[r, c] y_k[c]; thread per
// row, loads contiguous over the threads
template <class T>
__global__ void __launch_bounds__(256) fwd_off(SweepArgs a, const int2* chunks)
{
    __shared__ double yk[256];
    const int2 it = chunks[blockIdx.x];
    const int k = it.x, row0 = it.y;
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k], w = pl.lcol[k] - f + 1;
    const int64_t ld = pl.stride[k];
    const int nr = min(kChunk, (int)ld - row0);
    const T* L = static_cast<const T*>(a.panels) + pl.panel_off[k] + row0;
    const int32_t* g = a.rowg + a.rowg_off[k] + (row0 - w);
    const int tid = threadIdx.x;
    for (int rhs = 0; rhs < a.nrhs; ++rhs) {
        double* y = a.y + (int64_t)rhs * a.n;
        if (tid < w) yk[tid] = y[f + tid];
        __syncthreads();
        if (tid < nr) {
            const T* row = L + tid;
            double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int c = 0;
            for (; c + 8 <= w; c += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] += row[(c + u) * ld] * yk[c + u];
            }
            for (; c < w; ++c) v[0] += row[c * ld] * yk[c];
            unsafeAtomicAdd(y + g[tid], -(((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))));
        }
        __syncthreads();
    }
}

// ---- backward, off-diagonal rows: tacc[f + c] += sum_r L[r, c] x[g(r)];
// thread per column, each streaming down its own column of the chunk
template <class T>
__global__ void __launch_bounds__(256) bwd_off(SweepArgs a, const int2* chunks)
{
    __shared__ double xr[kChunk];
    const int2 it = chunks[blockIdx.x];
    const int k = it.x, row0 = it.y;
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k], w = pl.lcol[k] - f + 1;
    const int64_t ld = pl.stride[k];
    const int nr = min(kChunk, (int)ld - row0);
    const T* L = static_cast<const T*>(a.panels) + pl.panel_off[k] + row0;
    const int32_t* g = a.rowg + a.rowg_off[k] + (row0 - w);
    const int tid = threadIdx.x;
    for (int rhs = 0; rhs < a.nrhs; ++rhs) {
        const double* x = a.y + (int64_t)rhs * a.n;
        if (tid < nr) xr[tid] = x[g[tid]];
        __syncthreads();
        if (tid < w) {
            const T* col = L + (int64_t)tid * ld;
            double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int r = 0;
            for (; r + 8 <= nr; r += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] += col[r + u] * xr[r + u];
            }
            for (; r < nr; ++r) v[0] += col[r] * xr[r];
            unsafeAtomicAdd(a.tacc + (int64_t)rhs * a.n + f + tid,
                            ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])));
        }
        __syncthreads();
    }
}

// ---- backward, diagonal block: x_k <- D^T (y_k - t_k); thread c streams
// down column c of D
template <class T>
__global__ void __launch_bounds__(256) bwd_diag(SweepArgs a, const int32_t* cblks)
{
    __shared__ double zs[256];
    const int k = cblks[blockIdx.x];
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k], w = pl.lcol[k] - f + 1;
    const T* D = static_cast<const T*>(a.dinv) + pl.dinv_off[k];
    const int tid = threadIdx.x;
    for (int rhs = 0; rhs < a.nrhs; ++rhs) {
        double* y = a.y + (int64_t)rhs * a.n + f;
        const double* t = a.tacc + (int64_t)rhs * a.n + f;
        if (tid < w) zs[tid] = y[tid] - t[tid];
        __syncthreads();
        if (tid < w) {
            const T* col = D + (int64_t)tid * w;
            double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int p = tid;
            for (; p + 8 <= w; p += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] += col[p + u] * zs[p + u];
            }
            for (; p < w; ++p) v[0] += col[p] * zs[p];
            y[tid] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
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
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
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
// A is read through the symmetric row pattern (rptr, rcol) whose values are
// the input entries rval[q] (lower triangle mirrored).
// stats[0] = max_i |r_i| / (|A||x| + |b|)_i   (0/0 = 0, p/0 = inf)
// stats[1] = max |r_i|, stats[2] = max |x_i|, stats[3] = max |b_i|, stats[4] = max_i sum_j |a_ij|
__global__ void __launch_bounds__(256) residual_kernel(const int64_t* rptr, const int32_t* rcol, const int64_t* rval,
                                                       const double* vals, const double* x, const double* b,
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
            const double av = vals[rval[q]];
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
        atomicMax(stats + 0, m0);
        atomicMax(stats + 1, m1);
        atomicMax(stats + 2, m2);
        atomicMax(stats + 3, m3);
        atomicMax(stats + 4, m4);
    }
}

// ---- host launchers
static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

hipError_t launch_fwd_diag(const SweepArgs& a, const int32_t* cblks, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (a.f32) fwd_diag<float><<<count, 256, 0, s>>>(a, cblks);
    else fwd_diag<double><<<count, 256, 0, s>>>(a, cblks);
    return hipGetLastError();
}
hipError_t launch_fwd_off(const SweepArgs& a, const int2* chunks, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (a.f32) fwd_off<float><<<count, 256, 0, s>>>(a, chunks);
    else fwd_off<double><<<count, 256, 0, s>>>(a, chunks);
    return hipGetLastError();
}
hipError_t launch_bwd_off(const SweepArgs& a, const int2* chunks, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (a.f32) bwd_off<float><<<count, 256, 0, s>>>(a, chunks);
    else bwd_off<double><<<count, 256, 0, s>>>(a, chunks);
    return hipGetLastError();
}
hipError_t launch_bwd_diag(const SweepArgs& a, const int32_t* cblks, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (a.f32) bwd_diag<float><<<count, 256, 0, s>>>(a, cblks);
    else bwd_diag<double><<<count, 256, 0, s>>>(a, cblks);
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
    zero_u64<<<1, 64, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_axpy(double* x, const double* d, int64_t n, hipStream_t s)
{
    axpy_kernel<<<grid_for(n), 256, 0, s>>>(x, d, n);
    return hipGetLastError();
}
hipError_t launch_residual(const int64_t* rptr, const int32_t* rcol, const int64_t* rval, const double* vals,
                           const double* x, const double* b, int64_t ldb, double* r, int32_t n, int32_t nrhs,
                           unsigned long long* stats, hipStream_t s)
{
    residual_kernel<<<grid_for((int64_t)n * nrhs), 256, 0, s>>>(rptr, rcol, rval, vals, x, b, ldb, r, n, nrhs, stats);
    return hipGetLastError();
}

}  // namespace spx
