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
//   TRSM(k, rows)    64, 128 or 256 off-diagonal rows of panel k times
//                    L_kk^{-T}
//   UPDATE(k,j,r,c)  a 256x64 (or 128x128) tile of the outer product of panel
//                    k, subtracted into panel j with atomics; for a group of
//                    pieces of a split supernode, the sum of their products
//   SMALL(k)         a narrow column block (width <= 32, <= 128 rows): all
//                    three steps and every update tile of the block at once
// Dependencies are counters: FACT(j) becomes ready when every UPDATE tile
// into j is done, the TRSM tiles of k when FACT(k) is done, the UPDATE tiles
// of k when its last TRSM tile is done.  FACT, TRSM and the updates into the
// first facing block go to a high-priority queue that workers poll first.
// Products run on the matrix cores: v_mfma_f64_16x16x4f64 for the FP64
// factor, v_mfma_f32_16x16x4f32 for the FP32 factor of the refinement mode
// (whose 32x32 diagonal tiles are still factored and inverted in FP64), and
// split-BF16 products (v_mfma_f32_16x16x16_bf16) in the split mode.
#include "device.hpp"

namespace spx {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

#define AGENT __HIP_MEMORY_SCOPE_AGENT

// Pointers into device (global) memory.  The panels reach the tasks as
// generic pointers; typing them as global lets the compiler use global
// stores and atomics (scalar base, 32-bit lane offset) instead of flat ones.
template <class T>
struct Glob {
    typedef __attribute__((address_space(1))) T type;
};
template <class T>
__device__ __forceinline__ typename Glob<T>::type* glob(T* p)
{
    return (typename Glob<T>::type*)p;
}
// A generic pointer known to point into LDS, as an LDS pointer (never null:
// the cast then needs no null test)
template <class T>
__device__ __forceinline__ __attribute__((address_space(3))) T* lds(T* p)
{
    if (p == nullptr) __builtin_unreachable();
    return (__attribute__((address_space(3))) T*)p;
}

// The 16x16x4 matrix-core product of one element type.  Operand A lane l
// holds A[l%16][l/16], operand B lane l holds B[l/16][l%16]; the four result
// slots of lane l hold column l%16 of D, at the rows drow(v, l/16).
template <class T>
struct MM;
template <>
struct MM<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc mfma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int v, int lk) { return 4 * v + lk; }
};
template <>
struct MM<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc mfma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int v, int lk) { return 4 * lk + v; }
};

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
template <class T>
__device__ __forceinline__ const T* uni(const T* p)
{
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

template <class T>
__device__ __forceinline__ GOp make_gop(const T* base, int64_t count, int64_t off, int64_t si, int64_t sk)
{
    constexpr int e = (int)sizeof(T);
    GOp g;
    g.rs = __builtin_amdgcn_make_buffer_rsrc((void*)uni(base), (short)0, uni((int)(count * e)), 0x00020000);
    g.off = uni((int)(off * e));
    g.si = uni((int)(si * e));
    g.sk = uni((int)(sk * e));
    return g;
}

template <class T>
__device__ __forceinline__ T gload(const GOp& g, int voff);
template <>
__device__ __forceinline__ double gload<double>(const GOp& g, int voff)
{
    const u32x2 b = __builtin_amdgcn_raw_buffer_load_b64(g.rs, voff, 0, 0);
    return __builtin_bit_cast(double, b);
}
template <>
__device__ __forceinline__ float gload<float>(const GOp& g, int voff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(g.rs, voff, 0, 0));
}

// Byte offset of a masked-off buffer load: past the end of any array here,
// so the load returns zero (the value is discarded by a select anyway).
constexpr int kOffNone = 0x7f000000;

// Element at byte offset voff (per lane) + soff (wave-uniform) of g's array;
// stores outside the array are dropped.
__device__ __forceinline__ double gload_s(const GOp& g, int voff, int soff, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(g.rs, voff, soff, 0));
}
__device__ __forceinline__ float gload_s(const GOp& g, int voff, int soff, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(g.rs, voff, soff, 0));
}
__device__ __forceinline__ void gstore_s(const GOp& g, int voff, int soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), g.rs, voff, soff, 0);
}
__device__ __forceinline__ void gstore_s(const GOp& g, int voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), g.rs, voff, soff, 0);
}

// One wave accumulates a 64 x (16*NB) tile: acc += X Y^T, X(r, p) r < 64,
// Y(c, p) c < 16*NB, p < K (K rounded up to 8 reads zeros or is exact).  The
// whole tile is always computed (no per-block predicates); rows and columns
// beyond the caller's bounds produce results that are not stored.
// Y feeds operand A and X operand B (lane layout in MM), so
//   acc[bi][bj][v] = C(16*bj + l%16, 16*bi + drow(v, l/16))
// and the 16 lanes of a result slot cover 16 consecutive rows of C.  The
// inner dimension advances 8 at a time through register buffers: FP32 uses
// three (the operands of the next 16 in flight while the products of the
// current 8 are issued); FP64 two (the next 8 in flight): with a third, the
// 128 accumulator registers and the operands exceed the 256 registers of a
// wave at two workgroups per CU, and the spilled operands each cost a wait
// for every outstanding load.
template <int NB, class T, int RB = 4>
__device__ __forceinline__ void wave_gemm(typename MM<T>::acc (&acc)[NB][RB], const GOp& X, const GOp& Y, int K)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nchunks = (K + 7) >> 3;
    if (nchunks <= 0) return;
    int xo[2][RB], yo[2][NB];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int b = 0; b < RB; ++b) xo[u][b] = X.off + (16 * b + li) * X.si + (4 * u + lk) * X.sk;
#pragma unroll
        for (int b = 0; b < NB; ++b) yo[u][b] = Y.off + (16 * b + li) * Y.si + (4 * u + lk) * Y.sk;
    }
    const int dx = 8 * X.sk, dy = 8 * Y.sk;
    T xa[2][RB], ya[2][NB], xb[2][RB], yb[2][NB], xc[2][RB], yc[2][NB];
    // (scheduling barriers keep every group of loads ahead of the products
    // it is meant to overlap; left alone, the compiler sinks the FP32 loads
    // next to their uses and waits for them)
    auto load = [&](T (&xs)[2][RB], T (&ys)[2][NB], int ch) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int b = 0; b < RB; ++b) xs[u][b] = gload<T>(X, xo[u][b] + ch * dx);
#pragma unroll
            for (int b = 0; b < NB; ++b) ys[u][b] = gload<T>(Y, yo[u][b] + ch * dy);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto mma = [&](const T (&xs)[2][RB], const T (&ys)[2][NB]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj < RB; ++bj) acc[bi][bj] = MM<T>::mfma(ys[u][bi], xs[u][bj], acc[bi][bj]);
        __builtin_amdgcn_sched_barrier(0);
    };
    // (reads past the last chunk repeat it and are not used)
    const int last = nchunks - 1;
    if constexpr (sizeof(T) == 8) {
        (void)xc;
        (void)yc;
        load(xa, ya, 0);
        int ch = 0;
        for (; ch + 2 <= nchunks; ch += 2) {
            load(xb, yb, ch + 1);
            mma(xa, ya);
            load(xa, ya, min(ch + 2, last));
            mma(xb, yb);
        }
        if (ch < nchunks) mma(xa, ya);
    } else {
        load(xa, ya, 0);
        load(xb, yb, min(1, last));
        int ch = 0;
        for (; ch + 3 <= nchunks; ch += 3) {
            load(xc, yc, min(ch + 2, last));
            mma(xa, ya);
            load(xa, ya, min(ch + 3, last));
            mma(xb, yb);
            load(xb, yb, min(ch + 4, last));
            mma(xc, yc);
        }
        if (ch < nchunks) mma(xa, ya);
        if (ch + 1 < nchunks) mma(xb, yb);
    }
}

// L D L^T update products: acc += X (Y D)^T, the facing operand Y scaled by
// d_p (element p of Dg at p * Dg.sk: the diagonal of the source panel) just
// before the products, so its loads stay in flight with the others; two
// register buffers of 8 inner indices in both precisions (a separate
// function: the extra operand registers would change the allocation of the
// plain product, and a third FP32 buffer spills).
template <int NB, class T, int RB = 4>
__device__ __forceinline__ void wave_gemm_d(typename MM<T>::acc (&acc)[NB][RB], const GOp& X, const GOp& Y, int K,
                                          const GOp& Dg)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nchunks = (K + 7) >> 3;
    if (nchunks <= 0) return;
    int xo[2][RB], yo[2][NB];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int b = 0; b < RB; ++b) xo[u][b] = X.off + (16 * b + li) * X.si + (4 * u + lk) * X.sk;
#pragma unroll
        for (int b = 0; b < NB; ++b) yo[u][b] = Y.off + (16 * b + li) * Y.si + (4 * u + lk) * Y.sk;
    }
    const int dx = 8 * X.sk, dy = 8 * Y.sk;
    T xa[2][RB], ya[2][NB], da[2], xb[2][RB], yb[2][NB], db[2];
    // (scheduling barriers keep every group of loads ahead of the products
    // it is meant to overlap; left alone, the compiler sinks the FP32 loads
    // next to their uses and waits for them)
    auto load = [&](T (&xs)[2][RB], T (&ys)[2][NB], T (&ds)[2], int ch) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int b = 0; b < RB; ++b) xs[u][b] = gload<T>(X, xo[u][b] + ch * dx);
#pragma unroll
            for (int b = 0; b < NB; ++b) ys[u][b] = gload<T>(Y, yo[u][b] + ch * dy);
            ds[u] = gload<T>(Dg, Dg.off + (8 * ch + 4 * u + lk) * Dg.sk);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto mma = [&](const T (&xs)[2][RB], const T (&ys)[2][NB], const T (&ds)[2]) {
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) {
                const T yv = ys[u][bi] * ds[u];
#pragma unroll
                for (int bj = 0; bj < RB; ++bj) acc[bi][bj] = MM<T>::mfma(yv, xs[u][bj], acc[bi][bj]);
            }
        __builtin_amdgcn_sched_barrier(0);
    };
    // (reads past the last chunk repeat it and are not used)
    const int last = nchunks - 1;
    load(xa, ya, da, 0);
    int ch = 0;
    for (; ch + 2 <= nchunks; ch += 2) {
        load(xb, yb, db, ch + 1);
        mma(xa, ya, da);
        load(xa, ya, da, min(ch + 2, last));
        mma(xb, yb, db);
    }
    if (ch < nchunks) mma(xa, ya, da);
}

// Split-BF16 products (FP32 panels): each FP32 operand x is split into
// hi = bf16(x) (round to nearest) and lo = bf16(x - hi); the product is
// hi*hi + hi*lo + lo*hi on the BF16 matrix cores with FP32 accumulation
// (lo*lo is dropped: relative error about 2^-16 per product).  The inner
// dimension advances 16 at a time; lane (l%16, l/16) loads its FP32 operands
// at inner indices 4s + l/16 (s < 4), the order of the FP32 products, and
// packs them as the 4 BF16 values the 16x16x16 instruction takes from it at
// 4*(l/16) + s: the same permutation of the inner index for both operands,
// so the sum is unchanged.  Two raw buffers: the next 16 in flight while the
// current 16 are split and multiplied (with 32 per step, the 16x16x32 form,
// the buffers and accumulators exceed the registers and spill).
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(const float (&v)[4], s16x4& hi, s16x4& lo)
{
    bf16x4 h, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const __bf16 t = (__bf16)v[j];
        h[j] = t;
        l[j] = (__bf16)(v[j] - (float)t);
    }
    hi = __builtin_bit_cast(s16x4, h);
    lo = __builtin_bit_cast(s16x4, l);
}

template <int NB, int RB = 4>
__device__ __forceinline__ void wave_gemm_split(f4 (&acc)[NB][RB], const GOp& X, const GOp& Y, int K)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nchunks = (K + 15) >> 4;
    if (nchunks <= 0) return;
    int xo[RB], yo[NB];
#pragma unroll
    for (int b = 0; b < RB; ++b) xo[b] = X.off + (16 * b + li) * X.si + lk * X.sk;
#pragma unroll
    for (int b = 0; b < NB; ++b) yo[b] = Y.off + (16 * b + li) * Y.si + lk * Y.sk;
    const int dx = 4 * X.sk, dy = 4 * Y.sk;
    float xa[RB][4], ya[NB][4], xb[RB][4], yb[NB][4];
    auto load = [&](float (&xs)[RB][4], float (&ys)[NB][4], int ch) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int b = 0; b < RB; ++b) xs[b][s] = gload<float>(X, xo[b] + (4 * ch + s) * dx);
#pragma unroll
            for (int b = 0; b < NB; ++b) ys[b][s] = gload<float>(Y, yo[b] + (4 * ch + s) * dy);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto mma = [&](const float (&xs)[RB][4], const float (&ys)[NB][4]) {
        s16x4 xh[RB], xl[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) split_bf16(xs[b], xh[b], xl[b]);
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            s16x4 yh, yl;
            split_bf16(ys[bi], yh, yl);
#pragma unroll
            for (int bj = 0; bj < RB; ++bj) {
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(yh, xh[bj], acc[bi][bj], 0, 0, 0);
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(yh, xl[bj], acc[bi][bj], 0, 0, 0);
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(yl, xh[bj], acc[bi][bj], 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // (reads past the last chunk repeat it and are not used)
    const int last = nchunks - 1;
    load(xa, ya, 0);
    int ch = 0;
    for (; ch + 2 <= nchunks; ch += 2) {
        load(xb, yb, ch + 1);
        mma(xa, ya);
        load(xa, ya, min(ch + 2, last));
        mma(xb, yb);
    }
    if (ch < nchunks) mma(xa, ya);
}

// Split-BF16 L D L^T update products: the facing operand scaled by d_p in
// FP32 before it is split (as in wave_gemm_d).
template <int NB, int RB = 4>
__device__ __forceinline__ void wave_gemm_split_d(f4 (&acc)[NB][RB], const GOp& X, const GOp& Y, int K, const GOp& Dg)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nchunks = (K + 15) >> 4;
    if (nchunks <= 0) return;
    int xo[RB], yo[NB];
#pragma unroll
    for (int b = 0; b < RB; ++b) xo[b] = X.off + (16 * b + li) * X.si + lk * X.sk;
#pragma unroll
    for (int b = 0; b < NB; ++b) yo[b] = Y.off + (16 * b + li) * Y.si + lk * Y.sk;
    const int dx = 4 * X.sk, dy = 4 * Y.sk;
    float xa[RB][4], ya[NB][4], da[4], xb[RB][4], yb[NB][4], db[4];
    auto load = [&](float (&xs)[RB][4], float (&ys)[NB][4], float (&ds)[4], int ch) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int b = 0; b < RB; ++b) xs[b][s] = gload<float>(X, xo[b] + (4 * ch + s) * dx);
#pragma unroll
            for (int b = 0; b < NB; ++b) ys[b][s] = gload<float>(Y, yo[b] + (4 * ch + s) * dy);
            // inner index 16 ch + 4 s + l/16
            ds[s] = gload<float>(Dg, Dg.off + (16 * ch + 4 * s + lk) * Dg.sk);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    auto mma = [&](const float (&xs)[RB][4], const float (&ys)[NB][4], const float (&ds)[4]) {
        s16x4 xh[RB], xl[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) split_bf16(xs[b], xh[b], xl[b]);
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
            s16x4 yh, yl;
            float yv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) yv[q] = ys[bi][q] * ds[q];
            split_bf16(yv, yh, yl);
#pragma unroll
            for (int bj = 0; bj < RB; ++bj) {
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(yh, xh[bj], acc[bi][bj], 0, 0, 0);
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(yh, xl[bj], acc[bi][bj], 0, 0, 0);
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(yl, xh[bj], acc[bi][bj], 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // (reads past the last chunk repeat it and are not used)
    const int last = nchunks - 1;
    load(xa, ya, da, 0);
    int ch = 0;
    for (; ch + 2 <= nchunks; ch += 2) {
        load(xb, yb, db, ch + 1);
        mma(xa, ya, da);
        load(xa, ya, da, min(ch + 2, last));
        mma(xb, yb, db);
    }
    if (ch < nchunks) mma(xa, ya, da);
}

// acc += X Y^T over K inner indices: FP64 or FP32 products, or (FP32 panels
// with the split option) split-BF16 products; DS: acc += X (Y D)^T with the
// d_p read through Dg
template <int NB, class T, int RB = 4, bool DS = false>
__device__ __forceinline__ void tile_gemm(typename MM<T>::acc (&acc)[NB][RB], const GOp& X, const GOp& Y, int K, bool split,
                                          const GOp& Dg)
{
    if constexpr (sizeof(T) == 4) {
        if (split) {
            if constexpr (DS) wave_gemm_split_d<NB, RB>(acc, X, Y, K, Dg);
            else wave_gemm_split<NB, RB>(acc, X, Y, K);
            return;
        }
    }
    if constexpr (DS) wave_gemm_d<NB, T, RB>(acc, X, Y, K, Dg);
    else wave_gemm<NB, T, RB>(acc, X, Y, K);
}
template <int NB, class T, int RB = 4>
__device__ __forceinline__ void tile_gemm(typename MM<T>::acc (&acc)[NB][RB], const GOp& X, const GOp& Y, int K, bool split)
{
    tile_gemm<NB, T, RB, false>(acc, X, Y, K, split, X);
}

template <int NB, class A, int RB>
__device__ __forceinline__ void zero_acc(A (&acc)[NB][RB])
{
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = A{0, 0, 0, 0};
}

// epi(r, c, value) over a wave's accumulator, r < mv, c < nv
template <class T, int NB, int RB, class Epi>
__device__ __forceinline__ void wave_store(const typename MM<T>::acc (&acc)[NB][RB], int mv, int nv, Epi epi)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < RB; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * bj + li, c = 16 * bi + MM<T>::drow(v, lk);
                if (r < mv && c < nv) epi(r, c, acc[bi][bj][v]);
            }
}

// ---------------------------------------------------------------- FACT(k)
// 1/d from the hardware estimate and two Newton-Raphson steps
__device__ __forceinline__ double recip_nr(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    y = y * __builtin_fma(-d, y, 2.0);
    return y * __builtin_fma(-d, y, 2.0);
}

// The static pivoting threshold eps * max |a_ij| (0: off) sits in LDS after
// the 64-entry broadcast buffer bc and the 32-entry pivot buffer of the
// fused small items, written once by each worker at its start: a global
// load at the start of every tile factorization would wait for memory
// (each item begins with a cache invalidation) on the elimination chain.
constexpr int kThrSlot = 3 * kNB;   // offset from bc

// Cholesky factor and inverse of one 32x32 diagonal tile, in FP64, by one
// wave.  Lt (column-major, ld 33) holds the lower triangle of the tile; rows
// and columns >= jb hold the identity.  Lane r < 32 keeps row r of the tile,
// lane 32 + q keeps column q of X = L^{-1}, starting from the unit vector
// e_q.  One right-looking loop over the columns c serves both halves: the
// pivot l_cc is broadcast by readlane, column c is scaled by 1/l_cc (the
// pivot itself becomes sqrt of it), its entries l_ic go to LDS (bc), and every
// lane updates v[i] -= v[c] * l_ic for i > c.  For a row of the tile that is
// the Cholesky update of its remaining columns; for a column of X it is the
// forward substitution step x_iq -= l_ic x_cq after x_cq was divided by
// l_cc.  Entries above the diagonal of the tile rows are not meaningful and
// never read.  A pivot that is not > 0 records its column with atomicMin
// (NaN propagates).  Out: L in Lt (upper triangle zero), X in Dt.  NC (8,
// 16 or 32, >= jb) bounds the columns stepped through: the leading NC x NC
// part of Lt and Dt is written, the rest of the identity-padded tile is
// left as it is.
//
// LDL = true: the L D L^T form of the same loop (unit L): the pivot d is
// not square-rooted (a breakdown is a zero or non-finite d, found from the
// diagonal after the loop), a row keeps the
// unscaled value t of column c for its update (a_ri -= t l_ic) and stores
// t / d (d itself on the diagonal); on the identity rows the same steps give
// Y = D^{-1} L^{-1}.  Out: L (unit, d on the diagonal) in Lt, Y in Dt.
//
// Static pivoting (L D L^T): the common form (PIV false) only tracks the
// smallest |d| (one min per column, beside the dependency chain) and
// returns false before writing anything when it is below the threshold;
// the tile, still intact in Lt, is then factored again by the form with the
// replacement (PIV true).  With the test and replacement in every step, the
// scalar registers of the loop spill and each step waits longer.
template <class T, int NC, bool LDL, bool PIV>
__device__ __noinline__ bool tile_chol_inv_k(double* Lt, double* bc, T* Dt, int jb, int col0, int32_t* status)
{
    static_assert(NC == 8 || NC == 16 || NC == 32, "tile width");
    const double thr = LDL ? readlane_d(bc[kThrSlot], 0) : 0.0;
    double dmin = __builtin_inf();
    const int lane = threadIdx.x & 63;
    const int r = lane & 31;
    const bool upper = lane >= 32;
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double l = Lt[r + c * 33];
        v[c] = upper ? (c == r ? 1.0 : 0.0) : l;
    }
    // pivot of column c: inv = 1/sqrt(l_cc) from the hardware estimate and
    // two Newton-Raphson steps y <- y (3 - d y^2) / 2, s = d inv (a short
    // dependency chain; within a few ulps of the rounded values)
    int fail = 32;
    int nrep = 0;   // (L D L^T) pivots replaced by the static pivoting threshold thr
    auto pivot = [&](int c, double& s, double& inv) {
        double d = readlane_d(v[c], c);
        if constexpr (LDL) {
            if constexpr (PIV) {
                if (c < jb && fabs(d) < thr) {   // static pivoting (a uniform branch)
                    d = d < 0.0 ? -thr : thr;
                    ++nrep;
                }
            } else {
                dmin = fmin(dmin, fabs(d));   // (identity padding: pivots 1)
            }
            const double y = recip_nr(d);
            inv = y;
            s = d;
        } else {
            fail = (c < jb && !(d > 0.0) && fail == 32) ? c : fail;
            double y = __builtin_amdgcn_rsq(d);
            y = y * __builtin_fma(-0.5 * d, y * y, 1.5);
            y = y * __builtin_fma(-0.5 * d, y * y, 1.5);
            inv = y;
            s = d * y;
        }
    };
    double s, inv;
    pivot(0, s, inv);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        // L D L^T: every row is scaled by 1/d_c but updated with its unscaled
        // value, so the factor rows hold unit L (d_c on the diagonal) and the
        // identity rows end as rows of L^{-T} D^{-1}
        const double t = v[c];
        v[c] = lane == c ? s : t * inv;
        const double tu = LDL ? t : v[c];   // the factor of this column's update
        if (c < NC - 1) {
            // column c to bc[0..31] (the upper half writes the unused
            // bc[32..63]); LDS operations of one wave complete in order, so
            // the reads below see it (compiler barrier only)
            bc[lane] = v[c];
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            // column c+1 first: its pivot overlaps the rest of the update
            v[c + 1] -= tu * bc[c + 1];
            double sn, invn;
            pivot(c + 1, sn, invn);
#pragma unroll
            for (int i = c + 2; i < NC; ++i) v[i] -= tu * bc[i];
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            s = sn;
            inv = invn;
        }
        // keep the scheduler from interleaving column steps (register pressure)
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (LDL && !PIV) {
        if (dmin < thr) return false;   // a pivot to replace: the caller runs the PIV form
    }
    if constexpr (LDL) {   // breakdown: a zero or non-finite pivot among the first jb
        double dd = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) dd = lane == c ? v[c] : dd;
        const bool bad = !upper && r < jb && !(dd != 0.0 && dd - dd == 0.0);
        const uint64_t m = __ballot(bad);
        fail = m ? __builtin_ctzll(m) : 32;
    }
    if (lane == 0 && fail < jb) atomicMin(status, col0 + fail);
    if (LDL && lane == 0 && nrep > 0) atomicAdd(status + kStReplaced, nrep);
    if (r < NC && !upper) {
#pragma unroll
        for (int c = 0; c < NC; ++c) Lt[r + c * 33] = c <= r ? v[c] : 0.0;
    }
    if (r < NC && upper) {
#pragma unroll
        for (int c = 0; c < NC; ++c) Dt[c + r * 33] = c >= r ? (T)v[c] : T(0);
    }
    return true;
}

template <class T, int NC = 32, bool LDL = false>
__device__ __forceinline__ void tile_chol_inv(double* Lt, double* bc, T* Dt, int jb, int col0, int32_t* status)
{
    if (!tile_chol_inv_k<T, NC, LDL, false>(Lt, bc, Dt, jb, col0, status))
        tile_chol_inv_k<T, NC, LDL, true>(Lt, bc, Dt, jb, col0, status);
}

// Small product of the diagonal-block factorization: acc += X Y^T with
// X(i, p), i < 64, and Y(c, p), c < 16*NB, p < 32, given by loader functions
// that load unconditionally (no masks: callers arrange that entries outside
// the operands are zeros or only reach results that are not stored).  Fully
// unrolled in two halves of 16: the operand loads of a half are issued
// before its products.
template <int NB, class T, class LX, class LY>
__device__ __forceinline__ void wave_mm(typename MM<T>::acc (&acc)[NB][4], LX ldx, LY ldy)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        T xs[4][4], ys[4][NB];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int p = 16 * h + 4 * q + lk;
#pragma unroll
            for (int b = 0; b < 4; ++b) xs[q][b] = ldx(16 * b + li, p);
#pragma unroll
            for (int b = 0; b < NB; ++b) ys[q][b] = ldy(16 * b + li, p);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = MM<T>::mfma(ys[q][bi], xs[q][bj], acc[bi][bj]);
    }
}

// C(r, c) = f(old C(r, c), (X Y^T)(r, c)) for r < mv, c < nv, keep(r, c),
// with C(r, c) at byte offset C.off + r*C.si + c*C.sk of C's array; each
// offset is a per-lane part plus a wave-uniform part (scalar offset).  FP32
// requests the old values first, so that their latency overlaps the
// products; FP64 requests them all after the products (held across them, the
// old values and the accumulators exceed the registers and spill).  The
// stores are unconditional, masked elements going to an offset past the
// array where the hardware drops them: with a branch there the compiler
// sinks the loads of the old values into it, one round trip per element.
template <int NB, class T, class LX, class LY, class Keep, class F, class Also>
__device__ __forceinline__ void wave_mm_rmw(LX ldx, LY ldy, int mv, int nv, const GOp& C, Keep keep, F f, Also also)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // drow(v, lk) = MM<T>::drow(0, lk) + MM<T>::drow(v, 0)
    const int vl = C.off + li * C.si + MM<T>::drow(0, lk) * C.sk;
    auto voff = [&](int bi, int bj, int v) {
        const int r = 16 * bj + li, c = 16 * bi + MM<T>::drow(v, lk);
        return (r < mv && c < nv && keep(r, c)) ? vl : kOffNone;
    };
    auto soff = [&](int bi, int bj, int v) { return uni(16 * bj * C.si + (16 * bi + MM<T>::drow(v, 0)) * C.sk); };
    T old[NB][4][4];
    auto load_old = [&]() {
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int v = 0; v < 4; ++v) old[bi][bj][v] = gload_s(C, voff(bi, bj, v), soff(bi, bj, v), T(0));
    };
    if constexpr (sizeof(T) == 4) load_old();
    typename MM<T>::acc acc[NB][4];
    zero_acc(acc);
    wave_mm<NB, T>(acc, ldx, ldy);
    if constexpr (sizeof(T) == 8) load_old();
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T nv_ = f(old[bi][bj][v], acc[bi][bj][v]);
                gstore_s(C, voff(bi, bj, v), soff(bi, bj, v), nv_);
                also(16 * bj + li, 16 * bi + MM<T>::drow(v, lk), nv_);
            }
}

constexpr int kPbLd = 228;   // leading dimension of the LDS copy of the rows below a tile (<= 224 rows)

// Cholesky factorization of the w x w diagonal block (w <= 256) of panel k
// and the inverse D = L_kk^{-1}, by one workgroup, right-looking over 32
// columns at a time.  The running inverse uses the block form of L D = I:
// block row I of D is D_II (E_I - sum_{K<I} L_IK D_K), accumulated as the
// columns of L become final.  Step J (tile columns J .. J+jb):
//   1. the tile, fully updated, is factored and inverted by wave 0
//      (tile_chol_inv): L_JJ -> panel, D_JJ -> D;
//   2. the rows below: P = A[J+jb:w, J:J+jb] D_JJ^T -> panel and LDS (Pb);
//      block row J of D: D_J[:, 0:J] = D_JJ X_J[:, 0:J], in place;
//   3. trailing updates, 64x32 tiles dealt to the four waves:
//      A[J+jb:, J+jb:] -= P P^T (lower triangle) and
//      X[J+jb:, 0:J+jb] -= P D_J (columns J .. J+jb written for the first time).
// Products run on the matrix cores; P and D_JJ are read from LDS.
//
// LDL = true: L D L^T of the diagonal block (unit L with D on its diagonal,
// and Y = D^{-1} L^{-1} as the stored inverse, so that the panel solve and
// the rows below stay one product A_rows Y^T): the tile step is the L D L^T
// form of tile_chol_inv, the trailing update is A -= L (D L^T) and the rows
// of the running inverse take (L D) Y_J.
template <class T, bool LDL = false>
__device__ __noinline__ void task_fact(const SchedArgs& a, int k, double* Lt, T* Dt, T* Pb)
{
    typedef typename MM<T>::acc acc_t;
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k];
    const int w = pl.lcol[k] - f + 1;
    const int64_t ld = pl.stride[k];
    T* A = static_cast<T*>(a.panels) + pl.panel_off[k];
    T* D = static_cast<T*>(a.dinv) + pl.dinv_off[k];
    const int64_t nA = ld * w, nD = (int64_t)w * w;
    const GOp gA = make_gop(A, nA, 0, 1, ld);   // A(i, p) at i + p*ld
    const GOp gD = make_gop(D, nD, 0, 1, w);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double* bc = Lt + kNB * 33;
    __shared__ int s_next;   // next trailing tile to deal
    __shared__ double dcur[kNB];   // (L D L^T) this step's pivots
    bool ready = false;      // Lt/Dt already hold this step's factored tile
    // the off-diagonal tiles of the inverse here, or (a chain block with an
    // INV item) only its diagonal tiles, D_JJ
    const bool full = LDL || a.inv_item == nullptr || a.inv_item[k] < 0;
    for (int J = 0; J < w; J += kNB) {
        const int jb = min(kNB, w - J);
        const int R = w - J - jb;   // rows below the tile inside the block
        // 1. tile (identity padded) -> Lt; factor and invert (done ahead,
        // during the previous step's trailing updates, from the second step on)
        if (!ready) {
            for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
                const int r = idx & 31, c = idx >> 5;
                Lt[r + c * 33] = (r < jb && c < jb) ? (c <= r ? (double)A[(J + r) + (int64_t)(J + c) * ld] : 0.0)
                                                    : (r == c ? 1.0 : 0.0);
            }
            __syncthreads();
            if (wave == 0) tile_chol_inv<T, 32, LDL>(Lt, bc, Dt, jb, f + J, a.status);
        }
        if (tid == 0) s_next = 0;
        __syncthreads();
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            const int r = idx & 31, c = idx >> 5;
            if (r < jb && c <= r) {
                A[(J + r) + (int64_t)(J + c) * ld] = (T)Lt[r + c * 33];
                D[(J + r) + (int64_t)(J + c) * w] = Dt[r + c * 33];
            }
        }
        if (LDL && tid < kNB) dcur[tid] = Lt[tid + tid * 33];
        // 2a. rows below: P = A_rows D_JJ^T (wave v: rows 64v ..)
        const int r0 = 64 * wave;
        if (r0 < R) {
            acc_t acc[2][4];
            zero_acc(acc);
            const int gbase = gA.off + (J + jb + r0) * gA.si + J * gA.sk;
            // (R > 0 implies jb = 32: full inner range)
            wave_mm<2, T>(acc, [&](int i, int p) { return gload<T>(gA, gbase + i * gA.si + p * gA.sk); },
                          [&](int c, int p) { return Dt[c + p * 33]; });
            wave_store<T>(acc, min(64, R - r0), jb, [&](int r, int c, T v) {
                Pb[(r0 + r) + c * kPbLd] = v;
                A[(J + jb + r0 + r) + (int64_t)(J + c) * ld] = v;
            });
        }
        // 2b. block row J of D for columns < J (transposed: rows c of the
        // product are columns of D), each wave a 64-column slice, in place
        for (int c0 = 64 * wave; full && c0 < J; c0 += 64 * (kThreads / 64)) {
            acc_t acc[2][4];
            zero_acc(acc);
            // with jb < 32 (last step) the inner indices p >= jb read entries
            // of D below row w (finite: the top of the next column, or zero
            // past the array) that meet D_JJ[r][p] = 0 for r < jb
            wave_mm<2, T>(acc, [&](int i, int p) { return gload<T>(gD, gD.off + (J + p) * gD.si + (c0 + i) * gD.sk); },
                          [&](int c, int p) { return Dt[c + p * 33]; });
            wave_store<T>(acc, min(64, J - c0), jb,
                          [&](int r, int c, T v) { D[(J + c) + (int64_t)(c0 + r) * w] = v; });
        }
        __syncthreads();
        if (R == 0) break;
        // 3. trailing updates: syrk tiles (rt, ct) with ct*32 < rt*64 + 64,
        // then inverse tiles (rt, ct), ct*32 < J + jb, dealt to the waves one
        // at a time.  Tile 0 holds the whole next diagonal tile: the wave that
        // takes it also writes the tile's new lower entries (identity padded)
        // to Lt and then factors and inverts it, while the other waves go on
        // with the remaining tiles.
        const int nrt = (R + 63) >> 6, ncs = (R + 31) >> 5, nci = (J + jb + 31) >> 5;
        int nsyrk = 0;
        for (int rt = 0; rt < nrt; ++rt) nsyrk += min(ncs, 2 * rt + 2);
        const int ntiles = nsyrk + (full ? nrt * nci : 0);
        const int jn = min(kNB, R);   // width of the next tile
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&s_next, 1);
            t = __shfl(t, 0);
            if (t >= ntiles) break;
            int rt = 0, ct = t;
            const bool syrk = t < nsyrk;
            if (syrk) {
                while (ct >= min(ncs, 2 * rt + 2)) { ct -= min(ncs, 2 * rt + 2); ++rt; }
            } else {
                rt = (t - nsyrk) / nci;
                ct = (t - nsyrk) - rt * nci;
            }
            const int i0 = 64 * rt, c0 = 32 * ct;
            const int mv = min(64, R - i0);
            // rows i >= mv (and columns c >= nv below) only reach results
            // that are not stored; Pb is padded for their indices
            auto ldx = [&](int i, int p) { return Pb[(i0 + i) + p * kPbLd]; };
            // (L D L^T) the facing rows of the syrk tiles and the rows of the
            // inverse tiles carry D
            auto ldxd = [&](int i, int p) { return LDL ? (T)(Pb[(i0 + i) + p * kPbLd] * dcur[p]) : Pb[(i0 + i) + p * kPbLd]; };
            auto ldyd = [&](int c, int p) { return LDL ? (T)(Pb[(c0 + c) + p * kPbLd] * dcur[p]) : Pb[(c0 + c) + p * kPbLd]; };
            auto sub = [](T o, T v) { return o - v; };
            if (syrk) {
                const int nv = min(32, R - c0);
                GOp cA = gA;
                cA.off = uni(gA.off + (J + jb + i0) * gA.si + (J + jb + c0) * gA.sk);
                if (t == 0) {
                    for (int idx = lane; idx < kNB * kNB; idx += 64) {
                        const int r = idx & 31, c = idx >> 5;
                        Lt[r + c * 33] = r == c && r >= jn ? 1.0 : 0.0;
                    }
                    wave_mm_rmw<2, T>(
                        ldx, ldyd, mv, nv, cA, [&](int r, int c) { return r >= c; }, sub, [&](int r, int c, T v) {
                            if (r < jn && c < jn && c <= r) Lt[r + c * 33] = (double)v;
                        });
                    tile_chol_inv<T, 32, LDL>(Lt, bc, Dt, jn, f + J + jb, a.status);
                } else {
                    wave_mm_rmw<2, T>(
                        ldx, ldyd, mv, nv, cA, [&](int r, int c) { return i0 + r >= c0 + c; }, sub,
                        [](int, int, T) {});
                }
            } else {
                const int nv = min(32, J + jb - c0);
                auto ldy = [&](int c, int p) { return gload<T>(gD, gD.off + (J + p) * gD.si + (c0 + c) * gD.sk); };
                if (c0 >= J) {   // columns written for the first time
                    acc_t acc[2][4];
                    zero_acc(acc);
                    wave_mm<2, T>(acc, ldxd, ldy);
                    wave_store<T>(acc, mv, nv,
                                  [&](int r, int c, T v) { D[(J + jb + i0 + r) + (int64_t)(c0 + c) * w] = -v; });
                } else {
                    GOp cD = gD;
                    cD.off = uni(gD.off + (J + jb + i0) * gD.si + c0 * gD.sk);
                    wave_mm_rmw<2, T>(ldxd, ldy, mv, nv, cD, [](int, int) { return true; }, sub, [](int, int, T) {});
                }
            }
        }
        __syncthreads();
        ready = true;
    }
}

// ---------------------------------------------------------------- INV(k)
// The off-diagonal tiles of D = L_kk^{-1} after a FACT that stored L_kk and
// the diagonal tiles D_JJ = L_JJ^{-1} only (blocks of elimination chains: the
// inverse is then built beside the chain instead of inside FACT).  Block
// forward substitution on L D = I, column block c of D at a time:
//   D_Jc = -D_JJ (sum_{c <= K < J} L_JK D_Kc),   J = c+1 .. nb-1,
// one column block per wave (c = wave, wave + 4, ...).  Per step: S = the
// sum (32 x 32, inner dimension 32 (J - c), operands read from the panel and
// from D, the D_Kc written by this wave's earlier steps), S to LDS, then
// -D_JJ S on the matrix cores, written to D.  Rows of a partial last block
// beyond w only reach results that are not stored (operands past the
// arrays read zeros).
template <class T>
__device__ __noinline__ void task_inv(const SchedArgs& a, int k, T* Pb)
{
    typedef typename MM<T>::acc acc_t;
    const DevPlan& pl = a.pl;
    const int w = pl.lcol[k] - pl.fcol[k] + 1;
    const int64_t ld = pl.stride[k];
    const T* A = static_cast<const T*>(a.panels) + pl.panel_off[k];
    T* D = static_cast<T*>(a.dinv) + pl.dinv_off[k];
    const int nb = (w + kNB - 1) / kNB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    T* Sl = Pb + wave * (kNB * 33);   // this wave's S (32 x 32, ld 33)
    for (int c = wave; c + 1 < nb; c += kThreads / 64) {
        for (int J = c + 1; J < nb; ++J) {
            // S(r, q) = sum_p L(32J + r, 32c + p) D(32c + p, 32c + q)
            acc_t acc[2][2];
            zero_acc(acc);
            wave_gemm<2, T, 2>(acc, make_gop(A, ld * w, kNB * J + (int64_t)kNB * c * ld, 1, ld),
                               make_gop(D, (int64_t)w * w, kNB * c + (int64_t)kNB * c * w, w, 1), kNB * (J - c));
            wave_store<T>(acc, kNB, kNB, [&](int r, int q, T v) { Sl[r + q * 33] = v; });
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // (LDS operations of a wave complete in order)
            // D_Jc(r, q) = -sum_t D_JJ(r, t) S(t, q)
            const GOp gJ = make_gop(D, (int64_t)w * w, kNB * J + (int64_t)kNB * J * w, 1, w);
            acc_t acc2[2][2];
            zero_acc(acc2);
#pragma unroll
            for (int st = 0; st < kNB / 4; ++st) {
                const int t = 4 * st + lk;
                T xs[2], ys[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    xs[b] = gload<T>(gJ, gJ.off + (16 * b + li) * gJ.si + t * gJ.sk);
                    ys[b] = Sl[t + (16 * b + li) * 33];
                }
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) acc2[bi][bj] = MM<T>::mfma(ys[bi], xs[bj], acc2[bi][bj]);
            }
            const int jb = min(kNB, w - kNB * J);
            wave_store<T>(acc2, jb, kNB, [&](int r, int q, T v) {
                D[(kNB * J + r) + (int64_t)(kNB * c + q) * w] = -v;
            });
            // this wave's next steps read D_Jc: stores complete before their loads
            __builtin_amdgcn_s_waitcnt(0);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
    }
}

// ---------------------------------------------------------------- FACT(k), L U
// L U factorization without pivoting (the static pivoting of Section III:
// the elimination order is the analysis' order) of one 32x32 diagonal tile
// and the two inverses the panel solves use, in FP64, by one wave.  Lt
// (column-major, ld 33) holds the whole tile; rows and columns >= jb hold
// the identity.  Pass 1 keeps the tile twice: lane r < 32 holds row r, lane
// 32 + q holds column q.  Step c: the pivot u_cc is broadcast by readlane;
// the entries of column c below it become l_rc = a_rc / u_cc (in the row
// lanes, and in column lane c); every lane puts one value in LDS (row lane r
// its l_rc, column lane q its u_cq), so that row lane r > c updates
// a_rq -= l_rc u_cq (q > c) with u_cq from LDS and column lane q > c updates
// a_pq -= l_pc u_cq (p > c) with l_pc from LDS: the same operands in both
// copies.  Pass 2, from L\U in Lt: lane q < 32 forms column q of
// X = L^{-1} by forward substitution with the unit L (x_i -= l_ic x_c, i > c),
// lane 32 + q column q of Y = U^{-T} by forward substitution with U^T
// (y_c /= u_cc, then y_i -= u_ci y_c, i > c).  Out: L\U in Lt (unit L
// strictly below the diagonal, U on and above), X in Dt (column-major, ld
// 33), Y (rounded to T) in Yg[i + q*ldy] for q <= i < jb.  A zero or
// non-finite pivot among the first jb records its column with atomicMin.
//
// Static pivoting as in tile_chol_inv: the common form (PIV false) tracks
// the smallest |u_cc| and returns false, with Lt intact, when one is below
// the threshold; the PIV form replaces.
template <class T, bool PIV>
__device__ __noinline__ bool tile_lu_inv_k(double* Lt, double* bc, T* Dt, T* Yg, int ldy, int jb, int col0,
                                           int32_t* status)
{
    const double thr = readlane_d(bc[kThrSlot], 0);
    double dmin = __builtin_inf();
    const int lane = threadIdx.x & 63;
    const int r = lane & 31;
    const bool colh = lane >= 32;
    double v[32], invp[32];   // invp: the inverse pivots (uniform), for pass 2
#pragma unroll
    for (int c = 0; c < 32; ++c) v[c] = colh ? Lt[c + r * 33] : Lt[r + c * 33];
    // PIV: a replaced pivot only changes 1/u_cc here (the entries u_cc of
    // lanes r == c are not read again by the loop) and is written to the
    // tile's diagonal after it (uniform selects: a branch in the body stops
    // the full unroll and sends the arrays to scratch)
    const double ithr = PIV ? recip_nr(thr) : 0.0;
    uint32_t repmask = 0;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const double d = readlane_d(v[c], c);   // row lane c: u_cc
        double y = recip_nr(d);
        if constexpr (PIV) {
            const bool rp = c < jb && fabs(d) < thr;
            y = rp ? (d < 0.0 ? -ithr : ithr) : y;
            repmask |= rp ? 1u << c : 0u;
        } else {
            dmin = fmin(dmin, fabs(d));   // (identity padding: pivots 1)
        }
        invp[c] = y;
        if (!colh && r > c) v[c] *= y;   // l_rc
        // row lanes: l_rc (meaningful for r > c); column lanes: u_cq
        bc[lane] = v[c];
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // column lane c takes its scaled entries l_pc (p > c) from the row
        // lanes' values, the others update
        const double own = (r > c) ? v[c] : 0.0;
        const bool take = colh && r == c;
        const int bo = colh ? 0 : 32;
#pragma unroll
        for (int q = c + 1; q < 32; ++q) {
            const double b = bc[bo + q];
            v[q] = take ? b : v[q] - own * b;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!PIV) {
        if (dmin < thr) return false;   // a pivot to replace: the caller runs the PIV form
    }
    // breakdown: a zero or non-finite pivot among the first jb (after replacement)
    double dd = 0.0;
#pragma unroll
    for (int c = 0; c < 32; ++c) dd = (r == c) ? v[c] : dd;
    const bool replaced = (repmask >> r) & 1u;
    if (replaced) dd = dd < 0.0 ? -thr : thr;
    const bool bad = !colh && r < jb && !(dd != 0.0 && dd - dd == 0.0);
    const uint64_t m = __ballot(bad);
    if (lane == 0 && m) atomicMin(status, col0 + (int)__builtin_ctzll(m));
    if (lane == 0 && repmask) atomicAdd(status + kStReplaced, (int)__builtin_popcount(repmask));
    if (!colh) {
#pragma unroll
        for (int c = 0; c < 32; ++c) Lt[r + c * 33] = v[c];
        if (replaced) Lt[r + r * 33] = dd;
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    // pass 2: X (lanes < 32) and Y (lanes >= 32), column r of each
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = i == r ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        if (colh) v[c] *= invp[c];
        const double xc = v[c];
        // coefficient i: U(c, i) at c + 33 i for the Y lanes, L(i, c) at i + 33 c for the X lanes
        const int base = colh ? c : 33 * c, step = colh ? 33 : 1;
#pragma unroll
        for (int i = c + 1; i < 32; ++i) v[i] -= Lt[base + i * step] * xc;
        __builtin_amdgcn_sched_barrier(0);
    }
    if (!colh) {
#pragma unroll
        for (int c = 0; c < 32; ++c) Dt[c + r * 33] = c >= r ? (T)v[c] : T(0);
    } else if (r < jb) {
#pragma unroll
        for (int c = 0; c < 32; ++c)
            if (c >= r && c < jb) Yg[c + (int64_t)r * ldy] = (T)v[c];
    }
    return true;
}

template <class T>
__device__ __forceinline__ void tile_lu_inv(double* Lt, double* bc, T* Dt, T* Yg, int ldy, int jb, int col0,
                                            int32_t* status)
{
    if (!tile_lu_inv_k<T, false>(Lt, bc, Dt, Yg, ldy, jb, col0, status))
        tile_lu_inv_k<T, true>(Lt, bc, Dt, Yg, ldy, jb, col0, status);
}

// L U factorization of the w x w diagonal block (w <= 256) of panel k, in
// place in the L panel (unit L below the diagonal, U on and above), with the
// inverses X = L_kk^{-1} (L inverse array) and Y = U_kk^{-T} (U inverse
// array), both lower triangular, by one workgroup, right-looking over 32
// columns at a time.  Step J (tile columns J .. J+jb):
//   1. the tile, fully updated, is factored and inverted by wave 0
//      (tile_lu_inv): L\U_JJ -> panel, X_JJ -> X, Y_JJ -> Y;
//   2. rows below: P = A[J+jb:w, J:J+jb] Y_JJ^T (= L rows) -> panel and LDS;
//      columns to the right, transposed: Q = A[J:J+jb, J+jb:w]^T X_JJ^T
//      (= U^T rows) -> the panel's upper part (U_J,right); block rows J of
//      the inverses: X_J[:, 0:J] = X_JJ X_J[:, 0:J], Y_J[:, 0:J] = Y_JJ Y_J[:, 0:J];
//   3. trailing updates, 64x32 tiles dealt to the four waves:
//      A[J+jb:, J+jb:] -= P Q^T (the whole square), X[J+jb:, 0:J+jb] -= P X_J
//      and Y[J+jb:, 0:J+jb] -= Q Y_J (columns J .. J+jb written for the first
//      time).  The wave taking tile 0 (which holds the next diagonal tile)
//      writes it to LDS and factors it while the others go on.
// P is read from LDS, Q and the inverses' block rows from global memory
// (written by this workgroup earlier in the step).
template <class T>
__device__ __noinline__ void task_fact_lu(const SchedArgs& a, int k, double* Lt, T* Dt, T* Pb)
{
    typedef typename MM<T>::acc acc_t;
    const DevPlan& pl = a.pl;
    const int f = pl.fcol[k];
    const int w = pl.lcol[k] - f + 1;
    const int64_t ld = pl.stride[k];
    T* A = static_cast<T*>(a.panels) + pl.panel_off[k];
    T* X = static_cast<T*>(a.dinv) + pl.dinv_off[k];
    T* Y = X + a.uinv;
    const int64_t nA = ld * w, nD = (int64_t)w * w;
    const GOp gA = make_gop(A, nA, 0, 1, ld);   // A(i, p) at i + p*ld
    const GOp gX = make_gop(X, nD, 0, 1, w);
    const GOp gY = make_gop(Y, nD, 0, 1, w);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double* bc = Lt + kNB * 33;
    __shared__ int s_next;
    bool ready = false;
    for (int J = 0; J < w; J += kNB) {
        const int jb = min(kNB, w - J);
        const int R = w - J - jb;
        if (!ready) {
            for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
                const int r = idx & 31, c = idx >> 5;
                Lt[r + c * 33] = (r < jb && c < jb) ? (double)A[(J + r) + (int64_t)(J + c) * ld] : (r == c ? 1.0 : 0.0);
            }
            __syncthreads();
            if (wave == 0) tile_lu_inv<T>(Lt, bc, Dt, Y + J + (int64_t)J * w, w, jb, f + J, a.status);
        }
        if (tid == 0) s_next = 0;
        __syncthreads();
        for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
            const int r = idx & 31, c = idx >> 5;
            if (r < jb && c < jb) {
                A[(J + r) + (int64_t)(J + c) * ld] = (T)Lt[r + c * 33];
                if (c <= r) X[(J + r) + (int64_t)(J + c) * w] = Dt[r + c * 33];
            }
        }
        __syncthreads();   // Y_JJ (global, from wave 0) and the tile are in place
        const int r0 = 64 * wave;
        if (r0 < R) {
            // 2a. P = A_rows Y_JJ^T (R > 0 implies jb = 32)
            {
                acc_t acc[2][4];
                zero_acc(acc);
                const int gbase = gA.off + (J + jb + r0) * gA.si + J * gA.sk;
                wave_mm<2, T>(acc, [&](int i, int p) { return gload<T>(gA, gbase + i * gA.si + p * gA.sk); },
                              [&](int c, int p) { return gload<T>(gY, gY.off + (J + c) * gY.si + (J + p) * gY.sk); });
                wave_store<T>(acc, min(64, R - r0), jb, [&](int r, int c, T v) {
                    Pb[(r0 + r) + c * kPbLd] = v;
                    A[(J + jb + r0 + r) + (int64_t)(J + c) * ld] = v;
                });
            }
            // 2a'. Q = A[J:J+jb, right]^T X_JJ^T, stored as U_J,right
            {
                acc_t acc[2][4];
                zero_acc(acc);
                wave_mm<2, T>(acc,
                              [&](int i, int p) { return gload<T>(gA, gA.off + (J + p) * gA.si + (J + jb + r0 + i) * gA.sk); },
                              [&](int c, int p) { return Dt[c + p * 33]; });
                // (the upper rows of the inverse tile are zero: products over
                // p > c vanish)
                wave_store<T>(acc, min(64, R - r0), jb,
                              [&](int r, int c, T v) { A[(J + c) + (int64_t)(J + jb + r0 + r) * ld] = v; });
            }
        }
        // 2b. block rows J of X and Y for columns < J, in place; each wave a
        // 64-column slice of one of them
        for (int t = wave; t < 2 * ((J + 63) >> 6); t += kThreads / 64) {
            const bool isY = (t & 1) != 0;
            const int c0 = 64 * (t >> 1);
            const GOp& g = isY ? gY : gX;
            T* Z = isY ? Y : X;
            acc_t acc[2][4];
            zero_acc(acc);
            if (isY)
                wave_mm<2, T>(acc, [&](int i, int p) { return gload<T>(g, g.off + (J + p) * g.si + (c0 + i) * g.sk); },
                              [&](int c, int p) { return gload<T>(gY, gY.off + (J + c) * gY.si + (J + p) * gY.sk); });
            else
                wave_mm<2, T>(acc, [&](int i, int p) { return gload<T>(g, g.off + (J + p) * g.si + (c0 + i) * g.sk); },
                              [&](int c, int p) { return Dt[c + p * 33]; });
            wave_store<T>(acc, min(64, J - c0), jb, [&](int r, int c, T v) { Z[(J + c) + (int64_t)(c0 + r) * w] = v; });
        }
        __syncthreads();
        if (R == 0) break;
        // 3. trailing updates: A tiles (rt, ct) over the whole R x R square,
        // then X tiles and Y tiles (rt, ct), ct*32 < J + jb
        const int nrt = (R + 63) >> 6, ncs = (R + 31) >> 5, nci = (J + jb + 31) >> 5;
        const int nsq = nrt * ncs, ninv = nrt * nci;
        const int ntiles = nsq + 2 * ninv;
        const int jn = min(kNB, R);
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&s_next, 1);
            t = __shfl(t, 0);
            if (t >= ntiles) break;
            auto sub = [](T o, T v) { return o - v; };
            if (t < nsq) {
                const int rt = t / ncs, ct = t - rt * ncs;
                const int i0 = 64 * rt, c0 = 32 * ct;
                const int mv = min(64, R - i0), nv = min(32, R - c0);
                auto ldx = [&](int i, int p) { return Pb[(i0 + i) + p * kPbLd]; };
                auto ldq = [&](int c, int p) {
                    return gload<T>(gA, gA.off + (J + p) * gA.si + (J + jb + c0 + c) * gA.sk);
                };
                GOp cA = gA;
                cA.off = uni(gA.off + (J + jb + i0) * gA.si + (J + jb + c0) * gA.sk);
                if (t == 0) {
                    for (int idx = lane; idx < kNB * kNB; idx += 64) {
                        const int r = idx & 31, c = idx >> 5;
                        Lt[r + c * 33] = r == c && r >= jn ? 1.0 : 0.0;
                    }
                    wave_mm_rmw<2, T>(
                        ldx, ldq, mv, nv, cA, [](int, int) { return true; }, sub, [&](int r, int c, T v) {
                            if (r < jn && c < jn) Lt[r + c * 33] = (double)v;
                        });
                    tile_lu_inv<T>(Lt, bc, Dt, Y + (J + jb) + (int64_t)(J + jb) * w, w, jn, f + J + jb, a.status);
                } else {
                    wave_mm_rmw<2, T>(ldx, ldq, mv, nv, cA, [](int, int) { return true; }, sub, [](int, int, T) {});
                }
            } else {
                const bool isY = t >= nsq + ninv;
                const int u = t - nsq - (isY ? ninv : 0);
                const int rt = u / nci, ct = u - rt * nci;
                const int i0 = 64 * rt, c0 = 32 * ct;
                const int mv = min(64, R - i0), nv = min(32, J + jb - c0);
                const GOp& g = isY ? gY : gX;
                T* Z = isY ? Y : X;
                auto ldy = [&](int c, int p) { return gload<T>(g, g.off + (J + p) * g.si + (c0 + c) * g.sk); };
                auto ldp = [&](int i, int p) { return Pb[(i0 + i) + p * kPbLd]; };
                auto ldqr = [&](int i, int p) {
                    return gload<T>(gA, gA.off + (J + p) * gA.si + (J + jb + i0 + i) * gA.sk);
                };
                if (c0 >= J) {   // columns written for the first time
                    acc_t acc[2][4];
                    zero_acc(acc);
                    if (isY) wave_mm<2, T>(acc, ldqr, ldy);
                    else wave_mm<2, T>(acc, ldp, ldy);
                    wave_store<T>(acc, mv, nv,
                                  [&](int r, int c, T v) { Z[(J + jb + i0 + r) + (int64_t)(c0 + c) * w] = -v; });
                } else {
                    GOp cZ = g;
                    cZ.off = uni(g.off + (J + jb + i0) * g.si + c0 * g.sk);
                    if (isY) wave_mm_rmw<2, T>(ldqr, ldy, mv, nv, cZ, [](int, int) { return true; }, sub, [](int, int, T) {});
                    else wave_mm_rmw<2, T>(ldp, ldy, mv, nv, cZ, [](int, int) { return true; }, sub, [](int, int, T) {});
                }
            }
        }
        __syncthreads();
        ready = true;
    }
}

// ---------------------------------------------------------------- TRSM(k, rows)
// Rows [row0, row0+nrows) (nrows <= 64 * (4 / ceil(w / 64))) of panel k below its diagonal block
// are replaced by B L_kk^{-T} = B D^T.  Wave v computes the 64 output columns
// starting at 64v; the inner range stops at the diagonal of the lower
// triangular D.  poff / doff select the panel array and the inverse (L U:
// the L rows take U_kk^{-T}, giving A_off U_kk^{-1}; the U^T rows take
// L_kk^{-1}, giving A_up^T L_kk^{-T}).
// RB: 16-row blocks per wave tile (4: 64-row wave tiles; 1: the thin items
// of elimination chains, a quarter of the work per wave).
template <class T, int RB = 4>
__device__ __noinline__ void task_trsm(const SchedArgs& a, int k, int row0, int nrows, int64_t poff = 0,
                                       int64_t doff = 0)
{
    const DevPlan& pl = a.pl;
    const int w = pl.lcol[k] - pl.fcol[k] + 1;
    const int64_t ld = pl.stride[k];
    T* P = static_cast<T*>(a.panels) + poff + pl.panel_off[k];
    auto B = glob(P + row0);
    const T* D = static_cast<const T*>(a.dinv) + doff + pl.dinv_off[k];
    const int wave = threadIdx.x >> 6;
    typename MM<T>::acc acc[4][RB];
    zero_acc(acc);
    // (16 RB) x 64 wave tiles: ncb column blocks of the output, and 4/ncb
    // blocks of 16 RB rows (a chunk has 16 RB * (4/ncb) rows), so narrow
    // panels keep all four waves busy
    constexpr int TR = 16 * RB;
    const int ncb = (w + 63) >> 6, nrb = 4 / ncb;
    const int cb = wave % ncb, rb = wave / ncb;
    const int c0 = 64 * cb, r0 = TR * rb;
    const int nv = min(64, w - c0);
    const bool on = rb < nrb && nv > 0 && r0 < nrows;
    if (on)
        tile_gemm<4, T, RB>(acc, make_gop(P, ld * w, row0 + r0, 1, ld), make_gop(D, (int64_t)w * w, c0, 1, w),
                            min(w, c0 + 64), a.split != 0);
    __syncthreads();   // every wave has read all of B before any result is written
    if (on)
        wave_store<T>(acc, min(TR, nrows - r0), nv,
                      [&](int r, int c, T v) { B[(r0 + r) + (int64_t)(c0 + c) * ld] = v; });
}

// Rows [row0, row0+nrows) (nrows <= 64) of a chain block's panel below its
// diagonal block, by block forward substitution with the diagonal tiles of
// the inverse only (the rest of L_kk^{-1} is formed beside the chain, by the
// INV item):
//   X_J = (B_J - sum_{K<J} X_K L_JK^T) D_JJ^T,   J = 0 .. NBK-1   (X = B L_kk^{-T}),
// wave v taking rows 16v .. 16v+15.  The finished column blocks X_K stay in
// registers in the operand layout of the products (xop[K][s] = X(r, 32K + 4s
// + l/16), r = l%16); each new block passes once through LDS from the
// result layout to the operand layout.  NBK = number of 32-column blocks
// (every loop fully unrolled: a branch in them sends xop to scratch).
// Entries past a partial last block read zeros (operands past the arrays)
// or finite panel entries that only meet zeros of D.
template <class T, int NBK>
__device__ __noinline__ void task_trsm_subst(const SchedArgs& a, int k, int row0, int nrows, T* Pb)
{
    typedef typename MM<T>::acc acc_t;
    const DevPlan& pl = a.pl;
    const int w = pl.lcol[k] - pl.fcol[k] + 1;
    const int64_t ld = pl.stride[k];
    T* P = static_cast<T*>(a.panels) + pl.panel_off[k];
    const T* D = static_cast<const T*>(a.dinv) + pl.dinv_off[k];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = 16 * wave;
    if (r0 >= nrows) return;
    const int mv = min(16, nrows - r0);
    const GOp gP = make_gop(P, ld * w, row0 + r0, 1, ld);   // rows of this wave: X(r, j) at r + j*ld
    const GOp gL = make_gop(P, ld * w, 0, 1, ld);           // L_kk(i, j) at i + j*ld
    const GOp gD = make_gop(D, (int64_t)w * w, 0, 1, w);    // D(i, j) at i + j*w
    T* Sl = Pb + wave * (kNB * 17);   // this wave's 16 x 32 staging block (ld 17)
    T xop[NBK][8];
#pragma unroll
    for (int J = 0; J < NBK; ++J) {
        acc_t acc[2][1];
        zero_acc(acc);
        // the block of B, in the result layout: row li, column 16 bi + drow(v, l/16)
        T bj[2][4];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                bj[bi][v] = gload<T>(gP, gP.off + li * gP.si + (kNB * J + 16 * bi + MM<T>::drow(v, lk)) * gP.sk);
        // S = sum_{K<J} X_K L_JK^T: Y(c, p) = L(32J + c, 32K + p), X(r, p) = X_K
#pragma unroll
        for (int K = 0; K < J; ++K) {
            T y0[8], y1[8];
#pragma unroll
            for (int st = 0; st < 8; ++st) {
                const int pcol = kNB * K + 4 * st + lk;
                y0[st] = gload<T>(gL, (kNB * J + li) * gL.si + pcol * gL.sk);
                y1[st] = gload<T>(gL, (kNB * J + 16 + li) * gL.si + pcol * gL.sk);
            }
#pragma unroll
            for (int st = 0; st < 8; ++st) {
                acc[0][0] = MM<T>::mfma(y0[st], xop[K][st], acc[0][0]);
                acc[1][0] = MM<T>::mfma(y1[st], xop[K][st], acc[1][0]);
            }
        }
        // T_J = B_J - S, to the operand layout through LDS
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v) Sl[li + (16 * bi + MM<T>::drow(v, lk)) * 17] = bj[bi][v] - acc[bi][0][v];
        __atomic_signal_fence(__ATOMIC_SEQ_CST);   // (LDS operations of a wave complete in order)
        T tj[8];
#pragma unroll
        for (int st = 0; st < 8; ++st) tj[st] = Sl[li + (4 * st + lk) * 17];
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // X_J = T_J D_JJ^T: Y(c, t) = D(32J + c, 32J + t)
        acc_t acc2[2][1];
        zero_acc(acc2);
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int t = kNB * J + 4 * st + lk;
            const T d0 = gload<T>(gD, (kNB * J + li) * gD.si + t * gD.sk);
            const T d1 = gload<T>(gD, (kNB * J + 16 + li) * gD.si + t * gD.sk);
            acc2[0][0] = MM<T>::mfma(d0, tj[st], acc2[0][0]);
            acc2[1][0] = MM<T>::mfma(d1, tj[st], acc2[1][0]);
        }
        // X_J to the panel and, in the operand layout, to xop[J]
        auto out = glob(P);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 16 * bi + MM<T>::drow(v, lk);
                const T x = acc2[bi][0][v];
                Sl[li + c * 17] = x;
                if (li < mv && kNB * J + c < w) out[(row0 + r0 + li) + (int64_t)(kNB * J + c) * ld] = x;
            }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
        for (int st = 0; st < 8; ++st) xop[J][st] = Sl[li + (4 * st + lk) * 17];
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
}

template <class T>
__device__ __forceinline__ void trsm_subst(const SchedArgs& a, int k, int row0, int nrows, T* Pb)
{
    switch ((a.pl.lcol[k] - a.pl.fcol[k] + kNB) / kNB) {
    case 4: task_trsm_subst<T, 4>(a, k, row0, nrows, Pb); break;
    case 5: task_trsm_subst<T, 5>(a, k, row0, nrows, Pb); break;
    case 6: task_trsm_subst<T, 6>(a, k, row0, nrows, Pb); break;
    case 7: task_trsm_subst<T, 7>(a, k, row0, nrows, Pb); break;
    default: task_trsm_subst<T, 8>(a, k, row0, nrows, Pb); break;
    }
}

// ---------------------------------------------------------------- UPDATE
// W = L_k[row0 : row0+mrows] * L_k[col0 : col0+ncols]^T (inner dimension =
// width of k), C_j[rmap(row), rmap(col)] -= W on the lower triangle of j.
// rmap (precomputed from the symbolic structure) gives, for every panel row
// of k from the first block facing j on, its row inside panel j; for facing
// rows that is also the column of j.  Two tile shapes: ncols <= 64 and
// mrows <= 256 (the four waves cover 64 rows each), or 64 < ncols <= 128 and
// mrows <= 128 (the waves form a 2x2 grid of 64x64 wave tiles).  A merged
// item (np > 1, kind bits 8..) sums the products of the np consecutive
// pieces k-np+1 .. k of a split supernode (piece p's rows are k's rows
// shifted by fcol[k] - fcol[p]) before its one scatter.  LDL: each
// piece's product is L_p[rows] D_p L_p[cols]^T, D_p on the diagonal of panel p.
// LU: the tile covers the whole square of the facing rows (no triangle);
// W_L = L_k[rows] U^T_k[cols]^T goes to j's L panel (its square diagonal
// block included), and, for rows below j's diagonal block, W_U =
// U^T_k[rows] L_k[cols]^T to j's U^T panel.
// RB = 1: a thin tile of an elimination chain, at most 64 x 64, each wave
// 16 rows of it (a quarter of the work of a 64-row wave tile).
template <class T, bool LDL = false, bool LU = false, int RB = 4>
__device__ __noinline__ void task_update(const SchedArgs& a, const int4 d0, const int4 d1, int* rpos_g, int* cpos_g)
{
    // the row and column maps are LDS arrays of the calling kernel: stated,
    // so that their accesses are LDS operations without a generic-address
    // test (whether the compiler derives it depends on the set of callers)
    auto rpos = lds(rpos_g);
    auto cpos = lds(cpos_g);
    const DevPlan& pl = a.pl;
    const int k = d0.y, j = d0.z, row0 = d0.w, np = ((d0.x >> 8) & 15) + 1;
    const int mrows = d1.x, col0 = d1.y, ncols = d1.z, mbase = d1.w;
    const int64_t ldj = pl.stride[j];
    auto Cg = glob(static_cast<T*>(a.panels) + pl.panel_off[j]);
    const int tid = threadIdx.x, wave = tid >> 6;
    if (tid < mrows) rpos[tid] = a.rmap[mbase + row0 + tid];
    if (tid < ncols) cpos[tid] = a.rmap[mbase + col0 + tid];
    __syncthreads();
    const bool square = RB == 4 && ncols > 64;
    const int r0 = square ? 64 * (wave & 1) : 16 * RB * wave;
    const int c0 = square ? 64 * (wave >> 1) : 0;
    const int mv = min(16 * RB, mrows - r0), nv = min(64, ncols - c0);
    if (mv > 0 && nv > 0) {
        const int fk = pl.fcol[k];
        // half 0: W = X Y^T with X the rows and Y the facing rows of the L
        // panels (L U: Y from the U^T panels); half 1 (L U, rows below j's
        // diagonal block only): X from the U^T panels, Y from the L panels
        const int wj = pl.lcol[j] - pl.fcol[j] + 1;
        const int nhalf = (LU && rpos[r0 + mv - 1] >= wj) ? 2 : 1;
        for (int half = 0; half < nhalf; ++half) {
            typename MM<T>::acc acc[4][RB];
            zero_acc(acc);
            const int64_t xo = (LU && half == 1) ? a.upanel : 0, yo = (LU && half == 0) ? a.upanel : 0;
            for (int p = k - np + 1; p <= k; ++p) {
                const int fp = pl.fcol[p], w = pl.lcol[p] - fp + 1, sh = fk - fp;
                const int64_t ld = pl.stride[p];
                const T* A = static_cast<const T*>(a.panels) + pl.panel_off[p];
                if constexpr (LDL)
                    tile_gemm<4, T, RB, true>(acc, make_gop(A, ld * w, row0 + r0 + sh, 1, ld),
                                              make_gop(A, ld * w, col0 + c0 + sh, 1, ld), w, a.split != 0,
                                              make_gop(A, ld * w, 0, 0, ld + 1));
                else
                    tile_gemm<4, T, RB>(acc, make_gop(A + xo, ld * w, row0 + r0 + sh, 1, ld),
                                        make_gop(A + yo, ld * w, col0 + c0 + sh, 1, ld), w, a.split != 0);
            }
            if constexpr (LU) {
                auto Cu = Cg + (half == 1 ? a.upanel : 0);
                wave_store<T>(acc, mv, nv, [&](int r, int c, T v) {
                    const int tr = rpos[r0 + r], tc = cpos[c0 + c];
                    if (half == 0 || tr >= wj) __hip_atomic_fetch_add(Cu + (int64_t)tc * ldj + tr, -v, __ATOMIC_RELAXED, AGENT);
                });
            } else {
                wave_store<T>(acc, mv, nv, [&](int r, int c, T v) {
                    const int tr = rpos[r0 + r], tc = cpos[c0 + c];
                    if (tr >= tc) __hip_atomic_fetch_add(Cg + (int64_t)tc * ldj + tr, -v, __ATOMIC_RELAXED, AGENT);
                });
            }
        }
    }
}

// ---------------------------------------------------------------- queues
__device__ __forceinline__ void push_items(const SchedArgs& a, bool hp, int base, int first, int count)
{
    int32_t* q = hp ? a.hp_queue : a.queue;
    const int cap = hp ? a.hp_total : a.total_normal;
    for (int i = threadIdx.x; i < count; i += kThreads) {
        if (base + i < cap)
            __hip_atomic_store(&q[base + i], first + i, __ATOMIC_RELAXED, AGENT);
        else
            __hip_atomic_store(&a.status[kStAbort], 2, __ATOMIC_RELAXED, AGENT);   // more pushes than slots
    }
}

// Deterministic mode: queue the items of pair p (one thread).
__device__ __forceinline__ void push_pair(const SchedArgs& a, int p)
{
    const int4 q = a.pairs[p];
    const bool hp = q.w != 0;
    int32_t* qu = hp ? a.hp_queue : a.queue;
    const int cap = hp ? a.hp_total : a.total_normal;
    const int base = __hip_atomic_fetch_add(hp ? a.hp_tail : a.qtail, q.y, __ATOMIC_RELAXED, AGENT);
    for (int i = 0; i < q.y; ++i) {
        if (base + i < cap)
            __hip_atomic_store(&qu[base + i], q.x + i, __ATOMIC_RELAXED, AGENT);
        else
            __hip_atomic_store(&a.status[kStAbort], 2, __ATOMIC_RELAXED, AGENT);
    }
}

// Deterministic mode: the pairs of source k lose their panel dependency
// (all threads of the workgroup; out of line, so that the scheduler loop
// does not keep its registers).
__device__ __noinline__ void release_pairs(const SchedArgs& a, int k)
{
    for (int p = a.kpair[k] + threadIdx.x; p < a.kpair[k + 1]; p += kThreads)
        if (__hip_atomic_fetch_add(&a.pdep[p], -1, __ATOMIC_RELAXED, AGENT) == 1) push_pair(a, p);
}

// Count down one update tile of target j (any lane); queue j when it was the
// last one.
__device__ __forceinline__ void finish_update(const SchedArgs& a, int j)
{
    if (__hip_atomic_fetch_add(&a.fact_dep[j], -1, __ATOMIC_RELAXED, AGENT) != 1) return;
    const bool hp = a.hp_cblk[j] != 0;
    const int slot = __hip_atomic_fetch_add(hp ? a.hp_tail : a.qtail, 1, __ATOMIC_RELAXED, AGENT);
    if (slot < (hp ? a.hp_total : a.total_normal))
        __hip_atomic_store(&(hp ? a.hp_queue : a.queue)[slot], j, __ATOMIC_RELAXED, AGENT);
    else
        __hip_atomic_store(&a.status[kStAbort], 2, __ATOMIC_RELAXED, AGENT);
}

// ---------------------------------------------------------------- fused small block
// A column block of width w <= 32 with at most 128 panel rows as one item:
// the panel is read into LDS once; the diagonal block is factored and
// inverted (tile_chol_inv); the rows below become A_off D^T; every update
// tile of the block (fused-tile table) is formed from the LDS copy and
// scattered with the atomics of the update items; then the item counts its
// targets down.  Blocks at the bottom of the elimination
// tree of small systems are a few columns wide: as separate factor, solve
// and update items each paid several queue round trips and chains of
// dependent metadata loads for a few hundred flops.  Products accumulate in
// FP64 from the stored (type T) values.  LDL: the tile is factored as
// L D L^T (static pivoting as in FACT), the rows below become A_off Y^T with
// Y = D^{-1} L^{-1}, and the update products take d_t (FP64, from the
// factored tile) between the two rows.
constexpr int kSLd = kSmallRows + 1;   // leading dimension of the LDS panel copy
static_assert(kSLd * kNB * sizeof(float) + (kSmallMap + 8 * kSmallMaxUpd) * sizeof(int) +
                      kSmallMaxUpd * sizeof(int64_t) <= (kPbLd * kNB + 32) * sizeof(float),
              "small-block tables exceed the LDS row buffer");
static_assert((kSLd * kNB * sizeof(float) + (kSmallMap + 8 * kSmallMaxUpd) * sizeof(int)) % 8 == 0,
              "misaligned small-block offset table");
static_assert(kSmallRows * kNB % kThreads == 0, "rows below per thread");

template <class T, bool LDL = false>
__device__ __noinline__ void task_small(const SchedArgs& a, const int4 d0, const int4 d1, double* Lt, T* Dt, T* Pb)
{
    const DevPlan& pl = a.pl;
    const int k = d0.y;
    const int tfirst = d1.x, nupd = d1.y, mstart = d1.z, mlen = d1.w;
    const int f = pl.fcol[k];
    const int w = pl.lcol[k] - f + 1;
    const int ld = pl.stride[k];
    const int R = ld - w;   // rows below the diagonal block
    T* A = static_cast<T*>(a.panels) + pl.panel_off[k];
    T* D = static_cast<T*>(a.dinv) + pl.dinv_off[k];
    T* S = Pb;                                                // S[r + c*kSLd] for panel rows r >= w
    int* smap = reinterpret_cast<int*>(S + kSLd * kNB);       // row-map entries mstart ..
    int* dtab = smap + kSmallMap;                             // per tile: j, row0, mrows, col0, ncols, map base, ldj
    int64_t* dpo = reinterpret_cast<int64_t*>(dtab + 8 * kSmallMaxUpd);   // panel offset of the target
    double* bc = Lt + kNB * 33;
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
        const int r = idx & 31, c = idx >> 5;
        Lt[r + c * 33] = (r < w && c < w) ? (c <= r ? (double)A[r + (int64_t)c * ld] : 0.0) : (r == c ? 1.0 : 0.0);
    }
    for (int idx = tid; idx < R * w; idx += kThreads) {
        const int i = idx % R, c = idx / R;
        S[(w + i) + c * kSLd] = A[(w + i) + (int64_t)c * ld];
    }
    for (int idx = tid; idx < mlen; idx += kThreads) smap[idx] = a.rmap[mstart + idx];
    if (tid < nupd) {
        const int4* ft = a.ftab + 3 * (int64_t)(tfirst + tid);
        const int4 u0 = ft[0], u1 = ft[1], u2 = ft[2];
        int* e = dtab + 8 * tid;
        e[0] = u0.x;
        e[1] = u0.y;
        e[2] = u0.z;
        e[3] = u0.w;
        e[4] = u1.x;
        e[5] = u1.y - mstart;
        e[6] = u1.z;
        dpo[tid] = (int64_t)(uint32_t)u2.x | ((int64_t)u2.y << 32);
    }
    __syncthreads();
    if (wave == 0) {
        if (w <= 8)
            tile_chol_inv<T, 8, LDL>(Lt, bc, Dt, w, f, a.status);
        else if (w <= 16)
            tile_chol_inv<T, 16, LDL>(Lt, bc, Dt, w, f, a.status);
        else
            tile_chol_inv<T, 32, LDL>(Lt, bc, Dt, w, f, a.status);
    }
    __syncthreads();
    for (int idx = tid; idx < kNB * kNB; idx += kThreads) {
        const int r = idx & 31, c = idx >> 5;
        if (r < w && c <= r) {
            A[r + (int64_t)c * ld] = (T)Lt[r + c * 33];
            D[r + (int64_t)c * w] = Dt[r + c * 33];
        }
    }
    // rows below: P = A_off D^T, D lower triangular
    constexpr int kPer = kSmallRows * kNB / kThreads;
    double p[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = tid + q * kThreads;
        double acc = 0.0;
        if (idx < R * w) {
            const int i = idx % R, c = idx / R;
            for (int t = 0; t <= c; ++t) acc += (double)S[(w + i) + t * kSLd] * (double)Dt[c + t * 33];
        }
        p[q] = acc;
    }
    __syncthreads();   // every product has read its row of S
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = tid + q * kThreads;
        if (idx < R * w) {
            const int i = idx % R, c = idx / R;
            const T v = (T)p[q];
            S[(w + i) + c * kSLd] = v;
            A[(w + i) + (int64_t)c * ld] = v;
        }
    }
    __syncthreads();
    // update tiles: C_j[rmap(r), rmap(c)] -= P_r . P_c (L D L^T: P_r D P_c) on
    // the lower triangle of j
    double* dg = bc + 64;   // (L D L^T) the pivots d_t
    if (LDL && tid < w) dg[tid] = Lt[tid * 34];
    __syncthreads();
    for (int u = 0; u < nupd; ++u) {
        const int* e = dtab + 8 * u;
        const int row0 = e[1], mrows = e[2], col0 = e[3], ncols = e[4], mb = e[5], ldj = e[6];
        auto Cg = glob(static_cast<T*>(a.panels) + dpo[u]);
        for (int idx = tid; idx < mrows * ncols; idx += kThreads) {
            const int r = row0 + idx % mrows, c = col0 + idx / mrows;
            const int tr = smap[mb + r], tc = smap[mb + c];
            if (tr >= tc) {
                double acc = 0.0;
                if constexpr (LDL) {
                    for (int t = 0; t < w; ++t) acc += (double)S[r + t * kSLd] * dg[t] * (double)S[c + t * kSLd];
                } else {
                    for (int t = 0; t < w; ++t) acc += (double)S[r + t * kSLd] * (double)S[c + t * kSLd];
                }
                __hip_atomic_fetch_add(Cg + (int64_t)tc * ldj + tr, (T)(-acc), __ATOMIC_RELAXED, AGENT);
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();   // every atomic of the item has completed
    if (tid < nupd) finish_update(a, dtab[8 * tid]);
}

// ---------------------------------------------------------------- scheduler
// LDL: the L D L^T factor.  LU: the L U factor (two panel arrays; no fused
// small items).
template <class T, bool LDL = false, bool LU = false>
__global__ void __launch_bounds__(kThreads, 2) sched_kernel(SchedArgs a)
{
    __shared__ double Lt[kNB * 33 + 3 * kNB + 1];   // tile, bc, small-item pivots, pivot threshold
    __shared__ T Dt[kNB * 33];
    __shared__ __align__(16) T Pb[kPbLd * kNB + 32];   // + padding: tile row indices up to 255; small-block tables
    __shared__ int rpos[256], cpos[128];
    __shared__ int s_item;
    __shared__ int s_push[6];   // {hp first, hp count, hp base, normal first, normal count, normal base}
    __shared__ int s_rel;       // deterministic mode: source whose update pairs lose one dependency
    __shared__ int64_t s_t0, s_t1;
    const int tid = threadIdx.x;
    // Tickets of the two FIFO queues held by this worker and not yet served
    // (thread 0).  A ticket below the queue's total is always served: its item
    // is pushed eventually.  A high-priority ticket is taken only when the
    // next slot is already published, so that an idle worker picks up a
    // released critical item at once; a worker holding one serves whichever
    // of its two items is published first.
    // Items served by this worker are counted in a register and added to the
    // done count once, at exit.
    int my_slot = -1, hp_slot = -1, ndone = 0;
    if (tid == 0) {
        s_rel = -1;
        double thr = 0.0;   // (read after the first barrier of the loop)
        if ((LDL || LU) && a.pivot_eps > 0.0)
            thr = a.pivot_eps * __longlong_as_double(*reinterpret_cast<const long long*>(a.status + kStAmax));
        Lt[kNB * 33 + kThrSlot] = thr;
    }
    for (;;) {
        if (tid == 0) {
            int item = -1;
            s_t0 = wall_clock64();
            const int64_t t0 = s_t0;
            for (int spin = 0;; ++spin) {
                if ((spin & 15) == 0 && __hip_atomic_load(&a.status[kStAbort], __ATOMIC_RELAXED, AGENT) != 0) {
                    item = -1;
                    break;
                }
                if (hp_slot < 0) {
                    const int h = __hip_atomic_load(a.hp_head, __ATOMIC_RELAXED, AGENT);
                    if (h < a.hp_total && __hip_atomic_load(&a.hp_queue[h], __ATOMIC_RELAXED, AGENT) >= 0) {
                        const int t = __hip_atomic_fetch_add(a.hp_head, 1, __ATOMIC_RELAXED, AGENT);
                        hp_slot = t < a.hp_total ? t : -1;
                    }
                }
                if (hp_slot >= 0) {
                    item = __hip_atomic_load(&a.hp_queue[hp_slot], __ATOMIC_RELAXED, AGENT);
                    if (item >= 0) { hp_slot = -1; break; }
                }
                if (my_slot < 0) my_slot = __hip_atomic_fetch_add(a.qhead, 1, __ATOMIC_RELAXED, AGENT);
                if (my_slot < a.total_normal) {
                    item = __hip_atomic_load(&a.queue[my_slot], __ATOMIC_RELAXED, AGENT);
                    if (item >= 0) { my_slot = -1; break; }
                } else if (hp_slot < 0 && __hip_atomic_load(a.hp_head, __ATOMIC_RELAXED, AGENT) >= a.hp_total) {
                    item = -1;   // no ticket left to serve in either queue
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > a.timeout_ticks) {
                    __hip_atomic_store(&a.status[kStAbort], 1, __ATOMIC_RELAXED, AGENT);
                    item = -1;
                    break;
                }
            }
            if (item < 0) __hip_atomic_fetch_add(&a.status[kStDone], ndone, __ATOMIC_RELAXED, AGENT);
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
        const int kind = d0.x & 0xff;   // (bits 8..11 of an update: pieces merged - 1; bit 12: thin item)
        const bool thin = (d0.x & kThinItem) != 0;
        if (kind == kFact) {
            __builtin_amdgcn_s_setprio(3);
            if constexpr (LU) task_fact_lu<T>(a, d0.y, Lt, Dt, Pb);
            else task_fact<T, LDL>(a, d0.y, Lt, Dt, Pb);
            __builtin_amdgcn_s_setprio(0);
        } else if (kind == kTrsm) {
            __builtin_amdgcn_s_setprio(2);
            if constexpr (LU) {
                if (thin) {
                    task_trsm<T, 1>(a, d0.y, d0.z, d0.w, 0, a.uinv);
                    task_trsm<T, 1>(a, d0.y, d0.z, d0.w, a.upanel, 0);
                } else {
                    task_trsm<T>(a, d0.y, d0.z, d0.w, 0, a.uinv);
                    task_trsm<T>(a, d0.y, d0.z, d0.w, a.upanel, 0);
                }
            } else {
                if (d0.x & kSubstItem) {
                    if constexpr (!LDL) trsm_subst<T>(a, d0.y, d0.z, d0.w, Pb);
                } else if (thin) {
                    task_trsm<T, 1>(a, d0.y, d0.z, d0.w);
                } else {
                    task_trsm<T>(a, d0.y, d0.z, d0.w);
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else if (kind == kUpdate) {
            if (thin) task_update<T, LDL, LU, 1>(a, d0, d1, rpos, cpos);
            else task_update<T, LDL, LU>(a, d0, d1, rpos, cpos);
        } else if (kind == kInv) {
            if constexpr (!LDL && !LU) {
                __builtin_amdgcn_s_setprio(2);
                task_inv<T>(a, d0.y, Pb);
                __builtin_amdgcn_s_setprio(0);
            }
        } else if constexpr (!LU) {
            task_small<T, LDL>(a, d0, d1, Lt, Dt, Pb);
        }
        // every wave's stores and atomics have completed before the barrier
        // (FACT and TRSM items ran at raised wave priority: they are on the
        // elimination chain and share their CU with update tiles)
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid < 64 && (kind == kFact || kind == kTrsm || kind == kInv)) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (tid == 0) {
            int hf = 0, hc = 0, nf = 0, nc = 0;
            if (kind == kFact) {
                // the panel solves; a chain block (high priority) also its
                // INV item, in the normal queue
                if (a.hp_cblk[d0.y]) {
                    hf = a.trsm_first[d0.y];
                    hc = a.trsm_count[d0.y];
                    const int ii = a.inv_item ? a.inv_item[d0.y] : -1;
                    if (ii >= 0) { nf = ii; nc = 1; }
                } else {
                    nf = a.trsm_first[d0.y];
                    nc = a.trsm_count[d0.y];
                }
            } else if (kind == kTrsm) {
                if (__hip_atomic_fetch_add(&a.trsm_left[d0.y], -1, __ATOMIC_RELAXED, AGENT) == 1) {
                    if (a.npair > 0) {
                        s_rel = d0.y;   // its pairs, below
                    } else {
                        hf = a.upd_first[d0.y];
                        hc = a.upd_hp[d0.y];
                        nf = hf + hc;
                        nc = a.upd_count[d0.y] - hc;
                    }
                }
            } else if (kind == kUpdate) {
                if (__hip_atomic_fetch_add(&a.fact_dep[d0.z], -1, __ATOMIC_RELAXED, AGENT) == 1) {
                    if (a.hp_cblk[d0.z]) { hf = d0.z; hc = 1; }
                    else { nf = d0.z; nc = 1; }
                }
                if (a.npair > 0) {
                    // the pair's last item releases the next pair into the
                    // same target (which then cannot have released the target)
                    const int p = a.upair[item - a.ubase];
                    if (__hip_atomic_fetch_add(&a.pleft[p], -1, __ATOMIC_RELAXED, AGENT) == 1) {
                        const int4 q = a.pairs[p];
                        if (q.z >= 0 && __hip_atomic_fetch_add(&a.pdep[q.z], -1, __ATOMIC_RELAXED, AGENT) == 1) {
                            const int4 r = a.pairs[q.z];
                            if (r.w) { hf = r.x; hc = r.y; }
                            else { nf = r.x; nc = r.y; }
                        }
                    }
                }
            }
            s_push[0] = hf;
            s_push[1] = hc;
            s_push[2] = hc > 0 ? __hip_atomic_fetch_add(a.hp_tail, hc, __ATOMIC_RELAXED, AGENT) : 0;
            s_push[3] = nf;
            s_push[4] = nc;
            s_push[5] = nc > 0 ? __hip_atomic_fetch_add(a.qtail, nc, __ATOMIC_RELAXED, AGENT) : 0;
            ++ndone;
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
        if (s_rel >= 0) release_pairs(a, s_rel);   // deterministic mode
        __syncthreads();
        if (tid == 0) s_rel = -1;
    }
}

// ---------------------------------------------------------------- update microbenchmark
// The update tiles of one synthetic (source, target) pair, as a plain grid:
// block b runs tile b % ntiles ({row0, mrows, col0, ncols}) of source 0 into
// target 1 through the same task_update as the scheduler (row map base
// mbase).  Several calls of the grid, or one grid of several calls, measure
// the update kernel alone (the paper's update-kernel study).
template <class T, bool LDL>
__global__ void __launch_bounds__(kThreads, 2) update_bench_kernel(SchedArgs a, const int4* tiles, int ntiles, int mbase)
{
    __shared__ int rpos[256], cpos[128];
    const int4 t = tiles[blockIdx.x % ntiles];
    task_update<T, LDL, false>(a, int4{kUpdate, 0, 1, t.x}, int4{t.y, t.z, t.w, mbase}, rpos, cpos);
}

hipError_t launch_update_bench(const SchedArgs& a, bool f32, bool ldl, const int4* tiles, int ntiles, int mbase,
                               int copies, hipStream_t s)
{
    const int grid = ntiles * copies;
    if (f32 && ldl) update_bench_kernel<float, true><<<grid, kThreads, 0, s>>>(a, tiles, ntiles, mbase);
    else if (f32) update_bench_kernel<float, false><<<grid, kThreads, 0, s>>>(a, tiles, ntiles, mbase);
    else if (ldl) update_bench_kernel<double, true><<<grid, kThreads, 0, s>>>(a, tiles, ntiles, mbase);
    else update_bench_kernel<double, false><<<grid, kThreads, 0, s>>>(a, tiles, ntiles, mbase);
    return hipGetLastError();
}

// ---------------------------------------------------------------- set-up kernels
template <class T>
__global__ void fill_kernel(T* p, int64_t n, T v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_i32(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// panels[amap[p]] = values[p] (rounded to the panel type) for entries read
// by the factorization
template <class T>
__global__ void assemble_kernel(T* panels, const int64_t* amap, const double* values, int64_t nnz)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = amap[p];
        if (d >= 0) panels[d] = (T)values[p];
    }
}

// max |values[p]| over the entries the factorization reads (amap[p] >= 0),
// into two status words as the bits of a non-negative double (ordered like
// the doubles; a NaN value counts as larger than every number)
__global__ void absmax_kernel(const int64_t* amap, const double* values, int64_t nnz, int32_t* status)
{
    unsigned long long m = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        if (amap[p] >= 0) {
            const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(values[p]));
            m = b > m ? b : m;
        }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(reinterpret_cast<unsigned long long*>(status + kStAmax), m);
}

__global__ void zero_amax_kernel(int32_t* status)
{
    if (threadIdx.x < 2) status[kStAmax + threadIdx.x] = 0;
}

hipError_t launch_absmax(const int64_t* amap, const double* values, int64_t nnz, int32_t* status, hipStream_t s)
{
    zero_amax_kernel<<<1, 64, 0, s>>>(status);
    if (nnz > 0) {
        const int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 2048);
        absmax_kernel<<<blocks, 256, 0, s>>>(amap, values, nnz, status);
    }
    return hipGetLastError();
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
    for (int64_t i = t; i < a.npair; i += stride) {
        a.pdep[i] = a.pdep0[i];
        a.pleft[i] = a.pairs[i].y;
    }
    if (t == 0) {
        *a.qhead = 0;
        *a.qtail = nready_n;
        *a.hp_head = 0;
        *a.hp_tail = nready_hp;
        a.status[kStFail] = 0x7fffffff;
        a.status[kStAbort] = 0;
        a.status[kStDone] = 0;
        a.status[kStReplaced] = 0;
    }
}

// ---------------------------------------------------------------- host launchers
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    fill_kernel<double><<<blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    fill_kernel<float><<<blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    fill_i32<<<blocks, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_assemble(void* panels, bool f32, const int64_t* amap, const double* values, int64_t nnz,
                           hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
    if (f32) assemble_kernel<float><<<blocks, 256, 0, s>>>(static_cast<float*>(panels), amap, values, nnz);
    else assemble_kernel<double><<<blocks, 256, 0, s>>>(static_cast<double*>(panels), amap, values, nnz);
    return hipGetLastError();
}

// FP32 panels widened to FP64 (export of the refinement-mode factor)
__global__ void widen_kernel(double* dst, const float* src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

// dst[j] = panels[off[j]] widened to FP64 (the diagonal of every panel, one
// entry per column, for the log-determinant)
template <class T>
__global__ void gather_diag_kernel(double* dst, const T* panels, const int64_t* off, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)panels[off[i]];
}

hipError_t launch_gather_diag(double* dst, const void* panels, bool f32, const int64_t* off, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    if (f32) gather_diag_kernel<float><<<blocks, 256, 0, s>>>(dst, static_cast<const float*>(panels), off, n);
    else gather_diag_kernel<double><<<blocks, 256, 0, s>>>(dst, static_cast<const double*>(panels), off, n);
    return hipGetLastError();
}

hipError_t launch_widen(double* dst, const float* src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    widen_kernel<<<blocks, 256, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_sched_init(const SchedArgs& a, const int32_t* ready, int32_t nready, int32_t nready_hp,
                             const int32_t* fact_dep0, int32_t ncblk, hipStream_t s)
{
    const int64_t n = std::max<int64_t>(std::max<int64_t>(a.total_normal, a.hp_total), std::max(ncblk, a.npair));
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    sched_init<<<blocks, 256, 0, s>>>(a, ready, nready, nready_hp, fact_dep0, ncblk);
    return hipGetLastError();
}

int sched_blocks_per_cu(bool f32, bool ldlt, bool lu)
{
    int nb = 0;
    hipError_t e;
    if (lu)
        e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel<float, false, true>, kThreads, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel<double, false, true>, kThreads, 0);
    else if (f32 && ldlt)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel<float, true>, kThreads, 0);
    else if (f32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel<float>, kThreads, 0);
    else if (ldlt)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel<double, true>, kThreads, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sched_kernel<double>, kThreads, 0);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_sched(const SchedArgs& a, bool f32, bool lu, int grid, hipStream_t s)
{
    if (lu && f32) sched_kernel<float, false, true><<<grid, kThreads, 0, s>>>(a);
    else if (lu) sched_kernel<double, false, true><<<grid, kThreads, 0, s>>>(a);
    else if (f32 && a.ldlt) sched_kernel<float, true><<<grid, kThreads, 0, s>>>(a);
    else if (f32) sched_kernel<float><<<grid, kThreads, 0, s>>>(a);
    else if (a.ldlt) sched_kernel<double, true><<<grid, kThreads, 0, s>>>(a);
    else sched_kernel<double><<<grid, kThreads, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace spx
