// Multi-right-hand-side Jacobi-PCG: k independent CG recurrences that share
// every read of the operator (the three velocity components of a step and
// many wind scenarios solved at once).
//
// Vectors are n x k row-major (the k values of node i are contiguous).  A
// thread owns V consecutive columns of one row (V is the autotuned pack
// width) and, because the grid's thread count times V is a multiple of k,
// always the same V columns: its per-column partial sums need no atomics and
// are reduced deterministically (threads of a block in thread order, then
// blocks in block order by one small reduction kernel per step).  One
// iteration is five launches:
//   spmm      Q = mask_j(A P) per column, per-block partials of p_j^T q_j
//   reduce    gamma_j, alpha_j = rho_j / gamma_j (active columns)
//   update    x_j += alpha_j p_j, r_j -= alpha_j q_j, partials of r^T z, r^T r
//   reduce    rho_j', rr_j, beta_j, stop flags
//   pupdate   p_j = z_j + beta_j p_j (columns still active)
// Columns stop independently; a chunk of iterations is captured once into a
// HIP graph and replayed.
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "kernels.h"

namespace hns {

// Per-column CG state (device)
struct BCol {
    double rho, alpha, beta, gamma;
    double rr;        // recursive r^T r
    double ref;       // reference r^T r of the current recurrence segment
    double thr2;      // segment stops when rr <= thr2 * ref
    double bb;        // |b|^2 (projected for pure-Neumann columns)
    double tol2;      // tol^2
    double rr_true;   // last FP64 true residual r^T r
    double sumb;      // sum of the free entries of b
    double mean_b;    // mean removed from b (pure-Neumann columns)
    double mean_r;    // mean of the last FP64 residual (pure-Neumann projection)
    double wx;        // sum lumped_i x_i
    double nonfinite;
    int32_t stop;     // 0 active, 1 segment threshold reached, 2 breakdown, 3 b = 0, 4 done
    int32_t iter;     // iterations executed
    int32_t bit;      // Dirichlet bit (-1 none)
    int32_t singular; // pure-Neumann column
    int32_t mark;     // selects the column for the next one-off kernel
    int32_t fresh;    // next direction restarts from z (no beta)
};

namespace {

enum : int32_t {
    ACTIVE = 0, THRESH = 1, BREAK = 2, ZERO = 3, DONE = 4, FAILED = 5, EMPTY = 6, CAPPED = 7,
    BADRHS = 8
};

#define PACK_LOOP(t, np)                                                       \
    for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < (np); \
         t += (int64_t)gridDim.x * kBlock)

// The same walk by element e = t V and row i = e / K: the grid's thread count
// times V is a multiple of K (bgrid), so a thread keeps the columns of its
// first pack in every pass and its row advances by a constant (no 64-bit
// division per pack).
#define ROW_LOOP(e, i, n, K, V)                                                             \
    for (int64_t e = (blockIdx.x * (int64_t)kBlock + threadIdx.x) * (V), i = e / (K),       \
                 de_ = (int64_t)gridDim.x * kBlock * (V), di_ = de_ / (K);                  \
         e < (int64_t)(n) * (K); e += de_, i += di_)

// First column of the thread's packs in ROW_LOOP.
template <int V>
__device__ __forceinline__ int thread_col0(int K)
{
    return (int)((((int64_t)blockIdx.x * kBlock + threadIdx.x) * V) % K);
}

// True in every thread of the block when at least one of the K columns is
// running (stop == ACTIVE; mode 0) or is marked for a direction update
// (mode 1).  The per-iteration kernels return at once otherwise, so the
// iterations of a chunk that follow the last column's exit cost a launch
// each instead of a pass over the n x K block.
__device__ __forceinline__ bool any_column(const BCol *__restrict__ cols, int K, int mode);

__device__ __forceinline__ bool masked(const uint8_t *bc, int bit, int64_t i)
{
    return bc != nullptr && bit >= 0 && ((bc[i] >> bit) & 1u);
}

// Reduce the per-thread values acc[NV][V] of a block to per-column partials
// part[k][b * K + c] for the K columns; thread t owns columns j0(t) .. j0(t)+V-1
// with j0(t) = ((b * kBlock + t) * V) mod K.
template <int NV, int V>
__device__ void block_column_partials(double (&acc)[NV][V], int K, double *part)
{
    __shared__ double s[NV][V][kBlock];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int v = 0; v < V; ++v) s[k][v][threadIdx.x] = acc[k][v];
    __syncthreads();
    const int P = K / V;  // column groups
    const int64_t b = blockIdx.x;
    for (int c = threadIdx.x; c < K; c += kBlock) {
        const int g = c / V, v = c % V;
        int t0 = (int)(((int64_t)g - b * kBlock) % P);
        if (t0 < 0) t0 += P;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double sum = 0.0;
            for (int t = t0; t < kBlock; t += P) sum += s[k][v][t];
            part[(int64_t)k * gridDim.x * K + b * K + c] = sum;
        }
    }
}

// Sum of one column's partials over the G blocks (block order); result valid
// in thread 0.
__device__ double column_total(const double *part, int G, int K, int c)
{
    __shared__ double lds[kBlock / 64];
    double t = 0.0;
    for (int b = threadIdx.x; b < G; b += kBlock) t += part[(int64_t)b * K + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) s += lds[w];
    __syncthreads();
    return s;
}

template <typename T, int W>
struct alignas(sizeof(T) * W) BPack {
    T v[W];
};

template <int W, typename T>
__device__ __forceinline__ BPack<T, W> bld(const T *p, int64_t e)
{
    return *reinterpret_cast<const BPack<T, W> *>(p + e);
}

template <int W, typename T>
__device__ __forceinline__ void bst(T *p, int64_t e, const BPack<T, W> &v)
{
    *reinterpret_cast<BPack<T, W> *>(p + e) = v;
}

struct BOffsets {
    int32_t o[kMaxDiag];
};

struct BWideOffsets {
    int32_t o[kMaxDiagWide];
};

// ---------------------------------------------------------------------------
// SpMM: Q = mask_j(A P), optional per-column partials of p_j^T q_j
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool any_column(const BCol *__restrict__ cols, int K, int mode)
{
    int mine = 0;
    for (int c = threadIdx.x; c < K; c += blockDim.x)
        mine |= mode == 0 ? (cols[c].stop == ACTIVE) : (cols[c].mark != 0);
    return __syncthreads_or(mine) != 0;
}

// The Dirichlet bits of a thread's V columns.  A thread owns the same V
// columns in every pass of PACK_LOOP (the grid's thread count times V is a
// multiple of K), so the products read them once, before the loop, and only
// the row's byte of bc inside it, issued with the other loads: testing
// cols[j].bit and then bc[i] per column after the products serialised two
// memory round trips per column and pack.
template <int V>
struct ColBits {
    int bit[V];
};

template <int V>
__device__ __forceinline__ ColBits<V> thread_col_bits(const BCol *__restrict__ cols, int K)
{
    ColBits<V> cb;
    const int j0 = thread_col0<V>(K);
#pragma unroll
    for (int v = 0; v < V; ++v) cb.bit[v] = cols[j0 + v].bit;
    return cb;
}

__device__ __forceinline__ bool masked_byte(uint8_t b, int bit)
{
    return bit >= 0 && ((b >> bit) & 1u);
}

template <typename TV, typename TX, int V, bool DOT, int M>
__global__ __launch_bounds__(kBlock) void k_bspmm_sdia(int64_t n, int K, BOffsets offs,
                                                       const TV *__restrict__ dia,
                                                       const TX *__restrict__ P,
                                                       TX *__restrict__ Q,
                                                       const uint8_t *__restrict__ bc,
                                                       const BCol *__restrict__ cols,
                                                       double *__restrict__ part)
{
    if constexpr (DOT) {
        if (!any_column(cols, K, 0)) return;
    }
    double acc[1][V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[0][v] = 0.0;
    const ColBits<V> cbits = thread_col_bits<V>(cols, K);
    const int j0 = thread_col0<V>(K);
    // the iteration's product: a thread whose columns have all stopped
    // skips its rows (their q is not read again)
    bool mine = !DOT;
    if constexpr (DOT) {
#pragma unroll
        for (int v = 0; v < V; ++v) mine |= cols[j0 + v].stop == ACTIVE;
    }
    if (mine) ROW_LOOP(e, i, n, K, V)
    {
        const uint8_t bci = bc ? bc[i] : (uint8_t)0;
        const auto pi = bld<V>(P, e);
        const TX d = (TX)dia[i];
        TX s[V];
#pragma unroll
        for (int v = 0; v < V; ++v) s[v] = d * pi.v[v];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int64_t o = offs.o[k];
            const TV *u = dia + (int64_t)(k + 1) * n;
            const bool hu = i + o < n, hl = i >= o;
            const int64_t iu = hu ? i + o : i, il = hl ? i - o : i;
            const TX cu = hu ? (TX)u[i] : (TX)0;
            const TX cl = hl ? (TX)u[il] : (TX)0;
            const auto pu = bld<V>(P, iu * K + j0);
            const auto pl = bld<V>(P, il * K + j0);
#pragma unroll
            for (int v = 0; v < V; ++v) s[v] += cu * pu.v[v] + cl * pl.v[v];
        }
        BPack<TX, V> out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            out.v[v] = masked_byte(bci, cbits.bit[v]) ? (TX)0 : s[v];
            if constexpr (DOT) acc[0][v] += (double)pi.v[v] * (double)out.v[v];
        }
        bst<V>(Q, e, out);
    }
    if constexpr (DOT) block_column_partials<1, V>(acc, K, part);
}

// ---------------------------------------------------------------------------
// LDS-tiled product for the narrow symmetric-diagonal format.  A block owns
// tiles of T consecutive rows and one group of C columns; the rows its tile
// needs (row i reads rows i and i +- o_k) form a few clusters of nearby
// offsets, which the block stages into LDS with coalesced 16-byte loads
// (zeros outside [0, n)), so each value of P comes from global memory about
// (staged rows / T) times instead of 2 M + 1 times, and every term of a row
// then reads LDS.  Terms of a row in the order of k_bspmm_sdia: main, then
// (upper + lower) for each offset.  Each thread owns NP packs of 16 bytes of
// one row (PK columns each), the same columns in every tile; per-column
// partials of p^T q are reduced over the block in row order and stored at
// part[slot * K + column] (slot = the block's index within its column group).
// ---------------------------------------------------------------------------
// Workgroup b runs on XCD b mod 8 (round-robin dispatch): renumbered so that
// each XCD takes a contiguous eighth of the tiles (its L2 then holds the rows
// its neighbouring tiles stage again).
__device__ __forceinline__ int tile_block(int b, int G)
{
    return (G >= 8 && (G & 7) == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

struct TileMap {
    int32_t nclus;                        // clusters of staged rows
    int32_t rows;                         // staged rows in all
    int32_t lo[2 * kMaxDiag + 1];         // cluster c: rows i0 + lo[c] .. (cnt[c] of them)
    int32_t cnt[2 * kMaxDiag + 1];
    int32_t base[2 * kMaxDiag + 1];       // LDS row of the cluster's first staged row
    int32_t lrow[2 * kMaxDiag + 1];       // term t: LDS row of tile row 0 (t = 0 main,
                                          // 2k + 1 at + off[k], 2k + 2 at - off[k])
    int32_t off[kMaxDiag];
};

template <typename TV, typename TX, int C, int NP, int M>
__global__ __launch_bounds__(kBlock) void k_bspmm_tile(int64_t n, int K, TileMap tm,
                                                       const TV *__restrict__ dia,
                                                       const TX *__restrict__ P,
                                                       TX *__restrict__ Q,
                                                       const uint8_t *__restrict__ bc,
                                                       const BCol *__restrict__ cols,
                                                       double *__restrict__ part, int64_t ntiles,
                                                       int64_t tpb, int ngroups)
{
    constexpr int PK = 16 / sizeof(TX);      // columns per 16-byte pack
    constexpr int W = PK * NP;               // columns per thread
    constexpr int TPR = C / W;               // threads per tile row
    constexpr int T = kBlock / TPR;          // rows per tile
    constexpr int PPR = C / PK;              // packs per staged row
    constexpr int U = 8;                     // staging loads in flight per thread
    static_assert(C % W == 0 && kBlock % TPR == 0, "tile shape");
    extern __shared__ __align__(16) unsigned char smem[];
    TX *lds = reinterpret_cast<TX *>(smem);
    if (!any_column(cols, K, 0)) return;
    const int lb = tile_block(blockIdx.x, gridDim.x);
    const int group = lb % ngroups;
    const int64_t slot = lb / ngroups;
    const int c0 = group * C;
    const int tr = threadIdx.x / TPR;
    const int tc = (threadIdx.x % TPR) * W;
    int cbit[W];
#pragma unroll
    for (int v = 0; v < W; ++v) cbit[v] = cols[c0 + tc + v].bit;
    double acc[W];
#pragma unroll
    for (int v = 0; v < W; ++v) acc[v] = 0.0;
    const int64_t t0 = slot * tpb;
    const int64_t t1 = t0 + tpb < ntiles ? t0 + tpb : ntiles;
    const int total = tm.rows * PPR;
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t i0 = tile * T;
        // stage the clusters' rows: U loads in flight, then their stores
        for (int b0 = threadIdx.x; b0 < total; b0 += U * kBlock) {
            BPack<TX, PK> v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = b0 + u * kBlock;
#pragma unroll
                for (int e = 0; e < PK; ++e) v[u].v[e] = (TX)0;
                if (idx < total) {
                    const int lr = idx / PPR, pk = idx - lr * PPR;
                    int c = 0;
                    while (c + 1 < tm.nclus && lr >= tm.base[c + 1]) ++c;
                    const int64_t g = i0 + tm.lo[c] + (lr - tm.base[c]);
                    if (g >= 0 && g < n) v[u] = bld<PK>(P, g * K + c0 + pk * PK);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int idx = b0 + u * kBlock;
                if (idx < total) bst<PK>(lds, (int64_t)idx * PK, v[u]);
            }
        }
        __syncthreads();
        const int64_t i = i0 + tr;
        if (i < n) {
            // the row's operator entries first (all loads in flight)
            const uint8_t bci = bc ? bc[i] : (uint8_t)0;
            const TX d = (TX)dia[i];
            TX cu[M], cl[M];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t o = tm.off[k];
                const TV *u = dia + (int64_t)(k + 1) * n;
                cu[k] = (i + o < n) ? (TX)u[i] : (TX)0;
                cl[k] = (i >= o) ? (TX)u[i >= o ? i - o : 0] : (TX)0;
            }
            TX p0[W], s[W];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const auto pv = bld<PK>(lds, (int64_t)(tm.lrow[0] + tr) * C + tc + q * PK);
#pragma unroll
                for (int e = 0; e < PK; ++e) p0[q * PK + e] = pv.v[e];
            }
#pragma unroll
            for (int v = 0; v < W; ++v) s[v] = d * p0[v];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t ru = (int64_t)(tm.lrow[2 * k + 1] + tr) * C + tc;
                const int64_t rl = (int64_t)(tm.lrow[2 * k + 2] + tr) * C + tc;
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const auto pu = bld<PK>(lds, ru + q * PK);
                    const auto pl = bld<PK>(lds, rl + q * PK);
#pragma unroll
                    for (int e = 0; e < PK; ++e)
                        s[q * PK + e] += cu[k] * pu.v[e] + cl[k] * pl.v[e];
                }
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                BPack<TX, PK> out;
#pragma unroll
                for (int e = 0; e < PK; ++e) {
                    const int v = q * PK + e;
                    out.v[e] = masked_byte(bci, cbit[v]) ? (TX)0 : s[v];
                    acc[v] += (double)p0[v] * (double)out.v[e];
                }
                bst<PK>(Q, i * K + c0 + tc + q * PK, out);
            }
        }
        __syncthreads();
    }
    // per-column partials over the block's T rows, in row order
    double *red = reinterpret_cast<double *>(smem);   // T x C doubles (fits the staging area)
#pragma unroll
    for (int v = 0; v < W; ++v) red[tr * C + tc + v] = acc[v];
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += kBlock) {
        double sum = 0.0;
        for (int r = 0; r < T; ++r) sum += red[r * C + c];
        part[slot * K + c0 + c] = sum;
    }
}

// The same product for the wide symmetric-diagonal format: the offsets are a
// run-time count (up to kMaxDiagWide), visited in ascending order as above.
template <typename TV, typename TX, int V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_bspmm_sdia_wide(int64_t n, int K, int M,
                                                            BWideOffsets offs,
                                                            const TV *__restrict__ dia,
                                                            const TX *__restrict__ P,
                                                            TX *__restrict__ Q,
                                                            const uint8_t *__restrict__ bc,
                                                            const BCol *__restrict__ cols,
                                                            double *__restrict__ part)
{
    if constexpr (DOT) {
        if (!any_column(cols, K, 0)) return;
    }
    double acc[1][V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[0][v] = 0.0;
    const int64_t np = n * K / V;
    const ColBits<V> cbits = thread_col_bits<V>(cols, K);
    PACK_LOOP(t, np)
    {
        const int64_t e = t * V;
        const int64_t i = e / K;
        const uint8_t bci = bc ? bc[i] : (uint8_t)0;
        const auto pi = bld<V>(P, e);
        const TX d = (TX)dia[i];
        TX s[V];
#pragma unroll
        for (int v = 0; v < V; ++v) s[v] = d * pi.v[v];
#pragma unroll 4
        for (int k = 0; k < M; ++k) {
            const int64_t o = offs.o[k];
            const TV *u = dia + (int64_t)(k + 1) * n;
            const bool hu = i + o < n, hl = i >= o;
            const int64_t iu = hu ? i + o : i, il = hl ? i - o : i;
            const TX cu = hu ? (TX)u[i] : (TX)0;
            const TX cl = hl ? (TX)u[il] : (TX)0;
            const auto pu = bld<V>(P, iu * K + (e - i * K));
            const auto pl = bld<V>(P, il * K + (e - i * K));
#pragma unroll
            for (int v = 0; v < V; ++v) s[v] += cu * pu.v[v] + cl * pl.v[v];
        }
        BPack<TX, V> out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            out.v[v] = masked_byte(bci, cbits.bit[v]) ? (TX)0 : s[v];
            if constexpr (DOT) acc[0][v] += (double)pi.v[v] * (double)out.v[v];
        }
        bst<V>(Q, e, out);
    }
    if constexpr (DOT) block_column_partials<1, V>(acc, K, part);
}

template <typename TV, typename TX, int V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_bspmm_csr(int64_t n, int K,
                                                      const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ col,
                                                      const TV *__restrict__ val,
                                                      const TX *__restrict__ P,
                                                      TX *__restrict__ Q,
                                                      const uint8_t *__restrict__ bc,
                                                      const BCol *__restrict__ cols,
                                                      double *__restrict__ part)
{
    if constexpr (DOT) {
        if (!any_column(cols, K, 0)) return;
    }
    double acc[1][V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[0][v] = 0.0;
    const int64_t np = n * K / V;
    const ColBits<V> cbits = thread_col_bits<V>(cols, K);
    PACK_LOOP(t, np)
    {
        const int64_t e = t * V;
        const int64_t i = e / K;
        const uint8_t bci = bc ? bc[i] : (uint8_t)0;
        const int j0 = (int)(e - i * K);
        TX s[V];
#pragma unroll
        for (int v = 0; v < V; ++v) s[v] = 0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const TX a = (TX)val[k];
            const auto pc = bld<V>(P, (int64_t)col[k] * K + j0);
#pragma unroll
            for (int v = 0; v < V; ++v) s[v] += a * pc.v[v];
        }
        const auto pi = bld<V>(P, e);
        BPack<TX, V> out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            out.v[v] = masked_byte(bci, cbits.bit[v]) ? (TX)0 : s[v];
            if constexpr (DOT) acc[0][v] += (double)pi.v[v] * (double)out.v[v];
        }
        bst<V>(Q, e, out);
    }
    if constexpr (DOT) block_column_partials<1, V>(acc, K, part);
}

template <typename TV, typename TX, int V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_bspmm_sell(int64_t n, int K,
                                                       const int32_t *__restrict__ sptr,
                                                       const int32_t *__restrict__ col,
                                                       const TV *__restrict__ val,
                                                       const TX *__restrict__ P,
                                                       TX *__restrict__ Q,
                                                       const uint8_t *__restrict__ bc,
                                                       const BCol *__restrict__ cols,
                                                       double *__restrict__ part)
{
    if constexpr (DOT) {
        if (!any_column(cols, K, 0)) return;
    }
    double acc[1][V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[0][v] = 0.0;
    const int64_t np = n * K / V;
    const ColBits<V> cbits = thread_col_bits<V>(cols, K);
    PACK_LOOP(t, np)
    {
        const int64_t e = t * V;
        const int64_t i = e / K;
        const uint8_t bci = bc ? bc[i] : (uint8_t)0;
        const int j0 = (int)(e - i * K);
        const int64_t sl = i >> 6;
        const int lane = (int)(i & 63);
        const int32_t beg = sptr[sl];
        const int32_t w = (sptr[sl + 1] - beg) >> 6;
        TX s[V];
#pragma unroll
        for (int v = 0; v < V; ++v) s[v] = 0;
        for (int jj = 0; jj < w; ++jj) {
            const int32_t k = beg + jj * 64 + lane;
            const TX a = (TX)val[k];
            const auto pc = bld<V>(P, (int64_t)col[k] * K + j0);
#pragma unroll
            for (int v = 0; v < V; ++v) s[v] += a * pc.v[v];
        }
        const auto pi = bld<V>(P, e);
        BPack<TX, V> out;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            out.v[v] = masked_byte(bci, cbits.bit[v]) ? (TX)0 : s[v];
            if constexpr (DOT) acc[0][v] += (double)pi.v[v] * (double)out.v[v];
        }
        bst<V>(Q, e, out);
    }
    if constexpr (DOT) block_column_partials<1, V>(acc, K, part);
}

// ---------------------------------------------------------------------------
// Per-column reductions (one block per column)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bred_gamma(int K, const double *__restrict__ part,
                                                       int G, BCol *__restrict__ cols)
{
    const int c = blockIdx.x;
    const double g = column_total(part, G, K, c);
    if (threadIdx.x == 0) {
        BCol &s = cols[c];
        if (s.stop != ACTIVE) return;
        s.gamma = g;
        if (!(g > 0.0) || !isfinite(g)) {
            s.stop = BREAK;
            s.alpha = 0.0;
        } else {
            s.alpha = s.rho / g;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_bred_rho(int K, const double *__restrict__ part,
                                                     int G, BCol *__restrict__ cols)
{
    const int c = blockIdx.x;
    const double rz = column_total(part, G, K, c);
    const double rr = column_total(part + (int64_t)G * K, G, K, c);
    if (threadIdx.x == 0) {
        BCol &s = cols[c];
        s.mark = 0;
        s.fresh = 0;  // only the direction that opens a segment ignores beta
        if (s.stop != ACTIVE) return;
        s.iter += 1;
        s.rr = rr;
        if (!isfinite(rz) || !isfinite(rr)) {
            s.stop = BREAK;
            return;
        }
        if (rr <= s.thr2 * s.ref) {
            // segment ends: keep rho of this iteration's start, the next
            // segment's direction is z_new + (rho_new / rho) p
            s.stop = THRESH;
        } else {
            s.beta = rz / s.rho;
            s.rho = rz;
            s.mark = 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Vector updates
// ---------------------------------------------------------------------------
template <typename TX, typename TD, int V>
__global__ __launch_bounds__(kBlock) void k_bupdate(int64_t n, int K, TX *__restrict__ X,
                                                    TX *__restrict__ R,
                                                    const TX *__restrict__ P,
                                                    const TX *__restrict__ Q,
                                                    const TD *__restrict__ dinv,
                                                    const BCol *__restrict__ cols,
                                                    double *__restrict__ part)
{
    if (!any_column(cols, K, 0)) return;
    double acc[2][V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[0][v] = acc[1][v] = 0.0;
    // the thread's columns are the same in every pass: their state once
    const int j0 = thread_col0<V>(K);
    bool act[V];
    TX a[V];
    bool any = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const BCol &s = cols[j0 + v];
        act[v] = s.stop == ACTIVE;
        a[v] = (TX)s.alpha;
        any |= act[v];
    }
    if (any) ROW_LOOP(e, i, n, K, V)
    {
        auto xv = bld<V>(X, e);
        auto rv = bld<V>(R, e);
        const auto pv = bld<V>(P, e);
        const auto qv = bld<V>(Q, e);
        const TX d = (TX)dinv[i];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (!act[v]) continue;
            xv.v[v] = xv.v[v] + a[v] * pv.v[v];
            rv.v[v] = rv.v[v] - a[v] * qv.v[v];
            const TX z = d * rv.v[v];
            acc[0][v] += (double)rv.v[v] * (double)z;
            acc[1][v] += (double)rv.v[v] * (double)rv.v[v];
        }
        bst<V>(X, e, xv);
        bst<V>(R, e, rv);
    }
    block_column_partials<2, V>(acc, K, part);
}

// p = z + beta p for marked columns (fresh columns: p = z)
template <typename TX, typename TD, int V>
__global__ __launch_bounds__(kBlock) void k_bpupdate(int64_t n, int K, TX *__restrict__ P,
                                                     const TX *__restrict__ R,
                                                     const TD *__restrict__ dinv,
                                                     const BCol *__restrict__ cols)
{
    if (!any_column(cols, K, 1)) return;
    const int j0 = thread_col0<V>(K);
    bool mark[V], fresh[V];
    TX beta[V];
    bool any = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const BCol &s = cols[j0 + v];
        mark[v] = s.mark != 0;
        fresh[v] = s.fresh != 0;
        beta[v] = (TX)s.beta;
        any |= mark[v];
    }
    if (any) ROW_LOOP(e, i, n, K, V)
    {
        auto pv = bld<V>(P, e);
        const auto rv = bld<V>(R, e);
        const TX d = (TX)dinv[i];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (!mark[v]) continue;
            pv.v[v] = fresh[v] ? d * rv.v[v] : d * rv.v[v] + beta[v] * pv.v[v];
        }
        bst<V>(P, e, pv);
    }
}

// ---------------------------------------------------------------------------
// One-off kernels (elementwise over the n x K block, one element per thread)
// ---------------------------------------------------------------------------
#define ELEM_LOOP(e, ne)                                                       \
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < (ne); \
         e += (int64_t)gridDim.x * kBlock)

// sum, sum of squares and non-finite count of the free entries of b
__global__ __launch_bounds__(kBlock) void k_bbstats(int64_t n, int K, const double *__restrict__ B,
                                                    const uint8_t *__restrict__ bc,
                                                    const BCol *__restrict__ cols,
                                                    double *__restrict__ part)
{
    double acc[3][1] = {{0.0}, {0.0}, {0.0}};
    ELEM_LOOP(e, n * K)
    {
        const int64_t i = e / K;
        const int j = (int)(e - i * K);
        double b = masked(bc, cols[j].bit, i) ? 0.0 : B[e];
        if (!isfinite(b)) {
            acc[2][0] += 1.0;
            b = 0.0;
        }
        acc[0][0] += b;
        acc[1][0] += b * b;
    }
    block_column_partials<3, 1>(acc, K, part);
}

__global__ __launch_bounds__(kBlock) void k_bred_bstats(int64_t n, int K,
                                                        const double *__restrict__ part, int G,
                                                        BCol *__restrict__ cols)
{
    const int c = blockIdx.x;
    const double s = column_total(part, G, K, c);
    const double s2 = column_total(part + (int64_t)G * K, G, K, c);
    const double bad = column_total(part + 2 * (int64_t)G * K, G, K, c);
    if (threadIdx.x == 0) {
        BCol &b = cols[c];
        b.sumb = s;
        b.nonfinite = bad;
        b.mean_b = b.singular ? s / (double)n : 0.0;
        (void)s2;
    }
}

// R64 = mask(b - mean_b - Q64) for marked columns; partials of sum r, sum
// (b - mean_b)^2, sum r^2
__global__ __launch_bounds__(kBlock) void k_bresidual(int64_t n, int K,
                                                      const double *__restrict__ B,
                                                      const double *__restrict__ Q,
                                                      double *__restrict__ R,
                                                      const uint8_t *__restrict__ bc,
                                                      const BCol *__restrict__ cols,
                                                      double *__restrict__ part)
{
    double acc[3][1] = {{0.0}, {0.0}, {0.0}};
    ELEM_LOOP(e, n * K)
    {
        const int64_t i = e / K;
        const int j = (int)(e - i * K);
        const BCol &s = cols[j];
        if (!s.mark) continue;
        double b = B[e] - s.mean_b;
        double r = b - Q[e];
        if (masked(bc, s.bit, i)) b = r = 0.0;
        R[e] = r;
        acc[0][0] += r;
        acc[1][0] += b * b;
        acc[2][0] += r * r;
    }
    block_column_partials<3, 1>(acc, K, part);
}

// true residual statistics; decide per marked column: done, or continue
__global__ __launch_bounds__(kBlock) void k_bred_residual(int64_t n, int K,
                                                          const double *__restrict__ part, int G,
                                                          BCol *__restrict__ cols, double drop2,
                                                          int first)
{
    const int c = blockIdx.x;
    const double sr = column_total(part, G, K, c);
    const double sbb = column_total(part + (int64_t)G * K, G, K, c);
    const double srr = column_total(part + 2 * (int64_t)G * K, G, K, c);
    if (threadIdx.x == 0) {
        BCol &s = cols[c];
        if (!s.mark) return;
        const double mean = s.singular ? sr / (double)n : 0.0;
        const double rr = fmax(srr - (double)n * mean * mean, 0.0);
        s.mean_r = mean;
        s.rr_true = rr;
        if (first) {
            s.bb = sbb;
            if (!(sbb > 0.0)) {
                s.stop = ZERO;
                s.mark = 0;
                return;
            }
        }
        if (rr <= s.tol2 * s.bb) {
            s.stop = DONE;
            s.mark = 0;
            return;
        }
        if (s.stop == FAILED) {
            s.mark = 0;
            return;
        }
        // next segment: stop once the recursive residual fell by drop (or at tol)
        s.ref = rr;
        s.thr2 = fmax(drop2, s.tol2 * s.bb / rr);
        s.fresh = (first || s.stop == BREAK || drop2 == 0.0) ? 1 : 0;
    }
}

// Working residual of marked columns from the FP64 one (projected for
// pure-Neumann columns): r = (TX)(r64 - mean_r); partials of r^T z, r^T r.
template <typename TX, typename TD>
__global__ __launch_bounds__(kBlock) void k_bfrom64(int64_t n, int K,
                                                    const double *__restrict__ R64,
                                                    TX *__restrict__ R,
                                                    const TD *__restrict__ dinv,
                                                    const BCol *__restrict__ cols,
                                                    double *__restrict__ part)
{
    double acc[2][1] = {{0.0}, {0.0}};
    ELEM_LOOP(e, n * K)
    {
        const int64_t i = e / K;
        const int j = (int)(e - i * K);
        const BCol &s = cols[j];
        if (!s.mark) continue;
        const TX r = (TX)(R64[e] - s.mean_r);
        R[e] = r;
        const TX z = (TX)dinv[i] * r;
        acc[0][0] += (double)r * (double)z;
        acc[1][0] += (double)r * (double)r;
    }
    block_column_partials<2, 1>(acc, K, part);
}

// rho of the new segment; beta against the old rho unless fresh
__global__ __launch_bounds__(kBlock) void k_bred_restart(int K, const double *__restrict__ part,
                                                         int G, BCol *__restrict__ cols)
{
    const int c = blockIdx.x;
    const double rz = column_total(part, G, K, c);
    const double rr = column_total(part + (int64_t)G * K, G, K, c);
    if (threadIdx.x == 0) {
        BCol &s = cols[c];
        if (!s.mark) return;
        s.beta = s.fresh ? 0.0 : rz / s.rho;
        s.rho = rz;
        s.rr = rr;
        s.stop = (isfinite(rz) && rz > 0.0) ? ACTIVE : BREAK;
        if (s.stop != ACTIVE) s.mark = 0;
    }
}

// Mark exactly the columns listed in slots[0..count)
__global__ void k_bmark_list(int K, BCol *__restrict__ cols, const int32_t *__restrict__ slots,
                             int count)
{
    for (int c = threadIdx.x; c < K; c += blockDim.x) cols[c].mark = 0;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < count; ++q) cols[slots[q]].mark = 1;
}

// Column `slot` of B = b (contiguous n-vector); same column of X (and X32) = 0
__global__ __launch_bounds__(kBlock) void k_bset_column(int64_t n, int K, double *__restrict__ B,
                                                        double *__restrict__ X,
                                                        float *__restrict__ X32,
                                                        const double *__restrict__ b, int slot)
{
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        B[i * K + slot] = b[i];
        X[i * K + slot] = 0.0;
        if (X32) X32[i * K + slot] = 0.0f;
    }
}

// x = column `slot` of X, shifted to zero mass-weighted mean when `shift`
// (pure-Neumann columns; wx / wsum from cols[slot]), zeroed for b = 0
__global__ __launch_bounds__(kBlock) void k_bget_column(int64_t n, int K,
                                                        const double *__restrict__ X,
                                                        double *__restrict__ x, int slot,
                                                        const BCol *__restrict__ cols,
                                                        double wsum, int shift)
{
    const BCol &s = cols[slot];
    const double c = shift ? s.wx / wsum : 0.0;
    const bool zero = s.stop == ZERO;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        x[i] = zero ? 0.0 : X[i * K + slot] - c;
}

// x64 += x32, x32 = 0 for marked columns
__global__ __launch_bounds__(kBlock) void k_baccumulate(int64_t n, int K, double *__restrict__ X,
                                                        float *__restrict__ X32,
                                                        const BCol *__restrict__ cols)
{
    ELEM_LOOP(e, n * K)
    {
        const int j = (int)(e % K);
        if (!cols[j].mark) continue;
        X[e] += (double)X32[e];
        X32[e] = 0.0f;
    }
}

// Mark columns: mode 0 those with stop in {THRESH, BREAK}; mode 1 all
// columns; mode 2 the still active ones
__global__ void k_bmark(int K, BCol *__restrict__ cols, int mode)
{
    for (int c = threadIdx.x; c < K; c += blockDim.x) {
        BCol &s = cols[c];
        s.mark = mode == 1   ? 1
                 : mode == 2 ? (s.stop == ACTIVE ? 1 : 0)
                             : ((s.stop == THRESH || s.stop == BREAK) ? 1 : 0);
    }
}

// x = 0 on Dirichlet nodes (all entries of zero columns); x32 = 0
__global__ __launch_bounds__(kBlock) void k_bprepare(int64_t n, int K, double *__restrict__ X,
                                                     float *__restrict__ X32,
                                                     const uint8_t *__restrict__ bc,
                                                     const BCol *__restrict__ cols)
{
    ELEM_LOOP(e, n * K)
    {
        const int64_t i = e / K;
        const BCol &s = cols[e - i * K];
        if (s.stop == ZERO || masked(bc, s.bit, i)) X[e] = 0.0;
        if (X32) X32[e] = 0.0f;
    }
}

__global__ __launch_bounds__(kBlock) void k_bwdot(int64_t n, int K, const double *__restrict__ X,
                                                  const double *__restrict__ w,
                                                  double *__restrict__ part)
{
    double acc[1][1] = {{0.0}};
    ELEM_LOOP(e, n * K) acc[0][0] += w[e / K] * X[e];
    block_column_partials<1, 1>(acc, K, part);
}

__global__ __launch_bounds__(kBlock) void k_bred_wdot(int K, const double *__restrict__ part,
                                                      int G, BCol *__restrict__ cols)
{
    const int c = blockIdx.x;
    const double s = column_total(part, G, K, c);
    if (threadIdx.x == 0) cols[c].wx = s;
}

__global__ __launch_bounds__(kBlock) void k_bshift(int64_t n, int K, double *__restrict__ X,
                                                   const BCol *__restrict__ cols, double wsum)
{
    ELEM_LOOP(e, n * K)
    {
        const BCol &s = cols[e % K];
        if (s.singular && (s.stop == DONE || s.stop == ACTIVE || s.stop == THRESH))
            X[e] -= s.wx / wsum;
    }
}

hns_status bcheck(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", what, hipGetErrorString(e));
        return HNS_ERR_HIP;
    }
    return HNS_OK;
}

// grid (multiple of K / gcd) so that every thread keeps the same columns
int bgrid(int64_t packs, int K, int V)
{
    const int64_t tpg = (int64_t)kBlock * V;              // elements per block per sweep
    const int64_t g0 = K / std::gcd((int64_t)K, tpg);     // blocks per period of columns
    int64_t g = (packs + kBlock - 1) / kBlock;
    const int64_t cap = std::max<int64_t>(g0, (kMaxGrid / g0) * g0);
    g = std::min<int64_t>(g, cap);
    g = std::max<int64_t>(((g + g0 - 1) / g0) * g0, g0);
    return (int)g;
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================
struct BWorkspace {
    int64_t n = 0;
    int K = 0;
    bool mixed = false;
    void *block = nullptr;
    double *R64 = nullptr, *P64 = nullptr, *Q64 = nullptr;
    float *X32 = nullptr, *R32 = nullptr, *P32 = nullptr, *Q32 = nullptr;
    double *part = nullptr;  // 3 x kMaxGrid x K
    BCol *cols = nullptr;
    BCol *host = nullptr;    // pinned mirror
    // captured iteration chunks, keyed by chunk length, plan, precision and
    // the solution block they update (a few kept, oldest dropped first)
    struct ChunkGraph {
        hipGraphExec_t exec = nullptr;
        int chunk = 0, plan = 0, mixed = 0;
        const void *X = nullptr;
    };
    static constexpr size_t kGraphs = 16;
    std::vector<ChunkGraph> graphs;

    static size_t bytes_for(int64_t n, int K, bool mixed)
    {
        auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
        const size_t nk = (size_t)n * K;
        size_t b = 3 * al(nk * 8);
        if (mixed) b += 4 * al(nk * 4);
        b += al(3 * (size_t)kMaxGrid * K * 8) + al((size_t)K * sizeof(BCol));
        return b;
    }

    hns_status allocate(int64_t n_, int K_, bool mixed_)
    {
        n = n_;
        K = K_;
        mixed = mixed_;
        auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
        hipError_t e = hipMalloc(&block, bytes_for(n, K, mixed));
        if (e != hipSuccess) {
            block = nullptr;
            set_error("batched workspace of %zu bytes: %s", bytes_for(n, K, mixed),
                      hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        }
        const size_t nk = (size_t)n * K;
        char *c = (char *)block;
        R64 = (double *)c, c += al(nk * 8);
        P64 = (double *)c, c += al(nk * 8);
        Q64 = (double *)c, c += al(nk * 8);
        if (mixed) {
            X32 = (float *)c, c += al(nk * 4);
            R32 = (float *)c, c += al(nk * 4);
            P32 = (float *)c, c += al(nk * 4);
            Q32 = (float *)c, c += al(nk * 4);
        }
        part = (double *)c, c += al(3 * (size_t)kMaxGrid * K * 8);
        cols = (BCol *)c;
        HNS_TRY_HIP(hipHostMalloc((void **)&host, K * sizeof(BCol), hipHostMallocDefault));
        return HNS_OK;
    }

    void drop_graph()
    {
        for (auto &g : graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }

    ~BWorkspace()
    {
        drop_graph();
        if (block) (void)hipFree(block);
        if (host) (void)hipHostFree(host);
    }
};

void destroy_bworkspace(BWorkspace *w) { delete w; }

hns_status create_bworkspace(int64_t n, int K, bool mixed, BWorkspace **out)
{
    BWorkspace *w = new BWorkspace();
    hns_status st = w->allocate(n, K, mixed);
    if (st != HNS_OK) {
        delete w;
        *out = nullptr;
        return st;
    }
    *out = w;
    return HNS_OK;
}

size_t bworkspace_bytes(int64_t n, int K, bool mixed) { return BWorkspace::bytes_for(n, K, mixed); }

int bworkspace_k(const BWorkspace *w) { return w->K; }
bool bworkspace_mixed(const BWorkspace *w) { return w->mixed; }

namespace {

struct BCtx {
    hns_operator *op;
    BWorkspace *w;
    int K;
    int V;           // pack width of the iteration kernels
    const double *B;
    double *X;
    hipStream_t s;
    bool mixed;
    int tile = 0;    // tiled product shape (0: the grid-stride product of width V)
};

// A product plan as the autotuner records it: plan = V + 8 s, V the width of
// the grid-stride kernels (1, 2, 4), s the tiled product shape (0: none).
BCtx bctx(hns_operator *op, BWorkspace *w, int K, int plan, const double *B, double *X,
          hipStream_t s, bool mixed)
{
    BCtx c{op, w, K, plan & 7, B, X, s, mixed};
    c.tile = plan >> 3;
    return c;
}

hns_status pull(BCtx &c)
{
    HNS_TRY_HIP(hipMemcpyAsync(c.w->host, c.w->cols, c.K * sizeof(BCol), hipMemcpyDeviceToHost,
                               c.s));
    HNS_TRY_HIP(hipStreamSynchronize(c.s));
    return HNS_OK;
}

// Launches a kernel either on a stream or as the next node of a linear
// graph (hipGraphAddKernelNode, so no stream capture is involved and other
// threads' work on any stream cannot interfere with building the graph).
struct Launcher {
    hipStream_t s = nullptr;
    hipGraph_t g = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;

    template <typename Tuple, size_t... I>
    static void fill(void **params, Tuple &t, std::index_sequence<I...>)
    {
        ((params[I] = (void *)&std::get<I>(t)), ...);
    }

    template <typename... KArgs, typename... A>
    void operator()(void (*k)(KArgs...), int grid, int block, A... a)
    {
        with_lds(0, k, grid, block, a...);
    }

    // the same with `shm` bytes of dynamic LDS
    template <typename... KArgs, typename... A>
    void with_lds(size_t shm, void (*k)(KArgs...), int grid, int block, A... a)
    {
        if (err != hipSuccess) return;
        std::tuple<KArgs...> t(a...);
        void *params[sizeof...(KArgs)];
        fill(params, t, std::index_sequence_for<KArgs...>{});
        if (g) {
            hipKernelNodeParams p{};
            p.func = (void *)k;
            p.gridDim = dim3(grid);
            p.blockDim = dim3(block);
            p.sharedMemBytes = (unsigned int)shm;
            p.kernelParams = params;
            p.extra = nullptr;
            hipGraphNode_t node = nullptr;
            err = hipGraphAddKernelNode(&node, g, last ? &last : nullptr, last ? 1 : 0, &p);
            last = node;
        } else {
            err = hipLaunchKernel((const void *)k, dim3(grid), dim3(block), params, shm, s);
        }
    }

    hns_status status(const char *what) const
    {
        if (err != hipSuccess) {
            set_error("%s failed: %s", what, hipGetErrorString(err));
            return HNS_ERR_HIP;
        }
        return HNS_OK;
    }
};

template <typename TV, typename TX, int V, bool DOT>
void bspmm_launch(Launcher &L, const DevMatrix &A, int K, const TV *vals, const void *P, void *Q,
                  const uint8_t *bc, const BCol *cols, double *part, int G)
{
    if (A.fmt == HNS_FMT_SDIA && A.ndiag > kMaxDiag) {
        BWideOffsets o;
        for (int k = 0; k < kMaxDiagWide; ++k) o.o[k] = k < A.ndiag ? A.off[k] : 0;
        L(k_bspmm_sdia_wide<TV, TX, V, DOT>, G, kBlock, A.n, K, A.ndiag, o, vals, (const TX *)P,
          (TX *)Q, bc, cols, part);
    } else if (A.fmt == HNS_FMT_SDIA) {
        BOffsets o;
        for (int k = 0; k < kMaxDiag; ++k) o.o[k] = k < A.ndiag ? A.off[k] : 0;
#define HNS_SDIA_CASE(M)                                                              \
    case M:                                                                          \
        L(k_bspmm_sdia<TV, TX, V, DOT, M>, G, kBlock, A.n, K, o, vals, (const TX *)P, \
          (TX *)Q, bc, cols, part);                                                  \
        break;
        switch (A.ndiag) {
            HNS_SDIA_CASE(1) HNS_SDIA_CASE(2) HNS_SDIA_CASE(3) HNS_SDIA_CASE(4)
            HNS_SDIA_CASE(5) HNS_SDIA_CASE(6) HNS_SDIA_CASE(7) HNS_SDIA_CASE(8)
            HNS_SDIA_CASE(9) HNS_SDIA_CASE(10) HNS_SDIA_CASE(11) HNS_SDIA_CASE(12)
            HNS_SDIA_CASE(13) HNS_SDIA_CASE(14) HNS_SDIA_CASE(15) HNS_SDIA_CASE(16)
        }
#undef HNS_SDIA_CASE
    } else if (A.fmt == HNS_FMT_SELL) {
        L(k_bspmm_sell<TV, TX, V, DOT>, G, kBlock, A.n, K, (const int32_t *)A.slice_ptr,
          (const int32_t *)A.scol, vals, (const TX *)P, (TX *)Q, bc, cols, part);
    } else {
        L(k_bspmm_csr<TV, TX, V, DOT>, G, kBlock, A.n, K, (const int32_t *)A.rowptr,
          (const int32_t *)A.col, vals, (const TX *)P, (TX *)Q, bc, cols, part);
    }
}

// Tile shapes of k_bspmm_tile, (columns per tile, 16-byte packs per thread),
// per precision; rows per tile T = 256 * 16 / (C * sizeof) * NP ... see
// tile_rows.  Index 1.. of a shape is the `tile` choice of the autotuner (0:
// the grid-stride product).
struct TileShape {
    int C, NP;
};
constexpr int kTileShapes = kTileShapesAbi;
constexpr TileShape kTileShapes64[kTileShapes] = {{16, 2}, {8, 2}, {16, 1}};   // T = 64, 128, 32
constexpr TileShape kTileShapes32[kTileShapes] = {{32, 2}, {16, 2}, {16, 1}};  // T = 64, 128, 64
constexpr size_t kTileLds = 65536;   // bytes of LDS a tile may stage

int tile_rows(int C, int NP, size_t tx)
{
    const int W = (int)(16 / tx) * NP;
    return kBlock / (C / W);
}

// Staging plan of a tile of T rows: the distinct offsets 0, +-off[k], merged
// into clusters wherever the gap between neighbours is below T (a cluster
// [lo, hi] stages T + hi - lo rows).
void tile_plan(const DevMatrix &A, int T, TileMap *tm)
{
    std::vector<int> o = {0};
    for (int k = 0; k < A.ndiag; ++k) {
        o.push_back(A.off[k]);
        o.push_back(-A.off[k]);
    }
    std::sort(o.begin(), o.end());
    o.erase(std::unique(o.begin(), o.end()), o.end());
    memset(tm, 0, sizeof(*tm));
    std::vector<int> lo, hi;
    for (int v : o) {
        if (!lo.empty() && v - hi.back() < T)
            hi.back() = v;
        else {
            lo.push_back(v);
            hi.push_back(v);
        }
    }
    tm->nclus = (int)lo.size();
    int rows = 0;
    for (int c = 0; c < tm->nclus; ++c) {
        tm->lo[c] = lo[c];
        tm->cnt[c] = T + hi[c] - lo[c];
        tm->base[c] = rows;
        rows += tm->cnt[c];
    }
    tm->rows = rows;
    auto lrow = [&](int off) {
        for (int c = 0; c < tm->nclus; ++c)
            if (off >= lo[c] && off <= hi[c]) return tm->base[c] + (off - lo[c]);
        return 0;
    };
    tm->lrow[0] = lrow(0);
    for (int k = 0; k < A.ndiag; ++k) {
        tm->off[k] = A.off[k];
        tm->lrow[2 * k + 1] = lrow(A.off[k]);
        tm->lrow[2 * k + 2] = lrow(-A.off[k]);
    }
}

// Dynamic LDS bytes of tile shape `shape` (1-based) for K columns, or 0 when
// the shape does not apply (format, K not a multiple of C, too much LDS).
template <typename TX>
size_t tile_lds(const DevMatrix &A, int K, int shape)
{
    // the shapes are compiled for the 15-point P1 (7 upper diagonals) and the
    // 27-point Q1 (13) stencils
    if (shape < 1 || shape > kTileShapes || A.fmt != HNS_FMT_SDIA || A.unit ||
        (A.ndiag != 7 && A.ndiag != 13))
        return 0;
    const TileShape ts = sizeof(TX) == 8 ? kTileShapes64[shape - 1] : kTileShapes32[shape - 1];
    if (K % ts.C) return 0;
    const int T = tile_rows(ts.C, ts.NP, sizeof(TX));
    TileMap tm;
    tile_plan(A, T, &tm);
    const size_t b = std::max((size_t)tm.rows * ts.C * sizeof(TX), (size_t)T * ts.C * 8);
    return b <= kTileLds ? b : 0;
}

template <typename TX, int C, int NP>
int tile_launch_shape(Launcher &L, const DevMatrix &A, int K, const TX *vals, const void *P,
                      void *Q, const uint8_t *bc, const BCol *cols, double *part, size_t shm)
{
    if (A.ndiag != 7 && A.ndiag != 13) return -1;
    const int T = tile_rows(C, NP, sizeof(TX));
    TileMap tm;
    tile_plan(A, T, &tm);
    const int ngroups = K / C;
    const int64_t ntiles = (A.n + T - 1) / T;
    int64_t Gt = std::min<int64_t>(ntiles, kMaxGrid);
    // a whole number of XCDs' worth of blocks in all (the XCD renumbering)
    while (Gt > 1 && (Gt * ngroups) % 8) --Gt;
    const int64_t tpb = (ntiles + Gt - 1) / Gt;
    if (A.ndiag == 7)
        L.with_lds(shm, k_bspmm_tile<TX, TX, C, NP, 7>, (int)(Gt * ngroups), kBlock, A.n, K, tm,
                   vals, (const TX *)P, (TX *)Q, bc, cols, part, ntiles, tpb, ngroups);
    else
        L.with_lds(shm, k_bspmm_tile<TX, TX, C, NP, 13>, (int)(Gt * ngroups), kBlock, A.n, K,
                   tm, vals, (const TX *)P, (TX *)Q, bc, cols, part, ntiles, tpb, ngroups);
    return (int)Gt;
}

// Tiled product of shape `shape` (1-based); returns the number of partial
// slots per column it wrote (the G of k_bred_gamma), -1 if not applicable.
template <typename TX>
int bspmm_tile_launch(Launcher &L, const DevMatrix &A, int K, int shape, const TX *vals,
                      const void *P, void *Q, const uint8_t *bc, const BCol *cols, double *part)
{
    const size_t shm = tile_lds<TX>(A, K, shape);
    if (!shm) return -1;
    if constexpr (sizeof(TX) == 8) {
        switch (shape) {
        case 1: return tile_launch_shape<TX, 16, 2>(L, A, K, vals, P, Q, bc, cols, part, shm);
        case 2: return tile_launch_shape<TX, 8, 2>(L, A, K, vals, P, Q, bc, cols, part, shm);
        case 3: return tile_launch_shape<TX, 16, 1>(L, A, K, vals, P, Q, bc, cols, part, shm);
        }
    } else {
        switch (shape) {
        case 1: return tile_launch_shape<TX, 32, 2>(L, A, K, vals, P, Q, bc, cols, part, shm);
        case 2: return tile_launch_shape<TX, 16, 2>(L, A, K, vals, P, Q, bc, cols, part, shm);
        case 3: return tile_launch_shape<TX, 16, 1>(L, A, K, vals, P, Q, bc, cols, part, shm);
        }
    }
    return -1;
}

template <typename T>
const T *values_of(const DevMatrix &A)
{
    if (std::is_same<T, float>::value)
        return (const T *)(const void *)(A.fmt == HNS_FMT_SDIA   ? (const void *)A.dia32
                                         : A.fmt == HNS_FMT_SELL ? (const void *)A.sval32
                                                                 : (const void *)A.val32);
    return (const T *)(const void *)(A.fmt == HNS_FMT_SDIA   ? (const void *)A.dia
                                     : A.fmt == HNS_FMT_SELL ? (const void *)A.sval
                                                             : (const void *)A.val);
}

// plain FP64 product Q64 = mask_j(A X) (one element per thread)
hns_status spmm64(BCtx &c, const double *X)
{
    const DevMatrix &A = c.op->A;
    const int V = (c.K % c.V == 0) ? c.V : 1;   // the tuned pack width
    const int G = bgrid(A.n * (int64_t)c.K / V, c.K, V);
    Launcher L{c.s};
    if (V == 4)
        bspmm_launch<double, double, 4, false>(L, A, c.K, values_of<double>(A), X, c.w->Q64,
                                               c.op->bc, c.w->cols, nullptr, G);
    else if (V == 2)
        bspmm_launch<double, double, 2, false>(L, A, c.K, values_of<double>(A), X, c.w->Q64,
                                               c.op->bc, c.w->cols, nullptr, G);
    else
        bspmm_launch<double, double, 1, false>(L, A, c.K, values_of<double>(A), X, c.w->Q64,
                                               c.op->bc, c.w->cols, nullptr, G);
    return L.status("batched spmm (fp64)");
}

template <typename TX, typename TD, int V>
void iteration_v(BCtx &c, Launcher &L, TX *X, TX *R, TX *P, TX *Q, const TD *dinv)
{
    const DevMatrix &A = c.op->A;
    const int64_t np = A.n * (int64_t)c.K / V;
    const int G = bgrid(np, c.K, V);
    double *part = c.w->part;
    BCol *cols = c.w->cols;
    using TV = TX;
    int Gp = -1;
    if (c.tile > 0)
        Gp = bspmm_tile_launch<TX>(L, A, c.K, c.tile, values_of<TX>(A), P, Q, c.op->bc, cols,
                                   part);
    if (Gp < 0) {
        bspmm_launch<TV, TX, V, true>(L, A, c.K, values_of<TV>(A), P, Q, c.op->bc, cols, part, G);
        Gp = G;
    }
    L(k_bred_gamma, c.K, kBlock, c.K, (const double *)part, Gp, cols);
    L(k_bupdate<TX, TD, V>, G, kBlock, A.n, c.K, X, R, (const TX *)P, (const TX *)Q, dinv,
      (const BCol *)cols, part);
    L(k_bred_rho, c.K, kBlock, c.K, (const double *)part, G, cols);
    L(k_bpupdate<TX, TD, V>, G, kBlock, A.n, c.K, P, (const TX *)R, dinv, (const BCol *)cols);
}

template <typename TX, typename TD>
void iteration(BCtx &c, Launcher &L, TX *X, TX *R, TX *P, TX *Q, const TD *dinv)
{
    switch (c.V) {
    case 4: iteration_v<TX, TD, 4>(c, L, X, R, P, Q, dinv); break;
    case 2: iteration_v<TX, TD, 2>(c, L, X, R, P, Q, dinv); break;
    default: iteration_v<TX, TD, 1>(c, L, X, R, P, Q, dinv); break;
    }
}

hns_status enqueue_chunk(BCtx &c, Launcher &L, int count)
{
    for (int it = 0; it < count; ++it) {
        if (c.mixed)
            iteration<float, float>(c, L, c.w->X32, c.w->R32, c.w->P32, c.w->Q32,
                                    (const float *)c.op->dinv32);
        else
            iteration<double, double>(c, L, c.X, c.w->R64, c.w->P64, c.w->Q64,
                                      (const double *)c.op->dinv);
    }
    return L.status("batched iteration");
}

// A chunk of iterations, replayed from a graph when enabled.  The graph is
// built node by node (no stream capture) and bakes in the kernels (precision,
// pack width), the chunk length and every pointer; a workspace serves both
// precisions, so all of them key the cached graph.
hns_status run_chunk(BCtx &c, int count)
{
    BWorkspace *w = c.w;
    if (!c.op->use_graph) {
        Launcher L{c.s};
        return enqueue_chunk(c, L, count);
    }
    const int plan = c.V + 8 * c.tile;
    hipGraphExec_t exec = nullptr;
    for (const auto &g : w->graphs)
        if (g.chunk == count && g.plan == plan && g.X == c.X && g.mixed == (int)c.mixed)
            exec = g.exec;
    if (!exec) {
        hipGraph_t g = nullptr;
        HNS_TRY_HIP(hipGraphCreate(&g, 0));
        Launcher L;
        L.g = g;
        hns_status st = enqueue_chunk(c, L, count);
        if (st != HNS_OK) {
            (void)hipGraphDestroy(g);
            return st;
        }
        hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            set_error("graph instantiation failed: %s", hipGetErrorString(e));
            return HNS_ERR_HIP;
        }
        if (w->graphs.size() >= BWorkspace::kGraphs) {
            // drop the oldest once its replays have finished
            HNS_TRY_HIP(hipStreamSynchronize(c.s));
            (void)hipGraphExecDestroy(w->graphs.front().exec);
            w->graphs.erase(w->graphs.begin());
        }
        w->graphs.push_back({exec, count, plan, (int)c.mixed, c.X});
    }
    HNS_TRY_HIP(hipGraphLaunch(exec, c.s));
    return HNS_OK;
}

// FP64 true residual of the marked columns, then the per-column decision
hns_status true_residual(BCtx &c, double drop2, int first)
{
    const int64_t ne = c.op->n * (int64_t)c.K;
    const int G = bgrid(ne, c.K, 1);
    HNS_TRY(spmm64(c, c.X));
    k_bresidual<<<G, kBlock, 0, c.s>>>(c.op->n, c.K, c.B, c.w->Q64, c.w->R64, c.op->bc, c.w->cols,
                                       c.w->part);
    k_bred_residual<<<c.K, kBlock, 0, c.s>>>(c.op->n, c.K, c.w->part, G, c.w->cols, drop2, first);
    return bcheck("batched residual");
}

// New recurrence segment for the marked columns from R64
hns_status new_segment(BCtx &c)
{
    const int64_t ne = c.op->n * (int64_t)c.K;
    const int G = bgrid(ne, c.K, 1);
    if (c.mixed)
        k_bfrom64<float, float><<<G, kBlock, 0, c.s>>>(c.op->n, c.K, c.w->R64, c.w->R32,
                                                       c.op->dinv32, c.w->cols, c.w->part);
    else
        k_bfrom64<double, double><<<G, kBlock, 0, c.s>>>(c.op->n, c.K, c.w->R64, c.w->R64,
                                                         c.op->dinv, c.w->cols, c.w->part);
    k_bred_restart<<<c.K, kBlock, 0, c.s>>>(c.K, c.w->part, G, c.w->cols);
    const int Gp = bgrid(ne, c.K, 1);
    if (c.mixed)
        k_bpupdate<float, float, 1><<<Gp, kBlock, 0, c.s>>>(c.op->n, c.K, c.w->P32, c.w->R32,
                                                            c.op->dinv32, c.w->cols);
    else
        k_bpupdate<double, double, 1><<<Gp, kBlock, 0, c.s>>>(c.op->n, c.K, c.w->P64, c.w->R64,
                                                              c.op->dinv, c.w->cols);
    return bcheck("batched segment");
}

}  // namespace

hns_status solve_batched_impl(hns_operator *op, BWorkspace *w, int K, const int *bits,
                              const double *B, double *X, double tol, int max_iter, bool mixed,
                              int V, hipStream_t s, hns_solve_info *infos)
{
    BCtx c = bctx(op, w, K, V, B, X, s, mixed);
    const int64_t n = op->n;
    const int64_t ne = n * (int64_t)K;
    const double drop2 = mixed ? replace_drop_of(op, false) * replace_drop_of(op, false) : 0.0;
    // per-column set-up
    for (int j = 0; j < K; ++j) {
        BCol &h = w->host[j];
        memset(&h, 0, sizeof(BCol));
        h.bit = bits[j];
        h.singular = (op->kind == HNS_POISSON && bits[j] < 0) ? 1 : 0;
        h.tol2 = tol * tol;
        h.mark = 1;
        h.stop = ACTIVE;
    }
    HNS_TRY_HIP(hipMemcpyAsync(w->cols, w->host, K * sizeof(BCol), hipMemcpyHostToDevice, s));
    const int G1 = bgrid(ne, K, 1);
    k_bbstats<<<G1, kBlock, 0, s>>>(n, K, B, op->bc, w->cols, w->part);
    k_bred_bstats<<<K, kBlock, 0, s>>>(n, K, w->part, G1, w->cols);
    k_bprepare<<<G1, kBlock, 0, s>>>(n, K, X, mixed ? w->X32 : nullptr, op->bc, w->cols);
    HNS_TRY(bcheck("batched set-up"));
    HNS_TRY(pull(c));
    for (int j = 0; j < K; ++j)
        if (w->host[j].nonfinite > 0) {
            set_error("right-hand side column %d has non-finite entries", j);
            for (int q = 0; q < K; ++q) infos[q].status = HNS_ERR_INVALID;
            return HNS_ERR_INVALID;
        }
    HNS_TRY(true_residual(c, drop2, 1));
    HNS_TRY(new_segment(c));
    HNS_TRY(pull(c));
    int segments = 1;
    std::vector<int> iter_at_break(K, -1);
    // chunk length: check_every in the first segment (8, 16, ... up to it in
    // mixed precision, whose segments end at a fixed FP32 residual drop, a
    // few iterations), then the longest segment seen so far plus 2, so that
    // a replacement follows soon after the columns reach their threshold (the
    // launches of a chunk after every column has stopped return at once, but
    // still cost a launch each); the columns' arithmetic does not depend on it
    std::vector<int> seg_begin(K, 0);
    int seg_longest = 0;
    int grow = mixed ? std::min(8, op->check_every) : op->check_every;
    // a replacement serves every column that is waiting for one and costs a
    // product over the whole block (about two iterations): while other
    // columns are still running it waits up to kGrace iterations for them
    constexpr int kGrace = 2;
    int waited = -1;   // iterations run since a column first waited, -1: none waits
    for (;;) {
        int active = 0, need = 0, maxit = 0;
        bool stuck = false;
        for (int j = 0; j < K; ++j) {
            BCol &h = w->host[j];
            maxit = std::max(maxit, h.iter);
            if (h.stop == BREAK) {
                // a breakdown right after a fresh restart, with no iteration
                // done since the previous one, is final
                if (iter_at_break[j] == h.iter) {
                    h.stop = FAILED;
                    stuck = true;
                    continue;
                }
                iter_at_break[j] = h.iter;
            }
            if (h.stop == ACTIVE) ++active;
            if (h.stop == THRESH || h.stop == BREAK) ++need;
        }
        if (stuck)  // host copy is current (nothing in flight): publish FAILED
            HNS_TRY_HIP(hipMemcpyAsync(w->cols, w->host, K * sizeof(BCol), hipMemcpyHostToDevice,
                                       s));
        if (need > 0 && active > 0 && waited < kGrace && maxit < max_iter) {
            const int extra = std::min(kGrace - std::max(waited, 0), max_iter - maxit);
            HNS_TRY(run_chunk(c, extra));
            HNS_TRY(pull(c));
            waited = std::max(waited, 0) + extra;
            continue;
        }
        if (need > 0) {
            waited = -1;
            std::vector<int> restart;
            for (int j = 0; j < K; ++j) {
                const BCol &h = w->host[j];
                if (h.stop == THRESH) seg_longest = std::max(seg_longest, h.iter - seg_begin[j]);
                if (h.stop == THRESH || h.stop == BREAK) restart.push_back(j);
            }
            // collect corrections, recompute the FP64 residual of those columns
            k_bmark<<<1, kBlock, 0, s>>>(K, w->cols, 0);
            if (mixed) k_baccumulate<<<G1, kBlock, 0, s>>>(n, K, X, w->X32, w->cols);
            HNS_TRY(true_residual(c, drop2, 0));
            HNS_TRY(new_segment(c));
            HNS_TRY(pull(c));
            for (int j : restart) seg_begin[j] = w->host[j].iter;
            ++segments;
            continue;
        }
        if (active == 0 || maxit >= max_iter) break;
        int per = seg_longest > 0 ? std::max(4, seg_longest + 2) : grow;
        if (seg_longest == 0) grow = std::min(2 * grow, op->check_every);
        const int chunk = std::min(std::min(op->check_every, per), max_iter - maxit);
        HNS_TRY(run_chunk(c, chunk));
        HNS_TRY(pull(c));
    }
    // columns stopped by the iteration cap: collect their FP32 correction and
    // report their true residual
    int unfinished = 0;
    for (int j = 0; j < K; ++j) unfinished += (w->host[j].stop == ACTIVE);
    if (unfinished > 0) {
        k_bmark<<<1, kBlock, 0, s>>>(K, w->cols, 2);
        if (mixed) k_baccumulate<<<G1, kBlock, 0, s>>>(n, K, X, w->X32, w->cols);
        HNS_TRY(true_residual(c, 0.0, 0));
        HNS_TRY(bcheck("final residual"));
    }
    // zero right-hand sides give zero columns; Dirichlet entries are zero
    k_bprepare<<<G1, kBlock, 0, s>>>(n, K, X, nullptr, op->bc, w->cols);
    // pure-Neumann columns: zero mass-weighted mean
    bool any_singular = false;
    for (int j = 0; j < K; ++j) any_singular |= w->host[j].singular != 0;
    if (any_singular) {
        k_bwdot<<<G1, kBlock, 0, s>>>(n, K, X, op->lumped, w->part);
        k_bred_wdot<<<K, kBlock, 0, s>>>(K, w->part, G1, w->cols);
        k_bshift<<<G1, kBlock, 0, s>>>(n, K, X, w->cols, op->lumped_sum);
        HNS_TRY(bcheck("batched normalisation"));
    }
    HNS_TRY(pull(c));
    hns_status worst = HNS_OK;
    for (int j = 0; j < K; ++j) {
        const BCol &h = w->host[j];
        hns_solve_info &inf = infos[j];
        inf.iterations = h.iter;
        inf.outer_iterations = segments;
        inf.removed_mean = h.mean_b;
        inf.relres_true = h.bb > 0 ? std::sqrt(h.rr_true / h.bb) : 0.0;
        switch (h.stop) {
        case DONE:
        case ZERO: inf.status = HNS_OK; break;
        case BREAK:
        case FAILED: inf.status = HNS_ERR_BREAKDOWN; break;
        default: inf.status = HNS_NOT_CONVERGED; break;
        }
        if (h.stop == ZERO) inf.relres_true = 0.0;
        if (inf.status < 0 || (worst >= 0 && inf.status > worst)) worst = (hns_status)inf.status;
    }
    if (worst == HNS_ERR_BREAKDOWN) set_error("CG breakdown in at least one column");
    return worst;
}

// Time one DOT product of each pack width (1, 2, 4) and of each tiled shape
// that applies, on this workspace; times_us[0..2] the widths, [3..] the tiled
// shapes (-1 where not applicable); *best_plan = V + 8 s: V the fastest
// width (the iteration kernels' width), s the tiled shape if one beats it.
hns_status tune_batched(hns_operator *op, BWorkspace *w, int K, bool mixed, hipStream_t s,
                        double *times_us, int *best_plan)
{
    const int widths[3] = {1, 2, 4};
    hipEvent_t e0, e1;
    HNS_TRY_HIP(hipEventCreate(&e0));
    HNS_TRY_HIP(hipEventCreate(&e1));
    // columns of the tuning run: all active, no Dirichlet bits
    for (int j = 0; j < K; ++j) {
        memset(&w->host[j], 0, sizeof(BCol));
        w->host[j].bit = -1;
    }
    HNS_TRY_HIP(hipMemcpyAsync(w->cols, w->host, K * sizeof(BCol), hipMemcpyHostToDevice, s));
    const DevMatrix &A = op->A;
    const int64_t ne = A.n * (int64_t)K;
    double best = 1e300;
    int best_V = 1, best_tile = 0;
    auto time_it = [&](auto &&launch, double *out) -> hns_status {
        Launcher L{s};
        launch(L);
        HNS_TRY(L.status("tune"));
        const int reps = 10;
        HNS_TRY_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch(L);
        HNS_TRY_HIP(hipEventRecord(e1, s));
        HNS_TRY_HIP(hipEventSynchronize(e1));
        HNS_TRY(L.status("tune"));
        float ms = 0.0f;
        HNS_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
        *out = 1e3 * ms / reps;
        return HNS_OK;
    };
    for (int q = 0; q < 3; ++q) {
        const int V = widths[q];
        times_us[q] = -1.0;
        if (K % V) continue;
        const int G = bgrid(ne / V, K, V);
        auto launch = [&](Launcher &L) {
            if (mixed) {
                if (V == 1)
                    bspmm_launch<float, float, 1, true>(L, A, K, values_of<float>(A), w->P32,
                                                        w->Q32, nullptr, w->cols, w->part, G);
                else if (V == 2)
                    bspmm_launch<float, float, 2, true>(L, A, K, values_of<float>(A), w->P32,
                                                        w->Q32, nullptr, w->cols, w->part, G);
                else
                    bspmm_launch<float, float, 4, true>(L, A, K, values_of<float>(A), w->P32,
                                                        w->Q32, nullptr, w->cols, w->part, G);
            } else {
                if (V == 1)
                    bspmm_launch<double, double, 1, true>(L, A, K, values_of<double>(A),
                                                          w->P64, w->Q64, nullptr, w->cols,
                                                          w->part, G);
                else if (V == 2)
                    bspmm_launch<double, double, 2, true>(L, A, K, values_of<double>(A),
                                                          w->P64, w->Q64, nullptr, w->cols,
                                                          w->part, G);
                else
                    bspmm_launch<double, double, 4, true>(L, A, K, values_of<double>(A),
                                                          w->P64, w->Q64, nullptr, w->cols,
                                                          w->part, G);
            }
        };
        HNS_TRY(time_it(launch, &times_us[q]));
        if (times_us[q] < best) {
            best = times_us[q];
            best_V = V;
        }
    }
    const double best_stride = best;
    for (int sh = 1; sh <= kTileShapes; ++sh) {
        times_us[2 + sh] = -1.0;
        if (op->bspmm_tile == 0 || (op->bspmm_tile > 0 && op->bspmm_tile != sh)) continue;
        const bool ok = mixed ? tile_lds<float>(A, K, sh) > 0 : tile_lds<double>(A, K, sh) > 0;
        if (!ok) continue;
        auto launch = [&](Launcher &L) {
            if (mixed)
                bspmm_tile_launch<float>(L, A, K, sh, values_of<float>(A), w->P32, w->Q32,
                                         nullptr, w->cols, w->part);
            else
                bspmm_tile_launch<double>(L, A, K, sh, values_of<double>(A), w->P64, w->Q64,
                                          nullptr, w->cols, w->part);
        };
        HNS_TRY(time_it(launch, &times_us[2 + sh]));
        if (times_us[2 + sh] < best) {
            best = times_us[2 + sh];
            best_tile = sh;
        }
    }
    (void)best_stride;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *best_plan = best_V + 8 * best_tile;
    return HNS_OK;
}

// ---------------------------------------------------------------------------
// Product plans kept across processes: a small JSON object keyed by
// "arch|n|nnz|k|precision|format", in $HNS_TUNE_CACHE or else
// $XDG_CACHE_HOME/hns/bspmm_plans.json ($HOME/.cache when unset).  Unreadable
// or unwritable files are ignored (the autotuner then runs again).
// ---------------------------------------------------------------------------
namespace {

std::mutex g_plan_mutex;

std::string plan_cache_path()
{
    const char *e = getenv("HNS_TUNE_CACHE");
    if (e && *e) return e;
    const char *x = getenv("XDG_CACHE_HOME");
    const char *h = getenv("HOME");
    std::string dir = (x && *x) ? std::string(x) : (h && *h) ? std::string(h) + "/.cache" : "";
    return dir.empty() ? std::string() : dir + "/hns/bspmm_plans.json";
}

std::map<std::string, int> plan_cache_read(const std::string &path)
{
    std::map<std::string, int> m;
    FILE *f = path.empty() ? nullptr : fopen(path.c_str(), "r");
    if (!f) return m;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        const char *a = strchr(line, '"');
        const char *b = a ? strchr(a + 1, '"') : nullptr;
        const char *c = b ? strchr(b + 1, ':') : nullptr;
        if (!c) continue;
        int v = 0;
        if (sscanf(c + 1, "%d", &v) == 1) m[std::string(a + 1, b)] = v;
    }
    fclose(f);
    return m;
}

}  // namespace

std::string plan_key(const hns_operator *op, int K, bool mixed)
{
    int dev = 0;
    hipDeviceProp_t p{};
    std::string arch = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
    }
    const char *fmt = op->A.fmt == HNS_FMT_SDIA ? "sdia" : op->A.fmt == HNS_FMT_SELL ? "sell"
                                                                                     : "csr";
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|%lld|%lld|%d|%s|%s", arch.c_str(), (long long)op->n,
             (long long)op->A.nnz, K, mixed ? "fp32" : "fp64", fmt);
    return buf;
}

bool plan_cache_get(const std::string &key, int *plan)
{
    std::lock_guard<std::mutex> g(g_plan_mutex);
    const auto m = plan_cache_read(plan_cache_path());
    const auto it = m.find(key);
    if (it == m.end()) return false;
    *plan = it->second;
    return true;
}

void plan_cache_put(const std::string &key, int plan)
{
    std::lock_guard<std::mutex> g(g_plan_mutex);
    const std::string path = plan_cache_path();
    if (path.empty()) return;
    auto m = plan_cache_read(path);
    m[key] = plan;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fputs("{\n", f);
    size_t i = 0;
    for (const auto &kv : m)
        fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
    fputs("}\n", f);
    const bool ok = fclose(f) == 0;
    if (ok)
        (void)rename(tmp.c_str(), path.c_str());
    else
        (void)remove(tmp.c_str());
}

// Product plan of the batched iteration for (k, mode): the tunables when
// set, else the plan tuned earlier in this process, else the one kept in the
// plan cache for this (arch, n, nnz, k, precision, format), else the
// autotuner's (recorded in both).
hns_status batched_plan(hns_operator *op, BWorkspace *w, int k, bool mixed, hipStream_t s,
                        int *plan)
{
    if (op->bspmm_vec > 0) {
        const int V = (k % op->bspmm_vec == 0) ? op->bspmm_vec : 1;
        *plan = V + 8 * (op->bspmm_tile > 0 ? op->bspmm_tile : 0);
        return HNS_OK;
    }
    {
        std::lock_guard<std::mutex> g(op->ws_mutex);
        for (const auto &t : op->tuned)
            if (t[0] == k && t[1] == (int)mixed) {
                *plan = t[2];
                return HNS_OK;
            }
    }
    const std::string key = plan_key(op, k, mixed);
    const bool cacheable = op->bspmm_tile < 0;   // the default search only
    if (!(cacheable && plan_cache_get(key, plan))) {
        double times[3 + kTileShapesAbi];
        HNS_TRY(tune_batched(op, w, k, mixed, s, times, plan));
        if (cacheable) plan_cache_put(key, *plan);
    }
    std::lock_guard<std::mutex> g(op->ws_mutex);
    op->tuned.push_back({k, (int)mixed, *plan});
    return HNS_OK;
}

}  // namespace hns

// ===========================================================================
// Batch sessions: fixed-capacity slots that requests join and leave while the
// shared recurrence keeps running (continuous batching).  Every slot is one
// column of the n x K block; a free slot is an inactive column, so the
// captured iteration graphs stay valid as requests come and go.
// ===========================================================================
struct hns_batch {
    hns_operator *op = nullptr;
    hns::SlotSession *ss = nullptr;   // per-slot recurrences (then no block below)
    hns::BWorkspace *w = nullptr;
    double *B = nullptr;
    double *X = nullptr;
    int32_t *slot_buf = nullptr;  // device list of slots for k_bmark_list
    int K = 0;
    bool mixed = false;
    int V = 1;
    int segments = 0;
    std::vector<int> max_iter;
    std::vector<int> iter_at_break;
};

namespace hns {
namespace {

hns_status session_pull(hns_batch *bt, hipStream_t s)
{
    HNS_TRY_HIP(hipMemcpyAsync(bt->w->host, bt->w->cols, bt->K * sizeof(BCol),
                               hipMemcpyDeviceToHost, s));
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status session_push(hns_batch *bt, hipStream_t s)
{
    HNS_TRY_HIP(hipMemcpyAsync(bt->w->cols, bt->w->host, bt->K * sizeof(BCol),
                               hipMemcpyHostToDevice, s));
    return HNS_OK;
}

// Replacement / restart pass for columns at their segment threshold or
// broken down; caps columns at their iteration limit.  Host mirror current.
hns_status session_service(hns_batch *bt, hipStream_t s)
{
    BWorkspace *w = bt->w;
    const int K = bt->K;
    const int64_t n = bt->op->n;
    BCtx c = bctx(bt->op, w, K, bt->V, bt->B, bt->X, s, bt->mixed);
    const double drop2 = bt->mixed ? replace_drop_of(bt->op, false) * replace_drop_of(bt->op, false) : 0.0;
    const int G1 = bgrid(n * (int64_t)K, K, 1);
    for (int round = 0; round < 4; ++round) {
        bool changed = false;
        int need = 0;
        std::vector<int32_t> capped;
        for (int j = 0; j < K; ++j) {
            BCol &h = w->host[j];
            if (h.stop == BREAK) {
                if (bt->iter_at_break[j] == h.iter) {
                    h.stop = FAILED;  // broke down again with no iteration in between
                    changed = true;
                    continue;
                }
                bt->iter_at_break[j] = h.iter;
            }
            if ((h.stop == ACTIVE || h.stop == THRESH) && h.iter >= bt->max_iter[j]) {
                h.stop = CAPPED;
                capped.push_back(j);
                changed = true;
            } else if (h.stop == THRESH || h.stop == BREAK) {
                ++need;
            }
        }
        if (changed) HNS_TRY(session_push(bt, s));
        if (!capped.empty()) {
            // collect the FP32 correction of capped columns, report their residual
            HNS_TRY_HIP(hipMemcpyAsync(bt->slot_buf, capped.data(),
                                       capped.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            k_bmark_list<<<1, kBlock, 0, s>>>(K, w->cols, bt->slot_buf, (int)capped.size());
            if (bt->mixed) k_baccumulate<<<G1, kBlock, 0, s>>>(n, K, bt->X, w->X32, w->cols);
            HNS_TRY(true_residual(c, 0.0, 0));
        }
        if (need > 0) {
            k_bmark<<<1, kBlock, 0, s>>>(K, w->cols, 0);
            if (bt->mixed) k_baccumulate<<<G1, kBlock, 0, s>>>(n, K, bt->X, w->X32, w->cols);
            HNS_TRY(true_residual(c, drop2, 0));
            HNS_TRY(new_segment(c));
            ++bt->segments;
        }
        HNS_TRY(bcheck("session service"));
        if (capped.empty() && need == 0) return HNS_OK;
        HNS_TRY(session_pull(bt, s));
    }
    return HNS_OK;
}

}  // namespace
}  // namespace hns

using namespace hns;

extern "C" {

size_t hns_batch_footprint(const hns_operator *op, int capacity, uint32_t mode)
{
    if (!op || capacity < 1) return 0;
    if (slot_session_wanted(op, capacity))
        return slot_session_bytes(op, capacity, mode == HNS_MIXED);
    return bworkspace_bytes(op->n, capacity, mode == HNS_MIXED) +
           2 * (size_t)op->n * capacity * sizeof(double) + 256;
}

hns_status hns_batch_open(hns_operator *op, int capacity, uint32_t mode, hns_batch **out)
{
    if (!op || !out || capacity < 1 || capacity > 1024 || (mode != HNS_FP64 && mode != HNS_MIXED) ||
        (mode == HNS_MIXED && !op->dinv32)) {
        set_error("hns_batch_open: bad arguments");
        return HNS_ERR_INVALID;
    }
    if (op->A.fmt == HNS_MATRIX_FREE && (mode != HNS_FP64 || !slot_session_wanted(op, capacity))) {
        set_error("hns_batch_open: a matrix-free operator serves HNS_FP64 per-slot sessions only");
        return HNS_ERR_INVALID;
    }
    *out = nullptr;
    hns_batch *bt = new hns_batch();
    bt->op = op;
    bt->K = capacity;
    bt->mixed = (mode == HNS_MIXED);
    if (slot_session_wanted(op, capacity)) {
        const hns_status st = slot_session_open(op, capacity, bt->mixed, &bt->ss);
        if (st != HNS_OK) {
            delete bt;
            return st;
        }
        *out = bt;
        return HNS_OK;
    }
    bt->max_iter.assign(capacity, 0);
    bt->iter_at_break.assign(capacity, -1);
    hns_status st = create_bworkspace(op->n, capacity, bt->mixed, &bt->w);
    const size_t nk = (size_t)op->n * capacity;
    if (st == HNS_OK) {
        hipError_t e = hipMalloc((void **)&bt->B, 2 * nk * sizeof(double) + 256);
        if (e != hipSuccess) {
            bt->B = nullptr;
            set_error("batch session allocation failed: %s", hipGetErrorString(e));
            st = e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
        } else {
            bt->X = bt->B + nk;
            e = hipMalloc((void **)&bt->slot_buf, capacity * sizeof(int32_t));
            if (e != hipSuccess) {
                bt->slot_buf = nullptr;
                set_error("batch session allocation failed: %s", hipGetErrorString(e));
                st = HNS_ERR_OOM;
            }
        }
    }
    if (st == HNS_OK) {
        st = batched_plan(op, bt->w, capacity, bt->mixed, nullptr, &bt->V);
    }
    if (st == HNS_OK) {
        for (int j = 0; j < capacity; ++j) {
            memset(&bt->w->host[j], 0, sizeof(BCol));
            bt->w->host[j].stop = EMPTY;
            bt->w->host[j].bit = -1;
        }
        hipError_t e1 = hipMemset(bt->B, 0, 2 * nk * sizeof(double));
        hipError_t e2 = bt->mixed ? hipMemset(bt->w->X32, 0, nk * sizeof(float)) : hipSuccess;
        hipError_t e3 = hipMemcpy(bt->w->cols, bt->w->host, capacity * sizeof(BCol),
                                  hipMemcpyHostToDevice);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            set_error("batch session initialisation failed");
            st = HNS_ERR_HIP;
        }
    }
    if (st != HNS_OK) {
        hns_batch_close(bt);
        return st;
    }
    *out = bt;
    return HNS_OK;
}

void hns_batch_close(hns_batch *bt)
{
    if (!bt) return;
    if (bt->ss) {
        slot_session_close(bt->ss);
        delete bt;
        return;
    }
    (void)hipDeviceSynchronize();
    if (bt->w) destroy_bworkspace(bt->w);
    if (bt->B) (void)hipFree(bt->B);
    if (bt->slot_buf) (void)hipFree(bt->slot_buf);
    delete bt;
}

hns_status hns_batch_add(hns_batch *bt, int count, const int *slots, const int *mask_bits,
                         const double *const *b_devs, const double *tols, const int *max_iters,
                         void *stream)
{
    if (!bt || count < 1 || count > bt->K || !slots || !mask_bits || !b_devs || !tols ||
        !max_iters) {
        set_error("hns_batch_add: bad arguments");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    if (bt->ss)
        return slot_session_add(bt->ss, count, slots, mask_bits, b_devs, tols, max_iters, s);
    hns_operator *op = bt->op;
    BWorkspace *w = bt->w;
    const int K = bt->K;
    const int64_t n = op->n;
    HNS_TRY(session_pull(bt, s));
    for (int q = 0; q < count; ++q) {
        const int j = slots[q];
        if (j < 0 || j >= K || w->host[j].stop != EMPTY || !b_devs[q] || !(tols[q] > 0) ||
            max_iters[q] < 0 || mask_bits[q] < -1 || mask_bits[q] > 7 ||
            (mask_bits[q] >= 0 && !op->bc)) {
            set_error("hns_batch_add: slot %d is not free or its arguments are invalid", j);
            return HNS_ERR_INVALID;
        }
        for (int r = 0; r < q; ++r)
            if (slots[r] == j) {
                set_error("hns_batch_add: slot %d listed twice", j);
                return HNS_ERR_INVALID;
            }
    }
    for (int q = 0; q < count; ++q) {
        const int j = slots[q];
        k_bset_column<<<stream_grid(n), kBlock, 0, s>>>(n, K, bt->B, bt->X,
                                                        bt->mixed ? w->X32 : nullptr, b_devs[q], j);
        BCol &h = w->host[j];
        memset(&h, 0, sizeof(BCol));
        h.bit = mask_bits[q];
        h.singular = (op->kind == HNS_POISSON && mask_bits[q] < 0) ? 1 : 0;
        h.tol2 = tols[q] * tols[q];
        h.stop = ACTIVE;
        bt->max_iter[j] = max_iters[q];
        bt->iter_at_break[j] = -1;
    }
    HNS_TRY(bcheck("batch add"));
    HNS_TRY(session_push(bt, s));
    const int G1 = bgrid(n * (int64_t)K, K, 1);
    k_bbstats<<<G1, kBlock, 0, s>>>(n, K, bt->B, op->bc, w->cols, w->part);
    k_bred_bstats<<<K, kBlock, 0, s>>>(n, K, w->part, G1, w->cols);
    HNS_TRY(bcheck("batch add statistics"));
    HNS_TRY(session_pull(bt, s));
    std::vector<int32_t> ok;
    for (int q = 0; q < count; ++q) {
        const int j = slots[q];
        if (w->host[j].nonfinite > 0)
            w->host[j].stop = BADRHS;
        else
            ok.push_back(j);
    }
    HNS_TRY(session_push(bt, s));
    if (!ok.empty()) {
        HNS_TRY_HIP(hipMemcpyAsync(bt->slot_buf, ok.data(), ok.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, s));
        k_bmark_list<<<1, kBlock, 0, s>>>(K, w->cols, bt->slot_buf, (int)ok.size());
        BCtx c = bctx(op, w, K, bt->V, bt->B, bt->X, s, bt->mixed);
        const double drop2 = bt->mixed ? replace_drop_of(op, false) * replace_drop_of(op, false) : 0.0;
        HNS_TRY(true_residual(c, drop2, 1));
        HNS_TRY(new_segment(c));
    }
    HNS_TRY(bcheck("batch add residual"));
    HNS_TRY(session_pull(bt, s));
    return HNS_OK;
}

hns_status hns_batch_advance(hns_batch *bt, int iterations, void *stream, int *active_out)
{
    if (!bt || iterations < 0) {
        set_error("hns_batch_advance: bad arguments");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    if (bt->ss) return slot_session_advance(bt->ss, iterations, s, active_out);
    BCtx c = bctx(bt->op, bt->w, bt->K, bt->V, bt->B, bt->X, s, bt->mixed);
    HNS_TRY(session_pull(bt, s));
    int done = 0, active = 0;
    for (;;) {
        HNS_TRY(session_service(bt, s));
        active = 0;
        for (int j = 0; j < bt->K; ++j) active += (bt->w->host[j].stop == ACTIVE);
        if (active == 0 || done >= iterations) break;
        const int chunk = std::min(bt->op->check_every, iterations - done);
        HNS_TRY(run_chunk(c, chunk));
        HNS_TRY(session_pull(bt, s));
        done += chunk;
    }
    if (active_out) *active_out = active;
    return HNS_OK;
}

hns_status hns_batch_poll(hns_batch *bt, int *states, hns_solve_info *infos, void *stream)
{
    if (!bt || !states) {
        set_error("hns_batch_poll: bad arguments");
        return HNS_ERR_INVALID;
    }
    if (bt->ss) return slot_session_poll(bt->ss, states, infos);
    HNS_TRY(session_pull(bt, (hipStream_t)stream));
    for (int j = 0; j < bt->K; ++j) {
        const BCol &h = bt->w->host[j];
        states[j] = h.stop == EMPTY                                          ? 0
                    : (h.stop == ACTIVE || h.stop == THRESH || h.stop == BREAK) ? 1
                                                                             : 2;
        if (infos) {
            hns_solve_info &inf = infos[j];
            memset(&inf, 0, sizeof(inf));
            inf.iterations = h.iter;
            inf.outer_iterations = bt->segments;
            inf.removed_mean = h.mean_b;
            inf.relres_true = (h.bb > 0 && h.stop != ZERO) ? std::sqrt(h.rr_true / h.bb) : 0.0;
            inf.status = (h.stop == DONE || h.stop == ZERO)      ? HNS_OK
                         : (h.stop == FAILED || h.stop == BREAK) ? HNS_ERR_BREAKDOWN
                         : h.stop == BADRHS                      ? HNS_ERR_INVALID
                                                                 : HNS_NOT_CONVERGED;
        }
    }
    return HNS_OK;
}

hns_status hns_batch_take(hns_batch *bt, int slot, double *x_dev, hns_solve_info *info,
                          void *stream)
{
    if (!bt || slot < 0 || slot >= bt->K || !x_dev) {
        set_error("hns_batch_take: bad arguments");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    if (bt->ss) return slot_session_take(bt->ss, slot, x_dev, info, s);
    BWorkspace *w = bt->w;
    HNS_TRY(session_pull(bt, s));
    BCol &h = w->host[slot];
    if (h.stop == EMPTY || h.stop == ACTIVE || h.stop == THRESH || h.stop == BREAK) {
        set_error("hns_batch_take: slot %d has no finished solve", slot);
        return HNS_ERR_INVALID;
    }
    int states[1];
    (void)states;
    hns_solve_info inf;
    memset(&inf, 0, sizeof(inf));
    {
        std::vector<int> st(bt->K);
        std::vector<hns_solve_info> all(bt->K);
        HNS_TRY(hns_batch_poll(bt, st.data(), all.data(), stream));
        inf = all[slot];
    }
    const int64_t n = bt->op->n;
    const int K = bt->K;
    const bool shift = h.singular && (h.stop == DONE || h.stop == CAPPED);
    if (shift) {
        const int G1 = bgrid(n * (int64_t)K, K, 1);
        k_bwdot<<<G1, kBlock, 0, s>>>(n, K, bt->X, bt->op->lumped, w->part);
        k_bred_wdot<<<K, kBlock, 0, s>>>(K, w->part, G1, w->cols);
    }
    k_bget_column<<<stream_grid(n), kBlock, 0, s>>>(n, K, bt->X, x_dev, slot, w->cols,
                                                    bt->op->lumped_sum, shift ? 1 : 0);
    HNS_TRY(bcheck("batch take"));
    HNS_TRY(session_pull(bt, s));
    w->host[slot].stop = EMPTY;
    w->host[slot].mark = 0;
    HNS_TRY(session_push(bt, s));
    HNS_TRY_HIP(hipStreamSynchronize(s));
    if (info) *info = inf;
    return HNS_OK;
}

}  // extern "C"
