// HIP kernels of the Jacobi-preconditioned conjugate gradient (gfx950).
//
// One CG iteration (Remark 1 after Sec. 5 of the paper names PCG; the
// diagonal preconditioner is the DIAG part of Remark 2) is three launches:
//   spmv    q = A p (Dirichlet rows zeroed), per-block partials of p^T q
//   update  gamma = p^T q, alpha = rho / gamma, r -= alpha q,
//           z = D^-1 r (not stored), per-block partials of r^T z and r^T r
//   pupdate rho' = r^T z, rr = r^T r, beta = rho' / rho, stop flags,
//           x += alpha p, p = z + beta p
// With Jacobi scaling the same three launches run plain CG on
// D^-1/2 A D^-1/2 (unit diagonal, not stored; z = r; r^T r weighed by
// diag(A) for the stopping test).
// Each consumer kernel re-reduces the producer's per-block partials in every
// block, in one fixed order, so all blocks hold bit-identical scalars without
// a grid-wide fence, an atomic or an extra launch; block 0 records them.
// The scalars stay in device memory and every kernel exits at once when the
// stop flag is set, so the host enqueues a chunk of iterations and reads the
// flag once per chunk.  Reductions are deterministic: wavefront butterflies
// (64 lanes), the 4 wavefronts of a block through LDS, then the block
// partials in block order.  Dots accumulate in FP64 also when vectors are FP32.
//
// Precisions (template parameters): TV = matrix values, TX = vectors and
// arithmetic, TD = Jacobi diagonal.  FP64 is <double,double,double>, the FP32
// inner iteration <float,float,float>, and the FP32-storage variant
// <float,double,float> (FP32 matrix and diagonal, FP64 vectors).
//
// One-off reductions outside the iteration (right-hand-side statistics,
// residual norms, normalisation, recurrence starts) store per-block partials
// the same way and a one-workgroup launch re-reduces them into the scalars.
#include <atomic>
#include <cmath>
#include <tuple>
#include <type_traits>
#include <utility>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace hns {
namespace {

// One DPP move of a double (both 32-bit halves): lanes whose source lies
// outside the pattern (bound_ctrl) or whose row is masked off read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Wavefront sum through the DPP network instead of LDS permutes (all 64
// lanes active): row_shr 1, 2, 4, 8 leave each 16-lane row's sum in its
// lane 15, row_bcast 15 adds row 0's into row 1 and row 2's into row 3, and
// row_bcast 31 adds lane 31's into rows 2 and 3, so lane 63 holds the total,
// which every lane then reads.  A fixed order, the same in every wavefront.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_move<0x111, 0xf>(v);   // row_shr:1
    v += dpp_move<0x112, 0xf>(v);   // row_shr:2
    v += dpp_move<0x114, 0xf>(v);   // row_shr:4
    v += dpp_move<0x118, 0xf>(v);   // row_shr:8
    v += dpp_move<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_move<0x143, 0xc>(v);   // row_bcast:31
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Every block reduction of the path calls this with all 64 lanes active.
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

// Sums NV values over the block; the totals are valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * (kBlock / 64) + wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += lds[k * (kBlock / 64) + w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// Sums NV per-thread values over the block and stores them as the block's
// partials P[k * G + block] (plain stores: the consumer is a later launch).
template <int NV>
__device__ __forceinline__ void store_block_partials(double (&v)[NV], double *P)
{
    __shared__ double lds[NV * (kBlock / 64)];
    block_sum<NV>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) P[k * gridDim.x + blockIdx.x] = v[k];
    }
}

// Every block of the consumer sums the G partials of the producer in the same
// fixed order, so all blocks obtain bit-identical scalars.
template <int NV>
__device__ __forceinline__ void load_reduced(const double *__restrict__ P, int G,
                                             double (&out)[NV])
{
    __shared__ double lds[NV * (kBlock / 64)];
    // U independent loads per thread in flight at once (one L2 round trip
    // per U * kBlock partials), then added in increasing block order
    constexpr int U = NV == 1 ? 16 : 8;
    double t[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = 0.0;
    for (int b0 = threadIdx.x; b0 < G; b0 += U * kBlock) {
        double u[NV][U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int b = b0 + j * kBlock;
#pragma unroll
            for (int k = 0; k < NV; ++k) u[k][j] = b < G ? P[k * G + b] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
#pragma unroll
            for (int k = 0; k < NV; ++k) t[k] += u[k][j];
        }
    }
    // wavefront sums, then every thread adds the kBlock/64 of them from LDS
    // itself, in the order block_sum's thread 0 does (so the totals are
    // bit-identical to it): one block barrier instead of three
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = wave_sum(t[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * (kBlock / 64) + wid] = t[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += lds[k * (kBlock / 64) + w];
        out[k] = s;
    }
}

// Finishing launches of the one-off reductions (one workgroup): the producer
// kernel only stores its per-block partials, and this re-reduces them in the
// same fixed order as every CG consumer and records the totals.  A
// last-block-done pattern in the producer instead had every block take a
// device-scope atomic on one counter, serialised beyond the per-XCD L2s.
//
// Start of a recurrence: rho[0] = r^T z, rr = r^T r (bb = rr when asked),
// and the stop flag (3: b = 0, 2: non-finite, 1: already below tolerance).
__global__ __launch_bounds__(kBlock) void k_fin_start(const double *__restrict__ P, int G,
                                                      Scalars *__restrict__ sc, int bb_from_rr)
{
    double v[2];
    load_reduced<2>(P, G, v);
    if (threadIdx.x != 0) return;
    sc->rho[0] = v[0];
    sc->rr = v[1];
    sc->beta = 0.0;
    if (bb_from_rr) sc->bb = v[1];
    if (!(sc->bb > 0.0))
        sc->stop = 3;
    else if (!isfinite(v[0]) || !isfinite(v[1]))
        sc->stop = 2;
    else
        sc->stop = (v[1] <= sc->tol2 * sc->bb) ? 1 : 0;
}

// Statistics of b: sum, sum of squares, non-finite count
__global__ __launch_bounds__(kBlock) void k_fin_bstats(const double *__restrict__ P, int G,
                                                       Scalars *__restrict__ sc)
{
    double v[3];
    load_reduced<3>(P, G, v);
    if (threadIdx.x != 0) return;
    sc->sumb = v[0];
    sc->bb_raw = v[1];
    sc->nonfinite = v[2];
}

// True residual: sum of r, |b - shift|^2
__global__ __launch_bounds__(kBlock) void k_fin_residual(const double *__restrict__ P, int G,
                                                         Scalars *__restrict__ sc)
{
    double v[2];
    load_reduced<2>(P, G, v);
    if (threadIdx.x != 0) return;
    sc->sum_r = v[0];
    sc->bb = v[1];
}

// One sum into sc->rr (which = 0) or sc->wx (which = 1)
__global__ __launch_bounds__(kBlock) void k_fin_one(const double *__restrict__ P, int G,
                                                    Scalars *__restrict__ sc, int which)
{
    double v[1];
    load_reduced<1>(P, G, v);
    if (threadIdx.x != 0) return;
    if (which == 0)
        sc->rr = v[0];
    else
        sc->wx = v[0];
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each
// XCD works on one contiguous eighth of the rows (neighbour gathers of the
// SpMV then hit that XCD's own L2).
__device__ __forceinline__ int xcd_block(int b, int G)
{
    return (G >= 8 && (G & 7) == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ bool is_dirichlet(const uint8_t *bc, int bit, int64_t i)
{
    return bc != nullptr && ((bc[i] >> bit) & 1u);
}

#define GRID_STRIDE(i, n)                                                   \
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * kBlock)

// ---------------------------------------------------------------------------
// SpMV
// ---------------------------------------------------------------------------

// Sliced ELL, slice height 64 = one wavefront, one row per lane.  Each block
// owns a contiguous range of slices; its 4 wavefronts take every 4th slice.
template <typename TV, typename TX, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv_sell(int64_t n, int64_t nslices,
                                                      const int32_t *__restrict__ sptr,
                                                      const int32_t *__restrict__ col,
                                                      const TV *__restrict__ val,
                                                      const TX *__restrict__ x, TX *__restrict__ y,
                                                      const uint8_t *__restrict__ bc, int bit,
                                                      const Scalars *__restrict__ sc,
                                                      double *__restrict__ part)
{
    if constexpr (DOT) {
        if (sc->stop) return;
    }
    const int G = gridDim.x;
    const int lb = xcd_block(blockIdx.x, G);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t per = (nslices + G - 1) / G;
    const int64_t s0 = (int64_t)lb * per;
    const int64_t s1 = s0 + per < nslices ? s0 + per : nslices;
    double acc = 0.0;
    for (int64_t s = s0 + wid; s < s1; s += kBlock / 64) {
        const int32_t beg = sptr[s];
        const int32_t w = (sptr[s + 1] - beg) >> 6;
        const int32_t *c = col + beg + lane;
        const TV *v = val + beg + lane;
        TX sum = 0;
#pragma unroll 4
        for (int j = 0; j < w; ++j) sum += (TX)v[j * 64] * x[c[j * 64]];
        const int64_t row = s * 64 + lane;
        if (row < n) {
            if (is_dirichlet(bc, bit, row)) sum = 0;
            y[row] = sum;
            if constexpr (DOT) acc += (double)x[row] * (double)sum;
        }
    }
    if constexpr (DOT) {
        double v[1] = {acc};
        store_block_partials<1>(v, part);
    }
}

// CSR with 16 lanes per row (4 rows per wavefront); rows of a block are a
// contiguous range.
template <typename TV, typename TX, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(int64_t n, const int32_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col,
                                                     const TV *__restrict__ val,
                                                     const TX *__restrict__ x, TX *__restrict__ y,
                                                     const uint8_t *__restrict__ bc, int bit,
                                                     const Scalars *__restrict__ sc,
                                                     double *__restrict__ part)
{
    if constexpr (DOT) {
        if (sc->stop) return;
    }
    const int G = gridDim.x;
    const int lb = xcd_block(blockIdx.x, G);
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
    const int64_t per = (((n + G - 1) / G) + 15) / 16 * 16;
    const int64_t r0 = (int64_t)lb * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    double acc = 0.0;
    for (int64_t base = r0; base < r1; base += kBlock / 16) {
        const int64_t row = base + grp;
        TX sum = 0;
        if (row < r1) {
            const int32_t e = rowptr[row + 1];
            for (int32_t k = rowptr[row] + gl; k < e; k += 16) sum += (TX)val[k] * x[col[k]];
        }
        sum += __shfl_xor(sum, 8, 16);
        sum += __shfl_xor(sum, 4, 16);
        sum += __shfl_xor(sum, 2, 16);
        sum += __shfl_xor(sum, 1, 16);
        if (gl == 0 && row < r1) {
            if (is_dirichlet(bc, bit, row)) sum = 0;
            y[row] = sum;
            if constexpr (DOT) acc += (double)x[row] * (double)sum;
        }
    }
    if constexpr (DOT) {
        double v[1] = {acc};
        store_block_partials<1>(v, part);
    }
}

// Offsets of the upper diagonals, passed by value (kernel-argument memory)
struct DiaOffsets {
    int32_t o[kMaxDiag];
};

// Launch of kernel k on stream s.  With an event pair ev2 the dispatch itself
// records ev2[0] when the kernel starts and ev2[1] when it ends
// (hipExtLaunchKernel), so their interval is the kernel's own duration.
template <typename Tuple, size_t... I>
void arg_pointers(Tuple &t, void **p, std::index_sequence<I...>)
{
    ((p[I] = (void *)&std::get<I>(t)), ...);
}

template <typename... KArgs, typename... A>
hipError_t launch_k(void (*k)(KArgs...), int grid, int block, size_t shmem, hipStream_t s,
                    hipEvent_t *ev2, A... a)
{
    if (!ev2) {
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), shmem, s, a...);
        return hipGetLastError();
    }
    std::tuple<KArgs...> t(a...);
    void *params[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
    arg_pointers(t, params, std::index_sequence_for<KArgs...>{});
    return hipExtLaunchKernel((const void *)k, dim3(grid), dim3(block), params, shmem, s,
                              ev2[0], ev2[1], 0);
}

// R consecutive values starting at p (8-byte aligned only: a shifted row may
// start at an odd element; gfx950 global loads need no 16-byte alignment)
template <int R, typename T>
struct Run {
    T v[R];
};

template <int R, typename T>
__device__ __forceinline__ Run<R, T> ldrun(const T *p)
{
    Run<R, T> r;
    __builtin_memcpy(&r, p, sizeof(r));
    return r;
}

// Symmetric diagonal storage: row i reads the main diagonal, each upper
// diagonal at i (entry (i, i+o)) and at i-o (entry (i-o, i) = (i, i-o) by
// symmetry).  All loads are unit-stride across the wavefront (shifted copies
// of the same arrays), so there are no index arrays and no gathers.  Block b
// (after the XCD renumbering) owns rows [b rows, (b+1) rows).
//
// R = 1: one row per lane; every load is unconditional (indices clamped into
// range) so the 4 M + 2 loads of a row issue back to back, and out-of-range
// terms are dropped by a select afterwards.
// R = 2: two consecutive rows per lane with 16-byte loads (half as many load
// instructions); rows within the largest offset of either end take a
// per-row path with explicit range tests.  Both forms add the terms of a row
// in the same order: main, then (upper, lower) for each offset.
// UNIT: the symmetrically Jacobi-scaled operator D^-1/2 A D^-1/2, whose main
// diagonal is 1 and not stored; dia then holds the M upper diagonals only.
// Waves per SIMD the two-row FP64 form is compiled for, as (min, max):
// exactly 3 for the 15-point operator (M = 7: 162 VGPRs, every load of a lane
// in flight; measured faster than 4 waves at 102 VGPRs), else the default.
template <typename TV, typename TX, int M, int R>
constexpr bool sdia_three_waves()
{
    return sizeof(TV) == 8 && sizeof(TX) == 8 && R == 2 && M == 7;
}

template <typename TV, typename TX, bool DOT, int M, int R, bool UNIT = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(sdia_three_waves<TV, TX, M, R>() ? 3 : 1,
                                   sdia_three_waves<TV, TX, M, R>() ? 3 : 8)))
void k_spmv_sdia(int64_t n, int64_t rows, DiaOffsets offs,
                                                      const TV *__restrict__ dia,
                                                      const TX *__restrict__ x, TX *__restrict__ y,
                                                      const uint8_t *__restrict__ bc, int bit,
                                                      const Scalars *__restrict__ sc,
                                                      double *__restrict__ part)
{
    if constexpr (DOT) {
        if (sc->stop) return;
    }
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)lb * rows;
    const int64_t r1 = r0 + rows < n ? r0 + rows : n;
    constexpr int K0 = UNIT ? 0 : 1;   // array of the first upper diagonal
    double acc = 0.0;
    if constexpr (R == 1) {
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
            const TX xi = x[i];
            TX sum = UNIT ? xi : (TX)dia[i] * xi;
            TV up[M], lo[M];
            TX xu[M], xl[M];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t o = offs.o[k];
                const TV *u = dia + (int64_t)(k + K0) * n;
                const int64_t iu = i + o < n ? i + o : n - 1;
                const int64_t il = i >= o ? i - o : 0;
                up[k] = u[i];
                xu[k] = x[iu];
                lo[k] = u[il];
                xl[k] = x[il];
            }
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t o = offs.o[k];
                sum += (i + o < n) ? (TX)up[k] * xu[k] : (TX)0;
                sum += (i >= o) ? (TX)lo[k] * xl[k] : (TX)0;
            }
            if (is_dirichlet(bc, bit, i)) sum = 0;
            y[i] = sum;
            if constexpr (DOT) acc += (double)xi * (double)sum;
        }
    } else {
        const int64_t omax = offs.o[M - 1];
        for (int64_t i = r0 + (int64_t)threadIdx.x * R; i < r1; i += (int64_t)kBlock * R) {
            if (i >= omax && i + (R - 1) + omax < n) {
                // the Dirichlet bits first: tested between the products they
                // make the compiler hold all 4 M + 2 loads at once (182
                // VGPRs for M = 7 instead of 102)
                bool dm[R];
#pragma unroll
                for (int e = 0; e < R; ++e) dm[e] = is_dirichlet(bc, bit, i + e);
                const Run<R, TX> xi = ldrun<R>(x + i);
                Run<R, TV> d0;
                if constexpr (!UNIT) d0 = ldrun<R>(dia + i);
                Run<R, TV> up[M], lo[M];
                Run<R, TX> xu[M], xl[M];
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int64_t o = offs.o[k];
                    const TV *u = dia + (int64_t)(k + K0) * n;
                    up[k] = ldrun<R>(u + i);
                    xu[k] = ldrun<R>(x + i + o);
                    lo[k] = ldrun<R>(u + i - o);
                    xl[k] = ldrun<R>(x + i - o);
                }
                Run<R, TX> out;
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    TX sum = UNIT ? xi.v[e] : (TX)d0.v[e] * xi.v[e];
#pragma unroll
                    for (int k = 0; k < M; ++k) {
                        sum += (TX)up[k].v[e] * xu[k].v[e];
                        sum += (TX)lo[k].v[e] * xl[k].v[e];
                    }
                    if (dm[e]) sum = 0;
                    out.v[e] = sum;
                    if constexpr (DOT) acc += (double)xi.v[e] * (double)sum;
                }
                __builtin_memcpy(y + i, &out, sizeof(out));
            } else {
                for (int e = 0; e < R; ++e) {
                    const int64_t j = i + e;
                    if (j >= r1) break;
                    const TX xj = x[j];
                    TX sum = UNIT ? xj : (TX)dia[j] * xj;
                    for (int k = 0; k < M; ++k) {
                        const int64_t o = offs.o[k];
                        const TV *u = dia + (int64_t)(k + K0) * n;
                        if (j + o < n) sum += (TX)u[j] * x[j + o];
                        if (j >= o) sum += (TX)u[j - o] * x[j - o];
                    }
                    if (is_dirichlet(bc, bit, j)) sum = 0;
                    y[j] = sum;
                    if constexpr (DOT) acc += (double)xj * (double)sum;
                }
            }
        }
    }
    if constexpr (DOT) {
        double v[1] = {acc};
        store_block_partials<1>(v, part);
    }
}

// Fused multiply-add in the vector type (the direction and x updates of the
// scaled recurrence are written with it wherever they are evaluated, so that
// every evaluation of p' = r + beta p gives the same bits)
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Completion of a scaled CG iteration by every block (the direction
// update's prologue): rho', rr and the stopping decision from the update
// partials, recorded by block 0.  False when the iteration's update did not
// run (its tag is not the last recorded one).
template <typename TX>
__device__ __forceinline__ bool dir_prologue(Scalars *__restrict__ sc,
                                             const double *__restrict__ part_in, int G_in,
                                             int parity, uint32_t token, TX &alpha, TX &beta,
                                             bool &dir)
{
    const uint32_t tag = sc->xtoken;
    const double alpha_d = sc->alpha;
    double v[2];
    load_reduced<2>(part_in, G_in, v);
    if (tag != token) return false;
    const double rho_new = v[0], rr = v[1];
    const bool bad = !isfinite(rho_new) || !isfinite(rr);
    const bool conv = !bad && rr <= sc->tol2 * sc->bb;
    const double beta_d = rho_new / sc->rho[parity];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rho[parity ^ 1] = rho_new;
        sc->rr = rr;
        sc->beta = beta_d;
        sc->iter += 1;
        if (bad)
            sc->stop = 2;
        else if (conv)
            sc->stop = 1;
    }
    alpha = (TX)alpha_d;
    beta = (TX)beta_d;
    dir = !(bad || conv);
    return true;
}

// Direction update and product in one launch, for CG on the Jacobi-scaled
// operator (unit diagonal, M upper diagonals, z = r): completes iteration
// k (the one tagged `token`) and starts k + 1.  Every block forms rho', rr,
// beta and the stopping decision as the direction update does, then for its
// own rows x += alpha p_k and p_{k+1} = r + beta p_k (stored into pn, the
// other buffer), and forms q = A p_{k+1} with every neighbour value
// p_{k+1}[j] recomputed from r[j] and p_k[j] by the same expression: the
// products, the p^T q partials and all scalars are bit for bit those of the
// separate direction update and product.  Rows, their order and the order
// of the terms are those of k_spmv_sdia (UNIT, DOT).  On a stop
// (convergence or a non-finite scalar) only x is updated, and p_k is copied
// into pc, the buffer the caller reads p from after a chunk.
template <typename TX, int M, int R>
__global__ __launch_bounds__(kBlock)
void k_sdia_dir(int64_t n, int64_t rows, DiaOffsets offs, const TX *__restrict__ dia,
                const TX *__restrict__ po, const TX *__restrict__ r, TX *__restrict__ x,
                TX *__restrict__ pn, TX *pc, TX *__restrict__ q,
                const uint8_t *__restrict__ bc, int bit, Scalars *__restrict__ sc,
                const double *__restrict__ part_in, int G_in, double *__restrict__ part_out,
                int parity, uint32_t token)
{
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)lb * rows;
    const int64_t r1 = r0 + rows < n ? r0 + rows : n;
    // one row per lane: every load of a row (clamped indices, as in
    // k_spmv_sdia) in one batch; the thread's first row is loaded before the
    // prologue, so those loads overlap its wait for the update partials
    struct RowLoads {
        TX pi, ri, xi, up[M], lo[M], pu[M], ru[M], pl[M], rl[M];
        bool dm;
    };
    auto load_row = [&](int64_t i) {
        RowLoads L;
        L.pi = po[i];
        L.ri = r[i];
        L.xi = x[i];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int64_t o = offs.o[k];
            const TX *u = dia + (int64_t)k * n;
            const int64_t iu = i + o < n ? i + o : n - 1;
            const int64_t il = i >= o ? i - o : 0;
            L.up[k] = u[i];
            L.pu[k] = po[iu];
            L.ru[k] = r[iu];
            L.lo[k] = u[il];
            L.pl[k] = po[il];
            L.rl[k] = r[il];
        }
        L.dm = is_dirichlet(bc, bit, i);
        return L;
    };
    const int64_t i0 = r0 + threadIdx.x;
    RowLoads first;
    if constexpr (R == 1) {
        if (i0 < r1) first = load_row(i0);
    }
    TX alpha = 0, beta = 0;
    bool dir = true;
    if (!dir_prologue<TX>(sc, part_in, G_in, parity, token, alpha, beta, dir)) return;
    if (!dir) {
        for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
            const TX pi = po[i];
            x[i] = fma_t(alpha, pi, x[i]);
            if (pc != po) pc[i] = pi;
        }
        return;
    }
    double acc = 0.0;
    if constexpr (R == 1) {
        auto row = [&](int64_t i, const RowLoads &L) {
            const TX xo = fma_t(alpha, L.pi, L.xi);
            const TX xi = fma_t(beta, L.pi, L.ri);
            TX sum = xi;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t o = offs.o[k];
                const TX xu = fma_t(beta, L.pu[k], L.ru[k]);
                const TX xl = fma_t(beta, L.pl[k], L.rl[k]);
                sum += (i + o < n) ? L.up[k] * xu : (TX)0;
                sum += (i >= o) ? L.lo[k] * xl : (TX)0;
            }
            if (L.dm) sum = 0;
            x[i] = xo;
            pn[i] = xi;
            q[i] = sum;
            acc += (double)xi * (double)sum;
        };
        if (i0 < r1) row(i0, first);
        for (int64_t i = i0 + kBlock; i < r1; i += kBlock) row(i, load_row(i));
    } else {
        const int64_t omax = offs.o[M - 1];
        for (int64_t i = r0 + (int64_t)threadIdx.x * R; i < r1; i += (int64_t)kBlock * R) {
            if (i >= omax && i + (R - 1) + omax < n) {
                bool dm[R];
#pragma unroll
                for (int e = 0; e < R; ++e) dm[e] = is_dirichlet(bc, bit, i + e);
                // every load first (as in k_spmv_sdia), the stores last
                const Run<R, TX> pi = ldrun<R>(po + i), ri = ldrun<R>(r + i);
                Run<R, TX> xo = ldrun<R>(x + i);
                Run<R, TX> up[M], lo[M], pu[M], ru[M], pl[M], rl[M];
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int64_t o = offs.o[k];
                    const TX *u = dia + (int64_t)k * n;
                    up[k] = ldrun<R>(u + i);
                    pu[k] = ldrun<R>(po + i + o);
                    ru[k] = ldrun<R>(r + i + o);
                    lo[k] = ldrun<R>(u + i - o);
                    pl[k] = ldrun<R>(po + i - o);
                    rl[k] = ldrun<R>(r + i - o);
                }
                Run<R, TX> xi, out;
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    xo.v[e] = fma_t(alpha, pi.v[e], xo.v[e]);
                    xi.v[e] = fma_t(beta, pi.v[e], ri.v[e]);
                    TX sum = xi.v[e];
#pragma unroll
                    for (int k = 0; k < M; ++k) {
                        sum += up[k].v[e] * fma_t(beta, pu[k].v[e], ru[k].v[e]);
                        sum += lo[k].v[e] * fma_t(beta, pl[k].v[e], rl[k].v[e]);
                    }
                    if (dm[e]) sum = 0;
                    out.v[e] = sum;
                    acc += (double)xi.v[e] * (double)sum;
                }
                __builtin_memcpy(x + i, &xo, sizeof(xo));
                __builtin_memcpy(pn + i, &xi, sizeof(xi));
                __builtin_memcpy(q + i, &out, sizeof(out));
            } else {
                for (int e = 0; e < R; ++e) {
                    const int64_t j = i + e;
                    if (j >= r1) break;
                    const TX pj = po[j];
                    x[j] = fma_t(alpha, pj, x[j]);
                    const TX xj = fma_t(beta, pj, r[j]);
                    pn[j] = xj;
                    TX sum = xj;
                    for (int k = 0; k < M; ++k) {
                        const int64_t o = offs.o[k];
                        const TX *u = dia + (int64_t)k * n;
                        if (j + o < n) sum += u[j] * fma_t(beta, po[j + o], r[j + o]);
                        if (j >= o) sum += u[j - o] * fma_t(beta, po[j - o], r[j - o]);
                    }
                    if (is_dirichlet(bc, bit, j)) sum = 0;
                    q[j] = sum;
                    acc += (double)xj * (double)sum;
                }
            }
        }
    }
    double w[1] = {acc};
    store_block_partials<1>(w, part_out);
}

// The direction update that ends a chunk of fused iterations: completes the
// iteration tagged `token` from p_k in po, writing x += alpha p_k and, unless
// stopping, p_{k+1} = r + beta p_k into pc (po and pc may be one buffer:
// each element is read and written by one thread); on a stop p_k is copied
// into pc.  Rows as in k_sdia_dir.
template <typename TX>
__global__ __launch_bounds__(kBlock) void k_sdia_dir_close(int64_t n, int64_t rows,
                                                           const TX *po, const TX *__restrict__ r,
                                                           TX *__restrict__ x, TX *pc,
                                                           Scalars *__restrict__ sc,
                                                           const double *__restrict__ part_in,
                                                           int G_in, int parity, uint32_t token)
{
    TX alpha = 0, beta = 0;
    bool dir = true;
    if (!dir_prologue<TX>(sc, part_in, G_in, parity, token, alpha, beta, dir)) return;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)lb * rows;
    const int64_t r1 = r0 + rows < n ? r0 + rows : n;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kBlock) {
        const TX pi = po[i];
        x[i] = fma_t(alpha, pi, x[i]);
        pc[i] = dir ? fma_t(beta, pi, r[i]) : pi;
    }
}

// ---------------------------------------------------------------------------
// Jacobi scaling: point-Jacobi PCG on A is plain CG on D^-1/2 A D^-1/2 with
// the vectors x_S = D^1/2 x, r_S = D^-1/2 r, p_S = D^1/2 p (the same alpha,
// beta and iterates in exact arithmetic); the scaled operator has a unit
// diagonal, so neither the main diagonal nor D^-1 is read per iteration.
// ---------------------------------------------------------------------------

// s = d^-1/2 and w = (float) d from the main diagonal d of A
__global__ __launch_bounds__(kBlock) void k_jacobi_diag(int64_t n, const double *__restrict__ d,
                                                        double *__restrict__ sh,
                                                        float *__restrict__ w)
{
    GRID_STRIDE(i, n)
    {
        const double di = d[i];
        sh[i] = 1.0 / sqrt(di);
        w[i] = (float)di;
    }
}

// upper diagonal k of the scaled operator: a_{i, i+o} s_i s_{i+o}
__global__ __launch_bounds__(kBlock) void k_jacobi_scale(int64_t n, int ndiag, DiaOffsets offs,
                                                         const double *__restrict__ dia,
                                                         const double *__restrict__ sh,
                                                         double *__restrict__ out,
                                                         float *__restrict__ out32)
{
    GRID_STRIDE(i, n)
    {
        const double si = sh[i];
        for (int k = 0; k < ndiag; ++k) {
            const int64_t j = i + offs.o[k];
            const double v = j < n ? dia[(int64_t)(k + 1) * n + i] * si * sh[j] : 0.0;
            out[(int64_t)k * n + i] = v;
            if (out32) out32[(int64_t)k * n + i] = (float)v;
        }
    }
}

// Segment start from the FP64 true residual: r = (TX)(s r64), p = r, dx = 0;
// rho[0] = r^T r, rr = r64^T r64.  r64 and r may be the same array (each
// element is read before it is overwritten, by the same thread).
template <typename TX>
__global__ __launch_bounds__(kBlock) void k_scale_in(int64_t n, const double *r64, TX *r,
                                                     TX *__restrict__ p, TX *__restrict__ dx,
                                                     const double *__restrict__ sh,
                                                     Scalars *__restrict__ sc,
                                                     double *__restrict__ partials)
{
    double rho = 0.0, rr = 0.0;
    GRID_STRIDE(i, n)
    {
        const double ra = r64[i];
        const TX ri = (TX)(sh[i] * ra);
        r[i] = ri;
        p[i] = ri;
        dx[i] = (TX)0;
        rho += (double)ri * (double)ri;
        rr += ra * ra;
    }
    double v[2] = {rho, rr};
    store_block_partials<2>(v, partials);
}

// Segment end: x += s dx in FP64, dx = 0
template <typename TX>
__global__ __launch_bounds__(kBlock) void k_scale_out(int64_t n, double *__restrict__ x,
                                                      TX *__restrict__ dx,
                                                      const double *__restrict__ sh)
{
    GRID_STRIDE(i, n)
    {
        x[i] += sh[i] * (double)dx[i];
        dx[i] = (TX)0;
    }
}

// Residual replacement of the scaled FP32 recurrence: r = (float)(s r64);
// per-block partials of r^T r and r64^T r64 for the k_pupdate that follows.
__global__ __launch_bounds__(kBlock) void k_replace_rz_scaled(int64_t n,
                                                              const double *__restrict__ r64,
                                                              float *__restrict__ r,
                                                              const double *__restrict__ sh,
                                                              double *__restrict__ part_out)
{
    double rz = 0.0, rr = 0.0;
    GRID_STRIDE(i, n)
    {
        const double ra = r64[i];
        const float ri = (float)(sh[i] * ra);
        r[i] = ri;
        rz += (double)ri * (double)ri;
        rr += ra * ra;
    }
    double v[2] = {rz, rr};
    store_block_partials<2>(v, part_out);
}

// Offsets of the wide symmetric-diagonal format (kernel-argument memory)
struct WideOffsets {
    int32_t o[kMaxDiagWide];
};

// Symmetric diagonal storage with more upper diagonals than the unrolled
// kernel takes (Q2 bricks: 62).  Same layout, same per-row order of the
// terms (main, then (upper, lower) for each offset in ascending order), but
// the offsets are streamed in groups of 8 so that a group's 32 loads are in
// flight together without holding all 4 M of them in registers.  R rows per
// lane as in k_spmv_sdia; interior rows take R-wide loads, rows within the
// largest offset of either end the per-row path with range tests.
template <typename TV, typename TX, bool DOT, int R>
__global__ __launch_bounds__(kBlock) void k_spmv_sdia_wide(int64_t n, int64_t rows, int M,
                                                           WideOffsets offs,
                                                           const TV *__restrict__ dia,
                                                           const TX *__restrict__ x,
                                                           TX *__restrict__ y,
                                                           const uint8_t *__restrict__ bc, int bit,
                                                           const Scalars *__restrict__ sc,
                                                           double *__restrict__ part)
{
    constexpr int GK = 8;
    if constexpr (DOT) {
        if (sc->stop) return;
    }
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t r0 = (int64_t)lb * rows;
    const int64_t r1 = r0 + rows < n ? r0 + rows : n;
    const int64_t omax = offs.o[M - 1];
    const int Mfull = M - M % GK;
    double acc = 0.0;
    for (int64_t i = r0 + (int64_t)threadIdx.x * R; i < r1; i += (int64_t)kBlock * R) {
        if (i >= omax && i + (R - 1) + omax < n) {
            const Run<R, TX> xi = ldrun<R>(x + i);
            const Run<R, TV> d0 = ldrun<R>(dia + i);
            TX sum[R];
#pragma unroll
            for (int e = 0; e < R; ++e) sum[e] = (TX)d0.v[e] * xi.v[e];
            for (int k0 = 0; k0 < Mfull; k0 += GK) {
                Run<R, TV> up[GK], lo[GK];
                Run<R, TX> xu[GK], xl[GK];
#pragma unroll
                for (int g = 0; g < GK; ++g) {
                    const int64_t o = offs.o[k0 + g];
                    const TV *u = dia + (int64_t)(k0 + g + 1) * n;
                    up[g] = ldrun<R>(u + i);
                    xu[g] = ldrun<R>(x + i + o);
                    lo[g] = ldrun<R>(u + i - o);
                    xl[g] = ldrun<R>(x + i - o);
                }
#pragma unroll
                for (int g = 0; g < GK; ++g)
#pragma unroll
                    for (int e = 0; e < R; ++e) {
                        sum[e] += (TX)up[g].v[e] * xu[g].v[e];
                        sum[e] += (TX)lo[g].v[e] * xl[g].v[e];
                    }
            }
            for (int k = Mfull; k < M; ++k) {
                const int64_t o = offs.o[k];
                const TV *u = dia + (int64_t)(k + 1) * n;
                const Run<R, TV> up = ldrun<R>(u + i), lo = ldrun<R>(u + i - o);
                const Run<R, TX> xu = ldrun<R>(x + i + o), xl = ldrun<R>(x + i - o);
#pragma unroll
                for (int e = 0; e < R; ++e) {
                    sum[e] += (TX)up.v[e] * xu.v[e];
                    sum[e] += (TX)lo.v[e] * xl.v[e];
                }
            }
            Run<R, TX> out;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                out.v[e] = is_dirichlet(bc, bit, i + e) ? (TX)0 : sum[e];
                if constexpr (DOT) acc += (double)xi.v[e] * (double)out.v[e];
            }
            __builtin_memcpy(y + i, &out, sizeof(out));
        } else {
            for (int e = 0; e < R; ++e) {
                const int64_t j = i + e;
                if (j >= r1) break;
                const TX xj = x[j];
                TX sum = (TX)dia[j] * xj;
                for (int k = 0; k < M; ++k) {
                    const int64_t o = offs.o[k];
                    const TV *u = dia + (int64_t)(k + 1) * n;
                    if (j + o < n) sum += (TX)u[j] * x[j + o];
                    if (j >= o) sum += (TX)u[j - o] * x[j - o];
                }
                if (is_dirichlet(bc, bit, j)) sum = 0;
                y[j] = sum;
                if constexpr (DOT) acc += (double)xj * (double)sum;
            }
        }
    }
    if constexpr (DOT) {
        double v[1] = {acc};
        store_block_partials<1>(v, part);
    }
}

// ---------------------------------------------------------------------------
// CG vector updates
// ---------------------------------------------------------------------------

// V consecutive elements moved by one load/store instruction (16 bytes of TX)
template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
    T v[V];
};

// Elementwise loop over [0, n) in packs of V consecutive elements (V > 1
// needs 16-byte aligned arrays).  With per > 0, block b (after the XCD
// renumbering) owns packs [b per, (b+1) per) and block 0 also takes the
// scalar tail; with per == 0 packs and tail are dealt grid-stride.
template <int V, typename F>
__device__ __forceinline__ void for_packs(int64_t n, int64_t per, F &&body)
{
    const int64_t np = n / V;
    if (per > 0) {
        const int64_t j0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
        const int64_t j1 = j0 + per < np ? j0 + per : np;
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kBlock)
            body(j * V, std::integral_constant<int, V>());
        if constexpr (V > 1) {
            if (blockIdx.x == 0 && threadIdx.x < n - np * V)
                body(np * V + threadIdx.x, std::integral_constant<int, 1>());
        }
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < np; j += stride)
        body(j * V, std::integral_constant<int, V>());
    if constexpr (V > 1) {
        for (int64_t i = np * V + blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += stride)
            body(i, std::integral_constant<int, 1>());
    }
}

// for_packs for kernels that first need a block-wide prologue (the
// re-reduction of the previous kernel's partials): each thread issues the
// loads of its first pack before the prologue runs, so their memory latency
// overlaps the prologue, and loads every further pack before it processes
// the current one.  prologue() runs in every thread and returns the same
// value in all threads of a block; false ends the loop (returns false).
// (Loading all of a thread's packs before the prologue was measured slower:
// the extra registers halve the occupancy.)
template <int V, typename Load, typename Pro, typename Body>
__device__ __forceinline__ bool for_packs_ahead(int64_t n, int64_t per, Load &&load,
                                                Pro &&prologue, Body &&body)
{
    using IV = std::integral_constant<int, V>;
    using I1 = std::integral_constant<int, 1>;
    const int64_t np = n / V;
    int64_t j, j1, step;
    if (per > 0) {
        const int64_t j0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * per;
        j = j0 + threadIdx.x;
        j1 = j0 + per < np ? j0 + per : np;
        step = kBlock;
    } else {
        j = blockIdx.x * (int64_t)kBlock + threadIdx.x;
        j1 = np;
        step = (int64_t)gridDim.x * kBlock;
    }
    decltype(load(int64_t(0), IV())) cur{};
    if (j < j1) cur = load(j * V, IV());
    if (!prologue()) return false;
    while (j < j1) {
        const int64_t jn = j + step;
        decltype(cur) nxt{};
        if (jn < j1) nxt = load(jn * V, IV());
        body(j * V, cur);
        cur = nxt;
        j = jn;
    }
    if constexpr (V > 1) {
        if (per > 0) {
            if (blockIdx.x == 0 && threadIdx.x < n - np * V) {
                const int64_t i = np * V + threadIdx.x;
                body(i, load(i, I1()));
            }
        } else {
            for (int64_t i = np * V + blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += step)
                body(i, load(i, I1()));
        }
    }
    return true;
}

template <int W, typename T>
__device__ __forceinline__ Pack<T, W> ld(const T *p, int64_t i)
{
    return *reinterpret_cast<const Pack<T, W> *>(p + i);
}

template <int W, typename T>
__device__ __forceinline__ void st(T *p, int64_t i, const Pack<T, W> &v)
{
    *reinterpret_cast<Pack<T, W> *>(p + i) = v;
}

template <typename TX, typename TD, int W>
struct UpdatePacks {
    Pack<TX, W> r, q;
    Pack<TD, W> d;
};

template <typename TX, typename TD, int W>
struct DirPacks {
    Pack<TX, W> p, r;
    Pack<TD, W> d;
};

template <typename TX, typename TD, int W>
struct XDirPacks {
    Pack<TX, W> p, r, x;
    Pack<TD, W> d;
};

// r -= alpha q; partials of r^T D^-1 r and r^T r.  Block 0 records alpha and
// this iteration's tag, which the direction update needs to add alpha p to x.
// SC (CG on the Jacobi-scaled operator, r = D^-1/2 r_A): dinv holds the
// weights diag(A) instead, and the partials are r^T r and r^T diag(A) r, the
// latter being |r_A|^2 of the unscaled residual.
template <typename TX, typename TD, int V, bool SC = false>
__global__ __launch_bounds__(kBlock) void k_update(int64_t n, int64_t per, TX *__restrict__ r,
                                                   const TX *__restrict__ q,
                                                   const TD *__restrict__ dinv,
                                                   Scalars *__restrict__ sc,
                                                   const double *__restrict__ part_in, int G_in,
                                                   double *__restrict__ part_out, int parity,
                                                   uint32_t token)
{
    TX alpha = 0;
    auto load = [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        return UpdatePacks<TX, TD, W>{ld<W>(r, i), ld<W>(q, i), ld<W>(dinv, i)};
    };
    // the stop flag is read here, after the first pack's loads are issued and
    // beside the partials, rather than at entry: a stopped launch still ends
    // without a store, and a running one does not wait for the flag first
    auto prologue = [&]() {
        const int stopped = sc->stop;
        double g[1];
        load_reduced<1>(part_in, G_in, g);
        if (stopped) return false;
        const double gamma = g[0];
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sc->gamma = gamma;
                sc->stop = 2;
            }
            return false;
        }
        const double alpha_d = sc->rho[parity] / gamma;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->gamma = gamma;
            sc->alpha = alpha_d;
            sc->xtoken = token;
        }
        alpha = (TX)alpha_d;
        return true;
    };
    double rz = 0.0, rr = 0.0;
    auto body = [&](int64_t i, auto in) {
        constexpr int W = sizeof(in.r.v) / sizeof(TX);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            in.r.v[e] = in.r.v[e] - alpha * in.q.v[e];
            const double ri = (double)in.r.v[e];
            if constexpr (SC) {
                rz += ri * ri;
                rr += (double)in.d.v[e] * ri * ri;
            } else {
                const TX zi = (TX)in.d.v[e] * in.r.v[e];
                rz += ri * (double)zi;
                rr += ri * ri;
            }
        }
        st<W>(r, i, in.r);
    };
    if (!for_packs_ahead<V>(n, per, load, prologue, body)) return;
    double v[2] = {rz, rr};
    store_block_partials<2>(v, part_out);
}

// rho' = r^T z, rr = r^T r from the update partials; beta = rho' / rho;
// p = D^-1 r + beta p unless converged.  `count` is added to the iteration
// counter (0 when used after a residual replacement).
// SC: the Jacobi-scaled recurrence, z = r (dinv is not read).
template <typename TX, typename TD, int V = 1, bool SC = false>
__global__ __launch_bounds__(kBlock) void k_pupdate(int64_t n, int64_t per, TX *__restrict__ p,
                                                    const TX *__restrict__ r,
                                                    const TD *__restrict__ dinv,
                                                    Scalars *__restrict__ sc,
                                                    const double *__restrict__ part_in, int G_in,
                                                    int parity, int count)
{
    TX beta = 0;
    auto load = [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        if constexpr (SC)
            return DirPacks<TX, TD, W>{ld<W>(p, i), ld<W>(r, i), {}};
        else
            return DirPacks<TX, TD, W>{ld<W>(p, i), ld<W>(r, i), ld<W>(dinv, i)};
    };
    // the stop flag is read in the prologue, by every wave, and every wave
    // then passes the block barrier of the re-reduction: block 0 of this very
    // launch may raise the flag, and an entry test could let some waves of a
    // later block leave while the others sum LDS slots the leavers never wrote
    // (a block that sees the flag raised by block 0 here computes the same
    // stopping decision from the same partials)
    auto prologue = [&]() {
        const int stopped = sc->stop;
        double v[2];
        load_reduced<2>(part_in, G_in, v);
        if (stopped) return false;
        const double rho_new = v[0], rr = v[1];
        const bool bad = !isfinite(rho_new) || !isfinite(rr);
        const bool conv = !bad && rr <= sc->tol2 * sc->bb;
        const double beta_d = rho_new / sc->rho[parity];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rho[parity ^ 1] = rho_new;
            sc->rr = rr;
            sc->beta = beta_d;
            sc->iter += count;
            if (bad)
                sc->stop = 2;
            else if (conv)
                sc->stop = 1;
        }
        beta = (TX)beta_d;
        return !(bad || conv);
    };
    auto body = [&](int64_t i, auto in) {
        constexpr int W = sizeof(in.p.v) / sizeof(TX);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            if constexpr (SC)
                in.p.v[e] = fma_t(beta, in.p.v[e], in.r.v[e]);
            else
                in.p.v[e] = (TX)in.d.v[e] * in.r.v[e] + beta * in.p.v[e];
        }
        st<W>(p, i, in.p);
    };
    for_packs_ahead<V>(n, per, load, prologue, body);
}

// The direction update of a point-Jacobi iteration, completing it: when this
// iteration's update ran (its tag is recorded; written by an earlier launch,
// so every block reads it consistently), x += alpha p with the old p, then,
// unless the iteration converged or broke down, p = D^-1 r + beta p.  The
// entry test is the tag and not the stop flag: block 0 of this launch may
// raise the flag while other blocks still have their x update to do.
// SC: the Jacobi-scaled recurrence, z = r (dinv is not read).
template <typename TX, typename TD, int V = 1, bool SC = false>
__global__ __launch_bounds__(kBlock) void k_pupdate_x(int64_t n, int64_t per,
                                                      TX *__restrict__ x, TX *__restrict__ p,
                                                      const TX *__restrict__ r,
                                                      const TD *__restrict__ dinv,
                                                      Scalars *__restrict__ sc,
                                                      const double *__restrict__ part_in,
                                                      int G_in, int parity, uint32_t token)
{
    TX alpha = 0;
    TX beta = 0;
    bool dir = true;
    auto load = [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        if constexpr (SC)
            return XDirPacks<TX, TD, W>{ld<W>(p, i), ld<W>(r, i), ld<W>(x, i), {}};
        else
            return XDirPacks<TX, TD, W>{ld<W>(p, i), ld<W>(r, i), ld<W>(x, i), ld<W>(dinv, i)};
    };
    // the tag and alpha are read in the prologue (as the update reads its stop
    // flag), after the first pack's loads are issued
    auto prologue = [&]() {
        const uint32_t tag = sc->xtoken;
        const double alpha_d = sc->alpha;
        double v[2];
        load_reduced<2>(part_in, G_in, v);
        if (tag != token) return false;
        alpha = (TX)alpha_d;
        const double rho_new = v[0], rr = v[1];
        const bool bad = !isfinite(rho_new) || !isfinite(rr);
        const bool conv = !bad && rr <= sc->tol2 * sc->bb;
        const double beta_d = rho_new / sc->rho[parity];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rho[parity ^ 1] = rho_new;
            sc->rr = rr;
            sc->beta = beta_d;
            sc->iter += 1;
            if (bad)
                sc->stop = 2;
            else if (conv)
                sc->stop = 1;
        }
        beta = (TX)beta_d;
        dir = !(bad || conv);
        return true;
    };
    auto body = [&](int64_t i, auto in) {
        constexpr int W = sizeof(in.p.v) / sizeof(TX);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            if constexpr (SC)
                in.x.v[e] = fma_t(alpha, in.p.v[e], in.x.v[e]);
            else
                in.x.v[e] = in.x.v[e] + alpha * in.p.v[e];
        }
        st<W>(x, i, in.x);
        if (dir) {
#pragma unroll
            for (int e = 0; e < W; ++e) {
                if constexpr (SC)
                    in.p.v[e] = fma_t(beta, in.p.v[e], in.r.v[e]);
                else
                    in.p.v[e] = (TX)in.d.v[e] * in.r.v[e] + beta * in.p.v[e];
            }
            st<W>(p, i, in.p);
        }
    };
    for_packs_ahead<V>(n, per, load, prologue, body);
}

// (singular: r -= mean r) z = D^-1 r; p = z; rho[0] = r^T z; rr = r^T r.
template <typename TX, typename TD>
__global__ __launch_bounds__(kBlock) void k_init_dir(int64_t n, TX *__restrict__ r,
                                                     TX *__restrict__ p,
                                                     const TD *__restrict__ dinv, int singular,
                                                     Scalars *__restrict__ sc,
                                                     double *__restrict__ partials)
{
    const TX mean = singular ? (TX)(sc->sum_r / (double)n) : (TX)0;
    double rz = 0.0, rr = 0.0;
    GRID_STRIDE(i, n)
    {
        TX ri = r[i];
        if (singular) {
            ri -= mean;
            r[i] = ri;
        }
        const TX zi = (TX)dinv[i] * ri;
        p[i] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    double v[2] = {rz, rr};
    store_block_partials<2>(v, partials);
}

// ---------------------------------------------------------------------------
// Vertical-line (water column) block preconditioner
// ---------------------------------------------------------------------------
// The rows of the vertical-first numbering form columns of L consecutive
// nodes; z = M^-1 r solves each column's tridiagonal block (diagonal and the
// couplings to the nodes above and below) by the Thomas recurrences with
// precomputed inverse pivots w and masked off-diagonal e:
//   y_0 = r_0 w_0,  y_k = (r_k - e_{k-1} y_{k-1}) w_k,
//   z_{L-1} = y_{L-1},  z_k = y_k - (e_k w_k) z_{k+1}.
// A block owns NC whole columns: its rows are staged through LDS with
// coalesced loads, one lane per column runs the two recurrences, and the
// result goes back to HBM coalesced.

// Thomas recurrences of the columns staged in LDS: sr holds r (read), se, sw
// the factors, sy receives z; returns this lane's share of r^T z.
// The four arrays are disjoint regions of the block's LDS (restrict lets the
// loads of later steps, which do not depend on the recurrence, issue ahead of
// the earlier steps' stores; the unrolled loops give them room to).
// T = double (FP64 solves) or float (the inner iterations of mixed precision;
// r^T z is always summed in FP64).
template <typename T>
__device__ __forceinline__ double line_columns(int ncols, int L, const T *__restrict__ sr,
                                               const T *__restrict__ se,
                                               const T *__restrict__ sw, T *__restrict__ sy)
{
    double rz = 0.0;
    if ((int)threadIdx.x < ncols) {
        const int b = threadIdx.x * L;
        T y = sr[b] * sw[b];
        sy[b] = y;
#pragma unroll 4
        for (int k = 1; k < L; ++k) {
            y = (sr[b + k] - se[b + k - 1] * y) * sw[b + k];
            sy[b + k] = y;
        }
        T z = y;
        rz += (double)sr[b + L - 1] * (double)z;
#pragma unroll 4
        for (int k = L - 2; k >= 0; --k) {
            z = sy[b + k] - (se[b + k] * sw[b + k]) * z;
            sy[b + k] = z;
            rz += (double)sr[b + k] * (double)z;
        }
    }
    return rz;
}

template <typename T, int W>
struct XLinePacks {
    Pack<T, W> p, z, x;
};

template <typename T, int W>
struct LinePacks {
    Pack<T, W> p, z;
};

constexpr int kLineLds = 49152;   // bytes of LDS for the staged columns of one block
// rows of a block's columns a thread stages at most: a block stages at most
// kLineLds / (4 * 8) rows (4 FP64-sized arrays of its rows in LDS)
constexpr int kLineStage = (kLineLds / (4 * 8) + kBlock - 1) / kBlock;

// r -= alpha q; z = M^-1 r; partials of r^T z and r^T r.  Block 0 records
// alpha and the iteration tag (x += alpha p is done by k_pupdate_line_x).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_update_line(
    int64_t n, int L, int NC, T *__restrict__ r, const T *__restrict__ q, T *__restrict__ z,
    const T *__restrict__ lfac, Scalars *__restrict__ sc, const double *__restrict__ part_in,
    int G_in, double *__restrict__ part_out, int parity, uint32_t token)
{
    extern __shared__ double line_lds[];
    const int span = NC * L;   // at most kLineStage * kBlock rows (NC from kLineLds)
    T *sr = reinterpret_cast<T *>(line_lds), *se = sr + span, *sw = se + span, *sy = sw + span;
    const int64_t row0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * span;
    const int64_t left = n - row0;
    const int rows = left <= 0 ? 0 : (left < span ? (int)left : span);
    const T *le = lfac, *lw = lfac + n;
    // every load of the thread's rows is issued first, ahead of the partials
    // that alpha waits for (one round trip instead of one per row)
    T rv[kLineStage], qv[kLineStage], ev[kLineStage], wv[kLineStage];
#pragma unroll
    for (int u = 0; u < kLineStage; ++u) {
        const int t = threadIdx.x + u * kBlock;
        rv[u] = qv[u] = ev[u] = wv[u] = (T)0;
        if (t < rows) {
            const int64_t i = row0 + t;
            rv[u] = r[i];
            qv[u] = q[i];
            ev[u] = le[i];
            wv[u] = lw[i];
        }
    }
    // the stop flag is read beside the partials rather than before them
    const int stopped = sc->stop;
    double g[1];
    load_reduced<1>(part_in, G_in, g);
    if (stopped) return;
    const double gamma = g[0];
    if (!(gamma > 0.0) || !isfinite(gamma)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->gamma = gamma;
            sc->stop = 2;
        }
        return;
    }
    const double alpha_d = sc->rho[parity] / gamma;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gamma = gamma;
        sc->alpha = alpha_d;
        sc->xtoken = token;
    }
    const T alpha = (T)alpha_d;
    double rr = 0.0;
#pragma unroll
    for (int u = 0; u < kLineStage; ++u) {
        const int t = threadIdx.x + u * kBlock;
        if (t < rows) {
            const T ri = rv[u] - alpha * qv[u];
            r[row0 + t] = ri;
            sr[t] = ri;
            se[t] = ev[u];
            sw[t] = wv[u];
            rr += (double)ri * (double)ri;
        }
    }
    __syncthreads();
    const double rz = line_columns<T>(rows / L, L, sr, se, sw, sy);
    __syncthreads();
    for (int t = threadIdx.x; t < rows; t += kBlock) z[row0 + t] = sy[t];
    double v[2] = {rz, rr};
    store_block_partials<2>(v, part_out);
}

// Direction update of the line and IC(0) iterations, completing them as
// k_pupdate_x does for point Jacobi: when this iteration's update ran (its
// tag is recorded), x += alpha p with the old p; then rho' = r^T z, rr = r^T r
// from the partials, beta = rho'/rho and, unless converged or broken down,
// p = z + beta p.
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_pupdate_line_x(int64_t n, int64_t per,
                                                           T *__restrict__ x, T *__restrict__ p,
                                                           const T *__restrict__ z,
                                                           Scalars *__restrict__ sc,
                                                           const double *__restrict__ part_in,
                                                           int G_in, int parity, uint32_t token)
{
    T alpha = 0;
    T beta = 0;
    bool dir = true;
    auto load = [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        return XLinePacks<T, W>{ld<W>(p, i), ld<W>(z, i), ld<W>(x, i)};
    };
    // the tag and alpha are read in the prologue, after the first pack's
    // loads are issued (as in k_pupdate_x)
    auto prologue = [&]() {
        const uint32_t tag = sc->xtoken;
        const double alpha_d = sc->alpha;
        double v[2];
        load_reduced<2>(part_in, G_in, v);
        if (tag != token) return false;
        alpha = (T)alpha_d;
        const double rho_new = v[0], rr = v[1];
        const bool bad = !isfinite(rho_new) || !isfinite(rr);
        const bool conv = !bad && rr <= sc->tol2 * sc->bb;
        const double beta_d = rho_new / sc->rho[parity];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rho[parity ^ 1] = rho_new;
            sc->rr = rr;
            sc->beta = beta_d;
            sc->iter += 1;
            if (bad)
                sc->stop = 2;
            else if (conv)
                sc->stop = 1;
        }
        beta = (T)beta_d;
        dir = !(bad || conv);
        return true;
    };
    auto body = [&](int64_t i, auto in) {
        constexpr int W = sizeof(in.p.v) / sizeof(T);
#pragma unroll
        for (int e = 0; e < W; ++e) in.x.v[e] = in.x.v[e] + alpha * in.p.v[e];
        st<W>(x, i, in.x);
        if (dir) {
#pragma unroll
            for (int e = 0; e < W; ++e) in.p.v[e] = in.z.v[e] + beta * in.p.v[e];
            st<W>(p, i, in.p);
        }
    };
    for_packs_ahead<V>(n, per, load, prologue, body);
}

// (singular: r -= mean r); z = M^-1 r; p = z; rho[0] = r^T z; rr = r^T r.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init_line(int64_t n, int L, int NC,
                                                      T *__restrict__ r, T *__restrict__ p,
                                                      const T *__restrict__ lfac, int singular,
                                                      Scalars *__restrict__ sc,
                                                      double *__restrict__ partials)
{
    extern __shared__ double line_lds[];
    const T mean = singular ? (T)(sc->sum_r / (double)n) : (T)0;
    const int span = NC * L;
    T *sr = reinterpret_cast<T *>(line_lds), *se = sr + span, *sw = se + span, *sy = sw + span;
    const int64_t row0 = (int64_t)blockIdx.x * span;
    const int64_t left = n - row0;
    const int rows = left <= 0 ? 0 : (left < span ? (int)left : span);
    const T *le = lfac, *lw = lfac + n;
    double rr = 0.0;
    for (int t = threadIdx.x; t < rows; t += kBlock) {
        const int64_t i = row0 + t;
        T ri = r[i];
        if (singular) {
            ri -= mean;
            r[i] = ri;
        }
        sr[t] = ri;
        se[t] = le[i];
        sw[t] = lw[i];
        rr += (double)ri * (double)ri;
    }
    __syncthreads();
    const double rz = line_columns<T>(rows / L, L, sr, se, sw, sy);
    __syncthreads();
    for (int t = threadIdx.x; t < rows; t += kBlock) p[row0 + t] = sy[t];
    double v[2] = {rz, rr};
    store_block_partials<2>(v, partials);
}

// Residual replacement of a line-preconditioned mixed-precision segment: the
// FP32 residual becomes the FP64 true residual r64 (cast), z = M^-1 r, and the
// partials of r^T z and r^T r feed k_pdir_line (the counterpart of
// k_replace_rz for point Jacobi).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_replace_line(int64_t n, int L, int NC,
                                                         const double *__restrict__ r64,
                                                         T *__restrict__ r, T *__restrict__ z,
                                                         const T *__restrict__ lfac,
                                                         double *__restrict__ part_out)
{
    extern __shared__ double line_lds[];
    const int span = NC * L;
    T *sr = reinterpret_cast<T *>(line_lds), *se = sr + span, *sw = se + span, *sy = sw + span;
    const int64_t row0 = (int64_t)xcd_block(blockIdx.x, gridDim.x) * span;
    const int64_t left = n - row0;
    const int rows = left <= 0 ? 0 : (left < span ? (int)left : span);
    const T *le = lfac, *lw = lfac + n;
    double rr = 0.0;
    for (int t = threadIdx.x; t < rows; t += kBlock) {
        const int64_t i = row0 + t;
        const T ri = (T)r64[i];
        r[i] = ri;
        sr[t] = ri;
        se[t] = le[i];
        sw[t] = lw[i];
        rr += (double)ri * (double)ri;
    }
    __syncthreads();
    const double rz = line_columns<T>(rows / L, L, sr, se, sw, sy);
    __syncthreads();
    for (int t = threadIdx.x; t < rows; t += kBlock) z[row0 + t] = sy[t];
    double v[2] = {rz, rr};
    store_block_partials<2>(v, part_out);
}

// rho' = r^T z, rr = r^T r from the partials, beta = rho' / rho, p = z + beta p
// unless the recursive residual is already below the segment threshold (no
// iteration is counted: the direction after a residual replacement)
template <typename T, int V>
__global__ __launch_bounds__(kBlock) void k_pdir_line(int64_t n, int64_t per, T *__restrict__ p,
                                                      const T *__restrict__ z,
                                                      Scalars *__restrict__ sc,
                                                      const double *__restrict__ part_in,
                                                      int G_in, int parity)
{
    T beta = 0;
    auto load = [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        return LinePacks<T, W>{ld<W>(p, i), ld<W>(z, i)};
    };
    // stop flag read by every wave before the re-reduction's barrier (as in
    // k_pupdate: block 0 of this launch may raise it)
    auto prologue = [&]() {
        const int stopped = sc->stop;
        double v[2];
        load_reduced<2>(part_in, G_in, v);
        if (stopped) return false;
        const double rho_new = v[0], rr = v[1];
        const bool bad = !isfinite(rho_new) || !isfinite(rr);
        const bool conv = !bad && rr <= sc->tol2 * sc->bb;
        const double beta_d = rho_new / sc->rho[parity];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->rho[parity ^ 1] = rho_new;
            sc->rr = rr;
            sc->beta = beta_d;
            if (bad)
                sc->stop = 2;
            else if (conv)
                sc->stop = 1;
        }
        beta = (T)beta_d;
        return !(bad || conv);
    };
    auto body = [&](int64_t i, auto in) {
        constexpr int W = sizeof(in.p.v) / sizeof(T);
#pragma unroll
        for (int e = 0; e < W; ++e) in.p.v[e] = in.z.v[e] + beta * in.p.v[e];
        st<W>(p, i, in.p);
    };
    for_packs_ahead<V>(n, per, load, prologue, body);
}

// ---------------------------------------------------------------------------
// IC(0) in the multicolour order
// ---------------------------------------------------------------------------
// Rows of one colour are not coupled, so each triangular solve is one launch
// per colour, one lane per row (permuted positions [r0, r1)).  The factor
// rows of a colour are stored column-major (entry k of local row j at
// k nc + j), so a lane issues the loads of all its entries, then all its
// gathers of y, instead of one dependent index-then-value round trip per
// entry; the entries are subtracted in the row's order.  A row is taken in
// groups of WM entries held in registers (one group for the P1 stencils; the
// longer rows of the Q2 bricks take several).

// v - sum_k a_k y[c_k] over the len entries of local row j of a colour block
template <int WM>
__device__ __forceinline__ double ic_row_sum(double v, int len, int64_t j, int64_t nc,
                                             const int32_t *__restrict__ col,
                                             const double *__restrict__ val,
                                             const double *__restrict__ y)
{
    for (int k0 = 0; k0 < len; k0 += WM) {
        int32_t c[WM];
        double a[WM], yv[WM];
#pragma unroll
        for (int k = 0; k < WM; ++k) {
            c[k] = 0;
            a[k] = 0.0;
            if (k0 + k < len) {
                c[k] = col[(int64_t)(k0 + k) * nc + j];
                a[k] = val[(int64_t)(k0 + k) * nc + j];
            }
        }
#pragma unroll
        for (int k = 0; k < WM; ++k) {
            yv[k] = 0.0;
            if (k0 + k < len) yv[k] = y[c[k]];
        }
#pragma unroll
        for (int k = 0; k < WM; ++k)
            if (k0 + k < len) v -= a[k] * yv[k];
    }
    return v;
}

// forward: y_r = (r[perm_r] - sum_t L_rt y_t) / L_rr; col / val point at the
// colour's block
template <int WM>
__global__ __launch_bounds__(kBlock) void k_ic_forward(int64_t r0, int64_t r1,
                                                       const int32_t *__restrict__ perm,
                                                       const int64_t *__restrict__ lptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val,
                                                       const double *__restrict__ diag,
                                                       const double *__restrict__ r,
                                                       double *__restrict__ y)
{
    const int64_t nc = r1 - r0;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < nc;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t row = r0 + j;
        const int len = (int)(lptr[row + 1] - lptr[row]);
        const double v = ic_row_sum<WM>(r[perm[row]], len, j, nc, col, val, y);
        y[row] = v / diag[row];
    }
}

// backward: w_r = (y_r - sum_t U_rt w_t) / L_rr (U = L^T), in place in y;
// z[perm_r] = w_r
template <int WM>
__global__ __launch_bounds__(kBlock) void k_ic_backward(int64_t r0, int64_t r1,
                                                        const int32_t *__restrict__ perm,
                                                        const int64_t *__restrict__ uptr,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        const double *__restrict__ diag,
                                                        double *__restrict__ y,
                                                        double *__restrict__ z)
{
    const int64_t nc = r1 - r0;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < nc;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t row = r0 + j;
        const int len = (int)(uptr[row + 1] - uptr[row]);
        double v = ic_row_sum<WM>(y[row], len, j, nc, col, val, y);
        v /= diag[row];
        y[row] = v;
        z[perm[row]] = v;
    }
}

template <int W>
struct RQPacks {
    Pack<double, W> r, q;
};

// r -= alpha q (no partials: r^T z and r^T r follow the solves); block 0
// records alpha and the iteration tag for k_pupdate_line_x
template <int V>
__global__ __launch_bounds__(kBlock) void k_update_noz(int64_t n, int64_t per,
                                                       double *__restrict__ r,
                                                       const double *__restrict__ q,
                                                       Scalars *__restrict__ sc,
                                                       const double *__restrict__ part_in,
                                                       int G_in, int parity, uint32_t token)
{
    double alpha = 0.0;
    auto load = [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        return RQPacks<W>{ld<W>(r, i), ld<W>(q, i)};
    };
    // stop flag read by every wave before the re-reduction's barrier (block 0
    // of this launch may raise it on a breakdown)
    auto prologue = [&]() {
        const int stopped = sc->stop;
        double g[1];
        load_reduced<1>(part_in, G_in, g);
        if (stopped) return false;
        const double gamma = g[0];
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sc->gamma = gamma;
                sc->stop = 2;
            }
            return false;
        }
        alpha = sc->rho[parity] / gamma;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->gamma = gamma;
            sc->alpha = alpha;
            sc->xtoken = token;
        }
        return true;
    };
    auto body = [&](int64_t i, auto in) {
        constexpr int W = sizeof(in.r.v) / sizeof(double);
#pragma unroll
        for (int e = 0; e < W; ++e) in.r.v[e] = in.r.v[e] - alpha * in.q.v[e];
        st<W>(r, i, in.r);
    };
    for_packs_ahead<V>(n, per, load, prologue, body);
}

// per-block partials of r^T z and r^T r (consumed like the update's)
template <int V>
__global__ __launch_bounds__(kBlock) void k_dot_rz(int64_t n, int64_t per,
                                                   const double *__restrict__ r,
                                                   const double *__restrict__ z,
                                                   const Scalars *__restrict__ sc,
                                                   double *__restrict__ part_out)
{
    if (sc->stop) return;
    double rz = 0.0, rr = 0.0;
    for_packs<V>(n, per, [&](int64_t i, auto w) {
        constexpr int W = decltype(w)::value;
        const auto rv = ld<W>(r, i);
        const auto zv = ld<W>(z, i);
#pragma unroll
        for (int e = 0; e < W; ++e) {
            rz += rv.v[e] * zv.v[e];
            rr += rv.v[e] * rv.v[e];
        }
    });
    double v[2] = {rz, rr};
    store_block_partials<2>(v, part_out);
}

// p = z; rho[0] = r^T z; rr = r^T r (first direction of an IC(0) recurrence)
__global__ __launch_bounds__(kBlock) void k_init_from_z(int64_t n, const double *__restrict__ r,
                                                        const double *__restrict__ z,
                                                        double *__restrict__ p,
                                                        Scalars *__restrict__ sc,
                                                        double *__restrict__ partials)
{
    double rz = 0.0, rr = 0.0;
    GRID_STRIDE(i, n)
    {
        const double ri = r[i], zi = z[i];
        p[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    double v[2] = {rz, rr};
    store_block_partials<2>(v, partials);
}

// Residual replacement: the working residual becomes the FP64 true residual
// (converted to TX when dst is given, else src is the working residual), with
// per-block partials of r^T D^-1 r and r^T r for the k_pupdate that follows.
template <typename TX, typename TD>
__global__ __launch_bounds__(kBlock) void k_replace_rz(int64_t n, const double *__restrict__ src,
                                                       TX *__restrict__ dst,
                                                       const TD *__restrict__ dinv,
                                                       double *__restrict__ part_out)
{
    double rz = 0.0, rr = 0.0;
    GRID_STRIDE(i, n)
    {
        const TX ri = (TX)src[i];
        if (dst) dst[i] = ri;
        const TX zi = (TX)dinv[i] * ri;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    double v[2] = {rz, rr};
    store_block_partials<2>(v, part_out);
}

// ---------------------------------------------------------------------------
// One-off kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_bstats(int64_t n, const double *__restrict__ b,
                                                   const uint8_t *__restrict__ bc, int bit,
                                                   Scalars *__restrict__ sc,
                                                   double *__restrict__ partials)
{
    double s = 0.0, s2 = 0.0, bad = 0.0;
    GRID_STRIDE(i, n)
    {
        double bi = is_dirichlet(bc, bit, i) ? 0.0 : b[i];
        if (!isfinite(bi)) {
            bad += 1.0;
            bi = 0.0;
        }
        s += bi;
        s2 += bi * bi;
    }
    double v[3] = {s, s2, bad};
    store_block_partials<3>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_prepare_x(int64_t n, double *__restrict__ x,
                                                      const uint8_t *__restrict__ bc, int bit,
                                                      int zero_all)
{
    GRID_STRIDE(i, n)
    if (zero_all || is_dirichlet(bc, bit, i)) x[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_residual(int64_t n, const double *__restrict__ b,
                                                     const double *__restrict__ q,
                                                     double *__restrict__ r,
                                                     const uint8_t *__restrict__ bc, int bit,
                                                     int singular, Scalars *__restrict__ sc,
                                                     double *__restrict__ partials)
{
    const double shift = singular ? sc->sumb / (double)n : 0.0;
    double sr = 0.0, sbb = 0.0;
    GRID_STRIDE(i, n)
    {
        double bi = b[i] - shift;
        double ri = bi - q[i];
        if (is_dirichlet(bc, bit, i)) {
            bi = 0.0;
            ri = 0.0;
        }
        r[i] = ri;
        sr += ri;
        sbb += bi * bi;
    }
    double v[2] = {sr, sbb};
    store_block_partials<2>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_project_norm(int64_t n, double *__restrict__ r,
                                                         int singular, Scalars *__restrict__ sc,
                                                         double *__restrict__ partials)
{
    const double mean = singular ? sc->sum_r / (double)n : 0.0;
    double rr = 0.0;
    GRID_STRIDE(i, n)
    {
        double ri = r[i];
        if (singular) {
            ri -= mean;
            r[i] = ri;
        }
        rr += ri * ri;
    }
    double v[1] = {rr};
    store_block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_cast_scaled(int64_t n, const double *__restrict__ r64,
                                                        float *__restrict__ r32,
                                                        float *__restrict__ d32,
                                                        const Scalars *__restrict__ outer)
{
    const double inv = 1.0 / sqrt(outer->rr);
    GRID_STRIDE(i, n)
    {
        r32[i] = (float)(r64[i] * inv);
        d32[i] = 0.0f;
    }
}

__global__ __launch_bounds__(kBlock) void k_correct(int64_t n, double *__restrict__ x,
                                                    const float *__restrict__ d32,
                                                    const Scalars *__restrict__ outer)
{
    const double s = sqrt(outer->rr);
    GRID_STRIDE(i, n) x[i] += s * (double)d32[i];
}

__global__ __launch_bounds__(kBlock) void k_cast(int64_t n, const double *__restrict__ r64,
                                                 float *__restrict__ r32, float *__restrict__ x32)
{
    GRID_STRIDE(i, n)
    {
        r32[i] = (float)r64[i];
        x32[i] = 0.0f;
    }
}

// x64 += x32; x32 = 0 (the FP64 solution collects the FP32 corrections)
__global__ __launch_bounds__(kBlock) void k_accumulate(int64_t n, double *__restrict__ x64,
                                                       float *__restrict__ x32)
{
    GRID_STRIDE(i, n)
    {
        x64[i] += (double)x32[i];
        x32[i] = 0.0f;
    }
}

__global__ void k_set_threshold(Scalars *sc, double tol2, double bb)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->tol2 = tol2;
        sc->bb = bb;
        sc->stop = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_wdot(int64_t n, const double *__restrict__ w,
                                                 const double *__restrict__ x,
                                                 Scalars *__restrict__ sc,
                                                 double *__restrict__ partials)
{
    double s = 0.0;
    GRID_STRIDE(i, n) s += w[i] * x[i];
    double v[1] = {s};
    store_block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_shift(int64_t n, double *__restrict__ x,
                                                  const Scalars *__restrict__ sc, double wsum)
{
    const double c = sc->wx / wsum;
    GRID_STRIDE(i, n) x[i] -= c;
}

hns_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", what, hipGetErrorString(e));
        return HNS_ERR_HIP;
    }
    return HNS_OK;
}

// A product that could not be launched: the HIP error if there is one, else
// HNS_ERR_INVALID (the dispatcher has set the reason)
static hns_status spmv_failed(const char *what)
{
    const hns_status st = check_launch(what);
    return st != HNS_OK ? st : HNS_ERR_INVALID;
}

// Rows per block of the diagonal SpMV: R rows per lane (two for FP64
// vectors), `it` workgroup-sized passes per block, more passes when the grid
// would exceed the partials slots.
template <typename TX>
int sdia_rows(const DevMatrix &A)
{
    return sizeof(TX) == 8 ? A.rows_per_lane64() : 1;
}

template <typename TX>
Chunks sdia_chunks(const DevMatrix &A)
{
    const int R = sdia_rows<TX>(A);
    const int it = sizeof(TX) == 8 ? A.spmv_it64 : A.spmv_passes32();
    return chunks(A.n, (int64_t)kBlock * R * (it > 0 ? it : 1), (int64_t)kBlock * R,
                  sizeof(TX) == 8 ? kMaxPart : kMaxPartSpmv32);
}

template <typename TV, typename TX, bool DOT, int M, int R>
int sdia_launch_r(const DevMatrix &A, const TV *vals, const void *p, void *q, const uint8_t *bc,
                  int bit, const Scalars *sc, double *part, hipStream_t s, hipEvent_t *ev2)
{
    DiaOffsets offs;
    for (int k = 0; k < kMaxDiag; ++k) offs.o[k] = k < A.ndiag ? A.off[k] : 0;
    const Chunks c = sdia_chunks<TX>(A);
    if constexpr (DOT && std::is_same<TV, TX>::value) {
        if (A.unit) {
            if (launch_k(k_spmv_sdia<TV, TX, DOT, M, R, true>, c.grid, kBlock, 0, s, ev2, A.n,
                         c.per, offs, vals, (const TX *)p, (TX *)q, bc, bit, sc,
                         part) != hipSuccess)
                return -1;
            return c.grid;
        }
    }
    if (A.unit) return -1;   // the unit-diagonal form runs the CG products only
    if (launch_k(k_spmv_sdia<TV, TX, DOT, M, R>, c.grid, kBlock, 0, s, ev2, A.n, c.per, offs,
                 vals, (const TX *)p, (TX *)q, bc, bit, sc, part) != hipSuccess)
        return -1;
    return c.grid;
}

template <typename TV, typename TX, bool DOT, int M>
int sdia_launch(const DevMatrix &A, const TV *vals, const void *p, void *q, const uint8_t *bc,
                int bit, const Scalars *sc, double *part, hipStream_t s, hipEvent_t *ev2)
{
    if constexpr (sizeof(TX) == 8) {
        if (sdia_rows<TX>(A) == 2)
            return sdia_launch_r<TV, TX, DOT, M, 2>(A, vals, p, q, bc, bit, sc, part, s, ev2);
    }
    return sdia_launch_r<TV, TX, DOT, M, 1>(A, vals, p, q, bc, bit, sc, part, s, ev2);
}

template <typename TV, typename TX, bool DOT>
int sdia_wide_launch(const DevMatrix &A, const TV *vals, const void *p, void *q,
                     const uint8_t *bc, int bit, const Scalars *sc, double *part, hipStream_t s,
                     hipEvent_t *ev2)
{
    WideOffsets offs;
    for (int k = 0; k < kMaxDiagWide; ++k) offs.o[k] = k < A.ndiag ? A.off[k] : 0;
    const Chunks c = sdia_chunks<TX>(A);
    hipError_t e;
    if (sdia_rows<TX>(A) == 2)
        e = launch_k(k_spmv_sdia_wide<TV, TX, DOT, 2>, c.grid, kBlock, 0, s, ev2, A.n, c.per,
                     A.ndiag, offs, vals, (const TX *)p, (TX *)q, bc, bit, sc, part);
    else
        e = launch_k(k_spmv_sdia_wide<TV, TX, DOT, 1>, c.grid, kBlock, 0, s, ev2, A.n, c.per,
                     A.ndiag, offs, vals, (const TX *)p, (TX *)q, bc, bit, sc, part);
    return e == hipSuccess ? c.grid : -1;
}

template <typename TV, typename TX, bool DOT, int M = 1>
int sdia_dispatch(const DevMatrix &A, const TV *vals, const void *p, void *q, const uint8_t *bc,
                  int bit, const Scalars *sc, double *part, hipStream_t s, hipEvent_t *ev2)
{
    if constexpr (M <= kMaxDiag) {
        if (A.ndiag == M)
            return sdia_launch<TV, TX, DOT, M>(A, vals, p, q, bc, bit, sc, part, s, ev2);
        return sdia_dispatch<TV, TX, DOT, M + 1>(A, vals, p, q, bc, bit, sc, part, s, ev2);
    }
    if (A.ndiag > kMaxDiag && A.ndiag <= kMaxDiagWide && !A.unit)
        return sdia_wide_launch<TV, TX, DOT>(A, vals, p, q, bc, bit, sc, part, s, ev2);
    return -1;
}

// Launches q = A p (+ per-block partials of p^T q when DOT); returns the
// grid, i.e. the number of partials written (-1 if the launch failed).
// ev2: optional event pair recorded by the dispatch (kernel duration).
// ---------------------------------------------------------------------------
// Matrix-free bricks: y = (c_mass M + c_stiff K_nu) x element by element
// (the forms of Sec. 5 on Q1 / Q2 bricks with the tensor Gauss rule of
// order + 1 points per direction, the element the trilinear image of the
// reference cube through its corners).  With u = sum_b N_b x_b,
//   y_a = sum_g [ N_a(g) w det c_mass u(g)
//                 + sum_s dN_a/ds_s(g) w c_stiff sum_d adj(J)_sd nu_d (grad u)_d ],
// (grad u)_d = sum_s du/ds_s adj(J)_sd / det: the element matrix of the
// assembled operator applied to x_e, evaluated by sum factorisation (the
// tensor-product basis contracted one direction at a time, forward to the
// Gauss points and back).  One thread per Gauss point / local node, an
// element per (order+1)^3 lanes of a wavefront, the contractions through
// LDS.  Element results go to a scratch array at node-ordered positions (a
// node's contributions contiguous, in ascending element order); a second
// kernel sums each node's run (deterministic), zeroes Dirichlet rows and
// forms the p^T q partials.
// ---------------------------------------------------------------------------
struct MfTables {
    double V[3][3], D[3][3];     // basis a at point g: value, derivative
    double LV[2][3], LD[2][3];   // trilinear corner basis
    double gw[3];                // Gauss weights
    double coef[5];              // c_mass, c_stiff, nu_x, nu_y, nu_z
};

// Exchange through LDS between the lanes of one wavefront: its LDS
// operations complete in program order, so only the compiler must keep the
// reads after the writes (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_mf_element(int64_t ne,
                                                       const int32_t *__restrict__ nodes,
                                                       const double *__restrict__ corner,
                                                       const int32_t *__restrict__ pos,
                                                       const double *__restrict__ x, MfTables T,
                                                       double *__restrict__ Y,
                                                       const Scalars *__restrict__ sc)
{
    constexpr int Q = P + 1, NL = Q * Q * Q, EW = 64 / NL, EB = (kBlock / 64) * EW;
    if (sc && sc->stop) return;
    __shared__ double sV[3][3], sD[3][3], sLV[2][3], sLD[2][3], sW[3];
    __shared__ double a0[EB][NL], a1[EB][NL], a2[EB][NL], a3[EB][NL];
    __shared__ double b0[EB][NL], b1[EB][NL], b2[EB][NL];
    __shared__ double sX[EB][24];
    if (threadIdx.x < 9) {
        sV[threadIdx.x / 3][threadIdx.x % 3] = T.V[threadIdx.x / 3][threadIdx.x % 3];
        sD[threadIdx.x / 3][threadIdx.x % 3] = T.D[threadIdx.x / 3][threadIdx.x % 3];
    } else if (threadIdx.x < 15) {
        const int k = threadIdx.x - 9;
        sLV[k / 3][k % 3] = T.LV[k / 3][k % 3];
        sLD[k / 3][k % 3] = T.LD[k / 3][k % 3];
    } else if (threadIdx.x < 18) {
        sW[threadIdx.x - 15] = T.gw[threadIdx.x - 15];
    }
    const int lane = threadIdx.x & 63;
    const int slot = lane / NL, t = lane - slot * NL;
    const int es = (threadIdx.x >> 6) * EW + slot;   // element slot of the block
    const bool on = slot < EW;
    const int t0 = t % Q, t1 = (t / Q) % Q, t2 = t / (Q * Q);
    const double cm = T.coef[0], cs = T.coef[1];
    const double nu[3] = {T.coef[2], T.coef[3], T.coef[4]};
    __syncthreads();   // the tables; below, every element lives in one wavefront
    // the next group's x values and corners are loaded into registers while
    // the current group computes (a workgroup takes several groups in turn)
    constexpr int NC = (24 + NL - 1) / NL;   // corner values per lane
    const int64_t stride = (int64_t)gridDim.x * EB;
    double px = 0.0, pc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) pc[k] = 0.0;
    auto fetch = [&](int64_t e) {
        if (on && e < ne) {
            px = x[nodes[e * NL + t]];
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (t + k * NL < 24) pc[k] = corner[e * 24 + t + k * NL];
        }
    };
    fetch((int64_t)blockIdx.x * EB + es);
    for (int64_t e0 = (int64_t)blockIdx.x * EB; e0 < ne; e0 += stride) {
        const int64_t e = e0 + es;
        const bool act = on && e < ne;
        int32_t out = 0;
        if (act) {
            a0[es][t] = px;
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (t + k * NL < 24) sX[es][t + k * NL] = pc[k];
            out = pos[e * NL + t];
        }
        fetch(e + stride);
        wave_lds_sync();
        // forward, direction 0: thread (g0 = t0, a1 = t1, a2 = t2)
        if (act) {
            double v = 0.0, d = 0.0;
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const double xa = a0[es][a + Q * t1 + Q * Q * t2];
                v += sV[a][t0] * xa;
                d += sD[a][t0] * xa;
            }
            b0[es][t] = v;
            b1[es][t] = d;
        }
        wave_lds_sync();
        // direction 1: thread (g0, g1 = t1, a2)
        if (act) {
            double vv = 0.0, vd = 0.0, dv = 0.0;
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int k = t0 + Q * a + Q * Q * t2;
                vv += sV[a][t1] * b0[es][k];
                vd += sD[a][t1] * b0[es][k];
                dv += sV[a][t1] * b1[es][k];
            }
            a1[es][t] = vv;
            a2[es][t] = vd;
            a3[es][t] = dv;
        }
        wave_lds_sync();
        // direction 2, then the point's geometry and fluxes: thread g = t
        if (act) {
            double u = 0.0, us[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int k = t0 + Q * t1 + Q * Q * a;
                u += sV[a][t2] * a1[es][k];
                us[2] += sD[a][t2] * a1[es][k];
                us[1] += sV[a][t2] * a2[es][k];
                us[0] += sV[a][t2] * a3[es][k];
            }
            // J[r][d] = d x_r / d s_d from the 8 corners
            double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int c0 = c & 1, c1 = (c >> 1) & 1, c2 = c >> 2;
                const double g0 = sLD[c0][t0] * sLV[c1][t1] * sLV[c2][t2];
                const double g1 = sLV[c0][t0] * sLD[c1][t1] * sLV[c2][t2];
                const double g2 = sLV[c0][t0] * sLV[c1][t1] * sLD[c2][t2];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const double X = sX[es][3 * c + r];
                    J[r][0] += X * g0;
                    J[r][1] += X * g1;
                    J[r][2] += X * g2;
                }
            }
            double A[3][3];
            A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
            const double w = sW[t0] * sW[t1] * sW[t2];
            const double inv = 1.0 / det;
            double f[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                f[d] = nu[d] * ((us[0] * A[0][d] + us[1] * A[1][d] + us[2] * A[2][d]) * inv);
            // mass and reference fluxes at the point (arrays free since the
            // forward pass of direction 1): M -> b0, F_0 -> b1, F_1 -> b2, F_2 -> a0
            b0[es][t] = w * det * cm * u;
            b1[es][t] = w * cs * (A[0][0] * f[0] + A[0][1] * f[1] + A[0][2] * f[2]);
            b2[es][t] = w * cs * (A[1][0] * f[0] + A[1][1] * f[1] + A[1][2] * f[2]);
            a0[es][t] = w * cs * (A[2][0] * f[0] + A[2][1] * f[1] + A[2][2] * f[2]);
        }
        wave_lds_sync();
        // back, direction 2: thread (g0, g1, a2 = t2)
        if (act) {
            double ra = 0.0, rb = 0.0, rc = 0.0;
#pragma unroll
            for (int g = 0; g < Q; ++g) {
                const int k = t0 + Q * t1 + Q * Q * g;
                ra += sV[t2][g] * b0[es][k] + sD[t2][g] * a0[es][k];
                rb += sV[t2][g] * b2[es][k];
                rc += sV[t2][g] * b1[es][k];
            }
            a1[es][t] = ra;
            a2[es][t] = rb;
            a3[es][t] = rc;
        }
        wave_lds_sync();
        // direction 1: thread (g0, a1 = t1, a2)
        if (act) {
            double sa = 0.0, sc2 = 0.0;
#pragma unroll
            for (int g = 0; g < Q; ++g) {
                const int k = t0 + Q * g + Q * Q * t2;
                sa += sV[t1][g] * a1[es][k] + sD[t1][g] * a2[es][k];
                sc2 += sV[t1][g] * a3[es][k];
            }
            b0[es][t] = sa;
            b1[es][t] = sc2;
        }
        wave_lds_sync();
        // direction 0: thread (a0 = t0, a1, a2): the element's y at node t
        if (act) {
            double y = 0.0;
#pragma unroll
            for (int g = 0; g < Q; ++g) {
                const int k = g + Q * t1 + Q * Q * t2;
                y += sV[t0][g] * b0[es][k] + sD[t0][g] * b1[es][k];
            }
            Y[out] = y;
        }
        wave_lds_sync();
    }
}

// y_i = sum of node i's element results (its run of the scratch, ascending
// element order); zero on Dirichlet rows; per-block partials of x^T y
template <bool DOT>
__global__ __launch_bounds__(kBlock) void k_mf_gather(int64_t n, const int64_t *__restrict__ ptr,
                                                      const double *__restrict__ Y,
                                                      const double *__restrict__ x,
                                                      double *__restrict__ y,
                                                      const uint8_t *__restrict__ bc, int bit,
                                                      const Scalars *__restrict__ sc,
                                                      double *__restrict__ part)
{
    if constexpr (DOT) {
        if (sc->stop) return;
    }
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double s = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) s += Y[k];
        if (is_dirichlet(bc, bit, i)) s = 0.0;
        y[i] = s;
        if constexpr (DOT) acc += x[i] * s;
    }
    if constexpr (DOT) {
        double v[1] = {acc};
        store_block_partials<1>(v, part);
    }
}

template <int P, bool DOT>
int mf_launch_p(const DevMatrix &A, const double *x, double *y, const uint8_t *bc, int bit,
                const Scalars *sc, double *part, double *scratch, hipStream_t s,
                hipEvent_t *ev2)
{
    constexpr int NL = (P + 1) * (P + 1) * (P + 1), EB = (kBlock / 64) * (64 / NL);
    MfTables T;
    for (int a = 0; a < 3; ++a)
        for (int g = 0; g < 3; ++g) {
            T.V[a][g] = A.mf_V[a][g];
            T.D[a][g] = A.mf_D[a][g];
        }
    for (int a = 0; a < 2; ++a)
        for (int g = 0; g < 3; ++g) {
            T.LV[a][g] = A.mf_LV[a][g];
            T.LD[a][g] = A.mf_LD[a][g];
        }
    for (int g = 0; g < 3; ++g) T.gw[g] = A.mf_gw[g];
    for (int k = 0; k < 5; ++k) T.coef[k] = A.mf_coef[k];
    // about two workgroups per SIMD's share of the chip at a time, each taking
    // several groups of elements in turn (the loads of the next overlap)
    const int64_t blocks = (A.mf_ne + EB - 1) / EB;
    const int Ge = (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 2048));
    const int Gg = stream_grid(A.n);
    hipEvent_t e1[2] = {ev2 ? ev2[0] : nullptr, nullptr};
    hipEvent_t e2[2] = {nullptr, ev2 ? ev2[1] : nullptr};
    if (launch_k(k_mf_element<P>, Ge, kBlock, 0, s, ev2 ? e1 : nullptr, A.mf_ne,
                 (const int32_t *)A.mf_nodes, (const double *)A.mf_corner,
                 (const int32_t *)A.mf_pos, x, T, scratch,
                 DOT ? sc : (const Scalars *)nullptr) != hipSuccess)
        return -1;
    if (launch_k(k_mf_gather<DOT>, Gg, kBlock, 0, s, ev2 ? e2 : nullptr, A.n,
                 (const int64_t *)A.mf_ptr, (const double *)scratch, x, y, bc, bit, sc,
                 part) != hipSuccess)
        return -1;
    return Gg;
}

// Matrix-free product (FP64 only); returns the number of partials, -1 on a
// failed launch or without scratch.
template <bool DOT>
int mf_launch(const DevMatrix &A, const double *x, double *y, const uint8_t *bc, int bit,
              const Scalars *sc, double *part, double *scratch, hipStream_t s, hipEvent_t *ev2)
{
    if (!scratch) {
        set_error("matrix-free product without its element scratch");
        return -1;
    }
    if (A.mf_order == 1) return mf_launch_p<1, DOT>(A, x, y, bc, bit, sc, part, scratch, s, ev2);
    return mf_launch_p<2, DOT>(A, x, y, bc, bit, sc, part, scratch, s, ev2);
}

template <typename TV, typename TX, bool DOT>
int spmv_dispatch(const DevMatrix &A, const void *p, void *q, const uint8_t *bc, int bit,
                  const Scalars *sc, double *part, hipStream_t s, hipEvent_t *ev2 = nullptr,
                  double *mf_scratch = nullptr)
{
    const bool f32 = std::is_same<TV, float>::value;
    if (A.fmt == HNS_MATRIX_FREE) {
        if constexpr (std::is_same<TV, double>::value && std::is_same<TX, double>::value)
            return mf_launch<DOT>(A, (const double *)p, (double *)q, bc, bit, sc, part,
                                  mf_scratch, s, ev2);
        set_error("matrix-free operators compute FP64 products only");
        return -1;
    }
    if (A.fmt == HNS_FMT_SDIA) {
        const TV *vd = f32 ? (const TV *)(const void *)A.dia32 : (const TV *)(const void *)A.dia;
        return sdia_dispatch<TV, TX, DOT>(A, vd, p, q, bc, bit, sc, part, s, ev2);
    }
    const int G = spmv_grid(A);
    const TV *vs = f32 ? (const TV *)(const void *)A.sval32 : (const TV *)(const void *)A.sval;
    const TV *vc = f32 ? (const TV *)(const void *)A.val32 : (const TV *)(const void *)A.val;
    hipError_t e;
    if (A.fmt == HNS_FMT_SELL)
        e = launch_k(k_spmv_sell<TV, TX, DOT>, G, kBlock, 0, s, ev2, A.n, A.nslices,
                     A.slice_ptr, A.scol, vs, (const TX *)p, (TX *)q, bc, bit, sc, part);
    else
        e = launch_k(k_spmv_csr<TV, TX, DOT>, G, kBlock, 0, s, ev2, A.n, A.rowptr, A.col, vc,
                     (const TX *)p, (TX *)q, bc, bit, sc, part);
    return e == hipSuccess ? G : -1;
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }


// Event pairs of a timed iteration: ev[0..1] SpMV, ev[2..3] update,
// ev[4..5] direction update (each recorded by its kernel's dispatch).
// k_pupdate_line_x over the n rows: p and z are workspace vectors (16-byte
// aligned), x may be a row of a caller's array at an 8-byte offset, in which
// case one element per thread.  G_in: number of update partials.
template <typename T>
hns_status launch_pupdate_line_x(const IterArgs &a, int parity, int G_in, hipStream_t s,
                                 hipEvent_t *ev2)
{
    constexpr int V = 16 / sizeof(T);
    double *P2 = a.partials + kPartUpdate;
    if (aligned16(a.x)) {
        const Chunks cp = chunks(a.n / V, (int64_t)kBlock * a.A->vec_packs(), kBlock);
        HNS_TRY_HIP(launch_k(k_pupdate_line_x<T, V>, cp.grid, kBlock, 0, s, ev2, a.n, cp.per,
                             (T *)a.x, (T *)a.p, (const T *)a.z, a.sc, (const double *)P2, G_in,
                             parity, a.token));
    } else {
        const Chunks cp = chunks(a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
        HNS_TRY_HIP(launch_k(k_pupdate_line_x<T, 1>, cp.grid, kBlock, 0, s, ev2, a.n, cp.per,
                             (T *)a.x, (T *)a.p, (const T *)a.z, a.sc, (const double *)P2, G_in,
                             parity, a.token));
    }
    return HNS_OK;
}

// T = double: FP64 iteration; T = float: FP32 matrix, vectors and factors
// (inner iterations of mixed precision)
template <typename T>
hns_status line_iteration(const IterArgs &a, int parity, hipStream_t s, hipEvent_t *ev)
{
    const uint8_t *bc = a.bit < 0 ? nullptr : a.bc;
    double *P1 = a.partials + kPartSpmv;
    double *P2 = a.partials + kPartUpdate;
    const int L = a.line_len;
    const int NC = line_cols_per_block(L);
    const int Gl = line_grid(a.n, L);
    const int Gs = spmv_dispatch<T, T, true>(*a.A, a.p, a.q, bc, a.bit, a.sc, P1, s,
                                             ev ? ev : nullptr, a.mf);
    if (Gs < 0) return spmv_failed("spmv");
    HNS_TRY_HIP(launch_k(k_update_line<T>, Gl, kBlock, (size_t)4 * NC * L * sizeof(T), s,
                         ev ? ev + 2 : nullptr, a.n, L, NC, (T *)a.r, (const T *)a.q, (T *)a.z,
                         (const T *)a.lfac, a.sc, (const double *)P1, Gs, P2, parity, a.token));
    HNS_TRY(launch_pupdate_line_x<T>(a, parity, Gl, s, ev ? ev + 4 : nullptr));
    return check_launch("line-preconditioned cg iteration");
}

// z = M^-1 r with the IC(0) factor: one launch per colour and direction,
// rows taken 8 entries at a time where a colour's rows have at most 8, else
// 16 at a time
hns_status ic0_apply(const IC0Dev &F, const double *r, double *y, double *z, hipStream_t s)
{
    for (int c = 0; c < F.ncolors; ++c) {
        const int64_t r0 = F.cstart[c], r1 = F.cstart[c + 1];
        if (r1 <= r0) continue;
        const int32_t *col = F.lcol + F.lbase[c];
        const double *val = F.lval + F.lbase[c];
        if (F.lwidth[c] <= 8)
            k_ic_forward<8><<<stream_grid(r1 - r0), kBlock, 0, s>>>(r0, r1, F.perm, F.lptr, col,
                                                                     val, F.diag, r, y);
        else
            k_ic_forward<16><<<stream_grid(r1 - r0), kBlock, 0, s>>>(r0, r1, F.perm, F.lptr,
                                                                      col, val, F.diag, r, y);
    }
    for (int c = F.ncolors - 1; c >= 0; --c) {
        const int64_t r0 = F.cstart[c], r1 = F.cstart[c + 1];
        if (r1 <= r0) continue;
        const int32_t *col = F.ucol + F.ubase[c];
        const double *val = F.uval + F.ubase[c];
        if (F.uwidth[c] <= 8)
            k_ic_backward<8><<<stream_grid(r1 - r0), kBlock, 0, s>>>(r0, r1, F.perm, F.uptr,
                                                                      col, val, F.diag, y, z);
        else
            k_ic_backward<16><<<stream_grid(r1 - r0), kBlock, 0, s>>>(r0, r1, F.perm, F.uptr,
                                                                       col, val, F.diag, y, z);
    }
    return check_launch("ic0 triangular solves");
}

// Event pairs as in line_iteration; the triangular solves are not timed.
hns_status ic0_iteration(const IterArgs &a, int parity, hipStream_t s, hipEvent_t *ev)
{
    const uint8_t *bc = a.bit < 0 ? nullptr : a.bc;
    double *P1 = a.partials + kPartSpmv;
    double *P2 = a.partials + kPartUpdate;
    const bool vec = aligned16(a.x) && aligned16(a.r) && aligned16(a.p) && aligned16(a.q) &&
                     aligned16(a.z);
    const Chunks cu = chunks(vec ? a.n / 2 : a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
    const int Gs = spmv_dispatch<double, double, true>(*a.A, a.p, a.q, bc, a.bit, a.sc, P1, s,
                                                       ev ? ev : nullptr, a.mf);
    if (Gs < 0) return spmv_failed("spmv");
    if (vec) {
        HNS_TRY_HIP(launch_k(k_update_noz<2>, cu.grid, kBlock, 0, s, ev ? ev + 2 : nullptr, a.n,
                             cu.per, (double *)a.r, (const double *)a.q, a.sc,
                             (const double *)P1, Gs, parity, a.token));
    } else {
        HNS_TRY_HIP(launch_k(k_update_noz<1>, cu.grid, kBlock, 0, s, ev ? ev + 2 : nullptr, a.n,
                             cu.per, (double *)a.r, (const double *)a.q, a.sc,
                             (const double *)P1, Gs, parity, a.token));
    }
    double *z = (double *)a.z;
    HNS_TRY(ic0_apply(*a.ic, (const double *)a.r, a.y, z, s));
    if (vec)
        k_dot_rz<2><<<cu.grid, kBlock, 0, s>>>(a.n, cu.per, (const double *)a.r, z, a.sc, P2);
    else
        k_dot_rz<1><<<cu.grid, kBlock, 0, s>>>(a.n, cu.per, (const double *)a.r, z, a.sc, P2);
    HNS_TRY(check_launch("dot r.z"));
    HNS_TRY(launch_pupdate_line_x<double>(a, parity, cu.grid, s, ev ? ev + 4 : nullptr));
    return check_launch("ic0-preconditioned cg iteration");
}

template <typename TV, typename TX, typename TD>
hns_status iteration_impl(const IterArgs &a, int parity, hipStream_t s, hipEvent_t *ev)
{
    constexpr int V = 16 / sizeof(TX);  // elements per 16-byte pack
    const uint8_t *bc = a.bit < 0 ? nullptr : a.bc;
    double *P1 = a.partials + kPartSpmv;
    double *P2 = a.partials + kPartUpdate;
    // packs need every operand 16-byte aligned (a row of a 3 x n array with n
    // odd is not): fall back to one element per thread then
    const bool vec = aligned16(a.x) && aligned16(a.r) && aligned16(a.p) && aligned16(a.q) &&
                     aligned16(a.dinv);
    const Chunks cu = chunks(vec ? a.n / V : a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
    const int Gs = spmv_dispatch<TV, TX, true>(*a.A, a.p, a.q, bc, a.bit, a.sc, P1, s,
                                               ev ? ev : nullptr, a.mf);
    if (Gs < 0) return spmv_failed("spmv");
    hipEvent_t *eu = ev ? ev + 2 : nullptr, *ep = ev ? ev + 4 : nullptr;
    if (vec) {
        HNS_TRY_HIP(launch_k(k_update<TX, TD, V>, cu.grid, kBlock, 0, s, eu, a.n, cu.per,
                             (TX *)a.r, (const TX *)a.q, (const TD *)a.dinv, a.sc,
                             (const double *)P1, Gs, P2, parity, a.token));
        HNS_TRY_HIP(launch_k(k_pupdate_x<TX, TD, V>, cu.grid, kBlock, 0, s, ep, a.n, cu.per,
                             (TX *)a.x, (TX *)a.p, (const TX *)a.r, (const TD *)a.dinv, a.sc,
                             (const double *)P2, cu.grid, parity, a.token));
    } else {
        HNS_TRY_HIP(launch_k(k_update<TX, TD, 1>, cu.grid, kBlock, 0, s, eu, a.n, cu.per,
                             (TX *)a.r, (const TX *)a.q, (const TD *)a.dinv, a.sc,
                             (const double *)P1, Gs, P2, parity, a.token));
        HNS_TRY_HIP(launch_k(k_pupdate_x<TX, TD, 1>, cu.grid, kBlock, 0, s, ep, a.n, cu.per,
                             (TX *)a.x, (TX *)a.p, (const TX *)a.r, (const TD *)a.dinv, a.sc,
                             (const double *)P2, cu.grid, parity, a.token));
    }
    return check_launch("cg iteration");
}

// Point-Jacobi iteration of CG on the Jacobi-scaled operator (a.A unit
// diagonal, FP64 or FP32 values and vectors): the same three kernels without
// the reads of D^-1; a.wjac (diag(A), FP32) weighs the unscaled residual norm.
template <typename T>
bool scaled_vec(const IterArgs &a)
{
    return aligned16(a.x) && aligned16(a.r) && aligned16(a.p) && aligned16(a.q) &&
           aligned16(a.wjac);
}

template <typename T>
hns_status scaled_values(const IterArgs &a)
{
    if ((sizeof(T) == 4 ? (const void *)a.A->dia32 : (const void *)a.A->dia) == nullptr) {
        set_error("the Jacobi-scaled operator has no values in this precision");
        return HNS_ERR_INVALID;
    }
    return HNS_OK;
}

// r -= alpha q with the partials of the scaled recurrence (Gs product partials in)
template <typename T>
hns_status launch_update_scaled(const IterArgs &a, int parity, int Gs, hipStream_t s,
                                hipEvent_t *eu)
{
    constexpr int V = 16 / sizeof(T);
    double *P1 = a.partials + kPartSpmv;
    double *P2 = a.partials + kPartUpdate;
    const bool vec = scaled_vec<T>(a);
    const Chunks cu = chunks(vec ? a.n / V : a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
    if (vec)
        HNS_TRY_HIP(launch_k(k_update<T, float, V, true>, cu.grid, kBlock, 0, s, eu, a.n, cu.per,
                             (T *)a.r, (const T *)a.q, a.wjac, a.sc, (const double *)P1, Gs, P2,
                             parity, a.token));
    else
        HNS_TRY_HIP(launch_k(k_update<T, float, 1, true>, cu.grid, kBlock, 0, s, eu, a.n, cu.per,
                             (T *)a.r, (const T *)a.q, a.wjac, a.sc, (const double *)P1, Gs, P2,
                             parity, a.token));
    return HNS_OK;
}

template <typename T>
hns_status iteration_scaled(const IterArgs &a, int parity, hipStream_t s, hipEvent_t *ev)
{
    constexpr int V = 16 / sizeof(T);
    const uint8_t *bc = a.bit < 0 ? nullptr : a.bc;
    double *P1 = a.partials + kPartSpmv;
    double *P2 = a.partials + kPartUpdate;
    const bool vec = scaled_vec<T>(a);
    HNS_TRY(scaled_values<T>(a));
    const Chunks cu = chunks(vec ? a.n / V : a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
    const int Gs = spmv_dispatch<T, T, true>(*a.A, a.p, a.q, bc, a.bit, a.sc, P1, s,
                                             ev ? ev : nullptr, a.mf);
    if (Gs < 0) return spmv_failed("spmv (Jacobi-scaled)");
    hipEvent_t *eu = ev ? ev + 2 : nullptr, *ep = ev ? ev + 4 : nullptr;
    HNS_TRY(launch_update_scaled<T>(a, parity, Gs, s, eu));
    if (vec)
        HNS_TRY_HIP(launch_k(k_pupdate_x<T, float, V, true>, cu.grid, kBlock, 0, s, ep, a.n,
                             cu.per, (T *)a.x, (T *)a.p, (const T *)a.r, (const float *)nullptr,
                             a.sc, (const double *)P2, cu.grid, parity, a.token));
    else
        HNS_TRY_HIP(launch_k(k_pupdate_x<T, float, 1, true>, cu.grid, kBlock, 0, s, ep, a.n,
                             cu.per, (T *)a.x, (T *)a.p, (const T *)a.r, (const float *)nullptr,
                             a.sc, (const double *)P2, cu.grid, parity, a.token));
    return check_launch("cg iteration (Jacobi-scaled)");
}

// The fused direction update + product for M upper diagonals (dispatch on M)
template <typename T, int M = 1>
hipError_t launch_sdia_dir(const IterArgs &a, const T *po, T *pn, uint32_t token, int parity,
                           int G_in, hipStream_t s, hipEvent_t *ev2, int *grid)
{
    if constexpr (M <= kMaxDiag) {
        if (a.A->ndiag != M)
            return launch_sdia_dir<T, M + 1>(a, po, pn, token, parity, G_in, s, ev2, grid);
        DiaOffsets offs;
        for (int k = 0; k < kMaxDiag; ++k) offs.o[k] = k < a.A->ndiag ? a.A->off[k] : 0;
        const Chunks c = sdia_chunks<T>(*a.A);
        *grid = c.grid;
        const T *dia = sizeof(T) == 4 ? (const T *)a.A->dia32 : (const T *)a.A->dia;
        auto k = sdia_rows<T>(*a.A) == 2 ? k_sdia_dir<T, M, 2> : k_sdia_dir<T, M, 1>;
        return launch_k(k, c.grid, kBlock, 0, s, ev2, a.n, c.per, offs, dia,
                        po, (const T *)a.r, (T *)a.x, pn, (T *)a.p, (T *)a.q,
                        a.bit < 0 ? (const uint8_t *)nullptr : a.bc, a.bit, a.sc,
                        (const double *)(a.partials + kPartUpdate), G_in,
                        a.partials + kPartSpmv, parity, token);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T>
hns_status scaled_fused_step_t(const IterArgs &a, const void *po, void *pn, uint32_t prev_token,
                               int prev_parity, int parity, hipStream_t s, hipEvent_t *ev)
{
    HNS_TRY(scaled_values<T>(a));
    int Gs = -1;
    if (!po) {
        // the chunk's first iteration: p is complete, the plain product
        Gs = spmv_dispatch<T, T, true>(*a.A, a.p, a.q, a.bit < 0 ? nullptr : a.bc, a.bit, a.sc,
                                       a.partials + kPartSpmv, s, ev, a.mf);
        if (Gs < 0) return spmv_failed("spmv (Jacobi-scaled)");
    } else {
        constexpr int V = 16 / sizeof(T);
        const bool vec = scaled_vec<T>(a);
        const Chunks cu = chunks(vec ? a.n / V : a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
        if (launch_sdia_dir<T>(a, (const T *)po, (T *)pn, prev_token, prev_parity, cu.grid, s, ev,
                               &Gs) != hipSuccess)
            return spmv_failed("direction update + spmv (Jacobi-scaled)");
    }
    HNS_TRY(launch_update_scaled<T>(a, parity, Gs, s, ev ? ev + 2 : nullptr));
    return check_launch("fused cg iteration (Jacobi-scaled)");
}

template <typename T>
hns_status scaled_fused_close_t(const IterArgs &a, const void *po, uint32_t token, int parity,
                                hipStream_t s)
{
    constexpr int V = 16 / sizeof(T);
    const bool vec = scaled_vec<T>(a);
    const Chunks cu = chunks(vec ? a.n / V : a.n, (int64_t)kBlock * a.A->vec_packs(), kBlock);
    const Chunks c = sdia_chunks<T>(*a.A);
    HNS_TRY_HIP(launch_k(k_sdia_dir_close<T>, c.grid, kBlock, 0, s, nullptr, a.n, c.per,
                         (const T *)po, (const T *)a.r, (T *)a.x, (T *)a.p, a.sc,
                         (const double *)(a.partials + kPartUpdate), cu.grid, parity, token));
    return check_launch("direction update (Jacobi-scaled, end of chunk)");
}

}  // namespace

int stream_grid(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g < 1) g = 1;
    if (g >= 8) g &= ~int64_t(7);
    return (int)g;
}

int spmv_grid(const DevMatrix &A)
{
    int64_t units = (A.fmt == HNS_FMT_SELL)   ? (A.nslices + 3) / 4
                    : (A.fmt == HNS_FMT_SDIA) ? (A.n + kBlock - 1) / kBlock
                                              : (A.n + 15) / 16;
    int64_t g = units < kMaxGrid ? units : kMaxGrid;
    if (g < 1) g = 1;
    if (g >= 8) g &= ~int64_t(7);
    return (int)g;
}

Chunks chunks(int64_t units, int64_t per, int64_t quantum, int64_t cap)
{
    per = per < quantum ? quantum : (per + quantum - 1) / quantum * quantum;
    int64_t g = (units + per - 1) / per;
    if (g > cap) {
        // more units per block (whole quanta) to stay within the slots
        per = ((units + cap - 1) / cap + quantum - 1) / quantum * quantum;
        g = (units + per - 1) / per;
    }
    if (g < 1) g = 1;
    if (g >= 8) g = (g + 7) / 8 * 8;   // the few extra blocks find no units
    return {(int)g, per};
}

hns_status launch_spmv_plain(const DevMatrix &A, bool fp32, const void *p, void *q,
                             const uint8_t *bc, int bit, hipStream_t s, double *mf_scratch)
{
    if (bit < 0) bc = nullptr;
    int G;
    if (fp32)
        G = spmv_dispatch<float, float, false>(A, p, q, bc, bit, nullptr, nullptr, s);
    else
        G = spmv_dispatch<double, double, false>(A, p, q, bc, bit, nullptr, nullptr, s, nullptr,
                                                 mf_scratch);
    if (G < 0 && A.fmt == HNS_MATRIX_FREE) return HNS_ERR_INVALID;   // the reason is set
    return check_launch("spmv");
}

int line_cols_per_block(int line_len)
{
    if (line_len < 1) return 0;
    int nc = kLineLds / (4 * (int)sizeof(double) * line_len);
    return nc > 64 ? 64 : nc;   // one wavefront runs the recurrences
}

int line_grid(int64_t n, int line_len)
{
    const int nc = line_cols_per_block(line_len);
    if (nc < 1) return 0;
    const int64_t cols = n / line_len;
    int64_t g = (cols + nc - 1) / nc;
    if (g >= 8) g = (g + 7) / 8 * 8;
    return (int)g;
}

template <typename T>
static hns_status init_line_t(int64_t n, int line_len, T *r, T *p, const T *lfac, bool singular,
                              bool bb_from_rr, Scalars *sc, double *partials, hipStream_t s)
{
    const int NC = line_cols_per_block(line_len);
    const int G = line_grid(n, line_len);
    k_init_line<T><<<G, kBlock, (size_t)4 * NC * line_len * sizeof(T), s>>>(
        n, line_len, NC, r, p, lfac, singular ? 1 : 0, sc, partials + kPartMisc);
    HNS_TRY(check_launch("init_line"));
    k_fin_start<<<1, kBlock, 0, s>>>(partials + kPartMisc, G, sc, bb_from_rr ? 1 : 0);
    return check_launch("fin_start");
}

hns_status launch_init_line(int64_t n, int line_len, double *r, double *p, const double *lfac,
                            bool singular, bool bb_from_rr, Scalars *sc, double *partials,
                            hipStream_t s)
{
    return init_line_t<double>(n, line_len, r, p, lfac, singular, bb_from_rr, sc, partials, s);
}

hns_status launch_init_line(int64_t n, int line_len, float *r, float *p, const float *lfac,
                            bool singular, bool bb_from_rr, Scalars *sc, double *partials,
                            hipStream_t s)
{
    return init_line_t<float>(n, line_len, r, p, lfac, singular, bb_from_rr, sc, partials, s);
}

hns_status launch_replace_line(int64_t n, int line_len, const double *r64, float *r, float *z,
                               float *p, const float *lfac, Scalars *sc, double *partials,
                               int parity, int vec_it, hipStream_t s)
{
    const int NC = line_cols_per_block(line_len);
    const int G = line_grid(n, line_len);
    double *P2 = partials + kPartUpdate;
    k_replace_line<float><<<G, kBlock, (size_t)4 * NC * line_len * sizeof(float), s>>>(
        n, line_len, NC, r64, r, z, lfac, P2);
    HNS_TRY(check_launch("replace_line"));
    // p and z are workspace vectors (16-byte aligned)
    const Chunks cp = chunks(n / 4, (int64_t)kBlock * vec_it, kBlock);
    k_pdir_line<float, 4><<<cp.grid, kBlock, 0, s>>>(n, cp.per, p, z, sc, P2, G, parity);
    return check_launch("direction (line replacement)");
}

hns_status launch_init_ic0(int64_t n, const IC0Dev &F, const double *r, double *p, double *z,
                           double *y, Scalars *sc, double *partials, hipStream_t s)
{
    HNS_TRY(ic0_apply(F, r, y, z, s));
    k_init_from_z<<<stream_grid(n), kBlock, 0, s>>>(n, r, z, p, sc, partials + kPartMisc);
    HNS_TRY(check_launch("init_from_z"));
    k_fin_start<<<1, kBlock, 0, s>>>(partials + kPartMisc, stream_grid(n), sc, 0);
    return check_launch("init_ic0");
}

// ---------------------------------------------------------------------------
// Small systems: a chunk of CG iterations in one workgroup
// ---------------------------------------------------------------------------
constexpr int kSmallBlock = 1024;

// The operator as the small kernel reads it (passed by value)
struct SmallMat {
    int64_t n;
    uint32_t fmt;
    int ndiag;
    int32_t off[kMaxDiagWide];
    const int32_t *rowptr, *col;       // CSR
    const int32_t *slice_ptr, *scol;   // sliced ELL
};

// Sum over the 16 wavefronts of the workgroup; every thread reads the 16
// wave sums in the same order, so all obtain bit-identical totals.  No
// barrier follows the reads: each call site of an iteration has its own
// slots, and the block passes at least one other barrier before that site
// writes them again.
template <int NV>
__device__ __forceinline__ void small_block_sum(double (&v)[NV], double *lds)
{
    constexpr int NW = kSmallBlock / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum_dpp(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * NW + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += lds[k * NW + w];
        v[k] = t;
    }
}

// Row i of A p: diagonal storage in the order main, (upper, lower) per offset
// (as the multi-block kernels); sliced ELL and CSR in storage order.
template <typename TV, typename TX>
__device__ __forceinline__ TX small_row(const SmallMat &A, const TV *__restrict__ vals,
                                        const TX *__restrict__ p, int64_t i)
{
    const int64_t n = A.n;
    if (A.fmt == HNS_FMT_SDIA) {
        TX sum = (TX)vals[i] * p[i];
        for (int k = 0; k < A.ndiag; ++k) {
            const int64_t o = A.off[k];
            const TV *u = vals + (int64_t)(k + 1) * n;
            if (i + o < n) sum += (TX)u[i] * p[i + o];
            if (i >= o) sum += (TX)u[i - o] * p[i - o];
        }
        return sum;
    }
    TX sum = 0;
    if (A.fmt == HNS_FMT_SELL) {
        const int64_t sl = i >> 6;
        const int l = (int)(i & 63);
        const int32_t beg = A.slice_ptr[sl];
        const int32_t w = (A.slice_ptr[sl + 1] - beg) >> 6;
        for (int j = 0; j < w; ++j) sum += (TX)vals[beg + 64 * j + l] * p[A.scol[beg + 64 * j + l]];
        return sum;
    }
    for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) sum += (TX)vals[k] * p[A.col[k]];
    return sum;
}

// `count` iterations; each thread keeps the rows i = t, t + 1024, ... in all
// three phases, so only the product's reads of p at neighbouring rows need
// the barrier at the end of an iteration.  Per element the arithmetic is
// that of k_update and k_pupdate_x.
template <typename TV, typename TX, typename TD>
__global__ __launch_bounds__(kSmallBlock) void k_cg_small(SmallMat A, const TV *__restrict__ vals,
                                                          TX *__restrict__ x, TX *__restrict__ r,
                                                          TX *__restrict__ p, TX *__restrict__ q,
                                                          const TD *__restrict__ dinv,
                                                          const uint8_t *__restrict__ bc, int bit,
                                                          Scalars *__restrict__ sc, int count,
                                                          int parity)
{
    __shared__ double lds[3 * (kSmallBlock / 64)];   // p^T q, then r^T z and r^T r
    if (sc->stop) return;
    const int64_t n = A.n;
    double rho[2] = {sc->rho[0], sc->rho[1]};
    double gamma = sc->gamma, alpha_d = sc->alpha, beta_d = sc->beta, rr = sc->rr;
    const double limit = sc->tol2 * sc->bb;
    int stop = 0, done = 0;
    for (int it = 0; it < count; ++it) {
        double v1[1] = {0.0};
        for (int64_t i = threadIdx.x; i < n; i += kSmallBlock) {
            TX sum = small_row<TV, TX>(A, vals, p, i);
            if (is_dirichlet(bc, bit, i)) sum = 0;
            q[i] = sum;
            v1[0] += (double)p[i] * (double)sum;
        }
        small_block_sum<1>(v1, lds);
        gamma = v1[0];
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            stop = 2;
            break;
        }
        alpha_d = rho[parity] / gamma;
        const TX alpha = (TX)alpha_d;
        double v2[2] = {0.0, 0.0};
        for (int64_t i = threadIdx.x; i < n; i += kSmallBlock) {
            const TX ri = r[i] - alpha * q[i];
            r[i] = ri;
            const TX zi = (TX)dinv[i] * ri;
            v2[0] += (double)ri * (double)zi;
            v2[1] += (double)ri * (double)ri;
        }
        small_block_sum<2>(v2, lds + kSmallBlock / 64);
        const double rho_new = v2[0];
        rr = v2[1];
        const bool bad = !isfinite(rho_new) || !isfinite(rr);
        const bool conv = !bad && rr <= limit;
        beta_d = rho_new / rho[parity];
        const TX beta = (TX)beta_d;
        const bool dir = !(bad || conv);
        for (int64_t i = threadIdx.x; i < n; i += kSmallBlock) {
            const TX pi = p[i];
            x[i] = x[i] + alpha * pi;
            if (dir) p[i] = (TX)dinv[i] * r[i] + beta * pi;
        }
        rho[parity ^ 1] = rho_new;
        parity ^= 1;
        ++done;
        if (!dir) {
            stop = bad ? 2 : 1;
            break;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->rho[0] = rho[0];
        sc->rho[1] = rho[1];
        sc->gamma = gamma;
        sc->alpha = alpha_d;
        sc->beta = beta_d;
        sc->rr = rr;
        sc->iter += done;
        if (stop) sc->stop = stop;
    }
}

// The same chunk for up to 4 kSmallBlock rows: a thread keeps its rows' x,
// r, q and D^-1 in registers and the direction p lives in LDS (the product
// reads it at neighbouring rows), so an iteration touches global memory only
// for the matrix values; x, r and p are loaded at the start of the chunk and
// stored at its end.  Per element and per sum the arithmetic and order are
// those of k_cg_small.
// With VL the matrix values (diagonal storage, (ndiag + 1) n of them) are
// copied into LDS too, ahead of p, and every product reads them there.
template <typename TV, typename TX, typename TD, int ROWS, bool VL>
__global__ __launch_bounds__(kSmallBlock) void k_cg_small_lds(
    SmallMat A, const TV *__restrict__ gvals, TX *__restrict__ x, TX *__restrict__ r,
    TX *__restrict__ p, const TD *__restrict__ dinv, const uint8_t *__restrict__ bc, int bit,
    Scalars *__restrict__ sc, int count, int parity)
{
    extern __shared__ __align__(16) unsigned char small_dyn[];
    const int64_t nv = VL ? (int64_t)(A.ndiag + 1) * A.n : 0;
    const size_t vbytes = ((size_t)nv * sizeof(TV) + 15) & ~size_t(15);
    TV *svals = reinterpret_cast<TV *>(small_dyn);
    TX *sp = reinterpret_cast<TX *>(small_dyn + vbytes);
    __shared__ double lds[3 * (kSmallBlock / 64)];   // p^T q, then r^T z and r^T r
    if (sc->stop) return;
    const int64_t n = A.n;
    if constexpr (VL)
        for (int64_t k = threadIdx.x; k < nv; k += kSmallBlock) svals[k] = gvals[k];
    const TV *vals = VL ? (const TV *)svals : gvals;
    TX xr[ROWS], rv[ROWS], qv[ROWS], dv[ROWS];
    bool dm[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int64_t i = threadIdx.x + (int64_t)k * kSmallBlock;
        xr[k] = rv[k] = qv[k] = dv[k] = (TX)0;
        dm[k] = false;
        if (i < n) {
            xr[k] = x[i];
            rv[k] = r[i];
            dv[k] = (TX)dinv[i];
            dm[k] = is_dirichlet(bc, bit, i);
            sp[i] = p[i];
        }
    }
    __syncthreads();
    double rho[2] = {sc->rho[0], sc->rho[1]};
    double gamma = sc->gamma, alpha_d = sc->alpha, beta_d = sc->beta, rr = sc->rr;
    const double limit = sc->tol2 * sc->bb;
    int stop = 0, done = 0;
    for (int it = 0; it < count; ++it) {
        double v1[1] = {0.0};
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int64_t i = threadIdx.x + (int64_t)k * kSmallBlock;
            if (i < n) {
                TX sum = small_row<TV, TX>(A, vals, sp, i);
                if (dm[k]) sum = 0;
                qv[k] = sum;
                v1[0] += (double)sp[i] * (double)sum;
            }
        }
        small_block_sum<1>(v1, lds);
        gamma = v1[0];
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            stop = 2;
            break;
        }
        alpha_d = rho[parity] / gamma;
        const TX alpha = (TX)alpha_d;
        double v2[2] = {0.0, 0.0};
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int64_t i = threadIdx.x + (int64_t)k * kSmallBlock;
            if (i < n) {
                const TX ri = rv[k] - alpha * qv[k];
                rv[k] = ri;
                const TX zi = dv[k] * ri;
                v2[0] += (double)ri * (double)zi;
                v2[1] += (double)ri * (double)ri;
            }
        }
        small_block_sum<2>(v2, lds + kSmallBlock / 64);
        const double rho_new = v2[0];
        rr = v2[1];
        const bool bad = !isfinite(rho_new) || !isfinite(rr);
        const bool conv = !bad && rr <= limit;
        beta_d = rho_new / rho[parity];
        const TX beta = (TX)beta_d;
        const bool dir = !(bad || conv);
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int64_t i = threadIdx.x + (int64_t)k * kSmallBlock;
            if (i < n) {
                const TX pi = sp[i];
                xr[k] = xr[k] + alpha * pi;
                if (dir) sp[i] = dv[k] * rv[k] + beta * pi;
            }
        }
        rho[parity ^ 1] = rho_new;
        parity ^= 1;
        ++done;
        if (!dir) {
            stop = bad ? 2 : 1;
            break;
        }
        __syncthreads();
    }
    // a thread stores only its own rows, whose p it alone wrote
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        const int64_t i = threadIdx.x + (int64_t)k * kSmallBlock;
        if (i < n) {
            x[i] = xr[k];
            r[i] = rv[k];
            p[i] = sp[i];
        }
    }
    if (threadIdx.x == 0) {
        sc->rho[0] = rho[0];
        sc->rho[1] = rho[1];
        sc->gamma = gamma;
        sc->alpha = alpha_d;
        sc->beta = beta_d;
        sc->rr = rr;
        sc->iter += done;
        if (stop) sc->stop = stop;
    }
}

// LDS a single workgroup may take on gfx950 (160 KB), less the static arrays
constexpr size_t kSmallLdsBytes = 160 * 1024 - 1024;

template <typename TV, typename TX, typename TD, int ROWS, bool VL>
hipError_t launch_small_rows(const SmallMat &A, const TV *v, TX *x, TX *r, TX *p,
                             const TD *dinv, const uint8_t *bc, int bit, Scalars *sc, int count,
                             int parity, size_t shm, hipStream_t s)
{
    auto k = k_cg_small_lds<TV, TX, TD, ROWS, VL>;
    // raised once per instantiation to the largest size it may take
    static std::atomic<bool> raised{false};
    if (shm > 64 * 1024 && !raised.load(std::memory_order_acquire)) {
        const hipError_t e = hipFuncSetAttribute((const void *)k,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)kSmallLdsBytes);
        if (e != hipSuccess) return e;
        raised.store(true, std::memory_order_release);
    }
    hipLaunchKernelGGL(k, dim3(1), dim3(kSmallBlock), shm, s, A, v, x, r, p, dinv, bc, bit, sc,
                       count, parity);
    return hipGetLastError();
}

template <typename TV, typename TX, typename TD, bool VL>
hipError_t launch_small_vl(const SmallMat &A, const TV *v, TX *x, TX *r, TX *p, const TD *dinv,
                           const uint8_t *bc, int bit, Scalars *sc, int count, int parity,
                           size_t shm, hipStream_t s)
{
    switch ((A.n + kSmallBlock - 1) / kSmallBlock) {
    case 1:
        return launch_small_rows<TV, TX, TD, 1, VL>(A, v, x, r, p, dinv, bc, bit, sc, count,
                                                    parity, shm, s);
    case 2:
        return launch_small_rows<TV, TX, TD, 2, VL>(A, v, x, r, p, dinv, bc, bit, sc, count,
                                                    parity, shm, s);
    case 3:
        return launch_small_rows<TV, TX, TD, 3, VL>(A, v, x, r, p, dinv, bc, bit, sc, count,
                                                    parity, shm, s);
    default:
        return launch_small_rows<TV, TX, TD, 4, VL>(A, v, x, r, p, dinv, bc, bit, sc, count,
                                                    parity, shm, s);
    }
}

template <typename TV, typename TX, typename TD>
void launch_small_lds(const SmallMat &A, const TV *v, TX *x, TX *r, TX *p, const TD *dinv,
                      const uint8_t *bc, int bit, Scalars *sc, int count, int parity,
                      hipStream_t s)
{
    // the diagonal storage's values on chip too when they fit beside p
    const size_t pbytes = (size_t)A.n * sizeof(TX);
    const size_t vbytes = ((size_t)(A.ndiag + 1) * A.n * sizeof(TV) + 15) & ~size_t(15);
    if (A.fmt == HNS_FMT_SDIA && vbytes + pbytes <= kSmallLdsBytes &&
        launch_small_vl<TV, TX, TD, true>(A, v, x, r, p, dinv, bc, bit, sc, count, parity,
                                          vbytes + pbytes, s) == hipSuccess)
        return;
    (void)hipGetLastError();
    (void)launch_small_vl<TV, TX, TD, false>(A, v, x, r, p, dinv, bc, bit, sc, count, parity,
                                             pbytes, s);
}

hns_status launch_cg_small(const IterArgs &a, int parity, int count, hipStream_t s)
{
    const DevMatrix &M = *a.A;
    if (a.n > kSmallMaxN || (a.prec != Prec::F64 && a.prec != Prec::F32) || a.lfac || a.ic) {
        set_error("launch_cg_small: unsupported configuration");
        return HNS_ERR_INVALID;
    }
    SmallMat A{};
    A.n = M.n;
    A.fmt = M.fmt;
    A.ndiag = M.fmt == HNS_FMT_SDIA ? M.ndiag : 0;
    for (int k = 0; k < kMaxDiagWide; ++k) A.off[k] = k < A.ndiag ? M.off[k] : 0;
    A.rowptr = M.rowptr;
    A.col = M.col;
    A.slice_ptr = M.slice_ptr;
    A.scol = M.scol;
    const uint8_t *bc = a.bit < 0 ? nullptr : a.bc;
    // up to 4 rows per thread the vectors stay on chip for the whole chunk
    const bool on_chip = a.n <= 4 * (int64_t)kSmallBlock;
    if (a.prec == Prec::F64) {
        const double *v = M.fmt == HNS_FMT_SDIA ? M.dia : M.fmt == HNS_FMT_SELL ? M.sval : M.val;
        if (on_chip)
            launch_small_lds<double, double, double>(A, v, (double *)a.x, (double *)a.r,
                                                     (double *)a.p, (const double *)a.dinv, bc,
                                                     a.bit, a.sc, count, parity & 1, s);
        else
            k_cg_small<double, double, double><<<1, kSmallBlock, 0, s>>>(
                A, v, (double *)a.x, (double *)a.r, (double *)a.p, (double *)a.q,
                (const double *)a.dinv, bc, a.bit, a.sc, count, parity & 1);
    } else {
        const float *v = M.fmt == HNS_FMT_SDIA ? M.dia32 : M.fmt == HNS_FMT_SELL ? M.sval32 : M.val32;
        if (!v) {
            set_error("launch_cg_small: FP32 values not kept");
            return HNS_ERR_INVALID;
        }
        if (on_chip)
            launch_small_lds<float, float, float>(A, v, (float *)a.x, (float *)a.r,
                                                  (float *)a.p, (const float *)a.dinv, bc, a.bit,
                                                  a.sc, count, parity & 1, s);
        else
            k_cg_small<float, float, float><<<1, kSmallBlock, 0, s>>>(
                A, v, (float *)a.x, (float *)a.r, (float *)a.p, (float *)a.q,
                (const float *)a.dinv, bc, a.bit, a.sc, count, parity & 1);
    }
    return check_launch("small-system cg chunk");
}

hns_status launch_iteration(const IterArgs &a, int parity, hipStream_t s, hipEvent_t *ev)
{
    if (a.ic) {
        if (a.prec != Prec::F64) {
            set_error("the IC(0) preconditioner runs in FP64 only");
            return HNS_ERR_INVALID;
        }
        return ic0_iteration(a, parity, s, ev);
    }
    if (a.lfac) {
        if (a.prec == Prec::F64) return line_iteration<double>(a, parity, s, ev);
        if (a.prec == Prec::F32) return line_iteration<float>(a, parity, s, ev);
        set_error("the line preconditioner runs FP64 iterations or FP32 inner iterations");
        return HNS_ERR_INVALID;
    }
    if (a.wjac) {
        if (!a.A->unit || a.A->fmt != HNS_FMT_SDIA) {
            set_error("the Jacobi-scaled iteration needs the unit-diagonal operator");
            return HNS_ERR_INVALID;
        }
        if (a.prec == Prec::F64) return iteration_scaled<double>(a, parity, s, ev);
        if (a.prec == Prec::F32) return iteration_scaled<float>(a, parity, s, ev);
        set_error("the Jacobi-scaled iteration runs FP64 or FP32 recurrences");
        return HNS_ERR_INVALID;
    }
    switch (a.prec) {
    case Prec::F64: return iteration_impl<double, double, double>(a, parity, s, ev);
    case Prec::F32: return iteration_impl<float, float, float>(a, parity, s, ev);
    case Prec::F32Store: return iteration_impl<float, double, float>(a, parity, s, ev);
    }
    set_error("unknown precision");
    return HNS_ERR_INVALID;
}

bool scaled_fusable(const IterArgs &a)
{
    return a.wjac && !a.lfac && !a.ic && a.A->unit && a.A->fmt == HNS_FMT_SDIA &&
           a.A->ndiag >= 1 && a.A->ndiag <= kMaxDiag &&
           (a.prec == Prec::F64 || a.prec == Prec::F32);
}

hns_status launch_scaled_fused_step(const IterArgs &a, const void *po, void *pn,
                                    uint32_t prev_token, int prev_parity, int parity,
                                    hipStream_t s, hipEvent_t *ev)
{
    if (!scaled_fusable(a)) {
        set_error("the fused iteration runs CG on the unit-diagonal diagonal-storage operator");
        return HNS_ERR_INVALID;
    }
    if (a.prec == Prec::F64)
        return scaled_fused_step_t<double>(a, po, pn, prev_token, prev_parity, parity, s, ev);
    return scaled_fused_step_t<float>(a, po, pn, prev_token, prev_parity, parity, s, ev);
}

hns_status launch_scaled_fused_close(const IterArgs &a, const void *po, uint32_t token,
                                     int parity, hipStream_t s)
{
    if (!scaled_fusable(a)) {
        set_error("the fused iteration runs CG on the unit-diagonal diagonal-storage operator");
        return HNS_ERR_INVALID;
    }
    if (a.prec == Prec::F64) return scaled_fused_close_t<double>(a, po, token, parity, s);
    return scaled_fused_close_t<float>(a, po, token, parity, s);
}

hns_status launch_bstats(int64_t n, const double *b, const uint8_t *bc, int bit, Scalars *sc,
                         double *partials, hipStream_t s)
{
    if (bit < 0) bc = nullptr;
    k_bstats<<<stream_grid(n), kBlock, 0, s>>>(n, b, bc, bit, sc, partials + kPartMisc);
    HNS_TRY(check_launch("bstats"));
    k_fin_bstats<<<1, kBlock, 0, s>>>(partials + kPartMisc, stream_grid(n), sc);
    return check_launch("fin_bstats");
}

hns_status launch_prepare_x(int64_t n, double *x, const uint8_t *bc, int bit, bool zero_all,
                            hipStream_t s)
{
    if (bit < 0) bc = nullptr;
    k_prepare_x<<<stream_grid(n), kBlock, 0, s>>>(n, x, bc, bit, zero_all ? 1 : 0);
    return check_launch("prepare_x");
}

hns_status launch_residual(int64_t n, const double *b, const double *q, double *r,
                           const uint8_t *bc, int bit, bool singular, Scalars *sc,
                           double *partials, hipStream_t s)
{
    if (bit < 0) bc = nullptr;
    k_residual<<<stream_grid(n), kBlock, 0, s>>>(n, b, q, r, bc, bit, singular ? 1 : 0, sc,
                                                 partials + kPartMisc);
    HNS_TRY(check_launch("residual"));
    k_fin_residual<<<1, kBlock, 0, s>>>(partials + kPartMisc, stream_grid(n), sc);
    return check_launch("fin_residual");
}

hns_status launch_init_dir(int64_t n, Prec prec, void *r, void *p, const void *dinv,
                           bool singular, bool bb_from_rr, Scalars *sc, double *partials,
                           hipStream_t s)
{
    const int G = stream_grid(n);
    const int sg = singular ? 1 : 0, bf = bb_from_rr ? 1 : 0;
    double *P = partials + kPartMisc;
    switch (prec) {
    case Prec::F64:
        k_init_dir<double, double><<<G, kBlock, 0, s>>>(n, (double *)r, (double *)p,
                                                        (const double *)dinv, sg, sc, P);
        break;
    case Prec::F32:
        k_init_dir<float, float><<<G, kBlock, 0, s>>>(n, (float *)r, (float *)p,
                                                      (const float *)dinv, sg, sc, P);
        break;
    case Prec::F32Store:
        k_init_dir<double, float><<<G, kBlock, 0, s>>>(n, (double *)r, (double *)p,
                                                       (const float *)dinv, sg, sc, P);
        break;
    }
    HNS_TRY(check_launch("init_dir"));
    k_fin_start<<<1, kBlock, 0, s>>>(P, G, sc, bf);
    return check_launch("fin_start");
}

hns_status launch_replace_residual(int64_t n, Prec prec, const double *r64, void *r, void *p,
                                   const void *dinv, Scalars *sc, double *partials, int parity,
                                   hipStream_t s)
{
    const int Gu = stream_grid(n);
    double *P2 = partials + kPartUpdate;
    if (prec == Prec::F32) {
        k_replace_rz<float, float><<<Gu, kBlock, 0, s>>>(n, r64, (float *)r, (const float *)dinv,
                                                         P2);
        HNS_TRY(check_launch("replace_rz"));
        k_pupdate<float, float><<<Gu, kBlock, 0, s>>>(n, 0, (float *)p, (const float *)r,
                                                      (const float *)dinv, sc, P2, Gu, parity, 0);
    } else if (prec == Prec::F32Store) {
        k_replace_rz<double, float><<<Gu, kBlock, 0, s>>>(n, r64, nullptr, (const float *)dinv,
                                                          P2);
        HNS_TRY(check_launch("replace_rz"));
        k_pupdate<double, float><<<Gu, kBlock, 0, s>>>(n, 0, (double *)p, r64, (const float *)dinv,
                                                       sc, P2, Gu, parity, 0);
    } else {
        k_replace_rz<double, double><<<Gu, kBlock, 0, s>>>(n, r64, nullptr,
                                                           (const double *)dinv, P2);
        HNS_TRY(check_launch("replace_rz"));
        k_pupdate<double, double><<<Gu, kBlock, 0, s>>>(n, 0, (double *)p, r64,
                                                        (const double *)dinv, sc, P2, Gu, parity,
                                                        0);
    }
    return check_launch("pupdate (replacement)");
}

hns_status launch_scale_in(int64_t n, Prec prec, const double *r64, void *r, void *p, void *dx,
                           const double *s_half, Scalars *sc, double *partials, hipStream_t s)
{
    const int G = stream_grid(n);
    double *P = partials + kPartMisc;
    if (prec == Prec::F64)
        k_scale_in<double><<<G, kBlock, 0, s>>>(n, r64, (double *)r, (double *)p, (double *)dx,
                                                s_half, sc, P);
    else if (prec == Prec::F32)
        k_scale_in<float><<<G, kBlock, 0, s>>>(n, r64, (float *)r, (float *)p, (float *)dx,
                                               s_half, sc, P);
    else {
        set_error("the Jacobi-scaled recurrence runs in FP64 or FP32");
        return HNS_ERR_INVALID;
    }
    HNS_TRY(check_launch("scale_in"));
    k_fin_start<<<1, kBlock, 0, s>>>(P, G, sc, 0);
    return check_launch("fin_start");
}

hns_status launch_scale_out(int64_t n, Prec prec, double *x, void *dx, const double *s_half,
                            hipStream_t s)
{
    const int G = stream_grid(n);
    if (prec == Prec::F64)
        k_scale_out<double><<<G, kBlock, 0, s>>>(n, x, (double *)dx, s_half);
    else if (prec == Prec::F32)
        k_scale_out<float><<<G, kBlock, 0, s>>>(n, x, (float *)dx, s_half);
    else {
        set_error("the Jacobi-scaled recurrence runs in FP64 or FP32");
        return HNS_ERR_INVALID;
    }
    return check_launch("scale_out");
}

hns_status launch_replace_scaled(int64_t n, const double *r64, float *r, float *p,
                                 const double *s_half, Scalars *sc, double *partials, int parity,
                                 hipStream_t s)
{
    const int Gu = stream_grid(n);
    double *P2 = partials + kPartUpdate;
    k_replace_rz_scaled<<<Gu, kBlock, 0, s>>>(n, r64, r, s_half, P2);
    HNS_TRY(check_launch("replace_rz (Jacobi-scaled)"));
    k_pupdate<float, float, 1, true><<<Gu, kBlock, 0, s>>>(n, 0, p, (const float *)r, nullptr, sc,
                                                           P2, Gu, parity, 0);
    return check_launch("pupdate (Jacobi-scaled replacement)");
}

hns_status launch_jacobi_scale(int64_t n, int ndiag, const int32_t *off, const double *dia,
                               double *s_half, float *w, double *out, float *out32,
                               hipStream_t s)
{
    if (ndiag < 1 || ndiag > kMaxDiag) {
        set_error("Jacobi scaling of %d upper diagonals (1 to %d supported)", ndiag, kMaxDiag);
        return HNS_ERR_INVALID;
    }
    DiaOffsets offs;
    for (int k = 0; k < kMaxDiag; ++k) offs.o[k] = k < ndiag ? off[k] : 0;
    const int G = stream_grid(n);
    k_jacobi_diag<<<G, kBlock, 0, s>>>(n, dia, s_half, w);
    HNS_TRY(check_launch("jacobi_diag"));
    k_jacobi_scale<<<G, kBlock, 0, s>>>(n, ndiag, offs, dia, s_half, out, out32);
    return check_launch("jacobi_scale");
}

hns_status launch_project_norm(int64_t n, double *r, bool singular, Scalars *sc,
                               double *partials, hipStream_t s)
{
    k_project_norm<<<stream_grid(n), kBlock, 0, s>>>(n, r, singular ? 1 : 0, sc,
                                                     partials + kPartMisc);
    HNS_TRY(check_launch("project_norm"));
    k_fin_one<<<1, kBlock, 0, s>>>(partials + kPartMisc, stream_grid(n), sc, 0);
    return check_launch("fin_norm");
}

hns_status launch_cast_scaled(int64_t n, const double *r64, float *r32, float *d32,
                              const Scalars *outer, hipStream_t s)
{
    k_cast_scaled<<<stream_grid(n), kBlock, 0, s>>>(n, r64, r32, d32, outer);
    return check_launch("cast_scaled");
}

hns_status launch_correct(int64_t n, double *x, const float *d32, const Scalars *outer,
                          hipStream_t s)
{
    k_correct<<<stream_grid(n), kBlock, 0, s>>>(n, x, d32, outer);
    return check_launch("correct");
}

hns_status launch_cast(int64_t n, const double *r64, float *r32, float *x32, hipStream_t s)
{
    k_cast<<<stream_grid(n), kBlock, 0, s>>>(n, r64, r32, x32);
    return check_launch("cast");
}

hns_status launch_accumulate(int64_t n, double *x64, float *x32, hipStream_t s)
{
    k_accumulate<<<stream_grid(n), kBlock, 0, s>>>(n, x64, x32);
    return check_launch("accumulate");
}

hns_status launch_set_threshold(Scalars *sc, double tol2, double bb, hipStream_t s)
{
    k_set_threshold<<<1, 64, 0, s>>>(sc, tol2, bb);
    return check_launch("set_threshold");
}

hns_status launch_normalise(int64_t n, double *x, const double *lumped, double lumped_sum,
                            Scalars *sc, double *partials, hipStream_t s)
{
    k_wdot<<<stream_grid(n), kBlock, 0, s>>>(n, lumped, x, sc, partials + kPartMisc);
    HNS_TRY(check_launch("wdot"));
    k_fin_one<<<1, kBlock, 0, s>>>(partials + kPartMisc, stream_grid(n), sc, 1);
    HNS_TRY(check_launch("fin_wdot"));
    k_shift<<<stream_grid(n), kBlock, 0, s>>>(n, x, sc, lumped_sum);
    return check_launch("shift");
}

}  // namespace hns
