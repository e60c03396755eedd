// Kernel launchers of the hns library (device code lives in kernels.hip).
#pragma once

#include "hns_internal.h"

namespace hns {

// CG scalars kept on the device so that a chunk of iterations runs without
// host round trips.  rho is double-buffered by iteration parity: during
// iteration k (counted from the last restart) the kernels read rho[k & 1]
// and the last kernel writes the next value into rho[(k + 1) & 1], so no
// block ever reads a slot another block of the same launch writes.
struct Scalars {
    double rho[2];   // r^T z
    double alpha;    // rho / (p^T q)
    double beta;     // rho_new / rho
    double gamma;    // p^T q
    double rr;       // r^T r
    double bb;       // b^T b (after projection in the pure-Neumann case)
    double tol2;     // tol^2
    double sumb;     // sum of the free entries of b
    double bb_raw;   // sum of squares of the free entries of b
    double sum_r;    // sum of r (pure-Neumann projection)
    double wx;       // sum of lumped_i x_i (pure-Neumann normalisation)
    double nonfinite;
    int32_t stop;    // 0 running, 1 recursive residual below tolerance, 2 breakdown, 3 b = 0
    int32_t iter;    // CG iterations executed
    uint32_t xtoken; // tag of the last iteration whose update ran (x += alpha p pending)
};

// Layout of the per-workspace partial-sum buffer (doubles).  The FP32 SpMV
// may take twice kMaxPart workgroups (kMaxPartSpmv32): on the largest
// operators its rows per block stay at two workgroup passes.
constexpr int kMaxPartSpmv32 = 2 * kMaxPart;
constexpr int kPartSpmv = 0;                      // p^T q per SpMV block
constexpr int kPartUpdate = kMaxPartSpmv32;       // r^T z, r^T r per update block
constexpr int kPartMisc = kPartUpdate + 2 * kMaxPart;   // one-off reductions (3 values)
constexpr int kPartTotal = kPartMisc + 3 * kMaxPart;

// grid for a streaming kernel over n entries (multiple of 8 when >= 8)
int stream_grid(int64_t n);
// grid for the SpMV of a matrix in CSR or sliced ELL
int spmv_grid(const DevMatrix &A);

// Contiguous chunks: `grid` workgroups (a multiple of 8 when >= 8, at most
// `cap`) of `per` consecutive units each (a multiple of `quantum`, at least
// the requested per) cover `units` units.
struct Chunks {
    int grid;
    int64_t per;
};
Chunks chunks(int64_t units, int64_t per, int64_t quantum, int64_t cap = kMaxPart);

// Precision of one CG recurrence: matrix values / vectors / Jacobi diagonal
enum class Prec {
    F64,       // double / double / double
    F32,       // float  / float  / float   (inner iteration of the refinement)
    F32Store,  // float  / double / float   (FP32 storage, FP64 vectors)
};

struct IterArgs {
    const DevMatrix *A;
    Prec prec;
    int64_t n;
    void *x, *r, *p, *q;
    const void *dinv;
    const uint8_t *bc;
    int bit;
    Scalars *sc;
    double *partials;   // kPartTotal doubles
    // vertical-line preconditioner (FP64 only): when lfac is set, z = M^-1 r
    // by the column blocks of `line_len` consecutive rows; lfac holds the
    // masked off-diagonal (n) then the inverse pivots (n); z is an n-vector
    const void *lfac = nullptr;     // double (FP64) or float (F32) factors
    void *z = nullptr;              // z in the precision of the iteration
    int line_len = 0;
    // IC(0) preconditioner (FP64 only): when ic is set, z = M^-1 r by the
    // colour-by-colour triangular solves; y is an n-vector of scratch
    const IC0Dev *ic = nullptr;
    double *y = nullptr;
    // tag of this iteration (unique within a workspace, never 0): links the
    // point-Jacobi update to the direction update that completes it
    uint32_t token = 0;
    // Jacobi-scaled CG (point Jacobi on A as plain CG on D^-1/2 A D^-1/2):
    // when set, A is the unit-diagonal scaled operator, x, r, p, q are the
    // scaled vectors (x the correction D^1/2 dx of this segment, r = D^-1/2
    // r_A), dinv is not read, and wjac = diag(A) in FP32 weighs |r_A|^2
    const float *wjac = nullptr;
    // matrix-free operators: the element results of one product
    // (A->mf_scratch() doubles)
    double *mf = nullptr;
};

// One CG iteration = three launches:
//   spmv    q = mask(A p), per-block partials of p^T q
//   update  gamma = p^T q (every block sums the partials in the same order),
//           alpha = rho / gamma, r -= alpha q,
//           per-block partials of r^T D^-1 r and r^T r
//   pupdate rho' and rr from the partials, beta = rho' / rho, stop flags,
//           x += alpha p, then p = D^-1 r + beta p unless stopping
// With point Jacobi the x update rides in the direction update, which reads
// p anyway (one vector pass fewer); the line and IC(0) iterations keep it in
// their update kernels.
// ev (optional, 6 events) brackets the three kernels for timing.
hns_status launch_iteration(const IterArgs &a, int parity, hipStream_t s, hipEvent_t *ev);

// Fused iterations of CG on the Jacobi-scaled operator (a.wjac set, the
// unit-diagonal diagonal-storage operator): two launches per iteration, the
// direction update of iteration k riding in the product of k + 1, with p in
// two buffers (a.p and a spare).  A chunk is: step(po = nullptr) on a.p,
// then step(po = the previous iteration's p buffer, pn = the other) per
// further iteration, then close(po = the last buffer), which leaves p in a.p.
// prev_token / prev_parity name the iteration the step completes, a.token /
// parity the one it starts.  Same arithmetic as launch_iteration, bit for bit.
// ev: optional 4 events (product, update).
bool scaled_fusable(const IterArgs &a);
hns_status launch_scaled_fused_step(const IterArgs &a, const void *po, void *pn,
                                    uint32_t prev_token, int prev_parity, int parity,
                                    hipStream_t s, hipEvent_t *ev);
hns_status launch_scaled_fused_close(const IterArgs &a, const void *po, uint32_t token,
                                     int parity, hipStream_t s);

// `count` point-Jacobi CG iterations of a small system (n <= kSmallMaxN) in
// one workgroup: the same recurrence, device scalars and stop rule as
// `count` launch_iteration calls, with block barriers in place of the kernel
// boundaries (latency-bound sizes).  FP64 or FP32 (prec F64 / F32) only.
constexpr int64_t kSmallMaxN = 1 << 20;
hns_status launch_cg_small(const IterArgs &a, int parity, int count, hipStream_t s);

// q = mask(A p) without reductions (residuals and hns_apply)
hns_status launch_spmv_plain(const DevMatrix &A, bool fp32, const void *p, void *q,
                             const uint8_t *bc, int bit, hipStream_t s,
                             double *mf_scratch = nullptr);
// statistics of the free entries of b (sum, sum of squares, non-finite count)
hns_status launch_bstats(int64_t n, const double *b, const uint8_t *bc, int bit, Scalars *sc,
                         double *partials, hipStream_t s);
// x = 0 on Dirichlet nodes (everywhere when zero_all)
hns_status launch_prepare_x(int64_t n, double *x, const uint8_t *bc, int bit, bool zero_all,
                            hipStream_t s);
// r = mask(b - shift - q) (FP64), shift = sumb / n when singular; sum of r and
// of (b - shift)^2 into sc
hns_status launch_residual(int64_t n, const double *b, const double *q, double *r,
                           const uint8_t *bc, int bit, bool singular, Scalars *sc,
                           double *partials, hipStream_t s);
// (singular: r -= mean r) z = D^-1 r; p = z; rho[0] = r^T z; rr = r^T r; stop flag.
// bb_from_rr: set bb = rr (inner solves of the refinement loop)
hns_status launch_init_dir(int64_t n, Prec prec, void *r, void *p, const void *dinv,
                           bool singular, bool bb_from_rr, Scalars *sc, double *partials,
                           hipStream_t s);
// (singular: r -= mean r) rr = r^T r, FP64 residual of the refinement loop
// Columns per block of the line-preconditioned kernels (0 if the column is
// too long for one block's LDS) and the grid that covers all columns.
int line_cols_per_block(int line_len);
int line_grid(int64_t n, int line_len);

// Line-preconditioned first direction (FP64, or FP32 for the inner
// iterations of mixed precision): (singular: r -= mean r); z = M^-1 r; p = z;
// rho[0] = r^T z; rr = r^T r (and bb = rr if asked).
hns_status launch_init_line(int64_t n, int line_len, double *r, double *p, const double *lfac,
                            bool singular, bool bb_from_rr, Scalars *sc, double *partials,
                            hipStream_t s);
hns_status launch_init_line(int64_t n, int line_len, float *r, float *p, const float *lfac,
                            bool singular, bool bb_from_rr, Scalars *sc, double *partials,
                            hipStream_t s);
// Residual replacement of a line-preconditioned FP32 segment: r = (float) r64,
// z = M^-1 r, then rho' = r^T z, beta = rho' / rho[parity], p = z + beta p.
hns_status launch_replace_line(int64_t n, int line_len, const double *r64, float *r, float *z,
                               float *p, const float *lfac, Scalars *sc, double *partials,
                               int parity, int vec_it, hipStream_t s);

// IC(0) first direction (FP64): z = M^-1 r; p = z; rho[0] = r^T z; rr = r^T r.
hns_status launch_init_ic0(int64_t n, const IC0Dev &F, const double *r, double *p, double *z,
                           double *y, Scalars *sc, double *partials, hipStream_t s);

hns_status launch_project_norm(int64_t n, double *r, bool singular, Scalars *sc,
                               double *partials, hipStream_t s);
// r32 = (float)(r64 / sqrt(rr)), d32 = 0
hns_status launch_cast_scaled(int64_t n, const double *r64, float *r32, float *d32,
                              const Scalars *outer, hipStream_t s);
// x += sqrt(rr) * (double)d32
hns_status launch_correct(int64_t n, double *x, const float *d32, const Scalars *outer,
                          hipStream_t s);
// r32 = (float) r64, x32 = 0
hns_status launch_cast(int64_t n, const double *r64, float *r32, float *x32, hipStream_t s);
// x64 += x32, x32 = 0
hns_status launch_accumulate(int64_t n, double *x64, float *x32, hipStream_t s);
// sc->tol2 = tol2, sc->bb = bb, sc->stop = 0 (threshold of the next residual replacement)
hns_status launch_set_threshold(Scalars *sc, double tol2, double bb, hipStream_t s);
// The recurrence continues from the FP64 true residual r64: r = (TX) r64
// (r is ignored when the vectors are FP64 and r64 is the working residual),
// z = D^-1 r, rho' = r^T z, beta = rho' / rho[parity], p = z + beta p,
// rho[parity ^ 1] = rho'.  parity is that of the last executed iteration.
hns_status launch_replace_residual(int64_t n, Prec prec, const double *r64, void *r, void *p,
                                   const void *dinv, Scalars *sc, double *partials, int parity,
                                   hipStream_t s);
// Segment start of the Jacobi-scaled recurrence from the FP64 true residual
// r64 (already projected when singular): r = (TX)(s r64) with s = diag(A)^-1/2,
// p = r, dx = 0, rho[0] = r^T r, rr = r64^T r64, stop flag as launch_init_dir.
// r may alias r64 (FP64 recurrence: the scaled residual replaces it in place).
// prec F64 (TX = double) or F32 (TX = float).
hns_status launch_scale_in(int64_t n, Prec prec, const double *r64, void *r, void *p, void *dx,
                           const double *s_half, Scalars *sc, double *partials, hipStream_t s);
// Segment end: x += s dx (FP64), dx = 0.
hns_status launch_scale_out(int64_t n, Prec prec, double *x, void *dx, const double *s_half,
                            hipStream_t s);
// Residual replacement of the Jacobi-scaled FP32 recurrence: r = (float)(s r64),
// rho' = r^T r, rr = r64^T r64, beta = rho' / rho[parity], p = r + beta p.
hns_status launch_replace_scaled(int64_t n, const double *r64, float *r, float *p,
                                 const double *s_half, Scalars *sc, double *partials, int parity,
                                 hipStream_t s);
// The scaled operator: from the main diagonal d (array 0 of `dia`) s = d^-1/2
// and w = (float) d; out[k n + i] = dia[(k+1) n + i] s_i s_{i + off[k]} for the
// ndiag upper diagonals (0 past the last row), and its FP32 rounding when out32.
hns_status launch_jacobi_scale(int64_t n, int ndiag, const int32_t *off, const double *dia,
                               double *s_half, float *w, double *out, float *out32,
                               hipStream_t s);

// wx = sum lumped_i x_i ; then x -= wx / lumped_sum
hns_status launch_normalise(int64_t n, double *x, const double *lumped, double lumped_sum,
                            Scalars *sc, double *partials, hipStream_t s);

}  // namespace hns
