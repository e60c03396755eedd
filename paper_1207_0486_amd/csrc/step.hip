// Right-hand sides and corrections of one projection time step (Sec. 3,
// weak forms of Sec. 4 discretised as in Sec. 5), built from the auxiliary
// forms kept on a HNS_STEP_AUX operator.  All work runs in the kernels
// below and the library's CSR SpMV.
#include <cmath>

#include "kernels.h"

namespace hns {
namespace {

#define GRID_STRIDE(i, n)                                                   \
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * kBlock)

__device__ __forceinline__ bool dirichlet(const uint8_t *bc, int bit, int64_t i)
{
    return bc != nullptr && ((bc[i] >> bit) & 1u);
}

// y += a x
__global__ __launch_bounds__(kBlock) void k_axpy(int64_t n, double *__restrict__ y, double a,
                                                 const double *__restrict__ x)
{
    GRID_STRIDE(i, n) y[i] += a * x[i];
}

// y = a .* b
__global__ __launch_bounds__(kBlock) void k_hadamard(int64_t n, double *__restrict__ y,
                                                     const double *__restrict__ a,
                                                     const double *__restrict__ b)
{
    GRID_STRIDE(i, n) y[i] = a[i] * b[i];
}

// y = a x
__global__ __launch_bounds__(kBlock) void k_scale(int64_t n, double *__restrict__ y, double a,
                                                  const double *__restrict__ x)
{
    GRID_STRIDE(i, n) y[i] = a * x[i];
}

__global__ __launch_bounds__(kBlock) void k_mask(int64_t n, double *__restrict__ y,
                                                 const uint8_t *__restrict__ bc, int bit)
{
    GRID_STRIDE(i, n)
    if (dirichlet(bc, bit, i)) y[i] = 0.0;
}

// u = mask(ut - dt * g / m_L)
__global__ __launch_bounds__(kBlock) void k_correct_lumped(int64_t n, double *__restrict__ u,
                                                           const double *__restrict__ ut,
                                                           const double *__restrict__ g,
                                                           const double *__restrict__ mL, double dt,
                                                           const uint8_t *__restrict__ bc,
                                                           int bit)
{
    GRID_STRIDE(i, n) u[i] = dirichlet(bc, bit, i) ? 0.0 : ut[i] - dt * g[i] / mL[i];
}

// out_c[a] = int ((u . grad) u_c) phi_a over the tetrahedra around node a,
// for c = 1..3 (explicit advection of the velocity prediction).  On a
// tetrahedron with basis gradients g_b the gradient of u_c is the constant
// G_c = sum_b u_c(b) g_b; (u . grad) u_c = sum_b phi_b s_b with
// s_b = u(b) . G_c, and int phi_a phi_b = vol/20 (1 + delta_ab) gives the
// node's share vol/20 (s_a + sum_b s_b).  One lane per node sums its
// tetrahedra in ascending order (deterministic, no atomics); the geometry is
// recomputed from the coordinates (cofactors of the edge vectors).
__global__ __launch_bounds__(kBlock) void k_advection(int64_t n, const double *__restrict__ xyz,
                                                      const int32_t *__restrict__ tets,
                                                      const int64_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ itet,
                                                      const int8_t *__restrict__ iloc,
                                                      const double *__restrict__ u,
                                                      double *__restrict__ out)
{
    GRID_STRIDE(a, n)
    {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t s = ptr[a]; s < ptr[a + 1]; ++s) {
            const int32_t *t = tets + 4 * (int64_t)itet[s];
            const int la = iloc[s];
            int64_t v[4];
            double X[4][3], U[3][4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                v[b] = t[b];
#pragma unroll
                for (int d = 0; d < 3; ++d) X[b][d] = xyz[3 * v[b] + d];
#pragma unroll
                for (int c = 0; c < 3; ++c) U[c][b] = u[c * n + v[b]];
            }
            double e[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d) e[k][d] = X[k + 1][d] - X[0][d];
            double g[4][3];
            // cofactors: g_1 = e2 x e3 / D, g_2 = e3 x e1 / D, g_3 = e1 x e2 / D
            const double c1[3] = {e[1][1] * e[2][2] - e[1][2] * e[2][1],
                                  e[1][2] * e[2][0] - e[1][0] * e[2][2],
                                  e[1][0] * e[2][1] - e[1][1] * e[2][0]};
            const double c2[3] = {e[2][1] * e[0][2] - e[2][2] * e[0][1],
                                  e[2][2] * e[0][0] - e[2][0] * e[0][2],
                                  e[2][0] * e[0][1] - e[2][1] * e[0][0]};
            const double c3[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1],
                                  e[0][2] * e[1][0] - e[0][0] * e[1][2],
                                  e[0][0] * e[1][1] - e[0][1] * e[1][0]};
            const double D = e[0][0] * c1[0] + e[0][1] * c1[1] + e[0][2] * c1[2];
            const double inv = 1.0 / D;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                g[1][d] = c1[d] * inv;
                g[2][d] = c2[d] * inv;
                g[3][d] = c3[d] * inv;
                g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
            }
            const double w = D / 120.0;   // vol / 20
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double G[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int d = 0; d < 3; ++d) G[d] += U[c][b] * g[b][d];
                double sb[4], sum = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    sb[b] = U[0][b] * G[0] + U[1][b] * G[1] + U[2][b] * G[2];
                    sum += sb[b];
                }
                acc[c] += w * (sum + sb[la]);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c * n + a] = acc[c];
    }
}

// u = mask(x)  (copy with the Dirichlet entries of bit set to 0)
__global__ __launch_bounds__(kBlock) void k_copy_masked(int64_t n, double *__restrict__ y,
                                                        const double *__restrict__ x,
                                                        const uint8_t *__restrict__ bc, int bit)
{
    GRID_STRIDE(i, n) y[i] = dirichlet(bc, bit, i) ? 0.0 : x[i];
}

hns_status check(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", what, hipGetErrorString(e));
        return HNS_ERR_HIP;
    }
    return HNS_OK;
}

hns_status need_aux(const hns_operator *op)
{
    if (!op) {
        set_error("null operator");
        return HNS_ERR_INVALID;
    }
    if (!op->has_aux) {
        set_error("the operator was not assembled with HNS_STEP_AUX");
        return HNS_ERR_INVALID;
    }
    return HNS_OK;
}

}  // namespace
}  // namespace hns

using namespace hns;

extern "C" {

hns_status hns_apply_aux(hns_operator *op, int which, const double *x_dev, double *y_dev,
                         void *stream)
{
    HNS_TRY(need_aux(op));
    if (!x_dev || !y_dev || which < 0 || which > 7) {
        set_error("hns_apply_aux: bad arguments");
        return HNS_ERR_INVALID;
    }
    const DevMatrix *F = which == 0 ? &op->M
                       : which <= 3 ? &op->B[which - 1]
                       : which <= 6 ? &op->Bt[which - 4]
                                    : &op->Ms;
    hipStream_t s = (hipStream_t)stream;
    HNS_TRY(launch_spmv_plain(*F, false, x_dev, y_dev, nullptr, -1, s));
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_velocity_rhs(hns_operator *op, const double *u_dev, const double *p_dev,
                                 const double *theta_dev, const double *f_dev, double *b_dev,
                                 void *stream)
{
    HNS_TRY(need_aux(op));
    if (!u_dev || !b_dev) {
        set_error("hns_step_velocity_rhs: null velocity or output");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const int G = stream_grid(n);
    const double dt = op->dt;
    double *t0 = op->step_tmp, *t1 = op->step_tmp + n;
    for (int c = 0; c < 3; ++c) {
        double *b = b_dev + c * n;
        const double *uc = u_dev + c * n;
        HNS_TRY(launch_spmv_plain(op->M, false, uc, b, nullptr, -1, s));  // M u_c
        if (theta_dev && c < 2) {                                          // + dt M_s theta_c
            HNS_TRY(launch_spmv_plain(op->Ms, false, theta_dev + c * n, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, dt, t0);
            HNS_TRY(check("axpy"));
        }
        if (p_dev) {                                                       // + dt B_c^T p
            HNS_TRY(launch_spmv_plain(op->Bt[c], false, p_dev, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, dt, t0);
            HNS_TRY(check("axpy"));
        }
        if (f_dev && c < 2) {  // Coriolis: +dt M (f u_2) for c = 1, -dt M (f u_1) for c = 2
            const double *uo = u_dev + (c == 0 ? 1 : 0) * n;
            k_hadamard<<<G, kBlock, 0, s>>>(n, t1, f_dev, uo);
            HNS_TRY(check("hadamard"));
            HNS_TRY(launch_spmv_plain(op->M, false, t1, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, c == 0 ? dt : -dt, t0);
            HNS_TRY(check("axpy"));
        }
        if (op->bc) {
            k_mask<<<G, kBlock, 0, s>>>(n, b, op->bc, c);
            HNS_TRY(check("mask"));
        }
    }
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_pressure_rhs(hns_operator *op, const double *ut_dev, double *b_dev,
                                 void *stream)
{
    HNS_TRY(need_aux(op));
    if (!ut_dev || !b_dev || !(op->dt != 0.0)) {
        set_error("hns_step_pressure_rhs: null vector or zero time step");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const int G = stream_grid(n);
    double *t0 = op->step_tmp;
    for (int c = 0; c < 3; ++c) {
        HNS_TRY(launch_spmv_plain(op->B[c], false, ut_dev + c * n, t0, nullptr, -1, s));
        if (c == 0)
            k_scale<<<G, kBlock, 0, s>>>(n, b_dev, -1.0 / op->dt, t0);
        else
            k_axpy<<<G, kBlock, 0, s>>>(n, b_dev, -1.0 / op->dt, t0);
        HNS_TRY(check("pressure rhs"));
    }
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_correct(hns_operator *op, const double *ut_dev, const double *q_dev,
                            double *p_dev, double *u_dev, void *stream)
{
    HNS_TRY(need_aux(op));
    if (!ut_dev || !q_dev || !u_dev) {
        set_error("hns_step_correct: null vector");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const int G = stream_grid(n);
    double *t0 = op->step_tmp;
    if (p_dev) {
        k_axpy<<<G, kBlock, 0, s>>>(n, p_dev, 1.0, q_dev);
        HNS_TRY(check("pressure update"));
    }
    for (int c = 0; c < 3; ++c) {
        HNS_TRY(launch_spmv_plain(op->B[c], false, q_dev, t0, nullptr, -1, s));
        k_correct_lumped<<<G, kBlock, 0, s>>>(n, u_dev + c * n, ut_dev + c * n, t0, op->lumped,
                                              op->dt, op->bc, c);
        HNS_TRY(check("velocity correction"));
    }
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_advection(hns_operator *op, const double *u_dev, double *out_dev,
                              void *stream)
{
    HNS_TRY(need_aux(op));
    if (!u_dev || !out_dev || u_dev == out_dev) {
        set_error("hns_step_advection: null or aliased vectors");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    k_advection<<<stream_grid(op->n), kBlock, 0, s>>>(op->n, op->mesh_xyz, op->mesh_tets,
                                                       op->inc_ptr, op->inc_tet, op->inc_loc,
                                                       u_dev, out_dev);
    HNS_TRY(check("advection"));
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_velocity_rhs_bdf(hns_operator *op, double tau, double a1, const double *u_dev,
                                     double a2, const double *uprev_dev, const double *p_dev,
                                     const double *theta_dev, const double *f_dev,
                                     const double *adv_dev, double *b_dev, void *stream)
{
    HNS_TRY(need_aux(op));
    if (!u_dev || !b_dev || (a2 != 0.0 && !uprev_dev) || !std::isfinite(tau) ||
        !std::isfinite(a1) || !std::isfinite(a2)) {
        set_error("hns_step_velocity_rhs_bdf: null vector or non-finite coefficient");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const int G = stream_grid(n);
    double *t0 = op->step_tmp, *t1 = op->step_tmp + n;
    for (int c = 0; c < 3; ++c) {
        double *b = b_dev + c * n;
        HNS_TRY(launch_spmv_plain(op->M, false, u_dev + c * n, t0, nullptr, -1, s));
        k_scale<<<G, kBlock, 0, s>>>(n, b, a1, t0);                       // a1 M u_c
        HNS_TRY(check("scale"));
        if (a2 != 0.0) {                                                   // + a2 M u'_c
            HNS_TRY(launch_spmv_plain(op->M, false, uprev_dev + c * n, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, a2, t0);
            HNS_TRY(check("axpy"));
        }
        if (theta_dev && c < 2) {                                          // + tau M_s theta_c
            HNS_TRY(launch_spmv_plain(op->Ms, false, theta_dev + c * n, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, tau, t0);
            HNS_TRY(check("axpy"));
        }
        if (f_dev && c < 2) {  // Coriolis: +tau M (f u_2) for c = 1, -tau M (f u_1) for c = 2
            k_hadamard<<<G, kBlock, 0, s>>>(n, t1, f_dev, u_dev + (c == 0 ? 1 : 0) * n);
            HNS_TRY(check("hadamard"));
            HNS_TRY(launch_spmv_plain(op->M, false, t1, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, c == 0 ? tau : -tau, t0);
            HNS_TRY(check("axpy"));
        }
        if (adv_dev) {                                                     // - tau N_c(u)
            k_axpy<<<G, kBlock, 0, s>>>(n, b, -tau, adv_dev + c * n);
            HNS_TRY(check("axpy"));
        }
        if (p_dev) {                                                       // + tau B_c^T p
            HNS_TRY(launch_spmv_plain(op->Bt[c], false, p_dev, t0, nullptr, -1, s));
            k_axpy<<<G, kBlock, 0, s>>>(n, b, tau, t0);
            HNS_TRY(check("axpy"));
        }
        if (op->bc) {
            k_mask<<<G, kBlock, 0, s>>>(n, b, op->bc, c);
            HNS_TRY(check("mask"));
        }
    }
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_pressure_rhs_tau(hns_operator *op, double tau, const double *ut_dev,
                                     double *b_dev, void *stream)
{
    HNS_TRY(need_aux(op));
    if (!ut_dev || !b_dev || !(tau != 0.0) || !std::isfinite(tau)) {
        set_error("hns_step_pressure_rhs_tau: null vector or zero time step");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const int G = stream_grid(n);
    double *t0 = op->step_tmp;
    for (int c = 0; c < 3; ++c) {
        HNS_TRY(launch_spmv_plain(op->B[c], false, ut_dev + c * n, t0, nullptr, -1, s));
        if (c == 0)
            k_scale<<<G, kBlock, 0, s>>>(n, b_dev, -1.0 / tau, t0);
        else
            k_axpy<<<G, kBlock, 0, s>>>(n, b_dev, -1.0 / tau, t0);
        HNS_TRY(check("pressure rhs"));
    }
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

hns_status hns_step_correct_rhs(hns_operator *op, double tau, const double *ut_dev,
                                const double *q_dev, double *p_dev, double *rhs_dev,
                                void *stream)
{
    HNS_TRY(need_aux(op));
    if (!ut_dev || !q_dev || !rhs_dev || !std::isfinite(tau)) {
        set_error("hns_step_correct_rhs: null vector or non-finite time step");
        return HNS_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const int G = stream_grid(n);
    double *t0 = op->step_tmp, *t1 = op->step_tmp + n;
    if (p_dev) {
        k_axpy<<<G, kBlock, 0, s>>>(n, p_dev, 1.0, q_dev);
        HNS_TRY(check("pressure update"));
    }
    for (int c = 0; c < 3; ++c) {
        double *r = rhs_dev + c * n;
        HNS_TRY(launch_spmv_plain(op->M, false, ut_dev + c * n, t0, nullptr, -1, s));
        HNS_TRY(launch_spmv_plain(op->B[c], false, q_dev, t1, nullptr, -1, s));
        k_axpy<<<G, kBlock, 0, s>>>(n, t0, -tau, t1);
        HNS_TRY(check("axpy"));
        k_copy_masked<<<G, kBlock, 0, s>>>(n, r, t0, op->bc, op->bc ? c : -1);
        HNS_TRY(check("mask"));
    }
    HNS_TRY_HIP(hipStreamSynchronize(s));
    return HNS_OK;
}

}  // extern "C"
