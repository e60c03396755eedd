// Right-hand sides and corrections of one projection time step (Sec. 3,
// weak forms of Sec. 4 discretised as in Sec. 5), built from the auxiliary
// forms kept on a HNS_STEP_AUX operator.  All work runs in the kernels
// below and the library's CSR SpMV.
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

}  // extern "C"
