// Device assembly of the values of a P1 operator c_mass M + c_stiff K_nu
// (Sec. 4 forms, discretised in Sec. 5) on a pattern built on the host.
//
// The kernel does what the host assembly does, in the same order: one lane
// per row gathers the tetrahedra around its node in ascending order,
// recomputes each tetrahedron's hat-function gradients from the coordinates
// (cofactors of the edge vectors), and adds c_mass m_ab + c_stiff k_ab to
// the entries of its row.  Contraction of multiply-adds is switched off, so
// the values are bitwise those of the host assembly.
#include <cmath>

#include "hns_internal.h"

namespace hns {
namespace {

__global__ __launch_bounds__(256) void k_assemble_rows(
    int64_t n, const double *__restrict__ xyz, const int32_t *__restrict__ tets,
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ itet,
    const int8_t *__restrict__ iloc, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, double c_mass, double c_stiff, double nu_h, double nu_v,
    double *__restrict__ val, double *__restrict__ lumped, unsigned long long *__restrict__ bad)
{
#pragma clang fp contract(off)
    const double nu[3] = {nu_h, nu_h, nu_v};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r0 = rowptr[i], r1 = rowptr[i + 1];
        for (int32_t k = r0; k < r1; ++k) val[k] = 0.0;
        double mi = 0.0;
        for (int64_t s = ptr[i]; s < ptr[i + 1]; ++s) {
            const int32_t *t = tets + 4 * (int64_t)itet[s];
            const int a = iloc[s];
            const double *X0 = xyz + 3 * (int64_t)t[0];
            double e[3][3];
            for (int q = 0; q < 3; ++q) {
                const double *Xq = xyz + 3 * (int64_t)t[q + 1];
                for (int d = 0; d < 3; ++d) e[q][d] = Xq[d] - X0[d];
            }
            double c1[3], c2[3], c3[3];
            c1[0] = e[1][1] * e[2][2] - e[1][2] * e[2][1];
            c1[1] = e[1][2] * e[2][0] - e[1][0] * e[2][2];
            c1[2] = e[1][0] * e[2][1] - e[1][1] * e[2][0];
            c2[0] = e[2][1] * e[0][2] - e[2][2] * e[0][1];
            c2[1] = e[2][2] * e[0][0] - e[2][0] * e[0][2];
            c2[2] = e[2][0] * e[0][1] - e[2][1] * e[0][0];
            c3[0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
            c3[1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
            c3[2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
            const double D = e[0][0] * c1[0] + e[0][1] * c1[1] + e[0][2] * c1[2];
            const double vol = D / 6.0;
            if (!(vol > 0.0) || !isfinite(vol)) atomicMin(bad, (unsigned long long)itet[s]);
            const double inv = 1.0 / D;
            double g[4][3];
            for (int d = 0; d < 3; ++d) {
                g[1][d] = c1[d] * inv;
                g[2][d] = c2[d] * inv;
                g[3][d] = c3[d] * inv;
                g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
            }
            mi += vol / 4.0;
            for (int b = 0; b < 4; ++b) {
                double kk = 0.0;
                for (int d = 0; d < 3; ++d) kk += nu[d] * (g[a][d] * g[b][d]);
                kk *= vol;
                const double m = (a == b) ? vol / 10.0 : vol / 20.0;
                // position of column t[b] in the sorted row
                int32_t lo = r0, hi = r1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (col[mid] < t[b]) lo = mid + 1;
                    else hi = mid;
                }
                val[lo] += c_mass * m + c_stiff * kk;
            }
        }
        if (lumped) lumped[i] = mi;
    }
}

template <class T>
hns_status dev_copy(const T *src, size_t count, T **dst)
{
    *dst = nullptr;
    if (count == 0) return HNS_OK;
    hipError_t e = hipMalloc((void **)dst, count * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        set_error("device assembly: hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                  hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
    }
    if (src) HNS_TRY_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return HNS_OK;
}

}  // namespace

hns_status assemble_values_device(const hns_mesh *mesh, const std::vector<int64_t> &inc_ptr,
                                  const std::vector<int32_t> &inc_tet,
                                  const std::vector<int8_t> &inc_loc, HostCSR &A, double c_mass,
                                  double c_stiff, double nu_h, double nu_v,
                                  std::vector<double> *lumped)
{
    const int64_t n = mesh->n_nodes, ne = mesh->n_tets;
    const size_t nnz = A.col.size();
    double *xyz = nullptr, *val = nullptr, *lump = nullptr;
    int32_t *tets = nullptr, *itet = nullptr, *rowptr = nullptr, *col = nullptr;
    int64_t *ptr = nullptr;
    int8_t *iloc = nullptr;
    unsigned long long *bad = nullptr;
    const unsigned long long none = ~0ull;
    hns_status st = HNS_OK;
    auto run = [&]() -> hns_status {
        HNS_TRY(dev_copy(mesh->xyz, 3 * (size_t)n, &xyz));
        HNS_TRY(dev_copy(mesh->tets, 4 * (size_t)ne, &tets));
        HNS_TRY(dev_copy(inc_ptr.data(), inc_ptr.size(), &ptr));
        HNS_TRY(dev_copy(inc_tet.data(), inc_tet.size(), &itet));
        HNS_TRY(dev_copy(inc_loc.data(), inc_loc.size(), &iloc));
        HNS_TRY(dev_copy(A.rowptr.data(), A.rowptr.size(), &rowptr));
        HNS_TRY(dev_copy(A.col.data(), nnz, &col));
        HNS_TRY(dev_copy<double>(nullptr, nnz, &val));
        if (lumped) HNS_TRY(dev_copy<double>(nullptr, (size_t)n, &lump));
        HNS_TRY(dev_copy(&none, 1, &bad));
        int64_t g = (n + 255) / 256;
        if (g > 65536) g = 65536;
        k_assemble_rows<<<(int)g, 256>>>(n, xyz, tets, ptr, itet, iloc, rowptr, col, c_mass,
                                         c_stiff, nu_h, nu_v, val, lump, bad);
        HNS_TRY_HIP(hipGetLastError());
        unsigned long long first_bad = none;
        HNS_TRY_HIP(hipMemcpy(&first_bad, bad, sizeof(first_bad), hipMemcpyDeviceToHost));
        if (first_bad != none) {
            set_error("mesh: tetrahedron %llu has non-positive volume", first_bad);
            return HNS_ERR_MESH;
        }
        A.val.assign(nnz, 0.0);
        HNS_TRY_HIP(hipMemcpy(A.val.data(), val, nnz * sizeof(double), hipMemcpyDeviceToHost));
        if (lumped) {
            lumped->assign(n, 0.0);
            HNS_TRY_HIP(hipMemcpy(lumped->data(), lump, n * sizeof(double),
                                  hipMemcpyDeviceToHost));
        }
        return HNS_OK;
    };
    st = run();
    void *ptrs[] = {xyz, val, lump, tets, itet, rowptr, col, ptr, iloc, bad};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    return st;
}

}  // namespace hns
