// Device assembly of a P1 operator c_mass M + c_stiff K_nu (Sec. 4 forms,
// discretised in Sec. 5), in two forms:
//  - values on a pattern built on the host (compressed rows);
//  - the whole operator on the device: node-to-tetrahedron incidence
//    (counting sort, each node's list in ascending tetrahedron order), the
//    distinct upper offsets j - i of the element couplings, and the values
//    straight into symmetric diagonal storage, with D^-1, the lumped mass and
//    the structural nonzero count.
//
// Both kernels do what the host assembly does, in the same order: one lane
// per row gathers the tetrahedra around its node in ascending order,
// recomputes each tetrahedron's hat-function gradients from the coordinates
// (cofactors of the edge vectors), and adds c_mass m_ab + c_stiff k_ab to
// the entries of its row.  Contraction of multiply-adds is switched off, so
// the values are bitwise those of the host assembly.  The element couplings
// are bitwise symmetric (entry (i, j) and (j, i) sum the same products over
// the same tetrahedra in the same order), so diagonal storage keeps the upper
// triangle only, as the host conversion does.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>

#include "hns_internal.h"

namespace hns {
namespace {

// Hat-function gradients g and volume of tetrahedron t.
__device__ inline void tet_gradients(const double *__restrict__ xyz, const int32_t *t,
                                     double g[4][3], double &vol)
{
#pragma clang fp contract(off)
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
    vol = D / 6.0;
    const double inv = 1.0 / D;
    for (int d = 0; d < 3; ++d) {
        g[1][d] = c1[d] * inv;
        g[2][d] = c2[d] * inv;
        g[3][d] = c3[d] * inv;
        g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    }
}

// c_mass m_ab + c_stiff k_ab of one tetrahedron
__device__ inline double tet_entry(const double g[4][3], double vol, int a, int b,
                                   const double nu[3], double c_mass, double c_stiff)
{
#pragma clang fp contract(off)
    double kk = 0.0;
    for (int d = 0; d < 3; ++d) kk += nu[d] * (g[a][d] * g[b][d]);
    kk *= vol;
    const double m = (a == b) ? vol / 10.0 : vol / 20.0;
    return c_mass * m + c_stiff * kk;
}

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
            double g[4][3], vol;
            tet_gradients(xyz, t, g, vol);
            if (!(vol > 0.0) || !isfinite(vol)) atomicMin(bad, (unsigned long long)itet[s]);
            mi += vol / 4.0;
            for (int b = 0; b < 4; ++b) {
                // position of column t[b] in the sorted row
                int32_t lo = r0, hi = r1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (col[mid] < t[b]) lo = mid + 1;
                    else hi = mid;
                }
                val[lo] += tet_entry(g, vol, a, b, nu, c_mass, c_stiff);
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

// ---------------------------------------------------------------------------
// The whole operator on the device (diagonal storage)
// ---------------------------------------------------------------------------
namespace {

constexpr unsigned long long kNone = ~0ull;

int grid_for(int64_t units)
{
    int64_t g = (units + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

// Incidence counts per node; the first vertex entry (flat index) outside [0, n).
__global__ __launch_bounds__(256) void k_inc_count(int64_t m, int64_t n,
                                                   const int32_t *__restrict__ tets,
                                                   uint32_t *__restrict__ cnt,
                                                   unsigned long long *__restrict__ bad)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = tets[e];
        if (v < 0 || v >= n) {
            atomicMin(bad, (unsigned long long)e);
            continue;
        }
        atomicAdd(&cnt[v], 1u);
    }
}

// First non-finite coordinate (flat index).
__global__ __launch_bounds__(256) void k_check_coords(int64_t m, const double *__restrict__ xyz,
                                                      unsigned long long *__restrict__ bad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(xyz[i])) atomicMin(bad, (unsigned long long)i);
}

// Each tetrahedron into the next free place of the lists of its four vertices.
__global__ __launch_bounds__(256) void k_inc_fill(int64_t ne, const int32_t *__restrict__ tets,
                                                  uint32_t *__restrict__ cursor,
                                                  int32_t *__restrict__ itet)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
         e += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 4; ++a) {
            const uint32_t s = atomicAdd(&cursor[tets[4 * e + a]], 1u);
            itet[s] = (int32_t)e;
        }
}

// Each node's list in ascending tetrahedron order (insertion sort: a list
// holds the few tetrahedra around one node, 24 in the interior of a Kuhn
// lattice).  A list of up to kSortSlot entries is sorted in the thread's
// slot of LDS (entry k at buf[k * 256 + thread], so the lanes of a wavefront
// hit distinct banks) and read and written once; a longer one is sorted in
// place in global memory.  The result, ascending order of distinct values,
// is unique either way.
constexpr int kSortSlot = 48;

__global__ __launch_bounds__(256) void k_inc_sort(int64_t n, const uint32_t *__restrict__ ptr,
                                                  int32_t *__restrict__ itet)
{
    __shared__ int32_t buf[kSortSlot * 256];
    int32_t *mine = buf + threadIdx.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t lo = ptr[i], hi = ptr[i + 1];
        const uint32_t len = hi - lo;
        if (len <= (uint32_t)kSortSlot) {
            for (uint32_t k = 0; k < len; ++k) mine[k * 256] = itet[lo + k];
            for (uint32_t s = 1; s < len; ++s) {
                const int32_t t = mine[s * 256];
                uint32_t r = s;
                while (r > 0 && mine[(r - 1) * 256] > t) {
                    mine[r * 256] = mine[(r - 1) * 256];
                    --r;
                }
                mine[r * 256] = t;
            }
            for (uint32_t k = 0; k < len; ++k) itet[lo + k] = mine[k * 256];
            continue;
        }
        for (uint32_t s = lo + 1; s < hi; ++s) {
            const int32_t t = itet[s];
            uint32_t r = s;
            while (r > lo && itet[r - 1] > t) {
                itet[r] = itet[r - 1];
                --r;
            }
            itet[r] = t;
        }
    }
}

// flag[d] = 1 for every distance d = |t_a - t_b| > 0 between two vertices of
// one tetrahedron: the upper offsets of the element couplings.
__global__ __launch_bounds__(256) void k_offset_flags(int64_t ne, const int32_t *__restrict__ tets,
                                                      uint8_t *__restrict__ flag)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t t[4];
        for (int a = 0; a < 4; ++a) t[a] = tets[4 * e + a];
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                const int32_t d = t[a] > t[b] ? t[a] - t[b] : t[b] - t[a];
                if (d > 0) flag[d] = 1;
            }
    }
}

// The flagged offsets (at most cap of them listed, all counted).
__global__ __launch_bounds__(256) void k_offset_list(int64_t n, const uint8_t *__restrict__ flag,
                                                     uint32_t *__restrict__ count,
                                                     int32_t *__restrict__ out, int cap)
{
    for (int64_t d = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n;
         d += (int64_t)gridDim.x * blockDim.x)
        if (flag[d]) {
            const uint32_t k = atomicAdd(count, 1u);
            if (k < (uint32_t)cap) out[k] = (int32_t)d;
        }
}

struct UpperOffsets {
    int nd;
    int32_t off[kMaxDiag];
};

// Row i of c_mass M + c_stiff K_nu in diagonal storage: entry (i, i + off[k])
// at dia[(k + 1) n + i], the diagonal at dia[i]; the row's entries gathered
// over its tetrahedra in ascending order (the host loop's order for every
// entry).  Also 1 / a_ii (0 and the row reported where a_ii is not positive
// and finite), the lumped mass, FP32 copies, and the row's structural
// nonzeros (the diagonal and twice each present upper coupling) summed over
// the grid.
__global__ __launch_bounds__(256) void k_assemble_sdia(
    int64_t n, const double *__restrict__ xyz, const int32_t *__restrict__ tets,
    const uint32_t *__restrict__ ptr, const int32_t *__restrict__ itet, UpperOffsets O,
    double c_mass, double c_stiff, double nu_h, double nu_v, double *__restrict__ dia,
    float *__restrict__ dia32, double *__restrict__ dinv, float *__restrict__ dinv32,
    double *__restrict__ lumped, unsigned long long *__restrict__ bad_tet,
    unsigned long long *__restrict__ bad_row, unsigned long long *__restrict__ nnz)
{
#pragma clang fp contract(off)
    __shared__ unsigned long long block_nnz;
    if (threadIdx.x == 0) block_nnz = 0;
    __syncthreads();
    unsigned long long mine = 0;
    const double nu[3] = {nu_h, nu_h, nu_v};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc[kMaxDiag + 1];
#pragma unroll
        for (int q = 0; q <= kMaxDiag; ++q) acc[q] = 0.0;
        uint32_t present = 0;
        double mi = 0.0;
        for (uint32_t s = ptr[i]; s < ptr[i + 1]; ++s) {
            const int32_t e = itet[s];
            const int32_t *t = tets + 4 * (int64_t)e;
            int a = 0;
            while (a < 3 && t[a] != i) ++a;
            double g[4][3], vol;
            tet_gradients(xyz, t, g, vol);
            if (!(vol > 0.0) || !isfinite(vol)) atomicMin(bad_tet, (unsigned long long)e);
            mi += vol / 4.0;
            for (int b = 0; b < 4; ++b) {
                const int64_t d = (int64_t)t[b] - i;
                if (d < 0) continue;
                int slot = 0;
                for (int k = 0; k < O.nd; ++k)
                    if (O.off[k] == d) slot = k + 1;
                if (d > 0 && slot == 0) continue;   // not an element offset: cannot happen
                const double v = tet_entry(g, vol, a, b, nu, c_mass, c_stiff);
#pragma unroll
                for (int q = 0; q <= kMaxDiag; ++q)
                    if (q == slot) acc[q] += v;
                present |= 1u << slot;
            }
        }
#pragma unroll
        for (int q = 0; q <= kMaxDiag; ++q)
            if (q <= O.nd) {
                dia[(int64_t)q * n + i] = acc[q];
                if (dia32) dia32[(int64_t)q * n + i] = (float)acc[q];
            }
        double di = 0.0;
        if (acc[0] > 0.0 && isfinite(acc[0])) di = 1.0 / acc[0];
        else atomicMin(bad_row, (unsigned long long)i);
        dinv[i] = di;
        if (dinv32) dinv32[i] = (float)di;
        lumped[i] = mi;
        mine += 1ull + 2ull * (unsigned long long)__popc(present >> 1);
    }
    atomicAdd(&block_nnz, mine);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nnz, block_nnz);
}

}  // namespace

hns_status assemble_operator_device(const hns_mesh *mesh, double c_mass, double c_stiff,
                                    double nu_h, double nu_v, bool keep32, hns_operator *op,
                                    bool *applicable)
{
    *applicable = false;
    const int64_t n = mesh->n_nodes, ne = mesh->n_tets;
    // no element (no offsets) or incidence beyond 32-bit positions: the host path
    if (ne <= 0 || 4 * ne >= (int64_t)INT32_MAX) return HNS_OK;
    double *xyz = nullptr;
    int32_t *tets = nullptr, *itet = nullptr;
    uint32_t *ptr = nullptr, *cursor = nullptr;
    uint8_t *flag = nullptr;
    void *scan_tmp = nullptr;
    unsigned long long *misc = nullptr;   // bad vertex, bad coordinate, bad tetrahedron, bad row, nnz
    uint32_t *count = nullptr;
    int32_t *offs_dev = nullptr;
    DevMatrix A;
    double *dinv = nullptr, *lumped = nullptr;
    float *dinv32 = nullptr;
    auto run = [&]() -> hns_status {
        HNS_TRY(dev_copy(mesh->xyz, 3 * (size_t)n, &xyz));
        HNS_TRY(dev_copy(mesh->tets, 4 * (size_t)ne, &tets));
        HNS_TRY(dev_copy<uint32_t>(nullptr, (size_t)n + 1, &ptr));
        HNS_TRY(dev_copy<uint32_t>(nullptr, (size_t)n, &cursor));
        const unsigned long long init[6] = {kNone, kNone, kNone, kNone, 0ull, 0ull};
        HNS_TRY(dev_copy(init, 6, &misc));
        count = (uint32_t *)(misc + 5);
        HNS_TRY_HIP(hipMemset(cursor, 0, (size_t)n * sizeof(uint32_t)));
        // mesh checks: vertex indices first (nothing indexes with them before), then coordinates
        k_inc_count<<<grid_for(4 * ne), 256>>>(4 * ne, n, tets, cursor, misc + 0);
        HNS_TRY_HIP(hipGetLastError());
        k_check_coords<<<grid_for(3 * n), 256>>>(3 * n, xyz, misc + 1);
        HNS_TRY_HIP(hipGetLastError());
        unsigned long long bad[2];
        HNS_TRY_HIP(hipMemcpy(bad, misc, sizeof(bad), hipMemcpyDeviceToHost));
        if (bad[0] != kNone) {
            set_error("mesh: tetrahedron %lld references node %d outside [0,%lld)",
                      (long long)(bad[0] / 4), mesh->tets[bad[0]], (long long)n);
            return HNS_ERR_MESH;
        }
        if (bad[1] != kNone) {
            set_error("mesh: non-finite coordinate at node %lld", (long long)(bad[1] / 3));
            return HNS_ERR_MESH;
        }
        // list starts: ptr[0] = 0, ptr[i + 1] = counts of nodes 0..i
        HNS_TRY_HIP(hipMemset(ptr, 0, sizeof(uint32_t)));
        size_t tmp_bytes = 0;
        HNS_TRY_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_bytes, cursor, ptr + 1, (int)n));
        HNS_TRY_HIP(hipMalloc(&scan_tmp, tmp_bytes));
        HNS_TRY_HIP(hipcub::DeviceScan::InclusiveSum(scan_tmp, tmp_bytes, cursor, ptr + 1, (int)n));
        HNS_TRY_HIP(hipMemcpy(cursor, ptr, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice));
        HNS_TRY(dev_copy<int32_t>(nullptr, 4 * (size_t)ne, &itet));
        k_inc_fill<<<grid_for(ne), 256>>>(ne, tets, cursor, itet);
        HNS_TRY_HIP(hipGetLastError());
        k_inc_sort<<<grid_for(n), 256>>>(n, ptr, itet);
        HNS_TRY_HIP(hipGetLastError());
        // the distinct upper offsets
        HNS_TRY(dev_copy<uint8_t>(nullptr, (size_t)n, &flag));
        HNS_TRY_HIP(hipMemset(flag, 0, (size_t)n));
        k_offset_flags<<<grid_for(ne), 256>>>(ne, tets, flag);
        HNS_TRY_HIP(hipGetLastError());
        HNS_TRY(dev_copy<int32_t>(nullptr, kMaxDiag, &offs_dev));
        k_offset_list<<<grid_for(n), 256>>>(n, flag, count, offs_dev, kMaxDiag);
        HNS_TRY_HIP(hipGetLastError());
        uint32_t nd = 0;
        HNS_TRY_HIP(hipMemcpy(&nd, count, sizeof(nd), hipMemcpyDeviceToHost));
        // beyond the unrolled diagonal storage (or none): the host path chooses the format
        if (nd == 0 || nd > (uint32_t)kMaxDiag) return HNS_OK;
        UpperOffsets O{};
        O.nd = (int)nd;
        HNS_TRY_HIP(hipMemcpy(O.off, offs_dev, nd * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::sort(O.off, O.off + nd);
        // values
        A.n = n;
        A.fmt = HNS_FMT_SDIA;
        A.ndiag = O.nd;
        for (int k = 0; k < O.nd; ++k) A.off[k] = O.off[k];
        const size_t nv = (size_t)(O.nd + 1) * n;
        HNS_TRY(dev_copy<double>(nullptr, nv, &A.dia));
        if (keep32) HNS_TRY(dev_copy<float>(nullptr, nv, &A.dia32));
        HNS_TRY(dev_copy<double>(nullptr, (size_t)n, &dinv));
        if (keep32) HNS_TRY(dev_copy<float>(nullptr, (size_t)n, &dinv32));
        HNS_TRY(dev_copy<double>(nullptr, (size_t)n, &lumped));
        k_assemble_sdia<<<grid_for(n), 256>>>(n, xyz, tets, ptr, itet, O, c_mass, c_stiff, nu_h,
                                              nu_v, A.dia, A.dia32, dinv, dinv32, lumped,
                                              misc + 2, misc + 3, misc + 4);
        HNS_TRY_HIP(hipGetLastError());
        unsigned long long res[3];
        HNS_TRY_HIP(hipMemcpy(res, misc + 2, sizeof(res), hipMemcpyDeviceToHost));
        if (res[0] != kNone) {
            set_error("mesh: tetrahedron %llu has non-positive volume", res[0]);
            return HNS_ERR_MESH;
        }
        A.nnz = (int64_t)res[2];
        // the lumped total in node order, as the host path sums it
        std::vector<double> lh((size_t)n);
        HNS_TRY_HIP(hipMemcpy(lh.data(), lumped, (size_t)n * sizeof(double),
                              hipMemcpyDeviceToHost));
        double total = 0.0;
        for (double m : lh) total += m;
        op->n = n;
        op->A = A;
        op->dinv = dinv;
        op->dinv32 = dinv32;
        op->lumped = lumped;
        op->lumped_sum = total;
        op->bad_diag = res[1] == kNone ? -1 : (int64_t)res[1];
        A = DevMatrix();   // now owned by op
        dinv = lumped = nullptr;
        dinv32 = nullptr;
        *applicable = true;
        return HNS_OK;
    };
    const hns_status st = run();
    A.release();
    void *ptrs[] = {xyz, tets, itet, ptr, cursor, flag, scan_tmp, misc, offs_dev, dinv, lumped,
                    dinv32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    return st;
}

}  // namespace hns
