// Host assembly of the P1 operators and their upload to the device.
//
// Forms (Sec. 4, discretised in Sec. 5):
//   mass        M_ij  = int phi_i phi_j                       (eq. fofa_velo_pred_h, first term)
//   stiffness   K_ij  = int (nu grad phi_j) . grad phi_i,     (second term; nu = diag(nu_h,nu_h,nu_v))
//               also the pressure-increment operator of eq. fofa_q_cor_h
//   divergence  (B_c)_ij = int phi_i d phi_j / d x_c          (right-hand side of eq. fofa_q_cor_h,
//                                                              and int p div v through B_c^T)
//   surface     (M_s)_ij = int_{Gamma_s} phi_i phi_j ds       (wind-tension load)
//
// The assembly is row-wise: every row gathers the contributions of the
// tetrahedra around its node, in tetrahedron order, so rows are independent
// (threads need no atomics), entry (i,j) and (j,i) receive the same products
// in the same order (the matrix is bitwise symmetric), and the result does
// not depend on the thread count.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <thread>

#include "hns_internal.h"

namespace hns {

namespace {

template <class F>
void parallel_for(int64_t n, F &&f)
{
    unsigned nt = std::max(1u, std::thread::hardware_concurrency());
    nt = (unsigned)std::min<int64_t>(nt, std::max<int64_t>(1, n / 4096));
    if (nt <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        int64_t lo = t * chunk, hi = std::min<int64_t>(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto &t : th) t.join();
}

struct TetGeom {
    double g[4][3];  // gradients of the hat functions
    double vol;      // volume (positive for a valid tetrahedron)
};

// Hat-function gradients by cofactors: with edges e_a = X_a - X_0 (a=1..3)
// and D = e_1 . (e_2 x e_3), grad(lambda_1) = (e_2 x e_3)/D,
// grad(lambda_2) = (e_3 x e_1)/D, grad(lambda_3) = (e_1 x e_2)/D and
// grad(lambda_0) = -(sum of the other three); volume D/6.
inline void cross(const double *u, const double *v, double *w)
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

inline TetGeom tet_geometry(const double *xyz, const int32_t *t)
{
    const double *X0 = xyz + 3 * (int64_t)t[0];
    double e[3][3];
    for (int a = 0; a < 3; ++a) {
        const double *Xa = xyz + 3 * (int64_t)t[a + 1];
        for (int d = 0; d < 3; ++d) e[a][d] = Xa[d] - X0[d];
    }
    TetGeom G;
    double c1[3], c2[3], c3[3];
    cross(e[1], e[2], c1);
    cross(e[2], e[0], c2);
    cross(e[0], e[1], c3);
    double D = e[0][0] * c1[0] + e[0][1] * c1[1] + e[0][2] * c1[2];
    G.vol = D / 6.0;
    double inv = 1.0 / D;
    for (int d = 0; d < 3; ++d) {
        G.g[1][d] = c1[d] * inv;
        G.g[2][d] = c2[d] * inv;
        G.g[3][d] = c3[d] * inv;
        G.g[0][d] = -(G.g[1][d] + G.g[2][d] + G.g[3][d]);
    }
    return G;
}

// node -> incident tetrahedra (ascending tetrahedron index), as CSR
struct Incidence {
    std::vector<int64_t> ptr;
    std::vector<int32_t> tet;  // tetrahedron index
    std::vector<int8_t> loc;   // local vertex number of the node in that tetrahedron
};

// Counts and fills run in parallel (atomic per-node cursors); each node's
// list is then sorted by element index, so the result is the serial one.
Incidence build_incidence(int64_t n, int64_t ne, int nloc, const int32_t *conn)
{
    Incidence inc;
    std::vector<std::atomic<int64_t>> cnt(n);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) cnt[i].store(0, std::memory_order_relaxed);
    });
    parallel_for(ne, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo * nloc; e < hi * nloc; ++e)
            cnt[conn[e]].fetch_add(1, std::memory_order_relaxed);
    });
    inc.ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) inc.ptr[i + 1] = inc.ptr[i] + cnt[i].load();
    inc.tet.resize(inc.ptr[n]);
    inc.loc.resize(inc.ptr[n]);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) cnt[i].store(inc.ptr[i], std::memory_order_relaxed);
    });
    parallel_for(ne, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e)
            for (int a = 0; a < nloc; ++a) {
                const int64_t s = cnt[conn[e * nloc + a]].fetch_add(1, std::memory_order_relaxed);
                inc.tet[s] = (int32_t)e;
                inc.loc[s] = (int8_t)a;
            }
    });
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            // insertion sort of the (element, local vertex) pairs by element
            for (int64_t s = inc.ptr[i] + 1; s < inc.ptr[i + 1]; ++s) {
                const int32_t t = inc.tet[s];
                const int8_t l = inc.loc[s];
                int64_t r = s;
                while (r > inc.ptr[i] && inc.tet[r - 1] > t) {
                    inc.tet[r] = inc.tet[r - 1];
                    inc.loc[r] = inc.loc[r - 1];
                    --r;
                }
                inc.tet[r] = t;
                inc.loc[r] = l;
            }
        }
    });
    return inc;
}

// Sparsity: row i holds every node sharing an element with node i.
void build_pattern(int64_t n, int nloc, const int32_t *conn, const Incidence &inc, HostCSR &A)
{
    A.n = n;
    A.rowptr.assign(n + 1, 0);
    std::vector<int32_t> len(n);
    auto row_cols = [&](int64_t i, std::vector<int32_t> &buf) {
        buf.clear();
        for (int64_t s = inc.ptr[i]; s < inc.ptr[i + 1]; ++s)
            for (int b = 0; b < nloc; ++b) buf.push_back(conn[(int64_t)inc.tet[s] * nloc + b]);
        if (buf.empty()) buf.push_back((int32_t)i);  // isolated node: keep a diagonal
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    // one pass: every range of rows keeps its columns, then they are placed
    std::vector<std::pair<int64_t, std::vector<int32_t>>> parts;
    std::mutex pm;
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> buf, all;
        for (int64_t i = lo; i < hi; ++i) {
            row_cols(i, buf);
            len[i] = (int32_t)buf.size();
            all.insert(all.end(), buf.begin(), buf.end());
        }
        std::lock_guard<std::mutex> g(pm);
        parts.emplace_back(lo, std::move(all));
    });
    for (int64_t i = 0; i < n; ++i) A.rowptr[i + 1] = A.rowptr[i] + len[i];
    A.col.resize(A.rowptr[n]);
    A.val.assign(A.rowptr[n], 0.0);
    for (const auto &pt : parts)
        std::copy(pt.second.begin(), pt.second.end(), A.col.begin() + A.rowptr[pt.first]);
}

inline int64_t find_col(const HostCSR &A, int64_t row, int32_t c)
{
    const int32_t *b = A.col.data() + A.rowptr[row];
    const int32_t *e = A.col.data() + A.rowptr[row + 1];
    const int32_t *p = std::lower_bound(b, e, c);
    return (p != e && *p == c) ? (p - A.col.data()) : -1;
}

hns_status check_mesh(const hns_mesh *m)
{
    HNS_TRY(check_mesh_arrays(m));
    for (int64_t e = 0; e < 4 * m->n_tets; ++e)
        if (m->tets[e] < 0 || m->tets[e] >= m->n_nodes) {
            set_error("mesh: tetrahedron %lld references node %d outside [0,%lld)",
                      (long long)(e / 4), m->tets[e], (long long)m->n_nodes);
            return HNS_ERR_MESH;
        }
    for (int64_t i = 0; i < 3 * m->n_nodes; ++i)
        if (!std::isfinite(m->xyz[i])) {
            set_error("mesh: non-finite coordinate at node %lld", (long long)(i / 3));
            return HNS_ERR_MESH;
        }
    return HNS_OK;
}

}  // namespace

hns_status check_mesh_arrays(const hns_mesh *m)
{
    if (!m || m->n_nodes <= 0 || m->n_tets < 0 || !m->xyz || (m->n_tets > 0 && !m->tets)) {
        set_error("mesh: null arrays or non-positive sizes");
        return HNS_ERR_INVALID;
    }
    if (m->n_nodes >= (int64_t)INT32_MAX) {
        set_error("mesh: %lld nodes exceed the int32 index range", (long long)m->n_nodes);
        return HNS_ERR_INVALID;
    }
    return HNS_OK;
}

hns_status assemble_host(const hns_mesh *mesh, double c_mass, double c_stiff, double nu_h,
                         double nu_v, HostCSR &A, std::vector<double> *lumped, bool values_on_device)
{
    HNS_TRY(check_mesh(mesh));
    const int64_t n = mesh->n_nodes, ne = mesh->n_tets;
    const double *xyz = mesh->xyz;
    const int32_t *tets = mesh->tets;

    if (values_on_device) {
        // pattern here, values (and the volume check) by the device kernel
        Incidence inc = build_incidence(n, ne, 4, tets);
        build_pattern(n, 4, tets, inc, A);
        if ((int64_t)A.col.size() >= (int64_t)INT32_MAX) {
            set_error("operator has %zu nonzeros, beyond the int32 range", A.col.size());
            return HNS_ERR_INVALID;
        }
        return assemble_values_device(mesh, inc.ptr, inc.tet, inc.loc, A, c_mass, c_stiff, nu_h,
                                      nu_v, lumped);
    }

    // element validity first (positive volume)
    std::atomic<int64_t> bad{-1};
    parallel_for(ne, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            TetGeom G = tet_geometry(xyz, tets + 4 * e);
            if (!(G.vol > 0.0) || !std::isfinite(G.vol)) {
                bad.store(e);
                return;
            }
        }
    });
    if (bad.load() >= 0) {
        set_error("mesh: tetrahedron %lld has non-positive volume", (long long)bad.load());
        return HNS_ERR_MESH;
    }

    Incidence inc = build_incidence(n, ne, 4, tets);
    build_pattern(n, 4, tets, inc, A);
    if ((int64_t)A.col.size() >= (int64_t)INT32_MAX) {
        set_error("operator has %zu nonzeros, beyond the int32 range", A.col.size());
        return HNS_ERR_INVALID;
    }
    if (lumped) lumped->assign(n, 0.0);
    const double nu[3] = {nu_h, nu_h, nu_v};
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            double mi = 0.0;
            for (int64_t s = inc.ptr[i]; s < inc.ptr[i + 1]; ++s) {
                const int32_t *t = tets + 4 * (int64_t)inc.tet[s];
                const int a = inc.loc[s];
                TetGeom G = tet_geometry(xyz, t);
                mi += G.vol / 4.0;
                for (int b = 0; b < 4; ++b) {
                    double k = 0.0;
                    for (int d = 0; d < 3; ++d) k += nu[d] * (G.g[a][d] * G.g[b][d]);
                    k *= G.vol;
                    double m = (a == b) ? G.vol / 10.0 : G.vol / 20.0;
                    A.val[find_col(A, i, t[b])] += c_mass * m + c_stiff * k;
                }
            }
            if (lumped) (*lumped)[i] = mi;
        }
    });
    return HNS_OK;
}

hns_status assemble_divergence_host(const hns_mesh *mesh, const HostCSR &pattern, int comp,
                                    HostCSR &B)
{
    HNS_TRY(check_mesh(mesh));
    const int64_t n = mesh->n_nodes, ne = mesh->n_tets;
    Incidence inc = build_incidence(n, ne, 4, mesh->tets);
    B.n = n;
    B.rowptr = pattern.rowptr;
    B.col = pattern.col;
    B.val.assign(pattern.col.size(), 0.0);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t s = inc.ptr[i]; s < inc.ptr[i + 1]; ++s) {
                const int32_t *t = mesh->tets + 4 * (int64_t)inc.tet[s];
                TetGeom G = tet_geometry(mesh->xyz, t);
                // int_T phi_a d phi_b / d x_c = (vol / 4) * d phi_b / d x_c
                for (int b = 0; b < 4; ++b)
                    B.val[find_col(B, i, t[b])] += (G.vol / 4.0) * G.g[b][comp];
            }
    });
    return HNS_OK;
}

hns_status assemble_surface_mass_host(const hns_mesh *mesh, HostCSR &Ms)
{
    const int64_t n = mesh->n_nodes, nt = mesh->n_surf_tris;
    if (nt <= 0 || !mesh->surf_tris) {
        set_error("surface mass needs the surface triangles");
        return HNS_ERR_INVALID;
    }
    for (int64_t e = 0; e < 3 * nt; ++e)
        if (mesh->surf_tris[e] < 0 || mesh->surf_tris[e] >= n) {
            set_error("surface triangle %lld references a node out of range", (long long)(e / 3));
            return HNS_ERR_MESH;
        }
    Incidence inc = build_incidence(n, nt, 3, mesh->surf_tris);
    build_pattern(n, 3, mesh->surf_tris, inc, Ms);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t s = inc.ptr[i]; s < inc.ptr[i + 1]; ++s) {
                const int32_t *t = mesh->surf_tris + 3 * (int64_t)inc.tet[s];
                const int a = inc.loc[s];
                const double *P0 = mesh->xyz + 3 * (int64_t)t[0];
                const double *P1 = mesh->xyz + 3 * (int64_t)t[1];
                const double *P2 = mesh->xyz + 3 * (int64_t)t[2];
                double u[3], v[3], w[3];
                for (int d = 0; d < 3; ++d) {
                    u[d] = P1[d] - P0[d];
                    v[d] = P2[d] - P0[d];
                }
                cross(u, v, w);
                double area = 0.5 * std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
                for (int b = 0; b < 3; ++b)
                    Ms.val[find_col(Ms, i, t[b])] += (a == b) ? area / 6.0 : area / 12.0;
            }
    });
    return HNS_OK;
}

void transpose_values(const HostCSR &A, HostCSR &At)
{
    At.n = A.n;
    At.rowptr = A.rowptr;
    At.col = A.col;
    At.val.assign(A.val.size(), 0.0);
    parallel_for(A.n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i)
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
                At.val[k] = A.val[find_col(A, A.col[k], (int32_t)i)];
    });
}

// ---------------------------------------------------------------------------
// Device upload
// ---------------------------------------------------------------------------

size_t DevMatrix::bytes() const
{
    size_t b = 0;
    if (fmt == HNS_FMT_SDIA) {
        const size_t arrays = (size_t)ndiag + (unit ? 0 : 1);
        if (dia) b += arrays * n * 8;
        if (dia32) b += arrays * n * 4;
    } else if (fmt == HNS_FMT_CSR) {
        b += (size_t)(n + 1) * 4 + (size_t)nnz * 12;
        if (val32) b += (size_t)nnz * 4;
    } else if (fmt == HNS_MATRIX_FREE) {
        b += (size_t)mf_ne * (nloc() * 4 + 24 * 8) + (size_t)(n + 1) * 8 +
             (size_t)mf_ne * nloc() * 4;
    } else {
        b += (size_t)(nslices + 1) * 4 + (size_t)sell_len * 12;
        if (sval32) b += (size_t)sell_len * 4;
    }
    return b;
}

void DevMatrix::release()
{
    void *ptrs[] = {rowptr, col,    val,     val32,     slice_ptr, scol,  sval,
                    sval32, dia,    dia32,   mf_nodes,  mf_corner, mf_ptr, mf_pos};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    rowptr = col = slice_ptr = scol = nullptr;
    val = sval = dia = nullptr;
    val32 = sval32 = dia32 = nullptr;
    mf_nodes = mf_pos = nullptr;
    mf_corner = nullptr;
    mf_ptr = nullptr;
}

// Offsets j - i of the upper triangle when the matrix is bitwise symmetric
// and uses at most kMaxDiagWide distinct upper offsets; empty otherwise.
static std::vector<int32_t> symmetric_offsets(const HostCSR &h)
{
    // distinct upper offsets per range of rows, merged; then the bitwise
    // symmetry of values and pattern, in parallel
    std::vector<int32_t> offs;
    std::mutex om;
    std::atomic<bool> too_many{false}, asym{false};
    parallel_for(h.n, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> mine;
        for (int64_t i = lo; i < hi && !too_many.load(std::memory_order_relaxed); ++i)
            for (int32_t k = h.rowptr[i]; k < h.rowptr[i + 1]; ++k) {
                const int64_t d = (int64_t)h.col[k] - i;
                if (d <= 0) continue;
                if (std::find(mine.begin(), mine.end(), (int32_t)d) == mine.end()) {
                    mine.push_back((int32_t)d);
                    if ((int)mine.size() > kMaxDiagWide) {
                        too_many.store(true);
                        break;
                    }
                }
            }
        std::lock_guard<std::mutex> g(om);
        for (int32_t d : mine)
            if (std::find(offs.begin(), offs.end(), d) == offs.end()) offs.push_back(d);
    });
    if (too_many.load() || (int)offs.size() > kMaxDiagWide) return {};
    parallel_for(h.n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi && !asym.load(std::memory_order_relaxed); ++i)
            for (int32_t k = h.rowptr[i]; k < h.rowptr[i + 1]; ++k) {
                const int64_t j = h.col[k];
                if (j <= i) continue;
                const int64_t t = find_col(h, j, (int32_t)i);
                if (t < 0 || h.val[t] != h.val[k]) {
                    asym.store(true);
                    break;
                }
            }
    });
    if (asym.load()) return {};
    std::sort(offs.begin(), offs.end());
    return offs;
}

uint32_t choose_format(const HostCSR &h)
{
    // Diagonal storage reads (ndiag + 1) n values and no indices, zeros
    // included; beyond the unrolled kernels' limit it is taken only when that
    // is fewer bytes than the values and column indices of CSR.
    const std::vector<int32_t> offs = symmetric_offsets(h);
    if (!offs.empty()) {
        if ((int)offs.size() <= kMaxDiag) return HNS_FMT_SDIA;
        if ((double)(offs.size() + 1) * h.n * 8.0 < 12.0 * (double)h.nnz()) return HNS_FMT_SDIA;
    }
    // Sliced ELL pays when rows inside a 64-row slice have similar lengths
    // (padding stays small); the structured basin meshes give < 5 % padding.
    int64_t n = h.n, padded = 0;
    for (int64_t s = 0; s * kSlice < n; ++s) {
        int32_t w = 0;
        for (int64_t r = s * kSlice; r < std::min<int64_t>(n, (s + 1) * kSlice); ++r)
            w = std::max(w, h.rowptr[r + 1] - h.rowptr[r]);
        padded += (int64_t)w * kSlice;
    }
    return (padded <= h.nnz() + h.nnz() / 5) ? HNS_FMT_SELL : HNS_FMT_CSR;
}

template <class T>
static hns_status upload(const std::vector<T> &v, T **dst)
{
    *dst = nullptr;
    if (v.empty()) return HNS_OK;
    hipError_t e = hipMalloc((void **)dst, v.size() * sizeof(T));
    if (e != hipSuccess) {
        *dst = nullptr;
        set_error("hipMalloc of %zu bytes failed: %s", v.size() * sizeof(T), hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? HNS_ERR_OOM : HNS_ERR_HIP;
    }
    HNS_TRY_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return HNS_OK;
}

hns_status upload_matrix(const HostCSR &h, uint32_t fmt, bool keep32, DevMatrix &d)
{
    d.n = h.n;
    d.nnz = h.nnz();
    d.fmt = fmt;
    if (fmt == HNS_FMT_SDIA) {
        std::vector<int32_t> offs = symmetric_offsets(h);
        if (offs.empty()) {
            set_error("symmetric-diagonal storage needs a bitwise-symmetric matrix with at most "
                      "%d upper diagonal offsets",
                      kMaxDiagWide);
            return HNS_ERR_INVALID;
        }
        const int64_t n = h.n;
        d.ndiag = (int)offs.size();
        for (int k = 0; k < d.ndiag; ++k) d.off[k] = offs[k];
        std::vector<double> dia((size_t)(d.ndiag + 1) * n, 0.0);
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i)
                for (int32_t k = h.rowptr[i]; k < h.rowptr[i + 1]; ++k) {
                    const int64_t dj = (int64_t)h.col[k] - i;
                    if (dj < 0) continue;
                    int slot = 0;
                    if (dj > 0)
                        slot = 1 + (int)(std::lower_bound(offs.begin(), offs.end(), (int32_t)dj) -
                                         offs.begin());
                    dia[(size_t)slot * n + i] = h.val[k];
                }
        });
        HNS_TRY(upload(dia, &d.dia));
        if (keep32) {
            std::vector<float> d32(dia.begin(), dia.end());
            HNS_TRY(upload(d32, &d.dia32));
        }
        return HNS_OK;
    }
    if (fmt == HNS_FMT_CSR) {
        HNS_TRY(upload(h.rowptr, &d.rowptr));
        HNS_TRY(upload(h.col, &d.col));
        HNS_TRY(upload(h.val, &d.val));
        if (keep32) {
            std::vector<float> v32(h.val.begin(), h.val.end());
            HNS_TRY(upload(v32, &d.val32));
        }
        return HNS_OK;
    }
    // sliced ELL, slice height 64, padding entries point at the row itself
    // with value 0 (rows past n point at node n-1)
    const int64_t n = h.n;
    d.nslices = (n + kSlice - 1) / kSlice;
    std::vector<int32_t> sptr(d.nslices + 1, 0);
    for (int64_t s = 0; s < d.nslices; ++s) {
        int32_t w = 0;
        for (int64_t r = s * kSlice; r < std::min<int64_t>(n, (s + 1) * kSlice); ++r)
            w = std::max(w, h.rowptr[r + 1] - h.rowptr[r]);
        if ((int64_t)sptr[s] + (int64_t)w * kSlice >= (int64_t)INT32_MAX) {
            set_error("sliced-ELL storage exceeds the int32 range");
            return HNS_ERR_INVALID;
        }
        sptr[s + 1] = sptr[s] + w * kSlice;
    }
    d.sell_len = sptr[d.nslices];
    std::vector<int32_t> scol(d.sell_len);
    std::vector<double> sval(d.sell_len, 0.0);
    parallel_for(d.nslices, [&](int64_t lo, int64_t hi) {
        for (int64_t s = lo; s < hi; ++s) {
            int32_t w = (sptr[s + 1] - sptr[s]) / kSlice;
            for (int l = 0; l < kSlice; ++l) {
                int64_t r = s * kSlice + l;
                int32_t rr = (int32_t)std::min<int64_t>(r, n - 1);
                int32_t len = r < n ? h.rowptr[r + 1] - h.rowptr[r] : 0;
                for (int32_t j = 0; j < w; ++j) {
                    int64_t k = sptr[s] + (int64_t)j * kSlice + l;
                    if (j < len) {
                        scol[k] = h.col[h.rowptr[r] + j];
                        sval[k] = h.val[h.rowptr[r] + j];
                    } else {
                        scol[k] = rr;
                        sval[k] = 0.0;
                    }
                }
            }
        }
    });
    HNS_TRY(upload(sptr, &d.slice_ptr));
    HNS_TRY(upload(scol, &d.scol));
    HNS_TRY(upload(sval, &d.sval));
    if (keep32) {
        std::vector<float> v32(sval.begin(), sval.end());
        HNS_TRY(upload(v32, &d.sval32));
    }
    return HNS_OK;
}

// ---------------------------------------------------------------------------
// Brick elements (Sec. 5): Q2 velocity and Q1 pressure spaces
// ---------------------------------------------------------------------------
namespace {

// Reference tables at the tensor Gauss points (p + 1 per direction, exact
// for the mass and stiffness forms on parallelepipeds), reference cube
// [-1, 1]^3, local node (a, b, c) at a + (p+1) b + (p+1)^2 c.
struct BrickTables {
    int p = 0, q = 0, nloc = 0, nq = 0;
    std::vector<double> w;    // nq weights
    std::vector<double> N;    // nq x nloc basis values
    std::vector<double> dN;   // nq x nloc x 3 reference gradients
    std::vector<double> dC;   // nq x 8 x 3 reference gradients of the corner (trilinear) functions
};

// 1D Lagrange basis of degree p on the equispaced nodes of [-1, 1]
void basis_1d(int p, double s, double *v, double *d)
{
    if (p == 1) {
        v[0] = 0.5 * (1.0 - s);
        v[1] = 0.5 * (1.0 + s);
        d[0] = -0.5;
        d[1] = 0.5;
    } else {
        v[0] = 0.5 * s * (s - 1.0);
        v[1] = (1.0 - s) * (1.0 + s);
        v[2] = 0.5 * s * (s + 1.0);
        d[0] = s - 0.5;
        d[1] = -2.0 * s;
        d[2] = s + 0.5;
    }
}

BrickTables brick_tables(int p)
{
    BrickTables T;
    T.p = p;
    T.q = p + 1;
    T.nloc = T.q * T.q * T.q;
    T.nq = T.nloc;
    double gp[3], gw[3];
    if (p == 1) {
        const double g = std::sqrt(1.0 / 3.0);
        gp[0] = -g; gp[1] = g;
        gw[0] = gw[1] = 1.0;
    } else {
        const double g = std::sqrt(3.0 / 5.0);
        gp[0] = -g; gp[1] = 0.0; gp[2] = g;
        gw[0] = gw[2] = 5.0 / 9.0;
        gw[1] = 8.0 / 9.0;
    }
    T.w.resize(T.nq);
    T.N.resize((size_t)T.nq * T.nloc);
    T.dN.resize((size_t)T.nq * T.nloc * 3);
    T.dC.resize((size_t)T.nq * 24);
    const int q = T.q;
    for (int k = 0; k < q; ++k)
        for (int j = 0; j < q; ++j)
            for (int i = 0; i < q; ++i) {
                const int g = i + q * j + q * q * k;
                const double s[3] = {gp[i], gp[j], gp[k]};
                T.w[g] = gw[i] * gw[j] * gw[k];
                double v[3][3], d[3][3], lv[3][2], ld[3][2];
                for (int r = 0; r < 3; ++r) {
                    basis_1d(p, s[r], v[r], d[r]);
                    basis_1d(1, s[r], lv[r], ld[r]);
                }
                for (int c = 0; c < q; ++c)
                    for (int b = 0; b < q; ++b)
                        for (int a = 0; a < q; ++a) {
                            const int l = a + q * b + q * q * c;
                            T.N[(size_t)g * T.nloc + l] = v[0][a] * v[1][b] * v[2][c];
                            double *g3 = &T.dN[((size_t)g * T.nloc + l) * 3];
                            g3[0] = d[0][a] * v[1][b] * v[2][c];
                            g3[1] = v[0][a] * d[1][b] * v[2][c];
                            g3[2] = v[0][a] * v[1][b] * d[2][c];
                        }
                for (int c = 0; c < 8; ++c) {
                    const int a = c & 1, b = (c >> 1) & 1, e = c >> 2;
                    double *g3 = &T.dC[((size_t)g * 8 + c) * 3];
                    g3[0] = ld[0][a] * lv[1][b] * lv[2][e];
                    g3[1] = lv[0][a] * ld[1][b] * lv[2][e];
                    g3[2] = lv[0][a] * lv[1][b] * ld[2][e];
                }
            }
    return T;
}

// Element matrix c_mass M + c_stiff K_nu of one brick (nloc x nloc, row-major,
// exactly symmetric: the upper triangle is computed and mirrored) and the
// integrals of its basis functions.  Returns false if the Jacobian
// determinant is not positive at a quadrature point.
bool brick_matrix(const BrickTables &T, const double *xyz, const int32_t *h, double c_mass,
                  double c_stiff, const double nu[3], double *E, double *ints,
                  std::vector<double> &G)
{
    const int nloc = T.nloc, p = T.p, q = T.q;
    double X[8][3];
    for (int c = 0; c < 8; ++c) {
        const int l = (c & 1) * p + q * (((c >> 1) & 1) * p) + q * q * ((c >> 2) * p);
        for (int r = 0; r < 3; ++r) X[c][r] = xyz[3 * (int64_t)h[l] + r];
    }
    std::fill(E, E + (size_t)nloc * nloc, 0.0);
    std::fill(ints, ints + nloc, 0.0);
    G.resize((size_t)nloc * 3);
    for (int g = 0; g < T.nq; ++g) {
        // J[r][d] = d x_r / d s_d
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        const double *dc = &T.dC[(size_t)g * 24];
        for (int c = 0; c < 8; ++c)
            for (int r = 0; r < 3; ++r)
                for (int d = 0; d < 3; ++d) J[r][d] += X[c][r] * dc[3 * c + d];
        // adjugate: inv(J) = adj(J) / det
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
        if (!(det > 0.0) || !std::isfinite(det)) return false;
        const double inv = 1.0 / det;
        // physical gradient: grad phi_d = sum_s (d phi / d s_s) inv(J)[s][d]
        const double *dn = &T.dN[(size_t)g * nloc * 3];
        for (int a = 0; a < nloc; ++a)
            for (int d = 0; d < 3; ++d)
                G[3 * a + d] = (dn[3 * a] * A[0][d] + dn[3 * a + 1] * A[1][d] +
                                dn[3 * a + 2] * A[2][d]) * inv;
        const double wd = T.w[g] * det;
        const double *n = &T.N[(size_t)g * nloc];
        for (int a = 0; a < nloc; ++a) {
            ints[a] += wd * n[a];
            for (int b = a; b < nloc; ++b) {
                const double k = nu[0] * (G[3 * a] * G[3 * b]) +
                                 nu[1] * (G[3 * a + 1] * G[3 * b + 1]) +
                                 nu[2] * (G[3 * a + 2] * G[3 * b + 2]);
                E[(size_t)a * nloc + b] += wd * (c_mass * (n[a] * n[b]) + c_stiff * k);
            }
        }
    }
    for (int a = 0; a < nloc; ++a)
        for (int b = 0; b < a; ++b) E[(size_t)a * nloc + b] = E[(size_t)b * nloc + a];
    return true;
}

}  // namespace

hns_status assemble_hex_host(const hns_hex_mesh *mesh, double c_mass, double c_stiff,
                             double nu_h, double nu_v, HostCSR &A, std::vector<double> *lumped)
{
    if (!mesh || mesh->n_nodes <= 0 || mesh->n_hex < 0 || !mesh->xyz ||
        (mesh->n_hex > 0 && !mesh->hex)) {
        set_error("hex mesh: null arrays or non-positive sizes");
        return HNS_ERR_INVALID;
    }
    if (mesh->order != 1 && mesh->order != 2) {
        set_error("hex mesh: order must be 1 (Q1) or 2 (Q2), got %d", mesh->order);
        return HNS_ERR_INVALID;
    }
    if (mesh->n_nodes >= (int64_t)INT32_MAX) {
        set_error("hex mesh: %lld nodes exceed the int32 index range", (long long)mesh->n_nodes);
        return HNS_ERR_INVALID;
    }
    const int q = mesh->order + 1, nloc = q * q * q;
    const int64_t n = mesh->n_nodes, ne = mesh->n_hex;
    for (int64_t e = 0; e < ne * nloc; ++e)
        if (mesh->hex[e] < 0 || mesh->hex[e] >= n) {
            set_error("hex mesh: element %lld references node %d outside [0,%lld)",
                      (long long)(e / nloc), mesh->hex[e], (long long)n);
            return HNS_ERR_MESH;
        }
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(mesh->xyz[i])) {
            set_error("hex mesh: non-finite coordinate at node %lld", (long long)(i / 3));
            return HNS_ERR_MESH;
        }
    Incidence inc = build_incidence(n, ne, nloc, mesh->hex);
    build_pattern(n, nloc, mesh->hex, inc, A);
    if ((int64_t)A.col.size() >= (int64_t)INT32_MAX) {
        set_error("operator has %zu nonzeros, beyond the int32 range", A.col.size());
        return HNS_ERR_INVALID;
    }
    const BrickTables T = brick_tables(mesh->order);
    const double nu[3] = {nu_h, nu_h, nu_v};
    if (lumped) lumped->assign(n, 0.0);
    std::atomic<int64_t> bad{-1};
    // Each thread owns a range of rows and visits, in ascending order, every
    // element touching them (elements on a range boundary are computed by
    // both threads): a row sums its elements in ascending order whatever the
    // thread count, so the values are deterministic and, the element
    // matrices being exactly symmetric, bitwise symmetric.
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> els(inc.tet.begin() + inc.ptr[lo], inc.tet.begin() + inc.ptr[hi]);
        std::sort(els.begin(), els.end());
        els.erase(std::unique(els.begin(), els.end()), els.end());
        std::vector<double> E((size_t)nloc * nloc), ints(nloc), G;
        for (int32_t e : els) {
            const int32_t *h = mesh->hex + (int64_t)e * nloc;
            if (!brick_matrix(T, mesh->xyz, h, c_mass, c_stiff, nu, E.data(), ints.data(), G)) {
                bad.store(e);
                return;
            }
            for (int a = 0; a < nloc; ++a) {
                const int64_t i = h[a];
                if (i < lo || i >= hi) continue;
                for (int b = 0; b < nloc; ++b)
                    A.val[find_col(A, i, h[b])] += E[(size_t)a * nloc + b];
                if (lumped) (*lumped)[i] += ints[a];
            }
        }
    });
    if (bad.load() >= 0) {
        set_error("hex mesh: element %lld has a non-positive Jacobian determinant",
                  (long long)bad.load());
        return HNS_ERR_MESH;
    }
    return HNS_OK;
}

hns_status upload_matrix_free(const hns_hex_mesh *mesh, double c_mass, double c_stiff,
                              double nu_h, double nu_v, int64_t nnz, DevMatrix &d)
{
    const int p = mesh->order, q = p + 1, nloc = q * q * q;
    const int64_t n = mesh->n_nodes, ne = mesh->n_hex;
    if (ne * nloc >= (int64_t)INT32_MAX) {
        set_error("matrix-free bricks: %lld element nodes exceed the int32 range",
                  (long long)(ne * nloc));
        return HNS_ERR_INVALID;
    }
    d.n = n;
    d.nnz = nnz;
    d.fmt = HNS_MATRIX_FREE;
    d.mf_order = p;
    d.mf_ne = ne;
    d.mf_coef[0] = c_mass;
    d.mf_coef[1] = c_stiff;
    d.mf_coef[2] = nu_h;
    d.mf_coef[3] = nu_h;
    d.mf_coef[4] = nu_v;
    // 1D tables at the Gauss points (the points and weights of brick_tables)
    double gp[3] = {0, 0, 0};
    if (p == 1) {
        const double g = std::sqrt(1.0 / 3.0);
        gp[0] = -g;
        gp[1] = g;
        d.mf_gw[0] = d.mf_gw[1] = 1.0;
    } else {
        const double g = std::sqrt(3.0 / 5.0);
        gp[0] = -g;
        gp[1] = 0.0;
        gp[2] = g;
        d.mf_gw[0] = d.mf_gw[2] = 5.0 / 9.0;
        d.mf_gw[1] = 8.0 / 9.0;
    }
    for (int g = 0; g < q; ++g) {
        double v[3], dv[3], lv[2], ld[2];
        basis_1d(p, gp[g], v, dv);
        basis_1d(1, gp[g], lv, ld);
        for (int a = 0; a < q; ++a) {
            d.mf_V[a][g] = v[a];
            d.mf_D[a][g] = dv[a];
        }
        for (int a = 0; a < 2; ++a) {
            d.mf_LV[a][g] = lv[a];
            d.mf_LD[a][g] = ld[a];
        }
    }
    // corners: local node (a, b, c) with a, b, c in {0, p}, corner index
    // a' + 2 b' + 4 c' (a' = a / p)
    std::vector<double> corner((size_t)ne * 24);
    parallel_for(ne, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            const int32_t *h = mesh->hex + e * nloc;
            for (int c = 0; c < 8; ++c) {
                const int l = (c & 1) * p + q * (((c >> 1) & 1) * p) + q * q * ((c >> 2) * p);
                for (int r = 0; r < 3; ++r) corner[(size_t)e * 24 + 3 * c + r] =
                    mesh->xyz[3 * (int64_t)h[l] + r];
            }
        }
    });
    // node i's (element, local node) pairs in ascending element order at
    // positions ptr[i] .. ptr[i+1]; pos[e nloc + a] = the position of (e, a)
    Incidence inc = build_incidence(n, ne, nloc, mesh->hex);
    std::vector<int32_t> pos(inc.tet.size());
    for (size_t k = 0; k < pos.size(); ++k) pos[(size_t)inc.tet[k] * nloc + inc.loc[k]] = (int32_t)k;
    std::vector<int32_t> nodes(mesh->hex, mesh->hex + ne * nloc);
    HNS_TRY(upload(nodes, &d.mf_nodes));
    HNS_TRY(upload(corner, &d.mf_corner));
    HNS_TRY(upload(inc.ptr, &d.mf_ptr));
    HNS_TRY(upload(pos, &d.mf_pos));
    return HNS_OK;
}

void tet_incidence(int64_t n, int64_t ntet, const int32_t *tets, std::vector<int64_t> &ptr,
                   std::vector<int32_t> &tet, std::vector<int8_t> &loc)
{
    Incidence inc = build_incidence(n, ntet, 4, tets);
    ptr = std::move(inc.ptr);
    tet = std::move(inc.tet);
    loc = std::move(inc.loc);
}

}  // namespace hns
