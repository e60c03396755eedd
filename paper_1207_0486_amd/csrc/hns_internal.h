// Internal declarations of the hns library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "hns.h"

namespace hns {

void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

#define HNS_TRY_HIP(call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::hns::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                      \
            return HNS_ERR_HIP;                                                              \
        }                                                                                    \
    } while (0)

#define HNS_TRY(expr)                       \
    do {                                    \
        hns_status s_ = (expr);             \
        if (s_ < 0) return s_;              \
    } while (0)

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts)
constexpr int kSlice = 64;       // sliced-ELL slice height = one wavefront
constexpr int kMaxGrid = 2048;   // workgroups of the reducing kernels (multiple of 8 XCDs)
constexpr int kMaxPart = 4096;   // workgroups of the single-vector CG kernels (partials slots)
constexpr int kMaxDiag = 16;     // upper diagonals of the unrolled symmetric-diagonal kernels
constexpr int kMaxDiagWide = 64; // upper diagonals of the grouped (wide) kernels

// ---------------------------------------------------------------------------
// Host-side compressed sparse rows (assembly output)
// ---------------------------------------------------------------------------
struct HostCSR {
    int64_t n = 0;
    std::vector<int32_t> rowptr;  // n+1
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

// ---------------------------------------------------------------------------
// Device matrix in one of the storage formats, FP64 and optional FP32 values.
// ---------------------------------------------------------------------------
// FP64-vector diagonal SpMV: one row per lane below this many rows (more
// workgroups where the product is latency-bound), two at and above it
constexpr int64_t kOneRowMax = 250000;

struct DevMatrix {
    int64_t n = 0;
    int64_t nnz = 0;        // structural nonzeros (CSR)
    uint32_t fmt = HNS_FMT_CSR;
    // CSR
    int32_t *rowptr = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    float *val32 = nullptr;
    // sliced ELL: slice s holds rows [64 s, 64 s + 64); entry j of lane l is
    // at slice_ptr[s] + 64 j + l (column-major inside the slice)
    int64_t nslices = 0;
    int64_t sell_len = 0;   // padded entries
    int32_t *slice_ptr = nullptr;
    int32_t *scol = nullptr;
    double *sval = nullptr;
    float *sval32 = nullptr;
    // symmetric diagonal storage (ndiag <= kMaxDiag: unrolled kernels; up to
    // kMaxDiagWide: offsets streamed in groups of 8): the main diagonal and `ndiag` upper
    // diagonals at offsets off[0] < ... < off[ndiag-1]; array k (k = 0 main,
    // k >= 1 upper) holds entry (i, i + off[k-1]) at dia[k * n + i] (zero
    // where the entry is absent); the lower triangle is read by symmetry
    int ndiag = 0;
    int32_t off[kMaxDiagWide] = {0};
    double *dia = nullptr;
    float *dia32 = nullptr;
    // unit: a symmetrically Jacobi-scaled operator (main diagonal 1, not
    // stored): array k = 0 .. ndiag-1 holds upper diagonal k (unrolled
    // kernels only, products of the CG iteration only)
    bool unit = false;
    // launch shape of the single-vector CG kernels: workgroup-sized row
    // passes per block of the FP64-vector and FP32-vector diagonal SpMV, and
    // 16-byte packs per thread of the vector updates
    int spmv_it64 = 1;
    int spmv_it32 = 0;   // 0: by size, spmv_passes32()
    // workgroup-sized passes per block of the FP32-vector diagonal SpMV:
    // spmv_it32 when set, else 1 below 500K rows (more workgroups where the
    // product is latency-bound), 2 above
    int spmv_passes32() const { return spmv_it32 > 0 ? spmv_it32 : n < 500000 ? 1 : 2; }
    int vec_it = 0;   // 0: by size, vec_packs()
    // rows per lane of the FP64-vector diagonal SpMV: 1 or 2, 0 by size
    int spmv_rows64 = 0;
    int rows_per_lane64() const { return spmv_rows64 > 0 ? spmv_rows64 : n < kOneRowMax ? 1 : 2; }
    // packs per thread of the vector updates: vec_it when set, else more
    // workgroups on smaller operators (measured per pressure iteration on the
    // basin operators: 1 pack below 250K rows, 2 below 1M, 3 above)
    int vec_packs() const { return vec_it > 0 ? vec_it : n < 250000 ? 1 : n < 1000000 ? 2 : 3; }
    // matrix-free bricks (fmt == HNS_MATRIX_FREE): the product is computed
    // element by element; per element its (order+1)^3 nodes (mf_nodes) and
    // its 8 corner coordinates (mf_corner, 24 doubles); the (element, local
    // node) pairs that touch node i take positions mf_ptr[i] .. mf_ptr[i+1]
    // of the scratch, in ascending element order, and mf_pos[e nloc + a] is
    // the position of pair (e, a); the coefficients of c_mass M + c_stiff
    // K_nu and the 1D Gauss tables (host copies, kernel arguments)
    int mf_order = 0;
    int64_t mf_ne = 0;
    int32_t *mf_nodes = nullptr;
    double *mf_corner = nullptr;
    int64_t *mf_ptr = nullptr;
    int32_t *mf_pos = nullptr;
    double mf_coef[5] = {0, 0, 0, 0, 0};   // c_mass, c_stiff, nu_x, nu_y, nu_z
    double mf_gw[3] = {0, 0, 0};           // Gauss weights
    double mf_V[3][3] = {}, mf_D[3][3] = {};   // basis a at point g: value, derivative
    double mf_LV[2][3] = {}, mf_LD[2][3] = {}; // trilinear corner basis at point g
    // doubles of per-product scratch (element outputs) a solve needs
    size_t mf_scratch() const { return fmt == HNS_MATRIX_FREE ? (size_t)mf_ne * nloc() : 0; }
    int nloc() const { return (mf_order + 1) * (mf_order + 1) * (mf_order + 1); }

    size_t bytes() const;
    void release();
};

// IC(0) in the greedy multicolour order, host side (ic0.cpp)
struct IC0Host {
    int64_t n = 0;
    int ncolors = 0;
    std::vector<int32_t> perm;     // permuted position -> node
    std::vector<int64_t> cstart;   // first position of each colour (ncolors + 1)
    std::vector<int64_t> lptr;     // strict lower factor by permuted rows
    std::vector<int32_t> lcol;
    std::vector<double> lval;
    std::vector<int64_t> uptr;     // its transpose (strict upper) by permuted rows
    std::vector<int32_t> ucol;
    std::vector<double> uval;
    std::vector<double> diag;      // L_ii
};
hns_status ic0_factor_host(const HostCSR &A, const uint8_t *bc, int bit, IC0Host &F);

// IC(0) factor on the device
// On the device the strict lower factor L and its transpose U are kept per
// colour in column-major padded rows: colour c's rows r0..r1 (nc = r1 - r0)
// hold entry k of row r0 + j at [base[c] + k nc + j] for k < width[c] (the
// colour's longest row), in the order of the host rows; lptr / uptr give
// each row's length.  Padding entries are column 0, value 0, never read.
struct IC0Dev {
    int64_t n = 0;
    int ncolors = 0;
    std::vector<int64_t> cstart;   // host copy of the colour starts
    std::vector<int64_t> lbase, ubase;   // host: start of each colour's block
    std::vector<int32_t> lwidth, uwidth;  // host: each colour's longest row
    int32_t *perm = nullptr;
    int64_t *lptr = nullptr, *uptr = nullptr;
    int32_t *lcol = nullptr, *ucol = nullptr;
    double *lval = nullptr, *uval = nullptr, *diag = nullptr;
    size_t bytes = 0;
    void release();
};

struct Scalars;           // device-side CG scalars (kernels.hip)
struct Workspace;         // per-solve device buffers (solve.hip)
struct BWorkspace;        // multi-right-hand-side buffers (batched.hip)

}  // namespace hns

struct hns_operator {
    int device = 0;
    uint32_t flags = 0;
    uint32_t kind = 0;      // HNS_POISSON or HNS_HELMHOLTZ
    int64_t n = 0;
    double nu_h = 0, nu_v = 0, dt = 0;
    hns::DevMatrix A;
    double *dinv = nullptr;     // 1 / diag(A)
    float *dinv32 = nullptr;
    uint8_t *bc = nullptr;      // Dirichlet bits (device), may be null
    double *lumped = nullptr;   // M 1 (mass-weighted mean of the Neumann answer)
    double lumped_sum = 0.0;
    int64_t bad_diag = -1;      // first non-positive diagonal entry, -1 if none
    int assembly = 0;           // 0 host, 1 values on the device, 2 the whole operator there
    // auxiliary forms for the step right-hand sides
    hns::DevMatrix M, B[3], Bt[3], Ms;
    bool has_aux = false;
    double *step_tmp = nullptr;   // 3 n doubles of scratch for the step kernels
    // mesh on the device for the advection term (HNS_STEP_AUX): coordinates
    // (n x 3), tetrahedra (ntet x 4) and the node -> tetrahedron incidence
    int64_t ntet = 0;
    double *mesh_xyz = nullptr;
    int32_t *mesh_tets = nullptr;
    int64_t *inc_ptr = nullptr;
    int32_t *inc_tet = nullptr;
    int8_t *inc_loc = nullptr;
    // tunables
    int check_every = 32;
    int64_t small_n = 4096;       // single-workgroup CG chunks up to this many rows (0: never)
    double inner_tol = 1e-5;
    int max_outer = 30;
    int mixed_variant = 0;        // 0 FP32 + replacement, 1 restarted refinement,
                                  // 2 FP32 storage with FP64 vectors
    double replace_drop = 0;      // FP32 residual drop that triggers a replacement (0: by size)
    int use_graph = 0;
    // kernel timing (hns_profile_*)
    int profile = 0;
    double prof_ms[6] = {0, 0, 0, 0, 0, 0};
    int64_t prof_count[6] = {0, 0, 0, 0, 0, 0};
    // workspaces, reused across solves
    std::mutex ws_mutex;
    std::vector<hns::Workspace *> ws_free;
    std::vector<hns::BWorkspace *> bws_free;
    int bspmm_vec = 0;                     // 0: autotune per (k, mode); else 1, 2 or 4
    int bspmm_tile = -1;                   // tiled product: -1 autotune, 0 never, 1..3 shape
    std::vector<std::array<int, 3>> tuned; // (k, mixed, V) chosen by the autotuner
    // vertical-line preconditioner: the rows form water columns of line_len
    // consecutive nodes (0 when the numbering has none).  Host copies of the
    // column blocks (diagonal; coupling to the next node of the column, 0 at
    // the column top) and of the Dirichlet bits; device factors per mask
    // (index mask_bit + 1: masked off-diagonal, then inverse pivots, 2 n
    // doubles), built on first use.
    int line_len = 0;
    int precond = 0;                       // 0 point Jacobi, 1 vertical-line blocks
    std::vector<double> line_d, line_e;
    std::vector<uint8_t> bc_host;
    std::mutex line_mutex;
    double *line_fac[9] = {nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, nullptr, nullptr};
    float *line_fac32[9] = {nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, nullptr, nullptr};   // FP32 copies (mixed)
    // Jacobi scaling (jacobi_scaling = 1): point-Jacobi solves on an operator
    // in the unrolled symmetric-diagonal format run plain CG on the
    // unit-diagonal D^-1/2 A D^-1/2 (S, FP64 and, when A keeps FP32 values,
    // FP32), with s = D^-1/2 and w = diag(A) in FP32; built on first use
    // (under line_mutex).
    int jacobi_scaling = 1;
    // scaled point-Jacobi iterations in two launches (the direction update
    // inside the next product, p in two buffers; the same arithmetic):
    // -1 by vector size, 0 never, 1 always
    int fuse_dir = -1;
    // batch sessions: 0 per-slot recurrences up to 2 slots, the shared
    // multi-right-hand-side block above; 1 always the block; 2 always per slot
    int session_mode = 0;
    hns::DevMatrix S;
    double *jac_s = nullptr;
    float *jac_w = nullptr;
    // IC(0) preconditioner (precond = 2): host copy of the assembled matrix
    // (kept with HNS_KEEP_HOST) and the device factors per mask (index bit + 1)
    hns::HostCSR host_A;
    hns::IC0Dev *ic0_fac[9] = {nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr};
};

namespace hns {

// Drop of the FP32 recursive residual between FP64 residual replacements: the
// "replace_drop" tunable when set, else 1e-3 where the FP32 recurrence runs in
// one workgroup (the two host round trips of each replacement outweigh the
// iterations between them there) and 0.1 elsewhere.
inline double replace_drop_of(const hns_operator *op, bool one_workgroup)
{
    if (op->replace_drop > 0) return op->replace_drop;
    return one_workgroup ? 1e-3 : 0.1;
}

// per-slot batch sessions (solve.hip)
struct SlotSession;
bool slot_session_wanted(const hns_operator *op, int capacity);
size_t slot_session_bytes(const hns_operator *op, int capacity, bool mixed);
hns_status slot_session_open(hns_operator *op, int capacity, bool mixed, SlotSession **out);
void slot_session_close(SlotSession *ss);
hns_status slot_session_add(SlotSession *ss, int count, const int *slots, const int *mask_bits,
                            const double *const *b_devs, const double *tols,
                            const int *max_iters, hipStream_t s);
hns_status slot_session_advance(SlotSession *ss, int iterations, hipStream_t s, int *active_out);
hns_status slot_session_poll(SlotSession *ss, int *states, hns_solve_info *infos);
hns_status slot_session_take(SlotSession *ss, int slot, double *x_dev, hns_solve_info *info,
                             hipStream_t s);

// batched.hip
hns_status create_bworkspace(int64_t n, int K, bool mixed, BWorkspace **out);
void destroy_bworkspace(BWorkspace *w);
size_t bworkspace_bytes(int64_t n, int K, bool mixed);
int bworkspace_k(const BWorkspace *w);
bool bworkspace_mixed(const BWorkspace *w);
hns_status solve_batched_impl(hns_operator *op, BWorkspace *w, int K, const int *bits,
                              const double *B, double *X, double tol, int max_iter, bool mixed,
                              int V, hipStream_t s, hns_solve_info *infos);
// Product plan of the multi-right-hand-side solves: plan = V + 8 s, V the
// width (1, 2, 4) of the grid-stride iteration kernels, s the LDS-tiled
// product shape (0: none, 1..kTileShapesAbi).  tune_batched times the widths
// into times_us[0..2] and the tiled shapes into times_us[3..] (-1 where one
// does not apply) and returns the fastest plan; plan_cache_get/put read and
// write the plans kept across processes under plan_key(op, K, mixed).
constexpr int kTileShapesAbi = 3;
hns_status tune_batched(hns_operator *op, BWorkspace *w, int K, bool mixed, hipStream_t s,
                        double *times_us, int *best_plan);
std::string plan_key(const hns_operator *op, int K, bool mixed);
bool plan_cache_get(const std::string &key, int *plan);
void plan_cache_put(const std::string &key, int plan);
hns_status batched_plan(hns_operator *op, BWorkspace *w, int k, bool mixed, hipStream_t s,
                        int *plan);

// assemble.cpp
// null arrays, sizes and the int32 node range of a tetrahedral mesh
hns_status check_mesh_arrays(const hns_mesh *m);
// values_on_device: the pattern is built here, the values (and the element
// volume check) by a device kernel in the same order as the host loop
hns_status assemble_host(const hns_mesh *mesh, double c_mass, double c_stiff, double nu_h,
                         double nu_v, HostCSR &A, std::vector<double> *lumped,
                         bool values_on_device = false);
// assemble_gpu.hip
hns_status assemble_values_device(const hns_mesh *mesh, const std::vector<int64_t> &inc_ptr,
                                  const std::vector<int32_t> &inc_tet,
                                  const std::vector<int8_t> &inc_loc, HostCSR &A, double c_mass,
                                  double c_stiff, double nu_h, double nu_v,
                                  std::vector<double> *lumped);
// The whole operator on the device in symmetric diagonal storage (A, D^-1,
// FP32 copies with keep32, lumped mass and its total, first non-positive
// diagonal, structural nonzeros): bitwise the host path's operator.  Checks
// the vertex indices and coordinates itself (check_mesh_arrays first).
// *applicable = false, with op untouched, where the element offsets do not
// fit the unrolled diagonal storage (then the host path builds it).
hns_status assemble_operator_device(const hns_mesh *mesh, double c_mass, double c_stiff,
                                    double nu_h, double nu_v, bool keep32, hns_operator *op,
                                    bool *applicable);
hns_status assemble_divergence_host(const hns_mesh *mesh, const HostCSR &pattern, int comp,
                                    HostCSR &B);
hns_status assemble_surface_mass_host(const hns_mesh *mesh, HostCSR &Ms);
hns_status upload_matrix(const HostCSR &h, uint32_t fmt, bool keep32, DevMatrix &d);
// same pattern, transposed values (the pattern must be structurally symmetric)
void transpose_values(const HostCSR &A, HostCSR &At);
uint32_t choose_format(const HostCSR &h);
// brick elements of order 1 or 2: c_mass M + c_stiff K_nu and the integrals
// of the basis functions (lumped)
hns_status assemble_hex_host(const hns_hex_mesh *mesh, double c_mass, double c_stiff,
                             double nu_h, double nu_v, HostCSR &A, std::vector<double> *lumped);
// The matrix-free form of the same operator on the device (fmt, order,
// element nodes and corners, node -> element lists, coefficients, 1D tables)
hns_status upload_matrix_free(const hns_hex_mesh *mesh, double c_mass, double c_stiff,
                              double nu_h, double nu_v, int64_t nnz, DevMatrix &d);
// node -> incident tetrahedra in ascending tetrahedron order (CSR), with the
// node's local vertex number in each
void tet_incidence(int64_t n, int64_t ntet, const int32_t *tets, std::vector<int64_t> &ptr,
                   std::vector<int32_t> &tet, std::vector<int8_t> &loc);

}  // namespace hns
