// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <complex>
#include <map>
#include <string>
#include <vector>

#include "../../include/lt.h"

namespace lt {

using cdouble = std::complex<double>;
constexpr int kMaxRhs = 1000;  // right-hand sides per solve (the host flag buffer holds that many)
constexpr int kMaxTunedLevels = 16;
// Cells per grid.  The fused smoothers address a vector plane with 32-bit byte offsets
// (cell index times 8 for FP64 must stay below 2^32) and several kernels form 2 N in int.
constexpr long long kMaxCells = 1LL << 28;  // levels whose smoother tile shape can be tuned

// ---------------------------------------------------------------- errors
#define LT_HIP(...)                                                      \
    do {                                                                 \
        hipError_t e_ = (__VA_ARGS__);                                   \
        if (e_ != hipSuccess) {                                          \
            lt::set_last_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
            return LT_EHIP;                                              \
        }                                                                \
    } while (0)

#define LT_TRY(...)                   \
    do {                              \
        int rc_ = (__VA_ARGS__);      \
        if (rc_ < 0) return rc_;      \
    } while (0)

void set_last_error(const std::string& s);

// ------------------------------------------------------------- device buffers
// Grow-only device buffer: reallocates only when a larger size is requested.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int reserve(size_t n);
    void release();
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------- multigrid level
// Cell-centred FV operator on one level: (A x)_i = (D_i + tau m_i) x_i
//   - sum_a [ T_a[i] x_{i+e_a} + T_a[i-e_a] x_{i-e_a} ],
// T_a[i] is the face to the +a neighbour (0 for the last cell along a);
// D_i sums every face of the cell including walls; m_i is the lumped mass.
template <typename T> struct LevelView {
    int nx, ny, nz, N;
    const T* Tx;
    const T* Ty;
    const T* Tz;
    const T* D;
    const T* m;
};

struct Level {
    int n[3];
    int N;
    double h[3];
    int coarsened_from_fine[3];  // axes halved when this level was built from the finer one
    // distance from a zero-head wall to the first unknown, in units of h, per axis: 1/2 for
    // cell-centred unknowns at every level; 1 on the vertex grid of P1 elements, where an
    // aggregate of two moves it to delta / 2 + 1/4 (coarse wall terms and the prolongation's
    // wall weights follow it)
    double delta[3] = {0.5, 0.5, 0.5};
    // coefficients: [5][N] = Tx, Ty, Tz, D, m
    DevBuf c64, c32;
    LevelView<double> v64() const;
    LevelView<float> v32() const;
};

struct CoarseInverse {
    cdouble tau;
    DevBuf inv64, inv32;  // [N][N] complex (interleaved re, im), row-major
};

// Exact (K + tau M)^{-1} by block cyclic reduction over the slices of the last axis
// (exact.hip).  Level l has nl[l] blocks; its odd-positioned ones are eliminated with
// their inverses Dinv (slots dinv[l] ...) and, above level 0, P = Dinv F_{i-1}^T and
// Q = Dinv F_i (slots pm[l] ..., qm[l] ...) with their transposes (ptm[l] ..., qtm[l] ...).
// The reduction stops at level top, the first above 0 whose whole reduced system has at most
// kExactTail unknowns (level 0 for one slice): that system's dense inverse, [2][mtop][mtop]
// with mtop = nl[top] nb, is stored from double tail_off of mats on.
constexpr int kExactMaxBlock = 1024;  // cells per slice
constexpr int kExactTail = 1024;      // unknowns of the level solved by one dense inverse
constexpr int kExactCache = 4;        // factorised shifts kept per handle
struct ExactFactor {
    bool valid = false;
    cdouble tau;
    int nb = 0, n = 0;    // cells per slice, slices
    size_t ms = 0;        // doubles per dense block ([2][nb][nb])
    int top = 0;
    size_t mtop = 0, tail_off = 0;
    std::vector<int> nl;
    std::vector<size_t> dinv, pm, qm, ptm, qtm;
    DevBuf mats;
    unsigned long long tick = 0;
    void release();
};

}  // namespace lt

struct lt_handle {
    lt_grid grid;
    lt_bc bc;
    hipStream_t stream;
    int device = 0;  // HIP device current at setup
    int N;
    std::vector<lt::Level> levels;
    std::vector<lt::CoarseInverse> coarse_cache;
    std::vector<double> coarse_host;  // coarsest level coefficients [5][Nc] on the host
    lt::DevBuf kappa;                 // copy of the fine-grid conductivity (sensitivities)
    bool p1 = false;                  // P1 elements: the unknowns are the interior vertices of `cells`
    lt_grid cells{};                  // P1: the cell grid the triangulation comes from
    lt::DevBuf mstor;                 // S V per fine cell when water-table storage joins the mass
    // tile shape id of the fused 2D smoothers per level, [0]: FP64, [1]: FP32 (lt_autotune)
    int tiles[2][16] = {};
    double lnDbar = 0.0;              // mean of ln D over the fine grid (network features)
    // V-cycle vectors of a 3D grid in colour-planar order (cells of colour (x+y+z) & 1 = c
    // contiguous from c N/2 on), on the fine level and every level above the single-workgroup
    // ones; set at setup when each such level has an even nx
    bool cp3d = false;
    struct lt_unet* unet = nullptr;   // attached learned preconditioner (not owned)
    // workspaces (grow-only, owned by the handle); ws_gen changes whenever a
    // workspace or cached coarse inverse moves, which retires captured graphs
    std::map<std::string, lt::DevBuf> ws;
    unsigned long long ws_gen = 0;
    // captured refinement steps (hipGraphExec_t), keyed by everything they bake in
    // (the int records whether the step swaps the FP64 residual buffers)
    std::map<std::vector<unsigned long long>, std::pair<hipGraphExec_t, int>> graphs;
    unsigned long long graphs_gen = 0;  // ws_gen the cached graphs were captured at
    void* pinned = nullptr;  // small pinned host area for flags
    // allocation-free calls (lt_vcycle_noalloc): workspaces are carved from caller-side
    // device memory instead of the handle's own; with arena_plan set, carving only counts
    // the bytes a call would use and nothing is launched
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    bool arena_plan = false;
    lt::CoarseInverse arena_ci;       // coarse inverse built in the arena (not owned)
    int last_R = 0, last_jmax = 0;  // shape of the basis the last solve left in the workspaces
    // factorised shifts of the exact preconditioner (capacity reserved up front, so entries
    // never move), their use counter, and factorisations / milliseconds since the last reset
    std::vector<lt::ExactFactor> exact_cache;
    unsigned long long exact_tick = 0;
    int exact_factorizations = 0;
    double exact_factor_ms = 0.0;
    // profiling of one kernel family (opts.profile): event pairs and a byte counter
    int prof_target = 0;
    std::vector<hipEvent_t> prof_events;
    int prof_used = 0;
    unsigned long long* prof_counter = nullptr;  // device
    double prof_host_bytes = 0.0;  // bytes of profiled launches counted on the host
    ~lt_handle();
};

namespace lt {

// profiling helpers (api.hip)
int prof_begin(lt_handle* h, int family, unsigned long long** counter, hipEvent_t* ev0, hipEvent_t* ev1);
int prof_end(lt_handle* h, int family);

// workspace helper
template <typename T> T* wsp(lt_handle* h, const char* name, size_t count, int* rc) {
    if (h->arena || h->arena_plan) {
        // bump allocation from the arena, 256-byte aligned
        const size_t off = (h->arena_used + 255) & ~size_t(255);
        h->arena_used = off + count * sizeof(T);
        if (h->arena_plan) return reinterpret_cast<T*>(uintptr_t(256));  // a size count only
        if (h->arena_used > h->arena_cap) {
            *rc = LT_EINVAL;
            set_last_error(std::string("scratch too small for ") + name);
            return nullptr;
        }
        return reinterpret_cast<T*>(h->arena + off);
    }
    DevBuf& b = h->ws[name];
    void* before = b.p;
    int r = b.reserve(count * sizeof(T));
    if (r < 0) { *rc = r; return nullptr; }
    if (b.p != before) ++h->ws_gen;
    return b.as<T>();
}

// ------------------------------------------------------------- host planner
struct Plan {
    int ntimes = 0, nz = 0, nk = 0;     // nk = nz/2 shifts per time
    std::vector<cdouble> z;             // [ntimes * nk]
    std::vector<cdouble> wq;            // w_k * qhat(z_k)  [ntimes * nk]
    std::vector<double> omega;          // |wq| / max |wq| within the same time
    std::vector<cdouble> w;             // w_k alone (the initial head's term)  [ntimes * nk]
    std::vector<double> omega_init;     // |w| / max |w| within the same time
    std::vector<cdouble> tau_sched;     // cyclic preconditioner shifts
};
int talbot(int nz, double t, cdouble* z, cdouble* w);
// storage: convergence weights that also cover the storage-sensitivity contraction (lt_adjoint)
int make_plan(const double* times, int ntimes, int nz, double q, const lt_opts* o, Plan* p, bool storage = false);

// point weights as CSR (host)
struct PointsCSR {
    std::vector<int> off, cell;
    std::vector<double> wt;
};
int points_csr(const lt_grid& g, const lt_points* pts, PointsCSR* out);
// P1 handles: the basis functions at each point (barycentric coordinates in the triangle of
// the cell grid `cells` that contains it), over the interior vertices
int points_csr_p1(const lt_grid& cells, const lt_points* pts, PointsCSR* out);

// dense complex inverse (Gauss-Jordan with partial pivoting); returns 0 or LT_EINVAL if singular
int dense_inverse(int n, std::vector<cdouble>& a, std::vector<cdouble>& inv);

// one V-cycle of lt_vcycle (shared by the allocation-free variant)
int vcycle_call(lt_handle* h, cdouble tau, int precision, int nu1, int nu2, const double* b, double* x, int nvec);
// allocation-free calls: device address of the library's scratch array on the current
// device, taken once per device at setup (noalloc.hip)
int noalloc_init_device(int device);
void* noalloc_scratch(int device, size_t* bytes);

// ------------------------------------------------------------- exact preconditioner
// slice shape: nb cells per slice of the last axis, n slices
int exact_slices(const lt_handle* h, int* nb, int* n);
// the factorisation of K + tau M (cached per handle; the least recently used of
// kExactCache entries is replaced); synchronises the stream once
const ExactFactor* exact_factor(lt_handle* h, cdouble tau, int* rc);
// x = (K + tau M)^{-1} b for R complex vectors (right-hand side r at b + r brs, planes N
// apart; likewise x); enqueued on the handle's stream.  active (device [R] or nullptr):
// x of a right-hand side marked 0 is left untouched
int exact_apply(lt_handle* h, const ExactFactor* F, int R, const double* b, size_t brs, double* x, size_t xrs,
                const int* active = nullptr);
// bytes of dense blocks one exact_apply reads
size_t exact_matrix_bytes(const ExactFactor* F);

// ------------------------------------------------------------- multigrid
int mg_build(lt_handle* h, const double* kappa, const double* S, const lt_grid* p1_cells = nullptr);
const CoarseInverse* mg_coarse_inverse(lt_handle* h, cdouble tau, int* rc);
// One V-cycle on level 0 for R complex vectors: b0, x0 in the level-0 work arrays of
// precision T (x0 is overwritten).  active: device [R] mask or nullptr.
// Optional fusion of the fine-level post-smoother with one refinement step of the
// preconditioner solve (2D fused path only): u += e, rho_out = rho_in - (K + tau M) e,
// lo = (T) rho_out, part = per-tile ||rho_out||^2 (u of right-hand side r is
// u + r * ustride + *jcol * 2N).  When applied, *nparts is set to
// the number of partial sums per right-hand side and x0 is not written.
struct RefineArgs {
    double* u;
    size_t ustride;
    const int* jcol;  // device: u is advanced by jcol * 2N (nullptr: by 0)
    const double* rho_in;
    double* rho_out;
    void* lo;
    double* part;
    int* nparts;
    const int* list = nullptr;  // set by the cycle: its list of active right-hand sides (group_rhs), if any
};

// Workgroup b of nb remapped so that each of the 8 XCDs, which take workgroups in turn,
// works through one contiguous run of the grid: cells that neighbour each other in the
// vectors are then read through the same XCD's L2.  Identity when 8 does not divide nb.
// (Stencil kernels gain from it; on plain streaming kernels it measured slower: the
// XCDs then stream eight distant regions at once instead of one.)
__device__ __forceinline__ int xcd_block(int b, int nb) {
    return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

// Right-hand sides per thread of the 3D multigrid kernels and the refinement update.
constexpr int kSweepRhs = 4;

// The right-hand sides that a kernel serves in groups of RB.  With a list (list[0] = the
// number of active right-hand sides, list[1 + j] = the j-th active index in increasing
// order), group g takes active ones g RB .. g RB + RB - 1, so every group but the last is
// full and what a group loads once (coefficients, indices) serves RB right-hand sides;
// without one, group g takes g RB .. g RB + RB - 1 of all R.  -1: no right-hand side there.
template <int RB>
__device__ __forceinline__ void group_rhs(const int* __restrict__ list, int R, int g, int (&rs)[RB]) {
    const int n = list ? list[0] : R;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int j = g * RB + q;
        rs[q] = j < n ? (list ? list[1 + j] : j) : -1;
    }
}
template <typename T>
int mg_vcycle(lt_handle* h, cdouble tau, int nu1, int nu2, int R, const int* active,
              T* x0, const T* b0, RefineArgs* refine = nullptr);
template <typename T>
int apply_operator(lt_handle* h, int level, cdouble tau, const T* x, T* y, int R, const int* active);
template <typename S, typename D>
int convert_vectors(hipStream_t st, const S* in, D* out, size_t count);
// nvec complex vectors [nvec][2][N] converted between precisions, and between the natural
// order and the colour-planar order of an nx = cpnx, ny = cpny grid (dir 0: natural to
// colour-planar, 1: back); cpnx = 0: natural order on both sides
template <typename S, typename D>
int convert_vectors_cp(hipStream_t st, const S* in, D* out, int nvec, int N, int cpnx, int cpny, int dir);

}  // namespace lt
