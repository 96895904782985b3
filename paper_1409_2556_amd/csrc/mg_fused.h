// Fused multigrid kernels (mg_fused.hip).
#pragma once

#include "lt_internal.h"

namespace lt {

constexpr int kNumTiles = 4;               // tile shapes of the fused 2D kernels (tile_shape)
constexpr int kMinTileX = 16, kMinTileY = 8;  // smallest of them (sizes per-tile partial sums)
constexpr int kCoarseBlockCells = 1024;  // first level handled by the single-workgroup kernel
constexpr int kMaxCBLevels = 5;

struct T4 {
    double x, y, z, w;  // ghost parity of the -x, +x, -y, +y walls
};

template <typename T> struct CBLevel {
    int nx, ny, nz, N;
    int cox, coy, coz;  // axes halved to make this level from the finer one
    int off;            // cell offset of this level's vectors in LDS
    const T* Tx;
    const T* Ty;
    const T* Tz;
    const T* D;
    const T* m;
};

template <typename T> struct CBMeta {
    int nl;
    CBLevel<T> L[kMaxCBLevels];
    T ghost[6];
    int nu1, nu2;
    const T* inv;  // dense inverse of the coarsest level (interleaved complex) or nullptr
    int coarse_sweeps;
};

// interior cells per workgroup of tile shape `id` (0..kNumTiles-1)
int tile_shape(int id, int* tx, int* ty);
template <typename T>
int launch_pre2d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b, T* x, int cnx,
                 int cny, int cox, int coy, T* bc, int R, const int* active, unsigned long long* prof,
                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
int launch_post2d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b, const T* xin,
                  const T* ec, int cnx, int cny, int cox, int coy, T4 ghost, T* xout, int R, const int* active,
                  unsigned long long* prof, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// *nparts = number of per-tile partial sums per right-hand side written to part.
// ev0/ev1 (optional): events recorded at the start and end of this launch.
template <typename T>
int launch_post2d_refine(hipStream_t st, const LevelView<T>& L, const LevelView<double>& L64, T tr, T ti,
                         double tr64, double ti64, int nu, int tile, const T* b, const T* xin, const T* ec, int cnx,
                         int cny, int cox, int coy, T4 ghost, double* u, size_t ustride, const int* jcol,
                         const double* rho_in, double* rho_out, T* lo, double* part, int R, const int* active,
                         unsigned long long* prof, int* nparts, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
template <typename T>
int launch_coarse_block(hipStream_t st, const CBMeta<T>& M, T tr, T ti, const T* bin, T* xout, int R,
                        const int* active);

}  // namespace lt
