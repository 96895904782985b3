// Autotuner for the tile shape of the fused 2D smoothers.
//
// Per multigrid level the best tile differs: the fine level moves the most
// data and prefers wide tiles (less halo re-reading), the coarser levels
// have few cells and are latency-bound, where small tiles give more, shorter
// workgroups.  The tuner times whole preconditioner steps (V-cycle plus the
// fused FP64 refinement update, exactly as the Krylov loop runs them) with
// HIP events on the handle's stream, trying every shape on one level at a
// time from the finest down while keeping the others, and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "krylov.h"
#include "lt_internal.h"
#include "mg_fused.h"

namespace lt {
namespace {

template <typename T>
__global__ void k_tune_fill(T* __restrict__ v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = T(1) + T(0.25) * (T)(i % 7);
}

template <typename T>
int fill(hipStream_t st, T* v, size_t n) {
    k_tune_fill<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(v, n);
    LT_HIP(hipGetLastError());
    return 0;
}

// Levels handled by the fused tile kernels (above the single-workgroup coarse levels).
int fused_levels(const lt_handle* h) {
    int n = 0;
    for (const Level& L : h->levels) {
        if (L.N <= kCoarseBlockCells) break;
        ++n;
    }
    return std::min(n, kMaxTunedLevels);
}

template <typename T>
int time_steps(lt_handle* h, cdouble tau, int nu1, int nu2, int R, T* e, T* b, RefineArgs* ra, hipEvent_t ev0,
               hipEvent_t ev1, int reps, float* ms) {
    for (int k = 0; k < 2; ++k) LT_TRY(mg_vcycle<T>(h, tau, nu1, nu2, R, nullptr, e, b, ra));
    LT_HIP(hipEventRecord(ev0, h->stream));
    for (int k = 0; k < reps; ++k) LT_TRY(mg_vcycle<T>(h, tau, nu1, nu2, R, nullptr, e, b, ra));
    LT_HIP(hipEventRecord(ev1, h->stream));
    LT_HIP(hipEventSynchronize(ev1));
    LT_HIP(hipEventElapsedTime(ms, ev0, ev1));
    *ms /= reps;
    return 0;
}

template <typename T>
int tune(lt_handle* h, int nu1, int nu2, int R, int* tiles_out, int n_out, double* us_out) {
    const int p = sizeof(T) == 4 ? 1 : 0;
    const int nf = fused_levels(h);
    const size_t n2 = 2 * (size_t)h->N * R;
    int rc = 0;
    T* b = wsp<T>(h, "tune_b", n2, &rc);
    T* e = wsp<T>(h, "tune_e", n2, &rc);
    T* lo = wsp<T>(h, "tune_lo", n2, &rc);
    double* u = wsp<double>(h, "tune_u", n2, &rc);
    double* rho = wsp<double>(h, "tune_rho", n2, &rc);
    double* rho2 = wsp<double>(h, "tune_rho2", n2, &rc);
    const size_t ntiles = ((size_t)h->grid.n[0] + kMinTileX - 1) / kMinTileX *
                          (((size_t)h->grid.n[1] + kMinTileY - 1) / kMinTileY);
    double* part = wsp<double>(h, "tune_part", ntiles * R, &rc);
    if (!b || !e || !lo || !u || !rho || !rho2 || !part) return rc;
    LT_TRY(fill<T>(h->stream, b, n2));
    LT_TRY(fill<double>(h->stream, u, n2));
    LT_TRY(fill<double>(h->stream, rho, n2));
    int nparts = -1;
    // FP32 steps update rho in place and write its FP32 copy; FP64 steps write rho2
    RefineArgs ra{u, 2 * (size_t)h->N, nullptr, rho, p ? rho : rho2, p ? (void*)lo : nullptr, part, &nparts};
    // a representative shift: the diagonal scale of the fine operator, half real, half imaginary
    const cdouble tau(1e5, 1e5);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    LT_HIP(hipEventCreate(&ev0));
    if (hipEventCreate(&ev1) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        set_last_error("hipEventCreate failed");
        return LT_EHIP;
    }
    float best_ms = 0;
    int result = 0;
    const int reps = 10;
    // three interleaved rounds over the shapes, keeping each shape's fastest round, so
    // that a transient slowdown does not decide the choice
    for (int l = 0; l < nf && result == 0; ++l) {
        float tms[kNumTiles];
        for (int t = 0; t < kNumTiles; ++t) tms[t] = 1e30f;
        for (int round = 0; round < 3 && result == 0; ++round)
            for (int t = 0; t < kNumTiles && result == 0; ++t) {
                h->tiles[p][l] = t;
                float ms = 0;
                result = time_steps<T>(h, tau, nu1, nu2, R, e, b, &ra, ev0, ev1, reps, &ms);
                if (result == 0) tms[t] = std::min(tms[t], ms);
            }
        int best = 0;
        for (int t = 1; t < kNumTiles; ++t)
            if (tms[t] < tms[best]) best = t;
        h->tiles[p][l] = best;
        best_ms = tms[best];
    }
    if (result == 0 && nf == 0) {
        float ms = 0;
        result = time_steps<T>(h, tau, nu1, nu2, R, e, b, &ra, ev0, ev1, reps, &ms);
        best_ms = ms;
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (result < 0) return result;
    LT_HIP(hipStreamSynchronize(h->stream));
    for (const char* nm : {"tune_b", "tune_e", "tune_lo", "tune_u", "tune_rho", "tune_rho2", "tune_part"}) {
        h->ws[nm].release();
        h->ws.erase(nm);
        ++h->ws_gen;
    }
    for (int l = 0; l < n_out && l < kMaxTunedLevels; ++l) tiles_out[l] = l < nf ? h->tiles[p][l] : -1;
    if (us_out) *us_out = 1e3 * best_ms;
    return nf;
}

}  // namespace
}  // namespace lt

extern "C" {

int lt_tile_shape(int id, int* tx, int* ty) {
    if (!tx || !ty) return LT_EINVAL;
    return lt::tile_shape(id, tx, ty);
}

int lt_autotune(lt_handle* h, int precision, int nu1, int nu2, int nvec, int* tiles_out, int n_out,
                double* us_per_step) {
    if (!h || nvec < 1 || nvec > 1000 || n_out < 0 || (n_out > 0 && !tiles_out) ||
        (precision != LT_PREC_FP64 && precision != LT_PREC_MIXED)) {
        lt::set_last_error("lt_autotune: bad argument");
        return LT_EINVAL;
    }
    if (h->grid.ndim != 2 || nu1 < 1 || nu1 > 3 || nu2 < 1 || nu2 > 3) {
        // only the fused 2D smoothers have tile shapes
        for (int l = 0; l < n_out; ++l) tiles_out[l] = -1;
        if (us_per_step) *us_per_step = 0;
        return 0;
    }
    if (precision == LT_PREC_MIXED) return lt::tune<float>(h, nu1, nu2, nvec, tiles_out, n_out, us_per_step);
    return lt::tune<double>(h, nu1, nu2, nvec, tiles_out, n_out, us_per_step);
}

int lt_set_tiles(lt_handle* h, int precision, const int* tiles, int n) {
    if (!h || n < 0 || n > lt::kMaxTunedLevels || (n > 0 && !tiles) ||
        (precision != LT_PREC_FP64 && precision != LT_PREC_MIXED)) {
        lt::set_last_error("lt_set_tiles: bad argument");
        return LT_EINVAL;
    }
    for (int l = 0; l < n; ++l)
        if (tiles[l] < -1 || tiles[l] >= lt::kNumTiles) {
            lt::set_last_error("lt_set_tiles: unknown tile shape");
            return LT_EINVAL;
        }
    const int p = precision == LT_PREC_MIXED ? 1 : 0;
    for (int l = 0; l < lt::kMaxTunedLevels; ++l) h->tiles[p][l] = (l < n && tiles[l] >= 0) ? tiles[l] : 0;
    return LT_OK;
}

}  // extern "C"
