// The quasi-linear geostatistical inversion (Section 5.1, Algorithm 2) on the GPU.
//
// Unknowns s = ln kappa per cell, prior s ~ N(X beta, Q) with X a column of ones and Q the
// exponential covariance Q_ij = var exp(-|(x_i - x_j) / ell|) over the cell centres (the kernel
// of the paper's rough field), measurements y = h(s) + eps with eps ~ N(0, r I): heads at the
// observation wells and times, ordered (well, receiver, time).  A Gauss-Newton step at s_k:
//   h(s_k) by lt_solve, J = dh/ds by lt_adjoint (d phi / d ln kappa per cell),
//   Q J^T by k_cov_apply (the kernel matrix is evaluated tile by tile in LDS and never stored:
//     the grid-sized matrix the paper multiplies by FFT or an H-matrix costs O(N^2) exp here,
//     shared by 32 rows of J, against O(N^2 M) multiply-adds),
//   J Q J^T, J X and J s_k by reductions over the cells,
//   the saddle-point system of eq:inversion1 (M + 1 unknowns) by LU with partial pivoting on
//     the host, and s_{k+1} = X beta + Q J^T xi on the device.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lt_internal.h"

namespace lt {

namespace {

constexpr int kCT = 64;  // cells per tile of the covariance product (rows and columns)
constexpr int kCM = 32;  // vectors per workgroup of the covariance product
constexpr int kGT = 16;  // J Q J^T: output tile (rows and columns)
constexpr int kGK = 64;  // J Q J^T: cells per staged chunk

// cell centres scaled by the correlation lengths
struct CovGrid {
    int nx, ny, nz, ndim;
    double sx, sy, sz;  // h_a / ell_a: cell spacing in correlation lengths
};

__device__ inline void cov_coords(const CovGrid& g, int c, double* x, double* y, double* z) {
    const int ix = c % g.nx, iy = (c / g.nx) % g.ny, iz = c / (g.nx * g.ny);
    *x = (ix + 0.5) * g.sx;
    *y = g.ndim >= 2 ? (iy + 0.5) * g.sy : 0.0;
    *z = g.ndim >= 3 ? (iz + 0.5) * g.sz : 0.0;
}

// out[m][i] = sum_j var exp(-|x_i - x_j|) v[m][j] for m < M (rows of [M][N]).  Workgroup:
// 64 cells i times 32 vectors; thread (i, g) accumulates vectors g * 8 ... g * 8 + 7.  Each
// 64 x 64 tile of the kernel matrix is evaluated once into LDS and used by all 32 vectors.
__global__ __launch_bounds__(256) void k_cov_apply(CovGrid G, int N, double var, int M, const double* __restrict__ v,
                                                   double* __restrict__ out) {
    __shared__ double kt[kCT][kCT + 1];   // [j][i]
    __shared__ double vt[kCM][kCT + 1];   // [m][j]
    __shared__ double xj[3][kCT], xi[3][kCT];
    const int tid = threadIdx.x, il = tid % kCT, g = tid / kCT;
    const int i0 = blockIdx.x * kCT, m0 = blockIdx.y * kCM;
    if (tid < kCT) {
        const int i = min(i0 + tid, N - 1);
        cov_coords(G, i, &xi[0][tid], &xi[1][tid], &xi[2][tid]);
    }
    double acc[kCM / 4];
#pragma unroll
    for (int q = 0; q < kCM / 4; ++q) acc[q] = 0.0;
    for (int j0 = 0; j0 < N; j0 += kCT) {
        __syncthreads();  // the previous tile is no longer read
        if (tid < kCT) {
            const int j = min(j0 + tid, N - 1);
            cov_coords(G, j, &xj[0][tid], &xj[1][tid], &xj[2][tid]);
        }
#pragma unroll
        for (int q = 0; q < kCM * kCT / 256; ++q) {
            const int idx = tid + 256 * q;
            const int jj = idx % kCT, mm = idx / kCT;
            const int j = j0 + jj, m = m0 + mm;
            const bool ok = j < N && m < M;
            const double val = v[(size_t)(ok ? m : 0) * N + (ok ? j : 0)];
            vt[mm][jj] = ok ? val : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kCT * kCT / 256; ++q) {
            const int idx = tid + 256 * q;
            const int ii = idx % kCT, jj = idx / kCT;
            const double dx = xi[0][ii] - xj[0][jj], dy = xi[1][ii] - xj[1][jj], dz = xi[2][ii] - xj[2][jj];
            const double k = var * exp(-sqrt(dx * dx + dy * dy + dz * dz));
            kt[jj][ii] = j0 + jj < N ? k : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int jj = 0; jj < kCT; ++jj) {
            const double k = kt[jj][il];
#pragma unroll
            for (int q = 0; q < kCM / 4; ++q) acc[q] += k * vt[g * (kCM / 4) + q][jj];
        }
    }
    const int i = i0 + il;
    if (i < N) {
#pragma unroll
        for (int q = 0; q < kCM / 4; ++q) {
            const int m = m0 + g * (kCM / 4) + q;
            if (m < M) out[(size_t)m * N + i] = acc[q];
        }
    }
}

// Partial sums of G = A B^T over cell chunks: part[z][m][m'] = sum_{i in chunk z} A[m][i] B[m'][i]
// (A, B [M][N]); a 16 x 16 output tile per workgroup.
__global__ __launch_bounds__(256) void k_gram_part(int N, int M, int chunk, const double* __restrict__ A,
                                                   const double* __restrict__ B, double* __restrict__ part) {
    __shared__ double at[kGT][kGK + 1], bt[kGT][kGK + 1];
    const int tid = threadIdx.x, tm = tid / kGT, tn = tid % kGT;
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int c0 = blockIdx.z * chunk, c1 = min(N, c0 + chunk);
    double acc = 0.0;
    for (int k0 = c0; k0 < c1; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kGT * kGK / 256; ++q) {
            const int idx = tid + 256 * q;
            const int kk = idx % kGK, rr = idx / kGK;
            const int k = k0 + kk;
            const bool ok = k < c1;
            const int ma = m0 + rr, mb = n0 + rr;
            const double va = A[(size_t)((ok && ma < M) ? ma : 0) * N + (ok ? k : 0)];
            const double vb = B[(size_t)((ok && mb < M) ? mb : 0) * N + (ok ? k : 0)];
            at[rr][kk] = ok && ma < M ? va : 0.0;
            bt[rr][kk] = ok && mb < M ? vb : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kGK; ++kk) acc += at[tm][kk] * bt[tn][kk];
    }
    const int m = m0 + tm, n = n0 + tn;
    if (m < M && n < M) part[((size_t)blockIdx.z * M + m) * M + n] = acc;
}

__global__ __launch_bounds__(256) void k_sum_part(int len, int parts, const double* __restrict__ part,
                                                  double* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    double s = 0.0;
    for (int z = 0; z < parts; ++z) s += part[(size_t)z * len + e];
    out[e] = s;
}

// per row m of J [M][N]: out[m] = sum_i J[m][i] (J X), out[M + m] = sum_i J[m][i] s[i] (J s)
__global__ __launch_bounds__(256) void k_row_dots(int N, int M, const double* __restrict__ J,
                                                  const double* __restrict__ s, double* __restrict__ out) {
    __shared__ double r1[256], r2[256];
    const int m = blockIdx.x, tid = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = tid; i < N; i += 256) {
        const double j = J[(size_t)m * N + i];
        a += j;
        b += j * s[i];
    }
    r1[tid] = a;
    r2[tid] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            r1[tid] += r1[tid + w];
            r2[tid] += r2[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[m] = r1[0];
        out[M + m] = r2[0];
    }
}

// s_next[i] = beta + sum_m QJt[m][i] xi[m]
__global__ __launch_bounds__(256) void k_s_next(int N, int M, const double* __restrict__ QJt,
                                                const double* __restrict__ xi, double beta,
                                                double* __restrict__ s_next) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    double v = beta;
    for (int m = 0; m < M; ++m) v += QJt[(size_t)m * N + i] * xi[m];
    s_next[i] = v;
}

__global__ __launch_bounds__(256) void k_exp(int N, const double* __restrict__ s, double* __restrict__ kappa) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) kappa[i] = exp(s[i]);
}

inline unsigned nblk(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Dense solve A x = b (n x n, row-major, overwritten) by LU with partial pivoting.
int dense_solve(int n, std::vector<double>& A, std::vector<double>& b) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)p * n + k])) p = i;
        if (!(std::fabs(A[(size_t)p * n + k]) > 0.0)) return LT_EINVAL;
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
            std::swap(b[k], b[p]);
        }
        const double d = A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            const double f = A[(size_t)i * n + k] / d;
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double v = b[k];
        for (int j = k + 1; j < n; ++j) v -= A[(size_t)k * n + j] * b[j];
        b[k] = v / A[(size_t)k * n + k];
    }
    return 0;
}

CovGrid cov_grid(const lt_handle* h, const double* len) {
    const lt_grid& g = h->grid;
    return CovGrid{g.n[0], g.n[1], g.n[2], g.ndim, g.h[0] / len[0], g.ndim >= 2 ? g.h[1] / len[1] : 0.0,
                   g.ndim >= 3 ? g.h[2] / len[2] : 0.0};
}

int check_cov(const lt_handle* h, double var, const double* len) {
    if (!(var > 0.0) || !std::isfinite(var) || !len) return LT_EINVAL;
    for (int a = 0; a < h->grid.ndim; ++a)
        if (!(len[a] > 0.0) || !std::isfinite(len[a])) return LT_EINVAL;
    return 0;
}

}  // namespace

int cov_apply(lt_handle* h, double var, const double* len, int nvec, const double* v, double* out) {
    const int N = h->N;
    k_cov_apply<<<dim3(nblk(N, kCT), nblk(nvec, kCM)), 256, 0, h->stream>>>(cov_grid(h, len), N, var, nvec, v, out);
    LT_HIP(hipGetLastError());
    return 0;
}

}  // namespace lt

using namespace lt;

extern "C" {

int lt_cov_apply(lt_handle* h, double var, const double* len, int nvec, const double* v, double* out) {
    if (!h || !v || !out || nvec < 1 || check_cov(h, var, len) < 0) {
        set_last_error("lt_cov_apply: bad argument (var and lengths must be positive and finite)");
        return LT_EINVAL;
    }
    return cov_apply(h, var, len, nvec, v, out);
}

int lt_geostat_step(lt_handle* h, const lt_geostat* g, const double* y, const double* s, double* s_next,
                    double* hs_out, double* beta_out, lt_stats* stats) {
    if (!h || !g || !y || !s || !s_next || g->src.n < 1 || !g->src.xyz || g->obs.n < 1 || !g->obs.xyz ||
        !g->times || g->ntimes < 1 || !(g->r > 0.0) || !std::isfinite(g->r) ||
        check_cov(h, g->cov_var, g->cov_len) < 0) {
        set_last_error("lt_geostat_step: bad argument");
        return LT_EINVAL;
    }
    const int N = h->N;
    const long long Mll = (long long)g->src.n * g->obs.n * g->ntimes;
    if (Mll > 4096) {
        set_last_error("lt_geostat_step: at most 4096 measurements");
        return LT_EINVAL;
    }
    const int M = (int)Mll;
    hipStream_t st = h->stream;
    int rc = 0;
    double* J = wsp<double>(h, "gs_J", (size_t)M * N, &rc);
    double* QJt = wsp<double>(h, "gs_QJt", (size_t)M * N, &rc);
    double* hs = wsp<double>(h, "gs_hs", (size_t)M, &rc);
    double* dots = wsp<double>(h, "gs_dots", 2 * (size_t)M, &rc);
    double* Gm = wsp<double>(h, "gs_G", (size_t)M * M, &rc);
    const int KS = std::max(1, std::min(64, 256 / (int)(nblk(M, kGT) * nblk(M, kGT))));
    const int chunk = (int)((((size_t)N + KS - 1) / KS + kGK - 1) / kGK * kGK);
    double* part = wsp<double>(h, "gs_part", (size_t)KS * M * M, &rc);
    double* xi_d = wsp<double>(h, "gs_xi", (size_t)M, &rc);
    if (!J || !QJt || !hs || !dots || !Gm || !part || !xi_d) return rc;
    lt_sources src{g->src, g->q, nullptr};
    // h(s_k) at the observation wells, then J = dh/ds
    const int rs = lt_solve(h, &src, g->times, g->ntimes, &g->contour, &g->obs, g->opts, hs, stats);
    if (rs < 0) return rs;
    const int ra = lt_adjoint(h, &src, &g->obs, g->times, g->ntimes, &g->contour, g->opts, J, nullptr, nullptr);
    if (ra < 0) return ra;
    // Q J^T (rows Q J_m), J Q J^T, J X, J s_k
    LT_TRY(cov_apply(h, g->cov_var, g->cov_len, M, J, QJt));
    k_gram_part<<<dim3(nblk(M, kGT), nblk(M, kGT), KS), 256, 0, st>>>(N, M, chunk, J, QJt, part);
    LT_HIP(hipGetLastError());
    k_sum_part<<<nblk((size_t)M * M, 256), 256, 0, st>>>(M * M, KS, part, Gm);
    LT_HIP(hipGetLastError());
    k_row_dots<<<M, 256, 0, st>>>(N, M, J, s, dots);
    LT_HIP(hipGetLastError());
    std::vector<double> G((size_t)M * M), d(2 * (size_t)M), hh(M), yy(M);
    LT_HIP(hipMemcpyAsync(G.data(), Gm, G.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(d.data(), dots, d.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(hh.data(), hs, hh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(yy.data(), y, yy.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipStreamSynchronize(st));
    // the saddle-point system of eq:inversion1
    const int n1 = M + 1;
    std::vector<double> A((size_t)n1 * n1, 0.0), b(n1, 0.0);
    for (int m = 0; m < M; ++m) {
        for (int k = 0; k < M; ++k) A[(size_t)m * n1 + k] = G[(size_t)m * M + k];
        A[(size_t)m * n1 + m] += g->r;
        A[(size_t)m * n1 + M] = d[m];
        A[(size_t)M * n1 + m] = d[m];
        b[m] = yy[m] - hh[m] + d[M + m];
    }
    if (dense_solve(n1, A, b) < 0) {
        set_last_error("lt_geostat_step: the saddle-point system is singular");
        return LT_EINVAL;
    }
    const double beta = b[M];
    LT_HIP(hipMemcpyAsync(xi_d, b.data(), M * sizeof(double), hipMemcpyHostToDevice, st));
    k_s_next<<<nblk(N, 256), 256, 0, st>>>(N, M, QJt, xi_d, beta, s_next);
    LT_HIP(hipGetLastError());
    if (hs_out) LT_HIP(hipMemcpyAsync(hs_out, hs, M * sizeof(double), hipMemcpyDeviceToDevice, st));
    LT_HIP(hipStreamSynchronize(st));  // b (the host source of xi) goes out of scope
    if (beta_out) *beta_out = beta;
    return (rs > 0 || ra > 0) ? LT_WNOTCONV : LT_OK;
}

int lt_geostat_invert(const lt_grid* grid, const lt_bc* bc, const double* S, const lt_geostat* g,
                      const double* y, const double* s0, int iters, void* hip_stream, double* s_out,
                      double* misfit, double* step) {
    if (!grid || !S || !g || !y || !s0 || !s_out || iters < 1) {
        set_last_error("lt_geostat_invert: bad argument");
        return LT_EINVAL;
    }
    const long long Nll = (long long)grid->n[0] * grid->n[1] * grid->n[2];
    if (Nll < 2 || Nll > (1LL << 28)) {
        set_last_error("lt_geostat_invert: bad grid");
        return LT_EINVAL;
    }
    const size_t N = (size_t)Nll;
    const int M = g->src.n * g->obs.n * g->ntimes;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double *sa = nullptr, *sb = nullptr, *kap = nullptr, *hs = nullptr;
    auto cleanup = [&]() {
        if (sa) (void)hipFree(sa);
        if (sb) (void)hipFree(sb);
        if (kap) (void)hipFree(kap);
        if (hs) (void)hipFree(hs);
    };
    if (hipMalloc(&sa, N * sizeof(double)) != hipSuccess || hipMalloc(&sb, N * sizeof(double)) != hipSuccess ||
        hipMalloc(&kap, N * sizeof(double)) != hipSuccess ||
        hipMalloc(&hs, (size_t)std::max(M, 1) * sizeof(double)) != hipSuccess) {
        cleanup();
        set_last_error("lt_geostat_invert: hipMalloc failed");
        return LT_ENOMEM;
    }
    int ret = LT_OK;
    if (hipMemcpyAsync(sa, s0, N * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) ret = LT_EHIP;
    std::vector<double> hh(std::max(M, 1)), yy(std::max(M, 1)), va(N), vb(N);
    if (ret == LT_OK && (hipMemcpyAsync(yy.data(), y, M * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                         hipStreamSynchronize(st) != hipSuccess))
        ret = LT_EHIP;
    for (int k = 0; k < iters && ret >= 0; ++k) {
        k_exp<<<nblk(N, 256), 256, 0, st>>>((int)N, sa, kap);
        if (hipGetLastError() != hipSuccess) {
            ret = LT_EHIP;
            break;
        }
        lt_handle* h = nullptr;
        int r = lt_setup(grid, kap, S, bc, hip_stream, &h);
        if (r < 0) {
            ret = r;
            break;
        }
        r = lt_geostat_step(h, g, y, sa, sb, hs, nullptr, nullptr);
        if (r < 0) {
            lt_destroy(h);
            ret = r;
            break;
        }
        if (r > 0) ret = r;
        if (misfit || step) {
            if (hipMemcpyAsync(hh.data(), hs, M * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(va.data(), sa, N * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(vb.data(), sb, N * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                lt_destroy(h);
                ret = LT_EHIP;
                break;
            }
            double ms = 0.0, dn = 0.0, nn = 0.0;
            for (int m = 0; m < M; ++m) ms += (yy[m] - hh[m]) * (yy[m] - hh[m]);
            for (size_t i = 0; i < N; ++i) {
                dn += (vb[i] - va[i]) * (vb[i] - va[i]);
                nn += vb[i] * vb[i];
            }
            if (misfit) misfit[k] = ms / g->r;
            if (step) step[k] = nn > 0.0 ? std::sqrt(dn / nn) : 0.0;
        }
        lt_destroy(h);
        std::swap(sa, sb);
    }
    if (ret >= 0 && hipMemcpyAsync(s_out, sa, N * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
        ret = LT_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess && ret >= 0) ret = LT_EHIP;
    cleanup();
    return ret;
}

}  // extern "C"
