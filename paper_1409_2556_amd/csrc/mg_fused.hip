// Fused multigrid kernels.
//
// 2D levels: an LDS tile of TX x TY cells plus a halo runs nu full red-black
// Gauss-Seidel sweeps in one launch.  Every half-sweep updates the cells of
// one colour in a region one cell smaller than the last, so after nu sweeps
// (2 nu half-sweeps) the tile interior holds exactly what a global red-black
// sweep would produce (the halo is recomputed by neighbouring tiles, nothing
// is exchanged).  The pre-smoothing kernel starts from x = 0, keeps one more
// halo ring so the residual b - A x of the interior is exact, and restricts
// it (sum over the aggregate) to the coarse right-hand side in the same
// launch.  The post-smoothing kernel adds the prolongated coarse correction
// while loading its tile and writes to a separate buffer.
//
// Small levels (at most kCoarseBlockCells cells on the first of them) are
// handled by one workgroup per right-hand side that runs the remaining
// V-cycle in LDS, including the dense solve on the coarsest level.
#include "mg_fused.h"

namespace lt {

template <typename T> struct cx {
    T re, im;
};

// ------------------------------------------------------------------ 2D tiles
template <typename T, int H> struct Tile2D {
    static constexpr int EX = kTileX + 2 * H;
    static constexpr int EY = kTileY + 2 * H;
    T xr[EY][EX], xi[EY][EX];
    T br[EY][EX], bi[EY][EX];
    T tx[EY][EX], ty[EY][EX];
    T dr[EY][EX], di[EY][EX];
};

template <typename T, int H>
__device__ __forceinline__ void tile_sweeps(Tile2D<T, H>& s, int gx0, int gy0, int nx, int ny, int nhalf,
                                            int first_color) {
    constexpr int EX = Tile2D<T, H>::EX, EY = Tile2D<T, H>::EY;
    for (int hs = 0; hs < nhalf; ++hs) {
        const int color = (first_color + hs) & 1;
        const int sh = hs + 1;
        for (int c = threadIdx.x; c < EX * EY; c += blockDim.x) {
            const int lx = c % EX, ly = c / EX;
            if (lx < sh || lx >= EX - sh || ly < sh || ly >= EY - sh) continue;
            const int gx = gx0 + lx, gy = gy0 + ly;
            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
            if (((gx + gy) & 1) != color) continue;
            T ore = s.tx[ly][lx] * s.xr[ly][lx + 1] + s.tx[ly][lx - 1] * s.xr[ly][lx - 1] +
                    s.ty[ly][lx] * s.xr[ly + 1][lx] + s.ty[ly - 1][lx] * s.xr[ly - 1][lx];
            T oim = s.tx[ly][lx] * s.xi[ly][lx + 1] + s.tx[ly][lx - 1] * s.xi[ly][lx - 1] +
                    s.ty[ly][lx] * s.xi[ly + 1][lx] + s.ty[ly - 1][lx] * s.xi[ly - 1][lx];
            T nr = s.br[ly][lx] + ore, ni = s.bi[ly][lx] + oim;
            T dr = s.dr[ly][lx], di = s.di[ly][lx];
            T dd = dr * dr + di * di;
            s.xr[ly][lx] = (nr * dr + ni * di) / dd;
            s.xi[ly][lx] = (ni * dr - nr * di) / dd;
        }
        __syncthreads();
    }
}

// Load coefficients and b of the extended tile; cells outside the grid get zero
// couplings, zero b and a unit diagonal (they are never updated).
template <typename T, int H>
__device__ __forceinline__ void tile_load_common(Tile2D<T, H>& s, const LevelView<T>& L, T tr, T ti,
                                                 const T* __restrict__ br, const T* __restrict__ bi, int gx0,
                                                 int gy0) {
    constexpr int EX = Tile2D<T, H>::EX, EY = Tile2D<T, H>::EY;
    for (int c = threadIdx.x; c < EX * EY; c += blockDim.x) {
        const int lx = c % EX, ly = c / EX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
            const int i = gx + L.nx * gy;
            s.tx[ly][lx] = L.Tx[i];
            s.ty[ly][lx] = L.Ty[i];
            s.dr[ly][lx] = L.D[i] + tr * L.m[i];
            s.di[ly][lx] = ti * L.m[i];
            s.br[ly][lx] = br[i];
            s.bi[ly][lx] = bi[i];
        } else {
            s.tx[ly][lx] = 0;
            s.ty[ly][lx] = 0;
            s.dr[ly][lx] = 1;
            s.di[ly][lx] = 0;
            s.br[ly][lx] = 0;
            s.bi[ly][lx] = 0;
        }
    }
}

// Pre-smoothing from x = 0, then restriction of the residual.
template <typename T, int NU>
__global__ __launch_bounds__(256) void k_pre2d(LevelView<T> L, T tr, T ti, const T* __restrict__ b,
                                               T* __restrict__ x, int cnx, int cny, int cox, int coy,
                                               T* __restrict__ bc, const int* __restrict__ active) {
    constexpr int H = 2 * NU + 1;
    constexpr int EX = Tile2D<T, H>::EX, EY = Tile2D<T, H>::EY;
    __shared__ Tile2D<T, H> s;
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const int gx0 = blockIdx.x * kTileX - H, gy0 = blockIdx.y * kTileY - H;
    tile_load_common<T, H>(s, L, tr, ti, b + 2 * N * r, b + 2 * N * r + N, gx0, gy0);
    for (int c = threadIdx.x; c < EX * EY; c += blockDim.x) {
        const int lx = c % EX, ly = c / EX;
        s.xr[ly][lx] = 0;
        s.xi[ly][lx] = 0;
    }
    __syncthreads();
    tile_sweeps<T, H>(s, gx0, gy0, L.nx, L.ny, 2 * NU, 0);
    // interior -> x
    T* xr = x + 2 * N * r;
    T* xi = xr + N;
    for (int c = threadIdx.x; c < kTileX * kTileY; c += blockDim.x) {
        const int lx = H + c % kTileX, ly = H + c / kTileX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        if (gx < L.nx && gy < L.ny) {
            const int i = gx + L.nx * gy;
            xr[i] = s.xr[ly][lx];
            xi[i] = s.xi[ly][lx];
        }
    }
    // residual of the interior, summed per aggregate
    const int ctx = kTileX >> cox, cty = kTileY >> coy;
    const size_t Nc = (size_t)cnx * cny;
    for (int c = threadIdx.x; c < ctx * cty; c += blockDim.x) {
        const int X = blockIdx.x * ctx + c % ctx, Y = blockIdx.y * cty + c / ctx;
        if (X >= cnx || Y >= cny) continue;
        T ar = 0, ai = 0;
        for (int fy = (Y << coy); fy <= (Y << coy) + coy; ++fy)
            for (int fx = (X << cox); fx <= (X << cox) + cox; ++fx) {
                const int lx = fx - gx0, ly = fy - gy0;
                T ore = s.tx[ly][lx] * s.xr[ly][lx + 1] + s.tx[ly][lx - 1] * s.xr[ly][lx - 1] +
                        s.ty[ly][lx] * s.xr[ly + 1][lx] + s.ty[ly - 1][lx] * s.xr[ly - 1][lx];
                T oim = s.tx[ly][lx] * s.xi[ly][lx + 1] + s.tx[ly][lx - 1] * s.xi[ly][lx - 1] +
                        s.ty[ly][lx] * s.xi[ly + 1][lx] + s.ty[ly - 1][lx] * s.xi[ly - 1][lx];
                T axr = s.dr[ly][lx] * s.xr[ly][lx] - s.di[ly][lx] * s.xi[ly][lx] - ore;
                T axi = s.dr[ly][lx] * s.xi[ly][lx] + s.di[ly][lx] * s.xr[ly][lx] - oim;
                ar += s.br[ly][lx] - axr;
                ai += s.bi[ly][lx] - axi;
            }
        const size_t I = (size_t)X + (size_t)cnx * Y;
        bc[2 * Nc * r + I] = ar;
        bc[2 * Nc * r + Nc + I] = ai;
    }
}

// Cell-centred linear interpolation weights of one halved axis (ghost mirrored through the wall).
template <typename T>
__device__ __forceinline__ int prolong_axis(int f, int nc, int halved, T glo, T ghi, int* idx, T* w) {
    if (!halved) {
        idx[0] = f;
        w[0] = 1;
        return 1;
    }
    const int I = f >> 1;
    const int J = (f & 1) ? I + 1 : I - 1;
    idx[0] = I;
    if (J < 0) {
        w[0] = T(0.75) + T(0.25) * glo;
        return 1;
    }
    if (J >= nc) {
        w[0] = T(0.75) + T(0.25) * ghi;
        return 1;
    }
    w[0] = T(0.75);
    idx[1] = J;
    w[1] = T(0.25);
    return 2;
}

// x_out = post-smooth( x_in + P e_coarse )
template <typename T, int NU>
__global__ __launch_bounds__(256) void k_post2d(LevelView<T> L, T tr, T ti, const T* __restrict__ b,
                                                const T* __restrict__ xin, const T* __restrict__ ec, int cnx,
                                                int cny, int cox, int coy, T4 ghost, T* __restrict__ xout,
                                                const int* __restrict__ active) {
    constexpr int H = 2 * NU;
    constexpr int EX = Tile2D<T, H>::EX, EY = Tile2D<T, H>::EY;
    __shared__ Tile2D<T, H> s;
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const size_t Nc = (size_t)cnx * cny;
    const int gx0 = blockIdx.x * kTileX - H, gy0 = blockIdx.y * kTileY - H;
    tile_load_common<T, H>(s, L, tr, ti, b + 2 * N * r, b + 2 * N * r + N, gx0, gy0);
    const T* xr = xin + 2 * N * r;
    const T* xi = xr + N;
    const T* er = ec + 2 * Nc * r;
    const T* ei = er + Nc;
    for (int c = threadIdx.x; c < EX * EY; c += blockDim.x) {
        const int lx = c % EX, ly = c / EX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        T vr = 0, vi = 0;
        if (gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
            const int i = gx + L.nx * gy;
            int ix[2], iy[2];
            T wx[2], wy[2];
            const int nxp = prolong_axis<T>(gx, cnx, cox, (T)ghost.x, (T)ghost.y, ix, wx);
            const int nyp = prolong_axis<T>(gy, cny, coy, (T)ghost.z, (T)ghost.w, iy, wy);
            T pr = 0, pi = 0;
            for (int b2 = 0; b2 < nyp; ++b2)
                for (int a2 = 0; a2 < nxp; ++a2) {
                    const T w = wx[a2] * wy[b2];
                    const size_t J = (size_t)ix[a2] + (size_t)cnx * iy[b2];
                    pr += w * er[J];
                    pi += w * ei[J];
                }
            vr = xr[i] + pr;
            vi = xi[i] + pi;
        }
        s.xr[ly][lx] = vr;
        s.xi[ly][lx] = vi;
    }
    __syncthreads();
    tile_sweeps<T, H>(s, gx0, gy0, L.nx, L.ny, 2 * NU, 1);
    T* oxr = xout + 2 * N * r;
    T* oxi = oxr + N;
    for (int c = threadIdx.x; c < kTileX * kTileY; c += blockDim.x) {
        const int lx = H + c % kTileX, ly = H + c / kTileX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        if (gx < L.nx && gy < L.ny) {
            const int i = gx + L.nx * gy;
            oxr[i] = s.xr[ly][lx];
            oxi[i] = s.xi[ly][lx];
        }
    }
}

// ------------------------------------------------------------------ coarse levels in one workgroup
template <typename T>
__device__ __forceinline__ void cb_gs(const CBLevel<T>& L, T tr, T ti, T* xr, T* xi, const T* br, const T* bi,
                                      int color) {
    const int sy = L.nx, sz = L.nx * L.ny;
    for (int i = threadIdx.x; i < L.N; i += blockDim.x) {
        const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / sz;
        if (((x + y + z) & 1) != color) continue;
        T ore = 0, oim = 0;
        if (x + 1 < L.nx) { T t = L.Tx[i]; ore += t * xr[i + 1]; oim += t * xi[i + 1]; }
        if (x > 0) { T t = L.Tx[i - 1]; ore += t * xr[i - 1]; oim += t * xi[i - 1]; }
        if (y + 1 < L.ny) { T t = L.Ty[i]; ore += t * xr[i + sy]; oim += t * xi[i + sy]; }
        if (y > 0) { T t = L.Ty[i - sy]; ore += t * xr[i - sy]; oim += t * xi[i - sy]; }
        if (z + 1 < L.nz) { T t = L.Tz[i]; ore += t * xr[i + sz]; oim += t * xi[i + sz]; }
        if (z > 0) { T t = L.Tz[i - sz]; ore += t * xr[i - sz]; oim += t * xi[i - sz]; }
        T nr = br[i] + ore, ni = bi[i] + oim;
        T dr = L.D[i] + tr * L.m[i], di = ti * L.m[i];
        T dd = dr * dr + di * di;
        xr[i] = (nr * dr + ni * di) / dd;
        xi[i] = (ni * dr - nr * di) / dd;
    }
}

template <typename T>
__device__ __forceinline__ void cb_restrict(const CBLevel<T>& F, const CBLevel<T>& C, T tr, T ti, const T* xr,
                                            const T* xi, const T* br, const T* bi, T* cbr, T* cbi, T* cxr,
                                            T* cxi) {
    const int sy = F.nx, sz = F.nx * F.ny;
    for (int I = threadIdx.x; I < C.N; I += blockDim.x) {
        const int X = I % C.nx, Y = (I / C.nx) % C.ny, Z = I / (C.nx * C.ny);
        T ar = 0, ai = 0;
        for (int z = Z << C.coz; z <= (Z << C.coz) + C.coz; ++z)
            for (int y = Y << C.coy; y <= (Y << C.coy) + C.coy; ++y)
                for (int x = X << C.cox; x <= (X << C.cox) + C.cox; ++x) {
                    const int i = x + F.nx * (y + F.ny * z);
                    T ore = 0, oim = 0;
                    if (x + 1 < F.nx) { T t = F.Tx[i]; ore += t * xr[i + 1]; oim += t * xi[i + 1]; }
                    if (x > 0) { T t = F.Tx[i - 1]; ore += t * xr[i - 1]; oim += t * xi[i - 1]; }
                    if (y + 1 < F.ny) { T t = F.Ty[i]; ore += t * xr[i + sy]; oim += t * xi[i + sy]; }
                    if (y > 0) { T t = F.Ty[i - sy]; ore += t * xr[i - sy]; oim += t * xi[i - sy]; }
                    if (z + 1 < F.nz) { T t = F.Tz[i]; ore += t * xr[i + sz]; oim += t * xi[i + sz]; }
                    if (z > 0) { T t = F.Tz[i - sz]; ore += t * xr[i - sz]; oim += t * xi[i - sz]; }
                    T dr = F.D[i] + tr * F.m[i], di = ti * F.m[i];
                    ar += br[i] - (dr * xr[i] - di * xi[i] - ore);
                    ai += bi[i] - (dr * xi[i] + di * xr[i] - oim);
                }
        cbr[I] = ar;
        cbi[I] = ai;
        cxr[I] = 0;
        cxi[I] = 0;
    }
}

template <typename T>
__device__ __forceinline__ void cb_prolong(const CBLevel<T>& F, const CBLevel<T>& C, const T* g, T* xr, T* xi,
                                           const T* er, const T* ei) {
    for (int i = threadIdx.x; i < F.N; i += blockDim.x) {
        const int x = i % F.nx, y = (i / F.nx) % F.ny, z = i / (F.nx * F.ny);
        int ix[2], iy[2], iz[2];
        T wx[2], wy[2], wz[2];
        const int nxp = prolong_axis<T>(x, C.nx, C.cox, g[0], g[1], ix, wx);
        const int nyp = prolong_axis<T>(y, C.ny, C.coy, g[2], g[3], iy, wy);
        const int nzp = prolong_axis<T>(z, C.nz, C.coz, g[4], g[5], iz, wz);
        T pr = 0, pi = 0;
        for (int c = 0; c < nzp; ++c)
            for (int b = 0; b < nyp; ++b)
                for (int a = 0; a < nxp; ++a) {
                    const T w = wx[a] * wy[b] * wz[c];
                    const int J = ix[a] + C.nx * (iy[b] + C.ny * iz[c]);
                    pr += w * er[J];
                    pi += w * ei[J];
                }
        xr[i] += pr;
        xi[i] += pi;
    }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_block(CBMeta<T> M, T tr, T ti, const T* __restrict__ bin,
                                                       T* __restrict__ xout, const int* __restrict__ active) {
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    // per level: xr, xi, br, bi at offset 4 * off
    auto X = [&](int l) { return sm + 4 * (size_t)M.L[l].off; };
    const int n0 = M.L[0].N;
    {
        T* x = X(0);
        const T* b = bin + 2 * (size_t)n0 * r;
        for (int i = threadIdx.x; i < n0; i += blockDim.x) {
            x[i] = 0;
            x[n0 + i] = 0;
            x[2 * n0 + i] = b[i];
            x[3 * n0 + i] = b[n0 + i];
        }
    }
    __syncthreads();
    const int nl = M.nl;
    for (int l = 0; l < nl - 1; ++l) {
        const CBLevel<T>& L = M.L[l];
        T* p = X(l);
        for (int s = 0; s < M.nu1; ++s)
            for (int c = 0; c < 2; ++c) {
                cb_gs<T>(L, tr, ti, p, p + L.N, p + 2 * L.N, p + 3 * L.N, c);
                __syncthreads();
            }
        T* q = X(l + 1);
        const int nc = M.L[l + 1].N;
        cb_restrict<T>(L, M.L[l + 1], tr, ti, p, p + L.N, p + 2 * L.N, p + 3 * L.N, q + 2 * nc, q + 3 * nc, q,
                       q + nc);
        __syncthreads();
    }
    {
        const CBLevel<T>& L = M.L[nl - 1];
        T* p = X(nl - 1);
        if (M.inv) {
            for (int i = threadIdx.x; i < L.N; i += blockDim.x) {
                const T* row = M.inv + 2 * (size_t)L.N * i;
                T ar = 0, ai = 0;
                for (int j = 0; j < L.N; ++j) {
                    const T a = row[2 * j], bb = row[2 * j + 1];
                    const T vr = p[2 * L.N + j], vi = p[3 * L.N + j];
                    ar += a * vr - bb * vi;
                    ai += a * vi + bb * vr;
                }
                p[i] = ar;
                p[L.N + i] = ai;
            }
            __syncthreads();
        } else {
            for (int s = 0; s < M.coarse_sweeps; ++s)
                for (int c = 0; c < 2; ++c) {
                    cb_gs<T>(L, tr, ti, p, p + L.N, p + 2 * L.N, p + 3 * L.N, c);
                    __syncthreads();
                }
        }
    }
    for (int l = nl - 2; l >= 0; --l) {
        const CBLevel<T>& L = M.L[l];
        T* p = X(l);
        const T* q = X(l + 1);
        const int nc = M.L[l + 1].N;
        cb_prolong<T>(L, M.L[l + 1], M.ghost, p, p + L.N, q, q + nc);
        __syncthreads();
        for (int s = 0; s < M.nu2; ++s)
            for (int c = 1; c >= 0; --c) {
                cb_gs<T>(L, tr, ti, p, p + L.N, p + 2 * L.N, p + 3 * L.N, c);
                __syncthreads();
            }
    }
    {
        const T* x = X(0);
        T* o = xout + 2 * (size_t)n0 * r;
        for (int i = threadIdx.x; i < n0; i += blockDim.x) {
            o[i] = x[i];
            o[n0 + i] = x[n0 + i];
        }
    }
}

// ------------------------------------------------------------------ launchers
template <typename T>
int launch_pre2d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, const T* b, T* x, int cnx, int cny,
                 int cox, int coy, T* bc, int R, const int* active) {
    dim3 grid((L.nx + kTileX - 1) / kTileX, (L.ny + kTileY - 1) / kTileY, R);
    switch (nu) {
        case 1: k_pre2d<T, 1><<<grid, 256, 0, st>>>(L, tr, ti, b, x, cnx, cny, cox, coy, bc, active); break;
        case 2: k_pre2d<T, 2><<<grid, 256, 0, st>>>(L, tr, ti, b, x, cnx, cny, cox, coy, bc, active); break;
        case 3: k_pre2d<T, 3><<<grid, 256, 0, st>>>(L, tr, ti, b, x, cnx, cny, cox, coy, bc, active); break;
        default: set_last_error("fused smoother supports 1..3 sweeps"); return LT_EUNSUPPORTED;
    }
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_post2d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, const T* b, const T* xin,
                  const T* ec, int cnx, int cny, int cox, int coy, T4 ghost, T* xout, int R, const int* active) {
    dim3 grid((L.nx + kTileX - 1) / kTileX, (L.ny + kTileY - 1) / kTileY, R);
    switch (nu) {
        case 1: k_post2d<T, 1><<<grid, 256, 0, st>>>(L, tr, ti, b, xin, ec, cnx, cny, cox, coy, ghost, xout, active); break;
        case 2: k_post2d<T, 2><<<grid, 256, 0, st>>>(L, tr, ti, b, xin, ec, cnx, cny, cox, coy, ghost, xout, active); break;
        case 3: k_post2d<T, 3><<<grid, 256, 0, st>>>(L, tr, ti, b, xin, ec, cnx, cny, cox, coy, ghost, xout, active); break;
        default: set_last_error("fused smoother supports 1..3 sweeps"); return LT_EUNSUPPORTED;
    }
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_coarse_block(hipStream_t st, const CBMeta<T>& M, T tr, T ti, const T* bin, T* xout, int R,
                        const int* active) {
    size_t cells = 0;
    for (int l = 0; l < M.nl; ++l) cells += M.L[l].N;
    size_t shm = 4 * cells * sizeof(T);
    int threads = M.L[0].N >= 1024 ? 1024 : ((M.L[0].N + 63) / 64) * 64;
    if (threads < 64) threads = 64;
    k_coarse_block<T><<<R, threads, shm, st>>>(M, tr, ti, bin, xout, active);
    LT_HIP(hipGetLastError());
    return 0;
}

template int launch_pre2d<float>(hipStream_t, const LevelView<float>&, float, float, int, const float*, float*, int,
                                 int, int, int, float*, int, const int*);
template int launch_pre2d<double>(hipStream_t, const LevelView<double>&, double, double, int, const double*, double*,
                                  int, int, int, int, double*, int, const int*);
template int launch_post2d<float>(hipStream_t, const LevelView<float>&, float, float, int, const float*,
                                  const float*, const float*, int, int, int, int, T4, float*, int, const int*);
template int launch_post2d<double>(hipStream_t, const LevelView<double>&, double, double, int, const double*,
                                   const double*, const double*, int, int, int, int, T4, double*, int, const int*);
template int launch_coarse_block<float>(hipStream_t, const CBMeta<float>&, float, float, const float*, float*, int,
                                        const int*);
template int launch_coarse_block<double>(hipStream_t, const CBMeta<double>&, double, double, const double*, double*,
                                         int, const int*);

}  // namespace lt
