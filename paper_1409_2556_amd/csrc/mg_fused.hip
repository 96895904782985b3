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

#include <hip/hip_ext.h>

namespace lt {

template <typename T> struct cx {
    T re, im;
};

// ------------------------------------------------------------------ 2D tiles
// Colour-planar layout: cell (ly, lx) of the extended tile lives in plane (lx + ly) & 1 at
// ly * W + lx / 2.  The cells one half-sweep updates are then one plane, contiguous, so
// consecutive threads touch consecutive LDS banks (in row-major order every other word
// of a row, a two-way bank conflict on every access).  The plane size is 16 modulo 32,
// so the two colours of a row, loaded and stored by consecutive threads, also fall into
// different banks.
template <typename T, int H, int TX, int TY> struct Tile2D {
    static constexpr int EX = TX + 2 * H;
    static constexpr int EY = TY + 2 * H;
    static_assert(EX % 2 == 0, "tile rows hold whole colour pairs");
    static constexpr int W = EX / 2;  // cells of one colour in a row
    static constexpr int PL = EY * W + ((16 - (EY * W) % 32) + 32) % 32;
    static constexpr int NCELL = 2 * PL;
    T xr[NCELL], xi[NCELL];
    T br[NCELL], bi[NCELL];
    T tx[NCELL], ty[NCELL];
    T dr[NCELL], di[NCELL];  // inverse of the diagonal D + tau m
    __device__ static __forceinline__ int at(int ly, int lx) { return ((lx + ly) & 1) * PL + ly * W + (lx >> 1); }
    // cell (ly, lx) and its four neighbours (which lie in the other plane), from one parity
    __device__ static __forceinline__ void at5(int ly, int lx, int& c, int& e, int& w, int& n, int& so) {
        const int q = (lx + ly) & 1, k = lx >> 1;
        c = q * PL + ly * W + k;
        const int o = (1 - q) * PL + ly * W;
        e = o + ((lx + 1) >> 1);
        w = o + ((lx - 1) >> 1);
        n = o + W + k;
        so = o - W + k;
    }
};

// Element idx of an array with a uniform base: the byte offset is formed in 32 bits (every
// array these kernels index is far below 4 GiB), so the access takes the scalar base plus a
// 32-bit vector offset instead of a 64-bit address per thread.
template <typename T> __device__ __forceinline__ const T& el(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ T& el(T* base, unsigned idx) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}

// Sums of products are written as explicit fused multiply-adds in a fixed order, so every
// tile shape (a different template instance) rounds a cell's update identically.
template <typename T>
__device__ __forceinline__ T dot4(T a0, T b0, T a1, T b1, T a2, T b2, T a3, T b3) {
    return fma(a0, b0, fma(a1, b1, fma(a2, b2, a3 * b3)));
}

// nhalf half-sweeps of red-black Gauss-Seidel on the tile.  Threads walk the
// cells of the colour being updated only (half the cells of each row), and
// the tile holds the inverse of the complex diagonal, so an update is
// x = (b + off) / d with no division.
template <typename T, int H, int TX, int TY>
__device__ __forceinline__ void tile_sweeps(Tile2D<T, H, TX, TY>& s, int gx0, int gy0, int nx, int ny, int nhalf,
                                            int first_color) {
    using S = Tile2D<T, H, TX, TY>;
    constexpr int EX = S::EX, EY = S::EY, W = S::W, PL = S::PL;
    for (int hs = 0; hs < nhalf; ++hs) {
        const int color = (first_color + hs) & 1;
        const int q = (color + gx0 + gy0) & 1;  // the plane of this colour
        const int sh = hs + 1;
        const int nrow = EY - 2 * sh;
        for (int c = threadIdx.x; c < nrow * W; c += blockDim.x) {
            const int ly = sh + c / W, k = c % W;
            const int p = (q + ly) & 1;  // lx parity of this colour in row ly
            const int lx = 2 * k + p;
            if (lx < sh || lx >= EX - sh) continue;
            const int gx = gx0 + lx, gy = gy0 + ly;
            if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) continue;
            const int own = q * PL + ly * W + k;    // this cell
            const int oth = (1 - q) * PL + ly * W;  // row ly of the other colour
            const int e = oth + k + p, w = e - 1, n = oth + W + k, so = oth - W + k;
            const T ore = dot4(s.tx[own], s.xr[e], s.tx[w], s.xr[w], s.ty[own], s.xr[n], s.ty[so], s.xr[so]);
            const T oim = dot4(s.tx[own], s.xi[e], s.tx[w], s.xi[w], s.ty[own], s.xi[n], s.ty[so], s.xi[so]);
            const T nr = s.br[own] + ore, ni = s.bi[own] + oim;
            const T ir = s.dr[own], ii = s.di[own];
            s.xr[own] = fma(nr, ir, -(ni * ii));
            s.xi[own] = fma(nr, ii, ni * ir);
        }
        __syncthreads();
    }
}

// The two taps of prolong_axis with no branch on the count: a missing second tap gets
// weight 0 and the first tap's index (adding 0 * value leaves a sum unchanged, so sums
// over both taps equal sums over the taps prolong_axis returns).
template <typename T>
__device__ __forceinline__ void prolong_axis2(int f, int nc, int halved, T glo, T ghi, int& i0, int& i1, T& w0,
                                              T& w1) {
    if (!halved) {
        i0 = i1 = f;
        w0 = T(1);
        w1 = T(0);
        return;
    }
    const int I = f >> 1;
    const int J = (f & 1) ? I + 1 : I - 1;
    const bool lo = J < 0, hi = J >= nc;
    i0 = I;
    i1 = (lo || hi) ? I : J;
    w0 = lo ? T(0.75) + T(0.25) * glo : (hi ? T(0.75) + T(0.25) * ghi : T(0.75));
    w1 = (lo || hi) ? T(0) : T(0.25);
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

constexpr int kThreads = 256;  // every fused 2D kernel runs 256 threads

// Load coefficients and b of the extended tile; cells outside the grid get zero
// couplings, zero b and a unit diagonal (they are never updated).  Every
// thread issues the loads of all its cells before any is used (addresses are
// clamped into the grid, so no load depends on a branch), which keeps
// several loads in flight per thread instead of one cell at a time.  With
// PROLONG, x = xin + P e is formed from the coarse patch staged in pxr/pxi
// (which the caller loads and which may alias s.xr/s.xi: a barrier separates
// its last read from the first store here); otherwise x = 0.
template <typename T, int H, int TX, int TY, bool PROLONG>
__device__ __forceinline__ void tile_load(Tile2D<T, H, TX, TY>& s, const LevelView<T>& L, T tr, T ti,
                                          const T* __restrict__ br, const T* __restrict__ bi,
                                          const T* __restrict__ xr, const T* __restrict__ xi, int gx0, int gy0,
                                          const T* pxr, const T* pxi, int px0, int py0, int pnx, int cnx, int cny,
                                          int cox, int coy, T4 ghost) {
    constexpr int EX = Tile2D<T, H, TX, TY>::EX, EY = Tile2D<T, H, TX, TY>::EY;
    constexpr int NC = EX * EY, NL = (NC + kThreads - 1) / kThreads;
    T vtx[NL], vty[NL], vd[NL], vm[NL], vbr[NL], vbi[NL], vxr[NL], vxi[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int c = threadIdx.x + kThreads * k;
        const int lx = c % EX, ly = c / EX;
        const int gx = min(max(gx0 + lx, 0), L.nx - 1), gy = min(max(gy0 + ly, 0), L.ny - 1);
        const unsigned i = (unsigned)(gx + L.nx * gy);
        vtx[k] = el(L.Tx, i);
        vty[k] = el(L.Ty, i);
        vd[k] = el(L.D, i);
        vm[k] = el(L.m, i);
        vbr[k] = el(br, i);
        vbi[k] = el(bi, i);
        if (PROLONG) {
            vxr[k] = el(xr, i);
            vxi[k] = el(xi, i);
        }
    }
    if (PROLONG) {
        // coarse correction, interpolated from the staged patch
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int c = threadIdx.x + kThreads * k;
            const int gx = gx0 + c % EX, gy = gy0 + c / EX;
            if (c < NC && gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny) {
                int x0, x1, y0, y1;
                T wx0, wx1, wy0, wy1;
                prolong_axis2<T>(gx, cnx, cox, (T)ghost.x, (T)ghost.y, x0, x1, wx0, wx1);
                prolong_axis2<T>(gy, cny, coy, (T)ghost.z, (T)ghost.w, y0, y1, wy0, wy1);
                const int r0 = pnx * (y0 - py0) - px0, r1 = pnx * (y1 - py0) - px0;
                T pr = 0, pi = 0;
                pr = fma(wx0 * wy0, pxr[r0 + x0], pr);
                pi = fma(wx0 * wy0, pxi[r0 + x0], pi);
                pr = fma(wx1 * wy0, pxr[r0 + x1], pr);
                pi = fma(wx1 * wy0, pxi[r0 + x1], pi);
                pr = fma(wx0 * wy1, pxr[r1 + x0], pr);
                pi = fma(wx0 * wy1, pxi[r1 + x0], pi);
                pr = fma(wx1 * wy1, pxr[r1 + x1], pr);
                pi = fma(wx1 * wy1, pxi[r1 + x1], pi);
                vxr[k] += pr;
                vxi[k] += pi;
            }
        }
        __syncthreads();  // the patch may alias s.xr / s.xi
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int c = threadIdx.x + kThreads * k;
        if (c >= NC) continue;
        const int lx = c % EX, ly = c / EX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        const bool in = gx >= 0 && gx < L.nx && gy >= 0 && gy < L.ny;
        const int a = s.at(ly, lx);
        s.tx[a] = in ? vtx[k] : T(0);
        s.ty[a] = in ? vty[k] : T(0);
        // inverse of the diagonal D + tau m (1 outside the grid)
        const T dr = in ? fma(tr, vm[k], vd[k]) : T(1), di = in ? ti * vm[k] : T(0);
        const T rdd = T(1) / fma(dr, dr, di * di);
        s.dr[a] = dr * rdd;
        s.di[a] = -di * rdd;
        s.br[a] = in ? vbr[k] : T(0);
        s.bi[a] = in ? vbi[k] : T(0);
        s.xr[a] = (PROLONG && in) ? vxr[k] : T(0);
        s.xi[a] = (PROLONG && in) ? vxi[k] : T(0);
    }
}

// Stage the coarse cells the tile's prolongation reads (a patch of at most
// (EX/2 + 3) x EY or EX x (EY/2 + 3) cells) in pxr/pxi; returns its origin
// and width.  Followed by a barrier.
template <typename T, int H, int TX, int TY>
__device__ __forceinline__ void stage_patch(const T* __restrict__ er, const T* __restrict__ ei, int gx0, int gy0,
                                            int nx, int ny, int cnx, int cny, int cox, int coy, T* pxr, T* pxi,
                                            int* px0, int* py0, int* pnx) {
    constexpr int EX = Tile2D<T, H, TX, TY>::EX, EY = Tile2D<T, H, TX, TY>::EY;
    const int fx0 = max(gx0, 0), fx1 = min(gx0 + EX - 1, nx - 1);
    const int fy0 = max(gy0, 0), fy1 = min(gy0 + EY - 1, ny - 1);
    const int x0 = cox ? max((fx0 >> 1) - 1, 0) : fx0, x1 = cox ? min((fx1 >> 1) + 1, cnx - 1) : fx1;
    const int y0 = coy ? max((fy0 >> 1) - 1, 0) : fy0, y1 = coy ? min((fy1 >> 1) + 1, cny - 1) : fy1;
    const int w = x1 - x0 + 1, hgt = y1 - y0 + 1;
    constexpr int MAXP = (EX * (EY / 2 + 3) > (EX / 2 + 3) * EY) ? EX * (EY / 2 + 3) : (EX / 2 + 3) * EY;
    static_assert(MAXP <= Tile2D<T, H, TX, TY>::NCELL, "the patch is staged in one tile array");
    constexpr int NP = (MAXP + kThreads - 1) / kThreads;
    T vr[NP], vi[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int c = min((int)threadIdx.x + kThreads * k, w * hgt - 1);
        const unsigned J = (unsigned)((x0 + c % w) + cnx * (y0 + c / w));
        vr[k] = el(er, J);
        vi[k] = el(ei, J);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int c = threadIdx.x + kThreads * k;
        if (c < w * hgt) {
            pxr[c] = vr[k];
            pxi[c] = vi[k];
        }
    }
    *px0 = x0;
    *py0 = y0;
    *pnx = w;
    __syncthreads();
}

// Pre-smoothing from x = 0, then restriction of the residual.
template <typename T, int NU, int TX, int TY>
__global__ __launch_bounds__(256) void k_pre2d(LevelView<T> L, T tr, T ti, const T* __restrict__ b,
                                               T* __restrict__ x, int cnx, int cny, int cox, int coy,
                                               T* __restrict__ bc, const int* __restrict__ active,
                                               unsigned long long* __restrict__ prof, int Rtot) {
    constexpr int H = 2 * NU + 1;
    __shared__ Tile2D<T, H, TX, TY> s;
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const int gx0 = blockIdx.x * TX - H, gy0 = blockIdx.y * TY - H;
    tile_load<T, H, TX, TY, false>(s, L, tr, ti, b + 2 * N * r, b + 2 * N * r + N, nullptr, nullptr, gx0, gy0, nullptr,
                           nullptr, 0, 0, 0, cnx, cny, cox, coy, T4{});
    __syncthreads();
    tile_sweeps<T, H, TX, TY>(s, gx0, gy0, L.nx, L.ny, 2 * NU, 0);
    // interior -> x
    T* xr = x + 2 * N * r;
    T* xi = xr + N;
    for (int c = threadIdx.x; c < TX * TY; c += blockDim.x) {
        const int lx = H + c % TX, ly = H + c / TX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        if (gx < L.nx && gy < L.ny) {
            const unsigned i = (unsigned)(gx + L.nx * gy);
            el(xr, i) = s.xr[s.at(ly, lx)];
            el(xi, i) = s.xi[s.at(ly, lx)];
        }
    }
    // residual of the interior, summed per aggregate
    const int ctx = TX >> cox, cty = TY >> coy;
    const size_t Nc = (size_t)cnx * cny;
    T* bcr = bc + 2 * Nc * r;
    T* bci = bcr + Nc;
    for (int c = threadIdx.x; c < ctx * cty; c += blockDim.x) {
        const int X = blockIdx.x * ctx + c % ctx, Y = blockIdx.y * cty + c / ctx;
        if (X >= cnx || Y >= cny) continue;
        T ar = 0, ai = 0;
        for (int fy = (Y << coy); fy <= (Y << coy) + coy; ++fy)
            for (int fx = (X << cox); fx <= (X << cox) + cox; ++fx) {
                const int lx = fx - gx0, ly = fy - gy0;
                int c0, ce, cw, cn, cs;
                s.at5(ly, lx, c0, ce, cw, cn, cs);
                const T ore = dot4(s.tx[c0], s.xr[ce], s.tx[cw], s.xr[cw], s.ty[c0], s.xr[cn], s.ty[cs], s.xr[cs]);
                const T oim = dot4(s.tx[c0], s.xi[ce], s.tx[cw], s.xi[cw], s.ty[c0], s.xi[cn], s.ty[cs], s.xi[cs]);
                // the tile holds the inverse diagonal: take D + tau m from the level arrays
                const unsigned fi = (unsigned)(fx + L.nx * fy);
                const T dm = el(L.m, fi), dre = fma(tr, dm, el(L.D, fi)), dim = ti * dm;
                const T axr = fma(dre, s.xr[c0], -(dim * s.xi[c0])) - ore;
                const T axi = fma(dre, s.xi[c0], dim * s.xr[c0]) - oim;
                ar += s.br[c0] - axr;
                ai += s.bi[c0] - axi;
            }
        const unsigned I = (unsigned)(X + cnx * Y);
        el(bcr, I) = ar;
        el(bci, I) = ai;
    }
    if (prof && threadIdx.x == 0 && blockIdx.x == 0 && blockIdx.y == 0) {
        // algorithmic bytes of this right-hand side over the level (one count per
        // right-hand side and launch): b in, x out (complex), the coefficient arrays
        // Tx, Ty, D, m shared by the Rtot right-hand sides, coarse rhs out
        const double cell = 4.0 * sizeof(T) + 4.0 * sizeof(T) / Rtot;
        atomicAdd(prof, (unsigned long long)((double)L.N * cell + (double)Nc * 2.0 * sizeof(T)));
    }
}

// x_out = post-smooth( x_in + P e_coarse )
template <typename T, int NU, int TX, int TY>
__global__ __launch_bounds__(256) void k_post2d(LevelView<T> L, T tr, T ti, const T* __restrict__ b,
                                                const T* __restrict__ xin, const T* __restrict__ ec, int cnx,
                                                int cny, int cox, int coy, T4 ghost, T* __restrict__ xout,
                                                const int* __restrict__ active, unsigned long long* __restrict__ prof,
                                                int Rtot) {
    constexpr int H = 2 * NU;
    __shared__ Tile2D<T, H, TX, TY> s;
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const size_t Nc = (size_t)cnx * cny;
    const int gx0 = blockIdx.x * TX - H, gy0 = blockIdx.y * TY - H;
    const T* er = ec + 2 * Nc * r;
    int px0, py0, pnx;
    stage_patch<T, H, TX, TY>(er, er + Nc, gx0, gy0, L.nx, L.ny, cnx, cny, cox, coy, s.xr, s.xi, &px0, &py0,
                      &pnx);
    tile_load<T, H, TX, TY, true>(s, L, tr, ti, b + 2 * N * r, b + 2 * N * r + N, xin + 2 * N * r, xin + 2 * N * r + N,
                          gx0, gy0, s.xr, s.xi, px0, py0, pnx, cnx, cny, cox, coy, ghost);
    __syncthreads();
    tile_sweeps<T, H, TX, TY>(s, gx0, gy0, L.nx, L.ny, 2 * NU, 1);
    T* oxr = xout + 2 * N * r;
    T* oxi = oxr + N;
    for (int c = threadIdx.x; c < TX * TY; c += blockDim.x) {
        const int lx = H + c % TX, ly = H + c / TX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        if (gx < L.nx && gy < L.ny) {
            const unsigned i = (unsigned)(gx + L.nx * gy);
            el(oxr, i) = s.xr[s.at(ly, lx)];
            el(oxi, i) = s.xi[s.at(ly, lx)];
        }
    }
    if (prof && threadIdx.x == 0 && blockIdx.x == 0 && blockIdx.y == 0) {
        // algorithmic bytes of this right-hand side over the level: x in, b in, x out
        // (complex), shared coefficients, and the coarse correction in
        const double cell = 6.0 * sizeof(T) + 4.0 * sizeof(T) / Rtot;
        atomicAdd(prof, (unsigned long long)((double)L.N * cell + (double)Nc * 2.0 * sizeof(T)));
    }
}

// Fine-level post-smoothing fused with one step of the FP64 iterative
// refinement of the preconditioner solve: with e the V-cycle output,
//   u += e,  rho_out = rho_in - (K + tau M) e  (FP64 coefficients),
//   lo = (T) rho_out,  part[r][block] = ||rho_out||^2 over the block.
// One more halo ring than the plain post-smoother keeps e exact next to the
// interior, so A e is exact there.  rho_in and the input b of the tile may be
// the same buffer; rho_out and lo must not alias anything read here.
template <typename T, int NU, int TX, int TY>
__global__ __launch_bounds__(256) void k_post2d_refine(LevelView<T> L, LevelView<double> L64, T tr, T ti,
                                                       double tr64, double ti64, const T* __restrict__ b,
                                                       const T* __restrict__ xin, const T* __restrict__ ec,
                                                       int cnx, int cny, int cox, int coy, T4 ghost,
                                                       double* __restrict__ u, size_t ustride,
                                                       const int* __restrict__ jcol,
                                                       const double* rho_in, double* rho_out,
                                                       T* __restrict__ lo, double* __restrict__ part,
                                                       const int* __restrict__ active,
                                                       unsigned long long* __restrict__ prof, int Rtot) {
    constexpr int H = 2 * NU + 1;
    __shared__ Tile2D<T, H, TX, TY> s;
    __shared__ double red[4];
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const size_t Nc = (size_t)cnx * cny;
    const int gx0 = blockIdx.x * TX - H, gy0 = blockIdx.y * TY - H;
    const T* er = ec + 2 * Nc * r;
    int px0, py0, pnx;
    stage_patch<T, H, TX, TY>(er, er + Nc, gx0, gy0, L.nx, L.ny, cnx, cny, cox, coy, s.xr, s.xi, &px0, &py0,
                      &pnx);
    tile_load<T, H, TX, TY, true>(s, L, tr, ti, b + 2 * N * r, b + 2 * N * r + N, xin + 2 * N * r, xin + 2 * N * r + N,
                          gx0, gy0, s.xr, s.xi, px0, py0, pnx, cnx, cny, cox, coy, ghost);
    // the FP64 operands of the update do not depend on the sweeps: load them first so
    // their latency overlaps the LDS work
    double* ur = u + ustride * r + (jcol ? 2 * N * (size_t)*jcol : 0);
    double* ui = ur + N;
    const double* rin = rho_in + 2 * N * r;
    const double* rini = rin + N;
    double* rout = rho_out + 2 * N * r;
    double* routi = rout + N;
    T* lor = lo ? lo + 2 * N * r : nullptr;
    T* loi = lo ? lor + N : nullptr;
    constexpr int NI = (TX * TY + kThreads - 1) / kThreads;
    double vte[NI], vtw[NI], vtn[NI], vts[NI], vd[NI], vm[NI], vur[NI], vui[NI], vrr[NI], vri[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int c = min((int)threadIdx.x + kThreads * k, TX * TY - 1);
        const int gx = min(gx0 + H + c % TX, L.nx - 1), gy = min(gy0 + H + c / TX, L.ny - 1);
        const int i = gx + L.nx * gy;
        const unsigned iu = (unsigned)i;
        vte[k] = el(L64.Tx, iu);
        vtw[k] = el(L64.Tx, (unsigned)max(i - 1, 0));
        vtn[k] = el(L64.Ty, iu);
        vts[k] = el(L64.Ty, (unsigned)max(i - L.nx, 0));
        vd[k] = el(L64.D, iu);
        vm[k] = el(L64.m, iu);
        vur[k] = el((const double*)ur, iu);
        vui[k] = el((const double*)ui, iu);
        vrr[k] = el(rin, iu);
        vri[k] = el(rini, iu);
    }
    __syncthreads();
    tile_sweeps<T, H, TX, TY>(s, gx0, gy0, L.nx, L.ny, 2 * NU, 1);
    double acc = 0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int c = threadIdx.x + kThreads * k;
        const int lx = H + c % TX, ly = H + c / TX;
        const int gx = gx0 + lx, gy = gy0 + ly;
        if (c >= TX * TY || gx >= L.nx || gy >= L.ny) continue;
        const unsigned i = (unsigned)(gx + L.nx * gy);
        int c0, ce, cw, cn, cs;
        s.at5(ly, lx, c0, ce, cw, cn, cs);
        const double e0r = (double)s.xr[c0], e0i = (double)s.xi[c0];
        // (K + tau M) e with the FP64 operator; walls are in D, out-of-grid neighbours hold 0
        const double tE = vte[k], tW = gx > 0 ? vtw[k] : 0.0;
        const double tN = vtn[k], tS = gy > 0 ? vts[k] : 0.0;
        const double ore = dot4(tE, (double)s.xr[ce], tW, (double)s.xr[cw], tN, (double)s.xr[cn], tS, (double)s.xr[cs]);
        const double oim = dot4(tE, (double)s.xi[ce], tW, (double)s.xi[cw], tN, (double)s.xi[cn], tS, (double)s.xi[cs]);
        const double dre = fma(tr64, vm[k], vd[k]), dim = ti64 * vm[k];
        const double are = fma(dre, e0r, -(dim * e0i)) - ore;
        const double aim = fma(dre, e0i, dim * e0r) - oim;
        el(ur, i) = vur[k] + e0r;
        el(ui, i) = vui[k] + e0i;
        const double nre = vrr[k] - are, nim = vri[k] - aim;
        el(rout, i) = nre;
        el(routi, i) = nim;
        if (lo) {
            el(lor, i) = (T)nre;
            el(loi, i) = (T)nim;
        }
        acc += nre * nre + nim * nim;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        part[(size_t)r * gridDim.x * gridDim.y + blockIdx.x + (size_t)gridDim.x * blockIdx.y] =
            red[0] + red[1] + red[2] + red[3];
        if (prof && blockIdx.x == 0 && blockIdx.y == 0) {
            // algorithmic bytes of this right-hand side over the level: x in, b in
            // (T complex), shared T coefficients, coarse correction in, u in/out and rho
            // in/out (FP64 complex), lo out (T complex), FP64 coefficients (shared)
            const double cell = 4.0 * sizeof(T) + 4.0 * sizeof(T) / Rtot + 64.0 + (lo ? 2.0 * sizeof(T) : 0.0) +
                                32.0 / Rtot;
            atomicAdd(prof, (unsigned long long)((double)L.N * cell + (double)Nc * 2.0 * sizeof(T)));
        }
    }
}

// ------------------------------------------------------------------ coarse levels in one workgroup
// Thread i owns cell i of every level (levels have at most blockDim cells): its
// face transmissibilities, diagonal, right-hand side, neighbour indices and
// colour stay in registers, iterates and residuals go through LDS.
template <typename T> struct CBCell {
    T tw, te, ts, tn, tb, tt;  // faces to the -x, +x, -y, +y, -z, +z neighbours
    T dr, di;                  // D + tau m
    T ir, ii;                  // 1 / (D + tau m)
    T br, bi;                  // right-hand side of this level
    int x, y, z;               // coordinates of the cell
    int flags;                 // bits 0-5: neighbour exists at +x, -x, +y, -y, +z, -z; bit 6: colour
};

// Coefficients of cell i as loaded, before walls are applied.  Every address is valid
// whatever the cell (clamped), so the loads of all levels are issued before any is used.
template <typename T> struct CBRaw {
    T tx, txw, ty, tys, tz, tzb, d, m;
};

// D3: the levels have more than one layer (2D grids skip every z term)
template <typename T, bool D3>
__device__ __forceinline__ void cb_load_raw(const CBLevel<T>& L, int i, CBRaw<T>& q) {
    const int k = min(i, L.N - 1), sy = L.nx, sz = L.nx * L.ny;
    q.tx = L.Tx[k];
    q.txw = L.Tx[max(k - 1, 0)];
    q.ty = L.Ty[k];
    q.tys = L.Ty[max(k - sy, 0)];
    if (D3) {
        q.tz = L.Tz[k];
        q.tzb = L.Tz[max(k - sz, 0)];
    }
    q.d = L.D[k];
    q.m = L.m[k];
}

template <typename T, bool D3>
__device__ __forceinline__ void cb_make_cell(const CBLevel<T>& L, const CBRaw<T>& q, T tr, T ti, int i,
                                             CBCell<T>& c) {
    const int x = i % L.nx, y = (i / L.nx) % L.ny, z = D3 ? i / (L.nx * L.ny) : 0;
    c.x = x;
    c.y = y;
    c.z = z;
    c.flags = (x + 1 < L.nx) | ((x > 0) << 1) | ((y + 1 < L.ny) << 2) | ((y > 0) << 3) | ((z + 1 < L.nz) << 4) |
              ((z > 0) << 5) | (((x + y + z) & 1) << 6);
    // walls have zero couplings
    c.te = (x + 1 < L.nx) ? q.tx : T(0);
    c.tw = (x > 0) ? q.txw : T(0);
    c.tn = (y + 1 < L.ny) ? q.ty : T(0);
    c.ts = (y > 0) ? q.tys : T(0);
    if (D3) {
        c.tt = (z + 1 < L.nz) ? q.tz : T(0);
        c.tb = (z > 0) ? q.tzb : T(0);
    } else {
        c.tt = c.tb = T(0);
    }
    c.dr = q.d + tr * q.m;
    c.di = ti * q.m;
    const T dd = c.dr * c.dr + c.di * c.di;
    c.ir = c.dr / dd;
    c.ii = -c.di / dd;
}

// off = sum of couplings times neighbour values (a missing neighbour reads the cell itself with weight 0)
template <typename T, bool D3>
__device__ __forceinline__ void cb_off(const CBLevel<T>& L, const CBCell<T>& c, const T* xr, const T* xi, int i,
                                       T& ore, T& oim) {
    const int sy = L.nx, f = c.flags;
    const int e = (f & 1) ? i + 1 : i, w = (f & 2) ? i - 1 : i;
    const int n = (f & 4) ? i + sy : i, s = (f & 8) ? i - sy : i;
    ore = c.te * xr[e] + c.tw * xr[w] + c.tn * xr[n] + c.ts * xr[s];
    oim = c.te * xi[e] + c.tw * xi[w] + c.tn * xi[n] + c.ts * xi[s];
    if (D3) {
        const int sz = L.nx * L.ny;
        const int t = (f & 16) ? i + sz : i, b = (f & 32) ? i - sz : i;
        ore += c.tt * xr[t] + c.tb * xr[b];
        oim += c.tt * xi[t] + c.tb * xi[b];
    }
}

// one Gauss-Seidel update of cell i: x = (b + off) / (D + tau m)
template <typename T, bool D3>
__device__ __forceinline__ void cb_relax(const CBLevel<T>& L, const CBCell<T>& c, T* xr, T* xi, int i) {
    T ore, oim;
    cb_off<T, D3>(L, c, xr, xi, i, ore, oim);
    const T nr = c.br + ore, ni = c.bi + oim;
    xr[i] = nr * c.ir - ni * c.ii;
    xi[i] = nr * c.ii + ni * c.ir;
}

constexpr int kCBInvRegs = 8;  // inverse entries per lane held in registers from the kernel's start

template <typename T, int NLM, bool D3>
__global__ __launch_bounds__(1024) void k_coarse_block(CBMeta<T> M, T tr, T ti, const T* __restrict__ bin,
                                                       T* __restrict__ xout, const int* __restrict__ active) {
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);  // per level: xr, xi, rr, ri at 4 * off
    const int i = threadIdx.x;
    const int nl = M.nl;
    // Dense solve of the coarsest level, x = inv * r: P consecutive lanes share a row (P a
    // power of two, at most 64, as many as the block allows).  Each lane's entries of the
    // inverse are loaded now, so their latency overlaps the descent.
    int nc = 0;  // (compile-time indices only: a runtime index into the kernel argument
                 // struct becomes a chain of dependent scalar loads)
#pragma unroll
    for (int l = 0; l < NLM; ++l)
        if (l == nl - 1) nc = M.L[l].N;
    int P = 1, lp = 0;
    while (P < 64 && 2 * P * nc <= (int)blockDim.x) {
        P *= 2;
        ++lp;
    }
    const int row = i >> lp, seg = i & (P - 1);
    const bool inv_regs = M.inv && (nc + P - 1) / P <= kCBInvRegs;
    T ia[kCBInvRegs], ib[kCBInvRegs];
    if (inv_regs && row < nc) {
        const T* rowp = M.inv + 2 * (size_t)nc * row;
#pragma unroll
        for (int t = 0; t < kCBInvRegs; ++t) {
            const int j = seg + t * P;
            ia[t] = j < nc ? rowp[2 * j] : T(0);
            ib[t] = j < nc ? rowp[2 * j + 1] : T(0);
        }
    }
    CBRaw<T> raw[NLM];
#pragma unroll
    for (int l = 0; l < NLM; ++l)
        if (l < nl) cb_load_raw<T, D3>(M.L[l], i, raw[l]);
    CBCell<T> c[NLM];
#pragma unroll
    for (int l = 0; l < NLM; ++l)
        if (l < nl && i < M.L[l].N) cb_make_cell<T, D3>(M.L[l], raw[l], tr, ti, i, c[l]);
    {
        const int n0 = M.L[0].N;
        if (i < n0) {
            const T* b = bin + 2 * (size_t)n0 * r;
            c[0].br = b[i];
            c[0].bi = b[n0 + i];
            T* p = sm + 4 * (size_t)M.L[0].off;
            p[i] = 0;
            p[n0 + i] = 0;
        }
    }
    __syncthreads();
    // down
#pragma unroll
    for (int l = 0; l < NLM - 1; ++l) {
        if (l + 1 >= nl) break;
        const CBLevel<T>& L = M.L[l];
        T* xr = sm + 4 * (size_t)L.off;
        T* xi = xr + L.N;
        T* rr = xi + L.N;
        T* ri = rr + L.N;
        const bool own = i < L.N;
        const int par = own ? (c[l].flags >> 6) & 1 : 0;
        for (int sw = 0; sw < M.nu1; ++sw)
            for (int col = 0; col < 2; ++col) {
                if (own && par == col) cb_relax<T, D3>(L, c[l], xr, xi, i);
                __syncthreads();
            }
        if (own) {
            T ore, oim;
            cb_off<T, D3>(L, c[l], xr, xi, i, ore, oim);
            rr[i] = c[l].br - (c[l].dr * xr[i] - c[l].di * xi[i] - ore);
            ri[i] = c[l].bi - (c[l].dr * xi[i] + c[l].di * xr[i] - oim);
        }
        __syncthreads();
        const CBLevel<T>& C = M.L[l + 1];
        if (i < C.N) {
            // the aggregate of coarse cell i: up to two fine cells along each halved axis
            const int f0 = (c[l + 1].x << C.cox) + L.nx * ((c[l + 1].y << C.coy) + L.ny * (c[l + 1].z << C.coz));
            const int sy = L.nx, sz = L.nx * L.ny;
            T ar = 0, ai = 0;
#pragma unroll
            for (int dz = 0; dz < (D3 ? 2 : 1); ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx)
                        if (dz <= C.coz && dy <= C.coy && dx <= C.cox) {
                            const int f = f0 + dx + sy * dy + sz * dz;
                            ar += rr[f];
                            ai += ri[f];
                        }
            c[l + 1].br = ar;
            c[l + 1].bi = ai;
            T* q = sm + 4 * (size_t)C.off;
            q[i] = 0;
            q[C.N + i] = 0;
        }
        __syncthreads();
    }
    // coarsest level
#pragma unroll
    for (int l = 0; l < NLM; ++l) {
        if (l != nl - 1) continue;
        const CBLevel<T>& L = M.L[l];
        T* xr = sm + 4 * (size_t)L.off;
        T* xi = xr + L.N;
        T* rr = xi + L.N;
        T* ri = rr + L.N;
        const bool own = i < L.N;
        if (M.inv) {
            if (own) {
                rr[i] = c[l].br;
                ri[i] = c[l].bi;
            }
            __syncthreads();
            // the partial sums of a row's P lanes meet in a shuffle reduction
            const int n = L.N;
            T ar = 0, ai = 0;
            if (row < n) {
                if (inv_regs) {
#pragma unroll
                    for (int t = 0; t < kCBInvRegs; ++t) {
                        const int j = seg + t * P;
                        if (j < n) {
                            ar += ia[t] * rr[j] - ib[t] * ri[j];
                            ai += ia[t] * ri[j] + ib[t] * rr[j];
                        }
                    }
                } else {
                    const T* rowp = M.inv + 2 * (size_t)n * row;
                    for (int j = seg; j < n; j += P) {
                        const T a = rowp[2 * j], bb = rowp[2 * j + 1];
                        ar += a * rr[j] - bb * ri[j];
                        ai += a * ri[j] + bb * rr[j];
                    }
                }
            }
            for (int o = P / 2; o > 0; o >>= 1) {
                ar += __shfl_xor(ar, o, 64);
                ai += __shfl_xor(ai, o, 64);
            }
            if (row < n && seg == 0) {
                xr[row] = ar;
                xi[row] = ai;
            }
            __syncthreads();
        } else {
            const int par = own ? (c[l].flags >> 6) & 1 : 0;
            for (int sw = 0; sw < M.coarse_sweeps; ++sw)
                for (int col = 0; col < 2; ++col) {
                    if (own && par == col) cb_relax<T, D3>(L, c[l], xr, xi, i);
                    __syncthreads();
                }
        }
    }
    // up
#pragma unroll
    for (int l = NLM - 2; l >= 0; --l) {
        if (l + 1 >= nl) continue;
        const CBLevel<T>& L = M.L[l];
        const CBLevel<T>& C = M.L[l + 1];
        T* xr = sm + 4 * (size_t)L.off;
        T* xi = xr + L.N;
        const T* er = sm + 4 * (size_t)C.off;
        const T* ei = er + C.N;
        const bool own = i < L.N;
        if (own) {
            const int x = c[l].x, y = c[l].y, z = c[l].z;
            int ix[2], iy[2], iz[2];
            T wx[2], wy[2], wz[2];
            const int nxp = prolong_axis<T>(x, C.nx, C.cox, M.ghost[0], M.ghost[1], ix, wx);
            const int nyp = prolong_axis<T>(y, C.ny, C.coy, M.ghost[2], M.ghost[3], iy, wy);
            const int nzp = prolong_axis<T>(z, C.nz, C.coz, M.ghost[4], M.ghost[5], iz, wz);
            T pr = 0, pi = 0;
            for (int cz = 0; cz < nzp; ++cz)
                for (int cy = 0; cy < nyp; ++cy)
                    for (int cxx = 0; cxx < nxp; ++cxx) {
                        const T w = wx[cxx] * wy[cy] * wz[cz];
                        const int J = ix[cxx] + C.nx * (iy[cy] + C.ny * iz[cz]);
                        pr += w * er[J];
                        pi += w * ei[J];
                    }
            xr[i] += pr;
            xi[i] += pi;
        }
        __syncthreads();
        const int par = own ? (c[l].flags >> 6) & 1 : 0;
        for (int sw = 0; sw < M.nu2; ++sw)
            for (int col = 1; col >= 0; --col) {
                if (own && par == col) cb_relax<T, D3>(L, c[l], xr, xi, i);
                __syncthreads();
            }
    }
    {
        const int n0 = M.L[0].N;
        if (i < n0) {
            const T* x = sm + 4 * (size_t)M.L[0].off;
            T* o = xout + 2 * (size_t)n0 * r;
            o[i] = x[i];
            o[n0 + i] = x[n0 + i];
        }
    }
}

// ------------------------------------------------------------------ launchers
// Tile shapes (interior cells per workgroup); the id is what lt_autotune picks per level.
int tile_shape(int id, int* tx, int* ty) {
    static const int shapes[kNumTiles][2] = {{32, 16}, {64, 8}, {16, 16}, {16, 8}};
    if (id < 0 || id >= kNumTiles) return LT_EINVAL;
    *tx = shapes[id][0];
    *ty = shapes[id][1];
    return 0;
}

// Launch a kernel; with profiling events, through hipExtLaunchKernel so that the
// events bracket exactly this kernel's execution.
#define LT_LAUNCH(KERNEL, GRID, EV0, EV1, ...)                                              \
    do {                                                                                    \
        if (EV0)                                                                            \
            hipExtLaunchKernelGGL(KERNEL, GRID, dim3(kThreads), 0, st, EV0, EV1, 0, __VA_ARGS__); \
        else                                                                                \
            KERNEL<<<GRID, kThreads, 0, st>>>(__VA_ARGS__);                                 \
    } while (0)

// expands F(TX, TY) for the tile id, F(NU) for the sweep count
#define LT_TILE_SWITCH(id, F)                                                    \
    switch (id) {                                                                \
        case 0: F(32, 16); break;                                                \
        case 1: F(64, 8); break;                                                 \
        case 2: F(16, 16); break;                                                \
        case 3: F(16, 8); break;                                                 \
        default: set_last_error("unknown tile shape"); return LT_EINVAL;         \
    }

template <typename T>
int launch_pre2d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b, T* x, int cnx,
                 int cny, int cox, int coy, T* bc, int R, const int* active, unsigned long long* prof,
                 hipEvent_t ev0, hipEvent_t ev1) {
    if (nu < 1 || nu > 3) {
        set_last_error("fused smoother supports 1..3 sweeps");
        return LT_EUNSUPPORTED;
    }
#define LT_K(NU, X, Y)                                                                                \
    LT_LAUNCH((k_pre2d<T, NU, X, Y>), dim3((L.nx + X - 1) / X, (L.ny + Y - 1) / Y, R), ev0, ev1, L, tr, ti, b, \
              x, cnx, cny, cox, coy, bc, active, prof, R)
#define LT_T(X, Y) \
    if (nu == 1) LT_K(1, X, Y); else if (nu == 2) LT_K(2, X, Y); else LT_K(3, X, Y)
    LT_TILE_SWITCH(tile, LT_T)
#undef LT_T
#undef LT_K
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_post2d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b, const T* xin,
                  const T* ec, int cnx, int cny, int cox, int coy, T4 ghost, T* xout, int R, const int* active,
                  unsigned long long* prof, hipEvent_t ev0, hipEvent_t ev1) {
    if (nu < 1 || nu > 3) {
        set_last_error("fused smoother supports 1..3 sweeps");
        return LT_EUNSUPPORTED;
    }
#define LT_K(NU, X, Y)                                                                                 \
    LT_LAUNCH((k_post2d<T, NU, X, Y>), dim3((L.nx + X - 1) / X, (L.ny + Y - 1) / Y, R), ev0, ev1, L, tr, ti, b, \
              xin, ec, cnx, cny, cox, coy, ghost, xout, active, prof, R)
#define LT_T(X, Y) \
    if (nu == 1) LT_K(1, X, Y); else if (nu == 2) LT_K(2, X, Y); else LT_K(3, X, Y)
    LT_TILE_SWITCH(tile, LT_T)
#undef LT_T
#undef LT_K
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_post2d_refine(hipStream_t st, const LevelView<T>& L, const LevelView<double>& L64, T tr, T ti,
                         double tr64, double ti64, int nu, int tile, const T* b, const T* xin, const T* ec, int cnx,
                         int cny, int cox, int coy, T4 ghost, double* u, size_t ustride, const int* jcol,
                         const double* rho_in, double* rho_out, T* lo, double* part, int R, const int* active,
                         unsigned long long* prof, int* nparts, hipEvent_t ev0, hipEvent_t ev1) {
    if (nu < 1 || nu > 3) {
        set_last_error("fused smoother supports 1..3 sweeps");
        return LT_EUNSUPPORTED;
    }
#define LT_K(NU, X, Y)                                                                                        \
    LT_LAUNCH((k_post2d_refine<T, NU, X, Y>), dim3((L.nx + X - 1) / X, (L.ny + Y - 1) / Y, R), ev0, ev1, L, L64, \
              tr, ti, tr64, ti64, b, xin, ec, cnx, cny, cox, coy, ghost, u, ustride, jcol, rho_in, rho_out, lo,   \
              part, active, prof, R)
#define LT_T(X, Y)                                                          \
    *nparts = ((L.nx + X - 1) / X) * ((L.ny + Y - 1) / Y);                 \
    if (nu == 1) LT_K(1, X, Y); else if (nu == 2) LT_K(2, X, Y); else LT_K(3, X, Y)
    LT_TILE_SWITCH(tile, LT_T)
#undef LT_T
#undef LT_K
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_coarse_block(hipStream_t st, const CBMeta<T>& M, T tr, T ti, const T* bin, T* xout, int R,
                        const int* active) {
    size_t cells = 0;
    for (int l = 0; l < M.nl; ++l) cells += M.L[l].N;
    size_t shm = 4 * cells * sizeof(T);
    if (M.nl > kMaxCBLevels || M.L[0].N > 1024) {
        set_last_error("coarse block: too many levels or cells");
        return LT_EUNSUPPORTED;
    }
    int threads = ((M.L[0].N + 63) / 64) * 64;
    if (threads < 64) threads = 64;
    bool d3 = false;
    for (int l = 0; l < M.nl; ++l) d3 = d3 || M.L[l].nz > 1;
    if (M.nl <= 3) {
        if (d3)
            k_coarse_block<T, 3, true><<<R, threads, shm, st>>>(M, tr, ti, bin, xout, active);
        else
            k_coarse_block<T, 3, false><<<R, threads, shm, st>>>(M, tr, ti, bin, xout, active);
    } else {
        if (d3)
            k_coarse_block<T, kMaxCBLevels, true><<<R, threads, shm, st>>>(M, tr, ti, bin, xout, active);
        else
            k_coarse_block<T, kMaxCBLevels, false><<<R, threads, shm, st>>>(M, tr, ti, bin, xout, active);
    }
    LT_HIP(hipGetLastError());
    return 0;
}

template int launch_pre2d<float>(hipStream_t, const LevelView<float>&, float, float, int, int, const float*, float*,
                                 int, int, int, int, float*, int, const int*, unsigned long long*, hipEvent_t,
                                 hipEvent_t);
template int launch_pre2d<double>(hipStream_t, const LevelView<double>&, double, double, int, int, const double*,
                                  double*, int, int, int, int, double*, int, const int*, unsigned long long*,
                                  hipEvent_t, hipEvent_t);
template int launch_post2d<float>(hipStream_t, const LevelView<float>&, float, float, int, int, const float*,
                                  const float*, const float*, int, int, int, int, T4, float*, int, const int*,
                                  unsigned long long*, hipEvent_t, hipEvent_t);
template int launch_post2d<double>(hipStream_t, const LevelView<double>&, double, double, int, int, const double*,
                                   const double*, const double*, int, int, int, int, T4, double*, int, const int*,
                                   unsigned long long*, hipEvent_t, hipEvent_t);
template int launch_post2d_refine<float>(hipStream_t, const LevelView<float>&, const LevelView<double>&, float, float,
                                         double, double, int, int, const float*, const float*, const float*, int,
                                         int, int, int, T4, double*, size_t, const int*, const double*, double*,
                                         float*, double*, int, const int*, unsigned long long*, int*, hipEvent_t,
                                         hipEvent_t);
template int launch_post2d_refine<double>(hipStream_t, const LevelView<double>&, const LevelView<double>&, double,
                                          double, double, double, int, int, const double*, const double*,
                                          const double*, int, int, int, int, T4, double*, size_t, const int*,
                                          const double*, double*, double*, double*, int, const int*,
                                          unsigned long long*, int*, hipEvent_t, hipEvent_t);
template int launch_coarse_block<float>(hipStream_t, const CBMeta<float>&, float, float, const float*, float*, int,
                                        const int*);
template int launch_coarse_block<double>(hipStream_t, const CBMeta<double>&, double, double, const double*, double*,
                                         int, const int*);

}  // namespace lt
