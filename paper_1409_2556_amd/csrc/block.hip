// Block flexible GMRES for shifted systems: several right-hand sides share one block basis.
//
// Section 6 names block Krylov methods as the way to share work between the right-hand sides
// of the shifted systems.  This is the block form of Algorithm 1 (Section 3): the columns of
// each block of p right-hand sides start one basis, B = V_1 R_0; step j applies the
// preconditioner of that step to the block V_j (U_j = P(tau_j) V_j), orthogonalises
// S_j = M U_j against V_1 .. V_j (block CGS, twice) and takes the QR of the remainder by
// modified Gram-Schmidt inside the block, V_{j+1} H_{j+1, j}.  The flexible Arnoldi relation
// (K + z M) U_j = V_{j+1} ([I; 0] + Hbar_j (z I - T_j)) then reduces every shift to a block
// least-squares problem, solved by Givens rotations updated one step at a time (the matrix is
// block upper Hessenberg with p subdiagonals, since every H_{j+1, j} is upper triangular).
//
// Layout (device, FP64, complex vectors as [re plane][im plane] of N each):
//   V  [maxit + 1 slots][R][2][N]: basis index i of block b is slot i / p, column b p + i % p,
//      so a slot of every block is one contiguous batch for the preconditioner;
//   U  [maxit slots][R][2][N]; W [R][2][N] (the block being orthogonalised);
//   H  [nb][(maxit + 1) p][maxit p] complex, row-major;
//   per (block, shift): the rotated matrix Rm [maxit p columns][(maxit + 1) p rows], the
//   rotated right-hand side g [(maxit + 1) p rows][p], the rotations, the step count jd and
//   the converged flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "krylov.h"
#include "lt_internal.h"

namespace lt {
namespace {

constexpr int kBT = 256;      // threads of the vector kernels
constexpr int kBlockMax = 16;  // right-hand sides per block
constexpr int kLdsBytes = 32 * 1024;  // one (block, shift)'s new columns, or its right-hand side, in LDS

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
    return s;
}

// Dots V_{b,i}^* W_{b, c0 + c} for i in [i0, i0 + ni), c < nc (at most four), in two passes.
// First, each workgroup takes kDotE x 256 grid points of one block and kDotI of its basis vectors,
// holds the W columns there in registers and streams those vectors once: part[b][i][c][chunk] (one cross-wave reduction
// per vector for kDotE x 256 points).  Then k_bdots_fin sums the chunks into C[b][i][c0 + c] and
// adds them to Hacc[b hb + (i0 + i) hld + hcol + c] (complex).
constexpr int kDotE = 4;
constexpr int kDotI = 8;  // basis vectors per workgroup (more workgroups for short grids)
template <int NCM>
__global__ __launch_bounds__(kBT) void k_bdots_part(const double* __restrict__ V, int R, int p, int N, int i0,
                                                      int ni, const double* __restrict__ W, int c0, int nc,
                                                      double* __restrict__ part, int nchunk) {
    __shared__ double red[kBT / 64][2 * NCM];
    const int chunk = blockIdx.x, b = blockIdx.y, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t N2 = 2 * (size_t)N;
    int nn[kDotE];
    double wr[kDotE][NCM], wi[kDotE][NCM];
#pragma unroll
    for (int e = 0; e < kDotE; ++e) {
        nn[e] = (chunk * kDotE + e) * kBT + threadIdx.x;
#pragma unroll
        for (int c = 0; c < NCM; ++c) {
            wr[e][c] = wi[e][c] = 0.0;
            if (c < nc && nn[e] < N) {
                const double* w = W + ((size_t)b * p + c0 + c) * N2;
                wr[e][c] = w[nn[e]];
                wi[e][c] = w[nn[e] + N];
            }
        }
    }
    // this workgroup's basis vectors: i in [ia, ib) (blockIdx.z selects a group of kDotI)
    const int ia = blockIdx.z * kDotI, ib = min(ni, ia + kDotI);
    int sl = (i0 + ia) / p, cc = (i0 + ia) % p;  // slot and column of basis index i0 + i
    for (int i = ia; i < ib; ++i) {
        const double* q = V + ((size_t)sl * R + (size_t)b * p + cc) * N2;
        if (++cc == p) {
            cc = 0;
            ++sl;
        }
        double qr[kDotE], qi[kDotE];
#pragma unroll
        for (int e = 0; e < kDotE; ++e) {
            qr[e] = nn[e] < N ? q[nn[e]] : 0.0;
            qi[e] = nn[e] < N ? q[nn[e] + N] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < NCM; ++c) {
            if (c < nc) {
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int e = 0; e < kDotE; ++e) {
                    sr += qr[e] * wr[e][c] + qi[e] * wi[e][c];
                    si += qr[e] * wi[e][c] - qi[e] * wr[e][c];
                }
                sr = wave_sum(sr);
                si = wave_sum(si);
                if (lane == 0) {
                    red[wv][2 * c] = sr;
                    red[wv][2 * c + 1] = si;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * nc) {
            double s = 0.0;
            for (int q2 = 0; q2 < kBT / 64; ++q2) s += red[q2][threadIdx.x];
            const int c = threadIdx.x >> 1, im = threadIdx.x & 1;
            part[2 * ((((size_t)b * ni + i) * kBlockMax + c) * nchunk + chunk) + im] = s;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBT) void k_bdots_fin(const double* __restrict__ part, int ni, int nchunk, int p,
                                                     int i0, int c0, int nc, double* __restrict__ C, int ci,
                                                     double* __restrict__ Hacc, size_t hb, int hld, int hcol) {
    __shared__ double red[kBT / 64];
    const int i = blockIdx.x, b = blockIdx.y;
    for (int c = 0; c < nc; ++c) {
        const double* pp = part + 2 * ((((size_t)b * ni + i) * kBlockMax + c) * nchunk);
        double sr = 0.0, si = 0.0;
        for (int k = threadIdx.x; k < nchunk; k += kBT) {
            sr += pp[2 * k];
            si += pp[2 * k + 1];
        }
        sr = block_sum(sr, red);
        si = block_sum(si, red);
        if (threadIdx.x == 0) {
            double* o = C + 2 * (((size_t)b * ci + i) * p + c0 + c);
            o[0] = sr;
            o[1] = si;
            double* hh = Hacc + 2 * ((size_t)b * hb + (size_t)(i0 + i) * hld + hcol + c);
            hh[0] += sr;
            hh[1] += si;
        }
    }
}

// W_{b, c0 + c} -= sum_{i < ni} V_{b, i0 + i} C[b][i][c0 + c]; the coefficients of the block
// and the offsets of its basis vectors are staged in LDS (dynamic: ni nc complex, then ni
// offsets), so the loop over the vectors unrolls and keeps several loads in flight
// NCM: the column count rounded up to 1, 2 or 4 (the accumulators held in registers)
template <int NCM>
__global__ __launch_bounds__(kBT) void k_bupdate(const double* __restrict__ V, int R, int p, int N, int i0, int ni,
                                                   double* __restrict__ W, int c0, int nc,
                                                   const double* __restrict__ C, int ci) {
    extern __shared__ double cl[];  // [ni][nc][2], then [ni] offsets
    size_t* off = reinterpret_cast<size_t*>(cl + 2 * (size_t)ni * nc);
    const int b = blockIdx.y;
    const size_t N2 = 2 * (size_t)N;
    for (int e = threadIdx.x; e < ni * nc; e += kBT) {
        const int i = e / nc, c = e % nc;
        const double* s = C + 2 * (((size_t)b * ci + i) * p + c0 + c);
        cl[2 * e] = s[0];
        cl[2 * e + 1] = s[1];
    }
    for (int i = threadIdx.x; i < ni; i += kBT)
        off[i] = ((size_t)((i0 + i) / p) * R + (size_t)b * p + (i0 + i) % p) * N2;
    __syncthreads();
    const int n = blockIdx.x * kBT + threadIdx.x;
    if (n >= N) return;
    double ar[NCM], ai[NCM];
#pragma unroll
    for (int c = 0; c < NCM; ++c) {
        ar[c] = ai[c] = 0.0;
        if (c < nc) {
            const double* w = W + ((size_t)b * p + c0 + c) * N2;
            ar[c] = w[n];
            ai[c] = w[n + N];
        }
    }
#pragma unroll 4
    for (int i = 0; i < ni; ++i) {
        const double* q = V + off[i];
        const double qr = q[n], qi = q[n + N];
        const double* cc = cl + 2 * i * nc;
#pragma unroll
        for (int c = 0; c < NCM; ++c) {
            if (c < nc) {
                const double hr = cc[2 * c], hi = cc[2 * c + 1];
                ar[c] -= qr * hr - qi * hi;
                ai[c] -= qr * hi + qi * hr;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NCM; ++c) {
        if (c < nc) {
            double* w = W + ((size_t)b * p + c0 + c) * N2;
            w[n] = ar[c];
            w[n + N] = ai[c];
        }
    }
}

// Column c of every block scaled into Vout by 1 / nrm[b] (nrm from launch_norms), or zeroed
// when the remainder has lost rank: nrm <= 1e-14 of the block's largest column norm before
// orthogonalisation (scale); Hd[b hb + hrow hld + hcol] = nrm.
__global__ __launch_bounds__(kBT) void k_bscale(const double* __restrict__ W, int R, int p, int N, int c,
                                                  double* __restrict__ Vout, const double* __restrict__ nrm,
                                                  const double* __restrict__ scale, double* __restrict__ Hd, size_t hb,
                                                  int hld, int hrow, int hcol, int* __restrict__ brk) {
    const int b = blockIdx.y;
    const size_t N2 = 2 * (size_t)N, n = (size_t)blockIdx.x * kBT + threadIdx.x;
    const double nr = nrm[b];
    double sc = 0.0;
    for (int q = 0; q < p; ++q) sc = fmax(sc, scale[b * p + q]);
    const bool bad = !(nr > 1e-14 * sc);
    if (n < N2) Vout[((size_t)b * p + c) * N2 + n] = bad ? 0.0 : W[((size_t)b * p + c) * N2 + n] / nr;
    if (n == 0) {
        double* hh = Hd + 2 * ((size_t)b * hb + (size_t)hrow * hld + hcol);
        hh[0] = nr;
        hh[1] = 0.0;
        if (bad) brk[b] = 1;
    }
}

// W_r = m * U_r (the diagonal mass)
__global__ __launch_bounds__(kBT) void k_bmass(const double* __restrict__ U, const double* __restrict__ m, int N,
                                                 double* __restrict__ W) {
    const int n = blockIdx.x * kBT + threadIdx.x, r = blockIdx.y;
    if (n >= N) return;
    const size_t o = (size_t)r * 2 * N;
    const double mm = m[n];
    W[o + n] = mm * U[o + n];
    W[o + N + n] = mm * U[o + N + n];
}

// g of every (block, shift) = [R_0; 0] before the first step
__global__ void k_binit_g(const double* __restrict__ R0, int p, int nk, int grows, double* __restrict__ g) {
    const int id = blockIdx.x, b = id / nk;
    double* gg = g + 2 * (size_t)id * grows * p;
    for (int e = threadIdx.x; e < grows * p; e += blockDim.x) {
        const int row = e / p, c = e % p;
        const double* s = R0 + 2 * (((size_t)b * p + row) * p + c);
        gg[2 * e] = row < p ? s[0] : 0.0;
        gg[2 * e + 1] = row < p ? s[1] : 0.0;
    }
}

struct Rot {
    double c, sr, si;  // G = [c s; -conj(s) c], c real
};

__device__ inline void rot_apply(const Rot& G, double* a, double* b) {
    // (a, b) <- (c a + s b, -conj(s) a + c b)
    const double ar = a[0], ai = a[1], br = b[0], bi = b[1];
    a[0] = G.c * ar + (G.sr * br - G.si * bi);
    a[1] = G.c * ai + (G.sr * bi + G.si * br);
    b[0] = G.c * br - (G.sr * ar + G.si * ai);
    b[1] = G.c * bi - (G.sr * ai - G.si * ar);
}

// One step j of the block least squares of every (block, shift) still running: one wave per
// (block, shift), lane c < p owns new column (j - 1) p + c of ([I; 0] + Hbar (z_k - tau_j))
// and column c of g (both in LDS).  Old rotations are applied to the new columns, then each
// new column's p rotations (zeroing its rows col + p .. col + 1, bottom up) are made by its
// lane and applied by the lanes of the later new columns and of g.  Residual of column c:
// the norm of g's rows j p .. (j + 1) p - 1.
__global__ __launch_bounds__(64) void k_bls(int j, int p, int nk, int mx, const double* __restrict__ H, size_t hb,
                                              int hld, const double* __restrict__ zs, double taur, double taui,
                                              const double* __restrict__ wk, const double* __restrict__ bnorm,
                                              double tol, const int* __restrict__ brk, double* __restrict__ Rm,
                                              double* __restrict__ g, double* __restrict__ rot, int* __restrict__ jd,
                                              double* __restrict__ res, int* __restrict__ conv) {
    extern __shared__ double lds[];
    const int id = blockIdx.x, b = id / nk, k = id % nk, lane = threadIdx.x;
    if (conv[id]) return;
    const int grows = (mx + 1) * p, rows = (j + 1) * p, col0 = (j - 1) * p;
    double* cb = lds;                              // [p][grows][2]
    double* gb = lds + 2 * (size_t)p * grows;      // [p][grows][2]
    const double dzr = zs[2 * k] - taur, dzi = zs[2 * k + 1] - taui;
    for (int e = lane; e < p * rows; e += 64) {
        const int c = e / rows, row = e % rows, col = col0 + c;
        const double* hh = H + 2 * ((size_t)b * hb + (size_t)row * hld + col);
        double* o = cb + 2 * ((size_t)c * grows + row);
        o[0] = hh[0] * dzr - hh[1] * dzi + (row == col ? 1.0 : 0.0);
        o[1] = hh[0] * dzi + hh[1] * dzr;
        const double* gs = g + 2 * (((size_t)id * grows + row) * p + c);
        double* go = gb + 2 * ((size_t)c * grows + row);
        go[0] = gs[0];
        go[1] = gs[1];
    }
    __syncthreads();
    Rot* rt = reinterpret_cast<Rot*>(rot) + (size_t)id * mx * p * p;
    if (lane < p) {
        double* mycol = cb + 2 * (size_t)lane * grows;
        for (int cp = 0; cp < col0; ++cp)
            for (int q = 0; q < p; ++q) {
                const int kk = p - q;  // rows (cp + kk - 1, cp + kk)
                rot_apply(rt[(size_t)cp * p + q], mycol + 2 * (cp + kk - 1), mycol + 2 * (cp + kk));
            }
    }
    __syncthreads();
    for (int c = 0; c < p; ++c) {
        const int col = col0 + c;
        if (lane == c) {
            double* mycol = cb + 2 * (size_t)c * grows;
            for (int q = 0; q < p; ++q) {
                const int kk = p - q;
                double* a = mycol + 2 * (col + kk - 1);
                double* bb = mycol + 2 * (col + kk);
                const double na = hypot(a[0], a[1]), nb = hypot(bb[0], bb[1]);
                const double r = hypot(na, nb);
                Rot G;
                if (nb == 0.0) {
                    G = {1.0, 0.0, 0.0};
                } else if (na == 0.0) {
                    G = {0.0, bb[0] / nb, -bb[1] / nb};
                } else {
                    // s = (a / |a|) conj(b) / r
                    const double ur = a[0] / na, ui = a[1] / na;
                    G = {na / r, (ur * bb[0] + ui * bb[1]) / r, (ui * bb[0] - ur * bb[1]) / r};
                }
                rot_apply(G, a, bb);
                bb[0] = bb[1] = 0.0;
                rt[(size_t)col * p + q] = G;
            }
        }
        __syncthreads();
        if (lane < p) {
            for (int q = 0; q < p; ++q) {
                const int kk = p - q;
                const Rot G = rt[(size_t)col * p + q];
                if (lane > c) {
                    double* oc = cb + 2 * (size_t)lane * grows;
                    rot_apply(G, oc + 2 * (col + kk - 1), oc + 2 * (col + kk));
                }
                double* og = gb + 2 * (size_t)lane * grows;
                rot_apply(G, og + 2 * (col + kk - 1), og + 2 * (col + kk));
            }
        }
        __syncthreads();
    }
    // write back: the new columns' upper parts, g
    for (int e = lane; e < p * rows; e += 64) {
        const int c = e / rows, row = e % rows, col = col0 + c;
        const double* s = cb + 2 * ((size_t)c * grows + row);
        if (row <= col) {
            double* o = Rm + 2 * (((size_t)id * mx * p + col) * grows + row);
            o[0] = s[0];
            o[1] = s[1];
        }
        const double* gs = gb + 2 * ((size_t)c * grows + row);
        double* go = g + 2 * (((size_t)id * grows + row) * p + c);
        go[0] = gs[0];
        go[1] = gs[1];
    }
    double wr = 0.0;
    if (lane < p) {
        double s = 0.0;
        for (int row = j * p; row < rows; ++row) {
            const double* gs = gb + 2 * ((size_t)lane * grows + row);
            s += gs[0] * gs[0] + gs[1] * gs[1];
        }
        const double rr = sqrt(s) / bnorm[b * p + lane];
        res[(size_t)id * p + lane] = rr;
        wr = wk[k] * rr;
    }
    for (int o = 32; o > 0; o >>= 1) wr = fmax(wr, __shfl_xor(wr, o, 64));
    if (lane == 0) {
        jd[id] = j;
        if (!(wr > tol) || brk[b]) conv[id] = 1;
    }
}

// Y = Rm^{-1} g over the first jd p rows of every (block, shift); one workgroup each,
// column-oriented back substitution on g in LDS.
__global__ __launch_bounds__(kBT) void k_bsolve(int p, int nk, int mx, const double* __restrict__ Rm,
                                                  const double* __restrict__ g, const int* __restrict__ jd,
                                                  double* __restrict__ Y) {
    extern __shared__ double lds[];
    const int id = blockIdx.x;
    const int grows = (mx + 1) * p, n = jd[id] * p;
    double* gb = lds;  // [n][p][2]
    for (int e = threadIdx.x; e < n * p; e += kBT) {
        gb[2 * e] = g[2 * ((size_t)id * grows * p + e)];
        gb[2 * e + 1] = g[2 * ((size_t)id * grows * p + e) + 1];
    }
    __syncthreads();
    double* yo = Y + 2 * (size_t)id * mx * p * p;
    for (int i = n - 1; i >= 0; --i) {
        const double* ci = Rm + 2 * ((size_t)id * mx * p + i) * grows;  // column i
        const double dr = ci[2 * i], di = ci[2 * i + 1];
        const double dd = dr * dr + di * di;
        // y_i = g_i / R_ii for every column (each thread of the first p computes its own copy)
        double yr[kBlockMax], yi[kBlockMax];
#pragma unroll
        for (int c = 0; c < kBlockMax; ++c) {
            yr[c] = yi[c] = 0.0;
            if (c < p) {
                const double gr = gb[2 * (i * p + c)], gi = gb[2 * (i * p + c) + 1];
                yr[c] = (gr * dr + gi * di) / dd;
                yi[c] = (gi * dr - gr * di) / dd;
            }
        }
        __syncthreads();
        if (threadIdx.x < p) {
            yo[2 * (i * p + threadIdx.x)] = yr[threadIdx.x];
            yo[2 * (i * p + threadIdx.x) + 1] = yi[threadIdx.x];
        }
        for (int e = threadIdx.x; e < i * p; e += kBT) {
            const int l = e / p, c = e % p;
            const double rr = ci[2 * l], ri = ci[2 * l + 1];
            double ycr = 0.0, yci = 0.0;
#pragma unroll
            for (int q = 0; q < kBlockMax; ++q)
                if (q == c) {
                    ycr = yr[q];
                    yci = yi[q];
                }
            gb[2 * e] -= rr * ycr - ri * yci;
            gb[2 * e + 1] -= rr * yci + ri * ycr;
        }
        __syncthreads();
    }
}

// x[k][r] = sum_{i < jd p} U_{b, i} Y[b, k][i][c] (r = b p + c), kFormK shifts per thread, so
// that each basis vector is read once for every kFormK shifts (each shift has its own steps)
constexpr int kFormK = 8;
__global__ __launch_bounds__(kBT) void k_bform_x(const double* __restrict__ U, int R, int p, int N, int nk, int mx,
                                                   const int* __restrict__ jd, const double* __restrict__ Y,
                                                   double* __restrict__ x) {
    const int n = blockIdx.x * kBT + threadIdx.x, r = blockIdx.y, k0 = blockIdx.z * kFormK;
    if (n >= N) return;
    const int b = r / p, c = r % p;
    const size_t N2 = 2 * (size_t)N;
    int ni[kFormK];
    int nmax = 0;
#pragma unroll
    for (int q = 0; q < kFormK; ++q) {
        ni[q] = k0 + q < nk ? jd[b * nk + k0 + q] * p : 0;
        nmax = max(nmax, ni[q]);
    }
    double ar[kFormK], ai[kFormK];
#pragma unroll
    for (int q = 0; q < kFormK; ++q) ar[q] = ai[q] = 0.0;
    for (int i = 0, sl = 0, col = 0; i < nmax; ++i) {
        const double* u = U + ((size_t)sl * R + (size_t)b * p + col) * N2;
        if (++col == p) {
            col = 0;
            ++sl;
        }
        const double ur = u[n], ui = u[n + N];
#pragma unroll
        for (int q = 0; q < kFormK; ++q) {
            if (i < ni[q]) {
                const double* y = Y + 2 * ((size_t)(b * nk + k0 + q) * mx * p * p + (size_t)i * p + c);
                ar[q] += ur * y[0] - ui * y[1];
                ai[q] += ur * y[1] + ui * y[0];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kFormK; ++q) {
        if (k0 + q < nk) {
            double* o = x + ((size_t)(k0 + q) * R + r) * N2;
            o[n] = ar[q];
            o[n + N] = ai[q];
        }
    }
}

// Y = B - Y over R vectors (the residual of the operator's output Y)
__global__ __launch_bounds__(kBT) void k_bdiff(const double* __restrict__ B, double* __restrict__ Yv, size_t n2) {
    const size_t e = (size_t)blockIdx.x * kBT + threadIdx.x;
    if (e < n2) Yv[e] = B[e] - Yv[e];
}

unsigned nblk(size_t n) { return (unsigned)((n + kBT - 1) / kBT); }

// W_{b, c0 + c} -= sum_i V_{b, i0 + i} C[b][i][c0 + c] (dynamic LDS: coefficients, then offsets).
// Wider blocks go in groups of four columns: eight or sixteen accumulators per thread spill.
int launch_bupdate(hipStream_t st, const double* V, int R, int p, int nb, int N, int i0, int ni, double* W, int c0,
                   int nc, const double* C, int ci) {
    const dim3 g(nblk(N), nb);
    for (int g0 = 0; g0 < nc; g0 += 4) {
        const int m = std::min(4, nc - g0);
        const size_t lds = (2 * sizeof(double) * m + sizeof(size_t)) * (size_t)ni;
        if (m == 1)
            k_bupdate<1><<<g, kBT, lds, st>>>(V, R, p, N, i0, ni, W, c0 + g0, m, C, ci);
        else if (m == 2)
            k_bupdate<2><<<g, kBT, lds, st>>>(V, R, p, N, i0, ni, W, c0 + g0, m, C, ci);
        else
            k_bupdate<4><<<g, kBT, lds, st>>>(V, R, p, N, i0, ni, W, c0 + g0, m, C, ci);
        LT_HIP(hipGetLastError());
    }
    return 0;
}

// column c of every block normalised into the slot at Vout (norms by launch_norms over the
// columns b p + c, then scaled over the whole grid)
int launch_bnormalize(hipStream_t st, const double* W, int R, int p, int nb, int N, int c, double* Vout,
                      const double* scale, double* Hd, size_t hb, int hld, int hrow, int hcol, int* brk,
                      double* npart, double* nrm) {
    const size_t N2 = 2 * (size_t)N;
    LT_TRY(launch_norms(st, N, nb, (size_t)p * N2, W + (size_t)c * N2, npart, nrm, nullptr));
    k_bscale<<<dim3(nblk(N2), nb), kBT, 0, st>>>(W, R, p, N, c, Vout, nrm, scale, Hd, hb, hld, hrow, hcol, brk);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_bdots(hipStream_t st, const double* V, int R, int p, int nb, int N, int i0, int ni, const double* W,
                 int c0, int nc, double* part, double* C, int ci, double* Hacc, size_t hb, int hld, int hcol) {
    const int nchunk = (int)((N + kDotE * kBT - 1) / (kDotE * kBT));
    for (int g0 = 0; g0 < nc; g0 += 4) {  // four columns at a time: their W values stay in registers
        const int m = std::min(4, nc - g0);
        const dim3 g(nchunk, nb, (ni + kDotI - 1) / kDotI);
        if (m == 1)
            k_bdots_part<1><<<g, kBT, 0, st>>>(V, R, p, N, i0, ni, W, c0 + g0, m, part, nchunk);
        else if (m == 2)
            k_bdots_part<2><<<g, kBT, 0, st>>>(V, R, p, N, i0, ni, W, c0 + g0, m, part, nchunk);
        else
            k_bdots_part<4><<<g, kBT, 0, st>>>(V, R, p, N, i0, ni, W, c0 + g0, m, part, nchunk);
        LT_HIP(hipGetLastError());
        k_bdots_fin<<<dim3(ni, nb), kBT, 0, st>>>(part, ni, nchunk, p, i0, c0 + g0, m, C, ci, Hacc, hb, hld,
                                                  hcol + g0);
        LT_HIP(hipGetLastError());
    }
    return 0;
}

}  // namespace
}  // namespace lt

using namespace lt;

extern "C" {

int lt_shifted_solve_block(lt_handle* h, int nshift, const double* shifts, const double* weights, int ntau,
                           const double* taus, int nvec, int block, const double* b, const lt_opts* opts, double* x,
                           lt_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!h || nshift < 1 || !shifts || ntau < 1 || !taus || nvec < 1 || !b || !x) {
        set_last_error("lt_shifted_solve_block: bad argument");
        return LT_EINVAL;
    }
    if (block < 1 || block > kBlockMax || nvec % block || nvec > kMaxRhs || nshift > 1024) {
        set_last_error("lt_shifted_solve_block: block must be 1..16 and divide nvec (at most 1000); at most 1024 shifts");
        return LT_EINVAL;
    }
    lt_opts o;
    if (opts) {
        o = *opts;
    } else {
        lt_opts_default(&o);
    }
    if (!(o.tol > 0.0) || o.maxit < 1 || (o.precond != LT_PRECOND_GMG && o.precond != LT_PRECOND_EXACT) ||
        (o.precision != LT_PREC_FP64 && o.precision != LT_PREC_MIXED)) {
        set_last_error("lt_shifted_solve_block: tol > 0, maxit >= 1, precond GMG or EXACT, precision FP64 or MIXED");
        return LT_EINVAL;
    }
    for (int k = 0; k < nshift; ++k) {
        if (!std::isfinite(shifts[2 * k]) || !std::isfinite(shifts[2 * k + 1])) {
            set_last_error("lt_shifted_solve_block: shifts must be finite");
            return LT_EINVAL;
        }
        if (weights && !(weights[k] >= 0.0)) {
            set_last_error("lt_shifted_solve_block: weights must be non-negative");
            return LT_EINVAL;
        }
    }
    for (int t = 0; t < ntau; ++t)
        if (!std::isfinite(taus[2 * t]) || !std::isfinite(taus[2 * t + 1]) ||
            (o.precond == LT_PRECOND_GMG && taus[2 * t] < 0.0)) {
            set_last_error("lt_shifted_solve_block: taus must be finite, with Re(tau) >= 0 for multigrid");
            return LT_EINVAL;
        }
    const int p = block, R = nvec, nb = R / p, nk = nshift, N = h->N;
    const size_t N2 = 2 * (size_t)N;
    {
        const uintptr_t pb = (uintptr_t)b, px = (uintptr_t)x;
        const size_t bb = (size_t)R * N2 * sizeof(double), xb = (size_t)nk * bb;
        if (pb < px + xb && px < pb + bb) {
            set_last_error("lt_shifted_solve_block: x overlaps b");
            return LT_EINVAL;
        }
    }
    // the least squares keeps one (block, shift)'s rotated columns and right-hand side in LDS
    const int mx = std::min(o.maxit, kLdsBytes / (16 * p * p) - 1);
    if (mx < 1) {
        set_last_error("lt_shifted_solve_block: block too wide");
        return LT_EINVAL;
    }
    const int grows = (mx + 1) * p, hld = mx * p;
    const size_t hb = (size_t)grows * hld;
    hipStream_t st = h->stream;
    int rc = 0;
    double* V = wsp<double>(h, "bk_V", (size_t)(mx + 1) * R * N2, &rc);
    double* U = wsp<double>(h, "bk_U", (size_t)mx * R * N2, &rc);
    double* W = wsp<double>(h, "bk_W", (size_t)R * N2, &rc);
    double* C = wsp<double>(h, "bk_C", 2 * (size_t)nb * grows * p, &rc);
    double* H = wsp<double>(h, "bk_H", 2 * (size_t)nb * hb, &rc);
    double* R0 = wsp<double>(h, "bk_R0", 2 * (size_t)nb * p * p, &rc);
    double* Rm = wsp<double>(h, "bk_Rm", 2 * (size_t)nb * nk * hld * grows, &rc);
    double* g = wsp<double>(h, "bk_g", 2 * (size_t)nb * nk * grows * p, &rc);
    double* rot = wsp<double>(h, "bk_rot", 3 * (size_t)nb * nk * hld * p, &rc);
    double* Y = wsp<double>(h, "bk_Y", 2 * (size_t)nb * nk * hld * p, &rc);
    double* res = wsp<double>(h, "bk_res", (size_t)nb * nk * p, &rc);
    double* dev = wsp<double>(h, "bk_small", 2 * (size_t)nk + nk + 2 * (size_t)R + (size_t)nk * R + nb, &rc);
    int* ints = wsp<int>(h, "bk_ints", 2 * (size_t)nb * nk + nb, &rc);
    const int nbr = reduce_blocks(N, R);
    double* part = wsp<double>(h, "bk_part", (size_t)R * nbr, &rc);
    double* rho = wsp<double>(h, "bk_rho", (size_t)R * N2, &rc);
    double* ecorr = wsp<double>(h, "bk_e", (size_t)R * N2, &rc);
    const bool mixed = o.precond == LT_PRECOND_GMG && o.precision == LT_PREC_MIXED;
    double* lo = h->cp3d && !mixed ? wsp<double>(h, "bk_lo", (size_t)R * N2, &rc) : nullptr;
    float* lo32 = mixed ? wsp<float>(h, "bk_lo32", (size_t)R * N2, &rc) : nullptr;
    float* e32 = mixed ? wsp<float>(h, "bk_e32", (size_t)R * N2, &rc) : nullptr;
    double* dpart = wsp<double>(h, "bk_dpart", 2 * (size_t)nb * grows * kBlockMax * nblk(N), &rc);
    if (!V || !U || !W || !C || !H || !R0 || !Rm || !g || !rot || !Y || !res || !dev || !ints || !part || !rho ||
        !ecorr || (h->cp3d && !mixed && !lo) || (mixed && (!lo32 || !e32)) || !dpart)
        return rc ? rc : LT_ENOMEM;
    double* zs = dev;
    double* wk = zs + 2 * nk;
    double* bnorm = wk + nk;
    double* cnorm = bnorm + R;
    double* tres = cnorm + R;
    double* bcn = tres + (size_t)nk * R;  // [nb] norms of one column per block
    int* jd = ints;
    int* conv = jd + nb * nk;
    int* brk = conv + nb * nk;
    std::vector<double> hz(2 * (size_t)nk), hw(nk, 1.0);
    for (int k = 0; k < nk; ++k) {
        hz[2 * k] = shifts[2 * k];
        hz[2 * k + 1] = shifts[2 * k + 1];
        if (weights) hw[k] = weights[k];
    }
    LT_HIP(hipMemcpyAsync(zs, hz.data(), hz.size() * sizeof(double), hipMemcpyHostToDevice, st));
    LT_HIP(hipMemcpyAsync(wk, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice, st));
    LT_HIP(hipMemsetAsync(H, 0, 2 * (size_t)nb * hb * sizeof(double), st));
    LT_HIP(hipMemsetAsync(R0, 0, 2 * (size_t)nb * p * p * sizeof(double), st));
    LT_HIP(hipMemsetAsync(ints, 0, (2 * (size_t)nb * nk + nb) * sizeof(int), st));
    LT_TRY(launch_norms(st, N, R, N2, b, part, bnorm, nullptr));
    LT_HIP(hipMemcpyAsync(W, b, (size_t)R * N2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    {
        std::vector<double> hb0(R);
        LT_HIP(hipMemcpyAsync(hb0.data(), bnorm, R * sizeof(double), hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < R; ++r)
            if (!(hb0[r] > 0.0) || !std::isfinite(hb0[r])) {
                set_last_error("lt_shifted_solve_block: every right-hand side must be nonzero and finite");
                return LT_EINVAL;
            }
    }
    // B = V_1 R_0 by modified Gram-Schmidt inside each block (column c against columns < c,
    // twice): R_0[b][row][c], rows and columns 0 .. p - 1
    for (int c = 0; c < p; ++c) {
        for (int pass = 0; c > 0 && pass < 2; ++pass) {
            LT_TRY(launch_bdots(st, V, R, p, nb, N, 0, c, W, c, 1, dpart, C, grows, R0, (size_t)p * p, p, c));
            LT_TRY(launch_bupdate(st, V, R, p, nb, N, 0, c, W, c, 1, C, grows));
        }
        LT_TRY(launch_bnormalize(st, W, R, p, nb, N, c, V, bnorm, R0, (size_t)p * p, p, c, c, brk, part, bcn));
    }
    k_binit_g<<<nb * nk, kBT, 0, st>>>(R0, p, nk, grows, g);
    LT_HIP(hipGetLastError());
    const size_t ls_lds = 2 * 2 * sizeof(double) * (size_t)p * grows;
    std::vector<int> hconv((size_t)nb * nk);
    int steps = 0, vcycles = 0, factorizations = 0;
    double factor_ms = 0.0;
    bool done = false;
    for (int j = 1; j <= mx && !done; ++j) {
        steps = j;
        const double* tt = taus + 2 * ((j - 1) % ntau);
        const cdouble tau(tt[0], tt[1]);
        double* Vj = V + (size_t)(j - 1) * R * N2;
        double* Uj = U + (size_t)(j - 1) * R * N2;
        // U_j = P(tau_j) V_j for every column of every block
        if (o.precond == LT_PRECOND_EXACT) {
            const int f0 = h->exact_factorizations;
            const double m0 = h->exact_factor_ms;
            const ExactFactor* F = exact_factor(h, tau, &rc);
            if (!F) return rc;
            factorizations += h->exact_factorizations - f0;
            factor_ms += h->exact_factor_ms - m0;
            LT_TRY(exact_apply(h, F, R, Vj, N2, Uj, N2));
        } else {
            // V-cycle iteration to tol / 100 (the true residual gathers these inner residuals
            // through the combination coefficients y, whose sum is of order ten here): FP64
            // cycles, or FP32 cycles on an FP32 copy of the FP64 residual (opts.precision MIXED;
            // colour-planar on 3D grids), each correction added and the residual updated in FP64
            const LevelView<double> L0 = h->levels[0].v64();
            LT_HIP(hipMemcpyAsync(rho, Vj, (size_t)R * N2 * sizeof(double), hipMemcpyDeviceToDevice, st));
            if (lo) LT_TRY(convert_vectors_cp<double, double>(st, Vj, lo, R, N, h->grid.n[0], h->grid.n[1], 0));
            if (mixed)
                LT_TRY(convert_vectors_cp<double, float>(st, Vj, lo32, R, N, h->cp3d ? h->grid.n[0] : 0,
                                                          h->grid.n[1], 0));
            LT_HIP(hipMemsetAsync(Uj, 0, (size_t)R * N2 * sizeof(double), st));
            std::vector<double> hn(R);
            const int maxc = std::max(o.inner_max, 1) * 8;
            bool ok = false;
            for (int cyc = 0; cyc < maxc && !ok; ++cyc) {
                if (mixed) {
                    LT_TRY(mg_vcycle<float>(h, tau, o.nu1, o.nu2, R, nullptr, e32, lo32));
                    LT_TRY(launch_inner_update<float>(st, L0, tau, R, e32, Uj, N2, nullptr, rho, lo32, part, nullptr,
                                                      h->cp3d ? 1 : 0));
                } else {
                    LT_TRY(mg_vcycle<double>(h, tau, o.nu1, o.nu2, R, nullptr, ecorr, lo ? lo : rho));
                    LT_TRY(launch_inner_update<double>(st, L0, tau, R, ecorr, Uj, N2, nullptr, rho, lo, part,
                                                       nullptr, lo ? 1 : 0));
                }
                LT_TRY(launch_norms(st, N, R, N2, rho, part, cnorm, nullptr));
                LT_HIP(hipMemcpyAsync(hn.data(), cnorm, R * sizeof(double), hipMemcpyDeviceToHost, st));
                LT_HIP(hipStreamSynchronize(st));
                vcycles += R;
                ok = true;
                for (int r = 0; r < R; ++r) ok = ok && hn[r] <= 0.01 * o.tol;  // ||v|| = 1
            }
        }
        // S_j = M U_j, orthogonalised against V_1 .. V_j (block CGS, twice)
        k_bmass<<<dim3(nblk(N), R), kBT, 0, st>>>(Uj, h->levels[0].v64().m, N, W);
        LT_HIP(hipGetLastError());
        LT_TRY(launch_norms(st, N, R, N2, W, part, cnorm, nullptr));
        for (int pass = 0; pass < 2; ++pass) {
            LT_TRY(launch_bdots(st, V, R, p, nb, N, 0, j * p, W, 0, p, dpart, C, grows, H, hb, hld, (j - 1) * p));
            LT_TRY(launch_bupdate(st, V, R, p, nb, N, 0, j * p, W, 0, p, C, grows));
        }
        // V_{j+1} H_{j+1, j}: rows j p + c of columns (j - 1) p + c
        for (int c = 0; c < p; ++c) {
            for (int pass = 0; c > 0 && pass < 2; ++pass) {
                LT_TRY(launch_bdots(st, V, R, p, nb, N, j * p, c, W, c, 1, dpart, C, grows, H, hb, hld,
                                    (j - 1) * p + c));
                LT_TRY(launch_bupdate(st, V, R, p, nb, N, j * p, c, W, c, 1, C, grows));
            }
            LT_TRY(launch_bnormalize(st, W, R, p, nb, N, c, V + (size_t)j * R * N2, cnorm, H, hb, hld, j * p + c,
                                     (j - 1) * p + c, brk, part, bcn));
        }
        k_bls<<<nb * nk, 64, ls_lds, st>>>(j, p, nk, mx, H, hb, hld, zs, tau.real(), tau.imag(), wk, bnorm, o.tol,
                                           brk, Rm, g, rot, jd, res, conv);
        LT_HIP(hipGetLastError());
        LT_HIP(hipMemcpyAsync(hconv.data(), conv, hconv.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        done = true;
        for (int v : hconv) done = done && v;
    }
    k_bsolve<<<nb * nk, kBT, 2 * sizeof(double) * (size_t)mx * p * p, st>>>(p, nk, mx, Rm, g, jd, Y);
    LT_HIP(hipGetLastError());
    k_bform_x<<<dim3(nblk(N), R, (nk + kFormK - 1) / kFormK), kBT, 0, st>>>(U, R, p, N, nk, mx, jd, Y, x);
    LT_HIP(hipGetLastError());
    // FP64 true residuals ||b - (K + z_k M) x_k|| (W holds the operator's output, then the
    // residual), divided by ||b|| below
    for (int k = 0; k < nk; ++k) {
        LT_TRY(apply_operator<double>(h, 0, cdouble(hz[2 * k], hz[2 * k + 1]), x + (size_t)k * R * N2, W, R,
                                      nullptr));
        k_bdiff<<<nblk((size_t)R * N2), kBT, 0, st>>>(b, W, (size_t)R * N2);
        LT_HIP(hipGetLastError());
        LT_TRY(launch_norms(st, N, R, N2, W, part, tres + (size_t)k * R, nullptr));
    }
    std::vector<double> htr((size_t)nk * R), hbn(R);
    std::vector<int> hjd((size_t)nb * nk);
    LT_HIP(hipMemcpyAsync(htr.data(), tres, htr.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(hbn.data(), bnorm, R * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(hjd.data(), jd, hjd.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    LT_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < nk; ++k)
        for (int r = 0; r < R; ++r) htr[(size_t)k * R + r] /= hbn[r];
    double worst = 0.0;
    for (int k = 0; k < nk; ++k)
        for (int r = 0; r < R; ++r) worst = std::max(worst, hw[k] * htr[(size_t)k * R + r]);
    if (stats) {
        stats->n_rhs = R;
        stats->n_shifts = nk;
        stats->iters_max = steps;
        stats->vcycles = vcycles;
        stats->levels = (int)h->levels.size();
        stats->true_relres_max = worst;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->factorizations = factorizations;
        stats->factor_ms = factor_ms;
        stats->resolves = 0;
        if (stats->iters_per_rhs)
            for (int r = 0; r < R; ++r) {
                int it = 0;
                for (int k = 0; k < nk; ++k) it = std::max(it, hjd[(size_t)(r / p) * nk + k]);
                stats->iters_per_rhs[r] = it;
            }
        if (stats->true_relres)
            for (int r = 0; r < R; ++r)
                for (int k = 0; k < nk; ++k) stats->true_relres[(size_t)r * nk + k] = htr[(size_t)k * R + r];
    }
    return worst <= o.tol ? LT_OK : LT_WNOTCONV;
}

}  // extern "C"
