// FP64 kernels of the flexible shifted Arnoldi method (Section 3, Algorithm
// "Flexible FOM/GMRES for shifted systems"), batched over right-hand sides.
//
// Vectors of one right-hand side are complex SoA planes [2][N]; a batch is
// [R][2][N]; the basis is Q[R][jmax+1][2][N] and the preconditioned vectors
// U[R][jmax][2][N].  Reductions are two-stage with a fixed order, so results
// are deterministic.  Every kernel takes a per-RHS mask and skips converged
// right-hand sides.
#include "krylov.h"

#include <algorithm>

#include <cmath>

namespace lt {

static constexpr int kB = 256;
static constexpr int kGroup = 8;  // basis columns reduced together

struct c64 {
    double re, im;
};
__device__ __forceinline__ c64 cm(c64 a, c64 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c64 cmc(c64 a, c64 b) {  // conj(a) * b
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__device__ __forceinline__ c64 cd(c64 a, c64 b) {
    double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// Sum of v over the block (all threads get the result in lane 0 of wave 0; returned to thread 0).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduce `n` doubles per thread across the block; result written to out[0..n) by thread 0.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* out) {
    __shared__ double sh[kB / 64][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0;
            for (int q = 0; q < kB / 64; ++q) s += sh[q][k];
            out[k] = s;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- RHS and norms
__global__ void k_scatter_points(int R, int N, const int* __restrict__ off, const int* __restrict__ cell,
                                 const double* __restrict__ wt, double* __restrict__ b) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    for (int p = off[r]; p < off[r + 1]; ++p) b[(size_t)2 * N * r + cell[p]] += wt[p];
}

// partial[r][blk] = sum |x|^2 over the block's cells of vector r (stride between vectors: vstride)
__global__ void k_norm2_partial(int N, size_t vstride, const double* __restrict__ x, double* __restrict__ part,
                                const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    const double* xr = x + vstride * r;
    const double* xi = xr + N;
    double v[1] = {0};
    for (int i = blockIdx.x * kB + threadIdx.x; i < N; i += gridDim.x * kB) v[0] += xr[i] * xr[i] + xi[i] * xi[i];
    double o[1];
    block_reduce<1>(v, o);
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = o[0];
}

// beta[r] = ||b_r||, Q0 = b / beta
__global__ void k_norm_finalize(int R, int nb, const double* __restrict__ part, double* __restrict__ out) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double s = 0;
    for (int q = 0; q < nb; ++q) s += part[(size_t)r * nb + q];
    out[r] = sqrt(s);
}

__global__ void k_scale_into(int N, size_t instride, size_t outstride, const double* __restrict__ in,
                             const double* __restrict__ nrm, double* __restrict__ out) {
    int r = blockIdx.y;
    size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
    if (i >= 2 * (size_t)N) return;
    double s = nrm[r] > 0 ? 1.0 / nrm[r] : 0.0;
    out[outstride * r + i] = in[instride * r + i] * s;
}

// ---------------------------------------------------------------- inner refinement
// u <- 0, rho <- v = Q[:, j]; lo <- (T) rho
template <typename T>
__global__ void k_inner_init(int N, size_t qstride, double* __restrict__ v, double* __restrict__ u,
                             size_t ustride, double* __restrict__ rho, T* __restrict__ lo,
                             const int* __restrict__ active, const double* __restrict__ scale, int cpnx, int cpny) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
    if (i >= 2 * (size_t)N) return;
    double x = v[qstride * r + i];
    if (scale) {
        // normalisation of the new basis vector, deferred from the Gram-Schmidt step
        x *= scale[r];
        v[qstride * r + i] = x;
    }
    u[ustride * r + i] = 0.0;
    rho[2 * (size_t)N * r + i] = x;
    if (lo) {
        // the low-precision copy in the V-cycle's order (colour-planar when cpnx > 0)
        size_t o = i;
        if (cpnx) {
            const int plane = i >= (size_t)N ? 1 : 0, c = (int)(i - (size_t)plane * N);
            const int X = c % cpnx, Y = (c / cpnx) % cpny, Z = c / (cpnx * cpny);
            o = (size_t)plane * N + (size_t)(((X + Y + Z) & 1) * (N >> 1) + (c >> 1));
        }
        lo[2 * (size_t)N * r + o] = (T)x;
    }
}

// u += e; rho -= (K + tau M) e; lo = (T) rho; partial ||rho||^2
template <typename T>
__global__ void k_inner_update(LevelView<double> L, double tr, double ti, const T* __restrict__ e,
                               double* __restrict__ u, size_t ustride, const int* __restrict__ jcol,
                               double* __restrict__ rho, T* __restrict__ lo, double* __restrict__ part,
                               const int* __restrict__ active, int cp) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const T* er = e + 2 * N * r;
    const T* ei = er + N;
    double* ur = u + ustride * r + (jcol ? 2 * N * (size_t)*jcol : 0);
    double* rr = rho + 2 * N * r;
    double v[1] = {0};
    for (int i = blockIdx.x * kB + threadIdx.x; i < L.N; i += gridDim.x * kB) {
        int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
        // positions of e (the V-cycle's output): natural, or colour-planar, where every
        // neighbour has the other colour
        const int c = (x + y + z) & 1, half = L.N >> 1;
        const int own = cp ? c * half + (i >> 1) : i;
        auto ep = [&](int j) { return cp ? (1 - c) * half + (j >> 1) : j; };
        double sre = 0, sim = 0;
        if (x + 1 < L.nx) { double t = L.Tx[i]; const int q = ep(i + 1); sre += t * (double)er[q]; sim += t * (double)ei[q]; }
        if (x > 0) { double t = L.Tx[i - 1]; const int q = ep(i - 1); sre += t * (double)er[q]; sim += t * (double)ei[q]; }
        const int sy = L.nx, sz = L.nx * L.ny;
        if (y + 1 < L.ny) { double t = L.Ty[i]; const int q = ep(i + sy); sre += t * (double)er[q]; sim += t * (double)ei[q]; }
        if (y > 0) { double t = L.Ty[i - sy]; const int q = ep(i - sy); sre += t * (double)er[q]; sim += t * (double)ei[q]; }
        if (z + 1 < L.nz) { double t = L.Tz[i]; const int q = ep(i + sz); sre += t * (double)er[q]; sim += t * (double)ei[q]; }
        if (z > 0) { double t = L.Tz[i - sz]; const int q = ep(i - sz); sre += t * (double)er[q]; sim += t * (double)ei[q]; }
        double dre = L.D[i] + tr * L.m[i], dim = ti * L.m[i];
        double xre = (double)er[own], xim = (double)ei[own];
        double are = dre * xre - dim * xim - sre;
        double aim = dre * xim + dim * xre - sim;
        ur[i] += xre;
        ur[i + N] += xim;
        double nre = rr[i] - are, nim = rr[i + N] - aim;
        rr[i] = nre;
        rr[i + N] = nim;
        if (lo) {
            lo[2 * N * r + own] = (T)nre;
            lo[2 * N * r + N + own] = (T)nim;
        }
        v[0] += nre * nre + nim * nim;
    }
    double o[1];
    block_reduce<1>(v, o);
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = o[0];
}

// The same update for the RB right-hand sides of a group (group_rhs over the list of the
// cycle that produced e): a thread loads the FP64 coefficients and neighbour positions of
// its cells once for the group.  part[r * gridDim.x + block] as above.
template <typename T, int RB>
__global__ void k_inner_update_rb(LevelView<double> L, double tr, double ti, const T* __restrict__ e,
                                  double* __restrict__ u, size_t ustride, const int* __restrict__ jcol,
                                  double* __restrict__ rho, T* __restrict__ lo, double* __restrict__ part,
                                  const int* __restrict__ list, int R, int cp) {
    int rs[RB];
    group_rhs<RB>(list, R, blockIdx.y, rs);
    if (rs[0] < 0) return;
    const size_t N = L.N;
    const size_t jo = jcol ? 2 * N * (size_t)*jcol : 0;
    const int half = L.N >> 1, sy = L.nx, sz = L.nx * L.ny;
    double v[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) v[q] = 0.0;
    for (int i = blockIdx.x * kB + threadIdx.x; i < L.N; i += gridDim.x * kB) {
        const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
        // positions of e (the cycle's output): natural, or colour-planar, where every
        // neighbour has the other colour; a missing neighbour has coupling 0 and a valid index
        const int c = (x + y + z) & 1;
        const int own = cp ? c * half + (i >> 1) : i;
        const bool hx = x + 1 < L.nx, lx = x > 0, hy = y + 1 < L.ny, ly = y > 0, hz = z + 1 < L.nz, lz = z > 0;
        const int nb[6] = {hx ? i + 1 : i, lx ? i - 1 : i, hy ? i + sy : i, ly ? i - sy : i, hz ? i + sz : i,
                           lz ? i - sz : i};
        const double tc[6] = {hx ? L.Tx[i] : 0.0, lx ? L.Tx[i - 1] : 0.0, hy ? L.Ty[i] : 0.0,
                              ly ? L.Ty[i - sy] : 0.0, hz ? L.Tz[i] : 0.0, lz ? L.Tz[i - sz] : 0.0};
        int np[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) np[a] = cp ? (1 - c) * half + (nb[a] >> 1) : nb[a];
        const double dre = L.D[i] + tr * L.m[i], dim = ti * L.m[i];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = rs[q];
            if (r < 0) continue;
            const T* er = e + 2 * N * r;
            const T* ei = er + N;
            double sre = 0, sim = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                sre += tc[a] * (double)er[np[a]];
                sim += tc[a] * (double)ei[np[a]];
            }
            const double xre = (double)er[own], xim = (double)ei[own];
            const double are = dre * xre - dim * xim - sre;
            const double aim = dre * xim + dim * xre - sim;
            double* ur = u + ustride * r + jo;
            double* rr = rho + 2 * N * r;
            ur[i] += xre;
            ur[i + N] += xim;
            const double nre = rr[i] - are, nim = rr[i + N] - aim;
            rr[i] = nre;
            rr[i + N] = nim;
            if (lo) {
                lo[2 * N * r + own] = (T)nre;
                lo[2 * N * r + N + own] = (T)nim;
            }
            v[q] += nre * nre + nim * nim;
        }
    }
    double o[RB];
    block_reduce<RB>(v, o);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (rs[q] >= 0) part[(size_t)rs[q] * gridDim.x + blockIdx.x] = o[q];
    }
}

// inner_active[r] = active[r] && ||rho_r|| > eta_r && step + 1 < inner_max; counts vcycles.
// count[0] = right-hand sides still refining; count[1] = step + 1 if any right-hand
// side was refined in this step (the number of steps this outer iteration needed).
__global__ void k_inner_finalize(int R, int nb, const double* __restrict__ part, const int* __restrict__ active,
                                 const double* __restrict__ worst, double relax_tol, double tol,
                                 int inner_max, int* __restrict__ inner_active, int* __restrict__ vcycles,
                                 int* __restrict__ count, double* __restrict__ rprev, int* __restrict__ est) {
    __shared__ int cnt, any, more;
    const int step = count[2];  // refinement steps already taken in this outer iteration
    if (threadIdx.x == 0) {
        cnt = 0;
        any = 0;
        more = 0;
    }
    __syncthreads();
    // one wavefront per right-hand side sums its partial norms
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int r = threadIdx.x >> 6; r < R; r += nw) {
        if (!inner_active[r]) continue;  // (finished right-hand sides read nothing more)
        double s = 0;
        for (int q = lane; q < nb; q += 64) s += part[(size_t)r * nb + q];
        const double wr = worst[r], prev = rprev[r];
        const int act = active[r], vc = vcycles[r];
        s = wave_sum(s);
        if (lane == 0) {
            any = 1;
            double eta = relax_tol / fmax(wr, tol);
            eta = fmin(eta, 0.5);
            vcycles[r] = vc + 1;
            const double nrm = sqrt(s);
            rprev[r] = nrm;
            const int again = (nrm > eta) && (step + 1 < inner_max) && act;
            inner_active[r] = again;
            if (again) {
                atomicAdd(&cnt, 1);
                // steps still needed at the contraction this step showed (an estimate for
                // sizing the next batch of launches; the test above decides)
                const double q = prev > 0.0 ? nrm / prev : 1.0;
                int n = 1;
                if (q > 0.0 && q < 0.95) n = (int)ceil(log(eta / nrm) / log(q));
                n = max(1, min(n, inner_max - step - 1));
                atomicMax(&more, n);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        count[0] = cnt;
        if (any) count[1] = step + 1;
        count[2] = step + 1;
        est[0] = more;
    }
}

// bad[r] = active[r] && ||rho_r||^2 > 1 (the network guess made the unit residual worse);
// counts[2] = bit pattern of the worst residual ratio over the active right-hand sides
__global__ void k_net_guard(int R, int nb, const double* __restrict__ part, const int* __restrict__ active,
                            int* __restrict__ bad, int* __restrict__ counts) {
    __shared__ int nbad, nact;
    if (threadIdx.x == 0) { nbad = 0; nact = 0; }
    __syncthreads();
    __shared__ float worst;
    if (threadIdx.x == 0) worst = 0.0f;
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        int b = 0;
        if (active[r]) {
            double s = 0;
            for (int q = 0; q < nb; ++q) s += part[(size_t)r * nb + q];
            b = !(s <= 1.0);
            atomicAdd(&nact, 1);
            if (b) atomicAdd(&nbad, 1);
            // residual ratio ||rho|| / ||v|| left by the guess (v has unit norm); 1 if discarded
            const float ratio = b ? 1.0f : (float)sqrt(s);
            atomicMax((int*)&worst, __float_as_int(ratio));  // non-negative floats order like ints
        }
        bad[r] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        counts[0] += nact;
        counts[1] += nbad;
        counts[2] = __float_as_int(worst);
    }
}

// Residual-minimising multiple of the network's direction d for the residual v:
// w = (K + tau M) d (FP64), alpha = <w, v> / <w, w>.  part[r][blk] = (Re <w,v>, Im <w,v>, <w,w>).
template <typename T>
__global__ void k_net_dots(LevelView<double> L, double tr, double ti, const T* __restrict__ d,
                           const double* __restrict__ v, double* __restrict__ part, const int* __restrict__ active) {
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const size_t N = L.N;
    const T* dr = d + 2 * N * r;
    const T* di = dr + N;
    const double* vr = v + 2 * N * r;
    double acc[3] = {0, 0, 0};
    for (int i = blockIdx.x * kB + threadIdx.x; i < L.N; i += gridDim.x * kB) {
        const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
        const int sy = L.nx, sz = L.nx * L.ny;
        double sre = 0, sim = 0;
        if (x + 1 < L.nx) { double t = L.Tx[i]; sre += t * (double)dr[i + 1]; sim += t * (double)di[i + 1]; }
        if (x > 0) { double t = L.Tx[i - 1]; sre += t * (double)dr[i - 1]; sim += t * (double)di[i - 1]; }
        if (y + 1 < L.ny) { double t = L.Ty[i]; sre += t * (double)dr[i + sy]; sim += t * (double)di[i + sy]; }
        if (y > 0) { double t = L.Ty[i - sy]; sre += t * (double)dr[i - sy]; sim += t * (double)di[i - sy]; }
        if (z + 1 < L.nz) { double t = L.Tz[i]; sre += t * (double)dr[i + sz]; sim += t * (double)di[i + sz]; }
        if (z > 0) { double t = L.Tz[i - sz]; sre += t * (double)dr[i - sz]; sim += t * (double)di[i - sz]; }
        const double dre = L.D[i] + tr * L.m[i], dim = ti * L.m[i];
        const double wre = dre * (double)dr[i] - dim * (double)di[i] - sre;
        const double wim = dre * (double)di[i] + dim * (double)dr[i] - sim;
        const double xre = vr[i], xim = vr[i + N];
        acc[0] += wre * xre + wim * xim;   // Re conj(w) v
        acc[1] += wre * xim - wim * xre;   // Im conj(w) v
        acc[2] += wre * wre + wim * wim;
    }
    double o[3];
    block_reduce<3>(acc, o);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[((size_t)r * gridDim.x + blockIdx.x) * 3 + k] = o[k];
}

// d *= alpha_r (complex), alpha = <w, v> / <w, w> from the partial sums
template <typename T>
__global__ void k_net_scale(int N, int nb, const double* __restrict__ part, T* __restrict__ d,
                            const int* __restrict__ active) {
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    __shared__ double al[2];
    if (threadIdx.x == 0) {
        double a = 0, b = 0, c = 0;
        for (int q = 0; q < nb; ++q) {
            a += part[((size_t)r * nb + q) * 3];
            b += part[((size_t)r * nb + q) * 3 + 1];
            c += part[((size_t)r * nb + q) * 3 + 2];
        }
        al[0] = c > 0 ? a / c : 0.0;
        al[1] = c > 0 ? b / c : 0.0;
    }
    __syncthreads();
    const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
    if (i >= (size_t)N) return;
    T* dr = d + 2 * (size_t)N * r;
    const double xr = (double)dr[i], xi = (double)dr[i + N];
    dr[i] = (T)(al[0] * xr - al[1] * xi);
    dr[i + N] = (T)(al[0] * xi + al[1] * xr);
}

// ---------------------------------------------------------------- classical Gram-Schmidt (twice)
// Source vector: if `u` is given, s = m .* u (lumped mass, M u_j of the algorithm); else s = svec.
__device__ __forceinline__ c64 load_s(const double* __restrict__ m, const double* __restrict__ u,
                                      const double* __restrict__ s, size_t N, int i) {
    if (u) return {m[i] * u[i], m[i] * u[i + N]};
    return {s[i], s[i + N]};
}

// part[r][blk][c] = sum_i conj(Q_c(i)) s(i),  c < ncols; plus part[...][ncols] = ||s||^2 (real part)
__global__ void k_mdot(int N, int ncols, const double* __restrict__ Q, size_t qstride,
                       const double* __restrict__ m, const double* __restrict__ u, size_t ustride,
                       const double* __restrict__ s, size_t sstride, double* __restrict__ part, int pstride,
                       const int* __restrict__ active) {
    // blockIdx.z picks a group of kGroup basis columns (groups run side by side rather than
    // in turn); group 0 also accumulates ||s||^2
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const int c0 = blockIdx.z * kGroup;
    const double* Qr = Q + qstride * r;
    const double* ur = u ? u + ustride * r : nullptr;
    const double* sr = s ? s + sstride * r : nullptr;
    double* pr = part + ((size_t)r * gridDim.x + blockIdx.x) * pstride;
    const size_t NN = N;
    double v[2 * kGroup + 1];
#pragma unroll
    for (int k = 0; k < 2 * kGroup + 1; ++k) v[k] = 0;
    for (int i = blockIdx.x * kB + threadIdx.x; i < N; i += gridDim.x * kB) {
        c64 sv = load_s(m, ur, sr, NN, i);
        v[2 * kGroup] += sv.re * sv.re + sv.im * sv.im;
#pragma unroll
        for (int k = 0; k < kGroup; ++k) {
            int c = c0 + k;
            if (c < ncols) {
                const double* q = Qr + 2 * NN * c;
                c64 p = cmc({q[i], q[i + NN]}, sv);
                v[2 * k] += p.re;
                v[2 * k + 1] += p.im;
            }
        }
    }
    double o[2 * kGroup + 1];
    block_reduce<2 * kGroup + 1>(v, o);
    if (threadIdx.x == 0) {
        for (int k = 0; k < kGroup && c0 + k < ncols; ++k) {
            pr[2 * (c0 + k)] = o[2 * k];
            pr[2 * (c0 + k) + 1] = o[2 * k + 1];
        }
        if (blockIdx.z == 0) {
            pr[2 * ncols] = o[2 * kGroup];
            pr[2 * ncols + 1] = 0;
        }
    }
}

// coef[r][c] = sum over blocks of part  (c < ncols + 1: the last entry is ||s||^2)


// Hbar column j: h = h1 + h2, h_{j+1,j} = ||s||; scale for the new basis vector;
// breakdown (||s|| <= 1e-14 ||M u||) gives h_{j+1,j} = 0 and a zero vector.
__global__ void k_hcol_finalize(int R, int j, int nb, const double* __restrict__ c1, const double* __restrict__ c2,
                                int cstride, const double* __restrict__ part, double* __restrict__ H,
                                int hstride, size_t hrstride, double* __restrict__ scale,
                                const int* __restrict__ active) {
    int r = blockIdx.x;
    if (active && !active[r]) return;
    double* Hc = H + hrstride * r + (size_t)hstride * j;
    const double* a = c1 + (size_t)r * cstride;
    const double* b = c2 + (size_t)r * cstride;
    for (int c = threadIdx.x; c <= j; c += blockDim.x) {
        Hc[2 * c] = a[2 * c] + b[2 * c];
        Hc[2 * c + 1] = a[2 * c + 1] + b[2 * c + 1];
    }
    if (threadIdx.x == 0) {
        double s = 0;
        for (int q = 0; q < nb; ++q) s += part[(size_t)r * nb + q];
        double nrm = sqrt(s);
        double nrm0 = sqrt(a[2 * (j + 1)]);  // ||M u_j|| from the first pass
        bool breakdown = !(nrm > 1e-14 * nrm0);
        Hc[2 * (j + 1)] = breakdown ? 0.0 : nrm;
        Hc[2 * (j + 1) + 1] = 0.0;
        scale[r] = breakdown ? 0.0 : 1.0 / nrm;
    }
}

// out = s - sum_c Q_c coef_c (optional partial ||out||^2 into part[r][blk]), with the
// projection coefficients summed in the workgroup from the pass's partial dot products
// (one wavefront per column, lanes striding over the partials: every workgroup forms the
// same coefficients); workgroup 0 also stores them for the Hessenberg column.
// Dynamic LDS: 2 (ncols + 1) doubles.
__global__ void k_update_sum(int N, int ncols, const double* __restrict__ Q, size_t qstride,
                             const double* __restrict__ m, const double* __restrict__ u, size_t ustride,
                             const double* __restrict__ s, size_t sstride, const double* __restrict__ pin, int nbin,
                             int pstride, double* __restrict__ coef, int cstride, double* __restrict__ out,
                             size_t ostride, double* __restrict__ part, const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    extern __shared__ double cs[];
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int c = threadIdx.x >> 6; c <= ncols; c += nw) {
        double re = 0, im = 0;
        for (int q = lane; q < nbin; q += 64) {
            const double* p = pin + ((size_t)r * nbin + q) * pstride;
            re += p[2 * c];
            im += p[2 * c + 1];
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            cs[2 * c] = re;
            cs[2 * c + 1] = im;
            if (blockIdx.x == 0) {
                coef[(size_t)r * cstride + 2 * c] = re;
                coef[(size_t)r * cstride + 2 * c + 1] = im;
            }
        }
    }
    __syncthreads();
    const double* Qr = Q + qstride * r;
    const double* ur = u ? u + ustride * r : nullptr;
    const double* sr = s ? s + sstride * r : nullptr;
    double* orr = out + ostride * r;
    const size_t NN = N;
    double v[1] = {0};
    for (int i = blockIdx.x * kB + threadIdx.x; i < N; i += gridDim.x * kB) {
        c64 sv = load_s(m, ur, sr, NN, i);
        for (int c = 0; c < ncols; ++c) {
            const double* q = Qr + 2 * NN * c;
            c64 p = cm({q[i], q[i + NN]}, {cs[2 * c], cs[2 * c + 1]});
            sv.re -= p.re;
            sv.im -= p.im;
        }
        orr[i] = sv.re;
        orr[i + NN] = sv.im;
        v[0] += sv.re * sv.re + sv.im * sv.im;
    }
    if (part) {
        double o[1];
        block_reduce<1>(v, o);
        if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = o[0];
    }
}

// Start of an outer iteration: every active right-hand side refines, the step counters
// are cleared and the basis column is set (one launch instead of a copy, a fill and a store).
__global__ void k_iter_begin(int R, const int* __restrict__ active, int* __restrict__ inner_active,
                             int* __restrict__ count, int j, double* __restrict__ rprev) {
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        inner_active[r] = active[r];
        rprev[r] = 1.0;  // ||v_j||: the residual before the first step
    }
    if (threadIdx.x == 0) {
        count[1] = 0;
        count[2] = 0;
        count[3] = j;
    }
}


// ---------------------------------------------------------------- per-shift least squares
// One block per right-hand side, one thread per shift.  The Hessenberg matrix of shift z is
// Hbar(z; T) = [I; 0] + Hbar (z I - T) (eqn:shiftedarnoldimod): column j is e_j + (z - tau_j) h_j.
// Its QR factorisation is extended by one Givens rotation per column; |g_{j+1}| is the
// GMRES residual norm of the shift.
__global__ void k_ls_update(int R, int Ks, int j, double tau_re, double tau_im, const double* __restrict__ zs,
                            const double* __restrict__ omega, int rinit, double tol, int fom,
                            const double* __restrict__ H,
                            int hstride, size_t hrstride, const double* __restrict__ beta, LSState st,
                            int* __restrict__ active, int* __restrict__ mcols, double* __restrict__ worst,
                            int* __restrict__ conv_flags, const double* __restrict__ g0,
                            const double* __restrict__ bnorm) {
    int r = blockIdx.x;
    if (!active[r]) return;
    // right-hand sides from rinit on (the initial head's term) weigh their shifts by |w_k|
    const double* om = omega + (r >= rinit ? Ks : 0);
    extern __shared__ double sh[];  // h column, 2 (j + 2) doubles
    const double* Hc = H + hrstride * r + (size_t)hstride * j;
    for (int c = threadIdx.x; c < 2 * (j + 2); c += blockDim.x) sh[c] = Hc[c];
    __shared__ int notconv;
    __shared__ double wmax[kB / 64];
    if (threadIdx.x == 0) notconv = 0;
    __syncthreads();
    double myw = 0;
    for (int k = threadIdx.x; k < Ks; k += blockDim.x) {
        c64 dz = {zs[2 * k] - tau_re, zs[2 * k + 1] - tau_im};
        const size_t base = (size_t)r * Ks + k;  // pair index
        const size_t P = (size_t)R * Ks;
        // column entries col_i = delta_ij + dz * h_i, streamed through the previous rotations
        c64 cur = cm(dz, {sh[0], sh[1]});
        if (j == 0) cur.re += 1.0;
        for (int i = 0; i < j; ++i) {
            c64 nxt = cm(dz, {sh[2 * (i + 1)], sh[2 * (i + 1) + 1]});
            if (i + 1 == j) nxt.re += 1.0;
            double c = st.cs[(size_t)i * P + base];
            c64 s = {st.sn[2 * ((size_t)i * P + base)], st.sn[2 * ((size_t)i * P + base) + 1]};
            // [c s; -conj(s) c] [cur; nxt]
            c64 top = {c * cur.re + (s.re * nxt.re - s.im * nxt.im), c * cur.im + (s.re * nxt.im + s.im * nxt.re)};
            c64 bot = {-(s.re * cur.re + s.im * cur.im) + c * nxt.re, -(s.re * cur.im - s.im * cur.re) + c * nxt.im};
            size_t ri = (size_t)(j * (j + 1) / 2 + i) * P + base;
            st.Rm[2 * ri] = top.re;
            st.Rm[2 * ri + 1] = top.im;
            cur = bot;
        }
        c64 sub = cm(dz, {sh[2 * (j + 1)], sh[2 * (j + 1) + 1]});
        // new rotation zeroing `sub` into `cur`
        double na = hypot(cur.re, cur.im), nb = hypot(sub.re, sub.im);
        double c;
        c64 s, rr;
        if (nb == 0.0) {
            c = 1.0;
            s = {0.0, 0.0};
            rr = cur;
        } else if (na == 0.0) {
            c = 0.0;
            s = {sub.re / nb, -sub.im / nb};  // conj(sub)/|sub|
            rr = {nb, 0.0};
        } else {
            double nu = hypot(na, nb);
            c = na / nu;
            c64 ph = {cur.re / na, cur.im / na};                 // a / |a|
            c64 cb = {sub.re / nu, -sub.im / nu};                // conj(b) / nu
            s = cm(ph, cb);
            rr = {ph.re * nu, ph.im * nu};
        }
        size_t rj = (size_t)(j * (j + 1) / 2 + j) * P + base;
        st.Rm[2 * rj] = rr.re;
        st.Rm[2 * rj + 1] = rr.im;
        st.cs[(size_t)j * P + base] = c;
        st.sn[2 * ((size_t)j * P + base)] = s.re;
        st.sn[2 * ((size_t)j * P + base) + 1] = s.im;
        // g: g_j <- c g_j ; g_{j+1} = -conj(s) g_j
        c64 gj;
        if (j == 0) {
            gj = g0 ? c64{g0[2 * base], g0[2 * base + 1]} : c64{beta[r], 0.0};
        } else {
            gj = {st.g[2 * ((size_t)j * P + base)], st.g[2 * ((size_t)j * P + base) + 1]};
        }
        c64 gt = {c * gj.re, c * gj.im};
        c64 gn = {-(s.re * gj.re + s.im * gj.im), -(s.re * gj.im - s.im * gj.re)};
        st.g[2 * ((size_t)j * P + base)] = gt.re;
        st.g[2 * ((size_t)j * P + base) + 1] = gt.im;
        st.g[2 * ((size_t)(j + 1) * P + base)] = gn.re;
        st.g[2 * ((size_t)(j + 1) * P + base) + 1] = gn.im;
        // FOM: the square system's residual is |h_{j+1,j} y_j| = |g_{j+1}| / c (infinite when the
        // square system is singular, c = 0)
        const double bn = bnorm ? bnorm[r] : beta[r];
        double res = hypot(gn.re, gn.im) / bn;
        if (fom) res = c > 0.0 ? res / c : HUGE_VAL;
        if (fom && st.eta) {
            // eta = (z - tau_j) h_{j+1,j} y_j with y_j = g_j / cur, the square system's last
            // unknown (cur: its last diagonal entry before this step's rotation); the residual
            // of this pair is -eta v_{j+1}
            c64 e = {0.0, 0.0};
            if (na > 0.0) {
                const c64 sg = cm(sub, gj);
                const double d2 = cur.re * cur.re + cur.im * cur.im;
                e = {(sg.re * cur.re + sg.im * cur.im) / d2, (sg.im * cur.re - sg.re * cur.im) / d2};
            }
            st.eta[2 * base] = e.re;
            st.eta[2 * base + 1] = e.im;
        }
        double wres = om[k] * res;
        st.res[base] = res;
        myw = fmax(myw, wres);
        int ok = wres <= tol;
        conv_flags[base] = ok;
        if (!ok) atomicOr(&notconv, 1);
    }
    myw = fmax(myw, __shfl_xor(myw, 32, 64));
    myw = fmax(myw, __shfl_xor(myw, 16, 64));
    myw = fmax(myw, __shfl_xor(myw, 8, 64));
    myw = fmax(myw, __shfl_xor(myw, 4, 64));
    myw = fmax(myw, __shfl_xor(myw, 2, 64));
    myw = fmax(myw, __shfl_xor(myw, 1, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = myw;
    __syncthreads();
    if (threadIdx.x == 0) {
        double w = 0;
        for (int q = 0; q < (int)(blockDim.x + 63) / 64; ++q) w = fmax(w, wmax[q]);
        worst[r] = w;
        mcols[r] = j + 1;
        // a breakdown (h_{j+1,j} = 0) leaves every residual at zero: converged
        if (!notconv) active[r] = 0;
    }
}

// y = R^{-1} g for each pair, m = mcols[r] columns.  Y[r][j][k].
// FOM (fom != 0): the square system shares R and g except in the last row, whose entries
// before the last rotation are r_mm c and g_m / c, so y_m = g_m / (c^2 r_mm); the other
// rows back-substitute as before (c = 0, a singular square system, keeps the GMRES y).
__global__ void k_backsolve(int R, int Ks, const int* __restrict__ mcols, LSState st, double* __restrict__ Y,
                            int jmax, int fom) {
    int r = blockIdx.y;
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Ks) return;
    const int m = mcols[r];
    const size_t P = (size_t)R * Ks;
    const size_t base = (size_t)r * Ks + k;
    double* Yr = Y + (size_t)r * jmax * 2 * Ks;
    for (int j = m - 1; j >= 0; --j) {
        c64 acc = {st.g[2 * ((size_t)j * P + base)], st.g[2 * ((size_t)j * P + base) + 1]};
        for (int i = j + 1; i < m; ++i) {
            size_t ri = (size_t)(i * (i + 1) / 2 + j) * P + base;
            c64 Rji = {st.Rm[2 * ri], st.Rm[2 * ri + 1]};
            c64 yi = {Yr[(size_t)i * 2 * Ks + 2 * k], Yr[(size_t)i * 2 * Ks + 2 * k + 1]};
            c64 p = cm(Rji, yi);
            acc.re -= p.re;
            acc.im -= p.im;
        }
        size_t rj = (size_t)(j * (j + 1) / 2 + j) * P + base;
        c64 y = cd(acc, {st.Rm[2 * rj], st.Rm[2 * rj + 1]});
        if (fom && j == m - 1) {
            const double c = st.cs[(size_t)j * P + base];
            if (c > 0.0) {
                y.re /= c * c;
                y.im /= c * c;
            }
        }
        Yr[(size_t)j * 2 * Ks + 2 * k] = y.re;
        Yr[(size_t)j * 2 * Ks + 2 * k + 1] = y.im;
    }
}

// ---------------------------------------------------------------- receivers and the contour sum
// G[r][j][p] = sum_w w u_j(cell) for receiver p (B_r u_j).
__global__ void k_gather(int R, int N, int np, const int* __restrict__ off, const int* __restrict__ cell,
                         const double* __restrict__ wt, const double* __restrict__ U, size_t ustride, int j,
                         double* __restrict__ G, int jmax, const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const double* u = U + ustride * r + (size_t)2 * N * j;
    double re = 0, im = 0;
    for (int q = off[p]; q < off[p + 1]; ++q) {
        re += wt[q] * u[cell[q]];
        im += wt[q] * u[(size_t)N + cell[q]];
    }
    double* g = G + ((size_t)r * jmax + j) * 2 * np;
    g[2 * p] = re;
    g[2 * p + 1] = im;
}

// phi[s][p][t] = 2 Re sum_{k in t} ( wq_k sum_j G[s][j][p] Y[s][j][k]
//                                    + w_k sum_j G[r0][j][p] Y[r0][j][k] ),
// the second term (the initial head's right-hand side r0, factor 1) only when r0 >= 0;
// rows s < Rs are the wells (with Rs = 0 the one row holds the initial head's heads alone).
__device__ __forceinline__ double heads_term(int r, int p, int t, int nk, int Ks, int np, const double* __restrict__ wk,
                                             const double* __restrict__ G, const double* __restrict__ Y, int m,
                                             int jmax) {
    double acc = 0;
    for (int kk = 0; kk < nk; ++kk) {
        int k = t * nk + kk;
        c64 s = {0, 0};
        for (int j = 0; j < m; ++j) {
            const double* g = G + ((size_t)r * jmax + j) * 2 * np + 2 * p;
            const double* y = Y + ((size_t)r * jmax + j) * 2 * Ks + 2 * k;
            c64 pr = cm({g[0], g[1]}, {y[0], y[1]});
            s.re += pr.re;
            s.im += pr.im;
        }
        c64 w = {wk[2 * k], wk[2 * k + 1]};
        acc += w.re * s.re - w.im * s.im;
    }
    return acc;
}

__global__ void k_heads(int Rs, int r0, int np, int ntimes, int nk, const double* __restrict__ wq,
                        const double* __restrict__ w, const double* __restrict__ G, const double* __restrict__ Y,
                        const int* __restrict__ mcols, int jmax, double* __restrict__ phi, int accumulate) {
    const int rows = Rs > 0 ? Rs : 1;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * np * ntimes) return;
    int t = idx % ntimes, p = (idx / ntimes) % np, s = idx / (ntimes * np);
    const int Ks = ntimes * nk;
    double acc = 0;
    if (s < Rs) acc = heads_term(s, p, t, nk, Ks, np, wq, G, Y, mcols[s], jmax);
    if (r0 >= 0) acc += heads_term(r0, p, t, nk, Ks, np, w, G, Y, mcols[r0], jmax);
    phi[idx] = accumulate ? phi[idx] + 2.0 * acc : 2.0 * acc;
}

// ---------------------------------------------------------------- restarts
__global__ void k_fill_g0(int R, int Ks, const double* __restrict__ bnorm, double* __restrict__ g0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * Ks) return;
    g0[2 * i] = bnorm[i / Ks];
    g0[2 * i + 1] = 0.0;
}

// one workgroup row per right-hand side: the cycle's last basis vector becomes the next
// cycle's right-hand side, and each pair's coefficient on it is -eta
__global__ void k_restart_rhs(int R, int N, int Ks, const double* __restrict__ Q, size_t qstride,
                              const int* __restrict__ mcols, const int* __restrict__ restart,
                              const double* __restrict__ eta, double* __restrict__ b, double* __restrict__ g0) {
    const int r = blockIdx.y;
    if (!restart[r]) return;
    const size_t N2 = 2 * (size_t)N;
    const double* q = Q + qstride * r + N2 * mcols[r];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N2; i += (size_t)gridDim.x * blockDim.x)
        b[N2 * r + i] = q[i];
    if (blockIdx.x == 0)
        for (int k = threadIdx.x; k < Ks; k += blockDim.x) {
            const size_t pi = (size_t)r * Ks + k;
            g0[2 * pi] = -eta[2 * pi];
            g0[2 * pi + 1] = -eta[2 * pi + 1];
        }
}

__global__ void k_unscale_y(int R, int Ks, int jmax, const int* __restrict__ mcols, const double* __restrict__ g0,
                            const double* __restrict__ bnorm, double* __restrict__ Y) {
    const int r = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Ks) return;
    const size_t pi = (size_t)r * Ks + k;
    // sigma = g0 / bnorm; y <- y / sigma = y conj(sigma) / |sigma|^2
    const double sr = g0[2 * pi] / bnorm[r], si = g0[2 * pi + 1] / bnorm[r];
    const double d2 = sr * sr + si * si;
    double* Yr = Y + (size_t)r * jmax * 2 * Ks;
    for (int j = 0; j < mcols[r]; ++j) {
        double* y = Yr + (size_t)j * 2 * Ks + 2 * k;
        const double yr = y[0], yi = y[1];
        y[0] = d2 > 0.0 ? (yr * sr + yi * si) / d2 : 0.0;
        y[1] = d2 > 0.0 ? (yi * sr - yr * si) / d2 : 0.0;
    }
}

// b = M phi0 (real part; the imaginary plane stays as the caller cleared it)
__global__ void k_mass_rhs(int N, const double* __restrict__ m, const double* __restrict__ phi0,
                           double* __restrict__ b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) b[i] = m[i] * phi0[i];
}

// ---------------------------------------------------------------- true residual
// X[r][c][2][N] = sum_j U[r][j] Y[r][j][k0 + c], c < nc
__global__ void k_form_x(int N, int nc, int k0, int Ks, const double* __restrict__ U, size_t ustride,
                         const double* __restrict__ Y, int jmax, const int* __restrict__ mcols,
                         double* __restrict__ X) {
    constexpr int CMAX = 8;
    int r = blockIdx.y;
    int i = blockIdx.x * kB + threadIdx.x;
    if (i >= N) return;
    const int m = mcols[r];
    const size_t NN = N;
    for (int c0 = 0; c0 < nc; c0 += CMAX) {
        double are[CMAX], aim[CMAX];
        for (int c = 0; c < CMAX; ++c) are[c] = aim[c] = 0;
        for (int j = 0; j < m; ++j) {
            const double* u = U + ustride * r + 2 * NN * j;
            double ur = u[i], ui = u[i + NN];
            const double* y = Y + ((size_t)r * jmax + j) * 2 * Ks + 2 * (k0 + c0);
            for (int c = 0; c < CMAX && c0 + c < nc; ++c) {
                are[c] += ur * y[2 * c] - ui * y[2 * c + 1];
                aim[c] += ur * y[2 * c + 1] + ui * y[2 * c];
            }
        }
        for (int c = 0; c < CMAX && c0 + c < nc; ++c) {
            double* x = X + ((size_t)r * nc + c0 + c) * 2 * NN;
            x[i] = are[c];
            x[i + NN] = aim[c];
        }
    }
}

// part[(r*nc + c)][blk] = || b_r - (K + z_{k0+c} M) X[r][c] ||^2 over the block


// ---------------------------------------------------------------- true residuals from the basis
// With x_k = U y_k, the residual of shift k is b - sum_j y_jk (K u_j + z_k M u_j): the
// stencil is applied once per basis column (KU) and every shift's residual is then
// pointwise, so no solution vector is formed or re-read.
__global__ void k_apply_cols(LevelView<double> L, const double* __restrict__ U, size_t ustride,
                             const int* __restrict__ mcols, double* __restrict__ KU, size_t kstride) {
    const int j = blockIdx.y, r = blockIdx.z;
    if (j >= mcols[r]) return;
    const int i = blockIdx.x * kB + threadIdx.x;
    if (i >= L.N) return;
    const size_t N = L.N;
    const double* xr = U + ustride * r + 2 * N * j;
    const double* xi = xr + N;
    const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
    const int sy = L.nx, sz = L.nx * L.ny;
    double sre = 0, sim = 0;
    if (x + 1 < L.nx) { const double t = L.Tx[i]; sre += t * xr[i + 1]; sim += t * xi[i + 1]; }
    if (x > 0) { const double t = L.Tx[i - 1]; sre += t * xr[i - 1]; sim += t * xi[i - 1]; }
    if (y + 1 < L.ny) { const double t = L.Ty[i]; sre += t * xr[i + sy]; sim += t * xi[i + sy]; }
    if (y > 0) { const double t = L.Ty[i - sy]; sre += t * xr[i - sy]; sim += t * xi[i - sy]; }
    if (z + 1 < L.nz) { const double t = L.Tz[i]; sre += t * xr[i + sz]; sim += t * xi[i + sz]; }
    if (z > 0) { const double t = L.Tz[i - sz]; sre += t * xr[i - sz]; sim += t * xi[i - sz]; }
    double* o = KU + kstride * r + 2 * N * j;
    o[i] = L.D[i] * xr[i] - sre;
    o[i + N] = L.D[i] * xi[i] - sim;
}

template <int kTrK, bool STAGED>  // shifts per pass; y coefficients staged in LDS (m * kTrK of them)
__global__ __launch_bounds__(256) void k_true_res_cols(LevelView<double> L, int Ks, int k0, int kc, int jmax,
                                                       const double* __restrict__ U, size_t ustride,
                                                       const double* __restrict__ KU, size_t kstride,
                                                       const double* __restrict__ Y, const int* __restrict__ mcols,
                                                       const double* __restrict__ zs, const double* __restrict__ b,
                                                       double* __restrict__ part) {
    const int r = blockIdx.y;
    const int m = mcols[r];
    const size_t N = L.N;
    const double* br = b + 2 * N * r;
    const double* Yr = Y + (size_t)r * jmax * 2 * Ks;
    double v[kTrK], zr[kTrK], zi[kTrK];
#pragma unroll
    for (int c = 0; c < kTrK; ++c) {
        v[c] = 0;
        const int cc = min(c, kc - 1);
        zr[c] = zs[2 * (k0 + cc)];
        zi[c] = zs[2 * (k0 + cc) + 1];
    }
    const double* Ur = U + ustride * r;
    const double* KUr = KU + kstride * r;
    // this pass's y coefficients of every column, read by all lanes at once from LDS
    extern __shared__ double ys[];  // [m][kTrK] (re, im)
    if (STAGED) {
        for (int q = threadIdx.x; q < m * kTrK; q += blockDim.x) {
            const int j = q / kTrK, cc = min(q % kTrK, kc - 1);
            ys[2 * q] = Yr[(size_t)j * 2 * Ks + 2 * (k0 + cc)];
            ys[2 * q + 1] = Yr[(size_t)j * 2 * Ks + 2 * (k0 + cc) + 1];
        }
        __syncthreads();
    }
    for (int i = blockIdx.x * kB + threadIdx.x; i < L.N; i += gridDim.x * kB) {
        double ar[kTrK], ai[kTrK];
        const double b0 = br[i], b1 = br[i + N];
#pragma unroll
        for (int c = 0; c < kTrK; ++c) {
            ar[c] = b0;
            ai[c] = b1;
        }
        const double mi = L.m[i];
        // column j + 1 is loaded while column j is used
        double nu0 = 0, nu1 = 0, nk0 = 0, nk1 = 0;
        if (m > 0) {
            nu0 = Ur[i];
            nu1 = Ur[i + N];
            nk0 = KUr[i];
            nk1 = KUr[i + N];
        }
        for (int j = 0; j < m; ++j) {
            const double ur = mi * nu0, ui = mi * nu1, kr = nk0, ki = nk1;  // m u, K u
            if (j + 1 < m) {
                const size_t o = 2 * N * (j + 1) + i;
                nu0 = Ur[o];
                nu1 = Ur[o + N];
                nk0 = KUr[o];
                nk1 = KUr[o + N];
            }
            const double* y = STAGED ? ys + 2 * j * kTrK : Yr + (size_t)j * 2 * Ks + 2 * k0;
#pragma unroll
            for (int c = 0; c < kTrK; ++c) {
                const int cc = STAGED ? c : min(c, kc - 1);
                // t = K u + z m u;  acc -= y t
                const double tr = kr + (zr[c] * ur - zi[c] * ui), ti = ki + (zr[c] * ui + zi[c] * ur);
                const double yr = y[2 * cc], yi = y[2 * cc + 1];
                ar[c] -= yr * tr - yi * ti;
                ai[c] -= yr * ti + yi * tr;
            }
        }
#pragma unroll
        for (int c = 0; c < kTrK; ++c) v[c] += ar[c] * ar[c] + ai[c] * ai[c];
    }
    // block sums of the kc squared norms
    __shared__ double sh[kB / 64][kTrK];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kTrK; ++c) {
        const double t = wave_sum(v[c]);
        if (lane == 0) sh[w][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < kc) {
        double t = 0;
        for (int q = 0; q < kB / 64; ++q) t += sh[q][threadIdx.x];
        part[((size_t)r * Ks + k0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
}

// one wavefront per (right-hand side, shift)
__global__ void k_true_res_cols_finalize(int R, int Ks, int nb, const double* __restrict__ part,
                                         const double* __restrict__ beta, double* __restrict__ out) {
    const int idx = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
    if (idx >= R * Ks) return;
    double s = 0;
    for (int q = lane; q < nb; q += 64) s += part[(size_t)idx * nb + q];
    s = wave_sum(s);
    if (lane == 0) {
        const double bt = beta[idx / Ks];
        out[idx] = bt > 0 ? sqrt(s) / bt : 0.0;
    }
}

int launch_true_residual_cols(hipStream_t st, LevelView<double> L, int R, int Ks, int jmax, int mmax,
                              const double* U, size_t ustride, const double* Y, const int* mcols, const double* zs,
                              const double* b, const double* beta, double* KU, double* part, double* out) {
    const size_t kstride = (size_t)std::max(mmax, 1) * 2 * L.N;
    if (mmax > 0) {
        k_apply_cols<<<dim3((unsigned)((L.N + kB - 1) / kB), mmax, R), kB, 0, st>>>(L, U, ustride, mcols, KU, kstride);
    }
    const int nb = true_res_blocks(L.N, R);
    // shifts per pass: a multiple of 4 up to 32 that covers Ks with the fewest computed lanes
    int best = 32, cost = 1 << 30;
    for (int w = 4; w <= 32; w += 4) {
        const int c = (Ks + w - 1) / w * w + 8 * ((Ks + w - 1) / w);  // lanes plus a per-pass overhead
        if (c < cost) {
            cost = c;
            best = w;
        }
    }
    for (int k0 = 0; k0 < Ks; k0 += best) {
        const int kc = std::min(best, Ks - k0);
#define LT_TR(W)                                                                                                \
    if (sizeof(double) * 2 * W * (size_t)std::max(mmax, 1) <= 64 * 1024)                                    \
        k_true_res_cols<W, true><<<dim3(nb, R), kB, sizeof(double) * 2 * W * (size_t)std::max(mmax, 1), st>>>( \
            L, Ks, k0, kc, jmax, U, ustride, KU, kstride, Y, mcols, zs, b, part);                               \
    else                                                                                                        \
        k_true_res_cols<W, false><<<dim3(nb, R), kB, 0, st>>>(L, Ks, k0, kc, jmax, U, ustride, KU, kstride, Y,  \
                                                              mcols, zs, b, part)
        switch (best) {
            case 4: LT_TR(4); break;
            case 8: LT_TR(8); break;
            case 12: LT_TR(12); break;
            case 16: LT_TR(16); break;
            case 20: LT_TR(20); break;
            case 24: LT_TR(24); break;
            case 28: LT_TR(28); break;
            default: LT_TR(32); break;
        }
#undef LT_TR
    }
    k_true_res_cols_finalize<<<(unsigned)(((size_t)R * Ks * 64 + kB - 1) / kB), kB, 0, st>>>(R, Ks, nb, part, beta,
                                                                                              out);
    LT_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------- sensitivities
// Discrete adjoint of the heads (Section 5.2): with phi = (K + zM)^{-1} b_s and
// psi = (K + zM)^{-1} b_m (complex symmetric operator, no conjugation),
//   d/dp B_m phi = - psi^T (dK/dp + z dM/dp) phi,
// dT_f/dln k_c = T_f k_j / (k_c + k_j) for the face to neighbour j, dT_wall/dln k_c = T_wall,
// dm_c/dln S_c = m_c; the time-domain sensitivity is 2 Re sum_k w_k qhat_k (.).
// One thread per cell and per block of kSensS sources x kSensM receivers: the
// stencil of each field is loaded once per block and serves kSensS (or kSensM)
// pairs.  Indices past ns / nr are clamped (their results are not stored), so
// the loops unroll and all loads of a shift are in flight together.
constexpr int kSensS = 1;
constexpr int kSensM = 2;
__global__ __launch_bounds__(256) void k_sens(LevelView<double> L, const double* __restrict__ kappa,
                                              const double* __restrict__ mS, int ns, int nr,
                                              int nk, int t, int ntimes, const double* __restrict__ X,
                                              const double* __restrict__ zs, const double* __restrict__ wq,
                                              double* __restrict__ JK, double* __restrict__ JS) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= L.N) return;
    const int s0 = blockIdx.y * kSensS;
    const int m0 = blockIdx.z * kSensM;
    const size_t N = L.N;
    const int x = c % L.nx, y = (c / L.nx) % L.ny, z = c / (L.nx * L.ny);
    const int sy = L.nx, sz = L.nx * L.ny;
    // neighbours and face weights dT_f/dln k_c (zero where there is no face)
    int nb[6];
    double wf[6];
    const double kc = kappa[c];
    const int has[6] = {x > 0, x + 1 < L.nx, y > 0, y + 1 < L.ny, z > 0, z + 1 < L.nz};
    const int off[6] = {-1, 1, -sy, sy, -sz, sz};
    double tin = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        nb[f] = has[f] ? c + off[f] : c;
        double T = 0.0;
        if (has[f]) {
            if (f == 0) T = L.Tx[c - 1];
            if (f == 1) T = L.Tx[c];
            if (f == 2) T = L.Ty[c - sy];
            if (f == 3) T = L.Ty[c];
            if (f == 4) T = L.Tz[c - sz];
            if (f == 5) T = L.Tz[c];
        }
        tin += T;
        const double kj = kappa[nb[f]];
        wf[f] = has[f] ? T * kj / (kc + kj) : 0.0;
    }
    const double wall = L.D[c] - tin;  // walls of this cell; their T is proportional to k_c
    const double mc = mS[c];  // S V: the storage the parameter owns
    double aK[kSensS][kSensM], aS[kSensS][kSensM];
#pragma unroll
    for (int a = 0; a < kSensS; ++a)
#pragma unroll
        for (int q = 0; q < kSensM; ++q) aK[a][q] = aS[a][q] = 0.0;
    for (int kk = 0; kk < nk; ++kk) {
        const int k = t * nk + kk;
        const c64 w = {wq[2 * k], wq[2 * k + 1]};
        const c64 zw = cm(w, {zs[2 * k], zs[2 * k + 1]});
        c64 pc[kSensS], dph[kSensS][6];
#pragma unroll
        for (int a = 0; a < kSensS; ++a) {
            const int sa = min(s0 + a, ns - 1);
            const double* ph = X + ((size_t)sa * nk + kk) * 2 * N;
            pc[a] = {ph[c], ph[c + N]};
#pragma unroll
            for (int f = 0; f < 6; ++f) dph[a][f] = {pc[a].re - ph[nb[f]], pc[a].im - ph[nb[f] + N]};
        }
#pragma unroll
        for (int q = 0; q < kSensM; ++q) {
            const int m = min(m0 + q, nr - 1);
            const double* ps = X + ((size_t)(ns + m) * nk + kk) * 2 * N;
            const c64 qc = {ps[c], ps[c + N]};
            c64 dq[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) dq[f] = {qc.re - ps[nb[f]], qc.im - ps[nb[f] + N]};
#pragma unroll
            for (int a = 0; a < kSensS; ++a) {
                c64 g = cm(pc[a], qc);
                const c64 hs = {mc * g.re, mc * g.im};
                g.re *= wall;
                g.im *= wall;
#pragma unroll
                for (int f = 0; f < 6; ++f) {
                    const c64 p = cm(dph[a][f], dq[f]);
                    g.re += wf[f] * p.re;
                    g.im += wf[f] * p.im;
                }
                aK[a][q] += w.re * g.re - w.im * g.im;
                aS[a][q] += zw.re * hs.re - zw.im * hs.im;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < kSensS; ++a)
#pragma unroll
        for (int q = 0; q < kSensM; ++q) {
            const int sa = s0 + a, m = m0 + q;
            if (sa >= ns || m >= nr) continue;
            const size_t o = (((size_t)sa * nr + m) * ntimes + t) * N + c;
            if (JK) JK[o] = -2.0 * aK[a][q];
            if (JS) JS[o] = -2.0 * aS[a][q];
        }
}

// The same contraction with the fields staged in LDS.  For a fixed cell c the Jacobian is
// a product over the (shift, face) index,
//   J_K[s][m] = Re sum_k sum_f (w_k dphi_s,k,f) (dT_f/dln k_c dpsi_m,k,f) + Re sum_k (w_k wall_c phi_s,k) psi_m,k
//   J_S[s][m] = Re sum_k (w_k z_k m_c phi_s,k) psi_m,k,
// so a block of kSensCB cells stages, one shift at a time, the weighted differences of every
// source and receiver field once (kSensA source slots: six faces, the wall term and the
// storage term; kSensB receiver slots: six faces and the centre), and each thread forms
// TS sources x TM receivers of one cell from LDS.  Each field value is loaded once per
// block and shift instead of once per (source, receiver) pair.  CB cells per block; the
// launcher picks the shape whose threads all have work for the call's field counts.
constexpr int kSensA = 8, kSensB = 7;      // staged slots per source / receiver field
// doubles per staged field: 4 words past a multiple of 32 banks, so the consecutive fields
// the lanes of a wavefront read at once fall into different banks
constexpr int sens_fs(int CB) { return 2 * kSensA * CB + 2; }

template <int CB, int TS, int TM>
__global__ __launch_bounds__(256) void k_sens_tile(LevelView<double> L, const double* __restrict__ kappa,
                                                   const double* __restrict__ mS, int ns,
                                                   int nr, int nk, int t, int ntimes, const double* __restrict__ X,
                                                   const double* __restrict__ zs, const double* __restrict__ wq,
                                                   double* __restrict__ JK, double* __restrict__ JS) {
    constexpr int kSensCB = CB, kSensTPC = kB / CB, kSensTS = TS, kSensTM = TM, kSensFS = sens_fs(CB);
    static_assert(kSensFS >= 2 * kSensB * kSensCB && (2 * kSensFS) % 32 == 4, "staged field stride");
    extern __shared__ double sm[];
    // As[s][slot][cb], Bs[m][slot][cb] as (re, im) pairs
    double* As = sm;
    double* Bs = sm + (size_t)ns * kSensFS;
    const size_t N = L.N;
    const int cb = threadIdx.x / kSensTPC, g = threadIdx.x % kSensTPC + kSensTPC * blockIdx.y;
    // workgroups go to the 8 XCDs in turn; renumber them so each XCD takes one run of
    // consecutive cells and the short rows of output it writes complete lines in its own L2
    unsigned bx;
    {
        const unsigned W = gridDim.x, w = blockIdx.x, xk = w % 8u, per = W / 8u, extra = W % 8u;
        bx = xk * per + min(xk, extra) + w / 8u;
    }
    const int c0 = (int)bx * kSensCB;
    const int c = min(c0 + cb, (int)N - 1);
    // thread (si, mi) takes sources si + a nsg and receivers mi + q ntm: the lanes of a
    // wavefront then read consecutive fields
    const int nsg = (ns + kSensTS - 1) / kSensTS, ntm = (nr + kSensTM - 1) / kSensTM;
    const int si = g / ntm, mi = g % ntm;
    const bool work = g < nsg * ntm && c0 + cb < (int)N;
    // staging: thread j of the block takes (field, cell) items; every thread knows its staged
    // cell's neighbours and weights
    const int sy = L.nx, sz = L.nx * L.ny;
    // per staged cell: dT_f/dln k_c of its six faces, its wall term and its mass (once per block)
    __shared__ double Wf[6][kSensCB], Wall[kSensCB], Mc[kSensCB];
    __shared__ int Nb[7][kSensCB];  // the cell itself, then its six neighbours (itself where none)
    if (threadIdx.x < kSensCB) {
        const int q = threadIdx.x;
        const int cc = min(c0 + q, (int)N - 1);
        const int x = cc % L.nx, y = (cc / L.nx) % L.ny, z = cc / sz;
        const int has[6] = {x > 0, x + 1 < L.nx, y > 0, y + 1 < L.ny, z > 0, z + 1 < L.nz};
        const int off[6] = {-1, 1, -sy, sy, -sz, sz};
        const double kc = kappa[cc];
        double tin = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            double T = 0.0, wf = 0.0;
            if (has[e]) {
                if (e == 0) T = L.Tx[cc - 1];
                if (e == 1) T = L.Tx[cc];
                if (e == 2) T = L.Ty[cc - sy];
                if (e == 3) T = L.Ty[cc];
                if (e == 4) T = L.Tz[cc - sz];
                if (e == 5) T = L.Tz[cc];
                const double kj = kappa[cc + off[e]];
                wf = T * kj / (kc + kj);
            }
            tin += T;
            Wf[e][q] = wf;
            Nb[e + 1][q] = has[e] ? cc + off[e] : cc;
        }
        Nb[0][q] = cc;
        Wall[q] = L.D[cc] - tin;  // walls of this cell; their T is proportional to k_c
        Mc[q] = mS[cc];
    }
    double accK[kSensTS][kSensTM], accS[kSensTS][kSensTM];
#pragma unroll
    for (int a = 0; a < kSensTS; ++a)
#pragma unroll
        for (int q = 0; q < kSensTM; ++q) accK[a][q] = accS[a][q] = 0.0;
    const int nitems = (ns + nr) * kSensCB;
    // the seven stencil values (re, im) of staged item it = (field, cell) at shift kk
    auto fetch = [&](int it, int kk, double (&v)[14]) {
        const int f = it / kSensCB, q = it % kSensCB;
        const double* ph = X + ((size_t)f * nk + kk) * 2 * N;
        const double* phi = ph + N;
#pragma unroll
        for (int e = 0; e < 7; ++e) {
            const int nb = Nb[e][q];
            v[2 * e] = ph[nb];
            v[2 * e + 1] = phi[nb];
        }
    };
    auto stage = [&](int it, const double (&v)[14], c64 w, c64 zw) {
        const int f = it / kSensCB, q = it % kSensCB;  // field (sources first), staged cell
        const c64 pc = {v[0], v[1]};
        c64 d[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) d[e] = {pc.re - v[2 * e + 2], pc.im - v[2 * e + 3]};
        if (f < ns) {
            // w dphi per face, w wall phi, w z m phi
            const double wall = Wall[q], mc = Mc[q];
            double* a = As + (size_t)f * kSensFS + 2 * q;
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const c64 u = cm(w, d[e]);
                a[2 * e * kSensCB] = u.re;
                a[2 * e * kSensCB + 1] = u.im;
            }
            const c64 vw = cm(w, {wall * pc.re, wall * pc.im});
            const c64 vz = cm(zw, {mc * pc.re, mc * pc.im});
            a[2 * 6 * kSensCB] = vw.re;
            a[2 * 6 * kSensCB + 1] = vw.im;
            a[2 * 7 * kSensCB] = vz.re;
            a[2 * 7 * kSensCB + 1] = vz.im;
        } else {
            // dT_f/dln k_c dpsi per face, psi
            double* b = Bs + (size_t)(f - ns) * kSensFS + 2 * q;
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const double wf = Wf[e][q];
                b[2 * e * kSensCB] = wf * d[e].re;
                b[2 * e * kSensCB + 1] = wf * d[e].im;
            }
            b[2 * 6 * kSensCB] = pc.re;
            b[2 * 6 * kSensCB + 1] = pc.im;
        }
    };
    // each thread's first item of the next shift is loaded while the current shift is formed
    const int it0 = threadIdx.x;
    const bool h0 = it0 < nitems;
    double pv[14];
    __syncthreads();  // the neighbour table is written
    if (h0) fetch(it0, 0, pv);
    for (int kk = 0; kk < nk; ++kk) {
        const int k = t * nk + kk;
        const c64 w = {wq[2 * k], wq[2 * k + 1]};
        const c64 zw = cm(w, {zs[2 * k], zs[2 * k + 1]});
        __syncthreads();  // the previous shift's reads of the stage are done
        if (h0) stage(it0, pv, w, zw);
        for (int it = it0 + (int)blockDim.x; it < nitems; it += blockDim.x) {
            double v[14];
            fetch(it, kk, v);
            stage(it, v, w, zw);
        }
        __syncthreads();
        if (h0 && kk + 1 < nk) fetch(it0, kk + 1, pv);
        if (work) {
#pragma unroll
            for (int e = 0; e < kSensB; ++e) {
                c64 bv[kSensTM];
#pragma unroll
                for (int q = 0; q < kSensTM; ++q) {
                    const int m = min(mi + q * ntm, nr - 1);
                    const double* b = Bs + (size_t)m * kSensFS + 2 * (e * kSensCB + cb);
                    bv[q] = {b[0], b[1]};
                }
#pragma unroll
                for (int a = 0; a < kSensTS; ++a) {
                    const int sa = min(si + a * nsg, ns - 1);
                    const double* ap = As + (size_t)sa * kSensFS + 2 * (e * kSensCB + cb);
                    const c64 av = {ap[0], ap[1]};
#pragma unroll
                    for (int q = 0; q < kSensTM; ++q) accK[a][q] += av.re * bv[q].re - av.im * bv[q].im;
                    if (e == 6) {
                        // the storage term pairs the same receiver centre with slot 7
                        const double* zp = As + (size_t)sa * kSensFS + 2 * (7 * kSensCB + cb);
                        const c64 zv = {zp[0], zp[1]};
#pragma unroll
                        for (int q = 0; q < kSensTM; ++q) accS[a][q] += zv.re * bv[q].re - zv.im * bv[q].im;
                    }
                }
            }
        }
    }
    if (!work) return;
#pragma unroll
    for (int a = 0; a < kSensTS; ++a)
#pragma unroll
        for (int q = 0; q < kSensTM; ++q) {
            const int sa = si + a * nsg, m = mi + q * ntm;
            if (sa >= ns || m >= nr) continue;
            const size_t o = (((size_t)sa * nr + m) * ntimes + t) * N + c;
            if (JK) JK[o] = -2.0 * accK[a][q];
            if (JS) JS[o] = -2.0 * accS[a][q];
        }
}

template <int CB, int TS, int TM>
static void launch_sens_tile(hipStream_t st, LevelView<double> L, const double* kappa, const double* mS, int ns,
                             int nr, int nk, int t, int ntimes, const double* X, const double* zs, const double* wq,
                             double* JK, double* JS) {
    const size_t shm = sizeof(double) * (size_t)(ns + nr) * sens_fs(CB);
    const int groups = ((ns + TS - 1) / TS) * ((nr + TM - 1) / TM);
    const int tpc = kB / CB;
    dim3 grid((unsigned)((L.N + CB - 1) / CB), (unsigned)((groups + tpc - 1) / tpc));
    k_sens_tile<CB, TS, TM><<<grid, kB, shm, st>>>(L, kappa, mS, ns, nr, nk, t, ntimes, X, zs, wq, JK, JS);
}

// The same contraction for P1 elements (parameters per cell of the cell grid; fields on its
// interior vertices, zero at wall vertices).  dK/dln kappa_c is kappa_c times the cell's
// element stiffness at kappa = 1, which couples only the corners along the cell's edges:
// in 2D its four edges, each with hy / (2 hx) (x edges) or hx / (2 hy) (y edges); in 3D its
// twelve edges, an x edge with (tetrahedra holding it) x hy hz / (6 hx), two for the edges at
// (y, z) = (0, 0) and (1, 1), one for the other two (y and z edges alike).  dM/dln S_c puts
// S_c |e| / (d + 1) on each corner per element holding it: corner weights 1, 2, 2, 1 (v00,
// v10, v01, v11) times hx hy / 6 in 2D; 6 at v000 and v111, 2 elsewhere, times
// hx hy hz / 24 in 3D.  One thread per cell and per (source, kSensM receivers).
__global__ __launch_bounds__(256) void k_sens_p1(int ncx, int ncy, int ncz, double hx, double hy, double hz,
                                                 const double* __restrict__ kappa, const double* __restrict__ S,
                                                 int ns, int nr, int nk, int t, int ntimes, size_t N,
                                                 const double* __restrict__ X, const double* __restrict__ zs,
                                                 const double* __restrict__ wq, double* __restrict__ JK,
                                                 double* __restrict__ JS) {
    const int nc = ncx * ncy * ncz;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int s0 = blockIdx.y, m0 = blockIdx.z * kSensM;
    const bool d3 = ncz > 1;
    const int i = c % ncx, j = (c / ncx) % ncy, l = c / (ncx * ncy);
    const int nvx = ncx - 1, nvy = ncy - 1;
    // corners v(a, b, e), a + 2 b + 4 e; -1 on a wall
    int vi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int I = i + (q & 1), J = j + ((q >> 1) & 1), Kz = l + ((q >> 2) & 1);
        const bool in = I > 0 && I < ncx && J > 0 && J < ncy && (!d3 || (Kz > 0 && Kz < ncz));
        vi[q] = (q >= 4 && !d3) || !in ? -1 : (I - 1) + nvx * ((J - 1) + nvy * (d3 ? Kz - 1 : 0));
    }
    // edges (corner pair, weight at kappa = 1)
    int ea[12], eb[12];
    double ew[12];
    int ne = 0;
    if (!d3) {
        const double ax = hy / (2.0 * hx), ay = hx / (2.0 * hy);
        ea[0] = 0; eb[0] = 1; ew[0] = ax;  // (00, 10)
        ea[1] = 2; eb[1] = 3; ew[1] = ax;  // (01, 11)
        ea[2] = 0; eb[2] = 2; ew[2] = ay;  // (00, 01)
        ea[3] = 1; eb[3] = 3; ew[3] = ay;  // (10, 11)
        ne = 4;
    } else {
        const double ax = hy * hz / (6.0 * hx), ay = hx * hz / (6.0 * hy), az = hx * hy / (6.0 * hz);
        // x edges at (b, e): (0, 0) and (1, 1) in two tetrahedra, (1, 0) and (0, 1) in one
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = q & 1, e = q >> 1;
            ea[ne] = 2 * b + 4 * e; eb[ne] = 1 + 2 * b + 4 * e; ew[ne] = ax * (b == e ? 2.0 : 1.0); ++ne;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = q & 1, e = q >> 1;
            ea[ne] = a + 4 * e; eb[ne] = a + 2 + 4 * e; ew[ne] = ay * (a == e ? 2.0 : 1.0); ++ne;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = q & 1, b = q >> 1;
            ea[ne] = a + 2 * b; eb[ne] = a + 2 * b + 4; ew[ne] = az * (a == b ? 2.0 : 1.0); ++ne;
        }
    }
    double mw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (!d3) mw[q] = q >= 4 ? 0.0 : hx * hy / 6.0 * ((q == 0 || q == 3) ? 1.0 : 2.0);
        else mw[q] = hx * hy * hz / 24.0 * ((q == 0 || q == 7) ? 6.0 : 2.0);
    }
    const double kc = kappa[c], sc = S[c];
    double aK[kSensM], aS[kSensM];
#pragma unroll
    for (int q = 0; q < kSensM; ++q) aK[q] = aS[q] = 0.0;
    const int sa = min(s0, ns - 1);
    for (int kk = 0; kk < nk; ++kk) {
        const int k = t * nk + kk;
        const c64 w = {wq[2 * k], wq[2 * k + 1]};
        const c64 zw = cm(w, {zs[2 * k], zs[2 * k + 1]});
        const double* ph = X + ((size_t)sa * nk + kk) * 2 * N;
        c64 pv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[q] = vi[q] >= 0 ? c64{ph[vi[q]], ph[vi[q] + N]} : c64{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < kSensM; ++r) {
            const int m = min(m0 + r, nr - 1);
            const double* ps = X + ((size_t)(ns + m) * nk + kk) * 2 * N;
            c64 qv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) qv[q] = vi[q] >= 0 ? c64{ps[vi[q]], ps[vi[q] + N]} : c64{0.0, 0.0};
            c64 gK = {0.0, 0.0}, gS = {0.0, 0.0};
            for (int e = 0; e < ne; ++e) {
                const c64 dp = {pv[ea[e]].re - pv[eb[e]].re, pv[ea[e]].im - pv[eb[e]].im};
                const c64 dq = {qv[ea[e]].re - qv[eb[e]].re, qv[ea[e]].im - qv[eb[e]].im};
                const c64 p = cm(dp, dq);
                gK.re += ew[e] * p.re;
                gK.im += ew[e] * p.im;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const c64 p = cm(pv[q], qv[q]);
                gS.re += mw[q] * p.re;
                gS.im += mw[q] * p.im;
            }
            aK[r] += kc * (w.re * gK.re - w.im * gK.im);
            aS[r] += sc * (zw.re * gS.re - zw.im * gS.im);
        }
    }
    if (s0 >= ns) return;
#pragma unroll
    for (int r = 0; r < kSensM; ++r) {
        const int m = m0 + r;
        if (m >= nr) continue;
        const size_t o = (((size_t)s0 * nr + m) * ntimes + t) * nc + c;
        if (JK) JK[o] = -2.0 * aK[r];
        if (JS) JS[o] = -2.0 * aS[r];
    }
}

int launch_sens_p1(hipStream_t st, const lt_grid& cells, const double* kappa, const double* S, int ns, int nr,
                   int nk, int t, int ntimes, size_t N, const double* X, const double* zs, const double* wq,
                   double* JK, double* JS) {
    const int ncz = cells.ndim == 3 ? cells.n[2] : 1;
    const int nc = cells.n[0] * cells.n[1] * ncz;
    dim3 grid((unsigned)((nc + kB - 1) / kB), (unsigned)ns, (unsigned)((nr + kSensM - 1) / kSensM));
    k_sens_p1<<<grid, kB, 0, st>>>(cells.n[0], cells.n[1], ncz, cells.h[0], cells.h[1],
                                   cells.ndim == 3 ? cells.h[2] : 1.0, kappa, S, ns, nr, nk, t, ntimes, N, X, zs,
                                   wq, JK, JS);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_sens(hipStream_t st, LevelView<double> L, const double* kappa, const double* mS, int ns, int nr, int nk,
                int t, int ntimes, const double* X, const double* zs, const double* wq, double* JK, double* JS) {
    // 8 cells x (4 sources x 4 receivers per thread) when one block's 32 threads per cell cover
    // every (source, receiver) pair; else 4 cells x (5 x 4), several blocks per cell when needed
    const bool fit8 = ((ns + 3) / 4) * ((nr + 3) / 4) <= kB / 8 &&
                      sizeof(double) * (size_t)(ns + nr) * sens_fs(8) <= 64 * 1024;
    if (fit8) {
        launch_sens_tile<8, 4, 4>(st, L, kappa, mS, ns, nr, nk, t, ntimes, X, zs, wq, JK, JS);
    } else if (sizeof(double) * (size_t)(ns + nr) * sens_fs(4) <= 64 * 1024) {
        launch_sens_tile<4, 5, 4>(st, L, kappa, mS, ns, nr, nk, t, ntimes, X, zs, wq, JK, JS);
    } else {
        dim3 grid((unsigned)((L.N + kB - 1) / kB), (ns + kSensS - 1) / kSensS, (nr + kSensM - 1) / kSensM);
        k_sens<<<grid, kB, 0, st>>>(L, kappa, mS, ns, nr, nk, t, ntimes, X, zs, wq, JK, JS);
    }
    LT_HIP(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------- launchers
template <typename T>
int launch_net_scale(hipStream_t st, LevelView<double> L, cdouble tau, int R, T* d, const double* v, double* part,
                     const int* active) {
    const int nb = reduce_blocks(L.N, R);
    k_net_dots<T><<<dim3(nb, R), kB, 0, st>>>(L, tau.real(), tau.imag(), d, v, part, active);
    k_net_scale<T><<<dim3((L.N + kB - 1) / kB, R), kB, 0, st>>>(L.N, nb, part, d, active);
    LT_HIP(hipGetLastError());
    return 0;
}
template int launch_net_scale<float>(hipStream_t, LevelView<double>, cdouble, int, float*, const double*, double*,
                                     const int*);
template int launch_net_scale<double>(hipStream_t, LevelView<double>, cdouble, int, double*, const double*, double*,
                                      const int*);

int launch_net_guard(hipStream_t st, int R, int nb, const double* part, const int* active, int* bad, int* counts) {
    k_net_guard<<<1, 256, 0, st>>>(R, nb, part, active, bad, counts);
    LT_HIP(hipGetLastError());
    return 0;
}

static inline unsigned nb_for(size_t n) { return (unsigned)((n + kB - 1) / kB); }

int launch_scatter_points(hipStream_t st, int R, int N, const int* off, const int* cell, const double* wt,
                          double* b) {
    k_scatter_points<<<nb_for(R), kB, 0, st>>>(R, N, off, cell, wt, b);
    LT_HIP(hipGetLastError());
    return 0;
}

int reduce_blocks(int N, int R) {
    // about 4 cells per thread and at least a few hundred blocks overall
    int nb = (N + 4 * kB - 1) / (4 * kB);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return nb;
}

int true_res_blocks(int N, int R) {
    // enough workgroups to fill the chip (about 4096 over all right-hand sides), and no more:
    // each thread re-reads the uniform y coefficients of every column for every cell it takes,
    // so with many right-hand sides several cells per thread amortise those loads
    const int per_rhs = (4096 + R - 1) / std::max(R, 1);
    return std::max(1, std::min({1024, (N + kB - 1) / kB, per_rhs}));
}

int launch_norms(hipStream_t st, int N, int R, size_t vstride, const double* x, double* part, double* out,
                 const int* active) {
    int nb = reduce_blocks(N, R);
    k_norm2_partial<<<dim3(nb, R), kB, 0, st>>>(N, vstride, x, part, active);
    k_norm_finalize<<<nb_for(R), kB, 0, st>>>(R, nb, part, out);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_scale_into(hipStream_t st, int N, int R, size_t instride, size_t outstride, const double* in,
                      const double* nrm, double* out) {
    k_scale_into<<<dim3(nb_for(2 * (size_t)N), R), kB, 0, st>>>(N, instride, outstride, in, nrm, out);
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_inner_init(hipStream_t st, int N, int R, size_t qstride, double* v, double* u, size_t ustride,
                      double* rho, T* lo, const int* active, const double* scale, int cpnx, int cpny) {
    k_inner_init<T><<<dim3(nb_for(2 * (size_t)N), R), kB, 0, st>>>(N, qstride, v, u, ustride, rho, lo, active,
                                                                   scale, cpnx, cpny);
    LT_HIP(hipGetLastError());
    return 0;
}
template int launch_inner_init<double>(hipStream_t, int, int, size_t, double*, double*, size_t, double*,
                                       double*, const int*, const double*, int, int);
template int launch_inner_init<float>(hipStream_t, int, int, size_t, double*, double*, size_t, double*,
                                      float*, const int*, const double*, int, int);

int launch_iter_begin(hipStream_t st, int R, const int* active, int* inner_active, int* count, int j,
                      double* rprev) {
    k_iter_begin<<<1, 256, 0, st>>>(R, active, inner_active, count, j, rprev);
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_inner_update(hipStream_t st, LevelView<double> L, cdouble tau, int R, const T* e, double* u,
                        size_t ustride, const int* jcol, double* rho, T* lo, double* part, const int* inner_active,
                        int cp, const int* list) {
    int nb = reduce_blocks(L.N, R);
    if (list)
        k_inner_update_rb<T, kSweepRhs><<<dim3(nb, (R + kSweepRhs - 1) / kSweepRhs), kB, 0, st>>>(
            L, tau.real(), tau.imag(), e, u, ustride, jcol, rho, lo, part, list, R, cp);
    else
        k_inner_update<T><<<dim3(nb, R), kB, 0, st>>>(L, tau.real(), tau.imag(), e, u, ustride, jcol, rho, lo, part,
                                                      inner_active, cp);
    LT_HIP(hipGetLastError());
    return 0;
}
template int launch_inner_update<double>(hipStream_t, LevelView<double>, cdouble, int, const double*, double*,
                                         size_t, const int*, double*, double*, double*, const int*, int, const int*);
template int launch_inner_update<float>(hipStream_t, LevelView<double>, cdouble, int, const float*, double*,
                                        size_t, const int*, double*, float*, double*, const int*, int, const int*);

int launch_inner_finalize(hipStream_t st, int nb, int R, const double* part, const int* active, const double* worst,
                          double relax_tol, double tol, int inner_max, int* inner_active, int* vcycles, int* count,
                          double* rprev, int* est) {
    k_inner_finalize<<<1, 1024, 0, st>>>(R, nb, part, active, worst, relax_tol, tol, inner_max, inner_active,
                                         vcycles, count, rprev, est);
    LT_HIP(hipGetLastError());
    return 0;
}


// One CGS2 step for column j: Q[:, j+1] = normalised (I - Q Q^*)^2 (M u_j); Hbar column j.
int launch_cgs2(hipStream_t st, int N, int R, int j, const double* m, const double* U, size_t ustride, double* Q,
                size_t qstride, double* H, int hstride, size_t hrstride, double* part, int pstride, double* c1,
                double* c2, int cstride, double* scale, double* partn, const int* active) {
    int nb = reduce_blocks(N, R);
    int ncols = j + 1;
    const double* u = U + 2 * (size_t)N * j;
    double* qn = Q + 2 * (size_t)N * (j + 1);
    dim3 g(nb, R);
    const dim3 gd(nb, R, (ncols + kGroup - 1) / kGroup);
    const size_t shm = sizeof(double) * 2 * (ncols + 1);
    // first pass: coefficients of M u_j, then its projection; second pass on the result
    k_mdot<<<gd, kB, 0, st>>>(N, ncols, Q, qstride, m, u, ustride, nullptr, 0, part, pstride, active);
    k_update_sum<<<g, kB, shm, st>>>(N, ncols, Q, qstride, m, u, ustride, nullptr, 0, part, nb, pstride, c1, cstride,
                                     qn, qstride, nullptr, active);
    k_mdot<<<gd, kB, 0, st>>>(N, ncols, Q, qstride, nullptr, nullptr, 0, qn, qstride, part, pstride, active);
    k_update_sum<<<g, kB, shm, st>>>(N, ncols, Q, qstride, nullptr, nullptr, 0, qn, qstride, part, nb, pstride, c2,
                                     cstride, qn, qstride, partn, active);
    // Hessenberg column and 1 / ||q_{j+1}||; the next iteration's first read applies the scale
    k_hcol_finalize<<<R, 256, 0, st>>>(R, j, nb, c1, c2, cstride, partn, H, hstride, hrstride, scale, active);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_ls_update(hipStream_t st, int R, int Ks, int j, cdouble tau, const double* zs, const double* omega,
                     int rinit, double tol, bool fom, const double* H, int hstride, size_t hrstride,
                     const double* beta, const LSState& s, int* active, int* mcols, double* worst, int* conv,
                     const LSStart& start) {
    int threads = ((Ks + 63) / 64) * 64;
    if (threads > kB) threads = kB;
    size_t shm = sizeof(double) * 2 * (j + 2);
    k_ls_update<<<R, threads, shm, st>>>(R, Ks, j, tau.real(), tau.imag(), zs, omega, rinit, tol, fom ? 1 : 0, H,
                                         hstride, hrstride, beta, s, active, mcols, worst, conv, start.g0,
                                         start.bnorm);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_gather(hipStream_t st, int R, int N, int np, const int* off, const int* cell, const double* wt,
                  const double* U, size_t ustride, int j, double* G, int jmax, const int* active) {
    if (np == 0) return 0;
    k_gather<<<dim3(nb_for(np), R), kB, 0, st>>>(R, N, np, off, cell, wt, U, ustride, j, G, jmax, active);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_backsolve(hipStream_t st, int R, int Ks, const int* mcols, const LSState& s, double* Y, int jmax,
                     bool fom) {
    k_backsolve<<<dim3(nb_for(Ks), R), kB, 0, st>>>(R, Ks, mcols, s, Y, jmax, fom ? 1 : 0);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_heads(hipStream_t st, int Rs, int r0, int np, int ntimes, int nk, const double* wq, const double* w,
                 const double* G, const double* Y, const int* mcols, int jmax, double* phi, bool accumulate) {
    int tot = (Rs > 0 ? Rs : 1) * np * ntimes;
    if (tot == 0) return 0;
    k_heads<<<nb_for(tot), kB, 0, st>>>(Rs, r0, np, ntimes, nk, wq, w, G, Y, mcols, jmax, phi, accumulate ? 1 : 0);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_fill_g0(hipStream_t st, int R, int Ks, const double* bnorm, double* g0) {
    k_fill_g0<<<nb_for(R * Ks), kB, 0, st>>>(R, Ks, bnorm, g0);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_restart_rhs(hipStream_t st, int R, int N, int Ks, const double* Q, size_t qstride, const int* mcols,
                       const int* restart, const double* eta, double* b, double* g0) {
    const unsigned nbx = (unsigned)std::min<size_t>((2 * (size_t)N + kB - 1) / kB, 1024);
    k_restart_rhs<<<dim3(nbx, R), kB, 0, st>>>(R, N, Ks, Q, qstride, mcols, restart, eta, b, g0);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_unscale_y(hipStream_t st, int R, int Ks, int jmax, const int* mcols, const double* g0, const double* bnorm,
                     double* Y) {
    k_unscale_y<<<dim3((Ks + 63) / 64, R), 64, 0, st>>>(R, Ks, jmax, mcols, g0, bnorm, Y);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_mass_rhs(hipStream_t st, int N, const double* m, const double* phi0, double* b) {
    k_mass_rhs<<<nb_for(N), kB, 0, st>>>(N, m, phi0, b);
    LT_HIP(hipGetLastError());
    return 0;
}

int launch_form_x(hipStream_t st, int N, int R, int nc, int k0, int Ks, const double* U, size_t ustride,
                  const double* Y, int jmax, const int* mcols, double* X) {
    k_form_x<<<dim3(nb_for(N), R), kB, 0, st>>>(N, nc, k0, Ks, U, ustride, Y, jmax, mcols, X);
    LT_HIP(hipGetLastError());
    return 0;
}


}  // namespace lt
