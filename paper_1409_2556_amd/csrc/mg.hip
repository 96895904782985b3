// Geometric multigrid for the complex-shifted cell-centred FV operator K + tau M.
//
// Levels are built by aggregating 2 cells per coarsened axis.  The coarse
// transmissibility across an aggregate interface is the sum of the fine face
// transmissibilities on that interface times h_a / H_a (1/2 on a halved
// axis), which is exact for a homogeneous medium; walls scale the same way;
// the lumped mass is summed.  Axes are halved only while their spacing is
// within 1.5x of the finest spacing (semi-coarsening of anisotropic grids).
// Restriction sums the fine residuals of an aggregate (the FV balance of the
// coarse cell); prolongation is bilinear/trilinear in the cell centres with a
// ghost value mirrored through the wall (odd for zero Dirichlet, even for zero
// Neumann).  Smoothing is red-black Gauss-Seidel; the coarsest level is
// solved exactly with a dense inverse per preconditioner shift.
#include "lt_internal.h"
#include "mg_fused.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

namespace lt {

static constexpr int kBlock = 256;
static constexpr int kMaxCoarseDense = 512;

int DevBuf::reserve(size_t n) {
    if (n <= bytes) return 0;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, n) != hipSuccess) {
        p = nullptr;
        set_last_error("hipMalloc failed");
        return LT_ENOMEM;
    }
    bytes = n;
    return 0;
}
void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

LevelView<double> Level::v64() const {
    const double* b = c64.as<double>();
    return {n[0], n[1], n[2], N, b, b + N, b + 2 * (size_t)N, b + 3 * (size_t)N, b + 4 * (size_t)N};
}
LevelView<float> Level::v32() const {
    const float* b = c32.as<float>();
    return {n[0], n[1], n[2], N, b, b + N, b + 2 * (size_t)N, b + 3 * (size_t)N, b + 4 * (size_t)N};
}

// ------------------------------------------------------------------ helpers
template <typename T> struct cpx {
    T re, im;
};
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cpx<T> cdiv(cpx<T> a, cpx<T> b) {
    T d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// Colour-planar order (FP32 cycles of 3D grids, levels above the single-workgroup ones): the
// cells of colour c = (x + y + z) & 1 are stored contiguously from c N/2 on, in storage
// order (nx even), so a one-colour half-sweep reads and writes whole cache lines of one
// colour.  Position of cell i = (x, y, z):
__device__ __forceinline__ int cp_at(int i, int x, int y, int z, int N) {
    return ((x + y + z) & 1) * (N >> 1) + (i >> 1);
}

// Off-diagonal sum  sum_nbr T x_nbr  at cell i = (x, y, z) of plane pair (re, im).
template <typename T>
__device__ __forceinline__ cpx<T> offsum(const LevelView<T>& L, const T* xr, const T* xi, int i, int x,
                                         int y, int z) {
    cpx<T> s = {0, 0};
    if (x + 1 < L.nx) { T t = L.Tx[i]; s.re += t * xr[i + 1]; s.im += t * xi[i + 1]; }
    if (x > 0) { T t = L.Tx[i - 1]; s.re += t * xr[i - 1]; s.im += t * xi[i - 1]; }
    const int sy = L.nx;
    if (y + 1 < L.ny) { T t = L.Ty[i]; s.re += t * xr[i + sy]; s.im += t * xi[i + sy]; }
    if (y > 0) { T t = L.Ty[i - sy]; s.re += t * xr[i - sy]; s.im += t * xi[i - sy]; }
    const int sz = L.nx * L.ny;
    if (z + 1 < L.nz) { T t = L.Tz[i]; s.re += t * xr[i + sz]; s.im += t * xi[i + sz]; }
    if (z > 0) { T t = L.Tz[i - sz]; s.re += t * xr[i - sz]; s.im += t * xi[i - sz]; }
    return s;
}

// ------------------------------------------------------------------ assembly
// Fine-level coefficients from kappa and S.  out = [Tx, Ty, Tz, D(unused here), m],
// walls = [Wx, Wy, Wz] (wall transmissibility per axis, summed over both walls).
// A water-table wall adds sy * area to m (no conductive flux); mstor, when
// given, receives the storage part S V alone.
__global__ void k_fine_assemble(const double* __restrict__ kappa, const double* __restrict__ S, int nx,
                                int ny, int nz, int ndim, double hx, double hy, double hz, int4 bclo,
                                int4 bchi, double sy, double* __restrict__ out, double* __restrict__ walls,
                                double* __restrict__ mstor) {
    const int N = nx * ny * nz;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    double V = hx * hy * hz;
    double h[3] = {hx, hy, hz};
    int n[3] = {nx, ny, nz};
    int c[3] = {x, y, z};
    int stride[3] = {1, nx, nx * ny};
    int lo[3] = {bclo.x, bclo.y, bclo.z};
    int hi[3] = {bchi.x, bchi.y, bchi.z};
    double ki = kappa[i];
    double wt = 0.0;  // water-table storage of this cell's walls
    for (int a = 0; a < 3; ++a) {
        double T = 0.0, W = 0.0;
        if (a < ndim) {
            double area = V / h[a];
            if (c[a] + 1 < n[a]) {
                double kj = kappa[i + stride[a]];
                T = 2.0 * ki * kj / (ki + kj) * area / h[a];
            }
            if (c[a] == 0 && lo[a] == LT_BC_DIRICHLET0) W += 2.0 * ki * area / h[a];
            if (c[a] == n[a] - 1 && hi[a] == LT_BC_DIRICHLET0) W += 2.0 * ki * area / h[a];
            if (c[a] == 0 && lo[a] == LT_BC_WATER_TABLE) wt += sy * area;
            if (c[a] == n[a] - 1 && hi[a] == LT_BC_WATER_TABLE) wt += sy * area;
        }
        out[(size_t)a * N + i] = T;
        walls[(size_t)a * N + i] = W;
    }
    const double ms = S[i] * V;
    out[(size_t)4 * N + i] = ms + wt;
    if (mstor) mstor[i] = ms;
}

// Aggregate a fine level into a coarse one (see the file comment).
__global__ void k_coarsen(const double* __restrict__ fc, const double* __restrict__ fw, int fnx, int fny,
                          int fnz, int cnx, int cny, int cnz, int cox, int coy, int coz,
                          double* __restrict__ cc, double* __restrict__ cw, double3 wscale) {
    const int Nc = cnx * cny * cnz;
    const int Nf = fnx * fny * fnz;
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= Nc) return;
    int X = I % cnx, Y = (I / cnx) % cny, Z = I / (cnx * cny);
    int co[3] = {cox, coy, coz};
    int C[3] = {X, Y, Z};
    int k0[3], k1[3];
    for (int a = 0; a < 3; ++a) {
        k0[a] = co[a] ? 2 * C[a] : C[a];
        k1[a] = co[a] ? 2 * C[a] + 1 : C[a];
    }
    double Tsum[3] = {0, 0, 0}, Wsum[3] = {0, 0, 0}, msum = 0.0;
    for (int z = k0[2]; z <= k1[2]; ++z)
        for (int y = k0[1]; y <= k1[1]; ++y)
            for (int x = k0[0]; x <= k1[0]; ++x) {
                int f = x + fnx * (y + fny * z);
                int fc3[3] = {x, y, z};
                msum += fc[(size_t)4 * Nf + f];
                for (int a = 0; a < 3; ++a) {
                    Wsum[a] += fw[(size_t)a * Nf + f];
                    // only children on the +a interface of the aggregate carry the coarse face
                    if (fc3[a] == k1[a]) Tsum[a] += fc[(size_t)a * Nf + f];
                }
            }
    // wscale: the wall terms' correction where the wall is not half a spacing from the first
    // unknown (delta_fine / delta_coarse; 1 for cell-centred levels)
    const double ws[3] = {wscale.x, wscale.y, wscale.z};
    for (int a = 0; a < 3; ++a) {
        double fa = co[a] ? 0.5 : 1.0;
        cc[(size_t)a * Nc + I] = fa * Tsum[a];
        cw[(size_t)a * Nc + I] = fa * Wsum[a] * ws[a];
    }
    cc[(size_t)4 * Nc + I] = msum;
}

// D_i = sum_a (W_a[i] + T_a[i] + T_a[i - e_a]).
// P1 finite elements (Section 2.1's weak form) on a 2D cell grid ncx x ncy split into right
// triangles (each cell by its anti-diagonal), lumped mass, zero head on every wall, assembled
// on the interior vertices (ncx - 1) x (ncy - 1), x fastest.  A right triangle couples the
// two ends of its hypotenuse by zero, so the stiffness is a five-point stencil: the edge from
// vertex (I, J) to (I + 1, J) carries hy/hx times the mean kappa of the two cells beside it,
// the edge to (I, J + 1) hx/hy times theirs; an edge to a wall vertex is a wall term.  The
// lumped mass sums S |e| / 3 over the six triangles at the vertex.  Same layout as
// k_fine_assemble (Tx, Ty, Tz, D by k_finish_diag, m; walls per axis).
__global__ void k_p1_assemble(const double* __restrict__ kappa, const double* __restrict__ S, int ncx, int ncy,
                              double hx, double hy, double* __restrict__ out, double* __restrict__ walls) {
    const int nvx = ncx - 1, nvy = ncy - 1, N = nvx * nvy;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int x = i % nvx, y = i / nvx, I = x + 1, J = y + 1;  // vertex (I, J); cell (a, b) has corner (a, b) lowest
    const double kc00 = kappa[(I - 1) + ncx * (J - 1)], kc10 = kappa[I + ncx * (J - 1)];
    const double kc01 = kappa[(I - 1) + ncx * J], kc11 = kappa[I + ncx * J];
    const double ax = hy / hx, ay = hx / hy;
    const double e_right = ax * 0.5 * (kc10 + kc11);  // to (I + 1, J): cells (I, J - 1), (I, J)
    const double e_left = ax * 0.5 * (kc00 + kc01);   // to (I - 1, J): cells (I - 1, J - 1), (I - 1, J)
    const double e_up = ay * 0.5 * (kc01 + kc11);     // to (I, J + 1): cells (I - 1, J), (I, J)
    const double e_down = ay * 0.5 * (kc00 + kc10);  // to (I, J - 1): cells (I - 1, J - 1), (I, J - 1)
    const size_t n = N;
    out[i] = x + 1 < nvx ? e_right : 0.0;
    out[n + i] = y + 1 < nvy ? e_up : 0.0;
    out[2 * n + i] = 0.0;
    walls[i] = (x == 0 ? e_left : 0.0) + (x + 1 == nvx ? e_right : 0.0);
    walls[n + i] = (y == 0 ? e_down : 0.0) + (y + 1 == nvy ? e_up : 0.0);
    walls[2 * n + i] = 0.0;
    const double s00 = S[(I - 1) + ncx * (J - 1)], s10 = S[I + ncx * (J - 1)];
    const double s01 = S[(I - 1) + ncx * J], s11 = S[I + ncx * J];
    // six triangles: one of cell (I, J), two of (I - 1, J), two of (I, J - 1), one of (I - 1, J - 1)
    out[4 * n + i] = hx * hy / 6.0 * (s11 + 2.0 * s01 + 2.0 * s10 + s00);
}

// The same in 3D: each cell of an ncx x ncy x ncz grid split into the six path tetrahedra of
// the Kuhn subdivision (v000, v000 + e_a, v000 + e_a + e_b, v111 for every order of the axes).
// Their barycentric gradients are orthogonal for every pair of vertices off an axis, so the
// stiffness is a seven-point stencil on the interior vertices.  An x edge lies in six
// tetrahedra of its four cells: two of the cell beyond it in y and z and two of the one
// behind it in both, one of each of the other two; each adds kappa hy hz / (6 hx) (y and z
// edges alike).  A vertex lies in all six tetrahedra of the two cells it is the lowest or the
// highest corner of and in two of each of its other six cells, each adding S |e| / 4.
__global__ void k_p1_assemble3d(const double* __restrict__ kappa, const double* __restrict__ S, int ncx, int ncy,
                                int ncz, double hx, double hy, double hz, double* __restrict__ out,
                                double* __restrict__ walls) {
    const int nvx = ncx - 1, nvy = ncy - 1, nvz = ncz - 1, N = nvx * nvy * nvz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int x = i % nvx, y = (i / nvx) % nvy, z = i / (nvx * nvy);
    const int I = x + 1, J = y + 1, K = z + 1;
    auto kc = [&](int a, int b, int c) { return kappa[a + ncx * (b + ncy * c)]; };
    auto sc = [&](int a, int b, int c) { return S[a + ncx * (b + ncy * c)]; };
    // the edge from (I, J, K) along +x lies in cells (I, J - 1 .. J, K - 1 .. K); along -x in
    // cells (I - 1, ...); the cell that holds it as its (y, z) = (0, 0) or (1, 1) edge counts twice
    const double ax = hy * hz / (6.0 * hx), ay = hx * hz / (6.0 * hy), az = hx * hy / (6.0 * hz);
    const double xp = ax * (2.0 * kc(I, J - 1, K - 1) + 2.0 * kc(I, J, K) + kc(I, J - 1, K) + kc(I, J, K - 1));
    const double xm = ax * (2.0 * kc(I - 1, J - 1, K - 1) + 2.0 * kc(I - 1, J, K) + kc(I - 1, J - 1, K) +
                            kc(I - 1, J, K - 1));
    const double yp = ay * (2.0 * kc(I - 1, J, K - 1) + 2.0 * kc(I, J, K) + kc(I, J, K - 1) + kc(I - 1, J, K));
    const double ym = ay * (2.0 * kc(I - 1, J - 1, K - 1) + 2.0 * kc(I, J - 1, K) + kc(I, J - 1, K - 1) +
                            kc(I - 1, J - 1, K));
    const double zp = az * (2.0 * kc(I - 1, J - 1, K) + 2.0 * kc(I, J, K) + kc(I - 1, J, K) + kc(I, J - 1, K));
    const double zm = az * (2.0 * kc(I - 1, J - 1, K - 1) + 2.0 * kc(I, J, K - 1) + kc(I - 1, J, K - 1) +
                            kc(I, J - 1, K - 1));
    const size_t n = N;
    out[i] = x + 1 < nvx ? xp : 0.0;
    out[n + i] = y + 1 < nvy ? yp : 0.0;
    out[2 * n + i] = z + 1 < nvz ? zp : 0.0;
    walls[i] = (x == 0 ? xm : 0.0) + (x + 1 == nvx ? xp : 0.0);
    walls[n + i] = (y == 0 ? ym : 0.0) + (y + 1 == nvy ? yp : 0.0);
    walls[2 * n + i] = (z == 0 ? zm : 0.0) + (z + 1 == nvz ? zp : 0.0);
    const double six = sc(I, J, K) + sc(I - 1, J - 1, K - 1);
    const double two = sc(I - 1, J, K) + sc(I, J - 1, K) + sc(I, J, K - 1) + sc(I - 1, J - 1, K) +
                       sc(I - 1, J, K - 1) + sc(I, J - 1, K - 1);
    out[4 * n + i] = hx * hy * hz / 24.0 * (6.0 * six + 2.0 * two);
}

__global__ void k_finish_diag(double* __restrict__ c, const double* __restrict__ w, int nx, int ny, int nz) {
    const int N = nx * ny * nz;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
    double d = w[i] + w[(size_t)N + i] + w[(size_t)2 * N + i];
    d += c[i] + (x > 0 ? c[i - 1] : 0.0);
    d += c[(size_t)N + i] + (y > 0 ? c[(size_t)N + i - nx] : 0.0);
    d += c[(size_t)2 * N + i] + (z > 0 ? c[(size_t)2 * N + i - nx * ny] : 0.0);
    c[(size_t)3 * N + i] = d;
}

template <typename S, typename D>
__global__ void k_convert(const S* __restrict__ in, D* __restrict__ out, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (D)in[i];
}

template <typename S, typename D>
int convert_vectors(hipStream_t st, const S* in, D* out, size_t count) {
    if (count == 0) return 0;
    k_convert<S, D><<<(unsigned)((count + kBlock - 1) / kBlock), kBlock, 0, st>>>(in, out, count);
    LT_HIP(hipGetLastError());
    return 0;
}
template <typename S, typename D>
__global__ void k_convert_cp(const S* __restrict__ in, D* __restrict__ out, int N, int nx, int ny, int dir) {
    const size_t plane = blockIdx.y;  // vector * 2 + (re, im)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int X = i % nx, Y = (i / nx) % ny, Z = i / (nx * ny);
    const int p = cp_at(i, X, Y, Z, N);
    const size_t base = plane * N;
    if (dir == 0)
        out[base + p] = (D)in[base + i];
    else
        out[base + i] = (D)in[base + p];
}

template <typename S, typename D>
int convert_vectors_cp(hipStream_t st, const S* in, D* out, int nvec, int N, int cpnx, int cpny, int dir) {
    if (!cpnx) return convert_vectors<S, D>(st, in, out, 2 * (size_t)N * nvec);
    k_convert_cp<S, D><<<dim3((unsigned)((N + kBlock - 1) / kBlock), 2 * nvec), kBlock, 0, st>>>(in, out, N, cpnx, cpny, dir);
    LT_HIP(hipGetLastError());
    return 0;
}
template int convert_vectors_cp<double, float>(hipStream_t, const double*, float*, int, int, int, int, int);
template int convert_vectors_cp<float, double>(hipStream_t, const float*, double*, int, int, int, int, int);
template int convert_vectors_cp<double, double>(hipStream_t, const double*, double*, int, int, int, int, int);

template int convert_vectors<double, float>(hipStream_t, const double*, float*, size_t);
template int convert_vectors<float, double>(hipStream_t, const float*, double*, size_t);
template int convert_vectors<double, double>(hipStream_t, const double*, double*, size_t);
template int convert_vectors<float, float>(hipStream_t, const float*, float*, size_t);

// ------------------------------------------------------------------ smoothing and transfers
// y = (K + tau M) x for R vectors [R][2][N].
template <typename T>
__global__ void k_apply(LevelView<T> L, T tr, T ti, const T* __restrict__ x, T* __restrict__ y,
                        const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.N) return;
    const size_t N = L.N;
    const T* xr = x + 2 * N * r;
    const T* xi = xr + N;
    int X = i % L.nx, Y = (i / L.nx) % L.ny, Z = i / (L.nx * L.ny);
    cpx<T> off = offsum(L, xr, xi, i, X, Y, Z);
    cpx<T> d = {L.D[i] + tr * L.m[i], ti * L.m[i]};
    cpx<T> xv = {xr[i], xi[i]};
    cpx<T> dx = cmul(d, xv);
    y[2 * N * r + i] = dx.re - off.re;
    y[2 * N * r + N + i] = dx.im - off.im;
}

// One colour of red-black Gauss-Seidel (colour = parity of x + y + z).
template <typename T>
__global__ void k_gs_color(LevelView<T> L, T tr, T ti, int color, T* __restrict__ x,
                           const T* __restrict__ b, const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.N) return;
    int X = i % L.nx, Y = (i / L.nx) % L.ny, Z = i / (L.nx * L.ny);
    if (((X + Y + Z) & 1) != color) return;
    const size_t N = L.N;
    T* xr = x + 2 * N * r;
    T* xi = xr + N;
    const T* br = b + 2 * N * r;
    cpx<T> off = offsum(L, xr, xi, i, X, Y, Z);
    cpx<T> num = {br[i] + off.re, br[i + N] + off.im};
    cpx<T> d = {L.D[i] + tr * L.m[i], ti * L.m[i]};
    cpx<T> v = cdiv(num, d);
    xr[i] = v.re;
    xi[i] = v.im;
}

// The list of active right-hand sides that group_rhs reads, from R <= 1024 flags: one workgroup of 1024 threads, one flag per
// thread; positions from the wave's ballot and the counts of the waves before it.
__global__ void __launch_bounds__(1024) k_active_list(const int* __restrict__ active, int R, int* __restrict__ list) {
    __shared__ int wcount[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool on = t < R && active[t] != 0;
    const unsigned long long m = __ballot(on ? 1 : 0);
    if (lane == 0) wcount[w] = __popcll(m);
    __syncthreads();
    int base = 0, total = 0;
    for (int k = 0; k < 16; ++k) {
        base += k < w ? wcount[k] : 0;
        total += wcount[k];
    }
    if (on) list[1 + base + __popcll(m & ((1ull << lane) - 1ull))] = t;
    if (t == 0) list[0] = total;
}

// The same half-sweep with one thread per cell of the colour (nx even): thread k takes
// the k-th cell of that colour in storage order, so no lane idles.  A thread serves its
// cell for the RB right-hand sides of its group (group_rhs): the coefficients are loaded
// once and reused (they are shared by every right-hand side), and the RB updates are
// independent.  prof: per launch, prof_once bytes plus prof_bytes per right-hand side served.
template <typename T, int RB, bool CP>
__global__ void k_gs_color_half(LevelView<T> L, T tr, T ti, int color, T* __restrict__ x,
                                const T* __restrict__ b, const int* __restrict__ list, int R,
                                unsigned long long* __restrict__ prof, unsigned long long prof_bytes,
                                unsigned long long prof_once) {
    int rs[RB];
    group_rhs<RB>(list, R, blockIdx.y, rs);
    if (rs[0] < 0) return;
    if (prof && blockIdx.x == 0 && threadIdx.x == 0) {
        unsigned long long add = blockIdx.y == 0 ? prof_once : 0ull;
#pragma unroll
        for (int q = 0; q < RB; ++q) add += rs[q] >= 0 ? prof_bytes : 0ull;
        atomicAdd(prof, add);
    }
    const int W = L.nx >> 1;
    const int k = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (k >= (L.N >> 1)) return;
    const int row = k / W;  // y + ny z
    const int Y = row % L.ny, Z = row / L.ny;
    const int X = 2 * (k - row * W) + ((Y + Z + color) & 1);
    const int i = X + L.nx * row;
    const int sy = L.nx, sz = L.nx * L.ny;
    // neighbours in offsum's order (+x, -x, +y, -y, +z, -z); a missing one has coupling 0
    // and reads the cell itself
    const bool hx = X + 1 < L.nx, lx = X > 0, hy = Y + 1 < L.ny, ly = Y > 0, hz = Z + 1 < L.nz, lz = Z > 0;
    const int nb[6] = {hx ? i + 1 : i, lx ? i - 1 : i, hy ? i + sy : i, ly ? i - sy : i, hz ? i + sz : i,
                       lz ? i - sz : i};
    const T tc[6] = {hx ? L.Tx[i] : T(0), lx ? L.Tx[i - 1] : T(0), hy ? L.Ty[i] : T(0),
                     ly ? L.Ty[i - sy] : T(0), hz ? L.Tz[i] : T(0), lz ? L.Tz[i - sz] : T(0)};
    const cpx<T> d = {L.D[i] + tr * L.m[i], ti * L.m[i]};
    const size_t N = L.N;
    // positions in the vectors: this cell and its neighbours (all of the other colour; a
    // missing neighbour's position is a valid cell read with coupling 0)
    const int half = L.N >> 1;
    const int own = CP ? color * half + k : i;
    int np[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) np[a] = CP ? (1 - color) * half + (nb[a] >> 1) : nb[a];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int r = rs[q];
        if (r < 0) continue;
        T* xr = x + 2 * N * r;
        T* xi = xr + N;
        const T* br = b + 2 * N * r;
        cpx<T> off = {0, 0};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            off.re += tc[a] * xr[np[a]];
            off.im += tc[a] * xi[np[a]];
        }
        const cpx<T> num = {br[own] + off.re, br[own + N] + off.im};
        const cpx<T> v = cdiv(num, d);
        xr[own] = v.re;
        xi[own] = v.im;
    }
}

// prof (fine level, opts.profile = LT_PROF_SWEEP3D): every launch bracketed by HIP events
// on the stream and its algorithmic bytes counted: per active right-hand side, b of the
// colour's cells in, x of the other colour in, x of the colour out (complex: 12 bytes of T
// per cell in FP32 terms, 3 sizeof(T) per cell), plus, once per launch, the coefficients
// Tx, Ty, Tz of every cell and D, m of the colour's cells (4 sizeof(T) per cell).
// list: the active right-hand sides (group_rhs), or null for all R; active: their flags,
// for the one-thread-per-cell fallback of odd nx.
constexpr int kHalfSweepRhs = 8;  // right-hand sides per thread of a one-colour half-sweep

template <typename T>
static int gs_half_sweep(lt_handle* h, hipStream_t st, const LevelView<T>& L, T tr, T ti, int color, T* x,
                         const T* b, int R, const int* active, const int* list, bool fine, bool cp = false) {
    if ((L.nx & 1) == 0) {
        const dim3 grid((unsigned)((L.N / 2 + 255) / 256), (R + kHalfSweepRhs - 1) / kHalfSweepRhs);
        if (fine && h->prof_target == LT_PROF_SWEEP3D) {
            unsigned long long* pc = nullptr;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            LT_TRY(prof_begin(h, LT_PROF_SWEEP3D, &pc, &e0, &e1));
            const unsigned long long per = (unsigned long long)L.N * 3ull * sizeof(T);
            const unsigned long long once = (unsigned long long)L.N * 4ull * sizeof(T);
            if (cp)
                hipExtLaunchKernelGGL((k_gs_color_half<T, kHalfSweepRhs, true>), grid, dim3(256), 0, st, e0, e1, 0, L, tr,
                                      ti, color, x, b, list, R, pc, per, once);
            else
                hipExtLaunchKernelGGL((k_gs_color_half<T, kHalfSweepRhs, false>), grid, dim3(256), 0, st, e0, e1, 0, L, tr,
                                      ti, color, x, b, list, R, pc, per, once);
            LT_TRY(prof_end(h, LT_PROF_SWEEP3D));
        } else if (cp) {
            k_gs_color_half<T, kHalfSweepRhs, true><<<grid, 256, 0, st>>>(L, tr, ti, color, x, b, list, R, nullptr,
                                                                      0ull, 0ull);
        } else {
            k_gs_color_half<T, kHalfSweepRhs, false><<<grid, 256, 0, st>>>(L, tr, ti, color, x, b, list, R, nullptr,
                                                                       0ull, 0ull);
        }
    } else {
        k_gs_color<T><<<dim3((unsigned)((L.N + 255) / 256), R), 256, 0, st>>>(L, tr, ti, color, x, b, active);
    }
    LT_HIP(hipGetLastError());
    return 0;
}

// Coarse right-hand side = sum over the aggregate of the fine residual b - A x;
// the coarse iterate is cleared.  A thread serves its coarse cell for the RB right-hand
// sides of its group (group_rhs; the coefficients of the aggregate are loaded once).
template <typename T, int RB>
__global__ void k_resid_restrict(LevelView<T> F, int cnx, int cny, int cnz, int cox, int coy, int coz,
                                 T tr, T ti, const T* __restrict__ xf, const T* __restrict__ bf,
                                 T* __restrict__ bc, T* __restrict__ xc, const int* __restrict__ list, int R,
                                 int cpf, int cpc) {
    int rs[RB];
    group_rhs<RB>(list, R, blockIdx.y, rs);
    if (rs[0] < 0) return;
    const int Nc = cnx * cny * cnz;
    int I = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (I >= Nc) return;
    int Xc = I % cnx, Yc = (I / cnx) % cny, Zc = I / (cnx * cny);
    const size_t N = F.N;
    int x0 = cox ? 2 * Xc : Xc, x1 = cox ? 2 * Xc + 1 : Xc;
    int y0 = coy ? 2 * Yc : Yc, y1 = coy ? 2 * Yc + 1 : Yc;
    int z0 = coz ? 2 * Zc : Zc, z1 = coz ? 2 * Zc + 1 : Zc;
    cpx<T> acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = {0, 0};
    const int sy = F.nx, sz = F.nx * F.ny;
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const int i = x + F.nx * (y + F.ny * z);
                // neighbours in offsum's order; a missing one has coupling 0 and reads the cell
                const bool hx = x + 1 < F.nx, lx = x > 0, hy = y + 1 < F.ny, ly = y > 0, hz = z + 1 < F.nz,
                           lz = z > 0;
                const int nb[6] = {hx ? i + 1 : i, lx ? i - 1 : i, hy ? i + sy : i, ly ? i - sy : i,
                                   hz ? i + sz : i, lz ? i - sz : i};
                const T tc[6] = {hx ? F.Tx[i] : T(0), lx ? F.Tx[i - 1] : T(0), hy ? F.Ty[i] : T(0),
                                 ly ? F.Ty[i - sy] : T(0), hz ? F.Tz[i] : T(0), lz ? F.Tz[i - sz] : T(0)};
                const cpx<T> d = {F.D[i] + tr * F.m[i], ti * F.m[i]};
                // positions in the fine vectors (colour-planar: the neighbours have the other colour)
                const int c = (x + y + z) & 1, half = F.N >> 1;
                const int own = cpf ? c * half + (i >> 1) : i;
                int np[6];
#pragma unroll
                for (int a = 0; a < 6; ++a) np[a] = cpf ? (1 - c) * half + (nb[a] >> 1) : nb[a];
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    const int r = rs[q];
                    if (r < 0) continue;
                    const T* xr = xf + 2 * N * r;
                    const T* xi = xr + N;
                    const T* br = bf + 2 * N * r;
                    const T* bi = br + N;
                    cpx<T> off = {0, 0};
#pragma unroll
                    for (int a = 0; a < 6; ++a) {
                        off.re += tc[a] * xr[np[a]];
                        off.im += tc[a] * xi[np[a]];
                    }
                    const cpx<T> ax = cmul(d, cpx<T>{xr[own], xi[own]});
                    acc[q].re += br[own] - (ax.re - off.re);
                    acc[q].im += bi[own] - (ax.im - off.im);
                }
            }
    const size_t M = Nc;
    const int Ic = cpc ? cp_at(I, Xc, Yc, Zc, Nc) : I;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int r = rs[q];
        if (r < 0) continue;
        bc[2 * M * r + Ic] = acc[q].re;
        bc[2 * M * r + M + Ic] = acc[q].im;
        xc[2 * M * r + Ic] = 0;
        xc[2 * M * r + M + Ic] = 0;
    }
}

// x_fine += P e_coarse for the RB right-hand sides of a group (group_rhs).  A thread takes one
// position of the fine vectors (colour-planar when cpf) and forms the interpolation's taps
// once for the group: two per halved axis, an absent one with weight 0 at a valid index, so
// the eight loads of a right-hand side issue without a data-dependent loop.  c0only: colour-0
// cells only (positions below N/2 when cpf), for a post-smoother that starts with colour 1:
// that half-sweep sets every colour-1 cell from its colour-0 neighbours without reading it.
template <typename T, int RB>
__global__ void k_prolong_rb(int fnx, int fny, int fnz, int cnx, int cny, int cnz, int cox, int coy, int coz,
                             T glox, T ghix, T gloy, T ghiy, T gloz, T ghiz, const T* __restrict__ ec,
                             T* __restrict__ xf, const int* __restrict__ list, int R, int cpf, int cpc, int c0only) {
    int rs[RB];
    group_rhs<RB>(list, R, blockIdx.y, rs);
    if (rs[0] < 0) return;
    const int Nf = fnx * fny * fnz;
    const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;  // position in the fine vectors
    if (p >= ((c0only && cpf) ? (Nf >> 1) : Nf)) return;
    int c3[3];
    if (cpf) {
        const int half = Nf >> 1, c = p >= half ? 1 : 0, k = p - c * half, W = fnx >> 1;
        const int row = k / W;
        c3[1] = row % fny;
        c3[2] = row / fny;
        c3[0] = 2 * (k - row * W) + ((c3[1] + c3[2] + c) & 1);
    } else {
        c3[0] = p % fnx;
        c3[1] = (p / fnx) % fny;
        c3[2] = p / (fnx * fny);
        if (c0only && ((c3[0] + c3[1] + c3[2]) & 1)) return;
    }
    const int co[3] = {cox, coy, coz};
    const int cn[3] = {cnx, cny, cnz};
    const T glo[3] = {glox, gloy, gloz};
    const T ghi[3] = {ghix, ghiy, ghiz};
    int ia[3][2];
    T wa[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!co[a]) {
            ia[a][0] = ia[a][1] = c3[a];
            wa[a][0] = T(1);
            wa[a][1] = T(0);
            continue;
        }
        // cell-centred linear interpolation: 3/4 of the parent, 1/4 of its neighbour on the
        // child's side; beyond a wall the ghost mirrors the parent with parity glo / ghi
        const int I = c3[a] >> 1, J = (c3[a] & 1) ? I + 1 : I - 1;
        ia[a][0] = I;
        if (J < 0 || J >= cn[a]) {
            ia[a][1] = I;
            wa[a][0] = T(0.75) + T(0.25) * (J < 0 ? glo[a] : ghi[a]);
            wa[a][1] = T(0);
        } else {
            ia[a][1] = J;
            wa[a][0] = T(0.75);
            wa[a][1] = T(0.25);
        }
    }
    const int Mc = cnx * cny * cnz;
    int J[8];
    T W[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int a = t & 1, b = (t >> 1) & 1, c = t >> 2;
        W[t] = wa[0][a] * wa[1][b] * wa[2][c];
        const int idx = ia[0][a] + cnx * (ia[1][b] + cny * ia[2][c]);
        J[t] = cpc ? cp_at(idx, ia[0][a], ia[1][b], ia[2][c], Mc) : idx;
    }
    const size_t Nfs = Nf;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int r = rs[q];
        if (r < 0) continue;
        const T* er = ec + 2 * (size_t)Mc * r;
        const T* ei = er + Mc;
        cpx<T> acc = {0, 0};
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            acc.re += W[t] * er[J[t]];
            acc.im += W[t] * ei[J[t]];
        }
        xf[2 * Nfs * r + p] += acc.re;
        xf[2 * Nfs * r + Nfs + p] += acc.im;
    }
}

// The first half-sweep of red-black Gauss-Seidel from x = 0: colour-0 cells see only
// zero neighbours and take b / d, colour-1 cells stay 0.  Replaces clearing x and the
// first sweep of colour 0.  The RB right-hand sides of a group (group_rhs) per thread
// (D and m loaded once).
template <typename T, int RB>
__global__ void k_gs_first(LevelView<T> L, T tr, T ti, T* __restrict__ x, const T* __restrict__ b,
                           const int* __restrict__ list, int R, int cp) {
    int rs[RB];
    group_rhs<RB>(list, R, blockIdx.y, rs);
    if (rs[0] < 0) return;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;  // position in the vectors
    if (p >= L.N) return;
    int i = p, c0 = 0;
    if (cp) {
        // the cell at colour-planar position p
        const int half = L.N >> 1, c = p >= half ? 1 : 0, k = p - c * half, W = L.nx >> 1;
        const int row = k / W, Y = row % L.ny, Z = row / L.ny;
        i = 2 * (k - row * W) + ((Y + Z + c) & 1) + L.nx * row;
        c0 = c == 0;
    } else {
        const int X = i % L.nx, Y = (i / L.nx) % L.ny, Z = i / (L.nx * L.ny);
        c0 = ((X + Y + Z) & 1) == 0;
    }
    const cpx<T> d = {L.D[i] + tr * L.m[i], ti * L.m[i]};
    const size_t N = L.N;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int r = rs[q];
        if (r < 0) continue;
        T* xr = x + 2 * N * r;
        T* xi = xr + N;
        if (c0) {
            const T* br = b + 2 * N * r;
            const cpx<T> v = cdiv(cpx<T>{br[p], br[p + N]}, d);
            xr[p] = v.re;
            xi[p] = v.im;
        } else {
            xr[p] = 0;
            xi[p] = 0;
        }
    }
}

// x = Ainv b on the coarsest level (Ainv interleaved complex, row-major).
template <typename T>
__global__ void k_coarse_solve(int Nc, const T* __restrict__ inv, const T* __restrict__ b, T* __restrict__ x,
                               const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nc) return;
    const T* br = b + (size_t)2 * Nc * r;
    const T* bi = br + Nc;
    cpx<T> acc = {0, 0};
    const T* row = inv + (size_t)2 * Nc * i;
    for (int j = 0; j < Nc; ++j) {
        cpx<T> a = {row[2 * j], row[2 * j + 1]};
        cpx<T> v = {br[j], bi[j]};
        cpx<T> p = cmul(a, v);
        acc.re += p.re;
        acc.im += p.im;
    }
    x[(size_t)2 * Nc * r + i] = acc.re;
    x[(size_t)2 * Nc * r + Nc + i] = acc.im;
}

template <typename T>
__global__ void k_zero(T* __restrict__ x, size_t per, const int* __restrict__ active) {
    int r = blockIdx.y;
    if (active && !active[r]) return;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < per) x[per * r + i] = 0;
}

// ------------------------------------------------------------------ host side
static inline unsigned nblk(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int mg_build(lt_handle* h, const double* kappa, const double* S, const lt_grid* p1_cells) {
    const lt_grid& g = h->grid;
    hipStream_t st = h->stream;
    std::vector<Level>& lv = h->levels;
    lv.clear();
    Level f;
    for (int a = 0; a < 3; ++a) {
        f.n[a] = g.n[a];
        f.h[a] = g.h[a];
        f.coarsened_from_fine[a] = 0;
    }
    f.N = g.n[0] * g.n[1] * g.n[2];
    if (p1_cells)  // vertices: the walls lie one spacing out
        for (int a = 0; a < p1_cells->ndim; ++a) f.delta[a] = 1.0;
    lv.push_back(f);
    DevBuf walls_f, walls_c;
    LT_TRY(lv[0].c64.reserve(sizeof(double) * 5 * (size_t)f.N));
    LT_TRY(walls_f.reserve(sizeof(double) * 3 * (size_t)f.N));
    int4 lo = {h->bc.face[0], h->bc.face[2], h->bc.face[4], 0};
    int4 hi = {h->bc.face[1], h->bc.face[3], h->bc.face[5], 0};
    double* mstor = nullptr;
    if (h->bc.sy > 0.0) {
        LT_TRY(h->mstor.reserve(sizeof(double) * (size_t)f.N));
        mstor = h->mstor.as<double>();
    }
    if (p1_cells && p1_cells->ndim == 3)
        k_p1_assemble3d<<<nblk(f.N), kBlock, 0, st>>>(kappa, S, p1_cells->n[0], p1_cells->n[1], p1_cells->n[2],
                                                      p1_cells->h[0], p1_cells->h[1], p1_cells->h[2],
                                                      lv[0].c64.as<double>(), walls_f.as<double>());
    else if (p1_cells)
        k_p1_assemble<<<nblk(f.N), kBlock, 0, st>>>(kappa, S, p1_cells->n[0], p1_cells->n[1], p1_cells->h[0],
                                                    p1_cells->h[1], lv[0].c64.as<double>(), walls_f.as<double>());
    else
        k_fine_assemble<<<nblk(f.N), kBlock, 0, st>>>(kappa, S, f.n[0], f.n[1], f.n[2], g.ndim, f.h[0], f.h[1],
                                                       f.h[2], lo, hi, h->bc.sy, lv[0].c64.as<double>(),
                                                       walls_f.as<double>(), mstor);
    LT_HIP(hipGetLastError());
    k_finish_diag<<<nblk(f.N), kBlock, 0, st>>>(lv[0].c64.as<double>(), walls_f.as<double>(), f.n[0], f.n[1],
                                                f.n[2]);
    LT_HIP(hipGetLastError());
    // coarsen while useful
    while (true) {
        const Level& L = lv.back();
        if (L.N <= 64) break;
        double hmin = 1e300;
        for (int a = 0; a < g.ndim; ++a) hmin = std::min(hmin, L.h[a]);
        int co[3] = {0, 0, 0};
        bool any = false;
        for (int a = 0; a < g.ndim; ++a) {
            if (L.n[a] % 2 == 0 && L.n[a] > 2 && L.h[a] < 1.5 * hmin) {
                co[a] = 1;
                any = true;
            }
        }
        if (!any) break;
        Level C;
        double ws[3];
        for (int a = 0; a < 3; ++a) {
            C.n[a] = co[a] ? L.n[a] / 2 : L.n[a];
            C.h[a] = co[a] ? L.h[a] * 2 : L.h[a];
            C.coarsened_from_fine[a] = co[a];
            C.delta[a] = co[a] ? 0.5 * L.delta[a] + 0.25 : L.delta[a];
            // a wall term is kappa A / (delta h): the aggregation's rule holds it for delta = 1/2
            ws[a] = co[a] ? L.delta[a] / C.delta[a] : 1.0;
        }
        C.N = C.n[0] * C.n[1] * C.n[2];
        LT_TRY(C.c64.reserve(sizeof(double) * 5 * (size_t)C.N));
        LT_TRY(walls_c.reserve(sizeof(double) * 3 * (size_t)C.N));
        k_coarsen<<<nblk(C.N), kBlock, 0, st>>>(L.c64.as<double>(), walls_f.as<double>(), L.n[0], L.n[1],
                                                L.n[2], C.n[0], C.n[1], C.n[2], co[0], co[1], co[2],
                                                C.c64.as<double>(), walls_c.as<double>(),
                                                make_double3(ws[0], ws[1], ws[2]));
        LT_HIP(hipGetLastError());
        k_finish_diag<<<nblk(C.N), kBlock, 0, st>>>(C.c64.as<double>(), walls_c.as<double>(), C.n[0], C.n[1],
                                                    C.n[2]);
        LT_HIP(hipGetLastError());
        std::swap(walls_f, walls_c);
        lv.push_back(C);
        // keep the DevBufs owned by the vector (C's buffer pointer moved by copy)
        lv.back().c64 = C.c64;
        C.c64.p = nullptr;
    }
    for (Level& L : lv) {
        LT_TRY(L.c32.reserve(sizeof(float) * 5 * (size_t)L.N));
        LT_TRY(convert_vectors<double, float>(st, L.c64.as<double>(), L.c32.as<float>(), 5 * (size_t)L.N));
    }
    {
        // mean of ln D on the fine grid (features of the learned preconditioner)
        std::vector<double> D(f.N);
        LT_HIP(hipMemcpyAsync(D.data(), lv[0].c64.as<double>() + 3 * (size_t)f.N, sizeof(double) * f.N,
                              hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        double s = 0;
        for (double d : D) s += std::log(d);
        h->lnDbar = s / f.N;
    }
    // colour-planar V-cycle vectors for 3D grids whose levels above the single-workgroup ones
    // (those with more than kCoarseBlockCells cells, at most kMaxCBLevels below them) all
    // have an even number of cells along x
    {
        const int nl = (int)lv.size();
        int lc = nl;
        for (int l = 0; l < nl; ++l)
            if (lv[l].N <= kCoarseBlockCells) { lc = l; break; }
        bool ok = h->grid.ndim == 3 && lc > 0 && lc < nl && nl - lc <= kMaxCBLevels;
        for (int l = 0; l < lc && ok; ++l) ok = (lv[l].n[0] % 2) == 0;
        h->cp3d = ok;
    }
    // coarsest coefficients on the host for the dense coarse solve
    const Level& Lc = lv.back();
    h->coarse_host.resize(5 * (size_t)Lc.N);
    LT_HIP(hipMemcpyAsync(h->coarse_host.data(), Lc.c64.p, sizeof(double) * 5 * Lc.N, hipMemcpyDeviceToHost, st));
    LT_HIP(hipStreamSynchronize(st));
    walls_f.release();
    walls_c.release();
    return 0;
}

// Dense inverse of the coarsest level's K + tau M by Gauss-Jordan elimination with
// partial pivoting, in one workgroup on a working matrix [A | I] (n x 2n complex) in
// global memory; writes the inverse row-major as interleaved complex FP64 and FP32.
// The allocation-free path builds the coarse solve this way in its scratch; a singular
// pivot leaves NaN in the inverse.
__global__ __launch_bounds__(1024) void k_coarse_gj(LevelView<double> L, double tr, double ti, int n,
                                                    cpx<double>* __restrict__ Mw, double* __restrict__ inv64,
                                                    float* __restrict__ inv32) {
    __shared__ cpx<double> fac[kMaxCoarseDense];
    __shared__ double pv[1024];
    __shared__ int pix[1024];
    const int tid = threadIdx.x, nt = blockDim.x, w = 2 * n;
    const int sy = L.nx, sz = L.nx * L.ny;
    for (int e = tid; e < n * w; e += nt) {
        const int i = e / w, j = e % w;
        cpx<double> v = {0.0, 0.0};
        if (j < n) {
            const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / sz;
            if (j == i) v = {L.D[i] + tr * L.m[i], ti * L.m[i]};
            else if (x + 1 < L.nx && j == i + 1) v.re = -L.Tx[i];
            else if (x > 0 && j == i - 1) v.re = -L.Tx[i - 1];
            else if (y + 1 < L.ny && j == i + sy) v.re = -L.Ty[i];
            else if (y > 0 && j == i - sy) v.re = -L.Ty[i - sy];
            else if (z + 1 < L.nz && j == i + sz) v.re = -L.Tz[i];
            else if (z > 0 && j == i - sz) v.re = -L.Tz[i - sz];
        } else if (j - n == i) {
            v.re = 1.0;
        }
        Mw[e] = v;
    }
    __syncthreads();
    bool singular = false;
    for (int c = 0; c < n && !singular; ++c) {
        double best = -1.0;
        int bi = c;
        for (int r = c + tid; r < n; r += nt) {
            const cpx<double> v = Mw[(size_t)r * w + c];
            const double a = v.re * v.re + v.im * v.im;
            if (a > best) { best = a; bi = r; }
        }
        pv[tid] = best;
        pix[tid] = bi;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s && (pv[tid + s] > pv[tid] || (pv[tid + s] == pv[tid] && pix[tid + s] < pix[tid]))) {
                pv[tid] = pv[tid + s];
                pix[tid] = pix[tid + s];
            }
            __syncthreads();
        }
        const int pr = pix[0];
        singular = !(pv[0] > 0.0);
        if (singular) break;  // uniform: every thread read the same pv[0]
        if (pr != c)
            for (int j = tid; j < w; j += nt) {
                const cpx<double> a = Mw[(size_t)c * w + j];
                Mw[(size_t)c * w + j] = Mw[(size_t)pr * w + j];
                Mw[(size_t)pr * w + j] = a;
            }
        __syncthreads();
        const cpx<double> piv = Mw[(size_t)c * w + c];
        __syncthreads();
        const double d = piv.re * piv.re + piv.im * piv.im;
        const cpx<double> ip = {piv.re / d, -piv.im / d};
        for (int j = tid; j < w; j += nt) Mw[(size_t)c * w + j] = cmul(Mw[(size_t)c * w + j], ip);
        for (int r = tid; r < n; r += nt) fac[r] = Mw[(size_t)r * w + c];
        __syncthreads();
        for (int e = tid; e < n * w; e += nt) {
            const int r = e / w, j = e % w;
            if (r == c) continue;
            const cpx<double> f = fac[r], a = Mw[(size_t)c * w + j];
            cpx<double>& t = Mw[e];
            t.re -= f.re * a.re - f.im * a.im;
            t.im -= f.re * a.im + f.im * a.re;
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += nt) {
        const int i = e / n, j = e % n;
        const cpx<double> v = singular ? cpx<double>{NAN, NAN} : Mw[(size_t)i * w + n + j];
        inv64[2 * (size_t)e] = v.re;
        inv64[2 * (size_t)e + 1] = v.im;
        inv32[2 * (size_t)e] = (float)v.re;
        inv32[2 * (size_t)e + 1] = (float)v.im;
    }
}

// The coarse inverse of an allocation-free call, built on the GPU in the arena.
static const CoarseInverse* arena_coarse_inverse(lt_handle* h, cdouble tau, int* rc) {
    const Level& L = h->levels.back();
    const int n = L.N;
    if (n > kMaxCoarseDense) return nullptr;
    cpx<double>* Mw = wsp<cpx<double>>(h, "gj_work", 2 * (size_t)n * n, rc);
    double* i64 = wsp<double>(h, "gj_inv64", 2 * (size_t)n * n, rc);
    float* i32 = wsp<float>(h, "gj_inv32", 2 * (size_t)n * n, rc);
    if (!Mw || !i64 || !i32) return nullptr;
    h->arena_ci.tau = tau;
    h->arena_ci.inv64.p = i64;
    h->arena_ci.inv64.bytes = 2 * (size_t)n * n * sizeof(double);
    h->arena_ci.inv32.p = i32;
    h->arena_ci.inv32.bytes = 2 * (size_t)n * n * sizeof(float);
    if (!h->arena_plan) {
        k_coarse_gj<<<1, 1024, 0, h->stream>>>(L.v64(), tau.real(), tau.imag(), n, Mw, i64, i32);
        if (hipGetLastError() != hipSuccess) {
            *rc = LT_EHIP;
            set_last_error("coarse inverse kernel launch failed");
            return nullptr;
        }
    }
    return &h->arena_ci;
}

const CoarseInverse* mg_coarse_inverse(lt_handle* h, cdouble tau, int* rc) {
    *rc = 0;
    if (h->arena || h->arena_plan) return arena_coarse_inverse(h, tau, rc);
    for (const CoarseInverse& c : h->coarse_cache)
        if (c.tau == tau) return &c;
    const Level& L = h->levels.back();
    const int n = L.N;
    if (n > kMaxCoarseDense) { *rc = 0; return nullptr; }
    const double* c = h->coarse_host.data();
    const double *Tx = c, *Ty = c + n, *Tz = c + 2 * n, *D = c + 3 * n, *m = c + 4 * n;
    std::vector<cdouble> A((size_t)n * n, 0.0), inv;
    const int nx = L.n[0], ny = L.n[1];
    for (int i = 0; i < n; ++i) {
        int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        A[(size_t)i * n + i] = D[i] + tau * m[i];
        if (x + 1 < L.n[0]) A[(size_t)i * n + i + 1] = -Tx[i];
        if (x > 0) A[(size_t)i * n + i - 1] = -Tx[i - 1];
        if (y + 1 < L.n[1]) A[(size_t)i * n + i + nx] = -Ty[i];
        if (y > 0) A[(size_t)i * n + i - nx] = -Ty[i - nx];
        if (z + 1 < L.n[2]) A[(size_t)i * n + i + nx * ny] = -Tz[i];
        if (z > 0) A[(size_t)i * n + i - nx * ny] = -Tz[i - nx * ny];
    }
    if (dense_inverse(n, A, inv) != 0) { *rc = LT_EINVAL; set_last_error("singular coarse operator"); return nullptr; }
    if (h->coarse_cache.size() >= 16) {
        ++h->ws_gen;
        h->coarse_cache.front().inv64.release();
        h->coarse_cache.front().inv32.release();
        h->coarse_cache.erase(h->coarse_cache.begin());
    }
    h->coarse_cache.emplace_back();
    CoarseInverse& ci = h->coarse_cache.back();
    ci.tau = tau;
    std::vector<double> d64(2 * (size_t)n * n);
    std::vector<float> d32(2 * (size_t)n * n);
    for (size_t k = 0; k < (size_t)n * n; ++k) {
        d64[2 * k] = inv[k].real();
        d64[2 * k + 1] = inv[k].imag();
        d32[2 * k] = (float)inv[k].real();
        d32[2 * k + 1] = (float)inv[k].imag();
    }
    if ((*rc = ci.inv64.reserve(d64.size() * sizeof(double))) < 0) return nullptr;
    if ((*rc = ci.inv32.reserve(d32.size() * sizeof(float))) < 0) return nullptr;
    if (hipMemcpyAsync(ci.inv64.p, d64.data(), d64.size() * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(ci.inv32.p, d32.data(), d32.size() * sizeof(float), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        *rc = LT_EHIP;
        set_last_error("coarse inverse upload failed");
        return nullptr;
    }
    return &ci;
}

template <typename T> static LevelView<T> view(const Level& L);
template <> LevelView<double> view<double>(const Level& L) { return L.v64(); }
template <> LevelView<float> view<float>(const Level& L) { return L.v32(); }
template <typename T> static const T* inv_ptr(const CoarseInverse* c);
template <> const double* inv_ptr<double>(const CoarseInverse* c) { return c->inv64.as<double>(); }
template <> const float* inv_ptr<float>(const CoarseInverse* c) { return c->inv32.as<float>(); }

template <typename T>
int apply_operator(lt_handle* h, int level, cdouble tau, const T* x, T* y, int R, const int* active) {
    const Level& L = h->levels[level];
    dim3 grid(nblk(L.N), R);
    k_apply<T><<<grid, kBlock, 0, h->stream>>>(view<T>(L), (T)tau.real(), (T)tau.imag(), x, y, active);
    LT_HIP(hipGetLastError());
    return 0;
}
template int apply_operator<double>(lt_handle*, int, cdouble, const double*, double*, int, const int*);
template int apply_operator<float>(lt_handle*, int, cdouble, const float*, float*, int, const int*);

template <typename T>
int mg_vcycle(lt_handle* h, cdouble tau, int nu1, int nu2, int R, const int* active, T* x0, const T* b0,
              RefineArgs* refine) {
    hipStream_t st = h->stream;
    const int nl = (int)h->levels.size();
    const T tr = (T)tau.real(), ti = (T)tau.imag();
    int rc = 0;
    // first level small enough for the single-workgroup kernel
    int lc = nl;
    for (int l = 0; l < nl; ++l)
        if (h->levels[l].N <= kCoarseBlockCells) { lc = l; break; }
    const bool cb = lc < nl && nl - lc <= kMaxCBLevels;
    if (!cb) lc = nl - 1;  // generic path down to the coarsest level
    const bool fused2d = h->grid.ndim == 2 && nu1 >= 1 && nu1 <= 3 && nu2 >= 1 && nu2 <= 3;
    const bool fusedT = fused2d;
    // cycles of 3D grids keep the generic levels' vectors in colour-planar order (the handle
    // decided at setup whether every such level allows it); the single-workgroup levels use
    // the natural order
    const bool cp = !fused2d && h->cp3d && cb;
    auto cpl = [&](int l) { return cp && l < lc ? 1 : 0; };
    const int* tiles = h->tiles[sizeof(T) == 4 ? 1 : 0];
    auto tile_of = [&](int l) { return l < kMaxTunedLevels ? tiles[l] : 0; };
    const int tag = sizeof(T) == 8 ? 64 : 32;
    // level vectors (fixed arrays and stack names: this path is also the allocation-free one)
    constexpr int kMaxLv = 48;
    if (nl >= kMaxLv) {
        set_last_error("too many multigrid levels");
        return LT_EUNSUPPORTED;
    }
    T* xpre[kMaxLv + 1] = {};
    T* xpost[kMaxLv + 1] = {};
    T* bs[kMaxLv + 1] = {};
    char nm[32];
    bs[0] = const_cast<T*>(b0);
    for (int l = 0; l <= lc && l < nl; ++l) {
        const size_t per = 2 * (size_t)h->levels[l].N * R;
        if (l > 0) {
            snprintf(nm, sizeof(nm), "mgb%d_%d", tag, l);
            bs[l] = wsp<T>(h, nm, per, &rc);
            if (!bs[l]) return rc;
        }
        if (l == 0 && (!fusedT || lc == 0)) {
            xpre[0] = x0;
        } else {
            snprintf(nm, sizeof(nm), "mgx%d_%d", tag, l);
            xpre[l] = wsp<T>(h, nm, per, &rc);
            if (!xpre[l]) return rc;
        }
        if (fusedT && l > 0 && l < lc) {
            snprintf(nm, sizeof(nm), "mgy%d_%d", tag, l);
            xpost[l] = wsp<T>(h, nm, per, &rc);
        } else {
            xpost[l] = xpre[l];
        }
        if (!xpost[l]) return rc;
    }
    xpost[0] = x0;
    // the generic levels' kernels take the active right-hand sides as a list (group_rhs)
    int* alist = nullptr;
    if (!fused2d && active) {
        static_assert(kMaxRhs <= 1024, "k_active_list takes one flag per thread of 1024");
        alist = wsp<int>(h, "mgalist", (size_t)R + 1, &rc);
        if (!alist) return rc;
    }
    const CoarseInverse* ci = mg_coarse_inverse(h, tau, &rc);
    if (rc < 0) return rc;
    if (h->arena_plan) return 0;  // sizes counted, nothing launched
    if (alist) {
        k_active_list<<<1, 1024, 0, st>>>(active, R, alist);
        LT_HIP(hipGetLastError());
    }
    if (refine) refine->list = alist;
    // ghost parity of the correction at a wall: odd at a Dirichlet wall, even at
    // a no-flux one (a water-table wall carries no conductive flux either)
    const T gsign[2] = {T(-1), T(1)};
    auto g = [&](int face) { return gsign[h->bc.face[face] == LT_BC_DIRICHLET0 ? 0 : 1]; };
    // the same for the prolongation from level l + 1 to level l: at a zero-head wall the fine
    // unknown nearest it takes delta_l / (2 delta_{l+1}) of its aggregate's value (the linear
    // interpolation to zero at the wall), i.e. the ghost parity 4 delta_l / (2 delta_{l+1}) - 3,
    // which is -1 for cell-centred levels
    auto gl = [&](int l, int face) {
        if (h->bc.face[face] != LT_BC_DIRICHLET0) return T(1);
        const int a = face / 2;
        const Level& F = h->levels[l];
        const Level& Cl = h->levels[l + 1];
        if (!Cl.coarsened_from_fine[a]) return T(-1);
        return T(4.0 * F.delta[a] / (2.0 * Cl.delta[a]) - 3.0);
    };
    // ---- down
    for (int l = 0; l < lc; ++l) {
        const Level& L = h->levels[l];
        const Level& C = h->levels[l + 1];
        LevelView<T> v = view<T>(L);
        if (fused2d) {
            unsigned long long* pc = nullptr;
            const bool prof = l == 0 && h->prof_target == LT_PROF_PRE_FINE;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (prof) LT_TRY(prof_begin(h, LT_PROF_PRE_FINE, &pc, &e0, &e1));
            LT_TRY(launch_pre2d<T>(st, v, tr, ti, nu1, tile_of(l), bs[l], xpre[l], C.n[0], C.n[1], C.coarsened_from_fine[0],
                                   C.coarsened_from_fine[1], bs[l + 1], R, active, pc, e0, e1));
            if (prof) LT_TRY(prof_end(h, LT_PROF_PRE_FINE));
        } else {
            const size_t per = 2 * (size_t)L.N;
            dim3 grid(nblk(L.N), R);
            if (nu1 > 0) {
                // from x = 0 (level 0 here; coarser levels are cleared by the restriction)
                k_gs_first<T, kSweepRhs><<<dim3(nblk(L.N), (R + kSweepRhs - 1) / kSweepRhs), kBlock, 0, st>>>(
                    v, tr, ti, xpre[l], bs[l], alist, R, cpl(l));
                LT_TRY(gs_half_sweep<T>(h, st, v, tr, ti, 1, xpre[l], bs[l], R, active, alist, l == 0, cpl(l)));
            } else if (l == 0) {
                k_zero<T><<<dim3(nblk(per), R), kBlock, 0, st>>>(xpre[0], per, active);
            }
            for (int s = 1; s < nu1; ++s)
                for (int c = 0; c < 2; ++c)
                    LT_TRY(gs_half_sweep<T>(h, st, v, tr, ti, c, xpre[l], bs[l], R, active, alist, l == 0, cpl(l)));
            k_resid_restrict<T, kSweepRhs><<<dim3(nblk(C.N), (R + kSweepRhs - 1) / kSweepRhs), kBlock, 0, st>>>(
                v, C.n[0], C.n[1], C.n[2], C.coarsened_from_fine[0], C.coarsened_from_fine[1],
                C.coarsened_from_fine[2], tr, ti, xpre[l], bs[l], bs[l + 1], xpre[l + 1], alist, R, cpl(l),
                cpl(l + 1));
            LT_HIP(hipGetLastError());
        }
    }
    // ---- coarse levels
    if (cb) {
        CBMeta<T> M{};
        M.nl = nl - lc;
        int off = 0;
        for (int l = lc; l < nl; ++l) {
            const Level& L = h->levels[l];
            LevelView<T> v = view<T>(L);
            CBLevel<T>& c = M.L[l - lc];
            c.nx = L.n[0]; c.ny = L.n[1]; c.nz = L.n[2]; c.N = L.N;
            c.cox = L.coarsened_from_fine[0]; c.coy = L.coarsened_from_fine[1]; c.coz = L.coarsened_from_fine[2];
            c.off = off;
            off += L.N;
            c.Tx = v.Tx; c.Ty = v.Ty; c.Tz = v.Tz; c.D = v.D; c.m = v.m;
        }
        for (int f = 0; f < 6; ++f) M.ghost[f] = g(f);
        M.nu1 = nu1;
        M.nu2 = nu2;
        M.inv = ci ? inv_ptr<T>(ci) : nullptr;
        M.coarse_sweeps = 64;
        T* out = (lc == 0) ? x0 : xpre[lc];
        LT_TRY(launch_coarse_block<T>(st, M, tr, ti, bs[lc], out, R, active));
        xpost[lc] = out;
    } else {
        const Level& L = h->levels[lc];
        dim3 grid(nblk(L.N), R);
        if (lc == 0) {
            const size_t per = 2 * (size_t)L.N;
            k_zero<T><<<dim3(nblk(per), R), kBlock, 0, st>>>(x0, per, active);
        }
        if (ci) {
            k_coarse_solve<T><<<grid, kBlock, 0, st>>>(L.N, inv_ptr<T>(ci), bs[lc], xpre[lc], active);
        } else {
            LevelView<T> v = view<T>(L);
            for (int s = 0; s < 64; ++s)
                for (int c = 0; c < 2; ++c)
                    LT_TRY(gs_half_sweep<T>(h, st, v, tr, ti, c, xpre[lc], bs[lc], R, active, alist, lc == 0));
        }
        LT_HIP(hipGetLastError());
        xpost[lc] = xpre[lc];
    }
    // ---- up
    for (int l = lc - 1; l >= 0; --l) {
        const Level& L = h->levels[l];
        const Level& C = h->levels[l + 1];
        LevelView<T> v = view<T>(L);
        if (fused2d) {
            T4 gh = {(double)gl(l, 0), (double)gl(l, 1), (double)gl(l, 2), (double)gl(l, 3)};
            unsigned long long* pc = nullptr;
            const bool prof = l == 0 && h->prof_target == LT_PROF_POST_FINE;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (prof) LT_TRY(prof_begin(h, LT_PROF_POST_FINE, &pc, &e0, &e1));
            if (l == 0 && refine) {
                LT_TRY(launch_post2d_refine<T>(st, v, h->levels[0].v64(), tr, ti, tau.real(), tau.imag(), nu2,
                                               tile_of(0), bs[0],
                                               xpre[0], xpost[1], C.n[0], C.n[1], C.coarsened_from_fine[0],
                                               C.coarsened_from_fine[1], gh, refine->u, refine->ustride, refine->jcol,
                                               refine->rho_in, refine->rho_out, static_cast<T*>(refine->lo),
                                               refine->part, R, active, pc, refine->nparts, e0, e1));
            } else {
                LT_TRY(launch_post2d<T>(st, v, tr, ti, nu2, tile_of(l), bs[l], xpre[l], xpost[l + 1], C.n[0], C.n[1],
                                        C.coarsened_from_fine[0], C.coarsened_from_fine[1], gh, xpost[l], R, active,
                                        pc, e0, e1));
            }
            if (prof) LT_TRY(prof_end(h, LT_PROF_POST_FINE));
        } else {
            // the post-smoother below starts with colour 1, which overwrites those cells
            const int c0only = nu2 >= 1 ? 1 : 0;
            const size_t np = (c0only && cpl(l)) ? L.N / 2 : L.N;
            k_prolong_rb<T, kSweepRhs><<<dim3(nblk(np), (R + kSweepRhs - 1) / kSweepRhs), kBlock, 0, st>>>(
                L.n[0], L.n[1], L.n[2], C.n[0], C.n[1], C.n[2], C.coarsened_from_fine[0], C.coarsened_from_fine[1],
                C.coarsened_from_fine[2], gl(l, 0), gl(l, 1), gl(l, 2), gl(l, 3), gl(l, 4), gl(l, 5), xpost[l + 1], xpre[l],
                alist, R, cpl(l),
                cpl(l + 1), c0only);
            for (int s = 0; s < nu2; ++s)
                for (int c = 1; c >= 0; --c)
                    LT_TRY(gs_half_sweep<T>(h, st, v, tr, ti, c, xpre[l], bs[l], R, active, alist, l == 0, cpl(l)));
            xpost[l] = xpre[l];
            LT_HIP(hipGetLastError());
        }
    }
    return 0;
}
template int mg_vcycle<double>(lt_handle*, cdouble, int, int, int, const int*, double*, const double*,
                               RefineArgs*);
template int mg_vcycle<float>(lt_handle*, cdouble, int, int, int, const int*, float*, const float*, RefineArgs*);

}  // namespace lt
