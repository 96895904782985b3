// Exact shift-and-invert preconditioner: x = (K + tau M)^{-1} b in FP64, the factorised
// preconditioner of the flexible shifted Krylov method (Section 3: each (K + tau_j M) is
// factorised once and its inverse applied at every iteration that uses tau_j).
//
// The grid is cut into slices along its last axis (rows of nx cells in 2D, planes of nx ny
// cells in 3D).  K + tau M is then block tridiagonal: nb x nb diagonal blocks (the operator
// within one slice) and diagonal couplings -T between neighbouring slices.  Block cyclic
// reduction eliminates the odd-positioned blocks of each level, leaving a block tridiagonal
// system on the even ones, until one block is left.  Writing row i of a level as
// F_{i-1}^T x_{i-1} + D_i x_i + F_i x_{i+1} = b_i (the matrix is complex symmetric):
//   eliminated i:  Dinv_i = D_i^{-1},  P_i = Dinv_i F_{i-1}^T,  Q_i = Dinv_i F_i
//   kept p -> p/2: D'_p = D_p - F_{p-1}^T Q_{p-1} - F_p P_{p+1},  F'_p = -F_p Q_{p+1}
// At level 0 the couplings are diagonal and these products are elementwise.  A solve
// reduces the right-hand side level by level, b'_p = b_p - Q_{p-1}^T b_{p-1} - P_{p+1}^T
// b_{p+1}, solves the last block, and substitutes back, x_i = Dinv_i b_i - P_i x_{i-1} -
// Q_i x_{i+1}: 2 log2(slices) dependent stages, each a batch of independent dense block
// products (a block LDL^T sweep would take 2 x slices dependent stages).
//
// No pivoting.  For Im tau != 0 the Hermitian part of -i sign(Im tau) (K + tau M) is
// |Im tau| M, definite; every Schur complement and diagonal sub-block of a matrix with a
// definite Hermitian part has one too, so no pivot can vanish.  For real tau >= 0 the
// matrix is real symmetric positive definite wherever K + tau M is nonsingular.  A zero or
// non-finite pivot is reported as an error.
//
// Storage: every dense block is [2][nb][nb] float64 (real plane, then imaginary plane,
// row-major).  Vectors of the caller are [R][2][N] (slice q of right-hand side r, plane c at
// r * rstride + c * N + q * nb); reduced right-hand sides and partial solutions of the
// levels are [block][R][2][nb] workspaces.
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "lt_internal.h"

namespace lt {

namespace {

constexpr int kGJW = 16;   // Gauss-Jordan panel width
constexpr int kGJTI = 16;  // rows per workgroup of the Gauss-Jordan update
constexpr int kGT = 64;    // GEMM output tile
constexpr int kGK = 16;    // GEMM inner chunk

// The fine operator cut into slices of nb cells along its last axis.
struct ExOp {
    const double* Tx;
    const double* Ty;
    const double* D;
    const double* m;
    int nx, ndim, nb;
    double tr, ti;
};

// entry (a, b) of diagonal block q of K + tau M
__device__ inline void ex_a_elem(const ExOp& op, int q, int a, int b, double* re, double* im) {
    const size_t c = (size_t)q * op.nb;
    if (a == b) {
        *re = op.D[c + a] + op.tr * op.m[c + a];
        *im = op.ti * op.m[c + a];
        return;
    }
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    double v = 0.0;
    if (hi == lo + 1) v -= op.Tx[c + lo];  // Tx is 0 at the last cell of an x line
    if (op.ndim == 3 && hi == lo + op.nx) v -= op.Ty[c + lo];
    *re = v;
    *im = 0.0;
}

// Dense diagonal blocks q = q0 + qstep * s of K + tau M into out + s * ms.
__global__ __launch_bounds__(256) void k_ex_dense(ExOp op, int q0, int qstep, double* __restrict__ out, size_t ms) {
    const int s = blockIdx.y;
    const size_t nn = (size_t)op.nb * op.nb;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nn) return;
    const int a = (int)(e / op.nb), b = (int)(e % op.nb);
    double re, im;
    ex_a_elem(op, q0 + qstep * s, a, b, &re, &im);
    double* o = out + (size_t)s * ms;
    o[e] = re;
    o[nn + e] = im;
}

// Level 0 -> 1 with diagonal couplings f_q = -Tl[q nb + .] (slice q to q + 1):
//   D1_k = A_{2k} - (f_{2k-1} f_{2k-1}^T) o Dinv0[k-1] - (f_{2k} f_{2k}^T) o Dinv0[k]
//   F1_k = -(f_{2k} f_{2k+1}^T) o Dinv0[k]          (o: elementwise product)
// Dinv0[s] is the inverse of slice 2s + 1.
__global__ __launch_bounds__(256) void k_ex_schur0(ExOp op, int n, const double* __restrict__ Tl,
                                                   const double* __restrict__ dinv0, size_t ms,
                                                   double* __restrict__ Dn, double* __restrict__ Fn) {
    const int k = blockIdx.y, p = 2 * k;
    const int nb = op.nb;
    const size_t nn = (size_t)nb * nb;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nn) return;
    const int a = (int)(e / nb), b = (int)(e % nb);
    double re, im;
    ex_a_elem(op, p, a, b, &re, &im);
    if (p >= 1) {
        const double* g = dinv0 + (size_t)(k - 1) * ms;
        const double t = Tl[(size_t)(p - 1) * nb + a] * Tl[(size_t)(p - 1) * nb + b];
        re -= t * g[e];
        im -= t * g[nn + e];
    }
    if (p + 1 < n) {
        const double* g = dinv0 + (size_t)k * ms;
        const double t = Tl[(size_t)p * nb + a] * Tl[(size_t)p * nb + b];
        re -= t * g[e];
        im -= t * g[nn + e];
        if (p + 2 < n) {
            const double u = -Tl[(size_t)p * nb + a] * Tl[(size_t)(p + 1) * nb + b];
            double* f = Fn + (size_t)k * ms;
            f[e] = u * g[e];
            f[nn + e] = u * g[nn + e];
        }
    }
    double* d = Dn + (size_t)k * ms;
    d[e] = re;
    d[nn + e] = im;
}

// ------------------------------------------------------------------ inversion
// In-place Gauss-Jordan inversion without pivoting, kGJW pivots (one panel K) per step:
//   A_KK <- P^{-1};  A_KJ <- P^{-1} A_KJ;  A_IJ <- A_IJ - A_IK (P^{-1} A_KJ);  A_IK <- -A_IK P^{-1}
// (P = A_KK; I, J outside K).  After every panel A holds its inverse.  Step 1 (one
// workgroup per matrix): invert P in LDS and form the row panel.
__global__ __launch_bounds__(256) void k_gj_panel(double* __restrict__ mats, size_t ms, int nb, int k0,
                                                  int* __restrict__ flag) {
    double* Ar = mats + (size_t)blockIdx.x * ms;
    double* Ai = Ar + (size_t)nb * nb;
    const int w = min(kGJW, nb - k0);
    __shared__ double pr[kGJW][kGJW + 1], pi[kGJW][kGJW + 1];
    const int tid = threadIdx.x, i = tid / kGJW, j = tid % kGJW;
    const bool in = i < w && j < w;
    pr[i][j] = in ? Ar[(size_t)(k0 + i) * nb + k0 + j] : 0.0;
    pi[i][j] = in ? Ai[(size_t)(k0 + i) * nb + k0 + j] : 0.0;
    __syncthreads();
    for (int s = 0; s < w; ++s) {
        const double a = pr[s][s], b = pi[s][s];
        const double d = a * a + b * b;
        if (!(d > 0.0 && d <= 1.7976931348623157e308) && tid == 0) *flag = 1;
        const double ir = a / d, ii = -b / d;  // 1 / pivot
        double nr = 0.0, ni = 0.0;
        if (in) {
            const double xr = pr[i][j], xi = pi[i][j];
            if (i == s && j == s) {
                nr = ir;
                ni = ii;
            } else if (i == s) {
                nr = xr * ir - xi * ii;
                ni = xr * ii + xi * ir;
            } else if (j == s) {
                nr = -(xr * ir - xi * ii);
                ni = -(xr * ii + xi * ir);
            } else {
                const double cr = pr[i][s], ci = pi[i][s], rr = pr[s][j], ri = pi[s][j];
                const double tr = cr * rr - ci * ri, ti = cr * ri + ci * rr;  // a_is a_sj
                nr = xr - (tr * ir - ti * ii);
                ni = xi - (tr * ii + ti * ir);
            }
        }
        __syncthreads();
        if (in) {
            pr[i][j] = nr;
            pi[i][j] = ni;
        }
        __syncthreads();
    }
    if (in) {
        Ar[(size_t)(k0 + i) * nb + k0 + j] = pr[i][j];
        Ai[(size_t)(k0 + i) * nb + k0 + j] = pi[i][j];
    }
    // row panel R = P^{-1} A_KJ, column by column
    for (int c = tid; c < nb; c += 256) {
        if (c >= k0 && c < k0 + w) continue;
        double xr[kGJW], xi[kGJW];
#pragma unroll
        for (int t = 0; t < kGJW; ++t) {  // rows past w read row k0 (P^{-1} is zero there)
            const size_t o = (size_t)(k0 + (t < w ? t : 0)) * nb + c;
            xr[t] = Ar[o];
            xi[t] = Ai[o];
        }
#pragma unroll 1
        for (int t = 0; t < w; ++t) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int u = 0; u < kGJW; ++u) {  // P^{-1} is zero past w
                sr += pr[t][u] * xr[u] - pi[t][u] * xi[u];
                si += pr[t][u] * xi[u] + pi[t][u] * xr[u];
            }
            Ar[(size_t)(k0 + t) * nb + c] = sr;
            Ai[(size_t)(k0 + t) * nb + c] = si;
        }
    }
}

// Step 2: rows I (kGJTI per workgroup, rows of the panel skipped) get the rank-w update
// with the row panel, and their panel columns become -A_IK P^{-1}.  A workgroup owns its
// rows, so it reads its old A_IK before writing it.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ mats, size_t ms, int nb, int k0) {
    double* Ar = mats + (size_t)blockIdx.y * ms;
    double* Ai = Ar + (size_t)nb * nb;
    const int w = min(kGJW, nb - k0);
    const int i0 = blockIdx.x * kGJTI;
    __shared__ double cr[kGJTI][kGJW + 1], ci[kGJTI][kGJW + 1], pr[kGJW][kGJW + 1], pi[kGJW][kGJW + 1];
    const int tid = threadIdx.x, ii = tid / kGJW, t = tid % kGJW;
    {
        const int row = i0 + ii;
        const bool ok = row < nb && !(row >= k0 && row < k0 + w) && t < w;
        cr[ii][t] = ok ? Ar[(size_t)row * nb + k0 + t] : 0.0;
        ci[ii][t] = ok ? Ai[(size_t)row * nb + k0 + t] : 0.0;
        const bool okp = ii < w && t < w;
        pr[ii][t] = okp ? Ar[(size_t)(k0 + ii) * nb + k0 + t] : 0.0;
        pi[ii][t] = okp ? Ai[(size_t)(k0 + ii) * nb + k0 + t] : 0.0;
    }
    __syncthreads();
    for (int c = tid; c < nb; c += 256) {
        if (c >= k0 && c < k0 + w) continue;
        // keep the reads of C from LDS inside the loop (hoisted, 512 values would not fit in registers)
        asm volatile("" ::: "memory");
        // every load first (clamped rows; C and P^{-1} are zero past w), then the updates
        double rr[kGJW], ri[kGJW], xr[kGJTI], xi[kGJTI];
#pragma unroll
        for (int u = 0; u < kGJW; ++u) {
            const size_t o = (size_t)(k0 + (u < w ? u : 0)) * nb + c;
            rr[u] = Ar[o];
            ri[u] = Ai[o];
        }
#pragma unroll
        for (int r = 0; r < kGJTI; ++r) {
            const size_t o = (size_t)min(i0 + r, nb - 1) * nb + c;
            xr[r] = Ar[o];
            xi[r] = Ai[o];
        }
#pragma unroll
        for (int r = 0; r < kGJTI; ++r) {
            const int row = i0 + r;
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int u = 0; u < kGJW; ++u) {
                sr += cr[r][u] * rr[u] - ci[r][u] * ri[u];
                si += cr[r][u] * ri[u] + ci[r][u] * rr[u];
            }
            if (row < nb && !(row >= k0 && row < k0 + w)) {
                Ar[(size_t)row * nb + c] = xr[r] - sr;
                Ai[(size_t)row * nb + c] = xi[r] - si;
            }
        }
    }
    {
        const int row = i0 + ii;
        if (row < nb && !(row >= k0 && row < k0 + w) && t < w) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int u = 0; u < kGJW; ++u) {
                sr += cr[ii][u] * pr[u][t] - ci[ii][u] * pi[u][t];
                si += cr[ii][u] * pi[u][t] + ci[ii][u] * pr[u][t];
            }
            Ar[(size_t)row * nb + k0 + t] = -sr;
            Ai[(size_t)row * nb + k0 + t] = -si;
        }
    }
}

// ------------------------------------------------------------------ GEMM
// C_b = beta C_b + alpha op(A_b) op(B_b) for b < gridDim.z, complex nb x nb blocks at
// X0 + b * sX (doubles); op = transpose (not conjugate) when TA / TB is set.
template <int TA, int TB>
__global__ __launch_bounds__(256) void k_ex_gemm(int nb, double alpha, double beta, const double* __restrict__ A0,
                                                 size_t sA, const double* __restrict__ B0, size_t sB,
                                                 double* __restrict__ C0, size_t sC) {
    const size_t nn = (size_t)nb * nb;
    const double* Ar = A0 + (size_t)blockIdx.z * sA;
    const double* Ai = Ar + nn;
    const double* Br = B0 + (size_t)blockIdx.z * sB;
    const double* Bi = Br + nn;
    double* Cr = C0 + (size_t)blockIdx.z * sC;
    double* Ci = Cr + nn;
    const int r0 = blockIdx.y * kGT, c0 = blockIdx.x * kGT;
    __shared__ double asr[kGK][kGT + 1], asi[kGK][kGT + 1], bsr[kGK][kGT + 1], bsi[kGK][kGT + 1];
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    double accr[4][4] = {}, acci[4][4] = {};
    // this thread's tile entries: (row, k) of op(A) and (k, col) of op(B) for q < 4
    constexpr int Q = kGT * kGK / 256;
    int arow[Q], ak[Q], bk[Q], bcol[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int idx = tid + 256 * q;
        arow[q] = TA ? idx % kGT : idx / kGK;
        ak[q] = TA ? idx / kGT : idx % kGK;
        bcol[q] = TB ? idx / kGK : idx % kGT;
        bk[q] = TB ? idx % kGK : idx / kGT;
    }
    double ra[Q], ia[Q], rb[Q], ib[Q];  // the next chunk, in flight during the current one
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int gr = r0 + arow[q], gk = k0 + ak[q];
            const bool oka = gr < nb && gk < nb;
            const size_t oa = oka ? (TA ? (size_t)gk * nb + gr : (size_t)gr * nb + gk) : 0;
            ra[q] = Ar[oa];
            ia[q] = Ai[oa];
            if (!oka) ra[q] = ia[q] = 0.0;
            const int gc = c0 + bcol[q], gkb = k0 + bk[q];
            const bool okb = gc < nb && gkb < nb;
            const size_t ob = okb ? (TB ? (size_t)gc * nb + gkb : (size_t)gkb * nb + gc) : 0;
            rb[q] = Br[ob];
            ib[q] = Bi[ob];
            if (!okb) rb[q] = ib[q] = 0.0;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < nb; k0 += kGK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            asr[ak[q]][arow[q]] = ra[q];
            asi[ak[q]][arow[q]] = ia[q];
            bsr[bk[q]][bcol[q]] = rb[q];
            bsi[bk[q]][bcol[q]] = ib[q];
        }
        __syncthreads();
        if (k0 + kGK < nb) fetch(k0 + kGK);
#pragma unroll 4
        for (int k = 0; k < kGK; ++k) {
            double ar[4], ai[4], br[4], bi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ar[u] = asr[k][ty + 16 * u];
                ai[u] = asi[k][ty + 16 * u];
                br[u] = bsr[k][tx + 16 * u];
                bi[u] = bsi[k][tx + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    accr[u][v] += ar[u] * br[v] - ai[u] * bi[v];
                    acci[u][v] += ar[u] * bi[v] + ai[u] * br[v];
                }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gr = r0 + ty + 16 * u, gc = c0 + tx + 16 * v;
            if (gr < nb && gc < nb) {
                const size_t o = (size_t)gr * nb + gc;
                double cr = alpha * accr[u][v], ci = alpha * acci[u][v];
                if (beta != 0.0) {
                    cr += beta * Cr[o];
                    ci += beta * Ci[o];
                }
                Cr[o] = cr;
                Ci[o] = ci;
            }
        }
}

// ------------------------------------------------------------------ solve
// One block of R complex vectors: element (r, c, a) at p[r * rs + c * ps + a].
struct ExVec {
    const double* p;
    size_t rs, ps;
};

// One term  sign * S^T v  of a block product, S a stored dense block read as S[k][a] (each
// block is stored in the orientation its product needs).  When T1 is given, v is replaced by
// v + T1 o w1 (+ T2 o w2): level 0's back substitution folds its diagonal couplings into the
// product's input.
struct ExTerm {
    const double* S;
    double sign;
    ExVec v;
    const double* T1;
    ExVec w1;
    const double* T2;
    ExVec w2;
};

enum { kModeT0 = 0, kModeReduce = 2, kModeTop = 3, kModeBack = 4, kModeBack0 = 5 };

// Where the blocks of a level's vectors live: block i of right-hand side r, plane c at
// base + i * bstride + r * rs + c * ps.  Levels below the tail: [block][R][2][nb]; the tail
// level: [R][2][nl nb] (contiguous per right-hand side, for its dense product).
struct ExLay {
    size_t bstride, rs, ps;
};

struct ExSolve {
    int mode, nb, R, n, nl;           // n: slices; nl: blocks at this level; nb: rows (the tail: nl nb)
    const double* mats;
    size_t ms;                        // doubles per dense block
    size_t dinv, pm, qm, ptm, qtm;    // first slot of Dinv / P / Q / P^T / Q^T at this level
    const double* tail;               // the tail's dense inverse (kModeTop)
    const double* b;                  // caller's right-hand side, slice q at b + q nb
    size_t brs;
    double* x;                        // caller's solution
    size_t xrs;
    size_t N;                         // plane stride of the caller's vectors
    const double* Bl;                 // this level's reduced right-hand sides
    double* Bn;                       // the next level's
    double* Xl;                       // this level's solution blocks (or level 0's T = Dinv b)
    const double* Xn;                 // the next level's solution blocks
    ExLay ll, ln;                     // layouts of this level's and the next level's vectors
    const double* Tl;                 // couplings along the slicing axis (T of the last axis)
    const int* active;                // [R] or nullptr: the caller's x of a right-hand side marked 0 is kept
    int ks;                           // kModeTop: the inner dimension is split over ks workgroups ...
    double* part;                     // ... whose partial products go to part[ks][R][2][nb]
};

__device__ inline ExVec ws_vec(const double* base, const ExLay& L, int blk) {
    return ExVec{base + (size_t)blk * L.bstride, L.rs, L.ps};
}

constexpr int kExKG = 16;  // k-groups (waves) per row tile of a block product

// y (64 rows from a0, NR right-hand sides from r0) = y0 + sum_t sign_t S_t^T v_t.  Thread (a, g)
// takes row a0 + a and the inner indices k = g, g + KG, ...: per k a wave reads 64 consecutive
// entries of row k of each plane of S (coalesced) straight from HBM, and the right-hand sides'
// entries at k from LDS (the same address for every lane), where the workgroup stages them a
// slice at a time.  The matrices are read once and the loads of successive k are independent;
// 16 k-groups keep a thread's share of the inner dimension short (a few round trips to HBM).
// The KG partial sums of a row are added through LDS at the end.
// COMB: level 0's back substitution (the one mode whose term has couplings).
template <bool COMB, int NR>
__global__ __launch_bounds__(64 * kExKG) void k_ex_solve(ExSolve A) {
    constexpr int KG = kExKG;
    const int nb = A.nb, o = blockIdx.z;
    const int kp = blockIdx.y % A.ks;  // part of the inner dimension (kModeTop only; else 0 of 1)
    const int a0 = blockIdx.x * 64, r0 = (blockIdx.y / A.ks) * NR;
    const int kspan = (nb + A.ks - 1) / A.ks;
    const int kb = kp * kspan, ke = min(nb, kb + kspan);
    // up to three terms at fixed positions (S == nullptr: absent), so that they stay in registers
    ExTerm terms[3];
    const ExVec none{nullptr, 0, 0};
#pragma unroll
    for (int t = 0; t < 3; ++t) terms[t] = ExTerm{nullptr, 0.0, none, nullptr, none, nullptr, none};
    ExVec y0{nullptr, 0, 0};
    double* yp;
    size_t yrs, yps;
    bool to_caller = false;  // y is the caller's x (masked by active)
    auto mat = [&](size_t slot) { return A.mats + slot * A.ms; };
    const ExLay t0lay{2 * (size_t)A.R * nb, 2 * (size_t)nb, (size_t)nb};  // level 0's T = Dinv b
    switch (A.mode) {
    case kModeT0:  // T0[o] = Dinv0[o] b_{2o+1}
        yp = A.Xl + (size_t)o * t0lay.bstride;
        yrs = t0lay.rs;
        yps = t0lay.ps;
        terms[0] = ExTerm{mat(A.dinv + o), 1.0, ExVec{A.b + (size_t)(2 * o + 1) * nb, A.brs, A.N}, nullptr, none,
                          nullptr, none};
        break;
    case kModeReduce:  // B'_o = B_{2o} - Q_{2o-1}^T B_{2o-1} - P_{2o+1}^T B_{2o+1}
        yp = A.Bn + (size_t)o * A.ln.bstride;
        yrs = A.ln.rs;
        yps = A.ln.ps;
        y0 = ws_vec(A.Bl, A.ll, 2 * o);
        if (o >= 1)
            terms[0] = ExTerm{mat(A.qm + o - 1), -1.0, ws_vec(A.Bl, A.ll, 2 * o - 1), nullptr, none, nullptr, none};
        if (2 * o + 1 < A.nl)
            terms[1] = ExTerm{mat(A.pm + o), -1.0, ws_vec(A.Bl, A.ll, 2 * o + 1), nullptr, none, nullptr, none};
        break;
    case kModeTop:  // the tail's dense inverse on its right-hand side (one slice: the caller's vectors),
                    // or, split over ks, partial products into part
        if (A.ks > 1) {
            yp = A.part + (size_t)kp * A.R * 2 * nb;
            yrs = 2 * (size_t)nb;
            yps = nb;
        } else if (A.n == 1) {
            yp = A.x;
            yrs = A.xrs;
            yps = A.N;
            to_caller = true;
        } else {
            yp = A.Xl;
            yrs = A.ll.rs;
            yps = A.ll.ps;
        }
        terms[0] = ExTerm{A.tail, 1.0, A.n == 1 ? ExVec{A.b, A.brs, A.N} : ExVec{A.Bl, A.ll.rs, A.ll.ps}, nullptr,
                          none, nullptr, none};
        break;
    case kModeBack: {  // X_o = X'_{o/2} (even);  Dinv_s B_o - P_s X'_s - Q_s X'_{s+1} (odd, s = (o-1)/2)
        yp = A.Xl + (size_t)o * A.ll.bstride;
        yrs = A.ll.rs;
        yps = A.ll.ps;
        if (!(o & 1)) {
            y0 = ws_vec(A.Xn, A.ln, o / 2);
        } else {
            const int s = (o - 1) / 2;
            terms[0] = ExTerm{mat(A.dinv + s), 1.0, ws_vec(A.Bl, A.ll, o), nullptr, none, nullptr, none};
            terms[1] = ExTerm{mat(A.ptm + s), -1.0, ws_vec(A.Xn, A.ln, s), nullptr, none, nullptr, none};
            if (o + 1 < A.nl)
                terms[2] = ExTerm{mat(A.qtm + s), -1.0, ws_vec(A.Xn, A.ln, s + 1), nullptr, none, nullptr, none};
        }
        break;
    }
    default: {  // kModeBack0: x_o = X1_{o/2} (even);  Dinv0_s (b_o + T_{o-1} X1_s + T_o X1_{s+1}) (odd)
        yp = A.x + (size_t)o * nb;
        yrs = A.xrs;
        yps = A.N;
        to_caller = true;
        if (!(o & 1)) {
            y0 = ws_vec(A.Xn, A.ln, o / 2);
        } else {
            const int s = (o - 1) / 2;
            const bool right = o + 1 < A.n;
            terms[0] = ExTerm{mat(A.dinv + s), 1.0, ExVec{A.b + (size_t)o * nb, A.brs, A.N},
                              A.Tl + (size_t)(o - 1) * nb, ws_vec(A.Xn, A.ln, s),
                              right ? A.Tl + (size_t)o * nb : nullptr, right ? ws_vec(A.Xn, A.ln, s + 1) : none};
        }
        break;
    }
    }

    const int a = threadIdx.x % 64, g = threadIdx.x / 64;
    const int row = a0 + a;
    const int rowc = row < nb ? row : nb - 1;  // rows past nb read a valid entry, never written
    // one LDS buffer: a slice of the right-hand sides (KC inner indices x NR, the couplings of
    // level 0 already folded in), then the partial sums (KG x NR x 64, real and imaginary)
    constexpr int KC = 2048 / NR;
    __shared__ double2 lds[2048];
    double accr[NR], acci[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) accr[j] = acci[j] = 0.0;
    const size_t nn = (size_t)nb * nb;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const ExTerm& T = terms[t];
        if (!T.S) continue;
        const double* Sr = T.S + rowc;
        const double* Si = T.S + nn + rowc;
        for (int kc0 = kb; kc0 < ke; kc0 += KC) {
            const int kc = min(KC, ke - kc0);
            __syncthreads();  // the previous slice is no longer read
            for (int idx = threadIdx.x; idx < kc * NR; idx += 64 * KG) {
                const int kk = idx % kc, j = idx / kc;
                const int k = kc0 + kk;
                const size_t r = (size_t)min(r0 + j, A.R - 1);  // past R: computed and dropped
                double vr = T.v.p[r * T.v.rs + k], vi = T.v.p[r * T.v.rs + T.v.ps + k];
                if (COMB) {
                    if (T.T1) {
                        vr += T.T1[k] * T.w1.p[r * T.w1.rs + k];
                        vi += T.T1[k] * T.w1.p[r * T.w1.rs + T.w1.ps + k];
                    }
                    if (T.T2) {
                        vr += T.T2[k] * T.w2.p[r * T.w2.rs + k];
                        vi += T.T2[k] * T.w2.p[r * T.w2.rs + T.w2.ps + k];
                    }
                }
                lds[kk * NR + j] = make_double2(T.sign * vr, T.sign * vi);
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = g; kk < kc; kk += KG) {
                const size_t k = (size_t)(kc0 + kk);
                const double sr = Sr[k * nb], si = Si[k * nb];
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    const double2 v = lds[kk * NR + j];
                    accr[j] += sr * v.x - si * v.y;
                    acci[j] += sr * v.y + si * v.x;
                }
            }
        }
    }
    // add the KG groups' partial sums, JR right-hand sides at a time (KG x JR x 64 complex in LDS)
    constexpr int JR = NR < 2 ? NR : 2;
    double* redr = reinterpret_cast<double*>(lds);
    double* redi = redr + KG * JR * 64;
#pragma unroll
    for (int j0 = 0; j0 < NR; j0 += JR) {
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < JR; ++jj) {
            redr[(g * JR + jj) * 64 + a] = accr[j0 + jj];
            redi[(g * JR + jj) * 64 + a] = acci[j0 + jj];
        }
        __syncthreads();
        const int r = r0 + j0 + g;  // wave g < JR finishes right-hand side j0 + g
        if (g < JR && row < nb && r < A.R && !(to_caller && A.active && !A.active[r])) {
            double sr = 0.0, si = 0.0;
            if (y0.p) {
                sr = y0.p[(size_t)r * y0.rs + row];
                si = y0.p[(size_t)r * y0.rs + y0.ps + row];
            }
            for (int q = 0; q < KG; ++q) {
                sr += redr[(q * JR + g) * 64 + a];
                si += redi[(q * JR + g) * 64 + a];
            }
            yp[(size_t)r * yrs + row] = sr;
            yp[(size_t)r * yrs + yps + row] = si;
        }
    }
}

// Level 0 reduction with diagonal couplings: B1_k = b_{2k} + T_{2k-1} o T0[k-1] + T_{2k} o T0[k]
// (f = -T), one thread per (rhs, plane, cell) of one block; B1 in layout L1.
__global__ __launch_bounds__(256) void k_ex_reduce0(int nb, int R, int n, const double* __restrict__ b, size_t brs,
                                                    size_t N, const double* __restrict__ Tl,
                                                    const double* __restrict__ T0, double* __restrict__ B1,
                                                    ExLay L1) {
    const int k = blockIdx.y, p = 2 * k;
    const size_t bs = 2 * (size_t)R * nb;  // T0's block stride
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= bs) return;
    const int a = (int)(e % nb);
    const int c = (int)((e / nb) % 2);
    const int r = (int)(e / (2 * (size_t)nb));
    double v = b[(size_t)r * brs + (size_t)c * N + (size_t)p * nb + a];
    if (p >= 1) v += Tl[(size_t)(p - 1) * nb + a] * T0[(size_t)(k - 1) * bs + e];
    if (p + 1 < n) v += Tl[(size_t)p * nb + a] * T0[(size_t)k * bs + e];
    B1[(size_t)k * L1.bstride + (size_t)r * L1.rs + (size_t)c * L1.ps + a] = v;
}

// The tail's k-split partial products summed: X = sum_p part[p] (X and part [R][2][m]).
__global__ __launch_bounds__(256) void k_ex_sum_parts(size_t len, int ks, const double* __restrict__ part,
                                                      double* __restrict__ X) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= len) return;
    double v = 0.0;
    for (int p = 0; p < ks; ++p) v += part[(size_t)p * len + e];
    X[e] = v;
}

// The tail level's reduced system as one dense matrix of m = nl nb unknowns: diagonal blocks
// D_i, block (i, i + 1) F_i and block (i + 1, i) F_i^T.
__global__ __launch_bounds__(256) void k_ex_tail(int nb, int nl, const double* __restrict__ D,
                                                 const double* __restrict__ Fb, size_t ms, double* __restrict__ out) {
    const size_t m = (size_t)nl * nb, mm = m * m, nn = (size_t)nb * nb;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= mm) return;
    const size_t I = e / m, J = e % m;
    const int bi = (int)(I / nb), bj = (int)(J / nb), a = (int)(I % nb), c = (int)(J % nb);
    double re = 0.0, im = 0.0;
    if (bi == bj) {
        const double* g = D + (size_t)bi * ms;
        re = g[(size_t)a * nb + c];
        im = g[nn + (size_t)a * nb + c];
    } else if (bj == bi + 1) {
        const double* g = Fb + (size_t)bi * ms;
        re = g[(size_t)a * nb + c];
        im = g[nn + (size_t)a * nb + c];
    } else if (bi == bj + 1) {
        const double* g = Fb + (size_t)bj * ms;
        re = g[(size_t)c * nb + a];
        im = g[nn + (size_t)c * nb + a];
    }
    out[e] = re;
    out[mm + e] = im;
}

inline unsigned nblk(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// right-hand sides per workgroup: the smallest of 1, 2, 4, 8 that covers R (8 beyond)
inline int solve_nr(int R) { return R >= 8 ? 8 : R >= 4 ? (R == 4 ? 4 : 8) : R >= 2 ? (R == 2 ? 2 : 4) : 1; }

template <bool COMB, int NR>
hipError_t launch_nr(const ExSolve& A, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    hipExtLaunchKernelGGL((k_ex_solve<COMB, NR>), g, dim3(64 * kExKG), 0, st, e0, e1, 0, A);
    return hipGetLastError();
}

template <bool COMB>
hipError_t dispatch_nr(const ExSolve& A, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    switch (solve_nr(A.R)) {
    case 1: return launch_nr<COMB, 1>(A, g, st, e0, e1);
    case 2: return launch_nr<COMB, 2>(A, g, st, e0, e1);
    case 4: return launch_nr<COMB, 4>(A, g, st, e0, e1);
    default: return launch_nr<COMB, 8>(A, g, st, e0, e1);
    }
}

hipError_t dispatch_solve(const ExSolve& A, dim3 g, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    return A.mode == kModeBack0 ? dispatch_nr<true>(A, g, st, e0, e1) : dispatch_nr<false>(A, g, st, e0, e1);
}

// One block-product launch of a solve; with opts.profile = LT_PROF_EXACT it is bracketed by
// HIP events and its algorithmic bytes (dense blocks and vector blocks it must move) counted.
int launch_solve(lt_handle* h, const ExSolve& A, dim3 g, double bytes) {
    hipStream_t st = h->stream;
    if (h->prof_target == LT_PROF_EXACT) {
        unsigned long long* pc = nullptr;
        hipEvent_t e0, e1;
        LT_TRY(prof_begin(h, LT_PROF_EXACT, &pc, &e0, &e1));
        LT_HIP(dispatch_solve(A, g, st, e0, e1));
        h->prof_host_bytes += bytes;
        return prof_end(h, LT_PROF_EXACT);
    }
    LT_HIP(dispatch_solve(A, g, st, nullptr, nullptr));
    return 0;
}

int invert_batch(hipStream_t st, double* mats, size_t ms, int nb, int count, int* flag) {
    if (count <= 0) return 0;
    for (int k0 = 0; k0 < nb; k0 += kGJW) {
        k_gj_panel<<<count, 256, 0, st>>>(mats, ms, nb, k0, flag);
        LT_HIP(hipGetLastError());
        k_gj_update<<<dim3(nblk(nb, kGJTI), count), 256, 0, st>>>(mats, ms, nb, k0);
        LT_HIP(hipGetLastError());
    }
    return 0;
}

int gemm_batch(hipStream_t st, int nb, int count, int ta, int tb, double alpha, double beta, const double* A0,
               size_t sA, const double* B0, size_t sB, double* C0, size_t sC) {
    if (count <= 0) return 0;
    const dim3 g(nblk(nb, kGT), nblk(nb, kGT), count);
    if (!ta && !tb) k_ex_gemm<0, 0><<<g, 256, 0, st>>>(nb, alpha, beta, A0, sA, B0, sB, C0, sC);
    else if (ta && !tb) k_ex_gemm<1, 0><<<g, 256, 0, st>>>(nb, alpha, beta, A0, sA, B0, sB, C0, sC);
    else if (!ta && tb) k_ex_gemm<0, 1><<<g, 256, 0, st>>>(nb, alpha, beta, A0, sA, B0, sB, C0, sC);
    else k_ex_gemm<1, 1><<<g, 256, 0, st>>>(nb, alpha, beta, A0, sA, B0, sB, C0, sC);
    LT_HIP(hipGetLastError());
    return 0;
}

// copy count blocks src[i * sstep] -> dst[i] (block strides in matrices)
int copy_blocks(hipStream_t st, double* dst, const double* src, size_t ms, int sstep, int count) {
    for (int i = 0; i < count; ++i)
        LT_HIP(hipMemcpyAsync(dst + (size_t)i * ms, src + (size_t)i * sstep * ms, ms * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
    return 0;
}

}  // namespace

int exact_slices(const lt_handle* h, int* nb, int* n) {
    const lt_grid& g = h->grid;
    if (g.ndim == 3) {
        *nb = g.n[0] * g.n[1];
        *n = g.n[2];
    } else {
        *nb = g.n[0];
        *n = g.n[1];
    }
    return 0;
}

void ExactFactor::release() {
    mats.release();
    valid = false;
}

const ExactFactor* exact_factor(lt_handle* h, cdouble tau, int* rc) {
    *rc = 0;
    if (h->exact_cache.capacity() < (size_t)kExactCache) h->exact_cache.reserve(kExactCache);
    for (auto& f : h->exact_cache)
        if (f.valid && f.tau == tau) {
            f.tick = ++h->exact_tick;
            return &f;
        }
    if (!(std::isfinite(tau.real()) && std::isfinite(tau.imag()))) {
        *rc = LT_EINVAL;
        set_last_error("exact preconditioner: the shift is not finite");
        return nullptr;
    }
    // Shifts for which elimination without pivoting is safe: Im tau != 0, or a real tau
    // >= 0 with K + tau M positive definite (tau = 0 needs a zero-head wall, or K is singular)
    bool dirichlet = false;
    for (int f = 0; f < 2 * h->grid.ndim; ++f) dirichlet = dirichlet || h->bc.face[f] == LT_BC_DIRICHLET0;
    if (tau.imag() == 0.0 && (tau.real() < 0.0 || (tau.real() == 0.0 && !dirichlet))) {
        *rc = LT_EINVAL;
        set_last_error("exact preconditioner: a real shift must be > 0 (or 0 with a zero-head wall)");
        return nullptr;
    }
    int nb = 0, n = 0;
    exact_slices(h, &nb, &n);
    if (n > 65535) {  // one workgroup layer per slice in a launch
        *rc = LT_EINVAL;
        set_last_error("exact preconditioner: more than 65535 slices along the last axis");
        return nullptr;
    }
    if (nb > kExactMaxBlock) {
        *rc = LT_EINVAL;
        set_last_error("exact preconditioner: a slice along the last axis has " + std::to_string(nb) +
                       " cells (at most " + std::to_string(kExactMaxBlock) + ")");
        return nullptr;
    }
    // slot for the factor: a free one, else the least recently used
    if (h->exact_cache.size() < (size_t)kExactCache) h->exact_cache.emplace_back();
    ExactFactor* F = nullptr;
    for (auto& f : h->exact_cache)
        if (!f.valid) {
            F = &f;
            break;
        }
    if (!F) {
        F = &h->exact_cache[0];
        for (auto& f : h->exact_cache)
            if (f.tick < F->tick) F = &f;
    }
    F->valid = false;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = h->stream;
    F->tau = tau;
    F->nb = nb;
    F->n = n;
    F->ms = 2 * (size_t)nb * nb;
    F->nl.assign(1, n);
    while (F->nl.back() > 1) F->nl.push_back((F->nl.back() + 1) / 2);
    // the tail: the first level above 0 whose whole reduced system has at most kExactTail
    // unknowns (one slice: level 0 itself) is inverted as one dense matrix
    int top = 0;
    if (n > 1) {
        top = 1;
        while (top + 1 < (int)F->nl.size() && (size_t)F->nl[top] * nb > (size_t)kExactTail) ++top;
    }
    F->nl.resize(top + 1);
    F->top = top;
    F->mtop = (size_t)F->nl[top] * nb;
    F->dinv.assign(top + 1, 0);
    F->pm.assign(top + 1, 0);
    F->qm.assign(top + 1, 0);
    F->ptm.assign(top + 1, 0);
    F->qtm.assign(top + 1, 0);
    size_t slots = 0;
    for (int l = 0; l < top; ++l) {
        F->dinv[l] = slots;
        slots += F->nl[l] / 2;
    }
    for (int l = 1; l < top; ++l) {
        F->pm[l] = slots;
        slots += F->nl[l] / 2;
        F->qm[l] = slots;
        slots += F->nl[l] / 2;
        F->ptm[l] = slots;
        slots += F->nl[l] / 2;
        F->qtm[l] = slots;
        slots += F->nl[l] / 2;
    }
    F->tail_off = slots * F->ms;
    const size_t mt = F->mtop, mst = 2 * mt * mt;  // the tail's doubles
    const size_t ms = F->ms;
    *rc = F->mats.reserve((F->tail_off + mst) * sizeof(double));
    if (*rc < 0) return nullptr;
    double* M = F->mats.as<double>();
    double* Mt = M + F->tail_off;
    const int half = (n + 1) / 2;
    double* tmp = top >= 1 ? wsp<double>(h, "ex_tmp", 4 * (size_t)half * ms, rc) : nullptr;
    if (top >= 1 && !tmp) return nullptr;
    int* flag = wsp<int>(h, "ex_flag", 1, rc);
    if (!flag) return nullptr;
    const LevelView<double> L = h->levels[0].v64();
    ExOp op{L.Tx, L.Ty, L.D, L.m, h->grid.n[0], h->grid.ndim, nb, tau.real(), tau.imag()};
    const double* Tl = h->grid.ndim == 3 ? L.Tz : L.Ty;
    const size_t nn = (size_t)nb * nb;
    auto fail = [&](int r) {
        *rc = r;
        return nullptr;
    };
    int r = 0;
    if (hipMemsetAsync(flag, 0, sizeof(int), st) != hipSuccess) return fail(LT_EHIP);
    if (n == 1) {
        k_ex_dense<<<dim3(nblk(nn, 256), 1), 256, 0, st>>>(op, 0, 1, Mt, mst);
        if (hipGetLastError() != hipSuccess) return fail(LT_EHIP);
        if ((r = invert_batch(st, Mt, mst, nb, 1, flag)) < 0) return fail(r);
    } else {
        // level 0: invert the odd slices, then the Schur step onto the even ones
        const int e0 = n / 2;
        k_ex_dense<<<dim3(nblk(nn, 256), e0), 256, 0, st>>>(op, 1, 2, M + F->dinv[0] * ms, ms);
        if (hipGetLastError() != hipSuccess) return fail(LT_EHIP);
        if ((r = invert_batch(st, M + F->dinv[0] * ms, ms, nb, e0, flag)) < 0) return fail(r);
        double* Dc = tmp;
        double* Dx = tmp + (size_t)half * ms;
        double* Fc = tmp + 2 * (size_t)half * ms;
        double* Fx = tmp + 3 * (size_t)half * ms;
        k_ex_schur0<<<dim3(nblk(nn, 256), F->nl[1]), 256, 0, st>>>(op, n, Tl, M + F->dinv[0] * ms, ms, Dc, Fc);
        if (hipGetLastError() != hipSuccess) return fail(LT_EHIP);
        for (int l = 1; l < top; ++l) {
            const int nl = F->nl[l], el = nl / 2, nq = (nl - 1) / 2, nn1 = F->nl[l + 1];
            double* Dv = M + F->dinv[l] * ms;
            double* Pm = M + F->pm[l] * ms;
            double* Qm = M + F->qm[l] * ms;
            if ((r = copy_blocks(st, Dv, Dc + ms, ms, 2, el)) < 0) return fail(r);
            if ((r = invert_batch(st, Dv, ms, nb, el, flag)) < 0) return fail(r);
            // P_s = Dinv_s F_{2s}^T, Q_s = Dinv_s F_{2s+1}
            if ((r = gemm_batch(st, nb, el, 0, 1, 1.0, 0.0, Dv, ms, Fc, 2 * ms, Pm, ms)) < 0) return fail(r);
            if ((r = gemm_batch(st, nb, nq, 0, 0, 1.0, 0.0, Dv, ms, Fc + ms, 2 * ms, Qm, ms)) < 0) return fail(r);
            // and their transposes (Dinv is symmetric): P_s^T = F_{2s} Dinv_s, Q_s^T = F_{2s+1}^T Dinv_s
            if ((r = gemm_batch(st, nb, el, 0, 0, 1.0, 0.0, Fc, 2 * ms, Dv, ms, M + F->ptm[l] * ms, ms)) < 0)
                return fail(r);
            if ((r = gemm_batch(st, nb, nq, 1, 0, 1.0, 0.0, Fc + ms, 2 * ms, Dv, ms, M + F->qtm[l] * ms, ms)) < 0)
                return fail(r);
            // D'_k = D_{2k} - F_{2k-1}^T Q_{k-1} - F_{2k} P_k;  F'_k = -F_{2k} Q_k
            if ((r = copy_blocks(st, Dx, Dc, ms, 2, nn1)) < 0) return fail(r);
            if ((r = gemm_batch(st, nb, nn1 - 1, 1, 0, -1.0, 1.0, Fc + ms, 2 * ms, Qm, ms, Dx + ms, ms)) < 0)
                return fail(r);
            if ((r = gemm_batch(st, nb, el, 0, 0, -1.0, 1.0, Fc, 2 * ms, Pm, ms, Dx, ms)) < 0) return fail(r);
            if ((r = gemm_batch(st, nb, nq, 0, 0, -1.0, 0.0, Fc, 2 * ms, Qm, ms, Fx, ms)) < 0) return fail(r);
            std::swap(Dc, Dx);
            std::swap(Fc, Fx);
        }
        // the tail: level top's blocks (D_i in Dc, F_i in Fc) as one dense matrix, inverted
        k_ex_tail<<<nblk(mt * mt, 256), 256, 0, st>>>(nb, F->nl[top], Dc, Fc, ms, Mt);
        if (hipGetLastError() != hipSuccess) return fail(LT_EHIP);
        if ((r = invert_batch(st, Mt, mst, (int)mt, 1, flag)) < 0) return fail(r);
    }
    int hf = 0;
    if (hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_last_error("exact preconditioner: factorisation failed on the device");
        return fail(LT_EHIP);
    }
    if (hf) {
        set_last_error("exact preconditioner: zero or non-finite pivot (K + tau M singular for this shift)");
        return fail(LT_EINVAL);
    }
    F->valid = true;
    F->tick = ++h->exact_tick;
    h->exact_factor_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ++h->exact_factorizations;
    return F;
}

int exact_apply(lt_handle* h, const ExactFactor* F, int R, const double* b, size_t brs, double* x, size_t xrs,
                const int* active) {
    if (R <= 0) return 0;
    hipStream_t st = h->stream;
    const int nb = F->nb, n = F->n, top = F->top;
    const size_t m = F->mtop;
    ExSolve A{};
    A.nb = nb;
    A.R = R;
    A.n = n;
    A.mats = F->mats.as<double>();
    A.ms = F->ms;
    A.tail = F->mats.as<double>() + F->tail_off;
    A.b = b;
    A.brs = brs;
    A.x = x;
    A.xrs = xrs;
    A.N = (size_t)h->N;
    A.active = active;
    A.ks = 1;
    const LevelView<double> L = h->levels[0].v64();
    A.Tl = h->grid.ndim == 3 ? L.Tz : L.Ty;
    const int nr = solve_nr(R);
    const unsigned gx = nblk(nb, 64), gy = nblk(R, nr);
    // algorithmic bytes: a dense block, a block of R vectors
    const double mb = (double)F->ms * sizeof(double), vb = 2.0 * R * nb * sizeof(double);
    const double tb = 2.0 * m * m * sizeof(double);  // the tail's matrix
    if (n == 1) {
        A.mode = kModeTop;
        A.nl = 1;
        return launch_solve(h, A, dim3(gx, gy, 1), tb + 2 * vb);
    }
    // workspaces: T0 (n/2 blocks), B_l and X_l for l = 1..top, the tail's partial products
    const size_t bs = 2 * (size_t)R * nb;
    auto lay = [&](int l) {
        return l == top ? ExLay{(size_t)nb, 2 * m, m} : ExLay{bs, 2 * (size_t)nb, (size_t)nb};
    };
    std::vector<size_t> boff(top + 1, 0), xoff(top + 1, 0);
    size_t tot = (size_t)(n / 2) * bs;
    for (int l = 1; l <= top; ++l) {
        boff[l] = tot;
        tot += (size_t)F->nl[l] * bs;
        xoff[l] = tot;
        tot += (size_t)F->nl[l] * bs;
    }
    // the tail's product: split its inner dimension so that the launch fills the GPU
    const unsigned gxt = nblk(m, 64);
    int ks = (int)std::min<size_t>(16, std::max<size_t>(1, 256 / ((size_t)gxt * gy)));
    ks = (int)std::min<size_t>(ks, std::max<size_t>(1, m / 64));
    const size_t poff = tot;
    if (ks > 1) tot += (size_t)ks * R * 2 * m;
    int rc = 0;
    double* W = wsp<double>(h, "ex_vec", tot, &rc);
    if (!W) return rc;
    // level 0: T0 = Dinv0 b_odd, then B1
    A.mode = kModeT0;
    A.nl = n;
    A.dinv = F->dinv[0];
    A.Xl = W;
    LT_TRY(launch_solve(h, A, dim3(gx, gy, n / 2), (n / 2) * (mb + 2 * vb)));
    k_ex_reduce0<<<dim3(nblk(bs, 256), F->nl[1]), 256, 0, st>>>(nb, R, n, b, brs, A.N, A.Tl, W, W + boff[1], lay(1));
    LT_HIP(hipGetLastError());
    for (int l = 1; l < top; ++l) {
        A.mode = kModeReduce;
        A.nl = F->nl[l];
        A.pm = F->pm[l];
        A.qm = F->qm[l];
        A.Bl = W + boff[l];
        A.Bn = W + boff[l + 1];
        A.ll = lay(l);
        A.ln = lay(l + 1);
        const int nl = F->nl[l], nn1 = F->nl[l + 1];
        LT_TRY(launch_solve(h, A, dim3(gx, gy, nn1), (nn1 - 1 + nl / 2) * mb + (nl + nn1) * vb));
    }
    // the tail: X_top = (dense inverse) B_top, contiguous [R][2][m]
    A.mode = kModeTop;
    A.nl = F->nl[top];
    A.nb = (int)m;
    A.Bl = W + boff[top];
    A.Xl = W + xoff[top];
    A.ll = lay(top);
    A.ks = ks;
    A.part = W + poff;
    LT_TRY(launch_solve(h, A, dim3(gxt, gy * ks, 1), tb + 2.0 * R * m * sizeof(double) * (ks > 1 ? ks : 1)));
    if (ks > 1) {
        const size_t len = (size_t)R * 2 * m;
        k_ex_sum_parts<<<nblk(len, 256), 256, 0, st>>>(len, ks, W + poff, W + xoff[top]);
        LT_HIP(hipGetLastError());
    }
    A.nb = nb;
    A.ks = 1;
    for (int l = top - 1; l >= 1; --l) {
        A.mode = kModeBack;
        A.nl = F->nl[l];
        A.dinv = F->dinv[l];
        A.ptm = F->ptm[l];
        A.qtm = F->qtm[l];
        A.Bl = W + boff[l];
        A.Xl = W + xoff[l];
        A.Xn = W + xoff[l + 1];
        A.ll = lay(l);
        A.ln = lay(l + 1);
        const int nl = F->nl[l], el = nl / 2, nq = (nl - 1) / 2;
        LT_TRY(launch_solve(h, A, dim3(gx, gy, nl), (2 * el + nq) * mb + (el + F->nl[l + 1] + nl) * vb));
    }
    A.mode = kModeBack0;
    A.nl = n;
    A.dinv = F->dinv[0];
    A.Xn = W + xoff[1];
    A.ln = lay(1);
    return launch_solve(h, A, dim3(gx, gy, n), (n / 2) * mb + (n / 2 + F->nl[1] + n) * vb);
}

size_t exact_matrix_bytes(const ExactFactor* F) {
    // dense blocks one solve reads: level 0's inverses twice (reduction and back
    // substitution), Dinv, P, Q, P^T, Q^T of each eliminated block of the levels below the
    // tail (each once), and the tail's dense inverse once
    size_t blocks = F->n > 1 ? 2 * (size_t)(F->n / 2) : 0;
    for (int l = 1; l < F->top; ++l) {
        const int el = F->nl[l] / 2, nq = (F->nl[l] - 1) / 2;
        blocks += 3 * (size_t)el + 2 * (size_t)nq;
    }
    return blocks * F->ms * sizeof(double) + 2 * F->mtop * F->mtop * sizeof(double);
}

}  // namespace lt
