// Fused 3D multigrid smoothing: z-marching tiles.
//
// A workgroup owns an xy tile of TX x TY cells (plus a halo of H = 2 nu cells)
// and a run of CZ planes, and marches through the planes from bottom to top.
// Every thread owns one pair of cells (x even, x odd) of a tile row, so it
// holds exactly one cell of each red-black colour per plane.  The nu
// red-black sweeps are a pipeline of 2 nu half-sweep stages: at step t stage
// s updates the cells of its colour in plane t - s + 1.  Stage s needs the
// other colour of planes p - 1, p, p + 1 after stage s - 1; plane p + 1
// reached that state earlier in the same step (stages run in increasing s)
// and plane p - 1 has not yet been touched by stage s + 1 (it reaches it
// later in the same step), so one barrier per step orders everything and the
// update is done in place.  The z neighbours of a cell live in the owning
// thread's registers (a ring of planes); only the four in-plane neighbours
// go through LDS.  Each stage shrinks the valid region by one cell in x and
// y (the halo is recomputed by neighbouring tiles, nothing is exchanged) and
// by one plane at each end of the run, so after 2 nu stages the interior
// holds exactly what global red-black sweeps produce.
//
// Pre-smoothing starts from x = 0 (the first stage needs no neighbours),
// then forms the residual b - A x of the interior and sums it over each
// aggregate into the coarse right-hand side.  Post-smoothing adds the
// prolongated coarse correction as each plane is loaded and writes to a
// separate buffer.  A level thus takes two launches per V-cycle instead of
// one launch per half-sweep plus the transfers.
#include "mg_fused.h"

#include <hip/hip_ext.h>

namespace lt {

template <typename T> struct V2T;
template <> struct V2T<float> { using type = float2; };
template <> struct V2T<double> { using type = double2; };

template <int NU, int TX, int TY> struct G3 {
    static constexpr int H = 2 * NU;          // halo: one cell per stage
    static constexpr int EX = TX + 2 * H, EY = TY + 2 * H;
    static constexpr int W = EX / 2;          // cell pairs per tile row
    static constexpr int NT = W * EY;         // threads: one per pair column
    static constexpr int RW = W + 2;          // LDS row with a guard entry at both ends
    static constexpr int PLANE = (EY + 2) * RW;  // one colour of one plane, guard rows included
    static constexpr int NS = 2 * NU + 1;     // planes held in LDS
    static constexpr int LR = 2 * NU + 3;     // planes held in registers
    static_assert(TX % 2 == 0 && TY % 2 == 0, "tiles start on even cells");
    static_assert(NT <= 1024, "one workgroup");
};

template <typename T> __device__ __forceinline__ typename V2T<T>::type mk2(T a, T b) {
    typename V2T<T>::type v;
    v.x = a;
    v.y = b;
    return v;
}

// Element idx of an array with a uniform base, addressed with a 32-bit byte offset
// (lt_setup limits a grid to 2^28 cells, so idx * 8 < 2^31).
template <typename T> __device__ __forceinline__ T ld(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ void stv(T* base, unsigned idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T)) = v;
}

// Values of one plane as loaded, before they are sorted by colour.
template <typename T, bool PRE> struct Raw3 {
    T b0r, b0i, b1r, b1i, d0, d1, m0, m1;
    T txw, txm, txe, tn0, tn1, ts0, ts1, tz0, tz1;
    // post-smoothing: x_in of both cells and the coarse values of the prolongation,
    // [z tap][y tap][x index a, b, c] (re, im)
    T x0r, x0i, x1r, x1i;
    T cr[PRE ? 1 : 2][PRE ? 1 : 2][PRE ? 1 : 3], ci[PRE ? 1 : 2][PRE ? 1 : 2][PRE ? 1 : 3];
    T wz0, wz1;
};

// Per-thread geometry of a tile (constant over the march).
struct Lane3 {
    int k, ly, lpos;
    bool iny, in0, in1, hasw, hass;
    unsigned o0, o1, oxw, os0, os1;
    // prolongation: x and y taps of the pair's cells in the coarse plane
    unsigned cy0, cy1, cxa, cxb, cxc;
    float wy0, wy1, wa0, wb0, wb1, wc1;
};

template <typename T, int NU, int TX, int TY, bool PRE>
__global__ __launch_bounds__((G3<NU, TX, TY>::NT)) void k_smooth3d(
    LevelView<T> L, T tr, T ti, const T* __restrict__ b, const T* __restrict__ xin, const T* __restrict__ ec,
    T* __restrict__ xout, T* __restrict__ bc, int cnx, int cny, int cnz, int cox, int coy, int coz, G6 ghost,
    int CZ, int ntx, const int* __restrict__ active, unsigned long long* __restrict__ prof, int Rtot) {
    using G = G3<NU, TX, TY>;
    using V = typename V2T<T>::type;
    constexpr int H = G::H, W = G::W, RW = G::RW, PLANE = G::PLANE, NS = G::NS, LR = G::LR;
    constexpr int NST = 2 * NU;
    __shared__ V sx[NS][2][PLANE];
    __shared__ V sred[PRE ? 2 : 1][PRE ? G::NT : 1][2];
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int tid = threadIdx.x;
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const unsigned NXY = (unsigned)nx * ny;
    const size_t N = L.N;
    const int bx = blockIdx.x % ntx, by = blockIdx.x / ntx;
    const int gx0 = bx * TX - H, gy0 = by * TY - H;
    const int z0 = blockIdx.y * CZ, z1 = min(z0 + CZ, nz);
    const T* bre = b + 2 * N * r;
    const T* bim = bre + N;

    for (int c = tid; c < NS * 2 * PLANE; c += G::NT) (&sx[0][0][0])[c] = mk2<T>(T(0), T(0));

    Lane3 ln;
    ln.k = tid % W;
    ln.ly = tid / W;
    ln.lpos = (ln.ly + 1) * RW + ln.k + 1;
    const int gxa = gx0 + 2 * ln.k, gy = gy0 + ln.ly;
    ln.iny = gy >= 0 && gy < ny;
    ln.in0 = ln.iny && gxa >= 0 && gxa < nx;
    ln.in1 = ln.iny && gxa + 1 >= 0 && gxa + 1 < nx;
    ln.hasw = ln.in0 && gxa >= 1;
    ln.hass = gy >= 1;
    {
        const int cx0 = min(max(gxa, 0), nx - 1), cx1 = min(max(gxa + 1, 0), nx - 1);
        const int cy = min(max(gy, 0), ny - 1), cys = max(cy - 1, 0);
        ln.o0 = (unsigned)(cx0 + nx * cy);
        ln.o1 = (unsigned)(cx1 + nx * cy);
        ln.oxw = (unsigned)(max(cx0 - 1, 0) + nx * cy);
        ln.os0 = (unsigned)(cx0 + nx * cys);
        ln.os1 = (unsigned)(cx1 + nx * cys);
        if (!PRE) {
            // y taps (ghost mirrored through the wall; a missing tap has weight 0)
            if (coy) {
                const int I = cy >> 1, J = (cy & 1) ? I + 1 : I - 1;
                const bool lo = J < 0, hi = J >= cny;
                ln.cy0 = (unsigned)I;
                ln.cy1 = (unsigned)((lo || hi) ? I : J);
                ln.wy0 = lo ? 0.75f + 0.25f * (float)ghost.g[2] : (hi ? 0.75f + 0.25f * (float)ghost.g[3] : 0.75f);
                ln.wy1 = (lo || hi) ? 0.f : 0.25f;
            } else {
                ln.cy0 = ln.cy1 = (unsigned)cy;
                ln.wy0 = 1.f;
                ln.wy1 = 0.f;
            }
            // x taps of the pair: cell 0 = a, b; cell 1 = b, c
            if (cox) {
                const int X = min(cx0 >> 1, cnx - 1);
                const bool lo = X - 1 < 0, hi = X + 1 >= cnx;
                ln.cxa = (unsigned)(lo ? X : X - 1);
                ln.cxb = (unsigned)X;
                ln.cxc = (unsigned)(hi ? X : X + 1);
                ln.wa0 = lo ? 0.f : 0.25f;
                ln.wb0 = lo ? 0.75f + 0.25f * (float)ghost.g[0] : 0.75f;
                ln.wb1 = hi ? 0.75f + 0.25f * (float)ghost.g[1] : 0.75f;
                ln.wc1 = hi ? 0.f : 0.25f;
            } else {
                ln.cxa = ln.cxb = (unsigned)cx0;
                ln.cxc = (unsigned)cx1;
                ln.wa0 = 1.f;
                ln.wb0 = 0.f;
                ln.wb1 = 0.f;
                ln.wc1 = 1.f;
            }
        }
    }
    const int lodd = ln.ly & 1;
    const bool interior = ln.k >= H / 2 && ln.k < H / 2 + TX / 2 && ln.ly >= H && ln.ly < H + TY && ln.iny &&
                          gxa < nx;
    const size_t Nc = (size_t)cnx * cny * cnz;
    const T* ecr = PRE ? nullptr : ec + 2 * Nc * r;
    const T* eci = PRE ? nullptr : ecr + Nc;
    const T* xir = PRE ? nullptr : xin + 2 * N * r;
    const T* xii = PRE ? nullptr : xir + N;
    T* xor_ = xout + 2 * N * r;
    T* xoi = xor_ + N;
    T* bcr = PRE ? bc + 2 * Nc * r : nullptr;
    T* bci = PRE ? bcr + Nc : nullptr;
    const unsigned CXY = (unsigned)cnx * cny;

    // register ring: [slot][colour]
    T xr[LR][2], xi[LR][2], br[LR][2], bi[LR][2], dr[LR][2], di[LR][2];
    T tn[LR][2], ts[LR][2], tz[LR][2], tl[LR][2], tm[LR];
#pragma unroll
    for (int s = 0; s < LR; ++s) {
        tm[s] = T(0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            xr[s][c] = xi[s][c] = br[s][c] = bi[s][c] = di[s][c] = T(0);
            dr[s][c] = T(1);
            tn[s][c] = ts[s][c] = tz[s][c] = tl[s][c] = T(0);
        }
    }
    // restriction state (PRE): partial sums over the planes of the current aggregate
    T zr0 = 0, zi0 = 0, zr1 = 0, zi1 = 0;
    int pend = -1;  // coarse plane whose y partner sums wait in sred[pend & 1]

    const int pl0 = z0 - H, pl1 = z1 + H - 1;  // planes loaded
    // stage s touches the planes it must make valid: the interior plus (H - s) planes
    // beyond each end (pre-smoothing: one more, its residual needs one ring of x)
    auto in_range = [&](int p, int s) {
        const int ext = H - s + (PRE ? 1 : 0);
        return p >= max(z0 - ext, 0) && p < min(z1 + ext, nz);
    };

    Raw3<T, PRE> raw;
    auto load_raw = [&](int p) {
        if (p < 0 || p >= nz || p < pl0 || p > pl1) return;
        const unsigned zo = (unsigned)p * NXY;
        raw.b0r = ld(bre, zo + ln.o0);
        raw.b0i = ld(bim, zo + ln.o0);
        raw.b1r = ld(bre, zo + ln.o1);
        raw.b1i = ld(bim, zo + ln.o1);
        raw.d0 = ld(L.D, zo + ln.o0);
        raw.d1 = ld(L.D, zo + ln.o1);
        raw.m0 = ld(L.m, zo + ln.o0);
        raw.m1 = ld(L.m, zo + ln.o1);
        raw.txw = ld(L.Tx, zo + ln.oxw);
        raw.txm = ld(L.Tx, zo + ln.o0);
        raw.txe = ld(L.Tx, zo + ln.o1);
        raw.tn0 = ld(L.Ty, zo + ln.o0);
        raw.tn1 = ld(L.Ty, zo + ln.o1);
        raw.ts0 = ld(L.Ty, zo + ln.os0);
        raw.ts1 = ld(L.Ty, zo + ln.os1);
        raw.tz0 = ld(L.Tz, zo + ln.o0);
        raw.tz1 = ld(L.Tz, zo + ln.o1);
        if (!PRE) {
            raw.x0r = ld(xir, zo + ln.o0);
            raw.x0i = ld(xii, zo + ln.o0);
            raw.x1r = ld(xir, zo + ln.o1);
            raw.x1i = ld(xii, zo + ln.o1);
            int iz0, iz1;
            if (coz) {
                const int I = p >> 1, J = (p & 1) ? I + 1 : I - 1;
                const bool lo = J < 0, hi = J >= cnz;
                iz0 = I;
                iz1 = (lo || hi) ? I : J;
                raw.wz0 = lo ? T(0.75) + T(0.25) * (T)ghost.g[4] : (hi ? T(0.75) + T(0.25) * (T)ghost.g[5] : T(0.75));
                raw.wz1 = (lo || hi) ? T(0) : T(0.25);
            } else {
                iz0 = iz1 = p;
                raw.wz0 = T(1);
                raw.wz1 = T(0);
            }
            const unsigned cz[2] = {(unsigned)iz0 * CXY, (unsigned)iz1 * CXY};
            const unsigned cyo[2] = {ln.cy0 * (unsigned)cnx, ln.cy1 * (unsigned)cnx};
            const unsigned cxs[3] = {ln.cxa, ln.cxb, ln.cxc};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        raw.cr[a][bb][c] = ld(ecr, cz[a] + cyo[bb] + cxs[c]);
                        raw.ci[a][bb][c] = ld(eci, cz[a] + cyo[bb] + cxs[c]);
                    }
        }
    };

    // sort the loaded plane p into ring slot S by colour (out-of-grid planes are all zero)
    auto process = [&](int p, auto Sc) {
        constexpr int S = decltype(Sc)::value;
        const bool inz = p >= max(pl0, 0) && p <= min(pl1, nz - 1);
        const bool in0 = inz && ln.in0, in1 = inz && ln.in1;
        // per cell (position order)
        T b0r = in0 ? raw.b0r : T(0), b0i = in0 ? raw.b0i : T(0);
        T b1r = in1 ? raw.b1r : T(0), b1i = in1 ? raw.b1i : T(0);
        T e0r = T(1), e0i = T(0), e1r = T(1), e1i = T(0);
        if (in0) {
            const T a = fma(tr, raw.m0, raw.d0), c = ti * raw.m0, q = T(1) / fma(a, a, c * c);
            e0r = a * q;
            e0i = -c * q;
        }
        if (in1) {
            const T a = fma(tr, raw.m1, raw.d1), c = ti * raw.m1, q = T(1) / fma(a, a, c * c);
            e1r = a * q;
            e1i = -c * q;
        }
        const T tw = (inz && ln.hasw) ? raw.txw : T(0);
        const T tmid = (in0 && in1) ? raw.txm : T(0);
        const T te = in1 ? raw.txe : T(0);
        const T n0 = in0 ? raw.tn0 : T(0), n1 = in1 ? raw.tn1 : T(0);
        const T s0 = (in0 && ln.hass) ? raw.ts0 : T(0), s1 = (in1 && ln.hass) ? raw.ts1 : T(0);
        const T z0v = in0 ? raw.tz0 : T(0), z1v = in1 ? raw.tz1 : T(0);
        T x0r = T(0), x0i = T(0), x1r = T(0), x1i = T(0);
        if (!PRE) {
            T p0r = 0, p0i = 0, p1r = 0, p1i = 0;
            const T wz[2] = {raw.wz0, raw.wz1};
            const T wy[2] = {(T)ln.wy0, (T)ln.wy1};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) {
                    const T w = wz[a] * wy[bb];
                    const T a0 = w * (T)ln.wa0, b0 = w * (T)ln.wb0, b1 = w * (T)ln.wb1, c1 = w * (T)ln.wc1;
                    p0r = fma(a0, raw.cr[a][bb][0], fma(b0, raw.cr[a][bb][1], p0r));
                    p0i = fma(a0, raw.ci[a][bb][0], fma(b0, raw.ci[a][bb][1], p0i));
                    p1r = fma(b1, raw.cr[a][bb][1], fma(c1, raw.cr[a][bb][2], p1r));
                    p1i = fma(b1, raw.ci[a][bb][1], fma(c1, raw.ci[a][bb][2], p1i));
                }
            x0r = in0 ? raw.x0r + p0r : T(0);
            x0i = in0 ? raw.x0i + p0i : T(0);
            x1r = in1 ? raw.x1r + p1r : T(0);
            x1i = in1 ? raw.x1i + p1i : T(0);
        }
        // cell ce of the pair has colour 0
        const bool ce = ((ln.ly + p) & 1) != 0;
        br[S][0] = ce ? b1r : b0r;
        bi[S][0] = ce ? b1i : b0i;
        br[S][1] = ce ? b0r : b1r;
        bi[S][1] = ce ? b0i : b1i;
        dr[S][0] = ce ? e1r : e0r;
        di[S][0] = ce ? e1i : e0i;
        dr[S][1] = ce ? e0r : e1r;
        di[S][1] = ce ? e0i : e1i;
        tn[S][0] = ce ? n1 : n0;
        tn[S][1] = ce ? n0 : n1;
        ts[S][0] = ce ? s1 : s0;
        ts[S][1] = ce ? s0 : s1;
        tz[S][0] = ce ? z1v : z0v;
        tz[S][1] = ce ? z0v : z1v;
        // the x face into the neighbouring pair: cell 0 looks west, cell 1 east
        tl[S][0] = ce ? te : tw;
        tl[S][1] = ce ? tw : te;
        tm[S] = tmid;
        xr[S][0] = ce ? x1r : x0r;
        xi[S][0] = ce ? x1i : x0i;
        xr[S][1] = ce ? x0r : x1r;
        xi[S][1] = ce ? x0i : x1i;
        if (!PRE) {
            V* pl = &sx[(p + NS) % NS][0][0];
            pl[ln.lpos] = mk2<T>(xr[S][0], xi[S][0]);
            pl[PLANE + ln.lpos] = mk2<T>(xr[S][1], xi[S][1]);
        }
    };

    // one Gauss-Seidel update of the colour-C cell of plane p (ring slots S, below Sm, above Sp)
    auto relax = [&](int p, auto Sc, auto Smc, auto Spc, auto Cc) {
        constexpr int S = decltype(Sc)::value, Sm = decltype(Smc)::value, Sp = decltype(Spc)::value;
        constexpr int C = decltype(Cc)::value;
        V* pl = &sx[(p + NS) % NS][0][0];
        const V* oth = pl + (1 - C) * PLANE;
        // this cell sits at x parity e = (C + ly + p) & 1: its neighbour in the next pair is east (e = 1)
        const int e = lodd ^ ((p + C) & 1);
        const V vn = oth[ln.lpos + RW], vs = oth[ln.lpos - RW], vx = oth[ln.lpos + 2 * e - 1];
        T nr = fma(tn[S][C], vn.x, fma(ts[S][C], vs.x, fma(tl[S][C], vx.x, br[S][C])));
        T ni = fma(tn[S][C], vn.y, fma(ts[S][C], vs.y, fma(tl[S][C], vx.y, bi[S][C])));
        nr = fma(tm[S], xr[S][1 - C], fma(tz[S][C], xr[Sp][1 - C], fma(tz[Sm][1 - C], xr[Sm][1 - C], nr)));
        ni = fma(tm[S], xi[S][1 - C], fma(tz[S][C], xi[Sp][1 - C], fma(tz[Sm][1 - C], xi[Sm][1 - C], ni)));
        const T vr = fma(nr, dr[S][C], -(ni * di[S][C]));
        const T vi = fma(nr, di[S][C], ni * dr[S][C]);
        xr[S][C] = vr;
        xi[S][C] = vi;
        pl[C * PLANE + ln.lpos] = mk2<T>(vr, vi);
    };

    // residual b - A x of the colour-C cell of plane p (x final)
    auto resid = [&](int p, auto Sc, auto Smc, auto Spc, auto Cc, T& rr, T& ri) {
        constexpr int S = decltype(Sc)::value, Sm = decltype(Smc)::value, Sp = decltype(Spc)::value;
        constexpr int C = decltype(Cc)::value;
        const V* oth = &sx[(p + NS) % NS][1 - C][0];
        const int e = lodd ^ ((p + C) & 1);
        const V vn = oth[ln.lpos + RW], vs = oth[ln.lpos - RW], vx = oth[ln.lpos + 2 * e - 1];
        T orr = fma(tn[S][C], vn.x, fma(ts[S][C], vs.x, tl[S][C] * vx.x));
        T oi = fma(tn[S][C], vn.y, fma(ts[S][C], vs.y, tl[S][C] * vx.y));
        orr = fma(tm[S], xr[S][1 - C], fma(tz[S][C], xr[Sp][1 - C], fma(tz[Sm][1 - C], xr[Sm][1 - C], orr)));
        oi = fma(tm[S], xi[S][1 - C], fma(tz[S][C], xi[Sp][1 - C], fma(tz[Sm][1 - C], xi[Sm][1 - C], oi)));
        // D + tau m from its inverse
        const T q = T(1) / fma(dr[S][C], dr[S][C], di[S][C] * di[S][C]);
        const T ar = dr[S][C] * q, ai = -di[S][C] * q;
        const T axr = fma(ar, xr[S][C], -(ai * xi[S][C])) - orr;
        const T axi = fma(ar, xi[S][C], ai * xr[S][C]) - oi;
        rr = br[S][C] - axr;
        ri = bi[S][C] - axi;
    };

    auto flush_coarse = [&]() {
        // y partner sums of coarse plane `pend` (rows ly, ly + 1 with ly even)
        if (pend >= 0 && interior && (!coy || (ln.ly & 1) == 0)) {
            const int bsel = pend & 1;
            V a0 = sred[PRE ? bsel : 0][PRE ? tid : 0][0], a1 = sred[PRE ? bsel : 0][PRE ? tid : 0][1];
            if (coy) {
                const V c0 = sred[PRE ? bsel : 0][PRE ? tid + W : 0][0], c1 = sred[PRE ? bsel : 0][PRE ? tid + W : 0][1];
                a0.x += c0.x;
                a0.y += c0.y;
                a1.x += c1.x;
                a1.y += c1.y;
            }
            const int Y = coy ? gy >> 1 : gy;
            const unsigned base = (unsigned)pend * CXY + (unsigned)Y * cnx;
            if (cox) {
                const unsigned I = base + (unsigned)(gxa >> 1);
                stv(bcr, I, a0.x);
                stv(bci, I, a0.y);
            } else {
                stv(bcr, base + (unsigned)gxa, a0.x);
                stv(bci, base + (unsigned)gxa, a0.y);
                if (gxa + 1 < nx) {
                    stv(bcr, base + (unsigned)gxa + 1, a1.x);
                    stv(bci, base + (unsigned)gxa + 1, a1.y);
                }
            }
        }
        pend = -1;
    };

    // one step of the march at plane t; U = (t - pl0) mod LR
    auto step = [&](int t, auto Uc) {
        constexpr int U = decltype(Uc)::value;
        constexpr int S1 = (U + 1) % LR;
        if (PRE) flush_coarse();
        // plane t + 1 enters the ring; plane t + 2 is fetched
        process(t + 1, std::integral_constant<int, S1>{});
        load_raw(t + 2);
        // stages in increasing order
        if (PRE) {
            // stage 1 from x = 0: colour 0 = b / d, colour 1 = 0
            if (in_range(t, 1)) {
                constexpr int S = U % LR;
                const T vr = fma(br[S][0], dr[S][0], -(bi[S][0] * di[S][0]));
                const T vi = fma(br[S][0], di[S][0], bi[S][0] * dr[S][0]);
                xr[S][0] = vr;
                xi[S][0] = vi;
                xr[S][1] = xi[S][1] = T(0);
                V* pl = &sx[(t + NS) % NS][0][0];
                pl[ln.lpos] = mk2<T>(vr, vi);
                pl[PLANE + ln.lpos] = mk2<T>(T(0), T(0));
            }
        }
#pragma unroll
        for (int s0 = PRE ? 2 : 1; s0 <= NST; ++s0) {
            // (a compile-time loop: every index below is a constant after unrolling)
            const int p = t - s0 + 1;
            if (in_range(p, s0)) {
                auto go = [&](auto Sc) {
                    constexpr int S = decltype(Sc)::value;
                    constexpr int Sm = (S + LR - 1) % LR, Sp = (S + 1) % LR;
                    if (((PRE ? s0 - 1 : s0) & 1) == 0)
                        relax(p, Sc, std::integral_constant<int, Sm>{}, std::integral_constant<int, Sp>{},
                              std::integral_constant<int, 0>{});
                    else
                        relax(p, Sc, std::integral_constant<int, Sm>{}, std::integral_constant<int, Sp>{},
                              std::integral_constant<int, 1>{});
                };
                switch (s0) {  // slot of plane p = (U - s0 + 1) mod LR
#define LT_S(SS) case SS: go(std::integral_constant<int, ((U - SS + 1) % LR + LR) % LR>{}); break;
                    LT_S(1) LT_S(2) LT_S(3) LT_S(4) LT_S(5) LT_S(6)
#undef LT_S
                    default: break;
                }
            }
        }
        // final x of plane t - 2 nu + 1
        {
            const int p = t - NST + 1;
            constexpr int S = ((U - NST + 1) % LR + LR) % LR;
            if (p >= z0 && p < z1 && interior) {
                const bool ce = ((ln.ly + p) & 1) != 0;
                const unsigned zo = (unsigned)p * NXY;
                stv(xor_, zo + ln.o0, ce ? xr[S][1] : xr[S][0]);
                stv(xoi, zo + ln.o0, ce ? xi[S][1] : xi[S][0]);
                if (gxa + 1 < nx) {
                    stv(xor_, zo + ln.o1, ce ? xr[S][0] : xr[S][1]);
                    stv(xoi, zo + ln.o1, ce ? xi[S][0] : xi[S][1]);
                }
            }
        }
        if (PRE) {
            // residual of plane t - 2 nu, summed into the aggregate
            const int p = t - NST;
            constexpr int S = ((U - NST) % LR + LR) % LR;
            constexpr int Sm = (S + LR - 1) % LR, Sp = (S + 1) % LR;
            if (p >= z0 && p < z1) {
                T r0r, r0i, r1r, r1i;
                resid(p, std::integral_constant<int, S>{}, std::integral_constant<int, Sm>{},
                      std::integral_constant<int, Sp>{}, std::integral_constant<int, 0>{}, r0r, r0i);
                resid(p, std::integral_constant<int, S>{}, std::integral_constant<int, Sm>{},
                      std::integral_constant<int, Sp>{}, std::integral_constant<int, 1>{}, r1r, r1i);
                const bool ce = ((ln.ly + p) & 1) != 0;
                // position order
                T a0r = ce ? r1r : r0r, a0i = ce ? r1i : r0i, a1r = ce ? r0r : r1r, a1i = ce ? r0i : r1i;
                if (!(gxa + 1 < nx)) a1r = a1i = T(0);
                if (cox) {
                    a0r += a1r;
                    a0i += a1i;
                }
                zr0 += a0r;
                zi0 += a0i;
                zr1 += a1r;
                zi1 += a1i;
                if (!coz || (p & 1)) {
                    const int Z = coz ? p >> 1 : p;
                    sred[PRE ? (Z & 1) : 0][PRE ? tid : 0][0] = mk2<T>(zr0, zi0);
                    sred[PRE ? (Z & 1) : 0][PRE ? tid : 0][1] = mk2<T>(zr1, zi1);
                    zr0 = zi0 = zr1 = zi1 = T(0);
                    pend = Z;
                }
            }
        }
        __syncthreads();
    };

    // prologue: plane pl0 into slot 0, plane pl0 + 1 fetched
    load_raw(pl0);
    process(pl0, std::integral_constant<int, 0>{});
    load_raw(pl0 + 1);
    __syncthreads();
    const int tlast = PRE ? z1 - 1 + NST : z1 - 1 + NST - 1;
    for (int t0 = pl0; t0 <= tlast; t0 += LR) {
#define LT_U(UU) \
    if constexpr (LR > UU) { if (t0 + UU <= tlast) step(t0 + UU, std::integral_constant<int, UU>{}); }
        LT_U(0) LT_U(1) LT_U(2) LT_U(3) LT_U(4) LT_U(5) LT_U(6) LT_U(7) LT_U(8)
#undef LT_U
    }
    if (PRE) flush_coarse();

    if (prof && tid == 0 && blockIdx.x == 0 && blockIdx.y == 0) {
        // algorithmic bytes of this right-hand side over the level (one count per right-hand
        // side and launch): pre: b in, x out, coarse rhs out; post: x in, b in, x out, coarse
        // correction in; the coefficient arrays Tx, Ty, Tz, D, m are shared by the Rtot
        // right-hand sides
        const double cell = (PRE ? 4.0 : 6.0) * sizeof(T) + 5.0 * sizeof(T) / Rtot;
        atomicAdd(prof, (unsigned long long)((double)N * cell + (double)Nc * 2.0 * sizeof(T)));
    }
}

// ------------------------------------------------------------------ launchers
// z run per workgroup: the whole depth unless the launch would have fewer than
// ~4 workgroups per compute unit, then halved (kept even, at least 8 planes)
static int pick_cz(int nz, int nxy_tiles, int R) {
    int cz = nz + (nz & 1);
    while (cz > 8 && (long long)nxy_tiles * R * ((nz + cz - 1) / cz) < 1024) {
        cz = (cz + 1) / 2;
        cz += cz & 1;
    }
    return cz;
}

template <typename T, bool PRE>
static int launch_smooth3d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b,
                           const T* xin, const T* ec, T* xout, T* bc, int cnx, int cny, int cnz, int cox, int coy,
                           int coz, G6 ghost, int R, const int* active, unsigned long long* prof, hipEvent_t ev0,
                           hipEvent_t ev1) {
    if (sizeof(T) != 4 || nu < 1 || nu > 2) {
        set_last_error("fused 3D smoother: FP32 with 1 or 2 sweeps");
        return LT_EUNSUPPORTED;
    }
#define LT_K3(NU, X, Y)                                                                                         \
    do {                                                                                                       \
        using G = G3<NU, X, Y>;                                                                                \
        const int ntx = (L.nx + X - 1) / X, nty = (L.ny + Y - 1) / Y;                                          \
        const int cz = pick_cz(L.nz, ntx * nty, R);                                                            \
        const dim3 grid(ntx * nty, (L.nz + cz - 1) / cz, R);                                                   \
        if (ev0)                                                                                               \
            hipExtLaunchKernelGGL((k_smooth3d<T, NU, X, Y, PRE>), grid, dim3(G::NT), 0, st, ev0, ev1, 0, L, tr, ti, \
                                  b, xin, ec, xout, bc, cnx, cny, cnz, cox, coy, coz, ghost, cz, ntx, active, prof, R); \
        else                                                                                                   \
            k_smooth3d<T, NU, X, Y, PRE><<<grid, G::NT, 0, st>>>(L, tr, ti, b, xin, ec, xout, bc, cnx, cny, cnz,   \
                                                                 cox, coy, coz, ghost, cz, ntx, active, prof, R);   \
    } while (0)
#define LT_T3(X, Y) \
    if (nu == 1) LT_K3(1, X, Y); else LT_K3(2, X, Y)
    if constexpr (sizeof(T) == 4) {
        switch (tile) {
            case 0: LT_T3(32, 8); break;
            case 1: LT_T3(16, 8); break;
            default: set_last_error("unknown 3D tile shape"); return LT_EINVAL;
        }
    }
#undef LT_T3
#undef LT_K3
    LT_HIP(hipGetLastError());
    return 0;
}

template <typename T>
int launch_pre3d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b, T* x, int cnx,
                 int cny, int cnz, int cox, int coy, int coz, T* bc, int R, const int* active,
                 unsigned long long* prof, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_smooth3d<T, true>(st, L, tr, ti, nu, tile, b, nullptr, nullptr, x, bc, cnx, cny, cnz, cox, coy,
                                    coz, G6{}, R, active, prof, ev0, ev1);
}

template <typename T>
int launch_post3d(hipStream_t st, const LevelView<T>& L, T tr, T ti, int nu, int tile, const T* b, const T* xin,
                  const T* ec, int cnx, int cny, int cnz, int cox, int coy, int coz, G6 ghost, T* xout, int R,
                  const int* active, unsigned long long* prof, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_smooth3d<T, false>(st, L, tr, ti, nu, tile, b, xin, ec, xout, nullptr, cnx, cny, cnz, cox, coy,
                                     coz, ghost, R, active, prof, ev0, ev1);
}

template int launch_pre3d<float>(hipStream_t, const LevelView<float>&, float, float, int, int, const float*, float*,
                                 int, int, int, int, int, int, float*, int, const int*, unsigned long long*,
                                 hipEvent_t, hipEvent_t);
template int launch_pre3d<double>(hipStream_t, const LevelView<double>&, double, double, int, int, const double*,
                                  double*, int, int, int, int, int, int, double*, int, const int*,
                                  unsigned long long*, hipEvent_t, hipEvent_t);
template int launch_post3d<float>(hipStream_t, const LevelView<float>&, float, float, int, int, const float*,
                                  const float*, const float*, int, int, int, int, int, int, G6, float*, int,
                                  const int*, unsigned long long*, hipEvent_t, hipEvent_t);
template int launch_post3d<double>(hipStream_t, const LevelView<double>&, double, double, int, int, const double*,
                                   const double*, const double*, int, int, int, int, int, int, G6, double*, int,
                                   const int*, unsigned long long*, hipEvent_t, hipEvent_t);

}  // namespace lt
