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
// The inputs of a plane (right-hand side, coefficients, and for the
// post-smoother the incoming iterate and the coarse correction) are staged
// in LDS by direct global-to-LDS loads, MS planes at a time and one group of
// planes ahead (double buffered), so the loads of the next planes are in
// flight while the current ones are smoothed and no register holds them.
//
// Pre-smoothing starts from x = 0 (the first stage needs no neighbours),
// then forms the residual b - A x of the interior and sums it over each
// aggregate into the coarse right-hand side.  Post-smoothing adds the
// prolongated coarse correction as each plane enters and writes to a
// separate buffer.  A level thus takes two launches per V-cycle instead of
// one launch per half-sweep plus the transfers.  FP32 cycles, 1 or 2 sweeps,
// levels coarsened in x and y.
#include "mg_fused.h"

#include <hip/hip_ext.h>

namespace lt {

namespace {

typedef __attribute__((address_space(3))) void lds_void;

template <int NU, int TX, int TY> struct G3 {
    static constexpr int H = 2 * NU;          // halo: one cell per stage
    static constexpr int EX = TX + 2 * H, EY = TY + 2 * H;
    static constexpr int W = EX / 2;          // cell pairs per tile row
    static constexpr int NT = W * EY;         // threads: one per pair column
    static constexpr int RW = W + 2;          // LDS row with a guard entry at both ends
    static constexpr int PLANE = (EY + 2) * RW;  // one colour of one plane, guard rows included
    static constexpr int NS = 2 * NU + 1;     // planes of iterates in LDS
    static constexpr int LR = 2 * NU + 3;     // planes held in registers
    static constexpr int MS = 2;              // planes staged per group
    static constexpr int PW = W + 2, PH = EY / 2 + 2;  // coarse patch of the prolongation
    static constexpr int NCL = (PW * PH + NT - 1) / NT;  // coarse patch loads per thread and array
    static constexpr int CSL = 3;             // coarse planes a group of MS fine planes reads
    static_assert(TX % 2 == 0 && TY % 2 == 0, "tiles start on even cells");
    static_assert(NT <= 1024, "one workgroup");
    static_assert(MS == 2, "CSL covers two fine planes");
};

// staged values of one plane, per thread (position order: cell 0 = x even, cell 1 = x odd)
enum { B0R, B0I, B1R, B1I, D0, D1, M0, M1, TXM, TXE, TN0, TN1, TZ0, TZ1, X0R, X0I, X1R, X1I, NV_POST };
constexpr int NV_PRE = X0R;

// One dword per lane from global memory straight into LDS: lane i of the
// wavefront writes lds_wave[i].  lds_wave must be the same for the whole wavefront.
__device__ __forceinline__ void dma(const float* g, float* lds_wave) {
    __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)lds_wave, 4, 0, 0);
}

__device__ __forceinline__ float2 mk2(float a, float b) {
    float2 v;
    v.x = a;
    v.y = b;
    return v;
}

// Element idx of an array with a uniform base, addressed with a 32-bit byte offset
// (lt_setup limits a grid to 2^28 cells, so idx * 8 < 2^31).
__device__ __forceinline__ const float* at(const float* base, unsigned idx) {
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + idx * 4u);
}
__device__ __forceinline__ void stv(float* base, unsigned idx, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + idx * 4u) = v;
}

template <int K> using IC = std::integral_constant<int, K>;

}  // namespace

template <int NU, int TX, int TY, bool PRE>
__global__ __launch_bounds__((G3<NU, TX, TY>::NT)) void k_smooth3d(
    LevelView<float> L, float tr, float ti, const float* __restrict__ b, const float* __restrict__ xin,
    const float* __restrict__ ec, float* __restrict__ xout, float* __restrict__ bc, int cnx, int cny, int cnz,
    int coz, G6 ghost, int CZ, int ntx, const int* __restrict__ active, unsigned long long* __restrict__ prof,
    int Rtot) {
    using G = G3<NU, TX, TY>;
    using V = float2;
    constexpr int H = G::H, W = G::W, RW = G::RW, PLANE = G::PLANE, NS = G::NS, LR = G::LR, NT = G::NT;
    constexpr int MS = G::MS, PW = G::PW, PH = G::PH, NCL = G::NCL, CSL = G::CSL;
    constexpr int NST = 2 * NU;
    constexpr int NV = PRE ? NV_PRE : NV_POST;
    __shared__ V sx[NS][2][PLANE];
    __shared__ float stg[2 * MS][NV][NT];
    __shared__ float cst[PRE ? 1 : 2][PRE ? 1 : CSL][2][PRE ? 1 : NCL * NT];
    __shared__ V sred[PRE ? 2 : 1][PRE ? NT : 1];
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int tid = threadIdx.x;
    const int wv = tid & ~63;  // first thread of this wavefront
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const unsigned NXY = (unsigned)nx * ny;
    const size_t N = L.N;
    const int bx = blockIdx.x % ntx, by = blockIdx.x / ntx;
    const int gx0 = bx * TX - H, gy0 = by * TY - H;
    const int z0 = blockIdx.y * CZ, z1 = min(z0 + CZ, nz);
    const float* bre = b + 2 * N * r;
    const float* bim = bre + N;

    for (int c = tid; c < NS * 2 * PLANE; c += NT) (&sx[0][0][0])[c] = mk2(0.f, 0.f);

    // ---- per-thread geometry (constant over the march)
    const int k = tid % W, ly = tid / W;
    const int lpos = (ly + 1) * RW + k + 1;
    const int gxa = gx0 + 2 * k, gy = gy0 + ly;
    const bool iny = gy >= 0 && gy < ny;
    const bool lin0 = iny && gxa >= 0 && gxa < nx;
    const bool lin1 = iny && gxa + 1 >= 0 && gxa + 1 < nx;
    const bool hasw = lin0 && gxa >= 1 && k > 0;
    const bool hass = gy >= 1 && ly > 0;
    const int cx0 = min(max(gxa, 0), nx - 1), cx1 = min(max(gxa + 1, 0), nx - 1);
    const int cy = min(max(gy, 0), ny - 1);
    const unsigned o0 = (unsigned)(cx0 + nx * cy), o1 = (unsigned)(cx1 + nx * cy);
    const int lodd = ly & 1;
    const bool interior = k >= H / 2 && k < H / 2 + TX / 2 && ly >= H && ly < H + TY && iny && gxa < nx;
    // prolongation taps in the coarse patch (x and y halved; the patch starts one coarse
    // cell before the tile): rows pr0 (weight wy0), pr1 (wy1); cell 0 takes columns ca, cb,
    // cell 1 cb, cc; a tap beyond a wall folds into the boundary cell with the ghost parity
    int pr0 = 0, pr1 = 0, ca = 0, cb = 0, cc = 0;
    float wy0 = 0.f, wy1 = 0.f, wa0 = 0.f, wb0 = 0.f, wb1 = 0.f, wc1 = 0.f;
    const int px0 = (gx0 >> 1) - 1, py0 = (gy0 >> 1) - 1;
    if (!PRE) {
        const int Y = gy >> 1, J = (gy & 1) ? Y + 1 : Y - 1;
        const bool lo = J < 0, hi = J >= cny;
        pr0 = (Y - py0) * PW;
        pr1 = ((lo || hi) ? Y - py0 : J - py0) * PW;
        wy0 = lo ? 0.75f + 0.25f * (float)ghost.g[2] : (hi ? 0.75f + 0.25f * (float)ghost.g[3] : 0.75f);
        wy1 = (lo || hi) ? 0.f : 0.25f;
        const int X = gxa >> 1;
        const bool xlo = X - 1 < 0, xhi = X + 1 >= cnx;
        cb = X - px0;
        ca = xlo ? cb : cb - 1;
        cc = xhi ? cb : cb + 1;
        wa0 = xlo ? 0.f : 0.25f;
        wb0 = xlo ? 0.75f + 0.25f * (float)ghost.g[0] : 0.75f;
        wb1 = xhi ? 0.75f + 0.25f * (float)ghost.g[1] : 0.75f;
        wc1 = xhi ? 0.f : 0.25f;
    }
    const size_t Nc = (size_t)cnx * cny * cnz;
    const unsigned CXY = (unsigned)cnx * cny;
    const float* ecr = PRE ? nullptr : ec + 2 * Nc * r;
    const float* eci = PRE ? nullptr : ecr + Nc;
    const float* xir = PRE ? nullptr : xin + 2 * N * r;
    const float* xii = PRE ? nullptr : xir + N;
    float* xor_ = xout + 2 * N * r;
    float* xoi = xor_ + N;
    float* bcr = PRE ? bc + 2 * Nc * r : nullptr;
    float* bci = PRE ? bcr + Nc : nullptr;

    const int pl0 = z0 - H, pl1 = z1 + H - 1;  // planes the run reads
    const int qlo = max(pl0, 0), qhi = min(pl1, nz - 1);

    // ---- staging: group g holds planes pl0 + g MS + 1 .. pl0 + (g + 1) MS in buffer g & 1;
    // plane pl0 is staged in the last slot of buffer 1 before the march
    auto slot_of = [&](int q) {
        return q == pl0 ? 2 * MS - 1 : (((q - pl0 - 1) / MS) & 1) * MS + (q - pl0 - 1) % MS;
    };
    auto stage_plane = [&](int q, int sl) {
        if (q < qlo || q > qhi) return;
        const unsigned zo = (unsigned)q * NXY;
        float* s = &stg[sl][0][wv];
        dma(at(bre, zo + o0), s + B0R * NT);
        dma(at(bim, zo + o0), s + B0I * NT);
        dma(at(bre, zo + o1), s + B1R * NT);
        dma(at(bim, zo + o1), s + B1I * NT);
        dma(at(L.D, zo + o0), s + D0 * NT);
        dma(at(L.D, zo + o1), s + D1 * NT);
        dma(at(L.m, zo + o0), s + M0 * NT);
        dma(at(L.m, zo + o1), s + M1 * NT);
        dma(at(L.Tx, zo + o0), s + TXM * NT);
        dma(at(L.Tx, zo + o1), s + TXE * NT);
        dma(at(L.Ty, zo + o0), s + TN0 * NT);
        dma(at(L.Ty, zo + o1), s + TN1 * NT);
        dma(at(L.Tz, zo + o0), s + TZ0 * NT);
        dma(at(L.Tz, zo + o1), s + TZ1 * NT);
        if (!PRE) {
            dma(at(xir, zo + o0), s + X0R * NT);
            dma(at(xii, zo + o0), s + X0I * NT);
            dma(at(xir, zo + o1), s + X1R * NT);
            dma(at(xii, zo + o1), s + X1I * NT);
        }
    };
    // coarse planes the prolongation of fine plane q reads (taps I, J; J = I when missing)
    auto ztaps = [&](int q, int& I, int& J, float& w0, float& w1) {
        const int qq = min(max(q, 0), nz - 1);
        if (coz) {
            I = qq >> 1;
            const int j = (qq & 1) ? I + 1 : I - 1;
            const bool lo = j < 0, hi = j >= cnz;
            J = (lo || hi) ? I : j;
            w0 = lo ? 0.75f + 0.25f * (float)ghost.g[4] : (hi ? 0.75f + 0.25f * (float)ghost.g[5] : 0.75f);
            w1 = (lo || hi) ? 0.f : 0.25f;
        } else {
            I = J = qq;
            w0 = 1.f;
            w1 = 0.f;
        }
    };
    // lowest coarse plane read by fine planes qa..qb
    auto zlow = [&](int qa, int qb) {
        int I, J, lo = 1 << 30;
        float w0, w1;
        for (int q = qa; q <= qb; ++q) {
            ztaps(q, I, J, w0, w1);
            lo = min(lo, min(I, J));
        }
        return lo;
    };
    // coarse planes of fine planes qa..qb into coarse buffer cbuf (slot Z - zlow)
    auto stage_coarse = [&](int qa, int qb, int cbuf) {
        int I, J, zl = 1 << 30, zh = -1;
        float w0, w1;
        for (int q = qa; q <= qb; ++q) {
            ztaps(q, I, J, w0, w1);
            zl = min(zl, min(I, J));
            zh = max(zh, max(I, J));
        }
        for (int Z = zl; Z <= zh && Z - zl < CSL; ++Z) {
            const unsigned zo = (unsigned)Z * CXY;
#pragma unroll
            for (int kk = 0; kk < NCL; ++kk) {
                const int e = min(tid + kk * NT, PW * PH - 1);
                const int X = min(max(px0 + e % PW, 0), cnx - 1), Y = min(max(py0 + e / PW, 0), cny - 1);
                const unsigned J2 = zo + (unsigned)(X + cnx * Y);
                dma(at(ecr, J2), &cst[cbuf][Z - zl][0][kk * NT + wv]);
                dma(at(eci, J2), &cst[cbuf][Z - zl][1][kk * NT + wv]);
            }
        }
    };

    // ---- register ring: [slot][colour]
    float xr[LR][2], xi[LR][2], br[LR][2], bi[LR][2], dr[LR][2], di[LR][2];
    float tn[LR][2], ts[LR][2], tz[LR][2], tl[LR][2], tm[LR];
#pragma unroll
    for (int s = 0; s < LR; ++s) {
        tm[s] = 0.f;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            xr[s][c] = xi[s][c] = br[s][c] = bi[s][c] = di[s][c] = 0.f;
            dr[s][c] = 1.f;
            tn[s][c] = ts[s][c] = tz[s][c] = tl[s][c] = 0.f;
        }
    }
    float zr0 = 0.f, zi0 = 0.f;  // restriction: sum over the aggregate's planes so far
    int pend = -1;  // coarse plane whose y partner sums wait in sred[pend & 1]

    // stage s touches the planes it must make valid: the interior plus (H - s) planes
    // beyond each end (pre-smoothing: one more, its residual needs one ring of x)
    auto in_range = [&](int p, int s) {
        const int ext = H - s + (PRE ? 1 : 0);
        return p >= max(z0 - ext, 0) && p < min(z1 + ext, nz);
    };

    // plane p from its staging slot into ring slot S, sorted by colour (planes outside the
    // grid or the run are all zero)
    auto process = [&](int p, auto Sc) {
        constexpr int S = decltype(Sc)::value;
        const bool inz = p >= qlo && p <= qhi;
        const bool in0 = inz && lin0, in1 = inz && lin1;
        const float* sv = &stg[slot_of(p)][0][0];
        auto g = [&](int v) { return sv[v * NT + tid]; };
        const float b0r = in0 ? g(B0R) : 0.f, b0i = in0 ? g(B0I) : 0.f;
        const float b1r = in1 ? g(B1R) : 0.f, b1i = in1 ? g(B1I) : 0.f;
        float e0r = 1.f, e0i = 0.f, e1r = 1.f, e1i = 0.f;
        {
            const float a = fmaf(tr, g(M0), g(D0)), c = ti * g(M0), q = 1.f / fmaf(a, a, c * c);
            if (in0) {
                e0r = a * q;
                e0i = -c * q;
            }
        }
        {
            const float a = fmaf(tr, g(M1), g(D1)), c = ti * g(M1), q = 1.f / fmaf(a, a, c * c);
            if (in1) {
                e1r = a * q;
                e1i = -c * q;
            }
        }
        // the west face is the east face of the pair to the left, the south faces the
        // north faces of the row below (staged by those threads)
        const float tw = (inz && hasw) ? sv[TXE * NT + tid - 1] : 0.f;
        const float tmid = (in0 && in1) ? g(TXM) : 0.f;
        const float te = in1 ? g(TXE) : 0.f;
        const float n0 = in0 ? g(TN0) : 0.f, n1 = in1 ? g(TN1) : 0.f;
        const float s0 = (in0 && hass) ? sv[TN0 * NT + tid - W] : 0.f;
        const float s1 = (in1 && hass) ? sv[TN1 * NT + tid - W] : 0.f;
        const float z0v = in0 ? g(TZ0) : 0.f, z1v = in1 ? g(TZ1) : 0.f;
        float x0r = 0.f, x0i = 0.f, x1r = 0.f, x1i = 0.f;
        if (!PRE) {
            int I, J;
            float w0, w1;
            ztaps(p, I, J, w0, w1);
            const int cbuf = p == pl0 ? 1 : ((p - pl0 - 1) / MS) & 1;
            const int qa = p == pl0 ? pl0 : pl0 + ((p - pl0 - 1) / MS) * MS + 1;
            const int zl = zlow(qa, p == pl0 ? pl0 : qa + MS - 1);
            const float* PI = &cst[cbuf][I - zl][0][0];
            const float* PJ = &cst[cbuf][J - zl][0][0];
            constexpr int NP = NCL * NT;
            float p0r = 0.f, p0i = 0.f, p1r = 0.f, p1i = 0.f;
#pragma unroll
            for (int zz = 0; zz < 2; ++zz) {
                const float* P = zz ? PJ : PI;
                const float wz = zz ? w1 : w0;
#pragma unroll
                for (int yy = 0; yy < 2; ++yy) {
                    const int row = yy ? pr1 : pr0;
                    const float w = wz * (yy ? wy1 : wy0);
                    const float ar = P[row + ca], ai = P[NP + row + ca];
                    const float br2 = P[row + cb], bi2 = P[NP + row + cb];
                    const float cr = P[row + cc], ci = P[NP + row + cc];
                    p0r = fmaf(w * wa0, ar, fmaf(w * wb0, br2, p0r));
                    p0i = fmaf(w * wa0, ai, fmaf(w * wb0, bi2, p0i));
                    p1r = fmaf(w * wb1, br2, fmaf(w * wc1, cr, p1r));
                    p1i = fmaf(w * wb1, bi2, fmaf(w * wc1, ci, p1i));
                }
            }
            x0r = in0 ? g(X0R) + p0r : 0.f;
            x0i = in0 ? g(X0I) + p0i : 0.f;
            x1r = in1 ? g(X1R) + p1r : 0.f;
            x1i = in1 ? g(X1I) + p1i : 0.f;
        }
        // cell ce of the pair has colour 0
        const bool ce = ((ly + p) & 1) != 0;
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
            pl[lpos] = mk2(xr[S][0], xi[S][0]);
            pl[PLANE + lpos] = mk2(xr[S][1], xi[S][1]);
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
        const V vn = oth[lpos + RW], vs = oth[lpos - RW], vx = oth[lpos + 2 * e - 1];
        float nr = fmaf(tn[S][C], vn.x, fmaf(ts[S][C], vs.x, fmaf(tl[S][C], vx.x, br[S][C])));
        float ni = fmaf(tn[S][C], vn.y, fmaf(ts[S][C], vs.y, fmaf(tl[S][C], vx.y, bi[S][C])));
        nr = fmaf(tm[S], xr[S][1 - C], fmaf(tz[S][C], xr[Sp][1 - C], fmaf(tz[Sm][1 - C], xr[Sm][1 - C], nr)));
        ni = fmaf(tm[S], xi[S][1 - C], fmaf(tz[S][C], xi[Sp][1 - C], fmaf(tz[Sm][1 - C], xi[Sm][1 - C], ni)));
        const float vr = fmaf(nr, dr[S][C], -(ni * di[S][C]));
        const float vi = fmaf(nr, di[S][C], ni * dr[S][C]);
        xr[S][C] = vr;
        xi[S][C] = vi;
        pl[C * PLANE + lpos] = mk2(vr, vi);
    };

    // residual b - A x of the colour-C cell of plane p (x final)
    auto resid = [&](int p, auto Sc, auto Smc, auto Spc, auto Cc, float& rr, float& ri) {
        constexpr int S = decltype(Sc)::value, Sm = decltype(Smc)::value, Sp = decltype(Spc)::value;
        constexpr int C = decltype(Cc)::value;
        const V* oth = &sx[(p + NS) % NS][1 - C][0];
        const int e = lodd ^ ((p + C) & 1);
        const V vn = oth[lpos + RW], vs = oth[lpos - RW], vx = oth[lpos + 2 * e - 1];
        float orr = fmaf(tn[S][C], vn.x, fmaf(ts[S][C], vs.x, tl[S][C] * vx.x));
        float oi = fmaf(tn[S][C], vn.y, fmaf(ts[S][C], vs.y, tl[S][C] * vx.y));
        orr = fmaf(tm[S], xr[S][1 - C], fmaf(tz[S][C], xr[Sp][1 - C], fmaf(tz[Sm][1 - C], xr[Sm][1 - C], orr)));
        oi = fmaf(tm[S], xi[S][1 - C], fmaf(tz[S][C], xi[Sp][1 - C], fmaf(tz[Sm][1 - C], xi[Sm][1 - C], oi)));
        // D + tau m from its inverse
        const float q = 1.f / fmaf(dr[S][C], dr[S][C], di[S][C] * di[S][C]);
        const float ar = dr[S][C] * q, ai = -di[S][C] * q;
        const float axr = fmaf(ar, xr[S][C], -(ai * xi[S][C])) - orr;
        const float axi = fmaf(ar, xi[S][C], ai * xr[S][C]) - oi;
        rr = br[S][C] - axr;
        ri = bi[S][C] - axi;
    };

    auto flush_coarse = [&]() {
        // y partner sums of coarse plane `pend` (rows ly, ly + 1 with ly even; x and y halved)
        if (pend >= 0 && interior && (ly & 1) == 0) {
            const V a0 = sred[PRE ? (pend & 1) : 0][PRE ? tid : 0];
            const V c0 = sred[PRE ? (pend & 1) : 0][PRE ? tid + W : 0];
            const unsigned I = (unsigned)pend * CXY + (unsigned)(gy >> 1) * cnx + (unsigned)(gxa >> 1);
            stv(bcr, I, a0.x + c0.x);
            stv(bci, I, a0.y + c0.y);
        }
        pend = -1;
    };

    // one step of the march at plane t; U = (t - pl0) mod LR
    auto step = [&](int t, auto Uc) {
        constexpr int U = decltype(Uc)::value;
        constexpr int S1 = (U + 1) % LR;
        if (((t - pl0) % MS) == 0) {
            // group g = (t - pl0) / MS (planes t + 1 .. t + MS) has landed: stage group g + 1
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const int qa = t + MS + 1;
            const int sb = ((((t - pl0) / MS) + 1) & 1) * MS;
#pragma unroll
            for (int i = 0; i < MS; ++i) stage_plane(qa + i, sb + i);
            if (!PRE) stage_coarse(qa, qa + MS - 1, (((t - pl0) / MS) + 1) & 1);
        }
        if (PRE) flush_coarse();
        // plane t + 1 enters the ring
        process(t + 1, IC<S1>{});
        // stages in increasing order
        if (PRE) {
            // stage 1 from x = 0: colour 0 = b / d, colour 1 = 0
            if (in_range(t, 1)) {
                constexpr int S = U % LR;
                const float vr = fmaf(br[S][0], dr[S][0], -(bi[S][0] * di[S][0]));
                const float vi = fmaf(br[S][0], di[S][0], bi[S][0] * dr[S][0]);
                xr[S][0] = vr;
                xi[S][0] = vi;
                xr[S][1] = xi[S][1] = 0.f;
                V* pl = &sx[(t + NS) % NS][0][0];
                pl[lpos] = mk2(vr, vi);
                pl[PLANE + lpos] = mk2(0.f, 0.f);
            }
        }
        auto stage = [&](auto Sc) {
            constexpr int s0 = decltype(Sc)::value;
            constexpr int S = ((U - s0 + 1) % LR + LR) % LR;
            constexpr int Sm = (S + LR - 1) % LR, Sp = (S + 1) % LR;
            constexpr int C = (PRE ? s0 - 1 : s0) & 1;
            const int p = t - s0 + 1;
            if (in_range(p, s0)) relax(p, IC<S>{}, IC<Sm>{}, IC<Sp>{}, IC<C>{});
        };
        if (!PRE) stage(IC<1>{});
        stage(IC<2>{});
        if constexpr (NST >= 3) stage(IC<3>{});
        if constexpr (NST >= 4) stage(IC<4>{});
        // final x of plane t - 2 nu + 1
        {
            const int p = t - NST + 1;
            constexpr int S = ((U - NST + 1) % LR + LR) % LR;
            if (p >= z0 && p < z1 && interior) {
                const bool ce = ((ly + p) & 1) != 0;
                const unsigned zo = (unsigned)p * NXY;
                stv(xor_, zo + o0, ce ? xr[S][1] : xr[S][0]);
                stv(xoi, zo + o0, ce ? xi[S][1] : xi[S][0]);
                if (gxa + 1 < nx) {
                    stv(xor_, zo + o1, ce ? xr[S][0] : xr[S][1]);
                    stv(xoi, zo + o1, ce ? xi[S][0] : xi[S][1]);
                }
            }
        }
        if (PRE) {
            // residual of plane t - 2 nu, summed into the aggregate
            const int p = t - NST;
            constexpr int S = ((U - NST) % LR + LR) % LR;
            constexpr int Sm = (S + LR - 1) % LR, Sp = (S + 1) % LR;
            if (p >= z0 && p < z1) {
                float r0r, r0i, r1r, r1i;
                resid(p, IC<S>{}, IC<Sm>{}, IC<Sp>{}, IC<0>{}, r0r, r0i);
                resid(p, IC<S>{}, IC<Sm>{}, IC<Sp>{}, IC<1>{}, r1r, r1i);
                // the pair is one aggregate in x
                zr0 += r0r + r1r;
                zi0 += r0i + r1i;
                if (!coz || (p & 1)) {
                    const int Z = coz ? p >> 1 : p;
                    sred[PRE ? (Z & 1) : 0][PRE ? tid : 0] = mk2(zr0, zi0);
                    zr0 = zi0 = 0.f;
                    pend = Z;
                }
            }
        }
        __syncthreads();
    };

    // prologue: plane pl0 and the first group staged; pl0 into ring slot 0
    stage_plane(pl0, 2 * MS - 1);
    if (!PRE) stage_coarse(pl0, pl0, 1);
#pragma unroll
    for (int i = 0; i < MS; ++i) stage_plane(pl0 + 1 + i, i);
    if (!PRE) stage_coarse(pl0 + 1, pl0 + MS, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    process(pl0, IC<0>{});
    const int tlast = PRE ? z1 - 1 + NST : z1 - 1 + NST - 1;
    for (int t0 = pl0; t0 <= tlast; t0 += LR) {
#define LT_U(UU) \
    if constexpr (LR > UU) { if (t0 + UU <= tlast) step(t0 + UU, IC<UU>{}); }
        LT_U(0) LT_U(1) LT_U(2) LT_U(3) LT_U(4) LT_U(5) LT_U(6) LT_U(7) LT_U(8)
#undef LT_U
    }
    if (PRE) flush_coarse();
    // loads staged for planes beyond the run may still be in flight
    __builtin_amdgcn_s_waitcnt(0);

    if (prof && tid == 0 && blockIdx.x == 0 && blockIdx.y == 0) {
        // algorithmic bytes of this right-hand side over the level (one count per right-hand
        // side and launch): pre: b in, x out, coarse rhs out; post: x in, b in, x out, coarse
        // correction in (complex FP32); the coefficient arrays Tx, Ty, Tz, D, m are shared by
        // the Rtot right-hand sides
        const double cell = (PRE ? 16.0 : 24.0) + 20.0 / Rtot;
        atomicAdd(prof, (unsigned long long)((double)N * cell + (double)Nc * 8.0));
    }
}

// ------------------------------------------------------------------ launchers
// z run per workgroup: the whole depth unless the launch would have fewer than
// 1024 workgroups, then halved (kept even, at least 8 planes)
static int pick_cz(int nz, int nxy_tiles, int R) {
    int cz = nz + (nz & 1);
    while (cz > 8 && (long long)nxy_tiles * R * ((nz + cz - 1) / cz) < 1024) {
        cz = (cz + 1) / 2;
        cz += cz & 1;
    }
    return cz;
}

template <bool PRE>
static int launch_smooth3d(hipStream_t st, const LevelView<float>& L, float tr, float ti, int nu, int tile,
                           const float* b, const float* xin, const float* ec, float* xout, float* bc, int cnx,
                           int cny, int cnz, int cox, int coy, int coz, G6 ghost, int R, const int* active,
                           unsigned long long* prof, hipEvent_t ev0, hipEvent_t ev1) {
    if (nu < 1 || nu > 2 || !cox || !coy) {
        set_last_error("fused 3D smoother: 1 or 2 sweeps, x and y halved");
        return LT_EUNSUPPORTED;
    }
#define LT_K3(NU, X, Y)                                                                                        \
    do {                                                                                                      \
        using G = G3<NU, X, Y>;                                                                               \
        const int ntx = (L.nx + X - 1) / X, nty = (L.ny + Y - 1) / Y;                                         \
        const int cz = pick_cz(L.nz, ntx * nty, R);                                                           \
        const dim3 grid(ntx * nty, (L.nz + cz - 1) / cz, R);                                                  \
        if (ev0)                                                                                              \
            hipExtLaunchKernelGGL((k_smooth3d<NU, X, Y, PRE>), grid, dim3(G::NT), 0, st, ev0, ev1, 0, L, tr, ti, b, \
                                  xin, ec, xout, bc, cnx, cny, cnz, coz, ghost, cz, ntx, active, prof, R);     \
        else                                                                                                  \
            k_smooth3d<NU, X, Y, PRE><<<grid, G::NT, 0, st>>>(L, tr, ti, b, xin, ec, xout, bc, cnx, cny, cnz, coz, \
                                                              ghost, cz, ntx, active, prof, R);              \
    } while (0)
#define LT_T3(X, Y) \
    if (nu == 1) LT_K3(1, X, Y); else LT_K3(2, X, Y)
    switch (tile) {
        case 0: LT_T3(32, 8); break;
        case 1: LT_T3(16, 8); break;
        default: set_last_error("unknown 3D tile shape"); return LT_EINVAL;
    }
#undef LT_T3
#undef LT_K3
    LT_HIP(hipGetLastError());
    return 0;
}

template <>
int launch_pre3d<float>(hipStream_t st, const LevelView<float>& L, float tr, float ti, int nu, int tile,
                        const float* b, float* x, int cnx, int cny, int cnz, int cox, int coy, int coz, float* bc,
                        int R, const int* active, unsigned long long* prof, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_smooth3d<true>(st, L, tr, ti, nu, tile, b, nullptr, nullptr, x, bc, cnx, cny, cnz, cox, coy, coz,
                                 G6{}, R, active, prof, ev0, ev1);
}

template <>
int launch_post3d<float>(hipStream_t st, const LevelView<float>& L, float tr, float ti, int nu, int tile,
                         const float* b, const float* xin, const float* ec, int cnx, int cny, int cnz, int cox,
                         int coy, int coz, G6 ghost, float* xout, int R, const int* active,
                         unsigned long long* prof, hipEvent_t ev0, hipEvent_t ev1) {
    return launch_smooth3d<false>(st, L, tr, ti, nu, tile, b, xin, ec, xout, nullptr, cnx, cny, cnz, cox, coy, coz,
                                  ghost, R, active, prof, ev0, ev1);
}

// FP64 cycles keep the one-colour-per-launch kernels (mg.hip)
template <>
int launch_pre3d<double>(hipStream_t, const LevelView<double>&, double, double, int, int, const double*, double*,
                         int, int, int, int, int, int, double*, int, const int*, unsigned long long*, hipEvent_t,
                         hipEvent_t) {
    set_last_error("fused 3D smoother: FP32 only");
    return LT_EUNSUPPORTED;
}

template <>
int launch_post3d<double>(hipStream_t, const LevelView<double>&, double, double, int, int, const double*,
                          const double*, const double*, int, int, int, int, int, int, G6, double*, int, const int*,
                          unsigned long long*, hipEvent_t, hipEvent_t) {
    set_last_error("fused 3D smoother: FP32 only");
    return LT_EUNSUPPORTED;
}

}  // namespace lt
