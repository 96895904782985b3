// C ABI entry points and the batched flexible shifted Krylov driver.
//
// Method (Section 3): for each right-hand side b one flexible Arnoldi basis
// V_{m+1} and preconditioned vectors U_m are built with preconditioner shifts
// tau_j, and every contour shift z_k solves the small least-squares problem
// min || beta e_1 - Hbar(z_k; T_m) y ||, Hbar(z; T) = [I; 0] + Hbar (z I - T)
// (eqn:shiftedarnoldimod), x_k = U_m y_k.  The relation needs
// (K + tau_j M) u_j = v_j; the multigrid preconditioner is therefore refined
// (u_j += V-cycle(rho), rho = v_j - (K + tau_j M) u_j, in FP64) until
// ||rho|| <= relax * tol / (largest weighted shift residual so far): the
// residual gap this leaves is bounded by sum_j |y_j| ||rho_j|| and the
// relaxation keeps it below the tolerance (inexact Krylov).  The FP64 true
// residual of every (rhs, shift) is computed at exit.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "krylov.h"
#include "mg_fused.h"
#include "lt_internal.h"
#include "unet.h"

namespace lt {

static thread_local std::string g_last_error;
void set_last_error(const std::string& s) { g_last_error = s; }

}  // namespace lt

using namespace lt;

namespace lt {

// Events for one profiled launch: the launcher passes them to hipExtLaunchKernel,
// which records them at the start and end of that kernel's execution (no launch
// gap inside the interval).
int prof_begin(lt_handle* h, int family, unsigned long long** counter, hipEvent_t* ev0, hipEvent_t* ev1) {
    (void)family;
    if (h->prof_used + 2 > (int)h->prof_events.size()) {
        for (int k = 0; k < 256; ++k) {
            hipEvent_t e;
            LT_HIP(hipEventCreate(&e));
            h->prof_events.push_back(e);
        }
    }
    *ev0 = h->prof_events[h->prof_used];
    *ev1 = h->prof_events[h->prof_used + 1];
    *counter = h->prof_counter;
    return 0;
}

int prof_end(lt_handle* h, int family) {
    (void)family;
    h->prof_used += 2;
    return 0;
}

}  // namespace lt

lt_handle::~lt_handle() {
    for (Level& L : levels) {
        L.c64.release();
        L.c32.release();
    }
    for (CoarseInverse& c : coarse_cache) {
        c.inv64.release();
        c.inv32.release();
    }
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second.first);
    graphs.clear();
    for (auto& kv : ws) kv.second.release();
    kappa.release();
    mstor.release();
    for (lt::ExactFactor& f : exact_cache) f.release();
    if (pinned) (void)hipHostFree(pinned);
    for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
}

namespace {

struct DevPoints {
    int n = 0;
    int* off = nullptr;
    int* cell = nullptr;
    double* wt = nullptr;
};

int upload_points(lt_handle* h, const PointsCSR& c, const char* tag, DevPoints* d) {
    int rc = 0;
    d->n = (int)c.off.size() - 1;
    std::string t(tag);
    d->off = wsp<int>(h, (t + "_off").c_str(), c.off.size(), &rc);
    if (!d->off) return rc;
    size_t nn = std::max<size_t>(c.cell.size(), 1);
    d->cell = wsp<int>(h, (t + "_cell").c_str(), nn, &rc);
    if (!d->cell) return rc;
    d->wt = wsp<double>(h, (t + "_wt").c_str(), nn, &rc);
    if (!d->wt) return rc;
    LT_HIP(hipMemcpyAsync(d->off, c.off.data(), c.off.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
    if (!c.cell.empty()) {
        LT_HIP(hipMemcpyAsync(d->cell, c.cell.data(), c.cell.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
        LT_HIP(hipMemcpyAsync(d->wt, c.wt.data(), c.wt.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    }
    return 0;
}

int validate_opts(const lt_opts* o) {
    if (!o) return 0;
    if (!(o->tol > 0.0) || o->maxit < 1 || o->maxit > 2000 || o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 ||
        o->inner_max < 1 || !(o->relax > 0.0) || o->profile < 0 || o->profile > LT_PROF_EXACT ||
        (o->precond != LT_PRECOND_GMG && o->precond != LT_PRECOND_UNET_GMG && o->precond != LT_PRECOND_EXACT) ||
        !(o->net_keep >= 0.0) ||
        (o->graph != 0 && o->graph != 1) || (o->method != LT_METHOD_GMRES && o->method != LT_METHOD_FOM) ||
        (o->conv != LT_CONV_WEIGHTED && o->conv != LT_CONV_RELATIVE) || (o->tau_adapt != 0 && o->tau_adapt != 1) ||
        (o->precision != LT_PREC_FP64 && o->precision != LT_PREC_MIXED) || o->restart < 0 || o->restart > 2000) {
        set_last_error("invalid lt_opts");
        return LT_EINVAL;
    }
    if (o->restart > 0 && (o->precond != LT_PRECOND_EXACT || o->method != LT_METHOD_FOM)) {
        set_last_error("lt_opts.restart needs LT_PRECOND_EXACT and LT_METHOD_FOM (the residuals are collinear only "
                       "for FOM with an exact preconditioner)");
        return LT_EINVAL;
    }
    return 0;
}

// Everything the Krylov loop leaves on the device for the epilogues.
struct KrylovOut {
    int R = 0, Ks = 0, jmax = 0;
    double* U = nullptr;      // [R][jmax][2][N]
    size_t ustride = 0;
    double* Y = nullptr;      // [R][jmax][Ks] complex
    double* G = nullptr;      // [R][jmax][np] complex (receiver gathers of u_j)
    int* mcols = nullptr;     // [R]
    double* beta = nullptr;   // [R]
    double* b = nullptr;      // [R][2][N]
    double* zs = nullptr;     // [Ks] complex
    double* omega = nullptr;  // [2][Ks]: wells' weights, then the initial head's
    double* wq = nullptr;     // [Ks] complex
    double* w = nullptr;      // [Ks] complex (the initial head's factor-1 weights)
    int rinit = 0;            // first right-hand side weighed by w (R: none)
    int iters_max = 0, vcycles = 0;
    int net_applied = 0, net_rejected = 0, net_disabled_at = 0;
    bool converged = true;
    std::vector<int> notconv;  // [R] 1 where the Arnoldi stopped at maxit
    double* Q = nullptr;       // [R][jmax + 1][2][N] the basis V (column j unnormalised after its step)
    size_t qstride = 0;
    double* eta = nullptr;     // [R][Ks] complex: FOM's eta_k of each pair's last step
};

// A cycle of a restarted solve: the least-squares start (per-pair g_0, the original norms)
// and the steps taken before it (the preconditioner schedule continues from there).
struct RestartIn {
    LSStart start;
    int j0 = 0;
};

// One step of the iterative refinement of u_j ~ (K + tau M)^{-1} v_j for the
// right-hand sides still marked in inner_active: a V-cycle on the current
// residual, the FP64 update u_j += e, rho -= (K + tau M) e (fused into the
// fine post-smoother where the level allows), and the stopping test.  Only
// enqueues work; u_j is U advanced by the device column index jdev.
// *swapped = 1 when the FP64 residual moved to rho_next.
int refine_step(lt_handle* h, const lt_opts& o, int R, cdouble tau, double* U, size_t ustride, const int* jdev,
                float* e32, double* e64, float* lo32, float* lo32_next, double* lo64, double* rho, double* rho_next,
                double* part,
                const int* active, int* inner_active, const double* worst, int* vcyc, int* count, double* rprev,
                int* est, int* swapped) {
    hipStream_t st = h->stream;
    const LevelView<double> L0 = h->levels[0].v64();
    int nparts = -1;
    *swapped = 0;
    if (o.precision == LT_PREC_MIXED) {
        // the FP32 copy of rho is double-buffered so that halo loads of this
        // V-cycle's input never race with the fused update
        RefineArgs ra{U, ustride, jdev, rho, rho, lo32_next, part, &nparts};
        LT_TRY(mg_vcycle<float>(h, tau, o.nu1, o.nu2, R, inner_active, e32, lo32, &ra));
        if (nparts < 0) {
            LT_TRY(launch_inner_update<float>(st, L0, tau, R, e32, U, ustride, jdev, rho, lo32_next, part,
                                              inner_active, h->cp3d ? 1 : 0, ra.list));
            nparts = reduce_blocks(h->N, R);
        }
    } else {
        RefineArgs ra{U, ustride, jdev, rho, rho_next, nullptr, part, &nparts};
        // 3D grids: the cycle reads the colour-planar copy of rho, which the update refreshes
        LT_TRY(mg_vcycle<double>(h, tau, o.nu1, o.nu2, R, inner_active, e64, lo64 ? lo64 : rho, &ra));
        if (nparts < 0) {
            LT_TRY(launch_inner_update<double>(st, L0, tau, R, e64, U, ustride, jdev, rho, lo64, part,
                                               inner_active, lo64 ? 1 : 0, ra.list));
            nparts = reduce_blocks(h->N, R);
        } else {
            *swapped = 1;
        }
    }
    return launch_inner_finalize(st, nparts, R, part, active, worst, o.relax * o.tol, o.tol, o.inner_max,
                                 inner_active, vcyc, count, rprev, est);
}

// refine_step captured once as a HIP graph and replayed.  Everything a
// captured step bakes in is part of the key: sizes, options, the shift, the
// buffers, and the workspace generation (any reallocation retires all graphs).
int graph_step(lt_handle* h, const lt_opts& o, int R, cdouble tau, double* U, size_t ustride, const int* jdev,
               float* e32, double* e64, float* lo32, float* lo32_next, double* lo64, double* rho, double* rho_next,
               double* part,
               const int* active, int* inner_active, const double* worst, int* vcyc, int* count, double* rprev,
               int* est, int* swapped) {
    hipStream_t st = h->stream;
    int rc = 0;
    // the coarse inverse for tau is built on the host and uploaded: do it before capturing
    mg_coarse_inverse(h, tau, &rc);
    if (rc < 0) return rc;
    if (h->graphs_gen != h->ws_gen) {
        for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second.first);
        h->graphs.clear();
        h->graphs_gen = h->ws_gen;
    }
    auto bits = [](double v) {
        unsigned long long b;
        std::memcpy(&b, &v, sizeof(b));
        return b;
    };
    auto ptr = [](const void* p) { return (unsigned long long)(uintptr_t)p; };
    std::vector<unsigned long long> key = {
        (unsigned long long)o.precision, (unsigned long long)R, (unsigned long long)o.nu1, (unsigned long long)o.nu2,
        bits(tau.real()), bits(tau.imag()), bits(o.relax * o.tol), bits(o.tol), (unsigned long long)o.inner_max,
        ptr(U), ustride, ptr(jdev), ptr(e32), ptr(e64), ptr(lo32), ptr(lo32_next), ptr(lo64), ptr(rho), ptr(rho_next),
        ptr(part), ptr(active), ptr(inner_active), ptr(worst), ptr(vcyc), ptr(count), ptr(rprev), ptr(est),
        h->ws_gen};
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        if (h->graphs.size() >= 64) {
            for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second.first);
            h->graphs.clear();
        }
        const unsigned long long gen = h->ws_gen;
        LT_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int sw = 0;
        const int rcs = refine_step(h, o, R, tau, U, ustride, jdev, e32, e64, lo32, lo32_next, lo64, rho, rho_next, part,
                                    active, inner_active, worst, vcyc, count, rprev, est, &sw);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (rcs < 0 || ec != hipSuccess || h->ws_gen != gen) {
            if (g) (void)hipGraphDestroy(g);
            if (rcs < 0) return rcs;
            if (ec != hipSuccess) {
                set_last_error(std::string("capturing a refinement step: ") + hipGetErrorString(ec));
                return LT_EHIP;
            }
            // a workspace moved while capturing: launch this step directly
            return refine_step(h, o, R, tau, U, ustride, jdev, e32, e64, lo32, lo32_next, lo64, rho, rho_next, part,
                               active, inner_active, worst, vcyc, count, rprev, est, swapped);
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        LT_HIP(ei);
        it = h->graphs.emplace(key, std::make_pair(ex, sw)).first;
    }
    *swapped = it->second.second;
    LT_HIP(hipGraphLaunch(it->second.first, st));
    return 0;
}

// Batched flexible shifted GMRES for R right-hand sides b (device [R][2][N], already
// filled).  Gathers B_rec u_j for `rec` if given.  Right-hand sides from rinit on weigh
// their shifts by |w_k| (the initial head's term).  With `only` (host [R] flags), just
// those right-hand sides are solved; the others keep the basis, gathers and column
// counts of the previous call on the same workspace.
int run_krylov(lt_handle* h, const Plan& plan, const lt_opts& o, int R, int rinit, const DevPoints* rec,
               KrylovOut* out, const std::vector<int>* only = nullptr, const RestartIn* rin = nullptr) {
    hipStream_t st = h->stream;
    const int N = h->N;
    const int jmax = o.maxit;
    const int Ks = plan.ntimes * plan.nk;
    const size_t N2 = 2 * (size_t)N;
    int rc = 0;
    out->R = R;
    out->Ks = Ks;
    out->jmax = jmax;
    h->last_R = 0;  // set again once the basis is complete
    const size_t qstride = (size_t)(jmax + 1) * N2, ustride = (size_t)jmax * N2;
    double* Q = wsp<double>(h, "Q", (size_t)R * qstride, &rc);
    if (!Q) return rc;
    double* U = wsp<double>(h, "U", (size_t)R * ustride, &rc);
    if (!U) return rc;
    double* rho = wsp<double>(h, "rho", R * N2, &rc);
    if (!rho) return rc;
    const bool mixed = o.precision == LT_PREC_MIXED;
    float* lo32 = nullptr;
    float* e32 = nullptr;
    double* e64 = nullptr;
    double* rho_next = wsp<double>(h, "rho_next", R * N2, &rc);
    if (!rho_next) return rc;
    float* lo32_next = nullptr;
    if (mixed) {
        lo32 = wsp<float>(h, "lo32", R * N2, &rc);
        if (!lo32) return rc;
        lo32_next = wsp<float>(h, "lo32_next", R * N2, &rc);
        if (!lo32_next) return rc;
        e32 = wsp<float>(h, "e32", R * N2, &rc);
        if (!e32) return rc;
    } else {
        e64 = wsp<double>(h, "e64", R * N2, &rc);
        if (!e64) return rc;
    }
    // FP64 cycles of a 3D grid read a colour-planar copy of rho (the FP32 ones lo32)
    double* lo64 = nullptr;
    if (!mixed && h->cp3d) {
        lo64 = wsp<double>(h, "lo64", R * N2, &rc);
        if (!lo64) return rc;
    }
    const int hstride = 2 * (jmax + 2);
    const size_t hrstride = (size_t)jmax * hstride;
    double* H = wsp<double>(h, "H", (size_t)R * hrstride, &rc);
    if (!H) return rc;
    const int cstride = 2 * (jmax + 2);
    double* c1 = wsp<double>(h, "c1", (size_t)R * cstride, &rc);
    double* c2 = wsp<double>(h, "c2", (size_t)R * cstride, &rc);
    if (!c1 || !c2) return rc;
    const int nb = reduce_blocks(N, R);
    const int pstride = 2 * (jmax + 2);
    // per-tile partial sums of the fused refinement (the smallest tile shape has the most)
    const size_t ntiles = ((size_t)h->grid.n[0] + kMinTileX - 1) / kMinTileX *
                          (((size_t)h->grid.n[1] + kMinTileY - 1) / kMinTileY) * h->grid.n[2];
    double* part = wsp<double>(h, "part", (size_t)R * std::max((size_t)nb * pstride, ntiles), &rc);
    if (!part) return rc;
    double* small = wsp<double>(h, "small", 4 * (size_t)R, &rc);
    if (!small) return rc;
    double* partn = wsp<double>(h, "partn", (size_t)R * nb, &rc);  // norm partials of the Gram-Schmidt step
    if (!partn) return rc;
    double* scale = small;
    double* beta = small + R;
    double* worst = small + 2 * R;
    double* rprev = small + 3 * R;  // residual norms before the last refinement step
    int* ints = wsp<int>(h, "ints", 6 * (size_t)R + 12, &rc);  // netc has 3 entries at 5R + 4  // masks, counts, [count, steps needed], net stats
    if (!ints) return rc;
    int* active = ints;
    int* inner_active = ints + R;
    int* mcols = ints + 2 * R;
    int* vcyc = ints + 3 * R;
    int* count = ints + 4 * R;
    int* bad = ints + 4 * R + 4;      // [R] network guesses to discard
    int* netc = ints + 5 * R + 4;     // [3] applied, rejected, worst residual ratio (float bits)
    int* probe = ints + 5 * R + 8;    // [R] the one right-hand side the network is first tried on
    int* est = ints + 6 * R + 8;      // [1] estimated refinement steps still needed
    bool use_net = o.precond == LT_PRECOND_UNET_GMG && h->unet != nullptr;
    if (o.precond == LT_PRECOND_UNET_GMG &&
        (!h->unet || h->grid.ndim != 2 || h->grid.n[0] % 128 || h->grid.n[1] % 8)) {
        set_last_error("LT_PRECOND_UNET_GMG needs an attached network and a 2D grid with nx % 128 == 0, ny % 8 == 0");
        return LT_EINVAL;
    }
    const size_t P = (size_t)R * Ks;
    LSState ls;
    ls.Rm = wsp<double>(h, "Rm", 2 * P * ((size_t)jmax * (jmax + 1) / 2), &rc);
    ls.cs = wsp<double>(h, "cs", P * jmax, &rc);
    ls.sn = wsp<double>(h, "sn", 2 * P * jmax, &rc);
    ls.g = wsp<double>(h, "g", 2 * P * (jmax + 1), &rc);
    ls.res = wsp<double>(h, "res", P, &rc);
    if (o.method == LT_METHOD_FOM) {
        ls.eta = wsp<double>(h, "eta", 2 * P, &rc);
        if (!ls.eta) return rc;
    }
    const LSStart start = rin ? rin->start : LSStart();
    const int j0 = rin ? rin->j0 : 0;
    int* conv = wsp<int>(h, "conv", P, &rc);
    double* Y = wsp<double>(h, "Y", (size_t)R * jmax * 2 * Ks, &rc);
    double* tabs = wsp<double>(h, "tabs", 8 * (size_t)Ks, &rc);
    if (!ls.Rm || !ls.cs || !ls.sn || !ls.g || !ls.res || !conv || !Y || !tabs) return rc;
    double* G = nullptr;
    int np = rec ? rec->n : 0;
    if (np > 0) {
        G = wsp<double>(h, "G", (size_t)R * jmax * 2 * np, &rc);
        if (!G) return rc;
    }
    double* zs = tabs;
    double* wq = tabs + 2 * Ks;
    double* wk = tabs + 4 * Ks;
    double* omega = tabs + 6 * Ks;  // [2][Ks]
    {
        std::vector<double> t(8 * (size_t)Ks);
        for (int k = 0; k < Ks; ++k) {
            t[2 * k] = plan.z[k].real();
            t[2 * k + 1] = plan.z[k].imag();
            t[2 * Ks + 2 * k] = plan.wq[k].real();
            t[2 * Ks + 2 * k + 1] = plan.wq[k].imag();
            t[4 * Ks + 2 * k] = plan.w[k].real();
            t[4 * Ks + 2 * k + 1] = plan.w[k].imag();
            t[6 * Ks + k] = plan.omega[k];
            t[7 * Ks + k] = plan.omega_init[k];
        }
        LT_HIP(hipMemcpyAsync(tabs, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, st));
    }
    if (!h->pinned) LT_HIP(hipHostMalloc(&h->pinned, 4096, hipHostMallocDefault));
    int* hflag = static_cast<int*>(h->pinned);
    int* hact = hflag + 16;
    if (R > kMaxRhs) {
        set_last_error("at most " + std::to_string(kMaxRhs) + " right-hand sides per call");
        return LT_EINVAL;
    }
    double* b = out->b;
    int probe_rhs = -1;           // first right-hand side with a non-zero b
    bool net_confirmed = false;   // the network's probe guess paid for itself
    // beta, v_1 = b / beta, masks
    LT_TRY(launch_norms(st, N, R, N2, b, part, beta, nullptr));
    LT_TRY(launch_scale_into(st, N, R, N2, qstride, b, beta, Q));
    {
        std::vector<double> init(4 * (size_t)R, 0.0);
        for (int r = 0; r < R; ++r) init[2 * R + r] = 1.0;  // worst
        // scale, beta are device-computed; upload only worst (keep beta)
        LT_HIP(hipMemcpyAsync(worst, init.data() + 2 * R, R * sizeof(double), hipMemcpyHostToDevice, st));
        std::vector<double> hb(R);
        LT_HIP(hipMemcpyAsync(hb.data(), beta, R * sizeof(double), hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        std::vector<int> ii(6 * (size_t)R + 12, 0);
        for (int r = 0; r < R; ++r) ii[r] = hb[r] > 0.0 && (!only || (*only)[r]) ? 1 : 0;
        probe_rhs = -1;
        for (int r = 0; r < R && probe_rhs < 0; ++r)
            if (ii[r]) probe_rhs = r;
        if (probe_rhs >= 0) ii[5 * (size_t)R + 8 + probe_rhs] = 1;
        if (!only) {
            LT_HIP(hipMemcpyAsync(ints, ii.data(), ii.size() * sizeof(int), hipMemcpyHostToDevice, st));
        } else {
            // keep the column counts of the right-hand sides that are not solved again
            LT_HIP(hipMemcpyAsync(ints, ii.data(), 2 * (size_t)R * sizeof(int), hipMemcpyHostToDevice, st));
            LT_HIP(hipMemcpyAsync(ints + 3 * (size_t)R, ii.data() + 3 * (size_t)R, (ii.size() - 3 * (size_t)R) * sizeof(int),
                                  hipMemcpyHostToDevice, st));
        }
    }
    const LevelView<double> L0 = h->levels[0].v64();
    const double* m = L0.m;
    int* jdev = count + 3;  // basis column the refinement steps update (device)
    // captured steps need a stream of the handle's own (the legacy default stream cannot be captured)
    const bool use_graphs = o.graph && !h->prof_target && st != nullptr;
    int n_active = 0;
    for (int r = 0; r < R; ++r) n_active += (!only || (*only)[r]) ? 1 : 0;
    int j = 0;
    int inner_guess = 2;
    const bool debug = std::getenv("LT_DEBUG") != nullptr;
    const bool exact = o.precond == LT_PRECOND_EXACT;
    if (exact) {
        // factorise every shift of the schedule up front (each once; cached on the handle)
        for (size_t i = 0; i < plan.tau_sched.size() && i < (size_t)kExactCache; ++i) {
            exact_factor(h, plan.tau_sched[i], &rc);
            if (rc < 0) return rc;
        }
    }
    out->converged = false;
    // adaptive shifts: the weighted least-squares residuals of the last outer iteration
    std::vector<double> hres(o.tau_adapt ? (size_t)R * Ks : 0);
    std::vector<cdouble> cand;  // the exact preconditioner's candidates: the schedule's distinct shifts
    for (const cdouble& t : plan.tau_sched)
        if (std::find(cand.begin(), cand.end(), t) == cand.end()) cand.push_back(t);
    for (j = 0; j < jmax; ++j) {
        cdouble tau = plan.tau_sched[(j + j0) % plan.tau_sched.size()];
        if (o.tau_adapt && j > 0) {
            LT_HIP(hipMemcpyAsync(hres.data(), ls.res, hres.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            LT_HIP(hipMemcpyAsync(hact, active, R * sizeof(int), hipMemcpyDeviceToHost, st));
            LT_HIP(hipStreamSynchronize(st));
            double best = -1.0;
            int kbest = -1;
            for (int r = 0; r < R; ++r) {
                if (!hact[r]) continue;
                const std::vector<double>& om = r >= rinit ? plan.omega_init : plan.omega;
                for (int k = 0; k < Ks; ++k) {
                    const double w = om[k] * hres[(size_t)r * Ks + k];  // the convergence test's weighting
                    if (w > o.tol && w > best) {
                        best = w;
                        kbest = k;
                    }
                }
            }
            if (kbest >= 0) {
                const cdouble zc = plan.z[kbest];
                if (exact) {
                    tau = cand[0];
                    for (const cdouble& c : cand)
                        if (std::abs(c - zc) < std::abs(tau - zc)) tau = c;
                } else {
                    tau = zc.real() >= 0.0 ? zc : cdouble(0.0, zc.imag());
                }
            }
        }
        LT_TRY(launch_iter_begin(st, R, active, inner_active, count, j, rprev));  // jdev = count + 3
        double* uj = U + (size_t)j * N2;
        double* vj = Q + (size_t)j * N2;
        const double* vscale = j > 0 ? scale : nullptr;  // v_j is normalised by its first read
        if (exact) {
            // stop as soon as the last least-squares update converged every shift
            if (j > 0) {
                LT_HIP(hipMemcpyAsync(hact, active, R * sizeof(int), hipMemcpyDeviceToHost, st));
                LT_HIP(hipStreamSynchronize(st));
                n_active = 0;
                for (int r = 0; r < R; ++r) n_active += hact[r];
                if (n_active == 0) {
                    out->converged = true;
                    break;
                }
            }
            // u_j = (K + tau_j M)^{-1} v_j by the factorisation of tau_j: the Arnoldi relation
            // of the flexible method then holds to rounding, with no inner iteration
            const ExactFactor* F = exact_factor(h, tau, &rc);
            if (!F) return rc;
            LT_TRY(launch_inner_init<double>(st, N, R, qstride, vj, uj, ustride, rho, (double*)nullptr, active,
                                             vscale, 0, 0));
            LT_TRY(exact_apply(h, F, R, rho, N2, uj, ustride, active));
            LT_TRY(launch_cgs2(st, N, R, j, m, U, ustride, Q, qstride, H, hstride, hrstride, part, pstride, c1, c2,
                               cstride, scale, partn, active));
            if (np > 0)
                LT_TRY(launch_gather(st, R, N, np, rec->off, rec->cell, rec->wt, U, ustride, j, G, jmax, active));
            LT_TRY(launch_ls_update(st, R, Ks, j, tau, zs, omega, rinit, o.tol, o.method == LT_METHOD_FOM, H, hstride,
                                    hrstride, beta, ls, active, mcols, worst, conv, start));
            continue;
        }
        // inner refinement of u_j ~ (K + tau M)^{-1} v_j
        if (mixed)
            LT_TRY(launch_inner_init<float>(st, N, R, qstride, vj, uj, ustride, rho, lo32, active, vscale,
                                            h->cp3d ? h->grid.n[0] : 0, h->grid.n[1]));
        else
            LT_TRY(launch_inner_init<double>(st, N, R, qstride, vj, uj, ustride, rho, lo64, active, vscale,
                                             h->cp3d ? h->grid.n[0] : 0, h->grid.n[1]));
        if (use_net && probe_rhs >= 0) {
            // learned first guess u = alpha net(v), alpha minimising ||v - alpha (K + tau M) net(v)||;
            // rho = v - (K + tau M) u; discarded where it is not finite or does not help.  Until
            // a guess has paid for itself the network runs on one right-hand side only (a batch
            // of one), so a network that does not help costs one small application.
            UNet* net = &h->unet->net;
            const int nbr = reduce_blocks(N, R);
            const int* mask = net_confirmed ? active : probe;
            const int nb_net = net_confirmed ? R : 1;
            const size_t o0 = net_confirmed ? 0 : 2 * (size_t)N * probe_rhs;
            const int* amask = net_confirmed ? active : nullptr;
            if (mixed) {
                LT_TRY(unet_apply<float>(net, st, L0, h->lnDbar, tau, nb_net, lo32 + o0, e32 + o0, amask));
                LT_TRY(launch_net_scale<float>(st, L0, tau, R, e32, rho, part, mask));
                LT_TRY(launch_inner_update<float>(st, L0, tau, R, e32, uj, ustride, nullptr, rho, lo32, part, mask));
                LT_TRY(launch_net_guard(st, R, nbr, part, mask, bad, netc));
                LT_TRY(launch_inner_init<float>(st, N, R, qstride, vj, uj, ustride, rho, lo32, bad));
            } else {
                LT_TRY(unet_apply<double>(net, st, L0, h->lnDbar, tau, nb_net, rho + o0, e64 + o0, amask));
                LT_TRY(launch_net_scale<double>(st, L0, tau, R, e64, rho, part, mask));
                LT_TRY(launch_inner_update<double>(st, L0, tau, R, e64, uj, ustride, nullptr, rho, (double*)nullptr, part,
                                                   mask));
                LT_TRY(launch_net_guard(st, R, nbr, part, mask, bad, netc));
                LT_TRY(launch_inner_init<double>(st, N, R, qstride, vj, uj, ustride, rho, (double*)nullptr, bad));
            }
        }
        // The refinement steps expected from the previous outer iteration are
        // enqueued without waiting; finished right-hand sides are masked off on
        // the device, and the host checks only after that batch.
        // Later batches are sized by the finalize kernel's estimate of the steps still needed
        // (from each residual's contraction in the last step), so a short first batch costs
        // one more synchronisation rather than one per missing step.
        int step = 0, checks = 0;
        int batch = std::min(inner_guess, o.inner_max);
        while (step < o.inner_max) {
            ++checks;
            for (int b2 = 0; b2 < batch && step < o.inner_max; ++b2, ++step) {
                int swapped = 0;
                if (use_graphs && j > 0) {
                    LT_TRY(graph_step(h, o, R, tau, U, ustride, jdev, e32, e64, lo32, lo32_next, lo64, rho, rho_next, part,
                                      active, inner_active, worst, vcyc, count, rprev, est, &swapped));
                } else {
                    LT_TRY(refine_step(h, o, R, tau, U, ustride, jdev, e32, e64, lo32, lo32_next, lo64, rho, rho_next, part,
                                       active, inner_active, worst, vcyc, count, rprev, est, &swapped));
                }
                if (mixed) std::swap(lo32, lo32_next);
                if (swapped) std::swap(rho, rho_next);
            }
            LT_HIP(hipMemcpyAsync(hflag + 3, est, sizeof(int), hipMemcpyDeviceToHost, st));
            LT_HIP(hipMemcpyAsync(hflag, count, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
            // convergence flags as left by the previous outer iteration's least squares
            LT_HIP(hipMemcpyAsync(hact, active, R * sizeof(int), hipMemcpyDeviceToHost, st));
            if (use_net) LT_HIP(hipMemcpyAsync(hflag + 2, netc + 2, sizeof(int), hipMemcpyDeviceToHost, st));
            LT_HIP(hipStreamSynchronize(st));
            if (*hflag == 0) break;
            batch = std::max(1, hflag[3]);
        }
        if (use_net) {
            // keep the network only while its guess removes at least the fraction 1 - net_keep
            // of the residual; otherwise the V-cycle refinement alone continues
            float worst_ratio;
            std::memcpy(&worst_ratio, hflag + 2, sizeof(float));
            if (!(worst_ratio <= o.net_keep)) {
                use_net = false;
                out->net_disabled_at = j + 1;
            } else {
                net_confirmed = true;
            }
        }
        if (debug) {
            std::vector<int> vc(R);
            LT_HIP(hipMemcpy(vc.data(), vcyc, R * sizeof(int), hipMemcpyDeviceToHost));
            std::fprintf(stderr, "[lt] j=%d tau=(%.3g,%.3g) inner launched=%d needed=%d guess=%d checks=%d vcycles/rhs:",
                         j, tau.real(), tau.imag(), step, hflag[1], inner_guess, checks);
            for (int r = 0; r < R; ++r) std::fprintf(stderr, " %d", vc[r]);
            std::fprintf(stderr, "\n");
        }
        inner_guess = std::max(1, hflag[1]);
        n_active = 0;
        for (int r = 0; r < R; ++r) n_active += hact[r];
        if (n_active == 0) {
            out->converged = true;
            break;
        }
        // Arnoldi: v_{j+1} from M u_j by classical Gram-Schmidt with reorthogonalisation
        LT_TRY(launch_cgs2(st, N, R, j, m, U, ustride, Q, qstride, H, hstride, hrstride, part, pstride, c1, c2,
                           cstride, scale, partn, active));
        if (np > 0) LT_TRY(launch_gather(st, R, N, np, rec->off, rec->cell, rec->wt, U, ustride, j, G, jmax, active));
        LT_TRY(launch_ls_update(st, R, Ks, j, tau, zs, omega, rinit, o.tol, o.method == LT_METHOD_FOM, H, hstride,
                                hrstride, beta, ls, active, mcols, worst, conv, start));
    }
    LT_HIP(hipMemcpyAsync(hact, active, R * sizeof(int), hipMemcpyDeviceToHost, st));
    LT_HIP(hipStreamSynchronize(st));
    n_active = 0;
    out->notconv.assign(R, 0);
    for (int r = 0; r < R; ++r) {
        n_active += hact[r];
        out->notconv[r] = hact[r];
    }
    out->converged = n_active == 0;
    LT_TRY(launch_backsolve(st, R, Ks, mcols, ls, Y, jmax, o.method == LT_METHOD_FOM));
    std::vector<int> hm(R), hv(R), hn(2);
    LT_HIP(hipMemcpyAsync(hn.data(), netc, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(hm.data(), mcols, R * sizeof(int), hipMemcpyDeviceToHost, st));
    LT_HIP(hipMemcpyAsync(hv.data(), vcyc, R * sizeof(int), hipMemcpyDeviceToHost, st));
    LT_HIP(hipStreamSynchronize(st));
    out->iters_max = 0;
    out->vcycles = 0;
    out->net_applied = hn[0];
    out->net_rejected = hn[1];
    for (int r = 0; r < R; ++r) {
        out->iters_max = std::max(out->iters_max, hm[r]);
        out->vcycles += hv[r];
    }
    h->last_R = R;
    h->last_jmax = jmax;
    out->U = U;
    out->ustride = ustride;
    out->Y = Y;
    out->G = G;
    out->mcols = mcols;
    out->beta = beta;
    out->zs = zs;
    out->omega = omega;
    out->wq = wq;
    out->w = wk;
    out->rinit = rinit;
    out->Q = Q;
    out->qstride = qstride;
    out->eta = ls.eta;
    return 0;
}

// FP64 true residuals of every (rhs, shift); wr[r] receives each right-hand side's largest
// weighted value omega_k ||b - (K + z_k M) x_k|| / ||b||.
int true_residuals(lt_handle* h, const KrylovOut& k, const Plan& plan, lt_stats* stats, std::vector<double>* wr) {
    hipStream_t st = h->stream;
    const int N = h->N, R = k.R, Ks = k.Ks;
    int rc = 0;
    const int mmax = k.iters_max;
    double* KU = wsp<double>(h, "KU", (size_t)R * std::max(mmax, 1) * 2 * N, &rc);
    const int nb = true_res_blocks(N, R);
    double* part = wsp<double>(h, "tpart", (size_t)R * Ks * nb, &rc);
    double* tr = wsp<double>(h, "trel", (size_t)R * Ks, &rc);
    if (!KU || !part || !tr) return rc;
    LT_TRY(launch_true_residual_cols(st, h->levels[0].v64(), R, Ks, k.jmax, mmax, k.U, k.ustride, k.Y, k.mcols,
                                     k.zs, k.b, k.beta, KU, part, tr));
    std::vector<double> ht((size_t)R * Ks);
    LT_HIP(hipMemcpyAsync(ht.data(), tr, ht.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LT_HIP(hipStreamSynchronize(st));
    double mx = 0.0;
    wr->assign(R, 0.0);
    for (int r = 0; r < R; ++r) {
        const std::vector<double>& om = r >= k.rinit ? plan.omega_init : plan.omega;
        for (int kk = 0; kk < Ks; ++kk) (*wr)[r] = std::max((*wr)[r], om[kk] * ht[(size_t)r * Ks + kk]);
        mx = std::max(mx, (*wr)[r]);
    }
    if (stats) {
        stats->true_relres_max = mx;
        if (stats->true_relres) std::memcpy(stats->true_relres, ht.data(), ht.size() * sizeof(double));
    }
    return 0;
}

// The flexible Arnoldi of run_krylov, then the FP64 true residual as the judge: a
// right-hand side whose Arnoldi converged but whose weighted true residual misses tol
// (the gap that relaxed preconditioner solves leave, sum_j y_j rho_j) is solved again
// from the start with its own tolerance, and with it the inner tolerance relax * tol,
// scaled by 0.5 / excess (its own excess, rounded down to a power of two), and with four
// times the V-cycles allowed per preconditioner solve (a weak coarse-grid solve can need
// more than inner_max to reach the tighter inner tolerance); at most twice.  Right-hand sides with the same factor are solved again together; the factor
// depends on the right-hand side alone, so its result does not depend on which other
// right-hand sides share the call.  *ok: every (rhs, shift) meets tol by both residuals.
int solve_checked(lt_handle* h, const Plan& plan, const lt_opts& o, int R, int rinit, const DevPoints* rec,
                  KrylovOut* k, lt_stats* stats, int* resolves, bool* ok) {
    *resolves = 0;
    if (o.restart > 0) {
        set_last_error("lt_opts.restart: only lt_solve restarts");
        return LT_EUNSUPPORTED;
    }
    LT_TRY(run_krylov(h, plan, o, R, rinit, rec, k));
    std::vector<int> nc = k->notconv;
    int vcycles = k->vcycles, napp = k->net_applied, nrej = k->net_rejected;
    bool tr_ok = true;
    if (o.true_residual) {
        std::vector<double> wr;
        std::vector<int> tshift(R, 0);  // tolerance of rhs r: tol * 2^-tshift[r]
        for (int attempt = 0;; ++attempt) {
            LT_TRY(true_residuals(h, *k, plan, stats, &wr));
            std::map<int, std::vector<int>> groups;  // new tshift -> its right-hand sides
            tr_ok = true;
            for (int r = 0; r < R; ++r) {
                if (!(wr[r] <= o.tol)) {
                    tr_ok = false;
                    if (!nc[r]) {
                        const double excess = std::isfinite(wr[r]) ? std::min(wr[r] / o.tol, 1e6) : 1e6;
                        // 0.5 / excess rounded down to a power of two
                        const int e = (int)std::ceil(std::log2(2.0 * excess) - 1e-12);
                        tshift[r] += std::max(e, 1);
                        groups[tshift[r]].push_back(r);
                    }
                }
            }
            if (groups.empty() || attempt == 2) break;
            for (const auto& g : groups) {
                std::vector<int> redo(R, 0);
                for (int r : g.second) redo[r] = 1;
                lt_opts o2 = o;
                o2.tol = std::ldexp(o.tol, -g.first);
                o2.inner_max = std::min(o.inner_max << (2 * (attempt + 1)), 1000);
                *resolves += (int)g.second.size();
                LT_TRY(run_krylov(h, plan, o2, R, rinit, rec, k, &redo));
                for (int r : g.second) nc[r] = k->notconv[r];
                vcycles += k->vcycles;
                napp += k->net_applied;
                nrej += k->net_rejected;
            }
        }
    }
    k->vcycles = vcycles;
    k->net_applied = napp;
    k->net_rejected = nrej;
    bool conv = true;
    for (int r = 0; r < R; ++r) conv = conv && !nc[r];
    k->notconv = nc;
    k->converged = conv;
    *ok = conv && tr_ok;
    return 0;
}

// FFOM-Sh with the exact preconditioner, restarted every o.restart steps.  With FOM and an
// exact preconditioner the residual of every shift after m steps is -eta_k v_{m+1} (Section
// 3.1): one vector for all shifts of a right-hand side.  Each cycle is one run of the Krylov
// loop: the first on b with g_0 = ||b|| for every shift, each later one, for the right-hand
// sides not yet converged, on the previous cycle's last basis vector v_{m+1} with
// g_0 = -eta_k per shift.  Residuals are measured against the original ||b||, the
// preconditioner schedule continues across cycles, and the heads of the cycles are summed.
// The FP64 true residual of a pair is that of its right-hand side's last cycle (whose
// right-hand side is the residual left by the cycles before): with y / (g_0 / ||v||), the
// coefficients for the unit right-hand side v / ||v||, the usual kernels measure
// ||v - A U y|| / ||v||, which |g_0| / ||b|| turns into the pair's residual relative to ||b||.
int solve_restarted(lt_handle* h, const Plan& plan, const lt_opts& o, int R, int rinit, const DevPoints* rec, int ns,
                    int ntimes, double* phi_out, KrylovOut* k, lt_stats* stats, std::vector<int>* iters, bool* ok) {
    hipStream_t st = h->stream;
    const int N = h->N;
    const size_t N2 = 2 * (size_t)N;
    const int Ks = plan.ntimes * plan.nk;
    int rc = 0;
    const double* b0 = k->b;
    double* cb = wsp<double>(h, "rs_b", R * N2, &rc);                  // each cycle's right-hand sides
    double* g0 = wsp<double>(h, "rs_g0", 2 * (size_t)R * Ks, &rc);     // each pair's g_0 (complex)
    double* bn = wsp<double>(h, "rs_bnorm", R, &rc);                   // ||b||
    double* cn = wsp<double>(h, "rs_cnorm", R, &rc);                   // ||v|| of the last cycle
    double* npart = wsp<double>(h, "rs_part", (size_t)R * reduce_blocks(N, R), &rc);
    int* rflag = wsp<int>(h, "rs_flag", R, &rc);
    if (!cb || !g0 || !bn || !cn || !npart || !rflag) return rc;
    LT_TRY(launch_norms(st, N, R, N2, b0, npart, bn, nullptr));
    LT_TRY(launch_fill_g0(st, R, Ks, bn, g0));
    LT_HIP(hipMemcpyAsync(cb, b0, R * N2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    const size_t nphi = (size_t)(ns > 0 ? ns : 1) * rec->n * ntimes;
    LT_HIP(hipMemsetAsync(phi_out, 0, nphi * sizeof(double), st));
    // every cycle reserves the same basis, so a right-hand side that has finished keeps its
    // last cycle's basis, least-squares state and gathers until the end
    lt_opts oc = o;
    oc.maxit = o.restart;
    const int max_cycles = (o.maxit + o.restart - 1) / o.restart;
    std::vector<int> only(R, 1), mlast(R, 0), hm(R);
    iters->assign(R, 0);
    k->b = cb;
    int vcycles = 0;
    for (int c = 0; c < max_cycles; ++c) {
        RestartIn rin;
        rin.start.g0 = g0;
        rin.start.bnorm = bn;
        rin.j0 = c * o.restart;
        LT_TRY(run_krylov(h, plan, oc, R, rinit, rec, k, c ? &only : nullptr, &rin));
        vcycles += k->vcycles;
        // this cycle's heads: the right-hand sides it did not solve keep their earlier column
        // counts, which count zero in the sum
        LT_HIP(hipMemcpyAsync(hm.data(), k->mcols, R * sizeof(int), hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < R; ++r) {
            if (!only[r]) {
                hm[r] = 0;
            } else {
                mlast[r] = hm[r];
                (*iters)[r] += hm[r];
            }
        }
        LT_HIP(hipMemcpyAsync(k->mcols, hm.data(), R * sizeof(int), hipMemcpyHostToDevice, st));
        LT_TRY(launch_heads(st, ns, rinit < R ? rinit : -1, rec->n, ntimes, plan.nk, k->wq, k->w, k->G, k->Y,
                            k->mcols, k->jmax, phi_out, true));
        LT_HIP(hipStreamSynchronize(st));
        if (k->converged) break;
        // the right-hand sides that go on, from their collinear residuals
        for (int r = 0; r < R; ++r) only[r] = k->notconv[r];
        LT_HIP(hipMemcpyAsync(rflag, only.data(), R * sizeof(int), hipMemcpyHostToDevice, st));
        LT_TRY(launch_restart_rhs(st, R, N, Ks, k->Q, k->qstride, k->mcols, rflag, k->eta, cb, g0));
        LT_HIP(hipStreamSynchronize(st));
    }
    bool conv = true;
    for (int r = 0; r < R; ++r) conv = conv && !k->notconv[r];
    k->converged = conv;
    k->vcycles = vcycles;
    k->iters_max = 0;
    for (int r = 0; r < R; ++r) k->iters_max = std::max(k->iters_max, (*iters)[r]);
    LT_HIP(hipMemcpyAsync(k->mcols, mlast.data(), R * sizeof(int), hipMemcpyHostToDevice, st));
    bool tr_ok = true;
    if (o.true_residual) {
        const int mmax = *std::max_element(mlast.begin(), mlast.end());
        double* KU = wsp<double>(h, "KU", (size_t)R * std::max(mmax, 1) * N2, &rc);
        const int nb = true_res_blocks(N, R);
        double* part = wsp<double>(h, "tpart", (size_t)R * Ks * nb, &rc);
        double* tr = wsp<double>(h, "trel", (size_t)R * Ks, &rc);
        if (!KU || !part || !tr) return rc;
        LT_TRY(launch_norms(st, N, R, N2, cb, npart, cn, nullptr));
        LT_TRY(launch_unscale_y(st, R, Ks, k->jmax, k->mcols, g0, cn, k->Y));
        LT_TRY(launch_true_residual_cols(st, h->levels[0].v64(), R, Ks, k->jmax, mmax, k->U, k->ustride, k->Y,
                                         k->mcols, k->zs, cb, cn, KU, part, tr));
        std::vector<double> ht((size_t)R * Ks), hg((size_t)2 * R * Ks), hb(R);
        LT_HIP(hipMemcpyAsync(ht.data(), tr, ht.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        LT_HIP(hipMemcpyAsync(hg.data(), g0, hg.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        LT_HIP(hipMemcpyAsync(hb.data(), bn, R * sizeof(double), hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        double mx = 0.0;
        for (int r = 0; r < R; ++r) {
            const std::vector<double>& om = r >= rinit ? plan.omega_init : plan.omega;
            double wr = 0.0;
            for (int kk = 0; kk < Ks; ++kk) {
                const size_t pi = (size_t)r * Ks + kk;
                const double rel = hb[r] > 0.0 ? ht[pi] * std::hypot(hg[2 * pi], hg[2 * pi + 1]) / hb[r] : 0.0;
                ht[pi] = rel;
                wr = std::max(wr, om[kk] * rel);
            }
            mx = std::max(mx, wr);
            tr_ok = tr_ok && wr <= o.tol;
        }
        if (stats) {
            stats->true_relres_max = mx;
            if (stats->true_relres) std::memcpy(stats->true_relres, ht.data(), ht.size() * sizeof(double));
        }
    }
    *ok = conv && tr_ok;
    return 0;
}

int prof_start(lt_handle* h, int target) {
    h->prof_target = target;
    h->prof_used = 0;
    h->prof_host_bytes = 0.0;
    if (!target) return 0;
    int rc = 0;
    h->prof_counter = wsp<unsigned long long>(h, "prof_counter", 1, &rc);
    if (!h->prof_counter) return rc;
    LT_HIP(hipMemsetAsync(h->prof_counter, 0, sizeof(unsigned long long), h->stream));
    return 0;
}

int prof_finish(lt_handle* h, lt_stats* s) {
    if (!h->prof_target) {
        if (s) { s->prof_launches = 0; s->prof_ms = 0; s->prof_bytes = 0; }
        return 0;
    }
    LT_HIP(hipStreamSynchronize(h->stream));
    double ms = 0;
    for (int k = 0; k + 1 < h->prof_used; k += 2) {
        float e = 0;
        LT_HIP(hipEventElapsedTime(&e, h->prof_events[k], h->prof_events[k + 1]));
        ms += e;
    }
    unsigned long long bytes = 0;
    LT_HIP(hipMemcpy(&bytes, h->prof_counter, sizeof(bytes), hipMemcpyDeviceToHost));
    if (s) {
        s->prof_launches = h->prof_used / 2;
        s->prof_ms = ms;
        s->prof_bytes = (double)bytes + h->prof_host_bytes;
    }
    h->prof_target = 0;
    return 0;
}

void fill_stats(lt_stats* s, const KrylovOut& k, int nlev, double secs, int resolves, const lt_handle* h) {
    if (!s) return;
    s->resolves = resolves;
    s->factorizations = h->exact_factorizations;
    s->factor_ms = h->exact_factor_ms;
    s->n_rhs = k.R;
    s->n_shifts = k.Ks;
    s->iters_max = k.iters_max;
    s->vcycles = k.vcycles;
    s->net_applied = k.net_applied;
    s->net_rejected = k.net_rejected;
    s->net_disabled_at = k.net_disabled_at;
    s->levels = nlev;
    s->seconds = secs;
}

// Checks of an lt_sources (before any work).  adjoint: wells only, and receivers count
// towards the right-hand sides.
int check_sources(const lt_sources* src, int extra_rhs, bool adjoint, const char* who) {
    if (!src || src->pts.n < 0 || (src->pts.n > 0 && !src->pts.xyz)) {
        set_last_error(std::string(who) + ": bad sources");
        return LT_EINVAL;
    }
    if (adjoint && src->phi0) {
        set_last_error(std::string(who) + ": the sensitivities take wells only (phi0 must be NULL)");
        return LT_EUNSUPPORTED;
    }
    if (src->pts.n == 0 && (adjoint || !src->phi0)) {
        set_last_error(std::string(who) + ": no wells and no initial head");
        return LT_EINVAL;
    }
    if ((long long)src->pts.n + (src->phi0 ? 1 : 0) + extra_rhs > kMaxRhs) {
        set_last_error(std::string(who) + ": at most " + std::to_string(kMaxRhs) + " right-hand sides per call");
        return LT_EINVAL;
    }
    if (src->q)
        for (int i = 0; i < src->pts.n; ++i)
            if (!std::isfinite(src->q[i])) {
                set_last_error(std::string(who) + ": rates must be finite");
                return LT_EINVAL;
            }
    return 0;
}

// Weights of the wells' right-hand sides q_s B_s^T (heads are linear in the rates).
void scale_by_rates(const lt_sources* src, PointsCSR* c) {
    if (!src->q) return;
    for (int s = 0; s < src->pts.n; ++s)
        for (int e = c->off[s]; e < c->off[s + 1]; ++e) c->wt[e] *= src->q[s];
}

}  // namespace

namespace lt {

// One V-cycle on the handle's stream; FP32 cycles convert on entry and exit.  With
// h->arena_plan set, only the workspace bytes are counted and nothing is launched.
int vcycle_call(lt_handle* h, cdouble tau, int precision, int nu1, int nu2, const double* b, double* x, int nvec) {
    const size_t per = 2 * (size_t)h->N * nvec;
    int rc = 0;
    if (precision == LT_PREC_FP64) {
        if (!h->cp3d) return mg_vcycle<double>(h, tau, nu1, nu2, nvec, nullptr, x, b);
        // 3D: the cycle's vectors in colour-planar order
        double* bc = wsp<double>(h, "vc_b64", per, &rc);
        double* xc = wsp<double>(h, "vc_x64", per, &rc);
        if (!bc || !xc) return rc;
        if (!h->arena_plan)
            LT_TRY(convert_vectors_cp<double, double>(h->stream, b, bc, nvec, h->N, h->grid.n[0], h->grid.n[1], 0));
        LT_TRY(mg_vcycle<double>(h, tau, nu1, nu2, nvec, nullptr, xc, bc));
        if (h->arena_plan) return 0;
        return convert_vectors_cp<double, double>(h->stream, xc, x, nvec, h->N, h->grid.n[0], h->grid.n[1], 1);
    }
    float* bf = wsp<float>(h, "vc_b32", per, &rc);
    float* xf = wsp<float>(h, "vc_x32", per, &rc);
    if (!bf || !xf) return rc;
    // the FP32 cycle's vectors are colour-planar on 3D grids that allow it
    const int cpnx = h->cp3d ? h->grid.n[0] : 0;
    if (!h->arena_plan) LT_TRY(convert_vectors_cp<double, float>(h->stream, b, bf, nvec, h->N, cpnx, h->grid.n[1], 0));
    LT_TRY(mg_vcycle<float>(h, tau, nu1, nu2, nvec, nullptr, xf, bf));
    if (h->arena_plan) return 0;
    return convert_vectors_cp<float, double>(h->stream, xf, x, nvec, h->N, cpnx, h->grid.n[1], 1);
}

}  // namespace lt

extern "C" {

void lt_opts_default(lt_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->maxit = 200;
    o->precision = LT_PREC_FP64;
    o->n_tau = 1;
    o->tau_reim = nullptr;
    o->nu1 = 2;
    o->nu2 = 2;
    o->inner_max = 30;
    o->relax = 1.0;
    o->true_residual = 1;
    o->precond = LT_PRECOND_GMG;
    o->net_keep = 0.05;
    o->graph = 0;
}

const char* lt_strerror(int code) {
    switch (code) {
        case LT_OK: return "LT_OK";
        case LT_EINVAL: return "LT_EINVAL: invalid argument";
        case LT_EHIP: return "LT_EHIP: HIP runtime error";
        case LT_ENOMEM: return "LT_ENOMEM: out of memory";
        case LT_EUNSUPPORTED: return "LT_EUNSUPPORTED: not supported";
        case LT_WNOTCONV: return "LT_WNOTCONV: not converged within maxit";
        default: return "unknown lt status";
    }
}

const char* lt_last_error(void) { return lt::g_last_error.c_str(); }

int lt_setup(const lt_grid* grid, const double* kappa, const double* S, const lt_bc* bc, void* hip_stream,
             lt_handle** out) {
    if (!grid || !kappa || !S || !out) {
        set_last_error("lt_setup: NULL argument");
        return LT_EINVAL;
    }
    *out = nullptr;
    if (grid->ndim < 2 || grid->ndim > 3) {
        set_last_error("lt_setup: ndim must be 2 or 3");
        return LT_EINVAL;
    }
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1 || !(grid->h[a] > 0.0) || (a >= grid->ndim && grid->n[a] != 1)) {
            set_last_error("lt_setup: bad grid shape or spacing");
            return LT_EINVAL;
        }
    }
    long long Nll = (long long)grid->n[0] * grid->n[1] * grid->n[2];
    if (Nll < 2 || Nll > kMaxCells) {
        set_last_error("lt_setup: grid too small or too large (2 to 2^28 cells)");
        return LT_EINVAL;
    }
    lt_handle* h = new (std::nothrow) lt_handle();
    if (!h) return LT_ENOMEM;
    h->grid = *grid;
    if (bc)
        h->bc = *bc;
    else
        std::memset(&h->bc, 0, sizeof(h->bc));
    bool water_table = false;
    for (int f = 0; f < 6; ++f) {
        const int t = h->bc.face[f];
        if (t != LT_BC_DIRICHLET0 && t != LT_BC_NEUMANN0 && t != LT_BC_WATER_TABLE) {
            delete h;
            set_last_error("lt_setup: unknown boundary condition");
            return LT_EINVAL;
        }
        if (t == LT_BC_WATER_TABLE) {
            if (f / 2 >= grid->ndim) {
                delete h;
                set_last_error("lt_setup: a water-table face must lie on a grid axis");
                return LT_EINVAL;
            }
            water_table = true;
        }
    }
    if (!water_table)
        h->bc.sy = 0.0;
    else if (!(h->bc.sy >= 0.0) || !std::isfinite(h->bc.sy)) {
        delete h;
        set_last_error("lt_setup: the specific yield must be finite and >= 0");
        return LT_EINVAL;
    }
    h->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_last_error("lt_setup: no HIP device");
        return LT_EHIP;
    }
    h->N = (int)Nll;
    // the scratch of allocation-free calls: its address on this device, taken once per device
    int rc = noalloc_init_device(h->device);
    if (rc >= 0) rc = mg_build(h, kappa, S);
    if (rc >= 0) rc = h->kappa.reserve(sizeof(double) * (size_t)h->N);
    if (rc >= 0 && hipMemcpyAsync(h->kappa.p, kappa, sizeof(double) * (size_t)h->N, hipMemcpyDeviceToDevice,
                                  h->stream) != hipSuccess) {
        set_last_error("lt_setup: copying kappa failed");
        rc = LT_EHIP;
    }
    if (rc < 0) {
        delete h;
        return rc;
    }
    *out = h;
    return LT_OK;
}

int lt_setup_p1(const lt_grid* cells, const double* kappa, const double* S, void* hip_stream, lt_handle** out) {
    if (!cells || !kappa || !S || !out) {
        set_last_error("lt_setup_p1: NULL argument");
        return LT_EINVAL;
    }
    *out = nullptr;
    bool ok = cells->ndim == 2 || cells->ndim == 3;
    for (int a = 0; a < 3 && ok; ++a)
        ok = a < cells->ndim ? cells->n[a] >= 3 && cells->h[a] > 0.0 : cells->n[a] == 1;
    if (!ok) {
        set_last_error("lt_setup_p1: a 2D or 3D grid of at least 3 cells per axis with positive spacings");
        return LT_EINVAL;
    }
    const long long Nll = (long long)(cells->n[0] - 1) * (cells->n[1] - 1) *
                          (cells->ndim == 3 ? cells->n[2] - 1 : 1);
    if (Nll > kMaxCells) {
        set_last_error("lt_setup_p1: grid too large");
        return LT_EINVAL;
    }
    lt_handle* h = new (std::nothrow) lt_handle();
    if (!h) return LT_ENOMEM;
    h->p1 = true;
    h->cells = *cells;
    // the unknowns: the interior vertices, spaced like the cells
    h->grid = *cells;
    for (int a = 0; a < cells->ndim; ++a) h->grid.n[a] = cells->n[a] - 1;
    std::memset(&h->bc, 0, sizeof(h->bc));  // zero head on every wall
    h->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_last_error("lt_setup_p1: no HIP device");
        return LT_EHIP;
    }
    h->N = (int)Nll;
    int rc = noalloc_init_device(h->device);
    if (rc >= 0) rc = mg_build(h, kappa, S, &h->cells);
    // the parameters the sensitivities are taken to: kappa then S, per cell of `cells`
    const size_t nc = (size_t)cells->n[0] * cells->n[1] * (cells->ndim == 3 ? cells->n[2] : 1);
    if (rc >= 0) rc = h->kappa.reserve(2 * sizeof(double) * nc);
    if (rc >= 0 && (hipMemcpyAsync(h->kappa.p, kappa, sizeof(double) * nc, hipMemcpyDeviceToDevice, h->stream) !=
                        hipSuccess ||
                    hipMemcpyAsync(h->kappa.as<double>() + nc, S, sizeof(double) * nc, hipMemcpyDeviceToDevice,
                                   h->stream) != hipSuccess)) {
        set_last_error("lt_setup_p1: copying kappa and S failed");
        rc = LT_EHIP;
    }
    if (rc < 0) {
        delete h;
        return rc;
    }
    *out = h;
    return LT_OK;
}

void lt_destroy(lt_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int lt_level_shape(lt_handle* h, int level, int* n_out) {
    if (!h) return LT_EINVAL;
    int nl = (int)h->levels.size();
    if (level < 0 || level >= nl) return LT_EINVAL;
    if (n_out)
        for (int a = 0; a < 3; ++a) n_out[a] = h->levels[level].n[a];
    return nl;
}

int lt_talbot(int nz, double t, double* z_reim, double* w_reim) {
    if (!z_reim || !w_reim) return LT_EINVAL;
    std::vector<cdouble> z(nz / 2 > 0 ? nz / 2 : 1), w(z.size());
    int rc = talbot(nz, t, z.data(), w.data());
    if (rc < 0) return rc;
    for (int k = 0; k < nz / 2; ++k) {
        z_reim[2 * k] = z[k].real();
        z_reim[2 * k + 1] = z[k].imag();
        w_reim[2 * k] = w[k].real();
        w_reim[2 * k + 1] = w[k].imag();
    }
    return 0;
}

int lt_krylov_basis(lt_handle* h, int rhs, int mmax, double* V, double* U, double* Hbar, int* m_out) {
    if (!h || h->last_R < 1 || rhs < 0 || rhs >= h->last_R || mmax < 0) {
        set_last_error("lt_krylov_basis: no basis for this right-hand side");
        return LT_EINVAL;
    }
    hipStream_t st = h->stream;
    const int R = h->last_R, jmax = h->last_jmax;
    const size_t N2 = 2 * (size_t)h->N;
    const size_t qstride = (size_t)(jmax + 1) * N2, ustride = (size_t)jmax * N2;
    const int hstride = 2 * (jmax + 2);
    const double* Q = h->ws["Q"].as<double>();
    const double* Ud = h->ws["U"].as<double>();
    const double* Hd = h->ws["H"].as<double>();
    const int* ints = h->ws["ints"].as<int>();
    const double* small = h->ws["small"].as<double>();
    int m = 0;
    double scale = 0;
    LT_HIP(hipStreamSynchronize(st));
    LT_HIP(hipMemcpy(&m, ints + 2 * (size_t)R + rhs, sizeof(int), hipMemcpyDeviceToHost));  // mcols
    LT_HIP(hipMemcpy(&scale, small + rhs, sizeof(double), hipMemcpyDeviceToHost));
    if (m_out) *m_out = m;
    if (mmax < m) {
        set_last_error("lt_krylov_basis: mmax is smaller than the basis");
        return LT_EINVAL;
    }
    if (V && m > 0) {
        // the last column is kept unnormalised by the solver (its scale 1 / h_{m+1,m} is applied
        // by the next iteration's first read)
        LT_HIP(hipMemcpy(V, Q + qstride * rhs, (m + 1) * N2 * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < N2; ++i) V[(size_t)m * N2 + i] *= scale;
    }
    if (U && m > 0) LT_HIP(hipMemcpy(U, Ud + ustride * rhs, m * N2 * sizeof(double), hipMemcpyDeviceToHost));
    if (Hbar && m > 0) {
        std::vector<double> hc((size_t)m * hstride);
        LT_HIP(hipMemcpy(hc.data(), Hd + (size_t)jmax * hstride * rhs, hc.size() * sizeof(double),
                         hipMemcpyDeviceToHost));
        for (int j = 0; j < m; ++j)
            for (int i = 0; i <= m; ++i) {
                const bool in = i <= j + 1;
                Hbar[2 * ((size_t)j * (m + 1) + i)] = in ? hc[(size_t)j * hstride + 2 * i] : 0.0;
                Hbar[2 * ((size_t)j * (m + 1) + i) + 1] = in ? hc[(size_t)j * hstride + 2 * i + 1] : 0.0;
            }
    }
    return LT_OK;
}

int lt_apply_operator(lt_handle* h, int level, double tau_re, double tau_im, const double* x, double* y, int nvec) {
    if (!h || !x || !y || nvec < 1 || level < 0 || level >= (int)h->levels.size()) return LT_EINVAL;
    return apply_operator<double>(h, level, cdouble(tau_re, tau_im), x, y, nvec, nullptr);
}

int lt_vcycle(lt_handle* h, double tau_re, double tau_im, int precision, int nu1, int nu2, const double* b,
              double* x, int nvec) {
    if (!h || !b || !x || nvec < 1 || nvec > kMaxRhs || nu1 < 0 || nu2 < 0 || nu1 + nu2 < 1 ||
        (precision != LT_PREC_FP64 && precision != LT_PREC_MIXED))
        return LT_EINVAL;
    return vcycle_call(h, cdouble(tau_re, tau_im), precision, nu1, nu2, b, x, nvec);
}

int lt_solve(lt_handle* h, const lt_sources* src, const double* times, int ntimes, const lt_contour* contour,
             const lt_points* receivers, const lt_opts* opts, double* phi_out, lt_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!h || !times || ntimes < 1 || !contour || !receivers || receivers->n < 1 || !phi_out) {
        set_last_error("lt_solve: bad argument");
        return LT_EINVAL;
    }
    LT_TRY(check_sources(src, 0, false, "lt_solve"));
    for (int t = 0; t < ntimes; ++t)
        if (!(times[t] > 0.0) || !std::isfinite(times[t])) {
            set_last_error("lt_solve: times must be positive");
            return LT_EINVAL;
        }
    lt_opts o;
    if (opts) {
        LT_TRY(validate_opts(opts));
        o = *opts;
    } else {
        lt_opts_default(&o);
    }
    if (contour->nz < 2 || contour->nz % 2 || contour->nz > 512) {
        set_last_error("lt_solve: contour nz must be even, 2..512");
        return LT_EINVAL;
    }
    Plan plan;
    LT_TRY(make_plan(times, ntimes, contour->nz, 1.0, &o, &plan));
    PointsCSR sc, rcsr;
    if (h->p1) {
        LT_TRY(points_csr_p1(h->cells, &src->pts, &sc));
        LT_TRY(points_csr_p1(h->cells, receivers, &rcsr));
    } else {
        LT_TRY(points_csr(h->grid, &src->pts, &sc));
        LT_TRY(points_csr(h->grid, receivers, &rcsr));
    }
    scale_by_rates(src, &sc);
    DevPoints ds, dr;
    LT_TRY(upload_points(h, sc, "src", &ds));
    LT_TRY(upload_points(h, rcsr, "rec", &dr));
    const int ns = src->pts.n;
    const int R = ns + (src->phi0 ? 1 : 0);
    const int rinit = src->phi0 ? ns : R;
    const size_t N2 = 2 * (size_t)h->N;
    int rc = 0;
    double* b = wsp<double>(h, "b", R * N2, &rc);
    if (!b) return rc;
    LT_HIP(hipMemsetAsync(b, 0, R * N2 * sizeof(double), h->stream));
    if (ns > 0) LT_TRY(launch_scatter_points(h->stream, ns, h->N, ds.off, ds.cell, ds.wt, b));
    if (src->phi0) LT_TRY(launch_mass_rhs(h->stream, h->N, h->levels[0].v64().m, src->phi0, b + (size_t)ns * N2));
    KrylovOut k;
    k.b = b;
    h->exact_factorizations = 0;
    h->exact_factor_ms = 0.0;
    LT_TRY(prof_start(h, o.profile));
    int resolves = 0;
    bool ok = false;
    if (o.restart > 0) {
        std::vector<int> its;
        LT_TRY(solve_restarted(h, plan, o, R, rinit, &dr, ns, ntimes, phi_out, &k, stats, &its, &ok));
        LT_HIP(hipStreamSynchronize(h->stream));
        if (stats && stats->iters_per_rhs) std::memcpy(stats->iters_per_rhs, its.data(), R * sizeof(int));
    } else {
        LT_TRY(solve_checked(h, plan, o, R, rinit, &dr, &k, stats, &resolves, &ok));
        LT_TRY(launch_heads(h->stream, ns, src->phi0 ? ns : -1, dr.n, ntimes, plan.nk, k.wq, k.w, k.G, k.Y, k.mcols,
                            k.jmax, phi_out));
        LT_HIP(hipStreamSynchronize(h->stream));
        if (stats && stats->iters_per_rhs)
            LT_HIP(hipMemcpy(stats->iters_per_rhs, k.mcols, R * sizeof(int), hipMemcpyDeviceToHost));
    }
    LT_TRY(prof_finish(h, stats));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, k, (int)h->levels.size(), secs, resolves, h);
    return ok ? LT_OK : LT_WNOTCONV;
}

int lt_adjoint(lt_handle* h, const lt_sources* src, const lt_points* receivers, const double* times, int ntimes,
               const lt_contour* contour, const lt_opts* opts, double* dlnK, double* dlnS, lt_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!h || !receivers || receivers->n < 1 || !times || ntimes < 1 || !contour || (!dlnK && !dlnS)) {
        set_last_error("lt_adjoint: bad argument");
        return LT_EINVAL;
    }
    LT_TRY(check_sources(src, receivers->n, true, "lt_adjoint"));
    for (int t = 0; t < ntimes; ++t)
        if (!(times[t] > 0.0) || !std::isfinite(times[t])) {
            set_last_error("lt_adjoint: times must be positive");
            return LT_EINVAL;
        }
    lt_opts o;
    if (opts) {
        LT_TRY(validate_opts(opts));
        o = *opts;
    } else {
        lt_opts_default(&o);
    }
    if (contour->nz < 2 || contour->nz % 2 || contour->nz > 512) {
        set_last_error("lt_adjoint: contour nz must be even, 2..512");
        return LT_EINVAL;
    }
    Plan plan;
    LT_TRY(make_plan(times, ntimes, contour->nz, 1.0, &o, &plan, true));
    // right-hand sides: every well's q_s b_s, then every receiver's B_m^T (adjoint fields)
    const int ns = src->pts.n, nr = receivers->n, R = ns + nr;
    PointsCSR sc, rcsr, ac;
    if (h->p1) {
        LT_TRY(points_csr_p1(h->cells, &src->pts, &sc));
        LT_TRY(points_csr_p1(h->cells, receivers, &rcsr));
    } else {
        LT_TRY(points_csr(h->grid, &src->pts, &sc));
        LT_TRY(points_csr(h->grid, receivers, &rcsr));
    }
    scale_by_rates(src, &sc);
    ac = sc;
    for (int i = 0; i < nr; ++i) {
        for (int e = rcsr.off[i]; e < rcsr.off[i + 1]; ++e) {
            ac.cell.push_back(rcsr.cell[e]);
            ac.wt.push_back(rcsr.wt[e]);
        }
        ac.off.push_back((int)ac.cell.size());
    }
    DevPoints da;
    LT_TRY(upload_points(h, ac, "adj", &da));
    const size_t N2 = 2 * (size_t)h->N;
    int rc = 0;
    double* b = wsp<double>(h, "b", R * N2, &rc);
    if (!b) return rc;
    LT_HIP(hipMemsetAsync(b, 0, R * N2 * sizeof(double), h->stream));
    LT_TRY(launch_scatter_points(h->stream, R, h->N, da.off, da.cell, da.wt, b));
    KrylovOut k;
    k.b = b;
    h->exact_factorizations = 0;
    h->exact_factor_ms = 0.0;
    LT_TRY(prof_start(h, o.profile));
    int resolves = 0;
    bool ok = false;
    LT_TRY(solve_checked(h, plan, o, R, R, nullptr, &k, stats, &resolves, &ok));
    // nodal fields of one time at a time, then the cell-wise contraction
    const int nk = plan.nk;
    double* X = wsp<double>(h, "Xadj", (size_t)R * nk * N2, &rc);
    if (!X) return rc;
    for (int t = 0; t < ntimes; ++t) {
        LT_TRY(launch_form_x(h->stream, h->N, R, nk, t * nk, k.Ks, k.U, k.ustride, k.Y, k.jmax, k.mcols, X));
        if (h->p1) {
            const size_t nc = (size_t)h->cells.n[0] * h->cells.n[1] * (h->cells.ndim == 3 ? h->cells.n[2] : 1);
            const double* pk = h->kappa.as<double>();
            LT_TRY(launch_sens_p1(h->stream, h->cells, pk, pk + nc, ns, nr, nk, t, ntimes, (size_t)h->N, X, k.zs,
                                  k.wq, dlnK, dlnS));
            continue;
        }
        const LevelView<double> L0 = h->levels[0].v64();
        const double* mS = h->mstor.p ? h->mstor.as<double>() : L0.m;
        LT_TRY(launch_sens(h->stream, L0, h->kappa.as<double>(), mS, ns, nr, nk, t, ntimes, X, k.zs, k.wq, dlnK,
                           dlnS));
    }
    LT_HIP(hipStreamSynchronize(h->stream));
    if (stats && stats->iters_per_rhs)
        LT_HIP(hipMemcpy(stats->iters_per_rhs, k.mcols, R * sizeof(int), hipMemcpyDeviceToHost));
    LT_TRY(prof_finish(h, stats));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(stats, k, (int)h->levels.size(), secs, resolves, h);
    return ok ? LT_OK : LT_WNOTCONV;
}

// ---------------------------------------------------------------- learned preconditioner
static int unet_check_grid(const lt_handle* h) {
    if (h->grid.ndim != 2 || h->grid.n[0] % 128 || h->grid.n[1] % 8) {
        set_last_error("the network needs a 2D grid with nx % 128 == 0 and ny % 8 == 0");
        return LT_EUNSUPPORTED;
    }
    return 0;
}

int lt_unet_create(unsigned long long seed, void* hip_stream, lt_unet** out) {
    if (!out) return LT_EINVAL;
    *out = nullptr;
    lt_unet* u = new (std::nothrow) lt_unet();
    if (!u) return LT_ENOMEM;
    u->net.stream = static_cast<hipStream_t>(hip_stream);
    std::vector<float> p;
    unet_init_params(&u->net, seed, p);
    int rc = unet_upload(&u->net, u->net.stream, p.data());
    if (rc >= 0 && hipStreamSynchronize(u->net.stream) != hipSuccess) rc = LT_EHIP;
    if (rc < 0) {
        delete u;
        return rc;
    }
    *out = u;
    return LT_OK;
}

long long lt_unet_nparams(const lt_unet* u) { return u ? (long long)u->net.nparams : LT_EINVAL; }

int lt_unet_get_params(lt_unet* u, float* host) {
    if (!u || !host) return LT_EINVAL;
    LT_HIP(hipStreamSynchronize(u->net.stream));
    LT_HIP(hipMemcpy(host, u->net.ws["params"].p, u->net.nparams * sizeof(float), hipMemcpyDeviceToHost));
    return LT_OK;
}

int lt_unet_set_params(lt_unet* u, const float* host) {
    if (!u || !host) return LT_EINVAL;
    LT_TRY(unet_upload(&u->net, u->net.stream, host));
    u->net.adam_t = 0;
    LT_HIP(hipStreamSynchronize(u->net.stream));
    return LT_OK;
}

int lt_unet_apply(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r, double* e) {
    if (!u || !h || !r || !e || nvec < 1) return LT_EINVAL;
    LT_TRY(unet_check_grid(h));
    LT_TRY(unet_apply<double>(&u->net, h->stream, h->levels[0].v64(), h->lnDbar, cdouble(tau_re, tau_im), nvec, r,
                              e, nullptr));
    LT_HIP(hipStreamSynchronize(h->stream));
    return LT_OK;
}

static int unet_loss_grad(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r,
                          const double* e, float* loss) {
    LT_TRY(unet_check_grid(h));
    UNet* net = &u->net;
    hipStream_t st = h->stream;
    const LevelView<double> L0 = h->levels[0].v64();
    LT_TRY(unet_features<double>(net, st, L0, h->lnDbar, cdouble(tau_re, tau_im), nvec, r));
    LT_TRY(unet_forward(net, st, nvec, L0.ny, L0.nx));
    DevBuf& lb = net->ws["loss"];
    LT_TRY(lb.reserve(sizeof(float) * nvec));
    LT_TRY(unet_loss_and_grad(net, st, L0, nvec, e, lb.as<float>()));
    DevBuf& gb = net->ws["grad"];
    LT_TRY(gb.reserve(sizeof(float) * net->nparams));
    LT_HIP(hipMemsetAsync(gb.p, 0, sizeof(float) * net->nparams, st));
    LT_TRY(unet_backward(net, st, nvec, L0.ny, L0.nx, nullptr));
    if (loss) {
        std::vector<float> l(nvec);
        LT_HIP(hipMemcpyAsync(l.data(), lb.p, sizeof(float) * nvec, hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        double s = 0;
        for (float v : l) s += v;
        *loss = (float)(s / nvec);
    }
    return LT_OK;
}

int lt_unet_train_step(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r,
                       const double* e, float lr, float* loss) {
    if (!u || !h || !r || !e || nvec < 1 || !(lr >= 0.0f)) return LT_EINVAL;
    LT_TRY(unet_loss_grad(u, h, tau_re, tau_im, nvec, r, e, loss));
    if (lr > 0.0f) LT_TRY(unet_adam(&u->net, h->stream, lr));
    LT_HIP(hipStreamSynchronize(h->stream));
    return LT_OK;
}

int lt_unet_grad(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r, const double* e,
                 float* grad_host) {
    if (!u || !h || !r || !e || nvec < 1 || !grad_host) return LT_EINVAL;
    LT_TRY(unet_loss_grad(u, h, tau_re, tau_im, nvec, r, e, nullptr));
    LT_HIP(hipStreamSynchronize(h->stream));
    LT_HIP(hipMemcpy(grad_host, u->net.ws["grad"].p, u->net.nparams * sizeof(float), hipMemcpyDeviceToHost));
    return LT_OK;
}

int lt_unet_attach(lt_handle* h, lt_unet* u) {
    if (!h) return LT_EINVAL;
    if (u) LT_TRY(unet_check_grid(h));
    h->unet = u;
    return LT_OK;
}

void lt_unet_destroy(lt_unet* u) {
    if (!u) return;
    (void)hipStreamSynchronize(u->net.stream);
    delete u;
}

int lt_precond_solve(lt_handle* h, double tau_re, double tau_im, int nvec, const double* r, double* e, double tol,
                     int maxcycles) {
    if (!h || !r || !e || nvec < 1 || !(tol > 0.0) || maxcycles < 1) return LT_EINVAL;
    hipStream_t st = h->stream;
    const int N = h->N;
    const size_t N2 = 2 * (size_t)N;
    int rc = 0;
    double* rho = wsp<double>(h, "ps_rho", nvec * N2, &rc);
    double* x = wsp<double>(h, "ps_x", nvec * N2, &rc);
    const int nb = reduce_blocks(N, nvec);
    double* part = wsp<double>(h, "ps_part", (size_t)nvec * nb, &rc);
    double* nrm = wsp<double>(h, "ps_nrm", 2 * (size_t)nvec, &rc);
    // 3D grids: the cycle reads a colour-planar copy of the residual and returns its
    // correction in that order
    double* lo = h->cp3d ? wsp<double>(h, "ps_lo", nvec * N2, &rc) : nullptr;
    if (!rho || !x || !part || !nrm || (h->cp3d && !lo)) return rc;
    const cdouble tau(tau_re, tau_im);
    const LevelView<double> L0 = h->levels[0].v64();
    LT_HIP(hipMemcpyAsync(rho, r, nvec * N2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (lo) LT_TRY(convert_vectors_cp<double, double>(st, r, lo, nvec, N, h->grid.n[0], h->grid.n[1], 0));
    LT_HIP(hipMemsetAsync(e, 0, nvec * N2 * sizeof(double), st));
    LT_TRY(launch_norms(st, N, nvec, N2, r, part, nrm + nvec, nullptr));
    std::vector<double> hn(2 * (size_t)nvec);
    for (int c = 0; c < maxcycles; ++c) {
        LT_TRY(mg_vcycle<double>(h, tau, 2, 2, nvec, nullptr, x, lo ? lo : rho));
        LT_TRY(launch_inner_update<double>(st, L0, tau, nvec, x, e, N2, nullptr, rho, lo, part, nullptr, lo ? 1 : 0));
        LT_TRY(launch_norms(st, N, nvec, N2, rho, part, nrm, nullptr));
        LT_HIP(hipMemcpyAsync(hn.data(), nrm, 2 * nvec * sizeof(double), hipMemcpyDeviceToHost, st));
        LT_HIP(hipStreamSynchronize(st));
        bool done = true;
        for (int v = 0; v < nvec; ++v) done = done && hn[v] <= tol * hn[nvec + v];
        if (done) return LT_OK;
    }
    return LT_WNOTCONV;
}

int lt_shift_invert(lt_handle* h, double tau_re, double tau_im, int nvec, const double* b, double* x) {
    if (!h || !b || !x || nvec < 1 || nvec > kMaxRhs) {
        set_last_error("lt_shift_invert: bad argument");
        return LT_EINVAL;
    }
    const size_t bytes = (size_t)nvec * 2 * (size_t)h->N * sizeof(double);
    const uintptr_t pb = (uintptr_t)b, px = (uintptr_t)x;
    if (pb < px + bytes && px < pb + bytes) {
        set_last_error("lt_shift_invert: x overlaps b");
        return LT_EINVAL;
    }
    int rc = 0;
    const ExactFactor* F = exact_factor(h, cdouble(tau_re, tau_im), &rc);
    if (!F) return rc;
    return exact_apply(h, F, nvec, b, 2 * (size_t)h->N, x, 2 * (size_t)h->N);
}


}  // extern "C"
