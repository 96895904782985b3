// Host planner: Talbot contour, preconditioner shift schedule, point weights,
// and a dense complex inverse for the coarsest multigrid level.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "lt_internal.h"

namespace lt {

// Optimised Talbot contour of Trefethen, Weideman and Schmelzer (2006), the
// parameters the paper adopts (eq:talbot; error ~ 3.89^-N, Section 2.3):
//   z(theta) = (N/t) (-0.6122 + 0.5017 theta cot(0.6407 theta) + 0.2645 i theta).
// Trapezoid rule at the midpoints theta_k = -pi + (k - 1/2) 2 pi / N
// (eqn:quadrature): w_k = -(i/N) e^{z_k t} z'(theta_k), and the conjugate-
// symmetric half with Im z > 0 is summed as 2 Re (eqn:half).
int talbot(int nz, double t, cdouble* z, cdouble* w) {
    if (nz < 2 || nz % 2 != 0 || !(t > 0.0) || !std::isfinite(t)) {
        set_last_error("talbot: nz must be even and >= 2, t > 0");
        return LT_EINVAL;
    }
    const double a0 = -0.6122, a1 = 0.5017, al = 0.6407, nu = 0.2645;
    const double sc = nz / t;
    const int half = nz / 2;
    for (int k = 0; k < half; ++k) {
        // upper half: theta = (k + 1/2) 2 pi / N for k = 0 .. N/2 - 1
        double th = (k + 0.5) * 2.0 * M_PI / nz;
        double at = al * th;
        double sn = std::sin(at), cs = std::cos(at);
        double cot = cs / sn;
        cdouble zz(sc * (a0 + a1 * th * cot), sc * nu * th);
        cdouble dz(sc * a1 * (cot - at / (sn * sn)), sc * nu);
        z[k] = zz;
        w[k] = cdouble(0.0, -1.0 / nz) * std::exp(zz * t) * dz;
    }
    return 0;
}

int make_plan(const double* times, int ntimes, int nz, double q, const lt_opts* o, Plan* p, bool storage) {
    if (ntimes < 1 || !times) {
        set_last_error("need at least one time");
        return LT_EINVAL;
    }
    p->ntimes = ntimes;
    p->nz = nz;
    p->nk = nz / 2;
    p->z.assign((size_t)ntimes * p->nk, 0.0);
    p->wq.assign((size_t)ntimes * p->nk, 0.0);
    p->omega.assign((size_t)ntimes * p->nk, 0.0);
    p->w.assign((size_t)ntimes * p->nk, 0.0);
    p->omega_init.assign((size_t)ntimes * p->nk, 0.0);
    std::vector<cdouble> w(p->nk);
    for (int t = 0; t < ntimes; ++t) {
        LT_TRY(talbot(nz, times[t], &p->z[(size_t)t * p->nk], w.data()));
        double mx = 0.0, mz = 0.0, mw = 0.0;
        for (int k = 0; k < p->nk; ++k) {
            cdouble zk = p->z[(size_t)t * p->nk + k];
            cdouble v = w[k] * (q / zk);  // qhat(z) = q / z for a constant rate from t = 0
            p->wq[(size_t)t * p->nk + k] = v;
            p->w[(size_t)t * p->nk + k] = w[k];
            mx = std::max(mx, std::abs(v));
            mz = std::max(mz, std::abs(v * zk));
            mw = std::max(mw, std::abs(w[k]));
        }
        // the initial head's term M phi0 enters with factor 1: its shifts weigh by |w_k|
        for (int k = 0; k < p->nk; ++k)
            p->omega_init[(size_t)t * p->nk + k] =
                o->conv == LT_CONV_RELATIVE ? 1.0 : (mw > 0 ? std::abs(w[k]) / mw : 1.0);
        // Heads weigh shift k by |w_k qhat_k|.  The storage sensitivity weighs the same
        // fields by |w_k qhat_k z_k| (the z dM/dp term of Section 5.2), so for it each
        // shift must meet the stricter of the two weightings.
        for (int k = 0; k < p->nk; ++k) {
            const cdouble v = p->wq[(size_t)t * p->nk + k], zk = p->z[(size_t)t * p->nk + k];
            double a = mx > 0 ? std::abs(v) / mx : 1.0;
            if (storage && mz > 0) a = std::max(a, std::abs(v * zk) / mz);
            if (o->conv == LT_CONV_RELATIVE) a = 1.0;  // every shift to tol ||b||
            p->omega[(size_t)t * p->nk + k] = a;
        }
    }
    p->tau_sched.clear();
    if (o->tau_reim && o->n_tau > 0) {
        for (int i = 0; i < o->n_tau; ++i) p->tau_sched.emplace_back(o->tau_reim[2 * i], o->tau_reim[2 * i + 1]);
        return 0;
    }
    // Candidates: the rule of Section 3 takes the contour nodes of smallest and largest
    // real part over every time.  A V-cycle needs K + tau M with a non-negative real
    // shift, so for the multigrid preconditioners the candidates are restricted to that
    // half plane; the exact factorisation takes every node (the smallest real part is
    // then negative, with Im z != 0).
    const bool any_half_plane = o->precond == LT_PRECOND_EXACT;
    std::vector<cdouble> cand;
    for (const cdouble& z : p->z)
        if (any_half_plane || z.real() >= 0.0) cand.push_back(z);
    if (cand.empty()) cand.push_back(cdouble(0.0, 0.0));
    auto lessre = [](const cdouble& a, const cdouble& b) { return a.real() < b.real(); };
    cdouble t1 = *std::min_element(cand.begin(), cand.end(), lessre);
    cdouble t2 = *std::max_element(cand.begin(), cand.end(), lessre);
    int nt = o->n_tau <= 0 ? 1 : o->n_tau;
    if (nt == 1) {
        p->tau_sched = {t1};
    } else if (nt == 2) {
        p->tau_sched = {t1, t1, t1, t2, t2};
    } else {
        std::vector<cdouble> s = cand;
        std::sort(s.begin(), s.end(), [](const cdouble& a, const cdouble& b) { return std::abs(a) < std::abs(b); });
        cdouble tm = s[s.size() / 2];
        p->tau_sched = {t1, tm, t2};
    }
    return 0;
}

static void axis_weights(double x, double h, int n, int* i, double* w, int* cnt) {
    double u = x / h - 0.5;
    int i0 = (int)std::floor(u);
    double f = u - i0;
    if (i0 < 0) {
        i[0] = 0; w[0] = 1.0; *cnt = 1;
    } else if (i0 >= n - 1) {
        i[0] = n - 1; w[0] = 1.0; *cnt = 1;
    } else {
        i[0] = i0; w[0] = 1.0 - f; *cnt = 1;
        if (f > 0.0) { i[1] = i0 + 1; w[1] = f; *cnt = 2; }
    }
}

int points_csr(const lt_grid& g, const lt_points* pts, PointsCSR* out) {
    out->off.assign(1, 0);
    out->cell.clear();
    out->wt.clear();
    if (!pts || pts->n <= 0) return 0;
    if (!pts->xyz) {
        set_last_error("points: xyz is NULL");
        return LT_EINVAL;
    }
    for (int p = 0; p < pts->n; ++p) {
        int idx[3][2];
        double wt[3][2];
        int cnt[3];
        for (int a = 0; a < 3; ++a) {
            double x = pts->xyz[3 * p + a];
            if (a < g.ndim) {
                double L = g.n[a] * g.h[a];
                if (!(x >= 0.0 && x <= L)) {
                    set_last_error("points: coordinate outside the domain");
                    return LT_EINVAL;
                }
                axis_weights(x, g.h[a], g.n[a], idx[a], wt[a], &cnt[a]);
            } else {
                idx[a][0] = 0; wt[a][0] = 1.0; cnt[a] = 1;
            }
        }
        for (int c = 0; c < cnt[2]; ++c)
            for (int b = 0; b < cnt[1]; ++b)
                for (int a = 0; a < cnt[0]; ++a) {
                    double w = wt[0][a] * wt[1][b] * wt[2][c];
                    if (w == 0.0) continue;
                    out->cell.push_back(idx[0][a] + g.n[0] * (idx[1][b] + g.n[1] * idx[2][c]));
                    out->wt.push_back(w);
                }
        out->off.push_back((int)out->cell.size());
    }
    return 0;
}

int points_csr_p1(const lt_grid& c, const lt_points* pts, PointsCSR* out) {
    out->off.assign(1, 0);
    out->cell.clear();
    out->wt.clear();
    if (!pts || pts->n <= 0) return 0;
    if (!pts->xyz) {
        set_last_error("points: xyz is NULL");
        return LT_EINVAL;
    }
    const int nx = c.n[0], ny = c.n[1];
    const double hx = c.h[0], hy = c.h[1];
    if (c.ndim == 3) {
        // the Kuhn tetrahedron of the cell that holds the point: the path through the axes in
        // decreasing order of the local coordinates, with barycentric coordinates
        // (1 - c1, c1 - c2, c2 - c3, c3) for the sorted coordinates c1 >= c2 >= c3
        for (int p = 0; p < pts->n; ++p) {
            int cell[3], ax[3] = {0, 1, 2};
            double loc[3];
            for (int a = 0; a < 3; ++a) {
                const double x = pts->xyz[3 * p + a];
                if (!(x >= 0.0 && x <= c.n[a] * c.h[a])) {
                    set_last_error("points: coordinate outside the domain");
                    return LT_EINVAL;
                }
                cell[a] = std::min(std::max((int)std::floor(x / c.h[a]), 0), c.n[a] - 1);
                loc[a] = x / c.h[a] - cell[a];
            }
            std::sort(ax, ax + 3, [&](int u, int v) { return loc[u] > loc[v]; });
            int v[3] = {cell[0], cell[1], cell[2]};
            const double lam[4] = {1.0 - loc[ax[0]], loc[ax[0]] - loc[ax[1]], loc[ax[1]] - loc[ax[2]], loc[ax[2]]};
            for (int s = 0; s < 4; ++s) {
                if (s > 0) ++v[ax[s - 1]];
                bool wall = false;
                for (int a = 0; a < 3; ++a) wall = wall || v[a] <= 0 || v[a] >= c.n[a];
                if (wall || lam[s] == 0.0) continue;
                out->cell.push_back((v[0] - 1) + (c.n[0] - 1) * ((v[1] - 1) + (c.n[1] - 1) * (v[2] - 1)));
                out->wt.push_back(lam[s]);
            }
            out->off.push_back((int)out->cell.size());
        }
        return 0;
    }
    for (int p = 0; p < pts->n; ++p) {
        const double x = pts->xyz[3 * p], y = pts->xyz[3 * p + 1];
        if (!(x >= 0.0 && x <= nx * hx && y >= 0.0 && y <= ny * hy)) {
            set_last_error("points: coordinate outside the domain");
            return LT_EINVAL;
        }
        const int i = std::min(std::max((int)std::floor(x / hx), 0), nx - 1);
        const int j = std::min(std::max((int)std::floor(y / hy), 0), ny - 1);
        const double xi = x / hx - i, eta = y / hy - j;
        int vi[3], vj[3];
        double lam[3];
        if (xi + eta <= 1.0) {  // the triangle (i, j), (i + 1, j), (i, j + 1)
            vi[0] = i; vj[0] = j; lam[0] = 1.0 - xi - eta;
            vi[1] = i + 1; vj[1] = j; lam[1] = xi;
            vi[2] = i; vj[2] = j + 1; lam[2] = eta;
        } else {                // the triangle (i + 1, j + 1), (i, j + 1), (i + 1, j)
            vi[0] = i + 1; vj[0] = j + 1; lam[0] = xi + eta - 1.0;
            vi[1] = i; vj[1] = j + 1; lam[1] = 1.0 - xi;
            vi[2] = i + 1; vj[2] = j; lam[2] = 1.0 - eta;
        }
        for (int a = 0; a < 3; ++a) {
            // wall vertices hold zero head
            if (vi[a] <= 0 || vj[a] <= 0 || vi[a] >= nx || vj[a] >= ny || lam[a] == 0.0) continue;
            out->cell.push_back((vi[a] - 1) + (nx - 1) * (vj[a] - 1));
            out->wt.push_back(lam[a]);
        }
        out->off.push_back((int)out->cell.size());
    }
    return 0;
}

int dense_inverse(int n, std::vector<cdouble>& a, std::vector<cdouble>& inv) {
    inv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = std::abs(a[(size_t)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = std::abs(a[(size_t)r * n + c]);
            if (v > best) { best = v; piv = r; }
        }
        if (!(best > 0.0)) return LT_EINVAL;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)c * n + k], a[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        }
        cdouble d = 1.0 / a[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] *= d;
            inv[(size_t)c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            cdouble f = a[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return 0;
}

}  // namespace lt
