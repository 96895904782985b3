/*
 * lt.h -- C ABI of the Laplace-transform shifted-system solver for MI355X.
 *
 * The library computes heads of the groundwater equation
 *     S dphi/dt - div(kappa grad phi) = q delta(x - x_s),  phi(0) = 0
 * (eqn:timedomain, Section 2.1) at receiver points and measurement times by
 * the inverse Laplace transform on the optimised Talbot contour (eq:talbot,
 * eqn:quadrature, eqn:half, Section 2.2).  Each time needs the shifted
 * systems (K + z_k M) x_k = b for N_z/2 contour nodes z_k (eqn:multipleshifted,
 * Section 3); one flexible Arnoldi basis per right-hand side serves all of
 * them (eqn:shiftedarnoldimod, Algorithm "Flexible FOM/GMRES for shifted
 * systems").  The preconditioner (K + tau_j M)^{-1} is applied by a
 * geometric-multigrid V-cycle refined to a relaxed tolerance.
 *
 * Discretisation: cell-centred finite volumes on a regular grid, face
 * transmissibility = harmonic mean of kappa, zero-Dirichlet walls with the
 * boundary value at h/2, lumped storage m_i = S_i V_i.  Cells are numbered
 * with x fastest: (ix, iy, iz) -> ix + nx (iy + ny iz).
 *
 * Conventions for every entry point
 *   - "device" pointers are HIP device memory on the handle's device; "host"
 *     pointers are ordinary host memory.  All arrays are owned by the caller
 *     and only read or written during the call.
 *   - Complex device vectors are stored as two real planes per vector
 *     (all real parts, then all imaginary parts): [nvec][2][N].
 *   - All work is enqueued on the stream given to lt_setup; entry points that
 *     return results in host memory synchronise that stream before returning.
 *   - Return value: 0 = success, negative = error (nothing useful written),
 *     positive = warning (outputs hold the best estimate).  No exception or
 *     abort crosses this boundary.  lt_strerror() names every code.
 *   - A handle is used by one thread at a time.
 */
#ifndef LT_H
#define LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LT_OK = 0,
    LT_EINVAL = -1,       /* an argument is out of range or inconsistent      */
    LT_EHIP = -2,         /* a HIP runtime call failed                         */
    LT_ENOMEM = -3,       /* device or host allocation failed                  */
    LT_EUNSUPPORTED = -4, /* valid request this build does not implement       */
    LT_WNOTCONV = 1       /* maxit reached before every shift met the tolerance */
};

enum { LT_BC_DIRICHLET0 = 0, LT_BC_NEUMANN0 = 1, LT_BC_WATER_TABLE = 2 };
enum { LT_PREC_FP64 = 0, LT_PREC_MIXED = 1 };   /* V-cycle in FP64 or FP32   */
enum { LT_PROF_OFF = 0, LT_PROF_PRE_FINE = 1, LT_PROF_POST_FINE = 2, LT_PROF_SWEEP3D = 3, LT_PROF_EXACT = 4 };
enum { LT_PRECOND_GMG = 0, LT_PRECOND_UNET_GMG = 1, LT_PRECOND_EXACT = 2 };
enum { LT_METHOD_GMRES = 0, LT_METHOD_FOM = 1 };
enum { LT_CONV_WEIGHTED = 0, LT_CONV_RELATIVE = 1 };

typedef struct lt_handle lt_handle;

/* Regular grid: ndim in {2, 3}; n[a] cells and spacing h[a] per axis
 * (unused axes: n = 1, h = 1).  In 2D the depth is 1, so kappa is a
 * transmissivity and S a storativity. */
typedef struct {
    int ndim;
    int n[3];
    double h[3];
} lt_grid;

/* Boundary condition per wall, order -x, +x, -y, +y, -z, +z
 * (eqn:timedomain): LT_BC_DIRICHLET0 holds the head at zero,
 * LT_BC_NEUMANN0 carries no flux, LT_BC_WATER_TABLE is the linearised water
 * table, whose outward flux is -sy times the rate of change of the head.  A
 * water-table face carries no conductive flux; its storage sy * (face area)
 * joins the lumped mass of the cell behind it (the boundary term of M in
 * Section 2.1), so M = diag(S V) + that term.  sy is the specific yield of
 * every water-table face (finite, >= 0; ignored when no face has that type).
 * A water-table face must lie on one of the grid's ndim axes.  The storage
 * sensitivity (lt_adjoint) differentiates S V only: sy is not a parameter. */
typedef struct {
    int face[6];
    double sy;
} lt_bc;

/* n points (wells); host array xyz[3 n] of coordinates in the domain
 * [0, n_a h_a].  Each point is spread on the surrounding cell centres with
 * bilinear (trilinear) weights; a point within h/2 of a wall uses the
 * nearest cell along that axis.  Sources and receivers use the same rule,
 * so B_r (K + zM)^{-1} B_s^T is symmetric (reciprocity, Section 5.2). */
typedef struct {
    int n;
    const double* xyz;
} lt_points;

/* What drives a solve: the transformed semi-discrete system of Section 2.1,
 *     (K + z M) phi_hat(z) = sum_s qhat_s(z) b_s + M phi0,
 * with b_s the weights of well s (lt_points) and qhat_s(z) = q_s / z for a
 * constant rate q_s switched on at t = 0.  Heads are linear in the data, so
 * each well is solved as its own right-hand side q_s b_s and reported on its
 * own output row.
 *   pts   the pumping wells (pts.n >= 0).
 *   q     host [pts.n] pumping rate of each well (finite; 0 leaves the row
 *         zero); NULL: every rate 1.
 *   phi0  device float64 [N] initial head, or NULL for phi(0) = 0.  Its term
 *         M phi0 is one more right-hand side, weighed in the contour sum by
 *         w_k alone (factor 1, not qhat; the two-system split of Section 3),
 *         and its heads are added to every well's row.  With pts.n = 0 the
 *         output has one row holding the initial-value heads alone.
 * lt_adjoint takes wells only (phi0 must be NULL). */
typedef struct {
    lt_points pts;
    const double* q;
    const double* phi0;
} lt_sources;

/* Talbot contour with nz nodes on the full contour per time (nz even);
 * nz/2 shifted systems are solved per time (eqn:half). */
typedef struct {
    int nz;
} lt_contour;

/* Solver options.  Zero-initialise and set what you need; lt_opts_default()
 * fills the defaults.
 *   tol        weighted per-shift tolerance: shift k of time t is converged
 *              when |w_k qhat_k| ||r_k|| <= tol * max_{k' at t} |w_k' qhat_k'| ||b||
 *              (weights from eqn:half; residual bound of Proposition 1), i.e.
 *              omega_k ||r_k|| / ||b|| <= tol with omega_k the ratio of the
 *              two weights.  phi0's right-hand side weighs by |w_k| alone.
 *   maxit      maximum outer (Arnoldi) iterations per right-hand side.
 *   precision  LT_PREC_FP64 or LT_PREC_MIXED (V-cycle in FP32; Arnoldi,
 *              least squares, residuals and the contour sum stay FP64).
 *   n_tau      number of preconditioner shifts chosen from the contour nodes
 *              (1: the node of smallest non-negative real part; 2: that node
 *              three times, then the node of largest real part twice, repeated
 *              (the rule of Section 3); 3: smallest, median-|z| and largest
 *              real part in turn).  With LT_PRECOND_EXACT the candidates are
 *              all nodes, so the smallest real part may be negative, as in the
 *              paper's schedule (n_tau 1 is then its 'Single' solver, 2 its
 *              'Flexible' one, Section 4.1).  Ignored when tau_reim is given.
 *   tau_reim   optional host array [2 n_tau] of explicit shifts (re, im),
 *              used cyclically.
 *   nu1, nu2   red-black Gauss-Seidel sweeps before / after coarse correction.
 *   inner_max  maximum V-cycles per outer iteration (iterative refinement).
 *   relax      inner tolerance factor: the refinement stops when
 *              ||v - (K + tau M) u|| <= relax * tol / (worst weighted residual).
 *   true_residual  1 (default): compute the FP64 true residual of every
 *              (rhs, shift) at exit, report it in lt_stats, and let it decide
 *              the status and the re-solves described at lt_solve.  0: skip
 *              it; the status then rests on the least-squares residuals.
 *   profile    0: off.  LT_PROF_PRE_FINE / LT_PROF_POST_FINE: time every launch
 *              of the fine-grid pre- / post-smoothing kernel of a 2D grid with
 *              HIP events on the handle's stream and count its algorithmic
 *              bytes (reported in lt_stats.prof_*); LT_PROF_SWEEP3D: the same
 *              for every one-colour Gauss-Seidel half-sweep on the fine grid
 *              of a 3D grid; LT_PROF_EXACT: every dense block-product launch
 *              of the exact preconditioner's solves (LT_PRECOND_EXACT), whose
 *              algorithmic bytes are the dense blocks and vector blocks it
 *              must move.
 *   precond    LT_PRECOND_EXACT: each u_j = (K + tau_j M)^{-1} v_j is applied
 *              exactly (to rounding) by a factorisation of K + tau_j M made once
 *              per shift and kept on the handle (lt_shift_invert; the
 *              factorised shift-and-invert preconditioner of Section 3, so
 *              Algorithm 1 runs as printed, with no inner iteration).  FP64
 *              whatever `precision` says; nu1, nu2, inner_max, relax and graph
 *              are not used.  Limits are those of lt_shift_invert.
 *              LT_PRECOND_GMG: V-cycle refinement only.  LT_PRECOND_UNET_GMG:
 *              preconditioner solves start from the attached network's guess
 *              (lt_unet_attach, 2D grids whose nx is a multiple of 128 and ny of
 *              8).  The network is first tried on one right-hand side (a batch
 *              of one); once its guess passes the net_keep test it serves every
 *              right-hand side.  A guess that increases the residual is
 *              discarded, and the V-cycle refinement then proceeds as usual, so
 *              the V-cycle remains both the fallback and, through the true
 *              residual, the judge.
 *   net_keep   the network is switched off for the rest of the call after an
 *              outer iteration in which its guess left more than this fraction
 *              of some right-hand side's residual (default 0.05: it must do at
 *              least the work of about two V-cycles to pay for itself).
 *   graph      1: each refinement step (V-cycle, FP64 update, stopping
 *              test) is captured once as a HIP graph per shift, buffer set
 *              and size, and replayed; 0 (default): launched kernel by
 *              kernel.  Results are identical.  Needs a handle on a stream
 *              of its own (the legacy default stream cannot be captured;
 *              there, and when profiling, steps are launched directly).
 *   method     LT_METHOD_GMRES (default): per shift, y minimises the residual
 *              over the basis (FGMRES-Sh).  LT_METHOD_FOM: y solves the square
 *              Hessenberg system (FFOM-Sh), the other variant of the paper's
 *              flexible shifted algorithm (Section 3); its residual is the
 *              GMRES one divided by the cosine of the last Givens rotation.
 *   conv       LT_CONV_WEIGHTED (default): the weighted test under tol above.
 *              LT_CONV_RELATIVE: every shift until ||r_k|| <= tol ||b||, the
 *              plain relative residual test of the experiments in Section
 *              4.1 (stricter: shifts of small weight are solved as far as
 *              the others).
 *   tau_adapt  0 (default): preconditioner shifts from n_tau / tau_reim in
 *              turn.  1: after the first outer iteration each shift is
 *              chosen from the residual estimates (the a-posteriori
 *              estimate of Section 3, |w_k eta_k|: the least-squares residual
 *              of each shift, weighted as in the convergence test): the
 *              contour node with the largest weighted residual among those
 *              not yet converged, over all right-hand sides of the call,
 *              becomes the next shift (the V-cycle preconditioners take its
 *              projection onto Re tau >= 0, i Im z for a node left of the
 *              imaginary axis; LT_PRECOND_EXACT takes the nearest of the
 *              schedule's shifts, so nothing more is factorised).  The paper
 *              leaves the choice of shifts open (Sections 3 and 6); this is
 *              the build's own rule.  Costs one small device-to-host copy
 *              per outer iteration.
 *   restart    0 (default): one basis per solve, up to maxit columns.  m in 1..2000
 *              (lt_solve with LT_PRECOND_EXACT and LT_METHOD_FOM only, else
 *              LT_EINVAL; other calls return LT_EUNSUPPORTED): the basis
 *              restarts every m steps from the residuals, which FOM with an
 *              exact preconditioner makes collinear (Section 3.1: the residual
 *              of shift k after m steps is -eta_k v_{m+1}): the next cycle
 *              starts at v_{m+1}, and shift k's small problem takes -eta_k as
 *              its first right-hand-side entry.  maxit bounds the steps over
 *              all cycles (rounded up to whole cycles); the heads of the cycles
 *              are summed, and the true residual is that of each right-hand
 *              side's last cycle.  Extra device memory per right-hand side: one
 *              vector and one complex per shift. */
typedef struct {
    double tol;
    int maxit;
    int precision;
    int n_tau;
    const double* tau_reim;
    int nu1, nu2;
    int inner_max;
    double relax;
    int true_residual;
    int profile;
    int precond;
    double net_keep;
    int graph;
    int method;
    int conv;
    int tau_adapt;
    int restart;
} lt_opts;

/* Statistics of the last call.  Pointer members are optional host arrays the
 * caller provides (NULL to skip). */
typedef struct {
    int n_rhs;            /* right-hand sides solved                          */
    int n_shifts;         /* solved shifts per right-hand side                */
    int iters_max;        /* outer iterations of the slowest right-hand side  */
    int vcycles;          /* V-cycles applied, summed over right-hand sides   */
    int levels;           /* multigrid levels                                  */
    double true_relres_max;      /* max over (rhs, shift) of the weighted true residual
                                    omega_k ||b - (K + z_k M) x_k|| / ||b|| (compared with tol) */
    double seconds;              /* wall time of the call                    */
    int* iters_per_rhs;          /* [n_rhs] or NULL                          */
    double* true_relres;         /* [n_rhs][n_shifts] ||b - (K+zM)x|| / ||b|| or NULL
                                    (rows: the wells, then phi0's term if given) */
    int net_applied;             /* network guesses applied (rhs x outer iterations) */
    int net_rejected;            /* of which discarded by the residual guard      */
    int net_disabled_at;         /* outer iteration after which it was switched off (0: never) */
    int prof_launches;           /* profiled launches (opts.profile)          */
    double prof_ms;              /* their summed device time, milliseconds    */
    double prof_bytes;           /* their summed algorithmic bytes            */
    int resolves;                /* right-hand sides solved again because their
                                    weighted true residual missed tol          */
    int factorizations;          /* shifts factorised by this call (LT_PRECOND_EXACT;
                                    cached ones are reused, not counted)       */
    double factor_ms;            /* host wall time of those factorisations, ms */
} lt_stats;

void lt_opts_default(lt_opts* o);

/* Build the operator for conductivity kappa and storage S (device arrays of
 * grid cells, float64, x fastest; both strictly positive) and the multigrid
 * hierarchy.  hip_stream is a hipStream_t (NULL = the default stream); all
 * later work of the handle goes to it.  The handle copies what it needs, so
 * kappa and S may be freed after the call.  bc may be NULL (every wall zero
 * head).  LT_EINVAL for an unknown wall type, a water-table wall on an axis
 * beyond ndim, a specific yield that is negative or not finite, or fewer
 * than 2 or more than 2^28 cells (the fused smoothers address a vector with
 * 32-bit byte offsets); all checked before any device call.  Section 2.1 (semi-discrete system); the
 * finite-volume form is stated at the top of this file. */
int lt_setup(const lt_grid* grid, const double* kappa, const double* S, const lt_bc* bc,
             void* hip_stream, lt_handle** out);

/* The same handle for P1 finite elements (Section 2.1's weak form with
 * piecewise-linear basis functions) on a grid of cells: `cells` (ndim 2 or
 * 3, at least 3 cells per axis, n[2] = 1 in 2D, positive spacings).  2D: each
 * cell split by its anti-diagonal into two right triangles; 3D: each cell
 * split into the six path tetrahedra of the Kuhn subdivision (v000,
 * v000 + e_a, v000 + e_a + e_b, v111 for every order of the axes).  kappa
 * and S (device float64, per cell, x fastest) hold on all of a cell's
 * elements.  Every wall holds zero head; the unknowns are the interior
 * vertices, (n[0] - 1) x (n[1] - 1) [x (n[2] - 1)], x fastest.  The mass
 * matrix is lumped (M_ii = sum of S |e| / (d + 1) over the elements at
 * vertex i).  These elements couple no vertex pair off the axes, so K is a
 * five- or seven-point stencil on the vertices and every solver path
 * applies unchanged.  Wells and receivers
 * take the P1 basis functions at their position (barycentric coordinates in
 * their triangle).  lt_solve, lt_solve_batch, lt_shift_invert, lt_vcycle and
 * lt_precond_solve accept the handle, and so does lt_adjoint: its
 * sensitivities are then to ln kappa and ln S of every cell of `cells`.  Errors:
 * LT_EINVAL for a NULL argument or a bad grid, LT_EHIP for no device. */
int lt_setup_p1(const lt_grid* cells, const double* kappa, const double* S, void* hip_stream,
                lt_handle** out);

/* Heads phi[s][r][t] at receivers r and times t (host array times[ntimes],
 * strictly positive) for the wells and initial head of `src` (lt_sources):
 * the contour sum of eqn:half over the solutions of eqn:multipleshifted,
 * computed with the flexible shifted Krylov method of Section 3.
 * phi_out: device float64 [max(ns, 1)][nr][ntimes], ns = src->pts.n.
 * Status: the flexible Arnoldi stops when every shift meets opts.tol by its
 * least-squares residual; then (opts.true_residual = 1) the FP64 true
 * residual of every (rhs, shift) is computed, and a right-hand side whose
 * weighted true residual misses tol (relaxed preconditioner solves leave a
 * gap between the two) is solved again from the start with its tolerance,
 * and with it the inner tolerance, tightened by its own measured excess
 * (rounded to a power of two, so a right-hand side's result does not
 * depend on the others in the call) and four times the V-cycles per
 * preconditioner solve, at most twice (lt_stats.resolves).  LT_WNOTCONV if some shift still misses tol, by
 * either residual, after that (phi_out then holds the best estimate).
 * LT_EINVAL, before any work, for more than 1000 right-hand sides, a
 * non-finite rate, or neither wells nor phi0. */
int lt_solve(lt_handle* h, const lt_sources* src, const double* times, int ntimes,
             const lt_contour* contour, const lt_points* receivers, const lt_opts* opts,
             double* phi_out, lt_stats* stats);

/* Sensitivities of phi[s][r][t] to ln kappa and ln S of every cell
 * (Section 5.2, adjoint state through the Laplace transform), for the wells of
 * src (rates src->q as in lt_solve; src->phi0 must be NULL, else
 * LT_EUNSUPPORTED): forward fields for every well and adjoint fields for
 * every receiver (complex symmetric operator: no conjugation), contracted
 * cell by cell and summed over the contour.  dlnK, dlnS: device float64
 * [ns][nr][ntimes][N]; either may be NULL.  For a P1 handle (lt_setup_p1)
 * the last index runs over the cells of its cell grid instead, x fastest:
 * dK/dln kappa_c is kappa_c times the cell's element stiffness at kappa = 1,
 * dM/dln S_c its lumped element masses.  Every shift meets the stricter of
 * the heads' weighting |w_k qhat_k| and the storage term's |w_k qhat_k z_k|
 * in the convergence test.  Near steady state the storage sensitivity is a
 * vanishing sum of contour terms of its early-time size, so its error is set
 * by tol relative to that size, not to its own norm.  The status follows the
 * true residual as in lt_solve.  LT_EINVAL, before any work, for more than
 * 1000 wells and receivers together. */
int lt_adjoint(lt_handle* h, const lt_sources* src, const lt_points* receivers,
               const double* times, int ntimes, const lt_contour* contour, const lt_opts* opts,
               double* dlnK, double* dlnS, lt_stats* stats);

/* Block flexible GMRES for shifted systems (the block approach Section 6
 * proposes for many right-hand sides; Algorithm 1 of Section 3 with block
 * vectors): x_k = (K + z_k M)^{-1} b for every shift z_k and every column of
 * b, the columns taken in blocks of `block` consecutive right-hand sides that
 * share one basis.  Step j applies the preconditioner of tau_j =
 * taus[(j - 1) % ntau] to every column of the block's newest basis block
 * (LT_PRECOND_EXACT: the factorisation of K + tau_j M; LT_PRECOND_GMG:
 * V-cycles until each residual is below tol / 100, FP64 cycles, or with
 * opts.precision LT_PREC_MIXED FP32 cycles on an FP32 copy of the FP64
 * residual, corrections and residuals in FP64), orthogonalises M U_j
 * against the block basis by classical Gram-Schmidt, twice, and takes the QR
 * of the remainder by modified Gram-Schmidt; each (block, shift) then updates
 * its block least-squares problem by Givens rotations.  A shift of a block
 * stops when every column meets weights[k] ||r|| <= tol ||b||.
 *   shifts   host [nshift][2] (re, im), 1..1024; weights host [nshift] or NULL
 *   taus     host [ntau][2]; GMG needs Re(tau) >= 0
 *   b        device [nvec][2][N], every column nonzero; nvec <= 1000
 *   block    1..16, dividing nvec
 *   x        device [nshift][nvec][2][N] (written; must not overlap b)
 * opts: tol, maxit, precond (GMG or EXACT), precision (FP64 or MIXED), nu1,
 * nu2, inner_max (GMG: at most 8 inner_max V-cycles per step); other fields
 * are ignored.  The steps are
 * capped at 32768 / (16 block^2) - 1 (127 for blocks of 4, 31 for 8), where one
 * (block, shift)'s least-squares columns fill 32 KB of LDS.  Workspace on the
 * handle, with m the capped steps: about (2 m + 5) nvec 16 N bytes of vectors,
 * plus 16 (m block)^2 bytes of rotated least-squares columns per (block, shift).
 * The status follows the FP64 true residuals (stats.true_relres,
 * [nvec][nshift]): LT_WNOTCONV if a weighted one exceeds tol.
 * stats.iters_per_rhs gets each column's block's steps.  The columns of a
 * block must be linearly independent: a block of lower rank (a column
 * repeated, say) stops after its first step, and its true residuals report
 * it.  LT_EINVAL for bad sizes, non-finite shifts, a zero column, negative
 * weights, a negative Re(tau) with multigrid, or x overlapping b. */
int lt_shifted_solve_block(lt_handle* h, int nshift, const double* shifts, const double* weights, int ntau,
                           const double* taus, int nvec, int block, const double* b, const lt_opts* opts,
                           double* x, lt_stats* stats);

/* ---- batches of problems ----------------------------------------------
 * Every shift of every right-hand side of several problems, possibly on
 * grids of different shapes and dimensions, solved in one call: each item
 * is the argument list of one lt_solve (or lt_adjoint) on its own handle.
 * The shifted systems of all problems are independent (Section 3: one
 * basis per right-hand side serves its shifts; nothing couples right-hand
 * sides or problems), so the items run concurrently, one host thread per
 * item driving its handle's stream; the GPU interleaves the workgroups of
 * all streams.  Give every handle its own stream (lt_setup) for the items
 * to overlap; handles sharing a stream still give correct results, one
 * after another.  Every handle may appear once per call (handles are not
 * thread-safe), and a network attached to a handle whose item selects
 * LT_PRECOND_UNET_GMG may serve only that item.  Outputs and per-item
 * return codes (status) are the same as lt_solve's / lt_adjoint's for the
 * item alone: the kernels are deterministic, so results are bit-identical.
 * Returns the first negative status in item order if any item failed,
 * else LT_WNOTCONV if any item missed its tolerance, else LT_OK.
 * LT_EINVAL for n < 1, n > 64, a NULL items or handle, or the sharing
 * rules above (then no item runs). */
typedef struct {
    lt_handle* h;
    const lt_sources* src;
    const double* times;      /* host [ntimes] */
    int ntimes;
    const lt_contour* contour;
    const lt_points* receivers;
    const lt_opts* opts;      /* NULL: lt_opts_default */
    double* phi_out;          /* device float64 [max(ns, 1)][nr][ntimes] */
    lt_stats* stats;          /* or NULL */
    int status;               /* out: the item's return code */
} lt_solve_item;

typedef struct {
    lt_handle* h;
    const lt_sources* src;
    const lt_points* receivers;
    const double* times;      /* host [ntimes] */
    int ntimes;
    const lt_contour* contour;
    const lt_opts* opts;      /* NULL: lt_opts_default */
    double* dlnK;             /* device float64 [ns][nr][ntimes][N] or NULL */
    double* dlnS;             /* same shape or NULL (not both NULL) */
    lt_stats* stats;          /* or NULL */
    int status;               /* out */
} lt_adjoint_item;

int lt_solve_batch(lt_solve_item* items, int n);
int lt_adjoint_batch(lt_adjoint_item* items, int n);

/* Talbot nodes and weights for one time (host arrays of nz/2 complex values
 * as (re, im) pairs, nodes with Im z > 0 in increasing theta):
 * phi(t) ~ 2 Re sum_k w_k F(z_k).  eq:talbot, eqn:quadrature, eqn:half. */
int lt_talbot(int nz, double t, double* z_reim, double* w_reim);

/* y = (K + tau M) x on multigrid level `level` (0 = the fine grid) for nvec
 * complex device vectors [nvec][2][N_level], float64.  Test and diagnostic
 * entry point for the stencil (Section 2.1 operator). */
int lt_apply_operator(lt_handle* h, int level, double tau_re, double tau_im,
                      const double* x, double* y, int nvec);

/* x = one V-cycle for (K + tau M) x = b from x = 0 on the fine grid, nvec
 * complex device vectors [nvec][2][N] float64; precision as in lt_opts
 * (FP32 cycles convert on entry and exit).  Test entry point for the
 * preconditioner of Section 3 (here a multigrid approximation of the
 * shift-and-invert solve). */
int lt_vcycle(lt_handle* h, double tau_re, double tau_im, int precision, int nu1, int nu2,
              const double* b, double* x, int nvec);

/* lt_vcycle that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, layout and result as lt_vcycle; every
 * work vector of the cycle (level right-hand sides and iterates, the FP32
 * copies of b and x) and the dense inverse of the coarsest level (built on the
 * GPU for this shift) live in the library's static scratch array of 64 MiB per
 * device, whose address lt_setup takes once per device.  The call calls no
 * device allocator.  LT_EINVAL, before any work, when the cycle needs more than
 * 64 MiB (about 2D 256 x 256 with 8 right-hand sides in FP64; lt_last_error
 * names the size).  Every call on a GPU shares that GPU's scratch, so calls
 * that overlap on one GPU (other streams or host threads) race; the scratch
 * keeps the last call's contents, and nothing in it needs to start at zero.
 * The FP64 result agrees with lt_vcycle's to rounding (the coarse inverse is
 * formed on the GPU instead of the host); a singular coarse operator gives
 * NaN.  Works on handles from lt_setup only. */
int lt_vcycle_noalloc(lt_handle* h, double tau_re, double tau_im, int precision, int nu1, int nu2,
                      const double* b, double* x, int nvec);

/* ---- learned preconditioner -------------------------------------------
 * A 2D convolutional U-Net (4 levels, 16/32/64/64 channels, 3x3 kernels,
 * BF16 weights and activations, FP32 accumulation on the matrix cores) that
 * maps a residual r to an approximation of (K + tau M)^{-1} r on the grid of
 * a handle.  Its inputs per cell are r / rms(r), ln(D_i / mean D) and
 * tau m_i / D_i (D_i the diagonal of K); it predicts e D_i / rms(r).  It is
 * trained on the GPU with the library's own forward and backward kernels and
 * Adam; FP32 master weights live on the device.  Grids: 2D, nx a multiple of
 * 128, ny a multiple of 8.  Not part of the paper (which factorises
 * K + tau M); the flexible method of Section 3 admits any preconditioner. */
typedef struct lt_unet lt_unet;

/* New network with He-normal weights from `seed`; work goes to hip_stream. */
int lt_unet_create(unsigned long long seed, void* hip_stream, lt_unet** out);
/* Number of FP32 parameters. */
long long lt_unet_nparams(const lt_unet* u);
/* Copy the parameters to / from a host array of lt_unet_nparams floats. */
int lt_unet_get_params(lt_unet* u, float* host);
int lt_unet_set_params(lt_unet* u, const float* host);
/* e = network(r) for nvec complex device vectors [nvec][2][N] (float64) on the
 * grid of h with preconditioner shift tau. */
int lt_unet_apply(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r, double* e);
/* One training step on the pairs (r, e = (K + tau M)^{-1} r): loss = mean
 * over vectors of the relative error left after the best complex multiple
 * of the output, 1 - |<out, t>|^2 / (||out||^2 ||t||^2), t = e D / rms(r)
 * (the solver applies the output with the residual-minimising multiple, so
 * only its direction matters); Adam with learning rate lr (lr = 0: no update).
 * loss: host float (mean loss before the update) or NULL. */
int lt_unet_train_step(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r,
                       const double* e, float lr, float* loss);
/* Gradient of that loss with respect to the parameters (host array of
 * lt_unet_nparams floats); test entry point. */
int lt_unet_grad(lt_unet* u, lt_handle* h, double tau_re, double tau_im, int nvec, const double* r, const double* e,
                 float* grad_host);
/* Use u in lt_solve / lt_adjoint of h when opts.precond = LT_PRECOND_UNET_GMG
 * (NULL detaches).  The handle does not own the network. */
int lt_unet_attach(lt_handle* h, lt_unet* u);
void lt_unet_destroy(lt_unet* u);

/* e = (K + tau M)^{-1} r to relative residual tol by FP64 V-cycle iteration
 * (at most maxcycles), nvec complex device vectors [nvec][2][N]: accurate
 * preconditioner solves, used as training targets.  Returns LT_WNOTCONV if
 * tol is not reached. */
int lt_precond_solve(lt_handle* h, double tau_re, double tau_im, int nvec, const double* r, double* e, double tol,
                     int maxcycles);

/* ---- geostatistical inversion (Section 5.1, Algorithm 2) ---------------
 * Unknowns s = ln kappa per cell with the prior s ~ N(X beta, Q): X a column
 * of ones (one unknown constant mean) and Q the exponential covariance
 * Q(x, x') = cov_var exp(-|(x - x') / cov_len|) (per-axis lengths, the first
 * ndim used) over the cell centres.  Measurements y = h(s) + eps with
 * eps ~ N(0, r I): the heads of the wells src (rates q as in lt_sources) at
 * the observation wells obs and the times, ordered (well, receiver, time),
 * M = src.n obs.n ntimes of them (at most 4096).  opts (NULL: defaults) are
 * those of the forward (lt_solve) and adjoint (lt_adjoint) solves. */
typedef struct {
    lt_points src;
    const double* q;
    lt_points obs;
    const double* times;
    int ntimes;
    lt_contour contour;
    double cov_var;
    double cov_len[3];
    double r;
    const lt_opts* opts;
} lt_geostat;

/* out = Q v for nvec device vectors v, out [nvec][N] (float64; out must not
 * overlap v): the prior covariance product of Algorithm 2 (the paper forms
 * Q J^T by FFT or hierarchical matrices; here each tile of Q is evaluated
 * in LDS and never stored).  LT_EINVAL for nvec < 1 or a variance or length
 * that is not positive and finite. */
int lt_cov_apply(lt_handle* h, double var, const double* len, int nvec, const double* v, double* out);

/* One Gauss-Newton step of Algorithm 2 at s (device [N], the ln kappa the
 * handle was set up with: the caller keeps the two consistent): h(s) and
 * J = dh/ds (lt_solve, lt_adjoint), Q J^T, and the saddle-point system of
 * eq:inversion1 for xi and beta; s_next (device [N]) = X beta + Q J^T xi.
 * y: device [M]; hs (device [M] or NULL) receives h(s); *beta (or NULL) the
 * mean; stats (or NULL) those of the forward solve.  LT_WNOTCONV when a
 * forward or adjoint solve missed its tolerance (the step is still taken);
 * LT_EINVAL for bad arguments or a singular saddle-point system. */
int lt_geostat_step(lt_handle* h, const lt_geostat* g, const double* y, const double* s, double* s_next,
                    double* hs, double* beta, lt_stats* stats);

/* Algorithm 2 for iters Gauss-Newton steps from s0 (device [N]): each step
 * sets the operator up for kappa = exp(s_k) (lt_setup with grid, bc, S: S
 * device [N]) on hip_stream and calls lt_geostat_step.  s_out: device [N].
 * misfit (host [iters] or NULL): |y - h(s_k)|^2 / r at each step's start;
 * step (host [iters] or NULL): |s_{k+1} - s_k| / |s_{k+1}|. */
int lt_geostat_invert(const lt_grid* grid, const lt_bc* bc, const double* S, const lt_geostat* g,
                      const double* y, const double* s0, int iters, void* hip_stream, double* s_out,
                      double* misfit, double* step);

/* x = (K + tau M)^{-1} b exactly (to FP64 rounding) for nvec complex device
 * vectors b, x [nvec][2][N]: the factorised shift-and-invert preconditioner
 * of Section 3 (eqn for (K + z_k M)(K + tau M)^{-1}), the one LT_PRECOND_EXACT
 * applies.  The first call for a shift factorises K + tau M (block cyclic
 * reduction over the slices of the grid's last axis: rows of nx cells in 2D,
 * planes of nx ny cells in 3D; dense nb x nb complex blocks, about
 * 2 n nb^2 x 16 bytes of device memory for n slices of nb cells) and keeps
 * the factorisation on the handle (the last 4 shifts used); later calls with
 * the same shift only solve.  x must not overlap b.  No pivoting is done, so
 * the shift must be one for which none is needed: Im tau != 0 (the Hermitian
 * part of -i sign(Im tau) (K + tau M) is then definite), or real tau > 0, or
 * tau = 0 on a grid with a zero-head wall.  Errors: LT_EINVAL for nvec < 1
 * or > 1000, x overlapping b, any other shift, a slice of more than 1024
 * cells or more than 65535 slices, or a zero or non-finite pivot met on the way; LT_ENOMEM when the
 * factorisation does not fit.  Synchronises the handle's stream after a
 * factorisation, not after a solve. */
int lt_shift_invert(lt_handle* h, double tau_re, double tau_im, int nvec, const double* b, double* x);

/* ---- tile-shape autotuner ----------------------------------------------
 * The fused 2D smoothing kernels (fine and intermediate multigrid levels of
 * 2D grids) stage tiles of cells in LDS; the tile shape is chosen per level
 * and precision.  lt_autotune times preconditioner steps for nvec
 * right-hand sides on the handle's stream with every shape on one level at a
 * time (finest first, the others kept) and keeps the fastest: the choice is
 * stored in the handle and used by every later call.  tiles_out[n_out]
 * receives the shape id per level (-1 past the tuned levels);
 * *us_per_step the time of one step with the final choice (microseconds).
 * Returns the number of tuned levels (0 for 3D grids or nu outside 1..3,
 * which have no tile shapes), or a negative error code.  Results of later
 * solves do not depend on the shapes (each cell's arithmetic is the same;
 * only partial-sum order in residual norms differs).  A plain performance
 * knob, not part of the paper's method. */
int lt_autotune(lt_handle* h, int precision, int nu1, int nu2, int nvec, int* tiles_out, int n_out,
                double* us_per_step);
/* Set the tile shape ids per level (n <= 16; -1 or missing levels: shape 0),
 * e.g. from a cache of earlier lt_autotune results. */
int lt_set_tiles(lt_handle* h, int precision, const int* tiles, int n);
/* Interior cells (tx, ty) of tile shape `id`; LT_EINVAL for an unknown id. */
int lt_tile_shape(int id, int* tx, int* ty);

/* Diagnostic: the flexible Arnoldi relation that the last lt_solve or
 * lt_adjoint on h built for right-hand side `rhs` (eqn:shiftedarnoldimod;
 * Algorithm "Flexible FOM/GMRES for shifted systems"):
 *     M U_m = V_{m+1} Hbar_m,  V_{m+1}^H V_{m+1} = I,
 * u_j the preconditioned vectors, m the columns its shifts used (*m_out).
 * Host arrays, NULL to skip: V [mmax+1][2][N], U [mmax][2][N] (complex
 * planes), Hbar [mmax][mmax+1] complex (re, im) stored by column (column j
 * holds rows 0..m).  Only the first m (V: m+1) columns are written.  After a
 * breakdown (h_{m+1,m} = 0) the last column of V is zero.  LT_EINVAL if no
 * solve has run on h (or its basis was released by an error), rhs is out of
 * range, or mmax < m (then *m_out still receives m).  Synchronises the
 * handle's stream. */
int lt_krylov_basis(lt_handle* h, int rhs, int mmax, double* V, double* U, double* Hbar, int* m_out);

/* Number of cells per axis of multigrid level `level` (n_out[3]); returns
 * the number of levels, or a negative error code. */
int lt_level_shape(lt_handle* h, int level, int* n_out);

/* Name of a return code. */
const char* lt_strerror(int code);

/* Text describing the last error raised on the calling thread ("" if none). */
const char* lt_last_error(void);

/* Release the handle and everything it owns (NULL is accepted). */
void lt_destroy(lt_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* LT_H */
