/*
 * vp.h -- C ABI of the MI355X layer/volume potential library (libvp.so).
 *
 * Evaluates, at a set of targets, the 2-D Laplace potentials of the paper
 * "A lightweight, geometrically flexible fast algorithm for the evaluation of
 * layer and volume potentials" (Fryklund, Greengard, Jiang, Potter):
 *
 *   V[f](x)     = int_Omega G(x-y) f(y) dy                     (Sec. 1, eq. volpotposgreen)
 *   S[sigma](x) = int_dOmega G(x-y) sigma(y) ds_y              (Sec. 1, eq. slpot)
 *   D[mu](x)    = int_dOmega dG/dnu_y (x-y) mu(y) ds_y         (Sec. 1, eq. dlpot)
 *
 * with G(x) = -log|x| / (2 pi) and nu the outward normal.  Each potential is
 * split in time (Sec. 2) into a local part, evaluated per target from the
 * small-delta asymptotic expansions (Sec. 4), and a near/far history part,
 * evaluated on Fourier grids (Sec. 3: spread -> FFT -> diagonal multiply ->
 * inverse FFT -> interpolation).  All device work is hand-written HIP.
 *
 * Conventions common to every entry point
 *  - Array arguments are DEVICE pointers (hipMalloc / PyTorch CUDA tensors)
 *    unless a comment says "host".  Arrays are structure-of-arrays, float64
 *    (the geometry sign array is int8).  Jets are row-major [k][n]: row k of
 *    a jet array starts at element k*n.
 *  - The library copies what it keeps; it never retains a caller pointer
 *    after the call returns.  Outputs are written, not accumulated.
 *  - Every call returns a vp_status and never aborts.  On error nothing is
 *    written to outputs that the call did not already start writing, and
 *    vp_last_error() returns a message for the calling thread.
 *  - A plan is bound to the stream in its options; calls on one plan are not
 *    re-entrant (they share the plan's device workspace) and must be
 *    serialized by the caller.  Distinct plans may be used from different
 *    threads.  vp_eval/vp_volume/vp_layer only enqueue work on that stream:
 *    the output is ready once the stream is synchronized.  Without timing
 *    (vp_set_timing) an evaluation also runs the local part and the
 *    far-history level on a second stream the plan owns (default priority),
 *    forked from and joined back into the plan's stream by events inside the
 *    same call, so ordering against the plan's stream (and stream capture of
 *    it) is unchanged.  The output array is written on both streams between
 *    the fork and the join.
 */
#ifndef VP_H
#define VP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vp_plan_s* vp_plan_t;

typedef enum {
    VP_OK = 0,
    VP_ERR_ARG = 1,       /* invalid argument (NaN/inf, negative weight, bad sgn, n < 0, ...) */
    VP_ERR_OOM = 2,       /* device or host allocation failed                                  */
    VP_ERR_DEVICE = 3,    /* a HIP runtime call or kernel launch failed                        */
    VP_ERR_GEOMETRY = 4,  /* inputs violate the method's geometric assumptions                 */
    VP_ERR_TOL = 5,       /* tolerance cannot be met with the supported grid sizes             */
    VP_ERR_BUSY = 6,      /* resource in use (server capacity)                                 */
    VP_ERR_INTERNAL = 7
} vp_status;

typedef enum {
    VP_FP32 = 0,  /* spread / FFT / interpolation in float32 with float32 accumulation;
                     multiplier table built in float64, the zero-frequency (DC) term, the
                     local part and the final sum in float64                             */
    VP_FP64 = 1   /* everything in float64                                               */
} vp_precision;

enum { VP_KIND_V = 1, VP_KIND_S = 2, VP_KIND_D = 4 };

typedef struct {
    double tol;          /* target relative l_inf error of each result (default 1e-10)     */
    int precision;       /* vp_precision (default VP_FP64)                                  */
    double c_delta;      /* delta_1 = c_delta * dx^2, dx^2 = sum(w)/N (Sec. 6; default 3)  */
    double delta_ratio;  /* delta_2 / delta_1 (Sec. 2.2 uses 32; default 32)               */
    int order_v;         /* highest power of sqrt(delta) kept in V_L (default 4: delta^2)   */
    int order_s;         /* ... in S_L (default 3: delta^{3/2})                             */
    int order_d;         /* ... in D_L (default 3)                                          */
    int kinds;           /* VP_KIND_* bitmask this plan must support (default V|S|D)        */
    int fine_grid[2];    /* force fine-grid sizes F_NH, F_FH (0 = planner's choice)         */
    int spread_width[2]; /* force spreading widths w_NH, w_FH in grid cells (0 = planner)   */
    int tile;            /* spreading tile edge in grid cells (0 = planner); 16 spreads on
                            matrix cores (one 32x32 window of each tile in the MFMA
                            accumulators, either precision), 32 through LDS windows.  The
                            interpolation bins targets on the same edge, or with autotune on
                            whichever of 16 and 32 times faster                            */
    void* stream;        /* hipStream_t the plan's work is enqueued on (NULL = null stream) */
    int no_workspace;    /* 1: keep only the plan's resident data (sorted nodes, tables, geometry);
                            every evaluation then takes a stream-ordered workspace (grids,
                            spectra, strengths) -- the form the serving loop uses (default 0) */
    int autotune;        /* 1: choose each level's fine grid, spreading width and tile edge by
                            timing that level's kernels (spread, FFTs, interpolation) on the
                            device for every candidate that meets the tolerance, instead of the
                            static cost model; plan creation then runs kernels on the stream
                            and takes longer (default 0).  Forced fine_grid / spread_width /
                            tile values restrict the candidates.                              */
} vp_opts;

/* Fill opts with the defaults listed above. opts: host pointer. */
void vp_opts_default(vp_opts* opts);

/* Per-target local frame (Sec. 4): b = closest boundary point, r = |x - b|,
 * (nx, ny) = outward unit normal at b, x = b - sgn*r*nu_b, sgn = +1 inside,
 * 0 on the boundary, -1 outside; kappa = curvature at b (gamma''(0) in the
 * tangent-line frame whose second axis is the inward normal: > 0 on convex
 * arcs); gamma3, gamma4 = third and fourth derivatives of that local graph
 * (may be NULL: taken as 0; needed only by delta^{3/2} and higher layer
 * terms).  All arrays have n_tgt entries.  The closest-point computation is
 * the caller's (the paper treats it as geometry preprocessing, Sec. 2.2). */
typedef struct {
    const double* r;
    const double* nx;
    const double* ny;
    const double* kappa;
    const double* gamma3;
    const double* gamma4;
    const int8_t* sgn;
} vp_local_geom;

/* Build a plan for fixed nodes (the inputs of the history algorithm, Sec. 3):
 *   n_src volume quadrature nodes (src_x, src_y) with weights src_w >= 0
 *     (zero weights -- degenerate triangles -- and coincident nodes are legal);
 *   n_bnd boundary nodes (bnd_x, bnd_y) with outward unit normals
 *     (bnd_nx, bnd_ny) and weights bnd_w >= 0 (may be 0 / NULL if no layer
 *     potential is requested);
 *   n_tgt targets (tgt_x, tgt_y) with their local frame geom.
 * delta_1 = c_delta * sum(src_w)/n_src (or c_delta * mean(bnd_w)^2 without
 * volume nodes), delta_2 = delta_ratio * delta_1.  The planner chooses the
 * Fourier periods, mode counts, fine grids, spreading widths and tiles for
 * opts->tol, sorts nodes and targets into tiles and builds the float64
 * multiplier tables; it copies node data to the host for this (synchronizes
 * the stream).  Targets within 12 sqrt(delta_1) of the boundary with sgn=-1
 * are rejected (VP_ERR_GEOMETRY) if kinds includes V: the volume local
 * expansion is stated for targets in the closed domain.
 * out: host pointer receiving the plan.  opts: host pointer (NULL = defaults). */
vp_status vp_plan(vp_plan_t* out,
                  int64_t n_src, const double* src_x, const double* src_y, const double* src_w,
                  int64_t n_bnd, const double* bnd_x, const double* bnd_y,
                  const double* bnd_nx, const double* bnd_ny, const double* bnd_w,
                  int64_t n_tgt, const double* tgt_x, const double* tgt_y,
                  const vp_local_geom* geom, const vp_opts* opts);

/* Evaluate V[f] + S[sigma] + D[mu] at the plan's targets (history part with
 * one shared inverse FFT and interpolation per level, plus local parts; Secs.
 * 3-4).  Any density may be NULL (omitted); its kind must be in the plan.
 *   f_src      [n_src]     density at the volume nodes (the weights are the plan's)
 *   jet6       [6][n_tgt]  f, f_x, f_y, f_xx, f_xy, f_yy at each target (global axes);
 *                          required with f_src
 *   sigma      [n_bnd]     single-layer density at the boundary nodes
 *   sigma_jet3 [3][n_tgt]  sigma, sigma', sigma'' at each target's b, derivatives in
 *                          the tangent-line parametrization (Sec. 4); required with sigma
 *   mu         [n_bnd]     double-layer density at the boundary nodes
 *   mu_jet5    [5][n_tgt]  mu, mu', mu'', mu''', mu'''' at b (same parametrization);
 *                          required with mu
 *   out        [n_tgt]     float64 result (sum of the requested potentials)
 * (The jets and out are per target: with n_tgt = 0 they may be NULL.)
 * Enqueues on the plan's stream and returns. */
vp_status vp_eval(vp_plan_t plan, const double* f_src, const double* jet6,
                  const double* sigma, const double* sigma_jet3,
                  const double* mu, const double* mu_jet5, double* out);

/* V[f] only: vp_eval(plan, f_src, jet6, NULL, NULL, NULL, NULL, out). */
vp_status vp_volume(vp_plan_t plan, const double* f_src, const double* jet6, double* out);

/* S[sigma] + D[mu] (either may be NULL): vp_eval without the volume density. */
vp_status vp_layer(vp_plan_t plan, const double* sigma, const double* sigma_jet3,
                   const double* mu, const double* mu_jet5, double* out);

/* Dyadic refinement of the local layer parts (Sec. 4, subsection on computing
 * the local part with arbitrary precision).  S_L and D_L are accurate to the
 * truncation order of their small-time expansions in delta_1.  With J levels
 * the expansions are taken at delta* = delta_1 / 4^J, and the time slices
 * [delta_1/4^j, delta_1/4^(j-1)], j = 1..J, are added by direct quadrature
 * over an oversampled boundary (the slice kernels narrow by a factor two per
 * level, so the boundary must resolve the last one: e.g. every panel split
 * into 2^J).  The slices telescope into one kernel per boundary node, which
 * is what the device evaluates:
 *   S: (E1(rho^2 / 4 delta_1) - E1(rho^2 / 4 delta*)) / (4 pi),
 *   D: nu_y.(x - y) (exp(-rho^2 / 4 delta_1) - exp(-rho^2 / 4 delta*)) / (2 pi rho^2),
 * rho = |x - y|, summed over the nodes within 12 sqrt(delta_1) of the target.
 *
 * vp_refine_attach: attach J (1..8) and the oversampled boundary: n_fine nodes
 * (fine_x, fine_y) with outward unit normals (fine_nx, fine_ny) and quadrature
 * weights fine_w >= 0, plus the plan's targets again (tgt_x, tgt_y; n_tgt
 * entries) -- all device float64 arrays, copied.  Bins the nodes and lists the
 * targets within 12 sqrt(delta_1) of the boundary (synchronizes the plan's
 * stream).  Replaces an earlier attachment.  VP_ERR_ARG for NULL or
 * non-finite input, negative weights or J out of range.
 *
 * vp_layer_refine: ADD the refinement to out[n_tgt] (after vp_eval or
 * vp_layer has written it):
 *   S_L(delta*) - S_L(delta_1) + slices of S   (sigma_jet3 as in vp_eval; fine_sigma
 *                                               = sigma at the attached nodes)
 *   D_L(delta*) - D_L(delta_1) + slices of D   (mu_jet5, fine_mu likewise)
 * A pair may be NULL (kind omitted); its kind must be in the plan.  Computed
 * in float64 for either plan precision.  Enqueues on the plan's stream.
 * VP_ERR_ARG without an attachment. */
vp_status vp_refine_attach(vp_plan_t plan, int levels, int64_t n_fine, const double* fine_x,
                           const double* fine_y, const double* fine_nx, const double* fine_ny,
                           const double* fine_w, const double* tgt_x, const double* tgt_y);
vp_status vp_layer_refine(vp_plan_t plan, const double* sigma_jet3, const double* fine_sigma,
                          const double* mu_jet5, const double* fine_mu, double* out);

/* ------------------------------------------------------------------------
 * Local frame and layer-density jets from a boundary given as panels.  The
 * local expansions of Sec. 4 need, per target, its closest boundary point b,
 * the distance r, the side, the outward normal and the curve's derivatives as
 * a graph over its tangent line at b (kappa, gamma3, gamma4: the second to
 * fourth derivatives), and the layer densities' derivatives along that line;
 * the paper leaves them to a geometry preprocessing step.  These two calls
 * compute them from the boundary nodes alone, for vp_plan's vp_local_geom and
 * vp_eval's jets.
 *
 * Boundary: n_pan >= 2 panels in order along the curve, counter-clockwise
 * (interior on the left), each with q nodes (5 <= q <= 32) at the
 * Gauss-Legendre points of its own parameter u in [-1, 1], ascending: node j
 * of panel p at bnd_x[p*q + j], bnd_y[p*q + j] (device, float64).  On a panel
 * each coordinate or density is its degree q-1 interpolant in u.
 *
 * vp_boundary_frame: per target (tgt_x, tgt_y: device, n_tgt), the closest
 * point b on the interpolated curve -- nearest node, then Newton on its panel,
 * continuing on the neighbouring panel when u leaves [-1, 1] (the closest point
 * for targets within the curve's local radius of curvature, a stationary
 * point of the distance at least as far otherwise) -- and at b:
 *   r, nx/ny (outward normal), kappa, gamma3, gamma4 (may be NULL), sgn (+1
 *   inside, -1 outside, 0 when r <= 1e-12 |x'(u)|, i.e. on the curve), and
 *   pan[i], u[i]: the panel and parameter of b, for vp_boundary_jets.
 * All outputs are device arrays of n_tgt.  Fourth derivatives of the
 * interpolant carry the nodal coordinates' rounding amplified near panel ends
 * (about 1e-5 relative in gamma4 on strongly curved boundaries).
 *
 * vp_boundary_jets: d^k s / d xi^k (k = 0..nder, nder <= 4) at each target's
 * b of a density s given at the nodes (dens, device, n_pan*q), xi along the
 * counter-clockwise tangent at b: out[k*n_tgt + i] -- the sigma_jet3 (nder =
 * 2) and mu_jet5 (nder = 4) layouts of vp_eval.  pan, u from
 * vp_boundary_frame (a pan outside [0, n_pan) gives NaN jets).
 *
 * Both enqueue on stream (a hipStream_t; NULL: the null stream), allocate
 * stream-ordered scratch of 3 n_pan q doubles, and return VP_ERR_ARG for q or
 * n_pan out of range and NULL arrays (n_tgt = 0 is a no-op). */
vp_status vp_boundary_frame(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y, int64_t n_tgt,
                            const double* tgt_x, const double* tgt_y, double* r, double* nx, double* ny,
                            double* kappa, double* gamma3, double* gamma4, int8_t* sgn, int32_t* pan, double* u,
                            void* stream);
vp_status vp_boundary_jets(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y, const double* dens,
                           int64_t n_tgt, const int32_t* pan, const double* u, int nder, double* out, void* stream);

/* vp_boundary_jets for callers that cannot allocate device memory: code
 * under HIP stream capture, tight serving or solver loops, hosts that forbid
 * hipMalloc.  Same arguments, kernels and results as vp_boundary_jets, but the
 * panel coefficients go to a fixed scratch array compiled into the library
 * (3 * VP_NOALLOC_MAX_NODES doubles, 1.5 MiB on every device the call runs
 * on, held until the process ends) instead of stream-ordered scratch; it calls
 * no hipMalloc/hipFree.  n_pan * q must not exceed VP_NOALLOC_MAX_NODES
 * (VP_ERR_ARG otherwise).  Every call on one device shares that device's
 * scratch: calls that overlap on the device (different streams or threads
 * without ordering between them) race and must be serialized by the caller;
 * calls on one stream are ordered.  The first call on a device looks up the
 * scratch's device address with that device current. */
#define VP_NOALLOC_MAX_NODES 65536
vp_status vp_boundary_jets_noalloc(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                                   const double* dens, int64_t n_tgt, const int32_t* pan, const double* u, int nder,
                                   double* out, void* stream);

/* ------------------------------------------------------------------------
 * Volume-density jets from the triangulation (the derivatives of f the
 * volume local part of Sec. 4, Lemma 4.1, takes, for a density known only at
 * the nodes of Sec. 2.2's triangles).
 *
 * x, y, f [6 n_tri] (device): the nodes of triangle j at 6j .. 6j+5 and f
 * there.  jet6 [6][6 n_tri] (device, out): f, f_x, f_y, f_xx, f_xy, f_yy at
 * each node from the quadratic interpolant of f at its triangle's six nodes
 * (vp_eval's jet6 for targets that are the volume nodes, in their order; the
 * value row is f itself).  The gradient is O(h^2) and the Hessian O(h)
 * accurate, so the volume potential with these jets carries an O(h^4)-like
 * error of its own (2.5e-5 relative on a 12k-node disk, 8e-7 at 48k): callers
 * who know f's derivatives pass those instead.  A triangle whose nodes do
 * not determine a quadratic (collinear nodes, a conic through all six) gets
 * NaN derivatives.  Enqueues one launch on stream (a hipStream_t; NULL: the
 * null stream), allocates nothing; VP_ERR_ARG for NULL arrays or n_tri < 0
 * (n_tri = 0 is a no-op). */
vp_status vp_volume_jets(int64_t n_tri, const double* x, const double* y, const double* f, double* jet6,
                         void* stream);

/* vp_volume_jets_patch: the same jets from the least-squares quadratic over
 * each triangle's six nodes and the six nodes of each of its edge neighbours:
 * nbr [3 n_tri] (device, int32), the triangle across each edge, -1 for none
 * (entries outside [0, n_tri), and the triangle itself, count as none).  The
 * six nodes of a sliver lie close to a line and do not fix the derivatives
 * across it; its neighbours' nodes do.  On the split square mesh the slivers'
 * gradient and Hessian errors then converge like those of the well-shaped
 * triangles (O(h^2) and O(h)).  Without neighbours the fit is the
 * interpolant of vp_volume_jets.  A patch whose nodes fix no quadratic gets
 * NaN derivatives.  One launch on stream, allocates nothing; VP_ERR_ARG for
 * NULL arrays or n_tri < 0 (n_tri = 0 is a no-op). */
vp_status vp_volume_jets_patch(int64_t n_tri, const double* x, const double* y, const double* f, const int32_t* nbr,
                               double* jet6, void* stream);

/* ------------------------------------------------------------------------
 * Interior Dirichlet problem -Lap u = f inside, u = g on the boundary, by
 * the representation u = V[f] + D[mu] (Sec. 1; the boundary integral
 * correction of Sec. 5): mu at the boundary nodes solves
 * D_int[mu] = g - V[f], D_int the interior limit of the double layer at each
 * node (f absent: the Laplace equation, u = D[mu]).  Restarted GMRES(restart) with
 * classical Gram-Schmidt applied twice, whose product is this library's evaluation: mu's
 * jets at the nodes from its panel interpolant (vp_boundary_jets), then
 * vp_eval of the double layer.
 *
 * plan: kind D (and V with a source); its boundary nodes are the n_pan*q panel nodes (bnd_x, bnd_y,
 *   device, the layout of vp_boundary_frame) and its targets are those same
 *   nodes, each with r = 0, sgn = +1 (the interior limit) and its frame from
 *   vp_boundary_frame at the nodes; pan, u: that call's locations.
 * g [n_pan*q] (device): boundary values.  f_src [n_src] (device): f at the
 *   plan's volume nodes, jet6 [6][n_pan*q] (device): f and its derivatives at
 *   the boundary nodes (vp_eval's layout); both NULL for f = 0.  V[f] at the
 *   nodes is one vp_volume call on the plan; its delta_1 (from the volume
 *   nodes) then serves the double layer too, as in the method.
 *   mu [n_pan*q] (device): in, the
 *   initial guess; out, the solution (the last iterate on VP_ERR_TOL).
 * tol: relative residual ||b - A mu|| / ||b|| (b = g - V[f], A = D_int), computed
 *   from mu itself: the solve returns VP_OK only when that residual is <= tol
 *   (each restart cycle begins with it; the Arnoldi recurrence's estimate
 *   only ends a cycle).  max_iter >= 1 bounds every operator product, those
 *   residuals included; restart in [1, 200].  iters, resid (host, may be
 *   NULL): products taken, and the last relative residual (computed from mu
 *   on VP_OK, the recurrence's estimate when max_iter ran out inside a
 *   cycle).  The Arnoldi steps run on the device without a host copy per
 *   step: the host enqueues the next step before reading the previous one's
 *   convergence flag (from mapped host memory), so a cycle that converges
 *   takes one more product than it uses (counted in iters).
 * Resolution: at a node the double layer's local part carries, from its
 *   delta^{3/2} term on, mu'' and mu' from the panel interpolant, of size
 *   delta_1^{3/2} |kappa| / h^2 next to mu/2 for a density varying on the
 *   node spacing h.  A boundary resolved far finer than sqrt(delta_1) makes
 *   the operator strongly non-normal and GMRES stalls (measured on circles:
 *   condition number 1.2e4 at chi = 1.1, 1.6e8 at 4; 1.9e-7 attainable at
 *   chi = 100).  With order_d >= 3 the solve computes
 *   chi = delta_1^{3/2} max|kappa| / h^2 over the panels (h = panel length / q,
 *   from the plan's boundary weights and its targets' kappa) and returns
 *   VP_ERR_GEOMETRY above 4 (above 2 for the exterior Dirichlet and Neumann
 *   operator of the next block, which degrades earlier: 9.4e7 at chi = 2),
 *   where residuals of data with every frequency stall above 1e-10.  Remedies: coarser panels (about sqrt(N) boundary nodes for N
 *   volume nodes keeps chi small), a smaller delta_1, or order_d <= 2.
 * Runs on the plan's stream and synchronizes it before returning.  Scratch
 * of about (restart + 11) n + restart^2 doubles, 24 bytes of mapped host
 * memory and two events are allocated by the first solve on the plan and kept
 * with it (the scratch grown if a later solve needs more; all freed by
 * vp_destroy).  VP_ERR_ARG for a
 * plan without D, or whose nodes or targets are not the n_pan*q panel nodes,
 * for only one of f_src and jet6, or for a source on a plan without V or
 * volume nodes; VP_ERR_GEOMETRY past the resolution limit;
 * VP_ERR_TOL when max_iter products do not reach tol. */
vp_status vp_dirichlet_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                             const int32_t* pan, const double* u, const double* g, const double* f_src,
                             const double* jet6, double* mu, double tol, int max_iter, int restart, int* iters,
                             double* resid);

/* ------------------------------------------------------------------------
 * The exterior Dirichlet and the interior Neumann problems (Sec. 5).  Both
 * solve A x = b at the nodes with A x = x/2 + D[x] + (w . x), that is
 * D_int[x] + x + sum_j w_j x_j (w = bnd_w, the boundary quadrature weights),
 * by the GMRES of vp_dirichlet_solve, on the same kind of plan (its targets
 * the boundary nodes with r = 0, sgn = +1 and their frames; pan, u from
 * vp_boundary_frame at the nodes).  bnd_w [n_pan*q] (device).
 *
 * vp_exterior_dirichlet_solve: Laplace's equation outside the curve with
 *   u = g on it and u bounded: u = D[mu] + (integral of mu) outside (the
 *   double layer with the kernel's +1), whose exterior limit on the boundary
 *   is mu/2 + D[mu] + (integral of mu) = g.  For growth A log|x - x0| at
 *   infinity use vp_exterior_dirichlet_solve_growth below (or pass
 *   g - A log|x' - x0| here).  mu [n_pan*q]: initial guess in,
 *   solution out.  With a volume source outside (u = V[f] + D_E[mu] +
 *   A log), pass g - V[f]: V[f] at the nodes and at exterior
 *   targets comes from plans on the same nodes traversed clockwise (panel
 *   and node order reversed, normals flipped), whose frames from
 *   vp_boundary_frame put the outside on their interior side, where the
 *   volume local part applies.
 * vp_neumann_solve: -Lap u = f inside with du/dnu = g on the boundary, by
 *   Green's representation u = V[f] + S[g] - D[u]; on the boundary
 *   u/2 + D[u] = V[f] + S[g].  The added integral of u removes the constants
 *   that operator annihilates, so ub [n_pan*q] (initial guess in, boundary
 *   values out) has zero boundary integral (u is fixed up to a constant;
 *   the data are consistent when the integral of g is minus that of f).
 *   The plan needs S and D (and V with a source: f_src at its volume nodes,
 *   jet6 [6][n_pan*q] f's jets at the boundary nodes, or both NULL).  g's
 *   jets come from its panel interpolant.  The interior solution is then
 *   vp_eval with f, sigma = g and mu = -ub on a plan with interior targets.
 *
 * Both synchronize the plan's stream, use the plan's solve scratch as
 * vp_dirichlet_solve does, count products and accept residuals as vp_dirichlet_solve does, and
 * return VP_ERR_ARG / VP_ERR_GEOMETRY (resolution limit 2) / VP_ERR_TOL as
 * it does (and VP_ERR_ARG for a NULL bnd_w, or a Neumann plan without S). */
vp_status vp_exterior_dirichlet_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x,
                                      const double* bnd_y, const double* bnd_w, const int32_t* pan, const double* u,
                                      const double* g, double* mu, double tol, int max_iter, int restart,
                                      int* iters, double* resid);
/* Growth at infinity of exterior solutions (Sec. 5, exterior representation
 * u = V[f] + D_E[mu] + A log|x - x0|): the problem fixes A (A = 0: bounded
 * solutions), and x0 is any point inside the curve (another interior point
 * changes the growth term by a function harmonic outside and vanishing at
 * infinity, which mu absorbs, so u does not change).
 *
 * vp_exterior_dirichlet_solve_growth: vp_exterior_dirichlet_solve with the
 *   data g - A log|x' - x0| formed on the device at the nodes (bnd_x,
 *   bnd_y); g is the boundary value of the whole solution (with a volume
 *   source, pass g - V[f] as there).  Same arguments, scratch, iteration
 *   count, residual and errors, plus VP_ERR_ARG for non-finite A, x0, y0.
 * vp_add_log_growth: out[i] += A log|(x[i], y[i]) - (x0, y0)| for n points
 *   (device arrays; no point may equal x0), enqueued on stream (a
 *   hipStream_t, NULL = null stream): the representation's last term at
 *   exterior targets, after the evaluation of D_E[mu] (and V[f]).
 *   VP_ERR_ARG for n < 0, NULL arrays with n > 0 or non-finite A, x0, y0. */
vp_status vp_exterior_dirichlet_solve_growth(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x,
                                             const double* bnd_y, const double* bnd_w, const int32_t* pan,
                                             const double* u, const double* g, double A, double x0, double y0,
                                             double* mu, double tol, int max_iter, int restart, int* iters,
                                             double* resid);
vp_status vp_add_log_growth(int64_t n, const double* x, const double* y, double A, double x0, double y0, double* out,
                            void* stream);
vp_status vp_neumann_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                           const double* bnd_w, const int32_t* pan, const double* u, const double* g,
                           const double* f_src, const double* jet6, double* ub, double tol, int max_iter,
                           int restart, int* iters, double* resid);

/* Release the plan and its device memory (synchronizes its stream). NULL is a no-op. */
vp_status vp_destroy(vp_plan_t plan);

/* Message for the last failing call on this thread ("" if none). Host string, owned
 * by the library, valid until the next call on this thread. */
const char* vp_last_error(void);

/* Planned parameters, for reporting.  All fields host values. */
typedef struct {
    double delta1, delta2, eps_hist;
    double period[2];     /* Fourier period P_NH, P_FH (history grids are P-periodic)        */
    double kmax[2];       /* cutoff wavenumbers                                               */
    double trunc_L;       /* far-history kernel truncation radius (far-history lemma, Sec. 2)   */
    int modes[2];         /* 2*M+1 Fourier modes per dimension, NH and FH                     */
    int fine[2];          /* fine-grid sizes F_NH, F_FH                                       */
    int width[2];         /* spreading widths                                                 */
    int tile[2];          /* tile edge in grid cells, NH and FH                                */
    int spread_mma[2];    /* 1: the level spreads on matrix cores                              */
    int precision;
    int64_t n_src, n_bnd, n_tgt;
    int64_t spread_records[2];  /* spread records per level (one per node)                   */
    size_t device_bytes;  /* device memory held by the plan                                   */
    size_t workspace_bytes; /* device memory one evaluation writes (the plan's own workspace, or
                               the stream-ordered one of a plan created with no_workspace)     */
    int autotuned;        /* 1 if the levels were chosen by measurement (opts.autotune)      */
    int tune_candidates[2]; /* candidates timed per level (0 without autotune)               */
    double level_ms[2];   /* measured time of the chosen candidate's level kernels (ms)      */
    int spread_terms[2];  /* terms of the per-tap kernel polynomials used in spreading         */
    int interp_terms[2];  /* terms of the values-only polynomials used in interpolation        */
    double spread_fit_err[2]; /* sampled max |polynomial - kernel| of the spreading table      */
    double interp_fit_err[2]; /* the same for the interpolation table                          */
    int interp_tile[2];   /* tile edge the targets are binned on for interpolation (autotune may
                             choose it apart from the spreading tile)                          */
} vp_plan_info;

/* Fill info (host pointer) with the plan's parameters. */
vp_status vp_get_plan_info(vp_plan_t plan, vp_plan_info* info);

/* Per-launch device timing of the most recent vp_eval on this plan, measured
 * with HIP events on the plan's stream (milliseconds, host array of 13):
 * [0] strengths, [1] spread NH, [2] spread FH, [3] row FFT NH, [4] row FFT FH,
 * [5] column FFT+multiply+inverse NH, [6] same FH, [7] row inverse FFT NH,
 * [8] same FH, [9] interpolation NH, [10] interpolation FH, [11] local part and
 * final sum, [12] total.  Enabled by vp_set_timing(plan, 1): a timed
 * evaluation runs every launch alone, in this order, on the plan's stream (an
 * untimed one overlaps the two levels on two streams and takes less than
 * [12]).  Reading it synchronizes on the last event. */
vp_status vp_set_timing(vp_plan_t plan, int enable);
vp_status vp_get_timing(vp_plan_t plan, double* ms13);

/* ------------------------------------------------------------------------
 * Batched evaluation.  Plans of uneven size are executed together: one
 * persistent kernel per stage (spreading and interpolation: one per distinct
 * spreading width) walks a device table of (instance, level, unit) segments
 * -- units are tiles, rows, columns or node chunks -- so every stage of every
 * instance shares the whole GPU.  Not in the
 * paper (which evaluates one problem on one core); it serves workloads made of
 * many independent meshes and densities.
 */
typedef struct vp_batch_s* vp_batch_t;

/* Per-instance arguments of one batched call (device pointers, as in vp_eval). */
typedef struct {
    const double* f_src;
    const double* jet6;
    const double* sigma;
    const double* sigma_jet3;
    const double* mu;
    const double* mu_jet5;
    double* out;
} vp_eval_args;

/* Group n plans (host array of handles; the plans must outlive the batch) for
 * batched calls that always pass the densities in kinds (VP_KIND_* mask).
 * All plans must share the precision; fine grids and spreading widths may
 * differ (spreading and interpolation take one launch per distinct width).
 * stream: hipStream_t for the batch (must not be the null stream if graphs are
 * used).  Copies its tables to the device (synchronous). */
vp_status vp_batch_create(vp_batch_t* out, int n, const vp_plan_t* plans, int kinds, void* stream);

/* Evaluate every instance: args is a host array of n entries.  use_graph != 0
 * captures the stage sequence into a hipGraph on the first call and replays it
 * afterwards (the per-call pointer table is copied to the device before each
 * replay).  Enqueues on the batch stream and returns. */
vp_status vp_batch_eval(vp_batch_t batch, const vp_eval_args* args, int use_graph);

/* Stage times of the batched launch.  vp_batch_set_timing(batch, 1) makes
 * vp_batch_eval record HIP events on the batch stream around each stage kind
 * (and run without the graph); vp_batch_get_timing waits for the last timed
 * call and writes VP_BATCH_STAGES times in ms (host array of n >= that):
 * grid zeroing, strengths, spreading (every width), row pass, column
 * transforms of double-layer channels, column pass with the multiply,
 * inverse row pass, interpolation (every width), local part.  VP_ERR_ARG
 * without a timed call or for n too small. */
#define VP_BATCH_STAGES 9
vp_status vp_batch_set_timing(vp_batch_t batch, int enable);
vp_status vp_batch_get_timing(vp_batch_t batch, float* ms, int n);

/* Release the batch (synchronizes its stream); the plans are not destroyed. */
vp_status vp_batch_destroy(vp_batch_t batch);

/* Message for the last failing batch call on this thread. */
const char* vp_batch_last_error(void);

/* ------------------------------------------------------------------------
 * Serving loop (continuous batching).  A host worker thread keeps a FIFO of
 * submitted requests.  Whenever in-flight slots and HBM are free it admits the
 * queued requests that fit -- in FIFO order, one precision at a time, a
 * request that does not fit never blocking smaller ones behind it -- and runs
 * them as one group: one persistent kernel per stage for all of them (the
 * batched execution of vp_batch_*), on an idle one of n_streams streams.  At
 * most one group per stream is in flight: while every stream is busy,
 * arrivals wait on the host and join the next group, so groups grow with the
 * load; groups on different streams overlap on the device.  Plans stay resident; each
 * running request holds a workspace block (grids, spectra, strengths) of its
 * HBM footprint rounded up to a size class (at most 1/8 more); blocks are
 * cached and reused once the group that used them completes, and the blocks
 * held -- in use plus cached -- never exceed the budget.  A group completes as a whole.  With max_wait_us
 * > 0 the worker holds the oldest queued request up to that long (unless a
 * full group is already queued) so that more requests join its group: larger
 * groups at the cost of up to that much added latency.  Not in the paper; it
 * serves streams of independent evaluations.
 */
typedef struct vp_server_s* vp_server_t;

typedef struct {
    size_t hbm_budget_bytes;  /* cap on the workspace memory held (in use + cached)          */
    int max_in_flight;        /* cap on concurrently running requests                        */
    int n_streams;            /* streams, and groups in flight (1..16)                       */
    int max_wait_us;          /* admission delay to gather a group (0: admit at once; >= 0)  */
} vp_server_opts;

/* One request: a plan (resident; create it with opts.no_workspace = 1 so it holds no
 * workspace of its own) and the densities/output of vp_eval (device pointers, ready --
 * their producing stream synchronized -- when submitted; they must stay valid and the
 * output untouched until the request completes). */
typedef struct {
    vp_plan_t plan;
    const double* f_src;
    const double* jet6;
    const double* sigma;
    const double* sigma_jet3;
    const double* mu;
    const double* mu_jet5;
    double* out;
} vp_request;

typedef struct {
    uint64_t submitted, completed, rejected, failed, deferred;  /* deferred: requests that waited for room */
    size_t peak_bytes;        /* largest in-flight workspace total                             */
    int peak_in_flight;       /* largest number of concurrently running requests              */
    double p50_s, p99_s, max_s, mean_s;  /* latency: submission -> completion observed        */
    double span_s;            /* first submission -> last completion                           */
    double targets_per_s;     /* completed target points / span_s                              */
    uint64_t groups;          /* launched groups (requests admitted together run as one group) */
    double mean_group;        /* requests per group                                            */
    size_t peak_held_bytes;   /* largest workspace memory held (in use + cached), <= budget    */
    uint64_t device_allocs;   /* workspace blocks allocated (the rest were reused from cache)  */
} vp_server_stats;

/* Start a server on the current device (opts: host pointer). */
vp_status vp_server_create(vp_server_t* out, const vp_server_opts* opts);
/* Queue a request (host struct); returns at once with a ticket (host pointer). */
vp_status vp_server_submit(vp_server_t srv, const vp_request* req, uint64_t* ticket);
/* done = 1 once the request finished; then result is its status (VP_ERR_OOM if it
 * exceeds the whole budget) and latency_s its latency.  result/latency_s may be NULL. */
vp_status vp_server_poll(vp_server_t srv, uint64_t ticket, int* done, vp_status* result, double* latency_s);
/* Block until the request finished or timeout_s passed (VP_ERR_BUSY on timeout). */
vp_status vp_server_wait(vp_server_t srv, uint64_t ticket, double timeout_s, vp_status* result, double* latency_s);
/* Counters and latency percentiles over all completed requests (stats: host pointer). */
vp_status vp_server_get_stats(vp_server_t srv, vp_server_stats* stats);
/* Finish queued and running requests, then stop the worker and free the server. */
vp_status vp_server_destroy(vp_server_t srv);
/* Message for the last failing server call on this thread. */
const char* vp_server_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VP_H */
