// Interior Dirichlet problem -Lap u = f inside, u = g on the boundary, by the
// representation u = V[f] + D[mu] (Sec. 1; the boundary integral correction of
// Sec. 5): mu on the boundary nodes solves D_int[mu] = g - V[f], where D_int is
// the interior limit of the double layer at each node and V[f] is this
// library's volume potential at the nodes (f = 0: the Laplace equation,
// u = D[mu]).  Restarted GMRES (Givens rotations) whose product is this
// library's evaluation:
// the density's jets at the nodes from its panel interpolant
// (vp_boundary_jets), then vp_eval of the double layer at the plan's targets,
// which are the nodes themselves with r = 0 and sgn = +1.  Each Arnoldi step
// orthogonalizes by classical Gram-Schmidt applied twice, every sum taken in a
// fixed order (the result does not depend on timing).  The step stays on the
// device: one kernel writes the new Hessenberg column, applies the Givens
// rotations, updates the residual estimate and the next basis vector's scale,
// and sets a done flag; it also writes that state into mapped host memory.
// The host enqueues step k + 1 before it looks at step k's flag, so the device
// never waits for the host; a step enqueued after the flag was set is wasted
// (at most one per cycle, and counted among the products).  The host reads the
// Hessenberg matrix once per cycle, to update x.  A solve ends only on a
// residual b - A x computed from x itself (each cycle starts from it), never on
// the Arnoldi recurrence's estimate alone.
//
// Resolution guard.  At a node (r = 0) the double layer's local part of
// Lemma 4.3 carries, from its delta^{3/2} term on, derivatives of the density
// (kappa mu'' and gamma3 mu'), which the solve takes from the panel
// interpolant.  For a density varying on the node spacing h these terms are
// of size delta^{3/2} |kappa| / h^2 next to the jump mu/2: once the boundary is
// resolved much finer than sqrt(delta_1), the discrete operator becomes
// strongly non-normal (interpolant derivatives are nilpotent on each panel)
// and GMRES stalls above the tolerance.  Measured with the direct-sum
// operator on circles (16-node panels, right-hand sides with every
// frequency): the condition number grows from 13 at
// chi = delta^{3/2} max|kappa| / h^2 = 0.05 to 1.2e4 at 1.1, 2.3e5 at 1.7
// (where GMRES(50) no longer reaches 1e-12) and 1.6e8 at 4 (1e-8 reached,
// 1e-10 not); for x/2 + D[x] + (w . x) the growth starts earlier (1.6e5 at
// chi = 0.6, 9.4e7 at 2).  Smooth data converge well past the first of these
// points, so the solves refuse chi above 4 (interior Dirichlet) and 2
// (exterior Dirichlet and Neumann), where the condition number passes 1e8,
// when the plan keeps those terms (order_d >= 3), with h = panel length / q.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "vp_geom.hpp"
#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kSolveThreads = 256;
constexpr int kDotBlocks = 256;
constexpr int kMaxRestart = 200;
constexpr int kSmallThreads = 1024;       // one workgroup per basis vector at small n
constexpr int64_t kSmallN = 1 << 16;      // up to this many nodes the projections take one launch

__global__ __launch_bounds__(kSolveThreads) void k_dot(int64_t n, const double* __restrict__ a,
                                                       const double* __restrict__ b, double* __restrict__ part)
{
    __shared__ double red[kSolveThreads / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s = fma(a[i], b[i], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

// part[j][b] = block b's partial sum of V_j . w over its grid-stride share, for
// the k1 vectors V_j = V + j ldv (grid: kDotBlocks x k1)
__global__ __launch_bounds__(kSolveThreads) void k_proj_part(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                             const double* __restrict__ w, double* __restrict__ part)
{
    __shared__ double red[kSolveThreads / 64];
    const double* v = V + (int64_t)blockIdx.y * ldv;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s = fma(v[i], w[i], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += red[k];
        part[(int64_t)blockIdx.y * kDotBlocks + blockIdx.x] = t;
    }
}

// out[j] (+)= V_j . w for n <= kSmallN in one launch: workgroup j sums the whole
// vector in a fixed order (grid: k1 workgroups of kSmallThreads)
__global__ __launch_bounds__(kSmallThreads) void k_proj_small(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                              const double* __restrict__ w, double* __restrict__ out,
                                                              int accumulate)
{
    __shared__ double red[kSmallThreads / 64];
    const double* v = V + (int64_t)blockIdx.x * ldv;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kSmallThreads) s = fma(v[i], w[i], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kSmallThreads / 64; ++k) t += red[k];
        out[blockIdx.x] = accumulate ? out[blockIdx.x] + t : t;
    }
}

// h[j] (+)= sum over b of part[j][b], a fixed binary tree per j (grid: k1 blocks of kDotBlocks threads)
__global__ __launch_bounds__(kDotBlocks) void k_proj_sum(const double* __restrict__ part, double* __restrict__ h,
                                                         int accumulate)
{
    __shared__ double t[kDotBlocks];
    t[threadIdx.x] = part[(int64_t)blockIdx.x * kDotBlocks + threadIdx.x];
    __syncthreads();
    for (int o = kDotBlocks / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) t[threadIdx.x] += t[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[blockIdx.x] = accumulate ? h[blockIdx.x] + t[0] : t[0];
}

// w -= sum_j c[j] V_j, j < k1 (c on the device)
__global__ __launch_bounds__(kSolveThreads) void k_sub_proj(int64_t n, int k1, const double* __restrict__ V,
                                                            int64_t ldv, const double* __restrict__ c,
                                                            double* __restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int j = 0; j < k1; ++j) s = fma(-c[j], V[(int64_t)j * ldv + i], s);
    w[i] = s;
}

// y += x + c[0] (c on the device: the weighted integral of x)
__global__ __launch_bounds__(kSolveThreads) void k_plus(int64_t n, const double* __restrict__ x,
                                                        const double* __restrict__ c, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += x[i] + c[0];
}

// out = in + A log |(x, y) - (x0, y0)|: the growth term of the exterior representation
// (in == out allowed)
__global__ __launch_bounds__(kSolveThreads) void k_log_growth(int64_t n, const double* __restrict__ x,
                                                              const double* __restrict__ y, double A, double x0,
                                                              double y0, const double* in, double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] + A * log(hypot(x[i] - x0, y[i] - y0));
}

// y = a x + b y (b = 0: y is not read, so uninitialized memory may be the target)
__global__ __launch_bounds__(kSolveThreads) void k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                                                         double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// out[0] = d32 * max over panels of max_j |kappa_j| / (sum_j w_j / q)^2 (one workgroup)
__global__ __launch_bounds__(kSolveThreads) void k_resolution(int64_t n_pan, int q, const double* __restrict__ w,
                                                              const double* __restrict__ kappa, double d32,
                                                              double* __restrict__ out)
{
    __shared__ double red[kSolveThreads / 64];
    double m = 0.0;
    for (int64_t p = threadIdx.x; p < n_pan; p += blockDim.x) {
        double len = 0.0, km = 0.0;
        for (int j = 0; j < q; ++j) {
            len += w[p * q + j];
            km = kappa ? fmax(km, fabs(kappa[p * q + j])) : 0.0;
        }
        const double h = len / q;
        m = fmax(m, d32 * km / (h * h));   // a zero-length panel gives inf (or NaN with kappa 0)
        if (m != m) m = INFINITY;
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t = fmax(t, red[k]);
        out[0] = t;
    }
}

// State of one restart cycle's Arnoldi recurrence, on the device (and mirrored
// into mapped host memory by k_arnoldi).
struct ArnoldiState {
    int done;       // the estimate reached tol, or the step broke down (h[k+1][k] = 0)
    int k;          // Hessenberg columns in use
    double rel;     // |z[k]| / ||b||: the recurrence's residual estimate
    double inv_hn;  // 1 / h[k+1][k] of the last step (0 after a breakdown)
};

// Start a cycle: z = (beta, 0, ...), state cleared (one thread)
__global__ void k_cycle_init(int m, double beta, double bnorm, double* __restrict__ z, ArnoldiState* __restrict__ st,
                             ArnoldiState* __restrict__ mirror)
{
    if (threadIdx.x != 0) return;
    z[0] = beta;
    for (int i = 1; i <= m; ++i) z[i] = 0.0;
    const ArnoldiState s0{0, 0, beta / bnorm, 0.0};
    *st = s0;
    *mirror = s0;
    __threadfence_system();
}

// Arnoldi step k of a cycle (one thread; nothing once the cycle is done):
// column k of H from hd (projections h[0..k], then ||w||^2), the earlier
// rotations applied to it, a new rotation zeroing h[k+1][k], and z rotated.
__global__ void k_arnoldi(int k, int m, const double* __restrict__ hd, double* __restrict__ H,
                          double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ z, double tol,
                          double bnorm, ArnoldiState* __restrict__ st, ArnoldiState* __restrict__ mirror)
{
    if (threadIdx.x != 0 || st->done) return;
    const int k1 = k + 1;
    for (int i = 0; i <= k; ++i) H[(int64_t)i * m + k] = hd[i];
    const double hn = sqrt(fmax(hd[k1], 0.0));
    for (int i = 0; i < k; ++i) {  // earlier rotations on the new column
        const double a = H[(int64_t)i * m + k], c = H[(int64_t)(i + 1) * m + k];
        H[(int64_t)i * m + k] = cs[i] * a + sn[i] * c;
        H[(int64_t)(i + 1) * m + k] = -sn[i] * a + cs[i] * c;
    }
    const double a = H[(int64_t)k * m + k];
    const double rr = hypot(a, hn);
    cs[k] = rr > 0.0 ? a / rr : 1.0;
    sn[k] = rr > 0.0 ? hn / rr : 0.0;
    H[(int64_t)k * m + k] = rr;
    H[(int64_t)k1 * m + k] = 0.0;
    z[k1] = -sn[k] * z[k];
    z[k] = cs[k] * z[k];
    ArnoldiState s1;
    s1.k = k1;
    s1.rel = fabs(z[k1]) / bnorm;
    s1.inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
    s1.done = (s1.rel <= tol || hn == 0.0) ? 1 : 0;
    *st = s1;
    *mirror = s1;
    __threadfence_system();
}

// y = x * inv_hn (the next basis vector; zero after a breakdown)
__global__ __launch_bounds__(kSolveThreads) void k_scale_dev(int64_t n, const double* __restrict__ x,
                                                             const ArnoldiState* __restrict__ st,
                                                             double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] * st->inv_hn;
}

constexpr double kChiInterior = 4.0;   // resolution limits of the guard above
constexpr double kChiPlus = 2.0;

struct Solver {
    vp_plan_t plan;
    int64_t n_pan, n;
    int q;
    const double *bx, *by, *upar;
    const int32_t* pan;
    hipStream_t st;
    const double* bw = nullptr;  // boundary weights: the operator x/2 + D[x] + (w . x) when set
    double* jets = nullptr;  // [5][n]
    double* gws = nullptr;   // [3][n]: panel coefficients of x, y and the density (the jets' scratch)
    double* part = nullptr;  // [kMaxRestart + 2][kDotBlocks]
    double* hd = nullptr;    // [kMaxRestart + 2]: projections of the current step, then its norm squared
    double* tmp = nullptr;   // [kMaxRestart + 1]: the second Gram-Schmidt pass's projections; last: w . x
    std::vector<double> h_part = std::vector<double>(kDotBlocks);

    vp_status launched()
    {
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? VP_OK : set_error(VP_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(e));
    }
    // out[j] (+)= V_j . w for j < k1, on the device
    vp_status project(const double* V, int k1, const double* w, double* out, bool accumulate)
    {
        if (n <= kSmallN) {
            hipLaunchKernelGGL(k_proj_small, dim3((unsigned)k1), dim3(kSmallThreads), 0, st, n, V, n, w, out,
                               accumulate ? 1 : 0);
            return launched();
        }
        hipLaunchKernelGGL(k_proj_part, dim3(kDotBlocks, (unsigned)k1), dim3(kSolveThreads), 0, st, n, V, n, w, part);
        hipLaunchKernelGGL(k_proj_sum, dim3((unsigned)k1), dim3(kDotBlocks), 0, st, part, out, accumulate ? 1 : 0);
        return launched();
    }
    // w -= V c over k1 vectors
    vp_status subtract(const double* V, int k1, const double* c, double* w)
    {
        hipLaunchKernelGGL(k_sub_proj, dim3((unsigned)((n + kSolveThreads - 1) / kSolveThreads)), dim3(kSolveThreads),
                           0, st, n, k1, V, n, c, w);
        return launched();
    }
    // Arnoldi step on w against V_0..V_k: two classical Gram-Schmidt passes,
    // leaving hd[0..k] (the projections) and hd[k+1] = ||w||^2 on the device
    vp_status orthogonalize(const double* V, int k, double* w)
    {
        const int k1 = k + 1;
        vp_status s = project(V, k1, w, hd, false);
        if (s == VP_OK) s = subtract(V, k1, hd, w);
        if (s == VP_OK) s = project(V, k1, w, tmp, false);
        if (s == VP_OK) s = subtract(V, k1, tmp, w);
        if (s != VP_OK) return s;
        hipLaunchKernelGGL(k_axpby, dim3((unsigned)((k1 + kSolveThreads - 1) / kSolveThreads)), dim3(kSolveThreads), 0,
                           st, (int64_t)k1, 1.0, tmp, 1.0, hd);
        if ((s = launched()) != VP_OK) return s;
        return project(w, 1, w, hd + k1, false);
    }

    // y = D_int[x], or D_int[x] + x + (w . x) = x/2 + D[x] + (w . x) with weights
    vp_status matvec(const double* x, double* y)
    {
        vp_status s = boundary_jets_ws(n_pan, q, bx, by, x, n, pan, upar, 4, jets, st, gws);
        if (s == VP_OK) s = vp_eval(plan, nullptr, nullptr, nullptr, nullptr, x, jets, y);
        if (s != VP_OK || !bw) return s;
        if ((s = project(bw, 1, x, tmp + kMaxRestart, false)) != VP_OK) return s;
        hipLaunchKernelGGL(k_plus, dim3((unsigned)((n + kSolveThreads - 1) / kSolveThreads)), dim3(kSolveThreads), 0,
                           st, n, x, tmp + kMaxRestart, y);
        return launched();
    }
    vp_status dot(const double* a, const double* b, double* out)
    {
        hipLaunchKernelGGL(k_dot, dim3(kDotBlocks), dim3(kSolveThreads), 0, st, n, a, b, part);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_part.data(), part, kDotBlocks * sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return set_error(VP_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(e));
        double t = 0.0;
        for (double v : h_part) t += v;  // fixed order
        *out = t;
        return VP_OK;
    }
    // b = g - A log |x' - x0| at the nodes
    vp_status minus_growth(const double* g, double A, double x0, double y0, double* b)
    {
        hipLaunchKernelGGL(k_log_growth, dim3((unsigned)((n + kSolveThreads - 1) / kSolveThreads)),
                           dim3(kSolveThreads), 0, st, n, bx, by, -A, x0, y0, g, b);
        return launched();
    }
    vp_status axpby(double a, const double* x, double b, double* y)
    {
        hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + kSolveThreads - 1) / kSolveThreads)), dim3(kSolveThreads), 0,
                           st, n, a, x, b, y);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? VP_OK : set_error(VP_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(e));
    }
};

vp_status check_solve_args(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                           const int32_t* pan, const double* u, const double* g, const double* x, double tol,
                           int max_iter, int restart)
{
    if (!plan) return set_error(VP_ERR_ARG, "plan is NULL");
    if (!(plan->kinds & VP_KIND_D)) return set_error(VP_ERR_ARG, "the plan does not support the double layer");
    if (n_pan < 2 || q < 5 || q > 32 || plan->n_bnd != n_pan * q || plan->n_tgt != plan->n_bnd)
        return set_error(VP_ERR_ARG, "the plan's boundary nodes and targets must be the n_pan*q panel nodes");
    if (!bnd_x || !bnd_y || !pan || !u || !g || !x) return set_error(VP_ERR_ARG, "NULL array");
    if (!(tol > 0 && tol < 1) || max_iter < 1 || restart < 1 || restart > kMaxRestart)
        return set_error(VP_ERR_ARG, "tol in (0,1), max_iter >= 1, restart in [1, 200]");
    return VP_OK;
}

vp_status check_source(vp_plan_t plan, const double* f_src, const double* jet6)
{
    if ((f_src == nullptr) != (jet6 == nullptr)) return set_error(VP_ERR_ARG, "f_src and jet6 go together");
    if (f_src && (!(plan->kinds & VP_KIND_V) || plan->n_src == 0))
        return set_error(VP_ERR_ARG, "a volume source needs a plan with volume nodes and the volume kind");
    return VP_OK;
}

// Restarted GMRES for A x = b at the nodes, A = D_int or, with weights bw,
// x/2 + D[x] + (w . x); make_rhs(S, b) writes b on the plan's stream.  x holds
// the initial guess on entry.
template <class MakeRhs>
vp_status gmres_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                      const int32_t* pan, const double* u, const double* bw, MakeRhs&& make_rhs, double* x,
                      double tol, int max_iter, int restart, int* iters, double* resid)
{
    const int64_t n = plan->n_bnd;
    const int m = restart;
    Solver S{plan, n_pan, n, q, bnd_x, bnd_y, u, pan, plan->stream};
    S.bw = bw;
    // scratch in one block kept on the plan (allocated by the first solve, grown if needed):
    // basis, w, b, jets, jet scratch, partial sums, projections, second-pass projections,
    // Hessenberg matrix, rotations (cos, sin), z, cycle state
    constexpr int kParts = 13;
    const size_t parts[kParts] = {(size_t)(m + 1) * n, (size_t)n, (size_t)n, (size_t)5 * n, (size_t)3 * n,
                                  (size_t)(kMaxRestart + 2) * kDotBlocks, (size_t)(kMaxRestart + 2),
                                  (size_t)(kMaxRestart + 1), (size_t)(m + 1) * m, (size_t)m, (size_t)m,
                                  (size_t)(m + 1), (sizeof(ArnoldiState) + 7) / 8};
    size_t need = 0;
    for (size_t c : parts) need += (c * sizeof(double) + 255) & ~(size_t)255;
    hipError_t e = hipSuccess;
    if (plan->solve_ws_bytes < need) {
        if (plan->solve_ws) (void)hipFree(plan->solve_ws);
        plan->solve_ws = nullptr;
        plan->solve_ws_bytes = 0;
        e = hipMalloc(&plan->solve_ws, need);
        if (e == hipSuccess) plan->solve_ws_bytes = need;
    }
    if (e == hipSuccess && !plan->solve_host) {
        e = hipHostMalloc(&plan->solve_host, sizeof(ArnoldiState), hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer(&plan->solve_host_dev, plan->solve_host, 0);
    }
    if (e == hipSuccess && !plan->solve_ev_made) {
        e = hipEventCreateWithFlags(&plan->solve_ev[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->solve_ev[1], hipEventDisableTiming);
        if (e == hipSuccess) plan->solve_ev_made = true;
    }
    double* ptr[kParts] = {};
    if (e == hipSuccess) {
        unsigned char* q = (unsigned char*)plan->solve_ws;
        for (int k = 0; k < kParts; ++k) {
            ptr[k] = (double*)q;
            q += (parts[k] * sizeof(double) + 255) & ~(size_t)255;
        }
    }
    double* V = ptr[0];  // [m+1][n] Krylov basis
    double* w = ptr[1];  // [n]
    double* b = ptr[2];  // [n] right-hand side
    S.jets = ptr[3];
    S.gws = ptr[4];
    S.part = ptr[5];
    S.hd = ptr[6];
    S.tmp = ptr[7];
    double* Hd = ptr[8];   // [m+1][m] Hessenberg matrix of the cycle, rotated
    double* csd = ptr[9];
    double* snd = ptr[10];
    double* zd = ptr[11];  // [m+1] rotated right-hand side of the least-squares problem
    ArnoldiState* std_ = (ArnoldiState*)ptr[12];
    ArnoldiState* mirror_dev = (ArnoldiState*)plan->solve_host_dev;
    volatile ArnoldiState* mirror = (volatile ArnoldiState*)plan->solve_host;
    vp_status s = e == hipSuccess ? VP_OK : set_error(VP_ERR_OOM, "solve workspace");
    if (s == VP_OK && plan->loc.order_d >= 3) {   // the resolution guard (header)
        const double chi_max = bw ? kChiPlus : kChiInterior;
        double chi = 0.0;
        hipLaunchKernelGGL(k_resolution, dim3(1), dim3(kSolveThreads), 0, S.st, n_pan, q, plan->d_w + plan->n_src,
                           plan->g_kappa, std::pow(plan->delta1, 1.5), S.hd);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&chi, S.hd, sizeof(double), hipMemcpyDeviceToHost, S.st);
        if (e == hipSuccess) e = hipStreamSynchronize(S.st);
        if (e != hipSuccess) {
            s = set_error(VP_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(e));
        } else if (!(chi <= chi_max)) {
            char msg[320];
            snprintf(msg, sizeof msg,
                     "boundary resolved too finely for the local expansion's density derivatives: "
                     "delta_1^1.5 max|kappa| / h^2 = %.3g exceeds %.2g (h = panel length / q); use coarser panels, "
                     "a smaller delta_1 (c_delta), or a plan with order_d <= 2", chi, chi_max);
            s = set_error(VP_ERR_GEOMETRY, msg);
        }
    }
    double bnorm = 0.0, rel = INFINITY;
    int it = 0;          // operator products, every one counted
    bool done = false;   // rel is a residual computed from x and is <= tol
    std::vector<double> H((size_t)(m + 1) * m), z(m + 1), y(m);
    auto Vc = [&](int k) { return V + (size_t)k * n; };
    auto dev_err = [&](hipError_t er) { return set_error(VP_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(er)); };
    if (s == VP_OK) s = make_rhs(S, b);
    if (s == VP_OK) s = S.dot(b, b, &bnorm);
    bnorm = std::sqrt(bnorm);
    if (s == VP_OK && bnorm == 0.0) {  // zero data: zero solution
        e = hipMemsetAsync(x, 0, (size_t)n * sizeof(double), S.st);
        if (e != hipSuccess) s = dev_err(e);
        rel = 0.0;
        done = true;
    }
    const unsigned gn = (unsigned)((n + kSolveThreads - 1) / kSolveThreads);
    while (s == VP_OK && !done && it < max_iter) {
        // r = b - A x in V_0: the residual of x itself
        if ((s = S.matvec(x, Vc(0))) != VP_OK) break;
        ++it;
        if ((s = S.axpby(1.0, b, -1.0, Vc(0))) != VP_OK) break;
        double beta = 0.0;
        if ((s = S.dot(Vc(0), Vc(0), &beta)) != VP_OK) break;
        beta = std::sqrt(beta);
        rel = beta / bnorm;
        if (rel <= tol) {
            done = true;
            break;
        }
        if (it >= max_iter) break;
        if ((s = S.axpby(0.0, b, 1.0 / beta, Vc(0))) != VP_OK) break;
        hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, S.st, m, beta, bnorm, zd, std_, mirror_dev);
        if ((s = S.launched()) != VP_OK) break;
        // steps on the device; the host checks step k's flag after enqueuing step k + 1
        int kq = 0;
        bool stop = false;
        while (kq < m && it < max_iter && !stop) {
            if ((s = S.matvec(Vc(kq), w)) != VP_OK) break;
            ++it;
            if ((s = S.orthogonalize(V, kq, w)) != VP_OK) break;
            hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(64), 0, S.st, kq, m, S.hd, Hd, csd, snd, zd, tol, bnorm, std_,
                               mirror_dev);
            hipLaunchKernelGGL(k_scale_dev, dim3(gn), dim3(kSolveThreads), 0, S.st, n, w, std_, Vc(kq + 1));
            if ((s = S.launched()) != VP_OK) break;
            if ((e = hipEventRecord(plan->solve_ev[kq & 1], S.st)) != hipSuccess) {
                s = dev_err(e);
                break;
            }
            ++kq;
            if (kq >= 2) {  // step kq - 2 has been followed by step kq - 1: wait for it, read its flag
                if ((e = hipEventSynchronize(plan->solve_ev[kq & 1])) != hipSuccess) {
                    s = dev_err(e);
                    break;
                }
                stop = mirror->done != 0;
            }
        }
        if (s != VP_OK) break;
        if ((e = hipStreamSynchronize(S.st)) != hipSuccess) {
            s = dev_err(e);
            break;
        }
        const int k = mirror->k;
        rel = mirror->rel;   // the recurrence's estimate; the next cycle checks it
        if (k == 0) break;
        // the cycle's rotated Hessenberg matrix and z, once per cycle; x += V y with H y = z
        e = hipMemcpy(H.data(), Hd, (size_t)k * m * sizeof(double), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(z.data(), zd, (size_t)k * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            s = dev_err(e);
            break;
        }
        for (int i = k - 1; i >= 0; --i) {
            double t = z[i];
            for (int j = i + 1; j < k; ++j) t -= H[(size_t)i * m + j] * y[j];
            y[i] = t / H[(size_t)i * m + i];
        }
        for (int i = 0; i < k && s == VP_OK; ++i) s = S.axpby(y[i], Vc(i), 1.0, x);
    }
    if (s == VP_OK) {
        e = hipStreamSynchronize(plan->stream);
        if (e != hipSuccess) s = set_error(VP_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(e));
    }
    if (iters) *iters = it;
    if (resid) *resid = rel;
    if (s == VP_OK && !done) s = set_error(VP_ERR_TOL, "GMRES did not reach the tolerance within max_iter products");
    return s;
}

}  // namespace
}  // namespace vp

using namespace vp;

extern "C" vp_status vp_dirichlet_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x,
                                        const double* bnd_y, const int32_t* pan, const double* u, const double* g,
                                        const double* f_src, const double* jet6, double* mu, double tol,
                                        int max_iter, int restart, int* iters, double* resid)
{
    vp_status s = check_solve_args(plan, n_pan, q, bnd_x, bnd_y, pan, u, g, mu, tol, max_iter, restart);
    if (s == VP_OK) s = check_source(plan, f_src, jet6);
    if (s != VP_OK) return s;
    auto rhs = [&](Solver& S, double* b) {  // b = g - V[f]
        if (!f_src) return S.axpby(1.0, g, 0.0, b);
        vp_status r = vp_volume(plan, f_src, jet6, b);
        return r == VP_OK ? S.axpby(1.0, g, -1.0, b) : r;
    };
    return gmres_solve(plan, n_pan, q, bnd_x, bnd_y, pan, u, nullptr, rhs, mu, tol, max_iter, restart, iters, resid);
}

extern "C" vp_status vp_exterior_dirichlet_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x,
                                                 const double* bnd_y, const double* bnd_w, const int32_t* pan,
                                                 const double* u, const double* g, double* mu, double tol,
                                                 int max_iter, int restart, int* iters, double* resid)
{
    vp_status s = check_solve_args(plan, n_pan, q, bnd_x, bnd_y, pan, u, g, mu, tol, max_iter, restart);
    if (s != VP_OK) return s;
    if (!bnd_w) return set_error(VP_ERR_ARG, "NULL array");
    auto rhs = [&](Solver& S, double* b) { return S.axpby(1.0, g, 0.0, b); };
    return gmres_solve(plan, n_pan, q, bnd_x, bnd_y, pan, u, bnd_w, rhs, mu, tol, max_iter, restart, iters, resid);
}

extern "C" vp_status vp_exterior_dirichlet_solve_growth(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x,
                                                        const double* bnd_y, const double* bnd_w, const int32_t* pan,
                                                        const double* u, const double* g, double A, double x0,
                                                        double y0, double* mu, double tol, int max_iter, int restart,
                                                        int* iters, double* resid)
{
    vp_status s = check_solve_args(plan, n_pan, q, bnd_x, bnd_y, pan, u, g, mu, tol, max_iter, restart);
    if (s != VP_OK) return s;
    if (!bnd_w) return set_error(VP_ERR_ARG, "NULL array");
    if (!std::isfinite(A) || !std::isfinite(x0) || !std::isfinite(y0))
        return set_error(VP_ERR_ARG, "non-finite growth coefficient or centre");
    auto rhs = [&](Solver& S, double* b) { return S.minus_growth(g, A, x0, y0, b); };
    return gmres_solve(plan, n_pan, q, bnd_x, bnd_y, pan, u, bnd_w, rhs, mu, tol, max_iter, restart, iters, resid);
}

extern "C" vp_status vp_add_log_growth(int64_t n, const double* x, const double* y, double A, double x0, double y0,
                                       double* out, void* stream)
{
    if (n < 0) return set_error(VP_ERR_ARG, "negative count");
    if (n == 0) return VP_OK;
    if (!x || !y || !out) return set_error(VP_ERR_ARG, "NULL array");
    if (!std::isfinite(A) || !std::isfinite(x0) || !std::isfinite(y0))
        return set_error(VP_ERR_ARG, "non-finite growth coefficient or centre");
    hipLaunchKernelGGL(k_log_growth, dim3((unsigned)((n + kSolveThreads - 1) / kSolveThreads)), dim3(kSolveThreads), 0,
                       (hipStream_t)stream, n, x, y, A, x0, y0, out, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? VP_OK : set_error(VP_ERR_DEVICE, std::string("growth term: ") + hipGetErrorString(e));
}

extern "C" vp_status vp_neumann_solve(vp_plan_t plan, int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                                      const double* bnd_w, const int32_t* pan, const double* u, const double* g,
                                      const double* f_src, const double* jet6, double* ub, double tol, int max_iter,
                                      int restart, int* iters, double* resid)
{
    vp_status s = check_solve_args(plan, n_pan, q, bnd_x, bnd_y, pan, u, g, ub, tol, max_iter, restart);
    if (s == VP_OK) s = check_source(plan, f_src, jet6);
    if (s != VP_OK) return s;
    if (!bnd_w) return set_error(VP_ERR_ARG, "NULL array");
    if (!(plan->kinds & VP_KIND_S)) return set_error(VP_ERR_ARG, "the plan does not support the single layer");
    auto rhs = [&](Solver& S, double* b) {  // b = V[f] + S[g]; g's jets staged in the product's jet buffer
        vp_status r = boundary_jets_ws(n_pan, q, bnd_x, bnd_y, g, S.n, pan, u, 2, S.jets, S.st, S.gws);
        return r == VP_OK ? vp_eval(plan, f_src, jet6, g, S.jets, nullptr, nullptr, b) : r;
    };
    return gmres_solve(plan, n_pan, q, bnd_x, bnd_y, pan, u, bnd_w, rhs, ub, tol, max_iter, restart, iters, resid);
}
