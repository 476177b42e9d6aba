// Local frame of each target and layer-density jets from a boundary given as
// Gauss-Legendre panels: the per-target geometry the local expansions of
// Sec. 4 take as input (closest boundary point b, distance, side, normal,
// curvature and the next two derivatives of the curve as a graph over its
// tangent line at b, and the densities' derivatives along that line).
//
// Panels: n_pan in order along the curve, counter-clockwise, each with q nodes
// at the Gauss-Legendre points of its own parameter u in [-1, 1] (ascending).
// On a panel a coordinate or a density is its degree q-1 interpolant in u,
// held as Legendre coefficients from the discrete transform
//     c_k = (2k+1)/2 sum_j w_j P_k(u_j) f_j      (exact for the interpolant),
// less the coefficients below the transform's rounding bound 4 q eps max|f|.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "vp_geom.hpp"
#include "vp_internal.hpp"

// Fixed scratch of the allocation-free jets (vp_boundary_jets_noalloc): the
// Legendre coefficients of x, y and the density, 3 n_pan q doubles for up to
// VP_NOALLOC_MAX_NODES nodes (1.5 MiB).  Every device the library runs on
// holds its own copy until the process ends.  In host code this name is a
// host-side stand-in: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[3 * VP_NOALLOC_MAX_NODES];

namespace vp {
namespace {

constexpr int kGeomQMax = 32;
constexpr int kGeomThreads = 256;
constexpr int kNewtonIters = 30;
constexpr double kOnCurve = 1e-12;  // r <= kOnCurve |x'(u*)|: on the boundary
constexpr int kPanTile = 256;       // panel circles staged per LDS tile

// Gauss-Legendre node j (ascending) and weight for q points, by Newton on P_q.
__device__ void gauss_legendre(int q, int j, double* x, double* w)
{
    const int k = q - 1 - j;  // roots from the top
    double t = cos(M_PI * (k + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = t;
        for (int n = 1; n < q; ++n) {
            const double p2 = ((2.0 * n + 1.0) * t * p1 - n * p0) / (n + 1.0);
            p0 = p1;
            p1 = p2;
        }
        dp = q * (t * p1 - p0) / (t * t - 1.0);
        const double dt = p1 / dp;
        t -= dt;
        // quadratic convergence: a step of a few ulps leaves t at rounding level (a
        // tighter test can miss, the iterate then alternating between neighbours)
        if (fabs(dt) <= 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(t))) break;
    }
    double p0 = 1.0, p1 = t;
    for (int n = 1; n < q; ++n) {
        const double p2 = ((2.0 * n + 1.0) * t * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    dp = q * (t * p1 - p0) / (t * t - 1.0);
    *x = t;
    *w = 2.0 / ((1.0 - t * t) * dp * dp);
}

// One workgroup per panel: Legendre coefficients of up to three node arrays
// (coef[a][pan][q]) and, with circ, the panel's node bounding circle.
__global__ __launch_bounds__(64) void k_panel_coef(int64_t n_pan, int q, const double* __restrict__ f0,
                                                   const double* __restrict__ f1, const double* __restrict__ f2,
                                                   double* __restrict__ c0, double* __restrict__ c1,
                                                   double* __restrict__ c2, double* __restrict__ circ)
{
    __shared__ double xs[kGeomQMax], ws[kGeomQMax], fv[3][kGeomQMax], fabsmax[3];
    __shared__ double Pk[kGeomQMax][kGeomQMax + 1];  // Pk[k][j] = P_k(u_j)
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const double* src[3] = {f0, f1, f2};
    double* dst[3] = {c0, c1, c2};
    if (t < q) {
        gauss_legendre(q, t, &xs[t], &ws[t]);
        for (int a = 0; a < 3; ++a) fv[a][t] = src[a] ? src[a][p * q + t] : 0.0;
    }
    __syncthreads();
    if (t < q) {  // P_0 .. P_{q-1} at this thread's node, by the three-term recurrence
        const double u = xs[t];
        double pk = 1.0, pkm1 = 0.0;
        Pk[0][t] = 1.0;
        for (int n = 0; n + 1 < q; ++n) {
            const double pn = ((2.0 * n + 1.0) * u * pk - n * pkm1) / (n + 1.0);
            pkm1 = pk;
            pk = pn;
            Pk[n + 1][t] = pk;
        }
    }
    if (t < 3) {
        double m = 0.0;
        for (int j = 0; j < q; ++j) m = fmax(m, fabs(fv[t][j]));
        fabsmax[t] = m;
    }
    if (circ && t == 0) {
        double cx = 0.0, cy = 0.0;
        for (int j = 0; j < q; ++j) {
            cx += fv[0][j];
            cy += fv[1][j];
        }
        cx /= q;
        cy /= q;
        double rr = 0.0;
        for (int j = 0; j < q; ++j) rr = fmax(rr, hypot(fv[0][j] - cx, fv[1][j] - cy));
        circ[3 * p] = cx;
        circ[3 * p + 1] = cy;
        circ[3 * p + 2] = rr;
    }
    __syncthreads();
    if (t < q) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < q; ++j) {
            const double pk = Pk[t][j];
            for (int a = 0; a < 3; ++a) acc[a] += ws[j] * pk * fv[a][j];
        }
        const double floor_scale = 4.0 * q * 2.220446049250313e-16;
        for (int a = 0; a < 3; ++a)
            if (dst[a]) {
                const double c = (2.0 * t + 1.0) / 2.0 * acc[a];
                dst[a][p * q + t] = fabs(c) < floor_scale * fabsmax[a] ? 0.0 : c;
            }
    }
}

// d[m] = (d^m/du^m) sum_k c_k P_k(u), m = 0..M.
template <int M>
__device__ void legendre_derivs(const double* __restrict__ c, int q, double u, double* d)
{
    double pk[M + 1], pkm1[M + 1];
#pragma unroll
    for (int m = 0; m <= M; ++m) {
        pkm1[m] = m == 0 ? 1.0 : 0.0;  // P_0
        pk[m] = m == 0 ? u : (m == 1 ? 1.0 : 0.0);  // P_1
        d[m] = c[0] * pkm1[m] + (q > 1 ? c[1] * pk[m] : 0.0);
    }
    for (int k = 1; k + 1 < q; ++k) {
        double pn[M + 1];
#pragma unroll
        for (int m = 0; m <= M; ++m)
            pn[m] = ((2.0 * k + 1.0) * (u * pk[m] + (m > 0 ? m * pk[m - 1] : 0.0)) - k * pkm1[m]) / (k + 1.0);
        const double ck = c[k + 1];
#pragma unroll
        for (int m = 0; m <= M; ++m) {
            d[m] += ck * pn[m];
            pkm1[m] = pk[m];
            pk[m] = pn[m];
        }
    }
}

// xi-derivatives g[0..4] of h(u(xi)) from xi[1..4] and h[0..4] (u-derivatives):
// inverse function, then Faa di Bruno.
__device__ void inverse_chain(const double* xi, const double* h, double* g)
{
    const double x1 = xi[1], x2 = xi[2], x3 = xi[3], x4 = xi[4];
    const double u1 = 1.0 / x1;
    const double u2 = -x2 * u1 * u1 * u1;
    const double u3 = (3.0 * x2 * x2 - x1 * x3) * u1 * u1 * u1 * u1 * u1;
    const double u4 = (-15.0 * x2 * x2 * x2 + 10.0 * x1 * x2 * x3 - x1 * x1 * x4) * u1 * u1 * u1 * u1 * u1 * u1 * u1;
    g[0] = h[0];
    g[1] = h[1] * u1;
    g[2] = h[2] * u1 * u1 + h[1] * u2;
    g[3] = h[3] * u1 * u1 * u1 + 3.0 * h[2] * u1 * u2 + h[1] * u3;
    g[4] = h[4] * u1 * u1 * u1 * u1 + 6.0 * h[3] * u1 * u1 * u2 + h[2] * (3.0 * u2 * u2 + 4.0 * u1 * u3) + h[1] * u4;
}

struct FrameArgs {
    int64_t n_pan, n_tgt;
    int q;
    const double *bx, *by, *cx, *cy, *circ, *tx, *ty;
    double *r, *nx, *ny, *kappa, *g3, *g4, *upar;
    int8_t* sgn;
    int32_t* pan;
};

// One thread per target: nearest node (panels pruned by their node circles),
// Newton on the panel interpolant, frame at the closest point.
__global__ __launch_bounds__(kGeomThreads) void k_frame(FrameArgs a)
{
    __shared__ double sc[3 * kPanTile];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = i < a.n_tgt;
    const double px = on ? a.tx[i] : 0.0, py = on ? a.ty[i] : 0.0;
    // pass 1: U = min over panels of (distance to the circle's centre + radius) bounds the nearest node
    double U = INFINITY;
    for (int64_t p0 = 0; p0 < a.n_pan; p0 += kPanTile) {
        const int nt = (int)min<int64_t>(kPanTile, a.n_pan - p0);
        __syncthreads();
        for (int k = threadIdx.x; k < 3 * nt; k += blockDim.x) sc[k] = a.circ[3 * p0 + k];
        __syncthreads();
        for (int k = 0; k < nt; ++k) {
            const double ex = px - sc[3 * k], ey = py - sc[3 * k + 1];
            U = fmin(U, sqrt(ex * ex + ey * ey) + sc[3 * k + 2]);
        }
    }
    // pass 2: nodes of the panels whose circle comes within U (lowest index on
    // ties), on squared distances
    double best = INFINITY;
    int64_t jbest = 0;
    for (int64_t p0 = 0; p0 < a.n_pan; p0 += kPanTile) {
        const int nt = (int)min<int64_t>(kPanTile, a.n_pan - p0);
        __syncthreads();
        for (int k = threadIdx.x; k < 3 * nt; k += blockDim.x) sc[k] = a.circ[3 * p0 + k];
        __syncthreads();
        for (int k = 0; k < nt; ++k) {
            const double ex = px - sc[3 * k], ey = py - sc[3 * k + 1], reach = U + sc[3 * k + 2];
            if (!on || ex * ex + ey * ey > reach * reach) continue;
            const int64_t jb = (p0 + k) * a.q;
            for (int j = 0; j < a.q; ++j) {
                const double dx0 = px - a.bx[jb + j], dy0 = py - a.by[jb + j];
                const double d = dx0 * dx0 + dy0 * dy0;
                if (d < best) {
                    best = d;
                    jbest = jb + j;
                }
            }
        }
    }
    if (!on) return;
    const int q = a.q;
    int64_t p = jbest / q;
    double xg, wg;
    gauss_legendre(q, (int)(jbest % q), &xg, &wg);
    double uu = xg;
    double dx[5], dy[5];
    for (int it = 0; it < kNewtonIters; ++it) {
        legendre_derivs<2>(a.cx + p * q, q, uu, dx);
        legendre_derivs<2>(a.cy + p * q, q, uu, dy);
        const double gx = dx[0] - px, gy = dy[0] - py;
        const double g = gx * dx[1] + gy * dy[1];
        const double gp = dx[1] * dx[1] + dy[1] * dy[1] + gx * dx[2] + gy * dy[2];
        const double un = uu - g / gp;
        if (un > 1.0) {
            p = (p + 1) % a.n_pan;
            uu = -1.0;
        } else if (un < -1.0) {
            p = (p - 1 + a.n_pan) % a.n_pan;
            uu = 1.0;
        } else {
            const bool done = fabs(un - uu) <= 1e-15;
            uu = un;
            if (done) break;
        }
    }
    legendre_derivs<4>(a.cx + p * q, q, uu, dx);
    legendre_derivs<4>(a.cy + p * q, q, uu, dy);
    const double sp = hypot(dx[1], dy[1]);
    const double tx = dx[1] / sp, ty = dy[1] / sp;
    const double nx = ty, ny = -tx;  // outward for a counter-clockwise curve
    const double ddx = px - dx[0], ddy = py - dy[0];
    const double r = hypot(ddx, ddy);
    double xi[5], eta[5], g[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        xi[m] = dx[m] * tx + dy[m] * ty;
        eta[m] = -(dx[m] * nx + dy[m] * ny);
    }
    inverse_chain(xi, eta, g);
    a.r[i] = r;
    a.nx[i] = nx;
    a.ny[i] = ny;
    a.kappa[i] = g[2];
    if (a.g3) a.g3[i] = g[3];
    if (a.g4) a.g4[i] = g[4];
    a.sgn[i] = (int8_t)(r <= kOnCurve * sp ? 0 : (ddx * nx + ddy * ny < 0.0 ? 1 : -1));
    a.pan[i] = (int32_t)p;
    a.upar[i] = uu;
}

__global__ __launch_bounds__(kGeomThreads) void k_jets(int64_t n_pan, int q, int64_t n_tgt, const double* __restrict__ cx,
                                                      const double* __restrict__ cy, const double* __restrict__ cs,
                                                      const int32_t* __restrict__ pan, const double* __restrict__ upar,
                                                      int nder, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tgt) return;
    const int64_t p = pan[i];
    const double uu = upar[i];
    if (p < 0 || p >= n_pan) {  // not a location from vp_boundary_frame: no read
        for (int k = 0; k <= nder; ++k) out[(int64_t)k * n_tgt + i] = NAN;
        return;
    }
    double dx[5], dy[5], ds[5], xi[5], g[5];
    legendre_derivs<4>(cx + p * q, q, uu, dx);
    legendre_derivs<4>(cy + p * q, q, uu, dy);
    legendre_derivs<4>(cs + p * q, q, uu, ds);
    const double sp = hypot(dx[1], dy[1]);
    const double tx = dx[1] / sp, ty = dy[1] / sp;
#pragma unroll
    for (int m = 0; m < 5; ++m) xi[m] = dx[m] * tx + dy[m] * ty;
    inverse_chain(xi, ds, g);
    for (int k = 0; k <= nder; ++k) out[(int64_t)k * n_tgt + i] = g[k];
}

vp_status gfail(vp_status s, const std::string& m) { return set_error(s, m); }

vp_status geom_check(int64_t n_pan, int q, const double* bx, const double* by, int64_t n_tgt)
{
    if (q < 5 || q > kGeomQMax) return gfail(VP_ERR_ARG, "panel size q must be in [5, 32]");
    if (n_pan < 2) return gfail(VP_ERR_ARG, "at least two panels");
    if (n_tgt < 0) return gfail(VP_ERR_ARG, "negative target count");
    if (!bx || !by) return gfail(VP_ERR_ARG, "NULL boundary nodes");
    return VP_OK;
}

hipError_t alloc_async(double** p, size_t n, hipStream_t st)
{
    return hipMallocAsync((void**)p, n * sizeof(double), st);
}

// Device address of the fixed scratch on the current device, looked up once
// per device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

vp_status scratch_address(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gfail(VP_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return gfail(VP_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return gfail(VP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return VP_OK;
}

}  // namespace

vp_status boundary_jets_ws(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y, const double* dens,
                           int64_t n_tgt, const int32_t* pan, const double* u, int nder, double* out, hipStream_t st,
                           double* ws)
{
    if (n_tgt == 0) return VP_OK;
    double* cx = ws;
    double* cy = ws + (size_t)n_pan * q;
    double* cs = ws + (size_t)2 * n_pan * q;
    hipLaunchKernelGGL(k_panel_coef, dim3((unsigned)n_pan), dim3(64), 0, st, n_pan, q, bnd_x, bnd_y, dens, cx, cy, cs,
                       (double*)nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_jets, dim3((unsigned)((n_tgt + kGeomThreads - 1) / kGeomThreads)), dim3(kGeomThreads), 0,
                           st, n_pan, q, n_tgt, cx, cy, cs, pan, u, nder, out);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return gfail(VP_ERR_DEVICE, std::string("boundary jets: ") + hipGetErrorString(e));
    return VP_OK;
}

}  // namespace vp

using namespace vp;

extern "C" vp_status vp_boundary_frame(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y, int64_t n_tgt,
                                       const double* tgt_x, const double* tgt_y, double* r, double* nx, double* ny,
                                       double* kappa, double* gamma3, double* gamma4, int8_t* sgn, int32_t* pan,
                                       double* u, void* stream)
{
    vp_status s = geom_check(n_pan, q, bnd_x, bnd_y, n_tgt);
    if (s != VP_OK) return s;
    if (n_tgt == 0) return VP_OK;
    if (!tgt_x || !tgt_y || !r || !nx || !ny || !kappa || !sgn || !pan || !u) return gfail(VP_ERR_ARG, "NULL output or target array");
    if (n_pan > INT32_MAX) return gfail(VP_ERR_ARG, "too many panels");
    hipStream_t st = (hipStream_t)stream;
    double *cx = nullptr, *cy = nullptr, *circ = nullptr;
    hipError_t e = alloc_async(&cx, (size_t)n_pan * q, st);
    if (e == hipSuccess) e = alloc_async(&cy, (size_t)n_pan * q, st);
    if (e == hipSuccess) e = alloc_async(&circ, (size_t)n_pan * 3, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_panel_coef, dim3((unsigned)n_pan), dim3(64), 0, st, n_pan, q, bnd_x, bnd_y,
                           (const double*)nullptr, cx, cy, (double*)nullptr, circ);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        FrameArgs a{n_pan, n_tgt, q, bnd_x, bnd_y, cx, cy, circ, tgt_x, tgt_y, r, nx, ny, kappa, gamma3, gamma4, u,
                    sgn, pan};
        hipLaunchKernelGGL(k_frame, dim3((unsigned)((n_tgt + kGeomThreads - 1) / kGeomThreads)), dim3(kGeomThreads), 0,
                           st, a);
        e = hipGetLastError();
    }
    if (cx) (void)hipFreeAsync(cx, st);
    if (cy) (void)hipFreeAsync(cy, st);
    if (circ) (void)hipFreeAsync(circ, st);
    if (e != hipSuccess)
        return gfail(e == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,
                    std::string("boundary frame: ") + hipGetErrorString(e));
    return VP_OK;
}

extern "C" vp_status vp_boundary_jets(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                                      const double* dens, int64_t n_tgt, const int32_t* pan, const double* u, int nder,
                                      double* out, void* stream)
{
    vp_status s = geom_check(n_pan, q, bnd_x, bnd_y, n_tgt);
    if (s != VP_OK) return s;
    if (nder < 0 || nder > 4) return gfail(VP_ERR_ARG, "nder must be in [0, 4]");
    if (n_tgt == 0) return VP_OK;
    if (!dens || !pan || !u || !out) return gfail(VP_ERR_ARG, "NULL density, location or output array");
    hipStream_t st = (hipStream_t)stream;
    double* ws = nullptr;  // coefficients of x, y and the density, one allocation
    hipError_t e = alloc_async(&ws, (size_t)3 * n_pan * q, st);
    if (e != hipSuccess)
        return gfail(e == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,
                    std::string("boundary jets: ") + hipGetErrorString(e));
    s = boundary_jets_ws(n_pan, q, bnd_x, bnd_y, dens, n_tgt, pan, u, nder, out, st, ws);
    (void)hipFreeAsync(ws, st);
    return s;
}

extern "C" vp_status vp_boundary_jets_noalloc(int64_t n_pan, int q, const double* bnd_x, const double* bnd_y,
                                              const double* dens, int64_t n_tgt, const int32_t* pan, const double* u,
                                              int nder, double* out, void* stream)
{
    vp_status s = geom_check(n_pan, q, bnd_x, bnd_y, n_tgt);
    if (s != VP_OK) return s;
    if (nder < 0 || nder > 4) return gfail(VP_ERR_ARG, "nder must be in [0, 4]");
    if (n_pan * q > VP_NOALLOC_MAX_NODES)
        return gfail(VP_ERR_ARG, "n_pan * q = " + std::to_string(n_pan * q) + " exceeds VP_NOALLOC_MAX_NODES = " +
                                     std::to_string(VP_NOALLOC_MAX_NODES));
    double* ws = nullptr;  // resolved before the n_tgt = 0 return: set-up on the first call either way
    if ((s = scratch_address(&ws)) != VP_OK) return s;
    if (n_tgt == 0) return VP_OK;
    if (!dens || !pan || !u || !out) return gfail(VP_ERR_ARG, "NULL density, location or output array");
    // k_panel_coef writes every coefficient the jets read, so nothing is cleared
    return boundary_jets_ws(n_pan, q, bnd_x, bnd_y, dens, n_tgt, pan, u, nder, out, (hipStream_t)stream, ws);
}
