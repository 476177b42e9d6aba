// Jets of the volume density at the volume nodes from per-triangle quadratic
// interpolants: f, f_x, f_y, f_xx, f_xy, f_yy, the derivatives the volume
// local part of Sec. 4 (Lemma 4.1) takes, when f is known only at the nodes of
// the triangulation of Sec. 2.2 (six nodes per triangle).
//
// A triangle's six nodes determine the quadratic through them.  It is fitted
// in the nodes' principal-axis coordinates, each axis scaled by its own
// spread (u = e1.(x - c)/s1, v = e2.(x - c)/s2): the same interpolant as in
// any affine coordinates, but its 6x6 system stays well conditioned on
// slivers, whose extents differ by orders of magnitude.  Derivatives come
// back to (x, y) through the constant Jacobian of that map.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "vp_internal.hpp"

namespace vp {
namespace {

constexpr int kJetThreads = 256;

// Solve the 6 x 6 system in A[.][0..5] with right-hand side A[.][6] by Gaussian
// elimination with partial pivoting; ok becomes false when a pivot is not above
// thr.  Every loop has compile-time bounds and the row exchange is done with
// selects at compile-time indices, so A stays in registers (a runtime row index
// would put the array in scratch memory).
__device__ __forceinline__ void solve6(double (&A)[6][7], double (&c)[6], double thr, bool& ok)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int p = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < 6; ++r)
            if (fabs(A[r][k]) > best) {
                best = fabs(A[r][k]);
                p = r;
            }
        if (!(best > thr)) ok = false;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const bool sw = r == p;
#pragma unroll
            for (int j = k; j < 7; ++j) {
                const double a = A[k][j], b = A[r][j];
                A[k][j] = sw ? b : a;
                A[r][j] = sw ? a : b;
            }
        }
        const double inv = best > 0.0 ? 1.0 / A[k][k] : 0.0;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const double m = A[r][k] * inv;
#pragma unroll
            for (int j = k; j < 7; ++j) A[r][j] -= m * A[k][j];
        }
    }
#pragma unroll
    for (int k = 5; k >= 0; --k) {
        double sum = A[k][6];
#pragma unroll
        for (int j = k + 1; j < 6; ++j) sum -= A[k][j] * c[j];
        c[k] = A[k][k] != 0.0 ? sum / A[k][k] : 0.0;
    }
}

// one thread per triangle; jet [6][6 n_tri], the nodes' order
__global__ __launch_bounds__(kJetThreads) void k_volume_jets(int64_t n_tri, const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             const double* __restrict__ f, double* __restrict__ jet)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    const int64_t n = 6 * n_tri;
    const int64_t o = 6 * t;
    double px[6], py[6], pf[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        px[l] = x[o + l];
        py[l] = y[o + l];
        pf[l] = f[o + l];
    }
    double cx = 0.0, cy = 0.0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        cx += px[l];
        cy += py[l];
    }
    cx /= 6.0;
    cy /= 6.0;
    double sxx = 0.0, sxy = 0.0, syy = 0.0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const double dx = px[l] - cx, dy = py[l] - cy;
        sxx += dx * dx;
        sxy += dx * dy;
        syy += dy * dy;
    }
    // principal axes of the nodes' spread
    const double half = 0.5 * (sxx - syy);
    const double rad = sqrt(half * half + sxy * sxy);
    const double l1 = 0.5 * (sxx + syy) + rad, l2 = 0.5 * (sxx + syy) - rad;
    double e1x, e1y;
    if (sxx >= syy) {
        e1x = l1 - syy;
        e1y = sxy;
    } else {
        e1x = sxy;
        e1y = l1 - sxx;
    }
    const double en = hypot(e1x, e1y);
    // else the nodes lie on a line within rounding (collinear sets give l2 ~ 1e-16 l1; a
    // sliver of aspect 1e4 has l2 ~ 1e-8 l1)
    bool ok = l1 > 0.0 && l2 > 1e-14 * l1;
    if (en > 0.0) {
        e1x /= en;
        e1y /= en;
    } else {  // isotropic spread: every direction is principal
        e1x = 1.0;
        e1y = 0.0;
    }
    const double e2x = -e1y, e2y = e1x;
    const double s1 = ok ? sqrt(l1 / 6.0) : 1.0, s2 = ok ? sqrt(l2 / 6.0) : 1.0;
    // rows [1, u, v, u^2, uv, v^2 | f]
    double A[6][7], uu[6], vv[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const double dx = px[l] - cx, dy = py[l] - cy;
        const double u = (e1x * dx + e1y * dy) / s1, v = (e2x * dx + e2y * dy) / s2;
        uu[l] = u;
        vv[l] = v;
        A[l][0] = 1.0;
        A[l][1] = u;
        A[l][2] = v;
        A[l][3] = u * u;
        A[l][4] = u * v;
        A[l][5] = v * v;
        A[l][6] = pf[l];
    }
    // a pivot below 1e-10 of the columns' scale (O(1) here) means the nodes do not
    // determine a quadratic
    double c[6];
    solve6(A, c, 1e-10, ok);
    // (u, v) = J (x - c): J rows e1/s1, e2/s2
    const double j00 = e1x / s1, j01 = e1y / s1, j10 = e2x / s2, j11 = e2y / s2;
    const double quu = 2.0 * c[3], quv = c[4], qvv = 2.0 * c[5];
    const double hxx = j00 * j00 * quu + 2.0 * j00 * j10 * quv + j10 * j10 * qvv;
    const double hxy = j00 * j01 * quu + (j00 * j11 + j10 * j01) * quv + j10 * j11 * qvv;
    const double hyy = j01 * j01 * quu + 2.0 * j01 * j11 * quv + j11 * j11 * qvv;
    const double bad = NAN;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const double qu = c[1] + 2.0 * c[3] * uu[l] + c[4] * vv[l];
        const double qv = c[2] + c[4] * uu[l] + 2.0 * c[5] * vv[l];
        jet[o + l] = pf[l];
        jet[n + o + l] = ok ? qu * j00 + qv * j10 : bad;
        jet[2 * n + o + l] = ok ? qu * j01 + qv * j11 : bad;
        jet[3 * n + o + l] = ok ? hxx : bad;
        jet[4 * n + o + l] = ok ? hxy : bad;
        jet[5 * n + o + l] = ok ? hyy : bad;
    }
}

// Principal axes (e1, e2 = e1 rotated by 90 degrees) and their spreads l1 >= l2 of
// the second moments sxx, sxy, syy.
__device__ inline void principal_axes(double sxx, double sxy, double syy, double& e1x, double& e1y, double& l1,
                                      double& l2)
{
    const double half = 0.5 * (sxx - syy);
    const double rad = sqrt(half * half + sxy * sxy);
    l1 = 0.5 * (sxx + syy) + rad;
    l2 = 0.5 * (sxx + syy) - rad;
    if (sxx >= syy) {
        e1x = l1 - syy;
        e1y = sxy;
    } else {
        e1x = sxy;
        e1y = l1 - sxx;
    }
    const double en = hypot(e1x, e1y);
    if (en > 0.0) {
        e1x /= en;
        e1y /= en;
    } else {  // isotropic spread: every direction is principal
        e1x = 1.0;
        e1y = 0.0;
    }
}

// One thread per triangle: the least-squares quadratic over the triangle's six
// nodes and the six nodes of each edge neighbour nbr[3 t + e] (entries outside
// [0, n_tri) and t itself are skipped), in the patch's principal-axis
// coordinates scaled by their spreads, from its 6 x 6 normal equations.  The
// fitted quadratic does not depend on the coordinates (quadratics are closed
// under affine maps); the scaling keeps the normal equations well conditioned.
constexpr int kPatchMax = 4;  // the triangle and up to three neighbours
__global__ __launch_bounds__(kJetThreads) void k_volume_jets_patch(int64_t n_tri, const double* __restrict__ x,
                                                                   const double* __restrict__ y,
                                                                   const double* __restrict__ f,
                                                                   const int32_t* __restrict__ nbr,
                                                                   double* __restrict__ jet)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    const int64_t n = 6 * n_tri;
    int64_t tri[kPatchMax];
    int nt = 0;
    tri[nt++] = t;
    for (int e = 0; e < 3; ++e) {
        const int64_t k = nbr[3 * t + e];
        if (k >= 0 && k < n_tri && k != t) tri[nt++] = k;
    }
    const double np = 6.0 * nt;
    // first and second moments in one pass, about the triangle's first node (no cancellation
    // for patches far from the origin)
    const double ox = x[6 * t], oy = y[6 * t];
    double mx = 0.0, my = 0.0, mxx = 0.0, mxy = 0.0, myy = 0.0;
    for (int a = 0; a < nt; ++a)
        for (int l = 0; l < 6; ++l) {
            const double dx = x[6 * tri[a] + l] - ox, dy = y[6 * tri[a] + l] - oy;
            mx += dx;
            my += dy;
            mxx += dx * dx;
            mxy += dx * dy;
            myy += dy * dy;
        }
    mx /= np;
    my /= np;
    const double cx = ox + mx, cy = oy + my;
    const double sxx = mxx - np * mx * mx, sxy = mxy - np * mx * my, syy = myy - np * my * my;
    double e1x, e1y, l1, l2;
    principal_axes(sxx, sxy, syy, e1x, e1y, l1, l2);
    bool ok = l1 > 0.0 && l2 > 1e-14 * l1;  // else the patch's nodes lie on a line within rounding
    const double e2x = -e1y, e2y = e1x;
    const double s1 = ok ? sqrt(l1 / np) : 1.0, s2 = ok ? sqrt(l2 / np) : 1.0;
    // normal equations [M | b], M = sum a a^T (upper triangle accumulated), b = sum a f,
    // a = (1, u, v, u^2, uv, v^2)
    double A[6][7];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 7; ++c) A[r][c] = 0.0;
    for (int a = 0; a < nt; ++a)
        for (int l = 0; l < 6; ++l) {
            const int64_t i = 6 * tri[a] + l;
            const double dx = x[i] - cx, dy = y[i] - cy;
            const double u = (e1x * dx + e1y * dy) / s1, v = (e2x * dx + e2y * dy) / s2;
            const double m[7] = {1.0, u, v, u * u, u * v, v * v, f[i]};
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = r; c < 7; ++c) A[r][c] += m[r] * m[c];
        }
#pragma unroll
    for (int r = 1; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < r; ++c) A[r][c] = A[c][r];
    // a pivot below 1e-11 of the point count (the scale of M here) means the patch does
    // not fix a quadratic
    double c[6];
    solve6(A, c, 1e-11 * np, ok);
    const double j00 = e1x / s1, j01 = e1y / s1, j10 = e2x / s2, j11 = e2y / s2;
    const double quu = 2.0 * c[3], quv = c[4], qvv = 2.0 * c[5];
    const double hxx = j00 * j00 * quu + 2.0 * j00 * j10 * quv + j10 * j10 * qvv;
    const double hxy = j00 * j01 * quu + (j00 * j11 + j10 * j01) * quv + j10 * j11 * qvv;
    const double hyy = j01 * j01 * quu + 2.0 * j01 * j11 * quv + j11 * j11 * qvv;
    const double bad = NAN;
    const int64_t o = 6 * t;
    for (int l = 0; l < 6; ++l) {
        const double dx = x[o + l] - cx, dy = y[o + l] - cy;
        const double u = (e1x * dx + e1y * dy) / s1, v = (e2x * dx + e2y * dy) / s2;
        const double qu = c[1] + 2.0 * c[3] * u + c[4] * v;
        const double qv = c[2] + c[4] * u + 2.0 * c[5] * v;
        jet[o + l] = f[o + l];
        jet[n + o + l] = ok ? qu * j00 + qv * j10 : bad;
        jet[2 * n + o + l] = ok ? qu * j01 + qv * j11 : bad;
        jet[3 * n + o + l] = ok ? hxx : bad;
        jet[4 * n + o + l] = ok ? hxy : bad;
        jet[5 * n + o + l] = ok ? hyy : bad;
    }
}

}  // namespace
}  // namespace vp

using namespace vp;

extern "C" vp_status vp_volume_jets(int64_t n_tri, const double* x, const double* y, const double* f, double* jet6,
                                    void* stream)
{
    if (n_tri < 0) return set_error(VP_ERR_ARG, "negative triangle count");
    if (n_tri == 0) return VP_OK;
    if (!x || !y || !f || !jet6) return set_error(VP_ERR_ARG, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_volume_jets, dim3((unsigned)((n_tri + kJetThreads - 1) / kJetThreads)), dim3(kJetThreads), 0,
                       st, n_tri, x, y, f, jet6);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VP_ERR_DEVICE, std::string("volume jets: ") + hipGetErrorString(e));
    return VP_OK;
}

extern "C" vp_status vp_volume_jets_patch(int64_t n_tri, const double* x, const double* y, const double* f,
                                          const int32_t* nbr, double* jet6, void* stream)
{
    if (n_tri < 0) return set_error(VP_ERR_ARG, "negative triangle count");
    if (n_tri == 0) return VP_OK;
    if (!x || !y || !f || !nbr || !jet6) return set_error(VP_ERR_ARG, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_volume_jets_patch, dim3((unsigned)((n_tri + kJetThreads - 1) / kJetThreads)),
                       dim3(kJetThreads), 0, st, n_tri, x, y, f, nbr, jet6);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(VP_ERR_DEVICE, std::string("volume jets: ") + hipGetErrorString(e));
    return VP_OK;
}
