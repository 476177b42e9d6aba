// Dyadic refinement of the local layer parts (Sec. 4, subsection on computing
// the local part with arbitrary precision).
//
// The local layer parts are the time integrals of the heat layer potentials
// over [0, delta_1], taken from small-time expansions whose error constant
// shrinks with the time step.  With J levels the expansions are evaluated at
// delta* = delta_1 / 4^J and the slices [delta_1/4^j, delta_1/4^(j-1)] are
// added by direct quadrature over an oversampled boundary.  Summed over j the
// slices telescope into the time integral over [delta*, delta_1], one smooth
// kernel per boundary node:
//   S:  (E1(rho^2 / 4 delta_1) - E1(rho^2 / 4 delta*)) / (4 pi)
//   D:  nu_y.(x - y) / (2 pi rho^2) (exp(-rho^2 / 4 delta_1) - exp(-rho^2 / 4 delta*))
// (both bounded as rho -> 0: ln(4^J) / (4 pi), and 0 times a bounded factor).
// The paper sums the slices level by level on per-level refinements (constant
// work per level); one kernel on the finest sampling gives the same integral
// with one pass over the nodes.
//
// Device layout: the oversampled nodes sorted by cell of a uniform grid of
// cell edge 6 sqrt(delta_1) (both kernels are below 1e-17 of their peak
// beyond 12 sqrt(delta_1)), a cell index, and the targets within
// 12 sqrt(delta_1) of the boundary, grouped by cell into units of at most 128.
// A workgroup takes a unit, one target per thread, and streams the nodes of
// the 5 x 5 surrounding cells through LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "vp_device.hpp"
#include "vp_internal.hpp"

namespace vp {

namespace {

constexpr double kRefineCut = 12.0;  // slice support, in units of sqrt(delta_1)
constexpr int kRefineReach = 2;      // cells of edge kRefineCut sqrt(delta_1) / 2: scan 5 x 5
constexpr int kRefineThreads = 128;  // targets per workgroup (one cell's)

// Exponential integral E1(z), z > 0, in float64: the power series
// (Abramowitz & Stegun 5.1.11) for z <= 1.5, otherwise the continued fraction
// (A&S 5.1.22) by the modified Lentz method.
__device__ double e1(double z)
{
    const double EULER = 0.57721566490153286061;
    if (z <= 1.5) {
        double t = 1.0, sum = 0.0;
        for (int k = 1; k < 60; ++k) {
            t *= -z / k;
            const double d = t / k;
            sum += d;
            if (fabs(d) < 1e-17 * fabs(sum)) break;
        }
        return -EULER - log(z) - sum;
    }
    // E1(z) = e^-z / (z + 1 - 1^2 / (z + 3 - 2^2 / (z + 5 - ...)))
    const double tiny = 1e-300;
    double b = z + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int k = 1; k < 200; ++k) {
        const double a = -(double)k * k;
        b += 2.0;
        d = 1.0 / (a * d + b);
        c = b + a / c;
        const double del = c * d;
        h *= del;
        if (fabs(del - 1.0) < 1e-16) break;
    }
    return h * exp(-z);
}

struct RefineArgs {
    int n_units;
    const int4* units;         // (cell, first, end) of near targets, one cell's targets per unit
    const int* near;
    const double* near_x;
    const double* near_y;
    const double *fx, *fy, *fnx, *fny, *fw;
    const int* perm;
    const int* cell_start;
    int ncx, ncy;
    double delta1, delta_star;
    int64_t n_tgt;
    const double *r, *kappa, *g3, *g4;
    const int8_t* sgn;
    int order_s, order_d;
    const double* sj;          // [3][n_tgt] or NULL
    const double* fine_sigma;  // [n_fine] or NULL
    const double* mj;          // [5][n_tgt] or NULL
    const double* fine_mu;     // [n_fine] or NULL
    double* out;
};

// One workgroup per unit: its targets (one per thread) share the cell, so the
// nodes of the surrounding cells are staged once per workgroup through LDS
// (with strength times weight folded in) and read by all threads as broadcasts.
__global__ __launch_bounds__(kRefineThreads) void k_refine(RefineArgs a)
{
    __shared__ double sx[kRefineThreads], sy[kRefineThreads], snx[kRefineThreads], sny[kRefineThreads];
    __shared__ double ss[kRefineThreads], sm[kRefineThreads];
    const int4 u = a.units[blockIdx.x];
    const int t = u.y + (int)threadIdx.x;
    const bool on = t < u.z;
    int i = 0;
    double x = 0.0, y = 0.0;
    if (on) {
        i = a.near[t];
        x = a.near_x[t];
        y = a.near_y[t];
    }
    const double q1 = 0.25 / a.delta1, qs = 0.25 / a.delta_star;
    const double cut2 = kRefineCut * kRefineCut * a.delta1;
    const double ln_ratio = log(a.delta1 / a.delta_star);
    const int cx = u.x % a.ncx, cy = u.x / a.ncx;
    const bool use_s = a.fine_sigma != nullptr, use_d = a.fine_mu != nullptr;
    double acc_s = 0.0, acc_d = 0.0;
    for (int jy = max(cy - kRefineReach, 0); jy <= min(cy + kRefineReach, a.ncy - 1); ++jy) {
        // the row's cells cx - reach .. cx + reach are contiguous in cell order
        const int k0 = a.cell_start[jy * a.ncx + max(cx - kRefineReach, 0)];
        const int k1 = a.cell_start[jy * a.ncx + min(cx + kRefineReach, a.ncx - 1) + 1];
        for (int kb = k0; kb < k1; kb += kRefineThreads) {
            const int kl = kb + (int)threadIdx.x;
            __syncthreads();  // the previous chunk has been read
            if (kl < k1) {
                const int o = a.perm[kl];
                sx[threadIdx.x] = a.fx[kl];
                sy[threadIdx.x] = a.fy[kl];
                snx[threadIdx.x] = a.fnx[kl];
                sny[threadIdx.x] = a.fny[kl];
                ss[threadIdx.x] = use_s ? a.fw[kl] * a.fine_sigma[o] : 0.0;
                sm[threadIdx.x] = use_d ? a.fw[kl] * a.fine_mu[o] : 0.0;
            }
            __syncthreads();
            const int nk = min(kRefineThreads, k1 - kb);
            if (on) {
                for (int k = 0; k < nk; ++k) {
                    const double dx = x - sx[k], dy = y - sy[k];
                    const double rho2 = dx * dx + dy * dy;
                    if (rho2 >= cut2) continue;
                    // the delta* terms vanish (below 1e-17) once qs rho^2 > 40, i.e. for
                    // most pairs: rho > 12.6 sqrt(delta*)
                    const double zs = rho2 * qs;
                    if (use_s) {
                        double ks = ln_ratio;
                        if (rho2 > 0.0) ks = zs > 40.0 ? e1(rho2 * q1) : e1(rho2 * q1) - e1(zs);
                        acc_s += ks * ss[k];
                    }
                    if (use_d && rho2 > 0.0) {
                        // exp(-q1 rho^2) - exp(-qs rho^2) = -exp(-q1 rho^2) expm1(-(qs - q1) rho^2)
                        const double e = exp(-q1 * rho2);
                        const double diff = zs > 40.0 ? e : -e * expm1(-(qs - q1) * rho2);
                        acc_d += (snx[k] * dx + sny[k] * dy) / rho2 * diff * sm[k];
                    }
                }
            }
        }
    }
    if (!on) return;
    const double PI = 3.14159265358979323846;
    double corr = acc_s / (4.0 * PI) + acc_d / (2.0 * PI);
    const double r = a.r[i], kap = a.kappa[i], sg = (double)a.sgn[i];
    const double g3 = a.g3 ? a.g3[i] : 0.0, g4 = a.g4 ? a.g4[i] : 0.0;
    const int64_t n = a.n_tgt;
    if (a.sj) {
        const double s0 = a.sj[i], s1 = a.sj[n + i], s2 = a.sj[2 * n + i];
        corr += dev::s_local_value(a.delta_star, r, sg, kap, g3, g4, s0, s1, s2, a.order_s) -
                dev::s_local_value(a.delta1, r, sg, kap, g3, g4, s0, s1, s2, a.order_s);
    }
    if (a.mj) {
        const double m[5] = {a.mj[i], a.mj[n + i], a.mj[2 * n + i], a.mj[3 * n + i], a.mj[4 * n + i]};
        corr += dev::d_local_value(a.delta_star, r, sg, kap, g3, g4, m, a.order_d) -
                dev::d_local_value(a.delta1, r, sg, kap, g3, g4, m, a.order_d);
    }
    a.out[i] += corr;
}

vp_status rfail(vp_status s, const std::string& m) { return set_error(s, m); }

template <typename T>
vp_status dl(std::vector<T>& v, const T* src, int64_t n, const char* what)
{
    v.resize(n);
    if (n == 0) return VP_OK;
    if (!src) return rfail(VP_ERR_ARG, std::string(what) + " is NULL");
    if (hipMemcpy(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
        return rfail(VP_ERR_DEVICE, std::string("copy of ") + what);
    return VP_OK;
}

template <typename T>
vp_status ul(Refinement& r, T** dst, const std::vector<T>& v, const char* what)
{
    *dst = nullptr;
    if (v.empty()) return VP_OK;
    void* q = nullptr;
    if (hipMalloc(&q, v.size() * sizeof(T)) != hipSuccess) return rfail(VP_ERR_OOM, std::string("hipMalloc ") + what);
    r.allocs.push_back(q);
    if (hipMemcpy(q, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return rfail(VP_ERR_DEVICE, std::string("copy of ") + what);
    *dst = (T*)q;
    return VP_OK;
}

}  // namespace

void refinement_free(Refinement& r)
{
    for (void* q : r.allocs) hipFree(q);
    r = Refinement{};
}

}  // namespace vp

using namespace vp;

extern "C" {

vp_status vp_refine_attach(vp_plan_t p, int levels, int64_t n_fine, const double* fine_x, const double* fine_y,
                           const double* fine_nx, const double* fine_ny, const double* fine_w, const double* tgt_x,
                           const double* tgt_y)
{
    if (!p) return rfail(VP_ERR_ARG, "plan is NULL");
    if (levels < 1 || levels > 8) return rfail(VP_ERR_ARG, "levels must be in 1..8");
    if (n_fine < 1 || n_fine > (int64_t)1 << 30) return rfail(VP_ERR_ARG, "n_fine out of range");
    if (p->n_tgt > ((int64_t)1 << 31) - 1) return rfail(VP_ERR_ARG, "too many targets");
    if (p->stream) hipStreamSynchronize(p->stream);
    std::vector<double> x, y, nx, ny, w, tx, ty, r;
    vp_status s;
    if ((s = dl(x, fine_x, n_fine, "fine_x")) != VP_OK || (s = dl(y, fine_y, n_fine, "fine_y")) != VP_OK ||
        (s = dl(nx, fine_nx, n_fine, "fine_nx")) != VP_OK || (s = dl(ny, fine_ny, n_fine, "fine_ny")) != VP_OK ||
        (s = dl(w, fine_w, n_fine, "fine_w")) != VP_OK || (s = dl(tx, tgt_x, p->n_tgt, "tgt_x")) != VP_OK ||
        (s = dl(ty, tgt_y, p->n_tgt, "tgt_y")) != VP_OK || (s = dl(r, (const double*)p->g_r, p->n_tgt, "r")) != VP_OK)
        return s;
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int64_t k = 0; k < n_fine; ++k) {
        if (!std::isfinite(x[k]) || !std::isfinite(y[k]) || !std::isfinite(nx[k]) || !std::isfinite(ny[k]) ||
            !std::isfinite(w[k]) || w[k] < 0.0)
            return rfail(VP_ERR_ARG, "non-finite fine node data or negative weight");
        xmin = std::min(xmin, x[k]);
        xmax = std::max(xmax, x[k]);
        ymin = std::min(ymin, y[k]);
        ymax = std::max(ymax, y[k]);
    }
    Refinement R;
    R.levels = levels;
    R.delta_star = p->delta1 / std::pow(4.0, levels);
    R.n_fine = n_fine;
    R.cell = kRefineCut * std::sqrt(p->delta1) / kRefineReach;
    R.x0 = xmin;
    R.y0 = ymin;
    R.ncx = std::max(1, (int)std::ceil((xmax - xmin) / R.cell) + 1);
    R.ncy = std::max(1, (int)std::ceil((ymax - ymin) / R.cell) + 1);
    if ((double)R.ncx * R.ncy > 1e8) return rfail(VP_ERR_ARG, "fine boundary extent too large for its cell grid");
    auto cell_of = [&](double px, double py) {
        const int cx = std::min(std::max((int)std::floor((px - R.x0) / R.cell), 0), R.ncx - 1);
        const int cy = std::min(std::max((int)std::floor((py - R.y0) / R.cell), 0), R.ncy - 1);
        return cy * R.ncx + cx;
    };
    const int ncell = R.ncx * R.ncy;
    std::vector<int> start(ncell + 1, 0), order(n_fine);
    std::vector<int> cid(n_fine);
    for (int64_t k = 0; k < n_fine; ++k) {
        cid[k] = cell_of(x[k], y[k]);
        start[cid[k] + 1]++;
    }
    for (int c = 0; c < ncell; ++c) start[c + 1] += start[c];
    std::vector<int> pos(start.begin(), start.end() - 1);
    for (int64_t k = 0; k < n_fine; ++k) order[pos[cid[k]]++] = (int)k;
    std::vector<double> sx(n_fine), sy(n_fine), snx(n_fine), sny(n_fine), sw(n_fine);
    for (int64_t k = 0; k < n_fine; ++k) {
        const int o = order[k];
        sx[k] = x[o];
        sy[k] = y[o];
        snx[k] = nx[o];
        sny[k] = ny[o];
        sw[k] = w[o];
    }
    // targets within the slices' support of the boundary, in cell order
    const double cut = kRefineCut * std::sqrt(p->delta1);
    std::vector<int> near;
    for (int64_t i = 0; i < p->n_tgt; ++i) {
        if (!std::isfinite(tx[i]) || !std::isfinite(ty[i])) return rfail(VP_ERR_ARG, "non-finite target");
        if (r[i] <= cut) near.push_back((int)i);
    }
    std::vector<int> ncid(near.size());
    for (size_t t = 0; t < near.size(); ++t) ncid[t] = cell_of(tx[near[t]], ty[near[t]]);
    std::vector<size_t> ord(near.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return ncid[a] < ncid[b]; });
    std::vector<int> nsorted(near.size());
    std::vector<double> nxs(near.size()), nys(near.size());
    for (size_t t = 0; t < near.size(); ++t) {
        nsorted[t] = near[ord[t]];
        nxs[t] = tx[nsorted[t]];
        nys[t] = ty[nsorted[t]];
    }
    R.n_near = (int)nsorted.size();
    // work units: runs of at most kRefineThreads near targets of one cell
    std::vector<int4> units;
    for (size_t t = 0; t < nsorted.size();) {
        const int c = ncid[ord[t]];
        size_t e = t;
        while (e < nsorted.size() && ncid[ord[e]] == c && e - t < (size_t)kRefineThreads) ++e;
        units.push_back(make_int4(c, (int)t, (int)e, 0));
        t = e;
    }
    R.n_units = (int)units.size();
    if ((s = ul(R, &R.x, sx, "fine nodes")) != VP_OK || (s = ul(R, &R.y, sy, "fine nodes")) != VP_OK ||
        (s = ul(R, &R.nx, snx, "fine normals")) != VP_OK || (s = ul(R, &R.ny, sny, "fine normals")) != VP_OK ||
        (s = ul(R, &R.w, sw, "fine weights")) != VP_OK || (s = ul(R, &R.perm, order, "fine order")) != VP_OK ||
        (s = ul(R, &R.cell_start, start, "cells")) != VP_OK || (s = ul(R, &R.near, nsorted, "near targets")) != VP_OK ||
        (s = ul(R, &R.near_x, nxs, "near targets")) != VP_OK || (s = ul(R, &R.near_y, nys, "near targets")) != VP_OK ||
        (s = ul(R, &R.units, units, "refinement units")) != VP_OK) {
        refinement_free(R);
        return s;
    }
    refinement_free(p->ref);
    p->ref = R;
    return VP_OK;
}

vp_status vp_layer_refine(vp_plan_t p, const double* sigma_jet3, const double* fine_sigma, const double* mu_jet5,
                          const double* fine_mu, double* out)
{
    if (!p) return rfail(VP_ERR_ARG, "plan is NULL");
    if (p->ref.levels == 0) return rfail(VP_ERR_ARG, "no refinement attached (vp_refine_attach)");
    if ((sigma_jet3 == nullptr) != (fine_sigma == nullptr)) return rfail(VP_ERR_ARG, "sigma_jet3 and fine_sigma come together");
    if ((mu_jet5 == nullptr) != (fine_mu == nullptr)) return rfail(VP_ERR_ARG, "mu_jet5 and fine_mu come together");
    if (sigma_jet3 && !(p->kinds & VP_KIND_S)) return rfail(VP_ERR_ARG, "plan does not support S");
    if (mu_jet5 && !(p->kinds & VP_KIND_D)) return rfail(VP_ERR_ARG, "plan does not support D");
    if (!out && p->n_tgt) return rfail(VP_ERR_ARG, "out is NULL");
    if (!sigma_jet3 && !mu_jet5) return VP_OK;
    const Refinement& R = p->ref;
    if (R.n_near == 0) return VP_OK;
    RefineArgs a;
    a.n_units = R.n_units;
    a.units = R.units;
    a.near = R.near;
    a.near_x = R.near_x;
    a.near_y = R.near_y;
    a.fx = R.x;
    a.fy = R.y;
    a.fnx = R.nx;
    a.fny = R.ny;
    a.fw = R.w;
    a.perm = R.perm;
    a.cell_start = R.cell_start;
    a.ncx = R.ncx;
    a.ncy = R.ncy;
    a.delta1 = p->delta1;
    a.delta_star = R.delta_star;
    a.n_tgt = p->n_tgt;
    a.r = p->g_r;
    a.kappa = p->g_kappa;
    a.g3 = p->g_g3;
    a.g4 = p->g_g4;
    a.sgn = p->g_sgn;
    a.order_s = p->loc.order_s;
    a.order_d = p->loc.order_d;
    a.sj = sigma_jet3;
    a.fine_sigma = fine_sigma;
    a.mj = mu_jet5;
    a.fine_mu = fine_mu;
    a.out = out;
    hipLaunchKernelGGL(k_refine, dim3(R.n_units), dim3(kRefineThreads), 0, p->stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rfail(VP_ERR_DEVICE, std::string("refinement launch: ") + hipGetErrorString(e));
    return VP_OK;
}

}  // extern "C"
