// Host planner and C ABI (include/vp.h).
//
// The planner turns the paper's parameter choices (Sec. 2.2 and Sec. 3) into
// a concrete, alias-free discretization of the near- and far-history Fourier
// integrals:
//   delta_1 = c_delta * dx^2 (Sec. 6), delta_2 = ratio * delta_1;
//   k_max from k^p exp(-k^2 delta) < eps (p = 1 when the double layer is
//   present, Sec. 3, input of the history algorithm);
//   the trapezoid rule in k with spacing dk = 2 pi / P periodizes the kernel
//   with period P, so P is chosen from the geometry: P_NH >= E + R (E =
//   largest extent of nodes and targets, R = reach of the near-history
//   kernel), and for the far history the kernel is truncated at radius
//   L = D + R (D = diameter bound) as in the Vico-type truncation of the far-history lemma (Sec. 2),
//   with P_FH >= E + L + R;
//   the sums of Step 2 and Step 4 are evaluated by type-1 spreading and
//   type-2 interpolation on a fine grid F >= sigma * (2M+1) with the
//   exponential-of-semicircle kernel; its Fourier transform is tabulated by
//   Gauss-Legendre quadrature and divided out (squared) in the multiplier.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

namespace {

thread_local std::string g_last_error;

vp_status fail(vp_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

#define VP_HIP(call, what)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            return fail(e_ == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,                  \
                        std::string(what) + ": " + hipGetErrorString(e_));                       \
        }                                                                                        \
    } while (0)

// Neumaier-compensated sum.
double ksum(const double* a, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double t = s + a[i];
        if (std::fabs(s) >= std::fabs(a[i])) c += (s - t) + a[i];
        else c += (a[i] - t) + s;
        s = t;
    }
    return s + c;
}

bool all_finite(const std::vector<double>& v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

// Smallest k > 0 with k^p exp(-k^2 delta) <= eps (decreasing branch).
double kmax_for(double delta, double eps, int p)
{
    const double le = std::log(1.0 / eps);
    double k = std::sqrt(le / delta);
    for (int it = 0; it < 50; ++it) {
        const double kn = std::sqrt((le + p * std::log(std::max(k, 1.0))) / delta);
        if (std::fabs(kn - k) < 1e-12 * k) break;
        k = kn;
    }
    return k;
}

// Gauss-Legendre nodes/weights on [-1,1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                double q0 = 1.0, q1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
                    q0 = q1;
                    q1 = q2;
                }
                const double dq = n * (z * q1 - q0) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dq * dq);
                break;
            }
        }
    }
}

// Fourier transform of the spreading kernel phi(x) = exp(beta (sqrt(1-(2x/w)^2) - 1)),
// |x| < w/2 (grid units), at integer frequencies m of an F-periodic grid:
// phihat(m) = int phi(x) exp(-2 pi i m x / F) dx.
std::vector<double> kernel_ft(int w, double beta, int F, int M)
{
    std::vector<double> gx, gw;
    gauss_legendre(std::max(2 * w + 40, 80), gx, gw);
    std::vector<double> out(M + 1);
    for (int m = 0; m <= M; ++m) {
        double s = 0.0;
        for (size_t q = 0; q < gx.size(); ++q) {
            const double z = gx[q];
            const double phi = std::exp(beta * (std::sqrt(1.0 - z * z) - 1.0));
            const double x = 0.5 * w * z;
            s += gw[q] * phi * std::cos(2.0 * M_PI * m * x / F);
        }
        out[m] = 0.5 * w * s;
    }
    return out;
}

// Near-history multiplier (exp(-k^2 d1) - exp(-k^2 d2)) / k^2 (Lemma 2.1), k -> 0 limit d2 - d1.
double mult_nh(double k2, double d1, double d2)
{
    if (k2 * (d2 - d1) < 1e-8) return (d2 - d1) - 0.5 * k2 * (d2 * d2 - d1 * d1);
    return std::exp(-k2 * d1) * (-std::expm1(-k2 * (d2 - d1))) / k2;
}

// Far-history multiplier exp(-k^2 d2) W_L(k) with the truncated-kernel transform
// W_L(k) = (1 - J0(L k))/k^2 - L log L J1(L k)/k (far-history lemma of Sec. 2, with radius L);
// for small L k the Bessel quotients use their Taylor series (limit L^2 (1 - 2 log L)/4).
double mult_fh(double k2, double d2, double L)
{
    const double k = std::sqrt(k2);
    const double x = L * k;
    double a, b;  // a = (1 - J0(x))/x^2, b = J1(x)/x
    if (x < 1e-2) {
        const double x2 = x * x;
        a = 0.25 - x2 / 64.0 + x2 * x2 / 2304.0;
        b = 0.5 - x2 / 16.0 + x2 * x2 / 384.0;
    } else {
        a = (1.0 - j0(x)) / (x * x);
        b = j1(x) / x;
    }
    const double W = L * L * (a - std::log(L) * b);
    return std::exp(-k2 * d2) * W;
}

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

int spread_width_for(double eps, double sigma)
{
    // exponential-of-semicircle kernel: error ~ exp(-pi w sqrt(1 - 1/sigma))
    const double w = std::ceil(std::log(1.0 / eps) / (M_PI * std::sqrt(1.0 - 1.0 / sigma))) + 1.0;
    return (int)std::max(2.0, w);
}

struct HostPoints {
    std::vector<double> x, y;  // all spread sources: volume nodes then boundary nodes
};

template <typename T>
vp_status dalloc(Plan& p, T** ptr, size_t count, const char* what)
{
    *ptr = nullptr;
    if (count == 0) return VP_OK;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) return fail(VP_ERR_OOM, std::string("hipMalloc ") + what + ": " + hipGetErrorString(e));
    p.allocs.push_back(q);
    p.device_bytes += count * sizeof(T);
    *ptr = (T*)q;
    return VP_OK;
}

vp_status dalloc_bytes(Plan& p, void** ptr, size_t bytes, const char* what)
{
    unsigned char* q = nullptr;
    vp_status s = dalloc(p, &q, bytes, what);
    *ptr = q;
    return s;
}

template <typename T>
vp_status upload(Plan& p, T** dst, const std::vector<T>& src, const char* what)
{
    vp_status s = dalloc(p, dst, src.size(), what);
    if (s != VP_OK) return s;
    if (!src.empty()) VP_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), what);
    return VP_OK;
}

template <typename T>
vp_status download(std::vector<T>& dst, const T* src, int64_t n, const char* what)
{
    dst.resize(n);
    if (n == 0) return VP_OK;
    if (!src) return fail(VP_ERR_ARG, std::string(what) + " is NULL");
    VP_HIP(hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost), what);
    return VP_OK;
}

void free_plan(vp_plan_s* p)
{
    if (!p) return;
    if (p->stream) hipStreamSynchronize(p->stream);
    else hipDeviceSynchronize();
    for (void* q : p->allocs) hipFree(q);
    p->allocs.clear();
    workspace_free(p->ws, nullptr, false);
    if (p->ev_made)
        for (auto& e : p->ev) hipEventDestroy(e);
    delete p;
}

// Sort points into tiles of one level; spread=true gives one record per
// touched tile, spread=false one record per point (tile of its support corner).
template <typename R>
vp_status build_records(Plan& p, int l, const std::vector<double>& x, const std::vector<double>& y,
                        const std::vector<int>& ids, bool spread, RecList* list)
{
    const LevelGeom& g = p.lv[l];
    const int T = g.T, ntx = g.ntx, w = g.w;
    const int ntiles = ntx * ntx;
    const size_t n = ids.size();
    std::vector<int> i0(n), j0(n);
    std::vector<R> sx(n), sy(n);
    for (size_t q = 0; q < n; ++q) {
        const int k = ids[q];
        const double tx = (x[k] - g.x0) / g.h;
        const double ty = (y[k] - g.y0) / g.h;
        const double ax = std::ceil(tx - 0.5 * w);
        const double ay = std::ceil(ty - 0.5 * w);
        if (ax < 0 || ay < 0 || ax + w > g.F || ay + w > g.F)
            return fail(VP_ERR_INTERNAL, "support outside the fine grid (planner margin)");
        i0[q] = (int)ax;
        j0[q] = (int)ay;
        sx[q] = (R)(ax - tx + 0.5 * w);   // fractional offset in [0, 1)
        sy[q] = (R)(ay - ty + 0.5 * w);
    }
    std::vector<int> cnt(ntiles + 1, 0);
    auto tiles_of = [&](size_t q, int& ax0, int& ax1, int& ay0, int& ay1) {
        if (spread) {
            ax0 = i0[q] / T;
            ax1 = (i0[q] + w - 1) / T;
            ay0 = j0[q] / T;
            ay1 = (j0[q] + w - 1) / T;
        } else {
            ax0 = ax1 = i0[q] / T;
            ay0 = ay1 = j0[q] / T;
        }
    };
    for (size_t q = 0; q < n; ++q) {
        int ax0, ax1, ay0, ay1;
        tiles_of(q, ax0, ax1, ay0, ay1);
        for (int ty = ay0; ty <= ay1; ++ty)
            for (int tx = ax0; tx <= ax1; ++tx) cnt[ty * ntx + tx + 1]++;
    }
    for (int t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
    const int64_t nrec = cnt[ntiles];
    if (nrec > INT32_MAX) return fail(VP_ERR_ARG, "too many (node, tile) records");
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    std::vector<int> rij(nrec), ridx(nrec);
    std::vector<R> rsx(nrec), rsy(nrec);
    for (size_t q = 0; q < n; ++q) {
        int ax0, ax1, ay0, ay1;
        tiles_of(q, ax0, ax1, ay0, ay1);
        for (int ty = ay0; ty <= ay1; ++ty)
            for (int tx = ax0; tx <= ax1; ++tx) {
                const int at = pos[ty * ntx + tx]++;
                rij[at] = i0[q] | (j0[q] << 16);
                rsx[at] = sx[q];
                rsy[at] = sy[q];
                ridx[at] = ids[q];
            }
    }
    RecList* L = list;
    vp_status s;
    if ((s = upload(p, &L->start, cnt, "tile starts")) != VP_OK) return s;
    if ((s = upload(p, &L->ij, rij, "records ij")) != VP_OK) return s;
    if ((s = upload(p, (R**)&L->dx, rsx, "records dx")) != VP_OK) return s;
    if ((s = upload(p, (R**)&L->dy, rsy, "records dy")) != VP_OK) return s;
    if ((s = upload(p, &L->idx, ridx, "records idx")) != VP_OK) return s;
    L->n = nrec;
    return VP_OK;
}

template <typename R>
vp_status build_level_tables(Plan& p, int l, const std::vector<double>& phihat, double d1, double d2)
{
    LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    const int M = g.M;
    const double s = g.dk / (2.0 * M_PI);
    const double scale = s * s;
    std::vector<R> mult((size_t)(M + 1) * (M + 1));
    for (int a = 0; a <= M; ++a)
        for (int c = 0; c <= M; ++c) {
            const double k2 = g.dk * g.dk * ((double)a * a + (double)c * c);
            const double m = (l == 0) ? mult_nh(k2, d1, d2) : mult_fh(k2, d2, p.L);
            const double ph = phihat[a] * phihat[c];
            mult[(size_t)a * (M + 1) + c] = (R)(scale * m / (ph * ph));
        }
    g.dc_coef = scale * ((l == 0) ? mult_nh(0.0, d1, d2) : mult_fh(0.0, d2, p.L));
    // Spreading kernel per tap as a polynomial in the node offset: tap a of a
    // node with offset d in [0,1) sits at z = ((2a - w) + (u + 1)) / w, u = 2d - 1.
    // Chebyshev interpolation at w+2 points, converted to monomials in u.
    {
        const int W = g.w, P = W + 2;
        std::vector<double> coef((size_t)W * P);
        std::vector<double> cn(P), fv(P);
        for (int j = 0; j < P; ++j) cn[j] = std::cos(M_PI * (j + 0.5) / P);
        for (int a = 0; a < W; ++a) {
            for (int j = 0; j < P; ++j) {
                const double z = ((2.0 * a - W) + (cn[j] + 1.0)) / W;
                const double q = 1.0 - z * z;
                fv[j] = q > 0 ? std::exp(-g.beta * z * z / (1.0 + std::sqrt(q))) : 0.0;
            }
            // Chebyshev coefficients
            std::vector<double> ch(P);
            for (int k = 0; k < P; ++k) {
                double sacc = 0.0;
                for (int j = 0; j < P; ++j) sacc += fv[j] * std::cos(M_PI * k * (j + 0.5) / P);
                ch[k] = (k == 0 ? 1.0 : 2.0) * sacc / P;
            }
            // monomial coefficients: T_k(u) via the recurrence on coefficient vectors
            std::vector<double> mono(P, 0.0), tkm1(P, 0.0), tk(P, 0.0), tkp1(P, 0.0);
            tkm1[0] = 1.0;                     // T_0
            if (P > 1) tk[1] = 1.0;            // T_1
            for (int i = 0; i < P; ++i) mono[i] += ch[0] * tkm1[i];
            if (P > 1)
                for (int i = 0; i < P; ++i) mono[i] += ch[1] * tk[i];
            for (int k = 2; k < P; ++k) {
                for (int i = 0; i < P; ++i) tkp1[i] = -tkm1[i] + ((i > 0) ? 2.0 * tk[i - 1] : 0.0);
                for (int i = 0; i < P; ++i) mono[i] += ch[k] * tkp1[i];
                tkm1.swap(tk);
                tk.swap(tkp1);
            }
            for (int i = 0; i < P; ++i) coef[(size_t)a * P + i] = mono[i];
        }
        vp_status st2;
        if ((st2 = upload(p, &b.horner, coef, "kernel polynomials")) != VP_OK) return st2;
    }
    std::vector<cplx<R>> tw(g.F / 2);
    for (int k = 0; k < g.F / 2; ++k) {
        const double ang = -2.0 * M_PI * (double)k / g.F;
        tw[k] = {(R)std::cos(ang), (R)std::sin(ang)};
    }
    vp_status st;
    if ((st = upload(p, (R**)&b.mult, mult, "multiplier")) != VP_OK) return st;
    if ((st = upload(p, (cplx<R>**)&b.tw, tw, "twiddles")) != VP_OK) return st;
    return VP_OK;
}

template <typename R>
vp_status build_plan_t(Plan& p, const std::vector<double>& sxv, const std::vector<double>& syv,
                       const std::vector<int>& vol_ids, const std::vector<int>& bnd_ids, const std::vector<double>& tx,
                       const std::vector<double>& ty, const std::vector<std::vector<double>>& phihat)
{
    vp_status s;
    std::vector<int> tids(p.n_tgt);
    std::iota(tids.begin(), tids.end(), 0);
    for (int l = 0; l < 2; ++l) {
        LevelBufs& b = p.lb[l];
        if ((s = build_records<R>(p, l, sxv, syv, vol_ids, true, &b.vol)) != VP_OK) return s;
        if ((s = build_records<R>(p, l, sxv, syv, bnd_ids, true, &b.bnd)) != VP_OK) return s;
        if ((s = build_records<R>(p, l, tx, ty, tids, false, &b.tgt)) != VP_OK) return s;
        if ((s = build_level_tables<R>(p, l, phihat[l], p.delta1, p.delta2)) != VP_OK) return s;
    }
    return VP_OK;
}

}  // namespace

vp_status set_error(vp_status s, const std::string& msg) { return fail(s, msg); }

// Workspace layout: grid, spec, spec2, hist per level, then strengths and dc,
// each 256-byte aligned inside one allocation.
static size_t workspace_layout(const Plan& p, Workspace* ws, unsigned char* base)
{
    const size_t rb = p.precision == VP_FP32 ? sizeof(float) : sizeof(double);
    size_t off = 0;
    auto take = [&](void** slot, size_t bytes) {
        if (slot) *slot = base ? base + off : nullptr;
        off += align256(std::max<size_t>(bytes, 1));
    };
    for (int l = 0; l < 2; ++l) {
        const LevelGeom& g = p.lv[l];
        const size_t F = g.F, M1 = g.M + 1;
        take(ws ? &ws->grid[l] : nullptr, (size_t)p.cmax * F * F * rb);
        take(ws ? &ws->spec[l] : nullptr, (size_t)p.cmax * M1 * F * 2 * rb);
        take(ws ? &ws->spec2[l] : nullptr, M1 * F * 2 * rb);
        take(ws ? &ws->hist[l] : nullptr, (size_t)std::max<int64_t>(p.n_tgt, 1) * rb);
    }
    take(ws ? &ws->str : nullptr, (size_t)p.cmax * std::max<int64_t>(p.n_src + p.n_bnd, 1) * rb);
    void* dcp = nullptr;
    take(ws ? &dcp : nullptr, sizeof(double));
    if (ws) ws->dc = (double*)dcp;
    return off;
}

size_t workspace_bytes(const Plan& p) { return workspace_layout(p, nullptr, nullptr); }

hipError_t workspace_alloc(const Plan& p, Workspace& ws, hipStream_t st, bool async)
{
    const size_t bytes = workspace_bytes(p);
    void* blk = nullptr;
    hipError_t e = async ? hipMallocAsync(&blk, bytes, st) : hipMalloc(&blk, bytes);
    if (e != hipSuccess) return e;
    ws = Workspace{};
    ws.block = blk;
    ws.bytes = bytes;
    workspace_layout(p, &ws, (unsigned char*)blk);
    return hipSuccess;
}

hipError_t workspace_free(Workspace& ws, hipStream_t st, bool async)
{
    hipError_t e = hipSuccess;
    if (ws.block) e = async ? hipFreeAsync(ws.block, st) : hipFree(ws.block);
    ws = Workspace{};
    return e;
}

vp_status eval_enqueue(Plan& p, const Workspace& ws, hipStream_t st, const double* f, const double* jet6,
                       const double* sigma, const double* sigma_jet3, const double* mu, const double* mu_jet5,
                       double* out, bool timing)
{
    if (!out && p.n_tgt) return fail(VP_ERR_ARG, "out is NULL");
    const bool use_v = f != nullptr;
    const bool use_s = sigma != nullptr;
    const bool use_d = mu != nullptr;
    if (!use_v && !use_s && !use_d) return fail(VP_ERR_ARG, "no density given");
    if (use_v && !(p.kinds & VP_KIND_V)) return fail(VP_ERR_ARG, "plan does not support V");
    if (use_s && !(p.kinds & VP_KIND_S)) return fail(VP_ERR_ARG, "plan does not support S");
    if (use_d && !(p.kinds & VP_KIND_D)) return fail(VP_ERR_ARG, "plan does not support D");
    if (use_v && !jet6) return fail(VP_ERR_ARG, "jet6 is required with f");
    if (use_s && !sigma_jet3) return fail(VP_ERR_ARG, "sigma_jet3 is required with sigma");
    if (use_d && !mu_jet5) return fail(VP_ERR_ARG, "mu_jet5 is required with mu");
    if (!ws.block) return fail(VP_ERR_ARG, "no workspace");
    const int C = use_d ? 3 : 1;
    if (timing && !p.ev_made) {
        for (auto& e : p.ev) VP_HIP(hipEventCreate(&e), "event create");
        p.ev_made = true;
    }
    auto mark = [&](int k) -> hipError_t { return timing ? hipEventRecord(p.ev[k], st) : hipSuccess; };
    VP_HIP(mark(0), "event");
    VP_HIP(launch_zero_dc(p, ws, st), "zero dc");
    VP_HIP(launch_strengths(p, ws, st, f, sigma, mu, C), "strengths");
    VP_HIP(mark(1), "event");
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_spread(p, ws, st, l, C, use_v, use_s || use_d), "spread");
        VP_HIP(mark(2 + l), "event");
    }
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_row_fft(p, ws, st, l, C), "row fft");
        VP_HIP(mark(4 + l), "event");
    }
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_col_fft(p, ws, st, l, C), "column fft");
        VP_HIP(mark(6 + l), "event");
    }
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_row_ifft(p, ws, st, l), "row ifft");
        VP_HIP(mark(8 + l), "event");
    }
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_interp(p, ws, st, l), "interp");
        VP_HIP(mark(10 + l), "event");
    }
    VP_HIP(launch_local(p, ws, st, jet6, sigma_jet3, mu_jet5, use_v, use_s, use_d, out), "local");
    VP_HIP(mark(12), "event");
    return VP_OK;
}

}  // namespace vp

using namespace vp;

extern "C" {

void vp_opts_default(vp_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->precision = VP_FP64;
    o->c_delta = 3.0;
    o->delta_ratio = 32.0;
    o->order_v = 4;
    o->order_s = 3;
    o->order_d = 3;
    o->kinds = VP_KIND_V | VP_KIND_S | VP_KIND_D;
    o->no_workspace = 0;
}

const char* vp_last_error(void) { return g_last_error.c_str(); }

vp_status vp_plan(vp_plan_t* out, int64_t n_src, const double* src_x, const double* src_y, const double* src_w,
                  int64_t n_bnd, const double* bnd_x, const double* bnd_y, const double* bnd_nx,
                  const double* bnd_ny, const double* bnd_w, int64_t n_tgt, const double* tgt_x,
                  const double* tgt_y, const vp_local_geom* geom, const vp_opts* opts_in)
{
    g_last_error.clear();
    if (!out) return fail(VP_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_src < 0 || n_bnd < 0 || n_tgt < 0) return fail(VP_ERR_ARG, "negative count");
    if (n_src + n_bnd + n_tgt > (int64_t)INT32_MAX) return fail(VP_ERR_ARG, "too many points (int32 indices)");
    if (n_tgt > 0 && !geom) return fail(VP_ERR_ARG, "geom is NULL");
    vp_opts o;
    if (opts_in) o = *opts_in;
    else vp_opts_default(&o);
    if (!(o.tol > 0 && o.tol < 1)) return fail(VP_ERR_ARG, "tol must be in (0,1)");
    if (o.precision != VP_FP32 && o.precision != VP_FP64) return fail(VP_ERR_ARG, "bad precision");
    if (!(o.c_delta > 0) || !(o.delta_ratio > 1)) return fail(VP_ERR_ARG, "c_delta > 0 and delta_ratio > 1 required");
    if (o.order_v < 0 || o.order_v > 4 || o.order_s < 0 || o.order_s > 4 || o.order_d < 0 || o.order_d > 4)
        return fail(VP_ERR_ARG, "local orders must be in 0..4");
    if (o.kinds & ~7) return fail(VP_ERR_ARG, "bad kinds mask");
    if ((o.kinds & VP_KIND_V) && n_src == 0) o.kinds &= ~VP_KIND_V;
    if ((o.kinds & (VP_KIND_S | VP_KIND_D)) && n_bnd == 0) o.kinds &= ~(VP_KIND_S | VP_KIND_D);
    if (o.kinds == 0) return fail(VP_ERR_ARG, "no potential kind has nodes");

    vp_plan_s* p = new (std::nothrow) vp_plan_s();
    if (!p) return fail(VP_ERR_OOM, "host allocation");
    p->opts = o;
    p->precision = o.precision;
    p->kinds = o.kinds;
    p->n_src = n_src;
    p->n_bnd = n_bnd;
    p->n_tgt = n_tgt;
    p->stream = (hipStream_t)o.stream;
    p->loc = {0.0, o.order_v, o.order_s, o.order_d};

    auto bail = [&](vp_status s) {
        free_plan(p);
        return s;
    };
    if (p->stream) {
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return bail(fail(VP_ERR_DEVICE, std::string("stream sync: ") + hipGetErrorString(e)));
    }

    // ---- inputs to the host
    std::vector<double> sx, sy, sw, bx, by, bnx, bny, bw, tx, ty;
    std::vector<double> gr, gnx, gny, gk, g3, g4;
    std::vector<int8_t> gs;
    vp_status s;
#define DL(v, ptr, n, name)                                            \
    if ((s = download(v, ptr, n, name)) != VP_OK) return bail(s);
    DL(sx, src_x, n_src, "src_x");
    DL(sy, src_y, n_src, "src_y");
    DL(sw, src_w, n_src, "src_w");
    const bool need_b = (o.kinds & (VP_KIND_S | VP_KIND_D)) != 0;
    DL(bx, bnd_x, need_b ? n_bnd : 0, "bnd_x");
    DL(by, bnd_y, need_b ? n_bnd : 0, "bnd_y");
    DL(bnx, bnd_nx, need_b ? n_bnd : 0, "bnd_nx");
    DL(bny, bnd_ny, need_b ? n_bnd : 0, "bnd_ny");
    DL(bw, bnd_w, need_b ? n_bnd : 0, "bnd_w");
    DL(tx, tgt_x, n_tgt, "tgt_x");
    DL(ty, tgt_y, n_tgt, "tgt_y");
    if (n_tgt) {
        DL(gr, geom->r, n_tgt, "geom.r");
        DL(gnx, geom->nx, n_tgt, "geom.nx");
        DL(gny, geom->ny, n_tgt, "geom.ny");
        DL(gk, geom->kappa, n_tgt, "geom.kappa");
        if (geom->gamma3) DL(g3, geom->gamma3, n_tgt, "geom.gamma3");
        if (geom->gamma4) DL(g4, geom->gamma4, n_tgt, "geom.gamma4");
        if ((s = download(gs, geom->sgn, n_tgt, "geom.sgn")) != VP_OK) return bail(s);
    }
#undef DL
    if (!need_b) p->n_bnd = 0;
    for (auto* v : {&sx, &sy, &sw, &bx, &by, &bnx, &bny, &bw, &tx, &ty, &gr, &gnx, &gny, &gk, &g3, &g4})
        if (!all_finite(*v)) return bail(fail(VP_ERR_ARG, "non-finite input value"));
    for (double v : sw)
        if (v < 0) return bail(fail(VP_ERR_ARG, "negative volume weight"));
    for (double v : bw)
        if (v < 0) return bail(fail(VP_ERR_ARG, "negative boundary weight"));
    for (double v : gr)
        if (v < 0) return bail(fail(VP_ERR_ARG, "negative target distance r"));
    for (int8_t v : gs)
        if (v < -1 || v > 1) return bail(fail(VP_ERR_ARG, "sgn must be -1, 0 or +1"));

    // ---- delta_1 (Sec. 6: delta = 3 dx^2, dx^2 = sum w / N)
    double dx2;
    if (p->n_src > 0 && (o.kinds & VP_KIND_V)) dx2 = ksum(sw.data(), n_src) / (double)n_src;
    else if (p->n_src > 0) dx2 = ksum(sw.data(), n_src) / (double)n_src;
    else {
        const double mb = ksum(bw.data(), p->n_bnd) / (double)p->n_bnd;
        dx2 = mb * mb;
    }
    if (!(dx2 > 0)) return bail(fail(VP_ERR_ARG, "zero total weight"));
    p->delta1 = o.c_delta * dx2;
    p->delta2 = o.delta_ratio * p->delta1;
    p->loc.delta = p->delta1;
    const double sd1 = std::sqrt(p->delta1);
    if ((o.kinds & VP_KIND_V) && n_tgt)
        for (int64_t i = 0; i < n_tgt; ++i)
            if (gs[i] < 0 && gr[i] <= 12.0 * sd1)
                return bail(fail(VP_ERR_GEOMETRY, "exterior target near the boundary with the volume kind"));

    // ---- geometry: bounding box, extent, diameter bound
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    auto box = [&](const std::vector<double>& X, const std::vector<double>& Y) {
        for (size_t i = 0; i < X.size(); ++i) {
            xmin = std::min(xmin, X[i]);
            xmax = std::max(xmax, X[i]);
            ymin = std::min(ymin, Y[i]);
            ymax = std::max(ymax, Y[i]);
        }
    };
    if (o.kinds & VP_KIND_V) box(sx, sy);
    if (need_b) box(bx, by);
    box(tx, ty);
    const double cx = 0.5 * (xmin + xmax), cy = 0.5 * (ymin + ymax);
    const double E = std::max({xmax - xmin, ymax - ymin, 1e-3 * sd1, 1e-12});
    // diameter bound: max width over 32 directions, divided by cos(pi/64)
    double D = 0.0;
    {
        const int nd = 32;
        std::vector<double> lo(nd, INFINITY), hi(nd, -INFINITY), cs(nd), sn(nd);
        for (int d = 0; d < nd; ++d) {
            cs[d] = std::cos(M_PI * d / nd);
            sn[d] = std::sin(M_PI * d / nd);
        }
        auto scan = [&](const std::vector<double>& X, const std::vector<double>& Y) {
            for (size_t i = 0; i < X.size(); ++i)
                for (int d = 0; d < nd; ++d) {
                    const double v = (X[i] - cx) * cs[d] + (Y[i] - cy) * sn[d];
                    lo[d] = std::min(lo[d], v);
                    hi[d] = std::max(hi[d], v);
                }
        };
        if (o.kinds & VP_KIND_V) scan(sx, sy);
        if (need_b) scan(bx, by);
        scan(tx, ty);
        for (int d = 0; d < nd; ++d) D = std::max(D, hi[d] - lo[d]);
        D = std::min(D / std::cos(M_PI / (2 * nd)), std::hypot(xmax - xmin, ymax - ymin));
        D = std::max(D, E);
    }

    // ---- history tolerance and reaches
    p->eps = std::max(o.tol * 0.05, 1e-15);
    const double le = std::log(1.0 / p->eps);
    const double R = 2.0 * std::sqrt(p->delta2 * le);
    p->L = D + R;
    const int pk = (o.kinds & VP_KIND_D) ? 1 : 0;
    const double kmax[2] = {kmax_for(p->delta1, p->eps, pk),
                            kmax_for(p->delta2, p->eps / std::max(1.0, p->L * p->L), pk)};
    double period[2] = {E + R, E + p->L + R};
    const int Cmax = (o.kinds & VP_KIND_D) ? 3 : 1;
    const int64_t n_pts = ((o.kinds & VP_KIND_V) ? n_src : 0) + (need_b ? n_bnd : 0);
    const int Fmax = (o.precision == VP_FP32) ? 8192 : 4096;
    std::vector<std::vector<double>> phihat(2);
    for (int l = 0; l < 2; ++l) {
        LevelGeom& g = p->lv[l];
        const double eps_s = p->eps * 0.1;
        int bestF = 0, bestw = 0, bestM = 0;
        double bestP = 0, bestcost = INFINITY;
        for (int attempt = 0; attempt < 4 && bestF == 0; ++attempt) {
            const double P = period[l] * (1.0 + 0.02 * attempt);
            const double dk = 2.0 * M_PI / P;
            const int M = (int)std::ceil(kmax[l] / dk);
            const int nmodes = 2 * M + 1;
            int F0 = 64;
            while (F0 < (int)std::ceil(1.2 * nmodes)) F0 *= 2;
            const int Flim = o.spread_width[l] > 0 ? Fmax : std::min(4 * F0, Fmax);
            for (int F = F0; F <= Flim; F *= 2) {
                if (o.fine_grid[l] > 0 && F != o.fine_grid[l]) continue;
                const double sigma = (double)F / (double)nmodes;
                const int w_req = std::max(spread_width_for(eps_s, sigma), kWMin);
                // a forced width is accepted only on grids fine enough for it to meet the tolerance
                if (o.spread_width[l] > 0 && w_req > o.spread_width[l]) continue;
                const int w = o.spread_width[l] > 0 ? o.spread_width[l] : w_req;
                if (w > kWMax) continue;
                const double h = P / F;
                // keep every support inside the grid without wrap-around
                if ((P - E) * 0.5 < (0.5 * w + 2.0) * h) continue;
                const double cost = (double)F * F * Cmax * 12.0 + (double)n_pts * w * w * 1.5 +
                                    (double)n_tgt * w * w * 1.0;
                if (cost < bestcost) {
                    bestcost = cost;
                    bestF = F;
                    bestw = w;
                    bestM = M;
                    bestP = P;
                }
            }
        }
        if (bestF == 0)
            return bail(fail(VP_ERR_TOL, "no supported fine grid meets the tolerance (level " + std::to_string(l) +
                                             ")"));
        g.F = bestF;
        g.logF = ilog2(bestF);
        g.M = bestM;
        g.w = bestw;
        g.period = bestP;
        g.dk = 2.0 * M_PI / bestP;
        g.h = bestP / bestF;
        g.x0 = cx - 0.5 * bestP;
        g.y0 = cy - 0.5 * bestP;
        const double sigma = (double)bestF / (2.0 * bestM + 1.0);
        g.beta = 0.97 * M_PI * bestw * (1.0 - 0.5 / sigma);
        int T = o.tile > 0 ? o.tile : 32;
        while (T > bestF) T /= 2;
        if (bestF % T) return bail(fail(VP_ERR_ARG, "tile must divide the fine grid"));
        g.T = T;
        g.ntx = bestF / T;
        phihat[l] = kernel_ft(bestw, g.beta, bestF, bestM);
        for (double v : phihat[l])
            if (!(v > 0)) return bail(fail(VP_ERR_INTERNAL, "spreading kernel transform not positive"));
    }

    // ---- spread sources: volume nodes then boundary nodes
    std::vector<double> ax(sx), ay(sy);
    ax.insert(ax.end(), bx.begin(), bx.end());
    ay.insert(ay.end(), by.begin(), by.end());
    std::vector<int> vol_ids, bnd_ids;
    if (o.kinds & VP_KIND_V)
        for (int64_t i = 0; i < n_src; ++i) vol_ids.push_back((int)i);
    if (need_b)
        for (int64_t j = 0; j < p->n_bnd; ++j) bnd_ids.push_back((int)(n_src + j));

    // ---- device node data
    std::vector<double> wall(sw);
    wall.insert(wall.end(), bw.begin(), bw.end());
    if (wall.empty()) wall.push_back(0.0);
    if ((s = upload(*p, &p->d_w, wall, "weights")) != VP_OK) return bail(s);
    if (need_b) {
        if ((s = upload(*p, &p->d_nx, bnx, "normals")) != VP_OK) return bail(s);
        if ((s = upload(*p, &p->d_ny, bny, "normals")) != VP_OK) return bail(s);
    }
    if (n_tgt) {
        if ((s = upload(*p, &p->g_r, gr, "geom")) != VP_OK) return bail(s);
        if ((s = upload(*p, &p->g_nx, gnx, "geom")) != VP_OK) return bail(s);
        if ((s = upload(*p, &p->g_ny, gny, "geom")) != VP_OK) return bail(s);
        if ((s = upload(*p, &p->g_kappa, gk, "geom")) != VP_OK) return bail(s);
        if (!g3.empty() && (s = upload(*p, &p->g_g3, g3, "geom")) != VP_OK) return bail(s);
        if (!g4.empty() && (s = upload(*p, &p->g_g4, g4, "geom")) != VP_OK) return bail(s);
        if ((s = upload(*p, &p->g_sgn, gs, "geom")) != VP_OK) return bail(s);
    }
    s = (o.precision == VP_FP32) ? build_plan_t<float>(*p, ax, ay, vol_ids, bnd_ids, tx, ty, phihat)
                                 : build_plan_t<double>(*p, ax, ay, vol_ids, bnd_ids, tx, ty, phihat);
    if (s != VP_OK) return bail(s);
    p->cmax = Cmax;
    if (!o.no_workspace) {
        hipError_t e = workspace_alloc(*p, p->ws, p->stream, false);
        if (e != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,
                             std::string("workspace: ") + hipGetErrorString(e)));
        p->device_bytes += p->ws.bytes;
    }
    for (int l = 0; l < 2; ++l) {
        const size_t lds_row = row_fft_lds_bytes(*p, l), lds_col = col_fft_lds_bytes(*p, l);
        const size_t lds_sp = spread_lds_bytes(*p, l, Cmax, need_b);
        if (lds_row > 160 * 1024 || lds_col > 160 * 1024 || lds_sp > 160 * 1024)
            return bail(fail(VP_ERR_TOL, "working set too large for LDS"));
    }
    *out = p;
    return VP_OK;
}

vp_status vp_eval(vp_plan_t p, const double* f, const double* jet6, const double* sigma, const double* sigma_jet3,
                  const double* mu, const double* mu_jet5, double* out)
{
    g_last_error.clear();
    if (!p) return fail(VP_ERR_ARG, "plan is NULL");
    if (p->ws.block) return eval_enqueue(*p, p->ws, p->stream, f, jet6, sigma, sigma_jet3, mu, mu_jet5, out, p->timing);
    // plan without its own workspace: a stream-ordered temporary one
    Workspace ws;
    hipError_t e = workspace_alloc(*p, ws, p->stream, true);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,
                    std::string("workspace: ") + hipGetErrorString(e));
    vp_status s = eval_enqueue(*p, ws, p->stream, f, jet6, sigma, sigma_jet3, mu, mu_jet5, out, p->timing);
    workspace_free(ws, p->stream, true);
    return s;
}

vp_status vp_volume(vp_plan_t p, const double* f, const double* jet6, double* out)
{
    return vp_eval(p, f, jet6, nullptr, nullptr, nullptr, nullptr, out);
}

vp_status vp_layer(vp_plan_t p, const double* sigma, const double* sigma_jet3, const double* mu,
                   const double* mu_jet5, double* out)
{
    return vp_eval(p, nullptr, nullptr, sigma, sigma_jet3, mu, mu_jet5, out);
}

vp_status vp_destroy(vp_plan_t p)
{
    g_last_error.clear();
    free_plan(p);
    return VP_OK;
}

vp_status vp_get_plan_info(vp_plan_t p, vp_plan_info* info)
{
    if (!p || !info) return fail(VP_ERR_ARG, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->delta1 = p->delta1;
    info->delta2 = p->delta2;
    info->eps_hist = p->eps;
    info->trunc_L = p->L;
    for (int l = 0; l < 2; ++l) {
        info->period[l] = p->lv[l].period;
        info->kmax[l] = p->lv[l].M * p->lv[l].dk;
        info->modes[l] = 2 * p->lv[l].M + 1;
        info->fine[l] = p->lv[l].F;
        info->width[l] = p->lv[l].w;
        info->spread_records[l] = p->lb[l].vol.n + p->lb[l].bnd.n;
    }
    info->tile = p->lv[0].T;
    info->precision = p->precision;
    info->n_src = p->n_src;
    info->n_bnd = p->n_bnd;
    info->n_tgt = p->n_tgt;
    info->device_bytes = p->device_bytes;
    info->workspace_bytes = workspace_bytes(*p);
    return VP_OK;
}

vp_status vp_set_timing(vp_plan_t p, int enable)
{
    if (!p) return fail(VP_ERR_ARG, "plan is NULL");
    p->timing = enable != 0;
    return VP_OK;
}

vp_status vp_get_timing(vp_plan_t p, double* ms)
{
    if (!p || !ms) return fail(VP_ERR_ARG, "NULL argument");
    if (!p->ev_made) return fail(VP_ERR_ARG, "timing was not enabled before the last evaluation");
    VP_HIP(hipEventSynchronize(p->ev[kTimedLaunches]), "event sync");
    for (int k = 0; k < kTimedLaunches; ++k) {
        float t = 0;
        VP_HIP(hipEventElapsedTime(&t, p->ev[k], p->ev[k + 1]), "elapsed");
        ms[k] = t;
    }
    float tot = 0;
    VP_HIP(hipEventElapsedTime(&tot, p->ev[0], p->ev[kTimedLaunches]), "elapsed");
    ms[kTimedLaunches] = tot;
    return VP_OK;
}

}  // extern "C"
