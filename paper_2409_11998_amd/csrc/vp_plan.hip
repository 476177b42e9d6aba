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
#include <thread>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

namespace {

thread_local std::string g_last_error;

// Host loops over millions of points or thousands of tiles run on up to
// kHostParts threads, each on its own contiguous range [b, e) of [0, n) (no
// shared writes); ranges shorter than grain stay on the calling thread.
// parallel_parts also passes the range's index k < kHostParts, so that each
// range can keep a partial result in a slot of its own.
constexpr int kHostParts = 16;

template <typename Fn>
void parallel_parts(int64_t n, int64_t grain, Fn&& fn)
{
    const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t nt =
        std::min<int64_t>(std::min<int64_t>(hw, kHostParts), (n + grain - 1) / std::max<int64_t>(grain, 1));
    if (nt <= 1) {
        fn(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int64_t k = 0; k < nt; ++k) th.emplace_back([&fn, n, nt, k] { fn((int)k, n * k / nt, n * (k + 1) / nt); });
    for (auto& t : th) t.join();
}

template <typename Fn>
void parallel_ranges(int64_t n, int64_t grain, Fn&& fn)
{
    parallel_parts(n, grain, [&fn](int, int64_t b, int64_t e) { fn(b, e); });
}

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

// true if pred holds for some element (ranges on host threads)
template <typename T, typename Pred>
bool any_parallel(const std::vector<T>& v, Pred pred)
{
    std::vector<char> hit(kHostParts, 0);
    parallel_parts((int64_t)v.size(), 1 << 18, [&](int k, int64_t b, int64_t e) {
        bool h = false;
        for (int64_t i = b; i < e && !h; ++i) h = pred(v[i]);
        hit[k] = h;
    });
    for (char c : hit)
        if (c) return true;
    return false;
}

bool all_finite(const std::vector<double>& v)
{
    return !any_parallel(v, [](double x) { return !std::isfinite(x); });
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
    refinement_free(p->ref);
    workspace_free(p->ws, nullptr, false);
    if (p->solve_ws) hipFree(p->solve_ws);
    if (p->solve_host) hipHostFree(p->solve_host);
    if (p->solve_ev_made)
        for (auto& e : p->solve_ev) hipEventDestroy(e);
    if (p->ev_made)
        for (auto& e : p->ev) hipEventDestroy(e);
    if (p->side_made) {
        hipStreamSynchronize(p->side);
        for (auto& e : p->fork) hipEventDestroy(e);
        hipStreamDestroy(p->side);
    }
    delete p;
}

// Sort points into tiles of one level: one record per point, in the tile
// holding its support corner.  With pitch > 0 (interpolation targets) the
// records of each tile are ordered in chunks of 32 with distinct residues of
// their window offset (j0 - gy0) * pitch + (i0 - gx0) modulo 32 wherever the
// tile allows, so that the 32 targets a wavefront handles together read 32
// different LDS banks.
// Host arrays of record building, kept across the builds of one vp_plan call
// (the autotuner builds a level once per candidate): reusing them saves
// allocating and first-touching hundreds of MB per build.  Released when the
// call returns (ScratchRelease in vp_plan).
template <typename R>
struct RecScratch {
    std::vector<int> i0, j0, rij, ridx, rij2, ridx2, hist;
    std::vector<R> sx, sy, rsx, rsy, rsx2, rsy2;
};
template <typename R>
RecScratch<R>& rec_scratch()
{
    thread_local RecScratch<R> s;
    return s;
}
struct ScratchRelease {
    ~ScratchRelease()
    {
        rec_scratch<float>() = RecScratch<float>();
        rec_scratch<double>() = RecScratch<double>();
    }
};

template <typename R>
vp_status build_records(Plan& p, int l, const std::vector<double>& x, const std::vector<double>& y,
                        const std::vector<int>& ids, RecList* list, int pitch = 0, int tile = 0)
{
    const LevelGeom& g = p.lv[l];
    const int T = tile > 0 ? tile : g.T, ntx = g.F / T, w = g.w;
    const int ntiles = ntx * ntx;
    const size_t n = ids.size();
    RecScratch<R>& S = rec_scratch<R>();
    std::vector<int>& i0 = S.i0;
    std::vector<int>& j0 = S.j0;
    std::vector<R>& sx = S.sx;
    std::vector<R>& sy = S.sy;
    i0.resize(n);
    j0.resize(n);
    sx.resize(n);
    sy.resize(n);
    std::vector<char> outside(kHostParts, 0);  // per range: a support left the grid
    parallel_parts((int64_t)n, 1 << 16, [&](int part, int64_t b, int64_t e) {
        bool out = false;
        for (int64_t q = b; q < e; ++q) {
            const int k = ids[q];
            const double tx = (x[k] - g.x0) / g.h;
            const double ty = (y[k] - g.y0) / g.h;
            const double ax = std::ceil(tx - 0.5 * w);
            const double ay = std::ceil(ty - 0.5 * w);
            if (ax < 0 || ay < 0 || ax + w > g.F || ay + w > g.F) {
                out = true;
                continue;
            }
            i0[q] = (int)ax;
            j0[q] = (int)ay;
            sx[q] = (R)(ax - tx + 0.5 * w);   // fractional offset in [0, 1)
            sy[q] = (R)(ay - ty + 0.5 * w);
        }
        outside[part] = out;
    });
    for (char c : outside)
        if (c) return fail(VP_ERR_INTERNAL, "support outside the fine grid (planner margin)");
    // counting sort by tile in 16 point ranges: per-range counts, then each
    // range places its points after the earlier ranges' points of the same tile
    // (the order within a tile is the points' order, as a sequential pass gives)
    constexpr int NR = 16;
    const bool split = n >= ((size_t)1 << 16);
    const int nr = split ? NR : 1;
    auto rng_of = [&](int r, int64_t& b, int64_t& e) {
        b = (int64_t)n * r / nr;
        e = (int64_t)n * (r + 1) / nr;
    };
    std::vector<int>& hist = S.hist;
    hist.assign((size_t)nr * ntiles, 0);
    auto tile_of = [&](int64_t q) { return (j0[q] / T) * ntx + i0[q] / T; };
    parallel_ranges(nr, 1, [&](int64_t rb, int64_t re) {
        for (int64_t r = rb; r < re; ++r) {
            int64_t b, e;
            rng_of((int)r, b, e);
            int* h = &hist[(size_t)r * ntiles];
            for (int64_t q = b; q < e; ++q) h[tile_of(q)]++;
        }
    });
    std::vector<int> cnt(ntiles + 1, 0);
    for (int t = 0; t < ntiles; ++t) {
        int c = 0;
        for (int r = 0; r < nr; ++r) c += hist[(size_t)r * ntiles + t];
        cnt[t + 1] = cnt[t] + c;
    }
    const int64_t nrec = cnt[ntiles];
    if (nrec > INT32_MAX) return fail(VP_ERR_ARG, "too many (node, tile) records");
    for (int t = 0; t < ntiles; ++t) {  // hist becomes each range's first position in each tile
        int at = cnt[t];
        for (int r = 0; r < nr; ++r) {
            const int c = hist[(size_t)r * ntiles + t];
            hist[(size_t)r * ntiles + t] = at;
            at += c;
        }
    }
    std::vector<int>& rij = S.rij;
    std::vector<int>& ridx = S.ridx;
    std::vector<R>& rsx = S.rsx;
    std::vector<R>& rsy = S.rsy;
    rij.resize(nrec);
    ridx.resize(nrec);
    rsx.resize(nrec);
    rsy.resize(nrec);
    parallel_ranges(nr, 1, [&](int64_t rb, int64_t re) {
        for (int64_t r = rb; r < re; ++r) {
            int64_t b, e;
            rng_of((int)r, b, e);
            int* pos = &hist[(size_t)r * ntiles];
            for (int64_t q = b; q < e; ++q) {
                const int at = pos[tile_of(q)]++;
                rij[at] = i0[q] | (j0[q] << 16);
                rsx[at] = sx[q];
                rsy[at] = sy[q];
                ridx[at] = ids[q];
            }
        }
    });
    if (pitch > 0) {
        constexpr int NB = 32;
        std::vector<int>& rij2 = S.rij2;
        std::vector<int>& ridx2 = S.ridx2;
        std::vector<R>& rsx2 = S.rsx2;
        std::vector<R>& rsy2 = S.rsy2;
        rij2 = rij;
        ridx2 = ridx;
        rsx2 = rsx;
        rsy2 = rsy;
        // tiles are independent: ranges of tiles with about equal record counts per thread
        const int nth = 16;
        std::vector<int> tcut(nth + 1, ntiles);
        tcut[0] = 0;
        for (int k = 1; k < nth; ++k)
            tcut[k] = (int)(std::lower_bound(cnt.begin(), cnt.end() - 1, (int)(nrec * k / nth)) - cnt.begin());
        for (int k = 1; k <= nth; ++k) tcut[k] = std::max(tcut[k], tcut[k - 1]);
        parallel_ranges(nth, 1, [&](int64_t kb, int64_t ke) {
            std::vector<std::vector<int>> grp(NB);
            std::vector<int> next(NB), order(NB);
            std::vector<std::pair<int, int>> chunk;  // (residue, record) of the chunk being formed
            for (int t = tcut[kb]; t < tcut[ke]; ++t) {
                const int b0 = cnt[t], b1 = cnt[t + 1];
                if (b1 - b0 < 2) continue;
                const int gx0 = (t % ntx) * T, gy0 = (t / ntx) * T;
                for (auto& v : grp) v.clear();
                for (int r = b0; r < b1; ++r) {
                    const int ii = (rij[r] & 0xffff) - gx0, jj = (rij[r] >> 16) - gy0;
                    grp[(jj * pitch + ii) % NB].push_back(r);
                }
                std::fill(next.begin(), next.end(), 0);
                // chunks of NB records: each takes one record from each of the residues
                // with the most records left (so all NB residues last as long as they
                // can), more from the largest only when fewer than NB remain; within a
                // chunk the records go in ascending residue (a full chunk: record q has
                // residue q, so any grouping of its lanes reads distinct banks)
                int out = b0;
                while (out < b1) {
                    const int chunk_end = std::min(b1, out + NB);
                    chunk.clear();
                    while ((int)chunk.size() < chunk_end - out) {
                        for (int k = 0; k < NB; ++k) order[k] = k;
                        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
                            return (int)grp[x].size() - next[x] > (int)grp[y].size() - next[y];
                        });
                        for (int k = 0; k < NB && (int)chunk.size() < chunk_end - out; ++k) {
                            const int g = order[k];
                            if (next[g] == (int)grp[g].size()) break;  // sorted: the rest are empty too
                            chunk.push_back({g, grp[g][next[g]++]});
                        }
                    }
                    std::stable_sort(chunk.begin(), chunk.end(),
                                     [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.first < y.first; });
                    for (const auto& c : chunk) {
                        const int r = c.second;
                        rij2[out] = rij[r];
                        ridx2[out] = ridx[r];
                        rsx2[out] = rsx[r];
                        rsy2[out] = rsy[r];
                        ++out;
                    }
                }
            }
        });
        rij.swap(rij2);
        ridx.swap(ridx2);
        rsx.swap(rsx2);
        rsy.swap(rsy2);
    }
    RecList* L = list;
    vp_status s;
    L->h_start = cnt;
    L->h_ij = rij;
    if ((s = upload(p, &L->start, cnt, "tile starts")) != VP_OK) return s;
    if ((s = upload(p, &L->ij, rij, "records ij")) != VP_OK) return s;
    if ((s = upload(p, (R**)&L->dx, rsx, "records dx")) != VP_OK) return s;
    if ((s = upload(p, (R**)&L->dy, rsy, "records dy")) != VP_OK) return s;
    if ((s = upload(p, &L->idx, ridx, "records idx")) != VP_OK) return s;
    L->n = nrec;
    return VP_OK;
}

// Work units of one level: each tile with records becomes one or more units
// of at most kUnitNodes volume / kUnitBnd boundary nodes (spreading on LDS;
// kUnitNodesMma / kUnitBndMma on matrix cores) or kUnitTargets targets
// (interpolation).
vp_status build_units(Plan& p, int l)
{
    LevelBufs& b = p.lb[l];
    const int ntiles = p.lv[l].ntx * p.lv[l].ntx;
    auto cnt_of = [&](const RecList& L, int t) { return L.h_start.empty() ? 0 : L.h_start[t + 1] - L.h_start[t]; };
    auto beg_of = [&](const RecList& L, int t) { return L.h_start.empty() ? 0 : L.h_start[t]; };
    b.h_sp_units.clear();
    b.h_sp_units_bnd.clear();
    b.h_in_units.clear();
    const int T = p.lv[l].T, w = p.lv[l].w, E = T + w - 1, ntx = p.lv[l].ntx;
    // most records of [a0, a1) of va and [b0, b1) of vb whose w x w supports share a window cell
    // (cov: the caller's (E + 1)^2 scratch)
    auto cover_of = [&](std::vector<int>& cov, int t, int a0, int a1, int b0, int b1) {
        std::fill(cov.begin(), cov.end(), 0);
        const int gx0 = (t % ntx) * T, gy0 = (t / ntx) * T;
        auto add = [&](const std::vector<int>& ij, int r0, int r1) {
            for (int r = r0; r < r1; ++r) {
                const int ii = (ij[r] & 0xffff) - gx0, jj = (ij[r] >> 16) - gy0;
                cov[(size_t)jj * (E + 1) + ii] += 1;
                cov[(size_t)jj * (E + 1) + ii + w] -= 1;
                cov[(size_t)(jj + w) * (E + 1) + ii] -= 1;
                cov[(size_t)(jj + w) * (E + 1) + ii + w] += 1;
            }
        };
        add(b.vol.h_ij, a0, a1);
        add(b.bnd.h_ij, b0, b1);
        int best = 0;
        for (int y = 0; y <= E; ++y)
            for (int x = 0; x <= E; ++x) {
                int v = cov[(size_t)y * (E + 1) + x];
                if (x > 0) v += cov[(size_t)y * (E + 1) + x - 1];
                if (y > 0) v += cov[(size_t)(y - 1) * (E + 1) + x];
                if (x > 0 && y > 0) v -= cov[(size_t)(y - 1) * (E + 1) + x - 1];
                cov[(size_t)y * (E + 1) + x] = v;
                best = std::max(best, v);
            }
        return best;
    };
    // a matrix-core unit is one wavefront's work: smaller units keep more
    // wavefronts in flight on dense tiles (and need no cover: no fixed point)
    const bool mma = p.lv[l].mma != 0;
    const int cap_v = mma ? kUnitNodesMma : kUnitNodes, cap_b = mma ? kUnitBndMma : kUnitBnd;
    for (int t = 0; t < ntiles; ++t) {
        const int nv = cnt_of(b.vol, t), nb = cnt_of(b.bnd, t);
        const int ku = std::max((nv + cap_v - 1) / cap_v, (nb + cap_b - 1) / cap_b);
        for (int k = 0; k < ku; ++k) {
            WorkUnit u;
            u.tile = t;
            u.a0 = beg_of(b.vol, t) + std::min(nv, k * cap_v);
            u.a1 = beg_of(b.vol, t) + std::min(nv, (k + 1) * cap_v);
            u.b0 = beg_of(b.bnd, t) + std::min(nb, k * cap_b);
            u.b1 = beg_of(b.bnd, t) + std::min(nb, (k + 1) * cap_b);
            u.cover = 0;
            b.h_sp_units.push_back(u);
        }
    }
    if (!mma)
        parallel_ranges((int64_t)b.h_sp_units.size(), 256, [&](int64_t u0, int64_t u1) {
            std::vector<int> cov((size_t)(E + 1) * (E + 1));
            for (int64_t k = u0; k < u1; ++k) {
                WorkUnit& u = b.h_sp_units[k];
                u.cover = cover_of(cov, u.tile, u.a0, u.a1, u.b0, u.b1);
            }
        });
    // a spread of the layers alone (the products of the boundary integral solves, the
    // float32 double-layer channels) takes only the units with boundary nodes; the
    // cover of the whole unit bounds its boundary part's
    for (const WorkUnit& u : b.h_sp_units)
        if (u.b1 > u.b0) {
            WorkUnit v = u;
            v.a1 = v.a0;
            b.h_sp_units_bnd.push_back(v);
        }
    // targets on the interpolation's own tiles
    const int ntiles_i = p.lv[l].ntxi * p.lv[l].ntxi;
    for (int t = 0; t < ntiles_i; ++t) {
        const int nt = cnt_of(b.tgt, t);
        for (int k = 0; k * kUnitTargets < nt; ++k) {
            WorkUnit u;
            u.tile = t;
            u.a0 = beg_of(b.tgt, t) + k * kUnitTargets;
            u.a1 = beg_of(b.tgt, t) + std::min(nt, (k + 1) * kUnitTargets);
            u.b0 = u.b1 = 0;
            u.cover = 0;
            b.h_in_units.push_back(u);
        }
    }
    vp_status s;
    if ((s = upload(p, &b.sp_units, b.h_sp_units, "spreading units")) != VP_OK) return s;
    if ((s = upload(p, &b.sp_units_bnd, b.h_sp_units_bnd, "boundary spreading units")) != VP_OK) return s;
    if ((s = upload(p, &b.in_units, b.h_in_units, "interpolation units")) != VP_OK) return s;
    return VP_OK;
}

// Spreading kernel piece of tap a over one grid cell, as a function of the
// node offset: the tap sits at z = ((2a - w) + (u + 1)) / w, u = 2d - 1.
static double tap_kernel(int W, int a, double u, double beta)
{
    const double z = ((2.0 * a - W) + (u + 1.0)) / W;
    const double q = 1.0 - z * z;
    return q > 0 ? std::exp(-beta * z * z / (1.0 + std::sqrt(q))) : 0.0;
}

// Chebyshev interpolation of every tap's piece at P points in u, converted
// to monomial coefficients ([W][P], constant term first).
static std::vector<double> fit_tap_polynomials(int W, int P, double beta)
{
    std::vector<double> coef((size_t)W * P);
    std::vector<double> cn(P), fv(P);
    for (int j = 0; j < P; ++j) cn[j] = std::cos(M_PI * (j + 0.5) / P);
    for (int a = 0; a < W; ++a) {
        for (int j = 0; j < P; ++j) fv[j] = tap_kernel(W, a, cn[j], beta);
        std::vector<double> ch(P);
        for (int k = 0; k < P; ++k) {
            double sacc = 0.0;
            for (int j = 0; j < P; ++j) sacc += fv[j] * std::cos(M_PI * k * (j + 0.5) / P);
            ch[k] = (k == 0 ? 1.0 : 2.0) * sacc / P;
        }
        // T_k(u) as monomials by the three-term recurrence on coefficient vectors
        std::vector<double> mono(P, 0.0), tkm1(P, 0.0), tk(P, 0.0), tkp1(P, 0.0);
        tkm1[0] = 1.0;
        if (P > 1) tk[1] = 1.0;
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
    return coef;
}

// Make the table exactly even, as the kernel is: tap w-1-a at u is tap a at -u, so
// its coefficients are tap a's with the odd ones negated (the middle tap of an odd
// width keeps only even terms); float32 plans then round every coefficient to
// float32, the values their kernels evaluate with.
static void settle_tap_table(std::vector<double>& coef, int W, int P, bool fp32)
{
    for (int a = 0; a < W; ++a) {
        const int m = W - 1 - a;
        for (int i = 0; i < P; ++i) {
            double& c = coef[(size_t)a * P + i];
            if (m < a) c = (i & 1) ? -coef[(size_t)m * P + i] : coef[(size_t)m * P + i];
            else if (m == a && (i & 1)) c = 0.0;
            if (fp32) c = (double)(float)c;
        }
    }
}

// Fourier transform of the kernel the device applies: tap a's piece is the
// polynomial coef[a] in u = 2d - 1 over the cell [a - w/2, a - w/2 + 1) of the
// support (grid units, node at the origin), so at F-periodic integer frequencies
// phihat(m) = sum_a int_0^1 p_a(2d - 1) cos(2 pi m (a - w/2 + d) / F) dd
// (the table is even, so the sine part vanishes).  Gauss-Legendre per cell,
// exact for the polynomial times the cosine to rounding (at most half a turn
// of phase per cell).
static std::vector<double> poly_kernel_ft(const std::vector<double>& coef, int W, int P, int F, int M)
{
    std::vector<double> gx, gw;
    gauss_legendre(P + 24, gx, gw);
    std::vector<double> val((size_t)W * gx.size());
    for (int a = 0; a < W; ++a)
        for (size_t q = 0; q < gx.size(); ++q) {
            double v = 0.0;
            for (int i = P - 1; i >= 0; --i) v = v * gx[q] + coef[(size_t)a * P + i];
            val[(size_t)a * gx.size() + q] = v;
        }
    std::vector<double> out(M + 1);
    for (int m = 0; m <= M; ++m) {
        double s = 0.0;
        for (int a = 0; a < W; ++a)
            for (size_t q = 0; q < gx.size(); ++q) {
                const double x = a - 0.5 * W + 0.5 * (gx[q] + 1.0);
                s += gw[q] * val[(size_t)a * gx.size() + q] * std::cos(2.0 * M_PI * m * x / F);
            }
        out[m] = 0.5 * s;   // dd = du / 2
    }
    return out;
}

// max |polynomial - kernel| over taps and 513 offsets per tap
static double tap_fit_error(const std::vector<double>& coef, int W, int P, double beta)
{
    double e = 0.0;
    for (int a = 0; a < W; ++a)
        for (int k = 0; k <= 512; ++k) {
            const double u = -1.0 + 2.0 * k / 512.0;
            double v = 0.0;
            for (int i = P - 1; i >= 0; --i) v = v * u + coef[(size_t)a * P + i];
            e = std::max(e, std::fabs(v - tap_kernel(W, a, u, beta)));
        }
    return e;
}

template <typename R>
vp_status build_level_tables(Plan& p, int l, double d1, double d2)
{
    LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    const int M = g.M;
    const double s = g.dk / (2.0 * M_PI);
    const double scale = s * s;
    const bool fp32 = p.precision == VP_FP32;
    // Spreading kernel per tap as a polynomial in the node offset (spreading
    // table, horner_terms(w) terms; interpolation table, interp_terms(w)), made
    // exactly even and, for the interpolation of float32 plans, rounded to float32.  The multiplier
    // divides by the transforms of exactly these polynomials, so the tables'
    // fit to the exponential of the semicircle is no error of the method's
    // discretization: the spread and the interpolation apply kernels whose
    // transforms are divided out exactly.
    const int W = g.w, P = horner_terms(W);
    const int PI = interp_terms(W, fp32);
    std::vector<double> coef = fit_tap_polynomials(W, P, g.beta);
    std::vector<double> coef_i = fit_tap_polynomials(W, PI, g.beta);
    settle_tap_table(coef, W, P, false);      // spreading taps are evaluated in float64
    settle_tap_table(coef_i, W, PI, fp32);    // interpolation taps in the plan's precision
    const std::vector<double> ph_s = poly_kernel_ft(coef, W, P, g.F, M);
    const std::vector<double> ph_i = poly_kernel_ft(coef_i, W, PI, g.F, M);
    for (int m = 0; m <= M; ++m)
        if (!(ph_s[m] > 0 && ph_i[m] > 0)) return fail(VP_ERR_INTERNAL, "spreading kernel transform not positive");
    std::vector<R> mult((size_t)(M + 1) * (M + 1));
    parallel_ranges(M + 1, 16, [&](int64_t a0, int64_t a1) {  // rows of the table
        for (int64_t a = a0; a < a1; ++a)
            for (int c = 0; c <= M; ++c) {
                const double k2 = g.dk * g.dk * ((double)a * a + (double)c * c);
                const double m = (l == 0) ? mult_nh(k2, d1, d2) : mult_fh(k2, d2, p.L);
                const double ph = ph_s[a] * ph_s[c] * ph_i[a] * ph_i[c];
                mult[(size_t)a * (M + 1) + c] = (R)(scale * m / ph);
            }
    });
    g.dc_coef = scale * ((l == 0) ? mult_nh(0.0, d1, d2) : mult_fh(0.0, d2, p.L));
    {
        g.fit_err[0] = tap_fit_error(coef, W, P, g.beta);
        g.fit_err[1] = tap_fit_error(coef_i, W, PI, g.beta);
        // bound on |d/dy tap value| = (2/h) |dp/du| over taps and offsets (sampled, 5% margin)
        double dm = 0.0;
        for (int a = 0; a < W; ++a)
            for (int k = 0; k <= 256; ++k) {
                const double u = -1.0 + 2.0 * k / 256.0;
                double pv = 0.0;
                for (int i = P - 1; i >= 1; --i) pv = pv * u + i * coef[(size_t)a * P + i];
                dm = std::max(dm, std::fabs(pv));
            }
        g.dmax = 1.05 * dm * 2.0 / g.h;
        vp_status st2;
        if ((st2 = upload(p, &b.horner, coef, "kernel polynomials")) != VP_OK) return st2;
        if ((st2 = upload(p, &b.horner_i, coef_i, "interpolation kernel polynomials")) != VP_OK) return st2;
        if (fp32) {  // the same values as float32, for the float32 interpolation
            const std::vector<float> cif(coef_i.begin(), coef_i.end());
            if ((st2 = upload(p, &b.horner_if, cif, "interpolation kernel polynomials (float32)")) != VP_OK)
                return st2;
        }
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

// Records, work units and tables of level l for the plan's current geometry.
template <typename R>
vp_status build_level(Plan& p, int l, const std::vector<double>& sxv, const std::vector<double>& syv,
                      const std::vector<int>& vol_ids, const std::vector<int>& bnd_ids, const std::vector<double>& tx,
                      const std::vector<double>& ty)
{
    vp_status s;
    std::vector<int> tids(p.n_tgt);
    std::iota(tids.begin(), tids.end(), 0);
    LevelBufs& b = p.lb[l];
    if ((s = build_records<R>(p, l, sxv, syv, vol_ids, &b.vol)) != VP_OK) return s;
    if ((s = build_records<R>(p, l, sxv, syv, bnd_ids, &b.bnd)) != VP_OK) return s;
    if ((s = build_records<R>(p, l, tx, ty, tids, &b.tgt, p.lv[l].Ti + p.lv[l].w - 1, p.lv[l].Ti)) != VP_OK) return s;
    // row bands: the supports' corner rows j0 of the records (spread: rows j0 .. j0 + w - 1;
    // interpolation: also row j0 + w, which an odd-width support reads with weight zero)
    {
        LevelGeom& g = p.lv[l];
        auto rows = [&](const RecList& L, int& lo, int& hi) {
            std::vector<int> plo(kHostParts, INT32_MAX), phi(kHostParts, -1);  // per range
            parallel_parts((int64_t)L.h_ij.size(), 1 << 16, [&](int part, int64_t b0, int64_t b1) {
                int a = INT32_MAX, z = -1;
                for (int64_t r = b0; r < b1; ++r) {
                    const int j0 = L.h_ij[r] >> 16;
                    a = std::min(a, j0);
                    z = std::max(z, j0);
                }
                plo[part] = a;
                phi[part] = z;
            });
            for (int k = 0; k < kHostParts; ++k) {
                lo = std::min(lo, plo[k]);
                hi = std::max(hi, phi[k]);
            }
        };
        // A band starts on a multiple of 8 rows and spans a multiple of 64: the row passes map
        // blocks to XCDs in contiguous eighths only when the row count is a multiple of 8, and
        // then each eighth starts on a 128-byte line of the column-major spectrum (8 complex
        // float64 values), so no line is shared by two XCDs' L2s (a 1780-row band without this
        // ran the float64 inverse row pass at 0.053 ms against 0.029 ms for all 2048 rows).
        auto align = [&](int a, int z, int& b0, int& b1) {
            if (z <= a) {
                b0 = b1 = 0;
                return;
            }
            b0 = a & ~7;
            const int c = (z - b0 + 63) & ~63;
            if (c >= g.F) {
                b0 = 0;
                b1 = g.F;
                return;
            }
            b0 = std::min(b0, g.F - c);
            b1 = b0 + c;
        };
        int lo = INT32_MAX, hi = -1;
        rows(b.vol, lo, hi);
        rows(b.bnd, lo, hi);
        align(lo, hi >= 0 ? std::min(g.F, hi + g.w) : lo, g.rd0, g.rd1);
        lo = INT32_MAX;
        hi = -1;
        rows(b.tgt, lo, hi);
        align(lo, hi >= 0 ? std::min(g.F, hi + g.w + 1) : lo, g.rt0, g.rt1);
    }
    if ((s = build_units(p, l)) != VP_OK) return s;
    if ((s = build_level_tables<R>(p, l, p.delta1, p.delta2)) != VP_OK) return s;
    return VP_OK;
}

// Give the interpolation its own tile edge (a divisor of the grid): false if none.
bool set_interp_tile(LevelGeom& g, int Ti)
{
    while (Ti > g.F) Ti /= 2;
    if (Ti < 1 || g.F % Ti) return false;
    g.Ti = Ti;
    g.ntxi = g.F / Ti;
    return true;
}

// A feasible discretization of one level.
struct LevelCand {
    int F, w, M;
    double P;       // period
    double cost;    // static cost model (used without autotune)
};

// Geometry of level l for candidate c and tile edge T.
vp_status set_level_geom(Plan& p, int l, const LevelCand& c, int T, double cx, double cy)
{
    LevelGeom& g = p.lv[l];
    g.F = c.F;
    g.logF = ilog2(c.F);
    g.M = c.M;
    g.w = c.w;
    g.period = c.P;
    g.dk = 2.0 * M_PI / c.P;
    g.h = c.P / c.F;
    g.x0 = cx - 0.5 * c.P;
    g.y0 = cy - 0.5 * c.P;
    const double sigma = (double)c.F / (2.0 * c.M + 1.0);
    g.beta = 0.97 * M_PI * c.w * (1.0 - 0.5 / sigma);
    while (T > c.F) T /= 2;
    if (T < 1 || c.F % T) return fail(VP_ERR_ARG, "tile must divide the fine grid");
    g.T = T;
    g.ntx = c.F / T;
    g.Ti = T;
    g.ntxi = g.ntx;
    g.mma = T == kMmaTile ? 1 : 0;  // both precisions: float32 or float64 matrix instructions
    // Float32 far-history levels spread the double layer as two channels of its own: through the
    // kernel derivative its grid holds a dipole layer of size ~1/h whose float32 rounding is white
    // noise, which the far-history multiplier amplifies at the lowest wavenumbers where the dipole
    // signal is smallest (measured on the square workload: 1.2e-5 with the derivative, growing
    // with the far-history grid); in channels of their own the noise is multiplied by k like the
    // signal.
    g.dip = (p.precision == VP_FP32 && (p.kinds & VP_KIND_D) && l == 1) ? 1 : 0;
    return VP_OK;
}

bool level_fits_lds(const Plan& p, int l)
{
    const size_t lim = 160 * 1024;
    return row_fft_lds_bytes(p, l) <= lim && col_fft_lds_bytes(p, l) <= lim && spread_lds_bytes(p, l) <= lim &&
           interp_lds_bytes_of(p, l) <= lim;
}

// Release what build_level allocated (allocations made after index mark).
void drop_level(Plan& p, int l, size_t mark, size_t bytes_before)
{
    for (size_t i = mark; i < p.allocs.size(); ++i) hipFree(p.allocs[i]);
    p.allocs.resize(mark);
    p.device_bytes = bytes_before;
    p.lb[l] = LevelBufs{};
}

// Device time (ms, best of 3 after one warm-up) of one level's kernels, in two
// parts: grid zeroing, strengths, spread, row FFT, column pass and row inverse
// FFT (*ms_grid), then the interpolation (*ms_interp), with the node weights
// standing in for the densities.  The first part depends on the spreading tile
// and not on the interpolation's, the second the other way round.
vp_status time_level(Plan& p, int l, double* ms_grid, double* ms_interp)
{
    const LevelGeom& g = p.lv[l];
    const size_t rb = p.precision == VP_FP32 ? sizeof(float) : sizeof(double);
    const size_t F = g.F, M1 = g.M + 1;
    const int64_t nstr = p.n_src + p.n_bnd + ((p.kinds & VP_KIND_D) ? 2 * p.n_bnd : 0);
    size_t off = 0;
    const size_t o_grid = off;
    off += align256(F * F * rb);
    const size_t o_spec = off;
    off += align256(M1 * F * 2 * rb);
    const size_t o_hist = off;
    off += align256((size_t)std::max<int64_t>(p.n_tgt, 1) * rb);
    const size_t o_str = off;
    off += align256((size_t)std::max<int64_t>(nstr, 1) * rb);
    const size_t o_dc = off;
    off += align256(kDcParts * sizeof(double));
    const size_t o_smax = off;
    off += align256(kSmaxEntries * sizeof(unsigned long long));
    size_t o_dip[4] = {0, 0, 0, 0};
    if (g.dip)
        for (int c = 0; c < 2; ++c) {
            o_dip[2 * c] = off;
            off += align256(F * F * rb);
            o_dip[2 * c + 1] = off;
            off += align256(M1 * F * 2 * rb);
        }
    unsigned char* blk = nullptr;
    VP_HIP(hipMalloc((void**)&blk, off), "autotune workspace");
    Workspace ws;
    ws.block = blk;
    ws.bytes = off;
    ws.grid[l] = blk + o_grid;
    ws.spec[l] = blk + o_spec;
    ws.hist[l] = blk + o_hist;
    ws.str = blk + o_str;
    ws.dc = (double*)(blk + o_dc);
    ws.smax = (unsigned long long*)(blk + o_smax);
    if (g.dip)
        for (int c = 0; c < 2; ++c) {
            ws.dgrid[c] = blk + o_dip[2 * c];
            ws.dspec[c] = blk + o_dip[2 * c + 1];
        }
    const bool uv = (p.kinds & VP_KIND_V) && p.n_src > 0;
    const bool ub = (p.kinds & (VP_KIND_S | VP_KIND_D)) && p.n_bnd > 0;
    const bool ud = (p.kinds & VP_KIND_D) && p.n_bnd > 0;
    const double* f = uv ? p.d_w : nullptr;
    const double* sig = ub && !ud ? p.d_w + p.n_src : nullptr;
    const double* mu = ud ? p.d_w + p.n_src : nullptr;
    hipStream_t st = p.stream;
    hipEvent_t e0 = nullptr, em = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&em);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    double best_g = INFINITY, best_i = INFINITY;
    for (int rep = 0; rep < 4 && err == hipSuccess; ++rep) {
        err = hipEventRecord(e0, st);
        if (err == hipSuccess) err = launch_zero(p, ws, st);
        if (err == hipSuccess) err = launch_strengths(p, ws, st, f, sig, mu);
        if (err == hipSuccess) err = launch_spread(p, ws, st, l, uv, ub, ud);
        if (err == hipSuccess) err = launch_row_fft(p, ws, st, l, ud);
        if (err == hipSuccess) err = launch_col_fft(p, ws, st, l, ud);
        if (err == hipSuccess) err = launch_row_ifft(p, ws, st, l);
        if (err == hipSuccess) err = hipEventRecord(em, st);
        if (err == hipSuccess) err = launch_interp(p, ws, st, l);
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float tg = 0, ti = 0;
        if (err == hipSuccess) err = hipEventElapsedTime(&tg, e0, em);
        if (err == hipSuccess) err = hipEventElapsedTime(&ti, em, e1);
        if (err == hipSuccess && rep > 0) {
            best_g = std::min(best_g, (double)tg);
            best_i = std::min(best_i, (double)ti);
        }
    }
    if (e0) hipEventDestroy(e0);
    if (em) hipEventDestroy(em);
    if (e1) hipEventDestroy(e1);
    hipFree(blk);
    if (err != hipSuccess) return fail(VP_ERR_DEVICE, std::string("autotune timing: ") + hipGetErrorString(err));
    *ms_grid = best_g;
    *ms_interp = best_i;
    return VP_OK;
}

}  // namespace

vp_status set_error(vp_status s, const std::string& msg) { return fail(s, msg); }

// Workspace layout: grid, spec, hist per level, then strengths and dc, each
// 256-byte aligned inside one allocation.
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
        take(ws ? &ws->grid[l] : nullptr, F * F * rb);
        take(ws ? &ws->spec[l] : nullptr, M1 * F * 2 * rb);
        take(ws ? &ws->hist[l] : nullptr, (size_t)std::max<int64_t>(p.n_tgt, 1) * rb);
        if (g.dip)
            for (int c = 0; c < 2; ++c) {
                take(ws ? &ws->dgrid[c] : nullptr, F * F * rb);
                take(ws ? &ws->dspec[c] : nullptr, M1 * F * 2 * rb);
            }
    }
    const int64_t nstr = p.n_src + p.n_bnd + ((p.kinds & VP_KIND_D) ? 2 * p.n_bnd : 0);
    take(ws ? &ws->str : nullptr, (size_t)std::max<int64_t>(nstr, 1) * rb);
    void* dcp = nullptr;
    take(ws ? &dcp : nullptr, kDcParts * sizeof(double));
    if (ws) ws->dc = (double*)dcp;
    void* smp = nullptr;
    take(ws ? &smp : nullptr, kSmaxEntries * sizeof(unsigned long long));
    if (ws) ws->smax = (unsigned long long*)smp;
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

void workspace_bind(const Plan& p, Workspace& ws, void* block, size_t bytes)
{
    ws = Workspace{};
    ws.block = block;
    ws.bytes = bytes;
    workspace_layout(p, &ws, (unsigned char*)block);
}

hipError_t workspace_free(Workspace& ws, hipStream_t st, bool async)
{
    hipError_t e = hipSuccess;
    if (ws.block) e = async ? hipFreeAsync(ws.block, st) : hipFree(ws.block);
    ws = Workspace{};
    return e;
}

vp_status eval_validate(const Plan& p, const double* f, const double* jet6, const double* sigma,
                        const double* sigma_jet3, const double* mu, const double* mu_jet5, const double* out)
{
    if (!out && p.n_tgt) return fail(VP_ERR_ARG, "out is NULL");
    const bool use_v = f != nullptr;
    const bool use_s = sigma != nullptr;
    const bool use_d = mu != nullptr;
    if (!use_v && !use_s && !use_d) return fail(VP_ERR_ARG, "no density given");
    if (use_v && !(p.kinds & VP_KIND_V)) return fail(VP_ERR_ARG, "plan does not support V");
    if (use_s && !(p.kinds & VP_KIND_S)) return fail(VP_ERR_ARG, "plan does not support S");
    if (use_d && !(p.kinds & VP_KIND_D)) return fail(VP_ERR_ARG, "plan does not support D");
    // the jets are per target: with no targets they may be NULL
    if (use_v && !jet6 && p.n_tgt) return fail(VP_ERR_ARG, "jet6 is required with f");
    if (use_s && !sigma_jet3 && p.n_tgt) return fail(VP_ERR_ARG, "sigma_jet3 is required with sigma");
    if (use_d && !mu_jet5 && p.n_tgt) return fail(VP_ERR_ARG, "mu_jet5 is required with mu");
    return VP_OK;
}

vp_status eval_enqueue(Plan& p, const Workspace& ws, hipStream_t st, const double* f, const double* jet6,
                       const double* sigma, const double* sigma_jet3, const double* mu, const double* mu_jet5,
                       double* out, bool timing)
{
    vp_status vs = eval_validate(p, f, jet6, sigma, sigma_jet3, mu, mu_jet5, out);
    if (vs != VP_OK) return vs;
    const bool use_v = f != nullptr;
    const bool use_s = sigma != nullptr;
    const bool use_d = mu != nullptr;
    if (!ws.block) return fail(VP_ERR_ARG, "no workspace");
    if (timing && !p.ev_made) {
        for (auto& e : p.ev) VP_HIP(hipEventCreate(&e), "event create");
        p.ev_made = true;
    }
    if (!timing) {
        // the two levels are independent from the strengths to the history values:
        // the far-history level's whole chain (spread, FFT passes, interpolation)
        // runs on the side stream beside the near-history level's, after the local
        // part (which needs neither level: memory-bound, it fills the matrix-core
        // spreads' idle bandwidth); the history values are added at the join
        if (!p.side_made) {
            hipStream_t sd = nullptr;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            hipError_t err = hipStreamCreateWithFlags(&sd, hipStreamNonBlocking);
            if (err == hipSuccess) err = hipEventCreateWithFlags(&e0, hipEventDisableTiming);
            if (err == hipSuccess) err = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
            if (err != hipSuccess) {  // release what was made; the next call tries again
                if (e0) (void)hipEventDestroy(e0);
                if (sd) (void)hipStreamDestroy(sd);
                VP_HIP(err, "side stream and events");
            }
            p.side = sd;
            p.fork[0] = e0;
            p.fork[1] = e1;
            p.side_made = true;
        }
        hipStream_t sd = p.side;
        VP_HIP(launch_zero(p, ws, st), "zero");
        VP_HIP(launch_strengths(p, ws, st, f, sigma, mu), "strengths");
        VP_HIP(hipEventRecord(p.fork[0], st), "fork");
        VP_HIP(hipStreamWaitEvent(sd, p.fork[0], 0), "fork");
        VP_HIP(launch_local(p, ws, sd, jet6, sigma_jet3, mu_jet5, use_v, use_s, use_d, out, kLocalPart),
               "local");
        VP_HIP(launch_spread(p, ws, sd, 1, use_v, use_s || use_d, use_d), "spread");
        VP_HIP(launch_row_fft(p, ws, sd, 1, use_d), "row fft");
        VP_HIP(launch_col_fft(p, ws, sd, 1, use_d), "column fft");
        VP_HIP(launch_row_ifft(p, ws, sd, 1), "row ifft");
        VP_HIP(launch_interp(p, ws, sd, 1), "interp");
        VP_HIP(hipEventRecord(p.fork[1], sd), "join");
        VP_HIP(launch_spread(p, ws, st, 0, use_v, use_s || use_d, use_d), "spread");
        VP_HIP(launch_row_fft(p, ws, st, 0, use_d), "row fft");
        VP_HIP(launch_col_fft(p, ws, st, 0, use_d), "column fft");
        VP_HIP(launch_row_ifft(p, ws, st, 0), "row ifft");
        VP_HIP(launch_interp(p, ws, st, 0), "interp");
        VP_HIP(hipStreamWaitEvent(st, p.fork[1], 0), "join");
        VP_HIP(launch_local(p, ws, st, jet6, sigma_jet3, mu_jet5, use_v, use_s, use_d, out, kLocalAddHistory),
               "history sum");
        return VP_OK;
    }
    auto mark = [&](int k) -> hipError_t { return hipEventRecord(p.ev[k], st); };
    VP_HIP(mark(0), "event");
    VP_HIP(launch_zero(p, ws, st), "zero");
    VP_HIP(launch_strengths(p, ws, st, f, sigma, mu), "strengths");
    VP_HIP(mark(1), "event");
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_spread(p, ws, st, l, use_v, use_s || use_d, use_d), "spread");
        VP_HIP(mark(2 + l), "event");
    }
    // timed: every launch on one stream, one per level, in the order of the timing slots
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_row_fft(p, ws, st, l, use_d), "row fft");
        VP_HIP(mark(4 + l), "event");
    }
    for (int l = 0; l < 2; ++l) {
        VP_HIP(launch_col_fft(p, ws, st, l, use_d), "column fft");
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
    o->autotune = 0;
}

const char* vp_last_error(void) { return g_last_error.c_str(); }

vp_status vp_plan(vp_plan_t* out, int64_t n_src, const double* src_x, const double* src_y, const double* src_w,
                  int64_t n_bnd, const double* bnd_x, const double* bnd_y, const double* bnd_nx,
                  const double* bnd_ny, const double* bnd_w, int64_t n_tgt, const double* tgt_x,
                  const double* tgt_y, const vp_local_geom* geom, const vp_opts* opts_in)
{
    g_last_error.clear();
    ScratchRelease scratch_release;  // record-building scratch lives for this call only
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

    // ---- inputs to the host (one copy per array, the copies on host threads)
    std::vector<double> sx, sy, sw, bx, by, bnx, bny, bw, tx, ty;
    std::vector<double> gr, gnx, gny, gk, g3, g4;
    std::vector<int8_t> gs;
    vp_status s;
    const bool need_b = (o.kinds & (VP_KIND_S | VP_KIND_D)) != 0;
    {
        struct Item {
            std::vector<double>* v;
            const double* src;
            int64_t n;
            const char* name;
        };
        std::vector<Item> items = {{&sx, src_x, n_src, "src_x"}, {&sy, src_y, n_src, "src_y"},
                                   {&sw, src_w, n_src, "src_w"}, {&tx, tgt_x, n_tgt, "tgt_x"},
                                   {&ty, tgt_y, n_tgt, "tgt_y"}};
        if (need_b)
            for (Item it : {Item{&bx, bnd_x, n_bnd, "bnd_x"}, Item{&by, bnd_y, n_bnd, "bnd_y"},
                            Item{&bnx, bnd_nx, n_bnd, "bnd_nx"}, Item{&bny, bnd_ny, n_bnd, "bnd_ny"},
                            Item{&bw, bnd_w, n_bnd, "bnd_w"}})
                items.push_back(it);
        if (n_tgt) {
            for (Item it : {Item{&gr, geom->r, n_tgt, "geom.r"}, Item{&gnx, geom->nx, n_tgt, "geom.nx"},
                            Item{&gny, geom->ny, n_tgt, "geom.ny"}, Item{&gk, geom->kappa, n_tgt, "geom.kappa"}})
                items.push_back(it);
            if (geom->gamma3) items.push_back({&g3, geom->gamma3, n_tgt, "geom.gamma3"});
            if (geom->gamma4) items.push_back({&g4, geom->gamma4, n_tgt, "geom.gamma4"});
        }
        for (const Item& it : items) {
            if (it.n > 0 && !it.src) return bail(fail(VP_ERR_ARG, std::string(it.name) + " is NULL"));
            it.v->resize(it.n);
        }
        std::vector<hipError_t> err(items.size(), hipSuccess);
        parallel_ranges((int64_t)items.size(), 1, [&](int64_t b, int64_t e) {
            for (int64_t k = b; k < e; ++k)
                if (items[k].n > 0)
                    err[k] = hipMemcpy(items[k].v->data(), items[k].src, items[k].n * sizeof(double),
                                       hipMemcpyDeviceToHost);
        });
        for (size_t k = 0; k < items.size(); ++k)
            if (err[k] != hipSuccess)
                return bail(fail(VP_ERR_DEVICE, std::string(items[k].name) + ": " + hipGetErrorString(err[k])));
        if (n_tgt && (s = download(gs, geom->sgn, n_tgt, "geom.sgn")) != VP_OK) return bail(s);
    }
    if (!need_b) p->n_bnd = 0;
    for (auto* v : {&sx, &sy, &sw, &bx, &by, &bnx, &bny, &bw, &tx, &ty, &gr, &gnx, &gny, &gk, &g3, &g4})
        if (!all_finite(*v)) return bail(fail(VP_ERR_ARG, "non-finite input value"));
    auto negative = [](double v) { return v < 0; };
    if (any_parallel(sw, negative)) return bail(fail(VP_ERR_ARG, "negative volume weight"));
    if (any_parallel(bw, negative)) return bail(fail(VP_ERR_ARG, "negative boundary weight"));
    if (any_parallel(gr, negative)) return bail(fail(VP_ERR_ARG, "negative target distance r"));
    if (any_parallel(gs, [](int8_t v) { return v < -1 || v > 1; }))
        return bail(fail(VP_ERR_ARG, "sgn must be -1, 0 or +1"));

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
        constexpr int nd = 32;
        std::vector<double> lo(nd, INFINITY), hi(nd, -INFINITY), cs(nd), sn(nd);
        for (int d = 0; d < nd; ++d) {
            cs[d] = std::cos(M_PI * d / nd);
            sn[d] = std::sin(M_PI * d / nd);
        }
        auto scan = [&](const std::vector<double>& X, const std::vector<double>& Y) {
            const int64_t n = (int64_t)X.size();
            std::vector<double> plo(kHostParts * nd, INFINITY), phi(kHostParts * nd, -INFINITY);  // per range
            parallel_parts(n, 1 << 16, [&](int part, int64_t b, int64_t e) {
                double l2[nd], h2[nd], c2[nd], s2[nd];  // this range's extremes, in registers
                for (int d = 0; d < nd; ++d) {
                    l2[d] = INFINITY;
                    h2[d] = -INFINITY;
                    c2[d] = cs[d];
                    s2[d] = sn[d];
                }
                const double* xp = X.data();
                const double* yp = Y.data();
                for (int64_t i = b; i < e; ++i) {
                    const double px = xp[i] - cx, py = yp[i] - cy;
                    for (int d = 0; d < nd; ++d) {
                        const double v = px * c2[d] + py * s2[d];
                        l2[d] = std::min(l2[d], v);
                        h2[d] = std::max(h2[d], v);
                    }
                }
                for (int d = 0; d < nd; ++d) {
                    plo[part * nd + d] = l2[d];
                    phi[part * nd + d] = h2[d];
                }
            });
            for (int k = 0; k < kHostParts; ++k)
                for (int d = 0; d < nd; ++d) {
                    lo[d] = std::min(lo[d], plo[k * nd + d]);
                    hi[d] = std::max(hi[d], phi[k * nd + d]);
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
    const int64_t n_pts = ((o.kinds & VP_KIND_V) ? n_src : 0) + (need_b ? n_bnd : 0);
    const int Fmax = 8192;   // both precisions; level_fits_lds rejects what the LDS cannot hold
    std::vector<LevelCand> cands[2];
    for (int l = 0; l < 2; ++l) {
        // The double layer is spread with the derivative of the spreading kernel,
        // whose aliasing error is amplified relative to the kernel's own; the
        // far-history multiplier weights the lowest wavenumbers most, where the
        // amplification is largest, so that level gets a 20x tighter kernel
        // tolerance (on the square workload one extra tap of width takes the
        // double-layer error from 1.3e-10 to 6e-12).
        const double eps_s = p->eps * 0.1 / ((l == 1 && (o.kinds & VP_KIND_D)) ? 20.0 : 1.0);
        for (int attempt = 0; attempt < 4 && cands[l].empty(); ++attempt) {
            const double P = period[l] * (1.0 + 0.02 * attempt);
            const double dk = 2.0 * M_PI / P;
            const int M = (int)std::ceil(kmax[l] / dk);
            const int nmodes = 2 * M + 1;
            int F0 = 64;
            while (F0 < (int)std::ceil(1.2 * nmodes)) F0 *= 2;
            const int Flim = (o.spread_width[l] > 0 || o.fine_grid[l] > 0) ? Fmax : std::min(4 * F0, Fmax);
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
                const double cost = (double)F * F * 12.0 + (double)n_pts * w * w * 1.5 +
                                    (double)n_tgt * w * w * 1.0;
                cands[l].push_back({F, w, M, P, cost});
            }
        }
        if (cands[l].empty())
            return bail(fail(VP_ERR_TOL, "no supported fine grid meets the tolerance (level " + std::to_string(l) +
                                             ")"));
        std::stable_sort(cands[l].begin(), cands[l].end(),
                         [](const LevelCand& a2, const LevelCand& b2) { return a2.cost < b2.cost; });
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

    // ---- levels: static cost model, or measured selection (opts.autotune)
    const bool fp32 = o.precision == VP_FP32;
    auto build = [&](int l) {
        return fp32 ? build_level<float>(*p, l, ax, ay, vol_ids, bnd_ids, tx, ty)
                    : build_level<double>(*p, l, ax, ay, vol_ids, bnd_ids, tx, ty);
    };
    std::vector<int> tiles;
    if (o.tile > 0) tiles.push_back(o.tile);
    else if (o.autotune) tiles = {32, 16};
    else tiles.push_back(0);  // by width, below
    p->autotuned = o.autotune ? 1 : 0;
    for (int l = 0; l < 2; ++l) {
        int best_c = -1, best_T = 0, best_Ti = 0;
        if (o.autotune) {
            // Each candidate grid is timed with each tile edge T, the interpolation on the
            // same edge.  The grid chain (zeroing to the inverse row pass) does not depend on
            // the interpolation's tile, nor the interpolation on the spreading tile, so a
            // candidate's time is its best grid chain plus its best interpolation, whichever
            // edges they were timed with (a spreading tile and another interpolation tile
            // may win together without being timed together).
            double best_ms = INFINITY;
            for (size_t ci = 0; ci < cands[l].size(); ++ci) {
                double g_best = INFINITY, i_best = INFINITY;
                int g_T = 0, i_T = 0;
                for (int T : tiles) {
                    if ((s = set_level_geom(*p, l, cands[l][ci], T, cx, cy)) != VP_OK) return bail(s);
                    if (!level_fits_lds(*p, l)) continue;
                    const size_t mark = p->allocs.size(), bytes0 = p->device_bytes;
                    if ((s = build(l)) != VP_OK) return bail(s);
                    double ms_g = INFINITY, ms_i = INFINITY;
                    s = time_level(*p, l, &ms_g, &ms_i);
                    drop_level(*p, l, mark, bytes0);
                    if (s != VP_OK) return bail(s);
                    p->tune_cands[l]++;
                    if (ms_g < g_best) {
                        g_best = ms_g;
                        g_T = T;
                    }
                    if (ms_i < i_best) {
                        i_best = ms_i;
                        i_T = T;
                    }
                }
                if (g_T > 0 && g_best + i_best < best_ms) {
                    best_ms = g_best + i_best;
                    best_c = (int)ci;
                    best_T = g_T;
                    best_Ti = i_T;
                }
            }
            p->level_ms[l] = best_ms;
        } else {
            for (size_t ci = 0; ci < cands[l].size() && best_c < 0; ++ci) {
                // without a measurement: the matrix-core spread for levels of width >= 12
                // (measured faster there in both precisions: float32 at widths 12-16, float64
                // at 13 and 16 on the square workload, 0.12 against 0.15-0.18 ms per level),
                // 32-cell tiles and the LDS path otherwise
                const int T = tiles[0] > 0 ? tiles[0] : (cands[l][ci].w >= 12 ? kMmaTile : 32);
                if ((s = set_level_geom(*p, l, cands[l][ci], T, cx, cy)) != VP_OK) return bail(s);
                if (level_fits_lds(*p, l)) {
                    best_c = (int)ci;
                    best_T = T;
                }
            }
        }
        if (best_c < 0) return bail(fail(VP_ERR_TOL, "working set too large for LDS"));
        if (o.autotune && tiles.size() == 1) {
            // a forced spreading tile: the interpolation timed again on the other edge
            for (int Ti : {32, 16}) {
                if ((s = set_level_geom(*p, l, cands[l][best_c], best_T, cx, cy)) != VP_OK) return bail(s);
                if (Ti == p->lv[l].T || !set_interp_tile(p->lv[l], Ti) || !level_fits_lds(*p, l)) continue;
                const size_t mark = p->allocs.size(), bytes0 = p->device_bytes;
                if ((s = build(l)) != VP_OK) return bail(s);
                double ms_g = INFINITY, ms_i = INFINITY;
                s = time_level(*p, l, &ms_g, &ms_i);
                drop_level(*p, l, mark, bytes0);
                if (s != VP_OK) return bail(s);
                p->tune_cands[l]++;
                if (ms_g + ms_i < p->level_ms[l]) {
                    p->level_ms[l] = ms_g + ms_i;
                    best_Ti = p->lv[l].Ti;
                }
            }
        }
        if ((s = set_level_geom(*p, l, cands[l][best_c], best_T, cx, cy)) != VP_OK) return bail(s);
        if (best_Ti > 0 && best_Ti != best_T) set_interp_tile(p->lv[l], best_Ti);
        if ((s = build(l)) != VP_OK) return bail(s);
    }
    if (!o.no_workspace) {
        hipError_t e = workspace_alloc(*p, p->ws, p->stream, false);
        if (e != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,
                             std::string("workspace: ") + hipGetErrorString(e)));
        p->device_bytes += p->ws.bytes;
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
    for (int l = 0; l < 2; ++l) {
        info->tile[l] = p->lv[l].T;
        info->spread_mma[l] = p->lv[l].mma;
        info->interp_tile[l] = p->lv[l].Ti;
        info->spread_terms[l] = horner_terms(p->lv[l].w);
        info->interp_terms[l] = interp_terms(p->lv[l].w, p->precision == VP_FP32);
        info->spread_fit_err[l] = p->lv[l].fit_err[0];
        info->interp_fit_err[l] = p->lv[l].fit_err[1];
    }
    info->precision = p->precision;
    info->n_src = p->n_src;
    info->n_bnd = p->n_bnd;
    info->n_tgt = p->n_tgt;
    info->device_bytes = p->device_bytes;
    info->workspace_bytes = workspace_bytes(*p);
    info->autotuned = p->autotuned;
    for (int l = 0; l < 2; ++l) {
        info->tune_candidates[l] = p->tune_cands[l];
        info->level_ms[l] = p->level_ms[l];
    }
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
