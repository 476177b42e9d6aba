// Per-plan HIP kernels for gfx950: thin __global__ wrappers over the device
// code in vp_device.hpp (one workgroup per unit: tile, row or column), and
// their launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vp_device.hpp"

namespace vp {

namespace {

using namespace dev;

template <typename R>
__global__ __launch_bounds__(kThreads) void k_strengths(int64_t n_src, int64_t n_bnd, const double* __restrict__ f,
                                                        const double* __restrict__ sigma, const double* __restrict__ mu,
                                                        const double* __restrict__ w, const double* __restrict__ nx,
                                                        const double* __restrict__ ny, R* __restrict__ str,
                                                        double* __restrict__ dc, unsigned long long* __restrict__ smax)
{
    dev_strengths<R>(n_src, n_bnd, f, sigma, mu, w, nx, ny, str, dc, smax, blockIdx.x);
}

// Zero the spread grids of both levels (and the double-layer channel grids, if
// any) and the zero-frequency / maximum accumulators.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_zero(R* __restrict__ a, int64_t na, R* __restrict__ b, int64_t nb,
                                                   R* __restrict__ c, R* __restrict__ d, int64_t ncd,
                                                   double* __restrict__ dc, unsigned long long* __restrict__ smax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    dev_zero<R>(a, na, i);
    dev_zero<R>(b, nb, i);
    if (c) {
        dev_zero<R>(c, ncd, i);
        dev_zero<R>(d, ncd, i);
    }
    if (i < kDcParts) dc[i] = 0.0;
    if (i < kSmaxEntries) smax[i] = 0ull;
}

template <typename R, int W>
__global__ __launch_bounds__(kThreads) void k_spread(LevelGeom g, RecView<R> vol, RecView<R> bnd,
                                                     const R* __restrict__ str, int64_t n_src, int64_t n_bnd,
                                                     R* __restrict__ grid, int use_vol, int use_bnd, int use_d,
                                                     const double* __restrict__ coef,
                                                     const unsigned long long* __restrict__ smax,
                                                     const WorkUnit* __restrict__ units)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    dev_spread<R, W>(smem_raw, g, vol, bnd, str, n_src, n_bnd, grid, use_vol, use_bnd, use_d, coef, smax,
                     units[xcd_unit(blockIdx.x, gridDim.x)]);
}

// Matrix-core spread (kMmaTile tiles; float32 or float64 matrix instructions by
// plan precision): one wavefront per work unit.
template <typename R, int W>
__global__ __launch_bounds__(kThreads) void k_spread_mma(LevelGeom g, RecView<R> vol, RecView<R> bnd,
                                                         const R* __restrict__ str, int64_t n_src, int64_t n_bnd,
                                                         R* __restrict__ grid, int use_vol, int use_bnd, int use_d,
                                                         const double* __restrict__ coef,
                                                         const WorkUnit* __restrict__ units, int n_units)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int u = xcd_unit(blockIdx.x, gridDim.x) * (kThreads / 64) + (threadIdx.x >> 6);
    if (u >= n_units) return;
    if constexpr (sizeof(R) == 4)
        dev_spread_mma<W>(smem_raw, g, vol, bnd, str, n_src, n_bnd, grid, use_vol, use_bnd, use_d, coef, units[u]);
    else
        dev_spread_mma64<W>(smem_raw, g, vol, bnd, str, n_src, n_bnd, grid, use_vol, use_bnd, use_d, coef,
                            units[u]);
}

// The FFT passes of one or two levels (and a level's double-layer channels) in
// one launch: blocks [0, n[0]) work on the first entry, the next n[1] on the
// second, and so on.
constexpr int kPairMax = 4;
template <typename R> struct LevelPair {
    LevelGeom g[kPairMax];
    R* grid[kPairMax];
    cplx<R>* spec[kPairMax];
    const cplx<R>* tw[kPairMax];
    const R* mult[kPairMax];
    const cplx<R>* dsp[kPairMax][2];  // column pass: the entry's transformed double-layer channels (or NULL)
    int n[kPairMax];
    int cnt;
    int total() const
    {
        int t = 0;
        for (int k = 0; k < cnt; ++k) t += n[k];
        return t;
    }
};

template <typename R>
__device__ __forceinline__ int pair_unit(const LevelPair<R>& P, int* lv)
{
    int b = blockIdx.x;
    int k = 0;
    while (k + 1 < P.cnt && b >= P.n[k]) b -= P.n[k++];
    *lv = k;
    return xcd_unit(b, P.n[k]);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_r2c(LevelPair<R> P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int l;
    const int u = pair_unit(P, &l);
    dev_row_r2c<R>(smem_raw, P.g[l], P.grid[l], P.tw[l], P.spec[l], u);
}

// The column pass runs one thread per radix-4 butterfly of its length-F FFTs
// (F / 4 threads, at least kThreads): few columns per CU, each a chain of
// dependent LDS passes, so the threads shorten every pass instead of queuing.
constexpr int kColThreadsMax = 1024;

template <typename R>
__global__ __launch_bounds__(kColThreadsMax) void k_col(LevelPair<R> P, int zero_dc)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int l;
    const int u = pair_unit(P, &l);
    dev_col<R>(smem_raw, P.g[l], P.spec[l], P.mult[l], P.tw[l], zero_dc, u, P.dsp[l][0], P.dsp[l][1]);
}

template <typename R>
__global__ __launch_bounds__(kColThreadsMax) void k_col_fwd(LevelPair<R> P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int l;
    const int u = pair_unit(P, &l);
    dev_col_fwd<R>(smem_raw, P.g[l], P.spec[l], P.tw[l], u);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_c2r(LevelPair<R> P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int l;
    const int u = pair_unit(P, &l);
    dev_row_c2r<R>(smem_raw, P.g[l], P.spec[l], P.tw[l], P.grid[l], u);
}

template <typename R, int W>
__global__ __launch_bounds__(kThreads) void k_interp(LevelGeom g, const R* __restrict__ grid, RecView<R> tgt,
                                                     R* __restrict__ hist, const typename TapT<R>::T* __restrict__ coef,
                                                     const WorkUnit* __restrict__ units)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    dev_interp<R, W>(smem_raw, g, grid, tgt, hist, coef, units[xcd_unit(blockIdx.x, gridDim.x)]);
}

__global__ __launch_bounds__(kThreads) void k_local(LocalArgs a)
{
    dev_local(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The interpolation tap table a kernel of plan precision R evaluates.
template <typename R>
inline const typename TapT<R>::T* tap_table(const double* d, const float* f)
{
    if constexpr (std::is_same<R, float>::value) return f;
    else return d;
}

inline unsigned grid_for(int64_t n, int per = kThreads)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers

size_t row_fft_lds_bytes(const Plan& p, int level)
{
    const size_t cb = p.precision == VP_FP32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    return (size_t)lds_padded_len(p.lv[level].F / 2) * cb;
}

size_t col_fft_lds_bytes(const Plan& p, int level)
{
    return p.precision == VP_FP32 ? col_lds_bytes<float>(p.lv[level].F) : col_lds_bytes<double>(p.lv[level].F);
}

hipError_t launch_strengths(const Plan& p, const Workspace& ws, hipStream_t st, const double* f, const double* sigma,
                            const double* mu)
{
    const int64_t n = p.n_src + p.n_bnd;
    const unsigned blocks = grid_for(n, p.precision == VP_FP32 ? str_chunk<float>() : str_chunk<double>());
    if (p.precision == VP_FP32)
        hipLaunchKernelGGL(k_strengths<float>, dim3(blocks), dim3(kThreads), 0, st, p.n_src, p.n_bnd, f, sigma, mu,
                           p.d_w, p.d_nx, p.d_ny, (float*)ws.str, ws.dc, ws.smax);
    else  // the zero-frequency sum is used by the float32 path only; the maxima scale fixed-point windows
        hipLaunchKernelGGL(k_strengths<double>, dim3(blocks), dim3(kThreads), 0, st, p.n_src, p.n_bnd, f, sigma, mu,
                           p.d_w, p.d_nx, p.d_ny, (double*)ws.str, (double*)nullptr, ws.smax);
    return hipGetLastError();
}

// The level whose double layer has channels of its own (-1: none) and whose
// channel buffers are present in ws.
static int dip_level(const Plan& p, const Workspace& ws)
{
    for (int l = 0; l < 2; ++l)
        if (p.lv[l].dip && ws.dgrid[0] && ws.grid[l]) return l;
    return -1;
}

hipError_t launch_zero(const Plan& p, const Workspace& ws, hipStream_t st)
{
    // the rows the spread writes, [rd0, rd1) of each level (the others are never
    // read); a level without a grid in ws (the planner's level timing) is skipped
    auto band = [&](int l) { return (int64_t)(p.lv[l].rd1 - p.lv[l].rd0) * p.lv[l].F; };
    auto first = [&](int l) { return (size_t)p.lv[l].rd0 * p.lv[l].F; };
    const int64_t n0 = ws.grid[0] ? band(0) : 0;
    const int64_t n1 = ws.grid[1] ? band(1) : 0;
    const int dl = dip_level(p, ws);
    const int64_t nd = dl >= 0 ? band(dl) : 0;
    const size_t od = dl >= 0 ? first(dl) : 0;
    const unsigned blocks = grid_for(std::max<int64_t>({n0, n1, nd, (int64_t)kSmaxEntries}));
    if (p.precision == VP_FP32)
        hipLaunchKernelGGL(k_zero<float>, dim3(blocks), dim3(kThreads), 0, st,
                           ws.grid[0] ? (float*)ws.grid[0] + first(0) : nullptr, n0,
                           ws.grid[1] ? (float*)ws.grid[1] + first(1) : nullptr, n1,
                           dl >= 0 ? (float*)ws.dgrid[0] + od : nullptr, dl >= 0 ? (float*)ws.dgrid[1] + od : nullptr,
                           nd, ws.dc, ws.smax);
    else
        hipLaunchKernelGGL(k_zero<double>, dim3(blocks), dim3(kThreads), 0, st,
                           ws.grid[0] ? (double*)ws.grid[0] + first(0) : nullptr, n0,
                           ws.grid[1] ? (double*)ws.grid[1] + first(1) : nullptr, n1,
                           dl >= 0 ? (double*)ws.dgrid[0] + od : nullptr,
                           dl >= 0 ? (double*)ws.dgrid[1] + od : nullptr, nd, ws.dc, ws.smax);
    return hipGetLastError();
}

size_t interp_lds_bytes_of(const Plan& p, int level)
{
    return interp_lds_bytes(p.lv[level].Ti, p.lv[level].w, p.precision == VP_FP32 ? sizeof(float) : sizeof(double));
}

size_t spread_lds_bytes(const Plan& p, int level)
{
    if (p.lv[level].mma) return (kThreads / 64) * (p.precision == VP_FP32 ? mma_wave_bytes() : mma64_wave_bytes());
    size_t a;
    return spread_lds_layout(p.lv[level].T, p.lv[level].w, p.precision == VP_FP32 ? sizeof(float) : sizeof(double),
                             &a);
}

#define VP_W_CASES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

// One spread launch of level l into grid from strengths str (indexed by node:
// volume nodes, then boundary nodes); smax: the fixed-point windows' strength bound.
template <typename R, int W>
static void spread_launch(const Plan& p, hipStream_t st, int l, size_t lds, const R* str,
                          const unsigned long long* smax, R* grid, int uv, int ub, int ud)
{
    const LevelGeom& g = p.lv[l];
    const LevelBufs& b = p.lb[l];
    const bool layers_only = !uv && ub;  // only the units with boundary nodes have work
    const unsigned nu = (unsigned)(layers_only ? b.h_sp_units_bnd.size() : b.h_sp_units.size());
    const WorkUnit* units = layers_only ? b.sp_units_bnd : b.sp_units;
    if (nu == 0) return;
    if (g.mma) {  // four units per workgroup, one per wavefront
        const unsigned nb = (nu + kThreads / 64 - 1) / (kThreads / 64);
        (void)hipFuncSetAttribute((const void*)k_spread_mma<R, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        hipLaunchKernelGGL((k_spread_mma<R, W>), dim3(nb), dim3(kThreads), lds, st, g, view<R>(b.vol), view<R>(b.bnd),
                           str, p.n_src, p.n_bnd, grid, uv, ub, ud, (const double*)b.horner, units, (int)nu);
        return;
    }
    (void)hipFuncSetAttribute((const void*)k_spread<R, W>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_spread<R, W>), dim3(nu), dim3(kThreads), lds, st, g, view<R>(b.vol), view<R>(b.bnd), str,
                       p.n_src, p.n_bnd, grid, uv, ub, ud, (const double*)b.horner, smax, units);
}

// A level with dip spreads the double layer as two more channels: the
// strengths mu nu_1 w and mu nu_2 w (stored after the node strengths, one per
// boundary node) with the kernel itself, into their own grids, bounded by the
// second strength maximum (max |mu nu w|_1).
template <typename R, int W>
static void spread_level(const Plan& p, const Workspace& ws, hipStream_t st, int l, size_t lds, int uv, int ub,
                         int ud)
{
    const R* str = (const R*)ws.str;
    const unsigned long long* smax = ws.smax;
    const bool dip = ud && ub && p.lv[l].dip && ws.dgrid[0];
    spread_launch<R, W>(p, st, l, lds, str, smax, (R*)ws.grid[l], uv, ub, dip ? 0 : ud);
    if (!dip) return;
    const int64_t n_all = p.n_src + p.n_bnd;
    for (int c = 0; c < 2; ++c)
        spread_launch<R, W>(p, st, l, lds, str + n_all + c * p.n_bnd - p.n_src, smax ? smax + kDcParts : nullptr,
                            (R*)ws.dgrid[c], 0, 1, 0);
}

template <typename R>
static hipError_t spread_t(const Plan& p, const Workspace& ws, hipStream_t st, int l, bool use_vol, bool use_bnd,
                           bool use_d)
{
    const LevelBufs& b = p.lb[l];
    const size_t lds = spread_lds_bytes(p, l);
    const int uv = use_vol && b.vol.start != nullptr;
    const int ub = use_bnd && b.bnd.start != nullptr;
    const int ud = use_d ? 1 : 0;
    switch (p.lv[l].w) {
#define VP_CASE(W)                                               \
    case W:                                                      \
        spread_level<R, W>(p, ws, st, l, lds, uv, ub, ud);       \
        break;
        VP_W_CASES(VP_CASE)
#undef VP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_spread(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool use_vol, bool use_bnd,
                         bool use_d)
{
    return p.precision == VP_FP32 ? spread_t<float>(p, ws, st, level, use_vol, use_bnd, use_d)
                                  : spread_t<double>(p, ws, st, level, use_vol, use_bnd, use_d);
}

// Entries of a fused FFT launch: level 0 or 1 alone, or both (level < 0);
// channels = true adds the double-layer channel grids of a level with dip as
// entries of their own (row pass); channels_only keeps just those (their
// forward column transforms).
template <typename R>
static LevelPair<R> level_pair(const Plan& p, const Workspace& ws, int level, int (*units)(const LevelGeom&),
                               bool channels, bool channels_only = false)
{
    LevelPair<R> P{};
    int k = 0;
    const int dl = dip_level(p, ws);
    for (int l = 0; l < 2; ++l) {
        if (level >= 0 && l != level) continue;
        if (!channels_only) {
            P.g[k] = p.lv[l];
            P.grid[k] = (R*)ws.grid[l];
            P.spec[k] = (cplx<R>*)ws.spec[l];
            P.tw[k] = (const cplx<R>*)p.lb[l].tw;
            P.mult[k] = (const R*)p.lb[l].mult;
            P.n[k] = units(p.lv[l]);
            ++k;
        }
        if (channels && l == dl)
            for (int c = 0; c < 2; ++c) {
                P.g[k] = p.lv[l];
                P.grid[k] = (R*)ws.dgrid[c];
                P.spec[k] = (cplx<R>*)ws.dspec[c];
                P.tw[k] = (const cplx<R>*)p.lb[l].tw;
                P.mult[k] = nullptr;
                P.n[k] = units(p.lv[l]);
                ++k;
            }
    }
    P.cnt = k;
    return P;
}

static int rows_of(const LevelGeom& g) { return g.rd1 - g.rd0; }   // forward row pass: the spread's rows
static int trows_of(const LevelGeom& g) { return g.rt1 - g.rt0; }  // inverse row pass: the targets' rows
static int cols_of(const LevelGeom& g) { return g.M + 1; }

static size_t pair_lds(const Plan& p, int level, size_t (*lds)(const Plan&, int))
{
    size_t m = 0;
    for (int l = 0; l < 2; ++l)
        if (level < 0 || l == level) m = std::max(m, lds(p, l));
    return m;
}

// dip_used: the evaluation spread the double layer into the channel grids
template <typename R>
static hipError_t row_fft_t(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool dip_used)
{
    const LevelPair<R> P = level_pair<R>(p, ws, level, rows_of, dip_used);
    if (P.total() > 0)
        hipLaunchKernelGGL(k_row_r2c<R>, dim3(P.total()), dim3(kThreads), pair_lds(p, level, row_fft_lds_bytes), st,
                           P);
    return hipGetLastError();
}

hipError_t launch_row_fft(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool dip_used)
{
    return p.precision == VP_FP32 ? row_fft_t<float>(p, ws, st, level, dip_used)
                                  : row_fft_t<double>(p, ws, st, level, dip_used);
}

template <typename R>
static hipError_t col_fft_t(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool dip_used)
{
    int f = 0;
    for (int l = 0; l < 2; ++l)
        if (level < 0 || l == level) f = std::max(f, p.lv[l].F);
    const int threads = std::min(kColThreadsMax, std::max(kThreads, f / 4));
    const int dl = dip_used ? dip_level(p, ws) : -1;
    if (dl >= 0 && (level < 0 || level == dl)) {
        const LevelPair<R> C = level_pair<R>(p, ws, dl, cols_of, true, true);
        hipLaunchKernelGGL((k_col_fwd<R>), dim3(C.total()), dim3(threads), col_fft_lds_bytes(p, dl), st, C);
    }
    LevelPair<R> P = level_pair<R>(p, ws, level, cols_of, false);
    if (dl >= 0)
        for (int k = 0; k < P.cnt; ++k)
            if (P.spec[k] == (cplx<R>*)ws.spec[dl]) {
                P.dsp[k][0] = (const cplx<R>*)ws.dspec[0];
                P.dsp[k][1] = (const cplx<R>*)ws.dspec[1];
            }
    const int zero_dc = p.precision == VP_FP32 ? 1 : 0;
    hipLaunchKernelGGL((k_col<R>), dim3(P.total()), dim3(threads), pair_lds(p, level, col_fft_lds_bytes), st, P,
                       zero_dc);
    return hipGetLastError();
}

hipError_t launch_col_fft(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool dip_used)
{
    return p.precision == VP_FP32 ? col_fft_t<float>(p, ws, st, level, dip_used)
                                  : col_fft_t<double>(p, ws, st, level, dip_used);
}

template <typename R>
static hipError_t row_ifft_t(const Plan& p, const Workspace& ws, hipStream_t st, int level)
{
    const LevelPair<R> P = level_pair<R>(p, ws, level, trows_of, false);
    if (P.total() > 0)
        hipLaunchKernelGGL(k_row_c2r<R>, dim3(P.total()), dim3(kThreads), pair_lds(p, level, row_fft_lds_bytes), st,
                           P);
    return hipGetLastError();
}

hipError_t launch_row_ifft(const Plan& p, const Workspace& ws, hipStream_t st, int level)
{
    return p.precision == VP_FP32 ? row_ifft_t<float>(p, ws, st, level) : row_ifft_t<double>(p, ws, st, level);
}

template <typename R, int W>
static void interp_launch(const Plan& p, const Workspace& ws, hipStream_t st, int l)
{
    const LevelGeom& g = p.lv[l];
    const LevelBufs& b = p.lb[l];
    const size_t lds = interp_lds_bytes(g.Ti, W, sizeof(R));
    const unsigned nu = (unsigned)b.h_in_units.size();
    if (nu == 0) return;
    hipLaunchKernelGGL((k_interp<R, W>), dim3(nu), dim3(kThreads), lds, st, g, (const R*)ws.grid[l],
                       view<R>(b.tgt), (R*)ws.hist[l], tap_table<R>(b.horner_i, b.horner_if),
                       (const WorkUnit*)b.in_units);
}

template <typename R>
static hipError_t interp_t(const Plan& p, const Workspace& ws, hipStream_t st, int l)
{
    switch (p.lv[l].w) {
#define VP_CASE(W)                           \
    case W:                                  \
        interp_launch<R, W>(p, ws, st, l);   \
        break;
        VP_W_CASES(VP_CASE)
#undef VP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_interp(const Plan& p, const Workspace& ws, hipStream_t st, int level)
{
    return p.precision == VP_FP32 ? interp_t<float>(p, ws, st, level) : interp_t<double>(p, ws, st, level);
}

hipError_t launch_local(const Plan& p, const Workspace& ws, hipStream_t st, const double* jet6, const double* sig_jet,
                        const double* mu_jet, bool use_v, bool use_s, bool use_d, double* out, int part)
{
    LocalArgs a{};
    a.part = part;
    a.n = p.n_tgt;
    a.delta = p.delta1;
    a.order_v = p.loc.order_v;
    a.order_s = p.loc.order_s;
    a.order_d = p.loc.order_d;
    a.r = p.g_r;
    a.nx = p.g_nx;
    a.ny = p.g_ny;
    a.kappa = p.g_kappa;
    a.g3 = p.g_g3;
    a.g4 = p.g_g4;
    a.sgn = p.g_sgn;
    a.jet6 = use_v ? jet6 : nullptr;
    a.sj = use_s ? sig_jet : nullptr;
    a.mj = use_d ? mu_jet : nullptr;
    a.h0 = ws.hist[0];
    a.h1 = ws.hist[1];
    a.fp32 = p.precision == VP_FP32;
    a.dc_weight = p.lv[0].dc_coef + p.lv[1].dc_coef;
    a.dc = a.fp32 ? ws.dc : nullptr;
    a.out = out;
    if (p.n_tgt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_local, dim3(grid_for(p.n_tgt)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace vp
