// Batched evaluation: many plans (instances of uneven size) executed by one
// persistent kernel per stage.  Each persistent kernel walks a device work
// table of (instance, level, unit) items -- tiles for spreading and
// interpolation, rows and columns for the FFT passes, node/target chunks for
// the strengths and the local part -- so small and large instances share the
// whole GPU in every stage.  Items of the costliest stages are sorted by
// estimated cost (largest first) and dealt round-robin to the resident
// workgroups.  The stage sequence can be captured once in a hipGraph and
// replayed; per-call density pointers live in a device table refreshed before
// each replay (a copy, not part of the graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "vp_device.hpp"

namespace vp {

namespace {

thread_local std::string b_last_error;

struct Item {
    int inst;
    int level;
    int unit;
};

// Device descriptors (plain data copied to device memory at batch creation).
struct LevelDesc {
    LevelGeom g;
    const int* vol_start; const int* vol_ij; const void* vol_dx; const void* vol_dy; const int* vol_idx;
    const int* bnd_start; const int* bnd_ij; const void* bnd_dx; const void* bnd_dy; const int* bnd_idx;
    const int* tgt_start; const int* tgt_ij; const void* tgt_dx; const void* tgt_dy; const int* tgt_idx;
    void* grid;
    void* spec;
    const void* mult;
    const void* tw;
    void* hist;
    const double* horner;
    const WorkUnit* sp_units;
    const WorkUnit* in_units;
};

struct InstDesc {
    int64_t n_src, n_bnd, n_tgt;
    const double* w;
    const double* nx;
    const double* ny;
    double* dc;
    unsigned long long* smax;
    void* str;
    dev::LocalArgs loc;  // geometry pointers and constants; per-call fields filled from CallDesc
    int has_vol, has_bnd;
};

struct CallDesc {
    const double* f;
    const double* jet6;
    const double* sigma;
    const double* sj;
    const double* mu;
    const double* mj;
    double* out;
};

template <typename R> __device__ inline RecView<R> vol_view(const LevelDesc& d)
{
    return RecView<R>{d.vol_start, d.vol_ij, (const R*)d.vol_dx, (const R*)d.vol_dy, d.vol_idx};
}
template <typename R> __device__ inline RecView<R> bnd_view(const LevelDesc& d)
{
    return RecView<R>{d.bnd_start, d.bnd_ij, (const R*)d.bnd_dx, (const R*)d.bnd_dy, d.bnd_idx};
}
template <typename R> __device__ inline RecView<R> tgt_view(const LevelDesc& d)
{
    return RecView<R>{d.tgt_start, d.tgt_ij, (const R*)d.tgt_dx, (const R*)d.tgt_dy, d.tgt_idx};
}

__global__ void kb_zero_dc(const InstDesc* __restrict__ inst, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * kDcParts; i += gridDim.x * blockDim.x) {
        inst[i / kDcParts].dc[i % kDcParts] = 0.0;
        if (i % kDcParts < 2) inst[i / kDcParts].smax[i % kDcParts] = 0ull;
    }
}

constexpr int kZeroChunk = kThreads * 64;  // grid cells per zeroing work unit

template <typename R>
__global__ __launch_bounds__(kThreads) void kb_zero(const LevelDesc* __restrict__ lv, const Item* __restrict__ items,
                                                    int n_items)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const LevelDesc& D = lv[2 * x.inst + x.level];
        const int64_t n = (int64_t)D.g.F * D.g.F;
        const int64_t i0 = (int64_t)x.unit * kZeroChunk;
        for (int64_t i = i0 + threadIdx.x; i < i0 + kZeroChunk; i += blockDim.x) dev::dev_zero<R>((R*)D.grid, n, i);
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kb_strengths(const InstDesc* __restrict__ inst,
                                                         const CallDesc* __restrict__ call,
                                                         const Item* __restrict__ items, int n_items)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const InstDesc& I = inst[x.inst];
        const CallDesc& K = call[x.inst];
        dev::dev_strengths<R>(I.n_src, I.n_bnd, K.f, K.sigma, K.mu, I.w, I.nx, I.ny, (R*)I.str,
                              sizeof(R) == 4 ? I.dc : nullptr, I.smax, x.unit);
    }
}

template <typename R, int W>
__global__ __launch_bounds__(kThreads) void kb_spread(const InstDesc* __restrict__ inst,
                                                      const LevelDesc* __restrict__ lv,
                                                      const Item* __restrict__ items, int n_items, int use_vol,
                                                      int use_bnd, int use_d)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const InstDesc& I = inst[x.inst];
        const LevelDesc& D = lv[2 * x.inst + x.level];
        const LevelGeom g = D.g;
        dev::dev_spread<R, W>(smem_raw, g, vol_view<R>(D), bnd_view<R>(D), (const R*)I.str, I.n_src, I.n_bnd,
                              (R*)D.grid, use_vol && I.has_vol, use_bnd && I.has_bnd, use_d, D.horner, I.smax,
                              D.sp_units[x.unit]);
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kb_row_r2c(const LevelDesc* __restrict__ lv, const Item* __restrict__ items,
                                                       int n_items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const LevelDesc& D = lv[2 * x.inst + x.level];
        const LevelGeom g = D.g;
        dev::dev_row_r2c<R>(smem_raw, g, (const R*)D.grid, (const cplx<R>*)D.tw, (cplx<R>*)D.spec, x.unit);
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kb_col(const LevelDesc* __restrict__ lv, const Item* __restrict__ items,
                                                   int n_items, int zero_dc)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const LevelDesc& D = lv[2 * x.inst + x.level];
        const LevelGeom g = D.g;
        dev::dev_col<R>(smem_raw, g, (cplx<R>*)D.spec, (const R*)D.mult, (const cplx<R>*)D.tw, zero_dc, x.unit);
        __syncthreads();
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kb_row_c2r(const LevelDesc* __restrict__ lv, const Item* __restrict__ items,
                                                       int n_items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const LevelDesc& D = lv[2 * x.inst + x.level];
        const LevelGeom g = D.g;
        dev::dev_row_c2r<R>(smem_raw, g, (const cplx<R>*)D.spec, (const cplx<R>*)D.tw, (R*)D.grid, x.unit);
        __syncthreads();
    }
}

template <typename R, int W>
__global__ __launch_bounds__(kThreads) void kb_interp(const LevelDesc* __restrict__ lv, const Item* __restrict__ items,
                                                      int n_items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        const LevelDesc& D = lv[2 * x.inst + x.level];
        const LevelGeom g = D.g;
        dev::dev_interp<R, W>(smem_raw, g, (const R*)D.grid, tgt_view<R>(D), (R*)D.hist, D.horner,
                              D.in_units[x.unit]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void kb_local(const InstDesc* __restrict__ inst,
                                                     const CallDesc* __restrict__ call,
                                                     const Item* __restrict__ items, int n_items, int use_v,
                                                     int use_s, int use_d)
{
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item x = items[it];
        dev::LocalArgs a = inst[x.inst].loc;
        const CallDesc& K = call[x.inst];
        a.jet6 = use_v ? K.jet6 : nullptr;
        a.sj = use_s ? K.sj : nullptr;
        a.mj = use_d ? K.mj : nullptr;
        a.out = K.out;
        dev::dev_local(a, (int64_t)x.unit * blockDim.x + threadIdx.x);
    }
}

}  // namespace

}  // namespace vp

using namespace vp;

// Stages of one batched evaluation (one persistent launch each, per level for
// the width-templated ones).
enum { ST_ZERO = 0, ST_STR, ST_SPREAD0, ST_SPREAD1, ST_ROW, ST_COL, ST_C2R, ST_INTERP0, ST_INTERP1, ST_LOCAL, ST_N };

// One group of plans executed together.
struct vp_batch_s {
    std::vector<vp_plan_t> plans;
    int n = 0;
    int precision = VP_FP64;
    int kinds = 0;  // densities every call passes (VP_KIND_*)
    int w[2] = {0, 0};
    hipStream_t stream = nullptr;
    InstDesc* d_inst = nullptr;
    LevelDesc* d_lv = nullptr;
    CallDesc* d_call = nullptr;
    std::vector<CallDesc> h_call;  // host copy of the per-call table (pageable: reusable once copied)
    Item* d_items = nullptr;
    int off[ST_N] = {0};   // stage offsets into d_items
    int cnt[ST_N] = {0};   // stage item counts
    size_t lds_spread[2] = {0, 0}, lds_interp[2] = {0, 0}, lds_row = 0, lds_col = 0;
    int cus = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool have_graph = false;
};

namespace {


vp_status bfail(vp_status s, const std::string& m)
{
    b_last_error = m;
    return s;
}

#define VP_BHIP(call, what)                                                                               \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return bfail(e_ == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE,                          \
                         std::string(what) + ": " + hipGetErrorString(e_));                               \
    } while (0)

unsigned persistent_grid(const vp_batch_s& b, int n_items, int per_cu)
{
    const int g = std::min(n_items, b.cus * per_cu);
    return (unsigned)std::max(g, 1);
}

#define VP_W_CASES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

template <typename R>
hipError_t launch_all(vp_batch_s& b, int use_v, int use_s, int use_d)
{
    hipStream_t st = b.stream;
    hipLaunchKernelGGL(kb_zero_dc, dim3(std::max(1, (b.n * kDcParts + 255) / 256)), dim3(256), 0, st, b.d_inst, b.n);
    const Item* it = b.d_items;
    hipLaunchKernelGGL(kb_zero<R>, dim3(persistent_grid(b, b.cnt[ST_ZERO], 8)), dim3(kThreads), 0, st, b.d_lv,
                       it + b.off[ST_ZERO], b.cnt[ST_ZERO]);
    hipLaunchKernelGGL(kb_strengths<R>, dim3(persistent_grid(b, b.cnt[ST_STR], 8)), dim3(kThreads), 0, st, b.d_inst,
                       b.d_call, it + b.off[ST_STR], b.cnt[ST_STR]);
    for (int l = 0; l < 2; ++l) {
        const int s = l ? ST_SPREAD1 : ST_SPREAD0;
        if (!b.cnt[s]) continue;
        const size_t lds = b.lds_spread[l];
        switch (b.w[l]) {
#define VP_CASE(W)                                                                                               \
    case W:                                                                                                      \
        hipFuncSetAttribute((const void*)kb_spread<R, W>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL((kb_spread<R, W>), dim3(persistent_grid(b, b.cnt[s], 4)), dim3(kThreads), lds, st,   \
                           b.d_inst, b.d_lv, it + b.off[s], b.cnt[s], use_v, use_s || use_d, use_d);            \
        break;
            VP_W_CASES(VP_CASE)
#undef VP_CASE
        default:
            return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(kb_row_r2c<R>, dim3(persistent_grid(b, b.cnt[ST_ROW], 8)), dim3(kThreads), b.lds_row, st,
                       b.d_lv, it + b.off[ST_ROW], b.cnt[ST_ROW]);
    const int zero_dc = b.precision == VP_FP32 ? 1 : 0;
    hipLaunchKernelGGL((kb_col<R>), dim3(persistent_grid(b, b.cnt[ST_COL], 4)), dim3(kThreads), b.lds_col, st,
                       b.d_lv, it + b.off[ST_COL], b.cnt[ST_COL], zero_dc);
    hipLaunchKernelGGL(kb_row_c2r<R>, dim3(persistent_grid(b, b.cnt[ST_C2R], 8)), dim3(kThreads), b.lds_row, st,
                       b.d_lv, it + b.off[ST_C2R], b.cnt[ST_C2R]);
    for (int l = 0; l < 2; ++l) {
        const int s = l ? ST_INTERP1 : ST_INTERP0;
        if (!b.cnt[s]) continue;
        const size_t lds = b.lds_interp[l];
        switch (b.w[l]) {
#define VP_CASE(W)                                                                                              \
    case W:                                                                                                     \
        hipLaunchKernelGGL((kb_interp<R, W>), dim3(persistent_grid(b, b.cnt[s], 8)), dim3(kThreads), lds, st,  \
                           b.d_lv, it + b.off[s], b.cnt[s]);                                                    \
        break;
            VP_W_CASES(VP_CASE)
#undef VP_CASE
        default:
            return hipErrorInvalidValue;
        }
    }
    hipLaunchKernelGGL(kb_local, dim3(persistent_grid(b, b.cnt[ST_LOCAL], 8)), dim3(kThreads), 0, st, b.d_inst,
                       b.d_call, it + b.off[ST_LOCAL], b.cnt[ST_LOCAL], use_v, use_s, use_d);
    return hipGetLastError();
}

void free_batch(vp_batch_s* b)
{
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    else hipDeviceSynchronize();
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    hipFree(b->d_inst);
    hipFree(b->d_lv);
    hipFree(b->d_call);
    hipFree(b->d_items);
    delete b;
}

}  // namespace

extern "C" {

const char* vp_batch_last_error(void) { return b_last_error.c_str(); }

vp_status vp_batch_create(vp_batch_t* out, int n, const vp_plan_t* plans, int kinds, void* stream)
{
    b_last_error.clear();
    if (!out || !plans || n <= 0) return bfail(VP_ERR_ARG, "need out, plans and n > 0");
    *out = nullptr;
    if (kinds <= 0 || (kinds & ~7)) return bfail(VP_ERR_ARG, "bad kinds mask");
    vp_batch_s* b = new (std::nothrow) vp_batch_s();
    if (!b) return bfail(VP_ERR_OOM, "host allocation");
    b->plans.assign(plans, plans + n);
    b->n = n;
    b->kinds = kinds;
    b->stream = (hipStream_t)stream;
    auto bail = [&](vp_status s) {
        free_batch(b);
        return s;
    };
    for (int i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        if (!plans[i]) return bail(bfail(VP_ERR_ARG, "NULL plan"));
        if (i == 0) {
            b->precision = p.precision;
            b->w[0] = p.lv[0].w;
            b->w[1] = p.lv[1].w;
        }
        if (p.precision != b->precision) return bail(bfail(VP_ERR_ARG, "plans differ in precision"));
        if (!p.ws.block) return bail(bfail(VP_ERR_ARG, "batched plans need their own workspace"));
        if (p.lv[0].w != b->w[0] || p.lv[1].w != b->w[1])
            return bail(bfail(VP_ERR_ARG, "plans differ in spreading width (use one width per level per batch)"));
        if ((kinds & VP_KIND_V) && !(p.kinds & VP_KIND_V)) return bail(bfail(VP_ERR_ARG, "a plan lacks V"));
        if ((kinds & VP_KIND_S) && !(p.kinds & VP_KIND_S)) return bail(bfail(VP_ERR_ARG, "a plan lacks S"));
        if ((kinds & VP_KIND_D) && !(p.kinds & VP_KIND_D)) return bail(bfail(VP_ERR_ARG, "a plan lacks D"));
    }
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        b->cus = prop.multiProcessorCount;
    // descriptors
    std::vector<InstDesc> hi(n);
    std::vector<LevelDesc> hl(2 * n);
    const bool fp32 = b->precision == VP_FP32;
    const size_t rb = fp32 ? sizeof(float) : sizeof(double);
    size_t lds_row = 0, lds_col = 0;
    size_t lds_sp[2] = {0, 0}, lds_in[2] = {0, 0};
    std::vector<std::vector<Item>> st(ST_N);
    std::vector<std::vector<double>> cost(ST_N);
    for (int i = 0; i < n; ++i) {
        Plan& p = *plans[i];
        InstDesc& I = hi[i];
        I.n_src = p.n_src;
        I.n_bnd = p.n_bnd;
        I.n_tgt = p.n_tgt;
        I.w = p.d_w;
        I.nx = p.d_nx;
        I.ny = p.d_ny;
        I.dc = p.ws.dc;
        I.smax = p.ws.smax;
        I.str = p.ws.str;
        I.has_vol = p.lb[0].vol.start != nullptr;
        I.has_bnd = p.lb[0].bnd.start != nullptr;
        dev::LocalArgs& a = I.loc;
        std::memset(&a, 0, sizeof(a));
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
        a.h0 = p.ws.hist[0];
        a.h1 = p.ws.hist[1];
        a.fp32 = fp32;
        a.dc_weight = p.lv[0].dc_coef + p.lv[1].dc_coef;
        a.dc = fp32 ? p.ws.dc : nullptr;
        const int64_t nn = p.n_src + p.n_bnd;
        for (int64_t u = 0; u * (int64_t)dev::kStrChunk < nn; ++u) {
            st[ST_STR].push_back({i, 0, (int)u});
            cost[ST_STR].push_back(1.0);
        }
        for (int64_t u = 0; u * kThreads < p.n_tgt; ++u) {
            st[ST_LOCAL].push_back({i, 0, (int)u});
            cost[ST_LOCAL].push_back(1.0);
        }
        for (int l = 0; l < 2; ++l) {
            const LevelGeom& g = p.lv[l];
            const LevelBufs& lb = p.lb[l];
            LevelDesc& D = hl[2 * i + l];
            D.g = g;
            D.vol_start = lb.vol.start; D.vol_ij = lb.vol.ij; D.vol_dx = lb.vol.dx; D.vol_dy = lb.vol.dy;
            D.vol_idx = lb.vol.idx;
            D.bnd_start = lb.bnd.start; D.bnd_ij = lb.bnd.ij; D.bnd_dx = lb.bnd.dx; D.bnd_dy = lb.bnd.dy;
            D.bnd_idx = lb.bnd.idx;
            D.tgt_start = lb.tgt.start; D.tgt_ij = lb.tgt.ij; D.tgt_dx = lb.tgt.dx; D.tgt_dy = lb.tgt.dy;
            D.tgt_idx = lb.tgt.idx;
            D.grid = p.ws.grid[l];
            D.spec = p.ws.spec[l];
            D.mult = lb.mult;
            D.tw = lb.tw;
            D.hist = p.ws.hist[l];
            D.horner = lb.horner;
            D.sp_units = lb.sp_units;
            D.in_units = lb.in_units;
            // cost-sorted spreading and interpolation items: one per work unit
            const int ss = l ? ST_SPREAD1 : ST_SPREAD0;
            const int si = l ? ST_INTERP1 : ST_INTERP0;
            for (size_t k = 0; k < lb.h_sp_units.size(); ++k) {
                const WorkUnit& u = lb.h_sp_units[k];
                st[ss].push_back({i, l, (int)k});
                cost[ss].push_back(1.0 + (double)(u.a1 - u.a0) + 4.0 * (u.b1 - u.b0));
            }
            for (size_t k = 0; k < lb.h_in_units.size(); ++k) {
                const WorkUnit& u = lb.h_in_units[k];
                st[si].push_back({i, l, (int)k});
                cost[si].push_back(1.0 + (double)(u.a1 - u.a0));
            }
            for (int64_t u = 0; u * kZeroChunk < (int64_t)g.F * g.F; ++u) {
                st[ST_ZERO].push_back({i, l, (int)u});
                cost[ST_ZERO].push_back(1.0);
            }
            for (int r = 0; r < g.F; ++r) {
                st[ST_ROW].push_back({i, l, r});
                cost[ST_ROW].push_back((double)g.F);
            }
            for (int m = 0; m <= g.M; ++m) {
                st[ST_COL].push_back({i, l, m});
                cost[ST_COL].push_back((double)g.F);
            }
            for (int r = 0; r < g.F; ++r) {
                st[ST_C2R].push_back({i, l, r});
                cost[ST_C2R].push_back((double)g.F);
            }
            lds_row = std::max(lds_row, (size_t)(g.F / 2) * 2 * rb);
            lds_col = std::max(lds_col, (size_t)g.F * 2 * rb);
            lds_sp[l] = std::max(lds_sp[l], spread_lds_bytes(p, l));
            lds_in[l] = std::max(lds_in[l], dev::interp_lds_bytes(g.T, g.w, rb));
        }
    }
    if (lds_row > 160 * 1024 || lds_col > 160 * 1024) return bail(bfail(VP_ERR_TOL, "FFT too long for LDS"));
    b->lds_row = lds_row;
    b->lds_col = lds_col;
    b->lds_spread[0] = lds_sp[0];
    b->lds_spread[1] = lds_sp[1];
    b->lds_interp[0] = lds_in[0];
    b->lds_interp[1] = lds_in[1];
    // cost-sorted (largest first) item order per stage
    std::vector<Item> all;
    for (int s = 0; s < ST_N; ++s) {
        std::vector<int> ord(st[s].size());
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return cost[s][a] > cost[s][c]; });
        b->off[s] = (int)all.size();
        b->cnt[s] = (int)ord.size();
        for (int k : ord) all.push_back(st[s][k]);
    }
    VP_BHIP(hipMalloc(&b->d_inst, n * sizeof(InstDesc)), "batch descriptors");
    VP_BHIP(hipMalloc(&b->d_lv, 2 * n * sizeof(LevelDesc)), "batch descriptors");
    VP_BHIP(hipMalloc(&b->d_call, n * sizeof(CallDesc)), "batch call table");
    b->h_call.resize(n);
    VP_BHIP(hipMalloc(&b->d_items, std::max<size_t>(all.size(), 1) * sizeof(Item)), "batch work table");
    VP_BHIP(hipMemcpy(b->d_inst, hi.data(), n * sizeof(InstDesc), hipMemcpyHostToDevice), "upload");
    VP_BHIP(hipMemcpy(b->d_lv, hl.data(), 2 * n * sizeof(LevelDesc), hipMemcpyHostToDevice), "upload");
    if (!all.empty())
        VP_BHIP(hipMemcpy(b->d_items, all.data(), all.size() * sizeof(Item), hipMemcpyHostToDevice), "upload");
    *out = b;
    return VP_OK;
}

vp_status vp_batch_eval(vp_batch_t b, const vp_eval_args* args, int use_graph)
{
    b_last_error.clear();
    if (!b || !args) return bfail(VP_ERR_ARG, "NULL argument");
    const int use_v = (b->kinds & VP_KIND_V) != 0;
    const int use_s = (b->kinds & VP_KIND_S) != 0;
    const int use_d = (b->kinds & VP_KIND_D) != 0;
    for (int i = 0; i < b->n; ++i) {
        const vp_eval_args& a = args[i];
        if (!a.out && b->plans[i]->n_tgt) return bfail(VP_ERR_ARG, "out is NULL");
        if (use_v && (!a.f_src || !a.jet6)) return bfail(VP_ERR_ARG, "f_src and jet6 required by the batch kinds");
        if (use_s && (!a.sigma || !a.sigma_jet3)) return bfail(VP_ERR_ARG, "sigma and sigma_jet3 required");
        if (use_d && (!a.mu || !a.mu_jet5)) return bfail(VP_ERR_ARG, "mu and mu_jet5 required");
        CallDesc& c = b->h_call[i];
        c.f = use_v ? a.f_src : nullptr;
        c.jet6 = use_v ? a.jet6 : nullptr;
        c.sigma = use_s ? a.sigma : nullptr;
        c.sj = use_s ? a.sigma_jet3 : nullptr;
        c.mu = use_d ? a.mu : nullptr;
        c.mj = use_d ? a.mu_jet5 : nullptr;
        c.out = a.out;
    }
    // from pageable memory the copy has consumed the host table when it returns
    VP_BHIP(hipMemcpyAsync(b->d_call, b->h_call.data(), b->n * sizeof(CallDesc), hipMemcpyHostToDevice, b->stream),
            "call table");
    if (use_graph) {
        if (!b->have_graph) {
            VP_BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
            hipError_t e = b->precision == VP_FP32 ? launch_all<float>(*b, use_v, use_s, use_d)
                                                   : launch_all<double>(*b, use_v, use_s, use_d);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return bfail(VP_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e ? e : e2));
            }
            b->graph = g;
            VP_BHIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
            b->have_graph = true;
        }
        VP_BHIP(hipGraphLaunch(b->exec, b->stream), "graph launch");
        return VP_OK;
    }
    hipError_t e = b->precision == VP_FP32 ? launch_all<float>(*b, use_v, use_s, use_d)
                                           : launch_all<double>(*b, use_v, use_s, use_d);
    VP_BHIP(e, "batch launch");
    return VP_OK;
}

vp_status vp_batch_destroy(vp_batch_t b)
{
    free_batch(b);
    return VP_OK;
}

}  // extern "C"
