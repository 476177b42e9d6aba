// Group execution: several (plan, workspace, densities) instances evaluated
// together by one kernel per stage over a table of all their units.  Used by the batched API
// (vp_batch_*: a fixed group, optionally replayed as a hipGraph) and by the
// serving loop (a group per admission of queued requests).
//
// Each stage is described by a short table of segments, one per (instance,
// level) -- or per instance for the node and target stages -- holding a unit
// count: tiles/units for spreading and interpolation, rows and columns for
// the FFT passes, chunks for zeroing, strengths and the local part.  Segments
// are padded to multiples of 8 items, each item is one workgroup, and an
// item decodes to (instance, level, unit) by binary search
// over the segment starts and the XCD-aware unit order within its segment,
// so every XCD works on contiguous units of each instance.  Spreading and
// interpolation are templated on the spreading width: one launch per distinct
// width, covering every (instance, level) with that width.  The potential
// kinds of an instance follow from which of its density pointers are set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "vp_device.hpp"
#include "vp_group.hpp"

namespace vp {

namespace {

thread_local std::string b_last_error;

constexpr int kZeroChunk = kThreads * 64;  // grid cells per zeroing unit

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

// The interpolation tap table of a level for plan precision R.
template <typename R> __device__ inline const typename dev::TapT<R>::T* interp_table(const LevelDesc& d)
{
    if constexpr (sizeof(R) == 4) return d.horner_if;
    else return d.horner_i;
}

// Descriptors (instances, levels, calls, segments) do not change while a
// kernel runs: they are read through the constant address space, which makes
// their loads scalar and lets the compiler treat the pointers they hold as
// global memory (global rather than flat loads, stores and atomics; uniform
// reads of tables such as the tap coefficients then also become scalar).
// (The host pass only type-checks device code and has no such address space.)
template <typename T> __device__ __forceinline__ T desc(const T* p, int64_t k)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) T*)p)[k];
#else
    return p[k];
#endif
}

// Item `it` of a stage -> (instance, level, unit); false for padding items.
__device__ __forceinline__ bool decode(const StageTab& t, int it, int& inst, int& level, int& unit)
{
    int lo = 0, hi = t.nseg - 1;
    while (lo < hi) {  // last segment with begin <= it
        const int mid = (lo + hi + 1) >> 1;
        if (desc(t.seg, mid).begin <= it) lo = mid;
        else hi = mid - 1;
    }
    const Seg s = desc(t.seg, lo);
    const int j = it - s.begin;
    const int padded = (s.count + 7) & ~7;
    if (j < 0 || j >= padded) return false;
    const int u = dev::xcd_unit(j, padded);
    if (u >= s.count) return false;
    inst = s.inst;
    level = s.level;
    unit = u;
    return true;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kg_zero(const InstDesc* __restrict__ inst, const LevelDesc* __restrict__ lv,
                                                    StageTab t)
{
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const LevelDesc D = desc(lv, 2 * i + l);
    const int64_t n = (int64_t)(D.g.rd1 - D.g.rd0) * D.g.F;  // the rows the spread writes
    const size_t o = (size_t)D.g.rd0 * D.g.F;
    const int64_t i0 = (int64_t)u * kZeroChunk;
    for (int64_t k = i0 + threadIdx.x; k < i0 + kZeroChunk; k += blockDim.x) {
        dev::dev_zero<R>((R*)D.grid + o, n, k);
        if (D.dgrid[0]) {
            dev::dev_zero<R>((R*)D.dgrid[0] + o, n, k);
            dev::dev_zero<R>((R*)D.dgrid[1] + o, n, k);
        }
    }
    if (l == 0 && u == 0) {  // the instance's accumulators, once
        const InstDesc I = desc(inst, i);
        if (threadIdx.x < kDcParts) I.dc[threadIdx.x] = 0.0;
        if (threadIdx.x < kSmaxEntries) I.smax[threadIdx.x] = 0ull;
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kg_strengths(const InstDesc* __restrict__ inst,
                                                         const CallDesc* __restrict__ call, StageTab t)
{
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const InstDesc I = desc(inst, i);
    const CallDesc K = desc(call, i);
    dev::dev_strengths<R>(I.n_src, I.n_bnd, K.f, K.sigma, K.mu, I.w, I.nx, I.ny, (R*)I.str,
                          sizeof(R) == 4 ? I.dc : nullptr, I.smax, u);
}

template <typename R, int W>
__global__ __launch_bounds__(kThreads) void kg_spread(const InstDesc* __restrict__ inst,
                                                      const LevelDesc* __restrict__ lv,
                                                      const CallDesc* __restrict__ call, StageTab t)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const InstDesc I = desc(inst, i);
    const CallDesc K = desc(call, i);
    const int ch = l >> 1;
    const LevelDesc D = desc(lv, 2 * i + (l & 1));
    // channel 0: the node strengths (volume, and boundary through the kernel
    // derivative unless the level has double-layer channels); channel ch >= 1:
    // mu nu_ch w on the boundary with the kernel itself.  One call site keeps
    // the register allocation of a single spread.
    const bool chan = ch != 0;
    const R* s = (const R*)I.str + (chan ? (I.n_src + I.n_bnd) + (ch - 1) * I.n_bnd - I.n_src : 0);
    R* grid = (R*)(ch == 0 ? D.grid : ch == 1 ? D.dgrid[0] : D.dgrid[1]);  // no dynamic index: stays scalar
    const int use_vol = !chan && K.f != nullptr && I.has_vol;
    const int use_bnd = chan || ((K.sigma != nullptr || K.mu != nullptr) && I.has_bnd);
    const int use_d = !chan && K.mu != nullptr && !D.dgrid[0];
    dev::dev_spread<R, W>(smem_raw, D.g, vol_view<R>(D), bnd_view<R>(D), s, I.n_src, I.n_bnd, grid, use_vol, use_bnd,
                          use_d, D.horner, chan ? I.smax + kDcParts : I.smax, D.sp_units[u]);
}

// Matrix-core spread: an item is four work units, one per wavefront.
template <typename R, int W>
__global__ __launch_bounds__(kThreads) void kg_spread_mma(const InstDesc* __restrict__ inst,
                                                          const LevelDesc* __restrict__ lv,
                                                          const CallDesc* __restrict__ call, StageTab t)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const InstDesc I = desc(inst, i);
    const CallDesc K = desc(call, i);
    const int ch = l >> 1;
    const LevelDesc D = desc(lv, 2 * i + (l & 1));
    const int unit = u * (kThreads / 64) + (threadIdx.x >> 6);
    if (unit >= D.n_sp_units) return;  // no barrier follows: each wavefront spreads its own unit
    const bool chan = ch != 0;  // as in kg_spread
    const R* s = (const R*)I.str + (chan ? (I.n_src + I.n_bnd) + (ch - 1) * I.n_bnd - I.n_src : 0);
    R* grid = (R*)(ch == 0 ? D.grid : ch == 1 ? D.dgrid[0] : D.dgrid[1]);
    const int use_vol = !chan && K.f != nullptr && I.has_vol;
    const int use_bnd = chan || ((K.sigma != nullptr || K.mu != nullptr) && I.has_bnd);
    const int use_d = !chan && K.mu != nullptr && !D.dgrid[0];
    if constexpr (sizeof(R) == 4)
        dev::dev_spread_mma<W>(smem_raw, D.g, vol_view<float>(D), bnd_view<float>(D), s, I.n_src, I.n_bnd, grid,
                               use_vol, use_bnd, use_d, D.horner, D.sp_units[unit]);
    else
        dev::dev_spread_mma64<W>(smem_raw, D.g, vol_view<double>(D), bnd_view<double>(D), s, I.n_src, I.n_bnd,
                                 grid, use_vol, use_bnd, use_d, D.horner, D.sp_units[unit]);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kg_row_r2c(const LevelDesc* __restrict__ lv, StageTab t)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const int ch = l >> 1;
    const LevelDesc D = desc(lv, 2 * i + (l & 1));
    const LevelGeom g = D.g;
    const R* grid = (const R*)(ch == 0 ? D.grid : ch == 1 ? D.dgrid[0] : D.dgrid[1]);
    cplx<R>* spec = (cplx<R>*)(ch == 0 ? D.spec : ch == 1 ? D.dspec[0] : D.dspec[1]);
    dev::dev_row_r2c<R>(smem_raw, g, grid, (const cplx<R>*)D.tw, spec, u);
}

// Forward column transforms of the double-layer channels (items of channel c >= 1).
template <typename R>
__global__ __launch_bounds__(kThreads) void kg_col_fwd(const LevelDesc* __restrict__ lv, StageTab t)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const int ch = l >> 1;
    const LevelDesc D = desc(lv, 2 * i + (l & 1));
    const LevelGeom g = D.g;
    if (ch) dev::dev_col_fwd<R>(smem_raw, g, (cplx<R>*)(ch == 1 ? D.dspec[0] : D.dspec[1]), (const cplx<R>*)D.tw, u);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kg_col(const LevelDesc* __restrict__ lv, const CallDesc* __restrict__ call,
                                                   StageTab t, int zero_dc)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const LevelDesc D = desc(lv, 2 * i + l);
    const LevelGeom g = D.g;
    const bool dip = D.dgrid[0] && desc(call, i).mu;  // the channels were spread and transformed
    dev::dev_col<R>(smem_raw, g, (cplx<R>*)D.spec, (const R*)D.mult, (const cplx<R>*)D.tw, zero_dc, u,
                    dip ? (const cplx<R>*)D.dspec[0] : nullptr, dip ? (const cplx<R>*)D.dspec[1] : nullptr);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void kg_row_c2r(const LevelDesc* __restrict__ lv, StageTab t)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const LevelDesc D = desc(lv, 2 * i + l);
    const LevelGeom g = D.g;
    dev::dev_row_c2r<R>(smem_raw, g, (const cplx<R>*)D.spec, (const cplx<R>*)D.tw, (R*)D.grid, u);
}

template <typename R, int W>
__global__ __launch_bounds__(kThreads) void kg_interp(const LevelDesc* __restrict__ lv, StageTab t)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    const LevelDesc D = desc(lv, 2 * i + l);
    const LevelGeom g = D.g;
    dev::dev_interp<R, W>(smem_raw, g, (const R*)D.grid, tgt_view<R>(D), (R*)D.hist, interp_table<R>(D),
                          D.in_units[u]);
}

__global__ __launch_bounds__(kThreads) void kg_local(const InstDesc* __restrict__ inst,
                                                     const CallDesc* __restrict__ call, StageTab t)
{
    const int it = blockIdx.x;  // one item per workgroup
    int i, l, u;
    if (it >= t.nitems || !decode(t, it, i, l, u)) return;
    dev::LocalArgs a = desc(inst, i).loc;
    const CallDesc K = desc(call, i);
    a.jet6 = K.jet6;
    a.sj = K.sj;
    a.mj = K.mj;
    a.out = K.out;
    dev::dev_local(a, (int64_t)u * blockDim.x + threadIdx.x);
}

#define VP_W_CASES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

// One workgroup per item, the count rounded up to a multiple of 8: workgroup
// i then runs on XCD i mod 8, and the dispatcher hands items to CUs as they
// free up, which balances units of very different cost (a fixed round-robin
// share per resident workgroup leaves most of them idle behind the few that
// drew the dense tiles).
unsigned item_grid(int n_items)
{
    return (unsigned)std::max((n_items + 7) & ~7, 8);
}

size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

}  // namespace

// ---------------------------------------------------------------------------
// Host side

void fill_instance(const Plan& p, const Workspace& ws, InstDesc& I, LevelDesc* D)
{
    const bool fp32 = p.precision == VP_FP32;
    std::memset(&I, 0, sizeof(I));
    I.n_src = p.n_src;
    I.n_bnd = p.n_bnd;
    I.n_tgt = p.n_tgt;
    I.w = p.d_w;
    I.nx = p.d_nx;
    I.ny = p.d_ny;
    I.dc = ws.dc;
    I.smax = ws.smax;
    I.str = ws.str;
    I.has_vol = p.lb[0].vol.start != nullptr;
    I.has_bnd = p.lb[0].bnd.start != nullptr;
    dev::LocalArgs& a = I.loc;
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
    a.h0 = ws.hist[0];
    a.h1 = ws.hist[1];
    a.fp32 = fp32;
    a.dc_weight = p.lv[0].dc_coef + p.lv[1].dc_coef;
    a.dc = fp32 ? ws.dc : nullptr;
    for (int l = 0; l < 2; ++l) {
        const LevelBufs& lb = p.lb[l];
        LevelDesc& d = D[l];
        std::memset(&d, 0, sizeof(d));
        d.g = p.lv[l];
        d.vol_start = lb.vol.start; d.vol_ij = lb.vol.ij; d.vol_dx = lb.vol.dx; d.vol_dy = lb.vol.dy;
        d.vol_idx = lb.vol.idx;
        d.bnd_start = lb.bnd.start; d.bnd_ij = lb.bnd.ij; d.bnd_dx = lb.bnd.dx; d.bnd_dy = lb.bnd.dy;
        d.bnd_idx = lb.bnd.idx;
        d.tgt_start = lb.tgt.start; d.tgt_ij = lb.tgt.ij; d.tgt_dx = lb.tgt.dx; d.tgt_dy = lb.tgt.dy;
        d.tgt_idx = lb.tgt.idx;
        d.grid = ws.grid[l];
        d.spec = ws.spec[l];
        if (p.lv[l].dip && ws.dgrid[0])
            for (int c = 0; c < 2; ++c) {
                d.dgrid[c] = ws.dgrid[c];
                d.dspec[c] = ws.dspec[c];
            }
        d.mult = lb.mult;
        d.tw = lb.tw;
        d.hist = ws.hist[l];
        d.horner = lb.horner;
        d.horner_i = lb.horner_i;
        d.horner_if = lb.horner_if;
        d.sp_units = lb.sp_units;
        d.in_units = lb.in_units;
        d.n_sp_units = (int)lb.h_sp_units.size();
    }
}

CallDesc make_call(const vp_eval_args& a)
{
    CallDesc c;
    c.f = a.f_src;
    c.jet6 = a.f_src ? a.jet6 : nullptr;
    c.sigma = a.sigma;
    c.sj = a.sigma ? a.sigma_jet3 : nullptr;
    c.mu = a.mu;
    c.mj = a.mu ? a.mu_jet5 : nullptr;
    c.out = a.out;
    return c;
}

void HostStage::add(int inst, int level, int count)
{
    if (count <= 0) return;
    seg.push_back({inst, level, count, nitems});
    nitems += (count + 7) & ~7;
}

vp_status group_build(const std::vector<const Plan*>& plans, const std::vector<Workspace>& ws,
                      const std::vector<vp_eval_args>& args, GroupPlan& G, int kinds)
{
    const int n = (int)plans.size();
    if (n == 0) return set_error(VP_ERR_ARG, "empty group");
    G = GroupPlan{};
    G.precision = plans[0]->precision;
    G.inst.resize(n);
    G.lv.resize(2 * n);
    G.call.resize(n);
    std::map<int, int> sp_of_w, in_of_w;
    for (int i = 0; i < n; ++i) {
        const Plan& p = *plans[i];
        if (p.precision != G.precision) return set_error(VP_ERR_ARG, "group mixes precisions");
        fill_instance(p, ws[i], G.inst[i], &G.lv[2 * i]);
        G.call[i] = make_call(args[i]);
        const int64_t nn = p.n_src + p.n_bnd;
        const int sc = G.precision == VP_FP32 ? dev::str_chunk<float>() : dev::str_chunk<double>();
        G.str.add(i, 0, (int)((nn + sc - 1) / sc));
        G.local.add(i, 0, (int)((p.n_tgt + kThreads - 1) / kThreads));
        for (int l = 0; l < 2; ++l) {
            const LevelGeom& g = p.lv[l];
            const LevelBufs& lb = p.lb[l];
            G.zero.add(i, l, (int)(((int64_t)(g.rd1 - g.rd0) * g.F + kZeroChunk - 1) / kZeroChunk));
            G.row.add(i, l, g.rd1 - g.rd0);
            G.col.add(i, l, g.M + 1);
            G.c2r.add(i, l, g.rt1 - g.rt0);
            G.row.lds = std::max(G.row.lds, row_fft_lds_bytes(p, l));
            G.c2r.lds = G.row.lds;
            G.col.lds = std::max(G.col.lds, col_fft_lds_bytes(p, l));
            // one stage per (width, spreading method)
            auto stage_for = [&](std::map<int, int>& idx, std::vector<HostStage>& v, int mma) -> HostStage& {
                const int key = 2 * g.w + mma;
                auto f = idx.find(key);
                if (f == idx.end()) {
                    idx[key] = (int)v.size();
                    v.emplace_back();
                    v.back().w = g.w;
                    v.back().mma = mma;
                    return v.back();
                }
                return v[f->second];
            };
            HostStage& sp = stage_for(sp_of_w, G.spread, g.mma);
            const int nsu = (int)lb.h_sp_units.size();
            const int sp_items = g.mma ? (nsu + kThreads / 64 - 1) / (kThreads / 64) : nsu;
            sp.add(i, l, sp_items);
            sp.lds = std::max(sp.lds, spread_lds_bytes(p, l));
            // the double-layer channels, when the calls pass mu
            if (G.lv[2 * i + l].dgrid[0] && (args[i].mu || (kinds & VP_KIND_D)) && p.n_bnd > 0)
                for (int c = 1; c <= 2; ++c) {
                    sp.add(i, l + 2 * c, sp_items);
                    G.row.add(i, l + 2 * c, g.rd1 - g.rd0);
                    G.colf.add(i, l + 2 * c, g.M + 1);
                    G.colf.lds = std::max(G.colf.lds, col_fft_lds_bytes(p, l));
                }
            HostStage& in = stage_for(in_of_w, G.interp, 0);
            in.add(i, l, (int)lb.h_in_units.size());
            in.lds = std::max(in.lds, interp_lds_bytes_of(p, l));
        }
    }
    // device image: inst | lv | call | segment tables (filled by group_tabs)
    G.off_inst = 0;
    G.off_lv = a16(G.off_inst + n * sizeof(InstDesc));
    G.off_call = a16(G.off_lv + 2 * n * sizeof(LevelDesc));
    G.off_seg = a16(G.off_call + n * sizeof(CallDesc));
    size_t nseg = G.zero.seg.size() + G.str.seg.size() + G.row.seg.size() + G.colf.seg.size() + G.col.seg.size() +
                  G.c2r.seg.size() + G.local.seg.size();
    for (auto& st : G.spread) nseg += st.seg.size();
    for (auto& st : G.interp) nseg += st.seg.size();
    G.bytes = a16(G.off_seg + nseg * sizeof(Seg));
    G.blob.assign(G.bytes, 0);
    std::memcpy(G.blob.data() + G.off_inst, G.inst.data(), n * sizeof(InstDesc));
    std::memcpy(G.blob.data() + G.off_lv, G.lv.data(), 2 * n * sizeof(LevelDesc));
    std::memcpy(G.blob.data() + G.off_call, G.call.data(), n * sizeof(CallDesc));
    return VP_OK;
}

GroupTabs group_tabs(GroupPlan& G, unsigned char* dev_base)
{
    GroupTabs T;
    T.inst = (const InstDesc*)(dev_base + G.off_inst);
    T.lv = (const LevelDesc*)(dev_base + G.off_lv);
    T.call = (CallDesc*)(dev_base + G.off_call);
    size_t off = G.off_seg;
    auto place = [&](const HostStage& h) {
        StageTab t;
        t.nseg = (int)h.seg.size();
        t.nitems = h.nitems;
        t.seg = (const Seg*)(dev_base + off);
        if (!h.seg.empty()) std::memcpy(G.blob.data() + off, h.seg.data(), h.seg.size() * sizeof(Seg));
        off += h.seg.size() * sizeof(Seg);
        return t;
    };
    T.zero = place(G.zero);
    T.str = place(G.str);
    T.row = place(G.row);
    T.colf = place(G.colf);
    T.col = place(G.col);
    T.c2r = place(G.c2r);
    T.local = place(G.local);
    for (auto& st : G.spread) T.spread.push_back(place(st));
    for (auto& st : G.interp) T.interp.push_back(place(st));
    return T;
}

// ev (optional): kBatchStages + 1 events, recorded before the first stage and
// after each stage kind (zero, strengths, spread, row pass, double-layer
// column transforms, column pass, inverse row pass, interpolation, local part).
template <typename R>
static hipError_t group_launch_t(const GroupPlan& G, const GroupTabs& T, hipStream_t st, hipEvent_t* ev)
{
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    if (T.zero.nitems)
        hipLaunchKernelGGL(kg_zero<R>, dim3(item_grid(T.zero.nitems)), dim3(kThreads), 0, st, T.inst,
                           T.lv, T.zero);
    mark(1);
    if (T.str.nitems)
        hipLaunchKernelGGL(kg_strengths<R>, dim3(item_grid(T.str.nitems)), dim3(kThreads), 0, st,
                           T.inst, T.call, T.str);
    mark(2);
    for (size_t k = 0; k < G.spread.size(); ++k) {
        const StageTab& t = T.spread[k];
        if (!t.nitems) continue;
        const size_t lds = G.spread[k].lds;
        if (G.spread[k].mma) {
            switch (G.spread[k].w) {
#define VP_CASE(W)                                                                                              \
    case W:                                                                                                     \
        (void)hipFuncSetAttribute((const void*)kg_spread_mma<R, W>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                  (int)lds);                                                                    \
        hipLaunchKernelGGL((kg_spread_mma<R, W>), dim3(item_grid(t.nitems)), dim3(kThreads), lds,               \
                           st, T.inst, T.lv, T.call, t);                                                        \
        break;
                VP_W_CASES(VP_CASE)
#undef VP_CASE
            default:
                return hipErrorInvalidValue;
            }
            continue;
        }
        switch (G.spread[k].w) {
#define VP_CASE(W)                                                                                              \
    case W:                                                                                                     \
        (void)hipFuncSetAttribute((const void*)kg_spread<R, W>, hipFuncAttributeMaxDynamicSharedMemorySize,    \
                                  (int)lds);                                                                    \
        hipLaunchKernelGGL((kg_spread<R, W>), dim3(item_grid(t.nitems)), dim3(kThreads), lds, st, \
                           T.inst, T.lv, T.call, t);                                                            \
        break;
            VP_W_CASES(VP_CASE)
#undef VP_CASE
        default:
            return hipErrorInvalidValue;
        }
    }
    mark(3);
    if (T.row.nitems)
        hipLaunchKernelGGL(kg_row_r2c<R>, dim3(item_grid(T.row.nitems)), dim3(kThreads), G.row.lds, st,
                           T.lv, T.row);
    mark(4);
    const int zero_dc = G.precision == VP_FP32 ? 1 : 0;
    if (T.colf.nitems)
        hipLaunchKernelGGL((kg_col_fwd<R>), dim3(item_grid(T.colf.nitems)), dim3(kThreads), G.colf.lds,
                           st, T.lv, T.colf);
    mark(5);
    if (T.col.nitems)
        hipLaunchKernelGGL((kg_col<R>), dim3(item_grid(T.col.nitems)), dim3(kThreads), G.col.lds, st,
                           T.lv, T.call, T.col, zero_dc);
    mark(6);
    if (T.c2r.nitems)
        hipLaunchKernelGGL(kg_row_c2r<R>, dim3(item_grid(T.c2r.nitems)), dim3(kThreads), G.c2r.lds, st,
                           T.lv, T.c2r);
    mark(7);
    for (size_t k = 0; k < G.interp.size(); ++k) {
        const StageTab& t = T.interp[k];
        if (!t.nitems) continue;
        const size_t lds = G.interp[k].lds;
        switch (G.interp[k].w) {
#define VP_CASE(W)                                                                                              \
    case W:                                                                                                     \
        hipLaunchKernelGGL((kg_interp<R, W>), dim3(item_grid(t.nitems)), dim3(kThreads), lds, st, \
                           T.lv, t);                                                                            \
        break;
            VP_W_CASES(VP_CASE)
#undef VP_CASE
        default:
            return hipErrorInvalidValue;
        }
    }
    mark(8);
    if (T.local.nitems)
        hipLaunchKernelGGL(kg_local, dim3(item_grid(T.local.nitems)), dim3(kThreads), 0, st, T.inst,
                           T.call, T.local);
    mark(9);
    return hipGetLastError();
}

hipError_t group_launch(const GroupPlan& G, const GroupTabs& T, hipStream_t st, hipEvent_t* ev)
{
    return G.precision == VP_FP32 ? group_launch_t<float>(G, T, st, ev) : group_launch_t<double>(G, T, st, ev);
}

size_t group_bytes_bound(size_t n)
{
    // descriptors, call table, and at most 14 segments per instance plus 6 for the
    // double-layer channels of a level with dip
    return a16(n * sizeof(InstDesc)) + a16(2 * n * sizeof(LevelDesc)) + a16(n * sizeof(CallDesc)) +
           a16(n * 24 * sizeof(Seg)) + 256;
}

vp_status group_enqueue(const std::vector<const Plan*>& plans, const std::vector<Workspace>& ws,
                        const std::vector<vp_eval_args>& args, void* dev_buf, unsigned char* host_buf,
                        size_t buf_bytes, hipStream_t st, bool* enqueued)
{
    *enqueued = false;
    GroupPlan G;
    vp_status s = group_build(plans, ws, args, G);
    if (s != VP_OK) return s;
    if (G.bytes > buf_bytes) return set_error(VP_ERR_INTERNAL, "group descriptor buffer too small");
    GroupTabs T = group_tabs(G, (unsigned char*)dev_buf);
    std::memcpy(host_buf, G.blob.data(), G.bytes);
    hipError_t e = hipMemcpyAsync(dev_buf, host_buf, G.bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        *enqueued = true;
        e = group_launch(G, T, st);
    }
    if (e != hipSuccess) return set_error(VP_ERR_DEVICE, std::string("group launch: ") + hipGetErrorString(e));
    return VP_OK;
}

}  // namespace vp

using namespace vp;

// A fixed group of plans, each with its own workspace.  Per-call tables are
// staged in a ring of pinned host slots; a slot is rewritten only after the
// copy that last read it has completed.
constexpr int kCallSlots = 4;

struct vp_batch_s {
    std::vector<vp_plan_t> plans;
    int n = 0;
    int kinds = 0;
    hipStream_t stream = nullptr;
    GroupPlan G;
    GroupTabs T;
    unsigned char* d_buf = nullptr;
    CallDesc* h_call[kCallSlots] = {};
    hipEvent_t call_ev[kCallSlots] = {};
    int next_slot = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool have_graph = false;
    bool timing = false;                    // record stage events (no graph) in vp_batch_eval
    hipEvent_t tev[kBatchStages + 1] = {};
};

namespace {

vp_status bfail(vp_status s, const std::string& m)
{
    b_last_error = m;
    return s;
}

void free_batch(vp_batch_s* b)
{
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    else hipDeviceSynchronize();
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    for (auto& e : b->tev)
        if (e) hipEventDestroy(e);
    hipFree(b->d_buf);
    for (int k = 0; k < kCallSlots; ++k) {
        if (b->h_call[k]) hipHostFree(b->h_call[k]);
        if (b->call_ev[k]) hipEventDestroy(b->call_ev[k]);
    }
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
    std::vector<const Plan*> pp(n);
    std::vector<Workspace> ws(n);
    std::vector<vp_eval_args> args(n);
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return bail(bfail(VP_ERR_ARG, "NULL plan"));
        const Plan& p = *plans[i];
        if (p.precision != plans[0]->precision) return bail(bfail(VP_ERR_ARG, "plans differ in precision"));
        if (!p.ws.block) return bail(bfail(VP_ERR_ARG, "batched plans need their own workspace"));
        if ((kinds & VP_KIND_V) && !(p.kinds & VP_KIND_V)) return bail(bfail(VP_ERR_ARG, "a plan lacks V"));
        if ((kinds & VP_KIND_S) && !(p.kinds & VP_KIND_S)) return bail(bfail(VP_ERR_ARG, "a plan lacks S"));
        if ((kinds & VP_KIND_D) && !(p.kinds & VP_KIND_D)) return bail(bfail(VP_ERR_ARG, "a plan lacks D"));
        pp[i] = &p;
        ws[i] = p.ws;
        std::memset(&args[i], 0, sizeof(args[i]));
    }
    vp_status s = group_build(pp, ws, args, b->G, kinds);   // every call passes the kinds' densities
    if (s != VP_OK) return bail(bfail(s, vp_last_error()));
    if (hipMalloc((void**)&b->d_buf, b->G.bytes) != hipSuccess) return bail(bfail(VP_ERR_OOM, "batch tables"));
    b->T = group_tabs(b->G, b->d_buf);
    if (hipMemcpy(b->d_buf, b->G.blob.data(), b->G.bytes, hipMemcpyHostToDevice) != hipSuccess)
        return bail(bfail(VP_ERR_DEVICE, "batch tables upload"));
    for (int k = 0; k < kCallSlots; ++k) {
        if (hipHostMalloc((void**)&b->h_call[k], n * sizeof(CallDesc), hipHostMallocDefault) != hipSuccess)
            return bail(bfail(VP_ERR_OOM, "pinned call table"));
        if (hipEventCreateWithFlags(&b->call_ev[k], hipEventDisableTiming) != hipSuccess)
            return bail(bfail(VP_ERR_DEVICE, "event"));
    }
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
    }
    // the slot's previous copy has completed before the slot is rewritten
    const int k = b->next_slot;
    b->next_slot = (k + 1) % kCallSlots;
    if (hipEventSynchronize(b->call_ev[k]) != hipSuccess) return bfail(VP_ERR_DEVICE, "call slot");
    for (int i = 0; i < b->n; ++i) {
        vp_eval_args c = args[i];
        if (!use_v) c.f_src = c.jet6 = nullptr;
        if (!use_s) c.sigma = c.sigma_jet3 = nullptr;
        if (!use_d) c.mu = c.mu_jet5 = nullptr;
        b->h_call[k][i] = make_call(c);
    }
    if (hipMemcpyAsync((void*)b->T.call, b->h_call[k], b->n * sizeof(CallDesc), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return bfail(VP_ERR_DEVICE, "call table");
    if (hipEventRecord(b->call_ev[k], b->stream) != hipSuccess) return bfail(VP_ERR_DEVICE, "call slot event");
    if (b->timing) {
        hipError_t e = group_launch(b->G, b->T, b->stream, b->tev);
        if (e != hipSuccess) return bfail(VP_ERR_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
        return VP_OK;
    }
    if (use_graph) {
        if (!b->have_graph) {
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return bfail(VP_ERR_DEVICE, "begin capture");
            hipError_t e = group_launch(b->G, b->T, b->stream, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return bfail(VP_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e ? e : e2));
            }
            b->graph = g;
            if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
                return bfail(VP_ERR_DEVICE, "graph instantiate");
            b->have_graph = true;
        }
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return bfail(VP_ERR_DEVICE, "graph launch");
        return VP_OK;
    }
    hipError_t e = group_launch(b->G, b->T, b->stream, nullptr);
    if (e != hipSuccess) return bfail(VP_ERR_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    return VP_OK;
}

vp_status vp_batch_set_timing(vp_batch_t b, int enable)
{
    b_last_error.clear();
    if (!b) return bfail(VP_ERR_ARG, "NULL batch");
    if (enable && !b->tev[0])
        for (auto& e : b->tev)
            if (hipEventCreate(&e) != hipSuccess) return bfail(VP_ERR_DEVICE, "event create");
    b->timing = enable != 0;
    return VP_OK;
}

vp_status vp_batch_get_timing(vp_batch_t b, float* ms, int n)
{
    b_last_error.clear();
    if (!b || !ms || n < kBatchStages) return bfail(VP_ERR_ARG, "NULL argument or n < VP_BATCH_STAGES");
    if (!b->tev[0]) return bfail(VP_ERR_ARG, "timing was never enabled");
    if (hipEventSynchronize(b->tev[kBatchStages]) != hipSuccess) return bfail(VP_ERR_DEVICE, "timing event");
    for (int k = 0; k < kBatchStages; ++k)
        if (hipEventElapsedTime(&ms[k], b->tev[k], b->tev[k + 1]) != hipSuccess)
            return bfail(VP_ERR_DEVICE, "no timed evaluation yet");
    return VP_OK;
}

vp_status vp_batch_destroy(vp_batch_t b)
{
    free_batch(b);
    return VP_OK;
}

}  // extern "C"
