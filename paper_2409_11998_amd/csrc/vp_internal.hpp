// Internal structures shared by the planner (vp_plan.hip) and the kernels
// (vp_kernels.hip).  Not part of the public ABI (include/vp.h is).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vp.h"

namespace vp {

constexpr int kWMax = 16;        // largest spreading width (grid cells per dimension)
constexpr int kWMin = 4;         // smallest spreading width
constexpr int kThreads = 256;    // threads per workgroup for grid kernels
constexpr int kDcParts = 64;     // partial sums of the zero-frequency term (one wavefront reads them)
// Strength maxima: kDcParts partial maxima per quantity (|strength|, |mu nu w|_1),
// so the strengths units' atomic maxima spread over as many addresses.
constexpr int kSmaxEntries = 2 * kDcParts;
// Terms of the per-tap polynomials of the spreading kernel (degree + 1).  Each
// tap's piece of the kernel over one grid cell is fitted in u = 2d - 1 by
// Chebyshev interpolation (converted to monomial form) with w + 2 terms: fit
// error at the kernel's own exp(-beta) level.  Fewer terms for float32 plans
// (10: value error below 2e-10) measurably raised the double-layer error,
// whose derivative taps need the fuller fit.
__host__ __device__ constexpr int horner_terms(int w) { return w + 2; }
// Interpolation evaluates kernel values only, so its table keeps just the
// terms the plan's arithmetic resolves: 10 for float32 (sampled fit error
// below 2e-10, or equal to the w + 2 fit's where the exp(-beta) floor rules,
// for every width and upsampling factor >= 1.1) and 13 for float64 (within
// 10% of the w + 2 fit for upsampling <= 1.5 and below 5e-14 beyond).
__host__ __device__ constexpr int interp_terms(int w, bool fp32)
{
    return (w + 2 < (fp32 ? 10 : 13)) ? w + 2 : (fp32 ? 10 : 13);
}
constexpr int kLocalAll = 0, kLocalPart = 1, kLocalAddHistory = 2;  // shares of the local kernel's sum
constexpr int kMmaTile = 16;     // tile edge of the matrix-core spread (window of 32 x 32 cells)

// Launches timed by vp_set_timing, in order: grid zeroing + strengths; spread NH, FH; row FFT NH,
// FH; column FFT NH, FH; row inverse NH, FH; interpolation NH, FH; local part.
constexpr int kTimedLaunches = 12;

template <typename R> struct cplx { R x, y; };

// One history level (near or far history, Sec. 3) as the kernels see it.
struct LevelGeom {
    int F;          // fine grid points per dimension (power of two)
    int logF;
    int M;          // retained Fourier modes: |m1|, |m2| <= M
    int w;          // spreading width (grid cells)
    int T;          // tile edge (grid cells); F % T == 0
    int ntx;        // tiles per dimension
    double beta;    // exponential-of-semicircle shape parameter
    double h;       // grid spacing P / F
    double x0, y0;  // coordinates of grid index 0
    double period;  // P
    double dk;      // 2 pi / P
    double dc_coef; // (dk/2pi)^2 * multiplier(0): the zero mode's kernel weight
    double dmax;    // max over taps and offsets of |d/dy tap value| (double-layer spreading bound)
    double fit_err[2]; // sampled max |polynomial - kernel| of the spreading and interpolation tables
    int mma;        // spread on matrix cores (kMmaTile tiles, either precision), else LDS atomics
    int Ti, ntxi;   // interpolation tile edge and tiles per dimension (targets are binned on their own tiles)
    // Double layer in channels of its own: mu nu_1 w and mu nu_2 w spread with the kernel itself into
    // two more grids, whose spectra enter the column pass as -i k_1 B_1 - i k_2 B_2 (float32
    // far-history levels; elsewhere the double layer goes through the kernel derivative).
    int dip;
    // Grid rows the history chain must handle: the spread writes only rows [rd0, rd1) (the
    // nodes' supports) and the interpolation reads only rows [rt0, rt1) (the targets'
    // supports, plus the zero-weight row below each odd-width support).  Zeroing and the
    // forward row pass cover the first band, the inverse row pass the second; the column
    // pass reads the first and writes the second.
    int rd0, rd1, rt0, rt1;
};

// A tile-sorted list of points of one level (CSR by tile): each point appears
// once, in the tile holding its support corner (i0, j0).
struct RecList {
    std::vector<int> h_start;  // host copy of start
    std::vector<int> h_ij;     // host copy of ij
    int* start = nullptr;  // [ntiles+1]
    int* ij = nullptr;     // packed absolute support corner i0 | j0 << 16
    void* dx = nullptr;    // R: i0 - t_x + w/2, in [0, 1)
    void* dy = nullptr;
    int* idx = nullptr;    // node index (volume nodes first, then boundary nodes) or target index
    int64_t n = 0;
};

template <typename R> struct RecView {
    const int* __restrict__ start;
    const int* __restrict__ ij;
    const R* __restrict__ dx;
    const R* __restrict__ dy;
    const int* __restrict__ idx;
};

template <typename R> inline RecView<R> view(const RecList& l)
{
    return RecView<R>{l.start, l.ij, (const R*)l.dx, (const R*)l.dy, l.idx};
}

// A workgroup's share of a tile: records [a0, a1) of one list and [b0, b1) of
// another (spreading: volume and boundary nodes; interpolation: targets).
// Dense tiles are split into several units, so that the number of
// workgroups follows the number of points rather than the number of tiles.
struct WorkUnit {
    int tile;
    int a0, a1;
    int b0, b1;
    int cover;  // spreading: most records of the unit whose supports share one window cell
};
constexpr int kUnitNodes = 1024;     // volume nodes per spreading unit
constexpr int kUnitBnd = 256;        // boundary nodes per spreading unit
constexpr int kUnitNodesMma = 128;   // volume nodes per matrix-core spreading unit (one wavefront)
constexpr int kUnitBndMma = 64;      // boundary nodes per matrix-core spreading unit
constexpr int kUnitTargets = 2048;   // targets per interpolation unit

// Device buffers of one level.  R = float or double (plan precision).
struct LevelBufs {
    RecList vol;               // volume nodes (spread)
    RecList bnd;               // boundary nodes (spread)
    RecList tgt;               // targets (interpolation)
    WorkUnit* sp_units = nullptr;  // spreading work units (tiles with nodes)
    WorkUnit* sp_units_bnd = nullptr;  // the units with boundary nodes, volume ranges emptied (layer-only spreads)
    WorkUnit* in_units = nullptr;  // interpolation work units (tiles with targets)
    std::vector<WorkUnit> h_sp_units, h_sp_units_bnd, h_in_units;
    void* mult = nullptr;      // R [M+1][M+1] (dk/2pi)^2 M(k) / (phihat(m1) phihat(m2))^2
    void* tw = nullptr;        // cplx<R> [F/2] twiddles exp(-2 pi i k / F)
    double* horner = nullptr;  // [w][w+2] per-tap polynomial of the spreading kernel in u = 2d - 1
    double* horner_i = nullptr; // [w][interp_terms] the same pieces, values-only fit for interpolation
    float* horner_if = nullptr; // float32 plans: the interpolation table as float32 (its values are float32)
};

// Per-evaluation device memory (everything an evaluation writes).  A plan may
// own one; the serving loop gives every in-flight request its own, so
// requests on one plan can overlap.
struct Workspace {
    void* grid[2] = {nullptr, nullptr};   // R [F][F] spread grids, reused for the inverse output
    void* spec[2] = {nullptr, nullptr};   // cplx<R> [M+1][F] half spectra (x-frequency major)
    void* dgrid[2] = {nullptr, nullptr};  // R [F][F] double-layer channel grids of the level with dip
    void* dspec[2] = {nullptr, nullptr};  // cplx<R> [M+1][F] their half spectra
    void* hist[2] = {nullptr, nullptr};   // R [n_tgt] history value at each target
    void* str = nullptr;                  // R [n_src + n_bnd (+ 2 n_bnd)] strengths (+ mu nu wG)
    double* dc = nullptr;                 // [kDcParts] float64 partial sums of the spread strengths
    unsigned long long* smax = nullptr;   // [2][kDcParts] partial maxima: bit patterns of |strength|, |mu nu wG|_1
    void* block = nullptr;                // single allocation holding all of the above
    size_t bytes = 0;
};

struct LocalParams {
    double delta;       // delta_1
    int order_v, order_s, order_d;
};

// Oversampled boundary of the dyadic refinement of the local layer parts
// (vp_refine_attach): nodes sorted by cell of a uniform grid of cell edge
// 6 sqrt(delta_1), and the targets within 12 sqrt(delta_1) of the boundary.
struct Refinement {
    int levels = 0;
    double delta_star = 0.0;
    int64_t n_fine = 0;
    double *x = nullptr, *y = nullptr, *nx = nullptr, *ny = nullptr, *w = nullptr;  // sorted by cell
    int* perm = nullptr;        // original index of each sorted node
    int* cell_start = nullptr;  // [ncx * ncy + 1]
    int ncx = 0, ncy = 0;
    double x0 = 0.0, y0 = 0.0, cell = 1.0;
    int n_near = 0;
    int n_units = 0;
    int4* units = nullptr;      // (cell, first, end) runs of near targets
    int* near = nullptr;        // target indices
    double *near_x = nullptr, *near_y = nullptr;
    std::vector<void*> allocs;
};

struct Plan {
    vp_opts opts{};
    int precision = VP_FP64;
    int kinds = 0;
    int64_t n_src = 0, n_bnd = 0, n_tgt = 0;
    double delta1 = 0, delta2 = 0, eps = 0, L = 0;
    LevelGeom lv[2]{};
    LevelBufs lb[2]{};
    LocalParams loc{};
    hipStream_t stream = nullptr;
    // node data in original order (device, float64)
    double* d_w = nullptr;       // [n_src + n_bnd]: volume weights then boundary weights
    double* d_nx = nullptr;      // [n_bnd] outward normal
    double* d_ny = nullptr;
    Workspace ws;                // the plan's own workspace (absent with opts.no_workspace)
    // target geometry (device, float64 / int8)
    double* g_r = nullptr;
    double* g_nx = nullptr;
    double* g_ny = nullptr;
    double* g_kappa = nullptr;
    double* g_g3 = nullptr;
    double* g_g4 = nullptr;
    int8_t* g_sgn = nullptr;
    size_t device_bytes = 0;
    std::vector<void*> allocs;
    bool timing = false;
    // measured selection of the levels (opts.autotune)
    int autotuned = 0;
    int tune_cands[2] = {0, 0};
    double level_ms[2] = {0.0, 0.0};
    hipEvent_t ev[kTimedLaunches + 1]{};  // before the first and after each timed launch
    bool ev_made = false;
    // An untimed evaluation runs the far-history level's chain (spread, FFT
    // passes, interpolation) on a second stream beside the near-history
    // level's: fork after the strengths, join before the local part.
    hipStream_t side = nullptr;
    hipEvent_t fork[2]{};
    bool side_made = false;
    Refinement ref;               // dyadic refinement of the local layer parts (optional)
    // scratch of the boundary integral solves (vp_solve.hip): allocated by the first
    // solve on the plan, grown when a later one needs more, freed with the plan
    void* solve_ws = nullptr;
    size_t solve_ws_bytes = 0;
    // host memory the solves' Arnoldi kernel writes its state into (mapped, so
    // the host reads it without a copy); allocated by the first solve
    void* solve_host = nullptr;
    void* solve_host_dev = nullptr;  // the same memory's device address
    hipEvent_t solve_ev[2]{};
    bool solve_ev_made = false;
};

// Free a plan's refinement data (vp_refine.hip).
void refinement_free(Refinement& r);

// Kernel launchers (vp_kernels.hip).  All enqueue on stream st and write into ws.
hipError_t launch_strengths(const Plan& p, const Workspace& ws, hipStream_t st, const double* f, const double* sigma,
                            const double* mu);
// Grids present in ws, zero-frequency partial sums and strength maxima to zero.
hipError_t launch_zero(const Plan& p, const Workspace& ws, hipStream_t st);
hipError_t launch_spread(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool use_vol, bool use_bnd,
                         bool use_d);
// FFT passes: level 0 or 1, or both levels in one launch (level < 0).
// dip_used: the evaluation spread the double layer into the channel grids of a
// level with dip (their row transforms join the row pass, their column
// transforms precede the column pass, which combines them).
hipError_t launch_row_fft(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool dip_used);
hipError_t launch_col_fft(const Plan& p, const Workspace& ws, hipStream_t st, int level, bool dip_used);
hipError_t launch_row_ifft(const Plan& p, const Workspace& ws, hipStream_t st, int level);
hipError_t launch_interp(const Plan& p, const Workspace& ws, hipStream_t st, int level);
// part: which share of the final sum the local kernel writes (kLocalAll: all of it;
// kLocalPart: the local part alone; kLocalAddHistory: the history values and zero mode
// added to what a kLocalPart pass wrote)
hipError_t launch_local(const Plan& p, const Workspace& ws, hipStream_t st, const double* jet6, const double* sig_jet,
                        const double* mu_jet, bool use_v, bool use_s, bool use_d, double* out, int part = kLocalAll);
size_t row_fft_lds_bytes(const Plan& p, int level);
size_t col_fft_lds_bytes(const Plan& p, int level);
size_t spread_lds_bytes(const Plan& p, int level);
size_t interp_lds_bytes_of(const Plan& p, int level);

// Workspace layout / allocation (vp_plan.hip).  async: stream-ordered
// (hipMallocAsync/hipFreeAsync on st), else plain hipMalloc/hipFree.
size_t workspace_bytes(const Plan& p);
hipError_t workspace_alloc(const Plan& p, Workspace& ws, hipStream_t st, bool async);
hipError_t workspace_free(Workspace& ws, hipStream_t st, bool async);
// Lay out a workspace in a caller-owned block of at least workspace_bytes(p).
void workspace_bind(const Plan& p, Workspace& ws, void* block, size_t bytes);
// Validate the densities of one evaluation against the plan.
vp_status eval_validate(const Plan& p, const double* f, const double* jet6, const double* sigma,
                        const double* sigma_jet3, const double* mu, const double* mu_jet5, const double* out);
// Validate densities against the plan and enqueue one evaluation on st into ws.
vp_status eval_enqueue(Plan& p, const Workspace& ws, hipStream_t st, const double* f, const double* jet6,
                       const double* sigma, const double* sigma_jet3, const double* mu, const double* mu_jet5,
                       double* out, bool timing);
// Thread-local error message shared by the C ABI entry points.
vp_status set_error(vp_status s, const std::string& msg);

}  // namespace vp

// The opaque handle of the C ABI is the plan itself.
struct vp_plan_s : vp::Plan {};
