#pragma once
// Device code shared by the per-plan kernels (vp_kernels.hip) and the batched
// persistent kernels (vp_batch.hip) for gfx950: strengths, spread, 2-D FFT with the history
// multiplier fused into the column pass, interpolation, local part.
//
// Data flow of one evaluation (history part, Sec. 3 Steps 1-4; local part,
// Sec. 4), per level (near history NH, far history FH):
//
//   strengths  c_j (per node, channel)          k_strengths
//   spread     b[g] = sum_j c_j phi(g - t_j)     k_spread     (tile-owned LDS accumulation)
//   row FFT    along x, real -> half spectrum    k_row_r2c    (keeps |m1| <= M only)
//   column     along y: FFT, multiply by         k_col        (channels combined: B0 - i k.B12)
//              (dk/2pi)^2 M(k)/phihat^2, IFFT
//   row IFFT   half spectrum -> real              k_row_c2r
//   interp     u(x_i) = sum_g a[g] phi(t_i - g)  k_interp     (tile grid staged in LDS)
//   local      V_L + S_L + D_L + history sum     k_local      (float64)
//
// Both FFTs are unnormalized (forward exp(-2 pi i), inverse exp(+2 pi i)); all
// constants live in the multiplier table built by the planner.
#include <hip/hip_runtime.h>

#include <cmath>

#include "vp_internal.hpp"

namespace vp {
namespace dev {


// Spreading kernel values of one node at its w taps.  The kernel is the
// exponential of semicircle exp(beta (sqrt(1 - z^2) - 1)), |z| < 1; tap a of a
// node with offset d in [0, 1) sits at z = ((2a - w) + 2d) / w.  The planner
// fits each tap as a polynomial of degree w+1 in u = 2d - 1 (Chebyshev
// interpolation in float64, monomial form, error at the kernel's own e^-beta
// level), so the values cost w(w+2) float64 FMAs with uniform (scalar-loaded)
// coefficients instead of w exponentials, square roots and divisions.
template <int W>
__device__ __forceinline__ void kernel_taps(double d, const double* __restrict__ coef, double* out)
{
    constexpr int P = W + 2;
    const double u = 2.0 * d - 1.0;
#pragma unroll
    for (int a = 0; a < W; ++a) {
        double acc = coef[a * P + P - 1];
#pragma unroll
        for (int k = P - 2; k >= 0; --k) acc = fma(acc, u, coef[a * P + k]);
        out[a] = acc;
    }
}

__device__ __forceinline__ int bitrev(int k, int logn)
{
    return logn ? (int)(__brev((unsigned)k) >> (32 - logn)) : 0;
}

// In-place radix-2 decimation-in-time FFT of n = 2^logn points held in LDS in
// bit-reversed order; output in natural order.  tw[k*tw_stride] =
// exp(-2 pi i k / n) for k < n/2.  Ends with a barrier.
template <typename R>
__device__ void lds_fft(cplx<R>* a, int logn, const cplx<R>* __restrict__ tw, int tw_stride, bool inverse)
{
    const int n = 1 << logn;
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        const int step = (n >> s) * tw_stride;
        for (int b = threadIdx.x; b < (n >> 1); b += blockDim.x) {
            const int pos = b & (half - 1);
            const int i = ((b >> (s - 1)) << s) + pos;
            const int j = i + half;
            cplx<R> wv = tw[pos * step];
            if (inverse) wv.y = -wv.y;
            const cplx<R> u = a[i];
            const cplx<R> v = a[j];
            const R tx = v.x * wv.x - v.y * wv.y;
            const R ty = v.x * wv.y + v.y * wv.x;
            a[i] = {u.x + tx, u.y + ty};
            a[j] = {u.x - tx, u.y - ty};
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Strengths per node and channel (the sums of Sec. 3, Step 2):
//   ch0 = f w (volume) + sigma wG (boundary), ch1 = mu nu1 wG, ch2 = mu nu2 wG.
// Also accumulates sum(ch0) in float64 (the zero-frequency term).
constexpr int kStrChunk = kThreads * 8;  // nodes per strengths work unit

template <typename R>
__device__ void dev_strengths(int64_t n_src, int64_t n_bnd, const double* __restrict__ f,
                              const double* __restrict__ sigma, const double* __restrict__ mu,
                              const double* __restrict__ w, const double* __restrict__ nx,
                              const double* __restrict__ ny, R* __restrict__ str, int C,
                              double* __restrict__ dc, int64_t unit)
{
    const int64_t n = n_src + n_bnd;
    double part = 0.0;
    const int64_t i1 = min(n, (unit + 1) * (int64_t)kStrChunk);
    for (int64_t i = unit * (int64_t)kStrChunk + threadIdx.x; i < i1; i += blockDim.x) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (i < n_src) {
            if (f) s0 = f[i] * w[i];
        } else {
            const int64_t j = i - n_src;
            const double wg = w[i];
            if (sigma) s0 = sigma[j] * wg;
            if (mu) {
                const double m = mu[j] * wg;
                s1 = m * nx[j];
                s2 = m * ny[j];
            }
        }
        str[i] = (R)s0;
        if (C == 3) {
            str[n + i] = (R)s1;
            str[2 * n + i] = (R)s2;
        }
        part += s0;
    }
    // wave reduction, then one float64 atomic per wave
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if ((threadIdx.x & 63) == 0 && part != 0.0) atomicAdd(dc, part);
}


// ---------------------------------------------------------------------------
// Spread (type-1 spreading, Sec. 3 Step 2 via the NUFFT): one workgroup owns a
// T x T tile of the fine grid and writes it once (no global atomics, no
// zero-fill pass).  A node's support starts at grid index i0 = ceil(t - w/2);
// its offset is stored as d = i0 - t + w/2 in [0, 1).
//
// The tile accumulates in LDS with float64 atomic adds in both precisions:
// on gfx950 a 64-lane ds_add_f32 costs ~190 cycles per CU against ~8.5 for
// ds_add_f64 (measured), so float32 plans form their products in float32 and
// round the tile to float32 once, when it is written to the grid.
//
// Single-channel records (volume nodes; boundary nodes when only sigma is
// spread): each wavefront stages a chunk of its records in LDS (the next
// chunk's loads are in flight meanwhile), computes their 2w kernel values
// with one (record, value) pair per lane, then walks the records one at a
// time with lanes mapped to taps: the 64 lanes of one no-return atomic touch
// 64 distinct cells of a w x w patch.  Double-layer boundary records (three
// strengths, few nodes) use one lane per record.
template <typename R> struct SpreadShape {
    static constexpr int kWaves = kThreads / 64;
    static constexpr int kRecs = 32;            // records staged per wave chunk (2 lanes each)
    static constexpr int kVals = 2 * kWMax;     // staged kernel values per record
};

// Dynamic LDS layout of k_spread (bytes): C padded float64 tiles | per-wave staging.
__host__ __device__ inline size_t spread_lds_layout(int T, int C, size_t rb, int waves, int recs, int vals,
                                                    size_t* off_stage)
{
    const size_t tiles = (size_t)C * T * (T + 1) * sizeof(double);
    const size_t stage = (size_t)waves * recs * ((vals + 3) * rb + sizeof(int));
    *off_stage = tiles;
    return tiles + stage;
}

template <typename R, int W, int C>
__device__ void dev_spread(unsigned char* smem_raw, const LevelGeom& g, const RecView<R>& vol, const RecView<R>& bnd,
                           const R* __restrict__ str, int64_t nstr, R* __restrict__ grid, int use_vol, int use_bnd,
                           const double* __restrict__ coef, int t)
{
    using SS = SpreadShape<R>;
    constexpr int NW = SS::kWaves;
    constexpr int RECS = SS::kRecs;
    constexpr int VS = SS::kVals;
    constexpr int WW = W * W;
    constexpr int NTAP = (WW + 63) / 64;
    const int T = g.T;
    const int TP = T + 1;
    const int TS = T * TP;
    size_t off_st;
    spread_lds_layout(T, C, sizeof(R), NW, RECS, VS, &off_st);
    double* tile = reinterpret_cast<double*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    R* stage = reinterpret_cast<R*>(smem_raw + off_st);
    R* vals = stage + (size_t)wv * RECS * (VS + 3);  // [RECS][VS] kernel values (x taps, then y taps)
    R* my_s = vals + RECS * VS;                     // [RECS] strengths
    R* my_d = my_s + RECS;                          // [RECS][2] offsets
    int* my_ij = reinterpret_cast<int*>(stage + (size_t)NW * RECS * (VS + 3)) + wv * RECS;

    const int gx0 = (t % g.ntx) * T;
    const int gy0 = (t / g.ntx) * T;
    for (int i = threadIdx.x; i < C * TS; i += blockDim.x) tile[i] = 0.0;
    __syncthreads();

    // this lane's taps: tap = lane + 64 k, (a, b) = (tap % W, tap / W)
    int ta[NTAP], tb[NTAP];
#pragma unroll
    for (int k = 0; k < NTAP; ++k) {
        const int tap = lane + 64 * k;
        tb[k] = tap / W;
        ta[k] = tap - tb[k] * W;
    }

    auto wave_path = [&](const RecView<R>& L) {
        const int r1 = L.start[t + 1];
        int base = L.start[t] + wv * RECS;
        int c_ij = 0, c_idx = 0;
        R c_dx = R(0), c_dy = R(0);
        if (lane < RECS && base + lane < r1) {
            c_ij = L.ij[base + lane];
            c_idx = L.idx[base + lane];
            c_dx = L.dx[base + lane];
            c_dy = L.dy[base + lane];
        }
        R c_s = (lane < RECS && base + lane < r1) ? str[c_idx] : R(0);
        for (; base < r1; base += NW * RECS) {
            const int nrec = min(RECS, r1 - base);
            if (lane < nrec) {
                my_ij[lane] = c_ij;
                my_s[lane] = c_s;
                my_d[2 * lane] = c_dx;
                my_d[2 * lane + 1] = c_dy;
            }
            const int nb = base + NW * RECS;
            const bool pre = lane < RECS && nb + lane < r1;
            if (pre) {
                c_ij = L.ij[nb + lane];
                c_idx = L.idx[nb + lane];
                c_dx = L.dx[nb + lane];
                c_dy = L.dy[nb + lane];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // kernel values: lane -> (record lane/2, axis lane%2), all W taps
            if ((lane >> 1) < nrec) {
                double pv[W];
                kernel_taps<W>((double)my_d[lane], coef, pv);
                R* dst = vals + (lane >> 1) * VS + (lane & 1) * W;
#pragma unroll
                for (int a = 0; a < W; ++a) dst[a] = (R)pv[a];
            }
            if (pre) c_s = str[c_idx];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int rr = 0; rr < nrec; ++rr) {
                const int p = my_ij[rr];
                const R sv = my_s[rr];
                const int i0 = (p & 0xffff) - gx0;
                const int j0 = (p >> 16) - gy0;
                const R* v = vals + rr * VS;
#pragma unroll
                for (int k = 0; k < NTAP; ++k) {
                    if (k + 1 < NTAP || lane + 64 * k < WW) {
                        const int x = i0 + ta[k];
                        const int y = j0 + tb[k];
                        if ((unsigned)x < (unsigned)T && (unsigned)y < (unsigned)T)
                            atomicAdd(&tile[y * TP + x], (double)(sv * v[ta[k]] * v[W + tb[k]]));
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    };

    if (use_vol) wave_path(vol);
    if (use_bnd && C == 1) wave_path(bnd);
    if (use_bnd && C == 3) {
        const int r1 = bnd.start[t + 1];
        for (int r = bnd.start[t] + threadIdx.x; r < r1; r += blockDim.x) {
            const int p = bnd.ij[r];
            const int i0 = (p & 0xffff) - gx0;
            const int j0 = (p >> 16) - gy0;
            const int k = bnd.idx[r];
            R sc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) sc[c] = str[c * nstr + k];
            double px[W], py[W];
            kernel_taps<W>((double)bnd.dx[r], coef, px);
            kernel_taps<W>((double)bnd.dy[r], coef, py);
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const int y = j0 + b;
                if (y < 0 || y >= T) continue;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const int x = i0 + a;
                    if (x < 0 || x >= T) continue;
                    const R v = (R)px[a] * (R)py[b];
#pragma unroll
                    for (int c = 0; c < C; ++c) atomicAdd(&tile[c * TS + y * TP + x], (double)(sc[c] * v));
                }
            }
        }
    }
    __syncthreads();
    const size_t F = g.F;
    for (int i = threadIdx.x; i < C * T * T; i += blockDim.x) {
        const int c = i / (T * T);
        const int l = i - c * T * T;
        const int y = l / T;
        const int x = l - y * T;
        grid[(size_t)c * F * F + (size_t)(gy0 + y) * F + gx0 + x] = (R)tile[c * TS + y * TP + x];
    }
}

// ---------------------------------------------------------------------------
// Row pass: real FFT along x of each row (length F via a complex FFT of length
// F/2), keeping only x-frequencies 0..M.  Output spec[c][m1][row] so that the
// column pass reads contiguous columns.
template <typename R>
__device__ void dev_row_r2c(unsigned char* smem_raw, const LevelGeom& g, const R* __restrict__ grid,
                            const cplx<R>* __restrict__ tw, cplx<R>* __restrict__ spec, int unit)
{
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int N = F >> 1;
    const int logN = g.logF - 1;
    const int M = g.M;
    const int row = unit % F;
    const int c = unit / F;
    const R* x = grid + ((size_t)c * F + row) * F;
    for (int n = threadIdx.x; n < N; n += blockDim.x) z[bitrev(n, logN)] = {x[2 * n], x[2 * n + 1]};
    __syncthreads();
    lds_fft(z, logN, tw, 2, false);
    for (int k = threadIdx.x; k <= M; k += blockDim.x) {
        const cplx<R> a = z[k];
        const cplx<R> b = z[(N - k) & (N - 1)];
        const R ex = (a.x + b.x) * R(0.5), ey = (a.y - b.y) * R(0.5);   // even-sample spectrum
        const R ox = (a.y + b.y) * R(0.5), oy = (b.x - a.x) * R(0.5);   // odd-sample spectrum
        const cplx<R> wk = tw[k];                                       // exp(-2 pi i k / F)
        cplx<R> X;
        X.x = ex + wk.x * ox - wk.y * oy;
        X.y = ey + wk.x * oy + wk.y * ox;
        spec[((size_t)c * (M + 1) + k) * F + row] = X;
    }
}

// ---------------------------------------------------------------------------
// Column pass for x-frequency m1 = unit: FFT along y of each channel,
// combine B0 - i k1 B1 - i k2 B2 (double layer: derivative of the kernel in
// the source variable), multiply by the level's table, inverse FFT along y.
template <typename R, int C>
__device__ void dev_col(unsigned char* smem_raw, const LevelGeom& g, const cplx<R>* __restrict__ spec,
                        const R* __restrict__ mult, const cplx<R>* __restrict__ tw, cplx<R>* __restrict__ spec2,
                        int zero_dc, int unit)
{
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    constexpr int PER = 8192 / kThreads;
    const int F = g.F;
    const int logF = g.logF;
    const int M = g.M;
    const int m1 = unit;
    const R dk = (R)g.dk;
    cplx<R> acc[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) acc[i] = {R(0), R(0)};
    for (int c = 0; c < C; ++c) {
        const cplx<R>* col = spec + ((size_t)c * (M + 1) + m1) * F;
        for (int q = threadIdx.x; q < F; q += blockDim.x) z[bitrev(q, logF)] = col[q];
        __syncthreads();
        lds_fft(z, logF, tw, 1, false);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + i * kThreads;
            if (q < F) {
                const cplx<R> v = z[q];
                if (c == 0) {
                    acc[i].x += v.x;
                    acc[i].y += v.y;
                } else {
                    const int m2 = q < (F >> 1) ? q : q - F;
                    const R kk = (c == 1) ? dk * R(m1) : dk * R(m2);
                    acc[i].x += kk * v.y;     // -i kk v
                    acc[i].y -= kk * v.x;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = threadIdx.x + i * kThreads;
        if (q < F) {
            const int m2 = q < (F >> 1) ? q : q - F;
            const int am = m2 < 0 ? -m2 : m2;
            R t = am <= M ? mult[(size_t)m1 * (M + 1) + am] : R(0);
            if (zero_dc && m1 == 0 && q == 0) t = R(0);
            z[bitrev(q, logF)] = {acc[i].x * t, acc[i].y * t};
        }
    }
    __syncthreads();
    lds_fft(z, logF, tw, 1, true);
    cplx<R>* out = spec2 + (size_t)m1 * F;
    for (int q = threadIdx.x; q < F; q += blockDim.x) out[q] = z[q];
}

// ---------------------------------------------------------------------------
// Row inverse: rebuild each row's Hermitian x-spectrum from m1 = 0..M (zero
// elsewhere) and inverse real FFT (complex FFT of length F/2).
template <typename R>
__device__ void dev_row_c2r(unsigned char* smem_raw, const LevelGeom& g, const cplx<R>* __restrict__ spec2,
                            const cplx<R>* __restrict__ tw, R* __restrict__ out, int unit)
{
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int N = F >> 1;
    const int logN = g.logF - 1;
    const int M = g.M;
    const int row = unit;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        cplx<R> a = {R(0), R(0)};
        cplx<R> b = {R(0), R(0)};
        if (k <= M) a = spec2[(size_t)k * F + row];
        const int kk = N - k;
        if (kk <= M) b = spec2[(size_t)kk * F + row];
        const R ex = a.x + b.x, ey = a.y - b.y;       // X[k] + conj(X[N-k])
        const R dx = a.x - b.x, dy = a.y + b.y;       // X[k] - conj(X[N-k])
        const cplx<R> wk = tw[k];                     // exp(-2 pi i k/F); use its conjugate
        const R ox = dx * wk.x + dy * wk.y;
        const R oy = dy * wk.x - dx * wk.y;
        z[bitrev(k, logN)] = {ex - oy, ey + ox};      // E + i O
    }
    __syncthreads();
    lds_fft(z, logN, tw, 2, true);
    R* o = out + (size_t)row * F;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const cplx<R> v = z[n];
        o[2 * n] = v.x;
        o[2 * n + 1] = v.y;
    }
}

// ---------------------------------------------------------------------------
// Interpolation (type-2, Sec. 3 Step 4 via the NUFFT): one workgroup per tile
// stages the (T+w-1)^2 grid window in LDS; each thread evaluates one target.
template <typename R, int W>
__device__ void dev_interp(unsigned char* smem_raw, const LevelGeom& g, const R* __restrict__ grid,
                           const RecView<R>& L, R* __restrict__ hist, const double* __restrict__ coef, int t)
{
    const int* __restrict__ start = L.start;
    const int* __restrict__ ij = L.ij;
    const R* __restrict__ sx = L.dx;
    const R* __restrict__ sy = L.dy;
    const int* __restrict__ idx = L.idx;
    R* reg = reinterpret_cast<R*>(smem_raw);
    const int T = g.T;
    const int E = T + W - 1;
    const int F = g.F;
    const int r0 = start[t];
    const int r1 = start[t + 1];
    if (r0 == r1) return;
    const int gx0 = (t % g.ntx) * T;
    const int gy0 = (t / g.ntx) * T;
    for (int i = threadIdx.x; i < E * E; i += blockDim.x) {
        const int y = i / E;
        const int x = i - y * E;
        const int gy = gy0 + y;
        const int gx = gx0 + x;
        reg[i] = (gx < F && gy < F) ? grid[(size_t)gy * F + gx] : R(0);
    }
    __syncthreads();
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const int p = ij[r];
        const int i0 = (p & 0xffff) - gx0;
        const int j0 = (p >> 16) - gy0;
        double px[W], py[W];
        kernel_taps<W>((double)sx[r], coef, px);
        kernel_taps<W>((double)sy[r], coef, py);
        R sum = R(0);
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const R* rowp = reg + (j0 + b) * E + i0;
            R acc = R(0);
#pragma unroll
            for (int a = 0; a < W; ++a) acc += (R)px[a] * rowp[a];
            sum += (R)py[b] * acc;
        }
        hist[idx[r]] = sum;
    }
}

// ---------------------------------------------------------------------------
// Local part (Sec. 4) and final float64 sum.  Expansions in c = r/sqrt(delta):
//   V_L: Lemma 4.5 with the delta^{3/2} factor (2 f_eta - kappa f);
//   S_L, D_L: Lemmas 4.1, 4.3 with the overall sign reversed (positive heat
//   kernel, outward normal, interior jump -mu/2).
// Beyond c = 12 the layer parts vanish and V_L = delta f + delta^2 lap f / 2.
struct LocalArgs {
    int64_t n;
    double delta;
    int order_v, order_s, order_d;
    const double* r;
    const double* nx;
    const double* ny;
    const double* kappa;
    const double* g3;
    const double* g4;
    const int8_t* sgn;
    const double* jet6;
    const double* sj;
    const double* mj;
    const void* h0;
    const void* h1;
    int fp32;
    double dc_weight;        // sum over levels of the zero-mode weight (float32 path)
    const double* dc;        // float64 sum of channel-0 strengths
    double* out;
};

__device__ __forceinline__ double hist_at(const void* h, int fp32, int64_t i)
{
    return fp32 ? (double)((const float*)h)[i] : ((const double*)h)[i];
}

__device__ void dev_local(const LocalArgs& a, int64_t i)
{
    if (i >= a.n) return;
    const double SQPI = 1.7724538509055160273;
    const double d = a.delta;
    const double sd = sqrt(d);
    const double r = a.r[i];
    const double c = r / sd;
    const bool near = c <= 12.0;
    const double kap = a.kappa[i];
    const double g3 = a.g3 ? a.g3[i] : 0.0;
    const double g4 = a.g4 ? a.g4[i] : 0.0;
    const double sg = (double)a.sgn[i];
    const double E = erfc(0.5 * c);
    const double e = exp(-0.25 * c * c);
    const double c2 = c * c, c3 = c2 * c;
    double u = hist_at(a.h0, a.fp32, i) + hist_at(a.h1, a.fp32, i);
    if (a.dc) u += a.dc_weight * (*a.dc);
    const int64_t n = a.n;
    if (a.jet6) {
        const double f = a.jet6[i], fx = a.jet6[n + i], fy = a.jet6[2 * n + i];
        const double fxx = a.jet6[3 * n + i], fxy = a.jet6[4 * n + i], fyy = a.jet6[5 * n + i];
        const double lap = fxx + fyy;
        double v = 0.0;
        if (!near) {
            if (a.order_v >= 2) v += d * f;
            if (a.order_v >= 4) v += 0.5 * d * d * lap;
        } else {
            const double ex = -a.nx[i], ey = -a.ny[i];     // inward normal (eta)
            const double tx = a.ny[i], ty = -a.nx[i];      // tangent (xi), sign irrelevant
            const double fe = fx * ex + fy * ey;
            const double fee = fxx * ex * ex + 2.0 * fxy * ex * ey + fyy * ey * ey;
            const double ftt = fxx * tx * tx + 2.0 * fxy * tx * ty + fyy * ty * ty;
            if (a.order_v >= 2)
                v += 0.25 * d * (2.0 * erf(0.5 * c) + 2.0 * e * c / SQPI - c2 * E + 2.0) * f;
            if (a.order_v >= 3)
                v += d * sd * ((4.0 - 2.0 * c2) * e + SQPI * c3 * E) * (2.0 * fe - kap * f) / (12.0 * SQPI);
            if (a.order_v >= 4) {
                const double c4 = c2 * c2;
                v += d * d / 48.0 *
                     (E * (4.0 * c4 * kap * fe - 3.0 * (c4 + 4.0) * fee + (c4 - 12.0) * ftt - 3.0 * c4 * kap * kap * f) +
                      2.0 * c * (c2 - 2.0) * e * (-4.0 * kap * fe + 3.0 * fee - ftt + 3.0 * kap * kap * f) / SQPI +
                      24.0 * (ftt + fee));
            }
        }
        u += v;
    }
    if (near && a.sj) {
        const double s0 = a.sj[i], s1 = a.sj[n + i], s2 = a.sj[2 * n + i];
        const double P1 = c * E - 2.0 * e / SQPI;
        const double Q = 2.0 * (c2 - 2.0) * e / SQPI - c3 * E;
        double s = 0.0;
        if (a.order_s >= 1) s += sd * 0.5 * s0 * P1;
        if (a.order_s >= 2) s += sg * d * c * kap * s0 * 0.25 * P1;
        if (a.order_s >= 3)
            s += d * sd * (s0 * kap * kap / 12.0 * (2.0 * c3 * E - (4.0 * c2 + 1.0) * e / SQPI) + s2 / 12.0 * Q);
        if (a.order_s >= 4)
            s += d * d * sg *
                 (c * kap * kap * kap * s0 / 16.0 * (3.0 * c3 * E - (6.0 * c2 - 2.0) * e / SQPI) +
                  c * kap * s2 / 8.0 * Q + c * s0 * g4 / 48.0 * Q + c * s1 * g3 / 12.0 * Q);
        u -= s;
    }
    if (near && a.mj) {
        const double m0 = a.mj[i], m1 = a.mj[n + i], m2 = a.mj[2 * n + i], m4 = a.mj[4 * n + i];
        double s = sg * 0.5 * m0 * E;
        if (a.order_d >= 1) s += sd * kap * m0 / (2.0 * SQPI) * e;
        if (a.order_d >= 2) s += d * sg * (3.0 * c * kap * kap * m0 / (8.0 * SQPI) * e + c * m2 * 0.25 * (2.0 * e / SQPI - c * E));
        const double A = 2.0 * (c2 + 1.0) * e / SQPI - c3 * E;
        const double B = 2.0 * (c2 + 4.0) * e / SQPI - c3 * E;
        if (a.order_d >= 3)
            s += d * sd * (5.0 * (c2 - 2.0) * kap * kap * kap * m0 / (16.0 * SQPI) * e + g4 * m0 / (4.0 * SQPI) * e +
                           kap * m2 * 0.25 * A + g3 * m1 / 12.0 * B);
        if (a.order_d >= 4) {
            s += d * d * sg *
                 (35.0 * c * kap * kap * kap * kap * m0 * (c2 - 6.0) / (128.0 * SQPI) * e +
                  5.0 * c * g3 * g3 * m0 / (12.0 * SQPI) * e + 5.0 * c * kap * g4 * m0 / (8.0 * SQPI) * e);
            s += d * d * sg * 5.0 * c * (kap * kap * m2 / 16.0 * A + kap * g3 * m1 / 24.0 * B);
            s += d * d * sg * c * m4 / 48.0 * (c3 * E - 2.0 * (c2 - 2.0) * e / SQPI);
        }
        u -= s;
    }
    a.out[i] = u;
}

}  // namespace dev
}  // namespace vp
