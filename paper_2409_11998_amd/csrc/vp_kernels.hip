// HIP kernels for gfx950: strengths, spread, 2-D FFT with the history
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

namespace {

// Exponential-of-semicircle spreading kernel exp(beta (sqrt(1 - z^2) - 1)) on
// |z| < 1, written as exp(-beta z^2 / (1 + sqrt(1 - z^2))): the direct form
// loses the exponent to cancellation near z = 0, where the kernel is largest.
// Tap a of a node with fractional offset d in [0,1) sits at
// z = ((2a - w) + 2d) / w.  Only 2w values are needed per node, so they are
// always evaluated in float64 (the exponent reaches beta ~ 20-35, and its
// float32 rounding would cost ~1e-7 relative per tap) and rounded once to the
// working precision for the w^2 products and sums.
template <typename R>
__device__ __forceinline__ R es_tap(int a, int w, R d, double beta, double inv_w)
{
    const double z = ((double)(2 * a - w) + 2.0 * (double)d) * inv_w;
    const double z2 = z * z;
    const double q = 1.0 - z2;
    return q > 0.0 ? (R)exp(-beta * z2 / (1.0 + sqrt(q))) : R(0);
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
template <typename R>
__global__ __launch_bounds__(kThreads) void k_strengths(int64_t n_src, int64_t n_bnd, const double* __restrict__ f,
                                                        const double* __restrict__ sigma, const double* __restrict__ mu,
                                                        const double* __restrict__ w, const double* __restrict__ nx,
                                                        const double* __restrict__ ny, R* __restrict__ str, int C,
                                                        double* __restrict__ dc)
{
    const int64_t n = n_src + n_bnd;
    double part = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
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
    __shared__ double red[kThreads];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(dc, red[0]);
}

__global__ void k_zero_dc(double* dc) { if (threadIdx.x == 0 && blockIdx.x == 0) *dc = 0.0; }

// ---------------------------------------------------------------------------
// Spread (type-1 spreading, Sec. 3 Step 2 via the NUFFT): one workgroup owns a
// T x T tile of the fine grid, accumulates in LDS the contributions of every
// node whose w x w support meets the tile, and writes the tile once (no
// global atomics, no zero-fill pass).  A node's support starts at grid index
// i0 = ceil(t - w/2); its offset is stored as d = i0 - t + w/2 in [0, 1).
template <typename R, int C>
__global__ __launch_bounds__(kThreads) void k_spread(LevelGeom g, const int* __restrict__ start,
                                                     const int* __restrict__ ij, const R* __restrict__ sx,
                                                     const R* __restrict__ sy, const int* __restrict__ idx,
                                                     const R* __restrict__ str, int64_t nstr, R* __restrict__ grid)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* tile = reinterpret_cast<R*>(smem_raw);
    const int T = g.T;
    const int TT = T * T;
    const int t = blockIdx.x;
    const int gx0 = (t % g.ntx) * T;
    const int gy0 = (t / g.ntx) * T;
    for (int i = threadIdx.x; i < C * TT; i += blockDim.x) tile[i] = R(0);
    __syncthreads();
    const double beta = g.beta;
    const double inv_w = 1.0 / g.w;
    const int w = g.w;
    const int r1 = start[t + 1];
    for (int r = start[t] + threadIdx.x; r < r1; r += blockDim.x) {
        const int p = ij[r];
        const int i0 = (p & 0xffff) - gx0;
        const int j0 = (p >> 16) - gy0;
        const R ox = sx[r];
        const R oy = sy[r];
        const int k = idx[r];
        R s[C];
#pragma unroll
        for (int c = 0; c < C; ++c) s[c] = str[c * nstr + k];
        R px[kWMax], py[kWMax];
#pragma unroll
        for (int a = 0; a < kWMax; ++a) {
            px[a] = a < w ? es_tap(a, w, ox, beta, inv_w) : R(0);
            py[a] = a < w ? es_tap(a, w, oy, beta, inv_w) : R(0);
        }
#pragma unroll
        for (int b = 0; b < kWMax; ++b) {
            const int y = j0 + b;
            if (b >= w || y < 0 || y >= T) continue;
#pragma unroll
            for (int a = 0; a < kWMax; ++a) {
                const int x = i0 + a;
                if (a >= w || x < 0 || x >= T) continue;
                const R v = px[a] * py[b];
#pragma unroll
                for (int c = 0; c < C; ++c) atomicAdd(&tile[c * TT + y * T + x], s[c] * v);
            }
        }
    }
    __syncthreads();
    const size_t F = g.F;
    for (int i = threadIdx.x; i < C * TT; i += blockDim.x) {
        const int c = i / TT;
        const int l = i - c * TT;
        const int y = l / T;
        const int x = l - y * T;
        grid[(size_t)c * F * F + (size_t)(gy0 + y) * F + gx0 + x] = tile[i];
    }
}

// ---------------------------------------------------------------------------
// Row pass: real FFT along x of each row (length F via a complex FFT of length
// F/2), keeping only x-frequencies 0..M.  Output spec[c][m1][row] so that the
// column pass reads contiguous columns.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_row_r2c(LevelGeom g, const R* __restrict__ grid,
                                                      const cplx<R>* __restrict__ tw, cplx<R>* __restrict__ spec)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int N = F >> 1;
    const int logN = g.logF - 1;
    const int M = g.M;
    const int row = blockIdx.x % F;
    const int c = blockIdx.x / F;
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
// Column pass for x-frequency m1 = blockIdx.x: FFT along y of each channel,
// combine B0 - i k1 B1 - i k2 B2 (double layer: derivative of the kernel in
// the source variable), multiply by the level's table, inverse FFT along y.
template <typename R, int C>
__global__ __launch_bounds__(kThreads) void k_col(LevelGeom g, const cplx<R>* __restrict__ spec,
                                                  const R* __restrict__ mult, const cplx<R>* __restrict__ tw,
                                                  cplx<R>* __restrict__ spec2, int zero_dc)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    constexpr int PER = 8192 / kThreads;
    const int F = g.F;
    const int logF = g.logF;
    const int M = g.M;
    const int m1 = blockIdx.x;
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
__global__ __launch_bounds__(kThreads) void k_row_c2r(LevelGeom g, const cplx<R>* __restrict__ spec2,
                                                      const cplx<R>* __restrict__ tw, R* __restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int N = F >> 1;
    const int logN = g.logF - 1;
    const int M = g.M;
    const int row = blockIdx.x;
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
template <typename R>
__global__ __launch_bounds__(kThreads) void k_interp(LevelGeom g, const R* __restrict__ grid,
                                                     const int* __restrict__ start, const int* __restrict__ ij,
                                                     const R* __restrict__ sx, const R* __restrict__ sy,
                                                     const int* __restrict__ idx, R* __restrict__ hist)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* reg = reinterpret_cast<R*>(smem_raw);
    const int T = g.T;
    const int w = g.w;
    const int E = T + w - 1;
    const int F = g.F;
    const int t = blockIdx.x;
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
    const double beta = g.beta;
    const double inv_w = 1.0 / w;
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const int p = ij[r];
        const int i0 = (p & 0xffff) - gx0;
        const int j0 = (p >> 16) - gy0;
        const R ox = sx[r];
        const R oy = sy[r];
        R px[kWMax], py[kWMax];
#pragma unroll
        for (int a = 0; a < kWMax; ++a) {
            px[a] = a < w ? es_tap(a, w, ox, beta, inv_w) : R(0);
            py[a] = a < w ? es_tap(a, w, oy, beta, inv_w) : R(0);
        }
        R sum = R(0);
#pragma unroll
        for (int b = 0; b < kWMax; ++b) {
            if (b < w) {
                const R* rowp = reg + (j0 + b) * E + i0;
                R acc = R(0);
#pragma unroll
                for (int a = 0; a < kWMax; ++a)
                    if (a < w) acc += px[a] * rowp[a];
                sum += py[b] * acc;
            }
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

__global__ __launch_bounds__(kThreads) void k_local(LocalArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    return (size_t)(p.lv[level].F / 2) * cb;
}

size_t col_fft_lds_bytes(const Plan& p, int level)
{
    const size_t cb = p.precision == VP_FP32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    return (size_t)p.lv[level].F * cb;
}

hipError_t launch_zero_dc(Plan& p)
{
    hipLaunchKernelGGL(k_zero_dc, dim3(1), dim3(64), 0, p.stream, p.d_dc);
    return hipGetLastError();
}

hipError_t launch_strengths(Plan& p, const double* f, const double* sigma, const double* mu, int C)
{
    const int64_t n = p.n_src + p.n_bnd;
    unsigned blocks = grid_for(n);
    if (blocks > 4096) blocks = 4096;
    if (p.precision == VP_FP32)
        hipLaunchKernelGGL(k_strengths<float>, dim3(blocks), dim3(kThreads), 0, p.stream, p.n_src, p.n_bnd, f, sigma,
                           mu, p.d_w, p.d_nx, p.d_ny, (float*)p.d_str, C, p.d_dc);
    else
        hipLaunchKernelGGL(k_strengths<double>, dim3(blocks), dim3(kThreads), 0, p.stream, p.n_src, p.n_bnd, f, sigma,
                           mu, p.d_w, p.d_nx, p.d_ny, (double*)p.d_str, C, p.d_dc);
    return hipGetLastError();
}

template <typename R>
static hipError_t spread_t(Plan& p, int l, int C)
{
    const LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    const unsigned ntiles = (unsigned)(g.ntx * g.ntx);
    const size_t lds = (size_t)C * g.T * g.T * sizeof(R);
    const int64_t nstr = p.n_src + p.n_bnd;
    if (C == 1)
        hipLaunchKernelGGL((k_spread<R, 1>), dim3(ntiles), dim3(kThreads), lds, p.stream, g, b.src_start, b.src_ij,
                           (const R*)b.src_sx, (const R*)b.src_sy, b.src_idx, (const R*)p.d_str, nstr, (R*)b.grid);
    else
        hipLaunchKernelGGL((k_spread<R, 3>), dim3(ntiles), dim3(kThreads), lds, p.stream, g, b.src_start, b.src_ij,
                           (const R*)b.src_sx, (const R*)b.src_sy, b.src_idx, (const R*)p.d_str, nstr, (R*)b.grid);
    return hipGetLastError();
}

hipError_t launch_spread(Plan& p, int level, int C)
{
    return p.precision == VP_FP32 ? spread_t<float>(p, level, C) : spread_t<double>(p, level, C);
}

template <typename R>
static hipError_t row_fft_t(Plan& p, int l, int C)
{
    const LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    hipLaunchKernelGGL(k_row_r2c<R>, dim3(g.F * C), dim3(kThreads), row_fft_lds_bytes(p, l), p.stream, g,
                       (const R*)b.grid, (const cplx<R>*)b.tw, (cplx<R>*)b.spec);
    return hipGetLastError();
}

hipError_t launch_row_fft(Plan& p, int level, int C)
{
    return p.precision == VP_FP32 ? row_fft_t<float>(p, level, C) : row_fft_t<double>(p, level, C);
}

template <typename R>
static hipError_t col_fft_t(Plan& p, int l, int C)
{
    const LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    const int zero_dc = p.precision == VP_FP32 ? 1 : 0;
    if (C == 1)
        hipLaunchKernelGGL((k_col<R, 1>), dim3(g.M + 1), dim3(kThreads), col_fft_lds_bytes(p, l), p.stream, g,
                           (const cplx<R>*)b.spec, (const R*)b.mult, (const cplx<R>*)b.tw, (cplx<R>*)b.spec2, zero_dc);
    else
        hipLaunchKernelGGL((k_col<R, 3>), dim3(g.M + 1), dim3(kThreads), col_fft_lds_bytes(p, l), p.stream, g,
                           (const cplx<R>*)b.spec, (const R*)b.mult, (const cplx<R>*)b.tw, (cplx<R>*)b.spec2, zero_dc);
    return hipGetLastError();
}

hipError_t launch_col_fft(Plan& p, int level, int C)
{
    return p.precision == VP_FP32 ? col_fft_t<float>(p, level, C) : col_fft_t<double>(p, level, C);
}

template <typename R>
static hipError_t row_ifft_t(Plan& p, int l)
{
    const LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    hipLaunchKernelGGL(k_row_c2r<R>, dim3(g.F), dim3(kThreads), row_fft_lds_bytes(p, l), p.stream, g,
                       (const cplx<R>*)b.spec2, (const cplx<R>*)b.tw, (R*)b.grid);
    return hipGetLastError();
}

hipError_t launch_row_ifft(Plan& p, int level)
{
    return p.precision == VP_FP32 ? row_ifft_t<float>(p, level) : row_ifft_t<double>(p, level);
}

template <typename R>
static hipError_t interp_t(Plan& p, int l)
{
    const LevelGeom& g = p.lv[l];
    LevelBufs& b = p.lb[l];
    const int E = g.T + g.w - 1;
    const size_t lds = (size_t)E * E * sizeof(R);
    hipLaunchKernelGGL(k_interp<R>, dim3(g.ntx * g.ntx), dim3(kThreads), lds, p.stream, g, (const R*)b.grid,
                       b.tgt_start, b.tgt_ij, (const R*)b.tgt_sx, (const R*)b.tgt_sy, b.tgt_idx, (R*)b.hist);
    return hipGetLastError();
}

hipError_t launch_interp(Plan& p, int level)
{
    return p.precision == VP_FP32 ? interp_t<float>(p, level) : interp_t<double>(p, level);
}

hipError_t launch_local(Plan& p, const double* jet6, const double* sig_jet, const double* mu_jet, bool use_v,
                        bool use_s, bool use_d, double* out)
{
    LocalArgs a{};
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
    a.h0 = p.lb[0].hist;
    a.h1 = p.lb[1].hist;
    a.fp32 = p.precision == VP_FP32;
    a.dc_weight = p.lv[0].dc_coef + p.lv[1].dc_coef;
    a.dc = a.fp32 ? p.d_dc : nullptr;
    a.out = out;
    if (p.n_tgt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_local, dim3(grid_for(p.n_tgt)), dim3(kThreads), 0, p.stream, a);
    return hipGetLastError();
}

}  // namespace vp
