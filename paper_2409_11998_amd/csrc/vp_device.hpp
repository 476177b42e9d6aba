#pragma once
// Device code shared by the per-plan kernels (vp_kernels.hip) and the batched
// group kernels (vp_batch.hip) for gfx950: strengths, spread, 2-D FFT with the history
// multiplier fused into the column pass, interpolation, local part.
//
// Data flow of one evaluation (history part, Sec. 3 Steps 1-4; local part,
// Sec. 4), per level (near history NH, far history FH):
//
//   strengths  c_j per node (and mu nu wG)       k_strengths
//   spread     b[g] = sum_j c_j phi(g - t_j)     k_spread     (LDS tile windows, global atomics)
//              + mu_j nu_j . grad_y phi(g - t_j)
//   row FFT    along x, real -> half spectrum    k_row_r2c    (keeps |m1| <= M only)
//   column     along y: FFT, multiply by         k_col        (in place)
//              (dk/2pi)^2 M(k)/phihat^2, IFFT
//   row IFFT   half spectrum -> real              k_row_c2r
//   interp     u(x_i) = sum_g a[g] phi(t_i - g)  k_interp     (tile grid staged in LDS)
//   local      V_L + S_L + D_L + history sum     k_local      (float64)
//
// Both FFTs are unnormalized (forward exp(-2 pi i), inverse exp(+2 pi i)); all
// constants live in the multiplier table built by the planner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "vp_internal.hpp"

namespace vp {
namespace dev {


// XCD-aware unit order.  Workgroups are dealt round-robin to the 8 XCDs
// (each with its own L2), so consecutive block indices land on different
// XCDs.  Giving each XCD a contiguous range of units (rows, columns, tiles)
// keeps neighbouring units -- which share cache lines of the strided spectrum
// and the tiles' overlapping windows -- in one L2.  Identity when n is not a
// multiple of 8.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_unit(int b, int n)
{
    if (n % kXcds) return b;
    return (b % kXcds) * (n / kXcds) + b / kXcds;
}

__device__ __forceinline__ int bitrev(int k, int logn)
{
    return logn ? (int)(__brev((unsigned)k) >> (32 - logn)) : 0;
}

// LDS FFT arrays are padded by one element per 32: bit-reversed and
// power-of-two strided accesses would otherwise put a whole wavefront on a
// few of the 64 LDS banks.  (Measured on the square workload against one per
// 16, one per 8, one per 4 and an XOR swizzle: the same row passes, and float64
// column passes 0.033 / 0.024 ms against 0.037 / 0.027 ms.)
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 5); }
__host__ __device__ constexpr int lds_padded_len(int n) { return n + (n >> 5); }

// Complex helpers of the LDS FFTs.
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> w)
{
    return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> twiddle(const cplx<R>* __restrict__ tw, int k, bool inverse)
{
    cplx<R> w = tw[k];
    if (inverse) w.y = -w.y;
    return w;
}

// In-place radix-2 decimation-in-time FFT of n = 2^logn points held in LDS in
// bit-reversed order; output in natural order.  tw[k*tw_stride] =
// exp(-2 pi i k / n) for k < n/2.  Ends with a barrier.
//
// Stage s combines pairs half = 2^(s-1) apart with twiddle tw[pos (n >> s)].
// Two consecutive stages run as one pass over quads (i, i+h, i+2h, i+3h),
// h = 2^(s-1): the same butterflies, twiddles and order, with half the
// barriers and half the LDS traffic; an odd last stage runs alone.
template <typename R>
__device__ void lds_fft(cplx<R>* a, int logn, const cplx<R>* __restrict__ tw, int tw_stride, bool inverse)
{
    const int n = 1 << logn;
    int s = 1;
    for (; s + 1 <= logn; s += 2) {
        const int h = 1 << (s - 1);
        const int st1 = (n >> s) * tw_stride;        // stage s
        const int st2 = (n >> (s + 1)) * tw_stride;  // stage s + 1
        for (int q = threadIdx.x; q < (n >> 2); q += blockDim.x) {
            const int pos = q & (h - 1);
            const int i = ((q >> (s - 1)) << (s + 1)) + pos;
            const cplx<R> w1 = twiddle(tw, pos * st1, inverse);
            cplx<R> e0 = a[lds_pad(i)], e1 = a[lds_pad(i + h)], e2 = a[lds_pad(i + 2 * h)], e3 = a[lds_pad(i + 3 * h)];
            cplx<R> t = cmul(e1, w1);
            e1 = {e0.x - t.x, e0.y - t.y};
            e0 = {e0.x + t.x, e0.y + t.y};
            t = cmul(e3, w1);
            e3 = {e2.x - t.x, e2.y - t.y};
            e2 = {e2.x + t.x, e2.y + t.y};
            const cplx<R> w2a = twiddle(tw, pos * st2, inverse);
            const cplx<R> w2b = twiddle(tw, (pos + h) * st2, inverse);
            t = cmul(e2, w2a);
            a[lds_pad(i)] = {e0.x + t.x, e0.y + t.y};
            a[lds_pad(i + 2 * h)] = {e0.x - t.x, e0.y - t.y};
            t = cmul(e3, w2b);
            a[lds_pad(i + h)] = {e1.x + t.x, e1.y + t.y};
            a[lds_pad(i + 3 * h)] = {e1.x - t.x, e1.y - t.y};
        }
        __syncthreads();
    }
    if (s == logn) {
        const int half = 1 << (s - 1);
        const int step = (n >> s) * tw_stride;
        for (int b = threadIdx.x; b < (n >> 1); b += blockDim.x) {
            const int pos = b & (half - 1);
            const int i = ((b >> (s - 1)) << s) + pos;
            const int j = i + half;
            const cplx<R> t = cmul(a[lds_pad(j)], twiddle(tw, pos * step, inverse));
            const cplx<R> u = a[lds_pad(i)];
            a[lds_pad(i)] = {u.x + t.x, u.y + t.y};
            a[lds_pad(j)] = {u.x - t.x, u.y - t.y};
        }
        __syncthreads();
    }
}

// In-place radix-2 decimation-in-frequency FFT: input in natural order, output
// in bit-reversed order (same twiddle convention as lds_fft).  Stages run from
// s = logn down to 1 (pairs 2^(s-1) apart: sum, and difference times
// tw[pos (n >> s)]), two consecutive stages per pass as in lds_fft.  Ends with
// a barrier.
template <typename R>
__device__ void lds_fft_dif(cplx<R>* a, int logn, const cplx<R>* __restrict__ tw, int tw_stride, bool inverse)
{
    const int n = 1 << logn;
    int s = logn;
    for (; s - 1 >= 1; s -= 2) {
        const int h = 1 << (s - 2);                  // half of stage s - 1
        const int st1 = (n >> s) * tw_stride;        // stage s (pairs 2h apart)
        const int st2 = (n >> (s - 1)) * tw_stride;  // stage s - 1 (pairs h apart)
        for (int q = threadIdx.x; q < (n >> 2); q += blockDim.x) {
            const int pos = q & (h - 1);
            const int i = ((q >> (s - 2)) << s) + pos;
            cplx<R> e0 = a[lds_pad(i)], e1 = a[lds_pad(i + h)], e2 = a[lds_pad(i + 2 * h)], e3 = a[lds_pad(i + 3 * h)];
            const cplx<R> wa = twiddle(tw, pos * st1, inverse);
            const cplx<R> wb = twiddle(tw, (pos + h) * st1, inverse);
            cplx<R> d = {e0.x - e2.x, e0.y - e2.y};
            e0 = {e0.x + e2.x, e0.y + e2.y};
            e2 = cmul(d, wa);
            d = {e1.x - e3.x, e1.y - e3.y};
            e1 = {e1.x + e3.x, e1.y + e3.y};
            e3 = cmul(d, wb);
            const cplx<R> w2 = twiddle(tw, pos * st2, inverse);
            d = {e0.x - e1.x, e0.y - e1.y};
            a[lds_pad(i)] = {e0.x + e1.x, e0.y + e1.y};
            a[lds_pad(i + h)] = cmul(d, w2);
            d = {e2.x - e3.x, e2.y - e3.y};
            a[lds_pad(i + 2 * h)] = {e2.x + e3.x, e2.y + e3.y};
            a[lds_pad(i + 3 * h)] = cmul(d, w2);
        }
        __syncthreads();
    }
    if (s == 1) {
        for (int b = threadIdx.x; b < (n >> 1); b += blockDim.x) {
            const int i = b << 1;  // half = 1, pos = 0: twiddle tw[0] = 1
            const cplx<R> u = a[lds_pad(i)];
            const cplx<R> v = a[lds_pad(i + 1)];
            const cplx<R> w = twiddle(tw, 0, inverse);
            a[lds_pad(i)] = {u.x + v.x, u.y + v.y};
            a[lds_pad(i + 1)] = cmul(cplx<R>{u.x - v.x, u.y - v.y}, w);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Strengths per node (the sums of Sec. 3, Step 2):
//   str[i]               = f w (volume node) or sigma wG (boundary node),
//   str[n + j]           = mu nu1 wG,   str[n + nb + j] = mu nu2 wG
// for boundary node j (n = all nodes, nb = boundary nodes; present only when
// mu is given).  Also accumulates sum(str[0..n)) in float64 (the
// zero-frequency term).
// Nodes per thread of a strengths work unit: float32 plans reduce strength
// maxima (and the zero-frequency sum) by one atomic per unit, so their units
// stay long; float64 plans reduce nothing and use short units (more of them in
// flight).  Loads go out kStrBatch nodes at a time.
constexpr int kStrBatch = 4;
template <typename R> __host__ __device__ constexpr int str_per() { return sizeof(R) == 4 ? 16 : 4; }
template <typename R> __host__ __device__ constexpr int str_chunk() { return kThreads * str_per<R>(); }

template <typename R>
__device__ void dev_strengths(int64_t n_src, int64_t n_bnd, const double* __restrict__ f,
                              const double* __restrict__ sigma, const double* __restrict__ mu,
                              const double* __restrict__ w, const double* __restrict__ nx,
                              const double* __restrict__ ny, R* __restrict__ str, double* __restrict__ dc,
                              unsigned long long* __restrict__ smax, int64_t unit)
{
    const int64_t n = n_src + n_bnd;
    double part = 0.0, m0 = 0.0, m1 = 0.0;
    constexpr int NB = str_per<R>() / kStrBatch;
    const int64_t i1 = min(n, (unit + 1) * (int64_t)str_chunk<R>());
    for (int bt = 0; bt < NB; ++bt) {
    const int64_t ib = unit * (int64_t)str_chunk<R>() + (int64_t)bt * kStrBatch * blockDim.x + threadIdx.x;
    double wv[kStrBatch], dv[kStrBatch];
#pragma unroll
    for (int k = 0; k < kStrBatch; ++k) {
        const int64_t i = ib + (int64_t)k * blockDim.x;
        wv[k] = 0.0;
        dv[k] = 0.0;
        if (i < i1) {
            wv[k] = w[i];
            if (i < n_src) {
                if (f) dv[k] = f[i];
            } else if (sigma) {
                dv[k] = sigma[i - n_src];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kStrBatch; ++k) {
        const int64_t i = ib + (int64_t)k * blockDim.x;
        if (i >= i1) break;
        const double s0 = dv[k] * wv[k];
        if (i >= n_src && mu) {
            const int64_t j = i - n_src;
            const double m = mu[j] * wv[k];
            const R gx = (R)(m * nx[j]), gy = (R)(m * ny[j]);
            str[n + j] = gx;
            str[n + n_bnd + j] = gy;
            m1 = fmax(m1, fabs((double)gx) + fabs((double)gy));
        }
        const R sr = (R)s0;
        str[i] = sr;
        part += s0;
        m0 = fmax(m0, fabs((double)sr));
    }
    }
    // workgroup reductions (wavefront shuffles, then LDS): the zero-frequency sum
    // (one float64 atomic per unit into one of kDcParts partial sums) and the
    // strength maxima the spread scales its fixed-point windows by (unsigned
    // atomic max on the bit patterns of non-negative doubles)
    __shared__ double red[3][kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) {
        part += __shfl_xor(part, o);
        m0 = fmax(m0, __shfl_xor(m0, o));
        m1 = fmax(m1, __shfl_xor(m1, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = part;
        red[1][threadIdx.x >> 6] = m0;
        red[2][threadIdx.x >> 6] = m1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, a = 0.0, b = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            t += red[0][k];
            a = fmax(a, red[1][k]);
            b = fmax(b, red[2][k]);
        }
        if (dc && t != 0.0) atomicAdd(dc + (unit % kDcParts), t);
        if (smax && a > 0.0) atomicMax(smax + (unit % kDcParts), (unsigned long long)__double_as_longlong(a));
        if (smax && b > 0.0)
            atomicMax(smax + kDcParts + (unit % kDcParts), (unsigned long long)__double_as_longlong(b));
    }
    __syncthreads();
}

// Zero fill of a spread grid (the spread accumulates into it with atomics).
template <typename R>
__device__ void dev_zero(R* __restrict__ p, int64_t n, int64_t i)
{
    if (i < n) p[i] = R(0);
}

// ---------------------------------------------------------------------------
// Spread (type-1 spreading, Sec. 3 Step 2 via the NUFFT).
//
// Every node is assigned to the T x T tile holding its support corner
// i0 = ceil(t - w/2) (its offset is stored as d = i0 - t + w/2 in [0, 1)), so
// its whole w x w support lies inside the tile's extended window of
// (T+w-1)^2 cells.  One workgroup accumulates a tile's window in LDS and adds
// the window to the grid with global atomics (the grid is zeroed first); the
// windows of neighbouring tiles overlap by w-1 cells.
//
// Window accumulation (measured on gfx950, cycles per 64-lane LDS atomic per
// CU: ds_add_u32 4.4, ds_add_u64 6.5, ds_add_f64 8.5, ds_add_f32 ~190):
//  - float64 plans: float64 atomics;
//  - float32 plans: 64-bit fixed point (int64 atomics).  Integer sums are
//    exact and independent of the order of the atomics.  Each unit's scale
//    comes from a bound on its window values, cover * max contribution, where
//    cover (from the planner) is the most records of the unit sharing one cell
//    and the maximum contribution follows from the evaluation's largest
//    strengths (|phi| <= 1, |d phi/dy| <= dmax); a contribution v becomes
//    round(v q) with q = 2^49 / bound.  The double-layer terms make the bound
//    up to ~1e4 times the volume contributions near a boundary; the 49-bit
//    range still resolves those to ~1e-11, far below float32 rounding (a
//    32-bit window, with 29 bits, would not).
//
// Single-strength nodes (volume nodes, and boundary nodes without a double
// layer): each wavefront takes chunks of 32 of the tile's nodes; lane pairs
// evaluate the kernel values of one node (x taps and y taps) into LDS, then
// the wavefront walks the chunk node by node with the 64 lanes mapped to taps
// (lane -> column a = lane % w, rows b = lane / w + k (64 / w)).  The next
// node's values are read before the current node's atomics are issued, and
// the node's corner and strength come from registers (readlane), so the loop
// keeps several LDS operations in flight.
//
// Double layer (Sec. 3, Step 2; Sec. 2.1): the transform factor -i k of the
// double-layer kernel is applied in space, by spreading mu nu . grad_y phi
// (the gradient of the spreading kernel in the source position) into the same
// grid: its Fourier transform is phihat(k) (-i k . nu mu) exp(-i k.y), which
// is exactly the double-layer term of the combined spectrum.  These boundary
// nodes take the same wavefront path with the tap derivatives staged beside
// the tap values.
template <typename R> struct SpreadShape {
    static constexpr int kWaves = kThreads / 64;
    // nodes per wavefront chunk (half as many double-layer nodes, which stage
    // twice the values); sized so that four workgroups fit in LDS
    static constexpr int kRecs = sizeof(R) == 4 ? 32 : 16;
};

__host__ __device__ inline int spread_pitch(int T, int W)
{
    const int E = T + W - 1;
    return E | 1;  // odd pitch: consecutive rows start in different LDS banks
}

// Dynamic LDS layout of the spread (bytes): window of 8-byte cells (int64 for
// float32 plans, float64 for float64 plans) | per wave: kernel values of a chunk
// (2 w per node; 4 w per double-layer node: x, y taps and their derivatives)
// and the chunk's offsets.
__host__ __device__ inline size_t spread_lds_layout(int T, int W, size_t rb, size_t* off_stage)
{
    const int E = T + W - 1;
    const size_t win = ((size_t)E * spread_pitch(T, W) * 8 + 15) & ~(size_t)15;  // 8-byte cells
    const int recs = rb == 4 ? SpreadShape<float>::kRecs : SpreadShape<double>::kRecs;
    const size_t stage = (size_t)SpreadShape<float>::kWaves * (recs * 2 * W + 2 * recs) * rb;
    *off_stage = win;
    return win + stage;
}

template <typename T>
__device__ __forceinline__ T lane_value(T v, int lane)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    } else {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __builtin_bit_cast(T, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    }
}

// Precision of the tap polynomials.  An error in the kernel values that is the
// same for every node at a given offset acts as a change of the kernel's shape,
// which the deconvolution by 1/phihat^2 amplifies near the band edge.  The
// planner therefore divides by the transforms of the very polynomials the
// device evaluates (the interpolation table of float32 plans with float32
// coefficients), so the only shape change left is the evaluation's own
// rounding, which varies from node to node like noise.  Spreading evaluates
// its taps in float64 in both precisions: its rounding noise lands on the grid,
// where the far-history multiplier amplifies it at low wavenumbers (float32
// taps raised the float32 error on the square workload from 6.8e-7 to 9.9e-7
// for 7% of spreading time).  Interpolation noise stays with its target and is
// not amplified, so float32 plans interpolate with float32 taps.
template <typename R> struct TapT { using T = double; };
template <> struct TapT<float> { using T = float; };

// Horner evaluation of one tap's polynomial and its derivative in u.
template <int P, typename H>
__device__ __forceinline__ void tap_value_deriv(const H* __restrict__ c, H u, H& v, H& dv)
{
    H p = c[P - 1], dp = H(0);
#pragma unroll
    for (int k = P - 2; k >= 0; --k) {
        dp = fma(dp, u, p);
        p = fma(p, u, c[k]);
    }
    v = p;
    dv = dp;
}

// The kernel is even: tap w-1-a at offset u equals tap a at -u.  With tap a's
// polynomial split as E(u^2) + u O(u^2) (ce[k] = c[2k], co[k] = c[2k+1]), one
// evaluation gives both taps.
template <int P, typename T>
__device__ __forceinline__ void tap_pair(const T* ce, const T* co, T u, T& v_a, T& v_mirror)
{
    const T u2 = u * u;
    T e = ce[(P + 1) / 2 - 1];
#pragma unroll
    for (int k = (P + 1) / 2 - 2; k >= 0; --k) e = fma(e, u2, ce[k]);
    T o = co[P / 2 - 1];
#pragma unroll
    for (int k = P / 2 - 2; k >= 0; --k) o = fma(o, u2, co[k]);
    v_a = fma(u, o, e);
    v_mirror = fma(-u, o, e);
}

// The same tap pair from coefficients that are equal on every lane (scalar
// registers): each polynomial is summed from its top term down as
// coefficient x power of u^2, the powers pw[k] = u^(2k) being shared by all
// pairs of a lane, so every coefficient is a multiplicand (or the final
// addend) and none has to be copied into a vector register first.
template <int P, typename T>
__device__ __forceinline__ void tap_pair_pow(const T* __restrict__ c, const T* pw, T u, T& v_a, T& v_mirror)
{
    constexpr int NE = (P + 1) / 2, NO = P / 2;
    static_assert(NO >= 2, "at least four terms");
    T e = c[2 * (NE - 1)] * pw[NE - 1];
#pragma unroll
    for (int k = NE - 2; k >= 1; --k) e = fma(c[2 * k], pw[k], e);
    e += c[0];
    T o = c[2 * (NO - 1) + 1] * pw[NO - 1];
#pragma unroll
    for (int k = NO - 2; k >= 1; --k) o = fma(c[2 * k + 1], pw[k], o);
    o += c[1];
    v_a = fma(u, o, e);
    v_mirror = fma(-u, o, e);
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Window cells: 64-bit fixed point (exact, order-independent integer sums,
// ds_add_u64 at 6.5 cycles) or float64 (ds_add_f64, 8.5 cycles).
struct CellFixed {
    using T = unsigned long long;
    static constexpr bool kScaled = true;
    static constexpr double kRange = 562949953421312.0;  // 2^49
    // round(v) via the 1.5 2^52 shift: exact for |v| < 2^51
    __device__ static T enc(double v)
    {
        const double t = v + 6755399441055744.0;
        return (T)(__double_as_longlong(t) - 0x4338000000000000LL);
    }
    __device__ static double dec(T a, double inv_q) { return (double)(long long)a * inv_q; }
};
struct CellF64 {
    using T = double;
    static constexpr bool kScaled = false;
    static constexpr double kRange = 1.0;
    __device__ static T enc(double v) { return v; }
    __device__ static double dec(T a, double) { return a; }
};

// max over the kDcParts partial maxima at smax (bit patterns of non-negative doubles)
__device__ __forceinline__ double smax_bound(const unsigned long long* __restrict__ smax)
{
    const int lane = threadIdx.x & 63;
    double m = lane < kDcParts ? __longlong_as_double((long long)smax[lane]) : 0.0;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    return m;
}

template <typename R, int W, typename FP>
__device__ void dev_spread_cells(unsigned char* smem_raw, const LevelGeom& g, const RecView<R>& vol,
                                 const RecView<R>& bnd, const R* __restrict__ str, int64_t n_src, int64_t n_bnd,
                                 R* __restrict__ grid, int use_vol, int use_bnd, int use_d,
                                 const double* __restrict__ coef, const unsigned long long* __restrict__ smax,
                                 const WorkUnit unit)
{
    using A = typename FP::T;
    static_assert(sizeof(A) == 8, "spread_lds_layout sizes the window for 8-byte cells");
    using SS = SpreadShape<R>;
    constexpr int NW = SS::kWaves;
    constexpr int RECS = SS::kRecs;
    constexpr int VST = RECS * 2 * W;     // staged values per wave chunk
    constexpr int RW = 64 / W;            // tap rows per atomic instruction
    constexpr int NI = (W + RW - 1) / RW; // atomic instructions per node
    using H = double;
    constexpr int P = horner_terms(W);
    constexpr int G = 64 / W;             // offset groups of the kernel-value evaluation
    const int T = g.T;
    const int E = T + W - 1;
    const int EP = spread_pitch(T, W);
    const int t = unit.tile;
    const int nv = use_vol ? unit.a1 - unit.a0 : 0;
    const int nbd = use_bnd ? unit.b1 - unit.b0 : 0;
    if (nv == 0 && nbd == 0) return;  // nothing lands in this unit (uniform across the workgroup)
    // scale of this unit's fixed-point window: the strength bound (plus the
    // derivative taps' when the unit spreads the double layer through them) times
    // the most records whose supports share one window cell
    R q = R(1);
    double inv_q = 1.0;
    if constexpr (FP::kScaled) {
        const bool dl = use_d && nbd > 0;
        const double cmax = smax_bound(smax) + (dl ? smax_bound(smax + kDcParts) * g.dmax : 0.0);
        const double bound = 1.01 * (double)unit.cover * cmax;
        if (!(bound > 0.0)) return;  // every contribution is zero
        q = (R)(FP::kRange / bound);
        inv_q = 1.0 / (double)q;
    }
    size_t off_st;
    spread_lds_layout(T, W, sizeof(R), &off_st);
    A* win = reinterpret_cast<A*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    R* vals = reinterpret_cast<R*>(smem_raw + off_st) + (size_t)wv * (VST + 2 * RECS);
    R* dd = vals + VST;  // [2 RECS] offsets of the chunk (x, y per node)

    const int gx0 = (t % g.ntx) * T;
    const int gy0 = (t / g.ntx) * T;
    for (int i = threadIdx.x; i < E * EP; i += blockDim.x) win[i] = A(0);
    __syncthreads();

    // tap of this lane: column ta, rows tb0 + k RW (k < NI)
    const int ta = lane % W;
    const int tb0 = lane / W;
    const bool lane_on = lane < RW * W;
    // kernel-value evaluation: lane -> tap ta, offset group tb0 (G groups); the
    // tap's polynomial coefficients stay in this lane's registers
    // single-strength nodes: lane (tap pair kp, group kg) evaluates taps kp and
    // w-1-kp from tap kp's polynomial in even and odd parts (coefficients in
    // registers); double-layer nodes: lane (tap ta, group tb0) evaluates value
    // and derivative with the tap's coefficients read from the (cached) table
    constexpr int NP = (W + 1) / 2;
    constexpr int GP = 64 / NP;
    const int kp = lane % NP;
    const int kg = lane / NP;
    const bool kon = lane < GP * NP;
    double ce[(P + 1) / 2], co[P / 2];
#pragma unroll
    for (int k = 0; k < (P + 1) / 2; ++k) ce[k] = coef[kp * P + 2 * k];
#pragma unroll
    for (int k = 0; k < P / 2; ++k) co[k] = coef[kp * P + 2 * k + 1];
    const int64_t n_all = n_src + n_bnd;
    const H dscale = (H)(-2.0 / g.h);  // d/dy of a tap value = -(2/h) d/du

    // DL = false: one strength per node; DL = true: double-layer boundary nodes,
    // value s phi_x phi_y + gx phi_x' phi_y + gy phi_x phi_y'.
    auto wave_path = [&](const RecView<R>& L, int r0, int r1, auto dl_tag) {
        constexpr bool DL = decltype(dl_tag)::value;
        constexpr int VS = DL ? 4 * W : 2 * W;
        constexpr int NR = DL ? RECS / 2 : RECS;  // nodes per chunk
        int base = r0 + wv * NR;
        int n_ij = 0, n_idx = 0;
        R n_dx = R(0), n_dy = R(0);
        if (lane < NR && base + lane < r1) {
            n_ij = L.ij[base + lane];
            n_idx = L.idx[base + lane];
            n_dx = L.dx[base + lane];
            n_dy = L.dy[base + lane];
        }
        const bool have0 = lane < NR && base + lane < r1;
        R n_s = have0 ? str[n_idx] : R(0);
        R n_gx = R(0), n_gy = R(0);
        if (DL && have0) {
            n_gx = str[n_all + (n_idx - n_src)];
            n_gy = str[n_all + n_bnd + (n_idx - n_src)];
        }
        for (; base < r1; base += NW * NR) {
            const int nrec = min(NR, r1 - base);
            const int c_ij = n_ij;
            const R c_s = n_s, c_gx = n_gx, c_gy = n_gy;
            const R c_dx = n_dx, c_dy = n_dy;
            // prefetch the next chunk of this wavefront
            const int nb = base + NW * NR;
            const bool pre = lane < NR && nb + lane < r1;
            if (pre) {
                n_ij = L.ij[nb + lane];
                n_idx = L.idx[nb + lane];
                n_dx = L.dx[nb + lane];
                n_dy = L.dy[nb + lane];
            }
            // kernel values: the chunk's offsets go to LDS (lane = 2 node + axis),
            // then lane (tap ta, group tb0) evaluates its tap for offsets tb0, tb0+G, ...
            {
                const R dxv = __shfl(c_dx, lane >> 1);
                const R dyv = __shfl(c_dy, lane >> 1);
                if (lane < 2 * NR) dd[lane] = (lane & 1) ? dyv : dxv;
                wave_sync_lds();
                const int nv2 = 2 * nrec;
                if constexpr (DL) {
                    if (lane_on) {
                        const double* cf = coef + ta * P;
                        for (int q = tb0; q < nv2; q += G) {
                            const H u = H(2) * (H)dd[q] - H(1);
                            R* dst = vals + (q >> 1) * VS + (q & 1) * W + ta;
                            H v, dv;
                            tap_value_deriv<P>(cf, u, v, dv);
                            dst[0] = (R)v;
                            dst[2 * W] = (R)(dscale * dv);
                        }
                    }
                } else if (kon) {
                    for (int q = kg; q < nv2; q += GP) {
                        const double u = 2.0 * (double)dd[q] - 1.0;
                        double va, vm;
                        tap_pair<P>(ce, co, u, va, vm);
                        R* dst = vals + (q >> 1) * VS + (q & 1) * W;
                        dst[kp] = (R)va;
                        if (kp != W - 1 - kp) dst[W - 1 - kp] = (R)vm;
                    }
                }
            }
            if (pre) {
                n_s = str[n_idx];
                if (DL) {
                    n_gx = str[n_all + (n_idx - n_src)];
                    n_gy = str[n_all + n_bnd + (n_idx - n_src)];
                }
            }
            wave_sync_lds();
            // node loop: lanes -> taps; the next node's values are read before
            // this node's atomics are issued
            auto load = [&](int rr, R& vx, R* vy, R& dvx, R* dvy) {
                const R* v = vals + rr * VS;
                vx = v[ta];
                if (DL) dvx = v[2 * W + ta];
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    const int b = min(tb0 + k * RW, W - 1);
                    vy[k] = v[W + b];
                    if (DL) dvy[k] = v[3 * W + b];
                }
            };
            R vx, vy[NI], dvx = R(0), dvy[NI];
            load(0, vx, vy, dvx, dvy);
            for (int rr = 0; rr < nrec; ++rr) {
                R vxn = R(0), vyn[NI], dvxn = R(0), dvyn[NI];
                if (rr + 1 < nrec) load(rr + 1, vxn, vyn, dvxn, dvyn);
                const int p = __builtin_amdgcn_readlane(c_ij, rr);
                const R s = lane_value(c_s, rr);
                const int i0 = (p & 0xffff) - gx0;
                const int j0 = (p >> 16) - gy0;
                A* row = win + (j0 + tb0) * EP + i0 + ta;
                if constexpr (DL) {
                    const R gx = lane_value(c_gx, rr), gy = lane_value(c_gy, rr);
                    const R sx = s * vx * q, gxx = gx * dvx * q, gyx = gy * vx * q;
#pragma unroll
                    for (int k = 0; k < NI; ++k)
                        if (lane_on && tb0 + k * RW < W)
                            atomicAdd(row + k * RW * EP, FP::enc(sx * vy[k] + gxx * vy[k] + gyx * dvy[k]));
                } else {
                    const R vxs = vx * s * q;
#pragma unroll
                    for (int k = 0; k < NI; ++k)
                        if (lane_on && tb0 + k * RW < W) atomicAdd(row + k * RW * EP, FP::enc(vxs * vy[k]));
                }
                vx = vxn;
                dvx = dvxn;
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    vy[k] = vyn[k];
                    dvy[k] = dvyn[k];
                }
            }
            wave_sync_lds();
        }
    };

    if (nv) wave_path(vol, unit.a0, unit.a1, std::false_type{});
    if (nbd && !use_d) wave_path(bnd, unit.b0, unit.b1, std::false_type{});
    if (nbd && use_d) wave_path(bnd, unit.b0, unit.b1, std::true_type{});
    __syncthreads();
    const int F = g.F;
    for (int i = threadIdx.x; i < E * E; i += blockDim.x) {
        const int y = i / E;
        const int x = i - y * E;
        const int gx = gx0 + x, gy = gy0 + y;
        if (gx < F && gy < F) {
            const A a = win[y * EP + x];
            if (a != A(0)) unsafeAtomicAdd(grid + (size_t)gy * F + gx, (R)FP::dec(a, inv_q));
        }
    }
}

// Window cells of a unit: float32 plans always use 64-bit fixed point.
// Float64 plans use it too for units that spread no double-layer derivative
// taps (the strengths alone bound their contributions, so 2^49 / (cover x
// bound) resolves each cell to ~1e-15 of the largest strength per record);
// units with derivative taps keep float64 cells, whose contributions the
// derivative bound would otherwise coarsen ~10^4-fold.
template <typename R, int W>
__device__ void dev_spread(unsigned char* smem_raw, const LevelGeom& g, const RecView<R>& vol, const RecView<R>& bnd,
                           const R* __restrict__ str, int64_t n_src, int64_t n_bnd, R* __restrict__ grid,
                           int use_vol, int use_bnd, int use_d, const double* __restrict__ coef,
                           const unsigned long long* __restrict__ smax, const WorkUnit unit)
{
    if constexpr (sizeof(R) == 8) {
        const bool dl = use_d && use_bnd && unit.b1 > unit.b0;
        if (dl || !smax) {
            dev_spread_cells<R, W, CellF64>(smem_raw, g, vol, bnd, str, n_src, n_bnd, grid, use_vol, use_bnd, use_d,
                                            coef, smax, unit);
            return;
        }
    }
    dev_spread_cells<R, W, CellFixed>(smem_raw, g, vol, bnd, str, n_src, n_bnd, grid, use_vol, use_bnd, use_d, coef,
                                      smax, unit);
}

// ---------------------------------------------------------------------------
// Spread on matrix cores (float32 plans, 16 x 16 tiles).
//
// A tile's window of 32 x 32 cells (the tile plus the w - 1 cells its nodes'
// supports reach beyond it, padded) receives
//     window[y][x] = sum_j phi_y,j(y) * (s_j phi_x,j(x)),
// a sum of outer products of two 32-vectors per node, each with w nonzero
// entries at the node's corner offset -- a rank-n update that one
// v_mfma_f32_32x32x2_f32 advances by two nodes while the whole window stays in
// the wavefront's accumulation registers (no LDS atomics).  A double-layer
// node adds gx phi_x' phi_y + gy phi_x phi_y' (Sec. 3, Step 2, through the
// kernel derivative as in the LDS path), which is two outer products:
// phi_y (x) (s phi_x + gx phi_x') and (gy phi_y') (x) phi_x.
//
// One wavefront per work unit.  Per chunk of 32 rank-1 terms the wavefront
// writes their factors into LDS rows of 32 entries (lane pairs: one record,
// x or y; each lane zeroes its own row, then evaluates the w taps in float64
// with the tap's coefficients uniform across the wavefront), then runs 16 matrix
// instructions reading the rows.  The next chunk's records are loaded while
// the current one is processed.  Each chunk's products accumulate in float32 in
// the matrix registers and are then added to a float64 copy of the window, which
// is added to the grid (float32) with global atomics.
//
// Measured on gfx950 (disk with 12M nodes, F = 4096 / 2048, w = 13 / 10):
// 0.51 / 0.44 ms against 1.01 / 0.67 ms for the LDS path.  The float64 form
// (four 16x16x4 blocks) was slower than the LDS path: float64 matrix
// instructions run at the vector rate on this chip.
constexpr int kMmaChunk = 32;  // rank-1 terms (factor-row pairs) per chunk
using mma_f32x16 = float __attribute__((ext_vector_type(16)));

// Factor rows are kMmaRow floats apart (32 used): a multiple of 4 for the
// 16-byte zeroing stores, and not a multiple of 64 dwords, so that the lanes'
// rows fall in different LDS banks.
constexpr int kMmaRow = 36;
__host__ __device__ constexpr size_t mma_wave_bytes() { return (size_t)kMmaChunk * 2 * kMmaRow * sizeof(float); }

template <int W>
__device__ void dev_spread_mma(unsigned char* smem_raw, const LevelGeom& g, const RecView<float>& vol,
                               const RecView<float>& bnd, const float* __restrict__ str, int64_t n_src,
                               int64_t n_bnd, float* __restrict__ grid, int use_vol, int use_bnd, int use_d,
                               const double* __restrict__ coef, const WorkUnit unit)
{
    constexpr int NPC = kMmaChunk;
    constexpr int P = horner_terms(W);
    static_assert(kMmaTile + W - 1 <= 32, "window of 32 cells");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    float* Ay = reinterpret_cast<float*>(smem_raw + (size_t)wv * mma_wave_bytes());  // [NPC][kMmaRow] y factors
    float* Bx = Ay + NPC * kMmaRow;                                                     // [NPC][kMmaRow] x factors
    const int t = unit.tile;
    const int gx0 = (t % g.ntx) * kMmaTile, gy0 = (t / g.ntx) * kMmaTile;
    const int nv = use_vol ? unit.a1 - unit.a0 : 0;
    const int nbd = use_bnd ? unit.b1 - unit.b0 : 0;
    if (nv == 0 && nbd == 0) return;  // uniform across the wavefront
    const int64_t n_all = n_src + n_bnd;
    const double dscale = -2.0 / g.h;  // d/dy of a tap value = -(2/h) d/du
    const int axis = lane & 1;         // 0: x factor, 1: y factor
    const int rec = lane >> 1;
    // each chunk accumulates from zero in the matrix registers (16 roundings);
    // the chunk's window is then added in float64, so the float32 rounding
    // does not build up over the unit's hundreds of nodes
    double win[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) win[r] = 0.0;

    auto path = [&](const RecView<float>& L, int r0, int r1, auto dl_tag) {
        constexpr bool DL = decltype(dl_tag)::value;
        constexpr int NRC = DL ? NPC / 2 : NPC;  // records per chunk
        int p_off = 0, p_idx = 0;
        float p_d = 0.f, p_s = 0.f, p_gx = 0.f, p_gy = 0.f;
        // this lane's record of the chunk at c0, its axis: the record first, its
        // strengths (gathered through the record's node index) one phase later,
        // so that neither load's latency stalls the wavefront
        auto fetch_rec = [&](int c0) {
            const int r = c0 + rec;
            if (rec < NRC && r < r1) {
                const int ij = L.ij[r];
                p_idx = L.idx[r];
                p_d = axis ? L.dy[r] : L.dx[r];
                p_off = axis ? (ij >> 16) - gy0 : (ij & 0xffff) - gx0;
            }
        };
        auto fetch_str = [&](int c0) {
            if (rec < NRC && c0 + rec < r1) {
                p_s = str[p_idx];
                if (DL) {
                    p_gx = str[n_all + (p_idx - n_src)];
                    p_gy = str[n_all + n_bnd + (p_idx - n_src)];
                }
            }
        };
        fetch_rec(r0);
        fetch_str(r0);
        for (int c0 = r0; c0 < r1; c0 += NRC) {
            const int n = min(NRC, r1 - c0);
            const int np = DL ? 2 * n : n;
            const double u = 2.0 * (double)p_d - 1.0;
            const int off = p_off;
            const double s_ = p_s, gx_ = p_gx, gy_ = p_gy;
            const bool more = c0 + NRC < r1;
            if (more) fetch_rec(c0 + NRC);
            // this lane's factor row(s): zero, then the w taps at the corner offset
            float* row = (axis ? Ay : Bx) + (DL ? 2 * rec : rec) * kMmaRow;
            if (rec < NRC) {
                const float4 z{};
#pragma unroll
                for (int k = 0; k < 8; ++k) reinterpret_cast<float4*>(row)[k] = z;
                if (DL) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) reinterpret_cast<float4*>(row + kMmaRow)[k] = z;
                }
            }
            const bool on = rec < n;
            if constexpr (!DL) {
                // the kernel is even: tap w-1-a at offset u is tap a at -u, so with
                // tap a's polynomial split as E(u^2) + u O(u^2) one evaluation gives both
                // (coefficients uniform across the wavefront: power form, so they stay
                // in scalar registers; the powers of u^2 serve every pair)
                double pw[(P + 1) / 2];
                pw[0] = 1.0;
                pw[1] = u * u;
#pragma unroll
                for (int k = 2; k < (P + 1) / 2; ++k) pw[k] = pw[k - 1] * pw[1];
                const double sc = axis == 0 ? s_ : 1.0;
#pragma unroll
                for (int a = 0; a < (W + 1) / 2; ++a) {
                    double va, vm;
                    tap_pair_pow<P>(coef + a * P, pw, u, va, vm);
                    if (on) {
                        row[off + a] = (float)(sc * va);
                        if (a != W - 1 - a) row[off + W - 1 - a] = (float)(sc * vm);
                    }
                }
            }
#pragma unroll 2
            for (int a = 0; a < (DL ? W : 0); ++a) {
                const double* ca = coef + a * P;  // uniform: scalar loads
                if constexpr (DL) {
                    double v = ca[P - 1], dv = 0.0;
#pragma unroll
                    for (int k = P - 2; k >= 0; --k) {
                        dv = fma(dv, u, v);
                        v = fma(v, u, ca[k]);
                    }
                    dv *= dscale;
                    if (on) {
                        if (axis == 0) {
                            row[off + a] = (float)(s_ * v + gx_ * dv);
                            row[kMmaRow + off + a] = (float)v;
                        } else {
                            row[off + a] = (float)v;
                            row[kMmaRow + off + a] = (float)(gy_ * dv);
                        }
                    }
                }
            }
            wave_sync_lds();
            if (more) fetch_str(c0 + NRC);  // the next chunk's node indices have arrived by now
            // rank-1 terms [0, np) (rows up to the next even index are zero)
            const int i = lane & 31;
            mma_f32x16 acc = {};
#pragma unroll 4
            for (int m = 0; m < np; m += 2) {
                const int r = m + (lane >> 5);
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(Ay[r * kMmaRow + i], Bx[r * kMmaRow + i], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) win[r] += (double)acc[r];
            wave_sync_lds();
        }
    };
    if (nv) path(vol, unit.a0, unit.a1, std::false_type{});
    if (nbd && !use_d) path(bnd, unit.b0, unit.b1, std::false_type{});
    if (nbd && use_d) path(bnd, unit.b0, unit.b1, std::true_type{});
    // result element r of lane l: window row (r % 4) + 8 (r / 4) + 4 (l / 32), column l % 32
    const int F = g.F;
    const int gx = gx0 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int gy = gy0 + (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
        const float v = (float)win[r];
        if (v != 0.f && gx < F && gy < F) unsafeAtomicAdd(grid + (size_t)gy * F + gx, v);
    }
}

// ---------------------------------------------------------------------------
// Spread on matrix cores for float64 plans (16 x 16 tiles, w <= 16).
//
// The same outer-product form as the float32 kernel above, with
// v_mfma_f64_16x16x4_f64: the window of 32 x 32 cells is four 16 x 16 blocks,
// each in four float64 accumulation registers per lane, and one instruction per
// block advances it by four rank-1 terms (a volume node is one term,
// (s phi_x) (x) phi_y; a double-layer node two, as above).  Accumulation stays
// in float64 throughout, so nothing is rounded to float32.
//
// Per chunk of 32 terms each lane evaluates the w taps of one (term, axis)
// (coefficients uniform across the wavefront: scalar registers) into compact
// LDS rows of w values with the term's corner offset beside them; the matrix
// step then gives lane (k, i) = (lane / 16, lane % 16) the entry of row
// 16 b + i of term k's factor, zero outside the factor's w taps.  No LDS
// atomics, and each row's zero (entry w, written once) serves every entry
// outside the taps: 6 LDS reads per lane per four terms, against w^2 LDS
// atomics per node in the LDS path.
//
// Lane layout of the instruction (checked on the device): lane 16 k + i
// supplies A[i][k] and B[k][i]; result element e of lane l is C[l / 16 + 4 e][l % 16].
constexpr int kM64Terms = 32;  // rank-1 terms per chunk
constexpr int kM64Row = 17;    // doubles per factor row: w taps and a zero (w <= 16; odd, so rows start in different banks)
using mma_f64x4 = double __attribute__((ext_vector_type(4)));
__host__ __device__ constexpr size_t mma64_wave_bytes()
{
    return (size_t)kM64Terms * 2 * kM64Row * sizeof(double) + (size_t)kM64Terms * 2 * sizeof(int);
}

template <int W>
__device__ void dev_spread_mma64(unsigned char* smem_raw, const LevelGeom& g, const RecView<double>& vol,
                                 const RecView<double>& bnd, const double* __restrict__ str, int64_t n_src,
                                 int64_t n_bnd, double* __restrict__ grid, int use_vol, int use_bnd, int use_d,
                                 const double* __restrict__ coef, const WorkUnit unit_in)
{
    constexpr int NT = kM64Terms;
    constexpr int P = horner_terms(W);
    static_assert(kMmaTile + W - 1 <= 32 && W < kM64Row, "window of 32 cells, rows of w taps and a zero");
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    unsigned char* base = smem_raw + (size_t)wv * mma64_wave_bytes();
    double* X = reinterpret_cast<double*>(base);  // [NT][kM64Row] x factors (strength folded in)
    double* Y = X + NT * kM64Row;                 // [NT][kM64Row] y factors
    int* OFF = reinterpret_cast<int*>(Y + NT * kM64Row);  // [NT][2] corner offsets (x, y) in the window
    // the unit is the wavefront's own: its fields are uniform (scalar loop control)
    WorkUnit unit;
    unit.tile = __builtin_amdgcn_readfirstlane(unit_in.tile);
    unit.a0 = __builtin_amdgcn_readfirstlane(unit_in.a0);
    unit.a1 = __builtin_amdgcn_readfirstlane(unit_in.a1);
    unit.b0 = __builtin_amdgcn_readfirstlane(unit_in.b0);
    unit.b1 = __builtin_amdgcn_readfirstlane(unit_in.b1);
    const int t = unit.tile;
    const int gx0 = (t % g.ntx) * kMmaTile, gy0 = (t / g.ntx) * kMmaTile;
    const int nv = use_vol ? unit.a1 - unit.a0 : 0;
    const int nbd = use_bnd ? unit.b1 - unit.b0 : 0;
    if (nv == 0 && nbd == 0) return;  // uniform across the wavefront
    const int64_t n_all = n_src + n_bnd;
    const double dscale = -2.0 / g.h;  // d/dy of a tap value = -(2/h) d/du
    const int axis = lane & 1;         // evaluation: 0 x factor, 1 y factor
    const int rec = lane >> 1;
    const int mk = lane >> 4, mi = lane & 15;  // matrix step: term mk of the four, row / column mi of a block
    mma_f64x4 acc[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[b][c] = mma_f64x4{0.0, 0.0, 0.0, 0.0};
    // entry W of every factor row stays zero (taps fill entries 0..W-1 only)
    X[lane * kM64Row + W] = 0.0;  // the wavefront's 64 rows: 32 x rows, then 32 y rows
    wave_sync_lds();

    auto path = [&](const RecView<double>& L, int r0, int r1, auto dl_tag) {
        constexpr bool DL = decltype(dl_tag)::value;
        constexpr int NRC = DL ? NT / 2 : NT;  // records per chunk
        int p_off = 0, p_idx = 0;
        double p_d = 0.0, p_s = 0.0, p_gx = 0.0, p_gy = 0.0;
        // this lane's record of the chunk at c0, its axis: the record first, its
        // strengths (gathered through the record's node index) one phase later,
        // so that neither load's latency stalls the wavefront
        auto fetch_rec = [&](int c0) {
            const int r = c0 + rec;
            if (rec < NRC && r < r1) {
                const int ij = L.ij[r];
                p_idx = L.idx[r];
                p_d = axis ? L.dy[r] : L.dx[r];
                p_off = axis ? (ij >> 16) - gy0 : (ij & 0xffff) - gx0;
            }
        };
        auto fetch_str = [&](int c0) {
            if (rec < NRC && c0 + rec < r1) {
                p_s = str[p_idx];
                if (DL) {
                    p_gx = str[n_all + (p_idx - n_src)];
                    p_gy = str[n_all + n_bnd + (p_idx - n_src)];
                }
            }
        };
        fetch_rec(r0);
        fetch_str(r0);
        for (int c0 = r0; c0 < r1; c0 += NRC) {
            const int n = min(NRC, r1 - c0);
            const int nterm = DL ? 2 * n : n;
            const double u = 2.0 * p_d - 1.0;
            const int off = p_off;
            const double s_ = p_s, gx_ = p_gx, gy_ = p_gy;
            const bool more = c0 + NRC < r1;
            if (more) fetch_rec(c0 + NRC);
            const bool on = rec < n;
            if constexpr (!DL) {
                // term rec: x row s phi_x, y row phi_y (tap pairs from the even kernel, as above)
                double* row = (axis ? Y : X) + rec * kM64Row;
                double pw[(P + 1) / 2];
                pw[0] = 1.0;
                pw[1] = u * u;
#pragma unroll
                for (int k = 2; k < (P + 1) / 2; ++k) pw[k] = pw[k - 1] * pw[1];
                const double sc = axis == 0 ? s_ : 1.0;
#pragma unroll
                for (int a = 0; a < (W + 1) / 2; ++a) {
                    double va, vm;
                    tap_pair_pow<P>(coef + a * P, pw, u, va, vm);
                    if (on) {
                        row[a] = sc * va;
                        if (a != W - 1 - a) row[W - 1 - a] = sc * vm;
                    }
                }
                if (on) OFF[2 * rec + axis] = off;
            } else {
                // terms 2 rec and 2 rec + 1: (s phi_x + gx phi_x') (x) phi_y and phi_x (x) (gy phi_y')
                double* r0w = (axis ? Y : X) + (2 * rec) * kM64Row;
                double* r1w = r0w + kM64Row;
#pragma unroll 2
                for (int a = 0; a < W; ++a) {
                    double v, dv;
                    tap_value_deriv<P>(coef + a * P, u, v, dv);  // uniform coefficients: scalar loads
                    dv *= dscale;
                    if (on) {
                        if (axis == 0) {
                            r0w[a] = s_ * v + gx_ * dv;
                            r1w[a] = v;
                        } else {
                            r0w[a] = v;
                            r1w[a] = gy_ * dv;
                        }
                    }
                }
                if (on) {
                    OFF[2 * (2 * rec) + axis] = off;
                    OFF[2 * (2 * rec + 1) + axis] = off;
                }
            }
            wave_sync_lds();
            if (more) fetch_str(c0 + NRC);  // the next chunk's node indices have arrived by now
            // matrix steps of four terms (terms past nterm contribute zero rows); the
            // factors of the next step are read before this step's instructions issue
            auto factors = [&](int m, double* a, double* b) {
                const int tm = m + mk;
                const bool live = tm < nterm;
                const int ox = live ? OFF[2 * tm] : 64, oy = live ? OFF[2 * tm + 1] : 64;
                const double* yr = Y + tm * kM64Row;
                const double* xr = X + tm * kM64Row;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    // entries outside the w taps (negative offsets wrap to large unsigned
                    // values) read the row's zero at index W
                    a[q] = yr[min((unsigned)(16 * q + mi - oy), (unsigned)W)];
                    b[q] = xr[min((unsigned)(16 * q + mi - ox), (unsigned)W)];
                }
            };
            double a[2], b[2];
            factors(0, a, b);
            for (int m = 0; m < nterm; m += 4) {
                double an[2], bn[2];
                if (m + 4 < nterm) factors(m + 4, an, bn);
#pragma unroll
                for (int by = 0; by < 2; ++by)
#pragma unroll
                    for (int bx = 0; bx < 2; ++bx)
                        acc[by][bx] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[by], b[bx], acc[by][bx], 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    a[q] = an[q];
                    b[q] = bn[q];
                }
            }
            wave_sync_lds();
        }
    };
    if (nv) path(vol, unit.a0, unit.a1, std::false_type{});
    if (nbd && !use_d) path(bnd, unit.b0, unit.b1, std::false_type{});
    if (nbd && use_d) path(bnd, unit.b0, unit.b1, std::true_type{});
    const int F = g.F;
#pragma unroll
    for (int by = 0; by < 2; ++by)
#pragma unroll
        for (int bx = 0; bx < 2; ++bx) {
            const int gx = gx0 + 16 * bx + mi;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gy = gy0 + 16 * by + mk + 4 * e;
                const double v = acc[by][bx][e];
                if (v != 0.0 && gx < F && gy < F) unsafeAtomicAdd(grid + (size_t)gy * F + gx, v);
            }
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
    const int row = g.rd0 + unit;  // the rows the spread wrote
    const R* x = grid + (size_t)row * F;
    for (int n = threadIdx.x; n < N; n += blockDim.x) z[lds_pad(bitrev(n, logN))] = {x[2 * n], x[2 * n + 1]};
    __syncthreads();
    lds_fft(z, logN, tw, 2, false);
    for (int k = threadIdx.x; k <= M; k += blockDim.x) {
        const cplx<R> a = z[lds_pad(k)];
        const cplx<R> b = z[lds_pad((N - k) & (N - 1))];
        const R ex = (a.x + b.x) * R(0.5), ey = (a.y - b.y) * R(0.5);   // even-sample spectrum
        const R ox = (a.y + b.y) * R(0.5), oy = (b.x - a.x) * R(0.5);   // odd-sample spectrum
        const cplx<R> wk = tw[k];                                       // exp(-2 pi i k / F)
        cplx<R> X;
        X.x = ex + wk.x * ox - wk.y * oy;
        X.y = ey + wk.x * oy + wk.y * ox;
        spec[(size_t)k * F + row] = X;
    }
}

// ---------------------------------------------------------------------------
// Column pass for x-frequency m1 = unit, in place: FFT along y, multiply by the
// level's table ((dk/2pi)^2 M(k) / phihat^2, zero outside |m2| <= M), inverse
// FFT along y.  The multipliers are loaded with the column.  Float32 columns
// also copy the twiddles into LDS next to the column when both fit in
// kColTwLds bytes, so no global read waits inside the chain of LDS passes
// (measured: 12% faster for F = 4096; float64 columns, whose 16-byte
// twiddles would add to the passes' LDS traffic, were 10% slower so).
constexpr size_t kColTwLds = 96 * 1024;
constexpr int kColPre = 4;  // multipliers held in registers per thread (the rest load late)

template <typename R>
__host__ __device__ inline bool col_stages_twiddles(int F)
{
    return sizeof(R) == 4 && (size_t)(lds_padded_len(F) + F / 2) * sizeof(cplx<R>) <= kColTwLds;
}

template <typename R>
__host__ __device__ inline size_t col_lds_bytes(int F)
{
    return (size_t)(lds_padded_len(F) + (col_stages_twiddles<R>(F) ? F / 2 : 0)) * sizeof(cplx<R>);
}

// dspec: with g.dip, the level's two double-layer channels (mu nu_c w spread with
// the kernel itself), already transformed along y by dev_col_fwd; each column
// adds -i k_1 B_1 - i k_2 B_2 to the forward transform before the multiply,
// the transform of the double layer's kernel derivative (Sec. 3, Step 2).
template <typename R>
__device__ void dev_col(unsigned char* smem_raw, const LevelGeom& g, cplx<R>* __restrict__ spec,
                        const R* __restrict__ mult, const cplx<R>* __restrict__ tw, int zero_dc, int unit,
                        const cplx<R>* __restrict__ dspec1 = nullptr, const cplx<R>* __restrict__ dspec2 = nullptr)
{
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int logF = g.logF;
    const int M = g.M;
    const int m1 = unit;
    cplx<R>* col = spec + (size_t)m1 * F;
    auto mult_at = [&](int q) -> R {
        const int m2 = q < (F >> 1) ? q : q - F;
        const int am = m2 < 0 ? -m2 : m2;
        R t = am <= M ? mult[(size_t)m1 * (M + 1) + am] : R(0);
        if (zero_dc && m1 == 0 && q == 0) t = R(0);
        return t;
    };
    // rows outside [rd0, rd1) hold no spread data (the row pass skipped them): zero
    for (int q = threadIdx.x; q < F; q += blockDim.x)
        z[lds_pad(bitrev(q, logF))] = (q >= g.rd0 && q < g.rd1) ? col[q] : cplx<R>{R(0), R(0)};
    R mv[kColPre];
#pragma unroll
    for (int k = 0; k < kColPre; ++k) {
        const int q = threadIdx.x + k * (int)blockDim.x;
        mv[k] = q < F ? mult_at(q) : R(0);
    }
    auto run = [&](const cplx<R>* twp) {
        lds_fft(z, logF, twp, 1, false);
        if (dspec1) {  // + (-i k_1) B_1 + (-i k_2) B_2 at the retained modes (the table is zero elsewhere)
            const cplx<R>* b1 = dspec1 + (size_t)m1 * F;
            const cplx<R>* b2 = dspec2 + (size_t)m1 * F;
            const R k1 = (R)(m1 * g.dk);
            for (int q = threadIdx.x; q < F; q += blockDim.x) {
                const int m2 = q < (F >> 1) ? q : q - F;
                if (m2 > M || m2 < -M) continue;
                const R k2 = (R)(m2 * g.dk);
                const cplx<R> a = b1[q], b = b2[q];
                z[lds_pad(q)].x += k1 * a.y + k2 * b.y;
                z[lds_pad(q)].y -= k1 * a.x + k2 * b.x;
            }
        }
#pragma unroll
        for (int k = 0; k < kColPre; ++k) {
            const int q = threadIdx.x + k * (int)blockDim.x;
            if (q < F) {
                z[lds_pad(q)].x *= mv[k];
                z[lds_pad(q)].y *= mv[k];
            }
        }
        for (int q = threadIdx.x + kColPre * (int)blockDim.x; q < F; q += blockDim.x) {
            const R t = mult_at(q);
            z[lds_pad(q)].x *= t;
            z[lds_pad(q)].y *= t;
        }
        __syncthreads();
        lds_fft_dif(z, logF, twp, 1, true);
    };
    if (col_stages_twiddles<R>(F)) {
        cplx<R>* twl = z + lds_padded_len(F);
        for (int k = threadIdx.x; k < (F >> 1); k += blockDim.x) twl[k] = tw[k];
        __syncthreads();
        run(twl);
    } else {
        __syncthreads();
        run(tw);
    }
    for (int q = g.rt0 + (int)threadIdx.x; q < g.rt1; q += blockDim.x) col[q] = z[lds_pad(bitrev(q, logF))];
}

// Forward transform along y of column m1 = unit, in place, natural order out
// (the double-layer channels of a level with dip, before its column pass).
template <typename R>
__device__ void dev_col_fwd(unsigned char* smem_raw, const LevelGeom& g, cplx<R>* __restrict__ spec,
                            const cplx<R>* __restrict__ tw, int unit)
{
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int logF = g.logF;
    cplx<R>* col = spec + (size_t)unit * F;
    for (int q = threadIdx.x; q < F; q += blockDim.x)
        z[lds_pad(bitrev(q, logF))] = (q >= g.rd0 && q < g.rd1) ? col[q] : cplx<R>{R(0), R(0)};
    __syncthreads();
    lds_fft(z, logF, tw, 1, false);
    for (int q = threadIdx.x; q < F; q += blockDim.x) col[q] = z[lds_pad(q)];
}

// ---------------------------------------------------------------------------
// Row inverse: rebuild each row's Hermitian x-spectrum from m1 = 0..M (zero
// elsewhere) and inverse real FFT (complex FFT of length F/2).
template <typename R>
__device__ void dev_row_c2r(unsigned char* smem_raw, const LevelGeom& g, const cplx<R>* __restrict__ spec,
                            const cplx<R>* __restrict__ tw, R* __restrict__ out, int unit)
{
    cplx<R>* z = reinterpret_cast<cplx<R>*>(smem_raw);
    const int F = g.F;
    const int N = F >> 1;
    const int logN = g.logF - 1;
    const int M = g.M;
    const int row = g.rt0 + unit;  // the rows the interpolation reads
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        cplx<R> a = {R(0), R(0)};
        cplx<R> b = {R(0), R(0)};
        if (k <= M) a = spec[(size_t)k * F + row];
        const int kk = N - k;
        if (kk <= M) b = spec[(size_t)kk * F + row];
        const R ex = a.x + b.x, ey = a.y - b.y;       // X[k] + conj(X[N-k])
        const R dx = a.x - b.x, dy = a.y + b.y;       // X[k] - conj(X[N-k])
        const cplx<R> wk = tw[k];                     // exp(-2 pi i k/F); use its conjugate
        const R ox = dx * wk.x + dy * wk.y;
        const R oy = dy * wk.x - dx * wk.y;
        z[lds_pad(bitrev(k, logN))] = {ex - oy, ey + ox};      // E + i O
    }
    __syncthreads();
    lds_fft(z, logN, tw, 2, true);
    R* o = out + (size_t)row * F;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const cplx<R> v = z[lds_pad(n)];
        o[2 * n] = v.x;
        o[2 * n + 1] = v.y;
    }
}

// ---------------------------------------------------------------------------
// Interpolation (type-2, Sec. 3 Step 4 via the NUFFT): one workgroup per tile
// stages the (T+w-1)^2 grid window in LDS (a target's support lies in the
// window because the target is filed under the tile of its support corner).
// Each wavefront takes chunks of 32 targets, two lanes per target, 32 apart:
// lane (target q, coordinate c) evaluates the w kernel values of q's offset
// along c in registers (tap pairs a, w-1-a from one polynomial in u^2; the
// coefficients are the same for every lane, so they come through scalar
// loads), the two lanes swap their values with v_permlane32_swap, and each
// sums half of q's support rows (odd w: the second half ends on a zero row
// below the window, with weight zero, so both halves run alike).  The LDS
// holds the window only.
constexpr int kInterpTargets = 32;  // targets per wavefront chunk

__host__ __device__ inline size_t interp_lds_bytes(int T, int W, size_t rb)
{
    const size_t E = (size_t)(T + W - 1);
    return ((E + 1) * E * rb + 15) & ~(size_t)15;  // window rows and the zero row
}

// The value of v held by lane l ^ 32 (the other half of the wavefront).
// v_permlane32_swap(a, b) exchanges the upper 32 lanes of a with the lower 32
// lanes of b; with a = b = v, the lower lanes find the upper lanes' values in
// the second result and the upper lanes find the lower lanes' in the first.
__device__ __forceinline__ unsigned lane_xor32(unsigned v, bool upper)
{
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return upper ? r[0] : r[1];
}
__device__ __forceinline__ float lane_xor32(float v, bool upper)
{
    return __builtin_bit_cast(float, lane_xor32(__builtin_bit_cast(unsigned, v), upper));
}
__device__ __forceinline__ double lane_xor32(double v, bool upper)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = lane_xor32((unsigned)b, upper);
    const unsigned hi = lane_xor32((unsigned)(b >> 32), upper);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename R, int W>
__device__ void dev_interp(unsigned char* smem_raw, const LevelGeom& g, const R* __restrict__ grid,
                           const RecView<R>& L, R* __restrict__ hist, const typename TapT<R>::T* __restrict__ coef,
                           const WorkUnit unit)
{
    using TT = typename TapT<R>::T;
    constexpr int P = interp_terms(W, sizeof(R) == 4);
    constexpr int NT = kInterpTargets;
    constexpr int HB = (W + 1) / 2;  // rows per half (odd w: the last row of the second half is the zero row)
    constexpr int NP = (W + 1) / 2;  // tap pairs (the middle tap of odd w pairs with itself)
    const int t = unit.tile;
    const int r0 = unit.a0;
    const int r1 = unit.a1;
    if (r0 == r1) return;
    const int T = g.Ti;
    const int E = T + W - 1;
    const int F = g.F;
    R* reg = reinterpret_cast<R*>(smem_raw);
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int gx0 = (t % g.ntxi) * T;
    const int gy0 = (t / g.ntxi) * T;
    // window rows 0..E-1 from the grid, row E zero (32 lanes per row, no division)
    for (int y = threadIdx.x >> 5; y <= E; y += blockDim.x >> 5) {
        const int gy = gy0 + y;
        for (int x = threadIdx.x & 31; x < E; x += 32) {
            const int gx = gx0 + x;
            reg[y * E + x] = (y < E && gx < F && gy < F) ? grid[(size_t)gy * F + gx] : R(0);
        }
    }
    __syncthreads();
    // Lane (q, half): target q = lane % 32 of the chunk; half = lane / 32 is the
    // coordinate of its kernel values (0: x, 1: y) and its rows [half HB, half HB + HB).
    // Each half-wavefront thus reads one relative row of 32 targets, whose window
    // offsets the target order makes distinct modulo 32: 32 different LDS banks.
    const int q = lane & 31;
    const bool upper = lane >= 32;
    for (int base = r0 + wv * NT; base < r1; base += (kThreads / 64) * NT) {
        const bool on = q < r1 - base;  // the same for both lanes of a target
        int p = 0, id = 0;
        R own[W];  // this lane's kernel values along its coordinate
#pragma unroll
        for (int a = 0; a < W; ++a) own[a] = R(0);
        if (on) {
            p = L.ij[base + q];
            id = L.idx[base + q];
            const TT u = TT(2) * (TT)(upper ? L.dy[base + q] : L.dx[base + q]) - TT(1);
            TT pw[(P + 1) / 2];
            pw[0] = TT(1);
            pw[1] = u * u;
#pragma unroll
            for (int k = 2; k < (P + 1) / 2; ++k) pw[k] = pw[k - 1] * pw[1];
#pragma unroll
            for (int kp = 0; kp < NP; ++kp) {
                TT va, vm;
                tap_pair_pow<P>(coef + kp * P, pw, u, va, vm);
                own[kp] = (R)va;
                if (kp != W - 1 - kp) own[W - 1 - kp] = (R)vm;
            }
        }
        // x values for both lanes (the lower lane's own), y weights of each lane's rows
        R px[W], wy[HB];
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const R o = lane_xor32(own[a], upper);
            px[a] = upper ? o : own[a];
            if (a < HB) wy[a] = upper ? (HB + a < W ? own[HB + a] : R(0)) : o;
        }
        R sum = R(0);
        if (on) {
            const int i0 = (p & 0xffff) - gx0;
            const int j0 = (p >> 16) - gy0;
            const R* rowp = reg + (j0 + (upper ? HB : 0)) * E + i0;
#pragma unroll
            for (int bb = 0; bb < HB; ++bb) {
                R acc = R(0);
#pragma unroll
                for (int a2 = 0; a2 < W; ++a2) acc += px[a2] * rowp[bb * E + a2];
                sum += wy[bb] * acc;
            }
        }
        sum += lane_xor32(sum, upper);
        if (on && !upper) hist[id] = sum;
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
    // kLocalAll: out = history values + zero mode + local part; kLocalPart: out = local part
    // only (it needs neither history level, so it can run beside them); kLocalAddHistory:
    // out = history values + zero mode + out (after a kLocalPart pass)
    int part;
};

// Sum of the kDcParts zero-frequency partial sums, by one wavefront (every
// lane of the wavefront must call it).
__device__ __forceinline__ double dc_total(const double* __restrict__ dc)
{
    double v = dc[threadIdx.x & 63];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double hist_at(const void* h, int fp32, int64_t i)
{
    return fp32 ? (double)((const float*)h)[i] : ((const double*)h)[i];
}

// Local single-layer part S_L[sigma] at one target (Lemma 4.1 with the overall
// sign reversed, as pinned against brute-force quadrature), for c = r/sqrt(d) <= 12.
__device__ inline double s_local_value(double d, double r, double sg, double kap, double g3, double g4, double s0,
                                       double s1, double s2, int order)
{
    const double SQPI = 1.7724538509055160273;
    const double sd = sqrt(d);
    const double c = r / sd;
    if (c > 12.0) return 0.0;
    const double E = erfc(0.5 * c);
    const double e = exp(-0.25 * c * c);
    const double c2 = c * c, c3 = c2 * c;
    const double P1 = c * E - 2.0 * e / SQPI;
    const double Q = 2.0 * (c2 - 2.0) * e / SQPI - c3 * E;
    double s = 0.0;
    if (order >= 1) s += sd * 0.5 * s0 * P1;
    if (order >= 2) s += sg * d * c * kap * s0 * 0.25 * P1;
    if (order >= 3) s += d * sd * (s0 * kap * kap / 12.0 * (2.0 * c3 * E - (4.0 * c2 + 1.0) * e / SQPI) + s2 / 12.0 * Q);
    if (order >= 4)
        s += d * d * sg *
             (c * kap * kap * kap * s0 / 16.0 * (3.0 * c3 * E - (6.0 * c2 - 2.0) * e / SQPI) + c * kap * s2 / 8.0 * Q +
              c * s0 * g4 / 48.0 * Q + c * s1 * g3 / 12.0 * Q);
    return -s;
}

// Local double-layer part D_L[mu] at one target (Lemma 4.3 with the overall
// sign reversed), for c = r/sqrt(d) <= 12; m[0..4] = mu and its derivatives at b.
__device__ inline double d_local_value(double d, double r, double sg, double kap, double g3, double g4,
                                       const double* m, int order)
{
    const double SQPI = 1.7724538509055160273;
    const double sd = sqrt(d);
    const double c = r / sd;
    if (c > 12.0) return 0.0;
    const double E = erfc(0.5 * c);
    const double e = exp(-0.25 * c * c);
    const double c2 = c * c, c3 = c2 * c;
    const double m0 = m[0], m1 = m[1], m2 = m[2], m4 = m[4];
    double s = sg * 0.5 * m0 * E;
    if (order >= 1) s += sd * kap * m0 / (2.0 * SQPI) * e;
    if (order >= 2) s += d * sg * (3.0 * c * kap * kap * m0 / (8.0 * SQPI) * e + c * m2 * 0.25 * (2.0 * e / SQPI - c * E));
    const double A = 2.0 * (c2 + 1.0) * e / SQPI - c3 * E;
    const double B = 2.0 * (c2 + 4.0) * e / SQPI - c3 * E;
    if (order >= 3)
        s += d * sd * (5.0 * (c2 - 2.0) * kap * kap * kap * m0 / (16.0 * SQPI) * e + g4 * m0 / (4.0 * SQPI) * e +
                       kap * m2 * 0.25 * A + g3 * m1 / 12.0 * B);
    if (order >= 4) {
        s += d * d * sg *
             (35.0 * c * kap * kap * kap * kap * m0 * (c2 - 6.0) / (128.0 * SQPI) * e +
              5.0 * c * g3 * g3 * m0 / (12.0 * SQPI) * e + 5.0 * c * kap * g4 * m0 / (8.0 * SQPI) * e);
        s += d * d * sg * 5.0 * c * (kap * kap * m2 / 16.0 * A + kap * g3 * m1 / 24.0 * B);
        s += d * d * sg * c * m4 / 48.0 * (c3 * E - 2.0 * (c2 - 2.0) * e / SQPI);
    }
    return -s;
}

__device__ void dev_local(const LocalArgs& a, int64_t i)
{
    const double dcv = a.dc && a.part != kLocalPart ? dc_total(a.dc) : 0.0;  // before any lane leaves
    if (i >= a.n) return;
    double u = 0.0;
    if (a.part != kLocalPart) {
        u = hist_at(a.h0, a.fp32, i) + hist_at(a.h1, a.fp32, i);
        if (a.dc) u += a.dc_weight * dcv;
        if (a.part == kLocalAddHistory) {
            a.out[i] = u + a.out[i];
            return;
        }
    }
    const double SQPI = 1.7724538509055160273;
    const double d = a.delta;
    const double sd = sqrt(d);
    const double r = a.r[i];
    const double c = r / sd;
    const bool near = c <= 12.0;
    const int64_t n = a.n;
    if (!near) {
        // beyond 12 sqrt(delta): only the interior limit of V_L inside the domain; outside it the
        // local part of V is exponentially small (f vanishes off the domain) and is zero (frame
        // and layer data not read)
        if (a.jet6 && a.sgn[i] >= 0) {
            const double f = a.jet6[i], lap = a.jet6[3 * n + i] + a.jet6[5 * n + i];
            double v = 0.0;
            if (a.order_v >= 2) v += d * f;
            if (a.order_v >= 4) v += 0.5 * d * d * lap;
            u += v;
        }
        a.out[i] = u;
        return;
    }
    const double kap = a.kappa[i];
    const double g3 = a.g3 ? a.g3[i] : 0.0;
    const double g4 = a.g4 ? a.g4[i] : 0.0;
    const double sg = (double)a.sgn[i];
    const double E = erfc(0.5 * c);
    const double e = exp(-0.25 * c * c);
    const double c2 = c * c, c3 = c2 * c;
    if (a.jet6) {
        const double f = a.jet6[i], fx = a.jet6[n + i], fy = a.jet6[2 * n + i];
        const double fxx = a.jet6[3 * n + i], fxy = a.jet6[4 * n + i], fyy = a.jet6[5 * n + i];
        double v = 0.0;
        const double ex = -a.nx[i], ey = -a.ny[i];     // inward normal (eta)
        const double tx = a.ny[i], ty = -a.nx[i];      // tangent (xi), sign irrelevant
        const double fe = fx * ex + fy * ey;
        const double fee = fxx * ex * ex + 2.0 * fxy * ex * ey + fyy * ey * ey;
        const double ftt = fxx * tx * tx + 2.0 * fxy * tx * ty + fyy * ty * ty;
        if (a.order_v >= 2) v += 0.25 * d * (2.0 * erf(0.5 * c) + 2.0 * e * c / SQPI - c2 * E + 2.0) * f;
        if (a.order_v >= 3)
            v += d * sd * ((4.0 - 2.0 * c2) * e + SQPI * c3 * E) * (2.0 * fe - kap * f) / (12.0 * SQPI);
        if (a.order_v >= 4) {
            const double c4 = c2 * c2;
            v += d * d / 48.0 *
                 (E * (4.0 * c4 * kap * fe - 3.0 * (c4 + 4.0) * fee + (c4 - 12.0) * ftt - 3.0 * c4 * kap * kap * f) +
                  2.0 * c * (c2 - 2.0) * e * (-4.0 * kap * fe + 3.0 * fee - ftt + 3.0 * kap * kap * f) / SQPI +
                  24.0 * (ftt + fee));
        }
        u += v;
    }
    if (a.sj) u += s_local_value(d, r, sg, kap, g3, g4, a.sj[i], a.sj[n + i], a.sj[2 * n + i], a.order_s);
    if (a.mj) {
        const double m[5] = {a.mj[i], a.mj[n + i], a.mj[2 * n + i], a.mj[3 * n + i], a.mj[4 * n + i]};
        u += d_local_value(d, r, sg, kap, g3, g4, m, a.order_d);
    }
    a.out[i] = u;
}

}  // namespace dev
}  // namespace vp
