// Periodic cubic-spline semi-Lagrangian sweep (Sec. 3).
//
// Per line of n points: omega = C^{-1} u with C = (1/6)(T + 4 + T^{-1}), T the
// cyclic shift, then u'_i = sum_q beta_q(alpha) omega_{i-s-2+q}, q = 0..3, with
// s = floor(sigma) mod n and alpha its fractional part.
//
// The periodic tridiagonal solve uses the factorisation
//   T + 4 + T^{-1} = -(1/r)(1 - r T)(1 - r T^{-1}),  r = sqrt(3) - 2,
// (r is the root of r^2 + 4r + 1 = 0 inside the unit circle), so that
//   omega = -6 r (1 - r T^{-1})^{-1} (1 - r T)^{-1} u:
// a causal first-order recursion y_i = u_i + r y_{i-1} followed by an
// anti-causal one w_i = y_i + r w_{i+1}, each started from its periodic
// closed form y_0 = (1 - r^n)^{-1} sum_k r^k u_{-k}, truncated where r^k is
// below the rounding unit of the storage type.  The factor -6r is folded
// into the evaluation weights.  Every line is held in LDS for the solve and
// the evaluation, so omega never reaches HBM: each dof is read and written
// once.
//
// Tiles: lines along a strided axis are staged as [n][L] (L adjacent lines,
// one per lane, contiguous along the fastest axis); lines along the
// contiguous axis as [R][n+3] (an odd row length for even n, against LDS
// bank conflicts; room for wrapped copies of a row's first points).  One
// thread per line runs the two recursions; all threads load, evaluate and
// store element-parallel with contiguous global accesses.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

#include "field.hpp"

namespace vp {
namespace {

constexpr int kBlock = 256;

template <typename T>
struct SplineParams {
    T r;          // sqrt(3) - 2
    T inv_geo;    // 1 / (1 - r^n)
    int n;        // points per line
    int K;        // terms of the truncated periodic start sums
};

// beta_q(alpha) * (-6 r): the cubic B-spline weights of the four
// coefficients omega_{m-1..m+2}, m = i - s - 1, at distance t = 1 - alpha.
template <typename T>
__device__ __forceinline__ void spline_weights(double sigma, int n, int& s,
                                               T wq[4]) {
    double alpha;
    const bool ok = split_shift(sigma, n, s, alpha);
    const double t = 1.0 - alpha;
    const double t2 = t * t, t3 = t2 * t;
    const double g = -6.0 * (1.7320508075688772 - 2.0) / 6.0;  // -6r/6
    double b0 = (1.0 - t) * (1.0 - t) * (1.0 - t);
    double b1 = 3.0 * t3 - 6.0 * t2 + 4.0;
    double b2 = -3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0;
    double b3 = t3;
    if (!ok) b0 = b1 = b2 = b3 = __builtin_nan("");
    wq[0] = T(g * b0);
    wq[1] = T(g * b1);
    wq[2] = T(g * b2);
    wq[3] = T(g * b3);
}

// Segmented in-place periodic solve, called by every thread of the block.
// The thread owning segment [b, e) of the line at p (element i at
// p[i * stride]) starts each recursion from the truncated periodic sum of its
// predecessors (causal) or successors (anti-causal), so the Q segments of a
// line run in parallel:
//   y_{b-1} = inv_geo sum_{k<K} r^k u_{b-1-k},  y_i = u_i + r y_{i-1};
//   w_e     = inv_geo sum_{k<K} r^k y_{e+k},    w_i = y_i + r w_{i+1}
// (indices mod n).  With K = n the start values are the exact periodic sums.
template <typename T>
__device__ __forceinline__ T geometric_sum_down(const T* p, int stride, int j, int cnt,
                                                T r, T& rk, T acc) {
    // acc + sum_{k<cnt} rk r^k p[(j - k) * stride], four loads in flight
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const T x0 = p[(j - k) * stride], x1 = p[(j - k - 1) * stride];
        const T x2 = p[(j - k - 2) * stride], x3 = p[(j - k - 3) * stride];
        acc = fma(rk, x0, acc);
        rk *= r;
        acc = fma(rk, x1, acc);
        rk *= r;
        acc = fma(rk, x2, acc);
        rk *= r;
        acc = fma(rk, x3, acc);
        rk *= r;
    }
    for (; k < cnt; ++k) {
        acc = fma(rk, p[(j - k) * stride], acc);
        rk *= r;
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ T geometric_sum_up(const T* p, int stride, int j, int cnt,
                                              T r, T& rk, T acc) {
    // acc + sum_{k<cnt} rk r^k p[(j + k) * stride], four loads in flight
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
        const T x0 = p[(j + k) * stride], x1 = p[(j + k + 1) * stride];
        const T x2 = p[(j + k + 2) * stride], x3 = p[(j + k + 3) * stride];
        acc = fma(rk, x0, acc);
        rk *= r;
        acc = fma(rk, x1, acc);
        rk *= r;
        acc = fma(rk, x2, acc);
        rk *= r;
        acc = fma(rk, x3, acc);
        rk *= r;
    }
    for (; k < cnt; ++k) {
        acc = fma(rk, p[(j + k) * stride], acc);
        rk *= r;
    }
    return acc;
}

// Segmented in-place periodic solve, called by every thread of the block.
// The thread owning segment [b, e) of the line at p (element i at
// p[i * stride]) starts each recursion from the truncated periodic sum of its
// predecessors (causal) or successors (anti-causal), so the Q segments of a
// line run in parallel:
//   y_{b-1} = inv_geo sum_{k<K} r^k u_{b-1-k},  y_i = u_i + r y_{i-1};
//   w_e     = inv_geo sum_{k<K} r^k y_{e+k},    w_i = y_i + r w_{i+1}
// (indices mod n).  With K = n the start values are the exact periodic sums.
template <typename T>
__device__ __forceinline__ void spline_solve_segment(T* p, int stride, int b, int e,
                                                     bool active,
                                                     const SplineParams<T>& sp) {
    const int n = sp.n;
    const int K = sp.K;
    const T r = sp.r;
    T y = T(0);
    if (active) {
        // indices b-1 down to b-K: first those >= 0, then n-1 downwards
        T rk = T(1);
        const int run = min(K, b);
        T acc = geometric_sum_down<T>(p, stride, b - 1, run, r, rk, T(0));
        acc = geometric_sum_down<T>(p, stride, n - 1, K - run, r, rk, acc);
        y = acc * sp.inv_geo;
    }
    __syncthreads();
    if (active) {
        int i = b;
        for (; i + 4 <= e; i += 4) {
            const T x0 = p[i * stride], x1 = p[(i + 1) * stride];
            const T x2 = p[(i + 2) * stride], x3 = p[(i + 3) * stride];
            y = fma(r, y, x0);
            p[i * stride] = y;
            y = fma(r, y, x1);
            p[(i + 1) * stride] = y;
            y = fma(r, y, x2);
            p[(i + 2) * stride] = y;
            y = fma(r, y, x3);
            p[(i + 3) * stride] = y;
        }
        for (; i < e; ++i) {
            y = fma(r, y, p[i * stride]);
            p[i * stride] = y;
        }
    }
    __syncthreads();
    T w = T(0);
    if (active) {
        // indices e up to e+K-1: first those < n, then 0 upwards
        T rk = T(1);
        const int start = e < n ? e : 0;
        const int run = min(K, n - start);
        T acc = geometric_sum_up<T>(p, stride, start, run, r, rk, T(0));
        acc = geometric_sum_up<T>(p, stride, 0, K - run, r, rk, acc);
        w = acc * sp.inv_geo;
    }
    __syncthreads();
    if (active) {
        int i = e - 1;
        for (; i - 3 >= b; i -= 4) {
            const T x0 = p[i * stride], x1 = p[(i - 1) * stride];
            const T x2 = p[(i - 2) * stride], x3 = p[(i - 3) * stride];
            w = fma(r, w, x0);
            p[i * stride] = w;
            w = fma(r, w, x1);
            p[(i - 1) * stride] = w;
            w = fma(r, w, x2);
            p[(i - 2) * stride] = w;
            w = fma(r, w, x3);
            p[(i - 3) * stride] = w;
        }
        for (; i >= b; --i) {
            w = fma(r, w, p[i * stride]);
            p[i * stride] = w;
        }
    }
    __syncthreads();
}

// j + 1 reduced into [0, n) for j in [0, n)
__device__ __forceinline__ int next_idx(int j, int n) { return j + 1 < n ? j + 1 : j + 1 - n; }

// first index i - s - 2 reduced into [0, n), for i, s in [0, n)
__device__ __forceinline__ int first_tap(int i, int s, int n) {
    int j = i - s - 2;
    j += j < 0 ? n : 0;
    j += j < 0 ? n : 0;
    return j;
}

// kFwdRho: the forward sweep that also writes the partial density of its
// output (x2 sweeps with 32- or 64-line tiles; the workgroup's columns);
// kFwdRhoMom: and the workgroup's sums of the four moments of its output
enum { kFwd = 0, kAdj = 1, kDshift = 2, kFwdRho = 3, kFwdRhoMom = 4 };

// Longest segment a thread owns: tiles hold at most kTileBytes, so a
// segment has at most kTileBytes / (kBlock * sizeof(T)) points.
template <typename T>
struct SegMax {
    static constexpr int value = 48 * 1024 / (256 * static_cast<int>(sizeof(T)));
};

// d beta_q / d alpha times -6r (derivative of spline_weights).
template <typename T>
__device__ __forceinline__ void spline_dweights(double sigma, int n, int& s, T wq[4]) {
    double alpha;
    const bool ok = split_shift_floor(sigma, n, s, alpha);
    const double t = 1.0 - alpha;
    const double g = -6.0 * (1.7320508075688772 - 2.0) / 6.0;  // -6r/6
    // 6 d beta_q / dt; d/d alpha = -d/dt
    double d0 = -3.0 * (1.0 - t) * (1.0 - t);
    double d1 = 9.0 * t * t - 12.0 * t;
    double d2 = -9.0 * t * t + 6.0 * t + 3.0;
    double d3 = 3.0 * t * t;
    if (!ok) d0 = d1 = d2 = d3 = __builtin_nan("");
    wq[0] = T(-g * d0);
    wq[1] = T(-g * d1);
    wq[2] = T(-g * d2);
    wq[3] = T(-g * d3);
}

// Transposed evaluation on a segment, in place, called by every thread:
// mu_k = w3 lam_{k+s-1} + w2 lam_{k+s} + w1 lam_{k+s+1} + w0 lam_{k+s+2}
// for k in [b, e) (the gather form of the four-tap scatter).
template <typename T, int SM = SegMax<T>::value>
__device__ __forceinline__ void transposed_taps(T* p, int stride, int b, int e, int s, int n,
                                                T w0, T w1, T w2, T w3, bool active) {
    T mu[SM];
    if (active) {
        int j = b + s - 1;
        if (j < 0) j += n;
        if (j >= n) j -= n;
        T c0 = p[j * stride];
        j = next_idx(j, n);
        T c1 = p[j * stride];
        j = next_idx(j, n);
        T c2 = p[j * stride];
        j = next_idx(j, n);
        T c3 = p[j * stride];
#pragma unroll
        for (int t = 0; t < SM; ++t) {
            if (b + t < e) {
                mu[t] = fma(w0, c3, fma(w1, c2, fma(w2, c1, w3 * c0)));
                c0 = c1;
                c1 = c2;
                c2 = c3;
                j = next_idx(j, n);
                c3 = p[j * stride];
            }
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int t = 0; t < SM; ++t)
            if (b + t < e) p[(b + t) * stride] = mu[t];
    }
    __syncthreads();
}

// Lines along a strided axis.  Thread t owns line l = t % L (L adjacent
// lines of the fastest axis) and segment q = t / L of that line, for the
// load, the solve and the evaluation alike.
//   kFwd:    fout = E(alpha) C^{-1} fin
//   kAdj:    fout = C^{-1} E(alpha)^T fin            (fin = adjoint of the output)
//   kDshift: g[line] = <lam, E'(alpha) C^{-1} fin>    (per-line shift derivative)
// LS bounds the thread's segment: the FP64 loads in flight, the shift
// derivative's lam and the transposed taps take that many registers.  LT > 0
// fixes the tile's line count L at compile time (64-line tiles, and FP64
// 32-line ones): the solve's strided LDS accesses then pair into two-address
// loads and stores.  (FP32 32-line tiles ran slower that way: the 288^4 x1
// sweep 12.5 against 11.4 ms.)
template <typename T, int AXIS, int MODE, int LS = SegMax<T>::value, int LT = 0>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LS == 16 ? 5 : 1)))
spline_col(const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ lam,
           double* __restrict__ g, const double* __restrict__ shift, ShiftMap sm,
           int64_t nlines, int64_t inner, int L_, SplineParams<T> sp, RhoFuse rf) {
    const int L = LT > 0 ? LT : L_;
    constexpr bool RHO = MODE == kFwdRho || MODE == kFwdRhoMom;
    constexpr bool MOM = MODE == kFwdRhoMom;
    constexpr bool FWD = MODE == kFwd || RHO;
    __shared__ double mred[MOM ? 4 * (kBlock / 64) : 1];
    double s_m = 0.0, s_a = 0.0, s_q = 0.0;   // W2 f, W2 |f|, W2 f^2 of this line
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[MODE == kDshift ? kBlock : 1];
    const int n = sp.n;
    T* buf = reinterpret_cast<T*>(smem);   // [n][L]

    // the tile holds lines line0 .. line0+nl-1 of the flattened (outer,
    // inner) line index; a tile may straddle two outer indices
    const int64_t line0 = static_cast<int64_t>(blockIdx.x) * L;
    const int nl = static_cast<int>(min(static_cast<int64_t>(L), nlines - line0));

    const int l = threadIdx.x % L;
    const int64_t line = line0 + min(l, nl - 1);
    const int64_t o = line / inner;
    const int64_t kl = line - o * inner;
    const int64_t lbase = o * n * inner + kl;       // element 0 of the thread's line
    const int Q = kBlock / L;
    const int S = (n + Q - 1) / Q;
    const int b = min(n, (static_cast<int>(threadIdx.x) / L) * S);
    const int e = min(n, b + S);
    const bool active = l < nl && b < e;
    const T* __restrict__ src = fin + lbase;
    // the line's shift first: loads complete in order, so the wait for it
    // then covers none of the line's or lam's loads
    const double sigma = active ? shift[shift_offset(sm, o, kl)] : 0.0;
    if (active) {
        if constexpr (sizeof(T) == 8) {
            // FP64: the whole segment's loads in flight at once (the tile
            // size already limits the occupancy), indices clamped to the
            // segment's last point, whose slot the clamped loads store again
            // (no branch for the compiler to sink a load into)
            constexpr int kSeg = LS;
            for (int i0 = b; i0 < e; i0 += kSeg) {
                T v[kSeg];
#pragma unroll
                for (int u = 0; u < kSeg; ++u)
                    v[u] = src[static_cast<int64_t>(min(i0 + u, e - 1)) * inner];
#pragma unroll
                for (int u = 0; u < kSeg; ++u) buf[min(i0 + u, e - 1) * L + l] = v[u];
            }
        } else {
            // FP32: batches of 12 loads (registers, not the tile, limit the
            // occupancy here)
            constexpr int kV = 12;
            int i = b;
            for (; i + kV <= e; i += kV) {
                T v[kV];
#pragma unroll
                for (int u = 0; u < kV; ++u) v[u] = src[static_cast<int64_t>(i + u) * inner];
#pragma unroll
                for (int u = 0; u < kV; ++u) buf[(i + u) * L + l] = v[u];
            }
            for (; i < e; ++i) buf[i * L + l] = src[static_cast<int64_t>(i) * inner];
        }
    }
    // shift derivative: the thread's segment of lam, in flight during the
    // solve (clamped indices, no branches between the loads)
    constexpr int SM = LS;
    T lv[MODE == kDshift ? SM : 1];
    if (MODE == kDshift && active) {
        const T* __restrict__ lm = lam + lbase;
#pragma unroll
        for (int t = 0; t < SM; ++t)
            lv[t] = lm[static_cast<int64_t>(min(b + t, e - 1)) * inner];
    }
    int s = 0;
    T w0 = T(0), w1 = T(0), w2 = T(0), w3 = T(0);
    if (active) {
        T wq[4];
        if (MODE == kDshift)
            spline_dweights<T>(sigma, n, s, wq);
        else
            spline_weights<T>(sigma, n, s, wq);
        w0 = wq[0];
        w1 = wq[1];
        w2 = wq[2];
        w3 = wq[3];
    }
    __syncthreads();
    if (MODE == kAdj) transposed_taps<T, LS>(buf + l, L, b, e, s, n, w0, w1, w2, w3, active);
    spline_solve_segment<T>(buf + l, L, b, e, active, sp);
    if (MODE == kAdj) {
        if (active) {
            T* __restrict__ dst = fout + lbase;
            for (int i = b; i < e; ++i) put_out(&dst[static_cast<int64_t>(i) * inner], buf[i * L + l]);
        }
        return;
    }
    double acc = 0.0;
    if (active) {
        // sliding window over omega_{i-s-2 .. i-s+1}
        T* __restrict__ dst = fout + lbase;
        int j = first_tap(b, s, n);
        T c0 = buf[j * L + l];
        j = next_idx(j, n);
        T c1 = buf[j * L + l];
        j = next_idx(j, n);
        T c2 = buf[j * L + l];
        j = next_idx(j, n);
        T c3 = buf[j * L + l];
        int i = b;
        // density weight of the velocity columns: the spline's velocity
        // nodes are one per cell with equal weights (checked on the host),
        // so the weight multiplies the wavefront's sums instead of every
        // value
        const double wk = RHO ? rf.g3.w[0] * rf.g3.h * (rf.g4.w[0] * rf.g4.h) : 0.0;
        if (FWD) {
            for (; i + 4 <= e; i += 4) {
                const int j4 = next_idx(j, n), j5 = next_idx(j4, n);
                const int j6 = next_idx(j5, n), j7 = next_idx(j6, n);
                const T c4 = buf[j4 * L + l], c5 = buf[j5 * L + l];
                const T c6 = buf[j6 * L + l], c7 = buf[j7 * L + l];
                const T o0 = fma(w3, c3, fma(w2, c2, fma(w1, c1, w0 * c0)));
                const T o1 = fma(w3, c4, fma(w2, c3, fma(w1, c2, w0 * c1)));
                const T o2 = fma(w3, c5, fma(w2, c4, fma(w1, c3, w0 * c2)));
                const T o3 = fma(w3, c6, fma(w2, c5, fma(w1, c4, w0 * c3)));
                put_out(&dst[static_cast<int64_t>(i) * inner], o0);
                put_out(&dst[static_cast<int64_t>(i + 1) * inner], o1);
                put_out(&dst[static_cast<int64_t>(i + 2) * inner], o2);
                put_out(&dst[static_cast<int64_t>(i + 3) * inner], o3);
                if (RHO) {
                    // the wavefront's 64 lines share i: sums over them
                    double vals[4] = {static_cast<double>(o0), static_cast<double>(o1),
                                      static_cast<double>(o2), static_cast<double>(o3)};
                    if (MOM) {
                        // (the x2 weight, equal for all nodes, is applied at the end)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            s_m += vals[q];
                            s_a += fabs(vals[q]);
                            s_q = fma(vals[q], vals[q], s_q);
                        }
                    }
                    // lanes of one segment: the whole wavefront (64-line
                    // tiles) or its halves (32-line tiles, two segments)
                    if (L == 64) {
                        const double r = wave_sum4_rows(vals[0], vals[1], vals[2], vals[3]);
                        if ((threadIdx.x & 15) == 0)
                            rf.part[static_cast<int64_t>(blockIdx.x) * n + i + ((threadIdx.x & 63) >> 4)] = wk * r;
                    } else {
                        const int gl = threadIdx.x & (L - 1);
                        const double r = group_reduce_scatter<4, 32>(vals, threadIdx.x & 63);
                        if (gl < 4) rf.part[static_cast<int64_t>(blockIdx.x) * n + i + gl] = wk * r;
                    }
                }
                c0 = c4;
                c1 = c5;
                c2 = c6;
                c3 = c7;
                j = j7;
            }
        }
        if (FWD) {
            for (; i < e; ++i) {
                const T o = fma(w3, c3, fma(w2, c2, fma(w1, c1, w0 * c0)));
                put_out(&dst[static_cast<int64_t>(i) * inner], o);
                if (RHO) {
                    double vals[1] = {static_cast<double>(o)};
                    if (MOM) {
                        s_m += vals[0];
                        s_a += fabs(vals[0]);
                        s_q = fma(vals[0], vals[0], s_q);
                    }
                    const double r = L == 64 ? group_reduce_scatter<1, 64>(vals, threadIdx.x & 63)
                                             : group_reduce_scatter<1, 32>(vals, threadIdx.x & 63);
                    if ((threadIdx.x & (L - 1)) == 0)
                        rf.part[static_cast<int64_t>(blockIdx.x) * n + i] = wk * r;
                }
                c0 = c1;
                c1 = c2;
                c2 = c3;
                j = next_idx(j, n);
                c3 = buf[j * L + l];
            }
        } else {
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                if (b + t < e) {
                    const T v = fma(w3, c3, fma(w2, c2, fma(w1, c1, w0 * c0)));
                    acc = fma(static_cast<double>(lv[t]), static_cast<double>(v), acc);
                    c0 = c1;
                    c1 = c2;
                    c2 = c3;
                    j = next_idx(j, n);
                    c3 = buf[j * L + l];
                }
            }
        }
    }
    if (MODE == kDshift) {
        red[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x < nl) {
            double t = 0.0;
            for (int q = 0; q < Q; ++q) t += red[q * L + threadIdx.x];
            g[line0 + threadIdx.x] = t;
        }
    }
    if (MOM) {
        // workgroup sums of W f, W |f|, W f^2, W |v|^2 f (|v|^2 constant on
        // a line); every thread of the tile is active on this path
        const int k32 = static_cast<int>(kl);   // velocity index (< 2^31 here)
        const int v1 = k32 / rf.n4;
        const int v2 = k32 - v1 * rf.n4;
        const double a1 = rf.g3.lo + (static_cast<double>(v1) + rf.g3.xi[0]) * rf.g3.h;
        const double a2 = rf.g4.lo + (static_cast<double>(v2) + rf.g4.xi[0]) * rf.g4.h;
        const double wv = rf.g3.h * rf.g4.h;
        const double f0 = rf.g1.h * wv * rf.g2.h;   // the weights (one node per cell)
        const int lane = threadIdx.x & 63;
        const int wave = threadIdx.x >> 6;
        // one wavefront sum of the four: row t of the wavefront holds sum t
        const double r = wave_sum4_rows(f0 * s_m, f0 * s_a, f0 * s_q,
                                        f0 * (a1 * a1 + a2 * a2) * s_m);
        if ((lane & 15) == 0) mred[(lane >> 4) * (kBlock / 64) + wave] = r;
        __syncthreads();
        if (threadIdx.x < 4) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) t += mred[threadIdx.x * (kBlock / 64) + w];
            rf.mom_part[static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x] = t;
        }
    }
}

// Lines along the contiguous axis.  The R rows of a tile are one contiguous
// range of memory: loads and stores run over it flat (consecutive lanes,
// consecutive addresses, no idle lanes at row ends); the solve gives thread t
// row r = t % R and segment q = t / R.  Modes as for spline_col; LS (shift
// derivative and transposed sweep) bounds the thread's segment, so that the
// registers that hold its lam through the solve, or its transposed taps,
// match the segment and not the longest one.  RW > 0 (shift derivative):
// the evaluation goes by rows instead, wavefront w taking rows w, w + 4, ...
// (RW of them) and lane l points l, l + 64, ... (CW of them), so that lam
// arrives by whole-row loads.
template <typename T, int MODE, int LS, int RW = 0, int CW = 0>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    LS == 16 || (RW > 0 && RW <= 8 && RW * CW * sizeof(T) <= 128) ? 6 : RW > 0 ? 5 : 1)))
spline_row(const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ lam,
           double* __restrict__ g, const double* __restrict__ shift, ShiftMap sm,
           int64_t nrows, int R, SplineParams<T> sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = sp.n;
    // rows padded by three: after the solve, the rows read by four-tap
    // windows get wrapped copies of their first three points there, so that
    // the taps of any point are consecutive
    const int ld = n + 3;
    T* buf = reinterpret_cast<T*>(smem);   // [R][n+3]
    T* wts = buf + R * ld;                 // [R][4]
    int* sh = reinterpret_cast<int*>(wts + 4 * R);

    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
    const int nr = static_cast<int>(min(static_cast<int64_t>(R), nrows - row0));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    constexpr int kWaves = kBlock / 64;
    // the row's shift first: loads complete in order, so the wait for it
    // then covers none of the tile's or lam's loads
    const double sigma = static_cast<int>(threadIdx.x) < nr
                             ? shift[shift_offset(sm, row0 + threadIdx.x, 0)] : 0.0;
    // the tile's rows are contiguous in memory: flat element e = r*n + i,
    // (r, i) advanced by kBlock elements per round; kUR loads in flight with
    // indices clamped to the last element, whose slot the clamped lanes
    // store again (no branch for the compiler to sink a load into)
    const int cnt = nr * n;
    const int dr = kBlock / n;
    const int di = kBlock - dr * n;
    {
        const T* __restrict__ src = fin + row0 * n;
        int r = static_cast<int>(threadIdx.x) / n;
        int i = static_cast<int>(threadIdx.x) - r * n;
        constexpr int kUR = 12;   // one batch per FP64 tile, two per FP32 tile
        for (int e0 = threadIdx.x; e0 < cnt; e0 += kUR * kBlock) {
            T v[kUR];
            int pos[kUR];
#pragma unroll
            for (int u = 0; u < kUR; ++u) {
                const int e = e0 + u * kBlock;
                v[u] = src[e < cnt ? e : cnt - 1];
                pos[u] = r * ld + i;
                r += dr;
                i += di;
                if (i >= n) {
                    i -= n;
                    ++r;
                }
            }
            const int lastpos = (nr - 1) * ld + n - 1;
#pragma unroll
            for (int u = 0; u < kUR; ++u) buf[e0 + u * kBlock < cnt ? pos[u] : lastpos] = v[u];
        }
    }
    // shift derivative: each thread's segment of lam (the solve's mapping:
    // row t % R, points [b, e)), loaded before the solve so that it arrives
    // while the solve runs
    constexpr int SM = LS;
    T lseg[MODE == kDshift && RW == 0 ? SM : 1];
    T lrow[RW > 0 ? RW * CW : 1];
    if constexpr (MODE == kDshift && RW > 0) {
        // the wavefront's rows of lam, read along the rows (clamped
        // indices; the out-of-tile values are never used)
        const T* __restrict__ lr = lam + row0 * n;
        const int last = cnt - 1;
#pragma unroll
        for (int k = 0; k < RW; ++k) {
#pragma unroll
            for (int m = 0; m < CW; ++m) {
                const int r = wave + kWaves * k;
                const int i = lane + 64 * m;
                lrow[k * CW + m] = lr[r < nr && i < n ? r * n + i : last];
            }
        }
    } else if (MODE == kDshift) {
        const int r = threadIdx.x % R;
        const int Q = kBlock / R;
        const int S = (n + Q - 1) / Q;
        const int b = min(n, (static_cast<int>(threadIdx.x) / R) * S);
        const int e = min(n, b + S);
        if (r < nr) {
            const T* __restrict__ lr = lam + (row0 + r) * n;
#pragma unroll
            for (int t = 0; t < SM; ++t)
                if (b + t < e) lseg[t] = lr[b + t];
        }
    }
    if (threadIdx.x < nr) {
        const int r = threadIdx.x;
        int s;
        T wq[4];
        if (MODE == kDshift)
            spline_dweights<T>(sigma, n, s, wq);
        else
            spline_weights<T>(sigma, n, s, wq);
        wts[4 * r + 0] = wq[0];
        wts[4 * r + 1] = wq[1];
        wts[4 * r + 2] = wq[2];
        wts[4 * r + 3] = wq[3];
        sh[r] = s;
    }
    __syncthreads();
    {
        const int r = threadIdx.x % R;
        const int Q = kBlock / R;
        const int S = (n + Q - 1) / Q;
        const int b = min(n, (static_cast<int>(threadIdx.x) / R) * S);
        const int e = min(n, b + S);
        const bool active = r < nr && b < e;
        if (MODE == kAdj)
            transposed_taps<T, LS>(buf + r * ld, 1, b, e, active ? sh[r] : 0, n,
                               active ? wts[4 * r] : T(0), active ? wts[4 * r + 1] : T(0),
                               active ? wts[4 * r + 2] : T(0), active ? wts[4 * r + 3] : T(0),
                               active);
        spline_solve_segment<T>(buf + r * ld, 1, b, e, active, sp);
    }
    // the evaluations that read windows row[j0 .. j0 + 3], j0 in [0, n) (the
    // forward rows, the shift derivative by rows): point n + k holds point
    // k mod n
    if constexpr (MODE == kFwd || (MODE == kDshift && RW > 0)) {
        for (int t = threadIdx.x; t < 3 * nr; t += kBlock) {
            const int r = t / 3;
            const int k = t - 3 * r;
            buf[r * ld + n + k] = buf[r * ld + (k < n ? k : k % n)];
        }
        __syncthreads();
    }
    if (MODE != kDshift && sizeof(T) == 8) {
        // FP64: row by row, the row's weights and shift held in registers
        for (int r = wave; r < nr; r += kWaves) {
            const T* row = buf + r * ld;
            T* __restrict__ dst = fout + (row0 + r) * n;
            if (MODE == kAdj) {
                for (int i = lane; i < n; i += 64) put_out(&dst[i], row[i]);
                continue;
            }
            const T w0 = wts[4 * r + 0], w1 = wts[4 * r + 1];
            const T w2 = wts[4 * r + 2], w3 = wts[4 * r + 3];
            const int s = sh[r];
            for (int i = lane; i < n; i += 64) {
                const T* c = row + first_tap(i, s, n);
                put_out(&dst[i], fma(w3, c[3], fma(w2, c[2], fma(w1, c[1], w0 * c[0]))));
            }
        }
        return;
    }
    if (MODE != kDshift) {
        // FP32 rows, forward and transposed: element-parallel in memory
        // order (no idle lanes at row ends), the forward taps read as
        // windows of the padded row
        T* __restrict__ dst = fout + row0 * n;
        int r = static_cast<int>(threadIdx.x) / n;
        int i = static_cast<int>(threadIdx.x) - r * n;
        for (int e = threadIdx.x; e < cnt; e += kBlock) {
            const T* row = buf + r * ld;
            if (MODE == kAdj) {
                put_out(&dst[e], row[i]);
            } else {
                const T* c = row + first_tap(i, sh[r], n);
                const T* w = wts + 4 * r;
                put_out(&dst[e], fma(w[3], c[3], fma(w[2], c[2], fma(w[1], c[1], w[0] * c[0]))));
            }
            r += dr;
            i += di;
            if (i >= n) {
                i -= n;
                ++r;
            }
        }
        return;
    }
    if constexpr (RW > 0) {
        // shift derivative by rows: per-lane sums of lam_i v_i in FP64 for
        // four rows at a time, whose wavefront sums one wave_sum4_rows gives
        // (lane 16k holds row k's)
#pragma unroll
        for (int k0 = 0; k0 < RW; k0 += 4) {
            double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int r = wave + kWaves * (k0 + kk);
                if (k0 + kk < RW && r < nr) {
                    const T* row = buf + r * ld;
                    const T w0 = wts[4 * r + 0], w1 = wts[4 * r + 1];
                    const T w2 = wts[4 * r + 2], w3 = wts[4 * r + 3];
                    const int s = sh[r];
#pragma unroll
                    for (int m = 0; m < CW; ++m) {
                        const int i = lane + 64 * m;
                        if (i < n) {
                            const T* c = row + first_tap(i, s, n);
                            const T v = fma(w3, c[3], fma(w2, c[2], fma(w1, c[1], w0 * c[0])));
                            a[kk] = fma(static_cast<double>(lrow[(k0 + kk) * CW + m]),
                                        static_cast<double>(v), a[kk]);
                        }
                    }
                }
            }
            const double t = wave_sum4_rows(a[0], a[1], a[2], a[3]);
            const int r = wave + kWaves * (k0 + (lane >> 4));
            if ((lane & 15) == 0 && r < nr) g[row0 + r] = t;
        }
        return;
    }
    // shift derivative: each thread runs the sliding window of the forward
    // evaluation (one LDS read per point) along its own segment and adds
    // lam_i v_i in FP64; the segments of a row meet in LDS
    {
        const int r = threadIdx.x % R;
        const int Q = kBlock / R;
        const int S = (n + Q - 1) / Q;
        const int q = static_cast<int>(threadIdx.x) / R;
        const int b = min(n, q * S);
        const int e = min(n, b + S);
        double acc = 0.0;
        if (r < nr && b < e) {
            const T* row = buf + r * ld;
            const T w0 = wts[4 * r + 0], w1 = wts[4 * r + 1];
            const T w2 = wts[4 * r + 2], w3 = wts[4 * r + 3];
            int j = first_tap(b, sh[r], n);
            T c0 = row[j];
            j = next_idx(j, n);
            T c1 = row[j];
            j = next_idx(j, n);
            T c2 = row[j];
            j = next_idx(j, n);
            T c3 = row[j];
#pragma unroll
            for (int t = 0; t < SM; ++t) {
                if (b + t < e) {
                    const T v = fma(w3, c3, fma(w2, c2, fma(w1, c1, w0 * c0)));
                    acc = fma(static_cast<double>(lseg[t]), static_cast<double>(v), acc);
                    c0 = c1;
                    c1 = c2;
                    c2 = c3;
                    j = next_idx(j, n);
                    c3 = row[j];
                }
            }
        }
        // (the tile is free: every thread is past its last read of it)
        __syncthreads();
        double* red = reinterpret_cast<double*>(smem);   // [Q][R]
        red[q * R + r] = acc;
        __syncthreads();
        if (static_cast<int>(threadIdx.x) < nr) {
            double t = 0.0;
            for (int qq = 0; qq < Q; ++qq) t += red[qq * R + threadIdx.x];
            g[row0 + threadIdx.x] = t;
        }
    }
}

template <typename T>
SplineParams<T> make_params(int n) {
    const double r = std::sqrt(3.0) - 2.0;
    SplineParams<T> sp;
    sp.r = T(r);
    sp.inv_geo = T(1.0 / (1.0 - std::pow(r, n)));
    sp.n = n;
    // |r|^K / (1 - |r|) below the rounding unit: K = 28 (double), 14 (float)
    const int kmax = sizeof(T) == 8 ? 28 : 14;
    sp.K = n < kmax ? n : kmax;
    return sp;
}

constexpr size_t kTileBytes = 48 * 1024;

// The fused x2 sweeps' column tiles may take 64 KiB (64-line FP64 tiles up
// to 128 points a line, so that a wavefront's lanes are one segment of 64
// lines and its sums are whole-wavefront sums; two workgroups a compute
// unit: 1023 against 1072 us at 128^4); the other sweeps keep 48 KiB (at
// 128^4 the plain FP64 sweeps ran 3-11 % slower with the larger tiles),
// within which every segment also fits the transposed and shift-derivative
// sweeps' register arrays (SegMax).
constexpr size_t kFwdTileBytes = 64 * 1024;

// lines per column tile: a power of two up to 64 within the LDS budget
int tile_lines(int n, size_t esize, size_t budget = kTileBytes) {
    int L = 64;
    while (L > 1 && static_cast<size_t>(n) * L * esize > budget) L /= 2;
    return L;
}

template <typename T, int MODE>
vp_status launch_spline(int axis, const int64_t dims[4], const void* fin,
                        void* fout, const void* lam, double* g, const double* shift,
                        const ShiftMap& sm, hipStream_t st, const RhoFuse& rf = RhoFuse{}) {
    int64_t outer = 1, inner = 1;
    for (int d = 0; d < axis; ++d) outer *= dims[d];
    for (int d = axis + 1; d < 4; ++d) inner *= dims[d];
    const int n = static_cast<int>(dims[axis]);
    const SplineParams<T> sp = make_params<T>(n);
    const T* in = static_cast<const T*>(fin);
    T* out = static_cast<T*>(fout);
    const T* lm = static_cast<const T*>(lam);
    if (axis < 3) {
        // tiles run over the flattened line index
        constexpr bool RHO = MODE == kFwdRho || MODE == kFwdRhoMom;
        const size_t budget = RHO ? kFwdTileBytes : kTileBytes;
        const int L = tile_lines(n, sizeof(T), budget);
        size_t lds = static_cast<size_t>(n) * L * sizeof(T);
        if ((MODE == kFwdRho || MODE == kFwdRhoMom) &&
            (axis != 1 || (L != 64 && L != 32) || inner % L || n % (kBlock / L) ||
             inner >= (int64_t(1) << 31)))
            return set_error(VP_ERR_UNSUPPORTED,
                             "fused x2 sweep needs 32- or 64-line tiles of equal segments");
        if (lds > budget)
            return set_error(VP_ERR_UNSUPPORTED,
                             "spline_advect: line of %d points too long for the LDS tile", n);
        if (lds > kTileBytes) {
            static std::atomic<bool> attr_set{false};
            if (!attr_set.load(std::memory_order_relaxed)) {
                // dynamic LDS beyond the default (one setting covers the axes)
                // (only the fused x2 sweeps take tiles over 48 KiB)
                const void* fns[3] = {
                    reinterpret_cast<const void*>(&spline_col<T, 1, MODE>),
                    reinterpret_cast<const void*>(&spline_col<T, 1, MODE, SegMax<T>::value, 64>),
                    reinterpret_cast<const void*>(&spline_col<T, 1, MODE, SegMax<T>::value, 32>)};
                for (const void* fn : fns)
                    VP_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   static_cast<int>(kFwdTileBytes)));
                attr_set.store(true, std::memory_order_relaxed);
            }
        }
        const int64_t nlines = outer * inner;
        const int64_t grid64 = (nlines + L - 1) / L;
        if (grid64 >= (int64_t(1) << 31))
            return set_error(VP_ERR_UNSUPPORTED, "spline_advect: grid too large");
        const unsigned grid = static_cast<unsigned>(grid64);
        if constexpr (MODE == kFwdRho || MODE == kFwdRhoMom) {
            if (L == 64)
                spline_col<T, 1, MODE, SegMax<T>::value, 64><<<grid, kBlock, lds, st>>>(
                    in, out, lm, g, shift, sm, nlines, inner, L, sp, rf);
            else if (L == 32 && sizeof(T) == 8)
                spline_col<T, 1, MODE, SegMax<T>::value, 32><<<grid, kBlock, lds, st>>>(
                    in, out, lm, g, shift, sm, nlines, inner, L, sp, rf);
            else
                spline_col<T, 1, MODE><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, nlines, inner, L, sp, rf);
        } else {
            auto go = [&](auto ls) {
                constexpr int LS = decltype(ls)::value;
                auto launch = [&](auto lt) {
                    constexpr int LT = decltype(lt)::value;
                    switch (axis) {
                        case 0:
                            spline_col<T, 0, MODE, LS, LT><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, nlines, inner, L, sp, rf);
                            break;
                        case 1:
                            spline_col<T, 1, MODE, LS, LT><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, nlines, inner, L, sp, rf);
                            break;
                        default:
                            spline_col<T, 2, MODE, LS, LT><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, nlines, inner, L, sp, rf);
                            break;
                    }
                };
                if (L == 64)
                    launch(std::integral_constant<int, 64>{});
                else if (L == 32 && sizeof(T) == 8)
                    launch(std::integral_constant<int, 32>{});
                else
                    launch(std::integral_constant<int, 0>{});
            };
            // segment of ceil(n / (kBlock / L)) points: 16 or 24 registers
            // where it fits (FP32 forward loads go in batches of 12 and take
            // none of them)
            const int Q = kBlock / L;
            const int S = (n + Q - 1) / Q;
            if constexpr (sizeof(T) == 4 && MODE == kFwd) {
                go(std::integral_constant<int, SegMax<T>::value>{});
            } else {
                if (S <= 16)
                    go(std::integral_constant<int, 16>{});
                else if (S <= 24 || sizeof(T) == 8)
                    go(std::integral_constant<int, 24>{});
                else
                    go(std::integral_constant<int, SegMax<T>::value>{});
            }
        }
        return check_launch("spline_col");
    }
    if constexpr (MODE == kFwdRho || MODE == kFwdRhoMom) {
        return set_error(VP_ERR_UNSUPPORTED, "fused density only on x2 sweeps");
    } else {
    // rows per tile: a power of two (so every segment fits SegMax) within
    // the LDS budget
    int R = 64;
    while (R > 1 && static_cast<size_t>(R) * (n + 1) * sizeof(T) > kTileBytes) R /= 2;
    if (static_cast<size_t>(R) * (n + 1) * sizeof(T) > kTileBytes)
        return set_error(VP_ERR_UNSUPPORTED,
                         "spline_advect: line of %d points too long for the LDS tile", n);
    // (the shift derivative adds its segment sums in the tile afterwards:
    // kBlock doubles)
    const size_t lds = std::max(static_cast<size_t>(R) * (n + 3) * sizeof(T) +
                                    static_cast<size_t>(R) * (4 * sizeof(T) + sizeof(int)),
                                MODE == kDshift ? kBlock * sizeof(double) : size_t(0));
    const int64_t grid64 = (outer + R - 1) / R;
    if (grid64 >= (int64_t(1) << 31))
        return set_error(VP_ERR_UNSUPPORTED, "spline_advect: grid too large");
    const unsigned grid = static_cast<unsigned>(grid64);
    if constexpr (MODE == kDshift || MODE == kAdj) {
        // segment of ceil(n / (kBlock / R)) points; 16 or 24 registers where
        // it fits (the FP64 shift derivative at 96 points, 12 a segment: 4
        // against 6 wavefronts a SIMD with the 24-point bound)
        const int Q = kBlock / R;
        const int S = (n + Q - 1) / Q;
        if constexpr (MODE == kDshift) {
            // by rows where a lane's share of lam is 12-20 FP64 or 16-40
            // FP32 values: rows per wavefront and 64-point chunks per row
            // (rows of at most 64, 96-128, 192 and 257-320 points in FP64;
            // at most 128, 192 and 257-320 in FP32); other lengths by
            // segments
            const int rw = R / (kBlock / 64), cw = (n + 63) / 64;
            auto rows = [&](auto rwc, auto cwc) {
                spline_row<T, MODE, 1, decltype(rwc)::value, decltype(cwc)::value>
                    <<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, outer, R, sp);
                return check_launch("spline_row");
            };
            using I16 = std::integral_constant<int, 16>;
            using I8 = std::integral_constant<int, 8>;
            using I4 = std::integral_constant<int, 4>;
            using I5 = std::integral_constant<int, 5>;
            using I3 = std::integral_constant<int, 3>;
            using I2 = std::integral_constant<int, 2>;
            using I1 = std::integral_constant<int, 1>;
            if (rw == 16 && cw == 1) return rows(I16{}, I1{});
            if constexpr (sizeof(T) == 8) {
                if (rw == 8 && cw == 2) return rows(I8{}, I2{});
                if (rw == 4 && cw == 3) return rows(I4{}, I3{});
                if (rw == 4 && cw == 5) return rows(I4{}, I5{});
            } else {
                if (rw == 16 && cw == 2) return rows(I16{}, I2{});
                if (rw == 8 && cw == 3) return rows(I8{}, I3{});
                if (rw == 8 && cw == 5) return rows(I8{}, I5{});
            }
        }
        if (S <= 16)
            spline_row<T, MODE, 16><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, outer, R, sp);
        else if (S <= 24 || sizeof(T) == 8)
            spline_row<T, MODE, 24><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, outer, R, sp);
        else
            spline_row<T, MODE, SegMax<T>::value><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm,
                                                                            outer, R, sp);
    } else {
        spline_row<T, MODE, 1><<<grid, kBlock, lds, st>>>(in, out, lm, g, shift, sm, outer, R, sp);
    }
    return check_launch("spline_row");
    }
}

}  // namespace

vp_status spline_advect_impl(int axis, vp_dtype dt, const int64_t dims[4],
                             const void* f_in, void* f_out, const double* shift,
                             const int64_t shift_stride[4], hipStream_t st, bool adjoint) {
    const ShiftMap sm = make_shift_map(axis, dims, shift_stride);
    if (dt == VP_F64)
        return adjoint ? launch_spline<double, kAdj>(axis, dims, f_in, f_out, nullptr, nullptr, shift, sm, st)
                       : launch_spline<double, kFwd>(axis, dims, f_in, f_out, nullptr, nullptr, shift, sm, st);
    return adjoint ? launch_spline<float, kAdj>(axis, dims, f_in, f_out, nullptr, nullptr, shift, sm, st)
                   : launch_spline<float, kFwd>(axis, dims, f_in, f_out, nullptr, nullptr, shift, sm, st);
}

vp_status spline_advect_rho_impl(vp_dtype dt, const int64_t dims[4], const void* f_in,
                                 void* f_out, const double* shift,
                                 const int64_t shift_stride[4], const RhoFuse& rf,
                                 hipStream_t st) {
    // (point grids: one node per cell on every axis, so the quadrature
    // weights of a velocity column and of an x2 node do not vary)
    if (rf.g1.m != 1 || rf.g2.m != 1 || rf.g3.m != 1 || rf.g4.m != 1)
        return set_error(VP_ERR_UNSUPPORTED, "fused spline x2 sweep: point grids only");
    const ShiftMap sm = make_shift_map(1, dims, shift_stride);
    if (dt == VP_F64)
        return rf.mom_part
                   ? launch_spline<double, kFwdRhoMom>(1, dims, f_in, f_out, nullptr, nullptr,
                                                       shift, sm, st, rf)
                   : launch_spline<double, kFwdRho>(1, dims, f_in, f_out, nullptr, nullptr,
                                                    shift, sm, st, rf);
    return rf.mom_part
               ? launch_spline<float, kFwdRhoMom>(1, dims, f_in, f_out, nullptr, nullptr, shift,
                                                  sm, st, rf)
               : launch_spline<float, kFwdRho>(1, dims, f_in, f_out, nullptr, nullptr, shift, sm,
                                               st, rf);
}

int spline_rho_group(vp_dtype dt, const int64_t dims[4]) {
    // the lanes of a segment must run the same evaluation steps: tiles of 64
    // lines (one segment per wavefront) or 32 (two), segments of equal length
    const int L = tile_lines(static_cast<int>(dims[1]), dtype_size(dt), kFwdTileBytes);
    if (L != 64 && L != 32) return 0;
    if ((dims[2] * dims[3]) % L || dims[1] % (kBlock / L)) return 0;
    if (dims[2] * dims[3] >= (int64_t(1) << 31)) return 0;   // 32-bit velocity index
    return L;
}

vp_status spline_dshift_impl(int axis, vp_dtype dt, const int64_t dims[4], const void* f_in,
                             const void* lam, const double* shift,
                             const int64_t shift_stride[4], double* g_line, hipStream_t st) {
    const ShiftMap sm = make_shift_map(axis, dims, shift_stride);
    if (dt == VP_F64)
        return launch_spline<double, kDshift>(axis, dims, f_in, nullptr, lam, g_line, shift, sm, st);
    return launch_spline<float, kDshift>(axis, dims, f_in, nullptr, lam, g_line, shift, sm, st);
}

}  // namespace vp

namespace {

vp_status check_spline_args(int axis, vp_dtype dt, const int64_t dims[4], const void* a,
                            const void* b, const double* shift,
                            const int64_t shift_stride[4], int64_t* total) {
    using namespace vp;
    if (axis < 0 || axis > 3) return set_error(VP_ERR_ARG, "axis %d not in 0..3", axis);
    if (dt != VP_F32 && dt != VP_F64) return set_error(VP_ERR_ARG, "bad dtype %d", (int)dt);
    vp_status rc = check_dims(dims, total);
    if (rc != VP_OK) return rc;
    if (!a || !b || !shift) return set_error(VP_ERR_ARG, "NULL pointer argument");
    return check_shift_strides(axis, dims, shift_stride);
}

}  // namespace

extern "C" vp_status spline_advect(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                                   const void* f_in, void* f_out,
                                   const double* shift,
                                   const int64_t shift_stride[4], void* stream) {
    using namespace vp;
    clear_error();
    if (degree != 3)
        return set_error(VP_ERR_UNSUPPORTED, "spline degree %d: only the cubic spline (3)",
                         degree);
    int64_t total = 0;
    vp_status rc = check_spline_args(axis, dt, dims, f_in, f_out, shift, shift_stride, &total);
    if (rc != VP_OK) return rc;
    if (ranges_overlap(f_in, f_out, static_cast<size_t>(total) * dtype_size(dt)))
        return set_error(VP_ERR_ALIAS, "f_in and f_out overlap");
    return spline_advect_impl(axis, dt, dims, f_in, f_out, shift, shift_stride,
                              static_cast<hipStream_t>(stream), false);
}

extern "C" vp_status spline_advect_adjoint(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                                           const void* lam_out, void* lam_in,
                                           const double* shift,
                                           const int64_t shift_stride[4], void* stream) {
    using namespace vp;
    clear_error();
    if (degree != 3)
        return set_error(VP_ERR_UNSUPPORTED, "spline degree %d: only the cubic spline (3)",
                         degree);
    int64_t total = 0;
    vp_status rc = check_spline_args(axis, dt, dims, lam_out, lam_in, shift, shift_stride,
                                     &total);
    if (rc != VP_OK) return rc;
    if (ranges_overlap(lam_out, lam_in, static_cast<size_t>(total) * dtype_size(dt)))
        return set_error(VP_ERR_ALIAS, "lam_out and lam_in overlap");
    return spline_advect_impl(axis, dt, dims, lam_out, lam_in, shift, shift_stride,
                              static_cast<hipStream_t>(stream), true);
}

extern "C" vp_status spline_advect_dshift(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                                          const void* f_in, const void* lam_out,
                                          const double* shift,
                                          const int64_t shift_stride[4], double* g_line,
                                          void* stream) {
    using namespace vp;
    clear_error();
    if (degree != 3)
        return set_error(VP_ERR_UNSUPPORTED, "spline degree %d: only the cubic spline (3)",
                         degree);
    int64_t total = 0;
    vp_status rc = check_spline_args(axis, dt, dims, f_in, lam_out, shift, shift_stride, &total);
    if (rc != VP_OK) return rc;
    if (!g_line) return set_error(VP_ERR_ARG, "NULL pointer argument");
    return spline_dshift_impl(axis, dt, dims, f_in, lam_out, shift, shift_stride, g_line,
                              static_cast<hipStream_t>(stream));
}
