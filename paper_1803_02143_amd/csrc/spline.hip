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
// contiguous axis as [R][n+1] (padded against LDS bank conflicts).  One
// thread per line runs the two recursions; all threads load, evaluate and
// store element-parallel with contiguous global accesses.
#include <cmath>

#include "vp4d_internal.hpp"

namespace vp {
namespace {

constexpr int kBlock = 256;
constexpr int kU = 8;  // loads issued back to back per thread

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
__device__ __forceinline__ void spline_solve_segment(T* p, int stride, int b, int e,
                                                     bool active,
                                                     const SplineParams<T>& sp) {
    const int n = sp.n;
    const T r = sp.r;
    T y = T(0);
    if (active) {
        T acc = T(0), rk = T(1);
        int j = b - 1;
        if (j < 0) j += n;
        for (int k = 0; k < sp.K; ++k) {
            acc = fma(rk, p[j * stride], acc);
            rk *= r;
            if (--j < 0) j += n;
        }
        y = acc * sp.inv_geo;
    }
    __syncthreads();
    if (active) {
        for (int i = b; i < e; ++i) {
            y = fma(r, y, p[i * stride]);
            p[i * stride] = y;
        }
    }
    __syncthreads();
    T w = T(0);
    if (active) {
        T acc = T(0), rk = T(1);
        int j = e;
        if (j >= n) j -= n;
        for (int k = 0; k < sp.K; ++k) {
            acc = fma(rk, p[j * stride], acc);
            rk *= r;
            if (++j >= n) j -= n;
        }
        w = acc * sp.inv_geo;
    }
    __syncthreads();
    if (active) {
        for (int i = e - 1; i >= b; --i) {
            w = fma(r, w, p[i * stride]);
            p[i * stride] = w;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int wrap(int j, int n) {
    while (j >= n) j -= n;
    return j;
}

// first index i - s - 2 reduced into [0, n)
__device__ __forceinline__ int first_tap(int i, int s, int n) {
    int j = i - s - 2;
    while (j < 0) j += n;
    return j;
}

// Lines along a strided axis.  Thread t owns line l = t % L (L adjacent
// lines of the fastest axis) and segment q = t / L of that line, for the
// load, the solve and the evaluation alike.
template <typename T, int AXIS>
__global__ void __launch_bounds__(kBlock)
spline_col(const T* __restrict__ fin, T* __restrict__ fout,
           const double* __restrict__ shift, ShiftMap sm, int64_t inner, int L,
           int64_t tiles_per_outer, SplineParams<T> sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = sp.n;
    T* buf = reinterpret_cast<T*>(smem);   // [n][L]

    const int64_t o = blockIdx.x / tiles_per_outer;
    const int64_t k0 = (blockIdx.x - o * tiles_per_outer) * L;
    const int nl = static_cast<int>(min(static_cast<int64_t>(L), inner - k0));
    const int64_t base = o * n * inner + k0;

    const int l = threadIdx.x % L;
    const int Q = kBlock / L;
    const int S = (n + Q - 1) / Q;
    const int b = min(n, (static_cast<int>(threadIdx.x) / L) * S);
    const int e = min(n, b + S);
    const bool active = l < nl && b < e;
    const T* __restrict__ src = fin + base + l;
    T* __restrict__ dst = fout + base + l;
    if (active) {
        // batches of kU independent loads keep many requests in flight
        int i = b;
        for (; i + kU <= e; i += kU) {
            T v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) v[u] = src[static_cast<int64_t>(i + u) * inner];
#pragma unroll
            for (int u = 0; u < kU; ++u) buf[(i + u) * L + l] = v[u];
        }
        for (; i < e; ++i) buf[i * L + l] = src[static_cast<int64_t>(i) * inner];
    }
    int s = 0;
    T w0 = T(0), w1 = T(0), w2 = T(0), w3 = T(0);
    if (active) {
        T wq[4];
        spline_weights<T>(shift[shift_offset(sm, o, k0 + l)], n, s, wq);
        w0 = wq[0];
        w1 = wq[1];
        w2 = wq[2];
        w3 = wq[3];
    }
    __syncthreads();
    spline_solve_segment<T>(buf + l, L, b, e, active, sp);
    if (active) {
        // sliding window over omega_{i-s-2 .. i-s+1}
        int j = first_tap(b, s, n);
        T c0 = buf[j * L + l];
        j = wrap(j + 1, n);
        T c1 = buf[j * L + l];
        j = wrap(j + 1, n);
        T c2 = buf[j * L + l];
        j = wrap(j + 1, n);
        T c3 = buf[j * L + l];
        for (int i = b; i < e; ++i) {
            T acc = w0 * c0;
            acc = fma(w1, c1, acc);
            acc = fma(w2, c2, acc);
            acc = fma(w3, c3, acc);
            dst[static_cast<int64_t>(i) * inner] = acc;
            c0 = c1;
            c1 = c2;
            c2 = c3;
            j = wrap(j + 1, n);
            c3 = buf[j * L + l];
        }
    }
}

// Lines along the contiguous axis.  Loads and stores are element-parallel
// (consecutive threads, consecutive addresses); the solve gives thread t
// row r = t % R and segment q = t / R.
template <typename T>
__global__ void __launch_bounds__(kBlock)
spline_row(const T* __restrict__ fin, T* __restrict__ fout,
           const double* __restrict__ shift, ShiftMap sm, int64_t nrows, int R,
           SplineParams<T> sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = sp.n;
    const int ld = n + 1;
    T* buf = reinterpret_cast<T*>(smem);   // [R][n+1]
    T* wts = buf + R * ld;                 // [R][4]
    int* sh = reinterpret_cast<int*>(wts + 4 * R);

    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
    const int nr = static_cast<int>(min(static_cast<int64_t>(R), nrows - row0));
    const int64_t base = row0 * n;
    const int cnt = nr * n;
    // row of element e: exact for e < 2^16 with the rounded reciprocal
    const float inv_n = 1.0f / static_cast<float>(n);
    {
        int e = threadIdx.x;
        for (; e + (kU - 1) * kBlock < cnt; e += kU * kBlock) {
            T v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) v[u] = fin[base + e + u * kBlock];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int q = e + u * kBlock;
                const int r = static_cast<int>((static_cast<float>(q) + 0.5f) * inv_n);
                buf[r * ld + (q - r * n)] = v[u];
            }
        }
        for (; e < cnt; e += kBlock) {
            const int r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv_n);
            buf[r * ld + (e - r * n)] = fin[base + e];
        }
    }
    if (threadIdx.x < nr) {
        const int r = threadIdx.x;
        int s;
        T wq[4];
        spline_weights<T>(shift[shift_offset(sm, row0 + r, 0)], n, s, wq);
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
        spline_solve_segment<T>(buf + r * ld, 1, b, e, r < nr && b < e, sp);
    }
    for (int e = threadIdx.x; e < cnt; e += kBlock) {
        const int r = static_cast<int>((static_cast<float>(e) + 0.5f) * inv_n);
        const int i = e - r * n;
        const T* row = buf + r * ld;
        const T* w = wts + 4 * r;
        const int j0 = first_tap(i, sh[r], n);
        T acc = w[0] * row[j0];
        acc = fma(w[1], row[wrap(j0 + 1, n)], acc);
        acc = fma(w[2], row[wrap(j0 + 2, n)], acc);
        acc = fma(w[3], row[wrap(j0 + 3, n)], acc);
        fout[base + e] = acc;
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

template <typename T>
vp_status launch_spline(int axis, const int64_t dims[4], const void* fin,
                        void* fout, const double* shift, const ShiftMap& sm,
                        hipStream_t st) {
    int64_t outer = 1, inner = 1;
    for (int d = 0; d < axis; ++d) outer *= dims[d];
    for (int d = axis + 1; d < 4; ++d) inner *= dims[d];
    const int n = static_cast<int>(dims[axis]);
    const SplineParams<T> sp = make_params<T>(n);
    const T* in = static_cast<const T*>(fin);
    T* out = static_cast<T*>(fout);
    if (axis < 3) {
        // lines per tile: a power of two dividing the fastest block when one
        // of at least 16 does, within the LDS budget
        int L = 64;
        while (L > 16 && inner % L) L /= 2;
        if (inner % L) L = 64;
        while (L > 1 && (static_cast<size_t>(n) * L * sizeof(T) > kTileBytes || L / 2 >= inner))
            L /= 2;
        const size_t lds = static_cast<size_t>(n) * L * sizeof(T);
        if (lds > 64 * 1024)
            return set_error(VP_ERR_UNSUPPORTED,
                             "spline_advect: line of %d points too long for the LDS tile", n);
        const int64_t tiles = (inner + L - 1) / L;
        const int64_t grid64 = outer * tiles;
        if (grid64 >= (int64_t(1) << 31))
            return set_error(VP_ERR_UNSUPPORTED, "spline_advect: grid too large");
        const unsigned grid = static_cast<unsigned>(grid64);
        switch (axis) {
            case 0:
                spline_col<T, 0><<<grid, kBlock, lds, st>>>(in, out, shift, sm, inner, L, tiles, sp);
                break;
            case 1:
                spline_col<T, 1><<<grid, kBlock, lds, st>>>(in, out, shift, sm, inner, L, tiles, sp);
                break;
            default:
                spline_col<T, 2><<<grid, kBlock, lds, st>>>(in, out, shift, sm, inner, L, tiles, sp);
                break;
        }
        return check_launch("spline_col");
    }
    int R = static_cast<int>(kTileBytes / ((static_cast<size_t>(n) + 1) * sizeof(T)));
    if (R > 64) R = 64;
    if (R < 1)
        return set_error(VP_ERR_UNSUPPORTED,
                         "spline_advect: line of %d points too long for the LDS tile", n);
    const size_t lds = static_cast<size_t>(R) * (n + 1) * sizeof(T) +
                       static_cast<size_t>(R) * (4 * sizeof(T) + sizeof(int));
    const int64_t grid64 = (outer + R - 1) / R;
    if (grid64 >= (int64_t(1) << 31))
        return set_error(VP_ERR_UNSUPPORTED, "spline_advect: grid too large");
    spline_row<T><<<static_cast<unsigned>(grid64), kBlock, lds, st>>>(in, out, shift, sm, outer, R, sp);
    return check_launch("spline_row");
}

}  // namespace

vp_status spline_advect_impl(int axis, vp_dtype dt, const int64_t dims[4],
                             const void* f_in, void* f_out, const double* shift,
                             const int64_t shift_stride[4], hipStream_t st) {
    const ShiftMap sm = make_shift_map(axis, dims, shift_stride);
    if (dt == VP_F64) return launch_spline<double>(axis, dims, f_in, f_out, shift, sm, st);
    return launch_spline<float>(axis, dims, f_in, f_out, shift, sm, st);
}

}  // namespace vp

extern "C" vp_status spline_advect(int axis, vp_dtype dt, const int64_t dims[4],
                                   const void* f_in, void* f_out,
                                   const double* shift,
                                   const int64_t shift_stride[4], void* stream) {
    using namespace vp;
    clear_error();
    if (axis < 0 || axis > 3) return set_error(VP_ERR_ARG, "axis %d not in 0..3", axis);
    if (dt != VP_F32 && dt != VP_F64) return set_error(VP_ERR_ARG, "bad dtype %d", (int)dt);
    int64_t total = 0;
    vp_status rc = check_dims(dims, &total);
    if (rc != VP_OK) return rc;
    if (!f_in || !f_out || !shift) return set_error(VP_ERR_ARG, "NULL pointer argument");
    rc = check_shift_strides(axis, dims, shift_stride);
    if (rc != VP_OK) return rc;
    if (ranges_overlap(f_in, f_out, static_cast<size_t>(total) * dtype_size(dt)))
        return set_error(VP_ERR_ALIAS, "f_in and f_out overlap");
    return spline_advect_impl(axis, dt, dims, f_in, f_out, shift, shift_stride,
                              static_cast<hipStream_t>(stream));
}
