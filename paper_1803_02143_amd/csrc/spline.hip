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

// In-place periodic solve on one line: element i at p[i * stride].
template <typename T>
__device__ __forceinline__ void spline_solve_line(T* p, int stride,
                                                  const SplineParams<T>& sp) {
    const int n = sp.n;
    const T r = sp.r;
    // causal: y_0 = inv_geo * sum_{k<K} r^k u_{(n-k) mod n}
    T acc = p[0];
    T rk = r;
    for (int k = 1; k < sp.K; ++k) {
        acc = fma(rk, p[(n - k) * stride], acc);
        rk *= r;
    }
    T y = acc * sp.inv_geo;
    p[0] = y;
    for (int i = 1; i < n; ++i) {
        y = fma(r, y, p[i * stride]);
        p[i * stride] = y;
    }
    // anti-causal: w_{n-1} = inv_geo * sum_{k<K} r^k y_{(n-1+k) mod n}
    acc = p[(n - 1) * stride];
    rk = r;
    for (int k = 1; k < sp.K; ++k) {
        acc = fma(rk, p[(k - 1) * stride], acc);
        rk *= r;
    }
    T w = acc * sp.inv_geo;
    p[(n - 1) * stride] = w;
    for (int i = n - 2; i >= 0; --i) {
        w = fma(r, w, p[i * stride]);
        p[i * stride] = w;
    }
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

template <typename T, int AXIS>
__global__ void __launch_bounds__(kBlock)
spline_col(const T* __restrict__ fin, T* __restrict__ fout,
           const double* __restrict__ shift, ShiftMap sm, int64_t inner, int L,
           int64_t tiles_per_outer, SplineParams<T> sp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = sp.n;
    T* buf = reinterpret_cast<T*>(smem);   // [n][L]
    T* wts = buf + n * L;                  // [L][4]
    int* sh = reinterpret_cast<int*>(wts + 4 * L);

    const int64_t o = blockIdx.x / tiles_per_outer;
    const int64_t k0 = (blockIdx.x - o * tiles_per_outer) * L;
    const int nl = static_cast<int>(min(static_cast<int64_t>(L), inner - k0));
    const int64_t base = o * n * inner + k0;

    const int lane = threadIdx.x % L;
    const int row_step = kBlock / L;
    if (lane < nl) {
        // batches of kU independent loads keep many requests in flight
        int i = threadIdx.x / L;
        for (; i + (kU - 1) * row_step < n; i += kU * row_step) {
            T v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                v[u] = fin[base + static_cast<int64_t>(i + u * row_step) * inner + lane];
#pragma unroll
            for (int u = 0; u < kU; ++u) buf[(i + u * row_step) * L + lane] = v[u];
        }
        for (; i < n; i += row_step)
            buf[i * L + lane] = fin[base + static_cast<int64_t>(i) * inner + lane];
    }
    __syncthreads();
    if (threadIdx.x < nl) {
        const int l = threadIdx.x;
        int s;
        T wq[4];
        spline_weights<T>(shift[shift_offset(sm, o, k0 + l)], n, s, wq);
        wts[4 * l + 0] = wq[0];
        wts[4 * l + 1] = wq[1];
        wts[4 * l + 2] = wq[2];
        wts[4 * l + 3] = wq[3];
        sh[l] = s;
        spline_solve_line<T>(buf + l, L, sp);
    }
    __syncthreads();
    if (lane < nl) {
        const T w0 = wts[4 * lane + 0], w1 = wts[4 * lane + 1];
        const T w2 = wts[4 * lane + 2], w3 = wts[4 * lane + 3];
        const int s = sh[lane];
        for (int i = threadIdx.x / L; i < n; i += row_step) {
            const int j0 = first_tap(i, s, n);
            const int j1 = wrap(j0 + 1, n), j2 = wrap(j0 + 2, n), j3 = wrap(j0 + 3, n);
            T acc = w0 * buf[j0 * L + lane];
            acc = fma(w1, buf[j1 * L + lane], acc);
            acc = fma(w2, buf[j2 * L + lane], acc);
            acc = fma(w3, buf[j3 * L + lane], acc);
            fout[base + i * inner + lane] = acc;
        }
    }
}

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
    __syncthreads();
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
        spline_solve_line<T>(buf + r * ld, 1, sp);
    }
    __syncthreads();
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
    // |r|^K below the rounding unit: K = 40 (double), 20 (float)
    const int kmax = sizeof(T) == 8 ? 40 : 20;
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
        int L = 64;
        while (L > 1 && (static_cast<size_t>(n) * L * sizeof(T) > kTileBytes ||
                         L / 2 >= inner))
            L /= 2;
        const size_t lds = static_cast<size_t>(n) * L * sizeof(T) +
                           static_cast<size_t>(L) * (4 * sizeof(T) + sizeof(int));
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
