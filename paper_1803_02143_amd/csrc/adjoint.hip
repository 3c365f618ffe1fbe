// Reverse-mode pieces that are not sweeps: the transposed density and the
// per-line shift-derivative reduction.
//
// The density rho(x1,x2) = sum_{c,e} W3_c W4_e f[x1][x2][c][e] (Sec. 2) is
// linear in f; its transpose broadcasts rho_bar over the velocity block of
// every (x1, x2) point with the same quadrature weights.  One wavefront per
// point, contiguous accesses, kU stores (and loads when accumulating) in
// flight.
#include <cmath>

#include "field.hpp"

namespace vp {
namespace {

constexpr int kBlk = 256;
constexpr int kU = 8;

__device__ __forceinline__ double node_weight_d(const AxisGrid& g, int64_t c) {
    return g.w[c % g.m] * g.h;
}

template <typename T, bool ACC>
__global__ void __launch_bounds__(kBlk)
density_adjoint_kernel(const double* __restrict__ rho_bar, T* __restrict__ lam, int n3,
                       int n4, AxisGrid g3, AxisGrid g4, int64_t nblk) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* wt3 = reinterpret_cast<double*>(smem);
    double* wt4 = wt3 + n3;
    for (int c = threadIdx.x; c < n3; c += kBlk) wt3[c] = node_weight_d(g3, c);
    for (int d = threadIdx.x; d < n4; d += kBlk) wt4[d] = node_weight_d(g4, d);
    __syncthreads();
    constexpr int kWaves = kBlk / 64;
    const int lane = threadIdx.x & 63;
    const int total = n3 * n4;
    const int step_c = 64 / n4;
    const int step_d = 64 - step_c * n4;
    const int c0 = lane / n4;
    const int d0 = lane - c0 * n4;
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * kWaves + (threadIdx.x >> 6); b < nblk;
         b += static_cast<int64_t>(gridDim.x) * kWaves) {
        T* __restrict__ blk = lam + b * total;
        const double rb = rho_bar[b];
        int c = c0, d = d0;
        for (int e = lane; e < total; e += kU * 64) {
            T old[kU];
            double w[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const bool ok = e + u * 64 < total;
                if (ACC) old[u] = blk[ok ? e + u * 64 : total - 1];
                w[u] = ok ? wt3[c] * wt4[d] : 0.0;
                c += step_c;
                d += step_d;
                if (d >= n4) {
                    d -= n4;
                    ++c;
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                if (e + u * 64 < total) {
                    const double v = rb * w[u];
                    put_out(&blk[e + u * 64], ACC ? static_cast<T>(static_cast<double>(old[u]) + v)
                                                  : static_cast<T>(v));
                }
            }
        }
    }
}

// out[b] = scale * sum_{k<K} g[b*K + k]: one wavefront per b.
__global__ void __launch_bounds__(kBlk)
line_sum(const double* __restrict__ g, int64_t nb, int K, double scale,
         double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t b = static_cast<int64_t>(blockIdx.x) * (kBlk / 64) + (threadIdx.x >> 6);
    if (b >= nb) return;
    double acc = 0.0;
    for (int k = lane; k < K; k += 64) acc += g[b * K + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) out[b] = scale * acc;
}

}  // namespace

vp_status density_adjoint_impl(int degree, vp_dtype dt, const int64_t dims[4],
                               const double* rho_bar, double len_v1, double len_v2,
                               void* lam, bool accumulate, hipStream_t st) {
    const AxisGrid g3 = axis_grid(degree, dims[2], 0.0, len_v1);
    const AxisGrid g4 = axis_grid(degree, dims[3], 0.0, len_v2);
    const int64_t nblk = dims[0] * dims[1];
    const int n3 = static_cast<int>(dims[2]), n4 = static_cast<int>(dims[3]);
    const size_t lds = sizeof(double) * (static_cast<size_t>(n3) + n4);
    if (lds > 48 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "velocity axes of %d x %d nodes too long", n3, n4);
    int64_t grid = (nblk + kBlk / 64 - 1) / (kBlk / 64);
    if (grid > 8192) grid = 8192;
    const unsigned g = static_cast<unsigned>(grid);
    if (dt == VP_F64) {
        double* l = static_cast<double*>(lam);
        if (accumulate)
            density_adjoint_kernel<double, true><<<g, kBlk, lds, st>>>(rho_bar, l, n3, n4, g3, g4, nblk);
        else
            density_adjoint_kernel<double, false><<<g, kBlk, lds, st>>>(rho_bar, l, n3, n4, g3, g4, nblk);
    } else {
        float* l = static_cast<float*>(lam);
        if (accumulate)
            density_adjoint_kernel<float, true><<<g, kBlk, lds, st>>>(rho_bar, l, n3, n4, g3, g4, nblk);
        else
            density_adjoint_kernel<float, false><<<g, kBlk, lds, st>>>(rho_bar, l, n3, n4, g3, g4, nblk);
    }
    return check_launch("density_adjoint");
}

vp_status line_sum_impl(const double* g, int64_t nb, int K, double scale, double* out,
                        hipStream_t st) {
    line_sum<<<blocks_for(nb, kBlk / 64), kBlk, 0, st>>>(g, nb, K, scale, out);
    return check_launch("line_sum");
}

}  // namespace vp

extern "C" vp_status vp_density_adjoint(int degree, vp_dtype dt, const int64_t dims[4],
                                        const double* rho_bar, double len_v1, double len_v2,
                                        void* lam, int accumulate, void* stream) {
    using namespace vp;
    clear_error();
    int64_t total = 0;
    vp_status rc = check_grid_args(degree, dt, dims, &total);
    if (rc != VP_OK) return rc;
    if (!rho_bar || !lam) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if (!(len_v1 > 0.0) || !(len_v2 > 0.0))
        return set_error(VP_ERR_ARG, "velocity box lengths must be positive");
    return density_adjoint_impl(degree, dt, dims, rho_bar, len_v1, len_v2, lam, accumulate != 0,
                                static_cast<hipStream_t>(stream));
}
