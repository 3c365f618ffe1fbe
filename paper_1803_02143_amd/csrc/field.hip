// Velocity moments (density and diagnostics) and initial conditions.
//
// rho(x1, x2) = int f dv (Sec. 2) and the diagnostics of Sec. 4 (mass, L1,
// L2, kinetic energy) are read-only reductions over the contiguous
// (v1, v2) block that belongs to every (x1, x2) point.  One wavefront owns
// one block: it reads the block with contiguous loads, weights every value
// with the nodal quadrature (Gauss-Legendre weights times the cell width for
// SLDG, the spacing for the spline grid) and reduces in FP64 by cross-lane
// shuffles.  No atomics, so results are deterministic.
#include <algorithm>
#include <cmath>

#include "vp4d_internal.hpp"
#include "field.hpp"

namespace vp {

AxisGrid axis_grid(int degree, int64_t n, double lo, double len) {
    AxisGrid a{};
    a.lo = lo;
    if (degree < 0) {
        a.m = 1;
        a.w[0] = 1.0;
        a.xi[0] = 0.5;
        a.h = len / static_cast<double>(n);
    } else {
        const NodeBasis& b = node_basis(degree);
        a.m = b.m;
        for (int j = 0; j < b.m; ++j) {
            a.w[j] = b.w[j];
            a.xi[j] = b.xi[j];
        }
        a.h = len / static_cast<double>(n / b.m);
    }
    return a;
}

namespace {

constexpr int kU = 8;  // loads issued back to back per thread

__device__ __forceinline__ double node_coord(const AxisGrid& g, int64_t c) {
    const int64_t cell = c / g.m;
    return g.lo + (static_cast<double>(cell) + g.xi[c - cell * g.m]) * g.h;
}

__device__ __forceinline__ double node_weight(const AxisGrid& g, int64_t c) {
    return g.w[c % g.m] * g.h;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per (x1,x2) point b: out[b] = sum_{c,e} W3_c W4_e f[b][c][e], and when DIAG
// also out[nblk + b] = sum W |f|, out[2 nblk + b] = sum W f^2 and
// out[3 nblk + b] = sum W (v1^2 + v2^2) f.  One wavefront per point (its
// N3*N4 values are contiguous), kU loads in flight per lane, cross-lane
// shuffle reduction; the weight tables are built once per workgroup.
template <typename T, bool DIAG>
__global__ void __launch_bounds__(kRedBlock)
velocity_reduce(const T* __restrict__ f, int n3, int n4, AxisGrid g3,
                AxisGrid g4, double* __restrict__ out, int64_t nblk) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* wt3 = reinterpret_cast<double*>(smem);
    double* wt4 = wt3 + n3;
    double* vq3 = wt4 + n4;              // v^2 tables, DIAG only
    double* vq4 = vq3 + (DIAG ? n3 : 0);

    for (int c = threadIdx.x; c < n3; c += kRedBlock) {
        wt3[c] = node_weight(g3, c);
        if (DIAG) {
            const double v = node_coord(g3, c);
            vq3[c] = v * v;
        }
    }
    for (int e = threadIdx.x; e < n4; e += kRedBlock) {
        wt4[e] = node_weight(g4, e);
        if (DIAG) {
            const double v = node_coord(g4, e);
            vq4[e] = v * v;
        }
    }
    __syncthreads();

    constexpr int kWaves = kRedBlock / 64;
    const int lane = threadIdx.x & 63;
    const int total = n3 * n4;
    // element e = c*n4 + d; (c, d) advance by 64 elements per round
    const int step_c = 64 / n4;
    const int step_d = 64 - step_c * n4;
    const int c0 = lane / n4;
    const int d0 = lane - c0 * n4;
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * kWaves + (threadIdx.x >> 6); b < nblk;
         b += static_cast<int64_t>(gridDim.x) * kWaves) {
        const T* __restrict__ blk = f + b * total;
        int c = c0, d = d0;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int e = lane; e < total; e += kU * 64) {
            T x[kU];
            int cc[kU], dd[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                // clamped index instead of a branch: all kU loads issue back to back
                const bool ok = e + u * 64 < total;
                x[u] = blk[ok ? e + u * 64 : total - 1];
                if (!ok) x[u] = T(0);
                cc[u] = ok ? c : 0;
                dd[u] = ok ? d : 0;
                c += step_c;
                d += step_d;
                if (d >= n4) {
                    d -= n4;
                    ++c;
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const double xv = static_cast<double>(x[u]);
                const double wv = wt3[cc[u]] * wt4[dd[u]];
                acc[0] = fma(wv, xv, acc[0]);
                if (DIAG) {
                    acc[1] = fma(wv, fabs(xv), acc[1]);
                    acc[2] = fma(wv * xv, xv, acc[2]);
                    acc[3] = fma(wv * xv, vq3[cc[u]] + vq4[dd[u]], acc[3]);
                }
            }
        }
        const double s0 = wave_sum64(acc[0]);
        if (DIAG) {
            const double s1 = wave_sum64(acc[1]);
            const double s2 = wave_sum64(acc[2]);
            const double s3 = wave_sum64(acc[3]);
            if (lane == 0) {
                out[b] = s0;
                out[nblk + b] = s1;
                out[2 * nblk + b] = s2;
                out[3 * nblk + b] = s3;
            }
        } else if (lane == 0) {
            out[b] = s0;
        }
    }
}

// The density without weight tables, one workgroup per point (its four
// wavefronts interleave 64-value chunks of the block, so a point is done four
// times sooner than by one wavefront and the last round of workgroups is
// short).  Thread t reads the elements e = t + 256 j.  When 256 P is a
// multiple of N4 m (m nodes per cell, the period of the weights), the
// element in slot k = j mod P of every round of P loads has the same
// (c mod m, e mod N4), so its weight W3_c W4_e is fixed per thread and slot:
// the weights live in registers and every value costs one FMA.
template <typename T, int P>
__global__ void __launch_bounds__(kRedBlock)
density_slots(const T* __restrict__ f, int n3, int n4, AxisGrid g3, AxisGrid g4,
              double* __restrict__ out, int64_t nblk) {
    __shared__ double red[kRedBlock / 64];
    const int tid = threadIdx.x;
    const int total = n3 * n4;
    double wk[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int e = tid + kRedBlock * k;
        const int c = e / n4;
        wk[k] = node_weight(g3, c) * node_weight(g4, e - c * n4);
    }
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
        const T* __restrict__ blk = f + b * total;
        double acc = 0.0;
        for (int q0 = tid; q0 < total; q0 += kRedBlock * P) {
            T x[P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int q = q0 + kRedBlock * k;
                x[k] = blk[q < total ? q : total - 1];
            }
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double xv = q0 + kRedBlock * k < total ? static_cast<double>(x[k]) : 0.0;
                acc = fma(wk[k], xv, acc);
            }
        }
        const double sw = wave_sum64(acc);
        if ((tid & 63) == 0) red[tid >> 6] = sw;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kRedBlock / 64; ++w) t += red[w];
            out[b] = t;
        }
        __syncthreads();
    }
}

// rho[a][j] = sum over the groups g of part[(a * groups + g) * n2 + j]:
// workgroup (j-block, a), lane -> j, wavefront w sums the groups g = w mod 4
// (four independent accumulators each), the four partial sums meet in LDS.
// A fixed order, so the result is reproducible.
__global__ void __launch_bounds__(256)
rho_from_parts(const double* __restrict__ part, int64_t groups, int64_t n2,
               double* __restrict__ rho) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t a = blockIdx.y;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    const int64_t jc = j < n2 ? j : n2 - 1;
    const double* __restrict__ p = part + a * groups * n2 + jc;
    // eight independent accumulators: eight loads of each wavefront in flight
    double t[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t g = wave;
    for (; g + 28 < groups; g += 32) {
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] += p[(g + 4 * u) * n2];
    }
    for (; g < groups; g += 4) t[0] += p[g * n2];
    red[wave][lane] = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    __syncthreads();
    if (wave == 0 && j < n2)
        rho[a * n2 + j] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

constexpr int kFinalBlock = 1024;

// out4 = (mass, L1, L2, kinetic) from per-workgroup sums of the fused x2
// sweep: thread t adds parts t, t + 1024, ... in order, then a fixed-order
// block reduction.
__global__ void __launch_bounds__(kFinalBlock)
moments_from_parts(const double* __restrict__ part, int64_t nparts, double* __restrict__ out4) {
    __shared__ double red[4][kFinalBlock / 64];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q = threadIdx.x; q < nparts; q += kFinalBlock)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += part[4 * q + k];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum64(acc[k]);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < kFinalBlock / 64; ++w) t += red[threadIdx.x][w];
        if (threadIdx.x == 2) t = sqrt(t);
        if (threadIdx.x == 3) t *= 0.5;
        out4[threadIdx.x] = t;
    }
}

// First stage of a long moments_from_parts: block b adds the parts of its
// contiguous chunk [b per, (b+1) per) (thread t: parts t, t + 256, ... of
// the chunk, then a fixed-order block reduction) into chunk[4 b + k].
constexpr int kChunkBlock = 256;
constexpr int kMaxChunks = 512;
__global__ void __launch_bounds__(kChunkBlock)
moments_chunks(const double* __restrict__ part, int64_t nparts, int64_t per,
               double* __restrict__ chunk) {
    __shared__ double red[4][kChunkBlock / 64];
    const int64_t q0 = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t q1 = min(nparts, q0 + per);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kChunkBlock)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += part[4 * q + k];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum64(acc[k]);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < kChunkBlock / 64; ++w) t += red[threadIdx.x][w];
        chunk[4 * static_cast<int64_t>(blockIdx.x) + threadIdx.x] = t;
    }
}

// out4 = (mass, L1, L2, kinetic) from the per-(x1,x2) partial sums.
__global__ void __launch_bounds__(kFinalBlock)
moments_final(const double* __restrict__ part, int n1, int n2, AxisGrid g1,
              AxisGrid g2, double* __restrict__ out4) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* wt1 = reinterpret_cast<double*>(smem);
    double* wt2 = wt1 + n1;
    __shared__ double red[4 * (kFinalBlock / 64)];
    for (int a = threadIdx.x; a < n1; a += kFinalBlock) wt1[a] = node_weight(g1, a);
    for (int b = threadIdx.x; b < n2; b += kFinalBlock) wt2[b] = node_weight(g2, b);
    __syncthreads();
    const int64_t nblk = static_cast<int64_t>(n1) * n2;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q0 = threadIdx.x; q0 < nblk; q0 += kU * kFinalBlock) {
        double x[kU][4], w[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t q = q0 + u * kFinalBlock;
            const bool ok = q < nblk;
            const int64_t qc = ok ? q : nblk - 1;   // clamped: no branch around the loads
            const int64_t a = qc / n2;
            w[u] = ok ? wt1[a] * wt2[qc - a * n2] : 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) x[u][k] = part[k * nblk + qc];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] = fma(w[u], x[u][k], acc[k]);
    }
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = wave_sum64(acc[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) red[wv * 4 + k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < kFinalBlock / 64; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) t[k] += red[i * 4 + k];
        out4[0] = t[0];
        out4[1] = t[1];
        out4[2] = sqrt(t[2]);
        out4[3] = 0.5 * t[3];
    }
}

struct IcParams {
    int kind;
    double eps, k, v0;
};

template <typename T>
__global__ void __launch_bounds__(256)
init_kernel(T* __restrict__ f, int64_t total, int64_t n2, int64_t n3,
            int64_t n4, AxisGrid g1, AxisGrid g2, AxisGrid g3, AxisGrid g4,
            IcParams p) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
         idx < total; idx += stride) {
        int64_t r = idx;
        const int64_t i4 = r % n4;
        r /= n4;
        const int64_t i3 = r % n3;
        r /= n3;
        const int64_t i2 = r % n2;
        const int64_t i1 = r / n2;
        const double x1 = node_coord(g1, i1), x2 = node_coord(g2, i2);
        const double v1 = node_coord(g3, i3), v2 = node_coord(g4, i4);
        double val;
        if (p.kind == 0) {
            val = (1.0 + p.eps * (cos(p.k * x1) + cos(p.k * x2))) *
                  exp(-0.5 * (v1 * v1 + v2 * v2)) * (0.5 / M_PI);
        } else {
            const double px = p.kind == 1
                                  ? 1.0 + p.eps * (cos(p.k * x1) + cos(p.k * x2))
                                  : 1.0 + p.eps * cos(p.k * x1) * cos(p.k * x2);
            const double a1 = v1 - p.v0, b1 = v1 + p.v0;
            const double a2 = v2 - p.v0, b2 = v2 + p.v0;
            const double g1v = exp(-0.5 * a1 * a1) + exp(-0.5 * b1 * b1);
            const double g2v = exp(-0.5 * a2 * a2) + exp(-0.5 * b2 * b2);
            val = px * g1v * g2v * (0.125 / M_PI);
        }
        f[idx] = static_cast<T>(val);
    }
}

template <typename T>
vp_status launch_reduce(bool diag, const int64_t dims[4], const void* f,
                        const AxisGrid& g3, const AxisGrid& g4, double* out,
                        hipStream_t st) {
    const int64_t nblk = dims[0] * dims[1];
    const int n3 = static_cast<int>(dims[2]), n4 = static_cast<int>(dims[3]);
    const size_t lds = (diag ? 2 : 1) * sizeof(double) * (static_cast<size_t>(n3) + n4);
    if (lds > 48 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "velocity axes of %d x %d nodes too long", n3, n4);
    if (nblk >= (int64_t(1) << 31))
        return set_error(VP_ERR_UNSUPPORTED, "too many (x1, x2) points");
    const T* fp = static_cast<const T*>(f);
    // one wavefront per (x1, x2) point, at most 8192 workgroups
    int64_t grid = (nblk + kRedBlock / 64 - 1) / (kRedBlock / 64);
    if (grid > 8192) grid = 8192;
    // register weights when the weight pattern repeats within a few rounds
    const int64_t nm = static_cast<int64_t>(n4) * g3.m;
    int64_t gg = kRedBlock;
    for (int64_t a = nm; a; ) { const int64_t t = gg % a; gg = a; a = t; }
    const int64_t period = nm / gg;    // P with 256 P = 0 mod (N4 m)
    const bool same_m = g3.m == g4.m;
    const unsigned gr = static_cast<unsigned>(grid);
    const unsigned gp = static_cast<unsigned>(nblk);   // one workgroup per point
    // (the density only: with the four moment sums, register weights cost
    // more occupancy than the table lookups they save)
#define VP_SLOTS(PP)                                                                          \
    if (!diag && same_m && period == PP) {                                                    \
        density_slots<T, PP><<<gp, kRedBlock, 0, st>>>(fp, n3, n4, g3, g4, out, nblk);        \
        return check_launch("density_slots");                                                 \
    }
    VP_SLOTS(1) VP_SLOTS(2) VP_SLOTS(3) VP_SLOTS(4) VP_SLOTS(6) VP_SLOTS(8) VP_SLOTS(9)
    VP_SLOTS(12)
#undef VP_SLOTS
    if (diag)
        velocity_reduce<T, true><<<gr, kRedBlock, lds, st>>>(fp, n3, n4, g3, g4, out, nblk);
    else
        velocity_reduce<T, false><<<gr, kRedBlock, lds, st>>>(fp, n3, n4, g3, g4, out, nblk);
    return check_launch("velocity_reduce");
}

}  // namespace

vp_status moments_from_parts_impl(const double* mom_part, int64_t nparts, double* chunk,
                                  double* out4, hipStream_t st) {
    // one block adds a few thousand parts quickly (two per thread); beyond
    // that the parts are first added in contiguous chunks of one part per
    // thread (more per thread only past kMaxChunks chunks), whose loads are
    // all in flight at once
    if (nparts > 2 * kFinalBlock && chunk) {
        const int64_t per = std::max<int64_t>(kChunkBlock, (nparts + kMaxChunks - 1) / kMaxChunks);
        const int64_t used = (nparts + per - 1) / per;
        moments_chunks<<<static_cast<unsigned>(used), kChunkBlock, 0, st>>>(mom_part, nparts,
                                                                           per, chunk);
        vp_status rc = check_launch("moments_chunks");
        if (rc != VP_OK) return rc;
        moments_from_parts<<<1, kFinalBlock, 0, st>>>(chunk, used, out4);
        return check_launch("moments_from_parts");
    }
    moments_from_parts<<<1, kFinalBlock, 0, st>>>(mom_part, nparts, out4);
    return check_launch("moments_from_parts");
}

size_t moments_chunk_doubles() { return 4 * static_cast<size_t>(kMaxChunks); }

int64_t rho_fuse_workgroups(int method, int degree, vp_dtype dt, const int64_t dims[4]) {
    const int64_t nvel = dims[2] * dims[3];
    if (method == 0) return sldg_rho_workgroups(dt, degree, dims);
    const int gsz = spline_rho_group(dt, dims);
    return gsz > 0 ? dims[0] * nvel / gsz : 0;
}

vp_status rho_from_parts_impl(const double* part, int64_t n1, int64_t groups, int64_t n2,
                              double* rho, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n2 + 63) / 64), static_cast<unsigned>(n1));
    rho_from_parts<<<grid, 256, 0, st>>>(part, groups, n2, rho);
    return check_launch("rho_from_parts");
}

vp_status density_impl(int degree, vp_dtype dt, const int64_t dims[4],
                       const void* f, double len_v1, double len_v2, double* rho,
                       hipStream_t st) {
    const AxisGrid g3 = axis_grid(degree, dims[2], 0.0, len_v1);
    const AxisGrid g4 = axis_grid(degree, dims[3], 0.0, len_v2);
    if (dt == VP_F64) return launch_reduce<double>(false, dims, f, g3, g4, rho, st);
    return launch_reduce<float>(false, dims, f, g3, g4, rho, st);
}

vp_status moments_partial_impl(int degree, vp_dtype dt, const int64_t dims[4],
                               const void* f, const double lo[4],
                               const double len[4], double* partial,
                               hipStream_t st) {
    const AxisGrid g3 = axis_grid(degree, dims[2], lo[2], len[2]);
    const AxisGrid g4 = axis_grid(degree, dims[3], lo[3], len[3]);
    if (dt == VP_F64) return launch_reduce<double>(true, dims, f, g3, g4, partial, st);
    return launch_reduce<float>(true, dims, f, g3, g4, partial, st);
}

vp_status moments_final_impl(int degree, const int64_t dims[4],
                             const double lo[4], const double len[4],
                             const double* partial, double* out4,
                             hipStream_t st) {
    const AxisGrid g1 = axis_grid(degree, dims[0], lo[0], len[0]);
    const AxisGrid g2 = axis_grid(degree, dims[1], lo[1], len[1]);
    const size_t lds = sizeof(double) * static_cast<size_t>(dims[0] + dims[1]);
    if (lds > 48 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "x axes too long for the moment reduction");
    moments_final<<<1, kFinalBlock, lds, st>>>(partial, static_cast<int>(dims[0]),
                                               static_cast<int>(dims[1]), g1, g2, out4);
    return check_launch("moments_final");
}

static vp_status check_degree_dims(int degree, const int64_t dims[4], int64_t* total) {
    if (degree < -1 || degree > VP_MAX_DEGREE)
        return set_error(VP_ERR_UNSUPPORTED, "degree %d not in -1..%d", degree, VP_MAX_DEGREE);
    vp_status rc = check_dims(dims, total);
    if (rc != VP_OK) return rc;
    if (degree >= 0)
        for (int d = 0; d < 4; ++d)
            if (dims[d] % (degree + 1))
                return set_error(VP_ERR_ARG, "dims[%d] = %lld not a multiple of %d", d,
                                 (long long)dims[d], degree + 1);
    return VP_OK;
}

vp_status check_grid_args(int degree, vp_dtype dt, const int64_t dims[4], int64_t* total) {
    if (dt != VP_F32 && dt != VP_F64) return set_error(VP_ERR_ARG, "bad dtype %d", (int)dt);
    return check_degree_dims(degree, dims, total);
}

}  // namespace vp

using namespace vp;

extern "C" vp_status vp_density(int degree, vp_dtype dt, const int64_t dims[4],
                                const void* f, double len_v1, double len_v2,
                                double* rho, void* stream) {
    clear_error();
    int64_t total = 0;
    vp_status rc = check_grid_args(degree, dt, dims, &total);
    if (rc != VP_OK) return rc;
    if (!f || !rho) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if (!(len_v1 > 0.0) || !(len_v2 > 0.0))
        return set_error(VP_ERR_ARG, "velocity box lengths must be positive");
    return density_impl(degree, dt, dims, f, len_v1, len_v2, rho,
                        static_cast<hipStream_t>(stream));
}

extern "C" size_t vp_moments_workspace(const int64_t dims[4]) {
    if (!dims || dims[0] < 1 || dims[1] < 1) return 0;
    return 4 * sizeof(double) * static_cast<size_t>(dims[0]) * static_cast<size_t>(dims[1]);
}

extern "C" vp_status vp_moments(int degree, vp_dtype dt, const int64_t dims[4],
                                const void* f, const double lo[4],
                                const double len[4], double* out4,
                                void* workspace, size_t ws_bytes, void* stream) {
    clear_error();
    int64_t total = 0;
    vp_status rc = check_grid_args(degree, dt, dims, &total);
    if (rc != VP_OK) return rc;
    if (!f || !out4 || !lo || !len) return set_error(VP_ERR_ARG, "NULL pointer argument");
    for (int d = 0; d < 4; ++d)
        if (!(len[d] > 0.0)) return set_error(VP_ERR_ARG, "len[%d] must be positive", d);
    if (!workspace || ws_bytes < vp_moments_workspace(dims))
        return set_error(VP_ERR_WORKSPACE, "workspace of %zu bytes needed",
                         vp_moments_workspace(dims));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* part = static_cast<double*>(workspace);
    rc = moments_partial_impl(degree, dt, dims, f, lo, len, part, st);
    if (rc != VP_OK) return rc;
    return moments_final_impl(degree, dims, lo, len, part, out4, st);
}

extern "C" vp_status vp_init(int kind, double eps, double k, double v0, int degree,
                             vp_dtype dt, const int64_t dims[4], const double lo[4],
                             const double len[4], void* f, void* stream) {
    clear_error();
    int64_t total = 0;
    vp_status rc = check_grid_args(degree, dt, dims, &total);
    if (rc != VP_OK) return rc;
    if (kind < 0 || kind > 2) return set_error(VP_ERR_ARG, "initial condition kind %d", kind);
    if (!f || !lo || !len) return set_error(VP_ERR_ARG, "NULL pointer argument");
    for (int d = 0; d < 4; ++d)
        if (!(len[d] > 0.0)) return set_error(VP_ERR_ARG, "len[%d] must be positive", d);
    AxisGrid g[4];
    for (int d = 0; d < 4; ++d) g[d] = axis_grid(degree, dims[d], lo[d], len[d]);
    IcParams p{kind, eps, k, v0};
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dt == VP_F64)
        init_kernel<double><<<static_cast<unsigned>(blocks), 256, 0, st>>>(
            static_cast<double*>(f), total, dims[1], dims[2], dims[3], g[0], g[1], g[2], g[3], p);
    else
        init_kernel<float><<<static_cast<unsigned>(blocks), 256, 0, st>>>(
            static_cast<float*>(f), total, dims[1], dims[2], dims[3], g[0], g[1], g[2], g[3], p);
    return check_launch("init_kernel");
}
