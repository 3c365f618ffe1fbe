// Periodic 2D Poisson solve for the electric field (Sec. 1, Eq. (1)).
//
// div E = rho - 1, curl E = 0  =>  E = -grad phi, -Lap phi = rho - 1, so in
// Fourier space E_hat = -i k rho_hat / |k|^2 for k != 0.  The transforms are
// dense discrete Fourier transforms, one axis at a time, with the twiddle
// factors exp(-2 pi i j/n) tabulated once per call (the grids are at most a
// few hundred points per axis, so O(n^3) work is microseconds).
//
// SLDG grids: the nodal density of every cell is first mapped to the values
// at m = degree+1 equidistant sub-cell midpoints (Q[p][l] = L_l((p+1/2)/m)),
// which together form a uniform grid of n points; the field is computed
// there and mapped back with Q^{-1}.  Modes with m1 = 0 = m2 and modes with
// m1 = n1/2 or m2 = n2/2 (even n) are set to zero.  The electric energy
// W = 1/2 int |E|^2 uses the nodal quadrature of the grid.
//
// Kernel sequence (all FP64, workspace = 4 complex n1 x n2 arrays plus the
// two twiddle tables):
//   transfer_in   rho -> C0 (uniform-grid values), twiddles
//   dft_rows      C0 -> C1          (transform along x2)
//   dft_cols      C1 -> C0 = E1_hat, C2 = E2_hat  (along x1, spectral solve)
//   idft_cols     C0 -> C1, C2 -> C3
//   idft_rows     C1, C3 -> real fields (E directly, or scratch for SLDG)
//   transfer_out  scratch -> E1, E2   (SLDG only)
//   energy        E1, E2 -> W
#include <cmath>

#include "field.hpp"

namespace vp {
namespace {

struct Cplx {
    double re, im;
};

struct Transfer {
    int m;
    double q[kMaxNodes][kMaxNodes];
};

__global__ void __launch_bounds__(256)
transfer_in(const double* __restrict__ rho, Cplx* __restrict__ c0,
            Cplx* __restrict__ tw1, Cplx* __restrict__ tw2, int n1, int n2,
            Transfer t, int use_q) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid < n1) {
        double s, c;
        sincospi(2.0 * static_cast<double>(gid) / n1, &s, &c);
        tw1[gid] = Cplx{c, -s};
    }
    if (gid < n2) {
        double s, c;
        sincospi(2.0 * static_cast<double>(gid) / n2, &s, &c);
        tw2[gid] = Cplx{c, -s};
    }
    if (gid >= static_cast<int64_t>(n1) * n2) return;
    const int a = static_cast<int>(gid / n2);
    const int b = static_cast<int>(gid - static_cast<int64_t>(a) * n2);
    double v;
    if (use_q) {
        const int m = t.m;
        const int pa = a % m, pb = b % m;
        const int a0 = a - pa, b0 = b - pb;
        v = 0.0;
        for (int p = 0; p < m; ++p) {
            double row = 0.0;
            for (int q = 0; q < m; ++q)
                row = fma(t.q[pb][q], rho[static_cast<int64_t>(a0 + p) * n2 + b0 + q], row);
            v = fma(t.q[pa][p], row, v);
        }
    } else {
        v = rho[gid];
    }
    c0[gid] = Cplx{v, 0.0};
}

// out[a][k] = sum_b in[a][b] * tw[(b k) mod n]   (conj twiddles if INV)
template <bool INV>
__global__ void __launch_bounds__(256)
dft_rows(const Cplx* __restrict__ in, Cplx* __restrict__ out,
         const Cplx* __restrict__ tw, int n1, int n2) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= static_cast<int64_t>(n1) * n2) return;
    const int a = static_cast<int>(gid / n2);
    const int k = static_cast<int>(gid - static_cast<int64_t>(a) * n2);
    const Cplx* row = in + static_cast<int64_t>(a) * n2;
    double re = 0.0, im = 0.0;
    int idx = 0;
    for (int b = 0; b < n2; ++b) {
        const Cplx x = row[b];
        const Cplx w = tw[idx];
        const double wi = INV ? -w.im : w.im;
        re = fma(x.re, w.re, fma(-x.im, wi, re));
        im = fma(x.re, wi, fma(x.im, w.re, im));
        idx += k;
        if (idx >= n2) idx -= n2;
    }
    out[gid] = Cplx{re, im};
}

// Column transform followed by the spectral solve.
__global__ void __launch_bounds__(256)
dft_cols_solve(const Cplx* __restrict__ in, Cplx* __restrict__ e1h,
               Cplx* __restrict__ e2h, const Cplx* __restrict__ tw, int n1,
               int n2, double L1, double L2) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= static_cast<int64_t>(n1) * n2) return;
    const int k1 = static_cast<int>(gid / n2);
    const int k2 = static_cast<int>(gid - static_cast<int64_t>(k1) * n2);
    double re = 0.0, im = 0.0;
    int idx = 0;
    for (int a = 0; a < n1; ++a) {
        const Cplx x = in[static_cast<int64_t>(a) * n2 + k2];
        const Cplx w = tw[idx];
        re = fma(x.re, w.re, fma(-x.im, w.im, re));
        im = fma(x.re, w.im, fma(x.im, w.re, im));
        idx += k1;
        if (idx >= n1) idx -= n1;
    }
    const int m1 = 2 * k1 <= n1 ? k1 : k1 - n1;
    const int m2 = 2 * k2 <= n2 ? k2 : k2 - n2;
    const bool nyq = ((n1 % 2 == 0) && 2 * k1 == n1) || ((n2 % 2 == 0) && 2 * k2 == n2);
    const double kx = 2.0 * M_PI * m1 / L1;
    const double ky = 2.0 * M_PI * m2 / L2;
    const double kk = kx * kx + ky * ky;
    if (nyq || kk == 0.0) {
        e1h[gid] = Cplx{0.0, 0.0};
        e2h[gid] = Cplx{0.0, 0.0};
        return;
    }
    // -i k (re + i im) / kk = k (im - i re) / kk
    const double s1 = kx / kk, s2 = ky / kk;
    e1h[gid] = Cplx{s1 * im, -s1 * re};
    e2h[gid] = Cplx{s2 * im, -s2 * re};
}

// Inverse transform along x1 of two fields: out[a][k2] = sum_k1 in[k1][k2] conj(tw[(a k1) mod n1])
__global__ void __launch_bounds__(256)
idft_cols2(const Cplx* __restrict__ in1, const Cplx* __restrict__ in2,
           Cplx* __restrict__ out1, Cplx* __restrict__ out2,
           const Cplx* __restrict__ tw, int n1, int n2) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= static_cast<int64_t>(n1) * n2) return;
    const int a = static_cast<int>(gid / n2);
    const int k2 = static_cast<int>(gid - static_cast<int64_t>(a) * n2);
    double r1 = 0.0, i1 = 0.0, r2 = 0.0, i2 = 0.0;
    int idx = 0;
    for (int k1 = 0; k1 < n1; ++k1) {
        const Cplx w = tw[idx];
        const double wr = w.re, wi = -w.im;
        const Cplx x = in1[static_cast<int64_t>(k1) * n2 + k2];
        const Cplx y = in2[static_cast<int64_t>(k1) * n2 + k2];
        r1 = fma(x.re, wr, fma(-x.im, wi, r1));
        i1 = fma(x.re, wi, fma(x.im, wr, i1));
        r2 = fma(y.re, wr, fma(-y.im, wi, r2));
        i2 = fma(y.re, wi, fma(y.im, wr, i2));
        idx += a;
        if (idx >= n1) idx -= n1;
    }
    out1[gid] = Cplx{r1, i1};
    out2[gid] = Cplx{r2, i2};
}

// Inverse transform along x2, real part, scaled by 1/(n1 n2).
__global__ void __launch_bounds__(256)
idft_rows2(const Cplx* __restrict__ in1, const Cplx* __restrict__ in2,
           double* __restrict__ e1, double* __restrict__ e2,
           const Cplx* __restrict__ tw, int n1, int n2) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= static_cast<int64_t>(n1) * n2) return;
    const int a = static_cast<int>(gid / n2);
    const int b = static_cast<int>(gid - static_cast<int64_t>(a) * n2);
    const Cplx* r1 = in1 + static_cast<int64_t>(a) * n2;
    const Cplx* r2 = in2 + static_cast<int64_t>(a) * n2;
    double s1 = 0.0, s2 = 0.0;
    int idx = 0;
    for (int k = 0; k < n2; ++k) {
        const Cplx w = tw[idx];
        // Re[(x.re + i x.im)(w.re - i w.im)] = x.re w.re + x.im w.im
        s1 = fma(r1[k].re, w.re, fma(r1[k].im, w.im, s1));
        s2 = fma(r2[k].re, w.re, fma(r2[k].im, w.im, s2));
        idx += b;
        if (idx >= n2) idx -= n2;
    }
    const double scale = 1.0 / (static_cast<double>(n1) * n2);
    e1[gid] = s1 * scale;
    e2[gid] = s2 * scale;
}

__global__ void __launch_bounds__(256)
transfer_out(const double* __restrict__ s1, const double* __restrict__ s2,
             double* __restrict__ e1, double* __restrict__ e2, int n1, int n2,
             Transfer t) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= static_cast<int64_t>(n1) * n2) return;
    const int a = static_cast<int>(gid / n2);
    const int b = static_cast<int>(gid - static_cast<int64_t>(a) * n2);
    const int m = t.m;
    const int pa = a % m, pb = b % m;
    const int a0 = a - pa, b0 = b - pb;
    double v1 = 0.0, v2 = 0.0;
    for (int p = 0; p < m; ++p) {
        double r1 = 0.0, r2 = 0.0;
        for (int q = 0; q < m; ++q) {
            const int64_t src = static_cast<int64_t>(a0 + p) * n2 + b0 + q;
            r1 = fma(t.q[pb][q], s1[src], r1);
            r2 = fma(t.q[pb][q], s2[src], r2);
        }
        v1 = fma(t.q[pa][p], r1, v1);
        v2 = fma(t.q[pa][p], r2, v2);
    }
    e1[gid] = v1;
    e2[gid] = v2;
}

__global__ void __launch_bounds__(256)
field_energy(const double* __restrict__ e1, const double* __restrict__ e2,
             int n1, int n2, AxisGrid g1, AxisGrid g2, double* __restrict__ W) {
    __shared__ double red[4];
    const int64_t n = static_cast<int64_t>(n1) * n2;
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += 256) {
        const int64_t a = q / n2;
        const int64_t b = q - a * n2;
        const double w = g1.w[a % g1.m] * g1.h * g2.w[b % g2.m] * g2.h;
        acc = fma(w, e1[q] * e1[q] + e2[q] * e2[q], acc);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) W[0] = 0.5 * (red[0] + red[1] + red[2] + red[3]);
}

}  // namespace

static size_t poisson_ws_bytes(int64_t n1, int64_t n2) {
    return sizeof(Cplx) * (4 * static_cast<size_t>(n1) * static_cast<size_t>(n2) +
                           static_cast<size_t>(n1) + static_cast<size_t>(n2));
}

vp_status poisson_impl(int degree, int64_t n1_, int64_t n2_, double L1, double L2,
                       const double* rho, double* E1, double* E2, double* W_el,
                       void* workspace, hipStream_t st) {
    const int n1 = static_cast<int>(n1_), n2 = static_cast<int>(n2_);
    const int64_t n = n1_ * n2_;
    Cplx* c0 = static_cast<Cplx*>(workspace);
    Cplx* c1 = c0 + n;
    Cplx* c2 = c1 + n;
    Cplx* c3 = c2 + n;
    Cplx* tw1 = c3 + n;
    Cplx* tw2 = tw1 + n1;
    Transfer tin{}, tout{};
    const bool sldg = degree >= 0;
    if (sldg) {
        const TransferPair& tp = transfer_pair(degree);
        tin.m = tout.m = tp.m;
        for (int i = 0; i < tp.m; ++i)
            for (int j = 0; j < tp.m; ++j) {
                tin.q[i][j] = tp.q[i][j];
                tout.q[i][j] = tp.qinv[i][j];
            }
    }
    const unsigned grid = blocks_for(n, 256);
    transfer_in<<<grid, 256, 0, st>>>(rho, c0, tw1, tw2, n1, n2, tin, sldg ? 1 : 0);
    vp_status rc = check_launch("transfer_in");
    if (rc != VP_OK) return rc;
    dft_rows<false><<<grid, 256, 0, st>>>(c0, c1, tw2, n1, n2);
    if ((rc = check_launch("dft_rows")) != VP_OK) return rc;
    dft_cols_solve<<<grid, 256, 0, st>>>(c1, c0, c2, tw1, n1, n2, L1, L2);
    if ((rc = check_launch("dft_cols_solve")) != VP_OK) return rc;
    idft_cols2<<<grid, 256, 0, st>>>(c0, c2, c1, c3, tw1, n1, n2);
    if ((rc = check_launch("idft_cols2")) != VP_OK) return rc;
    if (sldg) {
        double* s1 = reinterpret_cast<double*>(c0);   // c0, c2 are free again
        double* s2 = reinterpret_cast<double*>(c2);
        idft_rows2<<<grid, 256, 0, st>>>(c1, c3, s1, s2, tw2, n1, n2);
        if ((rc = check_launch("idft_rows2")) != VP_OK) return rc;
        transfer_out<<<grid, 256, 0, st>>>(s1, s2, E1, E2, n1, n2, tout);
        if ((rc = check_launch("transfer_out")) != VP_OK) return rc;
    } else {
        idft_rows2<<<grid, 256, 0, st>>>(c1, c3, E1, E2, tw2, n1, n2);
        if ((rc = check_launch("idft_rows2")) != VP_OK) return rc;
    }
    if (W_el) {
        const AxisGrid g1 = axis_grid(degree, n1_, 0.0, L1);
        const AxisGrid g2 = axis_grid(degree, n2_, 0.0, L2);
        field_energy<<<1, 256, 0, st>>>(E1, E2, n1, n2, g1, g2, W_el);
        if ((rc = check_launch("field_energy")) != VP_OK) return rc;
    }
    return VP_OK;
}

}  // namespace vp

extern "C" size_t vp_poisson_workspace(int degree, int64_t n1, int64_t n2) {
    (void)degree;
    if (n1 < 1 || n2 < 1) return 0;
    return vp::poisson_ws_bytes(n1, n2);
}

extern "C" vp_status vp_poisson(int degree, int64_t n1, int64_t n2, double L1,
                                double L2, const double* rho, double* E1,
                                double* E2, double* W_el, void* workspace,
                                size_t ws_bytes, void* stream) {
    using namespace vp;
    clear_error();
    if (degree < -1 || degree > VP_MAX_DEGREE)
        return set_error(VP_ERR_UNSUPPORTED, "degree %d not in -1..%d", degree, VP_MAX_DEGREE);
    if (n1 < 1 || n2 < 1 || n1 > 65536 || n2 > 65536 || n1 * n2 >= (int64_t(1) << 31))
        return set_error(VP_ERR_ARG, "grid %lld x %lld out of range", (long long)n1,
                         (long long)n2);
    if (degree >= 0 && (n1 % (degree + 1) || n2 % (degree + 1)))
        return set_error(VP_ERR_ARG, "grid not a multiple of degree+1");
    if (!(L1 > 0.0) || !(L2 > 0.0)) return set_error(VP_ERR_ARG, "box lengths must be positive");
    if (!rho || !E1 || !E2) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if (E1 == E2 || ranges_overlap(E1, E2, sizeof(double) * n1 * n2) ||
        ranges_overlap(rho, E1, sizeof(double) * n1 * n2) ||
        ranges_overlap(rho, E2, sizeof(double) * n1 * n2))
        return set_error(VP_ERR_ALIAS, "rho, E1 and E2 must not overlap");
    if (!workspace || ws_bytes < poisson_ws_bytes(n1, n2))
        return set_error(VP_ERR_WORKSPACE, "workspace of %zu bytes needed",
                         poisson_ws_bytes(n1, n2));
    return poisson_impl(degree, n1, n2, L1, L2, rho, E1, E2, W_el, workspace,
                        static_cast<hipStream_t>(stream));
}
