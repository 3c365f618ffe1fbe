// Periodic 2D Poisson solve for the electric field (Sec. 1, Eq. (1)).
//
// div E = rho - 1, curl E = 0  =>  E = -grad phi, -Lap phi = rho - 1, so in
// Fourier space E_hat = -i k rho_hat / |k|^2 for k != 0.  The transforms are
// dense discrete Fourier transforms along one axis at a time, each line
// staged in LDS together with its twiddle table exp(-2 pi i j/n) (the x grids
// have at most a few hundred points per axis, so the O(n^3) work is small;
// what matters is few launches and no dependent global loads).
//
// SLDG grids: the nodal density of every cell is first mapped to the values
// at m = degree+1 equidistant sub-cell midpoints (Q[p][l] = L_l((p+1/2)/m)),
// which together form a uniform grid of n points; the field is computed
// there and mapped back with Q^{-1}.  Modes with m1 = 0 = m2 and modes with
// m1 = n1/2 or m2 = n2/2 (even n) are set to zero.  The electric energy
// W = 1/2 int |E|^2 uses the nodal quadrature of the grid.
//
// Three kernels (plus a one-block sum when W is asked for):
//   rows_fwd  one workgroup per x1 row: Q map along both axes, DFT along x2
//   cols      one workgroup per x2 mode: DFT along x1, spectral solve,
//             inverse DFT along x1 of both field components, Q^{-1} map
//             along x1 (real coefficients: it commutes with the transform
//             along x2 and the real part taken after it)
//   rows_inv  one workgroup per x1 row: inverse DFT along x2, Q^{-1} map
//             along x2, E (and optionally the v-sweep shifts tau E/h_v),
//             per-workgroup energy partial sums
#include <cmath>
#include <mutex>

#include "field.hpp"

namespace vp {
namespace {

constexpr int kPB = 256;

struct Cplx {
    double re, im;
};

struct Transfer {
    int m;
    double q[kMaxNodes][kMaxNodes];
};

__device__ __forceinline__ void twiddles(Cplx* tw, int n) {
    for (int j = threadIdx.x; j < n; j += kPB) {
        double s, c;
        sincospi(2.0 * static_cast<double>(j) / n, &s, &c);
        tw[j] = Cplx{c, -s};
    }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < kPB / 64; ++k) s += red[k];
    return s;
}

__global__ void __launch_bounds__(kPB)
rows_fwd(const double* __restrict__ rho, Cplx* __restrict__ c1, int n1, int n2,
         Transfer t, int use_q) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cplx* tw = reinterpret_cast<Cplx*>(smem);        // n2
    double* row = reinterpret_cast<double*>(tw + n2);  // n2
    const int a = blockIdx.x;
    twiddles(tw, n2);
    if (use_q) {
        const int m = t.m;
        const int pa = a % m, a0 = a - pa;
        for (int b = threadIdx.x; b < n2; b += kPB) {
            const int pb = b % m, b0 = b - pb;
            double v = 0.0;
            for (int p = 0; p < m; ++p) {
                double r = 0.0;
                for (int q = 0; q < m; ++q)
                    r = fma(t.q[pb][q], rho[static_cast<int64_t>(a0 + p) * n2 + b0 + q], r);
                v = fma(t.q[pa][p], r, v);
            }
            row[b] = v;
        }
    } else {
        for (int b = threadIdx.x; b < n2; b += kPB)
            row[b] = rho[static_cast<int64_t>(a) * n2 + b];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n2; k += kPB) {
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int b = 0; b < n2; ++b) {
            const Cplx w = tw[idx];
            re = fma(row[b], w.re, re);
            im = fma(row[b], w.im, im);
            idx += k;
            if (idx >= n2) idx -= n2;
        }
        c1[static_cast<int64_t>(a) * n2 + k] = Cplx{re, im};
    }
}

__global__ void __launch_bounds__(kPB)
cols(const Cplx* __restrict__ c1, Cplx* __restrict__ g1, Cplx* __restrict__ g2,
     int n1, int n2, double L1, double L2, Transfer tinv, int use_q) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cplx* tw = reinterpret_cast<Cplx*>(smem);  // n1
    Cplx* col = tw + n1;                       // n1
    Cplx* eh = col + n1;                       // 2 n1: E1 hat, E2 hat
    Cplx* ex = eh + 2 * n1;                    // 2 n1: their inverse transforms
    const int k2 = blockIdx.x;
    twiddles(tw, n1);
    for (int a = threadIdx.x; a < n1; a += kPB) col[a] = c1[static_cast<int64_t>(a) * n2 + k2];
    __syncthreads();
    const int m2 = 2 * k2 <= n2 ? k2 : k2 - n2;
    const bool nyq2 = (n2 % 2 == 0) && 2 * k2 == n2;
    const double ky = 2.0 * M_PI * m2 / L2;
    for (int k1 = threadIdx.x; k1 < n1; k1 += kPB) {
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int a = 0; a < n1; ++a) {
            const Cplx x = col[a];
            const Cplx w = tw[idx];
            re = fma(x.re, w.re, fma(-x.im, w.im, re));
            im = fma(x.re, w.im, fma(x.im, w.re, im));
            idx += k1;
            if (idx >= n1) idx -= n1;
        }
        const int m1 = 2 * k1 <= n1 ? k1 : k1 - n1;
        const bool nyq = nyq2 || ((n1 % 2 == 0) && 2 * k1 == n1);
        const double kx = 2.0 * M_PI * m1 / L1;
        const double kk = kx * kx + ky * ky;
        if (nyq || kk == 0.0) {
            eh[k1] = Cplx{0.0, 0.0};
            eh[n1 + k1] = Cplx{0.0, 0.0};
        } else {
            // -i k (re + i im) / |k|^2 = k (im - i re) / |k|^2
            const double s1 = kx / kk, s2 = ky / kk;
            eh[k1] = Cplx{s1 * im, -s1 * re};
            eh[n1 + k1] = Cplx{s2 * im, -s2 * re};
        }
    }
    __syncthreads();
    // inverse transforms: one thread per (component, x1 point)
    for (int e = threadIdx.x; e < 2 * n1; e += kPB) {
        const int d = e >= n1 ? 1 : 0;
        const int a = e - d * n1;
        const Cplx* x = eh + d * n1;
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int k1 = 0; k1 < n1; ++k1) {
            const Cplx w = tw[idx];       // conj(w) for the inverse transform
            re = fma(x[k1].re, w.re, fma(x[k1].im, w.im, re));
            im = fma(x[k1].im, w.re, fma(-x[k1].re, w.im, im));
            idx += a;
            if (idx >= n1) idx -= n1;
        }
        ex[e] = Cplx{re, im};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * n1; e += kPB) {
        const int d = e >= n1 ? 1 : 0;
        const int a = e - d * n1;
        Cplx v;
        if (use_q) {
            // Q^{-1} along x1 within the cell of a
            const int m = tinv.m;
            const int pa = a % m, a0 = a - pa;
            v = Cplx{0.0, 0.0};
            for (int p = 0; p < m; ++p) {
                const Cplx y = ex[d * n1 + a0 + p];
                v.re = fma(tinv.q[pa][p], y.re, v.re);
                v.im = fma(tinv.q[pa][p], y.im, v.im);
            }
        } else {
            v = ex[e];
        }
        (d ? g2 : g1)[static_cast<int64_t>(a) * n2 + k2] = v;
    }
}

__global__ void __launch_bounds__(kPB)
rows_inv(const Cplx* __restrict__ g1, const Cplx* __restrict__ g2,
         double* __restrict__ E1, double* __restrict__ E2, int n1, int n2,
         Transfer t, int use_q, AxisGrid gx1, AxisGrid gx2,
         double* __restrict__ wpart, double* __restrict__ sig1,
         double* __restrict__ sig2, double s1, double s2) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kPB / 64];
    Cplx* tw = reinterpret_cast<Cplx*>(smem);            // n2
    Cplx* gl = tw + n2;                                  // 2 n2: the row of g1, g2
    double* eq = reinterpret_cast<double*>(gl + 2 * n2);  // 2 n2
    const int a = blockIdx.x;
    twiddles(tw, n2);
    for (int b = threadIdx.x; b < n2; b += kPB) {
        gl[b] = g1[static_cast<int64_t>(a) * n2 + b];
        gl[n2 + b] = g2[static_cast<int64_t>(a) * n2 + b];
    }
    __syncthreads();
    // inverse DFT along x2, real part, one thread per (component, x2 point)
    const double scale = 1.0 / (static_cast<double>(n1) * n2);
    for (int e = threadIdx.x; e < 2 * n2; e += kPB) {
        const int d = e >= n2 ? 1 : 0;
        const int b = e - d * n2;
        const Cplx* row = gl + d * n2;
        double sum = 0.0;
        int idx = 0;
        for (int k = 0; k < n2; ++k) {
            // Re[(x.re + i x.im)(w.re - i w.im)] = x.re w.re + x.im w.im
            sum = fma(row[k].re, tw[idx].re, fma(row[k].im, tw[idx].im, sum));
            idx += b;
            if (idx >= n2) idx -= n2;
        }
        eq[e] = sum * scale;
    }
    __syncthreads();
    double wsum = 0.0;
    const double wa = gx1.w[a % gx1.m] * gx1.h;
    for (int b = threadIdx.x; b < n2; b += kPB) {
        double v1, v2;
        if (use_q) {
            // Q^{-1} along x2 within the cell of b
            const int m = t.m;
            const int pb = b % m, b0 = b - pb;
            v1 = 0.0;
            v2 = 0.0;
            for (int q = 0; q < m; ++q) {
                v1 = fma(t.q[pb][q], eq[b0 + q], v1);
                v2 = fma(t.q[pb][q], eq[n2 + b0 + q], v2);
            }
        } else {
            v1 = eq[b];
            v2 = eq[n2 + b];
        }
        const int64_t gi = static_cast<int64_t>(a) * n2 + b;
        E1[gi] = v1;
        E2[gi] = v2;
        if (sig1) {
            sig1[gi] = s1 * v1;
            sig2[gi] = s2 * v2;
        }
        const double w = wa * (gx2.w[b % gx2.m] * gx2.h);
        wsum = fma(w, v1 * v1 + v2 * v2, wsum);
    }
    const double tot = block_sum(wsum, red);
    if (threadIdx.x == 0) wpart[a] = tot;
}

__global__ void __launch_bounds__(kPB)
energy_sum(const double* __restrict__ wpart, int nb, double* __restrict__ W) {
    __shared__ double red[kPB / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += kPB) s += wpart[i];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) W[0] = 0.5 * tot;
}

// ---------------------------------------------------------------- adjoint ---
// rho_bar = P_1^T G_1 + P_2^T G_2.  On the uniform grid each P_d is the real
// Fourier multiplier -i k_d/|k|^2, whose transpose has multiplier
// +i k_d/|k|^2; the SLDG cell maps enter transposed: G is mapped by Q^{-T}
// before the transforms and the result by Q^T after them.  With `wgrid` set,
// G_d is first multiplied by the quadrature weights of the x grid (the
// gradient of W = 1/2 sum w |E|^2 with respect to E is w E).

__global__ void __launch_bounds__(kPB)
adj_rows_fwd(const double* __restrict__ g1, const double* __restrict__ g2,
             Cplx* __restrict__ c1, Cplx* __restrict__ c2, int n1, int n2,
             Transfer tinv, int use_q, int weighted, AxisGrid gx1, AxisGrid gx2) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cplx* tw = reinterpret_cast<Cplx*>(smem);         // n2
    double* y1 = reinterpret_cast<double*>(tw + n2);  // n2
    double* y2 = y1 + n2;                              // n2
    const int a = blockIdx.x;
    twiddles(tw, n2);
    const int m = use_q ? tinv.m : 1;
    const int pa = a % m, a0 = a - pa;
    for (int b = threadIdx.x; b < n2; b += kPB) {
        const int pb = b % m, b0 = b - pb;
        double v1 = 0.0, v2 = 0.0;
        for (int p = 0; p < m; ++p) {
            double r1 = 0.0, r2 = 0.0;
            for (int q = 0; q < m; ++q) {
                const int64_t src = static_cast<int64_t>(a0 + p) * n2 + b0 + q;
                double x1 = g1[src], x2 = g2[src];
                if (weighted) {
                    const double w = gx1.w[(a0 + p) % gx1.m] * gx1.h * gx2.w[(b0 + q) % gx2.m] * gx2.h;
                    x1 *= w;
                    x2 *= w;
                }
                const double qq = use_q ? tinv.q[q][pb] : 1.0;
                r1 = fma(qq, x1, r1);
                r2 = fma(qq, x2, r2);
            }
            const double qp = use_q ? tinv.q[p][pa] : 1.0;
            v1 = fma(qp, r1, v1);
            v2 = fma(qp, r2, v2);
        }
        y1[b] = v1;
        y2[b] = v2;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n2; k += kPB) {
        double re1 = 0.0, im1 = 0.0, re2 = 0.0, im2 = 0.0;
        int idx = 0;
        for (int b = 0; b < n2; ++b) {
            const Cplx w = tw[idx];
            re1 = fma(y1[b], w.re, re1);
            im1 = fma(y1[b], w.im, im1);
            re2 = fma(y2[b], w.re, re2);
            im2 = fma(y2[b], w.im, im2);
            idx += k;
            if (idx >= n2) idx -= n2;
        }
        c1[static_cast<int64_t>(a) * n2 + k] = Cplx{re1, im1};
        c2[static_cast<int64_t>(a) * n2 + k] = Cplx{re2, im2};
    }
}

__global__ void __launch_bounds__(kPB)
adj_cols(const Cplx* __restrict__ c1, const Cplx* __restrict__ c2, Cplx* __restrict__ h,
         int n1, int n2, double L1, double L2) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cplx* tw = reinterpret_cast<Cplx*>(smem);  // n1
    Cplx* x1 = tw + n1;                        // n1
    Cplx* x2 = x1 + n1;                        // n1
    Cplx* rh = x2 + n1;                        // n1
    const int k2 = blockIdx.x;
    twiddles(tw, n1);
    for (int a = threadIdx.x; a < n1; a += kPB) {
        x1[a] = c1[static_cast<int64_t>(a) * n2 + k2];
        x2[a] = c2[static_cast<int64_t>(a) * n2 + k2];
    }
    __syncthreads();
    const int m2 = 2 * k2 <= n2 ? k2 : k2 - n2;
    const bool nyq2 = (n2 % 2 == 0) && 2 * k2 == n2;
    const double ky = 2.0 * M_PI * m2 / L2;
    for (int k1 = threadIdx.x; k1 < n1; k1 += kPB) {
        double r1 = 0.0, i1 = 0.0, r2 = 0.0, i2 = 0.0;
        int idx = 0;
        for (int a = 0; a < n1; ++a) {
            const Cplx w = tw[idx];
            r1 = fma(x1[a].re, w.re, fma(-x1[a].im, w.im, r1));
            i1 = fma(x1[a].re, w.im, fma(x1[a].im, w.re, i1));
            r2 = fma(x2[a].re, w.re, fma(-x2[a].im, w.im, r2));
            i2 = fma(x2[a].re, w.im, fma(x2[a].im, w.re, i2));
            idx += k1;
            if (idx >= n1) idx -= n1;
        }
        const int m1 = 2 * k1 <= n1 ? k1 : k1 - n1;
        const bool nyq = nyq2 || ((n1 % 2 == 0) && 2 * k1 == n1);
        const double kx = 2.0 * M_PI * m1 / L1;
        const double kk = kx * kx + ky * ky;
        if (nyq || kk == 0.0) {
            rh[k1] = Cplx{0.0, 0.0};
        } else {
            // i (kx Y1 + ky Y2) / |k|^2
            const double sr = (kx * r1 + ky * r2) / kk, si = (kx * i1 + ky * i2) / kk;
            rh[k1] = Cplx{-si, sr};
        }
    }
    __syncthreads();
    for (int a = threadIdx.x; a < n1; a += kPB) {
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int k1 = 0; k1 < n1; ++k1) {
            const Cplx w = tw[idx];       // conj(w) for the inverse transform
            const Cplx x = rh[k1];
            re = fma(x.re, w.re, fma(x.im, w.im, re));
            im = fma(x.im, w.re, fma(-x.re, w.im, im));
            idx += a;
            if (idx >= n1) idx -= n1;
        }
        h[static_cast<int64_t>(a) * n2 + k2] = Cplx{re, im};
    }
}

// Inverse DFT along x2 of m rows of g into eq[m][n2] (real part, scaled).
__device__ __forceinline__ void inverse_rows(const Cplx* __restrict__ g, int a0,
                                             int m, int n1, int n2, const Cplx* tw,
                                             Cplx* gl, double* eq) {
    for (int e = threadIdx.x; e < m * n2; e += kPB)
        gl[e] = g[static_cast<int64_t>(a0) * n2 + e];
    __syncthreads();
    const double scale = 1.0 / (static_cast<double>(n1) * n2);
    for (int e = threadIdx.x; e < m * n2; e += kPB) {
        const int p = e / n2;
        const int b = e - p * n2;
        const Cplx* row = gl + p * n2;
        double s = 0.0;
        int idx = 0;
        for (int k = 0; k < n2; ++k) {
            // Re[(x.re + i x.im)(w.re - i w.im)] = x.re w.re + x.im w.im
            s = fma(row[k].re, tw[idx].re, fma(row[k].im, tw[idx].im, s));
            idx += b;
            if (idx >= n2) idx -= n2;
        }
        eq[e] = s * scale;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kPB)
adj_rows_inv(const Cplx* __restrict__ h, double* __restrict__ rho_bar, int n1, int n2,
             Transfer t, int use_q) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int m = use_q ? t.m : 1;
    Cplx* tw = reinterpret_cast<Cplx*>(smem);   // n2
    Cplx* gl = tw + n2;                         // m * n2
    double* r = reinterpret_cast<double*>(gl + m * n2);   // m * n2
    const int a0 = blockIdx.x * m;
    twiddles(tw, n2);
    inverse_rows(h, a0, m, n1, n2, tw, gl, r);
    for (int e = threadIdx.x; e < m * n2; e += kPB) {
        const int p = e / n2;
        const int b = e - p * n2;
        double v;
        if (use_q) {
            const int pb = b % m, b0 = b - pb;
            v = 0.0;
            for (int pp = 0; pp < m; ++pp) {
                double acc = 0.0;
                for (int q = 0; q < m; ++q) acc = fma(t.q[q][pb], r[pp * n2 + b0 + q], acc);
                v = fma(t.q[pp][p], acc, v);
            }
        } else {
            v = r[e];
        }
        rho_bar[static_cast<int64_t>(a0 + p) * n2 + b] = v;
    }
}

}  // namespace

static size_t poisson_ws_bytes(int64_t n1, int64_t n2) {
    return sizeof(Cplx) * 3 * static_cast<size_t>(n1) * static_cast<size_t>(n2) +
           sizeof(double) * static_cast<size_t>(n1) + 256;
}

static size_t rows_inv_lds(int n2) {
    return sizeof(Cplx) * 3 * static_cast<size_t>(n2) + 2 * sizeof(double) * static_cast<size_t>(n2);
}

static size_t cols_lds(int n1) { return sizeof(Cplx) * 6 * static_cast<size_t>(n1); }

static size_t adj_rows_inv_lds(int m, int n2) {
    return sizeof(Cplx) * (static_cast<size_t>(n2) + static_cast<size_t>(m) * n2) +
           sizeof(double) * static_cast<size_t>(m) * n2;
}

vp_status poisson_impl_shift(int degree, int64_t n1_, int64_t n2_, double L1, double L2,
                             const double* rho, double* E1, double* E2, double* W_el,
                             void* workspace, double* sig1, double* sig2, double s1,
                             double s2, hipStream_t st) {
    const int n1 = static_cast<int>(n1_), n2 = static_cast<int>(n2_);
    const int64_t n = n1_ * n2_;
    Cplx* c1 = static_cast<Cplx*>(workspace);
    Cplx* g1 = c1 + n;
    Cplx* g2 = g1 + n;
    double* wpart = reinterpret_cast<double*>(g2 + n);
    Transfer t{};
    const bool sldg = degree >= 0;
    Transfer tinv{};
    if (sldg) {
        const TransferPair& tp = transfer_pair(degree);
        t.m = tinv.m = tp.m;
        for (int i = 0; i < tp.m; ++i)
            for (int j = 0; j < tp.m; ++j) {
                t.q[i][j] = tp.q[i][j];
                tinv.q[i][j] = tp.qinv[i][j];
            }
    }
    const size_t lds_inv = rows_inv_lds(n2);
    if (lds_inv > 64 * 1024 || cols_lds(n1) > 64 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "x grid %d x %d too large for the Poisson kernels",
                         n1, n2);
    const AxisGrid gx1 = axis_grid(degree, n1_, 0.0, L1);
    const AxisGrid gx2 = axis_grid(degree, n2_, 0.0, L2);
    rows_fwd<<<n1, kPB, n2 * (sizeof(Cplx) + sizeof(double)), st>>>(rho, c1, n1, n2, t,
                                                                     sldg ? 1 : 0);
    vp_status rc = check_launch("rows_fwd");
    if (rc != VP_OK) return rc;
    cols<<<n2, kPB, cols_lds(n1), st>>>(c1, g1, g2, n1, n2, L1, L2, tinv, sldg ? 1 : 0);
    if ((rc = check_launch("cols")) != VP_OK) return rc;
    const int nb = n1;
    rows_inv<<<nb, kPB, lds_inv, st>>>(g1, g2, E1, E2, n1, n2, tinv, sldg ? 1 : 0, gx1,
                                       gx2, wpart, sig1, sig2, s1, s2);
    if ((rc = check_launch("rows_inv")) != VP_OK) return rc;
    if (W_el) {
        energy_sum<<<1, kPB, 0, st>>>(wpart, nb, W_el);
        if ((rc = check_launch("energy_sum")) != VP_OK) return rc;
    }
    return VP_OK;
}

vp_status poisson_impl(int degree, int64_t n1, int64_t n2, double L1, double L2,
                       const double* rho, double* E1, double* E2, double* W_el,
                       void* workspace, hipStream_t st) {
    return poisson_impl_shift(degree, n1, n2, L1, L2, rho, E1, E2, W_el, workspace,
                              nullptr, nullptr, 0.0, 0.0, st);
}

vp_status poisson_adjoint_impl(int degree, int64_t n1_, int64_t n2_, double L1, double L2,
                               const double* g1, const double* g2, double* rho_bar,
                               void* workspace, bool weighted, hipStream_t st) {
    const int n1 = static_cast<int>(n1_), n2 = static_cast<int>(n2_);
    const int64_t n = n1_ * n2_;
    Cplx* c1 = static_cast<Cplx*>(workspace);
    Cplx* c2 = c1 + n;
    Cplx* h = c2 + n;
    Transfer t{}, tinv{};
    const bool sldg = degree >= 0;
    int m = 1;
    if (sldg) {
        const TransferPair& tp = transfer_pair(degree);
        m = tp.m;
        t.m = tinv.m = tp.m;
        for (int i = 0; i < tp.m; ++i)
            for (int j = 0; j < tp.m; ++j) {
                t.q[i][j] = tp.q[i][j];
                tinv.q[i][j] = tp.qinv[i][j];
            }
    }
    if (adj_rows_inv_lds(m, n2) > 64 * 1024 || static_cast<size_t>(4 * n1) * sizeof(Cplx) > 64 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "x grid %d x %d too large for the Poisson kernels",
                         n1, n2);
    const AxisGrid gx1 = axis_grid(degree, n1_, 0.0, L1);
    const AxisGrid gx2 = axis_grid(degree, n2_, 0.0, L2);
    adj_rows_fwd<<<n1, kPB, n2 * (sizeof(Cplx) + 2 * sizeof(double)), st>>>(
        g1, g2, c1, c2, n1, n2, tinv, sldg ? 1 : 0, weighted ? 1 : 0, gx1, gx2);
    vp_status rc = check_launch("adj_rows_fwd");
    if (rc != VP_OK) return rc;
    adj_cols<<<n2, kPB, 4 * n1 * sizeof(Cplx), st>>>(c1, c2, h, n1, n2, L1, L2);
    if ((rc = check_launch("adj_cols")) != VP_OK) return rc;
    adj_rows_inv<<<n1 / m, kPB, adj_rows_inv_lds(m, n2), st>>>(
        h, rho_bar, n1, n2, t, sldg ? 1 : 0);
    return check_launch("adj_rows_inv");
}

}  // namespace vp

// ------------------------------------------------ allocation-free variant ---
// The workspace of vp_poisson_noalloc: a device array of the library,
// sized for the largest grid that entry point accepts.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): its address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.
namespace {
constexpr size_t kNoAllocBytes =
    sizeof(vp::Cplx) * 3 * static_cast<size_t>(VP_POISSON_NOALLOC_MAX_POINTS) +
    sizeof(double) * 4096 + 256;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// The address of `scratch` on the current device (looked up on the first
// call on that device).
vp_status scratch_on_current_device(void** out) {
    using namespace vp;
    int dev = -1;
    VP_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(VP_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(VP_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VP_OK;
}

// Host checks shared by vp_poisson and vp_poisson_noalloc.
vp_status check_poisson_args(int degree, int64_t n1, int64_t n2, double L1, double L2,
                             const double* rho, const double* E1, const double* E2) {
    using namespace vp;
    if (degree < -1 || degree > VP_MAX_DEGREE)
        return set_error(VP_ERR_UNSUPPORTED, "degree %d not in -1..%d", degree, VP_MAX_DEGREE);
    if (n1 < 1 || n2 < 1 || n1 > 4096 || n2 > 4096)
        return set_error(VP_ERR_ARG, "grid %lld x %lld out of range", (long long)n1,
                         (long long)n2);
    if (degree >= 0 && (n1 % (degree + 1) || n2 % (degree + 1)))
        return set_error(VP_ERR_ARG, "grid not a multiple of degree+1");
    if (!(L1 > 0.0) || !(L2 > 0.0)) return set_error(VP_ERR_ARG, "box lengths must be positive");
    if (!rho || !E1 || !E2) return set_error(VP_ERR_ARG, "NULL pointer argument");
    const size_t nb = sizeof(double) * static_cast<size_t>(n1 * n2);
    if (ranges_overlap(E1, E2, nb) || ranges_overlap(rho, E1, nb) || ranges_overlap(rho, E2, nb))
        return set_error(VP_ERR_ALIAS, "rho, E1 and E2 must not overlap");
    return VP_OK;
}
}  // namespace

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
    vp_status rc = check_poisson_args(degree, n1, n2, L1, L2, rho, E1, E2);
    if (rc != VP_OK) return rc;
    if (!workspace || ws_bytes < poisson_ws_bytes(n1, n2))
        return set_error(VP_ERR_WORKSPACE, "workspace of %zu bytes needed",
                         poisson_ws_bytes(n1, n2));
    return poisson_impl(degree, n1, n2, L1, L2, rho, E1, E2, W_el, workspace,
                        static_cast<hipStream_t>(stream));
}

extern "C" vp_status vp_poisson_adjoint(int degree, int64_t n1, int64_t n2, double L1,
                                        double L2, const double* G1, const double* G2,
                                        double* rho_bar, void* workspace, size_t ws_bytes,
                                        void* stream) {
    using namespace vp;
    clear_error();
    if (degree < -1 || degree > VP_MAX_DEGREE)
        return set_error(VP_ERR_UNSUPPORTED, "degree %d not in -1..%d", degree, VP_MAX_DEGREE);
    if (n1 < 1 || n2 < 1 || n1 > 4096 || n2 > 4096)
        return set_error(VP_ERR_ARG, "grid %lld x %lld out of range", (long long)n1,
                         (long long)n2);
    if (degree >= 0 && (n1 % (degree + 1) || n2 % (degree + 1)))
        return set_error(VP_ERR_ARG, "grid not a multiple of degree+1");
    if (!(L1 > 0.0) || !(L2 > 0.0)) return set_error(VP_ERR_ARG, "box lengths must be positive");
    if (!G1 || !G2 || !rho_bar) return set_error(VP_ERR_ARG, "NULL pointer argument");
    const size_t nb = sizeof(double) * static_cast<size_t>(n1 * n2);
    if (ranges_overlap(rho_bar, G1, nb) || ranges_overlap(rho_bar, G2, nb))
        return set_error(VP_ERR_ALIAS, "rho_bar must not overlap G1 or G2");
    if (!workspace || ws_bytes < poisson_ws_bytes(n1, n2))
        return set_error(VP_ERR_WORKSPACE, "workspace of %zu bytes needed",
                         poisson_ws_bytes(n1, n2));
    return poisson_adjoint_impl(degree, n1, n2, L1, L2, G1, G2, rho_bar, workspace, false,
                                static_cast<hipStream_t>(stream));
}

extern "C" vp_status vp_poisson_noalloc(int degree, int64_t n1, int64_t n2, double L1,
                                        double L2, const double* rho, double* E1,
                                        double* E2, double* W_el, void* stream) {
    using namespace vp;
    clear_error();
    vp_status rc = check_poisson_args(degree, n1, n2, L1, L2, rho, E1, E2);
    if (rc != VP_OK) return rc;
    if (n1 * n2 > VP_POISSON_NOALLOC_MAX_POINTS || poisson_ws_bytes(n1, n2) > kNoAllocBytes)
        return set_error(VP_ERR_WORKSPACE,
                         "grid %lld x %lld: the allocation-free Poisson solve holds at most "
                         "%d points",
                         (long long)n1, (long long)n2, VP_POISSON_NOALLOC_MAX_POINTS);
    void* ws = nullptr;
    if ((rc = scratch_on_current_device(&ws)) != VP_OK) return rc;
    return poisson_impl(degree, n1, n2, L1, L2, rho, E1, E2, W_el, ws,
                        static_cast<hipStream_t>(stream));
}
