// SLDG translate-and-project sweep (Sec. 2, last part; Sec. 3, Eq. (5)).
//
// A line of n_c cells x m = degree+1 Gauss-Legendre dofs is shifted by
// sigma cells: with s = floor(sigma) mod n_c and alpha = sigma - floor(sigma),
// output cell i = A(alpha) u_{i-s-1} + B(alpha) u_{i-s}.  The per-line
// operator (s, A, B) is built in FP64 inside the kernel from the quadrature
// definition
//   A_jl = (alpha/w_j) sum_q w_q L_l(alpha xi_q + 1 - alpha) L_j(alpha xi_q)
//   B_jl = ((1-alpha)/w_j) sum_q w_q L_l((1-alpha) xi_q) L_j(alpha + (1-alpha) xi_q)
// (the (m)-point Gauss rule is exact for these degree-2l integrands) and
// rounded to the storage type T; the sweep itself is 2m FMAs per dof in T.
//
// Two kernels, both HBM-bound (each dof read once and written once):
//  * sldg_col  -- axes whose lines are strided (x1, x2, v1).  One thread per
//    line streams the cells of its line in memory order; adjacent threads own
//    adjacent lines, so every load and store of a wavefront is contiguous
//    along the fastest axis.  Each input cell is loaded exactly once: the
//    last cell is loaded first (it is the left neighbour of cell 0) and
//    reused at the end.
//  * sldg_row  -- the contiguous axis (v2).  A workgroup builds the
//    operators of R whole lines once, into LDS; every thread then produces
//    one output cell from its two input cells, which neighbouring lanes
//    share through the L1 cache.
//
// The transposed sweep (for reverse-mode differentiation) is the same
// gather with the transposed operators and the opposite offset:
// u_bar_c = B^T lam_{c+s} + A^T lam_{c+s+1}; both kernels take it as the
// template flag ADJ (A_eff = B^T on the first cell of the pair, B_eff = A^T on
// the second).  The shift derivative d <lam, sweep(u)> / d sigma of a line
// uses dA/dalpha and dB/dalpha from Leibniz' rule on the defining integrals:
//   A'_jl = (1/w_j)[L_l(1) L_j(alpha) - sum_q alpha w_q L_l'(alpha xi_q + 1 - alpha) L_j(alpha xi_q)]
//   B'_jl = (1/w_j)[-L_l(0) L_j(alpha) - sum_q (1-alpha) w_q L_l'((1-alpha) xi_q) L_j(alpha + (1-alpha) xi_q)]
#include "field.hpp"

namespace vp {
namespace {

constexpr int kBlock = 256;
constexpr int kU = 8;  // loads issued back to back per thread
constexpr int kSegCells = 8;  // output cells per thread of the segmented column sweep

template <int M>
__device__ __forceinline__ void lagrange_all(const NodeBasis& b, double t,
                                             double L[M]) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double p = 1.0;
#pragma unroll
        for (int k = 0; k < M; ++k)
            if (k != j) p *= (t - b.xi[k]) * b.rd[j][k];
        L[j] = p;
    }
}

// Builds the line operator.  alpha == 0 gives A = 0, B = I exactly, so a
// whole-cell shift is an exact permutation of the cells; a shift that
// split_shift rejects gives NaN entries.  (Branch-free selects keep A and B
// in registers.)
template <int M, typename T>
__device__ __forceinline__ void sldg_operator(const NodeBasis& b, double sigma,
                                              int nc, int& s, T A[M][M],
                                              T B[M][M]) {
    double alpha;
    const bool ok = split_shift(sigma, nc, s, alpha);
    const bool exact = alpha == 0.0;
    const double beta = 1.0 - alpha;
    double a[M][M], c[M][M];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int l = 0; l < M; ++l) a[j][l] = c[j][l] = 0.0;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        double lo[M], li[M], ro[M], ri[M];
        const double ta = alpha * b.xi[q];
        lagrange_all<M>(b, ta, lo);
        lagrange_all<M>(b, ta + beta, li);
        lagrange_all<M>(b, alpha + beta * b.xi[q], ro);
        lagrange_all<M>(b, beta * b.xi[q], ri);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double wl = b.w[q] * lo[j];
            const double wr = b.w[q] * ro[j];
#pragma unroll
            for (int l = 0; l < M; ++l) {
                a[j][l] = fma(wl, li[l], a[j][l]);
                c[j][l] = fma(wr, ri[l], c[j][l]);
            }
        }
    }
    const double nan = __builtin_nan("");
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double sa = alpha * b.inv_w[j];
        const double sb = beta * b.inv_w[j];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            const double av = exact ? 0.0 : a[j][l] * sa;
            const double bv = exact ? (j == l ? 1.0 : 0.0) : c[j][l] * sb;
            A[j][l] = T(ok ? av : nan);
            B[j][l] = T(ok ? bv : nan);
        }
    }
}

template <int M>
__device__ __forceinline__ void lagrange_deriv_all(const NodeBasis& b, double t,
                                                   double D[M]) {
#pragma unroll
    for (int l = 0; l < M; ++l) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            if (q == l) continue;
            double p = b.rd[l][q];
#pragma unroll
            for (int k = 0; k < M; ++k)
                if (k != l && k != q) p *= (t - b.xi[k]) * b.rd[l][k];
            acc += p;
        }
        D[l] = acc;
    }
}

// dA/dalpha and dB/dalpha of the line (NaN for a rejected shift).
template <int M, typename T>
__device__ __forceinline__ void sldg_operator_deriv(const NodeBasis& b, double sigma,
                                                    int nc, int& s, T dA[M][M],
                                                    T dB[M][M]) {
    double alpha;
    const bool ok = split_shift_floor(sigma, nc, s, alpha);
    const double beta = 1.0 - alpha;
    double la[M], l1[M], l0[M];
    lagrange_all<M>(b, alpha, la);
    lagrange_all<M>(b, 1.0, l1);
    lagrange_all<M>(b, 0.0, l0);
    double a[M][M], c[M][M];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int l = 0; l < M; ++l) {
            a[j][l] = la[j] * l1[l];
            c[j][l] = -la[j] * l0[l];
        }
#pragma unroll
    for (int q = 0; q < M; ++q) {
        double lo[M], di[M], ro[M], dr[M];
        const double ta = alpha * b.xi[q];
        lagrange_all<M>(b, ta, lo);
        lagrange_deriv_all<M>(b, ta + beta, di);
        lagrange_all<M>(b, alpha + beta * b.xi[q], ro);
        lagrange_deriv_all<M>(b, beta * b.xi[q], dr);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double wl = alpha * b.w[q] * lo[j];
            const double wr = beta * b.w[q] * ro[j];
#pragma unroll
            for (int l = 0; l < M; ++l) {
                a[j][l] = fma(-wl, di[l], a[j][l]);
                c[j][l] = fma(-wr, dr[l], c[j][l]);
            }
        }
    }
    const double nan = __builtin_nan("");
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int l = 0; l < M; ++l) {
            dA[j][l] = T(ok ? a[j][l] * b.inv_w[j] : nan);
            dB[j][l] = T(ok ? c[j][l] * b.inv_w[j] : nan);
        }
}

// (A, B) -> (B^T, A^T): the pair operators of the transposed sweep.
template <int M, typename T>
__device__ __forceinline__ void transpose_pair(T A[M][M], T B[M][M]) {
    T At[M][M], Bt[M][M];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int l = 0; l < M; ++l) {
            At[j][l] = A[l][j];
            Bt[j][l] = B[l][j];
        }
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int l = 0; l < M; ++l) {
            A[j][l] = Bt[j][l];
            B[j][l] = At[j][l];
        }
}

// One output cell: out_j = sum_l A_jl left_l + B_jl right_l, stored at
// out[j * stride].
template <int M, typename T>
__device__ __forceinline__ void sldg_cell(const T A[M][M], const T B[M][M],
                                          const T left[M], const T right[M],
                                          T* __restrict__ out, int64_t stride) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < M; ++l) acc = fma(A[j][l], left[l], acc);
#pragma unroll
        for (int l = 0; l < M; ++l) acc = fma(B[j][l], right[l], acc);
        put_out(&out[j * stride], acc);
    }
}

template <int M, typename T, int AXIS, bool ADJ>
__global__ void __launch_bounds__(kBlock)
sldg_col(const T* __restrict__ fin, T* __restrict__ fout,
         const double* __restrict__ shift, ShiftMap sm, int64_t outer, int nc,
         int64_t inner, NodeBasis basis) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (gid >= outer * inner) return;
    const int64_t o = gid / inner;
    const int64_t k = gid - o * inner;

    int s;
    T A[M][M], B[M][M];
    sldg_operator<M, T>(basis, shift[shift_offset(sm, o, k)], nc, s, A, B);
    if (ADJ) transpose_pair<M, T>(A, B);

    const int64_t cs = static_cast<int64_t>(M) * inner;  // cell stride
    const T* __restrict__ src = fin + o * nc * cs + k;
    T* __restrict__ dst = fout + o * nc * cs + k;

    T last[M], prev[M];
#pragma unroll
    for (int l = 0; l < M; ++l) {
        last[l] = src[(nc - 1) * cs + l * inner];
        prev[l] = last[l];
    }
    // output cell fed by input cells (c-1, c): c+s, or c-1-s for the transpose
    int i = ADJ ? nc - 1 - s : s;
    // chunks of CU cells: all their loads are issued before the first use
    constexpr int CU = (M <= 3 ? 4 : 2) * (sizeof(T) == 4 ? 2 : 1);
    int c = 0;
    for (; c + CU <= nc - 1; c += CU) {
        T cur[CU][M];
#pragma unroll
        for (int u = 0; u < CU; ++u)
#pragma unroll
            for (int l = 0; l < M; ++l) cur[u][l] = src[(c + u) * cs + l * inner];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            sldg_cell<M, T>(A, B, prev, cur[u], dst + i * cs, inner);
#pragma unroll
            for (int l = 0; l < M; ++l) prev[l] = cur[u][l];
            if (++i == nc) i = 0;
        }
    }
    for (; c < nc; ++c) {
        T cur[M];
        if (c < nc - 1) {
#pragma unroll
            for (int l = 0; l < M; ++l) cur[l] = src[c * cs + l * inner];
        } else {
#pragma unroll
            for (int l = 0; l < M; ++l) cur[l] = last[l];
        }
        sldg_cell<M, T>(A, B, prev, cur, dst + i * cs, inner);
#pragma unroll
        for (int l = 0; l < M; ++l) prev[l] = cur[l];
        if (++i == nc) i = 0;
    }
}

// Strided lines by row segments.  A thread forms the C output cells
// [q C, q C + C) of one line (fewer at the end of the line): output cell i
// reads input cells i + d and i + d + 1 (d = -s - 1, or s for the transpose),
// so the segment loads its C + 1 input cells at once, one of them the
// previous segment's last (a re-read that the caches serve).  Blocks run in
// memory order: when a workgroup's 256 lines share the outer index (inner a
// multiple of 256) block b is (outer o, segment q, column block kb) with kb
// fastest, so that the workgroups in flight cover a narrow band of rows
// instead of every row of their columns at once; otherwise b is (line
// block, segment) with the segment fastest.  Short-lived workgroups whose
// accesses advance through memory in block order stream like a plain copy,
// where one thread per whole line (sldg_col) keeps every row of the array
// in flight at the same time.
//
// With J > 1 (band blocks only) a thread takes J adjacent columns that share
// the shift (a shift that does not depend on the fastest axis), loaded as
// one vector per row: workgroups of 256 J columns and C = 8 / J cells, the
// same outputs per operator build over a shorter band of rows.
template <int M, typename T, bool ADJ, int C, bool BAND, int J>
__global__ void __launch_bounds__(kBlock)
sldg_seg(const T* __restrict__ fin, T* __restrict__ fout,
         const double* __restrict__ shift, ShiftMap sm, int64_t outer, int nc,
         int64_t inner, int nseg, NodeBasis basis) {
    static_assert(J == 1 || BAND, "stacked columns need band blocks");
    int64_t o, k;
    int q;
    if (BAND) {
        const int64_t nkb = inner / (J * kBlock);
        const int64_t b = blockIdx.x;
        const int64_t kb = b % nkb;
        const int64_t rest = b / nkb;
        q = static_cast<int>(rest % nseg);
        o = rest / nseg;
        k = (kb * kBlock + threadIdx.x) * J;
    } else {
        q = static_cast<int>(blockIdx.x % nseg);
        const int64_t line = static_cast<int64_t>(blockIdx.x / nseg) * kBlock + threadIdx.x;
        if (line >= outer * inner) return;
        o = line / inner;
        k = line - o * inner;
    }
    int s;
    T A[M][M], B[M][M];
    sldg_operator<M, T>(basis, shift[shift_offset(sm, o, k)], nc, s, A, B);
    if (ADJ) transpose_pair<M, T>(A, B);

    const int64_t cs = static_cast<int64_t>(M) * inner;  // cell stride
    const T* __restrict__ src = fin + o * nc * cs + k;
    T* __restrict__ dst = fout + o * nc * cs + k;
    const int i0 = q * C;
    // first input cell i0 + d, reduced into [0, nc)
    int c = ADJ ? i0 + s : i0 - s - 1;
    c += c < 0 ? nc : 0;
    c -= c >= nc ? nc : 0;
    if constexpr (J == 1) {
        T u[C + 1][M];
#pragma unroll
        for (int j = 0; j <= C; ++j) {
#pragma unroll
            for (int l = 0; l < M; ++l) u[j][l] = src[c * cs + l * inner];
            c = c + 1 == nc ? 0 : c + 1;
        }
#pragma unroll
        for (int j = 0; j < C; ++j)
            if (i0 + j < nc) sldg_cell<M, T>(A, B, u[j], u[j + 1], dst + (i0 + j) * cs, inner);
    } else {
        using VJ = T __attribute__((ext_vector_type(J)));
        VJ u[C + 1][M];
#pragma unroll
        for (int j = 0; j <= C; ++j) {
#pragma unroll
            for (int l = 0; l < M; ++l)
                u[j][l] = *reinterpret_cast<const VJ*>(src + c * cs + l * inner);
            c = c + 1 == nc ? 0 : c + 1;
        }
#pragma unroll
        for (int j = 0; j < C; ++j) {
            if (i0 + j < nc) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    VJ acc;
#pragma unroll
                    for (int e = 0; e < J; ++e) {
                        T a = T(0);
#pragma unroll
                        for (int l = 0; l < M; ++l) a = fma(A[m][l], u[j][l][e], a);
#pragma unroll
                        for (int l = 0; l < M; ++l) a = fma(B[m][l], u[j + 1][l][e], a);
                        acc[e] = a;
                    }
                    __builtin_nontemporal_store(acc, reinterpret_cast<VJ*>(dst + (i0 + j) * cs + m * inner));
                }
            }
        }
    }
}

// The x2 sweep with its output density formed on the way (forward only), by
// whole lines: the form for the shapes the row-segment form below does not
// take (degree above 3, x2 rows over 16 MB, x1 planes of 4 GB or more),
// launched with J = 1.  The x2 shift depends on v2 only, so a thread may
// take J velocity columns that share it: the same v2 and J consecutive v1
// nodes (columns k0 + j N4), with one operator for all of them.  Output cells are produced in order,
// every lane of a wavefront on the same cell: output i is fed by input
// cells (l0 + i, l0 + i + 1) mod n_c with l0 = n_c - 1 - s, which lanes load
// from their own (shift-dependent) rows.  A lane first adds W3 W4 f_out
// over its J columns; the wavefront then sums those per-cell values four at
// a time (`wave_sum4_rows`: a batch of CU cells gives CU (l+1) values, a
// multiple of four), and the four wavefronts' sums meet in LDS, where each
// workgroup writes the partial density of its 256 J velocity columns
// (N3 N4 / J must be a multiple of the workgroup size, so that a workgroup
// stays within one x1 index).  Every input cell is loaded once.  The x1
// plane is read and written as a buffer (it must hold less than 4 GB): the
// loads of a cell share one per-lane byte offset, the stores the lane's
// column offset, with the rest of each address uniform.  (A row-segmented form, as for the plain sweeps, ran slower here:
// its reductions come after all of its loads, with nothing left to overlap.)
template <int M, typename T, int J, bool MOM>
__global__ void __launch_bounds__(kBlock)
sldg_col_rho(const T* __restrict__ fin, T* __restrict__ fout,
             const double* __restrict__ shift, ShiftMap sm, int nc, int64_t inner,
             NodeBasis basis, RhoFuse rf) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = nc * M;
    double* rp = reinterpret_cast<double*>(smem);   // [kBlock / 64][N]
    const int bpo = static_cast<int>(inner / (J * kBlock));   // workgroups per x1 index
    const int o = static_cast<int>(blockIdx.x) / bpo;
    const int t = (static_cast<int>(blockIdx.x) - o * bpo) * kBlock + static_cast<int>(threadIdx.x);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int v1b = t / rf.n4;                      // J v1 nodes v1b J .. v1b J + J - 1
    const int v2 = t - v1b * rf.n4;
    const int64_t k0 = static_cast<int64_t>(v1b) * J * rf.n4 + v2;
    const int64_t js = rf.n4;                       // column step between them
    const double w4v = rf.g4.w[v2 % rf.g4.m] * rf.g4.h;
    double wk[J];
#pragma unroll
    for (int j = 0; j < J; ++j) wk[j] = rf.g3.w[(v1b * J + j) % rf.g3.m] * rf.g3.h * w4v;

    int s;
    T A[M][M], B[M][M];
    sldg_operator<M, T>(basis, shift[shift_offset(sm, o, k0)], nc, s, A, B);
    const int64_t cs = static_cast<int64_t>(M) * inner;
    // the x1 plane o of input and output as buffers; per lane one byte offset
    const uint32_t pb = static_cast<uint32_t>(nc * cs * sizeof(T));
    const __amdgpu_buffer_rsrc_t rin = buffer_of(fin + static_cast<int64_t>(o) * nc * cs, pb);
    const __amdgpu_buffer_rsrc_t rout = buffer_of(fout + static_cast<int64_t>(o) * nc * cs, pb);
    const uint32_t kb = static_cast<uint32_t>(k0 * sizeof(T));     // lane's byte offset
    const uint32_t cb = static_cast<uint32_t>(cs * sizeof(T));     // cell stride, bytes
    // input (cell c, dof l, column j); output (cell i, dof m, column j)
    auto ld = [&](int c, int l, int j) -> T {
        return buffer_load<T>(rin, static_cast<uint32_t>(c) * cb + kb,
                              static_cast<uint32_t>((l * inner + j * js) * sizeof(T)));
    };
    auto st = [&](int i, int m, int j, T v) {
        buffer_store_nt<T>(v, rout, kb, static_cast<uint32_t>((i * cs + m * inner + j * js) * sizeof(T)));
    };

    const int l0 = nc - 1 - s;
    T prev[J][M];
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int l = 0; l < M; ++l) prev[j][l] = ld(l0, l, j);
    int rc = l0 + 1 == nc ? 0 : l0 + 1;   // next input cell to load
    // moments: sums over the thread's columns of W2 W3 f, W2 W3 |f|,
    // W2 W3 f^2 and W2 W3 |v|^2 f (W4 and W1 are applied at the end)
    double s_m = 0.0, s_a = 0.0, s_q = 0.0, s_k = 0.0;
    double w2[M];
#pragma unroll
    for (int l = 0; l < M; ++l) w2[l] = MOM ? rf.g2.w[l] * rf.g2.h : 0.0;
    double w3[J], vv[J];
    if (MOM) {
        const double a2 = rf.g4.lo + (static_cast<double>(v2 / rf.g4.m) + rf.g4.xi[v2 % rf.g4.m]) * rf.g4.h;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int v1 = v1b * J + j;
            const double a1 = rf.g3.lo + (static_cast<double>(v1 / rf.g3.m) + rf.g3.xi[v1 % rf.g3.m]) * rf.g3.h;
            w3[j] = rf.g3.w[v1 % rf.g3.m] * rf.g3.h;
            vv[j] = a1 * a1 + a2 * a2;
        }
    }
    // output cell i from the thread's values, its weighted sums into vals
    auto cell = [&](int i, const T (&cur)[J][M], double* vals) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < M; ++l) acc = fma(A[m][l], prev[j][l], acc);
#pragma unroll
                for (int l = 0; l < M; ++l) acc = fma(B[m][l], cur[j][l], acc);
                st(i, m, j, acc);
                const double ov = static_cast<double>(acc);
                vals[m] = fma(wk[j], ov, vals[m]);
                if (MOM) {
                    const double wv = w2[m] * w3[j];
                    s_m = fma(wv, ov, s_m);
                    s_a = fma(wv, fabs(ov), s_a);
                    s_q = fma(wv * ov, ov, s_q);
                    s_k = fma(wv * vv[j], ov, s_k);
                }
            }
#pragma unroll
            for (int l = 0; l < M; ++l) prev[j][l] = cur[j][l];
        }
    };
    // cells whose loads are in flight together: about 12 loads, and whole
    // groups of four values to sum (CU (l+1) a multiple of 4)
    constexpr int CU4 = M % 4 == 0 ? 1 : (M % 2 == 0 ? 2 : 4);
    constexpr int CUW = 12 / (J * M);
    constexpr int CU = CUW > CU4 ? (CUW / CU4) * CU4 : CU4;
    constexpr int NV = CU * M;
    static_assert(NV % 4 == 0, "whole groups of four values");
    int i = 0;
    for (; i + CU <= nc - 1; i += CU) {
        T cur[CU][J][M];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            int c = rc + u;
            c -= c >= nc ? nc : 0;
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int l = 0; l < M; ++l) cur[u][j][l] = ld(c, l, j);
        }
        double vals[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vals[q] = 0.0;
#pragma unroll
        for (int u = 0; u < CU; ++u) cell(i + u, cur[u], vals + u * M);
#pragma unroll
        for (int g = 0; g < NV / 4; ++g) {
            const double r = wave_sum4_rows(vals[4 * g], vals[4 * g + 1], vals[4 * g + 2], vals[4 * g + 3]);
            if ((lane & 15) == 0) rp[wave * N + i * M + 4 * g + (lane >> 4)] = r;
        }
        rc += CU;
        rc -= rc >= nc ? nc : 0;
    }
    // the last cells one at a time; the right input of cell n_c - 1 is the
    // first input cell again
    constexpr int NT = (M + 3) / 4 * 4;
    for (; i < nc; ++i) {
        T cur[J][M];
        const int c = i < nc - 1 ? rc : l0;
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int l = 0; l < M; ++l) cur[j][l] = ld(c, l, j);
        double vals[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) vals[q] = 0.0;
        cell(i, cur, vals);
#pragma unroll
        for (int g = 0; g < NT / 4; ++g) {
            const double r = wave_sum4_rows(vals[4 * g], vals[4 * g + 1], vals[4 * g + 2], vals[4 * g + 3]);
            const int q = 4 * g + (lane >> 4);
            if ((lane & 15) == 0 && q < M) rp[wave * N + i * M + q] = r;
        }
        rc = rc + 1 == nc ? 0 : rc + 1;
    }
    if (MOM) {
        // W = W1 W2 W3 W4 (W2 W3 already in the sums)
        const double w1 = rf.g1.w[o % rf.g1.m] * rf.g1.h;
        const double f0 = w1 * w4v;
        double q[4] = {f0 * s_m, f0 * s_a, f0 * s_q, f0 * s_k};
        double* red = rp + (kBlock / 64) * N;   // [4][kBlock / 64]
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) q[t4] += __shfl_xor(q[t4], off, 64);
            if (lane == 0) red[t4 * (kBlock / 64) + wave] = q[t4];
        }
    }
    __syncthreads();
    for (int jj = threadIdx.x; jj < N; jj += kBlock) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) acc += rp[w * N + jj];
        rf.part[static_cast<int64_t>(blockIdx.x) * N + jj] = acc;
    }
    if (MOM && threadIdx.x < 4) {
        const double* red = rp + (kBlock / 64) * N;
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) acc += red[threadIdx.x * (kBlock / 64) + w];
        rf.mom_part[static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x] = acc;
    }
}

// The x2 sweep with its output density formed on the way, by row segments
// as `sldg_seg` (band blocks: x1 index o, segment q, block kb of 256 threads,
// kb fastest).  A thread takes J velocity columns that share the x2 shift
// (one v2, J consecutive v1 nodes: columns k0 + j N4) under one operator,
// forms the C output cells of its segment in each, and adds W3 W4 f_out over
// its columns into one value per output node; the wavefront sums those
// C (l+1) values four at a time (`wave_sum4_rows`), the four wavefronts'
// sums meet in LDS, and the workgroup writes its slice [q C (l+1),
// (q C + C)(l+1)) of the partial density of its 256 J columns, the layout
// of one group per 256 J columns.  The x1 plane is read and written as a
// buffer (less than 4 GB).
template <int M, typename T, int C, int J, bool MOM>
__global__ void __launch_bounds__(kBlock)
sldg_seg_rho(const T* __restrict__ fin, T* __restrict__ fout,
             const double* __restrict__ shift, ShiftMap sm, int nc, int64_t inner, int nseg,
             NodeBasis basis, RhoFuse rf) {
    constexpr int NV = C * M;
    static_assert(NV % 4 == 0, "whole groups of four values");
    __shared__ double red[kBlock / 64][NV + 4];
    const int nkb = static_cast<int>(inner / (J * kBlock));
    const int b = static_cast<int>(blockIdx.x);
    const int kb = b % nkb;
    const int rest = b / nkb;
    const int q = rest % nseg;
    const int o = rest / nseg;
    const int t = kb * kBlock + static_cast<int>(threadIdx.x);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int v1b = t / rf.n4;                      // v1 nodes v1b J .. v1b J + J - 1
    const int v2 = t - v1b * rf.n4;
    const int k0 = v1b * J * rf.n4 + v2;            // first column
    const double w4 = rf.g4.w[v2 % rf.g4.m] * rf.g4.h;
    double w3[J];
#pragma unroll
    for (int j = 0; j < J; ++j) w3[j] = rf.g3.w[(v1b * J + j) % rf.g3.m] * rf.g3.h;

    int s;
    T A[M][M], B[M][M];
    sldg_operator<M, T>(basis, shift[shift_offset(sm, o, k0)], nc, s, A, B);
    const int64_t cs = static_cast<int64_t>(M) * inner;
    const uint32_t pb = static_cast<uint32_t>(nc * cs * sizeof(T));
    const __amdgpu_buffer_rsrc_t rin = buffer_of(fin + static_cast<int64_t>(o) * nc * cs, pb);
    const __amdgpu_buffer_rsrc_t rout = buffer_of(fout + static_cast<int64_t>(o) * nc * cs, pb);
    const uint32_t kbyte = static_cast<uint32_t>(k0 * sizeof(T));
    const uint32_t cb = static_cast<uint32_t>(cs * sizeof(T));
    const uint32_t ib = static_cast<uint32_t>(inner * sizeof(T));
    const uint32_t jb = static_cast<uint32_t>(rf.n4 * sizeof(T));

    const int i0 = q * C;
    int c = i0 - s - 1;   // first input cell, reduced into [0, nc)
    c += c < 0 ? nc : 0;
    c -= c >= nc ? nc : 0;
    T u[C + 1][J][M];
#pragma unroll
    for (int i = 0; i <= C; ++i) {
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int l = 0; l < M; ++l)
                u[i][j][l] = buffer_load<T>(rin, static_cast<uint32_t>(c) * cb + kbyte, l * ib + j * jb);
        c = c + 1 == nc ? 0 : c + 1;
    }
    double vals[NV];
    // moments of column j: sums of W2 f, W2 |f|, W2 f^2 over its nodes
    double x_m[J], x_a[J], x_q[J];
#pragma unroll
    for (int j = 0; j < J; ++j) x_m[j] = x_a[j] = x_q[j] = 0.0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const bool live = i0 + i < nc;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double val = 0.0;
#pragma unroll
            for (int j = 0; j < J; ++j) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < M; ++l) acc = fma(A[m][l], u[i][j][l], acc);
#pragma unroll
                for (int l = 0; l < M; ++l) acc = fma(B[m][l], u[i + 1][j][l], acc);
                if (live)
                    buffer_store_nt<T>(acc, rout, kbyte,
                                       static_cast<uint32_t>((i0 + i) * cs * sizeof(T)) + m * ib + j * jb);
                const double ov = live ? static_cast<double>(acc) : 0.0;
                val = fma(w3[j], ov, val);
                if (MOM) {
                    const double w2 = rf.g2.w[m] * rf.g2.h;
                    x_m[j] = fma(w2, ov, x_m[j]);
                    x_a[j] = fma(w2, fabs(ov), x_a[j]);
                    x_q[j] = fma(w2 * ov, ov, x_q[j]);
                }
            }
            const int v = i * M + m;
            vals[v] = w4 * val;
            if (v % 4 == 3) {   // a group of four values is complete: sum it
                const double r = wave_sum4_rows(vals[v - 3], vals[v - 2], vals[v - 1], vals[v]);
                if ((lane & 15) == 0) red[wave][v - 3 + (lane >> 4)] = r;
            }
        }
    }
    if (MOM) {
        // W = W1 W2 W3 W4: W2 in the column sums, W3 per column, W1 W4 here
        const double a2 = rf.g4.lo + (static_cast<double>(v2 / rf.g4.m) + rf.g4.xi[v2 % rf.g4.m]) * rf.g4.h;
        double s_m = 0.0, s_a = 0.0, s_q = 0.0, s_k = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int v1 = v1b * J + j;
            const double a1 = rf.g3.lo + (static_cast<double>(v1 / rf.g3.m) + rf.g3.xi[v1 % rf.g3.m]) * rf.g3.h;
            s_m = fma(w3[j], x_m[j], s_m);
            s_a = fma(w3[j], x_a[j], s_a);
            s_q = fma(w3[j], x_q[j], s_q);
            s_k = fma(w3[j] * (a1 * a1 + a2 * a2), x_m[j], s_k);
        }
        const double f0 = rf.g1.w[o % rf.g1.m] * rf.g1.h * w4;
        const double r = wave_sum4_rows(f0 * s_m, f0 * s_a, f0 * s_q, f0 * s_k);
        if ((lane & 15) == 0) red[wave][NV + (lane >> 4)] = r;
    }
    __syncthreads();
    const int nv = min(C, nc - i0) * M;
    if (static_cast<int>(threadIdx.x) < nv) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) acc += red[w][threadIdx.x];
        rf.part[(static_cast<int64_t>(o) * nkb + kb) * (nc * M) + i0 * M + threadIdx.x] = acc;
    }
    if (MOM && threadIdx.x < 4) {
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) acc += red[w][NV + threadIdx.x];
        rf.mom_part[static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x] = acc;
    }
}

template <int M, typename T, bool ADJ>
__global__ void __launch_bounds__(kBlock)
sldg_row(const T* __restrict__ fin, T* __restrict__ fout,
         const double* __restrict__ shift, ShiftMap sm, int64_t nrows, int nc,
         int R, NodeBasis basis) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* stage = reinterpret_cast<T*>(smem);                 // kBlock * M
    T* ops = stage + kBlock * M;                           // R * 2 M^2
    int* sh = reinterpret_cast<int*>(ops + R * 2 * M * M);  // R

    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
    const int nr = static_cast<int>(min(static_cast<int64_t>(R), nrows - row0));
    const int lane = threadIdx.x & 63;
    T* wstage = stage + (threadIdx.x >> 6) * 64 * M;       // this wavefront's

    for (int r = threadIdx.x; r < nr; r += kBlock) {
        int s;
        T A[M][M], B[M][M];
        sldg_operator<M, T>(basis, shift[shift_offset(sm, row0 + r, 0)], nc, s,
                            A, B);
        if (ADJ) transpose_pair<M, T>(A, B);
        T* op = ops + r * 2 * M * M;
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int l = 0; l < M; ++l) {
                op[j * M + l] = A[j][l];
                op[M * M + j * M + l] = B[j][l];
            }
        sh[r] = s;
    }
    __syncthreads();

    // one thread per output cell; its two input cells come straight from
    // global memory (neighbouring lanes share them in the L1 cache), kB
    // cells' loads in flight together, clamped indices instead of branches
    const int N = nc * M;
    const int ncell = nr * nc;
    const T* __restrict__ u0 = fin + row0 * N;
    T* __restrict__ o0 = fout + row0 * N;
    constexpr int kB = M <= 3 ? 4 : 2;
    // (the same trip count for every thread: the staging below needs whole
    // wavefronts)
    for (int base = 0; base < ncell; base += kB * kBlock) {
        const int q0 = base + static_cast<int>(threadIdx.x);
        T ul[kB][M], ur[kB][M];
        int qq[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int q = min(q0 + b * kBlock, ncell - 1);
            const int r = q / nc;
            const int i = q - r * nc;
            const int s = sh[r];
            // forward: cells (i-s-1, i-s); transpose: cells (i+s, i+s+1)
            int left = ADJ ? i + s : i - s - 1;
            left += left < 0 ? nc : 0;
            left -= left >= nc ? nc : 0;
            int right = left + 1;
            right -= right >= nc ? nc : 0;
            qq[b] = q;
#pragma unroll
            for (int l = 0; l < M; ++l) {
                ul[b][l] = u0[r * N + left * M + l];
                ur[b][l] = u0[r * N + right * M + l];
            }
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int q = qq[b];
            const T* op = ops + (q / nc) * 2 * M * M;
            T out[M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < M; ++l) acc = fma(op[j * M + l], ul[b][l], acc);
#pragma unroll
                for (int l = 0; l < M; ++l) acc = fma(op[M * M + j * M + l], ur[b][l], acc);
                out[j] = acc;
            }
            // The wavefront's 64 cells are consecutive, so are their 64 M
            // outputs: staged through the wavefront's LDS slice they leave
            // as M whole-line stores instead of M stores of lane-strided
            // runs.  The lanes exchange values through the slice, so each
            // wave barrier sits between a release and an acquire fence of
            // wavefront scope: the writes of every lane are visible to the
            // reads of the others (and the next round's writes wait for
            // this round's reads).  On LDS these fences cost nothing.
#pragma unroll
            for (int j = 0; j < M; ++j) wstage[lane * M + j] = out[j];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int64_t e0 = static_cast<int64_t>(q0 + b * kBlock - lane) * M;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int64_t e = e0 + j * 64 + lane;
                if (e < static_cast<int64_t>(ncell) * M) put_out(&o0[e], wstage[j * 64 + lane]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Adjacent columns per thread of the segmented sweep (J) when the shift
// does not depend on the fastest axis: 16-byte loads, and a band of 8 / J
// cells; 1 when the grid does not divide into workgroups of 256 J columns.
int seg_columns(vp_dtype dt, int axis, const int64_t dims[4], bool shift_shared_v2) {
    if (axis > 2 || !shift_shared_v2) return 1;
    int64_t inner = 1;
    for (int d = axis + 1; d < 4; ++d) inner *= dims[d];
    int J = dt == VP_F64 ? 2 : 4;
    while (J > 1 && (dims[3] % J || (inner / J) % kBlock)) J /= 2;
    return J;
}

template <int M, typename T, bool ADJ>
vp_status launch_sldg(int axis, const int64_t dims[4], const void* fin,
                      void* fout, const double* shift, const ShiftMap& sm,
                      hipStream_t st, int jcols) {
    const NodeBasis& b = node_basis(M - 1);
    int64_t outer = 1, inner = 1;
    for (int d = 0; d < axis; ++d) outer *= dims[d];
    for (int d = axis + 1; d < 4; ++d) inner *= dims[d];
    const int nc = static_cast<int>(dims[axis] / M);
    const T* in = static_cast<const T*>(fin);
    T* out = static_cast<T*>(fout);
    // Band blocks (lines of whole workgroups of columns) pay off while one
    // row of the array is short: at 96^4 (7 MB rows along x1) they beat one
    // thread per whole line, at 192^4 and 288^4 (28-95 MB rows) they lose
    // to it; lines with fewer than 256 columns always run by segments.
    const bool band_ok = static_cast<size_t>(inner) * sizeof(T) <= (size_t(16) << 20);
    if (!band_ok) jcols = 1;
    if (axis < 3 && jcols > 1) {
        // (M <= 3: a vector of J columns per row of the segment)
        const int C = kSegCells / jcols;
        const int nseg = (nc + C - 1) / C;
        const int64_t nblk = outer * nseg * (inner / (jcols * kBlock));
        if constexpr (M <= 3) {
            if (nblk < (int64_t(1) << 31)) {
                const unsigned g = static_cast<unsigned>(nblk);
                if (jcols == 2)
                    sldg_seg<M, T, ADJ, kSegCells / 2, true, 2><<<g, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, nseg, b);
                else
                    sldg_seg<M, T, ADJ, kSegCells / 4, true, 4><<<g, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, nseg, b);
                return check_launch("sldg_seg");
            }
        }
    }
    if (axis < 3) {
        constexpr int C = kSegCells;
        const int nseg = (nc + C - 1) / C;
        const bool band = inner % kBlock == 0;
        const int64_t nblk = band ? outer * nseg * (inner / kBlock)
                                  : static_cast<int64_t>(blocks_for(outer * inner, kBlock)) * nseg;
        if ((band_ok || !band) && nblk < (int64_t(1) << 31)) {
            const unsigned g = static_cast<unsigned>(nblk);
            if (band)
                sldg_seg<M, T, ADJ, C, true, 1><<<g, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, nseg, b);
            else
                sldg_seg<M, T, ADJ, C, false, 1><<<g, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, nseg, b);
            return check_launch("sldg_seg");
        }
        // one thread per whole line
        const unsigned grid = blocks_for(outer * inner, kBlock);
        switch (axis) {
            case 0:
                sldg_col<M, T, 0, ADJ><<<grid, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, b);
                break;
            case 1:
                sldg_col<M, T, 1, ADJ><<<grid, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, b);
                break;
            default:
                sldg_col<M, T, 2, ADJ><<<grid, kBlock, 0, st>>>(in, out, shift, sm, outer, nc, inner, b);
                break;
        }
        return check_launch("sldg_col");
    }
    // rows per workgroup: two rounds of the cell loop (4 or 2 cells per
    // thread per round), so that the operator build is spread over enough
    // bytes; the R operators in LDS
    const size_t per_row = static_cast<size_t>(2 * M * M) * sizeof(T) + sizeof(int);
    int R = (M <= 3 ? 4 : 2) * 2 * kBlock / nc;
    if (R < 1) R = 1;
    if (R > kBlock) R = kBlock;
    const size_t lds = static_cast<size_t>(kBlock) * M * sizeof(T) + R * per_row;
    const unsigned grid = blocks_for(outer, R);
    sldg_row<M, T, ADJ><<<grid, kBlock, lds, st>>>(in, out, shift, sm, outer, nc, R, b);
    return check_launch("sldg_row");
}

template <typename T, bool ADJ>
vp_status dispatch_degree(int degree, int axis, const int64_t dims[4],
                          const void* fin, void* fout, const double* shift,
                          const ShiftMap& sm, hipStream_t st, int jcols) {
    switch (degree) {
        case 0: return launch_sldg<1, T, ADJ>(axis, dims, fin, fout, shift, sm, st, jcols);
        case 1: return launch_sldg<2, T, ADJ>(axis, dims, fin, fout, shift, sm, st, jcols);
        case 2: return launch_sldg<3, T, ADJ>(axis, dims, fin, fout, shift, sm, st, jcols);
        case 3: return launch_sldg<4, T, ADJ>(axis, dims, fin, fout, shift, sm, st, jcols);
        case 4: return launch_sldg<5, T, ADJ>(axis, dims, fin, fout, shift, sm, st, jcols);
        case 5: return launch_sldg<6, T, ADJ>(axis, dims, fin, fout, shift, sm, st, jcols);
        default: return set_error(VP_ERR_UNSUPPORTED, "degree %d", degree);
    }
}

template <int M, typename T, int J>
vp_status launch_sldg_rho_j(const int64_t dims[4], const void* fin, void* fout,
                            const double* shift, const ShiftMap& sm, const RhoFuse& rf,
                            hipStream_t st) {
    const NodeBasis& b = node_basis(M - 1);
    const int64_t outer = dims[0];
    const int64_t inner = dims[2] * dims[3];
    const int nc = static_cast<int>(dims[1] / M);
    const size_t lds = sizeof(double) * (kBlock / 64) * (static_cast<size_t>(dims[1]) + 4);
    if (dims[2] % J || (inner / J) % kBlock || lds > 48 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "fused x2 sweep needs whole workgroups of columns");
    if (static_cast<uint64_t>(dims[1] * inner) * sizeof(T) >= (uint64_t(1) << 32))
        return set_error(VP_ERR_UNSUPPORTED, "fused x2 sweep: an x1 plane of 4 GB or more");
    const unsigned grid = blocks_for(outer * inner / J, kBlock);
    if (rf.mom_part)
        sldg_col_rho<M, T, J, true><<<grid, kBlock, lds, st>>>(
            static_cast<const T*>(fin), static_cast<T*>(fout), shift, sm, nc, inner, b, rf);
    else
        sldg_col_rho<M, T, J, false><<<grid, kBlock, lds, st>>>(
            static_cast<const T*>(fin), static_cast<T*>(fout), shift, sm, nc, inner, b, rf);
    return check_launch("sldg_col_rho");
}

// Shape of the fused row-segment sweep: cells per segment (0: whole lines)
// and velocity columns per thread.
constexpr int kRhoSegJ32 = 2;   // FP32: columns per thread
constexpr int kRhoSegC32 = 8;   // FP32: cells per segment
// (degree 3 by whole lines: its row-segment form held 233-237 registers, two
// wavefronts a SIMD, and took 1010 against 820 us at 128^4)
constexpr int rho_seg_cells(int M, bool f32) {
    return M > 3 ? 0 : (f32 ? kRhoSegC32 : kSegCells);
}
constexpr int rho_seg_cols(int M, bool f32) { return f32 && M <= 3 ? kRhoSegJ32 : 1; }

// The fused x2 sweep runs by row segments where its band blocks apply:
// N3 N4 / J a multiple of 256, x2 rows of at most 16 MB, an x1 plane under
// 4 GB and degree <= 2; otherwise one thread per whole line (`sldg_col_rho`).
int rho_seg_stack(vp_dtype dt, int degree, const int64_t dims[4]) {
    const int64_t inner = dims[2] * dims[3];
    const size_t es = dtype_size(dt);
    const bool f32 = dt == VP_F32;
    const int C = rho_seg_cells(degree + 1, f32);
    if (C == 0) return 0;
    if (static_cast<size_t>(inner) * es > (size_t(16) << 20)) return 0;
    if (static_cast<uint64_t>(dims[1] * inner) * es >= (uint64_t(1) << 32)) return 0;
    int J = rho_seg_cols(degree + 1, f32);
    while (J > 1 && (dims[2] % J || (inner / J) % kBlock)) J /= 2;
    if ((inner / J) % kBlock) return 0;
    const int nc = static_cast<int>(dims[1] / (degree + 1));
    const int64_t nblk = dims[0] * ((nc + C - 1) / C) * (inner / (J * kBlock));
    return nblk < (int64_t(1) << 31) ? J : 0;
}

template <int M, typename T, int J>
vp_status launch_sldg_rho_seg(const int64_t dims[4], const void* fin, void* fout,
                              const double* shift, const ShiftMap& sm, const RhoFuse& rf,
                              hipStream_t st) {
    constexpr int C = rho_seg_cells(M, sizeof(T) == 4);
    if constexpr (C > 0) {
        const NodeBasis& b = node_basis(M - 1);
        const int64_t inner = dims[2] * dims[3];
        const int nc = static_cast<int>(dims[1] / M);
        const int nseg = (nc + C - 1) / C;
        const unsigned grid = static_cast<unsigned>(dims[0] * nseg * (inner / (J * kBlock)));
        if (rf.mom_part)
            sldg_seg_rho<M, T, C, J, true><<<grid, kBlock, 0, st>>>(
                static_cast<const T*>(fin), static_cast<T*>(fout), shift, sm, nc, inner, nseg, b, rf);
        else
            sldg_seg_rho<M, T, C, J, false><<<grid, kBlock, 0, st>>>(
                static_cast<const T*>(fin), static_cast<T*>(fout), shift, sm, nc, inner, nseg, b, rf);
        return check_launch("sldg_seg_rho");
    }
    return set_error(VP_ERR_UNSUPPORTED, "fused x2 sweep by segments: degree <= 2");
}

template <int M, typename T>
vp_status launch_sldg_rho(const int64_t dims[4], const void* fin, void* fout,
                          const double* shift, const ShiftMap& sm, const RhoFuse& rf,
                          hipStream_t st) {
    const vp_dtype dt = sizeof(T) == 8 ? VP_F64 : VP_F32;
    const int js = rho_seg_stack(dt, M - 1, dims);
    if (js == 1) return launch_sldg_rho_seg<M, T, 1>(dims, fin, fout, shift, sm, rf, st);
    if constexpr (rho_seg_cols(M, sizeof(T) == 4) >= 2)
        if (js == 2) return launch_sldg_rho_seg<M, T, 2>(dims, fin, fout, shift, sm, rf, st);
    if constexpr (rho_seg_cols(M, sizeof(T) == 4) >= 4)
        if (js == 4) return launch_sldg_rho_seg<M, T, 4>(dims, fin, fout, shift, sm, rf, st);
    if (sldg_rho_stack(dt, M - 1, dims) == 1)
        return launch_sldg_rho_j<M, T, 1>(dims, fin, fout, shift, sm, rf, st);
    return set_error(VP_ERR_UNSUPPORTED, "fused x2 sweep needs whole workgroups of columns");
}

template <typename T>
vp_status dispatch_rho(int degree, const int64_t dims[4], const void* fin, void* fout,
                       const double* shift, const ShiftMap& sm, const RhoFuse& rf,
                       hipStream_t st) {
    switch (degree) {
        case 0: return launch_sldg_rho<1, T>(dims, fin, fout, shift, sm, rf, st);
        case 1: return launch_sldg_rho<2, T>(dims, fin, fout, shift, sm, rf, st);
        case 2: return launch_sldg_rho<3, T>(dims, fin, fout, shift, sm, rf, st);
        case 3: return launch_sldg_rho<4, T>(dims, fin, fout, shift, sm, rf, st);
        case 4: return launch_sldg_rho<5, T>(dims, fin, fout, shift, sm, rf, st);
        case 5: return launch_sldg_rho<6, T>(dims, fin, fout, shift, sm, rf, st);
        default: return set_error(VP_ERR_UNSUPPORTED, "degree %d", degree);
    }
}

// ------------------------------------------------------ shift derivative ---

// Strided lines: one thread per line streams u in memory order and the
// adjoint lam of the output cells it forms (c+s), accumulating
// sum_j lam_j (A' u_{c-1} + B' u_c)_j in FP64.
template <int M, typename T, int AXIS>
__global__ void __launch_bounds__(kBlock)
sldg_dshift_col(const T* __restrict__ fin, const T* __restrict__ lam,
                const double* __restrict__ shift, ShiftMap sm, int64_t outer,
                int nc, int64_t inner, NodeBasis basis, double* __restrict__ g) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (gid >= outer * inner) return;
    const int64_t o = gid / inner;
    const int64_t k = gid - o * inner;
    int s;
    T dA[M][M], dB[M][M];
    sldg_operator_deriv<M, T>(basis, shift[shift_offset(sm, o, k)], nc, s, dA, dB);
    const int64_t cs = static_cast<int64_t>(M) * inner;
    const T* __restrict__ src = fin + o * nc * cs + k;
    const T* __restrict__ ls = lam + o * nc * cs + k;
    T prev[M];
#pragma unroll
    for (int l = 0; l < M; ++l) prev[l] = src[(nc - 1) * cs + l * inner];
    double acc = 0.0;
    int i = s;
    for (int c = 0; c < nc; ++c) {
        T cur[M], lv[M];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            cur[l] = src[c * cs + l * inner];
            lv[l] = ls[i * cs + l * inner];
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            T d = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) d = fma(dA[j][l], prev[l], d);
#pragma unroll
            for (int l = 0; l < M; ++l) d = fma(dB[j][l], cur[l], d);
            acc = fma(static_cast<double>(lv[j]), static_cast<double>(d), acc);
        }
#pragma unroll
        for (int l = 0; l < M; ++l) prev[l] = cur[l];
        if (++i == nc) i = 0;
    }
    g[gid] = acc;
}

// Contiguous lines: R lines per workgroup.  The lines' derivative operators
// are built once per line into LDS; then one thread per output cell forms
// lam_i . (A' u_{i-s-1} + B' u_{i-s}) with loads that neighbouring lanes
// share, and each line's cell terms are summed from LDS.
template <int M, typename T>
__global__ void __launch_bounds__(kBlock)
sldg_dshift_row(const T* __restrict__ fin, const T* __restrict__ lam,
                const double* __restrict__ shift, ShiftMap sm, int64_t nrows,
                int nc, int R, NodeBasis basis, double* __restrict__ g) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* part = reinterpret_cast<double*>(smem);           // R * nc cell terms
    T* ops = reinterpret_cast<T*>(part + R * nc);              // R * 2 M^2
    int* sh = reinterpret_cast<int*>(ops + R * 2 * M * M);     // R
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
    const int nr = static_cast<int>(min(static_cast<int64_t>(R), nrows - row0));
    for (int r = threadIdx.x; r < nr; r += kBlock) {
        int s;
        T dA[M][M], dB[M][M];
        sldg_operator_deriv<M, T>(basis, shift[shift_offset(sm, row0 + r, 0)], nc, s, dA, dB);
        T* op = ops + r * 2 * M * M;
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int l = 0; l < M; ++l) {
                op[j * M + l] = dA[j][l];
                op[M * M + j * M + l] = dB[j][l];
            }
        sh[r] = s;
    }
    __syncthreads();
    const int N = nc * M;
    const int ncell = nr * nc;
    const T* __restrict__ u0 = fin + row0 * N;
    const T* __restrict__ l0 = lam + row0 * N;
    constexpr int kB = 4;  // cells per thread whose loads are in flight together
    for (int q0 = threadIdx.x; q0 < ncell; q0 += kB * kBlock) {
        T ul[kB][M], ur[kB][M], lv[kB][M];
        int qq[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int q = min(q0 + b * kBlock, ncell - 1);
            const int r = q / nc;
            const int i = q - r * nc;
            int left = i - sh[r] - 1;
            left += left < 0 ? nc : 0;
            int right = left + 1;
            right -= right >= nc ? nc : 0;
            qq[b] = q;
#pragma unroll
            for (int l = 0; l < M; ++l) {
                ul[b][l] = u0[r * N + left * M + l];
                ur[b][l] = u0[r * N + right * M + l];
                lv[b][l] = l0[q * M + l];
            }
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int q = qq[b];
            const T* op = ops + (q / nc) * 2 * M * M;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                T d = T(0);
#pragma unroll
                for (int l = 0; l < M; ++l) d = fma(op[j * M + l], ul[b][l], d);
#pragma unroll
                for (int l = 0; l < M; ++l) d = fma(op[M * M + j * M + l], ur[b][l], d);
                acc = fma(static_cast<double>(lv[b][j]), static_cast<double>(d), acc);
            }
            if (q0 + b * kBlock < ncell) part[q] = acc;
        }
    }
    __syncthreads();
    // per-line sums; the start is skewed by the line index so that the
    // threads of a wavefront read different LDS banks
    for (int r = threadIdx.x; r < nr; r += kBlock) {
        double acc = 0.0;
        int c = r % nc;
        for (int k = 0; k < nc; ++k) {
            acc += part[r * nc + c];
            c = c + 1 == nc ? 0 : c + 1;
        }
        g[row0 + r] = acc;
    }
}

template <int M, typename T>
vp_status launch_dshift(int axis, const int64_t dims[4], const void* fin, const void* lam,
                        const double* shift, const ShiftMap& sm, double* g, hipStream_t st) {
    const NodeBasis& b = node_basis(M - 1);
    int64_t outer = 1, inner = 1;
    for (int d = 0; d < axis; ++d) outer *= dims[d];
    for (int d = axis + 1; d < 4; ++d) inner *= dims[d];
    const int nc = static_cast<int>(dims[axis] / M);
    const T* in = static_cast<const T*>(fin);
    const T* l = static_cast<const T*>(lam);
    if (axis < 3) {
        const unsigned grid = blocks_for(outer * inner, kBlock);
        switch (axis) {
            case 0: sldg_dshift_col<M, T, 0><<<grid, kBlock, 0, st>>>(in, l, shift, sm, outer, nc, inner, b, g); break;
            case 1: sldg_dshift_col<M, T, 1><<<grid, kBlock, 0, st>>>(in, l, shift, sm, outer, nc, inner, b, g); break;
            default: sldg_dshift_col<M, T, 2><<<grid, kBlock, 0, st>>>(in, l, shift, sm, outer, nc, inner, b, g); break;
        }
        return check_launch("sldg_dshift_col");
    }
    // lines per workgroup: about 2048 cells, at most 48 KiB of LDS
    const size_t per_row = static_cast<size_t>(nc) * sizeof(double) +
                           static_cast<size_t>(2 * M * M) * sizeof(T) + sizeof(int);
    int R = 2048 / nc;
    if (R < 1) R = 1;
    if (R > kBlock) R = kBlock;
    while (R > 1 && R * per_row > 48 * 1024) R /= 2;
    const size_t lds = R * per_row;
    if (lds > 64 * 1024)
        return set_error(VP_ERR_UNSUPPORTED, "sldg dshift: line of %d cells too long", nc);
    sldg_dshift_row<M, T><<<blocks_for(outer, R), kBlock, lds, st>>>(in, l, shift, sm, outer,
                                                                      nc, R, b, g);
    return check_launch("sldg_dshift_row");
}

template <typename T>
vp_status dispatch_dshift(int degree, int axis, const int64_t dims[4], const void* fin,
                          const void* lam, const double* shift, const ShiftMap& sm,
                          double* g, hipStream_t st) {
    switch (degree) {
        case 0: return launch_dshift<1, T>(axis, dims, fin, lam, shift, sm, g, st);
        case 1: return launch_dshift<2, T>(axis, dims, fin, lam, shift, sm, g, st);
        case 2: return launch_dshift<3, T>(axis, dims, fin, lam, shift, sm, g, st);
        case 3: return launch_dshift<4, T>(axis, dims, fin, lam, shift, sm, g, st);
        case 4: return launch_dshift<5, T>(axis, dims, fin, lam, shift, sm, g, st);
        case 5: return launch_dshift<6, T>(axis, dims, fin, lam, shift, sm, g, st);
        default: return set_error(VP_ERR_UNSUPPORTED, "degree %d", degree);
    }
}

}  // namespace

vp_status sldg_advect_impl(int axis, int degree, vp_dtype dt,
                           const int64_t dims[4], const void* f_in, void* f_out,
                           const double* shift, const int64_t shift_stride[4],
                           hipStream_t st, bool adjoint) {
    const ShiftMap sm = make_shift_map(axis, dims, shift_stride);
    int jc = degree <= 2 ? seg_columns(dt, axis, dims, shift_stride[3] == 0) : 1;
    // (vector loads and stores of J values: both arrays aligned to them)
    const uintptr_t al = static_cast<uintptr_t>(jc) * dtype_size(dt);
    if ((reinterpret_cast<uintptr_t>(f_in) | reinterpret_cast<uintptr_t>(f_out)) % al) jc = 1;
    if (dt == VP_F64)
        return adjoint
                   ? dispatch_degree<double, true>(degree, axis, dims, f_in, f_out, shift, sm, st, jc)
                   : dispatch_degree<double, false>(degree, axis, dims, f_in, f_out, shift, sm, st, jc);
    return adjoint
               ? dispatch_degree<float, true>(degree, axis, dims, f_in, f_out, shift, sm, st, jc)
               : dispatch_degree<float, false>(degree, axis, dims, f_in, f_out, shift, sm, st, jc);
}

int sldg_rho_stack(vp_dtype dt, int degree, const int64_t dims[4]) {
    const int64_t inner = dims[2] * dims[3];
    const int js = rho_seg_stack(dt, degree, dims);
    if (js > 0) return js;
    // whole lines (`sldg_col_rho`): one column a thread
    return inner % kBlock ? 0 : 1;
}

int64_t sldg_rho_workgroups(vp_dtype dt, int degree, const int64_t dims[4]) {
    const int js = rho_seg_stack(dt, degree, dims);
    if (js > 0) {
        const int nc = static_cast<int>(dims[1] / (degree + 1));
        const int C = rho_seg_cells(degree + 1, dt == VP_F32);
        return dims[0] * ((nc + C - 1) / C) * (dims[2] * dims[3] / (js * kBlock));
    }
    const int J = sldg_rho_stack(dt, degree, dims);
    return J > 0 ? dims[0] * dims[2] * dims[3] / (static_cast<int64_t>(kBlock) * J) : 0;
}

vp_status sldg_advect_rho_impl(int degree, vp_dtype dt, const int64_t dims[4],
                               const void* f_in, void* f_out, const double* shift,
                               const int64_t shift_stride[4], const RhoFuse& rf,
                               hipStream_t st) {
    if (sldg_rho_stack(dt, degree, dims) > 1 && shift_stride[2] != 0)
        return set_error(VP_ERR_UNSUPPORTED, "fused x2 sweep: the shift must not depend on v1");
    const ShiftMap sm = make_shift_map(1, dims, shift_stride);
    if (dt == VP_F64)
        return dispatch_rho<double>(degree, dims, f_in, f_out, shift, sm, rf, st);
    return dispatch_rho<float>(degree, dims, f_in, f_out, shift, sm, rf, st);
}

vp_status sldg_dshift_impl(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                           const void* f_in, const void* lam, const double* shift,
                           const int64_t shift_stride[4], double* g_line, hipStream_t st) {
    const ShiftMap sm = make_shift_map(axis, dims, shift_stride);
    if (dt == VP_F64)
        return dispatch_dshift<double>(degree, axis, dims, f_in, lam, shift, sm, g_line, st);
    return dispatch_dshift<float>(degree, axis, dims, f_in, lam, shift, sm, g_line, st);
}

}  // namespace vp

namespace {

vp_status check_sldg_args(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                          const void* a, const void* b, const double* shift,
                          const int64_t shift_stride[4], int64_t* total) {
    using namespace vp;
    if (axis < 0 || axis > 3) return set_error(VP_ERR_ARG, "axis %d not in 0..3", axis);
    if (degree < 0 || degree > VP_MAX_DEGREE)
        return set_error(VP_ERR_UNSUPPORTED, "degree %d not in 0..%d", degree,
                         VP_MAX_DEGREE);
    if (dt != VP_F32 && dt != VP_F64) return set_error(VP_ERR_ARG, "bad dtype %d", (int)dt);
    vp_status rc = check_dims(dims, total);
    if (rc != VP_OK) return rc;
    if (dims[axis] % (degree + 1))
        return set_error(VP_ERR_ARG, "dims[%d] = %lld is not a multiple of degree+1 = %d",
                         axis, (long long)dims[axis], degree + 1);
    if (!a || !b || !shift) return set_error(VP_ERR_ARG, "NULL pointer argument");
    return check_shift_strides(axis, dims, shift_stride);
}

}  // namespace

extern "C" vp_status sldg_advect(int axis, int degree, vp_dtype dt,
                                 const int64_t dims[4], const void* f_in,
                                 void* f_out, const double* shift,
                                 const int64_t shift_stride[4], void* stream) {
    using namespace vp;
    clear_error();
    int64_t total = 0;
    vp_status rc = check_sldg_args(axis, degree, dt, dims, f_in, f_out, shift, shift_stride,
                                   &total);
    if (rc != VP_OK) return rc;
    if (ranges_overlap(f_in, f_out, static_cast<size_t>(total) * dtype_size(dt)))
        return set_error(VP_ERR_ALIAS, "f_in and f_out overlap");
    return sldg_advect_impl(axis, degree, dt, dims, f_in, f_out, shift, shift_stride,
                            static_cast<hipStream_t>(stream), false);
}

extern "C" vp_status sldg_advect_adjoint(int axis, int degree, vp_dtype dt,
                                         const int64_t dims[4], const void* lam_out,
                                         void* lam_in, const double* shift,
                                         const int64_t shift_stride[4], void* stream) {
    using namespace vp;
    clear_error();
    int64_t total = 0;
    vp_status rc = check_sldg_args(axis, degree, dt, dims, lam_out, lam_in, shift,
                                   shift_stride, &total);
    if (rc != VP_OK) return rc;
    if (ranges_overlap(lam_out, lam_in, static_cast<size_t>(total) * dtype_size(dt)))
        return set_error(VP_ERR_ALIAS, "lam_out and lam_in overlap");
    return sldg_advect_impl(axis, degree, dt, dims, lam_out, lam_in, shift, shift_stride,
                            static_cast<hipStream_t>(stream), true);
}

extern "C" vp_status sldg_advect_dshift(int axis, int degree, vp_dtype dt,
                                        const int64_t dims[4], const void* f_in,
                                        const void* lam_out, const double* shift,
                                        const int64_t shift_stride[4], double* g_line,
                                        void* stream) {
    using namespace vp;
    clear_error();
    int64_t total = 0;
    vp_status rc = check_sldg_args(axis, degree, dt, dims, f_in, lam_out, shift,
                                   shift_stride, &total);
    if (rc != VP_OK) return rc;
    if (!g_line) return set_error(VP_ERR_ARG, "NULL pointer argument");
    return sldg_dshift_impl(axis, degree, dt, dims, f_in, lam_out, shift, shift_stride,
                            g_line, static_cast<hipStream_t>(stream));
}
