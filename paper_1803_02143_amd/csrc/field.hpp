// Internal entry points shared between the field kernels and the stepper.
#pragma once

#include "vp4d_internal.hpp"

namespace vp {

constexpr int kRedBlock = 256;

// Nodes of one axis: coordinate of dof c = lo + (c/m + xi[c%m]) h and its
// quadrature weight w[c%m] h.  The spline grid uses m = 1, xi = 1/2, w = 1.
struct AxisGrid {
    int m;
    double w[kMaxNodes];
    double xi[kMaxNodes];
    double h;
    double lo;
};
AxisGrid axis_grid(int degree, int64_t n, double lo, double len);

vp_status check_grid_args(int degree, vp_dtype dt, const int64_t dims[4],
                          int64_t* total);

// Density of the output of an x2 sweep, formed inside the sweep: every
// group of adjacent velocity columns that a workgroup (or wavefront) owns
// adds W3 W4 f_out over its columns into part[(x1 * groups + g) * N2 + j],
// and rho_from_parts sums the groups in a fixed order.
// With mom_part set, the sweep also adds up the moments of its output: each
// workgroup writes its sums of W f, W |f|, W f^2 and W |v|^2 f (W the 4D
// quadrature weight) to mom_part[4 * workgroup + q].
struct RhoFuse {
    double* part;        // device, x1 * groups * N2 doubles
    double* mom_part;    // device, 4 doubles per workgroup, or NULL
    AxisGrid g1, g2;     // x node weights (moments)
    AxisGrid g3, g4;     // velocity node weights and coordinates
    int n4;              // N4 (v2 nodes), to split the column index
};
// Velocity columns per group of the fused spline x2 sweep (0: no fused
// path for this grid); the SLDG one uses groups of 256 J columns when
// N3 N4 / J is a multiple of 256.
int spline_rho_group(vp_dtype dt, const int64_t dims[4]);
// Velocity columns per thread of the fused SLDG x2 sweep (J columns that
// share the x2 shift: one v2, J consecutive v1 nodes; J = 2 in FP32 by row
// segments, else 1), so a workgroup holds 256 J columns; 0 when N3 N4 is no
// multiple of 256 (no fused path).
int sldg_rho_stack(vp_dtype dt, int degree, const int64_t dims[4]);
// Workgroups of the fused SLDG x2 sweep that sums the moments (one moment
// partial each).
int64_t sldg_rho_workgroups(vp_dtype dt, int degree, const int64_t dims[4]);
vp_status sldg_advect_rho_impl(int degree, vp_dtype dt, const int64_t dims[4],
                               const void* f_in, void* f_out, const double* shift,
                               const int64_t shift_stride[4], const RhoFuse& rf,
                               hipStream_t st);
vp_status spline_advect_rho_impl(vp_dtype dt, const int64_t dims[4], const void* f_in,
                                 void* f_out, const double* shift,
                                 const int64_t shift_stride[4], const RhoFuse& rf,
                                 hipStream_t st);
vp_status rho_from_parts_impl(const double* part, int64_t n1, int64_t groups, int64_t n2,
                              double* rho, hipStream_t st);
// out4 = (mass, L1, L2, kinetic energy) from nparts workgroup sums (4 each);
// `chunk` (moments_chunk_doubles() doubles) holds the first stage of long sums
vp_status moments_from_parts_impl(const double* mom_part, int64_t nparts, double* chunk,
                                  double* out4, hipStream_t st);
size_t moments_chunk_doubles();
// workgroups of the fused x2 sweep (the number of mom_part entries / 4)
int64_t rho_fuse_workgroups(int method, int degree, vp_dtype dt, const int64_t dims[4]);

// Sweep (adjoint = false) or its transpose for fixed shifts (adjoint = true).
vp_status sldg_advect_impl(int axis, int degree, vp_dtype dt,
                           const int64_t dims[4], const void* f_in, void* f_out,
                           const double* shift, const int64_t shift_stride[4],
                           hipStream_t st, bool adjoint);
vp_status spline_advect_impl(int axis, vp_dtype dt, const int64_t dims[4],
                             const void* f_in, void* f_out, const double* shift,
                             const int64_t shift_stride[4], hipStream_t st, bool adjoint);
// g_line[line] = d <lam, sweep(f_in)> / d sigma_line (lines in outer-inner order)
vp_status sldg_dshift_impl(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                           const void* f_in, const void* lam, const double* shift,
                           const int64_t shift_stride[4], double* g_line, hipStream_t st);
vp_status spline_dshift_impl(int axis, vp_dtype dt, const int64_t dims[4], const void* f_in,
                             const void* lam, const double* shift,
                             const int64_t shift_stride[4], double* g_line, hipStream_t st);
vp_status density_impl(int degree, vp_dtype dt, const int64_t dims[4],
                       const void* f, double len_v1, double len_v2, double* rho,
                       hipStream_t st);
// partial[4][dims0*dims1]: per (x1,x2) sums of W f, W|f|, W f^2, W |v|^2 f
// over the velocity block (partial[0] is the density).
vp_status moments_partial_impl(int degree, vp_dtype dt, const int64_t dims[4],
                               const void* f, const double lo[4],
                               const double len[4], double* partial,
                               hipStream_t st);
vp_status moments_final_impl(int degree, const int64_t dims[4],
                             const double lo[4], const double len[4],
                             const double* partial, double* out4,
                             hipStream_t st);
vp_status poisson_impl(int degree, int64_t n1, int64_t n2, double L1, double L2,
                       const double* rho, double* E1, double* E2, double* W_el,
                       void* workspace, hipStream_t st);
// As poisson_impl, and also writes sig1 = s1*E1, sig2 = s2*E2 when sig1 != NULL.
vp_status poisson_impl_shift(int degree, int64_t n1, int64_t n2, double L1, double L2,
                             const double* rho, double* E1, double* E2, double* W_el,
                             void* workspace, double* sig1, double* sig2, double s1,
                             double s2, hipStream_t st);
// rho_bar = P_1^T G_1 + P_2^T G_2 (G weighted by the x quadrature when
// `weighted`); same workspace as poisson_impl.
vp_status poisson_adjoint_impl(int degree, int64_t n1, int64_t n2, double L1, double L2,
                               const double* g1, const double* g2, double* rho_bar,
                               void* workspace, bool weighted, hipStream_t st);
// lam (+)= rho_bar[x1][x2] W3[v1] W4[v2]
vp_status density_adjoint_impl(int degree, vp_dtype dt, const int64_t dims[4],
                               const double* rho_bar, double len_v1, double len_v2,
                               void* lam, bool accumulate, hipStream_t st);
// out[b] = scale * sum_{k<K} g[b*K + k]
vp_status line_sum_impl(const double* g, int64_t nb, int K, double scale, double* out,
                        hipStream_t st);

}  // namespace vp
