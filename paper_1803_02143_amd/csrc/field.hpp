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

vp_status sldg_advect_impl(int axis, int degree, vp_dtype dt,
                           const int64_t dims[4], const void* f_in, void* f_out,
                           const double* shift, const int64_t shift_stride[4],
                           hipStream_t st);
vp_status spline_advect_impl(int axis, vp_dtype dt, const int64_t dims[4],
                             const void* f_in, void* f_out, const double* shift,
                             const int64_t shift_stride[4], hipStream_t st);
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

}  // namespace vp
