/*
 * vp4d.h -- C ABI of the MI355X (gfx950) library for the split-step
 * semi-Lagrangian 2D-2V Vlasov-Poisson solver of Einkemmer,
 * "A comparison of semi-Lagrangian discontinuous Galerkin and spline based
 * Vlasov solvers in four dimensions" (arXiv:1803.02143).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  The distribution f(x1, x2, v1, v2) is a dense C-order array
 *   f[dims[0]][dims[1]][dims[2]][dims[3]] (v2 fastest), in device memory,
 *   with dims[d] degrees of freedom along axis d.  For the SLDG method
 *   dims[d] = n_cells[d] * (degree + 1) and the dof of cell c, node j sits at
 *   index c*(degree+1)+j with the Gauss-Legendre nodes in ascending order
 *   (Sec. 3, text around Eq. (5)).  For the spline method point i of axis d
 *   sits at lo[d] + (i + 1/2) * len[d] / dims[d].
 * Precision.  vp_dtype selects the storage and arithmetic type of f
 *   (VP_F32: float, VP_F64: double).  Shifts, operator coefficients,
 *   densities, fields, energies and moments are always double.
 * Pointers.  "device" pointers must be device (or managed) memory visible to
 *   the current HIP device; "host" pointers are read on the host before the
 *   call returns.  The caller owns every buffer; the library never frees or
 *   keeps a caller pointer past the call (vp_state keeps only its own memory).
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Work is enqueued asynchronously; no entry point synchronises
 *   the device except vp_timing_read.
 * Errors.  Arguments are validated on the host before anything is enqueued;
 *   on a non-OK status nothing has been enqueued, except VP_ERR_HIP, which
 *   reports a failed launch or allocation.  vp_last_error() returns a
 *   thread-local message describing the last non-OK status.  Shifts are read
 *   on the device: a non-finite shift, or one of magnitude above 2^62 cells,
 *   yields NaN on its line and never an out-of-range access.
 */
#ifndef VP4D_H
#define VP4D_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define VP4D_API __attribute__((visibility("default")))
#else
#define VP4D_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VP_OK = 0,
    VP_ERR_ARG = -1,          /* invalid argument (null pointer, bad size, ...) */
    VP_ERR_UNSUPPORTED = -2,  /* valid request this build does not implement   */
    VP_ERR_ALIAS = -3,        /* input and output buffers overlap              */
    VP_ERR_HIP = -4,          /* a HIP call failed; see vp_last_error()        */
    VP_ERR_WORKSPACE = -5     /* workspace missing or too small                */
} vp_status;

typedef enum { VP_F32 = 0, VP_F64 = 1 } vp_dtype;

/* Largest supported SLDG polynomial degree (degree 0..VP_MAX_DEGREE). */
#define VP_MAX_DEGREE 5

/*
 * sldg_advect -- one SLDG sweep along `axis` (Sec. 2 last part; Sec. 3 Eq. (5)).
 *
 * Every line of f along `axis` is translated by its own shift sigma (in
 * cells of that axis: u'(x) = u(x - sigma*h)) and L2-projected back onto
 * cell-wise polynomials of degree `degree`.  With n = floor(sigma) and
 * alpha = sigma - n, output cell i reads input cells i-n-1 and i-n (periodic)
 * and applies the (degree+1)x(degree+1) matrices A(alpha) and B(alpha).
 *
 *   axis          0..3 (x1, x2, v1, v2).
 *   degree        0..VP_MAX_DEGREE; dims[axis] % (degree+1) == 0.
 *   dt            storage/arithmetic type of f_in and f_out.
 *   dims          host, 4 entries >= 1, each < 2^31.
 *   f_in          device, read only.
 *   f_out         device, written; must not overlap f_in (VP_ERR_ALIAS).
 *   shift         device, double, read only.  The line with indices
 *                 (i0, i1, i2, i3) (i_axis ignored) reads
 *                 shift[sum_{d != axis} i_d * shift_stride[d]].
 *   shift_stride  host, 4 entries >= 0 with shift_stride[axis] == 0; a zero
 *                 stride broadcasts the shift along that axis.
 */
VP4D_API vp_status sldg_advect(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                      const void* f_in, void* f_out, const double* shift,
                      const int64_t shift_stride[4], void* stream);

/*
 * spline_advect -- one periodic cubic-spline sweep along `axis` (Sec. 3).
 *
 * Every line (n = dims[axis] equidistant points) is interpolated by the
 * periodic cubic spline sum_k omega_k S(x - x_k), with omega solving the
 * periodic tridiagonal system (1/6)(omega_{i-1} + 4 omega_i + omega_{i+1}) =
 * u_i, and the spline is evaluated at x_i - sigma*h.  sigma is in grid
 * points.  The coefficients omega stay on chip and are never written to
 * memory.  Arguments as for sldg_advect (any dims[axis] >= 1), except
 *   degree        the spline degree: must be 3 (the cubic B-spline of Sec. 3);
 *                 any other value is VP_ERR_UNSUPPORTED.
 */
VP4D_API vp_status spline_advect(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                        const void* f_in, void* f_out, const double* shift,
                        const int64_t shift_stride[4], void* stream);

/*
 * vp_density -- rho(x1, x2) = int f dv1 dv2 (Sec. 2).
 *
 *   degree   >= 0: SLDG, Gauss-Legendre quadrature in each v cell of width
 *            len_v/(dims/(degree+1)); -1: spline grid, rectangle rule with
 *            spacing len_v/dims.
 *   rho      device, double, dims[0]*dims[1] entries, row-major [x1][x2].
 */
VP4D_API vp_status vp_density(int degree, vp_dtype dt, const int64_t dims[4],
                     const void* f, double len_v1, double len_v2, double* rho,
                     void* stream);

/*
 * vp_poisson -- electric field of div E = rho - 1, curl E = 0 on the
 * periodic box [0,L1)x[0,L2) (Sec. 1, Eq. (1)), and W = 1/2 int |E|^2 dx.
 *
 * E = -grad phi, -Lap phi = rho - 1, solved with discrete Fourier transforms
 * on an n1 x n2 grid.  For degree >= 0 (SLDG) the nodal density is first
 * mapped, cell by cell, to the values at degree+1 equidistant sub-cell
 * midpoints (a uniform grid), and E is mapped back by the inverse map.
 * Fourier modes m = 0 and modes with m1 = n1/2 or m2 = n2/2 (even n) are
 * zeroed.  W uses the nodal quadrature of the grid.
 *
 *   rho       device, double [n1][n2], read only.
 *   E1, E2    device, double [n1][n2], written.
 *   W_el      device, one double, written (may be NULL).
 *   workspace device, at least vp_poisson_workspace(degree, n1, n2) bytes.
 */
VP4D_API vp_status vp_poisson(int degree, int64_t n1, int64_t n2, double L1, double L2,
                     const double* rho, double* E1, double* E2, double* W_el,
                     void* workspace, size_t ws_bytes, void* stream);
VP4D_API size_t vp_poisson_workspace(int degree, int64_t n1, int64_t n2);

/*
 * vp_poisson_noalloc -- vp_poisson for callers that cannot allocate device
 * memory or pass a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, result and
 * kernels as vp_poisson, without the workspace: the library keeps a static
 * device array of 12.6 MB on every device it runs on (held until the
 * process ends) and the call allocates nothing.
 *
 *   n1 * n2  at most VP_POISSON_NOALLOC_MAX_POINTS; a larger grid is
 *            VP_ERR_WORKSPACE (use vp_poisson with a workspace).
 * Every call on one device uses that device's array, which keeps the last
 * call's contents (nothing in it needs to start at zero).  Calls that
 * overlap in time on one device (different streams, different threads
 * without ordering) race on it; calls ordered on one stream do not.
 */
#define VP_POISSON_NOALLOC_MAX_POINTS (512 * 512)
VP4D_API vp_status vp_poisson_noalloc(int degree, int64_t n1, int64_t n2, double L1, double L2,
                             const double* rho, double* E1, double* E2, double* W_el,
                             void* stream);

/*
 * vp_moments -- diagnostics of Sec. 4: mass = int f, L1 = int |f|,
 * L2 = (int f^2)^(1/2), kinetic energy = 1/2 int (v1^2 + v2^2) f, with the
 * nodal quadrature of the grid (degree as in vp_density).
 *
 *   lo, len   host, 4 doubles each: the box [lo, lo+len) of every axis.
 *   out4      device, 4 doubles written in that order.
 *   workspace device, at least vp_moments_workspace(dims) bytes.
 */
VP4D_API vp_status vp_moments(int degree, vp_dtype dt, const int64_t dims[4],
                     const void* f, const double lo[4], const double len[4],
                     double* out4, void* workspace, size_t ws_bytes,
                     void* stream);
VP4D_API size_t vp_moments_workspace(const int64_t dims[4]);

/*
 * vp_init -- sample an initial condition at the nodes (the dofs are point
 * values, Sec. 3).
 *
 *   kind 0  Landau (Sec. 4, Eq. (6)):
 *           (2 pi)^-1 exp(-(v1^2+v2^2)/2) (1 + eps (cos k x1 + cos k x2)).
 *   kind 1  two-stream (Sec. 5, Eq. (7)) with the perturbation written as a
 *           sum: (8 pi)^-1 g(v1) g(v2) (1 + eps (cos k x1 + cos k x2)),
 *           g(v) = exp(-(v-v0)^2/2) + exp(-(v+v0)^2/2).
 *   kind 2  two-stream with the product perturbation of Eq. (7):
 *           (1 + eps cos k x1 cos k x2).
 *   degree  >= 0 SLDG nodes, -1 spline grid.
 *   f       device, written.
 */
VP4D_API vp_status vp_init(int kind, double eps, double k, double v0, int degree,
                  vp_dtype dt, const int64_t dims[4], const double lo[4],
                  const double len[4], void* f, void* stream);

/*
 * vp_state -- a solver instance that owns its scratch on the HIP device
 * current at vp_create: the two-dimensional arrays (density, field, shift
 * arrays, Poisson and moment workspaces) and, where the x2 sweep forms the
 * density of its output (see vp_strang_step), that sweep's partial sums:
 * N1 N2 N3 N4 / 256 doubles for SLDG, N1 N2 N3 N4 / 64 or / 32 for the spline
 * (at most 1/16 of the bytes of f).  f itself is always the caller's.  Not
 * thread safe; calls that share a state must be serialised by the caller.
 *
 * vp_create   method 0 = SLDG (degree 0..VP_MAX_DEGREE), 1 = cubic spline
 *             (degree ignored).  dims/lo/len as above (host).
 */
typedef struct vp_state vp_state;
VP4D_API vp_status vp_create(vp_state** st, int method, int degree, vp_dtype dt,
                    const int64_t dims[4], const double lo[4],
                    const double len[4]);
VP4D_API void vp_destroy(vp_state* st);

/*
 * vp_strang_step -- `nsteps` Strang steps (Sec. 2):
 *   f^{m+1} = exp(tau/2 A) exp(tau B) exp(tau/2 A) f^m,
 * each as the sweeps x1 (tau/2), x2 (tau/2), [rho -> E], v1 (tau E1),
 * v2 (tau E2), x1 (tau/2), x2 (tau/2).  x-sweep shifts are
 * (tau/2) v_d / h_{x_d} per v_d node; v-sweep shifts tau E_d(x1,x2) / h_{v_d}.
 *
 *   f        device, f^m on entry, f^{m+nsteps} on return.
 *   f_tmp    device, same size as f, scratch (ping-pong partner).
 *   W_trace  device, nsteps+1 doubles or NULL: W of f^m ... f^{m+nsteps}.
 *   moments  device, 4*(nsteps+1) doubles or NULL: mass, L1, L2, kinetic
 *            energy of the same states.
 * When the x2 sweep can form the density of its output, the x2 sweep that
 * precedes each field solve (and the diagnostics) does so, and the separate
 * read of f for rho is skipped; rho then differs from vp_density only in the
 * order of its FP64 additions.  Conditions: SLDG, N3*N4 a multiple of 256
 * and N2 <= 1532 (four wavefronts' partial sums in 48 KiB of LDS);
 * spline, N3*N4 < 2^31 and a multiple of the tile width L (64 lines when
 * N2 * 64 * sizeof(T) <= 48 KiB, else 32) with N2 a multiple of 256/L (and of
 * 16 for FP64 64-line tiles); for both, per-workgroup partial sums of at
 * most 1/16 of a state.
 */
VP4D_API vp_status vp_strang_step(vp_state* st, void* f, void* f_tmp, int nsteps,
                         double tau, double* W_trace, double* moments,
                         void* stream);

/*
 * vp_strang_run -- the same `nsteps` Strang steps with the state formed only
 * every `diag_every` steps.  Inside a segment of diag_every steps the closing
 * x half-steps of one step and the opening ones of the next are one x sweep
 * of the whole step (the exact free-streaming flows compose, Sec. 2:
 * exp(tau/2 A) exp(tau/2 A) = exp(tau A)), so a segment of k steps takes
 * 4k + 2 sweeps instead of 6k; the discrete result differs from
 * vp_strang_step (one projection instead of two per x flow) except for
 * diag_every = 1, where the two are identical.
 *
 *   nsteps     a multiple of diag_every >= 1 (else VP_ERR_ARG).
 *   W_trace    device, nsteps/diag_every + 1 doubles or NULL: W of f^0,
 *              f^{diag_every}, ..., f^{nsteps} (relative to the entry state).
 *   moments    device, 4*(nsteps/diag_every + 1) doubles or NULL.
 * Other arguments as for vp_strang_step.
 */
VP4D_API vp_status vp_strang_run(vp_state* st, void* f, void* f_tmp, int nsteps,
                        double tau, int diag_every, double* W_trace,
                        double* moments, void* stream);

/* ------------------------------------------------------------------------
 * Reverse mode.  Transposes are taken with respect to the Euclidean inner
 * product of the dof arrays, <a, b> = sum_i a_i b_i (the discrete map is
 * differentiated as it is computed).
 * ---------------------------------------------------------------------- */

/*
 * sldg_advect_adjoint -- transpose of sldg_advect for fixed shifts:
 * lam_in_c = B(alpha)^T lam_out_{c+n} + A(alpha)^T lam_out_{c+n+1} (cells
 * mod n_c, n = floor(sigma)).  Arguments as for sldg_advect with
 * (f_in, f_out) replaced by (lam_out, lam_in); they must not overlap.
 */
VP4D_API vp_status sldg_advect_adjoint(int axis, int degree, vp_dtype dt,
                              const int64_t dims[4], const void* lam_out, void* lam_in,
                              const double* shift, const int64_t shift_stride[4],
                              void* stream);

/*
 * sldg_advect_dshift -- derivative of <lam_out, sldg_advect(f_in)> with
 * respect to the shift of every line:
 * g_line[line] = sum_i lam_i . (A'(alpha) u_{i-n-1} + B'(alpha) u_{i-n}),
 * A' = dA/dalpha, B' = dB/dalpha from the defining integrals (Leibniz rule).
 *   g_line  device, double, one value per line: prod(dims)/dims[axis]
 *           entries in C order of the remaining axes.
 */
VP4D_API vp_status sldg_advect_dshift(int axis, int degree, vp_dtype dt,
                             const int64_t dims[4], const void* f_in, const void* lam_out,
                             const double* shift, const int64_t shift_stride[4],
                             double* g_line, void* stream);

/* spline_advect_adjoint -- transpose of spline_advect for fixed shifts,
 * C^{-1} E(alpha)^T lam_out (C is symmetric).  As sldg_advect_adjoint;
 * degree must be 3. */
VP4D_API vp_status spline_advect_adjoint(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                                const void* lam_out, void* lam_in, const double* shift,
                                const int64_t shift_stride[4], void* stream);

/* spline_advect_dshift -- per-line derivative of <lam_out, spline_advect(f_in)>
 * with respect to the shift (derivative of the B-spline weights); degree
 * must be 3. */
VP4D_API vp_status spline_advect_dshift(int axis, int degree, vp_dtype dt, const int64_t dims[4],
                               const void* f_in, const void* lam_out, const double* shift,
                               const int64_t shift_stride[4], double* g_line,
                               void* stream);

/*
 * vp_density_adjoint -- transpose of vp_density:
 * lam[x1][x2][c][e] (+)= rho_bar[x1][x2] * W3_c * W4_e, with the quadrature
 * weights of vp_density.  accumulate != 0 adds to lam, 0 overwrites it.
 */
VP4D_API vp_status vp_density_adjoint(int degree, vp_dtype dt, const int64_t dims[4],
                             const double* rho_bar, double len_v1, double len_v2,
                             void* lam, int accumulate, void* stream);

/*
 * vp_poisson_adjoint -- transpose of the field map of vp_poisson:
 * rho_bar = P_1^T G1 + P_2^T G2 where (E1, E2) = (P_1 rho, P_2 rho).  On the
 * uniform grid P_d^T = -P_d (an odd real Fourier multiplier); the SLDG cell
 * maps are transposed.  Workspace as vp_poisson.
 */
VP4D_API vp_status vp_poisson_adjoint(int degree, int64_t n1, int64_t n2, double L1, double L2,
                             const double* G1, const double* G2, double* rho_bar,
                             void* workspace, size_t ws_bytes, void* stream);

/*
 * vp_energy_gradient -- W = 1/2 sum w_a w_b (E1^2 + E2^2) of the state f
 * (written to W when not NULL, device) and lam = dW/df (written).
 */
VP4D_API vp_status vp_energy_gradient(vp_state* st, const void* f, void* lam, double* W,
                             void* stream);

/*
 * vp_strang_adjoint -- one Strang step backwards.  On entry lam holds
 * dJ/df^{m+1}; on return it holds dJ/df^m, for the step of size tau taken
 * from f = f^m (Sec. 2).  The step's internal states are recomputed from f;
 * the shift dependence of the acceleration sweeps on E(rho(f)) is carried
 * through the Poisson and density transposes.
 *   work  device, at least vp_strang_adjoint_workspace(st) bytes: two
 *         copies of f (each rounded up to 256 bytes) and one double per
 *         line of the longer velocity axis, 8 N1 N2 max(N3, N4) bytes.
 * f, lam and work must not overlap (VP_ERR_ALIAS); a workspace that is
 * too small is VP_ERR_WORKSPACE.  Enqueued on `stream`, asynchronous.
 */
VP4D_API size_t vp_strang_adjoint_workspace(const vp_state* st);
VP4D_API vp_status vp_strang_adjoint(vp_state* st, const void* f, void* lam, double tau,
                            void* work, size_t ws_bytes, void* stream);

/*
 * Kernel timers of a vp_state.  When enabled, vp_strang_step and
 * vp_strang_run record HIP events around their launches on `stream`.  vp_timing_read synchronises the
 * events recorded so far, adds their durations per category into ms[] and
 * counts[] (VP_TIMER_COUNT entries each, both host) and clears them.
 */
enum {
    VP_TIMER_SWEEP_X1 = 0, VP_TIMER_SWEEP_X2 = 1, VP_TIMER_SWEEP_V1 = 2,
    VP_TIMER_SWEEP_V2 = 3, VP_TIMER_FIELD = 4, VP_TIMER_DIAG = 5,
    VP_TIMER_SWEEP_X2_RHO = 6,  /* x2 sweeps that also form the density */
    VP_TIMER_COUNT = 7
};
VP4D_API vp_status vp_timing_enable(vp_state* st, int enable);
/*
 * vp_timing_select -- time only the categories whose bit (1 << VP_TIMER_x) is
 * set in `mask` (0: none; vp_timing_enable(st, 1) selects all).  Each timed
 * launch costs two event records on the stream, so a caller that needs one
 * category's durations selects only that one.  Bits at or above
 * VP_TIMER_COUNT are VP_ERR_ARG.
 */
VP4D_API vp_status vp_timing_select(vp_state* st, unsigned mask);
VP4D_API vp_status vp_timing_read(vp_state* st, double* ms, int64_t* counts);

/*
 * vp_copy_pattern -- a measurement aid: copies f_in to f_out (same shape,
 * dtype dt) with the global-memory access pattern of one family of sweep
 * kernels and no arithmetic, so that a sweep's rate can be read against
 * the bandwidth its own access pattern reaches on the device.
 *
 *   VP_PATTERN_CONTIGUOUS  flat, 16 bytes per lane (row sweeps; axis ignored)
 *   VP_PATTERN_TILES       lines along `axis` in tiles of 64 adjacent lines,
 *                          a quarter line per thread, its loads and then its
 *                          stores (spline column sweeps); dims[axis] <= 384
 *   VP_PATTERN_SEGMENTS    lines along `axis` by segments of 24 rows, one
 *                          thread per (segment, line), blocks in memory order
 *                          (row-segment SLDG sweeps)
 *   VP_PATTERN_LINES       lines along `axis`, one thread per whole line,
 *                          rows in memory order (the fused SLDG x2 sweep)
 *   axis       0..2 for the strided patterns.
 *   f_in/out   device, 16-byte aligned, not overlapping (VP_ERR_ALIAS).
 */
enum {
    VP_PATTERN_CONTIGUOUS = 0, VP_PATTERN_TILES = 1, VP_PATTERN_SEGMENTS = 2,
    VP_PATTERN_LINES = 3
};
VP4D_API vp_status vp_copy_pattern(int pattern, vp_dtype dt, const int64_t dims[4], int axis,
                          const void* f_in, void* f_out, void* stream);

/* Thread-local description of the last non-OK status ("" if none). */
VP4D_API const char* vp_last_error(void);

/* Library version string. */
VP4D_API const char* vp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VP4D_H */
