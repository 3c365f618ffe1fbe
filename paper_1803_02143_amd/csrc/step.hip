// Strang splitting time step (Sec. 2) on one HIP stream.
//
//   f^{m+1} = exp(tau/2 A) exp(tau B) exp(tau/2 A) f^m
//
// with A split into the x1 and x2 free-streaming sweeps and B into the v1
// and v2 acceleration sweeps (the directional parts commute, so the split
// adds no error).  E is computed from the density after the first half step
// and stays fixed during B, which leaves the density unchanged.  Every sweep
// reads one buffer and writes the other; six sweeps per step return the
// result to the caller's buffer.  No host synchronisation inside a step.
//
// The diagnostics of a state whose density and moments came with its closing
// x2 sweep (W from the Poisson solve of that density, the moment sums) run
// on a second stream of the state, with buffers of their own, while the next
// step's sweeps run on the caller's stream: the closing sweep writes its
// partial sums to those buffers, an event hands them to the second stream,
// and the next closing sweep waits for the diagnostics that read them.  The
// caller's stream waits for the last diagnostics before the call returns, so
// every result is ordered after the call on that stream.
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "field.hpp"

struct vp_state {
    int device;
    int method;  // 0 SLDG, 1 spline
    int degree;  // SLDG degree, -1 for the spline grid
    vp_dtype dt;
    int64_t dims[4];
    double lo[4], len[4];
    double h[4];  // shift unit per axis: cell width or grid spacing
    double* buf;  // one device allocation holding every 2D array below
    double *rho, *e1, *e2, *sig_v1, *sig_v2, *sig_x1, *sig_x2, *vnode1, *vnode2;
    double *sig_x1f, *sig_x2f;  // x shifts of a whole step (merged half-steps)
    double* rho_part;           // partial densities of the fused x2 sweep
    int64_t rho_groups;         // column groups per x1 (0: no fused x2 sweep)
    double* mom_part;           // its per-workgroup moment sums (4 each)
    double* mom_chunk;          // first-stage sums of long mom_part arrays
    int64_t mom_parts;          // workgroups of the fused x2 sweep
    double* partial;  // 4 * n1 * n2
    double *gs1, *gs2, *rho_bar;  // adjoint: shift gradients and transposed density
    void* pws;        // Poisson workspace
    // diagnostics on the second stream: partial densities of the closing x2
    // sweep, field arrays, Poisson workspace; events that order the streams
    hipStream_t side;
    hipEvent_t side_ready, side_done;
    double* rho_part_d;
    double *rho_d, *e1_d, *e2_d;
    void* pws_d;
    unsigned timing;   // bit t: timer category t records its launches
    std::vector<hipEvent_t> ev[VP_TIMER_COUNT];  // start/stop pairs
    std::vector<hipEvent_t> free_events;
};

namespace vp {
namespace {

__global__ void xshift(const double* __restrict__ v1, const double* __restrict__ v2,
                       int64_t n3, int64_t n4, double s1, double s2,
                       double* __restrict__ o1, double* __restrict__ o2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n3) o1[i] = s1 * v1[i];
    if (i < n4) o2[i] = s2 * v2[i];
}

hipEvent_t take_event(vp_state* st) {
    if (!st->free_events.empty()) {
        hipEvent_t e = st->free_events.back();
        st->free_events.pop_back();
        return e;
    }
    // timing only: no system-scope fence (cache writeback and invalidate)
    // at each record, which would cost the launches between the events time
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

void mark(vp_state* st, int timer, hipStream_t s) {
    if (!(st->timing >> timer & 1u)) return;
    hipEvent_t e = take_event(st);
    if (!e) return;
    (void)hipEventRecord(e, s);
    st->ev[timer].push_back(e);
}

// Shift strides of the step: x sweeps one value per v node, v sweeps one
// value per (x1, x2) point.
void step_strides(const vp_state* st, int axis, int64_t stride[4]) {
    stride[0] = stride[1] = stride[2] = stride[3] = 0;
    if (axis == 0) stride[2] = 1;
    else if (axis == 1) stride[3] = 1;
    else {
        stride[0] = st->dims[1];
        stride[1] = 1;
    }
}

vp_status sweep(vp_state* st, int axis, const void* in, void* out,
                const double* shift, hipStream_t s, bool adjoint = false) {
    int64_t stride[4];
    step_strides(st, axis, stride);
    if (!adjoint) mark(st, VP_TIMER_SWEEP_X1 + axis, s);
    vp_status rc = st->method == 0
                       ? sldg_advect_impl(axis, st->degree, st->dt, st->dims, in, out,
                                          shift, stride, s, adjoint)
                       : spline_advect_impl(axis, st->dt, st->dims, in, out, shift,
                                            stride, s, adjoint);
    if (!adjoint) mark(st, VP_TIMER_SWEEP_X1 + axis, s);
    return rc;
}

// The x2 sweep of a state whose density comes next: when the grid allows
// it, the sweep also writes the partial densities of its output (and the
// field then sums them instead of reading the state again).
vp_status sweep_x2_rho(vp_state* st, const void* in, void* out, const double* shift,
                       hipStream_t s, bool& fused, bool moments = false,
                       double* part = nullptr) {
    fused = st->rho_groups > 0;
    if (!fused) return sweep(st, 1, in, out, shift, s);
    int64_t stride[4];
    step_strides(st, 1, stride);
    RhoFuse rf{};
    rf.part = part ? part : st->rho_part;
    rf.mom_part = moments ? st->mom_part : nullptr;
    rf.g1 = axis_grid(st->degree, st->dims[0], st->lo[0], st->len[0]);
    rf.g2 = axis_grid(st->degree, st->dims[1], st->lo[1], st->len[1]);
    rf.g3 = axis_grid(st->degree, st->dims[2], st->lo[2], st->len[2]);
    rf.g4 = axis_grid(st->degree, st->dims[3], st->lo[3], st->len[3]);
    rf.n4 = static_cast<int>(st->dims[3]);
    mark(st, VP_TIMER_SWEEP_X2_RHO, s);
    vp_status rc = st->method == 0
                       ? sldg_advect_rho_impl(st->degree, st->dt, st->dims, in, out, shift,
                                              stride, rf, s)
                       : spline_advect_rho_impl(st->dt, st->dims, in, out, shift, stride, rf, s);
    mark(st, VP_TIMER_SWEEP_X2_RHO, s);
    return rc;
}

// W (and the moments) of the state just written by a fused closing x2
// sweep, from its partial sums (rho_part_d, mom_part), with the second
// stream's field arrays; s is the second stream.
vp_status diagnostics_fused(vp_state* st, double* W, double* mom, hipStream_t s) {
    mark(st, VP_TIMER_DIAG, s);
    vp_status rc = VP_OK;
    if (mom) rc = moments_from_parts_impl(st->mom_part, st->mom_parts, st->mom_chunk, mom, s);
    if (rc == VP_OK && W)
        rc = rho_from_parts_impl(st->rho_part_d, st->dims[0], st->rho_groups, st->dims[1],
                                 st->rho_d, s);
    if (rc == VP_OK && W)
        rc = poisson_impl(st->degree, st->dims[0], st->dims[1], st->len[0], st->len[1],
                          st->rho_d, st->e1_d, st->e2_d, W, st->pws_d, s);
    mark(st, VP_TIMER_DIAG, s);
    return rc;
}

// rho of the state f: from the fused sweep's partials, or a read of f.
vp_status density_of(vp_state* st, const void* f, bool fused, hipStream_t s) {
    if (fused)
        return rho_from_parts_impl(st->rho_part, st->dims[0], st->rho_groups, st->dims[1],
                                   st->rho, s);
    return density_impl(st->degree, st->dt, st->dims, f, st->len[2], st->len[3], st->rho, s);
}

vp_status dshift(vp_state* st, int axis, const void* f, const void* lam,
                 const double* shift, double* g_line, hipStream_t s) {
    int64_t stride[4];
    step_strides(st, axis, stride);
    return st->method == 0
               ? sldg_dshift_impl(axis, st->degree, st->dt, st->dims, f, lam, shift, stride,
                                  g_line, s)
               : spline_dshift_impl(axis, st->dt, st->dims, f, lam, shift, stride, g_line, s);
}

size_t f_bytes(const vp_state* st) {
    return static_cast<size_t>(st->dims[0] * st->dims[1] * st->dims[2] * st->dims[3]) *
           dtype_size(st->dt);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// W (and optionally the moments) of the state in f.
vp_status diagnostics(vp_state* st, const void* f, double* W, double* mom,
                      hipStream_t s) {
    mark(st, VP_TIMER_DIAG, s);
    vp_status rc;
    if (mom) {
        rc = moments_partial_impl(st->degree, st->dt, st->dims, f, st->lo, st->len,
                                  st->partial, s);
        if (rc == VP_OK)
            rc = moments_final_impl(st->degree, st->dims, st->lo, st->len, st->partial,
                                    mom, s);
        if (rc == VP_OK && W)
            rc = poisson_impl(st->degree, st->dims[0], st->dims[1], st->len[0],
                              st->len[1], st->partial, st->e1, st->e2, W, st->pws, s);
    } else {
        rc = density_impl(st->degree, st->dt, st->dims, f, st->len[2], st->len[3],
                          st->rho, s);
        if (rc == VP_OK)
            rc = poisson_impl(st->degree, st->dims[0], st->dims[1], st->len[0],
                              st->len[1], st->rho, st->e1, st->e2, W, st->pws, s);
    }
    mark(st, VP_TIMER_DIAG, s);
    return rc;
}

}  // namespace
}  // namespace vp

using namespace vp;

extern "C" vp_status vp_create(vp_state** out, int method, int degree, vp_dtype dt,
                               const int64_t dims[4], const double lo[4],
                               const double len[4]) {
    clear_error();
    if (!out) return set_error(VP_ERR_ARG, "st is NULL");
    *out = nullptr;
    if (method != 0 && method != 1) return set_error(VP_ERR_ARG, "method %d", method);
    const int deg = method == 1 ? -1 : degree;
    if (method == 0 && (degree < 0 || degree > VP_MAX_DEGREE))
        return set_error(VP_ERR_UNSUPPORTED, "degree %d", degree);
    int64_t total = 0;
    vp_status rc = check_grid_args(deg, dt, dims, &total);
    if (rc != VP_OK) return rc;
    if (!lo || !len) return set_error(VP_ERR_ARG, "NULL pointer argument");
    for (int d = 0; d < 4; ++d)
        if (!(len[d] > 0.0)) return set_error(VP_ERR_ARG, "len[%d] must be positive", d);
    if (dims[0] * dims[1] >= (int64_t(1) << 31))
        return set_error(VP_ERR_UNSUPPORTED, "x grid too large");

    int device = -1;
    VP_HIP_TRY(hipGetDevice(&device));
    vp_state* st = new (std::nothrow) vp_state();
    if (!st) return set_error(VP_ERR_ARG, "out of host memory");
    st->device = device;
    st->method = method;
    st->degree = deg;
    st->dt = dt;
    for (int d = 0; d < 4; ++d) {
        st->dims[d] = dims[d];
        st->lo[d] = lo[d];
        st->len[d] = len[d];
        st->h[d] = axis_grid(deg, dims[d], lo[d], len[d]).h;
    }
    const int64_t nx = dims[0] * dims[1];
    const size_t pws = vp_poisson_workspace(deg, dims[0], dims[1]);
    // the x2 sweep forms the density of its output in groups of velocity
    // columns: 256 J per workgroup for SLDG (J columns a thread), 64 or 32
    // per tile for the spline
    const int64_t nvel = dims[2] * dims[3];
    int64_t groups = 0;
    // (SLDG: whole workgroups of 256 J columns, and the four wavefronts' N2
    // partial sums in 48 KiB of LDS)
    if (method == 0 && sldg_rho_stack(dt, deg, dims) > 0 && 4 * (dims[1] + 4) * 8 <= 48 * 1024)
        groups = nvel / (256 * sldg_rho_stack(dt, deg, dims));
    if (method == 1 && spline_rho_group(dt, dims) > 0) groups = nvel / spline_rho_group(dt, dims);
    // (not worth more than a sixteenth of a state in partial sums)
    const size_t fbytes = static_cast<size_t>(total) * dtype_size(dt);
    if (static_cast<size_t>(dims[0] * groups * dims[1]) * sizeof(double) > fbytes / 16) groups = 0;
    const size_t npart = static_cast<size_t>(dims[0] * groups * dims[1]);
    const int64_t nwg = groups > 0 ? rho_fuse_workgroups(method, deg, dt, dims) : 0;
    // (with the second stream's partial densities, field arrays and Poisson
    // workspace)
    const size_t ndbl = static_cast<size_t>(nx) * (5 + 4 + 3 + 3) +
                        3 * static_cast<size_t>(dims[2] + dims[3]) +
                        2 * (pws / sizeof(double) + 64) + 2 * npart +
                        4 * static_cast<size_t>(nwg) + moments_chunk_doubles() + 32;
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, ndbl * sizeof(double));
    if (e != hipSuccess) {
        delete st;
        return set_error(VP_ERR_HIP, "hipMalloc of %zu bytes failed: %s", ndbl * sizeof(double),
                         hipGetErrorString(e));
    }
    double* p = static_cast<double*>(mem);
    st->buf = p;
    st->rho = p; p += nx;
    st->e1 = p; p += nx;
    st->e2 = p; p += nx;
    st->sig_v1 = p; p += nx;
    st->sig_v2 = p; p += nx;
    st->partial = p; p += 4 * nx;
    st->gs1 = p; p += nx;
    st->gs2 = p; p += nx;
    st->rho_bar = p; p += nx;
    st->sig_x1 = p; p += dims[2];
    st->sig_x2 = p; p += dims[3];
    st->vnode1 = p; p += dims[2];
    st->vnode2 = p; p += dims[3];
    st->sig_x1f = p; p += dims[2];
    st->sig_x2f = p; p += dims[3];
    st->rho_groups = groups;
    st->rho_part = p;
    p += npart;
    st->mom_parts = nwg;
    st->mom_part = p;
    p += 4 * nwg;
    st->mom_chunk = p;
    p += moments_chunk_doubles();
    st->rho_part_d = p;
    p += npart;
    st->rho_d = p; p += nx;
    st->e1_d = p; p += nx;
    st->e2_d = p; p += nx;
    p = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255));
    st->pws_d = p;
    p += pws / sizeof(double) + 32;
    p = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255));
    st->pws = p;
    // velocity node coordinates, used for the x-sweep shifts
    std::vector<double> v1(dims[2]), v2(dims[3]);
    const AxisGrid g3 = axis_grid(deg, dims[2], lo[2], len[2]);
    const AxisGrid g4 = axis_grid(deg, dims[3], lo[3], len[3]);
    for (int64_t c = 0; c < dims[2]; ++c)
        v1[c] = g3.lo + (static_cast<double>(c / g3.m) + g3.xi[c % g3.m]) * g3.h;
    for (int64_t c = 0; c < dims[3]; ++c)
        v2[c] = g4.lo + (static_cast<double>(c / g4.m) + g4.xi[c % g4.m]) * g4.h;
    e = hipMemcpy(st->vnode1, v1.data(), sizeof(double) * dims[2], hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(st->vnode2, v2.data(), sizeof(double) * dims[3], hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        delete st;
        return set_error(VP_ERR_HIP, "hipMemcpy failed: %s", hipGetErrorString(e));
    }
    // the second stream (default priority, not synchronising with the null
    // stream) and its two events
    st->side = nullptr;
    st->side_ready = st->side_done = nullptr;
    e = hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->side_ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->side_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (st->side_ready) (void)hipEventDestroy(st->side_ready);
        if (st->side) (void)hipStreamDestroy(st->side);
        (void)hipFree(mem);
        delete st;
        return set_error(VP_ERR_HIP, "stream or event creation failed: %s", hipGetErrorString(e));
    }
    st->timing = 0;
    *out = st;
    return VP_OK;
}

extern "C" void vp_destroy(vp_state* st) {
    if (!st) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != st->device) (void)hipSetDevice(st->device);
    (void)hipDeviceSynchronize();
    for (auto& v : st->ev)
        for (hipEvent_t e : v) (void)hipEventDestroy(e);
    for (hipEvent_t e : st->free_events) (void)hipEventDestroy(e);
    (void)hipEventDestroy(st->side_ready);
    (void)hipEventDestroy(st->side_done);
    (void)hipStreamDestroy(st->side);
    (void)hipFree(st->buf);
    if (cur != st->device) (void)hipSetDevice(cur);
    delete st;
}

namespace vp {
namespace {

// nsteps Strang steps in segments of `every` steps.  A segment opens with the
// x half-steps, joins the closing x half-steps of each step with the opening
// ones of the next into whole-step x sweeps, and closes with the x
// half-steps; the diagnostics of the state after each segment go to
// W_trace[j] / moments[4 j].  With every = 1 this is the plain Strang step.
// Every segment has an even number of sweeps, so the result is back in f.
vp_status strang_run(vp_state* st, void* f, void* f_tmp, int nsteps, double tau, int every,
                     double* W_trace, double* moments, hipStream_t s) {
    vp_status rc = VP_OK;
    const int64_t nv = st->dims[2] > st->dims[3] ? st->dims[2] : st->dims[3];
    // x-sweep shifts (tau/2) v / h_x and tau v / h_x, one value per velocity node
    xshift<<<blocks_for(nv, 256), 256, 0, s>>>(st->vnode1, st->vnode2, st->dims[2],
                                               st->dims[3], 0.5 * tau / st->h[0],
                                               0.5 * tau / st->h[1], st->sig_x1,
                                               st->sig_x2);
    if ((rc = check_launch("xshift")) != VP_OK) return rc;
    if (every > 1) {
        xshift<<<blocks_for(nv, 256), 256, 0, s>>>(st->vnode1, st->vnode2, st->dims[2],
                                                   st->dims[3], tau / st->h[0], tau / st->h[1],
                                                   st->sig_x1f, st->sig_x2f);
        if ((rc = check_launch("xshift")) != VP_OK) return rc;
    }
    const bool diag = W_trace || moments;
    if (diag && (rc = diagnostics(st, f, W_trace, moments, s)) != VP_OK) return rc;
    // diagnostics in flight on the second stream: the caller's stream waits
    // for them before returning, whatever the outcome
    bool side_used = false;
    struct Join {
        vp_state* st;
        hipStream_t s;
        bool& used;
        ~Join() {
            if (used) (void)hipStreamWaitEvent(s, st->side_done, 0);
        }
    } join{st, s, side_used};
    for (int seg = 0; seg < nsteps / every; ++seg) {
        bool fused = false;
        if ((rc = sweep(st, 0, f, f_tmp, st->sig_x1, s)) != VP_OK) return rc;
        if ((rc = sweep_x2_rho(st, f_tmp, f, st->sig_x2, s, fused)) != VP_OK) return rc;
        for (int j = 0; j < every; ++j) {
            mark(st, VP_TIMER_FIELD, s);
            rc = density_of(st, f, fused, s);
            // E of the current state and the v-sweep shifts tau E_d / h_{v_d}
            if (rc == VP_OK)
                rc = poisson_impl_shift(st->degree, st->dims[0], st->dims[1], st->len[0],
                                        st->len[1], st->rho, st->e1, st->e2, nullptr,
                                        st->pws, st->sig_v1, st->sig_v2, tau / st->h[2],
                                        tau / st->h[3], s);
            if (rc != VP_OK) return rc;
            mark(st, VP_TIMER_FIELD, s);
            if ((rc = sweep(st, 2, f, f_tmp, st->sig_v1, s)) != VP_OK) return rc;
            if ((rc = sweep(st, 3, f_tmp, f, st->sig_v2, s)) != VP_OK) return rc;
            const bool last = j == every - 1;
            if ((rc = sweep(st, 0, f, f_tmp, last ? st->sig_x1 : st->sig_x1f, s)) != VP_OK)
                return rc;
            if (!last)
                rc = sweep_x2_rho(st, f_tmp, f, st->sig_x2f, s, fused);
            else if (diag) {
                // the state of the diagnostics: its density and moments come
                // with the closing sweep, into the second stream's partial
                // sums (once the previous diagnostics have read them)
                if (side_used) VP_HIP_TRY(hipStreamWaitEvent(s, st->side_done, 0));
                rc = sweep_x2_rho(st, f_tmp, f, st->sig_x2, s, fused, moments != nullptr,
                                  st->rho_part_d);
            } else
                rc = sweep(st, 1, f_tmp, f, st->sig_x2, s);
            if (rc != VP_OK) return rc;
        }
        if (diag) {
            double* Wd = W_trace ? W_trace + seg + 1 : nullptr;
            double* md = moments ? moments + 4 * (seg + 1) : nullptr;
            if (fused) {
                VP_HIP_TRY(hipEventRecord(st->side_ready, s));
                VP_HIP_TRY(hipStreamWaitEvent(st->side, st->side_ready, 0));
                side_used = true;
                rc = diagnostics_fused(st, Wd, md, st->side);
                const hipError_t e = hipEventRecord(st->side_done, st->side);
                if (rc == VP_OK && e != hipSuccess)
                    rc = set_error(VP_ERR_HIP, "hipEventRecord failed: %s", hipGetErrorString(e));
            } else {
                rc = diagnostics(st, f, Wd, md, s);
            }
            if (rc != VP_OK) return rc;
        }
    }
    return VP_OK;
}

vp_status check_run_args(vp_state* st, void* f, void* f_tmp, int nsteps, double tau) {
    if (!st || !f || !f_tmp) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if (nsteps < 0) return set_error(VP_ERR_ARG, "nsteps %d < 0", nsteps);
    if (!(tau == tau) || tau > 1e300 || tau < -1e300) return set_error(VP_ERR_ARG, "tau not finite");
    if (ranges_overlap(f, f_tmp, f_bytes(st))) return set_error(VP_ERR_ALIAS, "f and f_tmp overlap");
    int cur = -1;
    VP_HIP_TRY(hipGetDevice(&cur));
    if (cur != st->device)
        return set_error(VP_ERR_ARG, "state belongs to device %d, current device is %d",
                         st->device, cur);
    return VP_OK;
}

}  // namespace
}  // namespace vp

extern "C" vp_status vp_strang_step(vp_state* st, void* f, void* f_tmp, int nsteps,
                                    double tau, double* W_trace, double* moments,
                                    void* stream) {
    clear_error();
    vp_status rc = check_run_args(st, f, f_tmp, nsteps, tau);
    if (rc != VP_OK) return rc;
    return strang_run(st, f, f_tmp, nsteps, tau, 1, W_trace, moments,
                      static_cast<hipStream_t>(stream));
}

extern "C" vp_status vp_strang_run(vp_state* st, void* f, void* f_tmp, int nsteps, double tau,
                                   int diag_every, double* W_trace, double* moments,
                                   void* stream) {
    clear_error();
    vp_status rc = check_run_args(st, f, f_tmp, nsteps, tau);
    if (rc != VP_OK) return rc;
    if (diag_every < 1) return set_error(VP_ERR_ARG, "diag_every %d < 1", diag_every);
    if (nsteps % diag_every)
        return set_error(VP_ERR_ARG, "nsteps %d is not a multiple of diag_every %d", nsteps,
                         diag_every);
    return strang_run(st, f, f_tmp, nsteps, tau, diag_every, W_trace, moments,
                      static_cast<hipStream_t>(stream));
}

extern "C" vp_status vp_timing_enable(vp_state* st, int enable) {
    clear_error();
    if (!st) return set_error(VP_ERR_ARG, "st is NULL");
    st->timing = enable != 0 ? (1u << VP_TIMER_COUNT) - 1u : 0u;
    return VP_OK;
}

extern "C" vp_status vp_timing_select(vp_state* st, unsigned mask) {
    clear_error();
    if (!st) return set_error(VP_ERR_ARG, "st is NULL");
    if (mask >> VP_TIMER_COUNT)
        return set_error(VP_ERR_ARG, "timer mask 0x%x has bits beyond the %d categories", mask,
                         static_cast<int>(VP_TIMER_COUNT));
    st->timing = mask;
    return VP_OK;
}

extern "C" vp_status vp_timing_read(vp_state* st, double* ms, int64_t* counts) {
    clear_error();
    if (!st || !ms || !counts) return set_error(VP_ERR_ARG, "NULL pointer argument");
    for (int t = 0; t < VP_TIMER_COUNT; ++t) {
        auto& v = st->ev[t];
        const size_t pairs = v.size() / 2;
        if (pairs) VP_HIP_TRY(hipEventSynchronize(v[2 * pairs - 1]));
        for (size_t i = 0; i < pairs; ++i) {
            float x = 0.f;
            VP_HIP_TRY(hipEventElapsedTime(&x, v[2 * i], v[2 * i + 1]));
            ms[t] += x;
            counts[t] += 1;
        }
        for (hipEvent_t e : v) st->free_events.push_back(e);
        v.clear();
    }
    return VP_OK;
}

extern "C" size_t vp_strang_adjoint_workspace(const vp_state* st) {
    if (!st) return 0;
    const int64_t nv = st->dims[2] > st->dims[3] ? st->dims[2] : st->dims[3];
    return 2 * align256(f_bytes(st)) +
           sizeof(double) * static_cast<size_t>(st->dims[0] * st->dims[1] * nv);
}

extern "C" vp_status vp_strang_adjoint(vp_state* st, const void* f, void* lam, double tau,
                                       void* work, size_t ws_bytes, void* stream) {
    clear_error();
    if (!st || !f || !lam || !work) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if (!(tau == tau) || tau > 1e300 || tau < -1e300) return set_error(VP_ERR_ARG, "tau not finite");
    if (ws_bytes < vp_strang_adjoint_workspace(st))
        return set_error(VP_ERR_WORKSPACE, "workspace of %zu bytes needed",
                         vp_strang_adjoint_workspace(st));
    const size_t fb = f_bytes(st);
    if (ranges_overlap(f, lam, fb)) return set_error(VP_ERR_ALIAS, "f and lam overlap");
    const size_t wb = vp_strang_adjoint_workspace(st);
    if (ranges_overlap2(f, fb, work, wb) || ranges_overlap2(lam, fb, work, wb))
        return set_error(VP_ERR_ALIAS, "workspace overlaps f or lam");
    int cur = -1;
    VP_HIP_TRY(hipGetDevice(&cur));
    if (cur != st->device)
        return set_error(VP_ERR_ARG, "state belongs to device %d, current device is %d",
                         st->device, cur);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // two state-sized buffers: P holds f2, Q holds f1, then f3, then the
    // adjoint between the v2 and v1 transposes
    unsigned char* w = static_cast<unsigned char*>(work);
    void* bufP = w;
    void* bufQ = w + align256(fb);
    double* gline = reinterpret_cast<double*>(w + 2 * align256(fb));
    const int64_t nx = st->dims[0] * st->dims[1];
    vp_status rc;

    const int64_t nv = st->dims[2] > st->dims[3] ? st->dims[2] : st->dims[3];
    xshift<<<blocks_for(nv, 256), 256, 0, s>>>(st->vnode1, st->vnode2, st->dims[2],
                                               st->dims[3], 0.5 * tau / st->h[0],
                                               0.5 * tau / st->h[1], st->sig_x1,
                                               st->sig_x2);
    if ((rc = check_launch("xshift")) != VP_OK) return rc;
    // backward through x2, x1 of the second half step (Q is still free)
    if ((rc = sweep(st, 1, lam, bufQ, st->sig_x2, s, true)) != VP_OK) return rc;
    if ((rc = sweep(st, 0, bufQ, lam, st->sig_x1, s, true)) != VP_OK) return rc;
    // recompute the states the shift derivatives need: f2 (P), f3 (Q)
    bool fused = false;
    if ((rc = sweep(st, 0, f, bufQ, st->sig_x1, s)) != VP_OK) return rc;
    if ((rc = sweep_x2_rho(st, bufQ, bufP, st->sig_x2, s, fused)) != VP_OK) return rc;
    rc = density_of(st, bufP, fused, s);
    if (rc == VP_OK)
        rc = poisson_impl_shift(st->degree, st->dims[0], st->dims[1], st->len[0], st->len[1],
                                st->rho, st->e1, st->e2, nullptr, st->pws, st->sig_v1,
                                st->sig_v2, tau / st->h[2], tau / st->h[3], s);
    if (rc != VP_OK) return rc;
    if ((rc = sweep(st, 2, bufP, bufQ, st->sig_v1, s)) != VP_OK) return rc;
    // v2 sweep: shift gradient with f3, then the transpose overwrites f3
    if ((rc = dshift(st, 3, bufQ, lam, st->sig_v2, gline, s)) != VP_OK) return rc;
    if ((rc = line_sum_impl(gline, nx, static_cast<int>(st->dims[2]), tau / st->h[3], st->gs2,
                            s)) != VP_OK)
        return rc;
    if ((rc = sweep(st, 3, lam, bufQ, st->sig_v2, s, true)) != VP_OK) return rc;
    // v1 sweep: shift gradient with f2, then transpose back into lam
    if ((rc = dshift(st, 2, bufP, bufQ, st->sig_v1, gline, s)) != VP_OK) return rc;
    if ((rc = line_sum_impl(gline, nx, static_cast<int>(st->dims[3]), tau / st->h[2], st->gs1,
                            s)) != VP_OK)
        return rc;
    if ((rc = sweep(st, 2, bufQ, lam, st->sig_v1, s, true)) != VP_OK) return rc;
    // field: dJ/dE -> rho_bar -> density transpose, added to the adjoint of f2
    rc = poisson_adjoint_impl(st->degree, st->dims[0], st->dims[1], st->len[0], st->len[1],
                              st->gs1, st->gs2, st->rho_bar, st->pws, false, s);
    if (rc == VP_OK)
        rc = density_adjoint_impl(st->degree, st->dt, st->dims, st->rho_bar, st->len[2],
                                  st->len[3], lam, true, s);
    if (rc != VP_OK) return rc;
    // backward through x2, x1 of the first half step
    if ((rc = sweep(st, 1, lam, bufP, st->sig_x2, s, true)) != VP_OK) return rc;
    return sweep(st, 0, bufP, lam, st->sig_x1, s, true);
}

extern "C" vp_status vp_energy_gradient(vp_state* st, const void* f, void* lam, double* W,
                                        void* stream) {
    clear_error();
    if (!st || !f || !lam) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if (ranges_overlap(f, lam, f_bytes(st))) return set_error(VP_ERR_ALIAS, "f and lam overlap");
    int cur = -1;
    VP_HIP_TRY(hipGetDevice(&cur));
    if (cur != st->device)
        return set_error(VP_ERR_ARG, "state belongs to device %d, current device is %d",
                         st->device, cur);
    hipStream_t s = static_cast<hipStream_t>(stream);
    vp_status rc = density_impl(st->degree, st->dt, st->dims, f, st->len[2], st->len[3],
                                st->rho, s);
    if (rc == VP_OK)
        rc = poisson_impl(st->degree, st->dims[0], st->dims[1], st->len[0], st->len[1], st->rho,
                          st->e1, st->e2, W, st->pws, s);
    if (rc == VP_OK)
        rc = poisson_adjoint_impl(st->degree, st->dims[0], st->dims[1], st->len[0], st->len[1],
                                  st->e1, st->e2, st->rho_bar, st->pws, true, s);
    if (rc == VP_OK)
        rc = density_adjoint_impl(st->degree, st->dt, st->dims, st->rho_bar, st->len[2],
                                  st->len[3], lam, false, s);
    return rc;
}
