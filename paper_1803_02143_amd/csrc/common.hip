// Host-side utilities of libvp4d: error state, argument checks, the
// Gauss-Legendre basis and the nodal <-> sub-cell-midpoint transfer maps.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "vp4d_internal.hpp"

namespace vp {

namespace {
thread_local char g_err[1024] = "";
}

vp_status set_error(vp_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

vp_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(VP_ERR_HIP, "launch of %s failed: %s", what,
                         hipGetErrorString(e));
    return VP_OK;
}

vp_status check_dims(const int64_t dims[4], int64_t* total) {
    if (!dims) return set_error(VP_ERR_ARG, "dims is NULL");
    int64_t t = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 1 || dims[d] >= (int64_t(1) << 31))
            return set_error(VP_ERR_ARG, "dims[%d] = %lld out of range [1, 2^31)",
                             d, (long long)dims[d]);
        if (t > (int64_t(1) << 58) / dims[d])
            return set_error(VP_ERR_ARG, "array of %lld x %lld x %lld x %lld is too large",
                             (long long)dims[0], (long long)dims[1],
                             (long long)dims[2], (long long)dims[3]);
        t *= dims[d];
    }
    if (total) *total = t;
    return VP_OK;
}

vp_status check_shift_strides(int axis, const int64_t dims[4],
                              const int64_t stride[4]) {
    if (!stride) return set_error(VP_ERR_ARG, "shift_stride is NULL");
    if (stride[axis] != 0)
        return set_error(VP_ERR_ARG, "shift_stride[axis] must be 0 (got %lld)",
                         (long long)stride[axis]);
    int64_t span = 0;
    for (int d = 0; d < 4; ++d) {
        if (stride[d] < 0 || stride[d] >= (int64_t(1) << 40))
            return set_error(VP_ERR_ARG, "shift_stride[%d] = %lld out of range",
                             d, (long long)stride[d]);
        if (d != axis) span += (dims[d] - 1) * stride[d];
    }
    if (span >= (int64_t(1) << 46))
        return set_error(VP_ERR_ARG, "shift array span too large");
    return VP_OK;
}

bool ranges_overlap(const void* a, const void* b, size_t bytes) {
    return ranges_overlap2(a, bytes, b, bytes);
}

bool ranges_overlap2(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a);
    const uintptr_t y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

ShiftMap make_shift_map(int axis, const int64_t dims[4], const int64_t stride[4]) {
    ShiftMap sm{};
    for (int d = 0; d < axis; ++d) {
        sm.out_dim[sm.n_out] = dims[d];
        sm.out_str[sm.n_out] = stride[d];
        ++sm.n_out;
    }
    for (int d = axis + 1; d < 4; ++d) {
        sm.in_dim[sm.n_in] = dims[d];
        sm.in_str[sm.n_in] = stride[d];
        ++sm.n_in;
    }
    return sm;
}

// ------------------------------------------------------------- GL basis ---
// Roots of the Legendre polynomial P_m by Newton's method from the standard
// Chebyshev-like first guesses, P_m and P_m' from the three-term recurrence;
// weights 2 / ((1 - x^2) P_m'(x)^2), then mapped to [0, 1].
static void gauss_legendre(int m, double* xi, double* w) {
    for (int i = 0; i < m; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int j = 2; j <= m; ++j) {
                const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (m == 1) p0 = 1.0;  // P_0
            dp = m * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        // final derivative at the converged root
        double p0 = 1.0, p1 = x;
        for (int j = 2; j <= m; ++j) {
            const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        if (m == 1) p0 = 1.0;
        dp = m * (x * p1 - p0) / (x * x - 1.0);
        xi[i] = 0.5 * (1.0 - x);                     // ascending on [0, 1]
        w[i] = 1.0 / ((1.0 - x * x) * dp * dp);      // half of 2/(...)
    }
}

const NodeBasis& node_basis(int degree) {
    static NodeBasis cache[kMaxNodes];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int d = 0; d <= VP_MAX_DEGREE; ++d) {
            NodeBasis& b = cache[d];
            std::memset(&b, 0, sizeof(b));
            b.m = d + 1;
            gauss_legendre(b.m, b.xi, b.w);
            for (int j = 0; j < b.m; ++j) {
                b.inv_w[j] = 1.0 / b.w[j];
                for (int k = 0; k < b.m; ++k)
                    b.rd[j][k] = (k == j) ? 0.0 : 1.0 / (b.xi[j] - b.xi[k]);
            }
        }
    });
    return cache[degree];
}

static double lagrange_host(const NodeBasis& b, int l, double t) {
    double p = 1.0;
    for (int k = 0; k < b.m; ++k)
        if (k != l) p *= (t - b.xi[k]) / (b.xi[l] - b.xi[k]);
    return p;
}

// Gauss-Jordan inverse with partial pivoting of an m x m matrix.
static void invert(int m, const double a_in[kMaxNodes][kMaxNodes],
                   double inv[kMaxNodes][kMaxNodes]) {
    double a[kMaxNodes][2 * kMaxNodes];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < 2 * m; ++j)
            a[i][j] = j < m ? a_in[i][j] : (j - m == i ? 1.0 : 0.0);
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
        if (p != c)
            for (int j = 0; j < 2 * m; ++j) std::swap(a[p][j], a[c][j]);
        const double piv = a[c][c];
        for (int j = 0; j < 2 * m; ++j) a[c][j] /= piv;
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * m; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) inv[i][j] = a[i][j + m];
}

const TransferPair& transfer_pair(int degree) {
    static TransferPair cache[kMaxNodes];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int d = 0; d <= VP_MAX_DEGREE; ++d) {
            const NodeBasis& b = node_basis(d);
            TransferPair& t = cache[d];
            std::memset(&t, 0, sizeof(t));
            t.m = b.m;
            for (int p = 0; p < b.m; ++p)
                for (int l = 0; l < b.m; ++l)
                    t.q[p][l] = lagrange_host(b, l, (p + 0.5) / b.m);
            invert(b.m, t.q, t.qinv);
        }
    });
    return cache[degree];
}

}  // namespace vp

extern "C" const char* vp_last_error(void) { return vp::g_err; }

extern "C" const char* vp_version(void) { return "vp4d 0.1 (gfx950)"; }
