// Internal declarations shared by the translation units of libvp4d.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "vp4d.h"

namespace vp {

constexpr int kMaxNodes = VP_MAX_DEGREE + 1;

// ----------------------------------------------------------- error state ---
vp_status set_error(vp_status code, const char* fmt, ...);
void clear_error();

#define VP_HIP_TRY(expr)                                                     \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            return ::vp::set_error(VP_ERR_HIP, "%s failed: %s (%s:%d)",      \
                                   #expr, hipGetErrorString(e_), __FILE__,   \
                                   __LINE__);                                \
    } while (0)

// Checks the launch that was just enqueued.
vp_status check_launch(const char* what);

// --------------------------------------------------------- 1D node basis ---
// Gauss-Legendre nodes on [0,1] (ascending), weights summing to one, and the
// reciprocal node differences used to evaluate Lagrange polynomials.
struct NodeBasis {
    int m;                               // nodes per cell (degree + 1)
    double xi[kMaxNodes];
    double w[kMaxNodes];
    double inv_w[kMaxNodes];
    double rd[kMaxNodes][kMaxNodes];     // rd[j][k] = 1/(xi_j - xi_k), k != j
};

// Fills `b` for polynomial degree 0..VP_MAX_DEGREE (host, cached).
const NodeBasis& node_basis(int degree);

// Values of the cell polynomial at m equidistant sub-cell midpoints
// (Q[p][l] = L_l((p+1/2)/m)) and the inverse map.
struct TransferPair {
    int m;
    double q[kMaxNodes][kMaxNodes];
    double qinv[kMaxNodes][kMaxNodes];
};
const TransferPair& transfer_pair(int degree);

// -------------------------------------------------------- argument checks ---
vp_status check_dims(const int64_t dims[4], int64_t* total);
vp_status check_shift_strides(int axis, const int64_t dims[4],
                              const int64_t stride[4]);
bool ranges_overlap(const void* a, const void* b, size_t bytes);
// [a, a+na) and [b, b+nb) intersect
bool ranges_overlap2(const void* a, size_t na, const void* b, size_t nb);

inline size_t dtype_size(vp_dtype dt) { return dt == VP_F64 ? 8 : 4; }

// Decomposes the index of a line into the strided shift offset.  The
// dimensions before the swept axis form the "outer" index, the ones after
// it the "inner" index (C order).
struct ShiftMap {
    int n_out, n_in;
    int64_t out_dim[3], out_str[3];
    int64_t in_dim[3], in_str[3];
};
ShiftMap make_shift_map(int axis, const int64_t dims[4], const int64_t stride[4]);

// (Unrolled with constant indices so that the map stays in registers.)
__device__ __forceinline__ int64_t shift_offset(const ShiftMap& sm, int64_t o,
                                                int64_t k) {
    int64_t off = 0;
#pragma unroll
    for (int d = 2; d >= 0; --d) {
        if (d < sm.n_out) {
            const int64_t q = o / sm.out_dim[d];
            off += (o - q * sm.out_dim[d]) * sm.out_str[d];
            o = q;
        }
    }
#pragma unroll
    for (int d = 2; d >= 0; --d) {
        if (d < sm.n_in) {
            const int64_t q = k / sm.in_dim[d];
            off += (k - q * sm.in_dim[d]) * sm.in_str[d];
            k = q;
        }
    }
    return off;
}

// Splits a shift into its cell offset reduced modulo n (0 <= s < n) and its
// fractional part alpha in [0, 1).  Returns false for a non-finite or absurdly
// large shift; s is then 0 so that every index stays in range.
__device__ __forceinline__ bool split_shift(double sigma, int n, int& s,
                                            double& alpha) {
    if (!(fabs(sigma) < 4.0e18)) {
        s = 0;
        alpha = 0.0;
        return false;
    }
    double fl = floor(sigma);
    alpha = sigma - fl;
    if (alpha >= 1.0) {  // a tiny negative sigma rounds alpha up to one
        fl += 1.0;
        alpha = 0.0;
    }
    long long q = static_cast<long long>(fl) % static_cast<long long>(n);
    if (q < 0) q += n;
    s = static_cast<int>(q);
    return true;
}

// The split for shift derivatives: the exact floor branch.  For sigma in
// [-2^-54, 0) the fraction sigma - floor(sigma) = 1 + sigma rounds to one;
// the forward sweeps move that case to (s + 1, 0), the same output, but a
// derivative must be taken in the cell that holds sigma, so here s stays
// floor(sigma) mod n and alpha = 1 (the derivative from the left of the
// whole cell).  Only an exactly integer sigma gives alpha = 0.
__device__ __forceinline__ bool split_shift_floor(double sigma, int n, int& s,
                                                  double& alpha) {
    if (!(fabs(sigma) < 4.0e18)) {
        s = 0;
        alpha = 0.0;
        return false;
    }
    const double fl = floor(sigma);
    alpha = sigma - fl;
    long long q = static_cast<long long>(fl) % static_cast<long long>(n);
    if (q < 0) q += n;
    s = static_cast<int>(q);
    return true;
}

// v from lane (lane ^ m), m a power of two known at compile time after
// unrolling: within a quad by DPP quad permutations, up to 16 by the
// swizzle crossbar (bit mode: and 0x1F, xor m), 32 by a lane permute.
__device__ __forceinline__ double xor_lanes(double v, int m) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (m) {
        case 1:
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
            break;
        case 2:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
            break;
        case 4:
            lo = __builtin_amdgcn_ds_swizzle(lo, 0x1F | (4 << 10));
            hi = __builtin_amdgcn_ds_swizzle(hi, 0x1F | (4 << 10));
            break;
        case 8:
            lo = __builtin_amdgcn_ds_swizzle(lo, 0x1F | (8 << 10));
            hi = __builtin_amdgcn_ds_swizzle(hi, 0x1F | (8 << 10));
            break;
        case 16:
            lo = __builtin_amdgcn_ds_swizzle(lo, 0x1F | (16 << 10));
            hi = __builtin_amdgcn_ds_swizzle(hi, 0x1F | (16 << 10));
            break;
        default:
            return __shfl_xor(v, m, 64);
    }
    return __hiloint2double(hi, lo);
}

// Reduce-scatter across groups of G lanes (G a power of two, V <= G <= 64):
// on entry every lane holds v[0..V-1]; on return lane l holds the sum over
// its group of the values with index l mod V (valid in lanes whose
// l mod G < V).  V - 1 + log2(G/V) shuffles instead of V full reductions.
template <int V, int G>
__device__ __forceinline__ double group_reduce_scatter(double* v, int lane) {
#pragma unroll
    for (int m = V / 2; m >= 1; m >>= 1) {
        const bool upper = (lane & m) != 0;
#pragma unroll
        for (int j = 0; j < m; ++j) {
            const double keep = upper ? v[j + m] : v[j];
            const double give = upper ? v[j] : v[j + m];
            v[j] = keep + xor_lanes(give, m);
        }
    }
    double r = v[0];
#pragma unroll
    for (int m = V; m < G; m <<= 1) r += xor_lanes(r, m);
    return r;
}

// Store of a sweep output.  Every output element is written once and read
// only by a later kernel, so the store is non-temporal: the line streams out
// to memory during this kernel instead of waiting dirty in the caches, where
// its write-back would fall into the next sweep.
template <typename T>
__device__ __forceinline__ void put_out(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Launch geometry helpers.
inline unsigned blocks_for(int64_t work, int per_block) {
    return static_cast<unsigned>((work + per_block - 1) / per_block);
}

}  // namespace vp
