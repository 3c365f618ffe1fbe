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
            double a = v[j], b = v[j + m];
            // (register operands for the selects: a select of two array
            // elements would otherwise become one load at a lane-dependent
            // index, a compare-and-select chain over all V elements)
            asm("" : "+v"(a), "+v"(b));
            const double keep = upper ? b : a;
            const double give = upper ? a : b;
            v[j] = keep + xor_lanes(give, m);
        }
    }
    double r = v[0];
#pragma unroll
    for (int m = V; m < G; m <<= 1) r += xor_lanes(r, m);
    return r;
}

// x + y after a half-wave exchange: with H = 32, lanes 0..31 return
// x(l) + x(l + 32) and lanes 32..63 return y(l - 32) + y(l); with H = 16 the
// same within each pair of 16-lane rows (even rows: x, odd rows: y).  One
// v_permlane{32,16}_swap per 32-bit half (gfx950): the swap exchanges the
// upper half of x with the lower half of y, so no lane has to select.
template <int H>
__device__ __forceinline__ double swap_add(double x, double y) {
    const unsigned xl = static_cast<unsigned>(__double2loint(x));
    const unsigned xh = static_cast<unsigned>(__double2hiint(x));
    const unsigned yl = static_cast<unsigned>(__double2loint(y));
    const unsigned yh = static_cast<unsigned>(__double2hiint(y));
    static_assert(H == 32 || H == 16, "half-wave or half-row pair exchange");
    if constexpr (H == 32) {
        const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        return __hiloint2double(static_cast<int>(hi[0]), static_cast<int>(lo[0])) +
               __hiloint2double(static_cast<int>(hi[1]), static_cast<int>(lo[1]));
    } else {
        const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        return __hiloint2double(static_cast<int>(hi[0]), static_cast<int>(lo[0])) +
               __hiloint2double(static_cast<int>(hi[1]), static_cast<int>(lo[1]));
    }
}

// v from lane (l + n) mod 16 of the same 16-lane row (DPP row rotation).
template <int n>
__device__ __forceinline__ double row_ror(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x120 + n, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x120 + n, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes of a wavefront of four values per lane: on return
// every lane of row r (lanes 16 r .. 16 r + 15) holds the sum of a_r.  Two
// half exchanges leave each lane one partial sum over four lanes
// {l, l ^ 16, l ^ 32, l ^ 48}, added across its row by four rotations.
__device__ __forceinline__ double wave_sum4_rows(double a0, double a1, double a2, double a3) {
    const double b0 = swap_add<32>(a0, a2);   // lanes < 32: a0, else a2
    const double b1 = swap_add<32>(a1, a3);   // lanes < 32: a1, else a3
    double c = swap_add<16>(b0, b1);          // row r: a_r
    c += row_ror<8>(c);
    c += row_ror<4>(c);
    c += row_ror<2>(c);
    c += row_ror<1>(c);
    return c;
}

// Raw buffer access for kernels whose addresses are a uniform base plus a
// 32-bit per-lane byte offset: the descriptor and the uniform part (soff)
// live in scalar registers, so a load or store costs no vector address
// arithmetic.  `bytes` (< 4 GB) bounds the offsets: the hardware returns 0
// for a load beyond it and drops such a store.  Word 3 of the descriptor:
// 32-bit data format, the value for gfx9 buffers.
// The caller's base and size are the same in every lane; the readfirstlane
// says so to the compiler, which otherwise may keep the descriptor in vector
// registers and loop over the lanes at every access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, uint32_t bytes) {
    const uint64_t a = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
    void* const p = reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(voff),
                                                                          static_cast<int>(soff), 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(voff),
                                                                          static_cast<int>(soff), 0));
}
// (non-temporal, as `put_out` below: cache policy bit 1)
template <typename T>
__device__ __forceinline__ void buffer_store_nt(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                uint32_t soff) {
    if constexpr (sizeof(T) == 8) {
        using U = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, static_cast<int>(voff),
                                              static_cast<int>(soff), 2);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r,
                                              static_cast<int>(voff), static_cast<int>(soff), 2);
    }
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
