// Copies of f with the global-memory access patterns of the sweep kernels,
// nothing computed: the bandwidth ceiling of each pattern on this device,
// against which the sweeps' rates are read (a sweep at the copy rate of its
// own pattern loses nothing to its arithmetic or its on-chip work).
//
//   VP_PATTERN_CONTIGUOUS  flat copy, 16 bytes per lane, one round per
//                          thread: the row sweeps (contiguous axis) read and
//                          write their tiles this way.
//   VP_PATTERN_TILES       strided lines in tiles of 64 adjacent lines, a
//                          quarter line per thread (all of its loads in
//                          flight, then its stores): the spline column tiles.
//   VP_PATTERN_SEGMENTS    strided lines by segments of 24 rows, one thread
//                          per (segment, line), blocks in memory order: the
//                          row-segment SLDG sweeps.
//   VP_PATTERN_LINES       strided lines, one thread per whole line walking
//                          it in memory order, 12 loads in flight: the fused
//                          SLDG x2 sweep.
#include <algorithm>
#include <cstdint>

#include "field.hpp"

namespace vp {
namespace {

constexpr int kBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kBlock)
copy_contiguous(const T* __restrict__ in, T* __restrict__ out, int64_t n) {
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    constexpr int kV = 16 / sizeof(T);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t nv = n / kV;
    if (i < nv) {
        const V v = reinterpret_cast<const V*>(in)[i];
        __builtin_nontemporal_store(v, reinterpret_cast<V*>(out) + i);
    }
    // the ragged end, element by element
    if (i < n - nv * kV) out[nv * kV + i] = in[nv * kV + i];
}

// 64 lines per workgroup, thread t: line t % 64, rows of quarter t / 64
template <typename T>
__global__ void __launch_bounds__(kBlock)
copy_tiles(const T* __restrict__ in, T* __restrict__ out, int64_t nlines, int64_t inner,
           int n) {
    constexpr int kL = 64;
    constexpr int kQ = kBlock / kL;
    constexpr int kMax = 24;                      // rows in flight per thread
    const int64_t line = static_cast<int64_t>(blockIdx.x) * kL + threadIdx.x % kL;
    if (line >= nlines) return;
    const int64_t o = line / inner;
    const int64_t k = line - o * inner;
    const int S = (n + kQ - 1) / kQ;
    const int b = min(n, static_cast<int>(threadIdx.x / kL) * S);
    const int e = min(n, b + S);
    const T* __restrict__ src = in + o * n * inner + k;
    T* __restrict__ dst = out + o * n * inner + k;
    // (clamped load indices, so that every load is issued before the first
    // use; only the stores are guarded)
    for (int i0 = b; i0 < e; i0 += kMax) {
        T v[kMax];
#pragma unroll
        for (int u = 0; u < kMax; ++u) v[u] = src[static_cast<int64_t>(min(i0 + u, e - 1)) * inner];
        // (whole chunks store without guards: guarded stores let the compiler
        // move each load next to its store, one load in flight at a time)
        if (i0 + kMax <= e) {
#pragma unroll
            for (int u = 0; u < kMax; ++u)
                __builtin_nontemporal_store(v[u], &dst[static_cast<int64_t>(i0 + u) * inner]);
        } else {
#pragma unroll
            for (int u = 0; u < kMax; ++u)
                if (i0 + u < e) __builtin_nontemporal_store(v[u], &dst[static_cast<int64_t>(i0 + u) * inner]);
        }
    }
}

// segments of kSeg rows; blocks (outer, segment, column block) when inner is
// a multiple of the workgroup, else (line block, segment)
template <typename T, bool BAND>
__global__ void __launch_bounds__(kBlock)
copy_segments(const T* __restrict__ in, T* __restrict__ out, int64_t outer, int64_t inner,
              int n, int nseg) {
    constexpr int kSeg = 24;
    int64_t o, k;
    int q;
    if (BAND) {
        const int64_t nkb = inner / kBlock;
        const int64_t b = blockIdx.x;
        const int64_t kb = b % nkb;
        const int64_t rest = b / nkb;
        q = static_cast<int>(rest % nseg);
        o = rest / nseg;
        k = kb * kBlock + threadIdx.x;
    } else {
        q = static_cast<int>(blockIdx.x % nseg);
        const int64_t line = static_cast<int64_t>(blockIdx.x / nseg) * kBlock + threadIdx.x;
        if (line >= outer * inner) return;
        o = line / inner;
        k = line - o * inner;
    }
    const T* __restrict__ src = in + o * n * inner + k;
    T* __restrict__ dst = out + o * n * inner + k;
    const int r0 = q * kSeg;
    T v[kSeg];
#pragma unroll
    for (int u = 0; u < kSeg; ++u) v[u] = src[static_cast<int64_t>(min(r0 + u, n - 1)) * inner];
    if (r0 + kSeg <= n) {
#pragma unroll
        for (int u = 0; u < kSeg; ++u)
            __builtin_nontemporal_store(v[u], &dst[static_cast<int64_t>(r0 + u) * inner]);
    } else {
#pragma unroll
        for (int u = 0; u < kSeg; ++u)
            if (r0 + u < n) __builtin_nontemporal_store(v[u], &dst[static_cast<int64_t>(r0 + u) * inner]);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
copy_lines(const T* __restrict__ in, T* __restrict__ out, int64_t outer, int64_t inner, int n) {
    constexpr int kU = 12;
    const int64_t line = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (line >= outer * inner) return;
    const int64_t o = line / inner;
    const int64_t k = line - o * inner;
    const T* __restrict__ src = in + o * n * inner + k;
    T* __restrict__ dst = out + o * n * inner + k;
    int r = 0;
    for (; r + kU <= n; r += kU) {
        T v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = src[static_cast<int64_t>(r + u) * inner];
#pragma unroll
        for (int u = 0; u < kU; ++u) __builtin_nontemporal_store(v[u], &dst[static_cast<int64_t>(r + u) * inner]);
    }
    for (; r < n; ++r) __builtin_nontemporal_store(src[static_cast<int64_t>(r) * inner], &dst[static_cast<int64_t>(r) * inner]);
}

template <typename T>
vp_status launch_pattern(int pattern, const int64_t dims[4], int axis, const void* fin,
                         void* fout, int64_t total, hipStream_t st) {
    const T* in = static_cast<const T*>(fin);
    T* out = static_cast<T*>(fout);
    int64_t outer = 1, inner = 1;
    for (int d = 0; d < axis; ++d) outer *= dims[d];
    for (int d = axis + 1; d < 4; ++d) inner *= dims[d];
    const int n = static_cast<int>(dims[axis]);
    int64_t blocks = 0;
    switch (pattern) {
        case VP_PATTERN_CONTIGUOUS:
            blocks = (total / (16 / static_cast<int64_t>(sizeof(T))) + kBlock - 1) / kBlock;
            blocks = std::max<int64_t>(blocks, 1);
            break;
        case VP_PATTERN_TILES:
            blocks = (outer * inner + 63) / 64;
            break;
        case VP_PATTERN_SEGMENTS:
            blocks = inner % kBlock == 0
                         ? outer * ((n + 23) / 24) * (inner / kBlock)
                         : ((outer * inner + kBlock - 1) / kBlock) * ((n + 23) / 24);
            break;
        default:
            blocks = (outer * inner + kBlock - 1) / kBlock;
            break;
    }
    if (blocks >= (int64_t(1) << 31)) return set_error(VP_ERR_UNSUPPORTED, "grid too large");
    const unsigned g = static_cast<unsigned>(blocks);
    switch (pattern) {
        case VP_PATTERN_CONTIGUOUS:
            copy_contiguous<T><<<g, kBlock, 0, st>>>(in, out, total);
            break;
        case VP_PATTERN_TILES:
            copy_tiles<T><<<g, kBlock, 0, st>>>(in, out, outer * inner, inner, n);
            break;
        case VP_PATTERN_SEGMENTS:
            if (inner % kBlock == 0)
                copy_segments<T, true><<<g, kBlock, 0, st>>>(in, out, outer, inner, n, (n + 23) / 24);
            else
                copy_segments<T, false><<<g, kBlock, 0, st>>>(in, out, outer, inner, n, (n + 23) / 24);
            break;
        default:
            copy_lines<T><<<g, kBlock, 0, st>>>(in, out, outer, inner, n);
            break;
    }
    return check_launch("vp_copy_pattern");
}

}  // namespace
}  // namespace vp

extern "C" vp_status vp_copy_pattern(int pattern, vp_dtype dt, const int64_t dims[4], int axis,
                                     const void* f_in, void* f_out, void* stream) {
    using namespace vp;
    clear_error();
    if (pattern < VP_PATTERN_CONTIGUOUS || pattern > VP_PATTERN_LINES)
        return set_error(VP_ERR_ARG, "pattern %d not in %d..%d", pattern, VP_PATTERN_CONTIGUOUS,
                         VP_PATTERN_LINES);
    if (dt != VP_F32 && dt != VP_F64) return set_error(VP_ERR_ARG, "bad dtype %d", (int)dt);
    int64_t total = 0;
    vp_status rc = check_dims(dims, &total);
    if (rc != VP_OK) return rc;
    if (pattern != VP_PATTERN_CONTIGUOUS && (axis < 0 || axis > 2))
        return set_error(VP_ERR_ARG, "axis %d: strided patterns run along axes 0..2", axis);
    if (pattern == VP_PATTERN_TILES && dims[axis] > 4 * 96)
        return set_error(VP_ERR_UNSUPPORTED, "tile pattern: lines of at most 384 points");
    if (!f_in || !f_out) return set_error(VP_ERR_ARG, "NULL pointer argument");
    if ((reinterpret_cast<uintptr_t>(f_in) | reinterpret_cast<uintptr_t>(f_out)) % 16)
        return set_error(VP_ERR_ARG, "f_in and f_out must be 16-byte aligned");
    if (ranges_overlap(f_in, f_out, static_cast<size_t>(total) * dtype_size(dt)))
        return set_error(VP_ERR_ALIAS, "f_in and f_out overlap");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    return dt == VP_F64 ? launch_pattern<double>(pattern, dims, axis, f_in, f_out, total, st)
                        : launch_pattern<float>(pattern, dims, axis, f_in, f_out, total, st);
}
