// Device helpers shared by the gfx950 kernels: storage types, 16-byte
// vector access widened to float32, streaming (non-temporal) access for data
// that is read or written once, and XCD-aware workgroup numbering.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmmk {

constexpr int kWave = 64;   // CDNA wavefront width (same as kWaveSize)
constexpr int kXcds = 8;    // MI355X: 8 accelerator dies, each with its own L2

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Storage types of A's values and B. 16-bit types travel as raw bits and are
// widened exactly to float32 (bf16: the upper half of a binary32 pattern;
// fp16: the hardware conversion, exact for every binary16 value).
struct F32 {
    using T = float;
    static constexpr int kVec16 = 4;  // elements per 16-byte access
};
struct BF16 {
    using T = uint16_t;
    static constexpr int kVec16 = 8;
};
struct F16 {
    using T = uint16_t;
    static constexpr int kVec16 = 8;
};

__device__ __forceinline__ float widen_bits(uint32_t h, BF16) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float widen_bits(uint32_t h, F16) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

// One element (A's values).
__device__ __forceinline__ float load_elem(const float* p, F32) { return __builtin_nontemporal_load(p); }
template <class S>
__device__ __forceinline__ float load_elem(const uint16_t* p, S) {
    return widen_bits(__builtin_nontemporal_load(p), S{});
}

// Unpack two 16-bit values held in one dword.
__device__ __forceinline__ void unpack2(uint32_t w, float* o, BF16) {
    o[0] = __uint_as_float(w << 16);
    o[1] = __uint_as_float(w & 0xffff0000u);
}
__device__ __forceinline__ void unpack2(uint32_t w, float* o, F16) {
    f16x2 h = __builtin_bit_cast(f16x2, w);
    o[0] = (float)h.x;
    o[1] = (float)h.y;
}

// VEC consecutive elements of a B row (cached load: B rows are reused).
template <class S, int VEC>
__device__ __forceinline__ void load_row(const typename S::T* p, float (&o)[VEC]);

template <>
__device__ __forceinline__ void load_row<F32, 4>(const float* p, float (&o)[4]) {
    f32x4 v = *reinterpret_cast<const f32x4*>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <>
__device__ __forceinline__ void load_row<F32, 1>(const float* p, float (&o)[1]) { o[0] = *p; }
template <>
__device__ __forceinline__ void load_row<BF16, 8>(const uint16_t* p, float (&o)[8]) {
    u32x4 v = *reinterpret_cast<const u32x4*>(p);
    unpack2(v.x, o + 0, BF16{}); unpack2(v.y, o + 2, BF16{});
    unpack2(v.z, o + 4, BF16{}); unpack2(v.w, o + 6, BF16{});
}
template <>
__device__ __forceinline__ void load_row<BF16, 1>(const uint16_t* p, float (&o)[1]) {
    o[0] = widen_bits(*p, BF16{});
}
template <>
__device__ __forceinline__ void load_row<F16, 8>(const uint16_t* p, float (&o)[8]) {
    u32x4 v = *reinterpret_cast<const u32x4*>(p);
    unpack2(v.x, o + 0, F16{}); unpack2(v.y, o + 2, F16{});
    unpack2(v.z, o + 4, F16{}); unpack2(v.w, o + 6, F16{});
}
template <>
__device__ __forceinline__ void load_row<F16, 1>(const uint16_t* p, float (&o)[1]) {
    o[0] = widen_bits(*p, F16{});
}

// Two entries at once for BF16 storage: acc[e] += v0 * b0[e] + v1 * b1[e]
// for the 8 elements of two raw 16-byte B-row chunks, with the values' BF16
// bits paired as (v0, v1). v_dot2_f32_bf16 forms both (exact) products and
// adds them to acc[e] in one instruction (measured on gfx950 within 1.6 *
// 2^-24 of |v0 b0| + |v1 b1| + |acc|, against 1.0 for one rounding), so a
// pair costs 8 byte permutes and 8 dot products instead of 16 widening
// instructions and 16 multiply-adds.
typedef short bf16x2_bits __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void dot2_pair_bf16(const u32x4& b0, const u32x4& b1,
                                               uint32_t vpair, float (&acc)[8]) {
    const bf16x2_bits v = __builtin_bit_cast(bf16x2_bits, vpair);
    const uint32_t w0[4] = {b0.x, b0.y, b0.z, b0.w};
    const uint32_t w1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        // (b0[2d], b1[2d]) and (b0[2d + 1], b1[2d + 1])
        const uint32_t lo = __builtin_amdgcn_perm(w1[d], w0[d], 0x05040100u);
        const uint32_t hi = __builtin_amdgcn_perm(w1[d], w0[d], 0x07060302u);
        acc[2 * d] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_bits, lo), v,
                                                     acc[2 * d], false);
        acc[2 * d + 1] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_bits, hi), v,
                                                         acc[2 * d + 1], false);
    }
}

// The BF16 bits of two values that came from BF16 storage (exact in float).
__device__ __forceinline__ uint32_t bf16_pair_bits(float v0, float v1) {
    return (__float_as_uint(v0) >> 16) | (__float_as_uint(v1) & 0xFFFF0000u);
}

// VEC float32 results to C (streaming store: C is written once).
template <int VEC>
__device__ __forceinline__ void store_out(float* p, const float (&a)[VEC]) {
    if constexpr (VEC % 4 == 0) {
#pragma unroll
        for (int e = 0; e < VEC; e += 4) {
            f32x4 v = {a[e], a[e + 1], a[e + 2], a[e + 3]};
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p + e));
        }
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) __builtin_nontemporal_store(a[e], p + e);
    }
}

// Read VEC float32 values (carry-out rows, dC rows).
template <int VEC>
__device__ __forceinline__ void load_f32(const float* p, float (&o)[VEC]) {
    if constexpr (VEC % 4 == 0) {
#pragma unroll
        for (int e = 0; e < VEC; e += 4) {
            f32x4 v = *reinterpret_cast<const f32x4*>(p + e);
            o[e] = v.x; o[e + 1] = v.y; o[e + 2] = v.z; o[e + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = p[e];
    }
}

template <int VEC>
__device__ __forceinline__ void store_f32(float* p, const float (&a)[VEC]) {
    if constexpr (VEC % 4 == 0) {
#pragma unroll
        for (int e = 0; e < VEC; e += 4) {
            f32x4 v = {a[e], a[e + 1], a[e + 2], a[e + 3]};
            *reinterpret_cast<f32x4*>(p + e) = v;
        }
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) p[e] = a[e];
    }
}

// Sum over aligned groups of 2^glog2 lanes (glog2 <= 6); every lane of a
// group receives its group's sum. Within 16-lane rows the exchanges are DPP
// moves (quad permutations, then the half-row and row mirrors), which stay
// inside the group at every step; wider groups exchange across rows with
// ds_bpermute. All lanes of a group must be active.
__device__ __forceinline__ float dpp_add(float v, int step) {
    int x = __float_as_int(v);
    switch (step) {
    case 0: x = __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: x = __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: x = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    default: x = __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, false); break; // row_mirror
    }
    return v + __int_as_float(x);
}

__device__ __forceinline__ float group_sum(float v, int glog2) {
    const int in_row = glog2 < 4 ? glog2 : 4;
    for (int s = 0; s < in_row; ++s) v = dpp_add(v, s);
    for (int off = 16; off < (1 << glog2); off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8). Renumber them so that each XCD works on one contiguous range of
// logical tiles: neighbouring rows then share that XCD's L2. A bijection on
// [0, nblocks); correctness never depends on the dispatch order.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
    const uint32_t q = nblocks / kXcds, r = nblocks % kXcds;
    const uint32_t x = bid % kXcds, idx = bid / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + idx;
}

// Processing order of the row tiles (a workgroup's rows) of row split and
// row blocks for matrices whose entries lie near a few diagonals far apart,
// such as the neighbour planes of a 3-D stencil (`plane` tiles apart): strips
// of `strip` consecutive tiles are taken through every plane before the next
// strip, so a B row that three planes use is reused after about three
// strips of rows instead of two whole planes. A bijection on
// [0, planes * plane) (plane a multiple of strip); later tiles keep their
// place; strip == 0 is the row order. Each row's sum is unchanged.
struct TileOrder {
    int64_t plane = 0, strip = 0, planes = 0;
};

__device__ __forceinline__ int64_t tile_order(int64_t t, const TileOrder& o) {
    if (o.strip == 0) return t;
    const int64_t per_strip = o.strip * o.planes;
    if (t >= o.planes * o.plane) return t;
    const int64_t s = t / per_strip, r = t - s * per_strip;
    const int64_t z = r / o.strip, w = r - z * o.strip;
    return z * o.plane + s * o.strip + w;
}

// The order for tiles of `tile_rows` rows out of a plan's plane and strip
// sizes in rows (row order when they are not whole numbers of tiles).
inline TileOrder make_tile_order(int64_t plane_rows, int64_t strip_rows, int64_t tile_rows,
                                 int64_t ntiles) {
    TileOrder o;
    if (strip_rows <= 0 || plane_rows <= 0 || tile_rows <= 0 || plane_rows % tile_rows ||
        strip_rows % tile_rows || plane_rows % strip_rows)
        return o;
    o.plane = plane_rows / tile_rows;
    o.strip = strip_rows / tile_rows;
    o.planes = ntiles / o.plane;
    if (o.planes < 2) o = TileOrder{};
    return o;
}

}  // namespace spmmk
