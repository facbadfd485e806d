// Row-split SpMM (paper Sec. 4.1, Fig. 3) for gfx950 wavefronts.
//
// The paper gives each row of A to one 32-lane warp whose lanes span 32
// columns of B: every lane loads one (column index, value) pair of the row,
// the pairs are broadcast across the warp with shuffles, and for each pair
// the whole warp reads one row of B with a coalesced access, so B and C are
// both touched row-major.
//
// On a 64-lane wavefront the same pattern is kept but the lane groups are
// sized for the actual n:
//   slot  = 2^g_log2 lanes that together cover vec * 2^g_log2 consecutive
//           columns of one B row (16-byte accesses when vec is the 16-byte
//           width), so one B row is a single coalesced request per slot;
//   team  = 2^ts_log2 slots that own one row of A. The slots of a team walk
//           disjoint entries of the row (entry t goes to slot t mod team
//           slots), so short rows still fill the wavefront ("thread per
//           row" granularity of Sec. 4.1 when the team is one slot) and
//           long rows get several B rows in flight per step.
// A team loads up to its lane count of (column, value) pairs with one
// coalesced access per lane and broadcasts them to its slots with ds_bpermute
// (the wave64 form of the paper's shuffle broadcast). Each slot keeps U
// B-row gathers in flight before it accumulates them (the ILP of Table 1).
// At the end of the row the team's slots are combined by a butterfly of
// lane exchanges and the first slot writes the C row once.
//
// The result is fully determined by the launch shape: the accumulation order
// inside a slot and the butterfly order are fixed.

#include "common.hpp"
#include "kernels.hpp"

namespace spmmk {

template <class S, int VEC, int U>
__global__ __launch_bounds__(kBlock) void k_rowsplit(const int* __restrict__ rowptr,
                                                      const int* __restrict__ colind,
                                                      const typename S::T* __restrict__ vals,
                                                      const typename S::T* __restrict__ B,
                                                      float* __restrict__ C, int64_t m, int n,
                                                      int64_t ld, int g_log2, int ts_log2) {
    const int lane = threadIdx.x & (kWave - 1);
    const int tl_log2 = g_log2 + ts_log2;  // lanes per team (log2), <= 6
    const int TL = 1 << tl_log2;
    const int team_base = lane & ~(TL - 1);
    const int tl = lane & (TL - 1);
    const int slot = tl >> g_log2;
    const int g = tl & ((1 << g_log2) - 1);
    const int col = blockIdx.y * (VEC << g_log2) + g * VEC;
    const bool col_ok = col < n;
    const int rpb_log2 = (6 - tl_log2) + 2;  // rows per workgroup: teams per wave * 4 waves
    const int64_t nblk = (m + (int64_t(1) << rpb_log2) - 1) >> rpb_log2;

    for (int64_t blk = xcd_remap(blockIdx.x, gridDim.x); blk < nblk; blk += gridDim.x) {
        const int64_t row = (blk << rpb_log2) + (threadIdx.x >> tl_log2);
        int p0 = 0, p1 = 0;
        if (row < m) {
            p0 = __builtin_nontemporal_load(rowptr + row);
            p1 = __builtin_nontemporal_load(rowptr + row + 1);
        }
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = 0.f;

        for (int base = p0; base < p1; base += TL) {
            const int cnt = min(TL, p1 - base);
            int my_c = 0;
            float my_v = 0.f;
            if (tl < cnt) {
                my_c = __builtin_nontemporal_load(colind + base + tl);
                my_v = load_elem(vals + base + tl, S{});
            }
            const int nsteps = (cnt + (1 << ts_log2) - 1) >> ts_log2;
            for (int s = 0; s < nsteps; s += U) {
                int c[U];
                float v[U];
                bool ok[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int idx = ((s + u) << ts_log2) + slot;  // entry index within the chunk
                    ok[u] = idx < cnt;
                    const int src = team_base + (idx & (TL - 1));
                    c[u] = __shfl(my_c, src, kWave);
                    const float vv = __shfl(my_v, src, kWave);
                    v[u] = ok[u] ? vv : 0.f;
                }
                float b[U][VEC];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (ok[u] && col_ok) {
                        load_row<S, VEC>(B + (int64_t)c[u] * ld + col, b[u]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) b[u][e] = 0.f;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] = fmaf(v[u], b[u][e], acc[e]);
                }
            }
        }
        // Combine the team's slots (lanes G, 2G, ... apart) by a butterfly.
        for (int off = 1 << g_log2; off < TL; off <<= 1) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] += __shfl_xor(acc[e], off, kWave);
        }
        if (slot == 0 && row < m && col_ok) store_out<VEC>(C + row * ld + col, acc);
    }
}

template <class S, int VEC, int U>
static hipError_t go(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                     const void* B, float* C, int64_t m, int64_t n, int64_t ld, hipStream_t st) {
    const int tl_log2 = s.g_log2 + s.ts_log2;
    const int64_t rows_per_block = int64_t(kWave >> tl_log2) * (kBlock / kWave);
    const int64_t need = (m + rows_per_block - 1) / rows_per_block;
    const uint32_t grid = (uint32_t)(need < (1 << 22) ? need : (1 << 22));
    hipLaunchKernelGGL((k_rowsplit<S, VEC, U>), dim3(grid, s.col_tiles), dim3(kBlock), 0, st,
                       rowptr, colind, static_cast<const typename S::T*>(vals),
                       static_cast<const typename S::T*>(B), C, m, (int)n, ld, s.g_log2,
                       s.ts_log2);
    return hipGetLastError();
}

template <class S, int VEC>
static hipError_t go_u(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       hipStream_t st) {
    switch (s.unroll) {
    case 1: return go<S, VEC, 1>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 2: return go<S, VEC, 2>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 4: return go<S, VEC, 4>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 8: return go<S, VEC, 8>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S>
static hipError_t go_v(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       hipStream_t st) {
    if (s.vec == S::kVec16) return go_u<S, S::kVec16>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    if (s.vec == 1) return go_u<S, 1>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    return hipErrorInvalidValue;
}

hipError_t launch_rowsplit(int dtype, const Shape& s, const int* rowptr, const int* colind,
                           const void* vals, const void* B, float* C, int64_t m, int64_t n,
                           int64_t ld, hipStream_t st) {
    if (s.g_log2 < 0 || s.ts_log2 < 0 || s.g_log2 + s.ts_log2 > 6) return hipErrorInvalidValue;
    switch (dtype) {
    case 0: return go_v<F32>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 1: return go_v<BF16>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    case 2: return go_v<F16>(s, rowptr, colind, vals, B, C, m, n, ld, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spmmk
