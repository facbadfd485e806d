// Merge-based SpMM (paper Sec. 4.2, Algorithm 1) for gfx950.
//
// Phase 1 (PARTITIONSPMM): the merge of the row ends a[i] = rowptr[i+1] with
// the entry indices b[j] = j is cut into pieces of W items (rows + entries)
// by a 2-D binary search on the diagonals d_p = min(p W, m + nnz) (the merge
// path of Sec. 4). At state (i, j) the next item is the end of row i when
// a[i] <= j, otherwise entry j, which belongs to row i. Coordinates depend
// only on A's structure, so a plan computes them once.
//
// Phase 2 (one workgroup per piece): the piece's row ends, column indices and
// values are staged in LDS with coalesced loads (GLOBALTOSHARED). The piece
// is split again, evenly, among the workgroup's slots (2^g_log2 lanes
// covering one B row of the column tile) by the same diagonal search on the
// LDS copy. Each slot walks its items in merge order: for an entry it
// gathers the B row (U gathers in flight) and accumulates value * row; for a
// row end it emits the running sum. A row whose entries all lie inside the
// slot is written straight to C. The first row a slot finishes may have
// started in earlier slots: it goes through LDS and is combined with the
// carry-outs of those slots in slot order (the segmented reduction of
// REDUCETOGLOBALSPMM). The sum for the row still open at the end of the piece
// is the piece's carry-out (row id plus n floats).
//
// Phase 3 (FIXCARRYOUT): rows that cross piece boundaries receive the
// carry-outs of the pieces before the one that finished them, added in piece
// order by a separate pass, since workgroups cannot wait for each other.
//
// Every row is written exactly once by Phase 2 and updated at most once by
// Phase 3; all sums run in an order fixed by (W, slot width), so results are
// deterministic for a plan.

#include <limits.h>

#include "common.hpp"
#include "kernels.hpp"

namespace spmmk {

__global__ __launch_bounds__(kBlock) void k_merge_partition(const int* __restrict__ rowptr,
                                                             int64_t m, int64_t nnz, int W,
                                                             int64_t P, int* __restrict__ coords) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    const int64_t total = m + nnz;
    const int64_t d = p * W < total ? p * W : total;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < m ? d : m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rowptr[mid + 1] + mid < d)
            lo = mid + 1;
        else
            hi = mid;
    }
    coords[2 * p] = (int)lo;
    coords[2 * p + 1] = (int)(d - lo);
}

template <class S, int VEC, int U>
__global__ __launch_bounds__(kBlock) void k_merge(const int* __restrict__ rowptr,
                                                   const int* __restrict__ colind,
                                                   const typename S::T* __restrict__ vals,
                                                   const typename S::T* __restrict__ B,
                                                   float* __restrict__ C, int m, int n, int64_t ld,
                                                   int g_log2, const int* __restrict__ coords,
                                                   int W, float* __restrict__ carry_vals,
                                                   int* __restrict__ carry_rows) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* s_head = reinterpret_cast<float*>(smem);     // [kBlock * VEC] first finished row per slot
    float* s_carry = s_head + kBlock * VEC;              // [kBlock * VEC] open row per slot
    float* s_val = s_carry + kBlock * VEC;               // [W]
    int* s_col = reinterpret_cast<int*>(s_val + W);      // [W]
    int* s_rowend = s_col + W;                           // [W] local row ends
    int* s_head_row = s_rowend + W;                      // [kBlock]
    int* s_carry_row = s_head_row + kBlock;              // [kBlock]

    const int tile = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = coords[2 * tile], j0 = coords[2 * tile + 1];
    const int i1 = coords[2 * tile + 2], j1 = coords[2 * tile + 3];
    const int nr = i1 - i0, nj = j1 - j0;

    for (int t = threadIdx.x; t < nr; t += kBlock)
        s_rowend[t] = __builtin_nontemporal_load(rowptr + i0 + 1 + t) - j0;
    for (int t = threadIdx.x; t < nj; t += kBlock) {
        s_col[t] = __builtin_nontemporal_load(colind + j0 + t);
        s_val[t] = load_elem(vals + j0 + t, S{});
    }
    const int G = 1 << g_log2;
    const int NS = kBlock >> g_log2;
    const int slot = threadIdx.x >> g_log2;
    const int g = threadIdx.x & (G - 1);
    if (g == 0) s_head_row[slot] = -1;
    __syncthreads();

    const int col = blockIdx.y * (VEC << g_log2) + g * VEC;
    const bool col_ok = col < n;
    const int items = nr + nj;
    const int ips = (items + NS - 1) / NS;
    const int d0 = min(slot * ips, items), d1 = min(d0 + ips, items);
    auto search = [&](int d) {
        int lo = max(0, d - nj), hi = min(d, nr);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_rowend[mid] + mid < d)
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    };
    const int rs = search(d0), js = d0 - rs;
    const int re = search(d1), je = d1 - re;

    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
    int r = rs;
    int rend = r < nr ? s_rowend[r] : INT_MAX;
    auto emit = [&]() {
        if (r == rs) {
            store_f32<VEC>(s_head + threadIdx.x * VEC, acc);
            if (g == 0) s_head_row[slot] = r;
        } else if (col_ok) {
            store_out<VEC>(C + (int64_t)(i0 + r) * ld + col, acc);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
        ++r;
        rend = r < nr ? s_rowend[r] : INT_MAX;
    };

    for (int jb = js; jb < je; jb += U) {
        int c[U];
        float v[U];
        float b[U][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = jb + u < je;
            c[u] = ok ? s_col[jb + u] : 0;
            v[u] = ok ? s_val[jb + u] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (jb + u < je && col_ok) {
                load_row<S, VEC>(B + (int64_t)c[u] * ld + col, b[u]);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) b[u][e] = 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = jb + u;
            if (j < je) {
                while (rend <= j) emit();
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = fmaf(v[u], b[u][e], acc[e]);
            }
        }
    }
    while (r < re) emit();
    store_f32<VEC>(s_carry + threadIdx.x * VEC, acc);
    if (g == 0) s_carry_row[slot] = re;
    __syncthreads();

    // First finished row of each slot: add the carry-outs of the earlier
    // slots that ended inside the same row, in slot order.
    const int h = s_head_row[slot];
    if (h >= 0 && col_ok) {
        int s0 = slot;
        while (s0 > 0 && s_carry_row[s0 - 1] == h) --s0;
        float tot[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) tot[e] = 0.f;
        for (int q = s0; q < slot; ++q) {
            float t[VEC];
            load_f32<VEC>(s_carry + (q * G + g) * VEC, t);
#pragma unroll
            for (int e = 0; e < VEC; ++e) tot[e] += t[e];
        }
        float hv[VEC];
        load_f32<VEC>(s_head + threadIdx.x * VEC, hv);
#pragma unroll
        for (int e = 0; e < VEC; ++e) tot[e] += hv[e];
        store_out<VEC>(C + (int64_t)(i0 + h) * ld + col, tot);
    }

    // Carry-out of the piece: the row open at its end (row i1), if the piece
    // holds any of its entries.
    if (slot == NS - 1) {
        bool open = false;
        if (i1 < m) {
            const int start_local = nr > 0 ? s_rowend[nr - 1] : rowptr[i0] - j0;
            open = nj > start_local;
        }
        if (open && col_ok) {
            int s0 = NS - 1;
            while (s0 > 0 && s_carry_row[s0 - 1] == nr) --s0;
            float tot[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) tot[e] = 0.f;
            for (int q = s0; q < NS; ++q) {
                float t[VEC];
                load_f32<VEC>(s_carry + (q * G + g) * VEC, t);
#pragma unroll
                for (int e = 0; e < VEC; ++e) tot[e] += t[e];
            }
            store_f32<VEC>(carry_vals + (int64_t)tile * n + col, tot);
        }
        if (g == 0 && blockIdx.y == 0) carry_rows[tile] = open ? i1 : -1;
    }
}

// Phase 3: one wavefront per piece; the first piece of every run of pieces
// that carry into the same row adds the run's carry-outs (in piece order) to
// that row of C.
__global__ __launch_bounds__(kWave) void k_merge_fixup(float* __restrict__ C, int64_t ld, int n,
                                                        const float* __restrict__ carry_vals,
                                                        const int* __restrict__ carry_rows,
                                                        int64_t P) {
    const int64_t p = blockIdx.x;
    const int r = carry_rows[p];
    if (r < 0) return;
    if (p > 0 && carry_rows[p - 1] == r) return;
    int64_t q_end = p + 1;
    while (q_end < P && carry_rows[q_end] == r) ++q_end;
    for (int c = threadIdx.x; c < n; c += kWave) {
        float s = 0.f;
        for (int64_t q = p; q < q_end; ++q) s += carry_vals[q * n + c];
        C[(int64_t)r * ld + c] += s;
    }
}

size_t merge_lds_bytes(int dtype, const Shape& s) {
    (void)dtype;
    return (size_t)2 * kBlock * s.vec * sizeof(float) + (size_t)3 * s.W * sizeof(int) +
           (size_t)2 * kBlock * sizeof(int);
}

hipError_t launch_merge_partition(const int* rowptr, int64_t m, int64_t nnz, int W, int64_t P,
                                  int* coords, hipStream_t st) {
    const int64_t threads = P + 1;
    const uint32_t grid = (uint32_t)((threads + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_merge_partition, dim3(grid), dim3(kBlock), 0, st, rowptr, m, nnz, W, P,
                       coords);
    return hipGetLastError();
}

template <class S, int VEC, int U>
static hipError_t go(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                     const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                     const int* coords, int64_t P, float* carry_vals, int* carry_rows,
                     hipStream_t st) {
    const size_t lds = merge_lds_bytes(0, s);
    hipLaunchKernelGGL((k_merge<S, VEC, U>), dim3((uint32_t)P, s.col_tiles), dim3(kBlock), lds,
                       st, rowptr, colind, static_cast<const typename S::T*>(vals),
                       static_cast<const typename S::T*>(B), C, (int)m, (int)n, ld, s.g_log2,
                       coords, s.W, carry_vals, carry_rows);
    return hipGetLastError();
}

template <class S, int VEC>
static hipError_t go_u(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       const int* coords, int64_t P, float* cv, int* cr, hipStream_t st) {
    switch (s.unroll) {
    case 1: return go<S, VEC, 1>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    case 2: return go<S, VEC, 2>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    case 4: return go<S, VEC, 4>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    case 8: return go<S, VEC, 8>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S>
static hipError_t go_v(const Shape& s, const int* rowptr, const int* colind, const void* vals,
                       const void* B, float* C, int64_t m, int64_t n, int64_t ld,
                       const int* coords, int64_t P, float* cv, int* cr, hipStream_t st) {
    if (s.vec == S::kVec16)
        return go_u<S, S::kVec16>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    if (s.vec == 1) return go_u<S, 1>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, cv, cr, st);
    return hipErrorInvalidValue;
}

hipError_t launch_merge(int dtype, const Shape& s, const int* rowptr, const int* colind,
                        const void* vals, const void* B, float* C, int64_t m, int64_t n,
                        int64_t ld, const int* coords, int64_t P, float* carry_vals,
                        int* carry_rows, hipStream_t st) {
    if (P <= 0) return hipSuccess;
    if (s.g_log2 < 0 || s.g_log2 > 6 || s.W < 1) return hipErrorInvalidValue;
    switch (dtype) {
    case 0: return go_v<F32>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, carry_vals, carry_rows, st);
    case 1: return go_v<BF16>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, carry_vals, carry_rows, st);
    case 2: return go_v<F16>(s, rowptr, colind, vals, B, C, m, n, ld, coords, P, carry_vals, carry_rows, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge_fixup(float* C, int64_t ld, int64_t n, const float* carry_vals,
                              const int* carry_rows, int64_t P, hipStream_t st) {
    if (P <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_fixup, dim3((uint32_t)P), dim3(kWave), 0, st, C, ld, (int)n,
                       carry_vals, carry_rows, P);
    return hipGetLastError();
}

// ------------------------------------------------------------------ statistics

__global__ __launch_bounds__(kBlock) void k_row_stats(const int* __restrict__ rowptr, int64_t m,
                                                       int* __restrict__ stats) {
    int mx = 0, nlong = 0, bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int len = rowptr[i + 1] - rowptr[i];
        mx = max(mx, len);
        nlong += len >= 1024;
        bad |= len < 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && rowptr[0] != 0) bad = 1;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off, kWave));
        nlong += __shfl_xor(nlong, off, kWave);
        bad |= __shfl_xor(bad, off, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMax(&stats[0], mx);
        atomicAdd(&stats[1], nlong);
        if (bad) atomicAnd(&stats[2], 0);
    }
}

hipError_t launch_row_stats(const int* rowptr, int64_t m, int* stats, hipStream_t st) {
    int64_t blocks = (m + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_row_stats, dim3((uint32_t)blocks), dim3(kBlock), 0, st, rowptr, m, stats);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_check_cols(const int* __restrict__ colind, int64_t nnz,
                                                        int64_t k, int* __restrict__ flags) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = colind[i];
        bad |= (c < 0) | ((int64_t)c >= k);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) bad |= __shfl_xor(bad, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicOr(&flags[0], 1);
}

hipError_t launch_check_cols(const int* colind, int64_t nnz, int64_t k, int* flags,
                             hipStream_t st) {
    int64_t blocks = (nnz + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_check_cols, dim3((uint32_t)blocks), dim3(kBlock), 0, st, colind, nnz, k,
                       flags);
    return hipGetLastError();
}

}  // namespace spmmk
