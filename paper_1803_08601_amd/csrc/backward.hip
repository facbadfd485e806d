// Backward kernels for L = <dC, A B> (not in the paper, whose Sec. 6 names
// A^T products as future work):
//   - the CSR of A^T, built once per structure by a stable LSD radix sort of
//     (column index, entry position) pairs with 8-bit digits. Stability keeps
//     the entries of each column in entry order, i.e. in increasing row of A,
//     so the result is unique and equals a sequential counting sort;
//   - the per-call gather AT_vals[q] = vals[perm[q]] (widened to float32);
//   - SDDMM: dvals[p] = <dC[row(p), :], B[colind[p], :]>.
// dB = A^T dC then runs through the forward kernels on the transposed CSR.

#include "common.hpp"
#include "kernels.hpp"
#include "rowblock.hpp"

namespace spmmk {

constexpr int kRadixMaxBits = 8;                   // digits of at most 8 bits per pass
constexpr int kRadix = 1 << kRadixMaxBits;
constexpr int kSortWaves = kBlock / kWave;         // wavefronts per tile
constexpr int kSortRounds = 8;                     // 64-item rounds per wavefront
constexpr int kSortTile = kBlock * kSortRounds;    // items per tile (one workgroup per tile)

// Index within the tile of round r of a lane: wavefront w owns the
// contiguous quarter [w * 512, (w + 1) * 512) of the tile.
__device__ __forceinline__ int sort_item(int w, int r, int lane) {
    return (w * kSortRounds + r) * kWave + lane;
}

// Per-tile digit counts: hist[d * ntiles + t] for the 2^bits digits.
__global__ __launch_bounds__(kBlock) void k_radix_hist(const int* __restrict__ keys, int64_t n,
                                                        int shift, int bits, int64_t ntiles,
                                                        int* __restrict__ hist) {
    __shared__ int cnt[kRadix];
    const int64_t t = blockIdx.x;
    const int radix = 1 << bits;
    if (threadIdx.x < radix) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = t * kSortTile;
    int key[kSortRounds];  // all loads in flight before the first count
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + r * kBlock + threadIdx.x;
        key[r] = i < n ? keys[i] : -1;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
        if (key[r] >= 0) atomicAdd(&cnt[(key[r] >> shift) & (radix - 1)], 1);
    __syncthreads();
    if (threadIdx.x < radix) hist[(int64_t)threadIdx.x * ntiles + t] = cnt[threadIdx.x];
}

// Device-wide exclusive scan of int32 in place, in three launches: per-chunk
// sums, a scan of the chunk sums by one workgroup, and the scan of each chunk
// from its offset. A chunk is kScanPer consecutive items per thread of a
// 256-thread workgroup.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kBlock * kScanPer;

__device__ __forceinline__ int block_exclusive_scan(int v, int* s_wave, int* total) {
    // inclusive scan within the wavefront, then across the four wavefronts
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) s_wave[w] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kBlock / kWave; ++q) {
        const int sw = s_wave[q];
        before += q < w ? sw : 0;
        all += sw;
    }
    *total = all;
    return before + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_sums(const int* __restrict__ a, int64_t len,
                                                       int* __restrict__ sums) {
    __shared__ int s_wave[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    int v = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        const int64_t i = base + q * kBlock + threadIdx.x;  // coalesced; order is irrelevant
        if (i < len) v += a[i];
    }
    int total;
    (void)block_exclusive_scan(v, s_wave, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of `len` ints in place by one workgroup of 1024 threads:
// each thread scans a contiguous chunk, chunk sums are scanned in LDS. Used
// for the chunk sums (a few thousand at most for any int32 entry count).
__global__ __launch_bounds__(1024) void k_scan_single(int* __restrict__ a, int64_t len) {
    __shared__ int sums[1024];
    const int64_t per = (len + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < len ? lo + per : len;
    int s = 0;
    for (int64_t i = lo; i < hi; ++i) s += a[i];
    sums[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
        const int v = threadIdx.x >= off ? sums[threadIdx.x - off] : 0;
        __syncthreads();
        sums[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x ? sums[threadIdx.x - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_chunks(int* __restrict__ a, int64_t len,
                                                         const int* __restrict__ offs) {
    __shared__ int s_wave[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = base + q < len ? a[base + q] : 0;
        sum += v[q];
    }
    int total;
    int run = offs[blockIdx.x] + block_exclusive_scan(sum, s_wave, &total);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < len) a[base + q] = run;
        run += v[q];
    }
}

int64_t scan_chunks(int64_t len) { return (len + kScanChunk - 1) / kScanChunk; }

static hipError_t exclusive_scan(int* a, int64_t len, int* sums, hipStream_t st) {
    const int64_t nb = scan_chunks(len);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_sums, dim3((uint32_t)nb), dim3(kBlock), 0, st, a, len, sums);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, sums, nb);
    hipLaunchKernelGGL(k_scan_chunks, dim3((uint32_t)nb), dim3(kBlock), 0, st, a, len, sums);
    return hipGetLastError();
}

hipError_t exclusive_scan_i32(int* a, int64_t len, int* sums, hipStream_t st) {
    return exclusive_scan(a, len, sums, st);
}

// Stable scatter of one digit pass, carrying two value arrays (entry
// position and row of A). One workgroup per tile; each wavefront loads its
// quarter of the tile into registers and counts its digits in LDS. The
// counts give every (wavefront, digit) pair its first slot in the tile sorted
// by digit; a wavefront then ranks its items round by round (lanes with equal
// digits find each other with one ballot per digit bit and take ranks in lane
// order), which sorts the tile in LDS stably. The sorted tile is written out
// in order: consecutive slots of one digit go to consecutive global
// positions, so the stores of a digit's run coalesce instead of each item
// being a separate store to a random place.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const int* __restrict__ keys_in,
                                                           const int* __restrict__ vals_in,
                                                           const int* __restrict__ rows_in,
                                                           int* __restrict__ keys_out,
                                                           int* __restrict__ vals_out,
                                                           int* __restrict__ rows_out, int64_t n,
                                                           int shift, int bits, int64_t ntiles,
                                                           const int* __restrict__ offs) {
    __shared__ int s_key[kSortTile], s_val[kSortTile], s_row[kSortTile];
    __shared__ int cursor[kSortWaves][kRadix];  // next slot of (wavefront, digit)
    __shared__ int delta[kRadix];  // global position of a digit's slot minus the slot
    __shared__ int s_wave[kSortWaves];
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int radix = 1 << bits, mask = radix - 1;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = t * kSortTile;
    const int tile_n = (int)(n - base < kSortTile ? n - base : kSortTile);
    int key[kSortRounds], val[kSortRounds], row[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const int j = sort_item(w, r, lane);
        const bool ok = j < tile_n;
        key[r] = ok ? keys_in[base + j] : 0;
        val[r] = ok ? vals_in[base + j] : 0;
        row[r] = ok ? rows_in[base + j] : 0;
    }
    for (int d = lane; d < radix; d += kWave) cursor[w][d] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
        if (sort_item(w, r, lane) < tile_n) atomicAdd(&cursor[w][(key[r] >> shift) & mask], 1);
    __syncthreads();
    {
        // thread d owns digit d: the tile's count, its exclusive scan over the
        // digits, then the first slot of each wavefront's run of that digit
        const int d = threadIdx.x;
        int c[kSortWaves];
        int total_d = 0;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) {
            c[q] = d < radix ? cursor[q][d] : 0;
            total_d += c[q];
        }
        int all;
        const int start = block_exclusive_scan(total_d, s_wave, &all);
        __syncthreads();
        if (d < radix) {
            int run = start;
#pragma unroll
            for (int q = 0; q < kSortWaves; ++q) {
                cursor[q][d] = run;
                run += c[q];
            }
            delta[d] = offs[(int64_t)d * ntiles + t] - start;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const bool ok = sort_item(w, r, lane) < tile_n;
        const int d = (key[r] >> shift) & mask;
        uint64_t match = __ballot(ok);
        for (int b = 0; b < bits; ++b) {
            const uint64_t ones = __ballot(ok && ((d >> b) & 1));
            match &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int slot = ok ? cursor[w][d] + __popcll(match & lt) : 0;
        __syncthreads();
        if (ok) {
            s_key[slot] = key[r];
            s_val[slot] = val[r];
            s_row[slot] = row[r];
            // the highest lane of each digit group advances that digit's cursor
            if ((match >> lane) == 1ull) cursor[w][d] = slot + 1;
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < tile_n; j += kBlock) {
        const int kk = s_key[j];
        const int pos = delta[(kk >> shift) & mask] + j;
        keys_out[pos] = kk;
        vals_out[pos] = s_val[j];
        rows_out[pos] = s_row[j];
    }
}

__global__ __launch_bounds__(kBlock) void k_iota(int* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int)i;
}

// AT_rowptr[c] = number of sorted keys below c, for c = 0..k.
__global__ __launch_bounds__(kBlock) void k_lower_bounds(const int* __restrict__ sorted, int64_t n,
                                                          int64_t k, int* __restrict__ out) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= k;
         c += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sorted[mid] < c) lo = mid + 1; else hi = mid;
        }
        out[c] = (int)lo;
    }
}

// rows[p] = the row of A holding entry p: one wavefront per row, its lanes
// writing the row's entries 64 at a time.
__global__ __launch_bounds__(kBlock) void k_row_ids(const int* __restrict__ rowptr, int64_t m,
                                                     int* __restrict__ rows) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < m;
         i += nw) {
        const int lo = rowptr[i], hi = rowptr[i + 1];
        for (int j = lo + lane; j < hi; j += kWave) rows[j] = (int)i;
    }
}

template <class S>
__global__ __launch_bounds__(kBlock) void k_gather_widen(const typename S::T* __restrict__ vals,
                                                          const int* __restrict__ perm, int64_t n,
                                                          float* __restrict__ out) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        float v[1];
        load_row<S, 1>(vals + perm[q], v);
        __builtin_nontemporal_store(v[0], out + q);
    }
}

static uint32_t grid_for(int64_t n, int64_t cap = 65536) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t transpose_build(const int* rowptr, const int* colind, int64_t m, int64_t k,
                           int64_t nnz, int* at_rowptr, int* at_colind, int* perm,
                           int* tmp_keys0, int* tmp_keys1, int* tmp_vals1, int* tmp_rows0,
                           int* scratch, hipStream_t st) {
    // keys: column indices; values: entry positions (end in `perm`) and rows
    // of A (end in `at_colind`)
    hipError_t e = hipMemcpyAsync(tmp_keys0, colind, sizeof(int) * nnz, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(nnz)), dim3(kBlock), 0, st, perm, nnz);
    hipLaunchKernelGGL(k_row_ids, dim3(grid_for(m * kWave)), dim3(kBlock), 0, st, rowptr, m,
                       tmp_rows0);
    int bits = 0;
    while (bits < 31 && (int64_t(1) << bits) < k) ++bits;
    // as few passes as digits of at most 8 bits allow, the bits spread evenly:
    // narrower digits mean longer runs per digit in a tile, so fewer stores
    const int passes = (bits + kRadixMaxBits - 1) / kRadixMaxBits;
    const int64_t ntiles = (nnz + kSortTile - 1) / kSortTile;
    int* hist = scratch;
    int* sums = scratch + ntiles * kRadix;
    int *kin = tmp_keys0, *kout = tmp_keys1, *vin = perm, *vout = tmp_vals1;
    int *rin = tmp_rows0, *rout = at_colind;
    int shift = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const int pbits = (bits - shift + (passes - ps) - 1) / (passes - ps);
        const int64_t hlen = ntiles << pbits;
        hipLaunchKernelGGL(k_radix_hist, dim3((uint32_t)ntiles), dim3(kBlock), 0, st, kin, nnz,
                           shift, pbits, ntiles, hist);
        e = exclusive_scan(hist, hlen, sums, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((uint32_t)ntiles), dim3(kBlock), 0, st, kin, vin,
                           rin, kout, vout, rout, nnz, shift, pbits, ntiles, hist);
        shift += pbits;
        int* tk = kin; kin = kout; kout = tk;
        int* tv = vin; vin = vout; vout = tv;
        int* tr = rin; rin = rout; rout = tr;
    }
    if (vin != perm) {
        e = hipMemcpyAsync(perm, vin, sizeof(int) * nnz, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    if (rin != at_colind) {
        e = hipMemcpyAsync(at_colind, rin, sizeof(int) * nnz, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_lower_bounds, dim3(grid_for(k + 1)), dim3(kBlock), 0, st, kin, nnz, k,
                       at_rowptr);
    return hipGetLastError();
}

int64_t transpose_scratch_len(int64_t nnz) {
    const int64_t hlen = ((nnz + kSortTile - 1) / kSortTile) * kRadix;
    return hlen + scan_chunks(hlen);
}

hipError_t launch_gather_widen(int dtype, const void* vals, const int* perm, int64_t n,
                               float* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    switch (dtype) {
    case 0: hipLaunchKernelGGL(k_gather_widen<F32>, dim3(grid_for(n)), dim3(kBlock), 0, st,
                               static_cast<const float*>(vals), perm, n, out); break;
    case 1: hipLaunchKernelGGL(k_gather_widen<BF16>, dim3(grid_for(n)), dim3(kBlock), 0, st,
                               static_cast<const uint16_t*>(vals), perm, n, out); break;
    case 2: hipLaunchKernelGGL(k_gather_widen<F16>, dim3(grid_for(n)), dim3(kBlock), 0, st,
                               static_cast<const uint16_t*>(vals), perm, n, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ SDDMM
//
// dvals[p] = <dC[row(p), :], B[colind[p], :]> on the merge pieces of the plan
// (the Phase 1 partition of Algorithm 1), so that the work per workgroup is
// the same whatever the row lengths: a 159k-entry row costs no more per entry
// than a short one. A workgroup stages its piece's row ends and column indices
// in LDS; its wavefronts split the piece evenly with the diagonal search on
// the LDS copy, and the slots of a wavefront (2^g_log2 lanes covering one
// column tile of a row) take its entries interleaved, finding each entry's
// row among the staged row ends. For U entries at a time a slot gathers the
// B row chunks, forms the partial dot products with the dC row chunk (kept
// in registers while the row lasts when the row fits one column tile), and
// sums its lanes with DPP row exchanges; the wavefront then writes the step's
// consecutive dvals with one store (lane g of a slot writing its g-th sum).
// No entry depends on another, so there is no carry-out.
template <class S, int VEC, int U, bool ONE_TILE>
__global__ __launch_bounds__(kBlock) void k_sddmm(const int* __restrict__ rowptr,
                                                   const int* __restrict__ colind,
                                                   const float* __restrict__ dC,
                                                   const typename S::T* __restrict__ B,
                                                   float* __restrict__ dvals, int n, int64_t ld,
                                                   int g_log2, int col_tiles,
                                                   const int* __restrict__ coords, int W) {
    extern __shared__ __align__(16) unsigned char smem[];
    int* s_col = reinterpret_cast<int*>(smem);  // [W]
    int* s_rowend = s_col + W;                  // [W] local row ends
    const int tile = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int i0 = coords[2 * tile], j0 = coords[2 * tile + 1];
    const int i1 = coords[2 * tile + 2], j1 = coords[2 * tile + 3];
    const int nr = i1 - i0, nj = j1 - j0;
    for (int t = threadIdx.x; t < nr; t += kBlock)
        s_rowend[t] = __builtin_nontemporal_load(rowptr + i0 + 1 + t) - j0;
    for (int t = threadIdx.x; t < nj; t += kBlock) s_col[t] = __builtin_nontemporal_load(colind + j0 + t);
    __syncthreads();

    const int G = 1 << g_log2;
    const int g = threadIdx.x & (G - 1);
    // The piece is split among the workgroup's wavefronts by the diagonal
    // search; inside a wavefront its SPW slots take interleaved entries (slot
    // s: entries s, s + SPW, ...), so they walk the same rows together.
    const int NW = kBlock / kWave;
    const int w = threadIdx.x / kWave;
    const int SPW = kWave >> g_log2;
    const int s = (threadIdx.x & (kWave - 1)) >> g_log2;
    const int items = nr + nj;
    const int ipw = (items + NW - 1) / NW;
    const int d0 = min(w * ipw, items), d1 = min(d0 + ipw, items);
    auto search = [&](int d) {
        int lo = max(0, d - nj), hi = min(d, nr);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_rowend[mid] + mid < d) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    int r = search(d0);
    const int js = d0 - r;
    const int je = d1 - search(d1);
    const int span = VEC << g_log2;
    // With one column tile the dC chunk of the current row stays in
    // registers and is reloaded when the walk reaches a new row; the slots of
    // a wavefront reach row ends together, so that branch is nearly uniform.
    int have = -1;
    float dh[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) dh[e] = 0.f;
    for (int jb = js + s; jb < je; jb += SPW * U) {
        int rr[U], c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = jb + u * SPW;
            if (j < je) {
                while (r < nr && s_rowend[r] <= j) ++r;  // rows that end before entry j
                c[u] = s_col[j];
            } else {
                c[u] = 0;
            }
            rr[u] = r;
        }
        float part[U];
        if constexpr (ONE_TILE) {
            const int col = g * VEC;
            const bool col_ok = col < n;
            float b[U][VEC];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (jb + u * SPW < je && col_ok) {
                    load_row<S, VEC>(B + (int64_t)c[u] * ld + col, b[u]);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) b[u][e] = 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (rr[u] != have) {
                    if (col_ok && jb + u * SPW < je)
                        load_f32<VEC>(dC + (int64_t)(i0 + rr[u]) * ld + col, dh);
                    have = rr[u];
                }
                part[u] = 0.f;
#pragma unroll
                for (int e = 0; e < VEC; ++e) part[u] = fmaf(dh[e], b[u][e], part[u]);
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) part[u] = 0.f;
            for (int t = 0; t < col_tiles; ++t) {
                const int col = t * span + g * VEC;
                const bool col_ok = col < n;
                float b[U][VEC], d[U][VEC];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (jb + u * SPW < je && col_ok) {
                        load_row<S, VEC>(B + (int64_t)c[u] * ld + col, b[u]);
                        load_f32<VEC>(dC + (int64_t)(i0 + rr[u]) * ld + col, d[u]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) b[u][e] = d[u][e] = 0.f;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) part[u] = fmaf(d[u][e], b[u][e], part[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) part[u] = group_sum(part[u], g_log2);
        if ((1 << g_log2) >= U) {
            // Every lane of a slot holds its U sums: lane g < U writes the
            // g-th (entry jb + g SPW), so one store covers the wavefront's
            // SPW * U consecutive entries of this step.
            float out = part[0];
#pragma unroll
            for (int u = 1; u < U; ++u)
                if (g == u) out = part[u];
            const int j = jb + g * SPW;
            if (g < U && j < je) __builtin_nontemporal_store(out, dvals + j0 + j);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (g == 0 && jb + u * SPW < je)
                    __builtin_nontemporal_store(part[u], dvals + j0 + jb + u * SPW);
        }
    }
}

// ------------------------------------------------------------------ A^T dC by scatter
//
// dB = A^T dC straight from A's CSR, without the transpose: every entry p of
// row i adds vals[p] * dC[i, :] into row colind[p] of dB with float atomic
// adds. The work is split on the same diagonal merge pieces as SDDMM (the
// LDS-staged row ends give each entry's row), so long rows cost no more per
// entry. A slot covers 4 * 2^g_log2 columns with its lanes interleaved
// (column base + e * 2^g_log2 + lane), so each atomic instruction of a slot
// updates consecutive floats of one dB row. The slot keeps the dC chunk of
// its current row in registers and reloads it when the walk reaches a new
// row. The order in which additions reach an element depends on timing:
// results are not bitwise repeatable (integer-valued data is exact).
constexpr int kScatterVec = 4;

__global__ __launch_bounds__(kBlock) void k_zero_rows(float* __restrict__ a, int64_t rows, int n,
                                                       int64_t ld) {
    const int64_t total = rows * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x)
        a[(q / n) * ld + q % n] = 0.f;
}

hipError_t launch_zero_f32(float* a, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_rows, dim3(grid_for(count)), dim3(kBlock), 0, st, a, count, 1,
                       int64_t(1));
    return hipGetLastError();
}

template <class S>
__global__ __launch_bounds__(kBlock) void k_scatter_t(const int* __restrict__ rowptr,
                                                       const int* __restrict__ colind,
                                                       const typename S::T* __restrict__ vals,
                                                       const float* __restrict__ dC,
                                                       float* __restrict__ dB, int n, int64_t ld,
                                                       int g_log2, int col_tiles,
                                                       const int* __restrict__ coords, int W) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* s_val = reinterpret_cast<float*>(smem);       // [W]
    int* s_col = reinterpret_cast<int*>(s_val + W);      // [W]
    int* s_rowend = s_col + W;                           // [W] local row ends
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
    __syncthreads();

    const int G = 1 << g_log2;
    const int NS = kBlock >> g_log2;
    const int slot = threadIdx.x >> g_log2;
    const int g = threadIdx.x & (G - 1);
    const int items = nr + nj;
    const int ips = (items + NS - 1) / NS;
    const int d0 = min(slot * ips, items), d1 = min(d0 + ips, items);
    auto search = [&](int d) {
        int lo = max(0, d - nj), hi = min(d, nr);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_rowend[mid] + mid < d) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    const int rs = search(d0);
    const int js = d0 - rs;
    const int je = d1 - search(d1);
    const int span = kScatterVec << g_log2;
    for (int t = 0; t < col_tiles; ++t) {
        const int base = t * span + g;
        int r = rs, have = -1;
        float d[kScatterVec];
        for (int j = js; j < je; ++j) {
            while (r < nr && s_rowend[r] <= j) ++r;  // rows that end before entry j
            if (r != have) {
#pragma unroll
                for (int e = 0; e < kScatterVec; ++e) {
                    const int col = base + e * G;
                    d[e] = col < n ? dC[(int64_t)(i0 + r) * ld + col] : 0.f;
                }
                have = r;
            }
            const float v = s_val[j];
            float* dst = dB + (int64_t)s_col[j] * ld;
#pragma unroll
            for (int e = 0; e < kScatterVec; ++e) {
                const int col = base + e * G;
                if (col < n) unsafeAtomicAdd(dst + col, v * d[e]);
            }
        }
    }
}

hipError_t launch_scatter_t(int dtype, const int* rowptr, const int* colind, const void* vals,
                            const float* dC, float* dB, int64_t k, int64_t n, int64_t ld,
                            const int* coords, int64_t P, int W, hipStream_t st) {
    if (k <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_rows, dim3(grid_for(k * n)), dim3(kBlock), 0, st, dB, k, (int)n, ld);
    if (P <= 0) return hipGetLastError();
    int g_log2 = 0;
    while (g_log2 < 6 && (int64_t(kScatterVec) << g_log2) < n) ++g_log2;
    const int span = kScatterVec << g_log2;
    const int col_tiles = (int)((n + span - 1) / span);
    const size_t lds = sizeof(int) * 3 * (size_t)W;
#define SCATTER_LAUNCH(SS, T)                                                                  \
    hipLaunchKernelGGL((k_scatter_t<SS>), dim3((uint32_t)P), dim3(kBlock), lds, st, rowptr,     \
                       colind, static_cast<const T*>(vals), dC, dB, (int)n, ld, g_log2,        \
                       col_tiles, coords, W)
    switch (dtype) {
    case 0: SCATTER_LAUNCH(F32, float); break;
    case 1: SCATTER_LAUNCH(BF16, uint16_t); break;
    case 2: SCATTER_LAUNCH(F16, uint16_t); break;
    default: return hipErrorInvalidValue;
    }
#undef SCATTER_LAUNCH
    return hipGetLastError();
}

template <class S, int VEC>
static hipError_t sddmm_go(int unroll, int g_log2, int col_tiles, const int* rowptr,
                           const int* colind, const float* dC, const void* B, float* dvals,
                           int64_t n, int64_t ld, const int* coords, int64_t P, int W,
                           hipStream_t st) {
    const size_t lds = sizeof(int) * 2 * (size_t)W;
    const typename S::T* Bp = static_cast<const typename S::T*>(B);
#define SDDMM_LAUNCH(UU)                                                                         \
    if (col_tiles == 1)                                                                          \
        hipLaunchKernelGGL((k_sddmm<S, VEC, UU, true>), dim3((uint32_t)P), dim3(kBlock), lds,   \
                           st, rowptr, colind, dC, Bp, dvals, (int)n, ld, g_log2, col_tiles,    \
                           coords, W);                                                           \
    else                                                                                         \
        hipLaunchKernelGGL((k_sddmm<S, VEC, UU, false>), dim3((uint32_t)P), dim3(kBlock), lds,  \
                           st, rowptr, colind, dC, Bp, dvals, (int)n, ld, g_log2, col_tiles,    \
                           coords, W)
    switch (unroll) {
    case 1: SDDMM_LAUNCH(1); break;
    case 2: SDDMM_LAUNCH(2); break;
    case 4: SDDMM_LAUNCH(4); break;
    case 8: SDDMM_LAUNCH(8); break;
    default: return hipErrorInvalidValue;
    }
#undef SDDMM_LAUNCH
    return hipGetLastError();
}

hipError_t launch_sddmm(int dtype, int vec, int unroll, int g_log2, int col_tiles,
                        const int* rowptr, const int* colind, const float* dC, const void* B,
                        float* dvals, int64_t n, int64_t ld, const int* coords, int64_t P, int W,
                        hipStream_t st) {
    if (P <= 0) return hipSuccess;
    switch (dtype) {
    case 0:
        if (vec == 4) return sddmm_go<F32, 4>(unroll, g_log2, col_tiles, rowptr, colind, dC, B, dvals, n, ld, coords, P, W, st);
        return sddmm_go<F32, 1>(unroll, g_log2, col_tiles, rowptr, colind, dC, B, dvals, n, ld, coords, P, W, st);
    case 1:
        if (vec == 8) return sddmm_go<BF16, 8>(unroll, g_log2, col_tiles, rowptr, colind, dC, B, dvals, n, ld, coords, P, W, st);
        return sddmm_go<BF16, 1>(unroll, g_log2, col_tiles, rowptr, colind, dC, B, dvals, n, ld, coords, P, W, st);
    case 2:
        if (vec == 8) return sddmm_go<F16, 8>(unroll, g_log2, col_tiles, rowptr, colind, dC, B, dvals, n, ld, coords, P, W, st);
        return sddmm_go<F16, 1>(unroll, g_log2, col_tiles, rowptr, colind, dC, B, dvals, n, ld, coords, P, W, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spmmk
