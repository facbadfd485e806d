// Row-block product: blocks of R consecutive rows of A walk the union of
// their columns, so each B row the block needs is gathered once per block.
// Lane layout as in row split (Sec. 4.1): a slot of 2^g_log2 lanes covers one
// B row (or column tile) with 16-byte accesses; a team of 2^ts_log2 slots owns
// one block and deals the block's union entries to its slots in turn; at the
// end the slots' partial sums are combined by a butterfly and the first slot
// writes the block's C rows.

#include <climits>
#include <type_traits>

#include "common.hpp"
#include "rowblock.hpp"

namespace spmmk {

constexpr uint32_t kColMask = (1u << kRowBlockColBits) - 1;

// Every row, one wavefront per row: column indices must strictly increase.
__global__ __launch_bounds__(kBlock) void k_rowblock_check_sorted(const int* __restrict__ rowptr,
                                                                  const int* __restrict__ colind,
                                                                  int64_t m, int* __restrict__ flag) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; i < m; i += nw) {
        const int lo = rowptr[i], hi = rowptr[i + 1];
        for (int j = lo + lane; j + 1 < hi; j += kWave) bad |= colind[j] >= colind[j + 1];
    }
    if (__ballot(bad) != 0ull && lane == 0) atomicOr(flag, 1);
}

// One thread per block: an R-way merge of the block's rows.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_rowblock_union(const int* __restrict__ rowptr,
                                                           const int* __restrict__ colind,
                                                           int64_t m, int R,
                                                           const int* __restrict__ ub_ptr,
                                                           int* __restrict__ out) {
    const int64_t mb = (m + R - 1) / R;
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= mb) return;
    int p[8], e[8], h[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t row = b * R + r;
        p[r] = e[r] = 0;
        if (r < R && row < m) {
            p[r] = rowptr[row];
            e[r] = rowptr[row + 1];
        }
        h[r] = p[r] < e[r] ? colind[p[r]] : INT_MAX;
    }
    int64_t o = FILL ? ub_ptr[b] : 0;
    int cnt = 0;
    for (;;) {
        int c = INT_MAX;
#pragma unroll
        for (int r = 0; r < 8; ++r) c = min(c, h[r]);
        if (c == INT_MAX) break;
        uint32_t set = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (h[r] == c) {
                set |= 1u << r;
                ++p[r];
                h[r] = p[r] < e[r] ? colind[p[r]] : INT_MAX;
            }
        }
        if (FILL) out[o + cnt] = (int)((uint32_t)c | (set << kRowBlockColBits));
        ++cnt;
    }
    if (!FILL) out[b] = cnt;
}

hipError_t launch_rowblock_check_sorted(const int* rowptr, const int* colind, int64_t m,
                                        int* flag, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    int64_t g = (m + (kBlock / kWave) - 1) / (kBlock / kWave);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_rowblock_check_sorted, dim3((uint32_t)g), dim3(kBlock), 0, st, rowptr,
                       colind, m, flag);
    return hipGetLastError();
}

hipError_t launch_rowblock_union(const int* rowptr, const int* colind, int64_t m, int R,
                                 const int* ub_ptr, int* out, hipStream_t st) {
    if (R < 1 || R > 8) return hipErrorInvalidValue;
    const int64_t mb = (m + R - 1) / R;
    if (mb <= 0) return hipSuccess;
    const dim3 grid((uint32_t)((mb + kBlock - 1) / kBlock));
    if (ub_ptr)
        hipLaunchKernelGGL(k_rowblock_union<true>, grid, dim3(kBlock), 0, st, rowptr, colind, m, R,
                           ub_ptr, out);
    else
        hipLaunchKernelGGL(k_rowblock_union<false>, grid, dim3(kBlock), 0, st, rowptr, colind, m,
                           R, nullptr, out);
    return hipGetLastError();
}

// RB values of one union entry from the staging area.
template <int RB>
__device__ __forceinline__ void read_vals(const float* p, float (&v)[RB]) {
    if constexpr (RB % 4 == 0) {
#pragma unroll
        for (int r = 0; r < RB; r += 4) {
            const f32x4 x = *reinterpret_cast<const f32x4*>(p + r);
            v[r] = x.x; v[r + 1] = x.y; v[r + 2] = x.z; v[r + 3] = x.w;
        }
    } else {
        const f32x2 x = *reinterpret_cast<const f32x2*>(p);
        v[0] = x.x; v[1] = x.y;
    }
}

template <class S, int VEC, int U, int RB, bool SHORT>
__global__ __launch_bounds__(kBlock) void k_rowblock(const int* __restrict__ rowptr,
                                                      const int* __restrict__ ub_ptr,
                                                      const int* __restrict__ words,
                                                      const typename S::T* __restrict__ vals,
                                                      const typename S::T* __restrict__ B,
                                                      float* __restrict__ C, int64_t m, int n,
                                                      int64_t ld, int g_log2, int ts_log2,
                                                      TileOrder ord) {
    // Each team stages its current chunk (two union entries per lane) here;
    // only lanes of the same wavefront read what a lane wrote.
    __shared__ int s_w[2 * kBlock];
    __shared__ __align__(16) float s_v[2 * kBlock * RB];

    const int lane = threadIdx.x & (kWave - 1);
    const int tl_log2 = g_log2 + ts_log2;  // lanes per team (log2), <= 6
    const int TL = 1 << tl_log2;
    const int G = 1 << g_log2;
    const int team_base = lane & ~(TL - 1);
    const int tl = lane & (TL - 1);
    const int slot = tl >> g_log2;
    const int g = tl & (G - 1);
    const int col = blockIdx.y * (VEC << g_log2) + g * VEC;
    const bool col_ok = col < n;
    const int teams_log2 = 8 - tl_log2;  // teams per workgroup of 256 lanes
    const int ebase = (threadIdx.x & ~(TL - 1)) * 2;  // the team's staging entries
    const uint64_t tmask = (TL == kWave ? ~0ull : ((1ull << TL) - 1)) << team_base;
    const uint64_t below = (1ull << lane) - 1;
    const int CH = 2 * TL;
    const int TS = 1 << ts_log2;  // slots per team

    auto b_row = [&](uint32_t c) -> const typename S::T* {
        if constexpr (SHORT) {
            const uint32_t off = __umul24(c, (uint32_t)(ld * sizeof(typename S::T))) +
                                 (uint32_t)(col * sizeof(typename S::T));
            return reinterpret_cast<const typename S::T*>(reinterpret_cast<const char*>(B) + off);
        } else {
            return B + (int64_t)c * ld + col;
        }
    };

    const int64_t mb = (m + RB - 1) / RB;
    const int64_t nblk = (mb + (int64_t(1) << teams_log2) - 1) >> teams_log2;
    for (int64_t t = xcd_remap(blockIdx.x, gridDim.x); t < nblk; t += gridDim.x) {
        const int64_t blk = tile_order(t, ord);
        const int64_t b = (blk << teams_log2) + (threadIdx.x >> tl_log2);
        int u0 = 0, u1 = 0;
        int first[RB];  // first value of each row of the block
#pragma unroll
        for (int r = 0; r < RB; ++r) first[r] = 0;
        if (b < mb) {
            u0 = ub_ptr[b];
            u1 = ub_ptr[b + 1];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int64_t row = b * RB + r;
                first[r] = row < m ? __builtin_nontemporal_load(rowptr + row) : 0;
            }
        }
        float acc[RB][VEC];

        // One walk over the block's union. Unmasked, every row takes
        // value * b for every union entry, with value 0 for a row that lacks
        // the column: exact (0 * b = 0) while b is finite. Masked, a row takes
        // only the entries it holds (the product's definition for any b).
        auto walk = [&](auto masked) {
            constexpr bool MASKED = decltype(masked)::value;
            int cur[RB];  // next unread value of each row
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                cur[r] = first[r];
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[r][e] = 0.f;
            }
            for (int base = u0; base < u1; base += CH) {  // the same for the whole team
                uint32_t w0 = 0, w1 = 0;
                if (base + tl < u1) w0 = (uint32_t)__builtin_nontemporal_load(words + base + tl);
                if (base + TL + tl < u1)
                    w1 = (uint32_t)__builtin_nontemporal_load(words + base + TL + tl);
                // Rank of each entry among the chunk's entries of row r (first
                // member of every lane's pair before the second): its value is
                // row r's next unread value plus that rank.
                float v0[RB], v1[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const bool h0 = (w0 >> (kRowBlockColBits + r)) & 1u;
                    const bool h1 = (w1 >> (kRowBlockColBits + r)) & 1u;
                    const uint64_t m0 = __ballot(h0) & tmask, m1 = __ballot(h1) & tmask;
                    const int n0 = __popcll(m0);
                    v0[r] = h0 ? load_elem(vals + cur[r] + __popcll(m0 & below), S{}) : 0.f;
                    v1[r] = h1 ? load_elem(vals + cur[r] + n0 + __popcll(m1 & below), S{}) : 0.f;
                    cur[r] += n0 + __popcll(m1);
                }
                // Staging is slot-major: entry j (dealt to slot j mod TS) sits at
                // (j mod TS) * 2G + j / TS, so each slot reads its entries from
                // consecutive places (constant offsets within an unrolled step).
                const int p0 = ((tl & (TS - 1)) << (g_log2 + 1)) + (tl >> ts_log2);
                const int p1 = (((TL + tl) & (TS - 1)) << (g_log2 + 1)) + ((TL + tl) >> ts_log2);
                // the previous chunk's reads are done (program order in the wave)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                s_w[ebase + p0] = (int)w0;
                s_w[ebase + p1] = (int)w1;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    s_v[(ebase + p0) * RB + r] = v0[r];
                    s_v[(ebase + p1) * RB + r] = v1[r];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

                const int cnt = min(CH, u1 - base);
                const int nvalid = (cnt - slot + TS - 1) >> ts_log2;  // this slot's entries
                const int* sw = s_w + ebase + (slot << (g_log2 + 1));
                const float* sv = s_v + (ebase + (slot << (g_log2 + 1))) * RB;
                // Whole steps of U entries. From U = 4 on two are in flight: the
                // gathers of step k + U are issued before the adds of step k wait
                // for theirs (the adds keep the entry order); below that one at a
                // time (two steps of two rows hold no more rows in flight than
                // one of four, and cost registers and loop work).
                auto gather = [&](int k0, uint32_t (&w)[U], float (&bv)[U][VEC]) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        w[u] = (uint32_t)sw[k0 + u];
                        load_row<S, VEC>(b_row(w[u] & kColMask), bv[u]);
                    }
                };
                auto add = [&](int k0, const uint32_t (&w)[U], const float (&bv)[U][VEC]) {
                    float v[U][RB];
#pragma unroll
                    for (int u = 0; u < U; ++u) read_vals<RB>(sv + (k0 + u) * RB, v[u]);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            if (!MASKED || ((w[u] >> (kRowBlockColBits + r)) & 1u)) {
#pragma unroll
                                for (int e2 = 0; e2 < VEC; ++e2)
                                    acc[r][e2] = fmaf(v[u][r], bv[u][e2], acc[r][e2]);
                            }
                        }
                    }
                };
                int k = 0;
                if (U < 4) {
                    for (; col_ok && k + U <= nvalid; k += U) {
                        uint32_t w[U];
                        float bv[U][VEC];
                        gather(k, w, bv);
                        add(k, w, bv);
                    }
                } else if (col_ok && nvalid >= U) {
                    uint32_t wA[U], wB[U];
                    float bA[U][VEC], bB[U][VEC];
                    gather(0, wA, bA);
                    for (;;) {
                        const bool nb = k + 2 * U <= nvalid;
                        if (nb) gather(k + U, wB, bB);
                        add(k, wA, bA);
                        k += U;
                        if (!nb) break;
                        const bool na = k + 2 * U <= nvalid;
                        if (na) gather(k + U, wA, bA);
                        add(k, wB, bB);
                        k += U;
                        if (!na) break;
                    }
                }
                // the last, partial step (every step when this lane's columns
                // lie past n)
                for (; k < nvalid; k += U) {
                    uint32_t w[U];
                    float v[U][RB];
                    float bv[U][VEC];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool ok = k + u < nvalid;
                        w[u] = ok ? (uint32_t)sw[k + u] : 0u;
                        if (ok) {
                            read_vals<RB>(sv + (k + u) * RB, v[u]);
                        } else {
#pragma unroll
                            for (int r = 0; r < RB; ++r) v[u][r] = 0.f;
                        }
                        if (ok && col_ok) {
                            load_row<S, VEC>(b_row(w[u] & kColMask), bv[u]);
                        } else {
#pragma unroll
                            for (int e2 = 0; e2 < VEC; ++e2) bv[u][e2] = 0.f;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int r = 0; r < RB; ++r) {
                            if (!MASKED || ((w[u] >> (kRowBlockColBits + r)) & 1u)) {
#pragma unroll
                                for (int e2 = 0; e2 < VEC; ++e2)
                                    acc[r][e2] = fmaf(v[u][r], bv[u][e2], acc[r][e2]);
                            }
                        }
                    }
                }
            }
        };
        walk(std::false_type{});
        // A non-finite b makes every accumulator of its lane non-finite (0 * b
        // is NaN for the rows without the column), and nothing else can turn
        // a finite sum non-finite except overflow: only then walk again, masked.
        bool bad = false;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < VEC; ++e) bad |= !__builtin_isfinite(acc[r][e]);
        if (__ballot(bad) & tmask) walk(std::true_type{});

        // combine the team's slots, then the first slot writes the block's rows
#pragma unroll
        for (int r = 0; r < RB; ++r)
            for (int off = G; off < TL; off <<= 1) {
#pragma unroll
                for (int e2 = 0; e2 < VEC; ++e2) acc[r][e2] += __shfl_xor(acc[r][e2], off, kWave);
            }
        if (slot == 0 && b < mb && col_ok) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int64_t row = b * RB + r;
                if (row < m) store_out<VEC>(C + row * ld + col, acc[r]);
            }
        }
    }
}

template <class S, int VEC, int U, int RB>
static hipError_t rowblock_go(const Shape& s, const ForwardArgs& a, const int* ub_ptr,
                              const int* words, hipStream_t st) {
    const typename S::T* vals = static_cast<const typename S::T*>(a.vals);
    const typename S::T* B = static_cast<const typename S::T*>(a.B);
    const int tl_log2 = s.g_log2 + s.ts_log2;
    const int64_t blocks_per_wg = int64_t(kBlock) >> tl_log2;
    const int64_t mb = (a.m + RB - 1) / RB;
    const int64_t need = (mb + blocks_per_wg - 1) / blocks_per_wg;
    const uint32_t grid = (uint32_t)(need < (1 << 22) ? need : (1 << 22));
    const TileOrder ord = make_tile_order(s.plane_rows, s.strip_rows, blocks_per_wg * RB, need);
    if (s.short_addr)
        hipLaunchKernelGGL((k_rowblock<S, VEC, U, RB, true>), dim3(grid, s.col_tiles), dim3(kBlock),
                           0, st, a.rowptr, ub_ptr, words, vals, B, a.C, a.m, (int)a.n, a.ld,
                           s.g_log2, s.ts_log2, ord);
    else
        hipLaunchKernelGGL((k_rowblock<S, VEC, U, RB, false>), dim3(grid, s.col_tiles),
                           dim3(kBlock), 0, st, a.rowptr, ub_ptr, words, vals, B, a.C, a.m,
                           (int)a.n, a.ld, s.g_log2, s.ts_log2, ord);
    return hipGetLastError();
}

template <class S, int VEC, int RB>
static hipError_t rowblock_u(const Shape& s, const ForwardArgs& a, const int* ub_ptr,
                             const int* words, hipStream_t st) {
    switch (s.unroll) {
    case 1: return rowblock_go<S, VEC, 1, RB>(s, a, ub_ptr, words, st);
    case 2: return rowblock_go<S, VEC, 2, RB>(s, a, ub_ptr, words, st);
    case 4: return rowblock_go<S, VEC, 4, RB>(s, a, ub_ptr, words, st);
    case 8: return rowblock_go<S, VEC, 8, RB>(s, a, ub_ptr, words, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S, int VEC>
static hipError_t rowblock_r(int R, const Shape& s, const ForwardArgs& a, const int* ub_ptr,
                             const int* words, hipStream_t st) {
    switch (R) {
    case 2: return rowblock_u<S, VEC, 2>(s, a, ub_ptr, words, st);
    case 4: return rowblock_u<S, VEC, 4>(s, a, ub_ptr, words, st);
    case 8: return rowblock_u<S, VEC, 8>(s, a, ub_ptr, words, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S>
static hipError_t rowblock_v(int R, const Shape& s, const ForwardArgs& a, const int* ub_ptr,
                             const int* words, hipStream_t st) {
    if (s.vec == S::kVec16) return rowblock_r<S, S::kVec16>(R, s, a, ub_ptr, words, st);
    if (s.vec == 1) return rowblock_r<S, 1>(R, s, a, ub_ptr, words, st);
    return hipErrorInvalidValue;
}

hipError_t launch_rowblock(int dtype, const Shape& s, int R, const ForwardArgs& a,
                           const int* ub_ptr, const int* words, hipStream_t st,
                           hipEvent_t ev_after) {
    if (a.m <= 0 || a.n <= 0) return hipSuccess;
    if (s.g_log2 < 0 || s.ts_log2 < 0 || s.g_log2 + s.ts_log2 > 6) return hipErrorInvalidValue;
    hipError_t e;
    switch (dtype) {
    case 0: e = rowblock_v<F32>(R, s, a, ub_ptr, words, st); break;
    case 1: e = rowblock_v<BF16>(R, s, a, ub_ptr, words, st); break;
    case 2: e = rowblock_v<F16>(R, s, a, ub_ptr, words, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e == hipSuccess && ev_after) e = hipEventRecord(ev_after, st);
    return e;
}

}  // namespace spmmk
