// Device-side tile functions of the SpMM kernels, shared by the single-product
// kernels and the batched persistent kernel.
#pragma once

#include <limits.h>

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace spmmk {

// ---------------------------------------------------------------- semirings
// The product over a semiring (Sec. 1 names SpMM as one instance of the
// GraphBLAS matrix product on a semiring): acc = acc (+) (v (x) b), partial
// results combined with (+), rows without entries give the identity. The
// ordinary product is PlusTimes (fused multiply-add). Entries a lane skips
// must leave acc unchanged: PlusTimes feeds them as 0 * 0, the others skip.
struct PlusTimes {
    static constexpr bool kZeroTermIsNeutral = true;
    __device__ static float zero() { return 0.f; }
    __device__ static float mac(float acc, float v, float b) { return fmaf(v, b, acc); }
    __device__ static float add(float x, float y) { return x + y; }
};
struct MinPlus {
    static constexpr bool kZeroTermIsNeutral = false;
    __device__ static float zero() { return __builtin_inff(); }
    __device__ static float mac(float acc, float v, float b) { return fminf(acc, v + b); }
    __device__ static float add(float x, float y) { return fminf(x, y); }
};
struct MaxPlus {
    static constexpr bool kZeroTermIsNeutral = false;
    __device__ static float zero() { return -__builtin_inff(); }
    __device__ static float mac(float acc, float v, float b) { return fmaxf(acc, v + b); }
    __device__ static float add(float x, float y) { return fmaxf(x, y); }
};
struct MaxTimes {
    static constexpr bool kZeroTermIsNeutral = false;
    __device__ static float zero() { return -__builtin_inff(); }
    __device__ static float mac(float acc, float v, float b) { return fmaxf(acc, v * b); }
    __device__ static float add(float x, float y) { return fmaxf(x, y); }
};

// ---------------------------------------------------------------- row split
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
// A team loads up to twice its lane count of (column, value) pairs with two
// coalesced accesses per lane and broadcasts them to its slots with
// ds_bpermute (the wave64 form of the paper's shuffle broadcast); the next
// chunk of pairs is loaded while the current one is processed. Each slot keeps U
// B-row gathers in flight before it accumulates them (the ILP of Table 1).
// At the end of the row the team's slots are combined by a butterfly of
// lane exchanges and the first slot writes the C row once.
//
// The result is fully determined by the launch shape: the accumulation order
// inside a slot and the butterfly order are fixed.

// One workgroup's rows of the row-split product (rows blk * R .. blk * R + R - 1
// with R = rows per workgroup) for column tile `coltile`. Row i's entries
// run from rowbeg[i] to rowend[i] (the whole row: rowptr and rowptr + 1);
// with `accumulate` the row's sum is added to C instead of written.
template <class S, int VEC, int U, class R = PlusTimes, bool SHORT = false>
__device__ __forceinline__ void rowsplit_block(const int* __restrict__ rowbeg,
                                               const int* __restrict__ rowend,
                                               const int* __restrict__ colind,
                                               const typename S::T* __restrict__ vals,
                                               const typename S::T* __restrict__ B,
                                               float* __restrict__ C, int64_t m, int n, int64_t ld,
                                               int g_log2, int ts_log2, int64_t blk, int coltile,
                                               bool accumulate) {
    const int lane = threadIdx.x & (kWave - 1);
    const int tl_log2 = g_log2 + ts_log2;  // lanes per team (log2), <= 6
    const int TL = 1 << tl_log2;
    const int team_base = lane & ~(TL - 1);
    const int tl = lane & (TL - 1);
    const int slot = tl >> g_log2;
    const int g = tl & ((1 << g_log2) - 1);
    const int col = coltile * (VEC << g_log2) + g * VEC;
    const bool col_ok = col < n;
    const int rpb_log2 = (6 - tl_log2) + 2;  // rows per workgroup: teams per wave * 4 waves

    const int64_t row = (blk << rpb_log2) + (threadIdx.x >> tl_log2);
    int p0 = 0, p1 = 0;
    if (row < m) {
        p0 = __builtin_nontemporal_load(rowbeg + row);
        p1 = __builtin_nontemporal_load(rowend + row);
    }
    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = R::zero();

    // A chunk is 2 * TL entries: lane tl holds entries tl and tl + TL. The
    // next chunk's pairs are loaded while the current one is processed.
    const int CH = 2 << tl_log2;
    int cc0 = 0, cc1 = 0;
    float cv0 = 0.f, cv1 = 0.f;
    auto load_pair = [&](int base, int& c0, float& v0, int& c1, float& v1) {
        const int t0 = base + tl, t1 = base + TL + tl;
        c0 = 0; v0 = 0.f; c1 = 0; v1 = 0.f;
        if (t0 < p1) {
            c0 = __builtin_nontemporal_load(colind + t0);
            v0 = load_elem(vals + t0, S{});
        }
        if (t1 < p1) {
            c1 = __builtin_nontemporal_load(colind + t1);
            v1 = load_elem(vals + t1, S{});
        }
    };
    if (p0 < p1) load_pair(p0, cc0, cv0, cc1, cv1);
    const int TS = 1 << ts_log2;
    const int G = 1 << g_log2;
    // Byte address of this lane's first pair in the team (ds_bpermute takes
    // a byte lane address); step k of a chunk reads entry (k << ts_log2) +
    // slot, held by lane team_base + that entry (first pair member, k < G) or
    // that entry - TL (second member).
    const int my4 = (team_base + slot) << 2;
    auto b_row = [&](int c) -> const typename S::T* {
        if constexpr (SHORT) {
            // B spans < 4 GiB and < 2^24 rows of < 2^24 bytes: a 24-bit
            // multiply and a 32-bit offset from B's base in scalar registers
            const uint32_t off = __umul24((uint32_t)c, (uint32_t)(ld * sizeof(typename S::T))) +
                                 (uint32_t)(col * sizeof(typename S::T));
            return reinterpret_cast<const typename S::T*>(reinterpret_cast<const char*>(B) + off);
        } else {
            return B + (int64_t)c * ld + col;
        }
    };
    for (int base = p0; base < p1; base += CH) {
        const int cnt = min(CH, p1 - base);
        const bool more = base + CH < p1;  // uniform within the team
        int nc0 = 0, nc1 = 0;
        float nv0 = 0.f, nv1 = 0.f;
        if (more) load_pair(base + CH, nc0, nv0, nc1, nv1);
        const int nsteps = (cnt + TS - 1) >> ts_log2;       // the same for the team
        const int nvalid = (cnt - slot + TS - 1) >> ts_log2;  // steps holding this slot's entries
        // Steps [kbeg, kend) read pair member (creg, vreg); sub4 shifts the
        // second member's entries back to lanes 0 .. TL - 1.
        auto run = [&](int kbeg, int kend, int creg, float vreg, int sub4) {
            const int lim = min(kend, nvalid);
            for (int k = kbeg; k < kend; k += U) {
                int c[U];
                float v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // every lane of the team takes part in both permutes
                    const int addr = my4 + (((k + u) << ts_log2) << 2) - sub4;
                    c[u] = __builtin_amdgcn_ds_bpermute(addr, creg);
                    v[u] = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(vreg)));
                }
                if (col_ok && k + U <= lim) {
                    // a whole block of this slot's entries: no per-entry checks
                    if constexpr (std::is_same<S, BF16>::value && VEC == 8 &&
                                  std::is_same<R, PlusTimes>::value && U % 2 == 0) {
                        // BF16: two entries at a time by paired dot products
                        u32x4 raw[U];
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            raw[u] = *reinterpret_cast<const u32x4*>(b_row(c[u]));
#pragma unroll
                        for (int u = 0; u < U; u += 2)
                            dot2_pair_bf16(raw[u], raw[u + 1], bf16_pair_bits(v[u], v[u + 1]),
                                           acc);
                    } else {
                        float b[U][VEC];
#pragma unroll
                        for (int u = 0; u < U; ++u) load_row<S, VEC>(b_row(c[u]), b[u]);
#pragma unroll
                        for (int u = 0; u < U; ++u) {
#pragma unroll
                            for (int e = 0; e < VEC; ++e) acc[e] = R::mac(acc[e], v[u], b[u][e]);
                        }
                    }
                } else {
                    bool ok[U];
                    float b[U][VEC];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        ok[u] = k + u < lim;
                        if (!ok[u]) v[u] = 0.f;
                        if (ok[u] && col_ok) {
                            load_row<S, VEC>(b_row(c[u]), b[u]);
                        } else {
#pragma unroll
                            for (int e = 0; e < VEC; ++e) b[u][e] = 0.f;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (R::kZeroTermIsNeutral || ok[u]) {
#pragma unroll
                            for (int e = 0; e < VEC; ++e) acc[e] = R::mac(acc[e], v[u], b[u][e]);
                        }
                    }
                }
            }
        };
        run(0, min(G, nsteps), cc0, cv0, 0);
        if (nsteps > G) run(G, nsteps, cc1, cv1, TL << 2);
        cc0 = nc0; cc1 = nc1; cv0 = nv0; cv1 = nv1;
    }
    // Combine the team's slots (lanes G, 2G, ... apart) by a butterfly.
    for (int off = 1 << g_log2; off < TL; off <<= 1) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = R::add(acc[e], __shfl_xor(acc[e], off, kWave));
    }
    if (slot == 0 && row < m && col_ok) {
        if (accumulate) {
            // earlier panels' sum first, then this panel's
            float old[VEC];
            load_f32<VEC>(C + row * ld + col, old);
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] = R::add(old[e], acc[e]);
        }
        store_out<VEC>(C + row * ld + col, acc);
    }
}

// ---------------------------------------------------------------- merge-based
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
//
// Nonzero split (Sec. 4, scheme (a); nz != 0): the same walk over pieces cut
// by nonzero count instead of by diagonal. A piece then holds W nonzeros and
// any number of row ends; the row ends are staged in LDS when at most W of
// them fall in the piece and read from global memory otherwise, and the
// piece is split among its slots by nonzeros as well (a 1-D search on the
// row ends), so a run of empty rows is emitted by one slot.

// Phase 2 for merge piece `tile` and column tile `coltile`; smem holds
// merge_lds_bytes() of LDS. Contains workgroup barriers: every thread of the
// workgroup must call it with the same arguments. NZ selects nonzero-split
// pieces.
template <class S, int VEC, int U, class R = PlusTimes, bool NZ = false>
__device__ __forceinline__ void merge_tile(const int* __restrict__ rowptr,
                                           const int* __restrict__ colind,
                                           const typename S::T* __restrict__ vals,
                                           const typename S::T* __restrict__ B,
                                           float* __restrict__ C, int m, int n, int64_t ld,
                                           int g_log2, const int* __restrict__ coords, int W,
                                           float* __restrict__ carry_vals,
                                           int* __restrict__ carry_rows, int tile, int coltile,
                                           unsigned char* smem) {
    float* s_head = reinterpret_cast<float*>(smem);     // [kBlock * VEC] first finished row per slot
    float* s_carry = s_head + kBlock * VEC;              // [kBlock * VEC] open row per slot
    float* s_val = s_carry + kBlock * VEC;               // [W]
    int* s_col = reinterpret_cast<int*>(s_val + W);      // [W]
    int* s_rowend = s_col + W;                           // [W] local row ends
    int* s_head_row = s_rowend + W;                      // [kBlock]
    int* s_carry_row = s_head_row + kBlock;              // [kBlock]

    const int i0 = coords[2 * tile], j0 = coords[2 * tile + 1];
    const int i1 = coords[2 * tile + 2], j1 = coords[2 * tile + 3];
    const int nr = i1 - i0, nj = j1 - j0;
    // Row ends local to the piece. A diagonal piece has nr + nj <= W items;
    // a nonzero-split piece may hold more than W row ends (empty rows).
    const bool rows_lds = !NZ || nr <= W;
    auto rowend = [&](int r) -> int {
        if constexpr (!NZ) return s_rowend[r];
        return rows_lds ? s_rowend[r] : rowptr[i0 + 1 + r] - j0;
    };

    if (rows_lds)
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

    const int col = coltile * (VEC << g_log2) + g * VEC;
    const bool col_ok = col < n;
    int rs, js, re, je;
    if constexpr (!NZ) {
        // even split of the piece's items by the diagonal search
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
        rs = search(d0); js = d0 - rs;
        re = search(d1); je = d1 - re;
    } else {
        // even split of the piece's nonzeros; a slot starts after the row
        // ends at or before its first nonzero (the first slot at the piece
        // start, which takes the piece's leading empty rows)
        const int eps = (nj + NS - 1) / NS;
        js = min(slot * eps, nj);
        je = min(js + eps, nj);
        auto ended_by = [&](int j) {
            int lo = 0, hi = nr;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (rowend(mid) <= j)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            return lo;
        };
        rs = slot == 0 ? 0 : ended_by(js);
        re = ended_by(je);
    }

    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = R::zero();
    int r = rs;
    int rend = r < nr ? rowend(r) : INT_MAX;
    auto emit = [&]() {
        if (r == rs) {
            store_f32<VEC>(s_head + threadIdx.x * VEC, acc);
            if (g == 0) s_head_row[slot] = r;
        } else if (col_ok) {
            store_out<VEC>(C + (int64_t)(i0 + r) * ld + col, acc);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = R::zero();
        ++r;
        rend = r < nr ? rowend(r) : INT_MAX;
    };

    constexpr bool kPairs = std::is_same<S, BF16>::value && VEC == 8 &&
                            std::is_same<R, PlusTimes>::value && U % 2 == 0;
    for (int jb = js; jb < je; jb += U) {
        int c[U];
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = jb + u < je;
            c[u] = ok ? s_col[jb + u] : 0;
            v[u] = ok ? s_val[jb + u] : 0.f;
        }
        if constexpr (kPairs) {
            // BF16: raw 16-byte chunks; two entries of one row at a time by
            // paired dot products, an entry alone where a row ends between
            u32x4 raw[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (jb + u < je && col_ok)
                    raw[u] = *reinterpret_cast<const u32x4*>(B + (int64_t)c[u] * ld + col);
                else
                    raw[u] = u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int u = 0; u < U; u += 2) {
                const int j = jb + u;
                if (j < je) {
                    while (rend <= j) emit();
                    if (j + 1 < je && rend > j + 1) {
                        dot2_pair_bf16(raw[u], raw[u + 1], bf16_pair_bits(v[u], v[u + 1]), acc);
                    } else {
                        float b[VEC];
                        unpack2(raw[u].x, b + 0, BF16{}); unpack2(raw[u].y, b + 2, BF16{});
                        unpack2(raw[u].z, b + 4, BF16{}); unpack2(raw[u].w, b + 6, BF16{});
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] = fmaf(v[u], b[e], acc[e]);
                        if (j + 1 < je) {
                            while (rend <= j + 1) emit();
                            unpack2(raw[u + 1].x, b + 0, BF16{}); unpack2(raw[u + 1].y, b + 2, BF16{});
                            unpack2(raw[u + 1].z, b + 4, BF16{}); unpack2(raw[u + 1].w, b + 6, BF16{});
#pragma unroll
                            for (int e = 0; e < VEC; ++e) acc[e] = fmaf(v[u + 1], b[e], acc[e]);
                        }
                    }
                }
            }
        } else {
            float b[U][VEC];
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
                    for (int e = 0; e < VEC; ++e) acc[e] = R::mac(acc[e], v[u], b[u][e]);
                }
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
        for (int e = 0; e < VEC; ++e) tot[e] = R::zero();
        for (int q = s0; q < slot; ++q) {
            float t[VEC];
            load_f32<VEC>(s_carry + (q * G + g) * VEC, t);
#pragma unroll
            for (int e = 0; e < VEC; ++e) tot[e] = R::add(tot[e], t[e]);
        }
        float hv[VEC];
        load_f32<VEC>(s_head + threadIdx.x * VEC, hv);
#pragma unroll
        for (int e = 0; e < VEC; ++e) tot[e] = R::add(tot[e], hv[e]);
        store_out<VEC>(C + (int64_t)(i0 + h) * ld + col, tot);
    }

    // Carry-out of the piece: the row open at its end (row i1), if the piece
    // holds any of its entries.
    if (slot == NS - 1) {
        bool open = false;
        if (i1 < m) {
            const int start_local = nr > 0 ? rowend(nr - 1) : rowptr[i0] - j0;
            open = nj > start_local;
        }
        if (open && col_ok) {
            int s0 = NS - 1;
            while (s0 > 0 && s_carry_row[s0 - 1] == nr) --s0;
            float tot[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) tot[e] = R::zero();
            for (int q = s0; q < NS; ++q) {
                float t[VEC];
                load_f32<VEC>(s_carry + (q * G + g) * VEC, t);
#pragma unroll
                for (int e = 0; e < VEC; ++e) tot[e] = R::add(tot[e], t[e]);
            }
            store_f32<VEC>(carry_vals + (int64_t)tile * n + col, tot);
        }
        if (g == 0 && coltile == 0) carry_rows[tile] = open ? i1 : -1;
    }
}

// Phase 3 for piece p: the first piece of every run of pieces that carry
// into the same row adds the run's carry-outs (in piece order) to that row of
// C. One wavefront per piece (lane = its lane index). The row ids of the
// piece and its neighbours are loaded together; a long run (a row spanning
// many pieces) is measured 64 pieces per round with a ballot and summed with
// eight carry-outs in flight, so its cost grows by one memory round trip per
// 64 pieces and per 8 pieces instead of two per piece.
constexpr int kFixupWaves = kBlock / kWave;  // pieces per fix-up workgroup
constexpr int kFixupBatch = 8;               // carry-outs in flight per lane

template <class R = PlusTimes>
__device__ __forceinline__ void merge_fixup_piece(float* __restrict__ C, int64_t ld, int n,
                                                  const float* __restrict__ carry_vals,
                                                  const int* __restrict__ carry_rows, int64_t P,
                                                  int64_t p, int lane) {
    if (p >= P) return;
    const int r = carry_rows[p];
    const int rprev = carry_rows[p > 0 ? p - 1 : 0];
    const int rnext = carry_rows[p + 1 < P ? p + 1 : p];
    if (r < 0 || (p > 0 && rprev == r)) return;
    int64_t q_end = p + 1;
    if (p + 1 < P && rnext == r) {
        q_end = p + 2;
        for (;;) {  // first piece at or after q_end that carries elsewhere
            const int64_t q = q_end + lane;
            const uint64_t other = __ballot(q >= P || carry_rows[q] != r);
            if (other) {
                q_end += __ffsll((unsigned long long)other) - 1;
                break;
            }
            q_end += kWave;
        }
    }
    for (int c = lane; c < n; c += kWave) {
        float s = R::zero();
        for (int64_t q = p; q < q_end; q += kFixupBatch) {
            float t[kFixupBatch];
#pragma unroll
            for (int u = 0; u < kFixupBatch; ++u)
                t[u] = q + u < q_end ? carry_vals[(q + u) * n + c] : 0.f;
#pragma unroll
            for (int u = 0; u < kFixupBatch; ++u)
                if (q + u < q_end) s = R::add(s, t[u]);
        }
        C[(int64_t)r * ld + c] = R::add(C[(int64_t)r * ld + c], s);
    }
}

// ---------------------------------------------------------------- kernels

template <class S, int VEC, int U, class R, bool SHORT>
__global__ __launch_bounds__(kBlock) void k_rowsplit(const int* __restrict__ rowbeg,
                                                      const int* __restrict__ rowend,
                                                      const int* __restrict__ colind,
                                                      const typename S::T* __restrict__ vals,
                                                      const typename S::T* __restrict__ B,
                                                      float* __restrict__ C, int64_t m, int n,
                                                      int64_t ld, int g_log2, int ts_log2,
                                                      TileOrder ord, int accumulate) {
    const int rpb_log2 = (6 - g_log2 - ts_log2) + 2;
    const int64_t nblk = (m + (int64_t(1) << rpb_log2) - 1) >> rpb_log2;
    for (int64_t t = xcd_remap(blockIdx.x, gridDim.x); t < nblk; t += gridDim.x)
        rowsplit_block<S, VEC, U, R, SHORT>(rowbeg, rowend, colind, vals, B, C, m, n, ld,
                                            g_log2, ts_log2, tile_order(t, ord), blockIdx.y,
                                            accumulate != 0);
}

template <class S, int VEC, int U, class R, bool NZ>
__global__ __launch_bounds__(kBlock) void k_merge(const int* __restrict__ rowptr,
                                                   const int* __restrict__ colind,
                                                   const typename S::T* __restrict__ vals,
                                                   const typename S::T* __restrict__ B,
                                                   float* __restrict__ C, int m, int n, int64_t ld,
                                                   int g_log2, const int* __restrict__ coords,
                                                   int W, float* __restrict__ carry_vals,
                                                   int* __restrict__ carry_rows) {
    extern __shared__ __align__(16) unsigned char smem[];
    merge_tile<S, VEC, U, R, NZ>(rowptr, colind, vals, B, C, m, n, ld, g_log2, coords, W,
                                 carry_vals, carry_rows, (int)xcd_remap(blockIdx.x, gridDim.x),
                                 blockIdx.y, smem);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_merge_fixup(float* __restrict__ C, int64_t ld, int n,
                                                         const float* __restrict__ carry_vals,
                                                         const int* __restrict__ carry_rows,
                                                         int64_t P) {
    const int64_t p = (int64_t)blockIdx.x * kFixupWaves + threadIdx.x / kWave;
    merge_fixup_piece<R>(C, ld, n, carry_vals, carry_rows, P, p, threadIdx.x & (kWave - 1));
}

// Host-side dispatch over storage type, vector width and unroll for one
// semiring (instantiated in the translation unit that owns the semiring).
template <class S, int VEC, int U, class R>
hipError_t launch_one(bool merge, const Shape& s, const ForwardArgs& a, hipStream_t st) {
    const typename S::T* vals = static_cast<const typename S::T*>(a.vals);
    const typename S::T* B = static_cast<const typename S::T*>(a.B);
    if (!merge) {
        const int tl_log2 = s.g_log2 + s.ts_log2;
        const int64_t rows_per_block = int64_t(kWave >> tl_log2) * (kBlock / kWave);
        const int64_t need = (a.m + rows_per_block - 1) / rows_per_block;
        const uint32_t grid = (uint32_t)(need < (1 << 22) ? need : (1 << 22));
        const TileOrder ord = make_tile_order(s.plane_rows, s.strip_rows, rows_per_block, need);
        const int* rowend = a.rowend ? a.rowend : a.rowptr + 1;
        if (s.short_addr)
            hipLaunchKernelGGL((k_rowsplit<S, VEC, U, R, true>), dim3(grid, s.col_tiles),
                               dim3(kBlock), 0, st, a.rowptr, rowend, a.colind, vals, B, a.C,
                               a.m, (int)a.n, a.ld, s.g_log2, s.ts_log2, ord, a.accumulate);
        else
            hipLaunchKernelGGL((k_rowsplit<S, VEC, U, R, false>), dim3(grid, s.col_tiles),
                               dim3(kBlock), 0, st, a.rowptr, rowend, a.colind, vals, B, a.C,
                               a.m, (int)a.n, a.ld, s.g_log2, s.ts_log2, ord, a.accumulate);
    } else {
        const dim3 grid((uint32_t)a.P, s.col_tiles);
        if (s.nz)
            hipLaunchKernelGGL((k_merge<S, VEC, U, R, true>), grid, dim3(kBlock),
                               merge_lds_bytes(0, s), st, a.rowptr, a.colind, vals, B, a.C,
                               (int)a.m, (int)a.n, a.ld, s.g_log2, a.coords, s.W, a.carry_vals,
                               a.carry_rows);
        else
            hipLaunchKernelGGL((k_merge<S, VEC, U, R, false>), grid, dim3(kBlock),
                               merge_lds_bytes(0, s), st, a.rowptr, a.colind, vals, B, a.C,
                               (int)a.m, (int)a.n, a.ld, s.g_log2, a.coords, s.W, a.carry_vals,
                               a.carry_rows);
    }
    return hipGetLastError();
}

template <class S, int VEC, class R>
hipError_t launch_u(bool merge, const Shape& s, const ForwardArgs& a, hipStream_t st) {
    switch (s.unroll) {
    case 1: return launch_one<S, VEC, 1, R>(merge, s, a, st);
    case 2: return launch_one<S, VEC, 2, R>(merge, s, a, st);
    case 4: return launch_one<S, VEC, 4, R>(merge, s, a, st);
    case 8: return launch_one<S, VEC, 8, R>(merge, s, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <class S, class R>
hipError_t launch_v(bool merge, const Shape& s, const ForwardArgs& a, hipStream_t st) {
    if (s.vec == S::kVec16) return launch_u<S, S::kVec16, R>(merge, s, a, st);
    if (s.vec == 1) return launch_u<S, 1, R>(merge, s, a, st);
    return hipErrorInvalidValue;
}

// The main kernel of one product (row split, or Phase 2 of the merge-based
// kernel) followed, for merge-based plans, by its Phase 3 fix-up.
template <class R>
hipError_t launch_forward(int dtype, bool merge, const Shape& s, const ForwardArgs& a,
                          hipStream_t st, hipEvent_t ev_after) {
    if (merge && a.P <= 0) return hipSuccess;
    if (s.g_log2 < 0 || s.ts_log2 < 0 || s.g_log2 + s.ts_log2 > 6 || s.W < 1)
        return hipErrorInvalidValue;
    hipError_t e;
    switch (dtype) {
    case 0: e = launch_v<F32, R>(merge, s, a, st); break;
    case 1: e = launch_v<BF16, R>(merge, s, a, st); break;
    case 2: e = launch_v<F16, R>(merge, s, a, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (ev_after) {
        e = hipEventRecord(ev_after, st);
        if (e != hipSuccess) return e;
    }
    if (merge && a.n > 0) {
        const uint32_t groups = (uint32_t)((a.P + kFixupWaves - 1) / kFixupWaves);
        hipLaunchKernelGGL((k_merge_fixup<R>), dim3(groups), dim3(kBlock), 0, st, a.C, a.ld,
                           (int)a.n, a.carry_vals, a.carry_rows, a.P);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace spmmk
