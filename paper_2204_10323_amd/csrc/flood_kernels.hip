// Kernels of libflood: the fused flood step for gfx950 (wave64), its device
// clock, and the FP64 reductions.
//
// One step (Methods, "Shallow Water Equations", eqs. 3-6) is ONE launch:
//   * block 0 is the clock block: it closes the volume budget of the previous
//     step, advances the FP64 clock and solves eq. (6) for the next step's
//     inflow, concurrently with the tiles;
//   * every other wave marches up one work item: a strip of 64*CPT loaded
//     columns (64*CPT - 4 output columns) over `rows` output rows.  The wave
//     keeps a rolling window of the last rows in registers; left/right
//     neighbours come from the adjacent lanes by cross-lane moves, so each
//     value is read from HBM once per strip.  The 2 halo columns at each strip
//     edge are recomputed redundantly by both strips with the same code, so a
//     face shared by two strips gets bit-identical values.
// Per cell and step the kernel reads h, z, n, qx, qy and writes h, qx, qy:
// 32 bytes in FP32, 64 in FP64.  Nothing here is a dense contraction, so there
// is no MFMA; the bound is HBM bandwidth.
#include <math.h>

#include <algorithm>
#include <atomic>

#include "flood_march.h"

namespace flood {

// The clock (one full wave): closes the budget of the previous step, advances
// the clock to the end of this step and prepares the inflow of the next step.
// Runs concurrently with the tiles of this step, which only read the current
// clock slot.
template <typename T, int VAR = 0>
__device__ void clock_wave(const StepArgs<T>& a) {
    const int lane = threadIdx.x & 63;
    DevCtl* ctl = a.ctl;
    const int cur = a.phase & 1, nxt = cur ^ 1;
    const ClockSlot ck = ctl->clk[cur];
    const double t_end = ctl->t_end;
    int last, done, nonfin;
    const double dt = step_dt<T>(a, ck, ctl->hmax[a.phase % 3], t_end, last, done, nonfin);

    double so = 0.0;
    for (int p = lane; p < a.npart; p += 64) so += a.part_prev[p];
    so = wave_sum(so);
    double si = 0.0;
    for (int p = lane; p < a.in_count; p += 64) si += (double)a.qin[a.in_first + p];
    si = wave_sum(si);

    ClockSlot nk = advance_clock(ck, dt, last, done, nonfin, si, a.dx, t_end);
    nk.v_out = ck.v_out + ck.dt_prev * a.dx * so;

    inflow_solve<T, VAR>(a, hydrograph<T>(a, nk.t), a.qin_next);
    if (lane == 0) {
        ctl->hmax[(a.phase + 2) % 3] = 0ull;
        ctl->clk[nxt] = nk;
    }
}

// One work item: strip s (columns), chunk c (rows).  Accumulates the ordered
// bits of the deepest new depth and the outflow discharge leaving the grid;
// with ACT, also whether any of the item's cells is wet (h > 0, or NaN) or
// changed its depth, or any face it stores (border faces included) carries a
// non-zero discharge.  VAR: method variant of the marcher and border faces.
template <typename T, int CPT, bool NTS, bool ACT = false, int VAR = 0>
__device__ void step_item(const StepArgs<T>& a, int s, int c, T dt, typename Ord<T>::U& hbits,
                          double& outacc, bool& moved) {
    constexpr int WL = 64 * CPT;  // loaded columns
    constexpr int WO = WL - 4;    // output columns
    const int lane = threadIdx.x & 63;
    const int nx = a.nx, ny = a.ny;
    const long long P = a.pitch;
    const int pcol = s * WO + lane * CPT;  // padded column of my first cell
    const unsigned ucol = (unsigned)pcol;  // lane offset from a row's start (row pointers are uniform)
    const unsigned boff = ucol * (unsigned)sizeof(T);
    const bool loads = pcol < nx + 2 * kHalo;
    const int j0 = c * a.rows;
    const int j1 = min(j0 + a.rows, ny);
    const StripGeo<CPT> G = strip_geo<CPT>(nx, s, WO, WL, lane);
    const bool south_chunk = (j0 == 0);
    StepK<T> K;
    K.dt = dt;
    K.gdt = T(a.g) * dt;
    K.inv_dx = T(1) / T(a.dx);
    K.h_eps = T(a.h_eps);
    K.qin = a.qin;
    K.W = 0.0;
    K.inflow_on = 0;
    K.pre = true;
    K.b_in = K.b_out = T(0);

    bool store_col[CPT];
    bool all_store = true, any_store = false;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int l = lane * CPT + m;
        store_col[m] = (l >= kHalo && l < WL - kHalo && G.i0 + m < nx);
        all_store = all_store && store_col[m];
        any_store = any_store || store_col[m];
    }

    T hN[CPT], zN[CPT], nN[CPT], qxN[CPT], qyN[CPT];
    // the inflow and outflow coefficient of a row on a west or east section,
    // loaded with the row by the strips at those borders
    const bool edge_we = G.west_strip || G.east_strip;
    const bool in_we = (a.in_side == SIDE_W || a.in_side == SIDE_E);
    const bool out_we = (a.out_side == SIDE_W || a.out_side == SIDE_E);
    T bN_in = T(0), bN_out = T(0);
    auto load_row = [&](int k) {
        if (edge_we) {
            const bool rr = (k >= 0 && k < ny);
            bN_in = (rr && in_we && a.qin) ? a.qin[k] : T(0);
            bN_out = (rr && out_we) ? a.kout[k] : T(0);
        }
        if (loads) {
            const long long o = (long long)(k + kHalo) * P;
            ldv<T, CPT>(at_byte(as_global(a.h_in) + o, boff), hN);
            ldv<T, CPT>(at_byte(as_global(a.z) + o, boff), zN);
            ldv<T, CPT>(at_byte(as_global(a.n) + o, boff), nN);
            ldv<T, CPT>(at_byte(as_global(a.qx_in) + o, boff), qxN);
            ldv<T, CPT>(at_byte(as_global(a.qy_in) + o, boff), qyN);
        } else {
#pragma unroll
            for (int m = 0; m < CPT; ++m) hN[m] = zN[m] = nN[m] = qxN[m] = qyN[m] = T(0);
        }
    };

    auto store_row = [&](int r, const T (&hv)[CPT], const T (&qxv)[CPT], const T (&qyv)[CPT]) {
        auto* const ho = as_global(a.h_out) + (long long)(r + kHalo) * P;
        auto* const qxr = as_global(a.qx_out) + (long long)(r + kHalo) * P;
        auto* const qyr = as_global(a.qy_out) + (long long)(r + kHalo) * P;
        if (all_store) {
            stv<T, CPT, NTS>(at_byte(ho, boff), hv);
            stv<T, CPT, NTS>(at_byte(qxr, boff), qxv);
            stv<T, CPT, NTS>(at_byte(qyr, boff), qyv);
        } else if (any_store) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (store_col[m]) {
                    ho[ucol + m] = hv[m];
                    qxr[ucol + m] = qxv[m];
                    qyr[ucol + m] = qyv[m];
                }
        }
    };
    // With plain stores (the persistent batch), FP32, without active tiles
    // (where the registers allow): an output row is stored at the start of the
    // next row's turn, before that turn's loads, so that waiting for the loads
    // covers the stores too instead of stalling on stores issued just before.
    constexpr bool kDefer = !NTS && !ACT && sizeof(T) == 4;
    T sh[CPT], sqx[CPT], sqy[CPT];
    int srow = 0;
    bool spend = false;

    Marcher<T, CPT, VAR> M;
    M.reset();
    load_row(j0 - 2);
    for (int k = j0 - 2; k <= j1 + 1; ++k) {
        T h0[CPT], z0[CPT], n0[CPT], qx0[CPT], qy0[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            h0[m] = hN[m]; z0[m] = zN[m]; n0[m] = nN[m]; qx0[m] = qxN[m]; qy0[m] = qyN[m];
        }
        K.b_in = bN_in;
        K.b_out = bN_out;
        if (kDefer && spend) {
            store_row(srow, sh, sqx, sqy);
            spend = false;
        }
        if (k < j1 + 1) load_row(k + 1);
        T hn[CPT], qxo[CPT], qyo[CPT], hold[CPT];
        if constexpr (ACT) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) hold[m] = M.h2[m];  // depth of row k-2 before the step
        }
        M.row(a, K, G, k, h0, z0, n0, qx0, qy0, hn, qxo, qyo);

        const int ko = k - 2;
        const bool in_item = (ko >= j0 && ko < j1);
        if constexpr (ACT) {
            if (in_item) {
#pragma unroll
                for (int m = 0; m < CPT; ++m) {
                    if (store_col[m])
                        moved = moved || !(hn[m] <= T(0)) || hn[m] != hold[m] || qxo[m] != T(0) ||
                                qyo[m] != T(0);
                    if (G.west_face[m]) moved = moved || qxo[m] != T(0);
                }
            } else if (ko == -1 && south_chunk) {
#pragma unroll
                for (int m = 0; m < CPT; ++m)
                    if (store_col[m]) moved = moved || qyo[m] != T(0);
            }
        }
        if (in_item) {
            if constexpr (kDefer) {
#pragma unroll
                for (int m = 0; m < CPT; ++m) {
                    sh[m] = hn[m]; sqx[m] = qxo[m]; sqy[m] = qyo[m];
                }
                srow = ko;
                spend = true;
            } else {
                store_row(ko, hn, qxo, qyo);
            }
        }
        row_books<T, CPT>(a, G, store_col, ko, in_item, south_chunk, hn, qxo, qyo, true, hbits,
                          outacc);
    }
    if (kDefer && spend) store_row(srow, sh, sqx, sqy);
}

// Does work item (s, c), whose cells are columns [s wo, (s + 1) wo) and rows
// [c rows, (c + 1) rows) of the grid, own a cell behind an inflow face?
template <typename T>
__device__ __forceinline__ bool feeds_inflow(const StepArgs<T>& a, int s, int c, int wo) {
    if (a.in_side < 0) return false;
    const int i0 = s * wo, i1 = min(i0 + wo, a.nx);
    const int j0 = c * a.rows, j1 = min(j0 + a.rows, a.ny);
    const int f0 = a.in_first, f1 = a.in_first + a.in_count;
    switch (a.in_side) {
    case SIDE_W: return i0 == 0 && j0 < f1 && f0 < j1;
    case SIDE_E: return i0 <= a.nx - 1 && a.nx - 1 < i1 && j0 < f1 && f0 < j1;
    case SIDE_S: return j0 == 0 && i0 < f1 && f0 < i1;
    case SIDE_N: return j1 == a.ny && i0 < f1 && f0 < i1;
    default: return false;
    }
}

// Must item (s, c) be computed in this step (active-tile skipping)?  A step
// leaves a cell as it is, with zero discharges on its faces, when the cell
// and its four neighbours hold no water: h <= 0 on both sides makes a face
// dry (h_f <= 0), so its discharge is 0 whatever the donor factors.  The
// four neighbours of an item's cells lie in the item or in the four items
// that share an edge with it, so the item may be skipped when those five
// items were dry and unchanged in the previous step (flags of step n-1 are
// 0).  The skipped item's output buffer holds its state of step n-2, which
// equals that of step n-1 when the item's own flag of step n-2 is 0 as well.
// Items behind an inflow face are always computed: the inflow can start at
// any step.
template <typename T>
__device__ __forceinline__ bool item_needed(const StepArgs<T>& a, int s, int c, int wo) {
    if (feeds_inflow<T>(a, s, c, wo)) return true;
    const int lane = threadIdx.x & 63;
    int v = 0;
    if (lane < 6) {
        // lanes 0-4: the item, west, east, south, north at step n-1; lane 5: the item at n-2
        const int ds = lane == 1 ? -1 : (lane == 2 ? 1 : 0);
        const int dc = lane == 3 ? -1 : (lane == 4 ? 1 : 0);
        const int ss = s + ds, cc = c + dc;
        const int sl = lane == 5 ? (a.phase + 1) % 3 : (a.phase + 2) % 3;
        if (ss >= 0 && ss < a.nstrips && cc >= 0 && cc < a.nchunks)
            v = a.act[sl * a.act_stride + (long long)cc * a.nstrips + ss];
    }
    return __ballot(v != 0) != 0ull;
}

// Work item `item` of one step (strip fastest): the marching tile, then the
// wave's deepest cell into the next max slot and its outflow partial sum;
// with ACT, first the skip test (unless SELECTED: the selection kernel made
// it), and last the item's flag of this step.
template <typename T, int CPT, bool NTS, bool ACT = false, int VAR = 0, bool SELECTED = false>
__device__ __forceinline__ void tile_item(const StepArgs<T>& a, int item) {
    // (in a batch, members without active tiles have no flags: a.act NULL)
    const bool act = ACT && a.act != nullptr;
    if (act && !SELECTED) {
        const int s = item % a.nstrips, c = item / a.nstrips;
        if (!item_needed<T>(a, s, c, 64 * CPT - 4)) {
            // nothing moves: no deeper cell, no outflow, flag 0
            if ((threadIdx.x & 63) == 0) {
                a.act[(a.phase % 3) * a.act_stride + item] = 0;
                const int slot = part_slot<T>(a, s, c);
                if (slot >= 0) a.part_cur[slot] = 0.0;
            }
            return;
        }
    }
    const ClockSlot ck = a.ctl->clk[a.phase & 1];
    int last, done, nonfin;
    const double dt64 = step_dt<T>(a, ck, a.ctl->hmax[a.phase % 3], a.ctl->t_end, last, done, nonfin);
    const int s = item % a.nstrips, c = item / a.nstrips;
    typename Ord<T>::U hb = 0;
    double outacc = 0.0;
    bool moved = false;
    step_item<T, CPT, NTS, ACT, VAR>(a, s, c, (T)dt64, hb, outacc, moved);
    hb = wave_max_key(hb);
    const int slot = part_slot<T>(a, s, c);
    if (slot >= 0) outacc = wave_sum(outacc);
    bool any_moved = false;
    if constexpr (ACT) any_moved = __ballot(moved) != 0ull;
    if ((threadIdx.x & 63) == 0) {
        if (hb) atomicMax(&a.ctl->hmax[(a.phase + 1) % 3], (unsigned long long)hb);
        if (slot >= 0) a.part_cur[slot] = outacc;
        if (act) a.act[(a.phase % 3) * a.act_stride + item] = any_moved ? 1 : 0;
    }
}

// Active tiles, per step: the skip test of every work item (one thread per
// item), an ordered compaction of the items that must be computed, and a
// persistent grid over that list.
template <typename T, int CPT>
__device__ __forceinline__ bool select_need(const StepArgs<T>& a, long long item) {
    const int s = (int)(item % a.nstrips), c = (int)(item / a.nstrips);
    if (feeds_inflow<T>(a, s, c, 64 * CPT - 4)) return true;
    const unsigned char* f1 = a.act + ((a.phase + 2) % 3) * a.act_stride;  // step n-1
    const unsigned char* f2 = a.act + ((a.phase + 1) % 3) * a.act_stride;  // step n-2
    return f1[item] || f2[item] || (s > 0 && f1[item - 1]) || (s + 1 < a.nstrips && f1[item + 1]) ||
           (c > 0 && f1[item - a.nstrips]) || (c + 1 < a.nchunks && f1[item + a.nstrips]);
}

// Items of this block that must be computed, and the ranks of its waves'.
__device__ __forceinline__ unsigned block_rank(bool need, unsigned& rank_in_block) {
    __shared__ unsigned wave_n[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(need);
    if (lane == 0) wave_n[w] = (unsigned)__popcll(mask);
    __syncthreads();
    unsigned before = 0, total = 0;
    for (int k = 0; k < 4; ++k) {
        before += (k < w) ? wave_n[k] : 0u;
        total += wave_n[k];
    }
    rank_in_block = before + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
    return total;
}

// Pass 1: skipped items get flag 0 and a zero outflow partial; each block
// counts the items that must be computed.
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_select_count(StepArgs<T> a, unsigned* block_n) {
    const long long items = (long long)a.nstrips * a.nchunks;
    const long long item = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool need = false;
    if (item < items) {
        need = select_need<T, CPT>(a, item);
        if (!need) {
            a.act[(a.phase % 3) * a.act_stride + item] = 0;
            const int slot = part_slot<T>(a, (int)(item % a.nstrips), (int)(item / a.nstrips));
            if (slot >= 0) a.part_cur[slot] = 0.0;
        }
    }
    unsigned rank;
    const unsigned n = block_rank(need, rank);
    if (threadIdx.x == 0) block_n[blockIdx.x] = n;
}

// Between passes 1 and 2 when there are many blocks: one block turns the
// per-block counts into exclusive offsets in place (a running scan over
// chunks of 256).
__global__ __launch_bounds__(256) void k_select_prefix(unsigned* block_n, unsigned nblocks) {
    __shared__ unsigned sc[256];
    unsigned carry = 0;
    for (unsigned b0 = 0; b0 < nblocks; b0 += 256) {
        const unsigned b = b0 + threadIdx.x;
        const unsigned v = b < nblocks ? block_n[b] : 0u;
        sc[threadIdx.x] = v;
        __syncthreads();
        for (unsigned d = 1; d < 256; d <<= 1) {  // inclusive scan
            const unsigned add = threadIdx.x >= d ? sc[threadIdx.x - d] : 0u;
            __syncthreads();
            sc[threadIdx.x] += add;
            __syncthreads();
        }
        if (b < nblocks) block_n[b] = carry + sc[threadIdx.x] - v;
        carry += sc[255];
        __syncthreads();
    }
}

// Pass 2: the items that must be computed, in raster order, at the offset the
// counts of the blocks before give (summed here, or taken from
// k_select_prefix when `prefixed`); the last block writes the total.
template <typename T, int CPT>
__global__ __launch_bounds__(256) void k_select_scatter(StepArgs<T> a, const unsigned* block_n,
                                                        int prefixed) {
    __shared__ unsigned part[256];
    const long long items = (long long)a.nstrips * a.nchunks;
    const long long item = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned base;
    if (prefixed) {
        base = block_n[blockIdx.x];
    } else {
        unsigned off = 0;
        for (unsigned b = threadIdx.x; b < blockIdx.x; b += blockDim.x) off += block_n[b];
        part[threadIdx.x] = off;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < (unsigned)w) part[threadIdx.x] += part[threadIdx.x + w];
            __syncthreads();
        }
        base = part[0];
    }
    const bool need = item < items && select_need<T, CPT>(a, item);
    unsigned rank;
    const unsigned n = block_rank(need, rank);
    if (need) a.act_list[base + rank] = (int)item;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) a.act_count[a.phase & 1] = base + n;
    // the step's work counters of the list kernel (one per group of blocks)
    if (blockIdx.x == 0 && threadIdx.x < 8) a.act_count[2 + (a.phase & 1) * 8 + threadIdx.x] = 0u;
}

// Pass 3: a persistent grid (block 0: the clock) that fits the device at
// once, so its size does not depend on the list and the launch can be
// captured.  Blocks go round-robin to the 8 XCDs; XCD x takes the x-th eighth
// of the list, a run of neighbouring items (shared halo rows meet in one L2)
// of the same length on every XCD wherever the water is.  (Fewer than 8
// blocks: each block takes its own share.)  Each wave takes one item by its
// index, then further ones from the group's counter as it finishes, so items
// of uneven cost spread over the waves as they free up.
// occupancy of the one-wave-per-item kernel (the loop must not cost a wave per SIMD)
template <typename T, int CPT>
__global__ __launch_bounds__(256, (sizeof(T) == 4 ? (CPT == 4 ? 3 : CPT == 2 ? 5 : 7)
                                                   : (CPT == 4 ? 1 : CPT == 2 ? 3 : 4)))
void k_step_list(StepArgs<T> a) {
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) clock_wave<T>(a);
        return;
    }
    const unsigned count = a.act_count[a.phase & 1];
    const unsigned nblk = gridDim.x - 1, b = blockIdx.x - 1;
    const unsigned groups = nblk < 8u ? nblk : 8u;
    const unsigned g = b % groups, per = (nblk - g + groups - 1u) / groups;  // blocks of group g
    const unsigned lo = (unsigned)((unsigned long long)count * g / groups);
    const unsigned hi = (unsigned)((unsigned long long)count * (g + 1u) / groups);
    const unsigned nw = per * 4u;
    unsigned* next = a.act_count + 2 + (a.phase & 1) * 8 + g;
    unsigned idx = lo + (b / groups) * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    while (idx < hi) {
        const int item = __builtin_amdgcn_readfirstlane(a.act_list[idx]);
        tile_item<T, CPT, true, true, 0, true>(a, item);
        unsigned k = 0;
        if ((threadIdx.x & 63) == 0) k = atomicAdd(next, 1u);
        idx = lo + nw + __builtin_amdgcn_readfirstlane(k);
    }
}

template <typename T, int CPT, bool ACT, int VAR>
__global__ __launch_bounds__(256) void k_step(StepArgs<T> a) {
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) clock_wave<T, VAR>(a);
        return;
    }
    // XCD-aware order: workgroups go round-robin to the 8 XCDs, so XCD x runs
    // blocks b with b % 8 == x.  Give each XCD one contiguous run of the
    // raster order (strip fastest), i.e. a horizontal band of the grid: the
    // strips that share boundary cache lines and the chunks that share halo
    // rows then meet in the same L2.
    const int nblk = gridDim.x - 1, b = blockIdx.x - 1;
    const int xcd = b & 7, q8 = nblk >> 3, r8 = nblk & 7;
    const int lin = xcd * q8 + min(xcd, r8) + (b >> 3);
    // the wave index is uniform across the wave: keep it (and everything
    // derived from it: strip, rows, loop counter, border tests) scalar
    const int wave = lin * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= a.nstrips * a.nchunks) return;
    tile_item<T, CPT, true, ACT, VAR>(a, wave);
}

// Persistent batch of independent members, one launch for many steps.
// Members are assigned to XCDs; a wave reads the id of the XCD it runs on and
// serves only that XCD's queue, so every member's data stays in one L2 and the
// hand-over between steps needs no L2 write-back: stores are complete in the
// shared L2 when the writer's vector memory counter drains, and a consumer
// drops its CU's L1 (agent-scope acquire) before reading.  The queue holds, step after step,
// for each member one clock entry and its tile items.  Entries of step k of a
// member wait only until that member's step k-1 is complete (its depth
// maximum and clock then exist), so members do not wait for each other and no
// grid-wide barrier is needed.  No co-residency is needed either: a wave
// takes an entry only while it runs, and an entry waits only for entries of
// lower queue index, which running waves of the same XCD took before it; so
// the lowest unfinished entry never waits and always completes, and a wave
// that has not started yet holds nothing anyone waits for.  Every XCD gets
// workgroups (the grid is a multiple of the CU count and workgroups go
// round-robin to the XCDs), and each of them drains its XCD's queue.  A wait
// longer than spin_limit sleeps sets *error and exits.
template <typename T, int CPT, bool ACT>
__global__ __launch_bounds__(256) void k_batch(BatchArgs<T> B) {
    const int lane = threadIdx.x & 63;
    const int x = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15);  // XCC_ID
    if (x >= B.nxcc) return;
    const int m_lo = B.xbegin[x], m_hi = B.xbegin[x + 1];
    if (m_lo >= m_hi) return;
    const int per_step = B.per_step[x];
    const unsigned long long total = (unsigned long long)per_step * (unsigned long long)B.nsteps;
    for (;;) {
        unsigned long long q = 0;
        if (lane == 0) q = atomicAdd(&B.next[x], 1ull);
        // wave-uniform from here on: scalar registers, scalar loads of the arguments
        q = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(q >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((unsigned)q);
        if (q >= total) break;
        const long long k = (long long)(q / (unsigned long long)per_step);
        const int r = (int)(q - (unsigned long long)k * per_step);
        int lo = m_lo, hi = m_hi - 1;      // member with first <= r, largest such
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (B.scen[mid].first <= r) lo = mid; else hi = mid - 1;
        }
        const int m = lo;
        const BatchScen<T>& S = B.scen[m];
        const int e = r - S.first;
        if (k > 0) {
            const unsigned long long need = (unsigned long long)k * (unsigned long long)(S.items + 1);
            int ok = 1;
            if (lane == 0) {
                long long spins = 0;
                while (__hip_atomic_load(&B.done[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > B.spin_limit) { ok = 0; break; }
                }
            }
            ok = __builtin_amdgcn_readfirstlane(ok);
            if (!ok) {
                if (lane == 0) atomicExch(B.error, 1);
                break;
            }
            // acquire: drop this CU's L1 copies (and clean L2 lines of
            // non-coherent memory) so the member's new data is read from L2
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const StepArgs<T>& a = S.a[(int)((S.n0 + k) % 6)];
        if (e == 0) clock_wave<T>(a);
        else tile_item<T, CPT, false, ACT>(a, e - 1);
        // release within the XCD: this wave's stores have reached L2
        __builtin_amdgcn_s_waitcnt(0);
        __asm__ volatile("" ::: "memory");
        if (lane == 0) atomicAdd(&B.done[m], 1ull);
    }
}

// Inflow applied by the first step after commit (the clock slot is set by the
// host): written into the buffer that step reads.
template <typename T, int VAR>
__global__ void k_prime(StepArgs<T> a) {
    inflow_solve<T, VAR>(a, hydrograph<T>(a, a.ctl->clk[a.phase & 1].t), const_cast<T*>(a.qin));
}

// Clock and budget as of now: report[] = {t, last_dt, steps, v_in, v_out, done, nonfinite}.
template <typename T>
__global__ void k_flush(StepArgs<T> a) {
    const int lane = threadIdx.x & 63;
    DevCtl* ctl = a.ctl;
    const ClockSlot ck = ctl->clk[a.phase & 1];
    double so = 0.0;
    for (int p = lane; p < a.npart; p += 64) so += a.part_prev[p];
    so = wave_sum(so);
    if (lane == 0) {
        const unsigned long long hb = ctl->hmax[a.phase % 3];
        ctl->report[0] = ck.t;
        ctl->report[1] = ck.last_dt;
        ctl->report[2] = (double)ck.steps;
        ctl->report[3] = ck.v_in;
        ctl->report[4] = ck.v_out + ck.dt_prev * a.dx * so;
        ctl->report[5] = !(ctl->t_end - ck.t > 0.0) ? 1.0 : 0.0;
        ctl->report[6] = (ck.nonfinite || Ord<T>::nonfinite(hb)) ? 1.0 : 0.0;
    }
}

// Fold the outflow partial sums of the last step into the clock slot and clear
// them, so the work decomposition (and with it the partial-sum slots) can
// change before the next step.
template <typename T>
__global__ void k_fold(StepArgs<T> a) {
    const int lane = threadIdx.x & 63;
    ClockSlot* ck = &a.ctl->clk[a.phase & 1];
    double so = 0.0;
    for (int p = lane; p < a.npart; p += 64) so += a.part_prev[p];
    so = wave_sum(so);
    if (lane == 0) {
        ck->v_out = ck->v_out + ck->dt_prev * a.dx * so;
        ck->dt_prev = 0.0;
    }
    for (int p = lane; p < a.npart; p += 64) const_cast<double*>(a.part_prev)[p] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_hmax_init(const T* h, long long pitch, int nx, int ny,
                                                   DevCtl* ctl) {
    unsigned long long b = 0;
    const long long ncell = (long long)nx * ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < ncell;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long j = idx / nx, i = idx - j * nx;
        const unsigned long long v = Ord<T>::bits(h[(j + kHalo) * pitch + i + kHalo]);
        b = v > b ? v : b;
    }
    b = wave_max_u64(b);
    if ((threadIdx.x & 63) == 0 && b) atomicMax(&ctl->hmax[0], b);
}

// FP64 volume: fixed grid, fixed-order block partials, then one block sums
// them in order -- deterministic.
template <typename T>
__global__ __launch_bounds__(256) void k_volume_part(const T* h, long long pitch, int nx, int ny,
                                                     double* part) {
    __shared__ double red[4];
    double s = 0.0;
    const long long ncell = (long long)nx * ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < ncell;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long j = idx / nx, i = idx - j * nx;
        s += (double)h[(j + kHalo) * pitch + i + kHalo];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ void k_volume_sum(const double* part, int nparts, double* out) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int p = lane; p < nparts; p += 64) s += part[p];
    s = wave_sum(s);
    if (lane == 0) *out = s;
}

// ----------------------------------------------------------------- launchers
int strip_width(int cpt) { return 64 * cpt - 4; }

// Blocks of k_step_list<T, CPT> the current device holds at once (queried
// once; prepare_step_list does it outside any graph capture).  Threads that
// query it together store the same value.
template <typename T, int CPT>
std::atomic<int>& list_resident() {
    static std::atomic<int> resident{0};
    return resident;
}

template <typename T, int CPT>
hipError_t query_list_resident() {
    std::atomic<int>& resident = list_resident<T, CPT>();
    if (resident.load(std::memory_order_relaxed) > 0) return hipSuccess;
    int per_cu = 0, ncu = 0, dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_list<T, CPT>, 256, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    resident.store(std::max(1, per_cu) * std::max(1, ncu), std::memory_order_relaxed);
    return hipSuccess;
}

template <typename T>
hipError_t prepare_step_list(int cpt) {
    switch (cpt) {
    case 1: return query_list_resident<T, 1>();
    case 2: return query_list_resident<T, 2>();
    case 4: return query_list_resident<T, 4>();
    default: return hipErrorInvalidValue;
    }
}

// The selection kernel, then the persistent list kernel with as many blocks
// as the device holds at once (but no more than the items need).
template <typename T, int CPT>
hipError_t launch_step_list(const StepArgs<T>& a, long long items, hipStream_t s) {
    hipError_t e = query_list_resident<T, CPT>();
    if (e != hipSuccess) return e;
    const int resident = list_resident<T, CPT>().load(std::memory_order_relaxed);
    const unsigned sel_blocks = (unsigned)std::max<long long>(1, (items + 255) / 256);
    // the per-block counts live after the list's `items` entries (capacity act_stride + blocks)
    unsigned* block_n = reinterpret_cast<unsigned*>(a.act_list + a.act_stride);
    hipLaunchKernelGGL((k_select_count<T, CPT>), dim3(sel_blocks), dim3(256), 0, s, a, block_n);
    // few blocks: each scatter block sums the counts before it; many: scan them first
    const int prefixed = sel_blocks > 2048 ? 1 : 0;
    if (prefixed) hipLaunchKernelGGL(k_select_prefix, dim3(1), dim3(256), 0, s, block_n, sel_blocks);
    hipLaunchKernelGGL((k_select_scatter<T, CPT>), dim3(sel_blocks), dim3(256), 0, s, a,
                       (const unsigned*)block_n, prefixed);
    const long long want = (items + 3) / 4;
    const unsigned blocks = (unsigned)(1 + std::min<long long>(want, resident));
    hipLaunchKernelGGL((k_step_list<T, CPT>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T, bool ACT, int VAR = 0>
hipError_t launch_step_act(const StepArgs<T>& a, int cpt, int blocks, hipStream_t s) {
    switch (cpt) {
    case 1: hipLaunchKernelGGL((k_step<T, 1, ACT, VAR>), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_step<T, 2, ACT, VAR>), dim3(blocks), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_step<T, 4, ACT, VAR>), dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step(const StepArgs<T>& a, int cpt, hipStream_t s) {
    const long long items = (long long)a.nstrips * a.nchunks;
    const int blocks = (int)(1 + (items + 3) / 4);
    if (a.variant) {
        // method variants run without active tiles
        if (a.act) return hipErrorInvalidValue;
        switch (a.variant) {
        case VAR_FRICTION_VECTOR:
            return launch_step_act<T, false, VAR_FRICTION_VECTOR>(a, cpt, blocks, s);
        case VAR_BOUNDARY_CELL_AREA:
            return launch_step_act<T, false, VAR_BOUNDARY_CELL_AREA>(a, cpt, blocks, s);
        case VAR_FRICTION_VECTOR | VAR_BOUNDARY_CELL_AREA:
            return launch_step_act<T, false, VAR_FRICTION_VECTOR | VAR_BOUNDARY_CELL_AREA>(a, cpt,
                                                                                        blocks, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (a.act) {
        // the flags (and list entries) of every item must fit in a slot
        if (items > a.act_stride) return hipErrorInvalidValue;
        // with a list: the selection kernels and a persistent grid over the
        // items to compute (best when few items hold water); without: one
        // wave per item that makes the skip test itself
        if (!a.act_list) return launch_step_act<T, true>(a, cpt, blocks, s);
        if (!a.act_count) return hipErrorInvalidValue;
        switch (cpt) {
        case 1: return launch_step_list<T, 1>(a, items, s);
        case 2: return launch_step_list<T, 2>(a, items, s);
        case 4: return launch_step_list<T, 4>(a, items, s);
        default: return hipErrorInvalidValue;
        }
    }
    return launch_step_act<T, false>(a, cpt, blocks, s);
}

__global__ void k_fill_bytes(unsigned char* p, long long n, unsigned char v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_bytes(unsigned char* p, long long n, unsigned char v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long want = (n + 255) / 256;
    const int blocks = (int)std::min<long long>(want, 2048);
    hipLaunchKernelGGL(k_fill_bytes, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prime(const StepArgs<T>& a, hipStream_t s) {
    if (a.variant & VAR_BOUNDARY_CELL_AREA)
        hipLaunchKernelGGL((k_prime<T, VAR_BOUNDARY_CELL_AREA>), dim3(1), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_prime<T, 0>), dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_flush(const StepArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL((k_flush<T>), dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fold(const StepArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fold<T>), dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T, int CPT, bool ACT>
hipError_t launch_batch_cpt(const BatchArgs<T>& b, int device, hipStream_t s, int* blocks_out) {
    int per_cu = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<T, CPT, ACT>, 256, 0);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    const int blocks = std::max(1, per_cu) * ncu;
    if (blocks_out) *blocks_out = blocks;
    // an ordinary launch: the queue needs no co-residency (see k_batch)
    hipLaunchKernelGGL((k_batch<T, CPT, ACT>), dim3(blocks), dim3(256), 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch(const BatchArgs<T>& b, int cpt, int device, hipStream_t s, int* blocks_out,
                        bool act) {
    switch (cpt) {
    case 1: return act ? launch_batch_cpt<T, 1, true>(b, device, s, blocks_out)
                       : launch_batch_cpt<T, 1, false>(b, device, s, blocks_out);
    case 2: return act ? launch_batch_cpt<T, 2, true>(b, device, s, blocks_out)
                       : launch_batch_cpt<T, 2, false>(b, device, s, blocks_out);
    case 4: return act ? launch_batch_cpt<T, 4, true>(b, device, s, blocks_out)
                       : launch_batch_cpt<T, 4, false>(b, device, s, blocks_out);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_hmax_init(const T* h, long long pitch, int nx, int ny, DevCtl* ctl,
                            hipStream_t s) {
    const long long ncell = (long long)nx * ny;
    int blocks = (int)((ncell + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL((k_hmax_init<T>), dim3(blocks), dim3(256), 0, s, h, pitch, nx, ny, ctl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_volume(const T* h, long long pitch, int nx, int ny, double* partials, int nparts,
                         double* out, hipStream_t s) {
    hipLaunchKernelGGL((k_volume_part<T>), dim3(nparts), dim3(256), 0, s, h, pitch, nx, ny,
                       partials);
    hipLaunchKernelGGL(k_volume_sum, dim3(1), dim3(64), 0, s, partials, nparts, out);
    return hipGetLastError();
}

template hipError_t prepare_step_list<float>(int);
template hipError_t prepare_step_list<double>(int);
template hipError_t launch_step<float>(const StepArgs<float>&, int, hipStream_t);
template hipError_t launch_step<double>(const StepArgs<double>&, int, hipStream_t);
template hipError_t launch_prime<float>(const StepArgs<float>&, hipStream_t);
template hipError_t launch_prime<double>(const StepArgs<double>&, hipStream_t);
template hipError_t launch_flush<float>(const StepArgs<float>&, hipStream_t);
template hipError_t launch_flush<double>(const StepArgs<double>&, hipStream_t);
template hipError_t launch_fold<float>(const StepArgs<float>&, hipStream_t);
template hipError_t launch_fold<double>(const StepArgs<double>&, hipStream_t);
template hipError_t launch_batch<float>(const BatchArgs<float>&, int, int, hipStream_t, int*, bool);
template hipError_t launch_batch<double>(const BatchArgs<double>&, int, int, hipStream_t, int*, bool);
template hipError_t launch_hmax_init<float>(const float*, long long, int, int, DevCtl*, hipStream_t);
template hipError_t launch_hmax_init<double>(const double*, long long, int, int, DevCtl*,
                                             hipStream_t);
template hipError_t launch_volume<float>(const float*, long long, int, int, double*, int, double*,
                                         hipStream_t);
template hipError_t launch_volume<double>(const double*, long long, int, int, double*, int,
                                          double*, hipStream_t);

}  // namespace flood
