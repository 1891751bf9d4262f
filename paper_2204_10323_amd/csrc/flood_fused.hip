// Two flood steps per launch (Methods, "Shallow Water Equations", eqs. 3-6).
//
// The single-step kernel reads the state once and writes it once per step,
// so a step costs at least 32 bytes per cell of HBM traffic.  Here one wave
// runs two row marchers on its strip: the second consumes the rows the first
// one emits, still in registers, so two steps cost one read and one write of
// the state.  A strip loads 64*CPT columns and outputs 64*CPT - 8 of them
// (each step needs two halo columns on each side).
//
// The second step's dt depends on the deepest cell of the intermediate state,
// a grid-wide maximum that exists only once the launch has ended.  The launch
// therefore runs the second step with the dt it would have if that maximum
// were small (the fixed dt, or dt_max, in both cases cut at t_end); the next
// launch computes the true dt from the maximum the tiles recorded and, if
// they differ, redoes both steps with the right dt from the launch's input,
// which the ping-pong buffers still hold.  Either way every step uses exactly
// the dt, inflow and arithmetic of the single-step kernel, so the two paths
// give the same bits.  When the CFL bound is close to active the launch makes
// one step only.
//
// Every wave derives the launch's plan from the device clock, so the number
// of steps a launch makes is decided on the device; launches past the
// requested count do nothing.
#include <math.h>

#include <algorithm>

#include "flood_march.h"

namespace flood {

// What a launch does; every wave computes the same plan.
struct Plan2 {
    int mode;            // 0 nothing, 1 one step, 2 two steps, 3 redo the last launch's two steps
    int in;              // buffer read; the launch writes buffer in ^ 1
    int verified;        // the state claimed by the last launch holds
    ClockSlot ck0;       // clock at the start of the first step
    ClockSlot ck1;       // clock at the start of the second step (t and nonfinite; complete in mode 3)
    double dt_a, dt_b;
    int last_a, done_a, nonfin_a, last_b, done_b, nonfin_b;
    long long gen;       // generation of the state the launch writes (a redo: the one it replaces)
};

// Whether to run a second step with a speculated dt: always with a fixed dt,
// and with the CFL clock when the bound is clear of dt_max: the deepest cell
// may deepen by 4 % within the step without making it active.  A guess that
// fails costs one redo launch; a launch that makes one step costs a second
// pass over the state, so a narrow margin pays (deep, wet grids run at dt_max
// with the bound close by).
template <typename T>
__device__ __forceinline__ bool spec_room(const StepArgs<T>& a, unsigned long long hb) {
    if (a.dt_fixed > 0.0) return true;
    const double hm = Ord<T>::value(hb);
    return !(hm > 0.0) || a.alpha * a.dx / sqrt(a.g * hm) >= 1.02 * a.dt_max;
}

template <typename T>
__device__ Plan2 make_plan(const Step2Args<T>& A) {
    const StepArgs<T>& a = A.a;
    const DevCtl* ctl = a.ctl;
    const Clock2& S = ctl->c2[A.phase & 1];
    const int gp = (A.phase + 2) % 3;
    const unsigned long long hmid = ctl->hm2[2 * gp], hend = ctl->hm2[2 * gp + 1];
    const double t_end = ctl->t_end;
    Plan2 P;
    P.mode = 0;
    P.verified = 1;
    P.dt_a = P.dt_b = 0.0;
    P.last_a = P.done_a = P.nonfin_a = P.last_b = P.done_b = P.nonfin_b = 0;
    double dt_true = 0.0;
    int lt = 0, dn = 0, nf = 0;
    if (S.pending) {
        dt_true = step_dt<T>(a, S.mid, hmid, t_end, lt, dn, nf);
        P.verified = (dt_true == S.dt_b) ? 1 : 0;
    }
    if (!P.verified) {
        P.mode = 3;
        P.gen = S.gen;
        P.in = S.cur ^ 1;
        P.ck0 = S.back;
        P.ck1 = S.mid;
        P.dt_a = S.dt_a;
        P.dt_b = dt_true;
        P.last_b = lt;
        P.done_b = dn;
        P.nonfin_b = nf;
        return P;
    }
    P.in = S.cur;
    P.gen = S.gen + 1;
    P.ck0 = S.ck;
    P.ck1 = S.ck;
    const long long remaining = ctl->target2 - S.vsteps;
    if (A.resolve || remaining <= 0) return P;
    P.dt_a = step_dt<T>(a, S.ck, hend, t_end, P.last_a, P.done_a, P.nonfin_a);
    P.ck1.t = P.last_a ? t_end : S.ck.t + P.dt_a;
    P.ck1.nonfinite = P.nonfin_a ? 1 : 0;
    if (remaining < 2 || !spec_room<T>(a, hend)) {
        P.mode = 1;
        return P;
    }
    P.mode = 2;
    P.dt_b = step_dt<T>(a, P.ck1, 0ull, t_end, P.last_b, P.done_b, P.nonfin_b);
    return P;
}

// Total inflow (per unit width) of a step starting at time t: eq. (6) solved
// and summed exactly as the single-step clock sums the stored magnitudes.
template <typename T>
__device__ double inflow_sum(const StepArgs<T>& a, double t) {
    const int lane = threadIdx.x & 63;
    if (a.in_count <= 0) return 0.0;
    const double Q = hydrograph<T>(a, t);
    if (!(Q > 0.0)) return 0.0;
    const double W = inflow_level(a.in_z, a.in_k, a.in_count, a.dx, Q);
    double si = 0.0;
    for (int p = lane; p < a.in_count; p += 64) si += (double)(T)(a.in_k[p] * pow53(W - a.in_z[p]));
    return wave_sum(si);
}

template <typename T>
__device__ double partial_sum(const double* part, int npart) {
    const int lane = threadIdx.x & 63;
    double so = 0.0;
    for (int p = lane; p < npart; p += 64) so += part[p];
    return wave_sum(so);
}

// The clock wave of a two-step launch: closes the outflow of the last launch
// once its state is known to hold, advances the clock over this launch's
// steps and publishes the next slot.
template <typename T>
__device__ void clock2_wave(const Step2Args<T>& A, const Plan2& P) {
    const StepArgs<T>& a = A.a;
    const int lane = threadIdx.x & 63;
    DevCtl* ctl = a.ctl;
    const Clock2 S = ctl->c2[A.phase & 1];
    const int gp = (A.phase + 2) % 3, g = A.phase % 3, gn = (A.phase + 1) % 3;
    const int pp = (A.phase + 1) & 1;  // parity of the last launch
    const double t_end = ctl->t_end;
    ClockSlot base = P.ck0;
    if (P.verified && S.nclose >= 1) {
        double so = partial_sum<T>(A.part_a[pp], a.npart);
        base.v_out = base.v_out + S.dt_a * a.dx * so;
        if (S.nclose == 2) {
            so = partial_sum<T>(A.part_b[pp], a.npart);
            base.v_out = base.v_out + S.dt_b * a.dx * so;
        }
    }
    Clock2 N = S;
    if (P.mode == 0) {
        N.ck = base;
        N.nclose = 0;
        N.pending = 0;
        if (lane == 0) {
            ctl->hm2[2 * g] = ctl->hm2[2 * gp];
            ctl->hm2[2 * g + 1] = ctl->hm2[2 * gp + 1];
        }
    } else {
        ClockSlot c1;
        if (P.mode == 3) {
            c1 = S.mid;
        } else {
            const double si = inflow_sum<T>(a, base.t);
            c1 = advance_clock(base, P.dt_a, P.last_a, P.done_a, P.nonfin_a, si, a.dx, t_end);
        }
        N.back = base;
        N.mid = c1;
        N.dt_a = P.dt_a;
        N.cur = P.in ^ 1;
        N.gen = P.gen;
        if (P.mode == 1) {
            N.ck = c1;
            N.dt_b = 0.0;
            N.nclose = 1;
            N.pending = 0;
            N.vsteps = S.vsteps + 1;
        } else {
            const double si = inflow_sum<T>(a, c1.t);
            N.ck = advance_clock(c1, P.dt_b, P.last_b, P.done_b, P.nonfin_b, si, a.dx, t_end);
            N.dt_b = P.dt_b;
            N.nclose = 2;
            N.pending = (P.mode == 2) ? 1 : 0;
            N.vsteps = S.vsteps + (P.mode == 2 ? 2 : 0);
        }
    }
    if (lane == 0) {
        ctl->hm2[2 * gn] = 0ull;
        ctl->hm2[2 * gn + 1] = 0ull;
        ctl->c2[(A.phase + 1) & 1] = N;
    }
}

// Whether the waves of strip s, rows [j0, j1) meet an inflow face: those
// solve eq. (6) themselves (the second step's time is not known before the
// launch).
template <typename T>
__device__ __forceinline__ bool needs_inflow(const StepArgs<T>& a, int s, int j0, int j1, int wo,
                                             int wl) {
    if (a.in_side < 0 || a.in_count <= 0) return false;
    const int f = a.in_first, e = a.in_first + a.in_count;
    const int c0 = s * wo - kHalo;  // real column of the strip's first loaded cell
    switch (a.in_side) {
    case SIDE_W: return s == 0 && j0 - 4 < e && j1 + 4 > f;
    case SIDE_E: return a.nx - 1 >= c0 && a.nx - 1 < c0 + wl && j0 - 4 < e && j1 + 4 > f;
    case SIDE_S: return j0 <= 4 && c0 < e && c0 + wl > f;
    default: return j1 + 3 >= a.ny && c0 < e && c0 + wl > f;
    }
}

// One work item of a two-step (two = true) or one-step launch: strip s,
// rows [j0, j1).  Row k enters marcher A; the row A emits (k - 2) enters
// marcher B with the bed and roughness of that row; B emits row k - 4.
// Values of A's emitted rows outside the grid are replaced by zeros, which is
// what the single-step kernel reads from the halo there.
// With ACT, `moved` records whether any row of the item that either step
// emits holds water (h > 0, or NaN), changed its depth in that step, or
// carries a non-zero discharge on a face the item stores (border faces
// included); A's rows beyond the item count too (conservative).
template <typename T, int CPT, bool ACT, bool GA>
__device__ void step2_item(const StepArgs<T>& a, const T* __restrict__ h_in,
                           const T* __restrict__ qx_in, const T* __restrict__ qy_in,
                           T* __restrict__ h_out, T* __restrict__ qx_out, T* __restrict__ qy_out,
                           const StepK<T>& KA, const StepK<T>& KB, bool two, int s, int j0, int j1,
                           typename Ord<T>::U& hbA, typename Ord<T>::U& hbB, double& outA,
                           double& outB, bool& moved) {
    constexpr int WL = 64 * CPT;  // loaded columns
    constexpr int WO = WL - 8;    // output columns (strip 0: two more on the left)
    const int lane = threadIdx.x & 63;
    const int nx = a.nx, ny = a.ny;
    const long long P = a.pitch;
    const int pcol = s * WO + lane * CPT;
    const unsigned ucol = (unsigned)pcol;  // lane offset from a row's start (row pointers are uniform)
    const unsigned boff = ucol * (unsigned)sizeof(T);
    const bool loads = pcol < nx + 2 * kHalo;
    const StripGeo<CPT> G = strip_geo<CPT>(nx, s, WO, WL, lane);
    const bool south_chunk = (j0 == 0);
    const int lo = (s == 0) ? kHalo : 2 * kHalo;

    bool store_col[CPT];
    bool all_store = true, any_store = false;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int l = lane * CPT + m;
        store_col[m] = (l >= lo && l < WL - 2 * kHalo && G.i0 + m < nx);
        all_store = all_store && store_col[m];
        any_store = any_store || store_col[m];
    }

    T hN[CPT], zN[CPT], nN[CPT], qxN[CPT], qyN[CPT];
    auto load_row = [&](int k) {
        if (loads && k >= -kHalo && k < ny + kHalo) {
            const long long o = (long long)(k + kHalo) * P;
            ldv<T, CPT>(at_byte(in_space<GA>(h_in) + o, boff), hN);
            ldv<T, CPT>(at_byte(in_space<GA>(a.z) + o, boff), zN);
            ldv<T, CPT>(at_byte(in_space<GA>(a.n) + o, boff), nN);
            ldv<T, CPT>(at_byte(in_space<GA>(qx_in) + o, boff), qxN);
            ldv<T, CPT>(at_byte(in_space<GA>(qy_in) + o, boff), qyN);
        } else {
#pragma unroll
            for (int m = 0; m < CPT; ++m) hN[m] = zN[m] = nN[m] = qxN[m] = qyN[m] = T(0);
        }
    };
    // active-tile flag of an emitted row (ro: its row index, hold: its depth before the step)
    auto mark = [&](int ro, const T (&hv)[CPT], const T (&hold)[CPT], const T (&qxv)[CPT],
                    const T (&qyv)[CPT]) {
        if (ro >= 0 && ro < ny) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                if (store_col[m])
                    moved = moved || !(hv[m] <= T(0)) || hv[m] != hold[m] || qxv[m] != T(0) ||
                            qyv[m] != T(0);
                if (G.west_face[m]) moved = moved || qxv[m] != T(0);
            }
        } else if (ro == -1 && south_chunk) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (store_col[m]) moved = moved || qyv[m] != T(0);
        }
    };
    auto store_row = [&](int r, const T (&hv)[CPT], const T (&qxv)[CPT], const T (&qyv)[CPT]) {
        const long long o = (long long)(r + kHalo) * P;
        auto* const ho = in_space<GA>(h_out) + o;
        auto* const qxr = in_space<GA>(qx_out) + o;
        auto* const qyr = in_space<GA>(qy_out) + o;
        if (all_store) {
            stv<T, CPT, true>(at_byte(ho, boff), hv);
            stv<T, CPT, true>(at_byte(qxr, boff), qxv);
            stv<T, CPT, true>(at_byte(qyr, boff), qyv);
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

    Marcher<T, CPT> MA, MB;
    MA.reset();
    MB.reset();
    T zd1[CPT], zd2[CPT], nd1[CPT], nd2[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) zd1[m] = zd2[m] = nd1[m] = nd2[m] = T(0);

    // FP32 without active tiles (where the registers allow): an output row is
    // stored at the start of the next row's turn, before that turn's loads, so
    // that waiting for the loads covers the stores too instead of stalling on
    // stores issued just before (about 2 % on the two-step launch).
    constexpr bool kDefer = sizeof(T) == 4 && !ACT && CPT <= 2;
    T sh[CPT], sqx[CPT], sqy[CPT];
    int srow = 0;
    bool spend = false;
    auto put_row = [&](int r, const T (&hv)[CPT], const T (&qxv)[CPT], const T (&qyv)[CPT]) {
        if constexpr (kDefer) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                sh[m] = hv[m]; sqx[m] = qxv[m]; sqy[m] = qyv[m];
            }
            srow = r;
            spend = true;
        } else {
            store_row(r, hv, qxv, qyv);
        }
    };

    const int kb = two ? j0 - 4 : j0 - 2;
    const int ke = two ? j1 + 3 : j1 + 1;
    load_row(kb);
    for (int k = kb; k <= ke; ++k) {
        T h0[CPT], z0[CPT], n0[CPT], qx0[CPT], qy0[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            h0[m] = hN[m]; z0[m] = zN[m]; n0[m] = nN[m]; qx0[m] = qxN[m]; qy0[m] = qyN[m];
        }
        if (kDefer && spend) {
            store_row(srow, sh, sqx, sqy);
            spend = false;
        }
        if (k < ke) load_row(k + 1);
        T hA[CPT], qxA[CPT], qyA[CPT], holdA[CPT];
        if constexpr (ACT) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) holdA[m] = MA.h2[m];
        }
        MA.row(a, KA, G, k, h0, z0, n0, qx0, qy0, hA, qxA, qyA);
        T zr[CPT], nr[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            zr[m] = zd2[m]; nr[m] = nd2[m];
            zd2[m] = zd1[m]; nd2[m] = nd1[m];
            zd1[m] = z0[m]; nd1[m] = n0[m];
        }
        const int ra = k - 2;
        const bool a_item = (ra >= j0 && ra < j1);
        if constexpr (ACT) {
            if (two ? (ra >= j0 - 2 && ra < j1 + 2) : (a_item || (ra == -1 && south_chunk)))
                mark(ra, hA, holdA, qxA, qyA);
        }
        if (!two) {
            if (a_item) put_row(ra, hA, qxA, qyA);
            row_books<T, CPT>(a, G, store_col, ra, a_item, south_chunk, hA, qxA, qyA, true, hbA,
                              outA);
            continue;
        }
        row_books<T, CPT>(a, G, store_col, ra, a_item, south_chunk, hA, qxA, qyA, false, hbA, outA);
        if (ra < j0 - 2) continue;
        const bool ra_real = (ra >= 0 && ra < ny);
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            if (!ra_real || G.outside[m]) hA[m] = qxA[m] = qyA[m] = T(0);
        T hB[CPT], qxB[CPT], qyB[CPT], holdB[CPT];
        if constexpr (ACT) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) holdB[m] = MB.h2[m];
        }
        MB.row(a, KB, G, ra, hA, zr, nr, qxA, qyA, hB, qxB, qyB);
        const int rb = ra - 2;
        const bool b_item = (rb >= j0 && rb < j1);
        if constexpr (ACT) {
            if (b_item || (rb == -1 && south_chunk)) mark(rb, hB, holdB, qxB, qyB);
        }
        if (b_item) put_row(rb, hB, qxB, qyB);
        row_books<T, CPT>(a, G, store_col, rb, b_item, south_chunk, hB, qxB, qyB, true, hbB, outB);
    }
    if (kDefer && spend) store_row(srow, sh, sqx, sqy);
}

template <typename T>
__device__ __forceinline__ void step_consts(const StepArgs<T>& a, double dt, StepK<T>& K) {
    K.dt = (T)dt;
    K.gdt = T(a.g) * K.dt;
    K.inv_dx = T(1) / T(a.dx);
    K.h_eps = T(a.h_eps);
    K.qin = nullptr;
    K.W = 0.0;
    K.inflow_on = 0;
}

template <typename T>
__device__ __forceinline__ void inflow_consts(const StepArgs<T>& a, double t, StepK<T>& K) {
    const double Q = hydrograph<T>(a, t);
    if (Q > 0.0) {
        K.W = inflow_level(a.in_z, a.in_k, a.in_count, a.dx, Q);
        K.inflow_on = 1;
    }
}

// Must item (s, c) be computed by a launch that writes generation gen
// (active-tile skipping)?  Over two steps a cell depends on the cells up to
// two away, which lie in the item and the 8 items around it (items are at
// least two cells tall and wide), so it may be skipped when those nine items
// were dry and unchanged in generation gen - 1, and the item itself also in
// gen - 2 (its output buffer still holds that state).  A redo reads the same
// slots as the launch it replaces and so skips the same items, whose output
// buffer that launch left untouched.  Items whose loaded region meets an
// inflow face are always computed.
template <typename T>
__device__ __forceinline__ bool item_needed2(const StepArgs<T>& a, int s, int c, long long gen) {
    const int lane = threadIdx.x & 63;
    int v = 0;
    if (lane < 10) {
        int ss = s + lane % 3 - 1, cc = c + lane / 3 - 1;
        long long sl = (gen + 2) % 3;  // generation gen - 1
        if (lane == 9) {
            ss = s;
            cc = c;
            sl = (gen + 1) % 3;        // generation gen - 2
        }
        if (ss >= 0 && ss < a.nstrips && cc >= 0 && cc < a.nchunks)
            v = a.act[sl * a.act_stride + (long long)cc * a.nstrips + ss];
    }
    return __ballot(v != 0) != 0ull;
}

// GA: row pointers typed global (they come from memory in the batch kernel)
template <typename T, int CPT, bool ACT, bool GA>
__device__ __forceinline__ void tile2_item(const Step2Args<T>& A, const Plan2& P, int item) {
    const StepArgs<T>& a = A.a;
    constexpr int WL = 64 * CPT, WO = WL - 8;
    const int s = item % a.nstrips, c = item / a.nstrips;
    const int j0 = c * a.rows, j1 = min(j0 + a.rows, a.ny);
    // the plan is the same in every lane; keep what steers control flow scalar
    const bool two = __builtin_amdgcn_readfirstlane(P.mode) != 1;
    const bool inflow = needs_inflow<T>(a, s, j0, j1, WO, WL);
    if constexpr (ACT) {
        if (!inflow && !item_needed2<T>(a, s, c, P.gen)) {
            // nothing moves: no deeper cell, no outflow, flag 0
            if ((threadIdx.x & 63) == 0) {
                a.act[(P.gen % 3) * a.act_stride + item] = 0;
                const int slot = part_slot<T>(a, s, c);
                if (slot >= 0) {
                    A.part_a[A.phase & 1][slot] = 0.0;
                    A.part_b[A.phase & 1][slot] = 0.0;
                }
            }
            return;
        }
    }
    StepK<T> KA, KB;
    step_consts<T>(a, P.dt_a, KA);
    step_consts<T>(a, P.dt_b, KB);
    if (inflow) {
        inflow_consts<T>(a, P.ck0.t, KA);
        if (two) inflow_consts<T>(a, P.ck1.t, KB);
    }
    const bool in1 = __builtin_amdgcn_readfirstlane(P.in) != 0;
    typename Ord<T>::U hbA = 0, hbB = 0;
    double oA = 0.0, oB = 0.0;
    bool moved = false;
    step2_item<T, CPT, ACT, GA>(a, in1 ? A.h[1] : A.h[0], in1 ? A.qx[1] : A.qx[0],
                            in1 ? A.qy[1] : A.qy[0], in1 ? A.h[0] : A.h[1],
                            in1 ? A.qx[0] : A.qx[1], in1 ? A.qy[0] : A.qy[1], KA, KB, two, s, j0,
                            j1, hbA, hbB, oA, oB, moved);
    hbA = wave_max_key(hbA);
    if (two) hbB = wave_max_key(hbB);
    const int slot = part_slot<T>(a, s, c);
    if (slot >= 0) {
        oA = wave_sum(oA);
        if (two) oB = wave_sum(oB);
    }
    bool any_moved = false;
    if constexpr (ACT) any_moved = __ballot(moved) != 0ull;
    if ((threadIdx.x & 63) == 0) {
        if constexpr (ACT) a.act[(P.gen % 3) * a.act_stride + item] = any_moved ? 1 : 0;
        unsigned long long* hm = a.ctl->hm2 + 2 * (A.phase % 3);
        if (two) {
            if (hbA) atomicMax(&hm[0], (unsigned long long)hbA);
            if (hbB) atomicMax(&hm[1], (unsigned long long)hbB);
        } else if (hbA) {
            atomicMax(&hm[1], (unsigned long long)hbA);
        }
        if (slot >= 0) {
            A.part_a[A.phase & 1][slot] = oA;
            if (two) A.part_b[A.phase & 1][slot] = oB;
        }
    }
}

template <typename T, int CPT, bool ACT>
// FP32 at 2 cells per lane: hold the register budget of three waves per SIMD
__global__ __launch_bounds__(256, (sizeof(T) == 4 && CPT == 2) ? 3 : 1) void k_step2(Step2Args<T> A) {
    const Plan2 P = make_plan<T>(A);
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) clock2_wave<T>(A, P);
        return;
    }
    if (P.mode == 0) return;
    // XCD-aware order, as in the single-step kernel: XCD x runs blocks
    // b % 8 == x and gets one contiguous horizontal band of work items.
    const int nblk = gridDim.x - 1, b = blockIdx.x - 1;
    const int xcd = b & 7, q8 = nblk >> 3, r8 = nblk & 7;
    const int lin = xcd * q8 + min(xcd, r8) + (b >> 3);
    // the wave index is uniform across the wave: keep it (and everything
    // derived from it: strip, rows, loop counter, border tests) scalar
    const int wave = lin * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= A.a.nstrips * A.a.nchunks) return;
    tile2_item<T, CPT, ACT, false>(A, P, wave);
}

// Persistent batch with two steps per queue entry: the two-step launches of
// many members in one launch.  Per XCD the queue holds, launch after launch,
// for each member its clock entry and its two-step work items; an entry of a
// member's launch l waits only until that member's launch l - 1 is complete.
// Every entry derives the launch's plan from the member's device clock, as the
// waves of a two-step launch do, so each member makes exactly the launches
// (steps, speculated second steps, redos) of its own two-step run, and its
// state is bitwise that of stepping it alone.  Queue, hand-over between
// launches and progress argument as in k_batch (flood_kernels.hip): an entry
// waits only for entries of lower queue index, which running waves took
// before it.
// (FP32: two waves per SIMD; with three the queue's state spills the row
// pointers of the marchers to scratch)
template <typename T, int CPT>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) void k_batch2(
    Batch2Args<T> B, const BatchScen2<T>* __restrict__ scen) {
    // scen is not written during the launch: its loads may be repeated instead of held
    const int lane = threadIdx.x & 63;
    const int x = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15);  // XCC_ID
    if (x >= B.nxcc) return;
    const int m_lo = B.xbegin[x], m_hi = B.xbegin[x + 1];
    if (m_lo >= m_hi) return;
    const int per = B.per_launch[x];
    const unsigned long long total = (unsigned long long)per * (unsigned long long)B.nlaunch;
    for (;;) {
        unsigned long long q = 0;
        if (lane == 0) q = atomicAdd(&B.next[x], 1ull);
        q = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(q >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((unsigned)q);
        if (q >= total) break;
        const long long l = (long long)(q / (unsigned long long)per);
        const int r = (int)(q - (unsigned long long)l * per);
        int lo = m_lo, hi = m_hi - 1;      // member with first <= r, largest such
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (scen[mid].first <= r) lo = mid; else hi = mid - 1;
        }
        const int m = lo;
        const BatchScen2<T>& S = scen[m];
        const int e = r - S.first;
        if (l > 0) {
            const unsigned long long need = (unsigned long long)l * (unsigned long long)(S.items + 1);
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
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        const Step2Args<T>& A = S.a2[l == B.nlaunch - 1 ? 1 : 0][(int)((B.l0 + l) % 6)];
        const Plan2 P = make_plan<T>(A);
        if (e == 0) clock2_wave<T>(A, P);
        else if (P.mode != 0) tile2_item<T, CPT, false, true>(A, P, e - 1);
        __builtin_amdgcn_s_waitcnt(0);
        __asm__ volatile("" ::: "memory");
        if (lane == 0) atomicAdd(&B.done[m], 1ull);
    }
}

template <typename T>
__global__ void k_enter2(StepArgs<T> a, int cur, long long target, int keep_gen) {
    if (threadIdx.x != 0) return;
    DevCtl* ctl = a.ctl;
    Clock2 S;
    S.ck = ctl->clk[a.phase & 1];
    S.back = S.ck;
    S.mid = S.ck;
    S.dt_a = S.dt_b = 0.0;
    S.vsteps = 0;
    S.cur = cur;
    S.pending = 0;
    S.nclose = 0;
    S.pad = 0;
    S.gen = keep_gen ? ctl->gen2 : 0;
    ctl->c2[0] = S;
    for (int q = 0; q < 4; ++q) ctl->hm2[q] = 0ull;
    ctl->hm2[4] = 0ull;
    ctl->hm2[5] = ctl->hmax[a.phase % 3];
    ctl->target2 = target;
}

template <typename T>
__global__ void k_leave2(StepArgs<T> a, Step2Args<T> A, long long launches) {
    const int lane = threadIdx.x & 63;
    DevCtl* ctl = a.ctl;
    const Clock2 S = ctl->c2[launches & 1];
    const int pl = (int)((launches - 1) % 6);
    ClockSlot ck = S.ck;
    if (S.nclose >= 1) {
        double so = partial_sum<T>(A.part_a[pl & 1], A.a.npart);
        ck.v_out = ck.v_out + S.dt_a * a.dx * so;
        if (S.nclose == 2) {
            so = partial_sum<T>(A.part_b[pl & 1], A.a.npart);
            ck.v_out = ck.v_out + S.dt_b * a.dx * so;
        }
    }
    ck.dt_prev = 0.0;
    inflow_solve<T>(a, hydrograph<T>(a, ck.t), const_cast<T*>(a.qin));
    for (int q = lane; q < a.npart; q += 64) const_cast<double*>(a.part_prev)[q] = 0.0;
    if (lane == 0) {
        ctl->clk[a.phase & 1] = ck;
        ctl->hmax[a.phase % 3] = ctl->hm2[2 * (pl % 3) + 1];
        ctl->hmax[(a.phase + 1) % 3] = 0ull;
        ctl->gen2 = S.gen;
    }
}

// ------------------------------------------------------------ launchers
int strip_width2(int cpt) { return 64 * cpt - 8; }

template <typename T, int CPT>
static hipError_t launch_step2_cpt(const Step2Args<T>& a, hipStream_t s) {
    const long long items = (long long)a.a.nstrips * a.a.nchunks;
    const unsigned blocks = (unsigned)(1 + (items + 3) / 4);
    if (a.a.act) {
        // the flags of every item must fit in a slot; the skip test needs
        // items at least two rows tall
        if (items > a.a.act_stride || a.a.rows < 2) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step2<T, CPT, true>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_step2<T, CPT, false>), dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_step2(const Step2Args<T>& a, int cpt, hipStream_t s) {
    switch (cpt) {
    case 1: return launch_step2_cpt<T, 1>(a, s);
    case 2: return launch_step2_cpt<T, 2>(a, s);
    case 4: return sizeof(T) == 4 ? launch_step2_cpt<T, 4>(a, s) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_enter2(const StepArgs<T>& single, long long target, int keep_gen, hipStream_t s) {
    // the single-step state at counter n lives in buffer n % 2, i.e. the
    // buffer of single.h_in; phase = n % 6
    hipLaunchKernelGGL((k_enter2<T>), dim3(1), dim3(64), 0, s, single, single.phase & 1, target,
                       keep_gen);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_leave2(const StepArgs<T>& single, const Step2Args<T>& a2, long long launches,
                         hipStream_t s) {
    if (launches < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_leave2<T>), dim3(1), dim3(64), 0, s, single, a2, launches);
    return hipGetLastError();
}

template <typename T, int CPT>
static hipError_t launch_batch2_cpt(const Batch2Args<T>& b, int device, hipStream_t s, int* blocks_out) {
    int per_cu = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch2<T, CPT>, 256, 0);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    const int blocks = std::max(1, per_cu) * ncu;
    if (blocks_out) *blocks_out = blocks;
    // an ordinary launch: the queue needs no co-residency (see k_batch2)
    hipLaunchKernelGGL((k_batch2<T, CPT>), dim3(blocks), dim3(256), 0, s, b, b.scen);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch2(const Batch2Args<T>& b, int cpt, int device, hipStream_t s, int* blocks_out) {
    switch (cpt) {
    case 1: return launch_batch2_cpt<T, 1>(b, device, s, blocks_out);
    case 2: return launch_batch2_cpt<T, 2>(b, device, s, blocks_out);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_batch2<float>(const Batch2Args<float>&, int, int, hipStream_t, int*);
template hipError_t launch_batch2<double>(const Batch2Args<double>&, int, int, hipStream_t, int*);
template hipError_t launch_step2<float>(const Step2Args<float>&, int, hipStream_t);
template hipError_t launch_step2<double>(const Step2Args<double>&, int, hipStream_t);
template hipError_t launch_enter2<float>(const StepArgs<float>&, long long, int, hipStream_t);
template hipError_t launch_enter2<double>(const StepArgs<double>&, long long, int, hipStream_t);
template hipError_t launch_leave2<float>(const StepArgs<float>&, const Step2Args<float>&, long long,
                                         hipStream_t);
template hipError_t launch_leave2<double>(const StepArgs<double>&, const Step2Args<double>&,
                                          long long, hipStream_t);

}  // namespace flood
