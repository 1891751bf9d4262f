// Several flood steps per launch (Methods, "Shallow Water Equations", eqs. 3-6).
//
// The single-step kernel reads the state once and writes it once per step,
// so a step costs at least 32 bytes per cell of HBM traffic.  Here one wave
// runs K row marchers (K = 2 or 3) on its strip: each consumes the rows the
// one before it emits, still in registers, so K steps cost one read and one
// write of the state.  A strip loads 64*CPT columns and outputs 64*CPT - 4K
// of them (each step needs two halo columns on each side).
//
// The dt of every step after a launch's first depends on the deepest cell of
// the state before it, a grid-wide maximum that exists only once the launch
// has ended.  The launch therefore runs those steps with the dt they would
// have if that maximum were small (the fixed dt, or dt_max, in both cases cut
// at t_end); the next launch computes the true dts from the maxima the tiles
// recorded and, at the first that differs, redoes the launch up to that step,
// with the right dt, from the launch's input, which the ping-pong buffers
// still hold.  Either way every step uses exactly the dt, inflow and
// arithmetic of the single-step kernel, so the paths give the same bits.
// When the CFL bound is close to active a launch makes fewer steps, down to
// one.  With a fixed dt (the paper's runs) a guess fails only on a non-finite
// state.
//
// Every wave derives the launch's plan from the device clock, so the number
// of steps a launch makes is decided on the device; launches past the
// requested count do nothing.
#include <math.h>

#include <algorithm>

#include "flood_march.h"

namespace flood {

// What a launch does; every wave computes the same plan.
struct FusedPlan {
    int ns;                 // steps the launch makes (0: nothing)
    int redo;               // it redoes the last launch up to that launch's first wrong dt
    int in;                 // buffer read; the launch writes buffer in ^ 1
    int verified;           // the state claimed by the last launch holds
    int spec;               // first step whose dt is speculated (ns: none)
    ClockSlot ck0;          // clock at the start of the launch
    double t[kFuseMax];     // time at the start of each step
    double dt[kFuseMax];
    int last[kFuseMax], done[kFuseMax], nonfin[kFuseMax];  // step_dt's flags (the last step of a redo; every step otherwise)
    long long gen;          // generation of the state the launch writes (a redo: the one it replaces)
};

// Whether to run step s (>= 1) of a launch with a speculated dt: always with a
// fixed dt, and with the CFL clock when the bound is clear of dt_max: the
// deepest cell may deepen by 2 % per step before s without making it active.
// A guess that fails costs one redo launch; a launch that makes fewer steps
// costs another pass over the state, so a narrow margin pays (deep, wet grids
// run at dt_max with the bound close by).
template <typename T>
__device__ __forceinline__ bool spec_room(const StepArgs<T>& a, unsigned long long hb, int s) {
    if (a.dt_fixed > 0.0) return true;
    const double hm = Ord<T>::value(hb);
    return !(hm > 0.0) || a.alpha * a.dx / sqrt(a.g * hm) >= (1.0 + 0.02 * s) * a.dt_max;
}

template <typename T>
__device__ __forceinline__ FusedPlan make_plan(const FusedArgs<T>& A) {
    const StepArgs<T>& a = A.a;
    const DevCtl* ctl = a.ctl;
    const FusedClock& S = ctl->cf[A.phase & 1];
    const unsigned long long* hm = ctl->hmf + kFuseMax * ((A.phase + 2) % 3);
    const double t_end = ctl->t_end;
    FusedPlan P;
    P.ns = 0;
    P.redo = 0;
    P.verified = 1;
#pragma unroll
    for (int s = 0; s < kFuseMax; ++s) {
        P.t[s] = P.dt[s] = 0.0;
        P.last[s] = P.done[s] = P.nonfin[s] = 0;
    }
    // check the last launch's speculated dts in order; the first that differs
    // from the dt of the state before its step is redone
    int bad = 0, lt = 0, dn = 0, nf = 0;
    double dt_true = 0.0;
    if (S.pending) {
#pragma unroll
        for (int s = 1; s < kFuseMax; ++s) {
            if (bad || s < S.spec || s >= S.nclose) continue;
            int l1 = 0, d1 = 0, n1 = 0;
            const double d = step_dt<T>(a, S.mid[s - 1], hm[s - 1], t_end, l1, d1, n1);
            if (d != S.dt[s]) {
                bad = s;
                dt_true = d;
                lt = l1;
                dn = d1;
                nf = n1;
            }
        }
    }
    if (bad) {
        P.verified = 0;
        P.redo = 1;
        P.ns = bad + 1;
        P.spec = P.ns;
        P.gen = S.gen;
        P.in = S.cur ^ 1;
        P.ck0 = S.back;
        P.t[0] = S.back.t;
#pragma unroll
        for (int s = 1; s < kFuseMax; ++s)
            if (s <= bad) P.t[s] = S.mid[s - 1].t;
#pragma unroll
        for (int s = 0; s < kFuseMax; ++s)
            if (s < bad) P.dt[s] = S.dt[s];
        // (the clock after each repeated step is the last launch's)
#pragma unroll
        for (int s = 1; s < kFuseMax; ++s)
            if (s == bad) {
                P.dt[s] = dt_true;
                P.last[s] = lt;
                P.done[s] = dn;
                P.nonfin[s] = nf;
            }
        return P;
    }
    P.in = S.cur;
    P.gen = S.gen + 1;
    P.ck0 = S.ck;
    P.spec = 0;
    const long long remaining = ctl->targetf - S.vsteps;
    if (A.resolve || remaining <= 0) return P;
    const unsigned long long hend = hm[kFuseMax - 1];
    ClockSlot c = S.ck;
    P.t[0] = c.t;
    P.dt[0] = step_dt<T>(a, c, hend, t_end, P.last[0], P.done[0], P.nonfin[0]);
    P.ns = 1;
    const long long nmax = remaining < (long long)A.K ? remaining : (long long)A.K;
#pragma unroll
    for (int s = 1; s < kFuseMax; ++s) {
        if (P.ns != s || s >= nmax || !spec_room<T>(a, hend, s)) continue;
        c.t = P.last[s - 1] ? t_end : c.t + P.dt[s - 1];
        c.nonfinite = P.nonfin[s - 1] ? 1 : 0;
        P.t[s] = c.t;
        P.dt[s] = step_dt<T>(a, c, 0ull, t_end, P.last[s], P.done[s], P.nonfin[s]);
        P.ns = s + 1;
    }
    P.spec = P.ns > 1 ? 1 : P.ns;
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

// The clock wave of a multi-step launch: closes the outflow of the last
// launch once its state is known to hold, advances the clock over this
// launch's steps and publishes the next slot.
template <typename T>
__device__ __forceinline__ void clock_wave_fused(const FusedArgs<T>& A, const FusedPlan& P) {
    const StepArgs<T>& a = A.a;
    const int lane = threadIdx.x & 63;
    DevCtl* ctl = a.ctl;
    const FusedClock S = ctl->cf[A.phase & 1];
    const int gp = (A.phase + 2) % 3, g = A.phase % 3, gn = (A.phase + 1) % 3;
    const int pp = (A.phase + 1) & 1;  // parity of the last launch
    const double t_end = ctl->t_end;
    ClockSlot base = P.ck0;
    if (P.verified) {
#pragma unroll
        for (int s = 0; s < kFuseMax; ++s)
            if (s < S.nclose) {
                const double so = partial_sum<T>(A.part[s][pp], a.npart);
                base.v_out = base.v_out + S.dt[s] * a.dx * so;
            }
    }
    FusedClock N = S;
    if (P.ns == 0) {
        N.ck = base;
        N.nclose = 0;
        N.pending = 0;
        if (lane == 0) {
            for (int q = 0; q < kFuseMax; ++q) ctl->hmf[kFuseMax * g + q] = ctl->hmf[kFuseMax * gp + q];
        }
    } else {
        ClockSlot c = base;
#pragma unroll
        for (int s = 0; s < kFuseMax; ++s) {
            if (s >= P.ns) continue;
            if (P.redo && s < P.ns - 1) {
                c = S.mid[s];  // a step the redo repeats with the same dt
            } else {
                const double si = inflow_sum<T>(a, c.t);
                c = advance_clock(c, P.dt[s], P.last[s], P.done[s], P.nonfin[s], si, a.dx, t_end);
            }
            if (s < kFuseMax - 1) N.mid[s] = c;
            N.dt[s] = P.dt[s];
        }
        N.back = base;
        N.ck = c;
        N.cur = P.in ^ 1;
        N.gen = P.gen;
        N.nclose = P.ns;
        N.spec = P.spec;
        N.pending = P.spec < P.ns ? 1 : 0;
        // a redo replaces the steps of the launch it repeats
        N.vsteps = P.redo ? S.vsteps - S.nclose + P.ns : S.vsteps + P.ns;
    }
    if (lane == 0) {
        for (int q = 0; q < kFuseMax; ++q) ctl->hmf[kFuseMax * gn + q] = 0ull;
        ctl->cf[(A.phase + 1) & 1] = N;
    }
}

// Whether the waves of strip s, rows [j0, j1) meet an inflow face in a
// launch of up to k steps (loaded rows j0 - 2k .. j1 + 2k - 1): those solve
// eq. (6) themselves (the later steps' times are not known before the launch).
template <typename T>
__device__ __forceinline__ bool needs_inflow(const StepArgs<T>& a, int s, int j0, int j1, int wo,
                                             int wl, int k) {
    if (a.in_side < 0 || a.in_count <= 0) return false;
    const int f = a.in_first, e = a.in_first + a.in_count;
    const int c0 = s * wo - kHalo;  // real column of the strip's first loaded cell
    const int r = 2 * k;
    switch (a.in_side) {
    case SIDE_W: return s == 0 && j0 - r < e && j1 + r > f;
    case SIDE_E: return a.nx - 1 >= c0 && a.nx - 1 < c0 + wl && j0 - r < e && j1 + r > f;
    case SIDE_S: return j0 <= r && c0 < e && c0 + wl > f;
    default: return j1 + r - 1 >= a.ny && c0 < e && c0 + wl > f;
    }
}

// One work item of a launch of NS steps (1 <= NS <= K) in the tiling of K
// steps per launch: strip s, rows [j0, j1).  Row k enters marcher 0; the row
// marcher t emits (k - 2 - 2t) enters marcher t + 1 with the bed and
// roughness of that row; the last marcher's rows are the output.  Values of
// an emitted row outside the grid are replaced by zeros before the next
// marcher, which is what the single-step kernel reads from the halo there.
// With ACT, `moved` records whether any row of the item that either step
// emits holds water (h > 0, or NaN), changed its depth in that step, or
// carries a non-zero discharge on a face the item stores (border faces
// included); rows of earlier steps beyond the item count too (conservative).
// hb[t], out[t]: deepest new depth and outflow of step t in the item.
// EDGE = false: an interior item, whose loaded rows and columns meet no
// border of the grid (strip neither the first nor the one holding the last
// column, rows j0 - 2K .. j1 + 2K - 1 within 1 .. ny - 1): the marchers and
// the bookkeeping drop their border code.
template <typename T, int CPT, int K, int NS, bool ACT, bool GA, bool EDGE>
__device__ __forceinline__ void fused_item(const StepArgs<T>& a, const T* __restrict__ h_in,
                           const T* __restrict__ qx_in, const T* __restrict__ qy_in,
                           T* __restrict__ h_out, T* __restrict__ qx_out, T* __restrict__ qy_out,
                           const StepK<T> (&KS)[kFuseMax], int s, int j0, int j1,
                           typename Ord<T>::U (&hb)[kFuseMax], double (&out)[kFuseMax],
                           bool& moved) {
    static_assert(NS >= 1 && NS <= K && K <= kFuseMax, "steps per launch");
    constexpr int WL = 64 * CPT;  // loaded columns
    constexpr int WO = WL - 4 * K;  // output columns (strip 0: 2K - 2 more on the left)
    const int lane = threadIdx.x & 63;
    const int nx = a.nx, ny = a.ny;
    const long long P = a.pitch;
    const int pcol = s * WO + lane * CPT;
    const unsigned ucol = (unsigned)pcol;  // lane offset from a row's start (row pointers are uniform)
    const unsigned boff = ucol * (unsigned)sizeof(T);
    const bool loads = pcol < nx + 2 * kHalo;
    const StripGeo<CPT> G = strip_geo<CPT>(nx, s, WO, WL, lane);
    const bool south_chunk = (j0 == 0);
    const int lo = (s == 0) ? kHalo : 2 * K;

    bool store_col[CPT];
    bool all_store = true, any_store = false;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int l = lane * CPT + m;
        store_col[m] = (l >= lo && l < WL - 2 * K && G.i0 + m < nx);
        all_store = all_store && store_col[m];
        any_store = any_store || store_col[m];
    }

    T hN[CPT], zN[CPT], nN[CPT], qxN[CPT], qyN[CPT];
    auto load_row = [&](int k) {
        if (!EDGE || (loads && k >= -kHalo && k < ny + kHalo)) {
            const long long o = (long long)(k + kHalo) * P;
            ldv<T, CPT>(at_byte(wave_uniform_ptr(in_space<GA>(h_in) + o), boff), hN);
            ldv<T, CPT>(at_byte(wave_uniform_ptr(in_space<GA>(a.z) + o), boff), zN);
            ldv<T, CPT>(at_byte(wave_uniform_ptr(in_space<GA>(a.n) + o), boff), nN);
            ldv<T, CPT>(at_byte(wave_uniform_ptr(in_space<GA>(qx_in) + o), boff), qxN);
            ldv<T, CPT>(at_byte(wave_uniform_ptr(in_space<GA>(qy_in) + o), boff), qyN);
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
        auto* const ho = wave_uniform_ptr(in_space<GA>(h_out) + o);
        auto* const qxr = wave_uniform_ptr(in_space<GA>(qx_out) + o);
        auto* const qyr = wave_uniform_ptr(in_space<GA>(qy_out) + o);
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

    Marcher<T, CPT> M[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) M[t].reset();
    // bed and roughness of the rows entered 1 .. 2 (NS - 1) rows ago: marcher
    // t takes row k - 2t
    constexpr int ND = NS > 1 ? 2 * (NS - 1) : 1;
    T zd[ND][CPT], nd[ND][CPT];
#pragma unroll
    for (int q = 0; q < ND; ++q)
#pragma unroll
        for (int m = 0; m < CPT; ++m) zd[q][m] = nd[q][m] = T(0);

    // FP32 without active tiles (where the registers allow): an output row is
    // stored at the start of the next row's turn, before that turn's loads, so
    // that waiting for the loads covers the stores too instead of stalling on
    // stores issued just before (about 2 % on the two-step launch).
    constexpr bool kDefer = sizeof(T) == 4 && !ACT && CPT <= 2 && K <= 2;
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

    // bookkeeping of an emitted row of step t (an interior item has no border
    // faces and no outflow: only its deepest cell)
    auto books = [&](auto tc, int r, bool in_item, const T (&hv)[CPT], const T (&qxv)[CPT],
                     const T (&qyv)[CPT], bool keep_edges) {
        constexpr int t = decltype(tc)::value;
        if constexpr (EDGE) {
            row_books<T, CPT>(a, G, store_col, r, in_item, south_chunk, hv, qxv, qyv, keep_edges,
                              hb[t], out[t]);
        } else if (in_item) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (store_col[m]) {
                    const typename Ord<T>::U b = Ord<T>::key(hv[m]);
                    hb[t] = b > hb[t] ? b : hb[t];
                }
        }
    };

    const int kb = j0 - 2 * NS;
    const int ke = j1 + 2 * NS - 1;
    load_row(kb);
    for (int k = kb; k <= ke; ++k) {
        // the prefetched row first, on every path: a wait the compiler places
        // after the deferred stores (where the paths with and without them
        // join) would wait for the stores too
        if constexpr (kDefer) wait_vector_memory();
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
        T hc[CPT], qxc[CPT], qyc[CPT], hold[CPT];
        if constexpr (ACT) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) hold[m] = M[0].h2[m];
        }
        M[0].template row<EDGE>(a, KS[0], G, k, h0, z0, n0, qx0, qy0, hc, qxc, qyc);
        // bed and roughness for the later marchers, then shift the delay line
        T zt[NS][CPT], nt[NS][CPT];
#pragma unroll
        for (int t = 1; t < NS; ++t)
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                zt[t][m] = zd[2 * t - 1][m];
                nt[t][m] = nd[2 * t - 1][m];
            }
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = ND - 1; q > 0; --q)
#pragma unroll
                for (int m = 0; m < CPT; ++m) {
                    zd[q][m] = zd[q - 1][m];
                    nd[q][m] = nd[q - 1][m];
                }
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                zd[0][m] = z0[m];
                nd[0][m] = n0[m];
            }
        }
        int r = k - 2;  // the row the marcher just run emitted
        bool go = true;
        // the chain with compile-time step indices (a runtime loop over the
        // marchers would put their state in private memory)
        static_for<0, NS>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            if (!go) return;
            if constexpr (t > 0) {
                if constexpr (EDGE) {
                    const bool real = (r >= 0 && r < ny);
#pragma unroll
                    for (int m = 0; m < CPT; ++m)
                        if (!real || G.outside[m]) hc[m] = qxc[m] = qyc[m] = T(0);
                }
                if constexpr (ACT) {
#pragma unroll
                    for (int m = 0; m < CPT; ++m) hold[m] = M[t].h2[m];
                }
                T hn[CPT], qxn[CPT], qyn[CPT];
                M[t].template row<EDGE>(a, KS[t], G, r, hc, zt[t], nt[t], qxc, qyc, hn, qxn, qyn);
#pragma unroll
                for (int m = 0; m < CPT; ++m) {
                    hc[m] = hn[m]; qxc[m] = qxn[m]; qyc[m] = qyn[m];
                }
                r -= 2;
            }
            const bool in_item = (r >= j0 && r < j1);
            if constexpr (t == NS - 1) {
                if constexpr (ACT) {
                    if (in_item || (r == -1 && south_chunk)) mark(r, hc, hold, qxc, qyc);
                }
                if (in_item) put_row(r, hc, qxc, qyc);
                books(tc, r, in_item, hc, qxc, qyc, true);
            } else {
                // rows the later steps of the item need: 2 more per step left
                const int reach = 2 * (NS - 1 - t);
                if constexpr (ACT) {
                    if (r >= j0 - reach && r < j1 + reach) mark(r, hc, hold, qxc, qyc);
                }
                books(tc, r, in_item, hc, qxc, qyc, false);
                if (r < j0 - reach) go = false;  // not yet computed from loaded rows only
            }
        });
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
    K.pre = false;
    K.b_in = K.b_out = T(0);
}

template <typename T>
__device__ __forceinline__ void inflow_consts(const StepArgs<T>& a, double t, StepK<T>& K) {
    const double Q = hydrograph<T>(a, t);
    if (Q > 0.0) {
        K.W = inflow_level(a.in_z, a.in_k, a.in_count, a.dx, Q);
        K.inflow_on = 1;
    }
}

// Must item (s, c) be computed by a launch of K = 2 or 3 steps that writes
// generation gen (active-tile skipping)?  Over K steps a cell depends on the
// cells up to K away, which lie in the item and the 8 items around it (items
// are at least K cells tall and wide), so it may be skipped when those nine
// items were dry and unchanged in generation gen - 1, and the item itself also
// in gen - 2 (its output buffer still holds that state).  A redo reads the same
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

// One work item of a multi-step launch in the tiling of K steps per launch.
// GA: row pointers typed global (they come from memory in the batch kernel).
template <typename T, int CPT, int K, bool ACT, bool GA>
__device__ __forceinline__ void fused_tile(const FusedArgs<T>& A, const FusedPlan& P, int item) {
    static_assert(!ACT || K <= 3, "active tiles: two or three steps per launch");
    const StepArgs<T>& a = A.a;
    constexpr int WL = 64 * CPT, WO = WL - 4 * K;
    const int s = item % a.nstrips, c = item / a.nstrips;
    const int j0 = c * a.rows, j1 = min(j0 + a.rows, a.ny);
    // the plan is the same in every lane; keep what steers control flow scalar
    const int ns = __builtin_amdgcn_readfirstlane(P.ns);
    const bool inflow = needs_inflow<T>(a, s, j0, j1, WO, WL, K);
    if constexpr (ACT) {
        if (!inflow && !item_needed2<T>(a, s, c, P.gen)) {
            // nothing moves: no deeper cell, no outflow, flag 0
            if ((threadIdx.x & 63) == 0) {
                a.act[(P.gen % 3) * a.act_stride + item] = 0;
                const int slot = part_slot<T>(a, s, c);
                if (slot >= 0) {
                    for (int t = 0; t < kFuseMax; ++t) A.part[t][A.phase & 1][slot] = 0.0;
                }
            }
            return;
        }
    }
    StepK<T> KS[kFuseMax];
#pragma unroll
    for (int t = 0; t < kFuseMax; ++t) {
        step_consts<T>(a, P.dt[t], KS[t]);
        if (inflow && t < ns) inflow_consts<T>(a, P.t[t], KS[t]);
        // the same in every lane: keep the constants of the marcher chain scalar
        KS[t].dt = wave_uniform(KS[t].dt);
        KS[t].gdt = wave_uniform(KS[t].gdt);
        KS[t].inv_dx = wave_uniform(KS[t].inv_dx);
        KS[t].h_eps = wave_uniform(KS[t].h_eps);
        KS[t].W = wave_uniform(KS[t].W);
        KS[t].inflow_on = wave_uniform(KS[t].inflow_on);
    }
    const bool in1 = __builtin_amdgcn_readfirstlane(P.in) != 0;
    typename Ord<T>::U hb[kFuseMax];
    double out[kFuseMax];
#pragma unroll
    for (int t = 0; t < kFuseMax; ++t) {
        hb[t] = 0;
        out[t] = 0.0;
    }
    bool moved = false;
    const T* hi = in1 ? A.h[1] : A.h[0];
    const T* qxi = in1 ? A.qx[1] : A.qx[0];
    const T* qyi = in1 ? A.qy[1] : A.qy[0];
    T* ho = in1 ? A.h[0] : A.h[1];
    T* qxo = in1 ? A.qx[0] : A.qx[1];
    T* qyo = in1 ? A.qy[0] : A.qy[1];
    // interior items (almost all of a large grid) run without border code
    const bool edge = s == 0 || s * WO - kHalo + WL > a.nx - 1 || j0 - 2 * K < 1 ||
                      j1 + 2 * K - 1 > a.ny - 1;
#define FUSED_ITEM(NSV, EDGEV)                                                                   \
    fused_item<T, CPT, K, NSV, ACT, GA, EDGEV>(a, hi, qxi, qyi, ho, qxo, qyo, KS, s, j0, j1, hb, \
                                                out, moved)
    if (ns == 1) {
        FUSED_ITEM(1, true);
    } else if (K == 2 || ns == 2) {
        if (edge) FUSED_ITEM(2, true);
        else FUSED_ITEM(2, false);
    } else if constexpr (K == 3) {
        if (edge) FUSED_ITEM(3, true);
        else FUSED_ITEM(3, false);
    }
#undef FUSED_ITEM
    const int slot = part_slot<T>(a, s, c);
#pragma unroll
    for (int t = 0; t < kFuseMax; ++t) {
        if (t >= ns) continue;
        hb[t] = wave_max_key(hb[t]);
        if (slot >= 0) out[t] = wave_sum(out[t]);
    }
    bool any_moved = false;
    if constexpr (ACT) any_moved = __ballot(moved) != 0ull;
    if ((threadIdx.x & 63) == 0) {
        if constexpr (ACT) a.act[(P.gen % 3) * a.act_stride + item] = any_moved ? 1 : 0;
        unsigned long long* hm = a.ctl->hmf + kFuseMax * (A.phase % 3);
#pragma unroll
        for (int t = 0; t < kFuseMax; ++t) {
            if (t >= ns) continue;
            // the last step's maximum goes to the last slot
            if (hb[t]) atomicMax(&hm[t == ns - 1 ? kFuseMax - 1 : t], (unsigned long long)hb[t]);
            if (slot >= 0) A.part[t][A.phase & 1][slot] = out[t];
        }
    }
}

// FP32 at 2 cells per lane: hold the register budget of three waves per SIMD
template <typename T, int CPT, int K, bool ACT>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && CPT == 2) ? 3 : 1) void k_fused(FusedArgs<T> A) {
    const FusedPlan P = make_plan<T>(A);
    if (blockIdx.x == 0) {
        if (threadIdx.x < 64) clock_wave_fused<T>(A, P);
        return;
    }
    if (P.ns == 0) return;
    // XCD-aware order, as in the single-step kernel: XCD x runs blocks
    // b % 8 == x and gets one contiguous horizontal band of work items.
    const int nblk = gridDim.x - 1, b = blockIdx.x - 1;
    const int xcd = b & 7, q8 = nblk >> 3, r8 = nblk & 7;
    const int lin = xcd * q8 + min(xcd, r8) + (b >> 3);
    // the wave index is uniform across the wave: keep it (and everything
    // derived from it: strip, rows, loop counter, border tests) scalar
    const int wave = lin * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= A.a.nstrips * A.a.nchunks) return;
    fused_tile<T, CPT, K, ACT, false>(A, P, wave);
}

// Persistent batch with K = 2 or 3 steps per queue entry: the K-step launches
// of many members in one launch.  Per XCD the queue holds, launch after
// launch, for each member its clock entry and its K-step work items; an entry
// of a member's launch l waits only until that member's launch l - 1 is
// complete.  Every entry derives the launch's plan from the member's device
// clock, as the waves of a K-step launch do, so each member makes exactly the
// launches (steps, speculated later steps, redos) of its own K-step run, and
// its state is bitwise that of stepping it alone.  Queue, hand-over between
// launches and progress argument as in k_batch (flood_kernels.hip): an entry
// waits only for entries of lower queue index, which running waves took
// before it.
// (FP32: two waves per SIMD; with three the queue's state spills the row
// pointers of the marchers to scratch)
template <typename T, int CPT, int K>
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
        const FusedArgs<T>& A = S.a2[l == B.nlaunch - 1 ? 1 : 0][(int)((B.l0 + l) % 6)];
        const FusedPlan P = make_plan<T>(A);
        if (e == 0) clock_wave_fused<T>(A, P);
        else if (P.ns != 0) fused_tile<T, CPT, K, false, true>(A, P, e - 1);
        __builtin_amdgcn_s_waitcnt(0);
        __asm__ volatile("" ::: "memory");
        if (lane == 0) atomicAdd(&B.done[m], 1ull);
    }
}

template <typename T>
__global__ void k_enter_fused(StepArgs<T> a, int cur, long long target, int keep_gen) {
    if (threadIdx.x != 0) return;
    DevCtl* ctl = a.ctl;
    FusedClock S;
    S.ck = ctl->clk[a.phase & 1];
    S.back = S.ck;
    for (int q = 0; q < kFuseMax - 1; ++q) S.mid[q] = S.ck;
    for (int q = 0; q < kFuseMax; ++q) S.dt[q] = 0.0;
    S.vsteps = 0;
    S.cur = cur;
    S.pending = 0;
    S.spec = 0;
    S.nclose = 0;
    S.gen = keep_gen ? ctl->genf : 0;
    ctl->cf[0] = S;
    for (int q = 0; q < 3 * kFuseMax; ++q) ctl->hmf[q] = 0ull;
    // launch 0 reads the slots of phase 2: the deepest cell of the state
    ctl->hmf[2 * kFuseMax + kFuseMax - 1] = ctl->hmax[a.phase % 3];
    ctl->targetf = target;
}

template <typename T>
__global__ void k_leave_fused(StepArgs<T> a, FusedArgs<T> A, long long launches) {
    const int lane = threadIdx.x & 63;
    DevCtl* ctl = a.ctl;
    const FusedClock S = ctl->cf[launches & 1];
    const int pl = (int)((launches - 1) % 6);
    ClockSlot ck = S.ck;
    for (int q = 0; q < kFuseMax; ++q)
        if (q < S.nclose) {
            const double so = partial_sum<T>(A.part[q][pl & 1], A.a.npart);
            ck.v_out = ck.v_out + S.dt[q] * a.dx * so;
        }
    ck.dt_prev = 0.0;
    inflow_solve<T>(a, hydrograph<T>(a, ck.t), const_cast<T*>(a.qin));
    for (int q = lane; q < a.npart; q += 64) const_cast<double*>(a.part_prev)[q] = 0.0;
    if (lane == 0) {
        ctl->clk[a.phase & 1] = ck;
        ctl->hmax[a.phase % 3] = ctl->hmf[kFuseMax * (pl % 3) + kFuseMax - 1];
        ctl->hmax[(a.phase + 1) % 3] = 0ull;
        ctl->genf = S.gen;
    }
}

// ------------------------------------------------------------ launchers
int strip_width_fused(int cpt, int k) { return 64 * cpt - 4 * k; }

template <typename T, int CPT, int K>
static hipError_t launch_fused_k(const FusedArgs<T>& a, hipStream_t s) {
    const long long items = (long long)a.a.nstrips * a.a.nchunks;
    const unsigned blocks = (unsigned)(1 + (items + 3) / 4);
    if (a.a.act) {
        // the flags of every item must fit in a slot; the skip test needs
        // items at least K rows tall
        if (items > a.a.act_stride || a.a.rows < K) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_fused<T, CPT, K, true>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_fused<T, CPT, K, false>), dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T, int CPT>
static hipError_t launch_fused_cpt(const FusedArgs<T>& a, hipStream_t s) {
    switch (a.K) {
    case 2: return launch_fused_k<T, CPT, 2>(a, s);
    case 3: return launch_fused_k<T, CPT, 3>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int cpt, hipStream_t s) {
    switch (cpt) {
    case 1: return launch_fused_cpt<T, 1>(a, s);
    case 2: return launch_fused_cpt<T, 2>(a, s);
    case 4: return sizeof(T) == 4 && a.K == 2 ? launch_fused_k<T, 4, 2>(a, s) : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_enter_fused(const StepArgs<T>& single, long long target, int keep_gen,
                              hipStream_t s) {
    // the single-step state at counter n lives in buffer n % 2, i.e. the
    // buffer of single.h_in; phase = n % 6
    hipLaunchKernelGGL((k_enter_fused<T>), dim3(1), dim3(64), 0, s, single, single.phase & 1, target,
                       keep_gen);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_leave_fused(const StepArgs<T>& single, const FusedArgs<T>& af, long long launches,
                              hipStream_t s) {
    if (launches < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_leave_fused<T>), dim3(1), dim3(64), 0, s, single, af, launches);
    return hipGetLastError();
}

template <typename T, int CPT, int K>
static hipError_t launch_batch2_k(const Batch2Args<T>& b, int device, hipStream_t s, int* blocks_out) {
    int per_cu = 0, ncu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch2<T, CPT, K>, 256, 0);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    const int blocks = std::max(1, per_cu) * ncu;
    if (blocks_out) *blocks_out = blocks;
    // an ordinary launch: the queue needs no co-residency (see k_batch2)
    hipLaunchKernelGGL((k_batch2<T, CPT, K>), dim3(blocks), dim3(256), 0, s, b, b.scen);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch2(const Batch2Args<T>& b, int cpt, int k, int device, hipStream_t s,
                         int* blocks_out) {
    if (k == 2) {
        switch (cpt) {
        case 1: return launch_batch2_k<T, 1, 2>(b, device, s, blocks_out);
        case 2: return launch_batch2_k<T, 2, 2>(b, device, s, blocks_out);
        default: return hipErrorInvalidValue;
        }
    }
    if (k == 3) {
        switch (cpt) {
        case 1: return launch_batch2_k<T, 1, 3>(b, device, s, blocks_out);
        case 2: return launch_batch2_k<T, 2, 3>(b, device, s, blocks_out);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_batch2<float>(const Batch2Args<float>&, int, int, int, hipStream_t, int*);
template hipError_t launch_batch2<double>(const Batch2Args<double>&, int, int, int, hipStream_t, int*);
template hipError_t launch_fused<float>(const FusedArgs<float>&, int, hipStream_t);
template hipError_t launch_fused<double>(const FusedArgs<double>&, int, hipStream_t);
template hipError_t launch_enter_fused<float>(const StepArgs<float>&, long long, int, hipStream_t);
template hipError_t launch_enter_fused<double>(const StepArgs<double>&, long long, int, hipStream_t);
template hipError_t launch_leave_fused<float>(const StepArgs<float>&, const FusedArgs<float>&,
                                              long long, hipStream_t);
template hipError_t launch_leave_fused<double>(const StepArgs<double>&, const FusedArgs<double>&,
                                               long long, hipStream_t);

}  // namespace flood
