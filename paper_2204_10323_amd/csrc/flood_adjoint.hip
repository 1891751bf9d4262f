// Reverse of one fixed-dt flood step on the GPU (every cell's adjoints are
// written by the one lane that owns it; no atomics).  Used by the checkpointed
// adjoint of the runtime to obtain gradients of a gauge misfit with respect to
// the per-cell Manning n and the inflow hydrograph samples.
//
// For the adjoints lh', lq' of the new state (the step computes the boundary
// faces (eq. 5, 6), then eq. (3) on the interior faces, then donor-cell
// scaling, then eq. (4)):
//   mu_f  = lq'_f + dt/dx (lh'_R - lh'_L)               applied face value
//   rho_c = sum over faces f drained by cell c of mu_f q*_f
//   mu*_f = mu_f r_d + nu_d sign(q*_f),  nu_d = rho_d dr_d/dO_d * dt/dx
//   lh_c  = lh'_c + rho_c dr_c/dh_c + sum_f mu*_f dq*_f/dh_c
//   lq_f  = mu*_f dq*_f/dq_f,     dL/dn_c += sum_f mu*_f dq*_f/dn_c
// One row-marching pass per reversed step computes both: each wave marches
// up a strip, evaluates every face once (the forward value and its
// derivatives), gets r, nu and rho dr/dh of a row as soon as the faces around
// it exist, and the adjoints and the Manning gradient of the row below that,
// keeping all of it in registers (no round trip through memory between the
// two).  A one-wave pass carries the inflow section through the water level W
// of eq. (6) to Q(t) and to the section's roughness.
// The forward quantities are recomputed with the step's own device
// functions, so the branches (dry face, limiter, donor) match the forward.
#include <math.h>

#include "flood_device.h"

namespace flood {

template <typename T>
struct FaceFwd {
    T qs, Pq, PL, PR, Pn;
};

// Eq. (3) on one interior face, with dq*/dq, dq*/dh_L, dq*/dh_R, dq*/dn_f.
// A max tie takes the left value; d|q|/dq = sign(q), sign(0) = 0.
template <typename T>
__device__ __forceinline__ FaceFwd<T> face_fwd(T hL, T hR, T zL, T zR, T nL, T nR, T q, T gdt,
                                               T inv_dx, T h_eps) {
    FaceFwd<T> f;
    const T etaL = hL + zL, etaR = hR + zR;
    f.qs = face_q<T>(etaL, etaR, zL, zR, nL, nR, q, gdt, inv_dx, h_eps);
    f.Pq = f.PL = f.PR = f.Pn = T(0);
    const T hf = fmax(etaL, etaR) - fmax(zL, zR);
    if (hf <= h_eps) return f;
    const T nf = T(0.5) * (nL + nR);
    const T grad = (etaR - etaL) * inv_dx;
    const T c73 = (hf * hf) * cbrt_t(hf);
    const T fr = gdt * (nf * nf);
    const T aq = fabs(q);
    const T den = T(1) + (fr * aq) / c73;
    const T sq = T((q > T(0)) - (q < T(0)));
    const T dden_dq = fr * sq / c73;
    const T dden_dhf = -(T(7) / T(3)) * fr * aq / (c73 * hf);
    const T dden_dnf = T(2) * gdt * nf * aq / c73;
    const T dqs_dhf = (-gdt * grad - f.qs * dden_dhf) / den;
    const T dqs_dgrad = (-gdt * hf) / den;
    f.Pq = (T(1) - f.qs * dden_dq) / den;
    f.Pn = -f.qs * dden_dnf / den;
    const T tieL = (etaL >= etaR) ? T(1) : T(0);
    f.PL = dqs_dhf * tieL - dqs_dgrad * inv_dx;
    f.PR = dqs_dhf * (T(1) - tieL) + dqs_dgrad * inv_dx;
    return f;
}

// FP32: the same derivatives from h_f^(-7/3) and 1/den as the forward face
// update computes them (hardware log2/exp2/reciprocal, about one ulp each), so
// q* has exactly the forward's bits and no cube root or division remains.
template <>
__device__ __forceinline__ FaceFwd<float> face_fwd<float>(float hL, float hR, float zL, float zR,
                                                          float nL, float nR, float q, float gdt,
                                                          float inv_dx, float h_eps) {
    FaceFwd<float> f;
    f.qs = f.Pq = f.PL = f.PR = f.Pn = 0.0f;
    const float etaL = hL + zL, etaR = hR + zR;
    const float hf = maxv(etaL, etaR) - maxv(zL, zR);
    if (hf <= h_eps) return f;
    // the forward value, operation for operation (face_q<float>)
    const float nf = 0.5f * (nL + nR);
    const float grad = (etaR - etaL) * inv_dx;
    const float num = q - (gdt * hf) * grad;
    const float m73 = fminf(__builtin_amdgcn_exp2f((-7.0f / 3.0f) * __builtin_amdgcn_logf(hf)), 3.0e38f);
    const float fr = gdt * (nf * nf);
    const float aq = fabsf(q);
    const float den = 1.0f + (fr * aq) * m73;
    const float rden = __builtin_amdgcn_rcpf(den);
    f.qs = num * rden;
    // its derivatives
    const float sq = (float)((q > 0.0f) - (q < 0.0f));
    const float dden_dq = (fr * sq) * m73;
    const float dden_dhf = ((-(7.0f / 3.0f) * fr) * aq) * (m73 * __builtin_amdgcn_rcpf(hf));
    const float dden_dnf = ((2.0f * gdt) * nf * aq) * m73;
    const float dqs_dhf = (-gdt * grad - f.qs * dden_dhf) * rden;
    const float dqs_dgrad = (-gdt * hf) * rden;
    f.Pq = (1.0f - f.qs * dden_dq) * rden;
    f.Pn = -(f.qs * dden_dnf) * rden;
    const float tieL = (etaL >= etaR) ? 1.0f : 0.0f;
    f.PL = dqs_dhf * tieL - dqs_dgrad * inv_dx;
    f.PR = dqs_dhf * (1.0f - tieL) + dqs_dgrad * inv_dx;
    return f;
}

enum { F_INT = 0, F_WALL = 1, F_IN = 2, F_OUT = 3 };

// Kind of the border face of cell (i, j) on `side` (the cell is on that edge);
// kb: the outflow coefficient kout[pos] (zero off the outflow side).
template <typename T>
__device__ __forceinline__ int border_kind(const AdjArgs<T>& a, int side, int pos, T kb) {
    if (a.in_side == side && pos >= a.in_first && pos < a.in_first + a.in_count) return F_IN;
    if (a.out_side == side && kb > T(0)) return F_OUT;
    return F_WALL;
}

// Outflow border value as the step computes it (border_q without inflow),
// with its derivatives in the edge cell's depth and roughness.
template <typename T>
__device__ __forceinline__ T outflow_fwd(const AdjArgs<T>& a, int side, T k, T h, T n, T& d_dh,
                                         T& d_dn) {
    const T hp = fmax(h, T(0));
    const T v = -k * pow53(hp);
    const T c = cbrt_t(hp);
    T dv_dh = (h > T(0)) ? -k * (T(5) / T(3)) * (c * c) : T(0);
    T dv_dn = pow53(hp) * T(sqrt(a.out_slope)) / (n * n);
    const bool ws = (side == SIDE_W || side == SIDE_S);
    d_dh = ws ? dv_dh : -dv_dh;
    d_dn = ws ? dv_dn : -dv_dn;
    return ws ? v : -v;
}

// A face of the reversed step: its forward value q*, the derivatives of q*
// (eq. 3: dq*/dq, dq*/dh_L, dq*/dh_R, dq*/dn_f; an outflow border face: its
// derivatives in the edge cell's depth in PL or PR and in the cell's n in Pn)
// and mu = lq'_f + dt/dx (lh'_R - lh'_L).
template <typename T>
struct AFace {
    T qs, Pq, PL, PR, Pn, mu;
};

template <typename T>
__device__ __forceinline__ AFace<T> aface_prev(const AFace<T>& e) {
    AFace<T> f;
    f.qs = from_prev(e.qs);
    f.Pq = from_prev(e.Pq);
    f.PL = from_prev(e.PL);
    f.PR = from_prev(e.PR);
    f.Pn = from_prev(e.Pn);
    f.mu = from_prev(e.mu);
    return f;
}

// The face between cells L and R (R on the +axis side).  lq: the adjoint of
// the face's new value; real_L/real_R: whether L and R lie in the grid; for a
// border face the edge cell's side, its position along it and the outflow
// coefficient there.
template <typename T>
__device__ __forceinline__ AFace<T> aface(const AdjArgs<T>& a, T hL, T hR, T zL, T zR, T nL, T nR,
                                          T q, T lq, T lhL, T lhR, bool real_L, bool real_R,
                                          int side, int pos, T kb, T gdt, T inv_dx, T h_eps,
                                          T dtdx) {
    AFace<T> f;
    f.qs = f.Pq = f.PL = f.PR = f.Pn = T(0);
    f.mu = lq + dtdx * (lhR - lhL);
    if (real_L && real_R) {
        const FaceFwd<T> F = face_fwd<T>(hL, hR, zL, zR, nL, nR, q, gdt, inv_dx, h_eps);
        f.qs = F.qs;
        f.Pq = F.Pq;
        f.PL = F.PL;
        f.PR = F.PR;
        f.Pn = F.Pn;
    } else if (real_L != real_R) {
        if (border_kind(a, side, pos, kb) == F_OUT) {
            T d_dh, d_dn;
            if (real_L) {
                f.qs = outflow_fwd(a, side, kb, hL, nL, d_dh, d_dn);
                f.PL = d_dh;
            } else {
                f.qs = outflow_fwd(a, side, kb, hR, nR, d_dh, d_dn);
                f.PR = d_dh;
            }
            f.Pn = d_dn;
        }
    }
    return f;
}

// Donor terms of the face for the cell on its right (cell_is_L = false) or
// left: mu* = mu r_d + nu_d sign(q*), the donor being the cell the face drains.
template <typename T>
__device__ __forceinline__ T face_mus(const AFace<T>& f, bool cell_is_L, T r_c, T nu_c, T r_nb,
                                      T nu_nb) {
    const bool donor_is_c = (f.qs > T(0)) == cell_is_L;
    const T r_d = donor_is_c ? r_c : r_nb;
    const T nu_d = donor_is_c ? nu_c : nu_nb;
    return f.mu * r_d + nu_d * T((f.qs > T(0)) - (f.qs < T(0)));
}

template <typename T>
__device__ void adj_inflow(const AdjArgs<T>& a, double t, const double* ain);

// The reverse of one step on strips of 60 output columns (one cell per lane,
// two halo columns on each side) and chunks of `rows` output rows: row k
// enters; the faces east of its cells and the faces between rows k-1 and k
// are evaluated; r, nu, kappa of row k-1 follow (its four faces exist); then
// the adjoints and the Manning gradient of row k-2 (r and nu of its four
// neighbours exist).  Block 0 runs the inflow pass of the step reversed just
// before (that step's kernel has completed; the two use different ain
// buffers and the inflow pass accumulates its roughness terms apart).
constexpr int kAdjWO = 60;

template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 5 : 1) void k_adj_march(AdjArgs<T> a) {
    if (blockIdx.x == 0) {
        if (a.bc_prev && threadIdx.x < 64) adj_inflow<T>(a, a.t_prev, a.ain_prev);
        return;
    }
    const int wave = (blockIdx.x - 1) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nstrips = (a.nx + kAdjWO - 1) / kAdjWO;
    const int nchunks = (a.ny + a.rows - 1) / a.rows;
    if (wave >= nstrips * nchunks) return;
    const int s = wave % nstrips, c = wave / nstrips;
    const int j0 = c * a.rows, j1 = min(j0 + a.rows, a.ny);
    const int lane = threadIdx.x & 63;
    const int nx = a.nx, ny = a.ny;
    const int i = s * kAdjWO - kHalo + lane;       // this lane's column
    const bool col_real = (i >= 0 && i < nx);
    const bool out_col = (lane >= 2 && lane < 62 && col_real);
    const bool loads = (i >= -kHalo && i < nx + kHalo);
    const long long P = a.pitch;
    const T dt = (T)a.dt, inv_dx = T(1) / T(a.dx), gdt = T(a.g) * dt, h_eps = T(a.h_eps);
    const T dtdx = dt * inv_dx;

    // row k (entering), row k-1, row k-2
    T h0 = 0, z0 = 0, n0 = 0, qx0 = 0, qy0 = 0, l0 = 0, lx0 = 0, ly0 = 0;
    T h1 = 0, z1 = 0, n1 = 0, qy1 = 0, l1 = 0, ly1 = 0;
    T l2 = 0;
    AFace<T> E1{}, E2{};        // faces east of the cells of rows k-1, k-2
    AFace<T> Y1{}, Y2{};        // faces between rows k-2|k-1 and k-3|k-2
    // r, nu (and kappa) of rows k-2 (r1 ...) and k-3 (r2 ...), before this
    // iteration computes those of row k-1 (r0 ...)
    T r1 = 1, nu1 = 0, kap1 = 0, r2 = 1, nu2 = 0;
    // the next row's values are loaded one iteration ahead, and with them the
    // Manning gradient of the row that iteration finishes (two rows behind)
    T fh, fz, fn, fqx, fqy, fl, flx, fly;
    double fgn = 0.0, gn_row = 0.0;
    // outflow coefficients at the borders: by row on a west or east outflow
    // side (fetched with the rows: kr0, kr1, kr2 for rows k, k-1, k-2), by
    // column on a south or north one (kc)
    const bool out_we = (a.out_side == SIDE_W || a.out_side == SIDE_E);
    const T kc = (!out_we && col_real) ? a.kout[i] : T(0);
    T fkr = T(0), kr0 = T(0), kr1 = T(0), kr2 = T(0);
    auto fetch = [&](int k) {
        fh = fz = fn = fqx = fqy = fl = flx = fly = T(0);
        fkr = (out_we && k >= 0 && k < ny) ? a.kout[k] : T(0);
        if (out_col && k - 2 >= j0 && k - 2 < j1) fgn = a.gn[(long long)(k - 2) * nx + i];
        if (loads && k >= -kHalo && k < ny + kHalo) {
            const long long o = (long long)(k + kHalo) * P + i + kHalo;
            fh = a.h[o];
            fz = a.z[o];
            fn = a.n[o];
            fqx = a.qx[o];
            fqy = a.qy[o];
            fl = a.lh1[o];
            flx = a.lqx1[o];
            fly = a.lqy1[o];
        }
    };
    fetch(j0 - 2);
    for (int k = j0 - 2; k <= j1 + 1; ++k) {
        h0 = fh; z0 = fz; n0 = fn; qx0 = fqx; qy0 = fqy; l0 = fl; lx0 = flx; ly0 = fly;
        gn_row = fgn;   // row k-2's
        kr2 = kr1; kr1 = kr0; kr0 = fkr;
        if (k < j1 + 1) fetch(k + 1);
        const bool row_real = (k >= 0 && k < ny);
        // Only what the output rows j0 .. j1-1 use is evaluated (the conditions
        // are uniform over the wave): r and nu of rows j0-1 .. j1, so the faces
        // east of rows j0-1 .. j1 and those between rows j0-2|j0-1 .. j1|j1+1.
        // faces east of the cells of row k (the lane at column -1 holds the
        // west border face of column 0)
        AFace<T> E0{};
        if (k >= j0 - 1 && k <= j1) {
            const T hn = from_next(h0), zn = from_next(z0), nn = from_next(n0), ln = from_next(l0);
            const bool nxt_real = (i + 1 >= 0 && i + 1 < nx);
            E0 = aface<T>(a, h0, hn, z0, zn, n0, nn, qx0, lx0, l0, ln, row_real && col_real,
                          row_real && nxt_real, col_real ? SIDE_E : SIDE_W, k, kr0, gdt, inv_dx,
                          h_eps, dtdx);
        }
        // faces between rows k-1 and k
        AFace<T> Y0{};
        if (k >= j0 - 1) {
            const bool prev_row_real = (k - 1 >= 0 && k - 1 < ny);
            Y0 = aface<T>(a, h1, h0, z1, z0, n1, n0, qy1, ly1, l1, l0, col_real && prev_row_real,
                          col_real && row_real, prev_row_real ? SIDE_N : SIDE_S, i, kc, gdt,
                          inv_dx, h_eps, dtdx);
        }
        // r, nu, kappa of row k-1: faces W (east face of the lane before), E, S, N
        T r0 = 1, nu0 = 0, kap0 = 0;
        if (k >= j0) {
            const T qW = from_prev(E1.qs), muW = from_prev(E1.mu);
            T out = max0_neg(qW);
            out += max0(E1.qs);
            out += max0_neg(Y1.qs);
            out += max0(Y0.qs);
            const T O = (dt * out) * inv_dx;
            const T hp = max0(h1);
            const bool lim = a.positivity && (O > hp);
            T rho = T(0);
            if (qW < T(0)) rho += muW * qW;
            if (E1.qs > T(0)) rho += E1.mu * E1.qs;
            if (Y1.qs < T(0)) rho += Y1.mu * Y1.qs;
            if (Y0.qs > T(0)) rho += Y0.mu * Y0.qs;
            r0 = lim ? donor_ratio<T>(hp, O) : T(1);
            nu0 = lim ? rho * (-hp / (O * O)) * dtdx : T(0);
            kap0 = (lim && h1 > T(0)) ? rho / O : T(0);
        }
        // adjoints of row k-2
        const int rb = k - 2;
        if (rb >= j0 && rb < j1) {
            // lane moves with every lane active (a disabled source lane gives no value)
            const AFace<T> W = aface_prev(E2);
            const T rW = from_prev(r1), nuW = from_prev(nu1), rE = from_next(r1), nuE = from_next(nu1);
            if (out_col) {
                T lh = l2 + kap1;
                T gnc = T(0), lqx = T(0), lqy = T(0);
                // west face (the cell on its right)
                if (i == 0) {
                    const int kind = border_kind(a, SIDE_W, rb, kr2);
                    if (kind == F_OUT) {
                        const T mus = face_mus(W, false, r1, nu1, r1, nu1);
                        lh += mus * W.PR;
                        gnc += mus * W.Pn;
                    } else if (kind == F_IN) {
                        a.ain[rb - a.in_first] = (double)W.mu;
                    }
                } else {
                    const T mus = face_mus(W, false, r1, nu1, rW, nuW);
                    lh += mus * W.PR;
                    gnc += T(0.5) * mus * W.Pn;
                }
                // east face (the cell on its left)
                if (i == nx - 1) {
                    const int kind = border_kind(a, SIDE_E, rb, kr2);
                    if (kind == F_OUT) {
                        const T mus = face_mus(E2, true, r1, nu1, r1, nu1);
                        lh += mus * E2.PL;
                        gnc += mus * E2.Pn;
                    } else if (kind == F_IN) {
                        a.ain[rb - a.in_first] = (double)(-E2.mu);
                    }
                } else {
                    const T mus = face_mus(E2, true, r1, nu1, rE, nuE);
                    lh += mus * E2.PL;
                    gnc += T(0.5) * mus * E2.Pn;
                    lqx = mus * E2.Pq;
                }
                // south face
                if (rb == 0) {
                    const int kind = border_kind(a, SIDE_S, i, kc);
                    if (kind == F_OUT) {
                        const T mus = face_mus(Y2, false, r1, nu1, r1, nu1);
                        lh += mus * Y2.PR;
                        gnc += mus * Y2.Pn;
                    } else if (kind == F_IN) {
                        a.ain[i - a.in_first] = (double)Y2.mu;
                    }
                } else {
                    const T mus = face_mus(Y2, false, r1, nu1, r2, nu2);
                    lh += mus * Y2.PR;
                    gnc += T(0.5) * mus * Y2.Pn;
                }
                // north face
                if (rb == ny - 1) {
                    const int kind = border_kind(a, SIDE_N, i, kc);
                    if (kind == F_OUT) {
                        const T mus = face_mus(Y1, true, r1, nu1, r1, nu1);
                        lh += mus * Y1.PL;
                        gnc += mus * Y1.Pn;
                    } else if (kind == F_IN) {
                        a.ain[i - a.in_first] = (double)(-Y1.mu);
                    }
                } else {
                    const T mus = face_mus(Y1, true, r1, nu1, r0, nu0);
                    lh += mus * Y1.PL;
                    gnc += T(0.5) * mus * Y1.Pn;
                    lqy = mus * Y1.Pq;
                }
                const long long o = (long long)(rb + kHalo) * P + i + kHalo;
                a.lh[o] = lh;
                a.lqx[o] = lqx;
                a.lqy[o] = lqy;
                a.gn[(long long)rb * nx + i] = gn_row + (double)gnc;
            }
        }
        // shift the window
        l2 = l1;
        h1 = h0; z1 = z0; n1 = n0; qy1 = qy0; l1 = l0; ly1 = ly0;
        E2 = E1; E1 = E0;
        Y2 = Y1; Y1 = Y0;
        r2 = r1; nu2 = nu1;
        r1 = r0; nu1 = nu0; kap1 = kap0;
    }
}

// Q(t) and its interpolation weights on the samples (k0, 1-w) and (k0+1, w).
__device__ __forceinline__ double hydro_weights(const double* ts, const double* qs, int ns, double t,
                                                int& k0, double& w) {
    if (t <= ts[0]) { k0 = 0; w = 0.0; return qs[0]; }
    if (t >= ts[ns - 1]) { k0 = ns - 1; w = 0.0; return qs[ns - 1]; }
    int lo = 0, hi = ns - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ts[mid] <= t) lo = mid; else hi = mid;
    }
    k0 = lo;
    w = (t - ts[lo]) / (ts[hi] - ts[lo]);
    return qs[lo] + (qs[hi] - qs[lo]) * w;
}

// Inflow section of the step that started at time t (one wave; needs that
// step's reverse kernel complete, which wrote ain): with G(W) = sum_c dx k_c (W - z_c)_+^{5/3} - Q = 0,
// dW/dQ = 1/D and dW/dk_j = -dx (W - z_j)^{5/3} / D, D = sum_c dx k_c (5/3)(W - z_c)^{2/3}.
template <typename T>
__device__ void adj_inflow(const AdjArgs<T>& a, double t, const double* ain) {
    const int lane = threadIdx.x & 63;
    const int nc = a.in_count;
    if (nc <= 0 || a.nsamp <= 0) return;
    int k0;
    double w;
    const double Q = hydro_weights(a.ts, a.qs, a.nsamp, t, k0, w);
    if (!(Q > 0.0)) return;
    const double W = inflow_level(a.in_z, a.in_k, nc, a.dx, Q);
    double D = 0.0, A = 0.0;
    for (int p = lane; p < nc; p += 64) {
        const double d = W - a.in_z[p];
        const double c = d > 0.0 ? cbrt(d) : 0.0;
        const double e = a.in_k[p] * (5.0 / 3.0) * (c * c);
        D += a.dx * e;
        A += ain[p] * e;
    }
    D = wave_sum(D);
    A = wave_sum(A);
    const double dLdQ = A / D;
    if (lane == 0) {
        a.gq[k0] += (k0 + 1 < a.nsamp && w > 0.0) ? (1.0 - w) * dLdQ : dLdQ;
        if (k0 + 1 < a.nsamp && w > 0.0) a.gq[k0 + 1] += w * dLdQ;
    }
    // the section's roughness terms go to gn_in (by section position): the
    // step kernel this pass runs in adds to gn at the same cells
    for (int p = lane; p < nc; p += 64) {
        const int pos = a.in_first + p;
        const int ci = (a.in_side == SIDE_W) ? 0 : (a.in_side == SIDE_E) ? a.nx - 1 : pos;
        const int cj = (a.in_side == SIDE_S) ? 0 : (a.in_side == SIDE_N) ? a.ny - 1 : pos;
        const double nc_ = (double)a.n[(long long)(cj + kHalo) * a.pitch + ci + kHalo];
        const double dLdk = pow53(W - a.in_z[p]) * (ain[p] - a.dx * A / D);
        a.gn_in[p] += dLdk * (-sqrt(a.in_slope) / (nc_ * nc_));
    }
}

// gn at the inflow cells += the inflow pass's roughness terms (after a sweep).
template <typename T>
__global__ void k_adj_fold_inflow(AdjArgs<T> a) {
    for (int p = threadIdx.x; p < a.in_count; p += blockDim.x) {
        const int pos = a.in_first + p;
        const int ci = (a.in_side == SIDE_W) ? 0 : (a.in_side == SIDE_E) ? a.nx - 1 : pos;
        const int cj = (a.in_side == SIDE_S) ? 0 : (a.in_side == SIDE_N) ? a.ny - 1 : pos;
        a.gn[(long long)cj * a.nx + ci] += a.gn_in[p];
    }
}

// The inflow pass on its own (the last step of a sweep).
template <typename T>
__global__ void k_adj_bc(AdjArgs<T> a) {
    adj_inflow<T>(a, a.t, a.ain);
}

// Depth at the gauge cells (flat j*nx + i) into dst[0 .. ng).
template <typename T>
__global__ void k_gauge_gather(const T* h, long long pitch, int nx, const int* gauges, int ng,
                               T* dst) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int c = gauges[g], j = c / nx, i = c - j * nx;
    dst[g] = h[(long long)(j + kHalo) * pitch + i + kHalo];
}

// Adjoint seeds of one observation: dl[g], or 2 (series[g] - obs[g]), added
// to the depth adjoint of the gauge cells.  Gauges are grouped by cell
// (cells[u] holds gauges list[ptr[u] .. ptr[u+1]) in gauge order), one thread
// per cell, so the sum is the same in every run.
template <typename T>
__global__ void k_gauge_seed(T* lh, long long pitch, int nx, const int* cells, const int* ptr,
                             const int* list, int nu, const T* series, const T* obs, const T* dl) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    T s = T(0);
    for (int k = ptr[u]; k < ptr[u + 1]; ++k) {
        const int g = list[k];
        s += dl ? dl[g] : T(2) * (series[g] - obs[g]);
    }
    const int c = cells[u], j = c / nx, i = c - j * nx;
    lh[(long long)(j + kHalo) * pitch + i + kHalo] += s;
}

int adjoint_rows(int nx, int ny) {
    // about 4096 work items (four waves per SIMD): a chunk of r rows costs r + 3
    // row iterations, so chunks stay as tall as the grid allows, between 4 and 32
    const long long strips = (nx + kAdjWO - 1) / kAdjWO;
    int r = 32;
    while (r > 4 && strips * ((ny + r - 1) / r) < 4096) r >>= 1;
    return r;
}

template <typename T>
hipError_t launch_adjoint_step(const AdjArgs<T>& a, hipStream_t s) {
    if (a.rows < 1) return hipErrorInvalidValue;
    const long long items = (long long)((a.nx + kAdjWO - 1) / kAdjWO) * ((a.ny + a.rows - 1) / a.rows);
    hipLaunchKernelGGL((k_adj_march<T>), dim3((unsigned)(1 + (items + 3) / 4)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_fold_inflow(const AdjArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_fold_inflow<T>), dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_inflow(const AdjArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_bc<T>), dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gauge_gather(const T* h, long long pitch, int nx, const int* gauges, int ng, T* dst,
                               hipStream_t s) {
    hipLaunchKernelGGL((k_gauge_gather<T>), dim3((ng + 255) / 256), dim3(256), 0, s, h, pitch, nx,
                       gauges, ng, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gauge_seed(T* lh, long long pitch, int nx, const int* cells, const int* ptr,
                             const int* list, int nu, const T* series, const T* obs, const T* dl,
                             hipStream_t s) {
    hipLaunchKernelGGL((k_gauge_seed<T>), dim3((nu + 255) / 256), dim3(256), 0, s, lh, pitch, nx,
                       cells, ptr, list, nu, series, obs, dl);
    return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_adjoint_fold_inflow<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adjoint_fold_inflow<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_adjoint_inflow<float>(const AdjArgs<float>&, hipStream_t);
template hipError_t launch_adjoint_inflow<double>(const AdjArgs<double>&, hipStream_t);
template hipError_t launch_gauge_gather<float>(const float*, long long, int, const int*, int, float*,
                                               hipStream_t);
template hipError_t launch_gauge_gather<double>(const double*, long long, int, const int*, int,
                                                double*, hipStream_t);
template hipError_t launch_gauge_seed<float>(float*, long long, int, const int*, const int*,
                                             const int*, int, const float*, const float*,
                                             const float*, hipStream_t);
template hipError_t launch_gauge_seed<double>(double*, long long, int, const int*, const int*,
                                              const int*, int, const double*, const double*,
                                              const double*, hipStream_t);

}  // namespace flood
