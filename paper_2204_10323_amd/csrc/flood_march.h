// The row-marching update of one step, shared by the single-step, batch and
// two-step kernels of libflood, so that each computes a cell with the same
// instructions and therefore the same bits.
#pragma once
#include "flood_device.h"

namespace flood {

// Strip geometry of a wave: which of its cells lie outside the grid, and
// which carry the west or east border face.
template <int CPT>
struct StripGeo {
    int i0;                     // real column of the wave's first cell
    bool west_strip, east_strip;
    bool outside[CPT], west_face[CPT], east_face[CPT];
};

// Constants of one step.  The inflow magnitudes of this step come from the
// array qin (filled by the previous step's clock wave), or, when qin is NULL,
// from the water level W of eq. (6) for this step (inflow_on = 0: no inflow).
template <typename T>
struct StepK {
    T dt, gdt, inv_dx, h_eps;
    const T* qin;
    double W;
    int inflow_on;
    // pre: the west and east border faces of the row take its inflow b_in and
    // outflow coefficient b_out from here (loaded with the row) instead of
    // loading them when the face is evaluated
    bool pre;
    T b_in, b_out;
};

// Inflow magnitude at position p along the inflow side: the same expression
// the inflow solve stores.
template <typename T>
__device__ __forceinline__ T inflow_at(const StepArgs<T>& a, const StepK<T>& K, int p) {
    if (K.qin) return K.qin[p];
    const int r = p - a.in_first;
    if (!K.inflow_on || r < 0 || r >= a.in_count) return T(0);
    return (T)(a.in_k[r] * pow53(K.W - a.in_z[r]));
}

// Border face value (eq. 5, 6), signed toward +axis: the inflow of this step,
// the Manning discharge of the edge cell's own depth on the outflow section,
// a closed wall everywhere else.  With VAR_BOUNDARY_CELL_AREA eq. (5) is taken
// literally: the outflow cell passes dx^2 h^{2/3} sqrt(S)/n, dx h^{2/3} sqrt(S)/n
// per unit width of its face.
template <typename T, int VAR = 0>
__device__ __forceinline__ T border_q(const StepArgs<T>& a, const StepK<T>& K, int side, int p,
                                      T h_edge) {
    const bool given = K.pre && (side == SIDE_W || side == SIDE_E);
    T v = T(0);
    if (a.in_side == side) v = given ? K.b_in : inflow_at<T>(a, K, p);
    if (a.out_side == side) {
        const T ko = given ? K.b_out : a.kout[p];
        if constexpr ((VAR & VAR_BOUNDARY_CELL_AREA) != 0)
            v -= ko * (T(a.dx) * pow23(fmax(h_edge, T(0))));
        else
            v -= ko * pow53(fmax(h_edge, T(0)));
    }
    return (side == SIDE_W || side == SIDE_S) ? v : -v;
}

// The row-marching update of one step on one strip: rows enter in increasing
// order; when row k enters, the row k-2 leaves with its new depth (eq. 4) and
// the applied discharges of its east and north faces.  The marcher keeps the
// two rows still needed (surface, bed, roughness, depths, tentative and
// applied discharges, donor factors) in registers.
// VAR selects a method variant (0: the paper's per-axis form); with
// VAR_FRICTION_VECTOR the friction term uses sqrt(q^2 + q_perp^2), q_perp the
// mean of the start-of-step discharges on the interior perpendicular faces of
// the two cells beside the face, which needs the previous row's x-discharges.
template <typename T, int CPT, int VAR = 0>
struct Marcher {
    T eta1[CPT], z1[CPT], n1[CPT], qy1[CPT], h1[CPT], h2[CPT];
    T qsx1[CPT], qsy2[CPT], r2[CPT], qnx2[CPT], qny3[CPT];
    T qxo1[CPT];  // start-of-step qx of row k-1 (vector friction only)

    __device__ __forceinline__ void reset() {
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            eta1[m] = z1[m] = n1[m] = qy1[m] = h1[m] = h2[m] = T(0);
            qsx1[m] = qsy2[m] = qnx2[m] = qny3[m] = T(0);
            r2[m] = T(1);
            if constexpr ((VAR & VAR_FRICTION_VECTOR) != 0) qxo1[m] = T(0);
        }
    }

    // Row k enters with its start-of-step h, z, n, qx, qy.  Out: hn, qxo, qyo
    // of row k-2 (meaningful for rows inside the grid).  EDGE = false: the
    // caller guarantees that the strip meets no border of the grid (every
    // lane's cells inside it) and that rows k-2 .. k are inside the grid and
    // not next to its south or north border, so the border code drops out.
    template <bool EDGE = true>
    __device__ __forceinline__ void row(const StepArgs<T>& a, const StepK<T>& K,
                                        const StripGeo<CPT>& G, int k, const T (&h0)[CPT],
                                        const T (&z0)[CPT], const T (&n0)[CPT],
                                        const T (&qx0)[CPT], const T (&qy0)[CPT], T (&hn)[CPT],
                                        T (&qxo)[CPT], T (&qyo)[CPT]) {
        const int ny = a.ny;
        const bool row_real = (k >= 0 && k < ny);

        // A: x-faces of row k (eq. 3), border faces from the boundary conditions.
        T eta0[CPT], qsx0[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) eta0[m] = h0[m] + z0[m];
        const T etaRn = from_next(eta0[0]), zRn = from_next(z0[0]), nRn = from_next(n0[0]);
        if constexpr ((VAR & VAR_FRICTION_VECTOR) != 0) {
            // perpendicular faces of an x-face of row k: the y-faces below
            // (row k-1's north faces) and above (row k's), of both cells;
            // border faces (rows -1 and ny-1) are left out of the mean
            const T qy1Rn = from_next(qy1[0]), qy0Rn = from_next(qy0[0]);
            const bool below = (k >= 1), above = (k <= ny - 2);
            const T wgt = (below && above) ? T(0.25) : T(0.5);
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const T eR = (m + 1 < CPT) ? eta0[(m + 1) % CPT] : etaRn;
                const T zR = (m + 1 < CPT) ? z0[(m + 1) % CPT] : zRn;
                const T nR = (m + 1 < CPT) ? n0[(m + 1) % CPT] : nRn;
                const T b1 = (m + 1 < CPT) ? qy1[(m + 1) % CPT] : qy1Rn;
                const T b0 = (m + 1 < CPT) ? qy0[(m + 1) % CPT] : qy0Rn;
                T ps = T(0);
                if (below) ps += (qy1[m] + b1);
                if (above) ps += (qy0[m] + b0);
                const T qp = ps * wgt;
                const T qm = sqrt(qx0[m] * qx0[m] + qp * qp);
                qsx0[m] = face_qm<T>(eta0[m], eR, z0[m], zR, n0[m], nR, qx0[m], qm, K.gdt,
                                     K.inv_dx, K.h_eps);
            }
        } else {
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const T eR = (m + 1 < CPT) ? eta0[(m + 1) % CPT] : etaRn;
                const T zR = (m + 1 < CPT) ? z0[(m + 1) % CPT] : zRn;
                const T nR = (m + 1 < CPT) ? n0[(m + 1) % CPT] : nRn;
                qsx0[m] = face_q<T>(eta0[m], eR, z0[m], zR, n0[m], nR, qx0[m], K.gdt, K.inv_dx, K.h_eps);
            }
        }
        if (EDGE && G.west_strip) {
            const T hRn = from_next(h0[0]);
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (G.west_face[m]) {
                    const T hR = (m + 1 < CPT) ? h0[(m + 1) % CPT] : hRn;
                    qsx0[m] = row_real ? border_q<T, VAR>(a, K, SIDE_W, k, hR) : T(0);
                }
        }
        if (EDGE && G.east_strip) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (G.east_face[m])
                    qsx0[m] = row_real ? border_q<T, VAR>(a, K, SIDE_E, k, h0[m]) : T(0);
        }

        // B: y-faces between rows k-1 and k.
        T qsy1[CPT];
        if constexpr ((VAR & VAR_FRICTION_VECTOR) != 0) {
            // perpendicular faces of the y-face above cell (i, k-1): the
            // x-faces west (column i-1) and east (column i) of the cells of
            // rows k-1 and k; west and east border faces are left out
            const T w1n = from_prev(qxo1[CPT - 1]), w0n = from_prev(qx0[CPT - 1]);
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const T w1 = (m > 0) ? qxo1[(m + CPT - 1) % CPT] : w1n;
                const T w0 = (m > 0) ? qx0[(m + CPT - 1) % CPT] : w0n;
                const int i = G.i0 + m;
                const bool west = (i >= 1), east = (i <= a.nx - 2);
                T ps = T(0);
                if (west) ps += (w1 + w0);
                if (east) ps += (qxo1[m] + qx0[m]);
                const T qp = ps * ((west && east) ? T(0.25) : T(0.5));
                const T qm = sqrt(qy1[m] * qy1[m] + qp * qp);
                qsy1[m] = face_qm<T>(eta1[m], eta0[m], z1[m], z0[m], n1[m], n0[m], qy1[m], qm,
                                     K.gdt, K.inv_dx, K.h_eps);
            }
        } else {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                qsy1[m] = face_q<T>(eta1[m], eta0[m], z1[m], z0[m], n1[m], n0[m], qy1[m], K.gdt,
                                    K.inv_dx, K.h_eps);
        }
        if (EDGE && k - 1 == -1) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                qsy1[m] = G.outside[m] ? T(0) : border_q<T, VAR>(a, K, SIDE_S, G.i0 + m, h0[m]);
        } else if (EDGE && k - 1 == ny - 1) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                qsy1[m] = G.outside[m] ? T(0) : border_q<T, VAR>(a, K, SIDE_N, G.i0 + m, h1[m]);
        }

        // C: donor scaling factor of row k-1.
        const bool row1_real = (k - 1 >= 0 && k - 1 < ny);
        const T qWn = from_prev(qsx1[CPT - 1]);
        T r1[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const T qW = (m > 0) ? qsx1[(m + CPT - 1) % CPT] : qWn;
            T out = max0_neg(qW);
            out += max0(qsx1[m]);
            out += max0_neg(qsy2[m]);
            out += max0(qsy1[m]);
            const T O = (K.dt * out) * K.inv_dx;
            const T hp = max0(h1[m]);
            const T rr = (O > hp) ? donor_ratio<T>(hp, O) : T(1);
            r1[m] = (a.positivity && (!EDGE || (row1_real && !G.outside[m]))) ? rr : T(1);
        }

        // D: applied discharges: x-faces of row k-1 and y-faces between rows k-2 and k-1.
        const T rRn = from_next(r1[0]);
        T qnx1[CPT], qny2[CPT];
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const T rR = (m + 1 < CPT) ? r1[(m + 1) % CPT] : rRn;
            qnx1[m] = qsx1[m] * (qsx1[m] > T(0) ? r1[m] : rR);
            qny2[m] = qsy2[m] * (qsy2[m] > T(0) ? r2[m] : r1[m]);
        }

        // E: depth of row k-2 (eq. 4).
        const T qnWn = from_prev(qnx2[CPT - 1]);
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const T qW = (m > 0) ? qnx2[(m + CPT - 1) % CPT] : qnWn;
            hn[m] = h2[m] + (K.dt * ((qW - qnx2[m]) + (qny3[m] - qny2[m]))) * K.inv_dx;
            qxo[m] = qnx2[m];
            qyo[m] = qny2[m];
        }

#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            h2[m] = h1[m]; h1[m] = h0[m];
            eta1[m] = eta0[m]; z1[m] = z0[m]; n1[m] = n0[m]; qy1[m] = qy0[m];
            qsx1[m] = qsx0[m]; qsy2[m] = qsy1[m]; r2[m] = r1[m];
            qnx2[m] = qnx1[m]; qny3[m] = qny2[m];
            if constexpr ((VAR & VAR_FRICTION_VECTOR) != 0) qxo1[m] = qx0[m];
        }
    }
};

template <int CPT>
__device__ __forceinline__ StripGeo<CPT> strip_geo(int nx, int s, int wo, int wl, int lane) {
    StripGeo<CPT> G;
    const int pcol = s * wo + lane * CPT;
    G.i0 = pcol - kHalo;
    G.west_strip = (s == 0);
    // the east border can sit in the halo of the second-last strip
    G.east_strip = (nx - 1 >= s * wo - kHalo) && (nx - 1 < s * wo - kHalo + wl);
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int i = G.i0 + m;
        G.outside[m] = (i < 0 || i >= nx);
        G.west_face[m] = (i == -1);
        G.east_face[m] = (i == nx - 1);
    }
    return G;
}

// The bookkeeping of an output row ko of a work item: the deepest new depth,
// the border faces kept for read-back (edge arrays) and the outflow leaving
// the grid.  Row -1 carries the south border faces.
template <typename T, int CPT>
__device__ __forceinline__ void row_books(const StepArgs<T>& a, const StripGeo<CPT>& G,
                                          const bool (&store_col)[CPT], int ko, bool in_item,
                                          bool south_chunk, const T (&hn)[CPT],
                                          const T (&qxo)[CPT], const T (&qyo)[CPT],
                                          bool keep_edges, typename Ord<T>::U& hbits,
                                          double& outacc) {
    const int ny = a.ny;
    if (in_item) {
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            if (store_col[m]) {
                const typename Ord<T>::U b = Ord<T>::key(hn[m]);
                hbits = b > hbits ? b : hbits;
            }
        if (G.west_strip) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (G.west_face[m]) {
                    if (keep_edges) a.edge_w[ko] = qxo[m];
                    if (a.out_side == SIDE_W && a.kout[ko] > T(0)) outacc -= (double)qxo[m];
                }
        }
        if (G.east_strip && a.out_side == SIDE_E) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (G.east_face[m] && store_col[m] && a.kout[ko] > T(0)) outacc += (double)qxo[m];
        }
        if (ko == ny - 1 && a.out_side == SIDE_N) {
#pragma unroll
            for (int m = 0; m < CPT; ++m)
                if (store_col[m] && a.kout[G.i0 + m] > T(0)) outacc += (double)qyo[m];
        }
    } else if (ko == -1 && south_chunk) {
#pragma unroll
        for (int m = 0; m < CPT; ++m)
            if (store_col[m]) {
                if (keep_edges) a.edge_s[G.i0 + m] = qyo[m];
                if (a.out_side == SIDE_S && a.kout[G.i0 + m] > T(0)) outacc -= (double)qyo[m];
            }
    }
}

// Outflow partial-sum slot of a work item, or -1 if it has no outflow face.
template <typename T>
__device__ __forceinline__ int part_slot(const StepArgs<T>& a, int s, int c) {
    switch (a.out_side) {
    case SIDE_W: return s == 0 ? c : -1;
    case SIDE_E: return s == a.nstrips - 1 ? c : -1;
    case SIDE_S: return c == 0 ? s : -1;
    case SIDE_N: return c == a.nchunks - 1 ? s : -1;
    default: return -1;
    }
}

}  // namespace flood
