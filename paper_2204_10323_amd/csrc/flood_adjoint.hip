// Reverse of one fixed-dt flood step on the GPU (gather form: every thread
// owns one cell and collects what it needs from its four faces and
// neighbours; no atomics).  Used by the checkpointed adjoint of the runtime to
// obtain gradients of a gauge misfit with respect to the per-cell Manning n
// and the inflow hydrograph samples.
//
// For the adjoints lh', lq' of the new state (the step computes the boundary
// faces (eq. 5, 6), then eq. (3) on the interior faces, then donor-cell
// scaling, then eq. (4)):
//   mu_f  = lq'_f + dt/dx (lh'_R - lh'_L)               applied face value
//   rho_c = sum over faces f drained by cell c of mu_f q*_f
//   mu*_f = mu_f r_d + nu_d sign(q*_f),  nu_d = rho_d dr_d/dO_d * dt/dx
//   lh_c  = lh'_c + rho_c dr_c/dh_c + sum_f mu*_f dq*_f/dh_c
//   lq_f  = mu*_f dq*_f/dq_f,     dL/dn_c += sum_f mu*_f dq*_f/dn_c
// Pass A computes r, nu and rho dr/dh per cell; pass B the adjoints and the
// Manning gradient; a one-wave pass carries the inflow section through the
// water level W of eq. (6) to Q(t) and to the section's roughness.
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

// Kind of the border face of cell (i, j) on `side` (the cell is on that edge).
template <typename T>
__device__ __forceinline__ int border_kind(const AdjArgs<T>& a, int side, int pos) {
    if (a.in_side == side && pos >= a.in_first && pos < a.in_first + a.in_count) return F_IN;
    if (a.out_side == side && a.kout[pos] > T(0)) return F_OUT;
    return F_WALL;
}

// Outflow border value as the step computes it (border_q without inflow),
// with its derivatives in the edge cell's depth and roughness.
template <typename T>
__device__ __forceinline__ T outflow_fwd(const AdjArgs<T>& a, int side, int pos, T h, T n, T& d_dh,
                                         T& d_dn) {
    const T k = a.kout[pos];
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

// The four faces of cell (i, j): 0 W, 1 E, 2 S, 3 N.  Neighbour offset, the
// face's discharge offset, whether the cell is the face's left cell, side.
struct FaceGeo {
    long long nb, fq;
    bool cell_is_L;
    int side, pos;
    bool border;
};

__device__ __forceinline__ FaceGeo face_geo(int f, long long o, long long P, int i, int j, int nx,
                                            int ny, const long long* qoff) {
    FaceGeo g;
    switch (f) {
    case 0: g = {o - 1, o - 1, false, SIDE_W, j, i == 0}; break;
    case 1: g = {o + 1, o, true, SIDE_E, j, i == nx - 1}; break;
    case 2: g = {o - P, o - P, false, SIDE_S, i, j == 0}; break;
    default: g = {o + P, o, true, SIDE_N, i, j == ny - 1}; break;
    }
    (void)qoff;
    return g;
}

// Pass A: per cell, the donor factor r of the forward step, and the
// limiter's adjoint terms nu = rho dr/dO dt/dx and kappa = rho dr/dh.
// An extra block column runs the inflow pass of the step reversed just
// before (its pass B is complete; pass A reads nothing that pass touches), so
// it overlaps this pass instead of following the previous one.
template <typename T>
__device__ void adj_inflow(const AdjArgs<T>& a, double t);

template <typename T>
__global__ __launch_bounds__(256) void k_adj_a(AdjArgs<T> a) {
    if (blockIdx.x == gridDim.x - 1) {
        if (a.bc_prev && blockIdx.y == 0 && threadIdx.x < 64) adj_inflow<T>(a, a.t_prev);
        return;
    }
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i >= a.nx) return;
    const long long P = a.pitch, o = (long long)(j + kHalo) * P + i + kHalo;
    const T dt = (T)a.dt, inv_dx = T(1) / T(a.dx), gdt = T(a.g) * dt, h_eps = T(a.h_eps);
    const T dtdx = dt * inv_dx;
    const T h = a.h[o], z = a.z[o], nn = a.n[o], eta = h + z;
    const T lh_c = a.lh1[o];
    T qs[4], mu[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const FaceGeo g = face_geo(f, o, P, i, j, a.nx, a.ny, nullptr);
        const T lq = (f == 0 || f == 1) ? a.lqx1[g.fq] : a.lqy1[g.fq];
        const T lnb = a.lh1[g.nb];
        mu[f] = lq + dtdx * (g.cell_is_L ? (lnb - lh_c) : (lh_c - lnb));
        if (g.border) {
            const int kind = border_kind(a, g.side, g.pos);
            T d1, d2;
            qs[f] = (kind == F_OUT) ? outflow_fwd(a, g.side, g.pos, h, nn, d1, d2) : T(0);
        } else {
            const T hb = a.h[g.nb], zb = a.z[g.nb], nb = a.n[g.nb], eb = hb + zb;
            const T q = (f == 0 || f == 1) ? a.qx[g.fq] : a.qy[g.fq];
            qs[f] = g.cell_is_L ? face_q<T>(eta, eb, z, zb, nn, nb, q, gdt, inv_dx, h_eps)
                                : face_q<T>(eb, eta, zb, z, nb, nn, q, gdt, inv_dx, h_eps);
        }
    }
    T out = fmax(T(0), -qs[0]);
    out += fmax(T(0), qs[1]);
    out += fmax(T(0), -qs[2]);
    out += fmax(T(0), qs[3]);
    const T O = (dt * out) * inv_dx;
    const T hp = fmax(h, T(0));
    const bool lim = a.positivity && (O > hp);
    T rho = T(0);
    if (qs[0] < T(0)) rho += mu[0] * qs[0];
    if (qs[1] > T(0)) rho += mu[1] * qs[1];
    if (qs[2] < T(0)) rho += mu[2] * qs[2];
    if (qs[3] > T(0)) rho += mu[3] * qs[3];
    a.rr[o] = lim ? donor_ratio<T>(hp, O) : T(1);
    a.nu[o] = lim ? rho * (-hp / (O * O)) * dtdx : T(0);
    a.kap[o] = (lim && h > T(0)) ? rho / O : T(0);
}

// Pass B: adjoints of the state and the Manning gradient of one cell.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_b(AdjArgs<T> a) {
    const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
    if (i >= a.nx) return;
    const long long P = a.pitch, o = (long long)(j + kHalo) * P + i + kHalo;
    const T dt = (T)a.dt, inv_dx = T(1) / T(a.dx), gdt = T(a.g) * dt, h_eps = T(a.h_eps);
    const T dtdx = dt * inv_dx;
    const T h = a.h[o], z = a.z[o], nn = a.n[o], eta = h + z;
    const T lh_c = a.lh1[o];
    const T r_c = a.rr[o], nu_c = a.nu[o];
    T lh = lh_c + a.kap[o];
    T gn = T(0), lqx = T(0), lqy = T(0);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const FaceGeo g = face_geo(f, o, P, i, j, a.nx, a.ny, nullptr);
        const T lq = (f == 0 || f == 1) ? a.lqx1[g.fq] : a.lqy1[g.fq];
        const T lnb = a.lh1[g.nb];
        const T mu = lq + dtdx * (g.cell_is_L ? (lnb - lh_c) : (lh_c - lnb));
        if (g.border) {
            const int kind = border_kind(a, g.side, g.pos);
            if (kind == F_OUT) {
                T d_dh, d_dn;
                const T qs = outflow_fwd(a, g.side, g.pos, h, nn, d_dh, d_dn);
                // the edge cell drains this face (outward discharge)
                const T mus = mu * r_c + nu_c * T((qs > T(0)) - (qs < T(0)));
                lh += mus * d_dh;
                gn += mus * d_dn;
            } else if (kind == F_IN) {
                // no donor inside the grid: the inflow is applied unscaled
                const T sgn_in = (g.side == SIDE_W || g.side == SIDE_S) ? T(1) : T(-1);
                a.ain[g.pos - a.in_first] = (double)(mu * sgn_in);
            }
        } else {
            const T hb = a.h[g.nb], zb = a.z[g.nb], nb = a.n[g.nb], eb = hb + zb;
            const T q = (f == 0 || f == 1) ? a.qx[g.fq] : a.qy[g.fq];
            const FaceFwd<T> F = g.cell_is_L
                                     ? face_fwd<T>(h, hb, z, zb, nn, nb, q, gdt, inv_dx, h_eps)
                                     : face_fwd<T>(hb, h, zb, z, nb, nn, q, gdt, inv_dx, h_eps);
            // donor: the left cell if the face flows toward +axis, else the right one
            const bool donor_is_c = (F.qs > T(0)) == g.cell_is_L;
            const T r_d = donor_is_c ? r_c : a.rr[g.nb];
            const T nu_d = donor_is_c ? nu_c : a.nu[g.nb];
            const T mus = mu * r_d + nu_d * T((F.qs > T(0)) - (F.qs < T(0)));
            lh += mus * (g.cell_is_L ? F.PL : F.PR);
            gn += T(0.5) * mus * F.Pn;
            if (f == 1) lqx = mus * F.Pq;
            if (f == 3) lqy = mus * F.Pq;
        }
    }
    a.lh[o] = lh;
    a.lqx[o] = lqx;
    a.lqy[o] = lqy;
    a.gn[(long long)j * a.nx + i] += (double)gn;
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
// step's pass B complete): with G(W) = sum_c dx k_c (W - z_c)_+^{5/3} - Q = 0,
// dW/dQ = 1/D and dW/dk_j = -dx (W - z_j)^{5/3} / D, D = sum_c dx k_c (5/3)(W - z_c)^{2/3}.
template <typename T>
__device__ void adj_inflow(const AdjArgs<T>& a, double t) {
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
        A += a.ain[p] * e;
    }
    D = wave_sum(D);
    A = wave_sum(A);
    const double dLdQ = A / D;
    if (lane == 0) {
        a.gq[k0] += (k0 + 1 < a.nsamp && w > 0.0) ? (1.0 - w) * dLdQ : dLdQ;
        if (k0 + 1 < a.nsamp && w > 0.0) a.gq[k0 + 1] += w * dLdQ;
    }
    for (int p = lane; p < nc; p += 64) {
        const int pos = a.in_first + p;
        const int ci = (a.in_side == SIDE_W) ? 0 : (a.in_side == SIDE_E) ? a.nx - 1 : pos;
        const int cj = (a.in_side == SIDE_S) ? 0 : (a.in_side == SIDE_N) ? a.ny - 1 : pos;
        const double nc_ = (double)a.n[(long long)(cj + kHalo) * a.pitch + ci + kHalo];
        const double dLdk = pow53(W - a.in_z[p]) * (a.ain[p] - a.dx * A / D);
        a.gn[(long long)cj * a.nx + ci] += dLdk * (-sqrt(a.in_slope) / (nc_ * nc_));
    }
}

// The inflow pass on its own (the last step of a sweep).
template <typename T>
__global__ void k_adj_bc(AdjArgs<T> a) {
    adj_inflow<T>(a, a.t);
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

template <typename T>
hipError_t launch_adjoint_step(const AdjArgs<T>& a, hipStream_t s) {
    const dim3 grid((a.nx + 255) / 256, a.ny);
    hipLaunchKernelGGL((k_adj_a<T>), dim3(grid.x + 1, grid.y), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_adj_b<T>), grid, dim3(256), 0, s, a);
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
