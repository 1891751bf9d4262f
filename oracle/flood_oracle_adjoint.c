/*
 * FP64 CPU reverse-mode derivative of the flood run (test infrastructure).
 *
 * Gradient of a gauge-misfit loss with respect to the per-cell Manning
 * coefficient n and the inflow hydrograph samples Q_k, for runs with a fixed
 * time step (the paper's own mode: a constant dt for all results, Methods,
 * "Shallow Water Equations").  The forward run is the oracle's step; every
 * state is kept (small grids only), then the steps are reversed one by one
 * with the chain rule written out in the order the step computes:
 *
 *   boundary faces  (eq. 5, 6)  ->  interior faces (eq. 3)  ->  donor-cell
 *   scaling  ->  depth update (eq. 4).
 *
 * Reverse of one step, for adjoints lh', lqx', lqy' of the new state:
 *   mu_f   = lq'_f + dt/dx (lh'_R - lh'_L)          adjoint of an applied face value
 *   rho_c  = sum over faces f that cell c drains of mu_f q*_f
 *   mu*_f  = mu_f r_d + nu_d sign(q*_f),  nu_d = rho_d d(r_d)/d(O_d) dO_d/dq*
 *            (d the donor of f; an inflow face has no donor: r = 1)
 *   lh_c   = lh'_c + rho_c dr_c/dh_c + sum_f mu*_f dq*_f/dh_c
 *   lq_f   = mu*_f dq*_f/dq_f,   grad n_c += sum_f mu*_f dq*_f/dn_c
 * and for the inflow section, with G(W) = sum_c dx k_c (W - z_c)_+^{5/3} - Q = 0
 * (eq. 6), k_c = sqrt(S_in)/n_c: dW/dQ = 1/D, dW/dk_j = -dx (W - z_j)^{5/3} / D,
 * D = sum_c dx k_c (5/3)(W - z_c)_+^{2/3}.  Q(t) is piecewise linear in the
 * samples, so dQ/dQ_k are the interpolation weights.
 * Choices at kinks: a max tie takes the left value; d|q|/dq = sign(q) with
 * sign(0) = 0; branches (dry face, active limiter, donor) follow the forward
 * values.  This file is written face by face ("scatter"), independently of
 * the GPU kernels.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "flood_oracle.h"

static double p53(double x)
{
    if (!(x > 0.0)) return 0.0;
    double c = cbrt(x);
    return x * (c * c);
}

static double p23(double x)  /* x^(2/3) for x > 0, else 0 */
{
    if (!(x > 0.0)) return 0.0;
    double c = cbrt(x);
    return c * c;
}

static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* Eq. (3) on one face with its partial derivatives. */
static double face_partials(double hL, double hR, double zL, double zR, double nL, double nR,
                            double q, double dx, double dt, double g, double h_eps,
                            double *Pq, double *PL, double *PR, double *Pn)
{
    double qs = orc_face_flux(hL, hR, zL, zR, nL, nR, q, dx, dt, g, h_eps);
    double etaL = hL + zL, etaR = hR + zR;
    double hf = fmax(etaL, etaR) - fmax(zL, zR);
    *Pq = *PL = *PR = *Pn = 0.0;
    if (hf <= h_eps) return qs;
    double nf = 0.5 * (nL + nR);
    double grad = (etaR - etaL) / dx;
    double num = q - ((g * hf) * dt) * grad;
    double c73 = (hf * hf) * cbrt(hf);                     /* hf^(7/3) */
    double fr = (g * dt) * (nf * nf);
    double den = 1.0 + (fr * fabs(q)) / c73;
    double dden_dq = fr * sgn(q) / c73;
    double dden_dhf = -(7.0 / 3.0) * fr * fabs(q) / (c73 * hf);
    double dden_dnf = 2.0 * (g * dt) * nf * fabs(q) / c73;
    double dnum_dhf = -(g * dt) * grad;
    double dnum_dgrad = -(g * hf) * dt;
    double dqs_dhf = (dnum_dhf - qs * dden_dhf) / den;
    double dqs_dgrad = dnum_dgrad / den;
    *Pq = (1.0 - qs * dden_dq) / den;
    *Pn = -qs * dden_dnf / den;
    double tieL = (etaL >= etaR) ? 1.0 : 0.0;
    *PL = dqs_dhf * tieL - dqs_dgrad / dx;
    *PR = dqs_dhf * (1.0 - tieL) + dqs_dgrad / dx;
    (void)num;
    return qs;
}

enum { K_INTERIOR = 0, K_WALL = 1, K_IN = 2, K_OUT = 3 };

typedef struct {
    int64_t nx, ny, nfx, nfy;
    /* per face (x faces first, then y faces): value, partials, kind, cells */
    double *qs, *Pq, *PL, *PR, *Pn, *mu, *mus;
    int *kind;
    int64_t *L, *R;          /* cell indices, -1 outside */
    double *O, *r, *rho, *nu;
    int *lim;
} adj_work;

static int64_t fidx_x(const adj_work *w, int64_t j, int64_t i) { return j * (w->nx + 1) + i; }
static int64_t fidx_y(const adj_work *w, int64_t j, int64_t i) { return w->nfx + j * w->nx + i; }

/* Side and position of a border cell's face, or -1. */
static int in_section(const orc_problem *p, int side, int first, int count, int32_t pos)
{
    (void)p;
    return (count > 0 && pos >= first && pos < first + count) ? side : -1;
}

/*
 * Reverse one step with fixed dt from state (h, qx, qy) at time t.  Inputs
 * lh1 [ny*nx], lqx1 [ny*(nx+1)], lqy1 [(ny+1)*nx] are the adjoints of the new
 * state; outputs lh, lqx, lqy the adjoints of (h, qx, qy); grad_n and grad_q
 * are accumulated.
 */
static void adj_step(const orc_problem *p, const double *z, const double *n, const double *h,
                     const double *qx, const double *qy, double t, const double *lh1,
                     const double *lqx1, const double *lqy1, double *lh, double *lqx, double *lqy,
                     double *grad_n, double *grad_q, adj_work *w)
{
    const int64_t nx = p->nx, ny = p->ny;
    const double dx = p->dx, g = p->g, dt = p->dt_fixed, cdt = dt / dx;
    const int64_t nf = w->nfx + w->nfy;

    /* inflow section at this step: W from eq. (6) */
    double Q = 0.0, W = 0.0;
    double *qin_c = NULL, *zc = NULL, *kc = NULL;
    if (p->in_count > 0) {
        zc = malloc(sizeof(double) * p->in_count);
        kc = malloc(sizeof(double) * p->in_count);
        qin_c = malloc(sizeof(double) * p->in_count);
        for (int32_t k = 0; k < p->in_count; k++) {
            int32_t pos = p->in_first + k;
            int64_t i = (p->in_side == SIDE_W) ? 0 : (p->in_side == SIDE_E) ? nx - 1 : pos;
            int64_t j = (p->in_side == SIDE_S) ? 0 : (p->in_side == SIDE_N) ? ny - 1 : pos;
            zc[k] = z[j * nx + i];
            kc[k] = sqrt(p->in_slope) / n[j * nx + i];
        }
        Q = orc_hydrograph(p->nsamp, p->ts, p->qs, t);
        W = orc_inflow_split(p->in_count, zc, kc, dx, Q, qin_c);
    }

    /* 1. faces of the forward step, with partials */
    for (int64_t j = 0; j < ny; j++)
        for (int64_t i = 0; i <= nx; i++) {
            int64_t f = fidx_x(w, j, i);
            w->L[f] = (i >= 1) ? j * nx + i - 1 : -1;
            w->R[f] = (i < nx) ? j * nx + i : -1;
            w->Pq[f] = w->PL[f] = w->PR[f] = w->Pn[f] = 0.0;
            if (i >= 1 && i < nx) {
                int64_t a = w->L[f], b = w->R[f];
                w->kind[f] = K_INTERIOR;
                w->qs[f] = face_partials(h[a], h[b], z[a], z[b], n[a], n[b], qx[f], dx, dt, g,
                                         p->h_eps, &w->Pq[f], &w->PL[f], &w->PR[f], &w->Pn[f]);
            } else {
                int side = (i == 0) ? SIDE_W : SIDE_E;
                double inward = (i == 0) ? 1.0 : -1.0;
                int64_t c = (i == 0) ? w->R[f] : w->L[f];
                w->kind[f] = K_WALL;
                w->qs[f] = 0.0;
                if (in_section(p, p->in_side, p->in_first, p->in_count, (int32_t)j) == side) {
                    w->kind[f] = K_IN;
                    w->qs[f] = inward * qin_c[j - p->in_first];
                } else if (in_section(p, p->out_side, p->out_first, p->out_count, (int32_t)j) == side) {
                    double hp = fmax(h[c], 0.0), ko = sqrt(p->out_slope) / n[c];
                    w->kind[f] = K_OUT;
                    w->qs[f] = -inward * ko * p53(hp);
                    w->PL[f] = -inward * ko * (5.0 / 3.0) * p23(hp) * (h[c] > 0.0);   /* d/dh_c */
                    w->Pn[f] = -inward * p53(hp) * (-sqrt(p->out_slope) / (n[c] * n[c])); /* d/dn_c */
                }
            }
        }
    for (int64_t j = 0; j <= ny; j++)
        for (int64_t i = 0; i < nx; i++) {
            int64_t f = fidx_y(w, j, i), fq = j * nx + i;
            w->L[f] = (j >= 1) ? (j - 1) * nx + i : -1;
            w->R[f] = (j < ny) ? j * nx + i : -1;
            w->Pq[f] = w->PL[f] = w->PR[f] = w->Pn[f] = 0.0;
            if (j >= 1 && j < ny) {
                int64_t a = w->L[f], b = w->R[f];
                w->kind[f] = K_INTERIOR;
                w->qs[f] = face_partials(h[a], h[b], z[a], z[b], n[a], n[b], qy[fq], dx, dt, g,
                                         p->h_eps, &w->Pq[f], &w->PL[f], &w->PR[f], &w->Pn[f]);
            } else {
                int side = (j == 0) ? SIDE_S : SIDE_N;
                double inward = (j == 0) ? 1.0 : -1.0;
                int64_t c = (j == 0) ? w->R[f] : w->L[f];
                w->kind[f] = K_WALL;
                w->qs[f] = 0.0;
                if (in_section(p, p->in_side, p->in_first, p->in_count, (int32_t)i) == side) {
                    w->kind[f] = K_IN;
                    w->qs[f] = inward * qin_c[i - p->in_first];
                } else if (in_section(p, p->out_side, p->out_first, p->out_count, (int32_t)i) == side) {
                    double hp = fmax(h[c], 0.0), ko = sqrt(p->out_slope) / n[c];
                    w->kind[f] = K_OUT;
                    w->qs[f] = -inward * ko * p53(hp);
                    w->PL[f] = -inward * ko * (5.0 / 3.0) * p23(hp) * (h[c] > 0.0);
                    w->Pn[f] = -inward * p53(hp) * (-sqrt(p->out_slope) / (n[c] * n[c]));
                }
            }
        }

    /* 2. donor scaling of the forward step, as the step computes it */
    for (int64_t j = 0; j < ny; j++)
        for (int64_t i = 0; i < nx; i++) {
            int64_t c = j * nx + i;
            double out = 0.0;
            out += fmax(0.0, -w->qs[fidx_x(w, j, i)]);
            out += fmax(0.0, w->qs[fidx_x(w, j, i + 1)]);
            out += fmax(0.0, -w->qs[fidx_y(w, j, i)]);
            out += fmax(0.0, w->qs[fidx_y(w, j + 1, i)]);
            double O = (dt * out) / dx, hp = fmax(h[c], 0.0);
            w->O[c] = O;
            w->lim[c] = p->positivity && (O > hp);
            w->r[c] = w->lim[c] ? hp / O : 1.0;
            w->rho[c] = 0.0;
        }

    /* 3. adjoint of each applied face value */
    for (int64_t f = 0; f < nf; f++) {
        double l1 = (w->kind[f] == K_INTERIOR) ? ((f < w->nfx) ? lqx1[f] : lqy1[f - w->nfx]) : 0.0;
        double hR = (w->R[f] >= 0) ? lh1[w->R[f]] : 0.0, hL = (w->L[f] >= 0) ? lh1[w->L[f]] : 0.0;
        w->mu[f] = l1 + cdt * (hR - hL);
    }
    /* 4. rho: what each cell sends out, weighted by the adjoints */
    for (int64_t f = 0; f < nf; f++) {
        if (w->kind[f] == K_IN) continue;
        int64_t d = (w->qs[f] > 0.0) ? w->L[f] : w->R[f];
        if (w->qs[f] != 0.0 && d >= 0) w->rho[d] += w->mu[f] * w->qs[f];
    }
    for (int64_t c = 0; c < nx * ny; c++) {
        double hp = fmax(h[c], 0.0);
        w->nu[c] = w->lim[c] ? w->rho[c] * (-hp / (w->O[c] * w->O[c])) * cdt : 0.0;
    }
    /* 5. adjoint of the unscaled face values */
    for (int64_t f = 0; f < nf; f++) {
        if (w->kind[f] == K_IN) { w->mus[f] = w->mu[f]; continue; }
        int64_t d = (w->qs[f] > 0.0) ? w->L[f] : w->R[f];
        double rd = (d >= 0) ? w->r[d] : 1.0, nud = (d >= 0) ? w->nu[d] : 0.0;
        w->mus[f] = w->mu[f] * rd + nud * sgn(w->qs[f]);
    }
    /* 6. cells: direct term and the limiter's dependence on the depth */
    for (int64_t c = 0; c < nx * ny; c++)
        lh[c] = lh1[c] + ((w->lim[c] && h[c] > 0.0) ? w->rho[c] / w->O[c] : 0.0);
    memset(lqx, 0, sizeof(double) * ny * (nx + 1));
    memset(lqy, 0, sizeof(double) * (ny + 1) * nx);
    /* 7. scatter the face derivatives */
    double *a_in = (p->in_count > 0) ? calloc(p->in_count, sizeof(double)) : NULL;
    for (int64_t f = 0; f < nf; f++) {
        double m = w->mus[f];
        if (w->kind[f] == K_INTERIOR) {
            lh[w->L[f]] += m * w->PL[f];
            lh[w->R[f]] += m * w->PR[f];
            grad_n[w->L[f]] += 0.5 * m * w->Pn[f];
            grad_n[w->R[f]] += 0.5 * m * w->Pn[f];
            if (f < w->nfx) lqx[f] = m * w->Pq[f];
            else lqy[f - w->nfx] = m * w->Pq[f];
        } else if (w->kind[f] == K_OUT) {
            int64_t c = (w->L[f] >= 0) ? w->L[f] : w->R[f];
            lh[c] += m * w->PL[f];
            grad_n[c] += m * w->Pn[f];
        } else if (w->kind[f] == K_IN) {
            int64_t c = (w->L[f] >= 0) ? w->L[f] : w->R[f];
            int64_t pos = (f < w->nfx) ? c / nx : c % nx;
            double inward = (w->R[f] >= 0 && w->L[f] < 0) ? 1.0 : -1.0;
            a_in[pos - p->in_first] = m * inward;
        }
    }
    /* 8. inflow: through W (eq. 6) to Q(t) and to k_c = sqrt(S_in)/n_c */
    if (p->in_count > 0 && Q > 0.0) {
        double D = 0.0, A = 0.0;
        for (int32_t k = 0; k < p->in_count; k++) {
            double e = kc[k] * (5.0 / 3.0) * p23(W - zc[k]);
            D += dx * e;
            A += a_in[k] * e;
        }
        double dLdQ = A / D;
        int32_t ns = p->nsamp;
        if (t <= p->ts[0]) grad_q[0] += dLdQ;
        else if (t >= p->ts[ns - 1]) grad_q[ns - 1] += dLdQ;
        else {
            int32_t k = 0;
            while (k + 1 < ns && p->ts[k + 1] <= t) k++;
            double wgt = (t - p->ts[k]) / (p->ts[k + 1] - p->ts[k]);
            grad_q[k] += (1.0 - wgt) * dLdQ;
            grad_q[k + 1] += wgt * dLdQ;
        }
        for (int32_t k = 0; k < p->in_count; k++) {
            int32_t pos = p->in_first + k;
            int64_t i = (p->in_side == SIDE_W) ? 0 : (p->in_side == SIDE_E) ? nx - 1 : pos;
            int64_t j = (p->in_side == SIDE_S) ? 0 : (p->in_side == SIDE_N) ? ny - 1 : pos;
            int64_t c = j * nx + i;
            double dLdk = p53(W - zc[k]) * (a_in[k] - dx * A / D);
            grad_n[c] += dLdk * (-sqrt(p->in_slope) / (n[c] * n[c]));
        }
    }
    free(a_in);
    free(zc);
    free(kc);
    free(qin_c);
}

/*
 * Fixed-dt run of nsteps steps from (h0, qx0, qy0) at t = 0 with gauge
 * observations of the depth at cells `gauges` after every obs_every steps;
 * series [nobs][ngauges] receives them, nobs = nsteps / obs_every.  The loss
 * is sum (series - obs)^2, or, when dl_dseries is given, its adjoint seeds are
 * dl_dseries.  grad_n [ny*nx] and grad_q [nsamp] receive dL/dn and dL/dQ_k.
 * Returns 0, 1 on bad arguments, 2 on a non-finite depth.
 */
int orc_adj_run(const orc_problem *p, const double *z, const double *n, const double *h0,
                const double *qx0, const double *qy0, int64_t nsteps, int32_t ngauges,
                const int64_t *gauges, int32_t obs_every, const double *obs, const double *dl_dseries,
                double *series, double *loss, double *grad_n, double *grad_q, int32_t nthreads)
{
    if (!p || !(p->dt_fixed > 0.0) || nsteps < 0 || obs_every < 1) return 1;
    /* the reverse is derived for the default readings only */
    if (p->friction_vector || p->boundary_cell_area) return 1;
    const int64_t nx = p->nx, ny = p->ny, nc = nx * ny;
    const int64_t nqx = ny * (nx + 1), nqy = (ny + 1) * nx;
    const int64_t nobs = nsteps / obs_every;
    double *H = malloc(sizeof(double) * nc * (nsteps + 1));
    double *QX = malloc(sizeof(double) * nqx * (nsteps + 1));
    double *QY = malloc(sizeof(double) * nqy * (nsteps + 1));
    double *T = malloc(sizeof(double) * (nsteps + 1));
    double *rbuf = malloc(sizeof(double) * nc);
    if (!H || !QX || !QY || !T || !rbuf) return 1;
    memcpy(H, h0, sizeof(double) * nc);
    memcpy(QX, qx0, sizeof(double) * nqx);
    memcpy(QY, qy0, sizeof(double) * nqy);
    orc_clock clk = {0};
    T[0] = 0.0;
    orc_problem pp = *p;
    pp.t_end = INFINITY;
    int rc = 0;
    for (int64_t s = 0; s < nsteps; s++) {
        double *h = H + nc * (s + 1), *qx = QX + nqx * (s + 1), *qy = QY + nqy * (s + 1);
        memcpy(h, H + nc * s, sizeof(double) * nc);
        memcpy(qx, QX + nqx * s, sizeof(double) * nqx);
        memcpy(qy, QY + nqy * s, sizeof(double) * nqy);
        if ((rc = orc_one_step(&pp, z, n, h, qx, qy, rbuf, &clk, nthreads > 0 ? nthreads : 1))) break;
        T[s + 1] = clk.t;
    }
    if (!rc) {
        double L = 0.0;
        for (int64_t o = 0; o < nobs; o++)
            for (int32_t k = 0; k < ngauges; k++) {
                double v = H[nc * ((o + 1) * obs_every) + gauges[k]];
                series[o * ngauges + k] = v;
                if (obs) L += (v - obs[o * ngauges + k]) * (v - obs[o * ngauges + k]);
            }
        *loss = L;
        adj_work w;
        w.nx = nx; w.ny = ny; w.nfx = nqx; w.nfy = nqy;
        int64_t nf = nqx + nqy;
        w.qs = calloc(nf, sizeof(double)); w.Pq = calloc(nf, sizeof(double));
        w.PL = calloc(nf, sizeof(double)); w.PR = calloc(nf, sizeof(double));
        w.Pn = calloc(nf, sizeof(double)); w.mu = calloc(nf, sizeof(double));
        w.mus = calloc(nf, sizeof(double)); w.kind = calloc(nf, sizeof(int));
        w.L = calloc(nf, sizeof(int64_t)); w.R = calloc(nf, sizeof(int64_t));
        w.O = calloc(nc, sizeof(double)); w.r = calloc(nc, sizeof(double));
        w.rho = calloc(nc, sizeof(double)); w.nu = calloc(nc, sizeof(double));
        w.lim = calloc(nc, sizeof(int));
        double *lh1 = calloc(nc, sizeof(double)), *lh = calloc(nc, sizeof(double));
        double *lqx1 = calloc(nqx, sizeof(double)), *lqx = calloc(nqx, sizeof(double));
        double *lqy1 = calloc(nqy, sizeof(double)), *lqy = calloc(nqy, sizeof(double));
        memset(grad_n, 0, sizeof(double) * nc);
        memset(grad_q, 0, sizeof(double) * (p->nsamp > 0 ? p->nsamp : 0));
        for (int64_t s = nsteps - 1; s >= 0; s--) {
            /* seed the adjoint of the state after step s from the observations */
            if ((s + 1) % obs_every == 0 && (s + 1) / obs_every <= nobs) {
                int64_t o = (s + 1) / obs_every - 1;
                for (int32_t k = 0; k < ngauges; k++) {
                    double v = series[o * ngauges + k];
                    lh1[gauges[k]] += dl_dseries ? dl_dseries[o * ngauges + k]
                                                 : 2.0 * (v - obs[o * ngauges + k]);
                }
            }
            adj_step(&pp, z, n, H + nc * s, QX + nqx * s, QY + nqy * s, T[s], lh1, lqx1, lqy1, lh,
                     lqx, lqy, grad_n, grad_q, &w);
            double *tmp;
            tmp = lh1; lh1 = lh; lh = tmp;
            tmp = lqx1; lqx1 = lqx; lqx = tmp;
            tmp = lqy1; lqy1 = lqy; lqy = tmp;
        }
        free(w.qs); free(w.Pq); free(w.PL); free(w.PR); free(w.Pn); free(w.mu); free(w.mus);
        free(w.kind); free(w.L); free(w.R); free(w.O); free(w.r); free(w.rho); free(w.nu);
        free(w.lim); free(lh1); free(lh); free(lqx1); free(lqx); free(lqy1); free(lqy);
    }
    free(H); free(QX); free(QY); free(T); free(rbuf);
    return rc;
}
