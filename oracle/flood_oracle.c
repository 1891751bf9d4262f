/*
 * FP64 CPU oracle for the local-inertial flood step (test infrastructure).
 *
 * This file is the plain, slow, obviously-correct definition that the GPU
 * library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does.  It
 * shares no code, header or constant with the GPU library.
 *
 * It follows the paper's Methods section ("Shallow Water Equations"):
 *   - staggered grid: depth at cell centres, discharge per unit width on the
 *     faces between cells;
 *   - eq. (3): semi-implicit face update of the discharge from the water
 *     surface gradient with Manning friction, per axis;
 *   - eq. (4): depth update from the discharge divergence;
 *   - eq. (5) and (6): Manning inflow (water level W solved so the section
 *     carries Q_in) and Manning outflow at each outflow cell;
 *   - all other border faces are closed walls (left unchanged, Appendix
 *     "Code structure", halo exchange paragraph).
 * Readings of points the paper leaves silent or garbled:
 *   - a dt multiplies the gravity term in the numerator of eq. (3);
 *   - |q| in the friction term is the same face's own discharge (1-D form);
 *   - h_f = max(eta_L, eta_R) - max(z_L, z_R), eta = h + z;
 *   - A in eq. (5) is the face section dx*h, i.e. q = h^{5/3} sqrt(S) / n;
 *   - face Manning n is the mean of the two cells; boundary faces use n_c;
 *   - a face is dry (q* = 0) when h_f <= h_eps;
 *   - donor-cell outflow scaling keeps depths non-negative conservatively;
 *   - dt = min(dt_max, alpha dx / sqrt(g h_max)) unless a fixed dt is given,
 *     the last step shortened to t_end;
 *   - Q_in is evaluated at the start of the step, piecewise linear in the
 *     hydrograph samples and constant beyond them; W by 64 bisections.
 * Two method variants, off by default, check how much results depend on two
 * of these readings:
 *   - friction_vector: |q| in the friction term of eq. (3) is the magnitude
 *     of the discharge vector at the face, sqrt(q^2 + q_perp^2), where q_perp
 *     is the mean of the start-of-step discharges on the perpendicular faces
 *     of the two cells beside the face (four faces; those on the border of
 *     the grid are left out of the mean).  This is the vector norm eq. (2)
 *     writes, instead of the per-axis 1-D form;
 *   - boundary_cell_area: eq. (5) and (6) taken literally, A = dx^2 and the
 *     hydraulic radius = the depth, so a boundary cell passes
 *     Q_c = dx^2 h^{2/3} sqrt(S) / n, i.e. q = dx h^{2/3} sqrt(S) / n per unit
 *     width of its border face.
 *
 * Layout (this file's own): h, z, n are [ny][nx]; qx is [ny][nx+1] with
 * qx[j][i] the face between cells i-1 and i (i = 0 the west border, i = nx
 * the east border); qy is [ny+1][nx] with qy[j][i] the face between rows j-1
 * and j (j = 0 the south border, j = ny the north border).  Positive
 * discharge points toward +x / +y.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "flood_oracle.h"

/* x^(5/3) for x > 0, else 0. */
static double pow53(double x)
{
    if (!(x > 0.0)) return 0.0;
    double c = cbrt(x);
    return x * (c * c);
}

/* x^(2/3) for x > 0, else 0. */
static double pow23(double x)
{
    if (!(x > 0.0)) return 0.0;
    double c = cbrt(x);
    return c * c;
}

/* Hydrograph Q_in(t): piecewise linear, constant outside the samples. */
double orc_hydrograph(int32_t ns, const double *ts, const double *qs, double t)
{
    if (ns <= 0) return 0.0;
    if (t <= ts[0]) return qs[0];
    if (t >= ts[ns - 1]) return qs[ns - 1];
    int32_t k = 0;
    while (k + 1 < ns && ts[k + 1] <= t) k++;
    return qs[k] + (qs[k + 1] - qs[k]) * ((t - ts[k]) / (ts[k + 1] - ts[k]));
}

/*
 * Eq. (6): the water level W at which the Manning discharges of the section
 * cells add up to Q.  kc = sqrt(S_in)/n_c; each cell passes dx*kc*(W-z_c)_+^{5/3}.
 * The sum is continuous and strictly increasing above min z, so W is unique;
 * it is bracketed and bisected 64 times.  Writes the per-unit-width face
 * discharge of every cell into q_out and returns W.
 */
double orc_inflow_split(int32_t nc, const double *zc, const double *kc, double dx,
                        double Q, double *q_out)
{
    if (nc <= 0) return 0.0;
    if (!(Q > 0.0)) {
        for (int32_t c = 0; c < nc; c++) q_out[c] = 0.0;
        return zc[0];
    }
    double lo = zc[0], hi = zc[0], ksum = 0.0;
    for (int32_t c = 0; c < nc; c++) {
        if (zc[c] < lo) lo = zc[c];
        if (zc[c] > hi) hi = zc[c];
        ksum += kc[c];
    }
    hi += pow(Q / (dx * ksum), 0.6);
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (lo + hi), F = 0.0;
        for (int32_t c = 0; c < nc; c++) F += dx * kc[c] * pow53(mid - zc[c]);
        F -= Q;
        if (F < 0.0) lo = mid; else hi = mid;
    }
    double W = 0.5 * (lo + hi);
    for (int32_t c = 0; c < nc; c++) q_out[c] = kc[c] * pow53(W - zc[c]);
    return W;
}

/*
 * Eq. (6) with eq. (5) taken literally (variant boundary_cell_area): each cell
 * passes Q_c = dx^2 kc (W - z_c)_+^{2/3}; the sum is continuous and strictly
 * increasing above min z.  At W = max z + (Q / (dx^2 sum kc))^{3/2} every cell
 * passes at least its share, so that bounds W from above; 64 bisections.
 * Writes the per-unit-width face discharge Q_c / dx of every cell into q_out
 * and returns W.
 */
double orc_inflow_split_area(int32_t nc, const double *zc, const double *kc, double dx,
                             double Q, double *q_out)
{
    if (nc <= 0) return 0.0;
    if (!(Q > 0.0)) {
        for (int32_t c = 0; c < nc; c++) q_out[c] = 0.0;
        return zc[0];
    }
    double lo = zc[0], hi = zc[0], ksum = 0.0;
    for (int32_t c = 0; c < nc; c++) {
        if (zc[c] < lo) lo = zc[c];
        if (zc[c] > hi) hi = zc[c];
        ksum += kc[c];
    }
    hi += pow(Q / (dx * dx * ksum), 1.5);
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (lo + hi), F = 0.0;
        for (int32_t c = 0; c < nc; c++) F += dx * (dx * kc[c] * pow23(mid - zc[c]));
        F -= Q;
        if (F < 0.0) lo = mid; else hi = mid;
    }
    double W = 0.5 * (lo + hi);
    for (int32_t c = 0; c < nc; c++) q_out[c] = dx * kc[c] * pow23(W - zc[c]);
    return W;
}

/* Cell (i, j) of entry k of a boundary section on `side`. */
static void side_cell(const orc_problem *p, int32_t side, int32_t k, int32_t *i, int32_t *j)
{
    switch (side) {
    case SIDE_W: *i = 0;          *j = k;          break;
    case SIDE_E: *i = p->nx - 1;  *j = k;          break;
    case SIDE_S: *i = k;          *j = 0;          break;
    default:     *i = k;          *j = p->ny - 1;  break;
    }
}

/* Address of the border face of that cell and the sign of "into the domain". */
static double *side_face(const orc_problem *p, double *qx, double *qy, int32_t side,
                         int32_t i, int32_t j, double *inward)
{
    int64_t nx = p->nx;
    switch (side) {
    case SIDE_W: *inward = 1.0;  return &qx[j * (nx + 1) + 0];
    case SIDE_E: *inward = -1.0; return &qx[j * (nx + 1) + nx];
    case SIDE_S: *inward = 1.0;  return &qy[(int64_t)0 * nx + i];
    default:     *inward = -1.0; return &qy[(int64_t)p->ny * nx + i];
    }
}

/*
 * Eq. (3) on one interior face between cells L and R (R on the +axis side).
 * q is the face's discharge at the start of the step, qm the discharge
 * magnitude in the friction term.
 */
static double face_flux_m(double hL, double hR, double zL, double zR, double nL, double nR,
                          double q, double qm, double dx, double dt, double g, double h_eps)
{
    double etaL = hL + zL, etaR = hR + zR;
    double hf = fmax(etaL, etaR) - fmax(zL, zR);
    if (hf <= h_eps) return 0.0;
    double nf = 0.5 * (nL + nR);
    double grad = (etaR - etaL) / dx;
    double num = q - ((g * hf) * dt) * grad;
    double den = 1.0 + (((g * dt) * (nf * nf)) * qm) / ((hf * hf) * cbrt(hf));
    return num / den;
}

/* Eq. (3) with the face's own |q| in the friction term (the 1-D form). */
double orc_face_flux(double hL, double hR, double zL, double zR, double nL, double nR,
                     double q, double dx, double dt, double g, double h_eps)
{
    return face_flux_m(hL, hR, zL, zR, nL, nR, q, fabs(q), dx, dt, g, h_eps);
}

/* Variant friction_vector: mean of the start-of-step y-discharges on the
 * faces of the two cells beside the x-face qx[j][i] (faces qy[jj][i-1] and
 * qy[jj][i] for jj = j, j + 1), border faces left out. */
static double perp_mean_x(const double *qy0, int64_t nx, int64_t ny, int64_t i, int64_t j)
{
    double s = 0.0;
    int k = 0;
    for (int64_t jj = j; jj <= j + 1; jj++) {
        if (jj < 1 || jj > ny - 1) continue;
        s += qy0[jj * nx + i - 1] + qy0[jj * nx + i];
        k += 2;
    }
    return k ? s / k : 0.0;
}

/* The same for the y-face qy[j][i]: x-discharges on the faces qx[j-1][ii] and
 * qx[j][ii] for ii = i, i + 1 (the west and east faces of the two cells). */
static double perp_mean_y(const double *qx0, int64_t nx, int64_t i, int64_t j)
{
    double s = 0.0;
    int k = 0;
    for (int64_t ii = i; ii <= i + 1; ii++) {
        if (ii < 1 || ii > nx - 1) continue;
        s += qx0[(j - 1) * (nx + 1) + ii] + qx0[j * (nx + 1) + ii];
        k += 2;
    }
    return k ? s / k : 0.0;
}

static int orc_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* One step of the method.  Returns 0, or 2 if a non-finite depth was found. */
int orc_one_step(const orc_problem *p, const double *z, const double *n,
                        double *h, double *qx, double *qy, double *r, orc_clock *clk,
                        int nth)
{
    const int64_t nx = p->nx, ny = p->ny;
    const double dx = p->dx, g = p->g;

    /* dt: fixed, or CFL-limited by the deepest cell; last step shortened. */
    double hmax = 0.0;
    int bad = 0;
    for (int64_t c = 0; c < nx * ny; c++) {
        if (!isfinite(h[c])) bad = 1;
        else if (h[c] > hmax) hmax = h[c];
    }
    if (bad) return 2;
    double dt;
    if (p->dt_fixed > 0.0) dt = p->dt_fixed;
    else if (hmax > 0.0) dt = fmin(p->dt_max, p->alpha * dx / sqrt(g * hmax));
    else dt = p->dt_max;
    int last = 0;
    if (isfinite(p->t_end)) {
        double rem = p->t_end - clk->t;
        if (!(rem > 0.0)) { clk->done = 1; return 0; }
        if (dt >= rem) { dt = rem; last = 1; }
    }

    /* Eq. (3) on every interior face (q^n read and q* written in place). */
    if (!p->friction_vector) {
#pragma omp parallel for num_threads(nth) schedule(static)
        for (int64_t j = 0; j < ny; j++) {
            for (int64_t i = 1; i < nx; i++) {
                int64_t L = j * nx + i - 1, R = j * nx + i;
                double *q = &qx[j * (nx + 1) + i];
                *q = orc_face_flux(h[L], h[R], z[L], z[R], n[L], n[R], *q, dx, dt, g, p->h_eps);
            }
            if (j >= 1) {
                for (int64_t i = 0; i < nx; i++) {
                    int64_t L = (j - 1) * nx + i, R = j * nx + i;
                    double *q = &qy[j * nx + i];
                    *q = orc_face_flux(h[L], h[R], z[L], z[R], n[L], n[R], *q, dx, dt, g, p->h_eps);
                }
            }
        }
    } else {
        /* the perpendicular discharges are read from a copy of q^n */
        double *qx0 = malloc(sizeof(double) * (size_t)(ny * (nx + 1)));
        double *qy0 = malloc(sizeof(double) * (size_t)((ny + 1) * nx));
        if (!qx0 || !qy0) { free(qx0); free(qy0); return 2; }
        memcpy(qx0, qx, sizeof(double) * (size_t)(ny * (nx + 1)));
        memcpy(qy0, qy, sizeof(double) * (size_t)((ny + 1) * nx));
#pragma omp parallel for num_threads(nth) schedule(static)
        for (int64_t j = 0; j < ny; j++) {
            for (int64_t i = 1; i < nx; i++) {
                int64_t L = j * nx + i - 1, R = j * nx + i;
                double q = qx0[j * (nx + 1) + i], qp = perp_mean_x(qy0, nx, ny, i, j);
                qx[j * (nx + 1) + i] = face_flux_m(h[L], h[R], z[L], z[R], n[L], n[R], q,
                                                   sqrt(q * q + qp * qp), dx, dt, g, p->h_eps);
            }
            if (j >= 1) {
                for (int64_t i = 0; i < nx; i++) {
                    int64_t L = (j - 1) * nx + i, R = j * nx + i;
                    double q = qy0[j * nx + i], qp = perp_mean_y(qx0, nx, i, j);
                    qy[j * nx + i] = face_flux_m(h[L], h[R], z[L], z[R], n[L], n[R], q,
                                                 sqrt(q * q + qp * qp), dx, dt, g, p->h_eps);
                }
            }
        }
        free(qx0);
        free(qy0);
    }

    /* Border faces: closed walls unless an inflow or outflow section sets them. */
    for (int64_t j = 0; j < ny; j++) { qx[j * (nx + 1)] = 0.0; qx[j * (nx + 1) + nx] = 0.0; }
    for (int64_t i = 0; i < nx; i++) { qy[i] = 0.0; qy[ny * nx + i] = 0.0; }

    /* Inflow, eq. (6), from Q_in at the start of the step. */
    double sum_in = 0.0;
    if (p->in_count > 0) {
        int32_t nc = p->in_count;
        double *zc = malloc(sizeof(double) * nc), *kc = malloc(sizeof(double) * nc);
        double *qc = malloc(sizeof(double) * nc);
        for (int32_t k = 0; k < nc; k++) {
            int32_t i, j;
            side_cell(p, p->in_side, p->in_first + k, &i, &j);
            zc[k] = z[(int64_t)j * nx + i];
            kc[k] = sqrt(p->in_slope) / n[(int64_t)j * nx + i];
        }
        double Q = orc_hydrograph(p->nsamp, p->ts, p->qs, clk->t);
        if (p->boundary_cell_area) orc_inflow_split_area(nc, zc, kc, dx, Q, qc);
        else orc_inflow_split(nc, zc, kc, dx, Q, qc);
        for (int32_t k = 0; k < nc; k++) {
            int32_t i, j;
            double inward;
            side_cell(p, p->in_side, p->in_first + k, &i, &j);
            double *f = side_face(p, qx, qy, p->in_side, i, j, &inward);
            *f = inward * qc[k];
            sum_in += qc[k];
        }
        free(zc); free(kc); free(qc);
    }
    /* Outflow: Manning discharge of each outflow cell from its own depth, outward only. */
    if (p->out_count > 0) {
        for (int32_t k = 0; k < p->out_count; k++) {
            int32_t i, j;
            double inward;
            side_cell(p, p->out_side, p->out_first + k, &i, &j);
            int64_t c = (int64_t)j * nx + i;
            double hc = fmax(h[c], 0.0);
            double q = sqrt(p->out_slope) / n[c] *
                       (p->boundary_cell_area ? dx * pow23(hc) : pow53(hc));
            double *f = side_face(p, qx, qy, p->out_side, i, j, &inward);
            *f = -inward * q;
        }
    }

    /* Donor-cell scaling: no cell may send out more water than it holds. */
    if (p->positivity) {
#pragma omp parallel for num_threads(nth) schedule(static)
        for (int64_t j = 0; j < ny; j++) {
            for (int64_t i = 0; i < nx; i++) {
                double out = 0.0;
                out += fmax(0.0, -qx[j * (nx + 1) + i]);       /* west face  */
                out += fmax(0.0, qx[j * (nx + 1) + i + 1]);    /* east face  */
                out += fmax(0.0, -qy[j * nx + i]);             /* south face */
                out += fmax(0.0, qy[(j + 1) * nx + i]);        /* north face */
                double O = (dt * out) / dx;
                double hp = fmax(h[j * nx + i], 0.0);
                r[j * nx + i] = (O > hp) ? hp / O : 1.0;
            }
        }
#pragma omp parallel for num_threads(nth) schedule(static)
        for (int64_t j = 0; j < ny; j++) {
            for (int64_t i = 0; i <= nx; i++) {          /* x-faces; donors outside the grid keep r = 1 */
                double *q = &qx[j * (nx + 1) + i];
                if (*q > 0.0 && i >= 1) *q *= r[j * nx + i - 1];
                else if (*q < 0.0 && i < nx) *q *= r[j * nx + i];
            }
        }
#pragma omp parallel for num_threads(nth) schedule(static)
        for (int64_t j = 0; j <= ny; j++) {
            for (int64_t i = 0; i < nx; i++) {           /* y-faces */
                double *q = &qy[j * nx + i];
                if (*q > 0.0 && j >= 1) *q *= r[(j - 1) * nx + i];
                else if (*q < 0.0 && j < ny) *q *= r[j * nx + i];
            }
        }
    }

    /* Eq. (4): depth from the divergence of the applied discharges. */
#pragma omp parallel for num_threads(nth) schedule(static)
    for (int64_t j = 0; j < ny; j++) {
        for (int64_t i = 0; i < nx; i++) {
            double qW = qx[j * (nx + 1) + i], qE = qx[j * (nx + 1) + i + 1];
            double qS = qy[j * nx + i], qN = qy[(j + 1) * nx + i];
            h[j * nx + i] = h[j * nx + i] + (dt * ((qW - qE) + (qS - qN))) / dx;
        }
    }

    /* Volume budget (applied boundary discharges) and clock. */
    double sum_out = 0.0;
    for (int32_t k = 0; k < p->out_count; k++) {
        int32_t i, j;
        double inward;
        side_cell(p, p->out_side, p->out_first + k, &i, &j);
        double *f = side_face(p, qx, qy, p->out_side, i, j, &inward);
        sum_out += -inward * *f;
    }
    clk->v_in += dt * dx * sum_in;
    clk->v_out += dt * dx * sum_out;
    clk->t = last ? p->t_end : clk->t + dt;
    clk->last_dt = dt;
    clk->steps += 1;
    if (last) clk->done = 1;
    return 0;
}

/*
 * Run up to nsteps steps in place.  Stops early (clk->done set) at t_end or
 * on a non-finite depth.  Returns 0 on success, 2 on a non-finite depth,
 * 1 on bad arguments.
 */
int orc_run(const orc_problem *p, const double *z, const double *n, double *h,
            double *qx, double *qy, orc_clock *clk, int64_t nsteps, int32_t nthreads)
{
    if (!p || p->nx < 1 || p->ny < 1 || !(p->dx > 0.0)) return 1;
    int nth = orc_threads(nthreads);
    double *r = malloc(sizeof(double) * (size_t)p->nx * (size_t)p->ny);
    if (!r) return 1;
    int rc = 0;
    for (int64_t s = 0; s < nsteps && !clk->done; s++) {
        rc = orc_one_step(p, z, n, h, qx, qy, r, clk, nth);
        if (rc) { clk->done = 2; break; }
    }
    free(r);
    return rc;
}

/* Volume dx^2 * sum(h) in FP64. */
double orc_volume(int32_t nx, int32_t ny, double dx, const double *h)
{
    double s = 0.0;
    for (int64_t c = 0; c < (int64_t)nx * ny; c++) s += h[c];
    return s * dx * dx;
}

int32_t orc_threads_used(int32_t nthreads) { return orc_threads(nthreads); }
