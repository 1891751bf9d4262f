/* Declarations shared by the two files of the FP64 CPU oracle (test
 * infrastructure only; nothing here is used by the GPU library). */
#ifndef FLOOD_ORACLE_H
#define FLOOD_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t nx, ny;
    double dx, g, alpha, dt_max, h_eps, dt_fixed, t_end;
    int32_t positivity;              /* 1 = donor-cell outflow scaling */
    int32_t in_side, in_first, in_count;
    double in_slope;
    int32_t nsamp;
    const double *ts, *qs;           /* hydrograph samples (s, m^3/s) */
    int32_t out_side, out_first, out_count;
    double out_slope;
    /* method variants (0 = the readings in flood_oracle.c's header) */
    int32_t friction_vector;         /* 1: |q| in eq. (3) is the discharge vector's magnitude */
    int32_t boundary_cell_area;      /* 1: A in eq. (5)/(6) is the cell area dx^2 */
} orc_problem;

typedef struct {
    double t, last_dt;
    int64_t steps;
    double v_in, v_out;
    int32_t done;                    /* 1 = reached t_end, 2 = non-finite depth */
} orc_clock;

enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };

int orc_one_step(const orc_problem *p, const double *z, const double *n, double *h, double *qx,
                 double *qy, double *r, orc_clock *clk, int nth);
double orc_hydrograph(int32_t ns, const double *ts, const double *qs, double t);
double orc_inflow_split(int32_t nc, const double *zc, const double *kc, double dx, double Q,
                        double *q_out);
double orc_inflow_split_area(int32_t nc, const double *zc, const double *kc, double dx, double Q,
                             double *q_out);
double orc_face_flux(double hL, double hR, double zL, double zR, double nL, double nR, double q,
                     double dx, double dt, double g, double h_eps);

#endif
