// Internal declarations shared by the runtime and the kernels of libflood.
// Not part of the public interface (include/flood.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flood {

// Padded device layout of every cell or face field: two halo rows above and
// below, two halo columns on the left, row pitch `pitch` elements (a multiple
// of 256 bytes, at least nx + 8).  Cell (i, j) lives at (j + 2) * pitch + i + 2.
// qx holds the face east of each cell, qy the face north of each cell; the
// west and south border faces live in the edge arrays edge_w[ny], edge_s[nx].
constexpr int kHalo = 2;

// One slot of the double-buffered device clock.
struct ClockSlot {
    double t;          // simulated time at the start of the step that reads it
    double dt_prev;    // dt of the step that produced this state (0 for a no-op step)
    double last_dt;    // dt of the last step with dt > 0
    double v_in;       // inflow volume applied so far (FP64)
    double v_out;      // outflow volume applied so far, up to the step before dt_prev's
    long long steps;   // steps taken with dt > 0
    int done;          // t reached t_end
    int nonfinite;     // a depth became NaN or infinite
};

// Most steps one launch makes (multi-step launches, flood_fused.hip).
constexpr int kFuseMax = 3;

// Clock of the multi-step launches, one slot per launch parity.  A launch
// claims the state it wrote.  When it ran steps with speculated dts (pending:
// steps spec .. nclose - 1), the next launch compares each with the dt the
// depth maximum of the state before it gives; at the first that differs it
// redoes the launch up to that step from the launch's input, which the
// ping-pong buffers still hold.
struct FusedClock {
    ClockSlot ck;                 // clock of the claimed state; v_out without the last launch's outflow
    ClockSlot back;               // clock at the start of the last launch (v_out complete)
    ClockSlot mid[kFuseMax - 1];  // clock after each step of the last launch but its last
    double dt[kFuseMax];          // dt of each step of the last launch
    long long vsteps;             // steps claimed since entering multi-step mode (dt = 0 steps included)
    int cur;                      // buffer holding the claimed state
    int pending;                  // some of the last launch's dts were speculated and are not checked yet
    int spec;                     // the last launch's first speculated step
    int nclose;                   // steps of the last launch (their outflow is not in ck.v_out)
    long long gen;                // launches that produced the claimed state (a redo keeps the count);
                                  // active-tile flags of a launch live in slot gen % 3
};

// Device control block of one context.
struct DevCtl {
    ClockSlot clk[2];            // read clk[n % 2], written clk[(n + 1) % 2] by step n
    unsigned long long hmax[3];  // deepest cell as ordered bits: read [n%3], max into [(n+1)%3]
    double t_end;                // effective end time (host may lower it between launches)
    double report[8];            // filled by the flush kernel
    // multi-step launches: launch p reads cf[p % 2] and writes cf[(p + 1) % 2];
    // its tiles put the deepest cell after its step s into
    // hmf[kFuseMax (p % 3) + s] for every step but the last, and after its
    // last step into hmf[kFuseMax (p % 3) + kFuseMax - 1]
    FusedClock cf[2];
    unsigned long long hmf[3 * kFuseMax];
    long long targetf;           // steps to claim before launches become no-ops
    long long genf;              // generation of the last multi-step run's claimed state
};

template <typename T>
struct StepArgs {
    const T* h_in;
    const T* qx_in;
    const T* qy_in;
    T* h_out;
    T* qx_out;
    T* qy_out;
    const T* z;
    const T* n;
    T* edge_w;          // west border face values of the new state [ny]
    T* edge_s;          // south border face values of the new state [nx]
    const T* kout;      // outflow coefficient sqrt(S_out)/n_c along the outflow side (0 elsewhere)
    const T* qin;       // inflow face magnitudes applied this step, along the inflow side
    T* qin_next;        // written by the clock block for the next step
    const double* in_z; // inflow-section bed elevations (FP64)
    const double* in_k; // inflow-section sqrt(S_in)/n_c (FP64)
    const double* ts;   // hydrograph times
    const double* qs;   // hydrograph discharges
    double* part_cur;   // outflow partial sums written by this step [npart]
    const double* part_prev;  // partial sums of the previous step
    DevCtl* ctl;
    long long pitch;
    int nx, ny;
    int in_side, in_first, in_count, nsamp;
    int out_side, out_first, out_count, npart;
    int positivity;
    int freeze;                   // 1: dt forced to 0 (exact no-op steps, for tiling trials)
    int nstrips, nchunks, rows;   // tiling: strips along x, chunks of `rows` rows along y
    int phase;                    // step index modulo 6
    double dx, g, alpha, dt_max, h_eps, dt_fixed;
    // active-tile skipping: per work item, one byte per step (slot = step
    // modulo 3) that says whether the item's cells were wet or changed; NULL:
    // every item is computed every step
    unsigned char* act;
    long long act_stride;         // bytes per slot (>= nstrips * nchunks)
    int* act_list;                // the items a step computes (filled by the selection kernel)
    unsigned* act_count;          // [2]: list length of the step, by step parity; then [2][8]
                                  // work counters of the list kernel's block groups
    // method variant: bit 0 = friction by the discharge vector's magnitude,
    // bit 1 = boundary cells with the cell area (eq. 5 and 6 taken literally)
    int variant;
};

enum { VAR_FRICTION_VECTOR = 1, VAR_BOUNDARY_CELL_AREA = 2 };

// A multi-step launch: the grid, boundary data and constants (with the
// tiling of K steps per launch) in `a`; both ping-pong buffers, since the
// launch decides on the device which one holds its input.
template <typename T>
struct FusedArgs {
    StepArgs<T> a;
    T* h[2];
    T* qx[2];
    T* qy[2];
    double* part[kFuseMax][2];  // outflow partial sums of each step of a launch, by launch parity
    int K;              // steps per launch (2 or 3): strips output 64 CPT - 4 K columns
    int phase;          // launch counter modulo 6
    int resolve;        // 1: only check (and if needed redo) the last launch
};

// One member of a batch: its step arguments for each step counter modulo 6
// (buffer parity and slot indices), the step counter at the start of the run,
// and its work.
template <typename T>
struct BatchScen {
    StepArgs<T> a[6];
    long long n0;       // member's step counter when the run starts
    int items;          // tile work items per step
    int first;          // offset of this member's (1 + items) queue entries within a step
};

// Members are bin-packed onto the XCDs; each XCD has its own queue, served
// only by the waves running on it, so a member's data never leaves one L2.
constexpr int kMaxXcc = 16;

template <typename T>
struct BatchArgs {
    const BatchScen<T>* scen;     // grouped by XCD: members [xbegin[x], xbegin[x+1]) run on XCD x
    int nxcc;
    int xbegin[kMaxXcc + 1];
    int per_step[kMaxXcc];        // per XCD: sum over its members of (1 + items)
    long long nsteps;
    unsigned long long* next;     // per XCD work-queue head
    unsigned long long* done;     // per member: queue entries completed (monotone)
    int* error;                   // set when a wait exceeds its spin limit
    long long spin_limit;
};

// A member of a batch run with K = 2 or 3 steps per queue entry: its K-step
// launch arguments by settling flag and launch counter modulo 6, and its work.
template <typename T>
struct BatchScen2 {
    FusedArgs<T> a2[2][6];  // [resolve][launch counter % 6]
    int items;              // K-step work items per launch
    int first;              // offset of this member's (1 + items) entries within a launch
};

// A K-step batch run: every member makes `nlaunch` K-step launches with
// counters l0 .. l0 + nlaunch - 1, the last of which only settles (checks, and
// if needed redoes, the previous launch's speculated steps).  Queue layout and
// hand-over as in BatchArgs.
template <typename T>
struct Batch2Args {
    const BatchScen2<T>* scen;
    int nxcc;
    int xbegin[kMaxXcc + 1];
    int per_launch[kMaxXcc];      // per XCD: sum over its members of (1 + items)
    long long l0, nlaunch;
    unsigned long long* next;
    unsigned long long* done;
    int* error;
    long long spin_limit;
};

// Reverse of one fixed-dt step (flood_adjoint.hip).
template <typename T>
struct AdjArgs {
    const T* h;            // state x^n (padded layout)
    const T* qx;
    const T* qy;
    const T* z;
    const T* n;
    const T* lh1;          // adjoint of x^{n+1}
    const T* lqx1;
    const T* lqy1;
    T* lh;                 // adjoint of x^n
    T* lqx;
    T* lqy;
    double* gn;            // dL/dn per cell, dense [ny][nx], accumulated
    double* ain;           // adjoint of the inflow magnitudes [in_count], written by this step
    const double* ain_prev;  // ... written by the step reversed just before (its inflow pass)
    double* gn_in;         // the inflow pass's dL/dn terms by section position [in_count], accumulated
    double* gq;            // dL/dQ_k [nsamp], accumulated
    int rows;              // output rows per work item of the reverse pass
    const T* kout;
    const double* in_z;
    const double* in_k;
    const double* ts;
    const double* qs;
    long long pitch;
    int nx, ny;
    int in_side, in_first, in_count, nsamp;
    int out_side, out_first, out_count;
    int positivity;
    double dx, g, dt, h_eps, in_slope, out_slope;
    double t;              // time at the start of the forward step
    int bc_prev;           // 1: the inflow pass of the step reversed just before is still due
    double t_prev;         // ... and that step's start time
};

// Host-side launchers (flood_kernels.hip, flood_adjoint.hip).
template <typename T>
hipError_t launch_step(const StepArgs<T>& a, int cpt, hipStream_t s);
// Size the persistent grid of the active-tile step for cells-per-lane cpt
// (an occupancy query; call it outside graph capture before the first such launch).
template <typename T>
hipError_t prepare_step_list(int cpt);
template <typename T>
hipError_t launch_prime(const StepArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_flush(const StepArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_fold(const StepArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_batch(const BatchArgs<T>& b, int cpt, int device, hipStream_t s, int* blocks_out,
                        bool act);  // act: some member skips work items (active tiles)
template <typename T>
hipError_t launch_hmax_init(const T* h, long long pitch, int nx, int ny, DevCtl* ctl,
                            hipStream_t s);
template <typename T>
hipError_t launch_volume(const T* h, long long pitch, int nx, int ny, double* partials,
                         int nparts, double* out, hipStream_t s);
// Sets n bytes at p to v (a kernel, so that it can sit in a captured graph).
hipError_t launch_fill_bytes(unsigned char* p, long long n, unsigned char v, hipStream_t s);

// Output rows per work item of the reverse pass on an nx x ny grid.
int adjoint_rows(int nx, int ny);
template <typename T>
hipError_t launch_adjoint_step(const AdjArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_adjoint_inflow(const AdjArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_adjoint_fold_inflow(const AdjArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_gauge_gather(const T* h, long long pitch, int nx, const int* gauges, int ng,
                               T* dst, hipStream_t s);
template <typename T>
hipError_t launch_gauge_seed(T* lh, long long pitch, int nx, const int* cells, const int* ptr,
                             const int* list, int nu, const T* series, const T* obs, const T* dl,
                             hipStream_t s);

// Multi-step launches (flood_fused.hip).  enter: the single-step state at
// step counter n (its budget folded) becomes slot 0 of the multi-step clock,
// with `target` steps to claim; keep_gen: continue the launch generation of
// the previous multi-step run (its active-tile flags still hold).  leave: the
// state claimed after `launches` launches becomes the single-step state at
// counter n2 (buffer n2 % 2 must hold it).
template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, int cpt, hipStream_t s);
template <typename T>
hipError_t launch_enter_fused(const StepArgs<T>& single, long long target, int keep_gen,
                              hipStream_t s);
template <typename T>
hipError_t launch_leave_fused(const StepArgs<T>& single, const FusedArgs<T>& af,
                              long long launches, hipStream_t s);
// A persistent batch launch with k = 2 or 3 steps per queue entry
// (flood_fused.hip).
template <typename T>
hipError_t launch_batch2(const Batch2Args<T>& b, int cpt, int k, int device, hipStream_t s,
                         int* blocks_out);

int strip_width(int cpt);                 // output columns per work item for cells-per-lane cpt
int strip_width_fused(int cpt, int k);    // the same for k steps per launch
constexpr int kVolumeParts = 1024;

}  // namespace flood
