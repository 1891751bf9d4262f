// Host runtime of libflood: contexts, input validation, device buffers, the
// captured multi-step graph and the C interface declared in include/flood.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flood.h"
#include "flood_internal.h"

using namespace flood;

// Device scratch of fl_batch_run_noalloc: the batch's member descriptors, the
// per-XCD queue heads, the per-member completion counters and the error flag,
// for callers that cannot allocate.  One copy per GPU, held until the process
// ends; every fl_batch_run_noalloc call on a GPU uses it (overlapping calls on
// one GPU race).  Host code must not pass `scratch` itself to a kernel: its
// device address comes from hipGetSymbolAddress (scratch_ptr below).
constexpr size_t kScratchBytes = 1u << 20;   // 1 MiB
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_create_error;

// Device address of `scratch` per device, taken once per device (at the first
// fl_create on it, with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

size_t elem_size(fl_precision p) { return p == FL_F64 ? sizeof(double) : sizeof(float); }

}  // namespace

struct fl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    fl_precision prec = FL_F32;
    std::string err;

    // grid and inputs (host copies, element type of the context, row stride nx)
    int nx = 0, ny = 0;
    double dx = 0.0;
    bool have_grid = false, have_z = false, have_n = false, have_state = false;
    std::vector<unsigned char> z, n, h0, qx0, qy0;
    double t0 = 0.0;
    int in_side = -1, in_first = 0, in_count = 0;
    double in_slope = 0.0;
    std::vector<double> ts, qs;
    int out_side = -1, out_first = 0, out_count = 0;
    double out_slope = 0.0;
    fl_params params{};

    // launch configuration (rows_req 0 = automatic)
    int cpt = 0, rows = 0, rows_req = 0;

    // device state
    bool committed = false;
    long long pitch = 0;
    int nstrips = 0, nchunks = 0, npart = 0;
    void *d_h[2] = {nullptr, nullptr}, *d_qx[2] = {nullptr, nullptr}, *d_qy[2] = {nullptr, nullptr};
    void *d_z = nullptr, *d_n = nullptr, *d_edge_w = nullptr, *d_edge_s = nullptr;
    void *d_kout = nullptr, *d_qin[2] = {nullptr, nullptr};
    double *d_in_z = nullptr, *d_in_k = nullptr, *d_ts = nullptr, *d_qs = nullptr;
    double *d_part[2] = {nullptr, nullptr}, *d_vol_part = nullptr, *d_vol = nullptr;
    DevCtl* d_ctl = nullptr;
    std::vector<void*> allocs;
    size_t dev_bytes = 0;
    // caller-owned device memory for the commit buffers (fl_bind_workspace)
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0, ws_used = 0;
    long long nstep = 0;  // steps enqueued since commit
    double v0 = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_k = 0;

    // multi-step launches (fl_set_fusion): steps per launch (1, or fuse_k),
    // the steps per launch of the committed multi-step tiling (0: none),
    // requested and effective tiling, outflow partial sums of each step of a
    // launch by launch parity
    int fuse = 1, fuse_k = 0, cpt2_req = 0, rows2_req = 0;
    int cpt2 = 0, rows2 = 0, nstrips2 = 0, nchunks2 = 0, npart2 = 0;
    double* d_part2[2 * kFuseMax] = {};
    hipGraph_t graph2 = nullptr;
    hipGraphExec_t graph2_exec = nullptr;
    int graph2_k = 0;

    // active-tile skipping (fl_set_active_tiles): per work item one flag byte
    // in each of three slots; sized for the smallest work items any tiling
    // can have.  The single-step path indexes the slots by step counter, the
    // two-step path by its device-side launch generation.  act_mode says which
    // path wrote them (0: stale) and act_at the step counter at which they
    // describe the state; any other path that moves the state leaves them
    // stale, and they are set to 1 (compute everything) before the next
    // skipping run.
    int active = 0, act_mode = 0;
    int act_cpt = 0, act_rows = 0;  // the single-step tiling (own or a batch's) the flags refer to
    unsigned char* d_act = nullptr;
    int* d_act_list = nullptr;        // items a single-step launch computes (selection kernel)
    int act_list_mode = 0;            // 1: single-step launches select a list first (fl_autotune)
    unsigned* d_act_count = nullptr;  // [2] their number, by step parity; [2 + 8 p + g] work counters
    long long act_stride = 0, act_at = -1;
    // method variant (fl_set_variant): bit 0 vector friction, bit 1 cell-area boundaries
    int variant = 0;

    // reverse mode (fl_adj_*): settings, checkpoints and the forward's record
    bool adj_setup = false;
    std::vector<int> gauges;
    int obs_every = 0, ckpt_req = 0;
    long long nobs_set = 0;
    std::vector<void*> adj_allocs;       // freed by a new setup, commit or destroy
    int* d_gauges = nullptr;
    int* d_gcell = nullptr;              // gauges grouped by cell: cells, offsets, gauge indices
    int ngcell = 0;
    void* d_obs = nullptr;
    void* d_series = nullptr;
    void* d_ck = nullptr;                // checkpoints: [nck][h, qx, qy fields]
    DevCtl* d_ck_ctl = nullptr;          // [nck]
    void* d_ck_qin = nullptr;            // [nck][side length]
    void* d_end = nullptr;               // the end-of-forward clock, inflow, partials, edges
    void* d_bwd = nullptr;               // scratch of the backward sweep (stores, adjoints, gradients)
    long long adj_n0 = 0, adj_nsteps = 0, adj_C = 0, adj_nck = 0, adj_nobs = 0;
    double adj_t0 = 0.0;
};

namespace {

fl_status fail(fl_ctx* c, fl_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

fl_status hip_fail(fl_ctx* c, hipError_t e, const char* what) {
    return fail(c, FL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// A HIP event destroyed when it goes out of scope, so that an early error
// return does not leak it.
struct Event {
    hipEvent_t e = nullptr;
    Event() = default;
    Event(const Event&) = delete;
    Event& operator=(const Event&) = delete;
    ~Event() {
        if (e) (void)hipEventDestroy(e);
    }
};

#define HIP_TRY(c, call)                                                  \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return hip_fail((c), e_, #call);            \
    } while (0)

size_t esz(const fl_ctx* c) { return elem_size(c->prec); }

double get_elem(const fl_ctx* c, const unsigned char* base, size_t idx) {
    if (c->prec == FL_F64) {
        double v;
        std::memcpy(&v, base + idx * sizeof(double), sizeof(double));
        return v;
    }
    float v;
    std::memcpy(&v, base + idx * sizeof(float), sizeof(float));
    return v;
}

// A pointer the caller declares to be on the device must be device (or
// managed) memory of the context's device; anything else would be read or
// written as device memory by a copy.  A host pointer makes the query fail:
// that error is cleared here so that it is not reported by a later call.
fl_status need_device(fl_ctx* c, const void* p, const char* what) {
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) (void)hipGetLastError();
    if (e != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) ||
        at.device != c->device)
        return fail(c, FL_EINVAL, std::string(what) + ": not device memory of the context's device");
    return FL_OK;
}

// Copies `rows` rows of row_bytes bytes from device memory (row pitch spitch)
// to host memory (row pitch dpitch) on stream s and waits for them.  Pitched
// rows go as 1D copies of whole row blocks through a host staging buffer of
// at most 64 MiB: pitched device-to-host copies into pageable memory have
// been seen to leave the destination untouched under rocprofv3, while 1D
// copies arrive.
fl_status rows_to_host(fl_ctx* c, unsigned char* dst, size_t dpitch, const unsigned char* src,
                       size_t spitch, size_t row_bytes, int rows, hipStream_t s) {
    if (rows <= 0 || row_bytes == 0) return FL_OK;
    if (dpitch == row_bytes && spitch == row_bytes) {
        HIP_TRY(c, hipMemcpyAsync(dst, src, row_bytes * rows, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        return FL_OK;
    }
    const int block = (int)std::max<size_t>(1, std::min<size_t>((size_t)rows, (size_t(64) << 20) / spitch));
    std::vector<unsigned char> stage((size_t)(block - 1) * spitch + row_bytes);
    for (int r0 = 0; r0 < rows; r0 += block) {
        const int n = std::min(block, rows - r0);
        HIP_TRY(c, hipMemcpyAsync(stage.data(), src + (size_t)r0 * spitch, (size_t)(n - 1) * spitch + row_bytes,
                                  hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
        for (int j = 0; j < n; ++j)
            std::memcpy(dst + (size_t)(r0 + j) * dpitch, stage.data() + (size_t)j * spitch, row_bytes);
    }
    return FL_OK;
}

// Copy ny rows of `cols` elements with stride `stride` from host or device
// memory into a dense host vector.
fl_status fetch_rows(fl_ctx* c, const void* src, int64_t stride, int rows_, int cols, int on_device,
                     std::vector<unsigned char>& out) {
    const size_t es = esz(c);
    out.resize((size_t)rows_ * cols * es);
    if (on_device) {
        HIP_TRY(c, hipSetDevice(c->device));
        if (fl_status st = need_device(c, src, "input array")) return st;
        if (fl_status st = rows_to_host(c, out.data(), cols * es, static_cast<const unsigned char*>(src),
                                        (size_t)stride * es, cols * es, rows_, nullptr))
            return st;
    } else {
        for (int j = 0; j < rows_; ++j)
            std::memcpy(out.data() + (size_t)j * cols * es,
                        static_cast<const unsigned char*>(src) + (size_t)j * stride * es, cols * es);
    }
    return FL_OK;
}

void invalidate(fl_ctx* c) { c->committed = false; }

void free_adjoint(fl_ctx* c) {
    for (void* p : c->adj_allocs) (void)hipFree(p);
    c->adj_allocs.clear();
    c->d_gauges = c->d_gcell = nullptr;
    c->ngcell = 0;
    c->d_obs = c->d_series = c->d_ck = c->d_ck_qin = c->d_end = c->d_bwd = nullptr;
    c->d_ck_ctl = nullptr;
    c->adj_setup = false;
    c->adj_nsteps = 0;
}

void free_device(fl_ctx* c) {
    free_adjoint(c);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_k = 0;
    if (c->graph2_exec) (void)hipGraphExecDestroy(c->graph2_exec);
    if (c->graph2) (void)hipGraphDestroy(c->graph2);
    c->graph2_exec = nullptr;
    c->graph2 = nullptr;
    c->graph2_k = 0;
    for (auto& q : c->d_part2) q = nullptr;
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    c->dev_bytes = 0;
    c->ws_used = 0;
    c->d_h[0] = c->d_h[1] = c->d_qx[0] = c->d_qx[1] = c->d_qy[0] = c->d_qy[1] = nullptr;
    c->d_z = c->d_n = c->d_edge_w = c->d_edge_s = c->d_kout = nullptr;
    c->d_qin[0] = c->d_qin[1] = nullptr;
    c->d_in_z = c->d_in_k = c->d_ts = c->d_qs = nullptr;
    c->d_part[0] = c->d_part[1] = c->d_vol_part = c->d_vol = nullptr;
    c->d_ctl = nullptr;
    c->committed = false;
}

size_t ws_round(size_t bytes) { return (std::max<size_t>(bytes, 256) + 255) & ~size_t(255); }

fl_status dalloc(fl_ctx* c, void** p, size_t bytes) {
    bytes = ws_round(bytes);
    if (c->ws) {
        if (c->ws_used + bytes > c->ws_bytes) {
            *p = nullptr;
            return fail(c, FL_ENOMEM, "bound workspace too small");
        }
        *p = c->ws + c->ws_used;
        c->ws_used += bytes;
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            return fail(c, e == hipErrorOutOfMemory ? FL_ENOMEM : FL_EHIP,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        c->allocs.push_back(*p);
        c->dev_bytes += bytes;
    }
    return hipMemsetAsync(*p, 0, bytes, c->stream) == hipSuccess
               ? FL_OK
               : fail(c, FL_EHIP, "hipMemsetAsync failed");
}

int side_len(const fl_ctx* c, int side) { return (side == FL_WEST || side == FL_EAST) ? c->ny : c->nx; }

void side_cell(const fl_ctx* c, int side, int k, int* i, int* j) {
    switch (side) {
    case FL_WEST: *i = 0; *j = k; break;
    case FL_EAST: *i = c->nx - 1; *j = k; break;
    case FL_SOUTH: *i = k; *j = 0; break;
    default: *i = k; *j = c->ny - 1; break;
    }
}

struct Tiling {
    int cpt, rows, nstrips, nchunks, npart;
};

Tiling tiling_of(const fl_ctx* c, int cpt, int rows) {
    Tiling t{cpt, rows, 0, 0, 0};
    t.nstrips = (c->nx + strip_width(cpt) - 1) / strip_width(cpt);
    t.nchunks = (c->ny + rows - 1) / rows;
    if (c->out_count > 0)
        t.npart = (c->out_side == FL_WEST || c->out_side == FL_EAST) ? t.nchunks : t.nstrips;
    return t;
}

template <typename T>
StepArgs<T> make_args(const fl_ctx* c, long long n, const Tiling& tl, int freeze = 0);

template <typename T>
StepArgs<T> make_args(const fl_ctx* c, long long n) {
    Tiling tl{c->cpt, c->rows, c->nstrips, c->nchunks, c->npart};
    return make_args<T>(c, n, tl, 0);
}

template <typename T>
StepArgs<T> make_args(const fl_ctx* c, long long n, const Tiling& tl, int freeze) {
    StepArgs<T> a{};
    const int p = (int)(n & 1), q = p ^ 1;
    a.h_in = (const T*)c->d_h[p];
    a.qx_in = (const T*)c->d_qx[p];
    a.qy_in = (const T*)c->d_qy[p];
    a.h_out = (T*)c->d_h[q];
    a.qx_out = (T*)c->d_qx[q];
    a.qy_out = (T*)c->d_qy[q];
    a.z = (const T*)c->d_z;
    a.n = (const T*)c->d_n;
    a.edge_w = (T*)c->d_edge_w;
    a.edge_s = (T*)c->d_edge_s;
    a.kout = (const T*)c->d_kout;
    a.qin = (const T*)c->d_qin[p];
    a.qin_next = (T*)c->d_qin[q];
    a.in_z = c->d_in_z;
    a.in_k = c->d_in_k;
    a.ts = c->d_ts;
    a.qs = c->d_qs;
    a.part_cur = c->d_part[p];
    a.part_prev = c->d_part[q];
    a.ctl = c->d_ctl;
    a.pitch = c->pitch;
    a.nx = c->nx;
    a.ny = c->ny;
    a.in_side = c->in_count > 0 ? c->in_side : -1;
    a.in_first = c->in_first;
    a.in_count = c->in_count;
    a.nsamp = (int)c->ts.size();
    a.out_side = c->out_count > 0 ? c->out_side : -1;
    a.out_first = c->out_first;
    a.out_count = c->out_count;
    a.npart = tl.npart;
    a.positivity = c->params.positivity;
    a.freeze = freeze;
    a.nstrips = tl.nstrips;
    a.nchunks = tl.nchunks;
    a.rows = tl.rows;
    a.phase = (int)(n % 6);
    a.dx = c->dx;
    a.g = c->params.g;
    a.alpha = c->params.alpha;
    a.dt_max = c->params.dt_max;
    a.h_eps = c->params.h_eps;
    a.dt_fixed = c->params.dt_fixed;
    a.act = nullptr;
    a.act_stride = 0;
    a.variant = c->variant;
    return a;
}

// The flags and list of active-tile skipping, for a single-step launch.
template <typename T>
void set_act(const fl_ctx* c, StepArgs<T>& a) {
    if (!c->active) return;
    a.act = c->d_act;
    a.act_stride = c->act_stride;
    a.act_list = c->act_list_mode ? c->d_act_list : nullptr;
    a.act_count = c->d_act_count;
}

// One step of the context's own run: with active-tile skipping when it is on.
template <typename T>
hipError_t enqueue_one_t(fl_ctx* c, long long n, hipStream_t s) {
    StepArgs<T> a = make_args<T>(c, n);
    set_act<T>(c, a);
    return launch_step<T>(a, c->cpt, s);
}

hipError_t enqueue_one(fl_ctx* c, long long n, hipStream_t s) {
    return c->prec == FL_F64 ? enqueue_one_t<double>(c, n, s) : enqueue_one_t<float>(c, n, s);
}

// Work decomposition of the k-step kernel: strip 0 outputs columns
// [0, W + 2k - 2), strip s > 0 columns [s W + 2k - 2, (s + 1) W + 2k - 2),
// W = strip_width_fused(cpt, k).
Tiling tiling_fused_of(const fl_ctx* c, int cpt, int rows, int k) {
    Tiling t{cpt, rows, 0, 0, 0};
    const int w = strip_width_fused(cpt, k);
    t.nstrips = std::max(1, (c->nx - (2 * k - 2) + w - 1) / w);
    t.nchunks = (c->ny + rows - 1) / rows;
    if (c->out_count > 0)
        t.npart = (c->out_side == FL_WEST || c->out_side == FL_EAST) ? t.nchunks : t.nstrips;
    return t;
}

// Launch arguments of k steps per launch with the k-step tiling tl (no
// active tiles).
template <typename T>
FusedArgs<T> make_args_fused_tl(const fl_ctx* c, long long launch, int resolve, const Tiling& tl,
                                int k, int freeze) {
    FusedArgs<T> A{};
    A.a = make_args<T>(c, 0, tl, freeze);
    for (int p = 0; p < 2; ++p) {
        A.h[p] = (T*)c->d_h[p];
        A.qx[p] = (T*)c->d_qx[p];
        A.qy[p] = (T*)c->d_qy[p];
        for (int q = 0; q < kFuseMax; ++q) A.part[q][p] = c->d_part2[2 * q + p];
    }
    A.K = k;
    A.phase = (int)(launch % 6);
    A.resolve = resolve;
    return A;
}

// Launch arguments of the context's multi-step launches.
template <typename T>
FusedArgs<T> make_args_fused(const fl_ctx* c, long long launch, int resolve, int freeze = 0) {
    const Tiling tl{c->cpt2, c->rows2, c->nstrips2, c->nchunks2, c->npart2};
    FusedArgs<T> A = make_args_fused_tl<T>(c, launch, resolve, tl, c->fuse_k, freeze);
    if (c->active) {
        // active-tile skipping in the multi-step launches (flags by generation)
        A.a.act = c->d_act;
        A.a.act_stride = c->act_stride;
    }
    return A;
}

hipError_t enqueue_fused(fl_ctx* c, long long launch, int resolve, hipStream_t s, int freeze = 0) {
    if (c->prec == FL_F64)
        return launch_fused<double>(make_args_fused<double>(c, launch, resolve, freeze), c->cpt2, s);
    return launch_fused<float>(make_args_fused<float>(c, launch, resolve, freeze), c->cpt2, s);
}

// L multi-step launches with launch counters 0 .. L-1 (L a multiple of 6, so
// the graph can be replayed whenever the counter is a multiple of 6).
fl_status capture_graph2(fl_ctx* c) {
    int K = c->params.steps_per_graph > 0 ? c->params.steps_per_graph / c->fuse_k : 60 / c->fuse_k;
    K = std::max(6, ((K + 5) / 6) * 6);
    hipStream_t cs;
    HIP_TRY(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < K && e == hipSuccess; ++k) e = enqueue_fused(c, k, 0, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) {
            e = hipGraphInstantiate(&c->graph2_exec, g, nullptr, nullptr, 0);
            c->graph2 = g;
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(c, e, "graph capture (multi-step)");
    c->graph2_k = K;
    return FL_OK;
}

fl_status capture_graph(fl_ctx* c) {
    int K = c->params.steps_per_graph > 0 ? c->params.steps_per_graph : 60;
    K = ((K + 5) / 6) * 6;
    hipStream_t cs;
    HIP_TRY(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int k = 0; k < K && e == hipSuccess; ++k) e = enqueue_one(c, k, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) {
            e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
            c->graph = g;
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(c, e, "graph capture");
    c->graph_k = K;
    return FL_OK;
}

fl_status upload_field(fl_ctx* c, void* dst, const std::vector<unsigned char>& src, int rows_,
                       int cols, long long dst_row0, long long dst_col0) {
    const size_t es = esz(c);
    unsigned char* d = static_cast<unsigned char*>(dst) + ((dst_row0)*c->pitch + dst_col0) * es;
    HIP_TRY(c, hipMemcpy2DAsync(d, c->pitch * es, src.data(), cols * es, cols * es, rows_,
                                hipMemcpyHostToDevice, c->stream));
    return FL_OK;
}

template <typename T>
void fill_host(std::vector<unsigned char>& v, size_t count, const std::vector<double>& vals) {
    v.resize(count * sizeof(T));
    T* p = reinterpret_cast<T*>(v.data());
    for (size_t k = 0; k < count; ++k) p[k] = (T)vals[k];
}

// 32 rows per work item on large grids (measured best on MI355X at 16384^2);
// fewer on small grids so that there are at least ~6000 waves (two rounds of
// resident waves) to spread over the 256 CUs.
int default_rows(int nx, int ny, int cpt) {
    const long long strips = (nx + strip_width(cpt) - 1) / strip_width(cpt);
    const long long r = (long long)ny * strips / 6144;
    return (int)std::max<long long>(8, std::min<long long>(32, r));
}

// Rows per work item of the k-step kernel: like the single-step kernel, at
// least ~6000 waves on small grids; on large grids 32 rows at two steps per
// launch and 48 at three (the 4k + 2 extra rows an item loads weigh more;
// both measured best on MI355X at 16384^2).
int default_rows_fused(int nx, int ny, int cpt, int k) {
    const int w = strip_width_fused(cpt, k);
    const long long strips = std::max(1, (nx - (2 * k - 2) + w - 1) / w);
    const long long r = (long long)ny * strips / 6144;
    return (int)std::max<long long>(8, std::min<long long>(k >= 3 ? 48 : 32, r));
}

// Fold the last step's outflow partial sums into the clock (see k_fold).
fl_status fold_budget(fl_ctx* c, const Tiling& tl) {
    if (c->prec == FL_F64)
        HIP_TRY(c, launch_fold<double>(make_args<double>(c, c->nstep, tl, 0), c->stream));
    else
        HIP_TRY(c, launch_fold<float>(make_args<float>(c, c->nstep, tl, 0), c->stream));
    return FL_OK;
}

// Bytes fl_commit takes for a grid: the same buffers, in the same order and
// rounding, as do_commit allocates, with every size that depends on the
// boundary data at its largest (sections up to the longest side, hydrographs
// up to 4096 samples).
// Flag bytes per step slot of active-tile skipping: enough for the smallest
// work items of either kernel (one cell per lane, one row).
long long act_slot_bytes(int nx, int ny) {
    const int w = std::min(strip_width(1), strip_width_fused(1, 2));
    return (long long)((nx + w - 1) / w) * ny;
}

// Entries of the active-tile list: one per work item, then one count per
// block of 256 items of the selection kernels.
long long act_list_ints(int nx, int ny) {
    const long long items = act_slot_bytes(nx, ny);
    return items + (items + 255) / 256 + 1;
}

size_t workspace_bytes(int nx, int ny, fl_precision prec, bool two_step, bool active) {
    const size_t es = elem_size(prec);
    const long long align = 256 / (long long)es;
    const long long pitch = ((nx + 8 + align - 1) / align) * align;
    const size_t field = (size_t)pitch * (ny + 2 * kHalo) * es;
    const size_t side = (size_t)std::max(nx, ny);
    size_t b = 0;
    b += 2 * (3 * ws_round(field) + ws_round(side * es) + ws_round(sizeof(double) * side));
    b += 2 * ws_round(field);
    b += ws_round((size_t)ny * es) + ws_round((size_t)nx * es) + ws_round(side * es);
    b += 2 * ws_round(sizeof(double) * side);
    b += 2 * ws_round(sizeof(double) * 4096);
    b += ws_round(sizeof(double) * kVolumeParts) + ws_round(sizeof(double)) + ws_round(sizeof(DevCtl));
    if (two_step) b += 2 * kFuseMax * ws_round(sizeof(double) * side);
    if (active)
        b += ws_round((size_t)(3 * act_slot_bytes(nx, ny))) +
             ws_round(sizeof(int) * (size_t)act_list_ints(nx, ny)) + ws_round(18 * sizeof(unsigned));
    return b;
}

fl_status do_commit(fl_ctx* c) {
    if (!c->have_grid || !c->have_z || !c->have_n)
        return fail(c, FL_ESTATE, "fl_commit needs fl_init_grid, fl_set_dem and fl_set_manning");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_device(c);
    const size_t es = esz(c);
    const int nx = c->nx, ny = c->ny;
    if (c->variant && (c->fuse >= 2 || c->active))
        return fail(c, FL_EINVAL,
                    "fl_commit: method variants run one step per launch without active tiles");
    if (c->ws && c->ws_bytes < workspace_bytes(nx, ny, c->prec, c->fuse >= 2, c->active != 0))
        return fail(c, FL_EINVAL, "fl_commit: the bound workspace is smaller than fl_workspace_bytes");
    if (c->cpt == 0) c->cpt = (c->prec == FL_F64) ? 2 : 4;
    c->rows = c->rows_req ? c->rows_req : default_rows(nx, ny, c->cpt);
    const long long align = 256 / (long long)es;
    c->pitch = ((nx + 8 + align - 1) / align) * align;
    {
        const Tiling tl = tiling_of(c, c->cpt, c->rows);
        c->nstrips = tl.nstrips;
        c->nchunks = tl.nchunks;
        c->npart = tl.npart;
    }
    const size_t field = (size_t)c->pitch * (ny + 2 * kHalo) * es;
    fl_status st;
    for (int p = 0; p < 2; ++p) {
        if ((st = dalloc(c, &c->d_h[p], field))) return st;
        if ((st = dalloc(c, &c->d_qx[p], field))) return st;
        if ((st = dalloc(c, &c->d_qy[p], field))) return st;
        if ((st = dalloc(c, &c->d_qin[p], (size_t)std::max(nx, ny) * es))) return st;
        // sized for any work decomposition (a batch may use another tiling)
        if ((st = dalloc(c, (void**)&c->d_part[p], sizeof(double) * std::max(nx, ny))))
            return st;
    }
    if ((st = dalloc(c, &c->d_z, field))) return st;
    if ((st = dalloc(c, &c->d_n, field))) return st;
    if ((st = dalloc(c, &c->d_edge_w, (size_t)ny * es))) return st;
    if ((st = dalloc(c, &c->d_edge_s, (size_t)nx * es))) return st;
    if ((st = dalloc(c, &c->d_kout, (size_t)std::max(nx, ny) * es))) return st;
    if ((st = dalloc(c, (void**)&c->d_in_z, sizeof(double) * std::max(1, c->in_count)))) return st;
    if ((st = dalloc(c, (void**)&c->d_in_k, sizeof(double) * std::max(1, c->in_count)))) return st;
    if ((st = dalloc(c, (void**)&c->d_ts, sizeof(double) * std::max<size_t>(1, c->ts.size()))))
        return st;
    if ((st = dalloc(c, (void**)&c->d_qs, sizeof(double) * std::max<size_t>(1, c->qs.size()))))
        return st;
    if ((st = dalloc(c, (void**)&c->d_vol_part, sizeof(double) * kVolumeParts))) return st;
    if ((st = dalloc(c, (void**)&c->d_vol, sizeof(double)))) return st;
    if ((st = dalloc(c, (void**)&c->d_ctl, sizeof(DevCtl)))) return st;
    c->d_act = nullptr;
    c->d_act_list = nullptr;
    c->d_act_count = nullptr;
    c->act_stride = 0;
    c->act_at = -1;
    if (c->active) {
        c->act_stride = act_slot_bytes(nx, ny);
        if ((st = dalloc(c, (void**)&c->d_act, (size_t)(3 * c->act_stride)))) return st;
        if ((st = dalloc(c, (void**)&c->d_act_list, sizeof(int) * (size_t)act_list_ints(nx, ny)))) return st;
        if ((st = dalloc(c, (void**)&c->d_act_count, 18 * sizeof(unsigned)))) return st;
    }

    // Host sources of the asynchronous uploads below stay alive until the
    // stream is synchronized at the end of this function (a copy from pageable
    // memory may still read its source after the call returns).
    std::vector<unsigned char> east, west, north, kb;
    // cell fields
    if ((st = upload_field(c, c->d_z, c->z, ny, nx, kHalo, kHalo))) return st;
    if ((st = upload_field(c, c->d_n, c->n, ny, nx, kHalo, kHalo))) return st;
    if (c->have_state) {
        if ((st = upload_field(c, c->d_h[0], c->h0, ny, nx, kHalo, kHalo))) return st;
        // qx (ny x (nx+1)): column 0 is the west border, columns 1..nx the east faces.
        east.resize((size_t)ny * nx * es);
        west.resize((size_t)ny * es);
        for (int j = 0; j < ny; ++j) {
            std::memcpy(east.data() + (size_t)j * nx * es, c->qx0.data() + ((size_t)j * (nx + 1) + 1) * es,
                        nx * es);
            std::memcpy(west.data() + (size_t)j * es, c->qx0.data() + (size_t)j * (nx + 1) * es, es);
        }
        if ((st = upload_field(c, c->d_qx[0], east, ny, nx, kHalo, kHalo))) return st;
        HIP_TRY(c, hipMemcpyAsync(c->d_edge_w, west.data(), west.size(), hipMemcpyHostToDevice,
                                  c->stream));
        // qy ((ny+1) x nx): row 0 is the south border, rows 1..ny the north faces.
        north.assign(c->qy0.begin() + (size_t)nx * es, c->qy0.end());
        if ((st = upload_field(c, c->d_qy[0], north, ny, nx, kHalo, kHalo))) return st;
        HIP_TRY(c, hipMemcpyAsync(c->d_edge_s, c->qy0.data(), (size_t)nx * es, hipMemcpyHostToDevice,
                                  c->stream));
    }
    // boundary data
    if (c->out_count > 0) {
        std::vector<double> k(side_len(c, c->out_side), 0.0);
        for (int p = 0; p < c->out_count; ++p) {
            int i, j;
            side_cell(c, c->out_side, c->out_first + p, &i, &j);
            k[c->out_first + p] = std::sqrt(c->out_slope) / get_elem(c, c->n.data(), (size_t)j * nx + i);
        }
        if (c->prec == FL_F64) fill_host<double>(kb, k.size(), k); else fill_host<float>(kb, k.size(), k);
        HIP_TRY(c, hipMemcpyAsync(c->d_kout, kb.data(), kb.size(), hipMemcpyHostToDevice, c->stream));
    }
    std::vector<double> iz(std::max(1, c->in_count), 0.0), ik(std::max(1, c->in_count), 0.0);
    for (int p = 0; p < c->in_count; ++p) {
        int i, j;
        side_cell(c, c->in_side, c->in_first + p, &i, &j);
        iz[p] = get_elem(c, c->z.data(), (size_t)j * nx + i);
        ik[p] = std::sqrt(c->in_slope) / get_elem(c, c->n.data(), (size_t)j * nx + i);
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_in_z, iz.data(), iz.size() * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_in_k, ik.data(), ik.size() * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    if (!c->ts.empty()) {
        HIP_TRY(c, hipMemcpyAsync(c->d_ts, c->ts.data(), c->ts.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_qs, c->qs.data(), c->qs.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    }
    // clock
    DevCtl ctl{};
    ctl.clk[0].t = c->t0;
    ctl.t_end = c->params.t_end;
    HIP_TRY(c, hipMemcpyAsync(c->d_ctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, c->stream));
    c->nstep = 0;
    if (c->prec == FL_F64) {
        HIP_TRY(c, launch_hmax_init<double>((const double*)c->d_h[0], c->pitch, nx, ny, c->d_ctl, c->stream));
        HIP_TRY(c, launch_prime<double>(make_args<double>(c, 0), c->stream));
        HIP_TRY(c, launch_volume<double>((const double*)c->d_h[0], c->pitch, nx, ny, c->d_vol_part,
                                         kVolumeParts, c->d_vol, c->stream));
    } else {
        HIP_TRY(c, launch_hmax_init<float>((const float*)c->d_h[0], c->pitch, nx, ny, c->d_ctl, c->stream));
        HIP_TRY(c, launch_prime<float>(make_args<float>(c, 0), c->stream));
        HIP_TRY(c, launch_volume<float>((const float*)c->d_h[0], c->pitch, nx, ny, c->d_vol_part,
                                        kVolumeParts, c->d_vol, c->stream));
    }
    HIP_TRY(c, hipMemcpyAsync(&c->v0, c->d_vol, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->v0 *= c->dx * c->dx;
    if (c->active) {
        // size the active-tile step's persistent grids before any capture
        for (int cp : {1, 2, 4}) {
            if (c->prec == FL_F64 && cp == 4) continue;
            HIP_TRY(c, c->prec == FL_F64 ? prepare_step_list<double>(cp) : prepare_step_list<float>(cp));
        }
    }
    if ((st = capture_graph(c))) return st;
    c->fuse_k = c->fuse >= 2 ? c->fuse : 0;
    if (c->fuse_k) {
        c->cpt2 = c->cpt2_req ? c->cpt2_req : (c->prec == FL_F64 ? 1 : 2);
        if (c->cpt2 == 4 && c->fuse_k != 2)
            return fail(c, FL_EINVAL, "fl_commit: 4 cells per lane run two steps per launch at most");
        c->rows2 = c->rows2_req ? c->rows2_req : default_rows_fused(nx, ny, c->cpt2, c->fuse_k);
        if (c->active && c->rows2 < c->fuse_k)
            return fail(c, FL_EINVAL,
                        "fl_commit: active tiles with k steps per launch need items of >= k rows");
        const Tiling t2 = tiling_fused_of(c, c->cpt2, c->rows2, c->fuse_k);
        c->nstrips2 = t2.nstrips;
        c->nchunks2 = t2.nchunks;
        c->npart2 = t2.npart;
        for (auto& q : c->d_part2)
            if ((st = dalloc(c, (void**)&q, sizeof(double) * std::max(nx, ny)))) return st;
        if ((st = capture_graph2(c))) return st;
    }
    c->committed = true;
    return FL_OK;
}

// Do the flags describe the state for single-step work items of tiling (cpt, rows)?
bool act_flags_hold(const fl_ctx* c, int cpt, int rows) {
    return c->act_mode == 1 && c->act_at == c->nstep && c->act_cpt == cpt && c->act_rows == rows;
}

fl_status enqueue_steps(fl_ctx* c, long long nsteps) {
    if (c->active && nsteps > 0 && !act_flags_hold(c, c->cpt, c->rows)) {
        // flags stale: compute every item in the next two steps
        HIP_TRY(c, launch_fill_bytes(c->d_act, 3 * c->act_stride, 1, c->stream));
    }
    while (nsteps > 0) {
        if (c->graph_exec && c->nstep % 6 == 0 && nsteps >= c->graph_k) {
            HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
            c->nstep += c->graph_k;
            nsteps -= c->graph_k;
        } else {
            HIP_TRY(c, enqueue_one(c, c->nstep, c->stream));
            c->nstep += 1;
            nsteps -= 1;
        }
    }
    if (c->active) {
        c->act_mode = 1;
        c->act_at = c->nstep;
        c->act_cpt = c->cpt;
        c->act_rows = c->rows;
    }
    return FL_OK;
}

// nsteps steps by multi-step launches of k = fuse_k steps.  The single-step
// state (budget folded) becomes the multi-step clock; about nsteps/k launches
// follow, then one that only settles the last launch's speculated dts
// (redoing it if needed); the claimed count is read back, and further rounds
// run if redos or shorter launches left steps over.  Finally the state
// becomes the single-step state again, at a step counter whose parity names
// the buffer that holds it.
template <typename T>
fl_status fused_steps_t(fl_ctx* c, long long nsteps, int freeze = 0) {
    fl_status st;
    {
        const Tiling tl{c->cpt, c->rows, c->nstrips, c->nchunks, c->npart};
        if ((st = fold_budget(c, tl))) return st;
    }
    // the flags of the previous two-step run still hold if nothing else moved
    // the state since; otherwise compute every item in the first two launches
    const bool keep = c->active && c->act_mode == 2 && c->act_at == c->nstep;
    if (c->active && !keep) HIP_TRY(c, launch_fill_bytes(c->d_act, 3 * c->act_stride, 1, c->stream));
    HIP_TRY(c, launch_enter_fused<T>(make_args<T>(c, c->nstep), nsteps, keep ? 1 : 0, c->stream));
    long long lc = 0;
    long long want = (nsteps + c->fuse_k - 1) / c->fuse_k;
    FusedClock slot{};
    for (int round = 0;; ++round) {
        while (want > 0) {
            if (!freeze && c->graph2_exec && lc % 6 == 0 && want >= c->graph2_k) {
                HIP_TRY(c, hipGraphLaunch(c->graph2_exec, c->stream));
                lc += c->graph2_k;
                want -= c->graph2_k;
            } else {
                HIP_TRY(c, enqueue_fused(c, lc, 0, c->stream, freeze));
                lc += 1;
                want -= 1;
            }
        }
        HIP_TRY(c, enqueue_fused(c, lc, 1, c->stream, freeze));
        lc += 1;
        HIP_TRY(c, hipMemcpyAsync(&slot, &c->d_ctl->cf[lc & 1], sizeof(slot), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (slot.pending) return fail(c, FL_EHIP, "multi-step launches: unsettled state");
        if (slot.vsteps >= nsteps) break;
        if (round >= 64) return fail(c, FL_EHIP, "multi-step launches: no progress");
        want = nsteps - slot.vsteps;  // enough even if every launch makes one step
    }
    long long n2 = c->nstep + nsteps;
    n2 += (n2 ^ (long long)slot.cur) & 1;
    HIP_TRY(c, launch_leave_fused<T>(make_args<T>(c, n2), make_args_fused<T>(c, 0, 0), lc, c->stream));
    c->nstep = n2;
    if (c->active) {
        c->act_mode = 2;
        c->act_at = n2;
    }
    return FL_OK;
}

fl_status run_steps(fl_ctx* c, long long nsteps) {
    if (c->fuse >= 2 && c->fuse_k >= 2 && nsteps >= 2)
        return c->prec == FL_F64 ? fused_steps_t<double>(c, nsteps) : fused_steps_t<float>(c, nsteps);
    return enqueue_steps(c, nsteps);
}

struct HostReport {
    double r[8];
};

fl_status read_report(fl_ctx* c, fl_report* out, bool with_volume) {
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->prec == FL_F64) {
        HIP_TRY(c, launch_flush<double>(make_args<double>(c, c->nstep), c->stream));
        if (with_volume)
            HIP_TRY(c, launch_volume<double>((const double*)c->d_h[c->nstep & 1], c->pitch, c->nx, c->ny,
                                             c->d_vol_part, kVolumeParts, c->d_vol, c->stream));
    } else {
        HIP_TRY(c, launch_flush<float>(make_args<float>(c, c->nstep), c->stream));
        if (with_volume)
            HIP_TRY(c, launch_volume<float>((const float*)c->d_h[c->nstep & 1], c->pitch, c->nx, c->ny,
                                            c->d_vol_part, kVolumeParts, c->d_vol, c->stream));
    }
    HostReport hr{};
    double vol = 0.0;
    HIP_TRY(c, hipMemcpyAsync(hr.r, c->d_ctl->report, sizeof(hr.r), hipMemcpyDeviceToHost, c->stream));
    if (with_volume)
        HIP_TRY(c, hipMemcpyAsync(&vol, c->d_vol, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out->t = hr.r[0];
    out->last_dt = hr.r[1];
    out->steps = (int64_t)hr.r[2];
    out->v0 = c->v0;
    out->v_in = hr.r[3];
    out->v_out = hr.r[4];
    out->v_now = vol * c->dx * c->dx;
    out->done = hr.r[5] != 0.0;
    out->nonfinite = hr.r[6] != 0.0;
    return out->nonfinite ? fail(c, FL_ENONFINITE, "a depth became non-finite; the clock stopped")
                          : FL_OK;
}

bool check_side(int side) { return side >= FL_WEST && side <= FL_NORTH; }

}  // namespace

extern "C" {

void fl_default_params(fl_params* p) {
    if (!p) return;
    p->g = 9.81;
    p->alpha = 0.7;
    p->dt_max = 0.1;
    p->h_eps = 1e-4;
    p->dt_fixed = 0.0;
    p->t_end = std::numeric_limits<double>::infinity();
    p->steps_per_graph = 60;
    p->positivity = 1;
}

fl_status fl_create(fl_ctx** out, int device, void* hip_stream, fl_precision prec) {
    if (!out) {
        g_create_error = "fl_create: NULL output pointer";
        return FL_EINVAL;
    }
    *out = nullptr;
    if (prec != FL_F32 && prec != FL_F64) {
        g_create_error = "fl_create: precision must be FL_F32 or FL_F64";
        return FL_EINVAL;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
        return FL_EHIP;
    }
    if (device < 0 || device >= ndev) {
        g_create_error = "fl_create: no such device";
        return FL_EINVAL;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(e);
        return FL_EHIP;
    }
    e = scratch_setup(device);
    if (e != hipSuccess) {
        g_create_error = std::string("fl_create: device scratch address: ") + hipGetErrorString(e);
        return FL_EHIP;
    }
    fl_ctx* c = new (std::nothrow) fl_ctx();
    if (!c) {
        g_create_error = "fl_create: out of host memory";
        return FL_ENOMEM;
    }
    c->device = device;
    c->prec = prec;
    fl_default_params(&c->params);
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
            delete c;
            return FL_EHIP;
        }
        c->own_stream = true;
    }
    *out = c;
    return FL_OK;
}

fl_status fl_init_grid(fl_ctx* c, int32_t nx, int32_t ny, double dx) {
    if (!c) return FL_EINVAL;
    if (nx < 1 || ny < 1) return fail(c, FL_EINVAL, "fl_init_grid: nx and ny must be >= 1");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(c, FL_EINVAL, "fl_init_grid: dx must be finite and > 0");
    // a row's byte offsets must fit 31 bits (the kernels address a row's
    // cells by 32-bit offsets from the row start)
    if ((long long)nx + 8 + 256 > (1LL << 28) || (long long)ny + 8 > (1LL << 30))
        return fail(c, FL_EINVAL, "fl_init_grid: grid too large");
    invalidate(c);
    c->nx = nx;
    c->ny = ny;
    c->dx = dx;
    c->have_grid = true;
    c->have_z = c->have_n = c->have_state = false;
    c->in_count = c->out_count = 0;
    c->in_side = c->out_side = -1;
    c->ts.clear();
    c->qs.clear();
    c->t0 = 0.0;
    c->ws = nullptr;
    c->ws_bytes = 0;
    return FL_OK;
}

size_t fl_workspace_bytes(int32_t nx, int32_t ny, fl_precision prec, uint32_t flags) {
    if (nx < 1 || ny < 1 || (prec != FL_F32 && prec != FL_F64) || (flags & ~3u)) return 0;
    if ((long long)nx + 8 + 256 > (1LL << 28) || (long long)ny + 8 > (1LL << 30)) return 0;
    return workspace_bytes(nx, ny, prec, (flags & 1u) != 0, (flags & 2u) != 0);
}

fl_status fl_bind_workspace(fl_ctx* c, void* dev_ptr, size_t bytes) {
    if (!c) return FL_EINVAL;
    if (!c->have_grid) return fail(c, FL_ESTATE, "fl_bind_workspace before fl_init_grid");
    if (dev_ptr) {
        if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0)
            return fail(c, FL_EINVAL, "fl_bind_workspace: pointer not 256-byte aligned");
        if (bytes < workspace_bytes(c->nx, c->ny, c->prec, false, false))
            return fail(c, FL_EINVAL, "fl_bind_workspace: smaller than fl_workspace_bytes");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    if (dev_ptr)
        if (fl_status st = need_device(c, dev_ptr, "fl_bind_workspace")) return st;
    if (c->stream) HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_device(c);
    c->ws = static_cast<unsigned char*>(dev_ptr);
    c->ws_bytes = dev_ptr ? bytes : 0;
    return FL_OK;
}

fl_status fl_set_dem(fl_ctx* c, const void* z, int64_t row_stride, int on_device) {
    if (!c) return FL_EINVAL;
    if (!c->have_grid) return fail(c, FL_ESTATE, "fl_set_dem before fl_init_grid");
    if (!z || row_stride < c->nx) return fail(c, FL_EINVAL, "fl_set_dem: NULL or row_stride < nx");
    std::vector<unsigned char> tmp;
    fl_status st = fetch_rows(c, z, row_stride, c->ny, c->nx, on_device, tmp);
    if (st) return st;
    const size_t cnt = (size_t)c->nx * c->ny;
    for (size_t k = 0; k < cnt; ++k)
        if (!std::isfinite(get_elem(c, tmp.data(), k)))
            return fail(c, FL_EINVAL, "fl_set_dem: non-finite elevation");
    c->z.swap(tmp);
    c->have_z = true;
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_manning(fl_ctx* c, const void* n, int64_t row_stride, int on_device) {
    if (!c) return FL_EINVAL;
    if (!c->have_grid) return fail(c, FL_ESTATE, "fl_set_manning before fl_init_grid");
    if (!n || row_stride < c->nx) return fail(c, FL_EINVAL, "fl_set_manning: NULL or row_stride < nx");
    std::vector<unsigned char> tmp;
    fl_status st = fetch_rows(c, n, row_stride, c->ny, c->nx, on_device, tmp);
    if (st) return st;
    const size_t cnt = (size_t)c->nx * c->ny;
    for (size_t k = 0; k < cnt; ++k) {
        double v = get_elem(c, tmp.data(), k);
        if (!(v > 0.0) || !std::isfinite(v))
            return fail(c, FL_EINVAL, "fl_set_manning: Manning n must be finite and > 0");
    }
    c->n.swap(tmp);
    c->have_n = true;
    invalidate(c);
    return FL_OK;
}

static bool overlaps(int s1, int f1, int c1, int s2, int f2, int c2) {
    if (c1 <= 0 || c2 <= 0 || s1 != s2) return false;
    return f1 < f2 + c2 && f2 < f1 + c1;
}

fl_status fl_set_inflow(fl_ctx* c, fl_side side, int32_t first, int32_t count, double slope,
                        const double* t_s, const double* q_m3s, int32_t nsamples) {
    if (!c) return FL_EINVAL;
    if (!c->have_grid) return fail(c, FL_ESTATE, "fl_set_inflow before fl_init_grid");
    if (count == 0) {
        c->in_count = 0;
        c->in_side = -1;
        c->ts.clear();
        c->qs.clear();
        invalidate(c);
        return FL_OK;
    }
    if (!check_side(side)) return fail(c, FL_EINVAL, "fl_set_inflow: bad side");
    if (count < 0 || first < 0 || first + (long long)count > side_len(c, side))
        return fail(c, FL_EINVAL, "fl_set_inflow: section outside the side");
    if (!(slope > 0.0) || !std::isfinite(slope)) return fail(c, FL_EINVAL, "fl_set_inflow: slope must be > 0");
    if (!t_s || !q_m3s || nsamples < 1 || nsamples > 4096)
        return fail(c, FL_EINVAL, "fl_set_inflow: need 1..4096 hydrograph samples");
    for (int k = 0; k < nsamples; ++k) {
        if (!std::isfinite(t_s[k]) || !std::isfinite(q_m3s[k]) || q_m3s[k] < 0.0)
            return fail(c, FL_EINVAL, "fl_set_inflow: samples must be finite with Q >= 0");
        if (k > 0 && !(t_s[k] > t_s[k - 1]))
            return fail(c, FL_EINVAL, "fl_set_inflow: sample times must increase strictly");
    }
    if (overlaps(side, first, count, c->out_side, c->out_first, c->out_count))
        return fail(c, FL_EINVAL, "fl_set_inflow: overlaps the outflow section");
    c->in_side = side;
    c->in_first = first;
    c->in_count = count;
    c->in_slope = slope;
    c->ts.assign(t_s, t_s + nsamples);
    c->qs.assign(q_m3s, q_m3s + nsamples);
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_outflow(fl_ctx* c, fl_side side, int32_t first, int32_t count, double slope) {
    if (!c) return FL_EINVAL;
    if (!c->have_grid) return fail(c, FL_ESTATE, "fl_set_outflow before fl_init_grid");
    if (count == 0) {
        c->out_count = 0;
        c->out_side = -1;
        invalidate(c);
        return FL_OK;
    }
    if (!check_side(side)) return fail(c, FL_EINVAL, "fl_set_outflow: bad side");
    if (count < 0 || first < 0 || first + (long long)count > side_len(c, side))
        return fail(c, FL_EINVAL, "fl_set_outflow: section outside the side");
    if (!(slope > 0.0) || !std::isfinite(slope)) return fail(c, FL_EINVAL, "fl_set_outflow: slope must be > 0");
    if (overlaps(side, first, count, c->in_side, c->in_first, c->in_count))
        return fail(c, FL_EINVAL, "fl_set_outflow: overlaps the inflow section");
    c->out_side = side;
    c->out_first = first;
    c->out_count = count;
    c->out_slope = slope;
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_params(fl_ctx* c, const fl_params* p) {
    if (!c) return FL_EINVAL;
    if (!p) return fail(c, FL_EINVAL, "fl_set_params: NULL");
    if (!(p->g > 0.0) || !std::isfinite(p->g)) return fail(c, FL_EINVAL, "fl_set_params: g must be > 0");
    if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return fail(c, FL_EINVAL, "fl_set_params: alpha must be in (0, 1]");
    if (!(p->dt_max > 0.0) || !std::isfinite(p->dt_max)) return fail(c, FL_EINVAL, "fl_set_params: dt_max must be > 0");
    if (!(p->h_eps >= 0.0) || !std::isfinite(p->h_eps)) return fail(c, FL_EINVAL, "fl_set_params: h_eps must be >= 0");
    if (!(p->dt_fixed >= 0.0) || !std::isfinite(p->dt_fixed)) return fail(c, FL_EINVAL, "fl_set_params: dt_fixed must be >= 0");
    if (std::isnan(p->t_end)) return fail(c, FL_EINVAL, "fl_set_params: t_end is NaN");
    if (p->steps_per_graph < 0) return fail(c, FL_EINVAL, "fl_set_params: steps_per_graph < 0");
    if (p->positivity != 0 && p->positivity != 1) return fail(c, FL_EINVAL, "fl_set_params: positivity must be 0 or 1");
    c->params = *p;
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_state(fl_ctx* c, const void* h, const void* qx, const void* qy, double t,
                       int on_device) {
    if (!c) return FL_EINVAL;
    if (!c->have_grid) return fail(c, FL_ESTATE, "fl_set_state before fl_init_grid");
    if (!h) return fail(c, FL_EINVAL, "fl_set_state: NULL depth");
    if (!std::isfinite(t)) return fail(c, FL_EINVAL, "fl_set_state: t must be finite");
    const int nx = c->nx, ny = c->ny;
    const size_t es = esz(c);
    std::vector<unsigned char> hh, qxx, qyy;
    fl_status st = fetch_rows(c, h, nx, ny, nx, on_device, hh);
    if (st) return st;
    for (size_t k = 0; k < (size_t)nx * ny; ++k) {
        double v = get_elem(c, hh.data(), k);
        if (!(v >= 0.0) || !std::isfinite(v)) return fail(c, FL_EINVAL, "fl_set_state: depth must be finite and >= 0");
    }
    if (qx) {
        if ((st = fetch_rows(c, qx, nx + 1, ny, nx + 1, on_device, qxx))) return st;
    } else {
        qxx.assign((size_t)ny * (nx + 1) * es, 0);
    }
    if (qy) {
        if ((st = fetch_rows(c, qy, nx, ny + 1, nx, on_device, qyy))) return st;
    } else {
        qyy.assign((size_t)(ny + 1) * nx * es, 0);
    }
    for (size_t k = 0; k < qxx.size() / es; ++k)
        if (!std::isfinite(get_elem(c, qxx.data(), k))) return fail(c, FL_EINVAL, "fl_set_state: non-finite qx");
    for (size_t k = 0; k < qyy.size() / es; ++k)
        if (!std::isfinite(get_elem(c, qyy.data(), k))) return fail(c, FL_EINVAL, "fl_set_state: non-finite qy");
    c->h0.swap(hh);
    c->qx0.swap(qxx);
    c->qy0.swap(qyy);
    c->t0 = t;
    c->have_state = true;
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_tiling(fl_ctx* c, int32_t cells_per_lane, int32_t rows_per_item) {
    if (!c) return FL_EINVAL;
    if (cells_per_lane != 0 && cells_per_lane != 1 && cells_per_lane != 2 && cells_per_lane != 4)
        return fail(c, FL_EINVAL, "fl_set_tiling: cells_per_lane must be 1, 2 or 4");
    if (c->prec == FL_F64 && cells_per_lane == 4)
        return fail(c, FL_EINVAL, "fl_set_tiling: FP64 supports 1 or 2 cells per lane");
    if (rows_per_item < 0) return fail(c, FL_EINVAL, "fl_set_tiling: rows_per_item < 0");
    if (cells_per_lane) c->cpt = cells_per_lane;
    if (rows_per_item) c->rows_req = rows_per_item;
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_fusion(fl_ctx* c, int32_t steps_per_launch, int32_t cells_per_lane,
                        int32_t rows_per_item) {
    if (!c) return FL_EINVAL;
    if (steps_per_launch < 1 || steps_per_launch > kFuseMax)
        return fail(c, FL_EINVAL, "fl_set_fusion: steps_per_launch must be 1, 2 or 3");
    if (cells_per_lane != 0 && cells_per_lane != 1 && cells_per_lane != 2 && cells_per_lane != 4)
        return fail(c, FL_EINVAL, "fl_set_fusion: cells_per_lane must be 1, 2 or 4");
    if (c->prec == FL_F64 && cells_per_lane == 4)
        return fail(c, FL_EINVAL, "fl_set_fusion: FP64 supports 1 or 2 cells per lane");
    if (rows_per_item < 0) return fail(c, FL_EINVAL, "fl_set_fusion: rows_per_item < 0");
    c->fuse = steps_per_launch;
    c->cpt2_req = cells_per_lane;
    c->rows2_req = rows_per_item;
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_variant(fl_ctx* c, int32_t friction, int32_t boundary) {
    if (!c) return FL_EINVAL;
    if ((friction != FL_FRICTION_FACE && friction != FL_FRICTION_VECTOR) ||
        (boundary != FL_BOUNDARY_SECTION && boundary != FL_BOUNDARY_CELL_AREA))
        return fail(c, FL_EINVAL, "fl_set_variant: unknown friction or boundary form");
    c->variant = (friction == FL_FRICTION_VECTOR ? VAR_FRICTION_VECTOR : 0) |
                 (boundary == FL_BOUNDARY_CELL_AREA ? VAR_BOUNDARY_CELL_AREA : 0);
    invalidate(c);
    return FL_OK;
}

fl_status fl_set_active_tiles(fl_ctx* c, int32_t on) {
    if (!c) return FL_EINVAL;
    if (on < 0 || on > 2) return fail(c, FL_EINVAL, "fl_set_active_tiles: on must be 0, 1 or 2");
    c->active = on != 0;
    c->act_list_mode = on == 2 ? 1 : 0;
    invalidate(c);
    return FL_OK;
}

fl_status fl_active_items(fl_ctx* c, int64_t* next_items, int64_t* total_items) {
    if (!c || !next_items || !total_items) return FL_EINVAL;
    if (!c->committed || !c->active)
        return fail(c, FL_ESTATE, "fl_active_items needs a context committed with active tiles on");
    HIP_TRY(c, hipSetDevice(c->device));
    if (c->fuse >= 2 && c->fuse_k >= 2 && c->act_mode == 2 && c->act_at == c->nstep) {
        // the next multi-step launch: the rule of the multi-step kernel's skip test
        const int ns = c->nstrips2, nc = c->nchunks2;
        const long long items = (long long)ns * nc;
        *total_items = items;
        long long gen = 0;
        std::vector<unsigned char> f1((size_t)items), f2((size_t)items);
        HIP_TRY(c, hipMemcpyAsync(&gen, &c->d_ctl->genf, sizeof(gen), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const long long g = gen + 1;
        HIP_TRY(c, hipMemcpyAsync(f1.data(), c->d_act + ((g + 2) % 3) * c->act_stride, (size_t)items,
                                  hipMemcpyDeviceToHost, c->stream));  // generation g - 1
        HIP_TRY(c, hipMemcpyAsync(f2.data(), c->d_act + ((g + 1) % 3) * c->act_stride, (size_t)items,
                                  hipMemcpyDeviceToHost, c->stream));  // generation g - 2
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const int K = c->fuse_k, r = 2 * K;
        const int wl = 64 * c->cpt2, wo = strip_width_fused(c->cpt2, K);
        const int f0 = c->in_first, fe = c->in_first + c->in_count;
        long long need = 0;
        for (int cc = 0; cc < nc; ++cc)
            for (int ss = 0; ss < ns; ++ss) {
                const int j0 = cc * c->rows2, j1 = std::min(j0 + c->rows2, c->ny);
                const int c0 = ss * wo - kHalo;
                bool in = false;
                if (c->in_count > 0) {
                    switch (c->in_side) {
                    case FL_WEST: in = ss == 0 && j0 - r < fe && j1 + r > f0; break;
                    case FL_EAST:
                        in = c->nx - 1 >= c0 && c->nx - 1 < c0 + wl && j0 - r < fe && j1 + r > f0;
                        break;
                    case FL_SOUTH: in = j0 <= r && c0 < fe && c0 + wl > f0; break;
                    default: in = j1 + r - 1 >= c->ny && c0 < fe && c0 + wl > f0; break;
                    }
                }
                bool act = in || f2[(size_t)cc * ns + ss];
                for (int dc = -1; dc <= 1 && !act; ++dc)
                    for (int ds = -1; ds <= 1 && !act; ++ds) {
                        const int s2 = ss + ds, c2 = cc + dc;
                        if (s2 >= 0 && s2 < ns && c2 >= 0 && c2 < nc) act = f1[(size_t)c2 * ns + s2] != 0;
                    }
                need += act ? 1 : 0;
            }
        *next_items = need;
        return FL_OK;
    }
    const int ns = c->nstrips, nc = c->nchunks;
    const long long items = (long long)ns * nc;
    *total_items = items;
    if (!act_flags_hold(c, c->cpt, c->rows)) {  // stale flags: the next step computes everything
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        *next_items = items;
        return FL_OK;
    }
    // the rule of the step kernel's skip test, for the step with counter n
    const long long n = c->nstep;
    std::vector<unsigned char> f1((size_t)items), f2((size_t)items);
    HIP_TRY(c, hipMemcpyAsync(f1.data(), c->d_act + ((n + 2) % 3) * c->act_stride, (size_t)items,
                              hipMemcpyDeviceToHost, c->stream));  // step n-1
    HIP_TRY(c, hipMemcpyAsync(f2.data(), c->d_act + ((n + 1) % 3) * c->act_stride, (size_t)items,
                              hipMemcpyDeviceToHost, c->stream));  // step n-2
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int wo = strip_width(c->cpt);
    const int f0 = c->in_first, fe = c->in_first + c->in_count;
    long long need = 0;
    for (int cc = 0; cc < nc; ++cc)
        for (int ss = 0; ss < ns; ++ss) {
            const int i0 = ss * wo, i1 = std::min(i0 + wo, c->nx);
            const int j0 = cc * c->rows, j1 = std::min(j0 + c->rows, c->ny);
            bool in = false;
            if (c->in_count > 0) {
                switch (c->in_side) {
                case FL_WEST: in = i0 == 0 && j0 < fe && f0 < j1; break;
                case FL_EAST: in = i0 <= c->nx - 1 && c->nx - 1 < i1 && j0 < fe && f0 < j1; break;
                case FL_SOUTH: in = j0 == 0 && i0 < fe && f0 < i1; break;
                default: in = j1 == c->ny && i0 < fe && f0 < i1; break;
                }
            }
            const long long k = (long long)cc * ns + ss;
            bool act = in || f1[k] || f2[k];
            if (ss > 0) act = act || f1[k - 1];
            if (ss + 1 < ns) act = act || f1[k + 1];
            if (cc > 0) act = act || f1[k - ns];
            if (cc + 1 < nc) act = act || f1[k + ns];
            need += act ? 1 : 0;
        }
    *next_items = need;
    return FL_OK;
}

fl_status fl_autotune(fl_ctx* c, const int32_t* candidates, int32_t ncand, int32_t trial_steps,
                      int32_t* best, double* best_ms) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_autotune before fl_commit");
    if (!candidates || ncand < 1 || trial_steps < 1) return fail(c, FL_EINVAL, "fl_autotune: no candidates");
    for (int k = 0; k < ncand; ++k) {
        const int cp = candidates[2 * k], rw = candidates[2 * k + 1];
        if ((cp != 1 && cp != 2 && cp != 4) || (c->prec == FL_F64 && cp == 4) || rw < 1)
            return fail(c, FL_EINVAL, "fl_autotune: bad candidate");
    }
    HIP_TRY(c, hipSetDevice(c->device));
    fl_status st;
    Tiling cur{c->cpt, c->rows, c->nstrips, c->nchunks, c->npart};
    if ((st = fold_budget(c, cur))) return st;
    Event e0, e1;
    HIP_TRY(c, hipEventCreate(&e0.e));
    HIP_TRY(c, hipEventCreate(&e1.e));
    double bt = 1e300;
    int bk = 0, bmode = c->act_list_mode;
    const int list_mode0 = c->act_list_mode;
    // under active tiles each tiling is timed with and without the selected list
    for (int kk = 0; kk < ncand * (c->active ? 2 : 1); ++kk) {
        const int k = c->active ? kk / 2 : kk;
        if (c->active) c->act_list_mode = kk % 2;
        const Tiling t = tiling_of(c, candidates[2 * k], candidates[2 * k + 1]);
        float ms = 0.f;
        // frozen steps (dt = 0): the state is streamed like a real step but
        // unchanged.  With active tiles they skip as real steps would: the
        // first two (untimed) compute every item and leave the flags of this
        // tiling, which mark the items that hold water or discharge.
        if (c->active) HIP_TRY(c, launch_fill_bytes(c->d_act, 3 * c->act_stride, 1, c->stream));
        for (int r = 0; r < 2 + trial_steps; ++r) {
            if (r == 2) HIP_TRY(c, hipEventRecord(e0.e, c->stream));
            hipError_t e;
            if (c->prec == FL_F64) {
                StepArgs<double> a = make_args<double>(c, c->nstep, t, 1);
                set_act<double>(c, a);
                e = launch_step<double>(a, t.cpt, c->stream);
            } else {
                StepArgs<float> a = make_args<float>(c, c->nstep, t, 1);
                set_act<float>(c, a);
                e = launch_step<float>(a, t.cpt, c->stream);
            }
            if (e != hipSuccess) return hip_fail(c, e, "fl_autotune trial");
            c->nstep += 1;
        }
        HIP_TRY(c, hipEventRecord(e1.e, c->stream));
        HIP_TRY(c, hipEventSynchronize(e1.e));
        HIP_TRY(c, hipEventElapsedTime(&ms, e0.e, e1.e));
        if ((st = fold_budget(c, t))) return st;
        if (ms < bt) {
            bt = ms;
            bk = k;
            bmode = c->act_list_mode;
        }
    }
    c->act_list_mode = c->active ? bmode : list_mode0;
    c->cpt = candidates[2 * bk];
    c->rows = c->rows_req = candidates[2 * bk + 1];
    const Tiling t = tiling_of(c, c->cpt, c->rows);
    c->nstrips = t.nstrips;
    c->nchunks = t.nchunks;
    c->npart = t.npart;
    // the captured multi-step graph holds the old decomposition
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    if ((st = capture_graph(c))) return st;
    c->act_at = -1;  // the flags describe the last candidate's items
    if (best) {
        best[0] = c->cpt;
        best[1] = c->rows;
    }
    if (best_ms) *best_ms = bt / trial_steps;
    return FL_OK;
}

fl_status fl_commit(fl_ctx* c) {
    if (!c) return FL_EINVAL;
    fl_status st = do_commit(c);
    if (st) free_device(c);
    return st;
}

fl_status fl_step(fl_ctx* c, int64_t nsteps) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_step before fl_commit");
    if (nsteps < 0) return fail(c, FL_EINVAL, "fl_step: nsteps < 0");
    HIP_TRY(c, hipSetDevice(c->device));
    return run_steps(c, nsteps);
}

fl_status fl_time_steps(fl_ctx* c, int64_t nsteps, double* elapsed_ms) {
    if (!c || !elapsed_ms) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_time_steps before fl_commit");
    HIP_TRY(c, hipSetDevice(c->device));
    Event e0, e1;
    HIP_TRY(c, hipEventCreate(&e0.e));
    HIP_TRY(c, hipEventCreate(&e1.e));
    HIP_TRY(c, hipEventRecord(e0.e, c->stream));
    fl_status st = run_steps(c, nsteps);
    HIP_TRY(c, hipEventRecord(e1.e, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1.e));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, e0.e, e1.e));
    *elapsed_ms = ms;
    return st;
}

fl_status fl_advance(fl_ctx* c, double seconds) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_advance before fl_commit");
    if (!(seconds >= 0.0) || !std::isfinite(seconds)) return fail(c, FL_EINVAL, "fl_advance: seconds must be finite and >= 0");
    fl_report r{};
    fl_status st = read_report(c, &r, false);
    if (st) return st;
    const double target = std::min(c->params.t_end, r.t + seconds);
    HIP_TRY(c, hipMemcpyAsync(&c->d_ctl->t_end, &target, sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    double t = r.t;
    double dt_guess = r.last_dt > 0.0 ? r.last_dt : c->params.dt_max;
    if (c->params.dt_fixed > 0.0) dt_guess = c->params.dt_fixed;
    while (t < target) {
        // Steps past the target are no-ops that still stream the state, so
        // launch no more than the remaining time needs at the last dt.
        long long want = (long long)std::ceil((target - t) / std::max(dt_guess, 1e-9));
        want = std::max<long long>(1, std::min<long long>(want, 20000));
        if ((st = enqueue_steps(c, want))) break;
        if ((st = read_report(c, &r, false))) break;
        if (r.steps == 0 && r.t <= t) break;
        t = r.t;
        if (r.done) break;
        dt_guess = r.last_dt > 0.0 ? r.last_dt : dt_guess;
    }
    const double tend = c->params.t_end;
    hipError_t e = hipMemcpyAsync(&c->d_ctl->t_end, &tend, sizeof(double), hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(c, e, "restore t_end");
    return FL_OK;
}

fl_status fl_get_depth(fl_ctx* c, void* dst, int64_t row_stride, int on_device) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_get_depth before fl_commit");
    if (!dst || row_stride < c->nx) return fail(c, FL_EINVAL, "fl_get_depth: NULL or row_stride < nx");
    HIP_TRY(c, hipSetDevice(c->device));
    if (on_device)
        if (fl_status st = need_device(c, dst, "fl_get_depth")) return st;
    const size_t es = esz(c);
    const unsigned char* src = static_cast<const unsigned char*>(c->d_h[c->nstep & 1]) +
                               ((size_t)kHalo * c->pitch + kHalo) * es;
    if (!on_device)
        return rows_to_host(c, static_cast<unsigned char*>(dst), row_stride * es, src, c->pitch * es,
                            c->nx * es, c->ny, c->stream);
    HIP_TRY(c, hipMemcpy2DAsync(dst, row_stride * es, src, c->pitch * es, c->nx * es, c->ny,
                                hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FL_OK;
}

fl_status fl_get_discharge(fl_ctx* c, void* qx, void* qy, int on_device) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_get_discharge before fl_commit");
    if (!qx || !qy) return fail(c, FL_EINVAL, "fl_get_discharge: NULL output");
    HIP_TRY(c, hipSetDevice(c->device));
    if (on_device) {
        if (fl_status st = need_device(c, qx, "fl_get_discharge qx")) return st;
        if (fl_status st = need_device(c, qy, "fl_get_discharge qy")) return st;
    }
    const size_t es = esz(c);
    const int nx = c->nx, ny = c->ny;
    const int p = c->nstep & 1;
    const size_t off = ((size_t)kHalo * c->pitch + kHalo) * es;
    unsigned char* dqx = static_cast<unsigned char*>(qx);
    unsigned char* dqy = static_cast<unsigned char*>(qy);
    if (!on_device) {
        fl_status st;
        if ((st = rows_to_host(c, dqx + es, (nx + 1) * es, static_cast<unsigned char*>(c->d_qx[p]) + off,
                               c->pitch * es, nx * es, ny, c->stream)) ||
            (st = rows_to_host(c, dqx, (nx + 1) * es, static_cast<unsigned char*>(c->d_edge_w), es, es, ny,
                               c->stream)) ||
            (st = rows_to_host(c, dqy, nx * es, static_cast<unsigned char*>(c->d_edge_s), nx * es, nx * es, 1,
                               c->stream)) ||
            (st = rows_to_host(c, dqy + nx * es, nx * es, static_cast<unsigned char*>(c->d_qy[p]) + off,
                               c->pitch * es, nx * es, ny, c->stream)))
            return st;
        return FL_OK;
    }
    const hipMemcpyKind kind = hipMemcpyDeviceToDevice;
    HIP_TRY(c, hipMemcpy2DAsync(dqx + es, (nx + 1) * es, static_cast<unsigned char*>(c->d_qx[p]) + off,
                                c->pitch * es, nx * es, ny, kind, c->stream));
    HIP_TRY(c, hipMemcpy2DAsync(dqx, (nx + 1) * es, c->d_edge_w, es, es, ny, kind, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dqy, c->d_edge_s, nx * es, kind, c->stream));
    HIP_TRY(c, hipMemcpy2DAsync(dqy + nx * es, nx * es, static_cast<unsigned char*>(c->d_qy[p]) + off,
                                c->pitch * es, nx * es, ny, kind, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FL_OK;
}

fl_status fl_get_report(fl_ctx* c, fl_report* r) {
    if (!c || !r) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_get_report before fl_commit");
    return read_report(c, r, true);
}

fl_status fl_get_state(fl_ctx* c, void* h, void* qx, void* qy, double* t, int on_device) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_get_state before fl_commit");
    if ((qx == nullptr) != (qy == nullptr))
        return fail(c, FL_EINVAL, "fl_get_state: give both qx and qy, or neither");
    fl_status st;
    if (h && (st = fl_get_depth(c, h, c->nx, on_device))) return st;
    if (qx && (st = fl_get_discharge(c, qx, qy, on_device))) return st;
    fl_report r{};
    st = read_report(c, &r, false);
    if (t) *t = r.t;
    return st;
}

fl_status fl_autotune_fusion(fl_ctx* c, int32_t trial_steps, int32_t* steps_per_launch,
                             double* ms_per_step) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_autotune_fusion before fl_commit");
    if (!c->d_part2[0] || !c->graph2_exec)
        return fail(c, FL_ESTATE,
                    "fl_autotune_fusion: commit with fl_set_fusion(ctx, 2 or 3, ...) first");
    if (trial_steps < 2) return fail(c, FL_EINVAL, "fl_autotune_fusion: trial_steps < 2");
    HIP_TRY(c, hipSetDevice(c->device));
    fl_status st;
    const Tiling tl{c->cpt, c->rows, c->nstrips, c->nchunks, c->npart};
    if ((st = fold_budget(c, tl))) return st;
    Event e0, e1;
    HIP_TRY(c, hipEventCreate(&e0.e));
    HIP_TRY(c, hipEventCreate(&e1.e));
    float ms1 = 0.f, ms2 = 0.f;
    // one step per launch: frozen steps (dt = 0 streams the state, leaves it
    // as it is).  With active tiles they skip as real steps would, after two
    // untimed steps that compute every item and set the flags.
    if (c->active) HIP_TRY(c, launch_fill_bytes(c->d_act, 3 * c->act_stride, 1, c->stream));
    const int warm = c->active ? 2 : 0;
    for (int r = 0; r < warm + trial_steps; ++r) {
        if (r == warm) HIP_TRY(c, hipEventRecord(e0.e, c->stream));
        hipError_t e;
        if (c->prec == FL_F64) {
            StepArgs<double> a = make_args<double>(c, c->nstep, tl, 1);
            set_act<double>(c, a);
            e = launch_step<double>(a, tl.cpt, c->stream);
        } else {
            StepArgs<float> a = make_args<float>(c, c->nstep, tl, 1);
            set_act<float>(c, a);
            e = launch_step<float>(a, tl.cpt, c->stream);
        }
        if (e != hipSuccess) return hip_fail(c, e, "fl_autotune_fusion trial");
        c->nstep += 1;
    }
    HIP_TRY(c, hipEventRecord(e1.e, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1.e));
    HIP_TRY(c, hipEventElapsedTime(&ms1, e0.e, e1.e));
    if ((st = fold_budget(c, tl))) return st;
    c->act_at = -1;
    // fuse_k steps per launch, as fl_step runs them (entry, launches,
    // settling, exit); with active tiles after an untimed run that sets the
    // flags
    if (c->active) {
        st = c->prec == FL_F64 ? fused_steps_t<double>(c, 4, 1) : fused_steps_t<float>(c, 4, 1);
        if (st) return st;
    }
    HIP_TRY(c, hipEventRecord(e0.e, c->stream));
    st = c->prec == FL_F64 ? fused_steps_t<double>(c, trial_steps, 1)
                           : fused_steps_t<float>(c, trial_steps, 1);
    if (st) return st;
    HIP_TRY(c, hipEventRecord(e1.e, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1.e));
    HIP_TRY(c, hipEventElapsedTime(&ms2, e0.e, e1.e));
    c->fuse = (ms2 < ms1) ? c->fuse_k : 1;
    if (steps_per_launch) *steps_per_launch = c->fuse;
    if (ms_per_step) *ms_per_step = (c->fuse >= 2 ? ms2 : ms1) / trial_steps;
    return FL_OK;
}

size_t fl_device_bytes(const fl_ctx* c) { return c ? c->dev_bytes : 0; }

}  // extern "C"

// ------------------------------------------------------------ reverse mode
namespace {

fl_status adalloc(fl_ctx* c, void** p, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, e == hipErrorOutOfMemory ? FL_ENOMEM : FL_EHIP,
                    std::string("hipMalloc (adjoint): ") + hipGetErrorString(e));
    }
    c->adj_allocs.push_back(*p);
    HIP_TRY(c, hipMemsetAsync(*p, 0, bytes, c->stream));
    return FL_OK;
}

size_t field_bytes(const fl_ctx* c) { return (size_t)c->pitch * (c->ny + 2 * kHalo) * esz(c); }
size_t side_bytes(const fl_ctx* c) { return (size_t)std::max(c->nx, c->ny) * esz(c); }

// Layout of the end-of-forward snapshot: clock block, both inflow buffers,
// both partial-sum buffers, and the west/south edge faces.
size_t end_bytes(const fl_ctx* c) {
    return sizeof(DevCtl) + 2 * side_bytes(c) + 2 * sizeof(double) * std::max(c->nx, c->ny) +
           ((size_t)c->ny + c->nx) * esz(c);
}

fl_status snapshot_end(fl_ctx* c, bool restore) {
    unsigned char* e = static_cast<unsigned char*>(c->d_end);
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    auto mv = [&](void* live, size_t bytes) -> hipError_t {
        hipError_t r = restore ? hipMemcpyAsync(live, e, bytes, k, c->stream)
                               : hipMemcpyAsync(e, live, bytes, k, c->stream);
        e += bytes;
        return r;
    };
    const size_t pb = sizeof(double) * std::max(c->nx, c->ny);
    HIP_TRY(c, mv(c->d_ctl, sizeof(DevCtl)));
    HIP_TRY(c, mv(c->d_qin[0], side_bytes(c)));
    HIP_TRY(c, mv(c->d_qin[1], side_bytes(c)));
    HIP_TRY(c, mv(c->d_part[0], pb));
    HIP_TRY(c, mv(c->d_part[1], pb));
    HIP_TRY(c, mv(c->d_edge_w, (size_t)c->ny * esz(c)));
    HIP_TRY(c, mv(c->d_edge_s, (size_t)c->nx * esz(c)));
    return FL_OK;
}

// The backward sweep.  Segments are reversed from the last to the first.  A
// segment's states are recomputed from its checkpoint into one of two state
// stores by the step kernel on the context's stream, while the previous
// segment (one store) is reversed on a second stream: the recompute touches
// only the store, the clock, the inflow and partial-sum buffers and the edge
// arrays, the reverse passes only the adjoint buffers and the Manning and
// hydrograph gradients, so the two overlap.  Events order each store's
// recompute after the reverse that last read it, and each reverse after its
// recompute.
template <typename T>
fl_status adj_backward_t(fl_ctx* c, const void* dl, double* grad_n, int grad_on_device,
                         double* grad_q) {
    const size_t fb = field_bytes(c), sb = side_bytes(c);
    const long long N = c->adj_nsteps, C = c->adj_C, n0 = c->adj_n0;
    const int nx = c->nx, ny = c->ny, ng = (int)c->gauges.size();
    const int nsamp = (int)c->ts.size();
    fl_status st;
    // scratch of the sweep, kept with the forward record for further sweeps
    if (!c->d_bwd) {
        const size_t bytes = fb * 3 * (C + 1) * 2 + fb * 6 + sizeof(double) * nx * ny +
                             3 * sizeof(double) * std::max(1, c->in_count) +
                             sizeof(double) * std::max(1, nsamp) + 256 * 8;
        hipError_t e = hipMalloc(&c->d_bwd, bytes);
        if (e != hipSuccess) {
            c->d_bwd = nullptr;
            return fail(c, FL_ENOMEM, std::string("adjoint scratch: ") + hipGetErrorString(e));
        }
        c->adj_allocs.push_back(c->d_bwd);
    }
    unsigned char* cur_b = static_cast<unsigned char*>(c->d_bwd);
    auto carve = [&](size_t bytes) {
        unsigned char* p = cur_b;
        cur_b += (bytes + 255) & ~size_t(255);
        return p;
    };
    void* store[2];
    store[0] = carve(fb * 3 * (C + 1));
    store[1] = carve(fb * 3 * (C + 1));
    void* lam = carve(fb * 6);
    double* gn = (double*)carve(sizeof(double) * nx * ny);
    // inflow adjoints by step parity (a step's kernel writes one while it runs
    // the inflow pass of the step reversed before from the other), and the
    // inflow pass's own roughness terms
    const size_t inb = sizeof(double) * std::max(1, c->in_count);
    double* ain = (double*)carve(3 * inb);
    double* ainb[2] = {ain, (double*)((unsigned char*)ain + inb)};
    double* gn_in = (double*)((unsigned char*)ain + 2 * inb);
    double* gq = (double*)carve(sizeof(double) * std::max(1, nsamp));
    HIP_TRY(c, hipMemsetAsync(lam, 0, fb * 6, c->stream));
    HIP_TRY(c, hipMemsetAsync(gn, 0, sizeof(double) * nx * ny, c->stream));
    HIP_TRY(c, hipMemsetAsync(ain, 0, 3 * inb, c->stream));
    HIP_TRY(c, hipMemsetAsync(gq, 0, sizeof(double) * std::max(1, nsamp), c->stream));
    void* d_dl = nullptr;
    struct Owned {
        void* dl = nullptr;
        hipStream_t as = nullptr;
        hipEvent_t ev[5] = {};
        ~Owned() {
            if (as) (void)hipStreamSynchronize(as);
            for (hipEvent_t e : ev)
                if (e) (void)hipEventDestroy(e);
            if (as) (void)hipStreamDestroy(as);
            if (dl) (void)hipFree(dl);
        }
    } own;
    if (dl) {
        const size_t bytes = (size_t)c->adj_nobs * ng * sizeof(T);
        HIP_TRY(c, hipMalloc(&own.dl, std::max<size_t>(bytes, 256)));
        d_dl = own.dl;
        HIP_TRY(c, hipMemcpyAsync(d_dl, dl, bytes, hipMemcpyDefault, c->stream));
    }
    // the reverse stream (default priority); events: recomputed[2], reversed[2], start
    HIP_TRY(c, hipStreamCreateWithFlags(&own.as, hipStreamNonBlocking));
    for (hipEvent_t& e : own.ev) HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipEvent_t* recomputed = own.ev;
    hipEvent_t* reversed = own.ev + 2;
    hipEvent_t start = own.ev[4];
    bool reversed_set[2] = {false, false};
    HIP_TRY(c, hipEventRecord(start, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(own.as, start, 0));
    auto F = [&](void* base, long long k) { return static_cast<unsigned char*>(base) + fb * k; };
    T* lamf[6];
    for (int k = 0; k < 6; ++k) lamf[k] = (T*)F(lam, k);
    int cur = 0;   // lamf[3*cur .. 3*cur+2] hold the adjoint of the later state
    // the host replays the device clock: t_{k+1} = t_k + dt (dt rounded to T)
    std::vector<double> tseq(N + 1);
    const double dtT = (double)(T)c->params.dt_fixed;
    tseq[0] = c->adj_t0;
    for (long long k = 0; k < N; ++k) tseq[k + 1] = tseq[k] + dtT;
    const T* series = (const T*)c->d_series;
    const T* obs = (const T*)c->d_obs;
    const T* dlT = (const T*)d_dl;
    hipError_t e = hipSuccess;
    // recompute segment sgi into store[sgi & 1] (context stream)
    auto recompute = [&](long long sgi) -> hipError_t {
        const int b = (int)(sgi & 1);
        void* sto = store[b];
        hipError_t r = hipSuccess;
        if (reversed_set[b]) r = hipStreamWaitEvent(c->stream, reversed[b], 0);
        const long long ks = sgi * C, ke = std::min(ks + C, N);
        // restore the checkpoint: clock, the inflow that step reads, the state
        const long long nstart = n0 + ks;
        if (r == hipSuccess)
            r = hipMemcpyAsync(c->d_ctl, c->d_ck_ctl + sgi, sizeof(DevCtl), hipMemcpyDeviceToDevice, c->stream);
        if (r == hipSuccess)
            r = hipMemcpyAsync(c->d_qin[nstart & 1], static_cast<unsigned char*>(c->d_ck_qin) + sb * sgi, sb,
                               hipMemcpyDeviceToDevice, c->stream);
        for (int f = 0; f < 3 && r == hipSuccess; ++f)
            r = hipMemcpyAsync(F(sto, f), static_cast<unsigned char*>(c->d_ck) + fb * (3 * sgi + f), fb,
                               hipMemcpyDeviceToDevice, c->stream);
        // recompute the segment, keeping every state
        for (long long k = ks; k < ke && r == hipSuccess; ++k) {
            StepArgs<T> a = make_args<T>(c, n0 + k);
            const long long si = k - ks;
            a.h_in = (const T*)F(sto, 3 * si + 0);
            a.qx_in = (const T*)F(sto, 3 * si + 1);
            a.qy_in = (const T*)F(sto, 3 * si + 2);
            a.h_out = (T*)F(sto, 3 * (si + 1) + 0);
            a.qx_out = (T*)F(sto, 3 * (si + 1) + 1);
            a.qy_out = (T*)F(sto, 3 * (si + 1) + 2);
            r = launch_step<T>(a, c->cpt, c->stream);
        }
        if (r == hipSuccess) r = hipEventRecord(recomputed[b], c->stream);
        return r;
    };
    // reverse segment sgi from store[sgi & 1] (reverse stream)
    auto reverse = [&](long long sgi) -> hipError_t {
        const int b = (int)(sgi & 1);
        void* sto = store[b];
        hipError_t r = hipStreamWaitEvent(own.as, recomputed[b], 0);
        const long long ks = sgi * C, ke = std::min(ks + C, N);
        for (long long k = ke - 1; k >= ks && r == hipSuccess; --k) {
            T* l1 = lamf[3 * cur];
            if ((k + 1) % c->obs_every == 0) {
                const long long o = (k + 1) / c->obs_every - 1;
                const int nu = c->ngcell;
                r = launch_gauge_seed<T>(l1, c->pitch, nx, c->d_gcell, c->d_gcell + nu,
                                         c->d_gcell + 2 * nu + 1, nu, series + o * ng,
                                         obs ? obs + o * ng : nullptr, dlT ? dlT + o * ng : nullptr,
                                         own.as);
                if (r != hipSuccess) break;
            }
            AdjArgs<T> a{};
            const long long si = k - ks;
            a.h = (const T*)F(sto, 3 * si + 0);
            a.qx = (const T*)F(sto, 3 * si + 1);
            a.qy = (const T*)F(sto, 3 * si + 2);
            a.z = (const T*)c->d_z;
            a.n = (const T*)c->d_n;
            a.lh1 = lamf[3 * cur];
            a.lqx1 = lamf[3 * cur + 1];
            a.lqy1 = lamf[3 * cur + 2];
            a.lh = lamf[3 * (1 - cur)];
            a.lqx = lamf[3 * (1 - cur) + 1];
            a.lqy = lamf[3 * (1 - cur) + 2];
            a.gn = gn;
            a.ain = ainb[k & 1];
            a.ain_prev = ainb[(k + 1) & 1];
            a.gn_in = gn_in;
            a.gq = gq;
            a.rows = adjoint_rows(nx, ny);
            a.kout = (const T*)c->d_kout;
            a.in_z = c->d_in_z;
            a.in_k = c->d_in_k;
            a.ts = c->d_ts;
            a.qs = c->d_qs;
            a.pitch = c->pitch;
            a.nx = nx;
            a.ny = ny;
            a.in_side = c->in_count > 0 ? c->in_side : -1;
            a.in_first = c->in_first;
            a.in_count = c->in_count;
            a.nsamp = nsamp;
            a.out_side = c->out_count > 0 ? c->out_side : -1;
            a.out_first = c->out_first;
            a.out_count = c->out_count;
            a.positivity = c->params.positivity;
            a.dx = c->dx;
            a.g = c->params.g;
            a.dt = c->params.dt_fixed;
            a.h_eps = c->params.h_eps;
            a.in_slope = c->in_slope;
            a.out_slope = c->out_slope;
            a.t = tseq[k];
            // the inflow pass of step k+1 (reversed just before) runs in this
            // step's kernel
            a.bc_prev = (k + 1 < N) ? 1 : 0;
            a.t_prev = (k + 1 < N) ? tseq[k + 1] : 0.0;
            r = launch_adjoint_step<T>(a, own.as);
            cur = 1 - cur;
            if (k == 0 && r == hipSuccess) r = launch_adjoint_inflow<T>(a, own.as);
            if (k == 0 && r == hipSuccess) r = launch_adjoint_fold_inflow<T>(a, own.as);
        }
        if (r == hipSuccess) r = hipEventRecord(reversed[b], own.as);
        reversed_set[b] = true;
        return r;
    };
    if (c->adj_nck > 0) e = recompute(c->adj_nck - 1);
    for (long long sgi = c->adj_nck - 1; sgi >= 0 && e == hipSuccess; --sgi) {
        if (sgi >= 1) e = recompute(sgi - 1);   // overlaps the reverse of segment sgi
        if (e == hipSuccess) e = reverse(sgi);
    }
    // the context stream continues after the last reverse
    if (e == hipSuccess) e = hipEventRecord(start, own.as);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, start, 0);
    if (e == hipSuccess) {
        e = hipMemcpyAsync(grad_n, gn, sizeof(double) * nx * ny,
                           grad_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    }
    std::vector<double> gqh(std::max(1, nsamp));
    if (e == hipSuccess)
        e = hipMemcpyAsync(gqh.data(), gq, sizeof(double) * gqh.size(), hipMemcpyDeviceToHost, c->stream);
    // back to the end of the forward run
    c->nstep = n0 + N;
    c->act_at = -1;
    if (e == hipSuccess && (st = snapshot_end(c, true))) return st;
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint sweep");
    if (grad_q)
        for (int k = 0; k < nsamp; ++k) grad_q[k] = gqh[k];
    return FL_OK;
}

template <typename T>
fl_status adj_forward_t(fl_ctx* c, long long N, void* series_out, int on_device, double* loss) {
    fl_report r{};
    fl_status st = read_report(c, &r, false);
    if (st) return st;
    const double dtT = (double)(T)c->params.dt_fixed;
    if (!(c->params.t_end >= r.t + dtT * (double)N * (1.0 + 1e-12)))
        return fail(c, FL_EINVAL, "fl_adj_forward: t_end falls inside the run");
    const long long nobs = N / c->obs_every;
    const int ng = (int)c->gauges.size();
    if (c->d_obs && c->nobs_set < nobs)
        return fail(c, FL_EINVAL, "fl_adj_forward: fewer observations set than the run takes");
    // release the record of an earlier forward run (keep gauges and observations)
    std::vector<void*> keep;
    for (void* p : c->adj_allocs)
        if (p == c->d_gauges || p == c->d_gcell || p == c->d_obs) keep.push_back(p);
        else (void)hipFree(p);
    c->adj_allocs = keep;
    c->d_series = c->d_ck = c->d_ck_qin = c->d_end = c->d_bwd = nullptr;
    c->d_ck_ctl = nullptr;
    c->adj_nsteps = 0;
    const long long C = c->ckpt_req > 0 ? c->ckpt_req
                                        : std::max<long long>(1, (long long)std::ceil(std::sqrt((double)N)));
    const long long nck = (N + C - 1) / C;
    const size_t fb = field_bytes(c), sb = side_bytes(c);
    if ((st = adalloc(c, &c->d_series, sizeof(T) * std::max<long long>(1, nobs) * ng))) return st;
    if ((st = adalloc(c, &c->d_ck, fb * 3 * nck))) return st;
    if ((st = adalloc(c, (void**)&c->d_ck_ctl, sizeof(DevCtl) * nck))) return st;
    if ((st = adalloc(c, &c->d_ck_qin, sb * nck))) return st;
    if ((st = adalloc(c, &c->d_end, end_bytes(c)))) return st;
    const long long n0 = c->nstep;
    long long k = 0;
    while (k < N) {
        if (k % C == 0) {
            const long long sgi = k / C;
            const int p = (int)(c->nstep & 1);
            HIP_TRY(c, hipMemcpyAsync(static_cast<unsigned char*>(c->d_ck) + fb * (3 * sgi + 0), c->d_h[p], fb,
                                      hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(static_cast<unsigned char*>(c->d_ck) + fb * (3 * sgi + 1), c->d_qx[p], fb,
                                      hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(static_cast<unsigned char*>(c->d_ck) + fb * (3 * sgi + 2), c->d_qy[p], fb,
                                      hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->d_ck_ctl + sgi, c->d_ctl, sizeof(DevCtl), hipMemcpyDeviceToDevice,
                                      c->stream));
            HIP_TRY(c, hipMemcpyAsync(static_cast<unsigned char*>(c->d_ck_qin) + sb * sgi, c->d_qin[p], sb,
                                      hipMemcpyDeviceToDevice, c->stream));
        }
        const long long next_ck = (k / C + 1) * C;
        const long long next_obs = (k / c->obs_every + 1) * c->obs_every;
        const long long next = std::min(std::min(next_ck, next_obs), N);
        // single-step launches: the step counter (buffer parity and clock
        // slots) must advance by exactly one per step for the recompute
        if ((st = enqueue_steps(c, next - k))) return st;
        k = next;
        if (k % c->obs_every == 0 && k / c->obs_every <= nobs) {
            const long long o = k / c->obs_every - 1;
            HIP_TRY(c, launch_gauge_gather<T>((const T*)c->d_h[c->nstep & 1], c->pitch, c->nx, c->d_gauges, ng,
                                              (T*)c->d_series + o * ng, c->stream));
        }
    }
    if ((st = snapshot_end(c, false))) return st;
    c->adj_n0 = n0;
    c->adj_nsteps = N;
    c->adj_C = C;
    c->adj_nck = nck;
    c->adj_nobs = nobs;
    c->adj_t0 = r.t;
    std::vector<T> sh((size_t)std::max<long long>(1, nobs) * ng), oh;
    HIP_TRY(c, hipMemcpyAsync(sh.data(), c->d_series, sizeof(T) * nobs * ng, hipMemcpyDeviceToHost, c->stream));
    if (c->d_obs) {
        oh.resize(sh.size());
        HIP_TRY(c, hipMemcpyAsync(oh.data(), c->d_obs, sizeof(T) * nobs * ng, hipMemcpyDeviceToHost, c->stream));
    }
    if (series_out)
        HIP_TRY(c, hipMemcpyAsync(series_out, c->d_series, sizeof(T) * nobs * ng,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double L = 0.0;
    if (c->d_obs)
        for (size_t q = 0; q < (size_t)nobs * ng; ++q) {
            const double d = (double)sh[q] - (double)oh[q];
            L += d * d;
        }
    if (loss) *loss = L;
    fl_report r2{};
    if ((st = read_report(c, &r2, false))) return st;
    return FL_OK;
}

}  // namespace

extern "C" {

fl_status fl_adj_setup(fl_ctx* c, const int32_t* gauge_cells, int32_t ngauges, int32_t obs_every,
                       const void* obs, int64_t nobs, int obs_on_device, int32_t ckpt_stride) {
    if (!c) return FL_EINVAL;
    if (!c->committed) return fail(c, FL_ESTATE, "fl_adj_setup before fl_commit");
    if (!(c->params.dt_fixed > 0.0))
        return fail(c, FL_EINVAL, "fl_adj_setup: the reverse mode needs a fixed time step (dt_fixed > 0)");
    if (c->variant)
        return fail(c, FL_EINVAL, "fl_adj_setup: the reverse mode is derived for the default method");
    if (!gauge_cells || ngauges < 1 || obs_every < 1 || ckpt_stride < 0 || (obs && nobs < 1))
        return fail(c, FL_EINVAL, "fl_adj_setup: need gauges, obs_every >= 1, ckpt_stride >= 0");
    for (int k = 0; k < ngauges; ++k)
        if (gauge_cells[k] < 0 || (long long)gauge_cells[k] >= (long long)c->nx * c->ny)
            return fail(c, FL_EINVAL, "fl_adj_setup: gauge cell outside the grid");
    HIP_TRY(c, hipSetDevice(c->device));
    if (obs && obs_on_device)
        if (fl_status st = need_device(c, obs, "fl_adj_setup obs")) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_adjoint(c);
    c->gauges.assign(gauge_cells, gauge_cells + ngauges);
    c->obs_every = obs_every;
    c->ckpt_req = ckpt_stride;
    fl_status st;
    if ((st = adalloc(c, (void**)&c->d_gauges, sizeof(int) * ngauges))) return st;
    HIP_TRY(c, hipMemcpyAsync(c->d_gauges, gauge_cells, sizeof(int) * ngauges, hipMemcpyHostToDevice, c->stream));
    std::vector<int> packed;   // read by an asynchronous upload until the synchronization below
    {   // gauges grouped by cell, each group in gauge order
        std::vector<int> idx(ngauges);
        for (int k = 0; k < ngauges; ++k) idx[k] = k;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return gauge_cells[a] < gauge_cells[b]; });
        std::vector<int> cells, ptr, list;
        for (int k = 0; k < ngauges; ++k) {
            if (k == 0 || gauge_cells[idx[k]] != gauge_cells[idx[k - 1]]) {
                cells.push_back(gauge_cells[idx[k]]);
                ptr.push_back(k);
            }
            list.push_back(idx[k]);
        }
        ptr.push_back(ngauges);
        c->ngcell = (int)cells.size();
        packed = cells;
        packed.insert(packed.end(), ptr.begin(), ptr.end());
        packed.insert(packed.end(), list.begin(), list.end());
        if ((st = adalloc(c, (void**)&c->d_gcell, sizeof(int) * packed.size()))) return st;
        HIP_TRY(c, hipMemcpyAsync(c->d_gcell, packed.data(), sizeof(int) * packed.size(),
                                  hipMemcpyHostToDevice, c->stream));
    }
    c->nobs_set = 0;
    if (obs) {
        const size_t bytes = esz(c) * (size_t)nobs * ngauges;
        if ((st = adalloc(c, &c->d_obs, bytes))) return st;
        HIP_TRY(c, hipMemcpyAsync(c->d_obs, obs, bytes, obs_on_device ? hipMemcpyDeviceToDevice
                                                                      : hipMemcpyHostToDevice, c->stream));
        c->nobs_set = nobs;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->adj_setup = true;
    return FL_OK;
}

fl_status fl_adj_forward(fl_ctx* c, int64_t nsteps, void* series, int on_device, double* loss) {
    if (!c) return FL_EINVAL;
    if (!c->committed || !c->adj_setup) return fail(c, FL_ESTATE, "fl_adj_forward needs fl_commit and fl_adj_setup");
    if (nsteps < 1) return fail(c, FL_EINVAL, "fl_adj_forward: nsteps < 1");
    HIP_TRY(c, hipSetDevice(c->device));
    if (series && on_device)
        if (fl_status st = need_device(c, series, "fl_adj_forward series")) return st;
    return c->prec == FL_F64 ? adj_forward_t<double>(c, nsteps, series, on_device, loss)
                             : adj_forward_t<float>(c, nsteps, series, on_device, loss);
}

fl_status fl_adj_backward(fl_ctx* c, const void* dl_dseries, double* grad_n, int grad_on_device,
                          double* grad_q) {
    if (!c) return FL_EINVAL;
    if (!c->committed || !c->adj_setup || c->adj_nsteps < 1)
        return fail(c, FL_ESTATE, "fl_adj_backward needs a completed fl_adj_forward");
    if (c->nstep != c->adj_n0 + c->adj_nsteps)
        return fail(c, FL_ESTATE, "fl_adj_backward: the context was stepped after fl_adj_forward");
    if (!grad_n) return fail(c, FL_EINVAL, "fl_adj_backward: NULL grad_n");
    if (!dl_dseries && !c->d_obs)
        return fail(c, FL_EINVAL, "fl_adj_backward: no observations set and no dL/dseries given");
    HIP_TRY(c, hipSetDevice(c->device));
    if (grad_on_device)
        if (fl_status st = need_device(c, grad_n, "fl_adj_backward grad_n")) return st;
    return c->prec == FL_F64 ? adj_backward_t<double>(c, dl_dseries, grad_n, grad_on_device, grad_q)
                             : adj_backward_t<float>(c, dl_dseries, grad_n, grad_on_device, grad_q);
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct fl_batch {
    std::vector<fl_ctx*> members;   // in the caller's order
    std::vector<int> order;         // queue order: members by decreasing work
    int device = 0;
    hipStream_t stream = nullptr;
    fl_precision prec = FL_F32;
    int cpt = 0, rows = 0;
    void* d_scen = nullptr;
    size_t scen_bytes = 0;
    unsigned long long* d_sync = nullptr;   // [0] queue head, [1..] per-member done counts
    int* d_error = nullptr;
    int last_blocks = 0;
    int fuse = 1, cpt2 = 0, rows2 = 0;   // steps per queue entry and the multi-step tiling
    void* d_scen2 = nullptr;
    size_t scen2_bytes = 0;
    std::vector<int> member_xcd;    // XCD each member runs on (planning scratch, sized at create)
    void* h_stage = nullptr;        // pinned host staging of the descriptors (fl_batch_run_noalloc)
    size_t h_stage_bytes = 0;
    std::string err;
};

namespace {

fl_status bfail(fl_batch* b, fl_status s, const std::string& msg) {
    if (b) b->err = msg;
    return s;
}

#define BHIP_TRY(b, call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return bfail((b), FL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

fl_status batch_check_members(fl_batch* b) {
    for (fl_ctx* c : b->members)
        if (!c->committed)
            return bfail(b, FL_ESTATE, "fl_batch: a member is not committed (re-commit after fl_set_*)");
    return FL_OK;
}

// Number of XCDs the batch's members are spread over.
int batch_xccs(const fl_batch* b) {
    int nxcc = 1;
    if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, b->device) != hipSuccess || nxcc < 1)
        nxcc = 1;
    return std::min(nxcc, kMaxXcc);
}

// The member descriptors of one launch into scen[S] (host memory) and the
// per-XCD queues of `ba`: members are bin-packed onto the XCDs, largest
// first onto the least loaded.  Allocates nothing.
template <typename T>
void batch_plan(fl_batch* b, int freeze, int nxcc, BatchScen<T>* scen, BatchArgs<T>& ba) {
    const int S = (int)b->members.size();
    long long load[kMaxXcc] = {};
    for (int k = 0; k < S; ++k) {    // b->order is by decreasing cell count
        const int m = b->order[k];
        int x = 0;
        for (int y = 1; y < nxcc; ++y)
            if (load[y] < load[x]) x = y;
        b->member_xcd[m] = x;
        load[x] += (long long)b->members[m]->nx * b->members[m]->ny;
    }
    ba.nxcc = nxcc;
    int idx = 0;
    for (int x = 0; x < nxcc; ++x) {
        ba.xbegin[x] = idx;
        int first = 0;
        for (int k = 0; k < S; ++k) {
            const int m = b->order[k];
            if (b->member_xcd[m] != x) continue;
            fl_ctx* c = b->members[m];
            const Tiling tl = tiling_of(c, b->cpt, b->rows);
            for (int r = 0; r < 6; ++r) {
                scen[idx].a[r] = make_args<T>(c, r, tl, freeze);
                if (c->active) {
                    // the member's flags, indexed by its step counter as in its own steps
                    scen[idx].a[r].act = c->d_act;
                    scen[idx].a[r].act_stride = c->act_stride;
                }
            }
            scen[idx].n0 = c->nstep;
            scen[idx].items = tl.nstrips * tl.nchunks;
            scen[idx].first = first;
            first += 1 + scen[idx].items;
            ++idx;
        }
        ba.per_step[x] = first;
    }
    ba.xbegin[nxcc] = idx;
}

// One batch launch of nsteps steps with the descriptors scen_host (S entries)
// copied to d_scen, the queue heads and completion counters at d_sync
// (kMaxXcc + S words) and the error flag at d_error.  Allocates nothing.
template <typename T>
fl_status batch_execute(fl_batch* b, long long nsteps, int freeze, float* ms, BatchArgs<T>& ba,
                        const BatchScen<T>* scen_host, BatchScen<T>* d_scen,
                        unsigned long long* d_sync, int* d_error) {
    const int S = (int)b->members.size();
    // Members' pending work is on their own streams; the batch runs on its own.
    for (fl_ctx* c : b->members) BHIP_TRY(b, hipStreamSynchronize(c->stream));
    // The partial-sum slots depend on the work decomposition: fold them
    // before switching to the batch tiling.
    for (fl_ctx* c : b->members) {
        Tiling own{c->cpt, c->rows, c->nstrips, c->nchunks, c->npart};
        if (fold_budget(c, own)) return bfail(b, FL_EHIP, c->err);
    }
    for (fl_ctx* c : b->members) BHIP_TRY(b, hipStreamSynchronize(c->stream));
    bool any_active = false;
    for (fl_ctx* c : b->members) {
        if (!c->active) continue;
        any_active = true;
        // flags of another tiling or another path: compute every item in the first two steps
        if (!act_flags_hold(c, b->cpt, b->rows))
            BHIP_TRY(b, launch_fill_bytes(c->d_act, 3 * c->act_stride, 1, b->stream));
    }
    BHIP_TRY(b, hipMemcpyAsync(d_scen, scen_host, sizeof(BatchScen<T>) * S, hipMemcpyHostToDevice,
                               b->stream));
    // zeroed by a kernel (also fine inside a captured graph)
    BHIP_TRY(b, launch_fill_bytes(reinterpret_cast<unsigned char*>(d_sync),
                                  (long long)(sizeof(unsigned long long) * (S + kMaxXcc)), 0, b->stream));
    BHIP_TRY(b, launch_fill_bytes(reinterpret_cast<unsigned char*>(d_error), sizeof(int), 0, b->stream));
    ba.scen = d_scen;
    ba.nsteps = nsteps;
    ba.next = d_sync;
    ba.done = d_sync + kMaxXcc;
    ba.error = d_error;
    ba.spin_limit = 1LL << 26;   // ~ seconds of s_sleep: a wait that long means a broken hand-over
    Event e0, e1;
    if (ms) {
        BHIP_TRY(b, hipEventCreate(&e0.e));
        BHIP_TRY(b, hipEventCreate(&e1.e));
        BHIP_TRY(b, hipEventRecord(e0.e, b->stream));
    }
    BHIP_TRY(b, launch_batch<T>(ba, b->cpt, b->device, b->stream, &b->last_blocks, any_active));
    if (ms) BHIP_TRY(b, hipEventRecord(e1.e, b->stream));
    int error = 0;
    BHIP_TRY(b, hipMemcpyAsync(&error, d_error, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    if (ms) BHIP_TRY(b, hipEventElapsedTime(ms, e0.e, e1.e));
    for (fl_ctx* c : b->members) {
        c->nstep += nsteps;
        if (c->active) {
            c->act_mode = 1;
            c->act_at = c->nstep;
            c->act_cpt = b->cpt;
            c->act_rows = b->rows;
        }
    }
    for (int k = 0; k < S; ++k) {
        fl_ctx* c = b->members[b->order[k]];
        if (fold_budget(c, tiling_of(c, b->cpt, b->rows))) return bfail(b, FL_EHIP, c->err);
        BHIP_TRY(b, hipStreamSynchronize(c->stream));
    }
    if (error) return bfail(b, FL_EHIP, "fl_batch_run: a wait for a member's previous step timed out");
    return FL_OK;
}

template <typename T>
fl_status batch_launch(fl_batch* b, long long nsteps, int freeze, float* ms) {
    const int S = (int)b->members.size();
    std::vector<BatchScen<T>> scen(S);
    BatchArgs<T> ba{};
    batch_plan<T>(b, freeze, batch_xccs(b), scen.data(), ba);
    const size_t bytes = sizeof(BatchScen<T>) * S;
    if (bytes > b->scen_bytes) {
        if (b->d_scen) (void)hipFree(b->d_scen);
        b->d_scen = nullptr;
        b->scen_bytes = 0;
        BHIP_TRY(b, hipMalloc(&b->d_scen, bytes));
        b->scen_bytes = bytes;
    }
    return batch_execute<T>(b, nsteps, freeze, ms, ba, scen.data(), (BatchScen<T>*)b->d_scen,
                            b->d_sync, b->d_error);
}

constexpr size_t round256(size_t v) { return (v + 255) & ~size_t(255); }

// Scratch layout of fl_batch_run_noalloc for S members: descriptors, then the
// queue heads and completion counters, then the error flag.
template <typename T>
constexpr size_t noalloc_bytes(size_t S) {
    return round256(sizeof(BatchScen<T>) * S) +
           round256(sizeof(unsigned long long) * (kMaxXcc + S)) + 256;
}
static_assert(noalloc_bytes<float>(FL_NOALLOC_MAX_MEMBERS) <= kScratchBytes &&
                  noalloc_bytes<double>(FL_NOALLOC_MAX_MEMBERS) <= kScratchBytes,
              "the device scratch must hold the largest batch fl_batch_run_noalloc accepts");

template <typename T>
fl_status batch_launch_noalloc(fl_batch* b, long long nsteps) {
    const int S = (int)b->members.size();
    if (S > FL_NOALLOC_MAX_MEMBERS)
        return bfail(b, FL_EINVAL, "fl_batch_run_noalloc: the batch has " + std::to_string(S) +
                                       " members; at most " + std::to_string(FL_NOALLOC_MAX_MEMBERS) +
                                       " fit the device scratch");
    unsigned char* base = static_cast<unsigned char*>(scratch_ptr(b->device));
    if (!base) return bfail(b, FL_EHIP, "fl_batch_run_noalloc: no device scratch address for this device");
    if (!b->h_stage || b->h_stage_bytes < sizeof(BatchScen<T>) * S)
        return bfail(b, FL_ESTATE, "fl_batch_run_noalloc: the batch has no host staging");
    BatchScen<T>* hs = static_cast<BatchScen<T>*>(b->h_stage);
    BatchArgs<T> ba{};
    batch_plan<T>(b, 0, batch_xccs(b), hs, ba);
    BatchScen<T>* d_scen = reinterpret_cast<BatchScen<T>*>(base);
    unsigned long long* d_sync =
        reinterpret_cast<unsigned long long*>(base + round256(sizeof(BatchScen<T>) * S));
    int* d_error = reinterpret_cast<int*>(base + round256(sizeof(BatchScen<T>) * S) +
                                          round256(sizeof(unsigned long long) * (kMaxXcc + S)));
    return batch_execute<T>(b, nsteps, 0, nullptr, ba, hs, d_scen, d_sync, d_error);
}

// Can the members run several steps per queue entry?  They need the
// multi-step buffers (committed after fl_set_fusion(ctx, 2 or 3, ...)) and no
// active tiles.
fl_status batch_check_two_step(fl_batch* b) {
    for (fl_ctx* c : b->members) {
        if (!c->d_part2[0])
            return bfail(b, FL_ESTATE, "several steps per queue entry: every member must be "
                                       "committed after fl_set_fusion(ctx, 2 or 3, ...)");
        if (c->active)
            return bfail(b, FL_EINVAL, "several steps per queue entry: members with active tiles "
                                       "run one step per entry");
    }
    return FL_OK;
}

// nsteps steps of every member with K = 2 or 3 steps per queue entry: the
// members' single-step state (budget folded) becomes their multi-step clock,
// as in fused_steps_t; a round of batched K-step launches (about nsteps/K plus
// one that settles) follows, further rounds only if redos or shorter launches
// left a member short; finally every member's state becomes its single-step
// state again.
template <typename T>
fl_status batch2_launch(fl_batch* b, long long nsteps, int freeze, float* ms) {
    fl_status st = batch_check_two_step(b);
    if (st) return st;
    const int K = b->fuse;
    const int S = (int)b->members.size();
    for (fl_ctx* c : b->members) BHIP_TRY(b, hipStreamSynchronize(c->stream));
    for (fl_ctx* c : b->members) {
        Tiling own{c->cpt, c->rows, c->nstrips, c->nchunks, c->npart};
        if (fold_budget(c, own)) return bfail(b, FL_EHIP, c->err);
    }
    for (fl_ctx* c : b->members) BHIP_TRY(b, hipStreamSynchronize(c->stream));
    for (fl_ctx* c : b->members)
        BHIP_TRY(b, launch_enter_fused<T>(make_args<T>(c, c->nstep), nsteps, 0, b->stream));
    // bin-pack onto the XCDs as the one-step batch does
    const int nxcc = batch_xccs(b);
    long long load[kMaxXcc] = {};
    for (int k = 0; k < S; ++k) {
        const int m = b->order[k];
        int x = 0;
        for (int y = 1; y < nxcc; ++y)
            if (load[y] < load[x]) x = y;
        b->member_xcd[m] = x;
        load[x] += (long long)b->members[m]->nx * b->members[m]->ny;
    }
    std::vector<BatchScen2<T>> scen(S);
    Batch2Args<T> ba{};
    ba.nxcc = nxcc;
    int idx = 0;
    for (int x = 0; x < nxcc; ++x) {
        ba.xbegin[x] = idx;
        int first = 0;
        for (int k = 0; k < S; ++k) {
            const int m = b->order[k];
            if (b->member_xcd[m] != x) continue;
            fl_ctx* c = b->members[m];
            const Tiling tl = tiling_fused_of(c, b->cpt2, b->rows2, K);
            for (int res = 0; res < 2; ++res)
                for (int ph = 0; ph < 6; ++ph)
                    scen[idx].a2[res][ph] = make_args_fused_tl<T>(c, ph, res, tl, K, freeze);
            scen[idx].items = tl.nstrips * tl.nchunks;
            scen[idx].first = first;
            first += 1 + scen[idx].items;
            ++idx;
        }
        ba.per_launch[x] = first;
    }
    ba.xbegin[nxcc] = idx;
    const size_t bytes = sizeof(BatchScen2<T>) * S;
    if (bytes > b->scen2_bytes) {
        if (b->d_scen2) (void)hipFree(b->d_scen2);
        b->d_scen2 = nullptr;
        b->scen2_bytes = 0;
        BHIP_TRY(b, hipMalloc(&b->d_scen2, bytes));
        b->scen2_bytes = bytes;
    }
    BHIP_TRY(b, hipMemcpyAsync(b->d_scen2, scen.data(), bytes, hipMemcpyHostToDevice, b->stream));
    ba.scen = (const BatchScen2<T>*)b->d_scen2;
    ba.next = b->d_sync;
    ba.done = b->d_sync + kMaxXcc;
    ba.error = b->d_error;
    ba.spin_limit = 1LL << 26;
    Event e0, e1;
    if (ms) {
        BHIP_TRY(b, hipEventCreate(&e0.e));
        BHIP_TRY(b, hipEventCreate(&e1.e));
        BHIP_TRY(b, hipEventRecord(e0.e, b->stream));
    }
    std::vector<FusedClock> slot(S);
    long long lc = 0, want = (nsteps + K - 1) / K;
    for (int round = 0;; ++round) {
        BHIP_TRY(b, launch_fill_bytes(reinterpret_cast<unsigned char*>(b->d_sync),
                                      (long long)(sizeof(unsigned long long) * (S + kMaxXcc)), 0,
                                      b->stream));
        BHIP_TRY(b, launch_fill_bytes(reinterpret_cast<unsigned char*>(b->d_error), sizeof(int), 0,
                                      b->stream));
        ba.l0 = lc;
        ba.nlaunch = want + 1;   // the last launch only settles
        BHIP_TRY(b, launch_batch2<T>(ba, b->cpt2, K, b->device, b->stream, &b->last_blocks));
        lc += want + 1;
        if (ms) BHIP_TRY(b, hipEventRecord(e1.e, b->stream));
        int error = 0;
        BHIP_TRY(b, hipMemcpyAsync(&error, b->d_error, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        for (int m = 0; m < S; ++m)
            BHIP_TRY(b, hipMemcpyAsync(&slot[m], &b->members[m]->d_ctl->cf[lc & 1], sizeof(FusedClock),
                                       hipMemcpyDeviceToHost, b->stream));
        BHIP_TRY(b, hipStreamSynchronize(b->stream));
        if (error) return bfail(b, FL_EHIP, "fl_batch_run: a wait for a member's previous launch timed out");
        long long short_by = 0;
        for (int m = 0; m < S; ++m) {
            if (slot[m].pending) return bfail(b, FL_EHIP, "multi-step batch: unsettled member state");
            short_by = std::max(short_by, nsteps - slot[m].vsteps);
        }
        if (short_by <= 0) break;
        if (round >= 64) return bfail(b, FL_EHIP, "multi-step batch: no progress");
        want = short_by;   // enough even if every launch makes one step
    }
    if (ms) BHIP_TRY(b, hipEventElapsedTime(ms, e0.e, e1.e));
    for (int m = 0; m < S; ++m) {
        fl_ctx* c = b->members[m];
        const Tiling tl = tiling_fused_of(c, b->cpt2, b->rows2, K);
        long long n2 = c->nstep + nsteps;
        n2 += (n2 ^ (long long)slot[m].cur) & 1;
        BHIP_TRY(b, launch_leave_fused<T>(make_args<T>(c, n2), make_args_fused_tl<T>(c, 0, 0, tl, K, 0),
                                          lc, b->stream));
        c->nstep = n2;
    }
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    return FL_OK;
}

fl_status batch_run(fl_batch* b, long long nsteps, int freeze, float* ms) {
    fl_status st = batch_check_members(b);
    if (st) return st;
    if (nsteps == 0) {
        if (ms) *ms = 0.f;
        return FL_OK;
    }
    BHIP_TRY(b, hipSetDevice(b->device));
    if (b->fuse >= 2 && nsteps >= 2)
        return b->prec == FL_F64 ? batch2_launch<double>(b, nsteps, freeze, ms)
                                 : batch2_launch<float>(b, nsteps, freeze, ms);
    return b->prec == FL_F64 ? batch_launch<double>(b, nsteps, freeze, ms)
                             : batch_launch<float>(b, nsteps, freeze, ms);
}

}  // namespace

extern "C" {

fl_status fl_batch_create(fl_batch** out, int32_t nmembers, fl_ctx* const* members) {
    if (!out) return FL_EINVAL;
    *out = nullptr;
    if (nmembers < 1 || !members) {
        g_create_error = "fl_batch_create: need at least one member";
        return FL_EINVAL;
    }
    for (int k = 0; k < nmembers; ++k) {
        if (!members[k] || !members[k]->committed) {
            g_create_error = "fl_batch_create: every member must be a committed context";
            return FL_ESTATE;
        }
        if (members[k]->device != members[0]->device || members[k]->prec != members[0]->prec) {
            g_create_error = "fl_batch_create: members must share device and precision";
            return FL_EINVAL;
        }
        if (members[k]->variant) {
            g_create_error = "fl_batch_create: batches run the default method (no fl_set_variant)";
            return FL_EINVAL;
        }
        for (int l = 0; l < k; ++l)
            if (members[l] == members[k]) {
                g_create_error = "fl_batch_create: a context appears twice";
                return FL_EINVAL;
            }
    }
    fl_batch* b = new (std::nothrow) fl_batch();
    if (!b) return FL_ENOMEM;
    b->members.assign(members, members + nmembers);
    b->device = members[0]->device;
    b->prec = members[0]->prec;
    b->cpt = b->prec == FL_F64 ? 2 : 4;
    b->rows = 16;
    hipError_t e = hipSetDevice(b->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_sync, sizeof(unsigned long long) * (nmembers + kMaxXcc));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_error, sizeof(int));
    // host staging of the descriptors for fl_batch_run_noalloc, sized for either precision
    b->h_stage_bytes = std::max(sizeof(BatchScen<float>), sizeof(BatchScen<double>)) * nmembers;
    if (e == hipSuccess) e = hipHostMalloc(&b->h_stage, b->h_stage_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        g_create_error = std::string("fl_batch_create: ") + hipGetErrorString(e);
        fl_batch_destroy(b);
        return FL_EHIP;
    }
    b->order.resize(nmembers);
    b->member_xcd.assign(nmembers, 0);
    for (int k = 0; k < nmembers; ++k) b->order[k] = k;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (long long)members[x]->nx * members[x]->ny > (long long)members[y]->nx * members[y]->ny;
    });
    *out = b;
    return FL_OK;
}

fl_status fl_batch_set_tiling(fl_batch* b, int32_t cells_per_lane, int32_t rows_per_item) {
    if (!b) return FL_EINVAL;
    if (cells_per_lane != 1 && cells_per_lane != 2 && cells_per_lane != 4)
        return bfail(b, FL_EINVAL, "fl_batch_set_tiling: cells_per_lane must be 1, 2 or 4");
    if (b->prec == FL_F64 && cells_per_lane == 4)
        return bfail(b, FL_EINVAL, "fl_batch_set_tiling: FP64 supports 1 or 2 cells per lane");
    if (rows_per_item < 1) return bfail(b, FL_EINVAL, "fl_batch_set_tiling: rows_per_item must be >= 1");
    b->cpt = cells_per_lane;
    b->rows = rows_per_item;
    return FL_OK;
}

fl_status fl_batch_set_fusion(fl_batch* b, int32_t steps_per_entry, int32_t cells_per_lane,
                              int32_t rows_per_item) {
    if (!b) return FL_EINVAL;
    if (steps_per_entry < 1 || steps_per_entry > 3)
        return bfail(b, FL_EINVAL, "fl_batch_set_fusion: steps_per_entry must be 1, 2 or 3");
    if (cells_per_lane != 0 && cells_per_lane != 1 && cells_per_lane != 2)
        return bfail(b, FL_EINVAL, "fl_batch_set_fusion: cells_per_lane must be 0, 1 or 2");
    if (rows_per_item < 0) return bfail(b, FL_EINVAL, "fl_batch_set_fusion: rows_per_item < 0");
    if (steps_per_entry >= 2) {
        fl_status st = batch_check_two_step(b);
        if (st) return st;
    }
    b->fuse = steps_per_entry;
    b->cpt2 = cells_per_lane ? cells_per_lane : (b->prec == FL_F64 ? 1 : 2);
    b->rows2 = rows_per_item ? rows_per_item : 64;
    return FL_OK;
}

fl_status fl_batch_run(fl_batch* b, int64_t nsteps) {
    if (!b) return FL_EINVAL;
    if (nsteps < 0) return bfail(b, FL_EINVAL, "fl_batch_run: nsteps < 0");
    return batch_run(b, nsteps, 0, nullptr);
}

fl_status fl_batch_run_noalloc(fl_batch* b, int64_t nsteps) {
    if (!b) return FL_EINVAL;
    if (nsteps < 0) return bfail(b, FL_EINVAL, "fl_batch_run_noalloc: nsteps < 0");
    fl_status st = batch_check_members(b);
    if (st) return st;
    if (nsteps == 0) return FL_OK;
    BHIP_TRY(b, hipSetDevice(b->device));
    return b->prec == FL_F64 ? batch_launch_noalloc<double>(b, nsteps)
                             : batch_launch_noalloc<float>(b, nsteps);
}

fl_status fl_batch_time(fl_batch* b, int64_t nsteps, double* elapsed_ms) {
    if (!b || !elapsed_ms) return FL_EINVAL;
    if (nsteps < 0) return bfail(b, FL_EINVAL, "fl_batch_time: nsteps < 0");
    float ms = 0.f;
    fl_status st = batch_run(b, nsteps, 0, &ms);
    *elapsed_ms = ms;
    return st;
}

fl_status fl_batch_autotune(fl_batch* b, const int32_t* candidates, int32_t ncand, int32_t trial_steps,
                            int32_t* best, double* best_ms) {
    if (!b || !candidates || ncand < 1 || trial_steps < 1) return FL_EINVAL;
    const bool two = b->fuse >= 2;
    int& cpt_ref = two ? b->cpt2 : b->cpt;
    int& rows_ref = two ? b->rows2 : b->rows;
    const int cpt0 = cpt_ref, rows0 = rows_ref;
    double best_t = 1e300;
    int bc = -1;
    for (int k = 0; k < ncand; ++k) {
        fl_status st = two ? fl_batch_set_fusion(b, b->fuse, candidates[2 * k], candidates[2 * k + 1])
                           : fl_batch_set_tiling(b, candidates[2 * k], candidates[2 * k + 1]);
        if (!st && two && candidates[2 * k] == 0)
            st = bfail(b, FL_EINVAL, "fl_batch_autotune: cells_per_lane must be 1 or 2");
        if (st) {
            cpt_ref = cpt0;
            rows_ref = rows0;
            return st;
        }
        float ms = 0.f;
        // Frozen steps (dt = 0) stream the whole state like real steps but leave it unchanged.
        // Members with active tiles first take two untimed steps that set their flags for
        // this tiling, so that the timed ones skip as real steps would.
        bool any_active = false;
        for (fl_ctx* c : b->members) any_active = any_active || c->active;
        if (any_active) st = batch_run(b, 2, 1, nullptr);
        if (!st) st = batch_run(b, trial_steps, 1, &ms);
        if (st) {
            cpt_ref = cpt0;
            rows_ref = rows0;
            return st;
        }
        if (ms < best_t) {
            best_t = ms;
            bc = k;
        }
    }
    cpt_ref = candidates[2 * bc];
    rows_ref = candidates[2 * bc + 1];
    if (best) {
        best[0] = cpt_ref;
        best[1] = rows_ref;
    }
    if (best_ms) *best_ms = best_t / trial_steps;
    return FL_OK;
}

const char* fl_batch_last_error(const fl_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }

void fl_batch_destroy(fl_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->d_scen) (void)hipFree(b->d_scen);
    if (b->d_scen2) (void)hipFree(b->d_scen2);
    if (b->d_sync) (void)hipFree(b->d_sync);
    if (b->d_error) (void)hipFree(b->d_error);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* fl_last_error(const fl_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

void fl_destroy(fl_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_device(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
