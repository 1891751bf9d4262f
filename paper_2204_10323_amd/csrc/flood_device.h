// Device helpers shared by the step, batch and adjoint kernels of libflood:
// the face update of eq. (3), the boundary values of eq. (5)/(6), the clock
// and the inflow solve.  One definition each, so a quantity recomputed by
// another kernel has the same bits.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <math.h>

#include "flood_internal.h"

namespace flood {

enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };

// ------------------------------------------------------------------ helpers
// Ordered bits of a depth for the max-reduction: negative -> 0, NaN above +inf.
template <typename T> struct Ord;
template <> struct Ord<float> {
    typedef unsigned U;  // the key in the working precision's width
    static __device__ __forceinline__ U key(float h) {
        if (h >= 0.0f) return __float_as_uint(h);
        if (h < 0.0f) return 0u;
        return 0x7fc00000u;
    }
    static __device__ __forceinline__ unsigned long long bits(float h) {
        if (h >= 0.0f) return (unsigned long long)__float_as_uint(h);
        if (h < 0.0f) return 0ull;
        return 0x7fc00000ull;
    }
    static __device__ __forceinline__ double value(unsigned long long b) {
        return (double)__uint_as_float((unsigned)b);
    }
    static __device__ __forceinline__ bool nonfinite(unsigned long long b) { return b >= 0x7f800000ull; }
};
template <> struct Ord<double> {
    typedef unsigned long long U;
    static __device__ __forceinline__ U key(double h) { return bits(h); }
    static __device__ __forceinline__ unsigned long long bits(double h) {
        if (h >= 0.0) return (unsigned long long)__double_as_longlong(h);
        if (h < 0.0) return 0ull;
        return 0x7ff8000000000000ull;
    }
    static __device__ __forceinline__ double value(unsigned long long b) {
        return __longlong_as_double((long long)b);
    }
    static __device__ __forceinline__ bool nonfinite(unsigned long long b) {
        return b >= 0x7ff0000000000000ull;
    }
};

__device__ __forceinline__ float cbrt_t(float x) { return cbrtf(x); }
__device__ __forceinline__ double cbrt_t(double x) { return cbrt(x); }

// x^(5/3) for x > 0, else 0.
template <typename T>
__device__ __forceinline__ T pow53(T x) {
    if (!(x > T(0))) return T(0);
    T c = cbrt_t(x);
    return x * (c * c);
}

// x^(2/3) for x > 0, else 0 (the literal reading of eq. 5).
template <typename T>
__device__ __forceinline__ T pow23(T x) {
    if (!(x > T(0))) return T(0);
    T c = cbrt_t(x);
    return c * c;
}

// Value held by the next (lane + 1) or previous (lane - 1) lane of the wave,
// by the wave-wide DPP shifts of GFX9 (wave_shl:1, wave_shr:1): a register
// move the ALU does in place, no LDS round trip.  The last (first) lane keeps
// its own value.
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ float from_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ __forceinline__ float from_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
__device__ __forceinline__ double from_next(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_next((int)(b & 0xffffffffll)), hi = dpp_next((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_prev(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_prev((int)(b & 0xffffffffll)), hi = dpp_prev((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ unsigned wave_max_key(unsigned v) {
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v);
__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long v) {
    return wave_max_u64(v);
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int o = 32; o >= 1; o >>= 1) {
        unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffull), o, 64);
        unsigned hi = __shfl_xor((unsigned)(v >> 32), o, 64);
        unsigned long long w = ((unsigned long long)hi << 32) | lo;
        v = w > v ? w : v;
    }
    return v;
}

// f(std::integral_constant<int, I>) for I = B .. E - 1, in order: a loop whose
// index is a compile-time constant in its body.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Wait until every vector memory operation of the wave has completed
// (vmcnt = 0; the export and LDS/scalar counters are left alone).
__device__ __forceinline__ void wait_vector_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// A value every lane of the wave holds: read it from the first lane, so that
// it lives in scalar registers (VALU results are vector registers even when
// uniform; a marcher chain's per-step constants would otherwise take ~7 VGPRs
// per step).
__device__ __forceinline__ float wave_uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Row accesses through pointers typed in the global address space.  Every
// field of the library is device memory.  Pointers a kernel reads from memory
// (a batch's member descriptors) rather than from its arguments would
// otherwise compile to flat accesses, which cannot take a scalar base address
// and are counted with the LDS and scalar-memory operations.  Kernels whose
// row pointers are launch arguments keep generic pointers (GA = false): the
// compiler already proves them global there, and the generic form schedules
// the two-step marcher's loads and stores better.
template <typename T>
struct Global { typedef __attribute__((address_space(1))) T type; };
template <typename T>
__device__ __forceinline__ typename Global<T>::type* as_global(T* p) {
    return (typename Global<T>::type*)p;
}
template <bool GA, typename T>
struct Space { typedef T type; };
template <typename T>
struct Space<true, T> { typedef typename Global<T>::type type; };
template <bool GA, typename T>
__device__ __forceinline__ typename Space<GA, T>::type* in_space(T* p) {
    return (typename Space<GA, T>::type*)p;
}
// V in the address space (and constness) of E
template <typename E, typename V>
struct Like { typedef V type; };
template <typename E, typename V>
struct Like<const E, V> { typedef const V type; };
template <typename E, typename V>
struct Like<__attribute__((address_space(1))) E, V> {
    typedef __attribute__((address_space(1))) V type;
};
template <typename E, typename V>
struct Like<const __attribute__((address_space(1))) E, V> {
    typedef const __attribute__((address_space(1))) V type;
};

// A pointer every lane holds (a row start): in scalar registers, so that a
// row access takes the scalar-base + 32-bit lane offset form, and the compiler
// does not keep a 64-bit per-lane address for every field across the row loop.
// (Formed as p plus a zero the compiler cannot see through, so that the
// pointer keeps its provenance and address space.)
template <typename P>
__device__ __forceinline__ P* wave_uniform_ptr(P* p) {
    const unsigned long long b = (unsigned long long)(__UINTPTR_TYPE__)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    const long long d = (long long)((((unsigned long long)hi << 32) | lo) - b);
    typedef typename Like<P, char>::type B;
    return reinterpret_cast<P*>(const_cast<B*>(reinterpret_cast<const B*>(p)) + d);
}

// Element at byte offset boff (32-bit, per lane) from a row start that is the
// same in every lane: the form the scalar-base + 32-bit-offset memory
// instructions take, with no per-lane 64-bit address arithmetic.
template <typename E>
__device__ __forceinline__ E* at_byte(E* row, unsigned boff) {
    typedef typename Like<E, char>::type B;
    return reinterpret_cast<E*>(reinterpret_cast<B*>(row) + boff);
}

// Vector load of a row segment (N consecutive elements) and vector store of the
// new state.  NT = true marks the store non-temporal: the new state is not
// read again within the launch, so it should not displace the halo rows and
// columns other waves still read.  Kernels that hand data to other waves
// inside one launch (the persistent batch) store normally, so the data is
// resident in L2 when the wave's memory counter drains.
template <typename T, int N>
struct NVec { typedef T type __attribute__((ext_vector_type(N))); };
template <typename T, int N>
struct alignas(sizeof(T) * N) VecT { T v[N]; };
template <typename T, int N>
__device__ __forceinline__ void ldv(const T* p, T (&o)[N]) {
    const VecT<T, N> t = *reinterpret_cast<const VecT<T, N>*>(p);
#pragma unroll
    for (int m = 0; m < N; ++m) o[m] = t.v[m];
}
template <typename T, int N>
__device__ __forceinline__ void ldv(const typename Global<T>::type* p, T (&o)[N]) {
    typedef const typename Global<typename NVec<T, N>::type>::type V;
    const typename NVec<T, N>::type t = *reinterpret_cast<V*>(p);
    // a byte copy out of the vector keeps the row registers out of private
    // memory (copied element by element, the compiler spilled the prefetched
    // row to scratch and waited for the loads at once)
    __builtin_memcpy(o, &t, sizeof(t));
}
template <typename T, int N, bool NT, typename E>
__device__ __forceinline__ void stv(E* p, const T (&o)[N]) {
    typename NVec<T, N>::type t;
#pragma unroll
    for (int m = 0; m < N; ++m) t[m] = o[m];
    typedef typename Like<E, typename NVec<T, N>::type>::type V;
    if (NT) __builtin_nontemporal_store(t, reinterpret_cast<V*>(p));
    else *reinterpret_cast<V*>(p) = t;
}

// ------------------------------------------------------------ the physics
// Eq. (3) on one face between cells L and R (R on the +axis side).  q is the
// face discharge at the start of the step; gdt = g*dt.  Flow depth h_f is the
// higher water surface minus the higher bed; a face with h_f <= h_eps is dry.
// Friction uses the face's own |q| (per-axis 1-D form) and n_f = (n_L+n_R)/2.
template <typename T>
__device__ __forceinline__ T face_q(T etaL, T etaR, T zL, T zR, T nL, T nR, T q, T gdt,
                                    T inv_dx, T h_eps) {
    T hf = fmax(etaL, etaR) - fmax(zL, zR);
    if (hf <= h_eps) return T(0);
    T nf = T(0.5) * (nL + nR);
    T grad = (etaR - etaL) * inv_dx;
    T num = q - (gdt * hf) * grad;
    T den = T(1) + ((gdt * (nf * nf)) * fabs(q)) / ((hf * hf) * cbrt_t(hf));
    return num / den;
}

// Maxima on the hot path.  For fmax the compiler first "canonicalises" every
// operand it cannot prove canonical (a value straight from memory, a lane
// move, a loop-carried register) with v_max_f32 x, x, x, which only quiets a
// signalling NaN: about 16 instructions per marcher row.  v_max_f32 itself
// already returns the other operand for a quiet NaN and a quiet NaN for a
// signalling one, which is what fmax returns, so FP32 takes it directly (the
// same instruction the compiler emits for fmax, minus the canonicalisation).
template <typename T>
__device__ __forceinline__ T maxv(T a, T b) { return fmax(a, b); }
template <>
__device__ __forceinline__ float maxv<float>(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// max(0, a) and max(0, -a)
template <typename T>
__device__ __forceinline__ T max0(T a) { return fmax(T(0), a); }
template <>
__device__ __forceinline__ float max0<float>(float a) {
    float r;
    asm("v_max_f32 %0, 0, %1" : "=v"(r) : "v"(a));
    return r;
}
template <typename T>
__device__ __forceinline__ T max0_neg(T a) { return fmax(T(0), -a); }
template <>
__device__ __forceinline__ float max0_neg<float>(float a) {
    float r;
    asm("v_max_f32_e64 %0, 0, -%1" : "=v"(r) : "v"(a));
    return r;
}

// FP32 face update: the same formula with h_f^(-7/3) = 2^(-(7/3) log2 h_f)
// and the quotient by the hardware reciprocal (v_log_f32, v_exp_f32,
// v_rcp_f32, about one ulp each) instead of cbrt and two correctly rounded
// divisions, which roughly halves the face's ALU work.  FP64 keeps the
// correctly rounded operations.
template <>
__device__ __forceinline__ float face_q<float>(float etaL, float etaR, float zL, float zR,
                                               float nL, float nR, float q, float gdt,
                                               float inv_dx, float h_eps) {
    float hf = maxv(etaL, etaR) - maxv(zL, zR);
    if (hf <= h_eps) return 0.0f;
    float nf = 0.5f * (nL + nR);
    float grad = (etaR - etaL) * inv_dx;
    float num = q - (gdt * hf) * grad;
    // clamped so that a film thin enough to overflow it (h_f < 3e-17, possible
    // only with h_eps below that) still gives 0 * large = 0 for q = 0, as the
    // division does
    float m73 = fminf(__builtin_amdgcn_exp2f((-7.0f / 3.0f) * __builtin_amdgcn_logf(hf)), 3.0e38f);
    float den = 1.0f + ((gdt * (nf * nf)) * fabsf(q)) * m73;
    return num * __builtin_amdgcn_rcpf(den);
}

// Eq. (3) with the discharge magnitude of the friction term given (qm), for
// the variant that takes the magnitude of the discharge vector at the face
// instead of the face's own |q|; same operations as face_q otherwise.
template <typename T>
__device__ __forceinline__ T face_qm(T etaL, T etaR, T zL, T zR, T nL, T nR, T q, T qm, T gdt,
                                     T inv_dx, T h_eps) {
    T hf = fmax(etaL, etaR) - fmax(zL, zR);
    if (hf <= h_eps) return T(0);
    T nf = T(0.5) * (nL + nR);
    T grad = (etaR - etaL) * inv_dx;
    T num = q - (gdt * hf) * grad;
    T den = T(1) + ((gdt * (nf * nf)) * qm) / ((hf * hf) * cbrt_t(hf));
    return num / den;
}
template <>
__device__ __forceinline__ float face_qm<float>(float etaL, float etaR, float zL, float zR,
                                                float nL, float nR, float q, float qm, float gdt,
                                                float inv_dx, float h_eps) {
    float hf = fmaxf(etaL, etaR) - fmaxf(zL, zR);
    if (hf <= h_eps) return 0.0f;
    float nf = 0.5f * (nL + nR);
    float grad = (etaR - etaL) * inv_dx;
    float num = q - (gdt * hf) * grad;
    float m73 = fminf(__builtin_amdgcn_exp2f((-7.0f / 3.0f) * __builtin_amdgcn_logf(hf)), 3.0e38f);
    float den = 1.0f + ((gdt * (nf * nf)) * qm) * m73;
    return num * __builtin_amdgcn_rcpf(den);
}

// Donor-cell factor r = h+/O of a cell whose outflow O exceeds its depth h+.
template <typename T>
__device__ __forceinline__ T donor_ratio(T hp, T O) { return hp / O; }
template <>
__device__ __forceinline__ float donor_ratio<float>(float hp, float O) {
    // an outflow so small that its reciprocal overflows takes the division
    if (O < 1.0e-30f) return hp / O;
    return fminf(hp * __builtin_amdgcn_rcpf(O), 1.0f);
}

// dt of this step from the clock slot and the deepest cell of the current
// state: the fixed step, or min(dt_max, alpha dx / sqrt(g h_max)); shortened to
// land on t_end; 0 once done or non-finite.  Rounded to T (the step uses it).
template <typename T>
__device__ __forceinline__ double step_dt(const StepArgs<T>& a, const ClockSlot& ck,
                                          unsigned long long hb, double t_end, int& last,
                                          int& done, int& nonfin) {
    last = 0;
    done = 0;
    nonfin = ck.nonfinite || Ord<T>::nonfinite(hb);
    if (nonfin || a.freeze) return 0.0;
    double dt;
    if (a.dt_fixed > 0.0) {
        dt = a.dt_fixed;
    } else {
        double hm = Ord<T>::value(hb);
        dt = hm > 0.0 ? fmin(a.dt_max, a.alpha * a.dx / sqrt(a.g * hm)) : a.dt_max;
    }
    double rem = t_end - ck.t;
    if (!(rem > 0.0)) {
        done = 1;
        return 0.0;
    }
    if (dt >= rem) {
        dt = rem;
        last = 1;
    }
    return (double)(T)dt;
}

// The clock after a step of length dt (flags from step_dt) whose inflow faces
// carried si in total (per unit width).  The outflow volume is added
// separately, once the step's partial sums exist.
__device__ __forceinline__ ClockSlot advance_clock(const ClockSlot& ck, double dt, int last,
                                                   int done, int nonfin, double si, double dx,
                                                   double t_end) {
    ClockSlot nk = ck;
    nk.t = last ? t_end : ck.t + dt;
    nk.dt_prev = dt;
    nk.last_dt = dt > 0.0 ? dt : ck.last_dt;
    nk.v_in = ck.v_in + dt * dx * si;
    nk.steps = ck.steps + (dt > 0.0 ? 1 : 0);
    nk.done = (done || last) ? 1 : 0;
    nk.nonfinite = nonfin ? 1 : 0;
    return nk;
}

// Q_in(t): piecewise linear between samples, constant outside.
template <typename T>
__device__ double hydrograph(const StepArgs<T>& a, double t) {
    const int ns = a.nsamp;
    if (ns <= 0) return 0.0;
    if (t <= a.ts[0]) return a.qs[0];
    if (t >= a.ts[ns - 1]) return a.qs[ns - 1];
    int lo = 0, hi = ns - 1;  // ts[lo] <= t < ts[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a.ts[mid] <= t) lo = mid; else hi = mid;
    }
    return a.qs[lo] + (a.qs[hi] - a.qs[lo]) * ((t - a.ts[lo]) / (a.ts[hi] - a.ts[lo]));
}

// Eq. (6) on one wave: the water level W with F(W) = sum_c dx k_c (W - z_c)_+^{5/3}
// - Q = 0 (k_c = sqrt(S_in)/n_c).  F is continuous, convex and strictly
// increasing above min z, so the root is unique, and Newton's method started
// where F >= 0 (the right end of the bracket [min z, max z + (Q/(dx sum k))^{3/5}])
// decreases monotonically onto it; it stops when an update no longer
// decreases W.  Every lane returns the same W.  Requires Q > 0 and nc > 0.
__device__ inline double inflow_level(const double* in_z, const double* in_k, int nc, double dx,
                                      double Q) {
    const int lane = threadIdx.x & 63;
    double hi = -1e300, ks = 0.0;
    for (int p = lane; p < nc; p += 64) {
        hi = fmax(hi, in_z[p]);
        ks += in_k[p];
    }
    hi = wave_max(hi);
    ks = wave_sum(ks);
    double W = hi + pow(Q / (dx * ks), 0.6);
    for (int it = 0; it < 60; ++it) {
        double F = 0.0, dF = 0.0;
        for (int p = lane; p < nc; p += 64) {
            const double d = W - in_z[p];
            if (d > 0.0) {
                const double c = cbrt(d);
                F += dx * in_k[p] * (d * (c * c));
                dF += dx * in_k[p] * (5.0 / 3.0) * (c * c);
            }
        }
        F = wave_sum(F) - Q;
        dF = wave_sum(dF);
        const double Wn = W - F / dF;
        if (!(Wn < W)) break;
        W = Wn;
    }
    return W;
}

// Eq. (6) with eq. (5) taken literally (A = dx^2, hydraulic radius = depth):
// the level W at which the cells pass dx^2 k_c (W - z_c)_+^{2/3} in total.
// The sum is concave in W, so it is bisected (64 times, FP64) between min z
// and max z + (Q / (dx^2 sum k))^{3/2}, where every cell passes at least its
// share.  One wave.
__device__ inline double inflow_level_area(const double* in_z, const double* in_k, int nc,
                                           double dx, double Q) {
    const int lane = threadIdx.x & 63;
    double lo = 1e300, hi = -1e300, ks = 0.0;
    for (int p = lane; p < nc; p += 64) {
        lo = fmin(lo, in_z[p]);
        hi = fmax(hi, in_z[p]);
        ks += in_k[p];
    }
    lo = -wave_max(-lo);
    hi = wave_max(hi);
    ks = wave_sum(ks);
    hi += pow(Q / (dx * dx * ks), 1.5);
    for (int it = 0; it < 64; ++it) {
        const double mid = 0.5 * (lo + hi);
        double F = 0.0;
        for (int p = lane; p < nc; p += 64) F += dx * (dx * in_k[p] * pow23(mid - in_z[p]));
        F = wave_sum(F) - Q;
        if (F < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// The inflow split on one wave: per-cell face discharges (per unit width)
// into dst[first .. first+count).
template <typename T, int VAR = 0>
__device__ void inflow_solve(const StepArgs<T>& a, double Q, T* dst) {
    const int lane = threadIdx.x & 63;
    const int nc = a.in_count;
    if (nc <= 0) return;
    if (!(Q > 0.0)) {
        for (int p = lane; p < nc; p += 64) dst[a.in_first + p] = T(0);
        return;
    }
    if constexpr ((VAR & VAR_BOUNDARY_CELL_AREA) != 0) {
        const double W = inflow_level_area(a.in_z, a.in_k, nc, a.dx, Q);
        for (int p = lane; p < nc; p += 64)
            dst[a.in_first + p] = (T)(a.dx * a.in_k[p] * pow23(W - a.in_z[p]));
    } else {
        const double W = inflow_level(a.in_z, a.in_k, nc, a.dx, Q);
        for (int p = lane; p < nc; p += 64) dst[a.in_first + p] = (T)(a.in_k[p] * pow53(W - a.in_z[p]));
    }
}


}  // namespace flood
