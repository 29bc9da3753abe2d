// Device helpers shared by the lattice kernels: vector loads, the one
// definition of the drift, FP64 block sums, and the FP64 tails that turn the
// volume sums of a pass into the scale-factor update and the diagnostics.
#pragma once

#include <math.h>

#include "ce_internal.hpp"

namespace ce {
namespace dev {

// Pointers into device memory, typed as global so loads and stores compile to
// global_* instructions (generic pointers taken from a struct would become
// flat_* accesses, which share the LDS wait counter).
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
using gcptr = const __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(void *p)
{
    return (gptr<T>)p;
}

template <typename T>
struct Quad {
    T v[4];
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// VEC consecutive x sites of one array.
template <typename T, int VEC>
struct Vec {
    T v[VEC];
};

__device__ __forceinline__ Vec<float, 2> load_vec2(gcptr<float> base, long long s)
{
    const f32x2 q = *(gcptr<f32x2>)(base + s);
    return Vec<float, 2>{{q.x, q.y}};
}
__device__ __forceinline__ Vec<double, 2> load_vec2(gcptr<double> base, long long s)
{
    const f64x2 q = *(gcptr<f64x2>)(base + s);
    return Vec<double, 2>{{q.x, q.y}};
}
// Stores of a pass's outputs: streaming (nontemporal), since nothing reads
// them again within the pass; this keeps L2 for the halo lines.
__device__ __forceinline__ void store_vec2(gptr<float> base, long long s, const Vec<float, 2> &q)
{
    f32x2 v;
    v.x = q.v[0];
    v.y = q.v[1];
    __builtin_nontemporal_store(v, (gptr<f32x2>)(base + s));
}
__device__ __forceinline__ void store_vec2(gptr<double> base, long long s, const Vec<double, 2> &q)
{
    f64x2 v;
    v.x = q.v[0];
    v.y = q.v[1];
    __builtin_nontemporal_store(v, (gptr<f64x2>)(base + s));
}

// Cache-policy bits of a buffer store on gfx950: sc0 (1) | nt (2) | sc1 (16).
constexpr int kStreamPolicy = 1 | 2 | 16;

__device__ __forceinline__ Quad<float> load_quad(gcptr<float> base, long long s)
{
    const f32x4 q = *(gcptr<f32x4>)(base + s);
    return Quad<float>{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ Quad<double> load_quad(gcptr<double> base, long long s)
{
    const f64x2 a = *(gcptr<f64x2>)(base + s);
    const f64x2 b = *(gcptr<f64x2>)(base + s + 2);
    return Quad<double>{{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ void store_quad(gptr<float> base, long long s, const Quad<float> &q)
{
    f32x4 v;
    v.x = q.v[0];
    v.y = q.v[1];
    v.z = q.v[2];
    v.w = q.v[3];
    __builtin_nontemporal_store(v, (gptr<f32x4>)(base + s));
}
// Streaming store of 4 FP32 values at element s of a plane whose base is the
// same in every lane (s < 2^29): a buffer store with system scope and the
// nontemporal hint (sc0 sc1 nt), the policy for data written once and not
// read again by the same kernel; measured, it leaves more of L2 to the halo
// rows other tiles still have to read.  Results are those of store_quad;
// only the cache policy differs.
__device__ __forceinline__ void store_quad_stream(gptr<float> plane, unsigned s, const Quad<float> &q)
{
    typedef float f4_t __attribute__((ext_vector_type(4)));
    f4_t v;
    v.x = q.v[0];
    v.y = q.v[1];
    v.z = q.v[2];
    v.w = q.v[3];
    // raw buffer: stride 0, num_records in bytes, gfx9 dword3 (32-bit data)
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)plane, (short)0, 0x7ffffff0, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)(s * 4u), 0, kStreamPolicy);
}
__device__ __forceinline__ void store_quad(gptr<double> base, long long s, const Quad<double> &q)
{
    f64x2 a, b;
    a.x = q.v[0];
    a.y = q.v[1];
    b.x = q.v[2];
    b.y = q.v[3];
    __builtin_nontemporal_store(a, (gptr<f64x2>)(base + s));
    __builtin_nontemporal_store(b, (gptr<f64x2>)(base + s + 2));
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Per-field coefficients of one pass, in the storage type.
template <typename T>
struct FieldCoef {
    T beta;  // deferred c-term coefficient
    T bm;    // beta * m, rounded once
    T r;     // reference derivative
    T m1;    // reference field at n+1, rounded once (potential only)
};

// Derivative at n+1/2 and drifted deviation at n+1.  The one definition used
// for a site's own value and for every neighbour value, so both are bitwise
// identical.
template <typename T>
__device__ __forceinline__ T fdot_of(T d, T p, const FieldCoef<T> &c)
{
    return fma_t(c.beta, d, p) + c.bm;
}
template <typename T>
__device__ __forceinline__ T drift(T d, T p, const FieldCoef<T> &c, T dt)
{
    return fma_t(dt, fdot_of(d, p, c) - c.r, d);
}

// Value of `v` held by the lane below / above (whole-wave DPP shift by one;
// lane 0 / lane 63 receive 0).
__device__ __forceinline__ float lane_from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Work item of the j-th round of block b in a persistent grid of `grid`
// blocks over `nitems` items, -1 when done.  The hardware places block b on
// XCD b mod 8; when the grid and the item count are multiples of 8, each XCD
// takes one contiguous eighth of the items (neighbouring items share that
// XCD's L2), else items go round robin.
__device__ __forceinline__ long long xcd_item(int b, int j, int grid, long long nitems)
{
    if ((grid & 7) == 0 && (nitems & 7) == 0) {
        const long long per = nitems >> 3;
        const long long idx = (long long)(b >> 3) + (long long)j * (grid >> 3);
        return idx < per ? (long long)(b & 7) * per + idx : -1;
    }
    const long long t = (long long)b + (long long)j * grid;
    return t < nitems ? t : -1;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum acc[0..NQ) over the block (blockDim.x a multiple of 64, red holding
// one row per wave); the totals land in red[0][q].  Fixed order.
template <int NQ>
__device__ __forceinline__ void block_sum(double (&acc)[NQ], double (*red)[kMaxSums])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; q++) red[wave][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double s = red[0][threadIdx.x];
        for (int w = 1; w < nwaves; w++) s += red[w][threadIdx.x];
        red[0][threadIdx.x] = s;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ double round_to_storage(double v)
{
    return (double)(T)v;
}

// a^k for an integer k (|k| <= 8), by repeated multiplication or division.
__device__ __forceinline__ double int_power(double a, int k)
{
    double r = 1.0;
    for (int j = 0; j < k; j++) r *= a;
    for (int j = 0; j < -k; j++) r /= a;
    return r;
}

template <typename T>
__device__ __forceinline__ void fill_pass_scalars(PassScalars<T> &ps, const Scalars *sc, const Lattice &lat,
                                                  double a1)
{
    const double a2 = a1 * a1;
    ps.beta = (T)sc->beta;
    for (int i = 0; i < kMaxFields; i++) {
        const bool on = i < lat.nf;
        ps.bm[i] = on ? (T)(sc->beta * sc->m[i]) : (T)0;
        ps.r[i] = on ? (T)sc->r[i] : (T)0;
        ps.m1[i] = on ? (T)sc->nx_m1[i] : (T)0;
        ps.m2a[i] = on ? (T)(a2 * lat.mu2[i]) : (T)0;
        ps.hm[i] = on ? (T)(0.5 * a2 * lat.mu2[i]) : (T)0;
    }
    // a term of degree D of the physical potential is coef a^(4 - D) in the
    // program variables
    for (int t = 0; t < kMaxTerms; t++)
        ps.tc[t] = t < lat.nterms ? (T)(lat.tcoef[t] * int_power(a1, 4 - lat.tdeg[t])) : (T)0;
}

// Derive the next step pass's coefficients from the scalar state (one thread).
__device__ __forceinline__ void publish_next_pass(const Lattice &lat, Scalars *sc)
{
#pragma clang fp contract(off)
    const double a2 = sc->a_next * sc->a_next;
    for (int i = 0; i < kMaxFields; i++) {
        const bool on = i < lat.nf;
        sc->nx_m1[i] = on ? sc->m[i] + lat.dt * sc->r[i] : 0.0;
        sc->nx_hm[i] = on ? 0.5 * a2 * lat.mu2[i] : 0.0;
    }
    fill_pass_scalars(sc->nxf, sc, lat, sc->a_next);
    fill_pass_scalars(sc->nxd, sc, lat, sc->a_next);
}

// FP64 tail after a step pass n -> n+1 (one thread).  Sums of field i at
// 6i: sum d, sum d^2, sum d Lap d, sum ubar^2, sum ubar, sum ubar d, all at
// n+1, with ubar = (fdot^{n+1/2} + p^{n+3/2})/2; last: sum V.
template <typename T>
__device__ __forceinline__ void step_tail(const Lattice &lat, const double *tot)
{
#pragma clang fp contract(off)
    Scalars *sc = lat.sc;
    const double Ns = (double)lat.nsites;
    const double dt = lat.dt;
    const double a1 = sc->a_next;
    const double y = sc->adot_half;
    double m1[kMaxFields], sumf2[kMaxFields], gsum = 0.0;
    ce_energy e;
    for (int i = 0; i < kMaxFields; i++) {
        e.kin[i] = e.grad[i] = e.mean[i] = e.mean_sq[i] = 0.0;
        if (i >= lat.nf) continue;
        const double *t = tot + kSumsPerField * i;
        m1[i] = sc->m[i] + dt * sc->r[i];
        sumf2[i] = Ns * m1[i] * m1[i] + 2.0 * m1[i] * t[0] + t[1];
        e.mean[i] = m1[i] + t[0] / Ns;
        e.mean_sq[i] = sumf2[i] / Ns;
        e.grad[i] = -0.5 * t[2] / Ns;
        gsum += e.grad[i];
    }
    // mean comoving potential at n+1, with the vacuum term a^4 V0
    const double a1sq = a1 * a1;
    const double V = tot[kSumsPerField * lat.nf] / Ns + a1sq * a1sq * lat.vacuum;
    double x = 0.0, abar = 0.0, c = 0.0;
    if (lat.expansion) {
        // a'^{n+3/2} from the time-centred kick of a' (quadratic in x; the
        // root continuous with a'^{n+1/2}, written without cancellation)
        const double S = lat.kappa * (2.0 / 3.0 * gsum + V) / a1;
        const double A = dt / (4.0 * a1);
        const double B = 1.0 + dt * y / (2.0 * a1);
        const double C = dt * y * y / (4.0 * a1) - y - dt * S;
        x = -2.0 * C / (B + sqrt(B * B - 4.0 * A * C));
        abar = 0.5 * (x + y);
        c = (S - abar * abar / a1) / a1;
    }
    const double beta1 = dt * c;
    // kinetic energy of u = (fdot^{n+1/2} + fdot^{n+3/2})/2 - (abar/a) f
    //                     = ubar + eta f,  eta = dt c/2 - abar/a
    const double eta = 0.5 * dt * c - abar / a1;
    double rho = V;
    int bad = 0;
    for (int i = 0; i < lat.nf; i++) {
        const double *t = tot + kSumsPerField * i;
        const double sum_uf = m1[i] * t[4] + t[5];
        e.kin[i] = 0.5 * (t[3] + 2.0 * eta * sum_uf + eta * eta * sumf2[i]) / Ns;
        rho += e.kin[i] + e.grad[i];
        // mean of fdot^{n+3/2} = mean p^{n+3/2} + beta_{n+1} mean f^{n+1},
        // mean p^{n+3/2} = 2 mean ubar - mean fdot^{n+1/2}
        const double fm = 2.0 * t[4] / Ns - sc->fdot_mean[i] + beta1 * e.mean[i];
        sc->m[i] = m1[i];
        sc->fdot_mean[i] = fm;
        sc->r[i] = round_to_storage<T>(fm);
    }
    for (int q = 0; q <= kSumsPerField * lat.nf; q++) bad |= !isfinite(tot[q]);
    bad |= !isfinite(x) || !isfinite(c);
    e.step = sc->step + 1;
    e.tau = sc->tau + dt;
    e.a = a1;
    e.adot = abar;
    e.hubble = abar / (a1 * a1);
    e.pot = V;
    e.rho = rho;
    e.friedmann_residual =
        (lat.expansion && abar != 0.0) ? (abar * abar - lat.kappa * rho / 3.0) / (abar * abar) : 0.0;
    e.nonfinite = bad;
    e.pad_ = 0;
    lat.ring[e.step % kLogCap] = e;

    sc->a = a1;
    sc->a_next = lat.expansion ? a1 + dt * x : 1.0;
    sc->adot_half = x;
    sc->beta = beta1;
    sc->tau = e.tau;
    sc->step = e.step;
    sc->cur ^= 1;
    if (sc->remaining > 0) sc->remaining -= 1;
    if (bad && sc->first_bad < 0) sc->first_bad = e.step;
    publish_next_pass(lat, sc);
}

// FP64 tail of the start-up pass.  Sums of field i at 6i: sum d, sum d^2,
// sum d Lap d, sum fdot(0)^2, sum p^{1/2}, (unused); last: sum V at a = 1.
template <typename T>
__device__ __forceinline__ void init_tail(const Lattice &lat, const double *tot)
{
#pragma clang fp contract(off)
    Scalars *sc = lat.sc;
    const double Ns = (double)lat.nsites;
    const double dt = lat.dt;
    ce_energy e;
    double gsum = 0.0, rho = 0.0;
    for (int i = 0; i < kMaxFields; i++) {
        e.kin[i] = e.grad[i] = e.mean[i] = e.mean_sq[i] = 0.0;
        if (i >= lat.nf) continue;
        const double *t = tot + kSumsPerField * i;
        const double m = sc->m[i];
        e.kin[i] = 0.5 * t[3] / Ns;
        e.grad[i] = -0.5 * t[2] / Ns;
        e.mean[i] = m + t[0] / Ns;
        e.mean_sq[i] = (Ns * m * m + 2.0 * m * t[0] + t[1]) / Ns;
        gsum += e.grad[i];
        rho += e.kin[i] + e.grad[i];
    }
    const double V = tot[kSumsPerField * lat.nf] / Ns + lat.vacuum;  // a = 1
    rho += V;
    double ap0 = 0.0, app0 = 0.0;
    if (lat.expansion) {
        ap0 = sqrt(lat.kappa * rho / 3.0);
        app0 = -ap0 * ap0 + lat.kappa * (2.0 / 3.0 * gsum + V);
    }
    const double aph = ap0 + 0.5 * dt * app0;
    // fdot^{1/2} = fdot(0) + a'(0) f + dt/2 (Lap f - V' + a''(0) f): the stored
    // half kick omits the two f terms, beta_0 = a'(0) + dt/2 a''(0).
    const double beta0 = aph;
    int bad = 0;
    for (int i = 0; i < lat.nf; i++) {
        const double fm = tot[kSumsPerField * i + 4] / Ns + beta0 * e.mean[i];
        sc->fdot_mean[i] = fm;
        sc->r[i] = round_to_storage<T>(fm);
    }
    for (int q = 0; q <= kSumsPerField * lat.nf; q++) bad |= !isfinite(tot[q]);
    bad |= !isfinite(ap0);   // a negative energy density cannot start an expanding run
    e.step = 0;
    e.tau = 0.0;
    e.a = 1.0;
    e.adot = ap0;
    e.hubble = ap0;
    e.pot = V;
    e.rho = rho;
    e.friedmann_residual =
        (lat.expansion && ap0 != 0.0) ? (ap0 * ap0 - lat.kappa * rho / 3.0) / (ap0 * ap0) : 0.0;
    e.nonfinite = bad;
    e.pad_ = 0;
    lat.ring[0] = e;
    sc->a = 1.0;
    sc->adot_half = aph;
    sc->a_next = lat.expansion ? 1.0 + dt * aph : 1.0;
    sc->beta = beta0;
    sc->tau = 0.0;
    sc->step = 0;
    sc->first_bad = bad ? 0 : -1;
    publish_next_pass(lat, sc);
}

// Partial sum q of block or tile `row`: one column per sum, so that the
// last block's reads of a column by consecutive threads are contiguous.
__device__ __forceinline__ double *partial_at(const Lattice &lat, int q, long long row)
{
    return lat.partials + (long long)q * lat.slots + row;
}

// Last-block reduction of the partial sums in a fixed order, then the FP64
// tail.  Every block calls this after writing its partials.  The `grid`
// blocks (this lattice's share of the launch) wrote `rows` rows of partials
// between them (one per block, or one per tile); the block that takes the
// last ticket reduces them in row order and clears the tile counters for the
// next launch (every other block has finished taking tiles by then).
//
// Ordering: the barrier completes the block's partial stores; the ticket
// increment is a release at agent scope (the L2 of this XCD writes back, no
// invalidate), so only the block that takes the last ticket pays an acquire,
// whose L2 invalidate would otherwise evict the halos that the other blocks
// on its XCD are about to re-read.
//
// Each thread sums rows threadIdx.x, + blockDim.x, ... in that order; with
// R > 1 it loads R of them before adding them, so R rows' loads are in
// flight at once (the sums, and so the result, are the same for every R).
template <typename T, int NQ, int MODE, int R = 1>
__device__ __forceinline__ void finish_pass(const Lattice &lat, int grid, int rows, double (*red)[kMaxSums])
{
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int t = __hip_atomic_fetch_add(lat.ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int last = t == (unsigned int)(grid - 1);
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;
    const int stride = (int)blockDim.x;
    int b = threadIdx.x;
    if constexpr (R > 1) {
        for (; b + (R - 1) * stride < rows; b += R * stride) {
            double v[R][NQ];
#pragma unroll
            for (int r = 0; r < R; r++) {
#pragma unroll
                for (int q = 0; q < NQ; q++)
                    v[r][q] = __hip_atomic_load(partial_at(lat, q, b + r * stride), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (int r = 0; r < R; r++)
#pragma unroll
                for (int q = 0; q < NQ; q++) acc[q] += v[r][q];
        }
    }
    for (; b < rows; b += stride) {
#pragma unroll
        for (int q = 0; q < NQ; q++)
            acc[q] += __hip_atomic_load(partial_at(lat, q, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<NQ>(acc, red);
    if (threadIdx.x == 0) {
        double tot[kMaxSums];
        for (int q = 0; q < NQ; q++) tot[q] = red[0][q];
        if (MODE == kStep)
            step_tail<T>(lat, tot);
        else
            init_tail<T>(lat, tot);
        __hip_atomic_store(lat.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int i = 1; i <= kTileCounters; i++)
            __hip_atomic_store(lat.ticket + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}


// All coefficients of one pass, computed once per thread from the lattice
// description and the FP64 scalar state.
template <typename T, int NF>
struct PassCoef {
    T dt, inv_dx2, lam, kick;
    T G[NF], m2a[NF];
    FieldCoef<T> cf[NF];
    T qlam;              // lambda / 4
    T hG[NF];            // G_j / 2
    T hm[NF];            // a^2 mu2_i / 2 at the kick
    bool has_mass;
    // polynomial model: terms of degree >= 1, scaled coefficients and exponents
    int nterms;
    T tc[kMaxTerms];
    int texp[kMaxTerms][NF];
};

__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Every coefficient is the same in all lanes; keep them in scalar registers.
template <typename T, int NF>
__device__ __forceinline__ void make_uniform(PassCoef<T, NF> &c)
{
    c.dt = uniform(c.dt);
    c.inv_dx2 = uniform(c.inv_dx2);
    c.lam = uniform(c.lam);
    c.kick = uniform(c.kick);
    c.qlam = uniform(c.qlam);
#pragma unroll
    for (int i = 0; i < NF; i++) {
        c.G[i] = uniform(c.G[i]);
        c.m2a[i] = uniform(c.m2a[i]);
        c.cf[i].beta = uniform(c.cf[i].beta);
        c.cf[i].bm = uniform(c.cf[i].bm);
        c.cf[i].r = uniform(c.cf[i].r);
        c.cf[i].m1 = uniform(c.cf[i].m1);
        c.hG[i] = uniform(c.hG[i]);
        c.hm[i] = uniform(c.hm[i]);
    }
    c.has_mass = __builtin_amdgcn_readfirstlane((int)c.has_mass) != 0;
}

template <typename T>
__device__ __forceinline__ T static_coef(double d, float f)
{
    if constexpr (sizeof(T) == 4)
        return f;
    else
        return d;
}

template <typename T>
using cscalars = const __attribute__((address_space(4))) Scalars *;

template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) PassScalars<T> &pass_scalars(cscalars<T> s)
{
    if constexpr (sizeof(T) == 4)
        return s->nxf;
    else
        return s->nxd;
}

// Coefficients of a pass.  A step pass reads the ones the previous tail
// published (scalar loads: the values are the same for every lane and this
// kernel writes them only after every block has read them); the start-up pass
// derives its own (beta = 0, a = 1, m unchanged).
template <typename T, int NF, int MODEL, int MODE>
__device__ __forceinline__ PassCoef<T, NF> make_coef(const Lattice &lat)
{
    PassCoef<T, NF> c;
    if constexpr (MODEL == kPoly) {
        c.nterms = __builtin_amdgcn_readfirstlane(lat.nterms);
        for (int t = 0; t < kMaxTerms; t++)
#pragma unroll
            for (int i = 0; i < NF; i++) c.texp[t][i] = __builtin_amdgcn_readfirstlane(lat.texp[t][i]);
        if (MODE == kStep) {
            const auto &ps = pass_scalars<T>((cscalars<T>)lat.sc);
            for (int t = 0; t < kMaxTerms; t++) c.tc[t] = ps.tc[t];
        } else {
            for (int t = 0; t < kMaxTerms; t++) c.tc[t] = uniform((T)lat.tcoef[t]);  // a = 1
        }
    }
    c.dt = static_coef<T>(lat.dt, lat.dt_f);
    c.inv_dx2 = static_coef<T>(lat.inv_dx2, lat.inv_dx2_f);
    c.lam = static_coef<T>(lat.lambda, lat.lambda_f);
    c.qlam = static_coef<T>(0.25 * lat.lambda, lat.qlam_f);
    c.has_mass = false;
#pragma unroll
    for (int i = 0; i < NF; i++) {
        c.G[i] = static_coef<T>(lat.G[i], lat.G_f[i]);
        c.hG[i] = static_coef<T>(0.5 * lat.G[i], lat.hG_f[i]);
        c.has_mass |= lat.mu2[i] != 0.0;
    }
    if (MODE == kStep) {
        const cscalars<T> cs = (cscalars<T>)lat.sc;
        const auto &ps = pass_scalars<T>(cs);
        c.kick = c.dt;
#pragma unroll
        for (int i = 0; i < NF; i++) {
            c.m2a[i] = ps.m2a[i];
            c.cf[i].beta = ps.beta;
            c.cf[i].bm = ps.bm[i];
            c.cf[i].r = ps.r[i];
            c.cf[i].m1 = ps.m1[i];
            c.hm[i] = ps.hm[i];
        }
    } else {
        const Scalars *sc = lat.sc;
        c.kick = (T)(0.5 * lat.dt);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            c.m2a[i] = (T)lat.mu2[i];
            c.hm[i] = (T)(0.5 * lat.mu2[i]);
            const double m = sc->m[i];
            c.cf[i].beta = (T)0;
            c.cf[i].bm = (T)0;
            c.cf[i].r = (T)0;
            c.cf[i].m1 = (T)m;
        }
        make_uniform(c);
    }
    return c;
}

// Own-site derivative at n+1/2 and deviation at n+1 (kInit: unchanged).
template <typename T, int NF, int MODE>
__device__ __forceinline__ void own_drift(const PassCoef<T, NF> &c, int i, T d, T p, T &fdot, T &d1)
{
    if (MODE == kStep) {
        fdot = fdot_of(d, p, c.cf[i]);
        d1 = fma_t(c.dt, fdot - c.cf[i].r, d);
    } else {
        fdot = p;
        d1 = d;
    }
}

// Neighbour deviation at n+1 (same arithmetic as own_drift).
template <typename T, int NF, int MODE>
__device__ __forceinline__ T nbr_drift(const PassCoef<T, NF> &c, int i, T d, T p)
{
    return (MODE == kStep) ? drift(d, p, c.cf[i], c.dt) : d;
}

// One site: potential derivative and kick, plus the site's terms of the
// volume sums added into `part` (storage type).
//   d1[i]   deviation of field i at n+1,  fdot[i] derivative at n+1/2,
//   lap[i]  Laplacian of d1 at the site;  pn[i] receives the new stored
//   derivative.  Every kernel calls this, so all kernels round alike.
// With FP32 storage the per-site terms are formed in FP32 and a thread adds
// its few sites in FP32 before folding them into its FP64 accumulators
// (flush_sums); with FP64 storage everything is FP64.
// Polynomial model at one site: V = sum_t tc_t prod_i v_i^e_ti and
// dV/dv_i = sum_t tc_t (d v_i^e_ti / dv_i) prod_{j != i} v_j^e_tj.  Powers
// come from repeated multiplication, the derivative of v^e alongside by the
// product rule ((v^k)' v + v^k = (v^(k+1))'), so no exponent is ever a
// floating-point factor.  Exponents and coefficients are uniform.
template <typename T, int NF>
__device__ __forceinline__ void poly_potential(const PassCoef<T, NF> &c, const T (&v)[NF], T &V, T (&dV)[NF])
{
    V = (T)0;
#pragma unroll
    for (int i = 0; i < NF; i++) dV[i] = (T)0;
    // unrolled over the term slots, so every table index is a constant and
    // the tables stay in scalar registers
#pragma unroll
    for (int t = 0; t < kMaxTerms; t++) {
        if (t >= c.nterms) break;
        T pw[NF], dpw[NF];
#pragma unroll
        for (int i = 0; i < NF; i++) {
            T x = (T)1, dx = (T)0;
            for (int k = 0; k < c.texp[t][i]; k++) {
                dx = fma_t(dx, v[i], x);
                x = x * v[i];
            }
            pw[i] = x;
            dpw[i] = dx;
        }
        T mono = pw[0];
#pragma unroll
        for (int i = 1; i < NF; i++) mono = mono * pw[i];
        V = fma_t(c.tc[t], mono, V);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            T prod = dpw[i];
#pragma unroll
            for (int j = 0; j < NF; j++)
                if (j != i) prod = prod * pw[j];
            dV[i] = fma_t(c.tc[t], prod, dV[i]);
        }
    }
}

template <typename T, int NF, int MODEL, int MODE, int NQ>
__device__ __forceinline__ void site_update(const PassCoef<T, NF> &c, const T (&d1)[NF], const T (&fdot)[NF],
                                            const T (&lap)[NF], T (&pn)[NF], T (&part)[NQ])
{
    if constexpr (MODEL == kPoly) {
        T v[NF], dV[NF], Vs;
#pragma unroll
        for (int i = 0; i < NF; i++) v[i] = c.cf[i].m1 + d1[i];
        poly_potential<T, NF>(c, v, Vs, dV);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            pn[i] = fma_t(c.kick, lap[i] - dV[i], fdot[i]);
            const T dd = d1[i];
            T *a = part + kSumsPerField * i;
            a[0] += dd;
            a[1] = fma_t(dd, dd, a[1]);
            a[2] = fma_t(dd, lap[i], a[2]);
            if (MODE == kStep) {
                const T ub = (T)0.5 * (fdot[i] + pn[i]);
                a[3] = fma_t(ub, ub, a[3]);
                a[4] += ub;
                a[5] = fma_t(ub, dd, a[5]);
            } else {
                a[3] = fma_t(fdot[i], fdot[i], a[3]);
                a[4] += pn[i];
            }
        }
        part[kSumsPerField * NF] += Vs;
        return;
    }
    T v[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) v[i] = c.cf[i].m1 + d1[i];
    T chi2 = (T)0;
#pragma unroll
    for (int j = 1; j < NF; j++) chi2 = fma_t(c.G[j] * v[j], v[j], chi2);
    const T v0sq = v[0] * v[0];
    T Vs = (c.qlam * v0sq) * v0sq;
#pragma unroll
    for (int i = 0; i < NF; i++) {
        T dV = (i == 0) ? fma_t(c.lam * v0sq, v[0], v[0] * chi2) : (c.G[i] * v0sq) * v[i];
        dV = fma_t(c.m2a[i], v[i], dV);
        pn[i] = fma_t(c.kick, lap[i] - dV, fdot[i]);
        const T dd = d1[i];
        T *a = part + kSumsPerField * i;
        a[0] += dd;
        a[1] = fma_t(dd, dd, a[1]);
        a[2] = fma_t(dd, lap[i], a[2]);
        if (MODE == kStep) {
            const T ub = (T)0.5 * (fdot[i] + pn[i]);
            a[3] = fma_t(ub, ub, a[3]);
            a[4] += ub;
            a[5] = fma_t(ub, dd, a[5]);
        } else {
            a[3] = fma_t(fdot[i], fdot[i], a[3]);
            a[4] += pn[i];
        }
        const T vsq = v[i] * v[i];
        if (i > 0) Vs = fma_t(c.hG[i] * v0sq, vsq, Vs);
        if (c.has_mass) Vs = fma_t(c.hm[i], vsq, Vs);
    }
    part[kSumsPerField * NF] += Vs;
}

template <typename T, int NQ>
__device__ __forceinline__ void clear_part(T (&part)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; q++) part[q] = (T)0;
}

template <typename T, int NQ>
__device__ __forceinline__ void flush_sums(const T (&part)[NQ], double (&acc)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] += (double)part[q];
}

}  // namespace dev
}  // namespace ce
