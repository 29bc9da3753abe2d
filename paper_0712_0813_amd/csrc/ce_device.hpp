// Device helpers shared by the lattice kernels: vector loads, the one
// definition of the drift, FP64 block sums, and the FP64 tails that turn the
// volume sums of a pass into the scale-factor update and the diagnostics.
#pragma once

#include <math.h>

#include "ce_internal.hpp"

namespace ce {
namespace dev {

template <typename T>
struct Quad {
    T v[4];
};

__device__ __forceinline__ Quad<float> load_quad(const float *base, long long s)
{
    float4 q = *reinterpret_cast<const float4 *>(base + s);
    return Quad<float>{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ Quad<double> load_quad(const double *base, long long s)
{
    double2 a = *reinterpret_cast<const double2 *>(base + s);
    double2 b = *reinterpret_cast<const double2 *>(base + s + 2);
    return Quad<double>{{a.x, a.y, b.x, b.y}};
}
__device__ __forceinline__ void store_quad(float *base, long long s, const Quad<float> &q)
{
    *reinterpret_cast<float4 *>(base + s) = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
}
__device__ __forceinline__ void store_quad(double *base, long long s, const Quad<double> &q)
{
    *reinterpret_cast<double2 *>(base + s) = make_double2(q.v[0], q.v[1]);
    *reinterpret_cast<double2 *>(base + s + 2) = make_double2(q.v[2], q.v[3]);
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

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum acc[0..NQ) over the block; the totals land in red[0][q].
template <int NQ>
__device__ __forceinline__ void block_sum(double (&acc)[NQ], double (*red)[kMaxSums])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = wave_sum(acc[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; q++) red[wave][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double s = red[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; w++) s += red[w][threadIdx.x];
        red[0][threadIdx.x] = s;
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ double round_to_storage(double v)
{
    return (double)(T)v;
}

// FP64 tail after a step pass n -> n+1 (one thread).  Sums of field i at
// 6i: sum d, sum d^2, sum d Lap d, sum ubar^2, sum ubar, sum ubar d, all at
// n+1, with ubar = (fdot^{n+1/2} + p^{n+3/2})/2; last: sum V.
template <typename T>
__device__ __noinline__ void step_tail(const Lattice &lat, const double *tot)
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
    const double V = tot[kSumsPerField * lat.nf] / Ns;
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
    if (bad && sc->first_bad < 0) sc->first_bad = e.step;
}

// FP64 tail of the start-up pass.  Sums of field i at 6i: sum d, sum d^2,
// sum d Lap d, sum fdot(0)^2, sum p^{1/2}, (unused); last: sum V at a = 1.
template <typename T>
__device__ __noinline__ void init_tail(const Lattice &lat, const double *tot)
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
    const double V = tot[kSumsPerField * lat.nf] / Ns;
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
}

// Last-block reduction of the per-block partial sums in a fixed order, then
// the FP64 tail.  Every block calls this after writing its partials.
template <typename T, int NQ, int MODE>
__device__ __forceinline__ void finish_pass(const Lattice &lat, double (*red)[kMaxSums])
{
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int t = atomicAdd(lat.ticket, 1u);
        s_last = (t == (unsigned int)(gridDim.x - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
        const double *row = lat.partials + (long long)b * kMaxSums;
#pragma unroll
        for (int q = 0; q < NQ; q++)
            acc[q] += __hip_atomic_load(row + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    }
}


// All coefficients of one pass, computed once per thread from the lattice
// description and the FP64 scalar state.
template <typename T, int NF>
struct PassCoef {
    T dt, inv_dx2, lam, kick;
    T G[NF], m2a[NF];
    FieldCoef<T> cf[NF];
    double m1d[NF];      // FP64 reference field at n+1
    double qlam_d;       // lambda / 4
    double hG_d[NF];     // G_j / 2
    double hm_d[NF];     // a^2 mu2_i / 2 at the kick
    bool has_mass;
};

template <typename T, int NF, int MODE>
__device__ __forceinline__ PassCoef<T, NF> make_coef(const Lattice &lat)
{
    PassCoef<T, NF> c;
    const Scalars *sc = lat.sc;
    c.dt = (T)lat.dt;
    c.inv_dx2 = (T)lat.inv_dx2;
    c.lam = (T)lat.lambda;
    c.qlam_d = 0.25 * lat.lambda;
    const double a_kick = (MODE == kStep) ? sc->a_next : 1.0;
    c.kick = (MODE == kStep) ? c.dt : (T)(0.5 * lat.dt);
    const double beta = (MODE == kStep) ? sc->beta : 0.0;
    const double a2 = a_kick * a_kick;
    c.has_mass = false;
#pragma unroll
    for (int i = 0; i < NF; i++) {
        c.G[i] = (T)lat.G[i];
        c.hG_d[i] = 0.5 * lat.G[i];
        c.hm_d[i] = 0.5 * a2 * lat.mu2[i];
        c.has_mass |= lat.mu2[i] != 0.0;
        c.m2a[i] = (T)(a2 * lat.mu2[i]);
        const double m = sc->m[i];
        c.m1d[i] = (MODE == kStep) ? m + lat.dt * sc->r[i] : m;
        c.cf[i].beta = (T)beta;
        c.cf[i].bm = (T)(beta * m);
        c.cf[i].r = (MODE == kStep) ? (T)sc->r[i] : (T)0;
        c.cf[i].m1 = (T)c.m1d[i];
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

// One site: potential derivative, kick, and the FP64 volume sums.
//   d1[i]   deviation of field i at n+1,  fdot[i] derivative at n+1/2,
//   lap[i]  Laplacian of d1 at the site;  pn[i] receives the new stored
//   derivative.  Every kernel calls this, so all kernels round alike.
template <typename T, int NF, int MODE, int NQ>
__device__ __forceinline__ void site_update(const PassCoef<T, NF> &c, const T (&d1)[NF], const T (&fdot)[NF],
                                            const T (&lap)[NF], T (&pn)[NF], double (&acc)[NQ])
{
    T v[NF];
    double vd[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) {
        v[i] = c.cf[i].m1 + d1[i];
        vd[i] = c.m1d[i] + (double)d1[i];
    }
    T chi2 = (T)0;
#pragma unroll
    for (int j = 1; j < NF; j++) chi2 = fma_t(c.G[j] * v[j], v[j], chi2);
    const T v0sq = v[0] * v[0];
    const double v0sqd = vd[0] * vd[0];
    double Vd = (c.qlam_d * v0sqd) * v0sqd;
#pragma unroll
    for (int i = 0; i < NF; i++) {
        T dV = (i == 0) ? fma_t(c.lam * v0sq, v[0], v[0] * chi2) : (c.G[i] * v0sq) * v[i];
        dV = fma_t(c.m2a[i], v[i], dV);
        pn[i] = fma_t(c.kick, lap[i] - dV, fdot[i]);
        const double dd = (double)d1[i];
        double *a = acc + kSumsPerField * i;
        a[0] += dd;
        a[1] = fma_t(dd, dd, a[1]);
        a[2] = fma_t(dd, (double)lap[i], a[2]);
        if (MODE == kStep) {
            const double ub = 0.5 * ((double)fdot[i] + (double)pn[i]);
            a[3] = fma_t(ub, ub, a[3]);
            a[4] += ub;
            a[5] = fma_t(ub, dd, a[5]);
        } else {
            const double pd = (double)fdot[i];
            a[3] = fma_t(pd, pd, a[3]);
            a[4] += (double)pn[i];
        }
        const double vsq = vd[i] * vd[i];
        if (i > 0) Vd = fma_t(c.hG_d[i] * v0sqd, vsq, Vd);
        if (c.has_mass) Vd = fma_t(c.hm_d[i], vsq, Vd);
    }
    acc[kSumsPerField * NF] += Vd;
}

}  // namespace dev
}  // namespace ce
