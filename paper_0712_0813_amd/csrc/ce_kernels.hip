// Generic (1-, 2-, 3-D) fused leapfrog pass, FP64 volume sums and the FP64
// scale-factor tail, plus the conversion and readback kernels.
//
// One pass advances every site by one step of the staggered leapfrog of the
// paper's "Parallel Algorithms" section: a drift of f by dt from the
// half-step derivative, then a kick of the derivative from the new f.
//
// Two exact rewritings of the state shape the kernels:
//  * Deferred c-term.  The kick at step n+1 needs c = a''/a at n+1, which
//    depends on volume means of f^{n+1}.  The kick is stored without the term
//    dt c^{n+1} f^{n+1}; the stored array p holds fdot - beta f, and each pass
//    first rebuilds fdot^{n+1/2} = p + beta_n f^n with the beta_n the previous
//    pass's tail computed.  The start-up pass folds a'(0) f + dt/2 a''(0) f
//    into beta_0.  Without expansion beta == 0.
//  * Homogeneous split.  f_i = m_i + d_i with the reference m_i an FP64
//    scalar and only the deviation d_i stored.  m_i moves with the FP64 mean
//    derivative r_i; d_i drifts with fdot - r_i.  The Laplacian sees only d_i,
//    so FP32 storage of a field sitting near 1 with 1e-3 fluctuations keeps
//    the fluctuations' full precision instead of losing it to the cancellation
//    f(x+e) + f(x-e) - 2 f(x) amplified by 1/dx^2.
#include <math.h>

#include "ce_internal.hpp"

namespace ce {

namespace {

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
__device__ void step_tail(const Lattice &lat, const double *tot)
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
__device__ void init_tail(const Lattice &lat, const double *tot)
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

template <typename T, int D, int NF, int MODE>
__global__ __launch_bounds__(kBlock) void pass_kernel(Lattice lat, int src)
{
    constexpr int NQ = kSumsPerField * NF + 1;
    __shared__ double red[kBlock / 64][kMaxSums];

    const int N = lat.N;
    const long long nquads = lat.nsites / 4;
    const T dt = (T)lat.dt;
    const T inv_dx2 = (T)lat.inv_dx2;
    const T lam = (T)lat.lambda;
    const Scalars *sc = lat.sc;
    const double a_kick = (MODE == kStep) ? sc->a_next : 1.0;
    const T kick = (MODE == kStep) ? dt : (T)(0.5 * lat.dt);
    const double beta = (MODE == kStep) ? sc->beta : 0.0;
    T G[NF], m2a[NF];
    FieldCoef<T> cf[NF];
    double m1d[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) {
        G[i] = (T)lat.G[i];
        m2a[i] = (T)(a_kick * a_kick * lat.mu2[i]);
        const double m = sc->m[i];
        m1d[i] = (MODE == kStep) ? m + lat.dt * sc->r[i] : m;
        cf[i].beta = (T)beta;
        cf[i].bm = (T)(beta * m);
        cf[i].r = (MODE == kStep) ? (T)sc->r[i] : (T)0;
        cf[i].m1 = (T)m1d[i];
    }
    const double a2d = a_kick * a_kick;

    const T *din[NF];
    const T *pin[NF];
    T *dout[NF];
    T *pout[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) {
        din[i] = static_cast<const T *>(lat.d[src][i]);
        pin[i] = static_cast<const T *>(lat.p[src][i]);
        dout[i] = static_cast<T *>(lat.d[src ^ 1][i]);
        pout[i] = static_cast<T *>(lat.p[src ^ 1][i]);
    }

    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;

    const long long stride = (long long)gridDim.x * kBlock;
    for (long long qd = (long long)blockIdx.x * kBlock + threadIdx.x; qd < nquads; qd += stride) {
        const long long s = qd * 4;
        const int x0 = (int)(s % N);
        const long long row = s / N;
        const long long rowbase = s - x0;
        const long long sl = rowbase + (x0 == 0 ? N - 1 : x0 - 1);
        const long long sr = rowbase + (x0 + 4 == N ? 0 : x0 + 4);
        long long sy[2] = {0, 0}, sz[2] = {0, 0};
        if (D >= 2) {
            const int y = (int)(row % N);
            sy[0] = s + (long long)((y == N - 1) ? -(N - 1) : 1) * N;
            sy[1] = s + (long long)((y == 0) ? (N - 1) : -1) * N;
        }
        if (D == 3) {
            const long long NN = (long long)N * N;
            const int z = (int)(row / N);
            sz[0] = s + (long long)((z == N - 1) ? -(N - 1) : 1) * NN;
            sz[1] = s + (long long)((z == 0) ? (N - 1) : -1) * NN;
        }

        T d1[NF][4], fdot[NF][4], lap[NF][4];
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const Quad<T> dc = load_quad(din[i], s);
            const Quad<T> pc = load_quad(pin[i], s);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if (MODE == kStep) {
                    fdot[i][e] = fdot_of(dc.v[e], pc.v[e], cf[i]);
                    d1[i][e] = fma_t(dt, fdot[i][e] - cf[i].r, dc.v[e]);
                } else {
                    fdot[i][e] = pc.v[e];
                    d1[i][e] = dc.v[e];
                }
            }
            T dl, dr;
            if (MODE == kStep) {
                dl = drift(din[i][sl], pin[i][sl], cf[i], dt);
                dr = drift(din[i][sr], pin[i][sr], cf[i], dt);
            } else {
                dl = din[i][sl];
                dr = din[i][sr];
            }
            T acc_l[4];
            acc_l[0] = (dl + d1[i][1]) - (T)2 * d1[i][0];
            acc_l[1] = (d1[i][0] + d1[i][2]) - (T)2 * d1[i][1];
            acc_l[2] = (d1[i][1] + d1[i][3]) - (T)2 * d1[i][2];
            acc_l[3] = (d1[i][2] + dr) - (T)2 * d1[i][3];
            if (D >= 2) {
                const Quad<T> da = load_quad(din[i], sy[0]), db = load_quad(din[i], sy[1]);
                const Quad<T> pa = load_quad(pin[i], sy[0]), pb = load_quad(pin[i], sy[1]);
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    T ya = (MODE == kStep) ? drift(da.v[e], pa.v[e], cf[i], dt) : da.v[e];
                    T yb = (MODE == kStep) ? drift(db.v[e], pb.v[e], cf[i], dt) : db.v[e];
                    acc_l[e] += (ya + yb) - (T)2 * d1[i][e];
                }
            }
            if (D == 3) {
                const Quad<T> da = load_quad(din[i], sz[0]), db = load_quad(din[i], sz[1]);
                const Quad<T> pa = load_quad(pin[i], sz[0]), pb = load_quad(pin[i], sz[1]);
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    T za = (MODE == kStep) ? drift(da.v[e], pa.v[e], cf[i], dt) : da.v[e];
                    T zb = (MODE == kStep) ? drift(db.v[e], pb.v[e], cf[i], dt) : db.v[e];
                    acc_l[e] += (za + zb) - (T)2 * d1[i][e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; e++) lap[i][e] = acc_l[e] * inv_dx2;
        }

        // potential derivative, kick and FP64 sums
        T pn[NF][4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            T v[NF];
            double vd[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) {
                v[i] = cf[i].m1 + d1[i][e];
                vd[i] = m1d[i] + (double)d1[i][e];
            }
            T chi2 = (T)0;
#pragma unroll
            for (int j = 1; j < NF; j++) chi2 = fma_t(G[j] * v[j], v[j], chi2);
            const T v0sq = v[0] * v[0];
            const double v0sqd = vd[0] * vd[0];
            double Vd = 0.25 * lat.lambda * v0sqd * v0sqd;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                T dV = (i == 0) ? lam * v0sq * v[0] + v[0] * chi2 : G[i] * v0sq * v[i];
                dV = fma_t(m2a[i], v[i], dV);
                pn[i][e] = fma_t(kick, lap[i][e] - dV, fdot[i][e]);
                const double dd = (double)d1[i][e];
                double *a = acc + kSumsPerField * i;
                a[0] += dd;
                a[1] += dd * dd;
                a[2] += dd * (double)lap[i][e];
                if (MODE == kStep) {
                    const double ub = 0.5 * ((double)fdot[i][e] + (double)pn[i][e]);
                    a[3] += ub * ub;
                    a[4] += ub;
                    a[5] += ub * dd;
                } else {
                    const double pd = (double)fdot[i][e];
                    a[3] += pd * pd;
                    a[4] += (double)pn[i][e];
                }
                if (i > 0) Vd += 0.5 * lat.G[i] * v0sqd * vd[i] * vd[i];
                Vd += 0.5 * a2d * lat.mu2[i] * vd[i] * vd[i];
            }
            acc[kSumsPerField * NF] += Vd;
        }
#pragma unroll
        for (int i = 0; i < NF; i++) {
            Quad<T> po;
#pragma unroll
            for (int e = 0; e < 4; e++) po.v[e] = pn[i][e];
            if (MODE == kStep) {
                Quad<T> dq;
#pragma unroll
                for (int e = 0; e < 4; e++) dq.v[e] = d1[i][e];
                store_quad(dout[i], s, dq);
                store_quad(pout[i], s, po);
            } else {
                // start-up: the derivative is updated in place, d is unchanged
                store_quad(const_cast<T *>(pin[i]), s, po);
            }
        }
    }

    block_sum<NQ>(acc, red);
    if (threadIdx.x < NQ) lat.partials[(long long)blockIdx.x * kMaxSums + threadIdx.x] = red[0][threadIdx.x];
    finish_pass<T, NQ, MODE>(lat, red);
}

template <typename T, int D, int NF>
hipError_t launch_typed(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    dim3 grid(lat.nblocks), block(kBlock);
    if (mode == kStep)
        hipLaunchKernelGGL((pass_kernel<T, D, NF, kStep>), grid, block, 0, st, lat, src);
    else
        hipLaunchKernelGGL((pass_kernel<T, D, NF, kInit>), grid, block, 0, st, lat, src);
    return hipGetLastError();
}

template <typename T, int D>
hipError_t launch_nf(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.nf) {
    case 1: return launch_typed<T, D, 1>(lat, src, mode, st);
    case 2: return launch_typed<T, D, 2>(lat, src, mode, st);
    case 3: return launch_typed<T, D, 3>(lat, src, mode, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_dims(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.dims) {
    case 1: return launch_nf<T, 1>(lat, src, mode, st);
    case 2: return launch_nf<T, 2>(lat, src, mode, st);
    case 3: return launch_nf<T, 3>(lat, src, mode, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void convert_kernel(const double *src, double ref, T *dst, long long n,
                                                        unsigned int *maxabs_bits)
{
    __shared__ float red[kBlock / 64];
    float m = 0.0f;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const double v = src[i];
        dst[i] = (T)(v - ref);
        m = fmaxf(m, (float)fabs(v));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = red[0];
        for (int w = 1; w < kBlock / 64; w++) b = fmaxf(b, red[w]);
        // non-negative floats order like their bit patterns (NaN sorts high)
        atomicMax(maxabs_bits, __float_as_uint(b));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void readback_kernel(const T *d, const T *p, const Scalars *sc, int field,
                                                         int started, long long first,
                                                         const long long *sites, long long n,
                                                         double *out_f, double *out_fdot)
{
    const double m = sc->m[field];
    FieldCoef<T> c;
    const double beta = started ? sc->beta : 0.0;
    c.beta = (T)beta;
    c.bm = (T)(beta * m);
    c.r = (T)0;
    c.m1 = (T)0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const long long k = sites ? sites[i] : first + i;
        const T dv = d[k];
        if (out_f) out_f[i] = m + (double)dv;
        if (out_fdot) out_fdot[i] = started ? (double)fdot_of(dv, p[k], c) : (double)p[k];
    }
}

int grid_for(long long n)
{
    long long b = (n + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

int pass_blocks(int dims, int N)
{
    long long ns = 1;
    for (int d = 0; d < dims; d++) ns *= N;
    long long b = (ns / 4 + kBlock - 1) / kBlock;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_pass(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    if (precision == CE_FP64) return launch_dims<double>(lat, src, mode, st);
    return launch_dims<float>(lat, src, mode, st);
}

hipError_t launch_convert(const double *src, double ref, void *dst, int precision, long long n,
                          unsigned int *maxabs_bits, hipStream_t st)
{
    dim3 grid(grid_for(n)), block(kBlock);
    if (precision == CE_FP64)
        hipLaunchKernelGGL(convert_kernel<double>, grid, block, 0, st, src, ref, static_cast<double *>(dst), n,
                           maxabs_bits);
    else
        hipLaunchKernelGGL(convert_kernel<float>, grid, block, 0, st, src, ref, static_cast<float *>(dst), n,
                           maxabs_bits);
    return hipGetLastError();
}

hipError_t launch_readback(const Lattice &lat, int precision, int buf, int field, int started,
                           long long first, const long long *sites, long long n, double *out_f,
                           double *out_fdot, hipStream_t st)
{
    dim3 grid(grid_for(n)), block(kBlock);
    if (precision == CE_FP64)
        hipLaunchKernelGGL(readback_kernel<double>, grid, block, 0, st,
                           static_cast<const double *>(lat.d[buf][field]),
                           static_cast<const double *>(lat.p[buf][field]), lat.sc, field, started, first,
                           sites, n, out_f, out_fdot);
    else
        hipLaunchKernelGGL(readback_kernel<float>, grid, block, 0, st,
                           static_cast<const float *>(lat.d[buf][field]),
                           static_cast<const float *>(lat.p[buf][field]), lat.sc, field, started, first,
                           sites, n, out_f, out_fdot);
    return hipGetLastError();
}

}  // namespace ce
