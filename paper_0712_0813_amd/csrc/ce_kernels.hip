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

#include "ce_device.hpp"

#ifndef CE_UNIT_MODEL
#error "compile this file once per model, with -DCE_UNIT_MODEL=0 and -DCE_UNIT_MODEL=1"
#endif

namespace ce {

namespace {

using namespace dev;

// Body of the direct pass: block b of the `grid` blocks this lattice gets.
template <typename T, int D, int NF, int MODEL, int MODE>
__device__ __forceinline__ void pass_body(const Lattice &lat, int src, int b, int grid)
{
    constexpr int NQ = kSumsPerField * NF + 1;
    __shared__ double red[kBlock / 64][kMaxSums];

    const int N = lat.N;
    const long long nquads = lat.nsites / 4;
    const PassCoef<T, NF> c = make_coef<T, NF, MODEL, MODE>(lat);

    gcptr<T> din[NF];
    gcptr<T> pin[NF];
    gptr<T> dout[NF];
    gptr<T> pout[NF];
#pragma unroll
    for (int i = 0; i < NF; i++) {
        din[i] = as_global<T>(lat.d[src][i]);
        pin[i] = as_global<T>(lat.p[src][i]);
        dout[i] = as_global<T>(lat.d[src ^ 1][i]);
        pout[i] = as_global<T>(lat.p[src ^ 1][i]);
    }

    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;

    const long long stride = (long long)grid * kBlock;
    for (long long qd = (long long)b * kBlock + threadIdx.x; qd < nquads; qd += stride) {
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

        T d1[4][NF], fdot[4][NF], lap[4][NF];
#pragma unroll
        for (int i = 0; i < NF; i++) {
            const Quad<T> dc = load_quad(din[i], s);
            const Quad<T> pc = load_quad(pin[i], s);
#pragma unroll
            for (int e = 0; e < 4; e++) own_drift<T, NF, MODE>(c, i, dc.v[e], pc.v[e], fdot[e][i], d1[e][i]);
            const T dl = nbr_drift<T, NF, MODE>(c, i, din[i][sl], pin[i][sl]);
            const T dr = nbr_drift<T, NF, MODE>(c, i, din[i][sr], pin[i][sr]);
            T pair[4];
            pair[0] = dl + d1[1][i];
            pair[1] = d1[0][i] + d1[2][i];
            pair[2] = d1[1][i] + d1[3][i];
            pair[3] = d1[2][i] + dr;
            if (D >= 2) {
                const Quad<T> da = load_quad(din[i], sy[0]), db = load_quad(din[i], sy[1]);
                const Quad<T> pa = load_quad(pin[i], sy[0]), pb = load_quad(pin[i], sy[1]);
#pragma unroll
                for (int e = 0; e < 4; e++)
                    pair[e] += nbr_drift<T, NF, MODE>(c, i, da.v[e], pa.v[e]) +
                               nbr_drift<T, NF, MODE>(c, i, db.v[e], pb.v[e]);
            }
            if (D == 3) {
                const Quad<T> da = load_quad(din[i], sz[0]), db = load_quad(din[i], sz[1]);
                const Quad<T> pa = load_quad(pin[i], sz[0]), pb = load_quad(pin[i], sz[1]);
#pragma unroll
                for (int e = 0; e < 4; e++)
                    pair[e] += nbr_drift<T, NF, MODE>(c, i, da.v[e], pa.v[e]) +
                               nbr_drift<T, NF, MODE>(c, i, db.v[e], pb.v[e]);
            }
#pragma unroll
            for (int e = 0; e < 4; e++) lap[e][i] = fma_t((T)(-2 * D), d1[e][i], pair[e]) * c.inv_dx2;
        }

        T pn[4][NF];
        T part[NQ];
        clear_part(part);
#pragma unroll
        for (int e = 0; e < 4; e++) site_update<T, NF, MODEL, MODE, NQ>(c, d1[e], fdot[e], lap[e], pn[e], part);
        flush_sums(part, acc);
#pragma unroll
        for (int i = 0; i < NF; i++) {
            Quad<T> po;
#pragma unroll
            for (int e = 0; e < 4; e++) po.v[e] = pn[e][i];
            if (MODE == kStep) {
                Quad<T> dq;
#pragma unroll
                for (int e = 0; e < 4; e++) dq.v[e] = d1[e][i];
                store_quad(dout[i], s, dq);
                store_quad(pout[i], s, po);
            } else {
                // start-up: the derivative is updated in place, d is unchanged
                store_quad(as_global<T>(lat.p[src][i]), s, po);
            }
        }
    }

    block_sum<NQ>(acc, red);
    if (threadIdx.x < NQ) *partial_at(lat, threadIdx.x, b) = red[0][threadIdx.x];
    finish_pass<T, NQ, MODE>(lat, grid, grid, red);
}

template <typename T, int D, int NF, int MODEL, int MODE>
__global__ __launch_bounds__(kBlock) void pass_kernel(Lattice lat, int src)
{
    pass_body<T, D, NF, MODEL, MODE>(lat, src, blockIdx.x, gridDim.x);
}

// Step pass over many lattices: block -> (lattice, its own block index), so
// every lattice's blocks and reduction order are those of a lone launch.
template <typename T, int D, int NF, int MODEL>
__global__ __launch_bounds__(kBlock) void pass_batched(const Lattice *lats, const int *blk_lat, int total)
{
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const int l = __builtin_amdgcn_readfirstlane(blk_lat[v]);
        const Lattice &lat = *(const Lattice *)((const __attribute__((address_space(4))) Lattice *)lats + l);
        if (lat.sc->remaining <= 0) continue;
        const int src = lat.sc->cur;
        pass_body<T, D, NF, MODEL, kStep>(lat, src, v - lat.first_block, lat.nblocks);
    }
}

template <typename T, int D, int NF, int MODEL>
hipError_t launch_typed(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    dim3 grid(lat.nblocks), block(kBlock);
    if (mode == kStep)
        hipLaunchKernelGGL((pass_kernel<T, D, NF, MODEL, kStep>), grid, block, 0, st, lat, src);
    else
        hipLaunchKernelGGL((pass_kernel<T, D, NF, MODEL, kInit>), grid, block, 0, st, lat, src);
    return hipGetLastError();
}

template <typename T, int D, int MODEL>
hipError_t launch_nf(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.nf) {
    case 1: return launch_typed<T, D, 1, MODEL>(lat, src, mode, st);
    case 2: return launch_typed<T, D, 2, MODEL>(lat, src, mode, st);
    case 3: return launch_typed<T, D, 3, MODEL>(lat, src, mode, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODEL>
hipError_t launch_dims(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.dims) {
    case 1: return launch_nf<T, 1, MODEL>(lat, src, mode, st);
    case 2: return launch_nf<T, 2, MODEL>(lat, src, mode, st);
    case 3: return launch_nf<T, 3, MODEL>(lat, src, mode, st);
    default: return hipErrorInvalidValue;
    }
}

// Step budgets of a class's lattices for the coming block (pool quotas).
__global__ __launch_bounds__(kBlock) void set_remaining_kernel(const Lattice *lats, const long long *vals, int n)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l < n) lats[l].sc->remaining = vals[l];
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
        // NaN counts as +inf so that the maximum reports it
        m = fmaxf(m, isnan(v) ? INFINITY : (float)fabs(v));
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

template <typename T, int D, int MODEL>
hipError_t batched_nf(const Lattice *lats, const int *blk_lat, int total, int grid, int nf, hipStream_t st)
{
    const dim3 g(grid), b(kBlock);
    switch (nf) {
    case 1: hipLaunchKernelGGL((pass_batched<T, D, 1, MODEL>), g, b, 0, st, lats, blk_lat, total); break;
    case 2: hipLaunchKernelGGL((pass_batched<T, D, 2, MODEL>), g, b, 0, st, lats, blk_lat, total); break;
    case 3: hipLaunchKernelGGL((pass_batched<T, D, 3, MODEL>), g, b, 0, st, lats, blk_lat, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MODEL>
hipError_t batched_dims(const Lattice *lats, const int *blk_lat, int total, int grid, int dims, int nf,
                        hipStream_t st)
{
    switch (dims) {
    case 1: return batched_nf<T, 1, MODEL>(lats, blk_lat, total, grid, nf, st);
    case 2: return batched_nf<T, 2, MODEL>(lats, blk_lat, total, grid, nf, st);
    case 3: return batched_nf<T, 3, MODEL>(lats, blk_lat, total, grid, nf, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int D, int MODEL>
int resident_nf(int nf)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (nf) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pass_batched<T, D, 1, MODEL>, kBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pass_batched<T, D, 2, MODEL>, kBlock, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pass_batched<T, D, 3, MODEL>, kBlock, 0); break;
    default: break;
    }
    return e == hipSuccess ? n : 0;
}

template <typename T, int MODEL>
int resident_dims(int dims, int nf)
{
    switch (dims) {
    case 1: return resident_nf<T, 1, MODEL>(nf);
    case 2: return resident_nf<T, 2, MODEL>(nf);
    case 3: return resident_nf<T, 3, MODEL>(nf);
    default: return 0;
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

// This unit's model (the source is compiled once per model).
constexpr int kUnit = CE_UNIT_MODEL;

template <>
hipError_t launch_direct_model<kUnit>(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    if (precision == CE_FP64) return launch_dims<double, kUnit>(lat, src, mode, st);
    return launch_dims<float, kUnit>(lat, src, mode, st);
}

template <>
hipError_t launch_batched_direct_model<kUnit>(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                              const Lattice &proto, int precision, hipStream_t st)
{
    if (precision == CE_FP64)
        return batched_dims<double, kUnit>(lats, blk_lat, total_blocks, grid, proto.dims, proto.nf, st);
    return batched_dims<float, kUnit>(lats, blk_lat, total_blocks, grid, proto.dims, proto.nf, st);
}

template <>
int direct_batched_resident_model<kUnit>(const Lattice &proto, int precision)
{
    return precision == CE_FP64 ? resident_dims<double, kUnit>(proto.dims, proto.nf)
                                : resident_dims<float, kUnit>(proto.dims, proto.nf);
}

#if CE_UNIT_MODEL == CE_MODEL_QUARTIC
// Model-independent functions, and the dispatch on the kernel family, then
// on the model, live in the quartic unit.

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
    if (lat.kind == kTiled3d) return launch_tiled(lat, precision, src, mode, st);
    if (lat.kind == kStream2d) return launch_stream2d(lat, precision, src, mode, st);
    return lat.model == kPoly ? launch_direct_model<kPoly>(lat, precision, src, mode, st)
                              : launch_direct_model<kQuartic>(lat, precision, src, mode, st);
}

hipError_t launch_batched(const Lattice *lats, const int *blk_lat, int total_blocks, int grid, const Lattice &proto,
                          int precision, hipStream_t st)
{
    if (grid < 1 || grid > total_blocks) return hipErrorInvalidValue;
    if (proto.kind == kTiled3d) return launch_batched_tiled(lats, blk_lat, total_blocks, grid, proto, precision, st);
    if (proto.kind == kStream2d)
        return launch_batched_stream2d(lats, blk_lat, total_blocks, grid, proto, precision, st);
    return proto.model == kPoly
               ? launch_batched_direct_model<kPoly>(lats, blk_lat, total_blocks, grid, proto, precision, st)
               : launch_batched_direct_model<kQuartic>(lats, blk_lat, total_blocks, grid, proto, precision, st);
}

int batched_resident_blocks(const Lattice &proto, int precision)
{
    if (proto.kind == kTiled3d) return tiled_batched_resident(proto, precision);
    if (proto.kind == kStream2d) return stream2d_batched_resident(proto, precision);
    return proto.model == kPoly ? direct_batched_resident_model<kPoly>(proto, precision)
                                : direct_batched_resident_model<kQuartic>(proto, precision);
}

hipError_t launch_set_remaining(const Lattice *lats, const long long *vals, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_remaining_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, lats, vals, n);
    return hipGetLastError();
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

#endif  // CE_UNIT_MODEL == CE_MODEL_QUARTIC

}  // namespace ce
