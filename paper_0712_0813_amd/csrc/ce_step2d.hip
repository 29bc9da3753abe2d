// Streaming 2-D leapfrog pass for gfx950.
//
// The lattice is cut into units of one 256-site x segment by `rows`
// consecutive y rows.  Each wavefront works one unit at a time: every lane
// owns 4 consecutive x sites (128-bit loads), walks the unit's rows and keeps
// the drifted deviation of rows y-1, y and y+1 in registers (the y
// neighbours).  x neighbours come from the adjacent lane by a whole-wave DPP
// shift; the two edge lanes of the wave fetch the site beyond the segment
// themselves (a cache hit: it is the neighbouring segment's data).  No LDS and
// no barrier in the row loop.  The four waves of a block take four
// consecutive units, and blocks walk groups of units in the XCD-contiguous
// order of the 3-D pass.  Sums and tail are shared with the other passes.
#include "ce_device.hpp"

#ifndef CE_UNIT_MODEL
#error "compile this file once per model, with -DCE_UNIT_MODEL=0 and -DCE_UNIT_MODEL=1"
#endif

namespace ce {
namespace {

using namespace dev;

constexpr int kSeg = 256;       // x sites per unit
constexpr int kVec = 4;         // x sites per lane
constexpr int kWaves = kBlock / 64;

// Store of one lane's 4 sites of a row whose base is uniform: streaming
// buffer store for FP32 (see store_quad_stream), plain nontemporal for FP64.
template <typename T>
__device__ __forceinline__ void store_row(gptr<T> row, unsigned x, const Quad<T> &q)
{
    if constexpr (sizeof(T) == 4)
        store_quad_stream(row, x, q);
    else
        store_quad(row, x, q);
}

template <typename T, int NF, int MODEL, int MODE>
__device__ __forceinline__ void stream2d_body(const Lattice &lat, int src, int b, int grid)
{
    constexpr int NQ = kSumsPerField * NF + 1;
    __shared__ double red[kWaves][kMaxSums];

    const int N = lat.N;
    const int rows = lat.zc;
    const int nseg = N / kSeg;
    const long long units = (long long)nseg * (N / rows);
    const long long ngroups = (units + kWaves - 1) / kWaves;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
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
    const bool left_edge = lane == 0, right_edge = lane == 63;

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; k++) acc[k] = 0.0;

    for (int j = 0;; j++) {
        const long long g = xcd_item(b, j, grid, ngroups);
        if (g < 0) break;
        const long long u = g * kWaves + wave;
        if (u >= units) continue;
        const int seg = (int)(u % nseg);
        const int y0 = (int)(u / nseg) * rows;
        const int x0 = seg * kSeg;
        const unsigned own_x = (unsigned)(x0 + kVec * lane);
        // the site beyond the segment edge that this lane needs, if any
        const unsigned edge_x = left_edge ? (unsigned)((x0 + N - 1) % N) : (unsigned)((x0 + kSeg) % N);
        const bool edge = left_edge || right_edge;

        T dm[NF][kVec], dcur[NF][kVec], fcur[NF][kVec], ecur[NF];
        {
            const long long base = (long long)((y0 + N - 1) % N) * N;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const Quad<T> dq = load_quad(din[i] + base, own_x);
                const Quad<T> pq = load_quad(pin[i] + base, own_x);
#pragma unroll
                for (int e = 0; e < kVec; e++) dm[i][e] = nbr_drift<T, NF, MODE>(c, i, dq.v[e], pq.v[e]);
            }
        }
        {
            const long long base = (long long)y0 * N;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const Quad<T> dq = load_quad(din[i] + base, own_x);
                const Quad<T> pq = load_quad(pin[i] + base, own_x);
#pragma unroll
                for (int e = 0; e < kVec; e++) own_drift<T, NF, MODE>(c, i, dq.v[e], pq.v[e], fcur[i][e], dcur[i][e]);
                ecur[i] = edge ? nbr_drift<T, NF, MODE>(c, i, (din[i] + base)[edge_x], (pin[i] + base)[edge_x]) : (T)0;
            }
        }
        // stored values of row y+1, loaded one iteration ahead of their use
        Quad<T> rd[NF], rp[NF];
        T red[NF], rep[NF];
        {
            const long long base = (long long)((y0 + 1) % N) * N;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                rd[i] = load_quad(din[i] + base, own_x);
                rp[i] = load_quad(pin[i] + base, own_x);
                red[i] = edge ? (din[i] + base)[edge_x] : (T)0;
                rep[i] = edge ? (pin[i] + base)[edge_x] : (T)0;
            }
        }
        for (int k = 0; k < rows; k++) {
            const int y = y0 + k;
            // issue the loads of row y+2 before working on row y
            Quad<T> qd[NF], qp[NF];
            T qed[NF], qep[NF];
            if (k + 1 < rows) {
                const long long qbase = (long long)((y + 2) % N) * N;
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    qd[i] = load_quad(din[i] + qbase, own_x);
                    qp[i] = load_quad(pin[i] + qbase, own_x);
                    qed[i] = edge ? (din[i] + qbase)[edge_x] : (T)0;
                    qep[i] = edge ? (pin[i] + qbase)[edge_x] : (T)0;
                }
            } else {
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    qd[i] = rd[i];
                    qp[i] = rp[i];
                    qed[i] = red[i];
                    qep[i] = rep[i];
                }
            }
            T pair[NF][kVec];
#pragma unroll
            for (int i = 0; i < NF; i++) {
                T xl = lane_from_left(dcur[i][kVec - 1]);
                T xr = lane_from_right(dcur[i][0]);
                if (left_edge) xl = ecur[i];
                if (right_edge) xr = ecur[i];
#pragma unroll
                for (int e = 0; e < kVec; e++) {
                    const T l = e == 0 ? xl : dcur[i][e - 1];
                    const T r = e == kVec - 1 ? xr : dcur[i][e + 1];
                    pair[i][e] = l + r;
                }
            }
            T dn1[NF][kVec], fn1[NF][kVec], en1[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) {
#pragma unroll
                for (int e = 0; e < kVec; e++) own_drift<T, NF, MODE>(c, i, rd[i].v[e], rp[i].v[e], fn1[i][e], dn1[i][e]);
                en1[i] = edge ? nbr_drift<T, NF, MODE>(c, i, red[i], rep[i]) : (T)0;
            }
            const long long obase = (long long)y * N;
            T part[NQ];
            clear_part(part);
#pragma unroll
            for (int e = 0; e < kVec; e++) {
                T d1s[NF], fds[NF], lap[NF], pn[NF];
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    const T pr = pair[i][e] + (dn1[i][e] + dm[i][e]);
                    lap[i] = fma_t((T)-4, dcur[i][e], pr) * c.inv_dx2;
                    d1s[i] = dcur[i][e];
                    fds[i] = fcur[i][e];
                }
                site_update<T, NF, MODEL, MODE, NQ>(c, d1s, fds, lap, pn, part);
#pragma unroll
                for (int i = 0; i < NF; i++) fcur[i][e] = pn[i];
            }
            flush_sums(part, acc);
#pragma unroll
            for (int i = 0; i < NF; i++) {
                Quad<T> dq, pq;
#pragma unroll
                for (int e = 0; e < kVec; e++) {
                    dq.v[e] = dcur[i][e];
                    pq.v[e] = fcur[i][e];
                }
                if (MODE == kStep) {
                    store_row(dout[i] + obase, own_x, dq);
                    store_row(pout[i] + obase, own_x, pq);
                } else {
                    store_row(as_global<T>(lat.p[src][i]) + obase, own_x, pq);
                }
#pragma unroll
                for (int e = 0; e < kVec; e++) {
                    dm[i][e] = dcur[i][e];
                    dcur[i][e] = dn1[i][e];
                    fcur[i][e] = fn1[i][e];
                }
                ecur[i] = en1[i];
                rd[i] = qd[i];
                rp[i] = qp[i];
                red[i] = qed[i];
                rep[i] = qep[i];
            }
        }
    }

    block_sum<NQ>(acc, red);
    if (threadIdx.x < NQ) *partial_at(lat, threadIdx.x, b) = red[0][threadIdx.x];
    finish_pass<T, NQ, MODE>(lat, grid, grid, red);
}

template <typename T, int NF, int MODEL, int MODE>
__global__ __launch_bounds__(kBlock) void stream2d_kernel(Lattice lat, int src)
{
    stream2d_body<T, NF, MODEL, MODE>(lat, src, blockIdx.x, gridDim.x);
}

template <typename T, int NF, int MODEL>
__global__ __launch_bounds__(kBlock) void stream2d_batched(const Lattice *lats, const int *blk_lat, int total)
{
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const int l = __builtin_amdgcn_readfirstlane(blk_lat[v]);
        const Lattice &lat = *(const Lattice *)((const __attribute__((address_space(4))) Lattice *)lats + l);
        if (lat.sc->remaining <= 0) continue;
        const int src = lat.sc->cur;
        stream2d_body<T, NF, MODEL, kStep>(lat, src, v - lat.first_block, lat.nblocks);
    }
}

template <typename T, int MODEL>
hipError_t launch_t(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    const dim3 grid(lat.nblocks), block(kBlock);
    switch (lat.nf * 2 + (mode == kInit)) {
    case 2: hipLaunchKernelGGL((stream2d_kernel<T, 1, MODEL, kStep>), grid, block, 0, st, lat, src); break;
    case 3: hipLaunchKernelGGL((stream2d_kernel<T, 1, MODEL, kInit>), grid, block, 0, st, lat, src); break;
    case 4: hipLaunchKernelGGL((stream2d_kernel<T, 2, MODEL, kStep>), grid, block, 0, st, lat, src); break;
    case 5: hipLaunchKernelGGL((stream2d_kernel<T, 2, MODEL, kInit>), grid, block, 0, st, lat, src); break;
    case 6: hipLaunchKernelGGL((stream2d_kernel<T, 3, MODEL, kStep>), grid, block, 0, st, lat, src); break;
    case 7: hipLaunchKernelGGL((stream2d_kernel<T, 3, MODEL, kInit>), grid, block, 0, st, lat, src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MODEL>
hipError_t batched_t(const Lattice *lats, const int *blk_lat, int total, int grid, int nf, hipStream_t st)
{
    const dim3 g(grid), b(kBlock);
    switch (nf) {
    case 1: hipLaunchKernelGGL((stream2d_batched<T, 1, MODEL>), g, b, 0, st, lats, blk_lat, total); break;
    case 2: hipLaunchKernelGGL((stream2d_batched<T, 2, MODEL>), g, b, 0, st, lats, blk_lat, total); break;
    case 3: hipLaunchKernelGGL((stream2d_batched<T, 3, MODEL>), g, b, 0, st, lats, blk_lat, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int MODEL>
int resident_batched_t(int nf)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (nf) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream2d_batched<T, 1, MODEL>, kBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream2d_batched<T, 2, MODEL>, kBlock, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream2d_batched<T, 3, MODEL>, kBlock, 0); break;
    default: break;
    }
    return e == hipSuccess ? n : 0;
}

}  // namespace

// This unit's model (the source is compiled once per model).
constexpr int kUnit = CE_UNIT_MODEL;

template <>
hipError_t launch_stream2d_model<kUnit>(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    if (precision == CE_FP64) return launch_t<double, kUnit>(lat, src, mode, st);
    return launch_t<float, kUnit>(lat, src, mode, st);
}

template <>
hipError_t launch_batched_stream2d_model<kUnit>(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                                const Lattice &proto, int precision, hipStream_t st)
{
    if (precision == CE_FP64) return batched_t<double, kUnit>(lats, blk_lat, total_blocks, grid, proto.nf, st);
    return batched_t<float, kUnit>(lats, blk_lat, total_blocks, grid, proto.nf, st);
}

template <>
int stream2d_batched_resident_model<kUnit>(const Lattice &proto, int precision)
{
    return precision == CE_FP64 ? resident_batched_t<double, kUnit>(proto.nf)
                                : resident_batched_t<float, kUnit>(proto.nf);
}

#if CE_UNIT_MODEL == CE_MODEL_QUARTIC
bool stream2d_fits(int dims, int N, int rows)
{
    return dims == 2 && N % kSeg == 0 && rows >= 1 && N % rows == 0;
}

long long stream2d_groups(int N, int rows)
{
    const long long units = (long long)(N / kSeg) * (N / rows);
    return (units + kWaves - 1) / kWaves;
}

int stream2d_resident_blocks()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream2d_kernel<float, 3, kQuartic, kStep>, kBlock, 0) != hipSuccess)
        return 0;
    return n;
}

hipError_t launch_stream2d(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    return lat.model == kPoly ? launch_stream2d_model<kPoly>(lat, precision, src, mode, st)
                              : launch_stream2d_model<kQuartic>(lat, precision, src, mode, st);
}

hipError_t launch_batched_stream2d(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                   const Lattice &proto, int precision, hipStream_t st)
{
    return proto.model == kPoly
               ? launch_batched_stream2d_model<kPoly>(lats, blk_lat, total_blocks, grid, proto, precision, st)
               : launch_batched_stream2d_model<kQuartic>(lats, blk_lat, total_blocks, grid, proto, precision, st);
}

int stream2d_batched_resident(const Lattice &proto, int precision)
{
    return proto.model == kPoly ? stream2d_batched_resident_model<kPoly>(proto, precision)
                                : stream2d_batched_resident_model<kQuartic>(proto, precision);
}
#endif  // CE_UNIT_MODEL == CE_MODEL_QUARTIC

}  // namespace ce
