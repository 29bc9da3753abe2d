// Tiled 3-D leapfrog pass for gfx950: z-streaming with an LDS plane tile.
//
// A 256-thread block owns an (x, y) tile of 4*LPR x 256/LPR sites and walks
// `zc` consecutive z planes.  Each thread owns one quad of 4 consecutive x
// sites (128-bit loads of every array).  Per plane it loads its quad of d and
// p once, drifts it, and keeps the drifted deviation for planes z-1, z, z+1 in
// registers (the z neighbours).  The drifted plane also goes to a
// triple-buffered LDS tile, with a one-site halo ring filled by four groups of
// threads; y neighbours are read from LDS, x neighbours come from the adjacent
// lane by a DPP row shift, and the tile's edge lanes take the halo column.
// With three LDS buffers one barrier per plane suffices.  Only the halo ring
// and the two extra planes per tile are read twice, from cache.
//
// The grid is persistent: each block walks tiles, and the tiles are numbered
// so that the blocks the hardware places on one XCD (block ids equal mod 8)
// work on one contiguous slab, keeping y halos in that XCD's L2.  The FP64
// volume sums and the scale-factor tail are those of the direct pass.
#include "ce_device.hpp"

namespace ce {
namespace {

using namespace dev;

__device__ __forceinline__ float lane_from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x111, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x101, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void lds_store_quad(float *p, const float (&v)[4])
{
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void lds_store_quad(double *p, const double (&v)[4])
{
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}
__device__ __forceinline__ Quad<float> lds_load_quad(const float *p)
{
    const float4 q = *reinterpret_cast<const float4 *>(p);
    return Quad<float>{{q.x, q.y, q.z, q.w}};
}
__device__ __forceinline__ Quad<double> lds_load_quad(const double *p)
{
    const double2 a = reinterpret_cast<const double2 *>(p)[0];
    const double2 b = reinterpret_cast<const double2 *>(p)[1];
    return Quad<double>{{a.x, a.y, b.x, b.y}};
}

// Tile number for the j-th tile of block b: XCD-contiguous when the grid and
// the tile count are multiples of 8, else plain round robin.  -1 when done.
__device__ __forceinline__ long long tile_of(int b, int j, int grid, long long ntiles)
{
    if ((grid & 7) == 0 && (ntiles & 7) == 0) {
        const long long per = ntiles >> 3;
        const long long idx = (long long)(b >> 3) + (long long)j * (grid >> 3);
        return idx < per ? (long long)(b & 7) * per + idx : -1;
    }
    const long long t = (long long)b + (long long)j * grid;
    return t < ntiles ? t : -1;
}

template <typename T, int NF, int MODE, int LPR>
__global__ __launch_bounds__(kBlock) void tiled3d_kernel(Lattice lat, int src)
{
    constexpr int NQ = kSumsPerField * NF + 1;
    constexpr int TX = 4 * LPR;
    constexpr int TY = kBlock / LPR;
    constexpr int PLANE = (TY + 2) * TX;
    constexpr int FSTRIDE = PLANE + 2 * TY;  // plane with halo rows, then left/right columns
    __shared__ __align__(16) T lds[3][NF][FSTRIDE];
    __shared__ double red[kBlock / 64][kMaxSums];

    const int N = lat.N;
    const int zc = lat.zc;
    const int ntx = N / TX, nty = N / TY;
    const long long ntiles = (long long)ntx * nty * (N / zc);
    const int t = threadIdx.x;
    const int q = t % LPR;  // own quad within the tile row
    const int y = t / LPR;  // own row within the tile
    const PassCoef<T, NF> c = make_coef<T, NF, MODE>(lat);

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

    // halo duties: one group of threads per side of the ring
    const bool top = t < LPR;                              // row y0-1, quad t
    const bool bottom = t >= 64 && t < 64 + LPR;           // row y0+TY, quad t-64
    const bool left = t >= 128 && t < 128 + TY;            // column x0-1, row t-128
    const bool right = t >= 192 && t < 192 + TY;           // column x0+TX, row t-192

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; k++) acc[k] = 0.0;

    const long long NN = (long long)N * N;
    for (int j = 0;; j++) {
        const long long tile = tile_of(blockIdx.x, j, gridDim.x, ntiles);
        if (tile < 0) break;
        const int tx = (int)(tile % ntx);
        const int ty = (int)((tile / ntx) % nty);
        const int z0 = (int)(tile / ((long long)ntx * nty)) * zc;
        const int x0 = tx * TX, y0 = ty * TY;
        const long long own_xy = (long long)(y0 + y) * N + x0 + 4 * q;
        long long halo_xy = 0;
        if (top) halo_xy = (long long)((y0 + N - 1) % N) * N + x0 + 4 * t;
        if (bottom) halo_xy = (long long)((y0 + TY) % N) * N + x0 + 4 * (t - 64);
        if (left) halo_xy = (long long)(y0 + t - 128) * N + (x0 + N - 1) % N;
        if (right) halo_xy = (long long)(y0 + t - 192) * N + (x0 + TX) % N;
        int halo_slot = 0;  // LDS offset of this thread's halo value(s)
        if (top) halo_slot = 4 * t;
        if (bottom) halo_slot = (TY + 1) * TX + 4 * (t - 64);
        if (left) halo_slot = PLANE + (t - 128);
        if (right) halo_slot = PLANE + TY + (t - 192);

        T dm[NF][4], dcur[NF][4], fcur[NF][4];
        // plane z0-1: own quad, drifted
        {
            const long long base = (long long)((z0 + N - 1) % N) * NN;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const Quad<T> dq = load_quad(din[i], base + own_xy);
                const Quad<T> pq = load_quad(pin[i], base + own_xy);
#pragma unroll
                for (int e = 0; e < 4; e++) dm[i][e] = nbr_drift<T, NF, MODE>(c, i, dq.v[e], pq.v[e]);
            }
        }
        // plane z0: own quad and halo ring into LDS buffer 0
        {
            const long long base = (long long)z0 * NN;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const Quad<T> dq = load_quad(din[i], base + own_xy);
                const Quad<T> pq = load_quad(pin[i], base + own_xy);
#pragma unroll
                for (int e = 0; e < 4; e++) own_drift<T, NF, MODE>(c, i, dq.v[e], pq.v[e], fcur[i][e], dcur[i][e]);
                lds_store_quad(&lds[0][i][(y + 1) * TX + 4 * q], dcur[i]);
                if (top || bottom) {
                    const Quad<T> hd = load_quad(din[i], base + halo_xy);
                    const Quad<T> hp = load_quad(pin[i], base + halo_xy);
                    T hv[4];
#pragma unroll
                    for (int e = 0; e < 4; e++) hv[e] = nbr_drift<T, NF, MODE>(c, i, hd.v[e], hp.v[e]);
                    lds_store_quad(&lds[0][i][halo_slot], hv);
                } else if (left || right) {
                    lds[0][i][halo_slot] = nbr_drift<T, NF, MODE>(c, i, din[i][base + halo_xy], pin[i][base + halo_xy]);
                }
            }
        }
        __syncthreads();

        for (int k = 0; k < zc; k++) {
            const int z = z0 + k;
            const int cb = k % 3, nb = (k + 1) % 3;
            const bool more = k + 1 < zc;  // the next plane is inside the tile
            const long long nbase = (long long)((z + 1) % N) * NN;
            // next plane: own quad (z neighbour) and, inside the tile, the halo ring
            Quad<T> nd[NF], np[NF];
            Quad<T> hd[NF], hp[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) {
                nd[i] = load_quad(din[i], nbase + own_xy);
                np[i] = load_quad(pin[i], nbase + own_xy);
                if (more && (top || bottom)) {
                    hd[i] = load_quad(din[i], nbase + halo_xy);
                    hp[i] = load_quad(pin[i], nbase + halo_xy);
                } else if (more && (left || right)) {
                    hd[i].v[0] = din[i][nbase + halo_xy];
                    hp[i].v[0] = pin[i][nbase + halo_xy];
                }
            }
            // in-plane neighbours of plane z from LDS and the adjacent lanes
            T pair[NF][4];
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const T *P = lds[cb][i];
                T xl = lane_from_left(dcur[i][3]);
                T xr = lane_from_right(dcur[i][0]);
                if (q == 0) xl = P[PLANE + y];
                if (q == LPR - 1) xr = P[PLANE + TY + y];
                const Quad<T> up = lds_load_quad(&P[y * TX + 4 * q]);
                const Quad<T> dn = lds_load_quad(&P[(y + 2) * TX + 4 * q]);
                pair[i][0] = xl + dcur[i][1];
                pair[i][1] = dcur[i][0] + dcur[i][2];
                pair[i][2] = dcur[i][1] + dcur[i][3];
                pair[i][3] = dcur[i][2] + xr;
#pragma unroll
                for (int e = 0; e < 4; e++) pair[i][e] += dn.v[e] + up.v[e];
            }
            // drift the next plane; publish it for the next iteration
            T dn1[NF][4], fn1[NF][4];
#pragma unroll
            for (int i = 0; i < NF; i++) {
#pragma unroll
                for (int e = 0; e < 4; e++) own_drift<T, NF, MODE>(c, i, nd[i].v[e], np[i].v[e], fn1[i][e], dn1[i][e]);
                if (more) {
                    lds_store_quad(&lds[nb][i][(y + 1) * TX + 4 * q], dn1[i]);
                    if (top || bottom) {
                        T hv[4];
#pragma unroll
                        for (int e = 0; e < 4; e++) hv[e] = nbr_drift<T, NF, MODE>(c, i, hd[i].v[e], hp[i].v[e]);
                        lds_store_quad(&lds[nb][i][halo_slot], hv);
                    } else if (left || right) {
                        lds[nb][i][halo_slot] = nbr_drift<T, NF, MODE>(c, i, hd[i].v[0], hp[i].v[0]);
                    }
                }
            }
            // Laplacian, kick, sums and stores of plane z
            const long long obase = (long long)z * NN + own_xy;
            T d1s[4][NF], fds[4][NF], lap[4][NF], pn[4][NF];
#pragma unroll
            for (int i = 0; i < NF; i++) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const T pr = pair[i][e] + (dn1[i][e] + dm[i][e]);
                    lap[e][i] = fma_t((T)-6, dcur[i][e], pr) * c.inv_dx2;
                    d1s[e][i] = dcur[i][e];
                    fds[e][i] = fcur[i][e];
                }
            }
#pragma unroll
            for (int e = 0; e < 4; e++) site_update<T, NF, MODE, NQ>(c, d1s[e], fds[e], lap[e], pn[e], acc);
#pragma unroll
            for (int i = 0; i < NF; i++) {
                Quad<T> po;
#pragma unroll
                for (int e = 0; e < 4; e++) po.v[e] = pn[e][i];
                if (MODE == kStep) {
                    Quad<T> dq;
#pragma unroll
                    for (int e = 0; e < 4; e++) dq.v[e] = dcur[i][e];
                    store_quad(dout[i], obase, dq);
                    store_quad(pout[i], obase, po);
                } else {
                    store_quad(const_cast<T *>(pin[i]), obase, po);
                }
            }
#pragma unroll
            for (int i = 0; i < NF; i++) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    dm[i][e] = dcur[i][e];
                    dcur[i][e] = dn1[i][e];
                    fcur[i][e] = fn1[i][e];
                }
            }
            __syncthreads();
        }
    }

    block_sum<NQ>(acc, red);
    if (threadIdx.x < NQ) lat.partials[(long long)blockIdx.x * kMaxSums + threadIdx.x] = red[0][threadIdx.x];
    finish_pass<T, NQ, MODE>(lat, red);
}

template <typename T, int NF, int LPR>
hipError_t launch_lpr(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    dim3 grid(lat.nblocks), block(kBlock);
    if (mode == kStep)
        hipLaunchKernelGGL((tiled3d_kernel<T, NF, kStep, LPR>), grid, block, 0, st, lat, src);
    else
        hipLaunchKernelGGL((tiled3d_kernel<T, NF, kInit, LPR>), grid, block, 0, st, lat, src);
    return hipGetLastError();
}

template <typename T, int NF>
hipError_t launch_nf(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.lpr) {
    case 8: return launch_lpr<T, NF, 8>(lat, src, mode, st);
    case 16: return launch_lpr<T, NF, 16>(lat, src, mode, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_t(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.nf) {
    case 1: return launch_nf<T, 1>(lat, src, mode, st);
    case 2: return launch_nf<T, 2>(lat, src, mode, st);
    case 3: return launch_nf<T, 3>(lat, src, mode, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int NF, int LPR>
int resident_for()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tiled3d_kernel<T, NF, kStep, LPR>, kBlock, 0) !=
        hipSuccess)
        return 0;
    return n;
}

template <typename T, int NF>
int resident_nf(int lpr)
{
    return lpr == 8 ? resident_for<T, NF, 8>() : resident_for<T, NF, 16>();
}

template <typename T>
int resident_t(int nf, int lpr)
{
    switch (nf) {
    case 1: return resident_nf<T, 1>(lpr);
    case 2: return resident_nf<T, 2>(lpr);
    default: return resident_nf<T, 3>(lpr);
    }
}

}  // namespace

bool tiled_fits(int dims, int N, int lpr, int zc)
{
    if (dims != 3 || (lpr != 8 && lpr != 16)) return false;
    const int TX = 4 * lpr, TY = kBlock / lpr;
    return N % TX == 0 && N % TY == 0 && zc >= 1 && N % zc == 0;
}

long long tiled_tiles(int N, int lpr, int zc)
{
    const int TX = 4 * lpr, TY = kBlock / lpr;
    return (long long)(N / TX) * (N / TY) * (N / zc);
}

int tiled_resident_blocks(int precision, int nf, int lpr)
{
    return precision == CE_FP64 ? resident_t<double>(nf, lpr) : resident_t<float>(nf, lpr);
}

hipError_t launch_tiled(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    if (precision == CE_FP64) return launch_t<double>(lat, src, mode, st);
    return launch_t<float>(lat, src, mode, st);
}

}  // namespace ce
