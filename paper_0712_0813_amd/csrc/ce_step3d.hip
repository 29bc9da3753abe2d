// Tiled 3-D leapfrog pass for gfx950: z-streaming with an LDS plane tile.
//
// A block of BS threads owns an (x, y) tile of VEC*LPR x BS/LPR sites and
// walks one chunk of its z column: the column is cut into ceil(N/zc) chunks
// of near-equal length (zc planes each when zc divides N).  Each thread owns VEC consecutive x sites
// (one 64- or 128-bit load per array).  Per plane it loads its own sites of d
// and p once, drifts them, and keeps the drifted deviation of planes z-1, z
// and z+1 in registers (the z neighbours).  The drifted plane also goes to a
// triple-buffered LDS tile whose one-site halo ring is filled by four groups
// of threads; y neighbours are read from LDS, x neighbours come from the
// adjacent lane by a whole-wave DPP shift, and the tile's edge lanes take the
// halo column instead.  With three LDS buffers one barrier per plane
// suffices.  Only the halo ring and the two extra planes per tile are read
// twice, from L2 when the tile that owns them has read them recently (about
// half of them at 1024^3).  FP32 outputs leave through streaming stores.
//
// The grid is persistent: each block walks tiles, and the tiles are numbered
// so that the blocks the hardware places on one XCD (block ids equal mod 8)
// work on one contiguous slab, so that y halos can come from that XCD's L2.
// In the lone pass the blocks of an XCD take their slab's tiles in order from
// a counter as they become free (in the batched pass, in a fixed order).  The
// FP64 volume sums are formed per tile and reduced in tile order when the
// lattice holds a partial row per tile, so no result depends on which block
// worked which tile; the sums and the scale-factor tail are otherwise those
// of the direct pass.
#include "ce_device.hpp"

#ifndef CE_UNIT_MODEL
#error "compile this file once per model, with -DCE_UNIT_MODEL=0 and -DCE_UNIT_MODEL=1"
#endif

namespace ce {
namespace {

using namespace dev;

template <typename T, int VEC>
__device__ __forceinline__ Vec<T, VEC> gload(gcptr<T> base, unsigned s)
{
    Vec<T, VEC> r;
    if constexpr (VEC == 4) {
        const Quad<T> q = load_quad(base, s);
#pragma unroll
        for (int e = 0; e < 4; e++) r.v[e] = q.v[e];
    } else {
        r = load_vec2(base, s);
    }
    return r;
}

template <typename T, int VEC>
__device__ __forceinline__ void gstore(gptr<T> base, unsigned s, const T (&v)[VEC])
{
    if constexpr (VEC == 4) {
        Quad<T> q;
#pragma unroll
        for (int e = 0; e < 4; e++) q.v[e] = v[e];
        if constexpr (sizeof(T) == 4)
            store_quad_stream(base, s, q);
        else
            store_quad(base, s, q);
    } else {
        Vec<T, 2> q;
        q.v[0] = v[0];
        q.v[1] = v[1];
        store_vec2(base, s, q);
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void lds_store(T *p, const T (&v)[VEC])
{
    if constexpr (sizeof(T) * VEC == 16) {
        f32x4 w;
        const float *f = reinterpret_cast<const float *>(v);
        w.x = f[0];
        w.y = f[1];
        w.z = f[2];
        w.w = f[3];
        *reinterpret_cast<f32x4 *>(p) = w;
    } else if constexpr (sizeof(T) * VEC == 8) {
        f32x2 w;
        const float *f = reinterpret_cast<const float *>(v);
        w.x = f[0];
        w.y = f[1];
        *reinterpret_cast<f32x2 *>(p) = w;
    } else {  // 4 doubles
        f64x2 a, b;
        a.x = v[0];
        a.y = v[1];
        b.x = v[2];
        b.y = v[3];
        reinterpret_cast<f64x2 *>(p)[0] = a;
        reinterpret_cast<f64x2 *>(p)[1] = b;
    }
}

template <typename T, int VEC>
__device__ __forceinline__ Vec<T, VEC> lds_load(const T *p)
{
    Vec<T, VEC> r;
    if constexpr (sizeof(T) * VEC == 16) {
        const f32x4 w = *reinterpret_cast<const f32x4 *>(p);
        float *f = reinterpret_cast<float *>(r.v);
        f[0] = w.x;
        f[1] = w.y;
        f[2] = w.z;
        f[3] = w.w;
    } else if constexpr (sizeof(T) * VEC == 8) {
        const f32x2 w = *reinterpret_cast<const f32x2 *>(p);
        float *f = reinterpret_cast<float *>(r.v);
        f[0] = w.x;
        f[1] = w.y;
    } else {
        const f64x2 a = reinterpret_cast<const f64x2 *>(p)[0];
        const f64x2 b = reinterpret_cast<const f64x2 *>(p)[1];
        r.v[0] = a.x;
        r.v[1] = a.y;
        r.v[2] = b.x;
        r.v[3] = b.y;
    }
    return r;
}

// Occupancy target for FP32 kernels with up to two fields: two sites per
// thread fit 128 VGPRs (four waves per SIMD) and four sites fit 168 (three)
// without spilling; the others are left to the compiler (larger states spill
// when squeezed).
template <typename T, int NF, int MODEL, int VEC>
struct WavesHint {
    static constexpr int value = (MODEL == kQuartic && NF <= 2) ? (sizeof(T) == 4 ? (VEC == 2 ? 4 : 3) : 2) : 1;
};

// Body of the tiled pass: block b of the `grid` blocks this lattice gets.
//
// Every thread with a halo duty (a row above or below the tile, or a column
// left or right of it) issues the same vector loads: a column thread loads
// the aligned group of VEC sites that holds its column site and keeps one
// element.  Halo rows and columns thus share one load path, so a plane's
// loads go out together and no halo load has to wait for registers that a
// pending load of the other branch writes (which would serialise the row
// threads' halo loads behind their own-site loads, one memory round trip
// each).
template <typename T, int NF, int MODEL, int MODE, int VEC, int LPR, int BS, bool DYN>
__device__ __forceinline__ void tiled3d_body(const Lattice &lat, int src, int b, int grid)
{
    constexpr int NQ = kSumsPerField * NF + 1;
    constexpr int TX = VEC * LPR;
    constexpr int TY = BS / LPR;
    constexpr int PLANE = (TY + 2) * TX;
    constexpr int FSTRIDE = PLANE + 2 * TY;  // plane with halo rows, then left/right columns
    constexpr int G4 = BS / 4;               // halo role groups start at 0, G4, 2 G4, 3 G4
    static_assert(LPR <= G4 && TY <= G4, "halo groups must fit");
    static_assert(LPR <= 64 && 64 % LPR == 0, "a tile row must lie inside one wavefront");
    __shared__ __align__(16) T lds[3][NF][FSTRIDE];
    __shared__ double red[BS / 64][kMaxSums];
    __shared__ unsigned int s_tile;

    const int N = lat.N;
    const int zc = lat.zc;
    const int ntx = N / TX, nty = N / TY;
    // the z column is cut into nz chunks of near-equal length (zc planes
    // each when zc divides N)
    const int nz = (N + zc - 1) / zc;
    const long long ntiles = (long long)ntx * nty * nz;
    const int t = threadIdx.x;
    const int q = t % LPR;  // own site group within the tile row
    const int y = t / LPR;  // own row within the tile
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

    // halo duties: one group of threads per side of the ring
    const bool top = t < LPR;                          // row y0-1, group t
    const bool bottom = t >= G4 && t < G4 + LPR;       // row y0+TY, group t-G4
    const bool left = t >= 2 * G4 && t < 2 * G4 + TY;  // column x0-1, row t-2G4
    const bool right = t >= 3 * G4 && t < 3 * G4 + TY; // column x0+TX, row t-3G4
    const bool hrow = top || bottom;
    const bool hcol = left || right;
    const bool hduty = hrow || hcol;

    double acc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; k++) acc[k] = 0.0;

    // Sums per tile when the lattice has a partial row for every tile: the
    // result is then the same whichever block worked a tile, and where there
    // are more tiles than blocks, blocks of the lone pass (DYN) take their
    // tiles in order from a counter, those of each XCD from its own slab's
    // counter, so that the tiles that share halo rows are worked at the same
    // time and no block idles at the end while others still hold several
    // tiles.  Otherwise tiles in the fixed XCD-contiguous order (one per
    // block when there are no more tiles than blocks), and sums per block
    // when the partial rows do not cover the tiles.
    const bool per_tile = ntiles <= lat.slots;
    const bool dyn = DYN && per_tile && ntiles > grid;
    const bool split8 = (grid & 7) == 0 && (ntiles & 7) == 0;
    const long long slab = split8 ? ntiles >> 3 : ntiles;
    const int counter = split8 ? 1 + (b & 7) : 1;
    const long long first_tile = split8 ? (long long)(b & 7) * slab : 0;
    const long long NN = (long long)N * N;
    for (int j = 0;; j++) {
        long long tile;
        if (dyn) {
            __syncthreads();  // every thread has read the previous s_tile
            if (threadIdx.x == 0)
                s_tile = __hip_atomic_fetch_add(lat.ticket + counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const long long idx = (long long)s_tile;
            tile = idx < slab ? first_tile + idx : -1;
        } else {
            tile = xcd_item(b, j, grid, ntiles);
        }
        if (tile < 0) break;
        const int tx = (int)(tile % ntx);
        const int ty = (int)((tile / ntx) % nty);
        const int chunk = (int)(tile / ((long long)ntx * nty));
        const int z0 = chunk * N / nz;
        const int zlen = (chunk + 1) * N / nz - z0;
        const int x0 = tx * TX, y0 = ty * TY;
        // offsets within one plane (< N^2, 32 bits); plane bases are uniform
        const unsigned own_xy = (unsigned)((y0 + y) * N + x0 + VEC * q);
        unsigned halo_xy = 0;
        int halo_slot = 0;  // LDS offset of this thread's halo value(s)
        if (top) {
            halo_xy = (unsigned)(((y0 + N - 1) % N) * N + x0 + VEC * t);
            halo_slot = VEC * t;
        } else if (bottom) {
            halo_xy = (unsigned)(((y0 + TY) % N) * N + x0 + VEC * (t - G4));
            halo_slot = (TY + 1) * TX + VEC * (t - G4);
        } else if (left) {
            halo_xy = (unsigned)((y0 + t - 2 * G4) * N + (x0 + N - VEC) % N);
            halo_slot = PLANE + (t - 2 * G4);
        } else if (right) {
            halo_xy = (unsigned)((y0 + t - 3 * G4) * N + (x0 + TX) % N);
            halo_slot = PLANE + TY + (t - 3 * G4);
        }

        T dm[NF][VEC], dcur[NF][VEC], fcur[NF][VEC];
        // plane z0-1: own sites, drifted
        {
            const long long base = (long long)((z0 + N - 1) % N) * NN;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const Vec<T, VEC> dq = gload<T, VEC>(din[i] + base, own_xy);
                const Vec<T, VEC> pq = gload<T, VEC>(pin[i] + base, own_xy);
#pragma unroll
                for (int e = 0; e < VEC; e++) dm[i][e] = nbr_drift<T, NF, MODE>(c, i, dq.v[e], pq.v[e]);
            }
        }
        // plane z0: own sites and halo ring into LDS buffer 0
        {
            const long long base = (long long)z0 * NN;
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const Vec<T, VEC> dq = gload<T, VEC>(din[i] + base, own_xy);
                const Vec<T, VEC> pq = gload<T, VEC>(pin[i] + base, own_xy);
#pragma unroll
                for (int e = 0; e < VEC; e++) own_drift<T, NF, MODE>(c, i, dq.v[e], pq.v[e], fcur[i][e], dcur[i][e]);
                lds_store<T, VEC>(&lds[0][i][(y + 1) * TX + VEC * q], dcur[i]);
                if (hduty) {
                    const Vec<T, VEC> hd = gload<T, VEC>(din[i] + base, halo_xy);
                    const Vec<T, VEC> hp = gload<T, VEC>(pin[i] + base, halo_xy);
                    if (hcol) {
                        lds[0][i][halo_slot] = nbr_drift<T, NF, MODE>(c, i, left ? hd.v[VEC - 1] : hd.v[0],
                                                                    left ? hp.v[VEC - 1] : hp.v[0]);
                    } else {
                        T hv[VEC];
#pragma unroll
                        for (int e = 0; e < VEC; e++) hv[e] = nbr_drift<T, NF, MODE>(c, i, hd.v[e], hp.v[e]);
                        lds_store<T, VEC>(&lds[0][i][halo_slot], hv);
                    }
                }
            }
        }
        __syncthreads();

        for (int k = 0; k < zlen; k++) {
            const int z = z0 + k;
            const int cb = k % 3, nb = (k + 1) % 3;
            const bool more = k + 1 < zlen;  // the next plane is inside the tile
            const long long nbase = (long long)((z + 1) % N) * NN;
            // next plane: own sites (z neighbours) and, inside the tile, the halo ring
            Vec<T, VEC> nd[NF], np[NF], hd[NF], hp[NF];
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const gcptr<T> dpl = din[i] + nbase, ppl = pin[i] + nbase;
                nd[i] = gload<T, VEC>(dpl, own_xy);
                np[i] = gload<T, VEC>(ppl, own_xy);
                if (more && hduty) {
                    hd[i] = gload<T, VEC>(dpl, halo_xy);
                    hp[i] = gload<T, VEC>(ppl, halo_xy);
                }
            }
            // in-plane neighbour pairs of plane z: x from adjacent lanes, y from LDS
            T pair[NF][VEC];
#pragma unroll
            for (int i = 0; i < NF; i++) {
                const T *P = lds[cb][i];
                T xl = lane_from_left(dcur[i][VEC - 1]);
                T xr = lane_from_right(dcur[i][0]);
                if (q == 0) xl = P[PLANE + y];
                if (q == LPR - 1) xr = P[PLANE + TY + y];
                const Vec<T, VEC> up = lds_load<T, VEC>(&P[y * TX + VEC * q]);
                const Vec<T, VEC> dn = lds_load<T, VEC>(&P[(y + 2) * TX + VEC * q]);
#pragma unroll
                for (int e = 0; e < VEC; e++) {
                    const T l = e == 0 ? xl : dcur[i][e - 1];
                    const T r = e == VEC - 1 ? xr : dcur[i][e + 1];
                    pair[i][e] = (l + r) + (dn.v[e] + up.v[e]);
                }
            }
            // drift the next plane; publish it for the next iteration
            T dn1[NF][VEC], fn1[NF][VEC];
#pragma unroll
            for (int i = 0; i < NF; i++) {
#pragma unroll
                for (int e = 0; e < VEC; e++) own_drift<T, NF, MODE>(c, i, nd[i].v[e], np[i].v[e], fn1[i][e], dn1[i][e]);
                if (more) {
                    lds_store<T, VEC>(&lds[nb][i][(y + 1) * TX + VEC * q], dn1[i]);
                    if (hrow) {
                        T hv[VEC];
#pragma unroll
                        for (int e = 0; e < VEC; e++) hv[e] = nbr_drift<T, NF, MODE>(c, i, hd[i].v[e], hp[i].v[e]);
                        lds_store<T, VEC>(&lds[nb][i][halo_slot], hv);
                    } else if (hcol) {
                        lds[nb][i][halo_slot] = nbr_drift<T, NF, MODE>(c, i, left ? hd[i].v[VEC - 1] : hd[i].v[0],
                                                                     left ? hp[i].v[VEC - 1] : hp[i].v[0]);
                    }
                }
            }
            // Laplacian, kick, sums and stores of plane z
            const long long obase = (long long)z * NN;
            T part[NQ];
            clear_part(part);
#pragma unroll
            for (int e = 0; e < VEC; e++) {
                T d1s[NF], fds[NF], lap[NF], pn[NF];
#pragma unroll
                for (int i = 0; i < NF; i++) {
                    const T pr = pair[i][e] + (dn1[i][e] + dm[i][e]);
                    lap[i] = fma_t((T)-6, dcur[i][e], pr) * c.inv_dx2;
                    d1s[i] = dcur[i][e];
                    fds[i] = fcur[i][e];
                }
                site_update<T, NF, MODEL, MODE, NQ>(c, d1s, fds, lap, pn, part);
#pragma unroll
                for (int i = 0; i < NF; i++) fcur[i][e] = pn[i];  // reuse: new stored derivative
            }
            flush_sums(part, acc);
#pragma unroll
            for (int i = 0; i < NF; i++) {
                if (MODE == kStep) {
                    gstore<T, VEC>(dout[i] + obase, own_xy, dcur[i]);
                    gstore<T, VEC>(pout[i] + obase, own_xy, fcur[i]);
                } else {
                    gstore<T, VEC>(as_global<T>(lat.p[src][i]) + obase, own_xy, fcur[i]);
                }
#pragma unroll
                for (int e = 0; e < VEC; e++) {
                    dm[i][e] = dcur[i][e];
                    dcur[i][e] = dn1[i][e];
                    fcur[i][e] = fn1[i][e];
                }
            }
            __syncthreads();
        }
        if (per_tile) {
            // this tile's row; the next tile starts its sums from zero
            block_sum<NQ>(acc, red);
            if (threadIdx.x < NQ) *partial_at(lat, threadIdx.x, tile) = red[0][threadIdx.x];
#pragma unroll
            for (int k = 0; k < NQ; k++) acc[k] = 0.0;
        }
    }

    if (!per_tile) {
        block_sum<NQ>(acc, red);
        if (threadIdx.x < NQ) *partial_at(lat, threadIdx.x, b) = red[0][threadIdx.x];
    }
    // up to a few thousand tile rows: several rows' loads in flight per thread
    finish_pass<T, NQ, MODE, (NQ <= 13 ? 4 : 2)>(lat, grid, per_tile ? (int)ntiles : grid, red);
}

template <typename T, int NF, int MODEL, int MODE, int VEC, int LPR, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(WavesHint<T, NF, MODEL, VEC>::value, 8))) void
tiled3d_kernel(Lattice lat, int src)
{
    tiled3d_body<T, NF, MODEL, MODE, VEC, LPR, BS, true>(lat, src, blockIdx.x, gridDim.x);
}

// Step pass over many lattices of one class; see pass_batched.
template <typename T, int NF, int MODEL, int VEC, int LPR, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(WavesHint<T, NF, MODEL, VEC>::value, 8))) void
tiled3d_batched(const Lattice *lats, const int *blk_lat, int total)
{
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        const int l = __builtin_amdgcn_readfirstlane(blk_lat[v]);
        const Lattice &lat = *(const Lattice *)((const __attribute__((address_space(4))) Lattice *)lats + l);
        if (lat.sc->remaining <= 0) continue;
        const int src = lat.sc->cur;
        tiled3d_body<T, NF, MODEL, kStep, VEC, LPR, BS, false>(lat, src, v - lat.first_block, lat.nblocks);
    }
}

// The tile shapes built: (sites per thread, lanes per row, block).
struct Shape {
    int vec, lpr, bs;
};
constexpr Shape kShapes[] = {{4, 16, 256}, {4, 8, 256}, {2, 32, 256}, {2, 32, 512},
                             {2, 16, 256}, {2, 16, 512}, {4, 64, 256}, {4, 64, 512}};

// LDS of one block; shapes above the 160 KiB a workgroup may hold are not built.
template <typename T, int NF, int VEC, int LPR, int BS>
constexpr bool lds_fits()
{
    constexpr int TX = VEC * LPR, TY = BS / LPR;
    return 3 * NF * ((TY + 2) * TX + 2 * TY) * (int)sizeof(T) + (BS / 64) * kMaxSums * 8 <= 160 * 1024;
}

template <typename T, int NF, int MODEL, int MODE, int VEC, int LPR, int BS>
hipError_t launch_one(const Lattice &lat, int src, hipStream_t st)
{
    if constexpr (lds_fits<T, NF, VEC, LPR, BS>()) {
        hipLaunchKernelGGL((tiled3d_kernel<T, NF, MODEL, MODE, VEC, LPR, BS>), dim3(lat.nblocks), dim3(BS), 0, st, lat, src);
        return hipGetLastError();
    } else {
        return hipErrorInvalidConfiguration;
    }
}

template <typename T, int NF, int MODEL, int VEC, int LPR, int BS>
hipError_t batched_one(const Lattice *lats, const int *blk_lat, int total, int grid, hipStream_t st)
{
    if constexpr (lds_fits<T, NF, VEC, LPR, BS>()) {
        hipLaunchKernelGGL((tiled3d_batched<T, NF, MODEL, VEC, LPR, BS>), dim3(grid), dim3(BS), 0, st, lats, blk_lat,
                           total);
        return hipGetLastError();
    } else {
        return hipErrorInvalidConfiguration;
    }
}

template <typename T, int NF, int MODEL, int VEC, int LPR, int BS>
int resident_batched_one()
{
    if constexpr (lds_fits<T, NF, VEC, LPR, BS>()) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tiled3d_batched<T, NF, MODEL, VEC, LPR, BS>, BS, 0) !=
            hipSuccess)
            return 0;
        return n;
    } else {
        return 0;
    }
}

template <typename T, int NF, int MODEL, int VEC, int LPR, int BS>
int resident_one()
{
    if constexpr (lds_fits<T, NF, VEC, LPR, BS>()) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tiled3d_kernel<T, NF, MODEL, kStep, VEC, LPR, BS>, BS, 0) !=
            hipSuccess)
            return 0;
        return n;
    } else {
        return 0;
    }
}

// Dispatch over the built shapes; `fn` receives the template instance.
template <typename T, int NF, int MODEL>
struct ByShape {
    template <int MODE>
    static hipError_t launch(const Lattice &lat, int src, hipStream_t st)
    {
        const int v = lat.vec, l = lat.lpr, b = lat.bs;
        if (v == 4 && l == 16 && b == 256) return launch_one<T, NF, MODEL, MODE, 4, 16, 256>(lat, src, st);
        if (v == 4 && l == 8 && b == 256) return launch_one<T, NF, MODEL, MODE, 4, 8, 256>(lat, src, st);
        if (v == 2 && l == 32 && b == 256) return launch_one<T, NF, MODEL, MODE, 2, 32, 256>(lat, src, st);
        if (v == 2 && l == 32 && b == 512) return launch_one<T, NF, MODEL, MODE, 2, 32, 512>(lat, src, st);
        if (v == 2 && l == 16 && b == 256) return launch_one<T, NF, MODEL, MODE, 2, 16, 256>(lat, src, st);
        if (v == 2 && l == 16 && b == 512) return launch_one<T, NF, MODEL, MODE, 2, 16, 512>(lat, src, st);
        if (v == 4 && l == 64 && b == 256) return launch_one<T, NF, MODEL, MODE, 4, 64, 256>(lat, src, st);
        if (v == 4 && l == 64 && b == 512) return launch_one<T, NF, MODEL, MODE, 4, 64, 512>(lat, src, st);
        return hipErrorInvalidValue;
    }
    static hipError_t batched(const Lattice *lats, const int *blk_lat, int total, int grid, int v, int l, int b,
                              hipStream_t st)
    {
        if (v == 4 && l == 16 && b == 256) return batched_one<T, NF, MODEL, 4, 16, 256>(lats, blk_lat, total, grid, st);
        if (v == 4 && l == 8 && b == 256) return batched_one<T, NF, MODEL, 4, 8, 256>(lats, blk_lat, total, grid, st);
        if (v == 2 && l == 32 && b == 256) return batched_one<T, NF, MODEL, 2, 32, 256>(lats, blk_lat, total, grid, st);
        if (v == 2 && l == 32 && b == 512) return batched_one<T, NF, MODEL, 2, 32, 512>(lats, blk_lat, total, grid, st);
        if (v == 2 && l == 16 && b == 256) return batched_one<T, NF, MODEL, 2, 16, 256>(lats, blk_lat, total, grid, st);
        if (v == 2 && l == 16 && b == 512) return batched_one<T, NF, MODEL, 2, 16, 512>(lats, blk_lat, total, grid, st);
        if (v == 4 && l == 64 && b == 256) return batched_one<T, NF, MODEL, 4, 64, 256>(lats, blk_lat, total, grid, st);
        if (v == 4 && l == 64 && b == 512) return batched_one<T, NF, MODEL, 4, 64, 512>(lats, blk_lat, total, grid, st);
        return hipErrorInvalidValue;
    }
    static int resident(int v, int l, int b)
    {
        if (v == 4 && l == 16 && b == 256) return resident_one<T, NF, MODEL, 4, 16, 256>();
        if (v == 4 && l == 8 && b == 256) return resident_one<T, NF, MODEL, 4, 8, 256>();
        if (v == 2 && l == 32 && b == 256) return resident_one<T, NF, MODEL, 2, 32, 256>();
        if (v == 2 && l == 32 && b == 512) return resident_one<T, NF, MODEL, 2, 32, 512>();
        if (v == 2 && l == 16 && b == 256) return resident_one<T, NF, MODEL, 2, 16, 256>();
        if (v == 2 && l == 16 && b == 512) return resident_one<T, NF, MODEL, 2, 16, 512>();
        if (v == 4 && l == 64 && b == 256) return resident_one<T, NF, MODEL, 4, 64, 256>();
        if (v == 4 && l == 64 && b == 512) return resident_one<T, NF, MODEL, 4, 64, 512>();
        return 0;
    }
    static int resident_batched(int v, int l, int b)
    {
        if (v == 4 && l == 16 && b == 256) return resident_batched_one<T, NF, MODEL, 4, 16, 256>();
        if (v == 4 && l == 8 && b == 256) return resident_batched_one<T, NF, MODEL, 4, 8, 256>();
        if (v == 2 && l == 32 && b == 256) return resident_batched_one<T, NF, MODEL, 2, 32, 256>();
        if (v == 2 && l == 32 && b == 512) return resident_batched_one<T, NF, MODEL, 2, 32, 512>();
        if (v == 2 && l == 16 && b == 256) return resident_batched_one<T, NF, MODEL, 2, 16, 256>();
        if (v == 2 && l == 16 && b == 512) return resident_batched_one<T, NF, MODEL, 2, 16, 512>();
        if (v == 4 && l == 64 && b == 256) return resident_batched_one<T, NF, MODEL, 4, 64, 256>();
        if (v == 4 && l == 64 && b == 512) return resident_batched_one<T, NF, MODEL, 4, 64, 512>();
        return 0;
    }
};

template <typename T, int MODEL>
hipError_t launch_t(const Lattice &lat, int src, Mode mode, hipStream_t st)
{
    switch (lat.nf) {
    case 1: return mode == kStep ? ByShape<T, 1, MODEL>::template launch<kStep>(lat, src, st)
                                 : ByShape<T, 1, MODEL>::template launch<kInit>(lat, src, st);
    case 2: return mode == kStep ? ByShape<T, 2, MODEL>::template launch<kStep>(lat, src, st)
                                 : ByShape<T, 2, MODEL>::template launch<kInit>(lat, src, st);
    case 3: return mode == kStep ? ByShape<T, 3, MODEL>::template launch<kStep>(lat, src, st)
                                 : ByShape<T, 3, MODEL>::template launch<kInit>(lat, src, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODEL>
hipError_t batched_t(const Lattice *lats, const int *blk_lat, int total, int grid, const Lattice &p, hipStream_t st)
{
    switch (p.nf) {
    case 1: return ByShape<T, 1, MODEL>::batched(lats, blk_lat, total, grid, p.vec, p.lpr, p.bs, st);
    case 2: return ByShape<T, 2, MODEL>::batched(lats, blk_lat, total, grid, p.vec, p.lpr, p.bs, st);
    case 3: return ByShape<T, 3, MODEL>::batched(lats, blk_lat, total, grid, p.vec, p.lpr, p.bs, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODEL>
int resident_batched_t(const Lattice &p)
{
    switch (p.nf) {
    case 1: return ByShape<T, 1, MODEL>::resident_batched(p.vec, p.lpr, p.bs);
    case 2: return ByShape<T, 2, MODEL>::resident_batched(p.vec, p.lpr, p.bs);
    default: return ByShape<T, 3, MODEL>::resident_batched(p.vec, p.lpr, p.bs);
    }
}

template <typename T, int MODEL>
int resident_t(int nf, int v, int l, int b)
{
    switch (nf) {
    case 1: return ByShape<T, 1, MODEL>::resident(v, l, b);
    case 2: return ByShape<T, 2, MODEL>::resident(v, l, b);
    default: return ByShape<T, 3, MODEL>::resident(v, l, b);
    }
}

}  // namespace

// This unit's model (the source is compiled once per model).
constexpr int kUnit = CE_UNIT_MODEL;

template <>
int tiled_resident_blocks_model<kUnit>(int precision, int nf, int vec, int lpr, int bs)
{
    return precision == CE_FP64 ? resident_t<double, kUnit>(nf, vec, lpr, bs)
                                : resident_t<float, kUnit>(nf, vec, lpr, bs);
}

template <>
hipError_t launch_batched_tiled_model<kUnit>(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                             const Lattice &proto, int precision, hipStream_t st)
{
    if (precision == CE_FP64) return batched_t<double, kUnit>(lats, blk_lat, total_blocks, grid, proto, st);
    return batched_t<float, kUnit>(lats, blk_lat, total_blocks, grid, proto, st);
}

template <>
int tiled_batched_resident_model<kUnit>(const Lattice &proto, int precision)
{
    return precision == CE_FP64 ? resident_batched_t<double, kUnit>(proto) : resident_batched_t<float, kUnit>(proto);
}

template <>
hipError_t launch_tiled_model<kUnit>(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    if (precision == CE_FP64) return launch_t<double, kUnit>(lat, src, mode, st);
    return launch_t<float, kUnit>(lat, src, mode, st);
}

#if CE_UNIT_MODEL == CE_MODEL_QUARTIC
// Model-independent functions and the dispatch on the model.

bool tiled_shape_built(int vec, int lpr, int bs)
{
    for (const Shape &s : kShapes)
        if (s.vec == vec && s.lpr == lpr && s.bs == bs) return true;
    return false;
}

bool tiled_fits(int dims, int N, int vec, int lpr, int bs, int zc)
{
    if (dims != 3 || !tiled_shape_built(vec, lpr, bs)) return false;
    const int TX = vec * lpr, TY = bs / lpr;
    return N % TX == 0 && N % TY == 0 && zc >= 1 && zc <= N;
}

long long tiled_tiles(int N, int vec, int lpr, int bs, int zc)
{
    const int TX = vec * lpr, TY = bs / lpr;
    return (long long)(N / TX) * (N / TY) * ((N + zc - 1) / zc);
}

int tiled_resident_blocks(int model, int precision, int nf, int vec, int lpr, int bs)
{
    return model == kPoly ? tiled_resident_blocks_model<kPoly>(precision, nf, vec, lpr, bs)
                          : tiled_resident_blocks_model<kQuartic>(precision, nf, vec, lpr, bs);
}

hipError_t launch_batched_tiled(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                const Lattice &proto, int precision, hipStream_t st)
{
    return proto.model == kPoly
               ? launch_batched_tiled_model<kPoly>(lats, blk_lat, total_blocks, grid, proto, precision, st)
               : launch_batched_tiled_model<kQuartic>(lats, blk_lat, total_blocks, grid, proto, precision, st);
}

int tiled_batched_resident(const Lattice &proto, int precision)
{
    return proto.model == kPoly ? tiled_batched_resident_model<kPoly>(proto, precision)
                                : tiled_batched_resident_model<kQuartic>(proto, precision);
}

hipError_t launch_tiled(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st)
{
    return lat.model == kPoly ? launch_tiled_model<kPoly>(lat, precision, src, mode, st)
                              : launch_tiled_model<kQuartic>(lat, precision, src, mode, st);
}
#endif  // CE_UNIT_MODEL == CE_MODEL_QUARTIC

}  // namespace ce
