// Radially binned power spectra of a field and of its time derivative.
//
// The paper's programs Fourier transform the fields to output spectra and lay
// the transform out in the field arrays with the last dimension padded from N
// to N + 2, where the Nyquist modes go ("Parallel Algorithms" section, last
// paragraphs).  Here each row's transform is kept the same way, as its
// N/2 + 1 complex values (N + 2 doubles), in a scratch buffer: the
// simulation's second ping-pong buffers, which are free between steps.  When
// they cannot hold all N/2 + 1 values of every row, the k_last range is done
// in chunks (each chunk re-reads the field).
//
//   rows kernel   last axis: real field row -> k_last in [k0, k0 + kc)
//   mid kernel    (3-D) second axis, in place
//   final kernel  first axis (2-D and 3-D), then |F|^2 into radial bins
//   reduce kernel per-block partial bins summed in a fixed order
//
// Binning is deterministic: one wavefront per block walks each line's
// elements in order of increasing |n_0| (the bin is then non-decreasing),
// sums runs of equal bins with a segmented scan across the wavefront and adds
// the run totals to the block's LDS histogram; blocks write partial
// histograms that one kernel sums in block order.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ce_device.hpp"
#include "ce_fft.hpp"
#include "ce_sim.hpp"

using namespace ce;
using namespace ce::host;
using namespace ce::fft;
using ce::dev::FieldCoef;
using ce::dev::fdot_of;

namespace {

constexpr int kSpecThreads = 256;
constexpr int kSpecLines = 1024;   // complex values of the line buffer (16 KiB): 1024 / N lines
constexpr int kMaxSpecN = 2048;
constexpr int kMaxGroups = 2048;   // blocks of the binning kernel
constexpr size_t kTwOffset = 0;    // twiddles at the start of the partial-sum buffer
constexpr size_t kOutOffset = 32768;

int spec_lines(int N) { return std::max(1, kSpecLines / N); }
// the first-axis kernel: one wavefront bins each line after its transform,
// so more lines per block only lengthen that serial part (measured: two
// lines of 1024 per block were slower than one)
int spec_final_lines(int N) { return spec_lines(N); }
// the middle axis: two line buffers per block (1024^3: 6.4 ms per pass
// against 7.6 ms with one; the rows are faster with one, 6.6 against 8.4 ms)
int spec_mid_lines(int N) { return std::max(1, 2 * kSpecLines / N); }

int nbins_of(int dims, int N)
{
    const long long m = (long long)dims * (N / 2) * (N / 2);
    long long r = (long long)sqrt((double)m);
    while (r * r > m) r--;
    while ((r + 1) * (r + 1) <= m) r++;
    return (int)r + 1;
}

// The transform buffer: rows [0, rows_a) of kc values in one free block,
// the rest in a second one.
struct ZBuf {
    double2 *a, *b;
    long long rows_a;
    int kc;
    __device__ double2 *row(long long r) const { return r < rows_a ? a + r * kc : b + (r - rows_a) * kc; }
};

__device__ inline int isqrt_ll(long long v)
{
    long long r = (long long)sqrt((double)v);
    while (r * r > v) r--;
    while ((r + 1) * (r + 1) <= v) r++;
    return (int)r;
}

// Last axis.  Row r of the field (N consecutive sites) -> Z[r * kc + k - k0].
template <typename T>
__global__ __launch_bounds__(kSpecThreads) void spec_rows_kernel(const T *__restrict__ d, const T *__restrict__ p,
                                                                const Scalars *sc, int field, int which, int started,
                                                                int N, int logN, long long rows, int k0,
                                                                const double2 *__restrict__ tw, ZBuf Z, int lpw)
{
    extern __shared__ double2 lds[];
    const int kc = Z.kc;
    const long long first = (long long)blockIdx.x * lpw;
    const int nl = (int)min((long long)lpw, rows - first);
    const double m = sc->m[field];
    FieldCoef<T> c;
    const double beta = started ? sc->beta : 0.0;
    c.beta = (T)beta;
    c.bm = (T)(beta * m);
    c.r = (T)0;
    c.m1 = (T)0;
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx >> logN, x = idx & (N - 1);
        double v = 0.0;
        if (l < nl) {
            const long long s = (first + l) * N + x;
            const T dv = d[s];
            if (which == 0)
                v = m + (double)dv;
            else
                v = started ? (double)fdot_of(dv, p[s], c) : (double)p[s];
        }
        lds[l * N + bitrev(x, logN)] = make_double2(v, 0.0);
    }
    __syncthreads();
    lds_fft<true>(lds, N, logN, lpw, tw);
    for (int idx = threadIdx.x; idx < lpw * kc; idx += blockDim.x) {
        const int l = idx / kc, kk = idx - l * kc;
        if (l < nl) Z.row(first + l)[kk] = lds[l * N + k0 + kk];
    }
}

// Second axis (3-D), in place: line (x0, kk), element x1 at Z[(x0 N + x1) kc + kk].
__global__ __launch_bounds__(kSpecThreads) void spec_mid_kernel(int N, int logN, const double2 *__restrict__ tw,
                                                               ZBuf Z, int lpw)
{
    extern __shared__ double2 lds[];
    const int kc = Z.kc;
    const long long lines = (long long)N * kc;
    const long long first = xcd_contiguous(blockIdx.x, gridDim.x) * lpw;
    const int nl = (int)min((long long)lpw, lines - first);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx % lpw, x1 = idx / lpw;
        double2 v = make_double2(0.0, 0.0);
        if (l < nl) {
            const long long line = first + l;
            const long long x0 = line / kc, kk = line % kc;
            v = Z.row(x0 * N + x1)[kk];
        }
        lds[l * N + bitrev(x1, logN)] = v;
    }
    __syncthreads();
    lds_fft<true>(lds, N, logN, lpw, tw);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx % lpw, n1 = idx / lpw;
        if (l < nl) {
            const long long line = first + l;
            const long long x0 = line / kc, kk = line % kc;
            Z.row(x0 * N + n1)[kk] = lds[l * N + n1];
        }
    }
}

// Segmented inclusive sums over the wavefront of runs of equal (non-
// decreasing) keys; the last lane of each run adds the run's totals to the
// histograms.  Called by all 64 lanes of one wavefront.
__device__ inline void bin_add(int key, double v, unsigned w, double *hp, unsigned *hc)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ko = __shfl_up(key, off, 64);
        const double vo = __shfl_up(v, off, 64);
        const unsigned wo = __shfl_up(w, off, 64);
        if (lane >= off && ko == key) {
            v += vo;
            w += wo;
        }
    }
    const int kn = __shfl_down(key, 1, 64);
    if (key >= 0 && (lane == 63 || kn != key)) {
        hp[key] += v;
        hc[key] += w;
    }
}

// Adds one transformed line (first-axis values x[0..N), natural order) to the
// histograms: the wavefront wv < nwb bins its contiguous part of the line's
// walk, whose elements come in order of |n0| (0, 1, -1, 2, -2, ..., -N/2) so
// that the bins are non-decreasing along it.  dims 3: line = n1 kc + kk;
// dims 2: line = kk.
__device__ inline void bin_line(const double2 *x, long long line, int dims, int N, int k0, int kc, int nwb, int wv,
                                double inv_norm, double *hp, unsigned *hc)
{
    const int halfN = N / 2;
    long long base2;
    int klast;
    if (dims == 3) {
        const int n1i = (int)(line / kc);
        const int n1 = n1i < halfN ? n1i : n1i - N;
        klast = k0 + (int)(line % kc);
        base2 = (long long)n1 * n1 + (long long)klast * klast;
    } else {
        klast = k0 + (int)line;
        base2 = (long long)klast * klast;
    }
    const unsigned wt = (klast == 0 || klast == halfN) ? 1u : 2u;
    const int seg = N / nwb;   // this wavefront's part of the walk
    const int e_end = (wv + 1) * seg;
    for (int e0 = wv * seg; e0 < e_end; e0 += 64) {
        const int e = e0 + (int)(threadIdx.x & 63);
        int key = -1;   // lanes past the part's end add nothing
        double v = 0.0;
        unsigned w = 0u;
        if (e < e_end) {
            const int pidx = e == 0 ? 0 : ((e & 1) ? (e + 1) >> 1 : N - (e >> 1));
            const int n0 = pidx < halfN ? pidx : pidx - N;
            const double2 X = x[pidx];
            key = isqrt_ll((long long)n0 * n0 + base2);
            v = (double)wt * (X.x * X.x + X.y * X.y) * inv_norm;
            w = wt;
        }
        bin_add(key, v, w, hp, hc);
    }
}

// First axis and binning.  dims 3: line (n1, kk), element x0 at
// Z[(x0 N + n1) kc + kk]; dims 2: line kk, element x0 at Z[x0 kc + kk];
// dims 1: the kc values of Z are the spectrum itself (no transform).
// partial[g][0..nb) accumulates the power, partial[g][nb..2nb) the counts.
// nwb wavefronts bin each line, wavefront w the w-th contiguous part of the
// line's walk, each into its own histogram; the block adds them in order.
//
// Order of the lines: an element read is 16 bytes of a 128-byte line of Z,
// whose other bytes belong to the neighbouring lines.  Each XCD (block b runs
// on XCD b % 8) takes one contiguous range of line groups and deals it out
// round-robin to its blocks, so the blocks running together on one L2 work
// on neighbouring lines and use each fetched line of Z whole.
__global__ __launch_bounds__(kSpecThreads) void spec_final_kernel(int dims, int N, int logN, int k0, int nb,
                                                                 double inv_norm, const double2 *__restrict__ tw,
                                                                 ZBuf Z, double *__restrict__ partial, int lpw,
                                                                 int nwb)
{
    const int kc = Z.kc;
    extern __shared__ double2 lds[];
    double *hp_all = reinterpret_cast<double *>(lds + lpw * N);   // [nwb][nb]
    unsigned *hc_all = reinterpret_cast<unsigned *>(hp_all + nwb * nb);  // [nwb][nb]
    for (int j = threadIdx.x; j < nwb * nb; j += blockDim.x) {
        hp_all[j] = 0.0;
        hc_all[j] = 0u;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    double *hp = hp_all + min(wv, nwb - 1) * nb;
    unsigned *hc = hc_all + min(wv, nwb - 1) * nb;
    const int halfN = N / 2;
    if (dims == 1) {
        // one line: k_last = k0 + kk, increasing
        if (blockIdx.x == 0 && threadIdx.x < 64) {
            for (int base = 0; base < kc; base += 64) {
                const int kk = base + (int)threadIdx.x;
                int key = -1;
                double v = 0.0;
                unsigned w = 0u;
                if (kk < kc) {
                    const int k = k0 + kk;
                    const unsigned wt = (k == 0 || k == halfN) ? 1u : 2u;
                    const double2 X = Z.row(0)[kk];
                    key = k;
                    v = (double)wt * (X.x * X.x + X.y * X.y) * inv_norm;
                    w = wt;
                }
                bin_add(key, v, w, hp, hc);
            }
        }
    } else {
        const long long lines = dims == 3 ? (long long)N * kc : (long long)kc;
        const long long groups = (lines + lpw - 1) / lpw;
        // this XCD's blocks: nx of them, the first at position vx of the
        // XCD-contiguous numbering; this block is the i-th
        const long long nblk = gridDim.x, nq = nblk / 8, nr = nblk % 8;
        const long long x = blockIdx.x % 8, i = blockIdx.x / 8;
        const long long nx = nq + (x < nr ? 1 : 0);
        const long long vx = x * nq + (x < nr ? x : nr);
        // groups split over the blocks in XCD-contiguous order; the XCD's
        // range is the union of its blocks' shares
        const long long per = groups / nblk, extra = groups % nblk;
        auto start_of = [&](long long v) { return v * per + (v < extra ? v : extra); };
        const long long g0 = start_of(vx), g1 = start_of(vx + nx);
        for (long long q = g0 + i; q < g1; q += nx) {
            const long long first = q * lpw;
            const int nl = (int)min((long long)lpw, lines - first);
            for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
                const int l = idx % lpw, x0 = idx / lpw;
                double2 val = make_double2(0.0, 0.0);
                if (l < nl) {
                    // 3-D: line = n1 kc + kk, element x0 in row x0 N + n1; 2-D: line kk, row x0
                    const long long line = first + l;
                    val = dims == 3 ? Z.row((long long)x0 * N + line / kc)[line % kc] : Z.row(x0)[line];
                }
                lds[l * N + bitrev(x0, logN)] = val;
            }
            __syncthreads();
            lds_fft<true>(lds, N, logN, lpw, tw);
            if (wv < nwb)
                for (int l = 0; l < nl; l++)
                    bin_line(lds + l * N, first + l, dims, N, k0, kc, nwb, wv, inv_norm, hp, hc);
            __syncthreads();
        }
    }
    __syncthreads();
    double *mine = partial + (size_t)blockIdx.x * 2 * nb;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
        double pw = 0.0;
        unsigned long long cnt = 0;
        for (int w = 0; w < nwb; w++) {
            pw += hp_all[w * nb + j];
            cnt += hc_all[w * nb + j];
        }
        mine[j] += pw;
        mine[nb + j] += (double)cnt;
    }
}

// Sum of the blocks' partial histograms, deterministic: 64 output values per
// block, one per lane; wavefront w adds the w-th contiguous range of blocks in
// order, and the wavefronts' sums are added in order.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void spec_reduce_kernel(const double *__restrict__ partial, int groups,
                                                                    int nb, double *__restrict__ out)
{
    __shared__ double red[kReduceThreads / 64][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const int per = (groups + nw - 1) / nw;
    const int g0 = min(groups, wv * per), g1 = min(groups, g0 + per);
    double acc = 0.0;
    if (j < 2 * nb)
        for (int g = g0; g < g1; g++) acc += partial[(size_t)g * 2 * nb + j];
    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && j < 2 * nb) {
        double t = red[0][lane];
        for (int w = 1; w < nw; w++) t += red[w][lane];
        out[j] = t;
    }
}

}  // namespace

extern "C" {

ce_status ce_spectrum_bins(const ce_sim *s, int32_t *nbins)
{
    if (!s || !nbins) return fail(CE_EINVAL, "NULL argument");
    *nbins = nbins_of(s->p.dims, s->p.N);
    return CE_OK;
}

ce_status ce_spectrum(ce_sim *s, int32_t field, double *power_f, double *power_fdot, double *count)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    if (s->loaded != (1u << s->p.nfields) - 1) return fail(CE_ESTATE, "fields not loaded");
    if (field < 0 || field >= s->p.nfields) return fail(CE_EINVAL, "field %d out of range", field);
    const int N = s->p.N, dims = s->p.dims;
    if (N > kMaxSpecN || (N & (N - 1)) != 0)
        return fail(CE_EINVAL, "spectra need N a power of two <= %d (got %d)", kMaxSpecN, N);
    int logN = 0;
    while ((1 << logN) < N) logN++;
    const int nb = nbins_of(dims, N);
    const int M = N / 2 + 1;
    long long rows = 1;
    for (int d = 1; d < dims; d++) rows *= N;
    // scratch: the transform buffer takes the two free ping-pong blocks (rows
    // split between them) when the partial histograms fit the staging chunk,
    // else one block, the other holding the partial histograms.  When the
    // buffer cannot hold all N/2 + 1 columns of every row, k_last is done in
    // chunks of kc columns.  The partial-sum buffer holds the twiddles and the
    // result.
    const int spare = 1 - s->cur;
    const size_t block = (size_t)s->p.nfields * s->lay.field_bytes;
    double2 *za = static_cast<double2 *>(s->lat.d[spare][0]);
    double2 *zb = static_cast<double2 *>(s->lat.p[spare][0]);
    const size_t staging_bytes = (size_t)s->lay.staging_elems * sizeof(double);
    const int lpw = spec_lines(N);
    const int lpw_final = spec_final_lines(N);
    const int lpw_mid = spec_mid_lines(N);
    auto groups_for = [&](int kc_) -> long long {
        const long long lines = dims == 3 ? (long long)N * kc_ : dims == 2 ? kc_ : 1;
        return dims == 1 ? 1 : (lines + lpw_final - 1) / lpw_final;
    };
    const size_t row_bytes_m = (size_t)M * sizeof(double2);
    const long long rows_a_m = (long long)(block / row_bytes_m);
    const bool split = rows_a_m + (long long)(block / row_bytes_m) >= rows &&
                       staging_bytes >= (size_t)2 * nb * sizeof(double);
    int kc;
    long long rows_a;
    double *partial;
    size_t stage_bytes;
    if (split) {
        kc = M;
        rows_a = std::min(rows_a_m, rows);
        partial = s->staging;
        stage_bytes = staging_bytes;
    } else {
        kc = (int)std::min<long long>(M, (long long)(block / ((size_t)rows * sizeof(double2))));
        rows_a = rows;
        const bool partial_in_block = block > staging_bytes;
        partial = partial_in_block ? reinterpret_cast<double *>(zb) : s->staging;
        stage_bytes = partial_in_block ? block : staging_bytes;
    }
    if (kc < 1) return fail(CE_EINVAL, "lattice too small for the spectrum scratch");
    const long long groups_needed = groups_for(kc);
    int G = (int)std::min<long long>({groups_needed, (long long)kMaxGroups,
                                      (long long)(stage_bytes / ((size_t)2 * nb * sizeof(double)))});
    if (G < 1) return fail(CE_EINVAL, "lattice too small for the spectrum scratch");
    if (dims == 1) G = 1;
    static_assert(kOutOffset >= (size_t)kMaxSpecN / 2 * sizeof(double2), "twiddles fit below the result");
    if (kOutOffset + (size_t)2 * nbins_of(3, kMaxSpecN) * sizeof(double) >
        (size_t)kMaxBlocks * kMaxSums * sizeof(double))
        return fail(CE_EDEVICE, "spectrum result does not fit the partial-sum buffer");
    char *pbase = reinterpret_cast<char *>(s->lat.partials);
    double2 *tw = reinterpret_cast<double2 *>(pbase + kTwOffset);
    double *out = reinterpret_cast<double *>(pbase + kOutOffset);
    hipStream_t st = s->stream;
    const size_t lds_line = (size_t)lpw * N * sizeof(double2);
    const size_t lds_mid = (size_t)lpw_mid * N * sizeof(double2);
    // as many binning wavefronts (2 or 1) as leave the block within 40 KiB of
    // LDS, so that four blocks fit a compute unit (1024^3: 8.4 ms per
    // first-axis pass, against 10.9 ms with four wavefronts at two blocks per
    // unit and 10.3 ms with one at six)
    int nwb = 1;
    for (int w = 2; w >= 1; w /= 2)
        if ((size_t)lpw_final * N * sizeof(double2) + (size_t)w * nb * (sizeof(double) + sizeof(unsigned)) <= 40960) {
            nwb = w;
            break;
        }
    const size_t lds_final =
        (size_t)lpw_final * N * sizeof(double2) + (size_t)nwb * nb * (sizeof(double) + sizeof(unsigned));
    const double inv_norm = 1.0 / pow((double)N, 2.0 * dims);
    const bool fp64 = s->p.precision == CE_FP64;

    CE_HIP(launch_twiddles(tw, N, st));
    for (int which = 0; which < 2; which++) {
        double *dst = which == 0 ? power_f : power_fdot;
        if (!dst && !(which == 0 && count)) continue;
        CE_HIP(hipMemsetAsync(partial, 0, (size_t)G * 2 * nb * sizeof(double), st));
        for (int k0 = 0; k0 < M; k0 += kc) {
            const int kcc = std::min(kc, M - k0);
            ZBuf Z;
            Z.a = za;
            Z.b = zb;
            Z.rows_a = rows_a;
            Z.kc = kcc;
            const dim3 blk(kSpecThreads);
            const dim3 grows((unsigned)((rows + lpw - 1) / lpw));
            if (fp64)
                hipLaunchKernelGGL(spec_rows_kernel<double>, grows, blk, lds_line, st,
                                   static_cast<const double *>(s->lat.d[s->cur][field]),
                                   static_cast<const double *>(s->lat.p[s->cur][field]), s->lat.sc, field, which,
                                   s->started ? 1 : 0, N, logN, rows, k0, tw, Z, lpw);
            else
                hipLaunchKernelGGL(spec_rows_kernel<float>, grows, blk, lds_line, st,
                                   static_cast<const float *>(s->lat.d[s->cur][field]),
                                   static_cast<const float *>(s->lat.p[s->cur][field]), s->lat.sc, field, which,
                                   s->started ? 1 : 0, N, logN, rows, k0, tw, Z, lpw);
            CE_HIP(hipGetLastError());
            if (dims == 3) {
                const long long mid_lines = (long long)N * kcc;
                hipLaunchKernelGGL(spec_mid_kernel, dim3((unsigned)((mid_lines + lpw_mid - 1) / lpw_mid)), blk, lds_mid,
                                   st, N, logN, tw, Z, lpw_mid);
                CE_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(spec_final_kernel, dim3(G), blk, lds_final, st, dims, N, logN, k0, nb, inv_norm,
                               tw, Z, partial, lpw_final, nwb);
            CE_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(spec_reduce_kernel, dim3((2 * nb + 63) / 64), dim3(kReduceThreads), 0, st, partial, G, nb,
                           out);
        CE_HIP(hipGetLastError());
        if (dst) CE_HIP(hipMemcpyAsync(dst, out, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, st));
        if (which == 0 && count)
            CE_HIP(hipMemcpyAsync(count, out + nb, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, st));
        CE_HIP(hipStreamSynchronize(st));
    }
    return CE_OK;
}

}  // extern "C"
