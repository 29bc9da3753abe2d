// Seeded Gaussian-random-field initial conditions generated on the device.
// The definition (mode amplitudes from Philox4x64-10 and Box-Muller, the
// band |n| <= N/4, the spectrum sigma_n, delta = Re sum_n c_n e^{2 pi i n.x/N})
// is stated with ce_init_spec in ce.h.
//
// The sum is evaluated as band-limited inverse FFTs, one axis at a time, on
// the Hermitian part H_n = (c_n + conj(c_{-n}))/2 (whose full sum is real and
// equals Re sum_n c_n e^{...}), keeping only the n_last >= 0 half:
//   3-D: modes (n0 in [-K,K], n1 in [-K,K], m in [0,K])
//        -> axis 0 (generated on the fly)  Y[x0][n1][m]
//        -> axis 1, in chunks of x0 rows   Z[x0][x1][m]
//        -> last axis, real part, weights 1 (m = 0) and 2 (m > 0), stored
//           straight into the storage arrays;
//   2-D: the same without the middle axis; 1-D: the last axis only.
// Each line transform is an in-place radix-2 FFT in LDS (ce_fft.hpp) with a
// table of N/2 FP64 twiddles.  Only the band (N/2 + 1 of N inputs per line)
// is read.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "ce_fft.hpp"

#include "ce_sim.hpp"

using namespace ce;
using namespace ce::host;
using namespace ce::fft;

namespace {

constexpr int kGenThreads = 256;
constexpr int kMaxGenN = 2048;
// complex values of LDS per workgroup (32 KiB): 2048 / N lines
constexpr int kLdsLines = 2048;

static_assert((size_t)kMaxBlocks * kMaxSums * sizeof(double) >= (size_t)kMaxGenN / 2 * 16,
              "the twiddle table lives in the partial-sum buffer");

struct GrfArgs {
    unsigned long long seed;
    int stream;            // 2 * field + kind
    int kind;              // 0: field, 1: time derivative
    int dims, N, K, logN;
    double k_unit;         // 2 pi / L
    double m_eff2;
    double amp;
    double inv_sqrt_vol;   // 1 / sqrt(L^dims)
};

// Philox4x64-10 (Salmon et al., SC 2011): round multipliers and Weyl key
// increments as published.
__device__ inline void philox4x64_10(unsigned long long c[4], unsigned long long k0, unsigned long long k1)
{
    const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const unsigned long long hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const unsigned long long hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const unsigned long long n0 = hi1 ^ c[1] ^ k0;
        const unsigned long long n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// c_n for the wave vector n[0..dims): sigma_n (X + iY), 0 outside the band.
__device__ double2 mode_amp(const GrfArgs &g, const int *n)
{
    long long n2 = 0, b = 0;
    const int W = 2 * g.K + 1;
    for (int j = 0; j < g.dims; j++) {
        n2 += (long long)n[j] * n[j];
        b = b * W + (n[j] + g.K);
    }
    if (n2 == 0 || n2 > (long long)g.K * g.K) return make_double2(0.0, 0.0);
    unsigned long long c[4] = {(unsigned long long)b, (unsigned long long)g.stream, 0ULL, 0ULL};
    philox4x64_10(c, g.seed, 0ULL);
    const double u1 = (double)((c[0] >> 11) + 1) * 0x1.0p-53;
    const double u2 = (double)(c[1] >> 11) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    const double k = g.k_unit * sqrt((double)n2);
    const double omega = sqrt(k * k + g.m_eff2);
    const double sigma = g.kind == 0 ? g.amp / sqrt(2.0 * omega) * g.inv_sqrt_vol
                                     : g.amp * sqrt(omega / 2.0) * g.inv_sqrt_vol;
    return make_double2(sigma * r * cs, sigma * r * sn);
}

// H_n = (c_n + conj(c_{-n})) / 2
__device__ double2 hermitian_mode(const GrfArgs &g, const int *n)
{
    int m[3];
    for (int j = 0; j < g.dims; j++) m[j] = -n[j];
    const double2 a = mode_amp(g, n), b = mode_amp(g, m);
    return make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
}

// First axis (dims 2 or 3), modes generated in place.  Line l: 3-D
// (n1 = l / (K+1) - K, m = l % (K+1)); 2-D m = l.  Output Y[x0 * lines + l].
__global__ __launch_bounds__(kGenThreads) void gen_axis0_kernel(GrfArgs g, const double2 *__restrict__ tw,
                                                               double2 *__restrict__ Y, int lines, int lpw)
{
    extern __shared__ double2 lds[];
    const int N = g.N, K = g.K;
    const int first = (int)xcd_contiguous(blockIdx.x, gridDim.x) * lpw;
    const int nl = min(lpw, lines - first);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx % lpw, p = idx / lpw;
        double2 v = make_double2(0.0, 0.0);
        const int n0 = p <= N / 2 ? p : p - N;
        if (l < nl && n0 >= -K && n0 <= K) {
            const int line = first + l;
            int n[3];
            n[0] = n0;
            if (g.dims == 3) {
                n[1] = line / (K + 1) - K;
                n[2] = line % (K + 1);
            } else {
                n[1] = line;
            }
            v = hermitian_mode(g, n);
        }
        lds[l * N + bitrev(p, g.logN)] = v;
    }
    __syncthreads();
    lds_fft<false>(lds, N, g.logN, lpw, tw);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx % lpw, x0 = idx / lpw;
        if (l < nl) Y[(long long)x0 * lines + first + l] = lds[l * N + x0];
    }
}

// Middle axis (3-D): rows x0 in [r0, r0 + rows); line (r, m), m fastest.
// In Y[x0][n1 + K][m], out Z[r][x1][m].
__global__ __launch_bounds__(kGenThreads) void axis1_kernel(GrfArgs g, const double2 *__restrict__ tw,
                                                           const double2 *__restrict__ Y, double2 *__restrict__ Z,
                                                           int r0, int rows, int lpw)
{
    extern __shared__ double2 lds[];
    const int N = g.N, K = g.K, M = K + 1, W = 2 * K + 1;
    const int lines = rows * M;
    const int first = (int)xcd_contiguous(blockIdx.x, gridDim.x) * lpw;
    const int nl = min(lpw, lines - first);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx % lpw, p = idx / lpw;
        double2 v = make_double2(0.0, 0.0);
        const int n1 = p <= N / 2 ? p : p - N;
        if (l < nl && n1 >= -K && n1 <= K) {
            const int line = first + l;
            const int r = line / M, m = line % M;
            v = Y[((long long)(r0 + r) * W + (n1 + K)) * M + m];
        }
        lds[l * N + bitrev(p, g.logN)] = v;
    }
    __syncthreads();
    lds_fft<false>(lds, N, g.logN, lpw, tw);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx % lpw, x1 = idx / lpw;
        if (l < nl) {
            const int line = first + l;
            const int r = line / M, m = line % M;
            Z[((long long)r * N + x1) * M + m] = lds[l * N + x1];
        }
    }
}

// Last axis: row r of Z (K+1 values, or the generated 1-D modes when Z is
// NULL) -> out[(row0 + r) * N + x] = (T)(Re sum + store_shift); the largest
// |Re sum + phys_shift| (NaN as +inf) goes to *maxabs_bits.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void last_axis_kernel(GrfArgs g, const double2 *__restrict__ tw,
                                                               const double2 *__restrict__ Z, int rows,
                                                               long long row0, T *__restrict__ out,
                                                               double store_shift, double phys_shift,
                                                               unsigned int *maxabs_bits, int lpw)
{
    extern __shared__ double2 lds[];
    __shared__ float red[kGenThreads / 64];
    const int N = g.N, K = g.K, M = K + 1;
    const int first = blockIdx.x * lpw;
    const int nl = min(lpw, rows - first);
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx >> g.logN, p = idx & (N - 1);
        double2 v = make_double2(0.0, 0.0);
        if (l < nl && p <= K) {
            if (Z) {
                v = Z[(long long)(first + l) * M + p];
            } else {
                int n[1] = {p};
                v = hermitian_mode(g, n);
            }
            if (p > 0) v = make_double2(2.0 * v.x, 2.0 * v.y);
        }
        lds[l * N + bitrev(p, g.logN)] = v;
    }
    __syncthreads();
    lds_fft<false>(lds, N, g.logN, lpw, tw);
    float mx = 0.0f;
    for (int idx = threadIdx.x; idx < lpw * N; idx += blockDim.x) {
        const int l = idx >> g.logN, x = idx & (N - 1);
        if (l < nl) {
            const double v = lds[l * N + x].x;
            out[(row0 + first + l) * N + x] = (T)(v + store_shift);
            const double ph = v + phys_shift;
            mx = fmaxf(mx, isnan(ph) ? INFINITY : (float)fabs(ph));
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = red[0];
        for (int w = 1; w < kGenThreads / 64; w++) b = fmaxf(b, red[w]);
        atomicMax(maxabs_bits, __float_as_uint(b));
    }
}

int lines_per_group(int N) { return std::max(1, kLdsLines / N); }

size_t lds_bytes(int N) { return (size_t)lines_per_group(N) * N * sizeof(double2); }

struct Region {
    char *p;
    size_t bytes;
};

// Generate one array (field i, kind) into dst.
ce_status generate_array(ce_sim *s, const GrfArgs &g, const double2 *tw, Region yreg, Region zreg, int zrows,
                         void *dst, double store_shift, double phys_shift, unsigned int *maxabs)
{
    const int N = g.N, K = g.K, M = K + 1;
    const int lpw = lines_per_group(N);
    const size_t lds = lds_bytes(N);
    const dim3 blk(kGenThreads);
    hipStream_t st = s->stream;
    const bool fp64 = s->p.precision == CE_FP64;
    auto last = [&](const double2 *Zp, int rows, long long row0) {
        const dim3 grd((rows + lpw - 1) / lpw);
        if (fp64)
            hipLaunchKernelGGL(last_axis_kernel<double>, grd, blk, lds, st, g, tw, Zp, rows, row0,
                               static_cast<double *>(dst), store_shift, phys_shift, maxabs, lpw);
        else
            hipLaunchKernelGGL(last_axis_kernel<float>, grd, blk, lds, st, g, tw, Zp, rows, row0,
                               static_cast<float *>(dst), store_shift, phys_shift, maxabs, lpw);
        return hipGetLastError();
    };
    if (g.dims == 1) {
        CE_HIP(last(nullptr, 1, 0));
        return CE_OK;
    }
    double2 *Y = reinterpret_cast<double2 *>(yreg.p);
    const int lines0 = g.dims == 3 ? (2 * K + 1) * M : M;
    hipLaunchKernelGGL(gen_axis0_kernel, dim3((lines0 + lpw - 1) / lpw), blk, lds, st, g, tw, Y, lines0, lpw);
    CE_HIP(hipGetLastError());
    if (g.dims == 2) {
        CE_HIP(last(Y, N, 0));
        return CE_OK;
    }
    double2 *Z = reinterpret_cast<double2 *>(zreg.p);
    for (int r0 = 0; r0 < N; r0 += zrows) {
        const int rows = std::min(zrows, N - r0);
        const int lines1 = rows * M;
        hipLaunchKernelGGL(axis1_kernel, dim3((lines1 + lpw - 1) / lpw), blk, lds, st, g, tw, Y, Z, r0, rows, lpw);
        CE_HIP(hipGetLastError());
        CE_HIP(last(Z, rows * N, (long long)r0 * N));
    }
    return CE_OK;
}

bool finite_nonneg(double v) { return isfinite(v) && v >= 0.0; }

}  // namespace

namespace ce {
namespace fft {

__global__ __launch_bounds__(kGenThreads) void twiddle_kernel(double2 *tw, int N)
{
    const int q = blockIdx.x * kGenThreads + threadIdx.x;
    if (q < N / 2) {
        double sn, cs;
        sincospi(2.0 * (double)q / (double)N, &sn, &cs);
        tw[q] = make_double2(cs, sn);
    }
}

hipError_t launch_twiddles(double2 *tw, int N, hipStream_t st)
{
    hipLaunchKernelGGL(twiddle_kernel, dim3((N / 2 + kGenThreads - 1) / kGenThreads), dim3(kGenThreads), 0, st, tw,
                       N);
    return hipGetLastError();
}

}  // namespace fft
}  // namespace ce

namespace {

// Scratch of ce_generate_fields_noalloc: the transform intermediates of one
// call live in this file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it only stands in for the symbol); it looks up each device's address
// once with hipGetSymbolAddress and uses that.
constexpr size_t kGenScratchBytes = (size_t)CE_GEN_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kGenScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device (looked up on first use there).
ce_status scratch_on_device(char **out)
{
    int dev = -1;
    CE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CE_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(CE_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return CE_OK;
}

// Both entry points: validate, place the transform intermediates (the
// simulation's spare buffers, a temporary for lattices too small for them,
// or, with `noalloc`, the static scratch), generate every array, start.
ce_status generate(ce_sim *s, const ce_init_spec *spec, bool noalloc)
{
    if (!s || !spec) return fail(CE_EINVAL, "NULL argument");
    if (s->started) return fail(CE_ESTATE, "fields already loaded and evolved");
    const int N = s->p.N, dims = s->p.dims, nf = s->p.nfields;
    if (N > kMaxGenN || (N & (N - 1)) != 0)
        return fail(CE_EINVAL, "device generation needs N a power of two <= %d (got %d)", kMaxGenN, N);
    if (!finite_nonneg(spec->amp)) return fail(CE_EINVAL, "amp must be finite and >= 0");
    for (int i = 0; i < nf; i++) {
        if (!isfinite(spec->background[i]) || !isfinite(spec->background_dot[i]))
            return fail(CE_EINVAL, "background values must be finite");
        if (!finite_nonneg(spec->m_eff2[i])) return fail(CE_EINVAL, "m_eff2[%d] must be finite and >= 0", i);
    }
    const int K = N / 4, M = K + 1;
    int logN = 0;
    while ((1 << logN) < N) logN++;

    const size_t ybytes = dims == 3 ? (size_t)N * (2 * K + 1) * M * sizeof(double2)
                                    : dims == 2 ? (size_t)N * M * sizeof(double2) : 0;
    const size_t rowbytes = dims == 3 ? (size_t)N * M * sizeof(double2) : 0;
    Region yreg{nullptr, 0}, zreg{nullptr, 0};
    int zrows = 0;
    char *temp = nullptr;
    if (noalloc) {
        // intermediates after the first axis, then as many rows of the
        // second axis as fit (the last axis works through them in chunks)
        const size_t yoff = (ybytes + kAlign - 1) / kAlign * kAlign;
        if (dims >= 2 && yoff + rowbytes > kGenScratchBytes)
            return fail(CE_EINVAL,
                        "N = %d in %d dimensions needs %zu bytes of scratch, more than the %zu of "
                        "ce_generate_fields_noalloc (use ce_generate_fields)",
                        N, dims, yoff + rowbytes, kGenScratchBytes);
        char *base = nullptr;
        const ce_status st = scratch_on_device(&base);
        if (st != CE_OK) return st;
        yreg = Region{base, ybytes};
        if (dims == 3) {
            zrows = (int)std::min<size_t>(N, (kGenScratchBytes - yoff) / rowbytes);
            zreg = Region{base + yoff, (size_t)zrows * rowbytes};
        }
    } else {
        // scratch: the second ping-pong buffers and the staging chunk are
        // unused until the run starts
        const size_t block = (size_t)nf * s->lay.field_bytes;
        const int spare = 1 - s->cur;
        Region regs[3] = {{static_cast<char *>(s->lat.d[spare][0]), block},
                          {static_cast<char *>(s->lat.p[spare][0]), block},
                          {reinterpret_cast<char *>(s->staging), (size_t)s->lay.staging_elems * sizeof(double)}};
        if (dims == 2) {
            for (const Region &r : regs)
                if (r.bytes >= ybytes && (!yreg.p || r.bytes < yreg.bytes)) yreg = r;
        } else if (dims == 3) {
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    if (a == b || regs[a].bytes < ybytes) continue;
                    const int rows = (int)std::min<size_t>(N, regs[b].bytes / rowbytes);
                    if (rows > zrows) {
                        zrows = rows;
                        yreg = regs[a];
                        zreg = regs[b];
                    }
                }
            if (zrows < 1) yreg.p = nullptr;
        }
        if (dims >= 2 && !yreg.p) {
            // lattices too small to hold the scratch in their own buffers
            const size_t zb = dims == 3 ? rowbytes * N : 0;
            CE_HIP(hipMalloc(&temp, ybytes + zb));
            yreg = Region{temp, ybytes};
            zreg = Region{temp + ybytes, zb};
            zrows = N;
        }
    }
    const double2 *tw = reinterpret_cast<const double2 *>(s->lat.partials);

    ce_status st = CE_OK;
    auto run = [&]() -> ce_status {
        CE_HIP(hipMemsetAsync(s->maxabs, 0, kAlign, s->stream));
        CE_HIP(launch_twiddles(reinterpret_cast<double2 *>(s->lat.partials), N, s->stream));
        double vol = 1.0;
        for (int d = 0; d < dims; d++) vol *= s->p.L;
        for (int i = 0; i < nf; i++) {
            // the homogeneous reference is the background itself: the
            // fluctuations have no n = 0 mode, so their volume mean is zero
            s->m_host[i] = spec->background[i];
            CE_HIP(hipMemcpyAsync(&s->lat.sc->m[i], &s->m_host[i], sizeof(double), hipMemcpyHostToDevice,
                                  s->stream));
            for (int kind = 0; kind < 2; kind++) {
                GrfArgs g;
                g.seed = spec->seed;
                g.stream = 2 * i + kind;
                g.kind = kind;
                g.dims = dims;
                g.N = N;
                g.K = K;
                g.logN = logN;
                g.k_unit = 2.0 * M_PI / s->p.L;
                g.m_eff2 = spec->m_eff2[i];
                g.amp = spec->amp;
                g.inv_sqrt_vol = 1.0 / sqrt(vol);
                void *dst = kind == 0 ? s->lat.d[s->cur][i] : s->lat.p[s->cur][i];
                const double store_shift = kind == 0 ? 0.0 : spec->background_dot[i];
                const double phys_shift = kind == 0 ? spec->background[i] : spec->background_dot[i];
                ce_status r = generate_array(s, g, tw, yreg, zreg, zrows, dst, store_shift, phys_shift,
                                             kind == 0 ? s->maxabs + i : s->maxabs + 3);
                if (r != CE_OK) return r;
            }
        }
        CE_HIP(hipStreamSynchronize(s->stream));
        return CE_OK;
    };
    st = run();
    if (temp) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipFree(temp);
    }
    if (st != CE_OK) return st;
    s->loaded = (1u << nf) - 1;
    return start_run(s);
}

}  // namespace

extern "C" {

ce_status ce_generate_fields(ce_sim *s, const ce_init_spec *spec)
{
    return generate(s, spec, false);
}

ce_status ce_generate_fields_noalloc(ce_sim *s, const ce_init_spec *spec)
{
    return generate(s, spec, true);
}

}  // extern "C"
