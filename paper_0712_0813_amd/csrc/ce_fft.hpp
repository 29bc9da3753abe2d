// Radix-2 FFT of FP64 complex lines held in LDS, shared by the device-side
// initial conditions and the spectra.
#pragma once

#include <hip/hip_runtime.h>

namespace ce {
namespace fft {

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 w, double2 b)  // conj(w) * b
{
    return make_double2(w.x * b.x + w.y * b.y, w.x * b.y - w.y * b.x);
}

__device__ inline int bitrev(int p, int logN) { return (int)(__brev((unsigned)p) >> (32 - logN)); }

// In-place DFT of `lines` lines of N values (N = 2^logN) held bit-reversed in
// LDS: sum_p v_p e^{s 2 pi i p x / N}, s = +1 (inverse, kForward false) or -1,
// no normalisation.  tw[q] = e^{2 pi i q/N} for q < N/2.  Every thread of the
// block must call it (it synchronises after each pass).
//
// Radix-2 decimation in time, two stages per pass: the four values
// i0, i0+h, i0+2h, i0+3h (i0 mod 4h < h) are closed under the stages of
// half-size h and 2h, so one thread takes them through both in registers.
// The arithmetic is exactly that of two separate radix-2 stages; only the
// LDS round trips and barriers are halved.
template <bool kForward>
__device__ void lds_fft(double2 *buf, int N, int logN, int lines, const double2 *__restrict__ tw)
{
    auto twiddled = [](double2 w, double2 v) { return kForward ? cmulc(w, v) : cmul(w, v); };
    int s = 0, half = 1;
    for (; s + 1 < logN; s += 2, half <<= 2) {
        const int quarterN = N >> 2;
        const int total = lines * quarterN;
        const int sh0 = logN - 1 - s, sh1 = logN - 2 - s;  // twiddle index j N / (2 h) and j' N / (4 h)
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int line = idx >> (logN - 2);
            const int b = idx & (quarterN - 1);
            const int j = b & (half - 1);
            const int i0 = ((b >> s) << (s + 2)) + j;
            double2 *x = buf + line * N;
            const double2 x0 = x[i0], x1 = x[i0 + half], x2 = x[i0 + 2 * half], x3 = x[i0 + 3 * half];
            const double2 w = tw[j << sh0];
            double2 t = twiddled(w, x1);
            const double2 y0 = cadd(x0, t), y1 = csub(x0, t);
            t = twiddled(w, x3);
            const double2 y2 = cadd(x2, t), y3 = csub(x2, t);
            t = twiddled(tw[j << sh1], y2);
            x[i0] = cadd(y0, t);
            x[i0 + 2 * half] = csub(y0, t);
            t = twiddled(tw[(j + half) << sh1], y3);
            x[i0 + half] = cadd(y1, t);
            x[i0 + 3 * half] = csub(y1, t);
        }
        __syncthreads();
    }
    if (s < logN) {
        // odd logN: one radix-2 stage of half-size h = N/2 left
        const int halfN = N >> 1;
        const int total = lines * halfN;
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int line = idx >> (logN - 1);
            const int j = idx & (halfN - 1);
            double2 *x = buf + line * N;
            const double2 t = twiddled(tw[j], x[j + half]);
            const double2 a = x[j];
            x[j] = cadd(a, t);
            x[j + half] = csub(a, t);
        }
        __syncthreads();
    }
}

// Blocks are dealt round-robin over the 8 XCDs (block b on XCD b % 8), each
// with its own L2.  Renumbering so that every XCD's blocks take one
// contiguous range keeps neighbouring lines (which share cache lines when a
// line's elements are strided) on one L2.  A bijection of [0, nblocks).
__device__ inline long long xcd_contiguous(long long b, long long nblocks)
{
    const long long q = nblocks / 8, r = nblocks % 8;
    const long long x = b % 8, i = b / 8;
    return x * q + (x < r ? x : r) + i;
}

// tw[q] = e^{2 pi i q/N}, q < N/2 (N a power of two).
hipError_t launch_twiddles(double2 *tw, int N, hipStream_t st);

}  // namespace fft
}  // namespace ce
