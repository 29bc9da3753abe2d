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
// block must call it (it synchronises after each stage).
template <bool kForward>
__device__ void lds_fft(double2 *buf, int N, int logN, int lines, const double2 *__restrict__ tw)
{
    const int halfN = N >> 1;
    const int total = lines * halfN;
    for (int half = 1, s = 0; half < N; half <<= 1, s++) {
        const int tshift = logN - 1 - s;  // twiddle index j * N / (2 half)
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int line = idx >> (logN - 1);
            const int b = idx & (halfN - 1);
            const int j = b & (half - 1);
            const int i0 = ((b - j) << 1) + j;
            double2 *x = buf + line * N;
            const double2 w = tw[j << tshift];
            const double2 t = kForward ? cmulc(w, x[i0 + half]) : cmul(w, x[i0 + half]);
            const double2 a = x[i0];
            x[i0] = cadd(a, t);
            x[i0 + half] = csub(a, t);
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
