/*
 * Plain FP64 CPU oracle for the seeded Gaussian-random-field initial
 * conditions that the GPU library can generate on the device.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code
 * and no header with the GPU library.
 *
 * Definition (written from the description of the initial spectrum, each
 * mode with a Gaussian complex amplitude, in the workloads' parameters; the
 * paper's programs start from such fluctuations but it states no recipe):
 *   K = N/4; wave vectors n = (n_0, .., n_{d-1}) with integer n_j in [-K, K];
 *   box index b(n) = sum_j (n_j + K) (2K+1)^(d-1-j)   (C order over the box);
 *   random words: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel
 *     random numbers: as easy as 1, 2, 3", SC 2011) with key (seed, 0) and
 *     counter (b(n), stream, 0, 0), stream = 2 * field + kind (kind 0: field,
 *     1: its time derivative); w0, w1 = the first two output words;
 *   uniforms u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1], u2 = (w1 >> 11) 2^-53;
 *   Box-Muller: X = sqrt(-2 ln u1) cos(2 pi u2), Y = sqrt(-2 ln u1) sin(2 pi u2);
 *   c_n = sigma_n (X + i Y) when 0 < |n|^2 <= K^2, else 0, with
 *     k = 2 pi |n| / L, omega = sqrt(k^2 + m_eff2),
 *     sigma_n = amp / sqrt(2 omega L^d)          (kind 0)
 *     sigma_n = amp sqrt(omega / 2) / sqrt(L^d)   (kind 1);
 *   delta(x) = Re sum_n c_n exp(2 pi i n.x / N), x integer site coordinates.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Philox4x64 round multipliers and key increments, from the publication. */
#define PH_M0 0xD2E7470EE14C6C93ULL
#define PH_M1 0xCA5A826395121157ULL
#define PH_W0 0x9E3779B97F4A7C15ULL
#define PH_W1 0xBB67AE8584CAA73BULL

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    const unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* One Philox4x64-10 block: out = bijection_key(ctr). */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(PH_M0, c0, &hi0, &lo0);
        mulhilo64(PH_M1, c2, &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* The two standard normal numbers of mode box index b in `stream`. */
void or_grf_normals(uint64_t seed, int64_t b, int32_t stream, double *X, double *Y)
{
    const uint64_t ctr[4] = {(uint64_t)b, (uint64_t)stream, 0, 0};
    const uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    or_philox4x64_10(ctr, key, w);
    const double u1 = (double)((w[0] >> 11) + 1) * 0x1.0p-53;
    const double u2 = (double)(w[1] >> 11) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(u1));
    const double t = 2.0 * M_PI * u2;
    *X = r * cos(t);
    *Y = r * sin(t);
}

/* sigma_n of a mode with integer |n|^2 = n2 (0 outside the band). */
static double sigma_of(int64_t n2, int32_t K, int32_t dims, double L, int32_t kind, double amp, double m_eff2)
{
    if (n2 <= 0 || n2 > (int64_t)K * K) return 0.0;
    const double k = 2.0 * M_PI * sqrt((double)n2) / L;
    const double omega = sqrt(k * k + m_eff2);
    const double vol = pow(L, dims);
    if (kind == 0) return amp / sqrt(2.0 * omega * vol);
    return amp * sqrt(omega / 2.0) / sqrt(vol);
}

/* c_n over the whole (2K+1)^dims box in C order (re, im: (2K+1)^dims each). */
void or_grf_modes(uint64_t seed, int32_t field, int32_t kind, int32_t dims, int32_t N, double L, double amp,
                  double m_eff2, double *re, double *im)
{
    const int32_t K = N / 4, W = 2 * K + 1;
    int64_t total = 1;
    for (int d = 0; d < dims; d++) total *= W;
    for (int64_t b = 0; b < total; b++) {
        int64_t rest = b, n2 = 0;
        for (int d = dims - 1; d >= 0; d--) {
            const int64_t nj = rest % W - K;
            rest /= W;
            n2 += nj * nj;
        }
        const double s = sigma_of(n2, K, dims, L, kind, amp, m_eff2);
        if (s == 0.0) {
            re[b] = 0.0;
            im[b] = 0.0;
            continue;
        }
        double X, Y;
        or_grf_normals(seed, b, 2 * field + kind, &X, &Y);
        re[b] = s * X;
        im[b] = s * Y;
    }
}

/* delta at `count` sites (C-order site indices) by direct summation over the
 * modes of the box (re, im from or_grf_modes). */
void or_grf_sites(int32_t dims, int32_t N, const double *re, const double *im, int64_t count,
                  const int64_t *sites, double *out)
{
    const int32_t K = N / 4, W = 2 * K + 1;
    int64_t total = 1;
    for (int d = 0; d < dims; d++) total *= W;
    for (int64_t q = 0; q < count; q++) {
        int64_t x[3] = {0, 0, 0}, rest = sites[q];
        for (int d = dims - 1; d >= 0; d--) {
            x[d] = rest % N;
            rest /= N;
        }
        double acc = 0.0;
        for (int64_t b = 0; b < total; b++) {
            if (re[b] == 0.0 && im[b] == 0.0) continue;
            int64_t r2 = b, phase = 0;
            for (int d = dims - 1; d >= 0; d--) {
                const int64_t nj = r2 % W - K;
                r2 /= W;
                phase += nj * x[d];
            }
            /* exact reduction of the phase n.x modulo N before the angle */
            phase %= N;
            if (phase < 0) phase += N;
            const double th = 2.0 * M_PI * (double)phase / (double)N;
            acc += re[b] * cos(th) - im[b] * sin(th);
        }
        out[q] = acc;
    }
}
