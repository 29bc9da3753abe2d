// Internal declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ce.h"

namespace ce {

constexpr int kMaxFields = CE_MAX_FIELDS;
constexpr int kMaxTerms = CE_MAX_TERMS;
// Model of the potential, a compile-time parameter of every pass kernel.
enum ModelKind { kQuartic = CE_MODEL_QUARTIC, kPoly = CE_MODEL_POLYNOMIAL };
constexpr int kLogCap = CE_ENERGY_LOG;
// FP64 volume sums per field (see the kernels for their meaning), plus sum V
constexpr int kSumsPerField = 6;
constexpr int kMaxSums = kSumsPerField * kMaxFields + 1;
constexpr int kBlock = 256;

// Per-field coefficients of one step pass in the storage type T.
template <typename T>
struct PassScalars {
    T beta;                 // deferred c-term coefficient
    T bm[kMaxFields];       // beta * m, rounded once
    T r[kMaxFields];        // reference derivative
    T m1[kMaxFields];       // reference field at n+1, rounded once
    T m2a[kMaxFields];      // a_{n+1}^2 mu2_i
    T hm[kMaxFields];       // a_{n+1}^2 mu2_i / 2
    T tc[kMaxTerms];        // polynomial model: coef_t a_{n+1}^(4 - D_t)
};

// FP64 scalar state of one lattice at integer step n, resident on the device.
//
// Storage split: field i at step n is f_i(x) = m[i] + d_i(x), with the
// homogeneous reference m[i] in FP64 and the deviation d_i in the storage
// type; the derivative at n+1/2 is fdot_i(x) = p_i(x) + beta (m[i] + d_i(x)).
struct Scalars {
    double a;          // a^n
    double a_next;     // a^{n+1} = a^n + dt a'^{n+1/2}
    double adot_half;  // a'^{n+1/2}
    double beta;       // deferred c-term coefficient (see above)
    double tau;
    long long step;
    long long first_bad;            // first step with a non-finite sum, -1 if none
    long long remaining;            // pool members: steps still to take (0: the lattice is idle)
    int cur;                        // pool members: buffer holding the current state
    int pad_cur;
    double m[kMaxFields];           // homogeneous reference of f_i at step n
    double fdot_mean[kMaxFields];   // volume mean of fdot_i^{n+1/2}
    double r[kMaxFields];           // fdot_mean rounded to the storage type
    // Coefficients of the next step pass, derived from the values above by
    // whoever wrote them last (start-up or step tail), in both storage types.
    // Kernels read them with scalar loads.
    PassScalars<float> nxf;
    PassScalars<double> nxd;
    double nx_m1[kMaxFields];       // m + dt r: FP64 reference at n+1
    double nx_hm[kMaxFields];       // a_{n+1}^2 mu2_i / 2
};

// One lattice as the kernels see it.  d[b][i], p[b][i]: buffer b (ping-pong)
// of field i, element type per precision.
struct Lattice {
    void *d[2][kMaxFields];
    void *p[2][kMaxFields];
    int dims, N, nf, expansion;
    long long nsites;
    double dt, inv_dx2, lambda, kappa, vacuum;
    double G[kMaxFields], mu2[kMaxFields];
    float dt_f, inv_dx2_f, lambda_f, G_f[kMaxFields];  // the same, rounded to FP32
    float qlam_f, hG_f[kMaxFields];                     // lambda/4, G/2 in FP32
    // polynomial model: the terms of degree >= 1 (constant terms are summed
    // into `vacuum`): coefficient, exponent per field, total degree
    int model, nterms;
    double tcoef[kMaxTerms];
    int texp[kMaxTerms][kMaxFields];
    int tdeg[kMaxTerms];
    Scalars *sc;
    double *partials;      // [kMaxSums][slots]: per sum, one entry per block or per tile (tiled pass)
    unsigned int *ticket;  // last-block counter, then the tiled pass's tile counters; 0 between launches
    int slots;             // entries per sum in `partials` (at least kMaxBlocks)
    ce_energy *ring;       // [kLogCap]
    int nblocks;           // blocks of the step launch (fixed per lattice)
    int kind;              // kDirect or kTiled3d
    int vec;               // tiled: consecutive x sites per thread (2 or 4)
    int lpr;               // tiled: threads per tile row (tile is vec*lpr x bs/lpr sites)
    int bs;                // tiled: threads per block
    int zc;                // tiled: planes streamed per tile; 2-D streaming: rows per unit
    int first_block;       // batched launches: this lattice's first block
};

enum Kind { kDirect = 0, kTiled3d = 1, kStream2d = 2 };
constexpr int kMaxBlocks = 4096;  // blocks per launch; partial-sum rows per lattice at least this
constexpr int kTileCounters = 8;  // the tiled pass's tile counters, one per XCD, after the ticket

enum Mode { kStep = 0, kInit = 1 };

// Launch one pass over `lat` reading buffer `src` and writing buffer 1-src
// (kStep) or updating the derivative of buffer `src` in place (kInit).
hipError_t launch_pass(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st);

// Each kernel family is compiled once per model (the source built with
// CE_UNIT_MODEL = kQuartic and = kPoly); these are the per-model entry points
// the dispatchers above pick from by lat.model.
template <int MODEL>
hipError_t launch_direct_model(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st);
template <int MODEL>
hipError_t launch_batched_direct_model(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                       const Lattice &proto, int precision, hipStream_t st);
template <int MODEL>
int direct_batched_resident_model(const Lattice &proto, int precision);
template <int MODEL>
hipError_t launch_tiled_model(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st);
template <int MODEL>
hipError_t launch_batched_tiled_model(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                      const Lattice &proto, int precision, hipStream_t st);
template <int MODEL>
int tiled_batched_resident_model(const Lattice &proto, int precision);
template <int MODEL>
int tiled_resident_blocks_model(int precision, int nf, int vec, int lpr, int bs);
template <int MODEL>
hipError_t launch_stream2d_model(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st);
template <int MODEL>
hipError_t launch_batched_stream2d_model(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                         const Lattice &proto, int precision, hipStream_t st);
template <int MODEL>
int stream2d_batched_resident_model(const Lattice &proto, int precision);
#define CE_DECLARE_MODEL_ENTRIES(M)                                                                             \
    template <> hipError_t launch_direct_model<M>(const Lattice &, int, int, Mode, hipStream_t);                \
    template <> hipError_t launch_batched_direct_model<M>(const Lattice *, const int *, int, int, const Lattice &, \
                                                          int, hipStream_t);                                     \
    template <> int direct_batched_resident_model<M>(const Lattice &, int);                                     \
    template <> hipError_t launch_tiled_model<M>(const Lattice &, int, int, Mode, hipStream_t);                 \
    template <> hipError_t launch_batched_tiled_model<M>(const Lattice *, const int *, int, int, const Lattice &, \
                                                         int, hipStream_t);                                      \
    template <> int tiled_batched_resident_model<M>(const Lattice &, int);                                      \
    template <> int tiled_resident_blocks_model<M>(int, int, int, int, int);                                    \
    template <> hipError_t launch_stream2d_model<M>(const Lattice &, int, int, Mode, hipStream_t);              \
    template <> hipError_t launch_batched_stream2d_model<M>(const Lattice *, const int *, int, int,             \
                                                            const Lattice &, int, hipStream_t);                  \
    template <> int stream2d_batched_resident_model<M>(const Lattice &, int);
CE_DECLARE_MODEL_ENTRIES(kQuartic)
CE_DECLARE_MODEL_ENTRIES(kPoly)
#undef CE_DECLARE_MODEL_ENTRIES

// Blocks a direct pass over this lattice uses (fixes the reduction order).
int pass_blocks(int dims, int N);
// Tiled 3-D pass: whether (N, lpr, zc) fits, its tile count, and the largest
// grid that keeps every block resident.
bool tiled_shape_built(int vec, int lpr, int bs);
bool tiled_fits(int dims, int N, int vec, int lpr, int bs, int zc);
long long tiled_tiles(int N, int vec, int lpr, int bs, int zc);
int tiled_resident_blocks(int model, int precision, int nf, int vec, int lpr, int bs);
hipError_t launch_tiled(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st);

// One step pass over many lattices of one class (same precision, dims,
// field count and kernel shape).  lats: device array of descriptors;
// blk_lat: lattice index of every per-lattice block (total_blocks entries).
// `grid` hardware blocks (1..total_blocks) walk the per-lattice blocks
// b, b + grid, ...; each per-lattice block computes exactly what block
// (b - first_block) of a lone launch of its lattice computes.  Each lattice
// reads its buffer parity from its scalar state and is skipped once its
// remaining-step count is 0.
hipError_t launch_batched(const Lattice *lats, const int *blk_lat, int total_blocks, int grid, const Lattice &proto,
                          int precision, hipStream_t st);
// Blocks of the class's batched kernel that fit on one compute unit.
int batched_resident_blocks(const Lattice &proto, int precision);
hipError_t launch_batched_tiled(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                const Lattice &proto, int precision, hipStream_t st);
int tiled_batched_resident(const Lattice &proto, int precision);

// 2-D streaming pass: units of 256 x sites by `rows` rows, four per block.
bool stream2d_fits(int dims, int N, int rows);
long long stream2d_groups(int N, int rows);
int stream2d_resident_blocks();
hipError_t launch_stream2d(const Lattice &lat, int precision, int src, Mode mode, hipStream_t st);
hipError_t launch_batched_stream2d(const Lattice *lats, const int *blk_lat, int total_blocks, int grid,
                                   const Lattice &proto, int precision, hipStream_t st);
int stream2d_batched_resident(const Lattice &proto, int precision);

// dst = (storage)(src - ref) for one chunk, plus running max |src| (as float bits).
hipError_t launch_convert(const double *src, double ref, void *dst, int precision, long long n,
                          unsigned int *maxabs_bits, hipStream_t st);
// storage -> FP64 readback of field `field`: f = m + d and the derivative as a
// step rebuilds it.  sites == NULL: the n consecutive sites from `first`;
// otherwise the n listed sites.
hipError_t launch_readback(const Lattice &lat, int precision, int buf, int field, int started,
                           long long first, const long long *sites, long long n, double *out_f,
                           double *out_fdot, hipStream_t st);

}  // namespace ce
