// Host runtime behind the C ABI in ce.h: parameter validation, device memory
// layout (library-owned or carved from a caller arena), loading with FP64 ->
// storage conversion, the start-up half step, step launches (plain or as
// captured step-block graphs), diagnostics and readback.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "ce_sim.hpp"

using namespace ce;
using namespace ce::host;

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace ce {
namespace host {

ce_status fail(ce_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}


long long sites_of(const ce_params *p)
{
    long long n = 1;
    for (int d = 0; d < p->dims; d++) n *= p->N;
    return n;
}

Layout layout_of(const ce_params *p)
{
    Layout L;
    const long long ns = sites_of(p);
    const size_t elem = p->precision == CE_FP64 ? 8 : 4;
    // partial-sum rows: one per block, and one per tile for tilings of up
    // to 16 N tiles of a 3-D lattice (the tiled pass sums per tile then)
    L.nblocks = p->dims == 3 ? (int)std::max<long long>(kMaxBlocks, 16LL * p->N) : kMaxBlocks;
    L.field_bytes = align_up((size_t)ns * elem);
    size_t off = 0;
    L.off_fields = off;
    off += 4 * (size_t)p->nfields * L.field_bytes;
    L.off_scalars = off;
    off += align_up(sizeof(Scalars));
    L.off_partials = off;
    off += align_up((size_t)L.nblocks * kMaxSums * sizeof(double));
    L.off_ticket = off;
    static_assert((1 + kTileCounters) * sizeof(unsigned int) <= kAlign, "ticket and tile counters share one line");
    off += kAlign;
    L.off_ring = off;
    off += align_up((size_t)kLogCap * sizeof(ce_energy));
    L.off_maxabs = off;
    off += kAlign;
    L.staging_elems = std::min<long long>(ns, kStagingElems);
    L.off_staging = off;
    off += align_up((size_t)L.staging_elems * sizeof(double));
    L.total = off;
    return L;
}

ce_status validate(const ce_params *p)
{
    if (!p) return fail(CE_EINVAL, "params is NULL");
    if (p->dims < 1 || p->dims > 3) return fail(CE_EINVAL, "dims must be 1, 2 or 3 (got %d)", p->dims);
    if (p->N < 4 || p->N % 4 != 0) return fail(CE_EINVAL, "N must be a multiple of 4 and >= 4 (got %d)", p->N);
    if (p->nfields < 1 || p->nfields > CE_MAX_FIELDS)
        return fail(CE_EINVAL, "nfields must be 1..%d (got %d)", CE_MAX_FIELDS, p->nfields);
    if (p->precision != CE_FP32 && p->precision != CE_FP64)
        return fail(CE_EINVAL, "precision must be CE_FP32 or CE_FP64");
    if (p->model != CE_MODEL_QUARTIC && p->model != CE_MODEL_POLYNOMIAL)
        return fail(CE_EINVAL, "unknown model %d", p->model);
    if (p->model == CE_MODEL_QUARTIC && p->nterms != 0)
        return fail(CE_EINVAL, "the quartic model takes no polynomial terms (nterms = %d)", p->nterms);
    if (p->model == CE_MODEL_POLYNOMIAL) {
        if (p->nterms < 1 || p->nterms > CE_MAX_TERMS)
            return fail(CE_EINVAL, "the polynomial model needs 1..%d terms (got %d)", CE_MAX_TERMS, p->nterms);
        if (p->lambda != 0.0 || p->vacuum != 0.0)
            return fail(CE_EINVAL, "the polynomial model takes lambda and vacuum as terms; set them to 0");
        for (int i = 0; i < CE_MAX_FIELDS; i++)
            if (p->G[i] != 0.0 || p->mu2[i] != 0.0)
                return fail(CE_EINVAL, "the polynomial model takes couplings and masses as terms; set G and mu2 to 0");
        for (int t = 0; t < p->nterms; t++) {
            const ce_term &tm = p->terms[t];
            if (!isfinite(tm.coef)) return fail(CE_EINVAL, "term %d: coefficient must be finite", t);
            int deg = 0;
            for (int i = 0; i < CE_MAX_FIELDS; i++) {
                if (tm.exp[i] < 0 || tm.exp[i] > CE_MAX_EXP)
                    return fail(CE_EINVAL, "term %d: exponent %d of field %d outside 0..%d", t, tm.exp[i], i,
                                CE_MAX_EXP);
                if (i >= p->nfields && tm.exp[i] != 0)
                    return fail(CE_EINVAL, "term %d: field %d does not exist (nfields = %d)", t, i, p->nfields);
                deg += tm.exp[i];
            }
            if (deg > CE_MAX_DEGREE)
                return fail(CE_EINVAL, "term %d: degree %d above %d", t, deg, CE_MAX_DEGREE);
        }
    }
    if (p->expansion != 0 && p->expansion != 1) return fail(CE_EINVAL, "expansion must be 0 or 1");
    if (!(p->L > 0) || !isfinite(p->L)) return fail(CE_EINVAL, "L must be positive and finite");
    if (!(p->dt > 0) || !isfinite(p->dt)) return fail(CE_EINVAL, "dt must be positive and finite");
    if (!(p->lambda >= 0) || !isfinite(p->lambda)) return fail(CE_EINVAL, "lambda must be >= 0");
    for (int i = 0; i < CE_MAX_FIELDS; i++) {
        if (!isfinite(p->G[i]) || p->G[i] < 0) return fail(CE_EINVAL, "G[%d] must be >= 0", i);
        if (!isfinite(p->mu2[i])) return fail(CE_EINVAL, "mu2[%d] must be finite", i);
    }
    if (!isfinite(p->vacuum)) return fail(CE_EINVAL, "vacuum must be finite");
    if (p->expansion && !(p->kappa > 0 && isfinite(p->kappa)))
        return fail(CE_EINVAL, "kappa must be positive with expansion");
    // site indices are 64-bit; 2^40 sites is far beyond any lattice that fits
    // in HBM.  The bound is checked before each multiplication: N^dims itself
    // can exceed 64 bits.
    long long ns = 1;
    for (int d = 0; d < p->dims; d++) {
        if (ns > (1LL << 40) / p->N) return fail(CE_EINVAL, "lattice too large (N^dims > 2^40 sites)");
        ns *= p->N;
    }
    const double dx = p->L / p->N;
    const double w = p->dt * 2.0 * sqrt((double)p->dims) / dx;
    if (!(w < 2.0))
        return fail(CE_EINVAL, "leapfrog unstable: dt*2*sqrt(dims)/dx = %g >= 2", w);
    return CE_OK;
}

void drop_graphs(ce_sim *s)
{
    for (int b = 0; b < 2; b++) {
        if (s->graph[b]) (void)hipGraphExecDestroy(s->graph[b]);
        s->graph[b] = nullptr;
    }
    s->graph_k = 0;
}

ce_status build_graph(ce_sim *s, int parity)
{
    if (!s->cap_stream) CE_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    CE_HIP(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int k = 0; k < s->step_block && err == hipSuccess; k++)
        err = launch_pass(s->lat, s->p.precision, (parity + k) & 1, kStep, s->cap_stream);
    hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(CE_EDEVICE, "step-block capture failed: %s",
                    hipGetErrorString(err != hipSuccess ? err : e2));
    }
    hipGraphExec_t ex = nullptr;
    err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return fail(CE_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(err));
    s->graph[parity] = ex;
    s->graph_k = s->step_block;
    return CE_OK;
}

ce_status device_cus(int *cus)
{
    int dev = 0;
    CE_HIP(hipGetDevice(&dev));
    CE_HIP(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    return CE_OK;
}

// Validate cfg for the lattice and fill the kernel-facing fields of lat.
ce_status apply_launch(ce_sim *s, const ce_launch &cfg)
{
    Lattice &lat = s->lat;
    if (cfg.grid < 0 || cfg.grid > kMaxBlocks) return fail(CE_EINVAL, "grid must be 0..%d", kMaxBlocks);
    if (cfg.kernel == CE_KERNEL_DIRECT) {
        int g = cfg.grid ? cfg.grid : pass_blocks(s->p.dims, s->p.N);
        lat.kind = kDirect;
        lat.vec = lat.lpr = lat.bs = lat.zc = 0;
        lat.nblocks = g;
    } else if (cfg.kernel == CE_KERNEL_TILED3D) {
        if (!tiled_shape_built(cfg.sites_per_thread, cfg.lanes_per_row, cfg.block))
            return fail(CE_EINVAL, "tiled shape (sites_per_thread=%d, lanes_per_row=%d, block=%d) is not built",
                        cfg.sites_per_thread, cfg.lanes_per_row, cfg.block);
        if (!tiled_fits(s->p.dims, s->p.N, cfg.sites_per_thread, cfg.lanes_per_row, cfg.block, cfg.planes))
            return fail(CE_EINVAL, "tiled launch (%d x %d tile, planes=%d) does not fit dims=%d N=%d",
                        cfg.sites_per_thread * cfg.lanes_per_row, cfg.block / cfg.lanes_per_row, cfg.planes,
                        s->p.dims, s->p.N);
        const long long tiles =
            tiled_tiles(s->p.N, cfg.sites_per_thread, cfg.lanes_per_row, cfg.block, cfg.planes);
        int g = cfg.grid;
        if (g == 0) {
            int cus = 0;
            ce_status st = device_cus(&cus);
            if (st != CE_OK) return st;
            const int per = tiled_resident_blocks(s->p.model, s->p.precision, s->p.nfields, cfg.sites_per_thread,
                                                  cfg.lanes_per_row, cfg.block);
            if (per < 1) return fail(CE_EDEVICE, "tiled kernel cannot be resident");
            // as many blocks as stay resident, then evened out so every block
            // walks the same number of tiles; a multiple of 8 keeps each
            // XCD on one contiguous slab of tiles
            long long resident = (long long)per * cus;
            if (resident > kMaxBlocks) resident = kMaxBlocks;
            const long long rounds = (tiles + resident - 1) / resident;
            long long want = (tiles + rounds - 1) / rounds;
            if (want >= 8) want = (want + 7) / 8 * 8;
            if (want > kMaxBlocks) want = kMaxBlocks / 8 * 8;
            g = (int)want;
        }
        lat.kind = kTiled3d;
        lat.vec = cfg.sites_per_thread;
        lat.lpr = cfg.lanes_per_row;
        lat.bs = cfg.block;
        lat.zc = cfg.planes;
        lat.nblocks = g;
    } else if (cfg.kernel == CE_KERNEL_STREAM2D) {
        if (!stream2d_fits(s->p.dims, s->p.N, cfg.planes))
            return fail(CE_EINVAL, "2-D streaming launch (rows=%d) does not fit dims=%d N=%d", cfg.planes,
                        s->p.dims, s->p.N);
        const long long groups = stream2d_groups(s->p.N, cfg.planes);
        int g = cfg.grid;
        if (g == 0) {
            int cus = 0;
            ce_status st = device_cus(&cus);
            if (st != CE_OK) return st;
            long long resident = (long long)stream2d_resident_blocks() * cus;
            if (resident < 1) return fail(CE_EDEVICE, "2-D streaming kernel cannot be resident");
            if (resident > kMaxBlocks) resident = kMaxBlocks;
            const long long rounds = (groups + resident - 1) / resident;
            long long want = (groups + rounds - 1) / rounds;
            if (want >= 8) want = (want + 7) / 8 * 8;
            if (want > kMaxBlocks) want = kMaxBlocks / 8 * 8;
            g = (int)want;
        }
        lat.kind = kStream2d;
        lat.vec = 4;
        lat.lpr = 64;
        lat.bs = kBlock;
        lat.zc = cfg.planes;
        lat.nblocks = g;
        // the shape is fixed: report it whatever the caller passed
        s->launch = ce_launch{CE_KERNEL_STREAM2D, 4, 64, kBlock, cfg.planes, cfg.grid};
        drop_graphs(s);
        return CE_OK;
    } else {
        return fail(CE_EINVAL, "unknown kernel %d", cfg.kernel);
    }
    s->launch = cfg;
    drop_graphs(s);
    return CE_OK;
}

// The library's default launch.  3-D lattices use the tiled kernel with the
// widest tile that divides N (256 x 4 sites, 4 per thread, then 64 x 16,
// then 32 x 32): wide tiles keep the x halo to 2 of every 8 cache lines.
// Large lattices keep every resident block busy with the longest chunks that
// give every block the same whole number (>= 2) of tiles (three of 342, 342
// and 340 planes at 1024^3); medium ones (N >= 64) get one tile per compute
// unit with the tallest chunks
// that allow it; smaller ones take the tallest chunks that leave three tiles
// per compute unit, or the direct kernel when they cannot give one tile per
// compute unit.
ce_launch default_launch(const ce_params *p, int cus)
{
    ce_launch c{CE_KERNEL_DIRECT, 0, 0, 0, 0, 0};
    if (p->dims == 2) {
        // rows per unit: the tallest (up to 64) that still gives every
        // compute unit a group of four units
        for (int rows = 64; rows >= 8; rows /= 2)
            if (stream2d_fits(2, p->N, rows) && (stream2d_groups(p->N, rows) >= cus || rows == 8)) {
                c.kernel = CE_KERNEL_STREAM2D;
                c.sites_per_thread = 4;
                c.lanes_per_row = 64;
                c.block = kBlock;
                c.planes = rows;
                return c;
            }
        return c;
    }
    if (p->dims != 3) return c;
    const int shapes[3][3] = {{4, 64, 256}, {4, 16, 256}, {4, 8, 256}};
    for (int a = 0; a < 3; a++) {
        const int v = shapes[a][0], l = shapes[a][1], bs = shapes[a][2];
        if (!tiled_fits(3, p->N, v, l, bs, p->N)) continue;
        // Large lattices: every block that fits stays resident (full
        // occupancy hides the most memory latency).  Each z chunk re-reads
        // two halo planes from memory, so chunks are as long as possible:
        // the fewest chunks per column that give every block the same whole
        // number (>= 2) of tiles.  Else short z chunks, so the last, partial
        // round of tiles is a small part of the pass.
        long long resident = (long long)tiled_resident_blocks(p->model, p->precision, p->nfields, v, l, bs) * cus;
        if (resident > kMaxBlocks) resident = kMaxBlocks;
        if (resident >= 8) resident = resident / 8 * 8;
        const long long cols = tiled_tiles(p->N, v, l, bs, p->N);
        for (int nz = 1; nz <= p->N / 64 && resident > 0; nz++) {
            const long long tiles = cols * nz;
            const int planes = (p->N + nz - 1) / nz;  // nz chunks of near-equal length
            if ((p->N + planes - 1) / planes == nz && tiles >= 2 * resident && tiles % resident == 0) {
                c.kernel = CE_KERNEL_TILED3D;
                c.sites_per_thread = v;
                c.lanes_per_row = l;
                c.block = bs;
                c.planes = planes;
                c.grid = (int)resident;
                return c;
            }
        }
        for (int z = 32; z >= 16 && resident > 0; z /= 2)
            if (p->N % z == 0 && tiled_tiles(p->N, v, l, bs, z) >= (z == 32 ? 8 : 4) * resident) {
                c.kernel = CE_KERNEL_TILED3D;
                c.sites_per_thread = v;
                c.lanes_per_row = l;
                c.block = bs;
                c.planes = z;
                c.grid = (int)resident;
                return c;
            }
    }
    if (p->N >= 64) {
        // Medium lattices (64^3 .. 256^3 and the like): one tile per compute
        // unit where the lattice has that many, with the tallest chunks that
        // still give them, else the shortest (2 planes).  Widest tiles first,
        // 512-thread blocks where the tile is 256 sites wide.  On 64^3,
        // 128^3 and 256^3 x 2 fields this is the fastest configuration found
        // by timing every shape and chunk length (128^3: 3.2x the direct pass).
        const int pref[5][3] = {{4, 64, 512}, {4, 64, 256}, {4, 16, 256}, {2, 32, 512}, {4, 8, 256}};
        for (int a = 0; a < 5; a++) {
            const int v = pref[a][0], l = pref[a][1], bs = pref[a][2];
            if (!tiled_fits(3, p->N, v, l, bs, 2) || p->N % 2) continue;
            int planes = 2;
            for (int z = 2; z <= p->N; z *= 2)
                if (p->N % z == 0 && tiled_tiles(p->N, v, l, bs, z) >= cus) planes = z;
            c.kernel = CE_KERNEL_TILED3D;
            c.sites_per_thread = v;
            c.lanes_per_row = l;
            c.block = bs;
            c.planes = planes;
            c.grid = 0;
            return c;
        }
    }
    for (int a = 0; a < 3; a++) {
        const int v = shapes[a][0], l = shapes[a][1], bs = shapes[a][2];
        if (!tiled_fits(3, p->N, v, l, bs, p->N)) continue;
        // smaller lattices: the tallest chunks that still give three tiles
        // per compute unit; the grid is evened over the rounds
        int planes = 0;
        for (int z = p->N; z >= 16; z /= 2) {
            if (p->N % z) continue;
            planes = z;
            if (tiled_tiles(p->N, v, l, bs, z) >= 3LL * cus) break;
        }
        if (planes == 0 || tiled_tiles(p->N, v, l, bs, planes) < cus) continue;
        c.kernel = CE_KERNEL_TILED3D;
        c.sites_per_thread = v;
        c.lanes_per_row = l;
        c.block = bs;
        c.planes = planes;
        return c;
    }
    return ce_launch{CE_KERNEL_DIRECT, 0, 0, 0, 0, 0};
}

}  // namespace host
}  // namespace ce

extern "C" {

const char *ce_last_error(void) { return g_err; }

ce_status ce_get_launch(const ce_sim *s, ce_launch *out)
{
    if (!s || !out) return fail(CE_EINVAL, "NULL argument");
    *out = s->launch;
    out->grid = s->lat.nblocks;
    return CE_OK;
}

ce_status ce_set_launch(ce_sim *s, const ce_launch *cfg)
{
    if (!s || !cfg) return fail(CE_EINVAL, "NULL argument");
    const ce_launch old = s->launch;
    const Lattice saved = s->lat;
    ce_status st = apply_launch(s, *cfg);
    if (st != CE_OK) {
        s->launch = old;
        s->lat = saved;
    }
    return st;
}

ce_status ce_required_bytes(const ce_params *p, size_t *out)
{
    ce_status st = validate(p);
    if (st != CE_OK) return st;
    if (!out) return fail(CE_EINVAL, "out is NULL");
    *out = layout_of(p).total;
    return CE_OK;
}

ce_status ce_create(const ce_params *p, ce_sim **out)
{
    ce_status st = validate(p);
    if (st != CE_OK) return st;
    if (!out) return fail(CE_EINVAL, "out is NULL");
    *out = nullptr;
    ce_sim *s = new (std::nothrow) ce_sim();
    if (!s) return fail(CE_ENOMEM, "host allocation failed");
    s->p = *p;
    s->lay = layout_of(p);
    const Layout &L = s->lay;
    if (p->arena) {
        if ((uintptr_t)p->arena % kAlign) {
            delete s;
            return fail(CE_EINVAL, "arena must be %zu-byte aligned", kAlign);
        }
        if (p->arena_bytes < L.total) {
            delete s;
            return fail(CE_ENOMEM, "arena holds %zu bytes, %zu needed", p->arena_bytes, L.total);
        }
        s->base = static_cast<char *>(p->arena);
    } else {
        hipError_t e = hipMalloc(&s->base, L.total);
        if (e != hipSuccess) {
            delete s;
            (void)hipGetLastError();
            return fail(CE_ENOMEM, "hipMalloc(%zu) failed: %s", L.total, hipGetErrorString(e));
        }
        s->own_mem = true;
    }
    if (p->stream) {
        s->stream = static_cast<hipStream_t>(p->stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ce_destroy(s);
            return fail(CE_EDEVICE, "stream creation failed: %s", hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    Lattice &lat = s->lat;
    memset(&lat, 0, sizeof(lat));
    for (int b = 0; b < 2; b++)
        for (int i = 0; i < p->nfields; i++) {
            lat.d[b][i] = s->base + L.off_fields + ((size_t)(b * p->nfields + i)) * L.field_bytes;
            lat.p[b][i] = s->base + L.off_fields + ((size_t)((2 + b) * p->nfields + i)) * L.field_bytes;
        }
    lat.dims = p->dims;
    lat.N = p->N;
    lat.nf = p->nfields;
    lat.expansion = p->expansion;
    lat.nsites = sites_of(p);
    lat.dt = p->dt;
    const double dx = p->L / p->N;
    lat.inv_dx2 = 1.0 / (dx * dx);
    lat.lambda = p->lambda;
    lat.kappa = p->kappa;
    lat.vacuum = p->vacuum;
    for (int i = 0; i < kMaxFields; i++) {
        lat.G[i] = i < p->nfields ? p->G[i] : 0.0;
        lat.mu2[i] = i < p->nfields ? p->mu2[i] : 0.0;
    }
    lat.G[0] = 0.0;
    // polynomial model: the terms of degree >= 1 go to the kernels; constant
    // terms are a vacuum energy (a^4 V0 in the program variables)
    lat.model = p->model;
    lat.nterms = 0;
    if (p->model == CE_MODEL_POLYNOMIAL) {
        for (int t = 0; t < p->nterms; t++) {
            const ce_term &tm = p->terms[t];
            int deg = 0;
            for (int i = 0; i < CE_MAX_FIELDS; i++) deg += tm.exp[i];
            if (deg == 0) {
                lat.vacuum += tm.coef;
                continue;
            }
            const int k = lat.nterms++;
            lat.tcoef[k] = tm.coef;
            lat.tdeg[k] = deg;
            for (int i = 0; i < kMaxFields; i++) lat.texp[k][i] = tm.exp[i];
        }
    }
    lat.dt_f = (float)lat.dt;
    lat.inv_dx2_f = (float)lat.inv_dx2;
    lat.lambda_f = (float)lat.lambda;
    lat.qlam_f = (float)(0.25 * lat.lambda);
    for (int i = 0; i < kMaxFields; i++) {
        lat.G_f[i] = (float)lat.G[i];
        lat.hG_f[i] = (float)(0.5 * lat.G[i]);
    }
    lat.sc = reinterpret_cast<Scalars *>(s->base + L.off_scalars);
    lat.partials = reinterpret_cast<double *>(s->base + L.off_partials);
    lat.ticket = reinterpret_cast<unsigned int *>(s->base + L.off_ticket);
    lat.slots = L.nblocks;
    lat.ring = reinterpret_cast<ce_energy *>(s->base + L.off_ring);
    {
        int cus = 0;
        ce_status st2 = device_cus(&cus);
        if (st2 == CE_OK) st2 = apply_launch(s, default_launch(p, cus));
        if (st2 != CE_OK) {
            const ce_status keep = st2;
            char msg[sizeof(g_err)];
            memcpy(msg, g_err, sizeof(msg));
            ce_destroy(s);
            memcpy(g_err, msg, sizeof(msg));
            return keep;
        }
    }
    s->maxabs = reinterpret_cast<unsigned int *>(s->base + L.off_maxabs);
    s->staging = reinterpret_cast<double *>(s->base + L.off_staging);

    Scalars init{};
    init.a = 1.0;
    init.a_next = 1.0;
    init.first_bad = -1;
    hipError_t e = hipMemcpyAsync(lat.sc, &init, sizeof(init), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(lat.ticket, 0, kAlign, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->maxabs, 0, kAlign, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        ce_destroy(s);
        return fail(CE_EDEVICE, "initialisation failed: %s", hipGetErrorString(e));
    }
    *out = s;
    return CE_OK;
}

ce_status ce_load_fields(ce_sim *s, int32_t first, int32_t count, const double *phi,
                         const double *phidot)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    if (s->started) return fail(CE_ESTATE, "fields already loaded and evolved");
    // compared without forming first + count, which could overflow
    if (first < 0 || count < 1 || first >= s->p.nfields || count > s->p.nfields - first)
        return fail(CE_EINVAL, "field range of %d fields from %d outside 0..%d", count, first, s->p.nfields);
    if (!phi || !phidot) return fail(CE_EINVAL, "phi and phidot must be non-NULL");
    const long long ns = s->lat.nsites;
    const long long chunk = s->lay.staging_elems;
    const size_t elem = s->p.precision == CE_FP64 ? 8 : 4;
    for (int i = 0; i < count; i++) {
        const int fi = first + i;
        // homogeneous reference: the mean of an evenly strided sample of at
        // most 2^16 sites.  Any value near the volume mean works (the stored
        // deviation is exact relative to it, and the reference then moves
        // with the mean derivative); the sample keeps the deviations at the
        // size of the fluctuations without a host pass over the whole field.
        const double *fsrc = phi + (long long)i * ns;
        const long long stride = std::max<long long>(1, ns >> 16);
        double part[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        long long cnt = 0;
        for (long long k = 0; k < ns; k += stride, cnt++) part[cnt & 7] += fsrc[k];
        const double acc = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
        s->m_host[fi] = acc / (double)cnt;
        if (!isfinite(s->m_host[fi])) return fail(CE_EINVAL, "initial field %d is not finite", fi);
        CE_HIP(hipMemcpyAsync(&s->lat.sc->m[fi], &s->m_host[fi], sizeof(double), hipMemcpyHostToDevice,
                              s->stream));
        for (int which = 0; which < 2; which++) {
            const double *src = (which == 0 ? phi : phidot) + (long long)i * ns;
            void *dst = which == 0 ? s->lat.d[s->cur][fi] : s->lat.p[s->cur][fi];
            const double ref = which == 0 ? s->m_host[fi] : 0.0;
            for (long long off = 0; off < ns; off += chunk) {
                const long long n = std::min(chunk, ns - off);
                CE_HIP(hipMemcpyAsync(s->staging, src + off, (size_t)n * sizeof(double),
                                      hipMemcpyHostToDevice, s->stream));
                CE_HIP(launch_convert(s->staging, ref, static_cast<char *>(dst) + (size_t)off * elem,
                                      s->p.precision, n, which == 0 ? s->maxabs + fi : s->maxabs + 3,
                                      s->stream));
            }
        }
        s->loaded |= 1u << fi;
    }
    CE_HIP(hipStreamSynchronize(s->stream));
    if (s->loaded != (1u << s->p.nfields) - 1) return CE_OK;
    return start_run(s);
}

}  // extern "C"

namespace ce {
namespace host {

ce_status start_run(ce_sim *s)
{
    // all fields present: stability including the potential's curvature,
    // bounded with the largest |f| of every field
    unsigned int bits[4];
    CE_HIP(hipMemcpy(bits, s->maxabs, sizeof(bits), hipMemcpyDeviceToHost));
    // a rejected set of fields must be loaded again; the maxima start over
    auto reject = [s]() -> ce_status {
        s->loaded = 0;
        CE_HIP(hipMemsetAsync(s->maxabs, 0, kAlign, s->stream));
        CE_HIP(hipStreamSynchronize(s->stream));
        return CE_EINVAL;
    };
    double M[CE_MAX_FIELDS] = {0, 0, 0};
    for (int i = 0; i < s->p.nfields; i++) {
        float v;
        memcpy(&v, &bits[i], sizeof(v));
        M[i] = v;
    }
    float vd;
    memcpy(&vd, &bits[3], sizeof(vd));
    if (!isfinite(vd)) {
        ce_status st = reject();
        return st != CE_EINVAL ? st : fail(CE_EINVAL, "initial derivatives are not finite");
    }
    double m2max = 0.0;
    for (int i = 0; i < s->p.nfields; i++) {
        if (!isfinite(M[i])) {
            ce_status st = reject();
            return st != CE_EINVAL ? st : fail(CE_EINVAL, "initial field %d is not finite", i);
        }
    }
    const int nf = s->p.nfields;
    for (int i = 0; i < nf; i++) {
        double m2;
        if (s->p.model == CE_MODEL_POLYNOMIAL) {
            // Gershgorin bound on the Hessian of V at |f_j| <= M_j (a = 1):
            // row i sums |d^2 V / df_i df_j| over j, term by term
            m2 = 0.0;
            const Lattice &L = s->lat;
            for (int t = 0; t < L.nterms; t++) {
                const double c = fabs(L.tcoef[t]);
                for (int j = 0; j < nf; j++) {
                    const int ei = L.texp[t][i], ej = L.texp[t][j];
                    double h = c;
                    for (int k = 0; k < nf; k++) {
                        int e = L.texp[t][k];
                        if (k == i) {
                            h *= (double)e;
                            e -= 1;
                        }
                        if (k == j) {
                            h *= (double)(k == i ? ei - 1 : ej);
                            e -= 1;
                        }
                        if (e < 0) {
                            h = 0.0;
                            break;
                        }
                        for (int q = 0; q < e; q++) h *= M[k];
                    }
                    m2 += h;
                }
            }
        } else if (i == 0) {
            m2 = 3.0 * s->p.lambda * M[0] * M[0] + s->p.mu2[0];
            for (int j = 1; j < nf; j++) m2 += s->p.G[j] * M[j] * M[j];
        } else {
            m2 = s->p.G[i] * M[0] * M[0] + s->p.mu2[i];
        }
        m2max = std::max(m2max, m2);
    }
    const double dx = s->p.L / s->p.N;
    const double w = s->p.dt * sqrt(4.0 * s->p.dims / (dx * dx) + m2max);
    if (!(w < 2.0)) {
        ce_status st = reject();
        return st != CE_EINVAL ? st
                               : fail(CE_EINVAL, "leapfrog unstable for these fields: dt*sqrt(4d/dx^2 + m^2_max) = %g >= 2", w);
    }
    CE_HIP(launch_pass(s->lat, s->p.precision, s->cur, kInit, s->stream));
    s->started = true;
    s->step = 0;
    return CE_OK;
}

}  // namespace host
}  // namespace ce

extern "C" {

ce_status ce_set_step_block(ce_sim *s, int32_t k)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    if (k < 0 || k > 4096) return fail(CE_EINVAL, "step block must be 0..4096");
    if (k != s->step_block) drop_graphs(s);
    s->step_block = k;
    return CE_OK;
}

ce_status ce_step(ce_sim *s, int64_t nsteps)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    if (nsteps < 0) return fail(CE_EINVAL, "nsteps must be >= 0");
    if (!s->started) return fail(CE_ESTATE, "load every field before stepping");
    long long left = nsteps;
    if (s->step_block > 0) {
        while (left >= s->step_block) {
            if (!s->graph[s->cur]) {
                ce_status st = build_graph(s, s->cur);
                if (st != CE_OK) return st;
            }
            CE_HIP(hipGraphLaunch(s->graph[s->cur], s->stream));
            s->cur = (s->cur + s->step_block) & 1;
            s->step += s->step_block;
            left -= s->step_block;
        }
    }
    for (; left > 0; left--) {
        CE_HIP(launch_pass(s->lat, s->p.precision, s->cur, kStep, s->stream));
        s->cur ^= 1;
        s->step += 1;
    }
    return CE_OK;
}

ce_status ce_time_steps(ce_sim *s, int64_t nsteps, float *ms)
{
    if (!s || !ms) return fail(CE_EINVAL, "NULL argument");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CE_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CE_EDEVICE, "hipEventCreate failed: %s", hipGetErrorString(err));
    }
    ce_status st = CE_OK;
    err = hipEventRecord(e0, s->stream);
    if (err == hipSuccess) {
        st = ce_step(s, nsteps);
        if (st == CE_OK) err = hipEventRecord(e1, s->stream);
        if (st == CE_OK && err == hipSuccess) err = hipEventSynchronize(e1);
        if (st == CE_OK && err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != CE_OK) return st;
    if (err != hipSuccess) return fail(CE_EDEVICE, "event timing failed: %s", hipGetErrorString(err));
    return CE_OK;
}

ce_status ce_sync(ce_sim *s)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    CE_HIP(hipStreamSynchronize(s->stream));
    return CE_OK;
}

ce_status ce_get_step(const ce_sim *s, int64_t *step)
{
    if (!s || !step) return fail(CE_EINVAL, "NULL argument");
    *step = s->step;
    return CE_OK;
}

ce_status ce_energies(ce_sim *s, ce_energy *out)
{
    if (!s || !out) return fail(CE_EINVAL, "NULL argument");
    if (!s->started) return fail(CE_ESTATE, "no diagnostics before every field is loaded");
    CE_HIP(hipStreamSynchronize(s->stream));
    CE_HIP(hipMemcpy(out, s->lat.ring + (s->step % kLogCap), sizeof(ce_energy), hipMemcpyDeviceToHost));
    Scalars sc;
    CE_HIP(hipMemcpy(&sc, s->lat.sc, sizeof(sc), hipMemcpyDeviceToHost));
    if (out->step != s->step)
        return fail(CE_EDEVICE, "diagnostics record for step %lld holds step %lld", (long long)s->step,
                    (long long)out->step);
    if (sc.first_bad >= 0)
        return fail(CE_ENONFINITE, "non-finite volume sum first at step %lld", sc.first_bad);
    return CE_OK;
}

ce_status ce_energy_log(ce_sim *s, int32_t count, ce_energy *out)
{
    if (!s || !out) return fail(CE_EINVAL, "NULL argument");
    if (!s->started) return fail(CE_ESTATE, "no diagnostics before every field is loaded");
    if (count < 1 || count > kLogCap || count > s->step + 1)
        return fail(CE_EINVAL, "count must be 1..min(%d, step+1)", kLogCap);
    CE_HIP(hipStreamSynchronize(s->stream));
    const long long first = s->step - count + 1;
    for (int k = 0; k < count;) {
        const long long idx = (first + k) % kLogCap;
        const int run = (int)std::min<long long>(count - k, kLogCap - idx);
        CE_HIP(hipMemcpy(out + k, s->lat.ring + idx, (size_t)run * sizeof(ce_energy),
                         hipMemcpyDeviceToHost));
        k += run;
    }
    return CE_OK;
}

ce_status ce_read_fields(ce_sim *s, double *f, double *fdot)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    if (s->loaded != (1u << s->p.nfields) - 1) return fail(CE_ESTATE, "fields not loaded");
    const long long ns = s->lat.nsites;
    const long long chunk = s->lay.staging_elems / 2;  // f and fdot share the staging block
    for (int i = 0; i < s->p.nfields; i++) {
        for (long long off = 0; off < ns; off += chunk) {
            const long long n = std::min(chunk, ns - off);
            double *df = s->staging;
            double *dp = s->staging + chunk;
            CE_HIP(launch_readback(s->lat, s->p.precision, s->cur, i, s->started ? 1 : 0, off, nullptr, n,
                                   f ? df : nullptr, fdot ? dp : nullptr, s->stream));
            if (f)
                CE_HIP(hipMemcpyAsync(f + (long long)i * ns + off, df, (size_t)n * sizeof(double),
                                      hipMemcpyDeviceToHost, s->stream));
            if (fdot)
                CE_HIP(hipMemcpyAsync(fdot + (long long)i * ns + off, dp, (size_t)n * sizeof(double),
                                      hipMemcpyDeviceToHost, s->stream));
            CE_HIP(hipStreamSynchronize(s->stream));
        }
    }
    return CE_OK;
}

ce_status ce_read_sites(ce_sim *s, int32_t field, int64_t count, const int64_t *sites, double *f,
                        double *fdot)
{
    if (!s) return fail(CE_EINVAL, "sim is NULL");
    if (s->loaded != (1u << s->p.nfields) - 1) return fail(CE_ESTATE, "fields not loaded");
    if (field < 0 || field >= s->p.nfields) return fail(CE_EINVAL, "field %d out of range", field);
    const long long per = s->lay.staging_elems / 3;
    if (count < 0 || count > (1LL << 20) || count > per)
        return fail(CE_EINVAL, "count must be 0..%lld", std::min(per, 1LL << 20));
    if (count == 0) return CE_OK;
    if (!sites) return fail(CE_EINVAL, "sites is NULL");
    const long long ns = s->lat.nsites;
    for (long long i = 0; i < count; i++)
        if (sites[i] < 0 || sites[i] >= ns) return fail(CE_EINVAL, "site %lld out of range", (long long)sites[i]);
    long long *dsites = reinterpret_cast<long long *>(s->staging);
    double *df = s->staging + per;
    double *dp = s->staging + 2 * per;
    CE_HIP(hipMemcpyAsync(dsites, sites, (size_t)count * sizeof(long long), hipMemcpyHostToDevice, s->stream));
    CE_HIP(launch_readback(s->lat, s->p.precision, s->cur, field, s->started ? 1 : 0, 0, dsites, count,
                           f ? df : nullptr, fdot ? dp : nullptr, s->stream));
    if (f) CE_HIP(hipMemcpyAsync(f, df, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (fdot) CE_HIP(hipMemcpyAsync(fdot, dp, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    CE_HIP(hipStreamSynchronize(s->stream));
    return CE_OK;
}

void ce_destroy(ce_sim *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    if (s->own_mem && s->base) (void)hipFree(s->base);
    delete s;
}

}  // extern "C"
