// Pool of independent lattices advanced together: admission within a byte
// budget, one batched launch per class of members per step, step blocks
// captured as graphs per pool composition, polling and retirement.
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "ce_sim.hpp"

namespace ce {
// lats[l].sc->remaining = vals[l] for l < n (device arrays); in ce_kernels.hip
hipError_t launch_set_remaining(const Lattice *lats, const long long *vals, int n, hipStream_t st);
}  // namespace ce

using namespace ce;
using namespace ce::host;

namespace {

struct Member {
    ce_sim *sim = nullptr;
    void *mem = nullptr;       // the member's device memory (pool-owned)
    size_t bytes = 0;
    long long remaining = 0;   // steps not yet enqueued (host mirror of the device count)
    long long init_remaining = 0;
    int init_cur = 0;
    long long finish_seq = -1; // block that holds the member's last step
    long long quota = -1;      // steps per block at most (-1: no limit)
};

// Members that can share one launch: same kernel instance.
// model, precision, dims, nf, kind, vec, lpr, bs
using ClassKey = std::tuple<int, int, int, int, int, int, int, int>;

ClassKey class_of(const ce_sim *s)
{
    return ClassKey(s->p.model, s->p.precision, s->p.dims, s->p.nfields, s->lat.kind, s->lat.vec, s->lat.lpr,
                    s->lat.bs);
}

struct ClassTable {
    int precision = CE_FP32;
    Lattice proto;               // any member: selects the kernel instance
    std::vector<Lattice> lats;   // descriptors, first_block filled
    std::vector<int> blk_lat;    // lattice index of every block
    Lattice *d_lats = nullptr;   // device copies (inside the pool's table buffer)
    int *d_blk = nullptr;
    int grid = 0;                // hardware blocks of the batched launch
    std::vector<Member *> mems;  // the member of each descriptor
    long long *d_rem = nullptr;  // step budgets for the next block (quotas)
};

}  // namespace

struct ce_pool {
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    long long next_id = 1;
    std::map<long long, Member> members;
    // launch tables for the current composition, double-buffered so that a
    // rebuild never waits for the block in flight (it rewrites the buffer
    // the block before that one used); graphs per buffer and block length
    bool dirty = true;
    std::vector<ClassTable> classes;
    struct TableBuf {
        char *d = nullptr;
        size_t bytes = 0;
        long long last_seq = -1;                // last block that read these tables
        std::map<int, hipGraphExec_t> graphs;   // by steps per block
    };
    TableBuf tbuf[2];
    int cur_buf = 0;
    int blocks_since_rebuild = 0;
    long long steps_run = 0;
    // per-block step budgets, used while any member has a quota: uploaded
    // from page-locked memory (one buffer per block parity) and written into
    // the members' remaining counts before the block
    long long *h_rem[2] = {};
    size_t h_rem_cap[2] = {};
    bool budgets_set = false;   // the last block ran with budgets below the remaining counts
    // one event per block, recorded on the pool stream after it
    static constexpr int kEvRing = 16;
    hipEvent_t block_ev[kEvRing] = {};
    long long seq = 0;                          // blocks enqueued
    // device memory of retired members, kept for reuse by size: freeing
    // would synchronise the device and stall the block in flight
    std::multimap<size_t, void *> free_mem;
    size_t cached = 0;
    // classes run their step chains on separate lanes (streams) inside a
    // block, so small classes overlap instead of queueing behind each other
    static constexpr int kLanes = 4;
    hipStream_t lanes[kLanes] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kLanes] = {};
    std::vector<int> lane_of;  // lane of each class
    // admissions load on their own stream, beside the running block; the
    // launch tables upload on another
    std::vector<hipStream_t> load_streams;   // idle load streams (one per admission in progress)
    std::vector<hipStream_t> all_load_streams;
    hipStream_t table_stream = nullptr;
    // members' own stream after admission: diagnostics and readback, which
    // the host issues after waiting for the block concerned
    hipStream_t read_stream = nullptr;
    // admissions may run on other host threads than the other calls (and
    // several at once, each on a load stream of its own): `mu` guards the
    // member map, the byte counts, the memory cache and the stream lists;
    // `admitting` counts admissions in progress, `idle` is signalled when it
    // drops to zero, and `closing` (set by ce_pool_destroy) turns later
    // admissions away
    std::mutex mu;
    std::condition_variable idle;
    int admitting = 0;
    bool closing = false;
};

namespace {

// The configuration members use: the tiled kernel (widest tile that fits,
// at most 64 planes per tile, more when needed to stay within the partial
// slots) with one tile per block, else the direct kernel with its usual grid.
ce_launch member_launch(const ce_params *p)
{
    ce_launch c{CE_KERNEL_DIRECT, 0, 0, 0, 0, pass_blocks(p->dims, p->N)};
    if (p->dims == 2 && stream2d_fits(2, p->N, 8)) {
        // one group of four units per block; the tallest units (up to 64
        // rows) that still give the member two blocks
        int rows = 64;
        while (rows > 8 && stream2d_groups(p->N, rows) < 2) rows /= 2;
        c.kernel = CE_KERNEL_STREAM2D;
        c.sites_per_thread = 4;
        c.lanes_per_row = 64;
        c.block = kBlock;
        c.planes = rows;
        c.grid = (int)std::min<long long>(stream2d_groups(p->N, rows), kMaxBlocks);
        return c;
    }
    if (p->dims != 3) return c;
    const int shapes[3][3] = {{4, 64, 256}, {4, 16, 256}, {4, 8, 256}};
    for (int a = 0; a < 3; a++) {
        const int v = shapes[a][0], l = shapes[a][1], bs = shapes[a][2];
        for (int z = std::min(p->N, 64); z <= p->N; z *= 2) {
            if (p->N % z || !tiled_fits(3, p->N, v, l, bs, z)) continue;
            const long long tiles = tiled_tiles(p->N, v, l, bs, z);
            if (tiles > kMaxBlocks) continue;
            c.kernel = CE_KERNEL_TILED3D;
            c.sites_per_thread = v;
            c.lanes_per_row = l;
            c.block = bs;
            c.planes = z;
            c.grid = (int)tiles;
            return c;
        }
    }
    return c;
}

void drop_graphs(ce_pool::TableBuf &T)
{
    for (auto &kv : T.graphs) (void)hipGraphExecDestroy(kv.second);
    T.graphs.clear();
}

// Wait until block s (and everything before it) has run.
ce_status wait_block(ce_pool *pl, long long s)
{
    if (s < 0 || s >= pl->seq) return CE_OK;
    if (pl->seq - s <= ce_pool::kEvRing)
        CE_HIP(hipEventSynchronize(pl->block_ev[s % ce_pool::kEvRing]));
    else
        CE_HIP(hipStreamSynchronize(pl->stream));  // its event was recorded again since
    return CE_OK;
}

void *take_cached(ce_pool *pl, size_t bytes)
{
    auto it = pl->free_mem.find(bytes);
    if (it == pl->free_mem.end()) return nullptr;
    void *m = it->second;
    pl->free_mem.erase(it);
    pl->cached -= bytes;
    return m;
}

// Free cached memory until `want` more bytes fit next to the members' and
// the cache's within the budget (hipFree synchronises the device).
ce_status trim_cache(ce_pool *pl, size_t want)
{
    while (!pl->free_mem.empty() && pl->used + pl->cached + want > pl->budget) {
        auto it = std::prev(pl->free_mem.end());
        CE_HIP(hipFree(it->second));
        pl->cached -= it->first;
        pl->free_mem.erase(it);
    }
    return CE_OK;
}

// Rebuild the per-class launch tables for the members with steps left.
ce_status ensure_lanes(ce_pool *pl)
{
    if (pl->fork_ev) return CE_OK;
    for (int l = 0; l < ce_pool::kLanes; l++) {
        CE_HIP(hipStreamCreateWithFlags(&pl->lanes[l], hipStreamNonBlocking));
        CE_HIP(hipEventCreateWithFlags(&pl->join_ev[l], hipEventDisableTiming));
    }
    CE_HIP(hipEventCreateWithFlags(&pl->fork_ev, hipEventDisableTiming));
    return CE_OK;
}

// Called with pl->mu held, after the block that last read the other table
// buffer has finished (the caller waits for it before taking the lock).
ce_status rebuild(ce_pool *pl)
{
    const int b = 1 - pl->cur_buf;
    ce_pool::TableBuf &T = pl->tbuf[b];
    drop_graphs(T);
    if (!pl->table_stream) CE_HIP(hipStreamCreateWithFlags(&pl->table_stream, hipStreamNonBlocking));
    std::map<ClassKey, ClassTable> by_class;
    for (auto &kv : pl->members) {
        Member &m = kv.second;
        if (m.remaining <= 0) continue;
        ClassTable &t = by_class[class_of(m.sim)];
        Lattice L = m.sim->lat;
        L.first_block = (int)t.blk_lat.size();
        if (t.lats.empty()) {
            t.proto = L;
            t.precision = m.sim->p.precision;
        }
        const int li = (int)t.lats.size();
        t.lats.push_back(L);
        t.mems.push_back(&m);
        t.blk_lat.insert(t.blk_lat.end(), L.nblocks, li);
    }
    pl->classes.clear();
    int cus = 0;
    {
        const ce_status st = device_cus(&cus);
        if (st != CE_OK) return st;
    }
    for (auto &kv : by_class) {
        // every hardware block stays resident and walks the class's
        // per-lattice blocks; more blocks than fit would queue behind full
        // compute units
        ClassTable &t = kv.second;
        const int per = batched_resident_blocks(t.proto, t.precision);
        if (per < 1) return fail(CE_EDEVICE, "batched kernel cannot be resident");
        const long long total = (long long)t.blk_lat.size();
        long long g = std::min<long long>(total, (long long)per * cus);
        if (g >= 8) g = g / 8 * 8;
        t.grid = (int)g;
    }
    {
        const ce_status st = ensure_lanes(pl);
        if (st != CE_OK) return st;
    }
    size_t need = 0;
    for (auto &kv : by_class) {
        need += align_up(kv.second.lats.size() * sizeof(Lattice)) + align_up(kv.second.blk_lat.size() * sizeof(int)) +
                align_up(kv.second.lats.size() * sizeof(long long));
        pl->classes.push_back(std::move(kv.second));
    }
    if (need > T.bytes) {
        if (T.d) CE_HIP(hipFree(T.d));
        T.d = nullptr;
        T.bytes = 0;
        const size_t want = std::max<size_t>(need * 2, 1 << 20);
        CE_HIP(hipMalloc(&T.d, want));
        T.bytes = want;
    }
    size_t off = 0;
    for (ClassTable &t : pl->classes) {
        t.d_lats = reinterpret_cast<Lattice *>(T.d + off);
        off += align_up(t.lats.size() * sizeof(Lattice));
        t.d_blk = reinterpret_cast<int *>(T.d + off);
        off += align_up(t.blk_lat.size() * sizeof(int));
        t.d_rem = reinterpret_cast<long long *>(T.d + off);
        off += align_up(t.lats.size() * sizeof(long long));
        CE_HIP(hipMemcpyAsync(t.d_lats, t.lats.data(), t.lats.size() * sizeof(Lattice), hipMemcpyHostToDevice,
                              pl->table_stream));
        CE_HIP(hipMemcpyAsync(t.d_blk, t.blk_lat.data(), t.blk_lat.size() * sizeof(int), hipMemcpyHostToDevice,
                              pl->table_stream));
    }
    // the upload runs beside the block in flight; the next launch is queued
    // only after it has landed
    CE_HIP(hipStreamSynchronize(pl->table_stream));
    pl->cur_buf = b;
    // lanes: largest class first onto the least loaded lane
    const int nc = (int)pl->classes.size();
    std::vector<double> work(nc, 0.0);
    for (int c = 0; c < nc; c++)
        for (const Lattice &L : pl->classes[c].lats) work[c] += (double)L.nsites * L.nf;
    std::vector<int> order(nc);
    for (int c = 0; c < nc; c++) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    double load[ce_pool::kLanes] = {};
    const int nl = std::max(1, std::min(nc, ce_pool::kLanes));
    pl->lane_of.assign(nc, 0);
    for (int c : order) {
        int best = 0;
        for (int l = 1; l < nl; l++)
            if (load[l] < load[best]) best = l;
        pl->lane_of[c] = best;
        load[best] += work[c];
    }
    pl->dirty = false;
    pl->blocks_since_rebuild = 0;
    return CE_OK;
}

hipError_t launch_class(const ClassTable &t, hipStream_t st)
{
    return launch_batched(t.d_lats, t.d_blk, (int)t.blk_lat.size(), t.grid, t.proto, t.precision, st);
}

// k steps of every class, ordered after the work already on `st` and ahead of
// what follows it.  One class runs its chain on `st`; several fork onto the
// lanes, each lane running the chains of its classes, and join again.
hipError_t launch_block(ce_pool *pl, hipStream_t st, int k)
{
    const int nc = (int)pl->classes.size();
    if (nc == 1) {
        for (int i = 0; i < k; i++) {
            const hipError_t e = launch_class(pl->classes[0], st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const int nl = std::min(nc, ce_pool::kLanes);
    hipError_t e = hipEventRecord(pl->fork_ev, st);
    for (int l = 0; l < nl && e == hipSuccess; l++) e = hipStreamWaitEvent(pl->lanes[l], pl->fork_ev, 0);
    for (int c = 0; c < nc && e == hipSuccess; c++)
        for (int i = 0; i < k && e == hipSuccess; i++) e = launch_class(pl->classes[c], pl->lanes[pl->lane_of[c]]);
    for (int l = 0; l < nl && e == hipSuccess; l++) {
        e = hipEventRecord(pl->join_ev[l], pl->lanes[l]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, pl->join_ev[l], 0);
    }
    return e;
}


ce_status build_pool_graph(ce_pool *pl, int k, hipGraphExec_t *out)
{
    if (!pl->cap_stream) CE_HIP(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    CE_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeRelaxed));
    hipError_t err = launch_block(pl, pl->cap_stream, k);
    const hipError_t e2 = hipStreamEndCapture(pl->cap_stream, &g);
    if (err != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(CE_EDEVICE, "pool capture failed: %s", hipGetErrorString(err != hipSuccess ? err : e2));
    }
    hipGraphExec_t exec = nullptr;
    err = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return fail(CE_EDEVICE, "pool graph instantiate failed: %s", hipGetErrorString(err));
    *out = exec;
    return CE_OK;
}

Member *find(ce_pool *pl, long long id)
{
    auto it = pl->members.find(id);
    return it == pl->members.end() ? nullptr : &it->second;
}

}  // namespace

extern "C" {

ce_status ce_pool_launch_for(const ce_params *p, ce_launch *out)
{
    ce_status st = validate(p);
    if (st != CE_OK) return st;
    if (!out) return fail(CE_EINVAL, "out is NULL");
    *out = member_launch(p);
    return CE_OK;
}

ce_status ce_pool_create(size_t budget_bytes, void *stream, ce_pool **out)
{
    if (!out) return fail(CE_EINVAL, "out is NULL");
    *out = nullptr;
    ce_pool *pl = new (std::nothrow) ce_pool();
    if (!pl) return fail(CE_ENOMEM, "host allocation failed");
    pl->budget = budget_bytes;
    if (stream) {
        pl->stream = static_cast<hipStream_t>(stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&pl->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete pl;
            return fail(CE_EDEVICE, "stream creation failed: %s", hipGetErrorString(e));
        }
        pl->own_stream = true;
    }
    *out = pl;
    return CE_OK;
}

namespace {

// Where an admitted member's state comes from: host fields, a generation
// spec or a grid image (exactly one set).
struct Source {
    const double *phi = nullptr, *phidot = nullptr;
    const ce_init_spec *spec = nullptr;
    const void *image = nullptr;
    size_t image_bytes = 0;
};

// Admission with an explicit member launch (cfg) or the default one.  static:
// an unnamed namespace inside extern "C" does not keep a C-linkage name local.
static ce_status admit(ce_pool *pl, const ce_params *p, const ce_launch *cfg, const Source &src, int64_t nsteps,
                int64_t *job_id)
{
    if (!pl || !p || !job_id) return fail(CE_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(CE_EINVAL, "nsteps must be >= 0");
    if (cfg && cfg->grid == 0) return fail(CE_EINVAL, "pool members need an explicit grid");
    ce_params q = *p;
    q.arena = nullptr;
    q.arena_bytes = 0;
    size_t bytes = 0;
    ce_status st = ce_required_bytes(&q, &bytes);
    if (st != CE_OK) return st;
    void *mem = nullptr;
    hipStream_t ls = nullptr;
    {
        // reserve the bytes, take cached memory of this size if any, and an
        // idle load stream
        std::lock_guard<std::mutex> g(pl->mu);
        if (pl->closing) return fail(CE_ESTATE, "the pool is being destroyed");
        if (bytes > pl->budget)
            return fail(CE_EINVAL, "admission needs %zu bytes, more than the pool's whole budget of %zu", bytes,
                        pl->budget);
        if (!pl->read_stream) CE_HIP(hipStreamCreateWithFlags(&pl->read_stream, hipStreamNonBlocking));
        if (pl->used + bytes > pl->budget)
            return fail(CE_EBUSY, "admission needs %zu bytes, %zu of %zu in use", bytes, pl->used, pl->budget);
        if (pl->load_streams.empty()) {
            hipStream_t n = nullptr;
            CE_HIP(hipStreamCreateWithFlags(&n, hipStreamNonBlocking));
            pl->all_load_streams.push_back(n);
            pl->load_streams.push_back(n);
        }
        ls = pl->load_streams.back();
        pl->load_streams.pop_back();
        pl->admitting++;
        pl->used += bytes;
        mem = take_cached(pl, bytes);
        if (!mem) st = trim_cache(pl, 0);
    }
    auto give_back = [&](void *m) {
        std::lock_guard<std::mutex> g(pl->mu);
        pl->used -= bytes;
        if (m) {
            pl->free_mem.emplace(bytes, m);
            pl->cached += bytes;
        }
        pl->load_streams.push_back(ls);
        if (--pl->admitting == 0) pl->idle.notify_all();
    };
    if (st != CE_OK) {
        give_back(nullptr);
        return st;
    }
    if (!mem && hipMalloc(&mem, bytes) != hipSuccess) {
        mem = nullptr;
        {
            std::lock_guard<std::mutex> g(pl->mu);
            st = trim_cache(pl, pl->budget);  // drop the whole cache, then try once more
        }
        if (st != CE_OK || hipMalloc(&mem, bytes) != hipSuccess) {
            give_back(nullptr);
            return st != CE_OK ? st : fail(CE_ENOMEM, "member allocation of %zu bytes failed", bytes);
        }
    }
    // the member loads on the pool's load stream, beside whatever block is
    // running on the pool stream; the host waits for its own load only
    q.stream = ls;
    q.arena = mem;
    q.arena_bytes = bytes;
    ce_sim *s = nullptr;
    st = ce_create(&q, &s);
    if (st == CE_OK) st = apply_launch(s, cfg ? *cfg : member_launch(&q));
    if (st == CE_OK) {
        if (src.image)
            st = ce_restore_image(s, src.image, src.image_bytes);
        else if (src.spec)
            st = ce_generate_fields(s, src.spec);
        else
            st = ce_load_fields(s, 0, q.nfields, src.phi, src.phidot);
    }
    // device copies of the member's step budget and buffer parity, read by
    // the batched kernels and updated by each step's tail
    const long long init_remaining = nsteps;
    const int init_cur = s ? s->cur : 0;
    if (st == CE_OK) {
        hipError_t e = hipMemcpyAsync(&s->lat.sc->remaining, &init_remaining, sizeof(long long),
                                      hipMemcpyHostToDevice, ls);
        if (e == hipSuccess) e = hipMemcpyAsync(&s->lat.sc->cur, &init_cur, sizeof(int), hipMemcpyHostToDevice, ls);
        if (e == hipSuccess) e = hipStreamSynchronize(ls);
        if (e != hipSuccess) st = fail(CE_EDEVICE, "admission failed: %s", hipGetErrorString(e));
    }
    if (st != CE_OK) {
        if (s) ce_destroy(s);
        give_back(mem);
        return st;
    }
    // the load stream goes back to the list for the next admission
    s->stream = pl->read_stream;
    std::lock_guard<std::mutex> g(pl->mu);
    pl->load_streams.push_back(ls);
    if (--pl->admitting == 0) pl->idle.notify_all();
    const long long id = pl->next_id++;
    Member &m = pl->members[id];
    m.sim = s;
    m.mem = mem;
    m.bytes = bytes;
    m.remaining = nsteps;
    m.init_remaining = nsteps;
    m.init_cur = init_cur;
    if (nsteps > 0) pl->dirty = true;
    *job_id = id;
    return CE_OK;
}

}  // namespace

ce_status ce_pool_admit(ce_pool *pl, const ce_params *p, const double *phi, const double *phidot, int64_t nsteps,
                        int64_t *job_id)
{
    Source src;
    src.phi = phi;
    src.phidot = phidot;
    return admit(pl, p, nullptr, src, nsteps, job_id);
}

ce_status ce_pool_admit_with_launch(ce_pool *pl, const ce_params *p, const ce_launch *launch, const double *phi,
                                    const double *phidot, int64_t nsteps, int64_t *job_id)
{
    if (!launch) return fail(CE_EINVAL, "launch is NULL");
    Source src;
    src.phi = phi;
    src.phidot = phidot;
    return admit(pl, p, launch, src, nsteps, job_id);
}

ce_status ce_pool_admit_generated(ce_pool *pl, const ce_params *p, const ce_launch *launch,
                                  const ce_init_spec *spec, int64_t nsteps, int64_t *job_id)
{
    if (!spec) return fail(CE_EINVAL, "spec is NULL");
    Source src;
    src.spec = spec;
    return admit(pl, p, launch, src, nsteps, job_id);
}

ce_status ce_pool_admit_image(ce_pool *pl, const void *image, size_t bytes, int64_t nsteps, int64_t *job_id)
{
    ce_params q;
    ce_status st = ce_image_params(image, bytes, &q);
    if (st != CE_OK) return st;
    // the member runs with the launch saved in the image (its grid is
    // explicit), so its continuation is bitwise the one it was saved from
    ce_image_header h;
    memcpy(&h, image, sizeof(h));
    Source src;
    src.image = image;
    src.image_bytes = bytes;
    return admit(pl, &q, &h.launch, src, nsteps, job_id);
}

ce_status ce_pool_set_member_launch(ce_pool *pl, int64_t job_id, const ce_launch *cfg)
{
    if (!pl || !cfg) return fail(CE_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(pl->mu);
    Member *m = find(pl, job_id);
    if (!m) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
    if (cfg->grid == 0) return fail(CE_EINVAL, "pool members need an explicit grid");
    // blocks in flight read the member's descriptor from the launch tables,
    // which hold copies; the change takes effect with the next block
    const ce_status st = ce_set_launch(m->sim, cfg);
    if (st == CE_OK) pl->dirty = true;
    return st;
}

ce_status ce_pool_run_block(ce_pool *pl, int32_t k)
{
    if (!pl) return fail(CE_EINVAL, "pool is NULL");
    if (k < 0 || k > 4096) return fail(CE_EINVAL, "k must be 0..4096");
    if (k == 0) return CE_OK;
    // at most two blocks in flight: the one running and this one; a rebuild
    // rewrites the table buffer the block before the running one read.
    // Both waits happen before taking the lock, so an admission on another
    // thread is not held up by them.
    {
        ce_status st = wait_block(pl, pl->seq - 2);
        if (st == CE_OK) st = wait_block(pl, pl->tbuf[1 - pl->cur_buf].last_seq);
        if (st != CE_OK) return st;
    }
    std::lock_guard<std::mutex> g(pl->mu);
    if (pl->dirty) {
        ce_status st = rebuild(pl);
        if (st != CE_OK) return st;
    }
    if (pl->classes.empty()) return CE_OK;
    if (!pl->block_ev[0])
        for (int i = 0; i < ce_pool::kEvRing; i++)
            CE_HIP(hipEventCreateWithFlags(&pl->block_ev[i], hipEventDisableTiming));
    ce_pool::TableBuf &T = pl->tbuf[pl->cur_buf];
    // step budgets: while any member has a quota (and once more after, to
    // restore the plain counts), write every member's budget for this block
    bool any_quota = false;
    for (const ClassTable &t : pl->classes)
        for (const Member *m : t.mems) any_quota |= m->quota >= 0;
    if (any_quota || pl->budgets_set) {
        size_t n = 0;
        for (const ClassTable &t : pl->classes) n += t.mems.size();
        const int hb = (int)(pl->seq & 1);  // the block that last used it has finished
        if (pl->h_rem_cap[hb] < n) {
            if (pl->h_rem[hb]) CE_HIP(hipHostFree(pl->h_rem[hb]));
            pl->h_rem[hb] = nullptr;
            pl->h_rem_cap[hb] = 0;
            const size_t cap = std::max<size_t>(n * 2, 256);
            CE_HIP(hipHostMalloc((void **)&pl->h_rem[hb], cap * sizeof(long long), hipHostMallocDefault));
            pl->h_rem_cap[hb] = cap;
        }
        size_t off = 0;
        for (const ClassTable &t : pl->classes) {
            const size_t n_c = t.mems.size();
            for (size_t l = 0; l < n_c; l++) {
                const Member *m = t.mems[l];
                pl->h_rem[hb][off + l] = m->quota >= 0 ? std::min(m->remaining, m->quota) : m->remaining;
            }
            CE_HIP(hipMemcpyAsync(t.d_rem, pl->h_rem[hb] + off, n_c * sizeof(long long), hipMemcpyHostToDevice,
                                  pl->stream));
            CE_HIP(launch_set_remaining(t.d_lats, t.d_rem, (int)n_c, pl->stream));
            off += n_c;
        }
        pl->budgets_set = any_quota;
    }
    // a composition that has just changed may change again after this block:
    // launch directly; capture a graph once the same composition repeats.
    // A capture is attempted only while no admission is running on another
    // thread (its HIP calls could invalidate the capture); a failed capture
    // falls back to launching the block directly.
    hipGraphExec_t graph = nullptr;
    if (k > 1 && pl->blocks_since_rebuild > 0) {
        auto it = T.graphs.find(k);
        if (it != T.graphs.end()) {
            graph = it->second;
        } else if (pl->admitting == 0) {
            // pl->mu is held: no admission can start until the capture ends
            hipGraphExec_t g = nullptr;
            if (build_pool_graph(pl, k, &g) == CE_OK) graph = T.graphs.emplace(k, g).first->second;
        }
    }
    if (graph)
        CE_HIP(hipGraphLaunch(graph, pl->stream));
    else
        CE_HIP(launch_block(pl, pl->stream, k));
    const long long s = pl->seq++;
    CE_HIP(hipEventRecord(pl->block_ev[s % ce_pool::kEvRing], pl->stream));
    T.last_seq = s;
    pl->blocks_since_rebuild++;
    pl->steps_run += k;
    bool finished_any = false;
    for (auto &kv : pl->members) {
        Member &m = kv.second;
        if (m.remaining <= 0) continue;
        long long adv = std::min<long long>(k, m.remaining);
        if (m.quota >= 0) adv = std::min(adv, m.quota);
        m.remaining -= adv;
        m.sim->step += adv;
        m.sim->cur ^= (int)(adv & 1);
        if (m.remaining == 0) {
            m.finish_seq = s;
            finished_any = true;
        }
    }
    if (finished_any) pl->dirty = true;  // drop idle members from the launches
    return CE_OK;
}

ce_status ce_pool_poll(ce_pool *pl, int64_t job_id, int32_t *done, ce_energy *out)
{
    if (!pl || !done) return fail(CE_EINVAL, "NULL argument");
    ce_sim *sim = nullptr;
    long long remaining = 0, finish_seq = -1;
    {
        std::lock_guard<std::mutex> g(pl->mu);
        Member *m = find(pl, job_id);
        if (!m) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
        sim = m->sim;
        remaining = m->remaining;
        finish_seq = m->finish_seq;
    }
    if (remaining > 0) {
        // steps still to enqueue: not done; its current state needs every
        // block enqueued so far
        *done = 0;
        if (!out) return CE_OK;
        CE_HIP(hipStreamSynchronize(pl->stream));
        return ce_energies(sim, out);
    }
    // only the block that holds its last step has to finish
    ce_status st = wait_block(pl, finish_seq);
    if (st != CE_OK) return st;
    *done = 1;
    return out ? ce_energies(sim, out) : CE_OK;
}

ce_status ce_pool_set_quota(ce_pool *pl, int64_t job_id, int64_t steps_per_block)
{
    if (!pl) return fail(CE_EINVAL, "pool is NULL");
    std::lock_guard<std::mutex> g(pl->mu);
    Member *m = find(pl, job_id);
    if (!m) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
    m->quota = steps_per_block < 0 ? -1 : steps_per_block;
    return CE_OK;
}

ce_status ce_pool_steps_left(const ce_pool *pl, int64_t job_id, int64_t *left)
{
    if (!pl || !left) return fail(CE_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(const_cast<ce_pool *>(pl)->mu);
    auto it = pl->members.find(job_id);
    if (it == pl->members.end()) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
    *left = it->second.remaining;
    return CE_OK;
}

ce_status ce_pool_retire(ce_pool *pl, int64_t job_id, double *f, double *fdot)
{
    if (!pl) return fail(CE_EINVAL, "pool is NULL");
    ce_sim *sim = nullptr;
    long long remaining = 0, finish_seq = -1;
    {
        std::lock_guard<std::mutex> g(pl->mu);
        Member *m = find(pl, job_id);
        if (!m) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
        sim = m->sim;
        remaining = m->remaining;
        finish_seq = m->finish_seq;
    }
    // the member's last block ran on the pool stream; its own stream (the
    // pool's read stream) does the readback
    const bool was_active = remaining > 0;
    if (was_active) {
        CE_HIP(hipStreamSynchronize(pl->stream));
    } else {
        const ce_status st = wait_block(pl, finish_seq);
        if (st != CE_OK) return st;
    }
    if (f || fdot) {
        ce_status st = ce_read_fields(sim, f, fdot);
        if (st != CE_OK) return st;
    }
    std::lock_guard<std::mutex> g(pl->mu);
    Member *m = find(pl, job_id);
    if (!m) return fail(CE_EINVAL, "pool member %lld was retired meanwhile", (long long)job_id);
    pl->used -= m->bytes;
    ce_destroy(m->sim);
    // no block still to run touches this memory: keep it for the next member
    pl->free_mem.emplace(m->bytes, m->mem);
    pl->cached += m->bytes;
    pl->members.erase(job_id);
    if (was_active) pl->dirty = true;
    return CE_OK;
}

ce_status ce_pool_save_member(ce_pool *pl, int64_t job_id, void *buf, size_t bytes)
{
    if (!pl) return fail(CE_EINVAL, "pool is NULL");
    ce_sim *sim = nullptr;
    long long remaining = 0, finish_seq = -1;
    {
        std::lock_guard<std::mutex> g(pl->mu);
        Member *m = find(pl, job_id);
        if (!m) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
        sim = m->sim;
        remaining = m->remaining;
        finish_seq = m->finish_seq;
    }
    // every step enqueued so far must have run: the host's step count and
    // buffer parity of the member then describe the device state
    if (remaining > 0) {
        CE_HIP(hipStreamSynchronize(pl->stream));
    } else {
        const ce_status st = wait_block(pl, finish_seq);
        if (st != CE_OK) return st;
    }
    return ce_save_image(sim, buf, bytes);
}

ce_status ce_pool_member_image_bytes(const ce_pool *pl, int64_t job_id, size_t *out)
{
    if (!pl || !out) return fail(CE_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(const_cast<ce_pool *>(pl)->mu);
    Member *m = find(const_cast<ce_pool *>(pl), job_id);
    if (!m) return fail(CE_EINVAL, "no pool member %lld", (long long)job_id);
    return ce_image_bytes(m->sim, out);
}

ce_status ce_pool_get_info(const ce_pool *pl, ce_pool_info *out)
{
    if (!pl || !out) return fail(CE_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(const_cast<ce_pool *>(pl)->mu);
    memset(out, 0, sizeof(*out));
    out->budget_bytes = pl->budget;
    out->used_bytes = pl->used;
    out->members = (int32_t)pl->members.size();
    for (const auto &kv : pl->members) out->active += kv.second.remaining > 0;
    out->classes = (int32_t)pl->classes.size();
    out->admitting = pl->admitting;
    out->steps_run = pl->steps_run;
    return CE_OK;
}

void ce_pool_destroy(ce_pool *pl)
{
    if (!pl) return;
    {
        // admissions in progress on other threads hold the pool's streams
        // and memory: wait for them, and turn away any that arrive meanwhile
        std::unique_lock<std::mutex> g(pl->mu);
        pl->closing = true;
        pl->idle.wait(g, [pl] { return pl->admitting == 0; });
    }
    if (pl->stream) (void)hipStreamSynchronize(pl->stream);
    for (ce_pool::TableBuf &T : pl->tbuf) {
        drop_graphs(T);
        if (T.d) (void)hipFree(T.d);
    }
    for (auto &kv : pl->members) {
        ce_destroy(kv.second.sim);
        if (kv.second.mem) (void)hipFree(kv.second.mem);
    }
    pl->members.clear();
    for (auto &kv : pl->free_mem) (void)hipFree(kv.second);
    pl->free_mem.clear();
    for (hipEvent_t e : pl->block_ev)
        if (e) (void)hipEventDestroy(e);
    for (long long *h : pl->h_rem)
        if (h) (void)hipHostFree(h);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    for (int l = 0; l < ce_pool::kLanes; l++) {
        if (pl->lanes[l]) (void)hipStreamDestroy(pl->lanes[l]);
        if (pl->join_ev[l]) (void)hipEventDestroy(pl->join_ev[l]);
    }
    if (pl->fork_ev) (void)hipEventDestroy(pl->fork_ev);
    std::vector<hipStream_t> streams = pl->all_load_streams;
    streams.push_back(pl->table_stream);
    streams.push_back(pl->read_stream);
    for (hipStream_t s : streams)
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    if (pl->own_stream && pl->stream) (void)hipStreamDestroy(pl->stream);
    delete pl;
}

}  // extern "C"
