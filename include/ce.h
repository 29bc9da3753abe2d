/*
 * ce.h -- C ABI of the MI355X (gfx950) lattice scalar-field evolution library.
 *
 * The library evolves interacting classical scalar fields on a periodic 1-, 2-
 * or 3-dimensional lattice, with or without a self-consistent expanding
 * background, by the staggered leapfrog described in the paper's "Parallel
 * Algorithms" section: field values f at integer times, their derivatives half
 * a step ahead, a drift of f by a full step followed by a kick of the
 * derivatives computed from the new field values.  Which runs are possible
 * (one, two or three dimensions; expansion on or off; a model potential with
 * its derivatives; masses, couplings, grid points and time step as run
 * parameters) follows the paper's Abstract and "Overview" section.
 *
 * Program units and equations (derived from the Friedmann-Robertson-Walker
 * equations; the paper states none):
 *   f_i   = a phi_i / phi_0, conformal time, lengths/times in 1/(sqrt(lambda) phi_0)
 *   f_i'' = Lap f_i - dV/df_i + (a''/a) f_i
 *   V     = lambda/4 f0^4 + sum_{j>=1} G_j/2 f0^2 fj^2 + a^2/2 sum_i mu2_i f_i^2 + a^4 V0
 *   a''   = -a'^2/a + kappa (2/3 Grad + V)/a        (Grad, V: volume means)
 *   check:  a'^2 = kappa rho/3, rho = Kin + Grad + V
 * mu2_i < 0 with a vacuum energy V0 > 0 gives the tachyonic / hybrid
 * potentials lambda/4 (phi^2 - v^2)^2: mu2_0 = -lambda v^2, V0 = lambda v^4/4.
 * Lap is the nearest-neighbour (2d+1)-point periodic stencil, dx = L/N.
 *
 * Conventions for every call:
 *  - Every function returns ce_status; nothing throws across the ABI.  On a
 *    failure ce_last_error() (thread-local) describes it and the object is
 *    unchanged, except for CE_ENONFINITE, where the state is kept as computed.
 *  - Host pointers are borrowed for the duration of the call only.
 *  - Device memory: the library owns what it allocates (hipMalloc).  When
 *    ce_params.arena is set, every device buffer of the simulation is carved
 *    from that caller-owned block instead and the library never frees it.
 *  - Work is queued asynchronously on ce_params.stream (a hipStream_t, e.g.
 *    PyTorch's current stream); NULL selects a stream the library creates.
 *    Calls that return host data synchronise that stream.
 *  - Arrays are C-ordered [field][i][j][k] with k contiguous; i is the first
 *    (slowest) spatial axis, the axis the paper slices into slabs.
 */
#ifndef CE_H
#define CE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CE_OK = 0,
    CE_EINVAL = -1,      /* bad argument or parameter set */
    CE_ENOMEM = -2,      /* device or host allocation failed / arena too small */
    CE_EDEVICE = -3,     /* a HIP call failed */
    CE_ESTATE = -4,      /* call not valid in the current state (e.g. step before load) */
    CE_ENONFINITE = -5,  /* a volume sum became NaN/Inf; state kept, step reported */
    CE_EBUSY = -6        /* pool admission refused: over the memory budget */
} ce_status;

enum { CE_FP32 = 0, CE_FP64 = 1 };   /* storage of f and its derivative; sums and a(t) always FP64 */
#define CE_MAX_FIELDS 3

/* Model potentials.  The paper's programs take the model as a file that
 * defines the potential and its derivatives ("Overview" section); here a run
 * names one of:
 *   CE_MODEL_QUARTIC     the potential V above (lambda, G, mu2, vacuum);
 *   CE_MODEL_POLYNOMIAL  a user-defined polynomial of the fields, given as
 *                        up to CE_MAX_TERMS terms of the physical potential
 *                            V(phi) = sum_t coef_t phi_0^e_t0 phi_1^e_t1 phi_2^e_t2
 *                        (program units, exponents 0..CE_MAX_EXP, total
 *                        degree D_t = sum_i e_ti <= CE_MAX_DEGREE).  In the
 *                        program variables f = a phi a term becomes
 *                        coef_t a^(4 - D_t) prod_i f_i^e_ti, and its derivative
 *                        with respect to f_i is taken term by term.  Mass
 *                        terms (degree 2), a vacuum energy (degree 0),
 *                        lambda phi^4 (degree 4), couplings phi^2 chi^2,
 *                        trilinear or sixth-order terms are all terms of this
 *                        form; lambda, G, mu2 and vacuum must be 0 with it. */
enum { CE_MODEL_QUARTIC = 0, CE_MODEL_POLYNOMIAL = 1 };
#define CE_MAX_TERMS 8
#define CE_MAX_EXP 6
#define CE_MAX_DEGREE 8
typedef struct {
    double coef;                  /* coefficient of the term in V(phi), finite */
    int32_t exp[CE_MAX_FIELDS];   /* exponent of each field, 0..CE_MAX_EXP (0 for fields beyond nfields) */
    int32_t pad_;
} ce_term;

typedef struct {
    int32_t dims;        /* 1, 2 or 3 */
    int32_t N;           /* points per edge; multiple of 4, >= 4 */
    int32_t nfields;     /* 1..CE_MAX_FIELDS; field 0 is the inflaton */
    int32_t precision;   /* CE_FP32 or CE_FP64 */
    int32_t model;       /* CE_MODEL_QUARTIC or CE_MODEL_POLYNOMIAL */
    int32_t expansion;   /* 0: a == 1 fixed; 1: self-consistent a(tau) */
    double L;            /* box edge (program units), dx = L/N */
    double dt;           /* time step (program units), > 0 */
    double lambda;       /* quartic self-coupling (1 in program units; 0 allowed) */
    double G[CE_MAX_FIELDS];   /* G_j = g_j^2/lambda for fields j >= 1; G[0] unused */
    double mu2[CE_MAX_FIELDS]; /* mass^2 of each field (program units), default 0; may be
                                  negative (tachyonic) */
    double kappa;        /* 8 pi (phi_0/M_p)^2; used only with expansion, > 0 there */
    double vacuum;       /* V0: constant term of the physical potential (program units),
                            a^4 V0 in the comoving potential; default 0 */
    int32_t nterms;      /* CE_MODEL_POLYNOMIAL: 1..CE_MAX_TERMS; else 0 */
    int32_t pad_;
    ce_term terms[CE_MAX_TERMS];  /* CE_MODEL_POLYNOMIAL: terms[0 .. nterms-1] */
    void *stream;        /* hipStream_t or NULL */
    void *arena;         /* optional caller-owned device memory, 256-byte aligned */
    size_t arena_bytes;  /* its size; see ce_required_bytes */
} ce_params;

/* Volume-averaged diagnostics at one integer step (comoving program units). */
typedef struct {
    int64_t step;
    double tau;
    double a;            /* a at this step */
    double adot;         /* a' at this step (mean of the two neighbouring half steps) */
    double hubble;       /* a'/a^2 */
    double kin[CE_MAX_FIELDS];    /* 1/2 <(f' - (a'/a) f)^2> */
    double grad[CE_MAX_FIELDS];   /* 1/2 <|grad f|^2> = -1/2 <f Lap f> */
    double pot;          /* <V> */
    double rho;          /* sum kin + sum grad + pot */
    double mean[CE_MAX_FIELDS];   /* <f_i> */
    double mean_sq[CE_MAX_FIELDS];/* <f_i^2> */
    double friedmann_residual;    /* (a'^2 - kappa rho/3)/a'^2; 0 without expansion */
    int32_t nonfinite;   /* 1 if any volume sum of this step was NaN/Inf */
    int32_t pad_;
} ce_energy;

typedef struct ce_sim ce_sim;   /* opaque, library-owned */

/* Device bytes one simulation with these parameters needs (for an arena). */
ce_status ce_required_bytes(const ce_params *p, size_t *out);

/* Create one run: the lattice and model the paper's programs take as run
 * parameters (dimension, grid points, box, time step, model potential,
 * couplings and masses, expansion on or off: Abstract, "Overview" section).
 * Validates p (ranges above, leapfrog stability of the Laplacian part
 * dt * 2 sqrt(dims) / dx < 2) and allocates device storage: 4 arrays per
 * field (field and derivative, each twice for the ping-pong) in the storage
 * type, plus the FP64 scalar state.  *out is library-owned until ce_destroy.
 * CE_EINVAL for a parameter out of range, CE_ENOMEM when device memory (or
 * the caller's arena) is too small; nothing is allocated on failure.  No
 * kernel runs. */
ce_status ce_create(const ce_params *p, ce_sim **out);

/* Copy initial data for fields first .. first+count-1.  phi and phidot are host
 * FP64 arrays [count][N^dims], C-ordered: the physical program-unit field and
 * its time derivative at tau = 0, a = 1.  When every field has been loaded the
 * library queues the start-up half step (derivatives moved to tau = dt/2) and
 * checks leapfrog stability including the potential's curvature. */
ce_status ce_load_fields(ce_sim *s, int32_t first, int32_t count,
                         const double *phi, const double *phidot);

/* Seeded initial conditions generated on the device: each field is its
 * homogeneous value plus a Gaussian random field of small fluctuations, the
 * starting point of the preheating runs the paper's programs are built for.
 * Definition (K = N/4; the same for every field i and kind, kind 0 the field
 * and 1 its time derivative):
 *   - wave vectors n with integer components in [-K, K]; box index
 *     b(n) = sum_j (n_j + K) (2K+1)^(dims-1-j);
 *   - random words: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel
 *     random numbers: as easy as 1, 2, 3", SC 2011), key (seed, 0), counter
 *     (b(n), 2 i + kind, 0, 0); w0, w1 its first two output words;
 *   - u1 = ((w0 >> 11) + 1) 2^-53, u2 = (w1 >> 11) 2^-53 and the Box-Muller
 *     pair X = sqrt(-2 ln u1) cos(2 pi u2), Y = sqrt(-2 ln u1) sin(2 pi u2);
 *   - c_n = sigma_n (X + iY) for 0 < |n|^2 <= K^2, else 0, with k = 2 pi |n|/L,
 *     omega = sqrt(k^2 + m_eff2[i]), sigma_n = amp / sqrt(2 omega L^dims)
 *     (kind 0) or amp sqrt(omega/2) / sqrt(L^dims) (kind 1);
 *   - phi_i(x) = background[i] + Re sum_n c_n exp(2 pi i n.x/N) (kind 0),
 *     phidot_i(x) = background_dot[i] + the same sum of the kind-1 modes.
 * The sums run as band-limited inverse FFTs on the device; results agree with
 * the definition to FP64 rounding. */
typedef struct {
    uint64_t seed;
    double amp;                           /* fluctuation amplitude, >= 0 */
    double background[CE_MAX_FIELDS];     /* homogeneous field values (program units) */
    double background_dot[CE_MAX_FIELDS]; /* homogeneous time derivatives */
    double m_eff2[CE_MAX_FIELDS];         /* effective mass^2 shaping each spectrum, >= 0 */
} ce_init_spec;

/* Generate every field as above and start the run exactly as ce_load_fields
 * does once all fields are present (stability check, start-up half step).
 * Needs N a power of two, N <= 2048; the transforms use the simulation's own
 * second buffers and staging as scratch, so no memory is allocated except for
 * lattices too small to hold the scratch there.  CE_ESTATE after the run has
 * started; CE_EINVAL for an unsupported N or a non-finite / negative spec. */
ce_status ce_generate_fields(ce_sim *s, const ce_init_spec *spec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * ce_generate_fields, with the same results bit for bit, but the transform
 * intermediates live in a file-scope device array of CE_GEN_SCRATCH_BYTES
 * (one per GPU, held until the process ends) instead of the simulation's
 * spare buffers or a temporary allocation, and the call allocates nothing.
 * The array of the current device is used, which must be the simulation's
 * device.  Every call on one GPU shares that array: calls that overlap on one
 * GPU (other threads, other simulations) race and must be serialised by the
 * caller.  Nothing in it needs to start at zero (every intermediate is written
 * before it is read); the call returns after its last use of it.  CE_EINVAL
 * when the lattice needs more scratch than that: 3-D up to N = 256 and 2-D
 * up to N = 2048 fit; 1-D needs none. */
#define CE_GEN_SCRATCH_BYTES (64u << 20)
ce_status ce_generate_fields_noalloc(ce_sim *s, const ce_init_spec *spec);

/* Advance nsteps >= 0 steps of the staggered leapfrog ("Parallel
 * Algorithms" section): per step, the field values move by a full step with
 * the half-step derivatives, the derivatives then move by a full step with
 * the second derivative computed from the new field values (nearest-neighbour
 * Laplacian, potential derivative, and with expansion the scale-factor
 * term), and the FP64 volume sums of that step give the scale factor and the
 * diagnostics.  Asynchronous on the simulation's stream; nothing is
 * allocated.  Before all fields are loaded: CE_ESTATE.  A non-finite volume
 * sum does not stop the steps; ce_energies reports it. */
ce_status ce_step(ce_sim *s, int64_t nsteps);

/* Synchronise and return the diagnostics of the current step: the
 * volume-averaged kinetic, gradient and potential energies, the scale factor
 * and its derivative, and per field <f> and <f^2>, at the integer step where
 * the paper's integrator holds the field values ("Parallel Algorithms"
 * section; the energies take the derivative time-centred there).  *out is
 * caller-owned.  Returns CE_ENONFINITE (with *out filled for the current
 * step) if any step so far produced a non-finite volume sum; ce_last_error()
 * names the first such step. */
ce_status ce_energies(ce_sim *s, ce_energy *out);

/* Diagnostics of the last `count` steps up to the current one (oldest first);
 * the library keeps the most recent CE_ENERGY_LOG steps. */
#define CE_ENERGY_LOG 1024
ce_status ce_energy_log(ce_sim *s, int32_t count, ce_energy *out);

/* Synchronise and copy the state to host FP64 arrays [nfields][N^dims]:
 * f at the current integer step n and its derivative at n + 1/2, the two
 * times at which the paper's integrator stores them.  Either pointer may be
 * NULL. */
ce_status ce_read_fields(ce_sim *s, double *f, double *fdot);

/* Synchronise and read `count` single sites of field `field` (site index in
 * the C-ordered lattice, 0 <= index < N^dims) into host arrays f[count] and
 * fdot[count], with the same meaning as ce_read_fields.  Either output may be
 * NULL.  count <= 1<<20 per call. */
ce_status ce_read_sites(ce_sim *s, int32_t field, int64_t count, const int64_t *sites,
                        double *f, double *fdot);

/* Current step count (host-side, no synchronisation). */
ce_status ce_get_step(const ce_sim *s, int64_t *step);

/* Kernel launch configuration of the per-step pass.  The volume sums are
 * reduced in an order fixed by this configuration, so results are bitwise
 * reproducible for a given configuration and agree to rounding across them. */
enum { CE_KERNEL_DIRECT = 0,    /* one quad of 4 x-sites per thread, neighbours from cache; any dims */
       CE_KERNEL_TILED3D = 1,   /* 3-D z-streaming through an LDS plane tile */
       CE_KERNEL_STREAM2D = 2 };/* 2-D y-streaming, one 256-site x segment per wavefront; N % 256 == 0 */
typedef struct {
    int32_t kernel;           /* CE_KERNEL_* */
    int32_t sites_per_thread; /* tiled: consecutive x sites per thread, 2 or 4 */
    int32_t lanes_per_row;    /* tiled: threads per tile row; tile x edge = sites_per_thread * lanes_per_row */
    int32_t block;            /* tiled: threads per block, 256 or 512; tile y edge = block / lanes_per_row */
    int32_t planes;           /* tiled: at most this many z planes per tile, 1..N (the z column is cut
                                 into ceil(N/planes) chunks of near-equal length);
                                 2-D streaming: rows per unit, divides N */
    int32_t grid;             /* blocks per pass, 1..4096; 0 = as many as stay resident, evened so every
                                 block walks the same number of tiles */
} ce_launch;
/* Tiled shapes built (sites_per_thread, lanes_per_row, block):
 * (4,16,256) (4,8,256) (2,32,256) (2,32,512) (2,16,256) (2,16,512) (4,64,256) (4,64,512). */

/* Current launch configuration (the library picks one in ce_create). */
ce_status ce_get_launch(const ce_sim *s, ce_launch *out);

/* Replace the launch configuration; CE_EINVAL if it does not fit the lattice.
 * Allowed at any time; captured step blocks are rebuilt. */
ce_status ce_set_launch(ce_sim *s, const ce_launch *cfg);

/* Steps per captured hipGraph inside ce_step (0 = plain launches).  Default 32. */
ce_status ce_set_step_block(ce_sim *s, int32_t k);

/* Advance nsteps steps like ce_step and return, in *ms, the time between two
 * HIP events recorded on the simulation's stream around them (synchronises). */
ce_status ce_time_steps(ce_sim *s, int64_t nsteps, float *ms);

/* Wait for all work queued on the simulation's stream. */
ce_status ce_sync(ce_sim *s);

/* End a run: wait for its queued work and free everything the simulation
 * allocated (never the caller's arena or stream).  NULL-safe; s must not be
 * used afterwards. */
void ce_destroy(ce_sim *s);

/* ---- Spectra -------------------------------------------------------------
 * The paper's programs Fourier transform the fields to output their spectra
 * ("Parallel Algorithms" section, last paragraphs).  For field i at the
 * current integer step n, with F(n) = N^-dims sum_x g(x) exp(-2 pi i n.x/N)
 * over integer wave vectors n (components in [-N/2, N/2)):
 *   power[j] = sum of |F(n)|^2 over the n with floor(|n|) = j, where g is the
 *              field f (power_f) or its derivative at n + 1/2 (power_fdot),
 *              both as ce_read_fields returns them;
 *   count[j] = the number of such n.
 * Bins j = 0 .. ce_spectrum_bins - 1 = floor(sqrt(dims) N/2).  By Parseval
 * sum_j power_f[j] is the volume mean of f^2.  k = 2 pi |n| / L in program
 * units.  Sums are deterministic for a given lattice configuration. */
ce_status ce_spectrum_bins(const ce_sim *s, int32_t *nbins);

/* Synchronise and compute the spectra of field `field` into host arrays of
 * ce_spectrum_bins doubles each (any may be NULL).  Needs N a power of two
 * <= 2048; the transforms use the simulation's second ping-pong buffers and
 * staging as scratch (free between steps), so nothing is allocated.
 * CE_ESTATE before every field is loaded. */
ce_status ce_spectrum(ce_sim *s, int32_t field, double *power_f, double *power_fdot, double *count);

/* ---- Grid images: save a run and resume it later -------------------------
 * The paper's programs can write a grid image from which a run continues to
 * later times ("Overview" section).  Here an image is one flat host byte
 * buffer holding the complete state of a simulation; a simulation restored
 * from it continues bit for bit as the saved one would have (the image also
 * carries the launch configuration, which fixes the reduction order).
 *
 * Layout, version 2 (host byte order, which is little-endian on every
 * platform the library builds for):
 *   [0, 512)        ce_image_header
 *   next            the FP64 scalar state (state_bytes; opaque: a, a', tau,
 *                   step, homogeneous references and pass coefficients)
 *   next            the diagnostics ring (ring_bytes = CE_ENERGY_LOG ce_energy
 *                   records, the record of step n in slot n % CE_ENERGY_LOG)
 *   next, per field i = 0 .. nfields-1:
 *                   d_i[N^dims] then p_i[N^dims] in the storage type (FP32 or
 *                   FP64; field_bytes each, C order): the field's deviation
 *                   from its homogeneous reference at step n and its derivative
 *                   at n + 1/2 in the library's deferred form.  ce_read_fields
 *                   on the restored simulation returns the paper's variables. */
#define CE_IMAGE_MAGIC "CEGRID\0\1"
#define CE_IMAGE_VERSION 2u
typedef struct {
    char     magic[8];          /* CE_IMAGE_MAGIC */
    uint32_t version;           /* CE_IMAGE_VERSION */
    uint32_t header_bytes;      /* 512 */
    int32_t  dims, N, nfields, precision, model, expansion;
    double   L, dt, lambda, G[CE_MAX_FIELDS], mu2[CE_MAX_FIELDS], kappa;
    int64_t  step;              /* integer step of the saved state */
    ce_launch launch;           /* launch configuration, grid resolved */
    uint64_t state_bytes, ring_bytes, field_bytes, total_bytes;
    double   vacuum;            /* ce_params.vacuum */
    int32_t  nterms;            /* ce_params.nterms and terms: the model polynomial */
    int32_t  pad_;
    ce_term  terms[CE_MAX_TERMS];
    uint8_t  reserved[120];     /* zero */
} ce_image_header;

/* Size in bytes of the simulation's image. */
ce_status ce_image_bytes(const ce_sim *s, size_t *out);

/* Synchronise and write the simulation's image into the host buffer `buf` of
 * `bytes` >= ce_image_bytes.  CE_ESTATE before every field is loaded. */
ce_status ce_save_image(ce_sim *s, void *buf, size_t bytes);

/* Read the run parameters out of an image header (no device work; stream and
 * arena come back NULL).  CE_EINVAL if buf is not a version-2 image of
 * `bytes` bytes. */
ce_status ce_image_params(const void *buf, size_t bytes, ce_params *out);

/* Replace the state of `s` by the image's: s must have been created with the
 * image's parameters (every field of ce_params except stream and arena equal,
 * bit for bit) and may be fresh or already running.  The image's launch
 * configuration is applied.  CE_EINVAL for a malformed image, a parameter
 * mismatch or an image of another build's scalar-state layout. */
ce_status ce_restore_image(ce_sim *s, const void *buf, size_t bytes);

/* ---- Pool: many independent lattices advanced together ------------------
 * Batched ensembles and serving.  Every admitted lattice (a "member") keeps
 * its state on the device between step blocks; a step advances every member
 * that still has steps left with one kernel launch per class of members
 * (same precision, dimension, field count and kernel shape), so many small
 * lattices fill the GPU that one alone cannot.  Each member is computed by
 * the same blocks and in the same reduction order as a lone simulation
 * launched with ce_pool_launch_for's configuration, so its results do not
 * depend on what else is in the pool (bitwise).  Member state counts against
 * the pool's byte budget; the memory of retired members is kept for reuse by
 * later members of the same size (and released when the budget needs it or
 * the pool is destroyed).  Steps run on the pool's stream; admissions load on
 * a stream of the pool's own, beside the block in flight.
 *
 * Threads: admissions (ce_pool_admit, ce_pool_admit_with_launch,
 * ce_pool_admit_generated, ce_pool_admit_image) may run on any number of host
 * threads at once, beside the other calls.  The other calls must not overlap
 * each other.  ce_pool_destroy may be called while admissions are in
 * progress: it waits for them to return before it frees anything, and an
 * admission that reaches the pool after ce_pool_destroy has begun returns
 * CE_ESTATE.  No call may begin after ce_pool_destroy has returned (the pool
 * no longer exists), so a caller stops or joins its admission threads before
 * it destroys the pool. */
typedef struct ce_pool ce_pool;   /* opaque, library-owned */
typedef struct {
    size_t budget_bytes;   /* admission budget */
    size_t used_bytes;     /* device bytes held by members */
    int32_t members;       /* admitted and not yet retired */
    int32_t active;        /* members with steps left */
    int32_t classes;       /* launches per pool step */
    int32_t admitting;     /* admissions in progress (on any thread) */
    int64_t steps_run;     /* pool steps taken so far */
} ce_pool_info;

/* Create a pool holding at most budget_bytes of member state.  stream as in
 * ce_params (NULL: the pool creates one). */
ce_status ce_pool_create(size_t budget_bytes, void *stream, ce_pool **out);

/* Admit one lattice: create it, load phi/phidot (as ce_load_fields, all
 * fields) and queue its start-up; it then takes part in the next nsteps pool
 * steps.  p->stream and p->arena are ignored.  CE_EBUSY (nothing allocated)
 * when its bytes do not fit the budget left now (retry after a retirement);
 * CE_EINVAL when they exceed the pool's whole budget (it can never fit);
 * CE_ESTATE once ce_pool_destroy has begun.  *job_id identifies it. */
ce_status ce_pool_admit(ce_pool *pl, const ce_params *p, const double *phi, const double *phidot,
                        int64_t nsteps, int64_t *job_id);

/* ce_pool_admit with the member's launch configuration given (validated as
 * ce_set_launch; the grid must be explicit, 1..4096). */
ce_status ce_pool_admit_with_launch(ce_pool *pl, const ce_params *p, const ce_launch *launch, const double *phi,
                                    const double *phidot, int64_t nsteps, int64_t *job_id);

/* ce_pool_admit with the initial fields generated on the device from `spec`
 * (as ce_generate_fields) instead of copied from the host; launch may be NULL
 * (the default member launch) or explicit as in ce_pool_admit_with_launch. */
ce_status ce_pool_admit_generated(ce_pool *pl, const ce_params *p, const ce_launch *launch,
                                  const ce_init_spec *spec, int64_t nsteps, int64_t *job_id);

/* The launch configuration a member with these parameters uses; setting it on
 * a lone simulation (ce_set_launch) reproduces the member's results bitwise. */
ce_status ce_pool_launch_for(const ce_params *p, ce_launch *out);

/* Replace a member's launch configuration (validated as ce_set_launch; the
 * grid may be any 1..4096).  Takes effect from the next block; a lone
 * simulation with the same configuration reproduces the member bitwise only
 * if the change precedes the member's first block (prefer
 * ce_pool_admit_with_launch). */
ce_status ce_pool_set_member_launch(ce_pool *pl, int64_t job_id, const ce_launch *cfg);

/* Enqueue min(k, steps left) steps of every active member, asynchronously
 * (k launches per class; a composition seen for a second block is captured
 * as a graph).  May be called again before the previous block has run. */
ce_status ce_pool_run_block(ce_pool *pl, int32_t k);

/* *done = 1 once the member has taken all its steps (waiting for the block
 * holding its last step, not for later blocks), else 0 without waiting.
 * *out (may be NULL) receives its diagnostics at its current step (for a
 * member with steps still to enqueue this waits for every block enqueued).
 * CE_ENONFINITE as in ce_energies. */
ce_status ce_pool_poll(ce_pool *pl, int64_t job_id, int32_t *done, ce_energy *out);

/* Let the member take at most steps_per_block steps in each following block
 * (0: pause it; negative: no limit, the default).  Its results do not
 * change; only when its steps run. */
ce_status ce_pool_set_quota(ce_pool *pl, int64_t job_id, int64_t steps_per_block);

/* Steps of the member not yet enqueued by ce_pool_run_block (no waiting). */
ce_status ce_pool_steps_left(const ce_pool *pl, int64_t job_id, int64_t *left);

/* Remove a member, first copying its fields as ce_read_fields does (f and fdot
 * may be NULL); its memory returns to the pool for reuse. */
ce_status ce_pool_retire(ce_pool *pl, int64_t job_id, double *f, double *fdot);

/* Grid image of a member (the layout of ce_save_image, with the member's
 * launch configuration), after every step enqueued for it so far has run;
 * the member stays in the pool.  With ce_pool_retire this evicts a member,
 * and ce_pool_admit_image (or a lone simulation restored from the image)
 * resumes it bit for bit. */
ce_status ce_pool_member_image_bytes(const ce_pool *pl, int64_t job_id, size_t *out);
ce_status ce_pool_save_member(ce_pool *pl, int64_t job_id, void *buf, size_t bytes);

/* Admit a member from a grid image (of a lone simulation or a pool member)
 * with nsteps more steps to take; it runs with the image's launch
 * configuration.  CE_EBUSY, CE_EINVAL and CE_ESTATE as ce_pool_admit; also
 * CE_EINVAL for a malformed image. */
ce_status ce_pool_admit_image(ce_pool *pl, const void *image, size_t bytes, int64_t nsteps, int64_t *job_id);

ce_status ce_pool_get_info(const ce_pool *pl, ce_pool_info *out);

/* Free the pool and every member still in it.  NULL-safe. */
void ce_pool_destroy(ce_pool *pl);

/* Measurement only (not part of the evolution): copy `bytes` from src to dst
 * (device buffers, 16-byte aligned) as `streams` (1, 2 or 4) equal parts that
 * one kernel of `grid` 256-thread blocks (0: 16 per compute unit) reads and
 * writes side by side with 128-bit loads and nontemporal stores; *ms receives
 * the mean time of `reps` launches on `stream` (NULL: the null stream) after
 * one warm-up launch.  2 * bytes / time is the read+write rate the memory
 * system reaches for a stream shaped like a step pass, beside the HBM peak.
 * bytes must be a multiple of 16 * streams. */
ce_status ce_stream_copy(const void *src, void *dst, size_t bytes, int32_t streams, int32_t grid, int32_t reps,
                         void *stream, float *ms);

/* Measurement only: the ceiling a streaming kernel can reach.  kind selects
 * a read+write copy of `bytes` from src to dst (CE_PROBE_COPY), a read of
 * `bytes` from src whose per-thread sums go to the first grid * 256 * 16
 * bytes of dst (CE_PROBE_READ), or a write of `bytes` to dst (CE_PROBE_WRITE;
 * src unused, may be NULL).  The bytes are split into `parts` (1 or 4) equal
 * side-by-side parts; each 256-thread block issues `unroll` (1, 2, 4 or 8)
 * independent 128-bit loads per part and thread before its first store.  nt:
 * bit 0 nontemporal loads, bit 1 nontemporal stores.  grid: blocks (0: 16 per
 * compute unit; at most 2^20).  *ms receives the mean time of `reps`
 * launches on `stream` (NULL: the null stream) after one warm-up launch.
 * Buffers are device memory, 16-byte aligned, `bytes` each (a multiple of
 * 16 * parts); CE_EINVAL otherwise. */
enum { CE_PROBE_COPY = 0, CE_PROBE_READ = 1, CE_PROBE_WRITE = 2 };
ce_status ce_stream_probe(int32_t kind, const void *src, void *dst, size_t bytes, int32_t parts, int32_t unroll,
                          int32_t nt, int32_t grid, int32_t reps, void *stream, float *ms);

/* Description of the last failure on this thread ("" if none). */
const char *ce_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CE_H */
