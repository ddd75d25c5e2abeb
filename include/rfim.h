/*
 * rfim.h -- C ABI of librfim.so: Exchange Monte Carlo (parallel tempering)
 * for the 3D random field Ising model on one AMD Instinct MI355X (gfx950).
 *
 * The method (Navarro, Huang, Deng, "Adaptive Multi-GPU Exchange Monte Carlo
 * for the 3D Random Field Ising Model", arXiv:1508.06268):
 *   - H = -J sum_<ij> s_i s_j - h sum_i h_i s_i on a periodic L^3 lattice,
 *     each bond counted once (Sec. 1, Eq. 1);
 *   - R replicas of one disorder realization at temperatures T_1 < ... < T_R,
 *     each evolved by checkerboard Metropolis sweeps: sites with
 *     (x+y+z) mod 2 = 0 first, then the others (Sec. 3.1 step 4, Sec. 3.2,
 *     Eq. 3);
 *   - every `exchange_every` sweeps, the per-replica energies are reduced
 *     and adjacent temperature slots (p, p+1) with p = k (mod 2) try to swap
 *     with probability min(1, e^Delta), Delta = (b_{p+1}-b_p)(E_{p+1}-E_p)
 *     (Sec. 3.1, Eq. 2, read with the Hukushima-Nemoto sign); temperatures
 *     move, configurations stay (Sec. 3.3);
 *   - adaptive insertion of temperatures at the midpoints of the intervals
 *     with the lowest exchange rates after short trial runs (Sec. 4).
 *
 * Conventions the paper leaves open, fixed here (and identical in the test
 * oracle, so that runs with +-1 fields are reproducible bit for bit):
 *   site i = x + L*(y + L*z); sublattice index j = i >> 1;
 *   Philox4x32-10, key = (lo32(seed), hi32(seed)), counter word 3 =
 *   (tag << 28) | realization;
 *     initial spins:  tag 1, ctr = (i >> 2, 0, r),      word i & 3, s = +1 iff >= 2^31;
 *     sweep t, col c: tag 2, ctr = (j >> 2, 2t + c, r), word j & 3 = u32;
 *     exchange k:     tag 3, ctr = (p, k, 0), U53 = ((w0 >> 11) 2^32 + w1) 2^-53;
 *   +-1 fields: accept iff dE <= 0 or u32 < min(floor(exp(-beta dE) 2^32), 2^32-1),
 *   thresholds built in FP64 on the host; energies exact integers;
 *   other fields: dE and exp(-beta dE) in FP32 on the device (rare decisions
 *   may differ from an FP64 evaluation; energies are FP64 sums).
 *
 * Ownership and threading.  The caller owns every host array; inputs are
 * copied, outputs are written into caller buffers of the documented size.
 * A handle owns its device memory (from hipMalloc, or from a provider given
 * to rfim_create_ex) and orders all its work on one HIP stream (its own, or
 * one set with rfim_set_stream); inside large streaming sweeps it forks half
 * of the replicas onto a second stream and joins it back before the exchange
 * step (rfim_set_concurrency), so callers see one stream.  That second
 * stream belongs to the library, one per (device, handle stream), shared by
 * the handles issuing on that stream.  One handle is used from one thread at
 * a time; different handles are independent.
 *
 * Errors.  Calls return RFIM_OK (0) or a negative status; constructors
 * return NULL.  rfim_last_error() gives a thread-local message for the last
 * failure.  Arguments are validated before any device work.  A kernel fault
 * surfaces as RFIM_EDEVICE at the next call that synchronizes.
 */
#ifndef RFIM_H
#define RFIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rfim rfim_t;

enum {
    RFIM_OK = 0,
    RFIM_EINVAL = -1,   /* bad argument */
    RFIM_ENOMEM = -2,   /* device or host allocation failed */
    RFIM_EDEVICE = -3,  /* HIP runtime or kernel error */
    RFIM_ESTATE = -4,   /* call not valid in the handle's state */
    RFIM_ECAP = -5,     /* beyond a capacity (R_cap, sweep counter 2^31-1) */
    RFIM_EBUSY = -6     /* pool budget exhausted (batch/serving calls) */
};

enum { RFIM_FIELDS_AUTO = -1, RFIM_FIELDS_BIMODAL = 0, RFIM_FIELDS_CONTINUOUS = 1 };

/*
 * Create one realization (Sec. 3.1 steps 1-3).
 *   L       even, 2 <= L <= 1024 (odd L breaks the periodic checkerboard).
 *   R       number of replicas / temperature slots, 1 <= R <= 65536.
 *   J, h    coupling and field strength, finite.
 *   fields  host [L^3] float, natural site order, finite.  Bimodal (exact
 *           integer path) iff every value is exactly +1 or -1.
 *   temps   host [R] double, finite, > 0, strictly ascending.
 *   seed    64-bit Philox key.  Realization id 0.
 * Returns NULL on failure (see rfim_last_error()).
 */
rfim_t *rfim_create(int L, int R, double J, double h, const float *fields,
                    const double *temps, uint64_t seed);

typedef struct rfim_params {
    int L, R;
    int R_cap;              /* >= R; capacity for adaptive growth (0 = R) */
    double J, h;
    const float *fields;    /* host [L^3] */
    const double *temps;    /* host [R] */
    uint64_t seed;
    uint32_t realization;   /* < 2^28; selects an independent stream */
    int field_kind;         /* RFIM_FIELDS_AUTO / _BIMODAL / _CONTINUOUS */
} rfim_params_t;

/* Device memory provider for one handle.  alloc(bytes, ctx) returns device
 * memory of at least `bytes` bytes, 16-byte aligned, usable from the
 * handle's stream(s), or NULL (the call then fails with RFIM_ENOMEM);
 * free(ptr, ctx) takes back a pointer alloc returned, after the handle's
 * work on it has finished.  Both run on the thread that called into the
 * library (create, rfim_set_measure, destroy).  A handle asks for one block
 * at create time (all its buffers), at most two more for its default
 * storage and shape (the bit arrays of handles that start in bits, the
 * second spin buffer of a slab shape), one when a slab shape is first set, two for
 * bit storage, and three when rfim_set_measure first turns the measurement
 * on.  A caching allocator (e.g. PyTorch's) can serve them. */
typedef struct rfim_alloc {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} rfim_alloc_t;

/* As rfim_create with the extra parameters.  alloc: where the handle's own
 * device memory comes from (copied; NULL: hipMalloc / hipFree).  hip_stream
 * is a hipStream_t owned by the caller (NULL: the handle creates its own). */
rfim_t *rfim_create_ex(const rfim_params_t *params, const rfim_alloc_t *alloc, void *hip_stream);

/*
 * n sweeps of all replicas; after every sweep that makes the global sweep
 * count a multiple of exchange_every (> 0), the energies are reduced and one
 * exchange step runs (Sec. 3.1 step 4).  exchange_every = 0: no exchange.
 * Asynchronous on the handle's stream.  RFIM_ECAP if the global sweep count
 * would pass 2^31 - 1.
 */
int rfim_sweep(rfim_t *h, int64_t n, int exchange_every);

/* Energies E[R] by temperature slot (ascending T), reduced on the device
 * from the current state.  Synchronizes. */
int rfim_energies(rfim_t *h, double *E);

/*
 * Adaptive temperatures (Sec. 4).  For each of `trials` trial runs: zero the
 * exchange counters, run sweeps_per_trial sweeps with exchange every
 * exchange_every (> 0) continuing the chain, compute each pair's rate
 * acc/att, and insert at most max_insert_per_trial new temperatures at the
 * midpoints (T_p + T_{p+1})/2 of the lowest-rate intervals (ties to the lower
 * slot) whose rate is below rate_threshold, while R stays <= R_cap.  A new
 * replica starts as a copy of the replica at the colder end p and gets the
 * next replica id.  Counters are zeroed after each insertion.
 * R_cap must not exceed the capacity given at creation.  Returns the new R
 * (>= 1) or a negative status.  Synchronizes.
 */
int rfim_adapt_temps(rfim_t *h, int trials, int64_t sweeps_per_trial,
                     int exchange_every, double rate_threshold,
                     int max_insert_per_trial, int R_cap);

/* Release the handle and its device memory.  NULL-safe.  Synchronizes. */
void rfim_destroy(rfim_t *h);

/* Thread-local message for the last failure on this thread. */
const char *rfim_last_error(void);

/* ---- additions: streams, observables, state, checkpoint ---- */

/* Issue future work on hip_stream (a hipStream_t owned by the caller, or
 * NULL for the handle's own stream).  Orders itself after pending work. */
int rfim_set_stream(rfim_t *h, void *hip_stream);
/* Block until the handle's pending work is done; RFIM_EDEVICE on fault. */
int rfim_synchronize(rfim_t *h);

int rfim_num_replicas(const rfim_t *h);
int rfim_lattice_size(const rfim_t *h);
int rfim_field_kind(const rfim_t *h);
/* Temperatures [R] by slot, ascending. */
int rfim_temps(const rfim_t *h, double *T);
/* Magnetisations M[R] = sum_i s_i by slot.  Synchronizes. */
int rfim_magnetizations(rfim_t *h, int64_t *M);
/* Energy pieces by replica id: bond sum B[R], field sum F[R] (FP64; exact
 * integers for +-1 fields), magnetisation M[R].  Synchronizes. */
int rfim_components(rfim_t *h, int64_t *B, double *F, int64_t *M);
/* Spins [R][L^3] (+-1, natural site order) by replica id.  Synchronizes. */
int rfim_get_spins(rfim_t *h, int8_t *s);
int rfim_set_spins(rfim_t *h, const int8_t *s);
/* Slot -> replica permutation t2r[R]. */
int rfim_get_perm(rfim_t *h, int32_t *t2r);
int rfim_set_perm(rfim_t *h, const int32_t *t2r);
/* Global sweep counter t and exchange counter k. */
int rfim_get_counters(rfim_t *h, uint64_t *t, uint64_t *k);
int rfim_set_counters(rfim_t *h, uint64_t t, uint64_t k);
/* Exchange attempts/acceptances per lower slot p, arrays of R-1. */
int rfim_exchange_stats(rfim_t *h, uint64_t *att, uint64_t *acc);
int rfim_reset_exchange_stats(rfim_t *h);

/* Measurements (Sec. 7): after every exchange step the energy E and
 * magnetisation M of the replica at each temperature slot are added to
 * per-slot sums.  obs = host [R][6]: count, sum E, sum E^2, sum |M|,
 * sum M^2, sum M^4 (FP64).  Reset at creation, by rfim_reset_observables
 * and by every insertion of rfim_adapt_temps (the slots change).
 * Synchronizes. */
int rfim_observables(rfim_t *h, double *obs);
int rfim_reset_observables(rfim_t *h);

/* Optional measurement for the correlation length (Sec. 7): with
 * RFIM_MEASURE_FOURIER set, every exchange step also adds, per slot,
 *   F = (1/(3N)) sum_mu [(sum_i s_i cos(K x_mu,i))^2 + (sum_i s_i sin(K x_mu,i))^2]
 * of the configuration now at that slot (K = 2 pi / L, mu over the three
 * axes; the printed formula's field h_i read as the spin s_i).  Costs two
 * small launches per exchange step and reads every spin once.  flags = 0
 * turns it off.  The first call with the flag allocates R_cap * L * 2L * 4
 * + (2L + 2 R_cap) * 8 bytes of device memory (RFIM_ENOMEM if that fails).
 * Works for standalone handles and for batch and pool items (their
 * batch's exchange steps measure them).  RFIM_EINVAL for unknown flags. */
#define RFIM_MEASURE_FOURIER 1
int rfim_set_measure(rfim_t *h, int flags);
/* fourier = host [R][2]: per slot, the number of samples and the sum of F
 * (FP64).  Reset with the other observables.  Synchronizes. */
int rfim_fourier(rfim_t *h, double *fourier);

/* Launch shape of the sweep kernels (no effect on results: every shape
 * gives bit-identical chains).  For L = 2^l >= 8: mode 0 streams every
 * half-sweep through HBM with nw in {1, 2, 4, 8} dwords (4 sites each, at
 * most one row: 4 nw <= L/2) per thread and wg in {64, 128, 256} threads
 * per workgroup; mode 1 (L <= 32, nw <= 4)
 * keeps each replica in one workgroup's LDS (wg in {64, ..., 1024}) for all
 * sweeps of an exchange interval.  Modes 2..4 (L = 16 or 32, standalone
 * handles only) cut each replica along z into nw in {2, 4, 8} slabs, one
 * workgroup each (wg in {128, ..., 1024}), so that few replicas still
 * cover every CU: a launch runs up to mode - 1 sweeps in LDS on the slab
 * and 2 (mode - 1) halo planes per side, recomputing the halo instead of
 * waiting for the neighbouring workgroups; the slab must be at least two
 * planes thick, the box (slab plus halos) at most L planes and 64 KB, and
 * the box at most 2 wg work items of 8 sites.  The first slab shape set on
 * a handle allocates a second spin buffer of R_cap * L^3 bytes
 * (RFIM_ENOMEM if that fails).  Other L have the single shape (0, 0, 0).
 * A new handle starts from a shape chosen by L from measurements on gfx950
 * (rfim_get_launch_shape reports it): (1, 1, 64), (1, 2, 256), (1, 4, 1024)
 * at L = 8, 16, 32, (0, 4, 128) above; a standalone handle with continuous
 * fields at L = 32 and R_cap <= 64 starts on the slab shape (3, 4, 1024)
 * when its second spin buffer can be allocated.
 * RFIM_EINVAL for a shape not valid for the handle's L. */
int rfim_set_launch_shape(rfim_t *h, int mode, int nw, int wg);
int rfim_get_launch_shape(const rfim_t *h, int *mode, int *nw, int *wg);

/* Streams a streaming-mode half-sweep runs on (no effect on results).
 * Replicas do not interact between exchange steps, so the library can run
 * the half-sweeps of replicas [0, R/2) on the handle stream and those of
 * [R/2, R) on a second stream (the library's, one per device and handle
 * stream, on a hardware queue of its own), forked from and joined back into
 * the handle stream by events around every exchange interval; the two launch
 * sequences then fill each other's start-up and drain time.  streams = 0:
 * automatic (two streams when each half holds at least 2^22 sites of one
 * colour, 2^23 for the bit sweep with +-1 fields), 1: always one stream, 2:
 * two streams whenever R >= 2.  Only streaming shapes (mode 0, power-of-two
 * L) and bit storage are affected.  RFIM_EINVAL for other values. */
int rfim_set_concurrency(rfim_t *h, int streams);
int rfim_get_concurrency(const rfim_t *h);

/*
 * Update order of the sweeps.  RFIM_ORDER_CHECKERBOARD (default): the plain
 * two-colour checkerboard, sites with (x+y+z) mod 2 = 0 then the others
 * (Sec. 3.2, Eq. 3), independent of launch shapes.  RFIM_ORDER_TILES: the
 * double checkerboard with multi-hit updates (Sec. 3.2; the mh runs of
 * Sec. 5.2): the lattice is cut into tiles of tx * ty * tz sites whose
 * coarse colour is (x/tx + y/ty + z/tz) mod 2; each sweep visits the tiles
 * of coarse colour 0, then those of colour 1, and each visit runs `hits`
 * local sweeps of the tile (its colour-0 sites, then its colour-1 sites)
 * while every site outside it stays as it is.  Hit m of sweep t draws the
 * sweep words of plain sweep t*hits + m (tag 2, ctr = (j >> 2,
 * 2(t*hits + m) + c, r)), so with hits = 1 only the order differs from the
 * plain sweep.  The chain then depends on the tile shape.
 *   Valid for power-of-two L >= 16: tx a multiple of 8; tx, ty, tz each
 *   dividing L into an even number of tiles; (tx/8)*ty*tz a multiple of 64
 *   in [64, 1024]; 1 <= hits <= 65536.  Sweeps need
 *   (sweep counter + n) * hits <= 2^31 (RFIM_ECAP otherwise).
 * Energies, exchanges and adaptive insertion are unchanged.  The order is
 * not part of a checkpoint (set it again after rfim_load).  RFIM_ESTATE for
 * batch and pool items (they sweep in the plain order).  Synchronizes.
 */
/*
 * Spin storage.  RFIM_SPINS_BYTES: one byte per spin.  RFIM_SPINS_BITS:
 * one bit per spin (multi-spin coding): per replica and colour, N/64 words
 * of 32 same-colour sites; the sweep forms neighbour counts with a
 * bit-sliced adder and takes the same decisions with the same random words,
 * so the chain is unchanged, with 1/8 of the bytes per spin-flip attempt.
 * Bits are valid for L = 64, 128 or 256 in the plain checkerboard order
 * without the Fourier measurement (RFIM_EINVAL / RFIM_ESTATE otherwise,
 * RFIM_ENOMEM if the bit arrays, R_cap * L^3 / 8 bytes plus L^3 / 8 for
 * +-1 fields or 4 L^3 for continuous fields (a copy of the fields in the
 * bit sweep's order), allocated on first use, cannot be had).  A handle
 * made by rfim_create / rfim_create_ex / rfim_load at L = 64..256 starts
 * in bits, every other handle in bytes; rfim_set_launch_shape (its
 * shapes are the byte kernels'), rfim_set_measure with the Fourier flag and
 * rfim_set_update_order with tiles switch a handle to bytes.  Calls that
 * read or write spins (energies, spins, checkpoints, adaptive insertion)
 * work in either storage.  RFIM_ESTATE for batch and pool items (bytes).
 * Asynchronous on the handle's stream.
 */
enum { RFIM_SPINS_BYTES = 0, RFIM_SPINS_BITS = 1 };
int rfim_set_spin_storage(rfim_t *h, int storage);
/* RFIM_SPINS_BYTES or RFIM_SPINS_BITS. */
int rfim_get_spin_storage(const rfim_t *h);

enum { RFIM_ORDER_CHECKERBOARD = 0, RFIM_ORDER_TILES = 1 };
int rfim_set_update_order(rfim_t *h, int order, int tx, int ty, int tz, int hits);
/* The current order; tx = ty = tz = 0 and hits = 1 for the plain order. */
int rfim_get_update_order(const rfim_t *h, int *order, int *tx, int *ty, int *tz, int *hits);

/* Checkpoint: the whole chain state (parameters, fields, temperatures,
 * spins, permutation, counters, exchange statistics) as a byte blob.
 * rfim_save with buf == NULL stores the needed size in *len.  A handle
 * restored with rfim_load continues the chain bit for bit. */
int rfim_save(rfim_t *h, void *buf, size_t *len);
rfim_t *rfim_load(const void *buf, size_t len, void *hip_stream);

/* ---- batches: many independent realizations per launch ------------- */

/*
 * A batch advances n independent realizations together (realization-level
 * parallelism, the natural choice the paper sets aside for single large
 * lattices in Sec. 8).  Every item must have L a power of two >= 8; items
 * may differ in L, R, J, h, field kind, seed and realization id.  Items that
 * share (L, field kind) form a class whose sweeps run in one launch (one per
 * half-sweep when streaming, one per exchange interval when LDS-resident);
 * one launch runs the exchange steps of all items; a full exchange interval
 * is captured once as a HIP graph and replayed.  Each item's chain is
 * bit-identical to the same realization run alone with rfim_create_ex.
 *   items      host [n] parameter blocks (copied); n in [1, 65536].
 *   hip_stream caller's hipStream_t or NULL (the batch creates its own).
 * Returns NULL on failure.
 */
typedef struct rfim_batch rfim_batch_t;
rfim_batch_t *rfim_batch_create(int n, const rfim_params_t *items, void *hip_stream);
void rfim_batch_destroy(rfim_batch_t *b);
int rfim_batch_size(const rfim_batch_t *b);
/* All items advance n sweeps with exchange every exchange_every sweeps (of
 * the batch's common sweep counter).  Asynchronous. */
int rfim_batch_sweep(rfim_batch_t *b, int64_t n, int exchange_every);
int rfim_batch_synchronize(rfim_batch_t *b);
/* Borrowed handle of item i for the observables and state calls (energies,
 * spins, permutation, counters, statistics, save).  Owned by the batch:
 * rfim_destroy ignores it; rfim_sweep, rfim_adapt_temps, rfim_set_counters
 * and rfim_set_launch_shape on it return RFIM_ESTATE. */
rfim_t *rfim_batch_item(rfim_batch_t *b, int i);
/* Launch shape of the class (L, field_kind) (see rfim_set_launch_shape;
 * modes 0 and 1), or RFIM_MODE_BITS: shape (RFIM_MODE_BITS, 0, 0) at L = 64,
 * 128 or 256 keeps the class's items in one bit per spin (see
 * rfim_set_spin_storage), each item swept on its own, all sweeps of an
 * exchange interval before the next item of its stream (two streams from
 * 2^23 sites of one colour per half, split by items or, for one item, by
 * replicas); a byte shape takes them back to bytes.  Items in bit storage
 * refuse the Fourier measurement and a storage switch of their own
 * (RFIM_ESTATE).  Used by the autotuner.  No effect on results.  Classes
 * at L = 64, 128 and 256 start in bit storage (in bytes if its arrays
 * cannot be had), the others on the default launch shape of a single
 * realization.  RFIM_EINVAL for slab or invalid shapes; RFIM_ENOMEM if bit
 * arrays cannot be had (the class keeps its shape).  Synchronizes. */
enum { RFIM_MODE_BITS = 5 };
int rfim_batch_set_shape(rfim_batch_t *b, int L, int field_kind, int mode, int nw, int wg);
/* Temporal blocking of large streaming classes (an optimisation of the
 * realization-level parallelism of Sec. 8; no effect on results).  A
 * streaming class holding more than 2 * bytes of spins runs as two lanes on
 * two streams, each a sequence of groups of consecutive items with at most
 * `bytes` of spins (at least one item each), and a group runs all sweeps of
 * an exchange interval before the next group of its lane, so that the
 * groups in flight stay in the on-package cache instead of the whole class
 * streaming through HBM once per half-sweep.  Default 96 MiB (two groups
 * in flight within the 256 MB cache); 0 turns it off (one or two lanes
 * over the whole class, every half-sweep over all its items).  RFIM_EINVAL
 * for 0 < bytes < 1 MiB.  Synchronizes.  Pools (below) use the default. */
int rfim_batch_set_group_bytes(rfim_batch_t *b, int64_t bytes);
int64_t rfim_batch_get_group_bytes(const rfim_batch_t *b);

/* ---- pools: continuous batching for serving ------------------------- */

/*
 * A pool is a batch whose membership changes while it runs.  Realizations
 * are admitted against a device-memory budget (each reserves what its
 * parameters need at R_cap), advance together in quanta of whole exchange
 * intervals (each keeps its own sweep and exchange counters; an admitted
 * realization starts at t = 0), may run one adaptive insertion step in
 * place between quanta, and are released when done.  A realization's
 * chain is the same as run alone with rfim_create_ex + rfim_adapt_temps +
 * rfim_sweep on the same schedule.  Items need L a power of two >= 8.
 */
typedef struct rfim_pool rfim_pool_t;
rfim_pool_t *rfim_pool_create(size_t hbm_budget_bytes, void *hip_stream);
void rfim_pool_destroy(rfim_pool_t *p);
/* Device bytes a realization with these parameters reserves (0 if the
 * parameters are invalid): its buffers at R_cap and, at L = 64, 128 or 256,
 * the bit arrays a class in bit storage adds (R_cap L^3 / 8 bytes plus
 * L^3 / 8 for +-1 fields or 4 L^3 for continuous fields), whatever the
 * class shape. */
size_t rfim_pool_bytes_needed(const rfim_params_t *params);
/* Admit: a slot id >= 0, RFIM_EBUSY if the budget cannot hold it now (try
 * again after a release), or another negative status.  The slot has no
 * schedule: the caller advances it with rfim_pool_step, runs its insertion
 * steps with rfim_pool_adapt and decides when it is done. */
int rfim_pool_admit(rfim_pool_t *p, const rfim_params_t *params);

/* A realization request with the adaptive schedule of Sec. 4 and the
 * realization-level parallelism of Sec. 8: `trials` trial runs of
 * sweeps_per_trial sweeps, each followed by one insertion step (rates below
 * rate_threshold, at most max_insert_per_trial new temperatures, R bounded
 * by params.R_cap; see rfim_adapt_temps), then production_sweeps sweeps.
 * The exchange interval is the one rfim_pool_step is called with. */
typedef struct rfim_job {
    rfim_params_t params;
    int trials;                 /* >= 0 */
    int64_t sweeps_per_trial;   /* >= 1 when trials > 0 */
    double rate_threshold;
    int max_insert_per_trial;   /* >= 0 */
    int64_t production_sweeps;  /* >= 1 */
} rfim_job_t;
/* Admit a job: as rfim_pool_admit, but the pool runs the schedule itself:
 * every rfim_pool_step advances the slot, runs its insertion step when a
 * trial run ends, and marks it finished when its production sweeps are
 * done; a finished slot is no longer stepped and is reported by
 * rfim_pool_poll until released.  RFIM_EINVAL for a schedule with a
 * negative count, an empty trial run or no production sweeps, RFIM_ECAP
 * if its sweeps pass 2^31 - 1. */
int rfim_pool_admit_job(rfim_pool_t *p, const rfim_job_t *job);

/* Every slot that is admitted and not finished advances `quantum` sweeps
 * (a multiple of exchange_every; every slot must be at an exchange
 * boundary; for a job, its next schedule boundary must lie a multiple of
 * `quantum` sweeps ahead, else RFIM_EINVAL before any work).  Asynchronous,
 * except that it synchronizes when a job's trial run ends (the insertion
 * step reads the exchange counters). */
int rfim_pool_step(rfim_pool_t *p, int quantum, int exchange_every);

/* Finished jobs not yet released: writes up to `max` slot ids (ascending)
 * into done[] and returns how many it wrote; with max = 0 (done may be
 * NULL) returns how many there are.  Host-side state only; no device
 * work. */
int rfim_pool_poll(rfim_pool_t *p, int *done, int max);

/* The state of a slot (finished or not).  The caller sets `capacity` and
 * the array pointers (each may be NULL to skip it); the library fills R,
 * the arrays by temperature slot (ascending T), the slot's sweep and
 * exchange counters, the spin-flip attempts issued for it and whether its
 * schedule is complete.  RFIM_ECAP if an array is given and capacity < R
 * (R is still written).  Synchronizes. */
typedef struct rfim_result {
    int R;                      /* out */
    int capacity;               /* in: entries each non-NULL array holds */
    double *temps;              /* out [R] */
    double *energies;           /* out [R], E of the replica at each slot */
    int64_t *magnetizations;    /* out [R] */
    int32_t *perm;              /* out [R], slot -> replica id */
    uint64_t sweeps, exchanges; /* out: counters t and k of the slot */
    uint64_t attempts;          /* out: R * L^3 per sweep, summed */
    int finished;               /* out: 1 once its schedule is complete */
} rfim_result_t;
int rfim_pool_result(rfim_pool_t *p, int slot, rfim_result_t *res);

/* One adaptive insertion step (Sec. 4) for a slot from the exchange
 * counters it accumulated since its last reset (admission or previous
 * step); see rfim_adapt_temps.  Synchronizes; returns the new R.
 * RFIM_ESTATE for a job's slot (the pool runs its insertions). */
int rfim_pool_adapt(rfim_pool_t *p, int slot, double rate_threshold, int max_insert, int R_cap);
/* Release a slot (finished or not) and its device memory.  Synchronizes. */
int rfim_pool_release(rfim_pool_t *p, int slot);
/* Borrowed handle of a slot for observables and state (see
 * rfim_batch_item). */
rfim_t *rfim_pool_item(rfim_pool_t *p, int slot);
/* Slots admitted and not released (finished jobs included). */
int rfim_pool_active(const rfim_pool_t *p);
size_t rfim_pool_reserved(const rfim_pool_t *p);
/* Shape of the class (L, field_kind) for items admitted from now on and,
 * at the next step, for the items already there (see rfim_batch_set_shape,
 * RFIM_MODE_BITS included; the same defaults).  Synchronizes. */
int rfim_pool_set_shape(rfim_pool_t *p, int L, int field_kind, int mode, int nw, int wg);
int rfim_pool_synchronize(rfim_pool_t *p);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * per-replica energies E_r = -J B_r - h F_r of rfim_energies, computed from
 * spin configurations and fields that the caller keeps on the device, with
 * nothing allocated and nothing synchronized.
 *   L           even, 2 <= L <= 1024.
 *   R           1 <= R <= RFIM_NOALLOC_MAX_PARTIALS (2^18).
 *   J, h        finite.
 *   d_spins     device [R][L^3] int8, each +1 or -1, natural site order
 *               i = x + L*(y + L*z) (the layout rfim_get_spins returns).
 *   d_fields    device [L^3] float, natural site order.
 *   d_E         device [R] double, written: E of configuration r.
 *   hip_stream  hipStream_t of the current device (NULL: its null stream);
 *               the work is queued there and the call returns at once.
 * B counts each bond once (forward partners along x, y, z, periodic), as in
 * rfim_energies; +-1 fields give the same values bit for bit, other fields
 * agree to FP64 rounding (another summation order).  The partial sums live
 * in a fixed 4 MiB device array of the library that every GPU it runs on
 * holds until the process ends; it is shared by every call on that GPU, so
 * calls that overlap on one GPU (two streams, two threads) race and must be
 * ordered by the caller.  Errors: RFIM_EINVAL (bad argument), RFIM_ECAP
 * (R too large), RFIM_EDEVICE (launch failure), all before any work is
 * queued.
 */
#define RFIM_NOALLOC_MAX_PARTIALS (1 << 18)
int rfim_energies_noalloc(int L, int R, double J, double h, const int8_t *d_spins, const float *d_fields,
                          double *d_E, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
