// Host runtime and C ABI of librfim.so (see include/rfim.h).  Validates
// arguments, owns device memory and the stream, builds the acceptance
// tables, sequences the sweep / energy / exchange kernels, and runs the
// adaptive temperature insertion of Sec. 4 between trial runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "rfim.h"
#include "rfim_internal.h"

using rfim_dev::Lattice;

namespace {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(RFIM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

constexpr int kMaxR = 65536;
constexpr uint64_t kMaxSweeps = 0x7FFFFFFFull;

// A stream for concurrent lanes of work.  It is created with a CU mask that
// enables every CU of the device: the runtime gives such a stream a hardware
// queue of its own instead of one shared round-robin from its pool of
// GPU_MAX_HW_QUEUES queues, so two lanes cannot end up serialized on one
// queue by the order in which the process happened to create its streams.
// Falls back to an ordinary non-blocking stream.
hipError_t create_lane_stream(hipStream_t *s) {
    *s = nullptr;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && ncu > 0) {
        std::vector<uint32_t> mask((size_t)(ncu + 31) / 32, 0u);
        for (int c = 0; c < ncu; ++c) mask[(size_t)c >> 5] |= 1u << (c & 31);
        e = hipExtStreamCreateWithCUMask(s, (uint32_t)mask.size(), mask.data());
        if (e == hipSuccess) return e;
    }
    (void)hipGetLastError();
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

// The second stream of the two-stream sweeps, one per (device, handle
// stream) and shared by every handle issuing on that stream, reference
// counted.  Each call forks from and joins back into its handle stream, so
// handles sharing a stream also share its order on the second stream.  A
// second stream that no handle holds any more stays alive and is bound to
// the next handle stream on its device that needs one: a loop that creates
// and destroys handles one at a time then reuses one hardware queue instead
// of setting up a new one per handle.  Their number is the largest number
// of handle streams in use at once on a device.
struct SideStream {
    hipStream_t main;
    int device;
    hipStream_t side;
    int refs;
};
std::mutex g_side_mu;
std::vector<SideStream> g_side;

hipError_t acquire_side_stream(hipStream_t main, hipStream_t *side) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_side_mu);
    SideStream *idle = nullptr;
    for (auto &s : g_side) {
        if (s.device != dev) continue;
        if (s.main == main && s.refs > 0) {
            ++s.refs;
            *side = s.side;
            return hipSuccess;
        }
        if (s.refs == 0 && (!idle || s.main == main)) idle = &s;
    }
    if (idle) {
        idle->main = main;
        idle->refs = 1;
        *side = idle->side;
        return hipSuccess;
    }
    hipStream_t q = nullptr;
    if ((e = create_lane_stream(&q)) != hipSuccess) return e;
    g_side.push_back({main, dev, q, 1});
    *side = q;
    return hipSuccess;
}

// Drops one reference; the stream itself stays for reuse (every call that
// forked work onto it has joined it back into its handle stream, which the
// handle synchronizes before it lets go).
void release_side_stream(hipStream_t side) {
    if (!side) return;
    std::lock_guard<std::mutex> lock(g_side_mu);
    for (auto &s : g_side)
        if (s.side == side) {
            if (s.refs > 0) --s.refs;
            return;
        }
}

}  // namespace

namespace rfim_host {

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

}  // namespace rfim_host

struct rfim {
    // parameters
    int L = 0, N = 0, half = 0, R = 0, R_cap = 0, log2L = -1, kind = 0;
    double J = 0, h = 0;
    uint64_t seed = 0;
    uint32_t rho = 0;
    std::vector<float> fields;      // natural order, as given
    std::vector<double> T;          // by slot
    // host mirrors of the device counters
    uint64_t t = 0, k = 0;
    // stream; a second stream takes half of the replicas of large streaming
    // sweeps (fork and join through events on the handle stream).  The
    // second stream is shared by every handle that issues on the same
    // stream (see acquire_side_stream).
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t aux = nullptr;
    hipStream_t aux_for = nullptr;  // the handle stream `aux` was acquired for
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int concurrency = 0;            // see rfim_set_concurrency
    // update order: 0 plain checkerboard, 1 double checkerboard of tiles
    // with multi-hit updates (rfim_set_update_order)
    int order = 0;
    rfim_dev::TileShape tiles = {0, 0, 0, 1};
    // spin storage: bytes in d_spins, or one bit per spin in d_bits
    // (rfim_set_spin_storage; the byte array is then a mirror brought up to
    // date before any call that reads it)
    bool bits_mode = false;
    uint32_t *d_bits = nullptr, *d_fbw = nullptr;
    float *d_fhw = nullptr;          // continuous fields in the bit sweep's order
    // slab shapes (mode >= 2) read one spin buffer and write the other;
    // d_spins is always the current one, d_spins_alt the other, and
    // d_spins_own the second buffer as allocated (freed with the handle)
    uint8_t *d_spins_alt = nullptr, *d_spins_own = nullptr;
    rfim_alloc_t alloc = {nullptr, nullptr, nullptr};   // device memory provider (rfim_create_ex)
    // optional Fourier measurement (rfim_set_measure)
    int measure = 0;
    int32_t *d_fpart = nullptr;
    double *d_trig = nullptr, *d_fobs = nullptr;
    // device memory: one allocation (d_arena, see arena_layout) carved into
    // the buffers below; the measurement buffers are allocated on demand
    void *d_arena = nullptr;
    uint8_t *d_spins = nullptr, *d_fbits = nullptr;
    float *d_fhf = nullptr, *d_fraw = nullptr, *d_betaf = nullptr;
    uint32_t *d_thr = nullptr;
    double *d_beta = nullptr, *d_part = nullptr, *d_E = nullptr, *d_Mr = nullptr, *d_obs = nullptr;
    int32_t *d_t2r = nullptr, *d_r2t = nullptr;
    uint64_t *d_att = nullptr, *d_acc = nullptr, *d_ctrs = nullptr;
    int64_t *d_B = nullptr, *d_M = nullptr;
    double *d_F = nullptr;
    int nblk = 1;
    int mode = 0, nw = 0, wg = 0;   // launch shape (see rfim_set_launch_shape)
    // device copy of lattice() and the workgroup maps of the sweep launches
    Lattice lat_host;
    Lattice *d_lat = nullptr;
    uint2 *d_smap = nullptr, *d_rmap = nullptr;
    size_t smap_cap = 0;
    int smap_n = 0;
    bool in_batch = false;          // owned by a batch: no standalone launches

    Lattice lattice() const {
        Lattice a;
        a.L = L;
        a.N = N;
        a.half = half;
        a.R = R;
        a.log2L = log2L;
        a.kind = kind;
        a.Jf = (float)J;
        a.J = J;
        a.h = h;
        a.key0 = (uint32_t)seed;
        a.key1 = (uint32_t)(seed >> 32);
        a.rho = rho;
        a.spins = d_spins;
        a.fbits = d_fbits;
        a.fhf = d_fhf;
        a.fraw = d_fraw;
        a.thr = d_thr;
        a.betaf = d_betaf;
        a.beta = d_beta;
        a.t2r = d_t2r;
        a.r2t = d_r2t;
        a.att = d_att;
        a.acc = d_acc;
        a.ctrs = d_ctrs;
        a.part = d_part;
        a.pstride = R_cap;
        a.nblk = nblk;
        a.mode = mode;
        a.nw = nw;
        a.wg = wg;
        a.E = d_E;
        a.Mr = d_Mr;
        a.obs = d_obs;
        a.bits = bits_mode ? d_bits : nullptr;
        a.fbw = d_fbw;
        a.fhw = d_fhw;
        return a;
    }
};

namespace {

// The handle's own device memory, from its provider or hipMalloc.
int dev_alloc(rfim *h, void **p, size_t bytes) {
    *p = nullptr;
    if (h->alloc.alloc) {
        *p = h->alloc.alloc(bytes, h->alloc.ctx);
        if (!*p) return fail(RFIM_ENOMEM, "device memory provider returned NULL for %zu bytes", bytes);
        return RFIM_OK;
    }
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RFIM_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    return RFIM_OK;
}

void dev_free(rfim *h, void *p) {
    if (!p) return;
    if (h->alloc.free)
        h->alloc.free(p, h->alloc.ctx);
    else
        (void)hipFree(p);
}

void free_device(rfim *h) {
    dev_free(h, h->d_arena);
    dev_free(h, h->d_fpart);
    dev_free(h, h->d_trig);
    dev_free(h, h->d_fobs);
    dev_free(h, (void *)h->d_bits);
    dev_free(h, (void *)h->d_fbw);
    dev_free(h, (void *)h->d_fhw);
    dev_free(h, (void *)h->d_spins_own);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    release_side_stream(h->aux);
    h->aux = nullptr;
    h->aux_for = nullptr;
}

int validate(const rfim_params_t *p, int *kind_out) {
    if (!p) return fail(RFIM_EINVAL, "params is NULL");
    if (p->L < 2 || p->L > 1024 || (p->L & 1))
        return fail(RFIM_EINVAL, "L must be even with 2 <= L <= 1024 (got %d)", p->L);
    const int R_cap = p->R_cap == 0 ? p->R : p->R_cap;
    if (p->R < 1 || p->R > kMaxR) return fail(RFIM_EINVAL, "R must be in [1, %d] (got %d)", kMaxR, p->R);
    if (R_cap < p->R || R_cap > kMaxR)
        return fail(RFIM_EINVAL, "R_cap must be in [R, %d] (got %d)", kMaxR, R_cap);
    if (!p->fields || !p->temps) return fail(RFIM_EINVAL, "fields and temps must not be NULL");
    if (!std::isfinite(p->J) || !std::isfinite(p->h)) return fail(RFIM_EINVAL, "J and h must be finite");
    if (p->realization >= (1u << 28)) return fail(RFIM_EINVAL, "realization id must be < 2^28");
    for (int t = 0; t < p->R; ++t) {
        if (!std::isfinite(p->temps[t]) || !(p->temps[t] > 0.0))
            return fail(RFIM_EINVAL, "temps must be finite and > 0 (temps[%d])", t);
        if (t > 0 && !(p->temps[t] > p->temps[t - 1]))
            return fail(RFIM_EINVAL, "temps must be strictly ascending (temps[%d])", t);
    }
    const size_t N = (size_t)p->L * p->L * p->L;
    bool bimodal = true;
    for (size_t i = 0; i < N; ++i) {
        const float f = p->fields[i];
        if (!std::isfinite(f)) return fail(RFIM_EINVAL, "fields must be finite (fields[%zu])", i);
        if (f != 1.0f && f != -1.0f) bimodal = false;
    }
    int kind;
    if (p->field_kind == RFIM_FIELDS_AUTO) kind = bimodal ? 0 : 1;
    else if (p->field_kind == RFIM_FIELDS_BIMODAL || p->field_kind == RFIM_FIELDS_CONTINUOUS) kind = p->field_kind;
    else return fail(RFIM_EINVAL, "field_kind must be -1, 0 or 1");
    if (kind == 0 && !bimodal) return fail(RFIM_EINVAL, "bimodal field kind needs every field = +-1");
    *kind_out = kind;
    return RFIM_OK;
}

// Metropolis thresholds for +-1 fields.  The device indexes them by
// idx = (up << 2) | (b << 1) | f: up = number of +1 neighbours (0..6),
// b = 1 iff s_i = +1, f = 1 iff h_i = +1.  With s = 2b-1, the flip costs
// dE = 2(J a + h c), a = s (2 up - 6) = s_i n_i, c = s (2f - 1) = s_i h_i.
// FP64 on the host: thr = floor(exp(-beta dE) 2^32) clamped to 2^32 - 1;
// entries with dE <= 0 are always accepted.
double index_delta(const rfim *h, int idx) {
    const int up = idx >> 2, b = (idx >> 1) & 1, f = idx & 1;
    const int s = 2 * b - 1;
    const int a = s * (2 * up - 6);
    const int c = s * (2 * f - 1);
    return 2.0 * (h->J * (double)a + h->h * (double)c);
}

int upload_tables(rfim *h) {
    std::vector<uint32_t> thr((size_t)h->R * 32, 0u);
    std::vector<double> beta(h->R);
    std::vector<float> betaf(h->R);
    // Accept iff dE <= 0 or u32 < floor(e^(-beta dE) 2^32) (clamped to
    // 2^32 - 1), stored as "u32 <= entry": the bound minus one, all ones
    // where dE <= 0, and a never bit in entry 31 where the bound is 0.
    for (int t = 0; t < h->R; ++t) {
        beta[t] = 1.0 / h->T[t];
        betaf[t] = (float)beta[t];
        uint32_t never = 0;
        for (int idx = 0; idx < 28; ++idx) {
            uint32_t &e = thr[(size_t)t * 32 + idx];
            const double dE = index_delta(h, idx);
            if (dE <= 0.0) {
                e = 0xFFFFFFFFu;
                continue;
            }
            const double scaled = std::ldexp(std::exp(-(beta[t] * dE)), 32);
            const uint32_t bound = scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)std::floor(scaled);
            if (bound == 0) {
                never |= 1u << idx;
                e = 0;
            } else {
                e = bound - 1u;
            }
        }
        thr[(size_t)t * 32 + 31] = never;
    }
    HIPCHK(hipMemcpyAsync(h->d_thr, thr.data(), thr.size() * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_beta, beta.data(), beta.size() * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_betaf, betaf.data(), betaf.size() * 4, hipMemcpyHostToDevice, h->stream));
    // pageable sources: make sure the copies are consumed before the vectors die
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

// Natural site order <-> colour-split layout (index only, no arithmetic of
// the method): site i of colour c goes to [c][i >> 1].
template <class F>
void for_each_site(int L, F f) {
    const size_t N = (size_t)L * L * L;
    for (size_t i = 0; i < N; ++i) {
        const int x = (int)(i % L), y = (int)((i / L) % L), z = (int)(i / ((size_t)L * L));
        f(i, (x + y + z) & 1, i >> 1);
    }
}

// A handle's device buffers live in one allocation, in this order, each
// piece on a 256-byte boundary (byte offsets; absent pieces have size 0).
struct ArenaLayout {
    size_t spins, fbits, fhf, fraw, thr, betaf, beta, t2r, r2t, att, acc, ctrs, part, E, Mr, obs, B, M, F,
        lat, rmap, smap, total;
    size_t smap_cap;   // streaming workgroup-map entries (0 for other L)
};

ArenaLayout arena_layout(int L, int R_cap, int kind) {
    const size_t N = (size_t)L * L * L, Rc = (size_t)R_cap;
    const bool pow2 = L >= 8 && (L & (L - 1)) == 0;
    // partials sized for the shape with the most workgroups per replica,
    // maps for the streaming shape with the most workgroups per replica
    size_t maxblk = 64, maxw = 1;
    if (pow2)
        for (int nw : {1, 2, 4, 8})
            for (int wg : {64, 128, 256})
                if (rfim_dev::shape_valid(L, 0, nw, wg)) {
                    maxblk = std::max(maxblk, (size_t)rfim_dev::blocks_per_replica(L, 0, nw, wg));
                    maxw = std::max(maxw, (size_t)rfim_dev::stream_blocks_per_replica(L, nw, wg));
                }
    ArenaLayout a{};
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    a.spins = take(Rc * N);
    a.fbits = take(kind == 0 ? N : 0);
    a.fhf = take(kind == 0 ? 0 : N * sizeof(float));
    a.fraw = take(kind == 0 ? 0 : N * sizeof(float));
    a.thr = take(Rc * 32 * sizeof(uint32_t));
    a.betaf = take(Rc * sizeof(float));
    a.beta = take(Rc * sizeof(double));
    a.t2r = take(Rc * sizeof(int32_t));
    a.r2t = take(Rc * sizeof(int32_t));
    a.att = take(Rc * sizeof(uint64_t));
    a.acc = take(Rc * sizeof(uint64_t));
    a.ctrs = take(2 * sizeof(uint64_t));
    a.part = take(Rc * maxblk * 3 * sizeof(double));
    a.E = take(Rc * sizeof(double));
    a.Mr = take(Rc * sizeof(double));
    a.obs = take(Rc * 6 * sizeof(double));
    a.B = take(Rc * sizeof(int64_t));
    a.M = take(Rc * sizeof(int64_t));
    a.F = take(Rc * sizeof(double));
    a.lat = take(sizeof(Lattice));
    a.rmap = take(Rc * sizeof(uint2));
    a.smap_cap = pow2 ? Rc * maxw : 0;
    a.smap = take(a.smap_cap * sizeof(uint2));
    a.total = off;
    return a;
}

int alloc_device(rfim *h) {
    h->nblk = rfim_dev::blocks_per_replica(h->L, h->mode, h->nw, h->wg);
    const ArenaLayout a = arena_layout(h->L, h->R_cap, h->kind);
    int rc;
    if ((rc = dev_alloc(h, &h->d_arena, a.total))) return rc;
    char *b = (char *)h->d_arena;
    h->d_spins = (uint8_t *)(b + a.spins);
    if (h->kind == 0) {
        h->d_fbits = (uint8_t *)(b + a.fbits);
    } else {
        h->d_fhf = (float *)(b + a.fhf);
        h->d_fraw = (float *)(b + a.fraw);
    }
    h->d_thr = (uint32_t *)(b + a.thr);
    h->d_betaf = (float *)(b + a.betaf);
    h->d_beta = (double *)(b + a.beta);
    h->d_t2r = (int32_t *)(b + a.t2r);
    h->d_r2t = (int32_t *)(b + a.r2t);
    h->d_att = (uint64_t *)(b + a.att);
    h->d_acc = (uint64_t *)(b + a.acc);
    h->d_ctrs = (uint64_t *)(b + a.ctrs);
    h->d_part = (double *)(b + a.part);
    h->d_E = (double *)(b + a.E);
    h->d_Mr = (double *)(b + a.Mr);
    h->d_obs = (double *)(b + a.obs);
    h->d_B = (int64_t *)(b + a.B);
    h->d_M = (int64_t *)(b + a.M);
    h->d_F = (double *)(b + a.F);
    h->d_lat = (Lattice *)(b + a.lat);
    h->d_rmap = (uint2 *)(b + a.rmap);
    h->smap_cap = a.smap_cap;
    h->d_smap = a.smap_cap ? (uint2 *)(b + a.smap) : nullptr;
    return RFIM_OK;
}

int upload_fields(rfim *h) {
    const size_t N = (size_t)h->N, half = N / 2;
    if (h->kind == 0) {
        std::vector<uint8_t> fb(N);
        for_each_site(h->L, [&](size_t i, int c, size_t j) { fb[c * half + j] = h->fields[i] > 0.0f ? 4 : 0; });
        HIPCHK(hipMemcpyAsync(h->d_fbits, fb.data(), N, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    } else {
        std::vector<float> hf(N), raw(N);
        for_each_site(h->L, [&](size_t i, int c, size_t j) {
            raw[c * half + j] = h->fields[i];
            hf[c * half + j] = (float)(h->h * (double)h->fields[i] - 6.0 * h->J);
        });
        HIPCHK(hipMemcpyAsync(h->d_fhf, hf.data(), N * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d_fraw, raw.data(), N * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return RFIM_OK;
}

int upload_perm(rfim *h, const std::vector<int32_t> &t2r) {
    std::vector<int32_t> r2t(h->R);
    for (int t = 0; t < h->R; ++t) r2t[t2r[t]] = t;
    HIPCHK(hipMemcpyAsync(h->d_t2r, t2r.data(), h->R * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_r2t, r2t.data(), h->R * 4, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int upload_counters(rfim *h) {
    uint64_t c[2] = {h->t, h->k};
    HIPCHK(hipMemcpyAsync(h->d_ctrs, c, sizeof c, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

// Upload the descriptor and rebuild the workgroup maps for the current R
// and launch shape (entries: (0 << 16 | replica, block)).
int sync_descriptor(rfim *h) {
    h->lat_host = h->lattice();
    HIPCHK(hipMemcpyAsync(h->d_lat, &h->lat_host, sizeof(Lattice), hipMemcpyHostToDevice, h->stream));
    std::vector<uint2> rmap(h->R);
    for (int r = 0; r < h->R; ++r) rmap[r] = make_uint2((uint32_t)r, 0u);
    HIPCHK(hipMemcpyAsync(h->d_rmap, rmap.data(), rmap.size() * sizeof(uint2), hipMemcpyHostToDevice, h->stream));
    std::vector<uint2> smap;
    if (h->log2L >= 3 && h->mode == 0) {
        const int wpr = rfim_dev::stream_blocks_per_replica(h->L, h->nw, h->wg);
        smap.resize((size_t)h->R * wpr);
        for (int r = 0; r < h->R; ++r)
            for (int b = 0; b < wpr; ++b) smap[(size_t)r * wpr + b] = make_uint2((uint32_t)r, (uint32_t)b);
        HIPCHK(hipMemcpyAsync(h->d_smap, smap.data(), smap.size() * sizeof(uint2), hipMemcpyHostToDevice, h->stream));
    }
    h->smap_n = (int)smap.size();
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

rfim_dev::Launch single_launch(const rfim *h) {
    rfim_dev::Launch ln;
    ln.single = &h->lat_host;
    ln.lats = h->d_lat;
    ln.map = h->mode == 1 ? h->d_rmap : h->d_smap;
    ln.nblocks = h->mode == 1 ? h->R : h->smap_n;
    ln.L = h->L;
    ln.kind = h->kind;
    ln.mode = h->mode;
    ln.nw = h->nw;
    ln.wg = h->wg;
    return ln;
}

int reset_stats(rfim *h) {
    HIPCHK(hipMemsetAsync(h->d_att, 0, (size_t)h->R_cap * 8, h->stream));
    HIPCHK(hipMemsetAsync(h->d_acc, 0, (size_t)h->R_cap * 8, h->stream));
    return RFIM_OK;
}

int reset_obs(rfim *h) {
    HIPCHK(hipMemsetAsync(h->d_obs, 0, (size_t)h->R_cap * 6 * sizeof(double), h->stream));
    if (h->d_fobs) HIPCHK(hipMemsetAsync(h->d_fobs, 0, (size_t)h->R_cap * 2 * sizeof(double), h->stream));
    return RFIM_OK;
}

// After an exchange step: the Fourier sample of every replica, by slot.
int measure_after_exchange(rfim *h, hipStream_t s) {
    if (!(h->measure & RFIM_MEASURE_FOURIER)) return RFIM_OK;
    HIPCHK(rfim_dev::launch_fourier(h->lattice(), h->d_fpart, h->d_trig, h->d_fobs, s));
    return RFIM_OK;
}

int download_perm(rfim *h, std::vector<int32_t> &t2r) {
    t2r.resize(h->R);
    HIPCHK(hipMemcpyAsync(t2r.data(), h->d_t2r, h->R * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

// Bit storage: bring the byte array up to date before code that reads it,
// and the bits after code that wrote it.
int bytes_from_bits(rfim *h) {
    if (h->bits_mode) HIPCHK(rfim_dev::launch_unpack_bits(h->lattice(), h->stream));
    return RFIM_OK;
}

int bits_from_bytes(rfim *h) {
    if (h->bits_mode) HIPCHK(rfim_dev::launch_pack_bits(h->lattice(), h->stream));
    return RFIM_OK;
}

int compute_components(rfim *h) {
    int rc;
    if ((rc = bytes_from_bits(h))) return rc;
    Lattice lat = h->lattice();
    HIPCHK(rfim_dev::launch_energy(lat, h->stream));
    HIPCHK(rfim_dev::launch_reduce(lat, h->d_B, h->d_F, h->d_M, h->stream));
    return RFIM_OK;
}

// Standalone continuous-field handles at L = 32 with at most this many
// replicas start on a slab shape (rfim_create_ex).
constexpr int kSlabDefaultMaxReplicas = 64;

// Default launch shape: lattices up to L = 32 run LDS-resident (streaming
// is launch-bound there), larger ones stream with four dwords per thread.
// The autotuner in the Python package measures and overrides these.
void default_shape(int L, int R, int *mode, int *nw, int *wg) {
    if (!(L >= 8 && (L & (L - 1)) == 0)) {
        *mode = 0; *nw = 0; *wg = 0;
        return;
    }
    // L <= 32: the LDS-resident shape, one replica per workgroup with one
    // chunk per thread per half-sweep (a whole exchange interval per
    // launch).  Measured on gfx950 at L = 32 against the best streaming
    // shape: +36-42 % (continuous fields, R = 64), +70 % (+-1 fields, R = 32);
    // streaming at L = 32 is launch-bound up to R ~ 128.
    if (L <= 32) {
        *mode = 1;
        *nw = L == 8 ? 1 : (L == 16 ? 2 : 4);
        *wg = L == 8 ? 64 : (L == 16 ? 256 : 1024);
        return;
    }
    // L >= 64: streaming, 4 dwords in 128-thread groups (whole rows of 8
    // dwords are no faster)
    *mode = 0;
    *nw = 4;
    *wg = 128;
    (void)R;
}

rfim *create_impl(const rfim_params_t *p, void *stream, int *err) {
    int kind = 0;
    *err = validate(p, &kind);
    if (*err) return nullptr;
    rfim *h = new (std::nothrow) rfim();
    if (!h) {
        *err = fail(RFIM_ENOMEM, "out of host memory");
        return nullptr;
    }
    h->L = p->L;
    h->N = p->L * p->L * p->L;
    h->half = h->N / 2;
    h->R = p->R;
    h->R_cap = p->R_cap == 0 ? p->R : p->R_cap;
    h->kind = kind;
    h->J = p->J;
    h->h = p->h;
    h->seed = p->seed;
    h->rho = p->realization;
    h->log2L = -1;
    if (p->L >= 8 && (p->L & (p->L - 1)) == 0) {
        int l = 0;
        while ((1 << l) < p->L) ++l;
        h->log2L = l;
    }
    default_shape(h->L, h->R_cap, &h->mode, &h->nw, &h->wg);
    h->fields.assign(p->fields, p->fields + h->N);
    h->T.assign(p->temps, p->temps + p->R);
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            *err = fail(RFIM_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
            delete h;
            return nullptr;
        }
        h->own_stream = true;
    }
    return h;
}

int init_device(rfim *h) {
    int rc;
    if ((rc = alloc_device(h))) return rc;
    if ((rc = upload_fields(h))) return rc;
    if ((rc = upload_tables(h))) return rc;
    std::vector<int32_t> ident(h->R);
    for (int t = 0; t < h->R; ++t) ident[t] = t;
    if ((rc = upload_perm(h, ident))) return rc;
    if ((rc = upload_counters(h))) return rc;
    if ((rc = reset_stats(h))) return rc;
    if ((rc = reset_obs(h))) return rc;
    if ((rc = sync_descriptor(h))) return rc;
    HIPCHK(rfim_dev::launch_init(h->lattice(), 0, h->R, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

void destroy_impl(rfim *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_device(h);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

// Streaming sweeps of two halves of the replicas on two streams: replicas
// never interact within an exchange interval, and the two launch sequences
// fill each other's start-up and drain time.  Worth it only for launches
// that are large on their own: from 2^22 sites of one colour per half (R >= 64
// at L = 64) for byte spins, from 2^23 for the bit sweep, whose launches are
// shortest (measured on gfx950 at L = 64, +-1 fields: R = 64 one stream runs
// 1196 attempts/ns against 827 split, at R = 128 the split wins, 1709 against
// 1575; continuous fields: 1128 against 957 at R = 64, 1421 against 1708 at
// R = 128).
constexpr long long kSplitMinAttempts = 1ll << 22;
constexpr long long kSplitMinAttemptsBits = 1ll << 23;

int ensure_aux(rfim *h) {
    if (h->aux && h->aux_for == h->stream) return RFIM_OK;
    if (h->aux) {                   // the handle stream changed since
        release_side_stream(h->aux);
        h->aux = nullptr;
    }
    HIPCHK(acquire_side_stream(h->stream, &h->aux));
    h->aux_for = h->stream;
    if (!h->ev_fork) HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    if (!h->ev_join) HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    return RFIM_OK;
}

int sweep_impl(rfim *h, int64_t n, int every) {
    h->lat_host = h->lattice();
    const Lattice &lat = h->lat_host;
    const rfim_dev::Launch ln = single_launch(h);
    const bool pow2 = h->log2L >= 3;
    const bool tiled = h->order == 1;
    const bool bitsm = h->bits_mode;
    const bool big = (long long)(h->R / 2) * h->half >=
                     (bitsm ? kSplitMinAttemptsBits : kSplitMinAttempts);
    const bool split = !tiled && pow2 && (bitsm || h->mode == 0) && h->R >= 2 &&
                       (h->concurrency == 2 || (h->concurrency == 0 && big));
    rfim_dev::Launch la = ln, lb = ln;
    const int ra = split ? h->R / 2 : h->R;
    if (split) {
        int rc;
        if ((rc = ensure_aux(h))) return rc;
        if (!bitsm) {
            const int wpr = ln.nblocks / h->R;
            la.nblocks = ra * wpr;
            lb.r0 = ra;
            lb.nblocks = (h->R - ra) * wpr;
        }
    }
    // Two streams: one fork at the start of the call and one join at its
    // end.  At each exchange step the streams meet once: the stream running
    // the step waits for the other's last half-sweep, runs the step (and the
    // measurement), and the other waits for it.  The step alternates between
    // the streams: whichever stream ran the previous step went on at once
    // while the other waited for it, so the other reaches the next step
    // later, and running the step there makes its own wait free -- one event
    // latency per interval on the critical path instead of two.  The first
    // step of a call runs on the second stream, which the fork delays.
    bool step_on_aux = true;
    if (split) {
        HIPCHK(hipEventRecord(h->ev_fork, h->stream));
        HIPCHK(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
    }
    int64_t remaining = n;
    while (remaining > 0) {
        int64_t to_next = every > 0 ? (int64_t)(every - (int64_t)(h->t % (uint64_t)every)) : remaining;
        const int m = (int)std::min<int64_t>(remaining, to_next);
        const bool exch = every > 0 && m == to_next;
        const bool fused = exch && !tiled && (bitsm || rfim_dev::fused_energy(lat));
        if (bitsm) {
            for (int q = 0; q < m; ++q) {
                const int e = fused && q == m - 1;
                HIPCHK(rfim_dev::launch_bits_sweep(lat, 0, ra, 0, q, 0, h->stream));
                if (split) HIPCHK(rfim_dev::launch_bits_sweep(lat, ra, h->R - ra, 0, q, 0, h->aux));
                HIPCHK(rfim_dev::launch_bits_sweep(lat, 0, ra, 1, q, e, h->stream));
                if (split) HIPCHK(rfim_dev::launch_bits_sweep(lat, ra, h->R - ra, 1, q, e, h->aux));
            }
        } else if (tiled) {
            for (int q = 0; q < m; ++q) {
                HIPCHK(rfim_dev::launch_tile_sweep(lat, h->tiles, 0, q, h->stream));
                HIPCHK(rfim_dev::launch_tile_sweep(lat, h->tiles, 1, q, h->stream));
            }
        } else if (pow2 && h->mode >= 2) {
            // slabs: up to mode - 1 sweeps per launch, alternating buffers
            const int K = rfim_dev::slab_sweeps_per_launch(h->mode);
            for (int q = 0; q < m;) {
                const int ns = std::min(K, m - q);
                const int e = fused && q + ns == m;
                HIPCHK(rfim_dev::launch_slab_sweep(lat, h->d_spins, h->d_spins_alt, h->mode, h->nw, h->wg, ns, q, e,
                                                   h->stream));
                std::swap(h->d_spins, h->d_spins_alt);
                q += ns;
            }
            h->lat_host = h->lattice();
        } else if (pow2 && h->mode == 1) {
            HIPCHK(rfim_dev::launch_resident(ln, m, fused ? 1 : 0, h->stream));
        } else if (pow2 && split) {
            for (int q = 0; q < m; ++q) {
                const int e = fused && q == m - 1;
                HIPCHK(rfim_dev::launch_stream_sweep(la, 0, q, 0, h->stream));
                HIPCHK(rfim_dev::launch_stream_sweep(lb, 0, q, 0, h->aux));
                HIPCHK(rfim_dev::launch_stream_sweep(la, 1, q, e, h->stream));
                HIPCHK(rfim_dev::launch_stream_sweep(lb, 1, q, e, h->aux));
            }
        } else if (pow2) {
            for (int q = 0; q < m; ++q) {
                HIPCHK(rfim_dev::launch_stream_sweep(ln, 0, q, 0, h->stream));
                HIPCHK(rfim_dev::launch_stream_sweep(ln, 1, q, fused && q == m - 1, h->stream));
            }
        } else {
            for (int q = 0; q < m; ++q) {
                HIPCHK(rfim_dev::launch_generic_sweep(lat, 0, q, h->stream));
                HIPCHK(rfim_dev::launch_generic_sweep(lat, 1, q, h->stream));
            }
        }
        if (exch) {
            hipStream_t xs = h->stream;
            if (split) {
                xs = step_on_aux ? h->aux : h->stream;
                hipStream_t other = step_on_aux ? h->stream : h->aux;
                HIPCHK(hipEventRecord(h->ev_join, other));
                HIPCHK(hipStreamWaitEvent(xs, h->ev_join, 0));
            }
            if (!fused) HIPCHK(rfim_dev::launch_energy(lat, xs));
            HIPCHK(rfim_dev::launch_exchange(h->d_lat, 1, m, xs));
            int rc;
            if ((rc = measure_after_exchange(h, xs))) return rc;
            if (split) {
                hipStream_t other = step_on_aux ? h->stream : h->aux;
                HIPCHK(hipEventRecord(h->ev_fork, xs));
                HIPCHK(hipStreamWaitEvent(other, h->ev_fork, 0));
                step_on_aux = !step_on_aux;
            }
            h->k += 1;
        } else {
            // the counter advance changes the sweep index both streams read:
            // join first (this is the last interval of the call)
            if (split) {
                HIPCHK(hipEventRecord(h->ev_join, h->aux));
                HIPCHK(hipStreamWaitEvent(h->stream, h->ev_join, 0));
            }
            HIPCHK(rfim_dev::launch_advance(lat, m, h->stream));
        }
        h->t += (uint64_t)m;
        remaining -= m;
    }
    if (split) {
        HIPCHK(hipEventRecord(h->ev_join, h->aux));
        HIPCHK(hipStreamWaitEvent(h->stream, h->ev_join, 0));
    }
    return RFIM_OK;
}

}  // namespace

// ===================================================================
// C ABI
// ===================================================================
extern "C" {

const char *rfim_last_error(void) { return g_error.c_str(); }

rfim_t *rfim_create_ex(const rfim_params_t *params, const rfim_alloc_t *alloc, void *hip_stream) {
    if (alloc && (!alloc->alloc || !alloc->free)) {
        fail(RFIM_EINVAL, "a device memory provider needs both alloc and free");
        return nullptr;
    }
    int err = 0;
    rfim *h = create_impl(params, hip_stream, &err);
    if (!h) return nullptr;
    if (alloc) h->alloc = *alloc;
    if (init_device(h)) {
        std::string msg = g_error;
        destroy_impl(h);
        g_error = msg;
        return nullptr;
    }
    // L = 64..256 defaults to one bit per spin, the faster storage there
    // for both field kinds (the same chain; measured on gfx950, continuous
    // fields: +19-25 % at L = 64, +32-50 % at L = 128); if its arrays cannot
    // be had the handle keeps byte spins
    if (rfim_dev::bits_valid(h->L) && rfim_set_spin_storage(h, RFIM_SPINS_BITS) != RFIM_OK) {
        (void)hipGetLastError();
        g_error.clear();
    }
    // continuous fields at L = 32 with few replicas: slabs of 8 planes, two
    // sweeps per launch, so that the replicas cover all CUs (measured on
    // gfx950 at R = 64: +14 % over one workgroup per replica; at R = 128 the
    // resident shape is faster); without the second spin buffer the handle
    // keeps the resident shape
    if (h->kind == 1 && h->L == 32 && h->R_cap <= kSlabDefaultMaxReplicas &&
        rfim_set_launch_shape(h, 3, 4, 1024) != RFIM_OK) {
        (void)hipGetLastError();
        g_error.clear();
    }
    return h;
}

rfim_t *rfim_create(int L, int R, double J, double h, const float *fields, const double *temps,
                    uint64_t seed) {
    rfim_params_t p;
    std::memset(&p, 0, sizeof p);
    p.L = L;
    p.R = R;
    p.R_cap = R;
    p.J = J;
    p.h = h;
    p.fields = fields;
    p.temps = temps;
    p.seed = seed;
    p.realization = 0;
    p.field_kind = RFIM_FIELDS_AUTO;
    return rfim_create_ex(&p, nullptr, nullptr);
}

void rfim_destroy(rfim_t *h) {
    if (h && h->in_batch) return;   // owned by its batch
    destroy_impl(h);
}

int rfim_set_stream(rfim_t *h, void *hip_stream) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    HIPCHK(hipStreamSynchronize(h->stream));
    if (h->own_stream && hip_stream) {
        HIPCHK(hipStreamDestroy(h->stream));
        h->own_stream = false;
        h->stream = (hipStream_t)hip_stream;
    } else if (hip_stream) {
        h->stream = (hipStream_t)hip_stream;
    } else if (!h->own_stream) {
        HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    return RFIM_OK;
}

int rfim_synchronize(rfim_t *h) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int rfim_sweep(rfim_t *h, int64_t n, int exchange_every) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (h->in_batch) return fail(RFIM_ESTATE, "batch items advance through rfim_batch_sweep");
    if (n < 0 || exchange_every < 0) return fail(RFIM_EINVAL, "n and exchange_every must be >= 0");
    if (h->t + (uint64_t)n > kMaxSweeps) return fail(RFIM_ECAP, "global sweep counter would pass 2^31-1");
    if (h->order == 1 && (h->t + (uint64_t)n) * (uint64_t)h->tiles.hits > (1ull << 31))
        return fail(RFIM_ECAP, "tile order: (sweep counter + n) * hits would pass 2^31");
    return sweep_impl(h, n, exchange_every);
}

int rfim_num_replicas(const rfim_t *h) { return h ? h->R : fail(RFIM_EINVAL, "handle is NULL"); }
int rfim_lattice_size(const rfim_t *h) { return h ? h->L : fail(RFIM_EINVAL, "handle is NULL"); }
int rfim_field_kind(const rfim_t *h) { return h ? h->kind : fail(RFIM_EINVAL, "handle is NULL"); }

int rfim_temps(const rfim_t *h, double *T) {
    if (!h || !T) return fail(RFIM_EINVAL, "NULL argument");
    std::copy(h->T.begin(), h->T.end(), T);
    return RFIM_OK;
}

int rfim_components(rfim_t *h, int64_t *B, double *F, int64_t *M) {
    if (!h || !B || !F || !M) return fail(RFIM_EINVAL, "NULL argument");
    int rc = compute_components(h);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(B, h->d_B, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(F, h->d_F, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(M, h->d_M, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int rfim_energies(rfim_t *h, double *E) {
    if (!h || !E) return fail(RFIM_EINVAL, "NULL argument");
    int rc = compute_components(h);
    if (rc) return rc;
    std::vector<double> byrep(h->R);
    HIPCHK(hipMemcpyAsync(byrep.data(), h->d_E, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    std::vector<int32_t> t2r;
    if ((rc = download_perm(h, t2r))) return rc;
    for (int t = 0; t < h->R; ++t) E[t] = byrep[t2r[t]];
    return RFIM_OK;
}

int rfim_magnetizations(rfim_t *h, int64_t *M) {
    if (!h || !M) return fail(RFIM_EINVAL, "NULL argument");
    int rc = compute_components(h);
    if (rc) return rc;
    std::vector<int64_t> byrep(h->R);
    HIPCHK(hipMemcpyAsync(byrep.data(), h->d_M, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    std::vector<int32_t> t2r;
    if ((rc = download_perm(h, t2r))) return rc;
    for (int t = 0; t < h->R; ++t) M[t] = byrep[t2r[t]];
    return RFIM_OK;
}

int rfim_get_spins(rfim_t *h, int8_t *s) {
    if (!h || !s) return fail(RFIM_EINVAL, "NULL argument");
    const size_t N = (size_t)h->N, half = N / 2;
    std::vector<uint8_t> dev((size_t)h->R * N);
    int rc;
    if ((rc = bytes_from_bits(h))) return rc;
    HIPCHK(hipMemcpyAsync(dev.data(), h->d_spins, dev.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int r = 0; r < h->R; ++r) {
        const uint8_t *src = dev.data() + (size_t)r * N;
        int8_t *dst = s + (size_t)r * N;
        for_each_site(h->L, [&](size_t i, int c, size_t j) { dst[i] = src[c * half + j] ? 1 : -1; });
    }
    return RFIM_OK;
}

int rfim_set_spins(rfim_t *h, const int8_t *s) {
    if (!h || !s) return fail(RFIM_EINVAL, "NULL argument");
    const size_t N = (size_t)h->N, half = N / 2;
    for (size_t q = 0; q < (size_t)h->R * N; ++q)
        if (s[q] != 1 && s[q] != -1) return fail(RFIM_EINVAL, "spins must be +-1 (index %zu)", q);
    std::vector<uint8_t> dev((size_t)h->R * N);
    for (int r = 0; r < h->R; ++r) {
        uint8_t *dst = dev.data() + (size_t)r * N;
        const int8_t *src = s + (size_t)r * N;
        for_each_site(h->L, [&](size_t i, int c, size_t j) { dst[c * half + j] = src[i] > 0 ? 1 : 0; });
    }
    HIPCHK(hipMemcpyAsync(h->d_spins, dev.data(), dev.size(), hipMemcpyHostToDevice, h->stream));
    int rc;
    if ((rc = bits_from_bytes(h))) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int rfim_get_perm(rfim_t *h, int32_t *t2r) {
    if (!h || !t2r) return fail(RFIM_EINVAL, "NULL argument");
    std::vector<int32_t> v;
    int rc = download_perm(h, v);
    if (rc) return rc;
    std::copy(v.begin(), v.end(), t2r);
    return RFIM_OK;
}

int rfim_set_perm(rfim_t *h, const int32_t *t2r) {
    if (!h || !t2r) return fail(RFIM_EINVAL, "NULL argument");
    std::vector<char> seen(h->R, 0);
    for (int t = 0; t < h->R; ++t) {
        if (t2r[t] < 0 || t2r[t] >= h->R || seen[t2r[t]]) return fail(RFIM_EINVAL, "t2r is not a permutation");
        seen[t2r[t]] = 1;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return upload_perm(h, std::vector<int32_t>(t2r, t2r + h->R));
}

int rfim_get_counters(rfim_t *h, uint64_t *t, uint64_t *k) {
    if (!h || !t || !k) return fail(RFIM_EINVAL, "NULL argument");
    uint64_t c[2];
    HIPCHK(hipMemcpyAsync(c, h->d_ctrs, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (c[0] != h->t || c[1] != h->k) return fail(RFIM_EDEVICE, "device counters out of step");
    *t = c[0];
    *k = c[1];
    return RFIM_OK;
}

int rfim_set_counters(rfim_t *h, uint64_t t, uint64_t k) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (h->in_batch) return fail(RFIM_ESTATE, "batch items share the batch's counters");
    if (t > kMaxSweeps || k > 0xFFFFFFFFull) return fail(RFIM_ECAP, "counter beyond its range");
    HIPCHK(hipStreamSynchronize(h->stream));
    h->t = t;
    h->k = k;
    return upload_counters(h);
}

int rfim_exchange_stats(rfim_t *h, uint64_t *att, uint64_t *acc) {
    if (!h || (h->R > 1 && (!att || !acc))) return fail(RFIM_EINVAL, "NULL argument");
    if (h->R < 2) return RFIM_OK;
    HIPCHK(hipMemcpyAsync(att, h->d_att, (h->R - 1) * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(acc, h->d_acc, (h->R - 1) * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int rfim_reset_exchange_stats(rfim_t *h) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    return reset_stats(h);
}

// One insertion step of the adaptive method (Sec. 4) from the exchange
// counters accumulated since the last reset: rates acc/att into a min-heap,
// the lowest-rate intervals below the threshold get a new temperature at
// their midpoint (at most max_insert, R <= R_cap), each new replica copies
// the colder end and takes the next replica id; slots are re-sorted and the
// counters reset.  Synchronizes; returns the new R.
static int insert_step(rfim *h, double rate_threshold, int max_insert, int R_cap) {
    int rc;
    const int R0 = h->R;
    std::vector<uint64_t> att(R0), acc(R0);
    HIPCHK(hipMemcpyAsync(att.data(), h->d_att, R0 * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(acc.data(), h->d_acc, R0 * 8, hipMemcpyDeviceToHost, h->stream));
    std::vector<int32_t> t2r;
    if ((rc = download_perm(h, t2r))) return rc;
    using Item = std::pair<double, int>;
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int p = 0; p + 1 < R0; ++p)
        if (att[p] > 0) heap.push({(double)acc[p] / (double)att[p], p});
    std::vector<int> picked;
    while (!heap.empty() && (int)picked.size() < max_insert && R0 + (int)picked.size() < R_cap) {
        Item it = heap.top();
        heap.pop();
        if (!(it.first < rate_threshold)) break;
        picked.push_back(it.second);
    }
    if (picked.empty()) {
        if ((rc = reset_stats(h))) return rc;
        HIPCHK(hipStreamSynchronize(h->stream));
        return h->R;
    }
    std::vector<std::pair<double, int32_t>> slots;
    for (int t = 0; t < R0; ++t) slots.push_back({h->T[t], t2r[t]});
    for (size_t q = 0; q < picked.size(); ++q) {
        const int p = picked[q];
        const int32_t id = R0 + (int32_t)q;
        slots.push_back({(h->T[p] + h->T[p + 1]) / 2.0, id});
        if (h->bits_mode) {
            const size_t words = (size_t)h->N / 32;     // both colours of one replica
            HIPCHK(hipMemcpyAsync(h->d_bits + (size_t)id * words, h->d_bits + (size_t)t2r[p] * words,
                                  words * 4, hipMemcpyDeviceToDevice, h->stream));
        } else {
            HIPCHK(hipMemcpyAsync(h->d_spins + (size_t)id * h->N, h->d_spins + (size_t)t2r[p] * h->N,
                                  (size_t)h->N, hipMemcpyDeviceToDevice, h->stream));
        }
    }
    std::sort(slots.begin(), slots.end(),
              [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
                  return a.first < b.first;
              });
    h->R = (int)slots.size();
    h->T.resize(h->R);
    std::vector<int32_t> nt2r(h->R);
    for (int t = 0; t < h->R; ++t) {
        h->T[t] = slots[t].first;
        nt2r[t] = slots[t].second;
    }
    if ((rc = upload_perm(h, nt2r))) return rc;
    if ((rc = upload_tables(h))) return rc;
    if ((rc = sync_descriptor(h))) return rc;
    if ((rc = reset_stats(h))) return rc;
    if ((rc = reset_obs(h))) return rc;      // the slots changed
    HIPCHK(hipStreamSynchronize(h->stream));
    return h->R;
}

int rfim_adapt_temps(rfim_t *h, int trials, int64_t sweeps_per_trial, int exchange_every,
                     double rate_threshold, int max_insert_per_trial, int R_cap) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (trials < 0 || sweeps_per_trial < 0 || exchange_every <= 0 || max_insert_per_trial < 0 ||
        std::isnan(rate_threshold))
        return fail(RFIM_EINVAL, "bad adapt arguments");
    if (h->in_batch) return fail(RFIM_ESTATE, "batch items cannot change R");
    if (R_cap > h->R_cap) return fail(RFIM_ECAP, "R_cap %d beyond the capacity %d given at create", R_cap, h->R_cap);
    if (h->t + (uint64_t)trials * (uint64_t)sweeps_per_trial > kMaxSweeps)
        return fail(RFIM_ECAP, "global sweep counter would pass 2^31-1");
    int rc;
    for (int trial = 0; trial < trials; ++trial) {
        // trial run, continuing the chain, with fresh exchange counters
        if ((rc = reset_stats(h))) return rc;
        if ((rc = sweep_impl(h, sweeps_per_trial, exchange_every))) return rc;
        if ((rc = insert_step(h, rate_threshold, max_insert_per_trial, R_cap)) < 0) return rc;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return h->R;
}

int rfim_observables(rfim_t *h, double *obs) {
    if (!h || !obs) return fail(RFIM_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(obs, h->d_obs, (size_t)h->R * 6 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int rfim_reset_observables(rfim_t *h) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    return reset_obs(h);
}

int rfim_set_launch_shape(rfim_t *h, int mode, int nw, int wg) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (h->in_batch) return fail(RFIM_ESTATE, "batch items take their class shape (rfim_batch_set_shape)");
    if (!rfim_dev::shape_valid(h->L, mode, nw, wg))
        return fail(RFIM_EINVAL, "launch shape (%d, %d, %d) not valid for L=%d", mode, nw, wg, h->L);
    int rc;
    if (h->bits_mode && (rc = rfim_set_spin_storage(h, RFIM_SPINS_BYTES))) return rc;   // shapes are the byte kernels'
    if (mode >= 2 && !h->d_spins_own) {
        if ((rc = dev_alloc(h, (void **)&h->d_spins_own, (size_t)h->R_cap * h->N))) return rc;
        h->d_spins_alt = h->d_spins_own;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->mode = mode;
    h->nw = nw;
    h->wg = wg;
    h->nblk = rfim_dev::blocks_per_replica(h->L, mode, nw, wg);
    return sync_descriptor(h);
}

int rfim_get_launch_shape(const rfim_t *h, int *mode, int *nw, int *wg) {
    if (!h || !mode || !nw || !wg) return fail(RFIM_EINVAL, "NULL argument");
    *mode = h->mode;
    *nw = h->nw;
    *wg = h->wg;
    return RFIM_OK;
}

int rfim_set_measure(rfim_t *h, int flags) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (flags & ~RFIM_MEASURE_FOURIER) return fail(RFIM_EINVAL, "unknown measurement flags %d", flags);
    int rc0;
    if (flags && h->bits_mode && (rc0 = rfim_set_spin_storage(h, RFIM_SPINS_BYTES))) return rc0;   // it reads bytes
    if ((flags & RFIM_MEASURE_FOURIER) && !h->d_fpart) {
        const size_t L = (size_t)h->L, Rc = (size_t)h->R_cap;
        if (dev_alloc(h, (void **)&h->d_fpart, Rc * L * 2 * L * sizeof(int32_t)) ||
            dev_alloc(h, (void **)&h->d_trig, 2 * L * sizeof(double)) ||
            dev_alloc(h, (void **)&h->d_fobs, Rc * 2 * sizeof(double))) {
            (void)hipGetLastError();
            dev_free(h, h->d_fpart);
            dev_free(h, h->d_trig);
            dev_free(h, h->d_fobs);
            h->d_fpart = nullptr;
            h->d_trig = nullptr;
            h->d_fobs = nullptr;
            return fail(RFIM_ENOMEM, "no device memory for the Fourier measurement");
        }
        // cos and sin of 2 pi v / L with the host libm (the same values the
        // reference computation uses)
        std::vector<double> trig(2 * L);
        for (size_t v = 0; v < L; ++v) {
            trig[v] = std::cos(2.0 * 3.14159265358979323846 * (double)v / (double)L);
            trig[L + v] = std::sin(2.0 * 3.14159265358979323846 * (double)v / (double)L);
        }
        HIPCHK(hipMemcpyAsync(h->d_trig, trig.data(), trig.size() * sizeof(double), hipMemcpyHostToDevice,
                              h->stream));
        HIPCHK(hipMemsetAsync(h->d_fobs, 0, Rc * 2 * sizeof(double), h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->measure = flags;
    return RFIM_OK;
}

int rfim_fourier(rfim_t *h, double *fourier) {
    if (!h || !fourier) return fail(RFIM_EINVAL, "NULL argument");
    if (!h->d_fobs) {
        std::memset(fourier, 0, (size_t)h->R * 2 * sizeof(double));
        return RFIM_OK;
    }
    HIPCHK(hipMemcpyAsync(fourier, h->d_fobs, (size_t)h->R * 2 * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return RFIM_OK;
}

int rfim_set_concurrency(rfim_t *h, int streams) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (streams < 0 || streams > 2) return fail(RFIM_EINVAL, "streams must be 0, 1 or 2 (got %d)", streams);
    h->concurrency = streams;
    return RFIM_OK;
}

int rfim_get_concurrency(const rfim_t *h) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    return h->concurrency;
}

int rfim_set_update_order(rfim_t *h, int order, int tx, int ty, int tz, int hits) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (h->in_batch) return fail(RFIM_ESTATE, "batch and pool items sweep in the plain order");
    if (order != RFIM_ORDER_CHECKERBOARD && order != RFIM_ORDER_TILES)
        return fail(RFIM_EINVAL, "unknown update order %d", order);
    if (order == RFIM_ORDER_TILES) {
        int rc0;
        if (h->bits_mode && (rc0 = rfim_set_spin_storage(h, RFIM_SPINS_BYTES))) return rc0;   // tiles run on bytes
        const rfim_dev::TileShape ts = {tx, ty, tz, hits};
        if (!rfim_dev::tile_shape_valid(h->L, ts))
            return fail(RFIM_EINVAL,
                        "tiles (%d, %d, %d) x %d hits not valid for L=%d: L a power of two >= 16, tx a multiple "
                        "of 8, each side dividing L into an even number of tiles, (tx/8)*ty*tz a multiple of 64 "
                        "in [64, 1024], 1 <= hits <= 65536",
                        tx, ty, tz, hits, h->L);
        if (h->t * (uint64_t)hits > (1ull << 31))
            return fail(RFIM_ECAP, "tile order: sweep counter * hits would pass 2^31");
        HIPCHK(hipStreamSynchronize(h->stream));
        h->tiles = ts;
    } else {
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->order = order;
    return RFIM_OK;
}

namespace {

// Switch a handle's spin storage (a batch or pool item's too: its class
// shape decides); switching to bytes leaves the launch shape as it is.
int set_storage_impl(rfim *h, int storage) {
    if (storage == (h->bits_mode ? RFIM_SPINS_BITS : RFIM_SPINS_BYTES)) return RFIM_OK;
    if (storage == RFIM_SPINS_BITS) {
        if (!rfim_dev::bits_valid(h->L))
            return fail(RFIM_EINVAL, "one bit per spin needs L = 64, 128 or 256 (got %d)", h->L);
        if (h->order != RFIM_ORDER_CHECKERBOARD)
            return fail(RFIM_ESTATE, "one bit per spin runs the plain checkerboard order");
        if (h->measure) return fail(RFIM_ESTATE, "turn the Fourier measurement off first");
        if (!h->d_bits) {
            const size_t words = (size_t)h->R_cap * (size_t)h->N / 32;
            int rc = dev_alloc(h, (void **)&h->d_bits, words * 4);
            if (!rc && h->kind == 0) rc = dev_alloc(h, (void **)&h->d_fbw, (size_t)h->N / 8);
            if (!rc && h->kind == 1) rc = dev_alloc(h, (void **)&h->d_fhw, (size_t)h->N * sizeof(float));
            if (rc) {
                dev_free(h, (void *)h->d_bits);
                dev_free(h, (void *)h->d_fbw);
                h->d_bits = nullptr;
                h->d_fbw = nullptr;
                return rc;
            }
        }
        h->bits_mode = true;
        HIPCHK(rfim_dev::launch_pack_bits(h->lattice(), h->stream));
        h->nblk = rfim_dev::bits_blocks_per_replica(h->L);
    } else {
        HIPCHK(rfim_dev::launch_unpack_bits(h->lattice(), h->stream));
        h->bits_mode = false;
        h->nblk = rfim_dev::blocks_per_replica(h->L, h->mode, h->nw, h->wg);
    }
    return sync_descriptor(h);
}

}  // namespace

int rfim_set_spin_storage(rfim_t *h, int storage) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    if (h->in_batch)
        return fail(RFIM_ESTATE, "batch and pool items take their storage from the class shape "
                                 "(rfim_batch_set_shape / rfim_pool_set_shape)");
    if (storage != RFIM_SPINS_BYTES && storage != RFIM_SPINS_BITS)
        return fail(RFIM_EINVAL, "unknown spin storage %d", storage);
    return set_storage_impl(h, storage);
}

int rfim_get_spin_storage(const rfim_t *h) {
    if (!h) return fail(RFIM_EINVAL, "handle is NULL");
    return h->bits_mode ? RFIM_SPINS_BITS : RFIM_SPINS_BYTES;
}

int rfim_get_update_order(const rfim_t *h, int *order, int *tx, int *ty, int *tz, int *hits) {
    if (!h || !order || !tx || !ty || !tz || !hits) return fail(RFIM_EINVAL, "NULL argument");
    *order = h->order;
    *tx = h->order ? h->tiles.tx : 0;
    *ty = h->order ? h->tiles.ty : 0;
    *tz = h->order ? h->tiles.tz : 0;
    *hits = h->order ? h->tiles.hits : 1;
    return RFIM_OK;
}

// ---- checkpoint ----------------------------------------------------
// Blob: magic, version, L, R, R_cap, kind, J, h, seed, realization, t, k,
// T[R], fields[N], spins[R][N] (+-1, natural order), t2r[R], att[R], acc[R].
namespace {
constexpr uint64_t kMagic = 0x314D494652ull;  // "RFIM1"
struct Header {
    uint64_t magic, version;
    int32_t L, R, R_cap, kind;
    double J, h;
    uint64_t seed;
    uint32_t rho, pad;
    uint64_t t, k;
};
size_t blob_size(int L, int R) {
    const size_t N = (size_t)L * L * L;
    return sizeof(Header) + R * 8 + N * 4 + (size_t)R * N + R * 4 + 2 * (size_t)R * 8;
}
}  // namespace

int rfim_save(rfim_t *h, void *buf, size_t *len) {
    if (!h || !len) return fail(RFIM_EINVAL, "NULL argument");
    const size_t need = blob_size(h->L, h->R);
    if (!buf) {
        *len = need;
        return RFIM_OK;
    }
    if (*len < need) return fail(RFIM_EINVAL, "buffer too small (%zu < %zu)", *len, need);
    uint8_t *p = (uint8_t *)buf;
    Header hd;
    std::memset(&hd, 0, sizeof hd);
    hd.magic = kMagic;
    hd.version = 1;
    hd.L = h->L;
    hd.R = h->R;
    hd.R_cap = h->R_cap;
    hd.kind = h->kind;
    hd.J = h->J;
    hd.h = h->h;
    hd.seed = h->seed;
    hd.rho = h->rho;
    int rc = rfim_get_counters(h, &hd.t, &hd.k);
    if (rc) return rc;
    std::memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    std::memcpy(p, h->T.data(), h->R * 8);
    p += h->R * 8;
    std::memcpy(p, h->fields.data(), (size_t)h->N * 4);
    p += (size_t)h->N * 4;
    if ((rc = rfim_get_spins(h, (int8_t *)p))) return rc;
    p += (size_t)h->R * h->N;
    if ((rc = rfim_get_perm(h, (int32_t *)p))) return rc;
    p += h->R * 4;
    HIPCHK(hipMemcpyAsync(p, h->d_att, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    p += h->R * 8;
    HIPCHK(hipMemcpyAsync(p, h->d_acc, h->R * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *len = need;
    return RFIM_OK;
}

rfim_t *rfim_load(const void *buf, size_t len, void *hip_stream) {
    if (!buf || len < sizeof(Header)) {
        fail(RFIM_EINVAL, "checkpoint buffer too small");
        return nullptr;
    }
    Header hd;
    std::memcpy(&hd, buf, sizeof hd);
    if (hd.magic != kMagic || hd.version != 1) {
        fail(RFIM_EINVAL, "not an rfim checkpoint");
        return nullptr;
    }
    if (hd.L < 2 || hd.L > 1024 || hd.R < 1 || hd.R > kMaxR || len < blob_size(hd.L, hd.R)) {
        fail(RFIM_EINVAL, "corrupt checkpoint header");
        return nullptr;
    }
    const uint8_t *p = (const uint8_t *)buf + sizeof hd;
    const size_t N = (size_t)hd.L * hd.L * hd.L;
    rfim_params_t prm;
    std::memset(&prm, 0, sizeof prm);
    prm.L = hd.L;
    prm.R = hd.R;
    prm.R_cap = hd.R_cap;
    prm.J = hd.J;
    prm.h = hd.h;
    prm.seed = hd.seed;
    prm.realization = hd.rho;
    prm.field_kind = hd.kind;
    std::vector<double> T(hd.R);
    std::memcpy(T.data(), p, hd.R * 8);
    p += hd.R * 8;
    std::vector<float> f(N);
    std::memcpy(f.data(), p, N * 4);
    p += N * 4;
    prm.temps = T.data();
    prm.fields = f.data();
    rfim *h = rfim_create_ex(&prm, nullptr, hip_stream);
    if (!h) return nullptr;
    int rc = rfim_set_spins(h, (const int8_t *)p);
    p += (size_t)hd.R * N;
    if (!rc) {
        std::vector<int32_t> t2r(hd.R);
        std::memcpy(t2r.data(), p, hd.R * 4);
        rc = rfim_set_perm(h, t2r.data());
    }
    p += hd.R * 4;
    if (!rc) rc = rfim_set_counters(h, hd.t, hd.k);
    if (!rc) {
        hipError_t e1 = hipMemcpyAsync(h->d_att, p, hd.R * 8, hipMemcpyHostToDevice, h->stream);
        hipError_t e2 = hipMemcpyAsync(h->d_acc, p + hd.R * 8, hd.R * 8, hipMemcpyHostToDevice, h->stream);
        hipError_t e3 = hipStreamSynchronize(h->stream);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) rc = fail(RFIM_EDEVICE, "checkpoint upload failed");
    }
    if (rc) {
        std::string msg = g_error;
        destroy_impl(h);
        g_error = msg;
        return nullptr;
    }
    return h;
}

}  // extern "C"

// ===================================================================
// Batches: many independent realizations advanced together.  The sweeps of
// every realization that shares (L, field kind) go into one launch per
// half-sweep (streaming) or per exchange interval (LDS-resident), and one
// launch runs the exchange step of every realization; a full exchange
// interval is captured once in a HIP graph and replayed.
// ===================================================================
struct rfim_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<rfim *> items;
    Lattice *d_lats = nullptr;
    std::vector<Lattice> lats_host;
    struct Class {
        int L = 0, kind = 0, mode = 0, nw = 0, wg = 0;
        std::vector<int> members;
        uint2 *d_map = nullptr;
        size_t cap = 0;                 // entries d_map can hold
        int nblocks = 0;
    };
    std::vector<Class> classes;
    int64_t group_bytes = 96ll << 20;   // temporal blocking of large streaming classes (0: off)
    uint64_t t = 0, k = 0;
    hipGraphExec_t graph = nullptr;
    int graph_every = 0;
    std::vector<int> graph_measure;     // items' measurement flags the graph was captured with
    // side streams for classes (and halves of large streaming classes) that
    // run concurrently within an exchange interval; events fork them from
    // and join them back into `stream`
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
};

namespace {

static_assert(rfim_dev::kModeBits == RFIM_MODE_BITS, "the class mode of bit storage is the ABI's");

// A batch or pool item to its class shape: one bit per spin for
// (kModeBits, 0, 0), byte spins with that launch shape otherwise.
int item_apply_shape(rfim *h, int mode, int nw, int wg) {
    int rc;
    if (mode == rfim_dev::kModeBits) {
        if ((rc = set_storage_impl(h, RFIM_SPINS_BITS))) return rc;
        h->mode = mode;
        h->nw = 0;
        h->wg = 0;
        return sync_descriptor(h);
    }
    h->mode = mode;
    h->nw = nw;
    h->wg = wg;
    if (h->bits_mode) return set_storage_impl(h, RFIM_SPINS_BYTES);   // sets nblk from the shape
    h->nblk = rfim_dev::blocks_per_replica(h->L, mode, nw, wg);
    return sync_descriptor(h);
}

// A class shape batches and pools take (the single-realization shapes
// without the slabs, and the bit storage).
int check_class_shape(int L, int mode, int nw, int wg) {
    if (mode == rfim_dev::kModeBits) {
        if (!rfim_dev::bits_valid(L) || nw != 0 || wg != 0)
            return fail(RFIM_EINVAL, "bit storage (%d, 0, 0) needs L = 64, 128 or 256 (got L=%d, shape (%d, %d, %d))",
                        rfim_dev::kModeBits, L, mode, nw, wg);
        return RFIM_OK;
    }
    if (mode >= 2) return fail(RFIM_EINVAL, "slab shapes are for single realizations");
    if (!rfim_dev::shape_valid(L, mode, nw, wg))
        return fail(RFIM_EINVAL, "launch shape (%d, %d, %d) not valid for L=%d", mode, nw, wg, L);
    return RFIM_OK;
}

// Every member of class c to shape (mode, nw, wg), and the class with them;
// on failure the members go back to the class's shape.
int class_apply_shape(rfim_batch *b, rfim_batch::Class &c, int mode, int nw, int wg) {
    int rc;
    for (int i : c.members)
        if ((rc = item_apply_shape(b->items[i], mode, nw, wg))) {
            const std::string msg = g_error;
            for (int j : c.members) (void)item_apply_shape(b->items[j], c.mode, c.nw, c.wg);
            g_error = msg;
            return rc;
        }
    c.mode = mode;
    c.nw = mode == rfim_dev::kModeBits ? 0 : nw;
    c.wg = mode == rfim_dev::kModeBits ? 0 : wg;
    return RFIM_OK;
}

void batch_free(rfim_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (auto &c : b->classes)
        if (c.d_map) (void)hipFree(c.d_map);
    if (b->d_lats) (void)hipFree(b->d_lats);
    for (rfim *h : b->items) {
        h->stream = nullptr;      // the batch owns the stream
        h->own_stream = false;
        free_device(h);
        delete h;
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t e : b->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t q : b->aux) (void)hipStreamDestroy(q);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Descriptors of every item and the workgroup maps of every class.
int batch_build(rfim_batch *b) {
    const int n = (int)b->items.size();
    b->lats_host.resize(n);
    for (int i = 0; i < n; ++i) b->lats_host[i] = b->items[i]->lattice();
    HIPCHK(hipMemcpyAsync(b->d_lats, b->lats_host.data(), n * sizeof(Lattice), hipMemcpyHostToDevice, b->stream));
    std::vector<std::vector<uint2>> maps(b->classes.size());
    for (size_t ci = 0; ci < b->classes.size(); ++ci) {
        auto &c = b->classes[ci];
        std::vector<uint2> &map = maps[ci];
        for (int i : c.members) {
            const rfim *h = b->items[i];
            const uint32_t hi = (uint32_t)i << 16;
            if (c.mode == 1 || c.mode == rfim_dev::kModeBits) {     // one entry per replica
                for (int r = 0; r < h->R; ++r) map.push_back(make_uint2(hi | (uint32_t)r, 0u));
            } else {
                const int wpr = rfim_dev::stream_blocks_per_replica(c.L, c.nw, c.wg);
                for (int r = 0; r < h->R; ++r)
                    for (int g = 0; g < wpr; ++g) map.push_back(make_uint2(hi | (uint32_t)r, (uint32_t)g));
            }
        }
        c.nblocks = (int)map.size();
        if (map.size() > c.cap) {
            if (c.d_map) HIPCHK(hipFree(c.d_map));
            c.d_map = nullptr;
            c.cap = 0;
            const size_t cap = map.size() + map.size() / 2;
            hipError_t e = hipMalloc((void **)&c.d_map, cap * sizeof(uint2));
            if (e != hipSuccess) return fail(RFIM_ENOMEM, "hipMalloc(batch map): %s", hipGetErrorString(e));
            c.cap = cap;
        }
        if (!map.empty())
            HIPCHK(hipMemcpyAsync(c.d_map, map.data(), map.size() * sizeof(uint2), hipMemcpyHostToDevice, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->graph) {
        HIPCHK(hipGraphExecDestroy(b->graph));
        b->graph = nullptr;
        b->graph_every = 0;
    }
    return RFIM_OK;
}

rfim_dev::Launch class_launch(const rfim_batch *b, const rfim_batch::Class &c) {
    rfim_dev::Launch ln;
    ln.single = nullptr;
    ln.lats = b->d_lats;
    ln.map = c.d_map;
    ln.nblocks = c.nblocks;
    ln.L = c.L;
    ln.kind = c.kind;
    ln.mode = c.mode;
    ln.nw = c.nw;
    ln.wg = c.wg;
    return ln;
}

// Classes never share items, and the workgroups of one streaming launch
// are independent within a half-sweep, so an interval's launches form
// independent lanes: one per class, two for a streaming class of at least
// kSplitMinAttempts sites per half.  Lanes go round-robin (largest first)
// to the batch stream and up to kMaxSideStreams side streams.
constexpr int kMaxSideStreams = 3;

struct Lane {
    int mode;                           // the class's launch mode
    std::vector<rfim_dev::Launch> ln;   // one launch, or the groups of a large class in order
    long long work;
    bool fused;         // the class's sweep kernels write the energy partials
};

// True when the sweep kernels of class c write its items' energy partials
// (resident shapes, and streaming shapes with at most kMaxFusedBlocks
// workgroups per replica); other classes get the separate energy kernel
// before the exchange step.
bool class_fused(const rfim_batch *b, const rfim_batch::Class &c) {
    if (c.members.empty()) return true;
    return rfim_dev::fused_energy(b->items[c.members[0]]->lattice());
}

int ensure_side_streams(rfim_batch *b, int n) {
    if (!b->ev_fork) HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    while ((int)b->aux.size() < n) {
        hipStream_t q = nullptr;
        hipEvent_t e = nullptr;
        // plain streams: lanes of a batch made right after many short-lived
        // batches (the autotuner's probes) ran ~30 % slower on CU-masked
        // queues of their own
        HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        b->aux.push_back(q);
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->ev_join.push_back(e);
    }
    return RFIM_OK;
}

// Temporal blocking of large streaming classes.  A class whose spins exceed
// 2 kGroupBytes runs as two lanes (the two halves of its members, on two
// streams), and a lane as groups of consecutive members of at most
// kGroupBytes of spins (at least one member each): a group runs all sweeps
// of the interval before the next group of its lane starts, so the two
// groups in flight stay inside the 256 MB on-package cache across the
// interval's half-sweeps instead of the whole class streaming through HBM
// once per half-sweep.  kGroupBytes is rfim_batch::group_bytes
// (rfim_batch_set_group_bytes); 0 turns the blocking off.

// The lanes of one class (see above and the two-lane split).
void class_lanes(const rfim_batch *b, const rfim_batch::Class &c, std::vector<Lane> &lanes) {
    const rfim_dev::Launch ln = class_launch(b, c);
    if (c.mode == rfim_dev::kModeBits) {
        // one launch per half-sweep over every replica of the class (map
        // entries are replicas), or two launches of half the replicas each
        // on two lanes from kSplitMinAttemptsBits sites per half, as for
        // one realization
        const long long sites = (long long)ln.nblocks * c.L * c.L * c.L / 2;
        if (ln.nblocks >= 2 && sites / 2 >= kSplitMinAttemptsBits) {
            rfim_dev::Launch la = ln, lb = ln;
            la.nblocks = ln.nblocks / 2;
            lb.map = ln.map + la.nblocks;
            lb.nblocks = ln.nblocks - la.nblocks;
            lanes.push_back({c.mode, {la}, (long long)la.nblocks * c.L * c.L * c.L / 2, true});
            lanes.push_back({c.mode, {lb}, (long long)lb.nblocks * c.L * c.L * c.L / 2, true});
        } else if (ln.nblocks > 0) {
            lanes.push_back({c.mode, {ln}, sites, true});
        }
        return;
    }
    const bool fused = class_fused(b, c);
    const long long sites = (long long)ln.nblocks * (c.mode == 1 ? (long long)c.L * c.L * c.L / 2
                                                                  : 4ll * c.nw * c.wg);
    if (c.mode != 0) {
        lanes.push_back({c.mode, {ln}, sites, fused});
        return;
    }
    long long bytes = 0;
    for (int i : c.members) bytes += (long long)b->items[i]->R * b->items[i]->N;
    const long long kGroupBytes = b->group_bytes;
    if (kGroupBytes > 0 && bytes > 2 * kGroupBytes && c.members.size() > 1) {
        const int wpr = rfim_dev::stream_blocks_per_replica(c.L, c.nw, c.wg);
        const long long sites_per_block = 4ll * c.nw * c.wg;
        // groups of consecutive members
        std::vector<rfim_dev::Launch> groups;
        std::vector<long long> gb;
        int first = 0, nblk = 0;
        long long gbytes = 0;
        for (size_t q = 0; q <= c.members.size(); ++q) {
            const rfim *h = q < c.members.size() ? b->items[c.members[q]] : nullptr;
            const long long hb = h ? (long long)h->R * h->N : 0;
            if (nblk > 0 && (!h || gbytes + hb > kGroupBytes)) {
                rfim_dev::Launch lg = ln;
                lg.map = ln.map + first;
                lg.nblocks = nblk;
                groups.push_back(lg);
                gb.push_back(gbytes);
                first += nblk;
                nblk = 0;
                gbytes = 0;
            }
            if (h) {
                nblk += h->R * wpr;
                gbytes += hb;
            }
        }
        // two lanes: the groups up to half of the bytes, and the rest
        size_t cut = 0;
        long long acc = 0;
        while (cut + 1 < groups.size() && 2 * (acc + gb[cut]) <= bytes) acc += gb[cut++];
        if (cut == 0) cut = 1;
        for (int side = 0; side < 2; ++side) {
            Lane l{c.mode, {}, 0, fused};
            for (size_t g = side ? cut : 0; g < (side ? groups.size() : cut); ++g) {
                l.ln.push_back(groups[g]);
                l.work += (long long)groups[g].nblocks * sites_per_block;
            }
            if (!l.ln.empty()) lanes.push_back(l);
        }
        return;
    }
    if (ln.nblocks >= 16 && sites / 2 >= kSplitMinAttempts) {
        rfim_dev::Launch la = ln, lb = ln;
        la.nblocks = (ln.nblocks / 2) & ~7;
        lb.map = ln.map + la.nblocks;
        lb.nblocks = ln.nblocks - la.nblocks;
        lanes.push_back({c.mode, {la}, sites / 2, fused});
        lanes.push_back({c.mode, {lb}, sites / 2, fused});
    } else {
        lanes.push_back({c.mode, {ln}, sites, fused});
    }
}

// m sweeps of every item; exch: energies (fused) and one exchange step.
int batch_segment(rfim_batch *b, int m, bool exch) {
    std::vector<Lane> lanes;
    for (const auto &c : b->classes) class_lanes(b, c, lanes);
    std::stable_sort(lanes.begin(), lanes.end(), [](const Lane &x, const Lane &y) { return x.work > y.work; });
    const int nside = std::min((int)lanes.size() - 1, kMaxSideStreams);
    std::vector<hipStream_t> qs(1, b->stream);
    if (nside > 0) {
        int rc;
        if ((rc = ensure_side_streams(b, nside))) return rc;
        HIPCHK(hipEventRecord(b->ev_fork, b->stream));
        for (int j = 0; j < nside; ++j) {
            HIPCHK(hipStreamWaitEvent(b->aux[j], b->ev_fork, 0));
            qs.push_back(b->aux[j]);
        }
    }
    const int nq = (int)qs.size();
    for (size_t i = 0; i < lanes.size(); ++i)
        if (lanes[i].mode == 1)
            HIPCHK(rfim_dev::launch_resident(lanes[i].ln[0], m, exch ? 1 : 0, qs[i % nq]));
    // lane by lane, and in a lane group by group: a group's half-sweeps
    // follow one another on its stream
    for (size_t i = 0; i < lanes.size(); ++i)
        if (lanes[i].mode == 0 || lanes[i].mode == rfim_dev::kModeBits)
            for (const rfim_dev::Launch &lg : lanes[i].ln)
                for (int q = 0; q < m; ++q) {
                    const int e = exch && q == m - 1 && lanes[i].fused;
                    if (lanes[i].mode == 0) {
                        HIPCHK(rfim_dev::launch_stream_sweep(lg, 0, q, 0, qs[i % nq]));
                        HIPCHK(rfim_dev::launch_stream_sweep(lg, 1, q, e, qs[i % nq]));
                    } else {
                        HIPCHK(rfim_dev::launch_bits_batch(lg, 0, q, 0, qs[i % nq]));
                        HIPCHK(rfim_dev::launch_bits_batch(lg, 1, q, e, qs[i % nq]));
                    }
                }
    for (int j = 0; j < nside; ++j) {
        HIPCHK(hipEventRecord(b->ev_join[j], b->aux[j]));
        HIPCHK(hipStreamWaitEvent(b->stream, b->ev_join[j], 0));
    }
    if (exch) {
        // classes whose sweeps do not write energy partials: the separate
        // energy kernel, per item, once every lane has joined
        for (const auto &c : b->classes)
            if (!class_fused(b, c))
                for (int i : c.members) HIPCHK(rfim_dev::launch_energy(b->items[i]->lattice(), b->stream));
        HIPCHK(rfim_dev::launch_exchange(b->d_lats, (int)b->items.size(), m, b->stream));
        for (rfim *h : b->items) {
            int rc;
            if ((rc = measure_after_exchange(h, b->stream))) return rc;
        }
    } else {
        for (rfim *h : b->items) HIPCHK(rfim_dev::launch_advance(h->lattice(), m, b->stream));
    }
    return RFIM_OK;
}

// A graph replays an interval's launches without their host cost, which
// matters when the launches are short; when every launch is long the host
// keeps ahead anyway, and eager launches on the batch's own lane streams
// (each with a hardware queue of its own) also keep concurrent lanes
// apart, which a replayed graph's parallel branches did not always do
// (measured: the first graph of a process ran the two lanes of a 16 x
// R=128, L=64 class one after the other, 1400 against 1590 attempts/ns).
// Eager when the interval's launches average at least 2^26 attempts (tens
// of microseconds each); below that the graph's lower per-launch cost wins
// (256 realizations of L <= 32: 489 against 448 realizations/s).
constexpr long long kEagerAttemptsPerLaunch = 1ll << 26;

bool batch_prefers_graph(const rfim_batch *b, int every) {
    long long attempts = 0, launches = 1;       // the exchange step
    std::vector<Lane> lanes;
    for (const auto &c : b->classes) {
        long long per_sweep = 0;
        for (int i : c.members) per_sweep += (long long)b->items[i]->R * b->items[i]->N;
        attempts += per_sweep * every;
        lanes.clear();
        class_lanes(b, c, lanes);
        for (const Lane &l : lanes) launches += l.mode == 1 ? 1 : 2ll * every * (long long)l.ln.size();
    }
    return attempts < kEagerAttemptsPerLaunch * launches;
}

int batch_capture(rfim_batch *b, int every) {
    if (b->graph) {
        HIPCHK(hipGraphExecDestroy(b->graph));
        b->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    int rc0;
    // side streams and events exist before the capture starts
    if ((rc0 = ensure_side_streams(b, kMaxSideStreams))) return rc0;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = batch_segment(b, every, true);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(RFIM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(RFIM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    b->graph_every = every;
    return RFIM_OK;
}

void note_advance(rfim_batch *b, int m, bool exch) {
    b->t += (uint64_t)m;
    if (exch) b->k += 1;
    for (rfim *h : b->items) {
        h->t = b->t;
        h->k = b->k;
    }
}

}  // namespace

extern "C" {

rfim_batch_t *rfim_batch_create(int n, const rfim_params_t *items, void *hip_stream) {
    if (n < 1 || n > 65536 || !items) {
        fail(RFIM_EINVAL, "need 1 <= n <= 65536 items");
        return nullptr;
    }
    for (int i = 0; i < n; ++i) {
        int kind;
        if (validate(&items[i], &kind)) {
            std::string msg = g_error;
            fail(RFIM_EINVAL, "item %d: %s", i, msg.c_str());
            return nullptr;
        }
        const int L = items[i].L;
        if (!(L >= 8 && (L & (L - 1)) == 0)) {
            fail(RFIM_EINVAL, "item %d: batches need L a power of two >= 8 (got %d)", i, L);
            return nullptr;
        }
    }
    rfim_batch *b = new (std::nothrow) rfim_batch();
    if (!b) {
        fail(RFIM_ENOMEM, "out of host memory");
        return nullptr;
    }
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            fail(RFIM_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
            delete b;
            return nullptr;
        }
        b->own_stream = true;
    }
    for (int i = 0; i < n; ++i) {
        int err = 0;
        rfim *h = create_impl(&items[i], b->stream, &err);
        if (!h) {
            batch_free(b);
            return nullptr;
        }
        h->in_batch = true;
        b->items.push_back(h);
        if (init_device(h)) {
            std::string msg = g_error;
            batch_free(b);
            fail(RFIM_ENOMEM, "item %d: %s", i, msg.c_str());
            return nullptr;
        }
        // one class per (L, field kind), default shape of the class
        int ci = -1;
        for (size_t c = 0; c < b->classes.size(); ++c)
            if (b->classes[c].L == h->L && b->classes[c].kind == h->kind) ci = (int)c;
        if (ci < 0) {
            rfim_batch::Class c;
            c.L = h->L;
            c.kind = h->kind;
            c.mode = h->mode;
            c.nw = h->nw;
            c.wg = h->wg;
            b->classes.push_back(c);
            ci = (int)b->classes.size() - 1;
        }
        auto &c = b->classes[ci];
        c.members.push_back(i);
        h->mode = c.mode;
        h->nw = c.nw;
        h->wg = c.wg;
        h->nblk = rfim_dev::blocks_per_replica(h->L, c.mode, c.nw, c.wg);
    }
    // classes at L = 64..256 start in bit storage, as single realizations
    // do there (if its arrays cannot be had a class keeps byte spins)
    for (auto &c : b->classes)
        if (rfim_dev::bits_valid(c.L) && class_apply_shape(b, c, rfim_dev::kModeBits, 0, 0) != RFIM_OK) {
            (void)hipGetLastError();
            g_error.clear();
        }
    hipError_t e = hipMalloc((void **)&b->d_lats, n * sizeof(Lattice));
    if (e != hipSuccess) {
        batch_free(b);
        fail(RFIM_ENOMEM, "hipMalloc(batch descriptors): %s", hipGetErrorString(e));
        return nullptr;
    }
    if (batch_build(b)) {
        std::string msg = g_error;
        batch_free(b);
        g_error = msg;
        return nullptr;
    }
    return b;
}

void rfim_batch_destroy(rfim_batch_t *b) { batch_free(b); }

int rfim_batch_size(const rfim_batch_t *b) { return b ? (int)b->items.size() : fail(RFIM_EINVAL, "batch is NULL"); }

rfim_t *rfim_batch_item(rfim_batch_t *b, int i) {
    if (!b || i < 0 || i >= (int)b->items.size()) {
        fail(RFIM_EINVAL, "no such batch item");
        return nullptr;
    }
    return b->items[i];
}

int rfim_batch_set_shape(rfim_batch_t *b, int L, int field_kind, int mode, int nw, int wg) {
    if (!b) return fail(RFIM_EINVAL, "batch is NULL");
    int rc = check_class_shape(L, mode, nw, wg);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(b->stream));
    for (auto &c : b->classes) {
        if (c.L != L || c.kind != field_kind) continue;
        if ((rc = class_apply_shape(b, c, mode, nw, wg))) {
            const std::string msg = g_error;
            (void)batch_build(b);
            g_error = msg;
            return rc;
        }
    }
    return batch_build(b);
}

int rfim_batch_set_group_bytes(rfim_batch_t *b, int64_t bytes) {
    if (!b) return fail(RFIM_EINVAL, "batch is NULL");
    if (bytes != 0 && bytes < (1ll << 20)) return fail(RFIM_EINVAL, "group budget must be 0 or at least 1 MiB");
    HIPCHK(hipStreamSynchronize(b->stream));
    b->group_bytes = bytes;
    if (b->graph) {                 // the lanes change: capture again
        HIPCHK(hipGraphExecDestroy(b->graph));
        b->graph = nullptr;
        b->graph_every = 0;
    }
    return RFIM_OK;
}

int64_t rfim_batch_get_group_bytes(const rfim_batch_t *b) {
    if (!b) return fail(RFIM_EINVAL, "batch is NULL");
    return b->group_bytes;
}

int rfim_batch_sweep(rfim_batch_t *b, int64_t n, int exchange_every) {
    if (!b) return fail(RFIM_EINVAL, "batch is NULL");
    if (n < 0 || exchange_every < 0) return fail(RFIM_EINVAL, "n and exchange_every must be >= 0");
    if (b->t + (uint64_t)n > kMaxSweeps) return fail(RFIM_ECAP, "global sweep counter would pass 2^31-1");
    int64_t remaining = n;
    const int every = exchange_every;
    while (remaining > 0) {
        const int64_t to_next = every > 0 ? (int64_t)(every - (int64_t)(b->t % (uint64_t)every)) : remaining;
        const int m = (int)std::min<int64_t>(remaining, to_next);
        const bool exch = every > 0 && m == to_next;
        int rc;
        if (exch && m == every && batch_prefers_graph(b, every)) {
            std::vector<int> flags(b->items.size());
            for (size_t q = 0; q < b->items.size(); ++q) flags[q] = b->items[q]->measure;
            if (b->graph_every != every || b->graph_measure != flags) {
                if ((rc = batch_capture(b, every))) return rc;
                b->graph_measure = flags;
            }
            HIPCHK(hipGraphLaunch(b->graph, b->stream));
        } else if ((rc = batch_segment(b, m, exch))) {
            return rc;
        }
        note_advance(b, m, exch);
        remaining -= m;
    }
    return RFIM_OK;
}

int rfim_batch_synchronize(rfim_batch_t *b) {
    if (!b) return fail(RFIM_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->stream));
    return RFIM_OK;
}

}  // extern "C"

// ===================================================================
// Pools: a batch whose membership changes while it runs (continuous
// batching).  Realizations are admitted against a device-memory budget,
// advance together in quanta of whole exchange intervals (each with its own
// sweep and exchange counters), can run an adaptive insertion step in place
// between quanta, and are released when done.
// ===================================================================
struct rfim_pool {
    rfim_batch core;                    // stepped items (compacted), classes, descriptors
    std::vector<rfim *> slots;          // slot id -> item (nullptr when free)
    std::vector<size_t> slot_bytes;
    // Per slot, the schedule of a job admitted with rfim_pool_admit_job
    // (Sec. 4: trial runs with an insertion step after each, then the
    // production sweeps) and its progress.  Slots admitted with
    // rfim_pool_admit have none and are driven by the caller.
    struct Job {
        bool scheduled = false, finished = false;
        int trials = 0, trials_done = 0, max_insert = 0, R_cap = 0;
        int64_t S = 0, P = 0;           // sweeps per trial, production sweeps
        double threshold = 0.0;
        int64_t done = 0;               // sweeps run since admission
        uint64_t attempts = 0;          // spin-flip attempts issued
    };
    std::vector<Job> jobs;
    size_t budget = 0, reserved = 0;
    size_t lats_cap = 0;
    bool dirty = true;
    struct Shape { int L, kind, mode, nw, wg; };
    std::vector<Shape> shapes;          // per (L, kind) once seen or set
};

namespace {

// Device bytes one realization reserves: what alloc_device allocates and,
// at the L that bit storage takes, the bit arrays a bit-storage class
// shape adds (the spin bits and the fields in the bit sweep's order).
size_t device_bytes(int L, int R_cap, int kind) {
    size_t n = arena_layout(L, R_cap, kind).total;
    if (rfim_dev::bits_valid(L)) {
        const size_t N = (size_t)L * L * L;
        n += (size_t)R_cap * N / 8 + (kind == 0 ? N / 8 : N * sizeof(float));
    }
    return n;
}

rfim_pool::Shape &pool_shape(rfim_pool *p, int L, int kind) {
    for (auto &s : p->shapes)
        if (s.L == L && s.kind == kind) return s;
    rfim_pool::Shape s{L, kind, 0, 0, 0};
    if (rfim_dev::bits_valid(L))
        s.mode = rfim_dev::kModeBits;       // bit storage, as for single realizations there
    else
        default_shape(L, 0, &s.mode, &s.nw, &s.wg);
    p->shapes.push_back(s);
    return p->shapes.back();
}

int pool_apply_shape(rfim_pool *p, rfim *h) {
    const rfim_pool::Shape &s = pool_shape(p, h->L, h->kind);
    if (h->mode == s.mode && h->nw == s.nw && h->wg == s.wg) return RFIM_OK;
    return item_apply_shape(h, s.mode, s.nw, s.wg);
}

// Compact the active items, regroup them into classes and rebuild the
// descriptor table and the workgroup maps.
int pool_build(rfim_pool *p) {
    rfim_batch &b = p->core;
    b.items.clear();
    for (size_t q = 0; q < p->slots.size(); ++q)
        if (p->slots[q] && !p->jobs[q].finished) b.items.push_back(p->slots[q]);
    std::vector<rfim_batch::Class> old;
    old.swap(b.classes);
    for (int i = 0; i < (int)b.items.size(); ++i) {
        rfim *h = b.items[i];
        int rc = pool_apply_shape(p, h);
        if (rc) return rc;
        int ci = -1;
        for (size_t c = 0; c < b.classes.size(); ++c)
            if (b.classes[c].L == h->L && b.classes[c].kind == h->kind) ci = (int)c;
        if (ci < 0) {
            rfim_batch::Class c;
            c.L = h->L;
            c.kind = h->kind;
            c.mode = h->mode;
            c.nw = h->nw;
            c.wg = h->wg;
            for (auto &o : old)           // reuse the class's map buffer
                if (o.L == c.L && o.kind == c.kind && o.d_map) {
                    c.d_map = o.d_map;
                    c.cap = o.cap;
                    o.d_map = nullptr;
                }
            b.classes.push_back(c);
            ci = (int)b.classes.size() - 1;
        }
        b.classes[ci].members.push_back(i);
    }
    for (auto &o : old)                   // classes with no members left
        if (o.d_map) b.classes.push_back(o), b.classes.back().members.clear(), b.classes.back().nblocks = 0;
    if (b.items.size() > p->lats_cap) {
        if (b.d_lats) HIPCHK(hipFree(b.d_lats));
        b.d_lats = nullptr;
        p->lats_cap = std::max<size_t>(64, 2 * b.items.size());
        hipError_t e = hipMalloc((void **)&b.d_lats, p->lats_cap * sizeof(Lattice));
        if (e != hipSuccess) {
            p->lats_cap = 0;
            return fail(RFIM_ENOMEM, "hipMalloc(pool descriptors): %s", hipGetErrorString(e));
        }
    }
    if (!b.items.empty()) {
        int rc = batch_build(&b);
        if (rc) return rc;
    }
    p->dirty = false;
    return RFIM_OK;
}

}  // namespace

extern "C" {

size_t rfim_pool_bytes_needed(const rfim_params_t *params) {
    int kind = 0;
    if (validate(params, &kind)) return 0;
    return device_bytes(params->L, params->R_cap == 0 ? params->R : params->R_cap, kind);
}

rfim_pool_t *rfim_pool_create(size_t hbm_budget_bytes, void *hip_stream) {
    rfim_pool *p = new (std::nothrow) rfim_pool();
    if (!p) {
        fail(RFIM_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->budget = hbm_budget_bytes;
    if (hip_stream) {
        p->core.stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&p->core.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            fail(RFIM_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
            delete p;
            return nullptr;
        }
        p->core.own_stream = true;
    }
    return p;
}

void rfim_pool_destroy(rfim_pool_t *p) {
    if (!p) return;
    // hand every live item, the class maps, the descriptors and the stream
    // to a batch record and free that
    rfim_batch *b = new (std::nothrow) rfim_batch();
    if (b) {
        b->stream = p->core.stream;
        b->own_stream = p->core.own_stream;
        b->d_lats = p->core.d_lats;
        b->classes = p->core.classes;
        b->aux = p->core.aux;
        b->ev_join = p->core.ev_join;
        b->ev_fork = p->core.ev_fork;
        for (rfim *h : p->slots)
            if (h) b->items.push_back(h);
        batch_free(b);
    }
    delete p;
}

namespace {

int pool_admit_impl(rfim_pool_t *p, const rfim_params_t *params, const rfim_pool::Job &job) {
    if (!p) return fail(RFIM_EINVAL, "pool is NULL");
    int kind = 0;
    int rc = validate(params, &kind);
    if (rc) return rc;
    if (!(params->L >= 8 && (params->L & (params->L - 1)) == 0))
        return fail(RFIM_EINVAL, "pools need L a power of two >= 8 (got %d)", params->L);
    const int R_cap = params->R_cap == 0 ? params->R : params->R_cap;
    const size_t need = device_bytes(params->L, R_cap, kind);
    if (p->reserved + need > p->budget)
        return fail(RFIM_EBUSY, "budget: %zu reserved + %zu needed > %zu", p->reserved, need, p->budget);
    int err = 0;
    rfim *h = create_impl(params, p->core.stream, &err);
    if (!h) return err ? err : RFIM_EINVAL;
    h->in_batch = true;
    if ((rc = init_device(h)) || (rc = pool_apply_shape(p, h))) {
        std::string msg = g_error;
        h->stream = nullptr;
        free_device(h);
        delete h;
        g_error = msg;
        return rc;
    }
    int slot = -1;
    for (size_t s = 0; s < p->slots.size(); ++s)
        if (!p->slots[s]) {
            slot = (int)s;
            break;
        }
    if (slot < 0) {
        slot = (int)p->slots.size();
        p->slots.push_back(nullptr);
        p->slot_bytes.push_back(0);
        p->jobs.emplace_back();
    }
    p->slots[slot] = h;
    p->slot_bytes[slot] = need;
    p->jobs[slot] = job;
    p->reserved += need;
    p->dirty = true;
    return slot;
}

}  // namespace

int rfim_pool_admit(rfim_pool_t *p, const rfim_params_t *params) {
    return pool_admit_impl(p, params, rfim_pool::Job());
}

int rfim_pool_admit_job(rfim_pool_t *p, const rfim_job_t *job) {
    if (!p || !job) return fail(RFIM_EINVAL, "NULL argument");
    const rfim_params_t &prm = job->params;
    const int R_cap = prm.R_cap == 0 ? prm.R : prm.R_cap;
    if (job->trials < 0 || job->max_insert_per_trial < 0 || std::isnan(job->rate_threshold))
        return fail(RFIM_EINVAL, "bad job schedule: trials, max_insert_per_trial must be >= 0");
    if (job->trials > 0 && job->sweeps_per_trial < 1)
        return fail(RFIM_EINVAL, "bad job schedule: a trial run needs sweeps_per_trial >= 1");
    if (job->production_sweeps < 1) return fail(RFIM_EINVAL, "bad job schedule: production_sweeps must be >= 1");
    if ((uint64_t)job->trials * (uint64_t)std::max<int64_t>(job->sweeps_per_trial, 0) +
            (uint64_t)job->production_sweeps > kMaxSweeps)
        return fail(RFIM_ECAP, "job schedule passes the sweep counter limit 2^31-1");
    rfim_pool::Job j;
    j.scheduled = true;
    j.trials = job->trials;
    j.S = job->trials > 0 ? job->sweeps_per_trial : 0;
    j.P = job->production_sweeps;
    j.threshold = job->rate_threshold;
    j.max_insert = job->max_insert_per_trial;
    j.R_cap = R_cap;
    return pool_admit_impl(p, &prm, j);
}

int rfim_pool_release(rfim_pool_t *p, int slot) {
    if (!p || slot < 0 || slot >= (int)p->slots.size() || !p->slots[slot])
        return fail(RFIM_EINVAL, "no such pool slot");
    rfim *h = p->slots[slot];
    HIPCHK(hipStreamSynchronize(p->core.stream));
    h->stream = nullptr;
    free_device(h);
    delete h;
    p->slots[slot] = nullptr;
    p->jobs[slot] = rfim_pool::Job();
    p->reserved -= p->slot_bytes[slot];
    p->slot_bytes[slot] = 0;
    p->dirty = true;
    return RFIM_OK;
}

rfim_t *rfim_pool_item(rfim_pool_t *p, int slot) {
    if (!p || slot < 0 || slot >= (int)p->slots.size() || !p->slots[slot]) {
        fail(RFIM_EINVAL, "no such pool slot");
        return nullptr;
    }
    return p->slots[slot];
}

int rfim_pool_active(const rfim_pool_t *p) {
    if (!p) return fail(RFIM_EINVAL, "pool is NULL");
    int n = 0;
    for (rfim *h : p->slots) n += h != nullptr;
    return n;
}

size_t rfim_pool_reserved(const rfim_pool_t *p) { return p ? p->reserved : 0; }

int rfim_pool_set_shape(rfim_pool_t *p, int L, int field_kind, int mode, int nw, int wg) {
    if (!p) return fail(RFIM_EINVAL, "pool is NULL");
    int rc = check_class_shape(L, mode, nw, wg);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(p->core.stream));
    rfim_pool::Shape &s = pool_shape(p, L, field_kind);
    s.mode = mode;
    s.nw = nw;
    s.wg = wg;
    p->dirty = true;
    return RFIM_OK;
}

int rfim_pool_step(rfim_pool_t *p, int quantum, int exchange_every) {
    if (!p) return fail(RFIM_EINVAL, "pool is NULL");
    if (exchange_every < 1 || quantum < 1 || quantum % exchange_every)
        return fail(RFIM_EINVAL, "quantum must be a positive multiple of exchange_every >= 1");
    for (size_t q = 0; q < p->slots.size(); ++q) {
        const rfim *h = p->slots[q];
        const rfim_pool::Job &j = p->jobs[q];
        if (!h || j.finished) continue;
        if (h->t % (uint64_t)exchange_every)
            return fail(RFIM_ESTATE, "a pool item is not at an exchange boundary");
        if (h->t + (uint64_t)quantum > kMaxSweeps) return fail(RFIM_ECAP, "sweep counter would pass 2^31-1");
        if (j.scheduled) {
            // the job's next boundary (end of a trial run, or of the
            // production sweeps) must fall on a quantum boundary
            const int64_t next = j.trials_done < j.trials ? (int64_t)(j.trials_done + 1) * j.S
                                                          : (int64_t)j.trials * j.S + j.P;
            if ((next - j.done) % quantum)
                return fail(RFIM_EINVAL, "slot %zu: its schedule boundary at sweep %lld is not a multiple of the "
                            "quantum %d from sweep %lld", q, (long long)next, quantum, (long long)j.done);
        }
    }
    int rc;
    if (p->dirty && (rc = pool_build(p))) return rc;
    if (p->core.items.empty()) return RFIM_OK;
    for (int q = 0; q < quantum / exchange_every; ++q) {
        if ((rc = batch_segment(&p->core, exchange_every, true))) return rc;
        for (rfim *h : p->core.items) {
            h->t += (uint64_t)exchange_every;
            h->k += 1;
        }
    }
    // progress of scheduled jobs: the insertion step at the end of each
    // trial run (Sec. 4), completion at the end of the production sweeps
    for (size_t q = 0; q < p->slots.size(); ++q) {
        rfim *h = p->slots[q];
        rfim_pool::Job &j = p->jobs[q];
        if (!h || j.finished) continue;
        j.attempts += (uint64_t)h->R * (uint64_t)h->N * (uint64_t)quantum;
        if (!j.scheduled) continue;
        j.done += quantum;
        if (j.trials_done < j.trials && j.done == (int64_t)(j.trials_done + 1) * j.S) {
            const int R0 = h->R;
            if ((rc = insert_step(h, j.threshold, j.max_insert, j.R_cap)) < 0) return rc;
            if (rc != R0) p->dirty = true;
            ++j.trials_done;
        }
        if (j.trials_done == j.trials && j.done == (int64_t)j.trials * j.S + j.P) {
            j.finished = true;
            p->dirty = true;
        }
    }
    return RFIM_OK;
}

int rfim_pool_poll(rfim_pool_t *p, int *done, int max) {
    if (!p) return fail(RFIM_EINVAL, "pool is NULL");
    if (max < 0 || (max > 0 && !done)) return fail(RFIM_EINVAL, "done must hold max >= 0 slot ids");
    int n = 0;
    for (size_t q = 0; q < p->slots.size(); ++q)
        if (p->slots[q] && p->jobs[q].finished) {
            if (n < max) done[n] = (int)q;
            ++n;
        }
    return max == 0 ? n : std::min(n, max);
}

int rfim_pool_result(rfim_pool_t *p, int slot, rfim_result_t *res) {
    if (!p || slot < 0 || slot >= (int)p->slots.size() || !p->slots[slot])
        return fail(RFIM_EINVAL, "no such pool slot");
    if (!res) return fail(RFIM_EINVAL, "result is NULL");
    rfim *h = p->slots[slot];
    const rfim_pool::Job &j = p->jobs[slot];
    res->R = h->R;
    res->finished = j.finished ? 1 : 0;
    res->attempts = j.attempts;
    const bool arrays = res->temps || res->energies || res->magnetizations || res->perm;
    if (arrays && res->capacity < h->R)
        return fail(RFIM_ECAP, "result arrays hold %d entries, the slot has %d replicas", res->capacity, h->R);
    HIPCHK(hipStreamSynchronize(p->core.stream));
    res->sweeps = h->t;
    res->exchanges = h->k;
    int rc;
    if (res->temps) std::copy(h->T.begin(), h->T.end(), res->temps);
    if (res->energies && (rc = rfim_energies(h, res->energies))) return rc;
    if (res->magnetizations && (rc = rfim_magnetizations(h, res->magnetizations))) return rc;
    if (res->perm && (rc = rfim_get_perm(h, res->perm))) return rc;
    return RFIM_OK;
}

int rfim_pool_adapt(rfim_pool_t *p, int slot, double rate_threshold, int max_insert, int R_cap) {
    rfim *h = rfim_pool_item(p, slot);
    if (!h) return RFIM_EINVAL;
    if (p->jobs[slot].scheduled) return fail(RFIM_ESTATE, "slot %d runs its own schedule (rfim_pool_admit_job)", slot);
    if (max_insert < 0 || std::isnan(rate_threshold)) return fail(RFIM_EINVAL, "bad adapt arguments");
    if (R_cap > h->R_cap) return fail(RFIM_ECAP, "R_cap %d beyond the capacity %d given at admit", R_cap, h->R_cap);
    const int R0 = h->R;
    const int rc = insert_step(h, rate_threshold, max_insert, R_cap);
    if (rc < 0) return rc;
    if (rc != R0) p->dirty = true;
    return rc;
}

int rfim_pool_synchronize(rfim_pool_t *p) {
    if (!p) return fail(RFIM_EINVAL, "pool is NULL");
    HIPCHK(hipStreamSynchronize(p->core.stream));
    return RFIM_OK;
}

}  // extern "C"
