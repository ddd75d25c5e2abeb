/*
 * rfim_oracle.c -- plain single-threaded CPU oracle (TEST INFRASTRUCTURE
 * ONLY; see rfim_oracle.h).  Written for readability, not speed: every step
 * follows the paper's description in the paper's order, with the
 * conventions the paper leaves open written out where they are used.
 *
 * Compiled with -ffp-contract=off so that every floating-point expression is
 * evaluated exactly as written (no fused multiply-add).
 *
 * Conventions (the paper names no random number generator, no colour order,
 * no acceptance precision):
 *
 *  Lattice.  L even, N = L^3, site i = x + L*(y + L*z), periodic neighbours
 *  (x+-1, y, z), (x, y+-1, z), (x, y, z+-1).  Colour c(i) = (x+y+z) mod 2
 *  (Eq. 3).  Sublattice index j = i >> 1: for even L the pair {2j, 2j+1}
 *  holds exactly one site of each colour.
 *
 *  Random numbers.  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *  key = (lo32(seed), hi32(seed)), counter word 3 = (tag << 28) | rho where
 *  rho is the realization id (< 2^28).
 *    tag 1, initial spins:   ctr = (i >> 2, 0, r, .), word i & 3,
 *                            s = +1 iff word >= 2^31.
 *    tag 2, sweep t colour c: ctr = (j >> 2, 2t + c, r, .), word j & 3.
 *    tag 3, exchange step k:  ctr = (p, k, 0, .) for the pair (p, p+1),
 *                            U53 = ((w0 >> 11) * 2^32 + w1) * 2^-53.
 *
 *  Double checkerboard with multi-hit updates (optional order, Sec. 3.2 and
 *  Sec. 5.2; see tile_visits below): sweep t, local sweep (hit) m of a
 *  tile visit, site of colour c: tag 2, ctr = (j >> 2, 2 (t hits + m) + c,
 *  r, .), word j & 3 -- with hits = 1 the words of the plain sweep t.
 *
 *  Metropolis (Sec. 2, Sec. 3.1 step 4; textbook rule min(1, e^{-b dE})).
 *    dE = 2 s_i (J n_i + h h_i), n_i = sum of the six neighbour spins.
 *    Bimodal fields: classes (a, b) = (s_i n_i, s_i h_i); a uint32 threshold
 *    thr = min(floor(exp(-beta dE) * 2^32), 2^32 - 1) per temperature slot
 *    and class, built in FP64; accept iff dE <= 0 or u32 < thr.
 *    Continuous fields: dE in FP64; accept iff dE <= 0 or
 *    (double)u32 < exp(-beta dE) * 2^32.
 *
 *  Exchange (Sec. 3.1, Eq. 2; Sec. 3.3).  After every `every`-th sweep
 *  (global count), energies are recomputed from scratch; for every slot p
 *  with p = k (mod 2) and p + 1 < R: a = t2r[p], b = t2r[p+1],
 *  Delta = (beta_{p+1} - beta_p)(E_b - E_a); accept iff Delta >= 0 or
 *  U53 < exp(Delta); on accept swap t2r[p], t2r[p+1] and fix r2t.  k += 1.
 *
 *  Energy (Eq. 1): B = sum_i sum_{mu=x,y,z} s_i s_{i+mu} (3N forward bonds),
 *  F = sum_i h_i s_i, E = -(J*B) - (h*F).  B, F exact integers for bimodal
 *  fields; F a sequential FP64 sum for continuous fields.
 */
#include "rfim_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define TAG_INIT 1u
#define TAG_SWEEP 2u
#define TAG_EXCH 3u

struct orc {
    int L, N, R, R_cap;
    double J, h;
    int kind;               /* 0 bimodal, 1 continuous */
    uint64_t seed;
    uint32_t rho;
    float *f;               /* [N] fields as given */
    int8_t *fs;             /* [N] sign of field (bimodal) */
    int32_t *nb;            /* [N][6] neighbour site indices */
    int8_t *s;              /* [R_cap][N] spins by replica id */
    double *T;              /* [R_cap] temperature of slot */
    double *beta;           /* [R_cap] 1/T of slot */
    int32_t *t2r, *r2t;     /* [R_cap] */
    uint64_t t, k;          /* global sweep and exchange counters */
    uint64_t *att, *acc;    /* [R_cap] per lower slot of a pair */
    uint32_t *thr;          /* [R_cap][14] (bimodal) */
    uint8_t always[14];
    /* update order: 0 plain two-colour checkerboard; 1 double checkerboard
     * of tx * ty * tz tiles with `hits` local sweeps per tile visit */
    int order, tx, ty, tz, hits;
};

static char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition: ten rounds of two     */
/* 32x32->64 multiplications by fixed odd constants, with a Weyl       */
/* sequence key schedule.                                              */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t philox_word(const orc_t *o, uint32_t tag, uint32_t c0,
                            uint32_t c1, uint32_t c2, int word) {
    uint32_t ctr[4] = {c0, c1, c2, (tag << 28) | o->rho};
    uint32_t key[2] = {(uint32_t)o->seed, (uint32_t)(o->seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word];
}

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */
static int site_x(const orc_t *o, int i) { return i % o->L; }
static int site_y(const orc_t *o, int i) { return (i / o->L) % o->L; }
static int site_z(const orc_t *o, int i) { return i / (o->L * o->L); }
static int site_of(const orc_t *o, int x, int y, int z) {
    int L = o->L;
    x = (x + L) % L; y = (y + L) % L; z = (z + L) % L;
    return x + L * (y + L * z);
}
static int colour(const orc_t *o, int i) {
    return (site_x(o, i) + site_y(o, i) + site_z(o, i)) & 1;
}
/* The site of colour c in pair j = {2j, 2j+1}. */
static int site_of_pair(const orc_t *o, int j, int c) {
    int i0 = 2 * j;
    return colour(o, i0) == c ? i0 : i0 + 1;
}

/* ------------------------------------------------------------------ */
/* Acceptance thresholds (bimodal fields)                              */
/* ------------------------------------------------------------------ */
static double class_delta_e(const orc_t *o, int cls) {
    int k = cls >> 1, fb = cls & 1;
    int a = 2 * k - 6;      /* s_i * n_i */
    int b = 2 * fb - 1;     /* s_i * h_i */
    return 2.0 * (o->J * (double)a + o->h * (double)b);
}

static uint32_t threshold(double beta, double dE) {
    double p = exp(-(beta * dE));
    double scaled = ldexp(p, 32);
    if (scaled >= 4294967295.0) return 4294967295u;
    return (uint32_t)floor(scaled);
}

static void build_tables(orc_t *o) {
    for (int c = 0; c < 14; ++c) o->always[c] = class_delta_e(o, c) <= 0.0;
    for (int t = 0; t < o->R; ++t) {
        o->beta[t] = 1.0 / o->T[t];
        for (int c = 0; c < 14; ++c)
            o->thr[t * 14 + c] = o->always[c] ? 0xFFFFFFFFu
                                              : threshold(o->beta[t], class_delta_e(o, c));
    }
}

/* ------------------------------------------------------------------ */
/* Creation                                                            */
/* ------------------------------------------------------------------ */
orc_t *orc_create(int L, int R, double J, double h, const float *fields,
                  const double *temps, uint64_t seed, uint32_t realization,
                  int field_kind, int R_cap) {
    /* L <= 512: the neighbour table alone takes 24 N bytes (3.2 GB at
     * L = 512); larger lattices are replayed site by site in the tests */
    if (L < 2 || L > 512 || (L & 1)) { set_err("L must be even, 2..512"); return NULL; }
    if (R_cap == 0) R_cap = R;
    if (R < 1 || R_cap < R) { set_err("need 1 <= R <= R_cap"); return NULL; }
    if (!fields || !temps) { set_err("null input"); return NULL; }
    if (!isfinite(J) || !isfinite(h)) { set_err("J, h must be finite"); return NULL; }
    if (realization >= (1u << 28)) { set_err("realization id must be < 2^28"); return NULL; }
    for (int t = 0; t < R; ++t) {
        if (!isfinite(temps[t]) || temps[t] <= 0.0) { set_err("temps must be finite and > 0"); return NULL; }
        if (t > 0 && !(temps[t] > temps[t - 1])) { set_err("temps must be strictly ascending"); return NULL; }
    }
    int N = L * L * L;
    int bimodal = 1;
    for (int i = 0; i < N; ++i) {
        if (!isfinite(fields[i])) { set_err("fields must be finite"); return NULL; }
        if (fields[i] != 1.0f && fields[i] != -1.0f) bimodal = 0;
    }
    int kind = field_kind < 0 ? (bimodal ? 0 : 1) : field_kind;
    if (kind == 0 && !bimodal) { set_err("bimodal kind needs fields of +-1"); return NULL; }

    orc_t *o = (orc_t *)calloc(1, sizeof *o);
    o->L = L; o->N = N; o->R = R; o->R_cap = R_cap;
    o->J = J; o->h = h; o->kind = kind; o->seed = seed; o->rho = realization;
    o->f = (float *)malloc(sizeof(float) * (size_t)N);
    o->fs = (int8_t *)malloc((size_t)N);
    o->nb = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)N);
    o->s = (int8_t *)malloc((size_t)R_cap * (size_t)N);
    o->T = (double *)calloc((size_t)R_cap, sizeof(double));
    o->beta = (double *)calloc((size_t)R_cap, sizeof(double));
    o->t2r = (int32_t *)calloc((size_t)R_cap, sizeof(int32_t));
    o->r2t = (int32_t *)calloc((size_t)R_cap, sizeof(int32_t));
    o->att = (uint64_t *)calloc((size_t)R_cap, sizeof(uint64_t));
    o->acc = (uint64_t *)calloc((size_t)R_cap, sizeof(uint64_t));
    o->thr = (uint32_t *)calloc((size_t)R_cap * 14, sizeof(uint32_t));
    if (!o->f || !o->fs || !o->nb || !o->s || !o->T || !o->beta || !o->t2r ||
        !o->r2t || !o->att || !o->acc || !o->thr) {
        set_err("out of memory");
        orc_destroy(o);
        return NULL;
    }
    for (int i = 0; i < N; ++i) {
        o->f[i] = fields[i];
        o->fs[i] = fields[i] > 0.0f ? 1 : -1;
        int x = site_x(o, i), y = site_y(o, i), z = site_z(o, i);
        o->nb[6 * (size_t)i + 0] = site_of(o, x + 1, y, z);
        o->nb[6 * (size_t)i + 1] = site_of(o, x - 1, y, z);
        o->nb[6 * (size_t)i + 2] = site_of(o, x, y + 1, z);
        o->nb[6 * (size_t)i + 3] = site_of(o, x, y - 1, z);
        o->nb[6 * (size_t)i + 4] = site_of(o, x, y, z + 1);
        o->nb[6 * (size_t)i + 5] = site_of(o, x, y, z - 1);
    }
    for (int t = 0; t < R; ++t) {
        o->T[t] = temps[t];
        o->t2r[t] = t;
        o->r2t[t] = t;
    }
    build_tables(o);
    /* Step 3 of the method: an arbitrary starting configuration per replica,
     * here drawn from the INIT stream. */
    for (int r = 0; r < R; ++r)
        for (int i = 0; i < N; ++i) {
            uint32_t w = philox_word(o, TAG_INIT, (uint32_t)(i >> 2), 0u, (uint32_t)r, i & 3);
            o->s[(size_t)r * N + i] = w >= 0x80000000u ? 1 : -1;
        }
    return o;
}

void orc_destroy(orc_t *o) {
    if (!o) return;
    free(o->f); free(o->fs); free(o->nb); free(o->s); free(o->T); free(o->beta);
    free(o->t2r); free(o->r2t); free(o->att); free(o->acc); free(o->thr);
    free(o);
}

int orc_num_replicas(const orc_t *o) { return o->R; }
int orc_field_kind(const orc_t *o) { return o->kind; }

/* ------------------------------------------------------------------ */
/* Energy (Eq. 1)                                                      */
/* ------------------------------------------------------------------ */
static void replica_components(const orc_t *o, int r, int64_t *B, double *F,
                               int64_t *Fi, int64_t *M) {
    const int8_t *s = o->s + (size_t)r * o->N;
    int64_t bonds = 0, mag = 0, fint = 0;
    double fsum = 0.0;
    for (int i = 0; i < o->N; ++i) {
        /* forward bonds +x, +y, +z: each bond once */
        bonds += (int64_t)s[i] * s[o->nb[6 * (size_t)i + 0]];
        bonds += (int64_t)s[i] * s[o->nb[6 * (size_t)i + 2]];
        bonds += (int64_t)s[i] * s[o->nb[6 * (size_t)i + 4]];
        mag += s[i];
        fint += (int64_t)o->fs[i] * s[i];
        fsum += (double)o->f[i] * (double)s[i];
    }
    *B = bonds;
    *M = mag;
    *Fi = fint;
    *F = fsum;
}

static double replica_energy(const orc_t *o, int r) {
    int64_t B, Fi, M;
    double F;
    replica_components(o, r, &B, &F, &Fi, &M);
    double fpart = o->kind == 0 ? (double)Fi : F;
    return -(o->J * (double)B) - (o->h * fpart);
}

int orc_components(orc_t *o, int64_t *B, double *F, int64_t *M) {
    for (int r = 0; r < o->R; ++r) {
        int64_t b, fi, m;
        double f;
        replica_components(o, r, &b, &f, &fi, &m);
        B[r] = b;
        F[r] = o->kind == 0 ? (double)fi : f;
        M[r] = m;
    }
    return 0;
}

int orc_energies(orc_t *o, double *E) {
    for (int t = 0; t < o->R; ++t) E[t] = replica_energy(o, o->t2r[t]);
    return 0;
}

int orc_magnetizations(orc_t *o, int64_t *M) {
    for (int t = 0; t < o->R; ++t) {
        const int8_t *s = o->s + (size_t)o->t2r[t] * o->N;
        int64_t m = 0;
        for (int i = 0; i < o->N; ++i) m += s[i];
        M[t] = m;
    }
    return 0;
}

int orc_temps(const orc_t *o, double *T) {
    memcpy(T, o->T, sizeof(double) * (size_t)o->R);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Metropolis                                                          */
/* ------------------------------------------------------------------ */
static int neighbour_sum(const orc_t *o, const int8_t *s, int i) {
    int n = 0;
    for (int d = 0; d < 6; ++d) n += s[o->nb[6 * (size_t)i + d]];
    return n;
}

double orc_flip_delta(const orc_t *o, int r, int i) {
    const int8_t *s = o->s + (size_t)r * o->N;
    int si = s[i];
    int n = neighbour_sum(o, s, i);
    if (o->kind == 0) {
        int k = (si * n + 6) / 2;
        int fb = si * o->fs[i] > 0;
        return class_delta_e(o, 2 * k + fb);
    }
    double x = o->J * (double)n + o->h * (double)o->f[i];
    return 2.0 * (double)si * x;
}

/* One Metropolis decision for site i of replica r with random word u. */
static int accept_flip(const orc_t *o, const int8_t *s, int i, int slot, uint32_t u) {
    int si = s[i];
    int n = neighbour_sum(o, s, i);
    if (o->kind == 0) {
        int k = (si * n + 6) / 2;                 /* aligned neighbour slots */
        int fb = si * o->fs[i] > 0;               /* field aligned with spin */
        int cls = 2 * k + fb;
        if (o->always[cls]) return 1;
        return u < o->thr[slot * 14 + cls];
    }
    double x = o->J * (double)n + o->h * (double)o->f[i];
    double dE = 2.0 * (double)si * x;
    if (dE <= 0.0) return 1;
    double p = exp(-(o->beta[slot] * dE));
    return (double)u < ldexp(p, 32);
}

/* ------------------------------------------------------------------ */
/* Fourier observable of the correlation length (Sec. 7): at the       */
/* smallest nonzero wave number K = 2 pi / L, per configuration        */
/*   F = (1/(3N)) sum_mu [(sum_i s_i cos(K x_mu,i))^2                  */
/*                        + (sum_i s_i sin(K x_mu,i))^2],              */
/* mu over the three axes.  The printed sums carry the field h_i, which */
/* would make F a constant of the disorder; read as s_i, the usual     */
/* second-moment estimator.  Each inner sum is grouped by the          */
/* coordinate: n_mu(v) = sum of s_i over the plane x_mu,i = v (exact   */
/* integers), then sum_v cos(K v) n_mu(v) in FP64 with v ascending.    */
/* ------------------------------------------------------------------ */
int orc_fourier(const orc_t *o, double *F) {
    const int L = o->L;
    int64_t *n = calloc((size_t)3 * L, sizeof(int64_t));
    double *ck = malloc(sizeof(double) * (size_t)L), *sk = malloc(sizeof(double) * (size_t)L);
    if (!n || !ck || !sk) {
        free(n); free(ck); free(sk);
        set_err("out of memory");
        return -1;
    }
    for (int v = 0; v < L; ++v) {
        ck[v] = cos(2.0 * 3.14159265358979323846 * (double)v / (double)L);
        sk[v] = sin(2.0 * 3.14159265358979323846 * (double)v / (double)L);
    }
    for (int t = 0; t < o->R; ++t) {
        const int8_t *s = o->s + (size_t)o->t2r[t] * o->N;
        memset(n, 0, sizeof(int64_t) * (size_t)3 * L);
        for (int i = 0; i < o->N; ++i) {
            const int x = i % L, y = (i / L) % L, z = i / (L * L);
            n[x] += s[i];
            n[L + y] += s[i];
            n[2 * L + z] += s[i];
        }
        double c[3], sn[3];
        for (int mu = 0; mu < 3; ++mu) {
            c[mu] = 0.0;
            sn[mu] = 0.0;
            for (int v = 0; v < L; ++v) {
                c[mu] += ck[v] * (double)n[mu * L + v];
                sn[mu] += sk[v] * (double)n[mu * L + v];
            }
        }
        F[t] = (c[0] * c[0] + sn[0] * sn[0] + c[1] * c[1] + sn[1] * sn[1] + c[2] * c[2] + sn[2] * sn[2]) /
               (3.0 * (double)o->N);
    }
    free(n); free(ck); free(sk);
    return 0;
}

int orc_accept(const orc_t *o, int r, int i, uint32_t u) {
    if (r < 0 || r >= o->R || i < 0 || i >= o->N) return -1;
    return accept_flip(o, o->s + (size_t)r * o->N, i, o->r2t[r], u);
}

static void half_sweep(orc_t *o, int c) {
    int half = o->N / 2;
    for (int r = 0; r < o->R; ++r) {
        int8_t *s = o->s + (size_t)r * o->N;
        int slot = o->r2t[r];
        /* four consecutive sublattice sites share one Philox block */
        for (int g = 0; g < half / 4; ++g) {
            uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(2 * o->t + (uint64_t)c), (uint32_t)r,
                               (TAG_SWEEP << 28) | o->rho};
            uint32_t key[2] = {(uint32_t)o->seed, (uint32_t)(o->seed >> 32)};
            uint32_t w[4];
            orc_philox4x32_10(ctr, key, w);
            for (int q = 0; q < 4; ++q) {
                int i = site_of_pair(o, 4 * g + q, c);
                if (accept_flip(o, s, i, slot, w[q])) s[i] = (int8_t)-s[i];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Double checkerboard with multi-hit updates (Sec. 3.2, Sec. 5.2)     */
/* ------------------------------------------------------------------ */
/* The lattice is cut into tiles of tx * ty * tz sites; tile (X, Y, Z) =  */
/* (x / tx, y / ty, z / tz) has the coarse colour (X + Y + Z) mod 2.     */
/* Sweep t visits every tile of coarse colour 0, then every tile of      */
/* coarse colour 1 (the paper's two kernel executions per sweep).  A     */
/* visited tile runs `hits` local sweeps of the fine checkerboard: its   */
/* sites of colour 0, then its sites of colour 1 (Eq. 3), each the       */
/* Metropolis update of the plain sweep.  With L / t_mu even, two tiles  */
/* of one coarse colour never share a face, so every neighbour outside   */
/* the visited tile lies in a tile of the other coarse colour and stays  */
/* as it is while the tile runs.  Site i in hit m takes word j & 3 of    */
/* the tag-2 block (j >> 2, 2 (t hits + m) + c(i), r).                   */
static void tile_visits(orc_t *o, int coarse) {
    const int L = o->L, Dx = L / o->tx, Dy = L / o->ty, Dz = L / o->tz;
    for (int r = 0; r < o->R; ++r) {
        int8_t *s = o->s + (size_t)r * o->N;
        int slot = o->r2t[r];
        for (int Z = 0; Z < Dz; ++Z)
            for (int Y = 0; Y < Dy; ++Y)
                for (int X = 0; X < Dx; ++X) {
                    if (((X + Y + Z) & 1) != coarse) continue;
                    for (int m = 0; m < o->hits; ++m) {
                        uint32_t step = (uint32_t)(o->t * (uint64_t)o->hits + (uint64_t)m);
                        for (int c = 0; c < 2; ++c)
                            for (int z = Z * o->tz; z < (Z + 1) * o->tz; ++z)
                                for (int y = Y * o->ty; y < (Y + 1) * o->ty; ++y)
                                    for (int x = X * o->tx; x < (X + 1) * o->tx; ++x) {
                                        int i = site_of(o, x, y, z);
                                        if (colour(o, i) != c) continue;
                                        int j = i >> 1;
                                        uint32_t u = philox_word(o, TAG_SWEEP, (uint32_t)(j >> 2),
                                                                 2u * step + (uint32_t)c, (uint32_t)r, j & 3);
                                        if (accept_flip(o, s, i, slot, u)) s[i] = (int8_t)-s[i];
                                    }
                    }
                }
    }
}

int orc_set_update_order(orc_t *o, int order, int tx, int ty, int tz, int hits) {
    if (order == 0) {
        o->order = 0;
        return 0;
    }
    if (order != 1) { set_err("order must be 0 (checkerboard) or 1 (tiles)"); return -1; }
    const int L = o->L;
    const int t[3] = {tx, ty, tz};
    for (int d = 0; d < 3; ++d)
        if (t[d] < 1 || L % t[d] != 0 || ((L / t[d]) & 1)) {
            set_err("each tile side must divide L into an even number of tiles");
            return -1;
        }
    if (hits < 1) { set_err("hits must be >= 1"); return -1; }
    o->order = 1;
    o->tx = tx; o->ty = ty; o->tz = tz; o->hits = hits;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Exchange (Eq. 2, temperatures swapped as in Sec. 3.3)               */
/* ------------------------------------------------------------------ */
int orc_exchange_once(orc_t *o) {
    double *E = (double *)malloc(sizeof(double) * (size_t)o->R);
    for (int r = 0; r < o->R; ++r) E[r] = replica_energy(o, r);
    for (int p = (int)(o->k & 1); p + 1 < o->R; p += 2) {
        int a = o->t2r[p], b = o->t2r[p + 1];
        double delta = (o->beta[p + 1] - o->beta[p]) * (E[b] - E[a]);
        uint32_t ctr[4] = {(uint32_t)p, (uint32_t)o->k, 0u, (TAG_EXCH << 28) | o->rho};
        uint32_t key[2] = {(uint32_t)o->seed, (uint32_t)(o->seed >> 32)};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        double u53 = ldexp((double)(w[0] >> 11) * 4294967296.0 + (double)w[1], -53);
        o->att[p] += 1;
        if (delta >= 0.0 || u53 < exp(delta)) {
            o->t2r[p] = b;
            o->t2r[p + 1] = a;
            o->r2t[a] = p + 1;
            o->r2t[b] = p;
            o->acc[p] += 1;
        }
    }
    o->k += 1;
    free(E);
    return 0;
}

int orc_sweep(orc_t *o, int64_t n, int every) {
    if (n < 0 || every < 0) { set_err("n and every must be >= 0"); return -1; }
    if (o->t + (uint64_t)n > 0x7FFFFFFFull) { set_err("sweep counter limit 2^31-1"); return -5; }
    if (o->order == 1 && (o->t + (uint64_t)n) * (uint64_t)o->hits > 0x80000000ull) {
        set_err("sweep counter limit: (t + n) * hits must stay <= 2^31");
        return -5;
    }
    for (int64_t q = 0; q < n; ++q) {
        if (o->order == 1) {
            tile_visits(o, 0);
            tile_visits(o, 1);
        } else {
            half_sweep(o, 0);
            half_sweep(o, 1);
        }
        o->t += 1;
        if (every > 0 && o->t % (uint64_t)every == 0) orc_exchange_once(o);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* State access                                                        */
/* ------------------------------------------------------------------ */
int orc_get_spins(const orc_t *o, int8_t *s) {
    memcpy(s, o->s, (size_t)o->R * o->N);
    return 0;
}
int orc_set_spins(orc_t *o, const int8_t *s) {
    for (size_t q = 0; q < (size_t)o->R * o->N; ++q)
        if (s[q] != 1 && s[q] != -1) { set_err("spins must be +-1"); return -1; }
    memcpy(o->s, s, (size_t)o->R * o->N);
    return 0;
}
int orc_get_perm(const orc_t *o, int32_t *t2r) {
    memcpy(t2r, o->t2r, sizeof(int32_t) * (size_t)o->R);
    return 0;
}
int orc_set_perm(orc_t *o, const int32_t *t2r) {
    int *seen = (int *)calloc((size_t)o->R, sizeof(int));
    for (int t = 0; t < o->R; ++t) {
        if (t2r[t] < 0 || t2r[t] >= o->R || seen[t2r[t]]) {
            free(seen);
            set_err("not a permutation");
            return -1;
        }
        seen[t2r[t]] = 1;
    }
    free(seen);
    for (int t = 0; t < o->R; ++t) {
        o->t2r[t] = t2r[t];
        o->r2t[t2r[t]] = t;
    }
    return 0;
}
int orc_get_counters(const orc_t *o, uint64_t *t, uint64_t *k) {
    *t = o->t;
    *k = o->k;
    return 0;
}
int orc_set_counters(orc_t *o, uint64_t t, uint64_t k) {
    o->t = t;
    o->k = k;
    return 0;
}
int orc_exchange_stats(const orc_t *o, uint64_t *att, uint64_t *acc) {
    for (int p = 0; p + 1 < o->R; ++p) {
        att[p] = o->att[p];
        acc[p] = o->acc[p];
    }
    return 0;
}
int orc_reset_exchange_stats(orc_t *o) {
    memset(o->att, 0, sizeof(uint64_t) * (size_t)o->R_cap);
    memset(o->acc, 0, sizeof(uint64_t) * (size_t)o->R_cap);
    return 0;
}
int orc_thresholds(const orc_t *o, uint32_t *thr, uint8_t *always) {
    memcpy(thr, o->thr, sizeof(uint32_t) * 14 * (size_t)o->R);
    memcpy(always, o->always, 14);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Adaptive temperatures (Sec. 4)                                      */
/* ------------------------------------------------------------------ */
/* Min-heap of (rate, slot): the smallest rate on top, ties to the lower
 * slot. */
typedef struct { double rate; int p; } heap_item;

static int item_less(heap_item a, heap_item b) {
    return a.rate < b.rate || (a.rate == b.rate && a.p < b.p);
}
static void heap_push(heap_item *hp, int *n, heap_item it) {
    int q = (*n)++;
    hp[q] = it;
    while (q > 0) {
        int parent = (q - 1) / 2;
        if (!item_less(hp[q], hp[parent])) break;
        heap_item tmp = hp[q]; hp[q] = hp[parent]; hp[parent] = tmp;
        q = parent;
    }
}
static heap_item heap_pop(heap_item *hp, int *n) {
    heap_item top = hp[0];
    hp[0] = hp[--(*n)];
    int q = 0;
    for (;;) {
        int l = 2 * q + 1, r = l + 1, m = q;
        if (l < *n && item_less(hp[l], hp[m])) m = l;
        if (r < *n && item_less(hp[r], hp[m])) m = r;
        if (m == q) break;
        heap_item tmp = hp[q]; hp[q] = hp[m]; hp[m] = tmp;
        q = m;
    }
    return top;
}

/* One insertion step from the exchange counters accumulated since the last
 * reset (steps 2-7 below). */
int orc_insert_step(orc_t *o, double rate_threshold, int max_insert, int R_cap) {
    if (max_insert < 0) { set_err("bad insert arguments"); return -1; }
    if (R_cap > o->R_cap) { set_err("R_cap beyond the capacity given at create"); return -5; }
    /* 2-3. exchange rate of each adjacent pair into a min-heap */
    heap_item *hp = (heap_item *)malloc(sizeof(heap_item) * (size_t)(o->R + 1));
    int hn = 0;
    for (int p = 0; p + 1 < o->R; ++p)
        if (o->att[p] > 0)
            heap_push(hp, &hn, (heap_item){(double)o->acc[p] / (double)o->att[p], p});
    /* 4. lowest-rate intervals below the threshold, within the caps */
    int *picked = (int *)malloc(sizeof(int) * (size_t)(o->R + 1));
    int count = 0;
    while (hn > 0 && count < max_insert && o->R + count < R_cap) {
        heap_item it = heap_pop(hp, &hn);
        if (!(it.rate < rate_threshold)) break;
        picked[count++] = it.p;
    }
    free(hp);
    /* 5-6. midpoint temperature, new replica copies the colder end */
    int R0 = o->R;
    double *newT = (double *)malloc(sizeof(double) * (size_t)(R0 + count));
    int32_t *newrep = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R0 + count));
    for (int t = 0; t < R0; ++t) { newT[t] = o->T[t]; newrep[t] = o->t2r[t]; }
    for (int q = 0; q < count; ++q) {
        int p = picked[q];
        int id = R0 + q;
        newT[R0 + q] = (o->T[p] + o->T[p + 1]) / 2.0;
        newrep[R0 + q] = id;
        memcpy(o->s + (size_t)id * o->N, o->s + (size_t)o->t2r[p] * o->N, (size_t)o->N);
    }
    /* 7. re-sort the slots by temperature (insertion sort; the new
     * temperatures lie strictly inside distinct intervals) */
    int Rn = R0 + count;
    for (int a = 1; a < Rn; ++a) {
        double tv = newT[a];
        int32_t rv = newrep[a];
        int b = a - 1;
        while (b >= 0 && newT[b] > tv) {
            newT[b + 1] = newT[b];
            newrep[b + 1] = newrep[b];
            --b;
        }
        newT[b + 1] = tv;
        newrep[b + 1] = rv;
    }
    o->R = Rn;
    for (int t = 0; t < Rn; ++t) {
        o->T[t] = newT[t];
        o->t2r[t] = newrep[t];
        o->r2t[newrep[t]] = t;
    }
    build_tables(o);
    orc_reset_exchange_stats(o);
    free(newT);
    free(newrep);
    free(picked);
    return o->R;
}

int orc_adapt_temps(orc_t *o, int trials, int64_t sweeps_per_trial, int every,
                    double rate_threshold, int max_insert_per_trial, int R_cap) {
    if (trials < 0 || sweeps_per_trial < 0 || every <= 0 || max_insert_per_trial < 0) {
        set_err("bad adapt arguments");
        return -1;
    }
    if (R_cap > o->R_cap) { set_err("R_cap beyond the capacity given at create"); return -5; }
    for (int trial = 0; trial < trials; ++trial) {
        /* 1. a short trial run continuing the chain */
        orc_reset_exchange_stats(o);
        int rc = orc_sweep(o, sweeps_per_trial, every);
        if (rc) return rc;
        rc = orc_insert_step(o, rate_threshold, max_insert_per_trial, R_cap);
        if (rc < 0) return rc;
    }
    return o->R;
}
