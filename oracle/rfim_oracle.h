/*
 * rfim_oracle.h -- plain, single-threaded CPU oracle for the Exchange Monte
 * Carlo (parallel tempering) method on the 3D random field Ising model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the HIP implementation.
 *
 * What it computes, and where the paper defines it:
 *   - Hamiltonian H = -J sum_<ij> s_i s_j - h sum_i h_i s_i on a periodic L^3
 *     lattice, each bond counted once (Sec. 1, Eq. 1).
 *   - Checkerboard Metropolis: sites with (x+y+z) mod 2 = c are updated as
 *     one half-sweep, colour 0 then colour 1 (Sec. 2 and Sec. 3.2, Eq. 3);
 *     optionally the double checkerboard of tiles with multi-hit local
 *     sweeps (Sec. 3.2, Sec. 5.2).
 *   - Replica exchange between adjacent temperatures, odd/even alternation,
 *     acceptance min(1, e^Delta) with Delta = (b_{i+1}-b_i)(H(X_{i+1})-H(X_i))
 *     (Sec. 3.1, step 4, Eq. 2 -- printed with its cases swapped; the
 *     min(1, e^Delta) reading is the Hukushima-Nemoto rule the paper cites).
 *   - Temperatures move instead of configurations: slot->replica and
 *     replica->slot permutations (Sec. 3.3, "trs"/"rts").
 *   - Adaptive insertion of temperatures at the midpoint of the
 *     lowest-exchange-rate intervals after short trial runs (Sec. 4).
 *   - The Fourier observable of the correlation length (Sec. 7).
 *
 * Conventions the paper leaves open (random number generator, colour order,
 * counter mapping, acceptance precision) are fixed here and written out in
 * rfim_oracle.c next to the code that follows them.
 */
#ifndef RFIM_ORACLE_H
#define RFIM_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc_t;

/* L even, 2 <= L <= 512.  field_kind: -1 auto (bimodal iff every field is
 * exactly +-1), 0 bimodal, 1 continuous.  R_cap >= R bounds adaptive growth
 * (0 means R). */
orc_t *orc_create(int L, int R, double J, double h, const float *fields,
                  const double *temps, uint64_t seed, uint32_t realization,
                  int field_kind, int R_cap);
void orc_destroy(orc_t *o);
const char *orc_last_error(void);

int orc_num_replicas(const orc_t *o);
int orc_field_kind(const orc_t *o);

/* n sweeps; after a sweep that makes the global sweep count a multiple of
 * every (every > 0) an exchange step follows. */
int orc_sweep(orc_t *o, int64_t n, int every);

/* Update order of the sweeps.  order 0 (default): the plain two-colour
 * checkerboard.  order 1: the double checkerboard with multi-hit updates
 * (Sec. 3.2, Sec. 5.2): tiles of tx * ty * tz sites (each side dividing L
 * into an even number of tiles) in a coarse checkerboard; each sweep visits
 * the tiles of coarse colour 0, then those of colour 1, and each visit runs
 * `hits` local two-colour sweeps of the tile.  Sweeps then need
 * (t + n) * hits <= 2^31.  Returns 0 or -1. */
int orc_set_update_order(orc_t *o, int order, int tx, int ty, int tz, int hits);

/* Observables by temperature slot (ascending T). */
int orc_energies(orc_t *o, double *E);
int orc_magnetizations(orc_t *o, int64_t *M);
int orc_temps(const orc_t *o, double *T);

/* Energy pieces by replica id: bond sum B, field sum F, magnetisation M. */
int orc_components(orc_t *o, int64_t *B, double *F, int64_t *M);

/* State access (spins by replica id, natural site order i = x + L(y + L z),
 * values +-1). */
int orc_get_spins(const orc_t *o, int8_t *s);
int orc_set_spins(orc_t *o, const int8_t *s);
int orc_get_perm(const orc_t *o, int32_t *t2r);
int orc_set_perm(orc_t *o, const int32_t *t2r);
int orc_get_counters(const orc_t *o, uint64_t *t, uint64_t *k);
int orc_set_counters(orc_t *o, uint64_t t, uint64_t k);
int orc_exchange_stats(const orc_t *o, uint64_t *att, uint64_t *acc);
int orc_reset_exchange_stats(orc_t *o);

/* One exchange step with the current counter k (energies recomputed first). */
int orc_exchange_once(orc_t *o);

/* Energy change the sweep would use for flipping site i of replica r. */
double orc_flip_delta(const orc_t *o, int r, int i);

/* The sweep's own decision for site i of replica r (at its current slot)
 * with random word u: 1 flip, 0 keep, -1 bad arguments. */
int orc_accept(const orc_t *o, int r, int i, uint32_t u);

/* Fourier observable of the correlation length (Sec. 7) of the current
 * configuration at every slot: F[R], see rfim_oracle.c. */
int orc_fourier(const orc_t *o, double *F);

/* Acceptance thresholds the sweep uses for bimodal fields: thr[R][14],
 * always[14] (1 where Delta E <= 0).  Class index = 2*k + fb with k the
 * number of the six neighbour slots aligned with s_i and fb = 1 iff
 * s_i * h_i = +1. */
int orc_thresholds(const orc_t *o, uint32_t *thr, uint8_t *always);

/* Adaptive temperatures.  Returns the new R or a negative error. */
int orc_insert_step(orc_t *o, double rate_threshold, int max_insert, int R_cap);
int orc_adapt_temps(orc_t *o, int trials, int64_t sweeps_per_trial, int every,
                    double rate_threshold, int max_insert_per_trial, int R_cap);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif
