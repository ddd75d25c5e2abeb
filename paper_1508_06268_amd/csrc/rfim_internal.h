// Internal interface between the host runtime (rfim_api.hip) and the
// device kernels (rfim_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfim_dev {

// Device layout of one realization (all arrays in HBM):
//   spins  uint8 [R_cap][2][N/2]  colour-split; byte = 1 iff s = +1.
//          Colour c, sublattice index j holds site 2j or 2j+1 (whichever has
//          colour c).
//   fbits  uint8 [2][N/2]         +-1 fields: byte = 4 iff h_i = +1, else 0.
//   fhf    float [2][N/2]         continuous fields: (float)(h * h_i - 6 J).
//   fraw   float [2][N/2]         continuous fields: h_i as given.
//   thr    uint32 [R_cap][32]     per slot, +-1 fields, indexed by
//                                 (up << 2) | (b << 1) | f with up = number of
//                                 +1 neighbours, b = spin byte, f = field bit:
//                                 a flip is taken iff u32 <= entry, unless bit
//                                 idx of entry 31 (the slot's never mask) is
//                                 set.  Entry = 0xFFFFFFFF where dE <= 0,
//                                 else floor(e^(-beta dE) 2^32) - 1, or 0 with
//                                 the never bit where that floor is 0.
//   betaf  float [R_cap]          per slot, continuous fields.
//   beta   double [R_cap]         per slot (exchange).
//   t2r, r2t int32 [R_cap]; att, acc uint64 [R_cap]
//   ctrs   uint64 [2]             global sweep counter t, exchange counter k.
//   part   double [nblk][R_cap][3] energy partials (B, F, M) per block,
//                                 block-major so that consecutive replicas'
//                                 partials of one block are adjacent (the
//                                 reduction reads them coalesced);
//                                 nblk = blocks_per_replica(shape).
//   E      double [R_cap]         energy by replica id after a reduction.
//   Mr     double [R_cap]         magnetisation by replica id (same reduction).
//   obs    double [R_cap][6]      per slot, one sample per exchange step
//                                 (Sec. 7): count, sum E, sum E^2, sum |M|,
//                                 sum M^2, sum M^4.
struct Lattice {
    int L, N, half, R;          // R = replicas currently active
    int log2L;                  // >= 3 when L is a power of two, else -1
    int kind;                   // 0 bimodal, 1 continuous
    float Jf;
    double J, h;
    uint32_t key0, key1, rho;
    uint8_t *spins;
    const uint8_t *fbits;
    const float *fhf, *fraw;
    const uint32_t *thr;
    const float *betaf;
    const double *beta;
    int32_t *t2r, *r2t;
    uint64_t *att, *acc;
    uint64_t *ctrs;
    double *part;
    int nblk;                   // energy partials per replica
    int pstride;                // replicas per block row of part (R_cap)
    int mode;                   // power-of-two L: 0 streaming, 1 LDS-resident
    int nw, wg;                 // dwords per thread, threads per workgroup
    double *E;
    double *Mr;
    double *obs;
    // one bit per spin (rfim_set_spin_storage): bits uint32 [R_cap][2][N/64],
    // colour c, word w = sublattice indices 32w..32w+31 (index 32w+4b+q at
    // bit 8q+b), 1 iff s = +1; fbw uint32 [2][N/64] in the same order,
    // 1 iff h_i = +1 (+-1 fields).  Null while the spins live in `spins`.
    // fhw float [2][N/2]: continuous fields as in fhf, ordered for the bit
    // sweep: in colour c, the four values of sublattice indices
    // 32w+4b..32w+4b+3 (block b of word w) are float4 number
    // (8 (w/64) + b) 64 + w%64, so that the 64 threads of a wavefront read
    // block b of their words as 1 KiB in one piece (N/64 is a multiple of
    // 64 at every L that bit storage takes).
    uint32_t *bits;
    const uint32_t *fbw;
    const float *fhw;
};

// Above this many workgroups per replica the streaming sweep does not write
// energy partials; a separate energy kernel with 64 blocks does.
constexpr int kMaxFusedBlocks = 1024;

// Launch shapes.  Power-of-two L >= 8: mode 0 (streaming: one chunk of
// nw dwords per thread, wg in {64, 128, 256}), mode 1 (LDS-resident,
// L <= 32: one workgroup of wg threads per replica runs every sweep of an
// exchange interval) or modes 2..4 (slabs, L = 16..64: nw slabs per
// replica, mode - 1 sweeps per launch, wg threads).  Other L: generic
// kernel, shape (0, 0, 0).  Every shape gives bit-identical results.
bool shape_valid(int L, int mode, int nw, int wg);
// Batch and pool classes also take shape (kModeBits, 0, 0) at L = 64, 128
// or 256: one bit per spin, each item swept on its own by the bit sweep
// (the storage of a standalone handle is set with rfim_set_spin_storage
// instead).
constexpr int kModeBits = 5;
// Energy partials per replica for a shape (1 for resident, the workgroups
// per replica when the streaming sweep fuses the energy, else 64).
int blocks_per_replica(int L, int mode, int nw, int wg);
// Workgroups per replica of one streaming half-sweep launch.
int stream_blocks_per_replica(int L, int nw, int wg);
// True when the sweep kernels themselves write the energy partials.
bool fused_energy(const Lattice &lat);

// One launch over a set of realizations that share L, field kind and shape:
// lats = device array of descriptors; map = one entry per workgroup:
// x = (realization << 16) | replica, y = block within the replica
// (streaming) or 0 (resident).
struct Launch {
    const Lattice *lats;
    const uint2 *map;
    int nblocks;
    int L, kind, mode, nw, wg;
    // one realization: its descriptor, passed by value (lats and map
    // unused; blocks enumerate (replica, block) in order, from replica r0)
    const Lattice *single = nullptr;
    int r0 = 0;
};

// Slab sweeps (mode 2..4, L = 16 or 32): nslab workgroups per replica, each
// a z-slab of L/nslab planes with the halo recomputed, mode - 1 sweeps per
// launch at most; reads `src`, writes `dst` (a second spin buffer: the
// workgroups of a replica must not see each other's new planes).
int slab_sweeps_per_launch(int mode);
size_t slab_lds_bytes(int L, int mode, int nslab);
int slab_positions_per_thread(int L, int mode, int nslab, int wg);
hipError_t launch_slab_sweep(const Lattice &lat, const uint8_t *src, uint8_t *dst, int mode, int nslab, int wg,
                             int nsweep, int toff, int energy, hipStream_t s);

// Double-checkerboard order with multi-hit updates (Sec. 3.2, Sec. 5.2):
// tiles of tx * ty * tz sites, `hits` local sweeps per tile visit.  Valid
// for L = 2^l >= 16 with tx a multiple of 8, every side dividing L into an
// even number of tiles, (tx / 8) ty tz threads per workgroup in
// {64, 128, ..., 1024}, the staged box within 64 KB of LDS, 1 <= hits <=
// 65536.
struct TileShape {
    int tx, ty, tz, hits;
};
bool tile_shape_valid(int L, const TileShape &ts);
size_t tile_lds_bytes(const TileShape &ts);
// The tiles of coarse colour `coarse` of every replica at sweep t + toff.
hipError_t launch_tile_sweep(const Lattice &lat, const TileShape &ts, int coarse, int toff, hipStream_t s);

// One bit per spin: L = 2^l with 64 <= L <= 256.  Workgroups per replica
// of a bit half-sweep (each writes one energy partial with ENERGY).
bool bits_valid(int L);
int bits_blocks_per_replica(int L);
// Half-sweep of colour `colour` at sweep t + toff for replicas r0..r0+nrep-1
// (energy != 0 on colour 1: also the energy partials of the final state).
hipError_t launch_bits_sweep(const Lattice &lat, int r0, int nrep, int colour, int toff, int energy, hipStream_t s);
// The bit sweep over a batch class in bit storage: ln.map holds one entry
// per replica (x = (realization << 16) | replica), ln.nblocks entries.
hipError_t launch_bits_batch(const Launch &ln, int colour, int toff, int energy, hipStream_t s);
// Byte spins <-> bit spins of replicas [0, R) (and, to bits, the +-1 field
// words).
hipError_t launch_pack_bits(const Lattice &lat, hipStream_t s);
hipError_t launch_unpack_bits(const Lattice &lat, hipStream_t s);

hipError_t launch_init(const Lattice &lat, int r0, int r1, hipStream_t s);
// Streaming half-sweep of colour `colour` at sweep t + toff (power-of-two
// L); energy != 0 on colour 1 also writes the energy partials.
hipError_t launch_stream_sweep(const Launch &ln, int colour, int toff, int energy, hipStream_t s);
// Resident: nsweep whole sweeps in one launch (energy != 0: also the
// energy partials of the final state).
hipError_t launch_resident(const Launch &ln, int nsweep, int energy, hipStream_t s);
// Any even L, one realization.
hipError_t launch_generic_sweep(const Lattice &lat, int colour, int toff, hipStream_t s);
hipError_t launch_energy(const Lattice &lat, hipStream_t s);
hipError_t launch_reduce(const Lattice &lat, int64_t *B, double *F, int64_t *M, hipStream_t s);
// One exchange step for each of the n realizations in lats (device array).
hipError_t launch_exchange(const Lattice *lats, int n, int tadv, hipStream_t s);
hipError_t launch_advance(const Lattice &lat, int tadv, hipStream_t s);
// Fourier observable of every replica, accumulated by slot (rfim_measure.hip):
// part int32 [R_cap][L][2L] scratch, trig double [2][L] = cos, sin of
// 2 pi v / L, fobs double [R_cap][2] = (count, sum F).
hipError_t launch_fourier(const Lattice &lat, int32_t *part, const double *trig, double *fobs, hipStream_t s);

}  // namespace rfim_dev

namespace rfim_host {
// Records a message for rfim_last_error() (printf-style) and returns code.
int set_error(int code, const char *fmt, ...);
}  // namespace rfim_host
