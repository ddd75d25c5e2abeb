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
//   fbits  uint8 [2][N/2]         +-1 fields: byte = 1 iff h_i = +1.
//   fhf    float [2][N/2]         continuous fields: (float)(h * h_i).
//   fraw   float [2][N/2]         continuous fields: h_i as given.
//   thr    uint32 [R_cap][16]     per slot, +-1 fields: threshold by class
//                                 2k + fb (k = aligned neighbours, fb = field
//                                 aligned); 0xFFFFFFFF for dE <= 0 classes.
//   betaf  float [R_cap]          per slot, continuous fields.
//   beta   double [R_cap]         per slot (exchange).
//   t2r, r2t int32 [R_cap]; att, acc uint64 [R_cap]
//   ctrs   uint64 [2]             global sweep counter t, exchange counter k.
//   part   double [R_cap][nblk][3] energy partials (B, F, M) per block.
//   E      double [R_cap]         energy by replica id after a reduction.
struct Lattice {
    int L, N, half, R;          // R = replicas currently active
    int log2L;                  // >= 3 when L is a power of two, else -1
    int kind;                   // 0 bimodal, 1 continuous
    float Jf;
    double J, h;
    uint32_t key0, key1, rho;
    uint32_t always_mask;       // bit (2k+fb) set iff that class has dE <= 0
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
    int nblk;                   // energy blocks per replica
    double *E;
};

int energy_blocks_per_replica(int L);

hipError_t launch_init(const Lattice &lat, int r0, int r1, hipStream_t s);
hipError_t launch_sweep(const Lattice &lat, int colour, int toff, hipStream_t s);
hipError_t launch_energy(const Lattice &lat, hipStream_t s);
hipError_t launch_reduce(const Lattice &lat, int64_t *B, double *F, int64_t *M, hipStream_t s);
hipError_t launch_exchange(const Lattice &lat, int tadv, hipStream_t s);
hipError_t launch_advance(const Lattice &lat, int tadv, hipStream_t s);

}  // namespace rfim_dev
