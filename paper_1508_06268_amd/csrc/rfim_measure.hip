// Fourier observable of the correlation length (arXiv:1508.06268, Sec. 7)
// on the device, one sample per exchange step and temperature slot:
//   F = (1/(3N)) sum_mu [(sum_i s_i cos(K x_mu,i))^2 + (sum_i s_i sin(K x_mu,i))^2],
// K = 2 pi / L, mu over the three axes (the printed sums carry the field
// h_i; read with the spins s_i, the usual second-moment estimator).  Each
// inner sum is grouped by coordinate: integer plane sums n_mu(v) first
// (exact in any order), then sum_v cos(K v) n_mu(v) in FP64 with v
// ascending, so the result does not depend on the launch shape.
//
// Compiled with -ffp-contract=off like the other kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfim_internal.h"

namespace rfim_dev {

namespace {

// One wave per (z-plane, replica): row sums over x (indexed by y) by ballot
// and population count, column sums over y (indexed by x) in LDS, one
// entry per lane.  part[r][z][0..L) = row sums, [L..2L) = column sums.
__global__ __launch_bounds__(64) void plane_sums_kernel(Lattice lat, int32_t *part) {
    __shared__ int32_t cols[1024];
    const int L = lat.L, z = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
    for (int x = lane; x < L; x += 64) cols[x] = 0;
    const uint8_t *sp = lat.spins + (size_t)r * lat.N;
    int32_t *dst = part + ((size_t)r * L + z) * 2 * L;
    for (int y = 0; y < L; ++y) {
        int rs = 0;
        for (int x0 = 0; x0 < L; x0 += 64) {
            const int x = x0 + lane;
            const bool in = x < L;
            int s = 0;
            if (in) {
                const int i = x + L * (y + L * z);
                const int c = (x + y + z) & 1;
                s = 2 * (int)sp[(size_t)c * lat.half + (i >> 1)] - 1;
                cols[x] += s;
            }
            const uint64_t up = __ballot(in && s > 0), all = __ballot(in);
            rs += 2 * __popcll(up) - __popcll(all);
        }
        if (lane == 0) dst[y] = rs;
    }
    for (int x = lane; x < L; x += 64) dst[L + x] = cols[x];
}

// One wave per replica: plane sums along the three axes from the partials,
// then C_mu, S_mu and F in FP64 (one lane, v ascending), accumulated into
// the replica's current slot: fobs[slot] = (count, sum F).
__global__ __launch_bounds__(64) void fourier_kernel(Lattice lat, const int32_t *part, const double *trig,
                                                     double *fobs) {
    __shared__ int32_t n[3][1024];
    const int L = lat.L, r = blockIdx.x, lane = threadIdx.x;
    const int32_t *pr = part + (size_t)r * L * 2 * L;
    for (int v = lane; v < L; v += 64) {
        int32_t nx = 0, ny = 0, nz = 0;
        for (int z = 0; z < L; ++z) {
            nx += pr[(size_t)z * 2 * L + L + v];   // columns of plane z at x = v
            ny += pr[(size_t)z * 2 * L + v];       // rows of plane z at y = v
            nz += pr[(size_t)v * 2 * L + z];       // plane z = v, row z
        }
        n[0][v] = nx;
        n[1][v] = ny;
        n[2][v] = nz;
    }
    __syncthreads();
    if (lane != 0) return;
    double c[3], s[3];
    for (int mu = 0; mu < 3; ++mu) {
        c[mu] = 0.0;
        s[mu] = 0.0;
        for (int v = 0; v < L; ++v) {
            c[mu] += trig[v] * (double)n[mu][v];
            s[mu] += trig[L + v] * (double)n[mu][v];
        }
    }
    const double F = (c[0] * c[0] + s[0] * s[0] + c[1] * c[1] + s[1] * s[1] + c[2] * c[2] + s[2] * s[2]) /
                     (3.0 * (double)lat.N);
    double *o = fobs + 2 * (size_t)lat.r2t[r];
    o[0] += 1.0;
    o[1] += F;
}

}  // namespace

hipError_t launch_fourier(const Lattice &lat, int32_t *part, const double *trig, double *fobs, hipStream_t s) {
    hipLaunchKernelGGL(plane_sums_kernel, dim3(lat.L, lat.R), dim3(64), 0, s, lat, part);
    hipLaunchKernelGGL(fourier_kernel, dim3(lat.R), dim3(64), 0, s, lat, part, trig, fobs);
    return hipGetLastError();
}

}  // namespace rfim_dev
