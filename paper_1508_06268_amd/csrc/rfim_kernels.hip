// HIP kernels for gfx950: Philox4x32-10, initial spins, checkerboard
// Metropolis half-sweeps, per-replica energy reduction and the replica
// exchange step of the Exchange Monte Carlo method (arXiv:1508.06268,
// Sec. 3.1-3.3, Eq. 1-3).
//
// Compiled with -ffp-contract=off: every FP64 expression that feeds an
// exchange decision is evaluated exactly as written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfim_internal.h"

namespace rfim_dev {

namespace {

constexpr uint32_t kTagInit = 1u, kTagSweep = 2u, kTagExch = 3u;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products by fixed odd multipliers whose high halves are mixed
// with the other two words and the round key; the key follows a Weyl
// sequence.  Written from the published definition.
struct Words { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = (uint64_t)0xD2511F53u * c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t word_at(const Words &w, int q) {
    return q == 0 ? w.w0 : q == 1 ? w.w1 : q == 2 ? w.w2 : w.w3;
}

// exp(-beta dE) * 2^32 as an integer threshold in FP32 (continuous fields).
__device__ __forceinline__ uint32_t cont_threshold(float beta, float dE) {
    const float p = expf(-(beta * dE));
    const float scaled = fminf(p * 4294967296.0f, 4294967040.0f);
    return (uint32_t)scaled;
}

// ---------------------------------------------------------------------
// Initial spins (method step 3): replica r, natural sites 4g..4g+3 take
// the four words of block (g, 0, r) of the INIT stream.
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_kernel(Lattice lat, int r0) {
    const int G = lat.N >> 2;
    const int g = blockIdx.x * 256 + threadIdx.x;
    const int r = r0 + blockIdx.y;
    if (g >= G) return;
    const Words w = philox10((uint32_t)g, 0u, (uint32_t)r, (kTagInit << 28) | lat.rho, lat.key0,
                             lat.key1);
    uint8_t *base = lat.spins + (size_t)r * lat.N;
    const int L = lat.L;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * g + q;
        const int x = i % L, y = (i / L) % L, z = i / (L * L);
        const int c = (x + y + z) & 1;
        base[(size_t)c * lat.half + (i >> 1)] = word_at(w, q) >= 0x80000000u ? 1 : 0;
    }
}

// ---------------------------------------------------------------------
// Half-sweep, any even L: one thread per four consecutive sublattice
// sites j = 4g..4g+3 of colour c (one Philox block), each site located
// and its six neighbours gathered individually.
// ---------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void sweep_generic(Lattice lat, int colour, int toff) {
    const int G = lat.half >> 2;
    const int g = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (g >= G) return;
    const uint32_t t = (uint32_t)(lat.ctrs[0] + (uint64_t)toff);
    const Words w = philox10((uint32_t)g, 2u * t + (uint32_t)colour, (uint32_t)r,
                             (kTagSweep << 28) | lat.rho, lat.key0, lat.key1);
    const int slot = lat.r2t[r];
    const int L = lat.L;
    uint8_t *own = lat.spins + (size_t)r * lat.N + (size_t)colour * lat.half;
    const uint8_t *oth = lat.spins + (size_t)r * lat.N + (size_t)(1 - colour) * lat.half;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = 4 * g + q;
        const int i0 = 2 * j;
        const int x0 = i0 % L, y = (i0 / L) % L, z = i0 / (L * L);
        const int x = x0 + (((x0 + y + z) & 1) ^ colour);
        const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
        const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
        const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
        const int up = oth[(xp + L * (y + L * z)) >> 1] + oth[(xm + L * (y + L * z)) >> 1] +
                       oth[(x + L * (yp + L * z)) >> 1] + oth[(x + L * (ym + L * z)) >> 1] +
                       oth[(x + L * (y + L * zp)) >> 1] + oth[(x + L * (y + L * zm)) >> 1];
        const int b = own[j];
        const uint32_t u = word_at(w, q);
        bool accept;
        if (KIND == 0) {
            const int k = b ? up : 6 - up;
            const int fb = b == lat.fbits[(size_t)colour * lat.half + j];
            const int cls = 2 * k + fb;
            accept = ((lat.always_mask >> cls) & 1u) || u < lat.thr[slot * 16 + cls];
        } else {
            const float n = (float)(2 * up - 6);
            const float s = b ? 1.0f : -1.0f;
            const float xloc = lat.Jf * n + lat.fhf[(size_t)colour * lat.half + j];
            const float dE = 2.0f * s * xloc;
            accept = dE <= 0.0f || u < cont_threshold(lat.betaf[slot], dE);
        }
        if (accept) own[j] = (uint8_t)(b ^ 1);
    }
}

// ---------------------------------------------------------------------
// Half-sweep, L = 2^l >= 8.  One thread per four consecutive sublattice
// sites of one row: the four spin bytes, the six neighbour words and the
// field bytes are 32-bit loads, and the neighbour counts of the four sites
// are one packed byte-wise sum (each byte <= 6, so no carries).
//
// Colour-c site of pair m in row (y, z) sits at x = 2m + p, p = (c+y+z)&1;
// its x-neighbours of the other colour are pair m and pair m-1+2p of the
// same row, so the row's other-colour word shifted by one byte (with the
// byte from the adjacent word, wrapping in the row) supplies the second x
// neighbour.
// ---------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void sweep_pow2(Lattice lat, int colour, int toff, int wg_per_rep,
                                                   int remap) {
    __shared__ uint32_t sthr[16];
    int blk = blockIdx.x;
    if (remap) {
        // consecutive block ids go round-robin to the 8 XCDs; give each XCD a
        // contiguous range of tiles so that halo rows stay in its L2
        const int per = gridDim.x >> 3;
        blk = (blk & 7) * per + (blk >> 3);
    }
    const int r = blk / wg_per_rep;
    const int gb = blk - r * wg_per_rep;
    const int slot = lat.r2t[r];
    if (KIND == 0) {
        if (threadIdx.x < 16) sthr[threadIdx.x] = lat.thr[slot * 16 + threadIdx.x];
        __syncthreads();
    }
    const int l = lat.log2L;
    const int L = lat.L;
    const int g = gb * blockDim.x + threadIdx.x;
    const int j0 = 4 * g;
    const int hm = (L >> 1) - 1;                       // m bits
    const int ystep = L >> 1;
    const int ymask = (L - 1) << (l - 1);
    const int zstep = (L * L) >> 1;
    const int jmask = lat.half - 1;
    const int m0 = j0 & hm;
    const int row = j0 >> (l - 1);
    const int y = row & (L - 1), z = row >> l;
    const int p = (colour + y + z) & 1;
    const int jx = (j0 - m0) | ((m0 + (p ? 4 : -4)) & hm);
    const int jyp = (j0 & ~ymask) | ((j0 + ystep) & ymask);
    const int jym = (j0 & ~ymask) | ((j0 - ystep) & ymask);
    const int jzp = (j0 + zstep) & jmask;
    const int jzm = (j0 - zstep) & jmask;

    uint8_t *own = lat.spins + (size_t)r * lat.N + (size_t)colour * lat.half;
    const uint8_t *oth = lat.spins + (size_t)r * lat.N + (size_t)(1 - colour) * lat.half;
    const uint32_t Wown = *(const uint32_t *)(own + j0);
    const uint32_t W = *(const uint32_t *)(oth + j0);
    const uint32_t Wx = *(const uint32_t *)(oth + jx);
    const uint32_t Wyp = *(const uint32_t *)(oth + jyp);
    const uint32_t Wym = *(const uint32_t *)(oth + jym);
    const uint32_t Wzp = *(const uint32_t *)(oth + jzp);
    const uint32_t Wzm = *(const uint32_t *)(oth + jzm);
    // p = 1: bytes of pairs m0+1..m0+4; p = 0: bytes of pairs m0-1..m0+2
    const uint32_t Xs = p ? __builtin_amdgcn_alignbyte(Wx, W, 1) : __builtin_amdgcn_alignbyte(W, Wx, 3);
    const uint32_t U = W + Xs + Wyp + Wym + Wzp + Wzm;  // up-neighbour counts, per byte

    const uint32_t t = (uint32_t)(lat.ctrs[0] + (uint64_t)toff);
    const Words w = philox10((uint32_t)g, 2u * t + (uint32_t)colour, (uint32_t)r,
                             (kTagSweep << 28) | lat.rho, lat.key0, lat.key1);
    uint32_t flip = 0;
    if (KIND == 0) {
        const uint32_t Fw = *(const uint32_t *)(lat.fbits + (size_t)colour * lat.half + j0);
        const uint32_t Mb = Wown * 0xFFu;                      // 0x00 / 0xFF per byte
        const uint32_t K = (Mb & U) | (~Mb & (0x06060606u - U)); // aligned neighbours
        const uint32_t FB = ~(Wown ^ Fw) & 0x01010101u;         // field aligned
        const uint32_t CLS = (K << 1) | FB;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t cls = (CLS >> (8 * q)) & 0xFFu;
            const uint32_t u = word_at(w, q);
            uint32_t acc = u < sthr[cls] ? 1u : 0u;
            if (u == 0xFFFFFFFFu) acc = (lat.always_mask >> cls) & 1u;
            flip |= acc << (8 * q);
        }
    } else {
        const float4 hf = *(const float4 *)(lat.fhf + (size_t)colour * lat.half + j0);
        const float beta = lat.betaf[slot];
        const float hv[4] = {hf.x, hf.y, hf.z, hf.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int up = (U >> (8 * q)) & 0xFF;
            const float n = (float)(2 * up - 6);
            const float s = ((Wown >> (8 * q)) & 1u) ? 1.0f : -1.0f;
            const float xloc = lat.Jf * n + hv[q];
            const float dE = 2.0f * s * xloc;
            const uint32_t u = word_at(w, q);
            const bool acc = dE <= 0.0f || u < cont_threshold(beta, dE);
            flip |= (acc ? 1u : 0u) << (8 * q);
        }
    }
    if (flip) *(uint32_t *)(own + j0) = Wown ^ flip;
}

// ---------------------------------------------------------------------
// Energy partials (Eq. 1).  Every bond joins a colour-0 and a colour-1
// site, so B = sum over colour-1 sites of s_i n_i counts each bond once;
// F and M run over both colours.  Grid (nblk, R); fixed reduction order.
// ---------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void energy_kernel(Lattice lat) {
    const int G = lat.half >> 2;
    const int r = blockIdx.y;
    const int L = lat.L;
    const uint8_t *s0 = lat.spins + (size_t)r * lat.N;
    const uint8_t *s1 = s0 + lat.half;
    long long bsum = 0, msum = 0;
    double fsum = 0.0;
    for (int g = blockIdx.x * 256 + threadIdx.x; g < G; g += lat.nblk * 256) {
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * g + q;
            const int i0 = 2 * j;
            const int x0 = i0 % L, y = (i0 / L) % L, z = i0 / (L * L);
            const int x = x0 + (((x0 + y + z) & 1) ^ 1);   // the colour-1 site of pair j
            const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
            const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
            const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
            const int up = s0[(xp + L * (y + L * z)) >> 1] + s0[(xm + L * (y + L * z)) >> 1] +
                           s0[(x + L * (yp + L * z)) >> 1] + s0[(x + L * (ym + L * z)) >> 1] +
                           s0[(x + L * (y + L * zp)) >> 1] + s0[(x + L * (y + L * zm)) >> 1];
            const int b1 = s1[j], b0 = s0[j];
            const int sp1 = 2 * b1 - 1, sp0 = 2 * b0 - 1;
            bsum += sp1 * (2 * up - 6);
            msum += sp1 + sp0;
            if (lat.kind == 0) {
                const int f1 = 2 * lat.fbits[lat.half + j] - 1, f0 = 2 * lat.fbits[j] - 1;
                fsum += (double)(f1 * sp1 + f0 * sp0);
            } else {
                fsum += (double)lat.fraw[lat.half + j] * (double)sp1;
                fsum += (double)lat.fraw[j] * (double)sp0;
            }
        }
    }
    __shared__ double red[3][4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double vb = wave_sum((double)bsum), vm = wave_sum((double)msum), vf = wave_sum(fsum);
    if (lane == 0) {
        red[0][wave] = vb;
        red[1][wave] = vf;
        red[2][wave] = vm;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const double v = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) +
                         red[threadIdx.x][3];
        lat.part[((size_t)r * lat.nblk + blockIdx.x) * 3 + threadIdx.x] = v;
    }
}

__device__ __forceinline__ void replica_totals(const Lattice &lat, int r, double &B, double &F,
                                               double &M) {
    const double *pp = lat.part + (size_t)r * lat.nblk * 3;
    B = 0.0;
    F = 0.0;
    M = 0.0;
    for (int b = 0; b < lat.nblk; ++b) {
        B += pp[3 * b + 0];
        F += pp[3 * b + 1];
        M += pp[3 * b + 2];
    }
}

__device__ __forceinline__ double energy_of(const Lattice &lat, double B, double F) {
    return -(lat.J * B) - (lat.h * F);
}

// Totals per replica id; optional outputs for the observables calls.
__global__ __launch_bounds__(256) void reduce_kernel(Lattice lat, int64_t *Bout, double *Fout,
                                                     int64_t *Mout) {
    for (int r = threadIdx.x; r < lat.R; r += 256) {
        double B, F, M;
        replica_totals(lat, r, B, F, M);
        lat.E[r] = energy_of(lat, B, F);
        if (Bout) Bout[r] = (int64_t)B;
        if (Fout) Fout[r] = F;
        if (Mout) Mout[r] = (int64_t)M;
    }
}

// ---------------------------------------------------------------------
// Exchange step k (Eq. 2): pairs (p, p+1) with p = k mod 2; temperatures
// move through t2r / r2t (Sec. 3.3).  One workgroup.
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void exchange_kernel(Lattice lat, int tadv) {
    for (int r = threadIdx.x; r < lat.R; r += 256) {
        double B, F, M;
        replica_totals(lat, r, B, F, M);
        lat.E[r] = energy_of(lat, B, F);
    }
    const uint64_t k = lat.ctrs[1];
    __syncthreads();
    for (int p = (int)(k & 1) + 2 * (int)threadIdx.x; p + 1 < lat.R; p += 512) {
        const int a = lat.t2r[p], b = lat.t2r[p + 1];
        const double delta = (lat.beta[p + 1] - lat.beta[p]) * (lat.E[b] - lat.E[a]);
        const Words w = philox10((uint32_t)p, (uint32_t)k, 0u, (kTagExch << 28) | lat.rho, lat.key0,
                                 lat.key1);
        const double u53 = ((double)(w.w0 >> 11) * 4294967296.0 + (double)w.w1) * 0x1p-53;
        lat.att[p] += 1;
        if (delta >= 0.0 || u53 < exp(delta)) {
            lat.t2r[p] = b;
            lat.t2r[p + 1] = a;
            lat.r2t[a] = p + 1;
            lat.r2t[b] = p;
            lat.acc[p] += 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        lat.ctrs[0] += (uint64_t)tadv;
        lat.ctrs[1] = k + 1;
    }
}

__global__ void advance_kernel(uint64_t *ctrs, int tadv) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctrs[0] += (uint64_t)tadv;
}

}  // namespace

int energy_blocks_per_replica(int L) {
    const long long G = (long long)L * L * L / 8;
    long long nb = (G + 255) / 256;
    if (nb > 64) nb = 64;
    return (int)(nb < 1 ? 1 : nb);
}

hipError_t launch_init(const Lattice &lat, int r0, int r1, hipStream_t s) {
    if (r1 <= r0) return hipSuccess;
    const int G = lat.N >> 2;
    dim3 grid((G + 255) / 256, r1 - r0);
    hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, s, lat, r0);
    return hipGetLastError();
}

hipError_t launch_sweep(const Lattice &lat, int colour, int toff, hipStream_t s) {
    const int G = lat.half >> 2;
    if (lat.log2L >= 3) {
        const int wg = G < 256 ? G : 256;
        const int wg_per_rep = G / wg;
        const int nb = wg_per_rep * lat.R;
        const int remap = (nb % 8 == 0) ? 1 : 0;
        if (lat.kind == 0)
            hipLaunchKernelGGL(sweep_pow2<0>, dim3(nb), dim3(wg), 0, s, lat, colour, toff, wg_per_rep,
                               remap);
        else
            hipLaunchKernelGGL(sweep_pow2<1>, dim3(nb), dim3(wg), 0, s, lat, colour, toff, wg_per_rep,
                               remap);
    } else {
        dim3 grid((G + 255) / 256, lat.R);
        if (lat.kind == 0)
            hipLaunchKernelGGL(sweep_generic<0>, grid, dim3(256), 0, s, lat, colour, toff);
        else
            hipLaunchKernelGGL(sweep_generic<1>, grid, dim3(256), 0, s, lat, colour, toff);
    }
    return hipGetLastError();
}

hipError_t launch_energy(const Lattice &lat, hipStream_t s) {
    hipLaunchKernelGGL(energy_kernel, dim3(lat.nblk, lat.R), dim3(256), 0, s, lat);
    return hipGetLastError();
}

hipError_t launch_reduce(const Lattice &lat, int64_t *B, double *F, int64_t *M, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, lat, B, F, M);
    return hipGetLastError();
}

hipError_t launch_exchange(const Lattice &lat, int tadv, hipStream_t s) {
    hipLaunchKernelGGL(exchange_kernel, dim3(1), dim3(256), 0, s, lat, tadv);
    return hipGetLastError();
}

hipError_t launch_advance(const Lattice &lat, int tadv, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, lat.ctrs, tadv);
    return hipGetLastError();
}

}  // namespace rfim_dev
