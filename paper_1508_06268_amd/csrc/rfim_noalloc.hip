// Per-replica energy reduction (Eq. 1) for callers that cannot allocate
// device memory: spins and fields come from the caller's device buffers in
// natural site order, the energies go to a caller's device buffer, and the
// per-block partials live in a fixed device array of this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "rfim.h"
#include "rfim_internal.h"

namespace {

// (B, F) partial pairs; every GPU the library runs on holds its own copy
// until the process ends.
constexpr int kScratchPairs = RFIM_NOALLOC_MAX_PARTIALS;
constexpr int kMaxBlocks = 64;          // partials per replica at most
constexpr int kSitesPerBlock = 8192;    // below this many sites a replica gets fewer blocks
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[2 * kScratchPairs];

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block r * nb + b: sites [b * chunk, min(N, (b + 1) * chunk)) of replica r.
// B counts each bond once through its forward partner along x, y and z
// (periodic); F = sum f_i s_i in FP64.  Per thread in site order, then the
// wave's butterfly, then the four waves in order: the same sum on every
// call.
__global__ __launch_bounds__(256) void site_energy_partials(int L, int nb, long long N, long long chunk,
                                                            const int8_t *__restrict__ spins,
                                                            const float *__restrict__ fields,
                                                            double *__restrict__ part) {
    const int b = (int)(blockIdx.x % (unsigned)nb), r = (int)(blockIdx.x / (unsigned)nb);
    const int8_t *s = spins + (size_t)r * (size_t)N;
    const long long i0 = (long long)b * chunk;
    const long long i1 = min(N, i0 + chunk);
    const long long LL = (long long)L * L;
    double bsum = 0.0, fsum = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += 256) {
        const int x = (int)(i % L);
        const int y = (int)((i / L) % L);
        const int z = (int)(i / LL);
        const long long ix = x + 1 == L ? i - (L - 1) : i + 1;
        const long long iy = y + 1 == L ? i - (long long)(L - 1) * L : i + L;
        const long long iz = z + 1 == L ? i - (long long)(L - 1) * LL : i + LL;
        const int si = s[i];
        bsum += (double)(si * ((int)s[ix] + (int)s[iy] + (int)s[iz]));
        fsum += (double)fields[i] * (double)si;
    }
    __shared__ double red[2][4];
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const double wb = wave_total(bsum), wf = wave_total(fsum);
    if (lane == 0) {
        red[0][wave] = wb;
        red[1][wave] = wf;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const double v = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) + red[threadIdx.x][3];
        part[2 * ((size_t)r * nb + b) + threadIdx.x] = v;
    }
}

// E_r = -(J B_r) - (h F_r), the block partials added in block order.
__global__ __launch_bounds__(256) void site_energy_totals(int R, int nb, double J, double h,
                                                          const double *__restrict__ part, double *__restrict__ E) {
    const int r = (int)(blockIdx.x * 256 + threadIdx.x);
    if (r >= R) return;
    const double *p = part + 2 * (size_t)r * nb;
    double B = p[0], F = p[1];
    for (int b = 1; b < nb; ++b) {
        B += p[2 * b];
        F += p[2 * b + 1];
    }
    E[r] = -(J * B) - (h * F);
}

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// The device address of this GPU's copy of `scratch`, looked up once per
// device with that device current.  In host code the array's name is not a
// device address; only this pointer may reach kernels.
int scratch_on_current_device(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rfim_host::set_error(RFIM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return rfim_host::set_error(RFIM_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rfim_host::set_error(RFIM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return RFIM_OK;
}

}  // namespace

extern "C" int rfim_energies_noalloc(int L, int R, double J, double h, const int8_t *d_spins,
                                     const float *d_fields, double *d_E, void *hip_stream) {
    if (L < 2 || L > 1024 || (L & 1))
        return rfim_host::set_error(RFIM_EINVAL, "L must be even with 2 <= L <= 1024 (got %d)", L);
    if (R < 1) return rfim_host::set_error(RFIM_EINVAL, "R must be >= 1 (got %d)", R);
    if (R > kScratchPairs)
        return rfim_host::set_error(RFIM_ECAP, "R = %d beyond the %d replicas the fixed partial array holds", R,
                                    kScratchPairs);
    if (!d_spins || !d_fields || !d_E) return rfim_host::set_error(RFIM_EINVAL, "NULL device pointer");
    if (!std::isfinite(J) || !std::isfinite(h)) return rfim_host::set_error(RFIM_EINVAL, "J and h must be finite");
    const long long N = (long long)L * L * L;
    int nb = (int)std::min<long long>(kMaxBlocks, std::max<long long>(1, N / kSitesPerBlock));
    nb = std::min(nb, kScratchPairs / R);    // >= 1 since R <= kScratchPairs
    const long long chunk = (N + nb - 1) / nb;
    double *part = nullptr;
    int rc = scratch_on_current_device(&part);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(site_energy_partials, dim3((unsigned)(nb * R)), dim3(256), 0, s, L, nb, N, chunk, d_spins,
                       d_fields, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(site_energy_totals, dim3((R + 255) / 256), dim3(256), 0, s, R, nb, J, h,
                           (const double *)part, d_E);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return rfim_host::set_error(RFIM_EDEVICE, "energy launch: %s", hipGetErrorString(e));
    return RFIM_OK;
}
