// HIP kernels for gfx950: Philox4x32-10, initial spins, checkerboard
// Metropolis half-sweeps, per-replica energy reduction and the replica
// exchange step of the Exchange Monte Carlo method (arXiv:1508.06268,
// Sec. 3.1-3.3, Eq. 1-3).
//
// Compiled with -ffp-contract=off: every FP64 expression that feeds an
// exchange decision is evaluated exactly as written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "rfim_internal.h"

namespace rfim_dev {

namespace {

constexpr uint32_t kTagInit = 1u, kTagSweep = 2u, kTagExch = 3u;

// Pointers read from a descriptor table in memory are generic; typing them
// as global (address space 1) all the way to the access keeps loads and
// stores global_* rather than flat_* instructions.
#define GAS __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ GAS T *gptr(T *p) {
    return (GAS T *)p;
}

// Pointer to U in the address space (and constness) of pointer type P.
template <class P, class U> struct rebind_ptr;
template <class U> struct rebind_ptr<uint8_t *, U> { using type = U *; };
template <class U> struct rebind_ptr<const uint8_t *, U> { using type = const U *; };
template <class U> struct rebind_ptr<GAS uint8_t *, U> { using type = GAS U *; };
template <class U> struct rebind_ptr<GAS const uint8_t *, U> { using type = GAS const U *; };
template <class U> struct rebind_ptr<const float *, U> { using type = const U *; };
template <class U> struct rebind_ptr<GAS const float *, U> { using type = GAS const U *; };

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products by fixed odd multipliers whose high halves are mixed
// with the other two words and the round key; the key follows a Weyl
// sequence.  Written from the published definition.
struct Words { uint32_t w0, w1, w2, w3; };

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;

// Philox4x32-10 with the first round's product M0 * c0 given: a caller
// whose counters step by a constant can form it with one multiply-add.
__device__ __forceinline__ Words philox10_p(uint64_t a0, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = round == 0 ? a0 : (uint64_t)kPhiloxM0 * c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0, n2;
        if (round < 2) {
            // the first rounds still hold wave-uniform words: leave them to
            // the scalar unit
            n0 = (uint32_t)(b >> 32) ^ (c1 ^ k0);
            n2 = (uint32_t)(a >> 32) ^ (c3 ^ k1);
        } else if (round == 2) {
            // with a wave-uniform c0 and c2 at round 0 (one site block per
            // lane), c3 is still uniform here: one scalar XOR, one VALU XOR
            // (a three-input VALU XOR can read only one scalar operand)
            n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
            n2 = (uint32_t)(a >> 32) ^ (c3 ^ k1);
        } else {
            // three-input XOR in one VALU instruction (truth table 0x96)
            n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, k1, 0x96);
        }
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
    return philox10_p((uint64_t)kPhiloxM0 * c0, c0, c1, c2, c3, k0, k1);
}

// M0 x + c in one v_mad_u64_u32 (c a wave-uniform 64-bit addend; M0 from
// a VGPR, since one instruction reads one scalar operand).  Written out
// because the compiler folds M0 x + M0 b back into M0 (x + b), which costs
// the addition of b on top of the product.  The carry-out register is not
// read.
__device__ __forceinline__ uint64_t mad_m0(uint32_t x, uint32_t m0, uint64_t c) {
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(carry) : "v"(x), "v"(m0), "s"(c));
    return r;
}

__device__ __forceinline__ uint32_t word_at(const Words &w, int q) {
    return q == 0 ? w.w0 : q == 1 ? w.w1 : q == 2 ? w.w2 : w.w3;
}

// Continuous fields, one site, in FP32.  With up = number of +1 neighbours,
// J n + h h_i = 2J up + (h h_i - 6J) = y (the second term precomputed per
// site), and the flip costs dE = 2 s y.  With a = -2 beta log2(e),
// exp(-beta dE) = 2^(s a y): accept iff s a y >= 0 (dE <= 0) or
// u32 2^-32 < 2^(s a y).
__device__ __forceinline__ bool cont_accept(float up, float hfs, float twoJ, float a, bool up_spin,
                                            uint32_t u) {
    const float y = fmaf(twoJ, up, hfs);
    const float ta = a * y;
    const float t = up_spin ? ta : -ta;
    const float p = __builtin_amdgcn_exp2f(t);
    return t >= 0.0f || (float)u * 0x1p-32f < p;
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
            const int f = lat.fbits[(size_t)colour * lat.half + j] >> 2;
            const int idx = (up << 2) | (b << 1) | f;
            const uint32_t *tab = lat.thr + slot * 32;
            accept = u <= tab[idx] && !((tab[31] >> idx) & 1u);
        } else {
            const float a = -2.0f * 1.44269504088896341f * lat.betaf[slot];
            accept = cont_accept((float)up, lat.fhf[(size_t)colour * lat.half + j], 2.0f * lat.Jf, a, b != 0, u);
        }
        if (accept) own[j] = (uint8_t)(b ^ 1);
    }
}

// ---------------------------------------------------------------------
// Half-sweep, L = 2^l >= 8, on one chunk of NW x 4 consecutive sublattice
// sites of one row (NW Philox blocks): the spin bytes, the six neighbour
// words and the field bytes are NW-dword loads, and the neighbour counts of
// four sites are one packed byte-wise sum per dword (each byte <= 6, so no
// carries).
//
// Colour-c site of pair m in row (y, z) sits at x = 2m + p, p = (c+y+z)&1;
// its x-neighbours of the other colour are pair m and pair m-1+2p of the
// same row, so the row's other-colour bytes shifted by one (with one byte
// from the adjacent dword, wrapping in the row) supply the second x
// neighbour.
// ---------------------------------------------------------------------
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int NW> struct Vec;
template <> struct Vec<1> { using T = uint32_t; };
template <> struct Vec<2> { using T = u32x2; };
template <> struct Vec<4> { using T = u32x4; };

template <int NW, class P>
__device__ __forceinline__ void load_words(P base, uint32_t off, uint32_t (&w)[NW]) {
    if constexpr (NW == 8) {
        // two 16-byte loads
        uint32_t lo[4], hi[4];
        load_words<4>(base, off, lo);
        load_words<4>(base, off + 16u, hi);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w[q] = lo[q];
            w[q + 4] = hi[q];
        }
        return;
    } else {
    const typename Vec<NW>::T v = *(typename rebind_ptr<P, const typename Vec<NW>::T>::type)(base + off);
    if constexpr (NW == 1) {
        w[0] = v;
    } else if constexpr (NW == 2) {
        w[0] = v.x; w[1] = v.y;
    } else {
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    }
    }
}

template <int NW, class P>
__device__ __forceinline__ void store_words(P base, uint32_t off, const uint32_t (&w)[NW]) {
    if constexpr (NW == 8) {
        const uint32_t lo[4] = {w[0], w[1], w[2], w[3]}, hi[4] = {w[4], w[5], w[6], w[7]};
        store_words<4>(base, off, lo);
        store_words<4>(base, off + 16u, hi);
        return;
    } else {
    typename Vec<NW>::T v;
    if constexpr (NW == 1) {
        v = w[0];
    } else if constexpr (NW == 2) {
        v.x = w[0]; v.y = w[1];
    } else {
        v.x = w[0]; v.y = w[1]; v.z = w[2]; v.w = w[3];
    }
    *(typename rebind_ptr<P, typename Vec<NW>::T>::type)(base + off) = v;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Offsets (in sublattice bytes) of the other-colour words around a chunk.
struct Chunk {
    uint32_t p, jxw, jyp, jym, jzp, jzm;
};

template <int NW>
__device__ __forceinline__ Chunk chunk_geometry(uint32_t j0, uint32_t colour, uint32_t L, uint32_t l,
                                                uint32_t half) {
    Chunk c;
    const uint32_t hm = (L >> 1) - 1u;          // m bits of j
    const uint32_t ystep = L >> 1;
    const uint32_t ymask = (L - 1u) << (l - 1u);
    const uint32_t zstep = (L * L) >> 1;
    const uint32_t jmask = half - 1u;
    const uint32_t m0 = j0 & hm;
    const uint32_t row = j0 >> (l - 1u);
    c.p = (colour + row + (row >> l)) & 1u;     // (c + y + z) & 1
    // the one dword of the adjacent chunk that the x-shift needs
    c.jxw = (j0 - m0) | ((m0 + (c.p ? 4u * NW : 0u - 4u)) & hm);
    c.jyp = (j0 & ~ymask) | ((j0 + ystep) & ymask);
    c.jym = (j0 & ~ymask) | ((j0 - ystep) & ymask);
    c.jzp = (j0 + zstep) & jmask;
    c.jzm = (j0 - zstep) & jmask;
    return c;
}

// The other-colour words around a chunk: the chunk's own pair words W, the
// one dword of the adjacent chunk the x-shift needs, and the y+-1, z+-1 rows.
template <int NW> struct Around {
    uint32_t W[NW], Wx, Wyp[NW], Wym[NW], Wzp[NW], Wzm[NW];
};

template <int NW, class P>
__device__ __forceinline__ void load_around(P oth, uint32_t j0, const Chunk &c, Around<NW> &a) {
    load_words<NW>(oth, j0, a.W);
    a.Wx = *(typename rebind_ptr<P, const uint32_t>::type)(oth + c.jxw);
    load_words<NW>(oth, c.jyp, a.Wyp);
    load_words<NW>(oth, c.jym, a.Wym);
    load_words<NW>(oth, c.jzp, a.Wzp);
    load_words<NW>(oth, c.jzm, a.Wzm);
}

// Up-neighbour counts (per byte) of the NW words of a chunk.
template <int NW>
__device__ __forceinline__ void neighbour_sums(const Chunk &c, const Around<NW> &a, uint32_t (&U)[NW]) {
    // p = 1: bytes of pairs m+1..m+4 (bytes 1-3 of W[w], byte 0 of the next
    // word); p = 0: bytes of pairs m-1..m+2 (byte 3 of the previous word,
    // bytes 0-2 of W[w]).  One byte permute of {other word, W[w]}.
    const uint32_t sel = c.p ? 0x04030201u : 0x02010007u;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t nxt = (w + 1 < NW) ? a.W[w + 1 < NW ? w + 1 : 0] : a.Wx;
        const uint32_t prv = (w > 0) ? a.W[w > 0 ? w - 1 : 0] : a.Wx;
        const uint32_t Xs = __builtin_amdgcn_perm(c.p ? nxt : prv, a.W[w], sel);
        U[w] = a.W[w] + Xs + a.Wyp[w] + a.Wym[w] + a.Wzp[w] + a.Wzm[w];
    }
}

template <int NW, class P>
__device__ __forceinline__ void neighbour_counts(P oth, uint32_t j0, const Chunk &c, uint32_t (&W)[NW],
                                                 uint32_t (&U)[NW]) {
    Around<NW> a;
    load_around<NW>(oth, j0, c, a);
    neighbour_sums<NW>(c, a, U);
#pragma unroll
    for (int w = 0; w < NW; ++w) W[w] = a.W[w];
}

// Bit q set iff u_q <= t_q, for four sites.  The compares write four lane
// masks that an add-with-carry chain folds into one register (acc = 2 acc +
// mask), so each site costs two VALU instructions and no select.  gfx950
// wants two wait states between a VALU write of a lane mask and a VALU read
// of it: every mask is read three instructions after it is written, and the
// trailing nop covers reads after the block.
__device__ __forceinline__ uint32_t accept_bits(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t u3,
                                                uint32_t t0, uint32_t t1, uint32_t t2, uint32_t t3) {
    uint32_t acc;
    uint64_t c3, c2, c1, c0, cx;
    asm("v_cmp_le_u32_e64 %1, %9, %13\n\t"
        "v_cmp_le_u32_e64 %2, %8, %12\n\t"
        "v_cmp_le_u32_e64 %3, %7, %11\n\t"
        "v_cmp_le_u32_e64 %4, %6, %10\n\t"
        "v_cndmask_b32_e64 %0, 0, 1, %1\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %2\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %3\n\t"
        "v_addc_co_u32_e64 %0, %5, %0, %0, %4\n\t"
        "s_nop 1"
        : "=&v"(acc), "=&s"(c3), "=&s"(c2), "=&s"(c1), "=&s"(c0), "=&s"(cx)
        : "v"(u0), "v"(u1), "v"(u2), "v"(u3), "v"(t0), "v"(t1), "v"(t2), "v"(t3));
    return acc;
}

// The bit sweep's form: the four decisions of one Philox block shifted
// into four accumulators, f_q = 2 f_q + [u_q <= t_q].  Run over blocks 7
// down to 0, bit b of f_q ends as the flip of block b's site q, which is
// bit 8q + b of the word: byte q of the flips is f_q, with no per-block
// spreading.  Four compares and four add-with-carry per block; each mask
// is read four instructions after it is written (gfx950's VALU-mask
// hazard), and the trailing nop covers reads after the block.
__device__ __forceinline__ void accept_shift(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t u3,
                                             uint32_t t0, uint32_t t1, uint32_t t2, uint32_t t3,
                                             uint32_t &f0, uint32_t &f1, uint32_t &f2, uint32_t &f3) {
    uint64_t c0, c1, c2, c3, cx;
    asm("v_cmp_le_u32_e64 %4, %9, %13\n\t"
        "v_cmp_le_u32_e64 %5, %10, %14\n\t"
        "v_cmp_le_u32_e64 %6, %11, %15\n\t"
        "v_cmp_le_u32_e64 %7, %12, %16\n\t"
        "v_addc_co_u32_e64 %0, %8, %0, %0, %4\n\t"
        "v_addc_co_u32_e64 %1, %8, %1, %1, %5\n\t"
        "v_addc_co_u32_e64 %2, %8, %2, %2, %6\n\t"
        "v_addc_co_u32_e64 %3, %8, %3, %3, %7\n\t"
        "s_nop 1"
        : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3), "=&s"(c0), "=&s"(c1), "=&s"(c2), "=&s"(c3), "=&s"(cx)
        : "v"(u0), "v"(u1), "v"(u2), "v"(u3), "v"(t0), "v"(t1), "v"(t2), "v"(t3));
}

// Metropolis decisions of one Philox block's four sites (+-1 fields): the
// table entry sits at LDS byte address ((up << 2) | (s << 1) | f) * 4 and a
// site flips iff u <= entry.  `never` marks classes whose bound is 0 at this
// temperature: there u = 0 would pass, so with NEV those sites are
// corrected when some u is 0 (about one block in 2^30).  Returns the flips
// as one bit per byte.
template <bool NEV>
__device__ __forceinline__ uint32_t bimodal_flips(const uint32_t *sthr, uint32_t U, uint32_t Wown,
                                                  uint32_t F4, const Words &rw, uint32_t never) {
    const uint32_t A = (U << 4) | (Wown << 3) | F4;
    const uint8_t *tb = (const uint8_t *)sthr;
    const uint32_t a0 = A & 0xFFu, a1 = (A >> 8) & 0xFFu, a2 = (A >> 16) & 0xFFu, a3 = A >> 24;
    const uint32_t th0 = *(const uint32_t *)(tb + a0), th1 = *(const uint32_t *)(tb + a1);
    const uint32_t th2 = *(const uint32_t *)(tb + a2), th3 = *(const uint32_t *)(tb + a3);
    const uint32_t acc = accept_bits(rw.w0, rw.w1, rw.w2, rw.w3, th0, th1, th2, th3);
    // bit q of a 4-bit value to bit 8q: the shifted copies 0, 7, 14, 21
    // do not overlap, so the product has no carries
    uint32_t fl = __umul24(acc, 0x204081u) & 0x01010101u;
    if (NEV) {
        const uint32_t umin = min(min(rw.w0, rw.w1), min(rw.w2, rw.w3));
        if (umin == 0u) {
            if (rw.w0 == 0u && ((never >> (a0 >> 2)) & 1u)) fl &= ~0x1u;
            if (rw.w1 == 0u && ((never >> (a1 >> 2)) & 1u)) fl &= ~0x100u;
            if (rw.w2 == 0u && ((never >> (a2 >> 2)) & 1u)) fl &= ~0x10000u;
            if (rw.w3 == 0u && ((never >> (a3 >> 2)) & 1u)) fl &= ~0x1000000u;
        }
    }
    return fl;
}

// Float to unsigned integer with the hardware's saturation (values at or
// above 2^32, infinity included, give 0xFFFFFFFF; negative values give 0).
__device__ __forceinline__ uint32_t cvt_u32_sat(float x) {
    uint32_t r;
    asm("v_cvt_u32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Continuous fields.  With up = number of +1 neighbours of a site and s
// its spin bit, J n + h h_i = 2J up + (h h_i - 6J) = 2J up + hfs (the
// second term precomputed per site), the flip costs dE = 2 (2s - 1) y with
// y = 2J up + hfs, and e^(-beta dE) = 2^x with
//   x = a (2s - 1) y = a (2s - 1) 2J up + a (2s - 1) hfs,  a = -2 beta log2(e).
// The two site-independent factors depend only on (up, s) at a given
// temperature: a per-slot LDS table holds them, entry (up << 1) | s =
// {a (2s - 1) 2J up, a (2s - 1)}, so x costs one FMA per site.  The integer
// bound is floor(2^x 2^32), saturated; dE <= 0 gives x >= 0 and the bound
// 0xFFFFFFFF, which every u32 meets: one integer test u <= bound covers
// both cases of the Metropolis rule.
__device__ __forceinline__ void cont_table_fill(uint32_t *sthr, float beta, float Jf) {
    const uint32_t q = threadIdx.x;
    if (q < 14u) {
        const float a = -2.0f * 1.44269504088896341f * beta;
        const float sa = (q & 1u) ? a : -a;
        const float two_j_up = 2.0f * Jf * (float)(q >> 1);
        sthr[2 * q] = __float_as_uint(sa * two_j_up);
        sthr[2 * q + 1] = __float_as_uint(sa);
    }
}

// The bound of one site from its table entry (at LDS byte offset e) and hfs.
__device__ __forceinline__ uint32_t cont_bound(const uint8_t *tb, uint32_t e, float hfs) {
    const float2 c = *(const float2 *)(tb + e);
    const float x = fmaf(c.y, hfs, c.x);
    return cvt_u32_sat(__builtin_amdgcn_exp2f(x) * 0x1p32f);
}

// Continuous fields: four sites of one Philox block, byte q of A the table
// entry offset (up << 4) | (s << 3) of site q; bit q set iff site q flips.
__device__ __forceinline__ uint32_t continuous_acc_at(const uint32_t *sthr, uint32_t A, const f32x4 hf,
                                                      const Words &rw) {
    const uint8_t *tb = (const uint8_t *)sthr;
    const uint32_t b0 = cont_bound(tb, A & 0xFFu, hf.x), b1 = cont_bound(tb, __builtin_amdgcn_ubfe(A, 8u, 8u), hf.y);
    const uint32_t b2 = cont_bound(tb, (A >> 16) & 0xFFu, hf.z), b3 = cont_bound(tb, A >> 24, hf.w);
    return accept_bits(rw.w0, rw.w1, rw.w2, rw.w3, b0, b1, b2, b3);
}

// The same from up counts U and spins Wown one per byte.
__device__ __forceinline__ uint32_t continuous_acc(const uint32_t *sthr, uint32_t U, uint32_t Wown, const f32x4 hf,
                                                   const Words &rw) {
    return continuous_acc_at(sthr, (U << 4) | (Wown << 3), hf, rw);
}

// Continuous fields: four sites of one Philox block, the flips one bit
// per byte.
__device__ __forceinline__ uint32_t continuous_flips(const uint32_t *sthr, uint32_t U, uint32_t Wown,
                                                     const f32x4 hf, const Words &rw) {
    return __umul24(continuous_acc(sthr, U, Wown, hf, rw), 0x204081u) & 0x01010101u;
}

// The words a chunk's half-sweep update reads: its own words, the
// other-colour words around it and its fields.
template <int KIND, int NW> struct ChunkIn {
    Chunk c;
    uint32_t Wown[NW];
    Around<NW> a;
    f32x4 HF[NW];   // continuous fields (KIND 1)
};

// Issue every load of a chunk (F4: the +-1 field bits, KIND 0).  Callers put
// a scheduling barrier after it so the compiler does not sink a load next to
// its use: with many realizations in a launch the fields and rows miss in
// L2, and a load issued per Philox block would expose the memory latency
// each time.
template <int KIND, int NW, class PO, class PC, class PB, class PF>
__device__ __forceinline__ void chunk_load(const Lattice &lat, PO own, PC oth, PB fb_own, PF hf_own, uint32_t j0,
                                           uint32_t colour, ChunkIn<KIND, NW> &in, uint32_t (&F4)[NW]) {
    in.c = chunk_geometry<NW>(j0, colour, (uint32_t)lat.L, (uint32_t)lat.log2L, (uint32_t)lat.half);
    load_words<NW>(own, j0, in.Wown);
    load_around<NW>(oth, j0, in.c, in.a);
    if (KIND == 0) {
        load_words<NW>(fb_own, j0, F4);
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w)
            in.HF[w] = *(typename rebind_ptr<PF, const f32x4>::type)(hf_own + j0 + 4u * w);
    }
}

// The flip decisions of a loaded chunk; returns nonzero if any site flips,
// with the new own words in Wnew (and the other-colour words and neighbour
// sums the energy pass reuses in W and U).
template <int KIND, int NW, bool NEV>
__device__ __forceinline__ uint32_t chunk_flip(const Lattice &lat, const uint32_t *sthr, uint32_t never,
                                               const ChunkIn<KIND, NW> &in, const uint32_t (&F4)[NW],
                                               uint32_t g0, uint32_t c1, uint32_t r, float beta,
                                               uint32_t (&W)[NW], uint32_t (&U)[NW], uint32_t (&Wnew)[NW]) {
    neighbour_sums<NW>(in.c, in.a, U);
#pragma unroll
    for (int w = 0; w < NW; ++w) W[w] = in.a.W[w];
    const uint32_t c3 = (kTagSweep << 28) | lat.rho;
    uint32_t any = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const Words rw = philox10(g0 + (uint32_t)w, c1, r, c3, lat.key0, lat.key1);
        uint32_t fl;
        if (KIND == 0) {
            fl = bimodal_flips<NEV>(sthr, U[w], in.Wown[w], F4[w], rw, never);
        } else {
            fl = continuous_flips(sthr, U[w], in.Wown[w], in.HF[w], rw);
        }
        any |= fl;
        Wnew[w] = in.Wown[w] ^ fl;
    }
    return any;
}

// chunk_flip with the never-class correction only where this slot has such
// classes (a wave-uniform branch between two copies).
template <int KIND, int NW>
__device__ __forceinline__ uint32_t chunk_flip_any(const Lattice &lat, const uint32_t *sthr, uint32_t never,
                                                   const ChunkIn<KIND, NW> &in, const uint32_t (&F4)[NW],
                                                   uint32_t g0, uint32_t c1, uint32_t r, float beta,
                                                   uint32_t (&W)[NW], uint32_t (&U)[NW], uint32_t (&Wnew)[NW]) {
    if (KIND == 0 && never != 0u) return chunk_flip<KIND, NW, true>(lat, sthr, never, in, F4, g0, c1, r, beta, W, U, Wnew);
    return chunk_flip<KIND, NW, false>(lat, sthr, never, in, F4, g0, c1, r, beta, W, U, Wnew);
}

// One chunk's half-sweep update: load, then flip.
template <int KIND, int NW, class PO, class PC, class PB, class PF>
__device__ __forceinline__ uint32_t chunk_update_any(const Lattice &lat, const uint32_t *sthr, uint32_t never,
                                                     PO own, PC oth, PB fb_own, PF hf_own, uint32_t j0,
                                                     uint32_t g0, uint32_t colour, uint32_t c1, uint32_t r,
                                                     float beta, uint32_t (&W)[NW], uint32_t (&U)[NW],
                                                     uint32_t (&Wnew)[NW], uint32_t (&F4)[NW]) {
    ChunkIn<KIND, NW> in;
    chunk_load<KIND, NW>(lat, own, oth, fb_own, hf_own, j0, colour, in, F4);
    __builtin_amdgcn_sched_barrier(0);
    return chunk_flip_any<KIND, NW>(lat, sthr, never, in, F4, g0, c1, r, beta, W, U, Wnew);
}

// Energy pieces of a chunk of colour-1 sites and the colour-0 sites of the
// same pairs, from the final spins: every bond joins a colour-0 and a
// colour-1 site, so B = sum over colour-1 sites of s_i n_i counts each bond
// once; F and M take both colours.
template <int KIND, int NW, class PB, class PF>
__device__ __forceinline__ void chunk_energy(const Lattice &lat, const uint32_t (&S1)[NW],
                                             const uint32_t (&S0)[NW], const uint32_t (&U)[NW],
                                             const uint32_t (&F1)[NW], PB fb0, PF fr1, PF fr0, uint32_t j0,
                                             int &ksum, int &upsum, int &eqsum, double &fsum) {
    uint32_t F0[NW];
    if (KIND == 0) load_words<NW>(fb0, j0, F0);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t Mb = S1[w] * 0xFFu;                                // 0x00 / 0xFF per byte
        const uint32_t K = (Mb & U[w]) | (~Mb & (0x06060606u - U[w]));  // aligned neighbours
        ksum = (int)__builtin_amdgcn_sad_u8(K, 0u, (uint32_t)ksum);
        upsum = (int)__builtin_amdgcn_sad_u8(S1[w] + S0[w], 0u, (uint32_t)upsum);
        if (KIND == 0) {
            const uint32_t e1 = ~(S1[w] ^ (F1[w] >> 2)) & 0x01010101u;
            const uint32_t e0 = ~(S0[w] ^ (F0[w] >> 2)) & 0x01010101u;
            eqsum = (int)__builtin_amdgcn_sad_u8(e1 + e0, 0u, (uint32_t)eqsum);
        } else {
            const f32x4 f1 = *(typename rebind_ptr<PF, const f32x4>::type)(fr1 + j0 + 4u * w);
            const f32x4 f0 = *(typename rebind_ptr<PF, const f32x4>::type)(fr0 + j0 + 4u * w);
            const float a1[4] = {f1.x, f1.y, f1.z, f1.w}, a0[4] = {f0.x, f0.y, f0.z, f0.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                fsum += ((S1[w] >> (8 * q)) & 1u) ? (double)a1[q] : -(double)a1[q];
                fsum += ((S0[w] >> (8 * q)) & 1u) ? (double)a0[q] : -(double)a0[q];
            }
        }
    }
}

// Block-wide (B, F, M) partial in a fixed order; thread 0..2 write it.
template <int KIND, class PD>
__device__ __forceinline__ void block_partial(PD dst, int nsite, int ksum, int upsum, int eqsum,
                                              double fsum) {
    __shared__ double red[3][16];
    const int bpart = 2 * ksum - 6 * nsite;
    const int mpart = 2 * upsum - 2 * nsite;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // integer sums over the wave's active lanes (DPP reduction in the
    // device library; exact, so the order does not matter)
    const int vb = __ockl_wfred_add_i32(bpart), vm = __ockl_wfred_add_i32(mpart);
    const double vf = KIND == 0 ? (double)__ockl_wfred_add_i32(2 * eqsum - 2 * nsite) : wave_sum(fsum);
    if (lane == 0) {
        red[0][wave] = (double)vb;
        red[1][wave] = vf;
        red[2][wave] = (double)vm;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int nw = (int)((blockDim.x + 63) >> 6);
        double v = red[threadIdx.x][0];
        for (int q = 1; q < nw; ++q) v += red[threadIdx.x][q];
        dst[threadIdx.x] = v;
    }
}

// Streaming half-sweep: one chunk per thread; one launch covers every
// replica of every realization listed in the block map (entry: realization,
// (replica << 16) | block within the replica), or, for one realization,
// replicas r0, r0 + 1, ... in block order.  ENERGY (colour 1 of the last
// sweep before an exchange) also writes one energy partial per workgroup.
template <int KIND, int NW, int ENERGY, bool BATCH>
__global__ __launch_bounds__(256) void sweep_pow2(Lattice lat0, const Lattice *__restrict__ lats,
                                                   const uint2 *__restrict__ map, int colour, int toff,
                                                   int remap, int lwpr, int r0) {
    __shared__ __align__(16) uint32_t sthr[32];   // +-1 thresholds or the continuous-field table
    uint32_t blk = blockIdx.x;
    if (remap) {
        // consecutive block ids go round-robin to the 8 XCDs; give each XCD a
        // contiguous range of tiles so that halo rows stay in its L2
        const uint32_t per = gridDim.x >> 3;
        blk = (blk & 7u) * per + (blk >> 3);
    }
    uint32_t r, gb;
    if (BATCH) {
        const uint2 e = map[blk];
        r = e.x & 0xFFFFu;
        gb = e.y;
    } else {
        r = (uint32_t)r0 + (blk >> lwpr);
        gb = blk & ((1u << lwpr) - 1u);
    }
    const Lattice &lat = BATCH ? lats[map[blk].x >> 16] : lat0;
    const uint32_t g0 = (gb * blockDim.x + threadIdx.x) * NW;   // first Philox block
    const uint32_t j0 = 4u * g0;
    const uint32_t col = (uint32_t)colour;
    GAS uint8_t *spins = gptr(lat.spins);
    GAS uint8_t *own = spins + (size_t)r * lat.N + (size_t)col * lat.half;
    GAS const uint8_t *oth = spins + (size_t)r * lat.N + (size_t)(1 - col) * lat.half;
    GAS const uint8_t *fbits = gptr(lat.fbits);
    GAS const float *fhf = gptr(lat.fhf), *fraw = gptr(lat.fraw);
    // The chunk's loads go out first; the slot's table (r2t, then thr) is
    // fetched while they are in flight, so the workgroup's barrier on the
    // table costs the longer of the two chains rather than their sum.
    ChunkIn<KIND, NW> in;
    uint32_t F4[NW];
    chunk_load<KIND, NW>(lat, own, oth, fbits + (size_t)col * lat.half, fhf + (size_t)col * lat.half, j0, col, in,
                         F4);
    __builtin_amdgcn_sched_barrier(0);
    const int slot = gptr(lat.r2t)[r];
    const uint32_t t = (uint32_t)(gptr(lat.ctrs)[0] + (uint64_t)toff);
    uint32_t never = 0;
    const float beta = KIND == 1 ? gptr(lat.betaf)[slot] : 0.0f;
    if (KIND == 0) {
        if (threadIdx.x < 32u) sthr[threadIdx.x] = gptr(lat.thr)[slot * 32 + threadIdx.x];
        __syncthreads();
        never = __builtin_amdgcn_readfirstlane(sthr[31]);
    } else {
        cont_table_fill(sthr, beta, lat.Jf);
        __syncthreads();
    }
    uint32_t W[NW], U[NW], Wnew[NW];
    const uint32_t any = chunk_flip_any<KIND, NW>(lat, sthr, never, in, F4, g0, 2u * t + col, r, beta, W, U, Wnew);
    if (any) store_words<NW>(own, j0, Wnew);
    if (ENERGY) {
        int ksum = 0, upsum = 0, eqsum = 0;
        double fsum = 0.0;
        chunk_energy<KIND, NW>(lat, Wnew, W, U, F4, fbits, fraw + lat.half, fraw, j0, ksum, upsum, eqsum,
                               fsum);
        block_partial<KIND>(gptr(lat.part) + ((size_t)gb * lat.pstride + r) * 3, 4 * NW, ksum, upsum, eqsum,
                            fsum);
    }
}

// Resident sweeps (L = 2^l <= 32): one workgroup holds one replica's spins
// in LDS and runs `nsweep` whole sweeps (colour 0 then colour 1, a barrier
// between half-sweeps), then, if asked, the energy partial of the final
// state, and writes the spins back.  Fields stay in global memory (shared
// by every replica, so they live in L2).
template <int KIND, int NW, bool BATCH, bool ONE>
__global__ __launch_bounds__(1024) void sweep_resident(Lattice lat0, const Lattice *__restrict__ lats,
                                                        const uint2 *__restrict__ map, int nsweep,
                                                        int energy) {
    extern __shared__ uint4 lds_raw[];
    __shared__ __align__(16) uint32_t sthr[32];   // +-1 thresholds or the continuous-field table
    uint8_t *sp = (uint8_t *)lds_raw;                  // [2][half]
    // batch: map entry (realization << 16 | replica, 0)
    const Lattice &lat = BATCH ? lats[map[blockIdx.x].x >> 16] : lat0;
    const uint32_t r = BATCH ? (map[blockIdx.x].x & 0xFFFFu) : blockIdx.x;
    const uint32_t N = (uint32_t)lat.N, half = (uint32_t)lat.half;
    const int slot = gptr(lat.r2t)[r];
    GAS const u32x4 *src = (GAS const u32x4 *)(gptr(lat.spins) + (size_t)r * N);
    u32x4 *lds4 = (u32x4 *)lds_raw;
    for (uint32_t q = threadIdx.x; q < N / 16u; q += blockDim.x) lds4[q] = src[q];
    if (KIND == 0 && threadIdx.x < 32) sthr[threadIdx.x] = gptr(lat.thr)[slot * 32 + threadIdx.x];
    const float beta = KIND == 1 ? gptr(lat.betaf)[slot] : 0.0f;
    if (KIND == 1) cont_table_fill(sthr, beta, lat.Jf);
    const uint32_t t0 = (uint32_t)gptr(lat.ctrs)[0];
    GAS const uint8_t *fbits = gptr(lat.fbits);
    GAS const float *fhf = gptr(lat.fhf), *fraw = gptr(lat.fraw);
    const uint32_t nchunk = half / (4u * NW);
    __syncthreads();
    const uint32_t never = KIND == 0 ? __builtin_amdgcn_readfirstlane(sthr[31]) : 0u;
    if constexpr (ONE) {
        // every thread owns chunk threadIdx.x of both colours: its fields
        // are read once per launch and kept in registers
        const uint32_t g0 = threadIdx.x * NW, j0 = 4u * g0;
        uint32_t F4c[2][NW];
        f32x4 HFc[2][NW];
#pragma unroll
        for (int col = 0; col < 2; ++col) {
            if (KIND == 0) {
                load_words<NW>(fbits + (size_t)col * half, j0, F4c[col]);
            } else {
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    HFc[col][w] = *(GAS const f32x4 *)(fhf + (size_t)col * half + j0 + 4u * w);
            }
        }
        for (int sw = 0; sw < nsweep; ++sw) {
#pragma unroll
            for (int col = 0; col < 2; ++col) {
                uint8_t *own = sp + col * half;
                const uint8_t *oth = sp + (1u - col) * half;
                const uint32_t c1 = 2u * (t0 + (uint32_t)sw) + col;
                ChunkIn<KIND, NW> in;
                in.c = chunk_geometry<NW>(j0, (uint32_t)col, (uint32_t)lat.L, (uint32_t)lat.log2L, half);
                load_words<NW>(own, j0, in.Wown);
                load_around<NW>(oth, j0, in.c, in.a);
                if (KIND == 1) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) in.HF[w] = HFc[col][w];
                }
                uint32_t W[NW], U[NW], Wnew[NW];
                const uint32_t any = chunk_flip_any<KIND, NW>(lat, sthr, never, in, F4c[col], g0, c1, r, beta, W,
                                                              U, Wnew);
                if (any) store_words<NW>(own, j0, Wnew);
                __syncthreads();
            }
        }
    } else {
    for (int sw = 0; sw < nsweep; ++sw) {
        for (uint32_t col = 0; col < 2; ++col) {
            uint8_t *own = sp + col * half;
            const uint8_t *oth = sp + (1u - col) * half;
            const uint32_t c1 = 2u * (t0 + (uint32_t)sw) + col;
            for (uint32_t ch = threadIdx.x; ch < nchunk; ch += blockDim.x) {
                const uint32_t g0 = ch * NW, j0 = 4u * g0;
                uint32_t W[NW], U[NW], Wnew[NW], F4[NW];
                const uint32_t any = chunk_update_any<KIND, NW>(lat, sthr, never, own, oth, fbits + (size_t)col * half,
                                                            fhf + (size_t)col * half, j0, g0, col, c1, r, beta,
                                                            W, U, Wnew, F4);
                if (any) store_words<NW>(own, j0, Wnew);
            }
            __syncthreads();
        }
    }
    }
    if (energy) {
        int ksum = 0, upsum = 0, eqsum = 0;
        double fsum = 0.0;
        const uint8_t *s1 = sp + half, *s0 = sp;
        for (uint32_t ch = threadIdx.x; ch < nchunk; ch += blockDim.x) {
            const uint32_t j0 = 4u * NW * ch;
            const Chunk c = chunk_geometry<NW>(j0, 1u, (uint32_t)lat.L, (uint32_t)lat.log2L, half);
            uint32_t S1[NW], W[NW], U[NW], F1[NW];
            load_words<NW>(s1, j0, S1);
            neighbour_counts<NW>(s0, j0, c, W, U);
            if (KIND == 0) load_words<NW>(fbits + half, j0, F1);
            chunk_energy<KIND, NW>(lat, S1, W, U, F1, fbits, fraw + half, fraw, j0, ksum, upsum, eqsum, fsum);
        }
        // every thread covered 4*NW sites per chunk it took; nsite per thread
        // differs, so fold the affine offsets into the total instead
        const int nch = (int)((nchunk > threadIdx.x) ? (nchunk - 1 - threadIdx.x) / blockDim.x + 1 : 0);
        block_partial<KIND>(gptr(lat.part) + (size_t)r * 3, 4 * NW * nch, ksum, upsum, eqsum, fsum);
    }
    GAS u32x4 *dst = (GAS u32x4 *)(gptr(lat.spins) + (size_t)r * N);
    for (uint32_t q = threadIdx.x; q < N / 16u; q += blockDim.x) dst[q] = lds4[q];
}

// ---------------------------------------------------------------------
// Slab sweeps (L = 16 or 32): each replica is cut along z into S slabs of
// L/S planes, one workgroup per (replica, slab), so that a few replicas
// still fill every CU.  A launch runs `nsweep` whole sweeps of the plain
// order: the workgroup stages its slab and 2 nsweep halo planes on each
// side (both colours) in LDS and runs the 2 nsweep half-sweeps there,
// half-sweep s updating the planes [s + 1, P - 1 - s) of the box; the
// outer planes it updates are other slabs', recomputed here from the same
// inputs and the same random words, so the slab's own planes end exactly
// as in the plain sweep and no workgroup waits for another.  The slab goes
// to `dst` (reading from `src`: a workgroup must not see a neighbour's new
// planes), and with `energy` the workgroup writes the energy partial of
// its slab.
//
// Work item: SW dwords (4 SW sites) of one row of one colour.  Thread t
// owns the box positions t, t + blockDim, ... (NP of them) for the whole
// launch and keeps their fields, both colours, in registers; a position is
// updated at the half-steps whose plane range holds it.  A plane has
// L * L / (8 SW) items: at L = 32 a wave's positions share one plane, so
// the test is uniform per wave.
// ---------------------------------------------------------------------
template <int KIND, int NP>
__global__ __launch_bounds__(1024) void sweep_slabs(Lattice lat, const uint8_t *__restrict__ src,
                                                     uint8_t *__restrict__ dst, int S, int nsweep, int toff,
                                                     int energy) {
    constexpr int SW = 2;
    extern __shared__ uint4 lds_raw[];
    __shared__ __align__(16) uint32_t sthr[32];   // +-1 thresholds or the continuous-field table
    uint8_t *box = (uint8_t *)lds_raw;                     // [P][2][plane]
    const uint32_t L = (uint32_t)lat.L, half = (uint32_t)lat.half;
    const uint32_t rowb = L >> 1;                          // bytes per row of one colour
    const uint32_t nwr = L >> 3;                           // dwords per row of one colour
    const uint32_t lipr = (uint32_t)lat.log2L - 4u;        // log2 of items per row (nwr / SW)
    const uint32_t ipr = 1u << lipr;
    const uint32_t plane = L * rowb;                       // bytes per plane of one colour
    const uint32_t ipp = L << lipr;                        // items per plane
    const uint32_t slab = L / (uint32_t)S;
    const uint32_t H = 2u * (uint32_t)nsweep;
    const uint32_t P = slab + 2u * H;
    const uint32_t r = blockIdx.x / (uint32_t)S, sl = blockIdx.x % (uint32_t)S;
    const uint32_t z0 = sl * slab;
    GAS const uint8_t *rsrc = gptr(src) + (size_t)r * lat.N;
    const int slot = gptr(lat.r2t)[r];
    const float beta = KIND == 1 ? gptr(lat.betaf)[slot] : 0.0f;
    const uint32_t t0 = (uint32_t)(gptr(lat.ctrs)[0] + (uint64_t)toff);
    GAS const uint8_t *fbits = gptr(lat.fbits);
    GAS const float *fhf = gptr(lat.fhf), *fraw = gptr(lat.fraw);
    // the positions of this thread and their fields (issued first, so the
    // field loads overlap the staging loads)
    uint32_t pb[NP], py[NP], pz[NP], pw[NP];
    uint32_t F4c[2][NP][SW];
    f32x4 HFc[2][NP][SW];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const uint32_t pos = threadIdx.x + (uint32_t)k * blockDim.x;
        const uint32_t rem = pos & (ipp - 1u);
        pb[k] = pos / ipp;                                 // P or more when the position is past the box
        py[k] = rem >> lipr;
        pw[k] = SW * (rem & (ipr - 1u));
        pz[k] = (z0 + L - H + pb[k]) & (L - 1u);
        const uint32_t j0 = (pz[k] * L + py[k]) * rowb + 4u * pw[k];
        if (pb[k] < P) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (KIND == 0) {
                    load_words<SW>(fbits + (size_t)c * half, j0, F4c[c][k]);
                } else {
#pragma unroll
                    for (int w = 0; w < SW; ++w)
                        HFc[c][k][w] = *(GAS const f32x4 *)(fhf + (size_t)c * half + j0 + 4u * w);
                }
            }
        }
    }
    // stage the box, 16 bytes at a time: plane b of the box is z0 - H + b
    const uint32_t per_plane16 = plane >> 4;
    const uint32_t n16 = P * 2u * per_plane16;
    for (uint32_t e = threadIdx.x; e < n16; e += blockDim.x) {
        const uint32_t q = e % per_plane16, bc = e / per_plane16;   // bc = 2 b + c
        const uint32_t b = bc >> 1, c = bc & 1u;
        const uint32_t zg = (z0 + L - H + b) & (L - 1u);
        ((u32x4 *)box)[e] = *(GAS const u32x4 *)(rsrc + (size_t)c * half + (size_t)zg * plane + 16u * q);
    }
    if (KIND == 0 && threadIdx.x < 32u) sthr[threadIdx.x] = gptr(lat.thr)[slot * 32 + threadIdx.x];
    if (KIND == 1) cont_table_fill(sthr, beta, lat.Jf);
    const uint32_t *bw = (const uint32_t *)box;
    const uint32_t ppw = plane >> 2;                       // dwords per colour-plane
    __syncthreads();
    const uint32_t never = KIND == 0 ? __builtin_amdgcn_readfirstlane(sthr[31]) : 0u;
    for (int sw = 0; sw < nsweep; ++sw) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const uint32_t st = 2u * (uint32_t)sw + (uint32_t)c;
            const uint32_t c1 = 2u * (t0 + (uint32_t)sw) + (uint32_t)c;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (pb[k] >= st + 1u && pb[k] + 1u + st < P) {
                    const uint32_t b = pb[k], y = py[k], w0 = pw[k], zg = pz[k];
                    const uint32_t rown = (2u * b + (uint32_t)c) * ppw + y * nwr;
                    const uint32_t oth = (2u * b + 1u - (uint32_t)c) * ppw;
                    ChunkIn<KIND, SW> in;
                    in.c.p = ((uint32_t)c + y + zg) & 1u;
#pragma unroll
                    for (int w = 0; w < SW; ++w) {
                        in.Wown[w] = bw[rown + w0 + w];
                        in.a.W[w] = bw[oth + y * nwr + w0 + w];
                        in.a.Wyp[w] = bw[oth + ((y + 1u) & (L - 1u)) * nwr + w0 + w];
                        in.a.Wym[w] = bw[oth + ((y - 1u) & (L - 1u)) * nwr + w0 + w];
                        in.a.Wzp[w] = bw[oth + 2u * ppw + y * nwr + w0 + w];
                        in.a.Wzm[w] = bw[oth - 2u * ppw + y * nwr + w0 + w];
                        if (KIND == 1) in.HF[w] = HFc[c][k][w];
                    }
                    in.a.Wx = bw[oth + y * nwr + ((w0 + (in.c.p ? (uint32_t)SW : nwr - 1u)) & (nwr - 1u))];
                    const uint32_t g0 = ((pz[k] * L + y) * rowb >> 2) + w0;
                    uint32_t W[SW], U[SW], Wnew[SW];
                    const uint32_t any = chunk_flip_any<KIND, SW>(lat, sthr, never, in, F4c[c][k], g0, c1, r, beta,
                                                                  W, U, Wnew);
                    if (any) {
#pragma unroll
                        for (int w = 0; w < SW; ++w) ((uint32_t *)box)[rown + w0 + w] = Wnew[w];
                    }
                }
            }
            __syncthreads();
        }
    }
    if (energy) {
        // the slab's colour-1 items against the final colour-0 planes (the
        // last colour-0 half-sweep covered the slab and one plane each side)
        int ksum = 0, upsum = 0, eqsum = 0, nch = 0;
        double fsum = 0.0;
        for (uint32_t it = threadIdx.x; it < slab * ipp; it += blockDim.x, ++nch) {
            const uint32_t bs = it >> ((uint32_t)lat.log2L + lipr), rem = it & (ipp - 1u);
            const uint32_t b = H + bs, y = rem >> lipr, w0 = SW * (rem & (ipr - 1u));
            const uint32_t zg = z0 + bs;
            const uint32_t j0 = (zg * L + y) * rowb + 4u * w0;
            const uint32_t o0 = (2u * b) * ppw;
            Around<SW> a;
            Chunk cg;
            cg.p = (1u + y + zg) & 1u;
            uint32_t S1[SW], U[SW], F1[SW];
#pragma unroll
            for (int w = 0; w < SW; ++w) {
                a.W[w] = bw[o0 + y * nwr + w0 + w];
                a.Wyp[w] = bw[o0 + ((y + 1u) & (L - 1u)) * nwr + w0 + w];
                a.Wym[w] = bw[o0 + ((y - 1u) & (L - 1u)) * nwr + w0 + w];
                a.Wzp[w] = bw[o0 + 2u * ppw + y * nwr + w0 + w];
                a.Wzm[w] = bw[o0 - 2u * ppw + y * nwr + w0 + w];
                S1[w] = bw[(2u * b + 1u) * ppw + y * nwr + w0 + w];
                F1[w] = 0u;
            }
            a.Wx = bw[o0 + y * nwr + ((w0 + (cg.p ? (uint32_t)SW : nwr - 1u)) & (nwr - 1u))];
            neighbour_sums<SW>(cg, a, U);
            if (KIND == 0) load_words<SW>(fbits + half, j0, F1);
            chunk_energy<KIND, SW>(lat, S1, a.W, U, F1, fbits, fraw + half, fraw, j0, ksum, upsum, eqsum, fsum);
        }
        block_partial<KIND>(gptr(lat.part) + ((size_t)sl * lat.pstride + r) * 3, 4 * SW * nch, ksum, upsum, eqsum,
                            fsum);
    }
    // the slab's planes, both colours
    GAS uint8_t *rdst = gptr(dst) + (size_t)r * lat.N;
    const uint32_t m16 = slab * 2u * per_plane16;
    for (uint32_t e = threadIdx.x; e < m16; e += blockDim.x) {
        const uint32_t q = e % per_plane16, bc = e / per_plane16;
        const uint32_t bs = bc >> 1, c = bc & 1u;
        *(GAS u32x4 *)(rdst + (size_t)c * half + (size_t)(z0 + bs) * plane + 16u * q) =
            ((const u32x4 *)box)[(2u * (H + bs) + c) * per_plane16 + q];
    }
}

// ---------------------------------------------------------------------
// Double checkerboard with multi-hit updates (Sec. 3.2, Sec. 5.2): one
// workgroup per (replica, tile of the coarse colour), tile of tx * ty * tz
// sites (tx a multiple of 8).  The tile and a one-site halo around it are
// staged in LDS in the colour-split row layout of global memory: per colour
// and per row (y, z) of the box (the tile's rows and one halo row on each
// side in y and z), tx/2 bytes of the tile's sites with one dword before
// (the left neighbour tile's last four sites of that colour) and one after
// (the right neighbour's first four).  Every thread owns one dword (four
// consecutive sites of a colour in a row) of each colour and runs `hits`
// local sweeps -- its colour-0 dword, a barrier, its colour-1 dword, a
// barrier -- with the same neighbour sums and decisions as the streaming
// sweep; the halo is never written, so the neighbouring tiles stay frozen.
// Hit m of sweep t draws the tag-2 block (j >> 2, 2 (t hits + m) + c, r).
// Then the tile goes back to global memory.
// ---------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(1024) void sweep_tiles(Lattice lat, TileShape ts, int coarse, int toff) {
    extern __shared__ uint4 lds_raw[];
    __shared__ __align__(16) uint32_t sthr[32];   // +-1 thresholds or the continuous-field table
    uint8_t *box = (uint8_t *)lds_raw;
    const uint32_t L = (uint32_t)lat.L, half = (uint32_t)lat.half;
    const uint32_t tx = (uint32_t)ts.tx, ty = (uint32_t)ts.ty, tz = (uint32_t)ts.tz;
    const uint32_t dwr = tx >> 3;                   // tile dwords per row and colour
    const uint32_t rowb = 4u * (dwr + 2u);          // bytes per box row (with the halo dwords)
    const uint32_t by = ty + 2u;
    const uint32_t plane = rowb * by * (tz + 2u);   // bytes per colour
    // block -> (replica, tile of the coarse colour)
    const uint32_t dxh = L / tx / 2u, Dy = L / ty;
    const uint32_t ntile = dxh * Dy * (L / tz);
    const uint32_t r = blockIdx.x / ntile, q = blockIdx.x % ntile;
    const uint32_t Y = (q / dxh) % Dy, Z = q / (dxh * Dy);
    const uint32_t X = 2u * (q % dxh) + (((uint32_t)coarse + Y + Z) & 1u);
    const uint32_t x0 = X * tx, y0 = Y * ty, z0 = Z * tz;
    GAS uint8_t *spins = gptr(lat.spins) + (size_t)r * lat.N;
    const int slot = gptr(lat.r2t)[r];
    if (KIND == 0 && threadIdx.x < 32u) sthr[threadIdx.x] = gptr(lat.thr)[slot * 32 + threadIdx.x];
    const float beta = KIND == 1 ? gptr(lat.betaf)[slot] : 0.0f;
    if (KIND == 1) cont_table_fill(sthr, beta, lat.Jf);
    const uint32_t t = (uint32_t)(gptr(lat.ctrs)[0] + (uint64_t)toff);
    // stage the box: both colours, every row of the box, the tile's dwords
    // and the two halo dwords (x, y, z wrap around the periodic lattice)
    const uint32_t nbox = 2u * (dwr + 2u) * by * (tz + 2u);
    for (uint32_t e = threadIdx.x; e < nbox; e += blockDim.x) {
        const uint32_t d = e % (dwr + 2u), row = (e / (dwr + 2u)) % (by * (tz + 2u));
        const uint32_t c = e / ((dwr + 2u) * by * (tz + 2u));
        const uint32_t yy = row % by, zz = row / by;
        const uint32_t x = (x0 + L + 8u * d - 8u) & (L - 1u);
        const uint32_t y = (y0 + L + yy - 1u) & (L - 1u), z = (z0 + L + zz - 1u) & (L - 1u);
        const uint32_t j = (x + L * (y + L * z)) >> 1;
        *(uint32_t *)(box + c * plane + row * rowb + 4u * d) =
            *(GAS const uint32_t *)(spins + (size_t)c * half + j);
    }
    // this thread's dword: four sites of row (y0 + yy, z0 + zz) from
    // x0 + 8w, in each colour
    const uint32_t w = threadIdx.x % dwr, yy = (threadIdx.x / dwr) % ty, zz = threadIdx.x / (dwr * ty);
    const uint32_t j0 = (x0 + 8u * w + L * ((y0 + yy) + L * (z0 + zz))) >> 1;
    const uint32_t g0 = j0 >> 2;
    const uint32_t mid = ((zz + 1u) * by + (yy + 1u)) * rowb + 4u * (w + 1u);
    uint32_t F4[2][1] = {{0u}, {0u}};
    f32x4 HF[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (KIND == 0) {
            F4[c][0] = *(GAS const uint32_t *)(gptr(lat.fbits) + (size_t)c * half + j0);
        } else {
            HF[c] = *(GAS const f32x4 *)(gptr(lat.fhf) + (size_t)c * half + j0);
        }
    }
    __syncthreads();
    const uint32_t never = KIND == 0 ? __builtin_amdgcn_readfirstlane(sthr[31]) : 0u;
    const uint32_t p0 = (y0 + yy + z0 + zz) & 1u;   // (c + y + z) & 1 for colour 0
    for (int m = 0; m < ts.hits; ++m) {
        const uint32_t step = t * (uint32_t)ts.hits + (uint32_t)m;
#pragma unroll
        for (uint32_t c = 0; c < 2; ++c) {
            const uint8_t *oth = box + (1u - c) * plane;
            ChunkIn<KIND, 1> in;
            in.c.p = p0 ^ c;
            in.Wown[0] = *(const uint32_t *)(box + c * plane + mid);
            in.a.W[0] = *(const uint32_t *)(oth + mid);
            in.a.Wx = *(const uint32_t *)(oth + mid + (in.c.p ? 4u : 0u - 4u));
            in.a.Wyp[0] = *(const uint32_t *)(oth + mid + rowb);
            in.a.Wym[0] = *(const uint32_t *)(oth + mid - rowb);
            in.a.Wzp[0] = *(const uint32_t *)(oth + mid + rowb * by);
            in.a.Wzm[0] = *(const uint32_t *)(oth + mid - rowb * by);
            if (KIND == 1) in.HF[0] = HF[c];
            uint32_t Wn[1], Un[1], Wnew[1];
            const uint32_t any = chunk_flip_any<KIND, 1>(lat, sthr, never, in, F4[c], g0, 2u * step + c, r, beta,
                                                         Wn, Un, Wnew);
            if (any) *(uint32_t *)(box + c * plane + mid) = Wnew[0];
            __syncthreads();
        }
    }
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c)
        *(GAS uint32_t *)(spins + (size_t)c * half + j0) = *(const uint32_t *)(box + c * plane + mid);
}

// ---------------------------------------------------------------------
// One bit per spin (multi-spin coding), L = 2^l in [64, 256].  Colour c of
// replica r is N/64 words; word w holds sublattice indices 32w..32w+31,
// index 32w + 4b + q at bit 8q + b, so that the four sites of Philox block
// 8w + b sit at bit b of the four bytes.  A row (y, z) of one colour is
// L/64 consecutive words.  One thread per word of the updated colour: the
// other colour's words around it are the pair word W (the same indices), W
// shifted by one index along the row with the neighbouring word's end bit
// (index m-1 when (c+y+z) is even, m+1 when odd, as in the byte layout),
// and the words of rows y+-1 and z+-1.  A bit-sliced full-adder tree turns
// the six into three planes of the up count; a bit transpose of the class
// planes gives every Philox block's byte-per-site table offsets, the
// operands of the byte sweep's decision, which runs on the same random
// words, so the chain is the same.  (Two words per thread, tried, ran the
// two-stream half-sweep 8 % slower: fewer waves to hide latency.)
// ---------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
// position of sublattice index i (0..31) within its word
__host__ __device__ constexpr uint32_t bit_of_index(uint32_t i) { return 8u * (i & 3u) + (i >> 2); }

// Exchange the bits of a at positions i + sh with the bits of b at
// positions i, for the positions i that mask m selects.
__device__ __forceinline__ void swap_bit_groups(uint32_t &a, uint32_t &b, uint32_t sh, uint32_t m) {
    const uint32_t t = ((a >> sh) ^ b) & m;
    b ^= t;
    a ^= t << sh;
}

// Table offsets of all eight Philox blocks of a word at once.  Byte q of
// plane k holds bit b for block b; the table offset of site (b, q) wants
// those five bits side by side, at bits 2 (f), 3 (s), 4..6 (up count).  With
// planes 0, 1 and 7 zero that is an 8x8 bit transpose inside every byte:
// three rounds of swapping bit groups of 4, 2 and 1 between planes, after
// which plane b is byte-per-site offset word A[b] = (U << 4) | (S << 3) | (F << 2)
// of block b.
__device__ __forceinline__ void class_offsets(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t s, uint32_t f,
                                              uint32_t (&A)[8]) {
    uint32_t x[8] = {0u, 0u, f, s, u0, u1, u2, 0u};
#pragma unroll
    for (int k = 0; k < 4; ++k) swap_bit_groups(x[k], x[k + 4], 4u, 0x0F0F0F0Fu);
    swap_bit_groups(x[0], x[2], 2u, 0x33333333u);
    swap_bit_groups(x[1], x[3], 2u, 0x33333333u);
    swap_bit_groups(x[4], x[6], 2u, 0x33333333u);
    swap_bit_groups(x[5], x[7], 2u, 0x33333333u);
#pragma unroll
    for (int k = 0; k < 8; k += 2) swap_bit_groups(x[k], x[k + 1], 1u, 0x55555555u);
#pragma unroll
    for (int b = 0; b < 8; ++b) A[b] = x[b];
}

constexpr int kBitsThreads = 256;

// Word i of a colour's bit array, addressed as a wave-uniform base plus a
// 32-bit byte offset (one vector register per load instead of a 64-bit
// address; i < 2^30 at every L that bit storage takes).
__device__ __forceinline__ uint32_t bits_word(GAS const uint32_t *base, uint32_t i) {
    return *(GAS const uint32_t *)((GAS const char *)base + (i << 2));
}

// Flip bits of one word of the bit sweep (its 32 sites, eight Philox
// blocks), in the word's bit order.  NEV: the slot has classes that can
// never flip (+-1 fields), checked per block; the common case runs
// without that check.  (Interleaving the blocks' Philox chains by hand,
// two, four or eight at a time, was no faster: the sweep is bound by
// instruction issue, not by the chains' latency.)
template <int KIND, bool NEV>
__device__ __forceinline__ uint32_t word_flips(const uint32_t *sthr, uint32_t never, const uint32_t (&Acls)[8],
                                               const f32x4 (&HF)[8], uint32_t w, uint32_t m0v, uint32_t c1w,
                                               uint32_t r, uint32_t c3w, uint32_t key0, uint32_t key1) {
    const uint8_t *tb = (const uint8_t *)sthr;
    uint32_t f0 = 0, f1 = 0, f2 = 0, f3 = 0;
#pragma unroll
    for (int b = 7; b >= 0; --b) {
        // block counters 8w + b: the first product M0 (8w + b) is one
        // multiply-add of 8w with the constant M0 b
        const Words rw = philox10_p(mad_m0(8u * w, m0v, (uint64_t)kPhiloxM0 * (uint32_t)b), 8u * w + b, c1w, r,
                                    c3w, key0, key1);
        const uint32_t A = Acls[b];
        const uint32_t a0 = A & 0xFFu, a1 = __builtin_amdgcn_ubfe(A, 8u, 8u), a2 = (A >> 16) & 0xFFu, a3 = A >> 24;
        if (KIND == 0) {
            const uint32_t th0 = *(const uint32_t *)(tb + a0), th1 = *(const uint32_t *)(tb + a1);
            const uint32_t th2 = *(const uint32_t *)(tb + a2), th3 = *(const uint32_t *)(tb + a3);
            accept_shift(rw.w0, rw.w1, rw.w2, rw.w3, th0, th1, th2, th3, f0, f1, f2, f3);
            if (NEV) {
                // a class that can never flip at this temperature has entry
                // 0, which u = 0 would meet: clear the bit just shifted in
                const uint32_t umin = min(min(rw.w0, rw.w1), min(rw.w2, rw.w3));
                if (umin == 0u) {
                    if (rw.w0 == 0u && ((never >> (a0 >> 2)) & 1u)) f0 &= ~1u;
                    if (rw.w1 == 0u && ((never >> (a1 >> 2)) & 1u)) f1 &= ~1u;
                    if (rw.w2 == 0u && ((never >> (a2 >> 2)) & 1u)) f2 &= ~1u;
                    if (rw.w3 == 0u && ((never >> (a3 >> 2)) & 1u)) f3 &= ~1u;
                }
            }
        } else {
            const f32x4 hf = HF[b];
            const uint32_t t0 = cont_bound(tb, a0, hf.x), t1 = cont_bound(tb, a1, hf.y);
            const uint32_t t2 = cont_bound(tb, a2, hf.z), t3 = cont_bound(tb, a3, hf.w);
            accept_shift(rw.w0, rw.w1, rw.w2, rw.w3, t0, t1, t2, t3, f0, f1, f2, f3);
        }
    }
    return f0 | (f1 << 8) | (f2 << 16) | (f3 << 24);
}

__host__ __device__ constexpr int bits_wg(int L) { return L == 64 ? 128 : 256; }

// BATCH: the replicas of several realizations that share L and the field
// kind, one map entry per replica (x = (realization << 16) | replica) and
// 2^lbpr workgroups each; else replicas r0.. of lat0.
template <int KIND, int ENERGY, bool BATCH>
__global__ __launch_bounds__(kBitsThreads) void sweep_bits(Lattice lat0, const Lattice *__restrict__ lats,
                                                          const uint2 *__restrict__ map, int colour, int toff,
                                                          int r0, int lbpr, int remap) {
    __shared__ __align__(16) uint32_t sthr[32];   // +-1 thresholds or the continuous-field table
    uint32_t blk = blockIdx.x;
    if (remap) {
        const uint32_t per = gridDim.x >> 3;
        blk = (blk & 7u) * per + (blk >> 3);
    }
    const uint32_t e = BATCH ? map[blk >> lbpr].x : 0u;
    const Lattice &lat = BATCH ? lats[e >> 16] : lat0;
    const uint32_t r = BATCH ? (e & 0xFFFFu) : (uint32_t)r0 + (blk >> lbpr);
    const uint32_t gb = blk & ((1u << lbpr) - 1u);
    const uint32_t L = (uint32_t)lat.L, l = (uint32_t)lat.log2L;
    const uint32_t W1 = (uint32_t)lat.N >> 6;            // words per colour
    const uint32_t lrw = l - 6u, rw_ = 1u << lrw;        // words per row
    // w = (z L + y) rw_ + wr: the bit fields of wr, y and z side by side, so
    // a neighbour's word is w stepped inside one field and put back (the
    // step's carry or borrow out of the field masked off: periodic wrap)
    const uint32_t w = gb * blockDim.x + threadIdx.x;
    const uint32_t c = (uint32_t)colour;
    const uint32_t p = (c + (w >> lrw) + (w >> (lrw + l))) & 1u;      // (c + y + z) mod 2
    const uint32_t xm = rw_ - 1u, ym = (L - 1u) << lrw, zm = ym << l;
    const uint32_t wx = ((w + 2u * p - 1u) & xm) | (w & ~xm);          // the word holding index m -+ 1
    const uint32_t wyp = ((w + rw_) & ym) | (w & ~ym), wym = ((w - rw_) & ym) | (w & ~ym);
    const uint32_t wzp = ((w + (rw_ << l)) & zm) | (w & ~zm), wzm = ((w - (rw_ << l)) & zm) | (w & ~zm);
    GAS uint32_t *own = gptr(lat.bits) + ((size_t)r * 2u + c) * W1;
    GAS const uint32_t *oth = gptr(lat.bits) + ((size_t)r * 2u + (1u - c)) * W1;
    const uint32_t S = bits_word(own, w);
    const uint32_t W = bits_word(oth, w);
    const uint32_t Wn = bits_word(oth, wx);
    const uint32_t Wyp = bits_word(oth, wyp), Wym = bits_word(oth, wym);
    const uint32_t Wzp = bits_word(oth, wzp), Wzm = bits_word(oth, wzm);
    uint32_t F = 0;
    f32x4 HF[8];
    if (KIND == 0) {
        F = gptr(lat.fbw)[(size_t)c * W1 + w];
    } else {
        GAS const f32x4 *hf = (GAS const f32x4 *)(gptr(lat.fhw) + (size_t)c * lat.half) +
                              (size_t)(w >> 6) * 512u + (w & 63u);
#pragma unroll
        for (int b = 0; b < 8; ++b) HF[b] = hf[b * 64];
    }
    __builtin_amdgcn_sched_barrier(0);
    const int slot = gptr(lat.r2t)[r];
    const uint32_t t = (uint32_t)(gptr(lat.ctrs)[0] + (uint64_t)toff);
    uint32_t never = 0;
    const float beta = KIND == 1 ? gptr(lat.betaf)[slot] : 0.0f;
    if (KIND == 0) {
        if (threadIdx.x < 32u) sthr[threadIdx.x] = gptr(lat.thr)[slot * 32 + threadIdx.x];
        __syncthreads();
        never = __builtin_amdgcn_readfirstlane(sthr[31]);
    } else {
        cont_table_fill(sthr, beta, lat.Jf);
        __syncthreads();
    }
    // the x neighbour, index m-1 (p = 0) or m+1 (p = 1), in the interleaved
    // order: a step of one index is a step of one byte, with the carry
    // between byte 3 and byte 0 one bit along, and the end bit from the
    // neighbouring word of the row (around the row)
    const uint32_t Wx = p ? ((W >> 8) | ((W << 23) & 0x7F000000u) | (Wn << 31))
                          : ((W << 8) | ((W >> 23) & 0x000000FEu) | (Wn >> 31));
    // up count of the six neighbours in three bit planes
    const uint32_t s1 = xor3(W, Wx, Wyp), c1 = maj3(W, Wx, Wyp);
    const uint32_t s2 = xor3(Wym, Wzp, Wzm), c2 = maj3(Wym, Wzp, Wzm);
    const uint32_t U0 = s1 ^ s2, c3 = s1 & s2;
    const uint32_t U1 = xor3(c1, c2, c3), U2 = maj3(c1, c2, c3);
    const uint32_t c1w = 2u * t + c, c3w = (kTagSweep << 28) | lat.rho;
    uint32_t Acls[8];
    class_offsets(U0, U1, U2, S, KIND == 0 ? F : 0u, Acls);
    const uint32_t m0v = __builtin_amdgcn_readfirstlane(kPhiloxM0);   // held in one VGPR below
    // `never` is the same for the whole workgroup: the common case (no class
    // that can never flip) runs without the per-block check
    const uint32_t flips =
        KIND == 0 && never != 0u
            ? word_flips<KIND, true>(sthr, never, Acls, HF, w, m0v, c1w, r, c3w, lat.key0, lat.key1)
            : word_flips<KIND, false>(sthr, never, Acls, HF, w, m0v, c1w, r, c3w, lat.key0, lat.key1);
    const uint32_t Snew = S ^ flips;
    if (flips) *(GAS uint32_t *)((GAS char *)own + (w << 2)) = Snew;
    if (ENERGY) {
        // colour 1 of the last sweep before an exchange: the final state.
        // B counts each bond once through the colour-1 sites: sum of
        // s_i n_i = 2 K - 6 with K the aligned neighbours (up if s = +1,
        // 6 - up if s = -1).
        const uint32_t nS = ~Snew;
        const int up_on = __popc(U0 & Snew) + 2 * __popc(U1 & Snew) + 4 * __popc(U2 & Snew);
        const int up_off = __popc(U0 & nS) + 2 * __popc(U1 & nS) + 4 * __popc(U2 & nS);
        const int ksum = up_on + 6 * (32 - __popc(Snew)) - up_off;
        const int upsum = __popc(Snew) + __popc(W);
        int eqsum = 0;
        double fsum = 0.0;
        if (KIND == 0) {
            const uint32_t F0 = gptr(lat.fbw)[w];
            eqsum = __popc(~(Snew ^ F)) + __popc(~(W ^ F0));
        } else {
            GAS const float *f1 = gptr(lat.fraw) + lat.half + 32u * w;
            GAS const float *f0 = gptr(lat.fraw) + 32u * w;
#pragma unroll 8
            for (uint32_t i = 0; i < 32; ++i) {
                const uint32_t q = bit_of_index(i);
                fsum += ((Snew >> q) & 1u) ? (double)f1[i] : -(double)f1[i];
                fsum += ((W >> q) & 1u) ? (double)f0[i] : -(double)f0[i];
            }
        }
        block_partial<KIND>(gptr(lat.part) + ((size_t)gb * lat.pstride + r) * 3, 32, ksum, upsum, eqsum, fsum);
    }
}

// Byte spins <-> bit spins (one thread per 32-site word) and the +-1 field
// words.
__global__ __launch_bounds__(256) void pack_bits_kernel(Lattice lat) {
    const uint32_t W1 = (uint32_t)lat.N >> 6;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;     // word of (replica, colour)
    if (e >= (uint32_t)lat.R * 2u * W1) return;
    const uint8_t *src = lat.spins + (size_t)e * 32u;       // [r][c][32w..] matches the byte layout
    uint32_t v = 0;
#pragma unroll
    for (uint32_t i = 0; i < 32; ++i) v |= (uint32_t)(src[i] & 1u) << bit_of_index(i);
    lat.bits[e] = v;
    if (e < 2u * W1 && lat.kind == 0) {
        uint32_t f = 0;
        const uint8_t *fb = lat.fbits + (size_t)e * 32u;
#pragma unroll
        for (uint32_t i = 0; i < 32; ++i) f |= (uint32_t)((fb[i] >> 2) & 1u) << bit_of_index(i);
        ((uint32_t *)lat.fbw)[e] = f;
    }
    if (e < 2u * W1 && lat.kind == 1) {
        // word w of colour c: its eight float4 blocks to the bit sweep's order
        const uint32_t c = e / W1, w = e - c * W1;
        const f32x4 *src4 = (const f32x4 *)(lat.fhf + (size_t)c * lat.half) + (size_t)w * 8u;
        f32x4 *dst4 = (f32x4 *)(lat.fhw + (size_t)c * lat.half) + (size_t)(w >> 6) * 512u + (w & 63u);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) dst4[b * 64u] = src4[b];
    }
}

__global__ __launch_bounds__(256) void unpack_bits_kernel(Lattice lat) {
    const uint32_t W1 = (uint32_t)lat.N >> 6;
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= (uint32_t)lat.R * 2u * W1) return;
    const uint32_t v = lat.bits[e];
    uint8_t *dst = lat.spins + (size_t)e * 32u;
#pragma unroll
    for (uint32_t i = 0; i < 32; ++i) dst[i] = (uint8_t)((v >> bit_of_index(i)) & 1u);
}

// ---------------------------------------------------------------------
// Energy partials (Eq. 1).  Every bond joins a colour-0 and a colour-1
// site, so B = sum over colour-1 sites of s_i n_i counts each bond once;
// F and M run over both colours.  Grid (nblk, R); fixed reduction order.
// ---------------------------------------------------------------------
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
                const int f1 = (lat.fbits[lat.half + j] >> 1) - 1, f0 = (lat.fbits[j] >> 1) - 1;
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
        lat.part[((size_t)blockIdx.x * lat.pstride + r) * 3 + threadIdx.x] = v;
    }
}

__device__ __forceinline__ double energy_of(const Lattice &lat, double B, double F) {
    return -(lat.J * B) - (lat.h * F);
}

// ---------------------------------------------------------------------
// Exchange step k (Eq. 2): pairs (p, p+1) with p = k mod 2; temperatures
// move through t2r / r2t (Sec. 3.3).  One workgroup of kExchangeThreads.
// ---------------------------------------------------------------------
constexpr int kExchangeThreads = 1024;

// Energy and magnetisation of every replica from its partials (B, F, M per
// block, block-major).  Thread (g, r) sums blocks [g per, min((g+1) per,
// nblk)) of replica r in order -- consecutive threads take consecutive
// replicas, so every load is coalesced -- issuing up to 8 blocks' loads
// before it adds any, so the range costs a few memory round trips rather than
// one per block; then one thread per replica adds its G range sums in order.
// nblk need not be a power of two (the generic kernel's is not).  The order
// is fixed for a given launch shape and replica count, so FP64 totals are
// reproducible.  Writes E and Mr, and B, F, M when asked (observables).
template <int B>
__device__ __forceinline__ void sum_range(GAS const double *pp, size_t qstride, int q_end, double &b, double &f,
                                          double &m) {
    for (int q0 = 0; q0 < q_end; q0 += B) {
        // loads past the range re-read its last block (always in bounds, no
        // branch between the loads); their adds are skipped
        double vb[B], vf[B], vm[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            GAS const double *pq = pp + (size_t)min(q0 + j, q_end - 1) * qstride;
            vb[j] = pq[0];
            vf[j] = pq[1];
            vm[j] = pq[2];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const bool in = q0 + j < q_end;
            b = in ? b + vb[j] : b;
            f = in ? f + vf[j] : f;
            m = in ? m + vm[j] : m;
        }
    }
}

__device__ __forceinline__ void replica_totals(const Lattice &lat, int64_t *Bout = nullptr,
                                               double *Fout = nullptr, int64_t *Mout = nullptr,
                                               double *sE = nullptr, double *sM = nullptr) {
    __shared__ double red[kExchangeThreads * 3];
    const int R = lat.R, nblk = lat.nblk;
    int G = 1;
    while (2 * G <= nblk && 2 * G <= 64 && (long long)R * 2 * G <= kExchangeThreads) G *= 2;
    const int tile = kExchangeThreads / G, per = (nblk + G - 1) / G;
    const int g = (int)threadIdx.x / tile, rl = (int)threadIdx.x % tile;
    const int q_end = min(per, nblk - g * per);   // blocks in this thread's range (may be <= 0)
    const size_t qstride = (size_t)lat.pstride * 3;
    for (int r0 = 0; r0 < R; r0 += tile) {
        const int r = r0 + rl;
        double b = 0.0, f = 0.0, m = 0.0;
        if (r < R) {
            GAS const double *pp = gptr(lat.part) + ((size_t)g * per * lat.pstride + r) * 3;
            if (per == 1)       // the batch width follows the range (uniform per block)
                sum_range<1>(pp, qstride, q_end, b, f, m);
            else if (per == 2)
                sum_range<2>(pp, qstride, q_end, b, f, m);
            else if (per <= 4)
                sum_range<4>(pp, qstride, q_end, b, f, m);
            else
                sum_range<8>(pp, qstride, q_end, b, f, m);
        }
        red[3 * threadIdx.x + 0] = b;
        red[3 * threadIdx.x + 1] = f;
        red[3 * threadIdx.x + 2] = m;
        __syncthreads();
        if ((int)threadIdx.x < tile && r0 + (int)threadIdx.x < R) {
            double B = red[3 * threadIdx.x + 0], F = red[3 * threadIdx.x + 1], M = red[3 * threadIdx.x + 2];
            for (int q = 1; q < G; ++q) {
                const double *rr = red + 3 * (q * tile + threadIdx.x);
                B += rr[0];
                F += rr[1];
                M += rr[2];
            }
            const int rt = r0 + (int)threadIdx.x;
            const double E = energy_of(lat, B, F);
            lat.E[rt] = E;
            lat.Mr[rt] = M;
            if (sE) {
                sE[rt] = E;
                sM[rt] = M;
            }
            if (Bout) Bout[rt] = (int64_t)B;
            if (Fout) Fout[rt] = F;
            if (Mout) Mout[rt] = (int64_t)M;
        }
        __syncthreads();
    }
}

// Totals per replica id for the observables calls (same reduction as the
// exchange step, so both give the same bits).
__global__ __launch_bounds__(kExchangeThreads) void reduce_kernel(Lattice lat, int64_t *Bout, double *Fout,
                                                                  int64_t *Mout) {
    replica_totals(lat, Bout, Fout, Mout);
}

// The decision for pair (p, p+1) of exchange step k: Philox word pair ->
// a uniform double in [0, 1) with 53 random bits, accepted if Delta >= 0 or
// u < e^Delta.
__device__ __forceinline__ bool exchange_accept(const Lattice &lat, int p, uint64_t k, double delta) {
    const Words w = philox10((uint32_t)p, (uint32_t)k, 0u, (kTagExch << 28) | lat.rho, lat.key0, lat.key1);
    const double u53 = ((double)(w.w0 >> 11) * 4294967296.0 + (double)w.w1) * 0x1p-53;
    return delta >= 0.0 || u53 < exp(delta);
}

// One exchange step per workgroup (one realization each).  Up to
// kExchangeThreads replicas the step runs out of LDS: the permutation, the
// inverse temperatures, the slot's observable sums and the pair counters are
// loaded together with the energy partials, so the whole step costs about
// two memory round trips; more replicas take the same steps through global
// memory.
__global__ __launch_bounds__(kExchangeThreads) void exchange_kernel(const Lattice *__restrict__ lats, int tadv) {
    __shared__ double sE[kExchangeThreads], sM[kExchangeThreads];
    __shared__ int32_t st2r[kExchangeThreads];
    const Lattice &lat = lats[blockIdx.x];
    const uint64_t k = lat.ctrs[1];
    const int R = lat.R, t = (int)threadIdx.x;
    if (R <= kExchangeThreads) {
        // inputs that do not depend on the energies, fetched first
        const bool mine = t < R;
        const int tc = mine ? t : 0;
        // (global-typed loads: flat ones would also hold up the scalar waits)
        const int32_t my_t2r = gptr(lat.t2r)[tc];
        GAS const double *beta = gptr(lat.beta);
        const double my_beta = beta[tc], my_beta1 = beta[min(tc + 1, R - 1)];
        const bool pair = t + 1 < R && (t & 1) == (int)(k & 1);
        const int pc = min(tc, max(R - 2, 0));
        const uint64_t my_att = gptr(lat.att)[pc], my_acc = gptr(lat.acc)[pc];
        double o[6];
        GAS const double *orow = gptr(lat.obs) + 6 * (size_t)tc;
#pragma unroll
        for (int q = 0; q < 6; ++q) o[q] = orow[q];
        replica_totals(lat, nullptr, nullptr, nullptr, sE, sM);
        if (mine) st2r[t] = my_t2r;
        __syncthreads();
        // pairs (p, p+1) with p = k mod 2: thread p decides its pair; the
        // pairs are disjoint, so every slot is written by at most one thread
        if (pair) {
            const int a = st2r[t], b = st2r[t + 1];
            const double delta = (my_beta1 - my_beta) * (sE[b] - sE[a]);
            lat.att[t] = my_att + 1;
            if (exchange_accept(lat, t, k, delta)) {
                lat.acc[t] = my_acc + 1;
                st2r[t] = b;
                st2r[t + 1] = a;
                lat.t2r[t] = b;
                lat.t2r[t + 1] = a;
                lat.r2t[a] = t + 1;
                lat.r2t[b] = t;
            }
        }
        __syncthreads();
        // one measurement per exchange step (Sec. 7), by temperature slot
        if (mine) {
            const int a = st2r[t];
            const double e = sE[a], m = sM[a], m2 = m * m;
            double *op = lat.obs + 6 * (size_t)t;
            op[0] = o[0] + 1.0;
            op[1] = o[1] + e;
            op[2] = o[2] + e * e;
            op[3] = o[3] + fabs(m);
            op[4] = o[4] + m2;
            op[5] = o[5] + m2 * m2;
        }
    } else {
        replica_totals(lat);
        __syncthreads();
        for (int p = (int)(k & 1) + 2 * t; p + 1 < R; p += 2 * kExchangeThreads) {
            const int a = lat.t2r[p], b = lat.t2r[p + 1];
            const double delta = (lat.beta[p + 1] - lat.beta[p]) * (lat.E[b] - lat.E[a]);
            lat.att[p] += 1;
            if (exchange_accept(lat, p, k, delta)) {
                lat.t2r[p] = b;
                lat.t2r[p + 1] = a;
                lat.r2t[a] = p + 1;
                lat.r2t[b] = p;
                lat.acc[p] += 1;
            }
        }
        __syncthreads();
        for (int q = t; q < R; q += kExchangeThreads) {
            const int a = lat.t2r[q];
            const double e = lat.E[a], m = lat.Mr[a], m2 = m * m;
            double *o = lat.obs + 6 * (size_t)q;
            o[0] += 1.0;
            o[1] += e;
            o[2] += e * e;
            o[3] += fabs(m);
            o[4] += m2;
            o[5] += m2 * m2;
        }
    }
    if (threadIdx.x == 0) {
        lat.ctrs[0] += (uint64_t)tadv;
        lat.ctrs[1] = k + 1;
    }
}

__global__ void advance_kernel(uint64_t *ctrs, int tadv) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctrs[0] += (uint64_t)tadv;
}

}  // namespace

bool shape_valid(int L, int mode, int nw, int wg) {
    const bool pow2 = L >= 8 && (L & (L - 1)) == 0;
    if (!pow2) return mode == 0 && nw == 0 && wg == 0;      // generic kernel, fixed shape
    if (mode >= 2 && mode <= 4) {
        // slabs: nw = slabs per replica, mode - 1 sweeps per launch
        if (L != 16 && L != 32) return false;
        if (nw != 2 && nw != 4 && nw != 8) return false;
        if (L / nw < 2) return false;
        if (L / nw + 4 * slab_sweeps_per_launch(mode) > L) return false;   // the box must not wrap onto itself
        if (slab_lds_bytes(L, mode, nw) > 65536) return false;
        if (wg != 128 && wg != 256 && wg != 512 && wg != 1024) return false;
        return slab_positions_per_thread(L, mode, nw, wg) <= 2;
    }
    if (nw != 1 && nw != 2 && nw != 4 && nw != 8) return false;
    if (4 * nw > L / 2) return false;                        // a chunk lies inside one row
    const long long chunks = (long long)L * L * L / 8 / nw;  // per colour and replica
    if (mode == 0) {
        if (wg != 64 && wg != 128 && wg != 256) return false;
        return chunks % wg == 0 || chunks < wg;
    }
    if (mode == 1) {
        if (L > 32 || nw > 4) return false;                  // one replica must fit in LDS
        return wg == 64 || wg == 128 || wg == 256 || wg == 512 || wg == 1024;
    }
    return false;
}

int blocks_per_replica(int L, int mode, int nw, int wg) {
    const bool pow2 = L >= 8 && (L & (L - 1)) == 0;
    if (!pow2) {
        const long long G = (long long)L * L * L / 8;
        long long nb = (G + 255) / 256;
        if (nb > 64) nb = 64;
        return (int)(nb < 1 ? 1 : nb);
    }
    if (mode == 1) return 1;
    if (mode >= 2) return nw;                                // one partial per slab
    const long long chunks = (long long)L * L * L / 8 / nw;
    if (chunks < wg) return 1;
    const long long nb = chunks / wg;
    return nb > kMaxFusedBlocks ? 64 : (int)nb;
}

int stream_blocks_per_replica(int L, int nw, int wg) {
    const long long chunks = (long long)L * L * L / 8 / nw;
    const long long w = chunks < wg ? chunks : wg;
    return (int)(chunks / w);
}

bool fused_energy(const Lattice &lat) {
    if (lat.log2L < 3) return false;
    if (lat.mode >= 1) return true;
    const long long chunks = (long long)lat.N / 8 / lat.nw;
    return chunks <= (long long)lat.wg * kMaxFusedBlocks;
}

hipError_t launch_init(const Lattice &lat, int r0, int r1, hipStream_t s) {
    if (r1 <= r0) return hipSuccess;
    const int G = lat.N >> 2;
    dim3 grid((G + 255) / 256, r1 - r0);
    hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, s, lat, r0);
    return hipGetLastError();
}

template <int KIND, int ENERGY, bool BATCH>
static void launch_pow2(const Launch &ln, const Lattice &lat0, int colour, int toff, hipStream_t s) {
    const int remap = (ln.nblocks % 8 == 0) ? 1 : 0;
    // a replica smaller than one workgroup gets a workgroup of its size:
    // the block map counts one block per replica then, and every thread of
    // a block must own a chunk of that replica
    const long long chunks = (long long)ln.L * ln.L * ln.L / 8 / ln.nw;
    const int wg = chunks < ln.wg ? (int)chunks : ln.wg;
    const int lwpr = __builtin_ctzll((unsigned long long)(chunks / wg));   // a power of two
    const dim3 grid(ln.nblocks), block(wg);
    if (ln.nw == 8)
        hipLaunchKernelGGL((sweep_pow2<KIND, 8, ENERGY, BATCH>), grid, block, 0, s, lat0, ln.lats, ln.map, colour,
                           toff, remap, lwpr, ln.r0);
    else if (ln.nw == 4)
        hipLaunchKernelGGL((sweep_pow2<KIND, 4, ENERGY, BATCH>), grid, block, 0, s, lat0, ln.lats, ln.map, colour,
                           toff, remap, lwpr, ln.r0);
    else if (ln.nw == 2)
        hipLaunchKernelGGL((sweep_pow2<KIND, 2, ENERGY, BATCH>), grid, block, 0, s, lat0, ln.lats, ln.map, colour,
                           toff, remap, lwpr, ln.r0);
    else
        hipLaunchKernelGGL((sweep_pow2<KIND, 1, ENERGY, BATCH>), grid, block, 0, s, lat0, ln.lats, ln.map, colour,
                           toff, remap, lwpr, ln.r0);
}

// Workgroups of `kernel` one CU holds at once (0 if unknown), cached in
// `slot` (-1: not asked yet), and the current device's CU count.
static int resident_blocks_per_cu(std::atomic<int> &slot, const void *kernel, int wg, size_t lds) {
    int n = slot.load(std::memory_order_relaxed);
    if (n >= 0) return n;
    n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, wg, lds) != hipSuccess) {
        (void)hipGetLastError();
        n = 0;
    }
    slot.store(n, std::memory_order_relaxed);
    return n;
}

static int device_cus() {
    static std::atomic<int> cache[16] = {};
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (dev >= 0 && dev < 16 && (n = cache[dev].load(std::memory_order_relaxed)) > 0) return n;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (dev >= 0 && dev < 16) cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

template <int KIND, int NW, bool BATCH>
static void launch_res_nw(const Launch &ln, const Lattice &lat0, int nsweep, int energy, hipStream_t s) {
    const size_t lds = (size_t)ln.L * ln.L * ln.L;
    const dim3 grid(ln.nblocks), block(ln.wg);
    // one chunk per thread and colour: the register-field form, unless its
    // extra registers would leave fewer workgroups per CU than the plain
    // form while there are more workgroups than the device holds at once
    bool one = (long long)ln.L * ln.L * ln.L / 8 / NW == ln.wg;
    if (one) {
        // per instantiation, (L, wg) is fixed by chunks == wg up to the two
        // L of NW = 1; index the cache by L
        static std::atomic<int> occ[2][6] = {{-1, -1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1, -1}};
        const int li = ln.L == 8 ? 0 : (ln.L == 16 ? 1 : (ln.L == 32 ? 2 : 3));
        const int b1 = resident_blocks_per_cu(occ[1][li], (const void *)sweep_resident<KIND, NW, BATCH, true>,
                                              ln.wg, lds);
        const int b0 = resident_blocks_per_cu(occ[0][li], (const void *)sweep_resident<KIND, NW, BATCH, false>,
                                              ln.wg, lds);
        const long long cus = device_cus();
        if (b1 < b0 && (long long)ln.nblocks > cus * b1) one = false;
    }
    if (one)
        hipLaunchKernelGGL((sweep_resident<KIND, NW, BATCH, true>), grid, block, lds, s, lat0, ln.lats, ln.map,
                           nsweep, energy);
    else
        hipLaunchKernelGGL((sweep_resident<KIND, NW, BATCH, false>), grid, block, lds, s, lat0, ln.lats, ln.map,
                           nsweep, energy);
}

template <int KIND, bool BATCH>
static void launch_res(const Launch &ln, const Lattice &lat0, int nsweep, int energy, hipStream_t s) {
    if (ln.nw == 4)
        launch_res_nw<KIND, 4, BATCH>(ln, lat0, nsweep, energy, s);
    else if (ln.nw == 2)
        launch_res_nw<KIND, 2, BATCH>(ln, lat0, nsweep, energy, s);
    else
        launch_res_nw<KIND, 1, BATCH>(ln, lat0, nsweep, energy, s);
}

hipError_t launch_stream_sweep(const Launch &ln, int colour, int toff, int energy, hipStream_t s) {
    if (ln.nblocks == 0) return hipSuccess;
    const bool e = energy && colour == 1;
    const bool b = ln.single == nullptr;
    const Lattice lat0 = b ? Lattice{} : *ln.single;
    if (ln.kind == 0) {
        if (e) b ? launch_pow2<0, 1, true>(ln, lat0, colour, toff, s) : launch_pow2<0, 1, false>(ln, lat0, colour, toff, s);
        else b ? launch_pow2<0, 0, true>(ln, lat0, colour, toff, s) : launch_pow2<0, 0, false>(ln, lat0, colour, toff, s);
    } else {
        if (e) b ? launch_pow2<1, 1, true>(ln, lat0, colour, toff, s) : launch_pow2<1, 1, false>(ln, lat0, colour, toff, s);
        else b ? launch_pow2<1, 0, true>(ln, lat0, colour, toff, s) : launch_pow2<1, 0, false>(ln, lat0, colour, toff, s);
    }
    return hipGetLastError();
}

hipError_t launch_resident(const Launch &ln, int nsweep, int energy, hipStream_t s) {
    if (ln.nblocks == 0) return hipSuccess;
    const bool b = ln.single == nullptr;
    const Lattice lat0 = b ? Lattice{} : *ln.single;
    if (ln.kind == 0) b ? launch_res<0, true>(ln, lat0, nsweep, energy, s) : launch_res<0, false>(ln, lat0, nsweep, energy, s);
    else b ? launch_res<1, true>(ln, lat0, nsweep, energy, s) : launch_res<1, false>(ln, lat0, nsweep, energy, s);
    return hipGetLastError();
}

hipError_t launch_generic_sweep(const Lattice &lat, int colour, int toff, hipStream_t s) {
    const int G = lat.half >> 2;
    dim3 grid((G + 255) / 256, lat.R);
    if (lat.kind == 0)
        hipLaunchKernelGGL(sweep_generic<0>, grid, dim3(256), 0, s, lat, colour, toff);
    else
        hipLaunchKernelGGL(sweep_generic<1>, grid, dim3(256), 0, s, lat, colour, toff);
    return hipGetLastError();
}

int slab_sweeps_per_launch(int mode) { return mode >= 2 ? mode - 1 : 0; }

size_t slab_lds_bytes(int L, int mode, int nslab) {
    const int P = L / nslab + 4 * slab_sweeps_per_launch(mode);
    return (size_t)P * (size_t)L * L;          // both colours: L^2 / 2 bytes each
}

int slab_positions_per_thread(int L, int mode, int nslab, int wg) {
    const long long items = (long long)(L / nslab + 4 * slab_sweeps_per_launch(mode)) * L * L / 16;
    return (int)((items + wg - 1) / wg);
}

template <int KIND>
static void launch_slab_kind(const Lattice &lat, const uint8_t *src, uint8_t *dst, int np, int nslab, int wg,
                             size_t lds, int nsweep, int toff, int energy, hipStream_t s) {
    const dim3 grid((unsigned)(lat.R * nslab)), block((unsigned)wg);
    if (np == 1)
        hipLaunchKernelGGL((sweep_slabs<KIND, 1>), grid, block, lds, s, lat, src, dst, nslab, nsweep, toff, energy);
    else
        hipLaunchKernelGGL((sweep_slabs<KIND, 2>), grid, block, lds, s, lat, src, dst, nslab, nsweep, toff, energy);
}

hipError_t launch_slab_sweep(const Lattice &lat, const uint8_t *src, uint8_t *dst, int mode, int nslab, int wg,
                             int nsweep, int toff, int energy, hipStream_t s) {
    const size_t lds = slab_lds_bytes(lat.L, mode, nslab);
    const int np = slab_positions_per_thread(lat.L, mode, nslab, wg);
    if (np < 1 || np > 2 || nsweep < 1 || nsweep > slab_sweeps_per_launch(mode)) return hipErrorInvalidValue;
    if (lat.kind == 0)
        launch_slab_kind<0>(lat, src, dst, np, nslab, wg, lds, nsweep, toff, energy, s);
    else
        launch_slab_kind<1>(lat, src, dst, np, nslab, wg, lds, nsweep, toff, energy, s);
    return hipGetLastError();
}

bool tile_shape_valid(int L, const TileShape &ts) {
    if (L < 16 || L > 1024 || (L & (L - 1))) return false;
    const int t[3] = {ts.tx, ts.ty, ts.tz};
    for (int d = 0; d < 3; ++d)
        if (t[d] < 1 || L % t[d] != 0 || ((L / t[d]) & 1)) return false;
    if (ts.tx % 8 != 0) return false;
    const long long threads = (long long)(ts.tx / 8) * ts.ty * ts.tz;
    if (threads < 64 || threads > 1024 || threads % 64 != 0) return false;
    if (tile_lds_bytes(ts) > 65536) return false;
    return ts.hits >= 1 && ts.hits <= 65536;
}

size_t tile_lds_bytes(const TileShape &ts) {
    return 2u * (size_t)(4 * (ts.tx / 8 + 2)) * (size_t)(ts.ty + 2) * (size_t)(ts.tz + 2);
}

hipError_t launch_tile_sweep(const Lattice &lat, const TileShape &ts, int coarse, int toff, hipStream_t s) {
    const int ntile = (lat.L / ts.tx) * (lat.L / ts.ty) * (lat.L / ts.tz) / 2;
    const dim3 grid((unsigned)(ntile * lat.R)), block((unsigned)((ts.tx / 8) * ts.ty * ts.tz));
    if (lat.kind == 0)
        hipLaunchKernelGGL(sweep_tiles<0>, grid, block, tile_lds_bytes(ts), s, lat, ts, coarse, toff);
    else
        hipLaunchKernelGGL(sweep_tiles<1>, grid, block, tile_lds_bytes(ts), s, lat, ts, coarse, toff);
    return hipGetLastError();
}

bool bits_valid(int L) { return L == 64 || L == 128 || L == 256; }

int bits_blocks_per_replica(int L) { return (int)(((long long)L * L * L / 64) / bits_wg(L)); }

namespace {
template <bool BATCH>
void launch_bits(const Lattice &lat0, const Lattice *lats, const uint2 *map, int L, int kind, int r0, int nrep,
                 int colour, int toff, int energy, hipStream_t s) {
    const int bpr = bits_blocks_per_replica(L);
    const int lbpr = __builtin_ctz((unsigned)bpr);
    const int nb = bpr * nrep;
    const int remap = nb % 8 == 0 ? 1 : 0;
    const dim3 grid((unsigned)nb), block((unsigned)bits_wg(L));
    const bool e = energy && colour == 1;
    if (kind == 0) {
        if (e) hipLaunchKernelGGL((sweep_bits<0, 1, BATCH>), grid, block, 0, s, lat0, lats, map, colour, toff, r0, lbpr, remap);
        else hipLaunchKernelGGL((sweep_bits<0, 0, BATCH>), grid, block, 0, s, lat0, lats, map, colour, toff, r0, lbpr, remap);
    } else {
        if (e) hipLaunchKernelGGL((sweep_bits<1, 1, BATCH>), grid, block, 0, s, lat0, lats, map, colour, toff, r0, lbpr, remap);
        else hipLaunchKernelGGL((sweep_bits<1, 0, BATCH>), grid, block, 0, s, lat0, lats, map, colour, toff, r0, lbpr, remap);
    }
}
}  // namespace

hipError_t launch_bits_sweep(const Lattice &lat, int r0, int nrep, int colour, int toff, int energy, hipStream_t s) {
    if (nrep <= 0) return hipSuccess;
    launch_bits<false>(lat, nullptr, nullptr, lat.L, lat.kind, r0, nrep, colour, toff, energy, s);
    return hipGetLastError();
}

hipError_t launch_bits_batch(const Launch &ln, int colour, int toff, int energy, hipStream_t s) {
    if (ln.nblocks <= 0) return hipSuccess;
    launch_bits<true>(Lattice{}, ln.lats, ln.map, ln.L, ln.kind, 0, ln.nblocks, colour, toff, energy, s);
    return hipGetLastError();
}

hipError_t launch_pack_bits(const Lattice &lat, hipStream_t s) {
    const long long words = (long long)lat.R * 2 * (lat.N / 64);
    hipLaunchKernelGGL(pack_bits_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, lat);
    return hipGetLastError();
}

hipError_t launch_unpack_bits(const Lattice &lat, hipStream_t s) {
    const long long words = (long long)lat.R * 2 * (lat.N / 64);
    hipLaunchKernelGGL(unpack_bits_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, lat);
    return hipGetLastError();
}

hipError_t launch_energy(const Lattice &lat, hipStream_t s) {
    hipLaunchKernelGGL(energy_kernel, dim3(lat.nblk, lat.R), dim3(256), 0, s, lat);
    return hipGetLastError();
}

hipError_t launch_reduce(const Lattice &lat, int64_t *B, double *F, int64_t *M, hipStream_t s) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kExchangeThreads), 0, s, lat, B, F, M);
    return hipGetLastError();
}

hipError_t launch_exchange(const Lattice *lats, int n, int tadv, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(exchange_kernel, dim3(n), dim3(kExchangeThreads), 0, s, lats, tadv);
    return hipGetLastError();
}

hipError_t launch_advance(const Lattice &lat, int tadv, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, lat.ctrs, tadv);
    return hipGetLastError();
}

}  // namespace rfim_dev
