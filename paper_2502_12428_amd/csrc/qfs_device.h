// Device helpers shared by the libqfs kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qfs_common.h"

namespace qfs {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// Explicit global-memory accesses: generic (flat) accesses are counted by both
// the vector-memory and the LDS wait counters, which serialises prefetches
// against LDS reads.
#define QFS_GLOBAL __attribute__((address_space(1)))
__device__ inline v4i gload16(const uint8_t *p) { return *(const QFS_GLOBAL v4i *)(p); }
__device__ inline v4u gload16u(const uint8_t *p) { return *(const QFS_GLOBAL v4u *)(p); }
__device__ inline void gstore16(uint8_t *p, v4u v) { *(QFS_GLOBAL v4u *)(p) = v; }
__device__ inline void gstore4(uint8_t *p, unsigned v) { *(QFS_GLOBAL unsigned *)(p) = v; }
__device__ inline void gstore1(uint8_t *p, uint8_t v) { *(QFS_GLOBAL uint8_t *)(p) = v; }
__device__ inline uint8_t gload1(const uint8_t *p) { return *(const QFS_GLOBAL uint8_t *)(p); }

__constant__ B4Table kB4 = make_b4();
template <int P>
__constant__ ThetaTable<P> kTT = make_theta_table<P>();

__device__ inline int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Block-wide sum; `red` is LDS scratch of at least blockDim.x/64 ints.
__device__ inline int block_sum(int v, int *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int t = 0;
    for (int i = 0; i < nw; ++i) t += red[i];
    return t;
}

// b^P mod P^2 for 0 <= b < P
template <int P>
__device__ inline int pow_p_mod_p2(int b)
{
    int r = 1;
#pragma unroll
    for (int i = 0; i < P; ++i) r = (r * b) % (P * P);
    return r;
}

// Compact list of the nonzero terms of f (35 coefficients in LDS) into
// taps[0..n-1]: exponents e1, e2, e3 in bytes 0..2 and the coefficient in
// byte 3 (e4 = 4 - e1 - e2 - e3).  Called by the first wave of the block;
// returns n to that wave.
__device__ inline int compact_taps(const uint8_t *f35, uint32_t *taps)
{
    const int lane = threadIdx.x & 63;
    uint32_t te = 0;
    bool nz = false;
    if (lane < 35) {
        const uint32_t v = f35[lane];
        nz = v != 0;
        te = (kB4.e[lane] & 0xFFFFFFu) | (v << 24);
    }
    const uint64_t bal = __ballot(nz);
    if (nz) taps[__popcll(bal & ((1ull << lane) - 1ull))] = te;
    return __popcll(bal);
}

// f^J mod MOD in CNS order, computed in LDS by repeated multiplication with
// the nonzero terms of f (coefficients in [0, MOD)).  b0 and b1 must each hold
// C(4J+3,3) bytes, taps 35 words.  Returns the buffer holding the result.
// Must be called by every thread of the block.
template <int J, int MOD>
__device__ uint8_t *fpow_mod_lds(const uint8_t *f35, uint8_t *b0, uint8_t *b1, uint32_t *taps, int *ntap)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < 35; i += nt) b0[i] = f35[i];
    if (tid < 64) {
        const int n = compact_taps(f35, taps);
        if (tid == 0) *ntap = n;
    }
    __syncthreads();
    const int ntaps = *ntap;
    uint8_t *cur = b0, *nxt = b1;
    for (int j = 1; j < J; ++j) {
        const int n = 4 * (j + 1);
        const int len = (int)num_mono(n);
        for (int r = tid; r < len; r += nt) {
            int e1, e2, e3, e4;
            cns_unrank(n, r, e1, e2, e3, e4);
            int acc = 0;
            for (int k = 0; k < ntaps; ++k) {
                const uint32_t te = taps[k];
                const int t1 = te & 255, t2 = (te >> 8) & 255, t3 = (te >> 16) & 255, t4 = 4 - t1 - t2 - t3;
                if (e1 >= t1 && e2 >= t2 && e3 >= t3 && e4 >= t4)
                    acc += (int)(te >> 24) * cur[cns_rank(e2 - t2, e3 - t3, e4 - t4)];
            }
            nxt[r] = (uint8_t)(acc % MOD);
        }
        __syncthreads();
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return cur;
}

// g = f^(P-1) mod P
template <int P>
__device__ uint8_t *fpow_lds(const uint8_t *f35, uint8_t *b0, uint8_t *b1, uint32_t *taps, int *ntap)
{
    return fpow_mod_lds<P - 1, P>(f35, b0, b1, taps, ntap);
}

__device__ inline unsigned dot16(const v4u a, const v4u b, unsigned acc)
{
    acc = __builtin_amdgcn_udot4(a.x, b.x, acc, false);
    acc = __builtin_amdgcn_udot4(a.y, b.y, acc, false);
    acc = __builtin_amdgcn_udot4(a.z, b.z, acc, false);
    acc = __builtin_amdgcn_udot4(a.w, b.w, acc, false);
    return acc;
}

// Permute a (CNS order, LDS) into the coarse-part-major vector a_perm (LDS):
// for each c' (degree j < J) a segment of rs(j) bytes holding a[p c' + s]
// for s in S_j, zero padded.
template <int P>
__device__ inline void build_aperm(const uint8_t *a_cns, uint8_t *aperm)
{
    for (int i = threadIdx.x; i < ThetaGeo<P>::APERM; i += blockDim.x) {
        const unsigned src = kTT<P>.aperm_src[i];
        aperm[i] = src == 0xFFFFu ? 0 : a_cns[src];
    }
}

// Chunk ch (16 bytes) of Delta's Cartier-split layout, gathered through src.
template <int P, class Src>
__device__ __attribute__((always_inline)) inline v4u cartier_chunk(Src &src, int64_t ch)
{
    using TG = ThetaGeo<P>;
    constexpr int d = TG::d;
    int j = 0;
#pragma unroll
    for (int i = 1; i < TG::J; ++i)
        if (ch * 16 >= kTT<P>.roff[i]) j = i;
    const int nc = kTT<P>.rs[j] / 16;
    const int64_t local = ch - kTT<P>.roff[j] / 16;
    const int y = (int)(local / nc), m = (int)(local % nc);
    int y1, y2, y3, y4;
    cns_unrank(d - j, y, y1, y2, y3, y4);
    int cb = 0;
#pragma unroll
    for (int i = 1; i < TG::J; ++i)
        if (j == i) cb = TG::col_off(i);
    // the chunk's 16 columns (two 16-byte loads); column 16m is never padding
    const v4u *sg = (const v4u *)(kTT<P>.sig + cb + 16 * m);
    const v4u s0 = sg[0], s1 = sg[1];
    const unsigned sw[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
    const unsigned first = sw[0] & 0xFFFFu;
    // all 16 loads are issued unconditionally (padding reads column 16m's position) and masked after
    unsigned b[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const unsigned raw = (sw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
        const unsigned s = raw == 0xFFFFu ? first : raw;
        b[q] = src(P * y1 + (int)(s & 15), P * y2 + (int)((s >> 4) & 15), P * y3 + (int)((s >> 8) & 15),
                   P * y4 + (int)(s >> 12));
        if (raw == 0xFFFFu) b[q] = 0;
    }
    unsigned w[4] = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q >> 2] |= b[q] << (8 * (q & 3));
    return v4u{w[0], w[1], w[2], w[3]};
}

// Delta in the Cartier-split layout dl (global), built by 16-byte chunks:
// chunk m of row y in region j holds Delta[p y + sigma] for the region's
// columns 16m .. 16m+15 (sigma from the column table, zero for padding).
// src(x1, x2, x3, x4) returns Delta at a position of degree D.  Two chunks per
// thread and iteration keep 32 independent gathers in flight.
template <int P, class Src>
__device__ inline void cartier_split(Src &&src, uint8_t *dl)
{
    constexpr int64_t NCH = ThetaGeo<P>::BYTES / 16;
    const int64_t nt = blockDim.x;
    int64_t ch = threadIdx.x;
    for (; ch + nt < NCH; ch += 2 * nt) {
        const v4u a = cartier_chunk<P>(src, ch), b = cartier_chunk<P>(src, ch + nt);
        gstore16(dl + ch * 16, a);
        gstore16(dl + (ch + nt) * 16, b);
    }
    if (ch < NCH) gstore16(dl + ch * 16, cartier_chunk<P>(src, ch));
}

// theta(a) for the coarse parts of degree J0: row y of region J0 (Delta at
// p y + sigma) meets the a_perm segment of every c' of degree J0 at output
// r = y + c'.  Each row is read once (coalesced across the block); the dot
// products are added into the 32-bit sums in LDS.
template <int P, int J0>
__device__ __attribute__((always_inline)) inline void theta_region(const uint8_t *__restrict__ dl,
                                                                   const uint8_t *aperm, uint32_t *sums)
{
    using TG = ThetaGeo<P>;
    constexpr int d = TG::d, RS = TG::rs(J0), NC = RS / 16, NCPJ = (int)num_mono(J0), CP0 = TG::cp_off(J0);
    constexpr int NROW = (int)num_mono(d - J0);
    constexpr int64_t ROFF = TG::region_off(J0);
    constexpr int KB = NC < 8 ? NC : 8;
    for (int y = threadIdx.x; y < NROW; y += blockDim.x) {
        int y1, y2, y3, y4;
        cns_unrank(d - J0, y, y1, y2, y3, y4);
        const uint8_t *row = dl + ROFF + (int64_t)y * RS;
        unsigned dots[NCPJ];
#pragma unroll
        for (int c = 0; c < NCPJ; ++c) dots[c] = 0;
        for (int k0 = 0; k0 < NC; k0 += KB) {
            v4u rv[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) rv[k] = (k0 + k < NC) ? gload16u(row + 16 * (k0 + k)) : v4u{0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < NCPJ; ++c) {
                const uint8_t *av = aperm + kTT<P>.cp_seg[CP0 + c] + 16 * k0;
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (k0 + k < NC) dots[c] = dot16(rv[k], *(const v4u *)(av + 16 * k), dots[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < NCPJ; ++c) {
            const uint32_t cp = kTT<P>.cprime[CP0 + c];
            atomicAdd(&sums[cns_rank(y2 + (int)((cp >> 8) & 255), y3 + (int)((cp >> 16) & 255), y4 + (int)(cp >> 24))],
                      dots[c]);
        }
    }
}

template <int P, int J0>
__device__ __attribute__((always_inline)) inline void theta_regions(const uint8_t *dl, const uint8_t *aperm,
                                                                    uint32_t *sums)
{
    if constexpr (J0 < ThetaGeo<P>::J) {
        theta_region<P, J0>(dl, aperm, sums);
        theta_regions<P, J0 + 1>(dl, aperm, sums);
    }
}

// out[r] = theta(a)[r] mod P for r in B_d (CNS order, LDS), from a_perm (LDS)
// and Delta in the Cartier-split layout (global):
//   theta(a)[r] = sum over c' <= r of < a_perm[c'] , DeltaRow_j(r - c') >
// (Section 3.4, with the matches of Section 4.2).  sums: C(4P-1,3) words of
// LDS.  Must be called by every thread of the block.
template <int P>
__device__ inline void theta_full(const uint8_t *__restrict__ dl, const uint8_t *aperm, uint32_t *sums, uint8_t *out)
{
    constexpr int LG = (int)num_mono(ThetaGeo<P>::d);
    for (int i = threadIdx.x; i < LG; i += blockDim.x) sums[i] = 0;
    __syncthreads();
    theta_regions<P, 0>(dl, aperm, sums);
    __syncthreads();
    for (int i = threadIdx.x; i < LG; i += blockDim.x) out[i] = (uint8_t)(sums[i] % P);
}

}  // namespace qfs
