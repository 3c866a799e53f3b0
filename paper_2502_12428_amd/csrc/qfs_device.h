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

// g = f^(P-1) mod P in CNS order, computed in LDS by repeated multiplication
// with the nonzero terms of f.  b0 and b1 must each hold C(4P-1,3) bytes,
// taps 35 words.  Returns the buffer holding the result.  Must be called by
// every thread of the block.
template <int P>
__device__ uint8_t *fpow_lds(const uint8_t *f35, uint8_t *b0, uint8_t *b1, uint32_t *taps, int *ntap)
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
    for (int j = 1; j < P - 1; ++j) {
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
            nxt[r] = (uint8_t)(acc % P);
        }
        __syncthreads();
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    return cur;
}

// Address of the Delta coefficient at 4-d position x (sum D) in the
// Cartier-split layout: region j = |x mod p| / p, row rank(x div p), column
// sidx(x mod p).
template <int P>
__device__ inline int64_t theta_addr(int x1, int x2, int x3, int x4)
{
    const int s1 = x1 % P, s2 = x2 % P, s3 = x3 % P, s4 = x4 % P;
    const int j = (s1 + s2 + s3 + s4) / P;
    const int code = ((s1 * P + s2) * P + s3) * P + s4;
    return kTT<P>.roff[j] + cns_rank(x2 / P, x3 / P, x4 / P) * kTT<P>.rs[j] + kTT<P>.sidx[code];
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

// out[r] = theta(a)[r] mod P for r in B_d (CNS order, LDS), from a_perm (LDS)
// and Delta in the Cartier-split layout (global):
//   theta(a)[r] = sum_{c' <= r} < a_perm[c'] , DeltaRow_j(r - c') >.
template <int P>
__device__ inline void theta_full(const uint8_t *__restrict__ dl, const uint8_t *aperm, uint8_t *out)
{
    using TG = ThetaGeo<P>;
    constexpr int d = TG::d;
    constexpr int LG = (int)num_mono(d);
    for (int r = threadIdx.x; r < LG; r += blockDim.x) {
        int r1, r2, r3, r4;
        cns_unrank(d, r, r1, r2, r3, r4);
        unsigned acc = 0;
        for (int cp = 0; cp < TG::NCP; ++cp) {
            const uint32_t c = kTT<P>.cprime[cp];
            const int c1 = c & 255, c2 = (c >> 8) & 255, c3 = (c >> 16) & 255, c4 = c >> 24;
            if (r1 < c1 || r2 < c2 || r3 < c3 || r4 < c4) continue;
            const int j = kTT<P>.cp_j[cp];
            const int rsj = kTT<P>.rs[j];
            const uint8_t *row = dl + kTT<P>.roff[j] + cns_rank(r2 - c2, r3 - c3, r4 - c4) * rsj;
            const uint8_t *av = aperm + kTT<P>.cp_seg[cp];
            for (int k = 0; k < rsj; k += 16)
                acc = dot16(gload16u(row + k), *(const v4u *)(av + k), acc);
        }
        out[r] = (uint8_t)(acc % P);
    }
}

// c(theta(a)) = theta(a)[e] mod P, the only coefficient the height test reads
// (Section 3.4): a block-wide dot product over the NCP segments.
template <int P>
__device__ inline int theta_test(const uint8_t *__restrict__ dl, const uint8_t *aperm, int *red)
{
    using TG = ThetaGeo<P>;
    unsigned part = 0;
    // one 16-byte chunk per thread iteration; chunk -> c' by scanning segments
    for (int ch = threadIdx.x; ch < TG::APERM / 16; ch += blockDim.x) {
        const int off = ch * 16;
        int cp = 0;
        while (cp + 1 < TG::NCP && kTT<P>.cp_seg[cp + 1] <= off) ++cp;
        const uint32_t c = kTT<P>.cprime[cp];
        const int c1 = c & 255, c2 = (c >> 8) & 255, c3 = (c >> 16) & 255, c4 = c >> 24;
        const int j = kTT<P>.cp_j[cp];
        const int64_t row = kTT<P>.roff[j] +
                            cns_rank(P - 1 - c2, P - 1 - c3, P - 1 - c4) * kTT<P>.rs[j];
        (void)c1;
        part = dot16(gload16u(dl + row + (off - kTT<P>.cp_seg[cp])), *(const v4u *)(aperm + off), part);
    }
    return block_sum((int)(part % P), red) % P;
}

}  // namespace qfs
