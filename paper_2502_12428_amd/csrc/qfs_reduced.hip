// Heights from the reduced form of Algorithm 3 (qfs_height_reduced).
//
// With D = Delta_1(f) (Algorithm 1 applied to f itself) and H = f^(p-2) mod p,
// the binomial theorem mod p^2 gives Delta_1(f^(p-1)) = phi(Q) - D phi(H) mod p
// (phi raises every exponent to p times itself), and since the splitting u of
// Algorithm 2 is p^-1-linear, theta(a) = c(a) Q - H u(D a) for forms a of
// degree 4(p-1), c(a) the coefficient of (x1..x4)^(p-1).  Along Algorithm 3's
// loop every tested a has c(a) = 0 until the height is found, so
// theta^(k-1)(g) = H v_k for quartics v_1 = f, v_(k+1) = -u(D H v_k), and the
// test reads c(H v_k) = sum_r v_k[r] H[e - r].  One workgroup per surface
// (persistent over the deep queue of stage 1) forms H and D in LDS, then
// applies v -> u(D (H v)) (the sign does not change which tests vanish) until
// a test is nonzero or the bound is reached.
#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

// Threads per workgroup.  At p = 11 the LDS buffers allow three workgroups per compute
// unit, so each takes more threads.
__host__ __device__ constexpr int red_nt(int p) { return p == 11 ? 512 : 256; }
// At p = 11 (few workgroups per compute unit) the inner sums run branch-free, so that
// their LDS reads are in flight together; at p <= 7 skipping the terms that do not
// apply is faster.
__host__ __device__ constexpr bool red_branch_free(int p) { return p == 11; }

template <int P>
struct RedGeo {
    static constexpr int DH = 4 * (P - 2), DF = 4 * P, d = 4 * (P - 1);
    static constexpr int LH = (int)num_mono(DH), LF = (int)num_mono(DF), LG = (int)num_mono(d);
    static constexpr int LHA = (LH + 15) / 16 * 16, LFA = (LF + 15) / 16 * 16;
};

// The next exponent after (e1, e2, e3, e4) in descending lex order of a fixed
// degree (the CNS rank grows by one).
__device__ inline void cns_next(int &e1, int &e2, int &e3, int &e4)
{
    if (e3 > 0) {
        --e3;
        ++e4;
    } else if (e2 > 0) {
        --e2;
        e3 = e4 + 1;
        e4 = 0;
    } else {
        --e1;
        e2 = e4 + 1;
        e4 = 0;
    }
}

// out[r] = sum over the quartic exponents t <= x_r of cf[t] in[rank(x_r - t)] mod MOD
// for the positions r of degree n; cf holds the 35 coefficients of a quartic in CNS
// order (the same for the whole block, read into scalar registers).  Each thread takes
// a contiguous run of positions and steps through them with cns_next.  With
// S = x2 + x3 + x4 and L = x3 + x4 the input rank is
// tet3(S - (4 - t1)) + tri2(L - (t3 + t4)) + x4 - t4, so a position needs five values
// of tet3 (they change with x1) and five of tri2 (they change with the line), and
// x >= t componentwise is one borrow test on the packed exponent bytes.
template <int MOD, int NT, bool BF>
__device__ inline void mul_quartic(int n, const uint8_t *in, uint8_t *out, const uint8_t *cf35)
{
    constexpr B4Table b4 = make_b4();
    int cf[35];
#pragma unroll
    for (int k = 0; k < 35; ++k) cf[k] = __builtin_amdgcn_readfirstlane((int)cf35[k]);
    const int len = (int)num_mono(n), per = (len + NT - 1) / NT;
    const int r0 = threadIdx.x * per, r1 = min(len, r0 + per);
    if (r0 >= r1) return;
    int x1, x2, x3, x4;
    cns_unrank(n, r0, x1, x2, x3, x4);
    unsigned t1s[5], t2s[5];
    int cS = -1, cL = -1;
    for (int r = r0; r < r1; ++r) {
        const int S = x2 + x3 + x4, L = x3 + x4;
        if (S != cS) {
            cS = S;
#pragma unroll
            for (int k = 0; k < 5; ++k) t1s[k] = tet3((unsigned)(S - k));
        }
        if (L != cL) {
            cL = L;
#pragma unroll
            for (int k = 0; k < 5; ++k) t2s[k] = tri2((unsigned)(L - k));
        }
        // byte i holds 0x80 + x_i: subtracting t leaves the top bit set iff x_i >= t_i
        const uint32_t xp = ((uint32_t)x1 | (uint32_t)x2 << 8 | (uint32_t)x3 << 16 | (uint32_t)x4 << 24) | 0x80808080u;
        int acc = 0;
#pragma unroll
        for (int k = 0; k < 35; ++k) {
            constexpr uint32_t H = 0x80808080u;
            const uint32_t te = b4.e[k];
            const int t1 = (int)(te & 255u), t3 = (int)((te >> 16) & 255u), t4 = (int)(te >> 24);
            if constexpr (BF) {  // a term with x < t reads position 0 and adds zero
                const bool ok = ((xp - te) & H) == H;
                const unsigned idx = ok ? t1s[4 - t1] + t2s[t3 + t4] + (unsigned)(x4 - t4) : 0u;
                acc += (ok ? cf[k] : 0) * (int)in[idx];
            } else if (cf[k] != 0 && ((xp - te) & H) == H) {
                acc += cf[k] * in[t1s[4 - t1] + t2s[t3 + t4] + (unsigned)(x4 - t4)];
            }
        }
        out[r] = (uint8_t)(acc % MOD);
        cns_next(x1, x2, x3, x4);
    }
}

template <int P>
__global__ __launch_bounds__(red_nt(P)) void k_reduced(Stage1Args a)
{
    using G = RedGeo<P>;
    constexpr int NT = red_nt(P);
    constexpr bool BF = red_branch_free(P);
    constexpr int P2 = P * P, d = G::d;
    static_assert(G::LFA >= G::LG, "M shares the second F buffer");
    __shared__ __align__(16) uint8_t f35[48], v_l[48], hb0[G::LHA], fb0[G::LFA], fb1[G::LFA];
    __shared__ uint32_t wsum[35];
    __shared__ int s_err, s_test;
    const int tid = threadIdx.x, lane = tid & 63, pi = prime_index(P);
    const int count = a.counters[CNT_COUNT + pi];
    for (int pos = blockIdx.x; pos < count; pos += gridDim.x) {
        const int surf = a.queue[pi][pos];
        if (tid < 35) f35[tid] = (uint8_t)(a.f[(size_t)surf * 35 + tid] % P);
        if (tid == 0) s_err = 0;
        __syncthreads();
        // F^j mod p^2 for j = 1..p by multiplication with f (degree 4j); on the way
        // H = F^(p-2) mod p = f^(p-2) mod p (degree 4(p-2))
        if (tid < 35) fb0[tid] = f35[tid];
        __syncthreads();
        uint8_t *cur = fb0, *nxt = fb1;
        if (P - 2 == 1 && tid < 35) hb0[tid] = f35[tid];
        for (int j = 1; j < P; ++j) {
            mul_quartic<P2, NT, BF>(4 * (j + 1), cur, nxt, f35);
            __syncthreads();
            uint8_t *t = cur;
            cur = nxt;
            nxt = t;
            if (j + 1 == P - 2)
                for (int r = tid; r < G::LH; r += NT) hb0[r] = (uint8_t)(cur[r] % P);
        }
        const uint8_t *H = hb0;
        uint8_t *Dl = cur;
        uint8_t *M = nxt;
        // D = (F^p - sum_I a_I^p x^(pI)) / p mod p, in place (Algorithm 1 on f)
        {
            constexpr int per = (G::LF + NT - 1) / NT;
            const int r0 = tid * per, rend = min(G::LF, r0 + per);
            int x1 = 0, x2 = 0, x3 = 0, x4 = 0;
            if (r0 < rend) cns_unrank(G::DF, r0, x1, x2, x3, x4);
            for (int r = r0; r < rend; ++r, cns_next(x1, x2, x3, x4)) {
                int val = Dl[r];
                if (x1 % P == 0 && x2 % P == 0 && x3 % P == 0 && x4 % P == 0) {
                    val -= pow_p_mod_p2<P>(f35[cns_rank(x2 / P, x3 / P, x4 / P)]);
                    if (val < 0) val += P2;
                }
                if (val % P) s_err = 1;
                Dl[r] = (uint8_t)(val / P);
            }
        }
        if (tid < 35) v_l[tid] = f35[tid];
        __syncthreads();
        int h = 0;
        for (int k = 2; k <= a.bound; ++k) {
            // M = H v (degree 4(p-1))
            if (tid < 35) wsum[tid] = 0;
            mul_quartic<P, NT, BF>(d, H, M, v_l);
            __syncthreads();
            // w[r'] = u(D M)[r'] = sum_c M[c] D[p r' + e - c] for the 35 quartic exponents r'.
            // The index y = p r' + e - c is nonnegative iff floor(c_i / p) <= r'_i (a borrow
            // test on packed bytes), and its rank is A[r'2 + r'3 + r'4] + B[r'3 + r'4] + p r'4 + p - 1 - c4
            // with A[s] = tet3(p s + 3(p-1) - (c2 + c3 + c4)) and B[l] = tri2(p l + 2(p-1) - (c3 + c4)).
            unsigned w[35];
#pragma unroll
            for (int q = 0; q < 35; ++q) w[q] = 0;
            {
                constexpr B4Table b4 = make_b4();
                constexpr int per = (G::LG + NT - 1) / NT;
                const int c0 = tid * per, cend = min(G::LG, c0 + per);
                int c1 = 0, c2 = 0, c3 = 0, c4 = 0;
                if (c0 < cend) cns_unrank(d, c0, c1, c2, c3, c4);
                for (int c = c0; c < cend; ++c, cns_next(c1, c2, c3, c4)) {
                    const unsigned mc = M[c];
                    if (!mc) continue;
                    const uint32_t kp = (uint32_t)(c1 / P) | (uint32_t)(c2 / P) << 8 | (uint32_t)(c3 / P) << 16 |
                                        (uint32_t)(c4 / P) << 24;
                    const int Sc = c2 + c3 + c4, Lc = c3 + c4;
                    unsigned A[5], B[5];
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        A[k] = tet3((unsigned)(P * k + 3 * (P - 1) - Sc));
                        B[k] = tri2((unsigned)(P * k + 2 * (P - 1) - Lc));
                    }
                    const unsigned base4 = (unsigned)(P - 1 - c4);
#pragma unroll
                    for (int q = 0; q < 35; ++q) {
                        constexpr uint32_t H8 = 0x80808080u;
                        const uint32_t rb = b4.e[q];
                        const int r2 = (int)((rb >> 8) & 255u), r3 = (int)((rb >> 16) & 255u), r4 = (int)(rb >> 24);
                        if constexpr (BF) {
                            const bool ok = (((rb | H8) - kp) & H8) == H8;
                            const unsigned idx = ok ? A[r2 + r3 + r4] + B[r3 + r4] + (unsigned)(P * r4) + base4 : 0u;
                            w[q] += (ok ? mc : 0u) * Dl[idx];
                        } else if ((((rb | H8) - kp) & H8) == H8) {
                            w[q] += mc * Dl[A[r2 + r3 + r4] + B[r3 + r4] + (unsigned)(P * r4) + base4];
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 35; ++q) {
                const int s = wave_sum((int)w[q]);
                if (lane == 0) atomicAdd(&wsum[q], (uint32_t)s);
            }
            __syncthreads();
            // v <- w mod p, and the test c(H v) = sum_r v[r] H[e - r]
            if (tid < 64) {
                int t = 0;
                if (tid < 35) {
                    const unsigned vq = wsum[tid] % P;
                    v_l[tid] = (uint8_t)vq;
                    const uint32_t rb = kB4.e[tid];
                    const int r1 = (int)(rb & 255u), r2 = (int)((rb >> 8) & 255u), r3 = (int)((rb >> 16) & 255u),
                              r4 = (int)(rb >> 24);
                    if (r1 <= P - 1 && r2 <= P - 1 && r3 <= P - 1 && r4 <= P - 1)
                        t = (int)vq * H[cns_rank(P - 1 - r2, P - 1 - r3, P - 1 - r4)];
                }
                t = wave_sum(t);
                if (tid == 0) s_test = t % P;
            }
            __syncthreads();
            if (s_test != 0) {
                h = k;
                break;
            }
        }
        if (tid == 0) a.heights[surf] = s_err ? -5 /* QFS_EARITH */ : h;
        __syncthreads();
    }
}

// The kernel walks its queue with a grid stride, so workgroups beyond those that fit
// on the device at once would start only after others have finished: the grid is
// at most the resident count.
template <int P>
static hipError_t launch_reduced_p(const Stage1Args &a, int nwg, hipStream_t s)
{
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_reduced<P>, red_nt(P), 0)) != hipSuccess) return e;
    if (per_cu > 0 && ncu > 0 && nwg > ncu * per_cu) nwg = ncu * per_cu;
    hipLaunchKernelGGL(k_reduced<P>, dim3(nwg), dim3(red_nt(P)), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduced(int p, const Stage1Args &a, int nwg, hipStream_t s)
{
    if (a.batch <= 0 || nwg <= 0) return hipSuccess;
    switch (p) {
    case 3: return launch_reduced_p<3>(a, nwg, s);
    case 5: return launch_reduced_p<5>(a, nwg, s);
    case 7: return launch_reduced_p<7>(a, nwg, s);
    case 11: return launch_reduced_p<11>(a, nwg, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qfs
