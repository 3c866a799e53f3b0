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

constexpr int RED_NT = 256;

template <int P>
struct RedGeo {
    static constexpr int DH = 4 * (P - 2), DF = 4 * P, d = 4 * (P - 1);
    static constexpr int LH = (int)num_mono(DH), LF = (int)num_mono(DF), LG = (int)num_mono(d);
    static constexpr int LHA = (LH + 15) / 16 * 16, LFA = (LF + 15) / 16 * 16;
};

template <int P>
__global__ __launch_bounds__(RED_NT) void k_reduced(Stage1Args a)
{
    using G = RedGeo<P>;
    constexpr int P2 = P * P, d = G::d;
    static_assert(G::LFA >= G::LG, "M shares the second F buffer");
    __shared__ __align__(16) uint8_t f35[48], v_l[48], hb0[G::LHA], hb1[G::LHA], fb0[G::LFA], fb1[G::LFA];
    __shared__ uint32_t taps[35], vtaps[35], wsum[35];
    __shared__ int ntap, nvt, s_err, s_test;
    const int tid = threadIdx.x, lane = tid & 63, pi = prime_index(P);
    const int count = a.counters[CNT_COUNT + pi];
    for (int pos = blockIdx.x; pos < count; pos += gridDim.x) {
        const int surf = a.queue[pi][pos];
        if (tid < 35) f35[tid] = (uint8_t)(a.f[(size_t)surf * 35 + tid] % P);
        if (tid == 0) s_err = 0;
        __syncthreads();
        // H = f^(p-2) mod p (degree 4(p-2)); F^p mod p^2 (degree 4p)
        const uint8_t *H = fpow_mod_lds<P - 2, P>(f35, hb0, hb1, taps, &ntap);
        uint8_t *Dl = fpow_mod_lds<P, P2>(f35, fb0, fb1, taps, &ntap);
        uint8_t *M = Dl == fb0 ? fb1 : fb0;
        // D = (F^p - sum_I a_I^p x^(pI)) / p mod p, in place (Algorithm 1 on f)
        for (int r = tid; r < G::LF; r += RED_NT) {
            int x1, x2, x3, x4;
            cns_unrank(G::DF, r, x1, x2, x3, x4);
            int val = Dl[r];
            if (x1 % P == 0 && x2 % P == 0 && x3 % P == 0 && x4 % P == 0) {
                val -= pow_p_mod_p2<P>(f35[cns_rank(x2 / P, x3 / P, x4 / P)]);
                if (val < 0) val += P2;
            }
            if (val % P) s_err = 1;
            Dl[r] = (uint8_t)(val / P);
        }
        if (tid < 35) v_l[tid] = f35[tid];
        __syncthreads();
        int h = 0;
        for (int k = 2; k <= a.bound; ++k) {
            // M = H v (degree 4(p-1)), from the nonzero terms of v
            if (tid < 64) {
                const int n = compact_taps(v_l, vtaps);
                if (tid == 0) nvt = n;
            }
            if (tid < 35) wsum[tid] = 0;
            __syncthreads();
            const int nv = nvt;
            for (int c = tid; c < G::LG; c += RED_NT) {
                int x1, x2, x3, x4;
                cns_unrank(d, c, x1, x2, x3, x4);
                int acc = 0;
                for (int t = 0; t < nv; ++t) {
                    const uint32_t te = vtaps[t];
                    const int t1 = te & 255, t2 = (te >> 8) & 255, t3 = (te >> 16) & 255, t4 = 4 - t1 - t2 - t3;
                    if (x1 >= t1 && x2 >= t2 && x3 >= t3 && x4 >= t4)
                        acc += (int)(te >> 24) * H[cns_rank(x2 - t2, x3 - t3, x4 - t4)];
                }
                M[c] = (uint8_t)(acc % P);
            }
            __syncthreads();
            // w[r'] = u(D M)[r'] = sum_c M[c] D[p r' + e - c] for the 35 quartic exponents r'
            unsigned w[35];
#pragma unroll
            for (int q = 0; q < 35; ++q) w[q] = 0;
            for (int c = tid; c < G::LG; c += RED_NT) {
                const unsigned mc = M[c];
                if (!mc) continue;
                int c1, c2, c3, c4;
                cns_unrank(d, c, c1, c2, c3, c4);
#pragma unroll
                for (int q = 0; q < 35; ++q) {
                    const uint32_t rb = kB4.e[q];
                    const int y1 = P * (int)(rb & 255u) + P - 1 - c1, y2 = P * (int)((rb >> 8) & 255u) + P - 1 - c2,
                              y3 = P * (int)((rb >> 16) & 255u) + P - 1 - c3, y4 = P * (int)(rb >> 24) + P - 1 - c4;
                    if (y1 >= 0 && y2 >= 0 && y3 >= 0 && y4 >= 0) w[q] += mc * Dl[cns_rank(y2, y3, y4)];
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

hipError_t launch_reduced(int p, const Stage1Args &a, int nwg, hipStream_t s)
{
    if (a.batch <= 0 || nwg <= 0) return hipSuccess;
    switch (p) {
    case 3: hipLaunchKernelGGL(k_reduced<3>, dim3(nwg), dim3(RED_NT), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_reduced<5>, dim3(nwg), dim3(RED_NT), 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_reduced<7>, dim3(nwg), dim3(RED_NT), 0, s, a); break;
    case 11: hipLaunchKernelGGL(k_reduced<11>, dim3(nwg), dim3(RED_NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qfs
