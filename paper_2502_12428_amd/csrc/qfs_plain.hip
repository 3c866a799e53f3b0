// Plain per-surface height path: vector-ALU kernels only, one surface at a
// time, no matrix cores and no batching.  It is the comparison baseline for
// the batched path.  Polynomials are dense dehomogenised cubes: the
// coefficient of x1^a x2^b x3^c x4^(n-a-b-c) at [(a*(n+1) + b)*(n+1) + c].
//
// Per surface: start (g = f^(p-1), Fedder's test, A_1 = g~), p-1 products
// A_{k+1} = A_k * g~ mod p^2 (the last one with the Delta_1 epilogue of
// Algorithm 1), then up to bound-1 theta launches (Algorithm 3's loop), then
// finish.  Launches after the surface is decided return at once.
#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

namespace {

struct PlainHdr {
    int done;
    int height;
    int ntaps;
    int err;
};

template <int P>
struct PlainLayout {
    static constexpr int d = 4 * (P - 1), D = P * d;
    static constexpr int LG = (int)num_mono(d);
    static constexpr size_t hdr = 0;
    static constexpr size_t g = 256;
    static constexpr size_t taps = g + align256(LG);
    static constexpr size_t tapv = taps + align256((size_t)LG * 4);
    static constexpr size_t a0 = tapv + align256(LG);
    static constexpr size_t a1 = a0 + align256(LG);
    static constexpr size_t cube_bytes = (size_t)(D + 1) * (D + 1) * (D + 1);
    static constexpr size_t cA = a1 + align256(LG);
    static constexpr size_t cB = cA + align256(cube_bytes);
    static constexpr size_t total = cB + align256(cube_bytes);
};

template <int P>
__global__ __launch_bounds__(256) void k_plain_start(const uint8_t *f, uint8_t *ws)
{
    using L = PlainLayout<P>;
    constexpr int d = L::d, LG = L::LG, S = d + 1;
    __shared__ __align__(16) uint8_t f35[64];
    __shared__ __align__(16) uint8_t b0[(LG + 15) / 16 * 16], b1[(LG + 15) / 16 * 16];
    __shared__ int bad, ntaps, fnt;
    __shared__ uint32_t ftaps[35];
    PlainHdr *hdr = (PlainHdr *)(ws + L::hdr);
    const int tid = threadIdx.x;
    if (tid == 0) {
        bad = 0;
        ntaps = 0;
    }
    __syncthreads();
    if (tid < 35) {
        const int v = f[tid];
        f35[tid] = (uint8_t)(v % P);
        if (v >= P) atomicOr(&bad, 1);
    }
    __syncthreads();
    const uint8_t *g = fpow_lds<P>(f35, b0, b1, ftaps, &fnt);
    uint8_t *gw = ws + L::g;
    uint32_t *taps = (uint32_t *)(ws + L::taps);
    uint8_t *tapv = ws + L::tapv;
    uint8_t *A = ws + L::cA;
    for (int i = tid; i < S * S * S; i += 256) A[i] = 0;
    __syncthreads();
    for (int r = tid; r < LG; r += 256) {
        gw[r] = g[r];
        int e1, e2, e3, e4;
        cns_unrank(d, r, e1, e2, e3, e4);
        A[(e1 * S + e2) * S + e3] = g[r];
        if (g[r]) {
            const int k = atomicAdd(&ntaps, 1);
            taps[k] = pack3(e1, e2, e3);
            tapv[k] = g[r];
        }
    }
    __syncthreads();
    if (tid == 0) {
        const bool deep = g[Prime<P>::e_index] == 0;
        hdr->ntaps = ntaps;
        hdr->err = 0;
        if (bad) {
            hdr->done = 1;
            hdr->height = -1; /* QFS_EINVAL */
        } else {
            hdr->done = deep ? 0 : 1;
            hdr->height = deep ? 0 : 1;
        }
    }
}

// A_{k+1} = A_k * g~ mod p^2 on the cube of degree n = (k+1) d; thread per cube position.
template <int P>
__global__ __launch_bounds__(256) void k_plain_mul(int k, uint8_t *ws)
{
    using L = PlainLayout<P>;
    constexpr int d = L::d, D = L::D, P2 = P * P;
    const PlainHdr *hdr = (const PlainHdr *)(ws + L::hdr);
    if (hdr->done) return;
    const int nk = k * d, n = nk + d, Sk = nk + 1, S = n + 1;
    const uint8_t *Ain = ws + ((k & 1) ? L::cA : L::cB);
    uint8_t *Aout = ws + ((k & 1) ? L::cB : L::cA);
    const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pos >= (int64_t)S * S * S) return;
    const int r3 = (int)(pos % S), r2 = (int)((pos / S) % S), r1 = (int)(pos / ((int64_t)S * S));
    const bool last = (k == P - 1);
    if (r1 + r2 + r3 > n) {
        Aout[pos] = 0;
        return;
    }
    const uint32_t *taps = (const uint32_t *)(ws + L::taps);
    const uint8_t *tapv = ws + L::tapv;
    const int nt = hdr->ntaps;
    int acc = 0;
    for (int t = 0; t < nt; ++t) {
        const uint32_t tp = taps[t];
        const int y1 = r1 - unp0(tp), y2 = r2 - unp1(tp), y3 = r3 - unp2(tp);
        if (y1 < 0 || y2 < 0 || y3 < 0 || y1 > nk || y2 > nk || y3 > nk) continue;
        acc += tapv[t] * Ain[((int64_t)y1 * Sk + y2) * Sk + y3];
    }
    int val = acc % P2;
    if (!last) {
        Aout[pos] = (uint8_t)val;
        return;
    }
    // Delta_1 epilogue (Algorithm 1): subtract b^p at p*J, divide by p
    const int r4 = D - r1 - r2 - r3;
    if (r1 % P == 0 && r2 % P == 0 && r3 % P == 0) {
        const uint8_t *gw = ws + L::g;
        const int bj = gw[cns_rank(r2 / P, r3 / P, r4 / P)];
        val -= pow_p_mod_p2<P>(bj);
        if (val < 0) val += P2;
    }
    if (val % P) atomicOr((int *)&((PlainHdr *)(ws + L::hdr))->err, 1);
    Aout[pos] = (uint8_t)(val / P);
}

// a_next = theta(a) with Delta in the cube Aout of the last product; one wave per output r.
template <int P>
__global__ __launch_bounds__(64) void k_plain_theta(int h, int bound, uint8_t *ws)
{
    using L = PlainLayout<P>;
    constexpr int d = L::d, D = L::D, LG = L::LG, S = D + 1;
    PlainHdr *hdr = (PlainHdr *)(ws + L::hdr);
    if (hdr->done) return;
    if (hdr->err) {
        if (threadIdx.x == 0 && blockIdx.x == 0) {
            hdr->done = 1;
            hdr->height = -5; /* QFS_EARITH */
        }
        return;
    }
    const uint8_t *dc = ws + (((P - 1) & 1) ? L::cB : L::cA);
    const uint8_t *a = ws + ((h & 1) ? L::a1 : L::a0);
    uint8_t *out = ws + ((h & 1) ? L::a0 : L::a1);
    if (h == 2) a = ws + L::g;
    const int r = blockIdx.x;
    int r1, r2, r3, r4;
    cns_unrank(d, r, r1, r2, r3, r4);
    int acc = 0;
    for (int c = threadIdx.x; c < LG; c += 64) {
        const int av = a[c];
        if (!av) continue;
        int c1, c2, c3, c4;
        cns_unrank(d, c, c1, c2, c3, c4);
        const int x1 = P * r1 + P - 1 - c1, x2 = P * r2 + P - 1 - c2, x3 = P * r3 + P - 1 - c3,
                  x4 = P * r4 + P - 1 - c4;
        if (x1 < 0 || x2 < 0 || x3 < 0 || x4 < 0) continue;
        acc += av * dc[((int64_t)x1 * S + x2) * S + x3];
    }
    acc = wave_sum(acc % P) % P;
    if (threadIdx.x == 0) {
        out[r] = (uint8_t)acc;
        if (r == Prime<P>::e_index && acc != 0) {
            hdr->height = h;
            hdr->done = 1;
        }
    }
}

__global__ void k_plain_finish(const uint8_t *ws, int32_t *height)
{
    const PlainHdr *hdr = (const PlainHdr *)ws;
    *height = hdr->height;
}

template <int P>
hipError_t plain_surface(const uint8_t *f35, int bound, int32_t *height, uint8_t *ws, hipStream_t s)
{
    using L = PlainLayout<P>;
    hipLaunchKernelGGL(k_plain_start<P>, dim3(1), dim3(256), 0, s, f35, ws);
    for (int k = 1; k < P; ++k) {
        const int64_t S = (int64_t)(k + 1) * L::d + 1;
        const int64_t n = S * S * S;
        hipLaunchKernelGGL(k_plain_mul<P>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k, ws);
    }
    for (int h = 2; h <= bound; ++h)
        hipLaunchKernelGGL(k_plain_theta<P>, dim3(L::LG), dim3(64), 0, s, h, bound, ws);
    hipLaunchKernelGGL(k_plain_finish, dim3(1), dim3(1), 0, s, (const uint8_t *)ws, height);
    return hipGetLastError();
}

}  // namespace

size_t plain_scratch_bytes(int p)
{
    switch (p) {
    case 3: return PlainLayout<3>::total;
    case 5: return PlainLayout<5>::total;
    case 7: return PlainLayout<7>::total;
    case 11: return PlainLayout<11>::total;
    }
    return 0;
}

hipError_t launch_plain_surface(int p, const uint8_t *f35, int bound, int32_t *height, uint8_t *scratch,
                                hipStream_t s)
{
    switch (p) {
    case 3: return plain_surface<3>(f35, bound, height, scratch, s);
    case 5: return plain_surface<5>(f35, bound, height, scratch, s);
    case 7: return plain_surface<7>(f35, bound, height, scratch, s);
    case 11: return plain_surface<11>(f35, bound, height, scratch, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace qfs
