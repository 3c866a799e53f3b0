// Batched height and Delta_1 kernels for gfx950.
//
// Stage 1 (one workgroup per surface): g = f^(p-1) mod p and Fedder's test
//   (g not in m^[p] iff its coefficient at (x1..x4)^(p-1) is nonzero, the only
//   monomial of degree 4(p-1) outside m^[p] -- Section 3.4).  Surfaces that
//   fail it ("deep" surfaces) are compacted into a per-prime queue together
//   with g.
// Deep kernel (persistent; each workgroup pops surfaces from the queue):
//   g~^p mod p^2 (Algorithm 1) as m^NF for the multiplier m = f~^J mod p^2,
//   by the chain A_{k+1} = A_k * m (k = 1..NF-1) on int8 matrix cores with
//   int32 accumulation, the Delta_1 epilogue fused into the last product
//   (Algorithm 1), then the theta loop of Algorithm 3 with its
//   one-coefficient test.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

template <int P>
__constant__ PlanTable<P> kPT = kPlanTable<P>;

// ---------------------------------------------------------------------------
// reset
// ---------------------------------------------------------------------------
__global__ void k_reset(int32_t *counters)
{
    for (int i = threadIdx.x; i < CNT_WORDS; i += blockDim.x) counters[i] = 0;
}

hipError_t launch_reset(int32_t *counters, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stage 1: Fedder's test for every surface, then g = f^(p-1) for the queued ones
// ---------------------------------------------------------------------------
template <int P>
__constant__ CapTable<P> kCap = make_cap_table<P>();

constexpr int S1_NT = 64;  // one wave per surface
constexpr int S1_LDS = 48 + 35 * 4 + 2 * ((11 * 11 * 11 + 15) / 16 * 16);

// Coefficient of (x1 x2 x3 x4)^(P-1) in f^(P-1) mod P (Fedder's criterion,
// Section 2.2): the powers f^j are kept only on the monomials whose exponents
// are all <= P-1 (a P^3 cube indexed by x1, x2, x3; x4 follows from the
// degree), which determines that coefficient exactly.  One wave.
template <int P>
__device__ int fedder_coefficient(const uint8_t *f35, uint8_t *lds)
{
    constexpr int C3 = (P * P * P + 15) / 16 * 16;
    uint32_t *taps = (uint32_t *)(lds + 48);
    uint8_t *cur = lds + 48 + 35 * 4, *nxt = cur + C3;
    const int lane = threadIdx.x;
    const int nt = compact_taps(f35, taps);
    for (int i = lane; i < kCap<P>.len[1]; i += S1_NT) {
        const uint32_t m = kCap<P>.m[kCap<P>.off[1] + i];
        const int x1 = m & 255, x2 = (m >> 8) & 255, x3 = (m >> 16) & 255, x4 = m >> 24;
        cur[(x1 * P + x2) * P + x3] = f35[cns_rank(x2, x3, x4)];
    }
    __syncthreads();
    for (int j = 1; j < P - 1; ++j) {
        const int off = kCap<P>.off[j + 1], len = kCap<P>.len[j + 1];
        for (int i = lane; i < len; i += S1_NT) {
            const uint32_t m = kCap<P>.m[off + i];
            const int x1 = m & 255, x2 = (m >> 8) & 255, x3 = (m >> 16) & 255, x4 = m >> 24;
            int acc = 0;
            for (int k = 0; k < nt; ++k) {
                const uint32_t te = taps[k];
                const int t1 = te & 255, t2 = (te >> 8) & 255, t3 = (te >> 16) & 255, t4 = 4 - t1 - t2 - t3;
                if (x1 >= t1 && x2 >= t2 && x3 >= t3 && x4 >= t4)
                    acc += (int)(te >> 24) * cur[((x1 - t1) * P + (x2 - t2)) * P + (x3 - t3)];
            }
            nxt[(x1 * P + x2) * P + x3] = (uint8_t)(acc % P);
        }
        __syncthreads();
        uint8_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    return cur[((P - 1) * P + (P - 1)) * P + (P - 1)];
}

template <int P>
__device__ void stage1_one(const Stage1Args &a, int surf, uint8_t *lds)
{
    uint8_t *f35 = lds;
    const int lane = threadIdx.x, pi = prime_index(P);
    int v = 0;
    if (lane < 35) {
        v = a.f[(size_t)surf * 35 + lane];
        f35[lane] = (uint8_t)(v % P);
    }
    const bool bad = __ballot(v >= P) != 0;
    __syncthreads();
    if (a.mode == MODE_HEIGHT) {
        if (bad) {
            if (lane == 0) a.heights[surf] = -1; /* QFS_EINVAL */
            return;
        }
        const bool deep = fedder_coefficient<P>(f35, lds) == 0;
        if (lane == 0) {
            if (!deep || a.bound < 2)
                a.heights[surf] = deep ? 0 : 1;
            else
                a.queue[pi][atomicAdd(&a.counters[CNT_COUNT + pi], 1)] = surf;
        }
    } else if (lane == 0) {
        a.queue[pi][surf] = surf;
        if (a.status) a.status[surf] = bad ? -1 : 0;
        if (surf == 0) a.counters[CNT_COUNT + pi] = a.batch;
    }
}

__global__ __launch_bounds__(S1_NT) void k_stage1(Stage1Args a)
{
    __shared__ __align__(16) uint8_t lds[S1_LDS];
    const int surf = blockIdx.x;
    const int p = a.fixed_p > 0 ? a.fixed_p : a.p[surf];
    const int pi = prime_index(p);
    if (pi < 0 || !((a.present_mask >> pi) & 1)) {
        if (threadIdx.x == 0) {
            if (a.mode == MODE_HEIGHT) a.heights[surf] = -4; /* QFS_EUNSUPPORTED */
            else if (a.status) a.status[surf] = -4;
        }
        return;
    }
    switch (p) {
    case 3: stage1_one<3>(a, surf, lds); break;
    case 5: stage1_one<5>(a, surf, lds); break;
    case 7: stage1_one<7>(a, surf, lds); break;
    case 11: stage1_one<11>(a, surf, lds); break;
    }
}

hipError_t launch_stage1(const Stage1Args &a, hipStream_t s)
{
    if (a.batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage1, dim3(a.batch), dim3(S1_NT), 0, s, a);
    return hipGetLastError();
}

// g = f^(P-1) mod P for the queued surfaces of prime P (persistent: workgroup
// b takes queue positions b, b + grid, ...), into gq (and g_out in MODE_DELTA).
template <int P>
__global__ __launch_bounds__(256) void k_gpow(Stage1Args a)
{
    constexpr int LG = Prime<P>::len_g, LGA = (LG + 15) / 16 * 16;
    __shared__ __align__(16) uint8_t f35[64], b0[LGA], b1[LGA];
    __shared__ uint32_t taps[35];
    __shared__ int ntap;
    const int tid = threadIdx.x, pi = prime_index(P);
    const int count = a.counters[CNT_COUNT + pi];
    for (int pos = blockIdx.x; pos < count; pos += gridDim.x) {
        const int surf = a.queue[pi][pos];
        if (tid < 35) f35[tid] = (uint8_t)(a.f[(size_t)surf * 35 + tid] % P);
        __syncthreads();
        const uint8_t *g = fpow_lds<P>(f35, b0, b1, taps, &ntap);
        uint8_t *dst = a.gq[pi] + (size_t)pos * LG;
        for (int i = tid; i < LG; i += blockDim.x) dst[i] = g[i];
        if (a.mode == MODE_DELTA && a.g_out) {
            uint8_t *go = a.g_out + (size_t)surf * LG;
            for (int i = tid; i < LG; i += blockDim.x) go[i] = g[i];
        }
        __syncthreads();
    }
}

bool gpow_needed(int p)
{
    switch (p) {
    case 3: return !g_from_chain<3>();
    case 5: return !g_from_chain<5>();
    case 7: return !g_from_chain<7>();
    case 11: return !g_from_chain<11>();
    }
    return true;
}

hipError_t launch_gpow(int p, const Stage1Args &a, int nwg, hipStream_t s)
{
    if (a.batch <= 0 || nwg <= 0) return hipSuccess;
    switch (p) {
    case 3: hipLaunchKernelGGL(k_gpow<3>, dim3(nwg), dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_gpow<5>, dim3(nwg), dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL(k_gpow<7>, dim3(nwg), dim3(256), 0, s, a); break;
    case 11: hipLaunchKernelGGL(k_gpow<11>, dim3(nwg), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// plan: output tile lists (base tiles of the super-tiles, and shell lists)
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_plan(uint32_t *plan)
{
    using X = GeoX<P>;
    constexpr int dm = X::dm, NF = X::NF;
    const int kind = blockIdx.x / NF, k = blockIdx.x % NF;  // 0 base, 1 shell, 2 band, 3 band shell
    if (kind == 1 ? (k > NF - 2) : kind == 3 ? (k < 1 || k > NF - 2) : (k < 1)) return;
    const int m = (k + 1) * dm;
    uint32_t *out = plan + (kind == 0 ? kPT<P>.boff[k] : kind == 1 ? kPT<P>.foff[k] : kind == 2 ? kPT<P>.noff[k]
                                                                                          : kPT<P>.hoff[k]);
    __shared__ int cnt[256];
    const int tid = threadIdx.x;
    if (kind == 0 || kind == 2) {
        // blocks of base units, a contiguous range of block indices per thread
        const bool band = kind == 2;
        auto keep = [&](uint32_t t) { return !band || band_tile_packed<P>(m, t); };
        const PlanBlocks nb = plan_blocks(m);
        const int nblk = nb.n1 * nb.n2 * nb.n3;
        const int per = (nblk + 255) / 256;
        const int b0 = min(nblk, tid * per), b1 = min(nblk, b0 + per);
        int mine = 0;
        for (int b = b0; b < b1; ++b) mine += plan_block_emit(m, b, keep, [](int, uint32_t) {});
        cnt[tid] = mine;
        __syncthreads();
        int off = 0;
        for (int i = 0; i < tid; ++i) off += cnt[i];
        for (int b = b0; b < b1; ++b) off += plan_block_emit(m, b, keep, [&](int i, uint32_t t) { out[off + i] = t; });
        __syncthreads();
        // bounding box of every group of 16 entries
        const int len = (int)(band ? kPT<P>.nlen[k] : kPT<P>.blen[k]);
        uint32_t *gb = plan + (band ? kPT<P>.ngoff[k] : kPT<P>.gboff[k]);
        for (int g = tid; g * 16 < len; g += 256) {
            int m1 = 0, m2 = 0, m3 = 0, l1 = 1 << 15, l2 = 1 << 15, l3 = 1 << 15, wl = 1 << 15, wh = 0;
            for (int i = g * 16; i < len && i < g * 16 + 16; ++i) {
                const uint32_t t = out[i];
                const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t), w = T1 * c1 + T2 * c2 + T3 * c3;
                m1 = max(m1, c1);
                m2 = max(m2, c2);
                m3 = max(m3, c3);
                l1 = min(l1, c1);
                l2 = min(l2, c2);
                l3 = min(l3, c3);
                wl = min(wl, w);
                wh = max(wh, w);
            }
            gb[4 * g] = (uint32_t)m1 | ((uint32_t)m2 << 16);
            gb[4 * g + 1] = (uint32_t)m3 | ((uint32_t)l1 << 16);
            gb[4 * g + 2] = (uint32_t)l2 | ((uint32_t)l3 << 16);
            gb[4 * g + 3] = (uint32_t)wl | ((uint32_t)wh << 16);
        }
        return;
    }
    // shell lists: one column slab c1 per thread, any order
    const int cap = kind == 3 ? P * P - 1 : CAP_NONE;
    const int cm = shell_cmax<P>(k, cap);
    const int c1 = tid;
    int mine = 0;
    if (c1 <= cm)
        for (int c2 = 0; c2 <= cm; ++c2) {
            int lo = 0, hi = -1;
            shell_c3_range<P>(k, cap, c1, c2, lo, hi);
            if (hi >= lo) mine += hi - lo + 1;
        }
    cnt[c1] = mine;
    __syncthreads();
    if (c1 <= cm) {
        int off = 0;
        for (int i = 0; i < c1; ++i) off += cnt[i];
        for (int c2 = 0; c2 <= cm; ++c2) {
            int lo = 0, hi = -1;
            shell_c3_range<P>(k, cap, c1, c2, lo, hi);
            for (int c3 = lo; c3 <= hi; ++c3) out[off++] = pack3(c1, c2, c3);
        }
    }
}

hipError_t launch_plan(int p, uint32_t *plan, hipStream_t s)
{
    switch (p) {
    case 3: hipLaunchKernelGGL(k_plan<3>, dim3(4 * Geo<3>::NF), dim3(256), 0, s, plan); break;
    case 5: hipLaunchKernelGGL(k_plan<5>, dim3(4 * Geo<5>::NF), dim3(256), 0, s, plan); break;
    case 7: hipLaunchKernelGGL(k_plan<7>, dim3(4 * Geo<7>::NF), dim3(256), 0, s, plan); break;
    case 11: hipLaunchKernelGGL(k_plan<11>, dim3(4 * Geo<11>::NF), dim3(256), 0, s, plan); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deep kernel
// ---------------------------------------------------------------------------
// Threads per deep workgroup (one workgroup per CU: the W blocks fill most of
// the LDS), and how many list entries ahead the input fragments are loaded.
#ifndef QFS_DEEP_NT
#define QFS_DEEP_NT 512
#endif
#ifndef QFS_DEEP_PF
#define QFS_DEEP_PF 4
#endif
// Deep workgroups one compute unit must be able to hold (registers per wave are sized for it).
#ifndef QFS_DEEP_MINWG
#define QFS_DEEP_MINWG 1
#endif
#ifndef QFS_DEEP_NB
#define QFS_DEEP_NB 4
#endif
constexpr int DEEP_NT = QFS_DEEP_NT, DEEP_NW = DEEP_NT / 64, DEEP_NB = QFS_DEEP_NB, DEEP_PF = QFS_DEEP_PF;

template <int P>
__constant__ DeltaTableX<P> kDX = make_delta_table_x<P>();

// Geometry of the Cartier split read straight from Delta's tile box.  The
// rows of every region whose coarse part starts (y1, y2, y3) read only the
// positions x with floor(x_i / p) = y_i (i = 1..3): a block of NT1 x NT1 x NT3
// tiles (p consecutive positions meet at most (p+1)/2 tiles of 2 and
// (p+2)/4 + 1 tiles of 4), staged position-major as W1 x W2 x W3 bytes.  Each
// block feeds NCH 16-byte chunks, one per column chunk of every region; a wave
// takes U blocks at a time.
template <int P>
struct SplitGeo {
    static constexpr int NT1 = (P + 1) / 2, NT3 = (P + 2) / 4 + 1, NTB = NT1 * NT1 * NT3;
    static constexpr int W1 = 2 * NT1, W2 = 2 * NT1, W3 = 4 * NT3, CUBE = W1 * W2 * W3;
    static constexpr int NCH = ThetaGeo<P>::NCOL / 16;
    static constexpr int U = NCH >= 64 ? 1 : 64 / NCH;
    static constexpr int NL = (U * NTB + 63) / 64;  // tile loads per lane and group of U blocks
    static constexpr int STAGE = U * CUBE;          // LDS bytes per wave
    static constexpr int NCUBE = (int)num_mono(4 * (P - 1));
};
// The coarse blocks (y1, y2, y3), y1 + y2 + y3 <= 4(p-1), packed 8 bits each.
template <int P>
struct CubeTable {
    uint32_t c[SplitGeo<P>::NCUBE];
};
template <int P>
constexpr CubeTable<P> make_cube_table()
{
    CubeTable<P> t{};
    constexpr int d = 4 * (P - 1);
    int n = 0;
    for (int y1 = 0; y1 <= d; ++y1)
        for (int y2 = 0; y1 + y2 <= d; ++y2)
            for (int y3 = 0; y1 + y2 + y3 <= d; ++y3) t.c[n++] = (uint32_t)y1 | ((uint32_t)y2 << 8) | ((uint32_t)y3 << 16);
    return t;
}
template <int P>
__constant__ CubeTable<P> kCube = make_cube_table<P>();

template <int P>
struct DeepLds {
    using X = GeoX<P>;
    static constexpr int LG = Prime<P>::len_g;
    static constexpr int LGA = (LG + 15) / 16 * 16;
    static constexpr int APA = (ThetaGeo<P>::APERM + 15) / 16 * 16;
    static constexpr int WB = w_in_lds<P>() ? (int)((X::W_BYTES + 15) / 16 * 16) : 0;
    // the multiplier m = f~^J mod p^2 (J < p-1; for J = p-1, m = g~ is g itself)
    static constexpr bool OWN_M = Geo<P>::J < P - 1;
    static constexpr int LMA = OWN_M ? (int)((num_mono(X::dm) + 15) / 16 * 16) : 0;
    static constexpr int off_w = 0;
    static constexpr int off_g = off_w + WB;
    static constexpr int off_m0 = off_g + LGA;
    static constexpr int off_m1 = off_m0 + LMA;
    static constexpr int off_taps = off_m1 + LMA;
    static constexpr int off_aperm = off_taps + (OWN_M ? 48 * 4 : 0);
    static constexpr int off_toff = off_aperm + APA;
    static constexpr int off_widx = off_toff + 4 * (X::NVXP + 4);
    static constexpr int off_qbox = off_widx + 8 * (X::NVXP + 4);
    static constexpr int off_qlist = off_qbox + 16 * X::NQX;
    static constexpr int QSTRIDE = X::NQX + DEEP_PF;  // a wave's needed-quad list, padded
    static constexpr int off_red = off_qlist + ((2 * QSTRIDE * (DEEP_NT / 64) + 15) / 16 * 16);
    static constexpr int off_sig = off_red + 4 * 64;  // the Cartier split's column table
    static constexpr int off_sums = off_sig + (ThetaGeo<P>::NCOL * 2 + 15) / 16 * 16;
    // theta's sums, or (not at the same time) the Cartier split's staging blocks
    static constexpr int SUMS = 4 * LGA > DEEP_NW * SplitGeo<P>::STAGE ? 4 * LGA : DEEP_NW * SplitGeo<P>::STAGE;
    static constexpr int bytes = off_sums + SUMS;
};

template <int P>
__device__ inline int64_t box_tile(int c1, int c2, int c3)
{
    using X = GeoX<P>;
    return ((int64_t)(c1 + X::H1) * X::B2 + (c2 + X::H2)) * X::B3 + (c3 + X::H3);
}

// W[v][s][s'] = m[T*v + s - s'] for v in V (dehomogenised, zero outside the
// simplex of degree dm); block NV is all zero.
template <int P>
__device__ void build_w(const uint8_t *g, uint8_t *W)
{
    using X = GeoX<P>;
    constexpr int d = X::dm;
    for (int row = threadIdx.x; row < (X::NV + 1) * 16; row += blockDim.x) {
        const int v = row >> 4, s = row & 15;
        const int s1 = s >> 3, s2 = (s >> 2) & 1, s3 = s & 3;
        unsigned w[4] = {0, 0, 0, 0};
        if (v < X::NV) {
            const uint32_t dl = kDX<P>.vpacked[v];
            const int b1 = T1 * unp0(dl) + s1, b2 = T2 * unp1(dl) + s2, b3 = T3 * unp2(dl) + s3;
            // 16 unconditional LDS reads (outside the simplex: index 0, masked after)
            unsigned val[16];
#pragma unroll
            for (int sp = 0; sp < 16; ++sp) {
                const int x1 = b1 - (sp >> 3), x2 = b2 - ((sp >> 2) & 1), x3 = b3 - (sp & 3);
                const int x4 = d - x1 - x2 - x3;
                const bool in = x1 >= 0 && x2 >= 0 && x3 >= 0 && x4 >= 0;
                val[sp] = g[in ? cns_rank(x2, x3, x4) : 0];
                if (!in) val[sp] = 0;
            }
#pragma unroll
            for (int sp = 0; sp < 16; ++sp) w[sp >> 2] |= val[sp] << (8 * (sp & 3));
        }
        *(v4u *)(W + (size_t)row * 16) = v4u{w[0], w[1], w[2], w[3]};
    }
}

// A_1 = m on the shell list 0 (every tile with w(c) <= 2 dm + 4; zero beyond degree dm).
template <int P>
__device__ void init_a1(const uint8_t *g, const uint32_t *list, int ntiles, uint8_t *A)
{
    constexpr int d = GeoX<P>::dm;
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
        const uint32_t t = list[i];
        const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t);
        unsigned w[4] = {0, 0, 0, 0};
        if (T1 * c1 + T2 * c2 + T3 * c3 <= d) {
            unsigned val[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int x1 = T1 * c1 + (s >> 3), x2 = T2 * c2 + ((s >> 2) & 1), x3 = T3 * c3 + (s & 3);
                const int x4 = d - x1 - x2 - x3;
                val[s] = g[x4 >= 0 ? cns_rank(x2, x3, x4) : 0];
                if (x4 < 0) val[s] = 0;
            }
#pragma unroll
            for (int s = 0; s < 16; ++s) w[s >> 2] |= val[s] << (8 * (s & 3));
        }
        gstore16(A + box_tile<P>(c1, c2, c3) * 16, v4u{w[0], w[1], w[2], w[3]});
    }
}

// Zero the tiles of a shell list: the next product reads them as zeros.
template <int P>
__device__ void zero_shell(const uint32_t *list, int ntiles, uint8_t *A)
{
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
        const uint32_t t = list[i];
        gstore16(A + box_tile<P>(unp0(t), unp1(t), unp2(t)) * 16, v4u{0, 0, 0, 0});
    }
}

// x mod p^2 for an accumulator 0 <= x <= C(4J+3,3) (p^2-1)^2 < 2^24 (a sum of
// products of two residues below p^2), in five full-rate fp32 operations instead
// of 32-bit integer multiplies: q = floor(x / p^2) = floor((x + 1/2) / p^2) is
// the truncation of one fma -- (x + 1/2)/p^2 lies at least 1/(2 p^2) from the
// integers and the fma's error stays below that on this range (every x is
// checked on the host) -- and x - q p^2 is an integer below 2^24, exact in fp32.
// (Multipliers with a larger bound take the integer remainder.)
template <int P>
__device__ __attribute__((always_inline)) inline unsigned mod_p2(int x)
{
    constexpr int64_t BOUND = num_mono(4 * Geo<P>::J) * (int64_t)(P * P - 1) * (P * P - 1);
    if constexpr (BOUND < (int64_t)1 << 24) {
        constexpr float C1 = 1.0f / (float)(P * P), C2 = 0.5f / (float)(P * P);
        const float xf = (float)x;
        const float q = __builtin_truncf(__builtin_fmaf(xf, C1, C2));
        return (unsigned)__builtin_fmaf(-q, (float)(P * P), xf);
    } else {
        return (unsigned)x % (unsigned)(P * P);
    }
}

struct EpiCtx {
    int mode;
    bool win;         // capped chain: only the window p^2-1-d <= x_i <= p^2-1 is formed and checked
    uint8_t *dout;    // MODE_DELTA: Delta in CNS order for this surface
    const uint8_t *g; // LDS
    int *err;         // LDS flag
};

// Delta_1 epilogue for the four positions s = 4 kg + v of output tile c:
// D = (g~^p - sum_J b_J^p x^(pJ)) / p mod p (Algorithm 1, lines 3-5).
// Returns the four values packed in a word (byte v for position 4 kg + v;
// positions beyond degree D, and in the capped chain outside the window, give 0).  MODE_DELTA also scatters them to the
// caller's array in CNS order.
template <int P>
__device__ __attribute__((always_inline)) inline unsigned epilogue(int c1, int c2, int c3, int kg, v4i acc,
                                                                   const EpiCtx &ec)
{
    constexpr int P2 = P * P, D = 4 * P * (P - 1);
    const int x1 = T1 * c1 + (kg >> 1), x2 = T2 * c2 + (kg & 1);
    const bool j12 = (x1 % P == 0) && (x2 % P == 0);
    unsigned packed = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int x3 = T3 * c3 + v;
        const int x4 = D - x1 - x2 - x3;
        if (x4 < 0) continue;
        if (ec.win) {
            constexpr int E = P2 - 1, LO = E - 4 * (P - 1);
            if (x1 < LO || x1 > E || x2 < LO || x2 > E || x3 < LO || x3 > E || x4 < LO || x4 > E) continue;
        }
        int val = (int)mod_p2<P>(acc[v]);
        if (j12 && x3 % P == 0) {
            const int bj = ec.g[cns_rank(x2 / P, x3 / P, x4 / P)];
            val -= pow_p_mod_p2<P>(bj);
            if (val < 0) val += P2;
        }
        if (val % P) *ec.err = 1;
        const unsigned dv = (unsigned)(val / P);
        packed |= dv << (8 * v);
        if (ec.mode == MODE_DELTA) gstore1(ec.dout + cns_rank(x2, x3, x4), (uint8_t)dv);
    }
    return packed;
}

// One wave computes NB groups of 16 base tiles (groups gfirst .. gfirst+NB-1
// of the list) and their four shifts, i.e. 4 * NB output groups of
// A_{k+1} = A_k * g~.  Per quad of offsets delta it loads one input fragment
// per group (the 16 tiles q - delta) and one W fragment per shift (blocks
// W_{delta + Delta_s}), then issues 4 * NB products
// D[s][tile] += W[s][(delta, s')] * A[(delta, s')][tile].
template <int P, int NB>
__device__ __attribute__((always_inline)) inline void mfma_set(const uint32_t *list, const uint32_t *gbox, int nbase, int gfirst, int nk, int cap,
                         const uint8_t *W, const uint8_t *__restrict__ Ain, uint8_t *Aout, bool last,
                         const int *toff_l, const uint32_t *widx_l, const uint32_t *qbox_l, uint16_t *qlist,
                         const EpiCtx &ec)
{
    using X = GeoX<P>;
    constexpr int P2 = P * P;
    const int lane = threadIdx.x & 63, kg = lane >> 4, col = lane & 15;

    int64_t base[NB];
    bool ok[NB], gex[NB];
    uint32_t tpk[NB];
    // the set's bounding box from the groups' boxes (uniform loads)
    int smax1 = 0, smax2 = 0, smax3 = 0, swmin = 1 << 30, smin1 = 1 << 30, smin2 = 1 << 30, smin3 = 1 << 30, swmax = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int g0 = (gfirst + b) * 16;
        gex[b] = g0 < nbase;
        const int idx = g0 + col;
        ok[b] = idx < nbase;
        const uint32_t t = gex[b] ? list[ok[b] ? idx : g0] : 0u;
        tpk[b] = t;
        base[b] = box_tile<P>(unp0(t), unp1(t), unp2(t));
        if (gex[b]) {
            const uint32_t *gb = gbox + 4 * (gfirst + b);
            const uint32_t w0 = gb[0], w1 = gb[1], w2 = gb[2], w3 = gb[3];
            smax1 = max(smax1, (int)(w0 & 0xFFFFu));
            smax2 = max(smax2, (int)(w0 >> 16));
            smax3 = max(smax3, (int)(w1 & 0xFFFFu));
            smin1 = min(smin1, (int)(w1 >> 16));
            smin2 = min(smin2, (int)(w2 & 0xFFFFu));
            smin3 = min(smin3, (int)(w2 >> 16));
            swmin = min(swmin, (int)(w3 & 0xFFFFu));
            swmax = max(swmax, (int)(w3 >> 16));
        }
    }
    smax1 = uniform(smax1);
    smax2 = uniform(smax2);
    smax3 = uniform(smax3);
    smin1 = uniform(smin1);
    smin2 = uniform(smin2);
    smin3 = uniform(smin3);
    swmin = uniform(swmin);
    swmax = uniform(swmax);
    v4i acc[4][NB];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[s][b] = v4i{0, 0, 0, 0};

    // A quad whose input tiles q - delta all lie outside A_k (a negative
    // coordinate, or weight above deg A_k; in the capped chain also outside
    // the cap) contributes nothing and is skipped.  For the quads that are
    // processed, every group and every shift is multiplied: tiles outside A_k
    // read the zero halo or the zeroed shell and the zero W block adds
    // nothing, so the products stay exact and the loop has no branches
    // around the matrix instructions.
    // the quads this set needs, in order, into the wave's list in LDS
    int nq = 0;
    for (int q0 = 0; q0 < X::NQX; q0 += 64) {
        const int q = q0 + lane;
        bool nd = false;
        if (q < X::NQX)
            nd = quad_needed(smax1, smax2, smax3, swmin, smin1, smin2, smin3, swmax, nk, cap, qbox_l[4 * q],
                             (int)qbox_l[4 * q + 1], qbox_l[4 * q + 2], (int)qbox_l[4 * q + 3]);
        const uint64_t m = __ballot(nd);
        if (nd) qlist[nq + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)q;
        nq += __popcll(m);
    }
    nq = uniform(nq);
    // pad to a multiple of the prefetch depth with the null quad (index NQX:
    // offset 0, zero W blocks)
    {
        const int npad = (DEEP_PF - nq % DEEP_PF) % DEEP_PF;
        if (lane < npad) qlist[nq + lane] = (uint16_t)X::NQX;
        nq += npad;
    }

    // byte offsets of the tiles inside the box fit in 32 bits
    uint32_t boff[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) boff[b] = (uint32_t)base[b] * 16u;
    const uint32_t wrow = (uint32_t)col * 16u;
    // Software pipeline over the list.  For list entry e the steps are, each
    // one loop step before the next: read its quad index; read its tile offset
    // and packed W-block indices; issue its input-fragment loads into slot
    // e mod DEEP_PF (DEEP_PF entries ahead of its products); read its W
    // fragments from LDS; issue its 4 x NB products.  So no LDS round trip
    // sits right before the matrix instructions.  Entries past the end
    // repeat the last one (the list is padded with null quads).
#define QFS_ENTRY(I) ((I) < nq ? (I) : nq - 1)
    // index data of entry I from its quad q
#define QFS_INDEX(Q)                                                                               \
    do {                                                                                           \
        tn = toff_l[4 * (Q) + kg];                                                                 \
        wan = widx_l[2 * (4 * (Q) + kg)];                                                          \
        wbn = widx_l[2 * (4 * (Q) + kg) + 1];                                                      \
    } while (0)
    // slot J <- the staged entry: W indices and input fragments
#define QFS_LOAD_B(J)                                                                              \
    do {                                                                                           \
        const uint32_t to_ = (uint32_t)tn * 16u;                                                   \
        wa[J] = wan;                                                                               \
        wb[J] = wbn;                                                                               \
        _Pragma("unroll") for (int b = 0; b < NB; ++b) bf[J][b] = gload16(Ain + (boff[b] - to_));  \
    } while (0)
    // W fragments (four shifts) of the entry in slot J into buffer K
#define QFS_LOAD_W(K, J)                                                                                   \
    do {                                                                                                   \
        _Pragma("unroll") for (int s = 0; s < 4; ++s)                                                      \
        {                                                                                                  \
            const uint32_t wi = ((s < 2 ? wa[J] : wb[J]) >> (16 * (s & 1))) & 0xFFFFu;                      \
            wf[K][s] = w_in_lds<P>() ? *(const v4i *)(W + wi * 256u + wrow) : gload16(W + wi * 256u + wrow); \
        }                                                                                                  \
    } while (0)
    // the 4 x NB products of the entry in slot J with W buffer K
#define QFS_PRODUCTS(K, J)                                                                         \
    do {                                                                                           \
        _Pragma("unroll") for (int s = 0; s < 4; ++s)                                              \
            _Pragma("unroll") for (int b = 0; b < NB; ++b)                                         \
                acc[s][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wf[K][s], bf[J][b], acc[s][b], 0, 0, 0); \
    } while (0)

    static_assert(DEEP_PF % 2 == 0, "W buffers alternate per entry");
    if (nq > 0) {
        v4i bf[DEEP_PF][NB], wf[2][4];
        uint32_t wa[DEEP_PF], wb[DEEP_PF];
        int tn;
        uint32_t wan, wbn;
#pragma unroll
        for (int j = 0; j < DEEP_PF; ++j) {
            QFS_INDEX(uniform(qlist[QFS_ENTRY(j)]));
            QFS_LOAD_B(j);
            __builtin_amdgcn_sched_barrier(0);
        }
        QFS_LOAD_W(0, 0);
        QFS_INDEX(uniform(qlist[QFS_ENTRY(DEEP_PF)]));
        int qv = qlist[QFS_ENTRY(DEEP_PF + 1)];
        __builtin_amdgcn_sched_barrier(0);
        // at the top of an iteration slot j holds entry i + j, the staged index
        // data is entry i + DEEP_PF's and qv holds entry i + DEEP_PF + 1's quad
        for (int i = 0; i < nq; i += DEEP_PF) {
#pragma unroll
            for (int j = 0; j < DEEP_PF; ++j) {
                QFS_LOAD_W((j + 1) & 1, (j + 1) % DEEP_PF);
                __builtin_amdgcn_sched_barrier(0);
                QFS_PRODUCTS(j & 1, j);
                __builtin_amdgcn_sched_barrier(0);
                QFS_LOAD_B(j);
                const int q_ = uniform(qv);
                qv = qlist[QFS_ENTRY(i + j + DEEP_PF + 2)];
                QFS_INDEX(q_);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
#undef QFS_ENTRY
#undef QFS_INDEX
#undef QFS_LOAD_B
#undef QFS_LOAD_W
#undef QFS_PRODUCTS

    constexpr int64_t SH1 = (int64_t)X::B2 * X::B3, SH2 = X::B3;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!gex[b] || !ok[b]) continue;
        const int c1 = unp0(tpk[b]), c2 = unp1(tpk[b]), c3 = unp2(tpk[b]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int d1 = s & 1, d2 = s >> 1;
            unsigned packed = 0;
            if (!last) {
#pragma unroll
                for (int v = 0; v < 4; ++v) packed |= mod_p2<P>(acc[s][b][v]) << (8 * v);
            } else {
                packed = epilogue<P>(c1 + d1, c2 + d2, c3, kg, acc[s][b], ec);
            }
            gstore4(Aout + (base[b] + d1 * SH1 + d2 * SH2) * 16 + 4 * kg, packed);
        }
    }
}

// c(theta(a)) = sum_c a[c] Delta[(p+1) e - c] mod p, read from Delta's tile box:
// the only coefficient of theta(a) the height test needs (Section 3.4).
template <int P>
__device__ int theta_test_box(const uint8_t *dbox, const uint8_t *a, int *red)
{
    constexpr int d = 4 * (P - 1), LG = (int)num_mono(d), E = P * P - 1;
    unsigned part = 0;
    for (int c = threadIdx.x; c < LG; c += blockDim.x) {
        const unsigned av = a[c];
        if (!av) continue;
        int c1, c2, c3, c4;
        cns_unrank(d, c, c1, c2, c3, c4);
        const int x1 = E - c1, x2 = E - c2, x3 = E - c3;
        const int64_t t = box_tile<P>(x1 >> 1, x2 >> 1, x3 >> 2);
        part += av * gload1(dbox + t * 16 + (x1 & 1) * 8 + (x2 & 1) * 4 + (x3 & 3));
    }
    return block_sum((int)(part % P), red) % P;
}

// g = A mod p for the chain link A = f~^(p-1) mod p^2 in a tile box, into g_l
// (LDS, CNS order) and, if given, out.
template <int P>
__device__ void g_from_box(const uint8_t *A, uint8_t *g_l, uint8_t *out)
{
    constexpr int d = 4 * (P - 1), LG = (int)num_mono(d);
    for (int r = threadIdx.x; r < LG; r += blockDim.x) {
        int x1, x2, x3, x4;
        cns_unrank(d, r, x1, x2, x3, x4);
        const uint8_t v =
            (uint8_t)(gload1(A + box_tile<P>(x1 >> 1, x2 >> 1, x3 >> 2) * 16 + (x1 & 1) * 8 + (x2 & 1) * 4 + (x3 & 3)) % P);
        g_l[r] = v;
        if (out) gstore1(out + r, v);
    }
}

// Delta in the Cartier-split layout dl (global) from its tile box.  A wave
// takes groups of U coarse blocks (SplitGeo); it keeps the tile loads of the
// next SPLIT_DEPTH - 1 groups in flight in registers, stages one group's tiles
// position-major in its LDS stage, and assembles the group's chunks there.  A
// lane always builds the same column chunk (region j, columns 16m..16m+15) of
// row y = (y1, y2, y3, d - j - y1 - y2 - y3); in the staged block the byte of
// column sigma lies at base(p y mod T) + lin(sigma), so the lane keeps its 16
// lin(sigma) and adds one base per block.  stage: DEEP_NW * STAGE bytes of LDS;
// sig_l: the column table (LDS).  A wave's LDS operations complete in issue
// order, so the stage needs only a compiler barrier between its writes and
// reads (a memory fence would also wait for the prefetched tile loads).
constexpr int SPLIT_DEPTH = 4;
template <int P>
__device__ void cartier_split_box(const uint8_t *__restrict__ dbox, uint8_t *dl, uint8_t *stage, const uint16_t *sig_l)
{
    using TG = ThetaGeo<P>;
    using SG = SplitGeo<P>;
    using X = GeoX<P>;
    constexpr int d = TG::d, NJ = TG::J, NCUBE = SG::NCUBE;
    constexpr int NT1 = SG::NT1, NT3 = SG::NT3, NTB = SG::NTB, U = SG::U, NL = SG::NL;
    constexpr int W2 = SG::W2, W3 = SG::W3, CUBE = SG::CUBE;
    constexpr int KPL = (U * SG::NCH + 63) / 64;  // chunks per lane and group
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint8_t *st = stage + wave * SG::STAGE;
    // the tiles of the U blocks from coarse index t0 into registers
    auto load_group = [&](int t0, v4u *v) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int i = lane + 64 * l, u = i / NTB, r = i % NTB;
            v[l] = v4u{0, 0, 0, 0};
            if (u < U && t0 + u < NCUBE) {
                const uint32_t cb = kCube<P>.c[t0 + u];
                const int c1 = ((P * (int)(cb & 255u)) >> 1) + r / (NT1 * NT3),
                          c2 = ((P * (int)((cb >> 8) & 255u)) >> 1) + (r / NT3) % NT1,
                          c3 = ((P * (int)(cb >> 16)) >> 2) + r % NT3;
                if (c1 <= X::C1 && c2 <= X::C2 && c3 < X::C3) v[l] = gload16u(dbox + box_tile<P>(c1, c2, c3) * 16);
            }
        }
    };
    // this lane's chunks: block u of the group, region j, column chunk m, and the
    // staged offsets lin(sigma) of its 16 columns (two per word; pad: bit q set)
    int ku[KPL], kj[KPL], km[KPL], krs[KPL];
    int64_t kro[KPL];
    unsigned klin[KPL][8], kpad[KPL];
#pragma unroll
    for (int c = 0; c < KPL; ++c) {
        const int k = lane + 64 * c, kc = k % SG::NCH;
        ku[c] = k < U * SG::NCH ? k / SG::NCH : U;  // U: no chunk
        int j = 0;
#pragma unroll
        for (int r = 1; r < NJ; ++r)
            if (kc * 16 >= TG::col_off(r)) j = r;
        int cb = 0;
        krs[c] = 0;
        kro[c] = 0;
#pragma unroll
        for (int r = 0; r < NJ; ++r)
            if (j == r) {
                cb = TG::col_off(r);
                krs[c] = TG::rs(r);
                kro[c] = TG::region_off(r);
            }
        kj[c] = j;
        km[c] = kc - cb / 16;
        kpad[c] = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const unsigned sv = sig_l[cb + 16 * km[c] + q];
            const unsigned lin = sv == 0xFFFFu ? 0u
                                               : ((sv & 15u) * W2 + ((sv >> 4) & 15u)) * W3 + ((sv >> 8) & 15u);
            if (sv == 0xFFFFu) kpad[c] |= 1u << q;
            if (q & 1)
                klin[c][q >> 1] |= lin << 16;
            else
                klin[c][q >> 1] = lin;
        }
    }
    const int stride = nw * U;
    v4u ring[SPLIT_DEPTH][NL];
#pragma unroll
    for (int s = 0; s < SPLIT_DEPTH; ++s)
        if (wave * U + s * stride < NCUBE) load_group(wave * U + s * stride, ring[s]);
    for (int tb = wave * U; tb < NCUBE; tb += SPLIT_DEPTH * stride) {
#pragma unroll
        for (int s = 0; s < SPLIT_DEPTH; ++s) {
            const int t0 = tb + s * stride;
            if (t0 >= NCUBE) break;
            // tile (i1, i2, i3) of block u: its rows (s1, s2) of 4 bytes to positions (2 i1 + s1, 2 i2 + s2, 4 i3..4 i3 + 3)
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int i = lane + 64 * l;
                if (i < U * NTB) {
                    const int u = i / NTB, r = i % NTB;
                    const int i1 = r / (NT1 * NT3), i2 = (r / NT3) % NT1, i3 = r % NT3;
                    uint8_t *blk = st + u * CUBE + 4 * i3;
                    *(unsigned *)(blk + ((2 * i1) * W2 + 2 * i2) * W3) = ring[s][l].x;
                    *(unsigned *)(blk + ((2 * i1) * W2 + 2 * i2 + 1) * W3) = ring[s][l].y;
                    *(unsigned *)(blk + ((2 * i1 + 1) * W2 + 2 * i2) * W3) = ring[s][l].z;
                    *(unsigned *)(blk + ((2 * i1 + 1) * W2 + 2 * i2 + 1) * W3) = ring[s][l].w;
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (t0 + SPLIT_DEPTH * stride < NCUBE) load_group(t0 + SPLIT_DEPTH * stride, ring[s]);
#pragma unroll
            for (int c = 0; c < KPL; ++c) {
                const int u = ku[c];
                if (u >= U || t0 + u >= NCUBE) continue;
                const uint32_t cb = kCube<P>.c[t0 + u];
                const int y1 = (int)(cb & 255u), y2 = (int)((cb >> 8) & 255u), y3 = (int)(cb >> 16);
                const int y4 = d - kj[c] - y1 - y2 - y3;
                if (y4 < 0) continue;
                const uint8_t *blk = st + u * CUBE + ((((P * y1) & 1) * W2 + ((P * y2) & 1)) * W3 + ((P * y3) & 3));
                unsigned w[4] = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    unsigned b = blk[(klin[c][q >> 1] >> (16 * (q & 1))) & 0xFFFFu];
                    if ((kpad[c] >> q) & 1u) b = 0;
                    w[q >> 2] |= b << (8 * (q & 3));
                }
                gstore16(dl + kro[c] + (int64_t)cns_rank(y2, y3, y4) * krs[c] + 16 * km[c], v4u{w[0], w[1], w[2], w[3]});
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// Delta at a position x (degree D) from its tile box.
template <int P>
struct BoxDelta {
    const uint8_t *dbox;
    __device__ uint8_t operator()(int x1, int x2, int x3, int) const
    {
        return gload1(dbox + box_tile<P>(x1 >> 1, x2 >> 1, x3 >> 2) * 16 + (x1 & 1) * 8 + (x2 & 1) * 4 + (x3 & 3));
    }
};

// The chain A_{k+1} = A_k * m, k = 1..NF-1, into the two tile boxes, from the
// W blocks and m already in place: in full, or (band) only the super-tiles
// that the height-2 test depends on, ending in the window of Delta it reads.
// A_NF ends in buf[(NF-1) & 1].  When g_from_chain<P>(), g is read off the
// link A_{(p-1)/J} into g_l (and g_out) before the last product needs it.
template <int P>
__device__ __attribute__((always_inline)) inline void run_chain(bool band, const uint32_t *plan, const uint8_t *m_l,
                                                               const uint8_t *W, uint8_t *buf0, uint8_t *buf1,
                                                               const int *toff_l, const uint32_t *widx_l,
                                                               const uint32_t *qbox_l, uint16_t *qlist_w, EpiCtx ec,
                                                               uint8_t *g_l, uint8_t *g_out)
{
    constexpr int d = GeoX<P>::dm, NF = GeoX<P>::NF;
    const int wave = uniform(threadIdx.x >> 6);
    const int cap = band ? P * P - 1 : CAP_NONE;
    init_a1<P>(m_l, plan + kPT<P>.foff[0], (int)kPT<P>.flen[0], buf0);
    __syncthreads();
    for (int k = 1; k < NF; ++k) {
        const uint8_t *Ain = (k & 1) ? buf0 : buf1;
        uint8_t *Aout = (k & 1) ? buf1 : buf0;
        const int nbase = (int)(band ? kPT<P>.nlen[k] : kPT<P>.blen[k]);
        const uint32_t *list = plan + (band ? kPT<P>.noff[k] : kPT<P>.boff[k]);
        const uint32_t *gbox = plan + (band ? kPT<P>.ngoff[k] : kPT<P>.gboff[k]);
        const bool last = (k == NF - 1);
        ec.win = band && last;
        // whole rounds of DEEP_NB-group sets, one per wave; the groups left
        // over go out in sets of DEEP_NB/2 so that more waves share the tail
        const int ngroups = (nbase + 15) / 16;
        const int rounds = ngroups / (DEEP_NB * DEEP_NW);
        for (int i = 0; i < rounds; ++i)
            mfma_set<P, DEEP_NB>(list, gbox, nbase, (i * DEEP_NW + wave) * DEEP_NB, k * d, cap, W, Ain, Aout, last, toff_l,
                                 widx_l, qbox_l, qlist_w, ec);
        constexpr int NB2 = DEEP_NB / 2;
        for (int g = rounds * DEEP_NB * DEEP_NW + wave * NB2; g < ngroups; g += DEEP_NW * NB2)
            mfma_set<P, NB2>(list, gbox, nbase, g, k * d, cap, W, Ain, Aout, last, toff_l, widx_l, qbox_l, qlist_w, ec);
        if (!last)
            zero_shell<P>(plan + (band ? kPT<P>.hoff[k] : kPT<P>.foff[k]), (int)(band ? kPT<P>.hlen[k] : kPT<P>.flen[k]),
                          Aout);
        __syncthreads();
        if constexpr (g_from_chain<P>()) {
            // A_{k+1} = f~^(p-1) mod p^2; the next barrier precedes the last product
            if (k + 1 == (P - 1) / Geo<P>::J) g_from_box<P>(Aout, g_l, g_out);
        }
    }
}

// Persistent deep kernel: each workgroup pops surfaces (queue positions) and
// owns one slot (two tile boxes and the Cartier-split Delta).
//  BAND (MODE_HEIGHT): the capped chain and the first test; h = 2 (or, for
//    bound 2, infinity) is written at once, other surfaces go to the second queue.
//  !BAND: the full chain g~^p with the Delta_1 epilogue, then (MODE_HEIGHT)
//    Algorithm 3's theta loop, or (MODE_DELTA) Delta written out in CNS order.
template <int P, bool BAND>
__global__ __launch_bounds__(DEEP_NT, QFS_DEEP_MINWG) void k_deep(DeepArgs a)
{
    using PR = Prime<P>;
    using X = GeoX<P>;
    using L = DeepLds<P>;
    constexpr int LG = PR::len_g;
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *g_l = lds + L::off_g;
    uint8_t *aperm = lds + L::off_aperm;
    int *toff_l = (int *)(lds + L::off_toff);
    uint32_t *widx_l = (uint32_t *)(lds + L::off_widx);
    uint32_t *qbox_l = (uint32_t *)(lds + L::off_qbox);
    uint16_t *qlist_l = (uint16_t *)(lds + L::off_qlist);
    int *red = (int *)(lds + L::off_red);
    uint32_t *sums = (uint32_t *)(lds + L::off_sums);
    uint16_t *sig_l = (uint16_t *)(lds + L::off_sig);
    __shared__ int s_pos, s_err;

    const int tid = threadIdx.x, wave = uniform(tid >> 6);
    const int pi = prime_index(P);
    uint8_t *slot = a.slots + (size_t)blockIdx.x * a.slot_bytes;
    uint8_t *wg = slot;
    uint8_t *bufs = slot + (w_in_lds<P>() ? 0 : align256(X::W_BYTES));
    uint8_t *buf[2] = {bufs, bufs + align256(X::BOX_BYTES)};
    uint8_t *dl = bufs + 2 * align256(X::BOX_BYTES);
    uint8_t *W = w_in_lds<P>() ? lds + L::off_w : wg;

    const bool q2 = !BAND && a.from_q2;
    const int count = a.counters[(q2 ? CNT_Q2 : CNT_COUNT) + pi];
    const int popc = (q2 ? CNT_POP2 : CNT_POP) + pi;
    if ((int)blockIdx.x >= count) return;  // more workgroups than surfaces: nothing to do
    for (int i = tid; i < X::NVXP; i += DEEP_NT) {
        toff_l[i] = kDX<P>.toff[i];
        widx_l[2 * i] = kDX<P>.widx[i][0];
        widx_l[2 * i + 1] = kDX<P>.widx[i][1];
    }
    if (tid < 4) {  // the null quad
        toff_l[X::NVXP + tid] = 0;
        widx_l[2 * (X::NVXP + tid)] = widx_l[2 * (X::NVXP + tid) + 1] = (uint32_t)X::NV | ((uint32_t)X::NV << 16);
    }
    if (!BAND)
        for (int i = tid; i < ThetaGeo<P>::NCOL; i += DEEP_NT) sig_l[i] = kTT<P>.sig[i];
    for (int i = tid; i < X::NQX; i += DEEP_NT) {
        qbox_l[4 * i] = kDX<P>.qmin[i];
        qbox_l[4 * i + 1] = (uint32_t)kDX<P>.qwmax[i];
        qbox_l[4 * i + 2] = kDX<P>.qmax[i];
        qbox_l[4 * i + 3] = (uint32_t)kDX<P>.qwmin[i];
    }
    // the halo (tiles with a negative coordinate) of both boxes is read as zero and never written
    if (a.zero_halo)
        for (int64_t t = tid; t < X::BOX_TILES; t += DEEP_NT) {
            const int i3 = (int)(t % X::B3);
            const int64_t r = t / X::B3;
            const int i2 = (int)(r % X::B2), i1 = (int)(r / X::B2);
            if (i1 < X::H1 || i2 < X::H2 || i3 < X::H3) {
                gstore16(buf[0] + t * 16, v4u{0, 0, 0, 0});
                gstore16(buf[1] + t * 16, v4u{0, 0, 0, 0});
            }
        }

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            s_pos = atomicAdd(&a.counters[popc], 1);
            s_err = 0;
        }
        __syncthreads();
        const int pos = s_pos;
        if (pos >= count) break;
        const int qpos = q2 ? a.queue2[pos] : pos;  // position in the first queue
        const int surf = a.queue[qpos];
        if constexpr (!g_from_chain<P>())
            for (int i = tid; i < LG; i += DEEP_NT) g_l[i] = a.gq[(size_t)qpos * LG + i];
        const uint8_t *m_l = g_l;
        if constexpr (L::OWN_M) {
            __shared__ __align__(16) uint8_t f35[48];
            __shared__ int ntap;
            if (tid < 35) f35[tid] = (uint8_t)(a.f[(size_t)surf * 35 + tid] % P);
            __syncthreads();
            m_l = fpow_mod_lds<Geo<P>::J, P * P>(f35, lds + L::off_m0, lds + L::off_m1, (uint32_t *)(lds + L::off_taps),
                                                 &ntap);
        }
        __syncthreads();
        build_w<P>(m_l, W);
        __syncthreads();

        EpiCtx ec;
        ec.mode = a.mode;
        ec.win = false;
        ec.dout = a.delta_out ? a.delta_out + (size_t)surf * PR::len_D : nullptr;
        ec.g = g_l;
        ec.err = &s_err;
        uint16_t *qlist_w = qlist_l + wave * L::QSTRIDE;
        uint8_t *g_out = a.mode == MODE_DELTA && a.g_out ? a.g_out + (size_t)surf * LG : nullptr;
        run_chain<P>(BAND, a.plan, m_l, W, buf[0], buf[1], toff_l, widx_l, qbox_l, qlist_w, ec, g_l, g_out);
        const bool err = s_err != 0;

        if (BAND) {
            // h = 2 needs only the window of Delta the first test reads
            int hv = -1;
            if (err)
                hv = -5; /* QFS_EARITH */
            else if (theta_test_box<P>(buf[(X::NF - 1) & 1], g_l, red) != 0)
                hv = 2;
            else if (a.bound == 2)
                hv = 0;
            if (tid == 0) {
                if (hv != -1)
                    a.heights[surf] = hv;
                else
                    a.queue2[atomicAdd(&a.counters[CNT_Q2 + pi], 1)] = qpos;
            }
            continue;
        }
        if (a.mode == MODE_DELTA) {
            if (tid == 0 && err && a.status) a.status[surf] = -5; /* QFS_EARITH */
            continue;
        }
        if (err) {
            if (tid == 0) a.heights[surf] = -5;
            continue;
        }
        // Algorithm 3's loop: the test at h reads c(theta(a)) only, a = theta^(h-2)(g);
        // theta(a) in full is formed when the surface goes on to the next h.
        // Surfaces from the second queue are known to fail the test at h = 2.
        const uint8_t *dbox = buf[(X::NF - 1) & 1];
        int h = 0;
        const bool h2 = !q2 && theta_test_box<P>(dbox, g_l, red) != 0;
        if (h2) h = 2;
        if (!h2 && a.bound > 2) {
            cartier_split_box<P>(dbox, dl, (uint8_t *)sums, sig_l);
            for (int hh = 3; hh <= a.bound; ++hh) {
                build_aperm<P>(g_l, aperm);
                __syncthreads();
                theta_full<P>(dl, aperm, sums, g_l);
                __syncthreads();
                if (theta_test_box<P>(dbox, g_l, red) != 0) {
                    h = hh;
                    break;
                }
            }
        }
        if (tid == 0) a.heights[surf] = h;
    }
}

// LDS limit of the deep kernels, set once per process (before any launch, so
// also before a graph capture)
template <int P, bool BAND>
static hipError_t deep_attr()
{
    static const hipError_t attr = hipFuncSetAttribute((const void *)k_deep<P, BAND>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)DeepLds<P>::bytes);
    return attr;
}

hipError_t prepare_deep(int p)
{
    hipError_t e = hipErrorInvalidValue;
    switch (p) {
    case 3: e = deep_attr<3, true>(); return e != hipSuccess ? e : deep_attr<3, false>();
    case 5: e = deep_attr<5, true>(); return e != hipSuccess ? e : deep_attr<5, false>();
    case 7: e = deep_attr<7, true>(); return e != hipSuccess ? e : deep_attr<7, false>();
    case 11: e = deep_attr<11, true>(); return e != hipSuccess ? e : deep_attr<11, false>();
    }
    return e;
}

template <int P, bool BAND>
static hipError_t launch_deep_pb(const DeepArgs &a, int nslots, hipStream_t s)
{
    const hipError_t attr = deep_attr<P, BAND>();
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_deep<P, BAND>), dim3(nslots), dim3(DEEP_NT), DeepLds<P>::bytes, s, a);
    return hipGetLastError();
}

template <int P>
static hipError_t launch_deep_p(bool band, const DeepArgs &a, int nslots, hipStream_t s)
{
    return band ? launch_deep_pb<P, true>(a, nslots, s) : launch_deep_pb<P, false>(a, nslots, s);
}

hipError_t launch_deep(int p, bool band, const DeepArgs &a, int nslots, hipStream_t s)
{
    switch (p) {
    case 3: return launch_deep_p<3>(band, a, nslots, s);
    case 5: return launch_deep_p<5>(band, a, nslots, s);
    case 7: return launch_deep_p<7>(band, a, nslots, s);
    case 11: return launch_deep_p<11>(band, a, nslots, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// MFMA instructions per surface (host): the deep kernel's skip tests depend
// only on the geometry, so this replays them.
// ---------------------------------------------------------------------------
template <int P>
static int64_t mfma_count_p(bool band)
{
    using X = GeoX<P>;
    constexpr int d = X::dm, E = P * P - 1;
    static const DeltaTableX<P> DX = make_delta_table_x<P>();
    int64_t total = 0;
    for (int k = 1; k < X::NF; ++k) {
        const int n = (k + 1) * d, nk = k * d, cap = band ? E : (1 << 20);
        std::vector<uint32_t> tiles;  // the list in k_plan's order
        const PlanBlocks nb = plan_blocks(n);
        for (int b = 0; b < nb.n1 * nb.n2 * nb.n3; ++b)
            plan_block_emit(n, b, [&](uint32_t t) { return !band || band_tile_packed<P>(n, t); },
                            [&](int, uint32_t t) { tiles.push_back(t); });
        const int nt = (int)tiles.size();
        if (nt != (band ? kPlanTable<P>.nlen[k] : kPlanTable<P>.blen[k])) return -1;  // list lengths disagree
        const int ngroups = (nt + 15) / 16;
        const int rounds = ngroups / (DEEP_NB * DEEP_NW);
        // (first group, groups) of every set k_deep multiplies
        std::vector<std::pair<int, int>> sets;
        for (int g = 0; g < rounds * DEEP_NB * DEEP_NW; g += DEEP_NB) sets.push_back({g, DEEP_NB});
        for (int g = rounds * DEEP_NB * DEEP_NW; g < ngroups; g += DEEP_NB / 2) sets.push_back({g, DEEP_NB / 2});
        for (const auto &st : sets) {
            int m1 = 0, m2 = 0, m3 = 0, wmin = 1 << 30, l1 = 1 << 30, l2 = 1 << 30, l3 = 1 << 30, wmax = 0;
            for (int g = st.first * 16; g < std::min(nt, (st.first + st.second) * 16); ++g) {
                const uint32_t t = tiles[g];
                m1 = std::max(m1, unp0(t));
                m2 = std::max(m2, unp1(t));
                m3 = std::max(m3, unp2(t));
                l1 = std::min(l1, unp0(t));
                l2 = std::min(l2, unp1(t));
                l3 = std::min(l3, unp2(t));
                wmin = std::min(wmin, T1 * unp0(t) + T2 * unp1(t) + T3 * unp2(t));
                wmax = std::max(wmax, T1 * unp0(t) + T2 * unp1(t) + T3 * unp2(t));
            }
            int nq = 0;
            for (int q = 0; q < X::NQX; ++q)
                nq += quad_needed(m1, m2, m3, wmin, l1, l2, l3, wmax, nk, cap, DX.qmin[q], DX.qwmax[q], DX.qmax[q],
                                  DX.qwmin[q]);
            nq += (DEEP_PF - nq % DEEP_PF) % DEEP_PF;  // null-quad padding
            total += (int64_t)nq * 4 * st.second;
        }
    }
    return total;
}

int64_t mfma_count(int p, bool band)
{
    static int64_t cache[2][4] = {{-1, -1, -1, -1}, {-1, -1, -1, -1}};
    const int pi = prime_index(p);
    if (pi < 0) return -1;
    int64_t &c = cache[band ? 1 : 0][pi];
    if (c == -1) {
        switch (p) {
        case 3: c = mfma_count_p<3>(band); break;
        case 5: c = mfma_count_p<5>(band); break;
        case 7: c = mfma_count_p<7>(band); break;
        case 11: c = mfma_count_p<11>(band); break;
        }
    }
    return c;
}

// ---------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------
int64_t len_g_of(int p)
{
    return num_mono(4 * (p - 1));
}

static size_t slot_bytes_of(int p)
{
    switch (p) {
    case 3: return slot_bytes<3>();
    case 5: return slot_bytes<5>();
    case 7: return slot_bytes<7>();
    case 11: return slot_bytes<11>();
    }
    return 0;
}

static size_t plan_bytes_of(int p)
{
    switch (p) {
    case 3: return (size_t)plan_words<3>() * 4;
    case 5: return (size_t)plan_words<5>() * 4;
    case 7: return (size_t)plan_words<7>() * 4;
    case 11: return (size_t)plan_words<11>() * 4;
    }
    return 0;
}

// The slot area is held to SLOT_AREA_MAX (fewer persistent workgroups beyond it).
constexpr size_t SLOT_AREA_MAX = (size_t)96 << 30;

BatchLayout make_batch_layout(const bool present[4], int batch, int slots)
{
    BatchLayout L;
    size_t off = align256(CNT_WORDS * sizeof(int32_t));
    for (int i = 0; i < 4; ++i) {
        L.present[i] = present[i];
        if (!present[i]) continue;
        const int p = kPrimes[i];
        L.queue[i] = off;
        off += align256((size_t)batch * sizeof(int32_t));
        L.queue2[i] = off;
        off += align256((size_t)batch * sizeof(int32_t));
        L.gq[i] = off;
        off += align256((size_t)batch * (size_t)len_g_of(p));
        L.plan[i] = off;
        off += align256(plan_bytes_of(p));
        // `slots` persistent workgroups (one per compute unit by default), the
        // slot area held to SLOT_AREA_MAX (a p = 11 slot is 242 MB)
        int ns = slots;
        const size_t cap = SLOT_AREA_MAX / slot_bytes_of(p);
        if ((size_t)ns > cap) ns = (int)cap;
        if (ns > batch) ns = batch;
        L.nslots[i] = ns > 0 ? ns : 1;
        L.slot_stride[i] = slot_bytes_of(p);
    }
    // the deep kernels of different primes run one after another and share the slot area
    size_t slots_total = 0;
    for (int i = 0; i < 4; ++i)
        if (present[i]) {
            const size_t need = (size_t)L.nslots[i] * L.slot_stride[i];
            if (need > slots_total) slots_total = need;
        }
    L.slots = off;
    off += align256(slots_total);
    L.total = off;
    return L;
}

}  // namespace qfs
