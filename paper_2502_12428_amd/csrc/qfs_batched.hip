// Batched height and Delta_1 kernels for gfx950.
//
// Stage 1 (one workgroup per surface): g = f^(p-1) mod p and Fedder's test
//   (g not in m^[p] iff its coefficient at (x1..x4)^(p-1) is nonzero, the only
//   monomial of degree 4(p-1) outside m^[p] -- Section 3.4).  Surfaces that
//   fail it ("deep" surfaces) are compacted into a per-prime queue together
//   with g.
// Deep kernel (persistent; each workgroup pops surfaces from the queue):
//   g~^p mod p^2 by the chain A_{k+1} = A_k * g~ (k = 1..p-1) on int8 matrix
//   cores with int32 accumulation (Algorithm 1, line 2), the Delta_1 epilogue
//   fused into the last product (Algorithm 1, lines 3-5), then the theta loop
//   of Algorithm 3 with its one-coefficient test.
#include <algorithm>
#include <vector>

#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

template <int P>
__constant__ PlanTable<P> kPT = make_plan_table<P>();

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
// stage 1
// ---------------------------------------------------------------------------
template <int P>
__device__ void stage1_one(const Stage1Args &a, int surf, uint8_t *lds)
{
    using PR = Prime<P>;
    constexpr int LG = PR::len_g;
    constexpr int LGA = (LG + 15) / 16 * 16;
    uint8_t *f35 = lds;
    int *flag = (int *)(lds + 48);
    uint8_t *b0 = lds + 64, *b1 = b0 + LGA;
    const int tid = threadIdx.x, pi = prime_index(P);
    if (tid == 0) flag[0] = 0;
    __syncthreads();
    if (tid < 35) {
        const int v = a.f[(size_t)surf * 35 + tid];
        f35[tid] = (uint8_t)(v % P);
        if (v >= P) atomicOr(flag, 1);
    }
    __syncthreads();
    const bool bad = flag[0] != 0;
    const uint8_t *g = fpow_lds<P>(f35, b0, b1);
    const bool deep = g[PR::e_index] == 0;
    if (a.mode == MODE_HEIGHT) {
        if (bad) {
            if (tid == 0) a.heights[surf] = -1; /* QFS_EINVAL */
            return;
        }
        if (!deep || a.bound < 2) {
            if (tid == 0) a.heights[surf] = deep ? 0 : 1;
            return;
        }
        __syncthreads();
        if (tid == 0) flag[1] = atomicAdd(&a.counters[CNT_COUNT + pi], 1);
        __syncthreads();
        const int pos = flag[1];
        if (tid == 0) a.queue[pi][pos] = surf;
        uint8_t *dst = a.gq[pi] + (size_t)pos * LG;
        for (int i = tid; i < LG; i += blockDim.x) dst[i] = g[i];
    } else {
        if (tid == 0) {
            a.queue[pi][surf] = surf;
            if (a.status) a.status[surf] = bad ? -1 : 0;
            if (surf == 0) a.counters[CNT_COUNT + pi] = a.batch;
        }
        uint8_t *dst = a.gq[pi] + (size_t)surf * LG;
        for (int i = tid; i < LG; i += blockDim.x) dst[i] = g[i];
        if (a.g_out) {
            uint8_t *go = a.g_out + (size_t)surf * LG;
            for (int i = tid; i < LG; i += blockDim.x) go[i] = g[i];
        }
    }
}

__global__ __launch_bounds__(256) void k_stage1(Stage1Args a)
{
    extern __shared__ __align__(16) uint8_t lds[];
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

size_t dyn_lds_stage1(int max_p)
{
    const int64_t lg = len_g_of(max_p);
    return 64 + 2 * (size_t)((lg + 15) / 16 * 16);
}

hipError_t launch_stage1(const Stage1Args &a, int max_p, hipStream_t s)
{
    if (a.batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage1, dim3(a.batch), dim3(256), dyn_lds_stage1(max_p), s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// plan: output tile lists
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_plan(uint32_t *plan)
{
    constexpr int d = 4 * (P - 1);
    const int k = blockIdx.x;
    const int n = (k + 1) * d;
    uint32_t *out = plan + kPT<P>.off[k];
    __shared__ int cnt[256];
    const int c1 = threadIdx.x;
    int mine = 0;
    if (T1 * c1 <= n)
        for (int c2 = 0; T1 * c1 + T2 * c2 <= n; ++c2) mine += (n - T1 * c1 - T2 * c2) / T3 + 1;
    cnt[c1] = mine;
    __syncthreads();
    if (T1 * c1 <= n) {
        int off = 0;
        for (int i = 0; i < c1; ++i) off += cnt[i];
        for (int c2 = 0; T1 * c1 + T2 * c2 <= n; ++c2)
            for (int c3 = 0; T1 * c1 + T2 * c2 + T3 * c3 <= n; ++c3) out[off++] = pack3(c1, c2, c3);
    }
}

hipError_t launch_plan(int p, uint32_t *plan, hipStream_t s)
{
    switch (p) {
    case 3: hipLaunchKernelGGL(k_plan<3>, dim3(3), dim3(256), 0, s, plan); break;
    case 5: hipLaunchKernelGGL(k_plan<5>, dim3(5), dim3(256), 0, s, plan); break;
    case 7: hipLaunchKernelGGL(k_plan<7>, dim3(7), dim3(256), 0, s, plan); break;
    case 11: hipLaunchKernelGGL(k_plan<11>, dim3(11), dim3(256), 0, s, plan); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deep kernel
// ---------------------------------------------------------------------------
constexpr int DEEP_NT = 512, DEEP_NW = DEEP_NT / 64, DEEP_NB = 4;

template <int P>
struct DeepLds {
    static constexpr int LG = Prime<P>::len_g;
    static constexpr int LGA = (LG + 15) / 16 * 16;
    static constexpr int APA = (ThetaGeo<P>::APERM + 15) / 16 * 16;
    static constexpr int off_g = 0;
    static constexpr int off_aperm = off_g + LGA;
    static constexpr int off_toff = off_aperm + APA;
    static constexpr int off_red = off_toff + 4 * Geo<P>::NVP;
    static constexpr int bytes = off_red + 4 * 32;
};

template <int P>
__device__ inline int64_t box_tile(int c1, int c2, int c3)
{
    using G = Geo<P>;
    return ((int64_t)(c1 + G::H1) * G::B2 + (c2 + G::H2)) * G::B3 + (c3 + G::H3);
}

// Fill W[delta][s][s'] = g~[T*delta + s - s'] (dehomogenised, zero outside the simplex of degree d).
template <int P>
__device__ void build_w(const uint8_t *g, uint8_t *W)
{
    using G = Geo<P>;
    constexpr int d = G::d;
    for (int row = threadIdx.x; row < G::NVP * 16; row += blockDim.x) {
        const int q = row >> 4, s = row & 15;
        const int s1 = s >> 3, s2 = (s >> 2) & 1, s3 = s & 3;
        unsigned w[4] = {0, 0, 0, 0};
        if (q < G::NV) {
            const uint32_t dl = kDT<P>.packed[q];
            const int b1 = T1 * unp0(dl) + s1, b2 = T2 * unp1(dl) + s2, b3 = T3 * unp2(dl) + s3;
            for (int sp = 0; sp < 16; ++sp) {
                const int x1 = b1 - (sp >> 3), x2 = b2 - ((sp >> 2) & 1), x3 = b3 - (sp & 3);
                const int x4 = d - x1 - x2 - x3;
                unsigned v = 0;
                if (x1 >= 0 && x2 >= 0 && x3 >= 0 && x4 >= 0) v = g[cns_rank(x2, x3, x4)];
                w[sp >> 2] |= v << (8 * (sp & 3));
            }
        }
        *(v4u *)(W + (size_t)row * 16) = v4u{w[0], w[1], w[2], w[3]};
    }
}

// A_1 = g~ on the tiles with w(c) <= 2d (zero beyond degree d).
template <int P>
__device__ void init_a1(const uint8_t *g, const uint32_t *list, int ntiles, uint8_t *A)
{
    constexpr int d = 4 * (P - 1);
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
        const uint32_t t = list[i];
        const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t);
        unsigned w[4] = {0, 0, 0, 0};
        if (T1 * c1 + T2 * c2 + T3 * c3 <= d) {
            for (int s = 0; s < 16; ++s) {
                const int x1 = T1 * c1 + (s >> 3), x2 = T2 * c2 + ((s >> 2) & 1), x3 = T3 * c3 + (s & 3);
                const int x4 = d - x1 - x2 - x3;
                if (x4 >= 0) w[s >> 2] |= (unsigned)g[cns_rank(x2, x3, x4)] << (8 * (s & 3));
            }
        }
        *(v4u *)(A + box_tile<P>(c1, c2, c3) * 16) = v4u{w[0], w[1], w[2], w[3]};
    }
}

// Zero the tiles of `list` with w(c) > n (the shell the next product reads beyond degree n).
template <int P>
__device__ void zero_shell(const uint32_t *list, int ntiles, int n, uint8_t *A)
{
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
        const uint32_t t = list[i];
        const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t);
        if (T1 * c1 + T2 * c2 + T3 * c3 > n) *(v4u *)(A + box_tile<P>(c1, c2, c3) * 16) = v4u{0, 0, 0, 0};
    }
}

template <int P>
__device__ inline int ntiles_of_list(int k)
{
    return (int)kPT<P>.len[k];
}

struct EpiCtx {
    int mode;
    uint8_t *dl;      // MODE_HEIGHT: Delta in the Cartier-split layout
    uint8_t *dout;    // MODE_DELTA: Delta in CNS order for this surface
    const uint8_t *g; // LDS
    int *err;         // LDS flag
};

// One wave computes NB groups of 16 output tiles of A_{k+1} = A_k * g~:
// for each quad of 4 offsets, D[s][tile] += W_quad[s][(delta,s')] * A_tile[(delta,s')].
template <int P>
__device__ void mfma_set(const uint32_t *list, int ntiles, int gs, int nk, const uint8_t *__restrict__ W,
                         const uint8_t *__restrict__ Ain, uint8_t *Aout, bool last, const int *toff_l,
                         const EpiCtx &ec)
{
    using G = Geo<P>;
    constexpr int NB = DEEP_NB;
    constexpr int P2 = P * P;
    constexpr int D = G::D;
    const int lane = threadIdx.x & 63, kg = lane >> 4, col = lane & 15;

    int64_t base[NB];
    bool ok[NB], gex[NB];
    int gmax1[NB], gmax2[NB], gmax3[NB], gwmin[NB];
    uint32_t tpk[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int g0 = (gs * NB + b) * 16;
        gex[b] = g0 < ntiles;
        const int idx = g0 + col;
        ok[b] = idx < ntiles;
        const uint32_t t = gex[b] ? list[ok[b] ? idx : g0] : 0u;
        tpk[b] = t;
        const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t);
        base[b] = box_tile<P>(c1, c2, c3);
        gmax1[b] = uniform(wave_max(c1));
        gmax2[b] = uniform(wave_max(c2));
        gmax3[b] = uniform(wave_max(c3));
        gwmin[b] = uniform(wave_min(T1 * c1 + T2 * c2 + T3 * c3));
    }
    v4i acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = v4i{0, 0, 0, 0};

    for (int q = 0; q < G::NQ; ++q) {
        const uint32_t qmin = kDT<P>.qmin[q];
        const int qw = kDT<P>.qwmax[q];
        const int qm1 = unp0(qmin), qm2 = unp1(qmin), qm3 = unp2(qmin);
        bool need[NB];
        bool any = false;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            need[b] = gex[b] && gmax1[b] >= qm1 && gmax2[b] >= qm2 && gmax3[b] >= qm3 && gwmin[b] - qw <= nk;
            any |= need[b];
        }
        if (!any) continue;
        const v4i wf = *(const v4i *)(W + (size_t)q * 1024 + lane * 16);
        const int to = toff_l[4 * q + kg];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!need[b]) continue;
            const v4i bf = *(const v4i *)(Ain + (base[b] - to) * 16);
            acc[b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wf, bf, acc[b], 0, 0, 0);
        }
    }

#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (!gex[b] || !ok[b]) continue;
        if (!last) {
            unsigned packed = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) packed |= (unsigned)(acc[b][v] % P2) << (8 * v);
            *(unsigned *)(Aout + base[b] * 16 + 4 * kg) = packed;
            continue;
        }
        // Delta_1 epilogue: D = (g~^p - sum_J b_J^p x^(pJ)) / p mod p
        const int c1 = unp0(tpk[b]), c2 = unp1(tpk[b]), c3 = unp2(tpk[b]);
        const int x1 = T1 * c1 + (kg >> 1), x2 = T2 * c2 + (kg & 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int x3 = T3 * c3 + v;
            const int x4 = D - x1 - x2 - x3;
            if (x4 < 0) continue;
            int val = acc[b][v] % P2;
            if (x1 % P == 0 && x2 % P == 0 && x3 % P == 0) {
                const int bj = ec.g[cns_rank(x2 / P, x3 / P, x4 / P)];
                val -= pow_p_mod_p2<P>(bj);
                if (val < 0) val += P2;
            }
            if (val % P) *ec.err = 1;
            const uint8_t dv = (uint8_t)(val / P);
            if (ec.mode == MODE_HEIGHT)
                ec.dl[theta_addr<P>(x1, x2, x3, x4)] = dv;
            else
                ec.dout[cns_rank(x2, x3, x4)] = dv;
        }
    }
}

template <int P>
__global__ __launch_bounds__(DEEP_NT, 1) void k_deep(DeepArgs a)
{
    using PR = Prime<P>;
    using G = Geo<P>;
    using L = DeepLds<P>;
    constexpr int LG = PR::len_g;
    constexpr int d = PR::d;
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *g_l = lds + L::off_g;
    uint8_t *aperm = lds + L::off_aperm;
    int *toff_l = (int *)(lds + L::off_toff);
    int *red = (int *)(lds + L::off_red);
    __shared__ int s_pos, s_err;

    const int tid = threadIdx.x, wave = tid >> 6;
    const int pi = prime_index(P);
    uint8_t *slot = a.slots + (size_t)blockIdx.x * a.slot_bytes;
    uint8_t *W = slot;
    uint8_t *buf[2] = {slot + align256(G::W_BYTES), slot + align256(G::W_BYTES) + align256(G::BOX_BYTES)};
    uint8_t *dl = slot + align256(G::W_BYTES) + 2 * align256(G::BOX_BYTES);

    for (int i = tid; i < G::NVP; i += DEEP_NT) toff_l[i] = kDT<P>.toff[i];
    // the halo (tiles with a negative coordinate) of both boxes is read as zero and never written
    for (int64_t t = tid; t < G::BOX_TILES; t += DEEP_NT) {
        const int i3 = (int)(t % G::B3);
        const int64_t r = t / G::B3;
        const int i2 = (int)(r % G::B2), i1 = (int)(r / G::B2);
        if (i1 < G::H1 || i2 < G::H2 || i3 < G::H3) {
            *(v4u *)(buf[0] + t * 16) = v4u{0, 0, 0, 0};
            *(v4u *)(buf[1] + t * 16) = v4u{0, 0, 0, 0};
        }
    }
    const int count = a.counters[CNT_COUNT + pi];

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            s_pos = atomicAdd(&a.counters[CNT_POP + pi], 1);
            s_err = 0;
        }
        __syncthreads();
        const int pos = s_pos;
        if (pos >= count) break;
        const int surf = a.queue[pos];
        for (int i = tid; i < LG; i += DEEP_NT) g_l[i] = a.gq[(size_t)pos * LG + i];
        __syncthreads();
        build_w<P>(g_l, W);
        init_a1<P>(g_l, a.plan + kPT<P>.off[1], ntiles_of_list<P>(1), buf[0]);
        __syncthreads();

        EpiCtx ec;
        ec.mode = a.mode;
        ec.dl = dl;
        ec.dout = a.delta_out ? a.delta_out + (size_t)surf * PR::len_D : nullptr;
        ec.g = g_l;
        ec.err = &s_err;
        for (int k = 1; k < P; ++k) {
            const uint8_t *Ain = buf[(k - 1) & 1];
            uint8_t *Aout = buf[k & 1];
            const int ntiles = ntiles_of_list<P>(k);
            const int nsets = ((ntiles + 15) / 16 + DEEP_NB - 1) / DEEP_NB;
            const bool last = (k == P - 1);
            const uint32_t *list = a.plan + kPT<P>.off[k];
            for (int gs = wave; gs < nsets; gs += DEEP_NW)
                mfma_set<P>(list, ntiles, gs, k * d, W, Ain, Aout, last, toff_l, ec);
            if (!last) zero_shell<P>(a.plan + kPT<P>.off[k + 1], ntiles_of_list<P>(k + 1), (k + 1) * d, Aout);
            __syncthreads();
        }
        const bool err = s_err != 0;

        if (a.mode == MODE_DELTA) {
            if (tid == 0 && err && a.status) a.status[surf] = -5; /* QFS_EARITH */
            continue;
        }
        if (err) {
            if (tid == 0) a.heights[surf] = -5;
            continue;
        }
        // Algorithm 3's loop: the test reads c(theta(a)) only; theta(a) in full
        // is needed only when the surface goes on to the next h.
        int h = 0;
        for (int hh = 2; hh <= a.bound; ++hh) {
            build_aperm<P>(g_l, aperm);
            __syncthreads();
            const int t = theta_test<P>(dl, aperm, red);
            if (t != 0) {
                h = hh;
                break;
            }
            if (hh == a.bound) break;
            theta_full<P>(dl, aperm, g_l);
            __syncthreads();
        }
        if (tid == 0) a.heights[surf] = h;
    }
}

template <int P>
static hipError_t launch_deep_p(const DeepArgs &a, int nslots, hipStream_t s)
{
    const size_t lds = DeepLds<P>::bytes;
    hipLaunchKernelGGL(k_deep<P>, dim3(nslots), dim3(DEEP_NT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_deep(int p, const DeepArgs &a, int nslots, hipStream_t s)
{
    switch (p) {
    case 3: return launch_deep_p<3>(a, nslots, s);
    case 5: return launch_deep_p<5>(a, nslots, s);
    case 7: return launch_deep_p<7>(a, nslots, s);
    case 11: return launch_deep_p<11>(a, nslots, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// MFMA instructions per surface (host): the deep kernel's skip test depends
// only on the geometry, so this replays it.
// ---------------------------------------------------------------------------
template <int P>
static int64_t mfma_count_p()
{
    using G = Geo<P>;
    constexpr int d = G::d;
    static const DeltaTable<P> DT = make_delta_table<P>();
    int64_t total = 0;
    for (int k = 1; k < P; ++k) {
        const int n = (k + 1) * d, nk = k * d;
        std::vector<uint32_t> tiles;
        for (int c1 = 0; T1 * c1 <= n; ++c1)
            for (int c2 = 0; T1 * c1 + T2 * c2 <= n; ++c2)
                for (int c3 = 0; T1 * c1 + T2 * c2 + T3 * c3 <= n; ++c3) tiles.push_back(pack3(c1, c2, c3));
        const int nt = (int)tiles.size();
        for (int g0 = 0; g0 < nt; g0 += 16) {
            int m1 = 0, m2 = 0, m3 = 0, wmin = 1 << 30;
            for (int j = 0; j < 16 && g0 + j < nt; ++j) {
                const uint32_t t = tiles[g0 + j];
                m1 = std::max(m1, unp0(t));
                m2 = std::max(m2, unp1(t));
                m3 = std::max(m3, unp2(t));
                wmin = std::min(wmin, T1 * unp0(t) + T2 * unp1(t) + T3 * unp2(t));
            }
            for (int q = 0; q < G::NQ; ++q) {
                const uint32_t qm = DT.qmin[q];
                if (m1 >= unp0(qm) && m2 >= unp1(qm) && m3 >= unp2(qm) && wmin - DT.qwmax[q] <= nk) ++total;
            }
        }
    }
    return total;
}

int64_t mfma_count(int p)
{
    static int64_t cache[4] = {-1, -1, -1, -1};
    const int pi = prime_index(p);
    if (pi < 0) return -1;
    if (cache[pi] < 0) {
        switch (p) {
        case 3: cache[pi] = mfma_count_p<3>(); break;
        case 5: cache[pi] = mfma_count_p<5>(); break;
        case 7: cache[pi] = mfma_count_p<7>(); break;
        case 11: cache[pi] = mfma_count_p<11>(); break;
        }
    }
    return cache[pi];
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

BatchLayout make_batch_layout(const bool present[4], int batch, int n_cu)
{
    BatchLayout L;
    size_t off = align256(CNT_WORDS * sizeof(int32_t));
    for (int i = 0; i < 4; ++i) {
        L.present[i] = present[i];
        if (!present[i]) continue;
        const int p = kPrimes[i];
        L.queue[i] = off;
        off += align256((size_t)batch * sizeof(int32_t));
        L.gq[i] = off;
        off += align256((size_t)batch * (size_t)len_g_of(p));
        L.plan[i] = off;
        off += align256(plan_bytes_of(p));
        // one persistent workgroup per compute unit; p = 11 boxes are large, so fewer
        int ns = p == 11 ? (n_cu < 64 ? n_cu : 64) : n_cu;
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
