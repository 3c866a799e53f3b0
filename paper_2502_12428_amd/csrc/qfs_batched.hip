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
#include <cstdlib>
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
// plan: output tile lists (base tiles of the super-tiles, and shell lists)
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_plan(uint32_t *plan)
{
    using X = GeoX<P>;
    constexpr int d = 4 * (P - 1);
    const bool is_base = blockIdx.x < P;
    const int k = is_base ? blockIdx.x : blockIdx.x - P;
    if (is_base ? (k < 1) : (k > P - 2)) return;
    const int m = is_base ? (k + 1) * d : (k + 2) * d + 4;
    uint32_t *out = plan + (is_base ? kPT<P>.boff[k] : kPT<P>.foff[k]);
    __shared__ int cnt[256];
    const int c1 = threadIdx.x;
    const int step = is_base ? 2 : 1;
    const bool mine_slab = (c1 % step == 0) && T1 * c1 <= m && (is_base || c1 <= X::C1);
    int mine = 0;
    if (mine_slab)
        for (int c2 = 0; T1 * c1 + T2 * c2 <= m && (is_base || c2 <= X::C2); c2 += step) {
            int top = (m - T1 * c1 - T2 * c2) / T3;
            if (!is_base && top > X::C3 - 1) top = X::C3 - 1;
            mine += top + 1;
        }
    cnt[c1] = mine;
    __syncthreads();
    if (mine_slab) {
        int off = 0;
        for (int i = 0; i < c1; ++i) off += cnt[i];
        for (int c2 = 0; T1 * c1 + T2 * c2 <= m && (is_base || c2 <= X::C2); c2 += step) {
            int top = (m - T1 * c1 - T2 * c2) / T3;
            if (!is_base && top > X::C3 - 1) top = X::C3 - 1;
            for (int c3 = 0; c3 <= top; ++c3) out[off++] = pack3(c1, c2, c3);
        }
    }
}

hipError_t launch_plan(int p, uint32_t *plan, hipStream_t s)
{
    switch (p) {
    case 3: hipLaunchKernelGGL(k_plan<3>, dim3(6), dim3(256), 0, s, plan); break;
    case 5: hipLaunchKernelGGL(k_plan<5>, dim3(10), dim3(256), 0, s, plan); break;
    case 7: hipLaunchKernelGGL(k_plan<7>, dim3(14), dim3(256), 0, s, plan); break;
    case 11: hipLaunchKernelGGL(k_plan<11>, dim3(22), dim3(256), 0, s, plan); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deep kernel
// ---------------------------------------------------------------------------
constexpr int DEEP_NT = 512, DEEP_NW = DEEP_NT / 64, DEEP_NB = 4;

template <int P>
__constant__ DeltaTableX<P> kDX = make_delta_table_x<P>();

template <int P>
struct DeepLds {
    using X = GeoX<P>;
    static constexpr int LG = Prime<P>::len_g;
    static constexpr int LGA = (LG + 15) / 16 * 16;
    static constexpr int APA = (ThetaGeo<P>::APERM + 15) / 16 * 16;
    static constexpr int WB = w_in_lds<P>() ? (int)((X::W_BYTES + 15) / 16 * 16) : 0;
    static constexpr int off_w = 0;
    static constexpr int off_g = off_w + WB;
    static constexpr int off_aperm = off_g + LGA;
    static constexpr int off_toff = off_aperm + APA;
    static constexpr int off_widx = off_toff + 4 * (X::NVXP + 4);
    static constexpr int off_qbox = off_widx + 8 * (X::NVXP + 4);
    static constexpr int off_qlist = off_qbox + 8 * X::NQX;
    static constexpr int off_red = off_qlist + ((2 * (X::NQX + 1) * (DEEP_NT / 64) + 15) / 16 * 16);
    static constexpr int bytes = off_red + 4 * 64;
};

template <int P>
__device__ inline int64_t box_tile(int c1, int c2, int c3)
{
    using X = GeoX<P>;
    return ((int64_t)(c1 + X::H1) * X::B2 + (c2 + X::H2)) * X::B3 + (c3 + X::H3);
}

// W[v][s][s'] = g~[T*v + s - s'] for v in V (dehomogenised, zero outside the
// simplex of degree d); block NV is all zero.
template <int P>
__device__ void build_w(const uint8_t *g, uint8_t *W)
{
    using X = GeoX<P>;
    constexpr int d = X::d;
    for (int row = threadIdx.x; row < (X::NV + 1) * 16; row += blockDim.x) {
        const int v = row >> 4, s = row & 15;
        const int s1 = s >> 3, s2 = (s >> 2) & 1, s3 = s & 3;
        unsigned w[4] = {0, 0, 0, 0};
        if (v < X::NV) {
            const uint32_t dl = kDX<P>.vpacked[v];
            const int b1 = T1 * unp0(dl) + s1, b2 = T2 * unp1(dl) + s2, b3 = T3 * unp2(dl) + s3;
            for (int sp = 0; sp < 16; ++sp) {
                const int x1 = b1 - (sp >> 3), x2 = b2 - ((sp >> 2) & 1), x3 = b3 - (sp & 3);
                const int x4 = d - x1 - x2 - x3;
                unsigned val = 0;
                if (x1 >= 0 && x2 >= 0 && x3 >= 0 && x4 >= 0) val = g[cns_rank(x2, x3, x4)];
                w[sp >> 2] |= val << (8 * (sp & 3));
            }
        }
        *(v4u *)(W + (size_t)row * 16) = v4u{w[0], w[1], w[2], w[3]};
    }
}

// A_1 = g~ on the shell list 0 (every tile with w(c) <= 2d + 4; zero beyond degree d).
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
        gstore16(A + box_tile<P>(c1, c2, c3) * 16, v4u{w[0], w[1], w[2], w[3]});
    }
}

// Zero the tiles of a shell list with w(c) > n: the next product reads them as zeros.
template <int P>
__device__ void zero_shell(const uint32_t *list, int ntiles, int n, uint8_t *A)
{
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
        const uint32_t t = list[i];
        const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t);
        if (T1 * c1 + T2 * c2 + T3 * c3 > n) gstore16(A + box_tile<P>(c1, c2, c3) * 16, v4u{0, 0, 0, 0});
    }
}

struct EpiCtx {
    int mode;
    uint8_t *dout;    // MODE_DELTA: Delta in CNS order for this surface
    const uint8_t *g; // LDS
    int *err;         // LDS flag
};

// Delta_1 epilogue for the four positions s = 4 kg + v of output tile c:
// D = (g~^p - sum_J b_J^p x^(pJ)) / p mod p (Algorithm 1, lines 3-5).
// Returns the four values packed in a word (byte v for position 4 kg + v;
// positions beyond degree D give 0).  MODE_DELTA also scatters them to the
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
        int val = acc[v] % P2;
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

// One wave computes NB groups of 16 base tiles and their four shifts, i.e.
// 4 * NB output groups of A_{k+1} = A_k * g~.  Per quad of offsets delta it
// loads one input fragment per group (the 16 tiles q - delta) and one W
// fragment per shift (blocks W_{delta + Delta_s}), then issues up to
// 4 * NB products D[s][tile] += W[s][(delta, s')] * A[(delta, s')][tile].
template <int P>
__device__ __attribute__((always_inline)) inline void mfma_set(const uint32_t *list, int nbase, int gs, int nk, const uint8_t *W,
                         const uint8_t *__restrict__ Ain, uint8_t *Aout, bool last, const int *toff_l,
                         const uint32_t *widx_l, const uint32_t *qbox_l, uint16_t *qlist, const EpiCtx &ec)
{
    using X = GeoX<P>;
    constexpr int NB = DEEP_NB;
    constexpr int P2 = P * P;
    const int lane = threadIdx.x & 63, kg = lane >> 4, col = lane & 15;

    int64_t base[NB];
    bool ok[NB], gex[NB];
    int gmax1[NB], gmax2[NB], gmax3[NB], gwmin[NB];
    uint32_t tpk[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int g0 = (gs * NB + b) * 16;
        gex[b] = g0 < nbase;
        const int idx = g0 + col;
        ok[b] = idx < nbase;
        const uint32_t t = gex[b] ? list[ok[b] ? idx : g0] : 0u;
        tpk[b] = t;
        const int c1 = unp0(t), c2 = unp1(t), c3 = unp2(t);
        base[b] = box_tile<P>(c1, c2, c3);
        gmax1[b] = uniform(wave_max(c1));
        gmax2[b] = uniform(wave_max(c2));
        gmax3[b] = uniform(wave_max(c3));
        gwmin[b] = uniform(wave_min(T1 * c1 + T2 * c2 + T3 * c3));
    }
    v4i acc[4][NB];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[s][b] = v4i{0, 0, 0, 0};

    // Bounding box of the set's tiles.  A quad whose input tiles q - delta all lie
    // outside A_k (a negative coordinate, or weight above deg A_k) contributes
    // nothing and is skipped.  For the quads that are processed, every group and
    // every shift is multiplied: tiles outside A_k read the zero halo or the
    // zeroed shell and the zero W block adds nothing, so the products stay exact
    // and the loop has no branches around the matrix instructions.
    int smax1 = 0, smax2 = 0, smax3 = 0, swmin = 1 << 30;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if (gex[b]) {
            smax1 = max(smax1, gmax1[b]);
            smax2 = max(smax2, gmax2[b]);
            smax3 = max(smax3, gmax3[b]);
            swmin = min(swmin, gwmin[b]);
        }
    // the quads this set needs, in order, into the wave's list in LDS
    int nq = 0;
    for (int q0 = 0; q0 < X::NQX; q0 += 64) {
        const int q = q0 + lane;
        bool nd = false;
        if (q < X::NQX) {
            const uint32_t qmin = qbox_l[2 * q];
            nd = smax1 >= (int)unp0(qmin) - 1 && smax2 >= (int)unp1(qmin) - 1 && smax3 >= (int)unp2(qmin) &&
                 swmin - (int)qbox_l[2 * q + 1] <= nk;
        }
        const uint64_t m = __ballot(nd);
        if (nd) qlist[nq + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)q;
        nq += __popcll(m);
    }
    nq = uniform(nq);
    // pad to an even count with the null quad (index NQX: offset 0, zero W blocks)
    if (nq & 1) {
        if (lane == 0) qlist[nq] = (uint16_t)X::NQX;
        ++nq;
    }

    // byte offsets of the tiles inside the box fit in 32 bits
    uint32_t boff[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) boff[b] = (uint32_t)base[b] * 16u;
    const uint32_t wrow = (uint32_t)col * 16u;
    // input fragments of the list entry i (clamped to the last entry)
#define QFS_LOAD_B(BF, I)                                                                          \
    do {                                                                                           \
        const int q_ = uniform(qlist[(I) < nq ? (I) : nq - 1]);                                    \
        const uint32_t to_ = (uint32_t)toff_l[4 * q_ + kg] * 16u;                                  \
        _Pragma("unroll") for (int b = 0; b < NB; ++b) BF[b] = gload16(Ain + (boff[b] - to_));     \
    } while (0)
    // W fragments of list entry i for the four shifts, then the 4 x NB products
#define QFS_PRODUCTS(BF, I)                                                                                \
    do {                                                                                                   \
        const int q_ = uniform(qlist[I]);                                                                  \
        const uint32_t w01_ = widx_l[2 * (4 * q_ + kg)], w23_ = widx_l[2 * (4 * q_ + kg) + 1];              \
        v4i wf_[4];                                                                                        \
        _Pragma("unroll") for (int s = 0; s < 4; ++s)                                                      \
        {                                                                                                  \
            const uint32_t wi = ((s < 2 ? w01_ : w23_) >> (16 * (s & 1))) & 0xFFFFu;                        \
            wf_[s] = w_in_lds<P>() ? *(const v4i *)(W + wi * 256u + wrow) : gload16(W + wi * 256u + wrow);  \
        }                                                                                                  \
        _Pragma("unroll") for (int s = 0; s < 4; ++s)                                                      \
            _Pragma("unroll") for (int b = 0; b < NB; ++b)                                                 \
                acc[s][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(wf_[s], BF[b], acc[s][b], 0, 0, 0);       \
    } while (0)

    // two fragment sets alternate; each is refilled two entries ahead of its use
    if (nq > 0) {
        v4i bfa[NB], bfb[NB];
        QFS_LOAD_B(bfa, 0);
        __builtin_amdgcn_sched_barrier(0);
        QFS_LOAD_B(bfb, 1);
        __builtin_amdgcn_sched_barrier(0);
        for (int i = 0; i < nq; i += 2) {
            QFS_PRODUCTS(bfa, i);
            __builtin_amdgcn_sched_barrier(0);
            QFS_LOAD_B(bfa, i + 2);
            __builtin_amdgcn_sched_barrier(0);
            QFS_PRODUCTS(bfb, i + 1);
            __builtin_amdgcn_sched_barrier(0);
            QFS_LOAD_B(bfb, i + 3);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#undef QFS_LOAD_B
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
                for (int v = 0; v < 4; ++v) packed |= (unsigned)(acc[s][b][v] % P2) << (8 * v);
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

// Copy Delta from its tile box into the Cartier-split layout used by theta_full.
template <int P>
__device__ void box_to_theta(const uint8_t *dbox, const uint32_t *list, int nbase, uint8_t *dl)
{
    constexpr int D = 4 * P * (P - 1);
    for (int i = threadIdx.x; i < nbase * 4; i += blockDim.x) {
        const uint32_t t = list[i >> 2];
        const int s = i & 3;
        const int c1 = unp0(t) + (s & 1), c2 = unp1(t) + (s >> 1), c3 = unp2(t);
        const v4u tile = gload16u(dbox + box_tile<P>(c1, c2, c3) * 16);
#pragma unroll
        for (int pos = 0; pos < 16; ++pos) {
            const int x1 = T1 * c1 + (pos >> 3), x2 = T2 * c2 + ((pos >> 2) & 1), x3 = T3 * c3 + (pos & 3);
            const int x4 = D - x1 - x2 - x3;
            if (x4 < 0) continue;
            const unsigned word = pos < 4 ? tile.x : pos < 8 ? tile.y : pos < 12 ? tile.z : tile.w;
            gstore1(dl + theta_addr<P>(x1, x2, x3, x4), (uint8_t)((word >> (8 * (pos & 3))) & 255u));
        }
    }
}

template <int P>
__global__ __launch_bounds__(DEEP_NT, 1) void k_deep(DeepArgs a)
{
    using PR = Prime<P>;
    using X = GeoX<P>;
    using L = DeepLds<P>;
    constexpr int LG = PR::len_g;
    constexpr int d = PR::d;
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *g_l = lds + L::off_g;
    uint8_t *aperm = lds + L::off_aperm;
    int *toff_l = (int *)(lds + L::off_toff);
    uint32_t *widx_l = (uint32_t *)(lds + L::off_widx);
    uint32_t *qbox_l = (uint32_t *)(lds + L::off_qbox);
    uint16_t *qlist_l = (uint16_t *)(lds + L::off_qlist);
    int *red = (int *)(lds + L::off_red);
    __shared__ int s_pos, s_err;

    const int tid = threadIdx.x, wave = uniform(tid >> 6);
    const int pi = prime_index(P);
    uint8_t *slot = a.slots + (size_t)blockIdx.x * a.slot_bytes;
    uint8_t *wg = slot;
    uint8_t *bufs = slot + (w_in_lds<P>() ? 0 : align256(X::W_BYTES));
    uint8_t *buf[2] = {bufs, bufs + align256(X::BOX_BYTES)};
    uint8_t *dl = bufs + 2 * align256(X::BOX_BYTES);
    uint8_t *W = w_in_lds<P>() ? lds + L::off_w : wg;

    const int count = a.counters[CNT_COUNT + pi];
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
    for (int i = tid; i < X::NQX; i += DEEP_NT) {
        qbox_l[2 * i] = kDX<P>.qmin[i];
        qbox_l[2 * i + 1] = (uint32_t)kDX<P>.qwmax[i];
    }
    // the halo (tiles with a negative coordinate) of both boxes is read as zero and never written
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
        init_a1<P>(g_l, a.plan + kPT<P>.foff[0], (int)kPT<P>.flen[0], buf[0]);
        __syncthreads();

        EpiCtx ec;
        ec.mode = a.mode;
        ec.dout = a.delta_out ? a.delta_out + (size_t)surf * PR::len_D : nullptr;
        ec.g = g_l;
        ec.err = &s_err;
        for (int k = 1; k < P; ++k) {
            const uint8_t *Ain = buf[(k - 1) & 1];
            uint8_t *Aout = buf[k & 1];
            const int nbase = (int)kPT<P>.blen[k];
            const int nsets = ((nbase + 15) / 16 + DEEP_NB - 1) / DEEP_NB;
            const bool last = (k == P - 1);
            const uint32_t *list = a.plan + kPT<P>.boff[k];
            for (int gs = wave; gs < nsets; gs += DEEP_NW)
                mfma_set<P>(list, nbase, gs, k * d, W, Ain, Aout, last, toff_l, widx_l, qbox_l, qlist_l + wave * (X::NQX + 1), ec);
            if (!last) zero_shell<P>(a.plan + kPT<P>.foff[k], (int)kPT<P>.flen[k], (k + 1) * d, Aout);
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
        const uint8_t *dbox = buf[(P - 1) & 1];
        int h = 0;
        bool split = false;
        for (int hh = 2; hh <= a.bound; ++hh) {
            const int t = theta_test_box<P>(dbox, g_l, red);
            if (t != 0) {
                h = hh;
                break;
            }
            if (hh == a.bound) break;
            if (!split) {
                box_to_theta<P>(dbox, a.plan + kPT<P>.boff[P - 1], (int)kPT<P>.blen[P - 1], dl);
                split = true;
            }
            build_aperm<P>(g_l, aperm);
            __syncthreads();
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
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)k_deep<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
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
// MFMA instructions per surface (host): the deep kernel's skip tests depend
// only on the geometry, so this replays them.
// ---------------------------------------------------------------------------
template <int P>
static int64_t mfma_count_p()
{
    using X = GeoX<P>;
    constexpr int d = X::d;
    static const DeltaTableX<P> DX = make_delta_table_x<P>();
    int64_t total = 0;
    for (int k = 1; k < P; ++k) {
        const int n = (k + 1) * d, nk = k * d;
        std::vector<uint32_t> tiles;
        for (int c1 = 0; T1 * c1 <= n; c1 += 2)
            for (int c2 = 0; T1 * c1 + T2 * c2 <= n; c2 += 2)
                for (int c3 = 0; T1 * c1 + T2 * c2 + T3 * c3 <= n; ++c3) tiles.push_back(pack3(c1, c2, c3));
        const int nt = (int)tiles.size();
        const int ngroups = (nt + 15) / 16;
        for (int gs = 0; gs * DEEP_NB < ngroups; ++gs) {
            int m1 = 0, m2 = 0, m3 = 0, wmin = 1 << 30;
            for (int g = gs * DEEP_NB * 16; g < std::min(nt, (gs + 1) * DEEP_NB * 16); ++g) {
                const uint32_t t = tiles[g];
                m1 = std::max(m1, unp0(t));
                m2 = std::max(m2, unp1(t));
                m3 = std::max(m3, unp2(t));
                wmin = std::min(wmin, T1 * unp0(t) + T2 * unp1(t) + T3 * unp2(t));
            }
            for (int q = 0; q < X::NQX; ++q) {
                const uint32_t qm = DX.qmin[q];
                if (m1 >= (int)unp0(qm) - 1 && m2 >= (int)unp1(qm) - 1 && m3 >= (int)unp2(qm) &&
                    wmin - DX.qwmax[q] <= nk)
                    total += 4 * DEEP_NB;
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

// Persistent workgroups per compute unit for p <= 7 (QFS_DEEP_WGS_PER_CU, 1..8; default 1).
static int deep_wgs_per_cu()
{
    const char *e = getenv("QFS_DEEP_WGS_PER_CU");
    int v = e ? atoi(e) : 1;
    return v < 1 ? 1 : v > 8 ? 8 : v;
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
        int ns = p == 11 ? (n_cu < 64 ? n_cu : 64) : n_cu * deep_wgs_per_cu();
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
