// Internal host/device interface of libqfs: workspace layouts and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "qfs_common.h"

namespace qfs {

constexpr int kPrimes[4] = {3, 5, 7, 11};
__host__ __device__ constexpr int prime_index(int p)
{
    return p == 3 ? 0 : p == 5 ? 1 : p == 7 ? 2 : p == 11 ? 3 : -1;
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// counters at the head of the batched workspace (int32 each)
// per-prime counters (index + prime_index): deep surfaces queued, popped, errors,
// surfaces left for the full chain (second queue), popped from it
enum { CNT_COUNT = 0, CNT_POP = 4, CNT_ERR = 8, CNT_Q2 = 12, CNT_POP2 = 16, CNT_WORDS = 64 };

enum { MODE_HEIGHT = 0, MODE_DELTA = 1 };

// Order of a base list.  In base units u = (c1/2, c2/2, c3) the base tiles of
// degree m form the simplex u1 + u2 + u3 <= m/4 (T = (2,2,4)).  The list runs
// through blocks of PB1 x PB2 x PB3 base units in lexicographic order, and
// through each block lexicographically, so that the 64 tiles one wave
// multiplies and the few hundred a workgroup has in flight are compact in all
// three coordinates: their input windows overlap and stay in L2.
#ifndef QFS_PLAN_B1
#define QFS_PLAN_B1 1
#endif
#ifndef QFS_PLAN_B2
#define QFS_PLAN_B2 1
#endif
#ifndef QFS_PLAN_B3
#define QFS_PLAN_B3 1
#endif
constexpr int PB1 = QFS_PLAN_B1, PB2 = QFS_PLAN_B2, PB3 = QFS_PLAN_B3;
static_assert(T1 == 2 && T2 == 2 && T3 == 4, "base-list order assumes 2x2x4 tiles");

struct PlanBlocks {
    int n1, n2, n3;
};
__host__ __device__ inline PlanBlocks plan_blocks(int m)
{
    return {(m / 4) / PB1 + 1, (m / 4) / PB2 + 1, (m / 4) / PB3 + 1};
}
// Calls emit(i, tile) for the i-th base tile of block b = (b1 n2 + b2) n3 + b3
// that keep(tile) accepts; returns the number of such tiles.
template <class K, class F>
__host__ __device__ inline int plan_block_emit(int m, int b, K &&keep, F &&emit)
{
    const int M = m / 4;
    const PlanBlocks nb = plan_blocks(m);
    const int b3 = b % nb.n3, b2 = (b / nb.n3) % nb.n2, b1 = b / (nb.n3 * nb.n2);
    if (PB1 * b1 + PB2 * b2 + PB3 * b3 > M) return 0;
    int n = 0;
    for (int u1 = b1 * PB1; u1 < (b1 + 1) * PB1; ++u1)
        for (int u2 = b2 * PB2; u2 < (b2 + 1) * PB2; ++u2)
            for (int u3 = b3 * PB3; u3 < (b3 + 1) * PB3; ++u3)
                if (u1 + u2 + u3 <= M && keep(pack3(2 * u1, 2 * u2, u3))) emit(n++, pack3(2 * u1, 2 * u2, u3));
    return n;
}

// The height-2 test reads c(theta(g)) = sum_c g[c] Delta[(p+1)e - c] only
// (Section 3.4), i.e. Delta at the positions x with p^2-1-d <= x_i <= p^2-1
// for all four coordinates (d = 4(p-1), the degree of g).  Since
// A_{k+1}[x] = sum_t m[t] A_k[x - t] with t >= 0, those coefficients depend
// only on the coefficients of A_k whose four coordinates are all <= p^2-1.  The capped chain computes just the
// super-tiles that meet that region: band_tile tells whether the super-tile of
// base tile (c1, c2, c3) at output degree n does (for n = D, the window).
template <int P>
__host__ __device__ constexpr bool band_tile(int n, int c1, int c2, int c3)
{
    constexpr int d = 4 * (P - 1), D = P * d, E = P * P - 1;
    const int lo[3] = {T1 * c1, T2 * c2, T3 * c3};
    const int hi[3] = {T1 * c1 + 2 * T1 - 1, T2 * c2 + 2 * T2 - 1, T3 * c3 + T3 - 1};
    const int flo = n == D ? E - d : 0;
    int wlo = 0, whi = 0;
    for (int i = 0; i < 3; ++i) {
        const int a = lo[i] > flo ? lo[i] : flo, b = hi[i] < E ? hi[i] : E;
        if (a > b) return false;
        wlo += a;
        whi += b;
    }
    // the fourth coordinate n - |x| in [flo, E]
    return whi >= n - E && wlo <= n - flo;
}
template <int P>
__host__ __device__ constexpr bool band_tile_packed(int n, uint32_t t)
{
    return band_tile<P>(n, unp0(t), unp1(t), unp2(t));
}

// Whether a quad of offsets delta can contribute to a set of base tiles b:
// some input tile b - delta has no negative coordinate and minimum weight
// <= nk (it holds part of A_k), and, in the capped chain (cap = p^2-1;
// cap = CAP_NONE otherwise), can have every coordinate <= cap and maximum
// weight >= nk - cap.  m1..m3 / wmin: largest coordinates / smallest weight
// of the set's tiles; l1..l3 / wmax: smallest coordinates / largest weight.
// Quads are packed as pack3(lo1+1, lo2+1, lo3) and pack3(hi1+1, hi2+1, hi3).
constexpr int CAP_NONE = 1 << 20;
__host__ __device__ inline bool quad_needed(int m1, int m2, int m3, int wmin, int l1, int l2, int l3, int wmax,
                                            int nk, int cap, uint32_t qmin, int qwmax, uint32_t qmax, int qwmin)
{
    return m1 >= (int)unp0(qmin) - 1 && m2 >= (int)unp1(qmin) - 1 && m3 >= (int)unp2(qmin) && wmin - qwmax <= nk &&
           T1 * (l1 - ((int)unp0(qmax) - 1)) <= cap && T2 * (l2 - ((int)unp1(qmax) - 1)) <= cap &&
           T3 * (l3 - (int)unp2(qmax)) <= cap && wmax - qwmin + (T1 - 1) + (T2 - 1) + (T3 - 1) >= nk - cap;
}

// Output-tile lists of the deep kernel (packed with pack3), dm the degree of
// the multiplier and NF the number of factors of the chain:
//  base list k (k = 1..NF-1): base tiles of the 2x2 super-tiles of output
//    degree n = (k+1) dm: c1, c2 even, w(c) = 2 c1 + 2 c2 + 4 c3 <= n;
//  shell list 0: all tiles c >= 0 of the box with w(c) <= 2 dm + 4 (A_1 = m
//    and the zeros the first product reads beyond its degree);
//  shell list k (k = 1..NF-2): the tiles with (k+1) dm < w(c) <= (k+2) dm + 4,
//    zeroed after step k because step k+1 reads them;
//  band list k (k = 1..NF-1): the base tiles of list k that band_tile keeps;
//  band shell list k (k = 1..NF-2): the tiles of shell list k whose
//    coordinates are all T_i c_i <= p^2 - 1, the only ones the capped chain reads.
// The base and band lists come with the bounding box of every group of 16
// entries (4 words at gboff / ngoff: max c1 | max c2 << 16, max c3 | min c1
// << 16, min c2 | min c3 << 16, min w | max w << 16).
template <int P>
struct PlanTable {
    static constexpr int NF = Geo<P>::NF;
    int64_t blen[NF], boff[NF], flen[NF], foff[NF], nlen[NF], noff[NF], hlen[NF], hoff[NF], gboff[NF], ngoff[NF];
    int64_t words;
};
// The c3 range [lo, hi] (empty if lo > hi) of shell list k (cap = CAP_NONE)
// or band shell list k (cap = p^2 - 1) in the column (c1, c2).
template <int P>
__host__ __device__ constexpr void shell_c3_range(int k, int cap, int c1, int c2, int &lo, int &hi)
{
    using X = GeoX<P>;
    constexpr int dm = X::dm;
    const int n = k == 0 ? -1 : (k + 1) * dm, m = (k + 2) * dm + 4;
    const int r = T1 * c1 + T2 * c2;
    lo = r > n ? 0 : (n - r) / T3 + 1;
    hi = m < r ? -1 : (m - r) / T3;
    if (hi > X::C3 - 1) hi = X::C3 - 1;
    if (hi > cap / T3) hi = cap / T3;
}
// Largest c1 (and c2) of shell list k's columns.
template <int P>
__host__ __device__ constexpr int shell_cmax(int k, int cap)
{
    using X = GeoX<P>;
    const int m = (k + 2) * GeoX<P>::dm + 4;
    int c = m / T1;
    if (c > X::C1) c = X::C1;
    if (c > cap / T1) c = cap / T1;
    return c;
}
// Base tiles of degree n: base units u >= 0 with u1 + u2 + u3 <= n / 4.
constexpr int64_t base_tiles(int n)
{
    const int64_t u = n / 4;
    return (u + 1) * (u + 2) * (u + 3) / 6;
}
// Tiles of shell list k: the c3 range depends on c1 + c2 only, so the columns
// are counted per diagonal c1 + c2 = s (s + 1 of them for s <= cm, 2 cm - s + 1 beyond).
template <int P>
constexpr int64_t shell_tiles(int k, int cap)
{
    int64_t cnt = 0;
    const int cm = shell_cmax<P>(k, cap);
    for (int s = 0; s <= 2 * cm; ++s) {
        const int a = s <= cm ? s : cm, b = s - a;
        int lo = 0, hi = -1;
        shell_c3_range<P>(k, cap, a, b, lo, hi);
        if (hi >= lo) cnt += (int64_t)(hi - lo + 1) * (s <= cm ? s + 1 : 2 * cm - s + 1);
    }
    return cnt;
}
// Number of base tiles band_tile keeps at degree n.  For fixed (u1, u2) both
// weight conditions of band_tile are monotone in u3, so the kept u3 form an
// interval [lo, hi] (the host checks the count against the predicate).
template <int P>
constexpr int64_t band_tiles(int n)
{
    constexpr int d = 4 * (P - 1), D = P * d, E = P * P - 1, U = E / 4;
    const int flo = n == D ? E - d : 0;
    auto cdiv4 = [](int x) { return x <= 0 ? 0 : (x + 3) / 4; };
    int64_t cnt = 0;
    for (int u1 = 0; u1 <= U && 4 * u1 <= n; ++u1)
        for (int u2 = 0; u2 <= U && 4 * (u1 + u2) <= n; ++u2) {
            const int a1 = 4 * u1 > flo ? 4 * u1 : flo, b1 = 4 * u1 + 3 < E ? 4 * u1 + 3 : E;
            const int a2 = 4 * u2 > flo ? 4 * u2 : flo, b2 = 4 * u2 + 3 < E ? 4 * u2 + 3 : E;
            if (a1 > b1 || a2 > b2) continue;
            // min(4 u3 + 3, E) >= r and max(4 u3, flo) <= t
            const int r = n - E - b1 - b2, t = n - flo - a1 - a2;
            if (r > E || flo > t) continue;
            int lo = cdiv4(r - 3), hi = t / 4;
            const int lo_f = cdiv4(flo - 3), hi_n = n / 4 - u1 - u2;
            if (lo_f > lo) lo = lo_f;
            if (U < hi) hi = U;
            if (hi_n < hi) hi = hi_n;
            if (hi >= lo) cnt += hi - lo + 1;
        }
    return cnt;
}
template <int P>
constexpr PlanTable<P> make_plan_table()
{
    constexpr int dm = Geo<P>::dm, NF = Geo<P>::NF;
    PlanTable<P> t{};
    int64_t o = 0;
    for (int k = 0; k < NF; ++k) {
        t.boff[k] = o;
        t.blen[k] = k >= 1 ? base_tiles((k + 1) * dm) : 0;
        o += t.blen[k];
    }
    for (int k = 0; k < NF; ++k) {
        t.foff[k] = o;
        t.flen[k] = k <= NF - 2 ? shell_tiles<P>(k, CAP_NONE) : 0;
        o += t.flen[k];
    }
    for (int k = 0; k < NF; ++k) {
        t.noff[k] = o;
        t.nlen[k] = k >= 1 ? band_tiles<P>((k + 1) * dm) : 0;
        o += t.nlen[k];
    }
    for (int k = 0; k < NF; ++k) {
        t.hoff[k] = o;
        t.hlen[k] = k >= 1 && k <= NF - 2 ? shell_tiles<P>(k, P * P - 1) : 0;
        o += t.hlen[k];
    }
    for (int k = 0; k < NF; ++k) {
        t.gboff[k] = o;
        o += 4 * ((t.blen[k] + 15) / 16);
        t.ngoff[k] = o;
        o += 4 * ((t.nlen[k] + 15) / 16);
    }
    t.words = o;
    return t;
}
// evaluated once per translation unit
template <int P>
inline constexpr PlanTable<P> kPlanTable = make_plan_table<P>();
template <int P>
constexpr int64_t plan_words()
{
    return kPlanTable<P>.words;
}

// W blocks live in LDS when they fit next to the other per-surface tables.
template <int P>
__host__ __device__ constexpr bool w_in_lds()
{
    return GeoX<P>::W_BYTES <= 100 * 1024;
}

// Per persistent workgroup ("slot") of the deep kernel: the W blocks when
// they do not fit in LDS, two tile boxes for the chain m^k, and Delta in
// the Cartier-split layout.
template <int P>
__host__ __device__ constexpr size_t slot_bytes()
{
    return (w_in_lds<P>() ? 0 : align256(GeoX<P>::W_BYTES)) + 2 * align256(GeoX<P>::BOX_BYTES) +
           align256(ThetaGeo<P>::BYTES);
}

struct BatchLayout {
    size_t counters = 0;
    size_t queue[4] = {0, 0, 0, 0};
    size_t queue2[4] = {0, 0, 0, 0};
    size_t gq[4] = {0, 0, 0, 0};
    size_t plan[4] = {0, 0, 0, 0};
    size_t slots = 0;
    size_t slot_stride[4] = {0, 0, 0, 0};
    int nslots[4] = {0, 0, 0, 0};
    bool present[4] = {false, false, false, false};
    size_t total = 0;
};

// Layout for the primes marked in `present`, `batch` surfaces and up to
// `slots` persistent deep workgroups.
BatchLayout make_batch_layout(const bool present[4], int batch, int slots);

int64_t len_g_of(int p);

struct Stage1Args {
    int batch;
    int mode;
    int fixed_p;      // > 0: every surface has this prime (MODE_DELTA)
    int bound;
    const int32_t *p; // [batch] (MODE_HEIGHT)
    const uint8_t *f; // [batch][35]
    int32_t *heights; // MODE_HEIGHT
    int32_t *status;  // MODE_DELTA, may be null
    uint8_t *g_out;   // MODE_DELTA, may be null
    int32_t *counters;
    int32_t *queue[4];
    uint8_t *gq[4];
    int present_mask;
};

struct DeepArgs {
    int mode;
    int bound;
    int from_q2;    // full chain: take surfaces from the second queue (they passed the capped chain)
    int zero_halo;  // zero the boxes' halo first (not needed right after a launch on the same slots)
    int32_t *heights;
    int32_t *status;
    uint8_t *delta_out;
    int32_t *counters;
    const int32_t *queue;
    int32_t *queue2;  // positions in `queue` of the surfaces the capped chain left undecided
    const uint8_t *gq;
    const uint8_t *f;  // [batch][35], the quartics (the multiplier m = f~^J is formed from them)
    uint8_t *g_out;    // MODE_DELTA, may be null: g per surface when the chain forms it
    const uint32_t *plan;
    uint8_t *slots;
    size_t slot_bytes;
};

hipError_t launch_reset(int32_t *counters, hipStream_t s);
// Fedder's test per surface (MODE_HEIGHT; queues the deep ones) or queue every surface (MODE_DELTA)
hipError_t launch_stage1(const Stage1Args &a, hipStream_t s);
// g = f^(p-1) for the surfaces queued for prime p, on nwg persistent workgroups
hipError_t launch_gpow(int p, const Stage1Args &a, int nwg, hipStream_t s);
// whether the deep kernels of prime p take g from launch_gpow (else they read it off their chain)
bool gpow_needed(int p);
// qfs_height_reduced's per-surface kernel over the deep queue of prime p (nwg persistent workgroups)
hipError_t launch_reduced(int p, const Stage1Args &a, int nwg, hipStream_t s);
// the pure matrix-core loop: times `iters` iterations on nwg workgroups (waits for it), and its operation count
hipError_t mfma_peak(int iters, int nwg, int *sink, float *ms, hipStream_t s);
int64_t mfma_peak_ops(int iters, int nwg);
hipError_t launch_plan(int p, uint32_t *plan, hipStream_t s);
// band: the capped-chain kernel (MODE_HEIGHT), else the full-chain kernel
hipError_t launch_deep(int p, bool band, const DeepArgs &a, int nslots, hipStream_t s);
// set the deep kernels' launch attributes for prime p (idempotent)
hipError_t prepare_deep(int p);

// theta on caller-given Delta (CNS order): converts Delta into the
// Cartier-split layout, then iterates.
size_t theta_scratch_bytes(int p);
hipError_t launch_theta(int p, int batch, const uint8_t *delta, const uint8_t *a, uint8_t *out, int iters,
                        uint8_t *scratch, int nslots, hipStream_t s);

int64_t mfma_count(int p, bool band);

// plain per-surface path
size_t plain_scratch_bytes(int p);
hipError_t launch_plain_surface(int p, const uint8_t *f35, int bound, int32_t *height, uint8_t *scratch,
                                hipStream_t s);

}  // namespace qfs
