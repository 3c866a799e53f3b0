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
enum { CNT_COUNT = 0, CNT_POP = 4, CNT_ERR = 8, CNT_WORDS = 64 };

enum { MODE_HEIGHT = 0, MODE_DELTA = 1 };

// Output-tile lists of the deep kernel (packed with pack3):
//  base list k (k = 1..P-1): base tiles of the 2x2 super-tiles of output
//    degree n = (k+1) d: c1, c2 even, w(c) = 2 c1 + 2 c2 + 4 c3 <= n;
//  shell list k (k = 0..P-2): all tiles c >= 0 of the box with
//    w(c) <= (k+2) d + 4, the region the next product reads.
template <int P>
struct PlanTable {
    int64_t blen[P], boff[P], flen[P], foff[P];
    int64_t words;
};
template <int P>
constexpr int64_t base_tiles(int n)
{
    int64_t cnt = 0;
    for (int a = 0; T1 * a <= n; a += 2)
        for (int b = 0; T1 * a + T2 * b <= n; b += 2) cnt += (n - T1 * a - T2 * b) / T3 + 1;
    return cnt;
}
template <int P>
constexpr int64_t shell_tiles(int m)
{
    using X = GeoX<P>;
    int64_t cnt = 0;
    for (int a = 0; a <= X::C1 && T1 * a <= m; ++a)
        for (int b = 0; b <= X::C2 && T1 * a + T2 * b <= m; ++b) {
            int top = (m - T1 * a - T2 * b) / T3;
            if (top > X::C3 - 1) top = X::C3 - 1;
            cnt += top + 1;
        }
    return cnt;
}
template <int P>
constexpr PlanTable<P> make_plan_table()
{
    constexpr int d = 4 * (P - 1);
    PlanTable<P> t{};
    int64_t o = 0;
    for (int k = 0; k < P; ++k) {
        t.boff[k] = o;
        t.blen[k] = k >= 1 ? base_tiles<P>((k + 1) * d) : 0;
        o += t.blen[k];
    }
    for (int k = 0; k < P; ++k) {
        t.foff[k] = o;
        t.flen[k] = k <= P - 2 ? shell_tiles<P>((k + 2) * d + 4) : 0;
        o += t.flen[k];
    }
    t.words = o;
    return t;
}
template <int P>
constexpr int64_t plan_words()
{
    return make_plan_table<P>().words;
}

// W blocks live in LDS when they fit next to the other per-surface tables.
template <int P>
__host__ __device__ constexpr bool w_in_lds()
{
    return GeoX<P>::W_BYTES <= 100 * 1024;
}

// Per persistent workgroup ("slot") of the deep kernel: the W blocks when
// they do not fit in LDS, two tile boxes for the chain g~^k, and Delta in
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
    size_t gq[4] = {0, 0, 0, 0};
    size_t plan[4] = {0, 0, 0, 0};
    size_t slots = 0;
    size_t slot_stride[4] = {0, 0, 0, 0};
    int nslots[4] = {0, 0, 0, 0};
    bool present[4] = {false, false, false, false};
    size_t total = 0;
};

// Layout for the primes marked in `present`, `batch` surfaces and the given
// number of compute units.
BatchLayout make_batch_layout(const bool present[4], int batch, int n_cu);

int64_t len_g_of(int p);
size_t dyn_lds_stage1(int max_p);

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
    int32_t *heights;
    int32_t *status;
    uint8_t *delta_out;
    int32_t *counters;
    const int32_t *queue;
    const uint8_t *gq;
    const uint32_t *plan;
    uint8_t *slots;
    size_t slot_bytes;
};

hipError_t launch_reset(int32_t *counters, hipStream_t s);
hipError_t launch_stage1(const Stage1Args &a, int max_p, hipStream_t s);
hipError_t launch_plan(int p, uint32_t *plan, hipStream_t s);
hipError_t launch_deep(int p, const DeepArgs &a, int nslots, hipStream_t s);

// theta on caller-given Delta (CNS order): converts Delta into the
// Cartier-split layout, then iterates.
size_t theta_scratch_bytes(int p);
hipError_t launch_theta(int p, int batch, const uint8_t *delta, const uint8_t *a, uint8_t *out, int iters,
                        uint8_t *scratch, int nslots, hipStream_t s);

int64_t mfma_count(int p);

// plain per-surface path
size_t plain_scratch_bytes(int p);
hipError_t launch_plain_surface(int p, const uint8_t *f35, int bound, int32_t *height, uint8_t *scratch,
                                hipStream_t s);

}  // namespace qfs
