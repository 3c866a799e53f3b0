// theta^iters(a) for caller-given Delta (CNS order): the map "multiply then
// split" of Section 3.4, theta(a) = u(Delta a) with u from Algorithm 2.
// Each workgroup converts one surface's Delta into the Cartier-split layout
// in its scratch slot, then iterates theta with a in LDS.
#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

constexpr int THETA_NT = 512;

// Delta at a position x (degree D) from the caller's CNS-ordered array, reduced mod P.
template <int P>
struct CnsDelta {
    const uint8_t *ds;
    __device__ uint8_t operator()(int, int x2, int x3, int x4) const
    {
        return (uint8_t)(gload1(ds + cns_rank(x2, x3, x4)) % P);
    }
};

template <int P>
__global__ __launch_bounds__(THETA_NT) void k_theta(int batch, const uint8_t *__restrict__ delta,
                                                     const uint8_t *__restrict__ a, uint8_t *__restrict__ out,
                                                     int iters, uint8_t *scratch, size_t stride)
{
    using PR = Prime<P>;
    using TG = ThetaGeo<P>;
    constexpr int LG = PR::len_g;
    constexpr int LGA = (LG + 15) / 16 * 16;
    extern __shared__ __align__(16) uint8_t lds[];
    constexpr int APA = (TG::APERM + 15) / 16 * 16;
    uint8_t *a_l = lds;
    uint8_t *aperm = lds + LGA;
    uint32_t *sums = (uint32_t *)(lds + LGA + APA);
    uint8_t *dl = scratch + (size_t)blockIdx.x * stride;
    for (int surf = blockIdx.x; surf < batch; surf += gridDim.x) {
        const uint8_t *ds = delta + (size_t)surf * PR::len_D;
        cartier_split<P>(CnsDelta<P>{ds}, dl);
        for (int i = threadIdx.x; i < LG; i += THETA_NT) a_l[i] = (uint8_t)(a[(size_t)surf * LG + i] % P);
        __syncthreads();
        for (int it = 0; it < iters; ++it) {
            build_aperm<P>(a_l, aperm);
            __syncthreads();
            theta_full<P>(dl, aperm, sums, a_l);
            __syncthreads();
        }
        for (int i = threadIdx.x; i < LG; i += THETA_NT) out[(size_t)surf * LG + i] = a_l[i];
        __syncthreads();
    }
}

template <int P>
static size_t theta_lds()
{
    constexpr size_t LGA = (Prime<P>::len_g + 15) / 16 * 16;
    return LGA + (size_t)((ThetaGeo<P>::APERM + 15) / 16 * 16) + 4 * LGA;
}

size_t theta_scratch_bytes(int p)
{
    switch (p) {
    case 3: return align256(ThetaGeo<3>::BYTES);
    case 5: return align256(ThetaGeo<5>::BYTES);
    case 7: return align256(ThetaGeo<7>::BYTES);
    case 11: return align256(ThetaGeo<11>::BYTES);
    }
    return 0;
}

template <int P>
static hipError_t launch_theta_p(int grid, hipStream_t s, int batch, const uint8_t *delta, const uint8_t *a,
                                 uint8_t *out, int iters, uint8_t *scratch, size_t stride)
{
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)k_theta<P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)theta_lds<P>());
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_theta<P>, dim3(grid), dim3(THETA_NT), theta_lds<P>(), s, batch, delta, a, out, iters, scratch,
                       stride);
    return hipGetLastError();
}

hipError_t launch_theta(int p, int batch, const uint8_t *delta, const uint8_t *a, uint8_t *out, int iters,
                        uint8_t *scratch, int nslots, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    const int grid = batch < nslots ? batch : nslots;
    const size_t stride = theta_scratch_bytes(p);
    switch (p) {
    case 3: return launch_theta_p<3>(grid, s, batch, delta, a, out, iters, scratch, stride);
    case 5: return launch_theta_p<5>(grid, s, batch, delta, a, out, iters, scratch, stride);
    case 7: return launch_theta_p<7>(grid, s, batch, delta, a, out, iters, scratch, stride);
    case 11: return launch_theta_p<11>(grid, s, batch, delta, a, out, iters, scratch, stride);
    }
    return hipErrorInvalidValue;
}

}  // namespace qfs
