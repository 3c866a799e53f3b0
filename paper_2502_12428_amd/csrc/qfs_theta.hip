// theta^iters(a) for caller-given Delta (CNS order): the map "multiply then
// split" of Section 3.4, theta(a) = u(Delta a) with u from Algorithm 2.
// Each workgroup converts one surface's Delta into the Cartier-split layout
// in its scratch slot, then iterates theta with a in LDS.
#include "qfs_device.h"
#include "qfs_internal.h"

namespace qfs {

constexpr int THETA_NT = 512;

template <int P>
__global__ __launch_bounds__(THETA_NT) void k_theta(int batch, const uint8_t *__restrict__ delta,
                                                     const uint8_t *__restrict__ a, uint8_t *__restrict__ out,
                                                     int iters, uint8_t *scratch, size_t stride)
{
    using PR = Prime<P>;
    using TG = ThetaGeo<P>;
    constexpr int LG = PR::len_g;
    constexpr int LGA = (LG + 15) / 16 * 16;
    constexpr int D = PR::D;
    extern __shared__ __align__(16) uint8_t lds[];
    uint8_t *a_l = lds;
    uint8_t *aperm = lds + LGA;
    uint8_t *dl = scratch + (size_t)blockIdx.x * stride;
    for (int surf = blockIdx.x; surf < batch; surf += gridDim.x) {
        const uint8_t *ds = delta + (size_t)surf * PR::len_D;
        for (int64_t i = threadIdx.x; i < PR::len_D; i += THETA_NT) {
            int x1, x2, x3, x4;
            cns_unrank(D, i, x1, x2, x3, x4);
            dl[theta_addr<P>(x1, x2, x3, x4)] = (uint8_t)(ds[i] % P);
        }
        for (int i = threadIdx.x; i < LG; i += THETA_NT) a_l[i] = (uint8_t)(a[(size_t)surf * LG + i] % P);
        __syncthreads();
        for (int it = 0; it < iters; ++it) {
            build_aperm<P>(a_l, aperm);
            __syncthreads();
            theta_full<P>(dl, aperm, a_l);
            __syncthreads();
        }
        for (int i = threadIdx.x; i < LG; i += THETA_NT) out[(size_t)surf * LG + i] = a_l[i];
        __syncthreads();
    }
}

template <int P>
static size_t theta_lds()
{
    return (size_t)((Prime<P>::len_g + 15) / 16 * 16) + (size_t)((ThetaGeo<P>::APERM + 15) / 16 * 16);
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

hipError_t launch_theta(int p, int batch, const uint8_t *delta, const uint8_t *a, uint8_t *out, int iters,
                        uint8_t *scratch, int nslots, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    const int grid = batch < nslots ? batch : nslots;
    const size_t stride = theta_scratch_bytes(p);
    switch (p) {
    case 3: hipLaunchKernelGGL(k_theta<3>, dim3(grid), dim3(THETA_NT), theta_lds<3>(), s, batch, delta, a, out, iters, scratch, stride); break;
    case 5: hipLaunchKernelGGL(k_theta<5>, dim3(grid), dim3(THETA_NT), theta_lds<5>(), s, batch, delta, a, out, iters, scratch, stride); break;
    case 7: hipLaunchKernelGGL(k_theta<7>, dim3(grid), dim3(THETA_NT), theta_lds<7>(), s, batch, delta, a, out, iters, scratch, stride); break;
    case 11: hipLaunchKernelGGL(k_theta<11>, dim3(grid), dim3(THETA_NT), theta_lds<11>(), s, batch, delta, a, out, iters, scratch, stride); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qfs
