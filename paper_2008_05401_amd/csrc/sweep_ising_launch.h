// sweep_ising_launch.h -- launchers of the bit-packed Ising kernel for one
// compile-time (K, LW) pair; included only by the instantiation units
// sweep_ising_k*.hip, each of which compiles one pair (a parallel build).
#pragma once
#include "sweep_ising_impl.h"

namespace crbm {

template <int KT, int LW, int BH>
static hipError_t launch_ising_klwb(const SweepLaunch& P, int n_blocks, size_t lds, int nt, hipStream_t s)
{
    switch (nt) {
    case 64:
        hipLaunchKernelGGL((sweep_ising_kernel<KT, LW, 64, BH>), dim3(n_blocks), dim3(64), lds, s, P);
        break;
    case 256:
        hipLaunchKernelGGL((sweep_ising_kernel<KT, LW, 256, BH>), dim3(n_blocks), dim3(256), lds, s, P);
        break;
    case 512:
        hipLaunchKernelGGL((sweep_ising_kernel<KT, LW, 512, BH>), dim3(n_blocks), dim3(512), lds, s, P);
        break;
    case 1024:
        hipLaunchKernelGGL((sweep_ising_kernel<KT, LW, 1024, BH>), dim3(n_blocks), dim3(1024), lds, s, P);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KT, int LW>
hipError_t launch_ising_klw(const SweepLaunch& P, int BH, int n_blocks, size_t lds, int nt, hipStream_t s)
{
    if (BH == 4) return launch_ising_klwb<KT, LW, 4>(P, n_blocks, lds, nt, s);
    if (BH == 2) return launch_ising_klwb<KT, LW, 2>(P, n_blocks, lds, nt, s);
    return launch_ising_klwb<KT, LW, 1>(P, n_blocks, lds, nt, s);
}

}  // namespace crbm

#define CRBM_ISING_INSTANTIATE(KT, LW)                                                                            \
    namespace crbm {                                                                                              \
    template hipError_t launch_ising_klw<KT, LW>(const SweepLaunch&, int, int, size_t, int, hipStream_t);         \
    }
