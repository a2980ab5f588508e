// sweep_ising.h -- the bit-packed Ising fast path (sweep_ising.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "sweep_common.h"

namespace crbm {

bool ising_fast_supported(int K, int LW, int L);
// FP64 subset-sum tables of the filter rows (K LW 2^LW doubles, at most 16 KiB) for the
// exact free energy of the MH re-check
__host__ __device__ inline bool ising_fast_t64(int K, int LW) { return K * LW * (1 << LW) <= 2048; }
int ising_fast_threads(int L);
int ising_fast_rows(int L);
size_t ising_fast_lds_bytes(int K, int LW, int L);
hipError_t launch_ising_fast(const SweepLaunch& P, int K, int LW, int BH, int n_blocks, size_t lds, int nt,
                             hipStream_t s);

}  // namespace crbm
