// sweep_ising.hip -- bit-packed Ising fast path (placeholder: not yet enabled).
#include "sweep_ising.h"

namespace crbm {

bool ising_fast_supported(int, int, int) { return false; }
int ising_fast_threads(int) { return 256; }
size_t ising_fast_lds_bytes(int, int, int) { return 0; }
hipError_t launch_ising_fast(const SweepLaunch&, int, int, int, size_t, int, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace crbm
