// sweep_ising_kxl4.hip -- bit-packed Ising sweep kernels for a runtime K, Lw = 4.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(0, 4)
