// sweep_ising_kxl1.hip -- bit-packed Ising sweep kernels for a runtime K, Lw = 1.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(0, 1)
