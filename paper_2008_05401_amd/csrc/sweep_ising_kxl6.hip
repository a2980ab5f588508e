// sweep_ising_kxl6.hip -- bit-packed Ising sweep kernels for a runtime K, Lw = 6.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(0, 6)
