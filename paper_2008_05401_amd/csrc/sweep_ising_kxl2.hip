// sweep_ising_kxl2.hip -- bit-packed Ising sweep kernels for a runtime K, Lw = 2.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(0, 2)
