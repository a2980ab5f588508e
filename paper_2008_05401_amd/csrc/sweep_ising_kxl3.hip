// sweep_ising_kxl3.hip -- bit-packed Ising sweep kernels for a runtime K, Lw = 3.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(0, 3)
