// sweep_ising_kxl5.hip -- bit-packed Ising sweep kernels for a runtime K, Lw = 5.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(0, 5)
