// sweep_ising_k4l3.hip -- bit-packed Ising sweep kernels for K = 4, Lw = 3.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(4, 3)
