// sweep_ising_k2l2.hip -- bit-packed Ising sweep kernels for K = 2, Lw = 2.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(2, 2)
