// sweep_ising_k8l3.hip -- bit-packed Ising sweep kernels for K = 8, Lw = 3.
#include "sweep_ising_launch.h"
CRBM_ISING_INSTANTIATE(8, 3)
