// sweep_common.h -- job descriptors shared by the sweep kernels and the host
// side of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace crbm {

// One job as the kernels see it; lives in the job's device workspace.
struct JobDev {
    const float* W;
    const float* hb;
    const float* vb;
    const double* T;
    int8_t* state;
    int8_t* rbm_state;  // persistent CRBM replicas or nullptr
    ChainRec* rec;
    double* eps;        // Kitaev: singular values of every chain's current state [n_chains][L*L]
    double* trace;      // per-sweep energy ring buffer [n_chains][trace_len] or nullptr
    double* kitA;       // Kitaev: per-chain N x N global scratch (Jacobi re-check; eigen-step beyond L = 12)
    unsigned char* tab; // bit-packed Ising kernel: the job's table block (built at crbm_init)
    double J0, J1, J2;
    double mh_band_min; // least half-width of the MH re-check band
    uint64_t seed;
    int K, C, LW, target, L, n_chains, gibbs_k, burnin;
    uint32_t chain_offset;
    int init_state;
    int trace_len;
    int open_cols;  // CRBM windows stop at the column edge (locally connected CRBM)
    int n_edge;     // unshared filter banks per side; banks = 1 + 2 n_edge
    int boundary;   // target lattice: 0 periodic, 1 open columns
    int dense;      // fully connected RBM: W[K][C L^2], hbias[K], vbias[C L^2]
};

constexpr int MAX_JOBS_PER_LAUNCH = 128;
enum : int { MODE_SWEEP = 0, MODE_INIT = 1 };

// Kernel argument block of one launch: blocks [block_begin[j], block_begin[j+1])
// belong to job j, one block (or one block slice) per chain.
struct SweepLaunch {
    const JobDev* jobs[MAX_JOBS_PER_LAUNCH];
    int block_begin[MAX_JOBS_PER_LAUNCH + 1];
    int n_jobs;
    int n_sweeps;
    int mode;
    int pad;
};

size_t generic_lds_bytes(int K, int C, int LW, int L, int target, int banks, int dense);
// Kitaev eigen-step: largest L, and global scratch bytes per chain (0 while A fits in LDS)
int kitaev_max_l();
size_t kitaev_scratch_bytes(int L);
hipError_t launch_autocorr(const double* trace, int n, int len, int start, int max_lag, double c_win, double* out,
                           double* tau, int* window, hipStream_t s);
hipError_t launch_tempering_swap(const JobDev* job_dev, int n_pairs, int n_ladders, int q0, uint32_t round,
                                 int target, hipStream_t s);
size_t init_lds(int K, int C, int LW, int L, int target, int banks, int dense);
hipError_t launch_init(const SweepLaunch& P, int n_blocks, size_t lds, int nt, hipStream_t s);
hipError_t launch_generic(const SweepLaunch& P, int n_blocks, size_t lds, int nt, hipStream_t s);

}  // namespace crbm
