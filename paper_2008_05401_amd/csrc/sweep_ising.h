// sweep_ising.h -- the bit-packed Ising fast path (sweep_ising.hip and its
// instantiation units sweep_ising_k*.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "sweep_common.h"

namespace crbm {

bool ising_fast_supported(int K, int LW, int L);
// FP64 subset-sum tables of the filter rows (K LW 2^LW doubles, at most 16 KiB) for the
// exact free energy of the MH re-check
__host__ __device__ inline bool ising_fast_t64(int K, int LW) { return K * LW * (1 << LW) <= 2048; }

// Scalars of a job's table block (FP64 exp/log constants of the exact paths,
// the visible-unit constants and the free-energy bound per site).
constexpr int ISING_NDC = 27;
struct IsingTabConst {
    double dc[ISING_NDC];      // constants of exp_c / log_c
    double Bsite;              // bound on the float32 free-energy error per site
    float vb;                  // additive mode: -v_bias log2(e)
    float dAv;                 // Bernoulli band of a visible unit
    float vb_raw;              // v_bias
    float evbm;                // e^{-v_bias}
    float Sv;                  // |v_bias| + sum |W|
    int mult;                  // 1: product mode, 0: additive mode
    int pad[2];
};

// Byte layout of the per-job table block.  It is built once by crbm_init in the
// job's workspace and copied verbatim into the first `bytes` bytes of LDS by
// every workgroup of a sweep launch:
//   [0, off_const)      float32 tables: T1, T2, E1p (K LW 2^LW each), then K
//                       floats each of hbs, dAh, Sk, dApre, ehbm, ehbp, hbl, and
//                       the filters W (K LW^2);
//   [off_const, +256)   IsingTabConst;
//   [off_t64, bytes)    FP64 subset sums of the filter rows (ising_fast_t64 only).
struct IsingTabLayout {
    int off_const, off_t64, bytes;
};

__host__ __device__ inline IsingTabLayout ising_tab_layout(int K, int LW)
{
    const int tsz = K * LW * (1 << LW);
    IsingTabLayout t;
    t.off_const = ((3 * tsz + 7 * K + K * LW * LW) * 4 + 15) & ~15;
    t.off_t64 = t.off_const + 256;
    t.bytes = t.off_t64 + (ising_fast_t64(K, LW) ? ((tsz * 8 + 15) & ~15) : 0);
    return t;
}
static_assert(sizeof(IsingTabConst) <= 256, "constant block fits its slot");

int ising_fast_threads(int L);
int ising_fast_rows(int L);
size_t ising_fast_lds_bytes(int K, int LW, int L);
// bytes of the table block in the job's workspace
size_t ising_tab_bytes(int K, int LW);
// build the table block of a job (job descriptor already on the device)
hipError_t launch_ising_tables(const JobDev* job_dev, hipStream_t s);
// FP64 free energy of every chain's initial state into its record (after the
// generic initialisation, on the same stream); the LDS it needs
size_t ising_init_fe_lds_bytes(int K, int LW, int L);
hipError_t launch_ising_init_fe(const JobDev* job_dev, int n_chains, int K, int LW, int L, hipStream_t s);
hipError_t launch_ising_fast(const SweepLaunch& P, int K, int LW, int BH, int n_blocks, size_t lds, int nt,
                             hipStream_t s);

// instantiation units: one per compiled (K, LW) pair, KT = 0 for a runtime K
template <int KT, int LW>
hipError_t launch_ising_klw(const SweepLaunch& P, int BH, int n_blocks, size_t lds, int nt, hipStream_t s);

}  // namespace crbm
