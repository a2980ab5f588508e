// init.hip -- per-chain set-up of a job: optional initial state from the INIT
// Philox stream (i.i.d. +-1, as the Binomial(p=0.5) start of Alg. 1), the FP64
// CRBM free energy of the state (left to a kernel of the bit-packed sweep for
// its jobs) and its target (Ising E, M or Kitaev S, E_f, C_f); sums zeroed.  One workgroup per chain, byte-per-unit lattice in LDS.
#include "device_common.h"
#include "generic_blocks.h"
#include "kitaev_eig.h"
#include "sweep_common.h"

namespace crbm {

__host__ __device__ inline size_t init_lds_bytes(int K, int C, int LW, int L, int target, int banks, int dense)
{
    const size_t nv = (size_t)C * L * L;
    size_t o = 64 * 8;
    o += dense ? ((size_t)K * (nv + 1) + K + nv) * 4 : ((size_t)banks * (K * C * LW * LW + K) + C) * 4;
    o = (o + 15) / 16 * 16;
    o += (size_t)C * L * L;
    o = (o + 15) / 16 * 16;
    if (target == 1) o += kitaev_lds_bytes(L);
    return o;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void init_kernel(SweepLaunch P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int jb = 0;
    while (jb + 1 < P.n_jobs && (int)blockIdx.x >= P.block_begin[jb + 1]) ++jb;
    const JobDev& J = *P.jobs[jb];
    const int g = (int)blockIdx.x - P.block_begin[jb];
    if (g >= J.n_chains) return;
    const int K = J.K, C = J.C, LW = J.LW, L = J.L, LL = L * L;
    const int nb = 1 + 2 * J.n_edge, nvis = C * LL;
    const int nW = J.dense ? K * (nvis + 1) : nb * K * C * LW * LW;  // LDS floats of W
    const ConvGeo G{K, C, LW, L, J.open_cols, J.n_edge, J.dense};
    const int tid = threadIdx.x, NT = blockDim.x;
    double* red = (double*)smem;
    float* Ws = (float*)(smem + 64 * 8);
    float* hbs = Ws + nW;
    float* vbs = hbs + nb * K;
    const int nvb = J.dense ? nvis : C;
    size_t o = 64 * 8 + ((size_t)nW + nb * K + nvb) * 4;
    o = (o + 15) / 16 * 16;
    uint8_t* v = smem + o;
    o += (size_t)C * LL;
    o = (o + 15) / 16 * 16;
    double* kit = (double*)(smem + o);

    if (J.dense) {
        for (int q = tid; q < K * nvis; q += NT) Ws[(q / nvis) * (nvis + 1) + q % nvis] = J.W[q];
    } else {
        for (int q = tid; q < nW; q += NT) Ws[q] = J.W[q];
    }
    for (int q = tid; q < nb * K; q += NT) hbs[q] = J.hb[q];
    for (int q = tid; q < nvb; q += NT) vbs[q] = J.vb[q];
    const uint32_t gid = J.chain_offset + (uint32_t)g;
    const uint32_t k0 = (uint32_t)J.seed, k1 = (uint32_t)(J.seed >> 32);
    int8_t* state = J.state + (size_t)g * C * LL;
    if (J.init_state) {
        // a persistent CRBM replica starts as a copy of the chain's state
        int8_t* rbm = J.rbm_state ? J.rbm_state + (size_t)g * C * LL : nullptr;
        for (int q = tid; q < C * LL; q += NT) {
            const u32x4 r = philox10((uint32_t)q >> 2, 0u, gid, STREAM_INIT, k0, k1);
            const int8_t s = (word_of(r, q & 3) >> 31) ? (int8_t)1 : (int8_t)-1;
            state[q] = s;
            if (rbm) rbm[q] = s;
            v[q] = s > 0;
        }
    } else {
        for (int q = tid; q < C * LL; q += NT) v[q] = state[q] > 0;
    }
    __syncthreads();
    // jobs of the bit-packed Ising kernel get F from its table-driven FP64 routine,
    // launched right after this kernel
    const double F = J.tab ? 0.0 : free_energy_block(Ws, hbs, vbs, v, G, red);
    long long E = 0, M = 0;
    KitaevOut ko{0.0, 0.0, 0.0};
    if (J.target != 1) {
        ising_em_block(v, L, J.boundary, (long long*)red, E, M);
    } else {
        const int N = LL;
        const KitaevBufs kb = kitaev_bufs(kit, J.kitA ? J.kitA + (size_t)g * kitaev_chain_doubles(L) : nullptr, L);
        ko = kitaev_weight_block<BLOCK>(v, C, L, J.boundary, J.J0, J.J1, J.J2, 1.0 / J.T[g], kb, red);
        // singular values of the initial state, kept for temperature swaps
        if (J.eps)
            for (int q = tid; q < N; q += NT) J.eps[(size_t)g * N + q] = kb.eps[q];
    }
    if (tid == 0) {
        ChainRec R{};
        R.E = E;
        R.F = F;
        R.S = ko.S;
        R.Ef = ko.Ef;
        R.Cf = ko.Cf;
        R.S_bound = ko.B;
        J.rec[g] = R;
    }
}

size_t init_lds(int K, int C, int LW, int L, int target, int banks, int dense)
{
    return init_lds_bytes(K, C, LW, L, target, banks, dense);
}

hipError_t launch_init(const SweepLaunch& P, int n_blocks, size_t lds, int nt, hipStream_t s)
{
    // the Kitaev eigen-step runs with the thread count of the job's sweeps
    if (nt == 1024)
        hipLaunchKernelGGL(init_kernel<1024>, dim3(n_blocks), dim3(1024), lds, s, P);
    else if (nt == 512)
        hipLaunchKernelGGL(init_kernel<512>, dim3(n_blocks), dim3(512), lds, s, P);
    else
        hipLaunchKernelGGL(init_kernel<256>, dim3(n_blocks), dim3(256), lds, s, P);
    return hipGetLastError();
}

}  // namespace crbm
