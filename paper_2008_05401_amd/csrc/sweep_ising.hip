// sweep_ising.hip -- host side of the bit-packed Ising sweep (shape checks,
// LDS sizes, launch dispatch over the instantiation units) and the kernel that
// builds a job's table block once at crbm_init.
#include "sweep_ising_impl.h"

namespace crbm {

// ---------------------------------------------------------------------------
// Table block of one job (layout in sweep_ising.h), one workgroup, run once by
// crbm_init.  Because v and h are binary, filter row (k, a) contributes the sum
// s(p) of the taps selected by the Lw-bit pattern p:
//   product mode (every partial product within float32 range): T1 = e^{-s},
//     T2 = e^{-s} with the taps reversed (the adjoint pass), E1p = e^{+s}, each
//     the float32 rounding of the FP64 value;
//   additive mode: T1 = -s log2(e), T2 likewise reversed (float32 sums).
// T64 holds s(p) in FP64 for the exact free energy of the MH re-check.  The
// per-channel Bernoulli bands dAh, the visible band dAv and the per-site bound
// of the float32 free energy follow the error analysis of the kernel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ising_tables_kernel(const JobDev* __restrict__ jd)
{
    const JobDev& J = *jd;
    const int K = J.K, LW = J.LW, NP = 1 << LW, tsz = K * LW * NP;
    const int tid = threadIdx.x, NT = blockDim.x;
    const IsingTabLayout tl = ising_tab_layout(K, LW);
    unsigned char* base = J.tab;
    float* T1 = (float*)base;
    float* T2 = T1 + tsz;
    float* E1p = T2 + tsz;
    float* hbs = E1p + tsz;
    float* dAh = hbs + K;
    float* Sk = dAh + K;
    float* dApre = Sk + K;
    float* ehbm = dApre + K;
    float* ehbp = ehbm + K;
    float* hbl = ehbp + K;
    float* Wl = hbl + K;
    IsingTabConst* TC = (IsingTabConst*)(base + tl.off_const);
    double* T64 = ising_fast_t64(K, LW) ? (double*)(base + tl.off_t64) : nullptr;
    __shared__ float s_Sk[64], s_dApre[64];
    __shared__ float s_Sv;
    const float* __restrict__ W = J.W;
    constexpr float NLOG2E = -1.44269504088896341f;

    for (int q = tid; q < K * LW * LW; q += NT) Wl[q] = W[q];
    for (int k = tid; k < K; k += NT) {
        const float hb = J.hb[k];
        hbl[k] = hb;
        float s = fabsf(hb);
        for (int q = 0; q < LW * LW; ++q) s += fabsf(W[k * LW * LW + q]);
        Sk[k] = s;
        s_Sk[k] = s;
        hbs[k] = hb * NLOG2E;
        ehbm[k] = (float)exp(-(double)hb);
        ehbp[k] = (float)exp((double)hb);
    }
    if (tid == 0) {
        const float vb = J.vb[0];
        float s = fabsf(vb);
        for (int q = 0; q < K * LW * LW; ++q) s += fabsf(W[q]);
        TC->vb = vb * NLOG2E;
        TC->vb_raw = vb;
        TC->evbm = (float)exp(-(double)vb);
        TC->Sv = s;
        s_Sv = s;
        fill_dconst(TC->dc);
    }
    __syncthreads();
    // Product mode when every partial product stays well inside the float32
    // normal range: |log| of a hidden factor chain <= S_k, of a visible chain
    // <= S_v, of the free-energy product over channels <= sum_k S_k + K.
    float Smax = s_Sv, Ssum = 0.f;
    for (int k = 0; k < K; ++k) {
        Smax = fmaxf(Smax, s_Sk[k]);
        Ssum += s_Sk[k];
    }
    const bool mult = Smax < 80.f && Ssum + (float)K < 80.f;
    // subset sums of every filter row (T1: taps in order, T2: reversed)
    for (int idx = tid; idx < tsz; idx += NT) {
        const int p = idx & (NP - 1), ka = idx >> LW;
        const float* wr = W + ka * LW;  // (k * LW + a) * LW with C = 1
        if (mult) {
            double d1 = 0.0, d2 = 0.0;
            for (int b = 0; b < LW; ++b) {
                const double w = (double)wr[b];
                if ((p >> b) & 1) d1 += w;
                if ((p >> (LW - 1 - b)) & 1) d2 += w;
            }
            T1[idx] = (float)exp(-d1);
            T2[idx] = (float)exp(-d2);
            E1p[idx] = (float)exp(d1);
            if (T64) T64[idx] = d1;
        } else {
            float s1 = 0.f, s2 = 0.f;
            for (int b = 0; b < LW; ++b) {
                const float w = wr[b];
                if ((p >> b) & 1) s1 += w;
                if ((p >> (LW - 1 - b)) & 1) s2 += w;
            }
            T1[idx] = s1 * NLOG2E;
            T2[idx] = s2 * NLOG2E;
            E1p[idx] = 0.f;
            if (T64) {
                double d1 = 0.0;
                for (int b = 0; b < LW; ++b)
                    if ((p >> b) & 1) d1 += (double)wr[b];
                T64[idx] = d1;
            }
        }
    }
    for (int k = tid; k < K; k += NT) {
        float dp;
        if (mult) {
            // e^{-a} from LW+1 factors each rounded once, LW products
            dp = 0.f;
            dAh[k] = gamma_f32(2 * LW + 1) * 1.01f + 0x1p-22f;
        } else {
            // |a_f32 - a|: table sums <= LW-1 roundings, scaling 1, pre-activation LW + 1
            dp = gamma_f32(2 * LW + 3) * s_Sk[k] * 1.001f;
            // band of u(1 + 2^z) - 1: that error, 2 ulp of exp2, the fma, float u
            dAh[k] = dp + 0x1p-20f;
        }
        dApre[k] = dp;
        s_dApre[k] = dp;
    }
    __syncthreads();
    if (tid == 0) {
        TC->dAv = mult ? gamma_f32(2 * K * LW + 1) * 1.01f + 0x1p-22f
                       : gamma_f32(K * LW + LW + 3) * s_Sv * 1.001f + 0x1p-20f;
        // rigorous bound of the float32 free energy per site
        //   product mode: K factors (1 + e^{a_k}) with e^{a_k} from 2 LW + 1 roundings,
        //   one rounding per product step; the FP64 log of the product is exact enough;
        //   additive mode: pre-activation errors, exp2/log2 and product roundings, max terms
        float dAsum = 0.f;
        for (int k = 0; k < K; ++k) dAsum += s_dApre[k];
        TC->Bsite = mult ? (double)K * ((double)gamma_f32(2 * LW + 1) + 0x1p-24) * 1.02
                         : (double)dAsum + (double)(K + 2) * 0x1p-20 + (double)(K + 2) * 0x1p-24 * 1.5 * (double)Ssum;
        TC->mult = mult ? 1 : 0;
        TC->pad[0] = TC->pad[1] = 0;
    }
}

// ---------------------------------------------------------------------------
// FP64 free energy (Eq. free-energy_CRBM) of each chain's initial state for the
// jobs of the bit-packed kernel, one workgroup per chain, run by crbm_init after
// the generic initialisation (which leaves F to this kernel).  The state goes
// into a bit plane as in the sweep, and F comes from the same exact routine as
// the sweep's MH re-check: per site and channel the FP64 subset sums of the
// filter rows, the softplus terms in product form.
// ---------------------------------------------------------------------------
template <int LW>
__global__ __launch_bounds__(256) void ising_init_fe_kernel(const JobDev* __restrict__ jd)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const JobDev& J = *jd;
    const int g = blockIdx.x;
    const int K = J.K, L = J.L, lgL = 31 - __builtin_clz(L), tsz = K * LW * (1 << LW);
    const int tid = threadIdx.x, NT = blockDim.x;
    const int RS = (L >= 32 ? (L >> 5) : 1) + 1;
    const IsingTabLayout tl = ising_tab_layout(K, LW);
    {
        const uint4* __restrict__ src = (const uint4*)J.tab;
        uint4* dst = (uint4*)smem;
        for (int q = tid; q < tl.bytes / 16; q += NT) dst[q] = src[q];
    }
    const float* hbl = (const float*)smem + 3 * tsz + 6 * K;
    const float* Wl = hbl + K;
    const IsingTabConst& TC = *(const IsingTabConst*)(smem + tl.off_const);
    const double* T64 = ising_fast_t64(K, LW) ? (const double*)(smem + tl.off_t64) : nullptr;
    double* red = (double*)(smem + tl.bytes);
    uint32_t* pl = (uint32_t*)(red + 64);
    const int8_t* state = J.state + (size_t)g * L * L;
    // +-1 int8 lattice -> bit plane, four sites per lane (every lane of a wave
    // takes part in store_nibble)
    const int lgq = lgL - 2, nq = (L * L) >> 2, nrounds = (nq + NT - 1) / NT;
    for (int r = 0; r < nrounds; ++r) {
        const int Q = r * NT + tid;
        const bool active = Q < nq;
        const int i = active ? (Q >> lgq) : 0, m = active ? (Q & ((L >> 2) - 1)) : 0;
        uint32_t nib = 0;
        if (active) {
            const uint32_t w4 = ~*(const uint32_t*)(state + (i << lgL) + 4 * m);
            nib = ((w4 >> 7) & 1u) | ((w4 >> 14) & 2u) | ((w4 >> 21) & 4u) | ((w4 >> 28) & 8u);
        }
        store_nibble(pl, RS, L, i, m, nib, active);
    }
    __syncthreads();
    const double F = free_energy_exact<LW>(Wl, hbl, TC.vb_raw, pl, RS, L, K, red, TC.dc, T64);
    if (tid == 0) J.rec[g].F = F;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
bool ising_fast_supported(int K, int LW, int L)
{
    if (LW < 1 || LW > 6 || LW > L || K < 1 || K > 64) return false;
    if (!(L == 8 || L == 16 || L == 32 || L == 64 || L == 128 || L == 256)) return false;
    return ising_fast_lds_bytes(K, LW, L) <= 160 * 1024;
}

int ising_fast_rows(int L) { return L >= 32 ? 4 : 1; }

int ising_fast_threads(int L)
{
    const int nb = L * L / (4 * ising_fast_rows(L));
    if (nb <= 64) return 64;
    if (nb <= 1024) return 256;
    return 512;
}

size_t ising_tab_bytes(int K, int LW) { return (size_t)ising_tab_layout(K, LW).bytes; }

// LDS of one workgroup: the table block, 64 doubles of reduction scratch, then
// the three visible planes and the K hidden planes (bit-packed rows)
size_t ising_fast_lds_bytes(int K, int LW, int L)
{
    size_t o = ising_tab_bytes(K, LW);
    o += 64 * 8;
    const size_t RS = (L >= 32 ? (size_t)(L >> 5) : 1) + 1;
    o += (3 + (size_t)K) * (size_t)L * RS * 4;
    return o;
}

hipError_t launch_ising_tables(const JobDev* job_dev, hipStream_t s)
{
    hipLaunchKernelGGL(ising_tables_kernel, dim3(1), dim3(256), 0, s, job_dev);
    return hipGetLastError();
}

size_t ising_init_fe_lds_bytes(int K, int LW, int L)
{
    const size_t RS = (L >= 32 ? (size_t)(L >> 5) : 1) + 1;
    return ising_tab_bytes(K, LW) + 64 * 8 + (size_t)L * RS * 4;
}

hipError_t launch_ising_init_fe(const JobDev* job_dev, int n_chains, int K, int LW, int L, hipStream_t s)
{
    const size_t lds = ising_init_fe_lds_bytes(K, LW, L);
    const dim3 grid(n_chains), block(256);
    switch (LW) {
    case 1: hipLaunchKernelGGL(ising_init_fe_kernel<1>, grid, block, lds, s, job_dev); break;
    case 2: hipLaunchKernelGGL(ising_init_fe_kernel<2>, grid, block, lds, s, job_dev); break;
    case 3: hipLaunchKernelGGL(ising_init_fe_kernel<3>, grid, block, lds, s, job_dev); break;
    case 4: hipLaunchKernelGGL(ising_init_fe_kernel<4>, grid, block, lds, s, job_dev); break;
    case 5: hipLaunchKernelGGL(ising_init_fe_kernel<5>, grid, block, lds, s, job_dev); break;
    case 6: hipLaunchKernelGGL(ising_init_fe_kernel<6>, grid, block, lds, s, job_dev); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ising_fast(const SweepLaunch& P, int K, int LW, int BH, int n_blocks, size_t lds, int nt,
                             hipStream_t s)
{
    // channel counts of the configured workloads get unrolled instances
    if (K == 8 && LW == 5) return launch_ising_klw<8, 5>(P, BH, n_blocks, lds, nt, s);
    if (K == 8 && LW == 3) return launch_ising_klw<8, 3>(P, BH, n_blocks, lds, nt, s);
    if (K == 4 && LW == 3) return launch_ising_klw<4, 3>(P, BH, n_blocks, lds, nt, s);
    if (K == 2 && LW == 2) return launch_ising_klw<2, 2>(P, BH, n_blocks, lds, nt, s);
    switch (LW) {
    case 1: return launch_ising_klw<0, 1>(P, BH, n_blocks, lds, nt, s);
    case 2: return launch_ising_klw<0, 2>(P, BH, n_blocks, lds, nt, s);
    case 3: return launch_ising_klw<0, 3>(P, BH, n_blocks, lds, nt, s);
    case 4: return launch_ising_klw<0, 4>(P, BH, n_blocks, lds, nt, s);
    case 5: return launch_ising_klw<0, 5>(P, BH, n_blocks, lds, nt, s);
    case 6: return launch_ising_klw<0, 6>(P, BH, n_blocks, lds, nt, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace crbm
