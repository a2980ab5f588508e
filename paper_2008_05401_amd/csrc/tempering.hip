// tempering.hip -- temperature swaps of parallel tempering (App. B): states
// at neighbouring temperatures are exchanged with the probability of Eq.
// (acceptance) between two physical distributions.  A job's chains form a
// grid chain = rung * n_ladders + ladder; one launch handles one round, in
// which the pairs (rung q, rung q + 1), q = q0, q0 + 2, ..., of every ladder
// are disjoint, so every pair is one independent wave.
#include "device_common.h"
#include "kitaev_eig.h"
#include "sweep_common.h"

namespace crbm {

constexpr int SWAP_NT = 64;

__global__ __launch_bounds__(SWAP_NT) void tempering_swap_kernel(const JobDev* __restrict__ Jp, int n_ladders, int q0,
                                                                 uint32_t round)
{
    const JobDev& J = *Jp;
    const int pair = (int)blockIdx.x;
    const int q = q0 + 2 * (pair / n_ladders), l = pair - (pair / n_ladders) * n_ladders;
    const int a = q * n_ladders + l, b = a + n_ladders;
    if (b >= J.n_chains) return;
    const int tid = threadIdx.x;
    const int LL = J.L * J.L, nv = J.C * LL;
    ChainRec* Ra = J.rec + a;
    ChainRec* Rb = J.rec + b;
    const double ba = 1.0 / J.T[a], bb = 1.0 / J.T[b];
    const bool kitaev = J.target == 1;

    // log A = log P_a(x_b) + log P_b(x_a) - log P_a(x_a) - log P_b(x_b)
    double logA, Sab = 0.0, Sba = 0.0, Efab = 0.0, Efba = 0.0, Cfab = 0.0, Cfba = 0.0, Bab = 0.0, Bba = 0.0;
    const double dlam = kitaev ? kitaev_dlam(LL, J.J0, J.J1, J.J2) : 0.0;
    if (!kitaev) {
        logA = J.J0 * (ba - bb) * (double)(Ra->E - Rb->E);
    } else {
        const double* ea = J.eps + (size_t)a * LL;
        const double* eb = J.eps + (size_t)b * LL;
        for (int i = tid; i < LL; i += SWAP_NT) {
            const double xa = 0.5 * ba * eb[i], xb = 0.5 * bb * ea[i];
            Sab += log2cosh_d(xa);
            Sba += log2cosh_d(xb);
            Efab -= 0.5 * eb[i] * tanh(xa);
            Efba -= 0.5 * ea[i] * tanh(xb);
            const double ca = cosh(xa), cb = cosh(xb);
            Cfab += xa * xa / (ca * ca);
            Cfba += xb * xb / (cb * cb);
            // error bounds of the new S (as in the eigen-step), for states whose singular
            // values come from the fast route
            Bab += kitaev_bound_term(eb[i] * eb[i], ba, dlam);
            Bba += kitaev_bound_term(ea[i] * ea[i], bb, dlam);
        }
        Sab = wave_sum(Sab);
        Sba = wave_sum(Sba);
        Efab = wave_sum(Efab);
        Efba = wave_sum(Efba);
        Cfab = wave_sum(Cfab);
        Cfba = wave_sum(Cfba);
        Bab = wave_sum(Bab);
        Bba = wave_sum(Bba);
        logA = Sab + Sba - Ra->S - Rb->S;
    }
    const double lu = log(uniform53(J.seed, round, J.chain_offset + (uint32_t)a, STREAM_PT));
    if (!(lu < logA)) return;  // the same decision in every lane

    // swap the physical states (and the singular values)
    int8_t* xa = J.state + (size_t)a * nv;
    int8_t* xb = J.state + (size_t)b * nv;
    if (((nv & 15) | (int)(((uintptr_t)xa | (uintptr_t)xb) & 15)) == 0) {
        uint4* va = (uint4*)xa;
        uint4* vb = (uint4*)xb;
        for (int i = tid; i < (nv >> 4); i += SWAP_NT) {
            const uint4 t = va[i];
            va[i] = vb[i];
            vb[i] = t;
        }
    } else {
        for (int i = tid; i < nv; i += SWAP_NT) {
            const int8_t t = xa[i];
            xa[i] = xb[i];
            xb[i] = t;
        }
    }
    if (kitaev) {
        double* ea = J.eps + (size_t)a * LL;
        double* eb = J.eps + (size_t)b * LL;
        for (int i = tid; i < LL; i += SWAP_NT) {
            const double t = ea[i];
            ea[i] = eb[i];
            eb[i] = t;
        }
    }
    if (tid == 0) {
        const double F = Ra->F, Fb = Ra->F_bound;
        Ra->F = Rb->F;
        Ra->F_bound = Rb->F_bound;
        Rb->F = F;
        Rb->F_bound = Fb;
        if (!kitaev) {
            const long long E = Ra->E;
            Ra->E = Rb->E;
            Rb->E = E;
        } else {
            // states whose S came from the Jacobi route keep S_bound = 0 (their singular
            // values are the accurate ones)
            const double Sbnd_a = Rb->S_bound > 0.0 ? dlam * Bab + (double)(LL + 4) * 0x1p-53 * Sab : 0.0;
            const double Sbnd_b = Ra->S_bound > 0.0 ? dlam * Bba + (double)(LL + 4) * 0x1p-53 * Sba : 0.0;
            Ra->S = Sab;
            Ra->Ef = Efab;
            Ra->Cf = Cfab;
            Ra->S_bound = Sbnd_a;
            Rb->S = Sba;
            Rb->Ef = Efba;
            Rb->Cf = Cfba;
            Rb->S_bound = Sbnd_b;
        }
        Ra->n_swap += 1;
        Rb->n_swap += 1;
    }
}

hipError_t launch_tempering_swap(const JobDev* job_dev, int n_pairs, int n_ladders, int q0, uint32_t round,
                                 int target, hipStream_t s)
{
    (void)target;
    hipLaunchKernelGGL(tempering_swap_kernel, dim3(n_pairs), dim3(SWAP_NT), 0, s, job_dev, n_ladders, q0, round);
    return hipGetLastError();
}

}  // namespace crbm
