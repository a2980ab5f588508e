// sweep_generic.hip -- generic fused propose+accept sweep for gfx950.
//
// One workgroup owns one chain for the whole launch: the chain's lattice, the
// Gibbs intermediates and the filters sit in LDS, so HBM is touched only to
// load the state at the start and to store it at the end.  A sweep is
//   - gibbs_k block-Gibbs steps (App. B): hidden pass v -> h and visible pass
//     h -> v' of the convolutional conditionals, float32 pre-activations with a
//     guarded Bernoulli test (FP64 re-evaluation inside the error band);
//   - F(v') of Eq. (free-energy_CRBM) in FP64;
//   - the target: Ising E(v') (integer) or the Kitaev weight S(v') (FP64
//     eigen-step, kitaev_eig.h);
//   - the MH test of Eq. (acceptance) with the CRBM as the second replica;
//   - the observables of the state after the sweep.
// The lattice is stored one byte per unit here, which supports every L, C and
// filter size; the bit-packed kernel in sweep_ising.hip is the fast path for
// the Ising workloads.
#include "device_common.h"
#include "generic_blocks.h"
#include "kitaev_eig.h"
#include "sweep_common.h"

namespace crbm {

struct GenericLds {
    // byte offsets inside dynamic LDS
    int off_red, off_W, off_hb, off_vb, off_dah, off_dav, off_v, off_h, off_kit, total;
};

__host__ __device__ inline GenericLds generic_lds_layout(int K, int C, int LW, int L, int target, int banks,
                                                        int dense)
{
    GenericLds g;
    const int LL = L * L, nv = C * LL;
    int o = 0;
    auto al = [](int x, int a) { return (x + a - 1) / a * a; };
    g.off_red = o;
    o += 64 * 8;
    g.off_W = o;
    o += al(dense ? K * (nv + 1) * 4 : banks * K * C * LW * LW * 4, 16);
    g.off_hb = o;
    o += al(banks * K * 4, 16);
    g.off_vb = o;
    o += al((dense ? nv : C) * 4, 16);
    g.off_dah = o;
    o += al(banks * K * 4, 16);
    g.off_dav = o;
    o += al((dense ? nv : C) * 4, 16);
    g.off_v = o;
    o += al(3 * C * LL, 16);
    g.off_h = o;
    o += al(dense ? K : K * LL, 16);
    g.off_kit = o;
    if (target == 1) o += (int)kitaev_lds_bytes(L);
    g.total = al(o, 16);
    return g;
}

template <int NT>
__global__ __launch_bounds__(NT) void sweep_generic_kernel(SweepLaunch P)
{
    extern __shared__ __align__(16) unsigned char smem[];
    int jb = 0;
    while (jb + 1 < P.n_jobs && (int)blockIdx.x >= P.block_begin[jb + 1]) ++jb;
    const JobDev& J = *P.jobs[jb];
    const int g = (int)blockIdx.x - P.block_begin[jb];
    if (g >= J.n_chains) return;

    const int K = J.K, C = J.C, LW = J.LW, L = J.L, LL = L * L;
    const int nb = 1 + 2 * J.n_edge;
    const ConvGeo G{K, C, LW, L, J.open_cols, J.n_edge, J.dense};
    const int tid = threadIdx.x;
    const int nvis = C * LL;  // visible units
    const GenericLds lay = generic_lds_layout(K, C, LW, L, J.target, nb, J.dense);
    double* red = (double*)(smem + lay.off_red);
    long long* redi = (long long*)(smem + lay.off_red);
    float* Ws = (float*)(smem + lay.off_W);
    float* hbs = (float*)(smem + lay.off_hb);
    float* vbs = (float*)(smem + lay.off_vb);
    float* dAh = (float*)(smem + lay.off_dah);
    float* dAv = (float*)(smem + lay.off_dav);
    uint8_t* vb3 = (uint8_t*)(smem + lay.off_v);
    uint8_t* h = (uint8_t*)(smem + lay.off_h);
    double* kit = (double*)(smem + lay.off_kit);

    const int nW = K * C * LW * LW;
    if (G.dense) {
        for (int q = tid; q < K * nvis; q += NT) Ws[(q / nvis) * (nvis + 1) + q % nvis] = J.W[q];
        for (int q = tid; q < K; q += NT) hbs[q] = J.hb[q];
        for (int q = tid; q < nvis; q += NT) vbs[q] = J.vb[q];
        __syncthreads();
        // error bounds: hidden unit k sums nv terms, visible unit q sums K terms
        for (int k = tid; k < K; k += NT) {
            float s = fabsf(hbs[k]);
            for (int q = 0; q < nvis; ++q) s += fabsf(Ws[k * (nvis + 1) + q]);
            dAh[k] = gamma_f32(nvis + 2) * s * 1.001f;
        }
        for (int q = tid; q < nvis; q += NT) {
            float s = fabsf(vbs[q]);
            for (int k = 0; k < K; ++k) s += fabsf(Ws[k * (nvis + 1) + q]);
            dAv[q] = gamma_f32(K + 2) * s * 1.001f;
        }
    } else {
        for (int q = tid; q < nb * nW; q += NT) Ws[q] = J.W[q];
        for (int q = tid; q < nb * K; q += NT) hbs[q] = J.hb[q];
        for (int q = tid; q < C; q += NT) vbs[q] = J.vb[q];
        __syncthreads();
        // error bounds of the float32 pre-activations (recursive fma summation):
        // per bank and hidden channel; a visible unit sums terms of several banks,
        // so its bound takes the largest |W| over the banks term by term
        for (int bk = tid; bk < nb * K; bk += NT) {
            float s = fabsf(hbs[bk]);
            for (int q = 0; q < C * LW * LW; ++q) s += fabsf(Ws[bk * C * LW * LW + q]);
            dAh[bk] = gamma_f32(C * LW * LW + 2) * s * 1.001f;
        }
        for (int c = tid; c < C; c += NT) {
            float s = fabsf(vbs[c]);
            for (int k = 0; k < K; ++k)
                for (int q = 0; q < LW * LW; ++q) {
                    float m = 0.0f;
                    for (int b = 0; b < nb; ++b) m = fmaxf(m, fabsf(Ws[b * nW + (k * C + c) * LW * LW + q]));
                    s += m;
                }
            dAv[c] = gamma_f32(K * LW * LW + 2) * s * 1.001f;
        }
    }

    const uint32_t gid = J.chain_offset + (uint32_t)g;
    const uint32_t k0 = (uint32_t)J.seed, k1 = (uint32_t)(J.seed >> 32);
    int8_t* state = J.state + (size_t)g * C * LL;
    ChainRec* rec = J.rec + g;

    // load the state (crbm_init has generated it if asked to) into plane 0 and
    // a persistent CRBM replica, if the job keeps one, into plane 1
    const bool replica = J.rbm_state != nullptr;
    int8_t* rbm_state = replica ? J.rbm_state + (size_t)g * C * LL : nullptr;
    uint8_t* vcur0 = vb3;
    for (int q = tid; q < C * LL; q += NT) vcur0[q] = state[q] > 0;
    if (replica)
        for (int q = tid; q < C * LL; q += NT) vb3[C * LL + q] = rbm_state[q] > 0;
    __syncthreads();

    const double T = J.T[g];
    const double beta = 1.0 / T;
    const bool ising = J.target != 1;      // Ising or Gibbs-only (sums of channel 0)
    const bool gibbs_only = J.target == 2;

    // ---------------------------------------------------------------- sweeps
    __shared__ long long sh_t0;
    __shared__ int sh_acc, sh_flag;
    __shared__ long long sh_M;
    __shared__ ChainRec R;  // touched by thread 0 only; in LDS so that no lane holds it in registers
    if (tid == 0) {
        R = *rec;
        sh_t0 = R.sweeps;
    }
    long long Mcur = 0;
    if (ising) {
        long long Ed;
        ising_em_block(vcur0, L, J.boundary, redi, Ed, Mcur);
    } else {
        __syncthreads();
    }
    const uint32_t t0 = (uint32_t)sh_t0;
    int cur = 0, rbm = 1;
    int nre = 0;
    for (int it = 0; it < P.n_sweeps; ++it) {
        const uint32_t t = t0 + (uint32_t)it;
        int src = replica ? rbm : cur;
        for (int sub = 0; sub < J.gibbs_k; ++sub) {
            int dst = (src + 1) % 3;
            if (dst == cur) dst = (dst + 1) % 3;
            const uint8_t* vs = vb3 + src * C * LL;
            uint8_t* vd = vb3 + dst * C * LL;
            // hidden pass
            const int nh = G.dense ? K : K * LL, ngh = (nh + 3) >> 2;
            const uint32_t tagh = STREAM_HID | ((uint32_t)sub << 8), tagv = STREAM_VIS | ((uint32_t)sub << 8);
            auto hid_unit = [&](int q, uint32_t word) {
                if (G.dense) {
                    const float a = dense_hidden_f(Ws, hbs, vs, nvis, q);
                    bool near;
                    bool on = bernoulli_fast(a, word, dAh[q], near);
                    if (near) {
                        on = bernoulli_exact(dense_hidden_d(Ws, hbs, vs, nvis, q), word);
                        ++nre;
                    }
                    h[q] = on;
                } else {
                    const int k = q / LL, rr = q - k * LL, i = rr / L, j = rr - i * L;
                    const float a = preact_hidden_f(Ws, hbs, vs, G, k, i, j);
                    bool near;
                    bool on = bernoulli_fast(a, word, dAh[G.bank(j) * K + k], near);
                    if (near) {
                        on = bernoulli_exact(preact_hidden_d(Ws, hbs, vs, G, k, i, j), word);
                        ++nre;
                    }
                    h[q] = on;
                }
            };
            if (ngh < NT) {
                // fewer Philox blocks than lanes: a lane per unit (each lane draws its unit's block)
                for (int q = tid; q < nh; q += NT) {
                    const u32x4 r = philox10((uint32_t)q >> 2, t, gid, tagh, k0, k1);
                    hid_unit(q, word_of(r, q & 3));
                }
            } else {
                for (int gi = tid; gi < ngh; gi += NT) {
                    const u32x4 r = philox10((uint32_t)gi, t, gid, tagh, k0, k1);
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        if (4 * gi + w < nh) hid_unit(4 * gi + w, word_of(r, w));
                }
            }
            __syncthreads();
            // visible pass
            const int nv = C * LL, ngv = (nv + 3) >> 2;
            auto vis_unit = [&](int q, uint32_t word) {
                if (G.dense) {
                    const float b = dense_visible_f(Ws, vbs, h, K, nvis, q);
                    bool near;
                    bool on = bernoulli_fast(b, word, dAv[q], near);
                    if (near) {
                        on = bernoulli_exact(dense_visible_d(Ws, vbs, h, K, nvis, q), word);
                        ++nre;
                    }
                    vd[q] = on;
                } else {
                    const int c = q / LL, rr = q - c * LL, x = rr / L, y = rr - x * L;
                    const float b = preact_visible_f(Ws, vbs, h, G, c, x, y);
                    bool near;
                    bool on = bernoulli_fast(b, word, dAv[c], near);
                    if (near) {
                        on = bernoulli_exact(preact_visible_d(Ws, vbs, h, G, c, x, y), word);
                        ++nre;
                    }
                    vd[q] = on;
                }
            };
            if (ngv < NT) {
                for (int q = tid; q < nv; q += NT) {
                    const u32x4 r = philox10((uint32_t)q >> 2, t, gid, tagv, k0, k1);
                    vis_unit(q, word_of(r, q & 3));
                }
            } else {
                for (int gi = tid; gi < ngv; gi += NT) {
                    const u32x4 r = philox10((uint32_t)gi, t, gid, tagv, k0, k1);
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        if (4 * gi + w < nv) vis_unit(4 * gi + w, word_of(r, w));
                }
            }
            __syncthreads();
            src = dst;
        }
        const uint8_t* vp = vb3 + src * C * LL;
        double Fp = 0.0;
        long long Ep = 0, Mp = 0;
        KitaevOut ko{0.0, 0.0, 0.0};
        double* scratch = J.kitA ? J.kitA + (size_t)g * kitaev_chain_doubles(L) : nullptr;
        if (ising) {
            Fp = free_energy_block(Ws, hbs, vbs, vp, G, red);
            ising_em_block(vp, L, J.boundary, redi, Ep, Mp);
        } else {
            const KitaevBufs kb = kitaev_bufs(kit, scratch, L);
            bool f_done = false;
            if constexpr (NT == KITAEV_SMALL_NT) {
                if (LL <= KITAEV_WAVE_MAX_N) {
                    // F(x') on waves 1..3 while wave 0 forms the tridiagonal matrix
                    const auto fside = [=](int ft, int fnt) { return free_energy_part(Ws, hbs, vbs, vp, G, ft, fnt); };
                    ko = kitaev_weight_small(vp, C, L, J.boundary, J.J0, J.J1, J.J2, beta, kb.eps, kb.eps, red, fside,
                                             Fp);
                    f_done = true;
                }
            }
            if (!f_done) {
                Fp = free_energy_block(Ws, hbs, vbs, vp, G, red);
                ko = kitaev_weight_block<NT>(vp, C, L, J.boundary, J.J0, J.J1, J.J2, beta, kb, red);
            }
        }
        double lu = 0.0;
        if (tid == 0) {
            const double logr = ising ? (-beta * J.J0 * (double)(Ep - R.E) + (Fp - R.F)) : ((ko.S - R.S) + (Fp - R.F));
            lu = log(mh_uniform(J.seed, t, gid));
            int acc = gibbs_only ? 1 : (lu < logr);
            if (!ising) {
                // Kitaev: the fast S of both states carries a rigorous bound (B_S); F is FP64
                // with relative error far below 1e-12.  Inside the band both S come again
                // from the Jacobi route.
                double band = ko.B + R.S_bound + 1e-12 * (1.0 + fabs(ko.S) + fabs(R.S) + fabs(Fp) + fabs(R.F));
                band = fmax(band, J.mh_band_min);
                if (fabs(logr - lu) <= band) acc = 2;
            }
            sh_acc = acc;
        }
        __syncthreads();
        if (sh_acc == 2) {
            // re-check: singular values of M by one-sided Jacobi for the proposal (into the
            // LDS eps buffer, stored on acceptance) and, unless its cached S already came from
            // this route, for the current state (its stored singular values are replaced)
            ko = kitaev_weight_jacobi(vp, C, L, J.boundary, J.J0, J.J1, J.J2, beta, scratch, kit, red, &sh_flag);
            if (R.S_bound > 0.0) {
                const KitaevOut kc = kitaev_weight_jacobi(vb3 + cur * C * LL, C, L, J.boundary, J.J0, J.J1, J.J2,
                                                          beta, scratch, J.eps + (size_t)g * LL, red, &sh_flag);
                if (tid == 0) {
                    R.S = kc.S;
                    R.Ef = kc.Ef;
                    R.Cf = kc.Cf;
                    R.S_bound = 0.0;
                }
            }
            if (tid == 0) {
                const double logr = (ko.S - R.S) + (Fp - R.F);
                sh_acc = lu < logr;
                R.n_recheck += 1;
            }
            __syncthreads();
        }
        if (tid == 0) {
            const int acc = sh_acc;
            if (acc) {
                R.F = Fp;
                R.E = Ep;
                R.S = ko.S;
                R.Ef = ko.Ef;
                R.Cf = ko.Cf;
                R.S_bound = ko.B;
                R.n_acc += 1;
                sh_M = Mp;
            } else {
                sh_M = Mcur;
            }
            R.sweeps += 1;
            if (J.trace) J.trace[(size_t)g * J.trace_len + t % (uint32_t)J.trace_len] = ising ? (double)R.E : R.Ef;
            if ((long long)t >= (long long)J.burnin) {
                R.n_meas += 1;
                if (ising) {
                    const long long m = sh_M;
                    R.sumE += R.E;
                    R.sumE2 += R.E * R.E;
                    R.sumM += m;
                    R.sumAbsM += m < 0 ? -m : m;
                    R.sumM2 += m * m;
                } else {
                    R.kE += R.Ef;
                    R.kE2 += R.Ef * R.Ef;
                    R.kCf += R.Cf;
                }
            }
        }
        __syncthreads();
        // exchange: accepted -> x <- y', y <- x; rejected -> y <- y'
        if (sh_acc) {
            rbm = cur;
            cur = src;
            Mcur = Mp;
            if (!ising && J.eps)
                for (int q = tid; q < LL; q += NT) J.eps[(size_t)g * LL + q] = kit[q];
            __syncthreads();
        } else {
            rbm = src;
        }
    }
    // store the state(s) and the record
    const uint8_t* vc = vb3 + cur * C * LL;
    for (int q = tid; q < C * LL; q += NT) state[q] = vc[q] ? (int8_t)1 : (int8_t)-1;
    if (replica) {
        const uint8_t* vr = vb3 + rbm * C * LL;
        for (int q = tid; q < C * LL; q += NT) rbm_state[q] = vr[q] ? (int8_t)1 : (int8_t)-1;
    }
    const int tot = block_sum(nre, (int*)redi);
    if (tid == 0) {
        R.n_recheck += tot;
        *rec = R;
    }
}

template __global__ void sweep_generic_kernel<1024>(SweepLaunch);
template __global__ void sweep_generic_kernel<512>(SweepLaunch);
template __global__ void sweep_generic_kernel<256>(SweepLaunch);
template __global__ void sweep_generic_kernel<64>(SweepLaunch);

int kitaev_max_l() { return KITAEV_MAX_L; }

size_t kitaev_scratch_bytes(int L) { return kitaev_chain_doubles(L) * sizeof(double); }

size_t generic_lds_bytes(int K, int C, int LW, int L, int target, int banks, int dense)
{
    return (size_t)generic_lds_layout(K, C, LW, L, target, banks, dense).total;
}

hipError_t launch_generic(const SweepLaunch& P, int n_blocks, size_t lds, int nt, hipStream_t s)
{
    if (nt == 64) {
        hipLaunchKernelGGL(sweep_generic_kernel<64>, dim3(n_blocks), dim3(64), lds, s, P);
    } else if (nt == 1024) {
        hipLaunchKernelGGL(sweep_generic_kernel<1024>, dim3(n_blocks), dim3(1024), lds, s, P);
    } else if (nt == 512) {
        hipLaunchKernelGGL(sweep_generic_kernel<512>, dim3(n_blocks), dim3(512), lds, s, P);
    } else {
        hipLaunchKernelGGL(sweep_generic_kernel<256>, dim3(n_blocks), dim3(256), lds, s, P);
    }
    return hipGetLastError();
}

}  // namespace crbm
