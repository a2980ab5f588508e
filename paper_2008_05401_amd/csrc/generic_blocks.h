// generic_blocks.h -- workgroup-level building blocks on byte-per-unit
// lattices: FP64 and float32 pre-activations of single units, the FP64 CRBM
// free energy of a configuration and the Ising energy / magnetisation.
#pragma once
#include "device_common.h"

namespace crbm {

// FP64 hidden pre-activation of unit (k, i, j)
__device__ __forceinline__ double preact_hidden_d(const float* Ws, const float* hbs, const uint8_t* v, int K, int C,
                                                  int LW, int L, int k, int i, int j)
{
    (void)K;
    double acc = (double)hbs[k];
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < LW; ++a) {
            int ia = i + a;
            if (ia >= L) ia -= L;
            const uint8_t* row = v + (c * L + ia) * L;
            const float* wr = Ws + ((k * C + c) * LW + a) * LW;
            for (int b = 0; b < LW; ++b) {
                int jb = j + b;
                if (jb >= L) jb -= L;
                acc += (double)wr[b] * (double)row[jb];
            }
        }
    return acc;
}

__device__ __forceinline__ double preact_visible_d(const float* Ws, const float* vbs, const uint8_t* h, int K, int C,
                                                   int LW, int L, int c, int x, int y)
{
    double acc = (double)vbs[c];
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < LW; ++a) {
            int xa = x - a;
            if (xa < 0) xa += L;
            const uint8_t* row = h + (k * L + xa) * L;
            const float* wr = Ws + ((k * C + c) * LW + a) * LW;
            for (int b = 0; b < LW; ++b) {
                int yb = y - b;
                if (yb < 0) yb += L;
                acc += (double)wr[b] * (double)row[yb];
            }
        }
    return acc;
}

// float32 pre-activations (the fast path of the Bernoulli tests)
__device__ __forceinline__ float preact_hidden_f(const float* Ws, const float* hbs, const uint8_t* v, int C, int LW,
                                                 int L, int k, int i, int j)
{
    float acc = hbs[k];
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < LW; ++a) {
            int ia = i + a;
            if (ia >= L) ia -= L;
            const uint8_t* row = v + (c * L + ia) * L;
            const float* wr = Ws + ((k * C + c) * LW + a) * LW;
            for (int b = 0; b < LW; ++b) {
                int jb = j + b;
                if (jb >= L) jb -= L;
                acc = fmaf(wr[b], (float)row[jb], acc);
            }
        }
    return acc;
}

__device__ __forceinline__ float preact_visible_f(const float* Ws, const float* vbs, const uint8_t* h, int K, int C,
                                                  int LW, int L, int c, int x, int y)
{
    float acc = vbs[c];
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < LW; ++a) {
            int xa = x - a;
            if (xa < 0) xa += L;
            const uint8_t* row = h + (k * L + xa) * L;
            const float* wr = Ws + ((k * C + c) * LW + a) * LW;
            for (int b = 0; b < LW; ++b) {
                int yb = y - b;
                if (yb < 0) yb += L;
                acc = fmaf(wr[b], (float)row[yb], acc);
            }
        }
    return acc;
}

// F(v) in FP64 over the workgroup (all threads receive it)
__device__ inline double free_energy_block(const float* Ws, const float* hbs, const float* vbs, const uint8_t* v, int K,
                                    int C, int LW, int L, double* red)
{
    const int LL = L * L;
    double fl = 0.0;
    for (int q = threadIdx.x; q < K * LL; q += blockDim.x) {
        const int k = q / LL, r = q - k * LL, i = r / L, j = r - i * L;
        fl -= softplus_d(preact_hidden_d(Ws, hbs, v, K, C, LW, L, k, i, j));
    }
    for (int q = threadIdx.x; q < C * LL; q += blockDim.x) fl -= (double)vbs[q / LL] * (double)v[q];
    return block_sum(fl, red);
}

// Ising E/J and M of v (C = 1), over the workgroup
__device__ inline void ising_em_block(const uint8_t* v, int L, long long* red, long long& E, long long& M)
{
    long long el = 0, ml = 0;
    for (int q = threadIdx.x; q < L * L; q += blockDim.x) {
        const int i = q / L, j = q - i * L;
        const int s = 2 * (int)v[q] - 1;
        const int sd = 2 * (int)v[(i + 1 == L ? 0 : i + 1) * L + j] - 1;
        const int sr = 2 * (int)v[i * L + (j + 1 == L ? 0 : j + 1)] - 1;
        el -= s * (sd + sr);
        ml += s;
    }
    E = block_sum(el, red);
    M = block_sum(ml, red);
}

}  // namespace crbm
