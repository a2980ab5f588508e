// generic_blocks.h -- workgroup-level building blocks on byte-per-unit
// lattices: FP64 and float32 pre-activations of single units, the FP64 CRBM
// free energy of a configuration and the Ising energy / magnetisation.
//
// The convolutional layer is either the periodic CRBM (one filter bank; the
// window wraps in both directions) or the locally connected CRBM of Sec. IV.B:
// banks [1 + 2 ne][K][C][LW][LW] and hidden biases [1 + 2 ne][K], bank 0 shared
// by the bulk, banks 1..ne owned by the hidden columns 0..ne-1 and banks
// ne+1..2ne by the columns L-ne..L-1; with `open` the window stops at the
// column edge (columns past it count as v = 0) while rows stay periodic.
//
// With `dense` the layer is the fully connected RBM of the Sec. IV
// comparison: K hidden units, each connected to all nv = C L^2 visible units,
// W[K][nv] held in LDS with row stride nv + 1 (so that the lanes of a wave,
// one hidden unit each, hit distinct banks), hbias[K], vbias[nv].
#pragma once
#include "device_common.h"

namespace crbm {

struct ConvGeo {
    int K, C, LW, L, open, ne, dense;
    // filter bank of hidden column j
    __device__ __forceinline__ int bank(int j) const
    {
        return j < ne ? 1 + j : (j >= L - ne ? 1 + ne + (j - (L - ne)) : 0);
    }
    __device__ __forceinline__ int bank_size() const { return K * C * LW * LW; }
};

// Offsets b of the window that stay inside the lattice: all LW when the
// columns wrap; with open columns the hidden window j..j+LW-1 ends at L-1 and
// the visible unit y is reached from hidden columns y-b >= 0.  Loop bounds
// instead of in-loop exits keep the inner loops branch-free.
__device__ __forceinline__ int hidden_taps(const ConvGeo& G, int j) { return G.open ? min(G.LW, G.L - j) : G.LW; }
__device__ __forceinline__ int visible_taps(const ConvGeo& G, int y) { return G.open ? min(G.LW, y + 1) : G.LW; }

// The same pre-activations with the channel count and filter width known at
// compile time (periodic layer, one bank): every tap of a unit is unrolled, so
// its LDS loads issue together instead of one per loop trip.  The summation
// order is that of the general versions, so the results are identical.
template <typename T, int C_, int LW_>
__device__ __forceinline__ T preact_hidden_t(const float* Ws, const float* hbs, const uint8_t* v, int L, int k, int i,
                                             int j)
{
    T acc = (T)hbs[k];
#pragma unroll
    for (int c = 0; c < C_; ++c)
#pragma unroll
        for (int a = 0; a < LW_; ++a) {
            int ia = i + a;
            if (ia >= L) ia -= L;
            const uint8_t* row = v + (c * L + ia) * L;
            const float* wr = Ws + ((k * C_ + c) * LW_ + a) * LW_;
#pragma unroll
            for (int b = 0; b < LW_; ++b) {
                int jb = j + b;
                if (jb >= L) jb -= L;
                if constexpr (sizeof(T) == 4)
                    acc = fmaf(wr[b], (float)row[jb], acc);
                else
                    acc += (double)wr[b] * (double)row[jb];
            }
        }
    return acc;
}

template <typename T, int C_, int LW_>
__device__ __forceinline__ T preact_visible_t(const float* Ws, const float* vbs, const uint8_t* h, int K, int L, int c,
                                              int x, int y)
{
    T acc = (T)vbs[c];
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int a = 0; a < LW_; ++a) {
            int xa = x - a;
            if (xa < 0) xa += L;
            const uint8_t* row = h + (k * L + xa) * L;
            const float* wr = Ws + ((k * C_ + c) * LW_ + a) * LW_;
#pragma unroll
            for (int b = 0; b < LW_; ++b) {
                int yb = y - b;
                if (yb < 0) yb += L;
                if constexpr (sizeof(T) == 4)
                    acc = fmaf(wr[b], (float)row[yb], acc);
                else
                    acc += (double)wr[b] * (double)row[yb];
            }
        }
    return acc;
}

// layers with a compiled form: periodic, one bank, C in {1, 3}, 3 x 3 filters
__device__ __forceinline__ int compiled_form(const ConvGeo& G)
{
    if (G.open || G.ne != 0 || G.dense || G.LW != 3) return 0;
    return G.C == 3 ? 3 : (G.C == 1 ? 1 : 0);
}


// FP64 hidden pre-activation of unit (k, i, j)
__device__ __forceinline__ double preact_hidden_d(const float* Ws, const float* hbs, const uint8_t* v,
                                                  const ConvGeo& G, int k, int i, int j)
{
    switch (compiled_form(G)) {
    case 3: return preact_hidden_t<double, 3, 3>(Ws, hbs, v, G.L, k, i, j);
    case 1: return preact_hidden_t<double, 1, 3>(Ws, hbs, v, G.L, k, i, j);
    default: break;
    }
    const int C = G.C, LW = G.LW, L = G.L, nb = hidden_taps(G, j);
    const int bk = G.bank(j);
    const float* Wb = Ws + (size_t)bk * G.bank_size();
    double acc = (double)hbs[bk * G.K + k];
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < LW; ++a) {
            int ia = i + a;
            if (ia >= L) ia -= L;
            const uint8_t* row = v + (c * L + ia) * L;
            const float* wr = Wb + ((k * C + c) * LW + a) * LW;
            for (int b = 0; b < nb; ++b) {
                int jb = j + b;
                if (jb >= L) jb -= L;
                acc += (double)wr[b] * (double)row[jb];
            }
        }
    return acc;
}

// FP64 visible pre-activation of unit (c, x, y): every hidden unit it sees
// brings the filter bank of its own column
__device__ __forceinline__ double preact_visible_d(const float* Ws, const float* vbs, const uint8_t* h,
                                                   const ConvGeo& G, int c, int x, int y)
{
    switch (compiled_form(G)) {
    case 3: return preact_visible_t<double, 3, 3>(Ws, vbs, h, G.K, G.L, c, x, y);
    case 1: return preact_visible_t<double, 1, 3>(Ws, vbs, h, G.K, G.L, c, x, y);
    default: break;
    }
    const int K = G.K, C = G.C, LW = G.LW, L = G.L, nb = visible_taps(G, y);
    double acc = (double)vbs[c];
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < LW; ++a) {
            int xa = x - a;
            if (xa < 0) xa += L;
            const uint8_t* row = h + (k * L + xa) * L;
            const float* wr = Ws + ((k * C + c) * LW + a) * LW;
            if (G.ne == 0) {
                for (int b = 0; b < nb; ++b) {
                    int yb = y - b;
                    if (yb < 0) yb += L;
                    acc += (double)wr[b] * (double)row[yb];
                }
            } else {
                for (int b = 0; b < nb; ++b) {
                    int yb = y - b;
                    if (yb < 0) yb += L;
                    acc += (double)wr[(size_t)G.bank(yb) * G.bank_size() + b] * (double)row[yb];
                }
            }
        }
    return acc;
}

// float32 pre-activations (the fast path of the Bernoulli tests)
__device__ __forceinline__ float preact_hidden_f(const float* Ws, const float* hbs, const uint8_t* v, const ConvGeo& G,
                                                 int k, int i, int j)
{
    switch (compiled_form(G)) {
    case 3: return preact_hidden_t<float, 3, 3>(Ws, hbs, v, G.L, k, i, j);
    case 1: return preact_hidden_t<float, 1, 3>(Ws, hbs, v, G.L, k, i, j);
    default: break;
    }
    const int C = G.C, LW = G.LW, L = G.L, nb = hidden_taps(G, j);
    const int bk = G.bank(j);
    const float* Wb = Ws + (size_t)bk * G.bank_size();
    float acc = hbs[bk * G.K + k];
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < LW; ++a) {
            int ia = i + a;
            if (ia >= L) ia -= L;
            const uint8_t* row = v + (c * L + ia) * L;
            const float* wr = Wb + ((k * C + c) * LW + a) * LW;
            for (int b = 0; b < nb; ++b) {
                int jb = j + b;
                if (jb >= L) jb -= L;
                acc = fmaf(wr[b], (float)row[jb], acc);
            }
        }
    return acc;
}

__device__ __forceinline__ float preact_visible_f(const float* Ws, const float* vbs, const uint8_t* h, const ConvGeo& G,
                                                  int c, int x, int y)
{
    switch (compiled_form(G)) {
    case 3: return preact_visible_t<float, 3, 3>(Ws, vbs, h, G.K, G.L, c, x, y);
    case 1: return preact_visible_t<float, 1, 3>(Ws, vbs, h, G.K, G.L, c, x, y);
    default: break;
    }
    const int K = G.K, C = G.C, LW = G.LW, L = G.L, nb = visible_taps(G, y);
    float acc = vbs[c];
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < LW; ++a) {
            int xa = x - a;
            if (xa < 0) xa += L;
            const uint8_t* row = h + (k * L + xa) * L;
            const float* wr = Ws + ((k * C + c) * LW + a) * LW;
            if (G.ne == 0) {
                for (int b = 0; b < nb; ++b) {
                    int yb = y - b;
                    if (yb < 0) yb += L;
                    acc = fmaf(wr[b], (float)row[yb], acc);
                }
            } else {
                for (int b = 0; b < nb; ++b) {
                    int yb = y - b;
                    if (yb < 0) yb += L;
                    acc = fmaf(wr[(size_t)G.bank(yb) * G.bank_size() + b], (float)row[yb], acc);
                }
            }
        }
    return acc;
}

// ---- fully connected layer (W in LDS with row stride nv + 1)
__device__ __forceinline__ float dense_hidden_f(const float* Ws, const float* hbs, const uint8_t* v, int nv, int k)
{
    const float* w = Ws + (size_t)k * (nv + 1);
    float acc = hbs[k];
    for (int q = 0; q < nv; ++q) acc = fmaf(w[q], (float)v[q], acc);
    return acc;
}

__device__ __forceinline__ double dense_hidden_d(const float* Ws, const float* hbs, const uint8_t* v, int nv, int k)
{
    const float* w = Ws + (size_t)k * (nv + 1);
    double acc = (double)hbs[k];
    for (int q = 0; q < nv; ++q) acc += (double)w[q] * (double)v[q];
    return acc;
}

__device__ __forceinline__ float dense_visible_f(const float* Ws, const float* vbs, const uint8_t* h, int K, int nv,
                                                 int q)
{
    float acc = vbs[q];
    for (int k = 0; k < K; ++k) acc = fmaf(Ws[(size_t)k * (nv + 1) + q], (float)h[k], acc);
    return acc;
}

__device__ __forceinline__ double dense_visible_d(const float* Ws, const float* vbs, const uint8_t* h, int K, int nv,
                                                  int q)
{
    double acc = (double)vbs[q];
    for (int k = 0; k < K; ++k) acc += (double)Ws[(size_t)k * (nv + 1) + q] * (double)h[k];
    return acc;
}

// F(v) in FP64: thread t of nt adds its share of the terms (free_energy_part);
// free_energy_block sums the shares over the workgroup (all threads receive F)
__device__ inline double free_energy_part(const float* Ws, const float* hbs, const float* vbs, const uint8_t* v,
                                          const ConvGeo& G, int t, int nt)
{
    const int L = G.L, LL = L * L;
    double fl = 0.0;
    if (G.dense) {
        const int nv = G.C * LL;
        for (int k = t; k < G.K; k += nt) fl -= softplus_d(dense_hidden_d(Ws, hbs, v, nv, k));
        for (int q = t; q < nv; q += nt) fl -= (double)vbs[q] * (double)v[q];
        return fl;
    }
    if (LL >= nt) {
        // a lane per site: the K softplus terms in product form, sum_k max(a, 0) +
        // log prod_k (1 + e^{-|a|}), one log per site (each factor in (1, 2], K <= 64)
        for (int r = t; r < LL; r += nt) {
            const int i = r / L, j = r - i * L;
            double pos = 0.0, prod = 1.0;
            for (int k = 0; k < G.K; ++k) {
                const double a = preact_hidden_d(Ws, hbs, v, G, k, i, j);
                pos += a > 0.0 ? a : 0.0;
                prod *= 1.0 + exp(-fabs(a));
            }
            fl -= pos + log(prod);
        }
    } else {
        for (int q = t; q < G.K * LL; q += nt) {
            const int k = q / LL, r = q - k * LL, i = r / L, j = r - i * L;
            fl -= softplus_d(preact_hidden_d(Ws, hbs, v, G, k, i, j));
        }
    }
    for (int q = t; q < G.C * LL; q += nt) fl -= (double)vbs[q / LL] * (double)v[q];
    return fl;
}

__device__ inline double free_energy_block(const float* Ws, const float* hbs, const float* vbs, const uint8_t* v,
                                           const ConvGeo& G, double* red)
{
    return block_sum(free_energy_part(Ws, hbs, vbs, v, G, (int)threadIdx.x, (int)blockDim.x), red);
}

// Ising E/J and M of v (C = 1), over the workgroup; with open_cols the bond
// from column L-1 to column 0 is absent
__device__ inline void ising_em_block(const uint8_t* v, int L, int open_cols, long long* red, long long& E,
                                      long long& M)
{
    long long el = 0, ml = 0;
    for (int q = threadIdx.x; q < L * L; q += blockDim.x) {
        const int i = q / L, j = q - i * L;
        const int s = 2 * (int)v[q] - 1;
        const int sd = 2 * (int)v[(i + 1 == L ? 0 : i + 1) * L + j] - 1;
        const int sr = (open_cols && j + 1 == L) ? 0 : 2 * (int)v[i * L + (j + 1 == L ? 0 : j + 1)] - 1;
        el -= s * (sd + sr);
        ml += s;
    }
    E = block_sum(el, red);
    M = block_sum(ml, red);
}

}  // namespace crbm
