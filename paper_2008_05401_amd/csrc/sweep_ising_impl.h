// sweep_ising_impl.h -- bit-packed fused propose+accept sweep for Ising jobs
// (C = 1) on gfx950: device code, instantiated by the sweep_ising_k*.hip units.
//
// Layout.  One workgroup owns one chain for the whole launch.  Every lattice
// plane (current state, two proposal buffers, K hidden planes) is kept in LDS
// with one bit per unit: row i of a plane is RS = max(L/32,1)+1 32-bit words,
// the last word repeating the first (rows with L < 32 hold the row pattern
// repeated across the word), so that the 32-bit window that starts at any
// column j0 < L is a funnel shift of two adjacent words.
//
// Work split.  A lane handles "quads" of four horizontally adjacent sites
// (i, 4m..4m+3); for hidden channel k that is exactly one Philox block
// (counter (((k L + i) L + 4m) >> 2, sweep, chain, tag)), so no random word is
// wasted.  Quads are dealt in row-major order, so the lanes that share a
// 32-bit row word are adjacent and their nibbles are OR-combined with lane
// shuffles before one lane stores the word.
//
// Arithmetic.  Because v and h are binary, each filter row a contributes a sum
// of a subset of its Lw taps; the 2^Lw subset sums are tabulated per (k, a)
// once per job at crbm_init (T1 for the visible->hidden correlation, T2 with
// the taps reversed for the hidden->visible adjoint; ising_tables_kernel) and
// copied into LDS at the start of every launch, so a pre-activation costs Lw
// table reads instead of Lw^2 multiply-adds.  Pre-activations are float32
// with rigorous error bounds; a Bernoulli test whose float32 value lies inside
// its bound is recomputed in FP64 from the bit planes.  F(x') is summed from
// float32 softplus terms (product form per site: sum_k max(a,0) +
// log prod_k (1 + e^{-|a|})) with a rigorous bound B'; the MH test is decided
// in float32/FP64 only when |log r - log u| exceeds the sum of the bounds of
// F(x') and F(x), otherwise both free energies are recomputed in FP64.
// E(x') and M(x') are XOR/popcount counts over row words (exact).
#pragma once
#include "device_common.h"
#include "sweep_common.h"
#include "sweep_ising.h"

namespace crbm {

namespace {

__device__ __forceinline__ uint32_t window32(const uint32_t* row, int j0)
{
    const int w = j0 >> 5;
    const uint64_t x = (uint64_t)row[w] | ((uint64_t)row[w + 1] << 32);
    return (uint32_t)(x >> (j0 & 31));
}

__device__ __forceinline__ int bit_at(const uint32_t* row, int c) { return (int)((row[c >> 5] >> (c & 31)) & 1u); }

// OR over groups of lpw = 2, 4 or 8 adjacent lanes, result valid in the
// group's first lane (quad permutations xor 1, xor 2, then row_shl:4)
__device__ __forceinline__ uint32_t group_or(uint32_t x, int lpw)
{
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
    if (lpw >= 4) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
    if (lpw >= 8) x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x104, 0xF, 0xF, false);
    return x;
}

// Combine the nibbles of the lanes that share one row word and store it
// (plus the wrap copy).  Must be called by every lane of the wave.
__device__ __forceinline__ void store_nibble(uint32_t* plane, int RS, int L, int i, int m, uint32_t nib, bool active)
{
    const int lpw = L >= 32 ? 8 : (L >> 2);
    uint32_t x = active ? (nib << (4 * (m & (lpw - 1)))) : 0u;
    x = group_or(x, lpw);
    if (active && (m & (lpw - 1)) == 0) {
        uint32_t val = x;
        if (L == 8) {
            val |= val << 8;
            val |= val << 16;
        } else if (L == 16) {
            val |= val << 16;
        }
        uint32_t* row = plane + i * RS;
        const int w = L >= 32 ? (m >> 3) : 0;
        row[w] = val;
        if (w == 0) row[RS - 1] = val;
    }
}

// Set or clear bit (i, c) of a plane, including its copies (wrap word, row
// pattern repeated across the word for L < 32); atomic so that concurrent
// fixes of neighbouring bits are safe.
__device__ __forceinline__ void put_bit(uint32_t* plane, int RS, int L, int i, int c, bool on)
{
    uint32_t* row = plane + i * RS;
    uint32_t mask;
    int w;
    if (L >= 32) {
        w = c >> 5;
        mask = 1u << (c & 31);
    } else {
        w = 0;
        mask = 0;
        for (int p = c; p < 32; p += L) mask |= 1u << p;
    }
    if (on) {
        atomicOr(row + w, mask);
        if (w == 0) atomicOr(row + RS - 1, mask);
    } else {
        atomicAnd(row + w, ~mask);
        if (w == 0) atomicAnd(row + RS - 1, ~mask);
    }
}

// four bits of row i, columns 4m..4m+3
__device__ __forceinline__ uint32_t quad_bits(const uint32_t* plane, int RS, int L, int i, int m)
{
    const uint32_t* row = plane + i * RS;
    const int w = L >= 32 ? (m >> 3) : 0;
    const int sh = L >= 32 ? 4 * (m & 7) : 4 * m;
    return (row[w] >> sh) & 15u;
}

// E/J = -2L^2 + 2 (unsatisfied bonds) and M = 2 (up spins) - L^2 of a plane
__device__ inline void ising_em_bits(const uint32_t* pl, int L, int RS, long long* red, long long& E, long long& M)
{
    const int lgw = L >= 32 ? (31 - __builtin_clz(L)) - 5 : 0;  // log2(words per row)
    const int nwr = 1 << lgw;
    const uint32_t mask = L >= 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
    long long unsat = 0, ones = 0;
    for (int t = threadIdx.x; t < L * nwr; t += blockDim.x) {
        const int i = t >> lgw, w = t & (nwr - 1);
        const uint32_t* row = pl + i * RS;
        const uint32_t* dn = pl + ((i + 1) & (L - 1)) * RS;
        const uint32_t x = row[w] & mask;
        const uint32_t right = window32(row, (w << 5) + 1) & mask;
        unsat += __popc(x ^ right) + __popc((x ^ dn[w]) & mask);
        ones += __popc(x);
    }
    const long long su = block_sum(unsat, red);
    const long long so = block_sum(ones, red);
    E = -2LL * L * L + 2LL * su;
    M = 2LL * so - (long long)L * L;
}

// ---------------------------------------------------------------------------
// FP64 exp and log for the exact paths inside the sweep loop, with every
// constant read from a small LDS table: nothing of them is then held in
// registers across the hot passes.  exp: Cody-Waite reduction x = k ln2 + r
// (ln2 split as in fdlibm so that k ln2_hi is exact), Taylor series of e^r to
// r^13 (|r| <= ln2/2, truncation < 1e-17).  log: x = 2^e m, m in [sqrt(1/2),
// sqrt(2)), log m = 2 atanh(s) with s = (m-1)/(m+1), series to s^23.
// ---------------------------------------------------------------------------
constexpr int NDC = ISING_NDC;
enum { DC_LN2HI = 0, DC_LN2LO = 1, DC_INVLN2 = 2, DC_FACT = 3, DC_ODD = 15, DC_SQRTH = 26 };

__device__ inline void fill_dconst(double* c)
{
    c[DC_LN2HI] = 6.93147180369123816490e-01;
    c[DC_LN2LO] = 1.90821492927058770002e-10;
    c[DC_INVLN2] = 1.44269504088896338700e+00;
    double f = 1.0;
    for (int n = 2; n <= 13; ++n) {
        f *= (double)n;
        c[DC_FACT + n - 2] = 1.0 / f;  // 1/n!
    }
    for (int n = 1; n <= 11; ++n) c[DC_ODD + n - 1] = 1.0 / (double)(2 * n + 1);
    c[DC_SQRTH] = 0.70710678118654752440;
}

__device__ __forceinline__ double exp_c(double x, const double* c)
{
    const double kd = rint(x * c[DC_INVLN2]);
    double r = fma(-kd, c[DC_LN2HI], x);
    r = fma(-kd, c[DC_LN2LO], r);
    double p = c[DC_FACT + 11];
#pragma unroll
    for (int n = 12; n >= 2; --n) p = fma(p, r, c[DC_FACT + n - 2]);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)kd);
}

// x > 0, finite
__device__ __forceinline__ double log_c(double x, const double* c)
{
    int e;
    double m = frexp(x, &e);
    if (m < c[DC_SQRTH]) {
        m *= 2.0;
        e -= 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double q = c[DC_ODD + 10];
#pragma unroll
    for (int n = 10; n >= 1; --n) q = fma(q, z, c[DC_ODD + n - 1]);
    const double lm = fma(2.0 * s, z * q, 2.0 * s);
    return fma((double)e, c[DC_LN2HI], fma((double)e, c[DC_LN2LO], lm));
}

// log(1 + y), y >= 0
__device__ __forceinline__ double log1p_c(double y, const double* c)
{
    const double u = 1.0 + y;
    if (u == 1.0) return y;
    return log_c(u, c) * (y / (u - 1.0));
}

__device__ __forceinline__ double softplus_c(double x, const double* c)
{
    return (x > 0.0 ? x : 0.0) + log1p_c(exp_c(-fabs(x), c), c);
}

// h = [u < sigmoid(a)], u = (x + 0.5) 2^-32, in FP64
__device__ __forceinline__ bool bernoulli_exact_c(double a, uint32_t x, const double* c)
{
    const double u = ((double)x + 0.5) * 0x1p-32;
    return u < 1.0 / (1.0 + exp_c(-a, c));
}

template <int LW>
__device__ __forceinline__ double preact_h_exact(const float* __restrict__ W, float hb, const uint32_t* pl, int RS,
                                                 int L, int k, int i, int j)
{
    double acc = (double)hb;
#pragma unroll
    for (int a = 0; a < LW; ++a) {
        int ia = i + a;
        if (ia >= L) ia -= L;
        const uint32_t* row = pl + ia * RS;
#pragma unroll
        for (int b = 0; b < LW; ++b) {
            int jb = j + b;
            if (jb >= L) jb -= L;
            if (bit_at(row, jb)) acc += (double)W[(k * LW + a) * LW + b];
        }
    }
    return acc;
}

template <int LW>
__device__ __forceinline__ double preact_v_exact(const float* __restrict__ W, float vb, const uint32_t* hpl, int PL,
                                                 int RS, int L, int K, int x, int y)
{
    double acc = (double)vb;
#pragma unroll 1
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int a = 0; a < LW; ++a) {
            int xa = x - a;
            if (xa < 0) xa += L;
            const uint32_t* row = hpl + k * PL + xa * RS;
#pragma unroll
            for (int b = 0; b < LW; ++b) {
                int yb = y - b;
                if (yb < 0) yb += L;
                if (bit_at(row, yb)) acc += (double)W[(k * LW + a) * LW + b];
            }
        }
    return acc;
}

// FP64 free energy of a bit plane, over the workgroup.  Wl and hbl are LDS
// copies of the filters and hidden biases; channel-major so that a channel's
// taps are read by every lane at the same address.
template <int LW>
__device__ double free_energy_exact(const float* Wl, const float* hbl, float vb, const uint32_t* pl, int RS, int L,
                                    int K, double* red, const double* dc, const double* T64)
{
    const int LL = L * L, lgL = 31 - __builtin_clz(L), Lm = L - 1;
    double f = 0.0;
    if (T64) {
        // FP64 subset sums of the filter rows: a = h_b + sum_a T64[k][a][window bits]; the
        // softplus terms of a site in product form, sum_k max(a, 0) + log prod_k (1 + e^{-|a|})
        // (each factor in (1, 2], so the product of K <= 64 of them stays in range)
        constexpr int NP = 1 << LW;
        for (int q = threadIdx.x; q < LL; q += blockDim.x) {
            const int i = q >> lgL, j = q & Lm;
            uint32_t wb[LW];
#pragma unroll
            for (int a = 0; a < LW; ++a) wb[a] = window32(pl + ((i + a) & Lm) * RS, j) & (NP - 1);
            double pos = 0.0, prod = 1.0;
            for (int k = 0; k < K; ++k) {
                const double* Tk = T64 + k * LW * NP;
                double acc = (double)hbl[k];
#pragma unroll
                for (int a = 0; a < LW; ++a) acc += Tk[a * NP + wb[a]];
                pos += acc > 0.0 ? acc : 0.0;
                prod *= 1.0 + exp_c(-fabs(acc), dc);
            }
            f -= pos + log_c(prod, dc);
            if (bit_at(pl + i * RS, j)) f -= (double)vb;
        }
        return block_sum(f, red);
    }
    for (int k = 0; k < K; ++k) {
        const float* Wk = Wl + k * LW * LW;
        const double hb = (double)hbl[k];
        for (int q = threadIdx.x; q < LL; q += blockDim.x) {
            const int i = q >> lgL, j = q & Lm;
            double acc = hb;
#pragma unroll
            for (int a = 0; a < LW; ++a) {
                const uint32_t w = window32(pl + ((i + a) & Lm) * RS, j);
#pragma unroll
                for (int b2 = 0; b2 < LW; ++b2)
                    if ((w >> b2) & 1u) acc += (double)Wk[a * LW + b2];
            }
            f -= softplus_c(acc, dc);
        }
    }
    for (int q = threadIdx.x; q < LL; q += blockDim.x) {
        const int i = q >> lgL, j = q & Lm;
        if (bit_at(pl + i * RS, j)) f -= (double)vb;
    }
    return block_sum(f, red);
}

// acc[s] = bias + sum_a T[off[a][s]] as a shallow tree: all LW reads are
// issued before the first add, so LDS latency is paid once per channel
template <int LW>
__device__ __forceinline__ void table_sums(const float* __restrict__ T, const uint32_t (&off)[LW][4], float bias,
                                           float (&acc)[4])
{
    float v[LW][4];
#pragma unroll
    for (int a = 0; a < LW; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) v[a][s] = T[off[a][s]];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float t = v[0][s];
#pragma unroll
        for (int a = 1; a + 1 < LW; a += 2) t += v[a][s] + v[a + 1][s];
        if ((LW & 1) == 0) t += v[LW - 1][s];
        acc[s] = bias + t;
    }
}

// acc[s] = bias + sum_a T[a NP + idx[b + a][s]] (visible-to-hidden, rows below)
template <int LW, int R>
__device__ __forceinline__ void table_sums_fwd(const float* __restrict__ T, const uint32_t (&idx)[R][4], int b,
                                               float bias, float (&acc)[4])
{
    constexpr int NP = 1 << LW;
    float v[LW][4];
#pragma unroll
    for (int a = 0; a < LW; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) v[a][s] = T[a * NP + idx[b + a][s]];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float t = v[0][s];
#pragma unroll
        for (int a = 1; a + 1 < LW; a += 2) t += v[a][s] + v[a + 1][s];
        if ((LW & 1) == 0) t += v[LW - 1][s];
        acc[s] = bias + t;
    }
}

// part[s] = sum_a T[a NP + idx[b - a + LW - 1][s]] (hidden-to-visible, rows above)
template <int LW, int R>
__device__ __forceinline__ void table_sums_adj(const float* __restrict__ T, const uint32_t (&idx)[R][4], int b,
                                               float (&part)[4])
{
    constexpr int NP = 1 << LW;
    float v[LW][4];
#pragma unroll
    for (int a = 0; a < LW; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) v[a][s] = T[a * NP + idx[b - a + LW - 1][s]];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float t = v[0][s];
#pragma unroll
        for (int a = 1; a + 1 < LW; a += 2) t += v[a][s] + v[a + 1][s];
        if ((LW & 1) == 0) t += v[LW - 1][s];
        part[s] = t;
    }
}

// e[s] = bias * prod_a T[a NP + idx[b + a][s]] (tree order)
template <int LW, int R>
__device__ __forceinline__ void table_prods_fwd(const float* __restrict__ T, const uint32_t (&idx)[R][4], int b,
                                                float bias, float (&e)[4])
{
    constexpr int NP = 1 << LW;
    float v[LW][4];
#pragma unroll
    for (int a = 0; a < LW; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) v[a][s] = T[a * NP + idx[b + a][s]];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float t = v[0][s];
#pragma unroll
        for (int a = 1; a + 1 < LW; a += 2) t *= v[a][s] * v[a + 1][s];
        if ((LW & 1) == 0) t *= v[LW - 1][s];
        e[s] = bias * t;
    }
}

// part[s] = prod_a T[a NP + idx[b - a + LW - 1][s]]
template <int LW, int R>
__device__ __forceinline__ void table_prods_adj(const float* __restrict__ T, const uint32_t (&idx)[R][4], int b,
                                                float (&part)[4])
{
    constexpr int NP = 1 << LW;
    float v[LW][4];
#pragma unroll
    for (int a = 0; a < LW; ++a)
#pragma unroll
        for (int s = 0; s < 4; ++s) v[a][s] = T[a * NP + idx[b - a + LW - 1][s]];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float t = v[0][s];
#pragma unroll
        for (int a = 1; a + 1 < LW; a += 2) t *= v[a][s] * v[a + 1][s];
        if ((LW & 1) == 0) t *= v[LW - 1][s];
        part[s] = t;
    }
}

template <bool B>
struct flag_c {
    static constexpr bool value = B;
};

}  // namespace

// KT > 0: the number of hidden channels is a compile-time constant (loops over
// channels unrolled, table offsets become instruction immediates); KT == 0:
// runtime K.  L is a power of two in {8, ..., 256}.
// filter loop unroll: full for a compile-time K with one row per lane (more spills)
template <int KT, int BH>
struct KUnroll {
    static constexpr int value = (KT > 0 && BH == 1) ? KT : 1;
};

template <int KT, int LW, int NT, int BH>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void sweep_ising_kernel(SweepLaunch P)
{
    constexpr int NP = 1 << LW;
    // unroll factor of the channel loops (unrolling with rows > 1 runs out of registers)
    extern __shared__ __align__(16) unsigned char smem[];
    int jb = 0;
    while (jb + 1 < P.n_jobs && (int)blockIdx.x >= P.block_begin[jb + 1]) ++jb;
    const JobDev& J = *P.jobs[jb];
    const int g = (int)blockIdx.x - P.block_begin[jb];
    if (g >= J.n_chains) return;

    const int K = KT > 0 ? KT : J.K;
    const int L = J.L;
    const int lgL = 31 - __builtin_clz(L);
    const int Lm = L - 1;
    const int RS = (L >= 32 ? (L >> 5) : 1) + 1;
    const int PL = L * RS;
    const int lgq = lgL - 2;  // quads per row = L/4
    const int nq = (L * L) >> 2;          // quads of 4 sites (state load/store)
    const int nb = nq / BH;               // blocks of BH x 4 sites (the passes)
    const int nrounds = (nq + NT - 1) / NT;
    const int nbrounds = (nb + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int tsz = K * LW * NP;

    // tables: additive mode T1, T2 (exp2 domain); product mode E1 = e^{-s},
    // E2 = e^{-s} of the reversed rows, E1p = e^{+s}
    float* T1 = (float*)smem;
    float* T2 = T1 + tsz;
    float* E1p = T2 + tsz;
    float* hbs = E1p + tsz;    // additive: -h_b log2(e)
    float* dAh = hbs + K;      // Bernoulli band per channel
    float* Sk = dAh + K;       // S_k = |h_b| + sum |W_k|
    float* dApre = Sk + K;     // bound on |a_f32 - a| (additive mode)
    float* ehbm = dApre + K;   // e^{-h_b}
    float* ehbp = ehbm + K;    // e^{+h_b}
    float* hbl = ehbp + K;     // h_b
    float* Wl = hbl + K;       // the filters, for the exact paths
    const IsingTabLayout tl = ising_tab_layout(K, LW);
    const IsingTabConst& TC = *(const IsingTabConst*)(smem + tl.off_const);
    double* red = (double*)(smem + tl.bytes);
    uint32_t* vpl = (uint32_t*)(red + 64);
    uint32_t* hpl = vpl + 3 * PL;
    // FP64 subset sums of the filter rows for the exact free energy, when small enough
    const double* T64 = ising_fast_t64(K, LW) ? (const double*)(smem + tl.off_t64) : nullptr;
    const double* sh_dc = TC.dc;
    __shared__ long long sh_t0;
    __shared__ int sh_flag;
    // units whose float32 Bernoulli test fell inside its error band
    constexpr int QCAP = 512;
    __shared__ uint32_t nearq[QCAP];
    __shared__ int sh_qn;
    __shared__ ChainRec R;
    __shared__ double sh_Bcur;
    constexpr int LU_CHUNK = 64;
    __shared__ double sh_lu[LU_CHUNK];
    __shared__ long long sh_Mcur;
    __shared__ int sh_cur, sh_rbm;
    __shared__ double sh_Bchain;

    // the job's tables (built once at crbm_init) into LDS, 16 bytes per lane and step
    {
        const uint4* __restrict__ src = (const uint4*)J.tab;
        uint4* dst = (uint4*)smem;
        for (int q = tid; q < tl.bytes / 16; q += NT) dst[q] = src[q];
    }
    __syncthreads();
    const bool mult = TC.mult != 0;
    const uint32_t gid = J.chain_offset + (uint32_t)g;
    const uint32_t k0 = (uint32_t)J.seed, k1 = (uint32_t)(J.seed >> 32);
    int8_t* state = J.state + (size_t)g * L * L;
    ChainRec* rec = J.rec + g;

    // +-1 int8 lattice <-> bit plane (4 int8 per lane; +1 = 0x01, -1 = 0xFF)
    auto load_plane = [&](const int8_t* src, uint32_t* pl) {
        for (int r = 0; r < nrounds; ++r) {
            const int Q = r * NT + tid;
            const bool active = Q < nq;
            const int i = active ? (Q >> lgq) : 0, m = active ? (Q & ((L >> 2) - 1)) : 0;
            uint32_t nib = 0;
            if (active) {
                const uint32_t w4 = ~*(const uint32_t*)(src + (i << lgL) + 4 * m);
                nib = ((w4 >> 7) & 1u) | ((w4 >> 14) & 2u) | ((w4 >> 21) & 4u) | ((w4 >> 28) & 8u);
            }
            store_nibble(pl, RS, L, i, m, nib, active);
        }
    };
    auto store_plane = [&](const uint32_t* pl, int8_t* dst) {
        for (int r = 0; r < nrounds; ++r) {
            const int Q = r * NT + tid;
            if (Q < nq) {
                const int i = Q >> lgq, m = Q & ((L >> 2) - 1);
                const uint32_t nib = quad_bits(pl, RS, L, i, m);
                const uint32_t up = (nib & 1u) | ((nib & 2u) << 7) | ((nib & 4u) << 14) | ((nib & 8u) << 21);
                const uint32_t dn =
                    ((~nib) & 1u) | (((~nib) & 2u) << 7) | (((~nib) & 4u) << 14) | (((~nib) & 8u) << 21);
                *(uint32_t*)(dst + (i << lgL) + 4 * m) = up | (dn * 0xFFu);
            }
        }
    };
    // physical state in plane 0; a persistent CRBM replica in plane 1
    const bool replica = J.rbm_state != nullptr;
    int8_t* rbm_state = replica ? J.rbm_state + (size_t)g * L * L : nullptr;
    load_plane(state, vpl);
    if (replica) load_plane(rbm_state, vpl + PL);
    if (tid == 0) {
        R = *rec;
        sh_t0 = R.sweeps;
        sh_Bcur = R.F_bound;
    }
    __syncthreads();
    {
        long long Ecur_d, Mcur;
        ising_em_bits(vpl, L, RS, (long long*)red, Ecur_d, Mcur);
        if (tid == 0) {
            sh_Mcur = Mcur;
            sh_cur = 0;
            sh_rbm = 1;
        }
    }
    const uint32_t t0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh_t0);
    // rigorous bound of the float32 free energy of the chain: the per-site bound of the
    // table block times L^2; product mode adds, per lane, the float log2 of a number in
    // [0.5, 1], whose rounding to float and log2 instruction stay below 2^-21 (natural
    // log units)
    if (tid == 0) sh_Bchain = TC.Bsite * (double)L * (double)L + (mult ? (double)NT * 0x1p-21 : 0.0);
    __syncthreads();

    // State that lives across the passes (current plane, M of the current state,
    // chain bound) stays in LDS: the passes use every vector register.
    for (int it = 0; it < P.n_sweeps; ++it) {
        const int cur = __builtin_amdgcn_readfirstlane(sh_cur);
        const uint32_t t = t0 + (uint32_t)it;
        // log of the MH uniforms of the next LU_CHUNK sweeps, one per lane
        if ((it & (LU_CHUNK - 1)) == 0) {
            if (tid < LU_CHUNK && it + tid < P.n_sweeps) sh_lu[tid] = log_c(mh_uniform(J.seed, t + (uint32_t)tid, gid), sh_dc);
            __syncthreads();
        }
        // the Gibbs chain starts from the replica (persistent) or the physical state
        int src = replica ? __builtin_amdgcn_readfirstlane(sh_rbm) : cur;
        for (int sub = 0; sub < J.gibbs_k; ++sub) {
            int dst = src == 2 ? 0 : src + 1;
            if (dst == cur) dst = dst == 2 ? 0 : dst + 1;
            const uint32_t* vs = vpl + src * PL;
            uint32_t* vd = vpl + dst * PL;
            const uint32_t tagh = STREAM_HID | ((uint32_t)sub << 8);
            const uint32_t tagv = STREAM_VIS | ((uint32_t)sub << 8);
            if (tid == 0) sh_qn = 0;
            __syncthreads();
            // ---- hidden pass: h ~ P(h | v); a lane owns BH rows x 4 columns
            auto hidden_pass = [&](auto MT) {
                constexpr bool MULT = decltype(MT)::value;
                for (int r = 0; r < nbrounds; ++r) {
                    const int Q = r * NT + tid;
                    const bool active = Q < nb;
                    const int i0 = active ? (Q >> lgq) * BH : 0, m = active ? (Q & ((L >> 2) - 1)) : 0;
                    const int j0 = 4 * m;
                    uint32_t idx[BH + LW - 1][4];
#pragma unroll
                    for (int r2 = 0; r2 < BH + LW - 1; ++r2) {
                        const uint32_t w = window32(vs + ((i0 + r2) & Lm) * RS, j0);
#pragma unroll
                        for (int s = 0; s < 4; ++s) idx[r2][s] = (w >> s) & (NP - 1);
                    }
#pragma unroll KUnroll<KT, BH>::value
                    for (int k = 0; k < K; ++k) {
                        const float dk = dAh[k];
#pragma unroll
                        for (int b = 0; b < BH; ++b) {
                            const int i = i0 + b;
                            // e[s] = e^{-a} of the four units
                            float e[4];
                            if constexpr (MULT) {
                                table_prods_fwd<LW>(T1 + k * LW * NP, idx, b, ehbm[k], e);
                            } else {
                                float z[4];
                                table_sums_fwd<LW>(T1 + k * LW * NP, idx, b, hbs[k], z);
#pragma unroll
                                for (int s = 0; s < 4; ++s) e[s] = __builtin_amdgcn_exp2f(z[s]);
                            }
                            const u32x4 rn =
                                philox10_uk((uint32_t)((((k << lgL) + i) << lgL) + j0) >> 2, t, gid, tagh, k0, k1);
                            uint32_t nib = 0, nearb = 0;
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                const float u = fmaf((float)word_of(rn, s), 0x1p-32f, 0x1p-33f);
                                const float tt = fmaf(u, e[s], u - 1.0f);
                                nib |= (uint32_t)(tt < 0.0f) << s;
                                nearb |= (uint32_t)(fabsf(tt) <= dk) << s;
                            }
                            if (nearb != 0 && active) {
                                for (int s = 0; s < 4; ++s)
                                    if ((nearb >> s) & 1) {
                                        const int pos = atomicAdd(&sh_qn, 1);
                                        if (pos < QCAP)
                                            nearq[pos] = ((uint32_t)((k << lgL) + i) << lgL) + (uint32_t)(j0 + s);
                                    }
                            }
                            store_nibble(hpl + k * PL, RS, L, i, m, nib, active);
                        }
                        // keep the scheduler from hoisting the next channel's table reads
                        if (BH > 1) __builtin_amdgcn_sched_barrier(0);
                    }
                }
            };
            if (mult) hidden_pass(flag_c<true>{});
            else hidden_pass(flag_c<false>{});
            __syncthreads();
            {
                // FP64 decisions of the queued hidden units (exact-mode rescan on overflow)
                const int n = __builtin_amdgcn_readfirstlane(sh_qn);
                if (n > 0) {
                    if (n <= QCAP) {
                        for (int e = tid; e < n; e += NT) {
                            const uint32_t q = nearq[e];
                            const int k = (int)(q >> (2 * lgL)), i = (int)(q >> lgL) & Lm, j = (int)q & Lm;
                            const u32x4 rn = philox10_uk(q >> 2, t, gid, tagh, k0, k1);
                            const bool on =
                                bernoulli_exact_c(preact_h_exact<LW>(Wl, hbl[k], vs, RS, L, k, i, j), word_of(rn, j & 3), sh_dc);
                            put_bit(hpl + k * PL, RS, L, i, j, on);
                        }
                    } else {
                        for (int q = tid; q < (K << (2 * lgL)); q += NT) {
                            const int k = q >> (2 * lgL), i = (q >> lgL) & Lm, j = q & Lm;
                            const u32x4 rn = philox10_uk((uint32_t)q >> 2, t, gid, tagh, k0, k1);
                            const bool on =
                                bernoulli_exact_c(preact_h_exact<LW>(Wl, hbl[k], vs, RS, L, k, i, j), word_of(rn, j & 3), sh_dc);
                            put_bit(hpl + k * PL, RS, L, i, j, on);
                        }
                    }
                    if (tid == 0) R.n_recheck += n;
                    __syncthreads();
                    if (tid == 0) sh_qn = 0;
                    __syncthreads();
                }
            }
            // ---- visible pass: v' ~ P(v | h)
            auto visible_pass = [&](auto MT) {
                constexpr bool MULT = decltype(MT)::value;
                const float vb = TC.vb, evbm = TC.evbm, dAv = TC.dAv;
                for (int r = 0; r < nbrounds; ++r) {
                    const int Q = r * NT + tid;
                    const bool active = Q < nb;
                    const int x0 = active ? (Q >> lgq) * BH : 0, m = active ? (Q & ((L >> 2) - 1)) : 0;
                    const int y0 = 4 * m;
                    const int jst = (y0 - (LW - 1)) & Lm;
                    // additive: z = -b log2(e); product: e = e^{-b}
                    float acc[BH][4];
#pragma unroll
                    for (int b = 0; b < BH; ++b)
#pragma unroll
                        for (int s = 0; s < 4; ++s) acc[b][s] = MULT ? evbm : vb;
#pragma unroll KUnroll<KT, BH>::value
                    for (int k = 0; k < K; ++k) {
                        const uint32_t* hk = hpl + k * PL;
                        uint32_t idx[BH + LW - 1][4];
#pragma unroll
                        for (int r2 = 0; r2 < BH + LW - 1; ++r2) {
                            const uint32_t w = window32(hk + ((x0 - (LW - 1) + r2) & Lm) * RS, jst);
#pragma unroll
                            for (int s = 0; s < 4; ++s) idx[r2][s] = (w >> s) & (NP - 1);
                        }
#pragma unroll
                        for (int b = 0; b < BH; ++b) {
                            float part[4];
                            if constexpr (MULT) {
                                table_prods_adj<LW>(T2 + k * LW * NP, idx, b, part);
#pragma unroll
                                for (int s = 0; s < 4; ++s) acc[b][s] *= part[s];
                            } else {
                                table_sums_adj<LW>(T2 + k * LW * NP, idx, b, part);
#pragma unroll
                                for (int s = 0; s < 4; ++s) acc[b][s] += part[s];
                            }
                        }
                        if (BH > 1) __builtin_amdgcn_sched_barrier(0);
                    }
#pragma unroll
                    for (int b = 0; b < BH; ++b) {
                        const int x = x0 + b;
                        const u32x4 rn = philox10_uk((uint32_t)((x << lgL) + y0) >> 2, t, gid, tagv, k0, k1);
                        uint32_t nib = 0, nearb = 0;
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const float u = fmaf((float)word_of(rn, s), 0x1p-32f, 0x1p-33f);
                            const float e = MULT ? acc[b][s] : __builtin_amdgcn_exp2f(acc[b][s]);
                            const float tt = fmaf(u, e, u - 1.0f);
                            nib |= (uint32_t)(tt < 0.0f) << s;
                            nearb |= (uint32_t)(fabsf(tt) <= dAv) << s;
                        }
                        if (nearb != 0 && active) {
                            for (int s = 0; s < 4; ++s)
                                if ((nearb >> s) & 1) {
                                    const int pos = atomicAdd(&sh_qn, 1);
                                    if (pos < QCAP) nearq[pos] = ((uint32_t)x << lgL) + (uint32_t)(y0 + s);
                                }
                        }
                        store_nibble(vd, RS, L, x, m, nib, active);
                    }
                }
            };
            if (mult) visible_pass(flag_c<true>{});
            else visible_pass(flag_c<false>{});
            __syncthreads();
            {
                const int n = __builtin_amdgcn_readfirstlane(sh_qn);
                if (n > 0) {
                    if (n <= QCAP) {
                        for (int e = tid; e < n; e += NT) {
                            const uint32_t q = nearq[e];
                            const int x = (int)(q >> lgL), y = (int)q & Lm;
                            const u32x4 rn = philox10_uk(q >> 2, t, gid, tagv, k0, k1);
                            const bool on =
                                bernoulli_exact_c(preact_v_exact<LW>(Wl, TC.vb_raw, hpl, PL, RS, L, K, x, y), word_of(rn, y & 3), sh_dc);
                            put_bit(vd, RS, L, x, y, on);
                        }
                    } else {
                        for (int q = tid; q < (1 << (2 * lgL)); q += NT) {
                            const int x = q >> lgL, y = q & Lm;
                            const u32x4 rn = philox10_uk((uint32_t)q >> 2, t, gid, tagv, k0, k1);
                            const bool on =
                                bernoulli_exact_c(preact_v_exact<LW>(Wl, TC.vb_raw, hpl, PL, RS, L, K, x, y), word_of(rn, y & 3), sh_dc);
                            put_bit(vd, RS, L, x, y, on);
                        }
                    }
                    if (tid == 0) R.n_recheck += n;
                    __syncthreads();
                }
            }
            src = dst;
        }
        // ---- F(x') with its error bound, E(x'), M(x')
        const uint32_t* vp = vpl + src * PL;
        // per-lane share of -sum softplus(a') over the lane's sites
        auto fe_pass = [&](auto MT) -> double {
            constexpr bool MULT = decltype(MT)::value;
            double Floc = 0.0;
            double D = 1.0;  // product mode: prod over sites of prod_k (1 + e^{a_k}), renormalised
            int Dexp = 0;
            for (int r = 0; r < nbrounds; ++r) {
                const int Q = r * NT + tid;
                const bool active = Q < nb;
                const int i0 = active ? (Q >> lgq) * BH : 0, m = active ? (Q & ((L >> 2) - 1)) : 0;
                const int j0 = 4 * m;
                uint32_t idx[BH + LW - 1][4];
#pragma unroll
                for (int r2 = 0; r2 < BH + LW - 1; ++r2) {
                    const uint32_t w = window32(vp + ((i0 + r2) & Lm) * RS, j0);
#pragma unroll
                    for (int s = 0; s < 4; ++s) idx[r2][s] = (w >> s) & (NP - 1);
                }
                // additive: softplus(a)/ln 2 = max(z', 0) + log2(1 + 2^{-|z'|}), z' = a log2(e)
                float msum[BH][4], prod[BH][4];
#pragma unroll
                for (int b = 0; b < BH; ++b)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        msum[b][s] = 0.f;
                        prod[b][s] = 1.f;
                    }
#pragma unroll KUnroll<KT, BH>::value
                for (int k = 0; k < K; ++k) {
#pragma unroll
                    for (int b = 0; b < BH; ++b) {
                        if constexpr (MULT) {
                            float e[4];
                            table_prods_fwd<LW>(E1p + k * LW * NP, idx, b, ehbp[k], e);
#pragma unroll
                            for (int s = 0; s < 4; ++s) prod[b][s] = fmaf(prod[b][s], e[s], prod[b][s]);
                        } else {
                            float acc[4];
                            table_sums_fwd<LW>(T1 + k * LW * NP, idx, b, hbs[k], acc);
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                msum[b][s] += fmaxf(-acc[s], 0.f);
                                prod[b][s] = fmaf(prod[b][s], __builtin_amdgcn_exp2f(-fabsf(acc[s])), prod[b][s]);
                            }
                        }
                    }
                    if (BH > 1) __builtin_amdgcn_sched_barrier(0);
                }
                if (active) {
                    if constexpr (MULT) {
#pragma unroll
                        for (int b = 0; b < BH; ++b) {
                            double q = (double)prod[b][0] * (double)prod[b][1];
                            q *= (double)prod[b][2] * (double)prod[b][3];
                            int ex;
                            D = frexp(D * q, &ex);
                            Dexp += ex;
                        }
                    } else {
                        float fs = 0.f;
#pragma unroll
                        for (int b = 0; b < BH; ++b)
#pragma unroll
                            for (int s = 0; s < 4; ++s) fs += msum[b][s] + __builtin_amdgcn_logf(prod[b][s]);
                        Floc -= (double)fs * 0.693147180559945309;
                    }
                }
            }
            // D in [0.5, 1]: float log2 of it, error counted in the chain bound
            if constexpr (MULT)
                Floc = -((double)__builtin_amdgcn_logf((float)D) + (double)Dexp) * 0.693147180559945309;
            return Floc;
        };
        const double Floc = mult ? fe_pass(flag_c<true>{}) : fe_pass(flag_c<false>{});
        const double Fsp = block_sum(Floc, red);
        const double Bp = sh_Bchain + 1e-13 * fabs(Fsp);
        long long Ep, Mp;
        ising_em_bits(vp, L, RS, (long long*)red, Ep, Mp);
        const long long ones = (Mp + (long long)L * L) / 2;
        const double Fp = Fsp - (double)TC.vb_raw * (double)ones;
        double lu = 0.0;
        if (tid == 0) {
            const double logr = -(1.0 / J.T[g]) * J.J0 * (double)(Ep - R.E) + (Fp - R.F);
            lu = sh_lu[it & (LU_CHUNK - 1)];
            const double band =
                fmax(Bp + sh_Bcur + 1e-12 * (1.0 + fabs(logr) + fabs(Fp) + fabs(R.F)), J.mh_band_min);
            sh_flag = J.target == 2 ? 1 : ((fabs(logr - lu) > band) ? (lu < logr ? 1 : 0) : 2);
        }
        __syncthreads();
        int flag = __builtin_amdgcn_readfirstlane(sh_flag);
        double Fnew = Fp, Bnew = Bp, Fold = 0.0;
        if (flag == 2) {
            // inside the float32 band: decide with FP64 free energies of both states
            Fnew = free_energy_exact<LW>(Wl, hbl, TC.vb_raw, vp, RS, L, K, red, sh_dc, T64);
            // the cached F of the current state is already exact after an earlier re-check
            Fold = sh_Bcur > 0.0 ? free_energy_exact<LW>(Wl, hbl, TC.vb_raw, vpl + cur * PL, RS, L, K, red, sh_dc, T64)
                                 : R.F;
            Bnew = 0.0;
            if (tid == 0) {
                const double logr = -(1.0 / J.T[g]) * J.J0 * (double)(Ep - R.E) + (Fnew - Fold);
                sh_flag = lu < logr ? 1 : 0;
                R.F = Fold;
                sh_Bcur = 0.0;
                R.n_recheck += 1;
            }
            __syncthreads();
            flag = __builtin_amdgcn_readfirstlane(sh_flag);
        }
        if (tid == 0) {
            if (flag) {
                R.F = Fnew;
                sh_Bcur = Bnew;
                R.E = Ep;
                R.n_acc += 1;
            }
            R.sweeps += 1;
            if (J.trace) J.trace[(size_t)g * J.trace_len + t % (uint32_t)J.trace_len] = (double)R.E;
            if ((long long)t >= (long long)J.burnin) {
                const long long mm = flag ? Mp : sh_Mcur;
                R.n_meas += 1;
                R.sumE += R.E;
                R.sumE2 += R.E * R.E;
                R.sumM += mm;
                R.sumAbsM += mm < 0 ? -mm : mm;
                R.sumM2 += mm * mm;
            }
        }
        if (tid == 0) {
            // exchange: accepted -> x <- y', y <- x; rejected -> y <- y'
            if (flag) {
                sh_cur = src;
                sh_Mcur = Mp;
                sh_rbm = cur;
            } else {
                sh_rbm = src;
            }
        }
        __syncthreads();
    }
    // End of the launch.  The chain's pointers are derived again from the kernel
    // argument through an opaque copy of the job index, so that none of them is
    // held in registers across the sweep loop.
    int jbe = jb;
    asm volatile("" : "+s"(jbe));
    const JobDev& Je = *P.jobs[jbe];
    const int ge = (int)blockIdx.x - P.block_begin[jbe];
    store_plane(vpl + __builtin_amdgcn_readfirstlane(sh_cur) * PL, Je.state + (size_t)ge * L * L);
    if (Je.rbm_state)
        store_plane(vpl + __builtin_amdgcn_readfirstlane(sh_rbm) * PL, Je.rbm_state + (size_t)ge * L * L);
    if (tid == 0) {
        R.F_bound = sh_Bcur;
        Je.rec[ge] = R;
    }
}


}  // namespace crbm
