/*
 * crbm_oracle.c -- plain FP64 CPU oracle for convolutional-RBM-aided Monte
 * Carlo (Alcalde Puente & Eremin, "Convolutional restricted Boltzmann
 * machine aided Monte Carlo: an application to Ising and Kitaev models",
 * arXiv:2008.05401).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library. The GPU product path
 * shares no code with it: no headers, no helpers, no tables.
 *
 * Every routine is the plain definition written out, in double precision,
 * in the order the paper states it; there is no blocking, fusion or
 * reordering.  Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).
 *
 * Conventions (readings of the paper where it is silent; each one is also
 * listed with its reason in the design notes of the repository):
 *   - states at the boundary are +-1 int8, layout [chain][C][L][L];
 *     the RBM works on v = (s+1)/2 (App. A, first paragraph).
 *   - the "wrap around convolution" of Eq. (energy_CRBM) is taken as a
 *     cross-correlation with the filter anchored at its top-left element:
 *       a[k][i][j] = hb[k] + sum_{c,a,b} W[k][c][a][b] v[c][(i+a)%L][(j+b)%L]
 *     and the hidden->visible pass is its exact adjoint:
 *       b[c][x][y] = vb[c] + sum_{k,a,b} W[k][c][a][b] h[k][(x-a)%L][(y-b)%L].
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11),
 *     key = (seed lo, seed hi), counter = (unit>>2, sweep, chain, tag),
 *     word = unit & 3; tag = stream | substep<<8 with streams
 *     INIT=0, HID=1, VIS=2, MH=3.  Bernoulli: x -> u = (x+0.5)/2^32,
 *     unit on iff u < sigma(pre-activation).  MH: 53-bit uniform from
 *     words 0,1 of unit group 0.  INIT: s=+1 iff the top bit of the word is set.
 *   - the MH step uses the Gibbs kernel as proposal; because the Gibbs kernel
 *     is reversible with respect to exp(-F) (App. B, Gibbs sampling), the
 *     acceptance ratio of Eq. (acceptance) with one replica being the CRBM
 *     reduces to  log r = log P(x') - log P(x) + F(x') - F(x).
 *     Two forms: the CRBM replica refreshed from the physical state before
 *     every sweep, or a persistent CRBM replica y that the Gibbs steps advance
 *     and that is exchanged with the physical state x (App. B, parallel
 *     tempering with an exchange correction): accepted -> x <- y', y <- x.
 *   - open boundaries (Sec. IV.B): the target drops the bonds from column
 *     L-1 to column 0 (Ising: that nearest-neighbour bond; Kitaev: the x bond,
 *     so chains of x and y bonds end at the left and right sides while rows
 *     stay periodic); the locally connected CRBM keeps a shared bulk filter
 *     bank and unshared banks for the n_edge hidden columns at each side, and
 *     its filter windows do not wrap across the column edge.
 *   - temperature swaps of parallel tempering (Eq. (acceptance) between two
 *     physical temperatures), stream PT=4: chains sit on a ladder grid,
 *     chain g = rung * n_ladders + ladder; round r pairs rungs (q, q+1) for
 *     q = r%2, r%2+2, ...; the uniform of a pair is the 53-bit MH-form
 *     uniform of counter (0, r, chain index of the lower rung, PT).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as  */
/* 1, 2, 3", SC'11): 10 rounds of the 4x32 S-box, Weyl key schedule.  */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

ORC_API void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

enum { ST_INIT = 0, ST_HID = 1, ST_VIS = 2, ST_MH = 3, ST_PT = 4 };

/* the 32-bit word that belongs to unit q of a stream */
static uint32_t unit_word(uint64_t seed, uint32_t q, uint32_t t, uint32_t g, uint32_t tag)
{
    const uint32_t ctr[4] = {q >> 2, t, g, tag};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[q & 3u];
}

static double word_to_unit_interval(uint32_t x) { return ((double)x + 0.5) * 0x1p-32; }

/* 53-bit uniform in (0,1) from words 0,1 of unit group 0 of a stream */
static double uniform53(uint64_t seed, uint32_t t, uint32_t g, uint32_t tag)
{
    const uint32_t ctr[4] = {0u, t, g, tag};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    const uint64_t x = ((uint64_t)out[0] << 32) | (uint64_t)out[1];
    return ((double)(x >> 11) + 0.5) * 0x1p-53;
}

/* 53-bit MH uniform of chain g at sweep t, in (0,1) */
ORC_API double orc_mh_uniform(uint64_t seed, uint32_t t, uint32_t g) { return uniform53(seed, t, g, ST_MH); }

/* 53-bit uniform of a temperature swap: round r, chain index g of the lower rung */
ORC_API double orc_pt_uniform(uint64_t seed, uint32_t r, uint32_t g) { return uniform53(seed, r, g, ST_PT); }

/* Bernoulli uniform of unit q in stream `tag` */
ORC_API double orc_unit_uniform(uint64_t seed, uint32_t q, uint32_t t, uint32_t g, uint32_t tag)
{
    return word_to_unit_interval(unit_word(seed, q, t, g, tag));
}

/* ------------------------------------------------------------------ */
/* CRBM parameters                                                     */
/* ------------------------------------------------------------------ */
/* Filter banks: the periodic CRBM has one bank, W[K][C][Lw][Lw], hbias[K].
 * The locally connected CRBM of Sec. IV.B (open boundaries) has
 * 1 + 2 n_edge banks, W[1+2n_edge][K][C][Lw][Lw], hbias[1+2n_edge][K]:
 * bank 0 is shared by the bulk, banks 1..n_edge belong to the hidden columns
 * 0..n_edge-1 (left side) and banks n_edge+1..2n_edge to the columns
 * L-n_edge..L-1 (right side).  With open_cols the filter window does not wrap
 * across the column edge: visible columns beyond it count as v = 0.  Rows stay
 * periodic. */
/* dense = 1: the fully connected RBM that Sec. IV compares with (FRBM):
 * K hidden units, each connected to all C L^2 visible units, W[K][C][L][L]
 * with Lw = L, hbias[K], vbias[C][L][L] (one bias per visible unit). */
typedef struct {
    int32_t K, C, Lw;
    const float* W;     /* [banks][K][C][Lw][Lw] */
    const float* hbias; /* [banks][K] */
    const float* vbias; /* [C], or [C][L][L] when dense */
    int32_t open_cols, n_edge;
    int32_t dense;
} orc_params;

/* number of hidden units of a configuration of side L */
static int n_hidden(const orc_params* P, int L) { return P->dense ? P->K : P->K * L * L; }

static inline int wrap(int i, int L) { int r = i % L; return r < 0 ? r + L : r; }

/* filter bank of hidden column j */
static int bank_of(const orc_params* P, int j, int L)
{
    const int ne = P->n_edge;
    if (ne <= 0) return 0;
    if (j < ne) return 1 + j;
    if (j >= L - ne) return 1 + ne + (j - (L - ne));
    return 0;
}

/* visible column reached from column j by an offset, or -1 past an open edge */
static int column(const orc_params* P, int j, int L)
{
    if (P->open_cols) return (j >= 0 && j < L) ? j : -1;
    return wrap(j, L);
}

static double Wd(const orc_params* P, int bank, int k, int c, int a, int b)
{
    return (double)P->W[(((size_t)bank * P->K + k) * P->C + c) * P->Lw * P->Lw + a * P->Lw + b];
}

static double hbd(const orc_params* P, int bank, int k) { return (double)P->hbias[bank * P->K + k]; }

/* hidden pre-activations, Eq. (free-energy_CRBM) argument / App. B P(h|v):
 * a[k][i][j] = hb[k] + sum_{c,a,b} W[k][c][a][b] v[c][(i+a)%L][(j+b)%L]
 * with the bank of column j and, for open columns, no wrap in j  */
ORC_API void orc_hidden_preact(const orc_params* P, const uint8_t* v, int L, double* a_out)
{
    const int K = P->K, C = P->C, Lw = P->Lw;
    if (P->dense) {
        /* FRBM: a[k] = hb[k] + sum_q W[k][q] v[q] over all C L^2 visible units */
        const int nv = C * L * L;
        for (int k = 0; k < K; ++k) {
            double s = (double)P->hbias[k];
            for (int q = 0; q < nv; ++q) s += (double)P->W[(size_t)k * nv + q] * (double)v[q];
            a_out[k] = s;
        }
        return;
    }
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < L; ++j) {
                const int bk = bank_of(P, j, L);
                double s = hbd(P, bk, k);
                for (int c = 0; c < C; ++c)
                    for (int a = 0; a < Lw; ++a)
                        for (int b = 0; b < Lw; ++b) {
                            const int jj = column(P, j + b, L);
                            if (jj < 0) continue;
                            s += Wd(P, bk, k, c, a, b) * (double)v[(c * L + wrap(i + a, L)) * L + jj];
                        }
                a_out[(k * L + i) * L + j] = s;
            }
}

/* visible pre-activations, App. B P(v|h), the exact adjoint of the above:
 * b[c][x][y] = vb[c] + sum_{k,a,b} W[k][c][a][b] h[k][(x-a)%L][(y-b)%L]
 * where the hidden unit at column y-b brings its own bank  */
ORC_API void orc_visible_preact(const orc_params* P, const uint8_t* h, int L, double* b_out)
{
    const int K = P->K, C = P->C, Lw = P->Lw;
    if (P->dense) {
        /* FRBM: b[q] = vb[q] + sum_k W[k][q] h[k] */
        const int nv = C * L * L;
        for (int q = 0; q < nv; ++q) {
            double s = (double)P->vbias[q];
            for (int k = 0; k < K; ++k) s += (double)P->W[(size_t)k * nv + q] * (double)h[k];
            b_out[q] = s;
        }
        return;
    }
    for (int c = 0; c < C; ++c)
        for (int x = 0; x < L; ++x)
            for (int y = 0; y < L; ++y) {
                double s = (double)P->vbias[c];
                for (int k = 0; k < K; ++k)
                    for (int a = 0; a < Lw; ++a)
                        for (int b = 0; b < Lw; ++b) {
                            const int jj = column(P, y - b, L);
                            if (jj < 0) continue;
                            s += Wd(P, bank_of(P, jj, L), k, c, a, b) * (double)h[(k * L + wrap(x - a, L)) * L + jj];
                        }
                b_out[(c * L + x) * L + y] = s;
            }
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }
static double softplus(double x) { return (x > 0 ? x : 0.0) + log1p(exp(-fabs(x))); }
/* log(2 cosh x) */
static double log2cosh(double x) { const double ax = fabs(x); return ax + log1p(exp(-2.0 * ax)); }

/* CRBM free energy, Eq. (free-energy_CRBM), of one visible configuration v */
static double free_energy_v(const orc_params* P, const uint8_t* v, int L, double* scratch)
{
    const int C = P->C, n = L * L;
    orc_hidden_preact(P, v, L, scratch);
    double F = 0.0;
    if (P->dense) {
        for (int q = 0; q < C * n; ++q) F -= (double)P->vbias[q] * (double)v[q];
    } else {
        for (int c = 0; c < C; ++c) {
            double nv = 0.0;
            for (int q = 0; q < n; ++q) nv += (double)v[c * n + q];
            F -= (double)P->vbias[c] * nv;
        }
    }
    for (int q = 0; q < n_hidden(P, L); ++q) F -= softplus(scratch[q]);
    return F;
}

static void spins_to_visible(const int8_t* s, int C, int L, uint8_t* v)
{
    for (int q = 0; q < C * L * L; ++q) v[q] = (uint8_t)(s[q] > 0);
}

/* F for a batch of +-1 configurations, x[B][C][L][L] */
ORC_API void orc_free_energy(const orc_params* P, const int8_t* x, int B, int L, double* F_out)
{
    const int C = P->C, n = L * L;
#pragma omp parallel
    {
        uint8_t* v = (uint8_t*)malloc((size_t)C * n);
        double* a = (double*)malloc(sizeof(double) * (size_t)P->K * n);
#pragma omp for schedule(static)
        for (int b = 0; b < B; ++b) {
            spins_to_visible(x + (size_t)b * C * n, C, L, v);
            F_out[b] = free_energy_v(P, v, L, a);
        }
        free(v);
        free(a);
    }
}

/* ------------------------------------------------------------------ */
/* Targets                                                             */
/* ------------------------------------------------------------------ */
/* Ising energy of Sec. III in units of J: E/J = -sum_<ij> s_i s_j, each
 * nearest-neighbour bond of the square lattice counted once; rows are
 * periodic, columns too unless open_cols (then the bond from column L-1 to
 * column 0 is absent).  */
ORC_API int64_t orc_ising_energy(const int8_t* s, int L, int open_cols)
{
    int64_t e = 0;
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
            const int64_t sij = s[i * L + j];
            e -= sij * (int64_t)s[wrap(i + 1, L) * L + j];
            if (!(open_cols && j == L - 1)) e -= sij * (int64_t)s[i * L + wrap(j + 1, L)];
        }
    return e;
}

ORC_API int64_t orc_magnetization(const int8_t* s, int L)
{
    int64_t m = 0;
    for (int q = 0; q < L * L; ++q) m += s[q];
    return m;
}

/* Majorana hopping block of Sec. IV: honeycomb as a brick wall of unit
 * cells r=(i,j), black site b(r), white site w(r).  Bonds of b(i,j):
 * z -> w(i,j), x -> w(i,(j+1)%L), y -> w((i+1)%L,j).  Entry = 2 J_alpha u_alpha(r)
 * (from H = -i J sum u c_b c_w written as (i/4) sum A c c).  u is either
 * [3][L][L] (x, y, z channels) or, with C==1, the z-bond field eta alone
 * with u_x = u_y = +1.  M is N x N row-major, N = L*L, rows = black sites.
 * open_cols (Sec. IV.B): the x bonds from column L-1 to column 0 are absent,
 * so the chains of x and y bonds end at the left and right sides while the
 * chains of y and z bonds stay closed. */
ORC_API void orc_kitaev_matrix(const int8_t* u, int C, int L, const double J[3], int open_cols, double* M)
{
    const int N = L * L;
    memset(M, 0, sizeof(double) * (size_t)N * N);
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) {
            const int r = i * L + j;
            const double ux = (C == 3) ? (double)u[(0 * L + i) * L + j] : 1.0;
            const double uy = (C == 3) ? (double)u[(1 * L + i) * L + j] : 1.0;
            const double uz = (C == 3) ? (double)u[(2 * L + i) * L + j] : (double)u[i * L + j];
            M[(size_t)r * N + r] += 2.0 * J[2] * uz;
            if (!(open_cols && j == L - 1)) M[(size_t)r * N + (i * L + wrap(j + 1, L))] += 2.0 * J[0] * ux;
            M[(size_t)r * N + (wrap(i + 1, L) * L + j)] += 2.0 * J[1] * uy;
        }
}

/* Singular values of an N x N matrix by one-sided (Hestenes) Jacobi:
 * rotate column pairs until all are mutually orthogonal; the singular
 * values are then the column norms.  A is overwritten. */
ORC_API int orc_singular_values(double* A, int N, double* sv)
{
    const double tol = 1e-15;
    int sweep;
    for (sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < N - 1; ++p)
            for (int q = p + 1; q < N; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = 0; r < N; ++r) {
                    const double xp = A[(size_t)r * N + p], xq = A[(size_t)r * N + q];
                    al += xp * xp;
                    be += xq * xq;
                    ga += xp * xq;
                }
                if (ga == 0.0 || fabs(ga) <= tol * sqrt(al * be)) continue;
                rotated = 1;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                for (int r = 0; r < N; ++r) {
                    const double xp = A[(size_t)r * N + p], xq = A[(size_t)r * N + q];
                    A[(size_t)r * N + p] = cs * xp - sn * xq;
                    A[(size_t)r * N + q] = sn * xp + cs * xq;
                }
            }
        if (!rotated) break;
    }
    for (int c = 0; c < N; ++c) {
        double s = 0.0;
        for (int r = 0; r < N; ++r) s += A[(size_t)r * N + c] * A[(size_t)r * N + c];
        sv[c] = sqrt(s);
    }
    return sweep;
}

/* Gauge-field weight of Sec. IV: F(u) = -T sum_lambda log 2cosh(beta eps/2),
 * summed over the N singular values of M.  Returned are S = -beta F and the
 * fermion energy E_f = -sum (eps/2) tanh(beta eps/2) and the fluctuation term
 * Cf = sum (beta eps/2)^2 / cosh^2(beta eps/2) used by the specific heat. */
ORC_API double orc_kitaev_S(const int8_t* u, int C, int L, const double J[3], int open_cols, double beta,
                            double* eps_out, double* Ef_out, double* Cf_out)
{
    const int N = L * L;
    double* M = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* eps = (double*)malloc(sizeof(double) * (size_t)N);
    orc_kitaev_matrix(u, C, L, J, open_cols, M);
    orc_singular_values(M, N, eps);
    double S = 0.0, Ef = 0.0, Cf = 0.0;
    for (int l = 0; l < N; ++l) {
        const double x = 0.5 * beta * eps[l];
        S += log2cosh(x);
        Ef -= 0.5 * eps[l] * tanh(x);
        const double ch = cosh(x);
        Cf += (x * x) / (ch * ch);
    }
    if (eps_out) memcpy(eps_out, eps, sizeof(double) * (size_t)N);
    if (Ef_out) *Ef_out = Ef;
    if (Cf_out) *Cf_out = Cf;
    free(M);
    free(eps);
    return S;
}

/* batched target: Ising E (units of J, exact) or Kitaev S = -beta F */
ORC_API void orc_target(int target, const int8_t* x, int C, int B, int L, int open_cols, const double J[3],
                        const double* T, int64_t* E_out, double* S_out)
{
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < B; ++b) {
        const int8_t* s = x + (size_t)b * C * L * L;
        if (target == 0) {
            if (E_out) E_out[b] = orc_ising_energy(s, L, open_cols);
        } else {
            if (S_out) S_out[b] = orc_kitaev_S(s, C, L, J, open_cols, 1.0 / T[b], NULL, NULL, NULL);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Sampling                                                            */
/* ------------------------------------------------------------------ */
/* i.i.d. +-1 start, stream INIT (Alg. 1 initialises with Binomial(p=0.5)) */
ORC_API void orc_init_state(uint64_t seed, uint32_t g0, int n, int C, int L, int8_t* s)
{
    const int nv = C * L * L;
    for (int g = 0; g < n; ++g)
        for (int q = 0; q < nv; ++q)
            s[(size_t)g * nv + q] = (unit_word(seed, (uint32_t)q, 0u, g0 + (uint32_t)g, ST_INIT) >> 31) ? 1 : -1;
}

/* one block-Gibbs step v -> h -> v' of App. B; counts near-ties |u-sigma|<1e-12 */
ORC_API int64_t orc_gibbs_step(const orc_params* P, int L, const uint8_t* v, uint8_t* h, uint8_t* vout,
                               uint64_t seed, uint32_t t, uint32_t g, uint32_t substep, double* scratch)
{
    const int C = P->C, n = L * L;
    int64_t ties = 0;
    orc_hidden_preact(P, v, L, scratch);
    for (int q = 0; q < n_hidden(P, L); ++q) {
        const double u = orc_unit_uniform(seed, (uint32_t)q, t, g, ST_HID | (substep << 8));
        const double p = sigmoid(scratch[q]);
        if (fabs(u - p) < 1e-12) ++ties;
        h[q] = (uint8_t)(u < p);
    }
    orc_visible_preact(P, h, L, scratch);
    for (int q = 0; q < C * n; ++q) {
        const double u = orc_unit_uniform(seed, (uint32_t)q, t, g, ST_VIS | (substep << 8));
        const double p = sigmoid(scratch[q]);
        if (fabs(u - p) < 1e-12) ++ties;
        vout[q] = (uint8_t)(u < p);
    }
    return ties;
}

/* per-chain record kept between calls */
typedef struct {
    int64_t sweeps, n_acc, n_meas, pad0;
    int64_t sumE, sumE2, sumM, sumAbsM, sumM2; /* Ising, units of J */
    int64_t E;                                  /* Ising energy of current state */
    double F;                                   /* CRBM free energy of current state */
    double S, Ef, Cf;                           /* Kitaev -beta F, fermion energy, fluctuation */
    double kE, kE2, kCf;                        /* Kitaev sums */
    int64_t n_swap;                             /* accepted temperature swaps */
} orc_chain;

typedef struct {
    int32_t target; /* 0 Ising, 1 Kitaev, 2 plain Gibbs chain (no MH) */
    int32_t L, n_chains, gibbs_k, burnin;
    uint32_t g0;
    uint64_t seed;
    double J[3];
    int32_t boundary; /* target lattice: 0 periodic, 1 open columns (Sec. IV.B) */
} orc_run_desc;

/* record of the current state: cached F and target, zeroed sums */
ORC_API void orc_chain_init(const orc_params* P, const orc_run_desc* D, const double* T,
                            const int8_t* state, orc_chain* rec, double* eps)
{
    const int C = P->C, L = D->L, nv = C * L * L;
#pragma omp parallel
    {
        uint8_t* v = (uint8_t*)malloc((size_t)nv);
        double* a = (double*)malloc(sizeof(double) * (size_t)P->K * L * L);
#pragma omp for schedule(dynamic)
        for (int g = 0; g < D->n_chains; ++g) {
            const int8_t* s = state + (size_t)g * nv;
            orc_chain* R = rec + g;
            memset(R, 0, sizeof *R);
            spins_to_visible(s, C, L, v);
            R->F = free_energy_v(P, v, L, a);
            if (D->target != 1) {
                R->E = orc_ising_energy(s, L, D->boundary);
            } else {
                R->S = orc_kitaev_S(s, C, L, D->J, D->boundary, 1.0 / T[g], eps ? eps + (size_t)g * L * L : NULL, &R->Ef,
                                    &R->Cf);
            }
        }
        free(v);
        free(a);
    }
}

/* n_sweeps propose+accept sweeps of every chain, starting at sweep index t0.
 * One sweep: gibbs_k Gibbs steps from the current state (or, with `rbm` not
 * NULL, from the chain's persistent CRBM replica) give x'; then
 * Ising:  log r = -beta J (E(x') - E(x)) + F(x') - F(x)
 * Kitaev: log r =  S(x') - S(x)          + F(x') - F(x)
 * accept iff log u < log r.  After burn-in (sweep index >= burnin) the
 * observables of the state after the sweep are accumulated.
 * With a replica: accepted -> state <- x', replica <- old state; rejected ->
 * replica <- x'.  For Kitaev, `eps` (if not NULL) keeps the singular values
 * of every chain's current state, [n_chains][L*L].
 * ties[0] counts Gibbs near-ties, ties[1] counts |log r - log u| < 1e-6.
 * accept_log / energy_log (optional, [n_chains][n_sweeps]) record each sweep's
 * decision and the energy after it (Ising E/J, Kitaev E_f).  */
ORC_API void orc_run(const orc_params* P, const orc_run_desc* D, const double* T, int8_t* state, int8_t* rbm,
                     double* eps, uint32_t t0, int n_sweeps, orc_chain* rec, int64_t* ties, uint8_t* accept_log,
                     double* energy_log)
{
    const int C = P->C, L = D->L, n = L * L, nv = C * n;
    int64_t gt = 0, mt = 0;
#pragma omp parallel reduction(+ : gt, mt)
    {
        uint8_t* v = (uint8_t*)malloc((size_t)nv);
        uint8_t* v2 = (uint8_t*)malloc((size_t)nv);
        uint8_t* h = (uint8_t*)malloc((size_t)P->K * n);
        double* a = (double*)malloc(sizeof(double) * (size_t)(P->K > C ? P->K : C) * n);
        int8_t* sp = (int8_t*)malloc((size_t)nv);
        double* epsp = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(dynamic)
        for (int g = 0; g < D->n_chains; ++g) {
            int8_t* s = state + (size_t)g * nv;
            int8_t* y = rbm ? rbm + (size_t)g * nv : NULL;
            orc_chain* R = rec + g;
            const double beta = 1.0 / T[g];
            const uint32_t gid = D->g0 + (uint32_t)g;
            for (int it = 0; it < n_sweeps; ++it) {
                const uint32_t t = t0 + (uint32_t)it;
                spins_to_visible(y ? y : s, C, L, v);
                for (int k = 0; k < D->gibbs_k; ++k) {
                    gt += orc_gibbs_step(P, L, v, h, v2, D->seed, t, gid, (uint32_t)k, a);
                    memcpy(v, v2, (size_t)nv);
                }
                for (int q = 0; q < nv; ++q) sp[q] = v[q] ? 1 : -1;
                const double Fp = free_energy_v(P, v, L, a);
                double logr;
                int64_t Ep = 0;
                double Sp = 0, Efp = 0, Cfp = 0;
                if (D->target != 1) {
                    Ep = orc_ising_energy(sp, L, D->boundary);
                    logr = -beta * D->J[0] * (double)(Ep - R->E) + (Fp - R->F);
                } else {
                    Sp = orc_kitaev_S(sp, C, L, D->J, D->boundary, beta, epsp, &Efp, &Cfp);
                    logr = (Sp - R->S) + (Fp - R->F);
                }
                const double lu = log(orc_mh_uniform(D->seed, t, gid));
                /* target 2: plain Gibbs chain of the CRBM, every proposal accepted */
                if (D->target != 2 && fabs(logr - lu) < 1e-6) ++mt;
                const int acc = D->target == 2 ? 1 : (lu < logr);
                if (accept_log) accept_log[(size_t)g * n_sweeps + it] = (uint8_t)acc;
                if (acc) {
                    if (y) memcpy(y, s, (size_t)nv); /* the replica takes the old state */
                    memcpy(s, sp, (size_t)nv);
                    R->F = Fp;
                    if (D->target != 1) R->E = Ep;
                    else {
                        R->S = Sp;
                        R->Ef = Efp;
                        R->Cf = Cfp;
                        if (eps) memcpy(eps + (size_t)g * n, epsp, sizeof(double) * (size_t)n);
                    }
                    R->n_acc += 1;
                } else if (y) {
                    memcpy(y, sp, (size_t)nv); /* the replica keeps its Gibbs steps */
                }
                R->sweeps += 1;
                if (energy_log)
                    energy_log[(size_t)g * n_sweeps + it] = D->target != 1 ? (double)R->E : R->Ef;
                if ((int64_t)t >= (int64_t)D->burnin) {
                    R->n_meas += 1;
                    if (D->target != 1) {
                        const int64_t m = orc_magnetization(s, L);
                        R->sumE += R->E;
                        R->sumE2 += R->E * R->E;
                        R->sumM += m;
                        R->sumAbsM += m < 0 ? -m : m;
                        R->sumM2 += m * m;
                    } else {
                        R->kE += R->Ef;
                        R->kE2 += R->Ef * R->Ef;
                        R->kCf += R->Cf;
                    }
                }
            }
        }
        free(v);
        free(v2);
        free(h);
        free(a);
        free(sp);
        free(epsp);
    }
    if (ties) {
        ties[0] += gt;
        ties[1] += mt;
    }
}

/* One round of temperature swaps of parallel tempering (App. B, Eq.
 * (acceptance) between two physical temperatures).  Chains form a grid
 * g = rung * n_ladders + ladder; round r pairs rungs (q, q+1) for
 * q = r % 2, r % 2 + 2, ... < n_rungs - 1.  For a pair (a, b):
 *   Ising:  log A = J (beta_a - beta_b) (E_a - E_b)
 *   Kitaev: log A = S_a(x_b) + S_b(x_a) - S_a(x_a) - S_b(x_b),
 *           S_beta(x) = sum_lambda log 2cosh(beta eps_lambda(x) / 2)
 * accept iff log u < log A (u from stream PT).  On acceptance the two
 * physical states swap, with their cached E, F (and the singular values,
 * recomputing S, Ef, Cf at the new temperatures); sums, replicas and sweep
 * counters stay with the chain slot.  ties counts |log A - log u| < 1e-6. */
ORC_API void orc_tempering_swap(const orc_run_desc* D, int C, const double* T, int8_t* state, orc_chain* rec,
                                double* eps, int n_ladders, uint32_t round, int64_t* ties)
{
    const int L = D->L, n = L * L, nv = C * n;
    const int n_rungs = D->n_chains / n_ladders;
    int8_t* tmp = (int8_t*)malloc((size_t)nv);
    double* etmp = (double*)malloc(sizeof(double) * (size_t)n);
    for (int q = (int)(round & 1u); q + 1 < n_rungs; q += 2) {
        for (int l = 0; l < n_ladders; ++l) {
            const int a = q * n_ladders + l, b = (q + 1) * n_ladders + l;
            orc_chain *Ra = rec + a, *Rb = rec + b;
            const double ba = 1.0 / T[a], bb = 1.0 / T[b];
            double logA, Sab = 0, Sba = 0, Efab = 0, Efba = 0, Cfab = 0, Cfba = 0;
            if (D->target != 1) {
                logA = D->J[0] * (ba - bb) * (double)(Ra->E - Rb->E);
            } else {
                const double* ea = eps + (size_t)a * n;
                const double* eb = eps + (size_t)b * n;
                for (int i = 0; i < n; ++i) {
                    const double xa = 0.5 * ba * eb[i], xb = 0.5 * bb * ea[i];
                    Sab += log2cosh(xa);
                    Sba += log2cosh(xb);
                    Efab -= 0.5 * eb[i] * tanh(xa);
                    Efba -= 0.5 * ea[i] * tanh(xb);
                    Cfab += xa * xa / (cosh(xa) * cosh(xa));
                    Cfba += xb * xb / (cosh(xb) * cosh(xb));
                }
                logA = Sab + Sba - Ra->S - Rb->S;
            }
            const double lu = log(orc_pt_uniform(D->seed, round, D->g0 + (uint32_t)a));
            if (ties && fabs(logA - lu) < 1e-6) ++*ties;
            if (!(lu < logA)) continue;
            memcpy(tmp, state + (size_t)a * nv, (size_t)nv);
            memcpy(state + (size_t)a * nv, state + (size_t)b * nv, (size_t)nv);
            memcpy(state + (size_t)b * nv, tmp, (size_t)nv);
            const double F = Ra->F;
            Ra->F = Rb->F;
            Rb->F = F;
            if (D->target != 1) {
                const int64_t E = Ra->E;
                Ra->E = Rb->E;
                Rb->E = E;
            } else {
                memcpy(etmp, eps + (size_t)a * n, sizeof(double) * (size_t)n);
                memcpy(eps + (size_t)a * n, eps + (size_t)b * n, sizeof(double) * (size_t)n);
                memcpy(eps + (size_t)b * n, etmp, sizeof(double) * (size_t)n);
                Ra->S = Sab;
                Ra->Ef = Efab;
                Ra->Cf = Cfab;
                Rb->S = Sba;
                Rb->Ef = Efba;
                Rb->Cf = Cfba;
            }
            Ra->n_swap += 1;
            Rb->n_swap += 1;
        }
    }
    free(tmp);
    free(etmp);
}

/* ------------------------------------------------------------------ */
/* Gradient of F (the backward of the loss of Eq. (loss), Alg. 1)       */
/* dF/dW[k][c][a][b] = -sum_ij sigma(a[k][i][j]) v[c][(i+a)%L][(j+b)%L]  */
/* dF/dhb[k]         = -sum_ij sigma(a[k][i][j])                         */
/* dF/dvb[c]         = -sum_ij v[c][i][j]                                */
/* out = sum_n g_n dF(x_n)/dtheta; with several banks, hidden column j    */
/* contributes to the bank that owns it; dW, dhb have the banks' layout.  */
/* FRBM (dense): dF/dW[k][q] = -sigma(a[k]) v[q], dF/dhb[k] = -sigma(a[k]),*/
/* dF/dvb[q] = -v[q].                                                     */
/* ------------------------------------------------------------------ */
ORC_API void orc_grad(const orc_params* P, const int8_t* x, int B, int L, const double* gF,
                      double* dW, double* dhb, double* dvb)
{
    const int K = P->K, C = P->C, Lw = P->Lw, n = L * L;
    if (P->dense) {
        const int nv = C * n;
        memset(dW, 0, sizeof(double) * (size_t)K * nv);
        memset(dhb, 0, sizeof(double) * (size_t)K);
        memset(dvb, 0, sizeof(double) * (size_t)nv);
        uint8_t* v = (uint8_t*)malloc((size_t)nv);
        double* a = (double*)malloc(sizeof(double) * (size_t)K);
        for (int bi = 0; bi < B; ++bi) {
            const double g = gF[bi];
            spins_to_visible(x + (size_t)bi * nv, C, L, v);
            orc_hidden_preact(P, v, L, a);
            for (int k = 0; k < K; ++k) {
                const double sg = sigmoid(a[k]);
                dhb[k] -= g * sg;
                for (int q = 0; q < nv; ++q) dW[(size_t)k * nv + q] -= g * sg * (double)v[q];
            }
            for (int q = 0; q < nv; ++q) dvb[q] -= g * (double)v[q];
        }
        free(v);
        free(a);
        return;
    }
    const int nb = 1 + 2 * (P->n_edge > 0 ? P->n_edge : 0);
    const int nW = K * C * Lw * Lw;
    memset(dW, 0, sizeof(double) * (size_t)nb * nW);
    memset(dhb, 0, sizeof(double) * (size_t)nb * K);
    memset(dvb, 0, sizeof(double) * (size_t)C);
    uint8_t* v = (uint8_t*)malloc((size_t)C * n);
    double* a = (double*)malloc(sizeof(double) * (size_t)K * n);
    for (int bi = 0; bi < B; ++bi) {
        const double g = gF[bi];
        spins_to_visible(x + (size_t)bi * C * n, C, L, v);
        orc_hidden_preact(P, v, L, a);
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < L; ++i)
                for (int j = 0; j < L; ++j) {
                    const double sg = sigmoid(a[(k * L + i) * L + j]);
                    const int bk = bank_of(P, j, L);
                    dhb[bk * K + k] -= g * sg;
                    for (int c = 0; c < C; ++c)
                        for (int aa = 0; aa < Lw; ++aa)
                            for (int bb = 0; bb < Lw; ++bb) {
                                const int jj = column(P, j + bb, L);
                                if (jj < 0) continue;
                                dW[(size_t)bk * nW + ((k * C + c) * Lw + aa) * Lw + bb] -=
                                    g * sg * (double)v[(c * L + wrap(i + aa, L)) * L + jj];
                            }
                }
        for (int c = 0; c < C; ++c) {
            double nvc = 0.0;
            for (int q = 0; q < n; ++q) nvc += v[c * n + q];
            dvb[c] -= g * nvc;
        }
    }
    free(v);
    free(a);
}

ORC_API int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Harness only (timing of the CPU baseline): threads of the OpenMP loops over chains. */
ORC_API void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
