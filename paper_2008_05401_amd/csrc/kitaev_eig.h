// kitaev_eig.h -- workgroup-cooperative FP64 gauge-field weight of the Kitaev
// honeycomb model (Sec. IV): S(u) = sum_lambda log 2cosh(beta eps_lambda / 2)
// over the singular values eps of the Majorana hopping block M (N x N, N=L^2).
//
// GPU method of the fast route (a one-sided Jacobi SVD of M, below, serves only
// the rare re-checks of the MH test):
//   1. A = M^T M is assembled directly from the bond variables (each white
//      site has three black neighbours, so A has at most 7 non-zeros per row);
//      up to L = 12 A is held in LDS as a packed lower triangle (N(N+1)/2
//      doubles, 83 KiB at N = 144); for 12 < L <= 24 it no longer fits and is
//      stored in full (N x N, row-major) in a per-chain global scratch, where
//      every access of the reduction below is then a contiguous row;
//   2. Householder reduction of A to a symmetric tridiagonal matrix (d, e),
//      column by column in LDS, in panels of 8 columns when A is global;
//   3. every eigenvalue lambda_i of the tridiagonal matrix by multisection on
//      the Sturm count (division-free recurrence), a group of up to eight lanes
//      per eigenvalue (kitaev_eigs_groups);
//   4. eps_i = sqrt(max(lambda_i, 0)); S, the fermion energy and the
//      fluctuation term are reduced over the workgroup.
//
// Error bound carried with S (used by the MH test of the sweep).  Squaring M
// costs accuracy: eigenvalues of A carry an absolute error dlam, and S depends
// on lambda through f(lambda) = log 2cosh(beta sqrt(lambda) / 2), whose slope
// f'(lambda) = (beta / 4) tanh(beta sqrt(lambda) / 2) / sqrt(lambda) is at most
// (beta / 4) min(beta / 2, 1 / sqrt(lambda)) -- up to beta^2 / 8 for the small
// singular values, 5000 at T = 0.005.  The bound is
//   B_S = dlam sum_i (beta / 4) min(beta / 2, 1 / sqrt(max(lambda_i - dlam, 0)))
//         + (N + 4) 2^-53 S,
// the last term for the N log 2cosh evaluations and their sum.  dlam
// (kitaev_dlam) takes the normwise backward error of Householder
// tridiagonalisation in the textbook worst-case form, 4 N^2 2^-53 |A|_F (each
// of the N - 2 similarity steps is exact for a matrix within ~4 n 2^-53 |A|_F,
// n <= N the length of its dot products), with |A|_F <= |M|_F |M|_2 from the
// couplings alone (so the bound needs no norm of the state), plus the Sturm
// counts (exact for a tridiagonal matrix within a few ulp of T entrywise) and
// the final bisection bracket.  By Weyl's theorem every eigenvalue then moves
// by at most dlam.  The bound is a worst case: at L = 24, T = 0.005 it reaches
// ~1e-3 while the observed errors against LAPACK are ~1e-9.  Where the MH test
// falls inside the band, the decision is taken again from singular values of M
// itself by one-sided Jacobi (kitaev_weight_jacobi), which never squares M.
#pragma once
#include "device_common.h"
#include <type_traits>

namespace crbm {

// Wave minimum and maximum of a double by the same DPP pattern (exact, so the
// order does not matter).  Needs the whole wave active.
__device__ __forceinline__ double wave_min_dpp(double v)
{
    v = fmin(v, dpp_f64<0xB1>(v));
    v = fmin(v, dpp_f64<0x4E>(v));
    v = fmin(v, dpp_f64<0x141>(v));
    v = fmin(v, dpp_f64<0x140>(v));
    return fmin(fmin(readlane_t(v, 0), readlane_t(v, 16)), fmin(readlane_t(v, 32), readlane_t(v, 48)));
}

__device__ __forceinline__ double wave_max_dpp(double v)
{
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return fmax(fmax(readlane_t(v, 0), readlane_t(v, 16)), fmax(readlane_t(v, 32), readlane_t(v, 48)));
}

// Four workgroup sums at once, each added up exactly as block_sum adds it (so
// the results are the same), through one exchange in `red` (>= 4 nwaves
// entries) with two barriers instead of eight.
__device__ __forceinline__ void block_sum4(double& a, double& b, double& c, double& d, double* red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    const double wa = wave_sum(a), wb = wave_sum(b), wc = wave_sum(c), wd = wave_sum(d);
    if (lane == 0) {
        red[wid] = wa;
        red[nw + wid] = wb;
        red[2 * nw + wid] = wc;
        red[3 * nw + wid] = wd;
    }
    __syncthreads();
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int i = 0; i < nw; ++i) {
        s0 += red[i];
        s1 += red[nw + i];
        s2 += red[2 * nw + i];
        s3 += red[3 * nw + i];
    }
    __syncthreads();
    a = s0;
    b = s1;
    c = s2;
    d = s3;
}

__device__ __forceinline__ int tri(int i, int j) { return (i * (i + 1) >> 1) + j; }  // j <= i
__device__ __forceinline__ int tri_s(int i, int j) { return i >= j ? tri(i, j) : tri(j, i); }

struct KitaevOut {
    double S, Ef, Cf;
    double B;  // bound on |S - S_exact| (0 from the Jacobi route)
};

// |M|_2 <= 2 (|J_x| + |J_y| + |J_z|) (at most one bond of each kind per row and
// column) and |M|_F <= 2 sqrt(N (J_x^2 + J_y^2 + J_z^2)); dlam bounds the
// absolute error of every computed eigenvalue of A = M^T M (see above).
__host__ __device__ inline double kitaev_dlam(int N, double Jx, double Jy, double Jz)
{
    const double u = 0x1p-53;
    const double n2 = 2.0 * (fabs(Jx) + fabs(Jy) + fabs(Jz));
    const double nf = 2.0 * sqrt((double)N * (Jx * Jx + Jy * Jy + Jz * Jz));
    return 4.0 * (double)N * (double)N * u * nf * n2 + (16.0 * u + 1.2e-15) * n2 * n2;
}

// the share of one eigenvalue lambda (= eps^2) in B_S, without the factor dlam
__device__ __forceinline__ double kitaev_bound_term(double lam, double beta, double dlam)
{
    const double lo = lam - dlam;
    const double g = lo > 0.0 ? fmin(0.5 * beta, 1.0 / sqrt(lo)) : 0.5 * beta;
    return 0.25 * beta * g;
}

constexpr int KITAEV_LDS_MAX_L = 12;  // A packed in LDS up to here
constexpr int KITAEV_MAX_L = 24;      // A in a global scratch beyond

__host__ __device__ inline bool kitaev_a_in_lds(int L) { return L <= KITAEV_LDS_MAX_L; }

// doubles of the global scratch of A for one chain (0 when A lives in LDS)
__host__ __device__ inline size_t kitaev_global_doubles(int L)
{
    const size_t N = (size_t)L * L;
    return kitaev_a_in_lds(L) ? 0 : N * N;
}

// doubles of a chain's global scratch: N x N, for M of the Jacobi re-check and,
// beyond L = 12, A of the eigen-step (used one after the other)
__host__ __device__ inline size_t kitaev_chain_doubles(int L)
{
    const size_t N = (size_t)L * L;
    return N * N;
}

// panel width of the blocked reduction used when A is global
constexpr int KITAEV_NB = 8;

// One wave per configuration for N <= 64 (L <= 8) when the workgroup is a single
// wave: A in LDS in full with an odd row stride (lane i owns row i), then d, e,
// e^2 and the Householder vectors v and w.
constexpr int KITAEV_WAVE_MAX_N = 64;
// rows padded with zeros to a multiple of 8 columns (whole batches of eight
// loads), plus one to make the row stride odd
__host__ __device__ inline int kitaev_wave_cols(int N) { return (N + 7) & ~7; }
__host__ __device__ inline int kitaev_wave_stride(int N) { return kitaev_wave_cols(N) + 1; }
__host__ __device__ inline size_t kitaev_wave_lds_bytes(int L)
{
    const size_t N = (size_t)L * L, NC = (size_t)kitaev_wave_cols((int)N);
    return sizeof(double) * (N * (size_t)kitaev_wave_stride((int)N) + 3 * N + 2 * NC);
}

// LDS region: [A packed, or the N eigenvalues when A is global | d | e | hv | p | (A global:)
// the panel's reflectors V and their companions W, column-major, KITAEV_NB x N each, then
// 16 waves x 2 KITAEV_NB partial sums and 2 KITAEV_NB reduced ones]; for N <= 64 large
// enough for the one-wave layout as well
__host__ __device__ inline size_t kitaev_lds_bytes(int L)
{
    const size_t N = (size_t)L * L;
    const size_t blk = sizeof(double) * (kitaev_a_in_lds(L) ? N * (N + 1) / 2 + 4 * N
                                                            : 5 * N + 2 * (size_t)KITAEV_NB * N + 34 * (size_t)KITAEV_NB);
    if (N > (size_t)KITAEV_WAVE_MAX_N) return blk;
    const size_t wv = kitaev_wave_lds_bytes(L);
    return blk > wv ? blk : wv;
}

struct KitaevBufs {
    double *A, *d, *e, *hv, *p, *eps, *vw;
};

// buffers inside the LDS region `lds`; `a_global` is the chain's scratch of
// kitaev_global_doubles(L) doubles (unused up to L = 12).  eps aliases A in
// LDS (A is dead once the tridiagonal form is known).
__device__ inline KitaevBufs kitaev_bufs(double* lds, double* a_global, int L)
{
    const int N = L * L;
    const int first = kitaev_a_in_lds(L) ? N * (N + 1) / 2 : N;
    KitaevBufs b;
    b.A = kitaev_a_in_lds(L) ? lds : a_global;
    b.d = lds + first;
    b.e = b.d + N;
    b.hv = b.e + N;
    b.p = b.hv + N;
    b.eps = lds;
    b.vw = kitaev_a_in_lds(L) ? nullptr : b.p + N;
    return b;
}

// Address-space-qualified pointers for the out-of-line eigen-steps, so that they
// address LDS with ds instructions and the global scratch with global ones
// rather than with flat instructions
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) const uint8_t lds_u8c;
typedef __attribute__((address_space(1))) double glb_f64;
template <bool kFull>
struct kit_a {
    typedef lds_f64 type;
};
template <>
struct kit_a<true> {
    typedef glb_f64 type;
};
template <bool kFull>
using kit_a_t = typename kit_a<kFull>::type;

// Element (i, j) of A, i >= j for the packed form
template <bool kFull>
__device__ __forceinline__ int a_at(int i, int j, int N)
{
    return kFull ? i * N + j : tri(i, j);
}

// Sturm count at x of the tridiagonal matrix (d, e2 = e^2): the number of sign
// changes along the leading principal minors p_0 = 1, p_1, ..., p_N, which is the
// number of eigenvalues below x; p_N = pm 2^xe on return.  kGuard: an exact zero
// minor is replaced by -2^-100 times its predecessor (so it takes the opposite
// sign).  Without kGuard no step tests for zero: each step is one dependent FMA,
// the sign bits of eight minors are shifted into a word and their changes counted
// with one popcount, and the smallest |p_i| is tracked.  The minors are then those
// of the guarded count whenever none is zero, and the return value says whether
// one was (the caller then counts again with kGuard).
__device__ __forceinline__ uint32_t sign_word(double v) { return (uint32_t)((unsigned long long)__double_as_longlong(v) >> 32); }

template <bool kGuard>
__device__ __forceinline__ bool sturm_count(const lds_f64* d, const lds_f64* e2, int N, double x, int& cnt_out,
                                            int& xe_out, double& pm_out)
{
    double p0 = 1.0, p1 = d[0] - x;
    int cnt, xe = 0;
    double zmin = 1.0;
    uint32_t m = 0;
    if (kGuard) {
        if (p1 == 0.0) p1 = -0x1p-100;
        cnt = p1 < 0.0;
    } else {
        zmin = fabs(p1);
        m = sign_word(p1) >> 31;
        cnt = (int)m;
    }
    int i0 = 1;
    for (; i0 + 7 < N; i0 += 8) {
        double dv[8], ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            dv[u] = d[i0 + u];
            ev[u] = e2[i0 + u - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            double pn = fma(dv[u] - x, p1, -ev[u] * p0);
            if (kGuard) {
                if (pn == 0.0) pn = -0x1p-100 * p1;
                cnt += (pn < 0.0) != (p1 < 0.0);
            } else {
                zmin = fmin(zmin, fabs(pn));
                m = __builtin_amdgcn_alignbit(m, sign_word(pn), 31);  // (m << 1) | sign(pn)
            }
            p0 = p1;
            p1 = pn;
        }
        // bits 8..0 of m: signs of p_{i0-1} .. p_{i0+7}
        if (!kGuard) cnt += __builtin_popcount((m ^ (m >> 1)) & 0xffu);
        const bool big = fabs(p1) > 0x1p+100, small = fabs(p1) < 0x1p-100;
        const double f = big ? 0x1p-100 : (small ? 0x1p+100 : 1.0);
        xe += big ? 100 : (small ? -100 : 0);
        p0 *= f;
        p1 *= f;
    }
    for (; i0 < N; ++i0) {
        double pn = fma(d[i0] - x, p1, -e2[i0 - 1] * p0);
        if (kGuard) {
            if (pn == 0.0) pn = -0x1p-100 * p1;
            cnt += (pn < 0.0) != (p1 < 0.0);
        } else {
            zmin = fmin(zmin, fabs(pn));
            cnt += (int)((sign_word(pn) ^ sign_word(p1)) >> 31);
        }
        p0 = p1;
        p1 = pn;
    }
    cnt_out = cnt;
    xe_out = xe;
    pm_out = p1;
    return !kGuard && !(zmin > 0.0);
}

// ---------------------------------------------------------------------------
// Every eigenvalue of the symmetric tridiagonal matrix (d, e), e2 = e^2, by
// multisection on the Sturm count, over the whole workgroup: a group of G
// adjacent lanes per eigenvalue (G <= 8, the largest with
// nwaves floor(64 / G) >= N, further rounds when even G = 1 leaves eigenvalues
// over), lane `sub` of the group evaluating the point lo + (sub + 1) h,
// h = (hi - lo) / (G + 1), so the bracket shrinks (G + 1)-fold per step; the
// group finds its first point whose count exceeds the eigenvalue's index from
// a ballot.  With a table, a first pass of one count per thread at evenly
// spaced points narrows every group's starting bracket to two neighbouring
// points.  Once a group's bracket holds its eigenvalue alone, the points
// cluster around the secant root of p_N between the bracket's ends instead
// (regula falsi on the determinant, every bracket still certified by counts),
// which ends in a few steps what multisection would take some twenty for.
// The count comes from the division-free three-term recurrence
// p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}, p_i = det(T_i - x), one
// eigenvalue below x per sign change of p_i / p_{i-1}; an exact zero is
// replaced by -2^-100 p_{i-1} (the sign convention of the ratio form; the fast
// count of sturm_count leaves the test out and counts again only if a minor was
// zero), and the pair is rescaled by 2^-+100 every eight steps to stay in range;
// the operands of eight steps are read from LDS before the eight dependent steps.  The
// first lane of each group adds log 2cosh(beta eps / 2), the fermion energy,
// the fluctuation term and the share of eps in the bound B_S (without the factor
// dlam) to S, Ef, Cf, Bs, and stores eps = sqrt(max(lambda, 0)) to eps_out
// after a workgroup barrier (eps_out may alias the dead matrix, never d or e2).
// ---------------------------------------------------------------------------
__device__ __host__ inline int kitaev_group_size(int N, int nwaves)
{
    int G = 8;
    while (G > 1 && nwaves * (64 / G) < N) --G;
    return G;
}

typedef __attribute__((address_space(3))) int lds_i32;

// doubles of the table of kitaev_eigs_groups for a workgroup of nt threads
__host__ __device__ inline int kitaev_eig_table_doubles(int nt) { return 2 * nt; }

__device__ inline void kitaev_eigs_groups(const lds_f64* d, const lds_f64* e2, int N, double glo, double ghi,
                                          double tol, double beta, double dlam, lds_f64* eps_out, double& S,
                                          double& Ef, double& Cf, double& Bs, lds_f64* tab, bool use_tab)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6, nt = blockDim.x;
    const double scale = fmax(fabs(glo), fabs(ghi));
    const int G = kitaev_group_size(N, nw), per_wave = 64 / G, cap = nw * per_wave;
    const int gi = lane / G, sub = lane - gi * G;
    const int gbase = gi * G < 64 ? gi * G : 0;
    const unsigned long long gmask = ((1ull << G) - 1ull) << (gi * G);
    const int rounds = (N + cap - 1) / cap;
    const double lo0 = glo - (1e-14 * scale + 1e-300), hi0 = ghi + (1e-14 * scale + 1e-300);
    // With a table (use_tab; kitaev_eig_table_doubles(nt) doubles of LDS at tab,
    // clear of d, e2 and the N entries of eps_out): one first pass
    // in which thread t counts at lo0 + (t + 1) h0, h0 = (hi0 - lo0) / (nt + 1),
    // so that every group starts from the two neighbouring points whose counts
    // enclose its eigenvalue (their determinants known) instead of the whole
    // Gershgorin interval
    const double h0 = (hi0 - lo0) / (double)(nt + 1);
    lds_i32* tci = (lds_i32*)(tab + nt);
    if (use_tab) {
        const double x = lo0 + (double)(tid + 1) * h0;
        int c = 0, xe = 0;
        double pm = 1.0;
        if (sturm_count<false>(d, e2, N, x, c, xe, pm)) sturm_count<true>(d, e2, N, x, c, xe, pm);
        tab[tid] = pm;
        tci[2 * tid] = c;
        tci[2 * tid + 1] = xe;
        __syncthreads();
    }
    for (int rd = 0; rd < rounds; ++rd) {
        const int idx = rd * cap + wid * per_wave + gi;
        const bool mine = gi < per_wave && idx < N;
        double lo = lo0, hi = hi0;
        // counts and scaled determinants p_N = m 2^x at the bracket's ends (ends
        // not yet evaluated carry no determinant)
        int clo = 0, chi = N;
        double mlo = 0.0, mhi = 0.0;
        int xlo = 0, xhi = 0;
        bool flo = false, fhi = false, sec_failed = false;
        if (use_tab && mine) {
            // neighbouring table points a < b with count(a) <= idx < count(b), the
            // ends standing in for a = -1 (count 0) and b = nt (count N)
            int a = -1, b = nt;
            while (b - a > 1) {
                const int m = (a + b) >> 1;
                if (tci[2 * m] > idx)
                    b = m;
                else
                    a = m;
            }
            if (a >= 0) {
                lo = lo0 + (double)(a + 1) * h0;
                clo = tci[2 * a];
                mlo = tab[a];
                xlo = tci[2 * a + 1];
                flo = true;
            }
            if (b < nt) {
                hi = lo0 + (double)(b + 1) * h0;
                chi = tci[2 * b];
                mhi = tab[b];
                xhi = tci[2 * b + 1];
                fhi = true;
            }
        }
        int q = 4;  // the cluster spans w 2^-q; doubled after every hit (the secant error squares)
        bool live = mine;
        for (int it = 0; it < 256; ++it) {
            const double w = hi - lo;
            const double h = w / (double)(G + 1);
            // done: bracket small enough, or no representable progress left
            if (live && (!(w > tol) || !(lo + h > lo) || !(lo + (double)G * h < hi))) live = false;
            if (!__any(live)) break;
            // Point placement.  Multisection: lo + (s + 1) h.  Once the bracket holds
            // exactly this eigenvalue (counts idx and idx + 1 at its ends, whose
            // determinants then differ in sign) the G points go to a cluster of
            // spacing dd = w 2^-q / (G - 1) around the secant root of the
            // determinant; q doubles after each hit, and a cluster that misses the
            // root is followed by one multisection step and q = 4 again.
            bool sec = G >= 2 && flo && fhi && clo == idx && chi == idx + 1 && !sec_failed;
            double a0 = 0.0, dd = 0.0;
            if (sec) {
                const int de = xlo - xhi;
                double t;
                if (de > 1000)
                    t = 1.0;
                else if (de < -1000)
                    t = 0.0;
                else {
                    const double r = ldexp(mlo / mhi, de);  // p_N(lo) / p_N(hi) < 0
                    t = r / (r - 1.0);
                }
                dd = ldexp(w, -q) / (double)(G - 1);
                const double span = dd * (double)(G - 1);
                a0 = lo + w * t - 0.5 * span;
                a0 = fmin(fmax(a0, lo + dd), hi - span - dd);
                sec = a0 > lo && a0 + dd > a0 && a0 + span < hi;
            }
            const double x = sec ? a0 + (double)sub * dd : lo + (double)(sub + 1) * h;
            int cnt = 0, xe = 0;
            double pm = 1.0;
            if (live) {
                if (sturm_count<false>(d, e2, N, x, cnt, xe, pm)) sturm_count<true>(d, e2, N, x, cnt, xe, pm);
            }
            // the group's first point with more than idx eigenvalues below it
            const unsigned long long mg = (__ballot(live && cnt > idx) & gmask) >> (gi * G);
            const int s0 = mg ? __builtin_ctzll(mg) : G;
            // count and determinant at the points that become the new ends
            const int sl = gbase + (s0 > 0 ? s0 - 1 : 0), sh = gbase + (s0 < G ? s0 : G - 1);
            const int c_l = __shfl(cnt, sl), c_h = __shfl(cnt, sh);
            const double m_l = __shfl(pm, sl), m_h = __shfl(pm, sh);
            const int x_l = __shfl(xe, sl), x_h = __shfl(xe, sh);
            if (live) {
                auto pt = [&](int q) { return sec ? a0 + (double)q * dd : lo + (double)(q + 1) * h; };
                const double nlo = s0 > 0 ? pt(s0 - 1) : lo;
                const double nhi = s0 < G ? pt(s0) : hi;
                if (s0 > 0) {
                    clo = c_l;
                    mlo = m_l;
                    xlo = x_l;
                    flo = true;
                }
                if (s0 < G) {
                    chi = c_h;
                    mhi = m_h;
                    xhi = x_h;
                    fhi = true;
                }
                sec_failed = sec && (s0 == 0 || s0 == G);
                if (sec) q = sec_failed ? 4 : (q < 24 ? 2 * q : 48);
                lo = nlo;
                hi = nhi;
            }
        }
        __syncthreads();  // every lane has read d and e2 of this round; eps may overwrite the matrix
        if (mine && sub == 0) {
            const double lam = 0.5 * (lo + hi);
            const double eps = sqrt(lam > 0.0 ? lam : 0.0);
            eps_out[idx] = eps;
            const double xv = 0.5 * beta * eps;  // >= 0
            // log 2cosh(xv) = xv + log1p(e) with e = exp(-2 xv), the steps of
            // log2cosh_d; 1 / cosh^2(xv) = 4 e / (1 + e)^2 from the same e
            const double em = exp(-2.0 * xv), op = 1.0 + em;
            S += xv + log1p(em);
            Ef -= 0.5 * eps * tanh(xv);
            Cf += (xv * xv) * (4.0 * em / (op * op));
            Bs += kitaev_bound_term(lam, beta, dlam);
        }
    }
}

// v: 0/1 bytes of the proposal, C channels ([3][L][L] = x,y,z bonds, or [1][L][L] = z bonds).
// open_cols (Sec. IV.B): the x bonds from column L-1 to column 0 are absent.
// kFull: A stored in full (N x N) rather than as a packed lower triangle.
// kNarrow: an instance for 1024-thread callers (128 VGPRs); the other instance
// serves workgroups of up to 512 threads and so gets 256 registers
template <bool kFull, bool kNarrow>
__device__ __noinline__ KitaevOut kitaev_weight_block_t(lds_u8c* v, int C, int L, int open_cols, double Jx, double Jy,
                                                        double Jz, double beta, kit_a_t<kFull>* A, lds_f64* d,
                                                        lds_f64* e, lds_f64* hv, lds_f64* p, lds_f64* red,
                                                        lds_f64* eps_out, lds_f64* vw)
{
    const int N = L * L;
    const int tid = threadIdx.x, nt = blockDim.x;
    // 1. A = M^T M, row w owned by one thread (full form: its mirror image too)
    if (kFull) {
        for (int q = tid; q < N * N; q += nt) A[q] = 0.0;
    } else {
        for (int w = tid; w < N; w += nt) {
            for (int q = 0; q <= w; ++q) A[tri(w, q)] = 0.0;
        }
    }
    __syncthreads();
    for (int w = tid; w < N; w += nt) {
        const int i = w / L, j = w - (w / L) * L;
        // black neighbours of w(i,j): b(i,j) via z, b(i,j-1) via x (none at an
        // open left side), b(i-1,j) via y
        int bn[3];
        bn[0] = w;
        bn[1] = j == 0 ? (open_cols ? -1 : i * L + L - 1) : i * L + j - 1;
        bn[2] = (i == 0 ? L - 1 : i - 1) * L + j;
        for (int nb = 0; nb < 3; ++nb) {
            const int b = bn[nb];
            if (b < 0) continue;
            const int bi = b / L, bj = b - (b / L) * L;
            // white neighbours of b(bi,bj) and the matrix entries M[b][w']
            int wn[3];
            double wv[3];
            wn[0] = b;
            wn[1] = bj + 1 == L ? (open_cols ? -1 : bi * L) : bi * L + bj + 1;
            wn[2] = (bi + 1 == L ? 0 : bi + 1) * L + bj;
            const double vz = C == 3 ? (v[2 * N + b] ? 1.0 : -1.0) : (v[b] ? 1.0 : -1.0);
            const double vx = C == 3 ? (v[0 * N + b] ? 1.0 : -1.0) : 1.0;
            const double vy = C == 3 ? (v[1 * N + b] ? 1.0 : -1.0) : 1.0;
            wv[0] = 2.0 * Jz * vz;
            wv[1] = 2.0 * Jx * vx;
            wv[2] = 2.0 * Jy * vy;
            // M[b][w] may receive several bonds when L is tiny; sum them
            double mbw = 0.0;
            for (int t = 0; t < 3; ++t)
                if (wn[t] == w) mbw += wv[t];
            // skip duplicate black neighbours so that each b counts once
            bool dup = false;
            for (int t = 0; t < nb; ++t) dup |= (bn[t] == b);
            if (dup) continue;
            for (int t = 0; t < 3; ++t) {
                const int w2 = wn[t];
                if (w2 < 0) continue;
                bool dupw = false;
                for (int s = 0; s < t; ++s) dupw |= (wn[s] == w2);
                if (dupw || w2 > w) continue;
                double mbw2 = 0.0;
                for (int s = 0; s < 3; ++s)
                    if (wn[s] == w2) mbw2 += wv[s];
                A[a_at<kFull>(w, w2, N)] += mbw * mbw2;
                // A[w2][w] (w2 < w) is written by this thread only: thread w2 fills columns <= w2
                if (kFull && w2 != w) A[w2 * N + w] += mbw * mbw2;
            }
        }
    }
    __syncthreads();

    // 2. Householder tridiagonalisation.  Packed A in LDS, unblocked, per step k:
    //    v from column k, p = bet A22 v with G = 16 lanes per row (two
    //    accumulators each, swizzle-reduced), then
    //    A22 -= v w^T + w v^T with w = p - kk v, kk = (bet/2)(p.v), i.e.
    //    A22 -= v p^T + p v^T - 2 kk v v^T, one wave per row, lanes along it.
    //    Five barriers per step: the two reductions alternate between two LDS
    //    slots, so a slot is never rewritten while another wave still reads it.
    //    nt is a multiple of 64.
    constexpr int G = 16;
    const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
    const int grp = tid / G, gl = tid - (tid / G) * G, ngrp = nt / G;
    int slot = 0;
    auto reduce = [&](double x) -> double {
        x = wave_sum_dpp(x);
        lds_f64* r = red + 16 * slot;  // 16 waves at most
        slot ^= 1;
        if (lane == 0) r[wid] = x;
        __syncthreads();
        // all sixteen slots are read at once (one LDS latency instead of nw in a
        // row); those of absent waves are discarded by the select
        double t[16];
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const double rw = r[w];
            t[w] = w < nw ? rw : 0.0;
        }
#pragma unroll
        for (int h = 8; h >= 1; h >>= 1)
#pragma unroll
            for (int w = 0; w < h; ++w) t[w] += t[w + h];
        return t[0];
    };
    // column k below the diagonal: in the full form read as row k (symmetry)
    auto col = [&](int i, int k) -> double { return kFull ? A[k * N + i] : A[tri(i, k)]; };
    if constexpr (kFull) {
        // Blocked reduction (the A in global memory): panels of NB columns.  Within
        // a panel A keeps its values from the panel's start; column k is corrected
        // on the fly by the panel's earlier reflectors,
        //   a = A[:,k] - V W[k,:]^T - W V[k,:]^T,
        // the matrix-vector product likewise, p = bet (A22 v - V (W^T v) - W (V^T v)),
        // and w = p - kk v (kk = bet (p.v) / 2) joins W; after the panel one pass
        // applies A22 -= V W^T + W V^T.  One read of the trailing matrix per column
        // plus one read-write per panel, instead of three passes per column.
        constexpr int NB = KITAEV_NB;
        lds_f64* Vc = vw;           // V[l][i] = vw[l N + i]
        lds_f64* Wc = vw + NB * N;  // W[l][i]
        lds_f64* part = vw + 2 * NB * N;  // per-wave partial sums of t_W, t_V: [16 waves][2 NB]
        lds_f64* tvw = part + 32 * NB;    // t_W[l], t_V[l] (2 NB doubles) after their reduction
        for (int k0 = 0; k0 + 2 < N; k0 += NB) {
            const int nbk = min(NB, N - 2 - k0);
            for (int jj = 0; jj < nbk; ++jj) {
                const int k = k0 + jj;
                // corrected column k, rows i >= k: diagonal to d[k], the rest to hv
                double s2 = 0.0;
                for (int i = k + tid; i < N; i += nt) {
                    double a = A[(size_t)k * N + i];
                    for (int l = 0; l < jj; ++l)
                        a -= Vc[l * N + i] * Wc[l * N + k] + Wc[l * N + i] * Vc[l * N + k];
                    if (i == k) {
                        d[k] = a;
                    } else {
                        hv[i] = a;
                        s2 += a * a;
                    }
                }
                s2 = reduce(s2);  // also publishes hv and d[k]
                const double x0 = hv[k + 1];
                const double rest = s2 - x0 * x0;
                if (!(rest > 1e-300 * (s2 > 1.0 ? s2 : 1.0))) {
                    // nothing to annihilate: the reflector is the identity
                    for (int i = tid; i < N; i += nt) {
                        Vc[jj * N + i] = 0.0;
                        Wc[jj * N + i] = 0.0;
                    }
                    if (tid == 0) e[k] = x0;
                    __syncthreads();
                    continue;
                }
                const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
                const double bet = 1.0 / (s2 - x0 * alpha);  // 2 / (v^T v)
                if (tid == 0) e[k] = alpha;
                // v into column jj of V (hv stays as read: other waves may still be
                // reading x0 from it); per-thread shares of t_W = W^T v and t_V = V^T v
                lds_f64* vcol = Vc + jj * N;
                double tw[NB], tv[NB];
#pragma unroll
                for (int l = 0; l < NB; ++l) tw[l] = tv[l] = 0.0;
                for (int i = tid; i < N; i += nt) {
                    const double vi = i > k ? (i == k + 1 ? x0 - alpha : hv[i]) : 0.0;
                    Vc[jj * N + i] = vi;
                    if (i > k) {
#pragma unroll
                        for (int l = 0; l < NB; ++l)
                            if (l < jj) {
                                tw[l] += Wc[l * N + i] * vi;
                                tv[l] += Vc[l * N + i] * vi;
                            }
                    }
                }
#pragma unroll
                for (int l = 0; l < NB; ++l)
                    if (l < jj) {
                        const double a = wave_sum(tw[l]), b = wave_sum(tv[l]);
                        if (lane == 0) {
                            part[wid * 2 * NB + l] = a;
                            part[wid * 2 * NB + NB + l] = b;
                        }
                    }
                __syncthreads();
                if (tid < 2 * jj) {
                    const int slotl = tid < jj ? tid : NB + (tid - jj);
                    double t = 0.0;
                    for (int w = 0; w < nw; ++w) t += part[w * 2 * NB + slotl];
                    tvw[slotl] = t;
                }
                __syncthreads();
                // p = bet (A22 v - V t_W - W t_V), rows of A22 contiguous; G lanes per row
                double pvl = 0.0;
                for (int i = k + 1 + grp; i < N; i += ngrp) {
                    const kit_a_t<kFull>* row = A + (size_t)i * N;
                    double a0 = 0.0, a1 = 0.0;
                    int j = k + 1 + gl;
                    for (; j + G < N; j += 2 * G) {
                        a0 += row[j] * vcol[j];
                        a1 += row[j + G] * vcol[j + G];
                    }
                    if (j < N) a0 += row[j] * vcol[j];
                    double acc = row16_sum(a0 + a1);
                    if (gl == 0) {
                        for (int l = 0; l < jj; ++l) acc -= Vc[l * N + i] * tvw[l] + Wc[l * N + i] * tvw[NB + l];
                        p[i] = bet * acc;
                        pvl += bet * acc * vcol[i];
                    }
                }
                const double kk2 = bet * reduce(pvl);  // 2 kk; publishes p
                for (int i = tid; i < N; i += nt) Wc[jj * N + i] = i > k ? p[i] - 0.5 * kk2 * vcol[i] : 0.0;
                __syncthreads();
            }
            // A22 -= V W^T + W V^T over rows and columns >= k0 + nbk, a wave per row
            const int kt = k0 + nbk;
            for (int i = kt + wid; i < N; i += nw) {
                double vi[NB], wi[NB];
#pragma unroll
                for (int l = 0; l < NB; ++l) {
                    vi[l] = l < nbk ? Vc[l * N + i] : 0.0;
                    wi[l] = l < nbk ? Wc[l * N + i] : 0.0;
                }
                kit_a_t<kFull>* row = A + (size_t)i * N;
                for (int j = kt + lane; j < N; j += 64) {
                    double a = row[j];
#pragma unroll
                    for (int l = 0; l < NB; ++l) a -= vi[l] * Wc[l * N + j] + wi[l] * Vc[l * N + j];
                    row[j] = a;
                }
            }
            __syncthreads();
        }
    } else
    for (int k = 0; k + 2 < N; ++k) {
        // column k below the diagonal: its norm, and the entries of v except the
        // first (v_{k+1} = x0 - alpha is formed where it is used, and stored by
        // thread 0 before the next barrier)
        double s2 = 0.0;
        for (int i = k + 1 + tid; i < N; i += nt) {
            const double x = col(i, k);
            hv[i] = x;
            s2 += x * x;
        }
        s2 = reduce(s2);
        const double x0 = col(k + 1, k);
        const double rest = s2 - x0 * x0;
        if (!(rest > 1e-300 * (s2 > 1.0 ? s2 : 1.0))) {
            if (tid == 0) {
                d[k] = A[a_at<kFull>(k, k, N)];
                e[k] = x0;
            }
            continue;
        }
        const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
        const double bet = 1.0 / (s2 - x0 * alpha);  // 2 / (v^T v)
        const double v1 = x0 - alpha;
        if (tid == 0) hv[k + 1] = v1;
        // p = bet * A22 v and p.v.  Lane gl of a G-lane group takes the columns
        // j = k + 1 + gl + G m of every row, so it loads its v_j once per step into
        // registers; row i reads A[i][j] from the lower triangle (j <= i, contiguous)
        // or its mirror A[j][i], all loads of a row issued before the first product,
        // two rows per group in flight.  Columns j >= N read the valid entry of column
        // N - 1 and meet v_j = 0 (A is finite), so every load is unconditional.  The
        // number of column slots MV is the step's ceil((N - k - 1) / G), chosen from
        // three compiled widths outside the loops.
        double pvl = 0.0;
        auto matvec = [&](auto mvc) {
            constexpr int MV = decltype(mvc)::value;
            double hr[MV];
            int jc[MV], tj[MV];
#pragma unroll
            for (int m = 0; m < MV; ++m) {
                const int j = k + 1 + gl + G * m;
                jc[m] = j < N ? j : N - 1;
                tj[m] = tri(jc[m], 0);
                const double h = hv[jc[m]];
                hr[m] = j < N ? (j == k + 1 ? v1 : h) : 0.0;
            }
            auto row_dot = [&](int i, double (&t)[MV]) {
                const int rb = tri(i, 0);
#pragma unroll
                for (int m = 0; m < MV; ++m) t[m] = A[jc[m] <= i ? rb + jc[m] : tj[m] + i];
            };
            auto finish = [&](int i, double acc) {
                if (gl == 0) {
                    p[i] = bet * acc;
                    pvl += bet * acc * (i == k + 1 ? v1 : hv[i]);
                }
            };
            int i = k + 1 + grp;
            for (; i + ngrp < N; i += 2 * ngrp) {
                double t0[MV], t1[MV];
                row_dot(i, t0);
                row_dot(i + ngrp, t1);
                double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
                for (int m = 0; m < MV; m += 2) {
                    a0 = fma(t0[m], hr[m], a0);
                    b0 = fma(t1[m], hr[m], b0);
                    if (m + 1 < MV) {
                        a1 = fma(t0[m + 1], hr[m + 1], a1);
                        b1 = fma(t1[m + 1], hr[m + 1], b1);
                    }
                }
                const double acc0 = row16_sum(a0 + a1), acc1 = row16_sum(b0 + b1);
                finish(i, acc0);
                finish(i + ngrp, acc1);
            }
            if (i < N) {
                double t0[MV];
                row_dot(i, t0);
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int m = 0; m < MV; m += 2) {
                    a0 = fma(t0[m], hr[m], a0);
                    if (m + 1 < MV) a1 = fma(t0[m + 1], hr[m + 1], a1);
                }
                finish(i, row16_sum(a0 + a1));
            }
        };
        {
            static_assert(KITAEV_LDS_MAX_L * KITAEV_LDS_MAX_L <= 9 * G, "nine column slots cover a row");
            const int nm = (N - k - 1 + G - 1) / G;
            if (nm <= 3)
                matvec(std::integral_constant<int, 3>{});
            else if (nm <= 5)
                matvec(std::integral_constant<int, 5>{});
            else
                matvec(std::integral_constant<int, 9>{});
        }
        const double kk2 = bet * reduce(pvl);  // 2 kk; its barrier publishes p and hv[k + 1]
        // A22 -= v p^T + p v^T - 2 kk v v^T on the lower triangle.  The R = N - k - 1
        // trailing rows are paired, (k + 1 + t, N - 1 - t), a wave per pair; lane q
        // of 64-entry slot c takes column j = k + 1 + q + 64 c in both rows of the
        // pair (the short row ends at its diagonal), so p_j and v_j are read once
        // per step into registers and each entry costs one load and one store
        {
            // a pair's bookkeeping is wave-uniform (scalar); all loads of a pair are
            // issued before its first store, lanes past a row's end reading a valid
            // entry that is not written back.
            static_assert(KITAEV_LDS_MAX_L * KITAEV_LDS_MAX_L < 3 * 64, "a row must fit three slots");
            const int R = N - k - 1, npair = (R + 1) / 2;
            const int top = N * (N + 1) / 2 - 1;
            // slots per pair: ceil(R / 64), the longest row of the step
            auto pairs = [&](auto nslot) {
                constexpr int NSL = decltype(nslot)::value;
                double pj[NSL], vj[NSL];
#pragma unroll
                for (int c = 0; c < NSL; ++c) {
                    const int jj = k + 1 + lane + 64 * c;
                    const int jc = jj < N ? jj : N - 1;
                    pj[c] = p[jc];
                    vj[c] = hv[jc];
                }
                for (int t = __builtin_amdgcn_readfirstlane(wid); t < npair; t += nw) {
                    const int ra = k + 1 + t, rz = N - 1 - t;
                    const int la = t + 1, lz = rz == ra ? 0 : R - t;  // entries of the two rows
                    const int ba = tri(ra, 0) + k + 1, bz = tri(rz, 0) + k + 1;
                    const double va = hv[ra], vz = hv[rz];
                    const double ca = p[ra] - kk2 * va, cz = p[rz] - kk2 * vz;  // p_i - 2 kk v_i
                    double xa[NSL], xz[NSL];
#pragma unroll
                    for (int c = 0; c < NSL; ++c) {
                        const int q = lane + 64 * c;
                        const int ia = ba + q, iz = bz + q;
                        xa[c] = A[ia < top ? ia : top];
                        xz[c] = A[iz < top ? iz : top];
                    }
#pragma unroll
                    for (int c = 0; c < NSL; ++c) {
                        const int q = lane + 64 * c;
                        if (q < la) A[ba + q] = xa[c] - (va * pj[c] + ca * vj[c]);
                        if (q < lz) A[bz + q] = xz[c] - (vz * pj[c] + cz * vj[c]);
                    }
                }
            };
            if (R <= 64)
                pairs(std::integral_constant<int, 1>{});
            else if (R <= 128)
                pairs(std::integral_constant<int, 2>{});
            else
                pairs(std::integral_constant<int, 3>{});
        }
        if (tid == 0) {
            d[k] = A[a_at<kFull>(k, k, N)];
            e[k] = alpha;
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (N >= 2) {
            d[N - 2] = A[a_at<kFull>(N - 2, N - 2, N)];
            e[N - 2] = A[a_at<kFull>(N - 1, N - 2, N)];
        }
        d[N - 1] = A[a_at<kFull>(N - 1, N - 1, N)];
    }
    __syncthreads();
    // 3. the eigenvalues (kitaev_eigs_groups), within the Gershgorin bracket of the
    //    whole spectrum (widened to hold 0): thread t forms e_i^2 and the interval
    //    of rows i = t, t + nt, ..., then a wave min / max and one exchange
    lds_f64* ee = hv;  // e^2, hv is free now
    double* redg = (double*)red;
    double glo = 0.0, ghi = 0.0;
    {
        double lo = 0.0, hi = 0.0;
        for (int i = tid; i < N; i += nt) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - r);
            hi = fmax(hi, d[i] + r);
            if (i + 1 < N) ee[i] = e[i] * e[i];
        }
        lo = wave_min_dpp(lo);
        hi = wave_max_dpp(hi);
        if (lane == 0) {
            redg[wid] = lo;
            redg[nw + wid] = hi;
        }
        __syncthreads();
        for (int w = 0; w < nw; ++w) {
            glo = fmin(glo, redg[w]);
            ghi = fmax(ghi, redg[nw + w]);
        }
        __syncthreads();
    }
    const double tol = 4e-16 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
    const double dlam = kitaev_dlam(N, Jx, Jy, Jz);
    double S = 0.0, Ef = 0.0, Cf = 0.0, Bs = 0.0;
    // the table of the first count pass sits in the dead matrix, past the N eps
    const bool use_tab = !kFull && N * (N + 1) / 2 >= N + kitaev_eig_table_doubles(nt);
    kitaev_eigs_groups(d, ee, N, glo, ghi, tol, beta, dlam, eps_out, S, Ef, Cf, Bs, eps_out + N, use_tab);
    block_sum4(S, Ef, Cf, Bs, redg);
    KitaevOut o;
    o.S = S;
    o.Ef = Ef;
    o.Cf = Cf;
    o.B = dlam * Bs + (double)(N + 4) * 0x1p-53 * o.S;
    return o;
}

// ---------------------------------------------------------------------------
// The same eigen-step for N <= 64 (L <= 8) with a four-wave workgroup:
//   - wave 0 alone assembles A = M^T M (LDS, full, odd row stride) and
//     tridiagonalises it: lane i owns row i, so a Householder step is a wave
//     reduction for the column norm, one row-times-vector product and one
//     rank-2 update of the lane's own row, with the vectors v and w broadcast
//     through LDS; the wave needs no workgroup barrier (wave_sync orders its
//     LDS traffic), and the row loops run in batches of eight loads;
//   - all four waves then bracket the eigenvalues (kitaev_eigs_groups).
// The bound on S is the one of kitaev_weight_block_t.  blockDim.x == 256; v, lds
// and eps_out are LDS addresses.
// ---------------------------------------------------------------------------
constexpr int KITAEV_SMALL_NT = 256;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Householder steps of kitaev_tridiag_wave with the rows in registers (NCT
// columns, N <= NCT <= 40, NCT a multiple of 4): lane i holds row i of the
// trailing matrix; at step k lane k writes its row to cb (A's storage, dead once
// the rows are loaded), from which every lane reads its entry of column k
// (symmetry) and the diagonal; v and w go through LDS as well and are read by
// every lane (broadcast).
// Lanes <= k and >= N get v_i = w_i = 0, so their rows, and the columns j <= k,
// stay as they are; step k therefore touches the columns j >= J0 = 4 floor(k / 4)
// only, and the steps run in stretches of four with J0 known at compile time.
template <int NCT, int J0>
__device__ __forceinline__ void kitaev_tridiag_regs_step(double (&row)[NCT], int k, int N, int lane, lds_f64* cb,
                                                         lds_f64* d, lds_f64* e, lds_f64* vb, lds_f64* wb)
{
    if (lane == k) {
#pragma unroll
        for (int j = J0; j < NCT; ++j) cb[j] = row[j];
    }
    wave_sync();
    const bool act = lane < N && lane > k;
    const double x = act ? cb[lane] : 0.0;
    const double dk = cb[k];
    const double x0 = cb[k + 1];
    const double s2 = wave_sum_dpp(x * x);
    const double rest = s2 - x0 * x0;
    if (!(rest > 1e-300 * (s2 > 1.0 ? s2 : 1.0))) {
        if (lane == 0) {
            d[k] = dk;
            e[k] = x0;
        }
        wave_sync();
        return;
    }
    const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
    const double bet = 1.0 / (s2 - x0 * alpha);  // 2 / (v^T v)
    const double vi = lane == k + 1 ? x0 - alpha : x;
    if (lane < NCT) vb[lane] = vi;
    wave_sync();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    // v is read once and kept for the update.  Beyond 36 columns, eight columns
    // at a time: the scheduler may not hoist the loads of later chunks (their
    // registers would push the rows out of the register file)
    double vv[NCT];
#pragma unroll
    for (int j = J0; j < NCT; j += 4) {
#pragma unroll
        for (int t = 0; t < 4; ++t) vv[j + t] = vb[j + t];
        a0 = fma(row[j], vv[j], a0);
        a1 = fma(row[j + 1], vv[j + 1], a1);
        a2 = fma(row[j + 2], vv[j + 2], a2);
        a3 = fma(row[j + 3], vv[j + 3], a3);
        if (NCT > 36 && (j & 7) == 4) __builtin_amdgcn_sched_barrier(0);
    }
    const double p = act ? bet * ((a0 + a1) + (a2 + a3)) : 0.0;
    const double kk2 = bet * wave_sum_dpp(p * vi);  // 2 kk
    const double wi = act ? p - 0.5 * kk2 * vi : 0.0;
    if (lane < NCT) wb[lane] = wi;
    wave_sync();
#pragma unroll
    for (int j = J0; j < NCT; ++j) {
        row[j] = fma(-vi, wb[j], row[j]);
        row[j] = fma(-wi, vv[j], row[j]);
        if (NCT > 36 && (j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    if (lane == 0) {
        d[k] = dk;
        e[k] = alpha;
    }
    wave_sync();
}

template <int NCT>
__device__ __forceinline__ void kitaev_tridiag_regs(int N, int NS, int lane, lds_f64* A, lds_f64* d, lds_f64* e,
                                                    lds_f64* vb, lds_f64* wb)
{
    double row[NCT];
#pragma unroll
    for (int j = 0; j < NCT; ++j) row[j] = lane < N ? A[lane * NS + j] : 0.0;
    wave_sync();
    lds_f64* cb = A;
    int k = 0;
    auto stretch = [&](auto j0) {
        constexpr int J0 = decltype(j0)::value;
        if constexpr (J0 < NCT)
            for (; k + 2 < N && k < J0 + 4; ++k) kitaev_tridiag_regs_step<NCT, J0>(row, k, N, lane, cb, d, e, vb, wb);
    };
    stretch(std::integral_constant<int, 0>{});
    stretch(std::integral_constant<int, 4>{});
    stretch(std::integral_constant<int, 8>{});
    stretch(std::integral_constant<int, 12>{});
    stretch(std::integral_constant<int, 16>{});
    stretch(std::integral_constant<int, 20>{});
    stretch(std::integral_constant<int, 24>{});
    stretch(std::integral_constant<int, 28>{});
    stretch(std::integral_constant<int, 32>{});
    stretch(std::integral_constant<int, 36>{});
    // the trailing 2 x 2 block (or the single entry for N = 1)
    if (N >= 2) {
        if (lane == N - 2) {
#pragma unroll
            for (int j = 0; j < NCT; ++j) cb[j] = row[j];
        }
        wave_sync();
        if (lane == 0) {
            d[N - 2] = cb[N - 2];
            e[N - 2] = cb[N - 1];
        }
        wave_sync();
    }
    if (lane == N - 1) {
#pragma unroll
        for (int j = 0; j < NCT; ++j) cb[j] = row[j];
    }
    wave_sync();
    if (lane == 0) d[N - 1] = cb[N - 1];
    wave_sync();
}

__device__ __noinline__ void kitaev_tridiag_wave(lds_u8c* v, int C, int L, int open_cols, double Jx, double Jy,
                                                 double Jz, lds_f64* A, lds_f64* d, lds_f64* e, lds_f64* vb,
                                                 lds_f64* wb)
{
    const int N = L * L, NS = kitaev_wave_stride(N), NC = kitaev_wave_cols(N);
    const int lane = threadIdx.x & 63;
    // 1. A = M^T M; lane w fills A[w][w2] for w2 <= w and the mirror A[w2][w] (w2 < w),
    //    which no other lane writes.  Rows are zero up to NC columns, and so are v and w
    //    beyond N: the row loops then run whole batches of eight from an aligned start,
    //    the entries j <= k of v and w being zero as well
    if (lane < N)
        for (int q = 0; q < NS; ++q) A[lane * NS + q] = 0.0;
    if (lane >= N && lane < NC) {
        vb[lane] = 0.0;
        wb[lane] = 0.0;
    }
    wave_sync();
    if (lane < N) {
        const int w = lane;
        const int i = w / L, j = w - (w / L) * L;
        int bn[3];
        bn[0] = w;
        bn[1] = j == 0 ? (open_cols ? -1 : i * L + L - 1) : i * L + j - 1;
        bn[2] = (i == 0 ? L - 1 : i - 1) * L + j;
        for (int nb = 0; nb < 3; ++nb) {
            const int b = bn[nb];
            if (b < 0) continue;
            bool dup = false;
            for (int t = 0; t < nb; ++t) dup |= (bn[t] == b);
            if (dup) continue;
            const int bi = b / L, bj = b - (b / L) * L;
            int wn[3];
            double wv[3];
            wn[0] = b;
            wn[1] = bj + 1 == L ? (open_cols ? -1 : bi * L) : bi * L + bj + 1;
            wn[2] = (bi + 1 == L ? 0 : bi + 1) * L + bj;
            const double vz = C == 3 ? (v[2 * N + b] ? 1.0 : -1.0) : (v[b] ? 1.0 : -1.0);
            const double vx = C == 3 ? (v[0 * N + b] ? 1.0 : -1.0) : 1.0;
            const double vy = C == 3 ? (v[1 * N + b] ? 1.0 : -1.0) : 1.0;
            wv[0] = 2.0 * Jz * vz;
            wv[1] = 2.0 * Jx * vx;
            wv[2] = 2.0 * Jy * vy;
            double mbw = 0.0;
            for (int t = 0; t < 3; ++t)
                if (wn[t] == w) mbw += wv[t];
            for (int t = 0; t < 3; ++t) {
                const int w2 = wn[t];
                if (w2 < 0) continue;
                bool dupw = false;
                for (int s2 = 0; s2 < t; ++s2) dupw |= (wn[s2] == w2);
                if (dupw || w2 > w) continue;
                double mbw2 = 0.0;
                for (int s2 = 0; s2 < 3; ++s2)
                    if (wn[s2] == w2) mbw2 += wv[s2];
                A[w * NS + w2] += mbw * mbw2;
                if (w2 != w) A[w2 * NS + w] += mbw * mbw2;
            }
        }
    }
    wave_sync();
    // 2. Householder: step k annihilates column k below the subdiagonal; up to
    //    40 columns (L <= 6) with the rows in registers
    if (NC <= 8) return kitaev_tridiag_regs<8>(N, NS, lane, A, d, e, vb, wb);
    if (NC <= 16) return kitaev_tridiag_regs<16>(N, NS, lane, A, d, e, vb, wb);
    if (N <= 28) return kitaev_tridiag_regs<28>(N, NS, lane, A, d, e, vb, wb);
    if (N <= 36) return kitaev_tridiag_regs<36>(N, NS, lane, A, d, e, vb, wb);
    if (NC <= 40) return kitaev_tridiag_regs<40>(N, NS, lane, A, d, e, vb, wb);
    lds_f64* row = A + (lane < N ? lane : 0) * NS;
    const bool own = lane < N;
    for (int k = 0; k + 2 < N; ++k) {
        const bool act = own && lane > k;
        const double x = act ? row[k] : 0.0;
        const double s2 = wave_sum_dpp(x * x);
        const double x0 = readlane_t(x, k + 1);
        const double rest = s2 - x0 * x0;
        if (!(rest > 1e-300 * (s2 > 1.0 ? s2 : 1.0))) {
            if (lane == 0) {
                d[k] = A[k * NS + k];
                e[k] = x0;
            }
            continue;
        }
        const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
        const double bet = 1.0 / (s2 - x0 * alpha);  // 2 / (v^T v)
        const double vi = lane == k + 1 ? x0 - alpha : x;
        if (own) vb[lane] = vi;
        wave_sync();
        // v_j = 0 for j <= k and j >= N, so the batches start at the aligned column below k + 1
        const int j0 = (k + 1) & ~7;
        double p = 0.0;
        if (act) {
            double a[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) a[t] = 0.0;
            for (int jj = j0; jj < NC; jj += 8) {
                double r8[8], v8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    r8[t] = row[jj + t];
                    v8[t] = vb[jj + t];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) a[t] = fma(r8[t], v8[t], a[t]);
            }
            p = bet * (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
        }
        const double kk2 = bet * wave_sum_dpp(p * vi);  // 2 kk
        const double wi = p - 0.5 * kk2 * vi;
        if (own) wb[lane] = wi;
        wave_sync();
        if (act) {
            // the entries j <= k and j >= N get v_j = w_j = 0: written back unchanged
            for (int jj = j0; jj < NC; jj += 8) {
                double r8[8], v8[8], w8[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    r8[t] = row[jj + t];
                    v8[t] = vb[jj + t];
                    w8[t] = wb[jj + t];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) row[jj + t] = r8[t] - (vi * w8[t] + wi * v8[t]);
            }
        }
        if (lane == 0) {
            d[k] = A[k * NS + k];
            e[k] = alpha;
        }
        wave_sync();
    }
    if (lane == 0) {
        if (N >= 2) {
            d[N - 2] = A[(N - 2) * NS + N - 2];
            e[N - 2] = A[(N - 1) * NS + N - 2];
        }
        d[N - 1] = A[(N - 1) * NS + N - 1];
    }
    wave_sync();
}

// No side work for the waves that wait on the tridiagonal form
struct KitaevNoSide {
    __device__ double operator()(int, int) const { return 0.0; }
};

// Side: work for waves 1..3 while wave 0 tridiagonalises; thread tid - 64 of the
// 192 calls side(tid - 64, 192) and the returned shares are summed over the
// workgroup into side_sum (KitaevNoSide: nothing, side_sum untouched).
template <class Side>
__device__ __noinline__ KitaevOut kitaev_weight_small(const uint8_t* v_, int C, int L, int open_cols, double Jx,
                                                      double Jy, double Jz, double beta, double* lds, double* eps_out,
                                                      double* red, Side side, double& side_sum)
{
    const int N = L * L, NS = kitaev_wave_stride(N);
    const int tid = threadIdx.x, wid = tid >> 6;
    lds_u8c* v = (lds_u8c*)v_;
    const int NC = kitaev_wave_cols(N);
    lds_f64* A = (lds_f64*)lds;
    lds_f64* d = A + N * NS;
    lds_f64* e = d + N;
    lds_f64* ee = e + N;
    lds_f64* vb = ee + N;
    lds_f64* wb = vb + NC;
    lds_f64* eps_l = (lds_f64*)eps_out;
    double side_part = 0.0;
    if (wid != 0) side_part = side(tid - 64, (int)blockDim.x - 64);
    if (wid == 0) {
        kitaev_tridiag_wave(v, C, L, open_cols, Jx, Jy, Jz, A, d, e, vb, wb);
        // e^2 for the Sturm counts and the Gershgorin bracket of the whole
        // spectrum (widened to hold 0), lane i taking row i; vb is free again
        const int lane = tid;
        double lo = 0.0, hi = 0.0;
        if (lane < N) {
            const double r = (lane > 0 ? fabs(e[lane - 1]) : 0.0) + (lane + 1 < N ? fabs(e[lane]) : 0.0);
            lo = d[lane] - r;
            hi = d[lane] + r;
            if (lane + 1 < N) ee[lane] = e[lane] * e[lane];
        }
        lo = wave_min_dpp(lo);
        hi = wave_max_dpp(hi);
        if (lane == 0) {
            vb[0] = lo;
            vb[1] = hi;
        }
    }
    __syncthreads();
    const double glo = vb[0], ghi = vb[1];
    const double tol = 4e-16 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
    const double dlam = kitaev_dlam(N, Jx, Jy, Jz);
    double S = 0.0, Ef = 0.0, Cf = 0.0, Bs = 0.0;
    // the table of the first count pass sits in the dead matrix, past the N eps
    const bool use_tab = N * NS >= N + kitaev_eig_table_doubles((int)blockDim.x);
    kitaev_eigs_groups(d, ee, N, glo, ghi, tol, beta, dlam, eps_l, S, Ef, Cf, Bs, A + N, use_tab);
    block_sum4(S, Ef, Cf, Bs, red);
    if constexpr (!std::is_same<Side, KitaevNoSide>::value) side_sum = block_sum(side_part, red);
    KitaevOut o;
    o.S = S;
    o.Ef = Ef;
    o.Cf = Cf;
    o.B = dlam * Bs + (double)(N + 4) * 0x1p-53 * o.S;
    return o;
}

// S, E_f, C_f of the proposal v; the eigenvalues eps_lambda go to b.eps.  BLOCK
// is the caller's compile-time workgroup size: only 256-thread kernels reach the
// four-wave path, so its out-of-line functions get the register budget of a
// 256-thread workgroup rather than the 128 VGPRs of a 1024-thread one.
template <int BLOCK>
__device__ inline KitaevOut kitaev_weight_block(const uint8_t* v, int C, int L, int open_cols, double Jx, double Jy,
                                                double Jz, double beta, const KitaevBufs& b, double* red)
{
    if constexpr (BLOCK == KITAEV_SMALL_NT) {
        if (L * L <= KITAEV_WAVE_MAX_N) {
            double unused = 0.0;
            return kitaev_weight_small(v, C, L, open_cols, Jx, Jy, Jz, beta, b.eps, b.eps, red, KitaevNoSide{},
                                       unused);
        }
    }
    lds_u8c* vl = (lds_u8c*)v;
    constexpr bool kNarrow = BLOCK > 512;
    if (kitaev_a_in_lds(L))
        return kitaev_weight_block_t<false, kNarrow>(vl, C, L, open_cols, Jx, Jy, Jz, beta, (lds_f64*)b.A,
                                                     (lds_f64*)b.d, (lds_f64*)b.e, (lds_f64*)b.hv, (lds_f64*)b.p,
                                                     (lds_f64*)red, (lds_f64*)b.eps, nullptr);
    return kitaev_weight_block_t<true, kNarrow>(vl, C, L, open_cols, Jx, Jy, Jz, beta, (glb_f64*)b.A, (lds_f64*)b.d,
                                                (lds_f64*)b.e, (lds_f64*)b.hv, (lds_f64*)b.p, (lds_f64*)red,
                                                (lds_f64*)b.eps, (lds_f64*)b.vw);
}

// ---------------------------------------------------------------------------
// The re-check route: S, E_f, C_f from the singular values of M itself by
// one-sided (Hestenes) Jacobi, which never forms M^T M.  M is built column-major
// in the chain's global scratch Mc (N x N doubles); column pairs are
// orthogonalised in the round-robin order of a tournament (N' = N rounded up
// to even players, player N' - 1 fixed, the others rotating), so the N'/2
// pairs of a round are disjoint and run one per wave; a pair is rotated when
// |x_p . x_q| > 1e-15 |x_p| |x_q|, and the sweeps stop once a whole sweep
// rotates nothing (60 at most).  The singular values are then the column norms;
// they go to eps_out (LDS or global).  Slow (O(N^3) per sweep) and only used for
// the rare MH decisions inside the band of B_S.  nt a multiple of 64.
// ---------------------------------------------------------------------------
constexpr int KITAEV_JAC_MAXR = (KITAEV_MAX_L * KITAEV_MAX_L + 63) / 64;  // rows per lane

__device__ __noinline__ KitaevOut kitaev_weight_jacobi(const uint8_t* v, int C, int L, int open_cols, double Jx, double Jy,
                                          double Jz, double beta, double* __restrict__ Mc, double* eps_out,
                                          double* red, int* flag)
{
    const int N = L * L;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
    // M[b][w] at Mc[w N + b]; thread b fills row b (its three bonds), so no two
    // threads write one element
    for (int q = tid; q < N * N; q += nt) Mc[q] = 0.0;
    __syncthreads();
    for (int b = tid; b < N; b += nt) {
        const int i = b / L, j = b - (b / L) * L;
        const double sz = (C == 3 ? v[2 * N + b] : v[b]) ? 1.0 : -1.0;
        const double sx = C == 3 ? (v[b] ? 1.0 : -1.0) : 1.0;
        const double sy = C == 3 ? (v[N + b] ? 1.0 : -1.0) : 1.0;
        Mc[(size_t)b * N + b] += 2.0 * Jz * sz;
        if (!(open_cols && j == L - 1)) Mc[(size_t)(i * L + (j + 1 == L ? 0 : j + 1)) * N + b] += 2.0 * Jx * sx;
        Mc[(size_t)((i + 1 == L ? 0 : i + 1) * L + j) * N + b] += 2.0 * Jy * sy;
    }
    __syncthreads();
    const int Np = N + (N & 1);
    const int half = Np >> 1;
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int r = 0; r + 1 < Np; ++r) {
            for (int k = wid; k < half; k += nw) {
                // players k and Np - 1 - k of round r
                const int a = k, bq = Np - 1 - k;
                int p = a == Np - 1 ? a : (a + r) % (Np - 1);
                int q = bq == Np - 1 ? bq : (bq + r) % (Np - 1);
                if (p >= N || q >= N) continue;  // the idle player of an odd N
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double* xp = Mc + (size_t)p * N;
                double* xq = Mc + (size_t)q * N;
                double cp[KITAEV_JAC_MAXR], cq[KITAEV_JAC_MAXR];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int m = 0; m < KITAEV_JAC_MAXR; ++m) {
                    const int row = lane + 64 * m;
                    cp[m] = row < N ? xp[row] : 0.0;
                    cq[m] = row < N ? xq[row] : 0.0;
                    al += cp[m] * cp[m];
                    be += cq[m] * cq[m];
                    ga += cp[m] * cq[m];
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                rotated = 1;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
                for (int m = 0; m < KITAEV_JAC_MAXR; ++m) {
                    const int row = lane + 64 * m;
                    if (row < N) {
                        xp[row] = cs * cp[m] - sn * cq[m];
                        xq[row] = sn * cp[m] + cs * cq[m];
                    }
                }
            }
            __syncthreads();
        }
        // stop after a sweep without rotations (every wave has seen the same rounds)
        if (tid == 0) *flag = 0;
        __syncthreads();
        if (rotated && lane == 0) atomicOr(flag, 1);
        __syncthreads();
        const int any = *flag;
        __syncthreads();
        if (!any) break;
    }
    // column norms: one wave per column
    double S = 0.0, Ef = 0.0, Cf = 0.0;
    for (int c = wid; c < N; c += nw) {
        const double* xc = Mc + (size_t)c * N;
        double s2 = 0.0;
        for (int row = lane; row < N; row += 64) s2 += xc[row] * xc[row];
        s2 = wave_sum(s2);
        if (lane == 0) {
            const double eps = sqrt(s2);
            eps_out[c] = eps;
            const double xv = 0.5 * beta * eps;
            S += log2cosh_d(xv);
            Ef -= 0.5 * eps * tanh(xv);
            const double ch = cosh(xv);
            Cf += (xv * xv) / (ch * ch);
        }
    }
    KitaevOut o;
    o.S = block_sum(S, red);
    o.Ef = block_sum(Ef, red);
    o.Cf = block_sum(Cf, red);
    o.B = 0.0;
    return o;
}

}  // namespace crbm
