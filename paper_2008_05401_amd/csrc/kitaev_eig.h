// kitaev_eig.h -- workgroup-cooperative FP64 gauge-field weight of the Kitaev
// honeycomb model (Sec. IV): S(u) = sum_lambda log 2cosh(beta eps_lambda / 2)
// over the singular values eps of the Majorana hopping block M (N x N, N=L^2).
//
// GPU method (differs from a one-sided Jacobi SVD on purpose):
//   1. A = M^T M is assembled directly from the bond variables (each white
//      site has three black neighbours, so A has at most 7 non-zeros per row);
//      A is held in LDS as a packed lower triangle (N(N+1)/2 doubles);
//   2. Householder reduction of A to a symmetric tridiagonal matrix (d, e);
//   3. every eigenvalue lambda_i of the tridiagonal matrix by bisection on the
//      Sturm count, one thread per eigenvalue;
//   4. eps_i = sqrt(max(lambda_i, 0)); S, the fermion energy and the
//      fluctuation term are reduced over the workgroup.
// Eigenvalues of A are accurate to ~N * 2^-52 * |A| in absolute terms; since
// S depends on eps only through log 2cosh(beta eps / 2), whose derivative in
// lambda is bounded by beta^2 / 8, the error of S stays far below 1e-6.
#pragma once
#include "device_common.h"

namespace crbm {

__device__ __forceinline__ int tri(int i, int j) { return (i * (i + 1) >> 1) + j; }  // j <= i
__device__ __forceinline__ int tri_s(int i, int j) { return i >= j ? tri(i, j) : tri(j, i); }

struct KitaevOut {
    double S, Ef, Cf;
};

// LDS needs: A[N(N+1)/2], d[N], e[N], hv[N], p[N] doubles and `red` (>= 16 doubles).
// v: 0/1 bytes of the proposal, C channels ([3][L][L] = x,y,z bonds, or [1][L][L] = z bonds).
__device__ KitaevOut kitaev_weight_block(const uint8_t* v, int C, int L, double Jx, double Jy, double Jz,
                                         double beta, double* A, double* d, double* e, double* hv, double* p,
                                         double* red, double* eps_out = nullptr)
{
    const int N = L * L;
    const int tid = threadIdx.x, nt = blockDim.x;
    // 1. A = M^T M, row w owned by one thread
    for (int w = tid; w < N; w += nt) {
        for (int q = 0; q <= w; ++q) A[tri(w, q)] = 0.0;
    }
    __syncthreads();
    for (int w = tid; w < N; w += nt) {
        const int i = w / L, j = w - (w / L) * L;
        // black neighbours of w(i,j): b(i,j) via z, b(i,j-1) via x, b(i-1,j) via y
        int bn[3];
        bn[0] = w;
        bn[1] = i * L + (j == 0 ? L - 1 : j - 1);
        bn[2] = (i == 0 ? L - 1 : i - 1) * L + j;
        for (int nb = 0; nb < 3; ++nb) {
            const int b = bn[nb];
            const int bi = b / L, bj = b - (b / L) * L;
            // white neighbours of b(bi,bj) and the matrix entries M[b][w']
            int wn[3];
            double wv[3];
            wn[0] = b;
            wn[1] = bi * L + (bj + 1 == L ? 0 : bj + 1);
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
                bool dupw = false;
                for (int s = 0; s < t; ++s) dupw |= (wn[s] == w2);
                if (dupw || w2 > w) continue;
                double mbw2 = 0.0;
                for (int s = 0; s < 3; ++s)
                    if (wn[s] == w2) mbw2 += wv[s];
                A[tri(w, w2)] += mbw * mbw2;
            }
        }
    }
    __syncthreads();

    // 2. Householder tridiagonalisation of the packed symmetric A
    for (int k = 0; k + 2 < N; ++k) {
        double s2 = 0.0;
        for (int i = k + 1 + tid; i < N; i += nt) {
            const double x = A[tri(i, k)];
            s2 += x * x;
        }
        s2 = block_sum(s2, red);
        const double x0 = A[tri(k + 1, k)];
        const double rest = s2 - x0 * x0;
        if (!(rest > 1e-300 * (s2 > 1.0 ? s2 : 1.0))) {
            if (tid == 0) {
                d[k] = A[tri(k, k)];
                e[k] = x0;
            }
            continue;
        }
        const double alpha = x0 > 0.0 ? -sqrt(s2) : sqrt(s2);
        const double bet = 1.0 / (s2 - x0 * alpha);  // 2 / (v^T v)
        for (int i = k + 1 + tid; i < N; i += nt) hv[i] = (i == k + 1) ? (x0 - alpha) : A[tri(i, k)];
        __syncthreads();
        // p = bet * A22 v
        for (int i = k + 1 + tid; i < N; i += nt) {
            double acc = 0.0;
            for (int j = k + 1; j <= i; ++j) acc += A[tri(i, j)] * hv[j];
            for (int j = i + 1; j < N; ++j) acc += A[tri(j, i)] * hv[j];
            p[i] = bet * acc;
        }
        __syncthreads();
        double pv = 0.0;
        for (int i = k + 1 + tid; i < N; i += nt) pv += p[i] * hv[i];
        pv = block_sum(pv, red);
        const double kk = 0.5 * bet * pv;
        for (int i = k + 1 + tid; i < N; i += nt) p[i] -= kk * hv[i];  // p := w
        __syncthreads();
        // A22 -= v w^T + w v^T (lower triangle)
        const int m = N - k - 1;
        const int cnt = m * (m + 1) / 2;
        for (int idx = tid; idx < cnt; idx += nt) {
            // invert idx -> (ii, jj) with jj <= ii inside the trailing block
            int ii = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            while ((ii + 1) * (ii + 2) / 2 <= idx) ++ii;
            while (ii * (ii + 1) / 2 > idx) --ii;
            const int jj = idx - ii * (ii + 1) / 2;
            const int gi = ii + k + 1, gj = jj + k + 1;
            A[tri(gi, gj)] -= hv[gi] * p[gj] + p[gi] * hv[gj];
        }
        if (tid == 0) {
            d[k] = A[tri(k, k)];
            e[k] = alpha;
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (N >= 2) {
            d[N - 2] = A[tri(N - 2, N - 2)];
            e[N - 2] = A[tri(N - 1, N - 2)];
        }
        d[N - 1] = A[tri(N - 1, N - 1)];
    }
    __syncthreads();

    // 3. bisection, one thread per eigenvalue
    double S = 0.0, Ef = 0.0, Cf = 0.0;
    for (int idx = tid; idx < N; idx += nt) {
        double lo = 0.0, hi = 0.0;
        for (int i = 0; i < N; ++i) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < N ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - r);
            hi = fmax(hi, d[i] + r);
        }
        const double scale = fmax(fabs(lo), fabs(hi));
        const double pivmin = 1e-290 * fmax(1.0, scale * scale);
        lo -= 1e-14 * scale + 1e-300;
        hi += 1e-14 * scale + 1e-300;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (!(hi - lo > 4e-16 * scale + pivmin) || mid == lo || mid == hi) break;
            // number of eigenvalues < mid
            int count = 0;
            double q = d[0] - mid;
            if (fabs(q) < pivmin) q = -pivmin;
            count += q < 0.0;
            for (int i = 1; i < N; ++i) {
                q = d[i] - mid - e[i - 1] * e[i - 1] / q;
                if (fabs(q) < pivmin) q = -pivmin;
                count += q < 0.0;
            }
            if (count > idx) hi = mid;
            else lo = mid;
        }
        const double lam = 0.5 * (lo + hi);
        const double eps = sqrt(lam > 0.0 ? lam : 0.0);
        if (eps_out) eps_out[idx] = eps;  // may alias A: A is dead after the tridiagonalisation
        const double x = 0.5 * beta * eps;
        S += log2cosh_d(x);
        Ef -= 0.5 * eps * tanh(x);
        const double ch = cosh(x);
        Cf += (x * x) / (ch * ch);
    }
    KitaevOut o;
    o.S = block_sum(S, red);
    o.Ef = block_sum(Ef, red);
    o.Cf = block_sum(Cf, red);
    return o;
}

__host__ __device__ inline size_t kitaev_lds_bytes(int L)
{
    const size_t N = (size_t)L * L;
    return sizeof(double) * (N * (N + 1) / 2 + 4 * N);
}

}  // namespace crbm
