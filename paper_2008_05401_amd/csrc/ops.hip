// ops.hip -- stand-alone kernels of the C ABI: batched CRBM free energy,
// target energies (Ising E, Kitaev S) and the backward of F.  The CRBM may be
// the locally connected one of Sec. IV.B: `banks` = 1 + 2 ne filter banks
// ([banks][K][C][LW][LW], hidden biases [banks][K]), bank 0 for the bulk
// columns, banks 1..ne for the hidden columns 0..ne-1 and ne+1..2ne for
// L-ne..L-1; with `open` the windows stop at the column edge.
#include <mutex>

#include "device_common.h"
#include "kitaev_eig.h"
#include "ops.h"

namespace crbm {

__device__ __forceinline__ int bank_of_col(int j, int L, int ne)
{
    return j < ne ? 1 + j : (j >= L - ne ? 1 + ne + (j - (L - ne)) : 0);
}

// hidden columns [j0, j1) owned by filter bank `bank`
__device__ __forceinline__ void bank_columns(int bank, int L, int ne, int& j0, int& j1)
{
    if (bank == 0) {
        j0 = ne;
        j1 = L - ne;
    } else if (bank <= ne) {
        j0 = bank - 1;
        j1 = bank;
    } else {
        j0 = L - ne + (bank - ne - 1);
        j1 = j0 + 1;
    }
}

// ---------------------------------------------------------------------------
// F(x_b) of Eq. (free-energy_CRBM), FP64 terms and sums; one workgroup per state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void free_energy_kernel(const float* __restrict__ W, const float* __restrict__ hb,
                                                          const float* __restrict__ vb, int K, int C, int LW, int open,
                                                          int ne, const int8_t* __restrict__ x, int L,
                                                          double* __restrict__ F)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int LL = L * L, nW = K * C * LW * LW, nb = 1 + 2 * ne;
    double* red = (double*)smem;
    double* Wd = red + 64;
    double* hbd = Wd + nb * nW;
    uint8_t* v = (uint8_t*)(hbd + nb * K);
    const int8_t* xs = x + (size_t)blockIdx.x * C * LL;
    for (int q = threadIdx.x; q < nb * nW; q += blockDim.x) Wd[q] = (double)W[q];
    for (int q = threadIdx.x; q < nb * K; q += blockDim.x) hbd[q] = (double)hb[q];
    for (int q = threadIdx.x; q < C * LL; q += blockDim.x) v[q] = xs[q] > 0;
    __syncthreads();
    double fl = 0.0;
    for (int q = threadIdx.x; q < K * LL; q += blockDim.x) {
        const int k = q / LL, r = q - k * LL, i = r / L, j = r - i * L;
        const int bk = bank_of_col(j, L, ne);
        const int taps = open ? min(LW, L - j) : LW;  // window offsets inside the lattice
        double acc = hbd[bk * K + k];
        for (int c = 0; c < C; ++c)
            for (int a = 0; a < LW; ++a) {
                int ia = i + a;
                if (ia >= L) ia -= L;
                const uint8_t* row = v + (c * L + ia) * L;
                const double* wr = Wd + bk * nW + ((k * C + c) * LW + a) * LW;
                for (int b = 0; b < taps; ++b) {
                    int jb = j + b;
                    if (jb >= L) jb -= L;
                    acc += row[jb] ? wr[b] : 0.0;
                }
            }
        fl -= softplus_d(acc);
    }
    for (int q = threadIdx.x; q < C * LL; q += blockDim.x) fl -= (double)vb[q / LL] * (double)v[q];
    const double tot = block_sum(fl, red);
    if (threadIdx.x == 0) F[blockIdx.x] = tot;
}

// F of the fully connected RBM (Sec. IV comparison): W[K][nv], hbias[K],
// vbias[nv], nv = C L^2; FP64 terms and sums, one workgroup per state.
__global__ __launch_bounds__(256) void free_energy_dense_kernel(const float* __restrict__ W,
                                                                const float* __restrict__ hb,
                                                                const float* __restrict__ vb, int K, int nv,
                                                                const int8_t* __restrict__ x, double* __restrict__ F)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* red = (double*)smem;
    uint8_t* v = (uint8_t*)(red + 64);
    const int8_t* xs = x + (size_t)blockIdx.x * nv;
    for (int q = threadIdx.x; q < nv; q += blockDim.x) v[q] = xs[q] > 0;
    __syncthreads();
    double fl = 0.0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float* w = W + (size_t)k * nv;
        double acc = (double)hb[k];
        for (int q = 0; q < nv; ++q) acc += v[q] ? (double)w[q] : 0.0;
        fl -= softplus_d(acc);
    }
    for (int q = threadIdx.x; q < nv; q += blockDim.x) fl -= (double)vb[q] * (double)v[q];
    const double tot = block_sum(fl, red);
    if (threadIdx.x == 0) F[blockIdx.x] = tot;
}

size_t free_energy_dense_lds(int nv) { return 64 * 8 + (size_t)nv + 16; }

hipError_t launch_free_energy_dense(const float* W, const float* hb, const float* vb, int K, int nv, const int8_t* x,
                                    int B, double* F, hipStream_t s)
{
    hipLaunchKernelGGL(free_energy_dense_kernel, dim3(B), dim3(256), free_energy_dense_lds(nv), s, W, hb, vb, K, nv, x,
                       F);
    return hipGetLastError();
}

size_t free_energy_lds(int K, int C, int LW, int L, int banks)
{
    return 64 * 8 + (size_t)banks * (K * C * LW * LW + K) * 8 + (size_t)C * L * L + 16;
}

hipError_t launch_free_energy(const float* W, const float* hb, const float* vb, int K, int C, int LW, int open, int ne,
                              const int8_t* x, int B, int L, double* F, hipStream_t s)
{
    hipLaunchKernelGGL(free_energy_kernel, dim3(B), dim3(256), free_energy_lds(K, C, LW, L, 1 + 2 * ne), s, W, hb, vb,
                       K, C, LW, open, ne, x, L, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ising E/J = -sum_<ij> s_i s_j, exact int32; one workgroup per state.  With
// open_cols the bond from column L-1 to column 0 is absent.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void ising_energy_kernel(const int8_t* __restrict__ x, int L, int open_cols,
                                                           int32_t* __restrict__ E)
{
    __shared__ int red[16];
    const int LL = L * L;
    const int8_t* s = x + (size_t)blockIdx.x * LL;
    int el = 0;
    for (int q = threadIdx.x; q < LL; q += blockDim.x) {
        const int i = q / L, j = q - i * L;
        const int right = (open_cols && j + 1 == L) ? 0 : (int)s[i * L + (j + 1 == L ? 0 : j + 1)];
        el -= (int)s[q] * ((int)s[(i + 1 == L ? 0 : i + 1) * L + j] + right);
    }
    const int tot = block_sum(el, red);
    if (threadIdx.x == 0) E[blockIdx.x] = tot;
}

hipError_t launch_ising_energy(const int8_t* x, int B, int L, int open_cols, int32_t* E, hipStream_t s)
{
    hipLaunchKernelGGL(ising_energy_kernel, dim3(B), dim3(256), 0, s, x, L, open_cols, E);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kitaev S = sum log 2cosh(eps / 2T), FP64; one workgroup per configuration.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void kitaev_weight_kernel(const int8_t* __restrict__ x, int C, int L, int open_cols,
                                                          double Jx, double Jy, double Jz,
                                                          const double* __restrict__ T, double* __restrict__ S)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = L * L;
    double* red = (double*)smem;
    double* A = red + 64;
    uint8_t* v = (uint8_t*)A + kitaev_lds_bytes(L);  // past every layout of the eigen-step
    const int8_t* xs = x + (size_t)blockIdx.x * C * N;
    for (int q = threadIdx.x; q < C * N; q += blockDim.x) v[q] = xs[q] > 0;
    __syncthreads();
    // the stand-alone op keeps A in LDS (L <= 12)
    const KitaevOut o = kitaev_weight_block<NT>(v, C, L, open_cols, Jx, Jy, Jz, 1.0 / T[blockIdx.x],
                                                kitaev_bufs(A, nullptr, L), red);
    if (threadIdx.x == 0) S[blockIdx.x] = o.S;
}

size_t kitaev_weight_lds(int C, int L) { return 64 * 8 + kitaev_lds_bytes(L) + (size_t)C * L * L + 16; }

hipError_t launch_kitaev_weight(const int8_t* x, int B, int C, int L, int open_cols, double Jx, double Jy, double Jz,
                                const double* T, double* S, hipStream_t s)
{
    if (L * L >= 16)
        hipLaunchKernelGGL(kitaev_weight_kernel<1024>, dim3(B), dim3(1024), kitaev_weight_lds(C, L), s, x, C, L,
                           open_cols, Jx, Jy, Jz, T, S);
    else
        hipLaunchKernelGGL(kitaev_weight_kernel<256>, dim3(B), dim3(256), kitaev_weight_lds(C, L), s, x, C, L,
                           open_cols, Jx, Jy, Jz, T, S);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Backward of F.  Stage 1 (one workgroup per sample b): sigma(a) of every
// hidden unit from its FP64 pre-activation, kept in LDS as FP64 (as float32
// when K L^2 doubles do not fit, `sig64` = 0), then one thread per parameter p
// forms g_b dF(x_b)/dtheta_p in FP64 into part[b][p].  Stage 2: out[p] =
// sum_b part[b][p] in sample order, rounded once to float32.
// Parameters are ordered W[banks][K][C][LW][LW], hbias[banks][K], vbias[C];
// a bank's gradient sums over the hidden columns that bank owns.
// ---------------------------------------------------------------------------
template <typename SigT>
__device__ void grad_stage1_body(const float* __restrict__ W, const float* __restrict__ hb, int K, int C, int LW,
                                 int open, int ne, const int8_t* __restrict__ x, int L, const float* __restrict__ gF,
                                 double* __restrict__ part, unsigned char* smem)
{
    const int nb = 1 + 2 * ne;
    const int LL = L * L, nW = K * C * LW * LW, P = nb * (nW + K) + C;
    SigT* sg = (SigT*)smem;
    float* Ws = (float*)(sg + K * LL);
    uint8_t* v = (uint8_t*)(Ws + nb * nW);
    const int8_t* xs = x + (size_t)blockIdx.x * C * LL;
    for (int q = threadIdx.x; q < nb * nW; q += blockDim.x) Ws[q] = W[q];
    for (int q = threadIdx.x; q < C * LL; q += blockDim.x) v[q] = xs[q] > 0;
    __syncthreads();
    for (int q = threadIdx.x; q < K * LL; q += blockDim.x) {
        const int k = q / LL, r = q - k * LL, i = r / L, j = r - i * L;
        const int bk = bank_of_col(j, L, ne);
        const int taps = open ? min(LW, L - j) : LW;
        double acc = (double)hb[bk * K + k];
        for (int c = 0; c < C; ++c)
            for (int a = 0; a < LW; ++a) {
                int ia = i + a;
                if (ia >= L) ia -= L;
                const uint8_t* row = v + (c * L + ia) * L;
                const float* wr = Ws + bk * nW + ((k * C + c) * LW + a) * LW;
                for (int b = 0; b < taps; ++b) {
                    int jb = j + b;
                    if (jb >= L) jb -= L;
                    if (row[jb]) acc += (double)wr[b];
                }
            }
        sg[q] = (SigT)(1.0 / (1.0 + exp(-acc)));
    }
    __syncthreads();
    const double gb = (double)gF[blockIdx.x];
    double* out = part + (size_t)blockIdx.x * P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        double s = 0.0;
        if (p < nb * nW) {
            const int bank = p / nW, pw = p - bank * nW;
            const int b = pw % LW, a = (pw / LW) % LW, c = (pw / (LW * LW)) % C, k = pw / (C * LW * LW);
            const SigT* sk = sg + k * LL;
            // hidden columns of this bank whose tap b stays inside the lattice
            int j0, j1;
            bank_columns(bank, L, ne, j0, j1);
            if (open) j1 = min(j1, L - b);
            for (int i = 0; i < L; ++i) {
                int ia = i + a;
                if (ia >= L) ia -= L;
                const uint8_t* row = v + (c * L + ia) * L;
                const SigT* srow = sk + i * L;
                for (int j = j0; j < j1; ++j) {
                    int jb = j + b;
                    if (jb >= L) jb -= L;
                    s += row[jb] ? (double)srow[j] : 0.0;
                }
            }
        } else if (p < nb * (nW + K)) {
            const int q0 = p - nb * nW, bank = q0 / K, k = q0 - bank * K;
            const SigT* sk = sg + k * LL;
            int j0, j1;
            bank_columns(bank, L, ne, j0, j1);
            for (int i = 0; i < L; ++i)
                for (int j = j0; j < j1; ++j) s += (double)sk[i * L + j];
        } else {
            const uint8_t* vc = v + (p - nb * (nW + K)) * LL;
            for (int q = 0; q < LL; ++q) s += (double)vc[q];
        }
        out[p] = -gb * s;
    }
}

__global__ __launch_bounds__(256) void grad_stage1(const float* __restrict__ W, const float* __restrict__ hb, int K,
                                                   int C, int LW, int open, int ne, const int8_t* __restrict__ x,
                                                   int L, const float* __restrict__ gF, double* __restrict__ part,
                                                   int sig64)
{
    extern __shared__ __align__(16) unsigned char smem[];
    if (sig64)
        grad_stage1_body<double>(W, hb, K, C, LW, open, ne, x, L, gF, part, smem);
    else
        grad_stage1_body<float>(W, hb, K, C, LW, open, ne, x, L, gF, part, smem);
}

__global__ __launch_bounds__(256) void grad_stage2(const double* __restrict__ part, int B, int P, int nW, int K,
                                                   float* __restrict__ dW, float* __restrict__ dhb,
                                                   float* __restrict__ dvb)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += part[(size_t)b * P + p];
    if (p < nW) dW[p] = (float)s;
    else if (p < nW + K) dhb[p - nW] = (float)s;
    else dvb[p - nW - K] = (float)s;
}

// Backward of the fully connected RBM's F: parameters W[K][nv], hbias[K],
// vbias[nv]; dF/dW[k][q] = -sigma(a_k) v_q, dF/dhb[k] = -sigma(a_k),
// dF/dvb[q] = -v_q.  Stage 1 per sample as above (FP64 pre-activations and
// sigma), stage 2 shared.
__global__ __launch_bounds__(256) void grad_dense_stage1(const float* __restrict__ W, const float* __restrict__ hb,
                                                         int K, int nv, const int8_t* __restrict__ x,
                                                         const float* __restrict__ gF, double* __restrict__ part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int P = K * nv + K + nv;
    double* sg = (double*)smem;
    uint8_t* v = (uint8_t*)(sg + K);
    const int8_t* xs = x + (size_t)blockIdx.x * nv;
    for (int q = threadIdx.x; q < nv; q += blockDim.x) v[q] = xs[q] > 0;
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const float* w = W + (size_t)k * nv;
        double acc = (double)hb[k];
        for (int q = 0; q < nv; ++q)
            if (v[q]) acc += (double)w[q];
        sg[k] = 1.0 / (1.0 + exp(-acc));
    }
    __syncthreads();
    const double gb = (double)gF[blockIdx.x];
    double* out = part + (size_t)blockIdx.x * P;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        double s;
        if (p < K * nv) s = v[p % nv] ? sg[p / nv] : 0.0;
        else if (p < K * nv + K) s = sg[p - K * nv];
        else s = (double)v[p - K * nv - K];
        out[p] = -gb * s;
    }
}

size_t grad_dense_lds(int K, int nv) { return (size_t)K * 8 + (size_t)nv + 16; }

hipError_t launch_grad_dense(const float* W, const float* hb, int K, int nv, const int8_t* x, int B, const float* gF,
                             double* part, float* dW, float* dhb, float* dvb, hipStream_t s)
{
    const int P = K * nv + K + nv;
    if (B > 0) {
        hipLaunchKernelGGL(grad_dense_stage1, dim3(B), dim3(256), grad_dense_lds(K, nv), s, W, hb, K, nv, x, gF, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(grad_stage2, dim3((P + 255) / 256), dim3(256), 0, s, part, B, P, K * nv, K, dW, dhb, dvb);
    return hipGetLastError();
}

// LDS of grad_stage1: sigma of every hidden unit (FP64, or float32 when that
// does not fit 160 KiB), the filters, the sample's visible units
size_t grad_lds_sig(int K, int C, int LW, int L, int banks, int sig_bytes)
{
    return (size_t)K * L * L * sig_bytes + (size_t)banks * (K * C * LW * LW) * 4 + (size_t)C * L * L + 16;
}

bool grad_sig64(int K, int C, int LW, int L, int banks) { return grad_lds_sig(K, C, LW, L, banks, 8) <= 160 * 1024; }

size_t grad_lds(int K, int C, int LW, int L, int banks)
{
    return grad_lds_sig(K, C, LW, L, banks, grad_sig64(K, C, LW, L, banks) ? 8 : 4);
}

hipError_t launch_grad(const float* W, const float* hb, int K, int C, int LW, int open, int ne, const int8_t* x, int B,
                       int L, const float* gF, double* part, float* dW, float* dhb, float* dvb, hipStream_t s)
{
    const int nb = 1 + 2 * ne;
    const int P = nb * (K * C * LW * LW + K) + C;
    if (B > 0) {
        hipLaunchKernelGGL(grad_stage1, dim3(B), dim3(256), grad_lds(K, C, LW, L, nb), s, W, hb, K, C, LW, open, ne, x,
                           L, gF, part, grad_sig64(K, C, LW, L, nb) ? 1 : 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(grad_stage2, dim3((P + 255) / 256), dim3(256), 0, s, part, B, P, nb * K * C * LW * LW, nb * K,
                       dW, dhb, dvb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of crbm_grad_static, the gradient entry point for callers that cannot
// allocate: the per-sample partial gradients part[B][P] live in a file-scope
// device array instead of a caller workspace.  Every GPU the library runs on
// holds its own copy until the process ends; calls on one GPU share it.  In
// host code the array's name is only a stand-in: its device address is looked
// up once per device (with that device current) and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[GRAD_STATIC_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
}  // namespace

hipError_t grad_static_scratch(void** ptr)
{
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace crbm
