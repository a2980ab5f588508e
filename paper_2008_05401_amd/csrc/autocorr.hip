// autocorr.hip -- autocovariance and integrated autocorrelation time of
// per-chain observable series (the sampler diagnostic compared between the
// CRBM and Metropolis samplers in Sec. III and IV).  One workgroup per series;
// the series of chain g is x_i = trace[g][(start + i) mod len], i = 0..len-1:
//   C(t)    = 1/(len - t) sum_{i < len - t} (x_i - m)(x_{i+t} - m),  m = mean x
//   rho(t)  = C(t) / C(0)
//   tau(W)  = 1/2 + sum_{t=1..W} rho(t)
// and the window is the smallest W >= 1 with W >= c * tau(W) (automatic
// windowing; the paper does not state its estimator).  FP64 throughout; the
// series sits centred in LDS and every lag is one lane's sequential sum, so the
// summation order is fixed.
#include "device_common.h"
#include "sweep_common.h"

namespace crbm {

constexpr int AC_NT = 256;

__global__ __launch_bounds__(AC_NT) void autocorr_kernel(const double* __restrict__ trace, int len, int start,
                                                         int max_lag, double c_win, double* __restrict__ out,
                                                         double* __restrict__ tau, int* __restrict__ window)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* red = (double*)smem;  // 16 doubles
    double* x = red + 16;         // the series, centred, in time order
    const int g = (int)blockIdx.x, tid = threadIdx.x;
    const double* tr = trace + (size_t)g * len;
    double* o = out + (size_t)g * (max_lag + 1);
    double s = 0.0;
    for (int i = tid; i < len; i += AC_NT) {
        const int j = start + i < len ? start + i : start + i - len;
        const double v = tr[j];
        x[i] = v;
        s += v;
    }
    const double m = block_sum(s, red) / (double)len;
    for (int i = tid; i < len; i += AC_NT) x[i] -= m;
    __syncthreads();
    for (int t = tid; t <= max_lag; t += AC_NT) {
        double c = 0.0;
        for (int i = 0; i + t < len; ++i) c += x[i] * x[i + t];
        o[t] = c / (double)(len - t);
    }
    if (!tau) return;
    __syncthreads();  // the lags written above are visible to the workgroup
    if (tid == 0) {
        const double c0 = o[0];
        double tw = 0.5;
        int w = -1;
        if (c0 > 0.0) {
            for (int t = 1; t <= max_lag; ++t) {
                tw += o[t] / c0;
                if ((double)t >= c_win * tw) {
                    w = t;
                    break;
                }
            }
        }
        tau[g] = tw;
        window[g] = w;
    }
}

hipError_t launch_autocorr(const double* trace, int n, int len, int start, int max_lag, double c_win, double* out,
                           double* tau, int* window, hipStream_t s)
{
    const size_t lds = (16 + (size_t)len) * sizeof(double);
    hipLaunchKernelGGL(autocorr_kernel, dim3(n), dim3(AC_NT), lds, s, trace, len, start, max_lag, c_win, out, tau,
                       window);
    return hipGetLastError();
}

}  // namespace crbm
