// ops.h -- host-side launchers of the stand-alone kernels (ops.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace crbm {

// `open`, `ne`: the locally connected CRBM (windows stop at the column edge,
// 1 + 2 ne filter banks); open_cols: the open-column target lattice
size_t free_energy_lds(int K, int C, int LW, int L, int banks);
hipError_t launch_free_energy(const float* W, const float* hb, const float* vb, int K, int C, int LW, int open, int ne,
                              const int8_t* x, int B, int L, double* F, hipStream_t s);
hipError_t launch_ising_energy(const int8_t* x, int B, int L, int open_cols, int32_t* E, hipStream_t s);
size_t kitaev_weight_lds(int C, int L);
hipError_t launch_kitaev_weight(const int8_t* x, int B, int C, int L, int open_cols, double Jx, double Jy, double Jz,
                                const double* T, double* S, hipStream_t s);
size_t grad_lds(int K, int C, int LW, int L, int banks);
// 1: grad_stage1 keeps sigma of the hidden units in FP64 (else float32)
bool grad_sig64(int K, int C, int LW, int L, int banks);
// fully connected RBM: W[K][nv], hbias[K], vbias[nv], nv = C L^2
size_t free_energy_dense_lds(int nv);
hipError_t launch_free_energy_dense(const float* W, const float* hb, const float* vb, int K, int nv, const int8_t* x,
                                    int B, double* F, hipStream_t s);
size_t grad_dense_lds(int K, int nv);
hipError_t launch_grad_dense(const float* W, const float* hb, int K, int nv, const int8_t* x, int B, const float* gF,
                             double* part, float* dW, float* dhb, float* dvb, hipStream_t s);
// crbm_grad_static: the device address of this GPU's static scratch of
// GRAD_STATIC_BYTES (looked up once per device, with the device current)
constexpr size_t GRAD_STATIC_BYTES = (size_t)8 << 20;
hipError_t grad_static_scratch(void** ptr);
hipError_t launch_grad(const float* W, const float* hb, int K, int C, int LW, int open, int ne, const int8_t* x, int B,
                       int L, const float* gF, double* part, float* dW, float* dhb, float* dvb, hipStream_t s);

}  // namespace crbm
