// mf_mlp.hpp -- the con2prim-seed MLP (2 -> 64 -> 64 -> 1, tanh, bf16 weights,
// FP32 accumulation): launchers of the matrix-core kernels in mf_mlp.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_device.hpp"
#include "mf_params.hpp"

namespace mf {

constexpr int kMlpHidden = 64;
// W1[64][2], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int kMlpParams = 2 * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;

// Input/output normalisation of the seed network.
struct SeedNorm {
    float in_shift[2], in_scale[2];  // x = ((ln E, |M|/E) - shift) * scale
    float out_shift, out_scale;      // prediction = y * scale + shift
    int output;                      // 0: prediction = ln e; 1: = (E - e) E / |M|^2
};

// Seeded con2prim over n states (mode 1: MLP on the matrix cores, mode 2:
// conformal closed-form guess), FP64, tabulated EoS.
hipError_t con2prim_seeded(int64_t n, hipStream_t s, const C2PArgs<double>& a, const EosTable& eos, const float* P,
                           const SeedNorm& nrm, int mode);

// y[i] = MLP(X[i]) for B samples, X row-major (B, 2), all device pointers.
hipError_t mlp_forward(const float* P, const float* X, int64_t B, float* y, hipStream_t s);

// Gradient of mean((MLP(X) - T)^2) into grad[kMlpParams] and the loss into
// *loss (nullable); part is scratch of mlp_grad_partials(B) * (kMlpParams + 1) floats.
int64_t mlp_grad_partials(int64_t B);
hipError_t mlp_grad(const float* P, const float* X, const float* T, int64_t B, float* part, float* grad, float* loss,
                    hipStream_t s);

// One Adam step (step >= 1) on the FP32 master parameters.
hipError_t mlp_adam(float* P, const float* g, float* m, float* v, int step, float lr, float b1, float b2, float eps,
                    hipStream_t s);

}  // namespace mf
