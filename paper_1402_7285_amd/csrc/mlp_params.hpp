// Shapes of the RHS-cost MLP and launchers of its kernels (mlp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scocg_params.hpp"

namespace scocg {

enum {
    NIN = 16,                 // features per RHS
    NH = 64,                  // hidden units per layer (one wave)
    OFF_W1 = 0,
    OFF_B1 = OFF_W1 + NH * NIN,
    OFF_W2 = OFF_B1 + NH,
    OFF_B2 = OFF_W2 + NH * NH,
    OFF_W3 = OFF_B2 + NH,
    OFF_B3 = OFF_W3 + NH,
    NPARAM = OFF_B3 + 1,      // 5313
    NPARAM_PAD = 5376,
    GRAD_BLOCKS = 64,         // workgroups of the gradient kernel (4 waves each)
};

hipError_t launch_mlp_forward(const float* w, const float* x, int64_t n, float* y, hipStream_t st);
hipError_t launch_mlp_grad(const float* w, const float* x, const float* t, const int32_t* idx, int64_t m,
                           float* partial, float* loss_part, int nblocks, hipStream_t st);
hipError_t launch_mlp_adam(float* w, float* am, float* av, const float* partial, const float* loss_part,
                           int64_t nparts, int64_t m, float lr, int32_t step, float* grad, float* loss,
                           hipStream_t st);
hipError_t launch_features(const KParams& P, int bd, int has_S, float* feats, hipStream_t st);

}  // namespace scocg
