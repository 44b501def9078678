// Host-side state of the learned-bracket network (internal).
#pragma once
#include <stdint.h>

#include "abi_util.h"
#include "mlp.h"

constexpr int MLP_MAX_LAYERS = 9;

struct spec_mlp_s {
    int device = 0;
    int n = 0, width = 0, hidden = 0, nl = 0, bf16 = 1;
    int nextra = 0;  // 2: the features end with <x, v> and |x|^2 (dims[0] = 2 n + nextra)
    int dims[MLP_MAX_LAYERS + 1] = {};
    int64_t off[MLP_MAX_LAYERS] = {};  // parameter offset of layer l
    int64_t np = 0;
    float *dP = nullptr, *dG = nullptr, *dM = nullptr, *dV = nullptr;
    int step = 0;
    // standardisation of features (2n) and targets (2)
    float *dMu = nullptr, *dIsd = nullptr;
    float tmu[2] = {0.f, 0.f}, tsd[2] = {1.f, 1.f};
    // work buffers, capacity in rows
    int cap = 0;
    float* dX = nullptr;                  // cap x ld_in: features and a ones column
    float* dH[MLP_MAX_LAYERS] = {};       // cap x ld_h: GELU outputs and a ones column
    float* dZ[MLP_MAX_LAYERS] = {};       // cap x width: pre-activations
    float *dY = nullptr, *dDY = nullptr;  // cap x 2
    float *dD0 = nullptr, *dD1 = nullptr; // cap x width
    float* dT = nullptr;                  // cap x 2
    int32_t* dIdx = nullptr;
    double* dLoss = nullptr;

    int ld_in() const { return dims[0] + 1; }
    int ld_h() const { return width + 1; }
    void free_work();
    spec_status ensure(int rows, hipStream_t s);
};

namespace spec_host {

// Raw network on X (rows x ldx, with a ones column at dims[0]); output in net->dY.
spec_status mlp_forward_x(spec_mlp_s* net, int rows, const float* X, int ldx, hipStream_t s);
// Gradient of the loss whose output gradient is in net->dDY, for the inputs of
// the last mlp_forward_x; into g (np floats).
spec_status mlp_backward(spec_mlp_s* net, int rows, const float* X, int ldx, float* g, hipStream_t s);
// Standardised features of (x, v) into net->dX, then forward.
spec_status mlp_predict_rows(spec_mlp_s* net, int rows, const double* x, int ldx, const double* v, int ldv,
                             hipStream_t s);

}  // namespace spec_host
