// hhg_learned.h -- state of the learned smoothing correction (weights on the
// device, fallback threshold) and its kernel launchers (hhg_learned.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hhg_internal.h"

namespace hhg {

constexpr int LN_IN = 32, LN_H = 16;
constexpr int LN_NPARAM = LN_H * LN_IN + LN_H + LN_H * LN_H + LN_H + LN_H + 1;  // 801

struct LearnedState {
    bool ready = false;
    double fallback_rate = 1.0;  // largest accepted per-cycle residual ratio
    float *w32 = nullptr;        // FP32 copy of the BF16-rounded weights (801)
    uint16_t *wbf = nullptr;     // BF16 weights, MFMA operand layout
    float *gpart = nullptr;      // per-block weight-gradient partials
    int64_t gpart_blocks = 0;
    float *dgrad = nullptr;      // reduced gradient (801)
};

void learned_free(LearnedState &s);

// c[slot] = network output at every unknown slot (0 elsewhere)
template <typename T>
hipError_t launch_learned_forward(const LevelView<T> &L, const LearnedState &S, const T *r,
                                  float *c, hipStream_t st);
// gradient of sum_i g_i c_i w.r.t. the parameters: per-block partials then a
// deterministic reduction into S.dgrad
hipError_t launch_learned_backward(const LevelView<float> &L, const LearnedState &S,
                                   const float *r, const float *g, hipStream_t st);
// u += delta, delta_i = s_i c_i / D_i (s_i = neighbourhood max |r|)
template <typename T>
hipError_t launch_learned_apply(const LevelView<T> &L, const LearnedState &S, const T *r,
                                const T *invd, T *u, hipStream_t st);

}  // namespace hhg
