// hhg_learned.h -- state of the learned smoothing correction (weights on the
// device, fallback threshold) and its kernel launchers (hhg_learned.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hhg_internal.h"

namespace hhg {

constexpr int LN_IN = 32, LN_H = 16;
// the cycle of a learned solve at which the plain cycle's contraction is
// measured from the same iterate
constexpr int LEARNED_PROBE_CYCLE = 2;
constexpr int LN_NPARAM = LN_H * LN_IN + LN_H + LN_H * LN_H + LN_H + LN_H + 1;  // 817

struct LearnedState {
    bool ready = false;
    double fallback_rate = 1.0;     // largest accepted per-cycle residual ratio
    double plain_margin = 1.05;     // largest accepted ratio to the plain cycle's contraction (0: off)
    double omega = 2.0 / 3.0;       // damping of the Jacobi part of the step
    unsigned short *wbf = nullptr;  // BF16 parameters (817)
    float *w32 = nullptr;           // FP32 copy uploaded by the caller
    float *gpart = nullptr;         // per-block gradient partials
    int64_t gpart_blocks = 0;
    float *dgrad = nullptr;         // reduced gradient (817)
};

// c (and s c, s) per slot from the residual r at one level (FP32)
template <typename T>
hipError_t launch_learned_forward(const LevelView<T> &L, const LearnedState &S, const T *r,
                                  const float *logk, float *c, hipStream_t st);
hipError_t launch_learned_forward_full(const LevelView<float> &L, const LearnedState &S,
                                       const float *r, const float *logk, float *c, float *sc,
                                       float *s, hipStream_t st);
// gradient of sum_i g_i c_i into S.dgrad (817 floats, device)
int learned_bwd_blocks(const LevelView<float> &L);
hipError_t launch_learned_backward(const LevelView<float> &L, const LearnedState &S,
                                   const float *r, const float *logk, const float *g,
                                   hipStream_t st);
// the learned smoothing step in one pass: u += D^{-1}(omega r + s c(r, k))
hipError_t launch_learned_step(const LevelView<float> &L, const LearnedState &S, const float *r, const float *logk,
                               float *u, const float *invd, float omega, hipStream_t st);
hipError_t launch_learned_err(const float *e, const float *r, const float *sc, const float *invd,
                              float omega, float *e1, int64_t n, hipStream_t st);
hipError_t launch_learned_lossgrad(const float *ae1, const float *s, const float *invd,
                                   double inv_e0, float *g, int64_t n, hipStream_t st);
hipError_t launch_dot_owned(const float *a, const float *b, const uint8_t *own, int64_t n,
                            double *partial, int *nblk, hipStream_t st);
hipError_t launch_logk(const double *k, float *lk, int64_t n, hipStream_t st);
hipError_t launch_weights_bf16(const float *w, unsigned short *wb, int n, hipStream_t st);
hipError_t launch_pair(const double *r64, const double *us, const double *u, float *r, float *e,
                       int64_t n, hipStream_t st);

}  // namespace hhg
