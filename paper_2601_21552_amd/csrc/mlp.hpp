// Learned-scorer perceptron: sizes, parameter layout and the launchers.
#pragma once
#include <cstdint>

namespace scuba {

constexpr int kMlpF = 16;    // features per candidate variable
constexpr int kMlpH = 128;   // hidden width
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpF * kMlpH;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
constexpr int kMlpParams = kOffB3 + 1;

// All pointers are device pointers; work is queued on `stream`.
void mlp_sync(const float* master, uint16_t* wb, void* stream);
void mlp_forward(const uint16_t* wb, const float* master, const uint16_t* X, uint32_t B, uint16_t* A1,
                 uint16_t* A2, float* y, void* stream);
void mlp_backward(const uint16_t* wb, const uint16_t* X, const uint16_t* A1, const uint16_t* A2, const float* y,
                  const float* target, uint32_t B, uint16_t* dZ1, uint16_t* dZ2, float* grad, void* stream);
void mlp_adam(float* master, const float* grad, float* m, float* v, uint16_t* wb, uint32_t step, float lr,
              float beta1, float beta2, float eps, void* stream);

}  // namespace scuba
