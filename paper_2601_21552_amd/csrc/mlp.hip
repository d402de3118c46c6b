// Learned branching scorer on gfx950: a 3-layer perceptron F -> H -> H -> 1
// (F = 16 features, H = 128, ReLU) with bf16 weights and activations and
// fp32 accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16), trained
// by mean squared error with Adam on fp32 master weights.
//
// Parameter block (fp32 master, and the bf16 copy at the same offsets):
//   W1 [F x H] | b1 [H] | W2 [H x H] | b2 [H] | w3 [H] | b3 [1]
// bf16 storage points: inputs, weights, both hidden activations, and the two
// back-propagated pre-activation gradients (the operands of the gradient
// products).  Rounding is to nearest, ties to even.
#include <hip/hip_runtime.h>

#include <string>

#include "common.hpp"
#include "mlp.hpp"

namespace scuba {

#define HIP_OK(x)                                                                               \
  do {                                                                                          \
    hipError_t e_ = (x);                                                                        \
    if (e_ != hipSuccess) fail(SCUBA_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int F = kMlpF, H = kMlpH;

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return uint16_t((u >> 16) | 0x40);  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// One 16x16x16 bf16 product on the matrix cores.  Operand layout (64 lanes):
//   a: A[i][k] with i = lane % 16, k = 4*(lane/16) + e   (e = 0..3)
//   b: B[k][j] with j = lane % 16, k = 4*(lane/16) + e
//   c: C[i][j] with j = lane % 16, i = 4*(lane/16) + e
__device__ __forceinline__ f32x4 mma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- forward
// One workgroup of 8 waves per 16 batch rows; wave w owns hidden columns
// [16w, 16w+16).
__global__ __launch_bounds__(512) void mlp_fwd_kernel(const uint16_t* __restrict__ X, uint32_t B,
                                                     const uint16_t* __restrict__ wb,
                                                     const float* __restrict__ master,
                                                     uint16_t* __restrict__ A1, uint16_t* __restrict__ A2,
                                                     float* __restrict__ y) {
  __shared__ uint16_t sA1[16 * H];
  __shared__ uint16_t sA2[16 * H];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t r0 = blockIdx.x * 16;
  const uint32_t li = lane % 16, lk = 4 * (lane / 16);
  const uint32_t col = wave * 16 + li;
  // layer 1: K = F = 16, one product
  bf16x4 a, b;
  for (int e = 0; e < 4; e++) {
    const uint32_t row = r0 + li;
    a[e] = row < B ? short(X[size_t(row) * F + lk + e]) : short(0);
    b[e] = short(wb[kOffW1 + (lk + e) * H + col]);
  }
  f32x4 c = {0, 0, 0, 0};
  c = mma(a, b, c);
  for (int e = 0; e < 4; e++) {
    const uint32_t i = lk + e;   // row within the block
    const float z = c[e] + master[kOffB1 + col];
    sA1[i * H + col] = f2bf(z > 0.f ? z : 0.f);
  }
  __syncthreads();
  // layer 2: K = H
  c = f32x4{0, 0, 0, 0};
  for (uint32_t k0 = 0; k0 < uint32_t(H); k0 += 16) {
    for (int e = 0; e < 4; e++) {
      a[e] = short(sA1[li * H + k0 + lk + e]);
      b[e] = short(wb[kOffW2 + (k0 + lk + e) * H + col]);
    }
    c = mma(a, b, c);
  }
  for (int e = 0; e < 4; e++) {
    const uint32_t i = lk + e;
    const float z = c[e] + master[kOffB2 + col];
    sA2[i * H + col] = f2bf(z > 0.f ? z : 0.f);
  }
  __syncthreads();
  // outputs: activations to global, then y = A2 w3 + b3 (fixed order)
  for (uint32_t t = threadIdx.x; t < 16u * H; t += blockDim.x) {
    const uint32_t row = r0 + t / H;
    if (row < B) {
      A1[size_t(row) * H + t % H] = sA1[t];
      A2[size_t(row) * H + t % H] = sA2[t];
    }
  }
  if (threadIdx.x < 16) {
    const uint32_t row = r0 + threadIdx.x;
    if (row < B) {
      float acc = 0.f;
      for (int h = 0; h < H; h++) acc += bf2f(sA2[threadIdx.x * H + h]) * bf2f(wb[kOffW3 + h]);
      y[row] = acc + master[kOffB3];
    }
  }
}

// ---------------------------------------------------------------- backward
// dZ2 = bf16(dy w3^T * [A2 > 0]); dZ1 = bf16(dZ2 W2^T * [A1 > 0]), per 16
// rows; wave w owns columns [16w, 16w+16) of dZ1.
__global__ __launch_bounds__(512) void mlp_bwd_dz_kernel(const uint16_t* __restrict__ A1,
                                                        const uint16_t* __restrict__ A2,
                                                        const float* __restrict__ y,
                                                        const float* __restrict__ target, uint32_t B,
                                                        const uint16_t* __restrict__ wb,
                                                        uint16_t* __restrict__ dZ1,
                                                        uint16_t* __restrict__ dZ2) {
  __shared__ uint16_t sZ2[16 * H];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t r0 = blockIdx.x * 16;
  for (uint32_t t = threadIdx.x; t < 16u * H; t += blockDim.x) {
    const uint32_t row = r0 + t / H, h = t % H;
    uint16_t v = 0;
    if (row < B) {
      const float dy = 2.f * (y[row] - target[row]) / float(B);
      const float g = bf2f(A2[size_t(row) * H + h]) > 0.f ? dy * bf2f(wb[kOffW3 + h]) : 0.f;
      v = f2bf(g);
      dZ2[size_t(row) * H + h] = v;
    }
    sZ2[t] = v;
  }
  __syncthreads();
  const uint32_t li = lane % 16, lk = 4 * (lane / 16);
  const uint32_t col = wave * 16 + li;
  f32x4 c = {0, 0, 0, 0};
  bf16x4 a, b;
  for (uint32_t k0 = 0; k0 < uint32_t(H); k0 += 16) {
    for (int e = 0; e < 4; e++) {
      a[e] = short(sZ2[li * H + k0 + lk + e]);
      b[e] = short(wb[kOffW2 + col * H + k0 + lk + e]);   // (W2^T)[k][col] = W2[col][k]
    }
    c = mma(a, b, c);
  }
  for (int e = 0; e < 4; e++) {
    const uint32_t row = r0 + lk + e;
    if (row < B) {
      const uint16_t a1 = A1[size_t(row) * H + col];
      dZ1[size_t(row) * H + col] = f2bf(bf2f(a1) > 0.f ? c[e] : 0.f);
    }
  }
}

// Weight and bias gradients, one 512-thread workgroup per output block.
// Workgroups 0..63: 16x16 tiles of dW2 = A1^T dZ2; 64..71: tiles of
// dW1 = X^T dZ1.  Wave w of a tile reduces the batch rows 16(w + 8i) .. +15
// on the matrix cores; the eight waves' tiles are then added in wave order.
// Workgroups 72..75: b1 = sum_r dZ1[r], b2 = sum_r dZ2[r],
// w3 = sum_r A2[r] dy[r], b3 = sum_r dy[r]; thread t takes column t % H and
// the rows of slice t / H, and the slices' sums are added in slice order.
// Every sum is taken in an order fixed by B alone.
constexpr uint32_t kDwWaves = 8;
constexpr uint32_t kBiasSlices = 4;

// Sum over rows [r0, r1) of column h of one bias or w3 gradient term, in
// eight interleaved partial sums (eight loads in flight) added pairwise.
// W selects the term, so the loop body has no branch between a load and
// its use.
template <int W>
__device__ __forceinline__ float bias_rows(const uint16_t* __restrict__ M, const float* __restrict__ y,
                                           const float* __restrict__ target, uint32_t B, uint32_t h,
                                           uint32_t r0, uint32_t r1) {
  auto term = [&](uint32_t r) -> float {
    if constexpr (W < 2) return bf2f(M[size_t(r) * H + h]);
    const float dy = 2.f * (y[r] - target[r]) / float(B);
    if constexpr (W == 2) return bf2f(M[size_t(r) * H + h]) * dy;
    return dy;
  };
  float s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0;
  uint32_t r = r0;
  for (; r + 8 <= r1; r += 8) {
    s0 += term(r);
    s1 += term(r + 1);
    s2 += term(r + 2);
    s3 += term(r + 3);
    s4 += term(r + 4);
    s5 += term(r + 5);
    s6 += term(r + 6);
    s7 += term(r + 7);
  }
  for (; r < r1; r++) s0 += term(r);
  return ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
}

__global__ __launch_bounds__(512) void mlp_bwd_dw_kernel(const uint16_t* __restrict__ X,
                                                        const uint16_t* __restrict__ A1,
                                                        const uint16_t* __restrict__ A2,
                                                        const float* __restrict__ y,
                                                        const float* __restrict__ target, uint32_t B,
                                                        const uint16_t* __restrict__ dZ1,
                                                        const uint16_t* __restrict__ dZ2,
                                                        float* __restrict__ grad) {
  static_assert(kDwWaves * 64 == 512 && kBiasSlices * H == 512, "one 512-thread workgroup");
  __shared__ float part[kDwWaves * 64 * 4];
  const uint32_t tile = blockIdx.x;
  if (tile < 72) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t li = lane % 16, lk = 4 * (lane / 16);
    const bool w2 = tile < 64;
    const uint32_t ti = w2 ? tile / 8 : 0, tj = w2 ? tile % 8 : tile - 64;
    const uint16_t* L = w2 ? A1 : X;      // left operand, row-major [B x (H or F)]
    const uint32_t ld = w2 ? H : F;
    const uint16_t* R = w2 ? dZ2 : dZ1;   // right operand [B x H]
    f32x4 c = {0, 0, 0, 0};
    bf16x4 a, b;
    uint32_t k0 = 16 * wave;
#pragma unroll 2
    for (; k0 + 16 <= B; k0 += 16 * kDwWaves) {   // full 16-row chunks
      for (int e = 0; e < 4; e++) {
        const uint32_t k = k0 + lk + e;   // batch index
        a[e] = short(L[size_t(k) * ld + ti * 16 + li]);   // (L^T)[i][k]
        b[e] = short(R[size_t(k) * H + tj * 16 + li]);
      }
      c = mma(a, b, c);
    }
    if (k0 < B) {   // the ragged last chunk, at most one per wave
      for (int e = 0; e < 4; e++) {
        const uint32_t k = k0 + lk + e;
        a[e] = k < B ? short(L[size_t(k) * ld + ti * 16 + li]) : short(0);
        b[e] = k < B ? short(R[size_t(k) * H + tj * 16 + li]) : short(0);
      }
      c = mma(a, b, c);
    }
    for (int e = 0; e < 4; e++) part[(wave * 64 + lane) * 4 + e] = c[e];
    __syncthreads();
    if (wave == 0) {
      for (int e = 0; e < 4; e++) {
        float sum = 0.f;
        for (uint32_t w = 0; w < kDwWaves; w++) sum += part[(w * 64 + lane) * 4 + e];
        const uint32_t i = ti * 16 + lk + e, j = tj * 16 + li;
        grad[(w2 ? kOffW2 : kOffW1) + i * H + j] = sum;
      }
    }
    return;
  }
  const uint32_t which = tile - 72, h = threadIdx.x % H, slice = threadIdx.x / H;
  const uint32_t per = (B + kBiasSlices - 1) / kBiasSlices;
  const uint32_t r0 = min(B, slice * per), r1 = min(B, r0 + per);
  float v;
  if (which == 0) v = bias_rows<0>(dZ1, y, target, B, h, r0, r1);
  else if (which == 1) v = bias_rows<1>(dZ2, y, target, B, h, r0, r1);
  else if (which == 2) v = bias_rows<2>(A2, y, target, B, h, r0, r1);
  else v = bias_rows<3>(A2, y, target, B, h, r0, r1);
  part[slice * H + h] = v;
  __syncthreads();
  if (slice == 0 && (which != 3 || h == 0)) {
    float sum = 0.f;
    for (uint32_t k = 0; k < kBiasSlices; k++) sum += part[k * H + h];
    const uint32_t off = which == 0 ? kOffB1 : which == 1 ? kOffB2 : which == 2 ? kOffW3 : kOffB3;
    grad[off + h] = sum;
  }
}

// ---------------------------------------------------------------- Adam
__global__ void mlp_adam_kernel(float* __restrict__ master, const float* __restrict__ grad,
                                float* __restrict__ m, float* __restrict__ v, uint16_t* __restrict__ wb,
                                uint32_t step, float lr, float beta1, float beta2, float eps) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= uint32_t(kMlpParams)) return;
  const float g = grad[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * g;
  const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(beta1, float(step)));
  const float vh = vi / (1.f - powf(beta2, float(step)));
  const float p = master[i] - lr * mh / (sqrtf(vh) + eps);
  master[i] = p;
  wb[i] = f2bf(p);
}

__global__ void mlp_sync_kernel(const float* __restrict__ master, uint16_t* __restrict__ wb) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < uint32_t(kMlpParams)) wb[i] = f2bf(master[i]);
}

}  // namespace

void mlp_sync(const float* master, uint16_t* wb, void* stream) {
  hipLaunchKernelGGL(mlp_sync_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), master, wb);
  HIP_OK(hipGetLastError());
}

void mlp_forward(const uint16_t* wb, const float* master, const uint16_t* X, uint32_t B, uint16_t* A1,
                 uint16_t* A2, float* y, void* stream) {
  if (B == 0) return;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3((B + 15) / 16), dim3(512), 0, static_cast<hipStream_t>(stream), X, B,
                     wb, master, A1, A2, y);
  HIP_OK(hipGetLastError());
}

void mlp_backward(const uint16_t* wb, const uint16_t* X, const uint16_t* A1, const uint16_t* A2, const float* y,
                  const float* target, uint32_t B, uint16_t* dZ1, uint16_t* dZ2, float* grad, void* stream) {
  if (B == 0) return;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(mlp_bwd_dz_kernel, dim3((B + 15) / 16), dim3(512), 0, st, A1, A2, y, target, B, wb, dZ1,
                     dZ2);
  HIP_OK(hipGetLastError());
  hipLaunchKernelGGL(mlp_bwd_dw_kernel, dim3(76), dim3(512), 0, st, X, A1, A2, y, target, B, dZ1, dZ2, grad);
  HIP_OK(hipGetLastError());
}

void mlp_adam(float* master, const float* grad, float* m, float* v, uint16_t* wb, uint32_t step, float lr,
              float beta1, float beta2, float eps, void* stream) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), master, grad, m, v, wb, step, lr, beta1, beta2, eps);
  HIP_OK(hipGetLastError());
}

}  // namespace scuba
