// GELU activation of the learned budget's hidden layers (float32, device).
// Kept apart from the matrix-core code so that the CPU emulation of the
// device code can test it against the exact definition.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace twk {
namespace mlp {

// GELU(x) = x Phi(x), Phi the standard normal distribution function, through
// the tail q = erfc(|x| / sqrt 2): Phi(x) = 1 - q/2 for x >= 0 and q/2 for
// x < 0, so that the negative tail carries no cancellation.  erfc is the
// Chebyshev fit of Press et al. (Numerical Recipes, "erfcc"; fractional error
// below 1.2e-7), evaluated in float32 with the hardware reciprocal and
// exponential: relative error of GELU below 1e-5 and absolute error below
// 3e-7 for finite x, far below the bf16 rounding of the activations.
__device__ __forceinline__ float gelu_tail(float x) {
  const float u = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.5f, u, 1.0f));
  float p = 0.17087277f;
  p = __builtin_fmaf(p, t, -0.82215223f);
  p = __builtin_fmaf(p, t, 1.48851587f);
  p = __builtin_fmaf(p, t, -1.13520398f);
  p = __builtin_fmaf(p, t, 0.27886807f);
  p = __builtin_fmaf(p, t, -0.18628806f);
  p = __builtin_fmaf(p, t, 0.09678418f);
  p = __builtin_fmaf(p, t, 0.37409196f);
  p = __builtin_fmaf(p, t, 1.00002368f);
  p = __builtin_fmaf(p, t, -1.26551223f);
  // exp(p - u^2) as a power of two
  return t * __builtin_amdgcn_exp2f(__builtin_fmaf(-u, u, p) * 1.44269504088896341f);
}

__device__ inline float gelu(float x) {
  const float h = 0.5f * x * gelu_tail(x);
  return x >= 0.0f ? x - h : h;
}

__device__ inline float gelu_grad(float x) {
  const float hq = 0.5f * gelu_tail(x);
  const float cdf = x >= 0.0f ? 1.0f - hq : hq;
  // Phi'(x) = exp(-x^2 / 2) / sqrt(2 pi)
  return cdf + x * 0.39894228040143268f * __builtin_amdgcn_exp2f(x * x * -0.72134752044448170f);
}

}  // namespace mlp
}  // namespace twk
