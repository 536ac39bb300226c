// Activation functions of the layer-by-layer path (tanh form of GELU, as in
// the amplitude network's feed-forward block and phase MLP), shared by its
// kernels.
#pragma once

namespace nqs {

template <class T>
__device__ inline T gelu_tanh(T x) {
  const T c = T(0.7978845608028654);  // sqrt(2/pi)
  return T(0.5) * x * (T(1) + tanh(c * (x + T(0.044715) * x * x * x)));
}
template <class T>
__device__ inline T gelu_tanh_grad(T x) {
  const T c = T(0.7978845608028654);
  const T u = c * (x + T(0.044715) * x * x * x);
  const T t = tanh(u);
  return T(0.5) * (T(1) + t) + T(0.5) * x * (T(1) - t * t) * c * (T(1) + T(3 * 0.044715) * x * x);
}

}  // namespace nqs
