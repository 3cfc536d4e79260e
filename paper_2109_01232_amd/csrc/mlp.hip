// The parameter chooser's network 16-64-64-3 on the GPU: forward pass,
// mean-squared-error gradient and a fused Adam step.
//
// The network is tiny (5443 parameters, ~10.6 kFLOP per sample), so each
// kernel keeps the parameters in LDS; the gradient kernel runs as one block
// that stages the activations and deltas of a chunk of samples in LDS and
// then lets each thread accumulate a fixed set of parameters over the
// samples in order -- a deterministic reduction without atomics.
#include <hip/hip_runtime.h>
#include <math.h>

#include "gmresir.h"
#include "internal.hpp"

namespace {

constexpr int NIN = 16, NH = 64, NOUT = 3;
constexpr int O_W1 = 0, O_B1 = O_W1 + NIN * NH, O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH, O_W3 = O_B2 + NH,
              O_B3 = O_W3 + NH * NOUT, NPARAM = O_B3 + NOUT;
static_assert(NPARAM == 5443, "parameter count");

constexpr int TPB = 256;
constexpr int CH = 32;              // samples per chunk in the gradient kernel
constexpr int PAD = NH + 1;         // LDS row pitch (odd: no bank conflicts)
constexpr int PPT = (NPARAM + TPB - 1) / TPB;  // parameters owned per thread

__global__ __launch_bounds__(TPB) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ shift,
                                                     const float* __restrict__ scale, const float* __restrict__ X,
                                                     float* __restrict__ Y, int batch) {
  __shared__ float sp[NPARAM];
  __shared__ float s_shift[NIN], s_scale[NIN];
  for (int i = threadIdx.x; i < NPARAM; i += TPB) sp[i] = P[i];
  if (threadIdx.x < NIN) {
    s_shift[threadIdx.x] = shift[threadIdx.x];
    s_scale[threadIdx.x] = scale[threadIdx.x];
  }
  __syncthreads();
  const int s = blockIdx.x * TPB + threadIdx.x;
  if (s >= batch) return;
  float x[NIN];
#pragma unroll
  for (int i = 0; i < NIN; ++i) x[i] = (X[(size_t)s * NIN + i] - s_shift[i]) * s_scale[i];
  float h1[NH];
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    float a = sp[O_B1 + o];
#pragma unroll
    for (int i = 0; i < NIN; ++i) a += x[i] * sp[O_W1 + i * NH + o];
    h1[o] = tanhf(a);
  }
  float y[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) y[o] = sp[O_B3 + o];
  for (int o2 = 0; o2 < NH; ++o2) {
    float a = sp[O_B2 + o2];
#pragma unroll
    for (int i = 0; i < NH; ++i) a += h1[i] * sp[O_W2 + i * NH + o2];
    const float h2 = tanhf(a);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) y[o] += h2 * sp[O_W3 + o2 * NOUT + o];
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) Y[(size_t)s * NOUT + o] = y[o];
}

// Gradient of L = sum (y - t)^2 / (3 batch) into g[] (registers, PPT per
// thread: parameter p = threadIdx.x + TPB * q); loss into *loss_out (LDS).
__device__ void mlp_grad_block(const float* __restrict__ P, const float* __restrict__ shift,
                               const float* __restrict__ scale, const float* __restrict__ X,
                               const float* __restrict__ T, int batch, float* sp, float (&g)[PPT], float* loss_out) {
  __shared__ float s_x[CH * (NIN + 1)];
  __shared__ float s_h1[CH * PAD];
  __shared__ float s_h2[CH * PAD];
  __shared__ float s_d1[CH * PAD];
  __shared__ float s_d2[CH * PAD];
  __shared__ float s_dy[CH * 4];
  __shared__ float s_loss[CH];
  __shared__ float s_shift[NIN], s_scale[NIN];
  const int tid = threadIdx.x;
  for (int i = tid; i < NPARAM; i += TPB) sp[i] = P[i];
  if (tid < NIN) {
    s_shift[tid] = shift[tid];
    s_scale[tid] = scale[tid];
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) g[q] = 0.f;
  float loss = 0.f;
  const float inv_n = 2.f / (3.f * (float)batch);
  __syncthreads();
  for (int c0 = 0; c0 < batch; c0 += CH) {
    const int cn = min(CH, batch - c0);
    // per-sample forward and backward, one thread per sample
    if (tid < cn) {
      const int s = c0 + tid;
      float* x = s_x + tid * (NIN + 1);
      for (int i = 0; i < NIN; ++i) x[i] = (X[(size_t)s * NIN + i] - s_shift[i]) * s_scale[i];
      float* h1 = s_h1 + tid * PAD;
      for (int o = 0; o < NH; ++o) {
        float a = sp[O_B1 + o];
        for (int i = 0; i < NIN; ++i) a += x[i] * sp[O_W1 + i * NH + o];
        h1[o] = tanhf(a);
      }
      float* h2 = s_h2 + tid * PAD;
      float y[NOUT];
      for (int o = 0; o < NOUT; ++o) y[o] = sp[O_B3 + o];
      for (int o2 = 0; o2 < NH; ++o2) {
        float a = sp[O_B2 + o2];
        for (int i = 0; i < NH; ++i) a += h1[i] * sp[O_W2 + i * NH + o2];
        const float hv = tanhf(a);
        h2[o2] = hv;
        for (int o = 0; o < NOUT; ++o) y[o] += hv * sp[O_W3 + o2 * NOUT + o];
      }
      float* dy = s_dy + tid * 4;
      float ls = 0.f;
      for (int o = 0; o < NOUT; ++o) {
        const float d = y[o] - T[(size_t)s * NOUT + o];
        ls += d * d;
        dy[o] = inv_n * d;
      }
      s_loss[tid] = ls;
      float* d2 = s_d2 + tid * PAD;
      for (int i = 0; i < NH; ++i) {
        float a = 0.f;
        for (int o = 0; o < NOUT; ++o) a += dy[o] * sp[O_W3 + i * NOUT + o];
        d2[i] = a * (1.f - h2[i] * h2[i]);
      }
      float* d1 = s_d1 + tid * PAD;
      for (int i = 0; i < NH; ++i) {
        float a = 0.f;
        for (int o = 0; o < NH; ++o) a += d2[o] * sp[O_W2 + i * NH + o];
        d1[i] = a * (1.f - h1[i] * h1[i]);
      }
    }
    __syncthreads();
    if (tid == 0)
      for (int s = 0; s < cn; ++s) loss += s_loss[s];
    // each thread accumulates its parameters over the chunk, samples in order
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int p = tid + TPB * q;
      if (p >= NPARAM) break;
      float a = 0.f;
      if (p < O_B1) {
        const int i = p / NH, o = p % NH;
        for (int s = 0; s < cn; ++s) a += s_x[s * (NIN + 1) + i] * s_d1[s * PAD + o];
      } else if (p < O_W2) {
        const int o = p - O_B1;
        for (int s = 0; s < cn; ++s) a += s_d1[s * PAD + o];
      } else if (p < O_B2) {
        const int qq = p - O_W2, i = qq / NH, o = qq % NH;
        for (int s = 0; s < cn; ++s) a += s_h1[s * PAD + i] * s_d2[s * PAD + o];
      } else if (p < O_W3) {
        const int o = p - O_B2;
        for (int s = 0; s < cn; ++s) a += s_d2[s * PAD + o];
      } else if (p < O_B3) {
        const int qq = p - O_W3, i = qq / NOUT, o = qq % NOUT;
        for (int s = 0; s < cn; ++s) a += s_h2[s * PAD + i] * s_dy[s * 4 + o];
      } else {
        const int o = p - O_B3;
        for (int s = 0; s < cn; ++s) a += s_dy[s * 4 + o];
      }
      g[q] += a;
    }
    __syncthreads();
  }
  if (tid == 0) *loss_out = loss / (3.f * (float)batch);
  __syncthreads();
}

__global__ __launch_bounds__(TPB) void k_mlp_loss_grad(const float* __restrict__ P, const float* __restrict__ shift,
                                                       const float* __restrict__ scale, const float* __restrict__ X,
                                                       const float* __restrict__ T, int batch, float* __restrict__ G,
                                                       float* __restrict__ loss) {
  __shared__ float sp[NPARAM];
  __shared__ float s_loss;
  float g[PPT];
  mlp_grad_block(P, shift, scale, X, T, batch, sp, g, &s_loss);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + TPB * q;
    if (p < NPARAM) G[p] = g[q];
  }
  if (threadIdx.x == 0) *loss = s_loss;
}

__global__ __launch_bounds__(TPB) void k_mlp_train_step(float* __restrict__ P, float* __restrict__ M,
                                                        float* __restrict__ Vv, const float* __restrict__ shift,
                                                        const float* __restrict__ scale, const float* __restrict__ X,
                                                        const float* __restrict__ T, int batch, float lr, int step,
                                                        float* __restrict__ loss) {
  __shared__ float sp[NPARAM];
  __shared__ float s_loss;
  float g[PPT];
  mlp_grad_block(P, shift, scale, X, T, batch, sp, g, &s_loss);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step);
  const float c2 = 1.f - powf(b2, (float)step);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = threadIdx.x + TPB * q;
    if (p >= NPARAM) break;
    const float m = b1 * M[p] + (1.f - b1) * g[q];
    const float v = b2 * Vv[p] + (1.f - b2) * g[q] * g[q];
    M[p] = m;
    Vv[p] = v;
    P[p] = sp[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  }
  if (threadIdx.x == 0) *loss = s_loss;
}

}  // namespace

extern "C" {

int gmresir_mlp_forward(const float* params, const float* shift, const float* scale, const float* X, float* Y,
                        int32_t batch, void* stream) {
  if (!params || !shift || !scale || !X || !Y || batch < 1 || batch > (1 << 24)) {
    gir::set_error("gmresir_mlp_forward: bad arguments");
    return GMRESIR_ERR_INVALID_ARG;
  }
  const int g = (batch + TPB - 1) / TPB;
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(TPB), 0, (hipStream_t)stream, params, shift, scale, X, Y, batch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    gir::set_error("gmresir_mlp_forward: %s", hipGetErrorString(e));
    return GMRESIR_ERR_HIP;
  }
  return GMRESIR_OK;
}

int gmresir_mlp_loss_grad(const float* params, const float* shift, const float* scale, const float* X, const float* T,
                          int32_t batch, float* grad, float* loss, void* stream) {
  if (!params || !shift || !scale || !X || !T || !grad || !loss || batch < 1 || batch > 65536) {
    gir::set_error("gmresir_mlp_loss_grad: bad arguments");
    return GMRESIR_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_mlp_loss_grad, dim3(1), dim3(TPB), 0, (hipStream_t)stream, params, shift, scale, X, T, batch,
                     grad, loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    gir::set_error("gmresir_mlp_loss_grad: %s", hipGetErrorString(e));
    return GMRESIR_ERR_HIP;
  }
  return GMRESIR_OK;
}

int gmresir_mlp_train_step(float* params, float* adam_m, float* adam_v, const float* shift, const float* scale,
                           const float* X, const float* T, int32_t batch, float lr, int32_t step, float* loss,
                           void* stream) {
  if (!params || !adam_m || !adam_v || !shift || !scale || !X || !T || !loss || batch < 1 || batch > 65536 ||
      step < 1 || !(lr > 0.f)) {
    gir::set_error("gmresir_mlp_train_step: bad arguments");
    return GMRESIR_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_mlp_train_step, dim3(1), dim3(TPB), 0, (hipStream_t)stream, params, adam_m, adam_v, shift,
                     scale, X, T, batch, lr, step, loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    gir::set_error("gmresir_mlp_train_step: %s", hipGetErrorString(e));
    return GMRESIR_ERR_HIP;
  }
  return GMRESIR_OK;
}

}  // extern "C"
