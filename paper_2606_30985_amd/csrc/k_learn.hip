// Learned warm start of the measurement BP (edge-wise perceptron).
//
// The paper's BP starts from uniform messages and shows that a BP can land on
// another fixed point (Sec. "BP Fixed-Point Multiplicity").  Here a small
// network, trained on fixed points the method itself produced, proposes the
// measurement-BP messages of a layer; uniform-start BP stays the fallback and
// the reference.  Every component k of every directed edge message is one row:
//   x = (base_k, one_k, prev_k, has_prev, sqrt(chi) lam_k, k/chi, 1/sqrt(chi),
//        deg(u)/4, u is the observable site, dist(u, c)/(Lx+Ly),
//        dist(v, c) - dist(u, c), h dt, J dt, t, log chi / log chi_max, 0)
// where one = the outgoing message after one sweep from the uniform start
// (normalised), prev = the previous measurement's converged message (zero
// past its length), base = prev where it exists, else one.  The network
// predicts the correction y with m_warm = normalise(base + y).
// Weights and inputs enter the products as BF16 (round to nearest even),
// sums are float32 in a fixed order.  The edge messages are short (chi <=
// 256 entries) and the whole row count is 2 chi per bond, so the products
// are plain FMA loops (no MFMA tiling pays at this size).
#include <cmath>

#include "common.h"
#include "learn.h"

namespace hpt {
namespace {

__device__ inline float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

__device__ inline float wsum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wsum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sign making the sum non-negative (the largest-magnitude entry decides a
// zero sum); the Bethe sum is invariant to each message's sign
__device__ inline double edge_sign(double sum, double amax_signed) {
  if (sum > 0.0) return 1.0;
  if (sum < 0.0) return -1.0;
  return amax_signed < 0.0 ? -1.0 : 1.0;
}

// norm, sign of a vector of n doubles held by one wave
__device__ inline void norm_sign(const double* v, int n, double& inv, double& sg) {
  const int lane = threadIdx.x & 63;
  double s2 = 0.0, s1 = 0.0, am = 0.0;
  for (int k = lane; k < n; k += 64) {
    const double x = v[k];
    s2 += x * x;
    s1 += x;
    if (fabs(x) > fabs(am)) am = x;
  }
  s2 = wsum_d(s2);
  s1 = wsum_d(s1);
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_xor(am, o, 64);
    if (fabs(other) > fabs(am) || (fabs(other) == fabs(am) && other > am)) am = other;
  }
  inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  sg = edge_sign(s1, am);
}

__global__ __launch_bounds__(64) void learn_features_kernel(const LearnEdge* edges, LearnGlobals g, float* X,
                                                            float* base) {
  const LearnEdge e = edges[blockIdx.x];
  const int lane = threadIdx.x;
  double inv1, sg1, invp = 0.0, sgp = 1.0;
  norm_sign(e.one, e.chi, inv1, sg1);
  if (e.prev && e.chi_prev > 0) norm_sign(e.prev, e.chi_prev, invp, sgp);
  const float c = (float)e.chi;
  for (int k = lane; k < e.chi; k += 64) {
    const float one = (float)(sg1 * inv1 * e.one[k]);
    const bool hp = e.prev && k < e.chi_prev;
    const float prev = hp ? (float)(sgp * invp * e.prev[k]) : 0.0f;
    const float b = hp ? prev : one;
    float* x = X + (e.row0 + k) * LEARN_F;
    x[0] = b;
    x[1] = one;
    x[2] = prev;
    x[3] = hp ? 1.0f : 0.0f;
    x[4] = (float)(e.lam[k]) * sqrtf(c);
    x[5] = (float)k / c;
    x[6] = 1.0f / sqrtf(c);
    x[7] = e.deg * 0.25f;
    x[8] = e.obs;
    x[9] = e.dist;
    x[10] = e.dir;
    x[11] = g.h_dt;
    x[12] = g.J_dt;
    x[13] = g.t;
    x[14] = logf(c) * g.inv_log_chimax;
    x[15] = 0.0f;
    base[e.row0 + k] = b;
  }
}

// one thread per row; W1 and w2 (BF16-rounded) and b1 in LDS
__global__ __launch_bounds__(256) void learn_forward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                            int64_t rows, float* __restrict__ y) {
  __shared__ float W1[LEARN_H * LEARN_F];
  __shared__ float b1[LEARN_H], w2[LEARN_H];
  for (int i = threadIdx.x; i < LEARN_H * LEARN_F; i += blockDim.x) W1[i] = bf16r(P[i]);
  for (int i = threadIdx.x; i < LEARN_H; i += blockDim.x) {
    b1[i] = P[LEARN_H * LEARN_F + i];
    w2[i] = bf16r(P[LEARN_H * LEARN_F + LEARN_H + i]);
  }
  __syncthreads();
  const float b2 = P[LEARN_P - 1];
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
    float x[LEARN_F];
#pragma unroll
    for (int f = 0; f < LEARN_F; ++f) x[f] = bf16r(X[r * LEARN_F + f]);
    float acc = 0.0f;
    for (int j = 0; j < LEARN_H; ++j) {
      float z = b1[j];
#pragma unroll
      for (int f = 0; f < LEARN_F; ++f) z = fmaf(W1[j * LEARN_F + f], x[f], z);
      acc = fmaf(w2[j], tanhf(z), acc);
    }
    y[r] = acc + b2;
  }
}

__global__ __launch_bounds__(64) void learn_warm_kernel(const LearnEdge* edges, const float* base, const float* y) {
  const LearnEdge e = edges[blockIdx.x];
  const int lane = threadIdx.x;
  double s2 = 0.0, s1 = 0.0, am = 0.0;
  for (int k = lane; k < e.chi; k += 64) {
    const double m = (double)base[e.row0 + k] + (double)y[e.row0 + k];
    s2 += m * m;
    s1 += m;
    if (fabs(m) > fabs(am)) am = m;
  }
  s2 = wsum_d(s2);
  s1 = wsum_d(s1);
  for (int o = 32; o > 0; o >>= 1) {
    const double other = __shfl_xor(am, o, 64);
    if (fabs(other) > fabs(am) || (fabs(other) == fabs(am) && other > am)) am = other;
  }
  const double sg = edge_sign(s1, am);
  // a zero prediction falls back to the uniform start
  const double inv = s2 > 0.0 ? sg / sqrt(s2) : 0.0;
  for (int k = lane; k < e.chi; k += 64) {
    const double m = (double)base[e.row0 + k] + (double)y[e.row0 + k];
    e.out[k] = s2 > 0.0 ? m * inv : 1.0 / sqrt((double)e.chi);
  }
}

// targets of the training rows: T = normalise(m) - base for the converged
// message m of every edge (read through LearnEdge::one)
__global__ __launch_bounds__(64) void learn_targets_kernel(const LearnEdge* edges, const float* base, float* T) {
  const LearnEdge e = edges[blockIdx.x];
  double inv, sg;
  norm_sign(e.one, e.chi, inv, sg);
  for (int k = threadIdx.x; k < e.chi; k += 64)
    T[e.row0 + k] = (float)(sg * inv * e.one[k] - (double)base[e.row0 + k]);
}

// Workgroup j < LEARN_H: the 18 gradient entries of hidden unit j (W1[j, :],
// b1[j], w2[j]); workgroup LEARN_H: b2 and the loss.  Each thread sums its
// rows (r = tid, tid + 256, ...) in order, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void learn_backward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                             const float* __restrict__ y, const float* __restrict__ t,
                                                             int64_t rows, float* __restrict__ grad) {
  constexpr int NV = LEARN_F + 2;
  __shared__ float red[NV][256];
  const int j = blockIdx.x, tid = threadIdx.x;
  const float scale = 2.0f / (float)rows;
  float acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0f;
  if (j < LEARN_H) {
    float w[LEARN_F];
#pragma unroll
    for (int f = 0; f < LEARN_F; ++f) w[f] = bf16r(P[j * LEARN_F + f]);
    const float b1 = P[LEARN_H * LEARN_F + j];
    const float w2 = bf16r(P[LEARN_H * LEARN_F + LEARN_H + j]);
    for (int64_t r = tid; r < rows; r += 256) {
      float x[LEARN_F];
      float z = b1;
#pragma unroll
      for (int f = 0; f < LEARN_F; ++f) {
        x[f] = bf16r(X[r * LEARN_F + f]);
        z = fmaf(w[f], x[f], z);
      }
      const float a = tanhf(z);
      const float dy = scale * (y[r] - t[r]);
      const float dz = dy * w2 * (1.0f - a * a);
#pragma unroll
      for (int f = 0; f < LEARN_F; ++f) acc[f] = fmaf(dz, x[f], acc[f]);
      acc[LEARN_F] += dz;
      acc[LEARN_F + 1] = fmaf(dy, a, acc[LEARN_F + 1]);
    }
  } else {
    for (int64_t r = tid; r < rows; r += 256) {
      const float d = y[r] - t[r];
      acc[0] += scale * d;
      acc[1] = fmaf(d, d, acc[1]);
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) red[q][tid] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w)
#pragma unroll
      for (int q = 0; q < NV; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    if (j < LEARN_H) {
      for (int f = 0; f < LEARN_F; ++f) grad[j * LEARN_F + f] = red[f][0];
      grad[LEARN_H * LEARN_F + j] = red[LEARN_F][0];
      grad[LEARN_H * LEARN_F + LEARN_H + j] = red[LEARN_F + 1][0];
    } else {
      grad[LEARN_P - 1] = red[0][0];
      grad[LEARN_P] = red[1][0] / (float)rows;
    }
  }
}

__global__ void learn_adam_kernel(float* P, float* m, float* v, const float* g, int step, float lr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= LEARN_P) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)step));
  const float vh = vi / (1.0f - powf(b2, (float)step));
  P[i] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

int launch_learn_features(const LearnEdge* edges, int nedges, LearnGlobals g, float* X, float* base, hipStream_t s) {
  if (nedges <= 0) return 0;
  hipLaunchKernelGGL(learn_features_kernel, dim3(nedges), dim3(64), 0, s, edges, g, X, base);
  HPT_LAUNCH_CHECK("learn_features_kernel");
  return 0;
}

int launch_learn_forward(const float* params, const float* X, int64_t rows, float* y, hipStream_t s) {
  if (rows <= 0) return 0;
  const int64_t blocks = std::min<int64_t>(ceil_div(rows, 256), 4096);
  hipLaunchKernelGGL(learn_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, s, params, X, rows, y);
  HPT_LAUNCH_CHECK("learn_forward_kernel");
  return 0;
}

int launch_learn_warm(const LearnEdge* edges, int nedges, const float* base, const float* y, hipStream_t s) {
  if (nedges <= 0) return 0;
  hipLaunchKernelGGL(learn_warm_kernel, dim3(nedges), dim3(64), 0, s, edges, base, y);
  HPT_LAUNCH_CHECK("learn_warm_kernel");
  return 0;
}

int launch_learn_targets(const LearnEdge* edges, int nedges, const float* base, float* T, hipStream_t s) {
  if (nedges <= 0) return 0;
  hipLaunchKernelGGL(learn_targets_kernel, dim3(nedges), dim3(64), 0, s, edges, base, T);
  HPT_LAUNCH_CHECK("learn_targets_kernel");
  return 0;
}

int launch_learn_backward(const float* params, const float* X, const float* y, const float* t, int64_t rows,
                          float* grad, hipStream_t s) {
  if (rows <= 0) return -1;
  hipLaunchKernelGGL(learn_backward_kernel, dim3(LEARN_H + 1), dim3(256), 0, s, params, X, y, t, rows, grad);
  HPT_LAUNCH_CHECK("learn_backward_kernel");
  return 0;
}

int launch_learn_adam(float* params, float* m, float* v, const float* grad, int step, float lr, hipStream_t s) {
  if (step < 1) return -1;
  hipLaunchKernelGGL(learn_adam_kernel, dim3((LEARN_P + 255) / 256), dim3(256), 0, s, params, m, v, grad, step, lr);
  HPT_LAUNCH_CHECK("learn_adam_kernel");
  return 0;
}

}  // namespace hpt
