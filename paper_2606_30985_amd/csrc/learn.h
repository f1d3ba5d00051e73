// Learned warm start of the measurement BP: features of every component of
// every directed edge message, the edge-wise two-layer perceptron (BF16
// weights and inputs, float32 accumulation), its backward pass and the Adam
// update, and the writer of the warm messages (k_learn.hip).
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hpt {

constexpr int LEARN_F = 16;    // features per row
constexpr int LEARN_H = 128;   // hidden width
constexpr int LEARN_P = LEARN_H * LEARN_F + 2 * LEARN_H + 1;   // W1, b1, w2, b2

// One directed edge u -> v of the measurement BP.
struct LearnEdge {
  const double* prev;   // converged message of the previous measurement (chi_prev entries) or null
  const double* one;    // outgoing message after one sweep from the uniform start (unnormalised)
  const double* lam;    // Vidal values of the bond (chi entries)
  double* out;          // destination of the warm message (chi entries)
  int chi, chi_prev;
  int64_t row0;         // first row of this edge
  float deg, obs, dist, dir;
};

struct LearnGlobals {
  float h_dt, J_dt, t, inv_log_chimax;
};

// X (rows x LEARN_F, row-major) and base (rows) for every edge: one wave per edge
int launch_learn_features(const LearnEdge* edges, int nedges, LearnGlobals g, float* X, float* base, hipStream_t s);
// y = w2 . tanh(W1 x + b1) + b2 for every row (W1, w2 and x rounded to BF16)
int launch_learn_forward(const float* params, const float* X, int64_t rows, float* y, hipStream_t s);
// warm message of every edge: normalise(base + y) (L2, sum >= 0), written as float64
int launch_learn_warm(const LearnEdge* edges, int nedges, const float* base, const float* y, hipStream_t s);
// T = normalise(m) - base with m read through LearnEdge::one (converged messages)
int launch_learn_targets(const LearnEdge* edges, int nedges, const float* base, float* T, hipStream_t s);
// gradient of L = sum (y - t)^2 / rows with respect to the parameters (LEARN_P
// floats) and L itself in grad[LEARN_P]; fixed summation order
int launch_learn_backward(const float* params, const float* X, const float* y, const float* t, int64_t rows,
                          float* grad, hipStream_t s);
// one Adam step on params with moments m, v (step >= 1)
int launch_learn_adam(float* params, float* m, float* v, const float* grad, int step, float lr, hipStream_t s);

}  // namespace hpt
