// Stand-alone C ABI entry points of single steps of the gate update, on
// caller device buffers (no simulator handle): the float64 Gram of the
// CholeskyQR first pass (Sec. "Adaptive QR Decomposition", Eq. cholqr) and
// the float32 mode product of the absorb step (Sec. "Gate Update"); the
// switch and report of the launch-shape autotuner.
#include <cstdint>
#include <mutex>

#include "../../include/hpt.h"
#include "common.h"
#include "learn.h"
#include "tune.h"

// Scratch of hpt_gram64_noalloc: the per-split partial tiles live in this
// file-scope device array (one copy per GPU, held until the process ends)
// instead of a caller workspace.  Host code never passes the symbol itself to
// a kernel: it uses the device address from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[HPT_GRAM64_PART_MAX / 8];

namespace hpt {
namespace {

// device address of `scratch` on each GPU, looked up once per device with
// that device current (its first hpt_gram64_noalloc call)
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return HPT_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_hip_error(e, "hipGetSymbolAddress(scratch)");
      return HPT_EHIP;
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return HPT_OK;
}

// shared argument checks; *splits receives the row-split count
int gram64_args(const float* X, int64_t m, int32_t n, int64_t ldx, const double* G, int64_t ldg, int* splits) {
  if (m < 0 || n < 0 || m > 0x7fffffff - 64) return HPT_EINVAL;
  if (n == 0) {
    *splits = 0;
    return HPT_OK;
  }
  if ((!X && m > 0) || !G || ldx < m || ldg < n) return HPT_EINVAL;
  *splits = gram64_splits(m, n, (int64_t)(HPT_GRAM64_PART_MAX / 8));
  return HPT_OK;
}

}  // namespace
}  // namespace hpt

using namespace hpt;

extern "C" {

int hpt_gram64_workspace_bytes(int64_t m, int32_t n, uint64_t* bytes) {
  if (!bytes || m < 0 || n < 0 || m > 0x7fffffff - 64) return HPT_EINVAL;
  *bytes = n == 0 ? 0 : (uint64_t)gram64_splits(m, n, (int64_t)(HPT_GRAM64_PART_MAX / 8)) * n * n * 8;
  return HPT_OK;
}

int hpt_gram64(const float* X, int64_t m, int32_t n, int64_t ldx, double* G, int64_t ldg, void* workspace,
               uint64_t workspace_bytes, void* hip_stream) {
  int splits = 0;
  const int r = gram64_args(X, m, n, ldx, G, ldg, &splits);
  if (r || n == 0) return r;
  const uint64_t need = (uint64_t)splits * n * n * 8;
  if (!workspace || workspace_bytes < need) return HPT_ENOMEM;
  if (gram64_launch(X, ldx, (int)m, n, G, ldg, splits, (double*)workspace, (hipStream_t)hip_stream)) return HPT_EHIP;
  return HPT_OK;
}

int hpt_learn_forward(const float* params, const float* X, int64_t rows, float* y, void* hip_stream) {
  if (!params || rows < 0 || (rows > 0 && (!X || !y))) return HPT_EINVAL;
  return launch_learn_forward(params, X, rows, y, (hipStream_t)hip_stream) ? HPT_EHIP : HPT_OK;
}

int hpt_learn_backward(const float* params, const float* X, const float* y, const float* t, int64_t rows,
                       float* grad, void* hip_stream) {
  if (!params || !X || !y || !t || !grad || rows < 1) return HPT_EINVAL;
  return launch_learn_backward(params, X, y, t, rows, grad, (hipStream_t)hip_stream) ? HPT_EHIP : HPT_OK;
}

int hpt_learn_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr,
                   void* hip_stream) {
  if (!params || !m || !v || !grad || step < 1 || !(lr > 0.0f)) return HPT_EINVAL;
  return launch_learn_adam(params, m, v, grad, step, lr, (hipStream_t)hip_stream) ? HPT_EHIP : HPT_OK;
}

int hpt_bf16_mfma_sum(const float* a, float c, float* out, void* hip_stream) {
  if (!a || !out) return HPT_EINVAL;
  return bf16_mfma_sum(a, c, out, (hipStream_t)hip_stream) ? HPT_EHIP : HPT_OK;
}

int hpt_mode_product_f32(const float* src, float* dst, const float* S, int32_t n, int64_t inner, int64_t outer,
                         void* hip_stream) {
  if (!src || !dst || !S || n < 1 || n > 128 || inner < 1 || outer < 1) return HPT_EINVAL;
  if ((inner == 1 && outer < 16) || (inner > 1 && inner < 16) || inner * n >= ((int64_t)1 << 30)) return HPT_EINVAL;
  const int r = mode_product_f32(S, src, dst, n, inner, outer, (hipStream_t)hip_stream);
  return r < 0 ? HPT_EHIP : (r == 0 ? HPT_EINVAL : HPT_OK);
}

int hpt_autotune(int32_t mode) { return tune_set(mode) ? HPT_EINVAL : HPT_OK; }

int hpt_autotune_report(char* buf, uint64_t cap, uint64_t* needed) {
  if (!buf && cap > 0) return HPT_EINVAL;
  return tune_report(buf, cap, needed) ? HPT_EINVAL : HPT_OK;
}

int hpt_gram64_noalloc(const float* X, int64_t m, int32_t n, int64_t ldx, double* G, int64_t ldg,
                       void* hip_stream) {
  int splits = 0;
  const int r = gram64_args(X, m, n, ldx, G, ldg, &splits);
  if (r || n == 0) return r;
  if ((uint64_t)splits * n * n * 8 > HPT_GRAM64_PART_MAX) return HPT_EINVAL;   // n > HPT_GRAM64_NOALLOC_MAX_N
  double* part = nullptr;
  const int rs = scratch_on_current_device(&part);
  if (rs) return rs;
  if (gram64_launch(X, ldx, (int)m, n, G, ldg, splits, part, (hipStream_t)hip_stream)) return HPT_EHIP;
  return HPT_OK;
}

}  // extern "C"
