// Shared definitions of the libhpt HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <algorithm>

namespace hpt {

typedef __attribute__((ext_vector_type(4))) double d4;
typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8;

// Error handling: every HIP call in host code goes through HPT_HIP.
void set_hip_error(hipError_t e, const char* what);
#define HPT_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) {                             \
      ::hpt::set_hip_error(_e, #call);                  \
      return -3;                                        \
    }                                                   \
  } while (0)
#define HPT_LAUNCH_CHECK(what)                          \
  do {                                                  \
    hipError_t _e = hipGetLastError();                  \
    if (_e != hipSuccess) {                             \
      ::hpt::set_hip_error(_e, what);                   \
      return -3;                                        \
    }                                                   \
  } while (0)

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Batched, batch-reducing GEMM on MFMA (k_gemm.hip).
//   C[z] = alpha * sum_{r < R} op(A[z, r]) op(B[z, r]) + beta * C[z]
// column-major operands; op(A) is M x K, op(B) is K x N.  A[z, r] starts at
// A + z*sAz + r*sAr (same for B), C[z] at C + z*sCz.  Output type OutT is T
// or double; with splits > 1 partial tiles go through `part` (double,
// splits * Z * M * N entries) and a deterministic second pass.
template <typename T>
struct GemmDesc {
  int M, N, K, R, Z;
  const T* A; int64_t lda, sAz, sAr; int tA;
  const T* B; int64_t ldb, sBz, sBr; int tB;
  void* C; int64_t ldc, sCz; int c_double;
  double alpha, beta;
  int sym;   // op(B) = op(A)^T and M == N: only tiles on or above the diagonal
             // are computed, the result is mirrored (a SYRK)
  int acc64; // float inputs multiplied and accumulated in float64 (f64 MFMA)
  int bsplit; // float inputs: six bf16 MFMA products of the three-way bf16 split
              // of each operand, float32 accumulation (plain products only)
};
template <typename T>
int gemm(const GemmDesc<T>& d, double* part, int64_t part_cap, hipStream_t s);

// float64 Gram of float32 data (CholeskyQR first pass): row splits for a
// partial buffer of part_cap doubles, and the launch (part: splits n^2 doubles)
int gram64_splits(int64_t m, int n, int64_t part_cap);
int gram64_launch(const float* X, int64_t ldx, int m, int n, double* G, int64_t ldg, int splits, double* part,
                  hipStream_t s);

// process-wide event timing of the contraction launches; kind 0 gemm_pipe_kernel,
// 1 the float64-accumulated Gram of float data, 2 mode_product_kernel, 3 leg_gram_kernel, -1 all
int gemm_profile(int enable);
int gemm_profile_read(int kind, double* out4);
int gemm_profile_active();

// Mode product of the float32 form, dst = src x_axis S with the n x n factor
// S resident in LDS: dst[a, j, b] = sum_k S[j, k] src[a, k, b] for a < inner,
// b < outer (column-major).  Returns 1 when done, 0 when the shape is not
// served (n > 128, or a short leading extent; the caller uses gemm), < 0 on
// a HIP error.
int mode_product_f32(const float* S, const float* src, float* dst, int n, int64_t inner, int64_t outer,
                     hipStream_t s);

// Mode product of float32 data with a float64 factor in float64 arithmetic:
// dst[a, j, b] = sum_k S[j, k] src[a, k, b] (S n x n column-major), float64
// products and sums in increasing k, each result rounded once to float32.
// For the environment factors of the float32 form's Householder route, whose
// absorb/deabsorb pair must multiply to the projector to float64 accuracy.
// Returns 0, or < 0 on a HIP error / bad size.
int mode_product_f64acc(const double* S, const float* src, float* dst, int n, int64_t inner, int64_t outer,
                        hipStream_t s);

// One bf16 MFMA (16x16x32) summing 32 values a (device, float32, rounded to
// bf16) onto c in every output (out: 256 floats, device)
int bf16_mfma_sum(const float* a, float c, float* out, hipStream_t s);

// Leg Gram of the float32 form: out[i, j] (n x n, float64) = sum over a < inner,
// b < outer of psi[a, i, b] cur[a, j, b] (column-major), float32 MFMA products
// accumulated per workgroup, float64 partials (part, n^2 per workgroup, at
// most part_cap entries) summed in a fixed order.  Returns 1 when done, 0 when
// not served (n > 128), < 0 on a HIP error.
int leg_gram_f32(const float* psi, const float* cur, int n, int64_t inner, int64_t outer, double* out, double* part,
                 int64_t part_cap, hipStream_t s);

// Tensor permutation (k_permute.hip).
int permute_generic(const void* in, void* out, int ndim, const int64_t* dims,
                    const int* perm, int elem, hipStream_t s);
// out[a, c, b, p] = in[a, b, c, p] for an (A, B, C, P) column-major tensor.
int permute_swap_mid(const void* in, void* out, int64_t A, int64_t B, int64_t C,
                     int64_t P, int elem, hipStream_t s);

}  // namespace hpt
