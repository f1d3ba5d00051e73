// Small dense float64 factorisations of the gate update, one workgroup per
// problem (batched over the bonds of one colour and their environment legs).
//
//  * pseudo_sqrt: cyclic two-sided Jacobi eigensolver (round-robin parallel
//    ordering) and sqrt(M), M^{-1/2} with the eigenvalue cutoff
//    (paper Algorithm "Gate update", first step; Sec. "Gate Update" item 1).
//  * Householder QR with explicit Q (Sec. "Adaptive QR Decomposition",
//    Householder path) -- LAPACK dlarfg/dorg2r conventions, R diagonal >= 0.
//  * One-sided (Hestenes) Jacobi SVD (Sec. "Adaptive QR Decomposition",
//    paragraph "SVD and Truncation").
//  * Upper Cholesky and triangular inverse (Eq. cholqr, run as CholeskyQR2).
//  * A plain batched float64 GEMM for the few-hundred-wide R-core products.
#include "linalg.h"
#include "wave.h"

namespace hpt {

namespace {

// gate semantics of the batched jobs: no gate -> run; gate_zero -> run when
// *gate == 0; otherwise run when *gate != 0
__device__ inline bool gated_out(const int* gate, int gate_zero) {
  if (!gate) return false;
  return gate_zero ? (*gate != 0) : (*gate == 0);
}


// deterministic block sum: wave butterflies, then every thread adds the
// per-wave partials in the same order
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  return r;
}

// round-robin pairing: round r of n2 - 1, pair k of n2 / 2 (circle method)
__device__ inline void rr_pair(int r, int k, int n2, int& p, int& q) {
  const int m = n2 - 1;
  if (k == 0) {
    p = r;
    q = m;
  } else {
    p = (r + k) % m;
    q = (r - k + m) % m;
  }
}

__device__ inline void jacobi_rotation(double app, double aqq, double apq, double& c, double& s) {
  const double theta = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(theta) > 1e150)
    t = 0.5 / theta;
  else
    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  c = 1.0 / sqrt(t * t + 1.0);
  s = t * c;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pseudo_sqrt_kernel(const PsqJob* jobs, double eps_pinv) {
  const PsqJob job = jobs[blockIdx.x];
  const int n = job.n;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* A = job.work;
  double* V = job.work + (int64_t)n * n;
  __shared__ double cs_c[256], cs_s[256];
  __shared__ int s_rot;
  __shared__ double sh[16];
  __shared__ double s_w[512];

  for (int idx = tid; idx < n * n; idx += nt) {
    const int i = idx % n, j = idx / n;
    A[idx] = 0.5 * (job.M[i + j * n] + job.M[j + i * n]);
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int n2 = n + (n & 1);
  const int npairs = n2 / 2;
  if (n > 1) {
    for (int sweep = 0; sweep < 60; ++sweep) {
      if (tid == 0) s_rot = 0;
      __syncthreads();
      for (int r = 0; r < n2 - 1; ++r) {
        for (int k = tid; k < npairs; k += nt) {
          int p, q;
          rr_pair(r, k, n2, p, q);
          double c = 1.0, s = 0.0;
          if (p < n && q < n) {
            const double app = A[p + p * n], aqq = A[q + q * n], apq = A[p + q * n];
            if (apq != 0.0 && fabs(apq) > 1e-15 * sqrt(fabs(app * aqq))) {
              jacobi_rotation(app, aqq, apq, c, s);
              s_rot = 1;
            }
          }
          cs_c[k] = c;
          cs_s[k] = s;
        }
        __syncthreads();
        // rows p, q  (A <- J^T A)
        for (int idx = tid; idx < npairs * n; idx += nt) {
          const int k = idx / n, j = idx % n;
          const double s = cs_s[k];
          if (s == 0.0) continue;
          int p, q;
          rr_pair(r, k, n2, p, q);
          const double c = cs_c[k];
          const double ap = A[p + j * n], aq = A[q + j * n];
          A[p + j * n] = c * ap - s * aq;
          A[q + j * n] = s * ap + c * aq;
        }
        __syncthreads();
        // columns p, q  (A <- A J, V <- V J)
        for (int idx = tid; idx < npairs * n; idx += nt) {
          const int k = idx / n, i = idx % n;
          const double s = cs_s[k];
          if (s == 0.0) continue;
          int p, q;
          rr_pair(r, k, n2, p, q);
          const double c = cs_c[k];
          const double ap = A[i + p * n], aq = A[i + q * n];
          A[i + p * n] = c * ap - s * aq;
          A[i + q * n] = s * ap + c * aq;
          const double vp = V[i + p * n], vq = V[i + q * n];
          V[i + p * n] = c * vp - s * vq;
          V[i + q * n] = s * vp + c * vq;
        }
        __syncthreads();
        // the rotation annihilates (p, q) exactly; drop the rounding residue
        for (int k = tid; k < npairs; k += nt) {
          if (cs_s[k] == 0.0) continue;
          int p, q;
          rr_pair(r, k, n2, p, q);
          A[p + q * n] = 0.0;
          A[q + p * n] = 0.0;
        }
        __syncthreads();
      }
      if (!s_rot) break;
      __syncthreads();
    }
  }
  // eigenvalues, cutoff
  for (int i = tid; i < n; i += nt) s_w[i] = A[i + i * n];
  __syncthreads();
  double wmax = -1e308;
  for (int i = 0; i < n; ++i) wmax = fmax(wmax, s_w[i]);
  __syncthreads();
  if (!(wmax > 0.0)) {
    if (tid == 0) *job.ncut = -1;
    return;
  }
  if (tid == 0) {
    int cut = 0;
    for (int i = 0; i < n; ++i)
      if (!(s_w[i] > eps_pinv * wmax)) ++cut;
    *job.ncut = cut;
  }
  __syncthreads();
  // S = V f(w) V^T
  for (int idx = tid; idx < n * n; idx += nt) {
    const int i = idx % n, j = idx / n;
    double sq = 0.0, isq = 0.0;
    for (int k = 0; k < n; ++k) {
      const double w = s_w[k];
      if (!(w > eps_pinv * wmax)) continue;
      const double vv = V[i + k * n] * V[j + k * n];
      const double r = sqrt(w);
      sq += vv * r;
      isq += vv / r;
    }
    job.S[idx] = sq;
    job.Sinv[idx] = isq;
    if (job.S32) job.S32[idx] = (float)sq;
    if (job.Sinv32) job.Sinv32[idx] = (float)isq;
  }
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void householder_kernel(const QrJob<T>* jobs) {
  const QrJob<T> job = jobs[blockIdx.x];
  if (gated_out(job.gate, job.gate_zero)) return;
  const int m = job.m, n = job.n, k = m < n ? m : n;
  T* A = job.A;
  const int64_t lda = job.lda;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  __shared__ double sh[16];
  __shared__ double s_beta[1024];   // min(m, n) <= 1024 enforced by the caller
  constexpr int VMAX = 4096;        // reflectors of up to this length are staged in LDS
  __shared__ double s_v[VMAX];
  double* tau = job.tau;

  for (int j = 0; j < k; ++j) {
    // alpha is read before the barriers inside block_sum; thread 0 overwrites
    // A[j, j] only after them
    const double alpha = (double)A[j + j * lda];
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += blockDim.x) {
      const double x = (double)A[i + j * lda];
      part += x * x;
    }
    const double ss = block_sum(part, sh);
    double beta, t;
    if (ss == 0.0) {
      t = 0.0;
      beta = alpha;
    } else {
      const double sigma = sqrt(alpha * alpha + ss);
      beta = alpha >= 0.0 ? -sigma : sigma;
      t = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      for (int i = j + 1 + tid; i < m; i += blockDim.x)
        A[i + j * lda] = (T)((double)A[i + j * lda] * scal);
    }
    if (tid == 0) {
      tau[j] = t;
      s_beta[j] = beta;
      A[j + j * lda] = (T)beta;
    }
    __syncthreads();
    const bool staged = m - j - 1 <= VMAX;
    if (t != 0.0 && staged)
      for (int i = j + 1 + tid; i < m; i += blockDim.x) s_v[i - j - 1] = (double)A[i + j * lda];
    __syncthreads();
    if (t != 0.0) {
      // one wave per trailing column
      for (int c = j + 1 + wave; c < n; c += nw) {
        double w = 0.0;
        if (staged)
          for (int i = j + 1 + lane; i < m; i += 64) w += s_v[i - j - 1] * (double)A[i + c * lda];
        else
          for (int i = j + 1 + lane; i < m; i += 64) w += (double)A[i + j * lda] * (double)A[i + c * lda];
        w = wave_sum(w) + (double)A[j + c * lda];
        w *= t;
        if (lane == 0) A[j + c * lda] = (T)((double)A[j + c * lda] - w);
        if (staged)
          for (int i = j + 1 + lane; i < m; i += 64) A[i + c * lda] = (T)((double)A[i + c * lda] - s_v[i - j - 1] * w);
        else
          for (int i = j + 1 + lane; i < m; i += 64)
            A[i + c * lda] = (T)((double)A[i + c * lda] - (double)A[i + j * lda] * w);
      }
    }
    __syncthreads();
  }
  // R with non-negative diagonal
  for (int idx = tid; idx < k * n; idx += blockDim.x) {
    const int i = idx % k, c = idx / k;
    const double sg = s_beta[i] < 0.0 ? -1.0 : 1.0;
    double v = 0.0;
    if (c == i)
      v = s_beta[i] * sg;
    else if (c > i)
      v = (double)A[i + c * lda] * sg;
    job.R[i + (int64_t)c * job.ldr] = v;
  }
  __syncthreads();
  if (!job.form_q) return;
  for (int j = k - 1; j >= 0; --j) {
    const double t = tau[j];
    for (int c = j + 1 + wave; c < k; c += nw) {
      double w = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) w += (double)A[i + j * lda] * (double)A[i + c * lda];
      w = wave_sum(w) * t;
      if (lane == 0) A[j + c * lda] = (T)(-w);
      for (int i = j + 1 + lane; i < m; i += 64)
        A[i + c * lda] = (T)((double)A[i + c * lda] - (double)A[i + j * lda] * w);
    }
    __syncthreads();
    for (int i = tid; i < m; i += blockDim.x) {
      double v;
      if (i < j)
        v = 0.0;
      else if (i == j)
        v = 1.0 - t;
      else
        v = -t * (double)A[i + j * lda];
      A[i + j * lda] = (T)v;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < m * k; idx += blockDim.x) {
    const int i = idx % m, c = idx / m;
    if (s_beta[c] < 0.0) A[i + c * lda] = (T)(-(double)A[i + c * lda]);
  }
}

// ---------------------------------------------------------------------------
// Blocked Householder QR of one float64 m x n block per workgroup (m <= HBM):
// the same reflectors, R and explicit Q as householder_kernel, with the work
// reorganised into panels of HP columns (LAPACK's compact WY form,
// H_1 ... H_b = I - V T V^T).  A panel is factored in LDS; the trailing
// columns are then updated 16 at a time, staged through LDS, as
// C <- C - V T^T (V^T C); Q = H_1 ... H_k is accumulated backwards over the
// panels with C <- C - V T (V^T C).  Per panel step the sequential part
// touches only the panel's columns, and the products run on all 1024 threads.
constexpr int HP = 16;            // panel width
constexpr int HBM = 512;          // rows held in LDS
constexpr int HLD = HBM + 1;      // LDS column stride (odd: the 16 columns of a read use distinct banks)

// LDS: Vs, Cs [HLD x HP]; Ts, Ws, Ys [HP x HP]; Wp [4 x HP x HP]
constexpr size_t HB_LDS = (size_t)(2 * HLD * HP + 3 * HP * HP + 4 * HP * HP) * sizeof(double);

// partial dot products D[a + HP c] = sum_{i < mr} X[i + HLD a] Y[i + HLD c] for
// a < na, c < nc: four partial sums per entry over rows i = part (mod 4)
__device__ inline void hb_dots(const double* X, const double* Y, int mr, int na, int nc, double* Wp,
                               double* D) {
  const int tid = threadIdx.x, a = tid & 15, c = (tid >> 4) & 15, part = tid >> 8;
  double acc = 0.0;
  if (a < na && c < nc)
    for (int i = part; i < mr; i += 4) acc += X[i + HLD * a] * Y[i + HLD * c];
  Wp[part * HP * HP + a + HP * c] = acc;
  __syncthreads();
  if (tid < HP * HP)
    D[tid] = (Wp[tid] + Wp[HP * HP + tid]) + (Wp[2 * HP * HP + tid] + Wp[3 * HP * HP + tid]);
  __syncthreads();
}

// T (upper triangular, Ts[a + HP b]) of the panel's jb reflectors V (unit
// lower trapezoidal in Vs): T[b, b] = tau_b, T[a, b] = -tau_b sum_{a <= c < b}
// T[a, c] (V^T V)[c, b]; each row of T depends only on itself
__device__ inline void hb_build_T(const double* Vs, int mr, int jb, const double* tau, double* Ts, double* Ys,
                                  double* Wp) {
  hb_dots(Vs, Vs, mr, jb, jb, Wp, Ys);
  if (threadIdx.x < HP) {
    const int a = threadIdx.x;
    double row[HP];
#pragma unroll
    for (int b = 0; b < HP; ++b) {
      double v = 0.0;
      if (a < jb && b < jb) {
        if (b == a) {
          v = tau[b];
        } else if (b > a) {
          double acc = 0.0;
#pragma unroll
          for (int c = 0; c < HP; ++c)
            if (c >= a && c < b) acc += row[c] * Ys[c + HP * b];
          v = -tau[b] * acc;
        }
      }
      row[b] = v;
    }
#pragma unroll
    for (int b = 0; b < HP; ++b) Ts[a + HP * b] = row[b];
  }
  __syncthreads();
}

// C (mr x cw in memory at C, leading dimension ldc) <- C - V op(T) (V^T C),
// op(T) = T^T when trans (applying Q^T), T otherwise (applying Q)
__device__ inline void hb_apply(double* C, int64_t ldc, int mr, int cw, const double* Vs, const double* Ts,
                                int jb, bool trans, double* Cs, double* Ws, double* Ys, double* Wp) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < mr * cw; idx += blockDim.x) {
    const int i = idx % mr, c = idx / mr;
    Cs[i + HLD * c] = C[i + (int64_t)c * ldc];
  }
  __syncthreads();
  hb_dots(Vs, Cs, mr, jb, cw, Wp, Ws);
  if (tid < HP * HP) {
    const int a = tid & 15, c = tid >> 4;
    double v = 0.0;
    if (a < jb && c < cw) {
      if (trans)
        for (int b = 0; b <= a; ++b) v += Ts[b + HP * a] * Ws[b + HP * c];
      else
        for (int b = a; b < jb; ++b) v += Ts[a + HP * b] * Ws[b + HP * c];
    }
    Ys[a + HP * c] = v;
  }
  __syncthreads();
  for (int idx = tid; idx < mr * cw; idx += blockDim.x) {
    const int i = idx % mr, c = idx / mr;
    double v = Cs[i + HLD * c];
#pragma unroll
    for (int a = 0; a < HP; ++a)
      if (a < jb) v -= Vs[i + HLD * a] * Ys[a + HP * c];
    C[i + (int64_t)c * ldc] = v;
  }
  __syncthreads();
}

__global__ __launch_bounds__(1024) void householder_blocked_kernel(const QrJob<double>* jobs) {
  const QrJob<double> job = jobs[blockIdx.x];
  if (gated_out(job.gate, job.gate_zero)) return;
  const int m = job.m, n = job.n, k = m < n ? m : n;
  double* A = job.A;
  const int64_t lda = job.lda;
  double* tau = job.tau;
  extern __shared__ double hlds[];
  double* Vs = hlds;
  double* Cs = Vs + HLD * HP;
  double* Ts = Cs + HLD * HP;
  double* Ws = Ts + HP * HP;
  double* Ys = Ws + HP * HP;
  double* Wp = Ys + HP * HP;
  __shared__ double sh[16];
  __shared__ double s_beta[1024];   // min(m, n) <= 1024 enforced by the caller
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;

  for (int j0 = 0; j0 < k; j0 += HP) {
    const int jb = min(HP, k - j0), mr = m - j0;
    double* Ap = A + j0 + (int64_t)j0 * lda;
    for (int idx = tid; idx < mr * jb; idx += blockDim.x) {
      const int i = idx % mr, c = idx / mr;
      Vs[i + HLD * c] = Ap[i + (int64_t)c * lda];
    }
    __syncthreads();
    // unblocked factorisation of the panel in LDS
    for (int jj = 0; jj < jb; ++jj) {
      // alpha is read before the barriers inside block_sum
      const double alpha = Vs[jj + HLD * jj];
      double part = 0.0;
      for (int i = jj + 1 + tid; i < mr; i += blockDim.x) {
        const double x = Vs[i + HLD * jj];
        part += x * x;
      }
      const double ss = block_sum(part, sh);
      double beta, t;
      if (ss == 0.0) {
        t = 0.0;
        beta = alpha;
      } else {
        const double sigma = sqrt(alpha * alpha + ss);
        beta = alpha >= 0.0 ? -sigma : sigma;
        t = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);
        for (int i = jj + 1 + tid; i < mr; i += blockDim.x) Vs[i + HLD * jj] *= scal;
      }
      if (tid == 0) {
        tau[j0 + jj] = t;
        s_beta[j0 + jj] = beta;
      }
      __syncthreads();
      if (t != 0.0) {
        for (int c = jj + 1 + wave; c < jb; c += nw) {
          double w = 0.0;
          for (int i = jj + 1 + lane; i < mr; i += 64) w += Vs[i + HLD * jj] * Vs[i + HLD * c];
          w = (wave_sum(w) + Vs[jj + HLD * c]) * t;
          for (int i = jj + 1 + lane; i < mr; i += 64) Vs[i + HLD * c] -= Vs[i + HLD * jj] * w;
          if (lane == 0) Vs[jj + HLD * c] -= w;
        }
      }
      __syncthreads();
    }
    // panel back to memory: R above the diagonal, beta on it, v below
    for (int idx = tid; idx < mr * jb; idx += blockDim.x) {
      const int i = idx % mr, c = idx / mr;
      Ap[i + (int64_t)c * lda] = (i == c) ? s_beta[j0 + c] : Vs[i + HLD * c];
    }
    __syncthreads();
    if (j0 + jb >= n) break;
    // V: unit lower trapezoidal
    for (int idx = tid; idx < jb * jb; idx += blockDim.x) {
      const int a = idx % jb, c = idx / jb;
      if (a <= c) Vs[a + HLD * c] = (a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    hb_build_T(Vs, mr, jb, tau + j0, Ts, Ys, Wp);
    for (int c0 = j0 + jb; c0 < n; c0 += HP)
      hb_apply(A + j0 + (int64_t)c0 * lda, lda, mr, min(HP, n - c0), Vs, Ts, jb, true, Cs, Ws, Ys, Wp);
  }
  // R with non-negative diagonal
  for (int idx = tid; idx < k * n; idx += blockDim.x) {
    const int i = idx % k, c = idx / k;
    const double sg = s_beta[i] < 0.0 ? -1.0 : 1.0;
    double v = 0.0;
    if (c == i)
      v = s_beta[i] * sg;
    else if (c > i)
      v = A[i + (int64_t)c * lda] * sg;
    job.R[i + (int64_t)c * job.ldr] = v;
  }
  __syncthreads();
  if (!job.form_q) return;
  // Q = H_1 ... H_k (m x k), panels from the last: columns >= j0 + jb hold the
  // product of the later panels (rows < j0 zero), the panel's own columns
  // start as the identity
  for (int j0 = ((k - 1) / HP) * HP; j0 >= 0; j0 -= HP) {
    const int jb = min(HP, k - j0), mr = m - j0;
    double* Ap = A + j0 + (int64_t)j0 * lda;
    for (int idx = tid; idx < mr * jb; idx += blockDim.x) {
      const int i = idx % mr, c = idx / mr;
      Vs[i + HLD * c] = i < c ? 0.0 : (i == c ? 1.0 : Ap[i + (int64_t)c * lda]);
    }
    __syncthreads();
    for (int idx = tid; idx < m * jb; idx += blockDim.x) {
      const int i = idx % m, c = idx / m;
      A[i + (int64_t)(j0 + c) * lda] = (i == j0 + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    hb_build_T(Vs, mr, jb, tau + j0, Ts, Ys, Wp);
    for (int c0 = j0; c0 < k; c0 += HP)
      hb_apply(A + j0 + (int64_t)c0 * lda, lda, mr, min(HP, k - c0), Vs, Ts, jb, false, Cs, Ws, Ys, Wp);
  }
  for (int idx = tid; idx < m * k; idx += blockDim.x) {
    const int i = idx % m, c = idx / m;
    if (s_beta[c] < 0.0) A[i + (int64_t)c * lda] = -A[i + (int64_t)c * lda];
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void jacobi_svd_kernel(const SvdJob* jobs) {
  const SvdJob job = jobs[blockIdx.x];
  const int m = job.m, n = job.n;
  double* G = job.G;
  double* V = job.V;
  const int ldg = job.ldg, ldv = job.ldv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  __shared__ int s_rot, s_off;
  __shared__ double s_sig[1024];
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int n2 = n + (n & 1), npairs = n2 / 2;
  const double tol = 1e-15 * sqrt((double)m);
  __shared__ double s_dead2;
  {
    double f = 0.0;
    for (int idx = tid; idx < m * n; idx += blockDim.x) {
      const double x = G[idx % m + (idx / m) * ldg];
      f += x * x;
    }
    __shared__ double sh[16];
    f = block_sum(f, sh);
    if (tid == 0) s_dead2 = 1e-28 * f;
    __syncthreads();
  }
  const double dead2 = s_dead2;
  const int maxs = job.max_sweeps > 0 ? job.max_sweeps : 60;
  int sweep = 0;
  if (n > 1) {
    for (sweep = 0; sweep < maxs; ++sweep) {
      if (tid == 0) {
        s_rot = 0;
        s_off = 0;
      }
      __syncthreads();
      for (int r = 0; r < n2 - 1; ++r) {
        for (int k = wave; k < npairs; k += nw) {
          int p, q;
          rr_pair(r, k, n2, p, q);
          if (p >= n || q >= n) continue;
          double a = 0.0, b = 0.0, g = 0.0;
          for (int i = lane; i < m; i += 64) {
            const double x = G[i + p * ldg], y = G[i + q * ldg];
            a += x * x;
            b += y * y;
            g += x * y;
          }
          a = wave_sum(a);
          b = wave_sum(b);
          g = wave_sum(g);
          if (!(fmin(a, b) > dead2)) continue;
          const double rel = fabs(g) / sqrt(a * b);
          if (lane == 0 && rel == rel) atomicMax(&s_off, __float_as_int((float)fmin(rel, 1.0)));
          if (g == 0.0 || !(fabs(g) > tol * sqrt(a * b))) continue;
          double c, s;
          jacobi_rotation(a, b, g, c, s);
          for (int i = lane; i < m; i += 64) {
            const double x = G[i + p * ldg], y = G[i + q * ldg];
            G[i + p * ldg] = c * x - s * y;
            G[i + q * ldg] = s * x + c * y;
          }
          for (int i = lane; i < n; i += 64) {
            const double x = V[i + p * ldv], y = V[i + q * ldv];
            V[i + p * ldv] = c * x - s * y;
            V[i + q * ldv] = s * x + c * y;
          }
          if (lane == 0) s_rot = 1;
        }
        __syncthreads();
      }
      // no rotation, or every relative off-diagonal met in this sweep < 1e-12
      if (!s_rot || __int_as_float(s_off) < 1e-12f) break;
      __syncthreads();
    }
  }
  if (tid == 0 && job.sweeps) *job.sweeps = sweep + 1;
  // the loop ran to the cap without meeting either stopping rule
  if (tid == 0 && job.state) job.state[3] = (n > 1 && sweep >= maxs) ? 1 : 0;
  for (int p = wave; p < n; p += nw) {
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a += G[i + p * ldg] * G[i + p * ldg];
    a = wave_sum(a);
    if (lane == 0) s_sig[p] = sqrt(a);
  }
  __syncthreads();
  for (int p = tid; p < n; p += blockDim.x) {
    const double sp = s_sig[p];
    int rank = 0;
    for (int q = 0; q < n; ++q) {
      const double sq = s_sig[q];
      if (sq > sp || (sq == sp && q < p)) ++rank;
    }
    job.perm[rank] = p;
    job.s[rank] = sp;
  }
  if (tid == 0 && job.sweeps) *job.sweeps = sweep;
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Block one-sided Jacobi SVD.  Columns are grouped in blocks of w; a round
// pairs blocks by the circle method, and each workgroup takes one block pair
// of one job: it loads the 2w columns into LDS, runs one inner Jacobi sweep
// over all their pairs (one wave per pair), accumulates the 2w x 2w rotation
// J, writes the columns back and applies J to the same columns of V.
__global__ __launch_bounds__(256) void bj_init_kernel(const SvdJob* jobs) {
  const SvdJob job = jobs[blockIdx.x];
  for (int idx = threadIdx.x; idx < job.n * job.n; idx += blockDim.x) {
    const int i = idx % job.n, j = idx / job.n;
    job.V[i + (int64_t)j * job.ldv] = (i == j) ? 1.0 : 0.0;
  }
  if (job.fro2) {
    __shared__ double sh[16];
    double f = 0.0;
    for (int64_t idx = threadIdx.x; idx < (int64_t)job.m * job.n; idx += blockDim.x) {
      const double x = job.G[idx % job.m + (idx / job.m) * job.ldg];
      f += x * x;
    }
    f = block_sum(f, sh);
    if (threadIdx.x == 0) *job.fro2 = f;
  }
  if (threadIdx.x == 0) {
    job.state[0] = job.n < 2;
    job.state[1] = 0;
    job.state[2] = 0;
    job.state[3] = 0;
    job.state[5] = 0;
    job.state[6] = 0;
    if (job.sweeps) *job.sweeps = 0;
  }
}

__global__ void bj_sweep_begin_kernel(const SvdJob* jobs, int sweep) {
  const SvdJob job = jobs[blockIdx.x];
  if (threadIdx.x != 0 || job.state[0]) return;
  // done after a sweep without rotations, or one whose largest relative
  // off-diagonal |<g_p, g_q>| / (|g_p| |g_q|) stayed below 1e-12 (the
  // remaining rotations only shuffle rounding between near-degenerate columns)
  if (sweep > 0 && (job.state[1 + ((sweep - 1) & 1)] == 0 ||
                    __int_as_float(job.state[5 + ((sweep - 1) & 1)]) < 1e-12f)) {
    job.state[0] = 1;
    return;
  }
  job.state[1 + (sweep & 1)] = 0;
  job.state[5 + (sweep & 1)] = 0;
  if (job.sweeps) *job.sweeps = sweep + 1;
}

__global__ __launch_bounds__(1024) void bj_round_kernel(const SvdJob* jobs, int round, int sweep, int w) {
  const SvdJob job = jobs[blockIdx.y];
  if (job.state[0]) return;
  const int m = job.m, n = job.n;
  const int nb = (n + w - 1) / w, nb2 = nb + (nb & 1);
  if (round >= nb2 - 1 || (int)blockIdx.x >= nb2 / 2) return;
  int P, Q;
  rr_pair(round, blockIdx.x, nb2, P, Q);
  if (P >= nb || Q >= nb) return;
  extern __shared__ double lds[];
  const int W2 = 2 * w;
  double* J = lds;                 // W2 x W2, J[u + W2 t]
  double* Gs = lds + W2 * W2;      // column t at Gs + t * m
  __shared__ int cols[64];
  __shared__ int s_nc, s_rot, s_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) {
    int nc = 0;
    for (int t = 0; t < w; ++t)
      if (P * w + t < n) cols[nc++] = P * w + t;
    for (int t = 0; t < w; ++t)
      if (Q * w + t < n) cols[nc++] = Q * w + t;
    s_nc = nc;
    s_rot = 0;
    s_off = 0;
  }
  __syncthreads();
  const int nc = s_nc;
  for (int idx = tid; idx < nc * m; idx += blockDim.x) {
    const int t = idx / m, i = idx % m;
    Gs[idx] = job.G[i + (int64_t)cols[t] * job.ldg];
  }
  for (int idx = tid; idx < W2 * W2; idx += blockDim.x) J[idx] = (idx % W2 == idx / W2) ? 1.0 : 0.0;
  __syncthreads();
  const double tol = 1e-15 * sqrt((double)m);
  const double dead2 = job.fro2 ? 1e-28 * *job.fro2 : 0.0;
  const int nc2 = nc + (nc & 1);
  for (int r = 0; r < nc2 - 1; ++r) {
    for (int k = wave; k < nc2 / 2; k += nw) {
      int a, b;
      rr_pair(r, k, nc2, a, b);
      if (a >= nc || b >= nc) continue;
      double* ga = Gs + a * m;
      double* gb = Gs + b * m;
      double x2 = 0.0, y2 = 0.0, xy = 0.0;
      for (int i = lane; i < m; i += 64) {
        const double x = ga[i], y = gb[i];
        x2 += x * x;
        y2 += y * y;
        xy += x * y;
      }
      x2 = wave_sum(x2);
      y2 = wave_sum(y2);
      xy = wave_sum(xy);
      if (!(fmin(x2, y2) > dead2)) continue;
      const double rel = fabs(xy) / sqrt(x2 * y2);
      if (lane == 0 && rel == rel) atomicMax(&s_off, __float_as_int((float)fmin(rel, 1.0)));
      if (xy == 0.0 || !(fabs(xy) > tol * sqrt(x2 * y2))) continue;
      double c, sn;
      jacobi_rotation(x2, y2, xy, c, sn);
      for (int i = lane; i < m; i += 64) {
        const double x = ga[i], y = gb[i];
        ga[i] = c * x - sn * y;
        gb[i] = sn * x + c * y;
      }
      for (int u = lane; u < W2; u += 64) {
        const double x = J[u + W2 * a], y = J[u + W2 * b];
        J[u + W2 * a] = c * x - sn * y;
        J[u + W2 * b] = sn * x + c * y;
      }
      if (lane == 0) s_rot = 1;
    }
    __syncthreads();
  }
  if (tid == 0) atomicMax(&job.state[5 + (sweep & 1)], s_off);
  if (!s_rot) return;
  for (int idx = tid; idx < nc * m; idx += blockDim.x) {
    const int t = idx / m, i = idx % m;
    job.G[i + (int64_t)cols[t] * job.ldg] = Gs[idx];
  }
  // V[:, cols] <- V[:, cols] J, one row per thread
  for (int i = tid; i < n; i += blockDim.x) {
    double row[32];
    for (int u = 0; u < nc; ++u) row[u] = job.V[i + (int64_t)cols[u] * job.ldv];
    for (int t = 0; t < nc; ++t) {
      double acc = 0.0;
      for (int u = 0; u < nc; ++u) acc += row[u] * J[u + W2 * t];
      job.V[i + (int64_t)cols[t] * job.ldv] = acc;
    }
  }
  if (tid == 0) atomicAdd(&job.state[1 + (sweep & 1)], 1);
}

__global__ __launch_bounds__(1024) void bj_finish_kernel(const SvdJob* jobs) {
  const SvdJob job = jobs[blockIdx.x];
  const int m = job.m, n = job.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  __shared__ double s_sig[1024];
  for (int p = wave; p < n; p += nw) {
    double a = 0.0;
    for (int i = lane; i < m; i += 64) a += job.G[i + (int64_t)p * job.ldg] * job.G[i + (int64_t)p * job.ldg];
    a = wave_sum(a);
    if (lane == 0) s_sig[p] = sqrt(a);
  }
  __syncthreads();
  for (int p = tid; p < n; p += blockDim.x) {
    const double sp = s_sig[p];
    int rank = 0;
    for (int q = 0; q < n; ++q) {
      const double sq = s_sig[q];
      if (sq > sp || (sq == sp && q < p)) ++rank;
    }
    job.perm[rank] = p;
    job.s[rank] = sp;
  }
}

// Left-looking upper Cholesky; at step j every later column i needs the dot
// of columns j and i above row j: one wave per column, lanes over rows.
// Upper Cholesky G = R^T R, blocked right-looking with 16-column blocks (one
// workgroup per job, the working matrix in R, L2-resident):
//   (a) wave 0 factors the diagonal block in registers (lane l holds column
//       l of the block; the pivot test d > rel_tol * G_jj of the original
//       diagonal is taken on the updated diagonal, as column by column),
//   (b) every column j past the block solves R_kk^T x = A[k-block, j],
//   (c) the trailing upper triangle takes the rank-16 update A -= P^T P in
//       4 x 4 tiles (P = the block's rows of R).
// Three barriers per block instead of two per column.
constexpr int CB = 16;

__global__ __launch_bounds__(1024) void cholesky_kernel(const CholJob* jobs, double rel_tol) {
  const CholJob job = jobs[blockIdx.x];
  if (gated_out(job.gate, job.gate_zero)) return;
  const int n = job.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* R = job.R;
  const int64_t ldr = job.ldr;
  __shared__ double diag0[1024];
  __shared__ double Dk[CB][CB + 1];   // Dk[t][l] = R[k0 + t, k0 + l] of the factored block
  __shared__ int s_fail;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    const double g = job.G[i + (int64_t)j * job.ldg];
    if (i == j) diag0[i] = g;
    if (i <= j) R[i + (int64_t)j * ldr] = g;
  }
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    if (i > j) R[i + (int64_t)j * ldr] = 0.0;
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += CB) {
    const int kw = n - k0 < CB ? n - k0 : CB;
    const int k1 = k0 + kw;
    // (a) diagonal block in wave 0, in LDS (one wave's LDS operations execute
    // in order; the fences keep the compiler from reordering them)
    if (wave == 0) {
      for (int idx = lane; idx < CB * CB; idx += 64) {
        const int t = idx % CB, l = idx / CB;
        Dk[t][l] = (t <= l && l < kw) ? R[k0 + t + (int64_t)(k0 + l) * ldr] : 0.0;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      for (int j = 0; j < kw; ++j) {
        if (lane == 0) {
          double part = 0.0;
          for (int t = 0; t < j; ++t) part += Dk[t][j] * Dk[t][j];
          const double d = Dk[j][j] - part;
          const double g0 = diag0[k0 + j];
          if (!(d > rel_tol * g0) || !(g0 > 0.0))
            s_fail = k0 + j + 1;
          else
            Dk[j][j] = sqrt(d);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (s_fail) break;
        if (lane > j && lane < kw) {
          double part = 0.0;
          for (int t = 0; t < j; ++t) part += Dk[t][j] * Dk[t][lane];
          Dk[j][lane] = (Dk[j][lane] - part) / Dk[j][j];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      }
      if (!s_fail)
        for (int idx = lane; idx < CB * CB; idx += 64) {
          const int t = idx % CB, l = idx / CB;
          if (t <= l && l < kw) R[k0 + t + (int64_t)(k0 + l) * ldr] = Dk[t][l];
        }
    }
    __syncthreads();
    if (s_fail) {
      if (tid == 0) {
        *job.info = s_fail;
        if (job.fail) *job.fail = 1;
      }
      return;
    }
    // (b) panel: R[k-block, j] = R_kk^-T A[k-block, j] for j >= k1
    for (int j = k1 + tid; j < n; j += blockDim.x) {
      double* c = R + k0 + (int64_t)j * ldr;
      double x[CB];
      // an opaque zero keeps the block's reads inside this loop (hoisted out
      // of it, the 136 values would not fit the registers)
      int opq = 0;
      asm volatile("" : "+v"(opq));
      const double* D = &Dk[0][0] + opq;
#pragma unroll
      for (int t = 0; t < CB; ++t) {
        if (t < kw) {
          double a = c[t];
#pragma unroll
          for (int u = 0; u < t; ++u) a -= D[u * (CB + 1) + t] * x[u];
          x[t] = a / D[t * (CB + 1) + t];
        }
      }
#pragma unroll
      for (int t = 0; t < CB; ++t)
        if (t < kw) c[t] = x[t];
    }
    __syncthreads();
    // (c) trailing update of the upper triangle, 4 x 4 tiles (ti <= tj)
    const int m = n - k1;
    if (m > 0) {
      const int T = (m + 3) / 4;
      const int ntiles = T * (T + 1) / 2;
      for (int q = tid; q < ntiles; q += blockDim.x) {
        // tile index -> (ti, tj) with ti <= tj, column by column
        int tj = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while ((tj + 1) * (tj + 2) / 2 <= q) ++tj;
        while (tj * (tj + 1) / 2 > q) --tj;
        const int ti = q - tj * (tj + 1) / 2;
        const int i0 = k1 + 4 * ti, j0 = k1 + 4 * tj;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 2
        for (int t = 0; t < kw; ++t) {
          {
            double pi[4], pj[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              pi[a] = i0 + a < n ? R[k0 + t + (int64_t)(i0 + a) * ldr] : 0.0;
              pj[a] = j0 + a < n ? R[k0 + t + (int64_t)(j0 + a) * ldr] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) acc[a][b] += pi[a] * pj[b];
          }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = j0 + b;
          if (j >= n) continue;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int i = i0 + a;
            if (i <= j) R[i + (int64_t)j * ldr] -= acc[a][b];
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) *job.info = 0;
}

// Diagonal-pivoted Cholesky (rank-revealing CholeskyQR first pass): at each
// step the column with the largest remaining pivot is chosen; stop when it
// falls to tau times the largest diagonal entry.  One wave per column for the
// row update, lanes over the previous rows.
__global__ __launch_bounds__(1024) void piv_cholesky_kernel(const PivCholJob* jobs) {
  const PivCholJob job = jobs[blockIdx.x];
  const int n = job.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double* R = job.R;
  const int ldr = job.ldr;
  __shared__ double d[1024];
  __shared__ int used[1024];
  __shared__ double wbest[16];
  __shared__ int widx[16];
  __shared__ int s_p, s_stop;
  __shared__ double s_rjj, s_dmax;
  for (int i = tid; i < n; i += blockDim.x) {
    d[i] = job.G[i + (int64_t)i * job.ldg];
    used[i] = 0;
  }
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, d[i]);
    s_dmax = m;
  }
  __syncthreads();
  int j = 0;
  for (; j < n; ++j) {
    // argmax of the remaining pivots (ties -> smaller index)
    double best = -1.0;
    int bi = n;
    for (int i = tid; i < n; i += blockDim.x)
      if (!used[i] && (d[i] > best || (d[i] == best && i < bi))) {
        best = d[i];
        bi = i;
      }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      wbest[wave] = best;
      widx[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = -1.0;
      int p = n;
      for (int w = 0; w < nw; ++w)
        if (wbest[w] > b || (wbest[w] == b && widx[w] < p)) {
          b = wbest[w];
          p = widx[w];
        }
      s_stop = !(p < n && b > job.tau * s_dmax && b > 0.0);
      s_p = p;
      s_rjj = s_stop ? 0.0 : sqrt(b);
      if (!s_stop) job.sel[j] = p;
    }
    __syncthreads();
    if (s_stop) break;
    const int p = s_p;
    const double rjj = s_rjj;
    const double* Rp = R + (int64_t)p * ldr;
    for (int c = wave; c < n; c += nw) {
      double* Rc = R + (int64_t)c * ldr;
      if (c == p) {
        if (lane == 0) Rc[j] = rjj;
      } else if (used[c]) {
        if (lane == 0) Rc[j] = 0.0;
      } else {
        double part = 0.0;
        for (int k = lane; k < j; k += 64) part += Rp[k] * Rc[k];
        part = wave_sum(part);
        if (lane == 0) {
          const double v = (job.G[p + (int64_t)c * job.ldg] - part) / rjj;
          Rc[j] = v;
          d[c] -= v * v;
        }
      }
    }
    __syncthreads();
    if (tid == 0) used[p] = 1;
    __syncthreads();
  }
  if (tid == 0) *job.rank = j;
}

__global__ void sel_kernel(const SelJob* jobs) {
  const SelJob job = jobs[blockIdx.x];
  const int r = job.r, n = job.n;
  if (job.mode == 0) {
    for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
      const int i = idx % r, k = idx / r;
      job.out[i + (int64_t)k * job.ldout] = job.in[i + (int64_t)job.sel[k] * job.ldin];
    }
  } else {
    for (int idx = threadIdx.x; idx < n * r; idx += blockDim.x) {
      const int row = idx % n, c = idx / n;
      job.out[row + (int64_t)c * job.ldout] = 0.0;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
      const int k = idx % r, c = idx / r;
      job.out[job.sel[k] + (int64_t)c * job.ldout] = job.in[k + (int64_t)c * job.ldin];
    }
  }
}

// X = R^-1 of an upper-triangular n x n R (n <= 1024).  The columns of X are
// independent, so each workgroup takes one job's block of 16 columns
// [c0, c1) and forms its rows from the bottom in 16-row blocks:
// X[I, cols] = R_II^-1 (E[I, cols] - sum_{k >= r1} R[I, k] X[k, cols]).  The
// column block lives in LDS (rows below c1 are zero).  The block row of R is
// staged through LDS in chunks of 128 columns, loaded by all threads with 16
// consecutive rows of one column (128 bytes) per k, so the sums read LDS; the
// 16 x 16 inverse of R_II comes from back substitution by 16 threads on the
// staged diagonal block.
constexpr int TB = 16, TBP = TB + 1, TKC = 128, TKP = TKC + 1;

__global__ __launch_bounds__(256) void tri_inverse_kernel(const TriInvJob* jobs) {
  const TriInvJob job = jobs[blockIdx.y];
  if (gated_out(job.gate, job.gate_zero)) return;
  const int n = job.n;
  const int c0 = blockIdx.x * TB;
  if (c0 >= n) return;
  const int c1 = min(n, c0 + TB), cw = c1 - c0;
  const double* R = job.R;
  const int64_t ldr = job.ldr;
  extern __shared__ double tlds[];
  double* Rs = tlds;                       // Rs[t * TKP + kk] = R[r0 + t, k0 + kk]
  double* RI = Rs + TB * TKP;              // RI[t * TBP + q] = (R_II^-1)[t, q]
  double* E = RI + TB * TBP;               // E[t * TBP + u]: right-hand sides of the block row
  double* Xs = E + TB * TBP;               // Xs[k * TB + u] = X[k, c0 + u], k < c1
  const int tid = threadIdx.x, t = tid & 15, u = tid >> 4;
  auto stage_rows = [&](int r0, int kw, int k0, int kc) {
    for (int idx = tid; idx < TB * kc; idx += blockDim.x) {
      const int tt = idx & 15, kk = idx >> 4;
      Rs[tt * TKP + kk] = tt < kw ? R[r0 + tt + (int64_t)(k0 + kk) * ldr] : 0.0;
    }
  };
  for (int I = (c1 - 1) / TB; I >= 0; --I) {
    const int r0 = I * TB, kw = min(TB, n - r0), r1 = r0 + kw;
    // diagonal block
    stage_rows(r0, kw, r0, kw);
    __syncthreads();
    if (tid < kw) {
      // column v of R_II^-1: back substitution on R_II y = e_v
      const int v = tid;
      double y[TB];
#pragma unroll
      for (int a = TB - 1; a >= 0; --a) {
        double val = 0.0;
        if (a <= v) {
          double acc = (a == v) ? 1.0 : 0.0;
#pragma unroll
          for (int q = a + 1; q < TB; ++q)
            if (q <= v) acc -= Rs[a * TKP + q] * y[q];
          val = acc / Rs[a * TKP + a];
        }
        y[a] = val;
      }
#pragma unroll
      for (int a = 0; a < TB; ++a)
        if (a < kw) RI[a * TBP + v] = y[a];
    }
    double sacc = 0.0;
    for (int k0 = r1; k0 < c1; k0 += TKC) {
      const int kc = min(TKC, c1 - k0);
      __syncthreads();   // previous readers of Rs are done
      stage_rows(r0, kw, k0, kc);
      __syncthreads();
      if (t < kw && u < cw)
        for (int kk = 0; kk < kc; ++kk) sacc += Rs[t * TKP + kk] * Xs[(k0 + kk) * TB + u];
    }
    E[t * TBP + u] = ((r0 + t == c0 + u) ? 1.0 : 0.0) - sacc;
    __syncthreads();
    if (t < kw && u < cw) {
      double val = 0.0;
      for (int q = t; q < kw; ++q) val += RI[t * TBP + q] * E[q * TBP + u];
      Xs[(r0 + t) * TB + u] = val;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * cw; idx += blockDim.x) {
    const int i = idx % n, c = idx / n;
    job.Ri[i + (int64_t)(c0 + c) * job.ldri] = i < c1 ? Xs[i * TB + c] : 0.0;
  }
}

constexpr int SG = 64;   // output tile side
constexpr int SGK = 16;  // depth chunk

// Batched C = alpha op(A) op(B) + beta C on the float64 MFMA (16x16x4): a
// 64 x 64 tile of one job per workgroup, four waves in a 2 x 2 grid with 2 x 2
// MFMA blocks each, depth-16 chunks of op(A) and op(B) staged in LDS.  Sizes
// may come from device memory.
__global__ __launch_bounds__(256) void small_gemm_kernel(const SmallGemmJob* jobs) {
  const SmallGemmJob job = jobs[blockIdx.y];
  if (gated_out(job.gate, job.gate_zero)) return;
  const int M = job.M_dev ? *job.M_dev : job.M;
  const int N = job.N_dev ? *job.N_dev : job.N;
  const int K = job.K_dev ? *job.K_dev : job.K;
  const int tiles_m = (M + SG - 1) / SG, tiles_n = (N + SG - 1) / SG;
  if ((int)blockIdx.x >= tiles_m * tiles_n) return;
  const int i0 = (blockIdx.x % tiles_m) * SG, j0 = (blockIdx.x / tiles_m) * SG;
  __shared__ double As[SGK][SG + 1];  // As[k][i] = op(A)(i0 + i, k0 + k)
  __shared__ double Bs[SGK][SG + 1];  // Bs[k][j] = op(B)(k0 + k, j0 + j)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 4; ++e) acc[a][b][e] = 0.0;
  for (int k0 = 0; k0 < K; k0 += SGK) {
#pragma unroll
    for (int q = 0; q < SG * SGK / 256; ++q) {
      const int e = tid + 256 * q;
      {
        // contiguous axis of the stored A: i when not transposed, k otherwise
        const int i = job.tA ? e / SGK : e % SG, k = job.tA ? e % SGK : e / SG;
        const int gi = i0 + i, gk = k0 + k;
        double v = 0.0;
        if (gi < M && gk < K) v = job.tA ? job.A[gk + (int64_t)gi * job.lda] : job.A[gi + (int64_t)gk * job.lda];
        As[k][i] = v;
      }
      {
        const int j = job.tB ? e % SG : e / SGK, k = job.tB ? e / SG : e % SGK;
        const int gj = j0 + j, gk = k0 + k;
        double v = 0.0;
        if (gj < N && gk < K) v = job.tB ? job.B[gj + (int64_t)gk * job.ldb] : job.B[gk + (int64_t)gj * job.ldb];
        Bs[k][j] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SGK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double a[2], b[2];
      for (int x = 0; x < 2; ++x) a[x] = As[kr][wr * 32 + x * 16 + (lane & 15)];
      for (int y = 0; y < 2; ++y) b[y] = Bs[kr][wc * 32 + y * 16 + (lane & 15)];
      // operands swapped: the result blocks are C^T, so lanes run along C's rows
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[y], a[x], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int e = 0; e < 4; ++e) {
        const int gi = i0 + wr * 32 + x * 16 + (lane & 15);
        const int gj = j0 + wc * 32 + y * 16 + (lane >> 4) + 4 * e;
        if (gi >= M || gj >= N) continue;
        double* c = job.C + gi + (int64_t)gj * job.ldc;
        *c = job.alpha * acc[x][y][e] + (job.beta != 0.0 ? job.beta * *c : 0.0);
      }
}

}  // namespace

int launch_pseudo_sqrt(const PsqJob* jobs, int njobs, double eps_pinv, hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(pseudo_sqrt_kernel, dim3(njobs), dim3(256), 0, s, jobs, eps_pinv);
  HPT_LAUNCH_CHECK("pseudo_sqrt_kernel");
  return 0;
}

template <typename T>
int launch_householder(const QrJob<T>* jobs, int njobs, hipStream_t s, int mmax) {
  if (njobs <= 0) return 0;
  if (sizeof(T) == 8 && mmax >= 1 && mmax <= HBM) {
    hipLaunchKernelGGL(householder_blocked_kernel, dim3(njobs), dim3(1024), HB_LDS, s,
                       (const QrJob<double>*)jobs);
    HPT_LAUNCH_CHECK("householder_blocked_kernel");
    return 0;
  }
  hipLaunchKernelGGL(householder_kernel<T>, dim3(njobs), dim3(1024), 0, s, jobs);
  HPT_LAUNCH_CHECK("householder_kernel");
  return 0;
}
template int launch_householder<double>(const QrJob<double>*, int, hipStream_t, int);
template int launch_householder<float>(const QrJob<float>*, int, hipStream_t, int);

int launch_jacobi_svd(const SvdJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(njobs), dim3(1024), 0, s, jobs);
  HPT_LAUNCH_CHECK("jacobi_svd_kernel");
  return 0;
}

// after the last sweep: a job that is not done and whose last sweep still
// rotated above the 1e-12 relative off-diagonal has not converged
__global__ void bj_check_kernel(const SvdJob* jobs, int last) {
  const SvdJob job = jobs[blockIdx.x];
  if (threadIdx.x != 0) return;
  const bool conv = job.state[0] || job.state[1 + (last & 1)] == 0 ||
                    __int_as_float(job.state[5 + (last & 1)]) < 1e-12f;
  job.state[3] = conv ? 0 : 1;
}

// done = 1 when every job has converged
__global__ __launch_bounds__(256) void bj_all_done_kernel(const SvdJob* jobs, int njobs, int* done) {
  __shared__ int s_all;
  if (threadIdx.x == 0) s_all = 1;
  __syncthreads();
  for (int j = threadIdx.x; j < njobs; j += blockDim.x)
    if (!jobs[j].state[0]) s_all = 0;
  __syncthreads();
  if (threadIdx.x == 0) *done = s_all;
}

int launch_block_jacobi_svd(const SvdJob* jobs, const SvdJob* host, int njobs, hipStream_t s, int* done_dev,
                            volatile int* done_host, int max_sweeps) {
  if (njobs <= 0) return 0;
  int mmax = 1, nmax = 1;
  for (int j = 0; j < njobs; ++j) {
    mmax = std::max(mmax, host[j].m);
    nmax = std::max(nmax, host[j].n);
  }
  // block width: 16 columns per block when a pair of blocks fits in the
  // workgroup's LDS (leaving room for the kernel's static LDS)
  static int max_lds = 0;
  if (!max_lds) {
    int dev = 0;
    HPT_HIP(hipGetDevice(&dev));
    HPT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  }
  const size_t budget = (size_t)max_lds > 2048 ? (size_t)max_lds - 2048 : 0;
  int w = 16;
  while (w > 2 && (size_t)(2 * w * mmax + 4 * w * w) * 8 > budget) w /= 2;
  // one wave per column pair of a sub-round (w pairs over the 2w columns)
  const int bj_threads = 64 * std::max(4, std::min(16, w));
  const size_t lds = (size_t)(2 * w * mmax + 4 * w * w) * 8;
  if (lds > budget || njobs > 65535) return -1;
  const int nb = (nmax + w - 1) / w, nb2 = nb + (nb & 1);
  hipLaunchKernelGGL(bj_init_kernel, dim3(njobs), dim3(256), 0, s, jobs);
  HPT_LAUNCH_CHECK("bj_init_kernel");
  if (max_sweeps < 1) max_sweeps = 20;
  int last = -1;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    last = sweep;
    hipLaunchKernelGGL(bj_sweep_begin_kernel, dim3(njobs), dim3(64), 0, s, jobs, sweep);
    HPT_LAUNCH_CHECK("bj_sweep_begin_kernel");
    for (int r = 0; r < nb2 - 1; ++r) {
      hipLaunchKernelGGL(bj_round_kernel, dim3(std::max(1, nb2 / 2), njobs), dim3(bj_threads), lds, s, jobs, r,
                         sweep, w);
      HPT_LAUNCH_CHECK("bj_round_kernel");
    }
    // from the fourth sweep on, stop launching once every job has converged
    // (the check after sweep k sees the rotations of sweep k - 1)
    if (done_dev && done_host && sweep >= 3 && sweep + 1 < max_sweeps) {
      hipLaunchKernelGGL(bj_sweep_begin_kernel, dim3(njobs), dim3(64), 0, s, jobs, sweep + 1);
      HPT_LAUNCH_CHECK("bj_sweep_begin_kernel");
      hipLaunchKernelGGL(bj_all_done_kernel, dim3(1), dim3(256), 0, s, jobs, njobs, done_dev);
      HPT_LAUNCH_CHECK("bj_all_done_kernel");
      HPT_HIP(hipMemcpyAsync((void*)done_host, done_dev, sizeof(int), hipMemcpyDeviceToHost, s));
      HPT_HIP(hipStreamSynchronize(s));
      if (*done_host) break;
      ++sweep;   // that sweep has begun: run its rounds next
      last = sweep;
      for (int r = 0; r < nb2 - 1; ++r) {
        hipLaunchKernelGGL(bj_round_kernel, dim3(std::max(1, nb2 / 2), njobs), dim3(bj_threads), lds, s, jobs, r,
                           sweep, w);
        HPT_LAUNCH_CHECK("bj_round_kernel");
      }
    }
  }
  if (last >= 0) {
    hipLaunchKernelGGL(bj_check_kernel, dim3(njobs), dim3(64), 0, s, jobs, last);
    HPT_LAUNCH_CHECK("bj_check_kernel");
  }
  hipLaunchKernelGGL(bj_finish_kernel, dim3(njobs), dim3(1024), 0, s, jobs);
  HPT_LAUNCH_CHECK("bj_finish_kernel");
  return 0;
}

int launch_cholesky(const CholJob* jobs, int njobs, double rel_tol, hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(cholesky_kernel, dim3(njobs), dim3(1024), 0, s, jobs, rel_tol);
  HPT_LAUNCH_CHECK("cholesky_kernel");
  return 0;
}

int launch_tri_inverse(const TriInvJob* jobs, int njobs, hipStream_t s, int nmax) {
  if (njobs <= 0) return 0;
  if (nmax < 1 || nmax > 1024 || njobs > 65535) return -1;
  const size_t lds = (size_t)(TB * TKP + 2 * TB * TBP + TB * nmax) * sizeof(double);
  static int max_lds = 0;
  if (!max_lds) {
    int dev = 0;
    HPT_HIP(hipGetDevice(&dev));
    HPT_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  }
  if (lds > (size_t)max_lds) return -1;
  hipLaunchKernelGGL(tri_inverse_kernel, dim3((nmax + TB - 1) / TB, njobs), dim3(256), lds, s, jobs);
  HPT_LAUNCH_CHECK("tri_inverse_kernel");
  return 0;
}

int launch_piv_cholesky(const PivCholJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(piv_cholesky_kernel, dim3(njobs), dim3(1024), 0, s, jobs);
  HPT_LAUNCH_CHECK("piv_cholesky_kernel");
  return 0;
}

int launch_sel(const SelJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(sel_kernel, dim3(njobs), dim3(256), 0, s, jobs);
  HPT_LAUNCH_CHECK("sel_kernel");
  return 0;
}

int launch_small_gemm(const SmallGemmJob* jobs, const SmallGemmJob* host, int njobs, hipStream_t s) {
  if (njobs <= 0) return 0;
  int64_t tiles = 1;
  for (int j = 0; j < njobs; ++j)
    tiles = std::max<int64_t>(tiles, ceil_div(host[j].M, SG) * ceil_div(host[j].N, SG));
  if (tiles > 0x7fffffff || njobs > 65535) return -1;
  hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)tiles, njobs), dim3(256), 0, s, jobs);
  HPT_LAUNCH_CHECK("small_gemm_kernel");
  return 0;
}

}  // namespace hpt
