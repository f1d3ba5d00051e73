// Small dense float64 linear algebra on the device, one workgroup per
// problem, batched through arrays of job descriptors in device memory.
#pragma once
#include "common.h"

namespace hpt {

// sqrt(M) and its pseudo-inverse for a symmetric PSD chi x chi message.
struct PsqJob {
  const double* M;     // input, n x n column-major, leading dim n
  double* S;           // out: sqrt(M)
  double* Sinv;        // out: pseudo-inverse of sqrt(M)
  float* S32;          // optional float copies (may be null)
  float* Sinv32;
  double* work;        // 2 n^2 scratch
  int n;
  int* ncut;           // out: eigenvalues dropped
};

// Householder QR of a column-major m x n block in place (storage T,
// arithmetic float64).  R (min(m,n) x n, diag >= 0) goes to R; if form_q the
// explicit m x min(m,n) Q with matching signs overwrites A.  Runs only when
// (gate == nullptr || *gate != 0).
template <typename T>
struct QrJob {
  T* A; int64_t lda; int m, n;
  double* R; int ldr;
  double* tau;         // n scratch
  int form_q;
  const int* gate;
  int gate_zero;       // 1: run only when *gate == 0
};

// One-sided Jacobi SVD of an m x n (m >= n) float64 block in place.
// On exit column perm[i] of G holds sigma_i u_i, V (n x n) the right vectors,
// s[i] the singular values in descending order.
struct SvdJob {
  double* G; int ldg; int m, n;
  double* V; int ldv;
  double* s; int* perm;
  int* sweeps;
  int* state;          // 7 ints of scratch: done, 2 rotation counters (block variant), not converged
                       // within the sweep cap (both variants), -, 2 largest relative off-diagonals
                       // as float bits (block variant)
  double* fro2;        // block variant: 1 double of scratch (squared Frobenius norm); may be null
  int max_sweeps;      // one-sided variant: sweep cap (0: 60)
};
// Columns whose norm falls below 1e-14 of the Frobenius norm of G hold only
// rounding noise: pairs involving them are not rotated (otherwise the noise
// columns keep exchanging rounding errors with the large ones and the
// sweeps never settle).  Their singular values are reported as computed.

// Upper Cholesky G = R^T R of an n x n SPD block (G read, R written, may alias).
// *info = 0 on success, j+1 if pivot j fails the relative test.
struct CholJob {
  const double* G; int ldg; int n;
  double* R; int ldr;
  int* info;
  const int* gate;     // skip when *gate == 0 (null = always run)
  int gate_zero;       // 1: run only when *gate == 0 instead
  int* fail;           // optional: set to 1 when the factorisation fails
};

// Cholesky with diagonal pivoting of an n x n PSD Gram matrix, stopped when
// the largest remaining pivot is <= tau * max diag(G).  Row j of R (original
// column order) is written for j < rank; sel[j] is the column chosen at step
// j, so R[:, sel] is upper triangular.  *rank receives the number of steps.
struct PivCholJob {
  const double* G; int ldg; int n;
  double* R; int ldr;
  int* sel;
  int* rank;
  double tau;
};

// Rsel[i, k] = R[i, sel[k]] (gather, r x r) or W[sel[k], c] = Rs[k, c] with
// the other rows of W zero (scatter, n x r).
struct SelJob {
  int mode;            // 0 gather, 1 scatter
  const double* in; int ldin;
  double* out; int ldout;
  const int* sel; int r, n;
};

// Inverse of an upper-triangular n x n matrix.
struct TriInvJob {
  const double* R; int ldr; int n;
  double* Ri; int ldri;
  const int* gate;
  int gate_zero;       // 1: run only when *gate == 0
};

// Small batched float64 GEMM: C = alpha op(A) op(B) + beta C; sizes may be
// read from device memory (M_dev etc. override when non-null; the host
// fields M, N then hold upper bounds used to size the launch).
struct SmallGemmJob {
  int M, N, K;
  const int* M_dev; const int* N_dev; const int* K_dev;
  const double* A; int lda; int tA;
  const double* B; int ldb; int tB;
  double* C; int ldc;
  double alpha, beta;
  const int* gate;     // skip when *gate == 0 (null = always run)
  int gate_zero;       // 1: run only when *gate == 0 instead
};

int launch_pseudo_sqrt(const PsqJob* jobs, int njobs, double eps_pinv, hipStream_t s);
template <typename T>
// mmax: largest m of the jobs when known on the host (float64 blocks of up to
// 512 rows take the blocked kernel); 0 for the unblocked kernel
int launch_householder(const QrJob<T>* jobs, int njobs, hipStream_t s, int mmax = 0);
int launch_jacobi_svd(const SvdJob* jobs, int njobs, hipStream_t s);
// Block one-sided Jacobi: every launch of a round pairs column blocks of all
// jobs, one workgroup per block pair with the block columns in LDS.  Needs
// SvdJob::state; host holds the host copies of the jobs (sizes).
// With done_dev (device int) and done_host (pinned host int), the host checks
// convergence once per sweep from the fourth sweep on (one stream sync each)
// and stops launching when every job has converged.
int launch_block_jacobi_svd(const SvdJob* jobs, const SvdJob* host, int njobs, hipStream_t s, int* done_dev,
                            volatile int* done_host, int max_sweeps = 20);
int launch_cholesky(const CholJob* jobs, int njobs, double rel_tol, hipStream_t s);
// nmax: largest n of the jobs (<= 1024; sizes the LDS staging)
int launch_tri_inverse(const TriInvJob* jobs, int njobs, hipStream_t s, int nmax);
int launch_piv_cholesky(const PivCholJob* jobs, int njobs, hipStream_t s);
int launch_sel(const SelJob* jobs, int njobs, hipStream_t s);
int launch_small_gemm(const SmallGemmJob* jobs, const SmallGemmJob* host, int njobs, hipStream_t s);

}  // namespace hpt
