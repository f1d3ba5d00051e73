// R-core of the two-site gate (k_rcore.hip): bond matrix over the cut, gate
// on the Pauli pair, SVD, truncation, Vidal lambda, reconstruction factors.
#pragma once
#include "common.h"

namespace hpt {

// Per-bond device record shared by the R-core kernels of one colour.
struct BondCore {
  // inputs (set by the host)
  int chi_cut;            // current bond dimension
  int k[2];               // rows of R_i = min(m_i, 4 chi_cut)
  int q[2];               // rows of T_i = min(4 k_i, 4 chi_cut)
  int chol[2];            // 1: S_i = X_i and W_i = R_i^{-1} M'_i; 0: S_i = Q_i, W_i = M'_i
  int bqr[2];             // QR of B_i: 0 CholeskyQR2 (set to 1 when it fails), 1 Householder
  int chi_max;
  double eps_cut;
  const double* R[2];     // k_i x 4 chi_cut, ld ldR
  const double* Rinv[2];  // 4 chi_cut x 4 chi_cut (chol path)
  int ldR;
  double* B[2];           // 4 k_i x 4 chi_cut, becomes Q~_i (explicit) ; ld 4 k_i
  double* Tm[2];          // q_i x 4 chi_cut, R-factor of B_i ; ld ldT
  int ldT;
  double* tau;            // scratch for the B QRs, 2 * 4 chi_max
  double* G;              // core, max(q) x min(q), ld ldG
  int ldG;
  double* V;              // min(q) x min(q), ld ldG
  double* s;              // min(q)
  int* perm;              // min(q)
  double* Uc;             // q_0 x chi_new  (left vectors * sqrt(s)), ld ldG
  double* Vc;             // q_1 x chi_new
  double* Mf[2];          // 4 k_i x chi_new  = Q~_i * (Uc | Vc), ld 4 k_i
  double* Mp[2];          // k_i x 4 chi_new  rearranged Mf
  double* W[2];           // n_S_i x 4 chi_new, ld = n_S_i (= 4 chi_cut if chol else k_i)
  const double* z;        // sign projections of S_0: n_S_0 x 4
  double* msg[2];         // gauge message slots of this bond (chi_new x chi_new)
  double* lam;            // lambda out (chi_max)
  double* qs[2][8];       // float64 scratch of the CholeskyQR2 of B_i (4 chi_max x 4 chi_max each)
  double* pq[4];          // preconditioned core SVD: R, H = R^T, copy of Q, V of H (ld ldG each)
  // outputs
  int chi_new;
  int n4;                 // 4 * chi_new
  int status;             // 0 ok, 1 zero / non-finite spectrum
  int flags;
  int sweeps;
  double gate_err;
  double s0;
};

// gate factors of the XX coupling in the Pauli basis: G2 = sum_r F_r (x) H_r
struct GateFactors {
  double F[4][16];        // F_r[e, d] at [r][e + 4 d]
  double H[4][16];
};

int launch_rcore_build_B(BondCore* bonds, int nb, const GateFactors& g, hipStream_t s);
// Gram B_i^T B_i of the gated blocks (bqr[i] == 0) from R_i^T R_i in qs[i][5]
// into qs[i][0]
int launch_rcore_kron_gram(BondCore* bonds, int nb, const GateFactors& g, hipStream_t s);
// Preconditioned SVD of the core G (m x n, m >= n, ld ldG), after its
// Householder QR G = Q R (Q explicit in G, R in pq[0]): prep sets pq[1] = R^T
// and pq[2] = Q; the one-sided Jacobi then runs on R^T (pq[1], right vectors
// into pq[3]); finish rescales so that G = (Q V_H) diag(s) U_H^T reads as the
// plain SVD's output: pq[0] = V_H diag(sigma) (then G = pq[2] pq[0] by a GEMM)
// and V = H_out diag(1 / sigma).
int launch_rcore_precond_prep(BondCore* bonds, int nb, hipStream_t s);
int launch_rcore_precond_finish(BondCore* bonds, int nb, hipStream_t s);
int launch_rcore_select(BondCore* bonds, int nb, hipStream_t s);
int launch_rcore_rearrange(BondCore* bonds, int nb, hipStream_t s);
int launch_rcore_signs(BondCore* bonds, int nb, hipStream_t s);

}  // namespace hpt
