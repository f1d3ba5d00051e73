// Elementwise, reduction and BP kernels of libhpt (k_misc.hip).
#pragma once
#include "common.h"

namespace hpt {

// ---- field half-step (Sec. "Trotter Decomposition", Eq. trotter): rotate the X, Y Pauli slices of one site
template <typename T>
int launch_field(T* psi, int64_t slice, double gxx, double gxy, double gyx, double gyy,
                 hipStream_t s);

// ---- conversions / fills
int launch_d2f(const double* in, float* out, int64_t n, hipStream_t s);
int launch_fill_identity(double* M, int n, double scale, hipStream_t s);
int launch_fill_value(double* v, int64_t n, double value, hipStream_t s);
template <typename T>
int launch_fill_t(T* v, int64_t n, double value, hipStream_t s);
template <typename T>
int launch_scale_columns(T* A, int64_t lda, int64_t m, int ncols, const double* colscale,
                         hipStream_t s);

// ---- gauge BP: normalise + damp one batch of directed matrix messages.
// For message i: sym = (Mh + Mh^T)/2 normalised (Frobenius), Mn = normalise(
// (1-alpha) Mo + alpha sym); delta[i] = max |Mn - Mo|; Mo <- Mn.
struct GaugeNormJob {
  double* Mo;          // n x n, in/out
  const double* Mh;    // n x n
  int n;
};
int launch_gauge_norm(const GaugeNormJob* jobs, int njobs, double alpha, double* delta,
                      hipStream_t s);

// <A, B>_F of two n-element vectors; writes the value
struct DotJob {
  const double* a;
  const double* b;
  int64_t n;
  double* out;
};
int launch_dots(const DotJob* jobs, int njobs, hipStream_t s);

// log-space product: res[0] = sum_i sgn_i log|x_i| (sgn = +1 for numerators,
// -1 for denominators), res[1] = product of signs, res[2] = 1 if any x_i == 0
// among numerators, res[3] = 1 if any x_i == 0 among denominators,
// res[4] = max delta over n_delta entries of delta (if delta != null).
// Sweep control of the measurement BP (ctl non-null, ctl[0] = stop flag,
// ctl[1] = sweeps taken): the kernel does nothing once ctl[0] is set, else
// counts the sweep in ctl[1] and sets ctl[0] when res[4] < tol or res[4] is
// not finite.  The measurement-sweep launchers below take ctl as `stop` and
// return at once when it is set, so sweeps queued past convergence are no-ops.
int launch_log_product(const double* x, int n_num, int n_den, const double* delta, int n_delta,
                       double* res, hipStream_t s, double tol = 0.0, double* ctl = nullptr);

// ---- measurement BP (Sec. "Correlation Function via Belief Propagation"): contraction of a pinned slice with vectors
// on every leg except one.  out[a] = sum_{i,o} T[i + I*(a + nk*o)] x[i] y[o]
// with x, y Kronecker products of the incoming messages of the legs before
// and after the output leg.
struct MeasJob {
  const void* T;       // pinned slice (storage type)
  int64_t I, nk, O;
  int nx, ny;          // number of legs folded into x and y (each <= 3)
  const double* xm[3]; int xd[3];   // message pointers and dims, first leg fastest
  const double* ym[3]; int yd[3];
  double* x;           // scratch, I
  double* y;           // scratch, O
  double* S;           // scratch, I * nk (used when O > 1)
  double* out;         // nk
  // filled by meas_plan: block ranges of each stage and partial offsets
  int64_t bk0, bn0, bt0, br0;
  int64_t pn_off, pt_off;
};
// meas_plan fills the block ranges and partial offsets of the host jobs and
// returns the partial-buffer doubles they need; the caller then copies the
// jobs to the device and calls meas_launch.
int64_t meas_plan(MeasJob* jobs_host, int njobs, int64_t totals[4]);
int meas_launch(const MeasJob* jobs_dev, int njobs, const int64_t totals[4], int is_double,
                double* part, hipStream_t s, const double* stop = nullptr);

// One pass over a pinned slice T (rows x nL, column-major, last leg slowest):
// P[r] = sum_e T[r, e] mL[e] (T contracted with the last leg's message, for
// the other legs' outgoing messages) and out[e] = sum_r T[r, e] x[r] with
// x[r] = prod_l xm[l][r_l] over the other legs (the last leg's outgoing
// message).  Block partials of out go to part (nblk x nL), summed in a fixed
// order by a second kernel.  nL <= 1024.
struct LastLegJob {
  const void* T; int64_t rows; int nL;
  int nx; const double* xm[3]; int xd[3];   // messages of the other legs, first leg fastest
  const double* mL;    // nL
  double* P;           // rows
  double* part;        // nblk x nL
  double* out;         // nL
  int64_t nblk, b0;    // blocks of this job, first block in the launch (set by the launcher)
};
// blocks (rows of the partial buffer) a job of `rows` rows needs
int64_t last_leg_blocks(int64_t rows, int is_double);
// fills b0 / nblk of the host jobs and the largest nL; returns the launch's
// block count, -1 if a job is out of range (nL > 1024, rows >= 2^31 - block)
int64_t last_leg_plan(LastLegJob* jobs_host, int njobs, int is_double, int* max_nl);
int launch_last_leg(const LastLegJob* jobs_dev, int njobs, int64_t blocks, int max_nl,
                    int is_double, hipStream_t s, const double* stop = nullptr);

// normalise, sign continuity, damp, normalise; delta[i] = max |mn - mo|
struct MeasNormJob {
  double* mo;
  const double* mh;
  int n;
};
int launch_meas_norm(const MeasNormJob* jobs, int njobs, double alpha, double* delta,
                     hipStream_t s, const double* stop = nullptr);

// ---- sign weights: z[c + n*p] = sum_r A[r + lda*c] w(r + m*p) for an m x n
// matrix, p = 0..3, with w the SplitMix64 weights of the gauge-sign rule
template <typename T>
int launch_sign_projection(const T* A, int64_t lda, int64_t m, int n, double* z, double* part,
                           int64_t part_cap, hipStream_t s);

}  // namespace hpt
