// Elementwise and reduction kernels: field half-step (Sec. "Trotter Decomposition"), BP message
// normalisation and damping (Eq. bp, Eq. bp_tol, Eq. damping), measurement
// contractions of the pinned network (Sec. "Correlation Function via Belief
// Propagation", Eq. bethe_raw), the log-space sum with sign tracking
// (Eq. bethe), and the projections used by the gauge-sign rule.
#include <algorithm>
#include "misc.h"
#include "wave.h"

namespace hpt {

namespace {

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
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
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, sh[i]);
  return r;
}

inline int grid_for(int64_t n) {
  int64_t g = ceil_div(n, 256);
  return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void field_kernel(T* psi, int64_t slice, double gxx, double gxy, double gyx,
                             double gyy) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < slice;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)psi[i + slice], y = (double)psi[i + 2 * slice];
    psi[i + slice] = (T)(gxx * x + gxy * y);
    psi[i + 2 * slice] = (T)(gyx * x + gyy * y);
  }
}

__global__ void d2f_kernel(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

__global__ void fill_identity_kernel(double* M, int n, double scale) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n * n;
       i += (int64_t)gridDim.x * blockDim.x)
    M[i] = (i % n == i / n) ? scale : 0.0;
}

template <typename T>
__global__ void fill_kernel(T* v, int64_t n, double value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (T)value;
}

template <typename T>
__global__ void scale_columns_kernel(T* A, int64_t lda, int64_t m, int ncols,
                                     const double* colscale) {
  const int64_t total = m * ncols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i % m, c = i / m;
    A[r + c * lda] = (T)((double)A[r + c * lda] * colscale[c]);
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gauge_norm_kernel(const GaugeNormJob* jobs, double alpha,
                                                         double* delta) {
  const GaugeNormJob job = jobs[blockIdx.x];
  const int n = job.n;
  __shared__ double sh[16];
  double part = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    const double s = 0.5 * (job.Mh[i + j * n] + job.Mh[j + i * n]);
    part += s * s;
  }
  const double nrm2 = block_sum(part, sh);
  const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 1.0;
  part = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    const double s = 0.5 * (job.Mh[i + j * n] + job.Mh[j + i * n]) * inv;
    const double v = (1.0 - alpha) * job.Mo[idx] + alpha * s;
    part += v * v;
  }
  const double nn2 = block_sum(part, sh);
  const double inv2 = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 1.0;
  double dmax = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    const double s = 0.5 * (job.Mh[i + j * n] + job.Mh[j + i * n]) * inv;
    const double v = ((1.0 - alpha) * job.Mo[idx] + alpha * s) * inv2;
    dmax = fmax(dmax, fabs(v - job.Mo[idx]));
  }
  const double dm = block_max(dmax, sh);
  // all reads of Mo are complete (barriers inside block_max)
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    const double s = 0.5 * (job.Mh[i + j * n] + job.Mh[j + i * n]) * inv;
    job.Mo[idx] = ((1.0 - alpha) * job.Mo[idx] + alpha * s) * inv2;
  }
  if (threadIdx.x == 0) delta[blockIdx.x] = dm;
}

__global__ __launch_bounds__(256) void dots_kernel(const DotJob* jobs) {
  const DotJob job = jobs[blockIdx.x];
  __shared__ double sh[16];
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < job.n; i += blockDim.x) part += job.a[i] * job.b[i];
  const double r = block_sum(part, sh);
  if (threadIdx.x == 0) *job.out = r;
}

// Sweep gate of the measurement BP: the kernels of a sweep return at once
// when the flag a previous sweep's log_product_kernel raised is set (stop
// null: always run).  The flag is written only between kernels, so every
// workgroup of one launch sees the same value.
__device__ __forceinline__ bool stopped(const double* stop) { return stop && *(const volatile double*)stop != 0.0; }

__global__ __launch_bounds__(256) void log_product_kernel(const double* x, int n_num, int n_den,
                                                          const double* delta, int n_delta,
                                                          double* res, double tol, double* ctl) {
  if (stopped(ctl)) return;
  __shared__ double sh[16];
  double part = 0.0, neg = 0.0, zn = 0.0, zd = 0.0, dmax = 0.0;
  for (int i = threadIdx.x; i < n_num + n_den; i += blockDim.x) {
    const double v = x[i];
    const bool num = i < n_num;
    if (v == 0.0) {
      if (num) zn = 1.0; else zd = 1.0;
      continue;
    }
    part += (num ? 1.0 : -1.0) * log(fabs(v));
    if (v < 0.0) neg += 1.0;
  }
  if (delta)
    for (int i = threadIdx.x; i < n_delta; i += blockDim.x) dmax = fmax(dmax, delta[i]);
  const double s = block_sum(part, sh);
  const double ng = block_sum(neg, sh);
  const double a = block_max(zn, sh);
  const double b = block_max(zd, sh);
  const double d = block_max(dmax, sh);
  if (threadIdx.x == 0) {
    res[0] = s;
    res[1] = (((long long)ng) & 1) ? -1.0 : 1.0;
    res[2] = a;
    res[3] = b;
    res[4] = d;
    if (ctl) {   // one more sweep taken; stop at convergence or a non-finite residual
      ctl[1] += 1.0;
      if (d < tol || !isfinite(d)) ctl[0] = 1.0;
    }
  }
}

// ---------------------------------------------------------------------------
// measurement contraction stages; every stage launches exactly the blocks
// the jobs need (per-job block ranges, binary search of the job)
constexpr int MEAS_CHUNK = 256;  // o values per gemv_n block, i chunk = 64 * MEAS_CHUNK
constexpr int MEAS_TW = 4;       // waves per gemv_t block

__device__ inline int find_job(const MeasJob* jobs, int njobs, int64_t b, int which) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t st = which == 0 ? jobs[mid].bk0 : which == 1 ? jobs[mid].bn0 : which == 2 ? jobs[mid].bt0 : jobs[mid].br0;
    if (st <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void meas_kron_kernel(const MeasJob* jobs, int njobs, const double* stop) {
  if (stopped(stop)) return;
  const int j = find_job(jobs, njobs, blockIdx.x, 0);
  const MeasJob& job = jobs[j];
  const int64_t idx = (blockIdx.x - job.bk0) * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= job.I + job.O) return;
  const bool isx = idx < job.I;
  int64_t rem = isx ? idx : idx - job.I;
  const int nl = isx ? job.nx : job.ny;
  double v = 1.0;
  for (int l = 0; l < nl; ++l) {
    const int d = isx ? job.xd[l] : job.yd[l];
    const double* m = isx ? job.xm[l] : job.ym[l];
    v *= m[rem % d];
    rem /= d;
  }
  if (isx) job.x[idx] = v; else job.y[idx - job.I] = v;
}

// part[pn_off + oc * rows + r] = sum_{o in chunk oc} T[r + rows * o] y[o]
template <typename T>
__global__ void meas_gemv_n_kernel(const MeasJob* jobs, int njobs, double* part, const double* stop) {
  if (stopped(stop)) return;
  const int j = find_job(jobs, njobs, blockIdx.x, 1);
  const MeasJob& job = jobs[j];
  const int64_t rows = job.I * job.nk;
  const int64_t rb = ceil_div(rows, 256);
  const int64_t b = blockIdx.x - job.bn0;
  const int64_t r = (b % rb) * 256 + threadIdx.x;
  const int64_t oc = b / rb;
  if (r >= rows) return;
  const int64_t o0 = oc * MEAS_CHUNK;
  const int64_t o1 = o0 + MEAS_CHUNK < job.O ? o0 + MEAS_CHUNK : job.O;
  const T* Tp = (const T*)job.T;
  double acc = 0.0;
  for (int64_t o = o0; o < o1; ++o) acc += (double)Tp[r + rows * o] * job.y[o];
  part[job.pn_off + oc * rows + r] = acc;
}

__global__ void meas_gemv_n_reduce(const MeasJob* jobs, int njobs, const double* part, const double* stop) {
  if (stopped(stop)) return;
  const int j = find_job(jobs, njobs, blockIdx.x, 3);
  const MeasJob& job = jobs[j];
  const int64_t rows = job.I * job.nk;
  const int64_t r = (blockIdx.x - job.br0) * (int64_t)blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int64_t nch = ceil_div(job.O, MEAS_CHUNK);
  double acc = 0.0;
  for (int64_t c = 0; c < nch; ++c) acc += part[job.pn_off + c * rows + r];
  job.S[r] = acc;
}

// part[pt_off + a * nich + ic] = sum_{i in chunk ic} S[i + I a] x[i]; one wave per (a, ic)
template <typename T>
__global__ __launch_bounds__(256) void meas_gemv_t_kernel(const MeasJob* jobs, int njobs, double* part,
                                                          const double* stop) {
  if (stopped(stop)) return;
  const int j = find_job(jobs, njobs, blockIdx.x, 2);
  const MeasJob& job = jobs[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t chunk = 64 * MEAS_CHUNK;
  const int64_t nich = ceil_div(job.I, chunk);
  const int64_t w = (blockIdx.x - job.bt0) * MEAS_TW + wave;
  if (w >= nich * job.nk) return;
  const int64_t a = w / nich, ic = w % nich;
  const int64_t i0 = ic * chunk;
  const int64_t i1 = i0 + chunk < job.I ? i0 + chunk : job.I;
  double acc = 0.0;
  if (job.O > 1) {
    for (int64_t i = i0 + lane; i < i1; i += 64) acc += job.S[i + job.I * a] * job.x[i];
  } else {
    const T* Tp = (const T*)job.T;
    for (int64_t i = i0 + lane; i < i1; i += 64) acc += (double)Tp[i + job.I * a] * job.x[i];
  }
  acc = wave_sum(acc);
  if (lane == 0) part[job.pt_off + a * nich + ic] = acc;
}

__global__ void meas_gemv_t_reduce(const MeasJob* jobs, const double* part, const double* stop) {
  if (stopped(stop)) return;
  const MeasJob& job = jobs[blockIdx.x];
  const int64_t nich = ceil_div(job.I, 64 * MEAS_CHUNK);
  for (int64_t a = threadIdx.x; a < job.nk; a += blockDim.x) {
    double acc = 0.0;
    for (int64_t c = 0; c < nich; ++c) acc += part[job.pt_off + a * nich + c];
    job.out[a] = acc;
  }
}

// Rows per lane of the last-leg kernel: NV 16-byte vectors (4 floats or 2
// doubles each) per column; a block of 256 lanes covers 256 x that many rows.
// Three float vectors per lane (12 rows) measured best on the 10x10 chi=100
// sweep: two pay twice the per-column wave reductions, four need 180 VGPRs
// (two waves per SIMD) and leave fewer bytes in flight.  The kernel is held
// to 128 VGPRs (four waves per SIMD, no spills), 7% faster than 130.
constexpr int LL_MAXL = 1024;
template <typename T> struct LLShape {
  static constexpr int V = 16 / (int)sizeof(T);   // rows per vector
  static constexpr int NV = sizeof(T) == 4 ? 3 : 2;
  static constexpr int R = V * NV;                // rows per lane
  static constexpr int BR = 256 * R;              // rows per block
};
// 16-byte vectors in the global address space (plain global loads, waited on
// by the vector-memory counter alone)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = f32x4; };
template <> struct Vec16<double> { using type = f64x2; };
#define HPT_GLOBAL __attribute__((address_space(1)))

__device__ inline int find_ll(const LastLegJob* jobs, int njobs, int64_t b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].b0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Column loop of the last-leg kernel for one block.  VEC: the slice allows
// 16-byte loads (aligned base, rows a multiple of V); FULL: every row of the
// block is inside the slice, so no row guards.  All variants fold the same
// rows in the same order, so they give equal bits.
template <typename T, bool VEC, bool FULL>
__device__ __forceinline__ void ll_columns(const double* mL, const T* Tp, int rows, int nL,
                                           int rb, const double (&xr)[LLShape<T>::NV][LLShape<T>::V],
                                           double (&pacc)[LLShape<T>::NV][LLShape<T>::V],
                                           double* wp, int lane, int wave) {
  using S = LLShape<T>;
  constexpr int V = S::V, NV = S::NV;
  using VecT = typename Vec16<T>::type;
  typedef const T HPT_GLOBAL* GP;
  typedef const VecT HPT_GLOBAL* GVP;
  GP base = (GP)Tp + rb;   // this lane's first row of column 0
  auto load = [&](int e, T (&t)[NV][V]) {
    GP col = base + (int64_t)rows * e;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const bool in = FULL || rb + k * 64 * V < rows;
      if (VEC) {
        VecT x;
        if (in) x = *(GVP)(col + k * 64 * V);
        else x = VecT(0);
#pragma unroll
        for (int j = 0; j < V; ++j) t[k][j] = x[j];
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
          t[k][j] = (FULL || rb + k * 64 * V + j < rows) ? col[k * 64 * V + j] : T(0);
      }
    }
  };
  auto fold = [&](int e, const T (&t)[NV][V]) {
    const double me = mL[e];
    double sk[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const double x = (double)t[k][j];
        pacc[k][j] += x * me;
        s += x * xr[k][j];
      }
      sk[k] = s;
    }
    double s = sk[0];
#pragma unroll
    for (int k = 1; k < NV; ++k) s += sk[k];
    s = wave_sum(s);
    if (lane == 0) wp[wave * nL + e] = s;
  };
  // two register buffers; the prefetches in the loop are unconditional, so
  // each wait before a fold leaves the next column's loads in flight
  T a[NV][V], b[NV][V];
  load(0, a);
  int e = 0;
  for (; e + 3 <= nL; e += 2) {
    load(e + 1, b);
    fold(e, a);
    load(e + 2, a);
    fold(e + 1, b);
  }
  if (e + 2 == nL) {
    load(e + 1, b);
    fold(e, a);
    fold(e + 1, b);
  } else {
    fold(e, a);
  }
}

// One pass over the column-major slice T (rows x nL): out-partials
// part[blk, e] = sum_r T[r, e] x(r) with x the product of the other legs'
// messages, and P[r] = sum_e T[r, e] mL[e].  Lane vector k covers V
// consecutive rows; the 64 lanes of a wave read 1 KB contiguous per vector, a
// column is read as NV such vectors per lane and the next column's loads
// are issued before the current one is folded.  Per column each wave reduces
// its 64 lane sums once (DPP), so the reduction is paid once per 64 x R rows.
template <typename T>
__global__ __launch_bounds__(256, 4) void last_leg_kernel(const LastLegJob* jobs, int njobs, const double* stop) {
  if (stopped(stop)) return;
  using S = LLShape<T>;
  constexpr int V = S::V, NV = S::NV;
  // LDS: the 4 waves' column sums [4][nL], then the last leg's message (read
  // from LDS so that waiting for it never waits for the column loads in flight)
  extern __shared__ double wp[];
  const LastLegJob& job = jobs[find_ll(jobs, njobs, blockIdx.x)];
  const int blk = (int)(blockIdx.x - job.b0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = (int)job.rows;
  const int nL = job.nL;
  const T* Tp = (const T*)job.T;
  const bool vec = ((reinterpret_cast<uintptr_t>(Tp) & 15) == 0) && (rows % V == 0);
  const bool full = (int64_t)(blk + 1) * S::BR <= rows;
  const int rb = blk * S::BR + wave * (64 * S::R) + lane * V;

  double xr[NV][V], pacc[NV][V];
  const int nx = job.nx;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int r0 = rb + k * 64 * V;
    int idx[3] = {0, 0, 0};
    if (r0 < rows) {
      int rem = r0;
      for (int l = 0; l < nx; ++l) {
        idx[l] = rem % job.xd[l];
        rem /= job.xd[l];
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      pacc[k][j] = 0.0;
      double v = 0.0;
      if (r0 + j < rows) {
        v = 1.0;
        for (int l = 0; l < nx; ++l) v *= job.xm[l][idx[l]];
        // next row: first leg fastest, carry into the slower legs
        for (int l = 0; l < nx; ++l) {
          if (++idx[l] < job.xd[l]) break;
          idx[l] = 0;
        }
      }
      xr[k][j] = v;
    }
  }

  double* ml = wp + 4 * nL;
  for (int c = threadIdx.x; c < nL; c += blockDim.x) ml[c] = job.mL[c];
  __syncthreads();
  if (vec && full) ll_columns<T, true, true>(ml, Tp, rows, nL, rb, xr, pacc, wp, lane, wave);
  else if (vec) ll_columns<T, true, false>(ml, Tp, rows, nL, rb, xr, pacc, wp, lane, wave);
  else ll_columns<T, false, false>(ml, Tp, rows, nL, rb, xr, pacc, wp, lane, wave);

  double HPT_GLOBAL* P = (double HPT_GLOBAL*)job.P;
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int r = rb + k * 64 * V + j;
      if (r < rows) P[r] = pacc[k][j];
    }
  __syncthreads();
  for (int c = threadIdx.x; c < nL; c += blockDim.x)
    job.part[(int64_t)blk * nL + c] =
        (wp[c] + wp[nL + c]) + (wp[2 * nL + c] + wp[3 * nL + c]);
}

// out[e] = sum over blocks of part[blk, e]: 8 groups of 128 columns, fixed order
__global__ __launch_bounds__(1024) void last_leg_reduce(const LastLegJob* jobs, const double* stop) {
  if (stopped(stop)) return;
  const LastLegJob& job = jobs[blockIdx.x];
  __shared__ double red[8][129];
  const int c = threadIdx.x & 127, g = threadIdx.x >> 7;
  for (int e0 = 0; e0 < job.nL; e0 += 128) {
    const int e = e0 + c;
    double acc = 0.0;
    if (e < job.nL)
      for (int64_t b = g; b < job.nblk; b += 8) acc += job.part[b * job.nL + e];
    red[g][c] = acc;
    __syncthreads();
    if (g == 0 && e < job.nL) {
      double s = 0.0;
      for (int q = 0; q < 8; ++q) s += red[q][c];
      job.out[e] = s;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void meas_norm_kernel(const MeasNormJob* jobs, double alpha,
                                                        double* delta, const double* stop) {
  if (stopped(stop)) return;
  const MeasNormJob job = jobs[blockIdx.x];
  const int n = job.n;
  __shared__ double sh[16];
  double p1 = 0.0, p2 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    p1 += job.mh[i] * job.mh[i];
    p2 += job.mh[i] * job.mo[i];
  }
  const double nrm2 = block_sum(p1, sh);
  const double ov = block_sum(p2, sh);
  double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 1.0;
  if (ov * inv < 0.0) inv = -inv;   // sign continuity
  double p3 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = (1.0 - alpha) * job.mo[i] + alpha * job.mh[i] * inv;
    p3 += v * v;
  }
  const double nn2 = block_sum(p3, sh);
  const double inv2 = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 1.0;
  double dmax = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = ((1.0 - alpha) * job.mo[i] + alpha * job.mh[i] * inv) * inv2;
    dmax = fmax(dmax, fabs(v - job.mo[i]));
  }
  const double dm = block_max(dmax, sh);
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    job.mo[i] = ((1.0 - alpha) * job.mo[i] + alpha * job.mh[i] * inv) * inv2;
  if (threadIdx.x == 0) delta[blockIdx.x] = dm;
}

// ---------------------------------------------------------------------------
// SplitMix64 weights (Steele, Lea, Flood 2014): state_i = (i+1)*gamma and
// the 64-bit finaliser; w_i = (z >> 11) * 2^-53 - 1/2
__device__ inline double sign_weight(uint64_t i) {
  uint64_t z = (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

constexpr int SP_ROWS = 2048;
// part[(chunk * n + c) * 4 + p] = sum_{r in chunk} A[r, c] w(r + m p)
template <typename T>
__global__ __launch_bounds__(256) void sign_proj_kernel(const T* A, int64_t lda, int64_t m, int n,
                                                        double* part) {
  const int64_t chunk = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = chunk * SP_ROWS;
  const int64_t r1 = r0 + SP_ROWS < m ? r0 + SP_ROWS : m;
  for (int c = blockIdx.x * 4 + wave; c < n; c += gridDim.x * 4) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t r = r0 + lane; r < r1; r += 64) {
      const double a = (double)A[r + c * lda];
      for (int p = 0; p < 4; ++p) s[p] += a * sign_weight((uint64_t)(r + m * p));
    }
    for (int p = 0; p < 4; ++p) {
      const double v = wave_sum(s[p]);
      if (lane == 0) part[(chunk * n + c) * 4 + p] = v;
    }
  }
}

__global__ void sign_proj_reduce(const double* part, int64_t nchunks, int n, double* z) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < 4 * n;
       idx += gridDim.x * blockDim.x) {
    const int c = idx % n, p = idx / n;
    double s = 0.0;
    for (int64_t k = 0; k < nchunks; ++k) s += part[(k * n + c) * 4 + p];
    z[c + (int64_t)n * p] = s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
template <typename T>
int launch_field(T* psi, int64_t slice, double gxx, double gxy, double gyx, double gyy,
                 hipStream_t s) {
  if (slice <= 0) return 0;
  hipLaunchKernelGGL(field_kernel<T>, dim3(grid_for(slice)), dim3(256), 0, s, psi, slice, gxx,
                     gxy, gyx, gyy);
  HPT_LAUNCH_CHECK("field_kernel");
  return 0;
}
template int launch_field<double>(double*, int64_t, double, double, double, double, hipStream_t);
template int launch_field<float>(float*, int64_t, double, double, double, double, hipStream_t);

int launch_d2f(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(d2f_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  HPT_LAUNCH_CHECK("d2f_kernel");
  return 0;
}

int launch_fill_identity(double* M, int n, double scale, hipStream_t s) {
  hipLaunchKernelGGL(fill_identity_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, M, n,
                     scale);
  HPT_LAUNCH_CHECK("fill_identity_kernel");
  return 0;
}

int launch_fill_value(double* v, int64_t n, double value, hipStream_t s) {
  return launch_fill_t<double>(v, n, value, s);
}

template <typename T>
int launch_fill_t(T* v, int64_t n, double value, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, v, n, value);
  HPT_LAUNCH_CHECK("fill_kernel");
  return 0;
}
template int launch_fill_t<double>(double*, int64_t, double, hipStream_t);
template int launch_fill_t<float>(float*, int64_t, double, hipStream_t);

template <typename T>
int launch_scale_columns(T* A, int64_t lda, int64_t m, int ncols, const double* colscale,
                         hipStream_t s) {
  if (m <= 0 || ncols <= 0) return 0;
  hipLaunchKernelGGL(scale_columns_kernel<T>, dim3(grid_for(m * ncols)), dim3(256), 0, s, A, lda,
                     m, ncols, colscale);
  HPT_LAUNCH_CHECK("scale_columns_kernel");
  return 0;
}
template int launch_scale_columns<double>(double*, int64_t, int64_t, int, const double*,
                                          hipStream_t);
template int launch_scale_columns<float>(float*, int64_t, int64_t, int, const double*,
                                         hipStream_t);

int launch_gauge_norm(const GaugeNormJob* jobs, int njobs, double alpha, double* delta,
                      hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(gauge_norm_kernel, dim3(njobs), dim3(256), 0, s, jobs, alpha, delta);
  HPT_LAUNCH_CHECK("gauge_norm_kernel");
  return 0;
}

int launch_dots(const DotJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(dots_kernel, dim3(njobs), dim3(256), 0, s, jobs);
  HPT_LAUNCH_CHECK("dots_kernel");
  return 0;
}

int launch_log_product(const double* x, int n_num, int n_den, const double* delta, int n_delta,
                       double* res, hipStream_t s, double tol, double* ctl) {
  hipLaunchKernelGGL(log_product_kernel, dim3(1), dim3(256), 0, s, x, n_num, n_den, delta,
                     n_delta, res, tol, ctl);
  HPT_LAUNCH_CHECK("log_product_kernel");
  return 0;
}

int64_t last_leg_blocks(int64_t rows, int is_double) {
  return ceil_div(rows, is_double ? LLShape<double>::BR : LLShape<float>::BR);
}

int64_t last_leg_plan(LastLegJob* jobs, int njobs, int is_double, int* max_nl) {
  int64_t b = 0;
  int ml = 1;
  const int64_t br = is_double ? LLShape<double>::BR : LLShape<float>::BR;
  for (int j = 0; j < njobs; ++j) {
    // row indices are 32-bit inside the kernel (rows of the last block included)
    if (jobs[j].nL < 1 || jobs[j].nL > LL_MAXL || jobs[j].rows < 1 ||
        jobs[j].rows > 0x7fffffffll - br || jobs[j].nx < 0 || jobs[j].nx > 3)
      return -1;
    jobs[j].b0 = b;
    jobs[j].nblk = last_leg_blocks(jobs[j].rows, is_double);
    b += jobs[j].nblk;
    ml = std::max(ml, jobs[j].nL);
  }
  if (max_nl) *max_nl = ml;
  return b > 0x7fffffffll ? -1 : b;
}

int launch_last_leg(const LastLegJob* jobs_dev, int njobs, int64_t blocks, int max_nl,
                    int is_double, hipStream_t s, const double* stop) {
  if (njobs <= 0) return 0;
  if (blocks < 1 || blocks > 0x7fffffffll || max_nl < 1 || max_nl > LL_MAXL) return -1;
  const size_t lds = (size_t)5 * max_nl * sizeof(double);
  if (is_double)
    hipLaunchKernelGGL(last_leg_kernel<double>, dim3((unsigned)blocks), dim3(256), lds, s, jobs_dev, njobs, stop);
  else
    hipLaunchKernelGGL(last_leg_kernel<float>, dim3((unsigned)blocks), dim3(256), lds, s, jobs_dev, njobs, stop);
  HPT_LAUNCH_CHECK("last_leg_kernel");
  hipLaunchKernelGGL(last_leg_reduce, dim3(njobs), dim3(1024), 0, s, jobs_dev, stop);
  HPT_LAUNCH_CHECK("last_leg_reduce");
  return 0;
}

int64_t meas_plan(MeasJob* jobs, int njobs, int64_t totals[4]) {
  int64_t bk = 0, bn = 0, bt = 0, br = 0, part = 0;
  for (int j = 0; j < njobs; ++j) {
    MeasJob& q = jobs[j];
    q.bk0 = bk;
    bk += ceil_div(q.I + q.O, 256);
    const int64_t rows = q.I * q.nk;
    q.bn0 = bn;
    q.br0 = br;
    q.pn_off = part;
    if (q.O > 1) {
      bn += ceil_div(rows, 256) * ceil_div(q.O, MEAS_CHUNK);
      br += ceil_div(rows, 256);
      part += ceil_div(q.O, MEAS_CHUNK) * rows;
    }
    const int64_t nich = ceil_div(q.I, 64 * MEAS_CHUNK);
    q.bt0 = bt;
    bt += ceil_div(nich * q.nk, MEAS_TW);
    q.pt_off = part;
    part += nich * q.nk;
  }
  totals[0] = bk;
  totals[1] = bn;
  totals[2] = bt;
  totals[3] = br;
  return part;
}

int meas_launch(const MeasJob* jobs_dev, int njobs, const int64_t totals[4], int is_double,
                double* part, hipStream_t s, const double* stop) {
  if (njobs <= 0) return 0;
  for (int k = 0; k < 4; ++k)
    if (totals[k] > 0x7fffffffll) return -1;
  if (totals[0] > 0) {
    hipLaunchKernelGGL(meas_kron_kernel, dim3((unsigned)totals[0]), dim3(256), 0, s, jobs_dev, njobs, stop);
    HPT_LAUNCH_CHECK("meas_kron_kernel");
  }
  if (totals[1] > 0) {
    if (is_double)
      hipLaunchKernelGGL(meas_gemv_n_kernel<double>, dim3((unsigned)totals[1]), dim3(256), 0, s, jobs_dev,
                         njobs, part, stop);
    else
      hipLaunchKernelGGL(meas_gemv_n_kernel<float>, dim3((unsigned)totals[1]), dim3(256), 0, s, jobs_dev,
                         njobs, part, stop);
    HPT_LAUNCH_CHECK("meas_gemv_n_kernel");
    hipLaunchKernelGGL(meas_gemv_n_reduce, dim3((unsigned)totals[3]), dim3(256), 0, s, jobs_dev, njobs, part,
                       stop);
    HPT_LAUNCH_CHECK("meas_gemv_n_reduce");
  }
  if (totals[2] > 0) {
    if (is_double)
      hipLaunchKernelGGL(meas_gemv_t_kernel<double>, dim3((unsigned)totals[2]), dim3(256), 0, s, jobs_dev,
                         njobs, part, stop);
    else
      hipLaunchKernelGGL(meas_gemv_t_kernel<float>, dim3((unsigned)totals[2]), dim3(256), 0, s, jobs_dev,
                         njobs, part, stop);
    HPT_LAUNCH_CHECK("meas_gemv_t_kernel");
  }
  hipLaunchKernelGGL(meas_gemv_t_reduce, dim3(njobs), dim3(256), 0, s, jobs_dev, part, stop);
  HPT_LAUNCH_CHECK("meas_gemv_t_reduce");
  return 0;
}

int launch_meas_norm(const MeasNormJob* jobs, int njobs, double alpha, double* delta,
                     hipStream_t s, const double* stop) {
  if (njobs <= 0) return 0;
  hipLaunchKernelGGL(meas_norm_kernel, dim3(njobs), dim3(256), 0, s, jobs, alpha, delta, stop);
  HPT_LAUNCH_CHECK("meas_norm_kernel");
  return 0;
}

template <typename T>
int launch_sign_projection(const T* A, int64_t lda, int64_t m, int n, double* z, double* part,
                           int64_t part_cap, hipStream_t s) {
  const int64_t nch = ceil_div(m, SP_ROWS);
  if (nch * n * 4 > part_cap) return -2;
  if (nch > 65535) return -1;
  dim3 grid((unsigned)ceil_div(n, 4), (unsigned)nch);
  hipLaunchKernelGGL(sign_proj_kernel<T>, grid, dim3(256), 0, s, A, lda, m, n, part);
  HPT_LAUNCH_CHECK("sign_proj_kernel");
  hipLaunchKernelGGL(sign_proj_reduce, dim3((unsigned)ceil_div(4 * n, 256)), dim3(256), 0, s,
                     part, nch, n, z);
  HPT_LAUNCH_CHECK("sign_proj_reduce");
  return 0;
}
template int launch_sign_projection<double>(const double*, int64_t, int64_t, int, double*,
                                            double*, int64_t, hipStream_t);
template int launch_sign_projection<float>(const float*, int64_t, int64_t, int, double*, double*,
                                           int64_t, hipStream_t);

}  // namespace hpt
