// R-core of the two-site gate update (paper Sec. "Gate Update" items 3-6,
// Algorithm "Gate update", and the bond matrix RR4 = A1 A2^T of the
// implementation pipeline figure; Eq. truncation; Eq. vidal_norm).
//
// The paper forms the k1 D x k2 D bond matrix over the cut bond, applies the
// 16 x 16 gate to the Pauli pair and takes its SVD.  Here the XX coupling,
// whose Pauli transfer matrix has operator-Schmidt rank 4, is split as
// G2 = sum_r F_r (x) H_r, so the gated bond matrix factors as B1 B2^T with
// B_i (4 k_i x 4 chi_cut); after a QR of each B_i only the small core
// T1 T2^T (at most 4 chi_cut square) is decomposed.  Same singular values
// and vectors, a 16x smaller SVD at saturation.
#include "rcore.h"

namespace hpt {

namespace {

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
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

__global__ __launch_bounds__(256) void build_B_kernel(BondCore* bonds, GateFactors g) {
  BondCore& bc = bonds[blockIdx.x];
  const int i = blockIdx.y;
  const int chi = bc.chi_cut, k = bc.k[i];
  const double* R = bc.R[i];
  const int ldR = bc.ldR;
  double* B = bc.B[i];
  const int ldB = 4 * k;
  const double(*Fr)[16] = (i == 0) ? g.F : g.H;
  const int64_t total = (int64_t)4 * k * 4 * chi;
  for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int row = (int)(idx % ldB), col = (int)(idx / ldB);
    const int kk = row % k, e = row / k;
    const int c = col % chi, r = col / chi;
    double s = 0.0;
    for (int d = 0; d < 4; ++d) s += Fr[r][e + 4 * d] * R[kk + (int64_t)(c + chi * d) * ldR];
    B[row + (int64_t)col * ldB] = s;
  }
}

// B_i[(kk, e), (c, r)] = sum_d Fr[r][e + 4d] R_i[kk, c + chi d], so
// (B_i^T B_i)[(c, r), (c', r')] = sum_{d, d'} phi[d][d'][r][r'] (R_i^T R_i)[c + chi d, c' + chi d']
// with phi[d][d'][r][r'] = sum_e Fr[r][e + 4d] Fr[r'][e + 4d'].
__global__ __launch_bounds__(256) void kron_gram_kernel(BondCore* bonds, GateFactors g) {
  BondCore& bc = bonds[blockIdx.x];
  const int i = blockIdx.y;
  if (bc.bqr[i] != 0) return;
  const int chi = bc.chi_cut, n = 4 * chi;
  const double(*Fr)[16] = (i == 0) ? g.F : g.H;
  __shared__ double phi[256];
  for (int t = threadIdx.x; t < 256; t += blockDim.x) {
    const int d = t & 3, d2 = (t >> 2) & 3, r = (t >> 4) & 3, r2 = t >> 6;
    double v = 0.0;
    for (int e = 0; e < 4; ++e) v += Fr[r][e + 4 * d] * Fr[r2][e + 4 * d2];
    phi[t] = v;
  }
  __syncthreads();
  const double* RtR = bc.qs[i][5];
  double* GB = bc.qs[i][0];
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = blockIdx.z * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.z * blockDim.x) {
    const int row = (int)(idx % n), col = (int)(idx / n);
    const int c = row % chi, r = row / chi, c2 = col % chi, r2 = col / chi;
    double v = 0.0;
    for (int d = 0; d < 4; ++d)
      for (int d2 = 0; d2 < 4; ++d2)
        v += phi[d + 4 * d2 + 16 * r + 64 * r2] * RtR[(c + chi * d) + (int64_t)(c2 + chi * d2) * n];
    GB[idx] = v;
  }
}

__global__ __launch_bounds__(256) void precond_prep_kernel(BondCore* bonds) {
  BondCore& bc = bonds[blockIdx.x];
  const int q0 = bc.q[0], q1 = bc.q[1];
  const int m = q0 > q1 ? q0 : q1, n = q0 < q1 ? q0 : q1;
  const int ld = bc.ldG;
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += blockDim.x) {
    const int i = (int)(idx % n), j = (int)(idx / n);
    bc.pq[1][i + (int64_t)j * ld] = bc.pq[0][j + (int64_t)i * ld];   // H = R^T
  }
  for (int64_t idx = threadIdx.x; idx < (int64_t)m * n; idx += blockDim.x) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    bc.pq[2][i + (int64_t)j * ld] = bc.G[i + (int64_t)j * ld];       // Q
  }
}

// one wave per column p: sigma_p = |H_out[:, p]|, pq[0][:, p] = V_H[:, p] sigma_p,
// V[:, p] = H_out[:, p] / sigma_p (0 for a zero column)
__global__ __launch_bounds__(1024) void precond_finish_kernel(BondCore* bonds) {
  BondCore& bc = bonds[blockIdx.x];
  const int q0 = bc.q[0], q1 = bc.q[1];
  const int n = q0 < q1 ? q0 : q1;
  const int ld = bc.ldG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int p = wave; p < n; p += nw) {
    const double* h = bc.pq[1] + (int64_t)p * ld;
    double a = 0.0;
    for (int i = lane; i < n; i += 64) a += h[i] * h[i];
    a = wave_sum(a);
    const double sg = sqrt(a);
    const double inv = sg > 0.0 ? 1.0 / sg : 0.0;
    for (int i = lane; i < n; i += 64) {
      bc.pq[0][i + (int64_t)p * ld] = bc.pq[3][i + (int64_t)p * ld] * sg;
      bc.V[i + (int64_t)p * ld] = h[i] * inv;
    }
  }
}

__global__ __launch_bounds__(1024) void select_kernel(BondCore* bonds) {
  BondCore& bc = bonds[blockIdx.x];
  __shared__ double sh[16];
  __shared__ int s_keep;
  const int q0 = bc.q[0], q1 = bc.q[1];
  const int nsv = q0 < q1 ? q0 : q1;
  const bool transposed = q0 < q1;
  const double s0 = bc.s[0];
  if (!(s0 > 0.0) || !isfinite(s0)) {
    if (threadIdx.x == 0) {
      bc.status = 1;
      bc.chi_new = 0;
      bc.n4 = 0;
    }
    return;
  }
  if (threadIdx.x == 0) {
    int keep = 0;
    for (int j = 0; j < nsv; ++j)
      if (bc.s[j] >= bc.eps_cut * s0) ++keep;
    s_keep = keep < bc.chi_max ? keep : bc.chi_max;
  }
  __syncthreads();
  const int chi_new = s_keep;
  double pk = 0.0, pa = 0.0;
  for (int j = threadIdx.x; j < nsv; j += blockDim.x) {
    const double v = bc.s[j] * bc.s[j];
    pa += v;
    if (j < chi_new) pk += v;
  }
  const double sk = block_sum(pk, sh);
  const double sa = block_sum(pa, sh);
  const double inv = 1.0 / sqrt(sk);
  for (int j = threadIdx.x; j < chi_new; j += blockDim.x) bc.lam[j] = bc.s[j] * inv;
  // diag(lambda) into both directed gauge messages
  for (int idx = threadIdx.x; idx < chi_new * chi_new; idx += blockDim.x) {
    const int a = idx % chi_new, b = idx / chi_new;
    const double v = (a == b) ? bc.s[a] * inv : 0.0;
    bc.msg[0][idx] = v;
    bc.msg[1][idx] = v;
  }
  // scaled singular vectors
  const int ldG = bc.ldG;
  for (int idx = threadIdx.x; idx < (q0 + q1) * chi_new; idx += blockDim.x) {
    const bool left = idx < q0 * chi_new;
    const int e = left ? idx : idx - q0 * chi_new;
    const int len = left ? q0 : q1;
    const int r = e % len, j = e / len;
    const int p = bc.perm[j];
    const double sj = bc.s[j];
    const double rs = sqrt(sj);
    double v;
    if (left != transposed)  // vector stored in G's columns (scaled by sigma)
      v = bc.G[r + (int64_t)p * ldG] / sj * rs;
    else
      v = bc.V[r + (int64_t)p * ldG] * rs;
    if (left)
      bc.Uc[r + (int64_t)j * ldG] = v;
    else
      bc.Vc[r + (int64_t)j * ldG] = v;
  }
  if (threadIdx.x == 0) {
    bc.chi_new = chi_new;
    bc.n4 = 4 * chi_new;
    bc.gate_err = (sa - sk) / sa;
    bc.s0 = s0;
    bc.status = 0;
    int fl = 0;
    if (chi_new == bc.chi_max && chi_new < nsv && bc.s[chi_new - 1] - bc.s[chi_new] <= 1e-10 * s0)
      fl |= 1 << 4;
    bc.flags |= fl;
  }
}

// Mp_i[k, j + chi_new e] = Mf_i[k + k_i e, j]; on the Householder path Mp is W
__global__ __launch_bounds__(256) void rearrange_kernel(BondCore* bonds) {
  BondCore& bc = bonds[blockIdx.x];
  if (bc.status) return;
  const int i = blockIdx.y;
  const int k = bc.k[i], cn = bc.chi_new;
  const double* Mf = bc.Mf[i];
  double* dst = bc.chol[i] ? bc.Mp[i] : bc.W[i];
  const int64_t total = (int64_t)k * 4 * cn;
  for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int kk = (int)(idx % k), col = (int)(idx / k);
    const int j = col % cn, e = col / cn;
    dst[kk + (int64_t)col * k] = Mf[kk + (int64_t)k * e + (int64_t)j * 4 * k];
  }
}

// gauge-sign rule: flip channel j when <w, cv1_new[:, j, :]> < 0
__global__ __launch_bounds__(256) void signs_kernel(BondCore* bonds) {
  BondCore& bc = bonds[blockIdx.x];
  if (bc.status) return;
  const int cn = bc.chi_new;
  const int n0 = bc.chol[0] ? 4 * bc.chi_cut : bc.k[0];
  const int n1 = bc.chol[1] ? 4 * bc.chi_cut : bc.k[1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __shared__ double flip[1024];
  for (int j = wave; j < cn; j += nw) {
    double t = 0.0;
    for (int idx = lane; idx < 4 * n0; idx += 64) {
      const int r = idx % n0, p = idx / n0;
      t += bc.z[r + (int64_t)n0 * p] * bc.W[0][r + (int64_t)(j + cn * p) * n0];
    }
    t = wave_sum(t);
    if (lane == 0) flip[j] = t < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 4 * cn * n0; idx += blockDim.x) {
    const int col = idx / n0, j = col % cn;
    if (flip[j] < 0.0) bc.W[0][idx] = -bc.W[0][idx];
  }
  for (int idx = threadIdx.x; idx < 4 * cn * n1; idx += blockDim.x) {
    const int col = idx / n1, j = col % cn;
    if (flip[j] < 0.0) bc.W[1][idx] = -bc.W[1][idx];
  }
}

}  // namespace

int launch_rcore_build_B(BondCore* bonds, int nb, const GateFactors& g, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(build_B_kernel, dim3(nb, 2), dim3(256), 0, s, bonds, g);
  HPT_LAUNCH_CHECK("build_B_kernel");
  return 0;
}
int launch_rcore_kron_gram(BondCore* bonds, int nb, const GateFactors& g, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(kron_gram_kernel, dim3(nb, 2, 32), dim3(256), 0, s, bonds, g);
  HPT_LAUNCH_CHECK("kron_gram_kernel");
  return 0;
}
int launch_rcore_precond_prep(BondCore* bonds, int nb, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(precond_prep_kernel, dim3(nb), dim3(256), 0, s, bonds);
  HPT_LAUNCH_CHECK("precond_prep_kernel");
  return 0;
}
int launch_rcore_precond_finish(BondCore* bonds, int nb, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(precond_finish_kernel, dim3(nb), dim3(1024), 0, s, bonds);
  HPT_LAUNCH_CHECK("precond_finish_kernel");
  return 0;
}
int launch_rcore_select(BondCore* bonds, int nb, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(select_kernel, dim3(nb), dim3(1024), 0, s, bonds);
  HPT_LAUNCH_CHECK("select_kernel");
  return 0;
}
int launch_rcore_rearrange(BondCore* bonds, int nb, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(rearrange_kernel, dim3(nb, 2), dim3(256), 0, s, bonds);
  HPT_LAUNCH_CHECK("rearrange_kernel");
  return 0;
}
int launch_rcore_signs(BondCore* bonds, int nb, hipStream_t s) {
  if (nb <= 0) return 0;
  hipLaunchKernelGGL(signs_kernel, dim3(nb), dim3(256), 0, s, bonds);
  HPT_LAUNCH_CHECK("signs_kernel");
  return 0;
}

}  // namespace hpt
