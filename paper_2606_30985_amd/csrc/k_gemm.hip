// MFMA GEMM for the dense contractions of the gate update and of the BP
// environment products (paper Sec. "Gate Update": absorption, reconstruction
// and deabsorption are matrix products; Sec. "Adaptive QR Decomposition":
// the Gram matrix cv^T cv).
//
// One workgroup = 4 wave64s = one 64 x 64 output tile; each wave owns a
// 32 x 32 quadrant as 2 x 2 blocks of the 16x16x4 MFMA (f64 or f32).  A and B
// tiles of depth 16 are staged through LDS with loads coalesced along the
// contiguous axis of each operand.  The reduction space (batch r, k-chunks)
// can be split across workgroups; partial tiles are then summed in float64
// by a second, deterministic kernel.
#include <cstdlib>

#include "common.h"

namespace hpt {

namespace {

constexpr int TM = 64, TN = 64, TK = 16, PAD = 2;

__device__ inline d4 mfma_op(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma_op(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 type; };
template <> struct Acc<float> { typedef f4 type; };

__device__ inline void tile_of(int64_t bx, int tiles_m, int tiles_n, int sym, int& z, int& tm, int& tn) {
  if (!sym) {
    const int64_t tiles = (int64_t)tiles_m * tiles_n;
    z = (int)(bx / tiles);
    const int64_t t = bx % tiles;
    tm = (int)(t % tiles_m);
    tn = (int)(t / tiles_m);
    return;
  }
  // upper-triangular tiles (tm <= tn), column by column
  const int64_t tiles = (int64_t)tiles_m * (tiles_m + 1) / 2;
  z = (int)(bx / tiles);
  int64_t t = bx % tiles;
  int c = 0;
  while (t > c) {
    t -= c + 1;
    ++c;
  }
  tm = (int)t;
  tn = c;
}

// store one result element; for a symmetric product also its mirror
template <typename T>
__device__ inline void put(const GemmDesc<T>& d, int z, int gi, int gj, double v, int splits,
                           int split, double* part) {
  if (d.sym && gi > gj) return;
  if (splits > 1) {
    part[(((int64_t)split * d.Z + z) * d.N + gj) * d.M + gi] = v;
    return;
  }
  for (int rep = 0; rep < (d.sym && gi != gj ? 2 : 1); ++rep) {
    const int r = rep ? gj : gi, c = rep ? gi : gj;
    const int64_t off = (int64_t)z * d.sCz + r + (int64_t)c * d.ldc;
    if (d.c_double) {
      double* C = (double*)d.C;
      C[off] = d.alpha * v + (d.beta != 0.0 ? d.beta * C[off] : 0.0);
    } else {
      T* C = (T*)d.C;
      C[off] = (T)(d.alpha * v + (d.beta != 0.0 ? d.beta * (double)C[off] : 0.0));
    }
  }
}

// T: storage type of A and B; TC: MFMA type (T, or double for float inputs
// whose products must be accumulated in float64)
template <typename T, typename TC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmDesc<T> d, int tiles_m, int tiles_n,
                                                   int splits, int64_t chunks_per_r,
                                                   double* part) {
  typedef typename Acc<TC>::type acc_t;
  __shared__ TC As[TK][TM + PAD];
  __shared__ TC Bs[TK][TN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  int z, tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, d.sym, z, tm, tn);
  const int split = blockIdx.y;

  const int64_t total = (int64_t)d.R * chunks_per_r;
  const int64_t per = (total + splits - 1) / splits;
  const int64_t c_begin = (int64_t)split * per;
  const int64_t c_end = c_begin + per < total ? c_begin + per : total;

  acc_t acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  const T* Az = d.A + (int64_t)z * d.sAz;
  const T* Bz = d.B + (int64_t)z * d.sBz;
  const int row0 = tm * TM, col0 = tn * TN;

  for (int64_t c = c_begin; c < c_end; ++c) {
    const int64_t r = c / chunks_per_r;
    const int k0 = (int)((c % chunks_per_r) * TK);
    const T* Ar = Az + r * d.sAr;
    const T* Br = Bz + r * d.sBr;
    // stage op(A) tile (TM x TK) as As[k][i]
    if (!d.tA) {
      const int i = tid & 63;
      const int gi = row0 + i;
      for (int q = 0; q < 4; ++q) {
        const int k = (tid >> 6) + 4 * q;
        const int gk = k0 + k;
        TC v = 0;
        if (gi < d.M && gk < d.K) v = (TC)Ar[gi + (int64_t)gk * d.lda];
        As[k][i] = v;
      }
    } else {
      const int k = tid & 15;
      const int gk = k0 + k;
      for (int q = 0; q < 4; ++q) {
        const int i = (tid >> 4) + 16 * q;
        const int gi = row0 + i;
        TC v = 0;
        if (gi < d.M && gk < d.K) v = (TC)Ar[gk + (int64_t)gi * d.lda];
        As[k][i] = v;
      }
    }
    // stage op(B) tile (TK x TN) as Bs[k][j]
    if (!d.tB) {
      const int k = tid & 15;
      const int gk = k0 + k;
      for (int q = 0; q < 4; ++q) {
        const int j = (tid >> 4) + 16 * q;
        const int gj = col0 + j;
        TC v = 0;
        if (gj < d.N && gk < d.K) v = (TC)Br[gk + (int64_t)gj * d.ldb];
        Bs[k][j] = v;
      }
    } else {
      const int j = tid & 63;
      const int gj = col0 + j;
      for (int q = 0; q < 4; ++q) {
        const int k = (tid >> 6) + 4 * q;
        const int gk = k0 + k;
        TC v = 0;
        if (gj < d.N && gk < d.K) v = (TC)Br[gj + (int64_t)gk * d.ldb];
        Bs[k][j] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      TC a0 = As[kr][wr * 32 + (lane & 15)];
      TC a1 = As[kr][wr * 32 + 16 + (lane & 15)];
      TC b0 = Bs[kr][wc * 32 + (lane & 15)];
      TC b1 = Bs[kr][wc * 32 + 16 + (lane & 15)];
      // operands swapped (B fragment first): the MFMA then produces C^T
      // blocks whose lane index runs along C's contiguous row axis
      acc[0][0] = mfma_op(b0, a0, acc[0][0]);
      acc[0][1] = mfma_op(b1, a0, acc[0][1]);
      acc[1][0] = mfma_op(b0, a1, acc[1][0]);
      acc[1][1] = mfma_op(b1, a1, acc[1][1]);
    }
    __syncthreads();
  }

  // write out: block (bi, bj), register e -> row lane%16 and column
  // 4*(lane/16)+e for the f32 MFMA, lane/16 + 4*e for the f64 MFMA
  for (int bi = 0; bi < 2; ++bi)
    for (int bj = 0; bj < 2; ++bj)
      for (int e = 0; e < 4; ++e) {
        const int cloc = sizeof(TC) == 8 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
        const int gi = row0 + wr * 32 + bi * 16 + (lane & 15);
        const int gj = col0 + wc * 32 + bj * 16 + cloc;
        if (gi >= d.M || gj >= d.N) continue;
        put<T>(d, z, gi, gj, (double)acc[bi][bj][e], splits, split, part);
      }
}

// 128 x 128 tile, 4 waves of 64 x 64 (4 x 4 MFMA blocks each), depth-16
// chunks double-buffered in LDS with the next chunk prefetched into registers
// while the current one feeds the MFMAs.
constexpr int BT = 128, BPAD = 4;
template <typename T>
__global__ __launch_bounds__(256) void gemm_big_kernel(GemmDesc<T> d, int tiles_m, int tiles_n,
                                                       int splits, int64_t chunks_per_r,
                                                       double* part) {
  typedef typename Acc<T>::type acc_t;
  __shared__ T As[2][TK][BT + BPAD];
  __shared__ T Bs[2][TK][BT + BPAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  int z, tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, d.sym, z, tm, tn);
  const int split = blockIdx.y;
  const int64_t total = (int64_t)d.R * chunks_per_r;
  const int64_t per = (total + splits - 1) / splits;
  const int64_t c_begin = (int64_t)split * per;
  const int64_t c_end = c_begin + per < total ? c_begin + per : total;
  const T* Az = d.A + (int64_t)z * d.sAz;
  const T* Bz = d.B + (int64_t)z * d.sBz;
  const int row0 = tm * BT, col0 = tn * BT;

  acc_t acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  T ra[8], rb[8];
  auto load = [&](int64_t c) {
    const int64_t r = c / chunks_per_r;
    const int k0 = (int)((c % chunks_per_r) * TK);
    const T* Ar = Az + r * d.sAr;
    const T* Br = Bz + r * d.sBr;
    if (!d.tA) {
      const int i = tid & 127, gi = row0 + i;
      for (int q = 0; q < 8; ++q) {
        const int gk = k0 + (tid >> 7) + 2 * q;
        ra[q] = (gi < d.M && gk < d.K) ? Ar[gi + (int64_t)gk * d.lda] : (T)0;
      }
    } else {
      const int gk = k0 + (tid & 15);
      for (int q = 0; q < 8; ++q) {
        const int gi = row0 + (tid >> 4) + 16 * q;
        ra[q] = (gi < d.M && gk < d.K) ? Ar[gk + (int64_t)gi * d.lda] : (T)0;
      }
    }
    if (!d.tB) {
      const int gk = k0 + (tid & 15);
      for (int q = 0; q < 8; ++q) {
        const int gj = col0 + (tid >> 4) + 16 * q;
        rb[q] = (gj < d.N && gk < d.K) ? Br[gk + (int64_t)gj * d.ldb] : (T)0;
      }
    } else {
      const int j = tid & 127, gj = col0 + j;
      for (int q = 0; q < 8; ++q) {
        const int gk = k0 + (tid >> 7) + 2 * q;
        rb[q] = (gj < d.N && gk < d.K) ? Br[gj + (int64_t)gk * d.ldb] : (T)0;
      }
    }
  };
  auto store = [&](int buf) {
    if (!d.tA) {
      for (int q = 0; q < 8; ++q) As[buf][(tid >> 7) + 2 * q][tid & 127] = ra[q];
    } else {
      for (int q = 0; q < 8; ++q) As[buf][tid & 15][(tid >> 4) + 16 * q] = ra[q];
    }
    if (!d.tB) {
      for (int q = 0; q < 8; ++q) Bs[buf][tid & 15][(tid >> 4) + 16 * q] = rb[q];
    } else {
      for (int q = 0; q < 8; ++q) Bs[buf][(tid >> 7) + 2 * q][tid & 127] = rb[q];
    }
  };

  if (c_begin < c_end) {
    load(c_begin);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t c = c_begin; c < c_end; ++c) {
      const bool more = c + 1 < c_end;
      if (more) load(c + 1);
#pragma unroll
      for (int kk = 0; kk < TK / 4; ++kk) {
        const int kr = kk * 4 + (lane >> 4);
        T a[4], b[4];
        for (int i = 0; i < 4; ++i) a[i] = As[buf][kr][wr * 64 + i * 16 + (lane & 15)];
        for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kr][wc * 64 + j * 16 + (lane & 15)];
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) acc[i][j] = mfma_op(b[j], a[i], acc[i][j]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  for (int bi = 0; bi < 4; ++bi)
    for (int bj = 0; bj < 4; ++bj)
      for (int e = 0; e < 4; ++e) {
        const int cloc = sizeof(T) == 8 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
        const int gi = row0 + wr * 64 + bi * 16 + (lane & 15);
        const int gj = col0 + wc * 64 + bj * 16 + cloc;
        if (gi >= d.M || gj >= d.N) continue;
        put<T>(d, z, gi, gj, (double)acc[bi][bj][e], splits, split, part);
      }
}

template <typename T>
__global__ void gemm_reduce_kernel(GemmDesc<T> d, int splits, const double* part) {
  const int64_t mn = (int64_t)d.M * d.N;
  const int64_t total = mn * d.Z;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int z = (int)(idx / mn);
    const int64_t e = idx % mn;
    const int gi = (int)(e % d.M), gj = (int)(e / d.M);
    if (d.sym && gi > gj) continue;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += part[(((int64_t)k * d.Z + z) * d.N + gj) * d.M + gi];
    put<T>(d, z, gi, gj, s, 1, 0, nullptr);
  }
}

// Optional timing of every gemm_kernel launch with HIP events on the launch
// stream (process-wide), used to report the achieved MFMA rate.
constexpr int PROF_CAP = 4096;
struct GemmProfile {
  int on = 0;
  int n = 0;
  hipEvent_t ev[2 * PROF_CAP];
  double launches = 0, ms = 0, flops = 0, bytes = 0;
};
GemmProfile g_prof;

int prof_drain() {
  for (int i = 0; i < g_prof.n; ++i) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(g_prof.ev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
    if (e != hipSuccess) {
      set_hip_error(e, "gemm profile events");
      return -3;
    }
    g_prof.ms += t;
  }
  g_prof.n = 0;
  return 0;
}

}  // namespace

int gemm_profile(int enable) {
  if (enable && !g_prof.on) {
    for (int i = 0; i < 2 * PROF_CAP; ++i) HPT_HIP(hipEventCreate(&g_prof.ev[i]));
    g_prof.on = 1;
    g_prof.n = 0;
  } else if (!enable && g_prof.on) {
    int r = prof_drain();
    for (int i = 0; i < 2 * PROF_CAP; ++i) (void)hipEventDestroy(g_prof.ev[i]);
    g_prof.on = 0;
    if (r) return r;
  }
  g_prof.launches = g_prof.ms = g_prof.flops = g_prof.bytes = 0;
  return 0;
}

int gemm_profile_read(double* out4) {
  if (g_prof.on) {
    int r = prof_drain();
    if (r) return r;
  }
  out4[0] = g_prof.launches;
  out4[1] = g_prof.ms;
  out4[2] = g_prof.flops;
  out4[3] = g_prof.bytes;
  return 0;
}

template <typename T>
int gemm(const GemmDesc<T>& d, double* part, int64_t part_cap, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.Z <= 0) return 0;
  if (d.K <= 0 || d.R <= 0) return -1;  // callers never ask for an empty reduction
  // 64 x 64 tiles; HPT_GEMM_TILE=128 selects the 128 x 128 variant (tuning)
  static const int forced = [] {
    const char* e = getenv("HPT_GEMM_TILE");
    return e ? atoi(e) : 0;
  }();
  const bool big = !d.acc64 && forced == 128;
  const int tile = big ? BT : TM;
  const int tiles_m = (int)ceil_div(d.M, tile), tiles_n = (int)ceil_div(d.N, tile);
  if (d.sym && d.M != d.N) return -1;
  const int64_t tiles = (d.sym ? (int64_t)tiles_m * (tiles_m + 1) / 2 : (int64_t)tiles_m * tiles_n) * d.Z;
  const int64_t chunks_per_r = ceil_div(d.K, TK);
  const int64_t total = chunks_per_r * d.R;
  // split the reduction until the grid covers the chip several times over,
  // keeping at least 8 chunks of depth 16 per workgroup
  int splits = 1;
  const int64_t want = 2048;
  while (tiles * splits < want && total / (splits * 2) >= 8) splits *= 2;
  while (splits > 1 && (int64_t)splits * d.Z * d.M * d.N > part_cap) splits /= 2;
  dim3 grid((unsigned)tiles, (unsigned)splits);
  const bool prof = g_prof.on;
  if (prof) {
    if (g_prof.n == PROF_CAP) {
      const int r = prof_drain();
      if (r) return r;
    }
    HPT_HIP(hipEventRecord(g_prof.ev[2 * g_prof.n], s));
  }
  if (d.acc64 && sizeof(T) == 4)
    hipLaunchKernelGGL((gemm_kernel<T, double>), grid, dim3(256), 0, s, d, tiles_m, tiles_n, splits,
                       chunks_per_r, part);
  else if (big)
    hipLaunchKernelGGL(gemm_big_kernel<T>, grid, dim3(256), 0, s, d, tiles_m, tiles_n, splits,
                       chunks_per_r, part);
  else
    hipLaunchKernelGGL((gemm_kernel<T, T>), grid, dim3(256), 0, s, d, tiles_m, tiles_n, splits,
                       chunks_per_r, part);
  HPT_LAUNCH_CHECK("gemm_kernel");
  if (prof) {
    HPT_HIP(hipEventRecord(g_prof.ev[2 * g_prof.n + 1], s));
    g_prof.n++;
    g_prof.launches += 1;
    const double M = d.M, N = d.N, K = d.K, R = d.R, Z = d.Z;
    g_prof.flops += (d.sym ? 1.0 : 2.0) * M * N * K * R * Z;  // algorithmic: a SYRK does half
    const double za = d.sAz ? Z : 1.0, zb = d.sBz ? Z : 1.0;
    const double ra = d.sAr ? R : 1.0, rb = d.sBr ? R : 1.0;
    g_prof.bytes += sizeof(T) * (M * K * ra * za + K * N * rb * zb) +
                    (d.c_double ? 8.0 : (double)sizeof(T)) * M * N * Z;
  }
  if (splits > 1) {
    const int64_t n = (int64_t)d.M * d.N * d.Z;
    const int blocks = (int)(ceil_div(n, 256) < 65536 ? ceil_div(n, 256) : 65536);
    hipLaunchKernelGGL(gemm_reduce_kernel<T>, dim3(blocks), dim3(256), 0, s, d, splits, part);
    HPT_LAUNCH_CHECK("gemm_reduce_kernel");
  }
  return 0;
}

template int gemm<double>(const GemmDesc<double>&, double*, int64_t, hipStream_t);
template int gemm<float>(const GemmDesc<float>&, double*, int64_t, hipStream_t);

}  // namespace hpt
