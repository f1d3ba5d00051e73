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
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "tune.h"

namespace hpt {

#define RC_PROF(x) do { const int _r = (x); if (_r) return _r; } while (0)

namespace {

constexpr int TK = 16;

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

// Tile (2 WT) x (2 WT): four waves in a 2 x 2 grid, each owning WT x WT as
// (WT/16)^2 blocks of the 16x16x4 MFMA.  Depth-16 chunks of op(A) and op(B)
// are double-buffered in LDS; the next chunk is fetched into registers while
// the current one feeds the MFMAs, so global latency overlaps the math.
// T: storage type of A and B; TC: MFMA type (T, or double for float inputs
// whose products must be accumulated in float64).
template <typename T, typename TC, int WT>
__global__ __launch_bounds__(256) void gemm_pipe_kernel(GemmDesc<T> d, int tiles_m, int tiles_n,
                                                        int splits, int64_t chunks_per_r,
                                                        double* part) {
  typedef typename Acc<TC>::type acc_t;
  constexpr int BT = 2 * WT;           // tile side
  constexpr int NB = WT / 16;          // MFMA blocks per wave side
  constexpr int L = BT * TK / 256;     // elements per thread per operand
  constexpr int LP = 4;                // LDS row padding
  __shared__ TC As[2][TK][BT + LP];
  __shared__ TC Bs[2][TK][BT + LP];
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

  acc_t acc[NB][NB];
  for (int i = 0; i < NB; ++i)
    for (int j = 0; j < NB; ++j)
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0;

  // thread -> (row-or-col, k) coordinates of its L elements, per operand layout
  // contiguous-along-tile layout: x = tid % BT, k = tid / BT + (256 / BT) q
  // contiguous-along-k layout:    k = tid % 16, x = tid / 16 + 16 q
  TC ra[L], rb[L];
  auto load = [&](int64_t c) {
    const int64_t r = c / chunks_per_r;
    const int k0 = (int)((c % chunks_per_r) * TK);
    const T* Ar = Az + r * d.sAr;
    const T* Br = Bz + r * d.sBr;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      int i, k;
      if (!d.tA) { i = tid % BT; k = tid / BT + (256 / BT) * q; }
      else { k = tid & 15; i = (tid >> 4) + 16 * q; }
      const int gi = row0 + i, gk = k0 + k;
      ra[q] = (gi < d.M && gk < d.K) ? (TC)(d.tA ? Ar[gk + (int64_t)gi * d.lda] : Ar[gi + (int64_t)gk * d.lda]) : (TC)0;
    }
#pragma unroll
    for (int q = 0; q < L; ++q) {
      int j, k;
      if (d.tB) { j = tid % BT; k = tid / BT + (256 / BT) * q; }
      else { k = tid & 15; j = (tid >> 4) + 16 * q; }
      const int gj = col0 + j, gk = k0 + k;
      rb[q] = (gj < d.N && gk < d.K) ? (TC)(d.tB ? Br[gj + (int64_t)gk * d.ldb] : Br[gk + (int64_t)gj * d.ldb]) : (TC)0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < L; ++q) {
      if (!d.tA) As[buf][tid / BT + (256 / BT) * q][tid % BT] = ra[q];
      else As[buf][tid & 15][(tid >> 4) + 16 * q] = ra[q];
      if (d.tB) Bs[buf][tid / BT + (256 / BT) * q][tid % BT] = rb[q];
      else Bs[buf][tid & 15][(tid >> 4) + 16 * q] = rb[q];
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
        TC a[NB], b[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) a[i] = As[buf][kr][wr * WT + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < NB; ++j) b[j] = Bs[buf][kr][wc * WT + j * 16 + (lane & 15)];
        // operands swapped (B fragment first): the MFMA yields C^T blocks whose
        // lane index runs along C's contiguous row axis
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = mfma_op(b[j], a[i], acc[i][j]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // register e of block (bi, bj) -> row lane%16, column 4*(lane/16)+e for the
  // f32 MFMA and lane/16 + 4*e for the f64 MFMA
  for (int bi = 0; bi < NB; ++bi)
    for (int bj = 0; bj < NB; ++bj)
      for (int e = 0; e < 4; ++e) {
        const int cloc = sizeof(TC) == 8 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
        const int gi = row0 + wr * WT + bi * 16 + (lane & 15);
        const int gj = col0 + wc * WT + bj * 16 + cloc;
        if (gi >= d.M || gj >= d.N) continue;
        put<T>(d, z, gi, gj, (double)acc[bi][bj][e], splits, split, part);
      }
}

// ---------------------------------------------------------------------------
// Gram G = X^T X of a float32 matrix X (m x n, column-major, leading dimension
// ldx) with float64 products and sums (the Gram that feeds CholeskyQR2 in the
// float32 form).  Upper-triangular 64 x 64 tiles, four waves of 2 x 2 f64
// 16x16x4 MFMA blocks each; depth-16 chunks of rows of X are fetched as one
// float4 per thread (128-byte column segments per 8 lanes), kept as float in
// double-buffered LDS rows of stride 80 (16 mod 64 banks: the four k-rows an
// MFMA operand read touches land on disjoint banks) and widened to double on
// the way into the MFMA.  A diagonal tile reads its column block once and uses
// it for both operands.  16 x 16 blocks that lie past n or strictly below the
// diagonal issue no MFMA.  The rows of X are split over the grid; every
// split writes its partial tile (upper blocks) for a fixed-order reduction.
constexpr int G64_TK = 16, G64_SP = 80;

template <bool VEC>
__device__ inline float4 g64_load(const float* p, bool valid, bool full, int rem) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (!valid) return v;
  if (VEC && full) return *(const float4*)p;
  if (full || rem > 0) v.x = p[0];
  if (full || rem > 1) v.y = p[1];
  if (full || rem > 2) v.z = p[2];
  if (full || rem > 3) v.w = p[3];
  return v;
}

// VEC: ldx % 4 == 0 and X 16-byte aligned (float4 loads of whole chunks)
template <bool VEC>
__global__ __launch_bounds__(256) void gram64_kernel(const float* __restrict__ X, int64_t ldx, int m, int n,
                                                     int tiles, int splits, int chunks, double* __restrict__ part) {
  constexpr int BT = 64, TK = G64_TK, SP = G64_SP;
  constexpr int KQ = TK / 4, CPP = 256 / KQ;   // 4 threads per column, all 64 columns in one pass
  static_assert(CPP == BT, "one float4 per thread and operand");
  __shared__ float As[2][TK][SP];
  __shared__ float Bs[2][TK][SP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wr = wave >> 1, wc = wave & 1;
  // workgroup -> (tile, row split).  Workgroups go to the XCDs round-robin
  // (id mod 8); with splits a multiple of 8 every tile of one split runs on
  // the same XCD, one split after another, so the column blocks of X that
  // the tiles of a split share are fetched into that XCD's L2 once.
  const int L = blockIdx.x;
  int t, split;
  if (splits % 8 == 0) {
    const int j = L / 8;
    t = j % tiles;
    split = (j / tiles) * 8 + L % 8;
  } else {
    t = L % tiles;
    split = L / tiles;
  }
  // upper-triangular tile (tm <= tn), column by column
  int tn = 0;
  while (t > tn) { t -= tn + 1; ++tn; }
  const int tm = t;
  const bool diag = tm == tn;
  const int row0 = tm * BT, col0 = tn * BT;
  // 16-row blocks of G this wave computes: inside n and on or above the diagonal
  const int nb = (n + 15) / 16;
  bool run[2][2];
  bool active = false;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int rb = (row0 + wr * 32) / 16 + i, cb = (col0 + wc * 32) / 16 + j;
      run[i][j] = rb < nb && cb < nb && rb <= cb;
      active = active || run[i][j];
    }
  const int per = (chunks + splits - 1) / splits;
  const int c_begin = split * per;
  const int c_end = c_begin + per < chunks ? c_begin + per : chunks;
  const int kq = tid % KQ, cl = tid / KQ;
  const bool va = row0 + cl < n, vb = col0 + cl < n;
  const float* pa = X + (int64_t)(va ? row0 + cl : 0) * ldx + 4 * kq;
  const float* pb = X + (int64_t)(vb ? col0 + cl : 0) * ldx + 4 * kq;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = 0.0;
  float4 ra, rb;
  auto load = [&](int c) {
    const int k0 = c * TK;
    const bool full = k0 + TK <= m;
    const int rem = m - k0 - 4 * kq;
    ra = g64_load<VEC>(pa + k0, va, full, rem);
    if (!diag) rb = g64_load<VEC>(pb + k0, vb, full, rem);
  };
  auto store = [&](int buf) {
    As[buf][4 * kq + 0][cl] = ra.x; As[buf][4 * kq + 1][cl] = ra.y;
    As[buf][4 * kq + 2][cl] = ra.z; As[buf][4 * kq + 3][cl] = ra.w;
    if (!diag) {
      Bs[buf][4 * kq + 0][cl] = rb.x; Bs[buf][4 * kq + 1][cl] = rb.y;
      Bs[buf][4 * kq + 2][cl] = rb.z; Bs[buf][4 * kq + 3][cl] = rb.w;
    }
  };
  if (c_begin < c_end) {
    load(c_begin);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int c = c_begin; c < c_end; ++c) {
      const bool more = c + 1 < c_end;
      if (more) load(c + 1);
      if (active) {
        const float (*Bsrc)[SP] = diag ? As[buf] : Bs[buf];
#pragma unroll
        for (int kk = 0; kk < TK / 4; ++kk) {
          const int kr = kk * 4 + (lane >> 4);
          double a[2], b[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) a[i] = (double)As[buf][kr][wr * 32 + i * 16 + (lane & 15)];
#pragma unroll
          for (int j = 0; j < 2; ++j) b[j] = (double)Bsrc[kr][wc * 32 + j * 16 + (lane & 15)];
          // B fragment first: register e of block (i, j) is G[row lane%16, col lane/16 + 4 e]
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              if (run[i][j]) acc[i][j] = mfma_op(b[j], a[i], acc[i][j]);
        }
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  if (!active) return;
  double* out = part + (int64_t)split * n * n;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = row0 + wr * 32 + i * 16 + (lane & 15);
        const int gj = col0 + wc * 32 + j * 16 + (lane >> 4) + 4 * e;
        if (run[i][j] && gi < n && gj < n && gi <= gj) out[(int64_t)gj * n + gi] = acc[i][j][e];
      }
}

// ---------------------------------------------------------------------------
// Plain products C = A B for float32 A (M x K) and B (K x N), column-major,
// float32 C, in 128 x 80 tiles, in float32 or in split-bf16 form.
// Split-bf16: every operand element x is split to nearest into three bf16
// parts, x = h + m + l (h = bf16(x), m = bf16(x - h), l = x - h - m, which
// has at most 8 significant bits and is exact in bf16).  The product keeps
// the six terms down to relative order 2^-16, hh + hm + mh + mm + hl + lh;
// the dropped ml + lm + ll are below 2^-23 of |a b|, so the result carries
// float32-level error at the bf16 MFMA rate (gfx950 v_mfma_f32_16x16x32_bf16,
// 8 k-values per lane and operand).  Tile 128 x 80: four waves of 32 rows x
// 80 columns (2 x 5 blocks of 16 x 16), k-chunks of 32 split while staged
// into LDS (three bf16 planes per operand, rows of 80 bytes: 16-lane
// ds_read_b128 groups hit distinct banks).  Operands go into the MFMA with B
// first, so the 16 lanes of a result register run along C's rows.  The tiles
// of one XCD (workgroup id mod 8) form a contiguous range, the column tiles
// of a row strip adjacent, so a strip of A is fetched from HBM once.
constexpr int BS_BM = 128, BS_BN = 80, BS_KC = 32, BS_RS = 40;   // BS_RS: LDS row stride in bf16

__device__ inline void bsplit3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r = x - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

__device__ inline void bsplit_put(const float* v, __bf16* h0, __bf16* m0, __bf16* l0) {
  bf8 h, m, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    __bf16 a, b, c;
    bsplit3(v[e], a, b, c);
    h[e] = a; m[e] = b; l[e] = c;
  }
  *(bf8*)h0 = h;
  *(bf8*)m0 = m;
  *(bf8*)l0 = l;
}

// SPLIT = false: the same tiling in plain float32 (f32 16x16x4 MFMA, operands
// as floats in LDS rows of 36: the 16 rows x 4 k-values of an operand read
// fall on 64 distinct banks), the FP32 form's plain products.
constexpr int BS_RS32 = 36;

template <bool SPLIT>
__global__ __launch_bounds__(256) void tile_gemm_kernel(const float* __restrict__ A, int64_t lda,
                                                        const float* __restrict__ B, int64_t ldb,
                                                        float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                        int ntn, int64_t total, int64_t per_xcd) {
  constexpr int BM = BS_BM, BN = BS_BN, KC = BS_KC, RS = BS_RS, RS32 = BS_RS32;
  constexpr int LDS_BYTES = SPLIT ? 3 * (BM + BN) * RS * 2 : (BM + BN) * RS32 * 4;
  __shared__ __attribute__((aligned(16))) char smem[LDS_BYTES];
  __bf16* Ah = (__bf16*)smem;                 // split: planes h, m, l of A, then of B
  __bf16* Bh = Ah + 3 * BM * RS;
  float* Af = (float*)smem;                   // float32: A rows, then B columns
  float* Bf = Af + BM * RS32;
  const int64_t T = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (T >= total) return;
  const int row0 = (int)(T / ntn) * BM, col0 = (int)(T % ntn) * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // A staging: row ar of the tile, k-groups (8 k each) akg and akg + 2
  const int ar = tid & 127, akg = tid >> 7;
  const bool a_ok = row0 + ar < M;
  const float* Ap = A + (a_ok ? row0 + ar : 0);
  // B staging: units tid and tid + 256 (< 320) = (column u % 80, k-group u / 80)
  const int u1 = tid + 256;
  const bool u1_ok = u1 < BN * 4;
  const int bc0 = tid % BN, bk0 = tid / BN, bc1 = u1 % BN, bk1 = u1 / BN;
  const bool b0_ok = col0 + bc0 < N, b1_ok = u1_ok && col0 + bc1 < N;
  const float* Bp0 = B + (int64_t)(b0_ok ? col0 + bc0 : 0) * ldb;
  const float* Bp1 = B + (int64_t)(b1_ok ? col0 + bc1 : 0) * ldb;
  float ra[16], rb[16];
  auto load = [&](int k0) {
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * (akg + 2 * g) + e;
        ra[8 * g + e] = (a_ok && k < K) ? Ap[(int64_t)k * lda] : 0.f;
      }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k0e = k0 + 8 * bk0 + e, k1e = k0 + 8 * bk1 + e;
      rb[e] = (b0_ok && k0e < K) ? Bp0[k0e] : 0.f;
      rb[8 + e] = (b1_ok && k1e < K) ? Bp1[k1e] : 0.f;
    }
  };
  auto put8 = [&](const float* v, float* d) {
    *(float4*)d = make_float4(v[0], v[1], v[2], v[3]);
    *(float4*)(d + 4) = make_float4(v[4], v[5], v[6], v[7]);
  };
  f4 acc[2][5];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = (K + KC - 1) / KC;
  load(0);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();   // every wave is done reading the previous chunk
    if constexpr (SPLIT) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int off = ar * RS + 8 * (akg + 2 * g);
        bsplit_put(ra + 8 * g, Ah + off, Ah + BM * RS + off, Ah + 2 * BM * RS + off);
      }
      {
        const int off = bc0 * RS + 8 * bk0;
        bsplit_put(rb, Bh + off, Bh + BN * RS + off, Bh + 2 * BN * RS + off);
      }
      if (u1_ok) {
        const int off = bc1 * RS + 8 * bk1;
        bsplit_put(rb + 8, Bh + off, Bh + BN * RS + off, Bh + 2 * BN * RS + off);
      }
    } else {
#pragma unroll
      for (int g = 0; g < 2; ++g) put8(ra + 8 * g, Af + ar * RS32 + 8 * (akg + 2 * g));
      put8(rb, Bf + bc0 * RS32 + 8 * bk0);
      if (u1_ok) put8(rb + 8, Bf + bc1 * RS32 + 8 * bk1);
    }
    __syncthreads();
    if (c + 1 < nchunks) load((c + 1) * KC);
    if constexpr (SPLIT) {
      bf8 af[2][3];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int p = 0; p < 3; ++p)
          af[i][p] = *(const bf8*)(Ah + p * BM * RS + (32 * w + 16 * i + (lane & 15)) * RS + 8 * (lane >> 4));
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        bf8 bf[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) bf[p] = *(const bf8*)(Bh + p * BN * RS + (16 * j + (lane & 15)) * RS + 8 * (lane >> 4));
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          // the six products of this k-chunk, smallest terms first, start from
          // zero and join the running sum in one rounded float32 add: the sum
          // over K is not carried through the MFMA accumulator (measured: 4x
          // smaller worst-case error on sums of positive terms)
          f4 a = {0.f, 0.f, 0.f, 0.f};
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[0], af[i][2], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[2], af[i][0], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[1], af[i][1], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[0], af[i][1], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[1], af[i][0], a, 0, 0, 0);
          a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[0], af[i][0], a, 0, 0, 0);
          acc[i][j] += a;
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        const int ko = 4 * kk + (lane >> 4);
        float af[2], bf[5];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = Af[(32 * w + 16 * i + (lane & 15)) * RS32 + ko];
#pragma unroll
        for (int j = 0; j < 5; ++j) bf[j] = Bf[(16 * j + (lane & 15)) * RS32 + ko];
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
          for (int i = 0; i < 2; ++i) acc[i][j] = mfma_op(bf[j], af[i], acc[i][j]);
      }
    }
  }
  // register e of block (i, j): C[row 32 w + 16 i + lane % 16, column 16 j + 4 (lane / 16) + e]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = row0 + 32 * w + 16 * i + (lane & 15), cc = col0 + 16 * j + 4 * (lane >> 4) + e;
        if (r < M && cc < N) C[r + (int64_t)cc * ldc] = acc[i][j][e];
      }
}

// ---------------------------------------------------------------------------
// Plain float32 products C = A B (A M x K, B K x N, column-major) in the same
// 128 x 80 XCD-ordered tiles, f32 16x16x4 MFMA, k-chunks of 32.  Staging:
// A as float4 along rows (thread: 4 rows, k = kr + 8 g for g = 0..3), kept in
// LDS as k-rows of 144 floats (row-contiguous; 144 = 16 mod 64, so the four
// k-rows of an operand read use disjoint banks); B as float4 along k (eight
// threads per 32-k column segment), kept as columns of 36 floats.  Interior
// tiles and whole k-chunks of aligned operands take branch-free 16-byte
// loads; edge tiles and the last partial chunk take guarded element loads
// into the same layout.  The next chunk is fetched into registers while the
// current one feeds the MFMAs.
constexpr int F_SA = 144, F_SB = 36;

__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ B, int64_t ldb,
                                                       float* __restrict__ C, int64_t ldc, int M, int N, int K,
                                                       int ntn, int64_t total, int64_t per_xcd, int avec,
                                                       int bvec) {
  constexpr int BM = BS_BM, BN = BS_BN, KC = BS_KC, SA = F_SA, SB = F_SB;
  __shared__ __attribute__((aligned(16))) float As[KC * SA];
  __shared__ __attribute__((aligned(16))) float Bs[BN * SB];
  const int64_t T = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (T >= total) return;
  const int row0 = (int)(T / ntn) * BM, col0 = (int)(T % ntn) * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = tid & 31, kr = tid >> 5;   // A: rows 4q..4q+3, k-rows kr + 8 g
  const bool a_full = avec && row0 + BM <= M;
  const bool b_full = bvec && col0 + BN <= N;
  constexpr int NBU = BN * (KC / 4);       // B float4 units per chunk (640)
  float4 ra[4], rb[3];
  auto load = [&](int k0) {
    const bool kfull = k0 + KC <= K;
    if (a_full && kfull) {
      const float* ap = A + row0 + 4 * q + (int64_t)(k0 + kr) * lda;
#pragma unroll
      for (int g = 0; g < 4; ++g) ra[g] = *(const float4*)(ap + (int64_t)(8 * g) * lda);
    } else {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int k = k0 + kr + 8 * g;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = row0 + 4 * q + e;
          v[e] = (r < M && k < K) ? A[r + (int64_t)k * lda] : 0.f;
        }
        ra[g] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int u = tid + 256 * t;
      if (u >= NBU) break;
      const int c = col0 + (u >> 3), k = k0 + 4 * (u & 7);
      if (b_full && kfull) {
        rb[t] = *(const float4*)(B + k + (int64_t)c * ldb);
      } else {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (c < N && k + e < K) ? B[k + e + (int64_t)c * ldb] : 0.f;
        rb[t] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  };
  f4 acc[2][5];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = (K + KC - 1) / KC;
  load(0);
  for (int ch = 0; ch < nchunks; ++ch) {
    __syncthreads();   // every wave is done reading the previous chunk
#pragma unroll
    for (int g = 0; g < 4; ++g) *(float4*)(As + (kr + 8 * g) * SA + 4 * q) = ra[g];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int u = tid + 256 * t;
      if (u < NBU) *(float4*)(Bs + (u >> 3) * SB + 4 * (u & 7)) = rb[t];
    }
    __syncthreads();
    if (ch + 1 < nchunks) load((ch + 1) * KC);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int ko = 4 * kk + (lane >> 4);
      float af[2], bf[5];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[ko * SA + 32 * w + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 5; ++j) bf[j] = Bs[(16 * j + (lane & 15)) * SB + ko];
#pragma unroll
      for (int j = 0; j < 5; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][j] = mfma_op(bf[j], af[i], acc[i][j]);
    }
  }
  // register e of block (i, j): C[row 32 w + 16 i + lane % 16, column 16 j + 4 (lane / 16) + e]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = row0 + 32 * w + 16 * i + (lane & 15), cc = col0 + 16 * j + 4 * (lane >> 4) + e;
        if (r < M && cc < N) C[r + (int64_t)cc * ldc] = acc[i][j][e];
      }
}

// ---------------------------------------------------------------------------
// Mode products of the float32 form with the n x n factor resident in LDS
// (n <= 128), persistent workgroups of 4 waves, each wave streaming 16-row
// (or 16-column) strips of the tensor straight from HBM into MFMA operands.
// Padding of the LDS rows keeps the 64-lane operand reads free of bank
// conflicts.

// dst_z[a, j] = sum_k src_z[a, k] S[j, k]; src_z, dst_z inner x n (a fastest).
// A wave takes 16-row strips in turn and fetches the next strip's operands
// into registers while the MFMAs of the current one run.  The factor goes
// first into the MFMA, so result blocks are dst^T and the stores of 16 lanes
// run along a.
template <int NP, int KS>
__global__ __launch_bounds__(256) void mode_product_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                           const float* __restrict__ S, int n, int64_t inner,
                                                           int64_t Z, int64_t strips_per_z) {
  constexpr int NB = NP / 16;   // KS = ceil(n / 4) k-steps of 4 (<= NP / 4)
  constexpr int SP = NP + ((NP % 32) == 0 ? 16 : 0);   // row stride = 16 mod 32
  __shared__ float Sl[NP * SP];                         // Sl[k * SP + j] = S[j, k]
  for (int idx = threadIdx.x; idx < NP * NP; idx += blockDim.x) {
    const int j = idx % NP, k = idx / NP;
    Sl[k * SP + j] = (j < n && k < n) ? S[j + (int64_t)k * n] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t total = strips_per_z * Z;
  float y[KS], yn[KS];
  // 32-bit byte offsets inside one slice (inner * n < 2^30 is checked by
  // the launcher).  Rows past the end and k >= n read clamped, in-range
  // entries instead of being masked: rows past the end are never stored, and
  // the factor's rows k >= n are zero in LDS.
  auto fetch = [&](int64_t st, float* v) {
    const int64_t z = st / strips_per_z;
    const int64_t r = (st % strips_per_z) * 16 + r16;
    const uint32_t row = (uint32_t)(r < inner ? r : inner - 1);
    const char* base = (const char*)(src + z * inner * n);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const uint32_t k = (uint32_t)min(ks * 4 + kq, n - 1);
      // byte offset within the slice fits 32 bits: scalar base + vector offset
      v[ks] = *(const float*)(base + (row + k * (uint32_t)inner) * 4u);
    }
  };
  // the strip index is wave-uniform: keep it (and every base address) scalar
  int64_t st = blockIdx.x * (int64_t)(blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (st < total) fetch(st, y);
  for (; st < total; st += nwaves) {
    const int64_t nx = st + nwaves;
    if (nx < total) fetch(nx, yn);
    f4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = f4{0.f, 0.f, 0.f, 0.f};
    // an opaque zero keeps the factor reads inside the loop (hoisting all of
    // them out of the strip loop would need NP^2/16 registers per lane)
    int opq = 0;
    asm volatile("" : "+v"(opq));
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float* Sk = Sl + opq + (ks * 4 + kq) * SP + r16;
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Sk[cb * 16], y[ks], acc[cb], 0, 0, 0);
    }
    // block cb, register e: row a0 + r16, column 16 cb + 4 kq + e
    const int64_t z = st / strips_per_z;
    const int64_t row = (st % strips_per_z) * 16 + r16;
    if (row < inner) {
      float* Cz = dst + z * inner * n + row;
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int col = cb * 16 + 4 * kq + e;
          if (col < n) Cz[(int64_t)col * inner] = acc[cb][e];
        }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) y[ks] = yn[ks];
  }
}

// The same product in 32-row strips for even inner: lane (r16, kq) reads rows
// 2 r16 and 2 r16 + 1 of the strip as one float2 per k and feeds them to two
// MFMAs that share the factor operand, so block h of the result holds rows
// 2 r16 + h and the float2 stores of 16 lanes cover 128 contiguous bytes of a
// column (the 16-row form moves 64-byte pieces); half the load and factor
// read instructions per MFMA.  The factor is staged so that the NB <= 8
// values a lane needs at one k (rows j = 16 cb + r16) are two 16-byte LDS
// reads: Sl[k][h][r][c] = S[16 (4 h + c) + r, k] (each read of 16 lanes
// covers 256 contiguous bytes), only the 4 KS rows k the strip loop uses.
// Every output element sees the same MFMA operands in the same k order as in
// the 16-row form.
template <int NP, int KS>
__global__ __launch_bounds__(256, 3) void mode_product32_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                             const float* __restrict__ S, int n, int64_t inner,
                                                             int64_t Z, int64_t strips_per_z) {
  constexpr int NB = NP / 16;
  static_assert(NB <= 8, "two 16-byte factor reads per k");
  __shared__ float Sl[KS * 4 * 128];
  for (int idx = threadIdx.x; idx < KS * 4 * 128; idx += blockDim.x) {
    const int k = idx >> 7, cb = ((idx >> 6) & 1) * 4 + (idx & 3), r = (idx >> 2) & 15;
    const int j = cb * 16 + r;
    Sl[idx] = (cb < NB && j < n && k < n) ? S[j + (int64_t)k * n] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t total = strips_per_z * Z;
  float2 y[KS];
  // rows past the end read the clamped, in-range pair inner - 2, inner - 1
  // (never stored); k >= n read k = n - 1 (the factor's rows k >= n are zero)
  // opk is an opaque zero made inside the strip loop: without it the 25
  // loop-invariant row offsets k inner are hoisted out of the loop and held in
  // registers (spilled at three waves per SIMD)
  auto fetch = [&](int64_t st, float2* v, int opk) {
    const int64_t z = st / strips_per_z;
    const int64_t r = (st % strips_per_z) * 32 + 2 * r16;
    const uint32_t row = (uint32_t)(r < inner ? r : inner - 2);
    const char* base = (const char*)(src + z * inner * n);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const uint32_t k = (uint32_t)min(ks * 4 + kq + opk, n - 1);
      v[ks] = *(const float2*)(base + (row + k * (uint32_t)inner) * 4u);
    }
  };
  // no prefetch of the next strip (it would not fit the registers): a strip is
  // 350 MFMAs per wave, and the other waves of the SIMD cover its load latency
  int64_t st = blockIdx.x * (int64_t)(blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (; st < total; st += nwaves) {
    int opk = 0;
    asm volatile("" : "+v"(opk));
    fetch(st, y, opk);
    f4 acc0[NB], acc1[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      acc0[cb] = f4{0.f, 0.f, 0.f, 0.f};
      acc1[cb] = f4{0.f, 0.f, 0.f, 0.f};
    }
    int opq = 0;  // keeps the factor reads inside the strip loop
    asm volatile("" : "+v"(opq));
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const float* Sk = Sl + opq + (ks * 4 + kq) * 128 + 4 * r16;
      const f4 lo = *(const f4*)Sk;
      const f4 hi = NB > 4 ? *(const f4*)(Sk + 64) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const float a = cb < 4 ? lo[cb & 3] : hi[cb & 3];
        acc0[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, y[ks].x, acc0[cb], 0, 0, 0);
        acc1[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, y[ks].y, acc1[cb], 0, 0, 0);
      }
    }
    const int64_t z = st / strips_per_z;
    const int64_t row = (st % strips_per_z) * 32 + 2 * r16;
    if (row < inner) {
      char* Cz = (char*)(dst + z * inner * n);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t col = (uint32_t)(cb * 16 + 4 * kq + e + opk);
          if (col < (uint32_t)n)
            *(float2*)(Cz + ((uint32_t)row + col * (uint32_t)inner) * 4u) = make_float2(acc0[cb][e], acc1[cb][e]);
        }
    }
  }
}

// dst[j, b] = sum_k S[j, k] src[k, b]; src, dst n x outer (the leading leg).
// Each lane reads 4 consecutive k of one column (one 16-byte load when
// n % 4 == 0); the MFMA's reduction index is permuted accordingly (lane
// group kq supplies k = 16 kb + 4 kq + t at step t, and reads the same k of
// the factor), and the result blocks are dst^T, so stores run along j.
// 16-column strips, next strip fetched during the current one's MFMAs.  The
// factor sits in dynamic LDS as rows of 128 floats, Sl[k][h][r][c] =
// S[16 (4 h + c) + r, k] for k < n and one zero row k = n that every k >= n
// reads: the NB <= 8 values a lane needs at one k are two 16-byte reads.
template <int NP, bool VEC>
__global__ __launch_bounds__(256) void mode_product_lead_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                                const float* __restrict__ S, int n, int64_t outer) {
  constexpr int NB = NP / 16, KB = NP / 16;
  static_assert(NB <= 8, "two 16-byte factor reads per k");
  extern __shared__ float Sl[];
  const int rows = n < NP ? n + 1 : NP;
  for (int idx = threadIdx.x; idx < rows * 128; idx += blockDim.x) {
    const int k = idx >> 7, cb = ((idx >> 6) & 1) * 4 + (idx & 3), r = (idx >> 2) & 15;
    const int j = cb * 16 + r;
    Sl[idx] = (cb < NB && j < n && k < n) ? S[j + (int64_t)k * n] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t total = ceil_div(outer, 16);
  f4 x[KB], xn[KB];
  auto fetch = [&](int64_t st, f4* v) {
    const int64_t col = st * 16 + r16;
    const float* p = src + col * n + 4 * kq;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = kb * 16 + 4 * kq;
      f4 w{0.f, 0.f, 0.f, 0.f};
      if (col < outer) {
        if (VEC) {
          if (k < n) w = *(const f4*)(p + kb * 16);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (k + t < n) w[t] = p[kb * 16 + t];
        }
      }
      v[kb] = w;
    }
  };
  int64_t st = blockIdx.x * (int64_t)(blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (st < total) fetch(st, x);
  for (; st < total; st += nwaves) {
    const int64_t nx = st + nwaves;
    if (nx < total) fetch(nx, xn);
    f4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = f4{0.f, 0.f, 0.f, 0.f};
    int opq = 0;  // keeps the factor reads inside the strip loop
    asm volatile("" : "+v"(opq));
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float* Sk = Sl + min(kb * 16 + 4 * kq + t + opq, n) * 128 + 4 * r16;
        const f4 lo = *(const f4*)Sk;
        const f4 hi = NB > 4 ? *(const f4*)(Sk + 64) : f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[kb][t], cb < 4 ? lo[cb & 3] : hi[cb & 3], acc[cb], 0, 0, 0);
      }
    // block cb, register e: dst[16 cb + r16, b0 + 4 kq + e]
    const int64_t b0 = st * 16;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int j = cb * 16 + r16;
      if (j >= n) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t col = b0 + 4 * kq + e;
        if (col < outer) dst[j + col * n] = acc[cb][e];
      }
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) x[kb] = xn[kb];
  }
}

// Leg Gram of the float32 form: out[i, j] = sum over every other index of
// psi[.., i, ..] cur[.., j, ..] (n <= 128).  Each workgroup reduces a range
// of depth-16 chunks into the whole padded n x n block (four waves, 2 x 2
// quadrants of 16 x 16 MFMA blocks) and writes a float64 partial; a second
// pass sums the partials in a fixed order.  Chunk c covers 16 consecutive a
// of slice r (a fastest, stride 1: 16-byte loads of 4 a per lane), or, for
// the leading leg (inner == 1), 16 consecutive b with i fastest.  The MFMA's
// reduction index is permuted consistently on both operands.
template <int NP, bool LEAD, bool VEC>
__global__ __launch_bounds__(256) void leg_gram_kernel(const float* __restrict__ psi, const float* __restrict__ cur,
                                                       int n, int64_t inner, int64_t outer, int64_t chunks_per_r,
                                                       int64_t chunks_per_wg, double* __restrict__ part) {
  constexpr int NB = NP / 16, HB = (NB + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r16 = lane & 15, kq = lane >> 4;
  const int ib0 = (wave >> 1) * HB, jb0 = (wave & 1) * HB;
  f4 acc[HB][HB];
#pragma unroll
  for (int x = 0; x < HB; ++x)
#pragma unroll
    for (int y = 0; y < HB; ++y) acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t total = (LEAD ? 1 : outer) * chunks_per_r;
  const int64_t c0 = blockIdx.x * chunks_per_wg;
  const int64_t c1 = c0 + chunks_per_wg < total ? c0 + chunks_per_wg : total;
  auto load = [&](const float* T, int64_t c, int col) -> f4 {
    f4 v{0.f, 0.f, 0.f, 0.f};
    if (col >= n) return v;
    if (LEAD) {
      // k = 4 t + kq at step t: T[col, b0 + 4 t + kq], T is n x outer
      const int64_t b0 = c * 16 + kq;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (b0 + 4 * t < outer) v[t] = T[col + (b0 + 4 * t) * n];
    } else {
      // k = 4 kq + t at step t: T[a0 + 4 kq + t, col, r], T is inner x n x outer
      const int64_t r = c / chunks_per_r;
      const int64_t a = (c % chunks_per_r) * 16 + 4 * kq;
      const float* p = T + (r * n + col) * inner + a;
      if (VEC) {
        if (a < inner) v = *(const f4*)p;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (a + t < inner) v[t] = p[t];
      }
    }
    return v;
  };
  f4 xa[HB], yb[HB], xn[HB], yn[HB];
  if (c0 < c1) {
#pragma unroll
    for (int x = 0; x < HB; ++x) xa[x] = load(psi, c0, (ib0 + x) * 16 + r16);
#pragma unroll
    for (int y = 0; y < HB; ++y) yb[y] = load(cur, c0, (jb0 + y) * 16 + r16);
  }
  for (int64_t c = c0; c < c1; ++c) {
    // the next chunk's operands are in flight during this chunk's MFMAs
    if (c + 1 < c1) {
#pragma unroll
      for (int x = 0; x < HB; ++x) xn[x] = load(psi, c + 1, (ib0 + x) * 16 + r16);
#pragma unroll
      for (int y = 0; y < HB; ++y) yn[y] = load(cur, c + 1, (jb0 + y) * 16 + r16);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int x = 0; x < HB; ++x) {
        if (ib0 + x >= NB) continue;
#pragma unroll
        for (int y = 0; y < HB; ++y) {
          if (jb0 + y >= NB) continue;
          // cur first: the block is out^T, so lanes run along i
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(yb[y][t], xa[x][t], acc[x][y], 0, 0, 0);
        }
      }
#pragma unroll
    for (int x = 0; x < HB; ++x) xa[x] = xn[x];
#pragma unroll
    for (int y = 0; y < HB; ++y) yb[y] = yn[y];
  }
  // block (x, y), register e: out[16 (ib0 + x) + r16, 16 (jb0 + y) + 4 kq + e]
  double* out = part + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int x = 0; x < HB; ++x)
#pragma unroll
    for (int y = 0; y < HB; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = (ib0 + x) * 16 + r16, j = (jb0 + y) * 16 + 4 * kq + e;
        if (ib0 + x < NB && jb0 + y < NB && i < n && j < n) out[(int64_t)j * n + i] = (double)acc[x][y][e];
      }
}

// Leg Gram of the float32 form for inner > 1, inner % 4 == 0: the reduction
// index k = a + inner r is flattened over (a, r); chunks of 32 consecutive k
// of all n columns of both operands are fetched with 16-byte loads (8 lanes
// cover 128 contiguous bytes of one column), staged in LDS as [k][column],
// and fed to the MFMAs (four waves, 2 x 2 quadrants of 16 x 16 blocks of the
// padded n x n result).  The next chunk is fetched during this chunk's MFMAs.
template <int NP>
__global__ __launch_bounds__(256) void leg_gram_lds_kernel(const float* __restrict__ psi, const float* __restrict__ cur,
                                                           int n, uint32_t inner, uint32_t ktotal,
                                                           uint32_t chunks_per_wg, double* __restrict__ part) {
  constexpr int NB = NP / 16, HB = (NB + 1) / 2;
  constexpr int KC = 32;
  constexpr int SP = NP + 4;
  constexpr int PASSES = (NP + 31) / 32;
  __shared__ float As[KC * SP];   // As[k * SP + col]
  __shared__ float Bs[KC * SP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  const int ib0 = (wave >> 1) * HB, jb0 = (wave & 1) * HB;
  const int kg = tid & 7, cl = tid >> 3;
  f4 ra[PASSES], rb[PASSES];
  auto gload = [&](uint32_t c) {
    const uint32_t k = c * KC + 4 * kg;
    const bool kok = k < ktotal;
    const uint32_t r = kok ? k / inner : 0u;
    const uint32_t a = kok ? k - r * inner : 0u;
    const uint64_t base = (uint64_t)a + (uint64_t)inner * ((uint64_t)n * r);
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int col = cl + 32 * q;
      f4 x{0.f, 0.f, 0.f, 0.f}, y{0.f, 0.f, 0.f, 0.f};
      if (kok && col < n) {
        const uint64_t off = base + (uint64_t)inner * col;
        x = *(const f4*)(psi + off);
        y = *(const f4*)(cur + off);
      }
      ra[q] = x;
      rb[q] = y;
    }
  };
  f4 acc[HB][HB];
#pragma unroll
  for (int x = 0; x < HB; ++x)
#pragma unroll
    for (int y = 0; y < HB; ++y) acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};
  const uint32_t nchunks = (ktotal + KC - 1) / KC;
  const uint32_t c0 = blockIdx.x * chunks_per_wg;
  const uint32_t c1 = c0 + chunks_per_wg < nchunks ? c0 + chunks_per_wg : nchunks;
  if (c0 < c1) gload(c0);
  for (uint32_t c = c0; c < c1; ++c) {
    __syncthreads();   // the previous chunk's LDS reads are done
#pragma unroll
    for (int q = 0; q < PASSES; ++q) {
      const int col = cl + 32 * q;
      if (col < NP) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          As[(4 * kg + t) * SP + col] = ra[q][t];
          Bs[(4 * kg + t) * SP + col] = rb[q][t];
        }
      }
    }
    __syncthreads();
    if (c + 1 < c1) gload(c + 1);
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kr = 4 * ks + kq;
      float xa[HB], yb[HB];
#pragma unroll
      for (int x = 0; x < HB; ++x) xa[x] = (ib0 + x < NB) ? As[kr * SP + (ib0 + x) * 16 + r16] : 0.f;
#pragma unroll
      for (int y = 0; y < HB; ++y) yb[y] = (jb0 + y < NB) ? Bs[kr * SP + (jb0 + y) * 16 + r16] : 0.f;
#pragma unroll
      for (int x = 0; x < HB; ++x) {
        if (ib0 + x >= NB) continue;
#pragma unroll
        for (int y = 0; y < HB; ++y) {
          if (jb0 + y >= NB) continue;
          // cur first: the block is out^T, so lanes run along i
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(yb[y], xa[x], acc[x][y], 0, 0, 0);
        }
      }
    }
  }
  // block (x, y), register e: out[16 (ib0 + x) + r16, 16 (jb0 + y) + 4 kq + e]
  double* out = part + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int x = 0; x < HB; ++x)
#pragma unroll
    for (int y = 0; y < HB; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = (ib0 + x) * 16 + r16, j = (jb0 + y) * 16 + 4 * kq + e;
        if (ib0 + x < NB && jb0 + y < NB && i < n && j < n) out[(int64_t)j * n + i] = (double)acc[x][y][e];
      }
}

// sum of the split partials: 64 consecutive outputs per block, 16 groups of
// splits per output (fixed order, then a fixed LDS tree): deterministic
template <typename T>
__global__ __launch_bounds__(1024) void gemm_reduce_kernel(GemmDesc<T> d, int splits, const double* part) {
  __shared__ double red[16][65];
  const int64_t mn = (int64_t)d.M * d.N;
  const int64_t total = mn * d.Z;
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t idx = blockIdx.x * (int64_t)64 + el;
  double acc = 0.0;
  if (idx < total) {
    const int z = (int)(idx / mn);
    const int64_t e = idx % mn;
    const int gi = (int)(e % d.M), gj = (int)(e / d.M);
    for (int k = g; k < splits; k += 16) acc += part[(((int64_t)k * d.Z + z) * d.N + gj) * d.M + gi];
  }
  red[g][el] = acc;
  __syncthreads();
  if (g == 0 && idx < total) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) s += red[q][el];
    const int z = (int)(idx / mn);
    const int64_t e = idx % mn;
    const int gi = (int)(e % d.M), gj = (int)(e / d.M);
    if (!(d.sym && gi > gj)) put<T>(d, z, gi, gj, s, 1, 0, nullptr);
  }
}

// Optional timing of every contraction launch with HIP events on the launch
// stream (process-wide), per kernel kind, for the roofline report.
constexpr int PROF_CAP = 4096;
constexpr int PROF_KINDS = 5;   // 0 gemm_pipe_kernel, 1 float64-accumulated Gram (gram64_kernel), 2 mode_product_kernel,
                                 // 3 leg_gram_kernel, 4 split-bf16 GEMM (tile_gemm_kernel<true>)
struct GemmProfile {
  int on = 0;
  int n = 0;
  hipEvent_t ev[2 * PROF_CAP];
  int kind[PROF_CAP];
  double launches[PROF_KINDS] = {}, ms[PROF_KINDS] = {}, flops[PROF_KINDS] = {}, bytes[PROF_KINDS] = {};
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
    g_prof.ms[g_prof.kind[i]] += t;
  }
  g_prof.n = 0;
  return 0;
}

int prof_begin(hipStream_t s) {
  if (!g_prof.on) return 0;
  if (g_prof.n == PROF_CAP) {
    const int r = prof_drain();
    if (r) return r;
  }
  HPT_HIP(hipEventRecord(g_prof.ev[2 * g_prof.n], s));
  return 0;
}

int prof_end(hipStream_t s, int kind, double flops, double bytes) {
  if (!g_prof.on) return 0;
  HPT_HIP(hipEventRecord(g_prof.ev[2 * g_prof.n + 1], s));
  g_prof.kind[g_prof.n] = kind;
  g_prof.n++;
  g_prof.launches[kind] += 1;
  g_prof.flops[kind] += flops;
  g_prof.bytes[kind] += bytes;
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
  for (int k = 0; k < PROF_KINDS; ++k) g_prof.launches[k] = g_prof.ms[k] = g_prof.flops[k] = g_prof.bytes[k] = 0;
  return 0;
}

int gemm_profile_active() { return g_prof.on; }

int gemm_profile_read(int kind, double* out4) {
  if (kind < -1 || kind >= PROF_KINDS) return -1;
  if (g_prof.on) {
    int r = prof_drain();
    if (r) return r;
  }
  for (int q = 0; q < 4; ++q) out4[q] = 0;
  for (int k = 0; k < PROF_KINDS; ++k) {
    if (kind >= 0 && k != kind) continue;
    out4[0] += g_prof.launches[k];
    out4[1] += g_prof.ms[k];
    out4[2] += g_prof.flops[k];
    out4[3] += g_prof.bytes[k];
  }
  return 0;
}

// Row splits of the float64 Gram of an m x n X: doubled while the grid stays
// within ~4096 workgroups, every split keeps at least 16 chunks of rows and
// the partial tiles (splits x n x n doubles) fit part_cap.
int gram64_splits(int64_t m, int n, int64_t part_cap) {
  const int64_t tiles_m = ceil_div(n, 64);
  const int64_t tiles = tiles_m * (tiles_m + 1) / 2;
  const int64_t chunks = ceil_div(m, G64_TK);
  int splits = 1;
  while (splits < 128 && tiles * splits * 2 <= 4096 && chunks / (splits * 2) >= 16 &&
         (int64_t)splits * 2 * n * n <= part_cap)
    splits *= 2;
  return splits;
}

// G (n x n, leading dimension ldg, both triangles) = X^T X in float64 for a
// float32 X (m x n, column-major, leading dimension ldx): gram64_kernel writes
// every split's upper 16-blocks (all of them, zeros for an empty split) into
// part (splits x n x n doubles), gemm_reduce_kernel sums the splits in a fixed
// order and mirrors.  Nothing in part has to be cleared before the call.
int gram64_launch(const float* X, int64_t ldx, int m, int n, double* G, int64_t ldg, int splits, double* part,
                  hipStream_t s) {
  if (n <= 0) return 0;
  const int tiles_m = (int)ceil_div(n, 64);
  const int64_t tiles = (int64_t)tiles_m * (tiles_m + 1) / 2;
  const int chunks = (int)ceil_div(m, G64_TK);
  const bool vec = ldx % 4 == 0 && ((uintptr_t)X & 15) == 0;
  const unsigned grid = (unsigned)(tiles * splits);
  if (vec)
    hipLaunchKernelGGL(gram64_kernel<true>, dim3(grid), dim3(256), 0, s, X, ldx, m, n, (int)tiles, splits, chunks,
                       part);
  else
    hipLaunchKernelGGL(gram64_kernel<false>, dim3(grid), dim3(256), 0, s, X, ldx, m, n, (int)tiles, splits, chunks,
                       part);
  HPT_LAUNCH_CHECK("gram64_kernel");
  GemmDesc<float> d{};
  d.M = n; d.N = n; d.K = m; d.R = 1; d.Z = 1;
  d.A = X; d.lda = ldx; d.tA = 1;
  d.B = X; d.ldb = ldx; d.tB = 0;
  d.C = G; d.ldc = ldg; d.c_double = 1;
  d.alpha = 1.0; d.beta = 0.0; d.sym = 1; d.acc64 = 1;
  const int64_t blocks = ceil_div((int64_t)n * n, 64);
  hipLaunchKernelGGL(gemm_reduce_kernel<float>, dim3((unsigned)blocks), dim3(1024), 0, s, d, splits,
                     (const double*)part);
  HPT_LAUNCH_CHECK("gemm_reduce_kernel");
  return 0;
}

namespace {
// the float64-accumulated Gram G = X^T X of a float32 X, written whole
// (mirrored) into a float64 C, is served by gram64_kernel
bool gram64_eligible(const GemmDesc<float>& d, int64_t part_cap) {
  return d.acc64 && d.sym && d.R == 1 && d.Z == 1 && d.tA && !d.tB && d.A == d.B && d.lda == d.ldb &&
         d.c_double && d.M == d.N && d.K <= 0x7fffffff - G64_TK && (int64_t)d.M * d.M <= part_cap;
}

int gram64(const GemmDesc<float>& d, double* part, int64_t part_cap, hipStream_t s) {
  const int n = d.M, m = d.K;
  const int splits = gram64_splits(m, n, part_cap);
  RC_PROF(prof_begin(s));
  RC_PROF(gram64_launch(d.A, d.lda, m, n, (double*)d.C, d.ldc, splits, part, s));
  {
    const double N = n, K = m;
    // algorithmic: half the products of a full n x n product; X read once, G written once
    RC_PROF(prof_end(s, 1, N * N * K, 4.0 * K * N + 8.0 * N * N));
  }
  return 0;
}
}  // namespace

namespace {
// plain float32 products C = A B (no transposes, batches or scaling): the
// 128 x 80 XCD-ordered tiles, split-bf16 when asked for
bool tile_eligible(const GemmDesc<float>& d) {
  return !d.acc64 && !d.sym && !d.tA && !d.tB && d.R == 1 && d.Z == 1 && !d.c_double && d.alpha == 1.0 &&
         d.beta == 0.0;
}

int tile_gemm(const GemmDesc<float>& d, hipStream_t s) {
  const int ntn = (int)ceil_div(d.N, BS_BN);
  const int64_t total = ceil_div(d.M, BS_BM) * (int64_t)ntn;
  const int64_t per_xcd = ceil_div(total, 8);
  if (8 * per_xcd > 0x7fffffff) return -1;
  const dim3 grid((unsigned)(8 * per_xcd));
  RC_PROF(prof_begin(s));
  if (d.bsplit) {
    hipLaunchKernelGGL(tile_gemm_kernel<true>, grid, dim3(256), 0, s, d.A, d.lda, d.B, d.ldb, (float*)d.C, d.ldc,
                       d.M, d.N, d.K, ntn, total, per_xcd);
    HPT_LAUNCH_CHECK("tile_gemm_kernel<split>");
  } else {
    const int avec = ((reinterpret_cast<uintptr_t>(d.A) & 15) == 0) && d.lda % 4 == 0;
    const int bvec = ((reinterpret_cast<uintptr_t>(d.B) & 15) == 0) && d.ldb % 4 == 0;
    hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, s, d.A, d.lda, d.B, d.ldb, (float*)d.C, d.ldc,
                       d.M, d.N, d.K, ntn, total, per_xcd, avec, bvec);
    HPT_LAUNCH_CHECK("gemm_f32_kernel");
  }
  const double M = d.M, N = d.N, K = d.K;
  RC_PROF(prof_end(s, d.bsplit ? 4 : 0, 2.0 * M * N * K, 4.0 * (M * K + K * N + M * N)));
  return 0;
}
}  // namespace

template <typename T>
int gemm(const GemmDesc<T>& d, double* part, int64_t part_cap, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.Z <= 0) return 0;
  if (d.K <= 0 || d.R <= 0) return -1;  // callers never ask for an empty reduction
  // 64 x 64 tiles; HPT_GEMM_TILE=128 selects 128 x 128 tiles (tuning)
  static const int forced = [] {
    const char* e = getenv("HPT_GEMM_TILE");
    return e ? atoi(e) : 0;
  }();
  if constexpr (std::is_same<T, float>::value) {
    if (gram64_eligible(d, part_cap)) return gram64(d, part, part_cap, s);
    if (tile_eligible(d)) return tile_gemm(d, s);
  }
  const bool big = !d.acc64 && forced == 128;
  const int tile = big ? 128 : 64;
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
  RC_PROF(prof_begin(s));
  if (d.acc64 && sizeof(T) == 4)
    hipLaunchKernelGGL((gemm_pipe_kernel<T, double, 32>), grid, dim3(256), 0, s, d, tiles_m, tiles_n, splits,
                       chunks_per_r, part);
  else if (big)
    hipLaunchKernelGGL((gemm_pipe_kernel<T, T, 64>), grid, dim3(256), 0, s, d, tiles_m, tiles_n, splits,
                       chunks_per_r, part);
  else
    hipLaunchKernelGGL((gemm_pipe_kernel<T, T, 32>), grid, dim3(256), 0, s, d, tiles_m, tiles_n, splits,
                       chunks_per_r, part);
  HPT_LAUNCH_CHECK("gemm_kernel");
  {
    const double M = d.M, N = d.N, K = d.K, R = d.R, Z = d.Z;
    const double za = d.sAz ? Z : 1.0, zb = d.sBz ? Z : 1.0;
    const double ra = d.sAr ? R : 1.0, rb = d.sBr ? R : 1.0;
    // algorithmic: a SYRK does half the products; operands read once, result written once
    RC_PROF(prof_end(s, d.acc64 ? 1 : 0, (d.sym ? 1.0 : 2.0) * M * N * K * R * Z,
                     sizeof(T) * (M * K * ra * za + K * N * rb * zb) + (d.c_double ? 8.0 : (double)sizeof(T)) * M * N * Z));
  }
  if (splits > 1) {
    const int64_t n = (int64_t)d.M * d.N * d.Z;
    const int64_t blocks = ceil_div(n, 64);
    if (blocks > 0x7fffffff) return -1;
    hipLaunchKernelGGL(gemm_reduce_kernel<T>, dim3((unsigned)blocks), dim3(1024), 0, s, d, splits, part);
    HPT_LAUNCH_CHECK("gemm_reduce_kernel");
  }
  return 0;
}

template int gemm<double>(const GemmDesc<double>&, double*, int64_t, hipStream_t);
template int gemm<float>(const GemmDesc<float>&, double*, int64_t, hipStream_t);

namespace {
int resident_grid(const void* kernel, int threads, int64_t work_waves, size_t lds = 0) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t need = ceil_div(work_waves, threads / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)cus * per_cu));
}

template <int NP, int KS = NP / 4>
int launch_mode(const float* src, float* dst, const float* S, int n, int64_t inner, int64_t outer, hipStream_t s) {
  // Variants the autotuner chooses from (the same MFMAs in the same order for
  // every output): leading leg, the resident grid or two thirds of it; even
  // inner >= 32, 32-row strips on the resident grid or two thirds of it, or
  // 16-row strips.
  TuneCall tc;
  if (inner == 1) {
    const int64_t strips = ceil_div(outer, 16);
    const size_t lds = (size_t)(n < NP ? n + 1 : NP) * 128 * sizeof(float);
    const int cand = tune_pick(TUNE_MODE_LEAD, n, inner, outer, 2, &tc);
    tune_begin(&tc, s);
    if (n % 4 == 0) {
      int g = resident_grid((const void*)mode_product_lead_kernel<NP, true>, 256, strips, lds);
      if (cand == 1) g = std::max(1, 2 * g / 3);
      hipLaunchKernelGGL((mode_product_lead_kernel<NP, true>), dim3(g), dim3(256), lds, s, src, dst, S, n, outer);
    } else {
      int g = resident_grid((const void*)mode_product_lead_kernel<NP, false>, 256, strips, lds);
      if (cand == 1) g = std::max(1, 2 * g / 3);
      hipLaunchKernelGGL((mode_product_lead_kernel<NP, false>), dim3(g), dim3(256), lds, s, src, dst, S, n, outer);
    }
  } else {
    const bool even32 = inner % 2 == 0 && inner >= 32 && inner * n < ((int64_t)1 << 30);   // 32-bit byte offsets
    const int cand = even32 ? tune_pick(TUNE_MODE_STRIPS, n, inner, outer, 3, &tc) : 2;
    tune_begin(&tc, s);
    if (cand < 2) {
      const int64_t spz = ceil_div(inner, 32);
      int g = resident_grid((const void*)mode_product32_kernel<NP, KS>, 256, spz * outer);
      if (cand == 1) g = std::max(1, 2 * g / 3);
      hipLaunchKernelGGL((mode_product32_kernel<NP, KS>), dim3(g), dim3(256), 0, s, src, dst, S, n, inner, outer,
                         spz);
    } else {
      const int64_t spz = ceil_div(inner, 16);
      const int g = resident_grid((const void*)mode_product_kernel<NP, KS>, 256, spz * outer);
      hipLaunchKernelGGL((mode_product_kernel<NP, KS>), dim3(g), dim3(256), 0, s, src, dst, S, n, inner, outer, spz);
    }
  }
  tune_end(&tc, s);
  HPT_LAUNCH_CHECK("mode_product_kernel");
  return 0;
}
template <int NP>
int launch_leg_gram(const float* psi, const float* cur, int n, int64_t inner, int64_t outer, int64_t chunks_per_r,
                    int64_t cpw, int G, double* part, hipStream_t s) {
  if (inner > 1 && inner % 4 == 0 && inner * outer < ((int64_t)1 << 31)) {
    // flattened reduction index, chunks of 32
    const int64_t ktotal = inner * outer;
    const int64_t nch = ceil_div(ktotal, 32);
    const int64_t cw = ceil_div(nch, G);
    const int g2 = (int)ceil_div(nch, cw);
    hipLaunchKernelGGL((leg_gram_lds_kernel<NP>), dim3(g2), dim3(256), 0, s, psi, cur, n, (uint32_t)inner,
                       (uint32_t)ktotal, (uint32_t)cw, part);
    HPT_LAUNCH_CHECK("leg_gram_lds_kernel");
    return g2;
  }
  if (inner == 1)
    hipLaunchKernelGGL((leg_gram_kernel<NP, true, false>), dim3(G), dim3(256), 0, s, psi, cur, n, inner, outer,
                       chunks_per_r, cpw, part);
  else if (inner % 4 == 0)
    hipLaunchKernelGGL((leg_gram_kernel<NP, false, true>), dim3(G), dim3(256), 0, s, psi, cur, n, inner, outer,
                       chunks_per_r, cpw, part);
  else
    hipLaunchKernelGGL((leg_gram_kernel<NP, false, false>), dim3(G), dim3(256), 0, s, psi, cur, n, inner, outer,
                       chunks_per_r, cpw, part);
  HPT_LAUNCH_CHECK("leg_gram_kernel");
  return G;
}
}  // namespace

int leg_gram_f32(const float* psi, const float* cur, int n, int64_t inner, int64_t outer, double* out, double* part,
                 int64_t part_cap, hipStream_t s) {
  if (n < 1 || n > 128 || inner < 1 || outer < 1) return 0;
  const int64_t n2 = (int64_t)n * n;
  const int64_t chunks_per_r = inner == 1 ? ceil_div(outer, 16) : ceil_div(inner, 16);
  const int64_t total = (inner == 1 ? 1 : outer) * chunks_per_r;
  int64_t G = std::min<int64_t>(1024, part_cap / n2);
  G = std::min<int64_t>(G, total);
  if (G < 1) return 0;
  const int64_t cpw = ceil_div(total, G);
  G = ceil_div(total, cpw);
  RC_PROF(prof_begin(s));
  int r;
  switch ((n + 15) / 16) {
    case 1: r = launch_leg_gram<16>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    case 2: r = launch_leg_gram<32>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    case 3: r = launch_leg_gram<48>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    case 4: r = launch_leg_gram<64>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    case 5: r = launch_leg_gram<80>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    case 6: r = launch_leg_gram<96>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    case 7: r = launch_leg_gram<112>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
    default: r = launch_leg_gram<128>(psi, cur, n, inner, outer, chunks_per_r, cpw, (int)G, part, s); break;
  }
  if (r < 0) return r;
  const int parts = r;   // workgroups that wrote a partial
  {
    const double el = (double)inner * n * outer;
    RC_PROF(prof_end(s, 3, 2.0 * el * n, 4.0 * 2.0 * el + 8.0 * n2));
  }
  GemmDesc<float> d{};
  d.M = n; d.N = n; d.K = 1; d.R = 1; d.Z = 1;
  d.C = out; d.ldc = n; d.c_double = 1; d.alpha = 1.0; d.beta = 0.0;
  const int64_t blocks = ceil_div(n2, 64);
  hipLaunchKernelGGL(gemm_reduce_kernel<float>, dim3((unsigned)blocks), dim3(1024), 0, s, d, parts, (const double*)part);
  HPT_LAUNCH_CHECK("gemm_reduce_kernel");
  return 1;
}

// One v_mfma_f32_16x16x32_bf16 whose every output is sum_k bf16(a[k]) + c
// (the same 32 values a in every row, all ones in the other operand): shows
// how the instruction rounds its float32 sum (out: 64 lanes x 4 registers).
__global__ void bf16_mfma_sum_kernel(const float* __restrict__ a, float c, float* __restrict__ out) {
  const int l = threadIdx.x;
  bf8 x, y;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    x[t] = (__bf16)a[8 * (l / 16) + t];
    y[t] = (__bf16)1.0f;
  }
  f4 acc = {c, c, c, c};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(y, x, acc, 0, 0, 0);
#pragma unroll
  for (int e = 0; e < 4; ++e) out[4 * l + e] = acc[e];
}

int bf16_mfma_sum(const float* a, float c, float* out, hipStream_t s) {
  hipLaunchKernelGGL(bf16_mfma_sum_kernel, dim3(1), dim3(64), 0, s, a, c, out);
  HPT_LAUNCH_CHECK("bf16_mfma_sum_kernel");
  return 0;
}

// float64-arithmetic mode product of float32 data: one thread per
// (a, 8 consecutive j, b), the 8 sums carried in registers over k; consecutive
// threads take consecutive a, so the loads of src[a, k, b] are coalesced
__global__ __launch_bounds__(256) void mode_product_f64acc_kernel(const double* __restrict__ S,
                                                                  const float* __restrict__ src,
                                                                  float* __restrict__ dst, int n, int64_t inner,
                                                                  int64_t outer, int jblocks) {
  const int64_t total = inner * outer * jblocks;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = idx % inner;
    const int64_t r = idx / inner;
    const int j0 = (int)(r % jblocks) * 8;
    const int64_t b = r / jblocks;
    const float* sp = src + a + b * inner * n;
    double acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = 0.0;
    for (int k = 0; k < n; ++k) {
      const double x = (double)sp[(int64_t)k * inner];
      const double* Sk = S + (int64_t)k * n;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (j0 + t < n) acc[t] = fma(Sk[j0 + t], x, acc[t]);
    }
    float* dp = dst + a + b * inner * n;
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (j0 + t < n) dp[(int64_t)(j0 + t) * inner] = (float)acc[t];
  }
}

int mode_product_f64acc(const double* S, const float* src, float* dst, int n, int64_t inner, int64_t outer,
                        hipStream_t s) {
  if (n < 1 || inner < 1 || outer < 1) return -1;
  const int jblocks = (int)ceil_div(n, 8);
  const int64_t total = inner * outer * jblocks;
  const int64_t blocks = std::min<int64_t>(ceil_div(total, 256), 16384);
  hipLaunchKernelGGL(mode_product_f64acc_kernel, dim3((unsigned)blocks), dim3(256), 0, s, S, src, dst, n, inner,
                     outer, jblocks);
  HPT_LAUNCH_CHECK("mode_product_f64acc_kernel");
  return 0;
}

int mode_product_f32(const float* S, const float* src, float* dst, int n, int64_t inner, int64_t outer,
                     hipStream_t s) {
  if (n < 1 || n > 128 || inner < 1 || outer < 1) return 0;
  if (inner > 1 && inner < 16) return 0;
  if (inner * n >= ((int64_t)1 << 30)) return 0;  // 32-bit byte offsets inside a slice
  if (inner == 1 && outer < 16) return 0;
  RC_PROF(prof_begin(s));
  int r;
  switch ((n + 15) / 16) {
    case 1: r = launch_mode<16>(src, dst, S, n, inner, outer, s); break;
    case 2: r = launch_mode<32>(src, dst, S, n, inner, outer, s); break;
    case 3: r = launch_mode<48>(src, dst, S, n, inner, outer, s); break;
    case 4: r = launch_mode<64>(src, dst, S, n, inner, outer, s); break;
    case 5: r = launch_mode<80>(src, dst, S, n, inner, outer, s); break;
    case 6: r = launch_mode<96>(src, dst, S, n, inner, outer, s); break;
    case 7:
      // n in (96, 100] (chi_max = 100) needs 25 k-steps, not 28
      r = n <= 100 ? launch_mode<112, 25>(src, dst, S, n, inner, outer, s) : launch_mode<112>(src, dst, S, n, inner, outer, s);
      break;
    default: r = launch_mode<128>(src, dst, S, n, inner, outer, s); break;
  }
  if (r) return r;
  const double el = (double)inner * n * outer;
  RC_PROF(prof_end(s, 2, 2.0 * el * n, 4.0 * (2.0 * el + (double)n * n)));
  return 1;
}



}  // namespace hpt
