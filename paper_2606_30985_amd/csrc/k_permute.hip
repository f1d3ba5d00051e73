// Device tensor permutation (paper Sec. "GPU Tensor Permutation": the cut
// leg is moved next to the Pauli leg before QR and moved back afterwards,
// entirely on the device).
//
// The gate update only ever swaps two groups of axes between a fast group
// and the Pauli axis: [A, B, C, P] -> [A, C, B, P] (A = legs before the cut,
// B = the cut leg, C = legs after it).  When A is large the move is a gather
// of whole A-element rows (16-byte vectors); when A is small the (B, C) plane
// is transposed through a 64 x 64 LDS tile so that reads run along B and
// writes along C.  A generic
// rank <= 8 kernel (one thread per output element) serves everything else.
// All paths are plain copies: bit-exact.
#include <algorithm>

#include "common.h"
#include "tune.h"

namespace hpt {

namespace {

struct PermMeta {
  int ndim;
  int64_t out_dims[8];
  int64_t in_stride_of_out[8];  // input stride of the axis that is output axis k
};

template <typename E>
__global__ void permute_generic_kernel(const E* __restrict__ in, E* __restrict__ out,
                                       PermMeta m, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx, off = 0;
    for (int k = 0; k < m.ndim; ++k) {
      const int64_t c = rem % m.out_dims[k];
      rem /= m.out_dims[k];
      off += c * m.in_stride_of_out[k];
    }
    out[idx] = in[off];
  }
}

// out[a, c, b, p] = in[a, b, c, p] with A large: a gather of whole rows.  Both
// tensors are rows of A contiguous elements; output row c + C (b + B p) is
// input row b + B (c + C p).  Each thread moves one vector V of a row (16
// bytes when a row is a whole number of 16-byte vectors, else one element),
// the row index is split once per vector in 32-bit arithmetic (the caller
// guarantees rows * nv < 2^31; the loop counter itself is 64-bit), so loads
// and stores run along the rows.
template <typename V>
__global__ __launch_bounds__(256) void swap_rows_kernel(const V* __restrict__ in, V* __restrict__ out, int nv,
                                                        int B, int C, int total) {
  for (int64_t vv = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; vv < total;
       vv += (int64_t)gridDim.x * blockDim.x) {
    const int v = (int)vv;
    const int ro = v / nv, col = v - ro * nv;
    const int c = ro % C, t = ro / C;
    const int b = t % B, p = t / B;
    const int ri = b + B * (c + C * p);
    out[(int64_t)ro * nv + col] = in[(int64_t)ri * nv + col];
  }
}

// the same for tensors past the 32-bit range: 64-bit index arithmetic
template <typename V>
__global__ __launch_bounds__(256) void swap_rows64_kernel(const V* __restrict__ in, V* __restrict__ out, int64_t nv,
                                                          int64_t B, int64_t C, int64_t total) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < total; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ro = v / nv, col = v - ro * nv;
    const int64_t c = ro % C, t = ro / C;
    const int64_t b = t % B, p = t / B;
    out[ro * nv + col] = in[(b + B * (c + C * p)) * nv + col];
  }
}

template <typename V>
int launch_swap_rows(const void* in, void* out, int64_t nv, int64_t B, int64_t C, int64_t P, hipStream_t s) {
  const int64_t total = nv * B * C * P;
  const int grid = (int)std::min<int64_t>(ceil_div(total, 256), 262144);
  if (total < 0x7fffffff)
    hipLaunchKernelGGL(swap_rows_kernel<V>, dim3(grid), dim3(256), 0, s, (const V*)in, (V*)out, (int)nv, (int)B,
                       (int)C, (int)total);
  else
    hipLaunchKernelGGL(swap_rows64_kernel<V>, dim3(grid), dim3(256), 0, s, (const V*)in, (V*)out, nv, B, C, total);
  HPT_LAUNCH_CHECK("swap_rows_kernel");
  return 0;
}

// out[a, c, b, p] = in[a, b, c, p] with small A: tile (b, c) planes through LDS.
// grid.x over tiles of (B, C), grid.y over (a, p) slices.
constexpr int TT = 64;
template <typename E>
__global__ __launch_bounds__(256) void swap_mid_tile_kernel(const E* __restrict__ in,
                                                            E* __restrict__ out, int64_t A,
                                                            int64_t B, int64_t C,
                                                            int64_t tiles_b) {
  __shared__ E tile[TT][TT + 1];
  const int64_t tb = blockIdx.x % tiles_b, tc = blockIdx.x / tiles_b;
  const int64_t slice = blockIdx.y;  // a + A * p
  const int64_t a = slice % A, p = slice / A;
  const int64_t b0 = tb * TT, c0 = tc * TT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t in_base = a + A * (B * C * p);
  const int64_t out_base = a + A * (C * B * p);
  for (int r = ty; r < TT; r += 4) {
    const int64_t b = b0 + tx, c = c0 + r;
    if (b < B && c < C) tile[r][tx] = in[in_base + A * (b + B * c)];
  }
  __syncthreads();
  for (int r = ty; r < TT; r += 4) {
    const int64_t c = c0 + tx, b = b0 + r;
    if (b < B && c < C) out[out_base + A * (c + C * b)] = tile[tx][r];
  }
}

// out[c, b, p] = in[b, c, p] (A == 1) with B <= PB: a panel of all B rows and
// PC consecutive c is one contiguous block of the input (B * PC elements,
// read in order); each b of it is a run of PC contiguous outputs.
// grid.x over c panels, grid.y over p.
template <typename E, int PB, int PC>
__global__ __launch_bounds__(256) void swap_panel_smallb_kernel(const E* __restrict__ in, E* __restrict__ out,
                                                                int B, int64_t C) {
  __shared__ E tile[PC][PB + 1];
  const int64_t c0 = (int64_t)blockIdx.x * PC, p = blockIdx.y;
  const int pc = (int)(C - c0 < PC ? C - c0 : PC);
  const E* src = in + (p * C + c0) * B;
  const int n = pc * B;
  // (t / B, t % B) stepped along t without a division per element
  int j = (int)threadIdx.x / B, b = (int)threadIdx.x % B;
  const int sj = 256 / B, sb = 256 % B;
  for (int t = threadIdx.x; t < n; t += 256) {
    tile[j][b] = src[t];
    j += sj;
    b += sb;
    if (b >= B) {
      b -= B;
      ++j;
    }
  }
  __syncthreads();
  E* dst = out + p * C * B + c0;
  for (int t = threadIdx.x; t < PC * B; t += 256) {
    const int j = t % PC, b = t / PC;
    if (j < pc) dst[(int64_t)b * C + j] = tile[j][b];
  }
}

// out[c, b, p] = in[b, c, p] (A == 1) with C <= PC: each c of a panel of PB
// consecutive b is a run of PB contiguous inputs; the panel's outputs are
// one contiguous block (C * PB elements, written in order).
template <typename E, int PB, int PC>
__global__ __launch_bounds__(256) void swap_panel_smallc_kernel(const E* __restrict__ in, E* __restrict__ out,
                                                                int64_t B, int C) {
  __shared__ E tile[PC][PB + 1];
  const int64_t b0 = (int64_t)blockIdx.x * PB, p = blockIdx.y;
  const int pb = (int)(B - b0 < PB ? B - b0 : PB);
  const E* src = in + p * B * C + b0;
  for (int t = threadIdx.x; t < PB * C; t += 256) {
    const int i = t % PB, c = t / PB;
    if (i < pb) tile[c][i] = src[(int64_t)c * B + i];
  }
  __syncthreads();
  E* dst = out + (p * B + b0) * C;
  const int n = pb * C;
  int i = (int)threadIdx.x / C, c = (int)threadIdx.x % C;
  const int si = 256 / C, sc = 256 % C;
  for (int t = threadIdx.x; t < n; t += 256) {
    dst[t] = tile[c][i];
    i += si;
    c += sc;
    if (c >= C) {
      c -= C;
      ++i;
    }
  }
}

// Float32 panels with 16-byte accesses on both sides (the caller checks that
// every vector is aligned: B and C multiples of 4, 16-byte aligned tensors).
// 128 x 128 panels (66 KB of LDS): the scattered side moves 512-byte runs.
// smallb, B <= 128: the panel of all B rows and 128 consecutive c is read as
// one contiguous block of float4, each b's 128 outputs are written as 32
// float4.  (j, b) = divmod(4 u, B) once per vector, stepped inside it.
constexpr int VP = 128;
__global__ __launch_bounds__(256) void swap_panel_smallb_vec_kernel(const uint32_t* __restrict__ in,
                                                                    uint32_t* __restrict__ out, int B, int64_t C) {
  __shared__ uint32_t tile[VP][VP + 1];
  const int64_t c0 = (int64_t)blockIdx.x * VP, p = blockIdx.y;
  const int pc = (int)(C - c0 < VP ? C - c0 : VP);   // a multiple of 4 (C is)
  const uint4* src = (const uint4*)(in + (p * C + c0) * B);
  const int nu = pc * B / 4;
  for (int u = threadIdx.x; u < nu; u += 256) {
    const uint4 v = src[u];
    int j = 4 * u / B, b = 4 * u - j * B;
    const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      tile[j][b] = e[q];
      if (++b == B) {
        b = 0;
        ++j;
      }
    }
  }
  __syncthreads();
  uint32_t* dst = out + p * C * B + c0;
  const int nq = pc / 4;
  for (int w = threadIdx.x; w < nq * B; w += 256) {
    const int b = w / nq, j = 4 * (w - b * nq);
    *(uint4*)(dst + (int64_t)b * C + j) = make_uint4(tile[j][b], tile[j + 1][b], tile[j + 2][b], tile[j + 3][b]);
  }
}

// smallc, C <= 128: each c's run of 128 consecutive b is read as 32 float4,
// the panel's outputs (128 b x C, contiguous) are written as float4.
__global__ __launch_bounds__(256) void swap_panel_smallc_vec_kernel(const uint32_t* __restrict__ in,
                                                                    uint32_t* __restrict__ out, int64_t B, int C) {
  __shared__ uint32_t tile[VP][VP + 1];
  const int64_t b0 = (int64_t)blockIdx.x * VP, p = blockIdx.y;
  const int pb = (int)(B - b0 < VP ? B - b0 : VP);   // a multiple of 4 (B is)
  const uint32_t* src = in + p * B * C + b0;
  const int nq = pb / 4;
  for (int w = threadIdx.x; w < nq * C; w += 256) {
    const int c = w / nq, i = 4 * (w - c * nq);
    const uint4 v = *(const uint4*)(src + (int64_t)c * B + i);
    tile[c][i] = v.x;
    tile[c][i + 1] = v.y;
    tile[c][i + 2] = v.z;
    tile[c][i + 3] = v.w;
  }
  __syncthreads();
  uint4* dst = (uint4*)(out + (p * B + b0) * C);
  const int nu = pb * C / 4;
  for (int u = threadIdx.x; u < nu; u += 256) {
    int i = 4 * u / C, c = 4 * u - i * C;
    uint32_t e[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      e[q] = tile[c][i];
      if (++c == C) {
        c = 0;
        ++i;
      }
    }
    dst[u] = make_uint4(e[0], e[1], e[2], e[3]);
  }
}

template <typename E>
int launch_panel(const void* in, void* out, int64_t B, int64_t C, int64_t P, hipStream_t s) {
  // 128 x 64 panels (float32) or 128 x 32 (float64): 33 / 33 KB of LDS
  constexpr int PL = 128, PS = sizeof(E) == 4 ? 64 : 32;
  if (P > 65535) return -1;
  if (sizeof(E) == 4 && B % 4 == 0 && C % 4 == 0 && ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 15) == 0 &&
      (B <= VP || C <= VP)) {
    if (B <= VP) {
      const int64_t np = ceil_div(C, VP);
      if (np > 0x7fffffff) return -1;
      hipLaunchKernelGGL(swap_panel_smallb_vec_kernel, dim3((unsigned)np, (unsigned)P), dim3(256), 0, s,
                         (const uint32_t*)in, (uint32_t*)out, (int)B, C);
    } else {
      const int64_t np = ceil_div(B, VP);
      if (np > 0x7fffffff) return -1;
      hipLaunchKernelGGL(swap_panel_smallc_vec_kernel, dim3((unsigned)np, (unsigned)P), dim3(256), 0, s,
                         (const uint32_t*)in, (uint32_t*)out, B, (int)C);
    }
    HPT_LAUNCH_CHECK("swap_panel_vec_kernel");
    return 0;
  }
  if (B <= PL) {
    const int64_t np = ceil_div(C, PS);
    if (np > 0x7fffffff) return -1;
    hipLaunchKernelGGL((swap_panel_smallb_kernel<E, PL, PS>), dim3((unsigned)np, (unsigned)P), dim3(256), 0, s,
                       (const E*)in, (E*)out, (int)B, C);
  } else {
    const int64_t np = ceil_div(B, PS);
    if (np > 0x7fffffff) return -1;
    hipLaunchKernelGGL((swap_panel_smallc_kernel<E, PS, PL>), dim3((unsigned)np, (unsigned)P), dim3(256), 0, s,
                       (const E*)in, (E*)out, B, (int)C);
  }
  HPT_LAUNCH_CHECK("swap_panel_kernel");
  return 0;
}

// out[a, c, b, p] = in[a, b, c, p] through 64 x 64 LDS tiles of (b, c)
int launch_tile(const void* in, void* out, int64_t A, int64_t B, int64_t C, int64_t P, int elem, hipStream_t s) {
  const int64_t tiles_b = ceil_div(B, TT), tiles_c = ceil_div(C, TT);
  const int64_t slices = A * P;
  if (slices > 65535 || tiles_b * tiles_c > 0x7fffffff) return -1;
  dim3 grid((unsigned)(tiles_b * tiles_c), (unsigned)slices);
  if (elem == 8)
    hipLaunchKernelGGL(swap_mid_tile_kernel<uint64_t>, grid, dim3(256), 0, s,
                       (const uint64_t*)in, (uint64_t*)out, A, B, C, tiles_b);
  else
    hipLaunchKernelGGL(swap_mid_tile_kernel<uint32_t>, grid, dim3(256), 0, s,
                       (const uint32_t*)in, (uint32_t*)out, A, B, C, tiles_b);
  HPT_LAUNCH_CHECK("swap_mid_tile_kernel");
  return 0;
}

int grid_for(int64_t n) {
  int64_t g = ceil_div(n, 256);
  return (int)(g < 131072 ? (g > 0 ? g : 1) : 131072);
}

}  // namespace

int permute_generic(const void* in, void* out, int ndim, const int64_t* dims, const int* perm,
                    int elem, hipStream_t s) {
  if (ndim < 1 || ndim > 8 || (elem != 4 && elem != 8)) return -1;
  PermMeta m;
  m.ndim = ndim;
  int64_t in_stride[8];
  int64_t total = 1;
  bool seen[8] = {false, false, false, false, false, false, false, false};
  for (int k = 0; k < ndim; ++k) {
    if (dims[k] < 0) return -1;
    in_stride[k] = total;
    total *= dims[k];
  }
  for (int k = 0; k < ndim; ++k) {
    if (perm[k] < 0 || perm[k] >= ndim || seen[perm[k]]) return -1;
    seen[perm[k]] = true;
    m.out_dims[k] = dims[perm[k]];
    m.in_stride_of_out[k] = in_stride[perm[k]];
  }
  if (total == 0) return 0;
  if (elem == 8)
    hipLaunchKernelGGL(permute_generic_kernel<uint64_t>, dim3(grid_for(total)), dim3(256), 0, s,
                       (const uint64_t*)in, (uint64_t*)out, m, total);
  else
    hipLaunchKernelGGL(permute_generic_kernel<uint32_t>, dim3(grid_for(total)), dim3(256), 0, s,
                       (const uint32_t*)in, (uint32_t*)out, m, total);
  HPT_LAUNCH_CHECK("permute_generic_kernel");
  return 0;
}

int permute_swap_mid(const void* in, void* out, int64_t A, int64_t B, int64_t C, int64_t P,
                     int elem, hipStream_t s) {
  const int64_t total = A * B * C * P;
  if (total == 0) return 0;
  if (B == 1 || C == 1) {
    // nothing moves: a plain copy
    HPT_HIP(hipMemcpyAsync(out, in, (size_t)total * elem, hipMemcpyDeviceToDevice, s));
    return 0;
  }
  if (A >= 16) {
    const int64_t row_bytes = A * elem;
    const bool vec = row_bytes % 16 == 0 && ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 15) == 0;
    if (vec) return launch_swap_rows<uint4>(in, out, row_bytes / 16, B, C, P, s);
    if (elem == 8) return launch_swap_rows<uint64_t>(in, out, A, B, C, P, s);
    return launch_swap_rows<uint32_t>(in, out, A, B, C, P, s);
  }
  if (A == 1 && (B <= 128 || C <= 128) && P <= 65535) {
    // the cut leg is the first one (or goes back there): panel transposes or
    // 64 x 64 tiles, chosen by the autotuner (default: panels for float64,
    // 4.1-4.4 TB/s against 3.3-3.5 for the tiles; tiles for float32)
    TuneCall tc;
    const int cand = tune_pick(TUNE_PERMUTE_LEAD, elem, B, C * P, 2, &tc);
    const bool panel = (elem == 8) == (cand == 0);
    tune_begin(&tc, s);
    int r;
    if (panel)
      r = elem == 8 ? launch_panel<uint64_t>(in, out, B, C, P, s) : launch_panel<uint32_t>(in, out, B, C, P, s);
    else
      r = launch_tile(in, out, A, B, C, P, elem, s);
    tune_end(&tc, s);
    return r;
  }
  return launch_tile(in, out, A, B, C, P, elem, s);
}

}  // namespace hpt
