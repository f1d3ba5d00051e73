// Host engine of libhpt: memory model and arena carve, lattice topology,
// the Trotter layer (field half-steps, 4-colour gate sweep, gauge BP) and the
// measurement, all issued as stream-ordered launches of the HIP kernels.
//
// Paper: Sec. "Zero-Malloc Simulation Loop" (everything lives in one arena
// sized once), Sec. "Trotter Decomposition" (colours), Algorithm "Gate
// update", Sec. "Adaptive QR Decomposition", Sec. "BP Message Update",
// Sec. "Correlation Function via Belief Propagation", implementation
// pipeline figure (order of one time step), Table "Runtime diagnostic
// measures".
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <atomic>
#include <type_traits>
#include <vector>

#include "engine.h"

namespace hpt {

static thread_local std::string g_hip_error;
void set_hip_error(hipError_t e, const char* what) {
  g_hip_error = std::string(what) + ": " + hipGetErrorString(e);
}

namespace {

constexpr uint64_t ALIGN = 256;
inline uint64_t align_up(uint64_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// ---------------------------------------------------------------------------
// topology (site v = x + Lx y; legs U, D, L, R; bonds: horizontal row-major,
// then vertical row-major; colours H-even, H-odd, V-even, V-odd)
void build_topology(const hpt_config& c, std::vector<SiteInfo>& sites, std::vector<BondInfo>& bonds) {
  const int Lx = c.Lx, Ly = c.Ly;
  sites.assign(Lx * Ly, SiteInfo{});
  bonds.clear();
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x + 1 < Lx; ++x) bonds.push_back(BondInfo{x + Lx * y, x + 1 + Lx * y, x % 2, 0, 0});
  for (int y = 0; y + 1 < Ly; ++y)
    for (int x = 0; x < Lx; ++x) bonds.push_back(BondInfo{x + Lx * y, x + Lx * (y + 1), 2 + y % 2, 0, 0});
  auto find_bond = [&](int a, int b) {
    for (size_t i = 0; i < bonds.size(); ++i)
      if ((bonds[i].v1 == a && bonds[i].v2 == b) || (bonds[i].v1 == b && bonds[i].v2 == a)) return (int)i;
    return -1;
  };
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x < Lx; ++x) {
      const int v = x + Lx * y;
      SiteInfo& s = sites[v];
      s.deg = 0;
      const int nx[4] = {x, x, x - 1, x + 1}, ny[4] = {y - 1, y + 1, y, y};
      for (int l = 0; l < 4; ++l) {
        if (nx[l] < 0 || nx[l] >= Lx || ny[l] < 0 || ny[l] >= Ly) continue;
        const int u = nx[l] + Lx * ny[l];
        s.bond[s.deg] = find_bond(v, u);
        s.nbr[s.deg] = u;
        s.deg++;
      }
    }
  for (auto& b : bonds) {
    for (int l = 0; l < sites[b.v1].deg; ++l)
      if (sites[b.v1].nbr[l] == b.v2) b.pos1 = l;
    for (int l = 0; l < sites[b.v2].deg; ++l)
      if (sites[b.v2].nbr[l] == b.v1) b.pos2 = l;
  }
}

int validate(const hpt_config* c) {
  if (!c) return HPT_EINVAL;
  if (c->Lx < 1 || c->Ly < 1 || (int64_t)c->Lx * c->Ly < 2 || (int64_t)c->Lx * c->Ly > 1024) return HPT_EINVAL;
  if (!(c->dt != 0.0) || !std::isfinite(c->dt) || !std::isfinite(c->J) || !std::isfinite(c->h)) return HPT_EINVAL;
  if (c->chi_max < 1 || c->chi_max > 256) return HPT_EINVAL;
  const int cx = c->cx < 0 ? (c->Lx - 1) / 2 : c->cx, cy = c->cy < 0 ? (c->Ly - 1) / 2 : c->cy;
  if (cx >= c->Lx || cy >= c->Ly) return HPT_EINVAL;
  if (c->precision != HPT_FP64 && c->precision != HPT_FP32_MFMA && c->precision != HPT_FP32_BF16X6) return HPT_EINVAL;
  if (c->qr_mode != HPT_QR_ADAPTIVE && c->qr_mode != HPT_QR_HOUSEHOLDER) return HPT_EINVAL;
  if (c->chol_min_ratio < 1 || c->chol_min_cols < 1) return HPT_EINVAL;
  if (!(c->eps_cut < 1.0) || !(c->eps_pinv >= 0.0)) return HPT_EINVAL;
  if (!(c->bp_alpha > 0.0 && c->bp_alpha <= 1.0) || !(c->bp_tol > 0.0) || c->bp_max_sweeps < 1) return HPT_EINVAL;
  if (c->meas_alpha > 1.0) return HPT_EINVAL;
  if (!(c->qr_rank_tol < 1.0)) return HPT_EINVAL;
  if (c->trap_retry != 0 && c->trap_retry != 1) return HPT_EINVAL;
  if (c->trap_alpha > 1.0 || c->trap_sweeps < 1) return HPT_EINVAL;
  if (c->bp_init != HPT_BP_UNIFORM && c->bp_init != HPT_BP_WARM) return HPT_EINVAL;
  if (c->meas_init != HPT_BP_UNIFORM && c->meas_init != HPT_BP_LEARNED) return HPT_EINVAL;
  if (c->meas_graph != 0 && c->meas_graph != 1) return HPT_EINVAL;
  if (c->model_axes != HPT_AXES_PAPER && c->model_axes != HPT_AXES_ZZX) return HPT_EINVAL;
  if (c->svd_max_sweeps < 0) return HPT_EINVAL;
  // the storage of one interior site must stay addressable with 64-bit offsets
  // and its element count below 2^40
  const int maxdeg = (c->Lx >= 3 && c->Ly >= 3) ? 4 : ((c->Lx >= 3 || c->Ly >= 3) ? 3 : 2);
  if (4.0 * std::pow((double)c->chi_max, maxdeg) > 1.0e12) return HPT_EINVAL;
  return HPT_OK;
}

struct SlotSizes {
  uint64_t bytes;
};

// Walk the slot layout; when base != nullptr fill the pointers.
uint64_t slot_layout(int C, bool fp32, char* base, BondSlot* sl) {
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = align_up(off + bytes);
    return base ? (void*)(base + o) : nullptr;
  };
  const uint64_t C2 = (uint64_t)C * C, n4 = 4ull * C;
  for (int i = 0; i < 2; ++i)
    for (int e = 0; e < 3; ++e) {
      void* a = take(C2 * 8);
      void* b = take(C2 * 8);
      void* c = fp32 ? take(C2 * 4) : nullptr;
      void* d = fp32 ? take(C2 * 4) : nullptr;
      void* w = take(2 * C2 * 8);
      if (sl) {
        sl->S[i][e] = (double*)a;
        sl->Sinv[i][e] = (double*)b;
        sl->S32[i][e] = (float*)c;
        sl->Sinv32[i][e] = (float*)d;
        sl->eigwork[i][e] = (double*)w;
      }
    }
  void* nc = take(64);
  if (sl) sl->ncut = (int*)nc;
  for (int i = 0; i < 2; ++i) {
    void* r = take(n4 * n4 * 8);
    void* ri = take(n4 * n4 * 8);
    void* b = take(4 * n4 * n4 * 8);
    void* t = take(n4 * n4 * 8);
    void* mf = take(4 * n4 * (uint64_t)C * 8);
    void* mp = take(n4 * n4 * 8);
    void* w = take(n4 * n4 * 8);
    void* w32 = fp32 ? take(n4 * n4 * 4) : nullptr;
    if (sl) {
      sl->R[i] = (double*)r;
      sl->Rinv[i] = (double*)ri;
      sl->B[i] = (double*)b;
      sl->Tm[i] = (double*)t;
      sl->Mf[i] = (double*)mf;
      sl->Mp[i] = (double*)mp;
      sl->W[i] = (double*)w;
      sl->W32[i] = (float*)w32;
    }
  }
  void* tau = take(2 * n4 * 8);
  void* G = take(n4 * n4 * 8);
  void* V = take(n4 * n4 * 8);
  void* s = take(n4 * 8);
  void* perm = take(n4 * 4);
  void* Uc = take(n4 * (uint64_t)C * 8);
  void* Vc = take(n4 * (uint64_t)C * 8);
  void* z = take(n4 * 4 * 8);
  void* lam = take((uint64_t)C * 8);
  void* sst = take(64);
  for (int a = 0; a < 4; ++a) {
    void* q = take(n4 * n4 * 8);
    if (sl) sl->pq[a] = (double*)q;
  }
  for (int i = 0; i < 2; ++i) {
    for (int a = 0; a < 8; ++a) {
      void* q = fp32 ? take(n4 * n4 * 8) : nullptr;
      if (sl) sl->qa[i][a] = (double*)q;
    }
    void* qs = fp32 ? take(n4 * 4) : nullptr;
    void* qi = fp32 ? take(64) : nullptr;
    if (sl) {
      sl->qsel[i] = (int*)qs;
      sl->qinfo[i] = (int*)qi;
    }
  }
  if (sl) {
    sl->svd_state = (int*)sst;
    sl->tau = (double*)tau;
    sl->G = (double*)G;
    sl->V = (double*)V;
    sl->s = (double*)s;
    sl->perm = (int*)perm;
    sl->Uc = (double*)Uc;
    sl->Vc = (double*)Vc;
    sl->z = (double*)z;
    sl->lam = (double*)lam;
  }
  return off;
}

void make_carve(const hpt_config& c, Carve& cv) {
  std::vector<SiteInfo> sites;
  std::vector<BondInfo> bonds;
  build_topology(c, sites, bonds);
  const bool fp32 = c.precision != HPT_FP64;
  const uint64_t E = fp32 ? 4 : 8;
  const int C = c.chi_max;
  const int N = (int)sites.size(), nb = (int)bonds.size();
  uint64_t off = 0;
  int64_t tcap = 4;
  for (int v = 0; v < N; ++v) {
    const int64_t cap = 4 * ipow(C, sites[v].deg);
    tcap = std::max(tcap, cap);
    cv.psi_off[v] = off;
    off = align_up(off + cap * E);
  }
  cv.psi_off[N] = off;
  const uint64_t C2 = (uint64_t)C * C;
  cv.gmsg = off; off = align_up(off + 2ull * nb * C2 * 8);
  cv.gmsg_hat = off; off = align_up(off + 2ull * nb * C2 * 8);
  cv.gmsg32 = off; off = align_up(off + (fp32 ? 2ull * nb * C2 * 4 : 0));
  cv.mmsg = off; off = align_up(off + 2ull * nb * C * 8);
  cv.mmsg_hat = off; off = align_up(off + 2ull * nb * C * 8);
  cv.tcap = tcap;
  for (int i = 0; i < 3; ++i) {
    cv.t[i] = off;
    off = align_up(off + tcap * E);
  }
  const int64_t n4 = 4ll * C;
  cv.part_cap = std::max<int64_t>(1 << 22, 64 * n4 * n4);
  cv.part = off; off = align_up(off + cv.part_cap * 8);
  const int maxdeg = std::max(1, [&] { int d = 0; for (auto& s : sites) d = std::max(d, s.deg); return d; }());
  // measurement scratch: per site the contracted slice P (chi^(deg-1)), the
  // block partials of the last leg and the small contraction vectors, for
  // every site at once
  int64_t mneed = 0;
  for (auto& st : sites) mneed += 2 * ipow(C, std::max(st.deg - 1, 0)) + 4 * C * C + 64 * C + 64;
  cv.meas_scr_cap = std::max<int64_t>(1 << 20, mneed);
  (void)maxdeg;
  cv.meas_scr = off; off = align_up(off + cv.meas_scr_cap * 8);
  int mcb = 1;
  for (int col = 0; col < 4; ++col) {
    int n = 0;
    for (auto& b : bonds) n += b.colour == col;
    mcb = std::max(mcb, n);
  }
  cv.max_colour_bonds = mcb;
  cv.slot_bytes = slot_layout(C, fp32, nullptr, nullptr);
  cv.slots = off; off = align_up(off + cv.slot_bytes * mcb);
  cv.chol = off; off = align_up(off + 7 * n4 * n4 * 8 + n4 * n4 * 4 + 4 * n4 * 8 + n4 * 4 + 256);
  cv.small = off; off = align_up(off + (uint64_t)(N + nb + 64) * 8 + 2ull * nb * 8 + 16 * 8 +
                                 (uint64_t)mcb * sizeof(BondCore));
  cv.jobs_bytes = 4ull << 20;
  cv.jobs = off; off = align_up(off + cv.jobs_bytes);
  cv.learn_rows = 2ll * nb * C;
  cv.learn = off;
  off = align_up(off + (uint64_t)cv.learn_rows * (LEARN_F + 2) * 4);
  off = align_up(off + (uint64_t)cv.learn_rows * 8 + (uint64_t)nb * C * 8);
  cv.total = off;
}

// ---------------------------------------------------------------------------
// job staging: host pinned mirror -> device, bump allocation between syncs
int sync_stream(hpt_sim* s) {
  HPT_HIP(hipStreamSynchronize(s->stream));
  s->jobs_used = 0;
  return 0;
}

// elapsed milliseconds between two recorded events (waits for the second)
int event_ms(hipEvent_t a, hipEvent_t b, double* ms) {
  HPT_HIP(hipEventSynchronize(b));
  float f = 0.0f;
  HPT_HIP(hipEventElapsedTime(&f, a, b));
  *ms = f;
  return 0;
}

template <typename J>
int stage(hpt_sim* s, const J* host, int n, J** dev) {
  const uint64_t bytes = align_up(sizeof(J) * (uint64_t)std::max(n, 1));
  if (s->jobs_used + bytes > s->cv.jobs_bytes) {
    int rc = sync_stream(s);
    if (rc) return rc;
    if (bytes > s->cv.jobs_bytes) return HPT_ENOMEM;
  }
  std::memcpy(s->jobs_host + s->jobs_used, host, sizeof(J) * n);
  HPT_HIP(hipMemcpyAsync(s->jobs_dev + s->jobs_used, s->jobs_host + s->jobs_used, sizeof(J) * n,
                         hipMemcpyHostToDevice, s->stream));
  *dev = (J*)(s->jobs_dev + s->jobs_used);
  s->jobs_used += bytes;
  return 0;
}

#define RC(x)            \
  do {                   \
    int _r = (x);        \
    if (_r) return _r;   \
  } while (0)

int kres(int r) { return r == 0 ? 0 : (r == -3 ? HPT_EHIP : (r == -2 ? HPT_ENOMEM : HPT_EINVAL)); }
#define KR(x) RC(kres(x))

// ---------------------------------------------------------------------------
// contractions through the MFMA GEMM

// out[.., a, ..] = sum_b S[a, b] src[.., b, ..] on axis `axis` of a
// column-major tensor with dims[0..nd-1]
template <typename T>
int mode_product(hpt_sim* s, const T* src, T* dst, const int64_t* dims, int nd, int axis, const T* S) {
  int64_t inner = 1, outer = 1;
  for (int i = 0; i < axis; ++i) inner *= dims[i];
  for (int i = axis + 1; i < nd; ++i) outer *= dims[i];
  const int n = (int)dims[axis];
  if (sizeof(T) == 4) {
    // float32 form: the factor is resident in LDS
    const int r = mode_product_f32((const float*)S, (const float*)src, (float*)dst, n, inner, outer, s->stream);
    KR(r < 0 ? r : 0);
    if (r == 1) return 0;
  }
  GemmDesc<T> d{};
  if (inner == 1) {
    d.M = n; d.N = (int)outer; d.K = n; d.R = 1; d.Z = 1;
    d.A = S; d.lda = n; d.tA = 0;
    d.B = src; d.ldb = n; d.tB = 0;
    d.C = dst; d.ldc = n; d.c_double = 0;
  } else {
    d.M = (int)inner; d.N = n; d.K = n; d.R = 1; d.Z = (int)outer;
    d.A = src; d.lda = inner; d.sAz = inner * n; d.tA = 0;
    d.B = S; d.ldb = n; d.sBz = 0; d.tB = 1;
    d.C = dst; d.ldc = inner; d.sCz = inner * n; d.c_double = 0;
  }
  d.alpha = 1.0; d.beta = 0.0;
  KR(gemm<T>(d, s->part, s->cv.part_cap, s->stream));
  return 0;
}

// out[a, a'] = sum over every other index of psi[.., a, ..] cur[.., a', ..]
template <typename T>
int leg_gram(hpt_sim* s, const T* psi, const T* cur, const int64_t* dims, int nd, int axis, double* out) {
  int64_t inner = 1, outer = 1;
  for (int i = 0; i < axis; ++i) inner *= dims[i];
  for (int i = axis + 1; i < nd; ++i) outer *= dims[i];
  const int n = (int)dims[axis];
  if (sizeof(T) == 4) {
    const int r = leg_gram_f32((const float*)psi, (const float*)cur, n, inner, outer, out, s->part, s->cv.part_cap,
                               s->stream);
    KR(r < 0 ? r : 0);
    if (r == 1) return 0;
  }
  GemmDesc<T> d{};
  if (inner == 1) {
    d.M = n; d.N = n; d.K = (int)outer; d.R = 1; d.Z = 1;
    d.A = psi; d.lda = n; d.tA = 0;
    d.B = cur; d.ldb = n; d.tB = 1;
  } else {
    d.M = n; d.N = n; d.K = (int)inner; d.R = (int)outer; d.Z = 1;
    d.A = psi; d.lda = inner; d.sAr = inner * n; d.tA = 1;
    d.B = cur; d.ldb = inner; d.sBr = inner * n; d.tB = 0;
  }
  d.C = out; d.ldc = n; d.c_double = 1;
  d.alpha = 1.0; d.beta = 0.0;
  KR(gemm<T>(d, s->part, s->cv.part_cap, s->stream));
  return 0;
}

// C (m x n, double or T) = A (m x k) * B (k x n), plain column-major
template <typename T>
int matmul(hpt_sim* s, int64_t m, int64_t n, int64_t k, const T* A, int64_t lda, int tA, const T* B,
           int64_t ldb, int tB, void* C, int64_t ldc, int c_double) {
  GemmDesc<T> d{};
  d.M = (int)m; d.N = (int)n; d.K = (int)k; d.R = 1; d.Z = 1;
  d.A = A; d.lda = lda; d.tA = tA;
  d.B = B; d.ldb = ldb; d.tB = tB;
  d.C = C; d.ldc = ldc; d.c_double = c_double;
  d.alpha = 1.0; d.beta = 0.0;
  d.bsplit = s->bsplit;
  KR(gemm<T>(d, s->part, s->cv.part_cap, s->stream));
  return 0;
}

// G (n x n, double) = X^T X for X (m x n, column-major), as a SYRK
template <typename T>
int gram(hpt_sim* s, int64_t n, int64_t m, const T* X, int64_t ldx, double* G) {
  GemmDesc<T> d{};
  d.M = (int)n; d.N = (int)n; d.K = (int)m; d.R = 1; d.Z = 1;
  d.A = X; d.lda = ldx; d.tA = 1;
  d.B = X; d.ldb = ldx; d.tB = 0;
  d.C = G; d.ldc = n; d.c_double = 1;
  d.alpha = 1.0; d.beta = 0.0; d.sym = 1;
  d.acc64 = 1;  // products of float data accumulated in float64
  KR(gemm<T>(d, s->part, s->cv.part_cap, s->stream));
  return 0;
}

template <typename T> T* psi_of(hpt_sim* s, int v) { return (T*)s->sites[v].psi; }

void site_dims(hpt_sim* s, int v, int64_t* dims) {
  const SiteInfo& si = s->sites[v];
  for (int l = 0; l < si.deg; ++l) dims[l] = s->chi[si.bond[l]];
  dims[si.deg] = 4;
}

double* gmsg_slot(hpt_sim* s, int b, int dir) {
  return s->gmsg + (uint64_t)(2 * b + dir) * s->chi_max * s->chi_max;
}
double* gmsg_hat_slot(hpt_sim* s, int b, int dir) {
  return s->gmsg_hat + (uint64_t)(2 * b + dir) * s->chi_max * s->chi_max;
}
float* gmsg32_slot(hpt_sim* s, int b, int dir) {
  return s->gmsg32 + (uint64_t)(2 * b + dir) * s->chi_max * s->chi_max;
}
double* mmsg_slot(hpt_sim* s, int b, int dir) { return s->mmsg + (uint64_t)(2 * b + dir) * s->chi_max; }
double* mmsg_hat_slot(hpt_sim* s, int b, int dir) { return s->mmsg_hat + (uint64_t)(2 * b + dir) * s->chi_max; }
// direction index of the message leaving `src` along bond b
int dir_from(hpt_sim* s, int b, int src) { return s->bonds[b].v1 == src ? 0 : 1; }

// ---------------------------------------------------------------------------
// field half-step (Sec. "Trotter Decomposition", Eq. trotter)
template <typename T>
int apply_field_t(hpt_sim* s) {
  for (int v = 0; v < s->N; ++v) {
    int64_t dims[5];
    site_dims(s, v, dims);
    int64_t slice = 1;
    for (int l = 0; l < s->sites[v].deg; ++l) slice *= dims[l];
    KR(launch_field<T>(psi_of<T>(s, v), slice, s->g1[0], s->g1[1], s->g1[2], s->g1[3], s->stream));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// gate update (Algorithm "Gate update") of every bond of one colour
struct SitePlan {
  int v, cut, deg;
  int64_t dims[5];
  int nenv;
  int env_pos[3];
  int64_t m, n;
  int chol;
  int k;
  int deferred;     // float32 form: Gram taken, CholeskyQR2 algebra pending
  int was_deferred;
  int pinv_cut;     // an environment eigenvalue of this site was dropped
  int direct;       // float32 form, direct route: the storage holds the permuted,
                    // unabsorbed psi and the reconstruction multiplies it (no deabsorb)
};

template <typename T>
int phase_a_finish(hpt_sim* s, int i, BondSlot& sl, SitePlan& P);

template <typename T>
const T* env_S(BondSlot& sl, int i, int e, bool inv);
template <>
const double* env_S<double>(BondSlot& sl, int i, int e, bool inv) { return inv ? sl.Sinv[i][e] : sl.S[i][e]; }
template <>
const float* env_S<float>(BondSlot& sl, int i, int e, bool inv) { return inv ? sl.Sinv32[i][e] : sl.S32[i][e]; }

// Environment factor (sqrt(M) when inv is false, its pseudo-inverse when
// true) on one axis.  Float64 form: MFMA products in float64.  Float32 form:
// float64 factors in float64 arithmetic on the float32 data, so that an
// absorb/deabsorb pair multiplies to the projector to float64 accuracy.
template <typename T>
int env_product(hpt_sim* s, const T* src, T* dst, const int64_t* dims, int nd, int axis, BondSlot& sl, int i, int e,
                bool inv) {
  if constexpr (std::is_same<T, float>::value) {
    int64_t inner = 1, outer = 1;
    for (int q = 0; q < axis; ++q) inner *= dims[q];
    for (int q = axis + 1; q < nd; ++q) outer *= dims[q];
    KR(mode_product_f64acc(inv ? sl.Sinv[i][e] : sl.S[i][e], src, dst, (int)dims[axis], inner, outer, s->stream));
    return 0;
  } else {
    return mode_product<T>(s, src, dst, dims, nd, axis, env_S<T>(sl, i, e, inv));
  }
}

// dims of a site tensor with the cut leg moved next to the Pauli leg
void permuted_dims(const SitePlan& P, int64_t* pd) {
  int q = 0;
  for (int l = 0; l < P.deg; ++l)
    if (l != P.cut) pd[q++] = P.dims[l];
  pd[q++] = P.dims[P.cut];
  pd[q] = 4;
}

// Puts the tensor held in temporary ti into site v's storage.  The largest
// sites' storage and the temporaries are arena slices of the same size, so
// there the two slices trade places (the site's old storage becomes the
// temporary); smaller sites take a device copy of `bytes`.  Site storage is
// always reached through psi_of, never through a cached address.
int adopt_temp(hpt_sim* s, int v, int ti, uint64_t bytes) {
  SiteInfo& si = s->sites[v];
  if (si.cap == s->cv.tcap) {
    std::swap(si.psi, s->t[ti]);
    return 0;
  }
  HPT_HIP(hipMemcpyAsync(si.psi, s->t[ti], bytes, hipMemcpyDeviceToDevice, s->stream));
  return 0;
}

// Float32 form, direct route (a tall block for CholeskyQR2 and no environment
// eigenvalue dropped): Xraw = psi with the cut leg moved next to the Pauli leg
// is kept in the site's storage; its absorbed copy X = Xraw x_e sqrt(M_e)
// (float32 MFMA products) lives in a temporary only for the float64 Gram
// G1 = X^T X and the sign projection.  The reconstruction later multiplies
// Xraw itself: the environment products act on the rows of X and the
// reconstruction W on its columns, so (X W) x_e sqrt(M_e)^-1 = Xraw W
// exactly, and no deabsorb is needed.  (A float32 deabsorb factor would leave
// sqrt(M) sqrt(M)^-1 = 1 + O(eps32) on every environment leg of every gate, a
// coherent error that moves C(t) by a few 1e-6 over a 10x10 run.)
int phase_a_direct(hpt_sim* s, int i, BondSlot& sl, SitePlan& P) {
  float* psi = psi_of<float>(s, P.v);
  const int n = (int)P.n;
  const int64_t m = P.m;
  int64_t pd[5];
  permuted_dims(P, pd);
  float* xraw = psi;
  const bool need_perm = P.cut != P.deg - 1;
  if (need_perm) {
    int64_t A = 1, Cc = 1;
    for (int l = 0; l < P.cut; ++l) A *= P.dims[l];
    for (int l = P.cut + 1; l < P.deg; ++l) Cc *= P.dims[l];
    xraw = (float*)s->t[2];
    KR(permute_swap_mid(psi, xraw, A, P.dims[P.cut], Cc, 4, (int)sizeof(float), s->stream));
  }
  const float* X = xraw;
  int ti = 0;
  for (int e = 0; e < P.nenv; ++e) {
    float* dst = (float*)s->t[ti];
    ti ^= 1;
    RC(mode_product<float>(s, X, dst, pd, P.deg + 1, e, sl.S32[i][e]));
    X = dst;
  }
  RC(gram<float>(s, n, m, X, m, sl.qa[i][0]));
  if (i == 0) KR(launch_sign_projection<float>(X, m, m, n, sl.z, s->part, s->cv.part_cap, s->stream));
  if (need_perm) RC(adopt_temp(s, P.v, 2, sizeof(float) * m * n));
  P.direct = 1;
  P.deferred = 1;
  P.was_deferred = 1;
  return 0;
}

// A direct-route block whose CholeskyQR2 failed goes to Householder: absorb
// its environment in place (float64 factors), after which the block is an
// ordinary one (Q of X, deabsorb after the reconstruction).
int direct_to_framed(hpt_sim* s, int i, BondSlot& sl, SitePlan& P) {
  float* psi = psi_of<float>(s, P.v);
  int64_t pd[5];
  permuted_dims(P, pd);
  const float* src = psi;
  int ti = 0;
  for (int e = 0; e < P.nenv; ++e) {
    float* dst = (float*)s->t[ti];
    ti ^= 1;
    RC(env_product<float>(s, src, dst, pd, P.deg + 1, e, sl, i, e, false));
    src = dst;
  }
  if (src != psi) HPT_HIP(hipMemcpyAsync(psi, src, sizeof(float) * P.m * P.n, hipMemcpyDeviceToDevice, s->stream));
  P.direct = 0;
  return 0;
}

template <typename T>
int phase_a_site(hpt_sim* s, int b, int i, BondSlot& sl, SitePlan& P, uint32_t& flags) {
  const BondInfo& bi = s->bonds[b];
  const T* S_unused = nullptr;
  (void)S_unused;
  T* psi = psi_of<T>(s, P.v);
  P.direct = 0;
  P.deferred = 0;
  P.was_deferred = 0;
  const bool tall = s->cfg.qr_mode == HPT_QR_ADAPTIVE && P.m >= (int64_t)s->cfg.chol_min_ratio * P.n &&
                    P.n >= s->cfg.chol_min_cols;
  if constexpr (std::is_same<T, float>::value) {
    if (tall && !P.pinv_cut) return phase_a_direct(s, i, sl, P);
  }
  // absorb sqrt of each environment message (mode products, ping-pong)
  int64_t dims[5];
  for (int l = 0; l <= P.deg; ++l) dims[l] = P.dims[l];
  const T* src = psi;
  int ti = 0;
  const bool need_perm = P.cut != P.deg - 1;
  for (int e = 0; e < P.nenv; ++e) {
    const bool last = e == P.nenv - 1;
    T* dst;
    if (last && !need_perm && src != psi)
      dst = psi;
    else {
      dst = (T*)s->t[ti];
      ti ^= 1;
    }
    RC(env_product<T>(s, src, dst, dims, P.deg + 1, P.env_pos[e], sl, i, e, false));
    src = dst;
  }
  // permute [A, cut, C, P] -> [A, C, cut, P] into the site's own storage
  if (need_perm) {
    int64_t A = 1, Cc = 1;
    for (int l = 0; l < P.cut; ++l) A *= dims[l];
    for (int l = P.cut + 1; l < P.deg; ++l) Cc *= dims[l];
    T* dst = psi;
    if (src == psi) {  // no environment legs were absorbed: permute via a temp
      HPT_HIP(hipMemcpyAsync(s->t[0], psi, sizeof(T) * P.m * P.n, hipMemcpyDeviceToDevice, s->stream));
      src = (T*)s->t[0];
    }
    KR(permute_swap_mid(src, dst, A, dims[P.cut], Cc, 4, (int)sizeof(T), s->stream));
  } else if (src != psi) {
    HPT_HIP(hipMemcpyAsync(psi, src, sizeof(T) * P.m * P.n, hipMemcpyDeviceToDevice, s->stream));
  }
  // QR of X (m x n) held in psi's storage
  const int n = (int)P.n;
  const int64_t m = P.m;
  const int ldR = 4 * s->chi_max;
  P.chol = 0;
  const bool use_chol = tall;
  if (use_chol && s->fp32) {
    // float32 form: only the Gram here; the float64 algebra of every block of
    // the colour runs batched afterwards
    RC(gram<T>(s, n, m, psi, m, sl.qa[i][0]));
    P.deferred = 1;
    P.was_deferred = 1;
    return 0;
  }
  if (use_chol) {
    // rank-revealing CholeskyQR2: G1 = X^T X; pivoted Cholesky R1 (rank r,
    // exact structural zeros deflated); Q1 = X W1 with W1 = E_sel R1sel^{-1};
    // G2 = Q1^T Q1 = R2^T R2.  Then X = (Q1 R2^{-1}) (R2 R1) and Q = X W1 R2^{-1}.
    RC(gram<T>(s, n, m, psi, m, s->G1));
    // with tolerance 0 the pivoted factorisation stops at the first pivot
    // below 1e-13 of the largest and the block goes to Householder instead;
    // with a positive tolerance a failed second pass is retried with the
    // tolerance raised 100-fold (twice) before Householder is used
    const bool deflate = s->cfg_qr_tol > 0.0;
    double tol = deflate ? s->cfg_qr_tol : 1e-13;
    for (int attempt = 0; attempt < (deflate ? 3 : 1) && !P.chol; ++attempt, tol *= 100.0) {
    PivCholJob pj{s->G1, n, n, s->R1, n, s->sel, s->info + 1, tol};
    PivCholJob* pjd;
    RC(stage(s, &pj, 1, &pjd));
    KR(launch_piv_cholesky(pjd, 1, s->stream));
    HPT_HIP(hipMemcpyAsync(s->hscratch, s->info + 1, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    RC(sync_stream(s));
    int r = 0;
    std::memcpy(&r, s->hscratch, sizeof(int));
    if (r >= 1 && (deflate || r == n)) {
      if (r < n) flags |= HPT_FLAG_QR_RANK_DEFICIENT;
      SelJob g0{0, s->R1, n, s->G2, r, s->sel, r, n};
      SelJob* sjd;
      RC(stage(s, &g0, 1, &sjd));
      KR(launch_sel(sjd, 1, s->stream));
      TriInvJob tj{s->G2, r, r, s->Ri1, r, nullptr};
      TriInvJob* tjd;
      RC(stage(s, &tj, 1, &tjd));
      KR(launch_tri_inverse(tjd, 1, s->stream, 4 * s->chi_max));
      SelJob g1{1, s->Ri1, r, s->W1, n, s->sel, r, n};
      RC(stage(s, &g1, 1, &sjd));
      KR(launch_sel(sjd, 1, s->stream));
      const T* W1;
      if (sizeof(T) == 4) {
        KR(launch_d2f(s->W1, s->Ri32, (int64_t)n * r, s->stream));
        W1 = (const T*)s->Ri32;
      } else {
        W1 = (const T*)s->W1;
      }
      T* Q1 = (T*)s->t[0];
      RC(matmul<T>(s, m, r, n, psi, m, 0, W1, n, 0, Q1, m, 0));
      RC(gram<T>(s, r, m, Q1, m, s->G2));
      CholJob cj2{s->G2, r, r, s->R2, r, s->info, nullptr};
      CholJob* cjd;
      RC(stage(s, &cj2, 1, &cjd));
      KR(launch_cholesky(cjd, 1, 1e-13, s->stream));
      HPT_HIP(hipMemcpyAsync(s->hscratch, s->info, sizeof(int), hipMemcpyDeviceToHost, s->stream));
      RC(sync_stream(s));
      int info = 0;
      std::memcpy(&info, s->hscratch, sizeof(int));
      if (info == 0) {
        TriInvJob tj2{s->R2, r, r, s->Ri2, r, nullptr};
        RC(stage(s, &tj2, 1, &tjd));
        KR(launch_tri_inverse(tjd, 1, s->stream, 4 * s->chi_max));
        // R = R2 R1 (r x n, ld 4 chi_max), Rinv = W1 R2^{-1} (n x r)
        SmallGemmJob gj[2];
        std::memset(gj, 0, sizeof(gj));
        gj[0] = SmallGemmJob{r, n, r, nullptr, nullptr, nullptr, s->R2, r, 0, s->R1, n, 0, sl.R[i], ldR, 1.0, 0.0, nullptr};
        gj[1] = SmallGemmJob{n, r, r, nullptr, nullptr, nullptr, s->W1, n, 0, s->Ri2, r, 0, sl.Rinv[i], ldR, 1.0, 0.0, nullptr};
        SmallGemmJob* gjd;
        RC(stage(s, gj, 2, &gjd));
        KR(launch_small_gemm(gjd, gj, 2, s->stream));
        P.chol = 1;
        P.k = r;
      }
    }
    }
    if (!P.chol) flags |= HPT_FLAG_QR_FALLBACK;
  }
  (void)bi;
  return phase_a_finish<T>(s, i, sl, P);
}

// Householder QR of X when the Cholesky route was not taken or failed, then
// the sign projections of S_0 (X_0 or Q_0)
template <typename T>
int phase_a_finish(hpt_sim* s, int i, BondSlot& sl, SitePlan& P) {
  T* psi = psi_of<T>(s, P.v);
  const int n = (int)P.n;
  const int64_t m = P.m;
  if constexpr (std::is_same<T, float>::value) {
    if (P.direct) {
      if (P.chol) return 0;   // sign projection taken with the Gram
      RC(direct_to_framed(s, i, sl, P));
    }
  }
  if (!P.chol) {
    if (std::min<int64_t>(m, n) > 1024) return HPT_EINVAL;
    QrJob<T> qj{psi, m, (int)m, n, sl.R[i], 4 * s->chi_max, s->R1 /* tau scratch */, 1, nullptr, 0};
    QrJob<T>* qjd;
    RC(stage(s, &qj, 1, &qjd));
    KR(launch_householder<T>(qjd, 1, s->stream));
    P.k = (int)std::min<int64_t>(m, n);
  }
  if (i == 0) {
    const int ncols = P.chol ? n : P.k;
    KR(launch_sign_projection<T>(psi, m, m, ncols, sl.z, s->part, s->cv.part_cap, s->stream));
  }
  return 0;
}

// float32 form: the float64 algebra of the rank-revealing CholeskyQR2 of every
// deferred block of the colour, batched one workgroup per block.  With G1 =
// X^T X already formed: pivoted Cholesky R1 (rank r); W1 = E_sel R1sel^{-1};
// the second pass takes its Gram algebraically, G2 = W1^T G1 W1 = R2^T R2, in
// float64 rather than from an explicit float32 Q1 = X W1 (whose rounding would
// only add noise: Q is never formed, X W1 R2^{-1} is the basis used).  Then
// R = R2 R1 and Rinv = W1 R2^{-1}.  A block whose second Cholesky fails is
// retried with the deflation tolerance raised 100-fold (twice), then goes to
// Householder.
template <typename T>
int phase_a_batched(hpt_sim* s, std::vector<SitePlan>& plans, uint32_t& flags) {
  std::vector<int> pend;
  for (int p = 0; p < (int)plans.size(); ++p)
    if (plans[p].deferred) pend.push_back(p);
  const int ldR = 4 * s->chi_max;
  const bool deflate = s->cfg_qr_tol > 0.0;
  double tol = deflate ? s->cfg_qr_tol : 1e-13;
  for (int attempt = 0; attempt < (deflate ? 3 : 1) && !pend.empty(); ++attempt, tol *= 100.0) {
    const int np = (int)pend.size();
    std::vector<PivCholJob> pj;
    for (int p : pend) {
      BondSlot& sl = s->slots[p / 2];
      const int i = p % 2, n = (int)plans[p].n;
      pj.push_back(PivCholJob{sl.qa[i][0], n, n, sl.qa[i][1], n, sl.qsel[i], sl.qinfo[i] + 1, tol});
    }
    PivCholJob* pjd;
    RC(stage(s, pj.data(), np, &pjd));
    KR(launch_piv_cholesky(pjd, np, s->stream));
    for (int a = 0; a < np; ++a)
      HPT_HIP(hipMemcpyAsync(s->hscratch + 4 * a, s->slots[pend[a] / 2].qinfo[pend[a] % 2] + 1, sizeof(int),
                             hipMemcpyDeviceToHost, s->stream));
    RC(sync_stream(s));
    std::vector<int> rank(np), go;
    std::memcpy(rank.data(), s->hscratch, sizeof(int) * np);
    for (int a = 0; a < np; ++a) {
      const int r = rank[a], n = (int)plans[pend[a]].n;
      if (r >= 1 && r <= n && (deflate || r == n)) go.push_back(a);
    }
    std::vector<int> next;
    for (int a = 0; a < np; ++a)
      if (std::find(go.begin(), go.end(), a) == go.end()) next.push_back(pend[a]);
    if (!go.empty()) {
      const int ng = (int)go.size();
      std::vector<SelJob> gat, sca;
      std::vector<TriInvJob> ti;
      std::vector<SmallGemmJob> g1, g2;
      std::vector<CholJob> cj;
      for (int a : go) {
        const int p = pend[a], i = p % 2, r = rank[a], n = (int)plans[p].n;
        BondSlot& sl = s->slots[p / 2];
        double** q = sl.qa[i];
        gat.push_back(SelJob{0, q[1], n, q[2], r, sl.qsel[i], r, n});
        ti.push_back(TriInvJob{q[2], r, r, q[3], r, nullptr, 0});
        sca.push_back(SelJob{1, q[3], r, q[4], n, sl.qsel[i], r, n});
        SmallGemmJob a1{}, a2{};
        a1 = SmallGemmJob{n, r, n, nullptr, nullptr, nullptr, q[0], n, 0, q[4], n, 0, q[5], n, 1.0, 0.0, nullptr, 0};
        a2 = SmallGemmJob{r, r, n, nullptr, nullptr, nullptr, q[4], n, 1, q[5], n, 0, q[6], r, 1.0, 0.0, nullptr, 0};
        g1.push_back(a1);
        g2.push_back(a2);
        cj.push_back(CholJob{q[6], r, r, q[6], r, sl.qinfo[i], nullptr, 0, nullptr});
      }
      SelJob* sd;
      RC(stage(s, gat.data(), ng, &sd));
      KR(launch_sel(sd, ng, s->stream));
      TriInvJob* td;
      RC(stage(s, ti.data(), ng, &td));
      KR(launch_tri_inverse(td, ng, s->stream, 4 * s->chi_max));
      RC(stage(s, sca.data(), ng, &sd));
      KR(launch_sel(sd, ng, s->stream));
      SmallGemmJob* gd;
      RC(stage(s, g1.data(), ng, &gd));
      KR(launch_small_gemm(gd, g1.data(), ng, s->stream));
      RC(stage(s, g2.data(), ng, &gd));
      KR(launch_small_gemm(gd, g2.data(), ng, s->stream));
      CholJob* cd;
      RC(stage(s, cj.data(), ng, &cd));
      KR(launch_cholesky(cd, ng, 1e-13, s->stream));
      for (int a = 0; a < ng; ++a) {
        const int p = pend[go[a]];
        HPT_HIP(hipMemcpyAsync(s->hscratch + 4 * a, s->slots[p / 2].qinfo[p % 2], sizeof(int),
                               hipMemcpyDeviceToHost, s->stream));
      }
      RC(sync_stream(s));
      std::vector<int> info(ng);
      std::memcpy(info.data(), s->hscratch, sizeof(int) * ng);
      std::vector<TriInvJob> t2;
      std::vector<SmallGemmJob> fin;
      for (int a = 0; a < ng; ++a) {
        const int p = pend[go[a]], i = p % 2, r = rank[go[a]], n = (int)plans[p].n;
        if (info[a] != 0) {
          next.push_back(p);
          continue;
        }
        BondSlot& sl = s->slots[p / 2];
        double** q = sl.qa[i];
        t2.push_back(TriInvJob{q[6], r, r, q[7], r, nullptr, 0});
        // R = R2 R1 (r x n), Rinv = W1 R2^{-1} (n x r), both ld 4 chi_max
        fin.push_back(SmallGemmJob{r, n, r, nullptr, nullptr, nullptr, q[6], r, 0, q[1], n, 0, sl.R[i], ldR, 1.0, 0.0, nullptr, 0});
        fin.push_back(SmallGemmJob{n, r, r, nullptr, nullptr, nullptr, q[4], n, 0, q[7], r, 0, sl.Rinv[i], ldR, 1.0, 0.0, nullptr, 0});
        plans[p].chol = 1;
        plans[p].k = r;
        plans[p].deferred = 0;
        if (r < n) flags |= HPT_FLAG_QR_RANK_DEFICIENT;
      }
      if (!t2.empty()) {
        RC(stage(s, t2.data(), (int)t2.size(), &td));
        KR(launch_tri_inverse(td, (int)t2.size(), s->stream, 4 * s->chi_max));
        RC(stage(s, fin.data(), (int)fin.size(), &gd));
        KR(launch_small_gemm(gd, fin.data(), (int)fin.size(), s->stream));
      }
    }
    pend.swap(next);
  }
  for (int p : pend) {
    plans[p].deferred = 0;
    plans[p].chol = 0;
    flags |= HPT_FLAG_QR_FALLBACK;
  }
  // Householder for the blocks that failed, sign projections of every
  // deferred block's S_0
  for (int p = 0; p < (int)plans.size(); ++p) {
    SitePlan& P = plans[p];
    if (!P.was_deferred) continue;
    RC(phase_a_finish<T>(s, p % 2, s->slots[p / 2], P));
  }
  return 0;
}

template <typename T>
int phase_c_site(hpt_sim* s, int b, int i, BondSlot& sl, SitePlan& P, int cn) {
  T* psi = psi_of<T>(s, P.v);
  const int nS = P.chol ? (int)P.n : P.k;
  const int n4 = 4 * cn;
  const T* W;
  if (sizeof(T) == 4) {
    KR(launch_d2f(sl.W[i], sl.W32[i], (int64_t)nS * n4, s->stream));
    W = (const T*)sl.W32[i];
  } else {
    W = (const T*)sl.W[i];
  }
  T* out = (T*)s->t[0];
  RC(matmul<T>(s, P.m, n4, nS, psi, P.m, 0, W, nS, 0, out, P.m, 0));
  // new dims
  int64_t dims[5];
  for (int l = 0; l <= P.deg; ++l) dims[l] = P.dims[l];
  dims[P.cut] = cn;
  const T* src = out;
  int ti = 1;
  if (P.cut != P.deg - 1) {
    int64_t A = 1, Cc = 1;
    for (int l = 0; l < P.cut; ++l) A *= dims[l];
    for (int l = P.cut + 1; l < P.deg; ++l) Cc *= dims[l];
    // direct route: the reconstruction multiplied the unabsorbed psi, so the
    // inverse permutation is the last step and lands in the site's storage
    T* dst = P.direct ? psi : (T*)s->t[1];
    KR(permute_swap_mid(src, dst, A, Cc, cn, 4, (int)sizeof(T), s->stream));
    if (P.direct) return 0;
    src = dst;
    ti = 0;
  }
  if (P.direct) {   // src is the reconstruction in t[0]
    int64_t total = 4;
    for (int l = 0; l < P.deg; ++l) total *= dims[l];
    return adopt_temp(s, P.v, 0, sizeof(T) * total);
  }
  // deabsorb with the pseudo-inverse square roots; the last product lands in psi
  for (int e = 0; e < P.nenv; ++e) {
    const bool last = e == P.nenv - 1;
    T* dst = last ? psi : (T*)s->t[ti];
    RC(env_product<T>(s, src, dst, dims, P.deg + 1, P.env_pos[e], sl, i, e, true));
    if (!last) {
      src = dst;
      ti ^= 1;
    }
  }
  if (P.nenv == 0) {
    int64_t total = 4;
    for (int l = 0; l < P.deg; ++l) total *= dims[l];
    HPT_HIP(hipMemcpyAsync(psi, src, sizeof(T) * total, hipMemcpyDeviceToDevice, s->stream));
  }
  (void)b;
  return 0;
}

template <typename T>
int gate_colour(hpt_sim* s, const std::vector<int>& cbonds) {
  const int nb = (int)cbonds.size();
  if (nb == 0) return 0;
  if (nb > s->cv.max_colour_bonds) return HPT_EINVAL;
  std::vector<SitePlan> plans(2 * nb);
  uint32_t flags = 0;
  // environment pseudo square roots of every site in the colour
  std::vector<PsqJob> pj;
  for (int q = 0; q < nb; ++q) {
    const int b = cbonds[q];
    BondSlot& sl = s->slots[q];
    for (int i = 0; i < 2; ++i) {
      SitePlan& P = plans[2 * q + i];
      P.v = i == 0 ? s->bonds[b].v1 : s->bonds[b].v2;
      P.cut = i == 0 ? s->bonds[b].pos1 : s->bonds[b].pos2;
      P.deg = s->sites[P.v].deg;
      site_dims(s, P.v, P.dims);
      P.nenv = 0;
      P.m = 1;
      for (int l = 0; l < P.deg; ++l) {
        if (l == P.cut) continue;
        const int be = s->sites[P.v].bond[l];
        const int u = s->sites[P.v].nbr[l];
        const int ch = s->chi[be];
        PsqJob j{gmsg_slot(s, be, dir_from(s, be, u)), sl.S[i][P.nenv], sl.Sinv[i][P.nenv],
                 s->fp32 ? sl.S32[i][P.nenv] : nullptr, s->fp32 ? sl.Sinv32[i][P.nenv] : nullptr,
                 sl.eigwork[i][P.nenv], ch, sl.ncut + 3 * i + P.nenv};
        pj.push_back(j);
        P.env_pos[P.nenv++] = l;
        P.m *= ch;
      }
      P.n = 4ll * s->chi[b];
    }
  }
  if (!pj.empty()) {
    PsqJob* pjd;
    RC(stage(s, pj.data(), (int)pj.size(), &pjd));
    KR(launch_pseudo_sqrt(pjd, (int)pj.size(), s->cfg.eps_pinv, s->stream));
  }
  for (SitePlan& P : plans) P.pinv_cut = 0;
  if (s->fp32 && !pj.empty()) {
    // the route of each block depends on whether an environment eigenvalue
    // was dropped (the direct route needs sqrt(M) invertible on every leg)
    for (int q = 0; q < nb; ++q)
      HPT_HIP(hipMemcpyAsync(s->hscratch + 64 * q, s->slots[q].ncut, 6 * sizeof(int), hipMemcpyDeviceToHost,
                             s->stream));
    RC(sync_stream(s));
    for (int q = 0; q < nb; ++q) {
      const int* nc = (const int*)(s->hscratch + 64 * q);
      for (int i = 0; i < 2; ++i)
        for (int e = 0; e < plans[2 * q + i].nenv; ++e)
          if (nc[3 * i + e] != 0) plans[2 * q + i].pinv_cut = 1;
    }
  }
  // phase A: absorb, permute, QR
  for (int q = 0; q < nb; ++q)
    for (int i = 0; i < 2; ++i) RC(phase_a_site<T>(s, cbonds[q], i, s->slots[q], plans[2 * q + i], flags));
  if (s->fp32) RC(phase_a_batched<T>(s, plans, flags));
  // phase B: R-core of every bond of the colour
  std::vector<BondCore> cores(nb);
  const int C = s->chi_max, ldR = 4 * C;
  for (int q = 0; q < nb; ++q) {
    const int b = cbonds[q];
    BondSlot& sl = s->slots[q];
    BondCore& bc = cores[q];
    std::memset(&bc, 0, sizeof(bc));
    bc.chi_cut = s->chi[b];
    for (int i = 0; i < 2; ++i) {
      const SitePlan& P = plans[2 * q + i];
      bc.k[i] = P.k;
      bc.q[i] = std::min(4 * P.k, 4 * bc.chi_cut);
      bc.chol[i] = P.chol;
      bc.R[i] = sl.R[i];
      bc.Rinv[i] = sl.Rinv[i];
      bc.B[i] = sl.B[i];
      bc.Tm[i] = sl.Tm[i];
      bc.Mf[i] = sl.Mf[i];
      bc.Mp[i] = sl.Mp[i];
      bc.W[i] = sl.W[i];
      bc.msg[i] = gmsg_slot(s, b, i);
      // float32 form: CholeskyQR2 of B_i when it is tall (4 k_i >= 4 chi_cut)
      bc.bqr[i] = (s->fp32 && P.k >= bc.chi_cut) ? 0 : 1;
      for (int a = 0; a < 8; ++a) bc.qs[i][a] = sl.qa[i][a];
    }
    for (int a = 0; a < 4; ++a) bc.pq[a] = sl.pq[a];
    bc.chi_max = C;
    bc.eps_cut = s->cfg.eps_cut;
    bc.ldR = ldR;
    bc.ldT = ldR;
    bc.tau = sl.tau;
    bc.G = sl.G;
    bc.ldG = ldR;
    bc.V = sl.V;
    bc.s = sl.s;
    bc.perm = sl.perm;
    bc.Uc = sl.Uc;
    bc.Vc = sl.Vc;
    bc.z = sl.z;
    bc.lam = sl.lam;
  }
  // stage the records through the pinned scratch; it is next written by the
  // device-to-host copy at the end of this phase, which is stream-ordered after
  BondCore* cd = s->cores_dev;
  std::memcpy(s->hscratch, cores.data(), sizeof(BondCore) * nb);
  HPT_HIP(hipMemcpyAsync(cd, s->hscratch, sizeof(BondCore) * nb, hipMemcpyHostToDevice, s->stream));
  KR(launch_rcore_build_B(cd, nb, s->gf, s->stream));
  bool any_bchol = false;
  for (int q = 0; q < nb; ++q) any_bchol = any_bchol || cores[q].bqr[0] == 0 || cores[q].bqr[1] == 0;
  if (any_bchol) {
    // CholeskyQR2 of the tall B_i: G_B = B^T B assembled from R^T R (the gate
    // factors act on the Pauli pair only), R1 = chol(G_B), second pass taken
    // algebraically, G2 = R1^{-T} G_B R1^{-1} = R2^T R2; T_i = R2 R1 and
    // T_i^{-1} = R1^{-1} R2^{-1} (Q~_i = B_i T_i^{-1} is never formed).  A
    // failed Cholesky sets bqr[i] = 1 and B_i goes to Householder below.
    std::vector<SmallGemmJob> rtr, g1, g2, fin;
    std::vector<CholJob> c1, c2;
    std::vector<TriInvJob> t1, t2;
    for (int q = 0; q < nb; ++q)
      for (int i = 0; i < 2; ++i) {
        const BondCore& bc = cores[q];
        if (bc.bqr[i] != 0) continue;
        const int n = 4 * bc.chi_cut, k = bc.k[i];
        const int* gq = &cd[q].bqr[i];
        int* fq = &cd[q].bqr[i];
        double* const* x = bc.qs[i];
        int* info = s->slots[q].qinfo[i];
        rtr.push_back(SmallGemmJob{n, n, k, nullptr, nullptr, nullptr, bc.R[i], ldR, 1, bc.R[i], ldR, 0, x[5], n, 1.0, 0.0, gq, 1});
        c1.push_back(CholJob{x[0], n, n, x[1], n, info, gq, 1, fq});
        t1.push_back(TriInvJob{x[1], n, n, x[3], n, gq, 1});
        g1.push_back(SmallGemmJob{n, n, n, nullptr, nullptr, nullptr, x[0], n, 0, x[3], n, 0, x[4], n, 1.0, 0.0, gq, 1});
        g2.push_back(SmallGemmJob{n, n, n, nullptr, nullptr, nullptr, x[3], n, 1, x[4], n, 0, x[6], n, 1.0, 0.0, gq, 1});
        c2.push_back(CholJob{x[6], n, n, x[6], n, info, gq, 1, fq});
        t2.push_back(TriInvJob{x[6], n, n, x[7], n, gq, 1});
        fin.push_back(SmallGemmJob{n, n, n, nullptr, nullptr, nullptr, x[6], n, 0, x[1], n, 0, bc.Tm[i], ldR, 1.0, 0.0, gq, 1});
        fin.push_back(SmallGemmJob{n, n, n, nullptr, nullptr, nullptr, x[3], n, 0, x[7], n, 0, x[2], n, 1.0, 0.0, gq, 1});
      }
    const int nj = (int)c1.size();
    SmallGemmJob* gd;
    CholJob* chd;
    TriInvJob* tid;
    RC(stage(s, rtr.data(), nj, &gd));
    KR(launch_small_gemm(gd, rtr.data(), nj, s->stream));
    KR(launch_rcore_kron_gram(cd, nb, s->gf, s->stream));
    RC(stage(s, c1.data(), nj, &chd));
    KR(launch_cholesky(chd, nj, 1e-10, s->stream));
    RC(stage(s, t1.data(), nj, &tid));
    KR(launch_tri_inverse(tid, nj, s->stream, 4 * s->chi_max));
    RC(stage(s, g1.data(), nj, &gd));
    KR(launch_small_gemm(gd, g1.data(), nj, s->stream));
    RC(stage(s, g2.data(), nj, &gd));
    KR(launch_small_gemm(gd, g2.data(), nj, s->stream));
    RC(stage(s, c2.data(), nj, &chd));
    KR(launch_cholesky(chd, nj, 1e-10, s->stream));
    RC(stage(s, t2.data(), nj, &tid));
    KR(launch_tri_inverse(tid, nj, s->stream, 4 * s->chi_max));
    RC(stage(s, fin.data(), 2 * nj, &gd));
    KR(launch_small_gemm(gd, fin.data(), 2 * nj, s->stream));
  }
  {
    // Householder (explicit Q~_i into B_i) where bqr[i] != 0
    std::vector<QrJob<double>> qj;
    for (int q = 0; q < nb; ++q)
      for (int i = 0; i < 2; ++i) {
        const BondCore& bc = cores[q];
        qj.push_back(QrJob<double>{bc.B[i], 4 * bc.k[i], 4 * bc.k[i], 4 * bc.chi_cut, bc.Tm[i], ldR,
                                   s->slots[q].tau + i * 4 * C, 1, &cd[q].bqr[i], 0});
      }
    QrJob<double>* qd;
    RC(stage(s, qj.data(), (int)qj.size(), &qd));
    KR(launch_householder<double>(qd, (int)qj.size(), s->stream));
  }
  {
    std::vector<SmallGemmJob> gj;
    std::vector<SvdJob> sj;
    for (int q = 0; q < nb; ++q) {
      const BondCore& bc = cores[q];
      const int q0 = bc.q[0], q1 = bc.q[1], K = 4 * bc.chi_cut;
      SmallGemmJob j;
      std::memset(&j, 0, sizeof(j));
      if (q0 >= q1)
        j = SmallGemmJob{q0, q1, K, nullptr, nullptr, nullptr, bc.Tm[0], ldR, 0, bc.Tm[1], ldR, 1, bc.G, ldR, 1.0, 0.0, nullptr};
      else
        j = SmallGemmJob{q1, q0, K, nullptr, nullptr, nullptr, bc.Tm[1], ldR, 0, bc.Tm[0], ldR, 1, bc.G, ldR, 1.0, 0.0, nullptr};
      gj.push_back(j);
      sj.push_back(SvdJob{bc.G, ldR, std::max(q0, q1), std::min(q0, q1), bc.V, ldR, bc.s, bc.perm,
                          s->slots[q].svd_state + 4, s->slots[q].svd_state, (double*)(s->slots[q].svd_state + 8),
                          s->cfg.svd_max_sweeps});
    }
    SmallGemmJob* gd;
    RC(stage(s, gj.data(), nb, &gd));
    KR(launch_small_gemm(gd, gj.data(), nb, s->stream));
    // block Jacobi (many workgroups per SVD) when any core is wider than 64,
    // preconditioned: QR of the core, Jacobi on R^T (a graded core needs ~3x
    // fewer sweeps there), then back to the core's singular vectors
    int nmax = 0, mmax = 0;
    for (auto& j : sj) {
      nmax = std::max(nmax, j.n);
      mmax = std::max(mmax, j.m);
    }
    if (nmax > 64) {
      std::vector<QrJob<double>> qj;
      std::vector<SmallGemmJob> back;
      for (int q = 0; q < nb; ++q) {
        const BondCore& bc = cores[q];
        const int m = sj[q].m, n = sj[q].n;
        qj.push_back(QrJob<double>{bc.G, ldR, m, n, bc.pq[0], ldR, s->slots[q].tau, 1, nullptr, 0});
        sj[q].G = bc.pq[1];
        sj[q].m = n;
        sj[q].V = bc.pq[3];
        back.push_back(SmallGemmJob{m, n, n, nullptr, nullptr, nullptr, bc.pq[2], ldR, 0, bc.pq[0], ldR, 0, bc.G, ldR,
                                    1.0, 0.0, nullptr, 0});
      }
      QrJob<double>* qd;
      RC(stage(s, qj.data(), nb, &qd));
      KR(launch_householder<double>(qd, nb, s->stream, mmax));
      KR(launch_rcore_precond_prep(cd, nb, s->stream));
      SvdJob* sd;
      RC(stage(s, sj.data(), nb, &sd));
      KR(launch_block_jacobi_svd(sd, sj.data(), nb, s->stream, (int*)(s->res + 12),
                                 (volatile int*)(s->hscratch + s->hscratch_bytes - 64), s->cfg.svd_max_sweeps));
      KR(launch_rcore_precond_finish(cd, nb, s->stream));
      RC(stage(s, back.data(), nb, &gd));
      KR(launch_small_gemm(gd, back.data(), nb, s->stream));
    } else {
      SvdJob* sd;
      RC(stage(s, sj.data(), nb, &sd));
      KR(launch_jacobi_svd(sd, nb, s->stream));
    }
  }
  KR(launch_rcore_select(cd, nb, s->stream));
  {
    // Mf_i = Q~_i (U | V): Householder blocks hold Q~_i in B_i; CholeskyQR2
    // blocks use B_i (T_i^{-1} (U | V))
    std::vector<SmallGemmJob> tu, gj;
    for (int q = 0; q < nb; ++q) {
      const BondCore& bc = cores[q];
      for (int i = 0; i < 2; ++i) {
        const double* UV = i == 0 ? bc.Uc : bc.Vc;
        const int n = 4 * bc.chi_cut, m4 = 4 * bc.k[i];
        gj.push_back(SmallGemmJob{m4, C, bc.q[i], nullptr, &cd[q].chi_new, nullptr, bc.B[i], m4, 0, UV, ldR, 0,
                                  bc.Mf[i], m4, 1.0, 0.0, &cd[q].bqr[i], 0});
        if (bc.bqr[i] != 0) continue;
        tu.push_back(SmallGemmJob{n, C, n, nullptr, &cd[q].chi_new, nullptr, bc.qs[i][2], n, 0, UV, ldR, 0,
                                  bc.qs[i][5], n, 1.0, 0.0, &cd[q].bqr[i], 1});
        gj.push_back(SmallGemmJob{m4, C, n, nullptr, &cd[q].chi_new, nullptr, bc.B[i], m4, 0, bc.qs[i][5], n, 0,
                                  bc.Mf[i], m4, 1.0, 0.0, &cd[q].bqr[i], 1});
      }
    }
    SmallGemmJob* gd;
    if (!tu.empty()) {
      RC(stage(s, tu.data(), (int)tu.size(), &gd));
      KR(launch_small_gemm(gd, tu.data(), (int)tu.size(), s->stream));
    }
    RC(stage(s, gj.data(), (int)gj.size(), &gd));
    KR(launch_small_gemm(gd, gj.data(), (int)gj.size(), s->stream));
  }
  KR(launch_rcore_rearrange(cd, nb, s->stream));
  {
    std::vector<SmallGemmJob> gj;
    for (int q = 0; q < nb; ++q) {
      const BondCore& bc = cores[q];
      for (int i = 0; i < 2; ++i) {
        if (!bc.chol[i]) continue;
        const int n = 4 * bc.chi_cut;
        SmallGemmJob j{n, 4 * C, bc.k[i], nullptr, &cd[q].n4, nullptr, bc.Rinv[i], ldR, 0, bc.Mp[i], bc.k[i], 0,
                       bc.W[i], n, 1.0, 0.0, nullptr};
        gj.push_back(j);
      }
    }
    if (!gj.empty()) {
      SmallGemmJob* gd;
      RC(stage(s, gj.data(), (int)gj.size(), &gd));
      KR(launch_small_gemm(gd, gj.data(), (int)gj.size(), s->stream));
    }
  }
  KR(launch_rcore_signs(cd, nb, s->stream));
  // bring back chi_new, status, gate_err, flags and lambda
  const uint64_t core_bytes = sizeof(BondCore) * nb;
  HPT_HIP(hipMemcpyAsync(s->hscratch, cd, core_bytes, hipMemcpyDeviceToHost, s->stream));
  const uint64_t lam_off = align_up(core_bytes);
  for (int q = 0; q < nb; ++q)
    HPT_HIP(hipMemcpyAsync(s->hscratch + lam_off + (uint64_t)q * C * 8, s->slots[q].lam, C * 8,
                           hipMemcpyDeviceToHost, s->stream));
  int ncut_off = (int)(lam_off + (uint64_t)nb * C * 8);
  for (int q = 0; q < nb; ++q)
    HPT_HIP(hipMemcpyAsync(s->hscratch + ncut_off + q * 64, s->slots[q].ncut, 6 * sizeof(int),
                           hipMemcpyDeviceToHost, s->stream));
  for (int q = 0; q < nb; ++q)
    HPT_HIP(hipMemcpyAsync(s->hscratch + ncut_off + q * 64 + 40, s->slots[q].svd_state + 3, sizeof(int),
                           hipMemcpyDeviceToHost, s->stream));
  static const bool dbg_svd = getenv("HPT_DEBUG_SVD") != nullptr;
  if (dbg_svd)
    for (int q = 0; q < nb; ++q)
      HPT_HIP(hipMemcpyAsync(s->hscratch + ncut_off + q * 64 + 32, s->slots[q].svd_state + 4, sizeof(int),
                             hipMemcpyDeviceToHost, s->stream));
  RC(sync_stream(s));
  if (dbg_svd) {
    int mx = 0, sum = 0;
    for (int q = 0; q < nb; ++q) {
      const int sw = *(const int*)(s->hscratch + ncut_off + q * 64 + 32);
      mx = std::max(mx, sw);
      sum += sw;
    }
    fprintf(stderr, "[svd] step %d colour bonds %d: Jacobi sweeps max %d mean %.1f\n", s->step, nb, mx, (double)sum / nb);
  }
  std::memcpy(cores.data(), s->hscratch, core_bytes);
  for (int q = 0; q < nb; ++q) {
    const int b = cbonds[q];
    const BondCore& bc = cores[q];
    if (bc.status != 0) return HPT_ENUMERIC;
    if (!std::isfinite(bc.gate_err)) return HPT_ENUMERIC;
    const int* nc = (const int*)(s->hscratch + ncut_off + q * 64);
    for (int i = 0; i < 2; ++i)
      for (int e = 0; e < plans[2 * q + i].nenv; ++e) {
        if (nc[3 * i + e] < 0) return HPT_ENUMERIC;
        if (nc[3 * i + e] > 0) flags |= HPT_FLAG_PINV_CUT;
      }
    if (*(const int*)(s->hscratch + ncut_off + q * 64 + 40)) flags |= HPT_FLAG_SVD_NOT_CONVERGED;
    flags |= (uint32_t)bc.flags;
    s->layer_gate_err += bc.gate_err;
    s->lam[b].assign((const double*)(s->hscratch + lam_off + (uint64_t)q * C * 8),
                     (const double*)(s->hscratch + lam_off + (uint64_t)q * C * 8) + bc.chi_new);
  }
  // phase C: reconstruct, inverse permute, deabsorb
  for (int q = 0; q < nb; ++q)
    for (int i = 0; i < 2; ++i)
      RC(phase_c_site<T>(s, cbonds[q], i, s->slots[q], plans[2 * q + i], cores[q].chi_new));
  for (int q = 0; q < nb; ++q) s->chi[cbonds[q]] = cores[q].chi_new;
  s->layer_flags |= flags;
  return 0;
}

// ---------------------------------------------------------------------------
// gauge BP on the norm network (Sec. "BP Message Update", Eq. bp)

template <typename T>
const T* gmsg_T(hpt_sim* s, int b, int dir);
template <>
const double* gmsg_T<double>(hpt_sim* s, int b, int dir) { return gmsg_slot(s, b, dir); }
template <>
const float* gmsg_T<float>(hpt_sim* s, int b, int dir) { return gmsg32_slot(s, b, dir); }

// leave-one-out products: messages applied on every leg except the output one
template <typename T>
int loo(hpt_sim* s, int v, const T* cur, const std::vector<int>& rem, const int64_t* dims, int nd,
        int busy_mask) {
  const SiteInfo& si = s->sites[v];
  const T* psi = psi_of<T>(s, v);
  if (rem.size() == 1) {
    const int l = rem[0];
    const int b = si.bond[l];
    return leg_gram<T>(s, psi, cur, dims, nd, l, gmsg_hat_slot(s, b, dir_from(s, b, v)));
  }
  const size_t h = rem.size() / 2;
  std::vector<int> H1(rem.begin(), rem.begin() + h), H2(rem.begin() + h, rem.end());
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<int>& apply = pass == 0 ? H2 : H1;
    const std::vector<int>& keep = pass == 0 ? H1 : H2;
    const T* src = cur;
    int mask = busy_mask;
    int last_t = -1;
    for (size_t a = 0; a < apply.size(); ++a) {
      int ti = -1;
      for (int k = 0; k < 3; ++k)
        if (!(mask & (1 << k))) { ti = k; break; }
      if (ti < 0) return HPT_EINVAL;
      T* dst = (T*)s->t[ti];
      const int l = apply[a];
      const int b = si.bond[l];
      RC(mode_product<T>(s, src, dst, dims, nd, l, gmsg_T<T>(s, b, dir_from(s, b, si.nbr[l]))));
      if (last_t >= 0) mask &= ~(1 << last_t);
      mask |= 1 << ti;
      last_t = ti;
      src = dst;
    }
    RC(loo<T>(s, v, src, keep, dims, nd, mask));
  }
  return 0;
}

template <typename T>
int gauge_bp_t(hpt_sim* s, int init, int* sweeps_out, double* delta_out) {
  const int nbd = 2 * s->nb;
  if (init == HPT_BP_UNIFORM) {
    for (int b = 0; b < s->nb; ++b)
      for (int d = 0; d < 2; ++d)
        KR(launch_fill_identity(gmsg_slot(s, b, d), s->chi[b], 1.0 / std::sqrt((double)s->chi[b]), s->stream));
  }
  std::vector<GaugeNormJob> nj(nbd);
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) nj[2 * b + d] = GaugeNormJob{gmsg_slot(s, b, d), gmsg_hat_slot(s, b, d), s->chi[b]};
  std::vector<DotJob> dj;
  for (int v = 0; v < s->N; ++v) {
    const int b = s->sites[v].bond[0];
    const int u = s->sites[v].nbr[0];
    const int64_t c2 = (int64_t)s->chi[b] * s->chi[b];
    dj.push_back(DotJob{gmsg_hat_slot(s, b, dir_from(s, b, v)), gmsg_slot(s, b, dir_from(s, b, u)), c2, s->bethe_x + v});
  }
  for (int b = 0; b < s->nb; ++b) {
    const int64_t c2 = (int64_t)s->chi[b] * s->chi[b];
    dj.push_back(DotJob{gmsg_slot(s, b, 0), gmsg_slot(s, b, 1), c2, s->bethe_x + s->N + b});
  }
  int sweeps = 0;
  double delta = INFINITY;
  double res[5] = {0, 1, 0, 0, 0};
  const int maxs = s->cfg.bp_max_sweeps;
  while (sweeps < maxs) {
    if (s->fp32) KR(launch_d2f(s->gmsg, s->gmsg32, (int64_t)nbd * s->chi_max * s->chi_max, s->stream));
    for (int v = 0; v < s->N; ++v) {
      int64_t dims[5];
      site_dims(s, v, dims);
      std::vector<int> rem;
      for (int l = 0; l < s->sites[v].deg; ++l) rem.push_back(l);
      RC(loo<T>(s, v, psi_of<T>(s, v), rem, dims, s->sites[v].deg + 1, 0));
    }
    DotJob* djd;
    RC(stage(s, dj.data(), (int)dj.size(), &djd));
    KR(launch_dots(djd, (int)dj.size(), s->stream));
    GaugeNormJob* njd;
    RC(stage(s, nj.data(), nbd, &njd));
    KR(launch_gauge_norm(njd, nbd, s->cfg.bp_alpha, s->delta, s->stream));
    KR(launch_log_product(s->bethe_x, s->N, s->nb, s->delta, nbd, s->res, s->stream));
    HPT_HIP(hipMemcpyAsync(s->hscratch, s->res, 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    RC(sync_stream(s));
    std::memcpy(res, s->hscratch, sizeof(res));
    delta = res[4];
    ++sweeps;
    if (!std::isfinite(delta)) return HPT_ENUMERIC;
    if (delta < s->cfg.bp_tol) break;
  }
  if (res[2] != 0.0)
    s->bethe_norm = 0.0;
  else if (res[3] != 0.0)
    s->bethe_norm = NAN;
  else
    s->bethe_norm = res[1] * std::exp(res[0]);
  s->gauge_sweeps = sweeps;
  s->gauge_delta = delta;
  if (sweeps_out) *sweeps_out = sweeps;
  if (delta_out) *delta_out = delta;
  return 0;
}

// ---------------------------------------------------------------------------
// Per-site non-identity Pauli weight n(r, t) (Sec. "Operator Spreading and
// Lightcone Saturation"): with the gauge messages of the last gauge BP on
// every virtual leg, W_v = sum psi_v (x_e M_{e->v}) psi_v over the virtual
// legs is a 4 x 4 float64 Gram on the Pauli leg (mode products, then the leg
// Gram of the Pauli axis), and n_v = 1 - W_v[I, I] / tr W_v.  The spreading
// measures of Sec. "Spatial operator spreading" follow on the host:
// p = n / sum n, R_L1 = sum p |r - r_c|_1, R_L2 = sqrt(sum p |r - r_c|_2^2),
// S_frac = -sum p ln p / ln(number of sites) (Eq. sfrac).
template <typename T>
int pauli_weights_t(hpt_sim* s, double* n_out, double* stats) {
  if (s->fp32) KR(launch_d2f(s->gmsg, s->gmsg32, 2ll * s->nb * s->chi_max * s->chi_max, s->stream));
  if (16ll * s->N > s->cv.meas_scr_cap || 16ull * s->N * sizeof(double) + 64 > s->hscratch_bytes) return HPT_ENOMEM;
  double* W = s->meas_scr;
  for (int v = 0; v < s->N; ++v) {
    const SiteInfo& si = s->sites[v];
    int64_t dims[5];
    site_dims(s, v, dims);
    const int nd = si.deg + 1;
    const T* psi = psi_of<T>(s, v);
    const T* src = psi;
    for (int l = 0; l < si.deg; ++l) {
      T* dst = (T*)s->t[l & 1];
      const int b = si.bond[l];
      RC(mode_product<T>(s, src, dst, dims, nd, l, gmsg_T<T>(s, b, dir_from(s, b, si.nbr[l]))));
      src = dst;
    }
    RC(leg_gram<T>(s, psi, src, dims, nd, si.deg, W + 16ll * v));
  }
  HPT_HIP(hipMemcpyAsync(s->hscratch, W, 16ull * s->N * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  RC(sync_stream(s));
  const double* Wh = (const double*)s->hscratch;
  double tot = 0.0;
  for (int v = 0; v < s->N; ++v) {
    const double* w = Wh + 16ll * v;
    const double tr = w[0] + w[5] + w[10] + w[15];
    if (!std::isfinite(tr) || !(tr > 0.0)) return HPT_ENUMERIC;
    n_out[v] = 1.0 - w[0] / tr;
    tot += n_out[v];
  }
  if (stats) {
    const int Lx = s->cfg.Lx;
    const int cx = s->centre % Lx, cy = s->centre / Lx;
    double r1 = 0.0, r2 = 0.0, ent = 0.0;
    for (int v = 0; v < s->N; ++v) {
      const double p = tot > 0.0 ? n_out[v] / tot : 0.0;
      const int dx = v % Lx - cx, dy = v / Lx - cy;
      r1 += p * (std::abs(dx) + std::abs(dy));
      r2 += p * (double)(dx * dx + dy * dy);
      if (p > 0.0) ent -= p * std::log(p);
    }
    stats[0] = r1;
    stats[1] = std::sqrt(r2);
    stats[2] = ent / std::log((double)s->N);
  }
  return 0;
}

// measurement BP and the log-space Bethe sum (Sec. "Correlation Function via Belief
// Propagation", Eq. bethe)

// The launches of one measurement sweep: groups of sites whose scratch fits
// the measurement scratch and partial budgets, each one last-leg launch and
// one contraction launch.  The job arrays do not change between sweeps of one
// BP, so they are planned once, staged once per batch of sweeps and launched
// again for every sweep of the batch.
struct MeasGroup {
  std::vector<LastLegJob> ll;
  int64_t ll_blocks = 0;
  int max_nl = 1;
  std::vector<MeasJob> mj;
  int64_t totals[4] = {0, 0, 0, 0};
  LastLegJob* ll_dev = nullptr;
  MeasJob* mj_dev = nullptr;
};

// Per site, one read of the pinned slice T_v gives the last leg's outgoing
// message and P = T_v contracted with the last leg's incoming message; the
// other legs' outgoing messages come from P (float64, 1/chi of the slice)
// through the generic contraction jobs.
template <typename T>
int meas_sweep_plan(hpt_sim* s, bool only_first_leg, std::vector<MeasGroup>& groups) {
  groups.clear();
  groups.emplace_back();
  int64_t used = 0, pused = 0;
  auto close = [&]() -> int {
    MeasGroup& g = groups.back();
    if (!g.ll.empty()) {
      g.ll_blocks = last_leg_plan(g.ll.data(), (int)g.ll.size(), s->fp32 ? 0 : 1, &g.max_nl);
      if (g.ll_blocks < 0) return HPT_EINVAL;
    }
    if (!g.mj.empty() && meas_plan(g.mj.data(), (int)g.mj.size(), g.totals) > s->cv.part_cap) return HPT_ENOMEM;
    return 0;
  };
  auto in_msg = [&](const SiteInfo& si, int l) { return mmsg_slot(s, si.bond[l], dir_from(s, si.bond[l], si.nbr[l])); };
  auto out_msg = [&](const SiteInfo& si, int v, int l) { return mmsg_hat_slot(s, si.bond[l], dir_from(s, si.bond[l], v)); };
  for (int v = 0; v < s->N; ++v) {
    const SiteInfo& si = s->sites[v];
    int64_t dims[5];
    site_dims(s, v, dims);
    int64_t slice = 1;
    for (int l = 0; l < si.deg; ++l) slice *= dims[l];
    const int p = v == s->centre ? s->obs_p : 0;
    const T* Tv = psi_of<T>(s, v) + (int64_t)p * slice;
    const int L = si.deg - 1;
    const int64_t rows = slice / dims[L];
    LastLegJob lj;
    std::memset(&lj, 0, sizeof(lj));
    lj.T = Tv;
    lj.rows = rows;
    lj.nL = (int)dims[L];
    lj.nx = L;
    for (int l = 0; l < L; ++l) {
      lj.xm[l] = in_msg(si, l);
      lj.xd[l] = (int)dims[l];
    }
    lj.mL = in_msg(si, L);
    lj.out = out_msg(si, v, L);
    std::vector<MeasJob> js;
    const int64_t llb = last_leg_blocks(rows, s->fp32 ? 0 : 1);
    int64_t need = rows + llb * dims[L], pjob = 0;
    for (int k = 0; k < L; ++k) {
      if (only_first_leg && k > 0) break;
      MeasJob j;
      std::memset(&j, 0, sizeof(j));
      j.I = 1;
      j.O = 1;
      for (int l = 0; l < k; ++l) {
        j.I *= dims[l];
        j.xm[j.nx] = in_msg(si, l);
        j.xd[j.nx++] = (int)dims[l];
      }
      for (int l = k + 1; l < L; ++l) {
        j.O *= dims[l];
        j.ym[j.ny] = in_msg(si, l);
        j.yd[j.ny++] = (int)dims[l];
      }
      j.nk = dims[k];
      j.out = out_msg(si, v, k);
      need += j.I + j.O + (j.O > 1 ? j.I * j.nk : 0);
      pjob += (j.O > 1 ? ceil_div(j.O, 256) * j.I * j.nk : 0) + ceil_div(j.I, 64 * 256) * j.nk;
      js.push_back(j);
    }
    if (need > s->cv.meas_scr_cap || pjob > s->cv.part_cap) return HPT_ENOMEM;
    MeasGroup* g = &groups.back();
    if (used + need > s->cv.meas_scr_cap || pused + pjob > s->cv.part_cap || g->ll.size() >= 1024 ||
        g->mj.size() + js.size() > 4096) {
      RC(close());
      groups.emplace_back();
      g = &groups.back();
      used = 0;
      pused = 0;
    }
    lj.P = s->meas_scr + used;
    lj.part = lj.P + rows;
    used += rows + llb * dims[L];
    g->ll.push_back(lj);
    for (MeasJob& j : js) {
      j.T = lj.P;
      j.x = s->meas_scr + used;
      j.y = j.x + j.I;
      j.S = j.y + j.O;
      used += j.I + j.O + (j.O > 1 ? j.I * j.nk : 0);
      g->mj.push_back(j);
    }
    pused += pjob;
  }
  return close();
}

// bytes the staged arrays of a sweep take in the job region
uint64_t meas_stage_bytes(const std::vector<MeasGroup>& groups) {
  uint64_t b = 0;
  for (const MeasGroup& g : groups)
    b += align_up(sizeof(LastLegJob) * std::max<size_t>(g.ll.size(), 1)) +
         align_up(sizeof(MeasJob) * std::max<size_t>(g.mj.size(), 1));
  return b;
}

// stage every group's arrays (extra: bytes of further arrays the caller stages
// with them; a sync first if they would not all fit, so no stage call of the
// batch recycles the region)
int meas_sweep_stage(hpt_sim* s, std::vector<MeasGroup>& groups, uint64_t extra) {
  const uint64_t need = meas_stage_bytes(groups) + extra;
  if (need > s->cv.jobs_bytes) return HPT_ENOMEM;
  if (s->jobs_used + need > s->cv.jobs_bytes) RC(sync_stream(s));
  for (MeasGroup& g : groups) {
    if (!g.ll.empty()) RC(stage(s, g.ll.data(), (int)g.ll.size(), &g.ll_dev));
    if (!g.mj.empty()) RC(stage(s, g.mj.data(), (int)g.mj.size(), &g.mj_dev));
  }
  return 0;
}

// launch one sweep's outgoing-message contractions from the staged arrays
int meas_sweep_launch(hpt_sim* s, const std::vector<MeasGroup>& groups, const double* stop) {
  for (const MeasGroup& g : groups) {
    if (!g.ll.empty())
      KR(launch_last_leg(g.ll_dev, (int)g.ll.size(), g.ll_blocks, g.max_nl, s->fp32 ? 0 : 1, s->stream, stop));
    if (!g.mj.empty()) KR(meas_launch(g.mj_dev, (int)g.mj.size(), g.totals, 1, s->part, s->stream, stop));
  }
  return 0;
}

// One sweep's launches captured from a stream into an executable HIP graph
// (kernels only: no memset or copy nodes), replayed on the same stream;
// destroyed with the object.
struct SweepGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  SweepGraph() = default;
  SweepGraph(const SweepGraph&) = delete;
  SweepGraph& operator=(const SweepGraph&) = delete;
  ~SweepGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
  template <typename F>
  int capture(hipStream_t st, F&& launches) {
    HPT_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    const int rc = launches();
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc) return rc;
    HPT_HIP(e);
    HPT_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    return 0;
  }
  int launch(hipStream_t st) {
    HPT_HIP(hipGraphLaunch(exec, st));
    return 0;
  }
};

// Capture on the handle's own side stream (default priority; the handle's
// stream may be the null stream, which cannot be captured): the launch
// helpers target s->stream, so it points at the side stream meanwhile.  The
// graph is then launched on s->stream.
template <typename F>
int capture_sweep(hpt_sim* s, SweepGraph& g, F&& launches) {
  if (!s->cap_stream) HPT_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  hipStream_t keep = s->stream;
  s->stream = s->cap_stream;
  const int rc = g.capture(s->cap_stream, launches);
  s->stream = keep;
  return rc;
}

template <typename T>
int meas_outgoing(hpt_sim* s, bool only_first_leg) {
  std::vector<MeasGroup> groups;
  RC(meas_sweep_plan<T>(s, only_first_leg, groups));
  RC(meas_sweep_stage(s, groups, 0));
  return meas_sweep_launch(s, groups, nullptr);
}

// One measurement BP (fresh uniform start, damping alpha) and the Bethe sum.
struct MeasResult {
  double C, logC;
  int sign;
  int sweeps;
  double delta;
  uint32_t flags;   // BETHE_ZERO only
};

int dist_to(hpt_sim* s, int v) {
  const int Lx = s->cfg.Lx;
  return std::abs(v % Lx - s->centre % Lx) + std::abs(v / Lx - s->centre / Lx);
}

// Features of the learned warm start (rows: directed bond (b, d), then
// component k < chi_b): the previous measurement's messages are copied out,
// one sweep runs from the uniform start, and the feature kernel reads the
// copy, that sweep's outgoing messages and the Vidal values.  The messages
// of the previous measurement are put back afterwards.  Returns the edges
// through *edges_dev (staged) and the row count.
template <typename T>
int learn_features(hpt_sim* s, LearnEdge** edges_dev, int64_t* rows_out) {
  const int C = s->chi_max;
  HPT_HIP(hipMemcpyAsync(s->lprev, s->mmsg, 2ull * s->nb * C * 8, hipMemcpyDeviceToDevice, s->stream));
  // Vidal values through the pinned scratch (stream-ordered before any later
  // device-to-host copy into it)
  double* hl = (double*)s->hscratch;
  for (int b = 0; b < s->nb; ++b)
    for (int k = 0; k < C; ++k) hl[(int64_t)b * C + k] = k < (int)s->lam[b].size() ? s->lam[b][k] : 0.0;
  HPT_HIP(hipMemcpyAsync(s->llam, hl, (uint64_t)s->nb * C * 8, hipMemcpyHostToDevice, s->stream));
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d)
      KR(launch_fill_value(mmsg_slot(s, b, d), s->chi[b], 1.0 / std::sqrt((double)s->chi[b]), s->stream));
  RC(meas_outgoing<T>(s, false));
  std::vector<LearnEdge> ed;
  int64_t row = 0;
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) {
      const int u = d == 0 ? s->bonds[b].v1 : s->bonds[b].v2, v = d == 0 ? s->bonds[b].v2 : s->bonds[b].v1;
      LearnEdge e;
      e.prev = s->meas_chi[b] > 0 ? s->lprev + (uint64_t)(2 * b + d) * C : nullptr;
      e.one = mmsg_hat_slot(s, b, d);
      e.lam = s->llam + (uint64_t)b * C;
      e.out = mmsg_slot(s, b, d);
      e.chi = s->chi[b];
      e.chi_prev = s->meas_chi[b];
      e.row0 = row;
      e.deg = (float)s->sites[u].deg;
      e.obs = u == s->centre ? 1.0f : 0.0f;
      e.dist = (float)dist_to(s, u) / (float)(s->cfg.Lx + s->cfg.Ly);
      e.dir = (float)(dist_to(s, v) - dist_to(s, u));
      ed.push_back(e);
      row += s->chi[b];
    }
  if (row > s->cv.learn_rows) return HPT_ENOMEM;
  LearnGlobals g;
  g.h_dt = (float)(s->cfg.h * s->cfg.dt);
  g.J_dt = (float)(s->cfg.J * s->cfg.dt);
  g.t = (float)(s->step * s->cfg.dt);
  g.inv_log_chimax = s->chi_max > 1 ? (float)(1.0 / std::log((double)s->chi_max)) : 0.0f;
  RC(stage(s, ed.data(), (int)ed.size(), edges_dev));
  KR(launch_learn_features(*edges_dev, (int)ed.size(), g, s->lX, s->lbase, s->stream));
  *rows_out = row;
  return 0;
}

// learned: warm start from the network; reuse: the features of the previous
// call at this layer are still in the arena (rerun of the same BP)
template <typename T>
int meas_bp_t(hpt_sim* s, double alpha, MeasResult& mr, bool learned = false, bool reuse = false) {
  const int nbd = 2 * s->nb;
  int extra = 0;
  if (learned) {
    // warm start: m = normalise(base + y) with y the network's correction
    LearnEdge* ed;
    int64_t rows = 0;
    if (reuse) {
      std::vector<LearnEdge> e(nbd);
      for (int b = 0; b < s->nb; ++b)
        for (int d = 0; d < 2; ++d) {
          std::memset(&e[2 * b + d], 0, sizeof(LearnEdge));
          e[2 * b + d].out = mmsg_slot(s, b, d);
          e[2 * b + d].chi = s->chi[b];
          e[2 * b + d].row0 = rows;
          rows += s->chi[b];
        }
      RC(stage(s, e.data(), nbd, &ed));
    } else {
      RC(learn_features<T>(s, &ed, &rows));
    }
    KR(launch_learn_forward(s->meas_model, s->lX, rows, s->ly, s->stream));
    KR(launch_learn_warm(ed, nbd, s->lbase, s->ly, s->stream));
    extra = 1;   // the sweep taken for the features is counted
  } else {
    for (int b = 0; b < s->nb; ++b)
      for (int d = 0; d < 2; ++d)
        KR(launch_fill_value(mmsg_slot(s, b, d), s->chi[b], 1.0 / std::sqrt((double)s->chi[b]), s->stream));
  }
  std::vector<MeasNormJob> nj(nbd);
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) nj[2 * b + d] = MeasNormJob{mmsg_slot(s, b, d), mmsg_hat_slot(s, b, d), s->chi[b]};
  const double tol = s->cfg.meas_tol > 0.0 ? s->cfg.meas_tol : s->cfg.bp_tol;
  const int maxs = s->cfg.meas_max_sweeps > 0 ? s->cfg.meas_max_sweeps : s->cfg.bp_max_sweeps;
  // Sweeps are queued in batches of 1, 2, 4, then 8 between host checks: the
  // residual test runs on the device (ctl: stop flag, sweeps taken), sweeps
  // queued past the converged one do nothing, so the result and the sweep
  // count are those of a host check after every sweep.
  // The job arrays are staged once for the whole BP (nothing else is staged
  // until it ends, so the syncs between batches leave them in place) and one
  // sweep's launches are captured in a HIP graph that every sweep replays.
  std::vector<MeasGroup> groups;
  RC(meas_sweep_plan<T>(s, false, groups));
  double* ctl = s->res + 8;
  KR(launch_fill_value(ctl, 2, 0.0, s->stream));
  RC(meas_sweep_stage(s, groups, align_up(sizeof(MeasNormJob) * nbd)));
  MeasNormJob* njd;
  RC(stage(s, nj.data(), nbd, &njd));
  auto one_sweep = [&]() -> int {
    RC(meas_sweep_launch(s, groups, ctl));
    KR(launch_meas_norm(njd, nbd, alpha, s->delta, s->stream, ctl));
    KR(launch_log_product(s->bethe_x, 0, 0, s->delta, nbd, s->res, s->stream, tol, ctl));
    return 0;
  };
  SweepGraph sg;
  const bool graph = s->cfg.meas_graph != 0;
  if (graph) RC(capture_sweep(s, sg, one_sweep));
  int sweeps = 0, queued = 0, batch = 1;
  double delta = INFINITY;
  double res[10];
  while (queued < maxs) {
    const int nq = std::min(batch, maxs - queued);
    for (int q = 0; q < nq; ++q) RC(graph ? sg.launch(s->stream) : one_sweep());
    queued += nq;
    HPT_HIP(hipMemcpyAsync(s->hscratch, s->res, sizeof(res), hipMemcpyDeviceToHost, s->stream));
    RC(sync_stream(s));
    std::memcpy(res, s->hscratch, sizeof(res));
    delta = res[4];
    sweeps = (int)res[9];
    if (sweeps > 0 && !std::isfinite(delta)) return HPT_ENUMERIC;
    if (res[8] != 0.0) break;
    batch = std::min(2 * batch, 8);
  }
  // Bethe: vs_v = <out_{v -> leg0}, m_{leg0 -> v}>, Z_e = <m_{b,0}, m_{b,1}>
  RC(meas_outgoing<T>(s, true));
  std::vector<DotJob> dj;
  for (int v = 0; v < s->N; ++v) {
    const int b = s->sites[v].bond[0];
    const int u = s->sites[v].nbr[0];
    dj.push_back(DotJob{mmsg_hat_slot(s, b, dir_from(s, b, v)), mmsg_slot(s, b, dir_from(s, b, u)), s->chi[b], s->bethe_x + v});
  }
  for (int b = 0; b < s->nb; ++b) dj.push_back(DotJob{mmsg_slot(s, b, 0), mmsg_slot(s, b, 1), s->chi[b], s->bethe_x + s->N + b});
  DotJob* djd;
  RC(stage(s, dj.data(), (int)dj.size(), &djd));
  KR(launch_dots(djd, (int)dj.size(), s->stream));
  KR(launch_log_product(s->bethe_x, s->N, s->nb, nullptr, 0, s->res, s->stream));
  HPT_HIP(hipMemcpyAsync(s->hscratch, s->res, 5 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  RC(sync_stream(s));
  std::memcpy(res, s->hscratch, sizeof(res));
  mr.flags = 0;
  if (res[2] != 0.0) {
    mr.C = 0.0; mr.logC = -INFINITY; mr.sign = 0; mr.flags |= HPT_FLAG_BETHE_ZERO;
  } else if (res[3] != 0.0) {
    mr.C = NAN; mr.logC = NAN; mr.sign = 0; mr.flags |= HPT_FLAG_BETHE_ZERO;
  } else {
    mr.logC = res[0]; mr.sign = res[1] < 0 ? -1 : 1; mr.C = mr.sign * std::exp(mr.logC);
  }
  mr.sweeps = sweeps + extra;
  mr.delta = delta;
  for (int b = 0; b < s->nb; ++b) s->meas_chi[b] = s->chi[b];
  return 0;
}

template <typename T>
int measure_t(hpt_sim* s, hpt_measurement* out) {
  const double alpha = s->cfg.meas_alpha > 0.0 ? s->cfg.meas_alpha : s->cfg.bp_alpha;
  const double tol = s->cfg.meas_tol > 0.0 ? s->cfg.meas_tol : s->cfg.bp_tol;
  // the previous layer's measurement (for the trap rule)
  if (s->rec_step >= 0 && s->rec_step < s->step) {
    s->prv_step = s->rec_step;
    s->prv_C = s->rec_C;
    s->prv_gate_err = s->rec_gate_err;
  }
  if (s->phase_on) HPT_HIP(hipEventRecord(s->phase_ev[3], s->stream));
  MeasResult mr;
  const bool learned = s->cfg.meas_init == HPT_BP_LEARNED;
  if (learned && !s->meas_model) return HPT_ESTATE;
  RC(meas_bp_t<T>(s, alpha, mr, learned));
  uint32_t flags = s->layer_flags | mr.flags;
  if (mr.sweeps >= s->cfg.trap_sweeps && mr.delta < tol) flags |= HPT_FLAG_TRAP_CANDIDATE;
  // trap remediation (Sec. "BP Fixed-Point Multiplicity"): a candidate whose
  // C(t) fell below half of the previous layer's while the gate error grew
  // less than twofold is retried with the other damping; the retry stands
  // when it converges and is no longer such a drop
  if (s->cfg.trap_retry && s->prv_step >= 0 && s->prv_step < s->step && (flags & HPT_FLAG_TRAP_CANDIDATE) &&
      std::fabs(mr.C) < 0.5 * std::fabs(s->prv_C) &&
      (s->layer_gate_err < 2.0 * s->prv_gate_err || s->layer_gate_err == 0.0)) {
    const double alt = s->cfg.trap_alpha > 0.0 ? s->cfg.trap_alpha : (alpha >= 1.0 ? 0.5 : 0.8);
    MeasResult r2;
    RC(meas_bp_t<T>(s, alt, r2));
    if (r2.delta < tol && std::fabs(r2.C) >= 0.5 * std::fabs(s->prv_C)) {
      mr = r2;
      flags = (flags & ~HPT_FLAG_BETHE_ZERO) | r2.flags | HPT_FLAG_TRAP_REMEDIATED;
    } else {
      // the first value stands: rerun its BP (deterministic) so that the
      // measurement messages left in the handle are the ones of the reported C
      RC(meas_bp_t<T>(s, alpha, mr, learned, true));
      flags |= HPT_FLAG_TRAP_UNRESOLVED;
    }
  }
  if (s->phase_on) {
    HPT_HIP(hipEventRecord(s->phase_ev[4], s->stream));
    double m = 0.0;
    RC(event_ms(s->phase_ev[3], s->phase_ev[4], &m));
    s->phase_ms[2] += m;
    s->phase_count[2] += 1;
    s->phase_count[3] += mr.sweeps;
  }
  const double C = mr.C, logC = mr.logC, delta = mr.delta;
  const int sign = mr.sign, sweeps = mr.sweeps;
  s->rec_step = s->step;
  s->rec_C = C;
  s->rec_gate_err = s->layer_gate_err;
  if (delta >= tol) flags |= HPT_FLAG_BP_NOT_CONVERGED_MEAS;
  if (sweeps >= s->cfg.trap_sweeps && delta < tol) flags |= HPT_FLAG_TRAP_CANDIDATE;
  if (s->bethe_norm == s->bethe_norm && s->bethe_norm >= 2.0) flags |= HPT_FLAG_NORM_EXPLODED;
  int chimax = 1;
  for (int c : s->chi) chimax = std::max(chimax, c);
  out->step = s->step;
  out->t = s->step * s->cfg.dt;
  out->C = C;
  out->log_abs_C = logC;
  out->sign = sign;
  out->gate_err = s->layer_gate_err;
  out->bethe_norm = s->bethe_norm;
  out->max_S_over_logchi = s->layer_sfrac;
  out->gauge_sweeps = s->gauge_sweeps;
  out->meas_sweeps = sweeps;
  out->gauge_delta = s->gauge_delta;
  out->meas_delta = delta;
  out->chi_live_max = chimax;
  out->flags = flags;
  return 0;
}

template <typename T>
int layer_t(hpt_sim* s) {
  s->layer_gate_err = 0.0;
  s->layer_flags = 0;
  if (s->phase_on) HPT_HIP(hipEventRecord(s->phase_ev[0], s->stream));
  RC(apply_field_t<T>(s));
  for (int c = 0; c < 4; ++c) RC(gate_colour<T>(s, s->colour_bonds[c]));
  RC(apply_field_t<T>(s));
  if (s->phase_on) HPT_HIP(hipEventRecord(s->phase_ev[1], s->stream));
  s->gauge_sweeps = 0;
  s->gauge_delta = 0.0;
  if (s->cfg.gauge_bp) {
    RC(gauge_bp_t<T>(s, s->cfg.bp_init, nullptr, nullptr));
    if (s->gauge_delta >= s->cfg.bp_tol) s->layer_flags |= HPT_FLAG_BP_NOT_CONVERGED_GAUGE;
    if (s->gauge_sweeps >= s->cfg.trap_sweeps && s->gauge_delta < s->cfg.bp_tol) s->layer_flags |= HPT_FLAG_TRAP_CANDIDATE;
  }
  if (s->phase_on) {
    HPT_HIP(hipEventRecord(s->phase_ev[2], s->stream));
    double g = 0.0, b = 0.0;
    RC(event_ms(s->phase_ev[0], s->phase_ev[1], &g));
    RC(event_ms(s->phase_ev[1], s->phase_ev[2], &b));
    s->phase_ms[0] += g;
    s->phase_ms[1] += b;
    s->phase_count[0] += 1;
    s->phase_count[1] += s->gauge_sweeps;
  }
  double sf = 0.0;
  if (s->chi_max > 1)
    for (int b = 0; b < s->nb; ++b) {
      double S = 0.0;
      for (double l : s->lam[b]) {
        const double l2 = l * l;
        if (l2 > 0) S -= l2 * std::log(l2);
      }
      sf = std::max(sf, S / std::log((double)s->chi_max));
    }
  s->layer_sfrac = sf;
  s->step++;
  return 0;
}

// gate factors of exp(-i phi XX), phi = -J dt:
// G2 = c^2 Id(x)Id + s^2 X(x)X + (cs/2) (C(x)A + A(x)C), with X(P) = XPX,
// C(P) = i[X, P], A(P) = {X, P}  (real maps in the Pauli basis)
void make_gate_tables(hpt_sim* s) {
  const double phi = -s->cfg.J * s->cfg.dt;
  const double c = std::cos(phi), sn = std::sin(phi);
  double Id[16] = {0}, Xm[16] = {0}, Cm[16] = {0}, Am[16] = {0};
  auto at = [](double* M, int e, int d) -> double& { return M[e + 4 * d]; };
  for (int a = 0; a < 4; ++a) at(Id, a, a) = 1.0;
  at(Xm, 0, 0) = 1; at(Xm, 1, 1) = 1; at(Xm, 2, 2) = -1; at(Xm, 3, 3) = -1;
  at(Cm, 3, 2) = -2.0;  // Y -> -2 Z
  at(Cm, 2, 3) = 2.0;   // Z -> 2 Y
  at(Am, 1, 0) = 2.0;   // I -> 2 X
  at(Am, 0, 1) = 2.0;   // X -> 2 I
  for (int i = 0; i < 16; ++i) {
    s->gf.F[0][i] = c * c * Id[i]; s->gf.H[0][i] = Id[i];
    s->gf.F[1][i] = sn * sn * Xm[i]; s->gf.H[1][i] = Xm[i];
    s->gf.F[2][i] = 0.5 * c * sn * Cm[i]; s->gf.H[2][i] = Am[i];
    s->gf.F[3][i] = 0.5 * c * sn * Am[i]; s->gf.H[3][i] = Cm[i];
  }
  // field half-step exp(+i h dt/2 Z): X -> cos(h dt) X + sin(h dt) Y, Y -> cos(h dt) Y - sin(h dt) X
  const double th = s->cfg.h * s->cfg.dt;
  s->g1[0] = std::cos(th);   // x' = g1[0] x + g1[1] y
  s->g1[1] = -std::sin(th);
  s->g1[2] = std::sin(th);   // y' = g1[2] x + g1[3] y
  s->g1[3] = std::cos(th);
}

template <typename T>
int reset_t(hpt_sim* s) {
  s->meas_chi.assign(s->nb, 0);
  s->rec_step = s->prv_step = -1;
  s->rec_C = s->prv_C = s->rec_gate_err = s->prv_gate_err = 0.0;
  for (int b = 0; b < s->nb; ++b) {
    s->chi[b] = 1;
    s->lam[b].assign(1, 1.0);
  }
  for (int v = 0; v < s->N; ++v) {
    T* p = psi_of<T>(s, v);
    KR(launch_fill_t<T>(p, 4, 0.0, s->stream));
    KR(launch_fill_t<T>(p + (v == s->centre ? s->obs_p : 0), 1, 1.0, s->stream));
  }
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) KR(launch_fill_value(gmsg_slot(s, b, d), 1, 1.0, s->stream));
  s->step = 0;
  s->layer_gate_err = 0.0;
  s->layer_flags = 0;
  s->layer_sfrac = 0.0;
  s->gauge_sweeps = 0;
  s->gauge_delta = 0.0;
  s->bethe_norm = 1.0;
  return sync_stream(s);
}

}  // namespace
}  // namespace hpt

using namespace hpt;

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

int hpt_config_default(hpt_config* c) {
  if (!c) return HPT_EINVAL;
  std::memset(c, 0, sizeof(*c));
  c->Lx = 3; c->Ly = 3;
  c->J = 1.0; c->h = 1.0; c->dt = 0.05;
  c->chi_max = 8;
  c->cx = -1; c->cy = -1;
  c->precision = HPT_FP64;
  c->qr_mode = HPT_QR_ADAPTIVE;
  c->chol_min_ratio = 2;
  c->chol_min_cols = 16;
  c->eps_cut = -1.0;
  c->eps_pinv = 1e-12;
  c->bp_alpha = 0.5;
  c->bp_tol = 1e-10;
  c->bp_max_sweeps = 1000;
  c->bp_init = HPT_BP_UNIFORM;
  c->meas_alpha = -1.0;
  c->meas_tol = -1.0;
  c->meas_max_sweeps = 0;
  c->gauge_bp = 1;
  c->trap_sweeps = 30;
  c->qr_rank_tol = -1.0;
  c->trap_retry = 0;
  c->trap_alpha = -1.0;
  c->meas_graph = 1;
  return HPT_OK;
}

int hpt_required_bytes(const hpt_config* cfg, uint64_t* bytes) {
  const int r = validate(cfg);
  if (r) return r;
  if (!bytes) return HPT_EINVAL;
  Carve cv;
  make_carve(*cfg, cv);
  *bytes = cv.total;
  return HPT_OK;
}

int hpt_state_bytes(const hpt_config* cfg, uint64_t* bytes) {
  const int r = validate(cfg);
  if (r) return r;
  if (!bytes) return HPT_EINVAL;
  std::vector<SiteInfo> sites;
  std::vector<BondInfo> bonds;
  build_topology(*cfg, sites, bonds);
  const uint64_t E = cfg->precision != HPT_FP64 ? 4 : 8;
  uint64_t tot = 0;
  for (auto& s : sites) tot += 4ull * (uint64_t)ipow(cfg->chi_max, s.deg) * E;
  *bytes = tot;
  return HPT_OK;
}

int hpt_create(const hpt_config* cfg, void* arena, uint64_t arena_bytes, void* hip_stream, hpt_sim** out) {
  if (!out) return HPT_EINVAL;
  *out = nullptr;
  int r = validate(cfg);
  if (r) return r;
  hpt_sim* s = new (std::nothrow) hpt_sim();
  if (!s) return HPT_ENOMEM;
  s->cfg = *cfg;
  s->fp32 = cfg->precision != HPT_FP64;
  s->bsplit = cfg->precision == HPT_FP32_BF16X6;
  s->elem = s->fp32 ? 4 : 8;
  s->chi_max = cfg->chi_max;
  build_topology(*cfg, s->sites, s->bonds);
  s->N = (int)s->sites.size();
  s->nb = (int)s->bonds.size();
  const int cx = cfg->cx < 0 ? (cfg->Lx - 1) / 2 : cfg->cx, cy = cfg->cy < 0 ? (cfg->Ly - 1) / 2 : cfg->cy;
  s->centre = cx + cfg->Lx * cy;
  // HPT_AXES_ZZX is the paper's model conjugated by a Hadamard on every site:
  // same gates, observable X_c (initial operator and pinned index at the centre)
  s->obs_p = cfg->model_axes == HPT_AXES_ZZX ? 1 : 3;
  s->colour_bonds.assign(4, {});
  for (int b = 0; b < s->nb; ++b) s->colour_bonds[s->bonds[b].colour].push_back(b);
  s->chi.assign(s->nb, 1);
  s->lam.assign(s->nb, std::vector<double>(1, 1.0));
  make_carve(*cfg, s->cv);
  s->stream = (hipStream_t)hip_stream;
  if (arena) {
    if (arena_bytes < s->cv.total) { delete s; return HPT_ENOMEM; }
    if (((uintptr_t)arena) % ALIGN) { delete s; return HPT_EINVAL; }
    s->arena = (char*)arena;
    s->arena_bytes = arena_bytes;
    s->own_arena = false;
  } else {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, s->cv.total);
    if (e != hipSuccess) { set_hip_error(e, "hipMalloc(arena)"); delete s; return e == hipErrorOutOfMemory ? HPT_ENOMEM : HPT_EHIP; }
    s->arena = (char*)p;
    s->arena_bytes = s->cv.total;
    s->own_arena = true;
  }
  char* A = s->arena;
  for (int v = 0; v < s->N; ++v) {
    s->sites[v].psi = A + s->cv.psi_off[v];
    s->sites[v].cap = 4 * ipow(s->chi_max, s->sites[v].deg);
  }
  s->gmsg = (double*)(A + s->cv.gmsg);
  s->gmsg_hat = (double*)(A + s->cv.gmsg_hat);
  s->gmsg32 = s->fp32 ? (float*)(A + s->cv.gmsg32) : nullptr;
  s->mmsg = (double*)(A + s->cv.mmsg);
  s->mmsg_hat = (double*)(A + s->cv.mmsg_hat);
  for (int i = 0; i < 3; ++i) s->t[i] = A + s->cv.t[i];
  s->part = (double*)(A + s->cv.part);
  s->meas_scr = (double*)(A + s->cv.meas_scr);
  s->slots.resize(s->cv.max_colour_bonds);
  for (int q = 0; q < s->cv.max_colour_bonds; ++q)
    slot_layout(s->chi_max, s->fp32, A + s->cv.slots + (uint64_t)q * s->cv.slot_bytes, &s->slots[q]);
  {
    const uint64_t n4 = 4ull * s->chi_max, sz = n4 * n4 * 8;
    char* c = A + s->cv.chol;
    s->G1 = (double*)c; c += sz;
    s->R1 = (double*)c; c += sz;
    s->Ri1 = (double*)c; c += sz;
    s->G2 = (double*)c; c += sz;
    s->R2 = (double*)c; c += sz;
    s->Ri2 = (double*)c; c += sz;
    s->W1 = (double*)c; c += sz;
    s->Ri32 = (float*)c; c += n4 * n4 * 4;
    c += 4 * n4 * 8;
    s->sel = (int*)c; c += n4 * 4;
    s->info = (int*)c;
  }
  {
    char* c = A + s->cv.small;
    s->bethe_x = (double*)c; c += (uint64_t)(s->N + s->nb + 64) * 8;
    s->res = (double*)c; c += 16 * 8;
    s->delta = (double*)c; c += 2ull * s->nb * 8;
    c = (char*)(((uintptr_t)c + 255) / 256 * 256);
    s->cores_dev = (BondCore*)c;
  }
  {
    char* c = A + s->cv.learn;
    const int64_t R = s->cv.learn_rows;
    s->lX = (float*)c; c += R * LEARN_F * 4;
    s->lbase = (float*)c; c += R * 4;
    s->ly = (float*)c; c += R * 4;
    c = (char*)(((uintptr_t)c + 255) / 256 * 256);
    s->lprev = (double*)c; c += R * 8;
    s->llam = (double*)c;
    s->meas_model = nullptr;
  }
  s->jobs_dev = A + s->cv.jobs;
  s->jobs_used = 0;
  s->hscratch_bytes = (uint64_t)s->cv.max_colour_bonds * (sizeof(BondCore) + s->chi_max * 8 + 64) + (1 << 20) +
                      (uint64_t)s->nb * s->chi_max * 8;
  hipError_t e1 = hipHostMalloc((void**)&s->jobs_host, s->cv.jobs_bytes, hipHostMallocDefault);
  hipError_t e2 = hipHostMalloc((void**)&s->hscratch, s->hscratch_bytes, hipHostMallocDefault);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    set_hip_error(e1 != hipSuccess ? e1 : e2, "hipHostMalloc");
    if (e1 == hipSuccess) (void)hipHostFree(s->jobs_host);
    if (e2 == hipSuccess) (void)hipHostFree(s->hscratch);
    if (s->own_arena) (void)hipFree(s->arena);
    delete s;
    return HPT_EHIP;
  }
  make_gate_tables(s);
  // qr_rank_tol < 0: float64 form keeps CholeskyQR2 exact (any dependent
  // column sends the block to Householder), float32 form deflates columns
  // whose remaining pivot is below the float32 resolution of the Gram matrix
  s->cfg_qr_tol = cfg->qr_rank_tol >= 0.0 ? cfg->qr_rank_tol : (s->fp32 ? 1e-14 : 0.0);
  // eps_cut < 0: 1e-11 (the paper's default) in the float64 form; in the
  // float32 form singular values near 1e-7 s_0 are rounding noise of the
  // float32 site tensors, so the cutoff is raised to 1e-7 s_0 there
  if (s->cfg.eps_cut < 0.0) s->cfg.eps_cut = s->fp32 ? 1e-7 : 1e-11;
  r = s->fp32 ? reset_t<float>(s) : reset_t<double>(s);
  if (r) {
    hpt_destroy(s);
    return r;
  }
  *out = s;
  return HPT_OK;
}

int hpt_reset(hpt_sim* s) {
  if (!s) return HPT_EINVAL;
  return s->fp32 ? reset_t<float>(s) : reset_t<double>(s);
}

int hpt_step(hpt_sim* s, int32_t nsteps) {
  if (!s || nsteps < 0) return HPT_EINVAL;
  for (int i = 0; i < nsteps; ++i) {
    const int r = s->fp32 ? layer_t<float>(s) : layer_t<double>(s);
    if (r) return r;
  }
  return HPT_OK;
}

int hpt_run_batch(hpt_sim* const* sims, int32_t n, const int32_t* nsteps, hpt_measurement* const* out) {
  if (!sims || !nsteps || n < 0) return HPT_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!sims[i] || nsteps[i] < 0) return HPT_EINVAL;
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return HPT_EINVAL;
  }
  if (gemm_profile_active()) return HPT_ESTATE;
  // a pool of host threads, each driving whole runs on their own streams;
  // HPT_BATCH_PROGRESS set: one stderr line as each run completes
  const bool progress = getenv("HPT_BATCH_PROGRESS") != nullptr;
  std::atomic<int> next(0), err(0), done(0);
  auto worker = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n || err.load() != 0) return;
      hpt_sim* s = sims[i];
      for (int k = 0; k < nsteps[i]; ++k) {
        if (err.load() != 0) return;   // another run failed: stop at this layer boundary
        int r = s->fp32 ? layer_t<float>(s) : layer_t<double>(s);
        if (!r && out && out[i]) r = s->fp32 ? measure_t<float>(s, out[i] + k) : measure_t<double>(s, out[i] + k);
        if (r) {
          int z = 0;
          err.compare_exchange_strong(z, r);
          return;
        }
      }
      if (hipStreamSynchronize(s->stream) != hipSuccess) {
        int z = 0;
        err.compare_exchange_strong(z, (int)HPT_EHIP);
        return;
      }
      if (progress) {
        fprintf(stderr, "[batch] run %d done (%d layers), %d of %d\n", i, nsteps[i], done.fetch_add(1) + 1, n);
        fflush(stderr);
      }
    }
  };
  const int nt = std::max(1, std::min<int>(n, 16));
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
  return err.load();
}

int hpt_apply_field(hpt_sim* s) {
  if (!s) return HPT_EINVAL;
  const int r = s->fp32 ? apply_field_t<float>(s) : apply_field_t<double>(s);
  if (r) return r;
  return sync_stream(s);
}

int hpt_apply_bond(hpt_sim* s, int32_t bond) {
  if (!s || bond < 0 || bond >= s->nb) return HPT_EINVAL;
  std::vector<int> one(1, bond);
  s->layer_gate_err = 0.0;
  return s->fp32 ? gate_colour<float>(s, one) : gate_colour<double>(s, one);
}

int hpt_gauge_bp(hpt_sim* s, int32_t init, int32_t* sweeps, double* delta) {
  if (!s || (init != HPT_BP_UNIFORM && init != HPT_BP_WARM)) return HPT_EINVAL;
  return s->fp32 ? gauge_bp_t<float>(s, init, sweeps, delta) : gauge_bp_t<double>(s, init, sweeps, delta);
}

int hpt_measure(hpt_sim* s, hpt_measurement* out) {
  if (!s || !out) return HPT_EINVAL;
  return s->fp32 ? measure_t<float>(s, out) : measure_t<double>(s, out);
}

int hpt_pauli_weights(hpt_sim* s, double* n, int32_t cap, double* stats) {
  if (!s || !n || cap < s->N) return HPT_EINVAL;
  return s->fp32 ? pauli_weights_t<float>(s, n, stats) : pauli_weights_t<double>(s, n, stats);
}

int hpt_get_chi(hpt_sim* s, int32_t bond, int32_t* chi) {
  if (!s || !chi || bond < 0 || bond >= s->nb) return HPT_EINVAL;
  *chi = s->chi[bond];
  return HPT_OK;
}

int hpt_get_bond_spectrum(hpt_sim* s, int32_t bond, double* lam, int32_t cap, int32_t* chi) {
  if (!s || bond < 0 || bond >= s->nb) return HPT_EINVAL;
  const int n = (int)s->lam[bond].size();
  if (chi) *chi = n;
  if (lam) {
    if (cap < n) return HPT_EINVAL;
    for (int i = 0; i < n; ++i) lam[i] = s->lam[bond][i];
  }
  return HPT_OK;
}

int hpt_get_site_tensor(hpt_sim* s, int32_t site, double* host, uint64_t n, int32_t* dims) {
  if (!s || site < 0 || site >= s->N) return HPT_EINVAL;
  int64_t d[5];
  site_dims(s, site, d);
  const int deg = s->sites[site].deg;
  uint64_t tot = 1;
  for (int l = 0; l <= deg; ++l) {
    tot *= d[l];
    if (dims) dims[l] = (int32_t)d[l];
  }
  if (!host) return HPT_OK;
  if (n < tot) return HPT_EINVAL;
  if (sync_stream(s)) return HPT_EHIP;
  if (s->fp32) {
    std::vector<float> tmp(tot);
    HPT_HIP(hipMemcpy(tmp.data(), s->sites[site].psi, tot * 4, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < tot; ++i) host[i] = tmp[i];
  } else {
    HPT_HIP(hipMemcpy(host, s->sites[site].psi, tot * 8, hipMemcpyDeviceToHost));
  }
  return HPT_OK;
}

int hpt_set_site_tensor(hpt_sim* s, int32_t site, const double* host, const int32_t* dims) {
  if (!s || !host || !dims || site < 0 || site >= s->N) return HPT_EINVAL;
  const SiteInfo& si = s->sites[site];
  uint64_t tot = 1;
  for (int l = 0; l < si.deg; ++l) {
    if (dims[l] < 1 || dims[l] > s->chi_max) return HPT_EINVAL;
    tot *= dims[l];
  }
  if (dims[si.deg] != 4) return HPT_EINVAL;
  tot *= 4;
  for (uint64_t i = 0; i < tot; ++i)
    if (!std::isfinite(host[i])) return HPT_ENUMERIC;
  if (sync_stream(s)) return HPT_EHIP;
  if (s->fp32) {
    std::vector<float> tmp(tot);
    for (uint64_t i = 0; i < tot; ++i) tmp[i] = (float)host[i];
    HPT_HIP(hipMemcpy(si.psi, tmp.data(), tot * 4, hipMemcpyHostToDevice));
  } else {
    HPT_HIP(hipMemcpy(si.psi, host, tot * 8, hipMemcpyHostToDevice));
  }
  for (int l = 0; l < si.deg; ++l) {
    const int b = si.bond[l];
    if (s->chi[b] != dims[l]) {
      s->chi[b] = dims[l];
      s->lam[b].assign(dims[l], 1.0 / std::sqrt((double)dims[l]));
    }
  }
  return HPT_OK;
}

int hpt_get_messages(hpt_sim* s, int32_t bond, int32_t dir, double* host, int32_t cap) {
  if (!s || !host || bond < 0 || bond >= s->nb || dir < 0 || dir > 1) return HPT_EINVAL;
  const int c = s->chi[bond];
  if (cap < c * c) return HPT_EINVAL;
  if (sync_stream(s)) return HPT_EHIP;
  HPT_HIP(hipMemcpy(host, gmsg_slot(s, bond, dir), (uint64_t)c * c * 8, hipMemcpyDeviceToHost));
  return HPT_OK;
}

int hpt_set_messages(hpt_sim* s, int32_t bond, int32_t dir, const double* host, int32_t chi) {
  if (!s || !host || bond < 0 || bond >= s->nb || dir < 0 || dir > 1) return HPT_EINVAL;
  if (chi != s->chi[bond]) return HPT_EINVAL;
  for (int64_t i = 0; i < (int64_t)chi * chi; ++i)
    if (!std::isfinite(host[i])) return HPT_ENUMERIC;
  if (sync_stream(s)) return HPT_EHIP;
  HPT_HIP(hipMemcpy(gmsg_slot(s, bond, dir), host, (uint64_t)chi * chi * 8, hipMemcpyHostToDevice));
  return HPT_OK;
}

int hpt_get_meas_messages(hpt_sim* s, int32_t bond, int32_t dir, double* host, int32_t cap) {
  if (!s || !host || bond < 0 || bond >= s->nb || dir < 0 || dir > 1) return HPT_EINVAL;
  const int c = s->chi[bond];
  if (cap < c) return HPT_EINVAL;
  if (sync_stream(s)) return HPT_EHIP;
  HPT_HIP(hipMemcpy(host, mmsg_slot(s, bond, dir), (uint64_t)c * 8, hipMemcpyDeviceToHost));
  return HPT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// checkpoint image: header, bond dimensions, Vidal values, gauge messages,
// measurement messages, live site tensors; every section 256-byte aligned

namespace {

struct CkptHeader {
  char magic[8];
  int32_t version, Lx, Ly, chi_max, precision, N, nb, step;
  int32_t gauge_sweeps, rec_step, prv_step;
  uint32_t layer_flags;
  double J, h, dt;
  double layer_gate_err, layer_sfrac, gauge_delta, bethe_norm, rec_C, rec_gate_err, prv_C, prv_gate_err;
  uint64_t off_chi, off_lam, off_gmsg, off_mmsg, off_psi, total;
};
const char CKPT_MAGIC[8] = {'H', 'P', 'T', 'C', 'K', 'P', 'T', '1'};

// section offsets of an image for the bond dimensions chi
void ckpt_layout(const hpt_sim* s, const std::vector<int>& chi, CkptHeader& h) {
  uint64_t o = align_up(sizeof(CkptHeader));
  h.off_chi = o;
  o = align_up(o + 4ull * s->nb);
  h.off_lam = o;
  for (int c : chi) o += 8ull * c;
  o = align_up(o);
  h.off_gmsg = o;
  for (int c : chi) o += 2ull * 8 * c * c;
  o = align_up(o);
  h.off_mmsg = o;
  for (int c : chi) o += 2ull * 8 * c;
  o = align_up(o);
  h.off_psi = o;
  for (int v = 0; v < s->N; ++v) {
    uint64_t n = 4;
    for (int l = 0; l < s->sites[v].deg; ++l) n *= chi[s->sites[v].bond[l]];
    o = align_up(o + n * s->elem);
  }
  h.total = o;
}

// one copy between the image and the handle's device memory
int ckpt_copy(hpt_sim* s, char* img, uint64_t off, void* dev, uint64_t bytes, int where, bool save) {
  if (bytes == 0) return 0;
  if (where == HPT_MEM_DEVICE) {
    if (save)
      HPT_HIP(hipMemcpyAsync(img + off, dev, bytes, hipMemcpyDeviceToDevice, s->stream));
    else
      HPT_HIP(hipMemcpyAsync(dev, img + off, bytes, hipMemcpyDeviceToDevice, s->stream));
  } else {
    if (save)
      HPT_HIP(hipMemcpy(img + off, dev, bytes, hipMemcpyDeviceToHost));
    else
      HPT_HIP(hipMemcpy(dev, img + off, bytes, hipMemcpyHostToDevice));
  }
  return 0;
}

// the device sections (messages and site tensors) in image order
int ckpt_device_sections(hpt_sim* s, const CkptHeader& h, char* img, int where, bool save) {
  uint64_t o = h.off_gmsg;
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) {
      const uint64_t n = 8ull * s->chi[b] * s->chi[b];
      RC(ckpt_copy(s, img, o, gmsg_slot(s, b, d), n, where, save));
      o += n;
    }
  o = h.off_mmsg;
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) {
      const uint64_t n = 8ull * s->chi[b];
      RC(ckpt_copy(s, img, o, mmsg_slot(s, b, d), n, where, save));
      o += n;
    }
  o = h.off_psi;
  for (int v = 0; v < s->N; ++v) {
    uint64_t n = 4;
    for (int l = 0; l < s->sites[v].deg; ++l) n *= s->chi[s->sites[v].bond[l]];
    RC(ckpt_copy(s, img, o, s->sites[v].psi, n * s->elem, where, save));
    o = align_up(o + n * s->elem);
  }
  return 0;
}

}  // namespace

extern "C" {

int hpt_checkpoint_bytes(hpt_sim* s, uint64_t* bytes) {
  if (!s || !bytes) return HPT_EINVAL;
  CkptHeader h;
  ckpt_layout(s, s->chi, h);
  *bytes = h.total;
  return HPT_OK;
}

int hpt_checkpoint_save(hpt_sim* s, void* buf, uint64_t cap, int32_t where) {
  if (!s || !buf || (where != HPT_MEM_HOST && where != HPT_MEM_DEVICE)) return HPT_EINVAL;
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  ckpt_layout(s, s->chi, h);
  if (cap < h.total) return HPT_ENOMEM;
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.version = 1;
  h.Lx = s->cfg.Lx; h.Ly = s->cfg.Ly; h.chi_max = s->chi_max; h.precision = s->cfg.precision;
  h.N = s->N; h.nb = s->nb; h.step = s->step;
  h.gauge_sweeps = s->gauge_sweeps; h.rec_step = s->rec_step; h.prv_step = s->prv_step;
  h.layer_flags = s->layer_flags;
  h.J = s->cfg.J; h.h = s->cfg.h; h.dt = s->cfg.dt;
  h.layer_gate_err = s->layer_gate_err; h.layer_sfrac = s->layer_sfrac; h.gauge_delta = s->gauge_delta;
  h.bethe_norm = s->bethe_norm; h.rec_C = s->rec_C; h.rec_gate_err = s->rec_gate_err;
  h.prv_C = s->prv_C; h.prv_gate_err = s->prv_gate_err;
  // host part: header, chi, lambda
  std::vector<char> blob(h.off_gmsg, 0);
  std::memcpy(blob.data(), &h, sizeof(h));
  for (int b = 0; b < s->nb; ++b) std::memcpy(blob.data() + h.off_chi + 4ull * b, &s->chi[b], 4);
  uint64_t o = h.off_lam;
  for (int b = 0; b < s->nb; ++b) {
    std::memcpy(blob.data() + o, s->lam[b].data(), 8ull * s->chi[b]);
    o += 8ull * s->chi[b];
  }
  RC(sync_stream(s));
  char* img = (char*)buf;
  if (where == HPT_MEM_DEVICE)
    HPT_HIP(hipMemcpy(img, blob.data(), blob.size(), hipMemcpyHostToDevice));
  else
    std::memcpy(img, blob.data(), blob.size());
  RC(ckpt_device_sections(s, h, img, where, true));
  return sync_stream(s);
}

int hpt_checkpoint_load(hpt_sim* s, const void* buf, uint64_t bytes, int32_t where) {
  if (!s || !buf || (where != HPT_MEM_HOST && where != HPT_MEM_DEVICE)) return HPT_EINVAL;
  if (bytes < sizeof(CkptHeader)) return HPT_EINVAL;
  char* img = (char*)buf;
  RC(sync_stream(s));
  CkptHeader h;
  if (where == HPT_MEM_DEVICE)
    HPT_HIP(hipMemcpy(&h, img, sizeof(h), hipMemcpyDeviceToHost));
  else
    std::memcpy(&h, img, sizeof(h));
  if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != 1 || h.Lx != s->cfg.Lx || h.Ly != s->cfg.Ly ||
      h.chi_max != s->chi_max || h.precision != s->cfg.precision || h.N != s->N || h.nb != s->nb ||
      h.J != s->cfg.J || h.h != s->cfg.h || h.dt != s->cfg.dt || h.total > bytes || h.off_gmsg > h.total)
    return HPT_EINVAL;
  std::vector<char> blob(h.off_gmsg);
  if (where == HPT_MEM_DEVICE)
    HPT_HIP(hipMemcpy(blob.data(), img, blob.size(), hipMemcpyDeviceToHost));
  else
    std::memcpy(blob.data(), img, blob.size());
  std::vector<int> chi(s->nb);
  for (int b = 0; b < s->nb; ++b) {
    std::memcpy(&chi[b], blob.data() + h.off_chi + 4ull * b, 4);
    if (chi[b] < 1 || chi[b] > s->chi_max) return HPT_EINVAL;
  }
  CkptHeader chk;
  ckpt_layout(s, chi, chk);
  if (chk.total != h.total || chk.off_gmsg != h.off_gmsg || chk.off_psi != h.off_psi) return HPT_EINVAL;
  s->chi = chi;
  uint64_t o = h.off_lam;
  for (int b = 0; b < s->nb; ++b) {
    s->lam[b].resize(chi[b]);
    std::memcpy(s->lam[b].data(), blob.data() + o, 8ull * chi[b]);
    o += 8ull * chi[b];
  }
  s->step = h.step;
  s->gauge_sweeps = h.gauge_sweeps; s->rec_step = h.rec_step; s->prv_step = h.prv_step;
  s->layer_flags = h.layer_flags;
  s->layer_gate_err = h.layer_gate_err; s->layer_sfrac = h.layer_sfrac; s->gauge_delta = h.gauge_delta;
  s->bethe_norm = h.bethe_norm; s->rec_C = h.rec_C; s->rec_gate_err = h.rec_gate_err;
  s->prv_C = h.prv_C; s->prv_gate_err = h.prv_gate_err;
  RC(ckpt_device_sections(s, h, img, where, false));
  return sync_stream(s);
}

int hpt_meas_learn_rows(hpt_sim* s, int64_t* rows) {
  if (!s || !rows) return HPT_EINVAL;
  int64_t r = 0;
  for (int c : s->chi) r += 2 * c;
  *rows = r;
  return HPT_OK;
}

int hpt_meas_features(hpt_sim* s, float* X, float* base, int64_t cap) {
  if (!s || !X || !base) return HPT_EINVAL;
  int64_t need = 0;
  RC(hpt_meas_learn_rows(s, &need));
  if (cap < need) return HPT_ENOMEM;
  LearnEdge* ed;
  int64_t rows = 0;
  RC(s->fp32 ? learn_features<float>(s, &ed, &rows) : learn_features<double>(s, &ed, &rows));
  // the previous measurement's messages go back (the one sweep overwrote them)
  HPT_HIP(hipMemcpyAsync(s->mmsg, s->lprev, 2ull * s->nb * s->chi_max * 8, hipMemcpyDeviceToDevice, s->stream));
  HPT_HIP(hipMemcpyAsync(X, s->lX, (uint64_t)rows * LEARN_F * 4, hipMemcpyDeviceToDevice, s->stream));
  HPT_HIP(hipMemcpyAsync(base, s->lbase, (uint64_t)rows * 4, hipMemcpyDeviceToDevice, s->stream));
  return sync_stream(s);
}

int hpt_meas_targets(hpt_sim* s, const float* base, float* T, int64_t cap) {
  if (!s || !base || !T) return HPT_EINVAL;
  int64_t need = 0;
  RC(hpt_meas_learn_rows(s, &need));
  if (cap < need) return HPT_ENOMEM;
  std::vector<LearnEdge> e(2 * s->nb);
  int64_t row = 0;
  for (int b = 0; b < s->nb; ++b)
    for (int d = 0; d < 2; ++d) {
      LearnEdge& x = e[2 * b + d];
      std::memset(&x, 0, sizeof(x));
      x.one = mmsg_slot(s, b, d);
      x.chi = s->chi[b];
      x.row0 = row;
      row += s->chi[b];
    }
  LearnEdge* ed;
  RC(stage(s, e.data(), 2 * s->nb, &ed));
  KR(launch_learn_targets(ed, 2 * s->nb, base, T, s->stream));
  return sync_stream(s);
}

int hpt_set_meas_model(hpt_sim* s, const float* params) {
  if (!s) return HPT_EINVAL;
  s->meas_model = params;
  return HPT_OK;
}

int hpt_phase_timing(hpt_sim* s, int32_t enable) {
  if (!s) return HPT_EINVAL;
  RC(sync_stream(s));
  if (enable && !s->phase_on) {
    for (hipEvent_t& e : s->phase_ev) HPT_HIP(hipEventCreate(&e));
    s->phase_on = true;
  } else if (!enable && s->phase_on) {
    for (hipEvent_t e : s->phase_ev) (void)hipEventDestroy(e);
    s->phase_on = false;
  }
  for (double& m : s->phase_ms) m = 0.0;
  for (int64_t& c : s->phase_count) c = 0;
  return HPT_OK;
}

int hpt_phase_read(hpt_sim* s, double* out7) {
  if (!s || !out7) return HPT_EINVAL;
  for (int i = 0; i < 3; ++i) out7[i] = s->phase_ms[i];
  for (int i = 0; i < 4; ++i) out7[3 + i] = (double)s->phase_count[i];
  return HPT_OK;
}

int hpt_destroy(hpt_sim* s) {
  if (!s) return HPT_EINVAL;
  (void)hipStreamSynchronize(s->stream);
  if (s->phase_on)
    for (hipEvent_t e : s->phase_ev) (void)hipEventDestroy(e);
  if (s->jobs_host) (void)hipHostFree(s->jobs_host);
  if (s->hscratch) (void)hipHostFree(s->hscratch);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->own_arena && s->arena) (void)hipFree(s->arena);
  delete s;
  return HPT_OK;
}

const char* hpt_strerror(int code) {
  switch (code) {
    case HPT_OK: return "ok";
    case HPT_EINVAL: return "invalid argument";
    case HPT_ENOMEM: return "arena too small";
    case HPT_EHIP: return "HIP runtime error";
    case HPT_ENUMERIC: return "numerical failure";
    case HPT_ESTATE: return "invalid call order";
    default: return "unknown error";
  }
}

const char* hpt_last_hip_error(void) { return g_hip_error.c_str(); }

int hpt_profile_gemm(int32_t enable) {
  const int r = gemm_profile(enable);
  return r == 0 ? HPT_OK : HPT_EHIP;
}

int hpt_profile_gemm_read(double* out4) { return hpt_profile_read(-1, out4); }

int hpt_profile_read(int32_t kind, double* out4) {
  if (!out4 || kind < -1 || kind > 4) return HPT_EINVAL;
  const int r = gemm_profile_read(kind, out4);
  return r == 0 ? HPT_OK : HPT_EHIP;
}

int hpt_permute(const void* in, void* out, int32_t ndim, const int64_t* dims, const int32_t* perm,
                int32_t elem_size, void* hip_stream) {
  if (!in || !out || !dims || !perm || ndim < 1 || ndim > 8 || (elem_size != 4 && elem_size != 8)) return HPT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  // a swap of two adjacent axis groups is served by the tiled path
  int p[8];
  for (int k = 0; k < ndim; ++k) p[k] = perm[k];
  // detect out = [0..a-1, a+g..a+g+h-1, a..a+g-1, rest] (swap of group g and group h)
  for (int a = 0; a < ndim; ++a)
    for (int g = 1; a + g < ndim; ++g)
      for (int h = 1; a + g + h <= ndim; ++h) {
        bool ok = true;
        for (int k = 0; k < a && ok; ++k) ok = p[k] == k;
        for (int k = 0; k < h && ok; ++k) ok = p[a + k] == a + g + k;
        for (int k = 0; k < g && ok; ++k) ok = p[a + h + k] == a + k;
        for (int k = a + g + h; k < ndim && ok; ++k) ok = p[k] == k;
        if (!ok) continue;
        int64_t A = 1, B = 1, Cc = 1, P = 1;
        for (int k = 0; k < a; ++k) A *= dims[k];
        for (int k = a; k < a + g; ++k) B *= dims[k];
        for (int k = a + g; k < a + g + h; ++k) Cc *= dims[k];
        for (int k = a + g + h; k < ndim; ++k) P *= dims[k];
        const int rr = permute_swap_mid(in, out, A, B, Cc, P, elem_size, st);
        return rr == 0 ? HPT_OK : (rr == -3 ? HPT_EHIP : HPT_EINVAL);
      }
  int pp[8];
  for (int k = 0; k < ndim; ++k) pp[k] = perm[k];
  const int rr = permute_generic(in, out, ndim, dims, pp, elem_size, st);
  return rr == 0 ? HPT_OK : (rr == -3 ? HPT_EHIP : HPT_EINVAL);
}

}  // extern "C"
