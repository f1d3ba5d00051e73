/*
 * hpt.h -- C ABI of libhpt: Heisenberg-picture tensor-network dynamics of the
 * 2D transverse-field Ising model on one AMD Instinct MI355X (gfx950).
 *
 * Method: "GPU-First Heisenberg-Picture Tensor Network Dynamics for the 2D
 * Transverse-Field Ising Model".  The operator Z_c(t) is a network of real
 * Pauli-basis site tensors on an open Lx x Ly lattice (Sec. "Pauli Basis
 * Tensor Network"); each Trotter layer applies field and coupling gates
 * (Sec. "Trotter Decomposition", Eq. trotter) through the gate update of
 * Sec. "Gate Update" / Algorithm "Gate update", then belief-propagation
 * sweeps (Eq. bp, Eq. damping); C(t) = Tr[Z_c(t) Z_c]/2^N (Eq. autocorr) is
 * read out by the log-space Bethe sum with sign tracking (Eqs. bethe_raw,
 * ze, bethe).
 *
 * Conventions shared by every entry point:
 *   - Hamiltonian H = -J sum_<ij> X_i X_j - h sum_i Z_i (Eq. hamiltonian);
 *     one step is exp(+i h dt/2 sum Z) exp(+i J dt sum XX) exp(+i h dt/2 sum Z).
 *   - Sites v = x + Lx*y.  Legs of a site in the order U (x,y-1), D (x,y+1),
 *     L (x-1,y), R (x+1,y), absent legs omitted, then the Pauli leg
 *     p = 0 I, 1 X, 2 Y, 3 Z (Sec. "GPU Tensor Permutation" leg order).
 *   - Bonds: every horizontal ((x,y),(x+1,y)) in row-major order, then every
 *     vertical ((x,y),(x,y+1)) in row-major order.  Bond b joins v1 < v2.
 *     Colour: horizontal x even 0, x odd 1; vertical y even 2, y odd 3.
 *     Directed message dir 0 travels v1 -> v2, dir 1 travels v2 -> v1.
 *   - Host tensors are float64, column-major (first listed index fastest),
 *     dims = (chi of each present leg in U,D,L,R order, 4).
 *   - Every function returns 0 on success or a negative HPT_E* code; the
 *     handle is left usable after HPT_EINVAL / HPT_ENOMEM / HPT_ESTATE.
 *   - Calls on one handle are stream-ordered on the stream given at create
 *     and are not thread-safe; separate handles are independent.
 *   - The library allocates no device buffer after hpt_create (Sec.
 *     "Zero-Malloc Simulation Loop"); the runtime objects it makes later
 *     (the side stream and graphs of the measurement sweeps, the launch
 *     autotuner's events) are not buffers of the state.
 */
#ifndef HPT_H
#define HPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define HPT_OK        0
#define HPT_EINVAL   -1   /* bad argument: dims, centre, dt == 0, chi_max < 1, bond/site index */
#define HPT_ENOMEM   -2   /* arena smaller than hpt_required_bytes, checked before any launch */
#define HPT_EHIP     -3   /* HIP runtime error; hpt_last_hip_error() has its text */
#define HPT_ENUMERIC -4   /* non-finite data (host tensors given to a set call, bond
                                 matrices, gate errors), zero bond matrix */
#define HPT_ESTATE   -5   /* call order (e.g. library not initialised) */

/* precision */
#define HPT_FP64       0  /* plain form: every step in float64 */
#define HPT_FP32_MFMA  1  /* float32 site tensors and MFMA contractions; float64
                             Cholesky, R-core SVD, eigensolver, BP normalisation, Bethe sum */
#define HPT_FP32_BF16X6 2 /* HPT_FP32_MFMA with the plain float32 products (the reconstruction
                             X (R^-1 M') of every gate) taken as six bf16 MFMA products of the
                             round-to-nearest three-way bf16 split of each operand, accumulated
                             in float32 (BF16 split precision); everything else as HPT_FP32_MFMA.
                             On 10x10 chi_max=100 its C(t) departs from the FP64 form by up to
                             1.0e-5 over 30 layers (HPT_FP32_MFMA: 6.2e-7) */

/* QR strategy (Sec. "Adaptive QR Decomposition") */
#define HPT_QR_ADAPTIVE    0  /* CholeskyQR2 for tall blocks, Householder otherwise or on failure */
#define HPT_QR_HOUSEHOLDER 1  /* Householder everywhere */

/* BP initialisation */
#define HPT_BP_UNIFORM 0      /* gauge messages I/sqrt(chi) at the start of every layer */
#define HPT_BP_WARM    1      /* continue from the messages left by the gates */
#define HPT_BP_LEARNED 2      /* meas_init only: measurement messages proposed by the
                                 warm-start network of hpt_set_meas_model */

/* measurement flags */
#define HPT_FLAG_BP_NOT_CONVERGED_GAUGE (1u << 0)
#define HPT_FLAG_BP_NOT_CONVERGED_MEAS  (1u << 1)
#define HPT_FLAG_TRAP_CANDIDATE         (1u << 2)  /* sweeps >= trap_sweeps and delta < tol */
#define HPT_FLAG_NORM_EXPLODED          (1u << 3)  /* gauge Bethe norm >= 2 */
#define HPT_FLAG_DEGENERATE_CUT         (1u << 4)  /* s[chi_max-1] - s[chi_max] <= 1e-10 s[0] */
#define HPT_FLAG_PINV_CUT               (1u << 5)  /* an environment eigenvalue was dropped */
#define HPT_FLAG_BETHE_ZERO             (1u << 6)  /* some vs_v or Z_e was exactly zero */
#define HPT_FLAG_QR_FALLBACK            (1u << 7)  /* CholeskyQR2 failed, Householder used */
#define HPT_FLAG_TRAP_REMEDIATED        (1u << 9)  /* a verified trap was retried, the retry stands */
#define HPT_FLAG_TRAP_UNRESOLVED        (1u << 10) /* a verified trap was retried without success */
#define HPT_FLAG_QR_RANK_DEFICIENT      (1u << 8)  /* a QR block had numerically dependent columns
                                                      (deflated by the pivoted Cholesky) */
#define HPT_FLAG_SVD_NOT_CONVERGED      (1u << 11) /* an R-core SVD reached svd_max_sweeps */

typedef struct {
  int32_t Lx, Ly;          /* lattice, >= 1 each, Lx*Ly >= 2 */
  double  J, h, dt;        /* coupling, field, time step (dt != 0) */
  int32_t chi_max;         /* bond-dimension cap, >= 1 */
  int32_t cx, cy;          /* observable site; -1,-1 -> ((Lx-1)/2, (Ly-1)/2) */
  int32_t precision;       /* HPT_FP64 | HPT_FP32_MFMA | HPT_FP32_BF16X6 */
  int32_t qr_mode;         /* HPT_QR_ADAPTIVE | HPT_QR_HOUSEHOLDER */
  int32_t chol_min_ratio;  /* CholeskyQR2 needs rows >= chol_min_ratio * cols (default 2) */
  int32_t chol_min_cols;   /* ... and cols >= chol_min_cols (default 16); the paper's
                              rule (Sec. "Adaptive QR Decomposition") is ratio 150, cols 150 */
  double  eps_cut;         /* truncation cutoff relative to s_0 (Eq. truncation); < 0
                              (default): 1e-11 in the FP64 form, 1e-7 in the FP32 form */
  double  eps_pinv;        /* environment eigenvalue cutoff relative to the largest, 1e-12 */
  double  bp_alpha;        /* damping (Eq. damping), 0.5 */
  double  bp_tol;          /* max |change| stopping rule (Eq. bp_tol), 1e-10 */
  int32_t bp_max_sweeps;   /* 1000 */
  int32_t bp_init;         /* HPT_BP_UNIFORM | HPT_BP_WARM */
  double  meas_alpha;      /* measurement-BP damping; < 0 -> bp_alpha */
  double  meas_tol;        /* measurement-BP tolerance; <= 0 -> bp_tol */
  int32_t meas_max_sweeps; /* <= 0 -> bp_max_sweeps */
  int32_t gauge_bp;        /* 1: run gauge BP after every layer (default); 0: skip */
  int32_t trap_sweeps;     /* trap rule threshold (Sec. "BP Fixed-Point Multiplicity"), 30 */
  double  qr_rank_tol;     /* CholeskyQR2 deflates a column when its remaining pivot is
                              <= qr_rank_tol * max diag of the Gram matrix; 0: never
                              deflate (a dependent column sends the block to Householder);
                              < 0 (default): 0 in the FP64 form, 1e-14 in the FP32 form */
  int32_t trap_retry;      /* 1: remediate verified traps (Sec. "BP Fixed-Point Multiplicity",
                              trap remediation): when a BP of the layer needed >= trap_sweeps
                              sweeps to converge and C(t) fell below half of the previous
                              layer's value while the gate error grew less than twofold, the
                              measurement BP is rerun from a uniform start with trap_alpha;
                              the retry stands when it converges and is no such drop
                              (HPT_FLAG_TRAP_REMEDIATED), else HPT_FLAG_TRAP_UNRESOLVED.
                              The previous layer is the last hpt_measure at an earlier step.
                              0 (default): off */
  int32_t reserved0;
  double  trap_alpha;      /* damping of the retry; <= 0 (default): 0.5 when the measurement
                              damping is >= 1, else 0.8 */
  int32_t model_axes;      /* HPT_AXES_PAPER (default): H = -J sum XX - h sum Z (Eq.
                              hamiltonian), observable Z_c.  HPT_AXES_ZZX: H = -J sum ZZ
                              - h sum X, observable Z_c; computed as the paper's model
                              conjugated by a Hadamard on every site (same gates and
                              splitting, observable X_c) */
  int32_t svd_max_sweeps;  /* sweep cap of the R-core Jacobi SVDs; 0 (default): 20 for the
                              block Jacobi, 60 for the one-sided Jacobi.  A core that has
                              not converged within the cap keeps its last iterate and sets
                              HPT_FLAG_SVD_NOT_CONVERGED */
  int32_t meas_init;       /* HPT_BP_UNIFORM (default): measurement messages 1/sqrt(chi);
                              HPT_BP_LEARNED: warm start proposed by the network given with
                              hpt_set_meas_model (one extra sweep, counted in meas_sweeps,
                              computes its features) */
  int32_t meas_graph;      /* 1 (default): every measurement sweep replays one HIP graph of its
                              kernels; 0: the kernels are launched one by one.  Both queue the
                              sweeps in batches with the stop test on the device and give the
                              same results bit for bit */
} hpt_config;

/* model axes */
#define HPT_AXES_PAPER 0
#define HPT_AXES_ZZX   1

typedef struct {
  int32_t  step;               /* layers applied since reset */
  double   t;                  /* step * dt */
  double   C;                  /* Bethe estimate of C(t) (Eq. bethe) */
  double   log_abs_C;          /* sum log|vs_v| - sum log|Z_e| */
  int32_t  sign;               /* product of the signs, 0 if C == 0 */
  double   gate_err;           /* sum over bonds of the discarded weight in the last layer */
  double   bethe_norm;         /* gauge-BP Bethe estimate of Tr[O^2]/2^N */
  double   max_S_over_logchi;  /* max over bonds of S_e / log(chi_max) */
  int32_t  gauge_sweeps, meas_sweeps;
  double   gauge_delta, meas_delta;
  int32_t  chi_live_max;
  uint32_t flags;              /* HPT_FLAG_* of the last layer and this measurement */
} hpt_measurement;

typedef struct hpt_sim hpt_sim;

/* Fill *cfg with the defaults listed above (3x3, J = h = 1, dt = 0.05, chi_max 8, FP64). */
int hpt_config_default(hpt_config* cfg);

/* Device bytes the handle needs for cfg (analytic memory model, Sec. "Analytic
 * Memory Model" generalised to this library's workspace).  Host only, no GPU. */
int hpt_required_bytes(const hpt_config* cfg, uint64_t* bytes);

/* Paper's state term M_psi (Eq. mem_psi) for cfg, in bytes of the storage type. */
int hpt_state_bytes(const hpt_config* cfg, uint64_t* bytes);

/* Create a simulator.  arena: caller-owned device memory of arena_bytes
 * (>= hpt_required_bytes, 256-byte aligned) that must outlive the handle, or
 * NULL to let the library make one hipMalloc that hpt_destroy frees.
 * hip_stream: a hipStream_t (NULL = the null stream).  The state is reset to t = 0. */
int hpt_create(const hpt_config* cfg, void* arena, uint64_t arena_bytes,
               void* hip_stream, hpt_sim** out);

/* t = 0 state: psi_c = e_Z, psi_v = e_I elsewhere, every bond chi = 1, messages [[1]]. */
int hpt_reset(hpt_sim* sim);

/* nsteps Trotter layers: field half-step, 4-colour gate sweep, field
 * half-step, gauge BP (pipeline figure of Sec. "Implementation").  Returns
 * after the last layer's bond dimensions are known on the host. */
int hpt_step(hpt_sim* sim, int32_t nsteps);

/* One field half-step exp(+i h dt/2 Z) on every site (Sec. "Trotter Decomposition", Eq. trotter). */
int hpt_apply_field(hpt_sim* sim);

/* The two-site gate update of Algorithm "Gate update" on one bond. */
int hpt_apply_bond(hpt_sim* sim, int32_t bond);

/* Gauge BP on the norm network until delta < bp_tol or bp_max_sweeps (Sec. "BP Message Update").
 * init: HPT_BP_UNIFORM or HPT_BP_WARM.  sweeps/delta may be NULL. */
int hpt_gauge_bp(hpt_sim* sim, int32_t init, int32_t* sweeps, double* delta);

/* Measurement BP on the pinned network and log-space Bethe sum (Sec. "Correlation Function via
 * Belief Propagation", Eq. bethe),
 * plus the diagnostics of the last layer.  Synchronises the stream.  The
 * sweeps are queued in batches (1, 2, 4, then 8 between host checks), each a
 * replay of one HIP graph holding a sweep's kernels (captured once per call
 * on a side stream the handle creates at default priority, launched on the
 * handle's stream); the residual test runs on the device and sweeps queued
 * after the converged one do nothing, so C and meas_sweeps are those of a
 * test after every sweep. */
int hpt_measure(hpt_sim* sim, hpt_measurement* out);

/* Per-site non-identity Pauli weight n(r, t) of the current state (Sec.
 * "Operator Spreading and Lightcone Saturation": the weight of the Pauli
 * strings with a non-identity letter at r, as a fraction of all), estimated
 * with the gauge messages of the last gauge BP as the environment of every
 * virtual leg (exact on a tree): W_r = sum psi_r (x_e M_{e->r}) psi_r over
 * the virtual legs (4 x 4 on the Pauli leg, float64 Gram),
 * n[r] = 1 - W_r[I, I] / tr W_r, r = x + Lx y.  stats (may be NULL) receives
 * the spreading measures of Sec. "Spatial operator spreading" with
 * p = n / sum n: the mean Manhattan radius sum p |r - r_c|_1, the RMS
 * Euclidean radius sqrt(sum p |r - r_c|_2^2) and the spatial entropy fraction
 * -sum p ln p / ln N (Eq. sfrac).  n: host, cap >= N doubles.  Costs about one
 * gauge-BP sweep; synchronises the stream.  HPT_EINVAL for a null n or
 * cap < N, HPT_ENUMERIC for a zero or non-finite weight. */
int hpt_pauli_weights(hpt_sim* sim, double* n, int32_t cap, double* stats);

/* Live bond dimension of one bond. */
int hpt_get_chi(hpt_sim* sim, int32_t bond, int32_t* chi);

/* Vidal values lambda of the bond's last gate (cap >= chi), *chi receives the count. */
int hpt_get_bond_spectrum(hpt_sim* sim, int32_t bond, double* lam, int32_t cap, int32_t* chi);

/* Copy a site tensor to host (n >= product of dims); dims[0..deg] receive its shape. */
int hpt_get_site_tensor(hpt_sim* sim, int32_t site, double* host, uint64_t n, int32_t* dims);

/* Replace a site tensor; dims gives the chi of each present leg in U,D,L,R
 * order followed by 4.  Every bond's chi must agree with both end sites
 * before the next step: setting a tensor sets the chi of its bonds.
 * HPT_ENUMERIC (nothing changed) when an entry is not finite. */
int hpt_set_site_tensor(hpt_sim* sim, int32_t site, const double* host, const int32_t* dims);

/* Gauge message on bond/dir as a chi x chi column-major float64 matrix
 * (set: HPT_ENUMERIC, nothing changed, when an entry is not finite). */
int hpt_get_messages(hpt_sim* sim, int32_t bond, int32_t dir, double* host, int32_t cap);
int hpt_set_messages(hpt_sim* sim, int32_t bond, int32_t dir, const double* host, int32_t chi);

/* Measurement message (vector of length chi) of the last hpt_measure. */
int hpt_get_meas_messages(hpt_sim* sim, int32_t bond, int32_t dir, double* host, int32_t cap);

/* Batched form (independent runs, e.g. the step sizes of a multi-product-formula
 * set): advances every handle sims[i] by nsteps[i] layers, concurrently: a pool
 * of up to 16 host threads takes the runs in order, each run on its handle's
 * own stream, so the kernels of different runs overlap on the device.  When
 * out != NULL and out[i] != NULL, out[i][k] receives hpt_measure after layer k
 * of run i (caller-owned, nsteps[i] records).  Handles must be distinct; runs
 * are independent, so each trajectory equals the one hpt_step/hpt_measure
 * give for that handle alone.  Returns HPT_EINVAL for null or repeated
 * handles or a negative count, HPT_ESTATE while the contraction profile is
 * enabled (its counters are process-wide), else the first error of any run
 * (the other runs stop at their next layer).  Blocks until all runs are done. */
int hpt_run_batch(hpt_sim* const* sims, int32_t n, const int32_t* nsteps, hpt_measurement* const* out);

/* Checkpoint and resume (long runs; the benchmark's fixed saturated state).
 * The image holds the whole simulation state: live site tensors in the storage
 * type of the handle's precision, gauge and measurement messages, bond
 * dimensions, Vidal values, the layer counter and the diagnostics that the
 * next hpt_measure reads (trap rule).  A handle resumed from an image
 * continues bit-identically to the handle that wrote it (every kernel has a
 * fixed reduction order).
 * where: HPT_MEM_HOST (buf is host memory) or HPT_MEM_DEVICE (buf is device
 * memory on the handle's GPU).  buf is caller-owned.
 * hpt_checkpoint_bytes: size of the image of the current state.
 * hpt_checkpoint_save: writes the image; HPT_ENOMEM when cap is smaller than
 *   hpt_checkpoint_bytes (nothing written).  Synchronises the stream.
 * hpt_checkpoint_load: HPT_EINVAL when the image is not one of this library or
 *   was written by a handle with another lattice, chi_max, precision, J, h or
 *   dt, or when bytes is shorter than the image; the handle is unchanged then.
 *   Synchronises the stream. */
#define HPT_MEM_HOST   0
#define HPT_MEM_DEVICE 1
int hpt_checkpoint_bytes(hpt_sim* sim, uint64_t* bytes);
int hpt_checkpoint_save(hpt_sim* sim, void* buf, uint64_t cap, int32_t where);
int hpt_checkpoint_load(hpt_sim* sim, const void* buf, uint64_t bytes, int32_t where);

/* Per-phase timing of one handle with HIP events on its stream (the benchmark's
 * split of a layer): enable = 1 creates the events and clears the totals,
 * 0 removes them.  While enabled, every layer adds the milliseconds of its
 * gate phase (both field half-steps and the four colours) and of
 * its gauge BP, and every hpt_measure those of the measurement BP
 * and Bethe sum; each phase boundary waits for its event.
 * hpt_phase_read fills out7 = {gate ms, gauge-BP ms, measurement ms, layers,
 * gauge sweeps, measurements, measurement sweeps}. */
int hpt_phase_timing(hpt_sim* sim, int32_t enable);
int hpt_phase_read(hpt_sim* sim, double* out7);

/* Learned warm start of the measurement BP (an addition to the paper's method:
 * uniform-start BP stays the default and the reference; Sec. "BP Fixed-Point
 * Multiplicity" shows that the start decides which fixed point BP reaches).
 * A two-layer perceptron applied to every component k of every directed
 * message u -> v proposes a correction y to a base message:
 *   x (HPT_LEARN_FEATURES floats) = (base_k, one_k, prev_k, [k < chi_prev],
 *     sqrt(chi) lambda_k, k / chi, 1 / sqrt(chi), deg(u) / 4, [u = observable
 *     site], dist(u, c) / (Lx + Ly), dist(v, c) - dist(u, c), h dt, J dt, t,
 *     log chi / log chi_max, 0)
 *   one = the outgoing message after one sweep from the uniform start,
 *   prev = the previous hpt_measure's converged message on the same bond (its
 *   first chi_prev entries), both L2-normalised with a non-negative sum;
 *   base = prev_k where k < chi_prev, else one_k;
 *   y = w2 . tanh(W1 x + b1) + b2 with W1, w2 and x rounded to BF16, sums in
 *   float32; the warm message is normalise(base + y).
 * Rows are ordered by bond, then direction (0: v1 -> v2), then k.
 * Parameters: HPT_LEARN_PARAMS floats, device: W1 (HPT_LEARN_HIDDEN x
 * HPT_LEARN_FEATURES, row-major), b1, w2 (HPT_LEARN_HIDDEN each), b2.
 *
 * hpt_meas_learn_rows: row count for the current bond dimensions.
 * hpt_meas_features: X (rows x HPT_LEARN_FEATURES) and base (rows) of the
 *   current state, device buffers of cap rows (HPT_ENOMEM if short); runs the
 *   one sweep, leaves the previous measurement's messages in place.  Syncs.
 * hpt_meas_targets: after hpt_measure at the same state, T = m - base for the
 *   converged messages m (normalised as above).  Syncs.
 * hpt_set_meas_model: parameters (device, caller-owned, read at every
 *   hpt_measure with meas_init = HPT_BP_LEARNED; HPT_ESTATE there when null).
 * hpt_learn_forward: y (rows) for X (rows x HPT_LEARN_FEATURES), device.
 * hpt_learn_backward: grad (HPT_LEARN_PARAMS + 1 floats, device) = gradient of
 *   L = sum_r (y_r - t_r)^2 / rows, then L; fixed summation order.
 * hpt_learn_adam: one Adam step (beta 0.9, 0.999, eps 1e-8) at step >= 1 on
 *   params with moments m, v (HPT_LEARN_PARAMS floats each, device).
 * All stream-ordered on hip_stream (the handle's stream for the hpt_meas_*). */
#define HPT_LEARN_FEATURES 16
#define HPT_LEARN_HIDDEN   128
#define HPT_LEARN_PARAMS   (HPT_LEARN_HIDDEN * HPT_LEARN_FEATURES + 2 * HPT_LEARN_HIDDEN + 1)
int hpt_meas_learn_rows(hpt_sim* sim, int64_t* rows);
int hpt_meas_features(hpt_sim* sim, float* X, float* base, int64_t cap);
int hpt_meas_targets(hpt_sim* sim, const float* base, float* T, int64_t cap);
int hpt_set_meas_model(hpt_sim* sim, const float* params);
int hpt_learn_forward(const float* params, const float* X, int64_t rows, float* y, void* hip_stream);
int hpt_learn_backward(const float* params, const float* X, const float* y, const float* t, int64_t rows,
                       float* grad, void* hip_stream);
int hpt_learn_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr,
                   void* hip_stream);

int hpt_destroy(hpt_sim* sim);

const char* hpt_strerror(int code);
const char* hpt_last_hip_error(void);

/* Process-wide timing of the MFMA contraction kernels: when enabled, every
 * launch is bracketed by HIP events on its stream.  Enabling (again) clears
 * the counters.  hpt_profile_read waits for the recorded events and fills
 * out4 = {launches, total milliseconds, algorithmic flops (2 M N K per
 * product, half for a symmetric Gram), algorithmic bytes (operands read once,
 * result written once)} for one kernel kind: HPT_PROF_GEMM (gemm_pipe_kernel:
 * general tiled GEMM, and tile_gemm_kernel<float>: the plain float32
 * products), HPT_PROF_GRAM64 (gram64_kernel: float64 products
 * and accumulation of float32 data, the CholeskyQR Grams),
 * HPT_PROF_MODE (mode_product_kernel: float32 mode products with the factor
 * resident in LDS), HPT_PROF_LEGGRAM (leg_gram_kernel: float32 leg Grams of
 * the gauge BP, with their partial-sum pass), HPT_PROF_BSPLIT
 * (tile_gemm_kernel<split>: the split-bf16 products of HPT_FP32_BF16X6), or -1
 * for all of them.  hpt_profile_gemm_read(out4) is
 * hpt_profile_read(-1, out4).  For the roofline report of the contractions.
 * Returns HPT_EINVAL for a null out4 or an unknown kind. */
#define HPT_PROF_GEMM 0
#define HPT_PROF_GRAM64 1
#define HPT_PROF_MODE 2
#define HPT_PROF_LEGGRAM 3
#define HPT_PROF_BSPLIT 4
int hpt_profile_gemm(int32_t enable);
int hpt_profile_gemm_read(double* out4);
int hpt_profile_read(int32_t kind, double* out4);

/* Float64 Gram of float32 data, the first CholeskyQR pass of the gate update
 * (Sec. "Adaptive QR Decomposition", Eq. cholqr: G = X^T X of the absorbed,
 * permuted site matrix, here with float64 products and sums as the paper
 * recommends for the Gram).
 * X: device, float32, m x n column-major with leading dimension ldx >= m.
 * G: device, float64, n x n column-major with leading dimension ldg >= n;
 *    both triangles are written.
 * workspace: device scratch of at least hpt_gram64_workspace_bytes(m, n)
 *    bytes (per-split partial tiles, at most HPT_GRAM64_PART_MAX; its contents
 *    need no clearing and are overwritten), caller-owned.
 * The rows of X are reduced in a fixed order: the same inputs give the same G
 * bit for bit.  Stream-ordered on hip_stream, asynchronous.  n == 0 does
 * nothing.  Returns HPT_EINVAL for negative sizes, m >= 2^31 - 64, ldx < m,
 * ldg < n or null pointers (X may be null when m == 0: G = 0); HPT_ENOMEM for a short workspace (before any
 * launch); HPT_EHIP when a launch fails. */
#define HPT_GRAM64_PART_MAX (64ull << 20)
int hpt_gram64_workspace_bytes(int64_t m, int32_t n, uint64_t* bytes);
int hpt_gram64(const float* X, int64_t m, int32_t n, int64_t ldx, double* G, int64_t ldg, void* workspace,
               uint64_t workspace_bytes, void* hip_stream);

/* hpt_gram64 without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as hpt_gram64, except
 * that the per-split partial tiles live in a file-scope device array of
 * HPT_GRAM64_PART_MAX bytes inside the library (one per GPU, held until the
 * process ends; its address is looked up once per device on the first call,
 * with that device current).  The call allocates nothing.  Sizes with
 * n > HPT_GRAM64_NOALLOC_MAX_N (one split of n^2 doubles would not fit) return
 * HPT_EINVAL before any launch.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and must be serialised by the caller; calls ordered on one stream are safe.
 * The array holds the last call's partials; nothing needs clearing. */
#define HPT_GRAM64_NOALLOC_MAX_N 2896
int hpt_gram64_noalloc(const float* X, int64_t m, int32_t n, int64_t ldx, double* G, int64_t ldg,
                       void* hip_stream);

/* Diagnostic of the split-bf16 products (HPT_FP32_BF16X6): one
 * v_mfma_f32_16x16x32_bf16 instruction computing, in each of its 256 outputs,
 * c + sum_{k<32} bf16(a[k]).  a: 32 floats, out: 256 floats (64 lanes x 4
 * result registers), device.  Shows how the instruction rounds the float32
 * sum of its products (tests/test_gpu_bsplit_rounding.py). */
int hpt_bf16_mfma_sum(const float* a, float c, float* out, void* hip_stream);

/* Float32 mode product of the gate update's absorb step (Sec. "Gate Update"
 * item 1: a square root of an environment message applied to one leg of a
 * site tensor) and of the gauge-BP environment products, the kernels the
 * float32 form runs:
 *   dst[a, j, b] = sum_{k < n} S[j, k] src[a, k, b],  a < inner, b < outer,
 * all column-major float32 on the device (S n x n; src, dst inner x n x outer,
 * not overlapping).  Float32 MFMA products with float32 accumulation in
 * increasing k (groups of 4), so equal inputs give equal outputs bit for bit.
 * Shapes the MFMA kernels serve: 1 <= n <= 128, and inner == 1 with
 * outer >= 16 (the leading leg) or 16 <= inner with inner n < 2^30; other
 * shapes (and null pointers) return HPT_EINVAL before any launch.
 * Stream-ordered on hip_stream, asynchronous; HPT_EHIP when a launch fails. */
int hpt_mode_product_f32(const float* src, float* dst, const float* S, int32_t n, int64_t inner, int64_t outer,
                         void* hip_stream);

/* Launch-shape autotuner.  Some launches of the layer have variants that
 * compute every output with the same operations in the same order (so the
 * choice changes the time, never a result): the mode products of the absorb
 * step and of the gauge-BP environment products (32-row strips on the
 * resident grid or on two thirds of it, or 16-row strips; the leading leg:
 * the resident grid or two thirds of it) and the cut-leg moves from or to the
 * first position (Sec. "GPU Tensor Permutation": LDS panel transposes or
 * 64 x 64 tiles).  Per shape class the first calls run the variants in turn,
 * timed by HIP events read later without blocking; once each has been timed
 * twice the fastest is kept for the rest of the process.  Process-wide (all
 * handles and threads).
 * hpt_autotune: mode 1 = on (the default), 0 = off (the default variant
 *   everywhere), 2 = forget every measurement and decision.  HPT_EINVAL for
 *   another mode.
 * hpt_autotune_report: one text line per shape class, "site k0 k1 k2: t0 t1
 *   ... -> choice" (the best milliseconds of each variant, "-" when not yet
 *   timed; choice -1 while tuning), NUL-terminated and truncated to cap
 *   bytes; *needed (may be NULL) receives the full length + 1. */
int hpt_autotune(int32_t mode);
int hpt_autotune_report(char* buf, uint64_t cap, uint64_t* needed);

/* Permute a column-major tensor on the device (Sec. "GPU Tensor Permutation").
 * in/out: device pointers, not overlapping; ndim <= 8; dims of the input;
 * perm[k] = input axis that becomes output axis k; elem_size 4 or 8.
 * Bit-exact copy.  Stream-ordered on hip_stream. */
int hpt_permute(const void* in, void* out, int32_t ndim, const int64_t* dims,
                const int32_t* perm, int32_t elem_size, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* HPT_H */
