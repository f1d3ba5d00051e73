// Host-side state of one simulator handle: lattice topology, arena carve,
// per-colour gate workspace and the job staging area.
#pragma once
#include <vector>
#include <string>

#include "../../include/hpt.h"
#include "common.h"
#include "linalg.h"
#include "misc.h"
#include "rcore.h"
#include "learn.h"

namespace hpt {

struct SiteInfo {
  int deg;
  int bond[4];      // bond id of each leg, canonical U, D, L, R order
  int nbr[4];       // neighbour site of each leg
  int64_t cap;      // element capacity 4 * chi_max^deg
  void* psi;        // device pointer (storage type)
};

struct BondInfo {
  int v1, v2, colour;
  int pos1, pos2;   // leg axis carrying the bond at v1, v2
};

// Offsets of every device buffer inside the arena (bytes), computed by the
// memory model for a given config; `total` is hpt_required_bytes.
struct Carve {
  uint64_t psi_off[1024 + 1];
  uint64_t gmsg, gmsg_hat, gmsg32, mmsg, mmsg_hat;
  uint64_t t[3];
  int64_t tcap;     // elements per temp
  uint64_t part; int64_t part_cap;
  uint64_t meas_scr; int64_t meas_scr_cap;
  uint64_t slots; uint64_t slot_bytes; int max_colour_bonds;
  uint64_t chol;    // CholeskyQR2 scratch
  uint64_t small;   // scalars, bethe vectors, result arrays
  uint64_t jobs; uint64_t jobs_bytes;
  uint64_t learn; int64_t learn_rows;   // learned warm start: X, base, y, prev messages, Vidal values
  uint64_t total;
};

// Per-bond slot of the colour workspace (device pointers).
struct BondSlot {
  double* S[2][3];
  double* Sinv[2][3];
  float* S32[2][3];
  float* Sinv32[2][3];
  double* eigwork[2][3];
  int* ncut;        // 6 ints
  double* R[2];
  double* Rinv[2];
  double* B[2];
  double* Tm[2];
  double* tau;
  double* G;
  double* V;
  double* s;
  int* perm;
  double* Uc;
  double* Vc;
  double* Mf[2];
  double* Mp[2];
  double* W[2];
  float* W32[2];
  double* z;
  double* lam;
  int* svd_state;
  double* pq[4];    // preconditioned core SVD scratch (4 chi_max x 4 chi_max each)
  // float32 form: float64 scratch of the batched CholeskyQR2 steps, per side
  double* qa[2][8];
  int* qsel[2];
  int* qinfo[2];    // [0] Cholesky info, [1] pivoted-Cholesky rank
};

}  // namespace hpt

struct hpt_sim {
  hpt_config cfg;
  int N, nb, centre, chi_max;
  int obs_p;        // Pauli index of the observable at the centre (3 = Z; 1 = X for HPT_AXES_ZZX)
  bool fp32;
  bool bsplit;   // the split-bf16 form of the float32 GEMMs
  int elem;
  std::vector<hpt::SiteInfo> sites;
  std::vector<hpt::BondInfo> bonds;
  std::vector<std::vector<int>> colour_bonds;
  std::vector<int> chi;
  std::vector<std::vector<double>> lam;
  hipStream_t stream;
  hipStream_t cap_stream = nullptr;   // side stream for capturing the measurement sweep graph
  char* arena;
  uint64_t arena_bytes;
  bool own_arena;
  hpt::Carve cv;
  double* gmsg;
  double* gmsg_hat;
  float* gmsg32;
  double* mmsg;
  double* mmsg_hat;
  void* t[3];
  double* part;
  double* meas_scr;
  std::vector<hpt::BondSlot> slots;
  // CholeskyQR2 scratch
  double *G1, *R1, *Ri1, *G2, *R2, *Ri2, *W1;
  float* Ri32;
  int* sel;
  int* info;            // [0] Cholesky info, [1] pivoted-Cholesky rank
  double cfg_qr_tol;
  // small device arrays
  double* bethe_x;      // N + nb values
  double* res;          // 16 doubles: [0..4] log product, [8..9] measurement sweep control, [12..] Jacobi state
  double* delta;        // 2 nb
  hpt::BondCore* cores_dev;
  // job staging
  char* jobs_dev;
  char* jobs_host;      // pinned
  uint64_t jobs_used;
  // host pinned scratch for small D2H
  char* hscratch;
  uint64_t hscratch_bytes;
  hpt::GateFactors gf;
  double g1[4];
  // diagnostics of the last layer
  int step;
  double layer_gate_err;
  uint32_t layer_flags;
  double layer_sfrac;
  int gauge_sweeps;
  double gauge_delta;
  double bethe_norm;
  // last measurement (step, C, gate error) and the one of the layer before
  int rec_step, prv_step;
  double rec_C, rec_gate_err, prv_C, prv_gate_err;
  // learned warm start of the measurement BP
  float* lX;                    // learn_rows x LEARN_F features
  float* lbase;                 // learn_rows
  float* ly;                    // learn_rows
  double* lprev;                // copy of the previous measurement's messages (2 nb chi_max)
  double* llam;                 // Vidal values of every bond (nb chi_max)
  const float* meas_model;      // caller's parameters (LEARN_P floats, device) or null
  std::vector<int> meas_chi;    // chi of each bond at the last measurement (0: none)
  // per-phase timing (hpt_phase_timing): HIP events on the handle's stream
  bool phase_on;
  hipEvent_t phase_ev[5];
  double phase_ms[3];           // gate phase (field half-steps and gate updates), gauge BP, measurement
  int64_t phase_count[4];       // layers, gauge sweeps, measurements, measurement sweeps
};
