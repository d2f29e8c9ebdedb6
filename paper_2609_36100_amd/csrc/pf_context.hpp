// libpf context: the per-simulation state shared by the runtime translation
// units (single-grid runtime and the batched ensemble).
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <utility>
#include <vector>

#include "../../include/pf.h"
#include "pf_kernels.hpp"

namespace pf {

enum ColKind { CK_FFT = 0, CK_STAGE = 1, CK_ELASTIC = 2, CK_FWD_AC = 3, CK_COUNT = 4 };

// ---- ImEx-ARK tables ---------------------------------------------------------
struct ArkTable {
  int s;
  int order, emb_order;
  int has_emb;
  double AE[6][6], AI[6][6], bE[6], bI[6], bt[6];
};

inline ArkTable table_imex_euler() {
  ArkTable t;
  std::memset(&t, 0, sizeof(t));
  t.s = 2;
  t.order = 1;
  t.AE[1][0] = 1.0;
  t.AI[1][1] = 1.0;
  t.bE[0] = 1.0;
  t.bI[1] = 1.0;
  return t;
}

// ARK4(3)6L[2]SA (Kennedy & Carpenter 2003): published rational coefficients.
inline ArkTable table_ark436l() {
  ArkTable t;
  std::memset(&t, 0, sizeof(t));
  t.s = 6;
  t.order = 4;
  t.emb_order = 3;
  t.has_emb = 1;
  double(*E)[6] = t.AE;
  E[1][0] = 1.0 / 2.0;
  E[2][0] = 13861.0 / 62500.0;
  E[2][1] = 6889.0 / 62500.0;
  E[3][0] = -116923316275.0 / 2393684061468.0;
  E[3][1] = -2731218467317.0 / 15368042101831.0;
  E[3][2] = 9408046702089.0 / 11113171139209.0;
  E[4][0] = -451086348788.0 / 2902428689909.0;
  E[4][1] = -2682348792572.0 / 7519795681897.0;
  E[4][2] = 12662868775082.0 / 11960479115383.0;
  E[4][3] = 3355817975965.0 / 11060851509271.0;
  E[5][0] = 647845179188.0 / 3216320057751.0;
  E[5][1] = 73281519250.0 / 8382639484533.0;
  E[5][2] = 552539513391.0 / 3454668386233.0;
  E[5][3] = 3354512671639.0 / 8306763924573.0;
  E[5][4] = 4040.0 / 17871.0;
  const double b[6] = {82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0,
                       -2260.0 / 8211.0, 1.0 / 4.0};
  const double bt[6] = {4586570599.0 / 29645900160.0, 0.0, 178811875.0 / 945068544.0,
                        814220225.0 / 1159782912.0, -3700637.0 / 11593932.0, 61727.0 / 225920.0};
  double(*I)[6] = t.AI;
  const double g = 1.0 / 4.0;
  I[1][0] = g;
  I[1][1] = g;
  I[2][0] = 8611.0 / 62500.0;
  I[2][1] = -1743.0 / 31250.0;
  I[2][2] = g;
  I[3][0] = 5012029.0 / 34652500.0;
  I[3][1] = -654441.0 / 2922500.0;
  I[3][2] = 174375.0 / 388108.0;
  I[3][3] = g;
  I[4][0] = 15267082809.0 / 155376265600.0;
  I[4][1] = -71443401.0 / 120774400.0;
  I[4][2] = 730878875.0 / 902184768.0;
  I[4][3] = 2285395.0 / 8070912.0;
  I[4][4] = g;
  for (int j = 0; j < 6; ++j) {
    I[5][j] = b[j];
    t.bE[j] = b[j];
    t.bI[j] = b[j];
    t.bt[j] = bt[j];
  }
  return t;
}

// ARK2 of Giraldo, Kelly & Constantinescu (2013): three stages, second
// order, gamma = 1 - 1/sqrt 2, explicit last-row weight (3 + 2 sqrt 2)/6,
// first-order embedding.
inline ArkTable table_ark2() {
  ArkTable t;
  std::memset(&t, 0, sizeof(t));
  const double r2 = 1.41421356237309504880;
  const double g = 1.0 - 1.0 / r2, d = 1.0 / (2.0 * r2), al = (3.0 + 2.0 * r2) / 6.0;
  t.s = 3;
  t.order = 2;
  t.emb_order = 1;
  t.has_emb = 1;
  t.AE[1][0] = 2.0 * g;
  t.AE[2][0] = 1.0 - al;
  t.AE[2][1] = al;
  t.AI[1][0] = g;
  t.AI[1][1] = g;
  t.AI[2][0] = d;
  t.AI[2][1] = d;
  t.AI[2][2] = g;
  const double b[3] = {d, d, g};
  const double bt[3] = {(4.0 - r2) / 8.0, (4.0 - r2) / 8.0, d};
  for (int j = 0; j < 3; ++j) {
    t.bE[j] = b[j];
    t.bI[j] = b[j];
    t.bt[j] = bt[j];
  }
  return t;
}

// ARK3(2)4L[2]SA (Kennedy & Carpenter 2003): published rational coefficients.
inline ArkTable table_ark324l() {
  ArkTable t;
  std::memset(&t, 0, sizeof(t));
  t.s = 4;
  t.order = 3;
  t.emb_order = 2;
  t.has_emb = 1;
  const double g = 1767732205903.0 / 4055673282236.0;
  t.AE[1][0] = 1767732205903.0 / 2027836641118.0;
  t.AE[2][0] = 5535828885825.0 / 10492691773637.0;
  t.AE[2][1] = 788022342437.0 / 10882634858940.0;
  t.AE[3][0] = 6485989280629.0 / 16251701735622.0;
  t.AE[3][1] = -4246266847089.0 / 9704473918619.0;
  t.AE[3][2] = 10755448449292.0 / 10357097424841.0;
  t.AI[1][0] = 1767732205903.0 / 4055673282236.0;
  t.AI[1][1] = g;
  t.AI[2][0] = 2746238789719.0 / 10658868560708.0;
  t.AI[2][1] = -640167445237.0 / 6845629431997.0;
  t.AI[2][2] = g;
  const double b[4] = {1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0,
                       11266239266428.0 / 11593286722821.0, 1767732205903.0 / 4055673282236.0};
  const double bt[4] = {2756255671327.0 / 12835298489170.0, -10771552573575.0 / 22201958757719.0,
                        9247589265047.0 / 10645013368117.0, 2193209047091.0 / 5459859503100.0};
  for (int j = 0; j < 4; ++j) {
    t.AI[3][j] = b[j];
    t.bE[j] = b[j];
    t.bI[j] = b[j];
    t.bt[j] = bt[j];
  }
  return t;
}

// The table of a pf_method (IMEX Euler for an unknown value; callers validate).
inline ArkTable table_for(int method) {
  switch (method) {
    case PF_ARK2: return table_ark2();
    case PF_ARK324L: return table_ark324l();
    case PF_ARK436L: return table_ark436l();
    default: return table_imex_euler();
  }
}
inline bool method_ok(int method) {
  return method == PF_IMEX_EULER || method == PF_ARK2 || method == PF_ARK324L || method == PF_ARK436L;
}
inline bool method_embedded(int method) { return method == PF_ARK2 || method == PF_ARK324L || method == PF_ARK436L; }

inline bool fe_needed(const ArkTable& t, int i) {
  if (t.bE[i] != 0.0 || (t.has_emb && t.bt[i] != 0.0)) return true;
  for (int k = i + 1; k < t.s; ++k)
    if (t.AE[k][i] != 0.0) return true;
  return false;
}
inline bool fi_needed(const ArkTable& t, int i) {
  if (t.bI[i] != 0.0 || (t.has_emb && t.bI[i] - t.bt[i] != 0.0)) return true;
  for (int k = i + 1; k < t.s; ++k)
    if (t.AI[k][i] != 0.0) return true;
  return false;
}

// ---- context -----------------------------------------------------------------
}  // namespace pf

struct pf_ctx {
  pf_params p;
  hipStream_t stream = nullptr;
  int device = 0;
  pf::Geo g;
  pf::ModelK mk;
  pf::ArkTable tab;
  bool fe_need[6], fi_need[6];
  bool fi0_derived = false;  // F^I_1 = L y recomputed, never stored (explicit first stage)
  // the last stage forms the update and error sums (U into the last stage's
  // F^I buffer, E into the unused F^I_1 buffer); the update reads y, U, E, F^E_s
  bool fold_last = false;
  int mixed = 0;
  bool norm_real = false;  // WRMS of the error in real space (norm_space = 1)
  bool inhom = false;      // Reuss-averaged stiffness, Hu-Chen iteration (elastic_inhom = 1)
  pf::cx<double>* E6 = nullptr;  // inhom: six strain / polarisation spectra
  double* R6 = nullptr;          // inhom: six real strain fields
  double* LC6 = nullptr;         // inhom: the polarisation's per-point coefficients (six real fields)
  double* elmax = nullptr;       // inhom: largest strain change of the last update
  double* el_part = nullptr;     // inhom: per-block elastic energy sums

  bool owns = true;  // false for views whose buffers belong to an ensemble
  pf::cx<double>* y = nullptr;
  pf::cx<double>* ynew = nullptr;
  pf::cx<double>* ycopy = nullptr;  // norm_space = 1: the previous state, transformed back
  pf::cx<double>* FI[6] = {nullptr};
  void* FE[6] = {nullptr};  // cx<double> (FP64) or cx<float> (mixed)
  void* scratch = nullptr;  // T1 (4 fields) | T3 (3 fields) of the FFT precision
  size_t scratch_bytes = 0;
  double* partial = nullptr;
  double* red = nullptr;
  double* host_red = nullptr;  // pinned
  int nblk_red = 1024;

  // twiddle tables: 0 = z (N_z), 1 = y (N_y), 2 = x half length (M), 3 = x real length (N_x)
  pf::cx<double>* tw64[4] = {nullptr};
  pf::cx<float>* tw32[4] = {nullptr};

  // column-kernel tile variants (see col_tx) and the autotuner's timings
  int var[pf::CK_COUNT] = {1, 1, 1, 1};
  double tune_ms[pf::CK_COUNT][3] = {};
  int num_cu = 256;  // compute units of the device (persistent launches)

  // per-kernel-class HIP-event timing (off by default)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
  std::vector<std::pair<int, double>> prof_pending;  // (class, algorithmic bytes)
  double prof_ms[24] = {0}, prof_bytes[24] = {0};
  int64_t prof_n[24] = {0};

  int64_t ws_bytes = 0;
  double t = 0.0;
  double dt_next = 0.0;
  bool prev_rejected = false;  // the last attempt was rejected (caps the next proposal's growth)
  bool have_state = false;
  pf_stats st;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};


namespace pf {
// Shared by the runtime translation units (defined in pf_runtime.hip).
void ctx_setup(pf_ctx* c, const pf_params* p, hipStream_t stream);   // geometry, model, tables
void make_twiddles64(int n, cx<double>* host);
void make_twiddles32(int n, cx<float>* host);
// mass, volume fraction, threshold fraction and (want_F) total free energy of
// the context's current state; F is NaN without want_F
pf_status ctx_diagnostics(pf_ctx* c, bool want_F, double out[4]);
// ensemble member access (defined in pf_ensemble.hip)
int ens_members(const pf_ens* E);
int ens_member_n(const pf_ens* E, int m);
double ens_member_time(const pf_ens* E, int m);
hipStream_t ens_stream(const pf_ens* E);
pf_status ens_member_set(pf_ens* E, int m, const double* u, double t);
}  // namespace pf
