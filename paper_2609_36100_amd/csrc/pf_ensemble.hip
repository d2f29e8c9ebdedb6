// Batched ensembles: many independent simulations of uneven cubic sizes
// advanced together.
//
// The paper points at large ensembles of simulations (uncertainty
// quantification) as a use of faster-than-real-time runs (Discussion) and at
// tuning the parallel-loop tiling per architecture (Results, single-node
// performance).  Here every pass of the ImEx-ARK stage cycle is ONE kernel
// launch for the whole ensemble: a work list gives each member a contiguous
// range of work-groups, a work-group finds its member by binary search, and
// the member's grid size selects the inlined kernel body.  Step control
// (embedded error, WRMS, accept / reject, next step size) runs on the device
// per member, so one step of every member is a fixed sequence of launches
// that is captured once in a hipGraph and replayed.  The work-group size of
// each pass kind is chosen by an autotuner (two variants, timed on the
// ensemble itself).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/pf.h"
#include "pf_context.hpp"
#include "pf_kernels.hpp"

using namespace pf;

namespace pf {

// grid lengths the batched kernels are compiled for
#define PF_ENS_SIZES(X) X(32) X(48) X(64) X(96) X(128)

static bool ens_size_ok(int n) {
  switch (n) {
#define PF_C(N) case N:
    PF_ENS_SIZES(PF_C)
#undef PF_C
    return true;
    default:
      return false;
  }
}

// per-member device descriptor
template <typename T, typename TE>
struct EMemb {
  Geo g;
  ModelK mk;
  cx<double>* ybuf[2];
  cx<double>* FI[6];
  cx<TE>* FE[6];
  cx<T>* T1;
  cx<T>* T3;
  const cx<T>* twN;  // w_N: z, y and the x real length
  const cx<T>* twM;  // w_{N/2}: the packed x transform
};

// per-member integration state (device, mirrored on the host between calls)
// dt is the next attempt (the proposal dt_next capped by dt_max and clipped to
// t_final); dt_next is the controller's proposal itself, kept so that a later
// advance to a larger t_final resumes from it.
struct EState {
  double t, dt, tf, err, dt_last, dt_next;
  double rtol, atol, dt0, dt_min, dt_max;
  long long steps, attempts, rejects, n_rhs;
  int cur, done, rejrow, adaptive, max_rejects;
  int prevrej;  // the last attempt was rejected (caps the next proposal's growth)
};

struct StageCoef {
  double aE[6], aI[6], aii;
  int fi_out, fe_need;
  int fi0_from_y;  // F^I_1 = L(k) y formed in place (explicit first stage)
  // last stage: update / error sums into FI[stage] (U) and FI[0] (E), with
  // weights b and b - b~ (times each member's dt), as in the single grid
  int fold;
  double ub[6], eb[6], ubs, ebs;
};

struct FinCoef {
  double bE[6], bI[6], dE[6], dI[6];
  int s, want_err;
  int fi0_from_y;  // as in StageCoef
  int fold;        // y_new = U + ..., error = E + ... (U in FI[s-1], E in FI[0])
};

// kernel kinds with their own work list and work-group size
enum EKind { EK_STAGE = 0, EK_YFFT4, EK_YFFT3, EK_THETA, EK_ELASTIC, EK_DRIVE, EK_FWD_AC, EK_COUNT };
static const char* const ek_names[EK_COUNT] = {"stage_invz", "ypass4", "ypass3", "xpass_theta",
                                               "zpass_elastic", "xpass_drive", "zpass_fwd_ac"};

// Columns per work-group of eb threads for lines of n points: the largest
// power of two that fits, so every row segment starts on a 128-byte boundary
// (a width like 10 or 21 columns for the 48- and 96-point lines would make
// each segment straddle cache lines); the remaining threads idle.
constexpr int ens_tx(int eb, int n, int re) {
  const int tl = line_threads(n, re);
  const int fit = eb / tl < 1 ? 1 : eb / tl;
  int tx = 1;
  while (2 * tx <= fit) tx *= 2;
  return tx;
}
constexpr int ens_rb(int eb, int m) {
  const int tl = line_threads(m);
  return eb / tl < 1 ? 1 : eb / tl;
}
// LDS elements a work-group of eb threads needs for any size in the set
constexpr int ens_lds(int eb) {
  int mx = 0;
  const int ns[5] = {32, 48, 64, 96, 128};
  for (int i = 0; i < 5; ++i) {
    const int n = ns[i];
    const int c8 = n * (ens_tx(eb, n, 8) + 1), c4 = n * (ens_tx(eb, n, 4) + 1);
    const int r = ens_rb(eb, n / 2) * (n / 2 + 2);
    mx = c8 > mx ? c8 : mx;
    mx = c4 > mx ? c4 : mx;
    mx = r > mx ? r : mx;
  }
  return mx;
}

__device__ inline int find_member(const int* start, int M, int b) {
  int lo = 0, hi = M;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// ---- batched kernels -------------------------------------------------------
template <typename T, typename TE, int EB, int NP>
__global__ void __launch_bounds__(EB) kb_stage(const EMemb<T, TE>* mem, const EState* st, const int* start, int M,
                                               StageCoef sc) {
  __shared__ cx<T> lds[ens_lds(EB)];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;
  const EMemb<T, TE>& e = mem[m];
  const int tile = blockIdx.x - start[m];
  const double dt = st[m].dt;
  StageArgs<TE> sa;
  sa.y = e.ybuf[st[m].cur];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    sa.FE[j] = j < NP ? e.FE[j] : nullptr;
    sa.FI[j] = j < NP ? e.FI[j] : nullptr;
    sa.cE[j] = j < NP ? dt * sc.aE[j] : 0.0;
    sa.cI[j] = j < NP ? dt * sc.aI[j] : 0.0;
  }
  sa.nprev = NP;
  sa.gdt = dt * sc.aii;
  sa.FI_out = sc.fi_out ? e.FI[NP] : nullptr;
  sa.fi0_from_y = sc.fi0_from_y;
  sa.U_out = sc.fold ? e.FI[NP] : nullptr;
  sa.E_out = sc.fold ? e.FI[0] : nullptr;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    sa.ub[j] = sc.ub[j];
    sa.eb[j] = sc.eb[j];
  }
  sa.ubs = sc.ubs;
  sa.ebs = sc.ebs;
  sa.fdt = dt;
  sa.FEc_out = e.mk.fEa != 0.0 ? e.FE[NP] : nullptr;
  switch (e.g.nz) {
#define PF_C(N)                                                                                       \
  case N:                                                                                             \
    body_stage_invz<T, TE, N, ens_tx(EB, N, 8), 8, NP, true>(sa, e.g, e.mk, e.twN, e.T1, tile,        \
                                                              threadIdx.x, lds);                      \
    break;
    PF_ENS_SIZES(PF_C)
#undef PF_C
  }
}

template <typename T, typename TE, int EB, int S, int NF>
__global__ void __launch_bounds__(EB) kb_ypass(const EMemb<T, TE>* mem, const EState* st, const int* start, int M) {
  __shared__ cx<T> lds[ens_lds(EB)];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;
  const EMemb<T, TE>& e = mem[m];
  const int tile = blockIdx.x - start[m];
  cx<T>* buf = NF == 4 ? e.T1 : e.T3;
  switch (e.g.nz) {
#define PF_C(N)                                                                                             \
  case N:                                                                                                   \
    body_colfft<T, N, ens_tx(EB, N, 8), 8, S, 1, true>(buf, buf, e.g, NF, e.twN, (T)1, tile, threadIdx.x, lds); \
    break;
    PF_ENS_SIZES(PF_C)
#undef PF_C
  }
}

template <typename T, typename TE, int EB>
__global__ void __launch_bounds__(EB) kb_theta(const EMemb<T, TE>* mem, const EState* st, const int* start, int M) {
  __shared__ cx<T> lds[ens_lds(EB)];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;
  const EMemb<T, TE>& e = mem[m];
  const int tile = blockIdx.x - start[m];
  switch (e.g.nz) {
#define PF_C(N)                                                                                      \
  case N:                                                                                            \
    body_xpass_theta<T, N / 2, ens_rb(EB, N / 2), true>(e.T1, e.T3, e.g, e.twN, e.twM, tile,         \
                                                         threadIdx.x, lds);                          \
    break;
    PF_ENS_SIZES(PF_C)
#undef PF_C
  }
}

template <typename T, typename TE, int EB>
__global__ void __launch_bounds__(EB) kb_drive(const EMemb<T, TE>* mem, const EState* st, const int* start, int M) {
  __shared__ cx<T> lds[ens_lds(EB)];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;
  const EMemb<T, TE>& e = mem[m];
  const int tile = blockIdx.x - start[m];
  switch (e.g.nz) {
#define PF_C(N)                                                                                        \
  case N:                                                                                              \
    body_xpass_drive<T, N / 2, ens_rb(EB, N / 2), true>(e.T1, e.T3, e.g, e.mk, e.twN, e.twM, tile,    \
                                                         threadIdx.x, lds);                            \
    break;
    PF_ENS_SIZES(PF_C)
#undef PF_C
  }
}

template <typename T, typename TE, int EB>
__global__ void __launch_bounds__(EB) kb_elastic(const EMemb<T, TE>* mem, const EState* st, const int* start, int M,
                                                 int stage) {
  __shared__ cx<T> lds[ens_lds(EB)];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;
  const EMemb<T, TE>& e = mem[m];
  const int tile = blockIdx.x - start[m];
  const int acc = e.mk.fEa != 0.0 ? 1 : 0;
  switch (e.g.nz) {
#define PF_C(N)                                                                                           \
  case N:                                                                                                 \
    body_zpass_elastic<T, TE, N, ens_tx(EB, N, 4), 4, true>(e.T3, e.g, e.mk, e.twN, e.FE[stage], acc, tile, \
                                                            threadIdx.x, lds);                            \
    break;
    PF_ENS_SIZES(PF_C)
#undef PF_C
  }
}

template <typename T, typename TE, int EB>
__global__ void __launch_bounds__(EB) kb_fwd_ac(const EMemb<T, TE>* mem, const EState* st, const int* start, int M,
                                                int stage) {
  __shared__ cx<T> lds[ens_lds(EB)];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;
  const EMemb<T, TE>& e = mem[m];
  const int tile = blockIdx.x - start[m];
  switch (e.g.nz) {
#define PF_C(N)                                                                                          \
  case N:                                                                                                \
    body_zpass_fwd_ac<T, TE, N, ens_tx(EB, N, 8), 8, true>(e.T3, e.g, e.mk, e.twN, e.FE[stage], tile,   \
                                                           threadIdx.x, lds);                            \
    break;
    PF_ENS_SIZES(PF_C)
#undef PF_C
  }
}

// update + embedded error + WRMS partial sums; fixed work-group count per member
template <typename T, typename TE>
__global__ void __launch_bounds__(256) kb_finalize(const EMemb<T, TE>* mem, const EState* st, const int* start,
                                                   int M, FinCoef fc, double* partial) {
  __shared__ double sh[16];
  const int m = find_member(start, M, blockIdx.x);
  if (st[m].done) return;  // uniform per block: the partials of done members are never read
  const EMemb<T, TE>& e = mem[m];
  const Geo& g = e.g;
  const double dt = st[m].dt;
  const cx<double>* y = e.ybuf[st[m].cur];
  cx<double>* ynew = e.ybuf[1 - st[m].cur];
  const double rtol = st[m].rtol, atol = st[m].atol;
  const double sc = 1.0 / sqrt((double)g.nx * g.ny * g.nz);
  const long long nrow = (long long)g.nz * g.ny;
  const long long total = 4 * nrow * g.nxh;
  const int nb = start[m + 1] - start[m];
  const int lb = blockIdx.x - start[m];
  double acc = 0.0, bad = 0.0;
  for (long long i = lb * 256LL + threadIdx.x; i < total; i += 256LL * nb) {
    const int x = (int)(i % g.nxh);
    const long long fr = i / g.nxh;  // f * nrow + row
    const long long idx = fr * g.P + x;
    const cx<double> y0 = y[idx];
    // all the stage loads of one element are issued before any is used
    cx<double> fi[6], fe[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const bool hasI = j < fc.s && (fc.bI[j] != 0.0 || (fc.want_err && fc.dI[j] != 0.0));
      const bool hasE = j < fc.s && (fc.bE[j] != 0.0 || (fc.want_err && fc.dE[j] != 0.0));
      fi[j] = (hasI && !(j == 0 && fc.fi0_from_y)) ? e.FI[j][idx] : mk(0.0, 0.0);
      fe[j] = hasE ? to_d(e.FE[j][idx]) : mk(0.0, 0.0);
    }
    if (fc.fi0_from_y) {
      const int f = (int)(fr / nrow);
      const int row = (int)(fr % nrow);
      const int yy = row % g.ny, z = row / g.ny;
      const double kx = x * g.kfx, ky = mode_of(yy, g.ny) * g.kfy, kz = mode_of(z, g.nz) * g.kfz;
      const double k2 = kx * kx + ky * ky + kz * kz;
      fi[0] = lsym(e.mk, f, k2) * y0;
    }
    cx<double> inc = mk(0.0, 0.0), err = fc.fold ? e.FI[0][idx] : mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j >= fc.s) break;
      inc = inc + ((dt * fc.bI[j]) * fi[j] + (dt * fc.bE[j]) * fe[j]);
      err = err + ((dt * fc.dI[j]) * fi[j] + (dt * fc.dE[j]) * fe[j]);
    }
    const cx<double> yn = (fc.fold ? e.FI[fc.s - 1][idx] : y0) + inc;
    ynew[idx] = yn;
    if (!isfinite(yn.re) || !isfinite(yn.im)) bad += 1.0;
    if (fc.want_err) {
      const double mult = (x == 0 || 2 * x == g.nx) ? 1.0 : 2.0;
      const double ay = sqrt(y0.re * y0.re + y0.im * y0.im) * sc;
      const double wgt = 1.0 / (rtol * ay + atol);
      acc += mult * (err.re * err.re + err.im * err.im) * sc * sc * wgt * wgt;
    }
  }
  const double s0 = block_sum(acc, sh);
  const double s1 = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0;
    partial[2 * blockIdx.x + 1] = s1;
  }
}

__device__ inline double ctrl_factor(double dt, double err, int q, bool after_reject) {
  if (!isfinite(err)) return 0.25 * dt;
  double fac = err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -1.0 / (q + 1))));
  if (after_reject) fac = fmin(1.0, fac);
  return dt * fac;
}

// One work-group per member: sum its partials in a fixed order, then the
// accept / reject decision and the next step size (thread 0).
template <typename T, typename TE>
__global__ void __launch_bounds__(256) kb_control(const EMemb<T, TE>* mem, EState* st, const int* fstart,
                                                  const double* partial, int q, int has_emb, int nrhs) {
  __shared__ double sh[16];
  const int m = blockIdx.x;
  if (st[m].done) return;
  double a = 0.0, b = 0.0;
  for (int i = fstart[m] + threadIdx.x; i < fstart[m + 1]; i += blockDim.x) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x != 0) return;
  EState s = st[m];
  const Geo& g = mem[m].g;
  const double n3 = (double)g.nx * g.ny * g.nz;
  double err = has_emb ? sqrt(a / (4.0 * n3)) : 0.0;
  const bool finite = b == 0.0 && isfinite(err);
  if (!finite) err = INFINITY;
  bool ok;
  double nxt;
  if (s.adaptive) {
    ok = finite && err <= 1.0;
    nxt = fmax(ctrl_factor(s.dt, err, q, ok && s.prevrej != 0), s.dt_min);
    s.prevrej = ok ? 0 : 1;
  } else {
    ok = finite;
    nxt = s.dt0;
  }
  s.attempts += 1;
  s.n_rhs += nrhs;
  s.err = err;
  if (ok) {
    s.cur = 1 - s.cur;
    s.t += s.dt;
    s.steps += 1;
    s.dt_last = s.dt;
    s.rejrow = 0;
  } else {
    s.rejects += 1;
    s.rejrow += 1;
  }
  if (!finite && !s.adaptive) {
    s.done = 3;  // non-finite fixed-step run
  } else if (s.rejrow >= s.max_rejects) {
    s.done = 2;  // failed
  } else if (s.t >= s.tf * (1.0 - 1e-15)) {
    s.done = 1;
  }
  // next attempt: the controller's proposal (or dt0), capped and clipped to
  // t_final; the proposal itself is kept for a later advance
  s.dt_next = nxt;
  s.dt = fmin(fmin(nxt, s.dt_max), s.tf - s.t);
  st[m] = s;
}

}  // namespace pf

// ---- host side -------------------------------------------------------------------
struct pf_ens {
  int M = 0;
  int mixed = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<pf_params> prm;
  std::vector<pf_ctx*> views;
  std::vector<cx<double>*> yb0, yb1;  // state buffers 0 / 1 of each member
  std::vector<void*> allocs;
  void* mem_dev = nullptr;
  EState* st_dev = nullptr;
  EState* st_host = nullptr;  // pinned
  int* start[EK_COUNT][2] = {{nullptr}};
  int ntiles[EK_COUNT][2] = {{0}};
  int* fin_start = nullptr;
  int nfin = 0;
  double* partial = nullptr;
  int var[EK_COUNT] = {1, 1, 1, 1, 1, 1, 1};
  double tune_ms[EK_COUNT][2] = {{0}};
  ArkTable tab;
  bool fe_need[6], fi_need[6];
  bool fi0_derived = false;  // explicit first stage: F^I_1 = L y, never stored
  bool fold_last = false;    // last stage forms the update and error sums
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::map<int, std::pair<cx<double>*, cx<double>*>> tw64;  // N -> (w_N, w_{N/2})
  std::map<int, std::pair<cx<float>*, cx<float>*>> tw32;
  int64_t ws_bytes = 0;
  double elapsed_ms = 0.0;
};

#define PF_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return PF_ERR_HIP;           \
  } while (0)

static pf_status ens_alloc(pf_ens* E, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return PF_ERR_OOM;
  }
  E->allocs.push_back(*p);
  E->ws_bytes += (int64_t)bytes;
  return PF_OK;
}

template <int EB>
static int col_tiles(int n, int re) {
  const int tx = ens_tx(EB, n, re);
  return ((n / 2 + 1 + tx - 1) / tx) * n;
}
template <int EB>
static int row_tiles(int n) {
  const int rb = ens_rb(EB, n / 2);
  return (n * n + rb - 1) / rb;
}

template <int EB>
static int kind_tiles(int kind, int n) {
  switch (kind) {
    case EK_ELASTIC: return col_tiles<EB>(n, 4);
    case EK_THETA:
    case EK_DRIVE: return row_tiles<EB>(n);
    default: return col_tiles<EB>(n, 8);
  }
}

static pf_status build_lists(pf_ens* E) {
  for (int k = 0; k < EK_COUNT; ++k)
    for (int v = 0; v < 2; ++v) {
      std::vector<int> st(E->M + 1, 0);
      for (int m = 0; m < E->M; ++m)
        st[m + 1] = st[m] + (v ? kind_tiles<256>(k, E->prm[m].nz) : kind_tiles<128>(k, E->prm[m].nz));
      pf_status s = ens_alloc(E, (void**)&E->start[k][v], sizeof(int) * (E->M + 1));
      if (s != PF_OK) return s;
      PF_HIP(hipMemcpy(E->start[k][v], st.data(), sizeof(int) * (E->M + 1), hipMemcpyHostToDevice));
      E->ntiles[k][v] = st[E->M];
    }
  std::vector<int> fs(E->M + 1, 0);
  for (int m = 0; m < E->M; ++m) {
    const long long n = E->prm[m].nz;
    const long long total = 4 * n * n * (n / 2 + 1);
    fs[m + 1] = fs[m] + (int)std::min<long long>(1024, (total + 2047) / 2048);
  }
  E->nfin = fs[E->M];
  pf_status s = ens_alloc(E, (void**)&E->fin_start, sizeof(int) * (E->M + 1));
  if (s != PF_OK) return s;
  PF_HIP(hipMemcpy(E->fin_start, fs.data(), sizeof(int) * (E->M + 1), hipMemcpyHostToDevice));
  return ens_alloc(E, (void**)&E->partial, sizeof(double) * 2 * E->nfin);
}

template <typename T, typename TE>
static void launch_kind(pf_ens* E, int kind, int stage) {
  const EMemb<T, TE>* mem = (const EMemb<T, TE>*)E->mem_dev;
  const int v = E->var[kind];
  const int nb = E->ntiles[kind][v];
  const int* st = E->start[kind][v];
  hipStream_t s = E->stream;
  auto go = [&](auto EBC) {
    constexpr int EB = decltype(EBC)::value;
    switch (kind) {
      case EK_STAGE: {
        StageCoef sc;
        std::memset(&sc, 0, sizeof(sc));
        for (int j = 0; j < 6; ++j) {
          sc.aE[j] = (j < stage && E->fe_need[j]) ? E->tab.AE[stage][j] : 0.0;
          sc.aI[j] = (j < stage && E->fi_need[j]) ? E->tab.AI[stage][j] : 0.0;
        }
        sc.aii = E->tab.AI[stage][stage];
        sc.fi0_from_y = E->fi0_derived ? 1 : 0;
        sc.fi_out = (E->fi_need[stage] && !(stage == 0 && E->fi0_derived)) ? 1 : 0;
        if (E->fold_last && stage == E->tab.s - 1) {
          const ArkTable& tb = E->tab;
          sc.fold = 1;
          sc.fi_out = 0;
          for (int j = 0; j < stage; ++j) {  // b^E = b^I here (fold_last)
            sc.ub[j] = tb.bI[j];
            sc.eb[j] = tb.bI[j] - tb.bt[j];
          }
          sc.ubs = tb.bI[stage];
          sc.ebs = tb.bI[stage] - tb.bt[stage];
        }
        switch (stage) {
          case 0: kb_stage<T, TE, EB, 0><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, sc); break;
          case 1: kb_stage<T, TE, EB, 1><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, sc); break;
          case 2: kb_stage<T, TE, EB, 2><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, sc); break;
          case 3: kb_stage<T, TE, EB, 3><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, sc); break;
          case 4: kb_stage<T, TE, EB, 4><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, sc); break;
          default: kb_stage<T, TE, EB, 5><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, sc); break;
        }
        break;
      }
      case EK_YFFT4:
        if (stage < 0)
          kb_ypass<T, TE, EB, -1, 4><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M);
        else
          kb_ypass<T, TE, EB, +1, 4><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M);
        break;
      case EK_YFFT3:
        if (stage < 0)
          kb_ypass<T, TE, EB, -1, 3><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M);
        else
          kb_ypass<T, TE, EB, +1, 3><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M);
        break;
      case EK_THETA: kb_theta<T, TE, EB><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M); break;
      case EK_ELASTIC: kb_elastic<T, TE, EB><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, stage); break;
      case EK_DRIVE: kb_drive<T, TE, EB><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M); break;
      default: kb_fwd_ac<T, TE, EB><<<nb, EB, 0, s>>>(mem, E->st_dev, st, E->M, stage); break;
    }
  };
  if (v)
    go(std::integral_constant<int, 256>{});
  else
    go(std::integral_constant<int, 128>{});
}

// One attempted step of every active member: 6 x 9 pass launches, finalize, control.
template <typename T, typename TE>
static void enqueue_step(pf_ens* E) {
  const ArkTable& tb = E->tab;
  int nrhs = 0;
  for (int i = 0; i < tb.s; ++i) {
    launch_kind<T, TE>(E, EK_STAGE, i);
    if (!E->fe_need[i]) continue;
    ++nrhs;
    launch_kind<T, TE>(E, EK_YFFT4, +1);  // inverse y of the state
    launch_kind<T, TE>(E, EK_THETA, i);
    launch_kind<T, TE>(E, EK_YFFT3, -1);  // forward y of theta
    launch_kind<T, TE>(E, EK_ELASTIC, i);
    launch_kind<T, TE>(E, EK_YFFT3, +1);  // inverse y of the elastic potentials
    launch_kind<T, TE>(E, EK_DRIVE, i);
    launch_kind<T, TE>(E, EK_YFFT3, -1);  // forward y of the driving force
    launch_kind<T, TE>(E, EK_FWD_AC, i);
  }
  FinCoef fc;
  std::memset(&fc, 0, sizeof(fc));
  for (int j = 0; j < tb.s; ++j) {
    fc.bE[j] = E->fe_need[j] ? tb.bE[j] : 0.0;
    fc.bI[j] = E->fi_need[j] ? tb.bI[j] : 0.0;
    fc.dE[j] = (tb.has_emb && E->fe_need[j]) ? tb.bE[j] - tb.bt[j] : 0.0;
    fc.dI[j] = (tb.has_emb && E->fi_need[j]) ? tb.bI[j] - tb.bt[j] : 0.0;
  }
  fc.s = tb.s;
  fc.want_err = tb.has_emb;
  fc.fi0_from_y = E->fi0_derived ? 1 : 0;
  if (E->fold_last) {
    const int l = tb.s - 1;
    for (int j = 0; j < tb.s; ++j) fc.bE[j] = fc.bI[j] = fc.dE[j] = fc.dI[j] = 0.0;
    fc.bE[l] = tb.bE[l];
    fc.dE[l] = tb.bE[l] - tb.bt[l];
    fc.fi0_from_y = 0;
    fc.fold = 1;
  }
  const EMemb<T, TE>* mem = (const EMemb<T, TE>*)E->mem_dev;
  kb_finalize<T, TE><<<E->nfin, 256, 0, E->stream>>>(mem, E->st_dev, E->fin_start, E->M, fc, E->partial);
  kb_control<T, TE><<<E->M, 256, 0, E->stream>>>(mem, E->st_dev, E->fin_start, E->partial, tb.emb_order,
                                                  tb.has_emb, nrhs);
}

static void drop_graph(pf_ens* E) {
  if (E->exec) hipGraphExecDestroy(E->exec);
  if (E->graph) hipGraphDestroy(E->graph);
  E->exec = nullptr;
  E->graph = nullptr;
}

static pf_status capture_step(pf_ens* E) {
  drop_graph(E);
  PF_HIP(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
  if (E->mixed)
    enqueue_step<float, float>(E);
  else
    enqueue_step<double, double>(E);
  hipError_t e = hipStreamEndCapture(E->stream, &E->graph);
  if (e != hipSuccess) return PF_ERR_HIP;
  PF_HIP(hipGraphInstantiate(&E->exec, E->graph, nullptr, nullptr, 0));
  return PF_OK;
}

template <typename T, typename TE>
static pf_status build_members(pf_ens* E) {
  std::vector<EMemb<T, TE>> host(E->M);
  for (int m = 0; m < E->M; ++m) {
    pf_ctx* v = E->views[m];
    EMemb<T, TE>& e = host[m];
    std::memset(&e, 0, sizeof(e));
    e.g = v->g;
    e.mk = v->mk;
    e.ybuf[0] = v->y;
    e.ybuf[1] = v->ynew;
    for (int j = 0; j < 6; ++j) {
      e.FI[j] = v->FI[j];
      e.FE[j] = (cx<TE>*)v->FE[j];
    }
    e.T1 = (cx<T>*)v->scratch;
    e.T3 = e.T1 + 4 * v->g.fs;
    if constexpr (sizeof(T) == 8) {
      e.twN = v->tw64[0];
      e.twM = v->tw64[2];
    } else {
      e.twN = v->tw32[0];
      e.twM = v->tw32[2];
    }
  }
  pf_status s = ens_alloc(E, &E->mem_dev, sizeof(EMemb<T, TE>) * E->M);
  if (s != PF_OK) return s;
  PF_HIP(hipMemcpy(E->mem_dev, host.data(), sizeof(EMemb<T, TE>) * E->M, hipMemcpyHostToDevice));
  return PF_OK;
}

extern "C" {

pf_status pf_ensemble_init(int32_t n, const pf_params* per_member, void* stream, pf_ens** out) {
  if (!out || !per_member || n < 1 || n > 4096) return PF_ERR_ARG;
  *out = nullptr;
  const pf_params& p0 = per_member[0];
  for (int m = 0; m < n; ++m) {
    const pf_params& p = per_member[m];
    if (p.nx != p.ny || p.ny != p.nz || !ens_size_ok(p.nx)) return PF_ERR_UNSUPPORTED_SIZE;
    if (!method_embedded(p.method) || p.method != p0.method || p.precision != p0.precision ||
        p.adaptive != p0.adaptive)
      return PF_ERR_ARG;
    if (p.precision != PF_FP64 && p.precision != PF_MIXED) return PF_ERR_ARG;
    if (p.dx <= 0.0 || (p.adaptive && (p.rtol < 0.0 || p.atol <= 0.0))) return PF_ERR_ARG;
    if (p.norm_space != 0) return PF_ERR_ARG;  // ensembles take the k-space norm only
    if (p.elastic_inhom != 0) return PF_ERR_ARG;  // and the homogeneous elasticity
  }
  int ndev = 0;  // no usable device: a HIP error, before any allocation
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return PF_ERR_HIP;
  pf_ens* E = new (std::nothrow) pf_ens();
  if (!E) return PF_ERR_OOM;
  E->M = n;
  E->mixed = p0.precision == PF_MIXED;
  E->prm.assign(per_member, per_member + n);
  if (stream) {
    E->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&E->stream, hipStreamNonBlocking) != hipSuccess) {
      delete E;
      return PF_ERR_HIP;
    }
    E->own_stream = true;
  }
  E->tab = table_for(p0.method);
  for (int i = 0; i < 6; ++i) {
    E->fe_need[i] = fe_needed(E->tab, i);
    E->fi_need[i] = fi_needed(E->tab, i);
  }
  E->fi0_derived = E->tab.AI[0][0] == 0.0 && E->fi_need[0];
  {
    bool same_b = true;
    for (int j = 0; j < E->tab.s; ++j) same_b = same_b && E->tab.bE[j] == E->tab.bI[j];
    E->fold_last = E->tab.has_emb && same_b && E->fi0_derived && E->tab.s >= 2 && E->fe_need[E->tab.s - 1] &&
                   E->fi_need[E->tab.s - 1];
  }
  pf_status s = PF_OK;
  // per-size twiddle tables
  for (int m = 0; m < n && s == PF_OK; ++m) {
    const int N = per_member[m].nz;
    if (E->tw64.count(N)) continue;
    std::vector<cx<double>> a(N), b(N / 2);
    std::vector<cx<float>> af(N), bf(N / 2);
    make_twiddles64(N, a.data());
    make_twiddles64(N / 2, b.data());
    make_twiddles32(N, af.data());
    make_twiddles32(N / 2, bf.data());
    cx<double>*d0, *d1;
    cx<float>*f0, *f1;
    s = ens_alloc(E, (void**)&d0, sizeof(cx<double>) * N);
    if (s == PF_OK) s = ens_alloc(E, (void**)&d1, sizeof(cx<double>) * (N / 2));
    if (s == PF_OK) s = ens_alloc(E, (void**)&f0, sizeof(cx<float>) * N);
    if (s == PF_OK) s = ens_alloc(E, (void**)&f1, sizeof(cx<float>) * (N / 2));
    if (s != PF_OK) break;
    hipMemcpy(d0, a.data(), sizeof(cx<double>) * N, hipMemcpyHostToDevice);
    hipMemcpy(d1, b.data(), sizeof(cx<double>) * (N / 2), hipMemcpyHostToDevice);
    hipMemcpy(f0, af.data(), sizeof(cx<float>) * N, hipMemcpyHostToDevice);
    hipMemcpy(f1, bf.data(), sizeof(cx<float>) * (N / 2), hipMemcpyHostToDevice);
    E->tw64[N] = std::make_pair(d0, d1);
    E->tw32[N] = std::make_pair(f0, f1);
  }
  // per-member buffers and view contexts
  for (int m = 0; m < n && s == PF_OK; ++m) {
    pf_ctx* v = new (std::nothrow) pf_ctx();
    if (!v) {
      s = PF_ERR_OOM;
      break;
    }
    ctx_setup(v, &per_member[m], E->stream);
    v->owns = false;
    E->views.push_back(v);
    const Geo& g = v->g;
    const size_t k64 = sizeof(cx<double>) * 4 * (size_t)g.fs;
    const size_t fe = (E->mixed ? sizeof(cx<float>) : sizeof(cx<double>)) * 4 * (size_t)g.fs;
    const size_t tb = (E->mixed ? sizeof(cx<float>) : sizeof(cx<double>)) * 7 * (size_t)g.fs;
    const size_t rb = sizeof(double) * 4 * (size_t)g.nx * g.ny * g.nz;
    v->scratch_bytes = std::max(tb, rb);
    s = ens_alloc(E, (void**)&v->y, k64);
    if (s == PF_OK) s = ens_alloc(E, (void**)&v->ynew, k64);
    E->yb0.push_back(v->y);
    E->yb1.push_back(v->ynew);
    for (int i = 0; i < 6 && s == PF_OK; ++i) {
      s = ens_alloc(E, (void**)&v->FI[i], k64);
      if (s == PF_OK) s = ens_alloc(E, &v->FE[i], fe);
    }
    if (s == PF_OK) s = ens_alloc(E, &v->scratch, v->scratch_bytes);
    if (s == PF_OK) s = ens_alloc(E, (void**)&v->partial, sizeof(double) * 4 * v->nblk_red);
    if (s == PF_OK) s = ens_alloc(E, (void**)&v->red, sizeof(double) * 8);
    if (s == PF_OK && hipHostMalloc((void**)&v->host_red, sizeof(double) * 8, 0) != hipSuccess) s = PF_ERR_OOM;
    if (s != PF_OK) break;
    const int N = g.nz;
    v->tw64[0] = v->tw64[1] = v->tw64[3] = E->tw64[N].first;
    v->tw64[2] = E->tw64[N].second;
    v->tw32[0] = v->tw32[1] = v->tw32[3] = E->tw32[N].first;
    v->tw32[2] = E->tw32[N].second;
    if (hipMemsetAsync(v->y, 0, k64, E->stream) != hipSuccess) s = PF_ERR_HIP;
  }
  if (s == PF_OK) s = E->mixed ? build_members<float, float>(E) : build_members<double, double>(E);
  if (s == PF_OK) s = build_lists(E);
  if (s == PF_OK) s = ens_alloc(E, (void**)&E->st_dev, sizeof(EState) * n);
  if (s == PF_OK && hipHostMalloc((void**)&E->st_host, sizeof(EState) * n, 0) != hipSuccess) s = PF_ERR_OOM;
  if (s == PF_OK) {
    for (int m = 0; m < n; ++m) {
      EState& x = E->st_host[m];
      std::memset(&x, 0, sizeof(x));
      const pf_params& p = per_member[m];
      x.dt = p.dt0;
      x.dt_next = p.dt0;
      x.rtol = p.rtol;
      x.atol = p.atol;
      x.dt0 = p.dt0;
      x.dt_min = p.dt_min;
      x.dt_max = p.dt_max;
      x.adaptive = p.adaptive;
      x.max_rejects = p.max_rejects > 0 ? p.max_rejects : 10;
      x.done = 1;
    }
    if (hipStreamSynchronize(E->stream) != hipSuccess) s = PF_ERR_HIP;
  }
  if (s != PF_OK) {
    pf_ensemble_finalize(E);
    return s;
  }
  *out = E;
  return PF_OK;
}

void pf_ensemble_finalize(pf_ens* E) {
  if (!E) return;
  if (E->stream) hipStreamSynchronize(E->stream);
  drop_graph(E);
  for (pf_ctx* v : E->views) {
    if (v && v->host_red) hipHostFree(v->host_red);
    pf_finalize(v);
  }
  for (void* p : E->allocs) hipFree(p);
  if (E->st_host) hipHostFree(E->st_host);
  if (E->own_stream && E->stream) hipStreamDestroy(E->stream);
  delete E;
}

int32_t pf_ensemble_size_supported(int32_t n) { return ens_size_ok(n) ? 1 : 0; }

int64_t pf_ensemble_workspace_bytes(const pf_ens* E) { return E ? E->ws_bytes : 0; }

// The member's view context with y / ynew pointing at its current / spare
// state buffer.
static pf_status view_for(pf_ens* E, int32_t m, pf_ctx** v) {
  if (!E || m < 0 || m >= E->M) return PF_ERR_ARG;
  pf_ctx* c = E->views[m];
  const int cur = E->st_host[m].cur;
  c->y = cur ? E->yb1[m] : E->yb0[m];
  c->ynew = cur ? E->yb0[m] : E->yb1[m];
  *v = c;
  return PF_OK;
}

pf_status pf_ensemble_set_state(pf_ens* E, int32_t m, const double* c, const double* eta, int32_t on_device,
                                double t0) {
  if (!E || m < 0 || m >= E->M) return PF_ERR_ARG;
  E->st_host[m].cur = 0;  // state buffer 0 becomes current
  pf_ctx* v;
  pf_status s = view_for(E, m, &v);
  if (s != PF_OK) return s;
  s = pf_set_state(v, c, eta, on_device, t0);
  if (s != PF_OK) return s;
  EState& x = E->st_host[m];
  x.t = t0;
  x.dt = E->prm[m].dt0;
  x.dt_next = E->prm[m].dt0;
  x.steps = x.attempts = x.rejects = x.n_rhs = 0;
  x.rejrow = 0;
  x.prevrej = 0;
  x.done = 1;
  return PF_OK;
}

pf_status pf_ensemble_get_state(pf_ens* E, int32_t m, double* c, double* eta, int32_t on_device) {
  pf_ctx* v;
  pf_status s = view_for(E, m, &v);
  if (s != PF_OK) return s;
  return pf_get_state(v, c, eta, on_device);
}

pf_status pf_ensemble_get_state_hat(pf_ens* E, int32_t m, void* y_hat) {
  pf_ctx* v;
  pf_status s = view_for(E, m, &v);
  if (s != PF_OK) return s;
  return pf_get_state_hat(v, y_hat);
}

pf_status pf_ensemble_diagnostics(pf_ens* E, int32_t m, double* mass, double* vf, double* vf_thr) {
  pf_ctx* v;
  pf_status s = view_for(E, m, &v);
  if (s != PF_OK) return s;
  return pf_diagnostics(v, mass, vf, vf_thr);
}

pf_status pf_ensemble_free_energy(pf_ens* E, int32_t m, double* F) {
  pf_ctx* v;
  pf_status s = view_for(E, m, &v);
  if (s != PF_OK) return s;
  return pf_free_energy(v, F);
}

}  // extern "C"

namespace pf {
// Member access for the surrogate's ensemble advance (same library).
int ens_members(const pf_ens* E) { return E ? E->M : 0; }
int ens_member_n(const pf_ens* E, int m) { return (E && m >= 0 && m < E->M) ? E->prm[m].nz : 0; }
double ens_member_time(const pf_ens* E, int m) { return (E && m >= 0 && m < E->M) ? E->st_host[m].t : 0.0; }
hipStream_t ens_stream(const pf_ens* E) { return E ? E->stream : nullptr; }
// Sets member m's real-space state (device [4][n^3]) and time t, keeping its
// proposed step size and its step counters.
pf_status ens_member_set(pf_ens* E, int m, const double* u, double t) {
  if (!E || m < 0 || m >= E->M || !u) return PF_ERR_ARG;
  EState& x = E->st_host[m];
  x.cur = 0;
  pf_ctx* v;
  pf_status s = view_for(E, m, &v);
  if (s != PF_OK) return s;
  const long long P = (long long)v->g.nx * v->g.ny * v->g.nz;
  s = pf_set_state(v, u, u + P, 1, t);
  if (s != PF_OK) return s;
  x.t = t;
  x.rejrow = 0;
  x.done = 1;
  return PF_OK;
}
}  // namespace pf

extern "C" {

int64_t pf_ensemble_kspace_pitch(const pf_ens* E, int32_t m) {
  if (!E || m < 0 || m >= E->M) return 0;
  return E->views[m]->g.P;
}

pf_status pf_ensemble_advance(pf_ens* E, const double* t_final, int32_t max_steps, pf_stats* per_member) {
  if (!E || !t_final || max_steps < 1) return PF_ERR_ARG;
  for (int m = 0; m < E->M; ++m) {
    EState& x = E->st_host[m];
    x.tf = t_final[m];
    x.rejrow = 0;
    x.done = (x.t >= x.tf * (1.0 - 1e-15)) ? 1 : 0;
    if (!x.done) x.dt = std::min(std::min(x.dt_next, x.dt_max), x.tf - x.t);
  }
  PF_HIP(hipMemcpyAsync(E->st_dev, E->st_host, sizeof(EState) * E->M, hipMemcpyHostToDevice, E->stream));
  if (!E->exec) {
    pf_status s = capture_step(E);
    if (s != PF_OK) return s;
  }
  hipEvent_t e0, e1;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  PF_HIP(hipEventRecord(e0, E->stream));
  int steps = 0;
  pf_status status = PF_OK;
  const int chunk = 4;
  while (steps < max_steps) {
    for (int k = 0; k < chunk && steps < max_steps; ++k, ++steps) PF_HIP(hipGraphLaunch(E->exec, E->stream));
    PF_HIP(hipMemcpyAsync(E->st_host, E->st_dev, sizeof(EState) * E->M, hipMemcpyDeviceToHost, E->stream));
    PF_HIP(hipStreamSynchronize(E->stream));
    bool all = true;
    for (int m = 0; m < E->M; ++m) all = all && E->st_host[m].done != 0;
    if (all) break;
  }
  PF_HIP(hipEventRecord(e1, E->stream));
  PF_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  E->elapsed_ms += ms;
  for (int m = 0; m < E->M; ++m) {
    const EState& x = E->st_host[m];
    if (x.done == 2) status = PF_ERR_STEP_FAIL;
    if (x.done == 3 && status == PF_OK) status = PF_ERR_NONFINITE;
    if (x.done == 0 && status == PF_OK) status = PF_ERR_STATE;  // max_steps reached first
    if (per_member) {
      pf_stats& o = per_member[m];
      std::memset(&o, 0, sizeof(o));
      o.steps = x.steps;
      o.attempts = x.attempts;
      o.rejects = x.rejects;
      o.n_rhs = x.n_rhs;
      o.t = x.t;
      o.dt_last = x.dt_last;
      o.dt_next = x.dt_next;
      o.err_last = x.err;
      o.elapsed_ms = ms;
      o.mass = o.F = o.vf = o.vf_threshold = NAN;
      pf_ctx* v = nullptr;
      double d[4];
      if (view_for(E, m, &v) == PF_OK && v->have_state && ctx_diagnostics(v, true, d) == PF_OK) {
        o.mass = d[0];
        o.vf = d[1];
        o.vf_threshold = d[2];
        o.F = d[3];
      }
    }
  }
  return status;
}

pf_status pf_ensemble_autotune(pf_ens* E, int32_t reps) {
  if (!E || reps < 1) return PF_ERR_ARG;
  // time each kind on all members (state untouched: the stage arrays and
  // temporaries are overwritten, the state buffers only read)
  for (int m = 0; m < E->M; ++m) E->st_host[m].done = 0;
  PF_HIP(hipMemcpyAsync(E->st_dev, E->st_host, sizeof(EState) * E->M, hipMemcpyHostToDevice, E->stream));
  hipEvent_t e0, e1;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  for (int k = 0; k < EK_COUNT; ++k) {
    double best = 1e300;
    int bv = 1;
    for (int v = 0; v < 2; ++v) {
      E->var[k] = v;
      const int stage = (k == EK_YFFT4 || k == EK_YFFT3) ? 1 : 0;
      // the stage kernel differs per stage (number of previous stages, the
      // last stage's update sums): time the whole sequence of a step
      const int s0 = (k == EK_STAGE) ? 0 : stage;
      const int s1 = (k == EK_STAGE) ? E->tab.s : stage + 1;
      auto run = [&]() {
        for (int st = s0; st < s1; ++st) {
          if (E->mixed)
            launch_kind<float, float>(E, k, st);
          else
            launch_kind<double, double>(E, k, st);
        }
      };
      run();
      PF_HIP(hipEventRecord(e0, E->stream));
      for (int r = 0; r < reps; ++r) run();
      PF_HIP(hipEventRecord(e1, E->stream));
      PF_HIP(hipEventSynchronize(e1));
      PF_HIP(hipGetLastError());
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      E->tune_ms[k][v] = ms / reps;
      if (ms < best) {
        best = ms;
        bv = v;
      }
    }
    E->var[k] = bv;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  for (int m = 0; m < E->M; ++m) E->st_host[m].done = 1;
  drop_graph(E);  // re-captured with the chosen plans
  return PF_OK;
}

int32_t pf_ensemble_tuning_kinds(void) { return EK_COUNT; }

const char* pf_ensemble_tuning_name(int32_t k) { return (k >= 0 && k < EK_COUNT) ? ek_names[k] : ""; }

pf_status pf_ensemble_tuning_get(pf_ens* E, int32_t k, int32_t* block_threads, double* ms128, double* ms256) {
  if (!E || k < 0 || k >= EK_COUNT) return PF_ERR_ARG;
  if (block_threads) *block_threads = E->var[k] ? 256 : 128;
  if (ms128) *ms128 = E->tune_ms[k][0];
  if (ms256) *ms256 = E->tune_ms[k][1];
  return PF_OK;
}

pf_status pf_ensemble_tuning_set(pf_ens* E, int32_t k, int32_t block_threads) {
  if (!E || k < 0 || k >= EK_COUNT || (block_threads != 128 && block_threads != 256)) return PF_ERR_ARG;
  E->var[k] = block_threads == 256 ? 1 : 0;
  drop_graph(E);
  return PF_OK;
}

}  // extern "C"
