// libpf host runtime: context, workspace, stage pipeline, step control, C ABI.
//
// Time integration follows Methods, "Time integration": the ImEx-ARK stage
// and update formulas (Eq. ARK_method), the embedded solution
// (Eq. ARK_embedding), the WRMS test (Eqs. wrms_norm, wrms_weights) and the
// reject / recompute / accept cycle.  The implicit stage solve is the per-mode
// division the paper wraps as a custom linear solver; here it is fused into
// the first kernel of every stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/pf.h"
#include "pf_context.hpp"
#include "pf_inhom.hpp"
#include "pf_kernels.hpp"

using namespace pf;

// ---- supported line lengths --------------------------------------------
// Column passes (y, z) take N; row passes (x) take M = nx / 2.
#define PF_COL_SIZES(X)                                                                                  \
  X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64) X(80) X(96) X(128) X(160) X(168) X(192) X(256) X(320) X(336) \
  X(384) X(504) X(512)
#define PF_ROW_SIZES(X)                                                                                         \
  X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(64) X(80) X(84) X(96) X(128) X(160) X(168) X(192) \
  X(252) X(256)

template <class F>
static bool col_dispatch(int n, F&& f) {
  switch (n) {
#define PF_CASE(N)                          \
  case N:                                   \
    f(std::integral_constant<int, N>{});    \
    return true;
    PF_COL_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return false;
  }
}

template <class F>
static bool row_dispatch(int m, F&& f) {
  switch (m) {
#define PF_CASE(N)                          \
  case N:                                   \
    f(std::integral_constant<int, N>{});    \
    return true;
    PF_ROW_SIZES(PF_CASE)
#undef PF_CASE
    default:
      return false;
  }
}

static bool col_supported(int n) {
  return col_dispatch(n, [](auto) {});
}
static bool row_supported(int m) {
  return row_dispatch(m, [](auto) {});
}

// Column-pass tiles: TX consecutive kx columns per work-group, end radix RE.
// Two tile variants per kernel kind, chosen per context by the autotuner
// (pf_autotune): variant 0 gives each row segment `seg0` contiguous bytes,
// variant 1 twice that.  Small lines get wider tiles so a work-group has at
// least one full wavefront; lines shorter than 64 have only variant 0.
static const char* const ck_names[CK_COUNT] = {"colfft", "stage_invz", "zpass_elastic", "zpass_fwd_ac"};
// Largest end radix of each kind's line plan (elem_bytes: 16 FP64, 8 FP32
// complex values).  The FP64 elastic pass holds three fields in registers, so
// it takes narrower tiles and its ends stay at radix 4 where 16 divides the
// line length (half the registers per field of radix 8; radix 8 gained
// nothing at 512^3); lines that 36 divides but 16 does not (504) take radix-6
// ends, since the radix-3 ends they would otherwise get cost the pass a
// quarter more time.  In FP32 the three fields fit at radix 8 (113 VGPRs at
// 512: 8-column tiles ran 1.03 ms against 1.43 ms for 4-column radix-4 ones).
constexpr int col_re(int kind, int elem_bytes = 16) {
  return kind != CK_ELASTIC ? 8 : elem_bytes == 8 ? 8 : 6;
}
constexpr int col_tx(int n, int kind, int elem_bytes, int v) {
  const int seg = (kind == CK_ELASTIC ? 32 : 64) << ((n >= 64) ? v : 0);
  int tx = seg / elem_bytes;
  if (tx < 1) tx = 1;
  while (tx * line_threads(n, col_re(kind, elem_bytes)) < 64 && tx < 16) tx *= 2;
  // long lines with small end radices (504 in the elastic pass: 168 threads
  // per line) stay within 1024 threads per work-group
  while (tx > 1 && tx * line_threads(n, col_re(kind, elem_bytes)) > 1024) tx /= 2;
  return tx;
}
// Whether the wave-specialised column FFT (variant 2 of "colfft") exists for
// lines of length n with elements of elem_bytes.
static bool ws_supported(int n, int elem_bytes) {
  bool ok = false;
  col_dispatch(n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    ok = elem_bytes == 16 ? ws_ok<double, N, col_tx(N, CK_FFT, 16, 1)>()
                          : ws_ok<float, N, col_tx(N, CK_FFT, 8, 1)>();
  });
  return ok;
}
template <class F>
static void with_variant(int v, F&& f) {
  if (v)
    f(std::integral_constant<int, 1>{});
  else
    f(std::integral_constant<int, 0>{});
}
// Rows per row-pass work-group: about 256 threads.
constexpr int rb_of(int m) { return line_threads(m) >= 256 ? 1 : 256 / line_threads(m); }
// Rows per work-group of the stage cycle's theta and drive passes: 128
// threads where the line's thread count divides 128 (their drive pass ran
// 9-16 % faster so, their FP64 theta pass 3-8 %, at 512^3 and 256^3), else
// the general rule (lines of 42 or 84 threads would leave part-filled waves).
constexpr int rb_x(int m) {
  return line_threads(m) <= 128 && 128 % line_threads(m) == 0 ? 128 / line_threads(m) : rb_of(m);
}

#define PF_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return PF_ERR_HIP;           \
  } while (0)

static pf_status dalloc(pf_ctx* c, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return PF_ERR_OOM;
  }
  c->ws_bytes += (int64_t)bytes;
  return PF_OK;
}

template <typename T>
static void make_twiddles(int n, cx<T>* host) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n; ++j) {
    const long double a = 2.0L * pi * (long double)j / (long double)n;
    host[j].re = (T)cosl(a);
    host[j].im = (T)(-sinl(a));
  }
}

static pf_status upload_twiddles(pf_ctx* c, int slot, int n) {
  cx<double>* h64 = new (std::nothrow) cx<double>[n];
  cx<float>* h32 = new (std::nothrow) cx<float>[n];
  if (!h64 || !h32) {
    delete[] h64;
    delete[] h32;
    return PF_ERR_OOM;
  }
  make_twiddles<double>(n, h64);
  make_twiddles<float>(n, h32);
  pf_status s = dalloc(c, (void**)&c->tw64[slot], sizeof(cx<double>) * n);
  if (s == PF_OK) s = dalloc(c, (void**)&c->tw32[slot], sizeof(cx<float>) * n);
  if (s == PF_OK && hipMemcpy(c->tw64[slot], h64, sizeof(cx<double>) * n, hipMemcpyHostToDevice) != hipSuccess)
    s = PF_ERR_HIP;
  if (s == PF_OK && hipMemcpy(c->tw32[slot], h32, sizeof(cx<float>) * n, hipMemcpyHostToDevice) != hipSuccess)
    s = PF_ERR_HIP;
  delete[] h64;
  delete[] h32;
  return s;
}

template <typename T>
static const cx<T>* tw(const pf_ctx* c, int slot) {
  if constexpr (sizeof(T) == 8)
    return c->tw64[slot];
  else
    return c->tw32[slot];
}

static void setup_model(pf_ctx* c) {
  const pf_params& p = c->p;
  ModelK& m = c->mk;
  std::memset(&m, 0, sizeof(m));
  m.M = p.M;
  m.L = p.L;
  m.kc = p.kappa_c;
  m.ke = p.kappa_eta;
  m.ac = p.implicit_bulk_c ? 2.0 * p.W : 0.0;
  m.W = p.W;
  m.w = p.w;
  m.cm = p.c_m;
  m.cp = p.c_p;
  m.fEc = 2.0 * p.W * p.M * (p.c_p - p.c_m);
  m.fEa = (2.0 * p.W - m.ac) * p.M;
  m.C11 = p.C11;
  m.C12 = p.C12;
  m.C44 = p.C44;
  const double n3 = (double)p.nx * p.ny * p.nz;
  m.inv_n3 = 1.0 / n3;
  for (int v = 0; v < 3; ++v) {
    const double* e = p.eps_star[v];
    const double tr = e[0] + e[1] + e[2];
    for (int i = 0; i < 3; ++i) m.S[v][i] = p.C12 * tr + (p.C11 - p.C12) * e[i];
  }
  for (int v = 0; v < 3; ++v)
    for (int w = 0; w < 3; ++w) {
      double s = 0.0;
      for (int i = 0; i < 3; ++i) s += p.eps_star[v][i] * m.S[w][i];
      m.E[v][w] = s;
      m.B0[v][w] = p.mean_strain_mode == 0 ? s : 0.0;
    }
  for (int v = 0; v < 3; ++v) {
    double s = 0.0;
    if (p.mean_strain_mode == 0)
      for (int i = 0; i < 3; ++i) s += p.eps_bar[i] * m.S[v][i];
    m.hom[v] = -n3 * s;
  }
  if (p.elastic_inhom) {
    // cubic compliance from cubic stiffness: S11 = (C11 + C12) / D,
    // S12 = -C12 / D, D = (C11 - C12)(C11 + 2 C12); S44 = 1 / C44
    auto comp = [](double c11, double c12, double c44, double s[3]) {
      const double d = (c11 - c12) * (c11 + 2.0 * c12);
      s[0] = (c11 + c12) / d;
      s[1] = -c12 / d;
      s[2] = 1.0 / c44;
    };
    double sm[3], sp[3];
    comp(p.C11, p.C12, p.C44, sm);
    comp(p.C11p, p.C12p, p.C44p, sp);
    for (int i = 0; i < 3; ++i) {
      m.Sm[i] = sm[i];
      m.dS[i] = sp[i] - sm[i];
    }
    m.C0[0] = 0.5 * (p.C11 + p.C11p);
    m.C0[1] = 0.5 * (p.C12 + p.C12p);
    m.C0[2] = 0.5 * (p.C44 + p.C44p);
    for (int v = 0; v < 3; ++v)
      for (int i = 0; i < 3; ++i) {
        const double* e = p.eps_star[v];
        m.eps[v][i] = e[i];
        m.C0eps[v][i] = m.C0[0] * e[i] + m.C0[1] * (e[(i + 1) % 3] + e[(i + 2) % 3]);
      }
    for (int i = 0; i < 3; ++i) m.ebar[i] = p.eps_bar[i];
  }
}

// ---- launchers ----------------------------------------------------------------
template <typename T, typename TE, int NP>
static void launch_stage_np(pf_ctx* c, const StageArgs<TE>& sa, cx<T>* out) {
  const Geo& g = c->g;
  col_dispatch(g.nz, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    with_variant(c->var[CK_STAGE], [&](auto VC) {
      constexpr int RE = col_re(CK_STAGE);
      constexpr int TX = col_tx(N, CK_STAGE, sizeof(cx<T>), decltype(VC)::value);
      const int nbx = (g.nxh + TX - 1) / TX;
      k_stage_invz<T, TE, N, TX, RE, NP><<<dim3(nbx * g.ny), dim3(ColGeo<N, TX, RE>::THREADS), 0, c->stream>>>(
          sa, g, c->mk, tw<T>(c, 0), out);
    });
  });
}

template <typename T, typename TE>
static bool launch_stage_invz(pf_ctx* c, const StageArgs<TE>& sa, cx<T>* out, int do_fft) {
  if (!col_supported(c->g.nz)) return false;
  if (!do_fft) {
    k_combine<TE><<<dim3(1024), dim3(256), 0, c->stream>>>(sa, c->g, c->mk);
    return true;
  }
  switch (sa.nprev) {
    case 0: launch_stage_np<T, TE, 0>(c, sa, out); break;
    case 1: launch_stage_np<T, TE, 1>(c, sa, out); break;
    case 2: launch_stage_np<T, TE, 2>(c, sa, out); break;
    case 3: launch_stage_np<T, TE, 3>(c, sa, out); break;
    case 4: launch_stage_np<T, TE, 4>(c, sa, out); break;
    case 5: launch_stage_np<T, TE, 5>(c, sa, out); break;
    default: return false;
  }
  return true;
}

template <typename T, int S, int AXIS>
static bool launch_colfft(pf_ctx* c, const cx<T>* in, cx<T>* out, int nf, T scale) {
  const Geo& g = c->g;
  const int n = AXIS == 1 ? g.ny : g.nz;
  const int other = AXIS == 1 ? g.nz : g.ny;
  return col_dispatch(n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    const int var = c->var[CK_FFT];
    with_variant(var ? 1 : 0, [&](auto VC) {
      constexpr int RE = col_re(CK_FFT);
      constexpr int TX = col_tx(N, CK_FFT, sizeof(cx<T>), decltype(VC)::value);
      const int nbx = (g.nxh + TX - 1) / TX;
      if constexpr (ws_ok<T, N, TX, RE>()) {
        if (var == 2) {
          // persistent wave-specialised pass: one work-group per compute unit
          const long long items = (long long)nbx * other * nf;
          const int grid = (int)std::min<long long>(items, c->num_cu);
          k_colfft_ws<T, N, TX, RE, S, AXIS>
              <<<dim3(grid), dim3(ColGeo<N, TX, RE>::THREADS + WS_LOADERS), 0, c->stream>>>(
                  in, out, g, nf, tw<T>(c, AXIS == 1 ? 1 : 0), scale);
          return;
        }
      }
      k_colfft<T, N, TX, RE, S, AXIS><<<dim3(nbx * other), dim3(ColGeo<N, TX, RE>::THREADS), 0, c->stream>>>(
          in, out, g, nf, tw<T>(c, AXIS == 1 ? 1 : 0), scale);
    });
  });
}

template <typename T, typename TE>
static bool launch_zpass_elastic(pf_ctx* c, cx<T>* th, cx<TE>* FEc, int accumulate) {
  const Geo& g = c->g;
  return col_dispatch(g.nz, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    with_variant(c->var[CK_ELASTIC], [&](auto VC) {
      constexpr int RE = col_re(CK_ELASTIC, sizeof(cx<T>));
      constexpr int TX = col_tx(N, CK_ELASTIC, sizeof(cx<T>), decltype(VC)::value);
      const int nbx = (g.nxh + TX - 1) / TX;
      k_zpass_elastic<T, TE, N, TX, RE><<<dim3(nbx * g.ny), dim3(ColGeo<N, TX, RE>::THREADS), 0, c->stream>>>(
          th, g, c->mk, tw<T>(c, 0), FEc, accumulate);
    });
  });
}

template <typename T, typename TE>
static bool launch_zpass_fwd_ac(pf_ctx* c, const cx<T>* gk, cx<TE>* FE) {
  const Geo& g = c->g;
  return col_dispatch(g.nz, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    with_variant(c->var[CK_FWD_AC], [&](auto VC) {
      constexpr int RE = col_re(CK_FWD_AC);
      constexpr int TX = col_tx(N, CK_FWD_AC, sizeof(cx<T>), decltype(VC)::value);
      const int nbx = (g.nxh + TX - 1) / TX;
      k_zpass_fwd_ac<T, TE, N, TX, RE><<<dim3(nbx * g.ny), dim3(ColGeo<N, TX, RE>::THREADS), 0, c->stream>>>(
          gk, g, c->mk, tw<T>(c, 0), FE);
    });
  });
}

template <typename T>
static bool launch_xpass_theta(pf_ctx* c, const cx<T>* st, cx<T>* th) {
  const Geo& g = c->g;
  return row_dispatch(g.nx / 2, [&](auto MC) {
    constexpr int M = decltype(MC)::value;
    constexpr int RB = rb_x(M);
    const int nrows = g.nz * g.ny;
    k_xpass_theta<T, M, RB><<<dim3((nrows + RB - 1) / RB), dim3(RowGeo<M, RB>::THREADS), 0, c->stream>>>(
        st, th, g, tw<T>(c, 3), tw<T>(c, 2));
  });
}

template <typename T>
static bool launch_xpass_drive(pf_ctx* c, const cx<T>* st, cx<T>* el) {
  const Geo& g = c->g;
  return row_dispatch(g.nx / 2, [&](auto MC) {
    constexpr int M = decltype(MC)::value;
    constexpr int RB = rb_x(M);
    const int nrows = g.nz * g.ny;
    k_xpass_drive<T, M, RB><<<dim3((nrows + RB - 1) / RB), dim3(RowGeo<M, RB>::THREADS), 0, c->stream>>>(
        st, el, g, c->mk, tw<T>(c, 3), tw<T>(c, 2));
  });
}

static bool launch_xpass_r2c(pf_ctx* c, const double* re, cx<double>* out, int nf) {
  const Geo& g = c->g;
  return row_dispatch(g.nx / 2, [&](auto MC) {
    constexpr int M = decltype(MC)::value;
    constexpr int RB = rb_of(M);
    const int nrows = g.nz * g.ny;
    k_xpass_r2c<double, M, RB><<<dim3((nrows + RB - 1) / RB), dim3(RowGeo<M, RB>::THREADS), 0, c->stream>>>(
        re, out, g, nf, tw<double>(c, 3), tw<double>(c, 2));
  });
}

static bool launch_xpass_c2r(pf_ctx* c, const cx<double>* in, double* re, int nf, double scale) {
  const Geo& g = c->g;
  return row_dispatch(g.nx / 2, [&](auto MC) {
    constexpr int M = decltype(MC)::value;
    constexpr int RB = rb_of(M);
    const int nrows = g.nz * g.ny;
    k_xpass_c2r<double, M, RB><<<dim3((nrows + RB - 1) / RB), dim3(RowGeo<M, RB>::THREADS), 0, c->stream>>>(
        in, re, g, nf, scale, tw<double>(c, 3), tw<double>(c, 2));
  });
}

// ---- per-kernel-class timing --------------------------------------------------
enum KClass {
  KC_STAGE = 0, KC_YFFT, KC_THETA, KC_ELASTIC, KC_DRIVE, KC_ZFWD_AC, KC_FINAL,
  KC_XR2C, KC_XC2R, KC_ZFFT, KC_EL_K, KC_EL_TAU, KC_EL_STRAIN, KC_EL_DRIVE, KC_EL_LOCAL, KC_EL_ZGAMMA, KC_COUNT
};
static const char* const kc_names[KC_COUNT] = {
    "stage_invz", "ypass", "xpass_theta", "zpass_elastic", "xpass_drive",
    "zpass_fwd_ac", "finalize", "xpass_r2c", "xpass_c2r", "zpass",
    "el_kspace", "el_tau", "el_strain", "el_drive", "el_local", "el_zgamma"};

static void prof_begin(pf_ctx* c) {
  if (!c->prof_on) return;
  if (c->prof_used + 2 > c->prof_ev.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      c->prof_ev.push_back(e);
    }
  }
  hipEventRecord(c->prof_ev[c->prof_used], c->stream);
}

static void prof_end(pf_ctx* c, int cls, double bytes) {
  if (!c->prof_on || c->prof_used + 2 > c->prof_ev.size()) return;
  hipEventRecord(c->prof_ev[c->prof_used + 1], c->stream);
  c->prof_used += 2;
  c->prof_pending.push_back(std::make_pair(cls, bytes));
}

// Call after the stream has been synchronised.
static void prof_resolve(pf_ctx* c) {
  if (!c->prof_on) return;
  for (size_t i = 0; i < c->prof_pending.size(); ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]) == hipSuccess) {
      const int k = c->prof_pending[i].first;
      c->prof_ms[k] += ms;
      c->prof_n[k] += 1;
      c->prof_bytes[k] += c->prof_pending[i].second;
    }
  }
  c->prof_pending.clear();
  c->prof_used = 0;
}

// ---- inhomogeneous elasticity: the Hu-Chen iteration ---------------------------
template <int K>
static bool launch_el_rows(pf_ctx* c, const cx<double>* T1, cx<double>* out, double* mx) {
  const Geo& g = c->g;
  return row_dispatch(g.nx / 2, [&](auto MC) {
    constexpr int M = decltype(MC)::value;
    // 128-thread groups for the drive and local-coefficient kernels (0.64 ->
    // 0.58 ms and 0.27 -> 0.26 ms at 256^3), 256-thread ones for the strain
    // kernel (5 % slower at 128), the update and the energy sums
    constexpr int RB = (K == 2 || K == 4) ? rb_x(M) : rb_of(M);
    const int nb = (g.nz * g.ny + RB - 1) / RB;
    const dim3 blk(RowGeo<M, RB>::THREADS);
    const cx<double>* twN = tw<double>(c, 3);
    const cx<double>* twM = tw<double>(c, 2);
    if constexpr (K == 0)
      k_el_strain<M, RB><<<nb, blk, 0, c->stream>>>(c->E6, c->R6, g, twN, twM, mx);
    else if constexpr (K == 1)
      k_el_tau<M, RB><<<nb, blk, 0, c->stream>>>(c->LC6, c->R6, c->E6, g, twN, twM);
    else if constexpr (K == 4)
      k_el_local<M, RB><<<nb, blk, 0, c->stream>>>(T1, c->LC6, g, c->mk, twN, twM);
    else if constexpr (K == 2)
      k_el_drive<M, RB><<<nb, blk, 0, c->stream>>>(T1, c->R6, out, g, c->mk, twN, twM);
    else
      k_el_energy<M, RB><<<nb, blk, 0, c->stream>>>(T1, c->R6, g, c->mk, twN, twM, c->el_part);
  });
}
// Columns per work-group of the fused Green-operator z pass: at least 64
// threads, at least two columns; four (64-byte row segments) for lines of 32
// to 64 threads (128 to 256 points: at 256^3 0.48 ms against 0.55 ms for
// 2-column tiles, whose 32-byte segments leave cache lines half-written).
constexpr int el_ztx(int n) {
  return line_threads(n, 4) >= 32 ? (line_threads(n, 4) <= 64 ? 4 : 2) : 64 / line_threads(n, 4);
}

static bool launch_el_zgamma(pf_ctx* c, double scale) {
  const Geo& g = c->g;
  return col_dispatch(g.nz, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int TX = el_ztx(N);
    const int nbx = (g.nxh + TX - 1) / TX;
    k_el_zgamma<N, TX, 4><<<dim3(nbx * g.ny), dim3(ColGeo<N, TX, 4>::THREADS), 0, c->stream>>>(
        c->E6, g, c->mk, tw<double>(c, 0), scale);
  });
}

static int el_row_blocks(const pf_ctx* c) {
  int nb = 0;
  row_dispatch(c->g.nx / 2, [&](auto MC) {
    constexpr int M = decltype(MC)::value;
    nb = (c->g.nz * c->g.ny + rb_of(M) - 1) / rb_of(M);  // the energy kernel's groups
  });
  return nb;
}

// Strain of the periodic displacement at mechanical equilibrium for the order
// parameters in T1 (the state after its inverse z and y transforms): the
// start from theta~, then updates until the largest change of a strain
// component is <= el_tol or el_max_iter updates; the result is in R6.  With
// FE0, the explicit Cahn-Hilliard term (from H~, which the start has at hand)
// goes into FE0 (added with `accumulate`).  T3 and E6 are used as temporaries.
static pf_status el_solve(pf_ctx* c, cx<double>* T1, cx<double>* FE0, int accumulate) {
  const Geo& g = c->g;
  cx<double>* T3 = T1 + 4 * g.fs;
  const double nv = (double)g.nz * g.ny * g.nxh;
  const double fk = nv * sizeof(cx<double>), fr = (double)g.nx * g.ny * g.nz * sizeof(double);
  const long long modes = (long long)g.nz * g.ny * g.nxh;
  const int kgrid = (int)std::min<long long>((modes + 255) / 256, 16384);
  const double s = c->mk.inv_n3;
  bool ok = true;
  // E6 spectra -> R6 real strain (the z inverse only with `zinv`)
  auto back = [&](double* mx, bool zinv) {
    if (zinv) {
      prof_begin(c);
      ok = ok && launch_colfft<double, +1, 2>(c, c->E6, c->E6, 6, s);
      prof_end(c, KC_ZFFT, 12 * fk);
    }
    prof_begin(c);
    ok = ok && launch_colfft<double, +1, 1>(c, c->E6, c->E6, 6, 1.0);
    prof_end(c, KC_YFFT, 12 * fk);
    prof_begin(c);
    ok = ok && launch_el_rows<0>(c, nullptr, nullptr, mx);
    prof_end(c, KC_EL_STRAIN, 6 * fk + (mx ? 12 : 6) * fr);
  };
  prof_begin(c);
  ok = ok && launch_xpass_theta<double>(c, T1, T3);
  prof_end(c, KC_THETA, 6 * fk);
  prof_begin(c);
  ok = ok && launch_colfft<double, -1, 1>(c, T3, T3, 3, 1.0);
  prof_end(c, KC_YFFT, 6 * fk);
  prof_begin(c);
  ok = ok && launch_colfft<double, -1, 2>(c, T3, T3, 3, 1.0);
  prof_end(c, KC_ZFFT, 6 * fk);
  prof_begin(c);
  k_el_start<<<kgrid, 256, 0, c->stream>>>(T3, c->E6, FE0, accumulate, g, c->mk);
  prof_end(c, KC_EL_K, (9.0 + (FE0 ? (accumulate ? 2 : 1) : 0)) * fk);
  prof_begin(c);
  ok = ok && launch_el_rows<4>(c, T1, nullptr, nullptr);
  prof_end(c, KC_EL_LOCAL, 3 * fk + 6 * fr);
  back(nullptr, true);
  int it = 0;
  while (ok && it < c->p.el_max_iter) {
    prof_begin(c);
    ok = ok && launch_el_rows<1>(c, T1, nullptr, nullptr);
    prof_end(c, KC_EL_TAU, 6 * fk + 12 * fr);  // coefficients and strain read, six spectra written
    prof_begin(c);
    ok = ok && launch_colfft<double, -1, 1>(c, c->E6, c->E6, 6, 1.0);
    prof_end(c, KC_YFFT, 12 * fk);
    // forward z, Gamma0 and the scaled inverse z in one pass
    prof_begin(c);
    ok = ok && launch_el_zgamma(c, s);
    prof_end(c, KC_EL_ZGAMMA, 12 * fk);
    k_el_zero<<<1, 1, 0, c->stream>>>(c->elmax);
    back(c->elmax, false);
    ++it;
    if (!ok) break;
    PF_HIP(hipMemcpyAsync(&c->host_red[6], c->elmax, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PF_HIP(hipStreamSynchronize(c->stream));
    if (c->host_red[6] <= c->p.el_tol) break;  // a NaN change never stops early
  }
  if (!ok) return PF_ERR_UNSUPPORTED_SIZE;
  if (hipGetLastError() != hipSuccess) return PF_ERR_HIP;
  c->st.el_iterations += it;
  c->st.el_last = it;
  return PF_OK;
}

// The explicit right-hand side after the state's inverse z and y transforms,
// with the inhomogeneous elastic force: equilibrium strain, driving forces,
// forward transforms into FE (fields 1..3; field 0 from the strain's start).
static pf_status run_rhs_inhom(pf_ctx* c, cx<double>* T1, cx<double>* FE, int accumulate) {
  const Geo& g = c->g;
  cx<double>* T3 = T1 + 4 * g.fs;
  const double nv = (double)g.nz * g.ny * g.nxh;
  const double fk = nv * sizeof(cx<double>), fr = (double)g.nx * g.ny * g.nz * sizeof(double);
  pf_status st = el_solve(c, T1, FE, accumulate);
  if (st != PF_OK) return st;
  bool ok = true;
  prof_begin(c);
  ok = ok && launch_el_rows<2>(c, T1, T3, nullptr);
  prof_end(c, KC_EL_DRIVE, 7 * fk + 6 * fr);
  prof_begin(c);
  ok = ok && launch_colfft<double, -1, 1>(c, T3, T3, 3, 1.0);
  prof_end(c, KC_YFFT, 6 * fk);
  prof_begin(c);
  ok = ok && launch_zpass_fwd_ac<double, double>(c, T3, FE);
  prof_end(c, KC_ZFWD_AC, 6 * fk);
  if (!ok) return PF_ERR_UNSUPPORTED_SIZE;
  if (hipGetLastError() != hipSuccess) return PF_ERR_HIP;
  return PF_OK;
}

// ---- one stage: combine / implicit solve, then the explicit RHS chain ---------
template <typename T, typename TE>
static pf_status run_stage(pf_ctx* c, const StageArgs<TE>& sa, bool need_rhs, cx<TE>* FE_out) {
  cx<T>* T1 = (cx<T>*)c->scratch;
  cx<T>* T3 = T1 + 4 * c->g.fs;
  // algorithmic bytes: one valid half-spectrum field in T, TE and FP64
  const double nv = (double)c->g.nz * c->g.ny * c->g.nxh;
  const double fT = nv * sizeof(cx<T>), fE = nv * sizeof(cx<TE>), f64 = nv * sizeof(cx<double>);
  double b_stage = 4 * f64;  // state read
  const bool fold = sa.U_out != nullptr;
  for (int j = 0; j < sa.nprev; ++j) {
    const bool useF = fold && (sa.ub[j] != 0.0 || sa.eb[j] != 0.0);
    const bool useE = sa.cE[j] != 0.0 || useF;
    const bool useI = sa.cI[j] != 0.0 || useF;
    b_stage += 4 * ((useE ? fE : 0.0) + ((useI && !(j == 0 && sa.fi0_from_y)) ? f64 : 0.0));
  }
  b_stage += (sa.FI_out ? 4 * f64 : 0.0) + (sa.FEc_out ? fE : 0.0) + (need_rhs ? 4 * fT : 0.0);
  b_stage += fold ? 2 * 4 * f64 : 0.0;  // U and E
  prof_begin(c);
  if (!launch_stage_invz<T, TE>(c, sa, T1, need_rhs ? 1 : 0)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_STAGE, b_stage);
  if (need_rhs) {
    const int acc = (sa.FEc_out != nullptr) ? 1 : 0;
    bool ok = true;
    prof_begin(c);
    ok = ok && launch_colfft<T, +1, 1>(c, T1, T1, 4, (T)1);
    prof_end(c, KC_YFFT, 8 * fT);
    if constexpr (std::is_same<T, double>::value && std::is_same<TE, double>::value) {
      if (c->inhom) {
        if (!ok) return PF_ERR_UNSUPPORTED_SIZE;
        return run_rhs_inhom(c, T1, FE_out, acc);
      }
    }
    prof_begin(c);
    ok = ok && launch_xpass_theta<T>(c, T1, T3);
    prof_end(c, KC_THETA, 6 * fT);
    prof_begin(c);
    ok = ok && launch_colfft<T, -1, 1>(c, T3, T3, 3, (T)1);
    prof_end(c, KC_YFFT, 6 * fT);
    prof_begin(c);
    ok = ok && launch_zpass_elastic<T, TE>(c, T3, FE_out, acc);
    prof_end(c, KC_ELASTIC, 6 * fT + (acc ? 2 : 1) * fE);
    prof_begin(c);
    ok = ok && launch_colfft<T, +1, 1>(c, T3, T3, 3, (T)1);
    prof_end(c, KC_YFFT, 6 * fT);
    prof_begin(c);
    ok = ok && launch_xpass_drive<T>(c, T1, T3);
    prof_end(c, KC_DRIVE, 10 * fT);
    prof_begin(c);
    ok = ok && launch_colfft<T, -1, 1>(c, T3, T3, 3, (T)1);
    prof_end(c, KC_YFFT, 6 * fT);
    prof_begin(c);
    ok = ok && launch_zpass_fwd_ac<T, TE>(c, T3, FE_out);
    prof_end(c, KC_ZFWD_AC, 3 * fT + 3 * fE);
    if (!ok) return PF_ERR_UNSUPPORTED_SIZE;
  }
  if (hipGetLastError() != hipSuccess) return PF_ERR_HIP;
  return PF_OK;
}

template <typename T, typename TE>
static pf_status stages_and_finalize(pf_ctx* c, double dt, int* n_rhs) {
  const ArkTable& tb = c->tab;
  *n_rhs = 0;
  for (int i = 0; i < tb.s; ++i) {
    StageArgs<TE> sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.y = c->y;
    for (int j = 0; j < i; ++j) {
      sa.FE[j] = (const cx<TE>*)c->FE[j];
      sa.FI[j] = c->FI[j];
      sa.cE[j] = (c->fe_need[j] ? dt * tb.AE[i][j] : 0.0);
      sa.cI[j] = (c->fi_need[j] ? dt * tb.AI[i][j] : 0.0);
    }
    sa.nprev = i;
    sa.gdt = dt * tb.AI[i][i];
    sa.fi0_from_y = c->fi0_derived ? 1 : 0;
    sa.FI_out = (c->fi_need[i] && !(i == 0 && c->fi0_derived)) ? c->FI[i] : nullptr;
    if (c->fold_last && i == tb.s - 1) {
      sa.FI_out = nullptr;  // this stage's F^I enters U and E only
      sa.U_out = c->FI[i];
      sa.E_out = c->FI[0];
      for (int j = 0; j < i; ++j) {  // b^E = b^I here (fold_last); zero weights read nothing
        sa.ub[j] = tb.bI[j];
        sa.eb[j] = tb.bI[j] - tb.bt[j];
      }
      sa.ubs = tb.bI[i];
      sa.ebs = tb.bI[i] - tb.bt[i];
      sa.fdt = dt;
    }
    const bool need_rhs = c->fe_need[i];
    sa.FEc_out = (need_rhs && c->mk.fEa != 0.0) ? (cx<TE>*)c->FE[i] : nullptr;
    pf_status s = run_stage<T, TE>(c, sa, need_rhs, (cx<TE>*)c->FE[i]);
    if (s != PF_OK) return s;
    if (need_rhs) ++*n_rhs;
  }
  FinArgs<TE> fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.y = c->y;
  fa.ynew = c->ynew;
  for (int j = 0; j < tb.s; ++j) {
    fa.FE[j] = (const cx<TE>*)c->FE[j];
    fa.FI[j] = c->FI[j];
    fa.bE[j] = c->fe_need[j] ? dt * tb.bE[j] : 0.0;
    fa.bI[j] = c->fi_need[j] ? dt * tb.bI[j] : 0.0;
    fa.dE[j] = (tb.has_emb && c->fe_need[j]) ? dt * (tb.bE[j] - tb.bt[j]) : 0.0;
    fa.dI[j] = (tb.has_emb && c->fi_need[j]) ? dt * (tb.bI[j] - tb.bt[j]) : 0.0;
  }
  fa.s = tb.s;
  fa.want_err = tb.has_emb;
  fa.fi0_from_y = c->fi0_derived ? 1 : 0;
  if (c->fold_last) {  // everything but the last stage's F^E is in U and E
    const int l = tb.s - 1;
    for (int j = 0; j < tb.s; ++j) fa.bE[j] = fa.bI[j] = fa.dE[j] = fa.dI[j] = 0.0;
    fa.bE[l] = dt * tb.bE[l];
    fa.dE[l] = dt * (tb.bE[l] - tb.bt[l]);
    fa.fi0_from_y = 0;
    fa.U = c->FI[l];
    fa.E = c->FI[0];
  }
  fa.rtol = c->p.rtol;
  fa.atol = c->p.atol;
  fa.sc = 1.0 / std::sqrt((double)c->g.nx * c->g.ny * c->g.nz);
  fa.partial = c->partial;
  fa.err_out = (c->norm_real && tb.has_emb) ? c->FI[0] : nullptr;
  // y read + ynew write (4 complex FP64 fields each)
  double b_fin = 2.0 * 4 * c->g.nz * (double)c->g.ny * c->g.nxh * sizeof(cx<double>);
  if (fa.U) b_fin += 2.0 * 4 * c->g.nz * (double)c->g.ny * c->g.nxh * sizeof(cx<double>);  // U and E
  for (int j = 0; j < tb.s; ++j) {
    const double nv = 4.0 * c->g.nz * (double)c->g.ny * c->g.nxh;
    if ((fa.bI[j] != 0.0 || fa.dI[j] != 0.0) && !(j == 0 && fa.fi0_from_y)) b_fin += nv * sizeof(cx<double>);
    if (fa.bE[j] != 0.0 || fa.dE[j] != 0.0) b_fin += nv * sizeof(cx<TE>);
  }
  prof_begin(c);
  k_finalize<TE><<<dim3(c->nblk_red), dim3(256), 0, c->stream>>>(fa, c->g, c->mk);
  k_reduce_pairs<<<dim3(1), dim3(256), 0, c->stream>>>(c->partial, c->nblk_red, c->red);
  prof_end(c, KC_FINAL, b_fin);
  if (hipGetLastError() != hipSuccess) return PF_ERR_HIP;
  return PF_OK;
}

// Elementary I-controller (the paper leaves the formula to the integration
// library): dt * min(5, max(0.2, 0.9 err^(-1/(q+1)))), 0.25 dt after a
// non-finite attempt; `after_reject` (this attempt accepted, the previous one
// rejected) caps the factor at 1, the facmax = 1 rule of Hairer, Norsett and
// Wanner right after a rejection.
static double controller(double dt, double err, int q, bool after_reject) {
  if (!std::isfinite(err)) return 0.25 * dt;
  double fac;
  if (err == 0.0)
    fac = 5.0;
  else
    fac = std::min(5.0, std::max(0.2, 0.9 * std::pow(err, -1.0 / (q + 1))));
  if (after_reject) fac = std::min(1.0, fac);
  return dt * fac;
}



// ---- streaming-bandwidth probe kernels (measurement aid) ----------------------
namespace {
typedef double probe_d2 __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(256) k_probe_copy(const probe_d2* __restrict__ a, probe_d2* __restrict__ b,
                                                    long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) b[i] = a[i];
}
__global__ void __launch_bounds__(256) k_probe_read(const probe_d2* __restrict__ a, long long n,
                                                    double* __restrict__ sink) {
  double s = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const probe_d2 v = a[i];
    s += v.x + v.y;
  }
  if (s == -1.0) sink[0] = s;  // keeps the loads; never true for the zero-filled input
}
// eleven read streams and one write stream, the shape of the ARK4 update
__global__ void __launch_bounds__(256) k_probe_multi(const probe_d2* __restrict__ a, probe_d2* __restrict__ b,
                                                     long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    probe_d2 v[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) v[k] = a[i + k * n];
    probe_d2 acc = v[0];
#pragma unroll
    for (int k = 1; k < 11; ++k) acc += 0.5 * v[k];
    b[i] = acc;
  }
}
}  // namespace

namespace pf {
void ctx_setup(pf_ctx* c, const pf_params* p, hipStream_t stream) {
  c->p = *p;
  if (c->p.max_rejects <= 0) c->p.max_rejects = 10;
  c->stream = stream;
  hipGetDevice(&c->device);
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
    c->num_cu = ncu;
  c->mixed = p->precision == PF_MIXED;
  c->norm_real = p->norm_space == 1;
  c->inhom = p->elastic_inhom == 1;
  Geo& g = c->g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.nxh = p->nx / 2 + 1;
  g.P = (g.nxh + 7) / 8 * 8;
  g.fs = (long long)g.nz * g.ny * g.P;
  const double twopi = 6.283185307179586476925286766559;
  g.kfx = twopi / (p->nx * p->dx);
  g.kfy = twopi / (p->ny * p->dx);
  g.kfz = twopi / (p->nz * p->dx);
  setup_model(c);
  c->tab = table_for(p->method);
  for (int i = 0; i < c->tab.s; ++i) {
    c->fe_need[i] = fe_needed(c->tab, i);
    c->fi_need[i] = fi_needed(c->tab, i);
  }
  // explicit first stage: its value is the state, F^I_1 = L y is formed where used
  c->fi0_derived = c->tab.AI[0][0] == 0.0 && c->fi_need[0];
  {
    const int l = c->tab.s - 1;
    bool same_b = true;  // one weight set for the explicit and implicit parts
    for (int j = 0; j < c->tab.s; ++j) same_b = same_b && c->tab.bE[j] == c->tab.bI[j];
    c->fold_last = c->tab.has_emb && same_b && c->fi0_derived && l >= 1 && c->fe_need[l] && c->fi_need[l];
  }
  std::memset(&c->st, 0, sizeof(c->st));
  c->dt_next = p->dt0;
  c->st.dt_min_seen = 1e300;
}
void make_twiddles64(int n, cx<double>* host) { make_twiddles<double>(n, host); }
void make_twiddles32(int n, cx<float>* host) { make_twiddles<float>(n, host); }
}  // namespace pf

// ---- C ABI ---------------------------------------------------------------------
extern "C" {

pf_status pf_bandwidth_probe(int64_t bytes, int32_t reps, void* stream, double* copy_gbs, double* read_gbs,
                             double* multi_gbs) {
  if (bytes < (1 << 20) || reps < 1) return PF_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const long long n = bytes / 16;
  probe_d2 *a = nullptr, *b = nullptr;
  double* sink = nullptr;
  if (hipMalloc((void**)&a, 11 * 16 * (size_t)n) != hipSuccess) return PF_ERR_OOM;
  if (hipMalloc((void**)&b, 16 * (size_t)n) != hipSuccess || hipMalloc((void**)&sink, 8) != hipSuccess) {
    hipFree(a);
    hipFree(b);
    return PF_ERR_OOM;
  }
  pf_status res = PF_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMemsetAsync(a, 0, 11 * 16 * (size_t)n, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    res = PF_ERR_HIP;
  const int grid = 1024;
  auto best = [&](auto launch, double traffic) -> double {
    double b_ms = 1e300;
    launch();
    for (int r = 0; r < reps && res == PF_OK; ++r) {
      float ms = 0.f;
      if (hipEventRecord(e0, st) != hipSuccess) res = PF_ERR_HIP;
      launch();
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        res = PF_ERR_HIP;
      if (ms > 0.f && ms < b_ms) b_ms = ms;
    }
    return traffic / (b_ms * 1e-3) / 1e9;
  };
  const double bb = 16.0 * n;
  if (res == PF_OK) {
    const double c = best([&] { k_probe_copy<<<grid, 256, 0, st>>>(a, b, n); }, 2 * bb);
    const double r = best([&] { k_probe_read<<<grid, 256, 0, st>>>(a, n, sink); }, bb);
    const double m = best([&] { k_probe_multi<<<grid, 256, 0, st>>>(a, b, n); }, 12 * bb);
    if (hipGetLastError() != hipSuccess) res = PF_ERR_HIP;
    if (copy_gbs) *copy_gbs = c;
    if (read_gbs) *read_gbs = r;
    if (multi_gbs) *multi_gbs = m;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(st);
  hipFree(a);
  hipFree(b);
  hipFree(sink);
  return res;
}

#ifndef PF_BUILD_ID
#define PF_BUILD_ID "unversioned"
#endif
const char* pf_build_id(void) { return PF_BUILD_ID; }

const char* pf_status_string(pf_status s) {
  switch (s) {
    case PF_OK: return "PF_OK";
    case PF_ERR_ARG: return "PF_ERR_ARG";
    case PF_ERR_OOM: return "PF_ERR_OOM";
    case PF_ERR_HIP: return "PF_ERR_HIP";
    case PF_ERR_UNSUPPORTED_SIZE: return "PF_ERR_UNSUPPORTED_SIZE";
    case PF_ERR_STEP_FAIL: return "PF_ERR_STEP_FAIL";
    case PF_ERR_NONFINITE: return "PF_ERR_NONFINITE";
    case PF_ERR_STATE: return "PF_ERR_STATE";
  }
  return "PF_UNKNOWN_STATUS";
}

pf_status pf_default_params(pf_params* p) {
  if (!p) return PF_ERR_ARG;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 32;
  p->dx = 1.0;
  p->W = p->w = p->kappa_c = p->kappa_eta = p->M = p->L = 1.0;
  p->c_m = 0.02;
  p->c_p = 0.25;
  p->C11 = 250.0;
  p->C12 = 150.0;
  p->C44 = 120.0;
  for (int v = 0; v < 3; ++v)
    for (int i = 0; i < 3; ++i) p->eps_star[v][i] = (v == i) ? 0.0286 : 0.0067;
  p->mean_strain_mode = 0;
  p->implicit_bulk_c = 1;
  p->precision = PF_FP64;
  p->method = PF_ARK436L;
  p->adaptive = 0;
  p->dt0 = 1e-2;
  p->rtol = 1e-6;
  p->atol = 1e-9;
  p->dt_min = 0.0;
  p->dt_max = 1e300;
  p->max_rejects = 10;
  p->norm_space = 0;
  p->elastic_inhom = 0;
  p->C11p = p->C11;
  p->C12p = p->C12;
  p->C44p = p->C44;
  p->el_tol = 1e-16;
  p->el_max_iter = 50;
  return PF_OK;
}

int32_t pf_size_supported(int32_t n) {
  if (n < 8 || n > 512 || n % 8 != 0) return 0;
  return (col_supported(n) && row_supported(n / 2)) ? 1 : 0;
}

void pf_finalize(pf_ctx* c) {
  if (!c) return;
  if (!c->owns) {  // a view: buffers belong to the owner
    for (hipEvent_t e : c->prof_ev) hipEventDestroy(e);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    delete c;
    return;
  }
  hipFree(c->y);
  hipFree(c->ynew);
  hipFree(c->ycopy);
  hipFree(c->E6);
  hipFree(c->R6);
  hipFree(c->LC6);
  hipFree(c->elmax);
  hipFree(c->el_part);
  for (int i = 0; i < 6; ++i) {
    hipFree(c->FI[i]);
    hipFree(c->FE[i]);
  }
  hipFree(c->scratch);
  hipFree(c->partial);
  hipFree(c->red);
  if (c->host_red) hipHostFree(c->host_red);
  for (int s = 0; s < 4; ++s) {
    hipFree(c->tw64[s]);
    hipFree(c->tw32[s]);
  }
  for (hipEvent_t e : c->prof_ev) hipEventDestroy(e);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  delete c;
}

pf_status pf_init(const pf_params* p, void* stream, pf_ctx** out) {
  if (!p || !out) return PF_ERR_ARG;
  *out = nullptr;
  if (p->dx <= 0.0 || p->M < 0.0 || p->L < 0.0 || p->kappa_c < 0.0 || p->kappa_eta < 0.0)
    return PF_ERR_ARG;
  if (p->precision != PF_FP64 && p->precision != PF_MIXED) return PF_ERR_ARG;
  if (!method_ok(p->method)) return PF_ERR_ARG;
  if (p->adaptive && !method_embedded(p->method)) return PF_ERR_ARG;
  if (p->adaptive && (p->rtol < 0.0 || p->atol <= 0.0)) return PF_ERR_ARG;
  if (p->mean_strain_mode != 0 && p->mean_strain_mode != 1) return PF_ERR_ARG;
  if (p->norm_space != 0 && p->norm_space != 1) return PF_ERR_ARG;
  if (p->elastic_inhom != 0 && p->elastic_inhom != 1) return PF_ERR_ARG;
  if (p->elastic_inhom) {
    // stable cubic stiffnesses, FP64, a prescribed mean strain
    auto stable = [](double c11, double c12, double c44) {
      return c11 - c12 > 0.0 && c11 + 2.0 * c12 > 0.0 && c44 > 0.0;
    };
    if (!stable(p->C11, p->C12, p->C44) || !stable(p->C11p, p->C12p, p->C44p)) return PF_ERR_ARG;
    if (p->precision != PF_FP64 || p->mean_strain_mode != 0) return PF_ERR_ARG;
    if (!(p->el_tol >= 0.0) || p->el_max_iter < 0) return PF_ERR_ARG;
  }
  if (!pf_size_supported(p->nx) || !pf_size_supported(p->ny) || !pf_size_supported(p->nz))
    return PF_ERR_UNSUPPORTED_SIZE;

  int ndev = 0;  // no usable device: a HIP error, before any allocation
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return PF_ERR_HIP;
  pf_ctx* c = new (std::nothrow) pf_ctx();
  if (!c) return PF_ERR_OOM;
  ctx_setup(c, p, (hipStream_t)stream);
  const Geo& g = c->g;

  const size_t kbytes64 = sizeof(cx<double>) * 4 * (size_t)g.fs;
  const size_t fe_bytes = (c->mixed ? sizeof(cx<float>) : sizeof(cx<double>)) * 4 * (size_t)g.fs;
  const size_t tbytes = (c->mixed ? sizeof(cx<float>) : sizeof(cx<double>)) * 7 * (size_t)g.fs;
  const size_t rbytes = sizeof(double) * 4 * (size_t)g.nx * g.ny * g.nz;
  // a real-space norm holds the error and the previous state (8 real fields)
  c->scratch_bytes = std::max(tbytes, (c->norm_real ? 2 : 1) * rbytes);
  pf_status s = PF_OK;
  s = dalloc(c, (void**)&c->y, kbytes64);
  if (s == PF_OK) s = dalloc(c, (void**)&c->ynew, kbytes64);
  if (s == PF_OK && c->norm_real) s = dalloc(c, (void**)&c->ycopy, kbytes64);
  if (s == PF_OK && c->inhom) s = dalloc(c, (void**)&c->E6, sizeof(cx<double>) * 6 * (size_t)g.fs);
  if (s == PF_OK && c->inhom) s = dalloc(c, (void**)&c->R6, sizeof(double) * 6 * (size_t)g.nx * g.ny * g.nz);
  if (s == PF_OK && c->inhom) s = dalloc(c, (void**)&c->LC6, sizeof(double) * 6 * (size_t)g.nx * g.ny * g.nz);
  if (s == PF_OK && c->inhom) s = dalloc(c, (void**)&c->elmax, sizeof(double));
  if (s == PF_OK && c->inhom) s = dalloc(c, (void**)&c->el_part, sizeof(double) * (size_t)el_row_blocks(c));
  for (int i = 0; i < c->tab.s && s == PF_OK; ++i) {
    if (c->fi_need[i] || i == 0) s = dalloc(c, (void**)&c->FI[i], kbytes64);
    if (s == PF_OK && (c->fe_need[i] || i == 0)) s = dalloc(c, &c->FE[i], fe_bytes);
  }
  if (s == PF_OK) s = dalloc(c, &c->scratch, c->scratch_bytes);
  if (s == PF_OK) s = dalloc(c, (void**)&c->partial, sizeof(double) * 4 * c->nblk_red);
  if (s == PF_OK) s = dalloc(c, (void**)&c->red, sizeof(double) * 8);
  if (s == PF_OK && hipHostMalloc((void**)&c->host_red, sizeof(double) * 8, 0) != hipSuccess) s = PF_ERR_OOM;
  if (s == PF_OK) s = upload_twiddles(c, 0, g.nz);
  if (s == PF_OK) s = upload_twiddles(c, 1, g.ny);
  if (s == PF_OK) s = upload_twiddles(c, 2, g.nx / 2);
  if (s == PF_OK) s = upload_twiddles(c, 3, g.nx);
  if (s == PF_OK && (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess))
    s = PF_ERR_HIP;
  if (s == PF_OK && hipMemsetAsync(c->y, 0, kbytes64, c->stream) != hipSuccess) s = PF_ERR_HIP;
  if (s == PF_OK && hipStreamSynchronize(c->stream) != hipSuccess) s = PF_ERR_HIP;
  if (s != PF_OK) {
    pf_finalize(c);
    return s;
  }
  *out = c;
  return PF_OK;
}

int64_t pf_kspace_pitch(const pf_ctx* c) { return c ? c->g.P : 0; }
int64_t pf_workspace_bytes(const pf_ctx* c) { return c ? c->ws_bytes : 0; }
double pf_get_time(const pf_ctx* c) { return c ? c->t : 0.0; }

pf_status pf_set_dt(pf_ctx* c, double dt) {
  if (!c || !(dt > 0.0)) return PF_ERR_ARG;
  c->dt_next = dt;
  return PF_OK;
}

static double field_bytes64(const pf_ctx* c) {
  return (double)c->g.nz * c->g.ny * c->g.nxh * sizeof(cx<double>);
}
static double real_bytes64(const pf_ctx* c) { return (double)c->g.nz * c->g.ny * c->g.nx * sizeof(double); }

static pf_status forward3d_fp64(pf_ctx* c, const double* re, cx<double>* out, int nf) {
  const double fk = field_bytes64(c), fr = real_bytes64(c);
  prof_begin(c);
  if (!launch_xpass_r2c(c, re, out, nf)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_XR2C, nf * (fk + fr));
  prof_begin(c);
  if (!launch_colfft<double, -1, 1>(c, out, out, nf, 1.0)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_YFFT, 2 * nf * fk);
  prof_begin(c);
  if (!launch_colfft<double, -1, 2>(c, out, out, nf, 1.0)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_ZFFT, 2 * nf * fk);
  if (hipGetLastError() != hipSuccess) return PF_ERR_HIP;
  return PF_OK;
}

// inverse with 1/N^3 scaling; `in` is used as the intermediate (overwritten)
static pf_status inverse3d_fp64(pf_ctx* c, cx<double>* in, double* re, int nf) {
  const double s = c->mk.inv_n3;
  const double fk = field_bytes64(c), fr = real_bytes64(c);
  prof_begin(c);
  if (!launch_colfft<double, +1, 2>(c, in, in, nf, s)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_ZFFT, 2 * nf * fk);
  prof_begin(c);
  if (!launch_colfft<double, +1, 1>(c, in, in, nf, 1.0)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_YFFT, 2 * nf * fk);
  prof_begin(c);
  if (!launch_xpass_c2r(c, in, re, nf, 1.0)) return PF_ERR_UNSUPPORTED_SIZE;
  prof_end(c, KC_XC2R, nf * (fk + fr));
  if (hipGetLastError() != hipSuccess) return PF_ERR_HIP;
  return PF_OK;
}

pf_status pf_set_state(pf_ctx* c, const double* cfield, const double* eta, int32_t on_device, double t0) {
  if (!c || !cfield || !eta) return PF_ERR_ARG;
  const size_t n = (size_t)c->g.nx * c->g.ny * c->g.nz;
  double* stage = (double*)c->scratch;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  PF_HIP(hipMemcpyAsync(stage, cfield, n * sizeof(double), kind, c->stream));
  PF_HIP(hipMemcpyAsync(stage + n, eta, 3 * n * sizeof(double), kind, c->stream));
  pf_status s = forward3d_fp64(c, stage, c->y, 4);
  if (s != PF_OK) return s;
  PF_HIP(hipStreamSynchronize(c->stream));
  c->t = t0;
  c->have_state = true;
  c->prev_rejected = false;
  return PF_OK;
}

pf_status pf_get_state(pf_ctx* c, double* cfield, double* eta, int32_t on_device) {
  if (!c || !cfield || !eta) return PF_ERR_ARG;
  const size_t n = (size_t)c->g.nx * c->g.ny * c->g.nz;
  PF_HIP(hipMemcpyAsync(c->ynew, c->y, sizeof(cx<double>) * 4 * c->g.fs, hipMemcpyDeviceToDevice, c->stream));
  double* stage = (double*)c->scratch;
  pf_status s = inverse3d_fp64(c, c->ynew, stage, 4);
  if (s != PF_OK) return s;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  PF_HIP(hipMemcpyAsync(cfield, stage, n * sizeof(double), kind, c->stream));
  PF_HIP(hipMemcpyAsync(eta, stage + n, 3 * n * sizeof(double), kind, c->stream));
  PF_HIP(hipStreamSynchronize(c->stream));
  return PF_OK;
}

pf_status pf_get_state_hat(pf_ctx* c, void* y_hat) {
  if (!c || !y_hat) return PF_ERR_ARG;
  PF_HIP(hipMemcpyAsync(y_hat, c->y, sizeof(cx<double>) * 4 * c->g.fs, hipMemcpyDeviceToDevice, c->stream));
  PF_HIP(hipStreamSynchronize(c->stream));
  return PF_OK;
}

pf_status pf_set_state_hat(pf_ctx* c, const void* y_hat, double t0) {
  if (!c || !y_hat) return PF_ERR_ARG;
  PF_HIP(hipMemcpyAsync(c->y, y_hat, sizeof(cx<double>) * 4 * c->g.fs, hipMemcpyDeviceToDevice, c->stream));
  PF_HIP(hipStreamSynchronize(c->stream));
  c->t = t0;
  c->have_state = true;
  c->prev_rejected = false;
  return PF_OK;
}

pf_status pf_rhs(pf_ctx* c, double t, const void* y_hat, void* fI_hat, void* fE_hat) {
  (void)t;
  if (!c || !y_hat || !fI_hat || !fE_hat) return PF_ERR_ARG;
  pf_status s;
  if (!c->mixed) {
    StageArgs<double> sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.y = (const cx<double>*)y_hat;
    sa.FI_out = (cx<double>*)fI_hat;
    sa.FEc_out = c->mk.fEa != 0.0 ? (cx<double>*)fE_hat : nullptr;
    s = run_stage<double, double>(c, sa, true, (cx<double>*)fE_hat);
  } else {
    StageArgs<float> sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.y = (const cx<double>*)y_hat;
    sa.FI_out = (cx<double>*)fI_hat;
    cx<float>* fe = (cx<float>*)c->FE[0];
    sa.FEc_out = c->mk.fEa != 0.0 ? fe : nullptr;
    s = run_stage<float, float>(c, sa, true, fe);
    if (s == PF_OK) {
      k_convert<float, double><<<dim3(1024), dim3(256), 0, c->stream>>>(fe, (cx<double>*)fE_hat, c->g, 4);
      if (hipGetLastError() != hipSuccess) s = PF_ERR_HIP;
    }
  }
  if (s != PF_OK) return s;
  PF_HIP(hipStreamSynchronize(c->stream));
  prof_resolve(c);
  return PF_OK;
}

// Real-space WRMS of the step's error estimate (norm_space = 1): the error
// (stored by the finalize in FI[0]) and the previous state are transformed
// back to real space and weighted point by point; the sum of squares goes to
// red[2].
static pf_status wrms_real_space(pf_ctx* c) {
  const long long n = (long long)c->g.nx * c->g.ny * c->g.nz;
  double* re = (double*)c->scratch;
  double* ry = re + 4 * n;
  pf_status s = inverse3d_fp64(c, c->FI[0], re, 4);
  if (s != PF_OK) return s;
  PF_HIP(hipMemcpyAsync(c->ycopy, c->y, sizeof(cx<double>) * 4 * c->g.fs, hipMemcpyDeviceToDevice, c->stream));
  s = inverse3d_fp64(c, c->ycopy, ry, 4);
  if (s != PF_OK) return s;
  k_wrms_real<<<dim3(c->nblk_red), dim3(256), 0, c->stream>>>(re, ry, 4 * n, c->p.rtol, c->p.atol, c->partial);
  k_reduce_tuples<<<dim3(1), dim3(256), 0, c->stream>>>(c->partial, c->nblk_red, 1, c->red + 2);
  PF_HIP(hipGetLastError());
  return PF_OK;
}

pf_status pf_ark_step(pf_ctx* c, double dt, double* dt_next, double* err_out, int32_t* accepted) {
  if (!c || !(dt > 0.0) || !std::isfinite(dt)) return PF_ERR_ARG;
  if (!c->have_state) return PF_ERR_STATE;
  int n_rhs = 0;
  pf_status s = c->mixed ? stages_and_finalize<float, float>(c, dt, &n_rhs)
                         : stages_and_finalize<double, double>(c, dt, &n_rhs);
  if (s != PF_OK) return s;
  const bool real_norm = c->norm_real && c->tab.has_emb;
  if (real_norm) {
    s = wrms_real_space(c);
    if (s != PF_OK) return s;
  }
  PF_HIP(hipMemcpyAsync(c->host_red, c->red, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  PF_HIP(hipStreamSynchronize(c->stream));
  prof_resolve(c);
  const double n3 = (double)c->g.nx * c->g.ny * c->g.nz;
  double err = c->tab.has_emb ? std::sqrt(c->host_red[real_norm ? 2 : 0] / (4.0 * n3)) : 0.0;
  const bool finite = c->host_red[1] == 0.0 && std::isfinite(err);
  if (!finite) err = INFINITY;
  bool ok;
  double nxt;
  if (c->p.adaptive) {
    ok = finite && err <= 1.0;
    nxt = std::max(controller(dt, err, c->tab.emb_order, ok && c->prev_rejected), c->p.dt_min);
    c->prev_rejected = !ok;
  } else {
    ok = finite;
    nxt = c->p.dt0;
  }
  c->st.attempts += 1;
  c->st.n_rhs += n_rhs;
  c->st.err_last = err;
  if (ok) {
    std::swap(c->y, c->ynew);
    c->t += dt;
    c->st.steps += 1;
    c->st.dt_last = dt;
    c->st.dt_min_seen = std::min(c->st.dt_min_seen, dt);
    c->st.dt_max_seen = std::max(c->st.dt_max_seen, dt);
  } else {
    c->st.rejects += 1;
  }
  c->dt_next = nxt;
  c->st.dt_next = nxt;
  c->st.t = c->t;
  if (dt_next) *dt_next = nxt;
  if (err_out) *err_out = err;
  if (accepted) *accepted = ok ? 1 : 0;
  if (!finite && !c->p.adaptive) return PF_ERR_NONFINITE;
  return PF_OK;
}

pf_status pf_get_stats(pf_ctx* c, pf_stats* out) {
  if (!c || !out) return PF_ERR_ARG;
  c->st.t = c->t;
  if (c->have_state) {
    double d[4];
    pf_status s = ctx_diagnostics(c, true, d);
    if (s != PF_OK) return s;
    c->st.mass = d[0];
    c->st.vf = d[1];
    c->st.vf_threshold = d[2];
    c->st.F = d[3];
  } else {
    c->st.mass = c->st.vf = c->st.vf_threshold = c->st.F = NAN;
  }
  *out = c->st;
  return PF_OK;
}

pf_status pf_advance(pf_ctx* c, double t_final, pf_stats* out) {
  if (!c) return PF_ERR_ARG;
  if (!c->have_state) return PF_ERR_STATE;
  PF_HIP(hipEventRecord(c->ev0, c->stream));
  int rejects = 0;
  pf_status s = PF_OK;
  while (c->t < t_final * (1.0 - 1e-15)) {
    double dt = c->p.adaptive ? std::min(c->dt_next, c->p.dt_max) : std::min(c->p.dt0, c->p.dt_max);
    dt = std::min(dt, t_final - c->t);
    int32_t acc = 0;
    s = pf_ark_step(c, dt, nullptr, nullptr, &acc);
    if (s != PF_OK) break;
    if (acc) {
      rejects = 0;
    } else if (++rejects >= c->p.max_rejects) {
      s = PF_ERR_STEP_FAIL;
      break;
    }
  }
  PF_HIP(hipEventRecord(c->ev1, c->stream));
  PF_HIP(hipEventSynchronize(c->ev1));
  float ms = 0.f;
  hipEventElapsedTime(&ms, c->ev0, c->ev1);
  c->st.elapsed_ms += ms;
  if (out) {
    pf_status s2 = pf_get_stats(c, out);
    if (s == PF_OK) s = s2;
  }
  return s;
}

}  // extern "C"

// Diagnostics of the current state, all in FP64 on the device (the state is
// FP64 in both precisions): the real-space state from one inverse transform
// (into the scratch buffer, with the spare state buffer as the transform's
// intermediate); per-point sums of H, of the threshold count and of the bulk
// free-energy density; with want_F also the forward transform of
// theta_v = h(eta_v) and the reciprocal-space gradient and elastic energies.
// out: mass, vf, vf_threshold, F (F only with want_F).
namespace pf {
pf_status ctx_diagnostics(pf_ctx* c, bool want_F, double out[4]) {
  if (!c->have_state) return PF_ERR_STATE;
  const Geo& g = c->g;
  const long long n = (long long)g.nx * g.ny * g.nz;
  double el_sum = 0.0;
  if (want_F && c->inhom) {
    // elastic energy sum_r sigma : (eps_bar + eps_u - eps*) / 2 at the
    // equilibrium strain of the current state (FP64 contexts only)
    cx<double>* T1 = (cx<double>*)c->scratch;
    if (!launch_colfft<double, +1, 2>(c, c->y, T1, 4, c->mk.inv_n3) ||
        !launch_colfft<double, +1, 1>(c, T1, T1, 4, 1.0))
      return PF_ERR_UNSUPPORTED_SIZE;
    pf_status se = el_solve(c, T1, nullptr, 0);
    if (se != PF_OK) return se;
    if (!launch_el_rows<3>(c, T1, nullptr, nullptr)) return PF_ERR_UNSUPPORTED_SIZE;
    k_reduce_tuples<<<dim3(1), dim3(256), 0, c->stream>>>(c->el_part, el_row_blocks(c), 1, c->red + 6);
    PF_HIP(hipGetLastError());
    PF_HIP(hipMemcpyAsync(&c->host_red[6], c->red + 6, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PF_HIP(hipStreamSynchronize(c->stream));
    el_sum = c->host_red[6];
  }
  PF_HIP(hipMemcpyAsync(c->ynew, c->y, sizeof(cx<double>) * 4 * g.fs, hipMemcpyDeviceToDevice, c->stream));
  double* stage = (double*)c->scratch;
  pf_status s = inverse3d_fp64(c, c->ynew, stage, 4);
  if (s != PF_OK) return s;
  k_diag_real<<<dim3(c->nblk_red), dim3(256), 0, c->stream>>>(stage, n, c->mk, want_F ? 1 : 0, c->partial);
  k_reduce_tuples<<<dim3(1), dim3(256), 0, c->stream>>>(c->partial, c->nblk_red, 3, c->red);
  PF_HIP(hipGetLastError());
  cx<double> th0[3];
  if (want_F) {
    // theta~ into the spare state buffer (free again after the inverse transform)
    s = forward3d_fp64(c, stage + n, c->ynew, 3);
    if (s != PF_OK) return s;
    k_energy_kspace<<<dim3(c->nblk_red), dim3(256), 0, c->stream>>>(c->y, c->ynew, g, c->mk, c->partial);
    k_reduce_tuples<<<dim3(1), dim3(256), 0, c->stream>>>(c->partial, c->nblk_red, 2, c->red + 4);
    PF_HIP(hipGetLastError());
    for (int v = 0; v < 3; ++v)
      PF_HIP(hipMemcpyAsync(&th0[v], c->ynew + v * g.fs, sizeof(cx<double>), hipMemcpyDeviceToHost, c->stream));
  }
  PF_HIP(hipMemcpyAsync(c->host_red, c->red, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  cx<double> c0;
  PF_HIP(hipMemcpyAsync(&c0, c->y, sizeof(c0), hipMemcpyDeviceToHost, c->stream));
  PF_HIP(hipStreamSynchronize(c->stream));
  prof_resolve(c);
  const double* r = c->host_red;
  out[0] = c0.re / (double)n;
  out[1] = r[0] / (double)n;
  out[2] = r[1] / (double)n;
  out[3] = NAN;
  if (want_F) {
    // Eq. 1 on the grid: bulk sum + gradient and elastic energies (Parseval,
    // 1/(2 N^3)) + the prescribed mean strain's terms, times dx^3
    const pf_params& p = c->p;
    double F = r[2] + 0.5 * (r[4] + (c->inhom ? 0.0 : r[5])) / (double)n;
    if (c->inhom) {
      F += el_sum;  // includes the mean strain
    } else if (p.mean_strain_mode == 0) {
      const double* eb = p.eps_bar;
      double ebCeb = 0.0;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) ebCeb += eb[i] * eb[j] * (i == j ? p.C11 : p.C12);
      F += 0.5 * (double)n * ebCeb;
      // hom[v] = -N^3 eps*_v : C : eps_bar
      for (int v = 0; v < 3; ++v) F += c->mk.hom[v] / (double)n * th0[v].re;
    }
    out[3] = F * p.dx * p.dx * p.dx;
  }
  return PF_OK;
}
}  // namespace pf

extern "C" {

pf_status pf_diagnostics(pf_ctx* c, double* mass, double* vf, double* vf_thr) {
  if (!c) return PF_ERR_ARG;
  double out[4];
  pf_status s = ctx_diagnostics(c, false, out);
  if (s != PF_OK) return s;
  if (mass) *mass = out[0];
  if (vf) *vf = out[1];
  if (vf_thr) *vf_thr = out[2];
  return PF_OK;
}

pf_status pf_free_energy(pf_ctx* c, double* F) {
  if (!c || !F) return PF_ERR_ARG;
  double out[4];
  pf_status s = ctx_diagnostics(c, true, out);
  if (s != PF_OK) return s;
  *F = out[3];
  return PF_OK;
}

pf_status pf_fft3d(pf_ctx* c, int32_t dir, int32_t nf, void* in, void* out) {
  if (!c || !in || !out || nf < 1 || nf > 4 || (dir != -1 && dir != 1)) return PF_ERR_ARG;
  pf_status s = dir < 0 ? forward3d_fp64(c, (const double*)in, (cx<double>*)out, nf)
                        : inverse3d_fp64(c, (cx<double>*)in, (double*)out, nf);
  if (s != PF_OK) return s;
  PF_HIP(hipStreamSynchronize(c->stream));
  prof_resolve(c);
  return PF_OK;
}

pf_status pf_profile_enable(pf_ctx* c, int32_t on) {
  if (!c) return PF_ERR_ARG;
  PF_HIP(hipStreamSynchronize(c->stream));
  c->prof_pending.clear();
  c->prof_used = 0;
  for (int k = 0; k < 16; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_bytes[k] = 0.0;
    c->prof_n[k] = 0;
  }
  c->prof_on = on != 0;
  return PF_OK;
}

int32_t pf_profile_classes(void) { return KC_COUNT; }

const char* pf_profile_name(int32_t cls) {
  if (cls < 0 || cls >= KC_COUNT) return "";
  return kc_names[cls];
}

pf_status pf_profile_get(pf_ctx* c, int32_t cls, double* total_ms, int64_t* launches, double* bytes) {
  if (!c || cls < 0 || cls >= KC_COUNT) return PF_ERR_ARG;
  if (total_ms) *total_ms = c->prof_ms[cls];
  if (launches) *launches = c->prof_n[cls];
  if (bytes) *bytes = c->prof_bytes[cls];
  return PF_OK;
}

}  // extern "C"

// ---- autotuner: time each tile variant of each column kernel on this context
template <typename T, typename TE>
static pf_status autotune_impl(pf_ctx* c, int reps) {
  cx<T>* T1 = (cx<T>*)c->scratch;
  cx<T>* T3 = T1 + 4 * c->g.fs;
  int npairs = 0;
  while (npairs < 3 && c->FI[npairs] && c->FE[npairs]) ++npairs;
  StageArgs<TE> sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.y = c->y;
  for (int j = 0; j < npairs; ++j) {
    sa.FE[j] = (const cx<TE>*)c->FE[j];
    sa.FI[j] = c->FI[j];
    sa.cE[j] = 1e-3;
    sa.cI[j] = 1e-3;
  }
  sa.nprev = npairs;
  sa.gdt = 1e-3;
  sa.FI_out = c->FI[0];
  hipEvent_t e0, e1;
  PF_HIP(hipEventCreate(&e0));
  PF_HIP(hipEventCreate(&e1));
  for (int k = 0; k < CK_COUNT; ++k) {
    double best = 1e300;
    int best_v = 0;
    const int nvar = (k == CK_FFT && ws_supported(c->g.ny, sizeof(cx<T>)) && ws_supported(c->g.nz, sizeof(cx<T>)))
                         ? 3 : 2;
    for (int v = 0; v < nvar; ++v) {
      c->var[k] = v;
      auto run = [&]() {
        switch (k) {
          case CK_FFT: launch_colfft<T, -1, 1>(c, T1, T1, 4, (T)1); break;
          case CK_STAGE: launch_stage_invz<T, TE>(c, sa, T1, 1); break;
          case CK_ELASTIC: launch_zpass_elastic<T, TE>(c, T3, (cx<TE>*)c->FE[0], 0); break;
          default: launch_zpass_fwd_ac<T, TE>(c, T3, (cx<TE>*)c->FE[0]); break;
        }
      };
      run();
      PF_HIP(hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps; ++r) run();
      PF_HIP(hipEventRecord(e1, c->stream));
      PF_HIP(hipEventSynchronize(e1));
      PF_HIP(hipGetLastError());
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      c->tune_ms[k][v] = ms / reps;
      if (ms < best) {
        best = ms;
        best_v = v;
      }
    }
    c->var[k] = best_v;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return PF_OK;
}

extern "C" {

pf_status pf_autotune(pf_ctx* c, int32_t reps) {
  if (!c || reps < 1) return PF_ERR_ARG;
  return c->mixed ? autotune_impl<float, float>(c, reps) : autotune_impl<double, double>(c, reps);
}

int32_t pf_tuning_kinds(void) { return CK_COUNT; }

pf_status pf_tuning_get(pf_ctx* c, int32_t kind, int32_t* variant, int32_t* tile_cols, int32_t* end_radix,
                        double* ms_v0, double* ms_v1) {
  if (!c || kind < 0 || kind >= CK_COUNT) return PF_ERR_ARG;
  const int v = c->var[kind];
  const int eb = c->mixed ? (int)sizeof(cx<float>) : (int)sizeof(cx<double>);
  if (variant) *variant = v;
  if (tile_cols) *tile_cols = col_tx(c->g.nz, kind, eb, v ? 1 : 0);
  if (end_radix) *end_radix = plan(c->g.nz, col_re(kind, eb)).r[0];
  if (ms_v0) *ms_v0 = c->tune_ms[kind][0];
  if (ms_v1) *ms_v1 = c->tune_ms[kind][1];
  return PF_OK;
}

pf_status pf_tuning_set(pf_ctx* c, int32_t kind, int32_t variant) {
  if (!c || kind < 0 || kind >= CK_COUNT || variant < 0 || variant > 2) return PF_ERR_ARG;
  if (variant == 2 && !(kind == CK_FFT && ws_supported(c->g.ny, c->mixed ? 8 : 16) &&
                        ws_supported(c->g.nz, c->mixed ? 8 : 16)))
    return PF_ERR_ARG;
  c->var[kind] = variant;
  return PF_OK;
}

pf_status pf_tuning_ms(pf_ctx* c, int32_t kind, int32_t variant, double* ms) {
  if (!c || kind < 0 || kind >= CK_COUNT || variant < 0 || variant > 2 || !ms) return PF_ERR_ARG;
  *ms = c->tune_ms[kind][variant];
  return PF_OK;
}

const char* pf_tuning_name(int32_t kind) {
  if (kind < 0 || kind >= CK_COUNT) return "";
  return ck_names[kind];
}

}  // extern "C"
