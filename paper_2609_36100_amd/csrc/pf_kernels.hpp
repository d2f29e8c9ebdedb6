// HIP kernels of one ImEx-ARK stage for the pseudospectral phase-field model.
//
// A stage (Methods, "Time integration", Eq. ARK_stage, with the right-hand
// side of Eqs. composition / order) is nine HBM-streaming passes over the
// half spectrum [field][z][y][kx] (row pitch P complex values):
//
//  stage_invz    combine previous stage derivatives, implicit solve per mode,
//                F^I = L z, inverse z-FFT of the 4 state fields      (z pass)
//  ypass<+1>     inverse y-FFT of the 4 state fields                   (y pass)
//  xpass_theta   c2r of eta_v, theta_v = h(eta_v), r2c of theta_v      (x pass)
//  ypass<-1>     forward y-FFT of theta                                (y pass)
//  zpass_elastic forward z-FFT, per-mode elastic solve e~ = B(n) theta~,
//                explicit CH term, inverse z-FFT of e~                 (z pass)
//  ypass<+1>     inverse y-FFT of e~                                   (y pass)
//  xpass_drive   c2r of c, eta_v, e_v, driving force, r2c              (x pass)
//  ypass<-1>     forward y-FFT of the driving force                    (y pass)
//  zpass_fwd_ac  forward z-FFT, F^E_eta = -L g~                        (z pass)
//
// followed once per step by `finalize` (update, embedded error, WRMS partial
// sums).  z and y passes give each work-group TX consecutive kx columns of one
// plane so every global access is TX contiguous complex values; x passes give
// each work-group RB whole rows.  Line FFTs run in LDS with Stockham passes;
// inputs and outputs of a line stay in registers so the pointwise and
// per-mode work happens between the transforms without extra HBM traffic.
#pragma once

#include "pf_fft.hpp"

namespace pf {

// ---- geometry and model constants -----------------------------------------
struct Geo {
  int nx, ny, nz, nxh, P;
  long long fs;          // complex elements per field = nz * ny * P
  double kfx, kfy, kfz;  // 2 pi / (N_i dx)
};

struct ModelK {
  double M, L, kc, ke, ac;  // mobilities, gradient coefficients, implicit bulk
  double W, w, cm, cp;
  double fEc;               // 2 W M (c_p - c_m): explicit CH coefficient (split B)
  double fEa;               // (2W - a_c) M: extra explicit CH coefficient (split A)
  double E[3][3];           // eps*_v : C : eps*_w
  double B0[3][3];          // k = 0 kernel (E or 0)
  double S[3][3];           // diagonal of sigma*_v = C : eps*_v, [v][axis]
  double C11, C12, C44;
  double hom[3];            // N^3 * (-eps*_v : C : eps_bar), added to e~_v(0)
  double inv_n3;            // 1 / (nx ny nz)
  // inhomogeneous elasticity (Reuss average between matrix and precipitate)
  double Sm[3], dS[3];      // matrix compliance (S11, S12, S44; engineering shears), S_p - S_m
  double C0[3];             // reference stiffness (C_m + C_p) / 2
  double C0eps[3][3];       // (C0 eps*_v)_ii, [v][i]
  double eps[3][3];         // eigenstrain diagonals eps*_v, [v][i]
  double ebar[3];           // prescribed mean strain (diagonal)
};

__host__ __device__ inline int mode_of(int i, int n) { return (2 * i < n) ? i : i - n; }

// Implicit symbol L_f(k^2) for field f (0 = c, 1..3 = eta).
__device__ inline double lsym(const ModelK& m, int f, double k2) {
  return f == 0 ? -m.M * k2 * (m.ac + m.kc * k2) : -m.L * m.ke * k2;
}

// Khachaturyan kernel contraction e_v = sum_w B_vw(k) th_w for k != 0, with
// B_vw = E_vw - (S_v k) . Omega(k) . (S_w k),  Omega(k)^-1 = C_ijkl k_j k_l
// (S_v k componentwise).  Evaluated without forming B: q = sum_w (S_w k) th_w,
// p = Omega q (adjugate over determinant, Omega symmetric), then
// e_v = sum_w E_vw th_w - (S_v k) . p.  Uses k directly (Omega scales as
// 1/|k|^2, S k as |k|): no normalisation.
template <typename R>
__device__ inline void elastic_apply(const ModelK& m, R kx, R ky, R kz, const cx<R>* th, cx<R>* e) {
  const R C11 = (R)m.C11, C12 = (R)m.C12, C44 = (R)m.C44;
  const R a = C11 - C12 - (R)2 * C44;
  const R b = C12 + C44;
  const R k2 = kx * kx + ky * ky + kz * kz;
  // Omega^-1 (symmetric): C44 k^2 d_ik + b k_i k_k + a k_i^2 d_ik
  const R g00 = C44 * k2 + (b + a) * kx * kx;
  const R g11 = C44 * k2 + (b + a) * ky * ky;
  const R g22 = C44 * k2 + (b + a) * kz * kz;
  const R g01 = b * kx * ky, g02 = b * kx * kz, g12 = b * ky * kz;
  // adjugate
  const R A00 = g11 * g22 - g12 * g12;
  const R A11 = g00 * g22 - g02 * g02;
  const R A22 = g00 * g11 - g01 * g01;
  const R A01 = g02 * g12 - g01 * g22;
  const R A02 = g01 * g12 - g02 * g11;
  const R A12 = g01 * g02 - g00 * g12;
  const R idet = (R)1 / (g00 * A00 + g01 * A01 + g02 * A02);
  cx<R> q0 = mk<R>(0, 0), q1 = mk<R>(0, 0), q2 = mk<R>(0, 0);
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    q0 = q0 + ((R)m.S[w][0] * kx) * th[w];
    q1 = q1 + ((R)m.S[w][1] * ky) * th[w];
    q2 = q2 + ((R)m.S[w][2] * kz) * th[w];
  }
  const cx<R> p0 = idet * (A00 * q0 + A01 * q1 + A02 * q2);
  const cx<R> p1 = idet * (A01 * q0 + A11 * q1 + A12 * q2);
  const cx<R> p2 = idet * (A02 * q0 + A12 * q1 + A22 * q2);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    cx<R> acc = mk<R>(0, 0);
#pragma unroll
    for (int w = 0; w < 3; ++w) acc = acc + (R)m.E[v][w] * th[w];
    e[v] = acc - (((R)m.S[v][0] * kx) * p0 + ((R)m.S[v][1] * ky) * p1 + ((R)m.S[v][2] * kz) * p2);
  }
}

// Multiply a[t] by w^{S t j} (t = 1..R-1) where w^{-m} = tw[m]; only the
// powers 1, 2 (and 4) come from the table, the others are products of two
// table values (a few ulp).
template <int R, int S, typename T>
__device__ inline void apply_twiddles(cx<T>* a, const cx<T>* tw, int j) {
  if constexpr (R == 2) {
    a[1] = cmul(a[1], twiddle<S>(tw, j));
  } else {
    const cx<T> w1 = twiddle<S>(tw, j), w2 = twiddle<S>(tw, 2 * j);
    a[1] = cmul(a[1], w1);
    a[2] = cmul(a[2], w2);
    if constexpr (R >= 4) {
      const cx<T> w3 = cmul(w1, w2);
      a[3] = cmul(a[3], w3);
      if constexpr (R == 5) {
        a[4] = cmul(a[4], cmul(w2, w2));
      } else if constexpr (R == 6) {
        const cx<T> w4 = twiddle<S>(tw, 4 * j);
        a[4] = cmul(a[4], w4);
        a[5] = cmul(a[5], cmul(w4, w1));
      } else if constexpr (R == 7) {
        const cx<T> w4 = twiddle<S>(tw, 4 * j);
        a[4] = cmul(a[4], w4);
        a[5] = cmul(a[5], cmul(w4, w1));
        a[6] = cmul(a[6], cmul(w4, w2));
      } else if constexpr (R == 8) {
        const cx<T> w4 = twiddle<S>(tw, 4 * j);
        a[4] = cmul(a[4], w4);
        a[5] = cmul(a[5], cmul(w4, w1));
        a[6] = cmul(a[6], cmul(w4, w2));
        a[7] = cmul(a[7], cmul(w4, w3));
      }
    }
  }
}

// ---- line FFT in LDS -------------------------------------------------------
__host__ __device__ constexpr int plan_prod(int n, int q, int re) {
  Plan P = plan(n, re);
  int p = 1;
  for (int i = 0; i < q; ++i) p *= P.r[i];
  return p;
}

// Work-group barrier for LDS exchanges only: waits for this wavefront's LDS
// accesses, not for its outstanding global memory operations (a plain
// __syncthreads also drains in-flight global loads and stores, including
// loads that land in LDS).  The memory clobber keeps the compiler from moving
// memory accesses across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
template <bool LB>
__device__ inline void xbar() {
  if constexpr (LB)
    lds_barrier();
  else
    __syncthreads();
}

template <typename T, int N, int S, int Q, int RE, bool LB = false>
struct MidPass {
  template <class Buf>
  __device__ static inline void run(int tid, const cx<T>* tw, Buf buf, bool act) {
    constexpr Plan PL = plan(N, RE);
    if constexpr (Q < PL.np - 1) {
      constexpr int r = PL.r[Q];
      constexpr int p = plan_prod(N, Q, RE);
      constexpr int TL = N / PL.r[0];
      constexpr int NB = N / r;
      constexpr int PER = (NB + TL - 1) / TL;
      cx<T> v[PER][r];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int b = tid + j * TL;
        if (act && (PER * TL == NB || b < NB)) {
          const int k = b % p;
#pragma unroll
          for (int t = 0; t < r; ++t) v[j][t] = buf(b + t * NB);
          constexpr int step = N / (p * r);
          apply_twiddles<r, S>(v[j], tw, k * step);
          dft<r, S>(v[j]);
        }
      }
      xbar<LB>();
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int b = tid + j * TL;
        if (act && (PER * TL == NB || b < NB)) {
          const int k = b % p;
#pragma unroll
          for (int t = 0; t < r; ++t) buf((b - k) * r + k + t * p) = v[j][t];
        }
      }
      xbar<LB>();
      MidPass<T, N, S, Q + 1, RE, LB>::run(tid, tw, buf, act);
    }
  }
};

// In-place FFT of one line of length N by TL = N / r0 cooperating threads
// (r0 = the plan's end radix, at most RE).  On entry a[t] holds
// x[tid + t N/r0]; on exit X[tid + t N/r0].  Every thread of the work-group
// must call this the same number of times (it contains work-group barriers);
// the LDS region behind `buf` must hold N values.  Threads with act = false
// only take part in the barriers (work-groups shared by lines of different
// lengths have idle threads).
template <typename T, int N, int S, int RE = 8, bool LB = false, class Buf>
__device__ inline void line_fft(cx<T>* a, int tid, const cx<T>* tw, Buf buf, bool act = true) {
  constexpr Plan PL = plan(N, RE);
  static_assert(PL.ok, "unsupported line length");
  constexpr int R0 = PL.r[0];
  constexpr int TL = N / R0;
  dft<R0, S>(a);
  if constexpr (PL.np > 1) {
    xbar<LB>();
    if (act) {
#pragma unroll
      for (int t = 0; t < R0; ++t) buf(tid * R0 + t) = a[t];
    }
    xbar<LB>();
    MidPass<T, N, S, 1, RE, LB>::run(tid, tw, buf, act);
    if (act) {
#pragma unroll
      for (int t = 0; t < R0; ++t) a[t] = buf(tid + t * TL);
    }
    // last pass: p = N / R0, k = tid, twiddle w_N^{t tid}
    apply_twiddles<R0, S>(a, tw, tid);
    dft<R0, S>(a);
  }
}

// Work-groups are handed to the 8 XCDs round-robin.  Renumber them so each
// XCD processes a contiguous run of logical tiles: neighbouring column
// bundles (which share cache lines) then meet in the same L2.
__device__ inline int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, slot = b >> 3;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

template <typename T>
__device__ inline cx<T> ld(const cx<T>* p) { return *p; }

// Marks a value as computed at this point: the compiler may not move its
// arithmetic below here (an empty asm that reads and rewrites the registers).
template <typename T>
__device__ inline void pin(cx<T>& z) { asm volatile("" : "+v"(z.re), "+v"(z.im)); }

// Element i of an array at f, addressed as a uniform base plus a 32-bit byte
// offset: one field of the largest supported grid (512^3, row pitch 264) is
// 1.1 GB, so in-field offsets fit, and the compiler then keeps one VGPR per
// offset (shared by every field read at that position) instead of a 64-bit
// address per access.
template <typename E>
__device__ inline E& at32(E* f, uint32_t i) {
  return *reinterpret_cast<E*>(reinterpret_cast<char*>(f) + i * (uint32_t)sizeof(E));
}
template <typename E>
__device__ inline const E& at32(const E* f, uint32_t i) {
  return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(f) + i * (uint32_t)sizeof(E));
}

template <typename T>
__device__ inline cx<T> to_t(cx<double> z) { return mk<T>((T)z.re, (T)z.im); }
template <typename T>
__device__ inline cx<double> to_d(cx<T> z) { return mk<double>((double)z.re, (double)z.im); }

// ---- column-pass geometry -----------------------------------------------
template <int N, int TX, int RE>
struct ColGeo {
  static constexpr int R0 = plan(N, RE).r[0];
  static constexpr int TL = N / R0;
  static constexpr int THREADS = TX * TL;
  static constexpr int LD = TX + 1;  // LDS row pitch (padding)
};

// ---- K-A: stage combine + implicit solve + inverse z-FFT -------------------
template <typename TE>
struct StageArgs {
  const cx<double>* y;
  const cx<TE>* FE[6];
  const cx<double>* FI[6];
  double cE[6], cI[6];     // dt * A^E_ij, dt * A^I_ij for j < i
  int nprev;
  double gdt;              // dt * A^I_ii
  cx<double>* FI_out;      // F^I_i (may be null when unused)
  cx<TE>* FEc_out;         // split A: explicit CH part from z_c (may be null)
  // 1: F^I_1 is not read from FI[0] but formed as L(k) y.  With an explicit
  // first stage (A^I_11 = 0) the first stage value is the state itself, so
  // F^I_1 = L y exactly and the array is never stored.
  int fi0_from_y;
  // Last stage of an embedded method whose explicit and implicit weights
  // agree (b^E = b^I = b; one embedded b~), U_out non-null: the update and
  // error sums of the step (Eqs. ARK_method, ARK_embedding) over every term
  // but the last stage's explicit derivative are formed here, from values
  // this kernel loads anyway plus the last stage's own F^I (never stored):
  //   U = y + dt (sum_{j<i} ub_j (F^E_j + F^I_j) + ub_i F^I_i),
  //   E =     dt (sum_{j<i} eb_j (F^E_j + F^I_j) + eb_i F^I_i),
  // with ub = b and eb = b - b~ (zero where a stage array is not kept).  The
  // update then reads y, U, E and F^E_i.  One weight set for both parts keeps
  // the uniform operands few (they live in scalar registers).
  cx<double>* U_out;
  cx<double>* E_out;
  double ub[6], eb[6];  // indices < i; ub[i], eb[i] in ubs, ebs
  double ubs, ebs;
  double fdt;           // dt
};

// Stage combination for one element (Eq. ARK_stage restricted to the
// previous stages), then the implicit solve z = r / (1 - dt A^I_ii L(k)).
template <typename TE, int NP>
__device__ inline cx<double> stage_value(const StageArgs<TE>& sa, long long idx, double L, cx<double>* FIo,
                                         cx<TE>* FEo, double fea_k2, int f) {
  const cx<double> y0 = sa.y[idx];
  const bool fold = sa.U_out != nullptr;  // uniform
  cx<double> fe[NP > 0 ? NP : 1], fi[NP > 0 ? NP : 1];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const bool useF = fold && (sa.ub[j] != 0.0 || sa.eb[j] != 0.0);
    const bool useE = sa.cE[j] != 0.0 || useF;
    const bool useI = sa.cI[j] != 0.0 || useF;
    fe[j] = useE ? to_d(sa.FE[j][idx]) : mk(0.0, 0.0);
    if (j == 0 && sa.fi0_from_y)
      fi[0] = L * y0;
    else
      fi[j] = useI ? sa.FI[j][idx] : mk(0.0, 0.0);
  }
  cx<double> r = y0;
#pragma unroll
  for (int j = 0; j < NP; ++j) r = r + (sa.cE[j] * fe[j] + sa.cI[j] * fi[j]);
  const cx<double> zz = (sa.gdt != 0.0) ? (1.0 / (1.0 - sa.gdt * L)) * r : r;
  const cx<double> fin = L * zz;
  if (FIo) FIo[idx] = fin;
  if (f == 0 && FEo) FEo[idx] = to_t<TE>((-fea_k2) * zz);
  if (fold) {
    cx<double> u = sa.ubs * fin, e = sa.ebs * fin;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const cx<double> fj = fe[j] + fi[j];
      u = u + sa.ub[j] * fj;
      e = e + sa.eb[j] * fj;
    }
    sa.U_out[idx] = y0 + sa.fdt * u;
    sa.E_out[idx] = sa.fdt * e;
  }
  return zz;
}

template <typename T, typename TE, int N, int TX, int RE, int NP, bool GUARD = false>
__device__ inline void body_stage_invz(const StageArgs<TE>& sa, const Geo& g, const ModelK& m, const cx<T>* twz,
                                       cx<T>* out, int tile, int tid, cx<T>* lds) {
  using CG = ColGeo<N, TX, RE>;
  const bool act = !GUARD || tid < CG::THREADS;
  const int nbx = (g.nxh + TX - 1) / TX;
  const int xb = tile % nbx;
  const int y = tile / nbx;
  const int col = tid % TX;
  const int bf = tid / TX;
  const int x = xb * TX + col;
  const bool valid = act && x < g.nxh;
  const double kx = x * g.kfx;
  const double ky = mode_of(y, g.ny) * g.kfy;
  auto buf = [&](int pos) -> cx<T>& { return lds[pos * CG::LD + col]; };
  for (int f = 0; f < 4; ++f) {
    // combine + solve position by position into LDS (bounded unroll keeps the
    // stage-array loads of a few positions in flight, not all of them)
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < CG::R0; ++t) {
      const int z = bf + t * CG::TL;
      const long long idx = f * g.fs + ((long long)z * g.ny + y) * g.P + x;
      cx<double> r = mk(0.0, 0.0);
      if (valid) {
        const double kz = mode_of(z, g.nz) * g.kfz;
        const double k2 = kx * kx + ky * ky + kz * kz;
        r = m.inv_n3 * stage_value<TE, NP>(sa, idx, lsym(m, f, k2), sa.FI_out, sa.FEc_out, m.fEa * k2, f);
      }
      if (act) buf(z) = to_t<T>(r);
    }
    __syncthreads();
    cx<T> a[CG::R0];
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) a[t] = act ? buf(bf + t * CG::TL) : mk<T>(0, 0);
    line_fft<T, N, +1, RE>(a, bf, twz, buf, act);
    if (valid) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) {
        const int z = bf + t * CG::TL;
        out[f * g.fs + ((long long)z * g.ny + y) * g.P + x] = a[t];
      }
    }
  }
}

template <typename T, typename TE, int N, int TX, int RE, int NP>
__global__ void __launch_bounds__((ColGeo<N, TX, RE>::THREADS))
k_stage_invz(StageArgs<TE> sa, Geo g, ModelK m, const cx<T>* twz, cx<T>* __restrict__ out) {
  __shared__ cx<T> lds[N * ColGeo<N, TX, RE>::LD];
  body_stage_invz<T, TE, N, TX, RE, NP>(sa, g, m, twz, out, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, lds);
}

// Stage combination and implicit solve only (a stage whose explicit
// derivative is never used, e.g. the implicit stage of IMEX Euler).
template <typename TE>
__global__ void __launch_bounds__(256) k_combine(StageArgs<TE> sa, Geo g, ModelK m) {
  const long long nrow = (long long)g.nz * g.ny;
  const long long total = 4 * nrow * g.nxh;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % g.nxh);
    const long long fr = i / g.nxh;
    const int f = (int)(fr / nrow);
    const long long row = fr % nrow;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const double kx = x * g.kfx, ky = mode_of(y, g.ny) * g.kfy, kz = mode_of(z, g.nz) * g.kfz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const long long idx = fr * g.P + x;
    const double L = lsym(m, f, k2);
    const cx<double> y0 = sa.y[idx];
    cx<double> r = y0;
    for (int j = 0; j < sa.nprev; ++j) {
      if (sa.cE[j] != 0.0) r = r + sa.cE[j] * to_d(sa.FE[j][idx]);
      if (sa.cI[j] != 0.0) r = r + sa.cI[j] * ((j == 0 && sa.fi0_from_y) ? L * y0 : sa.FI[j][idx]);
    }
    const cx<double> zz = (sa.gdt != 0.0) ? (1.0 / (1.0 - sa.gdt * L)) * r : r;
    if (sa.FI_out) sa.FI_out[idx] = L * zz;
  }
}

// ---- generic column FFT along y or z (in or out of place) -----------------
// axis 1 = y (lines at fixed z), axis 2 = z (lines at fixed y).
template <typename T, int N, int TX, int RE, int S, int AXIS, bool GUARD = false>
__device__ inline void body_colfft(const cx<T>* in, cx<T>* out, const Geo& g, int nf, const cx<T>* tw, T scale,
                                   int tile, int tid, cx<T>* lds) {
  using CG = ColGeo<N, TX, RE>;
  const bool act = !GUARD || tid < CG::THREADS;
  const int nbx = (g.nxh + TX - 1) / TX;
  const int xb = tile % nbx;
  const int o = tile / nbx;  // fixed z (AXIS 1) or fixed y (AXIS 2)
  const int col = tid % TX;
  const int bf = tid / TX;
  const int x = xb * TX + col;
  const bool valid = act && x < g.nxh;
  const long long lstride = AXIS == 1 ? (long long)g.P : (long long)g.ny * g.P;
  const long long base = AXIS == 1 ? (long long)o * g.ny * g.P + x : (long long)o * g.P + x;
  auto buf = [&](int pos) -> cx<T>& { return lds[pos * CG::LD + col]; };
  for (int f = 0; f < nf; ++f) {
    cx<T> a[CG::R0];
    const long long fb = f * g.fs + base;
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) {
      const int q = bf + t * CG::TL;
      a[t] = valid ? in[fb + q * lstride] : mk<T>(0, 0);
    }
    line_fft<T, N, S, RE>(a, bf, tw, buf, act);
    if (valid) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) {
        const int q = bf + t * CG::TL;
        out[fb + q * lstride] = scale * a[t];
      }
    }
  }
}

// Column passes over several fields, software-pipelined: field f + 1 is
// loaded into registers while field f is transformed (LDS-only barriers,
// twiddles in LDS, so the loads stay in flight across the exchanges).  Used
// in FP32, where the second register set costs no occupancy; FP64 keeps the
// field-by-field body (it would drop from two work-groups per CU to one).
template <typename T, int N, int TX, int RE, int S, class LoadF, class StoreF>
__device__ inline void colfft_pipelined(int nf, int bf, bool valid, const cx<T>* twl, cx<T>* lds, int col,
                                        LoadF load, StoreF store) {
  using CG = ColGeo<N, TX, RE>;
  auto buf = [&](int pos) -> cx<T>& { return lds[pos * CG::LD + col]; };
  cx<T> a[CG::R0], b[CG::R0];
#pragma unroll
  for (int t = 0; t < CG::R0; ++t) a[t] = valid ? load(0, bf + t * CG::TL) : mk<T>(0, 0);
#pragma unroll 1
  for (int f = 0; f < nf; ++f) {
    if (f + 1 < nf) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) b[t] = valid ? load(f + 1, bf + t * CG::TL) : mk<T>(0, 0);
    }
    line_fft<T, N, S, RE, true>(a, bf, twl, buf, true);
    if (valid) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) store(f, bf + t * CG::TL, a[t]);
    }
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) a[t] = b[t];
  }
}

template <typename T, int N, int TX, int RE, int S, int AXIS>
__global__ void __launch_bounds__((ColGeo<N, TX, RE>::THREADS))
k_colfft(const cx<T>* in, cx<T>* out, Geo g, int nf, const cx<T>* tw, T scale) {
  using CG = ColGeo<N, TX, RE>;
  __shared__ cx<T> lds[N * CG::LD];
  if constexpr (sizeof(T) == 8) {
    body_colfft<T, N, TX, RE, S, AXIS>(in, out, g, nf, tw, scale, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x,
                                       lds);
  } else {
    __shared__ cx<T> twl[N];
    for (int j = threadIdx.x; j < N; j += CG::THREADS) twl[j] = tw[j];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nbx = (g.nxh + TX - 1) / TX;
    const int xb = tile % nbx;
    const int o = tile / nbx;
    const int col = threadIdx.x % TX;
    const int bf = threadIdx.x / TX;
    const int x = xb * TX + col;
    const long long lstride = AXIS == 1 ? (long long)g.P : (long long)g.ny * g.P;
    const long long base = AXIS == 1 ? (long long)o * g.ny * g.P + x : (long long)o * g.P + x;
    colfft_pipelined<T, N, TX, RE, S>(
        nf, bf, x < g.nxh, twl, lds, col, [&](int f, int q) { return in[f * g.fs + base + q * lstride]; },
        [&](int f, int q, cx<T> v) { out[f * g.fs + base + q * lstride] = scale * v; });
  }
}

// ---- wave-specialised column FFT (persistent) ------------------------------
// The plain column pass alternates a load phase and an FFT phase per
// work-group, so HBM idles while the butterflies run.  Here each work-group
// has CG::THREADS compute threads and WS_LOADERS loader threads and walks the
// items (field, tile) blockIdx.x, blockIdx.x + gridDim.x, ...: while the
// compute threads transform item i (exchanges in `xch`), the loader threads
// have item i + 1 copied from HBM straight into the landing buffer `land`
// (global_load_lds_dwordx4: 16 bytes per lane, lane l of a wavefront writing
// bytes [16 l, 16 l + 16) after the wavefront's LDS base), holding no
// registers meanwhile; the compute threads pick it up after the next barrier.
// Loader threads take part in every barrier of line_fft with act = false.
// The exchanges synchronise with LDS-only barriers so that neither the
// loaders' copies nor the compute threads' stores are drained at them, and
// the twiddles are read from LDS.  Columns past the last valid kx are loaded from a clamped in-row address and
// never stored (every column is transformed on its own).
constexpr int WS_LOADERS = 256;
template <typename T, int N, int TX, int RE = 8>
constexpr bool ws_ok() {
  constexpr int V = 16 / (int)sizeof(cx<T>);  // values per 16-byte copy
  return N >= 128 && TX % V == 0 && (N * TX) % (WS_LOADERS * V) == 0 &&
         TX * line_threads(N, RE) + WS_LOADERS <= 1024;
}

template <typename T>
__device__ inline void lds_dma16(const void* src, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}

template <typename T, int N, int TX, int RE, int S, int AXIS>
__global__ void __launch_bounds__((ColGeo<N, TX, RE>::THREADS + WS_LOADERS))
k_colfft_ws(const cx<T>* in, cx<T>* out, Geo g, int nf, const cx<T>* tw, T scale) {
  using CG = ColGeo<N, TX, RE>;
  static_assert(ws_ok<T, N, TX, RE>(), "loader tiling");
  constexpr int CT = CG::THREADS;
  constexpr int V = 16 / (int)sizeof(cx<T>);        // values per lane and load
  constexpr int PER_SWEEP = WS_LOADERS * V;          // values one sweep of all loaders moves
  constexpr int NE = N * TX / PER_SWEEP;             // sweeps per item
  static_assert(N * TX % PER_SWEEP == 0, "loader sweeps");
  __shared__ __attribute__((aligned(16))) cx<T> xch[N * CG::LD];
  __shared__ __attribute__((aligned(16))) cx<T> land[N * TX];
  __shared__ __attribute__((aligned(16))) cx<T> twl[N];  // twiddles: no global loads inside the loop
  const int tid = threadIdx.x;
  for (int j = tid; j < N; j += CT + WS_LOADERS) twl[j] = tw[j];
  const bool comp = tid < CT;
  const int lt = tid - CT;  // loader index
  const int col = tid % TX;
  const int bf = comp ? tid / TX : 0;
  const int nbx = (g.nxh + TX - 1) / TX;
  const long long ntile = (long long)nbx * (AXIS == 1 ? g.nz : g.ny);
  const long long nitems = ntile * nf;
  const long long lstride = AXIS == 1 ? (long long)g.P : (long long)g.ny * g.P;
  // start of item it's tile (column xb * TX) and the tile's first kx
  auto tile_base = [&](long long it, int& x0) -> long long {
    const int f = (int)(it / ntile);
    const long long tile = it % ntile;
    const int xb = (int)(tile % nbx);
    const long long o = tile / nbx;
    x0 = xb * TX;
    return f * g.fs + (AXIS == 1 ? o * g.ny * g.P : o * g.P);
  };
  // loader: copy item it into land
  auto load_item = [&](long long it) {
    int x0;
    const long long tb = tile_base(it, x0);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int flat = e * PER_SWEEP + lt * V;  // first of this lane's V values in land
      const int q = flat / TX, c0 = flat % TX;
      int x = x0 + c0;
      if (x > g.P - V) x = g.P - V;
      const int wave_first = e * PER_SWEEP + (lt & ~63) * V;
      lds_dma16<T>(in + tb + q * lstride + x, land + wave_first);
    }
  };
  auto xbuf = [&](int pos) -> cx<T>& { return xch[pos * CG::LD + col]; };
  long long it = blockIdx.x;
  if (!comp && it < nitems) {
    load_item(it);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  for (; it < nitems; it += gridDim.x) {
    const long long nxt = it + gridDim.x;
    cx<T> a[CG::R0];
    if (comp) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) a[t] = land[(bf + t * CG::TL) * TX + col];
    } else {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) a[t] = mk<T>(0, 0);
    }
    lds_barrier();  // the landing buffer has been read
    if (!comp && nxt < nitems) load_item(nxt);
    line_fft<T, N, S, RE, true>(a, bf, twl, xbuf, comp);
    if (comp) {
      int x0;
      const long long tb = tile_base(it, x0);
      if (x0 + col < g.nxh) {
#pragma unroll
        for (int t = 0; t < CG::R0; ++t) out[tb + x0 + col + (bf + t * CG::TL) * lstride] = scale * a[t];
      }
    } else {
      __builtin_amdgcn_s_waitcnt(0);
    }
    lds_barrier();  // the next item has landed (the loaders waited for their copies)
  }
}

// ---- K-E: forward z-FFT of theta, elastic solve, explicit CH, inverse z ----
template <typename T, typename TE, int N, int TX, int RE, bool GUARD = false, bool LB = false>
__device__ inline void body_zpass_elastic(cx<T>* th, const Geo& g, const ModelK& m, const cx<T>* twz, cx<TE>* FEc,
                                          int accumulate, int tile, int tid, cx<T>* lds) {
  using CG = ColGeo<N, TX, RE>;
  const bool act = !GUARD || tid < CG::THREADS;
  const int nbx = (g.nxh + TX - 1) / TX;
  const int xb = tile % nbx;
  const int y = tile / nbx;
  const uint32_t lstride = (uint32_t)(g.ny * g.P);
  // Thread-derived indices, rebuilt at each phase from an opaque copy of tid:
  // the compiler then recomputes them (and the LDS and global addresses made
  // from them) where they are used instead of holding them across the solve.
  struct Ix {
    int col, bf, x;
    uint32_t base;
    bool valid;
  };
  auto ix = [&]() {
    int tq = tid;
    asm volatile("" : "+v"(tq));
    Ix r;
    r.col = tq % TX;
    r.bf = tq / TX;
    r.x = xb * TX + r.col;
    r.valid = act && r.x < g.nxh;
    r.base = (uint32_t)(y * g.P + r.x);
    return r;
  };
  cx<T> a[3][CG::R0];
  // All three fields are loaded before the first transform.  With LB the
  // transforms synchronise with LDS-only barriers (twz then points to LDS), so
  // the loads of fields 1 and 2 stay in flight while field 0 is transformed,
  // and the stores of the inverse transforms overlap the next one.
  {
    const Ix I = ix();
#pragma unroll
    for (int v = 0; v < 3; ++v) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) {
        const int z = I.bf + t * CG::TL;
        a[v][t] = I.valid ? at32(th + v * g.fs, I.base + z * lstride) : mk<T>(0, 0);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const Ix I = ix();
    auto buf = [&](int pos) -> cx<T>& { return lds[pos * CG::LD + I.col]; };
    line_fft<T, N, -1, RE, LB>(a[v], I.bf, twz, buf, act);
  }
  // Every spectrum value is final here: left alone, the compiler sinks the
  // second half of the last butterflies past the first mode's solve and holds
  // their inputs as well.
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) pin(a[v][t]);
  {
    const Ix I = ix();
    const T kx = (T)(I.x * g.kfx);
    const T ky = (T)(mode_of(y, g.ny) * g.kfy);
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) {
      const int z = I.bf + t * CG::TL;
      const T kz = (T)(mode_of(z, g.nz) * g.kfz);
      cx<T> thv[3] = {a[0][t], a[1][t], a[2][t]};
      cx<T> e[3];
      const bool k0 = (I.x == 0) && (y == 0) && (z == 0);
      if (k0) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          cx<T> acc = mk<T>((T)m.hom[v], 0);
#pragma unroll
          for (int w = 0; w < 3; ++w) acc = acc + (T)m.B0[v][w] * thv[w];
          e[v] = acc;
        }
      } else {
        elastic_apply<T>(m, kx, ky, kz, thv, e);
      }
      if (I.valid) {
        const T k2 = kx * kx + ky * ky + kz * kz;
        cx<T> Hs = thv[0] + thv[1] + thv[2];
        cx<T> fe = ((T)m.fEc * k2) * Hs;
        const uint32_t idx = I.base + z * lstride;
        if (accumulate) {
          cx<TE> old = at32(FEc, idx);
          at32(FEc, idx) = mk<TE>((TE)(old.re + fe.re), (TE)(old.im + fe.im));
        } else {
          at32(FEc, idx) = mk<TE>((TE)fe.re, (TE)fe.im);
        }
      }
      const T s = (T)m.inv_n3;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        a[v][t] = s * e[v];
        pin(a[v][t]);
      }
      // one mode at a time: interleaving the solves only raises register pressure
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const Ix I = ix();
    auto buf = [&](int pos) -> cx<T>& { return lds[pos * CG::LD + I.col]; };
    line_fft<T, N, +1, RE, LB>(a[v], I.bf, twz, buf, act);
    if (I.valid) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) {
        const int z = I.bf + t * CG::TL;
        at32(th + v * g.fs, I.base + z * lstride) = a[v][t];
      }
    }
  }
}

template <typename T, typename TE, int N, int TX, int RE>
__global__ void __launch_bounds__((ColGeo<N, TX, RE>::THREADS))
k_zpass_elastic(cx<T>* __restrict__ th, Geo g, ModelK m, const cx<T>* twz, cx<TE>* __restrict__ FEc,
                int accumulate) {
  __shared__ cx<T> lds[N * ColGeo<N, TX, RE>::LD];
  __shared__ cx<T> twl[N];
  for (int j = threadIdx.x; j < N; j += ColGeo<N, TX, RE>::THREADS) twl[j] = twz[j];
  body_zpass_elastic<T, TE, N, TX, RE, false, true>(th, g, m, twl, FEc, accumulate,
                                                    xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, lds);
}

// ---- K-I: forward z-FFT of the AC driving force, F^E_eta = -L g~ ----------
template <typename T, typename TE, int N, int TX, int RE, bool GUARD = false>
__device__ inline void body_zpass_fwd_ac(const cx<T>* gk, const Geo& g, const ModelK& m, const cx<T>* twz,
                                         cx<TE>* FE, int tile, int tid, cx<T>* lds) {
  using CG = ColGeo<N, TX, RE>;
  const bool act = !GUARD || tid < CG::THREADS;
  const int nbx = (g.nxh + TX - 1) / TX;
  const int xb = tile % nbx;
  const int y = tile / nbx;
  const int col = tid % TX;
  const int bf = tid / TX;
  const int x = xb * TX + col;
  const bool valid = act && x < g.nxh;
  const long long lstride = (long long)g.ny * g.P;
  const long long base = (long long)y * g.P + x;
  auto buf = [&](int pos) -> cx<T>& { return lds[pos * CG::LD + col]; };
  const T nl = (T)(-m.L);
  for (int v = 0; v < 3; ++v) {
    cx<T> a[CG::R0];
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) {
      const int z = bf + t * CG::TL;
      a[t] = valid ? gk[v * g.fs + base + z * lstride] : mk<T>(0, 0);
    }
    line_fft<T, N, -1, RE>(a, bf, twz, buf, act);
    if (valid) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) {
        const int z = bf + t * CG::TL;
        cx<T> r = nl * a[t];
        FE[(1 + v) * g.fs + base + z * lstride] = mk<TE>((TE)r.re, (TE)r.im);
      }
    }
  }
}

template <typename T, typename TE, int N, int TX, int RE>
__global__ void __launch_bounds__((ColGeo<N, TX, RE>::THREADS))
k_zpass_fwd_ac(const cx<T>* __restrict__ gk, Geo g, ModelK m, const cx<T>* twz, cx<TE>* __restrict__ FE) {
  using CG = ColGeo<N, TX, RE>;
  __shared__ cx<T> lds[N * CG::LD];
  if constexpr (sizeof(T) == 8) {
    body_zpass_fwd_ac<T, TE, N, TX, RE>(gk, g, m, twz, FE, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, lds);
  } else {
    __shared__ cx<T> twl[N];
    for (int j = threadIdx.x; j < N; j += CG::THREADS) twl[j] = twz[j];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int nbx = (g.nxh + TX - 1) / TX;
    const int xb = tile % nbx;
    const int y = tile / nbx;
    const int col = threadIdx.x % TX;
    const int bf = threadIdx.x / TX;
    const int x = xb * TX + col;
    const long long lstride = (long long)g.ny * g.P;
    const long long base = (long long)y * g.P + x;
    const T nl = (T)(-m.L);
    colfft_pipelined<T, N, TX, RE, -1>(
        3, bf, x < g.nxh, twl, lds, col, [&](int f, int z) { return gk[f * g.fs + base + z * lstride]; },
        [&](int f, int z, cx<T> v) {
          const cx<T> r = nl * v;
          FE[(1 + f) * g.fs + base + z * lstride] = mk<TE>((TE)r.re, (TE)r.im);
        });
  }
}

// ---- row (x-axis) passes ---------------------------------------------------
template <int M, int RB>
struct RowGeo {
  static constexpr int R0 = plan(M).r[0];
  static constexpr int TL = M / R0;
  static constexpr int THREADS = RB * TL;
  static constexpr int LD = M + 2;
};

// The HBM reads of row_c2r on their own: raw[t] = src[bf + t TL], raw[R0] =
// src[M] (bf == 0), so a caller can have them in flight during other work.
template <typename T, int M, int RB>
__device__ inline void row_fetch(const cx<T>* src, bool rvalid, cx<T>* raw, int bf, bool act = true) {
  using RG = RowGeo<M, RB>;
#pragma unroll
  for (int t = 0; t < RG::R0; ++t) raw[t] = (act && rvalid) ? src[bf + t * RG::TL] : mk<T>(0, 0);
  raw[RG::R0] = (act && rvalid && bf == 0) ? src[M] : mk<T>(0, 0);
}

// row_c2r from values fetched by row_fetch.
// LB: LDS-only barriers (global loads and stores stay in flight across them).
template <typename T, int M, int RB, bool LB = false>
__device__ inline void row_c2r_regs(const cx<T>* raw, cx<T>* a, int bf, cx<T>* rbuf, const cx<T>* twN,
                                    const cx<T>* twM, bool act = true) {
  using RG = RowGeo<M, RB>;
  xbar<LB>();
  if (act) {
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) rbuf[bf + t * RG::TL] = raw[t];
    if (bf == 0) rbuf[M] = raw[RG::R0];
  }
  xbar<LB>();
  if (act) {
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const int k = bf + t * RG::TL;
      cx<T> xk = rbuf[k];
      cx<T> xmk = rbuf[M - k];
      if (k == 0) {
        xk.im = (T)0;
        xmk.im = (T)0;
      }
      a[t] = c2r_pre(xk, xmk, twN[k]);
    }
  }
  line_fft<T, M, +1, 8, LB>(a, bf, twM, [&](int pos) -> cx<T>& { return rbuf[pos]; }, act);
}

// c2r of one half-spectrum row src[0..M] into real pairs a[t] = (x_{2n}, x_{2n+1}),
// n = bf + t TL.  Unnormalised (full-spectrum sum).
template <typename T, int M, int RB>
__device__ inline void row_c2r(const cx<T>* src, bool rvalid, cx<T>* a, int bf, cx<T>* rbuf,
                               const cx<T>* twN, const cx<T>* twM, bool act = true) {
  using RG = RowGeo<M, RB>;
  cx<T> raw[RG::R0 + 1];
  row_fetch<T, M, RB>(src, rvalid, raw, bf, act);
  row_c2r_regs<T, M, RB>(raw, a, bf, rbuf, twN, twM, act);
}

// r2c of real pairs a[t] (n = bf + t TL) into half-spectrum row dst[0..M].
template <typename T, int M, int RB, bool LB = false>
__device__ inline void row_r2c(cx<T>* a, cx<T>* dst, bool rvalid, int bf, cx<T>* rbuf,
                               const cx<T>* twN, const cx<T>* twM, bool act = true) {
  using RG = RowGeo<M, RB>;
  line_fft<T, M, -1, 8, LB>(a, bf, twM, [&](int pos) -> cx<T>& { return rbuf[pos]; }, act);
  xbar<LB>();
  if (act) {
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) rbuf[bf + t * RG::TL] = a[t];
  }
  xbar<LB>();
  if (act && rvalid) {
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const int k = bf + t * RG::TL;
      const cx<T> zk = rbuf[k];
      const cx<T> zmk = rbuf[k == 0 ? 0 : M - k];
      dst[k] = r2c_post(zk, zmk, twN[k]);
    }
    if (bf == 0) {
      const cx<T> z0 = rbuf[0];
      dst[M] = mk<T>(z0.re - z0.im, (T)0);
    }
  }
}

template <typename T>
__device__ inline T hfun(T e) { return e * e * e * (e * ((T)6 * e - (T)15) + (T)10); }
template <typename T>
__device__ inline T dhfun(T e) {
  const T u = e * ((T)1 - e);
  return (T)30 * u * u;
}

// K-C: theta_v = h(eta_v) (rows of the 3 eta fields of `st` -> rows of `th`).
template <typename T, int M, int RB, bool GUARD = false>
__device__ inline void body_xpass_theta(const cx<T>* st, cx<T>* th, const Geo& g, const cx<T>* twN,
                                        const cx<T>* twM, int tile, int tid, cx<T>* lds) {
  using RG = RowGeo<M, RB>;
  const bool act = !GUARD || tid < RG::THREADS;
  const int rl = tid / RG::TL;
  const int bf = tid % RG::TL;
  const int row = tile * RB + rl;
  const bool rvalid = act && row < g.nz * g.ny;
  cx<T>* rbuf = lds + (act ? rl : 0) * RG::LD;
  const long long rb = (long long)(rvalid ? row : 0) * g.P;
  for (int v = 0; v < 3; ++v) {
    cx<T> a[RG::R0];
    row_c2r<T, M, RB>(st + (1 + v) * g.fs + rb, rvalid, a, bf, rbuf, twN, twM, act);
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) a[t] = mk<T>(hfun(a[t].re), hfun(a[t].im));
    row_r2c<T, M, RB>(a, th + v * g.fs + rb, rvalid, bf, rbuf, twN, twM, act);
  }
}

// Single-grid theta pass, software-pipelined: the rows of eta_{v+1} are
// requested before eta_v's transform back, and stay in flight across its
// exchanges (LDS-only barriers; the line-FFT twiddles are copied to LDS so
// that no global load issued after the prefetch has to wait for it).
template <typename T, int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_xpass_theta(const cx<T>* __restrict__ st, cx<T>* __restrict__ th, Geo g, const cx<T>* twN,
              const cx<T>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<T> lds[RB * RG::LD];
  __shared__ cx<T> tM[M], tN[M];
  for (int j = threadIdx.x; j < M; j += RG::THREADS) {
    tM[j] = twM[j];
    tN[j] = twN[j];
  }
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const bool rvalid = row < g.nz * g.ny;
  cx<T>* rbuf = lds + rl * RG::LD;
  const long long rb = (long long)(rvalid ? row : 0) * g.P;
  cx<T> raw[RG::R0 + 1];
  row_fetch<T, M, RB>(st + g.fs + rb, rvalid, raw, bf);
#pragma unroll 1
  for (int v = 0; v < 3; ++v) {
    cx<T> a[RG::R0];
    row_c2r_regs<T, M, RB, true>(raw, a, bf, rbuf, tN, tM);
    if (v < 2) row_fetch<T, M, RB>(st + (2 + v) * g.fs + rb, rvalid, raw, bf);
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) a[t] = mk<T>(hfun(a[t].re), hfun(a[t].im));
    row_r2c<T, M, RB, true>(a, th + v * g.fs + rb, rvalid, bf, rbuf, tN, tM);
  }
}

// K-G: g_v = h'(eta_v) (chi(c) + e_v) + 2 w eta_v (1 - eta_v)(1 - 2 eta_v).
template <typename T, int M, int RB, bool GUARD = false, bool LB = false>
__device__ inline void body_xpass_drive(const cx<T>* st, cx<T>* el, const Geo& g, const ModelK& m,
                                        const cx<T>* twN, const cx<T>* twM, int tile, int tid, cx<T>* lds) {
  using RG = RowGeo<M, RB>;
  const bool act = !GUARD || tid < RG::THREADS;
  const int rl = tid / RG::TL;
  const int bf = tid % RG::TL;
  const int row = tile * RB + rl;
  const bool rvalid = act && row < g.nz * g.ny;
  cx<T>* rbuf = lds + (act ? rl : 0) * RG::LD;
  const long long rb = (long long)(rvalid ? row : 0) * g.P;
  const T W = (T)m.W, cm = (T)m.cm, cp = (T)m.cp, w2 = (T)(2.0 * m.w);
  cx<T> chi[RG::R0];
  {
    cx<T> a[RG::R0];
    cx<T> raw[RG::R0 + 1];
    row_fetch<T, M, RB>(st + rb, rvalid, raw, bf, act);
    row_c2r_regs<T, M, RB, LB>(raw, a, bf, rbuf, twN, twM, act);
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const T c0 = a[t].re, c1 = a[t].im;
      chi[t] = mk<T>(W * ((c0 - cp) * (c0 - cp) - (c0 - cm) * (c0 - cm)),
                     W * ((c1 - cp) * (c1 - cp) - (c1 - cm) * (c1 - cm)));
    }
  }
  for (int v = 0; v < 3; ++v) {
    cx<T> et[RG::R0], a[RG::R0];
    if constexpr (sizeof(T) == 8) {
      // FP64: both rows of this variant are requested before either is
      // transformed (8% faster at 512^3; 8% slower in FP32, kept apart there)
      cx<T> raw_e[RG::R0 + 1];
      cx<T> raw_et[RG::R0 + 1];
      row_fetch<T, M, RB>(st + (1 + v) * g.fs + rb, rvalid, raw_et, bf, act);
      row_fetch<T, M, RB>(el + v * g.fs + rb, rvalid, raw_e, bf, act);
      row_c2r_regs<T, M, RB, LB>(raw_et, et, bf, rbuf, twN, twM, act);
      row_c2r_regs<T, M, RB, LB>(raw_e, a, bf, rbuf, twN, twM, act);
    } else {
      row_c2r<T, M, RB>(st + (1 + v) * g.fs + rb, rvalid, et, bf, rbuf, twN, twM, act);
      row_c2r<T, M, RB>(el + v * g.fs + rb, rvalid, a, bf, rbuf, twN, twM, act);
    }
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const T e0 = et[t].re, e1 = et[t].im;
      const T g0 = dhfun(e0) * (chi[t].re + a[t].re) + w2 * e0 * ((T)1 - e0) * ((T)1 - (T)2 * e0);
      const T g1 = dhfun(e1) * (chi[t].im + a[t].im) + w2 * e1 * ((T)1 - e1) * ((T)1 - (T)2 * e1);
      a[t] = mk<T>(g0, g1);
    }
    row_r2c<T, M, RB, LB>(a, el + v * g.fs + rb, rvalid, bf, rbuf, twN, twM, act);
  }
}

// Single-grid driving-force pass, software-pipelined like the theta pass (FP32):
// the eta row of variant v + 1 is requested before variant v's transform back
// and stays in flight across its exchanges; the elastic-potential row of
// variant v + 1 is requested after that transform and stays in flight across
// the eta row's transform (the first eta row with the composition row, the
// first elastic row after the composition row's transform).
template <typename T, int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_xpass_drive(const cx<T>* __restrict__ st, cx<T>* __restrict__ el, Geo g, ModelK m, const cx<T>* twN,
              const cx<T>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<T> lds[RB * RG::LD];
  // both twiddle tables in LDS: no global load issued after a prefetch has
  // to wait for it
  __shared__ cx<T> tM[M], tN[M];
  for (int j = threadIdx.x; j < M; j += RG::THREADS) {
    tM[j] = twM[j];
    tN[j] = twN[j];
  }
  if constexpr (sizeof(T) == 8) {
    // FP64: the prefetch registers would cut the occupancy from 3 to 2 waves
    // per SIMD; the plain body runs with LDS-only barriers instead, so each
    // variant's two rows load while nothing else waits for them and the
    // stores of the previous variant stay in flight
    body_xpass_drive<T, M, RB, false, true>(st, el, g, m, tN, tM, blockIdx.x, threadIdx.x, lds);
    return;
  }
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const bool rvalid = row < g.nz * g.ny;
  cx<T>* rbuf = lds + rl * RG::LD;
  const long long rb = (long long)(rvalid ? row : 0) * g.P;
  const T W = (T)m.W, cm = (T)m.cm, cp = (T)m.cp, w2 = (T)(2.0 * m.w);
  cx<T> raw_eta[RG::R0 + 1], raw_e[RG::R0 + 1];
  cx<T> chi[RG::R0];
  {
    cx<T> raw_c[RG::R0 + 1];
    row_fetch<T, M, RB>(st + rb, rvalid, raw_c, bf);
    row_fetch<T, M, RB>(st + g.fs + rb, rvalid, raw_eta, bf);
    cx<T> a[RG::R0];
    row_c2r_regs<T, M, RB, true>(raw_c, a, bf, rbuf, tN, tM);
    row_fetch<T, M, RB>(el + rb, rvalid, raw_e, bf);
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const T c0 = a[t].re, c1 = a[t].im;
      chi[t] = mk<T>(W * ((c0 - cp) * (c0 - cp) - (c0 - cm) * (c0 - cm)),
                     W * ((c1 - cp) * (c1 - cp) - (c1 - cm) * (c1 - cm)));
    }
  }
#pragma unroll 1
  for (int v = 0; v < 3; ++v) {
    cx<T> et[RG::R0], a[RG::R0];
    row_c2r_regs<T, M, RB, true>(raw_eta, et, bf, rbuf, tN, tM);
    row_c2r_regs<T, M, RB, true>(raw_e, a, bf, rbuf, tN, tM);
    if (v < 2) row_fetch<T, M, RB>(st + (2 + v) * g.fs + rb, rvalid, raw_eta, bf);
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const T e0 = et[t].re, e1 = et[t].im;
      const T g0 = dhfun(e0) * (chi[t].re + a[t].re) + w2 * e0 * ((T)1 - e0) * ((T)1 - (T)2 * e0);
      const T g1 = dhfun(e1) * (chi[t].im + a[t].im) + w2 * e1 * ((T)1 - e1) * ((T)1 - (T)2 * e1);
      a[t] = mk<T>(g0, g1);
    }
    row_r2c<T, M, RB, true>(a, el + v * g.fs + rb, rvalid, bf, rbuf, tN, tM);
    if (v < 2) row_fetch<T, M, RB>(el + (1 + v) * g.fs + rb, rvalid, raw_e, bf);
  }
}

// Standalone row r2c: real rows (length 2M, pitch 2M) -> half-spectrum rows.
template <typename T, int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_xpass_r2c(const T* __restrict__ re, cx<T>* __restrict__ out, Geo g, int nf,
            const cx<T>* twN, const cx<T>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<T> lds[RB * RG::LD];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<T>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  for (int f = 0; f < nf; ++f) {
    const cx<T>* src = reinterpret_cast<const cx<T>*>(re + ((long long)f * nrows + rr) * (2 * M));
    cx<T> a[RG::R0];
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) a[t] = rvalid ? src[bf + t * RG::TL] : mk<T>(0, 0);
    row_r2c<T, M, RB>(a, out + f * g.fs + rr * g.P, rvalid, bf, rbuf, twN, twM);
  }
}

// Standalone row c2r: half-spectrum rows -> real rows, times `scale`.
template <typename T, int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_xpass_c2r(const cx<T>* __restrict__ in, T* __restrict__ re, Geo g, int nf, T scale,
            const cx<T>* twN, const cx<T>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<T> lds[RB * RG::LD];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<T>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  for (int f = 0; f < nf; ++f) {
    cx<T> a[RG::R0];
    row_c2r<T, M, RB>(in + f * g.fs + rr * g.P, rvalid, a, bf, rbuf, twN, twM);
    if (rvalid) {
      cx<T>* dst = reinterpret_cast<cx<T>*>(re + ((long long)f * nrows + rr) * (2 * M));
#pragma unroll
      for (int t = 0; t < RG::R0; ++t) dst[bf + t * RG::TL] = scale * a[t];
    }
  }
}

// ---- reductions ------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum (blockDim.x multiple of 64, <= 1024); result valid in thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// ---- finalize: update, embedded error, WRMS partial sums ------------------
template <typename TE>
struct FinArgs {
  const cx<double>* y;
  cx<double>* ynew;
  const cx<TE>* FE[6];
  const cx<double>* FI[6];
  double bE[6], bI[6];   // update weights (times dt)
  double dE[6], dI[6];   // error weights (b - b~) times dt
  int s;
  int want_err;
  int fi0_from_y;         // F^I_1 = L(k) y (explicit first stage), FI[0] unread
  // partial sums from the last stage (null: off): y_new = U + sum(...),
  // error = E + sum(...); the weights then hold only the last stage's F^E term
  const cx<double>* U;
  const cx<double>* E;
  double rtol, atol, sc;  // sc = 1/sqrt(N^3)
  double* partial;        // [2 * gridDim.x]: sum of squares, non-finite count
  // non-null: the error estimate is also stored here (it may be E or FI[0]:
  // each element is read before it is written, by the same thread), for a
  // norm taken in real space
  cx<double>* err_out;
};

template <typename TE>
__global__ void __launch_bounds__(256) k_finalize(FinArgs<TE> fa, Geo g, ModelK m) {
  __shared__ double sh[16];
  // 32-bit indices: 4 nz ny (nx/2+1) < 2^31 on every supported grid
  const unsigned nrow = (unsigned)(g.nz * g.ny);
  const unsigned nxh = (unsigned)g.nxh;
  const unsigned total = 4u * nrow * nxh;
  double acc = 0.0, bad = 0.0;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const unsigned x = i % nxh;
    const unsigned fr = i / nxh;  // f * nrow + row
    const long long idx = (long long)fr * g.P + x;
    const cx<double> y0 = fa.y[idx];
    // every stage array this step reads is loaded before any is used, so the
    // loads of one element are in flight together (unused weights are zero)
    cx<double> fi[6], fe[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const bool hasI = j < fa.s && (fa.bI[j] != 0.0 || (fa.want_err && fa.dI[j] != 0.0));
      const bool hasE = j < fa.s && (fa.bE[j] != 0.0 || (fa.want_err && fa.dE[j] != 0.0));
      fi[j] = (hasI && !(j == 0 && fa.fi0_from_y)) ? fa.FI[j][idx] : mk(0.0, 0.0);
      fe[j] = hasE ? to_d(fa.FE[j][idx]) : mk(0.0, 0.0);
    }
    if (fa.fi0_from_y) {
      const unsigned f = fr / nrow, row = fr % nrow;
      const int yy = (int)(row % (unsigned)g.ny), z = (int)(row / (unsigned)g.ny);
      const double kx = (int)x * g.kfx, ky = mode_of(yy, g.ny) * g.kfy, kz = mode_of(z, g.nz) * g.kfz;
      const double k2 = kx * kx + ky * ky + kz * kz;
      fi[0] = lsym(m, (int)f, k2) * y0;
    }
    cx<double> inc = mk(0.0, 0.0), err = fa.E ? fa.E[idx] : mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j >= fa.s) break;
      inc = inc + (fa.bI[j] * fi[j] + fa.bE[j] * fe[j]);
      err = err + (fa.dI[j] * fi[j] + fa.dE[j] * fe[j]);
    }
    const cx<double> yn = (fa.U ? fa.U[idx] : y0) + inc;
    fa.ynew[idx] = yn;
    if (!isfinite(yn.re) || !isfinite(yn.im)) bad += 1.0;
    if (fa.err_out) fa.err_out[idx] = err;
    if (fa.want_err) {
      const double mult = (x == 0 || 2 * (int)x == g.nx) ? 1.0 : 2.0;
      const double ay = sqrt(y0.re * y0.re + y0.im * y0.im) * fa.sc;
      const double wgt = 1.0 / (fa.rtol * ay + fa.atol);
      const double e2 = (err.re * err.re + err.im * err.im) * fa.sc * fa.sc;
      acc += mult * e2 * wgt * wgt;
    }
  }
  const double s0 = block_sum(acc, sh);
  const double s1 = block_sum(bad, sh);
  if (threadIdx.x == 0) {
    fa.partial[2 * blockIdx.x] = s0;
    fa.partial[2 * blockIdx.x + 1] = s1;
  }
}

// Non-template kernels get internal linkage: this header is included by more
// than one translation unit.
namespace {

// Sums n (value, flag) partial pairs in a fixed order into out[0], out[1].
__global__ void __launch_bounds__(256) k_reduce_pairs(const double* partial, int n, double* out) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

// Real-space WRMS partial sums (Eqs. wrms_norm, wrms_weights applied point by
// point): sum_i (e_i / (rtol |y_i| + atol))^2 over n values of the error e and
// the previous state y, one value per block.
__global__ void __launch_bounds__(256) k_wrms_real(const double* e, const double* y, long long n, double rtol,
                                                   double atol, double* partial) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double w = e[i] / (rtol * fabs(y[i]) + atol);
    acc += w * w;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Sums n partial tuples of nv values (nv <= 4) in a fixed order into out[0..nv).
__global__ void __launch_bounds__(256) k_reduce_tuples(const double* partial, int n, int nv, double* out) {
  __shared__ double sh[16];
  for (int v = 0; v < nv; ++v) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += partial[nv * i + v];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) out[v] = a;
  }
}

// Real-space diagnostics over the fields u = [4][N] (c, eta_1..3), per block:
// sum of H = sum_v h(eta_v) (volume fraction), count of points with
// max_v eta_v > 1/2, and sum of the bulk free-energy density
// f = W (c - c_m)^2 (1 - H) + W (c - c_p)^2 H + w sum_v eta_v^2 (1 - eta_v)^2.
// With theta_out set, eta_v is replaced by theta_v = h(eta_v) in place (each
// point is read, then written, by one thread).
__global__ void __launch_bounds__(256) k_diag_real(double* u, long long npts, ModelK m, int theta_out,
                                                   double* partial) {
  __shared__ double sh[16];
  double hs = 0.0, cnt = 0.0, fb = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < npts;
       i += (long long)gridDim.x * blockDim.x) {
    const double c = u[i];
    const double e1 = u[npts + i], e2 = u[2 * npts + i], e3 = u[3 * npts + i];
    const double h1 = hfun(e1), h2 = hfun(e2), h3 = hfun(e3);
    const double H = h1 + h2 + h3;
    hs += H;
    cnt += fmax(e1, fmax(e2, e3)) > 0.5 ? 1.0 : 0.0;
    const double dw = e1 * e1 * (1.0 - e1) * (1.0 - e1) + e2 * e2 * (1.0 - e2) * (1.0 - e2) +
                      e3 * e3 * (1.0 - e3) * (1.0 - e3);
    fb += m.W * (c - m.cm) * (c - m.cm) * (1.0 - H) + m.W * (c - m.cp) * (c - m.cp) * H + m.w * dw;
    if (theta_out) {
      u[npts + i] = h1;
      u[2 * npts + i] = h2;
      u[3 * npts + i] = h3;
    }
  }
  hs = block_sum(hs, sh);
  cnt = block_sum(cnt, sh);
  fb = block_sum(fb, sh);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x] = hs;
    partial[3 * blockIdx.x + 1] = cnt;
    partial[3 * blockIdx.x + 2] = fb;
  }
}

// Reciprocal-space energy sums over the half spectrum, each mode counted with
// its multiplicity m(k) (1 for kx = 0 and the Nyquist plane, else 2), per
// block: the gradient energy kernel sum m k^2 (kappa_c |c~|^2 + kappa_eta
// sum_v |eta~_v|^2) of the state y, and the elastic energy kernel
// sum m sum_vw B_vw(k) Re(th~_v conj th~_w) of th~ = FFT(h(eta)) (3 fields),
// with B(0) the k = 0 rule.  Both still carry 1 / (2 N^3) and dx^3.
__global__ void __launch_bounds__(256) k_energy_kspace(const cx<double>* y, const cx<double>* th, Geo g, ModelK m,
                                                       double* partial) {
  __shared__ double sh[16];
  const long long nrow = (long long)g.nz * g.ny;
  const long long total = nrow * g.nxh;
  double gr = 0.0, el = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % g.nxh);
    const long long row = i / g.nxh;
    const int yy = (int)(row % g.ny), z = (int)(row / g.ny);
    const long long idx = row * g.P + x;
    const double kx = x * g.kfx, ky = mode_of(yy, g.ny) * g.kfy, kz = mode_of(z, g.nz) * g.kfz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double mult = (x == 0 || 2 * x == g.nx) ? 1.0 : 2.0;
    const cx<double> cc = y[idx];
    double eta2 = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const cx<double> e = y[(1 + v) * g.fs + idx];
      eta2 += e.re * e.re + e.im * e.im;
    }
    gr += mult * k2 * (m.kc * (cc.re * cc.re + cc.im * cc.im) + m.ke * eta2);
    cx<double> t[3], e[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) t[v] = th[v * g.fs + idx];
    if (x == 0 && yy == 0 && z == 0) {
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        e[v] = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < 3; ++w) e[v] = e[v] + m.B0[v][w] * t[w];
      }
    } else {
      elastic_apply<double>(m, kx, ky, kz, t, e);
    }
    double q = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) q += e[v].re * t[v].re + e[v].im * t[v].im;
    el += mult * q;
  }
  gr = block_sum(gr, sh);
  el = block_sum(el, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = gr;
    partial[2 * blockIdx.x + 1] = el;
  }
}

}  // namespace

// Element-wise copy with precision conversion over valid k-space entries.
template <typename TA, typename TB>
__global__ void __launch_bounds__(256) k_convert(const cx<TA>* a, cx<TB>* b, Geo g, int nf) {
  const long long total = (long long)nf * g.fs;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const cx<TA> v = a[i];
    b[i] = mk<TB>((TB)v.re, (TB)v.im);
  }
}

}  // namespace pf
