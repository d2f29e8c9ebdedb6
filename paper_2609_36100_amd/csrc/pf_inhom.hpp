// Inhomogeneous elasticity: Reuss-averaged stiffness solved by the Hu-Chen
// iteration (Methods, "Phase-field model formulation": Eq. u_gov with the
// Reuss average of the phases' stiffness; Methods, "MEUMAPPS C++ and the
// MEUMAPPS-SS application": the iterative approach of Hu and Chen).
//
// The local compliance is the linear interpolation S(r) = H S_p + (1 - H) S_m
// (H = sum_v h(eta_v)) of two cubic compliances, so the local stiffness
// C(r) = S(r)^-1 is cubic in the grid axes and has a closed form.  The strain
// of the periodic displacement is found by the polarisation iteration
//   tau = C0 eps* - (C(r) - C0)(eps_bar + eps_u - eps*),  eps_u <- Gamma0 tau,
// with the homogeneous reference C0 = (C_m + C_p) / 2 and Gamma0 the Green
// operator of C0 (per wavevector: p = Omega0(n) tau~ n,
// eps~_ij = (n_j p_i + n_i p_j) / 2, n along the wavevector with its Nyquist
// components zeroed).  The start drops (C - C0).  The elastic part of the
// Allen-Cahn driving force is h'(eta_v)[-sigma : eps*_v
// - 1/2 sigma : (S_p - S_m) : sigma].
//
// Passes of one right-hand side (T1: the state after its inverse z and y
// transforms; E6: six strain / polarisation spectra; R6: the six real strain
// fields, tensor components xx, yy, zz, yz, xz, xy; LC6: six real fields of
// per-point coefficients):
//   x theta -> y, z forward (3)            theta~
//   k_el_start        theta~ -> Gamma0 C0 eps*(theta~) into E6, F^E_c
//   x_el_local        T1 eta -> LC6 (the polarisation's per-point coefficients)
//   z, y inverse (6) -> x_el_strain        R6 = eps_u
//   repeat:  x_el_tau (LC6, R6 -> E6), y forward (6), k_el_zgamma (z forward,
//            Gamma0, z inverse), y inverse (6), x_el_strain (E6 -> R6, largest
//            change)
//   x_el_drive (T1, R6 -> T3 g) -> y forward, z forward to F^E_eta
#pragma once

#include "pf_kernels.hpp"

namespace pf {

// Cubic stiffness (C11, C12, C44, Voigt with engineering shears) of the
// interpolated compliance at H.
struct Cubic {
  double c11, c12, c44;
};
__device__ inline Cubic local_stiffness(const ModelK& m, double H) {
  const double s11 = m.Sm[0] + H * m.dS[0];
  const double s12 = m.Sm[1] + H * m.dS[1];
  const double s44 = m.Sm[2] + H * m.dS[2];
  const double d = (s11 - s12) * (s11 + 2.0 * s12);
  Cubic c;
  c.c11 = (s11 + s12) / d;
  c.c12 = -s12 / d;
  c.c44 = 1.0 / s44;
  return c;
}

// Unit vector along the derivative wavevector of mode (x, y, z): Nyquist
// components zeroed; false where nothing is left (k = 0 included).
__device__ inline bool deriv_normal(const Geo& g, int x, int y, int z, double n[3]) {
  const int my = mode_of(y, g.ny), mz = mode_of(z, g.nz);
  const double kx = (2 * x == g.nx) ? 0.0 : x * g.kfx;
  const double ky = (2 * my == -g.ny) ? 0.0 : my * g.kfy;
  const double kz = (2 * mz == -g.nz) ? 0.0 : mz * g.kfz;
  const double k2 = kx * kx + ky * ky + kz * kz;
  if (k2 == 0.0) return false;
  const double r = 1.0 / sqrt(k2);
  n[0] = kx * r;
  n[1] = ky * r;
  n[2] = kz * r;
  return true;
}

// eps~ = Gamma0(n) tau~ for one mode; tau, eps: tensor components
// xx, yy, zz, yz, xz, xy (complex).  Omega0 = (C0_ijkl n_j n_l)^-1 by its
// adjugate (symmetric).
__device__ inline void gamma0_apply(const ModelK& m, const double n[3], const cx<double> tau[6],
                                    cx<double> eps[6]) {
  const double a = m.C0[0] - m.C0[1] - 2.0 * m.C0[2];
  const double b = m.C0[1] + m.C0[2];
  const double g00 = m.C0[2] + (a + b) * n[0] * n[0];
  const double g11 = m.C0[2] + (a + b) * n[1] * n[1];
  const double g22 = m.C0[2] + (a + b) * n[2] * n[2];
  const double g01 = b * n[0] * n[1], g02 = b * n[0] * n[2], g12 = b * n[1] * n[2];
  const double A00 = g11 * g22 - g12 * g12;
  const double A11 = g00 * g22 - g02 * g02;
  const double A22 = g00 * g11 - g01 * g01;
  const double A01 = g02 * g12 - g01 * g22;
  const double A02 = g01 * g12 - g02 * g11;
  const double A12 = g01 * g02 - g00 * g12;
  const double idet = 1.0 / (g00 * A00 + g01 * A01 + g02 * A02);
  // t_i = tau_ij n_j
  const cx<double> t0 = n[0] * tau[0] + n[1] * tau[5] + n[2] * tau[4];
  const cx<double> t1 = n[0] * tau[5] + n[1] * tau[1] + n[2] * tau[3];
  const cx<double> t2 = n[0] * tau[4] + n[1] * tau[3] + n[2] * tau[2];
  const cx<double> p0 = idet * (A00 * t0 + A01 * t1 + A02 * t2);
  const cx<double> p1 = idet * (A01 * t0 + A11 * t1 + A12 * t2);
  const cx<double> p2 = idet * (A02 * t0 + A12 * t1 + A22 * t2);
  eps[0] = n[0] * p0;
  eps[1] = n[1] * p1;
  eps[2] = n[2] * p2;
  eps[3] = 0.5 * (n[2] * p1 + n[1] * p2);
  eps[4] = 0.5 * (n[2] * p0 + n[0] * p2);
  eps[5] = 0.5 * (n[1] * p0 + n[0] * p1);
}

// Non-template kernels get internal linkage (headers may be included by more
// than one translation unit).
namespace {

// Start of the iteration, per mode of the half spectrum: tau~ = C0 eps*(theta~)
// (diagonal), eps~ = Gamma0 tau~ into the six fields of e6; the explicit
// Cahn-Hilliard term F^E_c = fEc k^2 H~ into field 0 of FE (added to what is
// there with `accumulate`).
__global__ void __launch_bounds__(256) k_el_start(const cx<double>* th, cx<double>* e6, cx<double>* FE,
                                                  int accumulate, Geo g, ModelK m) {
  const long long nrow = (long long)g.nz * g.ny;
  const long long total = nrow * g.nxh;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % g.nxh);
    const long long row = i / g.nxh;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const long long idx = row * g.P + x;
    cx<double> t[3], Hs = mk(0.0, 0.0);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      t[v] = th[v * g.fs + idx];
      Hs = Hs + t[v];
    }
    cx<double> tau[6];
#pragma unroll
    for (int i3 = 0; i3 < 3; ++i3) {
      tau[i3] = mk(0.0, 0.0);
#pragma unroll
      for (int v = 0; v < 3; ++v) tau[i3] = tau[i3] + m.C0eps[v][i3] * t[v];
      tau[3 + i3] = mk(0.0, 0.0);
    }
    double n[3];
    cx<double> eps[6];
    if (deriv_normal(g, x, y, z, n)) {
      gamma0_apply(m, n, tau, eps);
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) eps[c] = mk(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) e6[c * g.fs + idx] = eps[c];
    const double kx = x * g.kfx, ky = mode_of(y, g.ny) * g.kfy, kz = mode_of(z, g.nz) * g.kfz;
    if (FE) {
      const cx<double> fe = (m.fEc * (kx * kx + ky * ky + kz * kz)) * Hs;
      FE[idx] = accumulate ? FE[idx] + fe : fe;
    }
  }
}

// Non-negative doubles order like their bit patterns: a block's largest change
// is merged into *mx with an integer atomic max.
__device__ inline void atomic_max_nonneg(double* mx, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(mx), (unsigned long long)__double_as_longlong(v));
}

__global__ void k_el_zero(double* p) { *p = 0.0; }

}  // namespace

// One update's Green-operator step fused with its z transforms, per column
// of TX consecutive kx at one y: forward z-FFT of the six polarisation
// spectra (after their forward y pass), eps~ = Gamma0(n) tau~ per mode,
// inverse z-FFT times `scale`, in place.  The six fields of a column stay in
// registers between the transforms (radix-4 ends keep them at four values per
// field and thread); columns past nxh transform zeros and store nothing.
template <int N, int TX, int RE>
__global__ void __launch_bounds__((ColGeo<N, TX, RE>::THREADS))
k_el_zgamma(cx<double>* __restrict__ e6, Geo g, ModelK m, const cx<double>* twz, double scale) {
  using CG = ColGeo<N, TX, RE>;
  __shared__ cx<double> lds[N * CG::LD];
  __shared__ cx<double> twl[N];
  for (int j = threadIdx.x; j < N; j += CG::THREADS) twl[j] = twz[j];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int nbx = (g.nxh + TX - 1) / TX;
  const int xb = tile % nbx, y = tile / nbx;
  const uint32_t lstride = (uint32_t)(g.ny * g.P);
  // thread-derived indices, rebuilt at each phase from an opaque copy of the
  // thread index so that they (and the addresses made from them) are not held
  // across the per-mode solves
  struct Ix {
    int col, bf, x;
    uint32_t base;
    bool valid;
  };
  auto ix = [&]() {
    int tq = (int)threadIdx.x;
    asm volatile("" : "+v"(tq));
    Ix r;
    r.col = tq % TX;
    r.bf = tq / TX;
    r.x = xb * TX + r.col;
    r.valid = r.x < g.nxh;
    r.base = (uint32_t)(y * g.P + r.x);
    return r;
  };
  cx<double> a[6][CG::R0];
  {
    const Ix I = ix();
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int t = 0; t < CG::R0; ++t)
        a[c][t] = I.valid ? at32(e6 + c * g.fs, I.base + (I.bf + t * CG::TL) * lstride) : mk(0.0, 0.0);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const Ix I = ix();
    line_fft<double, N, -1, RE, true>(a[c], I.bf, twl, [&](int pos) -> cx<double>& { return lds[pos * CG::LD + I.col]; },
                                      true);
  }
  // the spectra are final here (the compiler would otherwise finish the last
  // butterflies inside the per-mode loop and hold their inputs as well)
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) pin(a[c][t]);
  {
    const Ix I = ix();
#pragma unroll
    for (int t = 0; t < CG::R0; ++t) {
      const int z = I.bf + t * CG::TL;
      double nv[3];
      cx<double> tau[6], eps[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) tau[c] = a[c][t];
      if (I.valid && deriv_normal(g, I.x, y, z, nv)) {
        gamma0_apply(m, nv, tau, eps);
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) eps[c] = mk(0.0, 0.0);
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        a[c][t] = scale * eps[c];
        pin(a[c][t]);
      }
      __builtin_amdgcn_sched_barrier(0);  // one mode at a time
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const Ix I = ix();
    line_fft<double, N, +1, RE, true>(a[c], I.bf, twl, [&](int pos) -> cx<double>& { return lds[pos * CG::LD + I.col]; },
                                      true);
    if (I.valid) {
#pragma unroll
      for (int t = 0; t < CG::R0; ++t) at32(e6 + c * g.fs, I.base + (I.bf + t * CG::TL) * lstride) = a[c][t];
    }
  }
}

// Real strain rows from the six inverse-transformed spectra (c2r of each row),
// written to r6 (pitch nx per row, field stride nx ny nz); with mx, the
// largest change of any component against the values r6 held before is
// merged into *mx.
template <int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_el_strain(const cx<double>* __restrict__ e6, double* __restrict__ r6, Geo g, const cx<double>* twN,
            const cx<double>* twM, double* mx) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<double> lds[RB * RG::LD];
  __shared__ double wmax[RG::THREADS / 64 + 1];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<double>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  double dmax = 0.0;
  for (int f = 0; f < 6; ++f) {
    cx<double> a[RG::R0];
    row_c2r<double, M, RB>(e6 + f * g.fs + rr * g.P, rvalid, a, bf, rbuf, twN, twM);
    if (rvalid) {
      cx<double>* dst = reinterpret_cast<cx<double>*>(r6 + ((long long)f * nrows + rr) * (2 * M));
#pragma unroll
      for (int t = 0; t < RG::R0; ++t) {
        if (mx) {
          const cx<double> old = dst[bf + t * RG::TL];
          dmax = fmax(dmax, fmax(fabs(a[t].re - old.re), fabs(a[t].im - old.im)));
        }
        dst[bf + t * RG::TL] = a[t];
      }
    }
  }
  if (mx) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = 0.0;
      for (int w = 0; w < (RG::THREADS + 63) / 64; ++w) b = fmax(b, wmax[w]);
      atomic_max_nonneg(mx, b);
    }
  }
}

// Eigenstrain of one point (diagonal) from theta_1..3.
__device__ inline void eigen_diag(const ModelK& m, double t0, double t1, double t2, double es[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) es[i] = t0 * m.eps[0][i] + t1 * m.eps[1][i] + t2 * m.eps[2][i];
}

// The c2r of the three order parameters of one row of T1 into et[3][R0]
// (pairs of consecutive x).
template <int M, int RB>
__device__ inline void row_eta3(const cx<double>* st, long long rb, bool rvalid, cx<double> (*et)[RowGeo<M, RB>::R0],
                                int bf, cx<double>* rbuf, const cx<double>* twN, const cx<double>* twM,
                                const Geo& g) {
  // unrolled (a loop over v would index et at run time and put it in scratch
  // memory), one transform at a time
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    row_c2r<double, M, RB>(st + (1 + v) * g.fs + rb, rvalid, et[v], bf, rbuf, twN, twM);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The per-point coefficients of the polarisation, once per solve: with
// d = eps_bar + eps_u - eps* and C(r) - C0 = (d11, d12, d44) in Voigt form,
//   tau_j = C0 eps*_j - d11 d_j - d12 (d_k + d_l)     (normal; k, l the other axes)
//         = A_j - d11 u_j - d12 (u_k + u_l),
//   A_j   = (C0 eps*)_j + d11 (eps*_j - eps_bar_j) + d12 (eps*_k + eps*_l - eps_bar_k - eps_bar_l),
//   tau_s = -2 d44 u_s                                 (shear, tensor components),
// so an update does no division.  Written as six real fields A_0, A_1, A_2,
// d11, d12, d44 in the layout of the real strain (pairs of consecutive x),
// from the c2r of the order parameters of T1.
template <int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_el_local(const cx<double>* __restrict__ st, double* __restrict__ lc6, Geo g, ModelK m, const cx<double>* twN,
           const cx<double>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<double> lds[RB * RG::LD];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<double>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  const long long npair = (long long)nrows * M;
  cx<double> th[3][RG::R0];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    row_c2r<double, M, RB>(st + (1 + v) * g.fs + rr * g.P, rvalid, th[v], bf, rbuf, twN, twM);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (!rvalid) return;
  cx<double>* out = reinterpret_cast<cx<double>*>(lc6) + rr * M;
#pragma unroll
  for (int t = 0; t < RG::R0; ++t) {
    double o[2][6];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double t0 = hfun(h ? th[0][t].im : th[0][t].re);
      const double t1 = hfun(h ? th[1][t].im : th[1][t].re);
      const double t2 = hfun(h ? th[2][t].im : th[2][t].re);
      const Cubic C = local_stiffness(m, t0 + t1 + t2);
      const double d11 = C.c11 - m.C0[0], d12 = C.c12 - m.C0[1], d44 = C.c44 - m.C0[2];
      double es[3];
      eigen_diag(m, t0, t1, t2, es);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int k = (j + 1) % 3, l = (j + 2) % 3;
        o[h][j] = m.C0[0] * es[j] + m.C0[1] * (es[k] + es[l]) + d11 * (es[j] - m.ebar[j]) +
                  d12 * (es[k] + es[l] - m.ebar[k] - m.ebar[l]);
      }
      o[h][3] = d11;
      o[h][4] = d12;
      o[h][5] = d44;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) out[f * npair + bf + t * RG::TL] = mk(o[0][f], o[1][f]);
  }
}

// Polarisation rows from the real strain r6 and the per-point coefficients
// lc6 (k_el_local), r2c of each of the six tensor components into e6.  Fields
// are addressed as a uniform base plus a 32-bit pair index.
template <int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_el_tau(const double* __restrict__ lc6, const double* __restrict__ r6, cx<double>* __restrict__ e6, Geo g,
         const cx<double>* twN, const cx<double>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<double> lds[RB * RG::LD];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<double>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  const long long rb = rr * g.P;
  const long long npair = (long long)nrows * M;
  const cx<double>* s6 = reinterpret_cast<const cx<double>*>(r6);
  const cx<double>* lc = reinterpret_cast<const cx<double>*>(lc6);
  const uint32_t q0 = (uint32_t)(rr * M) + bf;
  // rows past the end read row 0 (rr = 0; in bounds) and store nothing
  auto ld = [&](const cx<double>* f, uint32_t q) { return at32(f, q); };
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    const int k = c == 2 ? 0 : c + 1, l = c == 0 ? 2 : c - 1;
    cx<double> a[RG::R0];
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const uint32_t q = q0 + t * RG::TL;
      const cx<double> A = ld(lc + c * npair, q), d11 = ld(lc + 3 * npair, q), d12 = ld(lc + 4 * npair, q);
      const cx<double> uj = ld(s6 + c * npair, q), uk = ld(s6 + k * npair, q), ul = ld(s6 + l * npair, q);
      a[t] = mk(A.re - d11.re * uj.re - d12.re * (uk.re + ul.re), A.im - d11.im * uj.im - d12.im * (uk.im + ul.im));
      if (t % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // four points' loads in flight at a time
    }
    row_r2c<double, M, RB>(a, e6 + c * g.fs + rb, rvalid, bf, rbuf, twN, twM);
  }
#pragma unroll 1
  for (int c = 3; c < 6; ++c) {
    cx<double> a[RG::R0];
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const uint32_t q = q0 + t * RG::TL;
      const cx<double> d44 = ld(lc + 5 * npair, q), u = ld(s6 + c * npair, q);
      a[t] = mk(-2.0 * d44.re * u.re, -2.0 * d44.im * u.im);
    }
    row_r2c<double, M, RB>(a, e6 + c * g.fs + rb, rvalid, bf, rbuf, twN, twM);
  }
}

// Stress at one point from the order parameters' theta and the strain.
struct PointStress {
  double s[6];   // xx, yy, zz, yz, xz, xy
  double d[3];   // normal components of eps_bar + eps_u - eps*
  double e[3];   // shear tensor components of eps_u
};
__device__ inline PointStress point_stress(const ModelK& m, double t0, double t1, double t2, const double u[6]) {
  PointStress p;
  const Cubic C = local_stiffness(m, t0 + t1 + t2);
  double es[3];
  eigen_diag(m, t0, t1, t2, es);
#pragma unroll
  for (int i = 0; i < 3; ++i) p.d[i] = m.ebar[i] + u[i] - es[i];
  p.s[0] = C.c11 * p.d[0] + C.c12 * (p.d[1] + p.d[2]);
  p.s[1] = C.c11 * p.d[1] + C.c12 * (p.d[2] + p.d[0]);
  p.s[2] = C.c11 * p.d[2] + C.c12 * (p.d[0] + p.d[1]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    p.e[i] = u[3 + i];
    p.s[3 + i] = 2.0 * C.c44 * u[3 + i];
  }
  return p;
}

// Driving-force rows with the inhomogeneous elastic term:
// g_v = h'(eta_v) (chi(c) - sigma : eps*_v - sigma : dS : sigma / 2) + 2 w eta_v (1 - eta_v)(1 - 2 eta_v),
// r2c into el (3 fields).
template <int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_el_drive(const cx<double>* __restrict__ st, const double* __restrict__ r6, cx<double>* __restrict__ el, Geo g,
           ModelK m, const cx<double>* twN, const cx<double>* twM) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<double> lds[RB * RG::LD];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<double>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  const long long rb = rr * g.P;
  const long long npair = (long long)nrows * M;
  const cx<double>* s6 = reinterpret_cast<const cx<double>*>(r6) + rr * M;
  cx<double> chi[RG::R0];
  {
    cx<double> a[RG::R0];
    row_c2r<double, M, RB>(st + rb, rvalid, a, bf, rbuf, twN, twM);
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const double c0 = a[t].re, c1 = a[t].im;
      chi[t] = mk(m.W * ((c0 - m.cp) * (c0 - m.cp) - (c0 - m.cm) * (c0 - m.cm)),
                  m.W * ((c1 - m.cp) * (c1 - m.cp) - (c1 - m.cm) * (c1 - m.cm)));
    }
  }
  cx<double> et[3][RG::R0];
  row_eta3<M, RB>(st, rb, rvalid, et, bf, rbuf, twN, twM, g);
#pragma unroll
  for (int t = 0; t < RG::R0; ++t) {
    const int q = bf + t * RG::TL;
    cx<double> uu[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) uu[c] = rvalid ? s6[c * npair + q] : mk(0.0, 0.0);
    double gv[3][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double e[3], u[6];
#pragma unroll
      for (int v = 0; v < 3; ++v) e[v] = h ? et[v][t].im : et[v][t].re;
#pragma unroll
      for (int c = 0; c < 6; ++c) u[c] = h ? uu[c].im : uu[c].re;
      const PointStress p = point_stress(m, hfun(e[0]), hfun(e[1]), hfun(e[2]), u);
      const double* s = p.s;
      const double quad = m.dS[0] * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2]) +
                          2.0 * m.dS[1] * (s[0] * s[1] + s[1] * s[2] + s[2] * s[0]) +
                          m.dS[2] * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
      const double ch = h ? chi[t].im : chi[t].re;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double sev = s[0] * m.eps[v][0] + s[1] * m.eps[v][1] + s[2] * m.eps[v][2];
        const double ev = e[v];
        gv[v][h] = dhfun(ev) * (ch - sev - 0.5 * quad) + 2.0 * m.w * ev * (1.0 - ev) * (1.0 - 2.0 * ev);
      }
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) et[v][t] = mk(gv[v][0], gv[v][1]);
  }
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    row_r2c<double, M, RB>(et[v], el + v * g.fs + rb, rvalid, bf, rbuf, twN, twM);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Elastic energy density sums, 1/2 sigma : (eps_bar + eps_u - eps*) over the
// points of each block (rows of T1 for the order parameters, r6 the strain).
template <int M, int RB>
__global__ void __launch_bounds__((RowGeo<M, RB>::THREADS))
k_el_energy(const cx<double>* __restrict__ st, const double* __restrict__ r6, Geo g, ModelK m,
            const cx<double>* twN, const cx<double>* twM, double* partial) {
  using RG = RowGeo<M, RB>;
  __shared__ cx<double> lds[RB * RG::LD];
  __shared__ double sh[16];
  const int rl = threadIdx.x / RG::TL;
  const int bf = threadIdx.x % RG::TL;
  const int row = blockIdx.x * RB + rl;
  const int nrows = g.nz * g.ny;
  const bool rvalid = row < nrows;
  cx<double>* rbuf = lds + rl * RG::LD;
  const long long rr = rvalid ? row : 0;
  const long long npair = (long long)nrows * M;
  const cx<double>* s6 = reinterpret_cast<const cx<double>*>(r6) + rr * M;
  cx<double> et[3][RG::R0];
  row_eta3<M, RB>(st, rr * g.P, rvalid, et, bf, rbuf, twN, twM, g);
  double acc = 0.0;
  if (rvalid) {
#pragma unroll
    for (int t = 0; t < RG::R0; ++t) {
      const int q = bf + t * RG::TL;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double u[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const cx<double> e = s6[c * npair + q];
          u[c] = h ? e.im : e.re;
        }
        const PointStress p = point_stress(m, hfun(h ? et[0][t].im : et[0][t].re),
                                           hfun(h ? et[1][t].im : et[1][t].re),
                                           hfun(h ? et[2][t].im : et[2][t].re), u);
        acc += 0.5 * (p.s[0] * p.d[0] + p.s[1] * p.d[1] + p.s[2] * p.d[2]) +
               (p.s[3] * p.e[0] + p.s[4] * p.e[1] + p.s[5] * p.e[2]);
      }
    }
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

}  // namespace pf
