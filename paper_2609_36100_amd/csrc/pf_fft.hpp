// Radix-2/3/4/5/6/7/8 Stockham FFT building blocks for gfx950.
//
// The paper moves every field between real and reciprocal space with 3D FFTs
// (Methods, "MEUMAPPS C++ and the MEUMAPPS-SS application"; "Scalable,
// performance-portable fast Fourier transforms": 1D transforms plus data
// reshapes).  Here a 3D transform is three HBM-streaming passes, one per axis;
// this header holds the per-line pieces every pass shares:
//
//  * cx<T>          interleaved complex value (T = float or double);
//  * dft<R,S>()     in-register R-point DFT, R in {2,3,4,5,8}, S = -1 forward
//                   (exp(-i...)), S = +1 inverse (unnormalised);
//  * Plan / plan()  compile-time radix sequence for a line of length n whose
//                   first and last radix are equal, so that a thread owns the
//                   same line positions before the first pass and after the
//                   last pass (inputs and outputs stay in registers across
//                   fused transforms);
//  * butterfly()    one Stockham autosort butterfly: reads x[b + t n/r],
//                   twiddles by w_{p r}^{t k} (k = b mod p), applies the
//                   r-point DFT and writes y[(b-k) r + k + t p];
//  * r2c/c2r helpers that turn an n-point real transform into an n/2-point
//                   complex one (even/odd packing).
//
// Everything here is __host__ __device__ so that the index arithmetic can be
// exercised on the CPU as well.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pf {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) {
  cx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T>
__host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
template <typename T>
__host__ __device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
// multiply by S*i  (S = +1 or -1)
template <int S, typename T>
__host__ __device__ inline cx<T> mul_si(cx<T> a) {
  return S > 0 ? mk(-a.im, a.re) : mk(a.im, -a.re);
}

// ---- small DFTs ---------------------------------------------------------
// X_k = sum_n a_n exp(S 2 pi i n k / R), written back into a[0..R-1].

template <int R, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<2, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    cx<T> t = a[0] - a[1];
    a[0] = a[0] + a[1];
    a[1] = t;
  }
};

template <int S, typename T>
struct Dft<4, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    cx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
    cx<T> t2 = a[1] + a[3], t3 = mul_si<S>(a[1] - a[3]);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  }
};

template <int S, typename T>
struct Dft<8, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    // split into even / odd samples, two 4-point DFTs, combine with w_8^{S k}
    cx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cx<T> o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, S, T>::run(e);
    Dft<4, S, T>::run(o);
    const T h = (T)0.70710678118654752440084436210484903928;  // 1/sqrt(2)
    cx<T> w1 = mk<T>(h, (T)S * h);       // exp(S i pi/4)
    cx<T> w3 = mk<T>(-h, (T)S * h);      // exp(S i 3pi/4)
    cx<T> o1 = cmul(o[1], w1);
    cx<T> o2 = mul_si<S>(o[2]);
    cx<T> o3 = cmul(o[3], w3);
    a[0] = e[0] + o[0];
    a[4] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[5] = e[1] - o1;
    a[2] = e[2] + o2;
    a[6] = e[2] - o2;
    a[3] = e[3] + o3;
    a[7] = e[3] - o3;
  }
};

template <int S, typename T>
struct Dft<3, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    const T s3 = (T)0.86602540378443864676372317075293618347;  // sin(2 pi/3)
    cx<T> t = a[1] + a[2];
    cx<T> m = a[0] - (T)0.5 * t;
    cx<T> d = mul_si<S>(s3 * (a[1] - a[2]));
    a[0] = a[0] + t;
    a[1] = m + d;
    a[2] = m - d;
  }
};

template <int S, typename T>
struct Dft<5, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    const T c1 = (T)0.30901699437494742410229341718281905886;   // cos(2 pi/5)
    const T c2 = (T)-0.80901699437494742410229341718281905886;  // cos(4 pi/5)
    const T s1 = (T)0.95105651629515357211643933337938214340;   // sin(2 pi/5)
    const T s2 = (T)0.58778525229247312916870595463907276860;   // sin(4 pi/5)
    cx<T> p1 = a[1] + a[4], m1 = a[1] - a[4];
    cx<T> p2 = a[2] + a[3], m2 = a[2] - a[3];
    cx<T> x0 = a[0];
    cx<T> r1 = x0 + c1 * p1 + c2 * p2;
    cx<T> r2 = x0 + c2 * p1 + c1 * p2;
    cx<T> i1 = mul_si<S>(s1 * m1 + s2 * m2);
    cx<T> i2 = mul_si<S>(s2 * m1 - s1 * m2);
    a[0] = x0 + p1 + p2;
    a[1] = r1 + i1;
    a[4] = r1 - i1;
    a[2] = r2 + i2;
    a[3] = r2 - i2;
  }
};

// Six points as two 3-point DFTs of the even and odd samples combined with
// w_6^{S k}: X_k = E_{k mod 3} + w_6^{S k} O_{k mod 3}.
template <int S, typename T>
struct Dft<6, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    cx<T> e[3] = {a[0], a[2], a[4]};
    cx<T> o[3] = {a[1], a[3], a[5]};
    Dft<3, S, T>::run(e);
    Dft<3, S, T>::run(o);
    const T s3 = (T)0.86602540378443864676372317075293618347;  // sin(pi/3)
    const cx<T> o1 = cmul(o[1], mk<T>((T)0.5, (T)S * s3));     // exp(S i pi/3)
    const cx<T> o2 = cmul(o[2], mk<T>((T)-0.5, (T)S * s3));    // exp(S i 2pi/3)
    a[0] = e[0] + o[0];
    a[3] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[4] = e[1] - o1;
    a[2] = e[2] + o2;
    a[5] = e[2] - o2;
  }
};

// Seven points: pair n with 7 - n, X_k = r_k + S i q_k and X_{7-k} = r_k - S i q_k
// with r_k = a_0 + sum_j cos(2 pi j k/7) (a_j + a_{7-j}) and
// q_k = sum_j sin(2 pi j k/7) (a_j - a_{7-j}), j = 1..3.
template <int S, typename T>
struct Dft<7, S, T> {
  __host__ __device__ static inline void run(cx<T>* a) {
    const T c1 = (T)0.62348980185873353052500488400423981063;   // cos(2 pi/7)
    const T c2 = (T)-0.22252093395631440428890256449679475947;  // cos(4 pi/7)
    const T c3 = (T)-0.90096886790241912623610231950744505117;  // cos(6 pi/7)
    const T s1 = (T)0.78183148246802980870844452667405775023;   // sin(2 pi/7)
    const T s2 = (T)0.97492791218182360701813168299393121723;   // sin(4 pi/7)
    const T s3 = (T)0.43388373911755812047576833284835875461;   // sin(6 pi/7)
    cx<T> p1 = a[1] + a[6], m1 = a[1] - a[6];
    cx<T> p2 = a[2] + a[5], m2 = a[2] - a[5];
    cx<T> p3 = a[3] + a[4], m3 = a[3] - a[4];
    cx<T> x0 = a[0];
    cx<T> r1 = x0 + c1 * p1 + c2 * p2 + c3 * p3;
    cx<T> r2 = x0 + c2 * p1 + c3 * p2 + c1 * p3;
    cx<T> r3 = x0 + c3 * p1 + c1 * p2 + c2 * p3;
    cx<T> i1 = mul_si<S>(s1 * m1 + s2 * m2 + s3 * m3);
    cx<T> i2 = mul_si<S>(s2 * m1 - s3 * m2 - s1 * m3);
    cx<T> i3 = mul_si<S>(s3 * m1 - s1 * m2 + s2 * m3);
    a[0] = x0 + p1 + p2 + p3;
    a[1] = r1 + i1;
    a[6] = r1 - i1;
    a[2] = r2 + i2;
    a[5] = r2 - i2;
    a[3] = r3 + i3;
    a[4] = r3 - i3;
  }
};

template <int R, int S, typename T>
__host__ __device__ inline void dft(cx<T>* a) {
  Dft<R, S, T>::run(a);
}

// ---- plans ----------------------------------------------------------------
struct Plan {
  int n;       // line length
  int np;      // number of passes
  int r[8];    // radices, r[0] == r[np-1]
  int ok;      // 1 when n is supported
};

// Radix sequence for a line of length n whose first and last radix (the "end"
// radix, at most remax) are equal.  Middle factors are taken greedily from
// {8, 4, 2, 3, 5, 7}.  ok = 0 when n has no such factorisation.
__host__ __device__ constexpr Plan plan(int n, int remax = 8) {
  Plan P{n, 0, {0, 0, 0, 0, 0, 0, 0, 0}, 0};
  if (n == 3 || n == 5 || n == 7 || ((n == 2 || n == 4 || n == 8) && n <= remax)) {
    P.np = 1;
    P.r[0] = n;
    P.ok = 1;
    return P;
  }
  int re = (remax >= 8 && n % 64 == 0) ? 8 : (remax >= 4 && n % 16 == 0) ? 4 : (n % 4 == 0) ? 2 : 0;
  // where radix 2 would be the alternative: radix-6 ends when 36 | n, else
  // radix-3 ends when 9 | n (504 = 6 * 14 * 6: four passes instead of six and a
  // third of the threads per line)
  if (re == 2 && remax >= 6 && n % 36 == 0)
    re = 6;
  else if (re == 2 && remax >= 3 && n % 9 == 0)
    re = 3;
  if (re == 0) return P;
  int m = n / (re * re);
  int mid[6] = {0, 0, 0, 0, 0, 0};
  int nm = 0;
  while (m % 8 == 0 && nm < 6) { mid[nm++] = 8; m /= 8; }
  while (m % 4 == 0 && nm < 6) { mid[nm++] = 4; m /= 4; }
  while (m % 2 == 0 && nm < 6) { mid[nm++] = 2; m /= 2; }
  while (m % 3 == 0 && nm < 6) { mid[nm++] = 3; m /= 3; }
  while (m % 5 == 0 && nm < 6) { mid[nm++] = 5; m /= 5; }
  while (m % 7 == 0 && nm < 6) { mid[nm++] = 7; m /= 7; }
  if (m != 1) return P;
  P.r[0] = re;
  for (int i = 0; i < nm; ++i) P.r[1 + i] = mid[i];
  P.r[1 + nm] = re;
  P.np = nm + 2;
  P.ok = 1;
  return P;
}

// Threads cooperating on one line: one butterfly each in the first/last pass.
__host__ __device__ constexpr int line_threads(int n, int remax = 8) { return n / plan(n, remax).r[0]; }

// Largest number of values a thread holds in any pass (registers per line).
__host__ __device__ constexpr int line_regs(int n) {
  Plan P = plan(n);
  int T = n / P.r[0];
  int mx = P.r[0];
  for (int q = 0; q < P.np; ++q) {
    int nb = n / P.r[q];
    int per = (nb + T - 1) / T;
    if (per * P.r[q] > mx) mx = per * P.r[q];
  }
  return mx;
}

// Twiddle w_n^{S j} from a table of w_n^{-j} = exp(-2 pi i j / n), j < n.
template <int S, typename T>
__host__ __device__ inline cx<T> twiddle(const cx<T>* tab, int j) {
  cx<T> w = tab[j];
  return S < 0 ? w : conj(w);
}

// One Stockham butterfly of radix R for line length n, at stride product p.
// `in(pos)` / `out(pos)` are accessors returning references.
template <int R, int S, typename T, class In, class Out>
__host__ __device__ inline void butterfly(int n, int p, int b, const cx<T>* tw, In in, Out out) {
  cx<T> a[R];
  const int nb = n / R;
  const int k = b % p;
#pragma unroll
  for (int t = 0; t < R; ++t) a[t] = in(b + t * nb);
  if (p > 1) {
    const int step = n / (p * R);  // w_{pR}^{t k} = w_n^{t k step}
#pragma unroll
    for (int t = 1; t < R; ++t) a[t] = cmul(a[t], twiddle<S>(tw, t * k * step));
  }
  dft<R, S>(a);
#pragma unroll
  for (int t = 0; t < R; ++t) out((b - k) * R + k + t * p) = a[t];
}

// Run-time radix dispatch of butterfly() (host reference path and tests).
template <int S, typename T, class In, class Out>
__host__ __device__ inline void butterfly_rt(int R, int n, int p, int b, const cx<T>* tw, In in, Out out) {
  switch (R) {
    case 2: butterfly<2, S, T>(n, p, b, tw, in, out); break;
    case 3: butterfly<3, S, T>(n, p, b, tw, in, out); break;
    case 4: butterfly<4, S, T>(n, p, b, tw, in, out); break;
    case 5: butterfly<5, S, T>(n, p, b, tw, in, out); break;
    case 6: butterfly<6, S, T>(n, p, b, tw, in, out); break;
    case 7: butterfly<7, S, T>(n, p, b, tw, in, out); break;
    case 8: butterfly<8, S, T>(n, p, b, tw, in, out); break;
    default: break;
  }
}

// ---- real <-> half-complex packing --------------------------------------
// A real line x of even length N is packed as z_j = x_{2j} + i x_{2j+1}
// (M = N/2 complex values).  With Z = FFT_M(z) (unnormalised, forward):
//   X_k = E_k + w_N^{-k} O_k,  E_k = (Z_k + conj Z_{M-k})/2,
//   O_k = (Z_k - conj Z_{M-k})/(2i),  k = 0..M  (Z_M = Z_0).
// Inverse (c2r, unnormalised full-spectrum sum with X_{N-k} = conj X_k):
//   Z'_k = (X_k + conj X_{M-k}) + i w_N^{+k} (X_k - conj X_{M-k}),
// and the unnormalised inverse M-point FFT of Z' gives x_{2j} + i x_{2j+1}.
// Imaginary parts of X_0 and X_M are dropped (a real line has none).

// X_k from Z_k and Z_{M-k}; wk = w_N^{-k} (table value).
template <typename T>
__host__ __device__ inline cx<T> r2c_post(cx<T> zk, cx<T> zmk, cx<T> wk) {
  cx<T> zc = conj(zmk);
  cx<T> e = (T)0.5 * (zk + zc);
  cx<T> d = (T)0.5 * (zk - zc);
  cx<T> o = mk(d.im, -d.re);  // d / i
  return e + cmul(wk, o);
}

// Z'_k from X_k and X_{M-k}; wk = w_N^{-k} (table value, conjugated here).
template <typename T>
__host__ __device__ inline cx<T> c2r_pre(cx<T> xk, cx<T> xmk, cx<T> wk) {
  cx<T> xc = conj(xmk);
  cx<T> s = xk + xc;
  cx<T> d = cmulc(xk - xc, wk);  // (X_k - conj X_{M-k}) w_N^{+k}
  return s + mul_si<1>(d);
}

}  // namespace pf
