// Host-side check of the FFT building blocks used by the gfx950 kernels:
// compile-time plans, radix-2/3/4/5/6/7/8 DFTs, the Stockham butterfly index and
// twiddle arithmetic, and the real<->half-complex packing.  Runs each line
// length through the plan's passes on the CPU and compares with a naive DFT
// evaluated in long double.  Prints one line per case: "<case> <n> <relerr>".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2609_36100_amd/csrc/pf_fft.hpp"

using namespace pf;
typedef cx<double> C;

static std::vector<C> table(int n) {
  std::vector<C> t(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n; ++j) {
    long double a = 2.0L * pi * j / n;
    t[j] = mk<double>((double)cosl(a), (double)-sinl(a));
  }
  return t;
}

template <int S>
static void stockham(std::vector<C>& x, const std::vector<C>& tw) {
  const int n = (int)x.size();
  Plan P = plan(n);
  std::vector<C> y(n);
  int p = 1;
  for (int q = 0; q < P.np; ++q) {
    const int r = P.r[q];
    for (int b = 0; b < n / r; ++b)
      butterfly_rt<S, double>(r, n, p, b, tw.data(), [&](int i) -> C& { return x[i]; },
                              [&](int i) -> C& { return y[i]; });
    x.swap(y);
    p *= r;
  }
}

static double naive_err(const std::vector<C>& in, const std::vector<C>& out, int S) {
  const int n = (int)in.size();
  const long double pi = 3.141592653589793238462643383279502884L;
  long double num = 0, den = 0;
  for (int k = 0; k < n; ++k) {
    long double re = 0, im = 0;
    for (int j = 0; j < n; ++j) {
      long double a = S * 2.0L * pi * (long double)((long long)j * k % n) / n;
      re += in[j].re * cosl(a) - in[j].im * sinl(a);
      im += in[j].re * sinl(a) + in[j].im * cosl(a);
    }
    num += (re - out[k].re) * (re - out[k].re) + (im - out[k].im) * (im - out[k].im);
    den += re * re + im * im;
  }
  return (double)sqrtl(num / den);
}

int main() {
  const int sizes[] = {4,  7,  8,   12,  16,  20,  24,  28,  32,  36,  40,  48,  56,  64,  72,  80, 84,
                       96, 128, 160, 168, 192, 252, 256, 320, 336, 384, 504, 512};
  srand(7);
  int fails = 0;
  for (int n : sizes) {
    Plan P = plan(n);
    if (!P.ok || P.r[0] != P.r[P.np - 1]) {
      printf("plan_bad %d 1\n", n);
      ++fails;
      continue;
    }
    int prod = 1;
    for (int q = 0; q < P.np; ++q) prod *= P.r[q];
    if (prod != n) {
      printf("plan_prod %d 1\n", n);
      ++fails;
    }
    std::vector<C> x(n);
    for (auto& v : x) v = mk<double>(rand() / (double)RAND_MAX - 0.5, rand() / (double)RAND_MAX - 0.5);
    auto tw = table(n);
    std::vector<C> f = x;
    stockham<-1>(f, tw);
    printf("fwd %d %.3e\n", n, naive_err(x, f, -1));
    std::vector<C> g = x;
    stockham<+1>(g, tw);
    printf("inv %d %.3e\n", n, naive_err(x, g, +1));
  }
  // real transforms of length N = 2M via packed M-point complex FFTs
  const int rsizes[] = {8, 16, 24, 32, 40, 48, 56, 64, 72, 96, 128, 168, 192, 256, 336, 504, 512};
  for (int N : rsizes) {
    const int M = N / 2;
    std::vector<double> xr(N);
    for (auto& v : xr) v = rand() / (double)RAND_MAX - 0.5;
    auto twN = table(N), twM = table(M);
    std::vector<C> z(M);
    for (int j = 0; j < M; ++j) z[j] = mk(xr[2 * j], xr[2 * j + 1]);
    stockham<-1>(z, twM);
    std::vector<C> X(M + 1);
    for (int k = 0; k < M; ++k) X[k] = r2c_post(z[k], z[(M - k) % M], twN[k]);
    X[M] = mk(z[0].re - z[0].im, 0.0);
    std::vector<C> xin(N), Xfull(N);
    for (int j = 0; j < N; ++j) xin[j] = mk(xr[j], 0.0);
    for (int k = 0; k <= M; ++k) Xfull[k] = X[k];
    for (int k = M + 1; k < N; ++k) Xfull[k] = conj(X[N - k]);
    printf("r2c %d %.3e\n", N, naive_err(xin, Xfull, -1));
    // c2r back (unnormalised full-spectrum sum) must give N * x
    std::vector<C> Z(M);
    for (int k = 0; k < M; ++k) {
      C xk = X[k], xmk = X[M - k];
      if (k == 0) { xk.im = 0; xmk.im = 0; }
      Z[k] = c2r_pre(xk, xmk, twN[k]);
    }
    stockham<+1>(Z, twM);
    double num = 0, den = 0;
    for (int j = 0; j < M; ++j) {
      double a = Z[j].re / N - xr[2 * j], b = Z[j].im / N - xr[2 * j + 1];
      num += a * a + b * b;
      den += xr[2 * j] * xr[2 * j] + xr[2 * j + 1] * xr[2 * j + 1];
    }
    printf("c2r %d %.3e\n", N, std::sqrt(num / den));
  }
  return fails;
}
