// Fourier neural operator surrogate: BF16 MFMA training and inference on gfx950.
//
// The learned form beside the method: a classic FNO maps the state
// (c, eta_1..3) on an n^3 grid to the increment of the state a fixed time
// later.  Architecture (width w, modes m, L layers, hidden h):
//   v0 = x W_lift + b_lift;  v_{l+1} = act(K_l v_l + v_l W_l + b_l);
//   out = GELU(v_L P1 + c1) P2 + c2,
//   K_l v = inverse truncated DFT( R_l . forward truncated DFT(v) ),
// retained modes kx < m and ky, kz in the m lowest positive and negative
// frequencies.  Activations are channel-last [point][channel] BF16.
//
// Dense contractions run on MFMA (gfx950 v_mfma_f32_32x32x16_bf16, FP32 accumulate):
//  * channel mixing (lift, W_l, P1, P2 and their data gradients) as
//    [points x K] x [K x N] GEMMs;
//  * every truncated-DFT stage as a small constant matrix G times batched
//    activation blocks, Out_b = G X_b, with layouts chosen so each stage is a
//    plain strided GEMM (and its backward the same kernel with G^T).
// The per-mode complex w x w mixing and the weight-gradient reductions over
// points run on FP32 vector ALUs.  Adam updates FP32 master weights and
// refreshes the BF16 working copies.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pf.h"
#include "pf_context.hpp"

namespace {

typedef unsigned short u16;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// gfx950's 32 x 32 x 16 BF16 MFMA (FP32 accumulate).  Lane l holds row l % 32
// of A and column l % 32 of B at k = 8 (l / 32) .. 8 (l / 32) + 7; the
// accumulator layout is that of every 32 x 32 MFMA (lane l, element i: row
// 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32).
__device__ inline f32x16 mfma16(bf16x4 a_lo, bf16x4 a_hi, bf16x4 b_lo, bf16x4 b_hi, f32x16 acc) {
  const s16x8 a = {a_lo[0], a_lo[1], a_lo[2], a_lo[3], a_hi[0], a_hi[1], a_hi[2], a_hi[3]};
  const s16x8 b = {b_lo[0], b_lo[1], b_lo[2], b_lo[3], b_hi[0], b_hi[1], b_hi[2], b_hi[3]};
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc,
                                                 0, 0, 0);
}

__host__ __device__ inline u16 f2bf(float f) {
  unsigned int u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (u16)(u >> 16);
}
__host__ __device__ inline float bf2f(u16 h) {
  unsigned int u = ((unsigned int)h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

__device__ inline float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_g(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__device__ inline bf16x4 ld4(const u16* p) { return *reinterpret_cast<const bf16x4*>(p); }

// A second contraction along the x lines that a channel-mixing GEMM can carry:
// for point p = line * R + x, adds sum_k G[x][k] X[line * xbs + k * ldx + n]
// (the truncated-DFT x stage whose result the GEMM would otherwise read back
// as a residual).  G row-major R x K (K % 4 == 0, zero beyond K); R % 32 == 0
// so that a wave's 32 points lie in one line.  G == nullptr: none.
struct LineTerm {
  const u16* G = nullptr;
  int K = 0, R = 0;
  const u16* X = nullptr;
  long long xbs = 0;
  int ldx = 0;
};

// ---- channel-mixing GEMM: Out[p][n] = epi(sum_k In[p][k] Bt[n][k] [+ line term]) ----
// K % 4 == 0 (zero beyond K), P % 128 == 0, N <= 32 * NT.  Epilogue: + bias[n] + resid[p][n],
// times GELU'(gpre[p][n]) (a data gradient through the activation), stores any
// of: f32 result, bf16 pre-activation, bf16 GELU(pre).
template <int NT>
__global__ void __launch_bounds__(256)
k_cm_gemm(const u16* __restrict__ In, int ldin, int K, const u16* __restrict__ Bt, int N,
          const float* __restrict__ bias, const float* __restrict__ resid, int ldres, float* __restrict__ outf,
          u16* __restrict__ outpre, u16* __restrict__ outact, int ldout, int accumulate, LineTerm lt,
          const u16* __restrict__ gpre) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * 32;
  const int lr = lane & 31, lg = lane >> 5;
  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
  for (int kk = 0; kk < K; kk += 16) {
    // K % 4 == 0: each 4-wide half of a lane's 8 values is all in or all out
    const int kb = kk + lg * 8;
    const bool in0 = kb < K, in1 = kb + 4 < K;
    bf16x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
    if (in0) a0 = ld4(In + (p0 + lr) * ldin + kb);
    if (in1) a1 = ld4(In + (p0 + lr) * ldin + kb + 4);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 32 + lr;
      bf16x4 b0 = {0, 0, 0, 0}, b1 = {0, 0, 0, 0};
      if (n < N && in0) b0 = ld4(Bt + (long long)n * K + kb);
      if (n < N && in1) b1 = ld4(Bt + (long long)n * K + kb + 4);
      acc[t] = mfma16(a0, a1, b0, b1, acc[t]);
    }
  }
  if (lt.G) {
    const long long line = p0 / lt.R;
    const int x = (int)(p0 % lt.R) + lr;
    const u16* Xb = lt.X + line * lt.xbs;
    for (int kk = 0; kk < lt.K; kk += 16) {
      const int kb = kk + lg * 8;
      const bool in0 = kb < lt.K, in1 = kb + 4 < lt.K;
      bf16x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
      if (in0) a0 = ld4(lt.G + (long long)x * lt.K + kb);
      if (in1) a1 = ld4(lt.G + (long long)x * lt.K + kb + 4);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = t * 32 + lr;
        bf16x4 b0 = {0, 0, 0, 0}, b1 = {0, 0, 0, 0};
        if (n < N && in0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) b0[j] = (short)Xb[(long long)(kb + j) * lt.ldx + n];
        }
        if (n < N && in1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) b1[j] = (short)Xb[(long long)(kb + 4 + j) * lt.ldx + n];
        }
        acc[t] = mfma16(a0, a1, b0, b1, acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 32 + lr;
    if (col >= N) continue;
    const float bb = bias ? bias[col] : 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const long long row = p0 + 8 * (i >> 2) + 4 * lg + (i & 3);
      float v = acc[t][i] + bb;
      if (resid) v += resid[row * ldres + col];
      const long long o = row * ldout + col;
      if (gpre) v *= gelu_g(bf2f(gpre[o]));
      if (outf) outf[o] = accumulate ? outf[o] + v : v;
      if (outpre) outpre[o] = f2bf(v);
      if (outact) outact[o] = f2bf(gelu_f(v));
    }
  }
}

// ---- small-matrix GEMM: Out_b[r][n] = sum_k G[r][k] X_b[k][n] ---------------
// G row-major R x K (K % 4 == 0, zero beyond K), X_b rows of stride ldx,
// batch stride xbs.
// Each wave owns 32 columns and 4 row tiles (128 rows); blockIdx.z picks the
// 128-row band, so stages with many rows (the inverse stages: 2n rows) spread
// over more waves.  A block's four waves cover wpb column groups of
// `bpb = 4 / wpb` batches (wpb = 1 for the 32-column x stages, so no wave of a
// block idles there).
__global__ void __launch_bounds__(256)
k_lm_gemm(const u16* __restrict__ G, int R, int K, const u16* __restrict__ X, long long xbs, int ldx, int Nc,
          float* __restrict__ outf, u16* __restrict__ outb, long long obs, int ldo, int accumulate, int wpb,
          long long batches) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 31, lg = lane >> 5;
  const long long b = (long long)blockIdx.y * (4 / wpb) + wave / wpb;
  if (b >= batches) return;  // no block-level synchronisation in this kernel
  const int n = (blockIdx.x * wpb + wave % wpb) * 32 + lr;
  const bool valid = n < Nc;
  const u16* Xb = X + b * xbs;
  {
    const int r0 = blockIdx.z * 128;
    f32x16 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
    for (int kk = 0; kk < K; kk += 16) {
      const int kb = kk + lg * 8;
      const bool in0 = kb < K, in1 = kb + 4 < K;  // K % 4 == 0
      bf16x4 b0 = {0, 0, 0, 0}, b1 = {0, 0, 0, 0};
      if (valid && in0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) b0[j] = (short)Xb[(long long)(kb + j) * ldx + n];
      }
      if (valid && in1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) b1[j] = (short)Xb[(long long)(kb + 4 + j) * ldx + n];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = r0 + t * 32 + lr;
        if (r0 + t * 32 < R) {
          bf16x4 a0 = {0, 0, 0, 0}, a1 = {0, 0, 0, 0};
          if (r < R && in0) a0 = ld4(G + (long long)r * K + kb);
          if (r < R && in1) a1 = ld4(G + (long long)r * K + kb + 4);
          acc[t] = mfma16(a0, a1, b0, b1, acc[t]);
        }
      }
    }
    if (valid) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int row = r0 + t * 32 + 8 * (i >> 2) + 4 * lg + (i & 3);
          if (row >= R) continue;
          const long long o = b * obs + (long long)row * ldo + n;
          const float v = acc[t][i];
          if (outf) outf[o] = accumulate ? outf[o] + v : v;
          if (outb) outb[o] = f2bf(accumulate ? bf2f(outb[o]) + v : v);
        }
    }
  }
}

// ---- per-mode complex mixing (FP32) -------------------------------------------
// S, T: [2][modes][w] (real block, imaginary block); R: [modes][w][w] (in, out).
// `batches` spectra one after another (stride 2 modes w), the same weights.
__global__ void __launch_bounds__(256)
k_mix_fwd(const float* __restrict__ S, const u16* __restrict__ Rr, const u16* __restrict__ Ri, float* __restrict__ T,
          int modes, int w, u16* __restrict__ Tb, int batches) {
  const long long gid = blockIdx.x * 256LL + threadIdx.x;
  const long long mo = (long long)modes * w;
  if (gid >= mo * batches) return;
  const long long bo = (gid / mo) * 2 * mo;  // this spectrum's offset
  S += bo;
  T += bo;
  Tb += bo;
  const long long id = gid % mo;
  const long long md = id / w;
  const int o = (int)(id % w);
  float tr = 0.f, ti = 0.f;
  for (int i = 0; i < w; ++i) {
    const float sr = S[md * w + i], si = S[mo + md * w + i];
    const float rr = bf2f(Rr[(md * w + i) * w + o]), ri = bf2f(Ri[(md * w + i) * w + o]);
    tr += rr * sr - ri * si;
    ti += rr * si + ri * sr;
  }
  T[md * w + o] = tr;
  T[mo + md * w + o] = ti;
  Tb[md * w + o] = f2bf(tr);
  Tb[mo + md * w + o] = f2bf(ti);
}

__global__ void __launch_bounds__(256)
k_mix_bwd_data(const float* __restrict__ dT, const u16* __restrict__ Rr, const u16* __restrict__ Ri,
               u16* __restrict__ dSb, int modes, int w) {
  const long long id = blockIdx.x * 256LL + threadIdx.x;
  if (id >= (long long)modes * w) return;
  const long long md = id / w;
  const int i = (int)(id % w);
  const long long mo = (long long)modes * w;
  float sr = 0.f, si = 0.f;
  for (int o = 0; o < w; ++o) {
    const float tr = dT[md * w + o], ti = dT[mo + md * w + o];
    const float rr = bf2f(Rr[(md * w + i) * w + o]), ri = bf2f(Ri[(md * w + i) * w + o]);
    sr += rr * tr + ri * ti;
    si += rr * ti - ri * tr;
  }
  dSb[md * w + i] = f2bf(sr);
  dSb[mo + md * w + i] = f2bf(si);
}

__global__ void __launch_bounds__(256)
k_mix_bwd_w(const float* __restrict__ S, const float* __restrict__ dT, float* __restrict__ gRr,
            float* __restrict__ gRi, int modes, int w) {
  const long long id = blockIdx.x * 256LL + threadIdx.x;
  if (id >= (long long)modes * w * w) return;
  const long long md = id / (w * w);
  const int i = (int)((id / w) % w), o = (int)(id % w);
  const long long mo = (long long)modes * w;
  const float sr = S[md * w + i], si = S[mo + md * w + i];
  const float tr = dT[md * w + o], ti = dT[mo + md * w + o];
  gRr[id] += sr * tr + si * ti;
  gRi[id] += sr * ti - si * tr;
}

// ---- weight gradients on MFMA: G[k][n] += sum_p A[p][k] D[p][n], gb[n] += sum_p D[p][n] ----
// The reduction runs over points, which are the slow index of both operands,
// so each block stages WG_PTS points of A (bf16) and D (f32, rounded to bf16)
// transposed into LDS ([channel][point], padded rows) and every wave feeds
// 32 of those points to the 32 x 32 x 16 MFMA for up to four 32 x 32
// output tiles [t0, t0 + 4) of the ceil(K/32) x ceil(N/32) tile grid.  The
// four waves' tiles are summed in LDS and each block writes one partial set
// part[block * KN + k * N + n] (KN = (K + 1) * N; row k = K holds the bias
// sums, written when t0 == 0); k_sum_partials adds the sets.  Requires lda % 4 == 0, K <= lda,
// channels K .. 4 ceil(K/4) of A zero, K, N <= 128, chunk % WG_PTS == 0.
constexpr int WG_PTS = 128;
constexpr int WG_LD = WG_PTS + 4;  // bf16 row pitch: 264 B rows keep the 8-byte MFMA reads spread over banks

__global__ void __launch_bounds__(256)
k_wgrad_mfma(const u16* __restrict__ A, int lda, int K, const float* __restrict__ D, int ldd, int N, long long P,
             int chunk, int t0, float* __restrict__ part) {
  // one buffer: the staged operands LA [k][p] and LD [n][p], reused at the end
  // for the cross-wave sum of the partial tiles (4 waves x 4 tiles x 1024 floats)
  __shared__ __attribute__((aligned(16))) u16 smem[2 * 128 * WG_LD];
  u16* LA = smem;
  u16* LD = smem + 128 * WG_LD;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 31, lg = lane >> 5;
  const int Nt = (N + 31) / 32;
  const int ntiles = min(4, ((K + 31) / 32) * Nt - t0);
  const int KN = (K + 1) * N;
  const int Kq = (K + 3) / 4;  // 4-channel groups of A staged per point
  for (int e = tid; e < 128 * WG_LD; e += 256) LA[e] = 0, LD[e] = 0;
  f32x16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
  float bsum = 0.f;  // bias sum of channel n = tid (tid < N)
  const long long pb = (long long)blockIdx.x * chunk;
  const long long pe = pb + chunk < P ? pb + chunk : P;
  for (long long p0 = pb; p0 < pe; p0 += WG_PTS) {
    __syncthreads();
    for (int e = tid; e < WG_PTS * Kq; e += 256) {
      const int pp = e / Kq, kg = e % Kq;
      const bf16x4 v = ld4(A + (p0 + pp) * lda + 4 * kg);
#pragma unroll
      for (int j = 0; j < 4; ++j) LA[(4 * kg + j) * WG_LD + pp] = (u16)v[j];
    }
    for (int e = tid; e < WG_PTS * N; e += 256) {
      const int pp = e / N, nn = e % N;
      LD[nn * WG_LD + pp] = f2bf(D[(p0 + pp) * ldd + nn]);
    }
    __syncthreads();
    if (tid < N) {
      float sacc = 0.f;
      for (int pp = 0; pp < WG_PTS; pp += 4) {
        const bf16x4 v = *reinterpret_cast<const bf16x4*>(LD + tid * WG_LD + pp);
        sacc += (bf2f((u16)v[0]) + bf2f((u16)v[1])) + (bf2f((u16)v[2]) + bf2f((u16)v[3]));
      }
      bsum += sacc;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= ntiles) break;
      const int tile = t0 + t, kt = tile / Nt, nt = tile % Nt;
      const u16* ra = LA + (kt * 32 + lr) * WG_LD + wave * 32 + lg * 8;
      const u16* rb = LD + (nt * 32 + lr) * WG_LD + wave * 32 + lg * 8;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // 8-byte LDS reads (rows are 8-byte aligned)
        const bf16x4 a0 = *reinterpret_cast<const bf16x4*>(ra + 16 * j);
        const bf16x4 a1 = *reinterpret_cast<const bf16x4*>(ra + 16 * j + 4);
        const bf16x4 b0 = *reinterpret_cast<const bf16x4*>(rb + 16 * j);
        const bf16x4 b1 = *reinterpret_cast<const bf16x4*>(rb + 16 * j + 4);
        acc[t] = mfma16(a0, a1, b0, b1, acc[t]);
      }
    }
  }
  // sum the four waves' tiles in LDS, then one partial set per block
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= ntiles) break;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = 8 * (i >> 2) + 4 * lg + (i & 3);
      red[(wave * 4 + t) * 1024 + row * 32 + lr] = acc[t][i];
    }
  }
  __syncthreads();
  float* dst = part + (long long)blockIdx.x * KN;
  for (int e = tid; e < ntiles * 1024; e += 256) {
    const int t = e >> 10, w = e & 1023;
    const int tile = t0 + t, kt = tile / Nt, nt = tile % Nt;
    const int k = kt * 32 + (w >> 5), n = nt * 32 + (w & 31);
    if (k < K && n < N)
      dst[k * N + n] = (red[t * 1024 + w] + red[(4 + t) * 1024 + w]) +
                       (red[(8 + t) * 1024 + w] + red[(12 + t) * 1024 + w]);
  }
  if (t0 == 0 && tid < N) dst[K * N + tid] = bsum;  // the bias row
}

// Adds nsets partial sets into gW / gb, for the entries of tiles [t0, t0 + 4)
// (and the bias row when t0 == 0).  A block sums 64 consecutive entries: its
// four groups of 64 threads take every fourth set, then combine in LDS.
__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ part, int nsets, int K, int N,
                                                      int t0, float* __restrict__ gW, float* __restrict__ gb) {
  __shared__ float sh[4][64];
  const int KN = (K + 1) * N;
  const int el = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  float s = 0.f;
  if (e < KN)
    for (int b = grp; b < nsets; b += 4) s += part[(long long)b * KN + e];
  sh[grp][el] = s;
  __syncthreads();
  if (grp != 0 || e >= KN) return;
  s = (sh[0][el] + sh[1][el]) + (sh[2][el] + sh[3][el]);
  const int k = e / N, n = e % N;
  if (k < K) {
    const int tile = (k / 32) * ((N + 31) / 32) + n / 32;
    if (tile < t0 || tile >= t0 + 4) return;
    gW[k * N + n] += s;
  } else if (t0 == 0) {
    gb[n] += s;
  }
}

// ---- elementwise ------------------------------------------------------------------
// dpre = dpost * GELU'(pre) (or dpost when last), f32 and bf16 copies.
__global__ void __launch_bounds__(256) k_gelu_bwd(const float* __restrict__ dpost, const u16* __restrict__ pre,
                                                  float* __restrict__ dpre, u16* __restrict__ dpreb, long long n,
                                                  int linear) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const float g = linear ? dpost[i] : dpost[i] * gelu_g(bf2f(pre[i]));
  dpre[i] = g;
  dpreb[i] = f2bf(g);
}

// per-channel input normalisation (x - shift) * inv, applied before rounding to bf16
struct InNorm {
  float shift[8];
  float inv[8];
};

// planar f32 [cin][P] (or f64) -> normalised bf16 [P][ld] zero padded
template <typename TI>
__global__ void __launch_bounds__(256) k_pack_input(const TI* __restrict__ x, long long P, int cin, int ld,
                                                    InNorm nm, u16* __restrict__ out) {
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= P) return;
  for (int c = 0; c < ld; ++c)
    out[p * ld + c] = c < cin ? f2bf((float)((x[c * P + p] - (TI)nm.shift[c]) * (TI)nm.inv[c])) : (u16)0;
}

// loss: out f32 [P][co] vs target (y - x) / scale (planar f32); writes dout
// (bf16 [P][ldd] padded, f32 [P][co]) and per-block squared-error partials
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ out, const float* __restrict__ x,
                                              const float* __restrict__ y, const float* __restrict__ scale,
                                              long long P, int co, int ldd, float* __restrict__ doutf,
                                              u16* __restrict__ doutb, double* __restrict__ part) {
  __shared__ double sh[4];
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  double s = 0.0;
  if (p < P) {
    const float inv = 2.0f / (float)((double)P * co);
    for (int c = 0; c < ldd; ++c) {
      float g = 0.f;
      if (c < co) {
        const float tgt = (y[c * P + p] - x[c * P + p]) / scale[c];
        const float d = out[p * co + c] - tgt;
        s += (double)d * d;
        g = d * inv;
        doutf[p * co + c] = g;
      }
      doutb[p * ldd + c] = f2bf(g);
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void __launch_bounds__(256) k_sum_d(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Adam on FP32 master weights; the gradient buffer is consumed (zeroed).
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                                              float* __restrict__ g, long long n, float lr, float b1, float b2,
                                              float eps, float gscale, float c1, float c2) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] * gscale;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  g[i] = 0.f;
}

// bf16 working copies: dst[r][c] = src[r*sr + c*sc] (transposes and padding)
__global__ void __launch_bounds__(256) k_to_bf16(const float* __restrict__ src, int rows, int cols, int ld_dst,
                                                 long long sr, long long sc, u16* __restrict__ dst) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= (long long)rows * ld_dst) return;
  const int r = (int)(i / ld_dst), c = (int)(i % ld_dst);
  dst[i] = c < cols ? f2bf(src[r * sr + c * sc]) : (u16)0;
}

// new_state[f][p] = state[f][p] + scale[f] * out[p][f]  (f64 planar state).
// st and res may be the same array (in-place advance): each element is read
// and then written by the same thread, so neither carries __restrict__.
__global__ void __launch_bounds__(256) k_apply(const double* st, const float* __restrict__ out,
                                               const float* __restrict__ scale, long long P, int co,
                                               double* res, double* __restrict__ part) {
  __shared__ double sh[4];
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  double dc = 0.0;
  if (p < P) {
    for (int f = 0; f < co; ++f) {
      const double d = (double)scale[f] * (double)out[p * co + f];
      res[f * P + p] = st[f * P + p] + d;
      if (f == 0) dc = d;
    }
  }
  for (int o = 32; o > 0; o >>= 1) dc += __shfl_xor(dc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// mass correction: c -= mean increment of c (the composition is conserved)
__global__ void __launch_bounds__(256) k_shift(double* __restrict__ c, long long P, const double* __restrict__ sum) {
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p < P) c[p] -= sum[0] / (double)P;
}

// partial sums of (a - b)^2 and b^2
__global__ void __launch_bounds__(256) k_rel_l2(const double* __restrict__ a, const double* __restrict__ b,
                                                long long n, double* __restrict__ part) {
  __shared__ double sh[2][4];
  double d2 = 0.0, b2 = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const double d = a[i] - b[i];
    d2 += d * d;
    b2 += b[i] * b[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o, 64);
    b2 += __shfl_xor(b2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = d2;
    sh[1][threadIdx.x >> 6] = b2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

}  // namespace

// ---- host side ----------------------------------------------------------------
// Kinds of work for the accounting of algorithmic bytes and flops
// (pf_fno_work): each launch counts its operands read once and its results
// written once, at their storage widths.
enum FnoKind { FK_LM = 0, FK_CM, FK_WGRAD, FK_WSUM, FK_MIX, FK_GELU, FK_ELEM, FK_COUNT };

struct pf_fno {
  pf_fno_config cfg;
  hipStream_t stream = nullptr;
  int acct = 0;  // accounting on
  bool fuse_x = false;  // x stages carried by the channel-mixing GEMMs (n % 32 == 0)
  double acct_bytes[FK_COUNT] = {}, acct_flops[FK_COUNT] = {};
  long long acct_n[FK_COUNT] = {};
  long long P = 0;
  int mode_count = 0;   // (2m)^2 m
  int cinp = 8, coutp = 8;  // padded channel counts (K % 8)
  int64_t nparams = 0;
  // parameter offsets in the flat FP32 vector
  long long o_Wl, o_bl, o_P1, o_c1, o_P2, o_c2;
  std::vector<long long> o_Rr, o_Ri, o_W, o_b;
  float *th = nullptr, *gr = nullptr, *am = nullptr, *av = nullptr;
  long long adam_t = 0;
  // bf16 working weights
  u16 *bWliftT = nullptr, *bP1T = nullptr, *bP1 = nullptr, *bP2T = nullptr, *bP2 = nullptr;
  std::vector<u16*> bWT, bW, bRr, bRi;
  // DFT matrices (forward and inverse stages, and their transposes)
  u16 *Gxf, *Gyf, *Gzf, *Gxi, *Gyi, *Gzi, *GxfT, *GyfT, *GzfT, *GxiT, *GyiT, *GziT;
  float* scale = nullptr;  // output scale per channel
  InNorm innorm;           // input normalisation (identity by default)
  // activations
  u16* xin = nullptr;
  std::vector<u16*> v, pre;
  std::vector<float*> S;
  u16 *hpre = nullptr, *hact = nullptr;
  u16 *A1 = nullptr, *A2 = nullptr, *A3 = nullptr, *Tb = nullptr, *B3 = nullptr, *B2 = nullptr;
  float *T = nullptr, *B1 = nullptr, *outf = nullptr;
  // backward buffers
  float *dvf = nullptr, *dvf2 = nullptr, *dpref = nullptr, *dpref2 = nullptr, *dT = nullptr, *dhf = nullptr;
  u16 *dvb = nullptr, *dpreb = nullptr, *dpreb2 = nullptr, *douthb = nullptr, *dhb = nullptr, *dSb = nullptr;
  float* part = nullptr;
  long long part_elems = 0;
  double* dpart = nullptr;
  double* dsum = nullptr;
  double* hsum = nullptr;  // pinned
  // batched inference over `bcap` samples (allocated on first use, grown on demand)
  int bcap = 0;
  std::vector<void*> ballocs;
  u16 *bxin = nullptr, *bv0 = nullptr, *bv1 = nullptr, *bA1 = nullptr, *bA2 = nullptr, *bTb = nullptr, *bB3 = nullptr,
      *bB2 = nullptr, *bhact = nullptr;
  float *bS = nullptr, *bT = nullptr, *bB1 = nullptr, *boutf = nullptr;
  double *bdpart = nullptr, *bdsum = nullptr;
  // ensemble surrogate advance: current, network and plain states of `ecap` members
  int ecap = 0;
  std::vector<void*> eallocs;
  double *eX = nullptr, *eY = nullptr, *eP = nullptr;
  // checked-advance buffers (allocated on first use)
  double* adv_next = nullptr;
  double* adv_ref = nullptr;
  double* l2_part = nullptr;
  double* l2_host = nullptr;  // pinned
  std::vector<void*> allocs;
};

#define FH(call)                                     \
  do {                                               \
    if ((call) != hipSuccess) return PF_ERR_HIP;     \
  } while (0)

static pf_status falloc(pf_fno* F, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return PF_ERR_OOM;
  }
  F->allocs.push_back(*p);
  return PF_OK;
}

static inline unsigned gdiv(long long n, int b) { return (unsigned)((n + b - 1) / b); }

static inline void account(pf_fno* F, int kind, double bytes, double flops) {
  if (!F->acct) return;
  F->acct_bytes[kind] += bytes;
  F->acct_flops[kind] += flops;
  F->acct_n[kind] += 1;
}

// Real DFT matrices for the six stages (see the header comment of this file).
static void build_dft(int n, int m, std::vector<std::vector<float>>& out) {
  const double pi = 3.14159265358979323846;
  std::vector<int> kx(m), kyz(2 * m);
  for (int i = 0; i < m; ++i) kx[i] = i;
  for (int i = 0; i < m; ++i) kyz[i] = i, kyz[m + i] = n - m + i;
  const int m2 = 2 * m;
  // x forward: rows (ri, kx) 2m, cols x n
  std::vector<float> xf(2 * m * n), xi(n * 2 * m), yf(2 * m2 * 2 * n), yi(2 * n * 2 * m2);
  for (int k = 0; k < m; ++k)
    for (int x = 0; x < n; ++x) {
      const double a = 2 * pi * kx[k] * x / n;
      xf[(0 * m + k) * n + x] = (float)cos(a);
      xf[(1 * m + k) * n + x] = (float)(-sin(a));
      const double w = (kx[k] == 0 ? 1.0 : 2.0) / ((double)n * n * n);
      xi[x * 2 * m + 0 * m + k] = (float)(w * cos(a));
      xi[x * 2 * m + 1 * m + k] = (float)(-w * sin(a));
    }
  // y / z forward: rows (ro, k) 2*m2, cols (y, ri) 2n ; inverse: rows (y, ro) 2n, cols (ri, k) 2*m2
  for (int k = 0; k < m2; ++k)
    for (int y = 0; y < n; ++y) {
      const double a = 2 * pi * kyz[k] * y / n;
      const float C = (float)cos(a), S = (float)sin(a);
      const int K2 = 2 * n;
      yf[(0 * m2 + k) * K2 + y * 2 + 0] = C;
      yf[(0 * m2 + k) * K2 + y * 2 + 1] = S;
      yf[(1 * m2 + k) * K2 + y * 2 + 0] = -S;
      yf[(1 * m2 + k) * K2 + y * 2 + 1] = C;
      const int Kq = 2 * m2;
      yi[(y * 2 + 0) * Kq + 0 * m2 + k] = C;
      yi[(y * 2 + 0) * Kq + 1 * m2 + k] = -S;
      yi[(y * 2 + 1) * Kq + 0 * m2 + k] = S;
      yi[(y * 2 + 1) * Kq + 1 * m2 + k] = C;
    }
  out = {xf, yf, yf, xi, yi, yi};
}

static std::vector<float> transpose(const std::vector<float>& a, int R, int K) {
  std::vector<float> t((size_t)R * K);
  for (int r = 0; r < R; ++r)
    for (int k = 0; k < K; ++k) t[(size_t)k * R + r] = a[(size_t)r * K + k];
  return t;
}

static pf_status upload_bf16(pf_fno* F, const std::vector<float>& h, u16** d) {
  std::vector<u16> b(h.size());
  for (size_t i = 0; i < h.size(); ++i) b[i] = f2bf(h[i]);
  pf_status s = falloc(F, (void**)d, sizeof(u16) * b.size());
  if (s != PF_OK) return s;
  if (hipMemcpy(*d, b.data(), sizeof(u16) * b.size(), hipMemcpyHostToDevice) != hipSuccess) return PF_ERR_HIP;
  return PF_OK;
}

// algorithmic bytes of one channel-mixing GEMM over `points` points
static double cm_bytes(double points, int K, int N, const float* bias, const float* resid, const float* outf,
                       const u16* outpre, const u16* outact, int accumulate) {
  double b = points * K * 2.0 + 2.0 * N * K + (bias ? 4.0 * N : 0.0);
  if (resid) b += points * N * 4.0;
  if (outf) b += points * N * (accumulate ? 8.0 : 4.0);
  if (outpre) b += points * N * 2.0;
  if (outact) b += points * N * 2.0;
  return b;
}

static void lm(pf_fno* F, const u16* G, int R, int K, const u16* X, long long xbs, int ldx, int Nc, int batches,
               float* outf, u16* outb, long long obs, int ldo, int accumulate) {
  const int wpb = Nc <= 32 ? 1 : (Nc <= 64 ? 2 : 4);  // waves per batch
  const double cols = (double)Nc * batches;
  account(F, FK_LM, 2.0 * R * K + 2.0 * K * cols + (outf ? (accumulate ? 8.0 : 4.0) : 2.0) * R * cols,
          2.0 * R * K * cols);
  // the batches in launches of at most 65535 blocks along y
  const long long per = 65535LL * (4 / wpb);
  for (long long b0 = 0; b0 < batches; b0 += per) {
    const long long nb = std::min<long long>(per, batches - b0);
    dim3 grid(gdiv(Nc, 32 * wpb), gdiv(nb, 4 / wpb), gdiv(R, 128));
    k_lm_gemm<<<grid, 256, 0, F->stream>>>(G, R, K, X + b0 * xbs, xbs, ldx, Nc, outf ? outf + b0 * obs : nullptr,
                                           outb ? outb + b0 * obs : nullptr, obs, ldo, accumulate, wpb, nb);
  }
}

static void cm_launch(pf_fno* F, long long points, const u16* In, int ldin, int K, const u16* Bt, int N,
                      const float* bias, const float* resid, int ldres, float* outf, u16* outpre, u16* outact,
                      int ldout, int accumulate, const LineTerm& lt, const u16* gpre = nullptr) {
  const unsigned grid = (unsigned)(points / 128);
  double bytes = cm_bytes((double)points, K, N, bias, resid, outf, outpre, outact, accumulate);
  double flops = 2.0 * points * K * N;
  if (lt.G) {
    bytes += 2.0 * lt.R * lt.K + (double)(points / lt.R) * lt.K * N * 2.0;
    flops += 2.0 * points * lt.K * N;
  }
  if (gpre) bytes += points * N * 2.0;
  account(F, FK_CM, bytes, flops);
  if (N <= 32)
    k_cm_gemm<1><<<grid, 256, 0, F->stream>>>(In, ldin, K, Bt, N, bias, resid, ldres, outf, outpre, outact, ldout,
                                               accumulate, lt, gpre);
  else
    k_cm_gemm<4><<<grid, 256, 0, F->stream>>>(In, ldin, K, Bt, N, bias, resid, ldres, outf, outpre, outact, ldout,
                                               accumulate, lt, gpre);
}

static void cm(pf_fno* F, const u16* In, int ldin, int K, const u16* Bt, int N, const float* bias, const float* resid,
               int ldres, float* outf, u16* outpre, u16* outact, int ldout, int accumulate,
               const LineTerm& lt = LineTerm(), const u16* gpre = nullptr) {
  cm_launch(F, F->P, In, ldin, K, Bt, N, bias, resid, ldres, outf, outpre, outact, ldout, accumulate, lt, gpre);
}

constexpr int kWgradBlocks = 512;  // blocks (point chunks) of one weight-gradient reduction

static void wgrad(pf_fno* F, const u16* A, int lda, int K, const float* D, int ldd, int N, float* gW, float* gb) {
  const long long per = (F->P + kWgradBlocks - 1) / kWgradBlocks;
  const int chunk = (int)((per + WG_PTS - 1) / WG_PTS * WG_PTS);
  const int nb = (int)gdiv(F->P, chunk);
  const int KN = (K + 1) * N;
  const int tiles = ((K + 31) / 32) * ((N + 31) / 32);
  const int ntx = (N + 31) / 32;
  for (int t0 = 0; t0 < tiles; t0 += 4) {
    // this launch's tiles: the K and N ranges it reads, the outputs it forms
    const int t1 = std::min(tiles, t0 + 4);
    double kk = 0.0, nn = 0.0, outs = 0.0;
    {
      int kmin = 1 << 30, kmax = 0, nmin = 1 << 30, nmax = 0;
      for (int t = t0; t < t1; ++t) {
        const int kt = t / ntx, nt = t % ntx;
        kmin = std::min(kmin, kt * 32);
        kmax = std::max(kmax, std::min(K, kt * 32 + 32));
        nmin = std::min(nmin, nt * 32);
        nmax = std::max(nmax, std::min(N, nt * 32 + 32));
        outs += (double)(std::min(K, kt * 32 + 32) - kt * 32) * (std::min(N, nt * 32 + 32) - nt * 32);
      }
      kk = kmax - kmin;
      nn = nmax - nmin;
    }
    account(F, FK_WGRAD, (double)F->P * (2.0 * kk + 4.0 * nn) + 4.0 * nb * KN, 2.0 * F->P * outs);
    k_wgrad_mfma<<<nb, 256, 0, F->stream>>>(A, lda, K, D, ldd, N, F->P, chunk, t0, F->part);
    account(F, FK_WSUM, 4.0 * nb * outs + 8.0 * outs, (double)nb * outs);
    k_sum_partials<<<gdiv(KN, 64), 256, 0, F->stream>>>(F->part, nb, K, N, t0, gW, gb);
  }
}

// refresh the bf16 working weights from the FP32 master vector
static void refresh(pf_fno* F) {
  const pf_fno_config& c = F->cfg;
  const int w = c.width, h = c.hidden;
  hipStream_t s = F->stream;
  auto cvt = [&](long long off, int rows, int cols, int ld, long long sr, long long sc, u16* dst) {
    k_to_bf16<<<gdiv((long long)rows * ld, 256), 256, 0, s>>>(F->th + off, rows, cols, ld, sr, sc, dst);
  };
  // W_lift^T [w][cinp]: dst[o][c] = W_lift[c][o]
  cvt(F->o_Wl, w, c.cin, F->cinp, 1, w, F->bWliftT);
  for (int l = 0; l < c.layers; ++l) {
    cvt(F->o_W[l], w, w, w, 1, w, F->bWT[l]);   // W^T[o][i] = W[i][o]
    cvt(F->o_W[l], w, w, w, w, 1, F->bW[l]);    // W[i][o]
    const long long nr = (long long)F->mode_count * w * w;
    k_to_bf16<<<gdiv(nr, 256), 256, 0, s>>>(F->th + F->o_Rr[l], 1, (int)nr, (int)nr, 0, 1, F->bRr[l]);
    k_to_bf16<<<gdiv(nr, 256), 256, 0, s>>>(F->th + F->o_Ri[l], 1, (int)nr, (int)nr, 0, 1, F->bRi[l]);
  }
  cvt(F->o_P1, h, w, w, 1, h, F->bP1T);        // P1^T [h][w]
  cvt(F->o_P1, w, h, h, h, 1, F->bP1);         // P1 [w][h]
  cvt(F->o_P2, c.cout, h, h, 1, c.cout, F->bP2T);  // P2^T [cout][h]
  cvt(F->o_P2, h, c.cout, F->coutp, c.cout, 1, F->bP2);  // P2 [h][coutp]
}

// per-mode mixing of `batches` spectra: S (f32) and R (bf16) in, T (f32) and Tb (bf16) out
static double mix_fwd_bytes(int modes, int w, int batches) {
  const double mo = (double)modes * w;
  return batches * (2.0 * mo * 4.0 + 2.0 * mo * (4.0 + 2.0)) + 2.0 * modes * (double)w * w * 2.0;
}

// the inverse x stage of a layer's spectral path as a line term (B2: the
// inverse y stage's output, one 2m x w block per x line)
static LineTerm x_inverse(const pf_fno* F, const u16* B2) {
  LineTerm lt;
  lt.G = F->Gxi;
  lt.K = 2 * F->cfg.modes;
  lt.R = F->cfg.n;
  lt.X = B2;
  lt.xbs = (long long)2 * F->cfg.modes * F->cfg.width;
  lt.ldx = F->cfg.width;
  return lt;
}

// forward pass for the packed input F->xin; leaves the result in F->outf
static void forward(pf_fno* F) {
  const pf_fno_config& c = F->cfg;
  const int n = c.n, w = c.width, m = c.modes, m2 = 2 * m, h = c.hidden;
  const long long P = F->P;
  const float* th = F->th;
  cm(F, F->xin, F->cinp, F->cinp, F->bWliftT, w, th + F->o_bl, nullptr, 0, nullptr, F->v[0], nullptr, w, 0);
  for (int l = 0; l < c.layers; ++l) {
    const u16* v = F->v[l];
    // forward truncated DFT: x (batch z,y), y (batch z), z
    lm(F, F->Gxf, 2 * m, n, v, (long long)n * w, w, w, n * n, nullptr, F->A1, (long long)2 * m * w, w, 0);
    lm(F, F->Gyf, 2 * m2, 2 * n, F->A1, (long long)n * 2 * m * w, m * w, m * w, n, nullptr, F->A2,
       (long long)2 * m2 * m * w, m * w, 0);
    const int Nz = m2 * m * w;
    lm(F, F->Gzf, 2 * m2, 2 * n, F->A2, 0, Nz, Nz, 1, F->S[l], nullptr, 0, Nz, 0);
    // per-mode mixing
    account(F, FK_MIX, mix_fwd_bytes(F->mode_count, w, 1), 8.0 * F->mode_count * w * w);
    k_mix_fwd<<<gdiv((long long)F->mode_count * w, 256), 256, 0, F->stream>>>(F->S[l], F->bRr[l], F->bRi[l], F->T,
                                                                               F->mode_count, w, F->Tb, 1);
    // inverse: z, y (batch z), x (batch z,y)
    lm(F, F->Gzi, 2 * n, 2 * m2, F->Tb, 0, Nz, Nz, 1, nullptr, F->B3, 0, Nz, 0);
    lm(F, F->Gyi, 2 * n, 2 * m2, F->B3, (long long)2 * m2 * m * w, m * w, m * w, n, nullptr, F->B2,
       (long long)2 * n * m * w, m * w, 0);
    // pointwise path, bias, the spectral part's inverse x stage (carried by the
    // channel-mixing GEMM when a wave's points lie in one line, else through
    // B1), activation (the last layer is linear)
    const bool last = l == c.layers - 1;
    if (F->fuse_x) {
      cm(F, v, w, w, F->bWT[l], w, th + F->o_b[l], nullptr, 0, nullptr, F->pre[l], last ? nullptr : F->v[l + 1], w, 0,
         x_inverse(F, F->B2));
    } else {
      lm(F, F->Gxi, n, 2 * m, F->B2, (long long)2 * m * w, w, w, n * n, F->B1, nullptr, (long long)n * w, w, 0);
      cm(F, v, w, w, F->bWT[l], w, th + F->o_b[l], F->B1, w, nullptr, F->pre[l], last ? nullptr : F->v[l + 1], w, 0);
    }
  }
  const u16* vL = F->pre[c.layers - 1];  // v_L = pre_{L-1}
  cm(F, vL, w, w, F->bP1T, h, th + F->o_c1, nullptr, 0, nullptr, F->hpre, F->hact, h, 0);
  cm(F, F->hact, h, h, F->bP2T, c.cout, th + F->o_c2, nullptr, 0, F->outf, nullptr, nullptr, c.cout, 0);
  (void)P;
}

// backward pass; the loss gradient is in F->douthb (bf16 [P][coutp]) and F->dvf2 (f32 [P][cout])
static void backward(pf_fno* F) {
  const pf_fno_config& c = F->cfg;
  const int n = c.n, w = c.width, m = c.modes, m2 = 2 * m, h = c.hidden, co = c.cout;
  const long long P = F->P;
  float* g = F->gr;
  // projection: out = hact P2 + c2
  wgrad(F, F->hact, h, h, F->dvf2, co, co, g + F->o_P2, g + F->o_c2);
  // d hpre = (d out P2^T) GELU'(hpre), formed in the GEMM's epilogue
  cm(F, F->douthb, F->coutp, F->coutp, F->bP2, h, nullptr, nullptr, 0, F->dhf, F->dhb, nullptr, h, 0, LineTerm(),
     F->hpre);
  wgrad(F, F->pre[c.layers - 1], w, w, F->dhf, h, h, g + F->o_P1, g + F->o_c1);
  const int Nz = m2 * m * w;
  // the spectral path's transposed stages from dpreb (bf16 d pre of the layer) down to A1
  auto spectral_back = [&](int l, const u16* dpreb) {
    lm(F, F->GxiT, 2 * m, n, dpreb, (long long)n * w, w, w, n * n, nullptr, F->B2, (long long)2 * m * w, w, 0);
    lm(F, F->GyiT, 2 * m2, 2 * n, F->B2, (long long)2 * n * m * w, m * w, m * w, n, nullptr, F->B3,
       (long long)2 * m2 * m * w, m * w, 0);
    lm(F, F->GziT, 2 * m2, 2 * n, F->B3, 0, Nz, Nz, 1, F->dT, nullptr, 0, Nz, 0);
    account(F, FK_MIX, 2.0 * F->mode_count * w * 4.0 * 2 + 2.0 * F->mode_count * (double)w * w * 8.0,
            8.0 * F->mode_count * w * w);
    account(F, FK_MIX, 2.0 * F->mode_count * w * (4.0 + 2.0) + 2.0 * F->mode_count * (double)w * w * 2.0,
            8.0 * F->mode_count * w * w);
    k_mix_bwd_w<<<gdiv((long long)F->mode_count * w * w, 256), 256, 0, F->stream>>>(
        F->S[l], F->dT, g + F->o_Rr[l], g + F->o_Ri[l], F->mode_count, w);
    k_mix_bwd_data<<<gdiv((long long)F->mode_count * w, 256), 256, 0, F->stream>>>(F->dT, F->bRr[l], F->bRi[l],
                                                                                   F->dSb, F->mode_count, w);
    lm(F, F->GzfT, 2 * n, 2 * m2, F->dSb, 0, Nz, Nz, 1, nullptr, F->A2, 0, Nz, 0);
    lm(F, F->GyfT, 2 * n, 2 * m2, F->A2, (long long)2 * m2 * m * w, m * w, m * w, n, nullptr, F->A1,
       (long long)2 * n * m * w, m * w, 0);
  };
  if (F->fuse_x) {
    // d v_l = d pre_l W^T + (transposed x stage of A1) in one GEMM, whose
    // epilogue applies GELU'(pre_{l-1}) to give d pre_{l-1} (f32 and bf16),
    // ping-ponging between two buffers; the last layer is linear
    LineTerm lt;
    lt.G = F->GxfT;
    lt.K = 2 * m;
    lt.R = n;
    lt.X = F->A1;
    lt.xbs = (long long)2 * m * w;
    lt.ldx = w;
    float* df[2] = {F->dpref, F->dpref2};
    u16* db[2] = {F->dpreb, F->dpreb2};
    int cur = 0;
    cm(F, F->dhb, h, h, F->bP1, w, nullptr, nullptr, 0, df[cur], db[cur], nullptr, w, 0);
    for (int l = c.layers - 1; l >= 0; --l) {
      wgrad(F, F->v[l], w, w, df[cur], w, w, g + F->o_W[l], g + F->o_b[l]);
      spectral_back(l, db[cur]);
      if (l > 0) {
        cm(F, db[cur], w, w, F->bW[l], w, nullptr, nullptr, 0, df[1 - cur], db[1 - cur], nullptr, w, 0, lt,
           F->pre[l - 1]);
        cur = 1 - cur;
      } else {
        cm(F, db[cur], w, w, F->bW[0], w, nullptr, nullptr, 0, F->dvf, nullptr, nullptr, w, 0, lt);
      }
    }
  } else {
    cm(F, F->dhb, h, h, F->bP1, w, nullptr, nullptr, 0, F->dvf, nullptr, nullptr, w, 0);
    for (int l = c.layers - 1; l >= 0; --l) {
      const bool last = l == c.layers - 1;
      account(F, FK_GELU, (double)P * w * (4.0 + 2.0 + 4.0 + 2.0), 20.0 * P * w);
      k_gelu_bwd<<<gdiv(P * w, 256), 256, 0, F->stream>>>(F->dvf, F->pre[l], F->dpref, F->dpreb, P * w,
                                                          last ? 1 : 0);
      wgrad(F, F->v[l], w, w, F->dpref, w, w, g + F->o_W[l], g + F->o_b[l]);
      spectral_back(l, F->dpreb);
      // pointwise data gradient plus the transposed x stage of the spectral path
      cm(F, F->dpreb, w, w, F->bW[l], w, nullptr, nullptr, 0, F->dvf, nullptr, nullptr, w, 0);
      lm(F, F->GxfT, n, 2 * m, F->A1, (long long)2 * m * w, w, w, n * n, F->dvf, nullptr, (long long)n * w, w, 1);
    }
  }
  // lift: v0 = x W_lift + b_lift
  wgrad(F, F->xin, F->cinp, c.cin, F->dvf, w, w, g + F->o_Wl, g + F->o_bl);
}

extern "C" {

pf_status pf_fno_create(const pf_fno_config* cfg, void* stream, pf_fno** out) {
  if (!cfg || !out) return PF_ERR_ARG;
  *out = nullptr;
  const pf_fno_config c = *cfg;
  if (c.n < 8 || c.n > 256 || c.n % 8 || c.width < 4 || c.width > 128 || c.width % 4 || c.modes < 2 ||
      c.modes % 2 || 2 * c.modes > c.n || c.layers < 1 || c.layers > 8 || c.hidden < 8 || c.hidden > 128 || c.hidden % 8 ||
      c.cin < 1 || c.cin > 8 || c.cout < 1 || c.cout > 8)
    return PF_ERR_ARG;
  int ndev = 0;  // no usable device: a HIP error, before any allocation
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return PF_ERR_HIP;
  pf_fno* F = new (std::nothrow) pf_fno();
  if (!F) return PF_ERR_OOM;
  F->cfg = c;
  F->stream = (hipStream_t)stream;
  F->P = (long long)c.n * c.n * c.n;
  for (int i = 0; i < 8; ++i) F->innorm.shift[i] = 0.f, F->innorm.inv[i] = 1.f;
  const int w = c.width, m = c.modes, m2 = 2 * m, h = c.hidden, n = c.n;
  F->mode_count = m2 * m2 * m;
  F->fuse_x = n % 32 == 0;
  // parameter layout (same order as the oracle)
  long long off = 0;
  F->o_Wl = off; off += (long long)c.cin * w;
  F->o_bl = off; off += w;
  for (int l = 0; l < c.layers; ++l) {
    F->o_Rr.push_back(off); off += (long long)F->mode_count * w * w;
    F->o_Ri.push_back(off); off += (long long)F->mode_count * w * w;
    F->o_W.push_back(off); off += (long long)w * w;
    F->o_b.push_back(off); off += w;
  }
  F->o_P1 = off; off += (long long)w * h;
  F->o_c1 = off; off += h;
  F->o_P2 = off; off += (long long)h * c.cout;
  F->o_c2 = off; off += c.cout;
  F->nparams = off;
  const long long P = F->P;
  pf_status s = PF_OK;
  auto A = [&](void** p, size_t b) {
    if (s == PF_OK) s = falloc(F, p, b);
  };
  A((void**)&F->th, 4 * off);
  A((void**)&F->gr, 4 * off);
  A((void**)&F->am, 4 * off);
  A((void**)&F->av, 4 * off);
  A((void**)&F->bWliftT, 2 * w * F->cinp);
  F->bWT.resize(c.layers);
  F->bW.resize(c.layers);
  F->bRr.resize(c.layers);
  F->bRi.resize(c.layers);
  for (int l = 0; l < c.layers; ++l) {
    A((void**)&F->bWT[l], 2 * w * w);
    A((void**)&F->bW[l], 2 * w * w);
    A((void**)&F->bRr[l], 2 * (size_t)F->mode_count * w * w);
    A((void**)&F->bRi[l], 2 * (size_t)F->mode_count * w * w);
  }
  A((void**)&F->bP1T, 2 * h * w);
  A((void**)&F->bP1, 2 * w * h);
  A((void**)&F->bP2T, 2 * c.cout * h);
  A((void**)&F->bP2, 2 * h * F->coutp);
  A((void**)&F->scale, 4 * 8);
  A((void**)&F->xin, 2 * P * F->cinp);
  F->v.resize(c.layers + 1);
  F->pre.resize(c.layers);
  F->S.resize(c.layers);
  for (int l = 0; l <= c.layers; ++l) A((void**)&F->v[l], 2 * P * w);
  const size_t spec = (size_t)2 * F->mode_count * w;
  for (int l = 0; l < c.layers; ++l) {
    A((void**)&F->pre[l], 2 * P * w);
    A((void**)&F->S[l], 4 * spec);
  }
  A((void**)&F->hpre, 2 * P * h);
  A((void**)&F->hact, 2 * P * h);
  const size_t a1 = (size_t)n * n * 2 * m * w, a2 = (size_t)n * 2 * m2 * m * w, b2 = (size_t)n * 2 * n * m * w;
  A((void**)&F->A1, 2 * std::max(a1, b2));
  A((void**)&F->A2, 2 * std::max(a2, (size_t)2 * n * m2 * m * w));
  A((void**)&F->A3, 2 * spec);
  A((void**)&F->Tb, 2 * spec);
  A((void**)&F->T, 4 * spec);
  A((void**)&F->B3, 2 * std::max((size_t)2 * n * m2 * m * w, a2));
  A((void**)&F->B2, 2 * std::max(b2, a1));
  if (!F->fuse_x) A((void**)&F->B1, 4 * P * w);
  A((void**)&F->outf, 4 * P * c.cout);
  A((void**)&F->dvf, 4 * P * w);
  A((void**)&F->dvf2, 4 * P * c.cout);
  A((void**)&F->dpref, 4 * P * w);
  A((void**)&F->dT, 4 * spec);
  A((void**)&F->dhf, 4 * P * h);
  A((void**)&F->dhb, 2 * P * h);
  A((void**)&F->dpreb, 2 * P * w);
  if (F->fuse_x) A((void**)&F->dpref2, 4 * P * w);
  if (F->fuse_x) A((void**)&F->dpreb2, 2 * P * w);
  A((void**)&F->douthb, 2 * P * F->coutp);
  A((void**)&F->dSb, 2 * spec);
  F->part_elems = (long long)kWgradBlocks * (std::max(std::max(w, h), 8) + 1) * std::max(std::max(w, h), 8);
  A((void**)&F->part, 4 * F->part_elems);
  A((void**)&F->dpart, 8 * (size_t)gdiv(P, 256));
  A((void**)&F->dsum, 8);
  if (s == PF_OK && hipHostMalloc((void**)&F->hsum, 8, 0) != hipSuccess) s = PF_ERR_OOM;
  if (s == PF_OK) {
    std::vector<std::vector<float>> G;
    build_dft(n, m, G);
    const int R[6] = {2 * m, 2 * m2, 2 * m2, n, 2 * n, 2 * n};
    const int K[6] = {n, 2 * n, 2 * n, 2 * m, 2 * m2, 2 * m2};
    u16** dst[6] = {&F->Gxf, &F->Gyf, &F->Gzf, &F->Gxi, &F->Gyi, &F->Gzi};
    u16** dstT[6] = {&F->GxfT, &F->GyfT, &F->GzfT, &F->GxiT, &F->GyiT, &F->GziT};
    for (int i = 0; i < 6 && s == PF_OK; ++i) {
      s = upload_bf16(F, G[i], dst[i]);
      if (s == PF_OK) s = upload_bf16(F, transpose(G[i], R[i], K[i]), dstT[i]);
    }
  }
  if (s == PF_OK) {
    std::vector<float> one(8, 1.0f);
    if (hipMemcpy(F->scale, one.data(), 32, hipMemcpyHostToDevice) != hipSuccess) s = PF_ERR_HIP;
    if (hipMemset(F->th, 0, 4 * off) != hipSuccess || hipMemset(F->gr, 0, 4 * off) != hipSuccess ||
        hipMemset(F->am, 0, 4 * off) != hipSuccess || hipMemset(F->av, 0, 4 * off) != hipSuccess)
      s = PF_ERR_HIP;
  }
  if (s != PF_OK) {
    pf_fno_destroy(F);
    return s;
  }
  *out = F;
  return PF_OK;
}

void pf_fno_destroy(pf_fno* F) {
  if (!F) return;
  if (F->stream) hipStreamSynchronize(F->stream);
  for (void* p : F->allocs) hipFree(p);
  for (void* p : F->ballocs) hipFree(p);
  for (void* p : F->eallocs) hipFree(p);
  if (F->hsum) hipHostFree(F->hsum);
  if (F->l2_host) hipHostFree(F->l2_host);
  delete F;
}

int64_t pf_fno_num_params(const pf_fno* F) { return F ? F->nparams : 0; }

pf_status pf_fno_set_params(pf_fno* F, const float* host) {
  if (!F || !host) return PF_ERR_ARG;
  FH(hipMemcpyAsync(F->th, host, 4 * F->nparams, hipMemcpyHostToDevice, F->stream));
  refresh(F);
  FH(hipMemsetAsync(F->am, 0, 4 * F->nparams, F->stream));
  FH(hipMemsetAsync(F->av, 0, 4 * F->nparams, F->stream));
  FH(hipMemsetAsync(F->gr, 0, 4 * F->nparams, F->stream));
  F->adam_t = 0;
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

pf_status pf_fno_get_params(pf_fno* F, float* host) {
  if (!F || !host) return PF_ERR_ARG;
  FH(hipMemcpyAsync(host, F->th, 4 * F->nparams, hipMemcpyDeviceToHost, F->stream));
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

pf_status pf_fno_get_grad(pf_fno* F, float* host) {
  if (!F || !host) return PF_ERR_ARG;
  FH(hipMemcpyAsync(host, F->gr, 4 * F->nparams, hipMemcpyDeviceToHost, F->stream));
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

pf_status pf_fno_load(pf_fno* F, const void* host, size_t bytes) {
  if (!F || !host) return PF_ERR_ARG;
  const size_t np = (size_t)F->nparams;
  if (bytes == 4 * np) return pf_fno_set_params(F, (const float*)host);
  if (bytes != 2 * np) return PF_ERR_ARG;
  // bfloat16 -> float32 is exact (the upper half of the float's bits)
  std::vector<float> w(np);
  const u16* h = (const u16*)host;
  for (size_t i = 0; i < np; ++i) w[i] = bf2f(h[i]);
  return pf_fno_set_params(F, w.data());
}
pf_status pf_fno_train_step(pf_fno* F, const float* x, const float* y, int32_t batch, float lr, float* loss) {
  if (!F || !x || !y || batch < 1 || !(lr > 0.f) || !std::isfinite(lr)) return PF_ERR_ARG;
  pf_status s = pf_fno_zero_grad(F);
  if (s != PF_OK) return s;
  const size_t per = (size_t)F->cfg.cin * (size_t)F->P;
  double tot = 0.0;
  for (int b = 0; b < batch; ++b) {
    double l = 0.0;
    s = pf_fno_grad(F, x + b * per, y + b * per, &l);
    if (s != PF_OK) return s;
    tot += l;
  }
  s = pf_fno_adam_step(F, lr, 0.9f, 0.999f, 1e-8f, 1.0f / (float)batch);
  if (s != PF_OK) return s;
  FH(hipStreamSynchronize(F->stream));
  if (loss) *loss = (float)(tot / batch);
  return PF_OK;
}
pf_status pf_fno_zero_grad(pf_fno* F) {
  if (!F) return PF_ERR_ARG;
  FH(hipMemsetAsync(F->gr, 0, 4 * F->nparams, F->stream));
  return PF_OK;
}

pf_status pf_fno_set_scale(pf_fno* F, const float* host_scale) {
  if (!F || !host_scale) return PF_ERR_ARG;
  FH(hipMemcpyAsync(F->scale, host_scale, 4 * F->cfg.cout, hipMemcpyHostToDevice, F->stream));
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

pf_status pf_fno_set_input_norm(pf_fno* F, const float* shift, const float* scale) {
  if (!F || !shift || !scale) return PF_ERR_ARG;
  for (int c = 0; c < F->cfg.cin; ++c)
    if (!(scale[c] > 0.f) || !std::isfinite(shift[c]) || !std::isfinite(scale[c])) return PF_ERR_ARG;
  for (int c = 0; c < 8; ++c) {
    F->innorm.shift[c] = c < F->cfg.cin ? shift[c] : 0.f;
    F->innorm.inv[c] = c < F->cfg.cin ? 1.f / scale[c] : 1.f;
  }
  return PF_OK;
}

pf_status pf_fno_forward(pf_fno* F, const float* x, float* out) {
  if (!F || !x || !out) return PF_ERR_ARG;
  account(F, FK_ELEM, (double)F->P * (4.0 * F->cfg.cin + 2.0 * F->cinp), 0.0);
  k_pack_input<float><<<gdiv(F->P, 256), 256, 0, F->stream>>>(x, F->P, F->cfg.cin, F->cinp, F->innorm, F->xin);
  forward(F);
  FH(hipMemcpyAsync(out, F->outf, 4 * F->P * F->cfg.cout, hipMemcpyDeviceToDevice, F->stream));
  FH(hipGetLastError());
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

pf_status pf_fno_grad(pf_fno* F, const float* x, const float* y, double* loss) {
  if (!F || !x || !y) return PF_ERR_ARG;
  account(F, FK_ELEM, (double)F->P * (4.0 * F->cfg.cin + 2.0 * F->cinp), 0.0);
  k_pack_input<float><<<gdiv(F->P, 256), 256, 0, F->stream>>>(x, F->P, F->cfg.cin, F->cinp, F->innorm, F->xin);
  forward(F);
  const unsigned nb = gdiv(F->P, 256);
  account(F, FK_ELEM, (double)F->P * F->cfg.cout * (4.0 * 4) + (double)F->P * F->coutp * 2.0, 0.0);
  k_loss<<<nb, 256, 0, F->stream>>>(F->outf, x, y, F->scale, F->P, F->cfg.cout, F->coutp, F->dvf2, F->douthb,
                                    F->dpart);
  k_sum_d<<<1, 256, 0, F->stream>>>(F->dpart, (int)nb, F->dsum);
  backward(F);
  FH(hipMemcpyAsync(F->hsum, F->dsum, 8, hipMemcpyDeviceToHost, F->stream));
  FH(hipGetLastError());
  FH(hipStreamSynchronize(F->stream));
  if (loss) *loss = F->hsum[0] / ((double)F->P * F->cfg.cout);
  return PF_OK;
}

pf_status pf_fno_adam_step(pf_fno* F, float lr, float beta1, float beta2, float eps, float grad_scale) {
  if (!F) return PF_ERR_ARG;
  F->adam_t += 1;
  const float c1 = 1.f - powf(beta1, (float)F->adam_t), c2 = 1.f - powf(beta2, (float)F->adam_t);
  account(F, FK_ELEM, 7.0 * 4.0 * F->nparams, 0.0);
  k_adam<<<gdiv(F->nparams, 256), 256, 0, F->stream>>>(F->th, F->am, F->av, F->gr, F->nparams, lr, beta1, beta2,
                                                       eps, grad_scale, c1, c2);
  refresh(F);
  FH(hipGetLastError());
  return PF_OK;
}

static constexpr int kL2Blocks = 512;
// pf_rel_l2_noalloc: devices it keeps a scratch address for, and the largest
// count it takes (the per-thread partial sums of 512 x 256 threads then add at
// most 2^24 squares each)
static constexpr int kMaxDevices = 64;
static constexpr int64_t kNoallocMaxN = (int64_t)1 << 41;

// ||a - b|| / ||b|| with caller-provided partials (device) and staging (pinned host)
static pf_status rel_l2_impl(hipStream_t s, const double* a, const double* b, long long n, double* part,
                             double* host, double* out) {
  k_rel_l2<<<kL2Blocks, 256, 0, s>>>(a, b, n, part);
  FH(hipGetLastError());
  FH(hipMemcpyAsync(host, part, sizeof(double) * 2 * kL2Blocks, hipMemcpyDeviceToHost, s));
  FH(hipStreamSynchronize(s));
  double d2 = 0.0, b2 = 0.0;
  for (int i = 0; i < kL2Blocks; ++i) {
    d2 += host[2 * i];
    b2 += host[2 * i + 1];
  }
  *out = b2 > 0.0 ? std::sqrt(d2 / b2) : std::sqrt(d2);
  return PF_OK;
}

// ---- allocation-free relative L2 ------------------------------------------------
// The partial sums of pf_rel_l2_noalloc live in a file-scope device array (one
// copy per GPU, held until the process ends).  In host code `scratch` names a
// host-side stand-in, not device memory: the array is only ever reached
// through the address hipGetSymbolAddress returns for the current device,
// looked up once per device on the entry point's first call there.
static __device__ __align__(256) double scratch[2 * kL2Blocks];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {nullptr};

static pf_status scratch_for_current_device(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PF_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PF_ERR_HIP;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return PF_OK;
}

pf_status pf_rel_l2_noalloc(const double* a, const double* b, int64_t n, void* stream, double* out) {
  if (!a || !b || n < 1 || !out) return PF_ERR_ARG;
  if (n > kNoallocMaxN) return PF_ERR_ARG;
  double* part = nullptr;
  pf_status st = scratch_for_current_device(&part);
  if (st != PF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // the same kernel and host-side summation order as pf_rel_l2; the host copy of
  // the partials is a stack array (no pinned or device allocation)
  double host[2 * kL2Blocks];
  k_rel_l2<<<kL2Blocks, 256, 0, s>>>(a, b, n, part);
  FH(hipGetLastError());
  FH(hipMemcpyAsync(host, part, sizeof(host), hipMemcpyDeviceToHost, s));
  FH(hipStreamSynchronize(s));
  double d2 = 0.0, b2 = 0.0;
  for (int i = 0; i < kL2Blocks; ++i) {
    d2 += host[2 * i];
    b2 += host[2 * i + 1];
  }
  *out = b2 > 0.0 ? std::sqrt(d2 / b2) : std::sqrt(d2);
  return PF_OK;
}

pf_status pf_rel_l2(const double* a, const double* b, int64_t n, void* stream, double* out) {
  if (!a || !b || n < 1 || !out) return PF_ERR_ARG;
  double* part = nullptr;
  double* host = nullptr;
  if (hipMalloc((void**)&part, sizeof(double) * 2 * kL2Blocks) != hipSuccess) return PF_ERR_OOM;
  if (hipHostMalloc((void**)&host, sizeof(double) * 2 * kL2Blocks, 0) != hipSuccess) {
    hipFree(part);
    return PF_ERR_OOM;
  }
  pf_status st = rel_l2_impl((hipStream_t)stream, a, b, n, part, host, out);
  hipStreamSynchronize((hipStream_t)stream);
  hipHostFree(host);
  hipFree(part);
  return st;
}

}  // extern "C"

// ---- batched inference ---------------------------------------------------------
static pf_status grow(std::vector<void*>& list, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return PF_ERR_OOM;
  }
  list.push_back(*p);
  return PF_OK;
}

// Inference buffers for B samples (the forward pass's activations, B times;
// no pre-activations or gradients are kept).
static pf_status ensure_batch(pf_fno* F, int B) {
  if (B <= F->bcap) return PF_OK;
  hipStreamSynchronize(F->stream);
  for (void* p : F->ballocs) hipFree(p);
  F->ballocs.clear();
  F->bcap = 0;
  const pf_fno_config& c = F->cfg;
  const size_t w = c.width, m = c.modes, m2 = 2 * m, h = c.hidden, n = c.n, P = (size_t)F->P, Bs = (size_t)B;
  const size_t Nz = m2 * m * w, spec = 2 * (size_t)F->mode_count * w;
  const size_t a1 = std::max(n * n * 2 * m * w, n * 2 * n * m * w);
  pf_status s = PF_OK;
  auto A = [&](void** p, size_t bytes) {
    if (s == PF_OK) s = grow(F->ballocs, p, bytes);
  };
  A((void**)&F->bxin, Bs * 2 * P * F->cinp);
  A((void**)&F->bv0, Bs * 2 * P * w);
  A((void**)&F->bv1, Bs * 2 * P * w);
  A((void**)&F->bA1, Bs * 2 * a1);
  A((void**)&F->bA2, Bs * 2 * 2 * n * Nz);
  A((void**)&F->bS, Bs * 4 * spec);
  A((void**)&F->bT, Bs * 4 * spec);
  A((void**)&F->bTb, Bs * 2 * spec);
  A((void**)&F->bB3, Bs * 2 * 2 * n * Nz);
  A((void**)&F->bB2, Bs * 2 * a1);
  if (!F->fuse_x) A((void**)&F->bB1, Bs * 4 * P * w);
  A((void**)&F->bhact, Bs * 2 * P * h);
  A((void**)&F->boutf, Bs * 4 * P * c.cout);
  A((void**)&F->bdpart, Bs * 8 * gdiv(F->P, 256));
  A((void**)&F->bdsum, Bs * 8);
  if (s != PF_OK) {
    for (void* p : F->ballocs) hipFree(p);
    F->ballocs.clear();
    return s;
  }
  F->bcap = B;
  return PF_OK;
}

static void cm_points(pf_fno* F, long long points, const u16* In, int ldin, int K, const u16* Bt, int N,
                      const float* bias, const float* resid, int ldres, float* outf, u16* outpre, u16* outact,
                      int ldout, const LineTerm& lt = LineTerm()) {
  cm_launch(F, points, In, ldin, K, Bt, N, bias, resid, ldres, outf, outpre, outact, ldout, 0, lt);
}

// The forward pass of B samples at once (inputs packed in bxin, outputs in
// boutf): every channel-mixing GEMM runs over the B n^3 points together and
// every truncated-DFT stage takes the B samples' lines as more batches of the
// same small GEMM, so the sums are those of the one-sample pass.
static void forward_batch(pf_fno* F, int B) {
  const pf_fno_config& c = F->cfg;
  const int n = c.n, w = c.width, m = c.modes, m2 = 2 * m, h = c.hidden;
  const long long PB = F->P * B;
  const long long Nz = (long long)m2 * m * w, spec = 2LL * F->mode_count * w;
  const float* th = F->th;
  cm_points(F, PB, F->bxin, F->cinp, F->cinp, F->bWliftT, w, th + F->o_bl, nullptr, 0, nullptr, F->bv0, nullptr, w);
  u16* v = F->bv0;
  u16* vn = F->bv1;
  for (int l = 0; l < c.layers; ++l) {
    lm(F, F->Gxf, 2 * m, n, v, (long long)n * w, w, w, B * n * n, nullptr, F->bA1, (long long)2 * m * w, w, 0);
    lm(F, F->Gyf, 2 * m2, 2 * n, F->bA1, (long long)n * 2 * m * w, m * w, m * w, B * n, nullptr, F->bA2,
       (long long)2 * m2 * m * w, m * w, 0);
    lm(F, F->Gzf, 2 * m2, 2 * n, F->bA2, 2LL * n * Nz, (int)Nz, (int)Nz, B, F->bS, nullptr, spec, (int)Nz, 0);
    account(F, FK_MIX, mix_fwd_bytes(F->mode_count, w, B), 8.0 * F->mode_count * w * w * B);
    k_mix_fwd<<<gdiv((long long)F->mode_count * w * B, 256), 256, 0, F->stream>>>(F->bS, F->bRr[l], F->bRi[l],
                                                                                   F->bT, F->mode_count, w,
                                                                                   F->bTb, B);
    lm(F, F->Gzi, 2 * n, 2 * m2, F->bTb, spec, (int)Nz, (int)Nz, B, nullptr, F->bB3, 2LL * n * Nz, (int)Nz, 0);
    lm(F, F->Gyi, 2 * n, 2 * m2, F->bB3, (long long)2 * m2 * m * w, m * w, m * w, B * n, nullptr, F->bB2,
       (long long)2 * n * m * w, m * w, 0);
    const bool last = l == c.layers - 1;
    if (F->fuse_x) {
      cm_points(F, PB, v, w, w, F->bWT[l], w, th + F->o_b[l], nullptr, 0, nullptr, last ? vn : nullptr,
                last ? nullptr : vn, w, x_inverse(F, F->bB2));
    } else {
      lm(F, F->Gxi, n, 2 * m, F->bB2, (long long)2 * m * w, w, w, B * n * n, F->bB1, nullptr, (long long)n * w, w,
         0);
      cm_points(F, PB, v, w, w, F->bWT[l], w, th + F->o_b[l], F->bB1, w, nullptr, last ? vn : nullptr,
                last ? nullptr : vn, w);
    }
    std::swap(v, vn);
  }
  cm_points(F, PB, v, w, w, F->bP1T, h, th + F->o_c1, nullptr, 0, nullptr, nullptr, F->bhact, h);
  cm_points(F, PB, F->bhact, h, h, F->bP2T, c.cout, th + F->o_c2, nullptr, 0, F->boutf, nullptr, nullptr, c.cout);
}

// next_b = state_b + scale * net(state_b), mean of c restored, for b < B
// (states / nexts: [B][cin][n^3] float64; next may equal state).
static pf_status apply_batch(pf_fno* F, const double* states, double* nexts, int B) {
  pf_status s = ensure_batch(F, B);
  if (s != PF_OK) return s;
  const long long P = F->P;
  const int ci = F->cfg.cin, co = F->cfg.cout;
  const unsigned nb = gdiv(P, 256);
  for (int b = 0; b < B; ++b) {
    account(F, FK_ELEM, (double)P * (8.0 * ci + 2.0 * F->cinp), 0.0);
    k_pack_input<double><<<nb, 256, 0, F->stream>>>(states + (long long)b * ci * P, P, ci, F->cinp, F->innorm,
                                                    F->bxin + (long long)b * P * F->cinp);
  }
  forward_batch(F, B);
  for (int b = 0; b < B; ++b) {
    double* nx = nexts + (long long)b * co * P;
    account(F, FK_ELEM, (double)P * co * (8.0 + 4.0 + 8.0), 0.0);
    k_apply<<<nb, 256, 0, F->stream>>>(states + (long long)b * ci * P, F->boutf + (long long)b * P * co, F->scale, P,
                                       co, nx, F->bdpart + (long long)b * nb);
    k_sum_d<<<1, 256, 0, F->stream>>>(F->bdpart + (long long)b * nb, (int)nb, F->bdsum + b);
    account(F, FK_ELEM, (double)P * 16.0, 0.0);
    k_shift<<<nb, 256, 0, F->stream>>>(nx, P, F->bdsum + b);
  }
  FH(hipGetLastError());
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

extern "C" {

pf_status pf_fno_work(pf_fno* F, int32_t enable, double* bytes, double* flops, int64_t* launches, int32_t kinds) {
  if (!F || kinds < 0 || (kinds > 0 && (!bytes || !flops || !launches))) return PF_ERR_ARG;
  for (int k = 0; k < kinds && k < FK_COUNT; ++k) {
    bytes[k] = F->acct_bytes[k];
    flops[k] = F->acct_flops[k];
    launches[k] = F->acct_n[k];
  }
  for (int k = FK_COUNT; k < kinds; ++k) {
    bytes[k] = flops[k] = 0.0;
    launches[k] = 0;
  }
  if (enable >= 0) {
    F->acct = enable ? 1 : 0;
    for (int k = 0; k < FK_COUNT; ++k) {
      F->acct_bytes[k] = F->acct_flops[k] = 0.0;
      F->acct_n[k] = 0;
    }
  }
  return PF_OK;
}

pf_status pf_fno_apply_batch(pf_fno* F, const double* states, double* nexts, int32_t batch) {
  if (!F || !states || !nexts || batch < 1 || F->cfg.cin != F->cfg.cout) return PF_ERR_ARG;
  return apply_batch(F, states, nexts, batch);
}

pf_status pf_fno_apply(pf_fno* F, const double* state, double* next) {
  if (!F || !state || !next || F->cfg.cin != F->cfg.cout) return PF_ERR_ARG;
  account(F, FK_ELEM, (double)F->P * (8.0 * F->cfg.cin + 2.0 * F->cinp), 0.0);
  k_pack_input<double><<<gdiv(F->P, 256), 256, 0, F->stream>>>(state, F->P, F->cfg.cin, F->cinp, F->innorm, F->xin);
  forward(F);
  const unsigned nb = gdiv(F->P, 256);
  account(F, FK_ELEM, (double)F->P * F->cfg.cout * (8.0 + 4.0 + 8.0), 0.0);
  k_apply<<<nb, 256, 0, F->stream>>>(state, F->outf, F->scale, F->P, F->cfg.cout, next, F->dpart);
  k_sum_d<<<1, 256, 0, F->stream>>>(F->dpart, (int)nb, F->dsum);
  account(F, FK_ELEM, (double)F->P * 16.0, 0.0);
  k_shift<<<nb, 256, 0, F->stream>>>(next, F->P, F->dsum);
  FH(hipGetLastError());
  FH(hipStreamSynchronize(F->stream));
  return PF_OK;
}

// one plain-solver interval: out = plain(state) over [0, delta]
static pf_status plain_interval(pf_ctx* plain, const double* in, double* out, long long P, double delta) {
  pf_status s = pf_set_state(plain, in, in + P, 1, 0.0);
  if (s != PF_OK) return s;
  s = pf_advance(plain, delta, nullptr);
  if (s != PF_OK) return s;
  return pf_get_state(plain, out, out + P, 1);
}

pf_status pf_fno_advance(pf_fno* F, pf_ctx* plain, double* state, int32_t n_adv, double delta,
                         int32_t check_every, double tol, pf_fno_stats* st) {
  if (!F || !plain || !state || !st || n_adv < 0 || !(delta > 0.0) || check_every < 1 || !(tol >= 0.0) ||
      F->cfg.cin != 4 || F->cfg.cout != 4)
    return PF_ERR_ARG;
  const long long P = F->P;
  const size_t bytes = sizeof(double) * 4 * P;
  if (!F->adv_next) {
    pf_status s = falloc(F, (void**)&F->adv_next, bytes);
    if (s == PF_OK) s = falloc(F, (void**)&F->adv_ref, bytes);
    if (s == PF_OK) s = falloc(F, (void**)&F->l2_part, sizeof(double) * 2 * kL2Blocks);
    if (s == PF_OK && hipHostMalloc((void**)&F->l2_host, sizeof(double) * 2 * kL2Blocks, 0) != hipSuccess)
      s = PF_ERR_OOM;
    if (s != PF_OK) return s;
  }
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  for (int32_t a = 0; a < n_adv; ++a) {
    if (st->plain_left > 0) {
      const auto t0 = clk::now();
      pf_status s = plain_interval(plain, state, state, P, delta);
      st->ms_plain += ms_since(t0);
      if (s != PF_OK) return s;
      st->plain += 1;
      st->plain_left -= 1;
      continue;
    }
    const bool check = st->since_check + 1 >= check_every;
    auto t0 = clk::now();
    pf_status s = pf_fno_apply(F, state, check ? F->adv_next : state);
    st->ms_surrogate += ms_since(t0);
    if (s != PF_OK) return s;
    st->surrogate += 1;
    st->since_check += 1;
    if (!check) continue;
    st->since_check = 0;
    st->checks += 1;
    t0 = clk::now();
    s = plain_interval(plain, state, F->adv_ref, P, delta);
    double err = 0.0;
    if (s == PF_OK) s = rel_l2_impl(F->stream, F->adv_next, F->adv_ref, P, F->l2_part, F->l2_host, &err);
    if (s != PF_OK) return s;
    st->err_last = err;
    if (!(err <= st->err_max)) st->err_max = err;
    const bool fail = !(err <= tol);
    if (fail) {
      st->fallbacks += 1;
      st->plain_left = check_every;
    }
    FH(hipMemcpyAsync(state, fail ? F->adv_ref : F->adv_next, bytes, hipMemcpyDeviceToDevice, F->stream));
    FH(hipStreamSynchronize(F->stream));
    st->ms_plain += ms_since(t0);
  }
  return PF_OK;
}

pf_status pf_fno_ensemble_advance(pf_fno* F, pf_ens* E, const int32_t* members, int32_t count, int32_t n_adv,
                                  double delta, int32_t check_every, double tol, pf_fno_stats* st) {
  if (!F || !E || !members || !st || count < 1 || n_adv < 0 || !(delta > 0.0) || check_every < 1 || !(tol >= 0.0) ||
      F->cfg.cin != 4 || F->cfg.cout != 4)
    return PF_ERR_ARG;
  const int M = pf::ens_members(E);
  for (int i = 0; i < count; ++i) {
    if (members[i] < 0 || members[i] >= M || pf::ens_member_n(E, members[i]) != F->cfg.n) return PF_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return PF_ERR_ARG;
  }
  const long long P = F->P;
  const size_t per = 4 * (size_t)P;
  if (count > F->ecap) {
    hipStreamSynchronize(F->stream);
    for (void* p : F->eallocs) hipFree(p);
    F->eallocs.clear();
    F->ecap = 0;
    pf_status s = grow(F->eallocs, (void**)&F->eX, sizeof(double) * per * count);
    if (s == PF_OK) s = grow(F->eallocs, (void**)&F->eY, sizeof(double) * per * count);
    if (s == PF_OK) s = grow(F->eallocs, (void**)&F->eP, sizeof(double) * per * count);
    if (s != PF_OK) return s;
    F->ecap = count;
  }
  if (!F->l2_part) {
    pf_status s = falloc(F, (void**)&F->l2_part, sizeof(double) * 2 * kL2Blocks);
    if (s == PF_OK && hipHostMalloc((void**)&F->l2_host, sizeof(double) * 2 * kL2Blocks, 0) != hipSuccess)
      s = PF_ERR_OOM;
    if (s != PF_OK) return s;
  }
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  hipStream_t es = pf::ens_stream(E);
  std::vector<double> t0(count), tf(M);
  for (int i = 0; i < count; ++i) {
    t0[i] = pf::ens_member_time(E, members[i]);
    pf_status s = pf_ensemble_get_state(E, members[i], F->eX + i * per, F->eX + i * per + P, 1);
    if (s != PF_OK) return s;
  }
  double ms_net = 0.0, ms_plain = 0.0;
  std::vector<char> due(count), plainm(count);
  for (int32_t a = 0; a < n_adv; ++a) {
    bool any_net = false, any_plain = false;
    for (int i = 0; i < count; ++i) {
      plainm[i] = st[i].plain_left > 0;
      due[i] = !plainm[i] && st[i].since_check + 1 >= check_every;
      any_net = any_net || !plainm[i];
      any_plain = any_plain || plainm[i] || due[i];
    }
    auto t1 = clk::now();
    if (any_net) {  // every member through the network in one batched pass
      pf_status s = apply_batch(F, F->eX, F->eY, count);
      if (s != PF_OK) return s;
    }
    ms_net += ms_since(t1);
    t1 = clk::now();
    if (any_plain) {  // the checks and the plain intervals: one ensemble advance
      for (int m = 0; m < M; ++m) tf[m] = pf::ens_member_time(E, m);
      for (int i = 0; i < count; ++i) {
        if (!(plainm[i] || due[i])) continue;
        pf_status s = pf::ens_member_set(E, members[i], F->eX + i * per, 0.0);
        if (s != PF_OK) return s;
        tf[members[i]] = delta;
      }
      pf_status s = pf_ensemble_advance(E, tf.data(), 1 << 30, nullptr);
      if (s != PF_OK) return s;
      for (int i = 0; i < count; ++i) {
        if (!(plainm[i] || due[i])) continue;
        s = pf_ensemble_get_state(E, members[i], F->eP + i * per, F->eP + i * per + P, 1);
        if (s != PF_OK) return s;
      }
      FH(hipStreamSynchronize(es));
    }
    for (int i = 0; i < count; ++i) {
      pf_fno_stats& x = st[i];
      const double* src;
      if (plainm[i]) {
        x.plain += 1;
        x.plain_left -= 1;
        src = F->eP + i * per;
      } else {
        x.surrogate += 1;
        x.since_check += 1;
        src = F->eY + i * per;
        if (due[i]) {
          x.since_check = 0;
          x.checks += 1;
          double err = 0.0;
          pf_status s = rel_l2_impl(F->stream, F->eY + i * per, F->eP + i * per, P, F->l2_part, F->l2_host, &err);
          if (s != PF_OK) return s;
          x.err_last = err;
          if (!(err <= x.err_max)) x.err_max = err;
          if (!(err <= tol)) {
            x.fallbacks += 1;
            x.plain_left = check_every;
            src = F->eP + i * per;
          }
        }
      }
      FH(hipMemcpyAsync(F->eX + i * per, src, sizeof(double) * per, hipMemcpyDeviceToDevice, F->stream));
    }
    FH(hipStreamSynchronize(F->stream));
    ms_plain += ms_since(t1);
  }
  for (int i = 0; i < count; ++i) {
    pf_status s = pf::ens_member_set(E, members[i], F->eX + i * per, t0[i] + n_adv * delta);
    if (s != PF_OK) return s;
    st[i].ms_surrogate += ms_net;
    st[i].ms_plain += ms_plain;
  }
  FH(hipStreamSynchronize(es));
  return PF_OK;
}

}  // extern "C"
