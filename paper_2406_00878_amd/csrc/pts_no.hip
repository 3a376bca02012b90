// Spectral neural operator for the learned initial space-time iterate (include/pts_no.h).
//
// Every matrix product runs in k_gemm (the MFMA tile of pts_mfma.hpp): float32 operands in
// memory, rounded to bfloat16 when staged into LDS, multiplied on MFMA 16x16x16 bf16 tiles
// with float32 accumulation. The separable trigonometric transforms of the spectral layers,
// the pointwise channel mixes (with bias and GELU in the epilogue), the projection to the
// temporal modes and all their transposes in the backward pass are strided views of that one
// kernel; reductions over the grid (weight gradients) split K across work-groups and sum the
// partial tiles in fixed order (deterministic). The temporal synthesis and encoding run in
// float32 vector arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/pts_no.h"
#include "pts_mfma.hpp"

namespace pts_no {

using pts_mm::BK;
using pts_mm::BM;
using pts_mm::BN;
using pts_mm::Gemm;
using pts_mm::gelu;

// grid: x = N tiles, y = M tiles, z = batch * ksplit
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  pts_mm::mm_tile(g, blockIdx.y * BM, blockIdx.x * BN, blockIdx.z / g.ksplit, blockIdx.z % g.ksplit);
}

// C_b = alpha * sum_s P[b][s] + beta C_b, summed over s in order
__global__ __launch_bounds__(256) void k_gemm_reduce(Gemm g, int batch) {
  const long total = (long)batch * g.M * g.N;
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long)gridDim.x * 256) {
    const int b = (int)(t / ((long)g.M * g.N));
    const long mn = t % ((long)g.M * g.N);
    const int m = (int)(mn / g.N), n = (int)(mn % g.N);
    float s = 0.f;
    for (int k = 0; k < g.ksplit; ++k) s += g.P[((long)b * g.ksplit + k) * g.M * g.N + mn];
    float* c = g.C + (long)b * g.bsc + (long)m * g.scm + (long)n * g.scn;
    *c = g.alpha * s + (g.beta != 0.f ? g.beta * *c : 0.f);
  }
}

// ------------------------------------------------------------------ elementwise
__device__ __forceinline__ float gelu_grad(float z) {
  const float a = 0.7978845608028654f * (z + 0.044715f * z * z * z);
  const float t = 1.f - 2.f / (expf(2.f * a) + 1.f);
  const float da = 0.7978845608028654f * (1.f + 3.f * 0.044715f * z * z);
  return 0.5f * (1.f + t) + 0.5f * z * (1.f - t * t) * da;
}

// Trigonometric basis phi[i][k] on n periodic nodes x_i = i/n: cos(2 pi k x), k < m;
// sin(2 pi (k - m + 1) x), m <= k < 2m - 1.
__global__ void k_basis(int n, int m, float* phi) {
  const int m2 = 2 * m - 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * m2) return;
  const int i = t / m2, k = t % m2;
  const double x = (double)i / n;
  const double v = k < m ? cos(2.0 * M_PI * k * x) : sin(2.0 * M_PI * (k - m + 1) * x);
  phi[t] = (float)v;
}

// v0[c][p] = lw[c] u0[p] + lb[c]
__global__ void k_lift(int C, long np, const float* __restrict__ lw, const float* __restrict__ lb,
                       const double* __restrict__ u0, float* __restrict__ v0) {
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < C * np; t += (long)gridDim.x * 256) {
    const int c = (int)(t / np);
    v0[t] = lw[c] * (float)u0[t % np] + lb[c];
  }
}

// dz = dy * gelu'(z)
__global__ void k_gelu_back(long n, const float* __restrict__ z, const float* __restrict__ dy,
                            float* __restrict__ dz) {
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) dz[t] = dy[t] * gelu_grad(z[t]);
}

// Spectral mixing: every complex Fourier mode of the band (|kx|, |ky| < m) is multiplied by a
// complex width x width matrix W = alpha + i beta. Coefficients live in the real basis
// (index q = a * m2 + b, row a = y, column b = x; cos k at k, sin k at m - 1 + k). For a
// frequency block kx, ky >= 1 with coefficients A (cos y cos x), B (cos y sin x), C (sin y cos x),
// D (sin y sin x), the amplitudes of exp(i(x + y)) and exp(i(x - y)) are
// (P_c - i P_s) and (M_c - i M_s) with P = ((A - D), (B + C)) / 2, M = ((A + D), (B - C)) / 2;
// multiplying by alpha + i beta maps a pair (c, s) to (alpha c + beta s, alpha s - beta c),
// and A' = P_c' + M_c', D' = M_c' - P_c', B' = P_s' + M_s', C' = P_s' - M_s'. alpha+ / beta+ /
// alpha- / beta- are the matrices R at (cos ky, cos kx) / (cos ky, sin kx) / (sin ky, cos kx) /
// (sin ky, sin kx). A block with one zero frequency is one (cos, sin) pair with alpha at the
// cosine and beta at the sine position; the mean is real.
struct Block {
  int n;       // 1, 2 or 4 coefficients
  int q[4];    // 4: cc, cs, sc, ss; 2: cos, sin; 1: mean
};
__device__ __forceinline__ Block block_of(int m, int ky, int kx) {
  const int m2 = 2 * m - 1;
  Block b;
  if (kx > 0 && ky > 0) {
    b.n = 4;
    b.q[0] = ky * m2 + kx;
    b.q[1] = ky * m2 + (m - 1 + kx);
    b.q[2] = (m - 1 + ky) * m2 + kx;
    b.q[3] = (m - 1 + ky) * m2 + (m - 1 + kx);
  } else if (kx > 0) {
    b.n = 2;
    b.q[0] = kx;
    b.q[1] = m - 1 + kx;
  } else if (ky > 0) {
    b.n = 2;
    b.q[0] = ky * m2;
    b.q[1] = (m - 1 + ky) * m2;
  } else {
    b.n = 1;
    b.q[0] = 0;
  }
  return b;
}

// Sum over the 32 lanes of each half of a wave (the halves stay separate).
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// what = mix(vhat). One wave per (frequency block, pair of output channels): each half of
// the wave takes one output channel and splits the input channels over its 32 lanes.
__global__ __launch_bounds__(256) void k_mix(int C, int m, const float* __restrict__ R, const float* __restrict__ vh,
                                             float* __restrict__ wh) {
  const int nb = m * m, Q = (2 * m - 1) * (2 * m - 1), pairs = C / 2;
  const int gw = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
  if (gw >= nb * pairs) return;  // uniform over the wave
  const int lane = threadIdx.x & 63, l = lane & 31;
  const int blk = gw / pairs, co = 2 * (gw % pairs) + (lane >> 5);
  const Block b = block_of(m, blk / m, blk % m);
  const long CC = (long)C * C;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  for (int c = l; c < C; c += 32) {
    const float* v = vh + (long)c * Q;
    const long o = (long)co * C + c;
    if (b.n == 4) {
      const float A = v[b.q[0]], B = v[b.q[1]], Cc = v[b.q[2]], D = v[b.q[3]];
      const float Pc = 0.5f * (A - D), Ps = 0.5f * (B + Cc), Mc = 0.5f * (A + D), Ms = 0.5f * (B - Cc);
      const float ap = R[b.q[0] * CC + o], bp = R[b.q[1] * CC + o], am = R[b.q[2] * CC + o], bm = R[b.q[3] * CC + o];
      s0 += ap * Pc + bp * Ps;
      s1 += ap * Ps - bp * Pc;
      s2 += am * Mc + bm * Ms;
      s3 += am * Ms - bm * Mc;
    } else if (b.n == 2) {
      const float A = v[b.q[0]], S = v[b.q[1]];
      const float al = R[b.q[0] * CC + o], be = R[b.q[1] * CC + o];
      s0 += al * A + be * S;
      s1 += al * S - be * A;
    } else {
      s0 += R[o] * v[0];
    }
  }
  s0 = half_sum(s0);
  s1 = half_sum(s1);
  s2 = half_sum(s2);
  s3 = half_sum(s3);
  if (l != 0) return;
  float* w = wh + (long)co * Q;
  if (b.n == 4) {  // s0..s3 = P_c', P_s', M_c', M_s'
    w[b.q[0]] = s0 + s2;
    w[b.q[3]] = s2 - s0;
    w[b.q[1]] = s1 + s3;
    w[b.q[2]] = s1 - s3;
  } else if (b.n == 2) {
    w[b.q[0]] = s0;
    w[b.q[1]] = s1;
  } else {
    w[0] = s0;
  }
}

// Adjoint of k_mix: dvhat (written) and dR (accumulated). One wave per (frequency block,
// pair of input channels); the lanes of each half split the output channels, so every dR
// entry has one writer.
__global__ __launch_bounds__(256) void k_mix_back(int C, int m, const float* __restrict__ R,
                                                  const float* __restrict__ vh, const float* __restrict__ dwh,
                                                  float* __restrict__ dvh, float* __restrict__ dR) {
  const int nb = m * m, Q = (2 * m - 1) * (2 * m - 1), pairs = C / 2;
  const int gw = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
  if (gw >= nb * pairs) return;  // uniform over the wave
  const int lane = threadIdx.x & 63, l = lane & 31;
  const int blk = gw / pairs, c = 2 * (gw % pairs) + (lane >> 5);
  const Block b = block_of(m, blk / m, blk % m);
  const long CC = (long)C * C;
  const float* v = vh + (long)c * Q;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
  if (b.n == 4) {
    const float A = v[b.q[0]], B = v[b.q[1]], Cc = v[b.q[2]], D = v[b.q[3]];
    const float Pc = 0.5f * (A - D), Ps = 0.5f * (B + Cc), Mc = 0.5f * (A + D), Ms = 0.5f * (B - Cc);
    for (int co = l; co < C; co += 32) {
      const float* d = dwh + (long)co * Q;
      const float dA = d[b.q[0]], dB = d[b.q[1]], dC = d[b.q[2]], dD = d[b.q[3]];
      const float dPc = dA - dD, dMc = dA + dD, dPs = dB + dC, dMs = dB - dC;
      const long o = (long)co * C + c;
      const float ap = R[b.q[0] * CC + o], bp = R[b.q[1] * CC + o], am = R[b.q[2] * CC + o], bm = R[b.q[3] * CC + o];
      g0 += ap * dPc - bp * dPs;
      g1 += bp * dPc + ap * dPs;
      g2 += am * dMc - bm * dMs;
      g3 += bm * dMc + am * dMs;
      dR[b.q[0] * CC + o] += dPc * Pc + dPs * Ps;
      dR[b.q[1] * CC + o] += dPc * Ps - dPs * Pc;
      dR[b.q[2] * CC + o] += dMc * Mc + dMs * Ms;
      dR[b.q[3] * CC + o] += dMc * Ms - dMs * Mc;
    }
  } else if (b.n == 2) {
    const float A = v[b.q[0]], S = v[b.q[1]];
    for (int co = l; co < C; co += 32) {
      const float* d = dwh + (long)co * Q;
      const float dA = d[b.q[0]], dS = d[b.q[1]];
      const long o = (long)co * C + c;
      const float al = R[b.q[0] * CC + o], be = R[b.q[1] * CC + o];
      g0 += al * dA - be * dS;
      g1 += be * dA + al * dS;
      dR[b.q[0] * CC + o] += dA * A + dS * S;
      dR[b.q[1] * CC + o] += dA * S - dS * A;
    }
  } else {
    const float A = v[0];
    for (int co = l; co < C; co += 32) {
      const long o = (long)co * C + c;
      g0 += R[o] * dwh[(long)co * Q];
      dR[o] += dwh[(long)co * Q] * A;
    }
  }
  g0 = half_sum(g0);
  g1 = half_sum(g1);
  g2 = half_sum(g2);
  g3 = half_sum(g3);
  if (l != 0) return;
  float* dv = dvh + (long)c * Q;
  if (b.n == 4) {  // g0..g3 = gradients of P_c, P_s, M_c, M_s
    dv[b.q[0]] = 0.5f * (g0 + g2);
    dv[b.q[3]] = 0.5f * (g2 - g0);
    dv[b.q[1]] = 0.5f * (g1 + g3);
    dv[b.q[2]] = 0.5f * (g1 - g3);
  } else if (b.n == 2) {
    dv[b.q[0]] = g0;
    dv[b.q[1]] = g1;
  } else {
    dv[0] = g0;
  }
}

constexpr int kMaxT = 64;  // temporal modes

// Temporal basis: Phi [nt][K] (float32) = Q of the thin QR of S[n][k] = sin(pi (k + 1/2)(n + 1) / nt)
// with a positive diagonal of R, formed as Cholesky QR in float64 (S^T S = L L^T, Q = S L^-T):
// the sines are close to orthogonal, so the Gram matrix is well conditioned. One work-group;
// S64 is [nt][K] float64 scratch.
__global__ __launch_bounds__(256) void k_tbasis(int nt, int K, double* __restrict__ S64, float* __restrict__ phi) {
  __shared__ double G[kMaxT][kMaxT + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nt * K; e += 256) {
    const int n = e / K, k = e % K;
    S64[e] = sin(M_PI * (k + 0.5) * (double)(n + 1) / (double)nt);
  }
  __syncthreads();
  for (int e = tid; e < K * K; e += 256) {
    const int a = e / K, b = e % K;
    if (a > b) continue;
    double g = 0.0;
    for (int n = 0; n < nt; ++n) g += S64[(long)n * K + a] * S64[(long)n * K + b];
    G[a][b] = g;
    G[b][a] = g;
  }
  __syncthreads();
  // Cholesky G = L L^T in place (lower triangle), column by column
  for (int j = 0; j < K; ++j) {
    if (tid == 0) {
      double d = G[j][j];
      for (int k = 0; k < j; ++k) d -= G[j][k] * G[j][k];
      G[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < K; i += 256) {
      double v = G[i][j];
      for (int k = 0; k < j; ++k) v -= G[i][k] * G[j][k];
      G[i][j] = v / G[j][j];
    }
    __syncthreads();
  }
  // rows of Q: L q = s (forward substitution), in place in S64
  for (int n = tid; n < nt; n += 256) {
    double* r = S64 + (long)n * K;
    for (int k = 0; k < K; ++k) {
      double v = r[k];
      for (int j = 0; j < k; ++j) v -= G[k][j] * r[j];
      r[k] = v / G[k][k];
      phi[(long)n * K + k] = (float)r[k];
    }
  }
}

// U[n][p] = u0[p] + sum_k Phi[n][k] (coef[k][p] + pb[k]) in float32, stored as float64.
// grid: x over points (grid-stride), y over chunks of kSynthLevels levels; the chunk's rows
// of Phi are staged in LDS.
// KT > 0 fixes K at compile time (no per-mode guards); KT = 0 is the generic form.
constexpr int kSynthLevels = 32;
template <int KT>
__global__ __launch_bounds__(256) void k_synth(int nt, int K, long np, const double* __restrict__ u0,
                                               const float* __restrict__ coef, const float* __restrict__ pb,
                                               const float* __restrict__ phi, double* __restrict__ U) {
  __shared__ float ph[kSynthLevels * kMaxT];
  const int n0 = blockIdx.y * kSynthLevels, n1 = min(nt, n0 + kSynthLevels);
  for (int e = threadIdx.x; e < (n1 - n0) * K; e += 256) ph[e] = phi[(long)n0 * K + e];
  __syncthreads();
  for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < np; p += (long)gridDim.x * 256) {
    constexpr int KM = KT ? KT : kMaxT;
    float c[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) c[k] = (KT || k < K) ? coef[(long)k * np + p] + pb[k] : 0.f;
    const double base = u0[p];
    for (int n = n0; n < n1; ++n) {
      const float* f = ph + (n - n0) * K;
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (KT || k < K) acc += f[k] * c[k];
      U[(long)n * np + p] = base + (double)acc;
    }
  }
}

// out[k][p] = scale * sum_n Phi[n][k] (A[n][p] - B[p or n][p]); with DIFF, B is [nt][np] and
// the block partial sums of (A - B)^2 go to part[blockIdx.x]; else B is u0 [np].
// 128 threads per block, grid-stride over points.
template <bool DIFF, int KT>
__global__ __launch_bounds__(128) void k_encode(int nt, int K, long np, const double* __restrict__ A,
                                                const double* __restrict__ B, const float* __restrict__ phi,
                                                float scale, float* __restrict__ out, double* __restrict__ part) {
  double lsum = 0.0;
  for (long p = (long)blockIdx.x * 128 + threadIdx.x; p < np; p += (long)gridDim.x * 128) {
    constexpr int KM = KT ? KT : kMaxT;
    float acc[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) acc[k] = 0.f;
    for (int n = 0; n < nt; ++n) {
      const double d = A[(long)n * np + p] - (DIFF ? B[(long)n * np + p] : B[p]);
      if (DIFF) lsum += d * d;
      const float df = (float)d;
      const float* f = phi + (long)n * K;
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (KT || k < K) acc[k] += f[k] * df;
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (KT || k < K) out[(long)k * np + p] = scale * acc[k];
  }
  if (DIFF) {
    __shared__ double red[128];
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int o = 64; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  }
}

// d = coef + pb - ctrue; dcoef = scale d; block partial sums of d^2 into part
__global__ __launch_bounds__(256) void k_coef_diff(int K, long np, const float* __restrict__ coef,
                                                   const float* __restrict__ pb, const float* __restrict__ ct,
                                                   float scale, float* __restrict__ dcoef,
                                                   double* __restrict__ part) {
  double acc = 0.0;
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < (long)K * np; t += (long)gridDim.x * 256) {
    const float d = coef[t] + pb[t / np] - ct[t];
    dcoef[t] = scale * d;
    acc += (double)d * (double)d;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// loss[0] += sum(part) / n: one work-group of 256, strided partial sums then a fixed tree
// (deterministic)
__global__ __launch_bounds__(256) void k_mse_finish(int nb, long n, const double* __restrict__ part,
                                                    double* __restrict__ loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] += red[0] / (double)n;
}

// Row sums (W == nullptr) or row dot products with a float64 vector w of a [rows][len] float
// array, in two passes: grid (kRowSlices, rows) writes per-slice partials to part, then
// k_row_fold adds each row's partials in order into out[row] (accumulated).
constexpr int kRowSlices = 64;
__global__ __launch_bounds__(256) void k_row_partial(long len, const float* __restrict__ a,
                                                     const double* __restrict__ w, float* __restrict__ part) {
  const int row = blockIdx.y, sl = blockIdx.x;
  const long chunk = (len + kRowSlices - 1) / kRowSlices;
  const long beg = (long)sl * chunk, end = min(len, beg + chunk);
  const float* r = a + (long)row * len;
  float s = 0.f;
  for (long t = beg + threadIdx.x; t < end; t += 256) s += w ? r[t] * (float)w[t] : r[t];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)row * kRowSlices + sl] = red[0];
}
__global__ void k_row_fold(int rows, const float* __restrict__ part, float* __restrict__ out) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  float s = 0.f;
  for (int i = 0; i < kRowSlices; ++i) s += part[(long)row * kRowSlices + i];
  out[row] += s;
}

__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float gs, float c1, float c2) {
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long)gridDim.x * 256) {
    const float gt = g[t] * gs;
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
  }
}


}  // namespace pts_no

using namespace pts_no;

namespace pts_internal {
void set_error(const char* msg);  // shared with pts_last_error (pts_api.hip)
}

namespace {

int nofail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  pts_internal::set_error(buf);
  return code;
}

#define NOCHK(expr)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) return nofail(PTS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int valid(const pts_no_config* c) {
  if (!c) return nofail(PTS_ERR_INVALID_ARG, "config is NULL");
  if (c->nx < 4 || c->ny < 4 || c->nt < 1) return nofail(PTS_ERR_INVALID_ARG, "grid/levels");
  if ((long long)c->nx * c->ny > (1ll << 24)) return nofail(PTS_ERR_INVALID_ARG, "grid too large");
  if (c->width < 16 || c->width > 64 || c->width % 16) return nofail(PTS_ERR_INVALID_ARG, "width %d", c->width);
  if (c->modes < 1 || c->modes > 32 || 2 * c->modes > std::min(c->nx, c->ny))
    return nofail(PTS_ERR_INVALID_ARG, "modes %d", c->modes);
  if (c->layers < 1 || c->layers > 8) return nofail(PTS_ERR_INVALID_ARG, "layers %d", c->layers);
  if (c->tmodes < 1 || c->tmodes > kMaxT || c->tmodes > c->nt)
    return nofail(PTS_ERR_INVALID_ARG, "tmodes %d", c->tmodes);
  return PTS_OK;
}

// parameter offsets (floats)
struct Par {
  size_t lw, lb, W[8], b[8], R[8], pw, pb, total;
};
Par par_layout(const pts_no_config* c) {
  Par P;
  const size_t C = c->width, Q = (size_t)(2 * c->modes - 1) * (2 * c->modes - 1);
  size_t o = 0;
  P.lw = o;
  o += C;
  P.lb = o;
  o += C;
  for (int l = 0; l < c->layers; ++l) {
    P.W[l] = o;
    o += C * C;
    P.b[l] = o;
    o += C;
    P.R[l] = o;
    o += Q * C * C;
  }
  P.pw = o;
  o += (size_t)c->tmodes * C;
  P.pb = o;
  o += c->tmodes;
  P.total = o;
  return P;
}

// workspace offsets (bytes, 256-aligned)
struct Ws {
  size_t phix, phiy, tphi, s64, v, z, vh, wh, t1, t2, coef, dcoef, dv, dv2, dz, dvh, dwh, part, gpart, tpart, rpart,
      total;
};
size_t al(size_t v) { return (v + 255) / 256 * 256; }
constexpr int kSplit = 32;
// K split of a product with `tiles` output tiles (all batches) and depth K: enough work-groups
// for two per compute unit, at least one K step of BK each, at most 16 ranges
int split_of(long tiles, int K) {
  const long want = (512 + tiles - 1) / tiles;
  return (int)std::max(1L, std::min({want, (long)(K / BK), 16L}));
}
long tiles_of(int M, int N, int batch) { return (long)((M + BM - 1) / BM) * ((N + BN - 1) / BN) * batch; }
constexpr int kPartSlots = 4096;  // loss partial sums (one per block of the loss kernels)
// B > 1: the forward buffers (activations, modes, coefficient fields, transform partials) of
// B samples at once (pts_no_forward_batched); the basis tables sit at the same offsets for
// every B, so one preparation serves either form.
Ws ws_layout(const pts_no_config* c, int B = 1) {
  Ws w;
  const size_t C = c->width, np = (size_t)c->nx * c->ny, m2 = 2 * c->modes - 1, Q = m2 * m2;
  const size_t CB = C * B;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = al(o + bytes);
    return at;
  };
  w.phix = take(c->nx * m2 * 4);
  w.phiy = take(c->ny * m2 * 4);
  w.tphi = take((size_t)c->nt * c->tmodes * 4);
  w.s64 = take((size_t)c->nt * c->tmodes * 8);
  w.v = take((c->layers + 1) * CB * np * 4);
  w.z = take(c->layers * CB * np * 4);
  w.vh = take(c->layers * CB * Q * 4);
  w.wh = take(CB * Q * 4);
  w.t1 = take(CB * c->ny * m2 * 4);
  w.t2 = take(CB * c->ny * m2 * 4);
  w.coef = take((size_t)B * c->tmodes * np * 4);
  w.dcoef = take((size_t)c->tmodes * np * 4);
  w.dv = take(C * np * 4);
  w.dv2 = take(C * np * 4);
  w.dz = take(C * np * 4);
  w.dvh = take(C * Q * 4);
  w.dwh = take(C * Q * 4);
  w.part = take(kPartSlots * 8);
  w.gpart = take((size_t)kSplit * std::max((size_t)c->tmodes, C) * C * 4);
  {  // partials of the two products onto the modes (x direction, then y direction per channel)
    const int M1 = (int)CB * c->ny, M2 = (int)m2;
    const size_t p1 = (size_t)split_of(tiles_of(M1, (int)m2, 1), c->nx) * M1 * m2;
    const size_t p2 = (size_t)split_of(tiles_of(M2, M2, (int)CB), c->ny) * CB * Q;
    w.tpart = take(std::max(p1, p2) * 4);
  }
  w.rpart = take((size_t)kMaxT * kRowSlices * 4);
  w.total = o;
  return w;
}

// out[row] += sum_t a[row][t] (w[t]) for rows x len (w may be NULL); part holds rows * kRowSlices floats
void row_reduce(hipStream_t s, int rows, long len, const float* a, const double* w, float* part, float* out) {
  hipLaunchKernelGGL(k_row_partial, dim3(kRowSlices, rows), dim3(256), 0, s, len, a, w, part);
  hipLaunchKernelGGL(k_row_fold, dim3((rows + 63) / 64), dim3(64), 0, s, rows, part, out);
}

// launches of k_synth / k_encode with the mode count fixed at compile time where it is 8, 16 or 32
void launch_synth(hipStream_t s, dim3 grid, int nt, int K, long np, const double* u0, const float* coef,
                  const float* pb, const float* phi, double* U) {
  auto k = K == 8 ? k_synth<8> : K == 16 ? k_synth<16> : K == 32 ? k_synth<32> : k_synth<0>;
  hipLaunchKernelGGL(k, grid, dim3(256), 0, s, nt, K, np, u0, coef, pb, phi, U);
}
template <bool DIFF>
void launch_encode(hipStream_t s, unsigned blocks, int nt, int K, long np, const double* A, const double* B,
                   const float* phi, float scale, float* out, double* part) {
  auto k = K == 8 ? k_encode<DIFF, 8> : K == 16 ? k_encode<DIFF, 16> : K == 32 ? k_encode<DIFF, 32> : k_encode<DIFF, 0>;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(128), 0, s, nt, K, np, A, B, phi, scale, out, part);
}

// work-groups of k_mix / k_mix_back: one wave per (frequency block, channel pair), 4 per group
unsigned mix_blocks(int C, int m) { return (unsigned)((m * m * (C / 2) + 3) / 4); }

unsigned eblocks(long n) { return (unsigned)std::min<long>((n + 255) / 256, 8192); }

// C = alpha op(A) op(B) + beta C via k_gemm; ksplit > 1 needs P scratch
int gemm(hipStream_t s, int M, int N, int K, float alpha, const float* A, long sam, long sak, long bsa,
         const float* B, long sbk, long sbn, long bsb, float beta, float* C, long scm, long scn, long bsc,
         int batch = 1, int ksplit = 1, float* P = nullptr, const float* bias = nullptr, float* act = nullptr) {
  Gemm g{A, B, C, M, N, K, sam, sak, bsa, sbk, sbn, bsb, scm, scn, bsc, alpha, beta, ksplit, P, bias, act};
  dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)(batch * ksplit));
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
  if (ksplit > 1) hipLaunchKernelGGL(k_gemm_reduce, dim3(eblocks((long)batch * M * N)), dim3(256), 0, s, g, batch);
  NOCHK(hipGetLastError());
  return PTS_OK;
}

struct Net {
  const pts_no_config* c;
  Par P;
  Ws W;
  char* ws;
  int C, CB, nx, ny, m2, Q;  // CB: channels of all samples of a batched forward (C otherwise)
  long np;
  float* f(size_t off) const { return (float*)(ws + off); }
  float* v(int l) const { return f(W.v) + (size_t)l * CB * np; }
  float* z(int l) const { return f(W.z) + (size_t)l * CB * np; }
  float* vh(int l) const { return f(W.vh) + (size_t)l * CB * Q; }
  void bind(const pts_no_config* cfg, void* w, int B = 1) {
    c = cfg;
    P = par_layout(cfg);
    W = ws_layout(cfg, B);
    ws = (char*)w;
    C = cfg->width;
    CB = C * B;
    nx = cfg->nx;
    ny = cfg->ny;
    m2 = 2 * cfg->modes - 1;
    Q = m2 * m2;
    np = (long)nx * ny;
  }
  // out = alpha phiy^T v phix for the C channels of v [C][ny][nx]; both products are deep
  // in K (nx, ny) with few output tiles, so they run split in K (partials summed in order)
  int to_modes(hipStream_t s, const float* vin, float* out, float alpha) {
    const float* phix = f(W.phix);
    const float* phiy = f(W.phiy);
    float* t1 = f(W.t1);
    float* tp = f(W.tpart);
    int rc = gemm(s, CB * ny, m2, nx, 1.f, vin, nx, 1, 0, phix, m2, 1, 0, 0.f, t1, m2, 1, 0, 1,
                  split_of(tiles_of(CB * ny, m2, 1), nx), tp);
    if (rc) return rc;
    return gemm(s, m2, m2, ny, alpha, phiy, 1, m2, 0, t1, m2, 1, (long)ny * m2, 0.f, out, m2, 1, Q, CB,
                split_of(tiles_of(m2, m2, CB), ny), tp);
  }
  // vh = (1/np) phiy^T v phix
  int forward_transform(hipStream_t s, const float* vin, float* vhat) { return to_modes(s, vin, vhat, 1.f / (float)np); }
  // out (+)= phiy what phix^T for C channels; beta = 0 writes, 1 accumulates
  int inverse_transform(hipStream_t s, const float* what, float* out, float beta) {
    const float* phix = f(W.phix);
    const float* phiy = f(W.phiy);
    float* t2 = f(W.t2);
    int rc = gemm(s, ny, m2, m2, 1.f, phiy, m2, 1, 0, what, m2, 1, Q, 0.f, t2, m2, 1, (long)ny * m2, CB);
    if (rc) return rc;
    return gemm(s, CB * ny, nx, m2, 1.f, t2, m2, 1, 0, phix, 1, m2, 0, beta, out, nx, 1, 0);
  }
  // gradients of a loss from dcoef = dL/dc (workspace) back through the network, accumulated
  int backward_from_coef(hipStream_t s, const float* params, const double* u0, float* grads) {
    int rc;
    const int K = c->tmodes;
    float* dco = f(W.dcoef);
    float* gp = f(W.gpart);
    float* vL = v(c->layers);
    // projection: dpw += dcoef v_L^T (K = np, split), dpb += rowsum(dcoef), dv = pw^T dcoef
    if ((rc = gemm(s, K, C, (int)np, 1.f, dco, np, 1, 0, vL, 1, np, 0, 1.f, grads + P.pw, C, 1, 0, 1, kSplit, gp)))
      return rc;
    row_reduce(s, K, np, dco, nullptr, f(W.rpart), grads + P.pb);
    float* dv = f(W.dv);
    float* dv2 = f(W.dv2);
    float* dz = f(W.dz);
    if ((rc = gemm(s, C, (int)np, K, 1.f, params + P.pw, 1, C, 0, dco, np, 1, 0, 0.f, dv, np, 1, 0))) return rc;
    const float* phix = f(W.phix);
    const float* phiy = f(W.phiy);
    for (int l = c->layers - 1; l >= 0; --l) {
      float* vin = v(l);
      hipLaunchKernelGGL(k_gelu_back, dim3(eblocks(C * np)), dim3(256), 0, s, C * np, z(l), dv, dz);
      row_reduce(s, C, np, dz, nullptr, f(W.rpart), grads + P.b[l]);
      // dW += dz v^T ; dv2 = W^T dz
      if ((rc = gemm(s, C, C, (int)np, 1.f, dz, np, 1, 0, vin, 1, np, 0, 1.f, grads + P.W[l], C, 1, 0, 1, kSplit,
                     gp)))
        return rc;
      if ((rc = gemm(s, C, (int)np, C, 1.f, params + P.W[l], 1, C, 0, dz, np, 1, 0, 0.f, dv2, np, 1, 0))) return rc;
      // spectral branch: dwhat = phiy^T dz phix (adjoint of the inverse transform)
      if ((rc = to_modes(s, dz, f(W.dwh), 1.f))) return rc;
      hipLaunchKernelGGL(k_mix_back, dim3(mix_blocks(C, c->modes)), dim3(256), 0, s, C, c->modes,
                         params + P.R[l], vh(l),
                         f(W.dwh), f(W.dvh), grads + P.R[l]);
      // dv2 += (1/np) phiy dvhat phix^T (adjoint of the forward transform)
      float* t2 = f(W.t2);
      if ((rc = gemm(s, ny, m2, m2, 1.f / (float)np, phiy, m2, 1, 0, f(W.dvh), m2, 1, Q, 0.f, t2, m2, 1,
                     (long)ny * m2, C)))
        return rc;
      if ((rc = gemm(s, C * ny, nx, m2, 1.f, t2, m2, 1, 0, phix, 1, m2, 0, 1.f, dv2, nx, 1, 0))) return rc;
      std::swap(dv, dv2);
    }
    // lift: dlw += sum_p dv0 u0, dlb += sum_p dv0
    row_reduce(s, C, np, dv, u0, f(W.rpart), grads + P.lw);
    row_reduce(s, C, np, dv, nullptr, f(W.rpart), grads + P.lb);
    NOCHK(hipGetLastError());
    return PTS_OK;
  }
};

}  // namespace

extern "C" {

size_t pts_no_param_count(const pts_no_config* cfg) {
  if (valid(cfg)) return 0;
  return par_layout(cfg).total;
}

size_t pts_no_workspace_bytes(const pts_no_config* cfg) {
  if (valid(cfg)) return 0;
  return ws_layout(cfg).total;
}

int pts_no_prepare(const pts_no_config* cfg, void* workspace, size_t workspace_bytes, pts_stream_t stream) {
  int rc = valid(cfg);
  if (rc) return rc;
  if (!workspace) return nofail(PTS_ERR_INVALID_ARG, "pts_no_prepare: NULL");
  if (workspace_bytes < ws_layout(cfg).total) return nofail(PTS_ERR_WORKSPACE, "pts_no_prepare: workspace");
  hipStream_t s = (hipStream_t)stream;
  Net n;
  n.bind(cfg, workspace);
  hipLaunchKernelGGL(k_basis, dim3((n.nx * n.m2 + 255) / 256), dim3(256), 0, s, n.nx, cfg->modes, n.f(n.W.phix));
  hipLaunchKernelGGL(k_basis, dim3((n.ny * n.m2 + 255) / 256), dim3(256), 0, s, n.ny, cfg->modes, n.f(n.W.phiy));
  hipLaunchKernelGGL(k_tbasis, dim3(1), dim3(256), 0, s, cfg->nt, cfg->tmodes, (double*)(n.ws + n.W.s64),
                     n.f(n.W.tphi));
  NOCHK(hipGetLastError());
  return PTS_OK;
}

int pts_no_gemm(int M, int N, int K, float alpha, const float* A, long sam, long sak, long bsa, const float* B,
                long sbk, long sbn, long bsb, float beta, float* C, long scm, long scn, long bsc, int batch,
                pts_stream_t stream) {
  if (M < 1 || N < 1 || K < 1 || batch < 1 || !A || !B || !C) return nofail(PTS_ERR_INVALID_ARG, "pts_no_gemm");
  return gemm((hipStream_t)stream, M, N, K, alpha, A, sam, sak, bsa, B, sbk, sbn, bsb, beta, C, scm, scn, bsc,
              batch);
}

int pts_no_forward(const pts_no_config* cfg, const float* params, const double* u0, double* U_pred, void* workspace,
                   size_t workspace_bytes, pts_stream_t stream) {
  int rc = valid(cfg);
  if (rc) return rc;
  if (!params || !u0 || !workspace) return nofail(PTS_ERR_INVALID_ARG, "pts_no_forward: NULL");
  if (workspace_bytes < ws_layout(cfg).total) return nofail(PTS_ERR_WORKSPACE, "pts_no_forward: workspace");
  hipStream_t s = (hipStream_t)stream;
  Net n;
  n.bind(cfg, workspace);
  const int C = n.C;
  const long np = n.np;
  hipLaunchKernelGGL(k_lift, dim3(eblocks(C * np)), dim3(256), 0, s, C, np, params + n.P.lw, params + n.P.lb, u0,
                     n.v(0));
  for (int l = 0; l < cfg->layers; ++l) {
    float* vin = n.v(l);
    float* z = n.z(l);
    // spectral part into z, then z += W v (pointwise channel mix)
    if ((rc = n.forward_transform(s, vin, n.vh(l)))) return rc;
    hipLaunchKernelGGL(k_mix, dim3(mix_blocks(C, cfg->modes)), dim3(256), 0, s, C, cfg->modes,
                       params + n.P.R[l], n.vh(l),
                       n.f(n.W.wh));
    if ((rc = n.inverse_transform(s, n.f(n.W.wh), z, 0.f))) return rc;
    // z += W v + b, v_{l+1} = GELU(z) in the product's epilogue
    if ((rc = gemm(s, C, (int)np, C, 1.f, params + n.P.W[l], C, 1, 0, vin, np, 1, 0, 1.f, z, np, 1, 0, 1, 1, nullptr,
                   params + n.P.b[l], n.v(l + 1))))
      return rc;
  }
  // coefficient fields coef[K][np] = pw v_L (bias added by the consumers)
  if ((rc = gemm(s, cfg->tmodes, (int)np, C, 1.f, params + n.P.pw, C, 1, 0, n.v(cfg->layers), np, 1, 0, 0.f,
                 n.f(n.W.coef), np, 1, 0)))
    return rc;
  if (U_pred) {
    dim3 grid(std::min<unsigned>((unsigned)((np + 255) / 256), 2048u),
              (unsigned)((cfg->nt + kSynthLevels - 1) / kSynthLevels));
    launch_synth(s, grid, cfg->nt, cfg->tmodes, np, u0, n.f(n.W.coef), params + n.P.pb, n.f(n.W.tphi), U_pred);
  }
  NOCHK(hipGetLastError());
  return PTS_OK;
}

size_t pts_no_workspace_bytes_batched(const pts_no_config* cfg, int batch) {
  if (valid(cfg) || batch < 1) return 0;
  return ws_layout(cfg, batch).total;
}

int pts_no_forward_batched(const pts_no_config* cfg, const float* params, int batch, const double* const* u0,
                           double* const* U_pred, void* workspace, size_t workspace_bytes, pts_stream_t stream) {
  int rc = valid(cfg);
  if (rc) return rc;
  if (batch < 1 || !params || !u0 || !U_pred || !workspace)
    return nofail(PTS_ERR_INVALID_ARG, "pts_no_forward_batched: NULL or empty batch");
  for (int b = 0; b < batch; ++b)
    if (!u0[b] || !U_pred[b]) return nofail(PTS_ERR_INVALID_ARG, "pts_no_forward_batched: sample %d: NULL", b);
  if (workspace_bytes < ws_layout(cfg, batch).total)
    return nofail(PTS_ERR_WORKSPACE, "pts_no_forward_batched: workspace");
  hipStream_t s = (hipStream_t)stream;
  Net n;
  n.bind(cfg, workspace, batch);
  const int C = n.C;
  const long np = n.np, cnp = (long)C * np;
  const long cq = (long)C * n.Q;
  const int K = cfg->tmodes;
  // activations of sample b at channel offset b C: the transforms run over all B C channels,
  // the channel mixes as B products sharing the weights
  for (int b = 0; b < batch; ++b)
    hipLaunchKernelGGL(k_lift, dim3(eblocks(C * np)), dim3(256), 0, s, C, np, params + n.P.lw, params + n.P.lb, u0[b],
                       n.v(0) + b * cnp);
  for (int l = 0; l < cfg->layers; ++l) {
    float* vin = n.v(l);
    float* z = n.z(l);
    if ((rc = n.forward_transform(s, vin, n.vh(l)))) return rc;
    for (int b = 0; b < batch; ++b)
      hipLaunchKernelGGL(k_mix, dim3(mix_blocks(C, cfg->modes)), dim3(256), 0, s, C, cfg->modes, params + n.P.R[l],
                         n.vh(l) + b * cq, n.f(n.W.wh) + b * cq);
    if ((rc = n.inverse_transform(s, n.f(n.W.wh), z, 0.f))) return rc;
    if ((rc = gemm(s, C, (int)np, C, 1.f, params + n.P.W[l], C, 1, 0, vin, np, 1, cnp, 1.f, z, np, 1, cnp, batch, 1,
                   nullptr, params + n.P.b[l], n.v(l + 1))))
      return rc;
  }
  if ((rc = gemm(s, K, (int)np, C, 1.f, params + n.P.pw, C, 1, 0, n.v(cfg->layers), np, 1, cnp, 0.f, n.f(n.W.coef),
                 np, 1, (long)K * np, batch)))
    return rc;
  dim3 grid(std::min<unsigned>((unsigned)((np + 255) / 256), 2048u),
            (unsigned)((cfg->nt + kSynthLevels - 1) / kSynthLevels));
  for (int b = 0; b < batch; ++b)
    launch_synth(s, grid, cfg->nt, K, np, u0[b], n.f(n.W.coef) + (size_t)b * K * np, params + n.P.pb, n.f(n.W.tphi),
                 U_pred[b]);
  NOCHK(hipGetLastError());
  return PTS_OK;
}

int pts_no_backward(const pts_no_config* cfg, const float* params, const double* u0, const double* U_pred,
                    const double* U_true, float* grads, double* loss, void* workspace, size_t workspace_bytes,
                    pts_stream_t stream) {
  int rc = valid(cfg);
  if (rc) return rc;
  if (!params || !u0 || !U_pred || !U_true || !grads || !loss || !workspace)
    return nofail(PTS_ERR_INVALID_ARG, "pts_no_backward: NULL");
  if (workspace_bytes < ws_layout(cfg).total) return nofail(PTS_ERR_WORKSPACE, "pts_no_backward: workspace");
  hipStream_t s = (hipStream_t)stream;
  Net n;
  n.bind(cfg, workspace);
  const long count = (long)cfg->nt * n.np;
  // dL/dc = Phi^T dL/dU with dL/dU = 2 (U_pred - U_true) / count; loss partials alongside
  double* part = (double*)(n.ws + n.W.part);
  const unsigned eb = (unsigned)std::min<long>((n.np + 127) / 128, kPartSlots);
  launch_encode<true>(s, eb, cfg->nt, cfg->tmodes, n.np, U_pred, U_true, n.f(n.W.tphi), (float)(2.0 / (double)count),
                      n.f(n.W.dcoef), part);
  hipLaunchKernelGGL(k_mse_finish, dim3(1), dim3(256), 0, s, (int)eb, count, part, loss);
  NOCHK(hipGetLastError());
  return n.backward_from_coef(s, params, u0, grads);
}

int pts_no_backward_coef(const pts_no_config* cfg, const float* params, const double* u0, const float* coef_true,
                         float* grads, double* loss, void* workspace, size_t workspace_bytes, pts_stream_t stream) {
  int rc = valid(cfg);
  if (rc) return rc;
  if (!params || !u0 || !coef_true || !grads || !loss || !workspace)
    return nofail(PTS_ERR_INVALID_ARG, "pts_no_backward_coef: NULL");
  if (workspace_bytes < ws_layout(cfg).total) return nofail(PTS_ERR_WORKSPACE, "pts_no_backward_coef: workspace");
  hipStream_t s = (hipStream_t)stream;
  Net n;
  n.bind(cfg, workspace);
  const long count = (long)cfg->nt * n.np;
  double* part = (double*)(n.ws + n.W.part);
  const unsigned eb = std::min<unsigned>(eblocks((long)cfg->tmodes * n.np), kPartSlots);
  hipLaunchKernelGGL(k_coef_diff, dim3(eb), dim3(256), 0, s, cfg->tmodes, n.np, n.f(n.W.coef), params + n.P.pb,
                     coef_true, (float)(2.0 / (double)count), n.f(n.W.dcoef), part);
  hipLaunchKernelGGL(k_mse_finish, dim3(1), dim3(256), 0, s, (int)eb, count, part, loss);
  NOCHK(hipGetLastError());
  return n.backward_from_coef(s, params, u0, grads);
}

int pts_no_encode(const pts_no_config* cfg, const double* u0, const double* U, float* coef, void* workspace,
                  size_t workspace_bytes, pts_stream_t stream) {
  int rc = valid(cfg);
  if (rc) return rc;
  if (!u0 || !U || !coef || !workspace) return nofail(PTS_ERR_INVALID_ARG, "pts_no_encode: NULL");
  if (workspace_bytes < ws_layout(cfg).total) return nofail(PTS_ERR_WORKSPACE, "pts_no_encode: workspace");
  hipStream_t s = (hipStream_t)stream;
  Net n;
  n.bind(cfg, workspace);
  const unsigned eb = (unsigned)std::min<long>((n.np + 127) / 128, 8192);
  launch_encode<false>(s, eb, cfg->nt, cfg->tmodes, n.np, U, u0, n.f(n.W.tphi), 1.f, coef, nullptr);
  NOCHK(hipGetLastError());
  return PTS_OK;
}

int pts_no_adam(size_t n, float* params, const float* grads, float* m, float* v, int step, float lr, float beta1,
                float beta2, float eps, float grad_scale, pts_stream_t stream) {
  if (!params || !grads || !m || !v || step < 1 || n == 0) return nofail(PTS_ERR_INVALID_ARG, "pts_no_adam");
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(eblocks((long)n)), dim3(256), 0, (hipStream_t)stream, (long)n, params, grads, m, v,
                     lr, beta1, beta2, eps, grad_scale, c1, c2);
  NOCHK(hipGetLastError());
  return PTS_OK;
}

}  // extern "C"
