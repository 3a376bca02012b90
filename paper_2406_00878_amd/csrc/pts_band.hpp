// Banded direct level solves without pivoting (Section 8: the paper solves each level's
// linear system by a direct solver for banded matrices without pivoting).
//
// For a Dirichlet problem in the x-fastest ordering of Section 3 the block A_n couples node i
// to i +- 1 and i +- nx: a band of half-width w = nx. It is factorised A_n = L_n U_n (L unit
// lower) without pivoting, in place in band storage B[row][w + col - row] (2w + 1 entries per
// row, zero outside the matrix). The levels' factorisations are independent (one work-group
// each, all levels in one launch); Eq. (7) then runs as a chain of forward and backward
// substitutions, level after level, du^n = U_n^{-1} L_n^{-1} (r^n + du^{n-1}).
//
// Used where the Chebyshev level solves have no convergence bound: blocks that are not
// diagonally dominant, or whose Jacobi iteration matrix may have complex eigenvalues of
// modulus above 1/sqrt(2) (central convection at cell Peclet numbers above 2).
#pragma once
#include <hip/hip_runtime.h>

#include "pts_device.hpp"

namespace pts {

constexpr int kBandMaxW = 64;  // half-bandwidth (nx) the band kernels handle

// Factorisation of level n = blockIdx.x: assemble the rows of A_n(U^n) (eval_point), then
// right-looking LU over a window of w + 1 rows held in LDS (row r in slot r % (w + 1)): at
// pivot k the rows k+1..k+w take their multipliers and the update from row k, row k goes to
// device memory and row k + w + 1 comes in. status[n] = 1 when a pivot is zero or not finite.
template <int FORM>
__global__ __launch_bounds__(256) void k_band_factor(KProb p0, const double* __restrict__ U, double* __restrict__ B,
                                                     int* __restrict__ status) {
  const int n = blockIdx.x;
  const KProb p = at_level(p0, n);
  const int nx = p.nx, ny = p.ny, w = nx, ld = 2 * w + 1, S = w + 1;
  const int ns = nx * ny;
  double* __restrict__ Bn = B + (size_t)n * ns * ld;
  const double* un = U + (size_t)n * ns;
  const double* bd = p.bdata ? p.bdata + (size_t)n * 2 * (nx + ny) : nullptr;
  for (size_t t = threadIdx.x; t < (size_t)ns * ld; t += blockDim.x) Bn[t] = 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const int x = i % nx, y = i / nx;
    const Nb u = gather<0>(p, un, bd, x, y);
    Row5 a;
    (void)eval_point<0, FORM>(p, u, x, y, a);
    double* row = Bn + (size_t)i * ld + w;  // row[c - i] holds column c
    row[0] = a.C;
    if (x > 0) row[-1] = a.W;
    if (x < nx - 1) row[1] = a.E;
    if (y > 0) row[-nx] = a.S;
    if (y < ny - 1) row[nx] = a.N;
  }
  __syncthreads();
  __shared__ double Wn[(kBandMaxW + 1) * (2 * kBandMaxW + 1)];
  __shared__ double mk[kBandMaxW + 1];
  const int first = min(S, ns);
  for (int t = threadIdx.x; t < first * ld; t += blockDim.x) Wn[t] = Bn[t];
  __syncthreads();
  int bad = 0;
  for (int k = 0, ks = 0; k < ns; ++k, ks = ks + 1 == S ? 0 : ks + 1) {  // ks = k % S
    const double* rk = Wn + ks * ld;
    const double piv = rk[w];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) bad = 1;
    const int ie = min(w, ns - 1 - k);  // rows below the pivot inside the band
    // multipliers l_{k+d,k} = a_{k+d,k} / piv, d = 1..ie (column k of row k+d sits at w - d)
    for (int d = 1 + threadIdx.x; d <= ie; d += blockDim.x) {
      double* rd = Wn + (ks + d < S ? ks + d : ks + d - S) * ld;
      const double m = rd[w - d] / piv;
      rd[w - d] = m;
      mk[d] = m;
    }
    __syncthreads();
    // trailing update a_{k+d,k+e} -= l_{k+d,k} u_{k,k+e}, d, e = 1..ie
    {
      const int e = 1 + (threadIdx.x & 63);
      if (e <= ie)
        for (int d = 1 + (threadIdx.x >> 6); d <= ie; d += blockDim.x >> 6)
          Wn[(ks + d < S ? ks + d : ks + d - S) * ld + w + e - d] -= mk[d] * rk[w + e];
    }
    __syncthreads();
    // row k is final: store it, load row k + w + 1 into its slot
    double* gk = Bn + (size_t)k * ld;
    const int kn = k + S;
    for (int t = threadIdx.x; t < ld; t += blockDim.x) {
      gk[t] = rk[t];
      if (kn < ns) Wn[ks * ld + t] = Bn[(size_t)kn * ld + t];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) status[n] = bad;
}

// Eq. (7) through the factors, level after level, in one wave: b = r^n + du^{n-1} (the -I
// block), L y = b row by row (lane j holds the product with y_{i-w+j}, then a wave sum),
// U x = y from the last row up; du^n = x. y and x live in LDS (ns <= kBandMaxW^2).
__global__ __launch_bounds__(64) void k_band_chain(int nx, int ny, int nt, const double* __restrict__ B,
                                                   const double* __restrict__ R, double* __restrict__ dU) {
  const int w = nx, ld = 2 * w + 1, ns = nx * ny;
  const int lane = threadIdx.x;
  __shared__ double y[kBandMaxW * kBandMaxW];
  for (int n = 0; n < nt; ++n) {
    const double* Bn = B + (size_t)n * ns * ld;
    const double* rn = R + (size_t)n * ns;
    const double* dp = n > 0 ? dU + (size_t)(n - 1) * ns : nullptr;
    double* xo = dU + (size_t)n * ns;
    for (int i = lane; i < ns; i += 64) y[i] = rn[i] + (dp ? dp[i] : 0.0);
    __syncthreads();
    // forward: y_i -= sum_{c = i-w}^{i-1} l_{i,c} y_c (lane j: column c = i - w + j)
    for (int i = 1; i < ns; ++i) {
      const int c = i - w + lane;
      double v = (lane < w && c >= 0) ? Bn[(size_t)i * ld + lane] * y[c] : 0.0;
      v = wave_sum(v);
      if (lane == 0) y[i] -= v;
      __syncthreads();
    }
    // backward: x_i = (y_i - sum_{c = i+1}^{i+w} u_{i,c} x_c) / u_{i,i} (x overwrites y)
    for (int i = ns - 1; i >= 0; --i) {
      const int c = i + 1 + lane;
      double v = (lane < w && c < ns) ? Bn[(size_t)i * ld + w + 1 + lane] * y[c] : 0.0;
      v = wave_sum(v);
      if (lane == 0) y[i] = (y[i] - v) / Bn[(size_t)i * ld + w];
      __syncthreads();
    }
    for (int i = lane; i < ns; i += 64) xo[i] = y[i];
    __syncthreads();
  }
}

}  // namespace pts
