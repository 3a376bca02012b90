// Theorem 1 in the paper's own form: the products P^l = A_1 A_2 ... A_l formed explicitly and
// every level solved on its own (Section 4, Eq. (8); Section 5, Eq. (9) and Algorithm 1).
//
//   P^1 = A_1,  P^l = P^{l-1} A_l;   rt^1 = r^1,  rt^l = P^{l-1} r^l + rt^{l-1};
//   P^l du^l = rt^l  for every l independently.
//
// Storage of P^l ("diamond"): the five-point blocks couple node (x, y) to (x + b, y + a) with
// |a| + |b| <= 1, so the product of l of them couples it to offsets with |a| + |b| <= l: the
// 2 l^2 + 2 l + 1 diagonals of the Section 5 remark. Entry e of row (x, y) holds the coupling
// to offset (a, b), entries ordered by a = -l..l, then b; planes [e][ny][nx] (x fastest).
// Each entry of P^l is a sum of at most five products (the Lemma of Section 5).
//
// The levels' systems are solved by banded LU without pivoting (the paper's direct solver for
// banded matrices), after the Section 7 diagonal preconditioner: every row of P^l and rt^l is
// divided by the row's diagonal entry. In the x-fastest ordering P^l has half-bandwidth
// w_l = min(l nx, N_s - 1); the band B_l[row][w_l + col - row] (2 w_l + 1 entries per row) is
// factorised by a right-looking blocked LU: per panel of kPb columns a panel factorisation
// (one work-group per level), a triangular solve for the panel's rows (U12) and the trailing
// update A22 -= L21 U12 (64 x 64 tiles over every level's band), all levels in each launch.
#pragma once
#include <hip/hip_runtime.h>

#include "pts_device.hpp"

namespace pts {

constexpr int kPb = 32;  // panel width of the blocked band LU

// Row of diagonal offset a (|a| <= l) in the diamond of radius l: entries before it.
__host__ __device__ inline int dia_base(int l, int a) {
  return a <= 0 ? (a + l) * (a + l) : l * l + 2 * l * a + 2 * a - a * a;
}
__host__ __device__ inline int dia_count(int l) { return 2 * l * l + 2 * l + 1; }
__host__ __device__ inline int dia_index(int l, int a, int b) { return dia_base(l, a) + b + (l - (a < 0 ? -a : a)); }
// (a, b) of entry e of the diamond of radius l
__device__ inline void dia_offset(int l, int e, int& a, int& b) {
  a = -l;
  while (a < l && dia_base(l, a + 1) <= e) ++a;
  b = e - dia_base(l, a) - (l - (a < 0 ? -a : a));
}

// P^l from P^{l-1} (radius l-1, Dp) and the rows of A_l (coef: planes C, W, E, S, N), one
// thread per (entry, node). l = 1: P^1 = A_1 (Dp unused).
__global__ __launch_bounds__(256) void k_prod_level(int nx, int ny, int l, const double* __restrict__ Dp,
                                                    const double* __restrict__ coef, double* __restrict__ Dc) {
  const size_t ns = (size_t)nx * ny;
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)dia_count(l) * ns) return;
  const int e = (int)(t / ns);
  const int i = (int)(t % ns);
  const int x = i % nx, y = i / nx;
  int a, b;
  dia_offset(l, e, a, b);
  // A's five entries: (da, db, plane) = (0,0,C) (0,-1,W) (0,1,E) (-1,0,S) (1,0,N)
  const int da[5] = {0, 0, 0, -1, 1}, db[5] = {0, -1, 1, 0, 0};
  double s = 0.0;
  if (l == 1) {
    for (int q = 0; q < 5; ++q)
      if (da[q] == a && db[q] == b) s = coef[(size_t)q * ns + i];
  } else {
    for (int q = 0; q < 5; ++q) {
      const int a1 = a - da[q], b1 = b - db[q];  // offset inside P^{l-1}
      if ((a1 < 0 ? -a1 : a1) + (b1 < 0 ? -b1 : b1) > l - 1) continue;
      const int kx = x + b1, ky = y + a1;  // the intermediate node k
      if (kx < 0 || kx >= nx || ky < 0 || ky >= ny) continue;
      s += Dp[(size_t)dia_index(l - 1, a1, b1) * ns + i] * coef[(size_t)q * ns + (size_t)ky * nx + kx];
    }
  }
  Dc[t] = s;
}

// rt^l = P^{l-1} r^l + rt^{l-1} (l >= 2; Dp of radius l-1), rt^1 = r^1. One thread per node.
__global__ __launch_bounds__(256) void k_prod_rhs(int nx, int ny, int l, const double* __restrict__ Dp,
                                                  const double* __restrict__ rl, const double* __restrict__ rt_prev,
                                                  double* __restrict__ rt) {
  const size_t ns = (size_t)nx * ny;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= (int)ns) return;
  if (l == 1) {
    rt[i] = rl[i];
    return;
  }
  const int x = i % nx, y = i / nx, r = l - 1;
  double s = 0.0;
  for (int a = -r; a <= r; ++a) {
    const int ky = y + a, br = r - (a < 0 ? -a : a);
    if (ky < 0 || ky >= ny) continue;
    const int e0 = dia_base(r, a);
    for (int b = -br; b <= br; ++b) {
      const int kx = x + b;
      if (kx < 0 || kx >= nx) continue;
      s += Dp[(size_t)(e0 + b + br) * ns + i] * rl[(size_t)ky * nx + kx];
    }
  }
  rt[i] = s + rt_prev[i];
}

// Band storage of P^l with the diagonal preconditioner: row i divided by p_ii, and rs_i =
// rt_i / p_ii (rt itself stays unscaled: the recursion reads it for the next level). One thread
// per (entry, node); the band (zeroed beforehand) takes the entries whose column node lies
// inside the grid.
__global__ __launch_bounds__(256) void k_prod_band(int nx, int ny, int l, int w, const double* __restrict__ Dc,
                                                   double* __restrict__ B, const double* __restrict__ rt,
                                                   double* __restrict__ rs) {
  const size_t ns = (size_t)nx * ny;
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)dia_count(l) * ns) return;
  const int e = (int)(t / ns);
  const int i = (int)(t % ns);
  const int x = i % nx, y = i / nx;
  int a, b;
  dia_offset(l, e, a, b);
  const int kx = x + b, ky = y + a;
  const double d = Dc[(size_t)dia_index(l, 0, 0) * ns + i];
  if (kx >= 0 && kx < nx && ky >= 0 && ky < ny) {
    const long col = (long)ky * nx + kx;
    B[(size_t)i * (2 * w + 1) + (size_t)(w + col - i)] = Dc[t] / d;
  }
  if (a == 0 && b == 0) rs[i] = rt[i] / d;
}

// Per-level parameters of the blocked band LU.
struct BandLevel {
  double* B;  // [ns][2w + 1]
  int w;
};

__device__ __forceinline__ double& bel(const BandLevel& L, int r, int c) {
  return L.B[(size_t)r * (2 * L.w + 1) + (L.w + c - r)];
}

// (a) panel [k0, k0 + kPb): unblocked LU of its columns over the rows the band reaches
// (one work-group per level, blockIdx.x). A zero or non-finite pivot sets *flag.
__global__ __launch_bounds__(256) void k_blu_panel(const BandLevel* __restrict__ lv, int ns, int k0,
                                                   int* __restrict__ flag) {
  const BandLevel L = lv[blockIdx.x];
  const int kend = min(k0 + kPb, ns);
  for (int c = k0; c < kend; ++c) {
    const double piv = bel(L, c, c);
    if (threadIdx.x == 0 && (!(fabs(piv) > 0.0) || !isfinite(piv))) atomicOr(flag, 1);
    const int rend = min(ns, c + L.w + 1);
    for (int r = c + 1 + threadIdx.x; r < rend; r += blockDim.x) bel(L, r, c) /= piv;
    __syncthreads();
    // rows c+1..rend-1, panel columns c+1..min(kend, c+w+1)-1: u_{c,c2} lies in the band, and
    // then so does a_{r,c2}
    const int nr = rend - c - 1, nc = min(kend, c + L.w + 1) - c - 1;
    for (int t = threadIdx.x; t < nr * nc; t += blockDim.x) {
      const int r = c + 1 + t / nc, c2 = c + 1 + t % nc;
      bel(L, r, c2) -= bel(L, r, c) * bel(L, c, c2);
    }
    __syncthreads();
  }
}

// (b) U12: rows [k0, k0 + kPb) of the columns [k0 + kPb, k0 + kPb + w) solved with the panel's
// unit lower triangle, one thread per column (grid.x over columns, grid.y = level).
__global__ __launch_bounds__(256) void k_blu_trsm(const BandLevel* __restrict__ lv, int ns, int k0) {
  const BandLevel L = lv[blockIdx.y];
  const int kend = min(k0 + kPb, ns);
  const int c2 = kend + blockIdx.x * 256 + threadIdx.x;
  if (c2 >= min(ns, kend + L.w)) return;
  for (int r = max(k0, c2 - L.w); r < kend; ++r) {
    double s = bel(L, r, c2);
    for (int m = max(max(k0, c2 - L.w), r - L.w); m < r; ++m) s -= bel(L, r, m) * bel(L, m, c2);
    bel(L, r, c2) = s;
  }
}

// (c) trailing update A22 -= L21 U12 over rows and columns [k0 + kPb, k0 + kPb + w), inside
// the band. One work-group per 64 x 64 tile: grid.x = tile (row-major over the level's tile
// grid), grid.y = level; the panel operands are staged in LDS (zero outside the band).
__global__ __launch_bounds__(256) void k_blu_gemm(const BandLevel* __restrict__ lv, int ns, int k0) {
  const BandLevel L = lv[blockIdx.y];
  const int kend = min(k0 + kPb, ns);
  const int span = min(ns, kend + L.w) - kend;  // rows / columns touched
  if (span <= 0) return;
  const int tn = (span + 63) / 64;
  if ((int)blockIdx.x >= tn * tn) return;
  const int r0 = kend + (blockIdx.x / tn) * 64, c0 = kend + (blockIdx.x % tn) * 64;
  // tiles wholly outside the band do nothing
  if (r0 - (c0 + 63) > L.w || c0 - (r0 + 63) > L.w) return;
  __shared__ double Ls[64][kPb + 1], Us[kPb][64 + 1];
  const int np = kend - k0;
  for (int t = threadIdx.x; t < 64 * kPb; t += 256) {
    const int rr = t / kPb, m = t % kPb, r = r0 + rr, k = k0 + m;
    Ls[rr][m] = (m < np && r < ns && r - k <= L.w) ? bel(L, r, k) : 0.0;
    const int mm = t / 64, cc = t % 64, c = c0 + cc, k2 = k0 + mm;
    Us[mm][cc] = (mm < np && c < ns && c - k2 <= L.w) ? bel(L, k2, c) : 0.0;
  }
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;  // 4 x 4 outputs per thread
  double acc[4][4] = {};
  for (int m = 0; m < kPb; ++m) {
    double lvv[4], uvv[4];
    for (int q = 0; q < 4; ++q) {
      lvv[q] = Ls[tr * 4 + q][m];
      uvv[q] = Us[m][tc * 4 + q];
    }
    for (int q = 0; q < 4; ++q)
      for (int p2 = 0; p2 < 4; ++p2) acc[q][p2] += lvv[q] * uvv[p2];
  }
  for (int q = 0; q < 4; ++q)
    for (int p2 = 0; p2 < 4; ++p2) {
      const int r = r0 + tr * 4 + q, c = c0 + tc * 4 + p2;
      if (r < ns && c < ns && r - c <= L.w && c - r <= L.w) bel(L, r, c) -= acc[q][p2];
    }
}

// Forward and backward substitution of every level with its factors (one work-group per
// level): y = L^{-1} rt, x = U^{-1} y, row by row with a block reduction over the band.
__global__ __launch_bounds__(256) void k_blu_solve(const BandLevel* __restrict__ lv, int ns,
                                                   const double* __restrict__ RT, double* __restrict__ dU) {
  const BandLevel L = lv[blockIdx.x];
  const double* rt = RT + (size_t)blockIdx.x * ns;
  double* x = dU + (size_t)blockIdx.x * ns;
  __shared__ double red[4];
  for (int i = threadIdx.x; i < ns; i += 256) x[i] = rt[i];
  __syncthreads();
  for (int i = 1; i < ns; ++i) {
    double s = 0.0;
    for (int m = max(0, i - L.w) + threadIdx.x; m < i; m += 256) s += bel(L, i, m) * x[m];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) x[i] -= (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
  for (int i = ns - 1; i >= 0; --i) {
    double s = 0.0;
    for (int m = i + 1 + threadIdx.x; m < min(ns, i + L.w + 1); m += 256) s += bel(L, i, m) * x[m];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) x[i] = (x[i] - ((red[0] + red[1]) + (red[2] + red[3]))) / bel(L, i, i);
    __syncthreads();
  }
}

}  // namespace pts
