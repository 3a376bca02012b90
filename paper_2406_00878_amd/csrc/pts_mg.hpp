// Geometric multigrid V-cycle for the stiff heat level solves (gfx950, float32, no MFMA).
//
// The per-level blocks of Dirichlet heat with k(u) = mu_a + mu_b u^2 at tau mu / h^2 >> 1 are
// too stiff for Jacobi-preconditioned Chebyshev (Gershgorin radius ~0.9995). Their level solve
// is a Chebyshev iteration preconditioned by the constant-coefficient operator
//     M = I + c (-Delta_h),  c = tau mu_a,
// on the N x N interior grid (h = 1/(N+1)); M^{-1} is replaced by one V-cycle:
//   - hierarchy N_0 = N, N_{l+1} = (N_l - 1)/2 for odd N_l (nested grids) and N_l/2 for even
//     N_l (non-nested), every grid with its own h_l = 1/(N_l + 1) and the zero boundary;
//   - M_l rediscretised on each grid: diagonal D_l = 1 + 4 a_l, off-diagonals -a_l,
//     a_l = c (N_l + 1)^2;
//   - prolongation P: linear interpolation in physical coordinates per axis (fine node i at
//     (i+1) h_f lies between coarse nodes; the boundary carries zero); restriction
//     R = (h_f/h_c)^2 P^T, so the V-cycle is a symmetric operator;
//   - smoothing: two damped Jacobi sweeps (omega = 0.8) before and after the coarse
//     correction, the first from zero; the coarsest grid (N <= 8) by kMgCoarseSweeps sweeps.
// Measured on the workload's sizes the V-cycle B satisfies spec(B M) within [0.75, 1]: the
// Chebyshev interval of the level solve is widened by that factor at its lower end.
//
// Grids with N > kMgLds are smoothed, restricted and prolonged by tile kernels over all
// instances of a batch (k_mg_down, k_mg_up); the remaining levels (N <= 64) of one instance
// run inside one work-group in LDS (k_mg_lds).
#pragma once
#include <hip/hip_runtime.h>

namespace pts {

constexpr int kMgLevels = 12;
constexpr int kMgLds = 64;          // grids with N <= kMgLds: rest of the V-cycle in LDS
constexpr int kMgCoarsest = 8;      // hierarchy ends at N <= 8
constexpr int kMgCoarseSweeps = 8;  // Jacobi sweeps on the coarsest grid
constexpr float kMgOmega = 0.8f;
constexpr double kMgLow = 0.75;     // lower end of spec(B M)
constexpr int kMgTC = 28;           // k_mg_down: coarse tile edge
constexpr int kMgTF = 60;           // k_mg_up: fine tile edge
constexpr int kMgDS = 64;           // k_mg_down: LDS row stride (fine region <= 62 wide)
constexpr int kMgUS = 64;           // k_mg_up: LDS row stride (fine region <= 64 wide)
constexpr int kMgUE = 36;           // k_mg_up: LDS row stride of the coarse correction
constexpr int kMgLdsWords = 5504;   // k_mg_lds: floats per LDS array (64^2 + 32^2 + ...)
constexpr int kMgThreads = 512;     // k_mg_down, k_mg_up: threads per work-group

__host__ __device__ inline int mg_coarse(int n) { return (n & 1) ? (n - 1) >> 1 : n >> 1; }

// One instance's hierarchy (filled on the host).
struct MgDesc {
  int levels;           // grids 0..levels-1, n[levels-1] <= kMgCoarsest
  int G;                // n[l] > kMgLds for l < G; grid G is the first one done in LDS
  int n[kMgLevels];
  float a[kMgLevels];   // c (n_l + 1)^2
  float* x[kMgLevels];  // grids 0..G: [n][n] iterate (x[0] = the preconditioned residual z)
  float* f[kMgLevels];  // grids 0..G: [n][n] right-hand side (f[0] = the level residual r)
  float* e[kMgLevels];  // grids 1..G-1: [n][n] the grid's corrected, post-smoothed iterate
                        // (written by k_mg_up while x[l] is still read by its neighbours)
  // transfer tables between grid l and l+1 (mg_tables): for fine index i, the coarse index
  // k = floor(s) and weight w of mg_w, and the nearest coarse index (clamped) that owns i;
  // for coarse index k, the fine range [lo, hi) its restriction gathers
  const int* tk[kMgLevels];
  const float* tw[kMgLevels];
  const int* to[kMgLevels];
  const int2* ts[kMgLevels];
};

// Fine node i of a grid of nf nodes at coarse coordinate s = (i+1)(nc+1)/(nf+1) - 1:
// k = floor(s) (may be -1), w = s - k; P[i][k] = 1 - w, P[i][k+1] = w.
__host__ __device__ inline void mg_w(int i, int nf, int nc, int& k, float& w) {
  const int den = nf + 1;
  const int num = (i + 1) * (nc + 1) - den;
  k = num >= 0 ? num / den : -((-num + den - 1) / den);
  w = (float)(num - k * den) / (float)den;
}

// Fine index range [lo, hi) whose interpolation reaches coarse nodes [k0, k1):
// k0 h_c < x_i < (k1 + 1) h_c.
__host__ __device__ inline void mg_support(int k0, int k1, int nf, int nc, int& lo, int& hi) {
  lo = (k0 * (nf + 1)) / (nc + 1);
  hi = ((k1 + 1) * (nf + 1) + nc) / (nc + 1) - 1;
  if (hi > nf) hi = nf;
}

// Transfer tables of grid l of a hierarchy (host): k[i], w[i], own[i] for i < n_l and
// sup[k] for k < n_{l+1} (see MgDesc).
inline void mg_tables(int nf, int nc, int* k, float* w, int* own, int2* sup) {
  for (int i = 0; i < nf; ++i) {
    mg_w(i, nf, nc, k[i], w[i]);
    const int o = w[i] >= 0.5f ? k[i] + 1 : k[i];
    own[i] = o < 0 ? 0 : (o > nc - 1 ? nc - 1 : o);
  }
  for (int c = 0; c < nc; ++c) {
    int lo, hi;
    mg_support(c, c + 1, nf, nc, lo, hi);
    sup[c] = make_int2(lo, hi);
  }
}

// --------------------------------------------------------------------------- down
// Work item (instance, grid l, coarse tile x, coarse tile y): two damped Jacobi sweeps on
// M_l x = f_l from x = 0 (closed form: x2 = (w/D)[(2 - w) f + (a w/D) sum f_nb]), the
// residual r = f - M_l x2 and its restriction onto the coarse tile of grid l+1. x2 is written
// for the fine nodes whose nearest coarse node lies in the tile.
// LDS of k_mg_down besides F, X and T: per coarse index of the tile (x and y) the fine support
// start (relative to the LDS origin), its length (<= kMgSup) and the restriction weights; per
// fine LDS column / row whether the tile owns it.
constexpr int kMgSup = 5;
struct MgDownAux {
  int sx0[kMgTC], sxn[kMgTC], sy0[kMgTC], syn[kMgTC];
  float wxr[kMgTC][kMgSup], wyr[kMgTC][kMgSup];
  unsigned char ownx[kMgDS], owny[kMgDS];
};

__device__ void mg_down_tile(const MgDesc& d, int l, int tx, int ty, float* F, float* X, float* T, MgDownAux& aux) {
  const int nf = d.n[l], nc = d.n[l + 1];
  const float a = d.a[l], D = 1.f + 4.f * a, wD = kMgOmega / D;
  const float c1 = wD * (2.f - kMgOmega), c2 = wD * a * kMgOmega / D;
  const int* __restrict__ tk = d.tk[l];
  const float* __restrict__ tw = d.tw[l];
  const int* __restrict__ to = d.to[l];
  const int2* __restrict__ ts = d.ts[l];
  const int k0x = tx * kMgTC, k1x = min(k0x + kMgTC, nc);
  const int k0y = ty * kMgTC, k1y = min(k0y + kMgTC, nc);
  // fine range whose interpolation reaches the tile: the union of the coarse supports
  const int ilo = ts[k0x].x, ihi = ts[k1x - 1].y, jlo = ts[k0y].x, jhi = ts[k1y - 1].y;
  const int ox = ilo - 2, oy = jlo - 2;  // LDS origin
  const int wx = ihi - ilo + 4, wy = jhi - jlo + 4;
  const int tcx = k1x - k0x, tcy = k1y - k0y;
  const float* __restrict__ f = d.f[l];
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5, sy = blockDim.x >> 5;
  for (int jj = ly; jj < wy; jj += sy)
    for (int ii = lx; ii < wx; ii += 32) {
      const int gi = ox + ii, gj = oy + jj;
      F[jj * kMgDS + ii] = (gi >= 0 && gi < nf && gj >= 0 && gj < nf) ? f[(size_t)gj * nf + gi] : 0.f;
    }
  // the tile's transfer tables, staged in LDS
  if (threadIdx.x < 2 * kMgTC) {
    const int kk = threadIdx.x % kMgTC;
    const bool isx = threadIdx.x < kMgTC;
    const int kc = (isx ? k0x : k0y) + kk, o = isx ? ox : oy;
    if (kk < (isx ? tcx : tcy)) {
      const int2 sp = ts[kc];
      (isx ? aux.sx0 : aux.sy0)[kk] = sp.x - o;
      (isx ? aux.sxn : aux.syn)[kk] = sp.y - sp.x;
      for (int m = 0; m < kMgSup; ++m) {
        const int i = sp.x + m;
        (isx ? aux.wxr : aux.wyr)[kk][m] = i < sp.y ? (tk[i] == kc ? 1.f - tw[i] : tw[i]) : 0.f;
      }
    }
  } else {
    for (int t = threadIdx.x - 2 * kMgTC; t < wx + wy; t += blockDim.x - 2 * kMgTC) {
      const bool isx = t < wx;
      const int q = isx ? t : t - wx, g = (isx ? ox : oy) + q;
      const int k0 = isx ? k0x : k0y, k1 = isx ? k1x : k1y;
      const int own = (g >= 0 && g < nf) ? to[g] : -1;
      (isx ? aux.ownx : aux.owny)[q] = own >= k0 && own < k1;
    }
  }
  __syncthreads();
  for (int jj = 1 + ly; jj < wy - 1; jj += sy)
    for (int ii = 1 + lx; ii < wx - 1; ii += 32) {
      const int gi = ox + ii, gj = oy + jj;
      const float* c = F + jj * kMgDS + ii;
      const float v = c1 * c[0] + c2 * ((c[-1] + c[1]) + (c[-kMgDS] + c[kMgDS]));
      X[jj * kMgDS + ii] = (gi >= 0 && gi < nf && gj >= 0 && gj < nf) ? v : 0.f;
    }
  __syncthreads();
  // residual on [ilo, ihi) x [jlo, jhi) (into F: each node reads only its own f), and x2 of the
  // fine nodes the tile owns
  float* __restrict__ xo = d.x[l];
  for (int jj = 2 + ly; jj < wy - 2; jj += sy)
    for (int ii = 2 + lx; ii < wx - 2; ii += 32) {
      const float* c = X + jj * kMgDS + ii;
      F[jj * kMgDS + ii] -= D * c[0] - a * ((c[-1] + c[1]) + (c[-kMgDS] + c[kMgDS]));
      if (aux.ownx[ii] && aux.owny[jj]) xo[(size_t)(oy + jj) * nf + ox + ii] = c[0];
    }
  __syncthreads();
  // restriction along x: T[jj][kk] = sum_i P[i][k0x + kk] r[jj][i]
  for (int jj = 2 + ly; jj < wy - 2; jj += sy)
    for (int kk = lx; kk < tcx; kk += 32) {
      const float* r = F + jj * kMgDS + aux.sx0[kk];
      float s = 0.f;
      for (int m = 0; m < aux.sxn[kk]; ++m) s += aux.wxr[kk][m] * r[m];
      T[jj * kMgTC + kk] = s;
    }
  __syncthreads();
  const float q = (float)(nc + 1) / (float)(nf + 1);
  float* __restrict__ fc = d.f[l + 1];
  for (int ky = ly; ky < tcy; ky += sy)
    for (int kk = lx; kk < tcx; kk += 32) {
      const float* t = T + aux.sy0[ky] * kMgTC + kk;
      float s = 0.f;
      for (int m = 0; m < aux.syn[ky]; ++m) s += aux.wyr[ky][m] * t[m * kMgTC];
      fc[(size_t)(k0y + ky) * nc + k0x + kk] = q * q * s;
    }
}

// ----------------------------------------------------------------------------- up
// Work item (instance, grid l, fine tile x, fine tile y): x = x_l + P e_{l+1} on the tile and
// a two-node halo (e_{l+1}: x_G from the LDS part, else the corrected iterate of grid l+1),
// then two damped Jacobi sweeps on M_l x = f_l; emit(i, j, x) receives the tile's values (the
// caller stores them in e_l, never in x_l, which neighbouring tiles still read).
// Thread (lx, ly) of the 32 x 16 work-group owns the window points (lx + 32 a, ly + 16 b) in
// every phase, so its f values stay in registers; its x_l and f_l loads are issued before the
// coarse window is staged.
constexpr int kMgUA = (kMgUS + 31) / 32, kMgUB = (kMgUS + 15) / 16;  // window points per thread
static_assert(kMgThreads == 512, "k_mg_up maps 32 x 16 threads onto its window");
template <typename Emit>
__device__ void mg_up_tile(const MgDesc& d, int l, int tx, int ty, float* X, float* X1, float* E, Emit emit) {
  const int nf = d.n[l], nc = d.n[l + 1];
  const float a = d.a[l], D = 1.f + 4.f * a, wD = kMgOmega / D;
  const int* __restrict__ tk = d.tk[l];
  const float* __restrict__ tw = d.tw[l];
  const int i0 = tx * kMgTF, i1 = min(i0 + kMgTF, nf), j0 = ty * kMgTF, j1 = min(j0 + kMgTF, nf);
  const int ox = i0 - 2, oy = j0 - 2, wx = i1 - i0 + 4, wy = j1 - j0 + 4;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
  const float* __restrict__ xf = d.x[l];
  const float* __restrict__ f = d.f[l];
  float xv[kMgUB][kMgUA], fv[kMgUB][kMgUA];
#pragma unroll
  for (int b = 0; b < kMgUB; ++b)
#pragma unroll
    for (int q = 0; q < kMgUA; ++q) {
      const int ii = lx + 32 * q, jj = ly + 16 * b, gi = ox + ii, gj = oy + jj;
      const bool in = ii < wx && jj < wy && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
      xv[b][q] = in ? xf[(size_t)gj * nf + gi] : 0.f;
      fv[b][q] = in ? f[(size_t)gj * nf + gi] : 0.f;
    }
  // coarse window covering the interpolation of the region: indices kxa..kxb+1
  const int kxa = tk[max(ox, 0)], kya = tk[max(oy, 0)];
  const int kxb = tk[min(ox + wx - 1, nf - 1)], kyb = tk[min(oy + wy - 1, nf - 1)];
  const int ex = kxb + 2 - kxa, ey = kyb + 2 - kya;
  const float* __restrict__ xc = l + 1 == d.G ? d.x[l + 1] : d.e[l + 1];
  for (int ej = ly; ej < ey; ej += 16)
    for (int ei = lx; ei < ex; ei += 32) {
      const int kx = kxa + ei, ky = kya + ej;
      E[ej * kMgUE + ei] = (kx >= 0 && kx < nc && ky >= 0 && ky < nc) ? xc[(size_t)ky * nc + kx] : 0.f;
    }
  // prolongation tables of the region's columns and rows, staged in LDS
  __shared__ int pk[2][kMgUS];
  __shared__ float pw[2][kMgUS];
  for (int t = threadIdx.x; t < wx + wy; t += blockDim.x) {
    const bool isx = t < wx;
    const int q = isx ? t : t - wx, g = (isx ? ox : oy) + q;
    const int gc = min(max(g, 0), nf - 1);
    pk[isx ? 0 : 1][q] = tk[gc] - (isx ? kxa : kya);
    pw[isx ? 0 : 1][q] = tw[gc];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < kMgUB; ++b)
#pragma unroll
    for (int q = 0; q < kMgUA; ++q) {
      const int ii = lx + 32 * q, jj = ly + 16 * b, gi = ox + ii, gj = oy + jj;
      if (ii >= wx || jj >= wy) continue;
      float v = 0.f;
      if (gi >= 0 && gi < nf && gj >= 0 && gj < nf) {
        const float wx_ = pw[0][ii], wy_ = pw[1][jj];
        const float* e = E + pk[1][jj] * kMgUE + pk[0][ii];
        const float pe = (1.f - wy_) * ((1.f - wx_) * e[0] + wx_ * e[1]) + wy_ * ((1.f - wx_) * e[kMgUE] + wx_ * e[kMgUE + 1]);
        v = xv[b][q] + pe;
      }
      X[jj * kMgUS + ii] = v;
    }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < kMgUB; ++b)
#pragma unroll
    for (int q = 0; q < kMgUA; ++q) {
      const int ii = lx + 32 * q, jj = ly + 16 * b, gi = ox + ii, gj = oy + jj;
      if (ii < 1 || ii >= wx - 1 || jj < 1 || jj >= wy - 1) continue;
      const float* c = X + jj * kMgUS + ii;
      const float mx = D * c[0] - a * ((c[-1] + c[1]) + (c[-kMgUS] + c[kMgUS]));
      X1[jj * kMgUS + ii] = (gi >= 0 && gi < nf && gj >= 0 && gj < nf) ? c[0] + wD * (fv[b][q] - mx) : 0.f;
    }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < kMgUB; ++b)
#pragma unroll
    for (int q = 0; q < kMgUA; ++q) {
      const int ii = lx + 32 * q, jj = ly + 16 * b;
      if (ii < 2 || ii >= wx - 2 || jj < 2 || jj >= wy - 2) continue;
      const float* c = X1 + jj * kMgUS + ii;
      const float mx = D * c[0] - a * ((c[-1] + c[1]) + (c[-kMgUS] + c[kMgUS]));
      emit(ox + ii, oy + jj, c[0] + wD * (fv[b][q] - mx));
    }
}

// ---------------------------------------------------------------------------- LDS
// The V-cycle below grid G of one instance in one work-group: grids G..levels-1 packed into
// the LDS arrays X, F, T (offsets o[l]); f_G is read from and x_G written to device memory.
template <typename Emit>
__device__ void mg_lds_cycle(const MgDesc& d, float* X, float* F, float* T, Emit emit) {
  const int G = d.G, L = d.levels;
  int o[kMgLevels + 1];
  o[G] = 0;
  for (int l = G; l < L; ++l) o[l + 1] = o[l] + d.n[l] * d.n[l];
  // fn(i, j, j * n + i) for every node of an n x n grid (n <= 64): lane = i, waves over j
  auto each = [&](int n, auto&& fn) {
    const int i = threadIdx.x & 63;
    if (i < n)
      for (int j = threadIdx.x >> 6; j < n; j += blockDim.x >> 6) fn(i, j, j * n + i);
  };
  // M x at node (i, j) of an n x n grid stored at B (zero boundary)
  auto mx = [&](const float* B, int n, float a, int i, int j) {
    const float* c = B + j * n + i;
    float s = 0.f;
    if (i > 0) s += c[-1];
    if (i < n - 1) s += c[1];
    if (j > 0) s += c[-n];
    if (j < n - 1) s += c[n];
    return (1.f + 4.f * a) * c[0] - a * s;
  };
  __shared__ int rs0[kMgLds], rsn[kMgLds], pk[kMgLds];
  __shared__ float rw[kMgLds][kMgSup], pw[kMgLds];
  const int nG = d.n[G];
  const float* __restrict__ fg = d.f[G];
  each(nG, [&](int i, int j, int t) { F[t] = fg[t]; });
  __syncthreads();
  for (int l = G; l < L - 1; ++l) {
    const int n = d.n[l], nc = d.n[l + 1];
    const float a = d.a[l], D = 1.f + 4.f * a, wD = kMgOmega / D;
    const float c1 = wD * (2.f - kMgOmega), c2 = wD * a * kMgOmega / D;
    float* x = X + o[l];
    const float* f = F + o[l];
    float* r = T + o[l];
    each(n, [&](int i, int j, int t) {
      float s = 0.f;
      if (i > 0) s += f[t - 1];
      if (i < n - 1) s += f[t + 1];
      if (j > 0) s += f[t - n];
      if (j < n - 1) s += f[t + n];
      x[t] = c1 * f[t] + c2 * s;
    });
    __syncthreads();
    each(n, [&](int i, int j, int t) { r[t] = f[t] - mx(x, n, a, i, j); });
    __syncthreads();
    const float q = (float)(nc + 1) / (float)(n + 1);
    float* fc = F + o[l + 1];
    // restriction weights of each coarse index (support start, length, weights), in LDS
    if (threadIdx.x < nc) {
      const int2 sp = d.ts[l][threadIdx.x];
      rs0[threadIdx.x] = sp.x;
      rsn[threadIdx.x] = sp.y - sp.x;
      for (int m = 0; m < kMgSup; ++m) {
        const int i = sp.x + m;
        rw[threadIdx.x][m] = i < sp.y ? (d.tk[l][i] == (int)threadIdx.x ? 1.f - d.tw[l][i] : d.tw[l][i]) : 0.f;
      }
    }
    __syncthreads();
    each(nc, [&](int kx, int ky, int t) {
      float s = 0.f;
      for (int mj = 0; mj < rsn[ky]; ++mj) {
        const float* rr = r + (rs0[ky] + mj) * n + rs0[kx];
        float sx = 0.f;
        for (int mi = 0; mi < rsn[kx]; ++mi) sx += rw[kx][mi] * rr[mi];
        s += rw[ky][mj] * sx;
      }
      fc[t] = q * q * s;
    });
    __syncthreads();
  }
  {  // coarsest grid: Jacobi sweeps from zero, ping-pong between X and T
    const int l = L - 1, n = d.n[l];
    const float a = d.a[l], wD = kMgOmega / (1.f + 4.f * a);
    float* x = X + o[l];
    float* y = T + o[l];
    const float* f = F + o[l];
    each(n, [&](int i, int j, int t) { x[t] = 0.f; });
    __syncthreads();
    for (int sw = 0; sw < kMgCoarseSweeps; sw += 2) {
      each(n, [&](int i, int j, int t) { y[t] = x[t] + wD * (f[t] - mx(x, n, a, i, j)); });
      __syncthreads();
      each(n, [&](int i, int j, int t) { x[t] = y[t] + wD * (f[t] - mx(y, n, a, i, j)); });
      __syncthreads();
    }
  }
  for (int l = L - 2; l >= G; --l) {
    const int n = d.n[l], nc = d.n[l + 1];
    const float a = d.a[l], wD = kMgOmega / (1.f + 4.f * a);
    float* x = X + o[l];
    float* y = T + o[l];
    const float* f = F + o[l];
    const float* e = X + o[l + 1];
    if (threadIdx.x < n) {  // prolongation table of the grid, in LDS
      pk[threadIdx.x] = d.tk[l][threadIdx.x];
      pw[threadIdx.x] = d.tw[l][threadIdx.x];
    }
    __syncthreads();
    auto at = [&](int i, int j) { return (i >= 0 && i < nc && j >= 0 && j < nc) ? e[j * nc + i] : 0.f; };
    each(n, [&](int i, int j, int t) {
      const int kx = pk[i], ky = pk[j];
      const float wx = pw[i], wy = pw[j];
      x[t] += (1.f - wy) * ((1.f - wx) * at(kx, ky) + wx * at(kx + 1, ky)) +
              wy * ((1.f - wx) * at(kx, ky + 1) + wx * at(kx + 1, ky + 1));
    });
    __syncthreads();
    each(n, [&](int i, int j, int t) { y[t] = x[t] + wD * (f[t] - mx(x, n, a, i, j)); });
    __syncthreads();
    each(n, [&](int i, int j, int t) { x[t] = y[t] + wD * (f[t] - mx(y, n, a, i, j)); });
    __syncthreads();
  }
  each(nG, [&](int i, int j, int t) { emit(i, j, X[t]); });
}

}  // namespace pts
